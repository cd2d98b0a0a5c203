// Frame-server kernel instances with F16 descriptor storage for 2 to 5 views.
#include "lf_internal.h"
#include "lf_serve_kernels.h"

namespace lfem {
ServeKernel pick_serve_f16_a(int K, int kind) { return pick_serve_range<1, 2, 5>(K, kind); }
}  // namespace lfem
