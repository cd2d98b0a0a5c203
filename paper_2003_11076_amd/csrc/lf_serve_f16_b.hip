// Frame-server kernel instances with F16 descriptor storage for 6 to 9 views.
#include "lf_internal.h"
#include "lf_serve_kernels.h"

namespace lfem {
ServeKernel pick_serve_f16_b(int K, int kind) { return pick_serve_range<1, 6, 9>(K, kind); }
}  // namespace lfem
