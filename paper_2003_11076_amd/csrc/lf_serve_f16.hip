// Frame-server kernel instance with F16 descriptor storage.
#include "lf_internal.h"
#include "lf_serve_kernels.h"

namespace lfem {
ServeKernel pick_serve_f16() { return (ServeKernel)lf_serve_kernel<1>; }
}  // namespace lfem
