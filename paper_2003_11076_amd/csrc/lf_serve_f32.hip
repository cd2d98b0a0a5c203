// Frame-server kernel instance with F32 descriptor storage.
#include "lf_internal.h"
#include "lf_serve_kernels.h"

namespace lfem {
ServeKernel pick_serve_f32() { return (ServeKernel)lf_serve_kernel<0>; }
}  // namespace lfem
