// Frame-server kernel instance with BF16 descriptor storage.
#include "lf_internal.h"
#include "lf_serve_kernels.h"

namespace lfem {
ServeKernel pick_serve_bf16() { return (ServeKernel)lf_serve_kernel<2>; }
}  // namespace lfem
