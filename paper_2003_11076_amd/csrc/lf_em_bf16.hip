// EM and frame-server kernel instances with BF16 descriptor storage.
#include "lf_em_dispatch.h"
#include "lf_serve_kernels.h"

namespace lfem {
EmKernel pick_em_bf16(int K, bool frac, bool exh, bool sym, bool share, bool enumerate) {
    return pick_em_storage<2>(K, frac, exh, sym, share, enumerate);
}
ServeKernel pick_serve_bf16() { return (ServeKernel)lf_serve_kernel<2>; }
}  // namespace lfem
