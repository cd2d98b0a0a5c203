// EM and frame-server kernel instances with F16 descriptor storage.
#include "lf_em_dispatch.h"
#include "lf_serve_kernels.h"

namespace lfem {
EmKernel pick_em_f16(int K, bool frac, bool exh, bool sym, bool share, bool enumerate) {
    return pick_em_storage<1>(K, frac, exh, sym, share, enumerate);
}
ServeKernel pick_serve_f16() { return (ServeKernel)lf_serve_kernel<1>; }
}  // namespace lfem
