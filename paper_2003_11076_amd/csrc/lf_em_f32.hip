// EM and frame-server kernel instances with F32 descriptor storage.
#include "lf_em_dispatch.h"
#include "lf_serve_kernels.h"

namespace lfem {
EmKernel pick_em_f32(int K, bool frac, bool exh, bool sym, bool share, bool enumerate) {
    return pick_em_storage<0>(K, frac, exh, sym, share, enumerate);
}
ServeKernel pick_serve_f32() { return (ServeKernel)lf_serve_kernel<0>; }
}  // namespace lfem
