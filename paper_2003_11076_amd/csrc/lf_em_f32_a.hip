// EM kernel instances with F32 descriptor storage for 2 to 5 views.
// Each storage format and view-count range is a translation unit of its own
// so that the instances compile in parallel.
#include "lf_em_dispatch.h"

namespace lfem {
EmKernel pick_em_f32_a(int K, bool frac, bool exh, bool sym, bool share, bool enumerate) {
    return pick_em_range<0, 2, 5>(K, frac, exh, sym, share, enumerate);
}
EmKernel pick_em_f32(int K, bool frac, bool exh, bool sym, bool share, bool enumerate) {
    if (K <= 5) return pick_em_f32_a(K, frac, exh, sym, share, enumerate);
    if (K <= 9) return pick_em_f32_b(K, frac, exh, sym, share, enumerate);
    return pick_em_f32_c(K, frac, exh, sym, share, enumerate);
}
}  // namespace lfem
