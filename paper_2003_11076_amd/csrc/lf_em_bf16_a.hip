// EM kernel instances with BF16 descriptor storage for 2 to 5 views.
// Each storage format and view-count range is a translation unit of its own
// so that the instances compile in parallel.
#include "lf_em_dispatch.h"

namespace lfem {
EmKernel pick_em_bf16_a(int K, bool frac, bool exh, bool sym, bool share, bool enumerate) {
    return pick_em_range<2, 2, 5>(K, frac, exh, sym, share, enumerate);
}
EmKernel pick_em_bf16(int K, bool frac, bool exh, bool sym, bool share, bool enumerate) {
    if (K <= 5) return pick_em_bf16_a(K, frac, exh, sym, share, enumerate);
    if (K <= 9) return pick_em_bf16_b(K, frac, exh, sym, share, enumerate);
    return pick_em_bf16_c(K, frac, exh, sym, share, enumerate);
}
}  // namespace lfem
