// EM kernel instances with F16 descriptor storage for 6 to 9 views.
// Each storage format and view-count range is a translation unit of its own
// so that the instances compile in parallel.
#include "lf_em_dispatch.h"

namespace lfem {
EmKernel pick_em_f16_b(int K, bool frac, bool exh, bool sym, bool share, bool enumerate) {
    return pick_em_range<1, 6, 9>(K, frac, exh, sym, share, enumerate);
}
}  // namespace lfem
