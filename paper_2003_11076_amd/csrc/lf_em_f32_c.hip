// EM kernel instances with F32 descriptor storage for 10 to 16 views.
// Each storage format and view-count range is a translation unit of its own
// so that the instances compile in parallel.
#include "lf_em_dispatch.h"

namespace lfem {
EmKernel pick_em_f32_c(int K, bool frac, bool exh, bool sym, bool share, bool enumerate) {
    return pick_em_range<0, 10, 16>(K, frac, exh, sym, share, enumerate);
}
}  // namespace lfem
