// Instantiation of the EM kernel for every view count, shift kind and sweep
// kind of one storage precision.  Each storage precision and range of view
// counts is compiled in its own translation unit (lf_em_{f32,f16,bf16}_{a,b,c}.hip).
#pragma once

#include "lf_em_kernels.h"
#include "lf_internal.h"

namespace lfem {

template <int K, int ST, int SW>
static EmKernel pick_em_fast(bool sym, bool enumerate) {
    if constexpr (SW == kSweepShared) {
        // The shared sweep keeps more state per lane: three waves per SIMD
        // (168 VGPRs, no spills) up to six views, measured faster than four
        // waves with the spills a 128-VGPR cap forces (plain workload 12 %,
        // precision 5 %); the compiler's own register count above that,
        // except for the enumeration E-step of seven to nine views, whose
        // 2^K loop gains more from three waves than the sweep loses
        if constexpr (K <= 6) {
            return sym ? (EmKernel)lf_em_kernel_w3<K, ST, false, SW, true>
                       : (EmKernel)lf_em_kernel_w3<K, ST, false, SW, false>;
        } else if constexpr (K <= 9) {
            if (enumerate)
                return sym ? (EmKernel)lf_em_kernel_w3<K, ST, false, SW, true>
                           : (EmKernel)lf_em_kernel_w3<K, ST, false, SW, false>;
            return sym ? (EmKernel)lf_em_kernel<K, ST, false, SW, true>
                       : (EmKernel)lf_em_kernel<K, ST, false, SW, false>;
        } else {
            return sym ? (EmKernel)lf_em_kernel<K, ST, false, SW, true>
                       : (EmKernel)lf_em_kernel<K, ST, false, SW, false>;
        }
    } else {
        // Occupancy per view count: the fast sweep of few views fits 96 or
        // 128 VGPRs with a few spills outside the sweep (five or four waves
        // per SIMD; FP32 descriptors carry two record paths and stay at four)
        if constexpr (K <= 5 && ST != 0) {
            return sym ? (EmKernel)lf_em_kernel_w5<K, ST, false, SW, true>
                       : (EmKernel)lf_em_kernel_w5<K, ST, false, SW, false>;
        } else if constexpr (K <= 6) {
            return sym ? (EmKernel)lf_em_kernel_w4<K, ST, false, SW, true>
                       : (EmKernel)lf_em_kernel_w4<K, ST, false, SW, false>;
        } else if constexpr (K <= 9) {
            // three waves per SIMD, with a tile wide enough for the LDS to hold them
            return sym ? (EmKernel)lf_em_kernel_w3<K, ST, false, SW, true>
                       : (EmKernel)lf_em_kernel_w3<K, ST, false, SW, false>;
        } else {
            return sym ? (EmKernel)lf_em_kernel<K, ST, false, SW, true>
                       : (EmKernel)lf_em_kernel<K, ST, false, SW, false>;
        }
    }
}

template <int K, int ST>
static EmKernel pick_em_k(bool frac, bool exh, bool sym, bool share, bool enumerate) {
    if (exh)
        return frac ? (EmKernel)lf_em_kernel<K, ST, true, kSweepExhaustive, false>
                    : (EmKernel)lf_em_kernel<K, ST, false, kSweepExhaustive, false>;
    if (frac) return (EmKernel)lf_em_kernel<K, ST, true, kSweepLane, false>;
    return share ? pick_em_fast<K, ST, kSweepShared>(sym, enumerate) : pick_em_fast<K, ST, kSweepLane>(sym, enumerate);
}

// The instance of view count K in [KLO, KHI] (nullptr outside it).
template <int ST, int KLO, int KHI>
static EmKernel pick_em_range(int K, bool frac, bool exh, bool sym, bool share, bool enumerate) {
    if constexpr (KLO > KHI) {
        return nullptr;
    } else {
        if (K == KLO) return pick_em_k<KLO, ST>(frac, exh, sym, share, enumerate);
        return pick_em_range<ST, KLO + 1, KHI>(K, frac, exh, sym, share, enumerate);
    }
}

}  // namespace lfem
