// Batched frame kernel of the frame server (gfx950).
//
// One launch covers every (frame, row tile) pair of a batch of admitted
// frames of one kernel key: the same storage format, view count and sweep
// kind, any size and level count.  Block b finds its frame through the
// batch's tile prefix table.  Each block runs the whole method for one row
// tile of serve_tile_width(K) pixels of one frame, with nothing written to HBM in
// between:
//   descriptors of the tile's windows, from three staged rows of R+G+B
//   (Sec. III-C) -> ray prior of each pixel's rays (Sec. III-B) -> n EM
//   iterations (Sec. III-C, III-D), with the plain context's sweeps ->
//   refocus of the static rays (Eq. 2).
// Tiles depend on nothing but their frame's inputs (and the stream's
// previous weights), so a frame gives the same bits alone or in any mix.
#pragma once

#include "lf_em_kernels.h"

namespace lfem {

// Row-tile width (the block size): 128 pixels, two waves.  Blocks of four
// waves (256 pixels) hold their LDS until their slowest wave ends, which
// measured a fifth slower with nine views.
__host__ __device__ constexpr int serve_tile_width(int K) { return (void)K, 128; }
constexpr int kServeTileMax = 128;
// Where a frame's LDS would otherwise limit the blocks a CU holds, a view's
// R+G+B rows are staged inside its own record window, and its records held
// in registers (this many per lane) until every lane has read the rows, for
// windows up to kServeHold tiles wide; other windows, and frames with LDS to
// spare, stage the rows in a scratch area after the records.
constexpr int kServeHold = 8;

// LDS record of a descriptor pair of storage ST as the serve kernel stages it:
// FP32 pairs as int16 Sobel responses (exact), the others as stored; the plain
// context's binary16 and int16 records of FP32 pairs decode to the same values.
template <int ST> constexpr int serve_rec_format() { return ST == 0 ? 3 : ST; }

template <int ST>
__device__ __forceinline__ typename Rec<serve_rec_format<ST>()>::T serve_rec(int gx, int gy) {
    const float sc = 1.0f / 4096.0f;  // exact: |G| <= 3060
    return stage_rec<serve_rec_format<ST>(), ST>(make_pair<ST>((float)gx * sc, (float)gy * sc));
}
constexpr int kServeMaxViews = 9;

// Sweep kinds of the serve kernel instances (one launch per kind):
// integer shifts of a unit-spaced symmetric array and of any array, shared
// by the wave's lanes under the prior bound; integer shifts with a search
// window, each lane on its own; fractional shifts.
constexpr int kServeSharedSym = 0, kServeShared = 1, kServeLane = 2, kServeFrac = 3, kServeKinds = 4;

struct ServeJob {
    EmArgs em;               // levels, prior, margins, view order, shape; em.mu_T, em.q, em.d_idx
    const uint8_t *views;    // [K][H][W][3]
    const float *S_P;        // [K][H][W]
    float *rgb;              // [H][W][3]
    float *q_out;            // [K][H][W] caller's copy of the weights (device), or null
    uint32_t *bad;           // count of invalid input values (checked inputs), or null
    int warm;                // em.q holds the stream's previous weights (the first weights)
    int check;               // count S_P outside [0,1] and mu_T not finite into *bad
    int ref, tiles_x, tile_start, n_tiles;
    int rows_in_place;       // stage each view's R+G+B rows inside its record window (else after the records)
    float tau;
};

template <int K, int ST, int KIND>
__device__ __forceinline__ void serve_tile(const ServeJob &job, int tile, unsigned char *lds) {
    constexpr bool FRAC = KIND == kServeFrac;
    constexpr bool SYM = KIND == kServeSharedSym;
    constexpr int RS = serve_rec_format<ST>();
    using R = typename Rec<RS>::T;
    const EmArgs &a = job.em;
    const int tid = threadIdx.x;
    const int y = tile / job.tiles_x;
    constexpr int TILE = serve_tile_width(K);
    const int x0 = (tile - y * job.tiles_x) * TILE;
    const int x = x0 + tid;
    const int W = a.W, H = a.H;
    const bool active = x < W;
    const size_t HW = (size_t)H * W;
    const size_t pix = (size_t)y * W + (active ? x : 0);

    Window w[K];
    int total;
    view_windows<K, FRAC>(a, x0, TILE, w, total);
    R *win = reinterpret_cast<R *>(lds);
    // rows of windows too wide to stage in place: after the records
    int16_t *scratch_rows = reinterpret_cast<int16_t *>(lds + (size_t)total * sizeof(R));

    // descriptor records of every window position (replicated border), view
    // by view: rows y-1, y, y+1 of R+G+B over the window's columns (+1
    // border), then the 3x3 Sobel responses.  The rows take 6 (len + 2)
    // bytes, the window's records 8 len (len >= the tile width), so a
    // window holds its own rows while its records wait in registers.
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int ulo = clampi(w[k].umin, 0, W - 1), uhi = clampi(w[k].umin + w[k].len - 1, 0, W - 1);
        const int c0 = max(ulo - 1, 0);
        const int nc = min(uhi + 1, W - 1) - c0 + 1;
        const bool in_place = job.rows_in_place && w[k].len <= kServeHold * TILE;   // uniform
        int16_t *lsum = in_place ? reinterpret_cast<int16_t *>(win + w[k].off) : scratch_rows;
        const uint8_t *v = job.views + (size_t)a.perm[k] * HW * 3;
        for (int i = tid; i < 3 * nc; i += TILE) {
            const int r = i / nc, c = c0 + (i - r * nc);
            const int yy = clampi(y + r - 1, 0, H - 1);
            const uint8_t *px = v + ((size_t)yy * W + c) * 3;
            lsum[i] = (int16_t)((int)px[0] + (int)px[1] + (int)px[2]);
        }
        __syncthreads();
        const int16_t *L0 = lsum, *L1 = L0 + nc, *L2 = L1 + nc;
        auto record = [&](int p) {
            const int uc = clampi(w[k].umin + p, 0, W - 1);
            const int cl = max(uc - 1, 0) - c0, cm = uc - c0, cr = min(uc + 1, W - 1) - c0;
            const int gx = (L0[cr] - L0[cl]) + 2 * (L1[cr] - L1[cl]) + (L2[cr] - L2[cl]);
            const int gy = (L2[cl] - L0[cl]) + 2 * (L2[cm] - L0[cm]) + (L2[cr] - L0[cr]);
            return serve_rec<ST>(gx, gy);
        };
        if (in_place) {
            R hold[kServeHold];
#pragma unroll
            for (int i = 0; i < kServeHold; ++i) {
                const int p = tid + i * TILE;
                if (p < w[k].len) hold[i] = record(p);
            }
            __syncthreads();   // every lane has read the rows before they are overwritten
#pragma unroll
            for (int i = 0; i < kServeHold; ++i) {
                const int p = tid + i * TILE;
                if (p < w[k].len) win[win_index(w[k], p)] = hold[i];
            }
        } else {
            for (int p = tid; p < w[k].len; p += TILE) win[win_index(w[k], p)] = record(p);
        }
        __syncthreads();
    }

    // 3) ray prior and first weights of each of the pixel's rays
    Lane<K> s;
    s.mu = 0.0f;
    s.L = 0.0f;
    s.best_j = 0;
    s.c = 0;
    s.f0 = make_float2(0.0f, 0.0f);
    s.n0 = 0.0f;
    bool work = active;   // pixel reconstructed (all of them unless dynamic-only)
    if (active) {
        s.mu = a.mu_T[pix];
        uint32_t nbad = job.check ? !(fabsf(s.mu) <= 1e6f) : 0u;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const size_t row = ((size_t)a.perm[k] * H + y) * W;
            float r, om;
            ray_prior_value(job.S_P + row, W, x, a.b[k], s.mu, ST, r, om);
            s.la[k] = (r > 0.0f ? logf(r) : -INFINITY) + a.lambda;
            s.lb[k] = (om > 0.0f ? logf(om) : -INFINITY);
            s.q[k] = job.warm ? a.q[row + x] : ((r >= job.tau) ? 1.0f : 0.0f);
            if (k == 0 && a.dyn_only) work = r < job.tau;    // kernel view 0 is the reference
            if (job.check) {
                const float sv = job.S_P[row + x];
                nbad += !(sv >= 0.0f && sv <= 1.0f);
            }
        }
        if (nbad) atomicAdd(job.bad, nbad);
        s.c = nearest_level(a, s.mu);
        s.best_j = s.c;
#pragma unroll
        for (int k = 0; k < K; ++k) s.idx0[k] = FRAC ? 0 : lane_index0(w[k], a.bi[k], a.dmin_i, x);
        fetch<K, RS, FRAC>(win, w[0], a, 0, x, 0, s.idx0[0], s.f0, s.n0);
    } else {
#pragma unroll
        for (int k = 0; k < K; ++k) s.q[k] = s.la[k] = s.lb[k] = 0.0f;
    }

    // 4) EM iterations: the plain context's sweeps (the same bits)
    const float Pc = kLn2 * __builtin_amdgcn_logf(a.gamma);
    int jlo, jhi, slo, shi;
    prior_window(a, work, s.mu, jlo, jhi);
    search_range(a, work, s.mu, slo, shi);
    for (int it = 0; it < a.n_iters; ++it) {
        if constexpr (KIND == kServeSharedSym || KIND == kServeShared) {
            (void)shared_iteration<K, RS, SYM>(win, w, a, x, x0, work, jlo, jhi, slo, shi, Pc, s, false);
        } else {
            if (work) em_iteration<K, RS, FRAC, false, false>(win, w, a, x, jlo, jhi, slo, shi, Pc, s, false);
        }
    }

    // 5) outputs: weights, level, refocus of the static rays
    if (active) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const size_t i = (size_t)a.perm[k] * HW + pix;
            a.q[i] = s.q[k];
            if (job.q_out) job.q_out[i] = s.q[k];
        }
        a.d_idx[pix] = s.best_j;
        float acc[3] = {0.0f, 0.0f, 0.0f};
        int n = 0;
        if (!FRAC) {
            int iacc[3] = {0, 0, 0};
            const int d = a.dmin_i + s.best_j * a.dstep_i;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (!(s.q[k] >= 0.5f)) continue;
                const int u = clampi(x - a.bi[k] * d, 0, W - 1);
                const uint8_t *px = job.views + (((size_t)a.perm[k] * H + y) * W + u) * 3;
                iacc[0] += px[0];
                iacc[1] += px[1];
                iacc[2] += px[2];
                ++n;
            }
            acc[0] = (float)iacc[0];
            acc[1] = (float)iacc[1];
            acc[2] = (float)iacc[2];
        } else {
            const float d = fmaf((float)s.best_j, a.d_step, a.d_min);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (!(s.q[k] >= 0.5f)) continue;
                int i0;
                float t, omt;
                footprint_precise(x, a.b[k], d, i0, t, omt);
                const uint8_t *r = job.views + ((size_t)a.perm[k] * H + y) * W * 3;
                const uint8_t *p0 = r + (size_t)clampi(i0, 0, W - 1) * 3;
                const uint8_t *p1 = r + (size_t)clampi(i0 + 1, 0, W - 1) * 3;
#pragma unroll
                for (int c = 0; c < 3; ++c) acc[c] += lerp((float)p0[c], (float)p1[c], t);
                ++n;
            }
        }
        float *o = job.rgb + pix * 3;
        if (!work || n == 0) {
            // a static reference ray (dynamic-only) or no static ray at all:
            // the reference pixel itself
            const uint8_t *c_ref = job.views + (((size_t)job.ref * H + y) * W + x) * 3;
#pragma unroll
            for (int c = 0; c < 3; ++c) o[c] = (float)c_ref[c] / 255.0f;
        } else {
            const float den = 255.0f * (float)n;
#pragma unroll
            for (int c = 0; c < 3; ++c) o[c] = acc[c] / den;
        }
    }
}

template <int K, int ST, int KIND>
__device__ __forceinline__ void serve_entry(const ServeJob *__restrict__ jobs, int n_jobs) {
    extern __shared__ __align__(16) unsigned char lds[];
    int j = 0;
    while (j + 1 < n_jobs && (int)blockIdx.x >= jobs[j + 1].tile_start) ++j;
    j = __builtin_amdgcn_readfirstlane(j);
    const ServeJob &job = jobs[j];
    // a frame's blocks start at a multiple of 8 (the blocks past its tiles
    // are padding); as in the plain EM launch, all tiles of a row go to one
    // XCD (block b to XCD b % 8), so that neighbouring tiles share their
    // halo in that XCD's L2; rows past the last whole group of 8 keep the
    // grid order
    const int local = (int)blockIdx.x - job.tile_start;
    if (local >= job.n_tiles) return;
    const int gx = job.tiles_x;
    int t = local;
    if (local < (job.n_tiles / gx / 8) * 8 * gx) {
        const int k = local >> 3;
        t = ((local & 7) + 8 * (k / gx)) * gx + k % gx;
    }
    serve_tile<K, ST, KIND>(job, t, lds);
}

// Register budgets as the plain context's instances: the shared sweep at
// three waves per SIMD up to six views and the compiler's own count above;
// the per-lane sweep at five (up to five FP16/BF16 views), four (up to six)
// or three waves (up to nine).
template <int K, int ST, int KIND>
__global__ __launch_bounds__(kServeTileMax) void lf_serve_kernel(const ServeJob *__restrict__ jobs, int n_jobs) {
    serve_entry<K, ST, KIND>(jobs, n_jobs);
}
template <int K, int ST, int KIND>
__global__ __launch_bounds__(kServeTileMax) __attribute__((amdgpu_waves_per_eu(5, 8))) void lf_serve_kernel_w5(
    const ServeJob *__restrict__ jobs, int n_jobs) {
    serve_entry<K, ST, KIND>(jobs, n_jobs);
}
template <int K, int ST, int KIND>
__global__ __launch_bounds__(kServeTileMax) __attribute__((amdgpu_waves_per_eu(4, 8))) void lf_serve_kernel_w4(
    const ServeJob *__restrict__ jobs, int n_jobs) {
    serve_entry<K, ST, KIND>(jobs, n_jobs);
}
template <int K, int ST, int KIND>
__global__ __launch_bounds__(kServeTileMax) __attribute__((amdgpu_waves_per_eu(3, 8))) void lf_serve_kernel_w3(
    const ServeJob *__restrict__ jobs, int n_jobs) {
    serve_entry<K, ST, KIND>(jobs, n_jobs);
}

using ServeKernel = void (*)(const ServeJob *, int);

template <int K, int ST, int KIND>
ServeKernel serve_instance() {
    if constexpr (KIND == kServeSharedSym || KIND == kServeShared) {
        if constexpr (K <= 6) return lf_serve_kernel_w3<K, ST, KIND>;
        else return lf_serve_kernel<K, ST, KIND>;
    } else {
        if constexpr (K <= 5 && ST != 0) return lf_serve_kernel_w5<K, ST, KIND>;
        else if constexpr (K <= 6) return lf_serve_kernel_w4<K, ST, KIND>;
        else return lf_serve_kernel_w3<K, ST, KIND>;
    }
}

// The instance of view count K in [KLO, KHI] (nullptr outside it).
template <int ST, int KLO, int KHI>
ServeKernel pick_serve_range(int K, int kind) {
    if constexpr (KLO > KHI) {
        return nullptr;
    } else {
        if (K == KLO) {
            switch (kind) {
                case kServeSharedSym: return serve_instance<KLO, ST, kServeSharedSym>();
                case kServeShared: return serve_instance<KLO, ST, kServeShared>();
                case kServeLane: return serve_instance<KLO, ST, kServeLane>();
                default: return serve_instance<KLO, ST, kServeFrac>();
            }
        }
        return pick_serve_range<ST, KLO + 1, KHI>(K, kind);
    }
}

}  // namespace lfem
