// Construction of the disparity prior mu_T (Sec. III-C, disparity prior):
// support points matched along the epipolar line over the full disparity
// range, those on dynamic objects dropped, support points of the other views
// transferred into the part of the reference occluded by dynamic objects,
// duplicates and inconsistent points removed, and mu_T interpolated
// piecewise-linearly over a Delaunay triangulation of the points.
//
// Device: integer Sobel responses, the matching of every grid point of every
// pass (one lane per point, all levels), the transfer of the other views'
// points with one point per reference pixel, the consistency filter, the
// ordering of the points by (y, u), the Delaunay triangulation (row strips
// and side pockets, then rounds of parallel edge flips) and its raster.
// Host (native C++): the four corners (nearest point of each), the rows'
// bounds, and the incremental Delaunay triangulation behind lf_triangulate
// (also the fallback should the flip rounds not settle).
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <vector>

#include "lf_delaunay.h"
#include "lf_em.h"
#include "lf_internal.h"

namespace lfem {

#define LF_HIP(call, what)                                 \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return hip_error(e_, what);  \
    } while (0)

__device__ __forceinline__ int pclamp(int v, int lo, int hi) { return min(max(v, lo), hi); }

// Flip rounds of the device triangulation before the host takes over (every
// round flips at least one edge; the scenes here settle in 5 to 25).
constexpr int kMaxFlipRounds = 4096;
// Flip rounds queued between two reads of the illegal-edge count.
constexpr int kRoundsPerCheck = 8;

// Integer Sobel responses (Gx, Gy) of L = R+G+B, replicated border.
// grid (ceil(W/256), H, K); g is [K][H][W].
__global__ __launch_bounds__(256) void lf_sobel_i16_kernel(const uint8_t *__restrict__ views, short2 *__restrict__ g,
                                                           int H, int W) {
    const int k = blockIdx.z, y = blockIdx.y;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= W) return;
    const uint8_t *v = views + (size_t)k * H * W * 3;
    int L[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const int yy = pclamp(y + r - 1, 0, H - 1);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const uint8_t *px = v + ((size_t)yy * W + pclamp(x + c - 1, 0, W - 1)) * 3;
            L[r][c] = (int)px[0] + (int)px[1] + (int)px[2];
        }
    }
    const int gx = (L[0][2] - L[0][0]) + 2 * (L[1][2] - L[1][0]) + (L[2][2] - L[2][0]);
    const int gy = (L[2][0] - L[0][0]) + 2 * (L[2][1] - L[0][1]) + (L[2][2] - L[0][2]);
    g[((size_t)k * H + y) * W + x] = make_short2((short)gx, (short)gy);
}

// One matching pass: grid points of view a against the views vs[].
struct MatchArgs {
    const short2 *g;     // [K][H][W]
    const float *S_P;    // [K][H][W]
    int32_t *level;      // [ny][nx] level of the unique best match, or -1
    int H, W, D, a, n_vs, nx, ny;
    int step, radius, texture_min, ratio_num, ratio_den, static_min;
    int dmin_i, dstep_i;
    float tau;
    int vs[LF_MAX_VIEWS];
    int db[LF_MAX_VIEWS];     // integer baseline of vs[i] minus that of a
    int side[LF_MAX_VIEWS];   // 1 when vs[i] lies right of a (larger baseline)
    int two_sides;            // views on both sides: the cost is the smaller side sum
};

// grid (ceil(nx*ny/128)), block 128; one lane per grid point.
__global__ __launch_bounds__(128) void lf_support_match_kernel(MatchArgs m) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m.nx * m.ny) return;
    const int ix = i % m.nx, iy = i / m.nx;
    const int x = m.step / 2 + ix * m.step, y = m.step / 2 + iy * m.step;
    const int H = m.H, W = m.W, r = m.radius;
    const size_t HW = (size_t)H * W;
    int j_out = -1;
    // static point with enough static pixels in its window
    const float *sp = m.S_P + (size_t)m.a * HW;
    bool ok = sp[(size_t)y * W + x] >= m.tau;
    if (ok) {
        int n_static = 0;
        for (int dy = -r; dy <= r; ++dy)
            for (int dx = -r; dx <= r; ++dx)
                n_static += sp[(size_t)pclamp(y + dy, 0, H - 1) * W + pclamp(x + dx, 0, W - 1)] >= m.tau;
        ok = n_static >= m.static_min;
    }
    const short2 *ga = m.g + (size_t)m.a * HW;
    if (ok) {
        long texture = 0;
        for (int dy = -r; dy <= r; ++dy)
            for (int dx = -r; dx <= r; ++dx) {
                const short2 v = ga[(size_t)pclamp(y + dy, 0, H - 1) * W + pclamp(x + dx, 0, W - 1)];
                texture += abs((int)v.x) + abs((int)v.y);
            }
        ok = texture >= m.texture_min;
    }
    if (ok) {
        // the four lowest (cost, level) pairs in lexicographic order: the
        // best, at most two levels next to it, and the best level further away
        long tc[4] = {LONG_MAX, LONG_MAX, LONG_MAX, LONG_MAX};
        int tj[4] = {INT_MAX, INT_MAX, INT_MAX, INT_MAX};
        for (int j = 0; j < m.D; ++j) {
            const int d = m.dmin_i + j * m.dstep_i;
            long s[2] = {0, 0};
            for (int t = 0; t < m.n_vs; ++t) {
                const short2 *gv = m.g + (size_t)m.vs[t] * HW;
                const int shift = m.db[t] * d;
                long c = 0;
                for (int dy = -r; dy <= r; ++dy) {
                    const size_t row = (size_t)pclamp(y + dy, 0, H - 1) * W;
                    for (int dx = -r; dx <= r; ++dx) {
                        const short2 A = ga[row + pclamp(x + dx, 0, W - 1)];
                        const short2 B = gv[row + pclamp(x + dx - shift, 0, W - 1)];
                        c += abs((int)A.x - (int)B.x) + abs((int)A.y - (int)B.y);
                    }
                }
                s[m.side[t]] += c;
            }
            const long cost = m.two_sides ? min(s[0], s[1]) : s[0] + s[1];
            // insert (cost, j); j increases, so a tie in cost keeps the earlier level first
            int pos = 4;
            while (pos > 0 && cost < tc[pos - 1]) --pos;
            if (pos < 4) {
                for (int q = 3; q > pos; --q) {
                    tc[q] = tc[q - 1];
                    tj[q] = tj[q - 1];
                }
                tc[pos] = cost;
                tj[pos] = j;
            }
        }
        const int best = tj[0];
        long second = -1;
        for (int q = 1; q < 4; ++q)
            if (tj[q] != INT_MAX && abs(tj[q] - best) >= 2) {
                second = tc[q];
                break;
            }
        const bool unique = second >= 0 ? tc[0] * m.ratio_den < second * m.ratio_num : true;
        if (unique) j_out = best;
    }
    m.level[i] = j_out;
}

// ---------------------------------------------------------------------------
// Candidate points.  Every point lies on a grid row (y = step/2 + iy * step):
// the reference's points at their grid column, the other views' points
// moved along the row.  Per-row maps [ny][W] hold each reference pixel's
// candidate (level, or -1, and view); no pixel holds two, since reference
// points need S_P_ref >= tau and moved points S_P_ref < tau, and moved points
// that land on one pixel keep the first (lowest pass, i.e. view, then grid
// order): the smallest key pass * n_grid + grid index claims the pixel.
// ---------------------------------------------------------------------------
struct CandArgs {
    const int32_t *lev;       // [n_pass][n_grid] matched level or -1
    const float *sp_ref;      // S_P of the reference view [H][W]
    unsigned long long *claim;  // [ny][W] smallest key of a point moved there
    int32_t *level;           // [ny][W] candidate level or -1
    int32_t *view;            // [ny][W] candidate's view
    int W, nx, ny, step, n_grid, dmin_i, dstep_i;
    float tau;
    int pass_view[LF_MAX_VIEWS];   // view of each pass (pass 0: the reference)
    int pass_bi[LF_MAX_VIEWS];     // its integer baseline
};

// grid (ceil(n_grid/256)), block 256: the reference's points (pass 0)
__global__ __launch_bounds__(256) void lf_cand_ref_kernel(CandArgs c) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= c.n_grid) return;
    const int j = c.lev[i];
    if (j < 0) return;
    const int ix = i % c.nx, iy = i / c.nx;
    const size_t m = (size_t)iy * c.W + c.step / 2 + ix * c.step;
    c.level[m] = j;
    c.view[m] = c.pass_view[0];
}

// The reference pixel a point of pass ps >= 1 moves to, or -1: inside the
// frame and dynamic in the reference (S_P_ref < tau).
__device__ __forceinline__ long moved_pixel(const CandArgs &c, int ps, int i, int &j) {
    j = c.lev[(size_t)ps * c.n_grid + i];
    if (j < 0) return -1;
    const int ix = i % c.nx, iy = i / c.nx;
    const int x = c.step / 2 + ix * c.step, y = c.step / 2 + iy * c.step;
    const long u = (long)x + (long)c.pass_bi[ps] * ((long)c.dmin_i + (long)j * c.dstep_i);
    if (u < 0 || u >= c.W) return -1;
    if (!(c.sp_ref[(size_t)y * c.W + u] < c.tau)) return -1;
    return (long)iy * c.W + u;
}

// grid (ceil(n_grid/256), n_pass - 1), block 256
__global__ __launch_bounds__(256) void lf_cand_claim_kernel(CandArgs c) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x, ps = blockIdx.y + 1;
    if (i >= c.n_grid) return;
    int j;
    const long m = moved_pixel(c, ps, i, j);
    if (m >= 0) atomicMin(&c.claim[m], (unsigned long long)ps * c.n_grid + i);
}

// grid as lf_cand_claim_kernel, after it
__global__ __launch_bounds__(256) void lf_cand_moved_kernel(CandArgs c) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x, ps = blockIdx.y + 1;
    if (i >= c.n_grid) return;
    int j;
    const long m = moved_pixel(c, ps, i, j);
    if (m >= 0 && c.claim[m] == (unsigned long long)ps * c.n_grid + i) {
        c.level[m] = j;
        c.view[m] = c.pass_view[ps];
    }
}

// Ordered compaction of a per-row map's entries (level >= 0) into points
// (u, y, level, view), by row then column.  grid (ny), block 256: the count
// of each row.
__global__ __launch_bounds__(256) void lf_row_count_kernel(const int32_t *__restrict__ level, int W,
                                                           int32_t *__restrict__ row_n) {
    __shared__ int part[4];
    const int iy = blockIdx.x, t = threadIdx.x;
    int n = 0;
    for (int x = t; x < W; x += 256) n += level[(size_t)iy * W + x] >= 0;
    part[t >> 6] = 0;
    __syncthreads();
    atomicAdd(&part[t >> 6], n);
    __syncthreads();
    if (t == 0) row_n[iy] = part[0] + part[1] + part[2] + part[3];
}

// One block: row_start[iy] = sum of row_n[0 .. iy), row_start[ny] the total.
__global__ __launch_bounds__(1024) void lf_row_scan_kernel(const int32_t *__restrict__ row_n, int ny,
                                                           int32_t *__restrict__ row_start) {
    __shared__ int part[1024];
    const int t = threadIdx.x, per = (ny + 1023) / 1024;
    const int beg = min(t * per, ny), end = min(beg + per, ny);
    int sum = 0;
    for (int i = beg; i < end; ++i) sum += row_n[i];
    part[t] = sum;
    __syncthreads();
    if (t == 0) {
        int acc = 0;
        for (int i = 0; i < 1024; ++i) {
            const int v = part[i];
            part[i] = acc;
            acc += v;
        }
        row_start[ny] = acc;
    }
    __syncthreads();
    int off = part[t];
    for (int i = beg; i < end; ++i) {
        row_start[i] = off;
        off += row_n[i];
    }
}

// grid (ny), block 256: each row's entries in column order from row_start.
__global__ __launch_bounds__(256) void lf_row_write_kernel(const int32_t *__restrict__ level,
                                                           const int32_t *__restrict__ view, int W, int step,
                                                           const int32_t *__restrict__ row_start,
                                                           int4 *__restrict__ out) {
    __shared__ int part[4];
    const int iy = blockIdx.x, t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int y = step / 2 + iy * step;
    int base = row_start[iy];
    for (int x0 = 0; x0 < W; x0 += 256) {
        const int x = x0 + t;
        const size_t m = (size_t)iy * W + x;
        const bool on = x < W && level[m] >= 0;
        const uint64_t b = __ballot(on);
        if (lane == 0) part[wv] = __popcll(b);
        __syncthreads();
        int before = 0, total = 0;
        for (int k = 0; k < 4; ++k) {
            before += k < wv ? part[k] : 0;
            total += part[k];
        }
        if (on) out[base + before + __popcll(b & ((1ull << lane) - 1ull))] = make_int4(x, y, level[m], view[m]);
        base += total;
        __syncthreads();
    }
}

// Consistency (one lane per candidate, candidates ordered by row then
// column): a candidate is kept with at least incon_min other candidates
// within R pixels in x and y and incon_levels levels.  The kept ones go to
// the per-row map `kept` (level, else -1).  grid (ceil(cap/256)); lanes past
// the number of candidates exit.
__global__ __launch_bounds__(256) void lf_consistency_kernel(const int4 *__restrict__ cand,
                                                             const int32_t *__restrict__ row_start, int ny, int W,
                                                             int step, int R, int L, int n_min,
                                                             int32_t *__restrict__ kept) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= row_start[ny]) return;
    const int4 c = cand[i];
    const int iy = (c.y - step / 2) / step;
    int cnt = 0;
    const int r_rows = R / step;
    for (int iy2 = max(iy - r_rows, 0); iy2 <= min(iy + r_rows, ny - 1) && cnt < n_min; ++iy2) {
        // first candidate of the row with u >= c.x - R
        int lo = row_start[iy2], hi = row_start[iy2 + 1];
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (cand[mid].x < c.x - R) lo = mid + 1;
            else hi = mid;
        }
        for (int k = lo; k < row_start[iy2 + 1] && cand[k].x <= c.x + R && cnt < n_min; ++k)
            cnt += k != i && abs(cand[k].z - c.z) <= L;
    }
    if (cnt >= n_min) kept[(size_t)iy * W + c.x] = c.z;
}

// ---------------------------------------------------------------------------
// Delaunay triangulation on the device (see lf_delaunay.h).  Points P in
// their output order; `order` lists them by (y, x) and row_start bounds the
// rows in it.
// ---------------------------------------------------------------------------

// One lane per strip between rows s and s + 1; the strips' triangles are
// stored in row order: strip s starts at sum over s' < s of
// (n_s' + n_s'+1 - 2) = row_start[s] + row_start[s+1] - row_start[1] - 2 s.
__global__ __launch_bounds__(64) void lf_dt_strips_kernel(const dt::Pt *__restrict__ P, const int *__restrict__ order,
                                                          const int *__restrict__ row_start, int n_rows,
                                                          int3 *__restrict__ tris) {
    const int st = blockIdx.x * blockDim.x + threadIdx.x;
    if (st >= n_rows - 1) return;
    int k = row_start[st] + row_start[st + 1] - row_start[1] - 2 * st;
    dt::zip_strip(P, order + row_start[st], row_start[st + 1] - row_start[st], order + row_start[st + 1],
                  row_start[st + 2] - row_start[st + 1], [&](int a, int b, int c) { tris[k++] = make_int3(a, b, c); });
}

// One lane: the left and the right side pocket after the strips (from
// `base`), at most `cap` triangles in all; the count goes to *n_out.  `work`
// holds 4 n_rows ints.
__global__ __launch_bounds__(64) void lf_dt_pockets_kernel(const dt::Pt *__restrict__ P, const int *__restrict__ order,
                                                           const int *__restrict__ row_start, int n_rows, int W,
                                                           int *__restrict__ work, int3 *__restrict__ tris, int base,
                                                           int cap, int *__restrict__ n_out) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int k = base;
    int *C = work;
    auto emit = [&](int a, int b, int c) {
        if (k < cap) tris[k] = make_int3(a, b, c);
        ++k;
    };
    for (int r = 0; r < n_rows; ++r) C[r] = order[row_start[r]];
    dt::side_pocket(P, C, n_rows, 0, -1, work + n_rows, emit);
    for (int r = 0; r < n_rows; ++r) C[r] = order[row_start[r + 1] - 1];
    dt::side_pocket(P, C, n_rows, W - 1, 1, work + n_rows, emit);
    *n_out = k;
}

// Flip rounds.  Edge e of triangle t (the edge opposite its vertex e) has the
// key min * n + max of its end points and the value 3 t + e; after sorting by
// key the two sides of an interior edge are neighbours.
__device__ __forceinline__ int tri_vertex(const int3 &v, int e) { return e == 0 ? v.x : (e == 1 ? v.y : v.z); }

__global__ __launch_bounds__(256) void lf_dt_edges_kernel(const int3 *__restrict__ tris, int T, int n,
                                                          unsigned long long *__restrict__ keys,
                                                          int *__restrict__ vals) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 3 * T) return;
    const int3 v = tris[i / 3];
    const int e = i % 3;
    const int a = tri_vertex(v, (e + 1) % 3), b = tri_vertex(v, (e + 2) % 3);
    keys[i] = (unsigned long long)min(a, b) * (unsigned long long)n + (unsigned long long)max(a, b);
    vals[i] = i;
}

// Neighbour links: after sorting the edges by key, the two sides of an
// interior edge are neighbours; nb[3 t + e] = 3 u + f links edge e of t
// with edge f of u (-1: an edge of the hull).
__global__ __launch_bounds__(256) void lf_dt_links_kernel(const unsigned long long *__restrict__ keys,
                                                          const int *__restrict__ vals, int m,
                                                          int *__restrict__ nb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m - 1 || keys[i] != keys[i + 1]) return;
    nb[vals[i]] = vals[i + 1];
    nb[vals[i + 1]] = vals[i];
}

// The triangles a flip of edge te rewrites: its two triangles and their four
// outer neighbours (-1 where the outer edge is on the hull).
__device__ __forceinline__ void flip_parts(const int *nb, int te, int other, int (&tri)[6]) {
    const int t = te / 3, e = te % 3, u = other / 3, f = other % 3;
    tri[0] = t;
    tri[1] = u;
    const int o[4] = {nb[3 * t + (e + 1) % 3], nb[3 * t + (e + 2) % 3], nb[3 * u + (f + 1) % 3],
                      nb[3 * u + (f + 2) % 3]};
#pragma unroll
    for (int k = 0; k < 4; ++k) tri[2 + k] = o[k] < 0 ? -1 : o[k] / 3;
}

// One round, part 1 (one lane per edge slot, each interior edge taken from
// its lower slot): an edge whose opposite vertex across it lies strictly
// inside its triangle's circumcircle is illegal; it claims, by an atomic
// minimum of its slot, the six triangles its flip rewrites.  The lowest
// illegal edge wins all of its claims, so every round flips at least one
// edge, and the flips that win theirs touch disjoint triangles.
__global__ __launch_bounds__(256) void lf_dt_mark_kernel(const int3 *__restrict__ tris, const dt::Pt *__restrict__ P,
                                                         const int *__restrict__ nb, int m,
                                                         int *__restrict__ claim, uint8_t *__restrict__ flag,
                                                         int *__restrict__ count) {
    const int te = blockIdx.x * blockDim.x + threadIdx.x;
    if (te >= m) return;
    flag[te] = 0;
    const int other = nb[te];
    if (other < te) return;   // a hull edge (-1), or taken from the other side
    const int t = te / 3, u = other / 3, f = other % 3;
    const int3 vt = tris[t];
    const int d = tri_vertex(tris[u], f);
    if (dt::incircle(P[vt.x], P[vt.y], P[vt.z], P[d]) <= 0) return;
    flag[te] = 1;
    atomicAdd(count, 1);
    int tri[6];
    flip_parts(nb, te, other, tri);
#pragma unroll
    for (int k = 0; k < 6; ++k)
        if (tri[k] >= 0) atomicMin(&claim[tri[k]], te);
}

// Part 2: the edges that won all their claims flip.  Edge (b, c) of
// t = (a, b, c) and u = (d, c, b) becomes (a, d): t = (a, b, d) and
// u = (a, d, c), both with positive orientation (an illegal edge's
// quadrilateral is convex), and the links of the six triangles follow.
__global__ __launch_bounds__(256) void lf_dt_flip_kernel(int3 *__restrict__ tris, int *__restrict__ nb,
                                                         const uint8_t *__restrict__ flag,
                                                         const int *__restrict__ claim, int m) {
    const int te = blockIdx.x * blockDim.x + threadIdx.x;
    if (te >= m || !flag[te]) return;
    const int other = nb[te];
    int tri[6];
    flip_parts(nb, te, other, tri);
#pragma unroll
    for (int k = 0; k < 6; ++k)
        if (tri[k] >= 0 && claim[tri[k]] != te) return;
    const int t = te / 3, e = te % 3, u = other / 3, f = other % 3;
    const int3 vt = tris[t];
    const int a = tri_vertex(vt, e), b = tri_vertex(vt, (e + 1) % 3), c = tri_vertex(vt, (e + 2) % 3);
    const int d = tri_vertex(tris[u], f);
    // outer neighbours: across (c, a) and (a, b) of t, (b, d) and (d, c) of u
    const int n_ca = nb[3 * t + (e + 1) % 3], n_ab = nb[3 * t + (e + 2) % 3];
    const int n_bd = nb[3 * u + (f + 1) % 3], n_dc = nb[3 * u + (f + 2) % 3];
    tris[t] = make_int3(a, b, d);   // edges: 0 (b, d), 1 (d, a), 2 (a, b)
    tris[u] = make_int3(a, d, c);   // edges: 0 (d, c), 1 (c, a), 2 (a, d)
    nb[3 * t + 0] = n_bd;
    nb[3 * t + 1] = 3 * u + 2;
    nb[3 * t + 2] = n_ab;
    nb[3 * u + 0] = n_dc;
    nb[3 * u + 1] = n_ca;
    nb[3 * u + 2] = 3 * t + 1;
    if (n_bd >= 0) nb[n_bd] = 3 * t + 0;
    if (n_ab >= 0) nb[n_ab] = 3 * t + 2;
    if (n_dc >= 0) nb[n_dc] = 3 * u + 0;
    if (n_ca >= 0) nb[n_ca] = 3 * u + 1;
}

// Raster of the triangulation: the lowest-index triangle containing each
// pixel (edges included), found with an atomic min so the result does not
// depend on the order of arrival.  grid (n_tri), block 256.
__global__ __launch_bounds__(256) void lf_prior_cover_kernel(const int4 *__restrict__ pts, const int3 *__restrict__ tris,
                                                             int n_tri, int32_t *__restrict__ owner, int H, int W) {
    const int t = blockIdx.x;
    if (t >= n_tri) return;
    const int3 tr = tris[t];
    const int4 a = pts[tr.x], b = pts[tr.y], c = pts[tr.z];
    const long A = (long)(b.x - a.x) * (c.y - a.y) - (long)(b.y - a.y) * (c.x - a.x);
    if (A == 0) return;
    const int x0 = max(min(a.x, min(b.x, c.x)), 0), x1 = min(max(a.x, max(b.x, c.x)), W - 1);
    const int y0 = max(min(a.y, min(b.y, c.y)), 0), y1 = min(max(a.y, max(b.y, c.y)), H - 1);
    const int bw = x1 - x0 + 1;
    const long n = (long)bw * (y1 - y0 + 1);
    for (long i = threadIdx.x; i < n; i += blockDim.x) {
        const int x = x0 + (int)(i % bw), y = y0 + (int)(i / bw);
        const long wa = (long)(b.x - x) * (c.y - y) - (long)(b.y - y) * (c.x - x);
        const long wb = (long)(c.x - x) * (a.y - y) - (long)(c.y - y) * (a.x - x);
        const long wc = (long)(a.x - x) * (b.y - y) - (long)(a.y - y) * (b.x - x);
        const bool inside = A > 0 ? (wa >= 0 && wb >= 0 && wc >= 0) : (wa <= 0 && wb <= 0 && wc <= 0);
        if (inside) atomicMin(&owner[(size_t)y * W + x], t);
    }
}

// mu_T of every pixel: barycentric interpolation in its triangle, in double
// with the interpolation written out in a fixed order (no contraction), or
// the level of the nearest point when no triangle covers it.  grid
// (ceil(W/256), H).
__global__ __launch_bounds__(256) void lf_prior_interp_kernel(const int4 *__restrict__ pts, int n_pts,
                                                              const int3 *__restrict__ tris,
                                                              const int32_t *__restrict__ owner, float *__restrict__ mu,
                                                              int H, int W, int D, double d_min, double d_step) {
#pragma clang fp contract(off)
    const int y = blockIdx.y;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= W) return;
    const int t = owner[(size_t)y * W + x];
    double v;
    if (t != INT_MAX) {
        const int3 tr = tris[t];
        const int4 a = pts[tr.x], b = pts[tr.y], c = pts[tr.z];
        const long A = (long)(b.x - a.x) * (c.y - a.y) - (long)(b.y - a.y) * (c.x - a.x);
        const long wa = (long)(b.x - x) * (c.y - y) - (long)(b.y - y) * (c.x - x);
        const long wb = (long)(c.x - x) * (a.y - y) - (long)(c.y - y) * (a.x - x);
        const long wc = (long)(a.x - x) * (b.y - y) - (long)(a.y - y) * (b.x - x);
        const double da = d_min + a.z * d_step, db = d_min + b.z * d_step, dc = d_min + c.z * d_step;
        const double s1 = (double)wa * da;
        const double s2 = (double)wb * db;
        const double s3 = (double)wc * dc;
        v = ((s1 + s2) + s3) / (double)A;
    } else if (n_pts == 0) {
        v = d_min + 0.5 * (D - 1) * d_step;
    } else {
        long best = -1;
        int lev = 0;
        for (int i = 0; i < n_pts; ++i) {
            const long dx = pts[i].x - x, dy = pts[i].y - y, d2 = dx * dx + dy * dy;
            if (best < 0 || d2 < best) {
                best = d2;
                lev = pts[i].z;
            }
        }
        v = d_min + lev * d_step;
    }
    mu[(size_t)y * W + x] = (float)v;
}

__global__ __launch_bounds__(256) void lf_prior_fill_kernel(int32_t *p, size_t n, int32_t v) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// Delaunay triangulation (incremental, Bowyer-Watson) with exact predicates on
// integer coordinates.  Three far vertices enclose the frame; triangles that
// use them are dropped at the end.  For frames up to 16384 pixels on a side
// the far vertices are far enough that every edge of the convex hull of the
// points is an edge of the result.
// ---------------------------------------------------------------------------
namespace {

struct P2 {
    long x, y;
};

inline long orient(const P2 &a, const P2 &b, const P2 &c) {
    return (b.x - a.x) * (c.y - a.y) - (b.y - a.y) * (c.x - a.x);
}

// > 0 when d lies strictly inside the circle through a, b, c (counter-clockwise)
inline int incircle(const P2 &a, const P2 &b, const P2 &c, const P2 &d) {
    const __int128 adx = a.x - d.x, ady = a.y - d.y, bdx = b.x - d.x, bdy = b.y - d.y, cdx = c.x - d.x,
                   cdy = c.y - d.y;
    const __int128 det = (adx * adx + ady * ady) * (bdx * cdy - bdy * cdx) -
                         (bdx * bdx + bdy * bdy) * (adx * cdy - ady * cdx) +
                         (cdx * cdx + cdy * cdy) * (adx * bdy - ady * bdx);
    return det > 0 ? 1 : (det < 0 ? -1 : 0);
}

struct Tri {
    int v[3];   // counter-clockwise
    int n[3];   // neighbour across the edge opposite v[i], -1 outside
    bool alive;
};

// Position of (x, y) along the Hilbert curve over a 2^15 x 2^15 grid (the
// published bit-by-bit construction: quadrant digit, then the rotation and
// reflection of the sub-square).
inline uint64_t hilbert_index(uint32_t x, uint32_t y) {
    const uint32_t n = 1u << 15;
    uint64_t d = 0;
    for (uint32_t s = n / 2; s > 0; s /= 2) {
        const uint32_t rx = (x & s) ? 1 : 0, ry = (y & s) ? 1 : 0;
        d += (uint64_t)s * s * ((3 * rx) ^ ry);
        if (ry == 0) {
            if (rx == 1) {
                x = n - 1 - x;
                y = n - 1 - y;
            }
            std::swap(x, y);
        }
    }
    return d;
}

class Delaunay {
  public:
    std::vector<P2> P;
    std::vector<Tri> T;
    int n_real = 0;

    // Points are inserted along the Hilbert curve: consecutive points are
    // near each other, so the walk to the next point is short and each
    // cavity small (row order would leave a long front of triangles on the
    // far vertices, each cavity growing with the row).  Where points are
    // cocircular the order decides which of the valid triangulations comes out.
    void run(const std::vector<P2> &pts) {
        n_real = (int)pts.size();
        P = pts;
        const long L = 1L << 26;
        P.push_back({-L, -L});
        P.push_back({3 * L, -L});
        P.push_back({-L, 3 * L});
        T.clear();
        T.reserve((size_t)6 * n_real + 16);
        T.push_back({{n_real, n_real + 1, n_real + 2}, {-1, -1, -1}, true});
        std::vector<std::pair<uint64_t, int>> order(n_real);
        for (int i = 0; i < n_real; ++i) order[i] = {hilbert_index((uint32_t)P[i].x, (uint32_t)P[i].y), i};
        std::sort(order.begin(), order.end());
        int last = 0;
        std::vector<int> bad, stack;
        std::vector<char> mark;
        struct Edge {
            int a, b, outer;
        };
        std::vector<Edge> edges;
        std::vector<std::pair<int, int>> by_a;
        for (int oi = 0; oi < n_real; ++oi) {
            const int i = order[oi].second;
            const int t0 = locate(P[i], last);
            if (t0 < 0) continue;   // a duplicate point
            // cavity: triangles whose circumcircle strictly holds the point
            bad.clear();
            stack.assign(1, t0);
            mark.resize(T.size(), 0);
            mark[t0] = 1;
            while (!stack.empty()) {
                const int t = stack.back();
                stack.pop_back();
                bad.push_back(t);
                for (int e = 0; e < 3; ++e) {
                    const int nb = T[t].n[e];
                    if (nb < 0 || mark[nb]) continue;
                    const Tri &u = T[nb];
                    if (incircle(P[u.v[0]], P[u.v[1]], P[u.v[2]], P[i]) > 0) {
                        mark[nb] = 1;
                        stack.push_back(nb);
                    }
                }
            }
            // boundary edges of the cavity, each with its outer neighbour
            edges.clear();
            for (int t : bad)
                for (int e = 0; e < 3; ++e) {
                    const int nb = T[t].n[e];
                    if (nb >= 0 && mark[nb]) continue;
                    edges.push_back({T[t].v[(e + 1) % 3], T[t].v[(e + 2) % 3], nb});
                }
            for (int t : bad) {
                T[t].alive = false;
                mark[t] = 0;
            }
            // fan of new triangles (a, b, i); each edge a->b is counter-clockwise
            // seen from inside the cavity, so (a, b, i) is counter-clockwise
            const int base = (int)T.size();
            for (size_t k = 0; k < edges.size(); ++k) {
                const Edge &E = edges[k];
                T.push_back({{E.a, E.b, i}, {-1, -1, E.outer}, true});
                if (E.outer >= 0)
                    for (int e = 0; e < 3; ++e) {
                        Tri &o = T[E.outer];
                        if (o.v[(e + 1) % 3] == E.b && o.v[(e + 2) % 3] == E.a) o.n[e] = base + (int)k;
                    }
            }
            // link the fan: triangle (a, b, i) meets (b, c, i) across edge b-i
            // (opposite a) and (z, a, i) across edge i-a (opposite b)
            by_a.resize(edges.size());
            for (size_t k = 0; k < edges.size(); ++k) by_a[k] = {edges[k].a, base + (int)k};
            std::sort(by_a.begin(), by_a.end());
            for (size_t k = 0; k < edges.size(); ++k) {
                Tri &t = T[base + (int)k];
                auto it = std::lower_bound(by_a.begin(), by_a.end(), std::make_pair(t.v[1], INT_MIN));
                if (it != by_a.end() && it->first == t.v[1]) {
                    t.n[0] = it->second;              // the triangle starting at b
                    T[it->second].n[1] = base + (int)k;   // it meets this one across i-b
                }
            }
            last = base;
            mark.resize(T.size(), 0);
        }
    }

    // triangles of real points only, counter-clockwise
    std::vector<int> triangles() const {
        std::vector<int> out;
        for (const Tri &t : T)
            if (t.alive && t.v[0] < n_real && t.v[1] < n_real && t.v[2] < n_real) {
                out.push_back(t.v[0]);
                out.push_back(t.v[1]);
                out.push_back(t.v[2]);
            }
        return out;
    }

  private:
    // a live triangle holding p (edges included), walking from `start`; -1
    // when p is already a vertex
    int locate(const P2 &p, int start) {
        int t = start;
        if (!T[t].alive) t = last_alive();
        for (size_t steps = 0; steps < 4 * T.size() + 16; ++steps) {
            const Tri &u = T[t];
            int next = -1;
            for (int e = 0; e < 3 && next < 0; ++e) {
                const P2 &a = P[u.v[(e + 1) % 3]], &b = P[u.v[(e + 2) % 3]];
                if (orient(a, b, p) < 0) next = u.n[e];
            }
            if (next < 0) return is_vertex(u, p) ? -1 : t;
            t = next;
        }
        // the walk did not settle: search every live triangle
        for (size_t k = 0; k < T.size(); ++k) {
            const Tri &u = T[k];
            if (!u.alive) continue;
            if (orient(P[u.v[0]], P[u.v[1]], p) >= 0 && orient(P[u.v[1]], P[u.v[2]], p) >= 0 &&
                orient(P[u.v[2]], P[u.v[0]], p) >= 0)
                return is_vertex(u, p) ? -1 : (int)k;
        }
        return -1;
    }
    bool is_vertex(const Tri &u, const P2 &p) const {
        for (int e = 0; e < 3; ++e)
            if (P[u.v[e]].x == p.x && P[u.v[e]].y == p.y) return true;
        return false;
    }
    int last_alive() const {
        for (int k = (int)T.size() - 1; k >= 0; --k)
            if (T[k].alive) return k;
        return 0;
    }
};

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

}  // namespace

}  // namespace lfem

using namespace lfem;

extern "C" lf_status lf_triangulate(const int32_t *xy, int32_t n, int32_t *tris, int32_t max_tris, int32_t *n_tris) {
    if (n < 0 || (n > 0 && !xy) || max_tris < 0) return set_error(LF_EINVAL, "bad arguments");
    for (int32_t i = 0; i < n; ++i)
        if (xy[2 * i] < 0 || xy[2 * i] > 16383 || xy[2 * i + 1] < 0 || xy[2 * i + 1] > 16383)
            return set_error(LF_EINVAL, "point %d outside [0, 16383]^2", i);
    std::vector<P2> pp(n);
    for (int32_t i = 0; i < n; ++i) pp[i] = {xy[2 * i], xy[2 * i + 1]};
    Delaunay dt;
    dt.run(pp);
    const std::vector<int> tv = dt.triangles();
    const int n_tri = (int)(tv.size() / 3);
    if (n_tris) *n_tris = n_tri;
    if (tris)
        for (int t = 0; t < std::min(n_tri, max_tris); ++t)
            for (int e = 0; e < 3; ++e) tris[3 * t + e] = tv[3 * t + e];
    return LF_OK;
}

extern "C" lf_status lf_build_prior(const lf_params *p, const lf_support_params *sp, const uint8_t *views,
                                    const float *S_P, float *mu_T, int32_t *points, int32_t max_points,
                                    int32_t *n_points, int32_t *tris, int32_t max_tris, int32_t *n_tris,
                                    void *hip_stream) {
    if (!p || !sp) return set_error(LF_EINVAL, "params and support params are required");
    lf_status st = validate_params(p);
    if (st != LF_OK) return st;
    if (!views || !S_P || !mu_T) return set_error(LF_EINVAL, "views, S_P and mu_T are required");
    if (p->W > 16384 || p->H > 16384) return set_error(LF_EINVAL, "the prior is built for frames up to 16384 pixels");
    if (sp->step < 1 || sp->radius < 0 || sp->radius > 7 || sp->ratio_den <= 0 || sp->ratio_num < 0 ||
        sp->incon_radius < 0 || sp->incon_levels < 0 || sp->texture_min < 0)
        return set_error(LF_EINVAL, "support params out of range");
    const Geometry g = make_geometry(p);
    if (g.frac) return set_error(LF_EINVAL, "the prior is built for integer baselines and levels only");
    const bool dev_in = p->flags & LF_INPUTS_ON_DEVICE;
    const bool dev_out = p->flags & LF_OUTPUTS_ON_DEVICE;
    const int K = p->K, H = p->H, W = p->W;
    const size_t HW = (size_t)H * W, KHW = HW * K;
    if (!dev_in) {
        for (size_t i = 0; i < KHW; ++i)
            if (!(S_P[i] >= 0.0f && S_P[i] <= 1.0f)) return set_error(LF_EINVAL, "S_P[%zu] outside [0,1]", i);
    }
    hipStream_t s = (hipStream_t)hip_stream;
    const int step = sp->step;
    const int nx = (W - step / 2 + step - 1) / step, ny = (H - step / 2 + step - 1) / step;
    const size_t n_grid = (size_t)std::max(nx, 0) * std::max(ny, 0);

    // device buffers: inputs (when on the host), Sobel responses, levels
    DevBuf b_views, b_sp, b_g, b_lev;
    const uint8_t *d_views = views;
    const float *d_sp = S_P;
    if (!dev_in) {
        LF_HIP(hipMalloc(&b_views.p, KHW * 3), "allocation");
        LF_HIP(hipMalloc(&b_sp.p, KHW * 4), "allocation");
        LF_HIP(hipMemcpyAsync(b_views.p, views, KHW * 3, hipMemcpyHostToDevice, s), "copy");
        LF_HIP(hipMemcpyAsync(b_sp.p, S_P, KHW * 4, hipMemcpyHostToDevice, s), "copy");
        d_views = (const uint8_t *)b_views.p;
        d_sp = (const float *)b_sp.p;
    }
    LF_HIP(hipMalloc(&b_g.p, KHW * sizeof(short2)), "allocation");
    LF_HIP(hipMalloc(&b_lev.p, std::max<size_t>(n_grid, 1) * K * 4), "allocation");
    hipLaunchKernelGGL(lf_sobel_i16_kernel, dim3((W + 255) / 256, H, K), dim3(256), 0, s, d_views, (short2 *)b_g.p, H,
                       W);
    LF_HIP(hipGetLastError(), "sobel launch");

    // passes: the reference against every other view, then each other view
    // against its non-reference neighbours
    std::vector<int> pass_view;
    for (int a = -1; a < K; ++a) {
        const int va = a < 0 ? p->ref : a;
        if (a >= 0 && a == p->ref) continue;
        MatchArgs m{};
        m.g = (const short2 *)b_g.p;
        m.S_P = d_sp;
        m.level = (int32_t *)b_lev.p + pass_view.size() * n_grid;
        m.H = H;
        m.W = W;
        m.D = p->D;
        m.a = va;
        m.nx = nx;
        m.ny = ny;
        m.step = step;
        m.radius = sp->radius;
        m.texture_min = sp->texture_min;
        m.ratio_num = sp->ratio_num;
        m.ratio_den = sp->ratio_den;
        m.static_min = sp->static_min;
        m.dmin_i = g.dmin_i;
        m.dstep_i = g.dstep_i;
        m.tau = p->tau_init;
        if (a < 0) {
            for (int k = 0; k < K; ++k)
                if (k != p->ref) m.vs[m.n_vs++] = k;
        } else {
            if (a - 1 >= 0 && a - 1 != p->ref) m.vs[m.n_vs++] = a - 1;
            if (a + 1 < K && a + 1 != p->ref) m.vs[m.n_vs++] = a + 1;
            if (m.n_vs == 0) continue;
        }
        int used[2] = {0, 0};
        for (int t = 0; t < m.n_vs; ++t) {
            m.db[t] = g.bi[m.vs[t]] - g.bi[va];
            m.side[t] = p->baselines[m.vs[t]] > p->baselines[va] ? 1 : 0;
            used[m.side[t]] = 1;
        }
        m.two_sides = used[0] && used[1];
        pass_view.push_back(va);
        if (n_grid > 0) {
            hipLaunchKernelGGL(lf_support_match_kernel, dim3((unsigned)((n_grid + 127) / 128)), dim3(128), 0, s, m);
            LF_HIP(hipGetLastError(), "support match launch");
        }
    }
    // candidates (per-row maps), their ordered list, the consistency filter
    // and the ordered list of the points kept, on the device
    const int n_pass = (int)pass_view.size();
    const size_t n_map = (size_t)std::max(ny, 0) * W;
    const size_t cap = std::max<size_t>(n_grid * n_pass, 1);
    DevBuf b_claim, b_level, b_view, b_kept, b_rown, b_rows, b_cand, b_pts0;
    LF_HIP(hipMalloc(&b_claim.p, std::max<size_t>(n_map, 1) * 8), "allocation");
    LF_HIP(hipMalloc(&b_level.p, std::max<size_t>(n_map, 1) * 4), "allocation");
    LF_HIP(hipMalloc(&b_view.p, std::max<size_t>(n_map, 1) * 4), "allocation");
    LF_HIP(hipMalloc(&b_kept.p, std::max<size_t>(n_map, 1) * 4), "allocation");
    LF_HIP(hipMalloc(&b_rown.p, (size_t)(std::max(ny, 0) + 1) * 4), "allocation");
    LF_HIP(hipMalloc(&b_rows.p, (size_t)(std::max(ny, 0) + 1) * 4), "allocation");
    LF_HIP(hipMalloc(&b_cand.p, cap * sizeof(int4)), "allocation");
    LF_HIP(hipMalloc(&b_pts0.p, cap * sizeof(int4)), "allocation");
    int32_t n_pts0 = 0;
    if (n_grid > 0) {
        const unsigned fill_blocks = (unsigned)((n_map + 255) / 256);
        // -1 in every int32 half: the claim keys start at the largest value
        hipLaunchKernelGGL(lf_prior_fill_kernel, dim3(2 * fill_blocks), dim3(256), 0, s, (int32_t *)b_claim.p,
                           2 * n_map, -1);
        hipLaunchKernelGGL(lf_prior_fill_kernel, dim3(fill_blocks), dim3(256), 0, s, (int32_t *)b_level.p, n_map, -1);
        hipLaunchKernelGGL(lf_prior_fill_kernel, dim3(fill_blocks), dim3(256), 0, s, (int32_t *)b_kept.p, n_map, -1);
        LF_HIP(hipGetLastError(), "fill launch");
        CandArgs c{};
        c.lev = (const int32_t *)b_lev.p;
        c.sp_ref = d_sp + (size_t)p->ref * HW;
        c.claim = (unsigned long long *)b_claim.p;
        c.level = (int32_t *)b_level.p;
        c.view = (int32_t *)b_view.p;
        c.W = W;
        c.nx = nx;
        c.ny = ny;
        c.step = step;
        c.n_grid = (int)n_grid;
        c.dmin_i = g.dmin_i;
        c.dstep_i = g.dstep_i;
        c.tau = p->tau_init;
        for (int ps = 0; ps < n_pass; ++ps) {
            c.pass_view[ps] = pass_view[ps];
            c.pass_bi[ps] = g.bi[pass_view[ps]];
        }
        const unsigned gb = (unsigned)((n_grid + 255) / 256);
        hipLaunchKernelGGL(lf_cand_ref_kernel, dim3(gb), dim3(256), 0, s, c);
        if (n_pass > 1) {
            hipLaunchKernelGGL(lf_cand_claim_kernel, dim3(gb, n_pass - 1), dim3(256), 0, s, c);
            hipLaunchKernelGGL(lf_cand_moved_kernel, dim3(gb, n_pass - 1), dim3(256), 0, s, c);
        }
        LF_HIP(hipGetLastError(), "candidate launch");
        int32_t *rown = (int32_t *)b_rown.p, *rows = (int32_t *)b_rows.p;
        hipLaunchKernelGGL(lf_row_count_kernel, dim3(ny), dim3(256), 0, s, (const int32_t *)b_level.p, W, rown);
        hipLaunchKernelGGL(lf_row_scan_kernel, dim3(1), dim3(1024), 0, s, rown, ny, rows);
        hipLaunchKernelGGL(lf_row_write_kernel, dim3(ny), dim3(256), 0, s, (const int32_t *)b_level.p,
                           (const int32_t *)b_view.p, W, step, rows, (int4 *)b_cand.p);
        hipLaunchKernelGGL(lf_consistency_kernel, dim3((unsigned)((cap + 255) / 256)), dim3(256), 0, s,
                           (const int4 *)b_cand.p, rows, ny, W, step, sp->incon_radius, sp->incon_levels,
                           sp->incon_min, (int32_t *)b_kept.p);
        LF_HIP(hipGetLastError(), "candidate list launch");
        // the points kept, ordered by (y, u) (the same row maps, counted again)
        hipLaunchKernelGGL(lf_row_count_kernel, dim3(ny), dim3(256), 0, s, (const int32_t *)b_kept.p, W, rown);
        hipLaunchKernelGGL(lf_row_scan_kernel, dim3(1), dim3(1024), 0, s, rown, ny, rows);
        hipLaunchKernelGGL(lf_row_write_kernel, dim3(ny), dim3(256), 0, s, (const int32_t *)b_kept.p,
                           (const int32_t *)b_view.p, W, step, rows, (int4 *)b_pts0.p);
        LF_HIP(hipGetLastError(), "point list launch");
        LF_HIP(hipMemcpyAsync(&n_pts0, rows + ny, 4, hipMemcpyDeviceToHost, s), "copy");
        LF_HIP(hipStreamSynchronize(s), "synchronize");
    }
    std::vector<int4> pts(n_pts0);
    if (n_pts0 > 0) {
        LF_HIP(hipMemcpyAsync(pts.data(), b_pts0.p, (size_t)n_pts0 * sizeof(int4), hipMemcpyDeviceToHost, s), "copy");
        LF_HIP(hipStreamSynchronize(s), "synchronize");
    }
    // the image corners at the level of the nearest point
    if (!pts.empty()) {
        const size_t n0 = pts.size();
        const int cx[4] = {0, W - 1, 0, W - 1}, cy[4] = {0, 0, H - 1, H - 1};
        for (int c = 0; c < 4; ++c) {
            bool dup = false;
            for (const int4 &q : pts) dup |= (q.x == cx[c] && q.y == cy[c]);
            if (dup) continue;
            long best = -1;
            int lv = 0;
            for (size_t i = 0; i < n0; ++i) {
                const long dx = pts[i].x - cx[c], dy = pts[i].y - cy[c], d2 = dx * dx + dy * dy;
                if (best < 0 || d2 < best) {
                    best = d2;
                    lv = pts[i].z;
                }
            }
            pts.push_back(make_int4(cx[c], cy[c], lv, -1));
        }
    }
    // triangulation on the device: rows of the points by (y, x) (the sorted
    // points with the corners merged in), strips and side pockets, then flip
    // rounds until no edge is illegal
    const int n_pts = (int)pts.size();
    DevBuf b_pts, b_tri, b_owner, b_mu;
    LF_HIP(hipMalloc(&b_pts.p, std::max(n_pts, 1) * sizeof(int4)), "allocation");
    if (n_pts) LF_HIP(hipMemcpyAsync(b_pts.p, pts.data(), n_pts * sizeof(int4), hipMemcpyHostToDevice, s), "copy");
    std::vector<int> tv;   // triangles for the caller (host)
    int n_tri = 0;
    bool on_device = false;
    if (n_pts >= 3 && W >= 2 && H >= 2) {
        std::vector<int> order(n_pts);
        auto by_yx = [&](int i, int j) { return pts[i].y != pts[j].y ? pts[i].y < pts[j].y : pts[i].x < pts[j].x; };
        {
            std::vector<int> real(n_pts0), corner(n_pts - n_pts0);
            for (int i = 0; i < n_pts0; ++i) real[i] = i;
            for (int i = n_pts0; i < n_pts; ++i) corner[i - n_pts0] = i;
            std::merge(real.begin(), real.end(), corner.begin(), corner.end(), order.begin(), by_yx);
        }
        std::vector<int> row_start;
        for (int i = 0; i < n_pts; ++i)
            if (i == 0 || pts[order[i]].y != pts[order[i - 1]].y) row_start.push_back(i);
        row_start.push_back(n_pts);
        const int n_rows = (int)row_start.size() - 1;
        // Euler: 2 n - h - 2 triangles, h the points on the frame's border
        int h = 0;
        for (const int4 &q : pts) h += q.x == 0 || q.x == W - 1 || q.y == 0 || q.y == H - 1;
        const int T = 2 * n_pts - h - 2;
        const int base = row_start[n_rows - 1] + row_start[n_rows] - row_start[1] - 2 * (n_rows - 1);
        const int cap_tri = std::max(T, base);   // the strips' count never exceeds T; room for them regardless
        std::vector<dt::Pt> P(n_pts);
        for (int i = 0; i < n_pts; ++i) P[i] = {pts[i].x, pts[i].y};
        const size_t m = (size_t)3 * T;
        DevBuf b_P, b_order, b_rows, b_work, b_keys, b_keys2, b_vals, b_vals2, b_claim, b_flag, b_cnt, b_temp, b_nb;
        LF_HIP(hipMalloc(&b_P.p, n_pts * sizeof(dt::Pt)), "allocation");
        LF_HIP(hipMalloc(&b_order.p, n_pts * 4), "allocation");
        LF_HIP(hipMalloc(&b_rows.p, (n_rows + 1) * 4), "allocation");
        LF_HIP(hipMalloc(&b_work.p, (size_t)4 * n_rows * 4), "allocation");
        LF_HIP(hipMalloc(&b_tri.p, std::max(cap_tri, 1) * sizeof(int3)), "allocation");
        LF_HIP(hipMalloc(&b_keys.p, m * 8), "allocation");
        LF_HIP(hipMalloc(&b_keys2.p, m * 8), "allocation");
        LF_HIP(hipMalloc(&b_vals.p, m * 4), "allocation");
        LF_HIP(hipMalloc(&b_vals2.p, m * 4), "allocation");
        LF_HIP(hipMalloc(&b_claim.p, std::max(T, 1) * 4), "allocation");
        LF_HIP(hipMalloc(&b_flag.p, m), "allocation");
        LF_HIP(hipMalloc(&b_cnt.p, 16), "allocation");
        LF_HIP(hipMemcpyAsync(b_P.p, P.data(), n_pts * sizeof(dt::Pt), hipMemcpyHostToDevice, s), "copy");
        LF_HIP(hipMemcpyAsync(b_order.p, order.data(), n_pts * 4, hipMemcpyHostToDevice, s), "copy");
        LF_HIP(hipMemcpyAsync(b_rows.p, row_start.data(), (n_rows + 1) * 4, hipMemcpyHostToDevice, s), "copy");
        const dt::Pt *dP = (const dt::Pt *)b_P.p;
        int3 *dtri = (int3 *)b_tri.p;
        int *cnt = (int *)b_cnt.p;
        if (n_rows > 1)
            hipLaunchKernelGGL(lf_dt_strips_kernel, dim3((n_rows - 1 + 63) / 64), dim3(64), 0, s, dP,
                               (const int *)b_order.p, (const int *)b_rows.p, n_rows, dtri);
        hipLaunchKernelGGL(lf_dt_pockets_kernel, dim3(1), dim3(64), 0, s, dP, (const int *)b_order.p,
                           (const int *)b_rows.p, n_rows, W, (int *)b_work.p, dtri, base, cap_tri, cnt + 1);
        LF_HIP(hipGetLastError(), "triangulation launch");
        int built = -1;
        LF_HIP(hipMemcpyAsync(&built, cnt + 1, 4, hipMemcpyDeviceToHost, s), "copy");
        LF_HIP(hipStreamSynchronize(s), "synchronize");
        if (built == T && T > 0) {
            // keys below n^2
            int end_bit = 1;
            while (end_bit < 64 && ((unsigned long long)n_pts * (unsigned long long)n_pts >> end_bit) != 0) ++end_bit;
            size_t temp_bytes = 0;
            unsigned long long *k0 = (unsigned long long *)b_keys.p, *k1 = (unsigned long long *)b_keys2.p;
            int *v0 = (int *)b_vals.p, *v1 = (int *)b_vals2.p;
            LF_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, temp_bytes, k0, k1, v0, v1, (int)m, 0, end_bit, s),
                   "sort size");
            LF_HIP(hipMalloc(&b_temp.p, std::max<size_t>(temp_bytes, 1)), "allocation");
            const unsigned eb = (unsigned)((m + 255) / 256);
            // links, once: the edges sorted by key
            LF_HIP(hipMalloc(&b_nb.p, m * 4), "allocation");
            hipLaunchKernelGGL(lf_dt_edges_kernel, dim3(eb), dim3(256), 0, s, (const int3 *)dtri, T, n_pts, k0, v0);
            LF_HIP(hipGetLastError(), "edge launch");
            LF_HIP(hipcub::DeviceRadixSort::SortPairs(b_temp.p, temp_bytes, k0, k1, v0, v1, (int)m, 0, end_bit, s),
                   "edge sort");
            hipLaunchKernelGGL(lf_prior_fill_kernel, dim3(eb), dim3(256), 0, s, (int32_t *)b_nb.p, m, -1);
            hipLaunchKernelGGL(lf_dt_links_kernel, dim3(eb), dim3(256), 0, s, (const unsigned long long *)k1,
                               (const int *)v1, (int)m, (int *)b_nb.p);
            LF_HIP(hipGetLastError(), "link launch");
            // rounds of independent flips, the count of illegal edges read
            // every kRoundsPerCheck rounds (rounds after the last flip find
            // nothing to do)
            const unsigned tb = (unsigned)((T + 255) / 256);
            for (int round = 0; round < kMaxFlipRounds && !on_device; round += kRoundsPerCheck) {
                for (int r = 0; r < kRoundsPerCheck; ++r) {
                    hipLaunchKernelGGL(lf_prior_fill_kernel, dim3(tb), dim3(256), 0, s, (int32_t *)b_claim.p,
                                       (size_t)T, INT_MAX);
                    hipLaunchKernelGGL(lf_prior_fill_kernel, dim3(1), dim3(256), 0, s, (int32_t *)cnt, (size_t)1, 0);
                    hipLaunchKernelGGL(lf_dt_mark_kernel, dim3(eb), dim3(256), 0, s, (const int3 *)dtri, dP,
                                       (const int *)b_nb.p, (int)m, (int *)b_claim.p, (uint8_t *)b_flag.p, cnt);
                    hipLaunchKernelGGL(lf_dt_flip_kernel, dim3(eb), dim3(256), 0, s, dtri, (int *)b_nb.p,
                                       (const uint8_t *)b_flag.p, (const int *)b_claim.p, (int)m);
                }
                LF_HIP(hipGetLastError(), "flip launch");
                int illegal = -1;
                LF_HIP(hipMemcpyAsync(&illegal, cnt, 4, hipMemcpyDeviceToHost, s), "copy");
                LF_HIP(hipStreamSynchronize(s), "synchronize");
                on_device = illegal == 0;
            }
        }
        if (on_device) {
            n_tri = T;
            tv.resize((size_t)3 * T);
            LF_HIP(hipMemcpyAsync(tv.data(), dtri, (size_t)T * sizeof(int3), hipMemcpyDeviceToHost, s), "copy");
            LF_HIP(hipStreamSynchronize(s), "synchronize");   // before the buffers of this block are freed
        }
    }
    if (!on_device) {
        // the host triangulation (no points, a degenerate frame, or flip
        // rounds that did not settle within kMaxFlipRounds)
        std::vector<P2> pp(pts.size());
        for (size_t i = 0; i < pts.size(); ++i) pp[i] = {pts[i].x, pts[i].y};
        Delaunay dtr;
        dtr.run(pp);
        tv = dtr.triangles();
        n_tri = (int)(tv.size() / 3);
        if (b_tri.p) {
            (void)hipFree(b_tri.p);
            b_tri.p = nullptr;
        }
        LF_HIP(hipMalloc(&b_tri.p, std::max(n_tri, 1) * sizeof(int3)), "allocation");
        if (n_tri) LF_HIP(hipMemcpyAsync(b_tri.p, tv.data(), n_tri * sizeof(int3), hipMemcpyHostToDevice, s), "copy");
    }

    // raster on the device
    LF_HIP(hipMalloc(&b_owner.p, HW * 4), "allocation");
    float *d_mu = mu_T;
    if (!dev_out) {
        LF_HIP(hipMalloc(&b_mu.p, HW * 4), "allocation");
        d_mu = (float *)b_mu.p;
    }
    hipLaunchKernelGGL(lf_prior_fill_kernel, dim3((unsigned)((HW + 255) / 256)), dim3(256), 0, s, (int32_t *)b_owner.p,
                       HW, INT_MAX);
    LF_HIP(hipGetLastError(), "fill launch");
    if (n_tri) {
        hipLaunchKernelGGL(lf_prior_cover_kernel, dim3(n_tri), dim3(256), 0, s, (const int4 *)b_pts.p,
                           (const int3 *)b_tri.p, n_tri, (int32_t *)b_owner.p, H, W);
        LF_HIP(hipGetLastError(), "cover launch");
    }
    hipLaunchKernelGGL(lf_prior_interp_kernel, dim3((W + 255) / 256, H), dim3(256), 0, s, (const int4 *)b_pts.p, n_pts,
                       (const int3 *)b_tri.p, (const int32_t *)b_owner.p, d_mu, H, W, p->D, (double)p->d_min,
                       (double)p->d_step);
    LF_HIP(hipGetLastError(), "interpolation launch");
    if (!dev_out) LF_HIP(hipMemcpyAsync(mu_T, d_mu, HW * 4, hipMemcpyDeviceToHost, s), "copy");
    LF_HIP(hipStreamSynchronize(s), "synchronize");
    if (n_points) *n_points = n_pts;
    if (n_tris) *n_tris = n_tri;
    if (points)
        for (int i = 0; i < std::min(n_pts, max_points); ++i) {
            points[4 * i] = pts[i].x;
            points[4 * i + 1] = pts[i].y;
            points[4 * i + 2] = pts[i].z;
            points[4 * i + 3] = pts[i].w;
        }
    if (tris)
        for (int t = 0; t < std::min(n_tri, max_tris); ++t)
            for (int e = 0; e < 3; ++e) tris[3 * t + e] = tv[3 * t + e];
    return LF_OK;
}
