// Internal declarations shared by the plain context (lf_em.hip) and the
// frame server (lf_server.hip).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "lf_em.h"

namespace lfem {

struct EmArgs;
struct RefocusArgs;
using EmKernel = void (*)(EmArgs);

EmKernel pick_em_f32(int K, bool frac, bool exh, bool sym, bool share, bool enumerate);
EmKernel pick_em_f16(int K, bool frac, bool exh, bool sym, bool share, bool enumerate);
EmKernel pick_em_bf16(int K, bool frac, bool exh, bool sym, bool share, bool enumerate);
// view-count ranges 2-5 (a), 6-9 (b) and 10-16 (c) of each storage format
#define LF_PICK_PART(name) EmKernel name(int K, bool frac, bool exh, bool sym, bool share, bool enumerate);
LF_PICK_PART(pick_em_f32_a) LF_PICK_PART(pick_em_f32_b) LF_PICK_PART(pick_em_f32_c)
LF_PICK_PART(pick_em_f16_a) LF_PICK_PART(pick_em_f16_b) LF_PICK_PART(pick_em_f16_c)
LF_PICK_PART(pick_em_bf16_a) LF_PICK_PART(pick_em_bf16_b) LF_PICK_PART(pick_em_bf16_c)
#undef LF_PICK_PART

struct ServeJob;
using ServeKernel = void (*)(const ServeJob *, int);
// frame-server instances of view counts 2-5 (a) and 6-9 (b) per storage format
ServeKernel pick_serve_f32_a(int K, int kind);
ServeKernel pick_serve_f32_b(int K, int kind);
ServeKernel pick_serve_f16_a(int K, int kind);
ServeKernel pick_serve_f16_b(int K, int kind);
ServeKernel pick_serve_bf16_a(int K, int kind);
ServeKernel pick_serve_bf16_b(int K, int kind);

// Integer-shift geometry: when every baseline and both level parameters are
// integers, footprints x - b_k d_j are exact integers and the kernels index
// directly; otherwise they interpolate (frac = true).
struct Geometry {
    bool frac;
    bool sym;   // integer shifts of a unit-spaced array centred on the reference, d_step = 1
    int dmin_i, dstep_i;
    int bi[LF_MAX_VIEWS];
};

// One device allocation carved into 256-byte aligned buffers.
struct ArenaPlan {
    struct Item {
        void **slot;
        size_t bytes;
    };
    std::vector<Item> items;
    template <class T>
    void add(T **slot, size_t bytes) {
        items.push_back({reinterpret_cast<void **>(slot), bytes});
    }
    size_t total() const {
        size_t t = 0;
        for (const Item &i : items) t += (i.bytes + 255) & ~(size_t)255;
        return t;
    }
};

struct DeviceArena {
    void *base = nullptr;
    size_t bytes = 0;
    lf_status allocate(const ArenaPlan &plan);
    void release();
};

EmArgs make_em_args(const lf_params *p, const Geometry &g, float lambda);
lf_status set_error(lf_status s, const char *fmt, ...);
lf_status hip_error(hipError_t e, const char *what);
lf_status validate_params(const lf_params *p);
lf_status validate_host_values(const lf_params *p, const float *S_P, const float *mu_T, const float *q_warm);
float derived_lambda(const lf_params *p);
Geometry make_geometry(const lf_params *p);
size_t em_window_pairs(const lf_params *p, const Geometry &g, int tile);
size_t em_window_widest(const lf_params *p, const Geometry &g, int tile);
size_t pair_bytes(int storage);
size_t rec_bytes(int storage);
int choose_tile(const lf_params *p, const Geometry &g, size_t lds_limit, size_t lds_per_cu, int vgprs,
                size_t *lds_out);

// Descriptors and ray prior of a frame (one launch).
hipError_t launch_load(const lf_params *p, const uint8_t *views, void *feat, const float *S_P, const float *mu_T,
                       const float *q_warm, float *rho, float *omr, float *q, uint32_t *bad, int check,
                       hipStream_t s);
hipError_t launch_median3(const lf_params *p, const float *in, float *out, hipStream_t s);
// Dynamic-only work list of a frame (span == 0: not dynamic-only).
struct DynPlan {
    int span;        // columns an item's pixels may spread over (multiple of 64)
    int split;       // items also limited in pixels predicted unbounded (shared sweep)
    int per_row;     // bound on a row's items
    int max_items;   // H * per_row
    size_t lds;      // block LDS of an item's windows
};
DynPlan dyn_plan(const lf_params *p, const Geometry &g, size_t lds_limit);
// Ints of the per-row scratch of the list: H counts and H * per_row items
// (first column, pixels).
size_t dyn_rows_ints(const lf_params *p, const DynPlan &d);
hipError_t launch_dyn_list(const lf_params *p, const EmArgs &a, const DynPlan &d, int *rows, int4 *items,
                           int *n_items, hipStream_t s);
hipError_t launch_em(const lf_params *p, const Geometry &g, EmArgs a, int tile, size_t lds, hipStream_t s,
                     const DynPlan *d);
hipError_t launch_refocus_frame(const lf_params *p, const Geometry &g, const uint8_t *views, const int32_t *d_idx,
                                const float *q, const float *rho, float *rgb, uint8_t *hole, float *rgb_med,
                                int median, int32_t *d_out, float *q_out, hipStream_t s);
hipError_t launch_objective_sum(const double *partials, int n_blocks, int n, double *objective, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, size_t n, uint32_t v, hipStream_t s);
// Row-tile width and block LDS of the EM kernel for these parameters on a device.
lf_status em_launch_shape(const lf_params *p, const Geometry &g, int device, int *tile, size_t *lds);
constexpr int kMaxItersPerLaunch = 64;

}  // namespace lfem
