// Allocation-free whole-frame entry point (lf_em_frame_noalloc): the work of
// lf_em_init, lf_em_iterate and lf_refocus with device inputs and outputs,
// with every intermediate buffer carved from one fixed device array instead
// of a context's allocation.
//
// The array `scratch` is a file-scope __device__ object: each GPU the library
// runs on holds its own copy, at its own address, until the process ends.
// Host code never passes the array's name to a kernel (in host code it names
// a host-side stand-in, not device memory); the device address of each GPU's
// copy is looked up once per device with hipGetSymbolAddress and used
// everywhere instead.
#include "lf_em.h"
#include "lf_em_kernels.h"
#include "lf_internal.h"

#include <algorithm>
#include <mutex>

namespace lfem {

static __device__ __align__(256) unsigned char scratch[LF_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

// Device address of this GPU's scratch array (the current device), looked up
// on the first call on the device.
static lf_status scratch_address(int device, unsigned char **out) {
    if (device < 0 || device >= kMaxDevices) return set_error(LF_EDEVICE, "device %d beyond %d", device, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return set_error(LF_EDEVICE, "scratch address on device %d: %s", device, hipGetErrorString(e));
        }
        g_scratch_ptr[device] = ptr;
    }
    *out = static_cast<unsigned char *>(g_scratch_ptr[device]);
    return LF_OK;
}

// Byte ranges of the frame's intermediate buffers inside the scratch array.
struct NoallocPlan {
    size_t feat, rho, omr, lpix, obj, rgb_med, bad, dyn_rows, dyn_items, dyn_n, total;
};

static size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

static NoallocPlan noalloc_plan(const lf_params *p, int n_blocks, int n_iters, int median, const DynPlan &d) {
    const size_t HW = (size_t)p->H * p->W, KHW = HW * p->K;
    NoallocPlan pl{};
    size_t o = 0;
    auto carve = [&](size_t bytes) {
        const size_t r = o;
        o += round256(bytes);
        return r;
    };
    pl.feat = carve(KHW * pair_bytes(p->storage));
    pl.rho = carve(KHW * 4);
    pl.omr = carve(KHW * 4);
    pl.lpix = carve(HW * 4);
    pl.obj = carve((size_t)std::min(n_iters, kMaxItersPerLaunch) * n_blocks * 8);
    pl.rgb_med = median ? carve(HW * 12) : 0;
    pl.bad = carve(4);
    if (d.span) {
        pl.dyn_rows = carve(dyn_rows_ints(p, d) * 4);
        pl.dyn_items = carve((size_t)d.max_items * 16);
        pl.dyn_n = carve(4);
    }
    pl.total = o;
    return pl;
}

}  // namespace lfem

using namespace lfem;

#define LF_HIP(call, what)                                 \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return hip_error(e_, what);  \
    } while (0)

extern "C" lf_status lf_em_frame_noalloc(const lf_params *p, const uint8_t *views, const float *S_P,
                                         const float *mu_T, const float *q_warm, int32_t n_iters, float *rgb,
                                         int32_t *d_idx, float *q, uint8_t *hole, int32_t median, double *objective,
                                         uint32_t *invalid, void *hip_stream) {
    lf_status st = validate_params(p);
    if (st != LF_OK) return st;
    if (!views || !S_P || !mu_T) return set_error(LF_EINVAL, "views, S_P and mu_T are required");
    if (!rgb || !d_idx || !q) return set_error(LF_EINVAL, "rgb, d_idx and q are required");
    if (n_iters < 1 || n_iters > 100000) return set_error(LF_EINVAL, "n_iters=%d outside [1,100000]", n_iters);
    if (median != 0 && median != 3) return set_error(LF_EINVAL, "median=%d must be 0 or 3", median);
    // every pointer is device memory here, whatever the flags say
    lf_params pp = *p;
    pp.flags = (pp.flags | LF_INPUTS_ON_DEVICE | LF_OUTPUTS_ON_DEVICE) & ~(uint32_t)LF_DEFERRED_CHECK;
    const hipStream_t s = (hipStream_t)hip_stream;
    int device = 0;
    LF_HIP(hipGetDevice(&device), "current device");
    unsigned char *base = nullptr;
    st = scratch_address(device, &base);
    if (st != LF_OK) return st;

    const Geometry g = make_geometry(&pp);
    int tile = 0;
    size_t lds = 0;
    st = em_launch_shape(&pp, g, device, &tile, &lds);
    if (st != LF_OK) return st;
    int lds_limit = 0;
    LF_HIP(hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, device), "device attribute");
    const DynPlan dyn = dyn_plan(&pp, g, (size_t)lds_limit);
    const int n_blocks = dyn.span ? dyn.max_items : ((pp.W + tile - 1) / tile) * pp.H;
    const NoallocPlan pl = noalloc_plan(&pp, n_blocks, n_iters, median, dyn);
    if (pl.total > LF_NOALLOC_SCRATCH_BYTES)
        return set_error(LF_EINVAL, "frame needs %zu bytes of scratch, above the fixed %zu", pl.total,
                         (size_t)LF_NOALLOC_SCRATCH_BYTES);

    void *feat = base + pl.feat;
    float *rho = reinterpret_cast<float *>(base + pl.rho);
    float *omr = reinterpret_cast<float *>(base + pl.omr);
    float *lpix = reinterpret_cast<float *>(base + pl.lpix);
    double *obj = reinterpret_cast<double *>(base + pl.obj);
    float *rgb_med = median ? reinterpret_cast<float *>(base + pl.rgb_med) : nullptr;
    uint32_t *bad = invalid ? invalid : reinterpret_cast<uint32_t *>(base + pl.bad);

    // the count of invalid input values starts at zero (a fill kernel, not a
    // memset, so that the call can be captured in a graph)
    LF_HIP(launch_fill_u32(bad, 1, 0u, s), "clear counter");
    LF_HIP(launch_load(&pp, views, feat, S_P, mu_T, q_warm, rho, omr, q, bad, 1, s), "load launch");

    EmArgs a = make_em_args(&pp, g, derived_lambda(&pp));
    if (dyn.span) {
        EmArgs da = a;
        da.feat = feat;
        da.rho = rho;
        da.q = q;
        da.mu_T = mu_T;
        da.d_idx = d_idx;
        da.lpix = lpix;
        da.seg_w = dyn.span;
        LF_HIP(launch_dyn_list(&pp, da, dyn, reinterpret_cast<int *>(base + pl.dyn_rows),
                               reinterpret_cast<int4 *>(base + pl.dyn_items), reinterpret_cast<int *>(base + pl.dyn_n), s),
               "dynamic-only work list");
        a.items = reinterpret_cast<const int4 *>(base + pl.dyn_items);
        a.n_items = reinterpret_cast<const int *>(base + pl.dyn_n);
    }
    a.feat = feat;
    a.rho = rho;
    a.omr = omr;
    a.mu_T = mu_T;
    a.q = q;
    a.d_idx = d_idx;
    a.lpix = lpix;
    a.obj = obj;
    for (int done = 0; done < n_iters;) {
        const int n = std::min(kMaxItersPerLaunch, n_iters - done);
        a.n_iters = n;
        a.seed_from_d = done > 0;
        a.want_obj = objective != nullptr;
        LF_HIP(launch_em(&pp, g, a, tile, lds, s, &dyn), "EM launch");
        if (objective) LF_HIP(launch_objective_sum(obj, n_blocks, n, objective + done, s), "objective launch");
        done += n;
    }
    LF_HIP(launch_refocus_frame(&pp, g, views, d_idx, q, rho, rgb, hole, rgb_med, median, nullptr, nullptr, s),
           "refocus launch");
    return LF_OK;
}
