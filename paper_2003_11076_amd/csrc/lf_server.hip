// Frame server: continuous batching of light-field frames from many streams.
//
// Frames are submitted by any thread.  Their host inputs are copied into a
// pinned staging arena at submission (when it is full the call returns
// LF_EAGAIN).  A service thread admits frames in arrival order as soon as
// their stream is idle and the HBM budget holds their buffers, groups every
// frame admitted at that moment into one batch, and launches the batch as
// one kernel (per storage format) covering all (frame, row tile) pairs, on
// one of several HIP streams, so batches overlap on the device.  When a
// batch's event completes, outputs are copied to the caller's buffers, the
// frame's weights stay on the device as its stream's warm start, memory is
// released and the caller's callback runs.  Kernel boundaries give the
// batches a coherent view of the inputs the copies wrote.
#include "lf_em.h"
#include "lf_internal.h"
#include "lf_serve_kernels.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

namespace lfem {

// First-fit allocator of byte ranges inside one allocation (256-byte granules).
class RangeAllocator {
  public:
    void reset(size_t size) {
        free_.clear();
        size_ = size & ~(size_t)255;
        if (size_) free_[0] = size_;
        used_ = peak_ = 0;
    }
    bool alloc(size_t bytes, size_t &off) {
        bytes = round(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            off = it->first;
            const size_t rest = it->second - bytes, start = it->first + bytes;
            free_.erase(it);
            if (rest) free_[start] = rest;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = round(bytes);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    static size_t round(size_t b) { return (b + 255) & ~(size_t)255; }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    size_t size() const { return size_; }

  private:
    std::map<size_t, size_t> free_;
    size_t size_ = 0, used_ = 0, peak_ = 0;
};

using Clock = std::chrono::steady_clock;

struct SrvFrame {
    int64_t id;
    int stream;
    lf_params p;
    Geometry g;
    float lambda;
    float *rgb_out;
    int32_t *d_out;
    float *q_out;
    lf_done_fn done;
    void *user;
    // pinned staging: inputs then outputs
    size_t h_off = 0, h_bytes = 0;
    size_t in_views, in_sp, in_mu, out_rgb, out_d, out_q, out_hole;
    // device: frame block (inputs, outputs but q) and the weights block
    size_t d_off = 0, d_bytes = 0, q_off = 0, q_bytes = 0;
    bool warm = false;
    int tiles_x = 0, n_tiles = 0;
    size_t lds = 0;
    Clock::time_point t_submit, t_admit, t_done;
    lf_status status = LF_OK;
};

struct SrvStream {
    bool busy = false;
    bool has_warm = false;
    int K = 0, H = 0, W = 0;
    size_t q_off = 0, q_bytes = 0;
    int64_t last_use = 0;      // completion order, for evicting the oldest warm start
};

struct SrvBatch {
    int slot;
    hipEvent_t ev;
    std::vector<SrvFrame *> frames;
};

constexpr size_t kMaxBatch = 16;

}  // namespace lfem

using namespace lfem;

struct lf_server {
    int device = 0;
    int n_iters = 8;
    int max_streams = 1;
    size_t lds_limit = 65536;
    // device arena
    char *dpool = nullptr;
    RangeAllocator dalloc;
    // pinned staging arena
    char *hpool = nullptr;
    RangeAllocator halloc;
    // streams of the device work
    static constexpr int kSlots = 3;
    hipStream_t hs[kSlots] = {};
    bool slot_busy[kSlots] = {};
    size_t djobs_off[kSlots] = {}, hjobs_off[kSlots] = {};   // job tables reserved per slot
    int64_t use_clock = 0;
    std::vector<SrvStream> streams;
    std::deque<SrvFrame *> pending;
    std::vector<SrvBatch *> inflight;
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv, cv_idle;
    bool stop = false;
    int64_t next_id = 0;
    // statistics
    int64_t submitted = 0, completed = 0, failed = 0, rejected = 0, batches = 0, batch_frames = 0;
    std::vector<double> lat_ms;
    Clock::time_point t_first, t_last;
    bool any = false;
    lf_status sticky = LF_OK;
    std::string sticky_msg;
};

namespace {

size_t frame_lds(const lf_params &p, const Geometry &g) {
    const size_t pairs = em_window_pairs(&p, g, kServeTile);
    return pairs * rec_bytes(p.storage) + 2 * 3 * (pairs + 2 * (size_t)p.K) + 64;
}

void fail_frame(SrvFrame *f, lf_status st) { f->status = st; }

// Launch one batch (caller holds the lock).  Returns false on a HIP error.
bool launch_batch(lf_server *s, SrvBatch *b, std::string &err) {
    hipStream_t st = s->hs[b->slot];
    const size_t nj = b->frames.size();
    // the slot's job tables (pinned and device), grouped by storage
    ServeJob *hj = reinterpret_cast<ServeJob *>(s->hpool + s->hjobs_off[b->slot]);
    ServeJob *dj = reinterpret_cast<ServeJob *>(s->dpool + s->djobs_off[b->slot]);
    int order = 0;
    size_t lds_max[3] = {0, 0, 0};
    int start[3] = {0, 0, 0}, count[3] = {0, 0, 0}, tiles[3] = {0, 0, 0};
    for (int stg = 0; stg < 3; ++stg) {
        start[stg] = order;
        for (SrvFrame *f : b->frames) {
            if (f->p.storage != stg) continue;
            const lf_params &p = f->p;
            const size_t HW = (size_t)p.H * p.W, KHW = HW * p.K;
            char *h = s->hpool + f->h_off;
            char *d = s->dpool + f->d_off;
            ServeJob &J = hj[order++];
            std::memset(&J, 0, sizeof J);
            J.em = make_em_args(&p, f->g, f->lambda);
            J.em.H = p.H;
            J.em.W = p.W;
            J.em.tile = kServeTile;
            J.em.n_iters = s->n_iters;
            // device layout of the frame block
            size_t o = 0;
            auto carve = [&](size_t bytes) { size_t r = o; o += RangeAllocator::round(bytes); return r; };
            const size_t o_views = carve(KHW * 3), o_sp = carve(KHW * 4), o_mu = carve(HW * 4), o_rgb = carve(HW * 12),
                         o_d = carve(HW * 4), o_hole = carve(HW);
            J.views = reinterpret_cast<const uint8_t *>(d + o_views);
            J.S_P = reinterpret_cast<const float *>(d + o_sp);
            J.em.mu_T = reinterpret_cast<const float *>(d + o_mu);
            J.rgb = reinterpret_cast<float *>(d + o_rgb);
            J.em.d_idx = reinterpret_cast<int32_t *>(d + o_d);
            J.hole = reinterpret_cast<uint8_t *>(d + o_hole);
            J.em.q = reinterpret_cast<float *>(s->dpool + f->q_off);
            J.q_warm = f->warm ? reinterpret_cast<const float *>(s->dpool + s->streams[f->stream].q_off) : nullptr;
            J.K = p.K;
            J.ref = p.ref;
            J.frac = f->g.frac ? 1 : 0;
            J.sym = f->g.sym ? 1 : 0;
            J.tiles_x = f->tiles_x;
            J.tile_start = tiles[stg];
            J.n_tiles = f->n_tiles;
            J.tau = p.tau_init;
            tiles[stg] += f->n_tiles;
            lds_max[stg] = std::max(lds_max[stg], f->lds);
            // inputs to the device
            hipError_t e;
            e = hipMemcpyAsync(d + o_views, h + f->in_views, KHW * 3, hipMemcpyHostToDevice, st);
            if (e == hipSuccess) e = hipMemcpyAsync(d + o_sp, h + f->in_sp, KHW * 4, hipMemcpyHostToDevice, st);
            if (e == hipSuccess) e = hipMemcpyAsync(d + o_mu, h + f->in_mu, HW * 4, hipMemcpyHostToDevice, st);
            if (e != hipSuccess) {
                err = hipGetErrorString(e);
                return false;
            }
        }
        count[stg] = order - start[stg];
    }
    hipError_t e = hipMemcpyAsync(dj, hj, nj * sizeof(ServeJob), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) {
        err = hipGetErrorString(e);
        return false;
    }
    for (int stg = 0; stg < 3; ++stg) {
        if (!count[stg]) continue;
        ServeKernel k = stg == 0 ? pick_serve_f32() : (stg == 1 ? pick_serve_f16() : pick_serve_bf16());
        hipLaunchKernelGGL(k, dim3(tiles[stg]), dim3(kServeTile), lds_max[stg], st, dj + start[stg], count[stg]);
        e = hipGetLastError();
        if (e != hipSuccess) {
            err = hipGetErrorString(e);
            return false;
        }
    }
    // outputs back to the pinned staging
    for (SrvFrame *f : b->frames) {
        const lf_params &p = f->p;
        const size_t HW = (size_t)p.H * p.W, KHW = HW * p.K;
        char *h = s->hpool + f->h_off;
        char *d = s->dpool + f->d_off;
        size_t o = 0;
        auto carve = [&](size_t bytes) { size_t r = o; o += RangeAllocator::round(bytes); return r; };
        carve(KHW * 3);
        carve(KHW * 4);
        carve(HW * 4);
        const size_t o_rgb = carve(HW * 12), o_d = carve(HW * 4), o_hole = carve(HW);
        e = hipMemcpyAsync(h + f->out_rgb, d + o_rgb, HW * 12, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(h + f->out_d, d + o_d, HW * 4, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(h + f->out_hole, d + o_hole, HW, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess && f->q_out)
            e = hipMemcpyAsync(h + f->out_q, s->dpool + f->q_off, KHW * 4, hipMemcpyDeviceToHost, st);
        if (e != hipSuccess) {
            err = hipGetErrorString(e);
            return false;
        }
    }
    e = hipEventRecord(b->ev, st);
    if (e != hipSuccess) {
        err = hipGetErrorString(e);
        return false;
    }
    return true;
}

// Admit frames and launch a batch if a device stream is free (lock held).
void schedule(lf_server *s) {
    int slot = -1;
    for (int i = 0; i < lf_server::kSlots; ++i)
        if (!s->slot_busy[i]) {
            slot = i;
            break;
        }
    if (slot < 0 || s->pending.empty()) return;
    SrvBatch *b = new SrvBatch();
    b->slot = slot;
    for (auto it = s->pending.begin(); it != s->pending.end() && b->frames.size() < kMaxBatch;) {
        SrvFrame *f = *it;
        SrvStream &ss = s->streams[f->stream];
        if (ss.busy) {
            ++it;
            continue;
        }
        const lf_params &p = f->p;
        const size_t HW = (size_t)p.H * p.W, KHW = HW * p.K;
        f->d_bytes = RangeAllocator::round(KHW * 3) + RangeAllocator::round(KHW * 4) + RangeAllocator::round(HW * 4) +
                     RangeAllocator::round(HW * 12) + RangeAllocator::round(HW * 4) + RangeAllocator::round(HW);
        f->q_bytes = KHW * 4;
        const bool same_shape = ss.has_warm && ss.K == p.K && ss.H == p.H && ss.W == p.W;
        if (ss.has_warm && !same_shape) {
            // shape changed: the stream starts cold, its old weights go
            s->dalloc.release(ss.q_off, ss.q_bytes);
            ss.has_warm = false;
        }
        size_t doff = 0, qoff = 0;
        bool fit = false;
        for (;;) {
            if (s->dalloc.alloc(f->d_bytes, doff)) {
                if (s->dalloc.alloc(f->q_bytes, qoff)) {
                    fit = true;
                    break;
                }
                s->dalloc.release(doff, f->d_bytes);
            }
            // nothing in flight or admitted will free memory: give up the
            // oldest warm start of an idle stream (that stream starts cold)
            if (!s->inflight.empty() || !b->frames.empty()) break;
            SrvStream *victim = nullptr;
            for (SrvStream &o : s->streams)
                if (o.has_warm && !o.busy && &o != &ss && (!victim || o.last_use < victim->last_use)) victim = &o;
            if (!victim) break;
            s->dalloc.release(victim->q_off, victim->q_bytes);
            victim->has_warm = false;
        }
        if (!fit) break;  // budget: wait for memory (arrival order is kept)
        f->d_off = doff;
        f->q_off = qoff;
        f->warm = same_shape;
        f->t_admit = Clock::now();
        ss.busy = true;
        b->frames.push_back(f);
        it = s->pending.erase(it);
    }
    if (b->frames.empty()) {
        delete b;
        return;
    }
    if (hipEventCreateWithFlags(&b->ev, hipEventDisableTiming) != hipSuccess) {
        s->sticky = LF_EDEVICE;
        s->sticky_msg = "event creation";
    }
    std::string err;
    if (s->sticky == LF_OK && !launch_batch(s, b, err)) {
        s->sticky = LF_EDEVICE;
        s->sticky_msg = "batch launch: " + err;
    }
    s->slot_busy[slot] = true;
    s->batches += 1;
    s->batch_frames += (int64_t)b->frames.size();
    s->inflight.push_back(b);
}

// Finish completed batches (lock held); callbacks are returned to run unlocked.
void reap(lf_server *s, std::vector<SrvFrame *> &finished) {
    for (auto it = s->inflight.begin(); it != s->inflight.end();) {
        SrvBatch *b = *it;
        hipError_t q = s->sticky == LF_OK ? hipEventQuery(b->ev) : hipSuccess;
        if (q == hipErrorNotReady) {
            ++it;
            continue;
        }
        const bool ok = (q == hipSuccess) && s->sticky == LF_OK;
        if (q != hipSuccess && q != hipErrorNotReady && s->sticky == LF_OK) {
            s->sticky = LF_EDEVICE;
            s->sticky_msg = hipGetErrorString(q);
        }
        for (SrvFrame *f : b->frames) {
            const lf_params &p = f->p;
            const size_t HW = (size_t)p.H * p.W, KHW = HW * p.K;
            const char *h = s->hpool + f->h_off;
            SrvStream &ss = s->streams[f->stream];
            if (ok) {
                std::memcpy(f->rgb_out, h + f->out_rgb, HW * 12);
                if (f->d_out) std::memcpy(f->d_out, h + f->out_d, HW * 4);
                if (f->q_out) std::memcpy(f->q_out, h + f->out_q, KHW * 4);
                // the frame's weights become the stream's warm start
                if (ss.has_warm) s->dalloc.release(ss.q_off, ss.q_bytes);
                ss.has_warm = true;
                ss.K = p.K;
                ss.H = p.H;
                ss.W = p.W;
                ss.q_off = f->q_off;
                ss.q_bytes = f->q_bytes;
                ss.last_use = ++s->use_clock;
            } else {
                fail_frame(f, LF_EDEVICE);
                s->dalloc.release(f->q_off, f->q_bytes);
            }
            s->dalloc.release(f->d_off, f->d_bytes);
            s->halloc.release(f->h_off, f->h_bytes);
            ss.busy = false;
            f->t_done = Clock::now();
            finished.push_back(f);
        }
        (void)hipEventDestroy(b->ev);
        s->slot_busy[b->slot] = false;
        delete b;
        it = s->inflight.erase(it);
    }
}

void service(lf_server *s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        std::vector<SrvFrame *> finished;
        reap(s, finished);
        schedule(s);
        const bool idle = s->pending.empty() && s->inflight.empty();
        if (!finished.empty()) {
            lk.unlock();
            for (SrvFrame *f : finished) {
                if (f->done) f->done(f->id, f->status, f->user);
            }
            lk.lock();
            for (SrvFrame *f : finished) {
                const double ms = std::chrono::duration<double, std::milli>(f->t_done - f->t_submit).count();
                if (f->status == LF_OK) {
                    s->completed += 1;
                    s->lat_ms.push_back(ms);
                } else {
                    s->failed += 1;
                }
                s->t_last = f->t_done;
                delete f;
            }
            s->cv_idle.notify_all();
            continue;
        }
        if (idle) {
            s->cv_idle.notify_all();
            if (s->stop) break;
            s->cv.wait(lk);
        } else if (!s->inflight.empty()) {
            // device work outstanding: poll its events at a short interval
            s->cv.wait_for(lk, std::chrono::microseconds(20));
        } else {
            s->cv.wait_for(lk, std::chrono::microseconds(200));
        }
    }
}

double percentile(std::vector<double> v, double q) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = q * (v.size() - 1);
    const size_t i = (size_t)pos;
    const double fr = pos - i;
    return i + 1 < v.size() ? v[i] * (1.0 - fr) + v[i + 1] * fr : v[i];
}

}  // namespace

extern "C" {

lf_status lf_server_create(lf_server **out, size_t hbm_budget_bytes, int32_t max_streams, int32_t n_iters,
                           size_t staging_bytes) {
    if (!out) return set_error(LF_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_streams < 1 || max_streams > 4096) return set_error(LF_EINVAL, "max_streams=%d outside [1,4096]", max_streams);
    if (n_iters < 0 || n_iters > 1000) return set_error(LF_EINVAL, "n_iters=%d outside [0,1000]", n_iters);
    if (hbm_budget_bytes < ((size_t)64 << 10)) return set_error(LF_EINVAL, "HBM budget below 64 KiB");
    if (staging_bytes == 0) staging_bytes = std::min(hbm_budget_bytes, (size_t)1 << 30);
    lf_server *s = new lf_server();
    s->n_iters = n_iters;
    s->max_streams = max_streams;
    s->streams.resize(max_streams);
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return set_error(LF_EDEVICE, "no HIP device");
    }
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, s->device) == hipSuccess) s->lds_limit = v;
    hipError_t e = hipMalloc((void **)&s->dpool, hbm_budget_bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        return set_error(LF_ENOMEM, "HBM arena of %zu bytes: %s", hbm_budget_bytes, hipGetErrorString(e));
    }
    s->dalloc.reset(hbm_budget_bytes);
    e = hipHostMalloc((void **)&s->hpool, staging_bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipFree(s->dpool);
        delete s;
        return set_error(LF_ENOMEM, "pinned staging of %zu bytes: %s", staging_bytes, hipGetErrorString(e));
    }
    s->halloc.reset(staging_bytes);
    for (int i = 0; i < lf_server::kSlots; ++i) {
        if (!s->dalloc.alloc(kMaxBatch * sizeof(ServeJob), s->djobs_off[i]) ||
            !s->halloc.alloc(kMaxBatch * sizeof(ServeJob), s->hjobs_off[i])) {
            (void)hipHostFree(s->hpool);
            (void)hipFree(s->dpool);
            delete s;
            return set_error(LF_EINVAL, "budget or staging too small for the job tables");
        }
    }
    for (int i = 0; i < lf_server::kSlots; ++i) {
        e = hipStreamCreateWithFlags(&s->hs[i], hipStreamNonBlocking);
        if (e != hipSuccess) {
            for (int j = 0; j < i; ++j) (void)hipStreamDestroy(s->hs[j]);
            (void)hipHostFree(s->hpool);
            (void)hipFree(s->dpool);
            delete s;
            return hip_error(e, "stream creation");
        }
    }
    s->worker = std::thread(service, s);
    *out = s;
    return LF_OK;
}

lf_status lf_submit_frame(lf_server *s, int32_t stream_id, const lf_params *p, const uint8_t *views, const float *S_P,
                          const float *mu_T, float *rgb_out, int32_t *d_out, float *q_out, lf_done_fn done,
                          void *user, int64_t *frame_id) {
    if (!s) return set_error(LF_EINVAL, "server is NULL");
    const Clock::time_point t_call = Clock::now();   // latency counts from the call
    lf_status st = validate_params(p);
    if (st != LF_OK) return st;
    if (stream_id < 0 || stream_id >= s->max_streams)
        return set_error(LF_EINVAL, "stream_id=%d outside [0,%d)", stream_id, s->max_streams);
    if (p->K > kServeMaxViews) return set_error(LF_EINVAL, "the server handles K <= %d views", kServeMaxViews);
    if (p->flags & (LF_INPUTS_ON_DEVICE | LF_OUTPUTS_ON_DEVICE | LF_EXHAUSTIVE_SWEEP))
        return set_error(LF_EINVAL, "the server takes host inputs and outputs, and of the flags only "
                                    "LF_PRIOR_WINDOW and LF_DYNAMIC_ONLY");
    if (!views || !S_P || !mu_T || !rgb_out) return set_error(LF_EINVAL, "views, S_P, mu_T and rgb_out are required");
    st = validate_host_values(p, S_P, mu_T, nullptr);
    if (st != LF_OK) return st;
    SrvFrame *f = new SrvFrame();
    f->p = *p;
    f->g = make_geometry(p);
    f->lambda = derived_lambda(p);
    f->stream = stream_id;
    f->rgb_out = rgb_out;
    f->d_out = d_out;
    f->q_out = q_out;
    f->done = done;
    f->user = user;
    f->tiles_x = (p->W + kServeTile - 1) / kServeTile;
    f->n_tiles = f->tiles_x * p->H;
    f->lds = frame_lds(*p, f->g);
    if (f->lds > s->lds_limit) {
        delete f;
        return set_error(LF_EINVAL, "disparity halo needs %zu bytes of LDS per tile, more than %zu", f->lds,
                         s->lds_limit);
    }
    const size_t HW = (size_t)p->H * p->W, KHW = HW * p->K;
    size_t o = 0;
    auto carve = [&](size_t bytes) { size_t r = o; o += RangeAllocator::round(bytes); return r; };
    f->in_views = carve(KHW * 3);
    f->in_sp = carve(KHW * 4);
    f->in_mu = carve(HW * 4);
    f->out_rgb = carve(HW * 12);
    f->out_d = carve(HW * 4);
    f->out_q = carve(KHW * 4);
    f->out_hole = carve(HW);
    f->h_bytes = o;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->sticky != LF_OK) {
            delete f;
            return set_error(s->sticky, "server failed earlier: %s", s->sticky_msg.c_str());
        }
        // a frame that could never fit the arenas is an argument error
        const size_t need = RangeAllocator::round(KHW * 3) + RangeAllocator::round(KHW * 4) +
                            RangeAllocator::round(HW * 4) + RangeAllocator::round(HW * 12) +
                            RangeAllocator::round(HW * 4) + RangeAllocator::round(HW) + RangeAllocator::round(KHW * 4);
        const size_t reserved = lf_server::kSlots * RangeAllocator::round(kMaxBatch * sizeof(ServeJob));
        if (f->h_bytes + reserved > s->halloc.size() || need + reserved > s->dalloc.size()) {
            delete f;
            return set_error(LF_EINVAL, "frame larger than the server's arenas");
        }
        if (!s->halloc.alloc(f->h_bytes, f->h_off)) {
            s->rejected += 1;
            delete f;
            return set_error(LF_EAGAIN, "staging full; retry when frames complete");
        }
        f->id = s->next_id++;
    }
    char *h = s->hpool + f->h_off;
    std::memcpy(h + f->in_views, views, KHW * 3);
    std::memcpy(h + f->in_sp, S_P, KHW * 4);
    std::memcpy(h + f->in_mu, mu_T, HW * 4);
    f->t_submit = t_call;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (!s->any) {
            s->any = true;
            s->t_first = f->t_submit;
        }
        s->submitted += 1;
        s->pending.push_back(f);
        if (frame_id) *frame_id = f->id;
    }
    s->cv.notify_one();
    return LF_OK;
}

lf_status lf_server_drain(lf_server *s) {
    if (!s) return set_error(LF_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv.notify_one();
    s->cv_idle.wait(lk, [&] { return s->pending.empty() && s->inflight.empty(); });
    if (s->sticky != LF_OK) return set_error(s->sticky, "%s", s->sticky_msg.c_str());
    return LF_OK;
}

lf_status lf_server_stats(lf_server *s, lf_server_stats_t *out) {
    if (!s || !out) return set_error(LF_EINVAL, "server or out is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(out, 0, sizeof *out);
    out->submitted = s->submitted;
    out->completed = s->completed;
    out->failed = s->failed;
    out->rejected = s->rejected;
    out->batches = s->batches;
    out->mean_batch_frames = s->batches ? (double)s->batch_frames / s->batches : 0.0;
    out->p50_ms = percentile(s->lat_ms, 0.50);
    out->p99_ms = percentile(s->lat_ms, 0.99);
    double sum = 0.0, mx = 0.0;
    for (double v : s->lat_ms) {
        sum += v;
        mx = std::max(mx, v);
    }
    out->mean_ms = s->lat_ms.empty() ? 0.0 : sum / s->lat_ms.size();
    out->max_ms = mx;
    out->wall_s = s->any ? std::chrono::duration<double>(s->t_last - s->t_first).count() : 0.0;
    out->frames_per_s = out->wall_s > 0 ? s->completed / out->wall_s : 0.0;
    out->hbm_in_use = (int64_t)s->dalloc.used();
    out->hbm_peak = (int64_t)s->dalloc.peak();
    return LF_OK;
}

lf_status lf_server_reset_stats(lf_server *s) {
    if (!s) return set_error(LF_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    s->submitted = s->completed = s->failed = s->rejected = s->batches = s->batch_frames = 0;
    s->lat_ms.clear();
    s->any = false;
    return LF_OK;
}

void lf_server_destroy(lf_server *s) {
    if (!s) return;
    (void)lf_server_drain(s);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (int i = 0; i < lf_server::kSlots; ++i) {
        (void)hipStreamSynchronize(s->hs[i]);
        (void)hipStreamDestroy(s->hs[i]);
    }
    (void)hipHostFree(s->hpool);
    (void)hipFree(s->dpool);
    delete s;
}

}  // extern "C"
