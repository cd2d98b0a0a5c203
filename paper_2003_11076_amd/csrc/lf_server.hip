// Frame server: continuous batching of light-field frames from many streams.
//
// Frames are submitted by any thread.  Host inputs are copied into a pinned
// staging arena at submission (when it is full the call returns LF_EAGAIN);
// device inputs are used in place.  A pool of workers, each with its own HIP
// stream, serves the queue: a free worker admits, in arrival order, every
// pending frame that shares the oldest admissible frame's kernel key
// (storage, view count, sweep kind), whose stream has no frame running and
// whose buffers fit the HBM budget, and runs them as one batch: host->device
// copies, one kernel launch covering all (frame, row tile) pairs, device->
// host copies.  Batches of different workers overlap on the device; frames
// that arrive while others run join the next batch.  When a batch's stream
// has finished, the worker copies host outputs out of the staging (holding
// no lock), releases memory, keeps each frame's weights on the device as its
// stream's warm start, and runs the callbacks.  Kernel boundaries give each
// batch a coherent view of the inputs the copies wrote.
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
#include <string>
#include <atomic>
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
    void reset_peak() { peak_ = used_; }

  private:
    std::map<size_t, size_t> free_;
    size_t size_ = 0, used_ = 0, peak_ = 0;
};

using Clock = std::chrono::steady_clock;

ServeKernel pick_serve(int storage, int K, int kind) {
    switch (storage) {
        case LF_F32: return K <= 5 ? pick_serve_f32_a(K, kind) : pick_serve_f32_b(K, kind);
        case LF_F16: return K <= 5 ? pick_serve_f16_a(K, kind) : pick_serve_f16_b(K, kind);
        default: return K <= 5 ? pick_serve_bf16_a(K, kind) : pick_serve_bf16_b(K, kind);
    }
}

struct SrvFrame {
    int64_t id;
    int stream;
    lf_params p;
    Geometry g;
    float lambda;
    int kind, key;            // sweep kind; kernel key (storage, K, kind): frames of one key share launches
    bool dev_in, dev_out;
    const uint8_t *views;     // caller's device inputs (dev_in)
    const float *S_P, *mu_T;
    float *rgb_out;
    int32_t *d_out;
    float *q_out;
    lf_done_fn done;
    void *user;
    // pinned staging: host inputs, then host outputs
    size_t h_off = 0, h_bytes = 0;
    size_t in_views = 0, in_sp = 0, in_mu = 0, out_rgb = 0, out_d = 0, out_q = 0;
    // device frame block: host inputs, and the outputs the caller does not
    // take in device memory
    size_t d_off = 0, d_bytes = 0;
    size_t o_views = 0, o_sp = 0, o_mu = 0, o_rgb = 0, o_d = 0;
    bool rgb_internal = false, d_internal = false;
    // the stream's weights block (K*H*W floats)
    size_t q_bytes = 0;
    bool warm = false;
    int tiles_x = 0, n_tiles = 0;
    size_t lds = 0;
    int rows_in_place = 0;   // R+G+B rows staged inside the record windows
    Clock::time_point t_submit, t_done;
    lf_status status = LF_OK;
};

struct SrvStream {
    bool busy = false;      // a frame of the stream is admitted and not yet finished
    bool has_q = false;     // a weights block of shape (K, H, W) is held
    bool warm = false;      // it holds a finished frame's weights
    int K = 0, H = 0, W = 0;
    size_t q_off = 0, q_bytes = 0;
    int64_t last_use = 0;   // completion order, for evicting the oldest warm start
};

constexpr size_t kMaxBatch = 16;
constexpr int kWorkers = 4;
constexpr int kIdleSpinUs = 200;   // an idle worker polls for new frames this long before sleeping

struct SrvWorker {
    hipStream_t hs = nullptr;
    size_t djobs_off = 0, hjobs_off = 0;   // job table + per-job invalid-value counters
    std::thread th;
};

size_t job_area_bytes() { return kMaxBatch * sizeof(ServeJob) + kMaxBatch * sizeof(uint32_t); }

}  // namespace lfem

using namespace lfem;

struct lf_server {
    int device = 0;
    int n_iters = 8;
    int max_streams = 1;
    size_t lds_limit = 65536;
    char *dpool = nullptr;        // device arena
    RangeAllocator dalloc;
    char *hpool = nullptr;        // pinned staging arena
    RangeAllocator halloc;
    SrvWorker workers[kWorkers];
    std::vector<SrvStream> streams;
    std::deque<SrvFrame *> pending;
    int inflight = 0;             // batches admitted and not yet finished
    bool hold = false;            // admission held (lf_server_hold)
    int64_t use_clock = 0;
    std::mutex mu;
    std::condition_variable cv, cv_idle;
    std::atomic<int64_t> arrivals{0};   // frames submitted (read by idle workers without the lock)
    bool stop = false;
    int64_t next_id = 0;
    // statistics
    int64_t submitted = 0, completed = 0, failed = 0, rejected = 0, batches = 0, batch_frames = 0, max_batch = 0;
    std::vector<double> lat_ms;
    Clock::time_point t_first, t_last;
    bool any = false;
    lf_status sticky = LF_OK;
    std::string sticky_msg;
};

namespace {

// LDS of a tile: the descriptor records of every view's window, then three
// int16 rows of intensity sums of one window at a time (+1 column of border
// on each side).
// LDS of a frame's blocks (8-byte records), and whether its R+G+B rows are
// staged in place: only when the scratch area after the records would leave
// a CU's LDS (160 KiB) fewer blocks than its registers allow (six two-wave
// blocks at three waves per SIMD up to six views, four above), since the
// in-place staging costs a barrier and registers per view.
size_t frame_lds(const lf_params &p, const Geometry &g, int *rows_in_place) {
    const int tile = serve_tile_width(p.K);
    const size_t pairs = em_window_pairs(&p, g, tile);
    const size_t widest = em_window_widest(&p, g, tile);
    const size_t rows = 2 * 3 * (widest + 2);
    const size_t with_rows = pairs * 8 + rows + 64;
    const size_t blocks = p.K <= 6 ? 6 : 4;
    if ((size_t)160 * 1024 / with_rows >= blocks || widest > (size_t)kServeHold * tile) {
        *rows_in_place = 0;
        return with_rows;
    }
    *rows_in_place = 1;
    return pairs * 8 + 64;
}

int frame_kind(const lf_params &p, const Geometry &g) {
    if (g.frac) return kServeFrac;
    if (p.flags & LF_PRIOR_WINDOW) return kServeLane;
    return g.sym ? kServeSharedSym : kServeShared;
}

// Admit one frame (lock held): its device block, and its stream's weights
// block (used in place by a frame of the same shape).  When nothing in flight
// will free memory (can_evict), the oldest warm starts of idle streams are
// given up until it fits, this stream's own last.
bool admit(lf_server *s, SrvFrame *f, SrvStream &ss, bool can_evict) {
    const lf_params &p = f->p;
    if (ss.has_q && !(ss.K == p.K && ss.H == p.H && ss.W == p.W)) {
        s->dalloc.release(ss.q_off, ss.q_bytes);   // shape changed: the stream starts cold
        ss.has_q = ss.warm = false;
    }
    for (;;) {
        size_t doff = 0, qoff = 0;
        bool ok = f->d_bytes == 0 || s->dalloc.alloc(f->d_bytes, doff);
        if (ok && !ss.has_q) {
            ok = s->dalloc.alloc(f->q_bytes, qoff);
            if (!ok && f->d_bytes) s->dalloc.release(doff, f->d_bytes);
        }
        if (ok) {
            f->d_off = doff;
            if (!ss.has_q) {
                ss.has_q = true;
                ss.warm = false;
                ss.K = p.K;
                ss.H = p.H;
                ss.W = p.W;
                ss.q_off = qoff;
                ss.q_bytes = f->q_bytes;
            }
            f->warm = ss.warm;
            return true;
        }
        if (!can_evict) return false;
        SrvStream *victim = nullptr;
        for (SrvStream &o : s->streams)
            if (o.has_q && !o.busy && &o != &ss && (!victim || o.last_use < victim->last_use)) victim = &o;
        if (!victim && ss.has_q) victim = &ss;
        if (!victim) return false;
        s->dalloc.release(victim->q_off, victim->q_bytes);
        victim->has_q = victim->warm = false;
    }
}

// Form a batch (lock held): pending frames in arrival order with the key of
// the first admissible one; a stream's frames stay in submission order.
void form_batch(lf_server *s, std::vector<SrvFrame *> &b) {
    int key = -1;
    std::vector<char> blocked((size_t)s->max_streams, 0);
    for (auto it = s->pending.begin(); it != s->pending.end() && b.size() < kMaxBatch;) {
        SrvFrame *f = *it;
        SrvStream &ss = s->streams[f->stream];
        if (ss.busy || blocked[f->stream] || (key >= 0 && f->key != key)) {
            blocked[f->stream] = 1;
            ++it;
            continue;
        }
        if (!admit(s, f, ss, b.empty() && s->inflight == 0)) break;   // memory: keep arrival order
        key = f->key;
        ss.busy = true;
        b.push_back(f);
        it = s->pending.erase(it);
    }
}

// Queue one batch on the worker's stream and wait for it (no lock held).
bool run_batch(lf_server *s, SrvWorker &wk, std::vector<SrvFrame *> &b, std::string &err) {
    const hipStream_t st = wk.hs;
    const size_t nj = b.size();
    ServeJob *hj = reinterpret_cast<ServeJob *>(s->hpool + wk.hjobs_off);
    ServeJob *dj = reinterpret_cast<ServeJob *>(s->dpool + wk.djobs_off);
    uint32_t *hbad = reinterpret_cast<uint32_t *>(s->hpool + wk.hjobs_off + kMaxBatch * sizeof(ServeJob));
    uint32_t *dbad = reinterpret_cast<uint32_t *>(s->dpool + wk.djobs_off + kMaxBatch * sizeof(ServeJob));
    int tiles = 0;
    size_t lds = 0;
    hipError_t e = hipSuccess;
    for (size_t i = 0; i < nj; ++i) {
        SrvFrame *f = b[i];
        const lf_params &p = f->p;
        const size_t HW = (size_t)p.H * p.W, KHW = HW * p.K;
        char *h = s->hpool + f->h_off;
        char *d = s->dpool + f->d_off;
        ServeJob &J = hj[i];
        std::memset(&J, 0, sizeof J);
        J.em = make_em_args(&p, f->g, f->lambda);
        J.em.tile = serve_tile_width(p.K);
        J.em.n_iters = s->n_iters;
        J.views = f->dev_in ? f->views : reinterpret_cast<const uint8_t *>(d + f->o_views);
        J.S_P = f->dev_in ? f->S_P : reinterpret_cast<const float *>(d + f->o_sp);
        J.em.mu_T = f->dev_in ? f->mu_T : reinterpret_cast<const float *>(d + f->o_mu);
        J.rgb = f->rgb_internal ? reinterpret_cast<float *>(d + f->o_rgb) : f->rgb_out;
        J.em.d_idx = f->d_internal ? reinterpret_cast<int32_t *>(d + f->o_d) : f->d_out;
        J.em.q = reinterpret_cast<float *>(s->dpool + s->streams[f->stream].q_off);
        J.q_out = f->dev_out ? f->q_out : nullptr;
        J.bad = dbad + i;
        J.warm = f->warm ? 1 : 0;
        J.check = f->dev_in ? 1 : 0;
        J.rows_in_place = f->rows_in_place;
        J.ref = p.ref;
        J.tiles_x = f->tiles_x;
        J.tile_start = tiles;
        J.n_tiles = f->n_tiles;
        J.tau = p.tau_init;
        hbad[i] = 0;
        tiles += (f->n_tiles + 7) & ~7;   // the next frame's blocks start at a multiple of 8
        lds = std::max(lds, f->lds);
        if (!f->dev_in) {
            e = hipMemcpyAsync(d + f->o_views, h + f->in_views, KHW * 3, hipMemcpyHostToDevice, st);
            if (e == hipSuccess) e = hipMemcpyAsync(d + f->o_sp, h + f->in_sp, KHW * 4, hipMemcpyHostToDevice, st);
            if (e == hipSuccess) e = hipMemcpyAsync(d + f->o_mu, h + f->in_mu, HW * 4, hipMemcpyHostToDevice, st);
            if (e != hipSuccess) break;
        }
    }
    // the job table and the zeroed counters in one copy
    if (e == hipSuccess) e = hipMemcpyAsync(dj, hj, job_area_bytes(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        ServeKernel k = pick_serve(b[0]->p.storage, b[0]->p.K, b[0]->kind);
        if (!k) {
            err = "no kernel instance for the frame";
            return false;
        }
        hipLaunchKernelGGL(k, dim3(tiles), dim3(serve_tile_width(b[0]->p.K)), lds, st, dj, (int)nj);
        e = hipGetLastError();
    }
    for (size_t i = 0; i < nj && e == hipSuccess; ++i) {
        SrvFrame *f = b[i];
        if (f->dev_out) continue;
        const lf_params &p = f->p;
        const size_t HW = (size_t)p.H * p.W, KHW = HW * p.K;
        char *h = s->hpool + f->h_off;
        char *d = s->dpool + f->d_off;
        e = hipMemcpyAsync(h + f->out_rgb, d + f->o_rgb, HW * 12, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess && f->d_out) e = hipMemcpyAsync(h + f->out_d, d + f->o_d, HW * 4, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess && f->q_out)
            e = hipMemcpyAsync(h + f->out_q, s->dpool + s->streams[f->stream].q_off, KHW * 4, hipMemcpyDeviceToHost,
                               st);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(hbad, dbad, nj * sizeof(uint32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        err = hipGetErrorString(e);
        (void)hipGetLastError();
        return false;
    }
    for (size_t i = 0; i < nj; ++i) {
        SrvFrame *f = b[i];
        if (hbad[i]) {
            f->status = set_error(LF_EINVAL, "frame %lld: %u input values invalid (S_P outside [0,1] or mu_T not "
                                             "finite)", (long long)f->id, hbad[i]);
            continue;
        }
        if (f->dev_out) continue;
        // host outputs out of the staging (no lock held)
        const lf_params &p = f->p;
        const size_t HW = (size_t)p.H * p.W, KHW = HW * p.K;
        const char *h = s->hpool + f->h_off;
        std::memcpy(f->rgb_out, h + f->out_rgb, HW * 12);
        if (f->d_out) std::memcpy(f->d_out, h + f->out_d, HW * 4);
        if (f->q_out) std::memcpy(f->q_out, h + f->out_q, KHW * 4);
    }
    return true;
}

// Finish a batch (lock held): memory, warm starts, statistics.
void finish_batch(lf_server *s, std::vector<SrvFrame *> &b, bool ok) {
    for (SrvFrame *f : b) {
        SrvStream &ss = s->streams[f->stream];
        if (!ok && f->status == LF_OK) f->status = LF_EDEVICE;
        if (f->status == LF_OK) {
            ss.warm = true;          // the frame's weights are the stream's warm start
            ss.last_use = ++s->use_clock;
        } else if (ss.has_q) {
            s->dalloc.release(ss.q_off, ss.q_bytes);   // weights of a failed frame are not kept
            ss.has_q = ss.warm = false;
        }
        if (f->d_bytes) s->dalloc.release(f->d_off, f->d_bytes);
        if (f->h_bytes) s->halloc.release(f->h_off, f->h_bytes);
        ss.busy = false;
        f->t_done = Clock::now();
    }
}

void record(lf_server *s, std::vector<SrvFrame *> &b) {
    for (SrvFrame *f : b) {
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
}

void worker_main(lf_server *s, int wi) {
    (void)hipSetDevice(s->device);
    SrvWorker &wk = s->workers[wi];
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        std::vector<SrvFrame *> b;
        bool spun = false;
        for (;;) {
            if (s->sticky != LF_OK) {
                // after a device failure every pending frame fails
                while (!s->pending.empty() && b.size() < kMaxBatch) {
                    SrvFrame *f = s->pending.front();
                    s->pending.pop_front();
                    f->status = s->sticky;
                    f->t_done = Clock::now();
                    b.push_back(f);
                }
                if (!b.empty()) break;
            } else if (!s->hold) {
                form_batch(s, b);
                if (!b.empty()) break;
            }
            if (s->stop && s->pending.empty() && s->inflight == 0) return;
            if (!spun) {
                // a short spin before sleeping: a frame submitted within
                // kIdleSpinUs of the worker going idle starts without the
                // wake-up latency of the wait
                spun = true;
                const int64_t seen = s->arrivals.load(std::memory_order_relaxed);
                lk.unlock();
                const Clock::time_point until = Clock::now() + std::chrono::microseconds(kIdleSpinUs);
                while (s->arrivals.load(std::memory_order_acquire) == seen && Clock::now() < until)
                    std::this_thread::yield();
                lk.lock();
                continue;
            }
            s->cv.wait(lk);
        }
        const bool failed_early = s->sticky != LF_OK;
        if (!failed_early) {
            s->inflight += 1;
            s->batches += 1;
            s->batch_frames += (int64_t)b.size();
            s->max_batch = std::max<int64_t>(s->max_batch, (int64_t)b.size());
            lk.unlock();
            std::string err;
            const bool ok = run_batch(s, wk, b, err);
            lk.lock();
            if (!ok && s->sticky == LF_OK) {
                s->sticky = LF_EDEVICE;
                s->sticky_msg = "batch: " + err;
            }
            finish_batch(s, b, ok);
            s->inflight -= 1;
        }
        // memory was released: other workers may admit now
        s->cv.notify_all();
        lk.unlock();
        for (SrvFrame *f : b)
            if (f->done) f->done(f->id, f->status, f->user);
        lk.lock();
        record(s, b);
        s->cv_idle.notify_all();
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

void server_free(lf_server *s) {
    for (SrvWorker &w : s->workers)
        if (w.hs) (void)hipStreamDestroy(w.hs);
    if (s->hpool) (void)hipHostFree(s->hpool);
    if (s->dpool) (void)hipFree(s->dpool);
    delete s;
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
    staging_bytes = std::max(staging_bytes, kWorkers * RangeAllocator::round(job_area_bytes()));
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
        s->dpool = nullptr;
        server_free(s);
        return set_error(LF_ENOMEM, "HBM arena of %zu bytes: %s", hbm_budget_bytes, hipGetErrorString(e));
    }
    s->dalloc.reset(hbm_budget_bytes);
    e = hipHostMalloc((void **)&s->hpool, staging_bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
        s->hpool = nullptr;
        server_free(s);
        return set_error(LF_ENOMEM, "pinned staging of %zu bytes: %s", staging_bytes, hipGetErrorString(e));
    }
    s->halloc.reset(staging_bytes);
    for (SrvWorker &w : s->workers) {
        if (!s->dalloc.alloc(job_area_bytes(), w.djobs_off) || !s->halloc.alloc(job_area_bytes(), w.hjobs_off)) {
            server_free(s);
            return set_error(LF_EINVAL, "budget or staging too small for the job tables");
        }
        e = hipStreamCreateWithFlags(&w.hs, hipStreamNonBlocking);
        if (e != hipSuccess) {
            w.hs = nullptr;
            server_free(s);
            return hip_error(e, "stream creation");
        }
    }
    for (int i = 0; i < kWorkers; ++i) s->workers[i].th = std::thread(worker_main, s, i);
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
    if (p->flags & (LF_EXHAUSTIVE_SWEEP | LF_DEFERRED_CHECK))
        return set_error(LF_EINVAL, "the server takes of the flags only LF_INPUTS_ON_DEVICE, LF_OUTPUTS_ON_DEVICE, "
                                    "LF_PRIOR_WINDOW and LF_DYNAMIC_ONLY");
    if (!views || !S_P || !mu_T || !rgb_out) return set_error(LF_EINVAL, "views, S_P, mu_T and rgb_out are required");
    SrvFrame *f = new SrvFrame();
    f->p = *p;
    f->dev_in = (p->flags & LF_INPUTS_ON_DEVICE) != 0;
    f->dev_out = (p->flags & LF_OUTPUTS_ON_DEVICE) != 0;
    if (!f->dev_in) {
        st = validate_host_values(p, S_P, mu_T, nullptr);
        if (st != LF_OK) {
            delete f;
            return st;
        }
    }
    f->g = make_geometry(p);
    f->lambda = derived_lambda(p);
    f->kind = frame_kind(*p, f->g);
    f->key = (p->storage * (kServeMaxViews + 1) + p->K) * kServeKinds + f->kind;
    f->stream = stream_id;
    f->views = views;
    f->S_P = S_P;
    f->mu_T = mu_T;
    f->rgb_out = rgb_out;
    f->d_out = d_out;
    f->q_out = q_out;
    f->done = done;
    f->user = user;
    f->tiles_x = (p->W + serve_tile_width(p->K) - 1) / serve_tile_width(p->K);
    f->n_tiles = f->tiles_x * p->H;
    f->lds = frame_lds(*p, f->g, &f->rows_in_place);
    if (f->lds > s->lds_limit) {
        delete f;
        return set_error(LF_EINVAL, "disparity halo needs %zu bytes of LDS per tile, more than %zu", f->lds,
                         s->lds_limit);
    }
    const size_t HW = (size_t)p->H * p->W, KHW = HW * p->K;
    {
        size_t o = 0;
        auto carve = [&](size_t bytes) { size_t r = o; o += RangeAllocator::round(bytes); return r; };
        if (!f->dev_in) {
            f->in_views = carve(KHW * 3);
            f->in_sp = carve(KHW * 4);
            f->in_mu = carve(HW * 4);
        }
        if (!f->dev_out) {
            f->out_rgb = carve(HW * 12);
            if (d_out) f->out_d = carve(HW * 4);
            if (q_out) f->out_q = carve(KHW * 4);
        }
        f->h_bytes = o;
    }
    {
        size_t o = 0;
        auto carve = [&](size_t bytes) { size_t r = o; o += RangeAllocator::round(bytes); return r; };
        if (!f->dev_in) {
            f->o_views = carve(KHW * 3);
            f->o_sp = carve(KHW * 4);
            f->o_mu = carve(HW * 4);
        }
        f->rgb_internal = !f->dev_out;
        f->d_internal = !f->dev_out || !d_out;
        if (f->rgb_internal) f->o_rgb = carve(HW * 12);
        if (f->d_internal) f->o_d = carve(HW * 4);
        f->d_bytes = o;
    }
    f->q_bytes = KHW * 4;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->sticky != LF_OK) {
            delete f;
            return set_error(s->sticky, "server failed earlier: %s", s->sticky_msg.c_str());
        }
        // a frame that could never fit the arenas is an argument error (with
        // every other stream's weights given up, a frame needs its own
        // block and its stream's weights)
        const size_t reserved = kWorkers * RangeAllocator::round(job_area_bytes());
        if (f->h_bytes + reserved > s->halloc.size() ||
            RangeAllocator::round(f->d_bytes) + RangeAllocator::round(f->q_bytes) + reserved > s->dalloc.size()) {
            delete f;
            return set_error(LF_EINVAL, "frame larger than the server's arenas");
        }
        if (f->h_bytes && !s->halloc.alloc(f->h_bytes, f->h_off)) {
            s->rejected += 1;
            delete f;
            return set_error(LF_EAGAIN, "staging full; retry when frames complete");
        }
        f->id = s->next_id++;
    }
    if (!f->dev_in) {
        char *h = s->hpool + f->h_off;
        std::memcpy(h + f->in_views, views, KHW * 3);
        std::memcpy(h + f->in_sp, S_P, KHW * 4);
        std::memcpy(h + f->in_mu, mu_T, HW * 4);
    }
    f->t_submit = t_call;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (!s->any) {
            s->any = true;
            s->t_first = f->t_submit;
        }
        s->submitted += 1;
        s->pending.push_back(f);
        s->arrivals.fetch_add(1, std::memory_order_release);
        if (frame_id) *frame_id = f->id;
    }
    s->cv.notify_one();
    return LF_OK;
}

lf_status lf_server_hold(lf_server *s, int32_t hold) {
    if (!s) return set_error(LF_EINVAL, "server is NULL");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->hold = hold != 0;
    }
    s->cv.notify_all();
    return LF_OK;
}

lf_status lf_server_drain(lf_server *s) {
    if (!s) return set_error(LF_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    s->hold = false;   // a held queue could never drain
    s->cv.notify_all();
    s->cv_idle.wait(lk, [&] { return s->pending.empty() && s->inflight == 0; });
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
    out->max_batch_frames = s->max_batch;
    return LF_OK;
}

lf_status lf_server_reset_stats(lf_server *s) {
    if (!s) return set_error(LF_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    s->submitted = s->completed = s->failed = s->rejected = s->batches = s->batch_frames = s->max_batch = 0;
    s->lat_ms.clear();
    s->any = false;
    s->dalloc.reset_peak();
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
    for (SrvWorker &w : s->workers)
        if (w.th.joinable()) w.th.join();
    for (SrvWorker &w : s->workers)
        if (w.hs) (void)hipStreamSynchronize(w.hs);
    server_free(s);
}

}  // extern "C"
