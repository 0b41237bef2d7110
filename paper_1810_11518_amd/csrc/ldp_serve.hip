// ldp_serve.hip -- continuous-batching request server (host code).
//
// Requests wait in arrival order until the device pool has room for their
// image, codes and histograms and a request slot is free.  A dispatcher
// thread admits as many waiting requests as fit (up to max_batch), copies
// their images to the pool and launches them as one persistent batch (a batch
// plan: device descriptor and work tables, device work queue, captured graph)
// on a free stream, then copies the results back.  Up to `depth` batches are
// in flight, so requests that arrive while earlier batches run are admitted as
// soon as memory and slots free up and run concurrently with them.  When a
// batch's completion event has fired its requests are reported done and their
// memory and slots are released.
//
// Pageable buffers go through a page-locked host mirror of the pool (same
// offsets and admission): the dispatcher packs a request's image into its
// mirror region, the kernel reads it there over the bus as it reads a
// page-locked caller's image and writes its codes and histograms there, and
// they are copied to the caller's buffers once the batch has finished.  No
// copy is enqueued: a copy from or to pageable memory would hold the
// dispatcher until it completes (results: until the batch has run), and every
// enqueued copy costs the dispatcher microseconds of runtime work.  The device
// pool serves pageable requests only when the mirror cannot be allocated.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include <sys/prctl.h>

#include "ldp_host.hpp"

namespace {

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

int64_t round256(int64_t n) { return (n + 255) & ~int64_t(255); }

// First-fit allocator over [0, size) with coalescing of neighbours.
class Pool {
public:
    explicit Pool(int64_t size) : size_(size) { free_[0] = size; }
    int64_t alloc(int64_t n)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                const int64_t off = it->first, rest = it->second - n;
                free_.erase(it);
                if (rest)
                    free_[off + n] = rest;
                used_ += n;
                return off;
            }
        }
        return -1;
    }
    void release(int64_t off, int64_t n)
    {
        used_ -= n;
        auto it = free_.emplace(off, n).first;
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
    int64_t used() const { return used_; }
    int64_t size() const { return size_; }

private:
    std::map<int64_t, int64_t> free_;
    int64_t size_, used_ = 0;
};

struct Req {
    int64_t id;
    const uint8_t *img;
    int32_t H, W;
    int64_t stride;
    uint8_t *codes;
    uint32_t *hist;
    // hist's device address when it is pinned host memory the GPU can write:
    // the kernel then writes the histograms there itself (no device copy and
    // no copy back); null otherwise
    uint32_t *hist_dev = nullptr;
    // the same for the image: the kernel reads it in place (no copy in)
    const uint8_t *img_dev = nullptr;
    double t_submit, t_admit = 0;
    int64_t off = -1, bytes = 0, img_bytes = 0, code_bytes = 0;
    bool waited_for_memory = false;
};

struct Batch {
    std::vector<Req *> reqs;
    int slot = -1;
    double t_launch = 0;
    int status = LDP_OK;
    bool staged = false;  // results are in the pool's page-locked mirror
};

}  // namespace

struct ldp_server {
    ldp_server_config cfg{};
    int64_t hist_bytes = 0;
    uint8_t *d_pool = nullptr;
    // page-locked mirror of d_pool for pageable requests (allocated at
    // creation for pools up to kEagerMirror bytes, else at first need; null if
    // that fails: such requests then copy from and to pageable memory directly)
    uint8_t *h_mirror = nullptr;
    uint8_t *d_mirror = nullptr;  // its address for the kernel
    bool mirror_tried = false;
    Pool *pool = nullptr;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    std::vector<ldp_batch_plan *> plans;
    std::vector<char> slot_busy;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Req *> pending;
    std::atomic<uint64_t> n_submitted{0};  // read by the dispatcher without the lock
    std::vector<Batch> inflight;
    std::deque<ldp_completion> done;
    int inflight_reqs = 0;
    bool stop = false;
    int64_t next_id = 0;
    ldp_server_stats st{};
    int device = 0;
    std::thread th;
};

namespace {

#ifndef LDP_SERVE_THREADS
#define LDP_SERVE_THREADS 1024
#endif
// Launch shape of the server's plans, for latency: batches are a few images,
// so each image is spread over many short lane tasks (one cell row per work
// item, row bands of >= 4 rows, large workgroups) rather than few long ones.
const ldp_tune kServeTune = {LDP_SERVE_THREADS, 0, 1, 0, {{INT64_MAX, 1, 4}}};

// The dispatcher spins (instead of sleeping) for this long after its last
// admission, launch or retirement, polling in slices of kSpinPollSeconds.
constexpr double kSpinSeconds = 200e-6;
constexpr double kSpinPollSeconds = 2e-6;

// Pools up to this size get their page-locked mirror at server creation.
constexpr int64_t kEagerMirror = int64_t(256) << 20;

uint8_t *mirror(ldp_server *s)
{
    if (s->cfg.flags & LDP_SERVER_NO_MIRROR)
        return nullptr;
    if (!s->h_mirror && !s->mirror_tried) {
        s->mirror_tried = true;
        void *d = nullptr;
        if (hipHostMalloc(&s->h_mirror, (size_t)s->cfg.pool_bytes) != hipSuccess) {
            s->h_mirror = nullptr;
            (void)hipGetLastError();
        } else if (hipHostGetDevicePointer(&d, s->h_mirror, 0) != hipSuccess || !d) {
            (void)hipGetLastError();
            (void)hipHostFree(s->h_mirror);
            s->h_mirror = nullptr;
        } else {
            s->d_mirror = static_cast<uint8_t *>(d);
        }
    }
    return s->h_mirror;
}

// Results of a finished batch from the pool's mirror to the callers' buffers.
void copy_out(ldp_server *s, const Batch &b)
{
    for (const Req *r : b.reqs) {
        const uint8_t *m = s->h_mirror + r->off + r->img_bytes;
        if (r->codes)
            std::memcpy(r->codes, m, (size_t)(r->H - 2) * (r->W - 2));
        if (!r->hist_dev)
            std::memcpy(r->hist, m + r->code_bytes, (size_t)s->hist_bytes);
    }
}

// Device work of one batch on its stream; returns a status.
int launch_batch(ldp_server *s, Batch &b)
{
    if (s->cfg.dry_run)
        return LDP_OK;
    hipStream_t st = s->streams[b.slot];
    bool copies = false;
    for (Req *r : b.reqs)
        copies = copies || r->bytes > 0;
    uint8_t *hm = copies ? mirror(s) : nullptr;
    b.staged = hm != nullptr;
    if (hm) {
        // The batch's pageable images packed into the mirror, which the
        // kernel then reads in place like a page-locked caller's image (and
        // writes codes and histograms to): no copy is enqueued at all.
        std::vector<ldp_image_desc> descs;
        descs.reserve(b.reqs.size());
        for (const Req *r : b.reqs) {
            uint8_t *m = hm + r->off, *dm = s->d_mirror + r->off;
            const uint8_t *img = r->img_dev;
            int64_t pitch = r->stride;
            if (!img) {
                if (r->stride == r->W)
                    std::memcpy(m, r->img, (size_t)r->H * r->W);
                else
                    for (int32_t y = 0; y < r->H; ++y)
                        std::memcpy(m + (size_t)y * r->W, r->img + (size_t)y * r->stride,
                                    (size_t)r->W);
                img = dm;
                pitch = r->W;
            }
            uint8_t *codes = r->codes ? dm + r->img_bytes : nullptr;
            uint32_t *hist = r->hist_dev ? r->hist_dev
                                         : reinterpret_cast<uint32_t *>(dm + r->img_bytes +
                                                                        r->code_bytes);
            descs.push_back({img, codes, hist, pitch, r->H, r->W});
        }
        const int rc = ldp::run_batch(s->plans[b.slot], descs.data(), (int32_t)descs.size(), st);
        if (rc != LDP_OK)
            return rc;
        return hipEventRecord(s->events[b.slot], st) == hipSuccess ? LDP_OK : LDP_ERR_HIP;
    }
    std::vector<ldp_image_desc> descs;
    descs.reserve(b.reqs.size());
    for (Req *r : b.reqs) {
        uint8_t *dimg = s->d_pool + r->off;
        uint8_t *dcodes = r->codes ? dimg + r->img_bytes : nullptr;
        uint32_t *dhist = r->hist_dev ? r->hist_dev
                                      : reinterpret_cast<uint32_t *>(dimg + r->img_bytes +
                                                                     r->code_bytes);
        if (r->img_dev) {
            descs.push_back({r->img_dev, dcodes, dhist, r->stride, r->H, r->W});
            continue;
        }
        const hipError_t e =
            r->stride == r->W
                ? hipMemcpyAsync(dimg, r->img, (size_t)r->H * r->W, hipMemcpyHostToDevice, st)
                : hipMemcpy2DAsync(dimg, r->W, r->img, r->stride, r->W, r->H,
                                   hipMemcpyHostToDevice, st);
        if (e != hipSuccess)
            return LDP_ERR_HIP;
        descs.push_back({dimg, dcodes, dhist, (int64_t)r->W, r->H, r->W});
    }
    int rc = ldp::run_batch(s->plans[b.slot], descs.data(), (int32_t)descs.size(), st);
    if (rc != LDP_OK)
        return rc;
    for (size_t i = 0; i < b.reqs.size(); ++i) {
        Req *r = b.reqs[i];
        if (!r->hist_dev &&
            hipMemcpyAsync(r->hist, descs[i].hist, s->hist_bytes, hipMemcpyDeviceToHost, st) !=
                hipSuccess)
            return LDP_ERR_HIP;
        if (r->codes && hipMemcpyAsync(r->codes, descs[i].codes, (size_t)(r->H - 2) * (r->W - 2),
                                       hipMemcpyDeviceToHost, st) != hipSuccess)
            return LDP_ERR_HIP;
    }
    return hipEventRecord(s->events[b.slot], st) == hipSuccess ? LDP_OK : LDP_ERR_HIP;
}

bool batch_finished(ldp_server *s, Batch &b, double t)
{
    if (s->cfg.dry_run)
        return t >= b.t_launch + s->cfg.dry_run_us * 1e-6;
    hipError_t e = hipEventQuery(s->events[b.slot]);
    if (e == hipErrorNotReady)
        return false;
    if (e != hipSuccess)
        b.status = LDP_ERR_HIP;
    return true;
}

void dispatcher(ldp_server *s)
{
    // timed waits of this thread end within ~1 us of their deadline instead
    // of the default 50 us timer slack (the completion polls below are 5 us)
    (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0UL, 0UL, 0UL);
    if (!s->cfg.dry_run)
        (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    double t_work = now_s();  // the last admission, launch or retirement
    for (;;) {
        bool progressed = false;
        // retire finished batches: copy staged results out (without the lock:
        // only this thread touches batches in flight, their pool regions and
        // slots), report, then free memory and slots
        double t = now_s();
        std::vector<Batch> fin;
        for (size_t i = 0; i < s->inflight.size();) {
            if (!batch_finished(s, s->inflight[i], t)) {
                ++i;
                continue;
            }
            fin.push_back(std::move(s->inflight[i]));
            s->inflight.erase(s->inflight.begin() + (long)i);
        }
        if (!fin.empty()) {
            bool staged = false;
            for (const Batch &b : fin)
                staged = staged || (b.staged && b.status == LDP_OK);
            if (staged) {
                lk.unlock();
                for (const Batch &b : fin)
                    if (b.staged && b.status == LDP_OK)
                        copy_out(s, b);
                t = now_s();
                lk.lock();
            }
            for (Batch &b : fin) {
                for (Req *r : b.reqs) {
                    if (r->bytes)
                        s->pool->release(r->off, r->bytes);
                    s->done.push_back({r->id, r->t_submit, r->t_admit, t, b.status,
                                       (int32_t)b.reqs.size()});
                    delete r;
                }
                s->inflight_reqs -= (int)b.reqs.size();
                s->st.completed += (int64_t)b.reqs.size();
                s->slot_busy[b.slot] = 0;
            }
            progressed = true;
        }
        if (progressed)
            s->cv_done.notify_all();
        // admit waiting requests in arrival order into a free launch slot
        int slot = -1;
        for (int i = 0; i < (int)s->slot_busy.size(); ++i)
            if (!s->slot_busy[i]) {
                slot = i;
                break;
            }
        if (slot >= 0 && !s->pending.empty()) {
            Batch b;
            b.slot = slot;
            while (!s->pending.empty() && (int)b.reqs.size() < s->cfg.max_batch &&
                   s->inflight_reqs + (int)b.reqs.size() < s->cfg.max_inflight) {
                Req *r = s->pending.front();
                // requests whose buffers are all read and written in place
                // need no pool space
                const int64_t off = r->bytes ? s->pool->alloc(r->bytes) : 0;
                if (off < 0) {
                    // head of line waits for memory
                    if (!r->waited_for_memory) {
                        r->waited_for_memory = true;
                        s->st.memory_waits += 1;
                    }
                    break;
                }
                r->off = off;
                r->t_admit = now_s();
                s->pending.pop_front();
                b.reqs.push_back(r);
            }
            if (!b.reqs.empty()) {
                s->slot_busy[slot] = 1;
                s->inflight_reqs += (int)b.reqs.size();
                s->st.peak_inflight = std::max(s->st.peak_inflight, s->inflight_reqs);
                s->st.peak_pool_bytes = std::max(s->st.peak_pool_bytes, s->pool->used());
                s->st.max_batch_seen = std::max(s->st.max_batch_seen, (int32_t)b.reqs.size());
                s->st.launches += 1;
                // device work without the lock: submit() keeps running
                lk.unlock();
                b.status = launch_batch(s, b);
                if (b.status != LDP_OK && !s->cfg.dry_run &&
                    hipEventRecord(s->events[slot], s->streams[slot]) != hipSuccess)
                    // copies enqueued before the failure may still write into
                    // this batch's pool regions: retire it only once they end
                    (void)hipStreamSynchronize(s->streams[slot]);
                b.t_launch = now_s();
                lk.lock();
                s->inflight.push_back(std::move(b));
                s->st.peak_batches = std::max(s->st.peak_batches, (int32_t)s->inflight.size());
                progressed = true;
            }
        }
        s->st.waiting = (int32_t)s->pending.size();
        if (s->stop && s->pending.empty() && s->inflight.empty())
            break;
        const double tnow = now_s();
        if (progressed) {
            t_work = tnow;
        } else if (!s->cfg.dry_run && tnow - t_work < kSpinSeconds) {
            // Busy within the last kSpinSeconds: spin for one short poll
            // interval with the lock released instead of sleeping, so a new
            // submission is admitted at once (a sleeping thread takes ~5-10
            // us to wake) and batches in flight are polled every ~2 us.
            const uint64_t seen = s->n_submitted.load(std::memory_order_acquire);
            lk.unlock();
            while (now_s() - tnow < kSpinPollSeconds &&
                   s->n_submitted.load(std::memory_order_acquire) == seen)
                __builtin_ia32_pause();
            lk.lock();
        } else if (s->inflight.empty()) {
            // idle: wait for a submission
            s->cv_work.wait_for(lk, std::chrono::milliseconds(2));
        } else {
            // batches in flight: poll their events every 5 us, and wake at
            // once for a submission
            s->cv_work.wait_for(lk, std::chrono::microseconds(5));
        }
    }
}

void release_server(ldp_server *s)
{
    for (ldp_batch_plan *p : s->plans)
        if (p)
            ldp_batch_plan_destroy(p);
    for (hipEvent_t e : s->events)
        if (e)
            (void)hipEventDestroy(e);
    for (hipStream_t st : s->streams)
        if (st)
            (void)hipStreamDestroy(st);
    if (s->d_pool)
        (void)hipFree(s->d_pool);
    if (s->h_mirror)
        (void)hipHostFree(s->h_mirror);
    delete s->pool;
    for (Req *r : s->pending)
        delete r;
    delete s;
}

}  // namespace

extern "C" {

double ldp_now(void) { return now_s(); }

int ldp_server_create(ldp_server **out, const ldp_server_config *cfg)
{
    if (!out || !cfg)
        return LDP_ERR_INVALID_ARG;
    *out = nullptr;
    const ldp_server_config c = *cfg;
    if (c.pool_bytes < 4096 || c.max_inflight < 1 || c.max_batch < 1 || c.depth < 1 ||
        c.depth > 8 || c.k < 1 || c.k > 8 || c.cells_y < 1 || c.cells_x < 1 ||
        c.cells_y > LDP_MAX_SIDE - 2 || c.cells_x > LDP_MAX_SIDE - 2 || c.dry_run_us < 0 ||
        (c.flags & ~LDP_SERVER_NO_MIRROR) != 0)
        return LDP_ERR_INVALID_ARG;
    ldp_server *s = new (std::nothrow) ldp_server();
    if (!s)
        return LDP_ERR_NO_MEMORY;
    s->cfg = c;
    s->hist_bytes = (int64_t)c.cells_y * c.cells_x * 256 * 4;
    s->pool = new Pool(c.pool_bytes);
    s->slot_busy.assign(c.depth, 0);
    if (!c.dry_run) {
        if (hipGetDevice(&s->device) != hipSuccess) {
            release_server(s);
            return LDP_ERR_HIP;
        }
        if (hipMalloc(&s->d_pool, (size_t)c.pool_bytes) != hipSuccess) {
            release_server(s);
            return LDP_ERR_NO_MEMORY;
        }
        if (c.pool_bytes <= kEagerMirror)
            (void)mirror(s);
        for (int i = 0; i < c.depth; ++i) {
            hipStream_t st = nullptr;
            hipEvent_t ev = nullptr;
            ldp_batch_plan *p = nullptr;
            if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
                if (st)
                    (void)hipStreamDestroy(st);
                release_server(s);
                return LDP_ERR_HIP;
            }
            s->streams.push_back(st);
            s->events.push_back(ev);
            // pixel capacity independent of the pool: images read in place
            // take no pool space, so a batch's pixels are bounded only by
            // max_batch images of the largest side
            const int64_t max_px = (int64_t)c.max_batch * LDP_MAX_SIDE * LDP_MAX_SIDE;
            int rc = ldp_batch_plan_create(&p, c.max_batch, max_px, c.k, c.cells_y, c.cells_x,
                                           &kServeTune);
            if (rc != LDP_OK) {
                release_server(s);
                return rc;
            }
            s->plans.push_back(p);
        }
        // Warm every launch slot: the first graph launch and the first copies
        // on a stream pay one-time runtime set-up (milliseconds), which would
        // otherwise land on the first requests that reach a slot once the
        // load spreads over several slots.
        uint8_t *h = nullptr;
        if (hipHostMalloc(&h, 4096) != hipSuccess) {
            release_server(s);
            return LDP_ERR_NO_MEMORY;
        }
        int wrc = LDP_OK;
        for (int i = 0; i < c.depth && wrc == LDP_OK; ++i) {
            hipStream_t st = s->streams[i];
            wrc = ldp::warm_plan(s->plans[i], st);
            if (wrc == LDP_OK &&
                (hipMemcpyAsync(s->d_pool, h, 4096, hipMemcpyHostToDevice, st) != hipSuccess ||
                 hipMemcpy2DAsync(s->d_pool, 32, h, 64, 32, 8, hipMemcpyHostToDevice, st) !=
                     hipSuccess ||
                 hipMemcpyAsync(h, s->d_pool, 4096, hipMemcpyDeviceToHost, st) != hipSuccess ||
                 hipStreamSynchronize(st) != hipSuccess))
                wrc = LDP_ERR_HIP;
        }
        (void)hipHostFree(h);
        if (wrc != LDP_OK) {
            release_server(s);
            return wrc;
        }
    }
    s->th = std::thread(dispatcher, s);
    *out = s;
    return LDP_OK;
}

int ldp_server_submit(ldp_server *s, const uint8_t *img, int32_t H, int32_t W, int64_t stride,
                      uint8_t *codes, uint32_t *hist, int64_t *id)
{
    if (!s || !img || !hist || !id || H < 3 || W < 3 || H > LDP_MAX_SIDE || W > LDP_MAX_SIDE ||
        stride < W || H - 2 < s->cfg.cells_y || W - 2 < s->cfg.cells_x)
        return LDP_ERR_INVALID_ARG;
    if ((int64_t)(H - 1) * W + W + 8 > ldp::kMaxExtent)
        return LDP_ERR_UNSUPPORTED;
    Req *r = new (std::nothrow) Req();
    if (!r)
        return LDP_ERR_NO_MEMORY;
    r->img = img;
    r->H = H;
    r->W = W;
    r->stride = stride;
    r->codes = codes;
    r->hist = hist;
    if (!s->cfg.dry_run) {
        // pinned host memory mapped for the GPU at its host address (unified
        // addressing): the kernel writes the histograms to `hist` itself
        hipPointerAttribute_t at{};
        if (hipPointerGetAttributes(&at, hist) == hipSuccess) {
            if (at.type == hipMemoryTypeHost && at.devicePointer != nullptr &&
                at.devicePointer == at.hostPointer)
                r->hist_dev = hist;
        } else {
            (void)hipGetLastError();  // leave no error from the query for the caller's next call
        }
        // and the image: read in place by the kernel, with its own pitch
        // (when that extent fits the kernel's 32-bit offsets)
        hipPointerAttribute_t ai{};
        if (hipPointerGetAttributes(&ai, img) == hipSuccess) {
            if (ai.type == hipMemoryTypeHost && ai.devicePointer != nullptr &&
                ai.devicePointer == ai.hostPointer &&
                (int64_t)(H - 1) * stride + W + 8 <= ldp::kMaxExtent)
                r->img_dev = img;
        } else {
            (void)hipGetLastError();
        }
    }
    r->img_bytes = r->img_dev ? 0 : round256((int64_t)H * W);
    r->code_bytes = codes ? round256((int64_t)(H - 2) * (W - 2)) : 0;
    r->bytes = r->img_bytes + r->code_bytes + (r->hist_dev ? 0 : round256(s->hist_bytes));
    std::lock_guard<std::mutex> lk(s->mu);
    if (r->bytes > s->pool->size()) {
        s->st.rejected += 1;
        delete r;
        return LDP_ERR_NO_MEMORY;
    }
    r->id = s->next_id++;
    r->t_submit = now_s();
    *id = r->id;
    s->pending.push_back(r);
    s->st.submitted += 1;
    s->n_submitted.fetch_add(1, std::memory_order_release);
    s->cv_work.notify_one();
    return LDP_OK;
}

int ldp_server_poll(ldp_server *s, ldp_completion *out, int32_t max, int32_t *n, int32_t wait_us)
{
    if (!s || !n || max < 0 || (max > 0 && !out))
        return LDP_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->done.empty() && wait_us > 0)
        s->cv_done.wait_for(lk, std::chrono::microseconds(wait_us),
                            [&] { return !s->done.empty(); });
    int32_t k = 0;
    while (k < max && !s->done.empty()) {
        out[k++] = s->done.front();
        s->done.pop_front();
    }
    *n = k;
    return LDP_OK;
}

int ldp_server_stats_get(ldp_server *s, ldp_server_stats *stats)
{
    if (!s || !stats)
        return LDP_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    *stats = s->st;
    stats->waiting = (int32_t)s->pending.size();
    return LDP_OK;
}

int ldp_server_destroy(ldp_server *s)
{
    if (!s)
        return LDP_ERR_INVALID_ARG;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_work.notify_one();
    }
    if (s->th.joinable())
        s->th.join();
    release_server(s);
    return LDP_OK;
}

}  // extern "C"
