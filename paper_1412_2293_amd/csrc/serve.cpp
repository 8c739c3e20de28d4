// Request server: continuous batching of trajectory requests on one GPU.
//
// Requests (a circuit, its noise, a trajectory count) arrive from any host thread.  Each is
// validated and planned at submission and split into trajectory batches of one fixed size.
// A worker thread admits batches in arrival order whenever a stream slot is idle and the
// caller's device pool has a free range large enough for the batch.  Each batch runs on its
// own HIP stream, so batches of different requests overlap on the device, and a request that
// arrives while others run starts as soon as a slot and memory free up.  Admission never
// lets the bytes in use exceed the pool.
//
// Every trajectory's result depends only on the circuit, the noise parameters, its global
// trajectory index and the plan.  The batch split, the neighbours in the mix and the stream
// a batch runs on change nothing, bit for bit.

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "internal.h"

using namespace qs;

namespace {

using Clock = std::chrono::steady_clock;

// First-fit allocator over [0, size) with 256-byte granules; neighbouring free ranges merge.
class Pool {
  public:
    explicit Pool(size_t size)
    {
        if (size) free_[0] = size;
    }
    bool alloc(size_t bytes, size_t &off)
    {
        bytes = align256(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= bytes) {
                off = it->first;
                size_t rest = it->second - bytes;
                free_.erase(it);
                if (rest) free_[off + bytes] = rest;
                used_ += bytes;
                peak_ = std::max(peak_, used_);
                return true;
            }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = align256(bytes);
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
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }

  private:
    size_t used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;
};

struct Job {
    uint64_t id = 0;
    TrajPrep prep;
    uint64_t init = 0;
    qs_noise nz{};
    bool has_noise = false;
    std::vector<double> e_per_traj;
    int T = 0;
    int64_t marked = -1;
    int chunk_T = 0;
    size_t chunk_bytes = 0;
    int next = 0, done = 0, inflight = 0, n_chunks = 0;
    bool admitted = false, blocked = false, finished = false;
    qs_status status = QS_OK;
    std::string err;
    std::vector<double> F, p, norm;
    Clock::time_point t_submit, t_admit, t_done;
};

struct Slot {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    double *pinned = nullptr;   // host-pinned landing area for the batch results
    bool busy = false;
    Job *job = nullptr;
    int traj0 = 0;
    size_t off = 0, bytes = 0;
    TrajRun run;
};

}  // namespace

struct qs_srv_s {
    qs_srv_config cfg{};
    int device = 0;
    char *pool_base = nullptr;
    Pool pool{0};
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Job *> queue;
    std::unordered_map<uint64_t, std::unique_ptr<Job>> jobs;
    uint64_t next_id = 1;
    bool stop = false;
    std::thread worker;
    Clock::time_point t0, busy_since;
    double busy_s = 0;
    int inflight = 0;
    qs_srv_stats stats{};

    double secs(Clock::time_point t) const { return std::chrono::duration<double>(t - t0).count(); }
    void loop();
    void retire_locked(Slot &s, hipError_t q);
    void fail_job_locked(Job *j, qs_status st, const std::string &msg);
};

void qs_srv_s::fail_job_locked(Job *j, qs_status st, const std::string &msg)
{
    if (j->status == QS_OK) {
        j->status = st;
        j->err = msg;
        stats.failed += 1;
    }
    // nothing more of a failed request is admitted
    if (j->next < j->T) {
        j->next = j->T;
        auto it = std::find(queue.begin(), queue.end(), j);
        if (it != queue.end()) queue.erase(it);
    }
}

void qs_srv_s::retire_locked(Slot &s, hipError_t q)
{
    Job *j = s.job;
    if (q == hipSuccess && j->status == QS_OK) {
        traj_finalize(j->prep, s.run, j->F.data() + s.traj0, j->p.empty() ? nullptr : j->p.data() + s.traj0,
                      j->norm.data() + s.traj0, nullptr);
        stats.trajectories += (uint64_t)s.run.T;
    } else if (q != hipSuccess) {
        fail_job_locked(j, QS_EDEVICE, std::string("serve: batch failed on the device: ") + hipGetErrorString(q));
    }
    pool.release(s.off, s.bytes);
    s.busy = false;
    s.job = nullptr;
    s.run = TrajRun();
    j->done += 1;
    j->inflight -= 1;
    inflight -= 1;
    if (inflight == 0) busy_s += std::chrono::duration<double>(Clock::now() - busy_since).count();
    if (j->inflight == 0 && j->next >= j->T) {
        j->finished = true;
        j->t_done = Clock::now();
        if (j->status == QS_OK) stats.completed += 1;
        cv_done.notify_all();
    }
}

void qs_srv_s::loop()
{
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        for (Slot &s : slots) {
            if (!s.busy) continue;
            hipError_t q = hipEventQuery(s.ev);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) (void)hipStreamSynchronize(s.st);
            retire_locked(s, q);
        }
        while (!queue.empty()) {
            auto fs = std::find_if(slots.begin(), slots.end(), [](const Slot &s) { return !s.busy; });
            if (fs == slots.end()) break;
            Job *j = queue.front();
            const int t = std::min(j->chunk_T, j->T - j->next);
            const size_t bytes = t == j->chunk_T ? j->chunk_bytes : traj_prep_bytes(j->prep, t);
            size_t off = 0;
            if (!pool.alloc(bytes, off)) {
                if (!j->blocked) stats.admission_waits += 1;
                j->blocked = true;
                break;
            }
            j->blocked = false;
            Slot &s = *fs;
            s.busy = true;
            s.job = j;
            s.traj0 = j->next;
            s.off = off;
            s.bytes = bytes;
            if (!j->admitted) {
                j->admitted = true;
                j->t_admit = Clock::now();
            }
            j->next += t;
            j->inflight += 1;
            j->n_chunks += 1;
            if (j->next >= j->T) queue.pop_front();
            if (inflight == 0) busy_since = Clock::now();
            inflight += 1;
            stats.chunks += 1;
            stats.peak_inflight = std::max<int32_t>(stats.peak_inflight, inflight);

            // the launch reads only the immutable plan of the job and this slot: no lock needed
            qs_noise nz = j->nz;
            nz.traj_base += (uint32_t)s.traj0;
            if (!j->e_per_traj.empty()) nz.e_per_traj = j->e_per_traj.data() + s.traj0;
            lk.unlock();
            qs_status v = traj_launch(j->prep, j->init, j->has_noise ? &nz : nullptr, t, j->marked,
                                      pool_base + off, bytes, s.st, s.pinned, s.run);
            std::string msg = v == QS_OK ? std::string() : std::string(qs_last_error());
            hipError_t er = v == QS_OK ? hipEventRecord(s.ev, s.st) : hipSuccess;
            if (v != QS_OK || er != hipSuccess) (void)hipStreamSynchronize(s.st);
            lk.lock();
            if (v != QS_OK) {
                fail_job_locked(j, v, msg);
                retire_locked(s, hipSuccess);
            } else if (er != hipSuccess) {
                retire_locked(s, er);
            }
        }
        stats.in_use_bytes = pool.used();
        stats.peak_bytes = pool.peak();
        if (stop && queue.empty() && inflight == 0) break;
        if (inflight == 0 && queue.empty()) {
            cv_work.wait(lk);
        } else {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
            lk.lock();
        }
    }
}

extern "C" {

qs_status qs_srv_create(const qs_srv_config *cfg, void *pool, size_t pool_bytes, qs_srv *out)
{
    clear_error();
    if (!cfg || !out) return fail(QS_EINVAL, "srv_create: NULL config or out");
    *out = nullptr;
    if (cfg->dtype != QS_C64 && cfg->dtype != QS_C128) return fail(QS_EINVAL, "srv_create: unknown dtype");
    if (cfg->max_inflight < 1 || cfg->max_inflight > 16)
        return fail(QS_EINVAL, "srv_create: max_inflight must be in 1..16");
    if (cfg->max_chunk_traj > 4096) return fail(QS_EINVAL, "srv_create: max_chunk_traj must be <= 4096");
    if (!pool || !aligned256(pool) || pool_bytes < 256)
        return fail(QS_EINVAL, "srv_create: pool must be non-NULL, 256-byte aligned and non-empty");
    hipPointerAttribute_t attr{};
    if (hipPointerGetAttributes(&attr, pool) != hipSuccess || attr.type != hipMemoryTypeDevice) {
        (void)hipGetLastError();
        return fail(QS_EINVAL, "srv_create: pool is not device memory");
    }
    auto srv = std::make_unique<qs_srv_s>();
    srv->cfg = *cfg;
    if (srv->cfg.max_chunk_traj <= 0) srv->cfg.max_chunk_traj = 256;
    srv->device = attr.device;
    srv->pool_base = (char *)pool;
    srv->pool = Pool(pool_bytes & ~size_t(255));
    srv->stats.pool_bytes = pool_bytes & ~size_t(255);
    int prev = 0;
    QS_HIP(hipGetDevice(&prev));
    QS_HIP(hipSetDevice(srv->device));
    srv->slots.resize(cfg->max_inflight);
    const size_t pin_bytes = sizeof(double) * 5 * (size_t)(srv->cfg.max_chunk_traj + 1);
    hipError_t e = hipSuccess;
    for (Slot &s : srv->slots) {
        if ((e = hipStreamCreateWithFlags(&s.st, hipStreamNonBlocking)) != hipSuccess) break;
        if ((e = hipEventCreateWithFlags(&s.ev, hipEventDisableTiming)) != hipSuccess) break;
        if ((e = hipHostMalloc((void **)&s.pinned, pin_bytes, hipHostMallocDefault)) != hipSuccess) break;
    }
    (void)hipSetDevice(prev);
    if (e != hipSuccess) {
        for (Slot &s : srv->slots) {
            if (s.pinned) (void)hipHostFree(s.pinned);
            if (s.ev) (void)hipEventDestroy(s.ev);
            if (s.st) (void)hipStreamDestroy(s.st);
        }
        return hip_fail(e, "srv_create");
    }
    srv->t0 = Clock::now();
    qs_srv_s *p = srv.release();
    p->worker = std::thread([p] { p->loop(); });
    *out = p;
    return QS_OK;
}

qs_status qs_srv_submit(qs_srv srv, const qs_gate *gates, int n_gates, int n, uint64_t init_index,
                        const qs_noise *nz, int T, int64_t marked, uint64_t *job_out)
{
    const auto t_arrive = Clock::now();   // planning counts toward the request's latency
    clear_error();
    if (!srv || !job_out) return fail(QS_EINVAL, "srv_submit: NULL server or job_out");
    if (T < 1) return fail(QS_EINVAL, "srv_submit: n_traj must be >= 1");
    if (init_index >= (1ull << std::min(std::max(n, 1), 63)))
        return fail(QS_EINVAL, "srv_submit: init_index out of range");
    if (marked >= 0 && n < 63 && marked >= (int64_t)(1ull << n))
        return fail(QS_EINVAL, "srv_submit: marked out of range");
    auto j = std::make_unique<Job>();
    qs_status v = traj_prepare(gates, n_gates, n, (qs_dtype)srv->cfg.dtype, &srv->cfg.plan, j->prep);
    if (v != QS_OK) return v;
    if (nz) {
        if (!std::isfinite(nz->e) || nz->e < 0) return fail(QS_EINVAL, "srv_submit: noise e must be finite and >= 0");
        j->nz = *nz;
        j->has_noise = true;
        if (nz->e_per_traj) {
            j->e_per_traj.assign(nz->e_per_traj, nz->e_per_traj + T);
            for (double e : j->e_per_traj)
                if (!std::isfinite(e) || e < 0)
                    return fail(QS_EINVAL, "srv_submit: per-trajectory e must be finite and >= 0");
            j->nz.e_per_traj = nullptr;
        }
        if ((uint64_t)nz->traj_base + (uint64_t)T > 0xffffffffull)
            return fail(QS_EINVAL, "srv_submit: traj_base + n_traj exceeds 2^32");
    }
    // batch size: the configured maximum, halved until one batch fits the whole pool
    const size_t cap = srv->stats.pool_bytes;
    int t = std::min(T, srv->cfg.max_chunk_traj);
    while (t > 1 && align256(traj_prep_bytes(j->prep, t)) > cap) t = (t + 1) / 2;
    const size_t b = traj_prep_bytes(j->prep, t);
    if (align256(b) > cap)
        return fail(QS_ENOMEM, "srv_submit: one trajectory needs " + std::to_string(b) +
                                   " bytes, more than the pool holds");
    j->chunk_T = t;
    j->chunk_bytes = b;
    j->init = init_index;
    j->T = T;
    j->marked = marked;
    j->F.assign(T, 0.0);
    if (marked >= 0) j->p.assign(T, 0.0);
    j->norm.assign(T, 0.0);
    j->t_submit = t_arrive;
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stop) return fail(QS_EBUSY, "srv_submit: server is shutting down");
    j->id = srv->next_id++;
    *job_out = j->id;
    srv->queue.push_back(j.get());
    srv->jobs.emplace(j->id, std::move(j));
    srv->stats.submitted += 1;
    srv->cv_work.notify_one();
    return QS_OK;
}

qs_status qs_srv_poll(qs_srv srv, uint64_t job, int *done)
{
    clear_error();
    if (!srv || !done) return fail(QS_EINVAL, "srv_poll: NULL argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->jobs.find(job);
    if (it == srv->jobs.end()) return fail(QS_EINVAL, "srv_poll: unknown job");
    *done = it->second->finished ? 1 : 0;
    return QS_OK;
}

qs_status qs_srv_wait(qs_srv srv, uint64_t job, double timeout_s)
{
    clear_error();
    if (!srv) return fail(QS_EINVAL, "srv_wait: NULL server");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->jobs.find(job);
    if (it == srv->jobs.end()) return fail(QS_EINVAL, "srv_wait: unknown job");
    Job *j = it->second.get();
    auto ready = [j] { return j->finished; };
    if (timeout_s < 0) {
        srv->cv_done.wait(lk, ready);
    } else if (!srv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready)) {
        return fail(QS_EBUSY, "srv_wait: timed out");
    }
    return QS_OK;
}

qs_status qs_srv_result(qs_srv srv, uint64_t job, double *fid_out, double *p_out, double *norm_out,
                        qs_srv_job_info *info)
{
    clear_error();
    if (!srv) return fail(QS_EINVAL, "srv_result: NULL server");
    std::unique_ptr<Job> j;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        auto it = srv->jobs.find(job);
        if (it == srv->jobs.end()) return fail(QS_EINVAL, "srv_result: unknown job");
        if (!it->second->finished) return fail(QS_EBUSY, "srv_result: job not finished");
        if (p_out && it->second->marked < 0) return fail(QS_EINVAL, "srv_result: p_out needs marked >= 0");
        j = std::move(it->second);
        srv->jobs.erase(it);
    }
    if (info) {
        std::memset(info, 0, sizeof *info);
        info->status = j->status;
        info->n_chunks = j->n_chunks;
        info->chunk_traj = j->chunk_T;
        info->chunk_bytes = j->chunk_bytes;
        info->t_submit = srv->secs(j->t_submit);
        info->t_admit = j->admitted ? srv->secs(j->t_admit) : info->t_submit;
        info->t_done = srv->secs(j->t_done);
        info->latency_s = info->t_done - info->t_submit;
        info->queue_s = info->t_admit - info->t_submit;
    }
    if (j->status != QS_OK) return fail(j->status, j->err);
    if (fid_out) std::memcpy(fid_out, j->F.data(), sizeof(double) * j->T);
    if (p_out) std::memcpy(p_out, j->p.data(), sizeof(double) * j->T);
    if (norm_out) std::memcpy(norm_out, j->norm.data(), sizeof(double) * j->T);
    return QS_OK;
}

qs_status qs_srv_stats_get(qs_srv srv, qs_srv_stats *out)
{
    clear_error();
    if (!srv || !out) return fail(QS_EINVAL, "srv_stats: NULL argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    *out = srv->stats;
    out->in_use_bytes = srv->pool.used();
    out->peak_bytes = srv->pool.peak();
    out->inflight = srv->inflight;
    out->queued = (int32_t)srv->queue.size();
    const auto now = Clock::now();
    out->busy_s = srv->busy_s + (srv->inflight ? std::chrono::duration<double>(now - srv->busy_since).count() : 0.0);
    out->elapsed_s = srv->secs(now);
    return QS_OK;
}

qs_status qs_srv_destroy(qs_srv srv)
{
    clear_error();
    if (!srv) return QS_OK;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        srv->cv_work.notify_one();
    }
    if (srv->worker.joinable()) srv->worker.join();
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(srv->device);
    for (Slot &s : srv->slots) {
        if (s.st) (void)hipStreamSynchronize(s.st);
        if (s.pinned) (void)hipHostFree(s.pinned);
        if (s.ev) (void)hipEventDestroy(s.ev);
        if (s.st) (void)hipStreamDestroy(s.st);
    }
    (void)hipSetDevice(prev);
    delete srv;
    return QS_OK;
}

}  // extern "C"
