// serve.cpp -- serving form: many independent systems on one GPU behind a request loop.
//
// A worker thread owns the GPU side. Requests queue in arrival order; the front request is
// admitted when its device footprint (system workspace, staging and thermo records) fits the
// remaining HBM budget and a free range of the caller's pool. An admitted system stays
// resident on its own stream. Its step sequence over one detection period (2 steps for
// detect_every = 2) is captured once into a hipGraph; every batch replays the graphs of all
// resident systems, each on its stream, so small systems run concurrently and the per-step
// host launch cost is one graph launch per system. A system whose remaining step count is
// shorter than the period finishes with ordinary launches. Finished systems are copied back to
// host memory and released; dcm_poll hands the result to the caller.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

struct Req {
    uint64_t ticket = 0;
    dcm_params p{};
    int64_t n = 0;
    int32_t nsteps = 0;
    std::vector<double> hx, hv;   // inputs; replaced by the outputs on completion
    dcm_status status = DCM_PENDING;
    std::string err;
    size_t off = 0, bytes = 0, ws_bytes = 0;
    dcm_system *sys = nullptr;
    hipStream_t stream = nullptr;
    hipGraphExec_t graph = nullptr;
    int period = 2;
    int32_t done_steps = 0;
    int last_record = 0;
    double *d_x = nullptr, *d_v = nullptr;
    dcm_thermo *d_th = nullptr;
    dcm_thermo last{};
};

int gcd(int a, int b) { return b ? gcd(b, a % b) : a; }

}  // namespace

struct dcm_server {
    size_t budget = 0, pool_bytes = 0, in_use = 0;
    uint8_t *pool = nullptr;
    int device = 0;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Req *> queue;
    std::map<uint64_t, Req *> reqs;
    std::vector<Req *> running;
    std::vector<std::pair<size_t, size_t>> free_list;   // (offset, size), sorted by offset
    std::thread worker;
    bool stop = false;
    uint64_t next_ticket = 1;
    dcm_server_stats stats{};
};

namespace {

bool pool_alloc(dcm_server *sv, size_t bytes, size_t *off)
{
    for (size_t q = 0; q < sv->free_list.size(); ++q) {
        auto &f = sv->free_list[q];
        if (f.second >= bytes) {
            *off = f.first;
            f.first += bytes;
            f.second -= bytes;
            if (f.second == 0) sv->free_list.erase(sv->free_list.begin() + (long)q);
            return true;
        }
    }
    return false;
}

void pool_free(dcm_server *sv, size_t off, size_t bytes)
{
    auto &fl = sv->free_list;
    size_t q = 0;
    while (q < fl.size() && fl[q].first < off) ++q;
    fl.insert(fl.begin() + (long)q, {off, bytes});
    if (q + 1 < fl.size() && fl[q].first + fl[q].second == fl[q + 1].first) {
        fl[q].second += fl[q + 1].second;
        fl.erase(fl.begin() + (long)q + 1);
    }
    if (q > 0 && fl[q - 1].first + fl[q - 1].second == fl[q].first) {
        fl[q - 1].second += fl[q].second;
        fl.erase(fl.begin() + (long)q);
    }
}

// Device footprint of a request: [workspace | x | v | thermo records of one period].
size_t footprint(const Req *r, size_t ws)
{
    return align_up(ws) + 2 * align_up(sizeof(double) * 3 * (size_t)r->n) +
           align_up(sizeof(dcm_thermo) * (size_t)r->period);
}

void release_device(Req *r)
{
    if (r->graph) (void)hipGraphExecDestroy(r->graph);
    if (r->sys) dcm_destroy(r->sys);
    if (r->stream) (void)hipStreamDestroy(r->stream);
    r->graph = nullptr;
    r->sys = nullptr;
    r->stream = nullptr;
}

// Admission: copy the state in, create the system (force evaluation k = 0), capture one period.
dcm_status start(dcm_server *sv, Req *r)
{
    uint8_t *base = sv->pool + r->off;
    r->d_x = (double *)(base + align_up(r->ws_bytes));
    r->d_v = (double *)((uint8_t *)r->d_x + align_up(sizeof(double) * 3 * (size_t)r->n));
    r->d_th = (dcm_thermo *)((uint8_t *)r->d_v + align_up(sizeof(double) * 3 * (size_t)r->n));
    if (hipStreamCreate(&r->stream) != hipSuccess) return DCM_E_HIP;
    const size_t nb = sizeof(double) * 3 * (size_t)r->n;
    if (hipMemcpyAsync(r->d_x, r->hx.data(), nb, hipMemcpyHostToDevice, r->stream) != hipSuccess ||
        hipMemcpyAsync(r->d_v, r->hv.data(), nb, hipMemcpyHostToDevice, r->stream) != hipSuccess)
        return DCM_E_HIP;
    dcm_status s = dcm_create(&r->p, r->n, base, r->ws_bytes, r->d_x, r->d_v, r->stream, &r->sys);
    if (s != DCM_OK) return s;
    if (r->nsteps >= r->period) {
        if (hipStreamBeginCapture(r->stream, hipStreamCaptureModeRelaxed) != hipSuccess) return DCM_E_HIP;
        const int64_t k0 = r->sys->k;
        const int cur0 = r->sys->cur;
        s = dcm_step(r->sys, r->period, r->stream, r->d_th);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(r->stream, &g);
        // capture records the launches without running them: restore the host-side state
        r->sys->k = k0;
        r->sys->cur = cur0;
        if (s != DCM_OK) return s;
        if (e != hipSuccess || !g) return DCM_E_HIP;
        e = hipGraphInstantiate(&r->graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return DCM_E_HIP;
    }
    return DCM_OK;
}

// One batch for one system: a period by graph replay, or the remaining steps eagerly.
void advance(Req *r)
{
    const int32_t left = r->nsteps - r->done_steps;
    if (left >= r->period && r->graph) {
        (void)hipGraphLaunch(r->graph, r->stream);
        r->sys->k += r->period;
        r->done_steps += r->period;
        r->last_record = r->period - 1;
    } else if (left > 0) {
        dcm_step(r->sys, left, r->stream, r->d_th);
        r->done_steps += left;
        r->last_record = left - 1;
    }
}

dcm_status finish(Req *r)
{
    int64_t k = 0;
    dcm_status s = dcm_get_state(r->sys, r->stream, r->d_x, r->d_v, nullptr, &k);
    if (s != DCM_OK) return s;
    const size_t nb = sizeof(double) * 3 * (size_t)r->n;
    if (hipMemcpyAsync(r->hx.data(), r->d_x, nb, hipMemcpyDeviceToHost, r->stream) != hipSuccess ||
        hipMemcpyAsync(r->hv.data(), r->d_v, nb, hipMemcpyDeviceToHost, r->stream) != hipSuccess ||
        hipMemcpyAsync(&r->last, r->d_th + r->last_record, sizeof(dcm_thermo), hipMemcpyDeviceToHost,
                       r->stream) != hipSuccess)
        return DCM_E_HIP;
    s = dcm_check(r->sys, r->stream);          // synchronizes the stream
    r->last.step = k;                          // replays re-use the captured step labels
    return s;
}

void worker_loop(dcm_server *sv)
{
    (void)hipSetDevice(sv->device);
    for (;;) {
        std::vector<Req *> admit;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            for (;;) {
                while (!sv->stop && !sv->queue.empty()) {
                    Req *r = sv->queue.front();
                    size_t off = 0;
                    if (sv->in_use + r->bytes > sv->budget || !pool_alloc(sv, r->bytes, &off)) break;
                    r->off = off;
                    sv->in_use += r->bytes;
                    sv->queue.pop_front();
                    admit.push_back(r);
                    sv->stats.admitted += 1;
                }
                if (!admit.empty() || !sv->running.empty()) break;
                if (sv->stop) return;
                sv->cv.wait(lk);
            }
        }
        for (Req *r : admit) {
            dcm_status s = start(sv, r);
            if (s != DCM_OK) {
                std::lock_guard<std::mutex> lk(sv->mu);
                r->status = s;
                r->err = dcm_last_error();
                release_device(r);
                pool_free(sv, r->off, r->bytes);
                sv->in_use -= r->bytes;
                sv->stats.completed += 1;
                sv->cv.notify_all();
                continue;
            }
            sv->running.push_back(r);
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->stats.running += 1;
        }
        for (Req *r : sv->running) advance(r);
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->stats.batches += 1;
        }
        std::vector<Req *> keep;
        for (Req *r : sv->running) {
            if (r->done_steps < r->nsteps) {
                (void)hipStreamSynchronize(r->stream);
                keep.push_back(r);
                continue;
            }
            dcm_status s = finish(r);
            std::string err = s == DCM_OK ? std::string() : std::string(dcm_last_error());
            release_device(r);
            std::lock_guard<std::mutex> lk(sv->mu);
            r->status = s;
            r->err = err;
            pool_free(sv, r->off, r->bytes);
            sv->in_use -= r->bytes;
            sv->stats.completed += 1;
            sv->stats.running -= 1;
            sv->cv.notify_all();
        }
        sv->running.swap(keep);
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            if (sv->stop && sv->running.empty()) {
                for (Req *r : sv->queue) { r->status = DCM_E_INVALID; r->err = "server destroyed"; }
                sv->queue.clear();
                return;
            }
        }
    }
}

}  // namespace

extern "C" {

dcm_status dcm_server_create(size_t hbm_budget, void *d_pool, size_t pool_bytes, dcm_stream_t stream,
                             dcm_server **out)
{
    if (!out || !d_pool || pool_bytes == 0 || ((uintptr_t)d_pool & (kAlign - 1)))
        return DCM_E_INVALID;
    if (hbm_budget == 0 || hbm_budget > pool_bytes) return DCM_E_INVALID;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return DCM_E_HIP;
    dcm_server *sv = new (std::nothrow) dcm_server();
    if (!sv) return DCM_E_INVALID;
    sv->budget = hbm_budget;
    sv->pool = (uint8_t *)d_pool;
    sv->pool_bytes = pool_bytes;
    sv->free_list.push_back({0, pool_bytes & ~(kAlign - 1)});
    if (hipGetDevice(&sv->device) != hipSuccess) {
        delete sv;
        return DCM_E_HIP;
    }
    sv->worker = std::thread(worker_loop, sv);
    *out = sv;
    return DCM_OK;
}

dcm_status dcm_submit(dcm_server *sv, const dcm_params *p, int64_t n, const double *h_x, const double *h_v,
                      int32_t nsteps, uint64_t *ticket)
{
    if (!sv || !p || !h_x || !h_v || !ticket || nsteps < 0) return DCM_E_INVALID;
    size_t ws = 0;
    dcm_status s = dcm_workspace_bytes(p, n, &ws);
    if (s != DCM_OK) return s;
    Req *r = new (std::nothrow) Req();
    if (!r) return DCM_E_INVALID;
    r->p = *p;
    r->n = n;
    r->nsteps = nsteps;
    r->period = p->detect_every > 0 ? 2 * p->detect_every / gcd(2, p->detect_every) : 2;
    r->ws_bytes = ws;
    r->bytes = footprint(r, ws);
    r->hx.assign(h_x, h_x + 3 * n);
    r->hv.assign(h_v, h_v + 3 * n);
    std::lock_guard<std::mutex> lk(sv->mu);
    if (r->bytes > sv->budget || r->bytes > sv->pool_bytes) {
        delete r;
        sv->stats.rejected += 1;
        return DCM_E_BUDGET;
    }
    r->ticket = sv->next_ticket++;
    sv->reqs[r->ticket] = r;
    sv->queue.push_back(r);
    sv->stats.submitted += 1;
    *ticket = r->ticket;
    sv->cv.notify_all();
    return DCM_OK;
}

dcm_status dcm_poll(dcm_server *sv, uint64_t ticket, double *h_x_out, double *h_v_out, dcm_thermo *h_last)
{
    if (!sv) return DCM_E_INVALID;
    Req *r = nullptr;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        auto it = sv->reqs.find(ticket);
        if (it == sv->reqs.end()) return DCM_E_UNKNOWN_TICKET;
        r = it->second;
        if (r->status == DCM_PENDING) return DCM_PENDING;
        sv->reqs.erase(it);
    }
    dcm_status s = r->status;
    if (s == DCM_OK) {
        if (h_x_out) std::memcpy(h_x_out, r->hx.data(), sizeof(double) * 3 * (size_t)r->n);
        if (h_v_out) std::memcpy(h_v_out, r->hv.data(), sizeof(double) * 3 * (size_t)r->n);
        if (h_last) *h_last = r->last;
    }
    delete r;
    return s;
}

dcm_status dcm_server_query(dcm_server *sv, dcm_server_stats *st)
{
    if (!sv || !st) return DCM_E_INVALID;
    std::lock_guard<std::mutex> lk(sv->mu);
    *st = sv->stats;
    st->queued = (int64_t)sv->queue.size();
    st->bytes_in_use = sv->in_use;
    return DCM_OK;
}

dcm_status dcm_server_destroy(dcm_server *sv)
{
    if (!sv) return DCM_OK;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
        sv->cv.notify_all();
    }
    if (sv->worker.joinable()) sv->worker.join();
    for (auto &kv : sv->reqs) delete kv.second;
    delete sv;
    return DCM_OK;
}

}  // extern "C"
