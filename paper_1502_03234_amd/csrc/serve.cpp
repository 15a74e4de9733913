// serve.cpp -- serving form: many independent systems on one GPU behind a request loop.
//
// A worker thread owns the GPU side. Requests queue in arrival order; the front request is
// admitted when its device footprint (system workspace, staging and thermo records) fits the
// remaining HBM budget and a free range of the caller's pool. An admitted system stays
// resident. Whenever the set of resident systems changes, the launch sequence of one detection
// period (2 steps for detect_every = 2) is recorded for every system without running it, and
// systems whose sequences name the same kernels in the same order form a group. Each position
// of a group's sequence becomes one batched launch over all of its systems' workgroups (their
// argument records in a device table, see launch.h), and the group's whole period is captured
// into one hipGraph. A batch replays every group's graph on the server's stream, so a period
// of all resident systems costs as many launches as a period of one system. A system whose
// remaining step count is shorter than the period finishes with ordinary launches on its own
// stream. Finished systems are copied back to host memory and released; dcm_poll hands the
// result to the caller.
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
#include "launch.h"

using dcm::current_recorder;
using dcm::Launch;
using dcm::Recorder;

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
    int period = 2;
    bool grouped = false;           // stepped by its group's graph in the current batch
    int32_t done_steps = 0;
    dcm_status failed = DCM_OK;     // a launch for this system failed: it completes with this
    int last_record = 0;
    double *d_x = nullptr, *d_v = nullptr;
    dcm_thermo *d_th = nullptr;
    dcm_thermo last{};
};

int gcd(int a, int b) { return b ? gcd(b, a % b) : a; }

// Systems stepped together: one recorded period per member, all naming the same kernels.
struct Group {
    std::vector<Req *> members;
    hipGraphExec_t graph = nullptr;
};

// Bytes of the pool kept for the batched launches' argument and workgroup tables.
size_t table_reserve(size_t pool_bytes)
{
    const size_t want = std::min<size_t>(pool_bytes / 16, (size_t)16 << 20);
    return want & ~(size_t)255;
}

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
    hipStream_t stream = nullptr;             // batched launches of all groups
    uint8_t *tables = nullptr;                // [table_bytes] at the end of the pool
    size_t table_bytes = 0;
    std::vector<uint8_t> table_host;          // host image of the tables (staging)
    std::vector<Group> groups;
    bool regroup = false;                     // the resident set changed since the last grouping
    hipEvent_t batch_done[2] = {nullptr, nullptr};   // ends of the last two batches
    int batch_parity = 0;
    bool in_flight = false;                   // the previous batch may still be running
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
    if (r->sys) dcm_destroy(r->sys);
    if (r->stream) (void)hipStreamDestroy(r->stream);
    r->sys = nullptr;
    r->stream = nullptr;
}

// Admission: copy the state in and create the system (force evaluation k = 0; synchronizes
// the system's stream).
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
    return dcm_create(&r->p, r->n, base, r->ws_bytes, r->d_x, r->d_v, r->stream, &r->sys);
}

// The launches of one period of r, recorded without running them. Recording advances the
// host-side state exactly as running would (step counter, ping-pong sets and sort buffers);
// a period is an even number of steps, so every buffer choice is back where it started and
// only the step counter needs restoring.
dcm_status record_period(Req *r, Recorder &rec)
{
    dcm_system *s = r->sys;
    const int64_t k0 = s->k;
    const int cur0 = s->cur;
    uint32_t *key0 = s->key, *val0 = s->val;
    current_recorder() = &rec;
    const dcm_status st = dcm_step(s, r->period, r->stream, r->d_th);
    current_recorder() = nullptr;
    s->k = k0;
    if (s->cur != cur0 || s->key != key0 || s->val != val0) return DCM_E_INVALID;
    return st;
}

bool same_sequence(const Recorder &a, const Recorder &b)
{
    if (a.ops.size() != b.ops.size()) return false;
    for (size_t q = 0; q < a.ops.size(); ++q)
        if (a.ops[q].batched != b.ops[q].batched || a.ops[q].threads != b.ops[q].threads ||
            a.ops[q].args.size() != b.ops[q].args.size())
            return false;
    return true;
}

void drop_groups(dcm_server *sv)
{
    for (Group &g : sv->groups)
        if (g.graph) (void)hipGraphExecDestroy(g.graph);
    sv->groups.clear();
}

// Table bytes of one group: per position, the members' argument records and first workgroups.
size_t group_table_bytes(const Recorder &rec, size_t m)
{
    size_t b = 0;
    for (const Launch &l : rec.ops) b += align_up(l.args.size() * m) + align_up(sizeof(uint32_t) * (m + 1));
    return b;
}

// Groups the systems that run whole periods this batch, writes their tables into the reserved
// part of the pool and captures one graph per group. Systems that fit no group (the tables
// are full, or recording failed) are stepped eagerly instead.
void regroup(dcm_server *sv)
{
    const auto t0 = std::chrono::steady_clock::now();
    (void)hipStreamSynchronize(sv->stream);     // tables of the previous grouping are free
    sv->in_flight = false;
    drop_groups(sv);
    for (Req *r : sv->running) r->grouped = false;
    std::vector<Recorder> recs;
    std::vector<std::vector<size_t>> members;   // indices into recs / cand
    std::vector<Req *> cand;
    for (Req *r : sv->running) {
        if (r->nsteps - r->done_steps < r->period) continue;
        Recorder rec;
        if (record_period(r, rec) != DCM_OK) continue;
        size_t gi = 0;
        while (gi < members.size() && !same_sequence(recs[members[gi][0]], rec)) ++gi;
        if (gi == members.size()) members.emplace_back();
        members[gi].push_back(recs.size());
        recs.push_back(std::move(rec));
        cand.push_back(r);
    }
    size_t used = 0;
    std::vector<uint8_t> &host = sv->table_host;
    for (const std::vector<size_t> &mem : members) {
        const Recorder &first_rec = recs[mem[0]];
        // as many members as the remaining table space holds
        size_t m = mem.size();
        while (m > 0 && used + group_table_bytes(first_rec, m) > sv->table_bytes) --m;
        if (m == 0) continue;
        struct Op { const void *fn; uint32_t threads, blocks; size_t tab, first; };
        std::vector<Op> ops;
        for (size_t q = 0; q < first_rec.ops.size(); ++q) {
            const size_t asz = first_rec.ops[q].args.size();
            Op op{first_rec.ops[q].batched, first_rec.ops[q].threads, 0, used, 0};
            for (size_t k = 0; k < m; ++k)
                std::memcpy(host.data() + used + k * asz, recs[mem[k]].ops[q].args.data(), asz);
            used += align_up(asz * m);
            op.first = used;
            uint32_t *fb = (uint32_t *)(host.data() + used);
            fb[0] = 0;
            for (size_t k = 0; k < m; ++k) fb[k + 1] = fb[k] + recs[mem[k]].ops[q].blocks;
            op.blocks = fb[m];
            used += align_up(sizeof(uint32_t) * (m + 1));
            ops.push_back(op);
        }
        Group g;
        for (size_t k = 0; k < m; ++k) g.members.push_back(cand[mem[k]]);
        if (hipStreamBeginCapture(sv->stream, hipStreamCaptureModeRelaxed) != hipSuccess) continue;
        for (const Op &op : ops) {
            if (op.blocks == 0) continue;
            void *tab = sv->tables + op.tab;
            void *fst = sv->tables + op.first;
            int nsys = (int)m;
            void *kargs[] = {&tab, &fst, &nsys};
            (void)hipLaunchKernel(op.fn, dim3(op.blocks), dim3(op.threads), kargs, 0, sv->stream);
        }
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(sv->stream, &graph);
        if (e == hipSuccess && graph) e = hipGraphInstantiate(&g.graph, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        if (e != hipSuccess || !g.graph) {
            (void)hipGetLastError();
            continue;
        }
        for (Req *r : g.members) r->grouped = true;
        sv->groups.push_back(std::move(g));
    }
    if (used) (void)hipMemcpyAsync(sv->tables, host.data(), used, hipMemcpyHostToDevice, sv->stream);
    (void)hipStreamSynchronize(sv->stream);     // the staging copy may be overwritten again
    sv->regroup = false;
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stats.groupings += 1;
    sv->stats.grouping_ms += ms;
}

// One batch: every group's period by graph replay on the server's stream, every other
// system its period (or its remaining steps) eagerly on its own stream.
void advance_all(dcm_server *sv)
{
    for (Group &g : sv->groups) {
        if (hipGraphLaunch(g.graph, sv->stream) == hipSuccess) continue;
        (void)hipGetLastError();
        // the members did not step: they end now, with the error, instead of with stale state
        for (Req *r : g.members) {
            r->failed = DCM_E_HIP;
            r->err = "hipGraphLaunch of the batched period failed";
            r->grouped = false;
            r->done_steps = r->nsteps;
        }
        sv->regroup = true;
    }
    int64_t grouped = 0, eager = 0;
    for (Req *r : sv->running) {
        const int32_t left = r->nsteps - r->done_steps;
        if (r->failed != DCM_OK) continue;
        if (r->grouped) {
            r->sys->k += r->period;
            r->done_steps += r->period;
            r->last_record = r->period - 1;
            if (r->nsteps - r->done_steps < r->period) sv->regroup = true;
            grouped += 1;
        } else if (left > 0) {
            const int32_t q = std::min(left, r->period);
            const dcm_status st = dcm_step(r->sys, q, r->stream, r->d_th);
            if (st != DCM_OK) {
                r->failed = st;
                r->err = dcm_last_error();
                r->done_steps = r->nsteps;
                continue;
            }
            r->done_steps += q;
            r->last_record = q - 1;
            eager += 1;
        }
    }
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stats.grouped_steps += grouped;
    sv->stats.eager_steps += eager;
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
            sv->regroup = true;
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->stats.running += 1;
        }
        if (sv->regroup) regroup(sv);
        advance_all(sv);
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->stats.batches += 1;
        }
        // Keep one batch in flight: wait for the previous batch, not this one, unless a system
        // has finished its steps in this batch (its results are read next) or the groups must
        // change (the tables are rewritten).
        bool finished = sv->regroup;
        for (Req *r : sv->running) finished = finished || r->done_steps >= r->nsteps;
        (void)hipEventRecord(sv->batch_done[sv->batch_parity], sv->stream);
        if (finished) {
            (void)hipStreamSynchronize(sv->stream);
            sv->in_flight = false;
        } else {
            if (sv->in_flight) (void)hipEventSynchronize(sv->batch_done[1 - sv->batch_parity]);
            sv->in_flight = true;
        }
        sv->batch_parity = 1 - sv->batch_parity;
        std::vector<Req *> keep;
        for (Req *r : sv->running) {
            if (r->done_steps < r->nsteps) {
                if (!r->grouped) (void)hipStreamSynchronize(r->stream);
                keep.push_back(r);
                continue;
            }
            sv->regroup = true;
            dcm_status s = r->failed != DCM_OK ? r->failed : finish(r);
            std::string err = s == DCM_OK ? std::string()
                              : (r->failed != DCM_OK ? r->err : std::string(dcm_last_error()));
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
                drop_groups(sv);
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
    sv->table_bytes = table_reserve(pool_bytes);
    sv->pool_bytes = (pool_bytes - sv->table_bytes) & ~(kAlign - 1);
    sv->tables = sv->pool + sv->pool_bytes;
    sv->free_list.push_back({0, sv->pool_bytes});
    sv->table_host.resize(sv->table_bytes);
    if (hipGetDevice(&sv->device) != hipSuccess || hipStreamCreate(&sv->stream) != hipSuccess ||
        hipEventCreateWithFlags(&sv->batch_done[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&sv->batch_done[1], hipEventDisableTiming) != hipSuccess) {
        if (sv->stream) (void)hipStreamDestroy(sv->stream);
        if (sv->batch_done[0]) (void)hipEventDestroy(sv->batch_done[0]);
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
    // neighbour lists decide their rebuilds on the host between launches, which a recorded
    // batch cannot do
    if (p->neighbor_list) return DCM_E_INVALID;
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
    drop_groups(sv);
    for (hipEvent_t e : sv->batch_done)
        if (e) (void)hipEventDestroy(e);
    if (sv->stream) (void)hipStreamDestroy(sv->stream);
    for (auto &kv : sv->reqs) delete kv.second;
    delete sv;
    return DCM_OK;
}

}  // extern "C"
