// Serving loop: many running simulations submit extrapolation requests; the server keeps
// their fields resident in HBM, admits work by an HBM budget and batches queued requests
// (across simulations and grid sizes) into launches on several streams, so that requests
// arriving while others run join the next launch as a stream and memory free up.  Object
// independence (main text, "Extrapolation of xi", third paragraph) makes every request,
// and every solid in it, independent of the others in its batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "rmx.h"
#include "rmx_core.h"
#include "rmx_ctx.h"

using namespace rmx;

namespace {

using Clock = std::chrono::steady_clock;

constexpr size_t kMaxQueue = 1 << 16;     // queued requests before RMX_E_BUSY
constexpr int kMaxBatchRequests = 64;     // requests fused into one launch chain
constexpr int kMaxBatchSolids = 4096;
constexpr int kMaxStreams = 16;

struct Sim {
    rmx_grid grid{};
    std::vector<rmx_solid> solids;   // fields owned by the server
    std::vector<const rmx_grid*> grids;
    void* mem = nullptr;
    size_t bytes = 0;
    bool busy = false;               // a request of this simulation is in flight
    int queued = 0;                  // requests waiting
};

struct Req {
    int64_t sim = 0;
    rmx_options opt{};
    Clock::time_point t_submit;
    double latency = 0.0;
    int status = RMX_OK;
    bool done = false;
    std::vector<rmx_solid_stats> stats;
};

struct Lane {
    rmx_ctx* ctx = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    std::vector<int64_t> tickets;    // requests in flight on this lane
    size_t n_solids = 0;
    bool busy = false;
};

bool same_class(const rmx_options& a, const rmx_options& b) {
    return a.r_s == b.r_s && a.r_max == b.r_max && a.normal_layers == b.normal_layers &&
           a.precision == b.precision;
}

}  // namespace

struct rmx_server {
    int device = 0;
    size_t budget = 0;
    std::mutex mu;
    std::condition_variable cv_work;   // scheduler: new request, completion, shutdown
    std::condition_variable cv_done;   // waiters
    std::thread sched;
    bool stop = false;
    std::unordered_map<int64_t, Sim> sims;
    int64_t next_sim = 1;
    std::deque<int64_t> queue;
    std::unordered_map<int64_t, Req> reqs;
    int64_t next_ticket = 1;
    std::vector<Lane> lanes;
    size_t resident = 0;               // bytes of registered fields
    size_t peak = 0;
};

namespace {

size_t lanes_ws(const rmx_server* s) {
    size_t t = 0;
    for (const auto& l : s->lanes) t += l.ctx ? l.ctx->ws_size : 0;
    return t;
}

size_t in_use(const rmx_server* s) { return s->resident + lanes_ws(s); }

void note_peak(rmx_server* s) { s->peak = std::max(s->peak, in_use(s)); }

// Give the workspaces of idle lanes back to the budget (caller holds the lock).
void release_idle_ws(rmx_server* s) {
    for (auto& l : s->lanes) {
        if (l.busy || !l.ctx || !l.ctx->ws || l.ctx->fixed) continue;
        (void)hipStreamSynchronize(l.stream);
        for (auto& kv : l.ctx->graphs) {
            if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
            if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
        }
        l.ctx->graphs.clear();
        (void)hipFree(l.ctx->ws);
        l.ctx->ws = nullptr;
        l.ctx->ws_size = 0;
        l.ctx->desc_valid = false;
    }
}

// Workspace bytes a batch of these solids needs on a lane; (size_t)-1 if it cannot be
// planned.  Server lanes grow their workspace to exactly this.
size_t batch_ws(const std::vector<const rmx_grid*>& g, const std::vector<rmx_solid>& sol,
                const rmx_options& opt, const Lane& lane) {
    Plan p;
    if (plan(g.data(), sol.data(), (int)sol.size(), &opt, lane.ctx->lds_limit, lane.ctx->cus,
             Tuning{}, &p) != RMX_OK)
        return (size_t)-1;
    return p.ws_bytes;
}

// Finish the requests of a lane whose launch completed (caller holds the lock).
void retire(rmx_server* s, Lane& lane) {
    const auto now = Clock::now();
    convert_stats(lane.ctx->stats_host, (int)lane.n_solids, lane.ctx->tmp_stats.data());
    size_t off = 0;
    for (int64_t t : lane.tickets) {
        Req& r = s->reqs[t];
        Sim& sim = s->sims[r.sim];
        const size_t n = sim.solids.size();
        r.stats.assign(lane.ctx->tmp_stats.begin() + off, lane.ctx->tmp_stats.begin() + off + n);
        off += n;
        r.status = RMX_OK;
        for (const auto& st : r.stats)
            if (st.status < 0) {
                r.status = st.status;
                break;
            }
        r.latency = std::chrono::duration<double>(now - r.t_submit).count();
        r.done = true;
        sim.busy = false;
    }
    lane.tickets.clear();
    lane.n_solids = 0;
    lane.busy = false;
}

void fail(rmx_server* s, int64_t t, int status) {
    Req& r = s->reqs[t];
    r.status = status;
    r.latency = std::chrono::duration<double>(Clock::now() - r.t_submit).count();
    r.done = true;
}

// Form a batch for an idle lane from the queue, in arrival order: the first request whose
// simulation is not in flight fixes the option class; later compatible requests join
// while the lane's workspace (grown within the budget) holds them.  Returns false if
// nothing could be started.
bool dispatch(rmx_server* s, Lane& lane) {
    std::vector<int64_t> pick;
    std::vector<const rmx_grid*> grids;
    std::vector<rmx_solid> solids;
    rmx_options cls{};
    for (auto it = s->queue.begin(); it != s->queue.end() && (int)pick.size() < kMaxBatchRequests;) {
        const int64_t t = *it;
        Req& r = s->reqs[t];
        Sim& sim = s->sims[r.sim];
        bool in_pick = false;
        for (int64_t q : pick)
            if (s->reqs[q].sim == r.sim) in_pick = true;
        if (sim.busy || in_pick || (!pick.empty() && !same_class(cls, r.opt)) ||
            solids.size() + sim.solids.size() > (size_t)kMaxBatchSolids) {
            ++it;
            continue;
        }
        std::vector<const rmx_grid*> g2 = grids;
        std::vector<rmx_solid> s2 = solids;
        g2.insert(g2.end(), sim.grids.begin(), sim.grids.end());
        s2.insert(s2.end(), sim.solids.begin(), sim.solids.end());
        const size_t need = batch_ws(g2, s2, pick.empty() ? r.opt : cls, lane);
        const size_t free_bytes = s->budget > in_use(s) ? s->budget - in_use(s) : 0;
        const size_t have = lane.ctx->ws_size;
        const bool fits = need != (size_t)-1 && (need <= have || need - have <= free_bytes);
        if (!fits) {
            if (pick.empty()) {
                // Alone it needs more than this lane can hold now.  If it cannot fit even
                // with every idle workspace returned, it never will: fail it alone.
                const size_t ws_all = lanes_ws(s);
                const size_t cap = s->budget > s->resident ? s->budget - s->resident : 0;
                bool others_busy = false;
                for (auto& l : s->lanes) others_busy |= l.busy;
                if (need == (size_t)-1 || need > cap) {
                    fail(s, t, need == (size_t)-1 ? RMX_E_ARG : RMX_E_BUDGET);
                    --sim.queued;
                    it = s->queue.erase(it);
                    s->cv_done.notify_all();
                    continue;
                }
                if (!others_busy && ws_all > lane.ctx->ws_size) {
                    release_idle_ws(s);   // frees this lane too; retried on the next pass
                    return false;
                }
                return false;   // wait for running work to return memory
            }
            break;
        }
        if (pick.empty()) cls = r.opt;
        pick.push_back(t);
        grids.swap(g2);
        solids.swap(s2);
        it = s->queue.erase(it);
        --sim.queued;
    }
    if (pick.empty()) return false;
    for (int64_t t : pick) s->sims[s->reqs[t].sim].busy = true;
    lane.tickets = pick;
    lane.n_solids = solids.size();
    lane.busy = true;
    int rc = ctx_stats_host(lane.ctx, (size_t)kStatWords * solids.size());
    if (rc == RMX_OK) {
        lane.ctx->tmp_stats.resize(solids.size());
        rc = run_batch(lane.ctx, grids.data(), solids.data(), (int)solids.size(), &cls,
                       lane.stream, false, 0, true, nullptr);
    }
    if (rc == RMX_OK && hipEventRecord(lane.ev, lane.stream) != hipSuccess) rc = RMX_E_HIP;
    note_peak(s);
    if (rc != RMX_OK) {
        (void)hipStreamSynchronize(lane.stream);
        for (int64_t t : pick) {
            fail(s, t, rc);
            s->sims[s->reqs[t].sim].busy = false;
        }
        lane.tickets.clear();
        lane.busy = false;
        s->cv_done.notify_all();
    }
    return true;
}

void scheduler(rmx_server* s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        bool any_busy = false;
        for (auto& lane : s->lanes) {
            if (lane.busy && hipEventQuery(lane.ev) == hipSuccess) {
                retire(s, lane);
                s->cv_done.notify_all();
            }
        }
        if (s->stop) {
            bool busy = false;
            for (auto& lane : s->lanes) busy |= lane.busy;
            if (!busy) break;
        }
        for (auto& lane : s->lanes) {
            if (!lane.busy && !s->queue.empty() && !s->stop) dispatch(s, lane);
            any_busy |= lane.busy;
        }
        if (any_busy)
            s->cv_work.wait_for(lk, std::chrono::microseconds(20));
        else
            s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty(); });
        if (s->stop && s->queue.empty()) {
            bool busy = false;
            for (auto& lane : s->lanes) busy |= lane.busy;
            if (!busy) break;
        }
    }
}

}  // namespace

extern "C" {

int rmx_server_create(int device, size_t hbm_budget_bytes, int32_t n_streams,
                      rmx_server** out) {
    if (!out) return RMX_E_ARG;
    *out = nullptr;
    if (hbm_budget_bytes == 0 || n_streams < 1 || n_streams > kMaxStreams) return RMX_E_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return RMX_E_ARG;
    if (hipSetDevice(device) != hipSuccess) return RMX_E_HIP;
    rmx_server* s = new rmx_server();
    s->device = device;
    s->budget = hbm_budget_bytes;
    s->lanes.resize(n_streams);
    for (auto& l : s->lanes) {
        if (rmx_create(device, 0, &l.ctx) != RMX_OK || !(l.ctx->exact_ws = true) ||
            hipStreamCreateWithFlags(&l.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&l.ev, hipEventDisableTiming) != hipSuccess) {
            rmx_server_destroy(s);
            return RMX_E_HIP;
        }
    }
    s->sched = std::thread(scheduler, s);
    *out = s;
    return RMX_OK;
}

int rmx_server_register(rmx_server* s, const rmx_grid* grid, const rmx_solid* templ,
                        int32_t n_solids, int64_t* sim_id) {
    if (!s || !grid || !templ || n_solids < 1 || !sim_id) return RMX_E_ARG;
    Sim sim;
    sim.grid = *grid;
    sim.solids.assign(templ, templ + n_solids);
    size_t bytes = 0;
    std::vector<size_t> off(n_solids);
    for (int i = 0; i < n_solids; ++i) {
        rmx_solid& t = sim.solids[i];
        t.xi = nullptr;
        t.labels = nullptr;
        t.xi_normal = nullptr;
        t.decisions = nullptr;
        const int rc = validate_solid(grid, &t, false);
        if (rc != RMX_OK) return rc;
        const size_t nc = (size_t)t.ext[0] * t.ext[1] * t.ext[2];
        off[i] = bytes;
        bytes += (24 * nc + 255) / 256 * 256 + (nc + 255) / 256 * 256;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (bytes > s->budget) return RMX_E_BUDGET;
    if (in_use(s) + bytes > s->budget) {
        release_idle_ws(s);
        if (in_use(s) + bytes > s->budget) return RMX_E_BUDGET;
    }
    if (hipSetDevice(s->device) != hipSuccess) return RMX_E_HIP;
    if (hipMalloc(&sim.mem, bytes) != hipSuccess) return RMX_E_HIP;
    char* base = static_cast<char*>(sim.mem);
    for (int i = 0; i < n_solids; ++i) {
        rmx_solid& t = sim.solids[i];
        const size_t nc = (size_t)t.ext[0] * t.ext[1] * t.ext[2];
        t.xi = reinterpret_cast<double*>(base + off[i]);
        t.labels = reinterpret_cast<int8_t*>(base + off[i] + (24 * nc + 255) / 256 * 256);
    }
    sim.bytes = bytes;
    const int64_t id = s->next_sim++;
    auto& ref = s->sims[id];
    ref = std::move(sim);
    ref.grids.assign(ref.solids.size(), &ref.grid);
    s->resident += bytes;
    note_peak(s);
    *sim_id = id;
    return RMX_OK;
}

int rmx_server_field(rmx_server* s, int64_t sim_id, int32_t solid, double** xi,
                     int8_t** labels) {
    if (!s) return RMX_E_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->sims.find(sim_id);
    if (it == s->sims.end()) return RMX_E_NOTFOUND;
    if (solid < 0 || solid >= (int)it->second.solids.size()) return RMX_E_ARG;
    if (xi) *xi = it->second.solids[solid].xi;
    if (labels) *labels = it->second.solids[solid].labels;
    return RMX_OK;
}

int rmx_server_submit(rmx_server* s, int64_t sim_id, const rmx_options* opt, int64_t* ticket) {
    if (!s || !ticket) return RMX_E_ARG;
    rmx_options o;
    rmx_default_options(&o);
    if (opt) o = *opt;
    int rc = validate_options(&o);
    if (rc != RMX_OK) return rc;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return RMX_E_ARG;
    auto it = s->sims.find(sim_id);
    if (it == s->sims.end()) return RMX_E_NOTFOUND;
    if (s->queue.size() >= kMaxQueue) return RMX_E_BUSY;
    const int64_t t = s->next_ticket++;
    Req& r = s->reqs[t];
    r.sim = sim_id;
    r.opt = o;
    r.t_submit = Clock::now();
    s->queue.push_back(t);
    ++it->second.queued;
    *ticket = t;
    s->cv_work.notify_one();
    return RMX_OK;
}

int rmx_server_wait(rmx_server* s, int64_t ticket, rmx_solid_stats* stats, double* latency_s) {
    if (!s) return RMX_E_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->reqs.find(ticket) == s->reqs.end()) return RMX_E_NOTFOUND;
    // The lock is released while waiting: a submit may rehash `reqs` (invalidating
    // iterators) and another waiter of the same ticket may take the result and erase it,
    // so the request is looked up again by its ticket each time this waiter wakes.
    bool gone = false;
    s->cv_done.wait(lk, [&] {
        const auto w = s->reqs.find(ticket);
        if (w == s->reqs.end()) {
            gone = true;
            return true;
        }
        return w->second.done;
    });
    if (gone) return RMX_E_NOTFOUND;
    const auto it = s->reqs.find(ticket);
    const Req& r = it->second;
    if (stats && !r.stats.empty())
        std::memcpy(stats, r.stats.data(), sizeof(rmx_solid_stats) * r.stats.size());
    if (latency_s) *latency_s = r.latency;
    const int status = r.status;
    s->reqs.erase(it);
    s->cv_done.notify_all();   // another waiter of this ticket now finds it gone
    return status;
}

int rmx_server_release(rmx_server* s, int64_t sim_id) {
    if (!s) return RMX_E_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->sims.find(sim_id);
    if (it == s->sims.end()) return RMX_E_NOTFOUND;
    if (it->second.busy || it->second.queued > 0) return RMX_E_BUSY;
    if (hipSetDevice(s->device) != hipSuccess) return RMX_E_HIP;
    (void)hipFree(it->second.mem);
    s->resident -= it->second.bytes;
    s->sims.erase(it);
    return RMX_OK;
}

int rmx_server_usage(rmx_server* s, size_t* used, size_t* peak) {
    if (!s) return RMX_E_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    if (used) *used = in_use(s);
    if (peak) *peak = s->peak;
    return RMX_OK;
}

int rmx_server_destroy(rmx_server* s) {
    if (!s) return RMX_E_ARG;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        // queued requests that never started fail; running ones finish
        for (int64_t t : s->queue) {
            fail(s, t, RMX_E_ARG);
            --s->sims[s->reqs[t].sim].queued;
        }
        s->queue.clear();
        s->cv_done.notify_all();
    }
    s->cv_work.notify_all();
    if (s->sched.joinable()) s->sched.join();
    (void)hipSetDevice(s->device);
    for (auto& l : s->lanes) {
        if (l.stream) (void)hipStreamSynchronize(l.stream);
        if (l.ctx) rmx_destroy(l.ctx);
        if (l.ev) (void)hipEventDestroy(l.ev);
        if (l.stream) (void)hipStreamDestroy(l.stream);
    }
    for (auto& kv : s->sims)
        if (kv.second.mem) (void)hipFree(kv.second.mem);
    delete s;
    return RMX_OK;
}

}  // extern "C"
