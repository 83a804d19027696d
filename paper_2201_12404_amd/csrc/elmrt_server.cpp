// elmrt_server.cpp -- a request loop over the C ABI of elmrt.h: jobs (problem
// statement, initial fields, step count) are queued, admitted in arrival
// order while their workspace fits a caller-owned device pool, kept resident,
// and advanced together in rounds: every round the first resident job in
// policy order (arrival, or least remaining work) and the later ones that fit
// a budget of cells that occupies the device form one batch per lattice and
// precision (elmrt_batch_*; a single job steps alone) that advances by the
// chunk or by the fewest steps any member still needs, so that jobs finish
// exactly; a job whose
// instability flag is seen set (polled after every round without waiting) is
// evicted and read out early.  A scheduling pass never waits for the device:
// it reads out the jobs whose last round has completed and uploads newly
// admitted ones on a second stream of the server's own, and enqueues the
// next round on the compute stream while fewer than two are in flight;
// finished jobs' memory returns to the pool once read out.  Built on the
// public entry points, and on the library's batch construction for tables
// that no kernel has read yet.
#include "../../include/elmrt.h"
#include "elmrt_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <string>
#include <thread>
#include <vector>

namespace {

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

elmrt_status sfail(elmrt_status st, const std::string& msg)
{
    elmrt::set_last_error(msg);
    return st;
}

// Lowest-address first-fit allocator over [0, size), 256-byte granules.
class Pool {
public:
    explicit Pool(size_t size) { free_[0] = size; }
    bool alloc(size_t bytes, size_t* off)
    {
        bytes = (bytes + 255) / 256 * 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            used_[*off] = bytes;
            return true;
        }
        return false;
    }
    void release(size_t off)
    {
        auto u = used_.find(off);
        if (u == used_.end()) return;
        size_t start = off, len = u->second;
        used_.erase(u);
        auto nx = free_.lower_bound(start);
        if (nx != free_.end() && nx->first == start + len) {
            len += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == start) {
                start = pv->first;
                len += pv->second;
                free_.erase(pv);
            }
        }
        free_[start] = len;
    }
    size_t free_bytes() const
    {
        size_t s = 0;
        for (auto& kv : free_) s += kv.second;
        return s;
    }

private:
    std::map<size_t, size_t> free_, used_;
};

enum JobState { QUEUED = 0, RESIDENT = 1, DONE = 2, FAILED = 3 };

struct Job {
    int64_t id = 0;
    elmrt_params p{};
    int D = 2;
    size_t N = 0;
    std::vector<double> rho0, u0;      // host inputs until admission
    int64_t steps = 0, done = 0;
    int64_t last_round = -1;            // round that enqueued the job's last steps
    int slot = -1;                      // word of the pinned flag array, or -1
    bool unstable = false;              // evicted: its flag was seen set
    size_t off = 0, bytes = 0;
    elmrt_sim* sim = nullptr;
    JobState state = QUEUED;
    double t_submit = 0, t_admit = 0, t_finish = 0;
    std::vector<double> rho, u;        // results
    double sums[4] = {0, 0, 0, 0};
    elmrt_status status = ELMRT_OK;
};

struct Group {                          // resident jobs of one (lattice, precision)
    elmrt_batch* batch = nullptr;
    std::vector<Job*> members;
    size_t off = 0;
    bool has_table = false;
    int64_t used_round = -1;            // last round that enqueued this batch's steps
};

struct RetiredTable {                   // pool memory of a replaced batch's job table
    size_t off;
    int64_t round;                      // free once this round's compute has completed
};

}  // namespace

struct elmrt_server {
    char* pool_base = nullptr;
    std::unique_ptr<Pool> pool;
    hipStream_t stream = nullptr;       // compute: the batches of resident jobs
    hipStream_t io = nullptr;           // uploads of admitted jobs, read-outs of finished ones
    hipEvent_t ev[2] = {nullptr, nullptr};   // end of each round's compute, alternating
    bool ev_recorded[2] = {false, false};
    int64_t round = 0;
    // pinned words the running jobs' instability flags are copied into after
    // every round (elmrt_poll_unstable), read without waiting
    uint32_t* flags = nullptr;
    std::vector<int> free_slots;
    int64_t chunk = 100;
    int64_t fill = 2 << 20;             // cells advanced per round (at least one job)
    int32_t policy = 0;                 // 0 arrival order, 1 shortest remaining work first,
                                        // 2 as 1 with the oldest job in every round
    int64_t next_id = 1;
    std::deque<Job*> queue;
    std::vector<Job*> resident;
    std::map<int64_t, std::unique_ptr<Job>> jobs;
    Group groups[4];                    // index 2 * lattice + precision
    std::vector<RetiredTable> retired;
    int64_t done_round = -1;            // every round <= this one has completed on the device
    int64_t lattice_updates = 0;        // cells x steps advanced

    ~elmrt_server()
    {
        (void)hipStreamSynchronize(stream);
        if (io) (void)hipStreamSynchronize(io);
        for (auto& g : groups)
            if (g.batch) elmrt_batch_destroy(g.batch);
        for (auto& kv : jobs)
            if (kv.second->sim) elmrt_destroy(kv.second->sim);
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
        if (io) (void)hipStreamDestroy(io);
        if (flags) (void)hipHostFree(flags);
    }
};

namespace {

elmrt_status admit(elmrt_server* s)
{
    while (!s->queue.empty()) {
        Job* j = s->queue.front();
        size_t off = 0;
        if (!s->pool->alloc(j->bytes, &off)) break;   // arrival order: wait for memory
        s->queue.pop_front();
        j->off = off;
        // upload and initialise on the io stream (init_fields waits for it),
        // then hand the job to the compute stream
        elmrt_status st = elmrt_create(&j->p, s->pool_base + off, j->bytes, s->io, &j->sim);
        if (st == ELMRT_OK) st = elmrt_init_fields(j->sim, j->rho0.data(), j->u0.data());
        if (st == ELMRT_OK) st = elmrt_set_stream(j->sim, s->stream);
        j->rho0.clear();
        j->rho0.shrink_to_fit();
        j->u0.clear();
        j->u0.shrink_to_fit();
        j->t_admit = now_s();
        if (st != ELMRT_OK) {
            j->status = st;
            j->state = FAILED;
            j->t_finish = j->t_admit;
            if (j->sim) elmrt_destroy(j->sim);
            j->sim = nullptr;
            s->pool->release(off);
            continue;
        }
        j->state = RESIDENT;
        if (!s->free_slots.empty()) {
            j->slot = s->free_slots.back();
            s->free_slots.pop_back();
            s->flags[j->slot] = 0u;
        }
        s->resident.push_back(j);
    }
    return ELMRT_OK;
}

// Read out a finished job on the io stream (its steps on the compute stream
// are complete) and return its memory to the pool.
elmrt_status retire(elmrt_server* s, Job* j)
{
    elmrt_set_stream(j->sim, s->io);
    j->rho.assign(j->N, 0.0);
    j->u.assign((size_t)j->D * j->N, 0.0);
    const elmrt_status st = elmrt_read_macros(j->sim, j->rho.data(), j->u.data(), j->sums);
    j->status = st;
    j->state = (st == ELMRT_OK || st == ELMRT_E_UNSTABLE) ? DONE : FAILED;
    j->t_finish = now_s();
    elmrt_destroy(j->sim);
    j->sim = nullptr;
    s->pool->release(j->off);
    if (j->slot >= 0) s->free_slots.push_back(j->slot);
    j->slot = -1;
    return ELMRT_OK;
}

// Return to the pool the tables of replaced batches whose last round has
// completed on the device.
void release_retired(elmrt_server* s)
{
    std::vector<RetiredTable> keep;
    for (const RetiredTable& t : s->retired) {
        if (t.round <= s->done_round) s->pool->release(t.off);
        else keep.push_back(t);
    }
    s->retired.swap(keep);
}

// Make group g's batch match its members (rebuilt when the set changed).  The
// old batch is released at once (it owns no device memory); its table's pool
// memory only after the last round that read it has completed, so the new
// table never lands on memory a kernel may still read, and the host need not
// wait for the device here.
elmrt_status sync_batch(elmrt_server* s, Group& g, const std::vector<Job*>& members)
{
    if (g.batch && members == g.members) return ELMRT_OK;
    if (g.batch) elmrt_batch_destroy(g.batch);
    g.batch = nullptr;
    if (g.has_table) {
        if (g.used_round < 0 || g.used_round <= s->done_round) s->pool->release(g.off);
        else s->retired.push_back({g.off, g.used_round});
    }
    g.has_table = false;
    g.used_round = -1;
    g.members = members;
    if (members.empty()) return ELMRT_OK;
    size_t bytes = 0;
    elmrt_status st = elmrt_batch_workspace_bytes((int32_t)members.size(), &bytes);
    if (st != ELMRT_OK) return st;
    if (!s->pool->alloc(bytes, &g.off)) return sfail(ELMRT_E_NOMEM, "pool has no room for a batch table");
    g.has_table = true;
    std::vector<elmrt_sim*> sims;
    for (Job* j : members) sims.push_back(j->sim);
    return elmrt::batch_create_fresh(sims.data(), (int32_t)sims.size(), s->pool_base + g.off, bytes, &g.batch);
}

// Wait until the compute enqueued by the rounds up to 'round' (whose event
// sits in 'slot') is complete.
elmrt_status wait_compute(elmrt_server* s, int slot, int64_t round)
{
    if (!s->ev_recorded[slot]) return ELMRT_OK;
    const hipError_t e = hipEventSynchronize(s->ev[slot]);
    if (e != hipSuccess) return sfail(ELMRT_E_DEVICE, std::string("hipEventSynchronize: ") + hipGetErrorString(e));
    s->done_round = std::max(s->done_round, round);
    return ELMRT_OK;
}

// Rounds known complete: the in-flight rounds' events, queried in order
// (no wait).  At most two rounds are in flight, so the two event slots (by
// round parity) are reused only once their round has completed.
void poll_done(elmrt_server* s)
{
    for (int64_t r = s->done_round + 1; r < s->round; ++r) {
        const int slot = (int)(r & 1);
        if (!s->ev_recorded[slot] || hipEventQuery(s->ev[slot]) != hipSuccess) break;
        s->done_round = r;
    }
}

// Relative device cost of one step of a cell: bytes per lattice update of
// the two-pass step (D2Q9 132 B, D3Q27 356 B).
double cell_cost(int D) { return D == 3 ? 356.0 / 132.0 : 1.0; }

// One scheduling pass, which never waits for the device: retire the jobs
// whose last round has completed (read-out on the io stream), admit queued
// jobs that fit the pool (upload and initialisation on the io stream), and,
// while fewer than two rounds are in flight, enqueue the next round on the
// compute stream.  A round advances resident jobs with steps left, in
// policy order (arrival, or least remaining work -- cells x steps -- first):
// the first one, and after it those that fit the rest of the fill budget:
// enough work to occupy the device, while the others wait their turn instead
// of slowing every running one down.
// Each (lattice, precision) group of the round is one batch (a group of one
// job steps through the single-simulation path); the costliest
// group advances by the chunk, a cheaper one by proportionally more steps (so
// that a small job beside a large one is not held to the large one's pace),
// and no group beyond the fewest steps any of its members still needs, so
// that every job stops exactly at its step count.  A job whose polled flag
// is seen set is evicted: not advanced further, read out as it stands.
elmrt_status round_once(elmrt_server* s, bool* progressed)
{
    *progressed = false;
    poll_done(s);
    release_retired(s);
    elmrt_status st;
    for (Job* j : s->resident)
        if (j->slot >= 0 && *(volatile uint32_t*)&s->flags[j->slot] != 0u) j->unstable = true;
    // retire the finished jobs whose last steps have completed
    std::vector<Job*> keep;
    for (Job* j : s->resident) {
        const bool finished = (j->done >= j->steps || j->unstable) && j->last_round <= s->done_round;
        if (!finished) {
            keep.push_back(j);
            continue;
        }
        if ((st = retire(s, j)) != ELMRT_OK) return st;
        *progressed = true;
    }
    s->resident.swap(keep);
    // admit the queued jobs that now fit
    const size_t before = s->queue.size();
    if ((st = admit(s)) != ELMRT_OK) return st;
    if (s->queue.size() != before) *progressed = true;
    if (s->round - 1 - s->done_round >= 2) return ELMRT_OK;   // the device is two rounds ahead
    std::vector<Job*> order;
    for (Job* j : s->resident)
        if (j->done < j->steps && !j->unstable) order.push_back(j);
    if (s->policy >= 1) {
        // resident is in arrival order: its first runnable job is the oldest
        Job* oldest = order.empty() ? nullptr : order.front();
        std::stable_sort(order.begin(), order.end(), [](const Job* a, const Job* b) {
            return (double)a->N * (double)(a->steps - a->done) < (double)b->N * (double)(b->steps - b->done);
        });
        if (s->policy == 2 && oldest) {   // the oldest first: it cannot starve
            order.erase(std::find(order.begin(), order.end(), oldest));
            order.insert(order.begin(), oldest);
        }
    }
    // the first job in order always runs; the others join while they fit the
    // rest of the fill budget, so that two jobs which each fill the device
    // are not put into one launch (it runs slower than the two alone)
    std::vector<Job*> running;
    int64_t cells = 0;
    for (Job* j : order) {
        if (!running.empty() && cells + (int64_t)j->N > s->fill) continue;
        running.push_back(j);
        cells += (int64_t)j->N;
    }
    const int cur = (int)(s->round & 1);
    if (!running.empty()) {
        std::vector<Job*> members[4];
        double cost[4] = {0, 0, 0, 0}, top = 0;
        for (Job* j : running) {
            const int gi = 2 * j->p.lattice + j->p.precision;
            members[gi].push_back(j);
            cost[gi] += (double)j->N * cell_cost(j->D);
        }
        for (double c : cost) top = std::max(top, c);
        for (int gi = 0; gi < 4; ++gi) {
            Group& g = s->groups[gi];
            // a group of one job advances through the single-simulation path
            // (the kernels of a job run alone, with no job table to read)
            const bool alone = members[gi].size() == 1;
            if ((st = sync_batch(s, g, alone ? std::vector<Job*>{} : members[gi])) != ELMRT_OK) return st;
            if (members[gi].empty()) continue;
            const double ratio = std::floor(top / cost[gi]);
            int64_t n = s->chunk * (int64_t)std::min(ratio, 1e6);
            for (Job* j : members[gi]) n = std::min(n, j->steps - j->done);
            if (alone) {
                if ((st = elmrt_step(members[gi][0]->sim, n)) != ELMRT_OK) return st;
            } else {
                if ((st = elmrt_batch_step(g.batch, n)) != ELMRT_OK) return st;
                g.used_round = s->round;
            }
            for (Job* j : members[gi]) {
                j->done += n;
                j->last_round = s->round;
                s->lattice_updates += (int64_t)j->N * n;
                if (j->slot >= 0 && (st = elmrt_poll_unstable(j->sim, &s->flags[j->slot])) != ELMRT_OK) return st;
            }
        }
        hipError_t e = hipEventRecord(s->ev[cur], s->stream);
        if (e != hipSuccess) return sfail(ELMRT_E_DEVICE, std::string("hipEventRecord: ") + hipGetErrorString(e));
        s->ev_recorded[cur] = true;
        ++s->round;
        *progressed = true;
    }
    if (s->resident.empty() && s->queue.empty()) {   // idle: release the batches and their tables
        for (int64_t r = s->done_round + 1; r < s->round; ++r)
            if ((st = wait_compute(s, (int)(r & 1), r)) != ELMRT_OK) return st;
        for (auto& g : s->groups)
            if ((st = sync_batch(s, g, {})) != ELMRT_OK) return st;
        release_retired(s);
    }
    return ELMRT_OK;
}

}  // namespace

extern "C" {

elmrt_status elmrt_server_create(void* dev_pool, size_t pool_bytes, void* stream, int64_t chunk_steps,
                                 elmrt_server** out)
{
    if (!out) return sfail(ELMRT_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!dev_pool || ((uintptr_t)dev_pool % 256) != 0) return sfail(ELMRT_E_INVALID, "pool is NULL or not 256-byte aligned");
    if (pool_bytes < 4096) return sfail(ELMRT_E_INVALID, "pool too small");
    if (chunk_steps < 1) return sfail(ELMRT_E_INVALID, "chunk_steps must be >= 1");
    elmrt_server* s = new elmrt_server;
    s->pool_base = (char*)dev_pool;
    s->pool.reset(new Pool(pool_bytes));
    s->stream = (hipStream_t)stream;
    s->chunk = chunk_steps;
    constexpr int kSlots = 4096;
    hipError_t e = hipStreamCreateWithFlags(&s->io, hipStreamNonBlocking);
    for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&s->ev[k], hipEventDisableTiming);
    if (e == hipSuccess) e = hipHostMalloc((void**)&s->flags, kSlots * sizeof(uint32_t), hipHostMallocDefault);
    for (int k = kSlots - 1; k >= 0 && e == hipSuccess; --k) s->free_slots.push_back(k);
    if (e != hipSuccess) {
        delete s;
        return sfail(ELMRT_E_DEVICE, std::string("server streams: ") + hipGetErrorString(e));
    }
    *out = s;
    return ELMRT_OK;
}

elmrt_status elmrt_server_set_fill(elmrt_server* s, int64_t cells)
{
    if (!s) return sfail(ELMRT_E_INVALID, "server is NULL");
    if (cells < 1) return sfail(ELMRT_E_INVALID, "fill must be >= 1 cell");
    s->fill = cells;
    return ELMRT_OK;
}

elmrt_status elmrt_server_set_policy(elmrt_server* s, int32_t policy)
{
    if (!s) return sfail(ELMRT_E_INVALID, "server is NULL");
    if (policy < 0 || policy > 2) return sfail(ELMRT_E_INVALID, "policy must be 0, 1 or 2");
    s->policy = policy;
    return ELMRT_OK;
}

elmrt_status elmrt_server_submit(elmrt_server* s, const elmrt_params* p, const double* rho0, const double* u0,
                                 int64_t steps, int64_t* job_id)
{
    if (!s) return sfail(ELMRT_E_INVALID, "server is NULL");
    if (!p || !rho0 || !u0) return sfail(ELMRT_E_INVALID, "params or fields are NULL");
    if (steps < 0) return sfail(ELMRT_E_INVALID, "steps < 0");
    size_t bytes = 0;
    elmrt_status st = elmrt_workspace_bytes(p, &bytes);
    if (st != ELMRT_OK) return sfail(st, std::string("job rejected: ") + elmrt_last_error());
    auto j = std::make_unique<Job>();
    j->id = s->next_id++;
    j->p = *p;
    j->D = p->lattice == ELMRT_D2Q9 ? 2 : 3;
    j->N = (size_t)(p->n[0] * p->n[1] * p->n[2]);
    j->rho0.assign(rho0, rho0 + j->N);
    j->u0.assign(u0, u0 + (size_t)j->D * j->N);
    j->steps = steps;
    j->bytes = bytes;
    j->t_submit = now_s();
    if (job_id) *job_id = j->id;
    s->queue.push_back(j.get());
    s->jobs[j->id] = std::move(j);
    return ELMRT_OK;
}

elmrt_status elmrt_server_run(elmrt_server* s, int32_t rounds, int32_t* queued, int32_t* resident)
{
    if (!s) return sfail(ELMRT_E_INVALID, "server is NULL");
    for (int32_t r = 0; r < rounds; ++r) {
        if (s->queue.empty() && s->resident.empty()) break;
        bool progressed = false;
        elmrt_status st = round_once(s, &progressed);
        if (st != ELMRT_OK) return st;
        // nothing to do until the device finishes a round: pause briefly
        // rather than spin
        if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(100));
    }
    if (queued) *queued = (int32_t)s->queue.size();
    if (resident) *resident = (int32_t)s->resident.size();
    return ELMRT_OK;
}

elmrt_status elmrt_server_job(elmrt_server* s, int64_t job_id, int32_t* state, double times[3], int64_t* steps_done)
{
    if (!s) return sfail(ELMRT_E_INVALID, "server is NULL");
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return sfail(ELMRT_E_INVALID, "unknown job");
    const Job* j = it->second.get();
    if (state) *state = (int32_t)j->state;
    if (times) {
        times[0] = j->t_submit;
        times[1] = j->t_admit;
        times[2] = j->t_finish;
    }
    if (steps_done) *steps_done = j->done;
    return ELMRT_OK;
}

elmrt_status elmrt_server_result(elmrt_server* s, int64_t job_id, double* rho, double* u, double* sums)
{
    if (!s) return sfail(ELMRT_E_INVALID, "server is NULL");
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return sfail(ELMRT_E_INVALID, "unknown job");
    Job* j = it->second.get();
    if (j->state == QUEUED || j->state == RESIDENT) return sfail(ELMRT_E_STATE, "job not finished");
    if (j->state == FAILED && j->rho.empty()) return sfail(j->status, "job failed");
    if (rho) std::copy(j->rho.begin(), j->rho.end(), rho);
    if (u) std::copy(j->u.begin(), j->u.end(), u);
    if (sums) std::copy(j->sums, j->sums + 4, sums);
    const elmrt_status st = j->status;
    // results are handed over once
    j->rho.clear();
    j->rho.shrink_to_fit();
    j->u.clear();
    j->u.shrink_to_fit();
    return st == ELMRT_E_UNSTABLE ? sfail(st, "job became unstable") : st;
}

elmrt_status elmrt_server_stats(elmrt_server* s, int64_t* lattice_updates, size_t* pool_free)
{
    if (!s) return sfail(ELMRT_E_INVALID, "server is NULL");
    if (lattice_updates) *lattice_updates = s->lattice_updates;
    if (pool_free) *pool_free = s->pool->free_bytes();
    return ELMRT_OK;
}

void elmrt_server_destroy(elmrt_server* s) { delete s; }

}  // extern "C"
