// pb_server.hip -- continuous-batching serving loop for linearized-PB solves.
//
// Requests (a molecule and a grid, mixed precision) queue on the host.  A request moves
// through: queued -> counting -> filling -> resident -> finishing -> done.  Coefficient builds
// and energy read-backs run on a second stream and each phase ends with an event the loop
// polls, so the host never blocks on them.  Each step of the loop
//   1. finishes the older of the two chunks kept in flight and reads every member's state
//      from one gathered copy;
//   2. advances builds whose phase has finished, and collects finished read-backs;
//   3. starts the read-back (final reliable update, energies) of problems that converged (or
//      ran out of iterations) once no chunk in flight still touches them;
//   4. starts builds for arrived requests while the resident count and the device-memory
//      budget allow;
//   5. launches one chunk for every resident problem: 16 CG iterations as batched launches
//      (each launch covers the tiles of all problems), then the batched reliable-update
//      kernels and a gather of all problem states.  Requests with the multigrid
//      preconditioner (worth it on large grids, where Jacobi-CG needs hundreds of iterations)
//      run their iterations as batched launches of their own (one launch per pass of the
//      V-cycle and of the CG step over all of them), then the batched restart from the true
//      residual where one is due, on a side stream that starts with the chunk and that the
//      gather waits for; the few that cannot be batched run their own launches on further
//      side streams.
// Every problem's blocks run the code and block numbering of its own solo launch, so a result
// does not depend on which other problems shared the batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <vector>

#include "pb_host.h"

using namespace pbk;

namespace {

constexpr int kChunkIters = 16;   // same chunk length as a solo mixed solve
constexpr int kServerTilePlanes = 32;   // long x-chunks: a batched launch has blocks to spare
constexpr int kMgStreams = 4;          // streams the multigrid problems are spread over
constexpr int kMgBatches = 4;          // batched multigrid groups per chunk (of PB_MG_MAX_BATCH)
// Multigrid problems converge in a few dozen iterations, so a fixed 16-iteration chunk with
// a second chunk in flight would launch many iterations that find the solve stopped.  Their
// chunks are sized instead: kMgFirst iterations, kMgSecond while the first is in flight, then
// the estimate from the residual decay seen so far (see mg_chunk_iters).
constexpr int kMgFirst = 12;
constexpr int kMgSecond = 6;

struct Request {
    pb_params prm;
    std::vector<double> xyz, rad, chg, bc;
    uint64_t id;
    double arrival;
    size_t est_bytes;
};

struct Active {
    pb_problem* pb;
    uint64_t id;
    double arrival;
    size_t counted;     // bytes of the memory budget held for it (its device memory, read-back included)
    int cancel;         // PB_ECANCELED or PB_ETIMEDOUT once cancelled: no more chunks, no read-back
    int launched;       // CG iterations launched for it
    int last_chunk;     // the last chunk that included it
    bool finished;      // converged, broke down or out of iterations; no more chunks
    bool mg;            // multigrid-preconditioned: its own launches on one of the side streams
    int lane;           // ... which one
    int pending;        // iterations launched in chunks not yet completed
    bool seen;          // snap holds the state after a completed chunk
    CGState snap;
};

struct Pending {        // a problem being built or read back on the build stream
    pb_problem* pb;
    uint64_t id;
    double arrival;
    int phase;          // 1 counting, 2 filling, 3 read-back
    size_t counted;     // bytes of the memory budget held for it: an estimate until the build ends
    int cancel;         // PB_ECANCELED or PB_ETIMEDOUT: dropped when its phase ends
};

struct Result {
    uint64_t id;
    pb_energy_out e;
    pb_solve_stats st;
    double done;
    int32_t code;
};

#define SCHK(expr)                                                                         \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return pbi_fail(PB_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));    \
    } while (0)

}  // namespace

struct pb_server {
    pb_ctx* ctx;     // batched iteration stream
    pb_ctx* bctx;    // build / energy stream
    int max_resident;
    size_t budget = 0, in_use = 0;   // in_use: sum of the `counted` bytes of all admitted requests
    size_t in_use_peak = 0;
    int64_t over_budget = 0;          // builds let past the budget (nothing else could free memory)
    double timeout_s = 0.0;           // per request, from its arrival (0: none)
    std::deque<Request> queue;
    std::vector<Active> act;
    std::vector<Pending> pend;
    std::vector<Result> done;
    std::chrono::steady_clock::time_point t0;
    // per in-flight slot: descriptors, offsets, gathered states (device and pinned host)
    ProbDev<float>* ddesc[2] = {nullptr, nullptr};
    int* doff[2] = {nullptr, nullptr};
    CGState* dgather[2] = {nullptr, nullptr};
    ProbDev<float>* hdesc[2] = {nullptr, nullptr};
    int* hoff[2] = {nullptr, nullptr};
    CGState* hgather[2] = {nullptr, nullptr};
    int cap[2] = {0, 0};
    std::vector<uint64_t> members[2];
    std::vector<int> members_n[2];   // iterations each member was given in the chunk
    hipEvent_t ev[2] = {};
    // multigrid problems run on side streams (a V-cycle is many small dependent launches;
    // several problems' launches overlap there); each chunk starts them after the chunk start
    // on the main stream and the main stream waits for them before the gather copy
    hipStream_t mgs[kMgStreams] = {};
    hipEvent_t start_ev[2] = {}, mg_ev[2][kMgStreams] = {};
    int next_lane = 0;
    bool inflight[2] = {false, false};
    int slot_chunk[2] = {-1, -1};
    int next = 0;
    int chunk_id = 0;
    int completed = -1;
    double t_wait = 0, t_retire = 0, t_admit = 0, t_launch = 0;   // host seconds per phase
    // sampled timing of the batched stencil launches (context profiling on)
    hipEvent_t pev[2][2 * kChunkIters];
    bool pev_made = false;
    bool prof_slot[2] = {false, false};
    std::vector<int64_t> prof_nu[2];     // interior unknowns of each member
    double prof_ms = 0, prof_bytes = 0;
    int64_t prof_launches = 0;
    // multigrid members run alone: the level-0 black half-sweep after the coarse correction
    // and the whole V-cycle of each chunk's first iteration, timed with events from a pool
    struct MgSample {
        uint64_t id;
        hipEvent_t e[4];
        int64_t nu;
    };
    std::vector<MgSample> mg_samples[2];
    std::vector<hipEvent_t> ev_pool;
    // batched multigrid chunks: launch tables, and per slot the batches launched (members,
    // their unknowns, iterations, four timing events per iteration)
    MGBatch mgb[2][kMgBatches];
    struct MgBatchRun {
        std::vector<uint64_t> ids;
        std::vector<int64_t> nu;
        int n;
        std::vector<hipEvent_t> ev;
    };
    std::vector<MgBatchRun> mg_batches[2];
    int64_t mg_batch_launches = 0;   // batched chunks launched
    double prof_mg_ms = 0, prof_mg_bytes = 0, prof_mg_vcycle_ms = 0;
    int64_t prof_mg_n = 0;
    double prof_mga_ms = 0, prof_mga_bytes = 0;   // the batched operator pass of the multigrid CG
    int64_t prof_mga_n = 0;
    // the energy N-body kernel of every request read back while build_ctx profiles
    double prof_nb_ms = 0, prof_nb_pairs = 0;
    int64_t prof_nb_n = 0;

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

void free_slot(pb_server* s, int k)
{
    if (s->ddesc[k]) s->ctx->free_fn(s->ddesc[k], s->ctx->user);
    if (s->doff[k]) s->ctx->free_fn(s->doff[k], s->ctx->user);
    if (s->dgather[k]) s->ctx->free_fn(s->dgather[k], s->ctx->user);
    if (s->hdesc[k]) (void)hipHostFree(s->hdesc[k]);
    if (s->hoff[k]) (void)hipHostFree(s->hoff[k]);
    if (s->hgather[k]) (void)hipHostFree(s->hgather[k]);
    s->ddesc[k] = nullptr;
    s->doff[k] = nullptr;
    s->dgather[k] = nullptr;
    s->hdesc[k] = nullptr;
    s->hoff[k] = nullptr;
    s->hgather[k] = nullptr;
    s->cap[k] = 0;
}

int ensure_slot(pb_server* s, int k, int P)
{
    if (s->cap[k] >= P) return PB_OK;
    free_slot(s, k);
    const int c = std::max(P, 8);
    s->ddesc[k] = (ProbDev<float>*)s->ctx->alloc(sizeof(ProbDev<float>) * c, s->ctx->user);
    s->doff[k] = (int*)s->ctx->alloc(sizeof(int) * 4 * (c + 1), s->ctx->user);
    s->dgather[k] = (CGState*)s->ctx->alloc(sizeof(CGState) * c, s->ctx->user);
    if (!s->ddesc[k] || !s->doff[k] || !s->dgather[k]) return pbi_fail(PB_ENOMEM, "batch descriptors");
    SCHK(hipHostMalloc((void**)&s->hdesc[k], sizeof(ProbDev<float>) * c, hipHostMallocDefault));
    SCHK(hipHostMalloc((void**)&s->hoff[k], sizeof(int) * 4 * (c + 1), hipHostMallocDefault));
    SCHK(hipHostMalloc((void**)&s->hgather[k], sizeof(CGState) * c, hipHostMallocDefault));
    s->cap[k] = c;
    return PB_OK;
}

// move a request's share of the budget count from `counted` to `bytes`
void charge(pb_server* s, size_t& counted, size_t bytes)
{
    s->in_use = s->in_use - std::min(s->in_use, counted) + bytes;
    counted = bytes;
    s->in_use_peak = std::max(s->in_use_peak, s->in_use);
}

// wait for the chunk in slot k and record every member's state
int complete_slot(pb_server* s, int k)
{
    if (!s->inflight[k]) return PB_OK;
    SCHK(hipEventSynchronize(s->ev[k]));
    s->inflight[k] = false;
    s->completed = std::max(s->completed, s->slot_chunk[k]);
    if (s->prof_slot[k]) {
        for (int it = 0; it < kChunkIters; ++it) {
            float ms = 0;
            SCHK(hipEventElapsedTime(&ms, s->pev[k][2 * it], s->pev[k][2 * it + 1]));
            s->prof_ms += ms;
        }
        s->prof_launches += kChunkIters;
    }
    // batched multigrid runs: iteration j of a batch ran for the members whose iteration count
    // grew by more than j over the chunk (a member that stops stays stopped until the chunk's
    // restart)
    for (auto& br : s->mg_batches[k]) {
        std::vector<int> done(br.ids.size(), 0);
        for (size_t q = 0; q < br.ids.size(); ++q)
            for (size_t m = 0; m < s->members[k].size(); ++m)
                if (s->members[k][m] == br.ids[q])
                    for (auto& a : s->act)
                        if (a.id == br.ids[q]) done[q] = s->hgather[k][m].iter_count - a.snap.iter_count;
        for (int j = 0; j < br.n && !br.ev.empty(); ++j) {
            double nu = 0.0;
            for (size_t q = 0; q < br.ids.size(); ++q)
                if (j < done[q]) nu += (double)br.nu[q];
            if (nu <= 0.0) continue;
            const hipEvent_t* e = br.ev.data() + 6 * j;
            float ap = 0, sw = 0, vc = 0;
            SCHK(hipEventElapsedTime(&ap, e[0], e[1]));
            SCHK(hipEventElapsedTime(&sw, e[3], e[4]));
            SCHK(hipEventElapsedTime(&vc, e[2], e[5]));
            // algorithmic bytes per unknown: the black half-sweep 10 (x of the other colour,
            // b, 1/D and the codes of the swept one read, x of the swept one written: 20 B per
            // node of that colour), the operator pass 20 (z, the old direction and the codes
            // read; the new direction and q written)
            s->prof_mg_ms += sw;
            s->prof_mg_vcycle_ms += vc;
            s->prof_mg_bytes += 10.0 * nu;
            s->prof_mg_n += 1;
            s->prof_mga_ms += ap;
            s->prof_mga_bytes += 20.0 * nu;
            s->prof_mga_n += 1;
        }
        for (auto e : br.ev) s->ev_pool.push_back(e);
    }
    s->mg_batches[k].clear();
    for (size_t m = 0; m < s->members[k].size(); ++m) {
        for (auto& a : s->act) {
            if (a.id != s->members[k][m] || a.last_chunk < s->slot_chunk[k]) continue;
            for (auto& smp : s->mg_samples[k]) {
                // the sampled (first) iteration of the chunk ran if any iteration did
                if (smp.id != a.id || s->hgather[k][m].iter_count <= a.snap.iter_count) continue;
                float sw = 0, vc = 0;
                SCHK(hipEventElapsedTime(&sw, smp.e[1], smp.e[2]));
                SCHK(hipEventElapsedTime(&vc, smp.e[0], smp.e[3]));
                s->prof_mg_ms += sw;
                s->prof_mg_vcycle_ms += vc;
                // algorithmic bytes per unknown of the FP32 half-sweep in the red-black layout:
                // x of the other colour, b, 1/D and the node codes of the swept colour read, x
                // of the swept colour written
                s->prof_mg_bytes += 10.0 * (double)smp.nu;
                s->prof_mg_n += 1;
            }
            if (s->prof_slot[k] && !a.mg) {
                // algorithmic bytes of the FP32 iteration kernel per unknown: read z, w, p, x
                // and the node code, write z, w, p, x
                const int done = s->hgather[k][m].iter_count - a.snap.iter_count;
                s->prof_bytes += (double)s->prof_nu[k][m] * 36.0 * (done > 0 ? done : 0);
            }
            a.snap = s->hgather[k][m];
            a.pending -= s->members_n[k][m];
            a.seen = true;
            const int stt = a.snap.status;
            if (stt == 1 || stt == 2 || a.launched >= a.pb->prm.max_iter) a.finished = true;
        }
    }
    for (auto& smp : s->mg_samples[k])
        for (int e = 0; e < 4; ++e) s->ev_pool.push_back(smp.e[e]);
    s->mg_samples[k].clear();
    return PB_OK;
}

void add_result(pb_server* s, uint64_t id, int code, const pb_energy_out* e, const pb_solve_stats* st)
{
    Result r;
    memset(&r, 0, sizeof r);
    r.id = id;
    r.code = code;
    if (e) r.e = *e;
    if (st) r.st = *st;
    r.done = s->now();
    s->done.push_back(r);
}

// something other than builds waiting for memory will release memory later
bool others_progressing(const pb_server* s, const Pending* self)
{
    if (!s->act.empty()) return true;
    for (const auto& p : s->pend)
        if (&p != self && p.phase >= 2) return true;
    return false;
}

// drop a pending problem (its phase event has completed) with a result code
void drop_pending(pb_server* s, size_t i, int code)
{
    Pending& p = s->pend[i];
    add_result(s, p.id, code, nullptr, nullptr);
    charge(s, p.counted, 0);
    pbi_problem_destroy(p.pb, false);
    s->pend.erase(s->pend.begin() + (long)i);
}

// advance builds and read-backs whose last phase has finished (never blocks)
int progress(pb_server* s)
{
    for (size_t i = 0; i < s->pend.size();) {
        Pending& p = s->pend[i];
        const int d = pbi_event_done(p.pb);
        if (d < 0) return d;
        if (!d) {
            ++i;
            continue;
        }
        int rc = PB_OK;
        if (p.cancel) {
            drop_pending(s, i, p.cancel);
            continue;
        }
        if (p.phase == 1) {
            // the counts are known: hold the budget for the request's actual cut list before
            // the build allocates it, or wait while other requests will free memory
            const size_t need = pbi_request_bytes(p.pb->prm, p.pb->na, nullptr, pbi_build_counted_cuts(p.pb));
            if (s->budget && need > s->budget) {
                drop_pending(s, i, pbi_fail(PB_ENOMEM, "request %llu needs %zu bytes, budget %zu",
                                            (unsigned long long)p.id, need, s->budget));
                continue;
            }
            if (s->budget && need > p.counted && s->in_use - p.counted + need > s->budget) {
                if (others_progressing(s, &p)) {
                    ++i;
                    continue;
                }
                ++s->over_budget;
            }
            charge(s, p.counted, need);
            rc = pbi_build_continue(p.pb);
            if (!rc)
                rc = p.pb->prm.precond == PB_PRECOND_MG ? pbi_mg_begin(p.pb, p.pb->ctx->stream) : pbi_mixed_begin(p.pb);
            if (!rc && hipEventRecord(p.pb->ev, p.pb->ctx->stream) != hipSuccess) rc = PB_EDEVICE;
            if (!rc) {
                p.phase = 2;
                ++i;
                continue;
            }
        } else if (p.phase == 2) {
            pbi_build_end(p.pb);
            // from here on the count is exact: what the problem holds and what its read-back
            // will allocate
            charge(s, p.counted, pb_problem_bytes(p.pb) + pbi_energy_bytes(p.pb));
            Active a;
            memset(&a.snap, 0, sizeof a.snap);
            a.pb = p.pb;
            a.id = p.id;
            a.arrival = p.arrival;
            a.counted = p.counted;
            a.cancel = 0;
            a.launched = 0;
            a.pending = 0;
            a.seen = false;
            a.last_chunk = -1;
            a.finished = false;
            a.mg = p.pb->prm.precond == PB_PRECOND_MG;
            a.lane = a.mg ? (s->next_lane++ % kMgStreams) : 0;
            s->act.push_back(a);
            s->pend.erase(s->pend.begin() + (long)i);
            continue;
        } else {
            pb_energy_out e;
            pb_solve_stats st;
            pbi_energy_end(p.pb, &e, &st);
            if (p.pb->prof_nbody_pairs > 0) {
                s->prof_nb_ms += p.pb->prof_nbody_ms;
                s->prof_nb_pairs += p.pb->prof_nbody_pairs;
                s->prof_nb_n += 1;
            }
            add_result(s, p.id, st.status, &e, &st);
            charge(s, p.counted, 0);
            pbi_problem_destroy(p.pb, false);  // its read-back event has completed
            s->pend.erase(s->pend.begin() + (long)i);
            continue;
        }
        // a phase failed: report and drop the problem
        add_result(s, p.id, rc, nullptr, nullptr);
        charge(s, p.counted, 0);
        pb_problem_free(p.pb);
        s->pend.erase(s->pend.begin() + (long)i);
    }
    return PB_OK;
}

// start the read-back of problems that stopped iterating and are in no chunk in flight
int retire(pb_server* s)
{
    for (size_t i = 0; i < s->act.size();) {
        Active& a = s->act[i];
        if (!(a.finished && a.last_chunk <= s->completed)) {
            ++i;
            continue;
        }
        const int rc = a.cancel ? a.cancel : pbi_energy_begin(a.pb, 1);
        if (rc) {
            add_result(s, a.id, rc, nullptr, nullptr);
            charge(s, a.counted, 0);
            pb_problem_free(a.pb);   // no chunk in flight touches it
        } else {
            s->pend.push_back(Pending{a.pb, a.id, a.arrival, 3, a.counted, 0});
        }
        s->act.erase(s->act.begin() + (long)i);
    }
    return PB_OK;
}

// requests past their time limit: queued ones complete at once, admitted ones are cancelled
// (an admitted problem is released once no launch in flight touches it)
void expire(pb_server* s)
{
    if (s->timeout_s <= 0.0) return;
    const double t = s->now();
    for (size_t i = 0; i < s->queue.size();) {
        const Request& q = s->queue[i];
        if (t - q.arrival > s->timeout_s) {
            add_result(s, q.id, PB_ETIMEDOUT, nullptr, nullptr);
            s->queue.erase(s->queue.begin() + (long)i);
        } else {
            ++i;
        }
    }
    for (auto& a : s->act)
        if (!a.cancel && t - a.arrival > s->timeout_s) {
            a.cancel = PB_ETIMEDOUT;
            a.finished = true;
        }
    for (auto& p : s->pend)
        if (!p.cancel && t - p.arrival > s->timeout_s) p.cancel = PB_ETIMEDOUT;
}

int building(const pb_server* s)
{
    int n = 0;
    for (const auto& p : s->pend) n += p.phase < 3;
    return n;
}

int admit(pb_server* s)
{
    const double t = s->now();
    while (!s->queue.empty() && s->queue.front().arrival <= t &&
           (int)s->act.size() + building(s) < s->max_resident) {
        Request& q = s->queue.front();
        if (s->budget && q.est_bytes > s->budget) {
            add_result(s, q.id, pbi_fail(PB_ENOMEM, "request %llu: estimated %zu bytes, budget %zu",
                                         (unsigned long long)q.id, q.est_bytes, s->budget),
                       nullptr, nullptr);
            s->queue.pop_front();
            continue;
        }
        if (s->budget && s->in_use + q.est_bytes > s->budget) break;  // wait for memory
        pb_params prm = q.prm;
        prm.bc_values = q.bc.empty() ? nullptr : q.bc.data();
        if (prm.tile_planes == 0) prm.tile_planes = kServerTilePlanes;
        pb_problem* pb = nullptr;
        const int rc = pbi_build_begin(s->bctx, &prm, (int64_t)q.rad.size(), q.xyz.data(), q.rad.data(),
                                       q.chg.data(), &pb);
        if (rc != PB_OK) {
            add_result(s, q.id, rc, nullptr, nullptr);
            s->queue.pop_front();
            continue;
        }
        size_t counted = 0;
        charge(s, counted, q.est_bytes);
        s->pend.push_back(Pending{pb, q.id, q.arrival, 1, counted, 0});
        s->queue.pop_front();
    }
    return PB_OK;
}

// Iterations to give a multigrid problem in the next chunk; 0 when the chunk in flight is
// expected to finish it (pbi_mg_next_chunk, from the state after its last completed chunk).
int mg_chunk_iters(const Active& a)
{
    if (!a.seen) return a.pending == 0 ? kMgFirst : kMgSecond;
    return pbi_mg_next_chunk(a.snap, a.pending, kChunkIters);
}

// an event from the pool (timing only: no system-scope fence, whose cache writeback would count)
int pool_event(pb_server* s, hipEvent_t* e)
{
    if (s->ev_pool.empty()) {
        hipEvent_t x;
        SCHK(hipEventCreateWithFlags(&x, hipEventDisableSystemFence));
        s->ev_pool.push_back(x);
    }
    *e = s->ev_pool.back();
    s->ev_pool.pop_back();
    return PB_OK;
}

int64_t unknowns(const pb_problem* pb)
{
    const Grid& g = pb->g;
    return (int64_t)(g.nx - 2) * (g.ny - 2) * (g.nz - 2);
}

int launch_chunk(pb_server* s, int k)
{
    // Jacobi members first (one batched chunk), then the multigrid members in batched groups,
    // then the multigrid members run alone; the gathered states follow the same order
    std::vector<Active*> mem, solo;
    std::vector<int> solo_n;
    std::vector<std::vector<Active*>> grp;
    std::vector<int> grp_n;
    for (auto& a : s->act) {
        if (a.finished) continue;
        if (!a.mg) {
            mem.push_back(&a);
            continue;
        }
        const int n = mg_chunk_iters(a);
        if (n <= 0) continue;
        if (!pbi_mg_batchable(a.pb)) {
            solo.push_back(&a);
            solo_n.push_back(n);
            continue;
        }
        // a group of one precision and smoothing counts with room left
        int gi = -1;
        for (size_t g = 0; g < grp.size(); ++g) {
            const pb_problem* f = grp[g][0]->pb;
            if ((int)grp[g].size() < PB_MG_MAX_BATCH && f->prm.precision == a.pb->prm.precision &&
                f->mg->nu == a.pb->mg->nu && f->mg->cs == a.pb->mg->cs) {
                gi = (int)g;
                break;
            }
        }
        if (gi < 0) {
            if ((int)grp.size() == kMgBatches) continue;   // no room in this chunk: the next one
            grp.emplace_back();
            grp_n.push_back(0);
            gi = (int)grp.size() - 1;
        }
        grp[gi].push_back(&a);
        grp_n[gi] = std::max(grp_n[gi], n);
    }
    int Q = (int)solo.size();
    for (auto& g : grp) Q += (int)g.size();
    const int P = (int)mem.size();
    s->members[k].clear();
    s->members_n[k].clear();
    if (P + Q == 0) return PB_OK;
    int rc = ensure_slot(s, k, P + Q);
    if (rc) return rc;
    BatchTotals t{0, 0, 0};
    int* o = s->hoff[k];
    for (int p = 0; p < P; ++p) {
        const ProbDev<float> d = pbi_probdev(mem[p]->pb);
        s->hdesc[k][p] = d;
        t.st = (t.st + 7) & ~7;   // block b of each problem on XCD b % 8, as in a solo launch
        o[p] = t.st;
        o[(P + 1) + p] = t.add;
        o[2 * (P + 1) + p] = t.res;
        t.st += d.ts.items;
        t.add += d.nadd;
        t.res += d.nbres;
        s->members[k].push_back(mem[p]->id);
        s->members_n[k].push_back(kChunkIters);
    }
    for (size_t g = 0; g < grp.size(); ++g)
        for (auto* a : grp[g]) {
            s->members[k].push_back(a->id);
            s->members_n[k].push_back(grp_n[g]);
        }
    for (size_t q = 0; q < solo.size(); ++q) {
        s->members[k].push_back(solo[q]->id);
        s->members_n[k].push_back(solo_n[q]);
    }
    o[P] = t.st;
    o[(P + 1) + P] = t.add;
    o[2 * (P + 1) + P] = t.res;
    hipStream_t st = s->ctx->stream;
    SCHK(hipEventRecord(s->start_ev[k], st));
    s->prof_slot[k] = s->ctx->profile != 0 && P > 0;
    if (s->prof_slot[k] && !s->pev_made) {
        for (int a = 0; a < 2; ++a)
            for (int e = 0; e < 2 * kChunkIters; ++e)
                SCHK(hipEventCreateWithFlags(&s->pev[a][e], hipEventDisableSystemFence));   // timing only
        s->pev_made = true;
    }
    s->prof_nu[k].clear();
    for (int p = 0; p < P; ++p) s->prof_nu[k].push_back(unknowns(mem[p]->pb));
    for (int q = 0; q < Q; ++q) s->prof_nu[k].push_back(0);
    if (P > 0) {
        SCHK(hipMemcpyAsync(s->ddesc[k], s->hdesc[k], sizeof(ProbDev<float>) * P, hipMemcpyHostToDevice, st));
        SCHK(hipMemcpyAsync(s->doff[k], s->hoff[k], sizeof(int) * 3 * (P + 1), hipMemcpyHostToDevice, st));
        SCHK(launch_batch_chunk(st, s->ddesc[k], s->doff[k], P, t, kChunkIters, s->dgather[k],
                                s->prof_slot[k] ? s->pev[k] : nullptr));
    }
    // group g on side stream g, the members alone on the stream of their lane
    bool used[kMgStreams] = {};
    for (size_t g = 0; g < grp.size(); ++g) used[g % kMgStreams] = true;
    for (auto* a : solo) used[a->lane] = true;
    for (int j = 0; j < kMgStreams; ++j)
        if (used[j]) SCHK(hipStreamWaitEvent(s->mgs[j], s->start_ev[k], 0));
    int slot = P;
    for (size_t g = 0; g < grp.size(); ++g) {
        hipStream_t ms = s->mgs[g % kMgStreams];
        std::vector<pb_problem*> pbs;
        pb_server::MgBatchRun br;
        br.n = grp_n[g];
        for (auto* a : grp[g]) {
            if (a->launched == 0 && (rc = pbi_mg_start(a->pb, ms))) return rc;
            pbs.push_back(a->pb);
            br.ids.push_back(a->id);
            br.nu.push_back(unknowns(a->pb));
        }
        if (s->ctx->profile) {
            br.ev.resize((size_t)6 * br.n);
            for (auto& e : br.ev)
                if ((rc = pool_event(s, &e))) return rc;
        }
        if (!s->mgb[k][g].alloc) {
            s->mgb[k][g].alloc = s->ctx->alloc;
            s->mgb[k][g].free_fn = s->ctx->free_fn;
            s->mgb[k][g].user = s->ctx->user;
        }
        if ((rc = pbi_mg_batch_chunk(pbs, ms, br.n, &s->mgb[k][g], s->dgather[k] + slot,
                                     br.ev.empty() ? nullptr : br.ev.data())))
            return rc;
        slot += (int)pbs.size();
        s->mg_batches[k].push_back(std::move(br));
        ++s->mg_batch_launches;
    }
    for (size_t q = 0; q < solo.size(); ++q) {
        pb_problem* pb = solo[q]->pb;
        hipStream_t ms = s->mgs[solo[q]->lane];
        hipEvent_t* sample = nullptr;
        if (s->ctx->profile && pb->mg && pb->mg->nlev > 1) {
            pb_server::MgSample smp;
            smp.id = solo[q]->id;
            for (int e = 0; e < 4; ++e)
                if ((rc = pool_event(s, &smp.e[e]))) return rc;
            smp.nu = unknowns(pb);
            s->mg_samples[k].push_back(smp);
            sample = s->mg_samples[k].back().e;
        }
        if ((rc = pbi_mg_chunk(pb, ms, solo_n[q], solo[q]->launched == 0, sample))) return rc;
        SCHK(hipMemcpyAsync(s->dgather[k] + slot, pb->st, sizeof(CGState), hipMemcpyDeviceToDevice, ms));
        ++slot;
    }
    for (int j = 0; j < kMgStreams; ++j)
        if (used[j]) {
            SCHK(hipEventRecord(s->mg_ev[k][j], s->mgs[j]));
            SCHK(hipStreamWaitEvent(st, s->mg_ev[k][j], 0));
        }
    SCHK(hipMemcpyAsync(s->hgather[k], s->dgather[k], sizeof(CGState) * (P + Q), hipMemcpyDeviceToHost, st));
    SCHK(hipEventRecord(s->ev[k], st));
    s->inflight[k] = true;
    s->slot_chunk[k] = s->chunk_id;
    for (auto* a : mem) {
        a->launched += kChunkIters;
        a->pending += kChunkIters;
        a->last_chunk = s->chunk_id;
    }
    for (size_t g = 0; g < grp.size(); ++g)
        for (auto* a : grp[g]) {
            a->launched += grp_n[g];
            a->pending += grp_n[g];
            a->last_chunk = s->chunk_id;
        }
    for (size_t q = 0; q < solo.size(); ++q) {
        solo[q]->launched += solo_n[q];
        solo[q]->pending += solo_n[q];
        solo[q]->last_chunk = s->chunk_id;
    }
    s->chunk_id++;
    return PB_OK;
}

}  // namespace

extern "C" {

int pb_server_create(pb_ctx* ctx, pb_ctx* build_ctx, int32_t max_resident, pb_server** out)
{
    if (!ctx || !build_ctx || !out || max_resident <= 0) return pbi_fail(PB_EINVAL, "bad argument");
    if (ctx->device != build_ctx->device) return pbi_fail(PB_EINVAL, "contexts on different devices");
    *out = nullptr;
    SCHK(hipSetDevice(ctx->device));
    pb_server* s = new pb_server();
    s->ctx = ctx;
    s->bctx = build_ctx;
    s->max_resident = max_resident;
    s->budget = ctx->budget;
    s->t0 = std::chrono::steady_clock::now();
    bool ok = true;
    for (int k = 0; k < 2; ++k) {
        ok = ok && hipEventCreateWithFlags(&s->ev[k], hipEventDisableTiming) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&s->start_ev[k], hipEventDisableTiming) == hipSuccess;
        for (int j = 0; j < kMgStreams; ++j)
            ok = ok && hipEventCreateWithFlags(&s->mg_ev[k][j], hipEventDisableTiming) == hipSuccess;
    }
    for (int j = 0; j < kMgStreams; ++j) ok = ok && hipStreamCreate(&s->mgs[j]) == hipSuccess;
    if (!ok) {
        pb_server_destroy(s);
        return pbi_fail(PB_EDEVICE, "server streams or events");
    }
    *out = s;
    return PB_OK;
}

double pb_server_now(const pb_server* s) { return s ? s->now() : 0.0; }

int pb_submit(pb_server* s, const pb_params* prm, int64_t n_atoms, const double* xyz, const double* radius,
              const double* charge, uint64_t request_id, double arrival_time_s)
{
    if (!s || !prm) return pbi_fail(PB_EINVAL, "NULL argument");
    if (prm->precision != PB_MIXED) return pbi_fail(PB_EINVAL, "the serving loop runs the mixed form only");
    if (prm->refine) return pbi_fail(PB_EINVAL, "the serving loop runs uniform grids only");
    if (n_atoms < 0 || (n_atoms > 0 && (!xyz || !radius || !charge))) return pbi_fail(PB_EINVAL, "bad atoms");
    Request q;
    q.prm = *prm;
    q.xyz.assign(xyz, xyz + 3 * n_atoms);
    q.rad.assign(radius, radius + n_atoms);
    q.chg.assign(charge, charge + n_atoms);
    if (prm->bc == PB_BC_USER && prm->bc_values) {
        const size_t nf = (size_t)prm->n[0] * prm->n[1] * prm->n[2];
        q.bc.assign(prm->bc_values, prm->bc_values + nf);
    }
    q.prm.bc_values = nullptr;
    q.id = request_id;
    q.arrival = arrival_time_s;
    q.est_bytes = pbi_request_bytes(*prm, n_atoms, radius, -1);
    s->queue.push_back(std::move(q));
    return PB_OK;
}

int pb_server_step(pb_server* s, int32_t* n_active, int32_t* n_queued)
{
    if (!s) return pbi_fail(PB_EINVAL, "NULL server");
    SCHK(hipSetDevice(s->ctx->device));
    const int k = s->next;
    double t = s->now(), t2;
    int rc = complete_slot(s, k);  // the slot about to be reused holds the older chunk
    t2 = s->now(); s->t_wait += t2 - t; t = t2;
    expire(s);
    if (!rc) rc = progress(s);
    if (!rc) rc = retire(s);
    t2 = s->now(); s->t_retire += t2 - t; t = t2;
    if (!rc) rc = admit(s);
    t2 = s->now(); s->t_admit += t2 - t; t = t2;
    if (!rc) rc = launch_chunk(s, k);
    t2 = s->now(); s->t_launch += t2 - t; t = t2;
    if (rc) return rc;
    if (s->inflight[k]) {
        s->next ^= 1;
    } else if (s->inflight[k ^ 1]) {
        // nothing new to launch: drain the other chunk so its finished problems can retire
        if ((rc = complete_slot(s, k ^ 1))) return rc;
        if ((rc = retire(s))) return rc;
        t2 = s->now(); s->t_wait += t2 - t; t = t2;
    } else if (!s->pend.empty()) {
        // only builds or read-backs are pending: wait for the oldest instead of spinning
        (void)hipEventSynchronize(s->pend.front().pb->ev);
        if ((rc = progress(s))) return rc;
        t2 = s->now(); s->t_wait += t2 - t; t = t2;
    }
    if (n_active) *n_active = (int32_t)(s->act.size() + s->pend.size());
    if (n_queued) *n_queued = (int32_t)s->queue.size();
    return PB_OK;
}

int pb_poll(pb_server* s, uint64_t* ids, pb_energy_out* results, pb_solve_stats* stats, double* done_time_s,
            int32_t* codes, int32_t max, int32_t* n_done)
{
    if (!s || !n_done || max < 0) return pbi_fail(PB_EINVAL, "bad argument");
    const int n = std::min<int>(max, (int)s->done.size());
    for (int i = 0; i < n; ++i) {
        const Result& r = s->done[i];
        if (ids) ids[i] = r.id;
        if (results) results[i] = r.e;
        if (stats) stats[i] = r.st;
        if (done_time_s) done_time_s[i] = r.done;
        if (codes) codes[i] = r.code;
    }
    s->done.erase(s->done.begin(), s->done.begin() + n);
    *n_done = n;
    return PB_OK;
}

int pb_cancel(pb_server* s, uint64_t request_id)
{
    if (!s) return pbi_fail(PB_EINVAL, "NULL server");
    for (size_t i = 0; i < s->queue.size(); ++i)
        if (s->queue[i].id == request_id) {
            add_result(s, request_id, PB_ECANCELED, nullptr, nullptr);
            s->queue.erase(s->queue.begin() + (long)i);
            return PB_OK;
        }
    for (auto& a : s->act)
        if (a.id == request_id && !a.cancel) {
            a.cancel = PB_ECANCELED;
            a.finished = true;
            return PB_OK;
        }
    for (auto& p : s->pend)
        if (p.id == request_id && !p.cancel) {
            p.cancel = PB_ECANCELED;
            return PB_OK;
        }
    return pbi_fail(PB_EINVAL, "request %llu is not queued or running", (unsigned long long)request_id);
}

int pb_server_set_timeout(pb_server* s, double seconds)
{
    if (!s || !(seconds >= 0.0) || !std::isfinite(seconds)) return pbi_fail(PB_EINVAL, "bad argument");
    s->timeout_s = seconds;
    return PB_OK;
}

int pb_server_memory(const pb_server* s, size_t* in_use, size_t* peak, int64_t* over_budget)
{
    if (!s) return pbi_fail(PB_EINVAL, "NULL server");
    if (in_use) *in_use = s->in_use;
    if (peak) *peak = s->in_use_peak;
    if (over_budget) *over_budget = s->over_budget;
    return PB_OK;
}

int pb_server_profile(const pb_server* s, double* stencil_ms_total, double* stencil_bytes_total,
                      int64_t* stencil_launches)
{
    if (!s) return pbi_fail(PB_EINVAL, "NULL server");
    if (stencil_ms_total) *stencil_ms_total = s->prof_ms;
    if (stencil_bytes_total) *stencil_bytes_total = s->prof_bytes;
    if (stencil_launches) *stencil_launches = s->prof_launches;
    return PB_OK;
}

int pb_server_profile_mg(const pb_server* s, double* sweep_ms_total, double* sweep_bytes_total,
                         double* vcycle_ms_total, int64_t* samples)
{
    if (!s) return pbi_fail(PB_EINVAL, "NULL server");
    if (sweep_ms_total) *sweep_ms_total = s->prof_mg_ms;
    if (sweep_bytes_total) *sweep_bytes_total = s->prof_mg_bytes;
    if (vcycle_ms_total) *vcycle_ms_total = s->prof_mg_vcycle_ms;
    if (samples) *samples = s->prof_mg_n;
    return PB_OK;
}

int pb_server_profile_mg_apply(const pb_server* s, double* ms_total, double* bytes_total, int64_t* launches)
{
    if (!s) return pbi_fail(PB_EINVAL, "NULL server");
    if (ms_total) *ms_total = s->prof_mga_ms;
    if (bytes_total) *bytes_total = s->prof_mga_bytes;
    if (launches) *launches = s->prof_mga_n;
    return PB_OK;
}

int pb_server_profile_energy(const pb_server* s, double* nbody_ms_total, double* pairs_total, int64_t* calls)
{
    if (!s) return pbi_fail(PB_EINVAL, "NULL server");
    if (nbody_ms_total) *nbody_ms_total = s->prof_nb_ms;
    if (pairs_total) *pairs_total = s->prof_nb_pairs;
    if (calls) *calls = s->prof_nb_n;
    return PB_OK;
}

int pb_server_times(const pb_server* s, double* out4)
{
    if (!s || !out4) return pbi_fail(PB_EINVAL, "NULL argument");
    out4[0] = s->t_wait;
    out4[1] = s->t_retire;
    out4[2] = s->t_admit;
    out4[3] = s->t_launch;
    return PB_OK;
}

void pb_server_destroy(pb_server* s)
{
    if (!s) return;
    (void)hipSetDevice(s->ctx->device);
    (void)hipStreamSynchronize(s->ctx->stream);
    (void)hipStreamSynchronize(s->bctx->stream);
    for (int j = 0; j < kMgStreams; ++j)
        if (s->mgs[j]) (void)hipStreamSynchronize(s->mgs[j]);
    for (auto& a : s->act) pb_problem_free(a.pb);
    for (auto& p : s->pend) pb_problem_free(p.pb);
    for (int j = 0; j < kMgStreams; ++j)
        if (s->mgs[j]) (void)hipStreamDestroy(s->mgs[j]);
    for (int k = 0; k < 2; ++k)
        for (auto& smp : s->mg_samples[k])
            for (int e = 0; e < 4; ++e) (void)hipEventDestroy(smp.e[e]);
    for (auto e : s->ev_pool) (void)hipEventDestroy(e);
    for (int k = 0; k < 2; ++k) {
        for (auto& br : s->mg_batches[k])
            for (auto e : br.ev) (void)hipEventDestroy(e);
        for (int g = 0; g < kMgBatches; ++g) {
            MGBatch& b = s->mgb[k][g];
            if (b.host) (void)hipHostFree(b.host);
            if (b.dev) b.free_fn(b.dev, b.user);
        }
    }
    for (int k = 0; k < 2; ++k) {
        free_slot(s, k);
        if (s->ev[k]) (void)hipEventDestroy(s->ev[k]);
        if (s->start_ev[k]) (void)hipEventDestroy(s->start_ev[k]);
        for (int j = 0; j < kMgStreams; ++j)
            if (s->mg_ev[k][j]) (void)hipEventDestroy(s->mg_ev[k][j]);
        if (s->pev_made)
            for (int e = 0; e < 2 * kChunkIters; ++e) (void)hipEventDestroy(s->pev[k][e]);
    }
    delete s;
}

}  // extern "C"
