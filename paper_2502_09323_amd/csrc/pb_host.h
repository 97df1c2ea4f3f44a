// pb_host.h -- host-side objects of libpb shared by the C ABI and the serving loop.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <utility>
#include <vector>

#include "pb_internal.h"

int pbi_fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

// Pinned host blocks kept for reuse: allocating and freeing pinned memory per problem costs
// milliseconds of host time, and freeing it waits for the device.  Blocks come in
// power-of-two sizes of at least 4 KiB; a block is handed back only once no copy that uses
// it can still be pending.  One host thread uses a context at a time.
struct PinnedPool {
    std::vector<std::pair<void*, size_t>> free_list;   // (block, capacity)
    static size_t capacity(size_t n)
    {
        size_t c = 4096;
        while (c < n) c <<= 1;
        return c;
    }
    // a block of at least n bytes and its capacity, or nullptr
    void* get(size_t n, size_t* cap)
    {
        const size_t c = capacity(n);
        for (size_t i = free_list.size(); i-- > 0;)
            if (free_list[i].second == c) {
                void* p = free_list[i].first;
                free_list.erase(free_list.begin() + (long)i);
                *cap = c;
                return p;
            }
        void* p = nullptr;
        if (hipHostMalloc(&p, c, hipHostMallocDefault) != hipSuccess) return nullptr;
        *cap = c;
        return p;
    }
    void put(void* p, size_t cap)
    {
        if (p) free_list.emplace_back(p, cap);
    }
    void release()
    {
        for (auto& b : free_list) (void)hipHostFree(b.first);
        free_list.clear();
    }
};

struct pb_ctx {
    int device;
    hipStream_t stream;
    pb_alloc_fn alloc;
    pb_free_fn free_fn;
    void* user;
    size_t budget;
    int profile;
    pbk::CGState* host_state;  // pinned, 2 slots for pipelined polling
    hipEvent_t ev[2];
    PinnedPool pinned;         // staging and read-back blocks of this context's problems
};

struct DevAlloc {
    pb_ctx* ctx;
    std::vector<std::pair<void*, size_t>> held;
    size_t bytes = 0;
    void* get(size_t n)
    {
        n = (n + 255) & ~(size_t)255;
        if (n == 0) n = 256;
        void* p = ctx->alloc(n, ctx->user);
        if (p) {
            held.emplace_back(p, n);
            bytes += n;
        }
        return p;
    }
    void put(void* p)
    {
        for (size_t i = 0; i < held.size(); ++i)
            if (held[i].first == p) {
                bytes -= held[i].second;
                ctx->free_fn(p, ctx->user);
                held.erase(held.begin() + (long)i);
                return;
            }
    }
    void release()
    {
        for (auto& h : held) ctx->free_fn(h.first, ctx->user);
        held.clear();
        bytes = 0;
    }
};

// temporaries of an asynchronous coefficient build
struct BuildTmp {
    pbk::Bins bn;
    int *bcnt = nullptr, *bstart = nullptr, *bcur = nullptr, *bids = nullptr;
    double* bxyzr = nullptr;  // the atoms' centres and radii in cell-list order
    uint32_t* cls = nullptr;
    int *bslots = nullptr, *bcuts = nullptr, *tot = nullptr;
    int nblk = 0;
    double* hpin = nullptr;   // pinned (context pool): atoms, charges, then the two counts
    size_t hpin_cap = 0;
    int* htot = nullptr;
    double* full = nullptr;   // device copy of user boundary values
    double* acell = nullptr;  // per cell-list slot: its atom's deposition cell, offsets and charge (8 doubles)
    double* dhpart = nullptr; // Debye-Hueckel partial sums per atom range and box node
};

struct pb_problem;

// one level of 2:1 refinement: the fine sub-lattice problem and the composite operator
struct RefineData {
    pb_problem* fine = nullptr;   // fine sub-lattice: geometry, cut list, energy read-back
    int nc[3] = {0, 0, 0};        // coarse cells per axis
    int brick = 4;
    double delta = 3.0;
    uint8_t* cells = nullptr;     // refinement flags of the coarse cells
    int64_t n_refined = 0;
    double* Kc = nullptr;         // coarse grid: K of the +x, +y, +z edges, lumped term [4][Nc]
    double* Kf = nullptr;         // fine sub-lattice, the same [4][Nf]
    uint8_t* rolec = nullptr;     // 1: coarse unknown
    uint8_t* rolef = nullptr;     // 1: fine unknown, 2: coincides with a coarse unknown, 3: hanging
    int64_t ng = 0;               // derived fine nodes (roles 2, 3)
    int64_t* gfine = nullptr;     // their fine element index
    int64_t* gpar = nullptr;      // [4*ng] coarse parents (unused slots repeat the first)
    int32_t* gnp = nullptr;       // parent counts 1, 2 or 4
    int64_t nr = 0;               // coarse nodes that are parents of derived fine nodes
    int64_t* rnode = nullptr;     // their coarse element index
    double *bc = nullptr, *rc = nullptr, *zc = nullptr, *pc = nullptr, *qc = nullptr, *dc = nullptr;
    double *bf = nullptr, *rf = nullptr, *zf = nullptr, *pf = nullptr, *qf = nullptr, *df = nullptr;
    // mixed precision: FP32 copies of K and D^-1 and the FP32 solver vectors (x: correction);
    // the FP64 r and q above then hold the true residual and the FP64 product
    float *Kc32 = nullptr, *Kf32 = nullptr;
    float *xc32 = nullptr, *rc32 = nullptr, *zc32 = nullptr, *pc32 = nullptr, *qc32 = nullptr, *dc32 = nullptr;
    float *xf32 = nullptr, *rf32 = nullptr, *zf32 = nullptr, *pf32 = nullptr, *qf32 = nullptr, *df32 = nullptr;
    double* part = nullptr;       // [3 * (nbc + nbf)] block partial sums
    int nbc = 0, nbf = 0;
    int64_t nunk_c = 0, nunk_f = 0, nhang = 0;
};

// multigrid preconditioner of a uniform problem (pb_mg.hip); level 0 is the problem's grid
constexpr int PB_MG_MAX_LEVELS = 12;
struct MGData {
    int nlev = 0;               // levels in use
    int nu = 1, cs = 4;         // sweeps per level and side, symmetric sweeps on the coarsest
    pbk::Grid g[PB_MG_MAX_LEVELS];
    void* K[PB_MG_MAX_LEVELS][3] = {};   // levels >= 1: K of the +x, +y, +z edges (element type)
    void* diag[PB_MG_MAX_LEVELS] = {};   // levels >= 1: diagonal
    void* dinv[PB_MG_MAX_LEVELS] = {};   // 1 / diagonal (level 0 too)
    void* x[PB_MG_MAX_LEVELS] = {};      // iterate (level 0: the CG vector z)
    void* b[PB_MG_MAX_LEVELS] = {};      // right-hand side (level 0: the CG residual)
    void* r[PB_MG_MAX_LEVELS] = {};      // residual at the red nodes (black entries 0)
    void *cr = nullptr, *cz = nullptr, *cp = nullptr, *cp2 = nullptr, *cq = nullptr;   // CG r, z, p (two), q
    void* cx = nullptr;         // CG x: the FP64 solution, or the FP32 correction (mixed)
    double* part = nullptr;     // [3 * nb] block partial sums
    int nb = 0;
    double* prz = nullptr;      // [nrz] r.z partial sums of the last half-sweep of a V-cycle
    int nrz = 0;
    // level 0 and the CG vectors are kept in the red-black layout (pb_mg.hip): Sh positions per
    // colour segment, Nrb elements per vector, and the node codes in that layout
    int Sh = 0;
    int64_t Nrb = 0;
    uint32_t* code_rb = nullptr;
    // natural-layout right-hand side and solution of level 0 for callers that work in that
    // layout (the two-level preconditioner of refined grids); made on first use
    void *nat_b = nullptr, *nat_x = nullptr;
    int ls = 0;                 // first level of the part of the V-cycle run in one block
    // the hierarchy's device descriptor, read by every kernel, and the launch tables of the
    // problem solved alone (device; solo_host holds what was copied there)
    void* dev = nullptr;
    void* solo_desc = nullptr;
    int* solo_off = nullptr;
    std::vector<char> solo_host;
};

// most problems of one batched multigrid launch
constexpr int PB_MG_MAX_BATCH = 64;

// launch tables of batched multigrid chunks: pinned staging and device memory, grown on demand
struct MGBatch {
    void* host = nullptr;
    void* dev = nullptr;
    size_t cap = 0;
    pb_alloc_fn alloc = nullptr;
    pb_free_fn free_fn = nullptr;
    void* user = nullptr;
};

struct pb_problem {
    pb_ctx* ctx;
    pb_params prm;
    int64_t na;
    pbk::Grid g;
    pbk::TileShape ts;
    pbk::Coef cf;
    double lB, kD;
    double ctr[3] = {0.0, 0.0, 0.0};   // centre of the atoms' bounding box (Atoms::cx, cy, cz)
    DevAlloc mem;
    // inputs
    double* xyzr = nullptr;
    double* q = nullptr;
    // coefficient maps
    uint32_t* code = nullptr;
    double* ck64 = nullptr;
    float* ck32 = nullptr;
    int* cutbase = nullptr;
    double* rhs = nullptr;
    double* gb = nullptr;
    double* x = nullptr;
    int64_t ncut = 0, nslot = 0;
    int64_t* cutkey = nullptr;
    double *alpha = nullptr, *kcut = nullptr, *rp = nullptr, *np = nullptr, *wp = nullptr;
    int* owner = nullptr;
    double *F = nullptr, *phip = nullptr, *pts = nullptr;
    // CG work: z = D^-1 r, w = D^-1 q and p, double buffered by iteration parity
    double* z64[2] = {nullptr, nullptr};
    double* w64[2] = {nullptr, nullptr};
    double* p64[2] = {nullptr, nullptr};
    float* d32 = nullptr;   // FP32 correction (the mixed form's x)
    float* z32[2] = {nullptr, nullptr};
    float* w32[2] = {nullptr, nullptr};
    float* p32[2] = {nullptr, nullptr};
    double *part = nullptr, *part_res = nullptr;
    pbk::CGState* st = nullptr;
    int nb = 0, nbres = 0;
    bool solved = false;
    BuildTmp* bt = nullptr;      // set while a build is in progress
    RefineData* ref = nullptr;   // set for a locally refined problem
    MGData* mg = nullptr;        // set once a multigrid-preconditioned solve has run
    hipEvent_t ev = nullptr;     // marks the end of the last asynchronous phase
    double* hout = nullptr;      // pinned (context pool): energy sums and the final CG state
    size_t hout_cap = 0;
    double* e_tmp[4] = {nullptr, nullptr, nullptr, nullptr};  // energy temporaries
    int e_nchunk = 0;

    // sampled kernel timings of the last solve (iteration kernel, tail kernel)
    double prof_stencil_ms = 0, prof_update_ms = 0;
    int prof_n = 0;
    // the energy N-body kernel of the last read-back, timed while profiling is on
    hipEvent_t nb_ev[2] = {nullptr, nullptr};
    bool nb_timed = false;
    double prof_nbody_ms = 0, prof_nbody_pairs = 0;
};


// asynchronous phases (all work on the problem's stream; pbi_event_done polls pb->ev)
int pbi_build_begin(pb_ctx* ctx, const pb_params* prm, int64_t na, const double* xyz, const double* rad,
                    const double* chg, pb_problem** out);
int pbi_build_continue(pb_problem* pb);
// the same for a sub-lattice whose node (i,j,k) is node (i,j,k) + off of the lattice given by
// prm's origin and spacing (atoms need only lie inside the sub-lattice)
int pbi_build_begin_sub(pb_ctx* ctx, const pb_params* prm, int64_t na, const double* xyz, const double* rad,
                        const double* chg, const int* off, pb_problem** out);
void pbi_build_end(pb_problem* pb);
// the cut edges counted by the first build phase (valid once its event has completed)
int64_t pbi_build_counted_cuts(const pb_problem* pb);
int pbi_event_done(pb_problem* pb);
void pbi_problem_destroy(pb_problem* pb, bool sync);   // sync=false: its event has completed
int pbi_energy_begin(pb_problem* pb, int finish_mixed);            // kernels + read-back
// take the device address of the allocation-free read-back's scratch array on `device` (the
// current device), once per device (pb_noalloc.hip)
int pbi_scratch_setup(int device);
// device bytes pbi_energy_begin allocates beyond what the problem holds
size_t pbi_energy_bytes(const pb_problem* pb);
// an upper estimate of the device bytes a mixed-form request holds at its peak (build,
// solve and energy read-back); ncut < 0: not yet counted, estimated from the atom radii
size_t pbi_request_bytes(const pb_params& p, int64_t na, const double* radius, int64_t ncut);
int pbi_energy_end(pb_problem* pb, pb_energy_out* out, pb_solve_stats* st);

// mixed-form solve split in steps for the serving loop (all work on the problem's stream)
int pbi_mixed_begin(pb_problem* pb);                              // buffers + first update
pbk::ProbDev<float> pbi_probdev(pb_problem* pb);

// locally refined problems (pb_refine.hip)
int pbi_refine_build(pb_problem* coarse, const double* xyz, const double* rad, const double* chg);
int pbi_refine_solve(pb_problem* pb, pbk::CGState* out);

// multigrid-preconditioned CG (pb_mg.hip)
int pbi_mg_solve(pb_problem* pb, pbk::CGState* out);
// the same in steps for the serving loop, all enqueued on stream s: the level hierarchy,
// then chunks of n iterations (first: x = 0 and the first residual before them; in mixed
// precision an iteration that follows a stop for a residual replacement runs that
// replacement instead of a step); finish folds a leftover FP32 correction into the solution
int pbi_mg_begin(pb_problem* pb, hipStream_t s);
// (sample: four events for the first iteration's V-cycle, or nullptr; see pb_get_profile)
int pbi_mg_chunk(pb_problem* pb, hipStream_t s, int n, bool first, hipEvent_t* sample);
int pbi_mg_finish(pb_problem* pb, hipStream_t s);
int pbi_mg_levels(const pb_problem* pb);
// Iterations to launch next for a problem whose last completed chunk ended in state st, with
// `pending` iterations launched since (at most cap; 0: the chunk in flight is expected to
// finish it).  At the mean rate at which the squared residual fell from ||b||^2 to rr over
// iter_count iterations it reaches the goal after some more; in mixed precision each residual
// replacement (one per delta2 of decrease, the last confirming convergence) takes an
// iteration of its own.  An estimate that falls short costs one more round trip; one that runs
// over, launches that return at once.
int pbi_mg_next_chunk(const pbk::CGState& st, int pending, int cap);
// x = 0 and the first residual of a multigrid problem, enqueued on s
int pbi_mg_start(pb_problem* pb, hipStream_t s);
// whether a problem can join batched multigrid chunks (more than one level, and no large
// coarsest level run in launches of its own)
bool pbi_mg_batchable(const pb_problem* pb);
// n iterations of every problem of pbs (at most PB_MG_MAX_BATCH, batchable, one precision and
// the same smoothing counts) in batched launches, then the problems' states into
// gather[0 .. pbs.size()) (device); ev (optional): 6 events per
// iteration, two around its operator pass, then four around its V-cycle and the first
// level-0 black half-sweep after the coarse correction
int pbi_mg_batch_chunk(const std::vector<pb_problem*>& pbs, hipStream_t s, int n, MGBatch* bb, pbk::CGState* gather,
                       hipEvent_t* ev);
// one V-cycle of pb's multigrid (set up by pbi_mg_begin, in pb's precision) on level 0:
// right-hand side pbi_mg_rhs0 (box nodes 0), correction in pbi_mg_sol0 (element type of the
// precision); gated on st running (status 0, ru 0) when st is given
void pbi_mg_vcycle_on(pb_problem* pb, hipStream_t s, const pbk::CGState* st);
void* pbi_mg_rhs0(pb_problem* pb);
void* pbi_mg_sol0(pb_problem* pb);
// one V-cycle on a vector over the padded level-0 layout (host arrays of g.N doubles)
int pbi_mg_vcycle_test(pb_problem* pb, const double* r_host, double* z_host);

// the problem's atoms as the kernels take them, with the centre of their bounding box
inline pbk::Atoms pbi_atoms(const pb_problem* pb)
{
    pbk::Atoms at{(int)pb->na, pb->xyzr, pb->q};
    at.cx = pb->ctr[0];
    at.cy = pb->ctr[1];
    at.cz = pb->ctr[2];
    return at;
}
