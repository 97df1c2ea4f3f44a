/*
 * pb.h -- C ABI of the MI355X (gfx950) linearized Poisson-Boltzmann grid solver.
 *
 * The library solves, on one GPU, the linearized Poisson-Boltzmann equation of
 * Sect. 2.1 (eq. LPBE) for a solute made of charged atom balls, discretized as in
 * Sect. 3 of the paper: a vertex-based Cartesian scheme whose condensed operator is a
 * 7-point stencil with one permittivity per grid edge (Sect. 3.1, eq. matrixequation),
 * the weighted harmonic average on edges that cross the molecular surface (Sect. 3.2,
 * eq. WHA), and the solvation energy read back from surface quantities only
 * (Sect. 3.3: Coulomb pair sum, flux-based polarization charges, and the ionic surface
 * integral of eq. energy_ion with the surface potential of eq. phi0).
 *
 * Units.  Lengths in Angstrom, charges in units of e, temperature in K, ionic strength
 * in mol/L of a 1:1 salt.  Energies are returned in kT, potentials in kT/e.
 *
 * Grid.  n[0] x n[1] x n[2] nodes, node (i,j,k) at origin + h*(i,j,k).  All nodes on the
 * box faces carry Dirichlet values; the unknowns are the interior nodes.  Host arrays
 * over the grid use the order ((i*n[1] + j)*n[2] + k), z fastest.
 *
 * Ownership.  The caller owns every input array; the library copies what it needs.
 * Device memory is obtained only through the allocator callbacks given to
 * pb_ctx_create and is returned through them by the matching *_free/destroy call.
 * All GPU work is issued on the stream given to pb_ctx_create.
 *
 * Errors.  Every int-returning call returns PB_OK (0) or a negative PB_E* code and
 * never aborts.  pb_last_error() returns a message describing the last failure on the
 * calling thread.
 */
#ifndef PB_H
#define PB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    PB_OK = 0,
    PB_EINVAL = -1,      /* bad parameters or atoms (checked on the host before any launch) */
    PB_ENOMEM = -2,      /* allocation failed or a request exceeds the memory budget */
    PB_ENOCONV = -3,     /* max_iter reached; the last iterate and statistics are returned */
    PB_EBREAKDOWN = -4,  /* CG breakdown: p.Ap <= 0 or a non-finite scalar */
    PB_EDEVICE = -5,     /* a HIP runtime call failed; see pb_last_error() */
    PB_ECANCELED = -6,   /* serving: the request was cancelled (pb_cancel) */
    PB_ETIMEDOUT = -7    /* serving: the request did not complete within the server's time limit */
};

enum { PB_BC_ZERO = 0, PB_BC_DH = 1, PB_BC_USER = 2 };
enum { PB_FP64 = 0, PB_MIXED = 1 };
enum { PB_PRECOND_JACOBI = 0, PB_PRECOND_MG = 1 };

typedef struct pb_ctx pb_ctx;
typedef struct pb_problem pb_problem;
typedef struct pb_server pb_server;

/* Device allocator: must return memory usable by kernels on the context's device and
 * stream, aligned to at least 256 bytes, or NULL on failure. */
typedef void* (*pb_alloc_fn)(size_t bytes, void* user);
typedef void (*pb_free_fn)(void* ptr, void* user);

/* Create a context on HIP device `device` issuing work on `hip_stream` (a hipStream_t;
 * NULL means the null stream).  `alloc`/`free_fn` are required.  `hbm_budget_bytes`
 * bounds the device memory of problems admitted by a server (0 = no bound).
 * Errors: PB_EINVAL (missing callbacks, bad device), PB_EDEVICE. */
int pb_ctx_create(int device, void* hip_stream, pb_alloc_fn alloc, pb_free_fn free_fn,
                  void* user, size_t hbm_budget_bytes, pb_ctx** out);
void pb_ctx_destroy(pb_ctx* ctx);

/* Message of the last failure on the calling thread ("" if none). */
const char* pb_last_error(void);

/* Problem statement (Sect. 2: eps_in, eps_out, ionic strength, temperature; Sect. 2.3:
 * box boundary conditions; Sect. 3: grid spacing). */
typedef struct {
    double eps_in;          /* solute relative permittivity (e.g. 2) */
    double eps_out;         /* solvent relative permittivity (e.g. 80) */
    double ionic_strength_M;/* 1:1 salt, mol/L (e.g. 0.145) */
    double temperature_K;   /* e.g. 298 */
    double h;               /* grid spacing, Angstrom */
    int32_t n[3];           /* nodes per axis, each in [3, 4096]; n[0]*n[1]*(n[2] + 31
                               pad nodes, rounded up to a multiple of 32) < 2^29 */
    double origin[3];       /* coordinates of node (0,0,0) */
    int32_t bc;             /* PB_BC_ZERO | PB_BC_DH | PB_BC_USER */
    const double* bc_values;/* PB_BC_USER: host array over the full grid; only box-face
                               entries are read.  Ignored otherwise. */
    int32_t precision;      /* PB_FP64, or PB_MIXED: FP32 coefficients, vectors and CG with
                               FP64 reliable updates (true residual, solution accumulation);
                               the Debye-Hueckel box values then use FP32 exponentials and
                               inverse distances with FP64 sums */
    double rtol;            /* stop when ||b - A x||_2 <= rtol ||b||_2 (FP64 path: CG
                               recursive residual; mixed: the FP64 true residual) */
    double inner_rtol;      /* PB_MIXED: reliable-update factor: the FP32 recursive residual
                               may drop by this factor before an FP64 true-residual update */
    int32_t max_iter;       /* bound on launched CG iterations */
    int32_t tile_planes;    /* planes per x-chunk of the iteration kernel's tiles: 0 = chosen
                               from the grid (short chunks on small grids, so that a solve
                               alone still spreads over the GPU; the serving loop takes 32
                               instead, as its launches hold many problems), else a multiple
                               of 4 in [4, 128].  It changes only the summation order of the
                               reductions: a problem gives bit-identical results with the
                               same value alone or in the serving loop. */
    int32_t refine;         /* 0: uniform grid.  2: de-refinement toward the box (the
                               paper's treatment of the box, Sect. 3.4, exploiting
                               de-refinement for more efficient BCs, with one
                               level): the grid given is the coarse far field, and every
                               coarse cell that meets the solute's extent (atom centres -/+
                               radii) widened by refine_shell_A on all three axes is split,
                               rounded up to bricks as below; use with PB_BC_ZERO on a box
                               far from the solute.  Otherwise as refine = 1.
                               1: one level of 2:1 local refinement (the
                               paper's octree restricted to one level, Sect. 3): a coarse cell
                               of size h is split into 8 cells of size h/2 when a crossing
                               point of the surface with the h/2 lattice lies within
                               refine_shell_A of it (distance to the closed cell), rounded up
                               to aligned bricks of refine_brick^3 coarse cells.  Nodes of the
                               fine cells that lie on a face or edge of an unrefined cell are
                               hanging: they take the mean of the 2 or 4 coarse nodes of that
                               edge or face (P), and the operator is P^T K P over cell-wise
                               assembled K.  Solved by Jacobi-CG over the unknowns of both
                               grids, in FP64 or, with PB_MIXED, in FP32 with FP64 reliable
                               updates (the refined-grid solution and energies are FP64 in
                               both).  Needs at least one atom and refined cells away from
                               the box faces (PB_EINVAL otherwise). */
    double refine_shell_A;  /* refine: distance in Angstrom (e.g. 3.0) */
    int32_t refine_brick;   /* refine: brick edge in coarse cells, 1..64 (e.g. 4) */
    int32_t precond;        /* PB_PRECOND_JACOBI: diagonal (the default).  PB_PRECOND_MG:
                               one geometric-multigrid V-cycle per CG step, smoothed by
                               red-black symmetric Gauss-Seidel (the paper's SSOR preconditioner
                               with omega = 1, Sect. 4, in an order a GPU can sweep in
                               parallel): levels take every second node while n-1 is even on
                               every axis (with one level the preconditioner is red-black
                               symmetric Gauss-Seidel itself); coarse edges combine the fine
                               ones in series along the edge and averaged across it; trilinear
                               interpolation and its transpose.  With refine: the symmetric
                               two-level preconditioner
                               of the composite system, z1 = w D^-1 r, z2 = z1 + I V(I^T (r -
                               A z1)), z = z2 + w D^-1 (r - A z2), w = 0.8, V one V-cycle of
                               the coarse grid's multigrid (from its own node-code map), I
                               the trilinear interpolation of the coarse grid to the
                               unknowns. */
    int32_t mg_smooth;      /* PB_PRECOND_MG: red-black sweeps before and after the coarse
                               correction on each level, 1..8 (0 = 1) */
    int32_t mg_coarse_sweeps; /* PB_PRECOND_MG: symmetric sweeps on the coarsest level,
                               1..64 (0 = 4) */
    int32_t mg_levels;      /* PB_PRECOND_MG: at most this many levels, 0..12 (0 = as many as
                               the grid allows, up to 12) */
} pb_params;

/* Build the coefficient maps of a problem on the device (paper Sect. 2.1 and 3.1-3.2):
 * atom cell list, solute/solvent node classification (a node is solute iff strictly
 * inside an atom ball), edge permittivities with the WHA on cut edges (alpha measured
 * from the solute end to the first exit from the union of balls), the cut-edge list with
 * crossing points and sphere normals, marching-cubes area weights, the trilinear load
 * 4 pi sum q_i w_n(r_i) (eq. RVop_), boundary values and their lift, and the Jacobi
 * diagonal.
 *   xyz    : host, 3*n_atoms doubles, atom centres (x0,y0,z0,x1,...)
 *   radius : host, n_atoms doubles, finite and >= 1e-6 A
 *   charge : host, n_atoms doubles
 * Every atom ball must lie strictly inside [origin + h, origin + (n-2) h] on each axis.
 * On success *out owns all device state of the problem.
 * Errors: PB_EINVAL (non-finite values, eps <= 0, n < 3, h <= 0, an atom too close to the
 * box, bad bc/precision, missing bc_values), PB_ENOMEM, PB_EDEVICE. */
int pb_build_coeffs(pb_ctx* ctx, const pb_params* params, int64_t n_atoms, const double* xyz,
                    const double* radius, const double* charge, pb_problem** out);

typedef struct {
    int32_t iters;          /* CG iterations (FP32 iterations in the mixed form) */
    int32_t outer_iters;    /* mixed: FP64 reliable updates after the first; FP64: 0 */
    int32_t status;         /* PB_OK, PB_ENOCONV or PB_EBREAKDOWN */
    int32_t reserved;
    double relres;          /* final relative residual (see pb_params.rtol) */
    double t_solve_s;       /* wall time of pb_solve */
} pb_solve_stats;

/* Solve A phi = b with preconditioned CG (the paper uses CG, Sect. 4; the preconditioner is
 * pb_params.precond: Jacobi, or the multigrid / two-level preconditioner), either in
 * FP64 throughout or as FP32 CG with FP64 reliable updates: whenever the FP32 recursive
 * residual has dropped by inner_rtol, the FP32 correction is added to the FP64 solution and
 * the FP32 residual is replaced by the FP64 true residual b - A x (exact coefficients), with
 * the search direction kept; convergence is judged on the FP64 true residual.  The solution
 * stays on the device.  Returns PB_OK, PB_ENOCONV or PB_EBREAKDOWN (stats filled in all
 * three cases), or PB_EDEVICE. */
int pb_solve(pb_problem* pb, pb_solve_stats* stats);

typedef struct {
    double e_coul;          /* sum_{i<j} q_i q_j /(eps_in r_ij)            (Sect. 3.3) */
    double e_pol;           /* 1/2 sum_i q_i sum_p q_p / |r_p - r_i|        (Sect. 3.3.1) */
    double e_ion;           /* eq. energy_ion with MC areas and eq. phi0     (Sect. 3.3.2) */
    double e_solv;          /* e_pol + e_ion */
    double e_total;         /* e_coul + e_pol + e_ion */
    double q_pol_total;     /* sum_p q_p, in e */
    double area_total;      /* sum of marching-cubes area weights, Angstrom^2 */
    int64_t n_cut;          /* number of cut edges (= polarization charges) */
    double t_energy_s;      /* wall time of pb_energy */
} pb_energy_out;

/* Binding energy of a complex from its two parts (paper Sect. 6.2, binding energy
 * calculation): ddG = dG_complex - dG_1 - dG_2, with dG the total electrostatic energy
 * e_coul + e_pol + e_ion (eq. energyPart), and the same difference for each component.  The
 * three energies must come from solves on the same grid (box, spacing and origin), so that
 * discretization errors largely cancel.  Host-only arithmetic; no device work.
 * Errors: PB_EINVAL (NULL argument). */
typedef struct {
    double ddg_total;
    double ddg_coul;
    double ddg_pol;
    double ddg_ion;
} pb_binding_out;

int pb_binding_ddg(const pb_energy_out* complex_e, const pb_energy_out* part1, const pb_energy_out* part2,
                   pb_binding_out* out);

/* Energy read-back after pb_solve.  phi_reac_per_atom (optional, host, n_atoms doubles)
 * receives phi_pol + phi_ion at each atom centre in kT/e.  Errors: PB_EINVAL (not
 * solved), PB_EDEVICE. */
int pb_energy(pb_problem* pb, pb_energy_out* out, double* phi_reac_per_atom);

/* pb_energy for callers that cannot allocate memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the same kernels and results, with no
 * device, pinned or pageable allocation.  The read-back's buffers (per cut edge: flux, surface
 * potential and the N-body point, 96 bytes; per atom: the N-body partial sums, Coulomb and
 * reaction potentials; the sums) live in one static device array of
 * pb_energy_noalloc_limit() bytes (128 MiB), which every device the library runs on holds
 * until the process ends; its address is taken when the first context on the device is
 * created.  When the N-body sum in pb_energy's chunking does not fit, fewer chunks are used
 * (only the order of the FP64 additions changes).  The energies go to *out, the reaction
 * potentials (kT/e, optional) to the caller's host array phi_reac_per_atom[n_atoms]; the
 * call returns when they are there.  Unlike pb_energy it leaves nothing with the problem, so
 * pb_copy_cut's F and phip stay those of the last pb_energy.  Every call on one device shares
 * the array: calls that overlap on one device (other host threads, other streams) race and
 * must be serialized by the caller.
 * Errors: PB_EINVAL (NULL argument, not solved), PB_ENOMEM (the problem needs more than the
 * limit even in one chunk: about 1.3M cut edges; use pb_energy), PB_EDEVICE. */
int pb_energy_noalloc(pb_problem* pb, pb_energy_out* out, double* phi_reac_per_atom);

/* Size in bytes of pb_energy_noalloc's static scratch array. */
size_t pb_energy_noalloc_limit(void);

/* Grid energy after pb_solve (Sect. 3.3, electrostatic energy), in kT: half the sum over
 * the interior grid nodes of the charge deposited there (trilinear weights of each atom's
 * cell, the right-hand side's charge term) times the potential there; charge that the
 * deposition would put on box nodes is left out, as in the right-hand side.  It includes the
 * grid's self-energy, which cancels in the difference of two solves of the same geometry and
 * grid: at the actual ionic strength and at zero ionic strength the difference estimates the
 * ionic energy without a volume integral.  *e_grid is a host double.  Uniform grids only.
 * Errors: PB_EINVAL (NULL argument, not solved, a locally refined problem), PB_ENOMEM,
 * PB_EDEVICE. */
int pb_grid_energy(pb_problem* pb, double* e_grid);

/* Copy the potential on the full grid (kT/e, box nodes hold the boundary values) into a
 * host array of n[0]*n[1]*n[2] doubles. */
int pb_copy_potential(const pb_problem* pb, double* host_phi);

/* Release all device memory of a problem (waits for its stream). */
void pb_problem_free(pb_problem* pb);

/* One V-cycle of the multigrid preconditioner of a PB_PRECOND_MG problem on a given vector
 * (parity tests; builds the level hierarchy on first use).
 *   r_host : host, nx*ny*nz doubles (z contiguous); values on box nodes are ignored
 *   z_host : host, nx*ny*nz doubles, written; box nodes 0.  In PB_MIXED the V-cycle runs in
 *            FP32 (r rounded to FP32 on the way in).
 *   levels : optional, receives the number of levels
 * Overwrites the solver's CG work vectors (not the solution).  PB_EINVAL for a problem
 * without the multigrid preconditioner. */
int pb_mg_vcycle(pb_problem* pb, const double* r_host, double* z_host, int32_t* levels);

/* Locally refined problems (refine = 1).  The fine cells live on a sub-lattice of the h/2
 * lattice: fine node (a,b,c) of it is node (a,b,c) + fine_offset of the lattice with the
 * problem's origin and spacing h/2 (coarse node (i,j,k) is lattice node (2i,2j,2k)). */
typedef struct {
    int32_t fine_n[3];        /* nodes of the fine sub-lattice per axis */
    int32_t fine_offset[3];
    int64_t refined_cells;    /* coarse cells split into fine cells */
    int64_t hanging_nodes;
    int64_t unknowns_coarse;  /* unknowns on the coarse grid and on the fine sub-lattice */
    int64_t unknowns_fine;
} pb_refine_stats;

/* Fills *out (all zero for a uniform problem). */
int pb_refine_info(const pb_problem* pb, pb_refine_stats* out);
/* Refinement flags of the coarse cells: host uint8[(n0-1)*(n1-1)*(n2-1)], cell (i,j,k) at
 * ((i*(n1-1) + j)*(n2-1) + k).  PB_EINVAL for a uniform problem. */
int pb_copy_refined_cells(const pb_problem* pb, uint8_t* host);
/* Potential (kT/e) on the fine sub-lattice after pb_solve, host doubles over fine_n in the
 * order ((a*fine_n[1] + b)*fine_n[2] + c); nodes of no fine cell hold 0.  pb_copy_potential
 * returns the coarse grid.  PB_EINVAL for a uniform problem. */
int pb_copy_fine_potential(const pb_problem* pb, double* host_phi);

/* --- inspection (used by the parity tests) ------------------------------------- */

/* Coefficient maps on the full grid (host arrays of n[0]*n[1]*n[2] entries, any may be
 * NULL): solute flag; edge coefficients K = h*eps_e of the edges to (i+1,j,k),
 * (i,j+1,k), (i,j,k+1) (0 where the edge leaves the grid); the operator diagonal
 * (0 on box nodes); the right-hand side including the boundary lift (0 on box nodes). */
int pb_copy_coeffs(const pb_problem* pb, uint8_t* solute, double* kx, double* ky, double* kz,
                   double* diag, double* rhs);

/* Number of cut edges of a built problem (or a negative error code).  For a refined problem:
 * those of its fine sub-lattice, where the surface and the energy read-back are. */
int64_t pb_num_cut(const pb_problem* pb);

/* Cut-edge list in ascending key order, key = 3*((i*n1 + j)*n2 + k) + axis of the edge's
 * low end (i,j,k).  Host arrays of m = pb_num_cut entries (rp, np: 3*m), any may be NULL.
 * F (flux K_e (phi_s - phi_w)) and phip (eq. phi0) are valid after pb_energy.  For a refined
 * problem the list of the fine sub-lattice (i, j, k and n on the sub-lattice, whose node 0
 * is fine-lattice node fine_offset of pb_refine_info). */
int pb_copy_cut(const pb_problem* pb, int64_t* key, double* alpha, double* rp, double* np,
                int64_t* owner, double* wp, double* F, double* phip);

/* Average duration in milliseconds of `reps` back-to-back launches of the fused stencil
 * kernel of the problem's CG (one launch = one operator application plus the
 * search-direction update and the p.Ap partial sums), FP64 or FP32 (fp32 != 0), timed with
 * HIP events on the problem's stream.  It overwrites the solver state: call pb_solve again
 * before pb_energy. */
int pb_time_stencil(pb_problem* pb, int32_t reps, int32_t fp32, double* avg_ms);

/* Turn on (1) or off (0) sampled HIP-event timing of the CG kernels: every 8th iteration's
 * stencil and update launches are bracketed by events on the context stream. */
int pb_ctx_set_profiling(pb_ctx* ctx, int on);

/* Average durations (ms) of the sampled stencil and update launches of the last pb_solve
 * (only iterations that did work are counted), and the number of samples.  For a
 * PB_PRECOND_MG solve with more than one level: the first level-0 black half-sweep after the
 * coarse correction, and the whole V-cycle. */
int pb_get_profile(const pb_problem* pb, double* stencil_ms_avg, double* update_ms_avg, int32_t* samples);

/* With profiling on in the problem's context: HIP-event time (ms) of the energy N-body
 * kernel (atoms x cut points, FP64; a12) of the last pb_energy, and its number of pairs
 * (n_atoms * n_cut); both 0 when it was not timed. */
int pb_get_energy_profile(const pb_problem* pb, double* nbody_ms, double* pairs);

/* Attainable-bandwidth reference: `reps` launches of a plain streaming copy of `bytes`
 * bytes between two buffers from the context allocator, timed with HIP events; *gbps is
 * (bytes read + bytes written) per second / 1e9. */
int pb_stream_copy(pb_ctx* ctx, size_t bytes, int32_t reps, double* gbps);

/* Bytes of device memory held by a problem. */
size_t pb_problem_bytes(const pb_problem* pb);

/* --- serving: continuous batching of many solves ----------------------------------- */

/* A serving loop for a stream of requests in the mixed form (the paper treats one molecule
 * at a time; solving many molecules, e.g. for binding free energies over complexes and
 * their parts, Sect. 6.2 (binding energy calculation), is the workload this serves).
 * Iteration kernels run on ctx's stream, coefficient builds and energy read-backs on
 * build_ctx's stream (same device).
 * Requests are admitted first-come first-served once arrived, while at most max_resident
 * problems are resident and ctx's hbm_budget_bytes (if non-zero) is not exceeded; all
 * resident problems advance together, 16 CG iterations per batched chunk.  Requests with
 * precond = PB_PRECOND_MG share batched multigrid launches (groups of up to
 * 64 requests of one precision and smoothing count; one whose coarsest level is
 * large runs its own launches), with chunks sized from each request's residual decay.  A
 * result equals that of a solve of the same request alone, bit for bit.
 * Errors: PB_EINVAL, PB_EDEVICE. */
int pb_server_create(pb_ctx* ctx, pb_ctx* build_ctx, int32_t max_resident, pb_server** out);

/* Seconds since the server was created (the clock of arrival and completion times). */
double pb_server_now(const pb_server* srv);

/* Queue a request (copied; params->precision must be PB_MIXED, refine 0).  It becomes eligible for
 * admission once pb_server_now() >= arrival_time_s.  A request whose estimated memory
 * exceeds the whole budget completes with code PB_ENOMEM. */
int pb_submit(pb_server* srv, const pb_params* params, int64_t n_atoms, const double* xyz,
              const double* radius, const double* charge, uint64_t request_id,
              double arrival_time_s);

/* One scheduling step: retire finished problems (energy read-back), admit arrived requests,
 * launch one chunk for all resident problems, and wait for the older of the two chunks kept
 * in flight.  Returns the resident and queued counts. */
int pb_server_step(pb_server* srv, int32_t* n_active, int32_t* n_queued);

/* Move up to max finished requests out of the server: ids, energies, solve statistics,
 * completion times (server clock) and result codes (PB_OK, PB_ENOCONV, PB_EBREAKDOWN,
 * PB_ENOMEM, PB_ECANCELED, PB_ETIMEDOUT, ...).  Any output array may be NULL. */
int pb_poll(pb_server* srv, uint64_t* ids, pb_energy_out* results, pb_solve_stats* stats,
            double* done_time_s, int32_t* codes, int32_t max, int32_t* n_done);

/* Cancel a queued or running request: it completes with code PB_ECANCELED (reported by
 * pb_poll) and no energies.  A running problem stops iterating at once and its device memory
 * is released when no launch in flight still uses it.  Errors: PB_EINVAL (NULL server, or the
 * request is not queued or running: unknown, already finished or already cancelled). */
int pb_cancel(pb_server* srv, uint64_t request_id);

/* Time limit per request, in seconds from its arrival time (0, the default: none).  A request
 * not finished within it completes with code PB_ETIMEDOUT and no energies, as if cancelled;
 * the limit is checked at every pb_server_step.  Errors: PB_EINVAL (negative or non-finite). */
int pb_server_set_timeout(pb_server* srv, double seconds);

/* Device-memory accounting of the serving loop against ctx's hbm_budget_bytes.  A request
 * holds an estimate from its atoms while it is queued for a build, an upper bound from its
 * counted cut edges while the build allocates, and then exactly the bytes its problem holds
 * plus those its energy read-back will allocate, until it completes.  in_use: the current
 * sum; peak: its largest value so far; over_budget: builds let past the budget because
 * nothing else running could free memory (a request that alone exceeds the budget fails with
 * PB_ENOMEM instead).  Any output may be NULL. */
int pb_server_memory(const pb_server* srv, size_t* in_use, size_t* peak, int64_t* over_budget);

/* Host seconds spent so far in the four phases of pb_server_step: waiting for chunks,
 * retiring (energy read-back), admitting (coefficient builds), launching. */
int pb_server_times(const pb_server* srv, double* out4);

/* With profiling on in ctx (pb_ctx_set_profiling): total HIP-event time (ms) of the batched
 * stencil launches, their algorithmic bytes (36 per interior unknown per CG iteration actually
 * performed), and the number of launches timed. */
int pb_server_profile(const pb_server* srv, double* stencil_ms_total, double* stencil_bytes_total,
                      int64_t* stencil_launches);

/* The same for the multigrid requests: for every iteration of the batched multigrid chunks
 * (and the first iteration of every chunk of a request run alone) in which at least one
 * request iterated, the HIP-event time (ms) of the level-0 black half-sweep after the coarse
 * correction and its algorithmic bytes (10 per interior unknown of the requests that
 * iterated: in the red-black layout x of the other colour, b, 1/D and the node codes of the
 * swept colour read, x of the swept colour written), the time of the whole
 * V-cycle, and the number of samples. */
int pb_server_profile_mg(const pb_server* srv, double* sweep_ms_total, double* sweep_bytes_total,
                         double* vcycle_ms_total, int64_t* samples);

/* The batched operator pass of the multigrid CG (q = A p with the new direction), timed the
 * same way: HIP-event time (ms), algorithmic bytes (20 per interior unknown of the requests
 * that iterated: z, the old direction and the node codes read, the new direction and q
 * written), and the number of launches timed. */
int pb_server_profile_mg_apply(const pb_server* srv, double* ms_total, double* bytes_total, int64_t* launches);

/* With profiling on in build_ctx: the HIP-event time (ms) of the energy N-body kernel summed
 * over every request read back, the pairs (n_atoms * n_cut) summed likewise, and the number
 * of such read-backs. */
int pb_server_profile_energy(const pb_server* srv, double* nbody_ms_total, double* pairs_total, int64_t* calls);

/* Wait for the device, release every resident problem and the server. */
void pb_server_destroy(pb_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* PB_H */
