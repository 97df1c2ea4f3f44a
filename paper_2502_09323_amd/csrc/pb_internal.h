// pb_internal.h -- device data layout and kernel launchers of libpb (gfx950).
//
// Node arrays live in a padded z-contiguous layout: node (i,j,k) is element
// ((i*ny + j)*S + k + Z0) with Z0 = 31 and S a multiple of 32, so that the first interior
// node of every z-row (k = 1) starts a 128-byte line for FP32 and FP64 data, and so does
// every 32-node tile row after it.  Padding elements are treated as Dirichlet nodes with
// value 0.
//
// Per node the solver keeps one 32-bit code instead of three edge coefficients:
//   bit 0      solute (node strictly inside an atom ball)
//   bit 1      box or padding node (Dirichlet)
//   bits 2..4  the edge to (i+1,j,k), (i,j+1,k), (i,j,k+1) crosses the molecular surface
//   bits 5..31 slot of the node in the compact cut-edge tables (valid if any of bits 2..4)
// An edge inside one medium has K = h*eps_in or h*eps_out; a cut edge reads its WHA value
// from ck[3*slot + axis].
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "pb.h"

namespace pbk {

constexpr uint32_t C_SOLUTE = 1u;
constexpr uint32_t C_BOX = 2u;
constexpr uint32_t C_CUTX = 4u;
constexpr int C_SLOT_SHIFT = 5;
constexpr int Z0 = 31;
constexpr int ZALIGN = 32;

// z-row stride of a grid with nz nodes along z
inline int64_t row_stride(int64_t nz) { return (nz + Z0 + ZALIGN - 1) / ZALIGN * ZALIGN; }

struct Grid {
    int nx, ny, nz;   // nodes per axis
    int S;            // z-row stride in elements
    int64_t N;        // storage elements nx*ny*S
    double h, ox, oy, oz;
    int off[3] = {0, 0, 0};   // node (i,j,k) sits at origin + h*(i + off[0], ...): a sub-lattice
                              // of a lattice with the same origin and spacing
    __host__ __device__ int64_t idx(int i, int j, int k) const
    {
        return ((int64_t)i * ny + j) * S + k + Z0;
    }
};

struct Bins {          // atom cell list: bins of edge bs covering the atom centres
    double lox, loy, loz, bs;
    int nbx, nby, nbz;
    const int* start;  // nbins + 1
    const int* ids;    // atom ids, ascending within each bin
};

// 1/sqrt(x) in FP64 for normal x: the hardware FP64 reciprocal square root estimate y
// (relative error d up to about 5e-8) refined by one step of the series (1 - e)^(-1/2) =
// 1 + e/2 + 3e^2/8 + ..., e = 1 - x y^2 = 2d + O(d^2): the first omitted term, 5e^3/16, is
// below FP64 rounding.  Five FP64 operations in place of a square root and a division.
__device__ __forceinline__ double rsqrt_fp64(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x, y * y, 1.0);
    return fma(y, e * fma(e, 0.375, 0.5), y);
}

struct Atoms {
    int n;
    const double* xyzr;  // 4 per atom: x, y, z, radius
    const double* q;
    // a point near the molecule (the centre of the atoms' bounding box): kernels that form a
    // squared distance in the expanded form |p|^2 + |a|^2 - 2 a.p take p and a relative to
    // it, so that its rounding error does not grow with the distance of the molecule from
    // the coordinate origin
    double cx = 0.0, cy = 0.0, cz = 0.0;
};

struct Coef {          // what the operator needs on the device
    double kin, kout, mass;  // h*eps_in, h*eps_out, h^3*eps_out*kD^2
};

// deterministic CG state, one per solve; written by single designated threads only (the
// one-block tail and reliable-update kernels), read by every block of the iteration kernel
struct CGState {
    double alpha;      // step the next iteration applies: x += alpha p_old, r -= alpha q_old
    double beta;       // p_new = D^-1 r_new + beta p_old
    double gamma;      // r.D^-1 r of the last iterate
    double bnorm2;     // ||b||^2 of the iterated system
    double rr;         // ||r||^2 of the last iterate (recursive residual)
    double pq;         // p.A p of the last iteration
    double stop2;      // the tail stops the iteration when rr <= stop2 ...
    double trig2;      // mixed: a reliable update runs once rr <= trig2 (Jacobi CG: at the
                       // chunk's end; multigrid: in the next iteration)
    double delta2;     // mixed: after an update trig2 = delta2 * ||r||^2
    double goal64;     // mixed: converged when the FP64 true ||b - A x||^2 <= goal64
    double rr64;       // mixed: FP64 true residual norm^2 at the last update
    int status;        // 0 running, 1 converged, 2 breakdown, 3 true-residual check requested
    int stop_status;   // ... and sets status = stop_status (1 for FP64, 3 for mixed)
    int iters;         // CG steps applied to x when the iteration stopped
    int iter_count;    // completed iteration kernels; its parity selects the buffers
    int ru;            // 1 while a reliable update is in progress
    int n_ru;          // reliable updates done
};

struct TileShape {     // tiling of the interior for the stencil kernel
    int LX;            // planes per x-chunk
    int nxc, njt, nkt; // chunks / tiles along x, y, z
    int items;         // nxc*njt*nkt
};

#ifndef PB_TILE_WAVES
#define PB_TILE_WAVES 4
#endif
constexpr int ZW = 32;              // z-extent of a tile of the iteration kernel (lanes per row)
constexpr int NWV = PB_TILE_WAVES;  // waves per block of the iteration kernel, two rows each
constexpr int TY = 2 * NWV;         // y-extent of a tile
static_assert(NWV >= 2 && TY <= 32, "tile shape");

// ---- build kernels (pb_build.hip) -----------------------------------------------------
// the cell list, and in xyzr_b (4 n doubles) the atoms' centres and radii in its order
hipError_t launch_bins(hipStream_t s, const Atoms& at, Bins& b, int* cnt, int* start, int* ids,
                       int* cursor, double* xyzr_b);
hipError_t launch_classify(hipStream_t s, const Grid& g, const Bins& b, const double* xyzr_b, uint32_t* code);
hipError_t launch_cutflags(hipStream_t s, const Grid& g, uint32_t* cls, int* blk_slots,
                           int* blk_cuts, int nblk);
hipError_t launch_scan2(hipStream_t s, int* a, int* b, int n, int* totals);
// exclusive scan of n ints into out[0 .. n] (out[n] = total; out may be in), one block
hipError_t launch_scan1(hipStream_t s, const int* in, int n, int* out);
hipError_t launch_assign(hipStream_t s, const Grid& g, const uint32_t* cls, uint32_t* code,
                         const int* blk_slots, const int* blk_cuts, int* cutbase, int64_t* cutkey);
hipError_t launch_cut_geom(hipStream_t s, const Grid& g, const Bins& b, const double* xyzr_b, const Atoms& at,
                           double eps_in, double eps_out, int64_t ncut, const int64_t* cutkey,
                           const uint32_t* code, double* alpha, double* kcut, double* rp,
                           double* np, int* owner, double* ck64, float* ck32);
// ac: scratch of 8 doubles per atom (in cell-list order: the atom's cell, offsets and charge)
hipError_t launch_deposit(hipStream_t s, const Grid& g, const Bins& b, const Atoms& at, double* ac, double* rhs);
// grid energy: part[nb] = scale * sum_a q_a sum_corners w x over interior nodes, with
// nb = grid_energy_blocks(at.n) and part holding nb + 1 doubles
int grid_energy_blocks(int n_atoms);
hipError_t launch_grid_energy(hipStream_t s, const Grid& g, const Atoms& at, const double* x, double scale,
                              double* part);
// Debye-Hueckel box values: the atoms are split into ranges of whole 256-atom chunks (as many
// ranges as kDhTargetBlocks blocks of kDhNodesPerBlock box nodes would ask for, at most
// kDhMaxRanges), each block sums one range for its patches of box-face nodes into
// part[range][node], and a second kernel adds the ranges in order
constexpr int kDhNodesPerBlock = 512;
constexpr int kDhMaxRanges = 16;
constexpr int64_t kDhTargetBlocks = 32768;
struct DhSplit {
    int64_t nbox;   // box nodes
    int tiles;      // box nodes / kDhNodesPerBlock (sizes the ranges)
    int per;        // atoms per range (a multiple of 256)
    int ranges;     // atom ranges (at most kDhMaxRanges)
};
DhSplit dh_split(const Grid& g, int n_atoms);
// constants of the table-driven exp(-kD r) of the FP64 Debye-Hueckel sum
constexpr int kDhTable = 2048;   // T[j] = 2^(j / kDhTable)
struct DhExp {
    double tscale;      // -kD kDhTable / ln 2
    double L;           // ln 2 / (kDhTable kD)
    double c1, c2, c3;  // Taylor coefficients of e^(-kD s): -kD, kD^2 / 2, -kD^3 / 6 (all 0 for kD = 0)
};
DhExp dh_exp_consts(double kD);
struct DhFaces {        // the six box faces as row-major U x V arrays of box nodes (FP64 sum)
    int64_t base[6];    // box-node index of each face's first node
    int U[6], V[6];
    int pv[6];          // thread patches per face row (along v)
    int64_t np[6];      // thread patches per face
    int tile0[7];       // first block of each face; tile0[6] = all blocks
};
DhFaces dh_faces(const Grid& g);
// part holds dh_split(g, at.n).ranges * nbox doubles
hipError_t launch_bc_dh(hipStream_t s, const Grid& g, const Atoms& at, double kD, double eps_out, double* part,
                        double* gb);
hipError_t launch_bc_dh32(hipStream_t s, const Grid& g, const Atoms& at, double kD, double eps_out, double* part,
                          double* gb);
hipError_t launch_bc_user(hipStream_t s, const Grid& g, const double* full, double* gb);
hipError_t launch_diag_lift(hipStream_t s, const Grid& g, const uint32_t* code, const double* ck64,
                            Coef c, const double* gb, double* rhs, float* dinv, double* diag);
hipError_t launch_mc_weights(hipStream_t s, const Grid& g, const uint32_t* code, const int* cutbase,
                             int64_t ncut, const int64_t* cutkey, const double* rp, double* wp);
hipError_t launch_fill(hipStream_t s, void* p, size_t bytes);
hipError_t launch_export_coeffs(hipStream_t s, const Grid& g, const uint32_t* code, const double* ck64, Coef c,
                                const double* rhs, uint8_t* sol, double* kx, double* ky, double* kz,
                                double* diag, double* b);
hipError_t launch_export_phi(hipStream_t s, const Grid& g, const double* x, const double* gb, double lB,
                             double* out);

// ---- solver kernels (pb_solve.hip) ------------------------------------------------------
TileShape make_tiles(const Grid& g, int planes);   // planes = 0: chosen from the grid

template <typename T>
struct CGBufs {
    T* x;
    T* z[2];           // D^-1 r; z, w and p are double buffered by iteration parity
    T* w[2];           // D^-1 q
    T* p[2];
    const T* ck;
    const uint32_t* code;
    double* part;      // [5*nb] per-block partial sums of the iteration kernel
    CGState* st;
    int nb;            // blocks of the iteration kernel (= tiles)
};

template <typename T>
hipError_t launch_cg_init(hipStream_t s, const Grid& g, const CGBufs<T>& B, Coef c, const double* b64, const T* bT);
hipError_t launch_cg_fin(hipStream_t s, const double* part, int nb, CGState* st, double rtol2);
template <typename T>
hipError_t launch_cg_iter(hipStream_t s, const Grid& g, const TileShape& ts, const CGBufs<T>& B, Coef c);
hipError_t launch_cg_tail(hipStream_t s, const double* part, int nb, CGState* st);
hipError_t launch_stream_copy(hipStream_t s, const void* a, void* b, size_t bytes);

// everything a batched launch needs to act for one problem
template <typename T>
struct ProbDev {
    Grid g;
    TileShape ts;
    Coef cf;
    CGBufs<T> B;          // FP32 CG state (x = FP32 correction, z = FP32 preconditioned residual)
    double* x64;          // FP64 solution
    const double* rhs;    // FP64 right-hand side
    const double* ck64;   // FP64 cut-edge coefficients
    double* part3;        // reliable-update partial sums [3][nbres]
    int nbres, nadd;      // block counts of the reliable-update kernels
};

struct BatchTotals {     // grid sizes of the batched launches (sums over the problems)
    int st, add, res;
};

// ev (optional): 2*iters events recorded around every batched iteration kernel
hipError_t launch_batch_chunk(hipStream_t s, const ProbDev<float>* D, const int* off, int P, const BatchTotals& t,
                              int iters, CGState* gather_out, hipEvent_t* ev);
int add_blocks(const Grid& g);

// mixed precision: FP32 CG with FP64 reliable updates (true residual + solution accumulation)
hipError_t launch_ru_begin(hipStream_t s, CGState* st);
hipError_t launch_ru_add(hipStream_t s, const Grid& g, CGState* st, double* x64, float* d32, float* const* p32,
                         int force);
hipError_t launch_ru_residual(hipStream_t s, const Grid& g, const uint32_t* code, const double* ck64, const float* ck32,
                              Coef c, const double* b, const double* x64, float* const* z32, double* part3, CGState* st);
hipError_t launch_ru_fin(hipStream_t s, CGState* st, const double* part3, int nbres, int init, double rtol2,
                         double delta2);
int residual_blocks(const Grid& g);

// ---- energy kernels (pb_energy.hip) -------------------------------------------------------
// a cut point as the N-body kernel reads it: r_p (3), the weighted normal u = w_p phi_p n_p
// (3), F_p, |r_p|^2, 2 r_p.u, and one pad
constexpr int CUT_POINT_DOUBLES = 10;
// the cut points are stored relative to the atoms' centre (at.cx, at.cy, at.cz)
hipError_t launch_edge_fields(hipStream_t s, const Grid& g, const Atoms& at, double eps_in, double eps_out,
                              int64_t ncut, const int64_t* cutkey, const uint32_t* code,
                              const double* alpha, const double* kcut, const double* x,
                              const double* gb, const double* wp, double* F, double* phip,
                              double* pts /* CUT_POINT_DOUBLES per cut point */, const double* rp,
                              const double* np);
hipError_t launch_nbody(hipStream_t s, const Atoms& at, int64_t ncut, const double* pts,
                        double* partial, int nchunk);
// phic: n_atoms * ncc partial Coulomb potentials, ncc = coulomb_chunks(n_atoms)
hipError_t launch_coulomb(hipStream_t s, const Atoms& at, double* phic, int ncc);
// out: ENERGY_OUT_DOUBLES (the five results, then per-block partial sums)
constexpr int ENERGY_OUT_DOUBLES = 16 + 5 * 256;
// the N-body partials: nchunk chunks, then room for their sums in groups (the reduction folds
// many chunks first); energy_partial_doubles gives the buffer's size
int64_t energy_partial_doubles(int n_atoms, int nchunk);
hipError_t launch_energy_reduce(hipStream_t s, const Atoms& at, double* partial, int nchunk,
                                const double* phic, int ncc, double eps_in, double eps_out, double lB,
                                double* phi_reac, double* out, const double* F, int64_t ncut,
                                const double* wp);
int nbody_chunks(int n_atoms, int64_t ncut);
int coulomb_chunks(int n_atoms);

}  // namespace pbk
