// pb_mg.hip -- CG preconditioned by one geometric-multigrid V-cycle (uniform grids).
//
// The paper solves with CG and an SSOR preconditioner (Sect. 4).  On a GPU a lexicographic
// SSOR sweep is sequential, so this solver orders the nodes red-black (node (i,j,k) is red
// when i+j+k is even; all neighbours of a red node are black) and uses symmetric red-black
// Gauss-Seidel -- SSOR with omega = 1 in that order -- as the smoother of a V-cycle:
//
//   levels      node I of level l+1 is node 2I of level l, while n-1 is even on every axis
//               (n >= 5); level 0 reads the operator from the node codes, the coarser
//               levels store K along +x, +y, +z and 1/diagonal per node
//   coarse K    along a coarse edge the two fine edges are in series (K1 K2 / (K1 + K2));
//               across it the 3 x 3 fine lines around it are averaged with weights
//               (1/4, 1/2, 1/4) per axis, times 4 (a coarse dual face holds four fine ones);
//               the coarse ionic term is P^T m
//   transfers   P trilinear, R = P^T
//   V-cycle     zero start; nu times (red, black); residual (zero on black nodes right after
//               a black half-sweep, so only red nodes are formed); restrict; recurse; add P e
//               (at the red nodes: the black half-sweep that follows replaces the black ones);
//               nu times (black, red); the coarsest level takes red, then (black, red) x cs.
//               Levels of at most 8192 unknowns run in one block (one launch).
//               Pre- and post-smoothing are adjoint and R = P^T: the V-cycle is symmetric
//               positive definite.  With one level it is red-black symmetric Gauss-Seidel.
//   CG          standard PCG (z = V-cycle(r)) with device-resident scalars; FP64, or FP32
//               with FP64 reliable updates (x64 += x32, r = b - A x64 in FP64, restart the
//               recurrence from the true residual, keeping the direction)
//
// Level 0 and the CG vectors use a red-black layout (each colour of a z-row in its own
// segment), the coarser levels the padded natural layout.  Every kernel is a batched launch:
// a table of block offsets maps each block to one problem of a set (its hierarchy described
// by a device-resident MGDev) and to a block of that problem's own launch, so one launch per
// pass serves every problem of the serving loop's multigrid requests, and a solo solve is a
// set of one.  A problem's blocks do the same work in the same order whatever the set, so a
// result does not depend on what it was batched with.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include "pb_host.h"
#include "pb_internal.h"
#include "pb_stencil.h"

using namespace pbk;

namespace {

#define RCHK(x)                                                                     \
    do {                                                                            \
        hipError_t e_ = (x);                                                        \
        if (e_ != hipSuccess) return pbi_fail(PB_EDEVICE, "%s", hipGetErrorString(e_)); \
    } while (0)

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// Every pointer that the kernels take from a hierarchy descriptor or a launch table points to
// global memory.  Typed so in the device pass, the loads through it are global loads, and a
// descriptor's fields are read with scalar loads, instead of flat loads whose addresses are
// formed per lane.  The host pass sees plain pointers (same size and layout): the host only
// writes the descriptors.
#if defined(__HIP_DEVICE_COMPILE__)
#define GMEM __attribute__((address_space(1)))
#else
#define GMEM
#endif
template <typename T>
__host__ __device__ inline GMEM T* gmem(T* p)
{
    return (GMEM T*)p;
}

// one coarse level as the kernels see it
template <typename T>
struct Lev {
    Grid g;
    const GMEM T *kx, *ky, *kz;   // K of the +x, +y, +z edges
    const GMEM T* diag;           // diagonal
    const GMEM T* dinv;           // 1 / diagonal
    GMEM T* x;                    // iterate
    const GMEM T* b;              // right-hand side
};

// the level-0 operator from the natural-layout node codes
template <typename T>
struct Op0 {
    const GMEM uint32_t* code;
    const GMEM T* ck;
    T kin, kout, mass;
};

// ---- level 0 in the red-black layout ----------------------------------------------------
// The vectors of level 0 (the CG vectors, the level's iterate, right-hand side, red residual
// and 1/D) and a copy of the node codes keep the two colours apart: row (i, j) holds its red
// nodes in one segment of Sh positions and its black nodes in the next, node k at position
// k >> 1.  A half-sweep then moves only lines of the colour it updates and of the other
// colour it reads, instead of whole lines of both.  Box and padding positions hold 0 in every
// vector (their codes carry C_BOX), so neighbour loads need no branch.  The neighbours of a
// node are all of the other colour: along x and y at the same position of the adjacent rows,
// along z at positions (k - 1) >> 1 and (k + 1) >> 1 of its own row.

struct RB {
    int nx, ny, nz;
    int Sh;        // positions per colour segment (a multiple of 32: 128-byte aligned segments)
    int64_t N;     // elements per vector: nx * ny * 2 * Sh
    int lw;        // a wave of a level-0 pass covers 2^lw positions of 64 >> lw rows
    __host__ __device__ int64_t at(int i, int j, int c, int m) const
    {
        return (((int64_t)i * ny + j) * 2 + c) * Sh + m;
    }
    __host__ __device__ int64_t idx(int i, int j, int k) const { return at(i, j, (i + j + k) & 1, k >> 1); }
};

inline RB rb_of(const Grid& g)
{
    RB r;
    r.nx = g.nx;
    r.ny = g.ny;
    r.nz = g.nz;
    r.Sh = ((g.nz + 1) / 2 + 31) / 32 * 32;
    r.N = (int64_t)g.nx * g.ny * 2 * r.Sh;
    // the interior positions of a row segment, (nz - 2) / 2 + 1, in as few idle lanes as
    // possible: 64, 32 or 16 positions per wave row (the widest of the least waste)
    const int P = (g.nz - 2) / 2 + 1;
    int best = 1 << 30;
    r.lw = 6;
    for (int lw = 6; lw >= 4; --lw) {
        const int w = 1 << lw, waste = (P + w - 1) / w * w - P;
        if (waste < best) {
            best = waste;
            r.lw = lw;
        }
    }
    return r;
}

template <typename T>
struct OpRB {
    const GMEM uint32_t* code;   // red-black layout
    const GMEM T* ck;
    T kin, kout, mass;
};

// one problem's hierarchy, solver vectors and state, as every kernel reads it (written once
// into device memory when the hierarchy is built)
template <typename T>
struct MGDev {
    RB rb;
    Grid g0;                     // level 0 in the natural layout (solution, right-hand side)
    OpRB<T> op;
    Op0<double> op64;            // FP64 operator from the natural codes (true residual)
    GMEM T *cr, *cz, *cp, *cp2, *cq, *cx, *dinv0, *r0;   // level 0: CG r, z, p (two), q, correction x; 1/D;
                                                        // red residual
    GMEM double* x64;            // FP64 solution (natural layout)
    const GMEM double* rhs;      // FP64 right-hand side (natural layout)
    int nlev, ls, nu, cs;        // levels, first level of the one-block part (ls == nlev: none)
    Lev<T> lv[PB_MG_MAX_LEVELS]; // levels >= 1
    GMEM T* r[PB_MG_MAX_LEVELS]; // red residual of levels >= 1
    GMEM CGState* st;
    GMEM double* part;           // [3 * nb] block partial sums
    GMEM double* prz;            // [nb] r.z partial sums of the last half-sweep
    int nb;                      // blocks of a level-0 pass
    int mixed;
    double rtol2, delta2;
};

// A batched launch: the problems, and the offsets of their blocks in this pass (P + 1; a
// problem may have none).
template <typename T>
struct Bt {
    const GMEM MGDev<T>* const GMEM* d;
    const GMEM int* off;
    int P;
};

// the problem of this block and the block's index in that problem's own launch
__device__ __forceinline__ int bt_find(const GMEM int* off, int P, int& local)
{
    const int b = (int)blockIdx.x;
    int lo = 0, hi = P;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= b)
            lo = mid;
        else
            hi = mid;
    }
    local = b - off[lo];
    return lo;
}

// which kernels run: those of a CG iteration (ru = 0) while the solve is running, those of a
// restart from the true residual (ru = 1) only while one is in progress; ungated (a V-cycle
// on its own); or gated on another state (the two-level preconditioner of refined grids)
struct GateSpec {
    const GMEM CGState* ext;
    int mode;   // 0 iteration, 1 restart, 2 none, 3 ext (running, ru 0; null: none), 4 running
};

__device__ __forceinline__ bool gated_out(const GateSpec& g, const GMEM CGState* st)
{
    if (g.mode == 2) return false;
    if (g.mode == 3) return g.ext && (g.ext->status != 0 || g.ext->ru != 0);
    if (g.mode == 4) return st->status != 0;
    return st->status != 0 || st->ru != g.mode;
}

// The block shape of the per-node passes: 64 lanes along z by 4 rows along y, each thread
// taking kPlanes x-planes, so that no thread divides to find its node and a launch has few
// enough blocks that one which finds the iteration stopped costs little.
constexpr int kPlanes = 4;
// level 0 (red-black layout): more x-planes per thread, so that fewer neighbour planes are
// read again at the edges of a block's slab
#ifndef PB_PLANES_RB
#define PB_PLANES_RB 8
#endif
constexpr int kPlanesRB = PB_PLANES_RB;

struct VB {   // a block of a problem's own 3-D launch
    int x, y, z;
};

__device__ __forceinline__ VB vb_of(int local, int gx, int gy)
{
    VB v;
    v.x = local % gx;
    const int t = local / gx;
    v.y = t % gy;
    v.z = t / gy;
    return v;
}

// tiles of 2^lw positions along a row: the interior nodes k = 1 ... nz - 2 sit at positions
// 0 ... (nz - 2) / 2 of their colour's segment; a block (4 waves) covers 4 * (64 >> lw) rows
__host__ __device__ inline int rb_gx(const RB& r) { return ((r.nz - 2) / 2 + 1 + (1 << r.lw) - 1) >> r.lw; }
__host__ __device__ inline int rb_rows(const RB& r) { return 4 * (64 >> r.lw); }
__host__ __device__ inline int rb_gy(const RB& r) { return (r.ny - 2 + rb_rows(r) - 1) / rb_rows(r); }
__host__ __device__ inline int rows_gy(int ny) { return (ny - 2 + 3) / 4; }

inline int rb_blocks(const RB& r) { return rb_gx(r) * rb_gy(r) * ((r.nx - 2 + kPlanesRB - 1) / kPlanesRB); }

// block `local` of a level-0 pass of nb blocks takes tile item(local): blocks are dealt to the
// 8 XCDs round-robin (a problem's blocks start at a multiple of 8), and this bijection gives
// each XCD one contiguous range of tiles (x fastest, then rows, then plane slabs), so that the
// neighbour rows and planes a tile reads were mostly brought into that XCD's L2 by the tiles
// just before it
__device__ __forceinline__ VB vb_rb(const RB& r, int local, int nb)
{
    const int q8 = nb >> 3, rem = nb & 7, xcd = local & 7;
    const int item = xcd * q8 + (xcd < rem ? xcd : rem) + (local >> 3);
    return vb_of(item, rb_gx(r), rb_gy(r));
}

// blocks along z of a coarse-level pass over all interior nodes or over the nodes of one colour
__host__ __device__ inline int lev_gx(const Grid& g, bool colour)
{
    const int nzl = colour ? (g.nz - 1) / 2 : g.nz - 2;
    return nzl > 0 ? (nzl + 63) / 64 : 1;
}

inline int lev_blocks(const Grid& g, bool colour)
{
    return lev_gx(g, colour) * rows_gy(g.ny) * ((g.nx - 2 + kPlanes - 1) / kPlanes);
}

__device__ __forceinline__ VB vb_lev(const Grid& g, bool colour, int local)
{
    return vb_of(local, lev_gx(g, colour), rows_gy(g.ny));
}

// red-black: this thread's row and position in plane p of its block; false outside the rows
__device__ __forceinline__ bool rb_slot(const VB& b, const RB& r, int p, int& i, int& j, int& m)
{
    const int lane = (int)(threadIdx.x & 63), w = 1 << r.lw;
    m = b.x * w + (lane & (w - 1));
    j = 1 + b.y * rb_rows(r) + (int)(threadIdx.x >> 6) * (64 >> r.lw) + (lane >> r.lw);
    i = 1 + b.z * kPlanesRB + p;
    return i <= r.nx - 2 && j <= r.ny - 2;
}

// z index of the node of colour c at position m of row (i, j), or -1 if it is not interior
__device__ __forceinline__ int rb_node(const RB& r, int i, int j, int c, int m)
{
    const int k = 2 * m + ((i + j + c) & 1);
    return (k >= 1 && k <= r.nz - 2) ? k : -1;
}

// A block's frame: a level-0 kernel addresses the vectors from the first element of plane
// i0 - 1 (i0 the block's first plane).  Every lane offset then fits in 32 bits, and the base of
// each vector is one scalar add per block, so that a load takes a scalar base and a 32-bit lane
// offset instead of a 64-bit address formed per lane.
struct RBFrame {
    int64_t org;   // element index of (i0 - 1, 0, colour 0, position 0)
    int i0;
};

__device__ __forceinline__ RBFrame rb_frame(const RB& r, const VB& vb)
{
    RBFrame f;
    f.i0 = 1 + vb.z * kPlanesRB;
    f.org = (int64_t)(f.i0 - 1) * r.ny * 2 * r.Sh;
    return f;
}

// offset of (i, j, c, m) in a frame (planes i0 - 1 ... i0 + kPlanesRB)
__device__ __forceinline__ uint32_t rb_rel(const RB& r, const RBFrame& f, int i, int j, int c, int m)
{
    return ((uint32_t)((i - f.i0 + 1) * r.ny + j) * 2u + (uint32_t)c) * (uint32_t)r.Sh + (uint32_t)m;
}

// element e of a frame's vector (base = the vector + the frame origin)
template <typename T>
__device__ __forceinline__ T ldf(const GMEM T* base, uint32_t e)
{
    return *(const GMEM T*)((const GMEM char*)base + e * (uint32_t)sizeof(T));
}
// the same as a non-temporal load: for data a pass reads once, so that it does not displace
// the lines of the vectors that neighbouring rows and planes read again
template <typename T>
__device__ __forceinline__ T ldf_nt(const GMEM T* base, uint32_t e)
{
    return __builtin_nontemporal_load((const GMEM T*)((const GMEM char*)base + e * (uint32_t)sizeof(T)));
}
template <typename T>
__device__ __forceinline__ GMEM T& stf(GMEM T* base, uint32_t e)
{
    return *(GMEM T*)((GMEM char*)base + e * (uint32_t)sizeof(T));
}

// frame offsets of a node and of its six neighbours (x-, x+, y-, y+, z-, z+)
struct RBNb {
    uint32_t e, xm, xp, ym, yp, zm, zp;
};

__device__ __forceinline__ RBNb rb_nb(const RB& r, const RBFrame& f, int i, int j, int c, int m, int k)
{
    RBNb n;
    n.e = rb_rel(r, f, i, j, c, m);
    const uint32_t eo = rb_rel(r, f, i, j, 1 - c, m);
    const uint32_t sx = (uint32_t)r.ny * 2u * (uint32_t)r.Sh, sy = 2u * (uint32_t)r.Sh;
    n.xm = eo - sx;
    n.xp = eo + sx;
    n.ym = eo - sy;
    n.yp = eo + sy;
    n.zm = eo - ((k & 1) ? 0u : 1u);
    n.zp = eo + ((k & 1) ? 1u : 0u);
    return n;
}

// In the red-black codes an interior node (whose natural code never carries C_BOX) carries
// C_BOX when none of its six edges is cut.
constexpr uint32_t C_RB_UNCUT = C_BOX;

// the six edge weights and the ionic term of node n whose code c is given (code = the frame's
// code base).  Uncut (every node of the wave carries C_RB_UNCUT): the six weights are the
// node's medium value (an uncut edge joins two nodes of one medium), the very values the
// table path gives, and the neighbours' codes are not read.
template <bool Uncut, typename T>
__device__ __forceinline__ stencil::NodeK<T> rb_k(const OpRB<T>& op, const GMEM uint32_t* code, const RBNb& n,
                                                  uint32_t c)
{
    stencil::NodeK<T> k;
    k.m = (c & C_SOLUTE) ? (T)0 : op.mass;
    if constexpr (Uncut) {
        const T b = (c & C_SOLUTE) ? op.kin : op.kout;
        k.xm = k.xp = k.ym = k.yp = k.zm = k.zp = b;
    } else {
        const T* ck = (const T*)op.ck;   // still a global pointer to the compiler (it follows the cast)
        k.xm = stencil::edgeK(ldf(code, n.xm), 0, ck, op.kin, op.kout);
        k.xp = stencil::edgeK(c, 0, ck, op.kin, op.kout);
        k.ym = stencil::edgeK(ldf(code, n.ym), 1, ck, op.kin, op.kout);
        k.yp = stencil::edgeK(c, 1, ck, op.kin, op.kout);
        k.zm = stencil::edgeK(ldf(code, n.zm), 2, ck, op.kin, op.kout);
        k.zp = stencil::edgeK(c, 2, ck, op.kin, op.kout);
    }
    return k;
}

// A level-0 stencil pass first loads the codes of all its thread's nodes (kPlanesRB x NC,
// NC colours per plane; C_RB_UNCUT where a slot has no node), then takes one of two
// branch-free bodies for the whole wave: the uncut one where every node of the wave carries
// C_RB_UNCUT, else the table one.  With no branch on loaded data inside the body, the loads of
// all planes can be in flight together.  The one-colour passes load these codes
// non-temporal (385^3: 3-5 % less time); the operator pass, which reads neighbours' codes
// too, keeps them cached.
template <int NC>
__device__ __forceinline__ bool rb_codes(const VB& vb, const RB& R, const RBFrame& F, const GMEM uint32_t* code,
                                         int c0, uint32_t (*cc)[NC])
{
    bool uncut = true;
#pragma unroll
    for (int p = 0; p < kPlanesRB; ++p) {
        int i, j, m;
        const bool ok = rb_slot(vb, R, p, i, j, m);
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            const int c = NC == 2 ? q : c0;
            const uint32_t e = rb_rel(R, F, i, j, c, m);
            cc[p][q] = (ok && rb_node(R, i, j, c, m) >= 0) ? (NC == 1 ? ldf_nt(code, e) : ldf(code, e)) : C_RB_UNCUT;
        }
    }
#pragma unroll
    for (int p = 0; p < kPlanesRB; ++p)
#pragma unroll
        for (int q = 0; q < NC; ++q) uncut = uncut && (cc[p][q] & C_RB_UNCUT) != 0;
    return __all(uncut) != 0;
}

// sum over the six edges of K * v(neighbour)
template <typename T, typename F>
__device__ __forceinline__ T rb_sum(const stencil::NodeK<T>& k, const RBNb& n, F v)
{
    return ((k.xm * v(n.xm) + k.xp * v(n.xp)) + (k.ym * v(n.ym) + k.yp * v(n.yp))) + (k.zm * v(n.zm) + k.zp * v(n.zp));
}

// ---- coarse levels (natural layout) ------------------------------------------------------

// sum over the six edges of node e of K * v(neighbour), and optionally the diagonal there
template <typename T, typename F>
__device__ __forceinline__ T nsum(const Lev<T>& L, int64_t e, F v, T* D = nullptr)
{
    const Grid& g = L.g;
    const int64_t sx = (int64_t)g.ny * g.S, sy = g.S;
    if (D) *D = L.diag[e];
    return ((L.kx[e - sx] * v(e - sx) + L.kx[e] * v(e + sx)) + (L.ky[e - sy] * v(e - sy) + L.ky[e] * v(e + sy))) +
           (L.kz[e - 1] * v(e - 1) + L.kz[e] * v(e + 1));
}

// interior node of this thread in plane r of its block (all nodes), or -1; red tells its colour
__device__ __forceinline__ int64_t this_node(const VB& b, const Grid& g, int r, bool& red)
{
    const int k = 1 + b.x * 64 + (int)(threadIdx.x & 63);
    const int j = 1 + b.y * 4 + (int)(threadIdx.x >> 6);
    const int i = 1 + b.z * kPlanes + r;
    if (k > g.nz - 2 || j > g.ny - 2 || i > g.nx - 2) return -1;
    red = ((i + j + k) & 1) == 0;
    return g.idx(i, j, k);
}

// interior node of colour c (0 red, 1 black) of this thread in plane r, or -1; with its indices
__device__ __forceinline__ int64_t this_colour_node(const VB& b, const Grid& g, int c, int r, int& i, int& j, int& k)
{
    const int m = b.x * 64 + (int)(threadIdx.x & 63);
    j = 1 + b.y * 4 + (int)(threadIdx.x >> 6);
    i = 1 + b.z * kPlanes + r;
    k = 1 + ((i + j + 1 + c) & 1) + 2 * m;
    if (k > g.nz - 2 || j > g.ny - 2 || i > g.nx - 2) return -1;
    return g.idx(i, j, k);
}

// node t of colour c in (i, j, m) order (one-block passes)
__device__ __forceinline__ int64_t colour_node(const Grid& g, int c, int t)
{
    const int M = (g.nz - 1) >> 1;
    const int rows = (g.nx - 2) * (g.ny - 2);
    if (M <= 0 || t >= rows * M) return -1;
    const int row = t / M, m = t - row * M;
    const int i = 1 + row / (g.ny - 2), j = 1 + row % (g.ny - 2);
    const int k = 1 + ((i + j + 1 + c) & 1) + 2 * m;
    if (k > g.nz - 2) return -1;
    return g.idx(i, j, k);
}

__device__ __forceinline__ int64_t interior_node(const Grid& g, int t, bool& red)
{
    const int nzi = g.nz - 2, nyi = g.ny - 2;
    const int row = t / nzi;
    const int k = 1 + (t - row * nzi);
    const int i = 1 + row / nyi, j = 1 + row % nyi;
    red = ((i + j + k) & 1) == 0;
    return g.idx(i, j, k);
}

__host__ __device__ inline int64_t colour_threads(const Grid& g)
{
    return (int64_t)(g.nx - 2) * (g.ny - 2) * ((g.nz - 1) >> 1);
}

__host__ __device__ inline int64_t interior_count(const Grid& g)
{
    return (int64_t)(g.nx - 2) * (g.ny - 2) * (g.nz - 2);
}

// P e at fine node (i, j, k): trilinear from the coarse corners of its coarse cell
template <typename T>
__device__ __forceinline__ T prolong_at(const Grid& gc, const GMEM T* __restrict__ ec, int i, int j, int k)
{
    const int i0 = i >> 1, i1 = (i + 1) >> 1, j0 = j >> 1, j1 = (j + 1) >> 1, k0 = k >> 1, k1 = (k + 1) >> 1;
    const T v = ((ec[gc.idx(i0, j0, k0)] + ec[gc.idx(i0, j0, k1)]) + (ec[gc.idx(i0, j1, k0)] + ec[gc.idx(i0, j1, k1)])) +
                ((ec[gc.idx(i1, j0, k0)] + ec[gc.idx(i1, j0, k1)]) + (ec[gc.idx(i1, j1, k0)] + ec[gc.idx(i1, j1, k1)]));
    return (T)0.125 * v;
}

// the level of a coarse-level pass: l, or the problem's coarsest for l < 0
template <typename T>
__device__ __forceinline__ int lev_index(const GMEM MGDev<T>& D, int l)
{
    return l < 0 ? D.nlev - 1 : l;
}

// the first smoothing step of coarse level l from a zero iterate: red x = b / D, then black
// x = (b + sum K x_red) / D with the red values formed on the fly (all interior nodes)
template <typename T>
__global__ void __launch_bounds__(256) kb_down1(Bt<T> B, int l, GateSpec gs)
{
    int local;
    const GMEM MGDev<T>& D = *B.d[bt_find(B.off, B.P, local)];
    if (gated_out(gs, D.st)) return;
    const Lev<T> L = D.lv[lev_index(D, l)];
    const VB vb = vb_lev(L.g, false, local);
    const GMEM T* __restrict__ b = L.b;
    const GMEM T* __restrict__ dinv = L.dinv;
#pragma unroll
    for (int r = 0; r < kPlanes; ++r) {
        bool red;
        const int64_t e = this_node(vb, L.g, r, red);
        if (e < 0) continue;
        if (red) {
            L.x[e] = b[e] * dinv[e];
        } else {
            const T s = nsum<T>(L, e, [&](int64_t n) { return b[n] * dinv[n]; });
            L.x[e] = (b[e] + s) * dinv[e];
        }
    }
}

// Gauss-Seidel on the nodes of colour c of coarse level l
template <typename T>
__global__ void __launch_bounds__(256) kb_sweep(Bt<T> B, int l, int c, GateSpec gs)
{
    int local;
    const GMEM MGDev<T>& D = *B.d[bt_find(B.off, B.P, local)];
    if (gated_out(gs, D.st)) return;
    const Lev<T> L = D.lv[lev_index(D, l)];
    const VB vb = vb_lev(L.g, true, local);
    const GMEM T* __restrict__ x = L.x;
#pragma unroll
    for (int r = 0; r < kPlanes; ++r) {
        int i, j, k;
        const int64_t e = this_colour_node(vb, L.g, c, r, i, j, k);
        if (e < 0) continue;
        const T s = nsum<T>(L, e, [&](int64_t n) { return x[n]; });
        L.x[e] = (L.b[e] + s) * L.dinv[e];
    }
}

// residual b - A x at the red nodes of coarse level l (after a black half-sweep the black
// residual is zero, and the black entries of r stay 0)
template <typename T>
__global__ void __launch_bounds__(256) kb_resid(Bt<T> B, int l, GateSpec gs)
{
    int local;
    const GMEM MGDev<T>& D = *B.d[bt_find(B.off, B.P, local)];
    if (gated_out(gs, D.st)) return;
    const Lev<T> L = D.lv[l];
    GMEM T* __restrict__ r = D.r[l];
    const VB vb = vb_lev(L.g, true, local);
    const GMEM T* __restrict__ x = L.x;
#pragma unroll
    for (int p = 0; p < kPlanes; ++p) {
        int i, j, k;
        const int64_t e = this_colour_node(vb, L.g, 0, p, i, j, k);
        if (e < 0) continue;
        T Dg;
        const T s = nsum<T>(L, e, [&](int64_t n) { return x[n]; }, &Dg);
        r[e] = L.b[e] - (Dg * x[e] - s);
    }
}

// coarse right-hand side P^T r on level l from the red residual of level l - 1: fine node 2I
// and its 12 red neighbours (two odd offsets, weight 1/4); the other 14 of the 27 are black.
// Level 0's residual is in the red-black layout.
template <typename T>
__global__ void __launch_bounds__(256) kb_restrict(Bt<T> B, int l, GateSpec gs)
{
    int local;
    const GMEM MGDev<T>& D = *B.d[bt_find(B.off, B.P, local)];
    if (gated_out(gs, D.st)) return;
    const Grid gc = D.lv[l].g;
    GMEM T* __restrict__ bc = const_cast<GMEM T*>(D.lv[l].b);
    const VB vb = vb_lev(gc, false, local);
#pragma unroll
    for (int p = 0; p < kPlanes; ++p) {
        bool red;
        const int64_t ec = this_node(vb, gc, p, red);
        if (ec < 0) continue;
        const int K = 1 + vb.x * 64 + (int)(threadIdx.x & 63);
        const int J = 1 + vb.y * 4 + (int)(threadIdx.x >> 6);
        const int I = 1 + vb.z * kPlanes + p;
        const int i = 2 * I, j = 2 * J, k = 2 * K;
        if (l == 1) {
            const GMEM T* __restrict__ r = D.r0;
            auto R = [&](int a, int b, int c) { return r[D.rb.idx(i + a, j + b, k + c)]; };
            const T xy = (R(-1, -1, 0) + R(-1, 1, 0)) + (R(1, -1, 0) + R(1, 1, 0));
            const T xz = (R(-1, 0, -1) + R(-1, 0, 1)) + (R(1, 0, -1) + R(1, 0, 1));
            const T yz = (R(0, -1, -1) + R(0, -1, 1)) + (R(0, 1, -1) + R(0, 1, 1));
            bc[ec] = R(0, 0, 0) + (T)0.25 * ((xy + xz) + yz);
        } else {
            const Grid gf = D.lv[l - 1].g;
            const GMEM T* __restrict__ r = D.r[l - 1];
            const int64_t sx = (int64_t)gf.ny * gf.S, sy = gf.S;
            const int64_t f = gf.idx(i, j, k);
            const T xy = (r[f - sx - sy] + r[f - sx + sy]) + (r[f + sx - sy] + r[f + sx + sy]);
            const T xz = (r[f - sx - 1] + r[f - sx + 1]) + (r[f + sx - 1] + r[f + sx + 1]);
            const T yz = (r[f - sy - 1] + r[f - sy + 1]) + (r[f + sy - 1] + r[f + sy + 1]);
            bc[ec] = r[f] + (T)0.25 * ((xy + xz) + yz);
        }
    }
}

// x += P e at the red nodes of coarse level l from level l + 1: post-smoothing starts with a
// black half-sweep, which replaces every black value from its red neighbours
template <typename T>
__global__ void __launch_bounds__(256) kb_prolong(Bt<T> B, int l, GateSpec gs)
{
    int local;
    const GMEM MGDev<T>& D = *B.d[bt_find(B.off, B.P, local)];
    if (gated_out(gs, D.st)) return;
    const Lev<T> L = D.lv[l];
    const Grid gc = D.lv[l + 1].g;
    const GMEM T* __restrict__ ec = D.lv[l + 1].x;
    const VB vb = vb_lev(L.g, true, local);
#pragma unroll
    for (int p = 0; p < kPlanes; ++p) {
        int i, j, k;
        const int64_t e = this_colour_node(vb, L.g, 0, p, i, j, k);
        if (e < 0) continue;
        L.x[e] += prolong_at(gc, ec, i, j, k);
    }
}

// the coarsest level in one block: red from zero, then (black, red) x cs
template <typename T>
__global__ void __launch_bounds__(256) kb_coarse(Bt<T> B, GateSpec gs)
{
    int local;
    const GMEM MGDev<T>& D = *B.d[bt_find(B.off, B.P, local)];
    if (gated_out(gs, D.st)) return;
    const Lev<T> L = D.lv[D.nlev - 1];
    const Grid& g = L.g;
    const int n = (int)interior_count(g), nc = (int)colour_threads(g);
    for (int t = threadIdx.x; t < n; t += 256) {
        bool red;
        const int64_t e = interior_node(g, t, red);
        L.x[e] = red ? L.b[e] * L.dinv[e] : (T)0;
    }
    __syncthreads();
    const GMEM T* __restrict__ x = L.x;
    for (int s = 0; s < 2 * D.cs; ++s) {
        const int c = (s & 1) ? 0 : 1;
        for (int t = threadIdx.x; t < nc; t += 256) {
            const int64_t e = colour_node(g, c, t);
            if (e < 0) continue;
            const T sum = nsum<T>(L, e, [&](int64_t m) { return x[m]; });
            L.x[e] = (L.b[e] + sum) * L.dinv[e];
        }
        __syncthreads();
    }
}

// ---- the small levels of a V-cycle in one block ------------------------------------------
// Levels of at most kSubcycleNodes unknowns would each cost several launches of a few
// microseconds that do little work; one block of kSubThreads threads runs the part of the
// V-cycle from level ls down (its right-hand side given) in one launch, with a block barrier
// between phases.  Same steps and order as the multi-launch path.
constexpr int kSubcycleNodes = 8192;
constexpr int kSubThreads = 1024;

template <typename T>
__device__ __forceinline__ void blk_sweep(const Lev<T>& L, int c)
{
    const int nc = (int)colour_threads(L.g);
    const GMEM T* __restrict__ x = L.x;
    for (int t = threadIdx.x; t < nc; t += kSubThreads) {
        const int64_t e = colour_node(L.g, c, t);
        if (e < 0) continue;
        const T s = nsum<T>(L, e, [&](int64_t m) { return x[m]; });
        L.x[e] = (L.b[e] + s) * L.dinv[e];
    }
    __syncthreads();
}

template <typename T>
__device__ __forceinline__ void blk_red_from_zero(const Lev<T>& L)
{
    const int nc = (int)colour_threads(L.g);
    for (int t = threadIdx.x; t < nc; t += kSubThreads) {
        const int64_t e = colour_node(L.g, 0, t);
        if (e >= 0) L.x[e] = L.b[e] * L.dinv[e];
    }
    __syncthreads();
}

template <typename T>
__global__ void __launch_bounds__(kSubThreads) kb_subcycle(Bt<T> B, GateSpec gs)
{
    int local;
    const GMEM MGDev<T>& D = *B.d[bt_find(B.off, B.P, local)];
    if (gated_out(gs, D.st)) return;
    const int l0 = D.ls, nl = D.nlev;
    // down: pre-smoothing, residual at the red nodes, restriction
    for (int l = l0; l + 1 < nl; ++l) {
        const Lev<T> L = D.lv[l];
        blk_red_from_zero(L);
        blk_sweep(L, 1);
        for (int v = 1; v < D.nu; ++v) {
            blk_sweep(L, 0);
            blk_sweep(L, 1);
        }
        const int nc = (int)colour_threads(L.g);
        const GMEM T* __restrict__ x = L.x;
        GMEM T* __restrict__ rl = D.r[l];
        for (int t = threadIdx.x; t < nc; t += kSubThreads) {
            const int64_t e = colour_node(L.g, 0, t);
            if (e < 0) continue;
            T Dg;
            const T s = nsum<T>(L, e, [&](int64_t m) { return x[m]; }, &Dg);
            rl[e] = L.b[e] - (Dg * x[e] - s);
        }
        __syncthreads();
        const Grid& gf = L.g;
        const Grid gc = D.lv[l + 1].g;
        const GMEM T* __restrict__ r = rl;
        GMEM T* bc = const_cast<GMEM T*>(D.lv[l + 1].b);
        const int n = (int)interior_count(gc);
        const int64_t sx = (int64_t)gf.ny * gf.S, sy = gf.S;
        for (int t = threadIdx.x; t < n; t += kSubThreads) {
            bool red;
            const int64_t ec = interior_node(gc, t, red);
            const int64_t q = ec - Z0;
            const int K = (int)(q % gc.S), J = (int)((q / gc.S) % gc.ny), I = (int)(q / ((int64_t)gc.ny * gc.S));
            const int64_t f = gf.idx(2 * I, 2 * J, 2 * K);
            const T xy = (r[f - sx - sy] + r[f - sx + sy]) + (r[f + sx - sy] + r[f + sx + sy]);
            const T xz = (r[f - sx - 1] + r[f - sx + 1]) + (r[f + sx - 1] + r[f + sx + 1]);
            const T yz = (r[f - sy - 1] + r[f - sy + 1]) + (r[f + sy - 1] + r[f + sy + 1]);
            bc[ec] = r[f] + (T)0.25 * ((xy + xz) + yz);
        }
        __syncthreads();
    }
    // coarsest: red from zero, then (black, red) x cs
    {
        const Lev<T> L = D.lv[nl - 1];
        blk_red_from_zero(L);
        for (int v = 0; v < D.cs; ++v) {
            blk_sweep(L, 1);
            blk_sweep(L, 0);
        }
    }
    // up: coarse correction, post-smoothing
    for (int l = nl - 2; l >= l0; --l) {
        const Lev<T> L = D.lv[l];
        const Grid gc = D.lv[l + 1].g;
        const GMEM T* __restrict__ ec = D.lv[l + 1].x;
        const int n = (int)colour_threads(L.g);
        for (int t = threadIdx.x; t < n; t += kSubThreads) {
            const int64_t e = colour_node(L.g, 0, t);   // red nodes only, as in kb_prolong
            if (e < 0) continue;
            const int64_t q = e - Z0;
            const int k = (int)(q % L.g.S), j = (int)((q / L.g.S) % L.g.ny), i = (int)(q / ((int64_t)L.g.ny * L.g.S));
            L.x[e] += prolong_at(gc, ec, i, j, k);
        }
        __syncthreads();
        for (int v = 0; v < D.nu; ++v) {
            blk_sweep(L, 1);
            blk_sweep(L, 0);
        }
    }
}

// ---- level 0 (red-black layout) ------------------------------------------------------------

__device__ __forceinline__ void bsum(double* v, int nv, double* sh)
{
    for (int t = 0; t < nv; ++t)
        for (int o = 32; o > 0; o >>= 1) v[t] += __shfl_xor(v[t], o, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0)
        for (int t = 0; t < nv; ++t) sh[4 * t + w] = v[t];
    __syncthreads();
    for (int t = 0; t < nv; ++t) v[t] = (sh[4 * t] + sh[4 * t + 1]) + (sh[4 * t + 2] + sh[4 * t + 3]);
}

// the first smoothing step from a zero iterate: red x = b / D, then black
// x = (b + sum K x_red) / D with the red values formed on the fly
template <typename T>
__global__ void __launch_bounds__(256) kb_rb_down1(Bt<T> B, GateSpec gs)
{
    int local;
    const GMEM MGDev<T>& D = *B.d[bt_find(B.off, B.P, local)];
    if (local >= D.nb) return;   // alignment padding between problems
    if (gated_out(gs, D.st)) return;
    const RB R = D.rb;
    const VB vb = vb_rb(R, local, D.nb);
    const RBFrame F = rb_frame(R, vb);
    const GMEM uint32_t* code = D.op.code + F.org;
    const GMEM T* b = D.cr + F.org;
    const GMEM T* dinv = D.dinv0 + F.org;
    GMEM T* x = D.cz + F.org;
    uint32_t cc[kPlanesRB][1];
    const bool uncut = rb_codes<1>(vb, R, F, code, 1, cc);
    auto body = [&](auto U) {
#pragma unroll
        for (int p = 0; p < kPlanesRB; ++p) {
            int i, j, m;
            if (!rb_slot(vb, R, p, i, j, m)) continue;
            if (rb_node(R, i, j, 0, m) >= 0) {
                const uint32_t e = rb_rel(R, F, i, j, 0, m);
                stf(x, e) = ldf(b, e) * ldf(dinv, e);
            }
            const int k = rb_node(R, i, j, 1, m);
            if (k >= 0) {
                const RBNb n = rb_nb(R, F, i, j, 1, m, k);
                const stencil::NodeK<T> K = rb_k<decltype(U)::value>(D.op, code, n, cc[p][0]);
                const T s = rb_sum(K, n, [&](uint32_t f) { return ldf(b, f) * ldf(dinv, f); });
                stf(x, n.e) = (ldf(b, n.e) + s) * ldf(dinv, n.e);
            }
        }
    };
    if (uncut)
        body(std::true_type{});
    else
        body(std::false_type{});
}

// Gauss-Seidel on the level-0 nodes of colour c; with dot (the last red half-sweep of a
// V-cycle) also the partial sums of r.z = b.x over all unknowns (the black ones are final
// after the black half-sweep), one per block
template <typename T, bool Dot>
__global__ void __launch_bounds__(256) kb_rb_sweep(Bt<T> B, int c, GateSpec gs)
{
    __shared__ double sh[8];
    int local;
    const GMEM MGDev<T>& D = *B.d[bt_find(B.off, B.P, local)];
    if (local >= D.nb) return;   // alignment padding between problems
    if (gated_out(gs, D.st)) return;
    const RB R = D.rb;
    const VB vb = vb_rb(R, local, D.nb);
    const RBFrame F = rb_frame(R, vb);
    const GMEM uint32_t* code = D.op.code + F.org;
    const GMEM T* b = D.cr + F.org;
    const GMEM T* dinv = D.dinv0 + F.org;
    GMEM T* x = D.cz + F.org;
    uint32_t cc[kPlanesRB][1];
    const bool uncut = rb_codes<1>(vb, R, F, code, c, cc);
    double v[1] = {0.0};
    auto body = [&](auto U) {
#pragma unroll
        for (int p = 0; p < kPlanesRB; ++p) {
            int i, j, m;
            if (!rb_slot(vb, R, p, i, j, m)) continue;
            const int k = rb_node(R, i, j, c, m);
            if (k >= 0) {
                const RBNb n = rb_nb(R, F, i, j, c, m, k);
                const stencil::NodeK<T> K = rb_k<decltype(U)::value>(D.op, code, n, cc[p][0]);
                const T s = rb_sum(K, n, [&](uint32_t f) { return ldf((const GMEM T*)x, f); });
                const T bn = ldf_nt(b, n.e);
                const T xn = (bn + s) * ldf_nt(dinv, n.e);
                stf(x, n.e) = xn;
                if constexpr (Dot) v[0] += (double)bn * (double)xn;
            }
            if constexpr (Dot) {
                if (rb_node(R, i, j, 1 - c, m) >= 0) {
                    const uint32_t eb = rb_rel(R, F, i, j, 1 - c, m);
                    v[0] += (double)ldf(b, eb) * (double)ldf((const GMEM T*)x, eb);
                }
            }
        }
    };
    if (uncut)
        body(std::true_type{});
    else
        body(std::false_type{});
    if constexpr (Dot) {
        bsum(v, 1, sh);
        if (threadIdx.x == 0) D.prz[local] = v[0];
    }
}

// residual b - A x at the red nodes of level 0 (the black residual is zero right after a
// black half-sweep), in the red segments of r0
template <typename T>
__global__ void __launch_bounds__(256) kb_rb_resid(Bt<T> B, GateSpec gs)
{
    int local;
    const GMEM MGDev<T>& D = *B.d[bt_find(B.off, B.P, local)];
    if (local >= D.nb) return;   // alignment padding between problems
    if (gated_out(gs, D.st)) return;
    const RB R = D.rb;
    const VB vb = vb_rb(R, local, D.nb);
    const RBFrame F = rb_frame(R, vb);
    const GMEM uint32_t* code = D.op.code + F.org;
    const GMEM T* b = D.cr + F.org;
    const GMEM T* x = D.cz + F.org;
    GMEM T* r = D.r0 + F.org;
    uint32_t cc[kPlanesRB][1];
    const bool uncut = rb_codes<1>(vb, R, F, code, 0, cc);
    auto body = [&](auto U) {
#pragma unroll
        for (int p = 0; p < kPlanesRB; ++p) {
            int i, j, m;
            if (!rb_slot(vb, R, p, i, j, m)) continue;
            const int k = rb_node(R, i, j, 0, m);
            if (k < 0) continue;
            const RBNb n = rb_nb(R, F, i, j, 0, m, k);
            const stencil::NodeK<T> K = rb_k<decltype(U)::value>(D.op, code, n, cc[p][0]);
            const T s = rb_sum(K, n, [&](uint32_t f) { return ldf(x, f); });
            stf(r, n.e) = ldf(b, n.e) - (K.diag() * ldf(x, n.e) - s);
        }
    };
    if (uncut)
        body(std::true_type{});
    else
        body(std::false_type{});
}

// x += P e at the red nodes of level 0 from level 1 (the black half-sweep that follows
// replaces the black ones)
template <typename T>
__global__ void __launch_bounds__(256) kb_rb_prolong(Bt<T> B, GateSpec gs)
{
    int local;
    const GMEM MGDev<T>& D = *B.d[bt_find(B.off, B.P, local)];
    if (local >= D.nb) return;   // alignment padding between problems
    if (gated_out(gs, D.st)) return;
    const RB R = D.rb;
    const VB vb = vb_rb(R, local, D.nb);
    const RBFrame F = rb_frame(R, vb);
    const Grid gc = D.lv[1].g;
    const GMEM T* __restrict__ ec = D.lv[1].x;
    GMEM T* x = D.cz + F.org;
#pragma unroll
    for (int p = 0; p < kPlanesRB; ++p) {
        int i, j, m;
        if (!rb_slot(vb, R, p, i, j, m)) continue;
        const int k = rb_node(R, i, j, 0, m);
        if (k < 0) continue;
        stf(x, rb_rel(R, F, i, j, 0, m)) += prolong_at(gc, ec, i, j, k);
    }
}

// ---- CG over the level-0 unknowns ----------------------------------------------------------

// The search direction is double buffered: an iteration with iter_count = ic reads the old
// direction from buffer ic & 1 and writes the new one to the other (iter_count counts the
// iterations that ran, so a restart between two iterations keeps the pairing).
template <typename T>
__device__ __forceinline__ const GMEM T* p_old(const GMEM CGState* st, const GMEM T* p0, const GMEM T* p1)
{
    return (st->iter_count & 1) ? p1 : p0;
}
template <typename T>
__device__ __forceinline__ GMEM T* p_new(const GMEM CGState* st, GMEM T* p0, GMEM T* p1)
{
    return (st->iter_count & 1) ? p0 : p1;
}

// p = z + beta p_old and q = A p at both nodes of each position in one pass (the new direction
// at the neighbours is formed on the fly from z and p_old, which box positions hold as 0);
// partial sums of p.q, one per block
template <typename T>
__global__ void __launch_bounds__(256) kb_rb_apply(Bt<T> B)
{
    __shared__ double sh[8];
    int local;
    const GMEM MGDev<T>& D = *B.d[bt_find(B.off, B.P, local)];
    if (local >= D.nb) return;   // alignment padding between problems
    const GMEM CGState* st = D.st;
    if (st->status != 0) return;
    const RB R = D.rb;
    const VB vb = vb_rb(R, local, D.nb);
    const RBFrame F = rb_frame(R, vb);
    const GMEM uint32_t* code = D.op.code + F.org;
    const GMEM T* z = D.cz + F.org;
    const GMEM T* po = p_old(st, (const GMEM T*)D.cp, (const GMEM T*)D.cp2) + F.org;
    GMEM T* pn = p_new(st, D.cp, D.cp2) + F.org;
    GMEM T* q = D.cq + F.org;
    const T beta = (T)st->beta;
    auto pd = [&](uint32_t f) { return ldf(z, f) + beta * ldf(po, f); };
    uint32_t cc[kPlanesRB][2];
    const bool uncut = rb_codes<2>(vb, R, F, code, 0, cc);
    double v[1] = {0.0};
    auto body = [&](auto U) {
#pragma unroll
        for (int p = 0; p < kPlanesRB; ++p) {
            int i, j, m;
            if (!rb_slot(vb, R, p, i, j, m)) continue;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int k = rb_node(R, i, j, c, m);
                if (k < 0) continue;
                const RBNb n = rb_nb(R, F, i, j, c, m, k);
                const stencil::NodeK<T> K = rb_k<decltype(U)::value>(D.op, code, n, cc[p][c]);
                const T pe = pd(n.e);
                const T qe = K.diag() * pe - rb_sum(K, n, pd);
                stf(pn, n.e) = pe;
                stf(q, n.e) = qe;
                v[0] += (double)pe * (double)qe;
            }
        }
    };
    if (uncut)
        body(std::true_type{});
    else
        body(std::false_type{});
    bsum(v, 1, sh);
    if (threadIdx.x == 0) D.part[local] = v[0];
}

// x += alpha p, r -= alpha q at the level-0 unknowns (box and padding positions hold 0 in p,
// q and r, and are left alone); partial sums of r.r (after the nb slots of the p.q sums)
template <typename T>
__global__ void __launch_bounds__(256) kb_rb_update(Bt<T> B)
{
    __shared__ double sh[8];
    int local;
    const GMEM MGDev<T>& D = *B.d[bt_find(B.off, B.P, local)];
    if (local >= D.nb) return;   // alignment padding between problems
    const GMEM CGState* st = D.st;
    if (st->status != 0) return;
    const RB R = D.rb;
    const VB vb = vb_rb(R, local, D.nb);
    const RBFrame F = rb_frame(R, vb);
    const GMEM T* p = p_new(st, D.cp, D.cp2) + F.org;
    GMEM T* x = D.cx + F.org;
    GMEM T* r = D.cr + F.org;
    const GMEM T* q = D.cq + F.org;
    const T a = (T)st->alpha;
    double v[1] = {0.0};
#pragma unroll
    for (int pl = 0; pl < kPlanesRB; ++pl) {
        int i, j, m;
        if (!rb_slot(vb, R, pl, i, j, m)) continue;
        for (int c = 0; c < 2; ++c) {
            if (rb_node(R, i, j, c, m) < 0) continue;
            const uint32_t e = rb_rel(R, F, i, j, c, m);
            // streamed once: non-temporal, and x (read again only by the next update or a
            // residual replacement) stored non-temporal; r stays cached for the V-cycle that
            // follows
            __builtin_nontemporal_store(ldf_nt((const GMEM T*)x, e) + a * ldf_nt(p, e), &stf(x, e));
            const T rv = ldf_nt((const GMEM T*)r, e) - a * ldf_nt(q, e);
            stf(r, e) = rv;
            v[0] += (double)rv * (double)rv;
        }
    }
    bsum(v, 1, sh);
    if (threadIdx.x == 0) D.part[D.nb + local] = v[0];
}

// partial sums of r.z at the level-0 unknowns (a single-level V-cycle forms no r.z itself)
template <typename T>
__global__ void __launch_bounds__(256) kb_rb_dot(Bt<T> B, GateSpec gs)
{
    __shared__ double sh[8];
    int local;
    const GMEM MGDev<T>& D = *B.d[bt_find(B.off, B.P, local)];
    if (local >= D.nb) return;   // alignment padding between problems
    if (gated_out(gs, D.st)) return;
    const RB R = D.rb;
    const VB vb = vb_rb(R, local, D.nb);
    const RBFrame F = rb_frame(R, vb);
    const GMEM T* r = D.cr + F.org;
    const GMEM T* z = D.cz + F.org;
    double v[1] = {0.0};
#pragma unroll
    for (int pl = 0; pl < kPlanesRB; ++pl) {
        int i, j, m;
        if (!rb_slot(vb, R, pl, i, j, m)) continue;
        for (int c = 0; c < 2; ++c) {
            if (rb_node(R, i, j, c, m) < 0) continue;
            const uint32_t e = rb_rel(R, F, i, j, c, m);
            v[0] += (double)ldf(r, e) * (double)ldf(z, e);
        }
    }
    bsum(v, 1, sh);
    if (threadIdx.x == 0) D.part[local] = v[0];
}

// the FP64 solution (natural layout) += the correction in the red-black layout, which is then
// cleared (with force, or where the iteration stopped for a restart)
template <typename T>
__global__ void __launch_bounds__(256) kb_rb_fold(Bt<T> B, int force)
{
    int local;
    const GMEM MGDev<T>& D = *B.d[bt_find(B.off, B.P, local)];
    if (local >= D.nb) return;   // alignment padding between problems
    if (!force && D.st->status != 3) return;
    const RB R = D.rb;
    const VB vb = vb_rb(R, local, D.nb);
#pragma unroll
    for (int p = 0; p < kPlanesRB; ++p) {
        int i, j, m;
        if (!rb_slot(vb, R, p, i, j, m)) continue;
        for (int c = 0; c < 2; ++c) {
            const int k = rb_node(R, i, j, c, m);
            if (k < 0) continue;
            const int64_t e = R.at(i, j, c, m);
            D.x64[D.g0.idx(i, j, k)] += (double)D.cx[e];
            D.cx[e] = (T)0;
        }
    }
}

// r = b - A x in FP64 from the natural-layout solution, right-hand side and codes, stored in
// the element type in the red-black layout; partial sums of the FP64 r.r in the third slot
// range, one per block.  force 2: x = 0 (the first residual), r = b without the operator (the
// same values: b - (D 0 - sum K 0) is b)
template <typename T>
__global__ void __launch_bounds__(256) kb_rb_true_res(Bt<T> B, int force)
{
    __shared__ double sh[8];
    int local;
    const GMEM MGDev<T>& D = *B.d[bt_find(B.off, B.P, local)];
    if (local >= D.nb) return;   // alignment padding between problems
    if (!force && D.st->status != 3) return;
    const RB R = D.rb;
    const Grid g = D.g0;
    const VB vb = vb_rb(R, local, D.nb);
    const GMEM double* __restrict__ x = D.x64;
    const int64_t sx = (int64_t)g.ny * g.S, sy = g.S;
    double v[1] = {0.0};
#pragma unroll
    for (int p = 0; p < kPlanesRB; ++p) {
        int i, j, m;
        if (!rb_slot(vb, R, p, i, j, m)) continue;
        for (int c = 0; c < 2; ++c) {
            const int k = rb_node(R, i, j, c, m);
            if (k < 0) continue;
            const int64_t e = g.idx(i, j, k);
            double rv = D.rhs[e];
            if (force != 2) {
                const stencil::NodeK<double> K = stencil::node_k(g, (const uint32_t*)D.op64.code,
                                                                 (const double*)D.op64.ck, D.op64.kin, D.op64.kout,
                                                                 D.op64.mass, e);
                const double s = ((K.xm * x[e - sx] + K.xp * x[e + sx]) + (K.ym * x[e - sy] + K.yp * x[e + sy])) +
                                 (K.zm * x[e - 1] + K.zp * x[e + 1]);
                rv -= K.diag() * x[e] - s;
            }
            D.cr[R.at(i, j, c, m)] = (T)rv;
            v[0] += rv * rv;
        }
    }
    bsum(v, 1, sh);
    if (threadIdx.x == 0) D.part[2 * D.nb + local] = v[0];
}

// ---- the scalar steps, one block per problem ------------------------------------------------

// sum of n partials in a fixed order (eight interleaved accumulators per thread keep many
// loads in flight)
__device__ __forceinline__ double psum(const GMEM double* __restrict__ a, int n)
{
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int t = threadIdx.x;
    for (; t + 7 * 256 < n; t += 8 * 256)
#pragma unroll
        for (int u = 0; u < 8; ++u) s[u] += a[t + u * 256];
    for (int u = 0; t < n; t += 256, ++u) s[u & 7] += a[t];
    return ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

template <typename T>
__global__ void __launch_bounds__(256) kb_alpha(Bt<T> B)
{
    __shared__ double sh[8];
    int local;
    const GMEM MGDev<T>& D = *B.d[bt_find(B.off, B.P, local)];
    GMEM CGState* st = D.st;
    if (st->status != 0) return;
    double v[1] = {psum(D.part, D.nb)};
    bsum(v, 1, sh);
    if (threadIdx.x == 0) {
        const double pq = v[0];
        st->pq = pq;
        if (!(pq > 0.0) || !isfinite(pq)) {
            st->status = 2;
            st->iters = st->iter_count;
        } else {
            st->alpha = st->gamma / pq;
        }
    }
}

// mode 0 (an iteration): beta = r.z / r.z_old, the iteration count and the stop test on the
// recursive r.r (status = stop_status once r.r <= stop2, or <= trig2 in mixed precision);
// mode 1 (first residual): beta = 0; mode 2 (after a residual replacement): the direction
// update that the stopped step skipped takes beta = r'.z' / (r.z of the step before);
// mode 3: mode 2 where a replacement has just run in this iteration (ru set), mode 0 otherwise.
// The r.z partials are those of the fused last half-sweep (prz), or of the dot pass (part)
// for a single-level V-cycle.
template <typename T>
__global__ void __launch_bounds__(256) kb_beta(Bt<T> B, int mode_arg)
{
    __shared__ double sh[8];
    int local;
    const GMEM MGDev<T>& D = *B.d[bt_find(B.off, B.P, local)];
    GMEM CGState* st = D.st;
    if (st->status != 0) return;
    // read by every thread before the block sums below; thread 0 writes ru after them
    const int mode = mode_arg == 3 ? (st->ru ? 2 : 0) : mode_arg;
    if (st->ru != (mode == 0 ? 0 : 1)) return;
    double v[2] = {psum(D.nlev > 1 ? D.prz : D.part, D.nb), mode == 0 ? psum(D.part + D.nb, D.nb) : 0.0};
    bsum(v, 2, sh);
    if (threadIdx.x == 0) {
        const double gm = v[0];
        if (mode == 0) {
            const double rr = v[1];
            st->iter_count += 1;
            st->beta = st->gamma > 0.0 ? gm / st->gamma : 0.0;
            st->rr = rr;
            if (!isfinite(gm) || !isfinite(rr)) {
                st->status = 2;
                st->iters = st->iter_count;
            } else if (rr <= st->stop2 || rr <= st->trig2) {
                st->status = st->stop_status;
                st->iters = st->iter_count;
            }
        } else if (mode == 1) {
            st->beta = 0.0;
            st->ru = 0;
        } else {
            st->beta = (st->gamma > 0.0 && st->beta > 0.0) ? gm * (st->beta / st->gamma) : 0.0;
            st->ru = 0;
        }
        st->gamma = gm;
        // the V-cycle is positive definite: r.z > 0 unless r = 0
        if (!isfinite(gm) || !(gm > 0.0)) {
            st->status = 2;
            st->iters = st->iter_count;
        }
    }
}

// after a true residual: the FP64 norm decides convergence; with init it sets the goals.  A
// restart that goes on sets ru, which lets the V-cycle, r.z and beta of the restart run.
template <typename T>
__global__ void __launch_bounds__(256) kb_ru_fin(Bt<T> B, int init, int force)
{
    __shared__ double sh[8];
    int local;
    const GMEM MGDev<T>& D = *B.d[bt_find(B.off, B.P, local)];
    GMEM CGState* st = D.st;
    if (!force && st->status != 3) return;
    double v[1] = {psum(D.part + 2 * D.nb, D.nb)};
    bsum(v, 1, sh);
    if (threadIdx.x == 0) {
        const double rr64 = v[0];
        if (init) {
            st->alpha = st->beta = st->gamma = st->pq = 0.0;
            st->bnorm2 = rr64;
            st->goal64 = D.rtol2 * rr64;
            st->stop2 = D.rtol2 * rr64;
            st->delta2 = D.mixed ? D.delta2 : 0.0;
            st->stop_status = D.mixed ? 3 : 1;
            st->iters = st->iter_count = st->ru = st->n_ru = 0;
        } else {
            st->n_ru += 1;
        }
        st->rr = rr64;
        st->rr64 = rr64;
        st->trig2 = st->delta2 * rr64;
        if (!isfinite(rr64)) {
            st->status = 2;
            st->iters = st->iter_count;
        } else if (rr64 <= st->goal64) {
            st->status = 1;
            st->iters = st->iter_count;
        } else {
            st->status = 0;
        }
        st->ru = st->status == 0 ? 1 : 0;
    }
}

// every problem's state into one array (the serving loop reads them back in one copy)
template <typename T>
__global__ void __launch_bounds__(64) kb_gather(Bt<T> B, CGState* out)
{
    int local;
    const int p = bt_find(B.off, B.P, local);
    const GMEM MGDev<T>& D = *B.d[p];
    const int n = (int)(sizeof(CGState) / sizeof(int));
    const int* s = (const int*)D.st;
    int* o = (int*)(out + p);
    for (int t = threadIdx.x; t < n; t += 64) o[t] = s[t];
}

// ---- set-up and test helpers (one problem) ------------------------------------------------

// codes in the red-black layout (C_BOX on box and padding positions); an interior node none
// of whose six edges is cut also carries C_RB_UNCUT
__global__ void __launch_bounds__(256) k_rb_code(Grid g, RB r, const uint32_t* __restrict__ code, uint32_t* __restrict__ out)
{
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < r.N; t += (int64_t)gridDim.x * 256) {
        const int m = (int)(t % r.Sh);
        const int64_t q = t / r.Sh;
        const int c = (int)(q & 1);
        const int64_t row = q >> 1;
        const int j = (int)(row % r.ny), i = (int)(row / r.ny);
        const int k = 2 * m + ((i + j + c) & 1);
        if (k >= r.nz) {
            out[t] = C_BOX;
            continue;
        }
        const int64_t e = g.idx(i, j, k);
        uint32_t cn = code[e];
        if (i >= 1 && i <= g.nx - 2 && j >= 1 && j <= g.ny - 2 && k >= 1 && k <= g.nz - 2) {
            const uint32_t cut = (cn & (7u * C_CUTX)) | (code[e - (int64_t)g.ny * g.S] & C_CUTX) |
                                 (code[e - g.S] & (C_CUTX << 1)) | (code[e - 1] & (C_CUTX << 2));
            if (!cut) cn |= C_RB_UNCUT;
        }
        out[t] = cn;
    }
}

// 1 / diagonal of the level-0 unknowns in the red-black layout (0 elsewhere)
template <typename T>
__global__ void __launch_bounds__(256) k_rb_diag0(Grid g, RB r, Op0<T> op, T* __restrict__ dinv)
{
    const VB vb = vb_rb(r, (int)blockIdx.x, (int)gridDim.x);
#pragma unroll
    for (int p = 0; p < kPlanesRB; ++p) {
        int i, j, m;
        if (!rb_slot(vb, r, p, i, j, m)) continue;
        for (int c = 0; c < 2; ++c) {
            const int k = rb_node(r, i, j, c, m);
            if (k < 0) continue;
            dinv[r.at(i, j, c, m)] =
                (T)1 / stencil::node_k(g, (const uint32_t*)op.code, (const T*)op.ck, op.kin, op.kout, op.mass, g.idx(i, j, k)).diag();
        }
    }
}

// natural-layout level-0 vector <-> red-black layout (interior nodes; the two-level
// preconditioner of refined grids hands its coarse right-hand side over in the natural layout)
template <typename T>
__global__ void __launch_bounds__(256) k_rb_convert(Grid g, RB r, T* __restrict__ nat, T* __restrict__ rbv, int to_rb,
                                                    GateSpec gs, const CGState* st)
{
    if (gated_out(gs, gmem(st))) return;
    const VB vb = vb_rb(r, (int)blockIdx.x, (int)gridDim.x);
#pragma unroll
    for (int p = 0; p < kPlanesRB; ++p) {
        int i, j, m;
        if (!rb_slot(vb, r, p, i, j, m)) continue;
        for (int c = 0; c < 2; ++c) {
            const int k = rb_node(r, i, j, c, m);
            if (k < 0) continue;
            if (to_rb)
                rbv[r.at(i, j, c, m)] = nat[g.idx(i, j, k)];
            else
                nat[g.idx(i, j, k)] = rbv[r.at(i, j, c, m)];
        }
    }
}

// ---- hierarchy set-up (FP64) ------------------------------------------------------------

struct FineSrc {            // the operator of the level being coarsened
    Grid g;
    const uint32_t* code;   // level 0: node-code map (else nullptr)
    const double* ck;
    double kin, kout, mass;
    const double *kx, *ky, *kz, *m;   // levels >= 1
    __device__ double K(int ax, int64_t e) const
    {
        if (code) return stencil::edgeK(code[e], ax, ck, kin, kout);
        return ax == 0 ? kx[e] : ax == 1 ? ky[e] : kz[e];
    }
    __device__ double M(int64_t e) const
    {
        if (code) return (code[e] & C_SOLUTE) ? 0.0 : mass;
        return m[e];
    }
};

__device__ __forceinline__ double series(double a, double b)
{
    const double t = a + b;
    return t > 0.0 ? a * b / t : 0.0;
}

// coarse K along each axis and the coarse ionic term, one thread per coarse node
__global__ void __launch_bounds__(256) k_coarsen(FineSrc F, Grid gc, double* kx, double* ky, double* kz, double* m)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t n = (int64_t)gc.nx * gc.ny * gc.nz;
    if (t >= n) return;
    const int K = (int)(t % gc.nz), J = (int)((t / gc.nz) % gc.ny), I = (int)(t / ((int64_t)gc.nz * gc.ny));
    const int64_t ec = gc.idx(I, J, K);
    const int C[3] = {I, J, K};
    const int nc[3] = {gc.nx, gc.ny, gc.nz};
    const double w3[3] = {0.25, 0.5, 0.25};
    double* out[3] = {kx, ky, kz};
    for (int ax = 0; ax < 3; ++ax) {
        const int t1 = ax == 0 ? 1 : 0, t2 = ax == 2 ? 1 : 2;
        bool ok = C[ax] <= nc[ax] - 2;
        ok = ok && C[t1] >= 1 && C[t1] <= nc[t1] - 2 && C[t2] >= 1 && C[t2] <= nc[t2] - 2;
        double acc = 0.0;
        if (ok) {
            for (int a = -1; a <= 1; ++a)
                for (int b = -1; b <= 1; ++b) {
                    int f[3] = {2 * I, 2 * J, 2 * K};
                    f[t1] += a;
                    f[t2] += b;
                    const int64_t e1 = F.g.idx(f[0], f[1], f[2]);
                    f[ax] += 1;
                    const int64_t e2 = F.g.idx(f[0], f[1], f[2]);
                    acc += w3[a + 1] * w3[b + 1] * series(F.K(ax, e1), F.K(ax, e2));
                }
        }
        out[ax][ec] = 4.0 * acc;
    }
    double mm = 0.0;
    if (I >= 1 && I <= gc.nx - 2 && J >= 1 && J <= gc.ny - 2 && K >= 1 && K <= gc.nz - 2) {
        for (int a = -1; a <= 1; ++a)
            for (int b = -1; b <= 1; ++b)
                for (int c = -1; c <= 1; ++c) {
                    const double w = (a ? 0.5 : 1.0) * (b ? 0.5 : 1.0) * (c ? 0.5 : 1.0);
                    mm += w * F.M(F.g.idx(2 * I + a, 2 * J + b, 2 * K + c));
                }
    }
    m[ec] = mm;
}

// 1 / diagonal at the interior nodes of a coarse level, and the element-type copies
template <typename T>
__global__ void __launch_bounds__(256) k_level_diag(Grid g, const double* kx, const double* ky, const double* kz,
                                                    const double* m, T* kxT, T* kyT, T* kzT, T* diagT, T* dinvT)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    if (t >= n) return;
    const int k = (int)(t % g.nz), j = (int)((t / g.nz) % g.ny), i = (int)(t / ((int64_t)g.nz * g.ny));
    const int64_t e = g.idx(i, j, k);
    kxT[e] = (T)kx[e];
    kyT[e] = (T)ky[e];
    kzT[e] = (T)kz[e];
    double D = 0.0, d = 0.0;
    if (i >= 1 && i <= g.nx - 2 && j >= 1 && j <= g.ny - 2 && k >= 1 && k <= g.nz - 2) {
        const int64_t sx = (int64_t)g.ny * g.S, sy = g.S;
        D = ((kx[e - sx] + kx[e]) + (ky[e - sy] + ky[e])) + ((kz[e - 1] + kz[e]) + m[e]);
        d = 1.0 / D;
    }
    diagT[e] = (T)D;
    dinvT[e] = (T)d;
}

}  // namespace

// ---- host side -----------------------------------------------------------------------------

namespace {

Grid coarse_grid(const Grid& f)
{
    Grid c = f;
    c.nx = (f.nx - 1) / 2 + 1;
    c.ny = (f.ny - 1) / 2 + 1;
    c.nz = (f.nz - 1) / 2 + 1;
    c.S = (int)row_stride(c.nz);
    c.N = (int64_t)c.nx * c.ny * c.S;
    c.h = 2.0 * f.h;
    return c;
}

bool can_coarsen(const Grid& g)
{
    const int n[3] = {g.nx, g.ny, g.nz};
    for (int d = 0; d < 3; ++d)
        if ((n[d] - 1) % 2 != 0 || (n[d] - 1) / 2 + 1 < 3) return false;
    return true;
}

// a coarsest level of at most this many unknowns runs in one block
constexpr int64_t kOneBlockCoarse = 32768;

template <typename T>
Op0<T> op0(const pb_problem* pb)
{
    Op0<T> o;
    o.code = gmem((const uint32_t*)pb->code);
    if constexpr (sizeof(T) == 8)
        o.ck = gmem((const T*)pb->ck64);
    else
        o.ck = gmem((const T*)pb->ck32);
    o.kin = (T)pb->cf.kin;
    o.kout = (T)pb->cf.kout;
    o.mass = (T)pb->cf.mass;
    return o;
}

// ---- launch plans --------------------------------------------------------------------------
// A plan lists, for a set of problems, how many blocks each has in every kind of pass: the
// level-0 passes (and the streaming CG passes, which use as many blocks), the one-block scalar
// steps, the one-block small levels, a one-block coarsest level, a large coarsest level
// (all nodes / one colour), and per coarse level l the pre/post-smoothing passes (all nodes /
// one colour) and the restriction onto it.  The block offsets of every pass kind go to the
// device in one table.
enum PassKind {
    K_RB0 = 0,
    K_ONE,
    K_SUB,
    K_COARSE1,
    K_CALL,
    K_CCOL,
    K_ALL,
    K_COL = K_ALL + PB_MG_MAX_LEVELS,
    K_RES = K_COL + PB_MG_MAX_LEVELS,
    K_N = K_RES + PB_MG_MAX_LEVELS
};

// blocks of one problem in each pass kind
void pass_counts(const MGData* G, int* cnt)
{
    for (int k = 0; k < K_N; ++k) cnt[k] = 0;
    const int L = G->nlev;
    cnt[K_RB0] = G->nb;
    cnt[K_ONE] = 1;
    if (L < 2) return;
    const int top = std::min(G->ls, L - 1);   // levels [1, top) smooth and restrict in launches of their own
    for (int l = 1; l < top; ++l) {
        cnt[K_ALL + l] = lev_blocks(G->g[l], false);
        cnt[K_COL + l] = lev_blocks(G->g[l], true);
    }
    for (int l = 1; l <= top; ++l) cnt[K_RES + l] = lev_blocks(G->g[l], false);
    if (G->ls < L) {
        cnt[K_SUB] = 1;
    } else if (interior_count(G->g[L - 1]) <= kOneBlockCoarse) {
        cnt[K_COARSE1] = 1;
    } else {
        cnt[K_CALL] = lev_blocks(G->g[L - 1], false);
        cnt[K_CCOL] = lev_blocks(G->g[L - 1], true);
    }
}

struct Plan {
    int P = 0;
    int total[K_N] = {};
    int top = 0;            // largest first level of the small-level part over the problems
    int nu = 1, cs = 4;
    bool single = false;    // one problem with a single level
    const void* desc = nullptr;   // device: P descriptor pointers
    const int* off = nullptr;     // device: K_N tables of P + 1 offsets
};

// the host tables of a plan: offs[k * (P + 1) + p]
void plan_tables(const std::vector<const MGData*>& Gs, Plan& pl, std::vector<int>& offs)
{
    const int P = (int)Gs.size();
    pl.P = P;
    offs.assign((size_t)K_N * (P + 1), 0);
    int cnt[K_N];
    for (int k = 0; k < K_N; ++k) pl.total[k] = 0;
    pl.top = 0;
    for (int p = 0; p < P; ++p) {
        pass_counts(Gs[p], cnt);
        // a problem's level-0 blocks start at a multiple of 8, so that its block b runs on XCD
        // b % 8 as in a launch of its own (the tile map depends on it)
        pl.total[K_RB0] = (pl.total[K_RB0] + 7) & ~7;
        for (int k = 0; k < K_N; ++k) {
            offs[(size_t)k * (P + 1) + p] = pl.total[k];
            pl.total[k] += cnt[k];
        }
        if (Gs[p]->nlev >= 2) pl.top = std::max(pl.top, std::min(Gs[p]->ls, Gs[p]->nlev - 1));
    }
    for (int k = 0; k < K_N; ++k) offs[(size_t)k * (P + 1) + P] = pl.total[k];
    pl.nu = P ? Gs[0]->nu : 1;
    pl.cs = P ? Gs[0]->cs : 4;
    pl.single = P == 1 && Gs[0]->nlev == 1;
}

template <typename T>
Bt<T> bt(const Plan& pl, int kind)
{
    return Bt<T>{(const GMEM MGDev<T>* const GMEM*)pl.desc, gmem((const int*)(pl.off + (size_t)kind * (pl.P + 1))), pl.P};
}

#define PLAUNCH(kind, threads, kernel, ...)                                                          \
    do {                                                                                             \
        if (pl.total[kind] > 0) kernel<<<pl.total[kind], threads, 0, s>>>(bt<T>(pl, kind), __VA_ARGS__); \
    } while (0)
#define PLAUNCH0(kind, threads, kernel)                                                              \
    do {                                                                                             \
        if (pl.total[kind] > 0) kernel<<<pl.total[kind], threads, 0, s>>>(bt<T>(pl, kind));           \
    } while (0)

// z = V-cycle(r) at level 0 for every problem of the plan; with ev, events around the whole
// V-cycle (ev[0], ev[3]) and around the first level-0 black half-sweep after the coarse
// correction (ev[1], ev[2]).  With more than one level the last half-sweep also writes the
// r.z partial sums (prz).
template <typename T>
void run_vcycle(hipStream_t s, const Plan& pl, GateSpec gs, hipEvent_t* ev = nullptr)
{
    if (pl.single) {
        // one level: red from zero and black, then red, then (black, red) x (cs - 1)
        PLAUNCH(K_RB0, 256, kb_rb_down1<T>, gs);
        PLAUNCH(K_RB0, 256, (kb_rb_sweep<T, false>), 0, gs);
        for (int v = 1; v < pl.cs; ++v) {
            PLAUNCH(K_RB0, 256, (kb_rb_sweep<T, false>), 1, gs);
            PLAUNCH(K_RB0, 256, (kb_rb_sweep<T, false>), 0, gs);
        }
        return;
    }
    if (ev) (void)hipEventRecord(ev[0], s);
    // level 0: pre-smoothing, red residual, restriction to level 1
    PLAUNCH(K_RB0, 256, kb_rb_down1<T>, gs);
    for (int v = 1; v < pl.nu; ++v) {
        PLAUNCH(K_RB0, 256, (kb_rb_sweep<T, false>), 0, gs);
        PLAUNCH(K_RB0, 256, (kb_rb_sweep<T, false>), 1, gs);
    }
    PLAUNCH(K_RB0, 256, kb_rb_resid<T>, gs);
    PLAUNCH(K_RES + 1, 256, kb_restrict<T>, 1, gs);
    // coarse levels above the one-block part (or above the coarsest level)
    for (int l = 1; l < pl.top; ++l) {
        PLAUNCH(K_ALL + l, 256, kb_down1<T>, l, gs);
        for (int v = 1; v < pl.nu; ++v) {
            PLAUNCH(K_COL + l, 256, kb_sweep<T>, l, 0, gs);
            PLAUNCH(K_COL + l, 256, kb_sweep<T>, l, 1, gs);
        }
        PLAUNCH(K_COL + l, 256, kb_resid<T>, l, gs);
        PLAUNCH(K_RES + l + 1, 256, kb_restrict<T>, l + 1, gs);
    }
    // the small levels in one block, or the coarsest level
    PLAUNCH(K_SUB, kSubThreads, kb_subcycle<T>, gs);
    PLAUNCH(K_COARSE1, 256, kb_coarse<T>, gs);
    if (pl.total[K_CALL] > 0) {
        // red, black in one pass, then red, then (black, red) x (cs - 1)
        PLAUNCH(K_CALL, 256, kb_down1<T>, -1, gs);
        PLAUNCH(K_CCOL, 256, kb_sweep<T>, -1, 0, gs);
        for (int v = 1; v < pl.cs; ++v) {
            PLAUNCH(K_CCOL, 256, kb_sweep<T>, -1, 1, gs);
            PLAUNCH(K_CCOL, 256, kb_sweep<T>, -1, 0, gs);
        }
    }
    for (int l = pl.top - 1; l >= 1; --l) {
        PLAUNCH(K_COL + l, 256, kb_prolong<T>, l, gs);
        for (int v = 0; v < pl.nu; ++v) {
            PLAUNCH(K_COL + l, 256, kb_sweep<T>, l, 1, gs);
            PLAUNCH(K_COL + l, 256, kb_sweep<T>, l, 0, gs);
        }
    }
    // level 0: coarse correction at the red nodes, post-smoothing; the last red half-sweep
    // also forms the r.z partial sums
    PLAUNCH(K_RB0, 256, kb_rb_prolong<T>, gs);
    if (ev) (void)hipEventRecord(ev[1], s);
    for (int v = 0; v < pl.nu; ++v) {
        PLAUNCH(K_RB0, 256, (kb_rb_sweep<T, false>), 1, gs);
        if (v == 0 && ev) (void)hipEventRecord(ev[2], s);
        if (v == pl.nu - 1)
            PLAUNCH(K_RB0, 256, (kb_rb_sweep<T, true>), 0, gs);
        else
            PLAUNCH(K_RB0, 256, (kb_rb_sweep<T, false>), 0, gs);
    }
    if (ev) (void)hipEventRecord(ev[3], s);
}

// one CG iteration of every problem of the plan (ev: the V-cycle's four events; ea: two
// events around the operator pass).  In mixed precision a problem whose last iteration
// stopped with status 3 (its FP32 residual reached its goal or fell by inner_rtol) skips the
// step and instead replaces its residual: fold the correction into the FP64 solution, r = b -
// A x in FP64 and the convergence test on it; the iteration's V-cycle and beta (mode 3) then
// serve the replaced residual.  A problem's replacement so follows the iteration that asked
// for it, wherever the chunks of iterations end.
template <typename T>
void run_iteration(hipStream_t s, const Plan& pl, hipEvent_t* ev = nullptr, hipEvent_t* ea = nullptr)
{
    const GateSpec gs{nullptr, 4};
    if (ea) (void)hipEventRecord(ea[0], s);
    PLAUNCH0(K_RB0, 256, kb_rb_apply<T>);
    if (ea) (void)hipEventRecord(ea[1], s);
    PLAUNCH0(K_ONE, 256, kb_alpha<T>);
    PLAUNCH0(K_RB0, 256, kb_rb_update<T>);
    if (sizeof(T) == 4) {
        PLAUNCH(K_RB0, 256, kb_rb_fold<T>, 0);
        PLAUNCH(K_RB0, 256, kb_rb_true_res<T>, 0);
        PLAUNCH(K_ONE, 256, kb_ru_fin<T>, 0, 0);
    }
    run_vcycle<T>(s, pl, gs, ev);
    if (pl.single) PLAUNCH(K_RB0, 256, kb_rb_dot<T>, gs);
    PLAUNCH(K_ONE, 256, kb_beta<T>, 3);
}

// restart from the true residual: fold the correction into the FP64 solution, r = b - A x in
// FP64, then z = V-cycle(r), r.z and beta.  With force it runs whatever the state (init: the
// first residual, x = 0); otherwise only where the iteration stopped with status 3.
template <typename T>
void run_restart(hipStream_t s, const Plan& pl, int init, int force)
{
    const GateSpec gs{nullptr, 1};
    // init: x = 0 (both parts were just cleared): nothing to fold, and r = b
    if (!init) PLAUNCH(K_RB0, 256, kb_rb_fold<T>, force);
    PLAUNCH(K_RB0, 256, kb_rb_true_res<T>, init ? 2 : force);
    PLAUNCH(K_ONE, 256, kb_ru_fin<T>, init, force);
    run_vcycle<T>(s, pl, gs);
    if (pl.single) PLAUNCH(K_RB0, 256, kb_rb_dot<T>, gs);
    PLAUNCH(K_ONE, 256, kb_beta<T>, init ? 1 : 2);
}

template <typename T>
Lev<T> level(const MGData* G, int l)
{
    Lev<T> L;
    L.g = G->g[l];
    L.kx = gmem((const T*)G->K[l][0]);
    L.ky = gmem((const T*)G->K[l][1]);
    L.kz = gmem((const T*)G->K[l][2]);
    L.diag = gmem((const T*)G->diag[l]);
    L.dinv = gmem((const T*)G->dinv[l]);
    L.x = gmem((T*)G->x[l]);
    L.b = gmem((const T*)G->b[l]);
    return L;
}

// the descriptor of a problem's hierarchy (host copy)
template <typename T>
MGDev<T> describe(const pb_problem* pb)
{
    const MGData* G = pb->mg;
    const pb_params& P = pb->prm;
    MGDev<T> d;
    memset((void*)&d, 0, sizeof d);
    d.rb = rb_of(pb->g);
    d.g0 = pb->g;
    const Op0<T> o = op0<T>(pb);
    d.op = OpRB<T>{gmem((const uint32_t*)G->code_rb), o.ck, o.kin, o.kout, o.mass};
    d.op64 = op0<double>(pb);
    d.cr = gmem((T*)G->cr);
    d.cz = gmem((T*)G->cz);
    d.cp = gmem((T*)G->cp);
    d.cp2 = gmem((T*)G->cp2);
    d.cq = gmem((T*)G->cq);
    d.cx = gmem((T*)G->cx);
    d.dinv0 = gmem((T*)G->dinv[0]);
    d.r0 = gmem((T*)G->r[0]);
    d.x64 = gmem(pb->x);
    d.rhs = gmem((const double*)pb->rhs);
    d.nlev = G->nlev;
    d.ls = G->ls;
    d.nu = G->nu;
    d.cs = G->cs;
    for (int l = 1; l < G->nlev; ++l) {
        d.lv[l] = level<T>(G, l);
        d.r[l] = gmem((T*)G->r[l]);
    }
    d.st = gmem(pb->st);
    d.part = gmem(G->part);
    d.prz = gmem(G->prz);
    d.nb = G->nb;
    d.mixed = P.precision == PB_MIXED ? 1 : 0;
    d.rtol2 = P.rtol * P.rtol;
    d.delta2 = P.inner_rtol * P.inner_rtol;
    return d;
}

// the level hierarchy, the solver vectors, the problem's descriptor and its one-problem
// plan, enqueued on stream s (no host wait); the FP64 coefficients the element-type copies
// are rounded from stay allocated with the problem
template <typename T>
int setup_levels(pb_problem* pb, MGData* G, hipStream_t s)
{
    const pb_params& P = pb->prm;
    G->g[0] = pb->g;
    G->nlev = 1;
    const int maxl = P.mg_levels > 0 ? std::min(P.mg_levels, PB_MG_MAX_LEVELS) : PB_MG_MAX_LEVELS;
    while (G->nlev < maxl && can_coarsen(G->g[G->nlev - 1])) {
        G->g[G->nlev] = coarse_grid(G->g[G->nlev - 1]);
        ++G->nlev;
    }
    // the first level from which every level has at most kSubcycleNodes unknowns (not 0)
    G->ls = G->nlev;
    while (G->ls - 1 >= 1 && interior_count(G->g[G->ls - 1]) <= kSubcycleNodes) --G->ls;
    // FP64 coefficients of every coarse level, then the element-type copies
    const double *pkx = nullptr, *pky = nullptr, *pkz = nullptr, *pm = nullptr;
    for (int l = 1; l < G->nlev; ++l) {
        const Grid& gc = G->g[l];
        double* c64 = (double*)pb->mem.get(sizeof(double) * 4 * (size_t)gc.N);
        if (!c64) return pbi_fail(PB_ENOMEM, "multigrid levels");
        RCHK(launch_fill(s, c64, sizeof(double) * 4 * (size_t)gc.N));
        double *kx = c64, *ky = c64 + gc.N, *kz = c64 + 2 * gc.N, *m = c64 + 3 * gc.N;
        FineSrc F;
        F.g = G->g[l - 1];
        F.code = l == 1 ? pb->code : nullptr;
        F.ck = pb->ck64;
        F.kin = pb->cf.kin;
        F.kout = pb->cf.kout;
        F.mass = pb->cf.mass;
        F.kx = pkx;
        F.ky = pky;
        F.kz = pkz;
        F.m = pm;
        const int64_t nn = (int64_t)gc.nx * gc.ny * gc.nz;
        k_coarsen<<<nblk(nn, 256), 256, 0, s>>>(F, gc, kx, ky, kz, m);
        // K (three), diagonal, 1/diagonal, and the level's residual, iterate and right-hand side
        T* v = (T*)pb->mem.get(sizeof(T) * 8 * (size_t)gc.N);
        if (!v) return pbi_fail(PB_ENOMEM, "multigrid levels");
        RCHK(launch_fill(s, v, sizeof(T) * 8 * (size_t)gc.N));
        for (int d = 0; d < 3; ++d) G->K[l][d] = v + d * gc.N;
        G->diag[l] = v + 3 * gc.N;
        G->dinv[l] = v + 4 * gc.N;
        G->r[l] = v + 5 * gc.N;
        G->x[l] = v + 6 * gc.N;
        G->b[l] = v + 7 * gc.N;
        k_level_diag<T><<<nblk(nn, 256), 256, 0, s>>>(gc, kx, ky, kz, m, (T*)G->K[l][0], (T*)G->K[l][1],
                                                       (T*)G->K[l][2], (T*)G->diag[l], (T*)G->dinv[l]);
        RCHK(hipGetLastError());
        pkx = kx;
        pky = ky;
        pkz = kz;
        pm = m;
    }
    // level 0 in the red-black layout: the codes, 1 / diagonal, the red residual and the CG
    // vectors r, z, p (two), q and the correction x (x and b of level 0 are z and r)
    const Grid& g0 = pb->g;
    const RB rb = rb_of(g0);
    G->Sh = rb.Sh;
    G->Nrb = rb.N;
    G->code_rb = (uint32_t*)pb->mem.get(sizeof(uint32_t) * (size_t)rb.N);
    if (!G->code_rb) return pbi_fail(PB_ENOMEM, "multigrid codes");
    k_rb_code<<<(unsigned)std::min<int64_t>(65536, nblk(rb.N, 256)), 256, 0, s>>>(g0, rb, pb->code, G->code_rb);
    T* v0 = (T*)pb->mem.get(sizeof(T) * 8 * (size_t)rb.N);
    if (!v0) return pbi_fail(PB_ENOMEM, "multigrid level-0 vectors");
    RCHK(launch_fill(s, v0, sizeof(T) * 8 * (size_t)rb.N));
    void** dst[8] = {&G->dinv[0], &G->r[0], &G->cr, &G->cz, &G->cp, &G->cp2, &G->cq, &G->cx};
    for (int v = 0; v < 8; ++v) *dst[v] = v0 + v * rb.N;
    G->nb = rb_blocks(rb);
    k_rb_diag0<T><<<G->nb, 256, 0, s>>>(g0, rb, op0<T>(pb), (T*)G->dinv[0]);
    G->x[0] = G->cz;
    G->b[0] = G->cr;
    G->nrz = G->nb;
    G->part = (double*)pb->mem.get(sizeof(double) * 4 * (size_t)G->nb);
    if (!G->part) return pbi_fail(PB_ENOMEM, "multigrid partial sums");
    G->prz = G->part + 3 * (size_t)G->nb;
    // the descriptor, the one-problem plan's tables and the pointer to the descriptor
    std::vector<const MGData*> one{G};
    Plan pl;
    std::vector<int> offs;
    plan_tables(one, pl, offs);
    const size_t dbytes = (sizeof(MGDev<T>) + 255) & ~(size_t)255;
    const size_t tbytes = sizeof(int) * offs.size();
    char* blob = (char*)pb->mem.get(dbytes + 256 + tbytes);
    if (!blob) return pbi_fail(PB_ENOMEM, "multigrid descriptor");
    G->dev = blob;
    G->solo_desc = blob + dbytes;
    G->solo_off = (int*)(blob + dbytes + 256);
    G->solo_host.assign(dbytes + 256 + tbytes, 0);
    const MGDev<T> d = describe<T>(pb);
    memcpy(G->solo_host.data(), &d, sizeof d);
    const void* dptr = G->dev;
    memcpy(G->solo_host.data() + dbytes, &dptr, sizeof dptr);
    memcpy(G->solo_host.data() + dbytes + 256, offs.data(), tbytes);
    // pageable source: the copy is complete when the call returns
    RCHK(hipMemcpyAsync(blob, G->solo_host.data(), G->solo_host.size(), hipMemcpyHostToDevice, s));
    RCHK(hipGetLastError());
    return PB_OK;
}

// the one-problem plan of a problem
Plan solo_plan(const pb_problem* pb)
{
    const MGData* G = pb->mg;
    std::vector<const MGData*> one{G};
    Plan pl;
    std::vector<int> offs;
    plan_tables(one, pl, offs);
    pl.desc = G->solo_desc;
    pl.off = G->solo_off;
    return pl;
}

template <typename T>
int begin_t(pb_problem* pb, hipStream_t s)
{
    const pb_params& P = pb->prm;
    if (!pb->mg) {
        pb->mg = new MGData();
        pb->mg->nu = P.mg_smooth > 0 ? P.mg_smooth : 1;
        pb->mg->cs = P.mg_coarse_sweeps > 0 ? P.mg_coarse_sweeps : 4;
        const int rc = setup_levels<T>(pb, pb->mg, s);
        if (rc) return rc;
    }
    return PB_OK;
}

// x = 0 and the first residual, enqueued on s
template <typename T>
int start_t(pb_problem* pb, hipStream_t s)
{
    MGData* G = pb->mg;
    RCHK(launch_fill(s, pb->x, sizeof(double) * (size_t)pb->g.N));
    RCHK(launch_fill(s, G->cx, sizeof(T) * (size_t)G->Nrb));
    RCHK(launch_fill(s, G->cp, sizeof(T) * (size_t)G->Nrb));
    RCHK(launch_fill(s, G->cp2, sizeof(T) * (size_t)G->Nrb));
    RCHK(launch_fill(s, pb->st, sizeof(CGState)));
    run_restart<T>(s, solo_plan(pb), 1, 1);
    RCHK(hipGetLastError());
    return PB_OK;
}

// n iterations enqueued on s; ev[it], where given, receives the four timing events of
// iteration it's V-cycle
// (ran[it], where given: receives the state's status as iteration it starts; 0 means the
// iteration runs, short of a breakdown in its alpha step: only its scalar steps change it)
template <typename T>
int chunk_t(pb_problem* pb, hipStream_t s, int n, hipEvent_t* const* ev, int* const* ran = nullptr)
{
    const Plan pl = solo_plan(pb);
    for (int it = 0; it < n; ++it) {
        if (ran && ran[it]) RCHK(hipMemcpyAsync(ran[it], &pb->st->status, sizeof(int), hipMemcpyDeviceToDevice, s));
        run_iteration<T>(s, pl, ev ? ev[it] : nullptr);
    }
    RCHK(hipGetLastError());
    return PB_OK;
}

// Pipelined like the Jacobi solve: a chunk of iterations is enqueued while the state of the
// previous one is read back, its length from the residual decay seen so far
// (pbi_mg_next_chunk), so that few iterations are launched past convergence.
template <typename T>
int solve_t(pb_problem* pb, CGState* out)
{
    pb_ctx* ctx = pb->ctx;
    hipStream_t s = ctx->stream;
    const pb_params& P = pb->prm;
    int rc = begin_t<T>(pb, s);
    if (!rc) rc = start_t<T>(pb, s);
    if (rc) return rc;
    const int M = 8;
    int launched = 0;
    // sampled timings (context profiling on): every 4th iteration while the V-cycle has
    // more than one level
    const bool prof = ctx->profile != 0 && pb->mg->nlev > 1;
    std::vector<hipEvent_t> evs;
    std::vector<int> ev_it;
    // per sample, the status as its iteration starts (a launch after a stop returns at once)
    constexpr int kMaxSamples = 128;
    int* ran_dev = nullptr;
    if (prof) {
        ran_dev = (int*)pb->mem.get(sizeof(int) * kMaxSamples);
        if (!ran_dev) return pbi_fail(PB_ENOMEM, "profiling flags");
    }
    auto enqueue = [&](int slot, int n) -> int {
        hipEvent_t* ev[M] = {};
        for (int it = 0; prof && it < n; ++it) {
            if ((launched + it) % 4 != 0 || evs.size() >= 4 * kMaxSamples) continue;
            for (int e = 0; e < 4; ++e) {
                // timing only: no system-scope fence, whose cache writeback of the data the
                // sampled kernels wrote would otherwise be counted in their time
                hipEvent_t x;
                RCHK(hipEventCreateWithFlags(&x, hipEventDisableSystemFence));
                evs.push_back(x);
            }
            ev_it.push_back(launched + it);
        }
        // pointers into evs only once it has stopped growing for this chunk
        int* ran[M] = {};
        for (size_t k = 0, it = 0; k < ev_it.size(); ++k)
            if (ev_it[k] >= launched && ev_it[k] < launched + n) {
                it = (size_t)(ev_it[k] - launched);
                ev[it] = &evs[4 * k];
                ran[it] = ran_dev + k;
            }
        const int r = chunk_t<T>(pb, s, n, prof ? ev : nullptr, prof ? ran : nullptr);
        if (r) return r;
        launched += n;
        RCHK(hipMemcpyAsync(&ctx->host_state[slot], pb->st, sizeof(CGState), hipMemcpyDeviceToHost, s));
        RCHK(hipEventRecord(ctx->ev[slot], s));
        return PB_OK;
    };
    // chunks in flight, oldest first (at most two): iterations and state slot
    int q_n[2] = {0, 0}, q_slot[2] = {0, 0}, qlen = 0, next_slot = 0;
    auto push = [&](int n) -> int {
        const int slot = next_slot;
        next_slot ^= 1;
        const int r = enqueue(slot, n);
        if (r) return r;
        q_n[qlen] = n;
        q_slot[qlen] = slot;
        ++qlen;
        return PB_OK;
    };
    if ((rc = push(std::min(M, P.max_iter)))) return rc;
    bool seen = false;
    CGState snap{};
    for (;;) {
        if (qlen < 2 && launched < P.max_iter) {
            int n = seen ? pbi_mg_next_chunk(snap, qlen ? q_n[0] : 0, M) : M;
            n = std::min(n, P.max_iter - launched);
            if (n > 0 && (rc = push(n))) return rc;
        }
        RCHK(hipEventSynchronize(ctx->ev[q_slot[0]]));
        snap = ctx->host_state[q_slot[0]];
        seen = true;
        q_n[0] = q_n[1];
        q_slot[0] = q_slot[1];
        --qlen;
        if (snap.status == 1 || snap.status == 2) break;
        if (qlen == 0 && launched >= P.max_iter) break;
    }
    // the correction into the FP64 solution (all of it in FP64; in the mixed form what is left
    // after the last restart)
    {
        const Plan pl = solo_plan(pb);
        PLAUNCH(K_RB0, 256, kb_rb_fold<T>, 1);
    }
    RCHK(hipMemcpyAsync(out, pb->st, sizeof(CGState), hipMemcpyDeviceToHost, s));
    RCHK(hipStreamSynchronize(s));
    if (prof) {
        // only iterations that ran: the state was running as the sampled iteration started
        std::vector<int> ran_h(ev_it.size(), 1);
        if (!ev_it.empty())
            RCHK(hipMemcpy(ran_h.data(), ran_dev, sizeof(int) * ev_it.size(), hipMemcpyDeviceToHost));
        pb->mem.put(ran_dev);
        for (size_t k = 0; k < ev_it.size(); ++k) {
            if (ran_h[k] != 0) continue;
            float a = 0, b = 0;
            RCHK(hipEventElapsedTime(&a, evs[4 * k + 1], evs[4 * k + 2]));
            RCHK(hipEventElapsedTime(&b, evs[4 * k], evs[4 * k + 3]));
            pb->prof_stencil_ms += a;
            pb->prof_update_ms += b;
            pb->prof_n += 1;
        }
        for (auto e : evs) (void)hipEventDestroy(e);
    }
    return PB_OK;
}

template <typename T>
void vcycle_natural(pb_problem* pb, hipStream_t s, const CGState* st)
{
    MGData* G = pb->mg;
    const RB rb = rb_of(pb->g);
    const GateSpec gs{gmem(st), 3};
    k_rb_convert<T><<<G->nb, 256, 0, s>>>(pb->g, rb, (T*)G->nat_b, (T*)G->cr, 1, gs, nullptr);
    run_vcycle<T>(s, solo_plan(pb), gs);
    k_rb_convert<T><<<G->nb, 256, 0, s>>>(pb->g, rb, (T*)G->nat_x, (T*)G->cz, 0, gs, nullptr);
}

void* natural_buffer(pb_problem* pb, void** slot)
{
    if (!pb->mg) return nullptr;
    if (!*slot) {
        const size_t bytes = (pb->prm.precision == PB_MIXED ? sizeof(float) : sizeof(double)) * (size_t)pb->g.N;
        *slot = pb->mem.get(bytes);
        if (*slot && launch_fill(pb->ctx->stream, *slot, bytes) != hipSuccess) return nullptr;
    }
    return *slot;
}

// ---- a batch of problems (the serving loop) --------------------------------------------------

template <typename T>
int batch_chunk_t(const std::vector<pb_problem*>& pbs, hipStream_t s, int n, MGBatch* bb, CGState* gather,
                  hipEvent_t* ev)
{
    std::vector<const MGData*> Gs;
    for (auto* pb : pbs) Gs.push_back(pb->mg);
    Plan pl;
    std::vector<int> offs;
    plan_tables(Gs, pl, offs);
    const int P = pl.P;
    // the plan's device tables: P descriptor pointers, then the offsets, through pinned staging
    const size_t need = sizeof(void*) * P + sizeof(int) * offs.size();
    if (bb->cap < need) {
        if (bb->host) (void)hipHostFree(bb->host);
        if (bb->dev) bb->free_fn(bb->dev, bb->user);
        bb->host = nullptr;
        bb->dev = nullptr;
        bb->cap = 0;
        const size_t c = std::max<size_t>(need, 16384);
        RCHK(hipHostMalloc(&bb->host, c, hipHostMallocDefault));
        bb->dev = bb->alloc(c, bb->user);
        if (!bb->dev) return pbi_fail(PB_ENOMEM, "multigrid batch tables");
        bb->cap = c;
    }
    char* h = (char*)bb->host;
    for (int p = 0; p < P; ++p) memcpy(h + sizeof(void*) * p, &pbs[p]->mg->dev, sizeof(void*));
    memcpy(h + sizeof(void*) * P, offs.data(), sizeof(int) * offs.size());
    RCHK(hipMemcpyAsync(bb->dev, bb->host, need, hipMemcpyHostToDevice, s));
    pl.desc = bb->dev;
    pl.off = (const int*)((char*)bb->dev + sizeof(void*) * P);
    for (int it = 0; it < n; ++it)
        run_iteration<T>(s, pl, ev ? ev + 6 * it + 2 : nullptr, ev ? ev + 6 * it : nullptr);
    if (gather) kb_gather<T><<<P, 64, 0, s>>>(bt<T>(pl, K_ONE), gather);
    RCHK(hipGetLastError());
    return PB_OK;
}

}  // namespace

int pbi_mg_next_chunk(const CGState& st, int pending, int cap)
{
    int need = cap;
    if (st.goal64 > 0.0 && st.rr > 0.0 && st.rr <= st.goal64) {
        need = 0;
    } else if (st.iter_count > 0 && st.rr > 0.0 && st.rr < st.bnorm2 && st.goal64 > 0.0) {
        const double rate = std::log(st.rr / st.bnorm2) / (double)st.iter_count;   // < 0
        if (rate < -1e-3) need = (int)std::min<double>(cap, std::ceil(std::log(st.goal64 / st.rr) / rate));
    }
    if (st.stop_status == 3) {
        // mixed precision: a residual replacement per delta2 of decrease, the last one
        // confirming convergence, each in an iteration of its own
        int rep = 1;
        if (st.delta2 > 0.0 && st.delta2 < 1.0 && st.goal64 > 0.0 && st.rr > st.goal64)
            rep = std::max(1, (int)std::ceil(std::log(st.goal64 / st.rr) / std::log(st.delta2)));
        need += rep;
    }
    int n = std::min(need - pending, cap);
    if (n < 0) n = 0;
    if (n == 0 && pending == 0) n = 1;   // nothing in flight: keep it moving
    return n;
}

int pbi_mg_solve(pb_problem* pb, CGState* out)
{
    if (pb->prm.precision == PB_MIXED) return solve_t<float>(pb, out);
    return solve_t<double>(pb, out);
}

int pbi_mg_begin(pb_problem* pb, hipStream_t s)
{
    if (pb->prm.precision == PB_MIXED) return begin_t<float>(pb, s);
    return begin_t<double>(pb, s);
}

int pbi_mg_start(pb_problem* pb, hipStream_t s)
{
    if (pb->prm.precision == PB_MIXED) return start_t<float>(pb, s);
    return start_t<double>(pb, s);
}

int pbi_mg_chunk(pb_problem* pb, hipStream_t s, int n, bool first, hipEvent_t* sample)
{
    int rc = PB_OK;
    std::vector<hipEvent_t*> ev((size_t)std::max(n, 1), nullptr);
    ev[0] = sample;
    if (pb->prm.precision == PB_MIXED) {
        if (first) rc = start_t<float>(pb, s);
        if (!rc) rc = chunk_t<float>(pb, s, n, ev.data());
    } else {
        if (first) rc = start_t<double>(pb, s);
        if (!rc) rc = chunk_t<double>(pb, s, n, ev.data());
    }
    return rc;
}

bool pbi_mg_batchable(const pb_problem* pb)
{
    const MGData* G = pb->mg;
    if (!G || G->nlev < 2) return false;
    // a large coarsest level (no one-block part) runs as launches of its own
    return G->ls < G->nlev || interior_count(G->g[G->nlev - 1]) <= kOneBlockCoarse;
}

int pbi_mg_batch_chunk(const std::vector<pb_problem*>& pbs, hipStream_t s, int n, MGBatch* bb, CGState* gather,
                       hipEvent_t* ev)
{
    if (pbs.empty()) return PB_OK;
    const pb_params& P0 = pbs[0]->prm;
    for (auto* pb : pbs) {
        const pb_params& P = pb->prm;
        if (!pbi_mg_batchable(pb) || P.precision != P0.precision || pb->mg->nu != pbs[0]->mg->nu ||
            pb->mg->cs != pbs[0]->mg->cs)
            return pbi_fail(PB_EINVAL, "multigrid batch: problems of different kinds");
    }
    if ((int)pbs.size() > PB_MG_MAX_BATCH) return pbi_fail(PB_EINVAL, "multigrid batch of %d problems", (int)pbs.size());
    if (P0.precision == PB_MIXED) return batch_chunk_t<float>(pbs, s, n, bb, gather, ev);
    return batch_chunk_t<double>(pbs, s, n, bb, gather, ev);
}

int pbi_mg_finish(pb_problem* pb, hipStream_t s)
{
    if (!pb->mg) return PB_OK;
    const Plan pl = solo_plan(pb);
    if (pb->prm.precision == PB_MIXED) {
        using T = float;
        PLAUNCH(K_RB0, 256, kb_rb_fold<T>, 1);
    } else {
        using T = double;
        PLAUNCH(K_RB0, 256, kb_rb_fold<T>, 1);
    }
    RCHK(hipGetLastError());
    return PB_OK;
}

int pbi_mg_levels(const pb_problem* pb) { return pb->mg ? pb->mg->nlev : 0; }

void pbi_mg_vcycle_on(pb_problem* pb, hipStream_t s, const CGState* st)
{
    if (pb->prm.precision == PB_MIXED)
        vcycle_natural<float>(pb, s, st);
    else
        vcycle_natural<double>(pb, s, st);
}

void* pbi_mg_rhs0(pb_problem* pb) { return natural_buffer(pb, &pb->mg->nat_b); }
void* pbi_mg_sol0(pb_problem* pb) { return natural_buffer(pb, &pb->mg->nat_x); }

int pbi_mg_vcycle_test(pb_problem* pb, const double* r_host, double* z_host)
{
    // one V-cycle on a host vector over the padded natural level-0 layout (test hook); the
    // conversion to and from the red-black layout is done here on the host
    hipStream_t s = pb->ctx->stream;
    const Grid& g = pb->g;
    const bool mixed = pb->prm.precision == PB_MIXED;
    int rc = pbi_mg_begin(pb, s);
    if (rc) return rc;
    MGData* G = pb->mg;
    const RB rb = rb_of(g);
    const GateSpec gate{nullptr, 2};
    std::vector<double> r64((size_t)rb.N, 0.0), z64((size_t)rb.N, 0.0);
    for (int i = 1; i < g.nx - 1; ++i)
        for (int j = 1; j < g.ny - 1; ++j)
            for (int k = 1; k < g.nz - 1; ++k) r64[(size_t)rb.idx(i, j, k)] = r_host[g.idx(i, j, k)];
    if (mixed) {
        std::vector<float> tmp((size_t)rb.N);
        for (size_t e = 0; e < tmp.size(); ++e) tmp[e] = (float)r64[e];
        RCHK(hipMemcpyAsync(G->cr, tmp.data(), sizeof(float) * tmp.size(), hipMemcpyHostToDevice, s));
        run_vcycle<float>(s, solo_plan(pb), gate);
        RCHK(hipMemcpyAsync(tmp.data(), G->cz, sizeof(float) * tmp.size(), hipMemcpyDeviceToHost, s));
        RCHK(hipStreamSynchronize(s));
        for (size_t e = 0; e < tmp.size(); ++e) z64[e] = tmp[e];
    } else {
        RCHK(hipMemcpyAsync(G->cr, r64.data(), sizeof(double) * r64.size(), hipMemcpyHostToDevice, s));
        run_vcycle<double>(s, solo_plan(pb), gate);
        RCHK(hipMemcpyAsync(z64.data(), G->cz, sizeof(double) * z64.size(), hipMemcpyDeviceToHost, s));
        RCHK(hipStreamSynchronize(s));
    }
    for (int64_t e = 0; e < g.N; ++e) z_host[e] = 0.0;
    for (int i = 1; i < g.nx - 1; ++i)
        for (int j = 1; j < g.ny - 1; ++j)
            for (int k = 1; k < g.nz - 1; ++k) z_host[g.idx(i, j, k)] = z64[(size_t)rb.idx(i, j, k)];
    RCHK(hipGetLastError());
    return PB_OK;
}
