// pb_mg.hip -- CG preconditioned by one geometric-multigrid V-cycle (uniform grids).
//
// The paper solves with CG and an SSOR preconditioner (Sect. 4).  On a GPU a lexicographic
// SSOR sweep is sequential, so this solver orders the nodes red-black (node (i,j,k) is red
// when i+j+k is even; all neighbours of a red node are black) and uses symmetric red-black
// Gauss-Seidel -- SSOR with omega = 1 in that order -- as the smoother of a V-cycle:
//
//   levels      node I of level l+1 is node 2I of level l, while n-1 is even on every axis
//               (n >= 5); level 0 reads the operator from the node-code map, the coarser
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
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
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

// one level as the kernels see it
template <typename T>
struct Lev {
    Grid g;
    const T *kx, *ky, *kz;   // levels >= 1: K of the +x, +y, +z edges
    const T* diag;           // levels >= 1: diagonal
    const T* dinv;           // 1 / diagonal (every level)
    T* x;                    // iterate (level 0: the CG vector z)
    const T* b;              // right-hand side (level 0: the CG residual r)
};

// the level-0 operator from the node-code map
template <typename T>
struct Op0 {
    const uint32_t* code;
    const T* ck;
    T kin, kout, mass;
};

// sum over the six edges of node e of a coarse level of K * v(neighbour), and optionally
// the diagonal there
template <typename T, typename F>
__device__ __forceinline__ T nsum(const Lev<T>& L, int64_t e, F v, T* D = nullptr)
{
    const Grid& g = L.g;
    const int64_t sx = (int64_t)g.ny * g.S, sy = g.S;
    if (D) *D = L.diag[e];
    return ((L.kx[e - sx] * v(e - sx) + L.kx[e] * v(e + sx)) + (L.ky[e - sy] * v(e - sy) + L.ky[e] * v(e + sy))) +
           (L.kz[e - 1] * v(e - 1) + L.kz[e] * v(e + 1));
}

// Per-node kernels run on a 3-D grid of 256-thread blocks, 64 lanes along z by 4 rows along
// y, each block layer covering kPlanes x-planes (a thread takes the same (j, k) slot in each),
// so that no thread divides to find its node and a launch has few enough blocks that one
// which finds the iteration stopped costs little.  A colour kernel gives lane m the m-th node
// of its colour in the row.
constexpr int kPlanes = 4;

inline dim3 node_grid(const Grid& g, bool colour)
{
    const int nzl = colour ? (g.nz - 1) / 2 : g.nz - 2;   // nodes per interior row
    return dim3((unsigned)std::max(1, (nzl + 63) / 64), (unsigned)((g.ny - 2 + 3) / 4),
                (unsigned)((g.nx - 2 + kPlanes - 1) / kPlanes));
}

// interior node of this thread in plane r of its block layer (all nodes), or -1; red tells
// its colour
__device__ __forceinline__ int64_t this_node(const Grid& g, int r, bool& red)
{
    const int k = 1 + (int)blockIdx.x * 64 + (int)(threadIdx.x & 63);
    const int j = 1 + (int)blockIdx.y * 4 + (int)(threadIdx.x >> 6);
    const int i = 1 + (int)blockIdx.z * kPlanes + r;
    if (k > g.nz - 2 || j > g.ny - 2 || i > g.nx - 2) return -1;
    red = ((i + j + k) & 1) == 0;
    return g.idx(i, j, k);
}

// interior node of colour c (0 red, 1 black) of this thread in plane r of its block layer,
// or -1; with its indices
__device__ __forceinline__ int64_t this_colour_node(const Grid& g, int c, int r, int& i, int& j, int& k)
{
    const int m = (int)blockIdx.x * 64 + (int)(threadIdx.x & 63);
    j = 1 + (int)blockIdx.y * 4 + (int)(threadIdx.x >> 6);
    i = 1 + (int)blockIdx.z * kPlanes + r;
    k = 1 + ((i + j + 1 + c) & 1) + 2 * m;
    if (k > g.nz - 2 || j > g.ny - 2 || i > g.nx - 2) return -1;
    return g.idx(i, j, k);
}

__device__ __forceinline__ int64_t this_colour_node(const Grid& g, int c, int r)
{
    int i, j, k;
    return this_colour_node(g, c, r, i, j, k);
}

// the same for the one-block coarsest solve: node t of colour c in (i, j, m) order
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

// which kernels of a chain run: those of a CG iteration (ru = 0) while the solve is running,
// those of a restart from the true residual (ru = 1) only while one is in progress; with no
// state (a V-cycle applied on its own) always
struct Gate {
    const CGState* st;
    int ru;
};

__device__ __forceinline__ bool halted(const Gate& g) { return g.st && (g.st->status != 0 || g.st->ru != g.ru); }

// the first smoothing step from a zero iterate in one pass: red x = b / D, then black
// x = (b + sum K x_red) / D with the red values formed on the fly
template <typename T>
__global__ void __launch_bounds__(256) k_down1(Lev<T> L, Gate st)
{
    if (halted(st)) return;
    const T* __restrict__ b = L.b;
    const T* __restrict__ dinv = L.dinv;
#pragma unroll
    for (int r = 0; r < kPlanes; ++r) {
        bool red;
        const int64_t e = this_node(L.g, r, red);
        if (e < 0) continue;
        if (red) {
            L.x[e] = b[e] * dinv[e];
        } else {
            const T s = nsum<T>(L, e, [&](int64_t n) { return b[n] * dinv[n]; });
            L.x[e] = (b[e] + s) * dinv[e];
        }
    }
}

// Gauss-Seidel on the nodes of one colour
template <typename T>
__global__ void __launch_bounds__(256) k_sweep(Lev<T> L, int c, Gate st)
{
    if (halted(st)) return;
    const T* __restrict__ x = L.x;
#pragma unroll
    for (int r = 0; r < kPlanes; ++r) {
        const int64_t e = this_colour_node(L.g, c, r);
        if (e < 0) continue;
        const T s = nsum<T>(L, e, [&](int64_t n) { return x[n]; });
        L.x[e] = (L.b[e] + s) * L.dinv[e];
    }
}

// residual b - A x at the red nodes (after a black half-sweep the black residual is zero,
// and the black entries of r stay 0)
template <typename T>
__global__ void __launch_bounds__(256) k_resid(Lev<T> L, T* __restrict__ r, Gate st)
{
    if (halted(st)) return;
    const T* __restrict__ x = L.x;
#pragma unroll
    for (int p = 0; p < kPlanes; ++p) {
        const int64_t e = this_colour_node(L.g, 0, p);
        if (e < 0) continue;
        T D;
        const T s = nsum<T>(L, e, [&](int64_t n) { return x[n]; }, &D);
        r[e] = L.b[e] - (D * x[e] - s);
    }
}

// coarse right-hand side P^T r: fine node 2I and its 12 red neighbours (two odd offsets,
// weight 1/4); the other 14 of the 27 are black, where r is zero
template <typename T>
__global__ void __launch_bounds__(256) k_restrict(Grid gf, const T* __restrict__ r, Grid gc, T* __restrict__ bc,
                                                  Gate st)
{
    if (halted(st)) return;
    const int64_t sx = (int64_t)gf.ny * gf.S, sy = gf.S;
#pragma unroll
    for (int p = 0; p < kPlanes; ++p) {
        bool red;
        const int64_t ec = this_node(gc, p, red);
        if (ec < 0) continue;
        const int K = 1 + (int)blockIdx.x * 64 + (int)(threadIdx.x & 63);
        const int J = 1 + (int)blockIdx.y * 4 + (int)(threadIdx.x >> 6);
        const int I = 1 + (int)blockIdx.z * kPlanes + p;
        const int64_t f = gf.idx(2 * I, 2 * J, 2 * K);
        const T xy = (r[f - sx - sy] + r[f - sx + sy]) + (r[f + sx - sy] + r[f + sx + sy]);
        const T xz = (r[f - sx - 1] + r[f - sx + 1]) + (r[f + sx - 1] + r[f + sx + 1]);
        const T yz = (r[f - sy - 1] + r[f - sy + 1]) + (r[f + sy - 1] + r[f + sy + 1]);
        bc[ec] = r[f] + (T)0.25 * ((xy + xz) + yz);
    }
}

// P e at fine node (i, j, k): trilinear from the coarse corners of its coarse cell
template <typename T>
__device__ __forceinline__ T prolong_at(const Grid& gc, const T* __restrict__ ec, int i, int j, int k)
{
    const int i0 = i >> 1, i1 = (i + 1) >> 1, j0 = j >> 1, j1 = (j + 1) >> 1, k0 = k >> 1, k1 = (k + 1) >> 1;
    const T v = ((ec[gc.idx(i0, j0, k0)] + ec[gc.idx(i0, j0, k1)]) + (ec[gc.idx(i0, j1, k0)] + ec[gc.idx(i0, j1, k1)])) +
                ((ec[gc.idx(i1, j0, k0)] + ec[gc.idx(i1, j0, k1)]) + (ec[gc.idx(i1, j1, k0)] + ec[gc.idx(i1, j1, k1)]));
    return (T)0.125 * v;
}

// x += P e at the red nodes: post-smoothing starts with a black half-sweep, which replaces
// every black value from its red neighbours, so the correction of the black ones is unused
template <typename T>
__global__ void __launch_bounds__(256) k_prolong(Grid gf, T* __restrict__ x, Grid gc, const T* __restrict__ ec,
                                                 Gate st)
{
    if (halted(st)) return;
#pragma unroll
    for (int p = 0; p < kPlanes; ++p) {
        int i, j, k;
        const int64_t e = this_colour_node(gf, 0, p, i, j, k);
        if (e < 0) continue;
        x[e] += prolong_at(gc, ec, i, j, k);
    }
}

// the coarsest level in one block: red from zero, then (black, red) x cs
template <typename T>
__global__ void __launch_bounds__(256) k_coarse(Lev<T> L, int cs, Gate st)
{
    if (halted(st)) return;
    const Grid& g = L.g;
    const int n = (int)interior_count(g), nc = (int)colour_threads(g);
    for (int t = threadIdx.x; t < n; t += 256) {
        bool red;
        const int64_t e = interior_node(g, t, red);
        L.x[e] = red ? L.b[e] * L.dinv[e] : (T)0;
    }
    __syncthreads();
    const T* __restrict__ x = L.x;
    for (int s = 0; s < 2 * cs; ++s) {
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
// V-cycle below the first such level (its right-hand side given) in one launch, with a block
// barrier between phases.  Same steps and order as the multi-launch path.
constexpr int kSubcycleNodes = 8192;
constexpr int kSubThreads = 1024;

template <typename T>
struct SubLevels {
    int nl;                          // levels, the last is the coarsest
    int nu, cs;
    Lev<T> lv[PB_MG_MAX_LEVELS];
    T* r[PB_MG_MAX_LEVELS];
};

template <typename T>
__device__ __forceinline__ void blk_sweep(const Lev<T>& L, int c)
{
    const int nc = (int)colour_threads(L.g);
    const T* __restrict__ x = L.x;
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
__global__ void __launch_bounds__(kSubThreads) k_subcycle(SubLevels<T> S, Gate st)
{
    if (halted(st)) return;
    // down: pre-smoothing, residual at the red nodes, restriction
    for (int l = 0; l + 1 < S.nl; ++l) {
        const Lev<T>& L = S.lv[l];
        blk_red_from_zero(L);
        blk_sweep(L, 1);
        for (int v = 1; v < S.nu; ++v) {
            blk_sweep(L, 0);
            blk_sweep(L, 1);
        }
        const int nc = (int)colour_threads(L.g);
        const T* __restrict__ x = L.x;
        for (int t = threadIdx.x; t < nc; t += kSubThreads) {
            const int64_t e = colour_node(L.g, 0, t);
            if (e < 0) continue;
            T D;
            const T s = nsum<T>(L, e, [&](int64_t m) { return x[m]; }, &D);
            S.r[l][e] = L.b[e] - (D * x[e] - s);
        }
        __syncthreads();
        const Grid& gf = L.g;
        const Grid& gc = S.lv[l + 1].g;
        const T* __restrict__ r = S.r[l];
        T* bc = const_cast<T*>(S.lv[l + 1].b);
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
        const Lev<T>& L = S.lv[S.nl - 1];
        blk_red_from_zero(L);
        for (int v = 0; v < S.cs; ++v) {
            blk_sweep(L, 1);
            blk_sweep(L, 0);
        }
    }
    // up: coarse correction, post-smoothing
    for (int l = S.nl - 2; l >= 0; --l) {
        const Lev<T>& L = S.lv[l];
        const Grid& gc = S.lv[l + 1].g;
        const T* __restrict__ ec = S.lv[l + 1].x;
        const int n = (int)colour_threads(L.g);
        for (int t = threadIdx.x; t < n; t += kSubThreads) {
            const int64_t e = colour_node(L.g, 0, t);   // red nodes only, as in k_prolong
            if (e < 0) continue;
            const int64_t q = e - Z0;
            const int k = (int)(q % L.g.S), j = (int)((q / L.g.S) % L.g.ny), i = (int)(q / ((int64_t)L.g.ny * L.g.S));
            L.x[e] += prolong_at(gc, ec, i, j, k);
        }
        __syncthreads();
        for (int v = 0; v < S.nu; ++v) {
            blk_sweep(L, 1);
            blk_sweep(L, 0);
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

// ---- CG over the level-0 unknowns ----------------------------------------------------------

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

// The search direction is double buffered: an iteration with iter_count = ic reads the old
// direction from buffer ic & 1 and writes the new one to the other (iter_count counts the
// iterations that ran, so a restart between two iterations keeps the pairing).
template <typename T>
__device__ __forceinline__ const T* p_old(const CGState* st, const T* p0, const T* p1)
{
    return (st->iter_count & 1) ? p1 : p0;
}
template <typename T>
__device__ __forceinline__ T* p_new(const CGState* st, T* p0, T* p1)
{
    return (st->iter_count & 1) ? p0 : p1;
}

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
    return r;
}

// the level-0 operator read from the codes in the red-black layout
template <typename T>
struct OpRB {
    const uint32_t* code;
    const T* ck;
    T kin, kout, mass;
};

// element indices of a node and of its six neighbours (x-, x+, y-, y+, z-, z+)
struct RBNb {
    int64_t e, xm, xp, ym, yp, zm, zp;
};

__device__ __forceinline__ RBNb rb_nb(const RB& r, int i, int j, int c, int m, int k)
{
    RBNb n;
    n.e = r.at(i, j, c, m);
    const int64_t eo = r.at(i, j, 1 - c, m);
    const int64_t sx = (int64_t)r.ny * 2 * r.Sh, sy = 2 * (int64_t)r.Sh;
    n.xm = eo - sx;
    n.xp = eo + sx;
    n.ym = eo - sy;
    n.yp = eo + sy;
    n.zm = eo - ((k & 1) ? 0 : 1);
    n.zp = eo + ((k & 1) ? 1 : 0);
    return n;
}

template <typename T>
__device__ __forceinline__ stencil::NodeK<T> rb_k(const OpRB<T>& op, const RBNb& n)
{
    const uint32_t c = op.code[n.e];
    stencil::NodeK<T> k;
    k.xm = stencil::edgeK(op.code[n.xm], 0, op.ck, op.kin, op.kout);
    k.xp = stencil::edgeK(c, 0, op.ck, op.kin, op.kout);
    k.ym = stencil::edgeK(op.code[n.ym], 1, op.ck, op.kin, op.kout);
    k.yp = stencil::edgeK(c, 1, op.ck, op.kin, op.kout);
    k.zm = stencil::edgeK(op.code[n.zm], 2, op.ck, op.kin, op.kout);
    k.zp = stencil::edgeK(c, 2, op.ck, op.kin, op.kout);
    k.m = (c & C_SOLUTE) ? (T)0 : op.mass;
    return k;
}

// sum over the six edges of K * v(neighbour), in the order of the natural-layout kernels
template <typename T, typename F>
__device__ __forceinline__ T rb_sum(const stencil::NodeK<T>& k, const RBNb& n, F v)
{
    return ((k.xm * v(n.xm) + k.xp * v(n.xp)) + (k.ym * v(n.ym) + k.yp * v(n.yp))) + (k.zm * v(n.zm) + k.zp * v(n.zp));
}

// 3-D launch over (position, row, x-plane group): 64 positions by 4 rows per block, kPlanes
// x-planes per thread
inline dim3 rb_grid(const RB& r)
{
    const int mh = (r.nz + 1) / 2;
    return dim3((unsigned)((mh + 63) / 64), (unsigned)((r.ny - 2 + 3) / 4), (unsigned)((r.nx - 2 + kPlanes - 1) / kPlanes));
}

// this thread's row and position in plane p of its block layer; false outside the interior rows
__device__ __forceinline__ bool rb_slot(const RB& r, int p, int& i, int& j, int& m)
{
    m = (int)blockIdx.x * 64 + (int)(threadIdx.x & 63);
    j = 1 + (int)blockIdx.y * 4 + (int)(threadIdx.x >> 6);
    i = 1 + (int)blockIdx.z * kPlanes + p;
    return i <= r.nx - 2 && j <= r.ny - 2;
}

// z index of the node of colour c at position m of row (i, j), or -1 if it is not interior
__device__ __forceinline__ int rb_node(const RB& r, int i, int j, int c, int m)
{
    const int k = 2 * m + ((i + j + c) & 1);
    return (k >= 1 && k <= r.nz - 2) ? k : -1;
}

__device__ __forceinline__ unsigned block_linear() { return (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x; }

// codes in the red-black layout (C_BOX on box and padding positions)
__global__ void __launch_bounds__(256) k_rb_code(Grid g, RB r, const uint32_t* __restrict__ code, uint32_t* __restrict__ out)
{
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < r.N; t += (int64_t)gridDim.x * 256) {
        const int m = (int)(t % r.Sh);
        const int64_t q = t / r.Sh;
        const int c = (int)(q & 1);
        const int64_t row = q >> 1;
        const int j = (int)(row % r.ny), i = (int)(row / r.ny);
        const int k = 2 * m + ((i + j + c) & 1);
        out[t] = k < r.nz ? code[g.idx(i, j, k)] : C_BOX;
    }
}

// 1 / diagonal of the level-0 unknowns in the red-black layout (0 elsewhere)
template <typename T>
__global__ void __launch_bounds__(256) k_rb_diag0(Grid g, RB r, Op0<T> op, T* __restrict__ dinv)
{
#pragma unroll
    for (int p = 0; p < kPlanes; ++p) {
        int i, j, m;
        if (!rb_slot(r, p, i, j, m)) continue;
        for (int c = 0; c < 2; ++c) {
            const int k = rb_node(r, i, j, c, m);
            if (k < 0) continue;
            dinv[r.at(i, j, c, m)] =
                (T)1 / stencil::node_k(g, op.code, op.ck, op.kin, op.kout, op.mass, g.idx(i, j, k)).diag();
        }
    }
}

// level-0 right-hand side b and iterate x (the CG vectors r and z), with 1/D
template <typename T>
struct Lev0 {
    RB r;
    const T* b;
    const T* dinv;
    T* x;
};

// the first smoothing step from a zero iterate: red x = b / D, then black
// x = (b + sum K x_red) / D with the red values formed on the fly
template <typename T>
__global__ void __launch_bounds__(256) k_rb_down1(Lev0<T> L, OpRB<T> op, Gate st)
{
    if (halted(st)) return;
    const T* __restrict__ b = L.b;
    const T* __restrict__ dinv = L.dinv;
#pragma unroll
    for (int p = 0; p < kPlanes; ++p) {
        int i, j, m;
        if (!rb_slot(L.r, p, i, j, m)) continue;
        if (rb_node(L.r, i, j, 0, m) >= 0) {
            const int64_t e = L.r.at(i, j, 0, m);
            L.x[e] = b[e] * dinv[e];
        }
        const int k = rb_node(L.r, i, j, 1, m);
        if (k >= 0) {
            const RBNb n = rb_nb(L.r, i, j, 1, m, k);
            const stencil::NodeK<T> K = rb_k(op, n);
            const T s = rb_sum(K, n, [&](int64_t f) { return b[f] * dinv[f]; });
            L.x[n.e] = (b[n.e] + s) * dinv[n.e];
        }
    }
}

// Gauss-Seidel on the nodes of colour c
template <typename T>
__global__ void __launch_bounds__(256) k_rb_sweep(Lev0<T> L, OpRB<T> op, int c, Gate st)
{
    if (halted(st)) return;
    const T* __restrict__ x = L.x;
#pragma unroll
    for (int p = 0; p < kPlanes; ++p) {
        int i, j, m;
        if (!rb_slot(L.r, p, i, j, m)) continue;
        const int k = rb_node(L.r, i, j, c, m);
        if (k < 0) continue;
        const RBNb n = rb_nb(L.r, i, j, c, m, k);
        const stencil::NodeK<T> K = rb_k(op, n);
        const T s = rb_sum(K, n, [&](int64_t f) { return x[f]; });
        L.x[n.e] = (L.b[n.e] + s) * L.dinv[n.e];
    }
}

// residual b - A x at the red nodes (the black residual is zero right after a black
// half-sweep), in the red segments of rr
template <typename T>
__global__ void __launch_bounds__(256) k_rb_resid(Lev0<T> L, OpRB<T> op, T* __restrict__ rr, Gate st)
{
    if (halted(st)) return;
    const T* __restrict__ x = L.x;
#pragma unroll
    for (int p = 0; p < kPlanes; ++p) {
        int i, j, m;
        if (!rb_slot(L.r, p, i, j, m)) continue;
        const int k = rb_node(L.r, i, j, 0, m);
        if (k < 0) continue;
        const RBNb n = rb_nb(L.r, i, j, 0, m, k);
        const stencil::NodeK<T> K = rb_k(op, n);
        const T s = rb_sum(K, n, [&](int64_t f) { return x[f]; });
        rr[n.e] = L.b[n.e] - (K.diag() * x[n.e] - s);
    }
}

// coarse right-hand side P^T r from the red residual of level 0: fine node 2I and its 12
// red neighbours (two odd offsets, weight 1/4); the other 14 of the 27 are black
template <typename T>
__global__ void __launch_bounds__(256) k_rb_restrict(RB rf, const T* __restrict__ r, Grid gc, T* __restrict__ bc,
                                                     Gate st)
{
    if (halted(st)) return;
#pragma unroll
    for (int p = 0; p < kPlanes; ++p) {
        bool red;
        const int64_t ec = this_node(gc, p, red);
        if (ec < 0) continue;
        const int K = 1 + (int)blockIdx.x * 64 + (int)(threadIdx.x & 63);
        const int J = 1 + (int)blockIdx.y * 4 + (int)(threadIdx.x >> 6);
        const int I = 1 + (int)blockIdx.z * kPlanes + p;
        const int i = 2 * I, j = 2 * J, k = 2 * K;
        auto R = [&](int a, int b, int c) { return r[rf.idx(i + a, j + b, k + c)]; };
        const T xy = (R(-1, -1, 0) + R(-1, 1, 0)) + (R(1, -1, 0) + R(1, 1, 0));
        const T xz = (R(-1, 0, -1) + R(-1, 0, 1)) + (R(1, 0, -1) + R(1, 0, 1));
        const T yz = (R(0, -1, -1) + R(0, -1, 1)) + (R(0, 1, -1) + R(0, 1, 1));
        bc[ec] = R(0, 0, 0) + (T)0.25 * ((xy + xz) + yz);
    }
}

// x += P e at the red nodes of level 0 (the black half-sweep that follows replaces the black ones)
template <typename T>
__global__ void __launch_bounds__(256) k_rb_prolong(RB rf, T* __restrict__ x, Grid gc, const T* __restrict__ ec,
                                                    Gate st)
{
    if (halted(st)) return;
#pragma unroll
    for (int p = 0; p < kPlanes; ++p) {
        int i, j, m;
        if (!rb_slot(rf, p, i, j, m)) continue;
        const int k = rb_node(rf, i, j, 0, m);
        if (k < 0) continue;
        x[rf.at(i, j, 0, m)] += prolong_at(gc, ec, i, j, k);
    }
}

// the last red half-sweep of a V-cycle on level 0 and the partial sums of r.z = b.x over all
// unknowns (the black ones are final after the black half-sweep), one per block
template <typename T>
__global__ void __launch_bounds__(256) k_rb_sweep_dot(Lev0<T> L, OpRB<T> op, Gate st, double* part)
{
    __shared__ double sh[8];
    if (halted(st)) return;
    const T* __restrict__ x = L.x;
    double v[1] = {0.0};
#pragma unroll
    for (int p = 0; p < kPlanes; ++p) {
        int i, j, m;
        if (!rb_slot(L.r, p, i, j, m)) continue;
        const int k = rb_node(L.r, i, j, 0, m);
        if (k >= 0) {
            const RBNb n = rb_nb(L.r, i, j, 0, m, k);
            const stencil::NodeK<T> K = rb_k(op, n);
            const T s = rb_sum(K, n, [&](int64_t f) { return x[f]; });
            const T xn = (L.b[n.e] + s) * L.dinv[n.e];
            L.x[n.e] = xn;
            v[0] += (double)L.b[n.e] * (double)xn;
        }
        if (rb_node(L.r, i, j, 1, m) >= 0) {
            const int64_t eb = L.r.at(i, j, 1, m);
            v[0] += (double)L.b[eb] * (double)x[eb];
        }
    }
    bsum(v, 1, sh);
    if (threadIdx.x == 0) part[block_linear()] = v[0];
}

// the single-level case (no coarser grid): red from zero, black, then (red, black) ... as the
// coarsest level runs, over the red-black level 0
// (k_rb_down1 gives red + black; the sweeps follow on the host side)

// ---- CG over the level-0 unknowns (red-black layout) ---------------------------------------

// p = z + beta p_old and q = A p at both nodes of each position in one pass (the new direction
// at the neighbours is formed on the fly from z and p_old, which box positions hold as 0);
// partial sums of p.q, one per block
template <typename T>
__global__ void __launch_bounds__(256) k_rb_apply(RB r, OpRB<T> op, const T* __restrict__ z, T* p0, T* p1,
                                                  T* __restrict__ q, double* part, const CGState* st)
{
    __shared__ double sh[8];
    if (st->status != 0) return;
    const T* __restrict__ po = p_old(st, (const T*)p0, (const T*)p1);
    T* __restrict__ pn = p_new(st, p0, p1);
    const T beta = (T)st->beta;
    auto pd = [&](int64_t f) { return z[f] + beta * po[f]; };
    double v[1] = {0.0};
#pragma unroll
    for (int p = 0; p < kPlanes; ++p) {
        int i, j, m;
        if (!rb_slot(r, p, i, j, m)) continue;
        for (int c = 0; c < 2; ++c) {
            const int k = rb_node(r, i, j, c, m);
            if (k < 0) continue;
            const RBNb n = rb_nb(r, i, j, c, m, k);
            const stencil::NodeK<T> K = rb_k(op, n);
            const T pe = pd(n.e);
            const T qe = K.diag() * pe - rb_sum(K, n, pd);
            pn[n.e] = pe;
            q[n.e] = qe;
            v[0] += (double)pe * (double)qe;
        }
    }
    bsum(v, 1, sh);
    if (threadIdx.x == 0) part[block_linear()] = v[0];
}

// x += alpha p, r -= alpha q over every element (box and padding positions hold 0 in p, q and
// r); partial sums of r.r (after the nb slots of the p.q sums)
template <typename T>
__global__ void __launch_bounds__(256) k_rb_update(int64_t N, T* __restrict__ x, T* __restrict__ r, T* p0, T* p1,
                                                   const T* __restrict__ q, double* part, int nb, const CGState* st)
{
    __shared__ double sh[8];
    if (st->status != 0) return;
    const T* __restrict__ p = p_new(st, p0, p1);
    const T a = (T)st->alpha;
    double v[1] = {0.0};
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < N; e += (int64_t)gridDim.x * 256) {
        x[e] += a * p[e];
        const T rv = r[e] - a * q[e];
        r[e] = rv;
        v[0] += (double)rv * (double)rv;
    }
    bsum(v, 1, sh);
    if (threadIdx.x == 0) part[nb + blockIdx.x] = v[0];
}

// partial sums of r.z over every element
template <typename T>
__global__ void __launch_bounds__(256) k_rb_dot(int64_t N, const T* __restrict__ r, const T* __restrict__ z,
                                                double* part, Gate st)
{
    __shared__ double sh[8];
    if (halted(st)) return;
    double v[1] = {0.0};
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < N; e += (int64_t)gridDim.x * 256)
        v[0] += (double)r[e] * (double)z[e];
    bsum(v, 1, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// the FP64 solution (natural layout) += the correction in the red-black layout, which is then
// cleared
template <typename T>
__global__ void __launch_bounds__(256) k_rb_fold(Grid g, RB r, double* __restrict__ x64, T* __restrict__ xc,
                                                 const CGState* st, int force)
{
    if (!force && st->status != 3) return;
#pragma unroll
    for (int p = 0; p < kPlanes; ++p) {
        int i, j, m;
        if (!rb_slot(r, p, i, j, m)) continue;
        for (int c = 0; c < 2; ++c) {
            const int k = rb_node(r, i, j, c, m);
            if (k < 0) continue;
            const int64_t e = r.at(i, j, c, m);
            x64[g.idx(i, j, k)] += (double)xc[e];
            xc[e] = (T)0;
        }
    }
}

// r = b - A x in FP64 from the natural-layout solution, right-hand side and codes, stored in
// the element type in the red-black layout; partial sums of the FP64 r.r in the third slot
// range, one per block
template <typename T>
__global__ void __launch_bounds__(256) k_rb_true_res(Grid g, RB r, Op0<double> op, const double* __restrict__ x,
                                                     const double* __restrict__ b, T* __restrict__ res, double* part,
                                                     int nb, const CGState* st, int force)
{
    __shared__ double sh[8];
    if (!force && st->status != 3) return;
    const int64_t sx = (int64_t)g.ny * g.S, sy = g.S;
    double v[1] = {0.0};
#pragma unroll
    for (int p = 0; p < kPlanes; ++p) {
        int i, j, m;
        if (!rb_slot(r, p, i, j, m)) continue;
        for (int c = 0; c < 2; ++c) {
            const int k = rb_node(r, i, j, c, m);
            if (k < 0) continue;
            const int64_t e = g.idx(i, j, k);
            const stencil::NodeK<double> K = stencil::node_k(g, op.code, op.ck, op.kin, op.kout, op.mass, e);
            const double s = ((K.xm * x[e - sx] + K.xp * x[e + sx]) + (K.ym * x[e - sy] + K.yp * x[e + sy])) +
                             (K.zm * x[e - 1] + K.zp * x[e + 1]);
            const double rv = b[e] - (K.diag() * x[e] - s);
            res[r.at(i, j, c, m)] = (T)rv;
            v[0] += rv * rv;
        }
    }
    bsum(v, 1, sh);
    if (threadIdx.x == 0) part[2 * nb + block_linear()] = v[0];
}

// natural-layout level-0 vector <-> red-black layout (interior nodes; the two-level
// preconditioner of refined grids hands its coarse right-hand side over in the natural layout)
template <typename T>
__global__ void __launch_bounds__(256) k_rb_convert(Grid g, RB r, T* __restrict__ nat, T* __restrict__ rbv, int to_rb,
                                                    Gate st)
{
    if (halted(st)) return;
#pragma unroll
    for (int p = 0; p < kPlanes; ++p) {
        int i, j, m;
        if (!rb_slot(r, p, i, j, m)) continue;
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

__global__ void __launch_bounds__(256) k_alpha(const double* part, int nb, CGState* st)
{
    __shared__ double sh[8];
    if (st->status != 0) return;
    double v[1] = {0.0};
    for (int t = threadIdx.x; t < nb; t += 256) v[0] += part[t];
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
// update that the stopped step skipped takes beta = r'.z' / (r.z of the step before)
// The r.z partials are prz[0 .. nrz) (those of the fused last half-sweep), or part[0 .. nb).
__global__ void __launch_bounds__(256) k_beta(const double* part, int nb, CGState* st, int mode,
                                              const double* prz, int nrz)
{
    __shared__ double sh[8];
    if (st->status != 0 || st->ru != (mode == 0 ? 0 : 1)) return;
    if (!prz) {
        prz = part;
        nrz = nb;
    }
    double v[2] = {0.0, 0.0};
    for (int t = threadIdx.x; t < nrz; t += 256) v[0] += prz[t];
    if (mode == 0)
        for (int t = threadIdx.x; t < nb; t += 256) v[1] += part[nb + t];
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
__global__ void __launch_bounds__(256) k_ru_fin(const double* part, int nb, CGState* st, int init, int mixed,
                                                double rtol2, double delta2, int force)
{
    __shared__ double sh[8];
    if (!force && st->status != 3) return;
    double v[1] = {0.0};
    for (int t = threadIdx.x; t < nb; t += 256) v[0] += part[2 * nb + t];
    bsum(v, 1, sh);
    if (threadIdx.x == 0) {
        const double rr64 = v[0];
        if (init) {
            st->alpha = st->beta = st->gamma = st->pq = 0.0;
            st->bnorm2 = rr64;
            st->goal64 = rtol2 * rr64;
            st->stop2 = rtol2 * rr64;
            st->delta2 = mixed ? delta2 : 0.0;
            st->stop_status = mixed ? 3 : 1;
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
Lev<T> level(const MGData* G, int l)
{
    Lev<T> L;
    L.g = G->g[l];
    L.kx = (const T*)G->K[l][0];
    L.ky = (const T*)G->K[l][1];
    L.kz = (const T*)G->K[l][2];
    L.diag = (const T*)G->diag[l];
    L.dinv = (const T*)G->dinv[l];
    L.x = (T*)G->x[l];
    L.b = (const T*)G->b[l];
    return L;
}

template <typename T>
Op0<T> op0(const pb_problem* pb)
{
    Op0<T> o;
    o.code = pb->code;
    if constexpr (sizeof(T) == 8)
        o.ck = (const T*)pb->ck64;
    else
        o.ck = (const T*)pb->ck32;
    o.kin = (T)pb->cf.kin;
    o.kout = (T)pb->cf.kout;
    o.mass = (T)pb->cf.mass;
    return o;
}

// ---- launches on the coarse levels (natural layout) --------------------------------------

template <typename T>
void launch_sweep(hipStream_t s, const Lev<T>& L, int c, Gate st)
{
    if (colour_threads(L.g) > 0) k_sweep<T><<<node_grid(L.g, true), 256, 0, s>>>(L, c, st);
}

// pre-smoothing (red, black) x nu from zero
template <typename T>
void launch_pre(hipStream_t s, int nu, const Lev<T>& L, Gate st)
{
    k_down1<T><<<node_grid(L.g, false), 256, 0, s>>>(L, st);
    for (int v = 1; v < nu; ++v) {
        launch_sweep<T>(s, L, 0, st);
        launch_sweep<T>(s, L, 1, st);
    }
}

// coarse correction and post-smoothing (black, red) x nu
template <typename T>
void launch_post(hipStream_t s, int nu, const Lev<T>& L, const Grid& gc, const T* ec, Gate st)
{
    k_prolong<T><<<node_grid(L.g, true), 256, 0, s>>>(L.g, L.x, gc, ec, st);
    for (int v = 0; v < nu; ++v) {
        launch_sweep<T>(s, L, 1, st);
        launch_sweep<T>(s, L, 0, st);
    }
}

template <typename T>
void launch_coarsest(hipStream_t s, const MGData* G, const Lev<T>& L, Gate st)
{
    if (interior_count(L.g) <= kOneBlockCoarse) {
        k_coarse<T><<<1, 256, 0, s>>>(L, G->cs, st);
        return;
    }
    // red, black in one pass, then red, then (black, red) x (cs - 1)
    launch_pre<T>(s, 1, L, st);
    launch_sweep<T>(s, L, 0, st);
    for (int v = 1; v < G->cs; ++v) {
        launch_sweep<T>(s, L, 1, st);
        launch_sweep<T>(s, L, 0, st);
    }
}

// ---- launches on level 0 (red-black layout) ------------------------------------------------

template <typename T>
OpRB<T> oprb(const pb_problem* pb)
{
    const Op0<T> o = op0<T>(pb);
    return OpRB<T>{pb->mg->code_rb, o.ck, o.kin, o.kout, o.mass};
}

template <typename T>
Lev0<T> lev0(const pb_problem* pb)
{
    const MGData* G = pb->mg;
    return Lev0<T>{rb_of(pb->g), (const T*)G->cr, (const T*)G->dinv[0], (T*)G->cz};
}

template <typename T>
void launch_rb_sweep(hipStream_t s, const Lev0<T>& L, const OpRB<T>& op, int c, Gate st)
{
    k_rb_sweep<T><<<rb_grid(L.r), 256, 0, s>>>(L, op, c, st);
}

// z = V-cycle(r) at level 0 (x of level 0 is z, b of level 0 is r); with ev, events around
// the whole V-cycle (ev[0], ev[3]) and around the first level-0 black half-sweep after the
// coarse correction (ev[1], ev[2]).  With more than one level the last half-sweep also writes
// the r.z partial sums to G->prz (G->nrz blocks); returns whether it did.
template <typename T>
bool launch_vcycle(hipStream_t s, const pb_problem* pb, Gate st, hipEvent_t* ev = nullptr)
{
    const MGData* G = pb->mg;
    const OpRB<T> op = oprb<T>(pb);
    const Lev0<T> L0 = lev0<T>(pb);
    const dim3 grid0 = rb_grid(L0.r);
    const int L = G->nlev;
    if (L == 1) {
        // one level: red from zero and black, then red, then (black, red) x (cs - 1)
        k_rb_down1<T><<<grid0, 256, 0, s>>>(L0, op, st);
        launch_rb_sweep<T>(s, L0, op, 0, st);
        for (int v = 1; v < G->cs; ++v) {
            launch_rb_sweep<T>(s, L0, op, 1, st);
            launch_rb_sweep<T>(s, L0, op, 0, st);
        }
        return false;
    }
    if (ev) (void)hipEventRecord(ev[0], s);
    // level 0: pre-smoothing, red residual, restriction to level 1
    k_rb_down1<T><<<grid0, 256, 0, s>>>(L0, op, st);
    for (int v = 1; v < G->nu; ++v) {
        launch_rb_sweep<T>(s, L0, op, 0, st);
        launch_rb_sweep<T>(s, L0, op, 1, st);
    }
    k_rb_resid<T><<<grid0, 256, 0, s>>>(L0, op, (T*)G->r[0], st);
    k_rb_restrict<T><<<node_grid(G->g[1], false), 256, 0, s>>>(L0.r, (const T*)G->r[0], G->g[1], (T*)G->b[1], st);
    // the first level from which every level has at most kSubcycleNodes unknowns (not 0)
    int ls = L;
    while (ls - 1 >= 1 && interior_count(G->g[ls - 1]) <= kSubcycleNodes) --ls;
    // pre-smoothing and restriction on the coarse levels above the one-block part (or above
    // the coarsest level)
    for (int l = 1; l < std::min(ls, L - 1); ++l) {
        const Lev<T> lv = level<T>(G, l);
        const Grid& gc = G->g[l + 1];
        T* r = (T*)G->r[l];
        launch_pre<T>(s, G->nu, lv, st);
        k_resid<T><<<node_grid(lv.g, true), 256, 0, s>>>(lv, r, st);
        k_restrict<T><<<node_grid(gc, false), 256, 0, s>>>(lv.g, r, gc, (T*)G->b[l + 1], st);
    }
    if (ls < L) {
        // levels ls.. in one block; its right-hand side was restricted above
        SubLevels<T> S;
        S.nl = L - ls;
        S.nu = G->nu;
        S.cs = G->cs;
        for (int l = ls; l < L; ++l) {
            S.lv[l - ls] = level<T>(G, l);
            S.r[l - ls] = (T*)G->r[l];
        }
        k_subcycle<T><<<1, kSubThreads, 0, s>>>(S, st);
    } else {
        launch_coarsest<T>(s, G, level<T>(G, L - 1), st);
    }
    for (int l = std::min(ls, L - 1) - 1; l >= 1; --l)
        launch_post<T>(s, G->nu, level<T>(G, l), G->g[l + 1], (const T*)G->x[l + 1], st);
    // level 0: coarse correction at the red nodes, post-smoothing; the last red half-sweep
    // also forms the r.z partial sums
    k_rb_prolong<T><<<grid0, 256, 0, s>>>(L0.r, L0.x, G->g[1], (const T*)G->x[1], st);
    if (ev) (void)hipEventRecord(ev[1], s);
    for (int v = 0; v < G->nu; ++v) {
        launch_rb_sweep<T>(s, L0, op, 1, st);
        if (v == 0 && ev) (void)hipEventRecord(ev[2], s);
        if (v == G->nu - 1)
            k_rb_sweep_dot<T><<<grid0, 256, 0, s>>>(L0, op, st, G->prz);
        else
            launch_rb_sweep<T>(s, L0, op, 0, st);
    }
    if (ev) (void)hipEventRecord(ev[3], s);
    return true;
}

// the level hierarchy and the solver vectors, enqueued on stream s (no host wait); the FP64
// coefficients the element-type copies are rounded from stay allocated with the problem
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
    // FP64 coefficients of every coarse level, then the element-type copies
    std::vector<double*> tmp;
    auto get64 = [&](int64_t n) -> double* {
        double* p = (double*)pb->mem.get(sizeof(double) * (size_t)n);
        if (p) tmp.push_back(p);
        return p;
    };
    const double *pkx = nullptr, *pky = nullptr, *pkz = nullptr, *pm = nullptr;
    for (int l = 1; l < G->nlev; ++l) {
        const Grid& gc = G->g[l];
        double *kx = get64(gc.N), *ky = get64(gc.N), *kz = get64(gc.N), *m = get64(gc.N);
        if (!kx || !ky || !kz || !m) return pbi_fail(PB_ENOMEM, "multigrid levels");
        RCHK(launch_fill(s, kx, sizeof(double) * (size_t)gc.N));
        RCHK(launch_fill(s, ky, sizeof(double) * (size_t)gc.N));
        RCHK(launch_fill(s, kz, sizeof(double) * (size_t)gc.N));
        RCHK(launch_fill(s, m, sizeof(double) * (size_t)gc.N));
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
        T* kT[3];
        for (int d = 0; d < 3; ++d) {
            kT[d] = (T*)pb->mem.get(sizeof(T) * (size_t)gc.N);
            if (!kT[d]) return pbi_fail(PB_ENOMEM, "multigrid levels");
            RCHK(launch_fill(s, kT[d], sizeof(T) * (size_t)gc.N));
            G->K[l][d] = kT[d];
        }
        T* dT = (T*)pb->mem.get(sizeof(T) * (size_t)gc.N);
        T* DT = (T*)pb->mem.get(sizeof(T) * (size_t)gc.N);
        if (!dT || !DT) return pbi_fail(PB_ENOMEM, "multigrid levels");
        RCHK(launch_fill(s, dT, sizeof(T) * (size_t)gc.N));
        RCHK(launch_fill(s, DT, sizeof(T) * (size_t)gc.N));
        G->dinv[l] = dT;
        G->diag[l] = DT;
        k_level_diag<T><<<nblk(nn, 256), 256, 0, s>>>(gc, kx, ky, kz, m, kT[0], kT[1], kT[2], DT, dT);
        RCHK(hipGetLastError());
        pkx = kx;
        pky = ky;
        pkz = kz;
        pm = m;
    }
    // coarse-level vectors (natural layout)
    for (int l = 1; l < G->nlev; ++l) {
        const Grid& g = G->g[l];
        void** dst[3] = {&G->r[l], &G->x[l], &G->b[l]};
        for (int v = 0; v < 3; ++v) {
            *dst[v] = pb->mem.get(sizeof(T) * (size_t)g.N);
            if (!*dst[v]) return pbi_fail(PB_ENOMEM, "multigrid vectors");
            RCHK(launch_fill(s, *dst[v], sizeof(T) * (size_t)g.N));
        }
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
    void** v0[8] = {&G->dinv[0], &G->r[0], &G->cr, &G->cz, &G->cp, &G->cp2, &G->cq, &G->cx};
    for (int v = 0; v < 8; ++v) {
        *v0[v] = pb->mem.get(sizeof(T) * (size_t)rb.N);
        if (!*v0[v]) return pbi_fail(PB_ENOMEM, "multigrid level-0 vectors");
        RCHK(launch_fill(s, *v0[v], sizeof(T) * (size_t)rb.N));
    }
    k_rb_diag0<T><<<rb_grid(rb), 256, 0, s>>>(g0, rb, op0<T>(pb), (T*)G->dinv[0]);
    G->x[0] = G->cz;
    G->b[0] = G->cr;
    {
        // one partial sum per block of the level-0 launches; the streaming kernels use as many
        const dim3 ng = rb_grid(rb);
        G->nb = (int)(ng.x * ng.y * ng.z);
        G->nrz = G->nb;
    }
    G->part = (double*)pb->mem.get(sizeof(double) * 3 * (size_t)G->nb);
    if (!G->part) return pbi_fail(PB_ENOMEM, "multigrid partial sums");
    G->prz = (double*)pb->mem.get(sizeof(double) * (size_t)G->nrz);
    if (!G->prz) return pbi_fail(PB_ENOMEM, "multigrid partial sums");
    RCHK(hipGetLastError());
    return PB_OK;
}

template <typename T>
void launch_iteration(hipStream_t s, const pb_problem* pb, CGState* st, hipEvent_t* ev = nullptr)
{
    const MGData* G = pb->mg;
    const RB rb = rb_of(pb->g);
    T *x = (T*)G->cx, *r = (T*)G->cr, *z = (T*)G->cz, *p0 = (T*)G->cp, *p1 = (T*)G->cp2, *q = (T*)G->cq;
    const Gate gate{st, 0};
    k_rb_apply<T><<<rb_grid(rb), 256, 0, s>>>(rb, oprb<T>(pb), z, p0, p1, q, G->part, st);
    k_alpha<<<1, 256, 0, s>>>(G->part, G->nb, st);
    k_rb_update<T><<<G->nb, 256, 0, s>>>(rb.N, x, r, p0, p1, q, G->part, G->nb, st);
    const bool fused = launch_vcycle<T>(s, pb, gate, ev);
    if (!fused) k_rb_dot<T><<<G->nb, 256, 0, s>>>(rb.N, r, z, G->part, gate);
    k_beta<<<1, 256, 0, s>>>(G->part, G->nb, st, 0, fused ? G->prz : nullptr, G->nrz);
}

// restart from the true residual: fold the correction into the FP64 solution, r = b - A x in
// FP64, then z = V-cycle(r), r.z and beta.  With force it runs whatever the state (init: the
// first residual, x = 0); otherwise only where the iteration stopped with status 3 (the FP32
// residual reached its goal or fell by inner_rtol).
template <typename T>
void launch_restart(hipStream_t s, pb_problem* pb, CGState* st, int init, int force)
{
    const MGData* G = pb->mg;
    const Grid& g = pb->g;
    const RB rb = rb_of(g);
    const pb_params& P = pb->prm;
    const bool mixed = sizeof(T) == 4;
    k_rb_fold<T><<<rb_grid(rb), 256, 0, s>>>(g, rb, pb->x, (T*)G->cx, st, force);
    const Op0<double> op64 = op0<double>(pb);
    k_rb_true_res<T><<<rb_grid(rb), 256, 0, s>>>(g, rb, op64, pb->x, pb->rhs, (T*)G->cr, G->part, G->nb, st, force);
    k_ru_fin<<<1, 256, 0, s>>>(G->part, G->nb, st, init, mixed ? 1 : 0, P.rtol * P.rtol, P.inner_rtol * P.inner_rtol,
                               force);
    const Gate gate{st, 1};
    const bool fused = launch_vcycle<T>(s, pb, gate);
    if (!fused) k_rb_dot<T><<<G->nb, 256, 0, s>>>(rb.N, (const T*)G->cr, (const T*)G->cz, G->part, gate);
    k_beta<<<1, 256, 0, s>>>(G->part, G->nb, st, init ? 1 : 2, fused ? G->prz : nullptr, G->nrz);
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
    launch_restart<T>(s, pb, pb->st, 1, 1);
    RCHK(hipGetLastError());
    return PB_OK;
}

// n iterations and the restart that follows them where one is due, enqueued on s; ev[it],
// where given, receives the four timing events of iteration it's V-cycle
// (ran[it], where given: receives the state's status as iteration it starts; 0 means the
// iteration runs, short of a breakdown in its alpha step: only its scalar steps change it)
template <typename T>
int chunk_t(pb_problem* pb, hipStream_t s, int n, hipEvent_t* const* ev, int* const* ran = nullptr)
{
    for (int it = 0; it < n; ++it) {
        if (ran && ran[it]) RCHK(hipMemcpyAsync(ran[it], &pb->st->status, sizeof(int), hipMemcpyDeviceToDevice, s));
        launch_iteration<T>(s, pb, pb->st, ev ? ev[it] : nullptr);
    }
    if (sizeof(T) == 4) launch_restart<T>(s, pb, pb->st, 0, 0);
    RCHK(hipGetLastError());
    return PB_OK;
}

// Pipelined like the Jacobi solve: chunks of iterations (each followed by the restart where
// one is due) are enqueued while the state of the previous chunk is read back.
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
    int launched = 0, c = 0;
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
    auto enqueue = [&](int slot) -> int {
        const int n = std::min(M, P.max_iter - launched);
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
    if ((rc = enqueue(0))) return rc;
    for (;;) {
        const bool more = launched < P.max_iter;
        if (more && (rc = enqueue((c + 1) & 1))) return rc;
        RCHK(hipEventSynchronize(ctx->ev[c & 1]));
        const CGState snap = ctx->host_state[c & 1];
        if (snap.status == 1 || snap.status == 2 || !more) break;
        ++c;
    }
    // the correction into the FP64 solution (all of it in FP64; in the mixed form what is left
    // after the last restart)
    {
        const RB rb = rb_of(pb->g);
        k_rb_fold<T><<<rb_grid(rb), 256, 0, s>>>(pb->g, rb, pb->x, (T*)pb->mg->cx, pb->st, 1);
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

}  // namespace

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

int pbi_mg_finish(pb_problem* pb, hipStream_t s)
{
    if (!pb->mg) return PB_OK;
    const RB rb = rb_of(pb->g);
    if (pb->prm.precision == PB_MIXED)
        k_rb_fold<float><<<rb_grid(rb), 256, 0, s>>>(pb->g, rb, pb->x, (float*)pb->mg->cx, pb->st, 1);
    else
        k_rb_fold<double><<<rb_grid(rb), 256, 0, s>>>(pb->g, rb, pb->x, (double*)pb->mg->cx, pb->st, 1);
    RCHK(hipGetLastError());
    return PB_OK;
}

int pbi_mg_levels(const pb_problem* pb) { return pb->mg ? pb->mg->nlev : 0; }

namespace {

template <typename T>
void vcycle_natural(pb_problem* pb, hipStream_t s, const CGState* st)
{
    MGData* G = pb->mg;
    const RB rb = rb_of(pb->g);
    const Gate gate{st, 0};
    k_rb_convert<T><<<rb_grid(rb), 256, 0, s>>>(pb->g, rb, (T*)G->nat_b, (T*)G->cr, 1, gate);
    launch_vcycle<T>(s, pb, gate);
    k_rb_convert<T><<<rb_grid(rb), 256, 0, s>>>(pb->g, rb, (T*)G->nat_x, (T*)G->cz, 0, gate);
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

}  // namespace

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
    const Gate gate{nullptr, 0};
    std::vector<double> r64((size_t)rb.N, 0.0), z64((size_t)rb.N, 0.0);
    for (int i = 1; i < g.nx - 1; ++i)
        for (int j = 1; j < g.ny - 1; ++j)
            for (int k = 1; k < g.nz - 1; ++k) r64[(size_t)rb.idx(i, j, k)] = r_host[g.idx(i, j, k)];
    if (mixed) {
        std::vector<float> tmp((size_t)rb.N);
        for (size_t e = 0; e < tmp.size(); ++e) tmp[e] = (float)r64[e];
        RCHK(hipMemcpyAsync(G->cr, tmp.data(), sizeof(float) * tmp.size(), hipMemcpyHostToDevice, s));
        launch_vcycle<float>(s, pb, gate);
        RCHK(hipMemcpyAsync(tmp.data(), G->cz, sizeof(float) * tmp.size(), hipMemcpyDeviceToHost, s));
        RCHK(hipStreamSynchronize(s));
        for (size_t e = 0; e < tmp.size(); ++e) z64[e] = tmp[e];
    } else {
        RCHK(hipMemcpyAsync(G->cr, r64.data(), sizeof(double) * r64.size(), hipMemcpyHostToDevice, s));
        launch_vcycle<double>(s, pb, gate);
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
