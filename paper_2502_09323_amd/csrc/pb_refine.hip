// pb_refine.hip -- one level of 2:1 local refinement with hanging nodes.
//
// The paper computes on a Cartesian octree with hierarchical refinement and handles its
// non-conforming (hanging) nodes as in its references (Sect. 3, before Sect. 3.1); the
// condensed operator of Sect. 3.1 is assembled cell by cell, every cell of size s adding
// (s/4) eps_e per edge and (s^3/8) kbar^2 per vertex.  This file builds and solves that
// operator for coarse cells of size H, some of which are split into 2x2x2 fine cells of size
// h = H/2:
//
//   refinement  a coarse cell is split when a crossing point of the surface with the fine
//               lattice lies within delta of it; the flags are rounded up to aligned bricks
//   grids       the coarse grid (all coarse nodes) and a fine sub-lattice covering the
//               refined bricks, each with explicit per-node coefficients: K of the +x, +y,
//               +z edges (the number of incident cells of that grid times s/4 eps_e) and the
//               lumped ionic term (incident cells times s^3/8 kbar^2)
//   unknowns    coarse nodes with an unrefined incident cell; fine nodes with a refined
//               incident cell, except those that coincide with a coarse unknown and the
//               hanging nodes (not coarse nodes, on the boundary of an unrefined coarse cell),
//               which take the mean of the 2 or 4 coarse nodes of the coarse edge or face
//               they lie on
//   operator    A = P^T K P: fill the derived fine values from the coarse ones (P), apply
//               each grid's cell contributions, and add the rows of the derived fine nodes
//               back to their coarse nodes (P^T)
//
// The solve is Jacobi-preconditioned CG over the unknowns of both grids (the diagonal of K
// at each unknown), with device-resident scalars and fixed-order reductions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "pb_host.h"
#include "pb_internal.h"
#include "pb_stencil.h"

using namespace pbk;

namespace {

constexpr double kPi = 3.14159265358979323846;

#define RCHK(expr)                                                                        \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return pbi_fail(PB_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));   \
    } while (0)

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

__device__ __forceinline__ void decode(const Grid& g, int64_t e, int& i, int& j, int& k)
{
    const int64_t row = e / g.S;
    k = (int)(e - row * g.S) - Z0;
    j = (int)(row % g.ny);
    i = (int)(row / g.ny);
}

struct Cells {             // refinement flags of the coarse cells
    const uint8_t* f;
    int nc[3];
    __device__ bool refined(int i, int j, int k) const
    {
        return f[((int64_t)i * nc[1] + j) * nc[2] + k] != 0;
    }
    __device__ bool valid(int i, int j, int k) const
    {
        return i >= 0 && j >= 0 && k >= 0 && i < nc[0] && j < nc[1] && k < nc[2];
    }
};

// ---- refinement rule ---------------------------------------------------------------------

// every coarse cell within delta of a crossing point is flagged (all writers store 1)
// de-refinement toward the box: a coarse cell is flagged when it meets the box
// [lo - delta, hi + delta] (the solute's extent widened by delta) on all three axes
__global__ void __launch_bounds__(256) k_mark_box(Grid gc, double lox, double loy, double loz, double hix, double hiy,
                                                  double hiz, double delta, uint8_t* flag, int nc0, int nc1, int nc2)
{
#pragma clang fp contract(off)
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t n = (int64_t)nc0 * nc1 * nc2;
    if (t >= n) return;
    const int k = (int)(t % nc2), j = (int)((t / nc2) % nc1), i = (int)(t / ((int64_t)nc2 * nc1));
    const int c[3] = {i, j, k};
    const double org[3] = {gc.ox, gc.oy, gc.oz}, lo[3] = {lox, loy, loz}, hi[3] = {hix, hiy, hiz};
    bool in = true;
    for (int d = 0; d < 3; ++d) {
        const double blo = org[d] + gc.h * (double)c[d];
        const double bhi = org[d] + gc.h * (double)(c[d] + 1);
        in = in && bhi >= lo[d] - delta && blo <= hi[d] + delta;
    }
    flag[t] = in ? 1 : 0;
}

__global__ void __launch_bounds__(256) k_mark(Grid gc, int64_t ncut, const double* __restrict__ rp, double delta,
                                              uint8_t* flag, int nc0, int nc1, int nc2)
{
#pragma clang fp contract(off)
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= ncut) return;
    const double org[3] = {gc.ox, gc.oy, gc.oz};
    const int nc[3] = {nc0, nc1, nc2};
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        const double a = floor((rp[3 * p + d] - delta - org[d]) / gc.h) - 1.0;
        const double b = floor((rp[3 * p + d] + delta - org[d]) / gc.h) + 1.0;
        lo[d] = a < 0.0 ? 0 : (int)a;
        hi[d] = b > (double)(nc[d] - 1) ? nc[d] - 1 : (int)b;
    }
    const double d2max = delta * delta;
    for (int i = lo[0]; i <= hi[0]; ++i)
        for (int j = lo[1]; j <= hi[1]; ++j)
            for (int k = lo[2]; k <= hi[2]; ++k) {
                const int c[3] = {i, j, k};
                double dd[3];
                for (int d = 0; d < 3; ++d) {
                    const double blo = org[d] + gc.h * (double)c[d];
                    const double bhi = org[d] + gc.h * (double)(c[d] + 1);
                    const double x = rp[3 * p + d];
                    const double e = blo - x > x - bhi ? blo - x : x - bhi;
                    dd[d] = e > 0.0 ? e : 0.0;
                }
                const double d2 = (dd[0] * dd[0] + dd[1] * dd[1]) + dd[2] * dd[2];
                if (d2 <= d2max) flag[((int64_t)i * nc1 + j) * nc2 + k] = 1;
            }
}

// brick flags: a brick is refined when any of its cells is flagged
__global__ void __launch_bounds__(256) k_bricks(const uint8_t* flag, int nc0, int nc1, int nc2, int B, int nb0,
                                                int nb1, int nb2, uint8_t* bf)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (int64_t)nb0 * nb1 * nb2) return;
    const int bk = (int)(t % nb2), bj = (int)((t / nb2) % nb1), bi = (int)(t / ((int64_t)nb1 * nb2));
    uint8_t r = 0;
    for (int i = bi * B; i < min((bi + 1) * B, nc0) && !r; ++i)
        for (int j = bj * B; j < min((bj + 1) * B, nc1) && !r; ++j)
            for (int k = bk * B; k < min((bk + 1) * B, nc2) && !r; ++k)
                r |= flag[((int64_t)i * nc1 + j) * nc2 + k];
    bf[t] = r;
}

__global__ void __launch_bounds__(256) k_cells_from_bricks(const uint8_t* bf, int nc0, int nc1, int nc2, int B,
                                                           int nb1, int nb2, uint8_t* cell)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (int64_t)nc0 * nc1 * nc2) return;
    const int k = (int)(t % nc2), j = (int)((t / nc2) % nc1), i = (int)(t / ((int64_t)nc1 * nc2));
    cell[t] = bf[((int64_t)(i / B) * nb1 + j / B) * nb2 + k / B];
}

// ---- coefficients ------------------------------------------------------------------------

__device__ __forceinline__ double edgeK(uint32_t c, int ax, const double* ck, const Coef& cf)
{
    return stencil::edgeK(c, ax, ck, cf.kin, cf.kout);
}

// coarse grid: K of the +axis edges and the lumped term from the unrefined incident cells;
// role 1 for a non-box node with an unrefined incident cell
__global__ void __launch_bounds__(256) k_coarse_coef(Grid g, Cells cl, const uint32_t* __restrict__ code, Coef cf,
                                                     double* __restrict__ K, uint8_t* __restrict__ role)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= g.N) return;
    int i, j, k;
    decode(g, e, i, j, k);
    double kx = 0.0, ky = 0.0, kz = 0.0, m = 0.0;
    uint8_t r = 0;
    if (k >= 0 && k < g.nz) {
        const uint32_t c = code[e];
        const double ke = (c & C_SOLUTE) ? cf.kin : cf.kout;
        const int n[3] = {i, j, k};
        double kk[3];
        for (int ax = 0; ax < 3; ++ax) {
            const int o1 = ax == 0 ? 1 : 0, o2 = ax == 2 ? 1 : 2;
            int cnt = 0;
            for (int s1 = 0; s1 < 2; ++s1)
                for (int s2 = 0; s2 < 2; ++s2) {
                    int cc[3] = {n[0], n[1], n[2]};
                    cc[o1] -= s1;
                    cc[o2] -= s2;
                    if (cl.valid(cc[0], cc[1], cc[2]) && !cl.refined(cc[0], cc[1], cc[2])) ++cnt;
                }
            kk[ax] = 0.25 * (double)cnt * ke;
        }
        int c8 = 0;
        for (int a = 0; a < 8; ++a) {
            const int ci = i - (a & 1), cj = j - ((a >> 1) & 1), ck2 = k - ((a >> 2) & 1);
            if (cl.valid(ci, cj, ck2) && !cl.refined(ci, cj, ck2)) ++c8;
        }
        kx = kk[0];
        ky = kk[1];
        kz = kk[2];
        m = (c & C_SOLUTE) ? 0.0 : 0.125 * (double)c8 * cf.mass;
        r = (!(c & C_BOX) && c8 > 0) ? 1 : 0;
    }
    K[e] = kx;
    K[g.N + e] = ky;
    K[2 * g.N + e] = kz;
    K[3 * g.N + e] = m;
    role[e] = r;
}

// fine sub-lattice: the same from the refined incident fine cells (a fine cell is refined when
// its coarse parent is); roles 1 unknown, 2 coincident with a coarse unknown, 3 hanging
__global__ void __launch_bounds__(256) k_fine_coef(Grid g, Grid gc, Cells cl, const uint32_t* __restrict__ code,
                                                   const double* __restrict__ ck, Coef cf,
                                                   const uint8_t* __restrict__ rolec, double* __restrict__ K,
                                                   uint8_t* __restrict__ role)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= g.N) return;
    int i, j, k;
    decode(g, e, i, j, k);
    double kk[3] = {0.0, 0.0, 0.0}, m = 0.0;
    uint8_t r = 0;
    if (k >= 0 && k < g.nz) {
        const uint32_t c = code[e];
        const int F[3] = {i + g.off[0], j + g.off[1], k + g.off[2]};   // global fine lattice
        auto fref = [&](int a, int b, int d) {   // fine cell (global) refined?
            if (a < 0 || b < 0 || d < 0) return false;
            const int ci = a >> 1, cj = b >> 1, ck2 = d >> 1;
            return cl.valid(ci, cj, ck2) && cl.refined(ci, cj, ck2);
        };
        for (int ax = 0; ax < 3; ++ax) {
            const int o1 = ax == 0 ? 1 : 0, o2 = ax == 2 ? 1 : 2;
            int cnt = 0;
            for (int s1 = 0; s1 < 2; ++s1)
                for (int s2 = 0; s2 < 2; ++s2) {
                    int cc[3] = {F[0], F[1], F[2]};
                    cc[o1] -= s1;
                    cc[o2] -= s2;
                    if (fref(cc[0], cc[1], cc[2])) ++cnt;
                }
            kk[ax] = cnt ? 0.25 * (double)cnt * edgeK(c, ax, ck, cf) : 0.0;
        }
        int c8 = 0;
        for (int a = 0; a < 8; ++a)
            if (fref(F[0] - (a & 1), F[1] - ((a >> 1) & 1), F[2] - ((a >> 2) & 1))) ++c8;
        m = (c & C_SOLUTE) ? 0.0 : 0.125 * (double)c8 * cf.mass;
        if (c8 > 0) {
            const bool even = !((F[0] | F[1] | F[2]) & 1);
            if (even) {
                r = rolec[gc.idx(F[0] >> 1, F[1] >> 1, F[2] >> 1)] ? 2 : 1;
            } else {
                // coarse cells whose closed box holds the node: an odd coordinate has one
                // candidate, an even one two
                bool hang = false;
                for (int s = 0; s < 8 && !hang; ++s) {
                    int cc[3];
                    bool ok = true;
                    for (int d = 0; d < 3; ++d) {
                        const int side = (s >> d) & 1;
                        if (F[d] & 1) {
                            if (side) ok = false;
                            cc[d] = (F[d] - 1) >> 1;
                        } else {
                            cc[d] = (F[d] >> 1) - 1 + side;
                        }
                    }
                    if (ok && cl.valid(cc[0], cc[1], cc[2]) && !cl.refined(cc[0], cc[1], cc[2])) hang = true;
                }
                r = hang ? 3 : 1;
            }
        }
    }
    K[e] = kk[0];
    K[g.N + e] = kk[1];
    K[2 * g.N + e] = kk[2];
    K[3 * g.N + e] = m;
    role[e] = r;
}

// own-grid diagonal: the six edge coefficients and the lumped term
__device__ __forceinline__ double own_diag(const Grid& g, const double* __restrict__ K, int64_t e)
{
    const int64_t sx = (int64_t)g.ny * g.S, sy = g.S;
    return ((K[e] + K[e - sx]) + (K[g.N + e] + K[g.N + e - sy])) + ((K[2 * g.N + e] + K[2 * g.N + e - 1]) + K[3 * g.N + e]);
}

__global__ void __launch_bounds__(256) k_diag(Grid g, const double* __restrict__ K, const uint8_t* __restrict__ role,
                                              double* __restrict__ D)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= g.N) return;
    D[e] = role[e] ? own_diag(g, K, e) : 0.0;
}

// a coarse unknown with a coincident fine node also carries that node's fine diagonal
__global__ void __launch_bounds__(256) k_diag_fix(int64_t ng, const int64_t* gfine, const int64_t* gpar,
                                                  const int32_t* gnp, const double* Df, double* Dc)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= ng || gnp[t] != 1) return;
    Dc[gpar[4 * t]] += Df[gfine[t]];
}

__global__ void __launch_bounds__(256) k_invert(int64_t n, const uint8_t* __restrict__ role, double* __restrict__ D)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    D[e] = (role[e] == 1 && D[e] > 0.0) ? 1.0 / D[e] : 0.0;
}

// Dirichlet lift on the coarse grid: b += K g over the edges to box nodes
__global__ void __launch_bounds__(256) k_lift(Grid g, const double* __restrict__ K, const uint8_t* __restrict__ role,
                                              const uint32_t* __restrict__ code, const double* __restrict__ gb,
                                              double* __restrict__ b)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= g.N || role[e] != 1) return;
    const int64_t st[3] = {(int64_t)g.ny * g.S, g.S, 1};
    double lift = 0.0;
    for (int ax = 0; ax < 3; ++ax) {
        if (code[e + st[ax]] & C_BOX) lift += K[ax * g.N + e] * gb[e + st[ax]];
        if (code[e - st[ax]] & C_BOX) lift += K[ax * g.N + e - st[ax]] * gb[e - st[ax]];
    }
    b[e] += lift;
}

// ---- operator and CG ---------------------------------------------------------------------

// derived fine values from the coarse ones
template <typename T>
__global__ void __launch_bounds__(256) k_fill(int64_t ng, const int64_t* __restrict__ gfine,
                                              const int64_t* __restrict__ gpar, const int32_t* __restrict__ gnp,
                                              const T* __restrict__ vc, T* __restrict__ vf, const CGState* st)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= ng || (st && st->status != 0)) return;
    const int np = gnp[t];
    T s = (T)0;
    for (int u = 0; u < np; ++u) s += vc[gpar[4 * t + u]];
    vf[gfine[t]] = s / (T)np;
}

// q = (cell contributions of this grid) p at every node with a role; 0 elsewhere
template <typename T>
__global__ void __launch_bounds__(256) k_apply(Grid g, const T* __restrict__ K, const uint8_t* __restrict__ role,
                                               const T* __restrict__ p, T* __restrict__ q, const CGState* st)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= g.N || (st && st->status != 0)) return;
    if (!role[e]) {
        q[e] = (T)0;
        return;
    }
    const int64_t sx = (int64_t)g.ny * g.S, sy = g.S;
    const T kxp = K[e], kxm = K[e - sx], kyp = K[g.N + e], kym = K[g.N + e - sy];
    const T kzp = K[2 * g.N + e], kzm = K[2 * g.N + e - 1];
    const T D = ((kxp + kxm) + (kyp + kym)) + ((kzp + kzm) + K[3 * g.N + e]);
    q[e] = D * p[e] - (((kxm * p[e - sx] + kxp * p[e + sx]) + (kym * p[e - sy] + kyp * p[e + sy])) +
                       (kzm * p[e - 1] + kzp * p[e + 1]));
}

// the rows of the derived fine nodes go to their coarse parents: one thread per coarse node
// that is a parent (rnode), gathering the derived fine nodes among the 27 fine nodes around it
// in fine-lattice order; the derived node at 2C + d is a child of C with weight 1 / 2^(number
// of nonzero components of d)
template <typename T>
__global__ void __launch_bounds__(256) k_restrict(int64_t nr, const int64_t* __restrict__ rnode, Grid gc, Grid gf,
                                                  const uint8_t* __restrict__ rolef, const T* __restrict__ vf,
                                                  T* __restrict__ vc, const CGState* st)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= nr || (st && st->status != 0)) return;
    const int64_t ec = rnode[t];
    int i, j, k;
    decode(gc, ec, i, j, k);
    const int F[3] = {2 * i - gf.off[0], 2 * j - gf.off[1], 2 * k - gf.off[2]};
    T s = (T)0;
    for (int a = -1; a <= 1; ++a)
        for (int b = -1; b <= 1; ++b)
            for (int c = -1; c <= 1; ++c) {
                const int f0 = F[0] + a, f1 = F[1] + b, f2 = F[2] + c;
                if (f0 < 0 || f1 < 0 || f2 < 0 || f0 >= gf.nx || f1 >= gf.ny || f2 >= gf.nz) continue;
                const int64_t ef = gf.idx(f0, f1, f2);
                if (rolef[ef] < 2) continue;
                const int np = 1 << ((a != 0) + (b != 0) + (c != 0));
                s += (T)(1.0 / np) * vf[ef];
            }
    vc[ec] += s;
}

// ---- the lists of derived fine nodes and of their coarse parents, built on the device -------

// whether fine element e is a derived node (role 2 or 3)
__device__ __forceinline__ bool derived_at(const Grid& gf, const uint8_t* rolef, int64_t e)
{
    return e < gf.N && rolef[e] >= 2;
}

// whether coarse element e is the parent of a derived fine node (one among the 27 around it)
__device__ __forceinline__ bool parent_at(const Grid& gc, const Grid& gf, const uint8_t* rolef, int64_t e)
{
    if (e >= gc.N) return false;
    int i, j, k;
    decode(gc, e, i, j, k);
    if (k < 0 || k >= gc.nz) return false;
    const int F[3] = {2 * i - gf.off[0], 2 * j - gf.off[1], 2 * k - gf.off[2]};
    for (int a = -1; a <= 1; ++a)
        for (int b = -1; b <= 1; ++b)
            for (int c = -1; c <= 1; ++c) {
                const int f0 = F[0] + a, f1 = F[1] + b, f2 = F[2] + c;
                if (f0 < 0 || f1 < 0 || f2 < 0 || f0 >= gf.nx || f1 >= gf.ny || f2 >= gf.nz) continue;
                if (rolef[gf.idx(f0, f1, f2)] >= 2) return true;
            }
    return false;
}

// rank of this thread's flag among the flagged threads of its block, in thread order (every
// thread of the block calls it)
__device__ __forceinline__ int block_rank(bool f, int* wsum)
{
    const int lane = (int)(threadIdx.x & 63), w = (int)(threadIdx.x >> 6);
    const unsigned long long m = __ballot(f);
    if (lane == 0) wsum[w] = __popcll(m);
    __syncthreads();
    int base = 0;
    for (int q = 0; q < w; ++q) base += wsum[q];
    return base + __popcll(m & ((1ull << lane) - 1ull));
}

// flagged elements per block of 256 (mode 0: derived fine nodes over the fine elements; 1:
// parents over the coarse elements)
__global__ void __launch_bounds__(256) k_list_count(int mode, Grid gc, Grid gf, const uint8_t* __restrict__ rolef,
                                                    int* __restrict__ cnt)
{
    __shared__ int wsum[4];
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool f = mode == 0 ? derived_at(gf, rolef, e) : parent_at(gc, gf, rolef, e);
    const int r = block_rank(f, wsum);
    (void)r;
    if (threadIdx.x == 0) cnt[blockIdx.x] = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
}

// the lists in element order from the scanned block counts (start): mode 0 the derived fine
// nodes (gfine), their parent counts (gnp) and their coarse parents (gpar, from the node's
// lattice coordinates: along an odd axis the two coarse nodes around it, along an even one
// the coarse node it lies on, in (a, b, c) order, unused slots repeating the first); a parent
// that is not a coarse unknown sets *bad.  Mode 1: the parents (rnode).
__global__ void __launch_bounds__(256) k_list_assign(int mode, Grid gc, Grid gf, const uint8_t* __restrict__ rolef,
                                                     const uint8_t* __restrict__ rolec, const int* __restrict__ start,
                                                     int64_t* gfine, int64_t* gpar, int32_t* gnp, int64_t* rnode,
                                                     int* bad)
{
    __shared__ int wsum[4];
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool f = mode == 0 ? derived_at(gf, rolef, e) : parent_at(gc, gf, rolef, e);
    const int64_t pos = (int64_t)start[blockIdx.x] + block_rank(f, wsum);
    if (!f) return;
    if (mode == 1) {
        rnode[pos] = e;
        return;
    }
    int i, j, k;
    decode(gf, e, i, j, k);
    const int F[3] = {i + gf.off[0], j + gf.off[1], k + gf.off[2]};   // global fine lattice
    int lo[3], hi[3], np = 1;
    for (int d = 0; d < 3; ++d) {
        if (F[d] & 1) {
            lo[d] = (F[d] - 1) / 2;
            hi[d] = (F[d] + 1) / 2;
            np *= 2;
        } else {
            lo[d] = hi[d] = F[d] / 2;
        }
    }
    if (np > 4) atomicOr(bad, 2);   // not a node of a coarse edge or face
    gfine[pos] = e;
    gnp[pos] = np;
    int u = 0;
    int64_t first = -1;
    for (int a = lo[0]; a <= hi[0]; ++a)
        for (int b = lo[1]; b <= hi[1]; ++b)
            for (int c = lo[2]; c <= hi[2]; ++c) {
                const int64_t pe = gc.idx(a, b, c);
                if (rolec[pe] != 1) atomicOr(bad, 1);
                if (first < 0) first = pe;
                if (u < 4) gpar[4 * pos + u] = pe;
                ++u;
            }
    for (; u < 4; ++u) gpar[4 * pos + u] = first;
}

// counters: [0] coarse unknowns, [1] fine unknowns, [2] hanging nodes
__global__ void __launch_bounds__(256) k_role_count(int64_t Nc, const uint8_t* __restrict__ rolec, int64_t Nf,
                                                    const uint8_t* __restrict__ rolef,
                                                    unsigned long long* __restrict__ out)
{
    unsigned long long v[3] = {0, 0, 0};
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < Nc; e += stride) v[0] += rolec[e] == 1;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < Nf; e += stride) {
        v[1] += rolef[e] == 1;
        v[2] += rolef[e] == 3;
    }
    for (int q = 0; q < 3; ++q) {
        for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o, 64);
        if ((threadIdx.x & 63) == 0 && v[q]) atomicAdd(out + q, v[q]);
    }
}

// refined coarse cells: out[3] counts them; bit 1 of out[4]: one touches the box boundary
// layer, bit 2: one lies outside the fine sub-lattice's cells [cl + 1, ch - 1)
__global__ void __launch_bounds__(256) k_cell_checks(Cells cl, int l0, int l1, int l2, int h0, int h1, int h2,
                                                     unsigned long long* __restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t n = (int64_t)cl.nc[0] * cl.nc[1] * cl.nc[2];
    bool ref = false;
    unsigned flags = 0;
    if (t < n && cl.f[t]) {
        ref = true;
        const int c[3] = {(int)(t / ((int64_t)cl.nc[1] * cl.nc[2])), (int)((t / cl.nc[2]) % cl.nc[1]),
                          (int)(t % cl.nc[2])};
        const int lo[3] = {l0, l1, l2}, hi[3] = {h0, h1, h2};
        for (int d = 0; d < 3; ++d) {
            if (c[d] == 0 || c[d] == cl.nc[d] - 1) flags |= 1u;
            if (c[d] < lo[d] + 1 || c[d] >= hi[d] - 1) flags |= 2u;
        }
    }
    const unsigned long long m = __ballot(ref);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(out + 3, (unsigned long long)__popcll(m));
    if (flags) atomicOr(out + 4, (unsigned long long)flags);
}

// charge loads accumulated on the host (unique elements): dst[idx[t]] = val[t]
__global__ void __launch_bounds__(256) k_scatter(int64_t n, const int64_t* __restrict__ idx,
                                                 const double* __restrict__ val, double* __restrict__ dst)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t < n) dst[idx[t]] = val[t];
}

// the loads of the derived fine nodes go to their coarse parents: each parent adds v / (its
// child's parent count) of every child with a nonzero load, in fine-lattice order
__global__ void __launch_bounds__(256) k_fold_load(int64_t nr, const int64_t* __restrict__ rnode, Grid gc, Grid gf,
                                                   const uint8_t* __restrict__ rolef, const double* __restrict__ bf,
                                                   double* __restrict__ bc)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= nr) return;
    const int64_t ec = rnode[t];
    int i, j, k;
    decode(gc, ec, i, j, k);
    const int F[3] = {2 * i - gf.off[0], 2 * j - gf.off[1], 2 * k - gf.off[2]};
    double h = bc[ec];
    for (int a = -1; a <= 1; ++a)
        for (int b = -1; b <= 1; ++b)
            for (int c = -1; c <= 1; ++c) {
                const int f0 = F[0] + a, f1 = F[1] + b, f2 = F[2] + c;
                if (f0 < 0 || f1 < 0 || f2 < 0 || f0 >= gf.nx || f1 >= gf.ny || f2 >= gf.nz) continue;
                const int64_t ef = gf.idx(f0, f1, f2);
                if (rolef[ef] < 2) continue;
                const double v = bf[ef];
                if (v == 0.0) continue;
                h += v / (double)(1 << ((a != 0) + (b != 0) + (c != 0)));
            }
    bc[ec] = h;
}

// ... and leave the derived fine nodes' own loads at zero
__global__ void __launch_bounds__(256) k_zero_derived(int64_t ng, const int64_t* __restrict__ gfine,
                                                      double* __restrict__ bf)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t < ng) bf[gfine[t]] = 0.0;
}

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

// The vector kernels run over both grids in one launch: blocks [0, nbc) take the coarse
// grid, the others the fine sub-lattice.
struct Split {
    int64_t Nc, Nf;
    int nbc;
    const uint8_t *rc, *rf;
    __device__ bool coarse() const { return (int)blockIdx.x < nbc; }
    __device__ int64_t first() const { return (coarse() ? blockIdx.x : blockIdx.x - nbc) * (int64_t)256 + threadIdx.x; }
    __device__ int64_t stride() const { return (coarse() ? nbc : (int64_t)gridDim.x - nbc) * (int64_t)256; }
    __device__ int64_t n() const { return coarse() ? Nc : Nf; }
    __device__ const uint8_t* role() const { return coarse() ? rc : rf; }
};

// partial sums of a.b over the unknowns of both grids
template <typename T>
__global__ void __launch_bounds__(256) k_dot(Split sp, const T* ac, const T* bc, const T* af, const T* bf,
                                             double* part, const CGState* st)
{
    __shared__ double sh[8];
    if (st->status != 0) return;
    const uint8_t* role = sp.role();
    const T* a = sp.coarse() ? ac : af;
    const T* b = sp.coarse() ? bc : bf;
    double v[1] = {0.0};
    for (int64_t e = sp.first(); e < sp.n(); e += sp.stride())
        if (role[e] == 1) v[0] += (double)a[e] * (double)b[e];
    bsum(v, 1, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
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

// x += alpha p, r -= alpha q, z = D^-1 r; partial sums of r.z and r.r
template <typename T>
__global__ void __launch_bounds__(256) k_update(Split sp, T* xc, T* rrc, T* zc, const T* pc, const T* qc, const T* dc,
                                                T* xf, T* rrf, T* zf, const T* pf, const T* qf, const T* df,
                                                double* part, int nb, const CGState* st)
{
    __shared__ double sh[8];
    if (st->status != 0) return;
    const bool coarse = sp.coarse();
    const uint8_t* role = sp.role();
    T* x = coarse ? xc : xf;
    T* r = coarse ? rrc : rrf;
    T* z = coarse ? zc : zf;
    const T* p = coarse ? pc : pf;
    const T* q = coarse ? qc : qf;
    const T* d = coarse ? dc : df;
    const T a = (T)st->alpha;
    double v[2] = {0.0, 0.0};
    for (int64_t e = sp.first(); e < sp.n(); e += sp.stride()) {
        if (role[e] != 1) continue;
        x[e] += a * p[e];
        const T rv = r[e] - a * q[e];
        r[e] = rv;
        const T zv = d[e] * rv;
        z[e] = zv;
        v[0] += (double)rv * (double)zv;
        v[1] += (double)rv * (double)rv;
    }
    bsum(v, 2, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = v[0];
        part[nb + blockIdx.x] = v[1];
    }
}

// beta = r.z / r.z_old and the stop test: status = stop_status once r.r falls to stop2 (the
// FP64 solve's goal; in mixed precision the FP32 goal) or to trig2 (mixed precision: the
// point at which the true residual is computed again); with mode 1 the first residual sets
// the reference norm (no beta)
__global__ void __launch_bounds__(256) k_beta(const double* part, int nb, CGState* st, int mode, double rtol2)
{
    __shared__ double sh[8];
    if (mode == 0 && st->status != 0) return;
    double v[2] = {0.0, 0.0};
    for (int t = threadIdx.x; t < nb; t += 256) {
        v[0] += part[t];
        v[1] += part[nb + t];
    }
    bsum(v, 2, sh);
    if (threadIdx.x == 0) {
        const double gm = v[0], rr = v[1];
        if (mode == 1) {          // init
            st->bnorm2 = rr;
            st->stop2 = rtol2 * rr;
            st->iter_count = 0;
            st->beta = 0.0;
        } else if (mode == 0) {   // an iteration
            st->iter_count += 1;
            st->beta = st->gamma > 0.0 ? gm / st->gamma : 0.0;
        }
        st->status = 0;
        st->gamma = gm;
        st->rr = rr;
        if (!isfinite(gm) || !isfinite(rr)) {
            st->status = 2;
            st->iters = st->iter_count;
        } else if (rr <= st->stop2 || rr <= st->trig2) {
            st->status = st->stop_status;
            st->iters = st->iter_count;
        }
    }
}

// p = z + beta p over the unknowns of one grid (init: beta = 0)
template <typename T>
__global__ void __launch_bounds__(256) k_pupd(int64_t N, const uint8_t* role, const T* z, T* p, const CGState* st)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= N || st->status != 0) return;
    p[e] = role[e] == 1 ? z[e] + (T)st->beta * p[e] : (T)0;
}

// ---- two-level preconditioner ----------------------------------------------------------------
// z = B r with B the symmetric two-level preconditioner: z1 = w D^-1 r, then the coarse-grid
// correction z2 = z1 + I_H V(I_H^T (r - A z1)) with V one V-cycle of the coarse grid's own
// multigrid (its operator from the coarse node-code map), then z = z2 + w D^-1 (r - A z2).
// I_H interpolates the coarse grid trilinearly to the unknowns: a coarse unknown takes its own
// node; a fine unknown at fine-lattice coordinates F takes coarse node F/2 along an even axis
// and the two nodes (F -+ 1)/2 with weight 1/2 along an odd one.  In the element type of the
// CG (FP64, or FP32 in the mixed form, whose reliable updates apply it ungated: st = null).

constexpr double kOmega = 0.8;   // smoother damping: w D^-1 A stays below 2 (SPD preconditioner)

__device__ __forceinline__ bool stopped(const CGState* st) { return st && st->status != 0; }

// z *= w at the unknowns
template <typename T>
__global__ void __launch_bounds__(256) k_zscale(Split sp, T* zc, T* zf, const CGState* st)
{
    if (stopped(st)) return;
    const uint8_t* role = sp.role();
    T* z = sp.coarse() ? zc : zf;
    for (int64_t e = sp.first(); e < sp.n(); e += sp.stride())
        if (role[e] == 1) z[e] *= (T)kOmega;
}

// q = r - q at the unknowns
template <typename T>
__global__ void __launch_bounds__(256) k_rsub(Split sp, const T* rc, const T* rf, T* qc, T* qf, const CGState* st)
{
    if (stopped(st)) return;
    const uint8_t* role = sp.role();
    const T* r = sp.coarse() ? rc : rf;
    T* q = sp.coarse() ? qc : qf;
    for (int64_t e = sp.first(); e < sp.n(); e += sp.stride())
        if (role[e] == 1) q[e] = r[e] - q[e];
}

// bH = I_H^T w over the coarse grid (0 on the box and the pads): the node's own value where it
// is a coarse unknown, plus the fine unknowns among the 27 fine nodes around it
template <typename T>
__global__ void __launch_bounds__(256) k_rest_h(Grid gc, Grid gf, const uint8_t* __restrict__ rolec,
                                                const uint8_t* __restrict__ rolef, const T* __restrict__ wc,
                                                const T* __restrict__ wf, T* __restrict__ bH, const CGState* st)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= gc.N || stopped(st)) return;
    int i, j, k;
    decode(gc, e, i, j, k);
    if (k < 1 || k > gc.nz - 2 || i < 1 || i > gc.nx - 2 || j < 1 || j > gc.ny - 2) {
        bH[e] = (T)0;
        return;
    }
    T v = rolec[e] == 1 ? wc[e] : (T)0;
    const int F[3] = {2 * i - gf.off[0], 2 * j - gf.off[1], 2 * k - gf.off[2]};
    const int nf[3] = {gf.nx, gf.ny, gf.nz};
    bool near = true;
    for (int d = 0; d < 3; ++d) near = near && F[d] >= -1 && F[d] <= nf[d];
    if (near)
        for (int a = -1; a <= 1; ++a)
            for (int b = -1; b <= 1; ++b)
                for (int c = -1; c <= 1; ++c) {
                    const int f0 = F[0] + a, f1 = F[1] + b, f2 = F[2] + c;
                    if (f0 < 0 || f1 < 0 || f2 < 0 || f0 >= nf[0] || f1 >= nf[1] || f2 >= nf[2]) continue;
                    const int64_t ef = gf.idx(f0, f1, f2);
                    if (rolef[ef] != 1) continue;
                    const T w = (a ? (T)0.5 : (T)1) * (b ? (T)0.5 : (T)1) * (c ? (T)0.5 : (T)1);
                    v += w * wf[ef];
                }
    bH[e] = v;
}

// z += I_H eH at the coarse unknowns
template <typename T>
__global__ void __launch_bounds__(256) k_prol_c(int64_t N, const uint8_t* __restrict__ rolec, const T* __restrict__ eH,
                                                T* __restrict__ zc, const CGState* st)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= N || stopped(st)) return;
    if (rolec[e] == 1) zc[e] += eH[e];
}

// z += I_H eH at the fine unknowns
template <typename T>
__global__ void __launch_bounds__(256) k_prol_f(Grid gf, Grid gc, const uint8_t* __restrict__ rolef,
                                                const T* __restrict__ eH, T* __restrict__ zf, const CGState* st)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= gf.N || stopped(st)) return;
    if (rolef[e] != 1) return;
    int i, j, k;
    decode(gf, e, i, j, k);
    const int F[3] = {i + gf.off[0], j + gf.off[1], k + gf.off[2]};
    T v = (T)0;
    for (int s3 = 0; s3 < 8; ++s3) {
        int I[3];
        T w = (T)1;
        bool ok = true;
        for (int d = 0; d < 3; ++d) {
            const int bit = (s3 >> d) & 1;
            if (F[d] & 1) {
                I[d] = (F[d] - 1) / 2 + bit;
                w *= (T)0.5;
            } else {
                I[d] = F[d] / 2;
                ok = ok && bit == 0;
            }
        }
        if (ok) v += w * eH[gc.idx(I[0], I[1], I[2])];
    }
    zf[e] += v;
}

// z += w D^-1 (r - q) at the unknowns; partial sums of r.z in part[0, nb)
template <typename T>
__global__ void __launch_bounds__(256) k_post(Split sp, T* zc, T* zf, const T* rc, const T* rf, const T* qc,
                                              const T* qf, const T* dc, const T* df, double* part, const CGState* st)
{
    __shared__ double sh[8];
    if (stopped(st)) return;
    const bool coarse = sp.coarse();
    const uint8_t* role = sp.role();
    T* z = coarse ? zc : zf;
    const T* r = coarse ? rc : rf;
    const T* q = coarse ? qc : qf;
    const T* d = coarse ? dc : df;
    double v[1] = {0.0};
    for (int64_t e = sp.first(); e < sp.n(); e += sp.stride()) {
        if (role[e] != 1) continue;
        const T zv = z[e] + (T)kOmega * d[e] * (r[e] - q[e]);
        z[e] = zv;
        v[0] += (double)r[e] * (double)zv;
    }
    bsum(v, 1, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// ---- mixed precision: reliable updates ------------------------------------------------------

__global__ void __launch_bounds__(256) k_to_f32(int64_t n, const double* __restrict__ a, float* __restrict__ b)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e < n) b[e] = (float)a[e];
}

// x64 += x32, x32 = 0 over both grids
__global__ void __launch_bounds__(256) k_fold(Split sp, double* xc, float* dc, double* xf, float* df)
{
    double* x = sp.coarse() ? xc : xf;
    float* d = sp.coarse() ? dc : df;
    const uint8_t* role = sp.role();
    for (int64_t e = sp.first(); e < sp.n(); e += sp.stride())
        if (role[e] == 1) {
            x[e] += (double)d[e];
            d[e] = 0.0f;
        }
}

// r64 = b - q64 on the unknowns (q64 = A x64 with the FP64 operator); partial sums of r.r
__global__ void __launch_bounds__(256) k_true_res(Split sp, const double* bc, const double* qc, double* rc,
                                                  const double* bf, const double* qf, double* rf, double* part)
{
    __shared__ double sh[8];
    const bool coarse = sp.coarse();
    const uint8_t* role = sp.role();
    const double* b = coarse ? bc : bf;
    const double* q = coarse ? qc : qf;
    double* r = coarse ? rc : rf;
    double v[1] = {0.0};
    for (int64_t e = sp.first(); e < sp.n(); e += sp.stride()) {
        const double rv = role[e] == 1 ? b[e] - q[e] : 0.0;
        r[e] = rv;
        v[0] += rv * rv;
    }
    bsum(v, 1, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// r32 = r64, z32 = D^-1 r32; partial sums of r.z and r.r
__global__ void __launch_bounds__(256) k_replace(Split sp, const double* r64c, float* rc, float* zc, const float* dc,
                                                 const double* r64f, float* rf, float* zf, const float* df,
                                                 double* part, int nb)
{
    __shared__ double sh[8];
    const bool coarse = sp.coarse();
    const uint8_t* role = sp.role();
    const double* r64 = coarse ? r64c : r64f;
    float* r = coarse ? rc : rf;
    float* z = coarse ? zc : zf;
    const float* d = coarse ? dc : df;
    double v[2] = {0.0, 0.0};
    for (int64_t e = sp.first(); e < sp.n(); e += sp.stride()) {
        const float rv = role[e] == 1 ? (float)r64[e] : 0.0f;
        const float zv = d[e] * rv;
        r[e] = rv;
        z[e] = zv;
        v[0] += (double)rv * (double)zv;
        v[1] += (double)rv * (double)rv;
    }
    bsum(v, 2, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = v[0];
        part[nb + blockIdx.x] = v[1];
    }
}

// after a residual replacement: part holds [r.z | r.r] of the FP32 residual and, after them,
// the FP64 r.r; the FP64 norm decides convergence.  With init the first replacement (x = 0,
// r = b) sets the goals.  A replacement follows a step whose direction update was skipped
// (status 3 stops the launches after beta), so the next direction update takes beta from the
// replaced residual.
__global__ void __launch_bounds__(256) k_ru_fin(const double* part, int nb, CGState* st, int init, double rtol2,
                                                double delta2)
{
    __shared__ double sh[12];
    double v[3] = {0.0, 0.0, 0.0};
    for (int t = threadIdx.x; t < nb; t += 256) {
        v[0] += part[t];
        v[1] += part[nb + t];
        v[2] += part[2 * nb + t];
    }
    bsum(v, 3, sh);
    if (threadIdx.x == 0) {
        const double gm = v[0], rr = v[1], rr64 = v[2];
        if (init) {
            st->bnorm2 = rr64;
            st->goal64 = rtol2 * rr64;
            st->stop2 = rtol2 * rr;
            st->delta2 = delta2;
            st->stop_status = 3;
            st->iter_count = 0;
            st->n_ru = 0;
            st->beta = 0.0;
        } else {
            // the direction continues from the replaced residual: its step was cut before
            // p was updated, so beta = r'.z' over r.z of the step before (gamma / beta)
            st->n_ru += 1;
            st->beta = (st->gamma > 0.0 && st->beta > 0.0) ? gm * (st->beta / st->gamma) : 0.0;
        }
        st->alpha = 0.0;
        st->gamma = gm;
        st->rr = rr;
        st->rr64 = rr64;
        st->trig2 = st->delta2 * rr;
        if (!isfinite(rr64) || !isfinite(gm)) {
            st->status = 2;
            st->iters = st->iter_count;
        } else if (rr64 <= st->goal64) {
            st->status = 1;
            st->iters = st->iter_count;
        } else {
            st->status = 0;
        }
    }
}

__global__ void k_state_init(CGState* st)
{
    st->alpha = st->beta = st->gamma = st->bnorm2 = st->rr = st->pq = 0.0;
    st->stop2 = st->trig2 = st->delta2 = st->goal64 = st->rr64 = 0.0;
    st->status = 0;
    st->stop_status = 1;
    st->iters = st->iter_count = st->ru = st->n_ru = 0;
}

// coarse nodes inside the refined region take the value of their fine node (for export)
__global__ void __launch_bounds__(256) k_sync_coarse(Grid gc, Grid gf, const uint8_t* rolec, const uint32_t* codec,
                                                     const double* xf, double* xc)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= gc.N || rolec[e] || (codec[e] & C_BOX)) return;
    int i, j, k;
    decode(gc, e, i, j, k);
    if (k < 0 || k >= gc.nz) return;
    const int a = 2 * i - gf.off[0], b = 2 * j - gf.off[1], c = 2 * k - gf.off[2];
    if (a < 0 || b < 0 || c < 0 || a >= gf.nx || b >= gf.ny || c >= gf.nz) return;
    xc[e] = xf[gf.idx(a, b, c)];
}

}  // namespace

// ---- host side -----------------------------------------------------------------------------

int pbi_refine_build(pb_problem* pb, const double* xyz, const double* rad, const double* chg)
{
    const pb_params& P = pb->prm;
    const Grid& gc = pb->g;
    hipStream_t s = pb->ctx->stream;
    RefineData* R = new RefineData();
    pb->ref = R;
    R->delta = P.refine_shell_A;
    R->brick = P.refine_brick;
    for (int d = 0; d < 3; ++d) R->nc[d] = P.n[d] - 1;
    const int64_t na = pb->na;
    if (na <= 0) return pbi_fail(PB_EINVAL, "refinement needs atoms");

    // fine sub-lattice: the bricks that can hold a cell within delta of the surface, plus one
    // coarse cell on every side
    const double H = P.h, o[3] = {P.origin[0], P.origin[1], P.origin[2]};
    int cl[3], ch[3];
    for (int d = 0; d < 3; ++d) {
        double lo = 1e300, hi = -1e300;
        for (int64_t a = 0; a < na; ++a) {
            lo = std::min(lo, xyz[3 * a + d] - rad[a]);
            hi = std::max(hi, xyz[3 * a + d] + rad[a]);
        }
        const int c0 = (int)std::floor((lo - R->delta - o[d]) / H) - 1;
        const int c1 = (int)std::floor((hi + R->delta - o[d]) / H) + 2;   // one past the last cell
        const int B = R->brick;
        cl[d] = (c0 / B) * B - 1;
        ch[d] = ((c1 + B - 1) / B) * B + 1;
        cl[d] = std::max(cl[d], 0);
        ch[d] = std::min(ch[d], R->nc[d]);
    }
    pb_params pf = P;
    pf.bc = PB_BC_ZERO;
    pf.bc_values = nullptr;
    pf.h = H / 2.0;
    pf.refine = 0;
    pf.precision = PB_FP64;
    int off[3];
    for (int d = 0; d < 3; ++d) {
        pf.n[d] = 2 * (ch[d] - cl[d]) + 1;
        off[d] = 2 * cl[d];
    }
    pb_problem* fp = nullptr;
    int rc = pbi_build_begin_sub(pb->ctx, &pf, na, xyz, rad, chg, off, &fp);
    if (rc) return rc;
    R->fine = fp;
    if (hipEventSynchronize(fp->ev) != hipSuccess) return pbi_fail(PB_EDEVICE, "fine build: counting failed");
    if ((rc = pbi_build_continue(fp))) return rc;
    if (hipEventSynchronize(fp->ev) != hipSuccess) return pbi_fail(PB_EDEVICE, "fine build failed");
    pbi_build_end(fp);
    const Grid& gf = fp->g;

    // refinement flags
    const int64_t ncell = (int64_t)R->nc[0] * R->nc[1] * R->nc[2];
    const int B = R->brick;
    const int nb[3] = {(R->nc[0] + B - 1) / B, (R->nc[1] + B - 1) / B, (R->nc[2] + B - 1) / B};
    R->cells = (uint8_t*)pb->mem.get((size_t)ncell);
    uint8_t* flag = (uint8_t*)pb->mem.get((size_t)ncell);
    uint8_t* bf = (uint8_t*)pb->mem.get((size_t)nb[0] * nb[1] * nb[2]);
    if (!R->cells || !flag || !bf) return pbi_fail(PB_ENOMEM, "refinement flags");
    RCHK(launch_fill(s, flag, (size_t)ncell));
    if (P.refine == 2) {
        double lo[3], hi[3];
        for (int d = 0; d < 3; ++d) {
            lo[d] = 1e300;
            hi[d] = -1e300;
            for (int64_t a = 0; a < na; ++a) {
                lo[d] = std::min(lo[d], xyz[3 * a + d] - rad[a]);
                hi[d] = std::max(hi[d], xyz[3 * a + d] + rad[a]);
            }
        }
        k_mark_box<<<nblk(ncell, 256), 256, 0, s>>>(gc, lo[0], lo[1], lo[2], hi[0], hi[1], hi[2], R->delta, flag,
                                                    R->nc[0], R->nc[1], R->nc[2]);
    } else if (fp->ncut > 0) {
        k_mark<<<nblk(fp->ncut, 256), 256, 0, s>>>(gc, fp->ncut, fp->rp, R->delta, flag, R->nc[0], R->nc[1], R->nc[2]);
    }
    k_bricks<<<nblk((int64_t)nb[0] * nb[1] * nb[2], 256), 256, 0, s>>>(flag, R->nc[0], R->nc[1], R->nc[2], B, nb[0], nb[1],
                                                                       nb[2], bf);
    k_cells_from_bricks<<<nblk(ncell, 256), 256, 0, s>>>(bf, R->nc[0], R->nc[1], R->nc[2], B, nb[1], nb[2], R->cells);
    RCHK(hipGetLastError());
    // the refined cells: counted and checked on the device; their flags come to the host for
    // the charge load below (whether an atom's coarse cell is refined)
    unsigned long long* cnt64 = (unsigned long long*)pb->mem.get(sizeof(unsigned long long) * 8);
    int* bad = (int*)pb->mem.get(sizeof(int) * 2);
    if (!cnt64 || !bad) return pbi_fail(PB_ENOMEM, "refinement counters");
    RCHK(launch_fill(s, cnt64, sizeof(unsigned long long) * 8));
    RCHK(launch_fill(s, bad, sizeof(int) * 2));
    Cells cells{R->cells, {R->nc[0], R->nc[1], R->nc[2]}};
    k_cell_checks<<<nblk(ncell, 256), 256, 0, s>>>(cells, cl[0], cl[1], cl[2], ch[0], ch[1], ch[2], cnt64);
    RCHK(hipGetLastError());
    std::vector<uint8_t> hcell((size_t)ncell);
    unsigned long long hc[8] = {};
    RCHK(hipMemcpyAsync(hcell.data(), R->cells, (size_t)ncell, hipMemcpyDeviceToHost, s));
    RCHK(hipMemcpyAsync(hc, cnt64, sizeof hc, hipMemcpyDeviceToHost, s));
    RCHK(hipStreamSynchronize(s));
    pb->mem.put(flag);
    pb->mem.put(bf);
    if (hc[4] & 1u) return pbi_fail(PB_EINVAL, "refined cells touch the box boundary layer");
    if (hc[4] & 2u) return pbi_fail(PB_EINVAL, "refined cell outside the fine sub-lattice");
    R->n_refined = (int64_t)hc[3];

    // coefficients and roles
    R->Kc = (double*)pb->mem.get(sizeof(double) * 4 * (size_t)gc.N);
    R->Kf = (double*)pb->mem.get(sizeof(double) * 4 * (size_t)gf.N);
    R->rolec = (uint8_t*)pb->mem.get((size_t)gc.N);
    R->rolef = (uint8_t*)pb->mem.get((size_t)gf.N);
    if (!R->Kc || !R->Kf || !R->rolec || !R->rolef) return pbi_fail(PB_ENOMEM, "refined coefficients");
    k_coarse_coef<<<nblk(gc.N, 256), 256, 0, s>>>(gc, cells, pb->code, pb->cf, R->Kc, R->rolec);
    k_fine_coef<<<nblk(gf.N, 256), 256, 0, s>>>(gf, gc, cells, fp->code, fp->ck64, fp->cf, R->rolec, R->Kf, R->rolef);
    RCHK(hipGetLastError());

    // the derived fine nodes (roles 2 and 3) with their coarse parents, and the coarse nodes
    // that are parents, as ordered compactions (block counts, a scan, then the lists), and the
    // role counts
    const unsigned nbD = nblk(gf.N, 256), nbP = nblk(gc.N, 256);
    int* startD = (int*)pb->mem.get(sizeof(int) * ((size_t)nbD + 1));
    int* startP = (int*)pb->mem.get(sizeof(int) * ((size_t)nbP + 1));
    if (!startD || !startP) return pbi_fail(PB_ENOMEM, "refinement lists");
    k_list_count<<<nbD, 256, 0, s>>>(0, gc, gf, R->rolef, startD);
    k_list_count<<<nbP, 256, 0, s>>>(1, gc, gf, R->rolef, startP);
    RCHK(launch_scan1(s, startD, (int)nbD, startD));
    RCHK(launch_scan1(s, startP, (int)nbP, startP));
    k_role_count<<<std::min<unsigned>(1024, nblk(std::max(gc.N, gf.N), 256)), 256, 0, s>>>(gc.N, R->rolec, gf.N,
                                                                                            R->rolef, cnt64);
    RCHK(hipGetLastError());
    int tot[2] = {0, 0};
    RCHK(hipMemcpyAsync(&tot[0], startD + nbD, sizeof(int), hipMemcpyDeviceToHost, s));
    RCHK(hipMemcpyAsync(&tot[1], startP + nbP, sizeof(int), hipMemcpyDeviceToHost, s));
    RCHK(hipMemcpyAsync(hc, cnt64, sizeof hc, hipMemcpyDeviceToHost, s));
    RCHK(hipStreamSynchronize(s));
    R->nunk_c = (int64_t)hc[0];
    R->nunk_f = (int64_t)hc[1];
    R->nhang = (int64_t)hc[2];
    R->ng = tot[0];
    R->nr = tot[1];
    R->gfine = (int64_t*)pb->mem.get(sizeof(int64_t) * (size_t)std::max<int64_t>(R->ng, 1));
    R->gpar = (int64_t*)pb->mem.get(sizeof(int64_t) * 4 * (size_t)std::max<int64_t>(R->ng, 1));
    R->gnp = (int32_t*)pb->mem.get(sizeof(int32_t) * (size_t)std::max<int64_t>(R->ng, 1));
    R->rnode = (int64_t*)pb->mem.get(sizeof(int64_t) * (size_t)std::max<int64_t>(R->nr, 1));
    if (!R->gfine || !R->gpar || !R->gnp || !R->rnode) return pbi_fail(PB_ENOMEM, "refinement lists");
    if (R->ng)
        k_list_assign<<<nbD, 256, 0, s>>>(0, gc, gf, R->rolef, R->rolec, startD, R->gfine, R->gpar, R->gnp, nullptr,
                                          bad);
    if (R->nr)
        k_list_assign<<<nbP, 256, 0, s>>>(1, gc, gf, R->rolef, R->rolec, startP, nullptr, nullptr, nullptr, R->rnode,
                                          bad);
    RCHK(hipGetLastError());

    // load: each charge on the corners of the cell that holds it (the fine cell inside a
    // refined coarse cell), 4 pi q trilinear, summed per node in atom order on the host; the
    // sums are scattered into the cleared vectors below, and the derived fine entries then go to
    // their parents
    std::vector<std::pair<int64_t, double>> depc, depf;
    for (int64_t a = 0; a < na; ++a) {
        int c[3];
        for (int d = 0; d < 3; ++d) {
            const double f = (xyz[3 * a + d] - o[d]) / H;
            double fl = std::floor(f);
            fl = std::min(std::max(fl, 0.0), (double)(P.n[d] - 2));
            c[d] = (int)fl;
        }
        const bool fine = hcell[((size_t)c[0] * R->nc[1] + c[1]) * R->nc[2] + c[2]] != 0;
        int base[3];
        double t[3];
        for (int d = 0; d < 3; ++d) {
            if (fine) {
                const double f = (xyz[3 * a + d] - o[d]) / (H / 2.0);
                double fl = std::floor(f);
                fl = std::min(std::max(fl, (double)(2 * c[d])), (double)(2 * c[d] + 1));
                base[d] = (int)fl - off[d];
                t[d] = f - fl;
            } else {
                const double f = (xyz[3 * a + d] - o[d]) / H;
                base[d] = c[d];
                t[d] = f - (double)c[d];
            }
        }
        for (int x = 0; x < 2; ++x)
            for (int y = 0; y < 2; ++y)
                for (int z = 0; z < 2; ++z) {
                    const double w = (x ? t[0] : 1.0 - t[0]) * (y ? t[1] : 1.0 - t[1]) * (z ? t[2] : 1.0 - t[2]);
                    const double v = 4.0 * kPi * chg[a] * w;
                    if (fine)
                        depf.emplace_back(gf.idx(base[0] + x, base[1] + y, base[2] + z), v);
                    else
                        depc.emplace_back(gc.idx(base[0] + x, base[1] + y, base[2] + z), v);
                }
    }
    // per element, 0 + the contributions in atom order (a stable sort keeps that order)
    auto sum_per_node = [](std::vector<std::pair<int64_t, double>>& d, std::vector<int64_t>& idx,
                           std::vector<double>& val) {
        std::stable_sort(d.begin(), d.end(),
                         [](const std::pair<int64_t, double>& x, const std::pair<int64_t, double>& y) {
                             return x.first < y.first;
                         });
        for (size_t u = 0; u < d.size();) {
            double acc = 0.0;
            size_t w = u;
            for (; w < d.size() && d[w].first == d[u].first; ++w) acc += d[w].second;
            idx.push_back(d[u].first);
            val.push_back(acc);
            u = w;
        }
    };
    std::vector<int64_t> ldc_i, ldf_i;
    std::vector<double> ldc_v, ldf_v;
    sum_per_node(depc, ldc_i, ldc_v);
    sum_per_node(depf, ldf_i, ldf_v);
    // solver vectors: b, r, z, p, q, D^-1 of each grid (x: the problems' own x)
    const size_t Nc = (size_t)gc.N, Nf = (size_t)gf.N;
    double** vc[6] = {&R->bc, &R->rc, &R->zc, &R->pc, &R->qc, &R->dc};
    double** vf[6] = {&R->bf, &R->rf, &R->zf, &R->pf, &R->qf, &R->df};
    for (int v = 0; v < 6; ++v) {
        *vc[v] = (double*)pb->mem.get(sizeof(double) * Nc);
        *vf[v] = (double*)pb->mem.get(sizeof(double) * Nf);
        if (!*vc[v] || !*vf[v]) return pbi_fail(PB_ENOMEM, "refined solver vectors");
        RCHK(launch_fill(s, *vc[v], sizeof(double) * Nc));
        RCHK(launch_fill(s, *vf[v], sizeof(double) * Nf));
    }
    std::vector<void*> tmp_dev;
    auto scatter = [&](const std::vector<int64_t>& idx, const std::vector<double>& val, double* dst) -> int {
        if (idx.empty()) return PB_OK;
        int64_t* di = (int64_t*)pb->mem.get(sizeof(int64_t) * idx.size());
        double* dv = (double*)pb->mem.get(sizeof(double) * val.size());
        if (!di || !dv) return pbi_fail(PB_ENOMEM, "refined charge load");
        tmp_dev.push_back(di);
        tmp_dev.push_back(dv);
        RCHK(hipMemcpyAsync(di, idx.data(), sizeof(int64_t) * idx.size(), hipMemcpyHostToDevice, s));
        RCHK(hipMemcpyAsync(dv, val.data(), sizeof(double) * val.size(), hipMemcpyHostToDevice, s));
        k_scatter<<<nblk((int64_t)idx.size(), 256), 256, 0, s>>>((int64_t)idx.size(), di, dv, dst);
        RCHK(hipGetLastError());
        return PB_OK;
    };
    if ((rc = scatter(ldc_i, ldc_v, R->bc))) return rc;
    if ((rc = scatter(ldf_i, ldf_v, R->bf))) return rc;
    if (R->nr) k_fold_load<<<nblk(R->nr, 256), 256, 0, s>>>(R->nr, R->rnode, gc, gf, R->rolef, R->bf, R->bc);
    if (R->ng) k_zero_derived<<<nblk(R->ng, 256), 256, 0, s>>>(R->ng, R->gfine, R->bf);
    k_lift<<<nblk(gc.N, 256), 256, 0, s>>>(gc, R->Kc, R->rolec, pb->code, pb->gb, R->bc);
    k_diag<<<nblk(gc.N, 256), 256, 0, s>>>(gc, R->Kc, R->rolec, R->dc);
    k_diag<<<nblk(gf.N, 256), 256, 0, s>>>(gf, R->Kf, R->rolef, R->df);
    if (R->ng) k_diag_fix<<<nblk(R->ng, 256), 256, 0, s>>>(R->ng, R->gfine, R->gpar, R->gnp, R->df, R->dc);
    k_invert<<<nblk(gc.N, 256), 256, 0, s>>>(gc.N, R->rolec, R->dc);
    k_invert<<<nblk(gf.N, 256), 256, 0, s>>>(gf.N, R->rolef, R->df);
    RCHK(hipGetLastError());
    R->nbc = (int)std::min<int64_t>(1024, (int64_t)nblk(gc.N, 256));
    R->nbf = (int)std::min<int64_t>(1024, (int64_t)nblk(gf.N, 256));
    R->part = (double*)pb->mem.get(sizeof(double) * 3 * (size_t)(R->nbc + R->nbf));
    if (!R->part) return pbi_fail(PB_ENOMEM, "refined partial sums");
    if (P.precision == PB_MIXED) {
        // FP32 operator and preconditioner, rounded once from the FP64 ones
        R->Kc32 = (float*)pb->mem.get(sizeof(float) * 4 * Nc);
        R->Kf32 = (float*)pb->mem.get(sizeof(float) * 4 * Nf);
        if (!R->Kc32 || !R->Kf32) return pbi_fail(PB_ENOMEM, "refined FP32 coefficients");
        float** wc[6] = {&R->xc32, &R->rc32, &R->zc32, &R->pc32, &R->qc32, &R->dc32};
        float** wf[6] = {&R->xf32, &R->rf32, &R->zf32, &R->pf32, &R->qf32, &R->df32};
        for (int v = 0; v < 6; ++v) {
            *wc[v] = (float*)pb->mem.get(sizeof(float) * Nc);
            *wf[v] = (float*)pb->mem.get(sizeof(float) * Nf);
            if (!*wc[v] || !*wf[v]) return pbi_fail(PB_ENOMEM, "refined FP32 solver vectors");
            RCHK(launch_fill(s, *wc[v], sizeof(float) * Nc));
            RCHK(launch_fill(s, *wf[v], sizeof(float) * Nf));
        }
        k_to_f32<<<nblk(4 * gc.N, 256), 256, 0, s>>>(4 * gc.N, R->Kc, R->Kc32);
        k_to_f32<<<nblk(4 * gf.N, 256), 256, 0, s>>>(4 * gf.N, R->Kf, R->Kf32);
        k_to_f32<<<nblk(gc.N, 256), 256, 0, s>>>(gc.N, R->dc, R->dc32);
        k_to_f32<<<nblk(gf.N, 256), 256, 0, s>>>(gf.N, R->df, R->df32);
        RCHK(hipGetLastError());
    }
    int hbad[2] = {0, 0};
    RCHK(hipMemcpyAsync(hbad, bad, sizeof hbad, hipMemcpyDeviceToHost, s));
    RCHK(hipStreamSynchronize(s));
    for (void* q : tmp_dev) pb->mem.put(q);
    pb->mem.put(startD);
    pb->mem.put(startP);
    pb->mem.put(cnt64);
    pb->mem.put(bad);
    if (hbad[0] & 1) return pbi_fail(PB_EINVAL, "a derived fine node has a parent that is not an unknown");
    if (hbad[0] & 2) return pbi_fail(PB_EINVAL, "a derived fine node is not on a coarse edge or face");
    return PB_OK;
}

namespace {

// the solver vectors of one grid in one precision
template <typename T>
struct GridVecs {
    T *x, *r, *z, *p, *q;
    const T *d, *K;
};

// w = A v over both grids with the operator of K arrays Kc, Kf (v's derived fine values are
// filled in first)
template <typename T>
void launch_apply_comp(hipStream_t s, const RefineData* R, const Grid& gc, const Grid& gf, const T* Kc, const T* Kf,
                       T* vc, T* vf, T* wc, T* wf, const CGState* st)
{
    if (R->ng) k_fill<T><<<nblk(R->ng, 256), 256, 0, s>>>(R->ng, R->gfine, R->gpar, R->gnp, vc, vf, st);
    k_apply<T><<<nblk(gc.N, 256), 256, 0, s>>>(gc, Kc, R->rolec, vc, wc, st);
    k_apply<T><<<nblk(gf.N, 256), 256, 0, s>>>(gf, Kf, R->rolef, vf, wf, st);
    if (R->nr)
        k_restrict<T><<<nblk(R->nr, 256), 256, 0, s>>>(R->nr, R->rnode, gc, gf, R->rolef, wf, wc,
                                                       st);
}

// z = B r in the element type T: on entry z = D^-1 r; the q vectors serve as scratch; the r.z
// partial sums go to part[0, nb).  st = null: ungated (inside a reliable update)
template <typename T>
void launch_two_level(hipStream_t s, pb_problem* pb, const Grid& gc, const Grid& gf, const Split& sp,
                      const GridVecs<T>& c, const GridVecs<T>& f, const CGState* st)
{
    RefineData* R = pb->ref;
    const int nb = R->nbc + R->nbf;
    T* bH = (T*)pbi_mg_rhs0(pb);
    T* eH = (T*)pbi_mg_sol0(pb);
    k_zscale<T><<<nb, 256, 0, s>>>(sp, c.z, f.z, st);
    launch_apply_comp<T>(s, R, gc, gf, c.K, f.K, c.z, f.z, c.q, f.q, st);
    k_rsub<T><<<nb, 256, 0, s>>>(sp, c.r, f.r, c.q, f.q, st);
    k_rest_h<T><<<nblk(gc.N, 256), 256, 0, s>>>(gc, gf, R->rolec, R->rolef, c.q, f.q, bH, st);
    pbi_mg_vcycle_on(pb, s, st);
    k_prol_c<T><<<nblk(gc.N, 256), 256, 0, s>>>(gc.N, R->rolec, eH, c.z, st);
    k_prol_f<T><<<nblk(gf.N, 256), 256, 0, s>>>(gf, gc, R->rolef, eH, f.z, st);
    launch_apply_comp<T>(s, R, gc, gf, c.K, f.K, c.z, f.z, c.q, f.q, st);
    k_post<T><<<nb, 256, 0, s>>>(sp, c.z, f.z, c.r, f.r, c.q, f.q, c.d, f.d, R->part, st);
}

// one composite CG iteration: q = P^T K P p, alpha, x and r, z = D^-1 r (or z = B r with
// two_level, the problem whose two-level preconditioner is used), beta, p
template <typename T>
void launch_iteration(hipStream_t s, const RefineData* R, const Grid& gc, const Grid& gf, const Split& sp,
                      const GridVecs<T>& c, const GridVecs<T>& f, CGState* st, pb_problem* two_level = nullptr)
{
    const int nb = R->nbc + R->nbf;
    if (R->ng) k_fill<T><<<nblk(R->ng, 256), 256, 0, s>>>(R->ng, R->gfine, R->gpar, R->gnp, c.p, f.p, st);
    k_apply<T><<<nblk(gc.N, 256), 256, 0, s>>>(gc, c.K, R->rolec, c.p, c.q, st);
    k_apply<T><<<nblk(gf.N, 256), 256, 0, s>>>(gf, f.K, R->rolef, f.p, f.q, st);
    if (R->nr)
        k_restrict<T><<<nblk(R->nr, 256), 256, 0, s>>>(R->nr, R->rnode, gc, gf, R->rolef, f.q, c.q,
                                                       st);
    k_dot<T><<<nb, 256, 0, s>>>(sp, c.p, c.q, f.p, f.q, R->part, st);
    k_alpha<<<1, 256, 0, s>>>(R->part, nb, st);
    k_update<T><<<nb, 256, 0, s>>>(sp, c.x, c.r, c.z, c.p, c.q, c.d, f.x, f.r, f.z, f.p, f.q, f.d, R->part, nb, st);
    if (two_level) launch_two_level<T>(s, two_level, gc, gf, sp, c, f, st);
    k_beta<<<1, 256, 0, s>>>(R->part, nb, st, 0, 0.0);
    k_pupd<T><<<nblk(gc.N, 256), 256, 0, s>>>(gc.N, R->rolec, c.z, c.p, st);
    k_pupd<T><<<nblk(gf.N, 256), 256, 0, s>>>(gf.N, R->rolef, f.z, f.p, st);
}

// mixed precision: fold the FP32 correction into x, r = b - A x with the FP64 operator, and
// restart the FP32 recurrence from it (the direction p is kept)
// (two_level: z = B r in place of D^-1 r after the replacement)
void launch_reliable_update(hipStream_t s, pb_problem* pb, const Split& sp, int init, double rtol2, double delta2,
                            bool two_level)
{
    RefineData* R = pb->ref;
    pb_problem* fp = R->fine;
    const Grid& gc = pb->g;
    const Grid& gf = fp->g;
    const int nb = R->nbc + R->nbf;
    k_fold<<<nb, 256, 0, s>>>(sp, pb->x, R->xc32, fp->x, R->xf32);
    if (R->ng)
        k_fill<double><<<nblk(R->ng, 256), 256, 0, s>>>(R->ng, R->gfine, R->gpar, R->gnp, pb->x, fp->x, nullptr);
    k_apply<double><<<nblk(gc.N, 256), 256, 0, s>>>(gc, R->Kc, R->rolec, pb->x, R->qc, nullptr);
    k_apply<double><<<nblk(gf.N, 256), 256, 0, s>>>(gf, R->Kf, R->rolef, fp->x, R->qf, nullptr);
    if (R->nr)
        k_restrict<double><<<nblk(R->nr, 256), 256, 0, s>>>(R->nr, R->rnode, gc, gf, R->rolef, R->qf,
                                                            R->qc, nullptr);
    k_true_res<<<nb, 256, 0, s>>>(sp, R->bc, R->qc, R->rc, R->bf, R->qf, R->rf, R->part + 2 * nb);
    k_replace<<<nb, 256, 0, s>>>(sp, R->rc, R->rc32, R->zc32, R->dc32, R->rf, R->rf32, R->zf32, R->df32, R->part, nb);
    if (two_level) {
        const GridVecs<float> c32{R->xc32, R->rc32, R->zc32, R->pc32, R->qc32, R->dc32, R->Kc32};
        const GridVecs<float> f32{R->xf32, R->rf32, R->zf32, R->pf32, R->qf32, R->df32, R->Kf32};
        launch_two_level<float>(s, pb, gc, gf, sp, c32, f32, nullptr);
    }
    k_ru_fin<<<1, 256, 0, s>>>(R->part, nb, pb->st, init, rtol2, delta2);
}

}  // namespace

// composite Jacobi-CG; fills the derived fine values of the solution at the end.  In mixed
// precision the iterations run in FP32 on a correction to the FP64 solution, and a reliable
// update (fold, FP64 true residual, restart) follows each time the FP32 residual norm falls by
// inner_rtol or reaches the goal; the FP64 residual decides convergence.
int pbi_refine_solve(pb_problem* pb, CGState* out)
{
    RefineData* R = pb->ref;
    pb_problem* fp = R->fine;
    const Grid& gc = pb->g;
    const Grid& gf = fp->g;
    hipStream_t s = pb->ctx->stream;
    const pb_params& P = pb->prm;
    const bool mixed = P.precision == PB_MIXED;
    const int nb = R->nbc + R->nbf;
    CGState* st = pb->st;
    const Split sp{gc.N, gf.N, R->nbc, R->rolec, R->rolef};
    const unsigned bc = nblk(gc.N, 256), bfn = nblk(gf.N, 256);
    const GridVecs<double> c64{pb->x, R->rc, R->zc, R->pc, R->qc, R->dc, R->Kc};
    const GridVecs<double> f64{fp->x, R->rf, R->zf, R->pf, R->qf, R->df, R->Kf};
    const GridVecs<float> c32{R->xc32, R->rc32, R->zc32, R->pc32, R->qc32, R->dc32, R->Kc32};
    const GridVecs<float> f32{R->xf32, R->rf32, R->zf32, R->pf32, R->qf32, R->df32, R->Kf32};
    // the two-level preconditioner (FP64): the coarse grid's multigrid hierarchy, once
    const bool two_level = P.precond == PB_PRECOND_MG;
    if (two_level && !pb->mg) {
        const int rc = pbi_mg_begin(pb, s);
        if (rc) return rc;
    }
    RCHK(launch_fill(s, pb->x, sizeof(double) * (size_t)gc.N));
    RCHK(launch_fill(s, fp->x, sizeof(double) * (size_t)gf.N));
    k_state_init<<<1, 1, 0, s>>>(st);
    if (mixed) {
        // x32 = 0; r = b, z = D^-1 r from the first reliable update; p = z
        RCHK(launch_fill(s, R->xc32, sizeof(float) * (size_t)gc.N));
        RCHK(launch_fill(s, R->xf32, sizeof(float) * (size_t)gf.N));
        launch_reliable_update(s, pb, sp, 1, P.rtol * P.rtol, P.inner_rtol * P.inner_rtol, two_level);
        k_pupd<float><<<bc, 256, 0, s>>>(gc.N, R->rolec, R->zc32, R->pc32, st);
        k_pupd<float><<<bfn, 256, 0, s>>>(gf.N, R->rolef, R->zf32, R->pf32, st);
    } else {
        // x = 0, r = b; the first update with alpha = 0 and p = q = 0 leaves x, r and forms z
        // and the norms; p = z
        RCHK(hipMemcpyAsync(R->rc, R->bc, sizeof(double) * (size_t)gc.N, hipMemcpyDeviceToDevice, s));
        RCHK(hipMemcpyAsync(R->rf, R->bf, sizeof(double) * (size_t)gf.N, hipMemcpyDeviceToDevice, s));
        RCHK(launch_fill(s, R->pc, sizeof(double) * (size_t)gc.N));
        RCHK(launch_fill(s, R->pf, sizeof(double) * (size_t)gf.N));
        RCHK(launch_fill(s, R->qc, sizeof(double) * (size_t)gc.N));
        RCHK(launch_fill(s, R->qf, sizeof(double) * (size_t)gf.N));
        k_update<double><<<nb, 256, 0, s>>>(sp, c64.x, c64.r, c64.z, c64.p, c64.q, c64.d, f64.x, f64.r, f64.z, f64.p,
                                            f64.q, f64.d, R->part, nb, st);
        if (two_level) launch_two_level<double>(s, pb, gc, gf, sp, c64, f64, st);
        k_beta<<<1, 256, 0, s>>>(R->part, nb, st, 1, P.rtol * P.rtol);
        k_pupd<double><<<bc, 256, 0, s>>>(gc.N, R->rolec, R->zc, R->pc, st);
        k_pupd<double><<<bfn, 256, 0, s>>>(gf.N, R->rolef, R->zf, R->pf, st);
    }
    RCHK(hipGetLastError());
    const int M = 16;
    int launched = 0;
    bool breakdown = false;
    CGState h;
    RCHK(hipMemcpyAsync(&h, st, sizeof(CGState), hipMemcpyDeviceToHost, s));
    RCHK(hipStreamSynchronize(s));
    while (h.status == 0 && launched < P.max_iter) {
        const int n = std::min(M, P.max_iter - launched);
        for (int it = 0; it < n; ++it) {
            if (mixed)
                launch_iteration<float>(s, R, gc, gf, sp, c32, f32, st, two_level ? pb : nullptr);
            else
                launch_iteration<double>(s, R, gc, gf, sp, c64, f64, st, two_level ? pb : nullptr);
        }
        RCHK(hipGetLastError());
        launched += n;
        RCHK(hipMemcpyAsync(&h, st, sizeof(CGState), hipMemcpyDeviceToHost, s));
        RCHK(hipStreamSynchronize(s));
        if (mixed && (h.status != 0 || launched >= P.max_iter)) {
            // status 3: the FP32 residual reached its goal or fell by inner_rtol
            breakdown = h.status == 2;
            launch_reliable_update(s, pb, sp, 0, 0.0, 0.0, two_level);
            if (!breakdown && launched < P.max_iter) {
                k_pupd<float><<<bc, 256, 0, s>>>(gc.N, R->rolec, R->zc32, R->pc32, st);
                k_pupd<float><<<bfn, 256, 0, s>>>(gf.N, R->rolef, R->zf32, R->pf32, st);
            }
            RCHK(hipGetLastError());
            RCHK(hipMemcpyAsync(&h, st, sizeof(CGState), hipMemcpyDeviceToHost, s));
            RCHK(hipStreamSynchronize(s));
            if (breakdown) break;
        }
    }
    // derived fine values of the solution, and the coarse copies of the fine-owned nodes
    if (R->ng)
        k_fill<double><<<nblk(R->ng, 256), 256, 0, s>>>(R->ng, R->gfine, R->gpar, R->gnp, pb->x, fp->x, nullptr);
    k_sync_coarse<<<bc, 256, 0, s>>>(gc, gf, R->rolec, pb->code, fp->x, pb->x);
    RCHK(hipGetLastError());
    RCHK(hipMemcpyAsync(out, st, sizeof(CGState), hipMemcpyDeviceToHost, s));
    RCHK(hipStreamSynchronize(s));
    if (breakdown && out->status != 1) out->status = 2;
    return PB_OK;
}
