// pb_build.hip -- coefficient-map construction on the GPU (gfx950).
//
// Steps (paper Sect. 2.1, 3.1, 3.2, 3.3.2):
//   atom cell list -> node classification (solute iff strictly inside an atom ball) ->
//   ordered compaction of the surface-crossing edges -> first-exit crossing geometry and
//   WHA edge coefficients -> trilinear charge load -> boundary values (Sect. 2.3) ->
//   diagonal, Jacobi inverse and boundary lift -> marching-cubes area weights.
//
// Every kernel is deterministic: no floating-point atomics, fixed summation orders.
// Geometry that decides a node's medium is evaluated without contraction so that the
// classification is bit-identical to the plain definition x = origin + h*i,
// d2 = (dx*dx + dy*dy) + dz*dz, solute iff d2 < R*R.
#include "pb_internal.h"
#include "pb_stencil.h"

#include <algorithm>
#include <type_traits>
#include <cmath>

namespace pbk {

namespace {

constexpr double kPi = 3.14159265358979323846;

__device__ __forceinline__ void decode(const Grid& g, int64_t e, int& i, int& j, int& k)
{
    int64_t row = e / g.S;
    k = (int)(e - row * g.S) - Z0;
    j = (int)(row % g.ny);
    i = (int)(row / g.ny);
}

__device__ __forceinline__ bool is_box(const Grid& g, int i, int j, int k)
{
    return i == 0 || j == 0 || k == 0 || i == g.nx - 1 || j == g.ny - 1 || k == g.nz - 1;
}

__device__ __forceinline__ double node_x(const Grid& g, int ax, int i)
{
#pragma clang fp contract(off)
    double o = ax == 0 ? g.ox : ax == 1 ? g.oy : g.oz;
    return o + g.h * (double)(i + g.off[ax]);
}

// range of bins to visit around point p (clamped); false when no atom can be within bs
__device__ __forceinline__ bool bin_range(const Bins& b, const double* p, int* lo, int* hi)
{
    const double l[3] = {b.lox, b.loy, b.loz};
    const int nb[3] = {b.nbx, b.nby, b.nbz};
    for (int d = 0; d < 3; ++d) {
        double f = floor((p[d] - l[d]) / b.bs);
        if (f < -1.0 || f > (double)nb[d]) return false;
        int c = (int)f;
        lo[d] = c - 1 < 0 ? 0 : c - 1;
        hi[d] = c + 1 > nb[d] - 1 ? nb[d] - 1 : c + 1;
    }
    return true;
}

// ---- cell list -----------------------------------------------------------------------

__device__ __forceinline__ int atom_bin(const Bins& b, const double* c)
{
    int x = (int)floor((c[0] - b.lox) / b.bs);
    int y = (int)floor((c[1] - b.loy) / b.bs);
    int z = (int)floor((c[2] - b.loz) / b.bs);
    return (x * b.nby + y) * b.nbz + z;
}

__global__ void k_bin_count(Atoms at, Bins b, int* cnt)
{
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= at.n) return;
    atomicAdd(&cnt[atom_bin(b, at.xyzr + 4 * a)], 1);
}

__global__ void k_bin_scatter(Atoms at, Bins b, int* cursor, int* ids)
{
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= at.n) return;
    int pos = atomicAdd(&cursor[atom_bin(b, at.xyzr + 4 * a)], 1);
    ids[pos] = a;
}

// the atoms' centres and radii in bin order (slot u holds atom ids[u]), so that the loops
// over a bin's atoms read them without first loading their ids
__global__ void k_bin_gather(Atoms at, const int* __restrict__ ids, double* __restrict__ xyzr_b)
{
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= at.n) return;
    const int a = ids[u];
    for (int d = 0; d < 4; ++d) xyzr_b[4 * u + d] = at.xyzr[4 * a + d];
}

// the scatter order depends on scheduling; sorting each bin makes the list deterministic
__global__ void k_bin_sort(int nbins, const int* start, int* ids)
{
    int bi = blockIdx.x * blockDim.x + threadIdx.x;
    if (bi >= nbins) return;
    int s = start[bi], e = start[bi + 1];
    for (int x = s + 1; x < e; ++x) {
        int v = ids[x];
        int y = x - 1;
        while (y >= s && ids[y] > v) {
            ids[y + 1] = ids[y];
            --y;
        }
        ids[y + 1] = v;
    }
}

// single-block exclusive scan of n ints into out[0..n] (out[n] = total; out may be in), in
// tiles of 4096: each thread takes four consecutive elements, the 1024 partial sums of a tile
// are scanned with wave shuffles and a pass over the 16 wave totals, and the running total
// carries from tile to tile.  Each element is read before it is written, by the same thread,
// so in == out is safe.
__global__ void __launch_bounds__(1024) k_scan1(const int* in, int n, int* out)
{
    __shared__ int wtot[16];
    const int lane = (int)(threadIdx.x & 63), w = (int)(threadIdx.x >> 6);
    int carry = 0;
    for (int base = 0; base < n; base += 4096) {
        const int e0 = base + 4 * (int)threadIdx.x;
        int v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = e0 + u < n ? in[e0 + u] : 0;
        const int s = (v[0] + v[1]) + (v[2] + v[3]);
        int incl = s;
        for (int off = 1; off < 64; off <<= 1) {
            const int t = __shfl_up(incl, off, 64);
            if (lane >= off) incl += t;
        }
        if (lane == 63) wtot[w] = incl;
        __syncthreads();
        int before = 0, total = 0;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int t = wtot[q];
            before += q < w ? t : 0;
            total += t;
        }
        int run = carry + before + incl - s;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (e0 + u < n) out[e0 + u] = run;
            run += v[u];
        }
        carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) out[n] = carry;
}

// ---- classification -------------------------------------------------------------------

__global__ void __launch_bounds__(256) k_classify(Grid g, Bins b, const double* __restrict__ xb, uint32_t* code)
{
#pragma clang fp contract(off)
    int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= g.N) return;
    int i, j, k;
    decode(g, e, i, j, k);
    if (k < 0 || k >= g.nz) {
        code[e] = C_BOX;
        return;
    }
    if (is_box(g, i, j, k)) {
        code[e] = C_BOX;
        return;
    }
    double p[3] = {node_x(g, 0, i), node_x(g, 1, j), node_x(g, 2, k)};
    uint32_t c = 0;
    int lo[3], hi[3];
    if (bin_range(b, p, lo, hi)) {
        for (int x = lo[0]; x <= hi[0] && !c; ++x)
            for (int y = lo[1]; y <= hi[1] && !c; ++y)
                for (int z = lo[2]; z <= hi[2] && !c; ++z) {
                    int bi = (x * b.nby + y) * b.nbz + z;
                    for (int t = b.start[bi]; t < b.start[bi + 1]; ++t) {
                        const double* a = xb + 4 * t;
                        double dx = p[0] - a[0], dy = p[1] - a[1], dz = p[2] - a[2];
                        double d2 = dx * dx + dy * dy + dz * dz;
                        if (d2 < a[3] * a[3]) {
                            c = C_SOLUTE;
                            break;
                        }
                    }
                }
    }
    code[e] = c;
}

// ---- ordered compaction of cut edges -----------------------------------------------------

__device__ __forceinline__ uint32_t cut_bits(const Grid& g, const uint32_t* cls, int64_t e)
{
    int i, j, k;
    decode(g, e, i, j, k);
    if (k < 0 || k >= g.nz) return 0;
    uint32_t s = cls[e] & C_SOLUTE, m = 0;
    if (i + 1 < g.nx && ((cls[e + (int64_t)g.ny * g.S] & C_SOLUTE) != s)) m |= 1u;
    if (j + 1 < g.ny && ((cls[e + g.S] & C_SOLUTE) != s)) m |= 2u;
    if (k + 1 < g.nz && ((cls[e + 1] & C_SOLUTE) != s)) m |= 4u;
    return m;
}

// exclusive block scan of one int over 256 threads (4 waves of 64)
__device__ __forceinline__ int block_exscan(int v, int* sh, int& total)
{
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int x = v;
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(x, o, 64);
        if (lane >= o) x += t;
    }
    if (lane == 63) sh[w] = x;
    __syncthreads();
    int off = 0;
    for (int q = 0; q < w; ++q) off += sh[q];
    total = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
    return off + x - v;
}

__global__ void __launch_bounds__(256) k_cutcount(Grid g, const uint32_t* cls, int* blk_slots, int* blk_cuts)
{
    __shared__ int sh[4];
    int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    uint32_t m = e < g.N ? cut_bits(g, cls, e) : 0;
    int t1, t2;
    block_exscan(m ? 1 : 0, sh, t1);
    block_exscan(__popc(m), sh, t2);
    if (threadIdx.x == 0) {
        blk_slots[blockIdx.x] = t1;
        blk_cuts[blockIdx.x] = t2;
    }
}

__global__ void __launch_bounds__(256) k_assign(Grid g, const uint32_t* cls, uint32_t* code,
                                                const int* blk_slots, const int* blk_cuts,
                                                int* cutbase, int64_t* cutkey)
{
    __shared__ int sh[4];
    int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    uint32_t m = e < g.N ? cut_bits(g, cls, e) : 0;
    int t1, t2;
    int ps = block_exscan(m ? 1 : 0, sh, t1) + blk_slots[blockIdx.x];
    int pc = block_exscan(__popc(m), sh, t2) + blk_cuts[blockIdx.x];
    if (e >= g.N) return;
    uint32_t c = cls[e] | (m << 2);
    if (m) {
        c |= (uint32_t)ps << C_SLOT_SHIFT;
        cutbase[ps] = pc;
        for (int ax = 0; ax < 3; ++ax)
            if (m & (1u << ax)) cutkey[pc++] = e * 4 + ax;
    }
    code[e] = c;
}

// ---- crossing geometry (first exit from the union of balls) -----------------------------

__global__ void __launch_bounds__(256) k_cut_geom(Grid g, Bins b, const double* __restrict__ xb, Atoms at,
                                                  double eps_in, double eps_out,
                                                  int64_t ncut, const int64_t* cutkey,
                                                  const uint32_t* code, double* alpha, double* kcut,
                                                  double* rp, double* np, int* owner, double* ck64,
                                                  float* ck32)
{
#pragma clang fp contract(off)
    int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= ncut) return;
    int64_t key = cutkey[c];
    int64_t e = key >> 2;
    int ax = (int)(key & 3);
    int i, j, k;
    decode(g, e, i, j, k);
    int lo_n[3] = {i, j, k}, hi_n[3] = {i, j, k};
    hi_n[ax] += 1;
    bool low_solute = (code[e] & C_SOLUTE) != 0;
    double s[3], w[3];
    for (int d = 0; d < 3; ++d) {
        double a = node_x(g, d, lo_n[d]), bb = node_x(g, d, hi_n[d]);
        s[d] = low_solute ? a : bb;
        w[d] = low_solute ? bb : a;
    }
    (void)w;
    double dir = low_solute ? 1.0 : -1.0;
    int lo[3], hi[3];
    double t = 0.0;
    int ow = -1;
    if (bin_range(b, s, lo, hi)) {
        for (;;) {
            double tn = t;
            for (int x = lo[0]; x <= hi[0]; ++x)
                for (int y = lo[1]; y <= hi[1]; ++y)
                    for (int z = lo[2]; z <= hi[2]; ++z) {
                        int bi = (x * b.nby + y) * b.nbz + z;
                        for (int u = b.start[bi]; u < b.start[bi + 1]; ++u) {
                            const double* a = xb + 4 * u;
                            double dperp2 = 0.0;
                            for (int d = 0; d < 3; ++d) {
                                if (d == ax) continue;
                                double dd = s[d] - a[d];
                                dperp2 = dperp2 + dd * dd;
                            }
                            double R2 = a[3] * a[3];
                            if (!(dperp2 < R2)) continue;
                            double half = sqrt(R2 - dperp2);
                            double tc = (a[ax] - s[ax]) * dir;
                            double clo = tc - half, chi = tc + half;
                            if (clo <= t && t < chi && chi > tn) tn = chi;
                        }
                    }
            if (tn == t) break;
            t = tn;
        }
        for (int x = lo[0]; x <= hi[0]; ++x)
            for (int y = lo[1]; y <= hi[1]; ++y)
                for (int z = lo[2]; z <= hi[2]; ++z) {
                    int bi = (x * b.nby + y) * b.nbz + z;
                    for (int u = b.start[bi]; u < b.start[bi + 1]; ++u) {
                        int id = b.ids[u];
                        const double* a = xb + 4 * u;
                        double dperp2 = 0.0;
                        for (int d = 0; d < 3; ++d) {
                            if (d == ax) continue;
                            double dd = s[d] - a[d];
                            dperp2 = dperp2 + dd * dd;
                        }
                        double R2 = a[3] * a[3];
                        if (!(dperp2 < R2)) continue;
                        double half = sqrt(R2 - dperp2);
                        double tc = (a[ax] - s[ax]) * dir;
                        double clo = tc - half, chi = tc + half;
                        if (chi == t && clo < t && (ow < 0 || id < ow)) ow = id;
                    }
                }
    }
    if (t > g.h) t = g.h;
    if (ow < 0) ow = 0;  // unreachable for a valid solute end; keeps indexing in range
    double al = t / g.h;
    double ee = 1.0 / (al / eps_in + (1.0 - al) / eps_out);
    double K = g.h * ee;
    alpha[c] = al;
    kcut[c] = K;
    const double* ao = at.xyzr + 4 * ow;
    for (int d = 0; d < 3; ++d) {
        double r = (d == ax) ? s[d] + dir * t : s[d];
        rp[3 * c + d] = r;
        np[3 * c + d] = (r - ao[d]) / ao[3];
    }
    owner[c] = ow;
    uint32_t slot = code[e] >> C_SLOT_SHIFT;
    ck64[3 * (int64_t)slot + ax] = K;
    ck32[3 * (int64_t)slot + ax] = (float)K;
}

// ---- load vector ------------------------------------------------------------------------

// per atom: the grid cell that receives its charge (floor of its grid coordinates, clamped
// to the cells of the grid) and its offsets in that cell: ac[6a + d] = t_d, ac[6a + 3 + d] =
// the cell index along d
// the grid cell holding atom a (its low corner, clamped into the grid) and the atom's
// fractional position in it along each axis
__device__ __forceinline__ void atom_cell(const Grid& g, const Atoms& at, int a, double* t, double* fl)
{
#pragma clang fp contract(off)
    const int nn[3] = {g.nx, g.ny, g.nz};
    const double org[3] = {g.ox, g.oy, g.oz};
    for (int d = 0; d < 3; ++d) {
        const double f = (at.xyzr[4 * a + d] - org[d]) / g.h - (double)g.off[d];
        double c = floor(f);
        if (c < 0) c = 0;
        if (c > nn[d] - 2) c = nn[d] - 2;
        t[d] = f - c;
        fl[d] = c;
    }
}

// per slot u of the cell list (atom ids[u]): the atom's deposition cell offsets t, its cell
// fl and its charge, 8 doubles in bin order
__global__ void __launch_bounds__(256) k_atom_cells(Grid g, Atoms at, const int* __restrict__ ids, double* ac)
{
    const int u = blockIdx.x * 256 + threadIdx.x;
    if (u >= at.n) return;
    const int a = ids[u];
    double t[3], fl[3];
    atom_cell(g, at, a, t, fl);
    for (int d = 0; d < 3; ++d) {
        ac[8 * u + d] = t[d];
        ac[8 * u + 3 + d] = fl[d];
    }
    ac[8 * u + 6] = at.q[a];
    ac[8 * u + 7] = 0.0;
}

// sum of v over the 256 threads of a block, the same value in every thread
__device__ __forceinline__ double block_total(double v, double* sh)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// Grid energy (Sect. 3.3, electrostatic energy): half the sum over grid nodes of the charge
// deposited there times the potential there.  Summed per atom instead of per node: atom a
// contributes q_a times the potential at the eight corners of its cell with the deposition's
// trilinear weights; box nodes hold no deposited charge and are left out.  part[b] = the
// sum over the atoms of block b.
__global__ void __launch_bounds__(256) k_grid_energy(Grid g, Atoms at, const double* __restrict__ x,
                                                     double* __restrict__ part)
{
#pragma clang fp contract(off)
    __shared__ double sh[4];
    const int a = blockIdx.x * 256 + threadIdx.x;
    double v = 0.0;
    if (a < at.n) {
        double t[3], fl[3];
        atom_cell(g, at, a, t, fl);
        const int c0[3] = {(int)fl[0], (int)fl[1], (int)fl[2]};
        for (int c = 0; c < 8; ++c) {
            const int i = c0[0] + ((c >> 2) & 1), j = c0[1] + ((c >> 1) & 1), k = c0[2] + (c & 1);
            if (is_box(g, i, j, k)) continue;
            double w = 1.0;
            w = w * ((c & 4) ? t[0] : 1.0 - t[0]);
            w = w * ((c & 2) ? t[1] : 1.0 - t[1]);
            w = w * ((c & 1) ? t[2] : 1.0 - t[2]);
            v += w * x[g.idx(i, j, k)];
        }
        v *= at.q[a];
    }
    v = block_total(v, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// one block: scale times the sum of part[0..nb), combined in a fixed order; written to part[nb]
__global__ void __launch_bounds__(256) k_grid_energy_total(double* part, int nb, double scale)
{
    __shared__ double sh[4];
    double v = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) v += part[b];
    v = block_total(v, sh);
    if (threadIdx.x == 0) part[nb] = scale * v;
}

// the bins that can hold an atom depositing charge at the node p: the atom's deposition cell
// is one of the eight cells around the node, so its centre lies within one spacing h of p on
// every axis (widened by h/1000, far beyond the rounding of either position); false when no
// bin is in reach.  The bin edge is at least 2h, so these bins are a sub-range of
// bin_range's, visited in the same order: the sum over the atoms is the same to the bit.
__device__ __forceinline__ bool bin_range_node(const Bins& b, const double* p, double h, int* lo, int* hi)
{
    const double l[3] = {b.lox, b.loy, b.loz};
    const int nb[3] = {b.nbx, b.nby, b.nbz};
    const double w = 1.001 * h;
    for (int d = 0; d < 3; ++d) {
        const double a = floor((p[d] - w - l[d]) / b.bs), c = floor((p[d] + w - l[d]) / b.bs);
        if (c < 0.0 || a > (double)(nb[d] - 1)) return false;
        lo[d] = a < 0.0 ? 0 : (int)a;
        hi[d] = c > (double)(nb[d] - 1) ? nb[d] - 1 : (int)c;
    }
    return true;
}

__global__ void __launch_bounds__(256) k_deposit(Grid g, Bins b, const double* __restrict__ ac, double* rhs)
{
#pragma clang fp contract(off)
    int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= g.N) return;
    int i, j, k;
    decode(g, e, i, j, k);
    if (k < 0 || k >= g.nz || is_box(g, i, j, k)) {
        rhs[e] = 0.0;
        return;
    }
    double p[3] = {node_x(g, 0, i), node_x(g, 1, j), node_x(g, 2, k)};
    const int nd[3] = {i, j, k};
    double sum = 0.0;
    int lo[3], hi[3];
    if (bin_range_node(b, p, g.h, lo, hi)) {
        for (int x = lo[0]; x <= hi[0]; ++x)
            for (int y = lo[1]; y <= hi[1]; ++y)
                for (int z = lo[2]; z <= hi[2]; ++z) {
                    int bi = (x * b.nby + y) * b.nbz + z;
                    for (int u = b.start[bi]; u < b.start[bi + 1]; ++u) {
                        const double* c6 = ac + 8 * u;
                        double w = 1.0;
                        bool corner = true;
                        for (int d = 0; d < 3; ++d) {
                            const int cl = (int)c6[3 + d];
                            const double t = c6[d];
                            if (nd[d] == cl) w = w * (1.0 - t);
                            else if (nd[d] == cl + 1) w = w * t;
                            else corner = false;
                        }
                        if (corner) sum += 4.0 * kPi * c6[6] * w;
                    }
                }
    }
    rhs[e] = sum;
}

// ---- boundary values ----------------------------------------------------------------------

__device__ __forceinline__ void box_node(const Grid& g, int64_t t, int& i, int& j, int& k)
{
    const int64_t fx = (int64_t)g.ny * g.nz, fy = (int64_t)(g.nx - 2) * g.nz,
                  fz = (int64_t)(g.nx - 2) * (g.ny - 2);
    if (t < 2 * fx) {
        i = t < fx ? 0 : g.nx - 1;
        int64_t r = t % fx;
        j = (int)(r / g.nz);
        k = (int)(r % g.nz);
    } else if ((t -= 2 * fx) < 2 * fy) {
        j = t < fy ? 0 : g.ny - 1;
        int64_t r = t % fy;
        i = 1 + (int)(r / g.nz);
        k = (int)(r % g.nz);
    } else {
        t -= 2 * fy;
        k = t < fz ? 0 : g.nz - 1;
        int64_t r = t % fz;
        i = 1 + (int)(r / (g.ny - 2));
        j = 1 + (int)(r % (g.ny - 2));
    }
}

__device__ __forceinline__ int64_t n_box(const Grid& g)
{
    return 2 * ((int64_t)g.ny * g.nz + (int64_t)(g.nx - 2) * g.nz + (int64_t)(g.nx - 2) * (g.ny - 2));
}

// exp(-kD r) for r >= 0 in FP64 by Tang's table-driven method (P. T. P. Tang, ACM TOMS 15(2),
// 1989) with the factor -kD folded into the constants: n = round(-kD r 2048 / ln 2), from the
// round-to-nearest of a 1.5 * 2^52 shift, and s = r + n L with L = ln 2 / (2048 kD), so that
// -kD r = (n / 2048) ln 2 - kD s with kD |s| <= ln 2 / 4096.  Then exp(-kD r) = 2^(n >> 11)
// 2^((n & 2047) / 2048) e^(-kD s), the last factor from its Taylor polynomial to degree 3
// (truncation under 4e-17 relative), the table T[j] = 2^(j / 2048) formed once per block.  L is
// one FP64 number: its rounding moves s by about r 1e-16, which changes the result by about
// kD r 1e-16 relative, the size of the rounding of the argument -kD r itself (Tang splits ln 2
// in two parts for an argument given exactly; here r carries a rounding of its own).
__device__ __forceinline__ double exp_dh(double r, const DhExp& E, const double* T)
{
    const double shift = 6755399441055744.0;   // 1.5 * 2^52
    const double t = fma(r, E.tscale, shift);
    const int n = __double2loint(t);
    const double s = fma(t - shift, E.L, r);
    const double p = fma(fma(fma(s, E.c3, E.c2), s, E.c1), s, 1.0);
    return ldexp(T[n & (kDhTable - 1)] * p, n >> 11);
}

// Debye-Hueckel values at the box nodes in FP64 (Sect. 2.3, the Debye-Hueckel form):
// g(x) = sum over atoms of q exp(-kD r) / (eps_out r).  The box nodes are taken face by face:
// on a face with normal axis w and in-plane axes u, v the squared distance separates,
// r^2 = (w0 - a_w)^2 + (u - a_u)^2 + (v - a_v)^2, so a thread that owns DH_PU x DH_PV nodes of
// a face forms the u and v terms of an atom once per row and column of its patch and each
// pair's r^2 in one add (2.75 operations per pair instead of four for |p|^2 + |a|^2 - 2 a.p),
// from exact coordinate differences taken relative to the atoms' centre.  Then 1/r by
// rsqrt_fp64, r = r^2 (1/r) and exp(-kD r) by exp_dh; without salt (kD = 0) the exponential is
// skipped.  A face's patches are numbered row by row (no padding to block tiles, so only the
// last patch of a row or column is partly outside the face), 256 to a block; block b takes
// block b % blocks of the faces and the atoms of range b / blocks (staged in LDS with the
// face's own w term); its partial sums go to part[range][node] (the box-node numbering of
// box_node), which k_bc_dh_sum adds up in range order.
constexpr int DH_PU = 2, DH_PV = 4;
constexpr int DH_GROUP = 32;   // atoms per FP32 partial sum of the mixed kernel   // nodes per thread along u, v

// a thread's patch of box-face nodes: its face (normal axis w, in-plane axes ua slower and va
// faster), the patch's first node (u0, v0) on the face's U x V array, and the coordinates,
// relative to the atoms' centre, of the face plane and of the patch's rows and columns
// (clamped to the face for a patch partly outside it)
struct DhPatch {
    int f, w, ua, va, U, V, u0, v0;
    bool act;
    double pw, pu[DH_PU], pv[DH_PV];
};

__device__ __forceinline__ DhPatch dh_patch(const Grid& g, const Atoms& at, const DhFaces& fc, int tile)
{
    DhPatch P;
    P.f = 0;
    while (P.f < 5 && tile >= fc.tile0[P.f + 1]) ++P.f;
    const int64_t patch = (int64_t)(tile - fc.tile0[P.f]) * 256 + threadIdx.x;
    P.w = P.f >> 1;
    P.ua = P.w == 0 ? 1 : 0;
    P.va = P.w == 2 ? 1 : 2;
    // a later axis's faces leave out the edge nodes that the earlier axes' faces hold
    const int ushift = P.w == 0 ? 0 : 1, vshift = P.w == 2 ? 1 : 0;
    P.U = fc.U[P.f];
    P.V = fc.V[P.f];
    P.u0 = (int)(patch / fc.pv[P.f]) * DH_PU;
    P.v0 = (int)(patch % fc.pv[P.f]) * DH_PV;
    P.act = patch < fc.np[P.f];
    const double cen[3] = {at.cx, at.cy, at.cz};
    const int nn[3] = {g.nx, g.ny, g.nz};
    P.pw = node_x(g, P.w, (P.f & 1) ? nn[P.w] - 1 : 0) - cen[P.w];
#pragma unroll
    for (int a = 0; a < DH_PU; ++a) P.pu[a] = node_x(g, P.ua, min(P.u0 + a, P.U - 1) + ushift) - cen[P.ua];
#pragma unroll
    for (int b = 0; b < DH_PV; ++b) P.pv[b] = node_x(g, P.va, min(P.v0 + b, P.V - 1) + vshift) - cen[P.va];
    return P;
}

// an atom's terms for the patch's face: (w0 - a_w)^2, a_u, a_v (relative to the atoms' centre)
__device__ __forceinline__ void dh_stage(const DhPatch& P, const Atoms& at, int a, double* out)
{
    const double* A = at.xyzr + 4 * a;
    const double cen[3] = {at.cx, at.cy, at.cz};
    const double dw = P.pw - (A[P.w] - cen[P.w]);
    out[0] = dw * dw;
    out[1] = A[P.ua] - cen[P.ua];
    out[2] = A[P.va] - cen[P.va];
}

// the squared distances of the patch's rows (with the face term) and columns to an atom
__device__ __forceinline__ void dh_terms(const DhPatch& P, const double* A, double* ru, double* rv)
{
#pragma unroll
    for (int a = 0; a < DH_PU; ++a) {
        const double d = P.pu[a] - A[1];
        ru[a] = fma(d, d, A[0]);
    }
#pragma unroll
    for (int b = 0; b < DH_PV; ++b) {
        const double d = P.pv[b] - A[2];
        rv[b] = d * d;
    }
}

__device__ __forceinline__ void dh_write(const DhPatch& P, const DhFaces& fc, const DhSplit& sp, int rg,
                                         const double (*s)[DH_PV], double* part)
{
#pragma unroll
    for (int a = 0; a < DH_PU; ++a)
#pragma unroll
        for (int b = 0; b < DH_PV; ++b)
            if (P.act && P.u0 + a < P.U && P.v0 + b < P.V)
                part[(int64_t)rg * sp.nbox + fc.base[P.f] + (int64_t)(P.u0 + a) * P.V + (P.v0 + b)] = s[a][b];
}

__global__ void __launch_bounds__(256) k_bc_dh(Grid g, Atoms at, DhExp E, DhSplit sp, DhFaces fc, double* part)
{
    __shared__ double sa[256 * 4];
    __shared__ double T[kDhTable];
    for (int j = threadIdx.x; j < kDhTable; j += 256) T[j] = exp2((double)j / kDhTable);
    const int tile = (int)(blockIdx.x % fc.tile0[6]), rg = (int)(blockIdx.x / fc.tile0[6]);
    const DhPatch P = dh_patch(g, at, fc, tile);
    double s[DH_PU][DH_PV];
#pragma unroll
    for (int a = 0; a < DH_PU; ++a)
#pragma unroll
        for (int b = 0; b < DH_PV; ++b) s[a][b] = 0.0;
    const bool salt = E.c1 != 0.0;
    const int a0 = rg * sp.per, a1 = min(at.n, a0 + sp.per);
    for (int base = a0; base < a1; base += 256) {
        const int at_i = base + threadIdx.x;
        __syncthreads();
        if (at_i < a1) {
            dh_stage(P, at, at_i, sa + 4 * threadIdx.x);
            sa[4 * threadIdx.x + 3] = at.q[at_i];
        }
        __syncthreads();
        const int m = a1 - base < 256 ? a1 - base : 256;
        if (!P.act) continue;
        auto body = [&](auto SALT) {
            for (int q = 0; q < m; ++q) {
                const double* A = sa + 4 * q;
                const double qq = A[3];
                double ru[DH_PU], rv[DH_PV];
                dh_terms(P, A, ru, rv);
#pragma unroll
                for (int a = 0; a < DH_PU; ++a)
#pragma unroll
                    for (int b = 0; b < DH_PV; ++b) {
                        const double r2 = ru[a] + rv[b];
                        const double y = rsqrt_fp64(r2);
                        if constexpr (decltype(SALT)::value)
                            s[a][b] = fma(qq * exp_dh(r2 * y, E, T), y, s[a][b]);
                        else
                            s[a][b] = fma(qq, y, s[a][b]);
                    }
            }
        };
        if (salt)
            body(std::true_type{});
        else
            body(std::false_type{});
    }
    dh_write(P, fc, sp, rg, s, part);
}

// The same sum for the mixed-precision form: the row and column terms of the squared
// distances in FP64 (as in k_bc_dh), rounded to FP32 once per atom and added in FP32, then the
// exponential and the inverse distance in FP32 (a few units in the last place, about 1e-7
// relative per term), summed in FP32 over groups of DH_GROUP atoms and the group sums in FP64
// (a group's rounding, about sqrt(DH_GROUP) units in the last place of its absolute sum, stays
// near the terms' own).  The box is tens of Angstrom from
// the surface, so these errors reach the surface potential screened by exp(-kD d) and stay
// far below the FP32 iteration's own rounding.  The hardware reciprocal square root and
// base-2 exponential are used directly: r^2 leaves the FP32 normal range only for an atom
// centre within 1e-19 A of a box node, where the sum is singular anyway, and an exponent
// below -126 gives 0 in place of a term under 1e-38.  Patches, ranges and partial sums as in
// k_bc_dh.
__global__ void __launch_bounds__(256) k_bc_dh32(Grid g, Atoms at, double kD, DhSplit sp, DhFaces fc, double* part)
{
    __shared__ double sa[256 * 3];
    __shared__ float sq[256];
    const int tile = (int)(blockIdx.x % fc.tile0[6]), rg = (int)(blockIdx.x / fc.tile0[6]);
    const DhPatch P = dh_patch(g, at, fc, tile);
    const float mk = (float)(-kD * 1.4426950408889634);   // -kD log2(e)
    double s[DH_PU][DH_PV];
#pragma unroll
    for (int a = 0; a < DH_PU; ++a)
#pragma unroll
        for (int b = 0; b < DH_PV; ++b) s[a][b] = 0.0;
    const int a0 = rg * sp.per, a1 = min(at.n, a0 + sp.per);
    for (int base = a0; base < a1; base += 256) {
        const int at_i = base + threadIdx.x;
        __syncthreads();
        if (at_i < a1) {
            dh_stage(P, at, at_i, sa + 3 * threadIdx.x);
            sq[threadIdx.x] = (float)at.q[at_i];
        }
        __syncthreads();
        const int m = a1 - base < 256 ? a1 - base : 256;
        if (!P.act) continue;
        // groups of DH_GROUP atoms summed in FP32, the group sums added in FP64
        for (int q0 = 0; q0 < m; q0 += DH_GROUP) {
            const int q1 = q0 + DH_GROUP < m ? q0 + DH_GROUP : m;
            float t[DH_PU][DH_PV];
#pragma unroll
            for (int a = 0; a < DH_PU; ++a)
#pragma unroll
                for (int b = 0; b < DH_PV; ++b) t[a][b] = 0.0f;
            for (int q = q0; q < q1; ++q) {
                double ru[DH_PU], rv[DH_PV];
                dh_terms(P, sa + 3 * q, ru, rv);
                float fu[DH_PU], fv[DH_PV];
#pragma unroll
                for (int a = 0; a < DH_PU; ++a) fu[a] = (float)ru[a];
#pragma unroll
                for (int b = 0; b < DH_PV; ++b) fv[b] = (float)rv[b];
                const float qq = sq[q];
#pragma unroll
                for (int a = 0; a < DH_PU; ++a)
#pragma unroll
                    for (int b = 0; b < DH_PV; ++b) {
                        const float r2 = fu[a] + fv[b];
                        const float ri = __builtin_amdgcn_rsqf(r2);
                        const float e = __builtin_amdgcn_exp2f(mk * (r2 * ri));
                        t[a][b] = fmaf(qq * e, ri, t[a][b]);
                    }
            }
#pragma unroll
            for (int a = 0; a < DH_PU; ++a)
#pragma unroll
                for (int b = 0; b < DH_PV; ++b) s[a][b] += (double)t[a][b];
        }
    }
    dh_write(P, fc, sp, rg, s, part);
}

// the box values from the partial sums of the atom ranges, added in range order
__global__ void __launch_bounds__(256) k_bc_dh_sum(Grid g, DhSplit sp, const double* part, double eps_out, double* gb)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= sp.nbox) return;
    double s = 0.0;
    for (int r = 0; r < sp.ranges; ++r) s += part[(int64_t)r * sp.nbox + t];
    int i, j, k;
    box_node(g, t, i, j, k);
    gb[g.idx(i, j, k)] = s / eps_out;
}

__global__ void __launch_bounds__(256) k_bc_user(Grid g, const double* full, double* gb)
{
    int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n_box(g)) return;
    int i, j, k;
    box_node(g, t, i, j, k);
    gb[g.idx(i, j, k)] = full[((int64_t)i * g.ny + j) * g.nz + k];
}

// ---- diagonal, Jacobi inverse, boundary lift ------------------------------------------------

__device__ __forceinline__ double edgeK(uint32_t c, int ax, const double* ck, const Coef& cf)
{
    return stencil::edgeK(c, ax, ck, cf.kin, cf.kout);
}

__global__ void __launch_bounds__(256) k_diag_lift(Grid g, const uint32_t* code, const double* ck,
                                                   Coef cf, const double* gb, double* rhs,
                                                   float* dinv, double* diag)
{
    int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= g.N) return;
    uint32_t c = code[e];
    if (c & C_BOX) {
        if (dinv) dinv[e] = 0.0f;
        if (diag) diag[e] = 0.0;
        return;
    }
    const int64_t sx = (int64_t)g.ny * g.S, sy = g.S;
    const int64_t nb[6] = {e - sx, e + sx, e - sy, e + sy, e - 1, e + 1};
    double K[6];
    K[0] = edgeK(code[e - sx], 0, ck, cf);
    K[1] = edgeK(c, 0, ck, cf);
    K[2] = edgeK(code[e - sy], 1, ck, cf);
    K[3] = edgeK(c, 1, ck, cf);
    K[4] = edgeK(code[e - 1], 2, ck, cf);
    K[5] = edgeK(c, 2, ck, cf);
    const double D = stencil::diag_sum(K[0], K[1], K[2], K[3], K[4], K[5], (c & C_SOLUTE) ? 0.0 : cf.mass);
    double lift = 0.0;
    for (int q = 0; q < 6; ++q)
        if (code[nb[q]] & C_BOX) lift += K[q] * gb[nb[q]];
    rhs[e] += lift;
    if (dinv) dinv[e] = (float)(1.0 / D);
    if (diag) diag[e] = D;
}

// ---- marching-cubes area weights ------------------------------------------------------------
// Cell corners are numbered x + 2y + 4z.  Cell edges 0..3 run along x at (y,z) = 00,10,01,11;
// 4..7 along y at (x,z) = 00,10,01,11; 8..11 along z at (x,y) = 00,10,01,11.

__device__ __forceinline__ double tri_area(const double* a, const double* b, const double* c)
{
    double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    double v[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    double x = u[1] * v[2] - u[2] * v[1];
    double y = u[2] * v[0] - u[0] * v[2];
    double z = u[0] * v[1] - u[1] * v[0];
    return 0.5 * sqrt(x * x + y * y + z * z);
}

// The surface in one cell as bit fields, so that nothing is indexed at run time from a
// private array: sm holds the solute flags of the 8 corners, each cut edge has two link
// slots (4-bit fields of lk[0], lk[1], 15 = empty) naming the cut edges it is joined to on
// the two faces it lies on.
__device__ __forceinline__ int nib(uint64_t w, int i) { return (int)((w >> (4 * i)) & 15u); }
__device__ __forceinline__ void set_nib(uint64_t& w, int i, int v)
{
    w = (w & ~((uint64_t)15 << (4 * i))) | ((uint64_t)v << (4 * i));
}
__device__ __forceinline__ void add_link(uint64_t* lk, int a, int b)
{
    if (nib(lk[0], a) == 15) set_nib(lk[0], a, b); else set_nib(lk[1], a, b);
    if (nib(lk[0], b) == 15) set_nib(lk[0], b, a); else set_nib(lk[1], b, a);
}

// index into the cut list of cut edge le of the cell whose corner codes are cc
__device__ __forceinline__ int64_t cell_cut_index(const uint32_t* cc, int le, const int* cutbase)
{
    const int lax = le >> 2, u = le & 1, v = (le >> 1) & 1;
    const int c0 = lax == 0 ? 2 * u + 4 * v : (lax == 1 ? u + 4 * v : u + 2 * v);
    uint32_t cd = cc[0];
#pragma unroll
    for (int q = 1; q < 8; ++q) cd = c0 == q ? cc[q] : cd;
    const uint32_t bits = (cd >> 2) & 7u;
    return (int64_t)cutbase[cd >> C_SLOT_SHIFT] + __popc(bits & ((1u << lax) - 1u));
}

// one thread per cut edge: its marching-cubes weight, the sum over its four cells of a third
// of the area of every triangle that touches it, each closed polygon triangulated as the
// average over all fan starting vertices
__global__ void __launch_bounds__(128) k_mc_weights(Grid g, const uint32_t* code, const int* cutbase,
                                                    int64_t ncut, const int64_t* cutkey,
                                                    const double* rp, double* wp)
{
    int64_t c = (int64_t)blockIdx.x * 128 + threadIdx.x;
    if (c >= ncut) return;
    // local edges: 0..3 along x at (y,z) = 00,10,01,11; 4..7 along y at (x,z); 8..11 along z at
    // (x,y); corners x + 2y + 4z; the faces (axis fa, side sd) and their four edges
    constexpr int kC0[12] = {0, 2, 4, 6, 0, 1, 4, 5, 0, 1, 2, 3};
    constexpr int kC1[12] = {1, 3, 5, 7, 2, 3, 6, 7, 4, 5, 6, 7};
    constexpr int kFace[6][4] = {{4, 6, 8, 10}, {5, 7, 9, 11},    // x = 0, x = 1
                                 {0, 2, 8, 9},  {1, 3, 10, 11},   // y = 0, y = 1
                                 {0, 1, 4, 5},  {2, 3, 6, 7}};    // z = 0, z = 1
    const int64_t key = cutkey[c];
    const int64_t e = key >> 2;
    const int ax = (int)(key & 3);
    const int a1 = ax == 0 ? 1 : 0, a2 = ax == 2 ? 1 : 2;
    const int64_t stride[3] = {(int64_t)g.ny * g.S, g.S, 1};
    double total = 0.0;
    for (int u = 0; u < 2; ++u)
        for (int v = 0; v < 2; ++v) {
            const int64_t base = e - u * stride[a1] - v * stride[a2];   // cell lower corner
            uint32_t cc[8];
            unsigned sm = 0;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                cc[q] = code[base + (q & 1) * stride[0] + ((q >> 1) & 1) * stride[1] + ((q >> 2) & 1) * stride[2]];
                sm |= (cc[q] & C_SOLUTE) << q;
            }
            unsigned cut = 0;
#pragma unroll
            for (int le = 0; le < 12; ++le) cut |= (((sm >> kC0[le]) ^ (sm >> kC1[le])) & 1u) << le;
            // this cell's copy of edge c: along ax, its low corner has bit a1 = u, bit a2 = v
            const int q0 = (u << a1) | (v << a2);
            const int me = ax == 0 ? ((q0 >> 1) & 1) + 2 * ((q0 >> 2) & 1)
                                   : (ax == 1 ? 4 + (q0 & 1) + 2 * ((q0 >> 2) & 1) : 8 + (q0 & 1) + 2 * ((q0 >> 1) & 1));
            uint64_t lk[2] = {~(uint64_t)0, ~(uint64_t)0};
#pragma unroll
            for (int f = 0; f < 6; ++f) {
                const int fa = f >> 1, sd = f & 1;
                int ncf = 0;
#pragma unroll
                for (int t = 0; t < 4; ++t) ncf += (cut >> kFace[f][t]) & 1u;
                if (ncf == 2) {
                    int x = -1, y = -1;
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        if ((cut >> kFace[f][t]) & 1u) {
                            if (x < 0) x = kFace[f][t]; else y = kFace[f][t];
                        }
                    add_link(lk, x, y);
                } else if (ncf == 4) {
                    // join the two cuts incident to the same solute corner
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        if (((q >> fa) & 1) != sd || !((sm >> q) & 1u)) continue;
                        int x = -1, y = -1;
#pragma unroll
                        for (int t = 0; t < 4; ++t) {
                            const int le = kFace[f][t];
                            if (kC0[le] == q || kC1[le] == q) {
                                if (x < 0) x = le; else y = le;
                            }
                        }
                        add_link(lk, x, y);
                    }
                }
            }
            // the polygon through me, in the order of its links, me first
            uint64_t loop = 0;
            int m = 0, prev = 15, cur = me;
            for (;;) {
                loop |= (uint64_t)cur << (4 * m);
                ++m;
                const int a = nib(lk[0], cur), b = nib(lk[1], cur);
                const int nxt = a != prev ? a : b;
                if (nxt == me || nxt == 15 || m >= 12) break;
                prev = cur;
                cur = nxt;
            }
            if (m < 3) continue;
            // fans from every start, triangles touching vertex 0 (me): from start 0 the
            // m - 2 triangles (0, t, t+1); from start s >= 1 the triangle (s, m-1, 0) when
            // s <= m-2 and (s, 0, 1) when s >= 2
            auto P = [&](int k) { return rp + 3 * cell_cut_index(cc, nib(loop, k), cutbase); };
            const double* p0 = P(0);
            const double* p1 = P(1);
            const double* pl = P(m - 1);
            double acc = 0.0;
            const double* pa = p1;
            for (int t = 1; t + 1 < m; ++t) {
                const double* pb = t + 1 == m - 1 ? pl : P(t + 1);
                acc += tri_area(p0, pa, pb);
                pa = pb;
            }
            for (int st = 1; st + 1 < m; ++st) acc += tri_area(st == 1 ? p1 : P(st), pl, p0);
            for (int st = 2; st < m; ++st) acc += tri_area(st == m - 1 ? pl : P(st), p0, p1);
            total += acc / (3.0 * (double)m);
        }
    wp[c] = total;
}

__global__ void k_zero(uint4* p, int64_t n)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (; t < n; t += st) p[t] = make_uint4(0, 0, 0, 0);
}

// ---- inspection exports (unpadded node order) -------------------------------------------------

__global__ void __launch_bounds__(256) k_export_coeffs(Grid g, const uint32_t* code, const double* ck, Coef cf,
                                                       const double* rhs, uint8_t* sol, double* kx,
                                                       double* ky, double* kz, double* diag, double* b)
{
    const int64_t u = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    if (u >= n) return;
    const int k = (int)(u % g.nz), j = (int)((u / g.nz) % g.ny), i = (int)(u / ((int64_t)g.nz * g.ny));
    const int64_t e = g.idx(i, j, k);
    const uint32_t c = code[e];
    if (sol) sol[u] = (uint8_t)(c & C_SOLUTE);
    if (kx) kx[u] = i + 1 < g.nx ? edgeK(c, 0, ck, cf) : 0.0;
    if (ky) ky[u] = j + 1 < g.ny ? edgeK(c, 1, ck, cf) : 0.0;
    if (kz) kz[u] = k + 1 < g.nz ? edgeK(c, 2, ck, cf) : 0.0;
    if (diag || b) {
        double D = 0.0, bv = 0.0;
        if (!(c & C_BOX)) {
            D = stencil::node_diag(g, code, ck, cf.kin, cf.kout, cf.mass, e);
            bv = rhs[e];
        }
        if (diag) diag[u] = D;
        if (b) b[u] = bv;
    }
}

__global__ void __launch_bounds__(256) k_export_phi(Grid g, const double* x, const double* gb, double lB,
                                                    double* out)
{
    const int64_t u = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    if (u >= n) return;
    const int k = (int)(u % g.nz), j = (int)((u / g.nz) % g.ny), i = (int)(u / ((int64_t)g.nz * g.ny));
    const int64_t e = g.idx(i, j, k);
    out[u] = lB * (x[e] + gb[e]);
}

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_fill(hipStream_t s, void* p, size_t bytes)
{
    // zero fill with a kernel (no memset nodes, so callers may capture it in a graph)
    int64_t n16 = (int64_t)(bytes / 16);
    if (n16 > 0) {
        unsigned g = nblk(n16, 256);
        if (g > 65536) g = 65536;
        k_zero<<<g, 256, 0, s>>>((uint4*)p, n16);
    }
    size_t rem = bytes - (size_t)n16 * 16;
    if (rem) return hipMemsetAsync((char*)p + n16 * 16, 0, rem, s);
    return hipGetLastError();
}

hipError_t launch_bins(hipStream_t s, const Atoms& at, Bins& b, int* cnt, int* start, int* ids,
                       int* cursor, double* xyzr_b)
{
    int nb = b.nbx * b.nby * b.nbz;
    hipError_t err = launch_fill(s, cnt, sizeof(int) * (size_t)nb);
    if (err != hipSuccess) return err;
    k_bin_count<<<nblk(at.n, 256), 256, 0, s>>>(at, b, cnt);
    k_scan1<<<1, 1024, 0, s>>>(cnt, nb, start);
    err = hipMemcpyAsync(cursor, start, sizeof(int) * (size_t)nb, hipMemcpyDeviceToDevice, s);
    if (err != hipSuccess) return err;
    k_bin_scatter<<<nblk(at.n, 256), 256, 0, s>>>(at, b, cursor, ids);
    k_bin_sort<<<nblk(nb, 256), 256, 0, s>>>(nb, start, ids);
    k_bin_gather<<<nblk(at.n, 256), 256, 0, s>>>(at, ids, xyzr_b);
    b.start = start;
    b.ids = ids;
    return hipGetLastError();
}

hipError_t launch_classify(hipStream_t s, const Grid& g, const Bins& b, const double* xyzr_b, uint32_t* code)
{
    k_classify<<<nblk(g.N, 256), 256, 0, s>>>(g, b, xyzr_b, code);
    return hipGetLastError();
}

hipError_t launch_cutflags(hipStream_t s, const Grid& g, uint32_t* cls, int* blk_slots, int* blk_cuts,
                           int nb)
{
    k_cutcount<<<nb, 256, 0, s>>>(g, cls, blk_slots, blk_cuts);
    return hipGetLastError();
}

hipError_t launch_scan1(hipStream_t s, const int* in, int n, int* out)
{
    k_scan1<<<1, 1024, 0, s>>>(in, n, out);
    return hipGetLastError();
}

hipError_t launch_scan2(hipStream_t s, int* a, int* b, int n, int* totals)
{
    // in-place exclusive scans through a copy: out[i] written after in[i] is read by the
    // same thread and only the carry crosses chunks, so in == out is safe
    k_scan1<<<1, 1024, 0, s>>>(a, n, a);
    k_scan1<<<1, 1024, 0, s>>>(b, n, b);
    hipError_t err = hipMemcpyAsync(totals, a + n, sizeof(int), hipMemcpyDeviceToDevice, s);
    if (err != hipSuccess) return err;
    err = hipMemcpyAsync(totals + 1, b + n, sizeof(int), hipMemcpyDeviceToDevice, s);
    if (err != hipSuccess) return err;
    return hipGetLastError();
}

hipError_t launch_assign(hipStream_t s, const Grid& g, const uint32_t* cls, uint32_t* code,
                         const int* blk_slots, const int* blk_cuts, int* cutbase, int64_t* cutkey)
{
    k_assign<<<nblk(g.N, 256), 256, 0, s>>>(g, cls, code, blk_slots, blk_cuts, cutbase, cutkey);
    return hipGetLastError();
}

hipError_t launch_cut_geom(hipStream_t s, const Grid& g, const Bins& b, const double* xyzr_b, const Atoms& at,
                           double eps_in, double eps_out, int64_t ncut, const int64_t* cutkey, const uint32_t* code,
                           double* alpha, double* kcut, double* rp, double* np, int* owner,
                           double* ck64, float* ck32)
{
    if (ncut == 0) return hipSuccess;
    k_cut_geom<<<nblk(ncut, 256), 256, 0, s>>>(g, b, xyzr_b, at, eps_in, eps_out, ncut, cutkey, code, alpha,
                                                kcut, rp, np, owner, ck64, ck32);
    return hipGetLastError();
}

hipError_t launch_deposit(hipStream_t s, const Grid& g, const Bins& b, const Atoms& at, double* ac, double* rhs)
{
    if (at.n > 0) k_atom_cells<<<nblk(at.n, 256), 256, 0, s>>>(g, at, b.ids, ac);
    k_deposit<<<nblk(g.N, 256), 256, 0, s>>>(g, b, ac, rhs);
    return hipGetLastError();
}

int grid_energy_blocks(int n_atoms) { return (int)nblk(n_atoms > 0 ? n_atoms : 1, 256); }

hipError_t launch_grid_energy(hipStream_t s, const Grid& g, const Atoms& at, const double* x, double scale,
                              double* part)
{
    const int nb = grid_energy_blocks(at.n);
    k_grid_energy<<<nb, 256, 0, s>>>(g, at, x, part);
    k_grid_energy_total<<<1, 256, 0, s>>>(part, nb, scale);
    return hipGetLastError();
}

DhExp dh_exp_consts(double kD)
{
    DhExp E{};
    if (kD == 0.0) return E;
    const long double ln2 = 0.693147180559945309417232121458176568L;
    E.L = (double)(ln2 / ((long double)kDhTable * (long double)kD));
    E.tscale = (double)(-(long double)kD * kDhTable / ln2);
    E.c1 = -kD;
    E.c2 = 0.5 * kD * kD;
    E.c3 = -kD * kD * kD / 6.0;
    return E;
}

DhFaces dh_faces(const Grid& g)
{
    DhFaces fc{};
    const int64_t fx = (int64_t)g.ny * g.nz, fy = (int64_t)(g.nx - 2) * g.nz;
    const int64_t fz = (int64_t)(g.nx - 2) * (g.ny - 2);
    const int U[3] = {g.ny, g.nx - 2, g.nx - 2}, V[3] = {g.nz, g.nz, g.ny - 2};
    const int64_t first[3] = {0, 2 * fx, 2 * fx + 2 * fy}, size[3] = {fx, fy, fz};
    fc.tile0[0] = 0;
    for (int f = 0; f < 6; ++f) {
        const int w = f >> 1;
        fc.base[f] = first[w] + (f & 1) * size[w];
        fc.U[f] = U[w];
        fc.V[f] = V[w];
        fc.pv[f] = (V[w] + DH_PV - 1) / DH_PV;
        fc.np[f] = (int64_t)((U[w] + DH_PU - 1) / DH_PU) * fc.pv[f];
        fc.tile0[f + 1] = fc.tile0[f] + (int)((fc.np[f] + 255) / 256);
    }
    return fc;
}

DhSplit dh_split(const Grid& g, int n_atoms)
{
    DhSplit sp;
    sp.nbox = 2 * ((int64_t)g.ny * g.nz + (int64_t)(g.nx - 2) * g.nz + (int64_t)(g.nx - 2) * (g.ny - 2));
    sp.tiles = (int)nblk(sp.nbox, kDhNodesPerBlock);
    const int chunks = std::max(1, (n_atoms + 255) / 256);
    // enough blocks to fill the device many times over (the last wave of blocks is then a small
    // part of the run), each with whole 256-atom chunks
    int r = (int)std::min<int64_t>(kDhMaxRanges, std::max<int64_t>(1, (kDhTargetBlocks + sp.tiles - 1) / sp.tiles));
    r = std::min(r, chunks);
    const int cpr = (chunks + r - 1) / r;
    sp.per = 256 * cpr;
    sp.ranges = (chunks + cpr - 1) / cpr;
    return sp;
}

hipError_t launch_bc_dh(hipStream_t s, const Grid& g, const Atoms& at, double kD, double eps_out, double* part,
                        double* gb)
{
    const DhSplit sp = dh_split(g, at.n);
    const DhFaces fc = dh_faces(g);
    k_bc_dh<<<(unsigned)(fc.tile0[6] * sp.ranges), 256, 0, s>>>(g, at, dh_exp_consts(kD), sp, fc, part);
    k_bc_dh_sum<<<(unsigned)nblk(sp.nbox, 256), 256, 0, s>>>(g, sp, part, eps_out, gb);
    return hipGetLastError();
}

hipError_t launch_bc_dh32(hipStream_t s, const Grid& g, const Atoms& at, double kD, double eps_out, double* part,
                          double* gb)
{
    const DhSplit sp = dh_split(g, at.n);
    const DhFaces fc = dh_faces(g);
    k_bc_dh32<<<(unsigned)(fc.tile0[6] * sp.ranges), 256, 0, s>>>(g, at, kD, sp, fc, part);
    k_bc_dh_sum<<<(unsigned)nblk(sp.nbox, 256), 256, 0, s>>>(g, sp, part, eps_out, gb);
    return hipGetLastError();
}

hipError_t launch_bc_user(hipStream_t s, const Grid& g, const double* full, double* gb)
{
    int64_t nbx = 2 * ((int64_t)g.ny * g.nz + (int64_t)(g.nx - 2) * g.nz + (int64_t)(g.nx - 2) * (g.ny - 2));
    k_bc_user<<<nblk(nbx, 256), 256, 0, s>>>(g, full, gb);
    return hipGetLastError();
}

hipError_t launch_diag_lift(hipStream_t s, const Grid& g, const uint32_t* code, const double* ck64,
                            Coef c, const double* gb, double* rhs, float* dinv, double* diag)
{
    k_diag_lift<<<nblk(g.N, 256), 256, 0, s>>>(g, code, ck64, c, gb, rhs, dinv, diag);
    return hipGetLastError();
}

hipError_t launch_export_coeffs(hipStream_t s, const Grid& g, const uint32_t* code, const double* ck64, Coef c,
                                const double* rhs, uint8_t* sol, double* kx, double* ky, double* kz,
                                double* diag, double* b)
{
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    k_export_coeffs<<<nblk(n, 256), 256, 0, s>>>(g, code, ck64, c, rhs, sol, kx, ky, kz, diag, b);
    return hipGetLastError();
}

hipError_t launch_export_phi(hipStream_t s, const Grid& g, const double* x, const double* gb, double lB,
                             double* out)
{
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    k_export_phi<<<nblk(n, 256), 256, 0, s>>>(g, x, gb, lB, out);
    return hipGetLastError();
}

hipError_t launch_mc_weights(hipStream_t s, const Grid& g, const uint32_t* code, const int* cutbase,
                             int64_t ncut, const int64_t* cutkey, const double* rp, double* wp)
{
    if (ncut == 0) return hipSuccess;
    k_mc_weights<<<nblk(ncut, 128), 128, 0, s>>>(g, code, cutbase, ncut, cutkey, rp, wp);
    return hipGetLastError();
}

}  // namespace pbk
