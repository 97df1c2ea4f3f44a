// pb_solve.hip -- Jacobi-preconditioned conjugate gradients on the condensed 7-point
// operator (paper Sect. 3.1, eq. matrixequation, with the edge permittivities of Sect. 3.2),
// matrix-free, for FP64 and FP32 data.
//
// One CG iteration is one pass over the vectors plus a one-block tail, with no host round
// trip.  The vectors kept are z = D^-1 r and w = D^-1 q (the preconditioned residual and
// operator image), p and x:
//   iter(it): per node  z = z_old - alpha w_old,  x += alpha p_old,  p = z + beta p_old,
//             q = A p,  w = q / D  (r = D z and q are formed where needed),
//             and per-block partial sums of p.q, r.z, r.r, z.q and q.D^-1 q
//   tail(it): reduce the partial sums in a fixed order, test convergence, and prepare the
//             next step: alpha = r.z / p.q, and beta from the next r.z, which follows from
//             the expansion (r - alpha q).D^-1 (r - alpha q) = r.z - 2 alpha z.q +
//             alpha^2 q.D^-1 q without another pass over the vectors.
// This is the iteration of Jacobi-preconditioned CG with the residual and solution updates
// of one step moved into the pass of the next; it reads z, w, p, x and the node code once
// and writes z, w, p and x once per iteration.  z, w and p are double buffered by iteration
// parity, because each tile also needs p on its halo, which it recomputes from the old
// vectors of its neighbours.  The scalars never leave the device and all reductions run in
// a fixed order, so a solve is run-to-run deterministic.
//
// The iteration kernel tiles the interior into columns of ZW (z) x TY (y) nodes and marches
// along x over a chunk of planes, carrying the x-neighbours in registers and staging the
// current plane with its y/z halo in LDS.  Tiles are numbered z-fastest and handed out so
// that each XCD gets one contiguous range of tiles, which keeps the halo rows of
// neighbouring tiles in the same L2.
#include "pb_internal.h"
#include "pb_stencil.h"

#include <cmath>
#include <type_traits>

namespace pbk {

namespace {

using namespace stencil;

// sum of NV doubles over a block of NW waves; every thread gets the totals (fixed order)
template <int NV, int NW = 4>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* sh)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int t = 0; t < NV; ++t) v[t] += __shfl_xor(v[t], o, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0)
#pragma unroll
        for (int t = 0; t < NV; ++t) sh[NW * t + w] = v[t];
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NV; ++t) {
        double a = sh[NW * t];
#pragma unroll
        for (int u = 1; u < NW; ++u) a += sh[NW * t + u];
        v[t] = a;
    }
}

template <typename T>
struct Old {   // the old vectors of one node, from which its new z and p follow
    T z, w, p;
    uint32_t c;
};

template <typename T>
struct K3 {    // coefficients of the +x, +y, +z edges of a node
    T x, y, z;
};

// element e of an array through a 32-bit byte offset from a uniform base (the grid is limited
// so that every offset fits), which lets every load and store use one offset register
template <typename T>
__device__ __forceinline__ const T& at(const T* base, uint32_t e)
{
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + e * (uint32_t)sizeof(T));
}
template <typename T>
__device__ __forceinline__ T& at(T* base, uint32_t e)
{
    return *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + e * (uint32_t)sizeof(T));
}

// One iteration over one tile.  The preconditioned residual z = D^-1 r and w = D^-1 q are
// kept instead of r and q, so a node's new p = (z - alpha w) + beta p_old needs no D^-1; the
// tile computes D of its own nodes from the edge coefficients it has for q = A p, and forms
// r = D z and q = D w there.
//
// A tile is ZW = 32 nodes along z (one 128-byte line of FP32 values: rows start on a line)
// by TY = 2*NWV rows along y; each wave holds two rows, each lane one node of a plane.
//
// Software pipeline along x: the old vectors of plane i+3 with their halo, and x of plane
// i+2, are loaded while plane i is computed, into register slots numbered by plane modulo 4;
// the loop body is unrolled four times so that every slot keeps its registers and no load in
// flight is ever copied (a copy would wait for it).  Two LDS buffers alternate by plane, so
// one barrier per plane suffices.
template <typename T>
__device__ __forceinline__ void iter_body(const Grid& g, const TileShape& ts, const CGBufs<T>& B, const Coef& cf,
                                          const int bid)
{
    __shared__ double sh[5 * NWV];
    __shared__ T sp[2][TY + 2][ZW + 2];   // p of plane i: rows j0-1..j0+TY, cols k0-1..k0+ZW
    __shared__ T sky[2][TY + 1][ZW];      // K of the +y edge: rows j0-1..j0+TY-1, cols k0..k0+ZW-1
    __shared__ T skz[2][TY][ZW + 1];      // K of the +z edge: own rows, cols k0-1..k0+ZW-1
    const CGState* st = B.st;
    if (st->status != 0) return;
    const int nw = st->iter_count & 1, od = nw ^ 1;
    const T aT = (T)st->alpha, bT = (T)st->beta;
    const T kin = (T)cf.kin, kout = (T)cf.kout, mass = (T)cf.mass;

    // XCD-aware bijective block -> tile map (blocks are dealt round-robin to 8 XCDs)
    const int W = ts.items, b = bid;
    const int q8 = W >> 3, rem = W & 7, xcd = b & 7;
    const int item = xcd * q8 + (xcd < rem ? xcd : rem) + (b >> 3);
    const int kt = item % ts.nkt;
    const int t2 = item / ts.nkt;
    const int jt = t2 % ts.njt;
    const int xc = t2 / ts.njt;
    const int k0 = 1 + kt * ZW, j0 = 1 + jt * TY;
    const int ib = 1 + xc * ts.LX;
    const int ie = (ib + ts.LX < g.nx - 1) ? ib + ts.LX : g.nx - 1;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int kl = lane & (ZW - 1), row = 2 * wv + (lane >> 5);

    const T* __restrict__ z_o = od ? B.z[1] : B.z[0];
    const T* __restrict__ w_o = od ? B.w[1] : B.w[0];
    const T* __restrict__ p_o = od ? B.p[1] : B.p[0];
    T* __restrict__ z_n = nw ? B.z[1] : B.z[0];
    T* __restrict__ w_n = nw ? B.w[1] : B.w[0];
    T* __restrict__ p_n = nw ? B.p[1] : B.p[0];
    T* __restrict__ x = B.x;
    const uint32_t* __restrict__ code = B.code;
    const T* __restrict__ ck = B.ck;
    const uint32_t sx = (uint32_t)g.ny * (uint32_t)g.S;

    // Out-of-interior positions are clamped onto box nodes, where every vector is 0: every
    // load below is unconditional and in bounds, and a clamped node has z = p = 0.
    auto clampj = [&](int j) { return j < 0 ? 0 : (j > g.ny - 1 ? g.ny - 1 : j); };
    auto clampk = [&](int k) { return k < 0 ? 0 : (k > g.nz - 1 ? g.nz - 1 : k); };
    auto load = [&](uint32_t e) {
        Old<T> v;
        v.z = at(z_o, e);
        v.w = at(w_o, e);
        v.p = at(p_o, e);
        v.c = at(code, e);
        return v;
    };
    auto znew = [&](const Old<T>& v) { return v.z - aT * v.w; };
    auto pnew = [&](const Old<T>& v) { return znew(v) + bT * v.p; };

    // own node (z = k0 + kl, y = j0 + row) and this thread's halo point
    const int k = k0 + kl, j = j0 + row;
    const bool valid = j <= g.ny - 2 && k <= g.nz - 2;
    const uint32_t eo = (uint32_t)g.idx(0, clampj(j), clampk(k));
    // halo: wave 0 holds rows j0-1 (lanes 0-31; needs p and K+y) and j0+TY (lanes 32-63; p),
    // wave 1 columns k0-1 (lanes 0..TY-1; p and K+z) and k0+ZW (lanes 32..32+TY-1; p); the
    // other lanes have no halo point (they load a node of their own tile and never use it)
    int hj = j0, hk = k0, hsel = 0;   // hsel: 1 row below, 2 row above, 3 column before, 4 column after
    if (wv == 0) {
        hsel = lane < 32 ? 1 : 2;
        hj = lane < 32 ? j0 - 1 : j0 + TY;
        hk = k0 + kl;
    } else if (wv == 1 && kl < TY) {
        hsel = lane < 32 ? 3 : 4;
        hj = j0 + kl;
        hk = lane < 32 ? k0 - 1 : k0 + ZW;
    }
    const uint32_t eh = (uint32_t)g.idx(0, clampj(hj), clampk(hk));
    const int hax = hsel == 1 ? 1 : 2;

    Old<T> rb[4];   // old vectors of the own node in planes, slot (plane - ib) % 4
    Old<T> hb[4];   // halo, same slots
    T xb[4];        // x of the own node, same slots
    K3<T> kr[2];    // coefficient-table reads of the own node, slot (plane - ib) % 2
    T hr[2];        // same for the halo
    T pm, pc, kxm;  // p of planes i-1 and i, K of the -x edge of plane i
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};   // p.q, r.z, r.r, z.q, q.D^-1 q (as D z w, D w w)

    // prologue: plane ib-1 (p, K+x), planes ib..ib+2 and their halo, x of ib and ib+1
    {
        const uint32_t i1 = (uint32_t)(ib + 1 < ie ? ib + 1 : ie), i2 = (uint32_t)(ib + 2 < ie ? ib + 2 : ie);
        const uint32_t h1 = (uint32_t)(ib + 1 < ie ? ib + 1 : ie - 1), h2 = (uint32_t)(ib + 2 < ie ? ib + 2 : ie - 1);
        const Old<T> a = load(eo + (uint32_t)(ib - 1) * sx);
        rb[0] = load(eo + (uint32_t)ib * sx);
        rb[1] = load(eo + i1 * sx);
        rb[2] = load(eo + i2 * sx);
        xb[0] = at(x, eo + (uint32_t)ib * sx);
        xb[1] = at(x, eo + h1 * sx);
        hb[0] = load(eh + (uint32_t)ib * sx);
        hb[1] = load(eh + h1 * sx);
        hb[2] = load(eh + h2 * sx);
        pm = pnew(a);
        kxm = edgeK(a.c, 0, ck, kin, kout);
        pc = pnew(rb[0]);
        kr[0].x = ck[ck_index(rb[0].c, 0)];
        kr[0].y = ck[ck_index(rb[0].c, 1)];
        kr[0].z = ck[ck_index(rb[0].c, 2)];
        hr[0] = ck[ck_index(hb[0].c, hax)];
    }

    // Load distances: own planes and halo 3 planes ahead, x 2 planes ahead, table reads
    // 1 plane ahead.  Loads complete in issue order as far as the wait counter is concerned,
    // so each step first issues what the next step needs (the table reads of plane i+1),
    // then the far prefetch.
    auto step = [&](const int i, auto slot) {
        constexpr int S0 = decltype(slot)::value;
        constexpr int S1 = (S0 + 1) & 3, S2 = (S0 + 2) & 3, S3 = (S0 + 3) & 3;
        constexpr int L = S0 & 1;
        // plane i+1 has arrived: its p, and its table reads
        const T px = pnew(rb[S1]);
        kr[L ^ 1].x = ck[ck_index(rb[S1].c, 0)];
        kr[L ^ 1].y = ck[ck_index(rb[S1].c, 1)];
        kr[L ^ 1].z = ck[ck_index(rb[S1].c, 2)];
        hr[L ^ 1] = ck[ck_index(hb[S1].c, hax)];
        __builtin_amdgcn_sched_barrier(0);   // keep the issue order: table reads, then prefetch
        // prefetch: own plane i+3 (never past plane ie, the last one this chunk needs), its
        // halo and x of plane i+2 (never past ie-1)
        {
            const uint32_t i3 = (uint32_t)(i + 3 < ie ? i + 3 : ie);
            const uint32_t h3 = (uint32_t)(i + 3 < ie ? i + 3 : ie - 1);
            const uint32_t i2 = (uint32_t)(i + 2 < ie ? i + 2 : ie - 1);
            rb[S3] = load(eo + i3 * sx);
            xb[S2] = at(x, eo + i2 * sx);
            hb[S3] = load(eh + h3 * sx);
        }
        __builtin_amdgcn_sched_barrier(0);

        // stage plane i in LDS: p and the +y/+z edge coefficients
        const uint32_t cc = rb[S0].c;
        const T Kxp = ck_blend(kr[L].x, cc, 0, kin, kout);
        sp[L][1 + row][1 + kl] = pc;
        sky[L][1 + row][kl] = ck_blend(kr[L].y, cc, 1, kin, kout);
        skz[L][row][1 + kl] = ck_blend(kr[L].z, cc, 2, kin, kout);
        {
            const T hv = pnew(hb[S0]);
            const T hK = ck_blend(hr[L], hb[S0].c, hax, kin, kout);
            if (hsel == 1) {
                sp[L][0][1 + kl] = hv;
                sky[L][0][kl] = hK;
            } else if (hsel == 2) {
                sp[L][TY + 1][1 + kl] = hv;
            } else if (hsel == 3) {
                sp[L][1 + kl][0] = hv;
                skz[L][kl][0] = hK;
            } else if (hsel == 4) {
                sp[L][1 + kl][ZW + 1] = hv;
            }
        }
        __syncthreads();
        const Old<T>& o = rb[S0];
        const T Kym = sky[L][row][kl], Kyp = sky[L][1 + row][kl];
        const T Kzm = skz[L][row][kl], Kzp = skz[L][row][1 + kl];
        const T D = diag_sum(kxm, Kxp, Kym, Kyp, Kzm, Kzp, (cc & C_SOLUTE) ? (T)0 : mass);
        const T p0 = pc;
        const T nbs = kxm * pm + Kxp * px + Kym * sp[L][row][1 + kl] + Kyp * sp[L][row + 2][1 + kl] +
                      Kzm * sp[L][1 + row][kl] + Kzp * sp[L][1 + row][2 + kl];
        const T qv = D * p0 - nbs;
        const T zv = znew(o);
        const T wq = qv / D;
        const T xv = xb[S0] + aT * o.p;
        // a lane outside the interior was clamped onto a box node, and a plane past the
        // chunk's last one stores onto the box face x = nx-1: the vectors there stay 0, so
        // the stores need no branch
        const bool ok = valid && i < ie;
        const uint32_t e = eo + (uint32_t)(i < ie ? i : g.nx - 1) * sx;
        // streaming stores: the new vectors are read again only in the next iteration,
        // after the whole grid has passed through the caches
        __builtin_nontemporal_store(ok ? zv : (T)0, &at(z_n, e));
        __builtin_nontemporal_store(ok ? wq : (T)0, &at(w_n, e));
        __builtin_nontemporal_store(ok ? p0 : (T)0, &at(p_n, e));
        __builtin_nontemporal_store(ok ? xv : (T)0, &at(x, e));
        const double dD = ok ? (double)D : 0.0;
        const double dz = (double)zv, dw = (double)wq, dq = (double)qv, dzD = dD * dz, dwD = dD * dw;
        acc[0] += ok ? (double)p0 * dq : 0.0;
        acc[1] += dzD * dz;
        acc[2] += dzD * dzD;
        acc[3] += dzD * dw;
        acc[4] += dwD * dw;
        kxm = Kxp;
        pm = p0;
        pc = px;
    };

    // Whole groups of four planes, so the loop body has no branch: a plane past the chunk's
    // last one (only in the last chunk along x, when its length is not a multiple of four)
    // is computed from clamped loads and stores its zeros onto the box face x = nx-1, whose
    // vectors are 0, like a lane outside the interior.
    using C0 = std::integral_constant<int, 0>;
    using C1 = std::integral_constant<int, 1>;
    using C2 = std::integral_constant<int, 2>;
    using C3 = std::integral_constant<int, 3>;
    for (int i = ib; i < ie; i += 4) {
        step(i, C0{});
        step(i + 1, C1{});
        step(i + 2, C2{});
        step(i + 3, C3{});
    }
    block_sum<5, NWV>(acc, sh);
    if (threadIdx.x == 0)
#pragma unroll
        for (int u = 0; u < 5; ++u) B.part[(int64_t)u * B.nb + bid] = acc[u];
}

template <typename T>
__global__ void __launch_bounds__(64 * NWV) k_cg_iter(Grid g, TileShape ts, CGBufs<T> B, Coef cf)
{
    iter_body(g, ts, B, cf, (int)blockIdx.x);
}

// one block: reduce the iteration's partial sums and set the scalars of the next iteration
__device__ __forceinline__ void tail_body(const double* __restrict__ part, int nb, CGState* st)
{
    __shared__ double sh[20];
    if (st->status != 0) return;
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int t = threadIdx.x; t < nb; t += 256)
#pragma unroll
        for (int u = 0; u < 5; ++u) v[u] += part[(int64_t)u * nb + t];
    block_sum<5>(v, sh);
    if (threadIdx.x != 0) return;
    const double pq = v[0], gm = v[1], rr = v[2], zq = v[3], qq = v[4];
    const int it = st->iter_count;
    st->iter_count = it + 1;
    st->rr = rr;
    st->pq = pq;
    if (!isfinite(pq) || !isfinite(gm) || !isfinite(rr) || !isfinite(zq) || !isfinite(qq)) {
        st->status = 2;
        st->iters = it;
        return;
    }
    double alpha = 0.0, beta = 0.0;
    if (pq > 0.0 && gm > 0.0) {
        alpha = gm / pq;
        const double gn = (gm - 2.0 * alpha * zq) + alpha * alpha * qq;
        beta = gn > 0.0 ? gn / gm : 0.0;
    }
    st->alpha = alpha;
    st->beta = beta;
    st->gamma = gm;
    if (rr <= st->stop2) {
        st->status = st->stop_status;
        st->iters = it;
    } else if (!(pq > 0.0)) {
        st->status = 2;
        st->iters = it;
    }
}

__global__ void __launch_bounds__(256) k_cg_tail(const double* __restrict__ part, int nb, CGState* st)
{
    tail_body(part, nb, st);
}

template <typename T>
struct Vec4;
template <>
struct Vec4<double> {
    using type = double4;
};
template <>
struct Vec4<float> {
    using type = float4;
};

// z_old = D^-1 b (the buffer the first iteration reads), x = 0, the other z and w, p of both
// parities = 0 (box and padding nodes are never written by the iteration and must read 0),
// partial sums of ||b||^2
template <typename T>
__global__ void __launch_bounds__(256) k_cg_init(Grid g, CGBufs<T> B, Coef cf, const double* b64, const T* bT)
{
    __shared__ double sh[4];
    const T kin = (T)cf.kin, kout = (T)cf.kout, mass = (T)cf.mass;
    double rr = 0.0;
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < g.N; e += stride) {
        const T bv = b64 ? (T)b64[e] : bT[e];
        T zv = (T)0;
        if (!(B.code[e] & C_BOX)) zv = bv / node_diag(g, B.code, B.ck, kin, kout, mass, e);
        B.x[e] = (T)0;
        B.z[0][e] = (T)0;
        B.z[1][e] = zv;
        B.w[0][e] = (T)0;
        B.w[1][e] = (T)0;
        B.p[0][e] = (T)0;
        B.p[1][e] = (T)0;
        rr += (double)bv * (double)bv;
    }
    double a[1] = {rr};
    block_sum<1>(a, sh);
    if (threadIdx.x == 0) B.part[blockIdx.x] = a[0];
}

__global__ void __launch_bounds__(256) k_cg_fin(const double* part, int nb, CGState* st, double rtol2)
{
    __shared__ double sh[4];
    double a[1] = {0.0};
    for (int t = threadIdx.x; t < nb; t += 256) a[0] += part[t];
    block_sum<1>(a, sh);
    if (threadIdx.x == 0) {
        const double rr = a[0];
        st->alpha = 0.0;
        st->beta = 0.0;
        st->gamma = 0.0;
        st->bnorm2 = rr;
        st->rr = rr;
        st->pq = 0.0;
        st->stop2 = rtol2 * rr;
        st->trig2 = -1.0;
        st->delta2 = 0.0;
        st->goal64 = 0.0;
        st->rr64 = 0.0;
        st->status = rr > 0.0 ? 0 : 1;
        st->stop_status = 1;
        st->iters = 0;
        st->iter_count = 0;
        st->ru = 0;
        st->n_ru = 0;
    }
}

// ---- mixed precision: FP32 CG with FP64 reliable updates ------------------------------------
// The FP32 iteration runs on; a reliable update takes the pending step of the last
// iteration, folds the FP32 correction into the FP64 solution and replaces the FP32
// residual by the FP64 true residual b - A x64 (FP64 operator, exact coefficients; stored as
// z = D^-1 r), keeping the search direction: the next iteration then continues with
// alpha = 0 and beta = r_true.z_true / r.z.  An update runs at a chunk end once the recursive residual has
// dropped by delta since the last one, or when the recursive residual reaches the target
// (the tail then stops with status 3).

__device__ __forceinline__ void ru_add_body(int64_t n4, CGState* st, double* __restrict__ x, float* __restrict__ d,
                                            const float* p0, const float* p1, int force, const int bid,
                                            const int nblk)
{
    const int s0 = st->status;
    const bool go = (s0 == 3) || (s0 == 0 && (force || st->rr <= st->trig2));
    if (!go) return;
    const double a = st->alpha;
    const float4* __restrict__ p = reinterpret_cast<const float4*>(((st->iter_count - 1) & 1) ? p1 : p0);
    const int64_t stride = (int64_t)nblk * 256;
    for (int64_t v = (int64_t)bid * 256 + threadIdx.x; v < n4; v += stride) {
        double4 xv = reinterpret_cast<double4*>(x)[v];
        const float4 dv = reinterpret_cast<const float4*>(d)[v];
        const float4 pv = p[v];
        xv.x += (double)dv.x + a * (double)pv.x;
        xv.y += (double)dv.y + a * (double)pv.y;
        xv.z += (double)dv.z + a * (double)pv.z;
        xv.w += (double)dv.w + a * (double)pv.w;
        reinterpret_cast<double4*>(x)[v] = xv;
        reinterpret_cast<float4*>(d)[v] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    if (bid == 0 && threadIdx.x == 0) st->ru = 1;
}

__global__ void __launch_bounds__(256) k_ru_add(int64_t n4, CGState* st, double* x, float* d, float* p0, float* p1,
                                                int force)
{
    ru_add_body(n4, st, x, d, p0, p1, force, (int)blockIdx.x, (int)gridDim.x);
}

// r_true = b - A x64 in FP64; z = r_true / D (D of the FP32 operator, as the iteration forms
// it) stored as FP32 into the buffer the next iteration reads; partial sums of ||r_true||^2
// (FP64) and of r.z, r.r as the FP32 iteration sees them (r = D z)
__device__ __forceinline__ void ru_residual_body(const Grid& g, const uint32_t* __restrict__ code,
                                                 const double* __restrict__ ck, const float* __restrict__ ck32,
                                                 const Coef& cf, const double* __restrict__ b,
                                                 const double* __restrict__ x, float* z0, float* z1,
                                                 double* __restrict__ part3, const CGState* st, const int bid,
                                                 const int nblk)
{
    __shared__ double sh[12];
    if (!st->ru) return;
    float* __restrict__ zout = ((st->iter_count - 1) & 1) ? z1 : z0;
    const int64_t e = (int64_t)bid * 256 + threadIdx.x;
    double v[3] = {0.0, 0.0, 0.0};
    if (e < g.N) {
        const uint32_t c = code[e];
        float out = 0.0f;
        if (!(c & C_BOX)) {
            const int64_t sx = (int64_t)g.ny * g.S, sy = g.S;
            const double Kxm = edgeK(code[e - sx], 0, ck, cf.kin, cf.kout);
            const double Kxp = edgeK(c, 0, ck, cf.kin, cf.kout);
            const double Kym = edgeK(code[e - sy], 1, ck, cf.kin, cf.kout);
            const double Kyp = edgeK(c, 1, ck, cf.kin, cf.kout);
            const double Kzm = edgeK(code[e - 1], 2, ck, cf.kin, cf.kout);
            const double Kzp = edgeK(c, 2, ck, cf.kin, cf.kout);
            const double D = ((Kxm + Kxp) + (Kym + Kyp)) + ((Kzm + Kzp) + ((c & C_SOLUTE) ? 0.0 : cf.mass));
            const double ax = D * x[e] - (Kxm * x[e - sx] + Kxp * x[e + sx] + Kym * x[e - sy] +
                                          Kyp * x[e + sy] + Kzm * x[e - 1] + Kzp * x[e + 1]);
            const double rv = b[e] - ax;
            v[0] = rv * rv;
            const float D32 = node_diag(g, code, ck32, (float)cf.kin, (float)cf.kout, (float)cf.mass, e);
            out = (float)rv / D32;
            const double dz = (double)out, dzD = (double)D32 * dz;
            v[1] = dzD * dz;
            v[2] = dzD * dzD;
        }
        zout[e] = out;
    }
    block_sum<3>(v, sh);
    if (threadIdx.x == 0) {
        part3[bid] = v[0];
        part3[nblk + bid] = v[1];
        part3[2 * nblk + bid] = v[2];
    }
}

__global__ void __launch_bounds__(256) k_ru_residual(Grid g, const uint32_t* __restrict__ code,
                                                     const double* __restrict__ ck, const float* __restrict__ ck32,
                                                     Coef cf, const double* __restrict__ b,
                                                     const double* __restrict__ x, float* z0, float* z1,
                                                     double* __restrict__ part3, const CGState* st)
{
    ru_residual_body(g, code, ck, ck32, cf, b, x, z0, z1, part3, st, (int)blockIdx.x, (int)gridDim.x);
}

__global__ void k_ru_begin(CGState* st)
{
    st->status = 0;
    st->iter_count = 0;
    st->ru = 1;
}

// one block: finish a reliable update (or, with init, set up the mixed iteration)
__device__ __forceinline__ void ru_fin_body(CGState* st, const double* part3, int nbres, int init, double rtol2,
                                            double delta2)
{
    __shared__ double sh[12];
    if (!st->ru) return;
    double v[3] = {0.0, 0.0, 0.0};
    for (int t = threadIdx.x; t < nbres; t += 256)
#pragma unroll
        for (int u = 0; u < 3; ++u) v[u] += part3[(int64_t)u * nbres + t];
    block_sum<3>(v, sh);
    if (threadIdx.x == 0) {
        const double rr64 = v[0], gm = v[1], rr = v[2];
        if (init) {
            st->beta = 0.0;
            st->bnorm2 = rr;
            st->pq = 0.0;
            st->stop2 = rtol2 * rr;
            st->delta2 = delta2;
            st->goal64 = rtol2 * rr64;
            st->stop_status = 3;
            st->iters = 0;
            st->iter_count = 0;
            st->n_ru = 0;
        } else {
            st->beta = st->gamma > 0.0 ? gm / st->gamma : 0.0;
            st->n_ru += 1;
        }
        st->alpha = 0.0;
        st->gamma = gm;
        st->rr = rr;
        st->rr64 = rr64;
        st->trig2 = st->delta2 * rr;
        if (rr64 <= st->goal64) {
            st->status = 1;
            st->iters = st->iter_count;
        } else {
            st->status = 0;
        }
        st->ru = 0;
    }
}

__global__ void __launch_bounds__(256) k_ru_fin(CGState* st, const double* part3, int nbres, int init, double rtol2,
                                                double delta2)
{
    ru_fin_body(st, part3, nbres, init, rtol2, delta2);
}

// plain streaming copy with non-temporal accesses: the attainable-bandwidth reference (and the
// kernel used to scale the HBM byte counters)
typedef float f4v __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) k_stream_copy(const f4v* __restrict__ a, f4v* __restrict__ b, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < n; v += stride) {
        const f4v x = __builtin_nontemporal_load(a + v);
        __builtin_nontemporal_store(x, b + v);
    }
}

// ---- batched launches: one launch advances every resident problem ---------------------------
// Block b of a batched launch belongs to the problem p with off[p] <= b < off[p+1] and acts as
// block b - off[p] of that problem's own launch, so each problem computes exactly what it
// computes when solved alone.  In the iteration launch off[p] is a multiple of 8.

__device__ __forceinline__ int find_prob(const int* __restrict__ off, int P, int b)
{
    int lo = 0, hi = P - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <typename T>
__global__ void __launch_bounds__(64 * NWV) kb_iter(const ProbDev<T>* __restrict__ D, const int* __restrict__ off, int P)
{
    const int p = __builtin_amdgcn_readfirstlane(find_prob(off, P, (int)blockIdx.x));
    const ProbDev<T> d = D[p];   // a uniform copy (scalar registers)
    // each problem's range starts at a multiple of 8, so its block b runs on XCD b % 8 as in
    // its own launch; the blocks that pad a range to the next multiple of 8 do nothing
    const int bid = (int)blockIdx.x - off[p];
    if (bid >= d.ts.items) return;
    iter_body(d.g, d.ts, d.B, d.cf, bid);
}

__global__ void __launch_bounds__(256) kb_tail(const ProbDev<float>* __restrict__ D)
{
    const ProbDev<float>& d = D[blockIdx.x];
    tail_body(d.B.part, d.B.nb, d.B.st);
}

__global__ void __launch_bounds__(256) kb_ru_add(const ProbDev<float>* __restrict__ D, const int* __restrict__ off, int P)
{
    const int p = __builtin_amdgcn_readfirstlane(find_prob(off, P, (int)blockIdx.x));
    const ProbDev<float>& d = D[p];
    ru_add_body(d.g.N / 4, d.B.st, d.x64, d.B.x, d.B.p[0], d.B.p[1], 0, (int)blockIdx.x - off[p], d.nadd);
}

__global__ void __launch_bounds__(256) kb_ru_residual(const ProbDev<float>* __restrict__ D, const int* __restrict__ off,
                                                      int P)
{
    const int p = __builtin_amdgcn_readfirstlane(find_prob(off, P, (int)blockIdx.x));
    const ProbDev<float>& d = D[p];
    ru_residual_body(d.g, d.B.code, d.ck64, d.B.ck, d.cf, d.rhs, d.x64, d.B.z[0], d.B.z[1], d.part3, d.B.st,
                     (int)blockIdx.x - off[p], d.nbres);
}

__global__ void __launch_bounds__(256) kb_ru_fin(const ProbDev<float>* __restrict__ D)
{
    const ProbDev<float>& d = D[blockIdx.x];
    ru_fin_body(d.B.st, d.part3, d.nbres, 0, 0.0, 0.0);
}

__global__ void kb_gather(const ProbDev<float>* __restrict__ D, int P, CGState* out)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < P) out[p] = *D[p].B.st;
}

}  // namespace

hipError_t launch_batch_chunk(hipStream_t s, const ProbDev<float>* D, const int* off, int P, const BatchTotals& t,
                              int iters, CGState* gather_out, hipEvent_t* ev)
{
    const int* off_st = off;
    const int* off_add = off + (P + 1);
    const int* off_res = off + 2 * (P + 1);
    for (int it = 0; it < iters; ++it) {
        if (ev) (void)hipEventRecord(ev[2 * it], s);
        kb_iter<float><<<t.st, 64 * NWV, 0, s>>>(D, off_st, P);
        if (ev) (void)hipEventRecord(ev[2 * it + 1], s);
        kb_tail<<<P, 256, 0, s>>>(D);
    }
    kb_ru_add<<<t.add, 256, 0, s>>>(D, off_add, P);
    kb_ru_residual<<<t.res, 256, 0, s>>>(D, off_res, P);
    kb_ru_fin<<<P, 256, 0, s>>>(D);
    kb_gather<<<(P + 63) / 64, 64, 0, s>>>(D, P, gather_out);
    return hipGetLastError();
}

hipError_t launch_stream_copy(hipStream_t s, const void* a, void* b, size_t bytes)
{
    const int64_t n = (int64_t)(bytes / 16);
    k_stream_copy<<<1024, 256, 0, s>>>((const f4v*)a, (f4v*)b, n);
    return hipGetLastError();
}

TileShape make_tiles(const Grid& g, int planes)
{
    TileShape t;
    t.njt = (g.ny - 2 + TY - 1) / TY;
    t.nkt = (g.nz - 2 + ZW - 1) / ZW;
    const int tiles = t.njt * t.nkt;
    int lx = planes;
    if (lx <= 0) {
        // chunk length along x: every chunk re-reads the planes next to it, so chunks stay
        // long; they are shortened (down to 8 planes) while the grid would give fewer than
        // 2048 tiles, so that the 256 CUs have several blocks each
        lx = 32;
        while (lx > 8 && (long)tiles * ((g.nx - 2 + lx - 1) / lx) < 2048) lx >>= 1;
    }
    t.LX = lx;
    t.nxc = (g.nx - 2 + lx - 1) / lx;
    t.items = tiles * t.nxc;
    return t;
}

template <typename T>
hipError_t launch_cg_init(hipStream_t s, const Grid& g, const CGBufs<T>& B, Coef c, const double* b64, const T* bT)
{
    k_cg_init<T><<<B.nb, 256, 0, s>>>(g, B, c, b64, bT);
    return hipGetLastError();
}

hipError_t launch_cg_fin(hipStream_t s, const double* part, int nb, CGState* st, double rtol2)
{
    k_cg_fin<<<1, 256, 0, s>>>(part, nb, st, rtol2);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cg_iter(hipStream_t s, const Grid& g, const TileShape& ts, const CGBufs<T>& B, Coef c)
{
    k_cg_iter<T><<<ts.items, 64 * NWV, 0, s>>>(g, ts, B, c);
    return hipGetLastError();
}

hipError_t launch_cg_tail(hipStream_t s, const double* part, int nb, CGState* st)
{
    k_cg_tail<<<1, 256, 0, s>>>(part, nb, st);
    return hipGetLastError();
}

template hipError_t launch_cg_init<double>(hipStream_t, const Grid&, const CGBufs<double>&, Coef, const double*,
                                           const double*);
template hipError_t launch_cg_init<float>(hipStream_t, const Grid&, const CGBufs<float>&, Coef, const double*,
                                          const float*);
template hipError_t launch_cg_iter<double>(hipStream_t, const Grid&, const TileShape&, const CGBufs<double>&, Coef);
template hipError_t launch_cg_iter<float>(hipStream_t, const Grid&, const TileShape&, const CGBufs<float>&, Coef);

int residual_blocks(const Grid& g) { return (int)((g.N + 255) / 256); }

int add_blocks(const Grid& g)
{
    int64_t nb = (g.N / 4 + 255) / 256;
    return (int)(nb > 4096 ? 4096 : (nb < 1 ? 1 : nb));
}

hipError_t launch_ru_add(hipStream_t s, const Grid& g, CGState* st, double* x64, float* d32, float* const* p32,
                         int force)
{
    k_ru_add<<<(unsigned)add_blocks(g), 256, 0, s>>>(g.N / 4, st, x64, d32, p32[0], p32[1], force);
    return hipGetLastError();
}

hipError_t launch_ru_residual(hipStream_t s, const Grid& g, const uint32_t* code, const double* ck64, const float* ck32,
                              Coef c, const double* b, const double* x64, float* const* z32, double* part3, CGState* st)
{
    k_ru_residual<<<(unsigned)residual_blocks(g), 256, 0, s>>>(g, code, ck64, ck32, c, b, x64, z32[0], z32[1], part3,
                                                               st);
    return hipGetLastError();
}

hipError_t launch_ru_begin(hipStream_t s, CGState* st)
{
    k_ru_begin<<<1, 1, 0, s>>>(st);
    return hipGetLastError();
}

hipError_t launch_ru_fin(hipStream_t s, CGState* st, const double* part3, int nbres, int init, double rtol2,
                         double delta2)
{
    k_ru_fin<<<1, 256, 0, s>>>(st, part3, nbres, init, rtol2, delta2);
    return hipGetLastError();
}

}  // namespace pbk
