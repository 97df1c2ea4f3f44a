// pb_solve.hip -- Jacobi-preconditioned conjugate gradients on the condensed 7-point
// operator (paper Sect. 3.1, eq. matrixequation, with the edge permittivities of Sect. 3.2),
// matrix-free, for FP64 and FP32 data.
//
// One CG iteration is two kernels and no host round trip:
//   stencil(par): reduce the previous r.z and r.r partials (every block, fixed order),
//                 test convergence, beta = rz/rz_old; then per tile
//                 p_new = D^-1 r + beta p_old (also on the halo), q = A p_new,
//                 partial sums of p_new.q
//   update(par):  reduce the p.q partials, alpha = rz/pq; x += alpha p, r -= alpha q,
//                 partial sums of r.(D^-1 r) and r.r
// The scalars never leave the device; every block reduces the same partial array in the
// same order, so all blocks agree bit for bit and the result is run-to-run deterministic.
//
// The stencil kernel tiles the interior into 64 (z, one wave) x TY (y, 4 waves x TY/4 rows)
// columns and marches along x over a chunk of planes, carrying the x-neighbours in
// registers and staging the current plane with its y/z halo in LDS.  Tiles are numbered
// z-fastest and handed out so that each XCD gets one contiguous range of tiles, which keeps
// the y-halo rows of neighbouring tiles in the same L2.
#include "pb_internal.h"

#include <cmath>

namespace pbk {

namespace {

__device__ __forceinline__ void block_sum2(double& a, double& b, double* sh)
{
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
    }
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) {
        sh[w] = a;
        sh[4 + w] = b;
    }
    __syncthreads();
    a = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    b = (sh[4] + sh[5]) + (sh[6] + sh[7]);
}

template <typename T>
__device__ __forceinline__ T eK(uint32_t c, int ax, const T* __restrict__ ck, T kin, T kout)
{
    if (c & (C_CUTX << ax)) return ck[3 * (int64_t)(c >> C_SLOT_SHIFT) + ax];
    return (c & C_SOLUTE) ? kin : kout;
}

// K of the edge from a node along +axis without a branch: a cut edge reads its WHA value
// from the compact table, an edge inside one medium takes h*eps of that medium.  The table
// is always read (slot 0 for uncut edges) and the result is blended arithmetically, so the
// load is never turned into a branch whose join would wait on every load in flight.
template <typename T>
__device__ __forceinline__ T edgeK(uint32_t c, int ax, const T* __restrict__ ck, T kin, T kout)
{
    const bool cut = (c & (C_CUTX << ax)) != 0;
    const int64_t ix = cut ? 3 * (int64_t)(c >> C_SLOT_SHIFT) + ax : 0;
    const T v = ck[ix];
    const T base = (c & C_SOLUTE) ? kin : kout;
    const T m = cut ? (T)1 : (T)0;
    return v * m + base * ((T)1 - m);
}

// the same split in two: the table index (any edge; slot 0 when uncut) and the blend
__device__ __forceinline__ int64_t ck_index(uint32_t c, int ax)
{
    return (c & (C_CUTX << ax)) ? 3 * (int64_t)(c >> C_SLOT_SHIFT) + ax : 0;
}

template <typename T>
__device__ __forceinline__ T ck_blend(T v, uint32_t c, int ax, T kin, T kout)
{
    const T base = (c & C_SOLUTE) ? kin : kout;
    const T m = (c & (C_CUTX << ax)) ? (T)1 : (T)0;
    return v * m + base * ((T)1 - m);
}

template <typename T>
struct Raw {   // what one node contributes to p_new = D^-1 r + beta p_old
    T r, po;
    float di;
    uint32_t c;
};

template <typename T>
struct K3 {    // coefficients of the +x, +y, +z edges of a node
    T x, y, z;
};

template <typename T>
__device__ __forceinline__ void stencil_body(const Grid& g, const TileShape& ts, const CGBufs<T>& B, const Coef& cf,
                                             const int bid)
{
    constexpr int RY = TY / 4;
    __shared__ double sh[8];
    __shared__ T sp[TY + 2][66];   // p_new of plane i: rows j0-1..j0+TY, cols k0-1..k0+64
    __shared__ T sky[TY + 1][64];  // K of the +y edge: rows j0-1..j0+TY-1, cols k0..k0+63
    __shared__ T skz[TY][65];      // K of the +z edge: own rows, cols k0-1..k0+63
    CGState* st = B.st;
    if (st->status != 0) return;
    const int par = st->iter_count & 1;

    double rz = 0.0, rr = 0.0;
    for (int t = threadIdx.x; t < B.nb2; t += 256) {
        rz += B.part2[t];
        rr += B.part2[B.nb2 + t];
    }
    block_sum2(rz, rr, sh);
    const bool first = bid == 0 && threadIdx.x == 0;
    if (rr <= st->stop2) {
        if (first) {
            st->status = st->stop_status;
            st->iters = st->iter_count;
            st->rr = rr;
        }
        return;
    }
    if (!isfinite(rz) || !isfinite(rr)) {
        if (first) st->status = 2;
        return;
    }
    const double beta = rz / st->rz[par ^ 1];
    if (first) {
        st->rz[par] = rz;
        st->rr = rr;
        st->par = par;
    }
    const T bT = (T)beta;
    const T kin = (T)cf.kin, kout = (T)cf.kout, mass = (T)cf.mass;

    // XCD-aware bijective block -> tile map (blocks are dealt round-robin to 8 XCDs)
    const int W = ts.items, b = bid;
    const int q8 = W >> 3, rem = W & 7, xcd = b & 7;
    const int item = xcd * q8 + (xcd < rem ? xcd : rem) + (b >> 3);
    const int kt = item % ts.nkt;
    const int t2 = item / ts.nkt;
    const int jt = t2 % ts.njt;
    const int xc = t2 / ts.njt;
    const int k0 = 1 + kt * 64, j0 = 1 + jt * TY;
    const int ib = 1 + xc * ts.LX;
    const int ie = (ib + ts.LX < g.nx - 1) ? ib + ts.LX : g.nx - 1;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;

    const T* __restrict__ r = B.r;
    const T* __restrict__ pold = B.p[par ^ 1];
    T* __restrict__ pnew = B.p[par];
    const float* __restrict__ dinv = B.dinv;
    const uint32_t* __restrict__ code = B.code;
    const T* __restrict__ ck = B.ck;
    const int64_t sx = (int64_t)g.ny * g.S;

    // Out-of-interior positions are clamped onto box nodes, where r = p = D^-1 = 0: every
    // load below is unconditional and in bounds, and a clamped node contributes p_new = 0.
    auto clampj = [&](int j) { return j < 0 ? 0 : (j > g.ny - 1 ? g.ny - 1 : j); };
    auto clampk = [&](int k) { return k < 0 ? 0 : (k > g.nz - 1 ? g.nz - 1 : k); };
    auto load = [&](int64_t e) {
        Raw<T> v;
        v.r = r[e];
        v.po = pold[e];
        v.di = dinv[e];
        v.c = code[e];
        return v;
    };
    auto pval = [&](const Raw<T>& v) { return (T)v.di * v.r + bT * v.po; };

    // own columns (z = k0 + lane, rows j0 + wv*RY + q) and this thread's halo point
    const int k = k0 + lane;
    const int kc = clampk(k);
    int64_t eo[RY];
    bool valid[RY];
#pragma unroll
    for (int q = 0; q < RY; ++q) {
        const int j = j0 + wv * RY + q;
        valid[q] = j <= g.ny - 2 && k <= g.nz - 2;
        eo[q] = g.idx(0, clampj(j), kc);
    }
    // halo: wave 0 row j0-1 (needs p and K+y), wave 1 row j0+TY (p), wave 2 column k0-1
    // (p and K+z), wave 3 column k0+64 (p); waves 2 and 3 use their first TY lanes
    int hj, hk;
    bool hact = true;
    if (wv == 0) { hj = j0 - 1; hk = k0 + lane; }
    else if (wv == 1) { hj = j0 + TY; hk = k0 + lane; }
    else { hact = lane < TY; hj = j0 + (lane < TY ? lane : TY - 1); hk = (wv == 2) ? k0 - 1 : k0 + 64; }
    const int64_t eh = g.idx(0, clampj(hj), clampk(hk));
    const int hax = wv == 0 ? 1 : 2;

    // prologue: plane ib-1 (p, K+x), ib (p, K), ib+1 (p, K), halo of ib (p, K)
    T pm[RY], pc[RY], px[RY], kxm[RY];
    uint32_t cc[RY], cxn[RY];   // node codes of planes i and i+1
    K3<T> kr[RY];               // raw table reads for the edge coefficients of plane i
    Raw<T> nxt[RY];
#pragma unroll
    for (int q = 0; q < RY; ++q) {
        const Raw<T> a = load(eo[q] + (int64_t)(ib - 1) * sx);
        const Raw<T> c0 = load(eo[q] + (int64_t)ib * sx);
        const Raw<T> c1 = load(eo[q] + (int64_t)(ib + 1) * sx);
        pm[q] = pval(a);
        kxm[q] = edgeK(a.c, 0, ck, kin, kout);
        pc[q] = pval(c0);
        cc[q] = c0.c;
        kr[q].x = ck[ck_index(c0.c, 0)];
        kr[q].y = ck[ck_index(c0.c, 1)];
        kr[q].z = ck[ck_index(c0.c, 2)];
        px[q] = pval(c1);
        cxn[q] = c1.c;
    }
    Raw<T> hraw = load(eh + (int64_t)ib * sx);
    T hv = pval(hraw);
    uint32_t hc = hraw.c;
    T hr = ck[ck_index(hc, hax)];

    T acc = (T)0;
    for (int i = ib; i < ie; ++i) {
        // prefetch: own plane i+2 (never past plane ie, the last one this chunk needs) and
        // the halo of plane i+1
        const int i2 = (i + 2 < ie) ? i + 2 : ie;
#pragma unroll
        for (int q = 0; q < RY; ++q) nxt[q] = load(eo[q] + (int64_t)i2 * sx);
        const Raw<T> hn = load(eh + (int64_t)(i + 1) * sx);

        // stage plane i in LDS: p_new and the +y/+z edge coefficients
        K3<T> kc3[RY];
#pragma unroll
        for (int q = 0; q < RY; ++q) {
            const int row = wv * RY + q;
            kc3[q].x = ck_blend(kr[q].x, cc[q], 0, kin, kout);
            kc3[q].y = ck_blend(kr[q].y, cc[q], 1, kin, kout);
            kc3[q].z = ck_blend(kr[q].z, cc[q], 2, kin, kout);
            sp[1 + row][1 + lane] = pc[q];
            sky[1 + row][lane] = kc3[q].y;
            skz[row][1 + lane] = kc3[q].z;
        }
        const T hK = ck_blend(hr, hc, hax, kin, kout);
        if (wv == 0) {
            sp[0][1 + lane] = hv;
            sky[0][lane] = hK;
        } else if (wv == 1) {
            sp[TY + 1][1 + lane] = hv;
        } else if (hact) {
            if (wv == 2) {
                sp[1 + lane][0] = hv;
                skz[lane][0] = hK;
            } else {
                sp[1 + lane][65] = hv;
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < RY; ++q) {
            const int row = wv * RY + q;
            const T Kym = sky[row][lane], Kyp = sky[1 + row][lane];
            const T Kzm = skz[row][lane], Kzp = skz[row][1 + lane];
            const T Kxp = kc3[q].x;
            const T D = ((kxm[q] + Kxp) + (Kym + Kyp)) + ((Kzm + Kzp) + ((cc[q] & C_SOLUTE) ? (T)0 : mass));
            const T p0 = pc[q];
            const T nbs = kxm[q] * pm[q] + Kxp * px[q] + Kym * sp[row][1 + lane] +
                          Kyp * sp[row + 2][1 + lane] + Kzm * sp[1 + row][lane] + Kzp * sp[1 + row][2 + lane];
            const T qv = D * p0 - nbs;
            // a lane outside the interior was clamped onto a box node, whose p and q stay
            // 0: it stores zeros there, so the stores need no branch
            const int64_t e = eo[q] + (int64_t)i * sx;
            pnew[e] = valid[q] ? p0 : (T)0;
            B.q[e] = valid[q] ? qv : (T)0;
            acc += valid[q] ? p0 * qv : (T)0;
        }
        __syncthreads();
        // rotate.  The coefficient lookups of plane i+1 are issued last, straight into the
        // registers that consume them, so no register copy waits on a load in flight and
        // the next step's prefetch loads are never waited for before they are needed.
#pragma unroll
        for (int q = 0; q < RY; ++q) {
            pm[q] = pc[q];
            kxm[q] = kc3[q].x;
            pc[q] = px[q];
            cc[q] = cxn[q];
            px[q] = pval(nxt[q]);
            cxn[q] = nxt[q].c;
        }
        hv = pval(hn);
        hc = hn.c;
#pragma unroll
        for (int q = 0; q < RY; ++q) {
            kr[q].x = ck[ck_index(cc[q], 0)];
            kr[q].y = ck[ck_index(cc[q], 1)];
            kr[q].z = ck[ck_index(cc[q], 2)];
        }
        hr = ck[ck_index(hc, hax)];
    }
    double a = (double)acc, dummy = 0.0;
    block_sum2(a, dummy, sh);
    if (threadIdx.x == 0) B.part1[bid] = a;
}

template <typename T>
__global__ void __launch_bounds__(256) k_cg_stencil(Grid g, TileShape ts, CGBufs<T> B, Coef cf)
{
    stencil_body(g, ts, B, cf, (int)blockIdx.x);
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

template <typename T>
__device__ __forceinline__ void update_body(int64_t n4, const CGBufs<T>& B, const int bid, const int nblk)
{
    __shared__ double sh[8];
    CGState* st = B.st;
    if (st->status != 0) return;
    const int par = st->par;
    double pq = 0.0, dummy = 0.0;
    for (int t = threadIdx.x; t < B.nb1; t += 256) pq += B.part1[t];
    block_sum2(pq, dummy, sh);
    const bool first = bid == 0 && threadIdx.x == 0;
    if (!(pq > 0.0) || !isfinite(pq)) {
        if (first) {
            st->status = 2;
            st->pq = pq;
        }
        return;
    }
    const T aT = (T)(st->rz[par] / pq);
    using V = typename Vec4<T>::type;
    V* __restrict__ x = reinterpret_cast<V*>(B.x);
    V* __restrict__ r = reinterpret_cast<V*>(B.r);
    const V* __restrict__ p = reinterpret_cast<const V*>(B.p[par]);
    const V* __restrict__ q = reinterpret_cast<const V*>(B.q);
    const float4* __restrict__ dv = reinterpret_cast<const float4*>(B.dinv);
    T rz = (T)0, rr = (T)0;
    const int64_t stride = (int64_t)nblk * 256;
    for (int64_t v = (int64_t)bid * 256 + threadIdx.x; v < n4; v += stride) {
        V xv = x[v], rv = r[v];
        const V pv = p[v], qv = q[v];
        const float4 d = dv[v];
        xv.x += aT * pv.x; xv.y += aT * pv.y; xv.z += aT * pv.z; xv.w += aT * pv.w;
        rv.x -= aT * qv.x; rv.y -= aT * qv.y; rv.z -= aT * qv.z; rv.w -= aT * qv.w;
        x[v] = xv;
        r[v] = rv;
        rz += rv.x * ((T)d.x * rv.x) + rv.y * ((T)d.y * rv.y) + rv.z * ((T)d.z * rv.z) + rv.w * ((T)d.w * rv.w);
        rr += rv.x * rv.x + rv.y * rv.y + rv.z * rv.z + rv.w * rv.w;
    }
    double a = (double)rz, c = (double)rr;
    block_sum2(a, c, sh);
    if (threadIdx.x == 0) {
        B.part2[bid] = a;
        B.part2[B.nb2 + bid] = c;
    }
    if (first) st->iter_count += 1;
}

template <typename T>
__global__ void __launch_bounds__(256) k_cg_update(int64_t n4, CGBufs<T> B)
{
    update_body(n4, B, (int)blockIdx.x, (int)gridDim.x);
}

template <typename T>
__global__ void __launch_bounds__(256) k_cg_init(int64_t n4, CGBufs<T> B, const double* b64, const T* bT)
{
    __shared__ double sh[8];
    using V = typename Vec4<T>::type;
    T rz = (T)0, rr = (T)0;
    const int64_t stride = (int64_t)gridDim.x * 256;
    V* x = reinterpret_cast<V*>(B.x);
    V* r = reinterpret_cast<V*>(B.r);
    V* p0 = reinterpret_cast<V*>(B.p[0]);
    V* p1 = reinterpret_cast<V*>(B.p[1]);
    V* q = reinterpret_cast<V*>(B.q);
    const float4* dv = reinterpret_cast<const float4*>(B.dinv);
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < n4; v += stride) {
        V bv;
        if (b64) {
            const double4 t = reinterpret_cast<const double4*>(b64)[v];
            bv.x = (T)t.x; bv.y = (T)t.y; bv.z = (T)t.z; bv.w = (T)t.w;
        } else {
            bv = reinterpret_cast<const V*>(bT)[v];
        }
        const float4 d = dv[v];
        V z0;
        z0.x = 0; z0.y = 0; z0.z = 0; z0.w = 0;
        x[v] = z0;
        p0[v] = z0;
        p1[v] = z0;
        q[v] = z0;
        r[v] = bv;
        rz += bv.x * ((T)d.x * bv.x) + bv.y * ((T)d.y * bv.y) + bv.z * ((T)d.z * bv.z) + bv.w * ((T)d.w * bv.w);
        rr += bv.x * bv.x + bv.y * bv.y + bv.z * bv.z + bv.w * bv.w;
    }
    double a = (double)rz, c = (double)rr;
    block_sum2(a, c, sh);
    if (threadIdx.x == 0) {
        B.part2[blockIdx.x] = a;
        B.part2[B.nb2 + blockIdx.x] = c;
    }
}

__global__ void __launch_bounds__(256) k_cg_fin(const double* part2, int nb2, CGState* st, double rtol2)
{
    __shared__ double sh[8];
    double rz = 0.0, rr = 0.0;
    for (int t = threadIdx.x; t < nb2; t += 256) {
        rz += part2[t];
        rr += part2[nb2 + t];
    }
    block_sum2(rz, rr, sh);
    if (threadIdx.x == 0) {
        st->rz[0] = rz;
        st->rz[1] = INFINITY;  // first iteration: beta = rz / inf = 0
        st->bnorm2 = rr;
        st->rr = rr;
        st->pq = 0.0;
        st->stop2 = rtol2 * rr;
        st->trig2 = -1.0;
        st->delta2 = 0.0;
        st->goal64 = 0.0;
        st->rr64 = 0.0;
        st->status = 0;
        st->stop_status = 1;
        st->iters = 0;
        st->iter_count = 0;
        st->par = 0;
        st->ru = 0;
        st->n_ru = 0;
        st->pad = 0;
    }
}

// ---- mixed precision: FP32 CG with FP64 reliable updates ------------------------------------
// The FP32 iteration runs on; a reliable update folds the FP32 correction into the FP64
// solution and replaces the FP32 residual by the FP64 true residual b - A x64 (FP64 operator,
// exact coefficients), keeping the search direction.  An update runs at a chunk end once the
// recursive residual has dropped by delta since the last one, or when the recursive residual
// reaches the target (the stencil kernel then stops with status 3).

__device__ __forceinline__ void ru_add_body(int64_t n4, CGState* st, double* x, float* d, int force, const int bid,
                                            const int nblk)
{
    const int s0 = st->status;
    const bool go = (s0 == 3) || (s0 == 0 && (force || st->rr <= st->trig2));
    if (!go) return;
    const int64_t stride = (int64_t)nblk * 256;
    for (int64_t v = (int64_t)bid * 256 + threadIdx.x; v < n4; v += stride) {
        double4 xv = reinterpret_cast<double4*>(x)[v];
        const float4 dv = reinterpret_cast<const float4*>(d)[v];
        xv.x += (double)dv.x; xv.y += (double)dv.y; xv.z += (double)dv.z; xv.w += (double)dv.w;
        reinterpret_cast<double4*>(x)[v] = xv;
        reinterpret_cast<float4*>(d)[v] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    if (bid == 0 && threadIdx.x == 0) st->ru = 1;
}

__global__ void __launch_bounds__(256) k_ru_add(int64_t n4, CGState* st, double* x, float* d, int force)
{
    ru_add_body(n4, st, x, d, force, (int)blockIdx.x, (int)gridDim.x);
}

__device__ __forceinline__ void ru_residual_body(const Grid& g, const uint32_t* __restrict__ code,
                                                 const double* __restrict__ ck, const Coef& cf,
                                                 const double* __restrict__ b, const double* __restrict__ x,
                                                 const float* __restrict__ dinv, float* __restrict__ r32,
                                                 double* __restrict__ part3, CGState* st, const int bid, const int nblk)
{
    __shared__ double sh[8];
    if (!st->ru) return;
    const int64_t e = (int64_t)bid * 256 + threadIdx.x;
    double rr64 = 0.0;
    float rz32 = 0.0f, rr32 = 0.0f;
    if (e < g.N) {
        const uint32_t c = code[e];
        float out = 0.0f;
        if (!(c & C_BOX)) {
            const int64_t sx = (int64_t)g.ny * g.S, sy = g.S;
            const double Kxm = eK(code[e - sx], 0, ck, cf.kin, cf.kout);
            const double Kxp = eK(c, 0, ck, cf.kin, cf.kout);
            const double Kym = eK(code[e - sy], 1, ck, cf.kin, cf.kout);
            const double Kyp = eK(c, 1, ck, cf.kin, cf.kout);
            const double Kzm = eK(code[e - 1], 2, ck, cf.kin, cf.kout);
            const double Kzp = eK(c, 2, ck, cf.kin, cf.kout);
            const double D = ((Kxm + Kxp) + (Kym + Kyp)) + ((Kzm + Kzp) + ((c & C_SOLUTE) ? 0.0 : cf.mass));
            const double ax = D * x[e] - (Kxm * x[e - sx] + Kxp * x[e + sx] + Kym * x[e - sy] +
                                          Kyp * x[e + sy] + Kzm * x[e - 1] + Kzp * x[e + 1]);
            const double rv = b[e] - ax;
            rr64 = rv * rv;
            out = (float)rv;
            rz32 = out * (dinv[e] * out);
            rr32 = out * out;
        }
        r32[e] = out;
    }
    double a = (double)rz32, c2 = (double)rr32;
    block_sum2(a, c2, sh);
    double dummy = 0.0;
    block_sum2(rr64, dummy, sh);
    if (threadIdx.x == 0) {
        part3[bid] = rr64;
        part3[nblk + bid] = a;
        part3[2 * nblk + bid] = c2;
    }
}

__global__ void __launch_bounds__(256) k_ru_residual(Grid g, const uint32_t* __restrict__ code,
                                                     const double* __restrict__ ck, Coef cf,
                                                     const double* __restrict__ b, const double* __restrict__ x,
                                                     const float* __restrict__ dinv, float* __restrict__ r32,
                                                     double* __restrict__ part3, CGState* st)
{
    ru_residual_body(g, code, ck, cf, b, x, dinv, r32, part3, st, (int)blockIdx.x, (int)gridDim.x);
}

__global__ void k_ru_begin(CGState* st)
{
    st->status = 0;
    st->ru = 1;
}

// one block: finish a reliable update (or, with init, set up the mixed iteration)
__device__ __forceinline__ void ru_fin_body(CGState* st, const double* part3, int nbres, double* part2, int nb2,
                                            int init, double rtol2, double delta2)
{
    __shared__ double sh[8];
    if (!st->ru) return;
    double rr64 = 0.0, rz = 0.0, rr = 0.0, dummy = 0.0;
    for (int t = threadIdx.x; t < nbres; t += 256) {
        rr64 += part3[t];
        rz += part3[nbres + t];
        rr += part3[2 * nbres + t];
    }
    block_sum2(rz, rr, sh);
    block_sum2(rr64, dummy, sh);
    for (int t = threadIdx.x; t < nb2; t += 256) {
        part2[t] = t == 0 ? rz : 0.0;
        part2[nb2 + t] = t == 0 ? rr : 0.0;
    }
    if (threadIdx.x == 0) {
        if (init) {
            st->rz[0] = rz;
            st->rz[1] = INFINITY;
            st->bnorm2 = rr;
            st->pq = 0.0;
            st->stop2 = rtol2 * rr;
            st->delta2 = delta2;
            st->goal64 = rtol2 * rr64;
            st->stop_status = 3;
            st->iters = 0;
            st->iter_count = 0;
            st->par = 0;
            st->n_ru = 0;
            st->pad = 0;
        } else {
            st->n_ru += 1;
        }
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

__global__ void __launch_bounds__(256) k_ru_fin(CGState* st, const double* part3, int nbres, double* part2,
                                                int nb2, int init, double rtol2, double delta2)
{
    ru_fin_body(st, part3, nbres, part2, nb2, init, rtol2, delta2);
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
// computes when solved alone.

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
__global__ void __launch_bounds__(256) kb_stencil(const ProbDev<T>* __restrict__ D, const int* __restrict__ off, int P)
{
    const int p = __builtin_amdgcn_readfirstlane(find_prob(off, P, (int)blockIdx.x));
    const ProbDev<T>& d = D[p];
    stencil_body(d.g, d.ts, d.B, d.cf, (int)blockIdx.x - off[p]);
}

template <typename T>
__global__ void __launch_bounds__(256) kb_update(const ProbDev<T>* __restrict__ D, const int* __restrict__ off, int P)
{
    const int p = __builtin_amdgcn_readfirstlane(find_prob(off, P, (int)blockIdx.x));
    const ProbDev<T>& d = D[p];
    update_body(d.g.N / 4, d.B, (int)blockIdx.x - off[p], d.B.nb2);
}

__global__ void __launch_bounds__(256) kb_ru_add(const ProbDev<float>* __restrict__ D, const int* __restrict__ off, int P)
{
    const int p = __builtin_amdgcn_readfirstlane(find_prob(off, P, (int)blockIdx.x));
    const ProbDev<float>& d = D[p];
    ru_add_body(d.g.N / 4, d.B.st, d.x64, d.B.x, 0, (int)blockIdx.x - off[p], d.nadd);
}

__global__ void __launch_bounds__(256) kb_ru_residual(const ProbDev<float>* __restrict__ D, const int* __restrict__ off,
                                                      int P)
{
    const int p = __builtin_amdgcn_readfirstlane(find_prob(off, P, (int)blockIdx.x));
    const ProbDev<float>& d = D[p];
    ru_residual_body(d.g, d.B.code, d.ck64, d.cf, d.rhs, d.x64, d.B.dinv, d.B.r, d.part3, d.B.st,
                     (int)blockIdx.x - off[p], d.nbres);
}

__global__ void __launch_bounds__(256) kb_ru_fin(const ProbDev<float>* __restrict__ D)
{
    const ProbDev<float>& d = D[blockIdx.x];
    ru_fin_body(d.B.st, d.part3, d.nbres, d.B.part2, d.B.nb2, 0, 0.0, 0.0);
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
    const int* off_up = off + (P + 1);
    const int* off_add = off + 2 * (P + 1);
    const int* off_res = off + 3 * (P + 1);
    for (int it = 0; it < iters; ++it) {
        if (ev) (void)hipEventRecord(ev[2 * it], s);
        kb_stencil<float><<<t.st, 256, 0, s>>>(D, off_st, P);
        if (ev) (void)hipEventRecord(ev[2 * it + 1], s);
        kb_update<float><<<t.up, 256, 0, s>>>(D, off_up, P);
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

TileShape make_tiles(const Grid& g)
{
    TileShape t;
    t.njt = (g.ny - 2 + TY - 1) / TY;
    t.nkt = (g.nz - 2 + 63) / 64;
    const int tiles = t.njt * t.nkt;
#ifdef PB_FORCE_LX
    int lx = PB_FORCE_LX;
#else
    // chunk length along x: every chunk re-reads the planes next to it, so chunks stay long;
    // they are shortened (down to 8 planes) while the grid would give fewer than 4096 tiles,
    // so that the 256 CUs have several blocks each
    int lx = 32;
    while (lx > 8 && (long)tiles * ((g.nx - 2 + lx - 1) / lx) < 4096) lx >>= 1;
#endif
    t.LX = lx;
    t.nxc = (g.nx - 2 + lx - 1) / lx;
    t.items = tiles * t.nxc;
    return t;
}

int update_blocks(const Grid& g)
{
    const int64_t n4 = g.N / 4;
    int64_t b = (n4 + 255) / 256;
    if (b > 512) b = 512;
    if (b < 1) b = 1;
    return (int)b;
}

template <typename T>
hipError_t launch_cg_init(hipStream_t s, const Grid& g, const CGBufs<T>& B, const double* b64, const T* bT)
{
    k_cg_init<T><<<B.nb2, 256, 0, s>>>(g.N / 4, B, b64, bT);
    return hipGetLastError();
}

hipError_t launch_cg_fin(hipStream_t s, double* part2, int nb2, CGState* st, double rtol2)
{
    k_cg_fin<<<1, 256, 0, s>>>(part2, nb2, st, rtol2);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cg_stencil(hipStream_t s, const Grid& g, const TileShape& ts, const CGBufs<T>& B, Coef c)
{
    k_cg_stencil<T><<<ts.items, 256, 0, s>>>(g, ts, B, c);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cg_update(hipStream_t s, const Grid& g, const CGBufs<T>& B)
{
    k_cg_update<T><<<B.nb2, 256, 0, s>>>(g.N / 4, B);
    return hipGetLastError();
}

template hipError_t launch_cg_init<double>(hipStream_t, const Grid&, const CGBufs<double>&, const double*,
                                           const double*);
template hipError_t launch_cg_init<float>(hipStream_t, const Grid&, const CGBufs<float>&, const double*,
                                          const float*);
template hipError_t launch_cg_stencil<double>(hipStream_t, const Grid&, const TileShape&,
                                              const CGBufs<double>&, Coef);
template hipError_t launch_cg_stencil<float>(hipStream_t, const Grid&, const TileShape&, const CGBufs<float>&,
                                             Coef);
template hipError_t launch_cg_update<double>(hipStream_t, const Grid&, const CGBufs<double>&);
template hipError_t launch_cg_update<float>(hipStream_t, const Grid&, const CGBufs<float>&);

int residual_blocks(const Grid& g) { return (int)((g.N + 255) / 256); }

int add_blocks(const Grid& g)
{
    int64_t nb = (g.N / 4 + 255) / 256;
    return (int)(nb > 4096 ? 4096 : (nb < 1 ? 1 : nb));
}

hipError_t launch_ru_add(hipStream_t s, const Grid& g, CGState* st, double* x64, float* d32, int force)
{
    k_ru_add<<<(unsigned)add_blocks(g), 256, 0, s>>>(g.N / 4, st, x64, d32, force);
    return hipGetLastError();
}

hipError_t launch_ru_residual(hipStream_t s, const Grid& g, const uint32_t* code, const double* ck64, Coef c,
                              const double* b, const double* x64, const float* dinv, float* r32, double* part3,
                              CGState* st)
{
    k_ru_residual<<<(unsigned)residual_blocks(g), 256, 0, s>>>(g, code, ck64, c, b, x64, dinv, r32, part3, st);
    return hipGetLastError();
}

hipError_t launch_ru_begin(hipStream_t s, CGState* st)
{
    k_ru_begin<<<1, 1, 0, s>>>(st);
    return hipGetLastError();
}

hipError_t launch_ru_fin(hipStream_t s, CGState* st, const double* part3, int nbres, double* part2, int nb2,
                         int init, double rtol2, double delta2)
{
    k_ru_fin<<<1, 256, 0, s>>>(st, part3, nbres, part2, nb2, init, rtol2, delta2);
    return hipGetLastError();
}

}  // namespace pbk
