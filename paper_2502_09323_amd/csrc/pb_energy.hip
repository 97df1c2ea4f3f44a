// pb_energy.hip -- solvation energy read back at the atoms (paper Sect. 3.3), FP64.
//
//   per cut edge p:  F_p   = K_e (phi_s - phi_w)                      flux of D_eff through
//                                                                      the edge's square
//                    phi_p = phi_s + (alpha/eps_in) eps_eff (phi_w - phi_s)   (eq. phi0)
//   per atom i:      S_F(i) = sum_p F_p / |r_p - r_i|
//                    S_D(i) = sum_p w_p phi_p (r_p - r_i).n_p / |r_p - r_i|^3
//   phi_pol(i) = (1/eps_out - 1/eps_in) S_F/(4 pi)      (polarization charges q_p at r_p)
//   phi_ion(i) = S_D/(4 pi) - S_F/(4 pi eps_out)        (eq. energy_ion)
//   E_pol = 1/2 lB sum q_i phi_pol(i),  E_ion = 1/2 lB sum q_i phi_ion(i),
//   E_coul = 1/2 lB sum_i q_i sum_{j != i} q_j /(eps_in r_ij)
//
// The atoms x cut-points sum is the FP64 vector-ALU hot spot: points are staged through
// LDS in tiles, each thread owns one atom, and the cut list is split into chunks whose
// per-atom partials are summed in chunk order, so the result does not depend on timing.
#include "pb_internal.h"

#include <cmath>

namespace pbk {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int NB_TILE = 256;

__device__ __forceinline__ void block_sum2(double& a, double& b, double* sh, int nw)
{
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
    }
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) {
        sh[w] = a;
        sh[16 + w] = b;
    }
    __syncthreads();
    a = 0.0;
    b = 0.0;
    for (int q = 0; q < nw; ++q) {
        a += sh[q];
        b += sh[16 + q];
    }
}

__global__ void __launch_bounds__(256) k_edge_fields(Grid g, double eps_in, double eps_out, int64_t ncut,
                                                     const int64_t* cutkey, const uint32_t* code,
                                                     const double* alpha, const double* kcut,
                                                     const double* x, const double* gb, const double* wp,
                                                     double* F, double* phip, double* pts,
                                                     const double* rp, const double* np)
{
    int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= ncut) return;
    const int64_t key = cutkey[c];
    const int64_t e = key >> 2;
    const int ax = (int)(key & 3);
    const int64_t st[3] = {(int64_t)g.ny * g.S, g.S, 1};
    const int64_t e2 = e + st[ax];
    const bool low_sol = (code[e] & C_SOLUTE) != 0;
    const int64_t s = low_sol ? e : e2, w = low_sol ? e2 : e;
    const double ps = x[s] + gb[s], pw = x[w] + gb[w];
    const double al = alpha[c];
    const double ee = 1.0 / (al / eps_in + (1.0 - al) / eps_out);
    const double f = g.h * ee * (ps - pw);
    const double pp = ps + (al / eps_in) * ee * (pw - ps);
    (void)kcut;
    F[c] = f;
    phip[c] = pp;
    double* o = pts + 8 * c;
    o[0] = rp[3 * c];
    o[1] = rp[3 * c + 1];
    o[2] = rp[3 * c + 2];
    o[3] = np[3 * c];
    o[4] = np[3 * c + 1];
    o[5] = np[3 * c + 2];
    o[6] = f;
    o[7] = wp[c] * pp;
}

// 1/sqrt(x) in FP64: the FP32 reciprocal square root as a start, then two Newton steps
// y <- y (3 - x y^2) / 2, each of which squares the relative error (about 1e-7 -> 1e-14 ->
// rounding level), in place of the library's FP64 square root and division
__device__ __forceinline__ double rsqrt_nr(double x)
{
    double y = (double)rsqrtf((float)x);
    y = y * (1.5 - 0.5 * (x * y * y));
    y = y * (1.5 - 0.5 * (x * y * y));
    return y;
}

// grid (ceil(n_atoms/512), nchunk), two atoms per thread (a and a + 256), so that each cut
// point read from LDS serves two pairs; partial[(chunk*n + i)*2 + {0,1}] = {S_F, S_D} over
// the chunk
__global__ void __launch_bounds__(256) k_nbody(Atoms at, int64_t ncut, const double* __restrict__ pts,
                                               double* __restrict__ partial, int64_t chunk_len)
{
    __shared__ double sp[NB_TILE * 8];
    const int a0 = blockIdx.x * 512 + threadIdx.x, a1 = a0 + 256;
    const bool act0 = a0 < at.n, act1 = a1 < at.n;
    double x0 = 0, y0 = 0, z0 = 0, x1 = 0, y1 = 0, z1 = 0;
    if (act0) {
        x0 = at.xyzr[4 * a0];
        y0 = at.xyzr[4 * a0 + 1];
        z0 = at.xyzr[4 * a0 + 2];
    }
    if (act1) {
        x1 = at.xyzr[4 * a1];
        y1 = at.xyzr[4 * a1 + 1];
        z1 = at.xyzr[4 * a1 + 2];
    } else {
        // an inactive slot evaluates the pairs of a far point, whose sums are discarded
        x1 = x0 + 1e3;
        y1 = y0;
        z1 = z0;
    }
    const int64_t p0 = (int64_t)blockIdx.y * chunk_len;
    int64_t p1 = p0 + chunk_len;
    if (p1 > ncut) p1 = ncut;
    double sf0 = 0.0, sd0 = 0.0, sf1 = 0.0, sd1 = 0.0;
    for (int64_t base = p0; base < p1; base += NB_TILE) {
        const int m = (int)((p1 - base) < NB_TILE ? (p1 - base) : NB_TILE);
        __syncthreads();
        for (int t = threadIdx.x; t < m * 8; t += 256) sp[t] = pts[base * 8 + t];
        __syncthreads();
        if (act0) {
            for (int u = 0; u < m; ++u) {
                const double* P = sp + 8 * u;
                const double dx0 = P[0] - x0, dy0 = P[1] - y0, dz0 = P[2] - z0;
                const double dx1 = P[0] - x1, dy1 = P[1] - y1, dz1 = P[2] - z1;
                const double r0 = rsqrt_nr(dx0 * dx0 + dy0 * dy0 + dz0 * dz0);
                const double r1 = rsqrt_nr(dx1 * dx1 + dy1 * dy1 + dz1 * dz1);
                const double dn0 = dx0 * P[3] + dy0 * P[4] + dz0 * P[5];
                const double dn1 = dx1 * P[3] + dy1 * P[4] + dz1 * P[5];
                sf0 += P[6] * r0;
                sd0 += P[7] * dn0 * (r0 * r0 * r0);
                sf1 += P[6] * r1;
                sd1 += P[7] * dn1 * (r1 * r1 * r1);
            }
        }
    }
    if (act0) {
        double* o = partial + ((int64_t)blockIdx.y * at.n + a0) * 2;
        o[0] = sf0;
        o[1] = sd0;
    }
    if (act1) {
        double* o = partial + ((int64_t)blockIdx.y * at.n + a1) * 2;
        o[0] = sf1;
        o[1] = sd1;
    }
}

// phi_coul(i) = sum_{j != i} q_j / r_ij  (divided by eps_in later)
__global__ void __launch_bounds__(256) k_coulomb(Atoms at, double* phic)
{
    __shared__ double sa[256 * 4];
    const int a = blockIdx.x * 256 + threadIdx.x;
    const bool act = a < at.n;
    double xi = 0, yi = 0, zi = 0;
    if (act) {
        xi = at.xyzr[4 * a];
        yi = at.xyzr[4 * a + 1];
        zi = at.xyzr[4 * a + 2];
    }
    double s = 0.0;
    for (int base = 0; base < at.n; base += 256) {
        const int j = base + threadIdx.x;
        __syncthreads();
        if (j < at.n) {
            sa[4 * threadIdx.x] = at.xyzr[4 * j];
            sa[4 * threadIdx.x + 1] = at.xyzr[4 * j + 1];
            sa[4 * threadIdx.x + 2] = at.xyzr[4 * j + 2];
            sa[4 * threadIdx.x + 3] = at.q[j];
        }
        __syncthreads();
        const int m = at.n - base < 256 ? at.n - base : 256;
        if (act)
            for (int u = 0; u < m; ++u) {
                if (base + u == a) continue;
                const double dx = sa[4 * u] - xi, dy = sa[4 * u + 1] - yi, dz = sa[4 * u + 2] - zi;
                s += sa[4 * u + 3] * rsqrt(dx * dx + dy * dy + dz * dz);
            }
    }
    if (act) phic[a] = s;
}

// single block of 1024: per-atom potentials and the energy sums, in fixed order
__global__ void __launch_bounds__(1024) k_energy_reduce(Atoms at, const double* partial, int nchunk,
                                                        const double* phic, double eps_in, double eps_out,
                                                        double lB, double* phi_reac, double* out,
                                                        const double* F, int64_t ncut, const double* wp)
{
    __shared__ double sh[32];
    const double fpi = 1.0 / (4.0 * kPi);
    double e_pol = 0.0, e_ion = 0.0, e_coul = 0.0, dummy = 0.0;
    for (int a = threadIdx.x; a < at.n; a += 1024) {
        double sf = 0.0, sd = 0.0;
        for (int c = 0; c < nchunk; ++c) {
            sf += partial[((int64_t)c * at.n + a) * 2];
            sd += partial[((int64_t)c * at.n + a) * 2 + 1];
        }
        const double ppol = (1.0 / eps_out - 1.0 / eps_in) * sf * fpi;
        const double pion = sd * fpi - sf * fpi / eps_out;
        const double q = at.q[a];
        e_pol += q * ppol;
        e_ion += q * pion;
        e_coul += q * phic[a] / eps_in;
        phi_reac[a] = lB * (ppol + pion);
    }
    block_sum2(e_pol, e_ion, sh, 16);
    block_sum2(e_coul, dummy, sh, 16);
    double fs = 0.0, ws = 0.0;
    for (int64_t c = threadIdx.x; c < ncut; c += 1024) {
        fs += F[c];
        ws += wp[c];
    }
    block_sum2(fs, ws, sh, 16);
    if (threadIdx.x == 0) {
        out[0] = 0.5 * lB * e_coul;
        out[1] = 0.5 * lB * e_pol;
        out[2] = 0.5 * lB * e_ion;
        out[3] = (1.0 / eps_out - 1.0 / eps_in) * fs * fpi;
        out[4] = ws;
    }
}

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

int nbody_chunks(int n_atoms, int64_t ncut)
{
    // enough blocks to fill 256 CUs several times, each chunk at least a few LDS tiles
    const int ab = (n_atoms + 511) / 512;   // blocks of k_nbody along the atoms
    int64_t want = (2048 + ab - 1) / ab;
    int64_t maxc = (ncut + 4 * NB_TILE - 1) / (4 * NB_TILE);
    if (want > maxc) want = maxc;
    if (want < 1) want = 1;
    if (want > 4096) want = 4096;
    return (int)want;
}

hipError_t launch_edge_fields(hipStream_t s, const Grid& g, double eps_in, double eps_out, int64_t ncut,
                              const int64_t* cutkey, const uint32_t* code, const double* alpha,
                              const double* kcut, const double* x, const double* gb, const double* wp,
                              double* F, double* phip, double* pts, const double* rp, const double* np)
{
    if (ncut == 0) return hipSuccess;
    k_edge_fields<<<nblk(ncut, 256), 256, 0, s>>>(g, eps_in, eps_out, ncut, cutkey, code, alpha, kcut, x, gb,
                                                   wp, F, phip, pts, rp, np);
    return hipGetLastError();
}

hipError_t launch_nbody(hipStream_t s, const Atoms& at, int64_t ncut, const double* pts, double* partial,
                        int nchunk)
{
    const int64_t len = (ncut + nchunk - 1) / nchunk;
    dim3 grid(nblk(at.n, 512), (unsigned)nchunk);
    k_nbody<<<grid, 256, 0, s>>>(at, ncut, pts, partial, len > 0 ? len : 1);
    return hipGetLastError();
}

hipError_t launch_coulomb(hipStream_t s, const Atoms& at, double* phic)
{
    k_coulomb<<<nblk(at.n, 256), 256, 0, s>>>(at, phic);
    return hipGetLastError();
}

hipError_t launch_energy_reduce(hipStream_t s, const Atoms& at, const double* partial, int nchunk,
                                const double* phic, double eps_in, double eps_out, double lB, double* phi_reac,
                                double* out, const double* F, int64_t ncut, const double* wp)
{
    k_energy_reduce<<<1, 1024, 0, s>>>(at, partial, nchunk, phic, eps_in, eps_out, lB, phi_reac, out, F, ncut,
                                       wp);
    return hipGetLastError();
}

}  // namespace pbk
