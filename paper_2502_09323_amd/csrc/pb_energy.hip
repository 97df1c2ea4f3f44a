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
// LDS in tiles, each thread owns a few atoms, and the cut list is split into chunks whose
// per-atom partials are summed in chunk order, so the result does not depend on timing.
#include "pb_internal.h"

#include <algorithm>
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

__global__ void __launch_bounds__(256) k_edge_fields(Grid g, Atoms at, double eps_in, double eps_out, int64_t ncut,
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
    double* o = pts + CUT_POINT_DOUBLES * c;
    // relative to the atoms' centre, as the N-body kernel takes the atoms
    const double px = rp[3 * c] - at.cx, py = rp[3 * c + 1] - at.cy, pz = rp[3 * c + 2] - at.cz;
    const double wphi = wp[c] * pp;
    const double ux = wphi * np[3 * c], uy = wphi * np[3 * c + 1], uz = wphi * np[3 * c + 2];
    o[0] = px;
    o[1] = py;
    o[2] = pz;
    o[3] = ux;
    o[4] = uy;
    o[5] = uz;
    o[6] = f;
    o[7] = fma(px, px, fma(py, py, pz * pz));
    o[8] = 2.0 * fma(px, ux, fma(py, uy, pz * uz));
    o[9] = 0.0;
}

// 1/sqrt(x) for the N-body sum: the hardware FP64 estimate y (relative error up to about
// 5.2e-8) and one Newton step y + y e / 2, e = 1 - x y^2.  The step leaves 3e^2/8, under 4e-15
// relative and of one sign, below the rounding of the read-back's sums over millions of cut
// points (about 1e-13 relative); four operations where rsqrt_fp64's series step takes five.
__device__ __forceinline__ double rsqrt_nb(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x, y * y, 1.0);
    return fma(0.5 * y, e, y);
}

constexpr int NB_ATOMS = 4;                       // atoms per thread
constexpr int NB_BLOCK_ATOMS = 256 * NB_ATOMS;    // atoms per block

// grid (ceil(n_atoms/NB_BLOCK_ATOMS), nchunk); thread t of block b owns the atoms
// b*NB_BLOCK_ATOMS + t + 256 k (k < NB_ATOMS), so that each cut point read from LDS serves
// NB_ATOMS pairs.  A cut point carries r_p, u_p = w_p phi_p n_p (the surface-potential weight
// folded into the normal), F_p, |r_p|^2 and 2 r_p.u_p, so that a pair needs no difference
// vector: with a = the atom centre,
//   |r_p - a|^2 = |r_p|^2 + |a|^2 - 2 a.r_p   and   2 (r_p - a).u_p = 2 r_p.u_p - 2 a.u_p,
// the first in one add and three fused multiply-adds, the second in three, with -2a and |a|^2
// held per atom.  Both r_p and a are taken relative to the centre of the atoms' bounding box
// (at.cx, at.cy, at.cz), so |r_p| and |a| are at most the molecule's half-diagonal plus an
// atom radius wherever the molecule sits.  The rounding error of r^2 is about
// (|r_p|^2 + |a|^2) eps: for a 65 A molecule (|r_p|, |a| < 115 A) below 3e-12 A^2, or 2e-12
// of the smallest squared distance (an atom radius squared, at least 1.44 A^2, as every cut
// point lies outside or on every ball).
// partial[(chunk*n + i)*2 + {0,1}] = {S_F, S_D} of atom i over the chunk.
__global__ void __launch_bounds__(256) k_nbody(Atoms at, int64_t ncut, const double* __restrict__ pts,
                                               double* __restrict__ partial, int64_t chunk_len)
{
    constexpr int PT = CUT_POINT_DOUBLES;
    __shared__ double sp[NB_TILE * PT];
    const int a0 = blockIdx.x * NB_BLOCK_ATOMS + threadIdx.x;
    double mx[NB_ATOMS], my[NB_ATOMS], mz[NB_ATOMS], aa[NB_ATOMS], sf[NB_ATOMS], sd[NB_ATOMS];
    double x0 = 0.0, y0 = 0.0, z0 = 0.0;
    if (a0 < at.n) {
        x0 = at.xyzr[4 * a0] - at.cx;
        y0 = at.xyzr[4 * a0 + 1] - at.cy;
        z0 = at.xyzr[4 * a0 + 2] - at.cz;
    }
#pragma unroll
    for (int k = 0; k < NB_ATOMS; ++k) {
        const int a = a0 + 256 * k;
        // an inactive slot evaluates the pairs of a far point, whose sums are discarded
        double x = x0 + 1e3 * k, y = y0, z = z0;
        if (k > 0 && a < at.n) {
            x = at.xyzr[4 * a] - at.cx;
            y = at.xyzr[4 * a + 1] - at.cy;
            z = at.xyzr[4 * a + 2] - at.cz;
        }
        mx[k] = -2.0 * x;
        my[k] = -2.0 * y;
        mz[k] = -2.0 * z;
        aa[k] = fma(x, x, fma(y, y, z * z));
        sf[k] = sd[k] = 0.0;
    }
    const int64_t p0 = (int64_t)blockIdx.y * chunk_len;
    int64_t p1 = p0 + chunk_len;
    if (p1 > ncut) p1 = ncut;
    for (int64_t base = p0; base < p1; base += NB_TILE) {
        const int m = (int)((p1 - base) < NB_TILE ? (p1 - base) : NB_TILE);
        __syncthreads();
        for (int t = threadIdx.x; t < m * PT; t += 256) sp[t] = pts[base * PT + t];
        __syncthreads();
        if (a0 < at.n) {
            for (int u = 0; u < m; ++u) {
                const double* P = sp + PT * u;
                const double px = P[0], py = P[1], pz = P[2], ux = P[3], uy = P[4], uz = P[5], f = P[6];
                const double pp = P[7], pu2 = P[8];
#pragma unroll
                for (int k = 0; k < NB_ATOMS; ++k) {
                    const double r2 = fma(mx[k], px, fma(my[k], py, fma(mz[k], pz, pp + aa[k])));
                    const double dn2 = fma(mx[k], ux, fma(my[k], uy, fma(mz[k], uz, pu2)));
                    const double r = rsqrt_nb(r2);
                    sf[k] = fma(f, r, sf[k]);
                    sd[k] = fma(dn2, (r * r) * r, sd[k]);
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < NB_ATOMS; ++k) {
        const int a = a0 + 256 * k;
        if (a < at.n) {
            double* o = partial + ((int64_t)blockIdx.y * at.n + a) * 2;
            o[0] = sf[k];
            o[1] = 0.5 * sd[k];
        }
    }
}

// phic[c*n + i] = sum over j != i in chunk c of q_j / r_ij  (divided by eps_in later); grid
// (ceil(n/256), nchunk), chunk c covering whole 256-atom tiles
__global__ void __launch_bounds__(256) k_coulomb(Atoms at, double* __restrict__ phic, int tiles_per_chunk)
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
    const int b0 = blockIdx.y * tiles_per_chunk * 256;
    int b1 = b0 + tiles_per_chunk * 256;
    if (b1 > at.n) b1 = at.n;
    for (int base = b0; base < b1; base += 256) {
        const int j = base + threadIdx.x;
        __syncthreads();
        if (j < at.n) {
            sa[4 * threadIdx.x] = at.xyzr[4 * j];
            sa[4 * threadIdx.x + 1] = at.xyzr[4 * j + 1];
            sa[4 * threadIdx.x + 2] = at.xyzr[4 * j + 2];
            sa[4 * threadIdx.x + 3] = at.q[j];
        }
        __syncthreads();
        const int m = b1 - base < 256 ? b1 - base : 256;
        if (act)
            for (int u = 0; u < m; ++u) {
                const double dx = sa[4 * u] - xi, dy = sa[4 * u + 1] - yi, dz = sa[4 * u + 2] - zi;
                const double t = sa[4 * u + 3] * rsqrt_fp64(fma(dx, dx, fma(dy, dy, dz * dz)));
                s += (base + u == a) ? 0.0 : t;   // the self term (not finite) is dropped by the select
            }
    }
    if (act) phic[(int64_t)blockIdx.y * at.n + a] = s;
}

constexpr int ER_BLOCKS = 256;   // most blocks of the energy reduction
constexpr int ER_FOLD = 16;      // chunk partials summed per group before the reduction

// out[(g*n + a)*2 + {0,1}] = the partials of atom a summed over chunks g*ER_FOLD ..
// g*ER_FOLD + ER_FOLD - 1 (those that exist), in chunk order; grid (ceil(n/256), groups)
__global__ void __launch_bounds__(256) k_chunk_fold(const double* __restrict__ partial, int nchunk, int n,
                                                    double* __restrict__ out)
{
    const int a = blockIdx.x * 256 + threadIdx.x;
    if (a >= n) return;
    const int c0 = blockIdx.y * ER_FOLD;
    const int c1 = c0 + ER_FOLD < nchunk ? c0 + ER_FOLD : nchunk;
    double sf = 0.0, sd = 0.0;
    for (int c = c0; c < c1; ++c) {
        sf += partial[((int64_t)c * n + a) * 2];
        sd += partial[((int64_t)c * n + a) * 2 + 1];
    }
    out[((int64_t)blockIdx.y * n + a) * 2] = sf;
    out[((int64_t)blockIdx.y * n + a) * 2 + 1] = sd;
}

// Energy reduction, first stage: each block takes the atoms and cut points b*256 + t +
// k*gridDim.x*256; an atom's potentials are its chunk partials summed in chunk order.
// part[5*b + {0..4}] = {sum q phi_pol, sum q phi_ion, sum q phi_coul, sum F, sum w} of block b.
__global__ void __launch_bounds__(256) k_energy_part(Atoms at, const double* __restrict__ partial, int nchunk,
                                                     const double* __restrict__ phic, int ncc, double eps_in,
                                                     double eps_out, double lB, double* __restrict__ phi_reac,
                                                     const double* __restrict__ F, int64_t ncut,
                                                     const double* __restrict__ wp, double* __restrict__ part)
{
    __shared__ double sh[32];
    const double fpi = 1.0 / (4.0 * kPi);
    double e_pol = 0.0, e_ion = 0.0, e_coul = 0.0, fs = 0.0, ws = 0.0, dummy = 0.0;
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t a = (int64_t)blockIdx.x * 256 + threadIdx.x; a < at.n; a += stride) {
        double sf = 0.0, sd = 0.0, pc = 0.0;
        for (int c = 0; c < nchunk; ++c) {
            sf += partial[((int64_t)c * at.n + a) * 2];
            sd += partial[((int64_t)c * at.n + a) * 2 + 1];
        }
        for (int c = 0; c < ncc; ++c) pc += phic[(int64_t)c * at.n + a];
        const double ppol = (1.0 / eps_out - 1.0 / eps_in) * sf * fpi;
        const double pion = sd * fpi - sf * fpi / eps_out;
        const double q = at.q[a];
        e_pol += q * ppol;
        e_ion += q * pion;
        e_coul += q * pc / eps_in;
        phi_reac[a] = lB * (ppol + pion);
    }
    for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < ncut; c += stride) {
        fs += F[c];
        ws += wp[c];
    }
    block_sum2(e_pol, e_ion, sh, 4);
    block_sum2(e_coul, fs, sh, 4);
    block_sum2(ws, dummy, sh, 4);
    if (threadIdx.x == 0) {
        double* o = part + 5 * blockIdx.x;
        o[0] = e_pol;
        o[1] = e_ion;
        o[2] = e_coul;
        o[3] = fs;
        o[4] = ws;
    }
}

// second stage, one block: the block sums in block order, and the energies
__global__ void __launch_bounds__(256) k_energy_final(const double* __restrict__ part, int nb, double eps_in,
                                                      double eps_out, double lB, double* __restrict__ out)
{
    __shared__ double sh[32];
    const double fpi = 1.0 / (4.0 * kPi);
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, dummy = 0.0;
    if ((int)threadIdx.x < nb)
        for (int k = 0; k < 5; ++k) v[k] = part[5 * threadIdx.x + k];
    block_sum2(v[0], v[1], sh, 4);
    block_sum2(v[2], v[3], sh, 4);
    block_sum2(v[4], dummy, sh, 4);
    if (threadIdx.x == 0) {
        out[0] = 0.5 * lB * v[2];
        out[1] = 0.5 * lB * v[0];
        out[2] = 0.5 * lB * v[1];
        out[3] = (1.0 / eps_out - 1.0 / eps_in) * v[3] * fpi;
        out[4] = v[4];
    }
}

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

// blocks of k_nbody resident on the device at once: its compute units times the blocks one
// compute unit holds (queried once, on the device current at the first call)
static int nbody_slots()
{
    static const int slots = [] {
        int dev = 0, cus = 0, per = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_nbody, 256, 0) != hipSuccess || per <= 0) per = 4;
        return cus * per;
    }();
    return slots;
}

int nbody_chunks(int n_atoms, int64_t ncut)
{
    // The blocks all carry the same work, so they run in rounds of nbody_slots() blocks; a
    // last round of a few blocks would leave most of the device idle for a whole block's run.
    // The grid is therefore the largest one of at most NB_ROUNDS rounds whose block count
    // falls just short of a whole number of rounds, each chunk at least 64 cut points.
    constexpr int NB_ROUNDS = 8;
    const int64_t ab = (n_atoms + NB_BLOCK_ATOMS - 1) / NB_BLOCK_ATOMS;   // blocks along the atoms
    const int64_t slots = nbody_slots();
    const int64_t maxc = std::max<int64_t>(1, (ncut + 63) / 64);
    for (int k = NB_ROUNDS; k >= 1; --k) {
        const int64_t c = k * slots / ab;
        if (c >= 1 && c <= maxc) return (int)c;
    }
    // fewer cut points than one round needs (one partial round), or more atom blocks than
    // NB_ROUNDS rounds hold (one chunk)
    return NB_ROUNDS * slots < ab ? 1 : (int)maxc;
}

hipError_t launch_edge_fields(hipStream_t s, const Grid& g, const Atoms& at, double eps_in, double eps_out, int64_t ncut,
                              const int64_t* cutkey, const uint32_t* code, const double* alpha,
                              const double* kcut, const double* x, const double* gb, const double* wp,
                              double* F, double* phip, double* pts, const double* rp, const double* np)
{
    if (ncut == 0) return hipSuccess;
    k_edge_fields<<<nblk(ncut, 256), 256, 0, s>>>(g, at, eps_in, eps_out, ncut, cutkey, code, alpha, kcut, x, gb,
                                                   wp, F, phip, pts, rp, np);
    return hipGetLastError();
}

hipError_t launch_nbody(hipStream_t s, const Atoms& at, int64_t ncut, const double* pts, double* partial,
                        int nchunk)
{
    const int64_t len = (ncut + nchunk - 1) / nchunk;
    dim3 grid(nblk(at.n, NB_BLOCK_ATOMS), (unsigned)nchunk);
    k_nbody<<<grid, 256, 0, s>>>(at, ncut, pts, partial, len > 0 ? len : 1);
    return hipGetLastError();
}

int coulomb_chunks(int n_atoms)
{
    const int ab = (n_atoms + 255) / 256, tiles = ab;
    int want = (2048 + ab - 1) / ab;
    if (want > tiles) want = tiles;
    if (want < 1) want = 1;
    return want;
}

hipError_t launch_coulomb(hipStream_t s, const Atoms& at, double* phic, int ncc)
{
    const int tiles = (at.n + 255) / 256;
    const int tpc = (tiles + ncc - 1) / ncc;
    k_coulomb<<<dim3(nblk(at.n, 256), (unsigned)ncc), 256, 0, s>>>(at, phic, tpc > 0 ? tpc : 1);
    return hipGetLastError();
}

int fold_chunks(int nchunk) { return nchunk > ER_FOLD ? (nchunk + ER_FOLD - 1) / ER_FOLD : 0; }

int64_t energy_partial_doubles(int n_atoms, int nchunk)
{
    return 2 * (int64_t)std::max(n_atoms, 1) * (nchunk + fold_chunks(nchunk));
}

hipError_t launch_energy_reduce(hipStream_t s, const Atoms& at, double* partial, int nchunk,
                                const double* phic, int ncc, double eps_in, double eps_out, double lB,
                                double* phi_reac, double* out, const double* F, int64_t ncut, const double* wp)
{
    const int nf = fold_chunks(nchunk);
    if (nf > 0 && at.n > 0) {
        // many chunks: sum them in groups first, so the per-atom loop below stays short
        double* folded = partial + 2 * (int64_t)at.n * nchunk;
        k_chunk_fold<<<dim3(nblk(at.n, 256), (unsigned)nf), 256, 0, s>>>(partial, nchunk, at.n, folded);
        partial = folded;
        nchunk = nf;
    }
    int64_t need = std::max<int64_t>(at.n, ncut);
    int nb = (int)std::min<int64_t>(ER_BLOCKS, std::max<int64_t>(1, (need + 255) / 256));
    k_energy_part<<<nb, 256, 0, s>>>(at, partial, nchunk, phic, ncc, eps_in, eps_out, lB, phi_reac, F, ncut, wp,
                                     out + 16);
    k_energy_final<<<1, 256, 0, s>>>(out + 16, nb, eps_in, eps_out, lB, out);
    return hipGetLastError();
}

}  // namespace pbk
