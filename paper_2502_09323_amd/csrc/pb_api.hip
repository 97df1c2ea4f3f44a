// pb_api.hip -- the C ABI of libpb: validation, device memory through the caller's
// allocator, and the order of kernel launches for build, solve and energy.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "pb_host.h"
#include "pb_internal.h"

using namespace pbk;

namespace {

thread_local std::string g_err;

}  // namespace

int pbi_fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

namespace {

#define fail pbi_fail

#define HIPCHK(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(PB_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),   \
                        __FILE__, __LINE__);                                                \
    } while (0)

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// physical constants (CODATA 2018) -> Bjerrum length (Angstrom) and kD^2 (1/Angstrom^2)
void reduced_constants(double T, double I, double eps_out, double* lB, double* kD2)
{
    const double e = 1.602176634e-19, kB = 1.380649e-23, NA = 6.02214076e23, eps0 = 8.8541878128e-12;
    const double pi = 3.14159265358979323846;
    const double lb_m = e * e / (4.0 * pi * eps0 * kB * T);
    *lB = lb_m * 1e10;
    // 1:1 salt: kD^2 = e^2 sum z^2 rho /(eps0 eps_out kB T) = 8 pi lB I NA 1e3 / eps_out  [1/m^2]
    *kD2 = 8.0 * pi * lb_m * I * NA * 1e3 / eps_out * 1e-20;
}

}  // namespace

namespace {

bool finite(double v) { return std::isfinite(v); }

int validate(const pb_params* p, int64_t na, const double* xyz, const double* rad, const double* chg)
{
    if (!p) return fail(PB_EINVAL, "params is NULL");
    if (!finite(p->eps_in) || !finite(p->eps_out) || p->eps_in <= 0 || p->eps_out <= 0)
        return fail(PB_EINVAL, "permittivities must be finite and > 0");
    if (!finite(p->ionic_strength_M) || p->ionic_strength_M < 0)
        return fail(PB_EINVAL, "ionic strength must be finite and >= 0");
    if (!finite(p->temperature_K) || p->temperature_K <= 0) return fail(PB_EINVAL, "temperature must be > 0");
    if (!finite(p->h) || p->h <= 0) return fail(PB_EINVAL, "grid spacing must be finite and > 0");
    for (int d = 0; d < 3; ++d) {
        if (p->n[d] < 3) return fail(PB_EINVAL, "n[%d] = %d < 3", d, p->n[d]);
        if (p->n[d] > 4096) return fail(PB_EINVAL, "n[%d] = %d > 4096", d, p->n[d]);
        if (!finite(p->origin[d])) return fail(PB_EINVAL, "origin must be finite");
    }
    {
        // the iteration kernel addresses FP64 vectors with 32-bit byte offsets
        const int64_t S = row_stride(p->n[2]);
        if ((int64_t)p->n[0] * p->n[1] * S >= ((int64_t)1 << 29))
            return fail(PB_EINVAL, "grid of %d x %d x %d nodes exceeds 2^29 stored nodes", p->n[0], p->n[1], p->n[2]);
    }
    if (p->bc != PB_BC_ZERO && p->bc != PB_BC_DH && p->bc != PB_BC_USER) return fail(PB_EINVAL, "bad bc");
    if (p->bc == PB_BC_USER && !p->bc_values) return fail(PB_EINVAL, "PB_BC_USER needs bc_values");
    if (p->precision != PB_FP64 && p->precision != PB_MIXED) return fail(PB_EINVAL, "bad precision");
    if (!finite(p->rtol) || p->rtol <= 0 || p->rtol >= 1) return fail(PB_EINVAL, "rtol must be in (0, 1)");
    if (p->precision == PB_MIXED && (!finite(p->inner_rtol) || p->inner_rtol <= 0 || p->inner_rtol >= 1))
        return fail(PB_EINVAL, "inner_rtol must be in (0, 1)");
    if (p->max_iter <= 0) return fail(PB_EINVAL, "max_iter must be > 0");
    if (p->tile_planes != 0 && (p->tile_planes < 4 || p->tile_planes > 128 || p->tile_planes % 4))
        return fail(PB_EINVAL, "tile_planes must be 0 or a multiple of 4 in [4, 128]");
    if (p->refine < 0 || p->refine > 2) return fail(PB_EINVAL, "refine must be 0, 1 or 2");
    if (p->refine) {
        if (!finite(p->refine_shell_A) || p->refine_shell_A < 0) return fail(PB_EINVAL, "refine_shell_A must be >= 0");
        if (p->refine_brick < 1 || p->refine_brick > 64) return fail(PB_EINVAL, "refine_brick must be in [1, 64]");
        if (na <= 0) return fail(PB_EINVAL, "refinement needs atoms");
    }
    if (p->precond != PB_PRECOND_JACOBI && p->precond != PB_PRECOND_MG)
        return fail(PB_EINVAL, "precond must be PB_PRECOND_JACOBI or PB_PRECOND_MG");
    if (p->precond == PB_PRECOND_MG) {
        if (p->mg_smooth < 0 || p->mg_smooth > 8) return fail(PB_EINVAL, "mg_smooth must be in [0, 8]");
        if (p->mg_coarse_sweeps < 0 || p->mg_coarse_sweeps > 64)
            return fail(PB_EINVAL, "mg_coarse_sweeps must be in [0, 64]");
        if (p->mg_levels < 0 || p->mg_levels > 12) return fail(PB_EINVAL, "mg_levels must be in [0, 12]");
    }
    if (na < 0 || na > (int64_t)1 << 26) return fail(PB_EINVAL, "bad atom count");
    if (na > 0 && (!xyz || !rad || !chg)) return fail(PB_EINVAL, "atom arrays are NULL");
    for (int64_t a = 0; a < na; ++a) {
        if (!finite(rad[a]) || rad[a] < 1e-6 || !finite(chg[a])) return fail(PB_EINVAL, "atom %lld: bad radius/charge", (long long)a);
        for (int d = 0; d < 3; ++d) {
            double c = xyz[3 * a + d];
            if (!finite(c)) return fail(PB_EINVAL, "atom %lld: non-finite coordinate", (long long)a);
            double lo = p->origin[d] + p->h, hi = p->origin[d] + p->h * (double)(p->n[d] - 2);
            if (!(c - rad[a] > lo && c + rad[a] < hi))
                return fail(PB_EINVAL, "atom %lld: ball not strictly inside the box interior on axis %d",
                            (long long)a, d);
        }
    }
    return PB_OK;
}

template <typename T>
T* dalloc(pb_problem* pb, size_t count, int* rc)
{
    void* p = pb->mem.get(sizeof(T) * count);
    if (!p) *rc = fail(PB_ENOMEM, "device allocation of %zu bytes failed", sizeof(T) * count);
    return (T*)p;
}

// Pipelined CG: launch chunks of iterations (for the mixed form each chunk ends with the
// reliable-update kernels, which do nothing unless an update is due) and poll the device
// state of the previous chunk while the next one runs.
template <typename T>
int run_cg(pb_problem* pb, const CGBufs<T>& B, int max_iter, bool mixed, CGState* out)
{
    pb_ctx* ctx = pb->ctx;
    hipStream_t s = ctx->stream;
    const int M = 16;
    int launched = 0, c = 0;
    const bool prof = ctx->profile != 0;
    std::vector<hipEvent_t> evs;
    std::vector<int> ev_it;
    auto enqueue = [&](int slot) -> int {
        int n = std::min(M, max_iter - launched);
        for (int t = 0; t < n; ++t) {
            const int it = launched + t;
            const bool sample = prof && (it % 8 == 0) && evs.size() < 3 * 256;
            hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr;
            if (sample) {
                HIPCHK(hipEventCreate(&e0));
                HIPCHK(hipEventCreate(&e1));
                HIPCHK(hipEventCreate(&e2));
                HIPCHK(hipEventRecord(e0, s));
            }
            HIPCHK(launch_cg_iter<T>(s, pb->g, pb->ts, B, pb->cf));
            if (sample) HIPCHK(hipEventRecord(e1, s));
            HIPCHK(launch_cg_tail(s, B.part, B.nb, B.st));
            if (sample) {
                HIPCHK(hipEventRecord(e2, s));
                evs.push_back(e0);
                evs.push_back(e1);
                evs.push_back(e2);
                ev_it.push_back(it);
            }
        }
        if (mixed) {
            HIPCHK(launch_ru_add(s, pb->g, B.st, pb->x, pb->d32, pb->p32, 0));
            HIPCHK(launch_ru_residual(s, pb->g, pb->code, pb->ck64, pb->ck32, pb->cf, pb->rhs, pb->x, pb->z32,
                                      pb->part_res, B.st));
            HIPCHK(launch_ru_fin(s, B.st, pb->part_res, pb->nbres, 0, 0.0, 0.0));
        }
        launched += n;
        HIPCHK(hipMemcpyAsync(&ctx->host_state[slot], B.st, sizeof(CGState), hipMemcpyDeviceToHost, s));
        HIPCHK(hipEventRecord(ctx->ev[slot], s));
        return PB_OK;
    };
    int rc = enqueue(0);
    if (rc) return rc;
    for (;;) {
        const bool more = launched < max_iter;
        if (more && (rc = enqueue((c + 1) & 1))) return rc;
        HIPCHK(hipEventSynchronize(ctx->ev[c & 1]));
        const CGState snap = ctx->host_state[c & 1];
        if ((snap.status != 0 && snap.status != 3) || !more) break;
        ++c;
    }
    if (mixed) {
        // a final update folds in the last correction when the iteration did not converge
        HIPCHK(launch_ru_add(s, pb->g, B.st, pb->x, pb->d32, pb->p32, 1));
        HIPCHK(launch_ru_residual(s, pb->g, pb->code, pb->ck64, pb->ck32, pb->cf, pb->rhs, pb->x, pb->z32,
                                  pb->part_res, B.st));
        HIPCHK(launch_ru_fin(s, B.st, pb->part_res, pb->nbres, 0, 0.0, 0.0));
    }
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipMemcpy(out, B.st, sizeof(CGState), hipMemcpyDeviceToHost));
    if (prof) {
        const int done = out->status == 1 ? out->iters : out->iter_count;
        double ts = 0, tu = 0;
        int n = 0;
        for (size_t k = 0; k < ev_it.size(); ++k) {
            if (ev_it[k] < done) {
                float a = 0, b = 0;
                HIPCHK(hipEventElapsedTime(&a, evs[3 * k], evs[3 * k + 1]));
                HIPCHK(hipEventElapsedTime(&b, evs[3 * k + 1], evs[3 * k + 2]));
                ts += a;
                tu += b;
                ++n;
            }
        }
        for (auto e : evs) (void)hipEventDestroy(e);
        pb->prof_stencil_ms += ts;
        pb->prof_update_ms += tu;
        pb->prof_n += n;
    }
    return PB_OK;
}

int ensure_cg64(pb_problem* pb)
{
    int rc = PB_OK;
    if (pb->z64[0]) return PB_OK;
    const size_t N = (size_t)pb->g.N;
    for (int k = 0; k < 2 && !rc; ++k) {
        pb->z64[k] = dalloc<double>(pb, N, &rc);
        if (!rc) pb->w64[k] = dalloc<double>(pb, N, &rc);
        if (!rc) pb->p64[k] = dalloc<double>(pb, N, &rc);
    }
    return rc;
}

int ensure_cg32(pb_problem* pb)
{
    int rc = PB_OK;
    if (pb->d32) return PB_OK;
    const size_t N = (size_t)pb->g.N;
    pb->d32 = dalloc<float>(pb, N, &rc);
    for (int k = 0; k < 2 && !rc; ++k) {
        pb->z32[k] = dalloc<float>(pb, N, &rc);
        if (!rc) pb->w32[k] = dalloc<float>(pb, N, &rc);
        if (!rc) pb->p32[k] = dalloc<float>(pb, N, &rc);
    }
    return rc;
}

template <typename T>
CGBufs<T> bufs(pb_problem* pb);

template <>
CGBufs<double> bufs<double>(pb_problem* pb)
{
    CGBufs<double> B;
    B.x = pb->x;
    for (int k = 0; k < 2; ++k) {
        B.z[k] = pb->z64[k];
        B.w[k] = pb->w64[k];
        B.p[k] = pb->p64[k];
    }
    B.ck = pb->ck64;
    B.code = pb->code;
    B.part = pb->part;
    B.st = pb->st;
    B.nb = pb->nb;
    return B;
}

template <>
CGBufs<float> bufs<float>(pb_problem* pb)
{
    CGBufs<float> B;
    B.x = pb->d32;
    for (int k = 0; k < 2; ++k) {
        B.z[k] = pb->z32[k];
        B.w[k] = pb->w32[k];
        B.p[k] = pb->p32[k];
    }
    B.ck = pb->ck32;
    B.code = pb->code;
    B.part = pb->part;
    B.st = pb->st;
    B.nb = pb->nb;
    return B;
}

}  // namespace

int pbi_mixed_begin(pb_problem* pb)
{
    int rc = ensure_cg32(pb);
    if (rc) return rc;
    hipStream_t s = pb->ctx->stream;
    const size_t N = (size_t)pb->g.N;
    const pb_params& P = pb->prm;
    HIPCHK(launch_fill(s, pb->x, sizeof(double) * N));
    HIPCHK(launch_fill(s, pb->d32, sizeof(float) * N));
    for (int k = 0; k < 2; ++k) {
        HIPCHK(launch_fill(s, pb->z32[k], sizeof(float) * N));
        HIPCHK(launch_fill(s, pb->w32[k], sizeof(float) * N));
        HIPCHK(launch_fill(s, pb->p32[k], sizeof(float) * N));
    }
    // first "update": z32 = D^-1 (b - A*0), the norms and the mixed iteration state
    HIPCHK(launch_ru_begin(s, pb->st));
    HIPCHK(launch_ru_residual(s, pb->g, pb->code, pb->ck64, pb->ck32, pb->cf, pb->rhs, pb->x, pb->z32, pb->part_res,
                              pb->st));
    HIPCHK(launch_ru_fin(s, pb->st, pb->part_res, pb->nbres, 1, P.rtol * P.rtol, P.inner_rtol * P.inner_rtol));
    return PB_OK;
}

// energy read-back: kernels and the read-back of the sums (and, with finish_mixed, the final
// reliable update and the CG state) behind pb->ev; pbi_energy_end collects after the event
int pbi_energy_begin(pb_problem* pb, int finish_mixed)
{
    hipStream_t s = pb->ctx->stream;
    int rc = PB_OK;
    const size_t nc1 = (size_t)std::max<int64_t>(pb->ncut, 1), na1 = (size_t)std::max<int64_t>(pb->na, 1);
    if (!pb->F) {
        pb->F = dalloc<double>(pb, nc1, &rc);
        if (!rc) pb->phip = dalloc<double>(pb, nc1, &rc);
        if (!rc) pb->pts = dalloc<double>(pb, CUT_POINT_DOUBLES * nc1, &rc);
        if (rc) return rc;
    }
    if (!pb->hout) {
        pb->hout = (double*)pb->ctx->pinned.get(16 * sizeof(double) + sizeof(CGState), &pb->hout_cap);
        if (!pb->hout) return fail(PB_EDEVICE, "pinned host allocation failed");
    }
    if (!pb->ev) HIPCHK(hipEventCreateWithFlags(&pb->ev, hipEventDisableTiming));
    pb->e_nchunk = nbody_chunks((int)std::max<int64_t>(pb->na, 1), pb->ncut);
    pb->e_tmp[0] = dalloc<double>(pb, (size_t)energy_partial_doubles((int)na1, pb->e_nchunk), &rc);   // partial sums
    const int ncc = coulomb_chunks((int)std::max<int64_t>(pb->na, 1));
    if (!rc) pb->e_tmp[1] = dalloc<double>(pb, na1 * (size_t)ncc, &rc);        // Coulomb potentials
    if (!rc) pb->e_tmp[2] = dalloc<double>(pb, na1, &rc);                      // reaction potentials
    if (!rc) pb->e_tmp[3] = dalloc<double>(pb, ENERGY_OUT_DOUBLES, &rc);       // energy sums
    if (rc) return rc;
    if (finish_mixed && pb->mg) {
        if ((rc = pbi_mg_finish(pb, s))) return rc;
    } else if (finish_mixed) {
        HIPCHK(launch_ru_add(s, pb->g, pb->st, pb->x, pb->d32, pb->p32, 1));
        HIPCHK(launch_ru_residual(s, pb->g, pb->code, pb->ck64, pb->ck32, pb->cf, pb->rhs, pb->x, pb->z32,
                                  pb->part_res, pb->st));
        HIPCHK(launch_ru_fin(s, pb->st, pb->part_res, pb->nbres, 0, 0.0, 0.0));
    }
    const Atoms at = pbi_atoms(pb);
    HIPCHK(launch_fill(s, pb->e_tmp[3], 16 * sizeof(double)));
    HIPCHK(launch_edge_fields(s, pb->g, at, pb->prm.eps_in, pb->prm.eps_out, pb->ncut, pb->cutkey, pb->code, pb->alpha,
                              pb->kcut, pb->x, pb->gb, pb->wp, pb->F, pb->phip, pb->pts, pb->rp, pb->np));
    pb->prof_nbody_ms = pb->prof_nbody_pairs = 0;
    pb->nb_timed = pb->ctx->profile && pb->na > 0 && pb->ncut > 0;
    if (pb->nb_timed && !pb->nb_ev[0])
        for (int e = 0; e < 2; ++e) HIPCHK(hipEventCreateWithFlags(&pb->nb_ev[e], hipEventDisableSystemFence));
    if (pb->na > 0) {
        if (pb->ncut > 0) {
            if (pb->nb_timed) HIPCHK(hipEventRecord(pb->nb_ev[0], s));
            HIPCHK(launch_nbody(s, at, pb->ncut, pb->pts, pb->e_tmp[0], pb->e_nchunk));
            if (pb->nb_timed) HIPCHK(hipEventRecord(pb->nb_ev[1], s));
        } else
            HIPCHK(launch_fill(s, pb->e_tmp[0], sizeof(double) * 2 * na1 * (size_t)pb->e_nchunk));
        HIPCHK(launch_coulomb(s, at, pb->e_tmp[1], ncc));
        HIPCHK(launch_energy_reduce(s, at, pb->e_tmp[0], pb->e_nchunk, pb->e_tmp[1], ncc, pb->prm.eps_in,
                                    pb->prm.eps_out, pb->lB, pb->e_tmp[2], pb->e_tmp[3], pb->F, pb->ncut, pb->wp));
    }
    HIPCHK(hipMemcpyAsync(pb->hout, pb->e_tmp[3], 16 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(pb->hout + 16, pb->st, sizeof(CGState), hipMemcpyDeviceToHost, s));
    HIPCHK(hipEventRecord(pb->ev, s));
    return PB_OK;
}

namespace {

size_t rounded(size_t n) { return n == 0 ? 256 : (n + 255) & ~(size_t)255; }   // as DevAlloc::get

// the energy read-back's buffers: F, phi_p and the N-body cut points (kept with the problem
// once made), then the partial sums, Coulomb potentials, reaction potentials and sums
size_t energy_bytes(int64_t na, int64_t ncut, bool with_cut_arrays)
{
    const size_t nc1 = (size_t)std::max<int64_t>(ncut, 1), na1 = (size_t)std::max<int64_t>(na, 1);
    size_t b = 0;
    if (with_cut_arrays) b += 2 * rounded(8 * nc1) + rounded(8 * (size_t)CUT_POINT_DOUBLES * nc1);
    const int nchunk = nbody_chunks((int)na1, ncut);
    const int ncc = coulomb_chunks((int)na1);
    b += rounded(8 * (size_t)energy_partial_doubles((int)na1, nchunk)) + rounded(8 * na1 * (size_t)ncc) +
         rounded(8 * na1) + rounded(8 * (size_t)ENERGY_OUT_DOUBLES);
    return b;
}

}  // namespace

size_t pbi_energy_bytes(const pb_problem* pb) { return energy_bytes(pb->na, pb->ncut, pb->F == nullptr); }

size_t pbi_request_bytes(const pb_params& p, int64_t na, const double* radius, int64_t ncut)
{
    const int64_t N = (int64_t)p.n[0] * p.n[1] * row_stride(p.n[2]);
    if (ncut < 0) {
        // before the build counts them: a lattice line along one axis meets a ball of radius R
        // at most twice and at most pi (R + h)^2 / h^2 such lines pass through it, so the cut
        // edges are fewer than 6 pi (R + h)^2 / h^2 per atom; overlapping balls hide most of
        // that (about a seventh at 0.5 A on the synthetic molecules), and a third of it is taken
        double e = 0.0;
        for (int64_t a = 0; a < na; ++a) {
            const double r = radius[a] + p.h;
            e += 2.0 * 3.14159265358979323846 * r * r / (p.h * p.h);
        }
        ncut = std::min<int64_t>((int64_t)e, 3 * N);
    }
    // per node: code, b, box values and the FP64 solution (28 B), the build's classes (4 B,
    // until the build ends), and the solver: six FP32 CG vectors and the correction (28 B), or
    // for the multigrid form eight FP32 vectors and the codes of level 0 in the red-black
    // layout (36 B, up to 40 B with its segment padding) and the coarser levels (64 B per
    // stored node in FP64 and FP32 copies; with the z-row padding of small levels they hold up
    // to a quarter of level 0's stored nodes)
    const size_t per_node = p.precond == PB_PRECOND_MG ? 28 + 4 + 40 + 16 : 28 + 4 + 28;
    // per cut edge: key, alpha, K, crossing point, normal, owner, area weight (84 B) and at
    // most one slot of the compact coefficient tables (40 B)
    const size_t per_cut = 124;
    // per atom: coordinates and charge (40 B); the cell list's ids, centres and radii in its
    // order, and deposition cells with charges (100 B)
    const size_t per_atom = 140;
    // the Debye-Hueckel partial sums of the build (at most kDhMaxRanges per box node)
    const int64_t nbox = 2 * ((int64_t)p.n[1] * p.n[2] + (int64_t)(p.n[0] - 2) * p.n[2] +
                              (int64_t)(p.n[0] - 2) * (p.n[1] - 2));
    const size_t dh = p.bc == PB_BC_DH ? (size_t)nbox * kDhMaxRanges * sizeof(double) : 0;
    return (size_t)N * per_node + (size_t)std::max<int64_t>(ncut, 1) * per_cut + (size_t)std::max<int64_t>(na, 1) * per_atom +
           energy_bytes(na, ncut, true) + dh + ((size_t)1 << 20);
}

int pbi_energy_end(pb_problem* pb, pb_energy_out* out, pb_solve_stats* stats)
{
    if (pb->nb_timed) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, pb->nb_ev[0], pb->nb_ev[1]) == hipSuccess) {
            pb->prof_nbody_ms = ms;
            pb->prof_nbody_pairs = (double)pb->na * (double)pb->ncut;
        }
        pb->nb_timed = false;
    }
    for (int t = 0; t < 4; ++t)
        if (pb->e_tmp[t]) {
            pb->mem.put(pb->e_tmp[t]);
            pb->e_tmp[t] = nullptr;
        }
    const double* h = pb->hout;
    memset(out, 0, sizeof *out);
    out->e_coul = h[0];
    out->e_pol = h[1];
    out->e_ion = h[2];
    out->e_solv = h[1] + h[2];
    out->e_total = h[0] + h[1] + h[2];
    out->q_pol_total = h[3];
    out->area_total = h[4];
    out->n_cut = pb->ncut;
    if (stats) {
        CGState st;
        memcpy(&st, h + 16, sizeof st);
        const pb_params& P = pb->prm;
        memset(stats, 0, sizeof *stats);
        stats->iters = st.status == 1 ? st.iters : st.iter_count;
        stats->outer_iters = st.n_ru;
        const double bn2 = P.rtol > 0 ? st.goal64 / (P.rtol * P.rtol) : 0.0;
        stats->relres = bn2 > 0 ? std::sqrt(st.rr64 / bn2) : 0.0;
        stats->status = st.status == 1 ? PB_OK : st.status == 2 ? PB_EBREAKDOWN : PB_ENOCONV;
    }
    return PB_OK;
}

ProbDev<float> pbi_probdev(pb_problem* pb)
{
    ProbDev<float> d;
    d.g = pb->g;
    d.ts = pb->ts;
    d.cf = pb->cf;
    d.B = bufs<float>(pb);
    d.x64 = pb->x;
    d.rhs = pb->rhs;
    d.ck64 = pb->ck64;
    d.part3 = pb->part_res;
    d.nbres = pb->nbres;
    d.nadd = add_blocks(pb->g);
    return d;
}

extern "C" {

const char* pb_last_error(void) { return g_err.c_str(); }

int pb_ctx_create(int device, void* hip_stream, pb_alloc_fn alloc, pb_free_fn free_fn, void* user,
                  size_t hbm_budget_bytes, pb_ctx** out)
{
    if (!out) return fail(PB_EINVAL, "out is NULL");
    *out = nullptr;
    if (!alloc || !free_fn) return fail(PB_EINVAL, "allocator callbacks are required");
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(PB_EINVAL, "device %d out of range (%d devices)", device, ndev);
    HIPCHK(hipSetDevice(device));
    {
        // the allocation-free energy read-back's scratch array: its address on this device
        const int rc = pbi_scratch_setup(device);
        if (rc) return rc;
    }
    pb_ctx* c = new pb_ctx();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->alloc = alloc;
    c->free_fn = free_fn;
    c->user = user;
    c->budget = hbm_budget_bytes;
    c->profile = 0;
    if (hipHostMalloc((void**)&c->host_state, 2 * sizeof(CGState), hipHostMallocDefault) != hipSuccess) {
        delete c;
        return fail(PB_EDEVICE, "hipHostMalloc failed");
    }
    for (int k = 0; k < 2; ++k)
        if (hipEventCreateWithFlags(&c->ev[k], hipEventDisableTiming) != hipSuccess) {
            delete c;
            return fail(PB_EDEVICE, "hipEventCreate failed");
        }
    *out = c;
    return PB_OK;
}

void pb_ctx_destroy(pb_ctx* c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (int k = 0; k < 2; ++k) (void)hipEventDestroy(c->ev[k]);
    (void)hipHostFree(c->host_state);
    c->pinned.release();
    delete c;
}

int pb_ctx_set_profiling(pb_ctx* c, int on)
{
    if (!c) return fail(PB_EINVAL, "ctx is NULL");
    c->profile = on;
    return PB_OK;
}

}  // extern "C"

// ---- coefficient build in three asynchronous phases ----------------------------------------
// begin:    atoms to the device, cell list, classification, counting of the cut edges; the
//           two counts come back through pinned memory behind an event
// continue: (counts known) allocation and the rest of the build, behind an event
// end:      release of the build temporaries
// pb_build_coeffs runs the three with waits in between; the serving loop polls the events.

namespace {

void release_tmp(pb_problem* pb)
{
    BuildTmp* t = pb->bt;
    if (!t) return;
    for (void* d : {(void*)t->bcnt, (void*)t->bstart, (void*)t->bcur, (void*)t->bids, (void*)t->bxyzr,
                    (void*)t->cls, (void*)t->bslots, (void*)t->bcuts, (void*)t->tot, (void*)t->full,
                    (void*)t->acell, (void*)t->dhpart})
        if (d) pb->mem.put(d);
    if (t->hpin) pb->ctx->pinned.put(t->hpin, t->hpin_cap);   // the build's copies have completed
    delete t;
    pb->bt = nullptr;
}

}  // namespace

void pbi_problem_destroy(pb_problem* pb, bool sync)
{
    if (!pb) return;
    (void)hipSetDevice(pb->ctx->device);
    if (sync) (void)hipStreamSynchronize(pb->ctx->stream);
    release_tmp(pb);
    if (pb->ref) {
        pbi_problem_destroy(pb->ref->fine, false);
        delete pb->ref;
        pb->ref = nullptr;
    }
    delete pb->mg;   // its arrays are held by pb->mem
    pb->mg = nullptr;
    if (pb->hout) pb->ctx->pinned.put(pb->hout, pb->hout_cap);   // no read-back is pending
    if (pb->ev) (void)hipEventDestroy(pb->ev);
    for (int e = 0; e < 2; ++e)
        if (pb->nb_ev[e]) (void)hipEventDestroy(pb->nb_ev[e]);
    pb->mem.release();
    delete pb;
}

int pbi_event_done(pb_problem* pb)
{
    const hipError_t e = hipEventQuery(pb->ev);
    if (e == hipSuccess) return 1;
    if (e == hipErrorNotReady) return 0;
    return fail(PB_EDEVICE, "hipEventQuery: %s", hipGetErrorString(e));
}

namespace {
int build_begin(pb_ctx* ctx, const pb_params* prm, int64_t na, const double* xyz, const double* rad,
                const double* chg, const int* off, pb_problem** out);
}

int pbi_build_begin(pb_ctx* ctx, const pb_params* prm, int64_t na, const double* xyz, const double* rad,
                    const double* chg, pb_problem** out)
{
    return build_begin(ctx, prm, na, xyz, rad, chg, nullptr, out);
}

int pbi_build_begin_sub(pb_ctx* ctx, const pb_params* prm, int64_t na, const double* xyz, const double* rad,
                        const double* chg, const int* off, pb_problem** out)
{
    return build_begin(ctx, prm, na, xyz, rad, chg, off, out);
}

namespace {
int build_begin(pb_ctx* ctx, const pb_params* prm, int64_t na, const double* xyz, const double* rad,
                const double* chg, const int* off, pb_problem** out)
{
    if (!ctx || !out) return fail(PB_EINVAL, "ctx/out is NULL");
    *out = nullptr;
    int rc;
    if (off) {
        // a sub-lattice: the atoms must lie inside it, whose first node sits at origin + h*off
        pb_params vp = *prm;
        for (int d = 0; d < 3; ++d) vp.origin[d] = prm->origin[d] + prm->h * (double)off[d];
        rc = validate(&vp, na, xyz, rad, chg);
    } else {
        rc = validate(prm, na, xyz, rad, chg);
    }
    if (rc) return rc;
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;

    pb_problem* pb = new pb_problem();
    pb->ctx = ctx;
    pb->prm = *prm;
    pb->prm.bc_values = nullptr;
    pb->na = na;
    pb->mem.ctx = ctx;
    pb->bt = new BuildTmp();
    BuildTmp& T = *pb->bt;
    Grid& g = pb->g;
    g.nx = prm->n[0];
    g.ny = prm->n[1];
    g.nz = prm->n[2];
    g.S = (int)row_stride(g.nz);
    g.N = (int64_t)g.nx * g.ny * g.S;
    g.h = prm->h;
    g.ox = prm->origin[0];
    g.oy = prm->origin[1];
    g.oz = prm->origin[2];
    if (off)
        for (int d = 0; d < 3; ++d) g.off[d] = off[d];
    pb->ts = make_tiles(g, prm->tile_planes);
    double kd2 = 0;
    reduced_constants(prm->temperature_K, prm->ionic_strength_M, prm->eps_out, &pb->lB, &kd2);
    pb->kD = std::sqrt(kd2);
    pb->cf.kin = prm->h * prm->eps_in;
    pb->cf.kout = prm->h * prm->eps_out;
    pb->cf.mass = prm->h * prm->h * prm->h * prm->eps_out * kd2;

    auto bail = [&](int code) {
        pbi_problem_destroy(pb, true);
        return code;
    };
#define CK(expr)                    \
    do {                            \
        int rc_ = (expr);           \
        if (rc_) return bail(rc_);  \
    } while (0)
#define HK(expr)                                                                              \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return bail(fail(PB_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)));      \
    } while (0)

    HK(hipEventCreateWithFlags(&pb->ev, hipEventDisableTiming));
    const size_t N = (size_t)g.N;
    const size_t na1 = (size_t)std::max<int64_t>(na, 1);
    pb->xyzr = dalloc<double>(pb, 4 * na1, &rc);
    CK(rc);
    pb->q = dalloc<double>(pb, na1, &rc);
    CK(rc);
    // pinned staging: atoms (x, y, z, R), charges, and the two counts read back later
    T.hpin = (double*)ctx->pinned.get(sizeof(double) * 5 * na1 + 64, &T.hpin_cap);
    if (!T.hpin) return bail(fail(PB_EDEVICE, "pinned host allocation failed"));
    double* hx = T.hpin;
    double* hq = T.hpin + 4 * na1;
    T.htot = (int*)(T.hpin + 5 * na1);
    double rmax = 0, lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (size_t a = 0; a < na1; ++a) {
        for (int d = 0; d < 4; ++d) hx[4 * a + d] = 0.0;
        hq[a] = 0.0;
    }
    for (int64_t a = 0; a < na; ++a) {
        for (int d = 0; d < 3; ++d) {
            hx[4 * a + d] = xyz[3 * a + d];
            lo[d] = a ? std::min(lo[d], xyz[3 * a + d]) : xyz[3 * a + d];
            hi[d] = a ? std::max(hi[d], xyz[3 * a + d]) : xyz[3 * a + d];
        }
        hx[4 * a + 3] = rad[a];
        hq[a] = chg[a];
        rmax = std::max(rmax, rad[a]);
    }
    HK(hipMemcpyAsync(pb->xyzr, hx, sizeof(double) * 4 * na1, hipMemcpyHostToDevice, s));
    HK(hipMemcpyAsync(pb->q, hq, sizeof(double) * na1, hipMemcpyHostToDevice, s));
    for (int d = 0; d < 3; ++d) pb->ctr[d] = na > 0 ? 0.5 * (lo[d] + hi[d]) : 0.0;
    const Atoms at = pbi_atoms(pb);

    // bins of edge >= R_max + h (and >= 2h) so that the 27 bins around a node or an edge end
    // hold every atom whose ball can touch it
    Bins& bn = T.bn;
    bn.bs = std::max(rmax + prm->h, 2.0 * prm->h);
    bn.lox = lo[0] - bn.bs;
    bn.loy = lo[1] - bn.bs;
    bn.loz = lo[2] - bn.bs;
    bn.nbx = (int)std::floor((hi[0] - bn.lox) / bn.bs) + 2;
    bn.nby = (int)std::floor((hi[1] - bn.loy) / bn.bs) + 2;
    bn.nbz = (int)std::floor((hi[2] - bn.loz) / bn.bs) + 2;
    const int nbins = bn.nbx * bn.nby * bn.nbz;
    T.bcnt = dalloc<int>(pb, (size_t)nbins + 1, &rc);
    CK(rc);
    T.bstart = dalloc<int>(pb, (size_t)nbins + 1, &rc);
    CK(rc);
    T.bcur = dalloc<int>(pb, (size_t)nbins + 1, &rc);
    CK(rc);
    T.bids = dalloc<int>(pb, na1, &rc);
    CK(rc);
    T.bxyzr = dalloc<double>(pb, 4 * (size_t)na1, &rc);
    CK(rc);
    if (na > 0) {
        HK(launch_bins(s, at, bn, T.bcnt, T.bstart, T.bids, T.bcur, T.bxyzr));
    } else {
        HK(launch_fill(s, T.bstart, sizeof(int) * ((size_t)nbins + 1)));
        bn.start = T.bstart;
        bn.ids = T.bids;
    }

    // classification and counting of the cut edges
    T.cls = dalloc<uint32_t>(pb, N, &rc);
    CK(rc);
    HK(launch_classify(s, g, bn, T.bxyzr, T.cls));
    T.nblk = (int)((N + 255) / 256);
    T.bslots = dalloc<int>(pb, (size_t)T.nblk + 1, &rc);
    CK(rc);
    T.bcuts = dalloc<int>(pb, (size_t)T.nblk + 1, &rc);
    CK(rc);
    T.tot = dalloc<int>(pb, 2, &rc);
    CK(rc);
    HK(launch_cutflags(s, g, T.cls, T.bslots, T.bcuts, T.nblk));
    HK(launch_scan2(s, T.bslots, T.bcuts, T.nblk, T.tot));
    HK(hipMemcpyAsync(T.htot, T.tot, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    if (prm->bc == PB_BC_USER) {
        const size_t nfull = (size_t)g.nx * g.ny * g.nz;
        T.full = dalloc<double>(pb, nfull, &rc);
        CK(rc);
        HK(hipMemcpy(T.full, prm->bc_values, sizeof(double) * nfull, hipMemcpyHostToDevice));
    }
    HK(hipEventRecord(pb->ev, s));
#undef CK
#undef HK
    *out = pb;
    return PB_OK;
}
}  // namespace

int pbi_build_continue(pb_problem* pb)
{
    BuildTmp& T = *pb->bt;
    const pb_params* prm = &pb->prm;
    const Grid& g = pb->g;
    hipStream_t s = pb->ctx->stream;
    int rc = PB_OK;
#define CK(expr)                    \
    do {                            \
        int rc_ = (expr);           \
        if (rc_) return rc_;        \
    } while (0)
    pb->nslot = T.htot[0];
    pb->ncut = T.htot[1];
    const size_t N = (size_t)g.N;
    const size_t ns1 = (size_t)std::max<int64_t>(pb->nslot, 1), nc1 = (size_t)std::max<int64_t>(pb->ncut, 1);
    const Atoms at = pbi_atoms(pb);

    pb->code = dalloc<uint32_t>(pb, N, &rc);
    CK(rc);
    pb->cutbase = dalloc<int>(pb, ns1, &rc);
    CK(rc);
    pb->cutkey = dalloc<int64_t>(pb, nc1, &rc);
    CK(rc);
    HIPCHK(launch_assign(s, g, T.cls, pb->code, T.bslots, T.bcuts, pb->cutbase, pb->cutkey));
    pb->ck64 = dalloc<double>(pb, 3 * ns1, &rc);
    CK(rc);
    pb->ck32 = dalloc<float>(pb, 3 * ns1, &rc);
    CK(rc);
    HIPCHK(launch_fill(s, pb->ck64, sizeof(double) * 3 * ns1));
    HIPCHK(launch_fill(s, pb->ck32, sizeof(float) * 3 * ns1));
    pb->alpha = dalloc<double>(pb, nc1, &rc);
    CK(rc);
    pb->kcut = dalloc<double>(pb, nc1, &rc);
    CK(rc);
    pb->rp = dalloc<double>(pb, 3 * nc1, &rc);
    CK(rc);
    pb->np = dalloc<double>(pb, 3 * nc1, &rc);
    CK(rc);
    pb->owner = dalloc<int>(pb, nc1, &rc);
    CK(rc);
    pb->wp = dalloc<double>(pb, nc1, &rc);
    CK(rc);
    HIPCHK(launch_cut_geom(s, g, T.bn, T.bxyzr, at, prm->eps_in, prm->eps_out, pb->ncut, pb->cutkey, pb->code, pb->alpha,
                           pb->kcut, pb->rp, pb->np, pb->owner, pb->ck64, pb->ck32));

    // load vector, boundary values, diagonal and lift
    pb->rhs = dalloc<double>(pb, N, &rc);
    CK(rc);
    pb->gb = dalloc<double>(pb, N, &rc);
    CK(rc);
    pb->x = dalloc<double>(pb, N, &rc);
    CK(rc);
    T.acell = dalloc<double>(pb, 8 * (size_t)std::max<int64_t>(pb->na, 1), &rc);
    CK(rc);
    HIPCHK(launch_deposit(s, g, T.bn, at, T.acell, pb->rhs));
    HIPCHK(launch_fill(s, pb->gb, sizeof(double) * N));
    HIPCHK(launch_fill(s, pb->x, sizeof(double) * N));
    if (prm->bc == PB_BC_DH && pb->na > 0) {
        const DhSplit sp = dh_split(g, at.n);
        T.dhpart = dalloc<double>(pb, (size_t)sp.ranges * sp.nbox, &rc);
        CK(rc);
        if (prm->precision == PB_MIXED)
            HIPCHK(launch_bc_dh32(s, g, at, pb->kD, prm->eps_out, T.dhpart, pb->gb));
        else
            HIPCHK(launch_bc_dh(s, g, at, pb->kD, prm->eps_out, T.dhpart, pb->gb));
    } else if (prm->bc == PB_BC_USER) {
        HIPCHK(launch_bc_user(s, g, T.full, pb->gb));
    }
    HIPCHK(launch_diag_lift(s, g, pb->code, pb->ck64, pb->cf, pb->gb, pb->rhs, nullptr, nullptr));
    HIPCHK(launch_mc_weights(s, g, pb->code, pb->cutbase, pb->ncut, pb->cutkey, pb->rp, pb->wp));

    // solver scalars and partial sums
    pb->nb = pb->ts.items;
    pb->nbres = residual_blocks(g);
    pb->part = dalloc<double>(pb, 5 * (size_t)pb->nb, &rc);
    CK(rc);
    pb->part_res = dalloc<double>(pb, 3 * (size_t)pb->nbres, &rc);
    CK(rc);
    pb->st = dalloc<CGState>(pb, 1, &rc);
    CK(rc);
#undef CK
    HIPCHK(hipEventRecord(pb->ev, s));
    return PB_OK;
}

void pbi_build_end(pb_problem* pb) { release_tmp(pb); }

int64_t pbi_build_counted_cuts(const pb_problem* pb) { return pb->bt ? pb->bt->htot[1] : pb->ncut; }

extern "C" {

int pb_build_coeffs(pb_ctx* ctx, const pb_params* prm, int64_t na, const double* xyz, const double* rad,
                    const double* chg, pb_problem** out)
{
    pb_problem* pb = nullptr;
    int rc = pbi_build_begin(ctx, prm, na, xyz, rad, chg, &pb);
    if (rc) return rc;
    if (hipEventSynchronize(pb->ev) != hipSuccess) rc = fail(PB_EDEVICE, "build: counting failed");
    if (!rc) rc = pbi_build_continue(pb);
    if (!rc && hipEventSynchronize(pb->ev) != hipSuccess) rc = fail(PB_EDEVICE, "build failed");
    if (rc) {
        pbi_problem_destroy(pb, true);
        return rc;
    }
    pbi_build_end(pb);
    if (prm->refine && (rc = pbi_refine_build(pb, xyz, rad, chg))) {
        pbi_problem_destroy(pb, true);
        return rc;
    }
    *out = pb;
    return PB_OK;
}

int pb_solve(pb_problem* pb, pb_solve_stats* stats)
{
    if (!pb || !stats) return fail(PB_EINVAL, "NULL argument");
    memset(stats, 0, sizeof *stats);
    pb_ctx* ctx = pb->ctx;
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const double t0 = now_s();
    pb->solved = false;
    pb->prof_stencil_ms = pb->prof_update_ms = 0;
    pb->prof_n = 0;
    int rc = PB_OK;
    const pb_params& P = pb->prm;
    int status = PB_OK;
    CGState st;
    if (pb->ref) {
        if ((rc = pbi_refine_solve(pb, &st))) return rc;
        stats->iters = st.status == 1 ? st.iters : st.iter_count;
        const double rr = P.precision == PB_MIXED ? st.rr64 : st.rr;
        stats->relres = st.bnorm2 > 0 ? std::sqrt(rr / st.bnorm2) : 0.0;
        stats->outer_iters = P.precision == PB_MIXED ? st.n_ru : 0;
        status = st.status == 1 ? PB_OK : st.status == 2 ? PB_EBREAKDOWN : PB_ENOCONV;
        stats->status = status;
        stats->t_solve_s = now_s() - t0;
        pb->solved = pb->ref->fine->solved = status == PB_OK || status == PB_ENOCONV;
        return status;
    }
    if (P.precond == PB_PRECOND_MG) {
        if ((rc = pbi_mg_solve(pb, &st))) return rc;
        stats->iters = st.status == 1 ? st.iters : st.iter_count;
        const double rr = P.precision == PB_MIXED ? st.rr64 : st.rr;
        stats->relres = st.bnorm2 > 0 ? std::sqrt(rr / st.bnorm2) : 0.0;
        stats->outer_iters = P.precision == PB_MIXED ? st.n_ru : 0;
        status = st.status == 1 ? PB_OK : st.status == 2 ? PB_EBREAKDOWN : PB_ENOCONV;
        stats->status = status;
        stats->t_solve_s = now_s() - t0;
        pb->solved = status == PB_OK || status == PB_ENOCONV;
        return status;
    }
    if (P.precision == PB_FP64 && (rc = ensure_cg64(pb))) return rc;
    if (P.precision == PB_FP64) {
        CGBufs<double> B = bufs<double>(pb);
        HIPCHK(launch_cg_init<double>(s, pb->g, B, pb->cf, pb->rhs, nullptr));
        HIPCHK(launch_cg_fin(s, pb->part, pb->nb, pb->st, P.rtol * P.rtol));
        rc = run_cg<double>(pb, B, P.max_iter, false, &st);
        if (rc) return rc;
        stats->iters = st.status == 1 ? st.iters : st.iter_count;
        stats->relres = st.bnorm2 > 0 ? std::sqrt(st.rr / st.bnorm2) : 0.0;
    } else {
        if ((rc = pbi_mixed_begin(pb))) return rc;
        CGBufs<float> B = bufs<float>(pb);
        rc = run_cg<float>(pb, B, P.max_iter, true, &st);
        if (rc) return rc;
        stats->iters = st.status == 1 ? st.iters : st.iter_count;
        stats->outer_iters = st.n_ru;
        const double bn2 = P.rtol > 0 ? st.goal64 / (P.rtol * P.rtol) : 0.0;
        stats->relres = bn2 > 0 ? std::sqrt(st.rr64 / bn2) : 0.0;
    }
    status = st.status == 1 ? PB_OK : st.status == 2 ? PB_EBREAKDOWN : PB_ENOCONV;
    HIPCHK(hipStreamSynchronize(s));
    stats->status = status;
    stats->t_solve_s = now_s() - t0;
    pb->solved = status == PB_OK || status == PB_ENOCONV;
    return status;
}

int pb_get_energy_profile(const pb_problem* pb, double* nbody_ms, double* pairs)
{
    if (!pb) return fail(PB_EINVAL, "NULL problem");
    const pb_problem* q = pb->ref ? pb->ref->fine : pb;   // a refined problem's energy runs on its fine lattice
    if (nbody_ms) *nbody_ms = q->prof_nbody_ms;
    if (pairs) *pairs = q->prof_nbody_pairs;
    return PB_OK;
}

int pb_get_profile(const pb_problem* pb, double* stencil_ms_avg, double* update_ms_avg, int32_t* samples)
{
    if (!pb) return fail(PB_EINVAL, "NULL problem");
    const int n = pb->prof_n;
    if (stencil_ms_avg) *stencil_ms_avg = n ? pb->prof_stencil_ms / n : 0.0;
    if (update_ms_avg) *update_ms_avg = n ? pb->prof_update_ms / n : 0.0;
    if (samples) *samples = n;
    return PB_OK;
}

int pb_energy(pb_problem* pb, pb_energy_out* out, double* phi_reac)
{
    if (!pb || !out) return fail(PB_EINVAL, "NULL argument");
    if (!pb->solved) return fail(PB_EINVAL, "pb_energy before a successful pb_solve");
    if (pb->ref) pb = pb->ref->fine;   // the cut edges all lie on the fine sub-lattice
    HIPCHK(hipSetDevice(pb->ctx->device));
    const double t0 = now_s();
    int rc = pbi_energy_begin(pb, 0);
    if (rc) return rc;
    if (hipEventSynchronize(pb->ev) != hipSuccess) rc = fail(PB_EDEVICE, "energy kernels failed");
    if (!rc && phi_reac && pb->na > 0) {
        hipError_t e = hipMemcpyAsync(phi_reac, pb->e_tmp[2], sizeof(double) * (size_t)pb->na, hipMemcpyDeviceToHost,
                                      pb->ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(pb->ctx->stream);
        if (e != hipSuccess) rc = fail(PB_EDEVICE, "per-atom copy: %s", hipGetErrorString(e));
    }
    const int rc2 = pbi_energy_end(pb, out, nullptr);
    if (!rc) rc = rc2;
    out->t_energy_s = now_s() - t0;
    return rc;
}

int pb_grid_energy(pb_problem* pb, double* e_grid)
{
    if (!pb || !e_grid) return fail(PB_EINVAL, "NULL argument");
    if (!pb->solved) return fail(PB_EINVAL, "pb_grid_energy before a successful pb_solve");
    if (pb->ref) return fail(PB_EINVAL, "pb_grid_energy: locally refined problems are not supported");
    *e_grid = 0.0;
    if (pb->na == 0) return PB_OK;
    HIPCHK(hipSetDevice(pb->ctx->device));
    hipStream_t s = pb->ctx->stream;
    const Atoms at = pbi_atoms(pb);
    const int nb = grid_energy_blocks(at.n);
    int rc = PB_OK;
    double* part = dalloc<double>(pb, (size_t)nb + 1, &rc);
    if (rc) return rc;
    hipError_t e = launch_grid_energy(s, pb->g, at, pb->x, 0.5 * pb->lB, part);
    if (e == hipSuccess) e = hipMemcpyAsync(e_grid, part + nb, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    pb->mem.put(part);
    if (e != hipSuccess) return fail(PB_EDEVICE, "grid energy: %s", hipGetErrorString(e));
    return PB_OK;
}

int pb_copy_potential(const pb_problem* pb, double* host_phi)
{
    if (!pb || !host_phi) return fail(PB_EINVAL, "NULL argument");
    pb_problem* p = const_cast<pb_problem*>(pb);
    HIPCHK(hipSetDevice(pb->ctx->device));
    hipStream_t s = pb->ctx->stream;
    const size_t n = (size_t)pb->g.nx * pb->g.ny * pb->g.nz;
    int rc = PB_OK;
    double* tmp = dalloc<double>(p, n, &rc);
    if (rc) return rc;
    hipError_t e = launch_export_phi(s, pb->g, pb->x, pb->gb, pb->lB, tmp);
    if (e == hipSuccess) e = hipMemcpyAsync(host_phi, tmp, sizeof(double) * n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    p->mem.put(tmp);
    if (e != hipSuccess) return fail(PB_EDEVICE, "export failed: %s", hipGetErrorString(e));
    return PB_OK;
}

int pb_copy_coeffs(const pb_problem* pb, uint8_t* sol, double* kx, double* ky, double* kz, double* diag,
                   double* rhs)
{
    if (!pb) return fail(PB_EINVAL, "NULL problem");
    pb_problem* p = const_cast<pb_problem*>(pb);
    HIPCHK(hipSetDevice(pb->ctx->device));
    hipStream_t s = pb->ctx->stream;
    const size_t n = (size_t)pb->g.nx * pb->g.ny * pb->g.nz;
    int rc = PB_OK;
    uint8_t* dsol = dalloc<uint8_t>(p, n, &rc);
    double* dk[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    double* hk[5] = {kx, ky, kz, diag, rhs};
    for (int t = 0; t < 5 && !rc; ++t)
        if (hk[t]) dk[t] = dalloc<double>(p, n, &rc);
    hipError_t e = hipSuccess;
    if (!rc) {
        e = launch_export_coeffs(s, pb->g, pb->code, pb->ck64, pb->cf, pb->rhs, dsol, dk[0], dk[1], dk[2], dk[3],
                                 dk[4]);
        if (e == hipSuccess && sol) e = hipMemcpyAsync(sol, dsol, n, hipMemcpyDeviceToHost, s);
        for (int t = 0; t < 5 && e == hipSuccess; ++t)
            if (hk[t]) e = hipMemcpyAsync(hk[t], dk[t], sizeof(double) * n, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    if (dsol) p->mem.put(dsol);
    for (int t = 0; t < 5; ++t)
        if (dk[t]) p->mem.put(dk[t]);
    if (rc) return rc;
    if (e != hipSuccess) return fail(PB_EDEVICE, "export failed: %s", hipGetErrorString(e));
    return PB_OK;
}

int64_t pb_num_cut(const pb_problem* pb)
{
    if (!pb) return fail(PB_EINVAL, "NULL problem");
    return pb->ref ? pb->ref->fine->ncut : pb->ncut;
}

int pb_copy_cut(const pb_problem* pb, int64_t* key, double* alpha, double* rp, double* np, int64_t* owner,
                double* wp, double* F, double* phip)
{
    if (!pb) return fail(PB_EINVAL, "NULL problem");
    // a refined problem's surface lies on its fine sub-lattice (the energy read-back's list)
    if (pb->ref) return pb_copy_cut(pb->ref->fine, key, alpha, rp, np, owner, wp, F, phip);
    HIPCHK(hipSetDevice(pb->ctx->device));
    hipStream_t s = pb->ctx->stream;
    const size_t m = (size_t)pb->ncut;
    if (m == 0) return PB_OK;
    if ((F || phip) && !pb->F) return fail(PB_EINVAL, "F/phip requested before pb_energy");
    std::vector<int64_t> sk(m);
    std::vector<int> ow(m);
    HIPCHK(hipMemcpyAsync(sk.data(), pb->cutkey, sizeof(int64_t) * m, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(ow.data(), pb->owner, sizeof(int) * m, hipMemcpyDeviceToHost, s));
    if (alpha) HIPCHK(hipMemcpyAsync(alpha, pb->alpha, sizeof(double) * m, hipMemcpyDeviceToHost, s));
    if (rp) HIPCHK(hipMemcpyAsync(rp, pb->rp, sizeof(double) * 3 * m, hipMemcpyDeviceToHost, s));
    if (np) HIPCHK(hipMemcpyAsync(np, pb->np, sizeof(double) * 3 * m, hipMemcpyDeviceToHost, s));
    if (wp) HIPCHK(hipMemcpyAsync(wp, pb->wp, sizeof(double) * m, hipMemcpyDeviceToHost, s));
    if (F) HIPCHK(hipMemcpyAsync(F, pb->F, sizeof(double) * m, hipMemcpyDeviceToHost, s));
    if (phip) HIPCHK(hipMemcpyAsync(phip, pb->phip, sizeof(double) * m, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const Grid& g = pb->g;
    for (size_t c = 0; c < m; ++c) {
        // storage element -> (i, j, k) -> unpadded key
        const int64_t e = sk[c] >> 2;
        const int ax = (int)(sk[c] & 3);
        const int64_t row = e / g.S;
        const int64_t k = e - row * g.S - Z0;
        const int64_t j = row % g.ny, i = row / g.ny;
        if (key) key[c] = 3 * ((i * g.ny + j) * g.nz + k) + ax;
        if (owner) owner[c] = ow[c];
    }
    return PB_OK;
}

int pb_binding_ddg(const pb_energy_out* c, const pb_energy_out* a, const pb_energy_out* b, pb_binding_out* out)
{
    if (!c || !a || !b || !out) return fail(PB_EINVAL, "NULL argument");
    out->ddg_coul = c->e_coul - a->e_coul - b->e_coul;
    out->ddg_pol = c->e_pol - a->e_pol - b->e_pol;
    out->ddg_ion = c->e_ion - a->e_ion - b->e_ion;
    out->ddg_total = c->e_total - a->e_total - b->e_total;
    return PB_OK;
}

int pb_mg_vcycle(pb_problem* pb, const double* r_host, double* z_host, int32_t* levels)
{
    if (!pb || !r_host || !z_host) return fail(PB_EINVAL, "NULL argument");
    if (pb->prm.precond != PB_PRECOND_MG) return fail(PB_EINVAL, "not a multigrid-preconditioned problem");
    HIPCHK(hipSetDevice(pb->ctx->device));
    const Grid& g = pb->g;
    std::vector<double> r((size_t)g.N, 0.0), z((size_t)g.N, 0.0);
    for (int i = 1; i < g.nx - 1; ++i)
        for (int j = 1; j < g.ny - 1; ++j)
            for (int k = 1; k < g.nz - 1; ++k)
                r[(size_t)g.idx(i, j, k)] = r_host[((size_t)i * g.ny + j) * g.nz + k];
    const int rc = pbi_mg_vcycle_test(pb, r.data(), z.data());
    if (rc) return rc;
    for (int i = 0; i < g.nx; ++i)
        for (int j = 0; j < g.ny; ++j)
            for (int k = 0; k < g.nz; ++k) z_host[((size_t)i * g.ny + j) * g.nz + k] = z[(size_t)g.idx(i, j, k)];
    if (levels) *levels = pbi_mg_levels(pb);
    return PB_OK;
}

int pb_time_stencil(pb_problem* pb, int32_t reps, int32_t fp32, double* avg_ms)
{
    if (!pb || !avg_ms || reps <= 0) return fail(PB_EINVAL, "bad argument");
    if (pb->ref) return fail(PB_EINVAL, "pb_time_stencil times the uniform-grid iteration kernel");
    HIPCHK(hipSetDevice(pb->ctx->device));
    hipStream_t s = pb->ctx->stream;
    int rc = fp32 ? ensure_cg32(pb) : ensure_cg64(pb);
    if (rc) return rc;
    hipEvent_t a, b;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    pb->solved = false;
    const double rtol2 = pb->prm.rtol * pb->prm.rtol;
    if (fp32) {
        CGBufs<float> B = bufs<float>(pb);
        HIPCHK(launch_cg_init<float>(s, pb->g, B, pb->cf, pb->rhs, nullptr));
        HIPCHK(launch_cg_fin(s, pb->part, pb->nb, pb->st, rtol2));
        HIPCHK(launch_cg_iter<float>(s, pb->g, pb->ts, B, pb->cf));
        HIPCHK(hipEventRecord(a, s));
        for (int t = 0; t < reps; ++t) HIPCHK(launch_cg_iter<float>(s, pb->g, pb->ts, B, pb->cf));
        HIPCHK(hipEventRecord(b, s));
    } else {
        CGBufs<double> B = bufs<double>(pb);
        HIPCHK(launch_cg_init<double>(s, pb->g, B, pb->cf, pb->rhs, nullptr));
        HIPCHK(launch_cg_fin(s, pb->part, pb->nb, pb->st, rtol2));
        HIPCHK(launch_cg_iter<double>(s, pb->g, pb->ts, B, pb->cf));
        HIPCHK(hipEventRecord(a, s));
        for (int t = 0; t < reps; ++t) HIPCHK(launch_cg_iter<double>(s, pb->g, pb->ts, B, pb->cf));
        HIPCHK(hipEventRecord(b, s));
    }
    HIPCHK(hipEventSynchronize(b));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *avg_ms = ms / reps;
    return PB_OK;
}

int pb_stream_copy(pb_ctx* ctx, size_t bytes, int32_t reps, double* gbps)
{
    if (!ctx || !gbps || reps <= 0 || bytes < 16) return fail(PB_EINVAL, "bad argument");
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    bytes &= ~(size_t)15;
    void* a = ctx->alloc(bytes, ctx->user);
    void* b = a ? ctx->alloc(bytes, ctx->user) : nullptr;
    if (!a || !b) {
        if (a) ctx->free_fn(a, ctx->user);
        return fail(PB_ENOMEM, "stream copy buffers");
    }
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = launch_fill(s, a, bytes);
    for (int t = 0; t < 2 && e == hipSuccess; ++t) e = launch_stream_copy(s, a, b, bytes);
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int t = 0; t < reps && e == hipSuccess; ++t) e = launch_stream_copy(s, a, b, bytes);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->free_fn(a, ctx->user);
    ctx->free_fn(b, ctx->user);
    if (e != hipSuccess) return fail(PB_EDEVICE, "stream copy: %s", hipGetErrorString(e));
    *gbps = 2.0 * (double)bytes * reps / (ms * 1e-3) / 1e9;
    return PB_OK;
}

size_t pb_problem_bytes(const pb_problem* pb) { return pb ? pb->mem.bytes : 0; }

void pb_problem_free(pb_problem* pb) { pbi_problem_destroy(pb, true); }

int pb_refine_info(const pb_problem* pb, pb_refine_stats* out)
{
    if (!pb || !out) return fail(PB_EINVAL, "NULL argument");
    memset(out, 0, sizeof *out);
    if (!pb->ref) return PB_OK;
    const RefineData* R = pb->ref;
    const Grid& gf = R->fine->g;
    out->fine_n[0] = gf.nx;
    out->fine_n[1] = gf.ny;
    out->fine_n[2] = gf.nz;
    for (int d = 0; d < 3; ++d) out->fine_offset[d] = gf.off[d];
    out->refined_cells = R->n_refined;
    out->hanging_nodes = R->nhang;
    out->unknowns_coarse = R->nunk_c;
    out->unknowns_fine = R->nunk_f;
    return PB_OK;
}

int pb_copy_refined_cells(const pb_problem* pb, uint8_t* host)
{
    if (!pb || !host) return fail(PB_EINVAL, "NULL argument");
    if (!pb->ref) return fail(PB_EINVAL, "not a refined problem");
    HIPCHK(hipSetDevice(pb->ctx->device));
    const RefineData* R = pb->ref;
    const size_t n = (size_t)R->nc[0] * R->nc[1] * R->nc[2];
    HIPCHK(hipMemcpyAsync(host, R->cells, n, hipMemcpyDeviceToHost, pb->ctx->stream));
    HIPCHK(hipStreamSynchronize(pb->ctx->stream));
    return PB_OK;
}

int pb_copy_fine_potential(const pb_problem* pb, double* host_phi)
{
    if (!pb || !host_phi) return fail(PB_EINVAL, "NULL argument");
    if (!pb->ref) return fail(PB_EINVAL, "not a refined problem");
    return pb_copy_potential(pb->ref->fine, host_phi);
}

}  // extern "C"
