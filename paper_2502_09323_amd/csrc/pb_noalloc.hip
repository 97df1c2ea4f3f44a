// pb_noalloc.hip -- the energy read-back without any allocation, for callers that cannot
// allocate device or pinned host memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid allocation).
//
// pb_energy allocates the read-back's buffers through the context allocator (and pinned host
// blocks for the sums).  pb_energy_noalloc runs the same kernels on the same problem, with
// every buffer beyond the problem's own state carved from one file-scope device array,
// `scratch`, and the sums copied straight into the caller's host memory.  Each device holds
// its own copy of the array for the life of the process; its address on a device is taken
// once, with hipGetSymbolAddress, when the first context on that device is created.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <mutex>

#include "pb_host.h"

using namespace pbk;

namespace {

constexpr size_t SCRATCH_BYTES = (size_t)128 << 20;   // 128 MiB on every device the library runs on
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};   // device address of `scratch` on each device (nullptr: not yet taken)

size_t up256(size_t n) { return (n + 255) & ~(size_t)255; }

// where the read-back's buffers sit in the scratch array, for a problem of na atoms and ncut
// cut edges with the N-body sum split in nchunk chunks; returns the bytes used
struct Layout {
    size_t F, phip, pts, partial, phic, reac, sums, end;
};

Layout layout(int64_t na, int64_t ncut, int nchunk, int ncc)
{
    const size_t nc1 = (size_t)std::max<int64_t>(ncut, 1), na1 = (size_t)std::max<int64_t>(na, 1);
    Layout L;
    size_t o = 0;
    L.F = o;
    o += up256(8 * nc1);
    L.phip = o;
    o += up256(8 * nc1);
    L.pts = o;
    o += up256(8 * (size_t)CUT_POINT_DOUBLES * nc1);
    L.partial = o;
    o += up256(8 * (size_t)energy_partial_doubles((int)na1, nchunk));
    L.phic = o;
    o += up256(8 * na1 * (size_t)ncc);
    L.reac = o;
    o += up256(8 * na1);
    L.sums = o;
    o += up256(8 * (size_t)ENERGY_OUT_DOUBLES);
    L.end = o;
    return L;
}

}  // namespace

int pbi_scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return pbi_fail(PB_EINVAL, "device %d: at most %d devices", device, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device]) return PB_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));   // the calling thread's device is `device`
    if (e != hipSuccess || !p)
        return pbi_fail(PB_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
    g_ptr[device] = p;
    return PB_OK;
}

extern "C" {

size_t pb_energy_noalloc_limit(void) { return SCRATCH_BYTES; }

int pb_energy_noalloc(pb_problem* pb, pb_energy_out* out, double* phi_reac)
{
    if (!pb || !out) return pbi_fail(PB_EINVAL, "NULL argument");
    if (pb->ref) pb = pb->ref->fine;   // the cut edges all lie on the fine sub-lattice
    const int dev = pb->ctx->device;
    void* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        base = dev >= 0 && dev < kMaxDevices ? g_ptr[dev] : nullptr;
    }
    if (!base) return pbi_fail(PB_EDEVICE, "pb_energy_noalloc: no scratch address for device %d", dev);
    // the same N-body split as pb_energy when it fits, else fewer chunks (the sums then differ
    // from pb_energy's only in the order of the FP64 additions)
    const int64_t na = pb->na, ncut = pb->ncut;
    const int na1 = (int)std::max<int64_t>(na, 1);
    const int ncc = coulomb_chunks(na1);
    int nchunk = nbody_chunks(na1, ncut);
    while (nchunk > 1 && layout(na, ncut, nchunk, ncc).end > SCRATCH_BYTES) nchunk = (nchunk + 1) / 2;
    const Layout L = layout(na, ncut, nchunk, ncc);
    if (L.end > SCRATCH_BYTES)
        return pbi_fail(PB_ENOMEM, "pb_energy_noalloc: %lld atoms and %lld cut edges need %zu bytes of scratch, "
                                   "the limit is %zu (use pb_energy)",
                        (long long)na, (long long)ncut, L.end, SCRATCH_BYTES);
    if (!pb->solved) return pbi_fail(PB_EINVAL, "pb_energy_noalloc before a successful pb_solve");
    if (hipSetDevice(dev) != hipSuccess) return pbi_fail(PB_EDEVICE, "hipSetDevice(%d) failed", dev);
    const double t0 = std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
    unsigned char* b = (unsigned char*)base;
    double* F = (double*)(b + L.F);
    double* phip = (double*)(b + L.phip);
    double* pts = (double*)(b + L.pts);
    double* partial = (double*)(b + L.partial);
    double* phic = (double*)(b + L.phic);
    double* reac = (double*)(b + L.reac);
    double* sums = (double*)(b + L.sums);
    hipStream_t s = pb->ctx->stream;
    const Atoms at = pbi_atoms(pb);
    hipError_t e = launch_fill(s, sums, 16 * sizeof(double));
    if (e == hipSuccess)
        e = launch_edge_fields(s, pb->g, at, pb->prm.eps_in, pb->prm.eps_out, ncut, pb->cutkey, pb->code, pb->alpha,
                               pb->kcut, pb->x, pb->gb, pb->wp, F, phip, pts, pb->rp, pb->np);
    if (e == hipSuccess && na > 0) {
        if (ncut > 0)
            e = launch_nbody(s, at, ncut, pts, partial, nchunk);
        else
            e = launch_fill(s, partial, sizeof(double) * 2 * (size_t)na1 * (size_t)nchunk);
        if (e == hipSuccess) e = launch_coulomb(s, at, phic, ncc);
        if (e == hipSuccess)
            e = launch_energy_reduce(s, at, partial, nchunk, phic, ncc, pb->prm.eps_in, pb->prm.eps_out, pb->lB, reac,
                                     sums, F, ncut, pb->wp);
    }
    double h[16];
    if (e == hipSuccess) e = hipMemcpyAsync(h, sums, sizeof h, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && phi_reac && na > 0)
        e = hipMemcpyAsync(phi_reac, reac, sizeof(double) * (size_t)na, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return pbi_fail(PB_EDEVICE, "pb_energy_noalloc: %s", hipGetErrorString(e));
    memset(out, 0, sizeof *out);
    out->e_coul = h[0];
    out->e_pol = h[1];
    out->e_ion = h[2];
    out->e_solv = h[1] + h[2];
    out->e_total = h[0] + h[1] + h[2];
    out->q_pol_total = h[3];
    out->area_total = h[4];
    out->n_cut = ncut;
    out->t_energy_s =
        std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count() - t0;
    return PB_OK;
}

}  // extern "C"
