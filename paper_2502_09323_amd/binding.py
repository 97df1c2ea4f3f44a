"""Thin ctypes binding of ``libpb.so`` (the C ABI declared in ``include/pb.h``).

Argument marshalling only: every step of the solve runs in the library's HIP kernels.
PyTorch supplies device memory (its caching allocator, through the library's allocator
callbacks) and the stream.  Loading fails loudly when the HIP library is missing.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# PB_LIB_PATH names another build of the library (the host-code sanitizer test's)
LIB_PATH = os.environ.get("PB_LIB_PATH") or os.path.join(_HERE, "libpb.so")

PB_OK, PB_EINVAL, PB_ENOMEM, PB_ENOCONV, PB_EBREAKDOWN, PB_EDEVICE = 0, -1, -2, -3, -4, -5
PB_ECANCELED, PB_ETIMEDOUT = -6, -7
PB_BC_ZERO, PB_BC_DH, PB_BC_USER = 0, 1, 2
PB_FP64, PB_MIXED = 0, 1
PB_PRECOND_JACOBI, PB_PRECOND_MG = 0, 1

EXPORTED = [
    "pb_ctx_create", "pb_ctx_destroy", "pb_last_error", "pb_build_coeffs", "pb_solve", "pb_energy",
    "pb_copy_potential", "pb_problem_free", "pb_copy_coeffs", "pb_num_cut", "pb_copy_cut",
    "pb_time_stencil", "pb_ctx_set_profiling", "pb_get_profile", "pb_problem_bytes", "pb_stream_copy",
    "pb_server_create", "pb_server_now", "pb_submit", "pb_server_step", "pb_poll", "pb_server_destroy",
    "pb_server_times", "pb_server_profile", "pb_refine_info", "pb_copy_refined_cells", "pb_copy_fine_potential",
    "pb_mg_vcycle", "pb_server_profile_mg", "pb_binding_ddg", "pb_get_energy_profile", "pb_server_profile_energy",
    "pb_grid_energy", "pb_cancel", "pb_server_set_timeout", "pb_server_memory", "pb_energy_noalloc",
    "pb_energy_noalloc_limit", "pb_server_profile_mg_apply",
]


class PbParams(C.Structure):
    _fields_ = [
        ("eps_in", C.c_double), ("eps_out", C.c_double), ("ionic_strength_M", C.c_double),
        ("temperature_K", C.c_double), ("h", C.c_double), ("n", C.c_int32 * 3),
        ("origin", C.c_double * 3), ("bc", C.c_int32), ("bc_values", C.c_void_p),
        ("precision", C.c_int32), ("rtol", C.c_double), ("inner_rtol", C.c_double),
        ("max_iter", C.c_int32), ("tile_planes", C.c_int32),
        ("refine", C.c_int32), ("refine_shell_A", C.c_double), ("refine_brick", C.c_int32),
        ("precond", C.c_int32), ("mg_smooth", C.c_int32), ("mg_coarse_sweeps", C.c_int32),
        ("mg_levels", C.c_int32),
    ]


class PbRefineStats(C.Structure):
    _fields_ = [("fine_n", C.c_int32 * 3), ("fine_offset", C.c_int32 * 3), ("refined_cells", C.c_int64),
                ("hanging_nodes", C.c_int64), ("unknowns_coarse", C.c_int64), ("unknowns_fine", C.c_int64)]


class PbSolveStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("outer_iters", C.c_int32), ("status", C.c_int32),
                ("reserved", C.c_int32), ("relres", C.c_double), ("t_solve_s", C.c_double)]


class PbEnergyOut(C.Structure):
    _fields_ = [("e_coul", C.c_double), ("e_pol", C.c_double), ("e_ion", C.c_double),
                ("e_solv", C.c_double), ("e_total", C.c_double), ("q_pol_total", C.c_double),
                ("area_total", C.c_double), ("n_cut", C.c_int64), ("t_energy_s", C.c_double)]


class PbBindingOut(C.Structure):
    _fields_ = [("ddg_total", C.c_double), ("ddg_coul", C.c_double), ("ddg_pol", C.c_double),
                ("ddg_ion", C.c_double)]


class PbError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libpb error {code}: {msg}")
        self.code = code


_lib = None
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


def load(path: str = LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libpb HIP library not found at {path}; run __graft_entry__.build()")
    # PyTorch brings up the HIP runtime first (its allocator and streams are the ones the
    # library is given), then the library is loaded into the same process
    import torch

    torch.cuda.is_available()
    L = C.CDLL(path)
    P, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    L.pb_ctx_create.argtypes = [C.c_int, P, ALLOC_FN, FREE_FN, P, C.c_size_t, C.POINTER(P)]
    L.pb_ctx_destroy.argtypes = [P]
    L.pb_ctx_destroy.restype = None
    L.pb_last_error.restype = C.c_char_p
    L.pb_build_coeffs.argtypes = [P, C.POINTER(PbParams), i64, P, P, P, C.POINTER(P)]
    L.pb_solve.argtypes = [P, C.POINTER(PbSolveStats)]
    L.pb_energy.argtypes = [P, C.POINTER(PbEnergyOut), P]
    L.pb_energy_noalloc.argtypes = [P, C.POINTER(PbEnergyOut), P]
    L.pb_energy_noalloc_limit.argtypes = []
    L.pb_energy_noalloc_limit.restype = C.c_size_t
    L.pb_copy_potential.argtypes = [P, P]
    L.pb_grid_energy.argtypes = [P, C.POINTER(C.c_double)]
    L.pb_problem_free.argtypes = [P]
    L.pb_problem_free.restype = None
    L.pb_copy_coeffs.argtypes = [P, P, P, P, P, P, P]
    L.pb_num_cut.argtypes = [P]
    L.pb_num_cut.restype = i64
    L.pb_copy_cut.argtypes = [P, P, P, P, P, P, P, P, P]
    L.pb_time_stencil.argtypes = [P, i32, i32, C.POINTER(C.c_double)]
    L.pb_ctx_set_profiling.argtypes = [P, C.c_int]
    L.pb_get_profile.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(i32)]
    L.pb_stream_copy.argtypes = [P, C.c_size_t, i32, C.POINTER(C.c_double)]
    L.pb_problem_bytes.argtypes = [P]
    L.pb_problem_bytes.restype = C.c_size_t
    L.pb_server_create.argtypes = [P, P, i32, C.POINTER(P)]
    L.pb_server_now.argtypes = [P]
    L.pb_server_now.restype = C.c_double
    L.pb_submit.argtypes = [P, C.POINTER(PbParams), i64, P, P, P, C.c_uint64, C.c_double]
    L.pb_server_step.argtypes = [P, C.POINTER(i32), C.POINTER(i32)]
    L.pb_poll.argtypes = [P, P, P, P, P, P, i32, C.POINTER(i32)]
    L.pb_server_times.argtypes = [P, P]
    L.pb_server_profile.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(i64)]
    L.pb_server_profile_mg.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                       C.POINTER(i64)]
    L.pb_server_destroy.argtypes = [P]
    L.pb_server_destroy.restype = None
    L.pb_cancel.argtypes = [P, C.c_uint64]
    L.pb_server_set_timeout.argtypes = [P, C.c_double]
    L.pb_server_memory.argtypes = [P, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t), C.POINTER(i64)]
    L.pb_refine_info.argtypes = [P, C.POINTER(PbRefineStats)]
    L.pb_copy_refined_cells.argtypes = [P, P]
    L.pb_copy_fine_potential.argtypes = [P, P]
    L.pb_mg_vcycle.argtypes = [P, P, P, C.POINTER(i32)]
    L.pb_get_energy_profile.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.pb_server_profile_energy.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(i64)]
    L.pb_server_profile_mg_apply.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(i64)]
    L.pb_binding_ddg.argtypes = [C.POINTER(PbEnergyOut), C.POINTER(PbEnergyOut), C.POINTER(PbEnergyOut),
                                 C.POINTER(PbBindingOut)]
    _lib = L
    return L


def _err(code: int):
    msg = _lib.pb_last_error()
    return PbError(code, msg.decode() if msg else "")


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class Context:
    """Device, stream and allocator (PyTorch's caching allocator) for problems."""

    def __init__(self, device: int = 0, stream=None, hbm_budget_bytes: int = 0):
        import torch
        L = load()
        self.device = device
        self._torch = torch
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        dev, strm = device, self.stream

        def _alloc(nbytes, user):
            try:
                return int(torch.cuda.caching_allocator_alloc(int(nbytes), dev, strm))
            except Exception:
                return None

        def _free(ptr, user):
            torch.cuda.caching_allocator_delete(int(ptr))

        self._cb = (ALLOC_FN(_alloc), FREE_FN(_free))
        h = C.c_void_p()
        rc = L.pb_ctx_create(device, C.c_void_p(self.stream.cuda_stream), self._cb[0], self._cb[1], None,
                             int(hbm_budget_bytes), C.byref(h))
        if rc != PB_OK:
            raise _err(rc)
        self.h = h
        # problems and servers made on this context: released before it, whatever order the
        # interpreter collects them in
        self._users = weakref.WeakSet()

    def set_profiling(self, on: bool):
        rc = _lib.pb_ctx_set_profiling(self.h, 1 if on else 0)
        if rc != PB_OK:
            raise _err(rc)

    def stream_copy_gbps(self, nbytes: int = 1 << 30, reps: int = 10) -> float:
        v = C.c_double()
        rc = _lib.pb_stream_copy(self.h, int(nbytes), int(reps), C.byref(v))
        if rc != PB_OK:
            raise _err(rc)
        return float(v.value)

    def close(self):
        if getattr(self, "h", None):
            for u in list(getattr(self, "_users", ())):
                u.close()
            _lib.pb_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _energy_struct(e: dict) -> PbEnergyOut:
    out = PbEnergyOut()
    for k, _ in PbEnergyOut._fields_:
        setattr(out, k, e.get(k, 0))
    return out


def binding_ddg(e_complex: dict, e_part1: dict, e_part2: dict) -> dict:
    """ddG of a complex from the energies of it and its two parts (pb_binding_ddg)."""
    out = PbBindingOut()
    a, b, c = _energy_struct(e_complex), _energy_struct(e_part1), _energy_struct(e_part2)
    rc = _lib.pb_binding_ddg(C.byref(a), C.byref(b), C.byref(c), C.byref(out))
    if rc != PB_OK:
        raise _err(rc)
    return {k: getattr(out, k) for k, _ in PbBindingOut._fields_}


def make_params(grid) -> PbParams:
    p = PbParams()
    p.eps_in, p.eps_out = float(grid.eps_in), float(grid.eps_out)
    p.ionic_strength_M, p.temperature_K = float(grid.ionic_M), float(grid.temp_K)
    p.h = float(grid.h)
    for d in range(3):
        p.n[d] = int(grid.n[d])
        p.origin[d] = float(grid.origin[d])
    p.bc = int(grid.bc)
    p.precision = int(grid.precision)
    p.rtol, p.inner_rtol = float(grid.rtol), float(grid.inner_rtol)
    p.max_iter = int(grid.max_iter)
    p.tile_planes = int(grid.tile_planes)
    p.refine = int(grid.refine)
    p.refine_shell_A = float(grid.refine_shell)
    p.refine_brick = int(grid.refine_brick)
    p.precond = int(grid.precond)
    p.mg_smooth = int(grid.mg_smooth)
    p.mg_coarse_sweeps = int(grid.mg_coarse_sweeps)
    p.mg_levels = int(grid.mg_levels)
    return p


class Problem:
    """One linearized-PB problem resident on the device."""

    def __init__(self, ctx: Context, mol, grid):
        L = load()
        self.ctx = ctx
        self.grid = grid
        self.n_atoms = int(mol.n)
        p = make_params(grid)
        keep = None
        if grid.bc == PB_BC_USER:
            keep = np.ascontiguousarray(grid.bc_values, dtype=np.float64).reshape(-1)
            p.bc_values = keep.ctypes.data_as(C.c_void_p)
        xyz = np.ascontiguousarray(mol.xyz, dtype=np.float64).reshape(-1)
        rad = np.ascontiguousarray(mol.radius, dtype=np.float64)
        chg = np.ascontiguousarray(mol.charge, dtype=np.float64)
        h = C.c_void_p()
        rc = L.pb_build_coeffs(ctx.h, C.byref(p), self.n_atoms, _ptr(xyz), _ptr(rad), _ptr(chg), C.byref(h))
        if rc != PB_OK:
            raise _err(rc)
        self.h = h
        ctx._users.add(self)

    @property
    def shape(self):
        return tuple(int(v) for v in self.grid.n)

    def solve(self) -> dict:
        st = PbSolveStats()
        rc = _lib.pb_solve(self.h, C.byref(st))
        if rc not in (PB_OK, PB_ENOCONV, PB_EBREAKDOWN):
            raise _err(rc)
        return dict(iters=st.iters, outer_iters=st.outer_iters, status=st.status, relres=st.relres,
                    t_solve_s=st.t_solve_s)

    def energy(self, per_atom: bool = False) -> dict:
        out = PbEnergyOut()
        pa = np.zeros(max(self.n_atoms, 1)) if per_atom else None
        rc = _lib.pb_energy(self.h, C.byref(out), _ptr(pa))
        if rc != PB_OK:
            raise _err(rc)
        d = {k: getattr(out, k) for k, _ in PbEnergyOut._fields_}
        if per_atom:
            d["phi_reac"] = pa[: self.n_atoms]
        return d

    def energy_noalloc(self, per_atom: bool = False) -> dict:
        """pb_energy without any allocation (the read-back's buffers in the library's static
        scratch array); per-atom potentials go to a host array allocated here, before the call."""
        out = PbEnergyOut()
        pa = np.zeros(max(self.n_atoms, 1)) if per_atom else None
        rc = _lib.pb_energy_noalloc(self.h, C.byref(out), _ptr(pa))
        if rc != PB_OK:
            raise _err(rc)
        d = {k: getattr(out, k) for k, _ in PbEnergyOut._fields_}
        if per_atom:
            d["phi_reac"] = pa[: self.n_atoms]
        return d

    def grid_energy(self) -> float:
        """Half the sum of the deposited node charges times the potential (kT); the
        difference of two solves of one geometry at two ionic strengths estimates E_ion."""
        e = C.c_double(0.0)
        rc = _lib.pb_grid_energy(self.h, C.byref(e))
        if rc != PB_OK:
            raise _err(rc)
        return e.value

    def potential(self) -> np.ndarray:
        phi = np.zeros(self.shape)
        rc = _lib.pb_copy_potential(self.h, _ptr(phi))
        if rc != PB_OK:
            raise _err(rc)
        return phi

    def refine_info(self) -> dict:
        st = PbRefineStats()
        rc = _lib.pb_refine_info(self.h, C.byref(st))
        if rc != PB_OK:
            raise _err(rc)
        return dict(fine_n=tuple(st.fine_n), fine_offset=tuple(st.fine_offset), refined_cells=st.refined_cells,
                    hanging_nodes=st.hanging_nodes, unknowns_coarse=st.unknowns_coarse,
                    unknowns_fine=st.unknowns_fine)

    def refined_cells(self) -> np.ndarray:
        out = np.zeros(tuple(int(v) - 1 for v in self.shape), dtype=np.uint8)
        rc = _lib.pb_copy_refined_cells(self.h, _ptr(out))
        if rc != PB_OK:
            raise _err(rc)
        return out

    def fine_potential(self) -> np.ndarray:
        info = self.refine_info()
        phi = np.zeros(info["fine_n"])
        rc = _lib.pb_copy_fine_potential(self.h, _ptr(phi))
        if rc != PB_OK:
            raise _err(rc)
        return phi

    def mg_vcycle(self, r: np.ndarray):
        """One V-cycle of the multigrid preconditioner on r (full grid); (z, levels)."""
        r = np.ascontiguousarray(r, dtype=np.float64)
        z = np.zeros(self.shape)
        lv = C.c_int32(0)
        rc = _lib.pb_mg_vcycle(self.h, _ptr(r), _ptr(z), C.byref(lv))
        if rc != PB_OK:
            raise _err(rc)
        return z, int(lv.value)

    def coeffs(self) -> dict:
        sh = self.shape
        sol = np.zeros(sh, np.uint8)
        arrs = {k: np.zeros(sh) for k in ("kx", "ky", "kz", "diag", "rhs")}
        rc = _lib.pb_copy_coeffs(self.h, _ptr(sol), *(_ptr(arrs[k]) for k in ("kx", "ky", "kz", "diag", "rhs")))
        if rc != PB_OK:
            raise _err(rc)
        arrs["solute"] = sol
        return arrs

    def num_cut(self) -> int:
        return int(_lib.pb_num_cut(self.h))

    def cut(self, fields: bool = False) -> dict:
        m = self.num_cut()
        d = dict(key=np.zeros(m, np.int64), alpha=np.zeros(m), rp=np.zeros((m, 3)), np=np.zeros((m, 3)),
                 owner=np.zeros(m, np.int64), wp=np.zeros(m))
        if fields:
            d["F"] = np.zeros(m)
            d["phip"] = np.zeros(m)
        rc = _lib.pb_copy_cut(self.h, _ptr(d["key"]), _ptr(d["alpha"]), _ptr(d["rp"]), _ptr(d["np"]),
                              _ptr(d["owner"]), _ptr(d["wp"]), _ptr(d.get("F")), _ptr(d.get("phip")))
        if rc != PB_OK:
            raise _err(rc)
        return d

    def time_stencil(self, reps: int = 20, fp32: bool = False) -> float:
        ms = C.c_double()
        rc = _lib.pb_time_stencil(self.h, int(reps), 1 if fp32 else 0, C.byref(ms))
        if rc != PB_OK:
            raise _err(rc)
        return float(ms.value)

    def profile(self) -> dict:
        a, b, n = C.c_double(), C.c_double(), C.c_int32()
        rc = _lib.pb_get_profile(self.h, C.byref(a), C.byref(b), C.byref(n))
        if rc != PB_OK:
            raise _err(rc)
        return dict(stencil_ms=a.value, update_ms=b.value, samples=n.value)

    def energy_profile(self) -> dict:
        a, b = C.c_double(), C.c_double()
        rc = _lib.pb_get_energy_profile(self.h, C.byref(a), C.byref(b))
        if rc != PB_OK:
            raise _err(rc)
        return dict(nbody_ms=a.value, nbody_pairs=b.value)

    def nbytes(self) -> int:
        return int(_lib.pb_problem_bytes(self.h))

    def close(self):
        if getattr(self, "h", None):
            _lib.pb_problem_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching serving loop (mixed form).  Iteration runs on ``ctx``'s stream,
    builds and energy read-backs on a second context with its own stream."""

    def __init__(self, ctx: Context, build_ctx: Context, max_resident: int = 64):
        load()
        self.ctx, self.build_ctx = ctx, build_ctx
        h = C.c_void_p()
        rc = _lib.pb_server_create(ctx.h, build_ctx.h, int(max_resident), C.byref(h))
        if rc != PB_OK:
            raise _err(rc)
        self.h = h
        ctx._users.add(self)
        build_ctx._users.add(self)

    def now(self) -> float:
        return float(_lib.pb_server_now(self.h))

    def submit(self, mol, grid, request_id: int, arrival_s: float | None = None):
        p = make_params(grid)
        keep = None
        if grid.bc == PB_BC_USER:
            keep = np.ascontiguousarray(grid.bc_values, dtype=np.float64).reshape(-1)
            p.bc_values = keep.ctypes.data_as(C.c_void_p)
        xyz = np.ascontiguousarray(mol.xyz, dtype=np.float64).reshape(-1)
        rad = np.ascontiguousarray(mol.radius, dtype=np.float64)
        chg = np.ascontiguousarray(mol.charge, dtype=np.float64)
        t = self.now() if arrival_s is None else float(arrival_s)
        rc = _lib.pb_submit(self.h, C.byref(p), int(mol.n), _ptr(xyz), _ptr(rad), _ptr(chg), int(request_id), t)
        if rc != PB_OK:
            raise _err(rc)

    def step(self):
        a, q = C.c_int32(), C.c_int32()
        rc = _lib.pb_server_step(self.h, C.byref(a), C.byref(q))
        if rc != PB_OK:
            raise _err(rc)
        return a.value, q.value

    def poll(self, max_n: int = 1024) -> list:
        ids = np.zeros(max_n, np.uint64)
        res = (PbEnergyOut * max_n)()
        sts = (PbSolveStats * max_n)()
        tdone = np.zeros(max_n)
        codes = np.zeros(max_n, np.int32)
        n = C.c_int32()
        rc = _lib.pb_poll(self.h, _ptr(ids), res, sts, _ptr(tdone), _ptr(codes), max_n, C.byref(n))
        if rc != PB_OK:
            raise _err(rc)
        out = []
        for i in range(n.value):
            d = {k: getattr(res[i], k) for k, _ in PbEnergyOut._fields_}
            d.update(iters=sts[i].iters, outer_iters=sts[i].outer_iters, status=sts[i].status, relres=sts[i].relres)
            d.update(id=int(ids[i]), done_s=float(tdone[i]), code=int(codes[i]))
            out.append(d)
        return out

    def profile(self) -> dict:
        a, b, n = C.c_double(), C.c_double(), C.c_int64()
        rc = _lib.pb_server_profile(self.h, C.byref(a), C.byref(b), C.byref(n))
        if rc != PB_OK:
            raise _err(rc)
        out = dict(stencil_ms=a.value, stencil_bytes=b.value, launches=n.value)
        c, d, e, m = C.c_double(), C.c_double(), C.c_double(), C.c_int64()
        rc = _lib.pb_server_profile_mg(self.h, C.byref(c), C.byref(d), C.byref(e), C.byref(m))
        if rc != PB_OK:
            raise _err(rc)
        out.update(mg_sweep_ms=c.value, mg_sweep_bytes=d.value, mg_vcycle_ms=e.value, mg_samples=m.value)
        f, g, k = C.c_double(), C.c_double(), C.c_int64()
        rc = _lib.pb_server_profile_energy(self.h, C.byref(f), C.byref(g), C.byref(k))
        if rc != PB_OK:
            raise _err(rc)
        out.update(nbody_ms=f.value, nbody_pairs=g.value, nbody_calls=k.value)
        a, b, n = C.c_double(), C.c_double(), C.c_int64()
        rc = _lib.pb_server_profile_mg_apply(self.h, C.byref(a), C.byref(b), C.byref(n))
        if rc != PB_OK:
            raise _err(rc)
        out.update(mg_apply_ms=a.value, mg_apply_bytes=b.value, mg_apply_launches=n.value)
        return out

    def cancel(self, request_id: int):
        rc = _lib.pb_cancel(self.h, int(request_id))
        if rc != PB_OK:
            raise _err(rc)

    def set_timeout(self, seconds: float):
        rc = _lib.pb_server_set_timeout(self.h, float(seconds))
        if rc != PB_OK:
            raise _err(rc)

    def memory(self) -> dict:
        a, b, c = C.c_size_t(), C.c_size_t(), C.c_int64()
        rc = _lib.pb_server_memory(self.h, C.byref(a), C.byref(b), C.byref(c))
        if rc != PB_OK:
            raise _err(rc)
        return dict(in_use=int(a.value), peak=int(b.value), over_budget=int(c.value))

    def times(self) -> dict:
        v = np.zeros(4)
        rc = _lib.pb_server_times(self.h, _ptr(v))
        if rc != PB_OK:
            raise _err(rc)
        return dict(wait=v[0], retire=v[1], admit=v[2], launch=v[3])

    def close(self):
        if getattr(self, "h", None):
            _lib.pb_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve(mol, grid, ctx: Context | None = None, per_atom: bool = False) -> dict:
    """Build, solve and read back the energy of one problem."""
    own = ctx is None
    ctx = ctx or Context()
    pb = Problem(ctx, mol, grid)
    try:
        st = pb.solve()
        en = pb.energy(per_atom=per_atom)
        en.update(st)
        en.update(pb.energy_profile())
        return en
    finally:
        pb.close()
        if own:
            ctx.close()
