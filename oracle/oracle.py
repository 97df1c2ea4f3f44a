"""Python driver of the plain FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py``.  The product path never imports it, and it imports
nothing from the product package.

Each function follows one step of the paper's method (see the header of ``oracle.c``
for the citations).  Arrays on the full node grid have shape (nx, ny, nz) with z
contiguous; the unknowns are the interior nodes in the same lexicographic order.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
import time
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SO = os.path.join(_HERE, "liborc.so")
_lib = None

BC_ZERO, BC_DH, BC_USER = 0, 1, 2


def build() -> str:
    """Compile the oracle into ``oracle/liborc.so`` (always recompiles)."""
    tmp = _SO + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        # PB_ORACLE_LIB names another build of oracle.c (the sanitizer test's)
        path = os.environ.get("PB_ORACLE_LIB") or _SO
        if path == _SO and not os.path.exists(_SO):
            build()
        L = C.CDLL(path)
        P = C.c_void_p
        i64, i32, d = C.c_int64, C.c_int32, C.c_double
        L.orc_constants.argtypes = [d, d, d, P, P]
        L.orc_classify.argtypes = [P, P, d, i64, P, P, P]
        L.orc_count_cut.argtypes = [P, P]
        L.orc_count_cut.restype = i64
        L.orc_cut_edges.argtypes = [P, P, d, i64, P, P, P, i64, P, P, P, P, P]
        L.orc_assemble.argtypes = [P, d, d, d, d, P, i64, P, P, P, P, P, P, P, P]
        L.orc_deposit.argtypes = [P, P, d, i64, P, P, P]
        L.orc_bc_dh.argtypes = [P, P, d, i64, P, P, d, d, P]
        L.orc_pcg.argtypes = [i64, P, P, P, P, P, d, i32, P, P]
        L.orc_mc_weights.argtypes = [P, P, i64, P, P, P]
        L.orc_edge_fields.argtypes = [P, d, d, d, P, i64, P, P, P, P, P]
        L.orc_surface_sums.argtypes = [i64, P, P, i64, P, P, P, P, P, P, P]
        L.orc_edge_coeffs.argtypes = [P, d, d, d, d, P, i64, P, P, P, P, P, P]
        L.orc_coulomb.argtypes = [i64, P, P, d]
        L.orc_coulomb.restype = d
        L.orc_num_threads.restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _n(grid):
    return np.asarray(grid.n, dtype=np.int32)


def _o(grid):
    return np.asarray(grid.origin, dtype=np.float64)


def num_threads() -> int:
    return int(lib().orc_num_threads())


# --- constants ---------------------------------------------------------------

def constants(temp_K: float, ionic_M: float, eps_out: float):
    """(Bjerrum length in Angstrom, kD in 1/Angstrom)."""
    lB = np.zeros(1)
    kd2 = np.zeros(1)
    lib().orc_constants(temp_K, ionic_M, eps_out, _p(lB), _p(kd2))
    return float(lB[0]), math.sqrt(float(kd2[0]))


# --- geometry ------------------------------------------------------------------

def classify(grid, mol) -> np.ndarray:
    n = _n(grid)
    sol = np.zeros(tuple(int(v) for v in grid.n), dtype=np.uint8)
    xyz = np.ascontiguousarray(mol.xyz, dtype=np.float64)
    rad = np.ascontiguousarray(mol.radius, dtype=np.float64)
    rc = lib().orc_classify(_p(n), _p(_o(grid)), float(grid.h), mol.n, _p(xyz), _p(rad), _p(sol))
    if rc != 0:
        raise RuntimeError(f"orc_classify failed ({rc})")
    return sol


@dataclass
class CutEdges:
    key: np.ndarray     # int64, 3 * (low node) + axis, ascending
    alpha: np.ndarray   # fraction of the edge on the solute side
    rp: np.ndarray      # (m, 3) crossing points
    np_: np.ndarray     # (m, 3) outward unit normals
    owner: np.ndarray   # int64 owning atom

    @property
    def m(self) -> int:
        return int(self.key.shape[0])


def cut_edges(grid, mol, solute: np.ndarray) -> CutEdges:
    n = _n(grid)
    sol = np.ascontiguousarray(solute, dtype=np.uint8)
    m = int(lib().orc_count_cut(_p(n), _p(sol)))
    key = np.zeros(m, np.int64)
    alpha = np.zeros(m)
    rp = np.zeros((m, 3))
    nrm = np.zeros((m, 3))
    owner = np.zeros(m, np.int64)
    xyz = np.ascontiguousarray(mol.xyz, dtype=np.float64)
    rad = np.ascontiguousarray(mol.radius, dtype=np.float64)
    rc = lib().orc_cut_edges(_p(n), _p(_o(grid)), float(grid.h), mol.n, _p(xyz), _p(rad),
                             _p(sol), m, _p(key), _p(alpha), _p(rp), _p(nrm), _p(owner))
    if rc != 0:
        raise RuntimeError(f"orc_cut_edges failed ({rc})")
    return CutEdges(key, alpha, rp, nrm, owner)


# --- load, boundary values, assembly --------------------------------------------

def deposit(grid, mol) -> np.ndarray:
    """4 pi sum_i q_i w_n(r_i) on the full grid."""
    b = np.zeros(tuple(int(v) for v in grid.n))
    xyz = np.ascontiguousarray(mol.xyz, dtype=np.float64)
    q = np.ascontiguousarray(mol.charge, dtype=np.float64)
    lib().orc_deposit(_p(_n(grid)), _p(_o(grid)), float(grid.h), mol.n, _p(xyz), _p(q), _p(b))
    return b


def boundary_values(grid, mol, kD: float) -> np.ndarray:
    """Full-grid array whose box-node entries hold the Dirichlet values."""
    shape = tuple(int(v) for v in grid.n)
    if grid.bc == BC_ZERO:
        return np.zeros(shape)
    if grid.bc == BC_USER:
        g = np.array(grid.bc_values, dtype=np.float64).reshape(shape)
        inner = g[1:-1, 1:-1, 1:-1]
        inner[...] = 0.0
        return g
    g = np.zeros(shape)
    xyz = np.ascontiguousarray(mol.xyz, dtype=np.float64)
    q = np.ascontiguousarray(mol.charge, dtype=np.float64)
    lib().orc_bc_dh(_p(_n(grid)), _p(_o(grid)), float(grid.h), mol.n, _p(xyz), _p(q),
                    float(grid.eps_out), float(kD), _p(g))
    return g


def assemble(grid, solute, cut: CutEdges, g_full, kbar2_out: float):
    """Cell-wise assembled CSR matrix over the interior unknowns and the BC lift."""
    import scipy.sparse as sp
    nu = grid.unknowns
    rowptr = np.zeros(nu + 1, np.int64)
    col = np.zeros(7 * nu, np.int64)
    val = np.zeros(7 * nu)
    lift = np.zeros(nu)
    nnz = np.zeros(1, np.int64)
    sol = np.ascontiguousarray(solute, dtype=np.uint8)
    g = np.ascontiguousarray(g_full, dtype=np.float64)
    rc = lib().orc_assemble(_p(_n(grid)), float(grid.h), float(grid.eps_in), float(grid.eps_out),
                            float(kbar2_out), _p(sol), cut.m, _p(cut.key), _p(cut.alpha), _p(g),
                            _p(rowptr), _p(col), _p(val), _p(lift), _p(nnz))
    if rc != 0:
        raise RuntimeError(f"orc_assemble failed ({rc})")
    k = int(nnz[0])
    A = sp.csr_matrix((val[:k].copy(), col[:k].copy(), rowptr), shape=(nu, nu))
    return A, lift


def edge_coeffs(grid, solute, cut: CutEdges, kbar2_out: float):
    """The assembled operator as full-grid fields (Kx, Ky, Kz, m): K[ax] at a node is the
    weight of its edge to the next node along ax, m its lumped ionic term."""
    shape = tuple(int(v) for v in grid.n)
    K = [np.zeros(shape) for _ in range(3)]
    m = np.zeros(shape)
    sol = np.ascontiguousarray(solute, dtype=np.uint8)
    rc = lib().orc_edge_coeffs(_p(_n(grid)), float(grid.h), float(grid.eps_in), float(grid.eps_out),
                               float(kbar2_out), _p(sol), cut.m, _p(cut.key), _p(cut.alpha),
                               _p(K[0]), _p(K[1]), _p(K[2]), _p(m))
    if rc != 0:
        raise RuntimeError(f"orc_edge_coeffs failed ({rc})")
    return K[0], K[1], K[2], m


def interior(a_full: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(a_full[1:-1, 1:-1, 1:-1]).reshape(-1)


def pcg(A, b, rtol: float, max_iter: int = 100000):
    """Jacobi-PCG; returns (x, iters, relres, status)."""
    nu = A.shape[0]
    x = np.zeros(nu)
    it = np.zeros(1, np.int32)
    rr = np.zeros(1)
    indptr = np.ascontiguousarray(A.indptr, dtype=np.int64)
    ind = np.ascontiguousarray(A.indices, dtype=np.int64)
    dat = np.ascontiguousarray(A.data, dtype=np.float64)
    bb = np.ascontiguousarray(b, dtype=np.float64)
    st = lib().orc_pcg(nu, _p(indptr), _p(ind), _p(dat), _p(bb), _p(x), float(rtol),
                       int(max_iter), _p(it), _p(rr))
    return x, int(it[0]), float(rr[0]), int(st)


# --- energies ---------------------------------------------------------------------

def mc_weights(grid, solute, cut: CutEdges) -> np.ndarray:
    wp = np.zeros(cut.m)
    sol = np.ascontiguousarray(solute, dtype=np.uint8)
    rp = np.ascontiguousarray(cut.rp)
    rc = lib().orc_mc_weights(_p(_n(grid)), _p(sol), cut.m, _p(cut.key), _p(rp), _p(wp))
    if rc != 0:
        raise RuntimeError(f"orc_mc_weights failed ({rc})")
    return wp


def edge_fields(grid, solute, cut: CutEdges, phi_full):
    F = np.zeros(cut.m)
    phip = np.zeros(cut.m)
    sol = np.ascontiguousarray(solute, dtype=np.uint8)
    phi = np.ascontiguousarray(phi_full, dtype=np.float64)
    lib().orc_edge_fields(_p(_n(grid)), float(grid.h), float(grid.eps_in), float(grid.eps_out),
                          _p(sol), cut.m, _p(cut.key), _p(cut.alpha), _p(phi), _p(F), _p(phip))
    return F, phip


def surface_sums(mol, cut: CutEdges, F, wp, phip, sel=None):
    sel = np.arange(mol.n, dtype=np.int64) if sel is None else np.asarray(sel, dtype=np.int64)
    SF = np.zeros(sel.shape[0])
    SD = np.zeros(sel.shape[0])
    xyz = np.ascontiguousarray(mol.xyz, dtype=np.float64)
    lib().orc_surface_sums(sel.shape[0], _p(sel), _p(xyz), cut.m, _p(np.ascontiguousarray(cut.rp)),
                           _p(np.ascontiguousarray(cut.np_)), _p(F), _p(wp), _p(phip), _p(SF), _p(SD))
    return SF, SD


def coulomb(mol, eps_in: float) -> float:
    xyz = np.ascontiguousarray(mol.xyz, dtype=np.float64)
    q = np.ascontiguousarray(mol.charge, dtype=np.float64)
    return float(lib().orc_coulomb(mol.n, _p(xyz), _p(q), float(eps_in)))


def energies(grid, mol, solute, cut: CutEdges, phi_full, lB: float, sel=None):
    """Energy components in kT and per-atom reaction potentials in kT/e.

    E_pol = 1/2 lB sum_i q_i (1/eps_out - 1/eps_in) S_F(i)
    E_ion = 1/2 lB sum_i q_i (S_D(i) - S_F(i)/eps_out)
    """
    wp = mc_weights(grid, solute, cut)
    F, phip = edge_fields(grid, solute, cut, phi_full)
    SF, SD = surface_sums(mol, cut, F, wp, phip, sel)
    ei, eo = float(grid.eps_in), float(grid.eps_out)
    q = mol.charge if sel is None else mol.charge[np.asarray(sel)]
    phi_pol = (1.0 / eo - 1.0 / ei) * SF
    phi_ion = SD - SF / eo
    out = dict(
        e_pol=0.5 * lB * float(np.dot(q, phi_pol)),
        e_ion=0.5 * lB * float(np.dot(q, phi_ion)),
        q_pol_total=float((1.0 / eo - 1.0 / ei) * F.sum() / (4.0 * math.pi)),
        area_total=float(wp.sum()),
        n_cut=cut.m,
        phi_reac=lB * (phi_pol + phi_ion),
        phi_pol=lB * phi_pol,
        phi_ion=lB * phi_ion,
        F=F, wp=wp, phip=phip,
    )
    if sel is None:
        out["e_coul"] = lB * coulomb(mol, ei)
        out["e_solv"] = out["e_pol"] + out["e_ion"]
        out["e_total"] = out["e_coul"] + out["e_solv"]
    return out


def grid_energy(grid, mol, phi_full, lB: float) -> float:
    """Grid energy in kT (Sect. 3.3, electrostatic energy): one half of the sum over the grid
    nodes of the fixed charge mapped onto each node times the potential there.  The node
    charges are the right-hand side's deposition divided by 4 pi, on the interior nodes only
    (the right-hand side holds no charge on box nodes).  The difference of two solves of one
    geometry, at the actual ionic strength and at zero, estimates the ionic energy."""
    Q = interior(deposit(grid, mol)) / (4.0 * math.pi)
    return 0.5 * lB * float(np.dot(Q, interior(phi_full)))


# --- the whole pipeline -------------------------------------------------------------

@dataclass
class OracleRun:
    lB: float
    kD: float
    solute: np.ndarray
    cut: CutEdges
    A: object
    b: np.ndarray
    g: np.ndarray
    phi: np.ndarray      # full grid, box nodes hold the Dirichlet values
    iters: int
    relres: float
    status: int
    energy: dict
    times: dict


def run(mol, grid, rtol: float = 1e-12, max_iter: int = 100000, sel=None,
        solver: str = "pcg", want_energy: bool = True) -> OracleRun:
    """Geometry -> assembly -> load -> Jacobi-PCG (or dense solve) -> energies."""
    t0 = time.perf_counter()
    lB, kD = constants(grid.temp_K, grid.ionic_M, grid.eps_out)
    sol = classify(grid, mol)
    cut = cut_edges(grid, mol, sol)
    g = boundary_values(grid, mol, kD)
    A, lift = assemble(grid, sol, cut, g, grid.eps_out * kD * kD)
    b = interior(deposit(grid, mol)) + lift
    t1 = time.perf_counter()
    if solver == "dense":
        x = np.linalg.solve(A.toarray(), b)
        it, rr, st = 0, float(np.linalg.norm(b - A @ x) / max(np.linalg.norm(b), 1e-300)), 0
    else:
        x, it, rr, st = pcg(A, b, rtol, max_iter)
    t2 = time.perf_counter()
    phi = g.copy()
    phi[1:-1, 1:-1, 1:-1] = x.reshape(tuple(int(v) - 2 for v in grid.n))
    en = energies(grid, mol, sol, cut, phi, lB, sel) if want_energy else {}
    t3 = time.perf_counter()
    return OracleRun(lB, kD, sol, cut, A, b, g, phi, it, rr, st, en,
                     dict(build=t1 - t0, solve=t2 - t1, energy=t3 - t2))
