"""Locally refined grids for the CPU oracle: one level of 2:1 refinement with hanging nodes.

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` (and nothing in the product path).  It
imports nothing from the product package.

The paper discretizes on a Cartesian octree with hierarchical refinement and treats the
non-conforming (hanging) nodes as in its references (Sect. 3, before Sect. 3.1); the
discrete operator of Sect. 3.1 (eq. matrixequation) is assembled cell by cell.  This module
builds that discrete problem for one refinement level:

* mesh.  Coarse cells of size H over the box; a coarse cell is split into 2x2x2 fine cells
  of size h = H/2 when a surface crossing point of the fine lattice lies within
  ``delta`` of the cell, rounded up to aligned bricks of ``brick``^3 coarse cells (the
  rule implemented by ``orc_refine_cells`` in ``oracle.c``).  Every mesh vertex is a node
  of the fine lattice (spacing h, 2n-1 nodes per axis); coarse node (i,j,k) is fine node
  (2i,2j,2k).
* operator.  Every cell of size s adds (s/4) eps_e to the Laplacian of each of its 12 edges
  and (s^3/8) kbar^2 to the diagonal at each of its 8 vertices (vertex quadrature).  A fine
  edge crossing the surface takes the weighted harmonic average of eq. WHA; coarse edges
  never cross the surface (cells around a crossing are refined).
* hanging nodes.  A fine vertex that is not a coarse node and lies on the boundary of an
  unrefined coarse cell is constrained to the mean of the coarse nodes at the ends of the
  coarse edge (2 parents) or at the corners of the coarse face (4 parents) it lies on:
  the trilinear interpolant of the coarse cell.  With P the map from free values to all
  vertex values, the system matrix is P^T K P and the load P^T b (Dirichlet box nodes
  eliminated as in the uniform case).
* load.  A charge deposits trilinearly on the corners of the cell that contains it: the
  fine cell inside a refined coarse cell, the coarse cell otherwise.
* energy.  All cut edges lie inside the refined region, where the energy read-back of
  Sect. 3.3 runs on the fine lattice exactly as on a uniform grid of spacing h.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, replace

import numpy as np

from oracle import oracle as O


def fine_grid(grid):
    """The fine lattice: spacing h/2, 2n-1 nodes per axis, same origin and physics."""
    return replace(grid, n=tuple(2 * int(v) - 1 for v in grid.n), h=float(grid.h) / 2.0)


def refine_cells(grid, rp: np.ndarray, delta: float, brick: int) -> np.ndarray:
    """uint8 flags over the coarse cells, shape (nx-1, ny-1, nz-1)."""
    n = O._n(grid)
    out = np.zeros(tuple(int(v) - 1 for v in grid.n), dtype=np.uint8)
    L = O.lib()
    import ctypes as C
    L.orc_refine_cells.argtypes = [C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_int32, C.c_int64,
                                   C.c_void_p, C.c_void_p]
    L.orc_refine_cells.restype = C.c_int64
    rpc = np.ascontiguousarray(rp, dtype=np.float64).reshape(-1, 3)
    cnt = L.orc_refine_cells(O._p(n), O._p(O._o(grid)), float(grid.h), float(delta), int(brick),
                             rpc.shape[0], O._p(rpc), O._p(out))
    if cnt < 0:
        raise MemoryError("orc_refine_cells")
    return out


def refine_cells_box(grid, lo, hi, delta: float, brick: int) -> np.ndarray:
    """De-refinement toward the box (the paper's Sect. 3.4, exploiting de-refinement for more efficient BCs): every coarse cell that
    meets the box [lo - delta, hi + delta] on all three axes is split (lo, hi: the solute's
    extent, atom centres -/+ radii), rounded up to aligned bricks like refine_cells; the rest
    of the domain, out to the box where the null Dirichlet values are applied, stays coarse."""
    nc = [int(v) - 1 for v in grid.n]
    H = float(grid.h)
    flag = np.ones(nc, bool)
    for d in range(3):
        c = np.arange(nc[d])
        blo = grid.origin[d] + H * c
        bhi = grid.origin[d] + H * (c + 1)
        ok = (bhi >= lo[d] - delta) & (blo <= hi[d] + delta)
        shape = [1, 1, 1]
        shape[d] = nc[d]
        flag &= ok.reshape(shape)
    out = np.zeros(nc, np.uint8)
    nb = [(v + brick - 1) // brick for v in nc]
    bf = np.zeros(nb, bool)
    idx = np.argwhere(flag)
    bf[idx[:, 0] // brick, idx[:, 1] // brick, idx[:, 2] // brick] = True
    I, J, K = np.meshgrid(*[np.arange(v) for v in nc], indexing="ij")
    out[...] = bf[I // brick, J // brick, K // brick]
    return out


def solute_extent(mol):
    lo = (mol.xyz - mol.radius[:, None]).min(axis=0)
    hi = (mol.xyz + mol.radius[:, None]).max(axis=0)
    return lo, hi


_AX = np.eye(3, dtype=np.int64)


def _edges_of_cells(corner0: np.ndarray, step: int):
    """(u, v, axis) fine coordinates of the 12 edges of cells with low corner corner0."""
    us, vs, axs = [], [], []
    for a in range(3):
        o1, o2 = [d for d in range(3) if d != a]
        for b in (0, 1):
            for c in (0, 1):
                off = np.zeros(3, np.int64)
                off[o1] = b * step
                off[o2] = c * step
                u = corner0 + off
                us.append(u)
                vs.append(u + step * _AX[a])
                axs.append(np.full(u.shape[0], a, np.int64))
    return np.concatenate(us), np.concatenate(vs), np.concatenate(axs)


def _corners_of_cells(corner0: np.ndarray, step: int) -> np.ndarray:
    return np.concatenate([corner0 + step * np.array([x, y, z], np.int64)
                           for x in (0, 1) for y in (0, 1) for z in (0, 1)])


@dataclass
class RefinedRun:
    lB: float
    kD: float
    refined: np.ndarray      # coarse-cell flags
    fgrid: object            # fine lattice GridSpec
    solute: np.ndarray       # fine-lattice media
    cut: O.CutEdges          # fine-lattice cut edges
    A: object                # P^T K P over the free vertices
    b: np.ndarray
    free: np.ndarray         # fine-lattice ids of the free vertices, in unknown order
    hanging: np.ndarray      # fine-lattice ids of the hanging vertices
    phi: np.ndarray          # fine lattice, NaN where there is no mesh vertex
    iters: int
    relres: float
    status: int
    energy: dict
    times: dict


def refined_run(mol, grid, delta: float = 3.0, brick: int = 4, rtol: float = 1e-12, max_iter: int = 100000,
                solver: str = "pcg", want_energy: bool = True, mode: str = "surface") -> RefinedRun:
    """Geometry -> refinement -> constrained assembly -> load -> solve -> energies."""
    t0 = time.perf_counter()
    lB, kD = O.constants(grid.temp_K, grid.ionic_M, grid.eps_out)
    kb2 = float(grid.eps_out) * kD * kD
    H = float(grid.h)
    h = H / 2.0
    n = np.array([int(v) for v in grid.n], np.int64)
    fg = fine_grid(grid)
    nf = np.array([int(v) for v in fg.n], np.int64)
    NF = int(nf.prod())

    sol = O.classify(fg, mol)
    cut = O.cut_edges(fg, mol, sol)
    if mode == "box":
        lo, hi = solute_extent(mol)
        ref = refine_cells_box(grid, lo, hi, delta, brick).astype(bool)
    else:
        ref = refine_cells(grid, cut.rp, delta, brick).astype(bool)
    if ref[0].any() or ref[-1].any() or ref[:, 0].any() or ref[:, -1].any() or ref[:, :, 0].any() or ref[:, :, -1].any():
        raise ValueError("refined cells touch the box boundary layer")

    def fid(c):
        return (c[:, 0] * nf[1] + c[:, 1]) * nf[2] + c[:, 2]

    solf = sol.reshape(-1).astype(bool)
    ei, eo = float(grid.eps_in), float(grid.eps_out)

    # unrefined coarse cells
    cc = np.argwhere(~ref).astype(np.int64) * 2
    u, v, a = _edges_of_cells(cc, 2)
    iu, iv = fid(u), fid(v)
    if (solf[iu] != solf[iv]).any():
        raise AssertionError("a coarse edge crosses the surface")
    w_c = (H / 4.0) * np.where(solf[iu], ei, eo)
    cor_c = fid(_corners_of_cells(cc, 2))
    m_c = (H ** 3 / 8.0) * kb2 * (~solf[cor_c])

    # fine cells of the refined coarse cells
    rc = np.argwhere(ref).astype(np.int64) * 2
    fc = np.concatenate([rc + np.array([x, y, z], np.int64) for x in (0, 1) for y in (0, 1) for z in (0, 1)])
    fu, fv, fa = _edges_of_cells(fc, 1)
    jf, jv = fid(fu), fid(fv)
    key = 3 * jf + fa
    pos = np.searchsorted(cut.key, key)
    pos_c = np.minimum(pos, max(cut.m - 1, 0))
    is_cut = (cut.m > 0) & (cut.key[pos_c] == key) if cut.m > 0 else np.zeros(key.shape, bool)
    alpha = np.where(is_cut, cut.alpha[pos_c] if cut.m > 0 else 0.0, 0.0)
    eps_e = np.where(is_cut, 1.0 / (alpha / ei + (1.0 - alpha) / eo), np.where(solf[jf], ei, eo))
    if (~is_cut & (solf[jf] != solf[jv])).any():
        raise AssertionError("an edge with endpoints in different media is not in the cut list")
    w_f = (h / 4.0) * eps_e
    cor_f = fid(_corners_of_cells(fc, 1))
    m_f = (h ** 3 / 8.0) * kb2 * (~solf[cor_f])

    import scipy.sparse as sp
    eu = np.concatenate([iu, jf])
    ev = np.concatenate([iv, jv])
    ew = np.concatenate([w_c, w_f])
    cor = np.concatenate([cor_c, cor_f])
    mass = np.concatenate([m_c, m_f])
    rows = np.concatenate([eu, ev, eu, ev, cor])
    cols = np.concatenate([eu, ev, ev, eu, cor])
    vals = np.concatenate([ew, ew, -ew, -ew, mass])
    K = sp.coo_matrix((vals, (rows, cols)), shape=(NF, NF)).tocsr()

    # every cut edge must be interior to the refined region (four refined fine cells)
    if cut.m:
        kk = cut.key // 3
        ax = cut.key % 3
        fi = np.stack([kk // (nf[1] * nf[2]), (kk // nf[2]) % nf[1], kk % nf[2]], axis=1)
        ok = np.ones(cut.m, bool)
        o1 = np.where(ax == 0, 1, 0)   # the two axes across the edge
        o2 = np.where(ax == 2, 1, 2)
        for s1 in (0, 1):
            for s2 in (0, 1):
                c = fi.copy()
                c[np.arange(cut.m), o1] -= s1
                c[np.arange(cut.m), o2] -= s2
                inside = (c >= 0).all(axis=1) & (c < nf - 1).all(axis=1)
                cc2 = np.clip(c // 2, 0, n - 2)
                ok &= inside & ref[cc2[:, 0], cc2[:, 1], cc2[:, 2]]
        if not ok.all():
            raise AssertionError("a cut edge touches an unrefined cell")

    # vertices, box nodes, hanging nodes
    verts = np.unique(np.concatenate([cor_c, cor_f]))
    vc = np.stack([verts // (nf[1] * nf[2]), (verts // nf[2]) % nf[1], verts % nf[2]], axis=1)
    box = ((vc == 0) | (vc == nf - 1)).any(axis=1)
    odd = (vc % 2) == 1
    hang = np.zeros(verts.shape[0], bool)
    anyodd = odd.any(axis=1)
    # coarse cells whose closed box holds the vertex: odd axis -> (f-1)/2, even -> f/2-1 or f/2
    for s in range(8):
        cidx = np.empty_like(vc)
        valid = anyodd.copy()
        for d in range(3):
            side = (s >> d) & 1
            cand = np.where(odd[:, d], (vc[:, d] - 1) // 2, vc[:, d] // 2 - 1 + side)
            valid &= ~(odd[:, d] & (side == 1))   # an odd axis has a single candidate
            valid &= (cand >= 0) & (cand <= n[d] - 2)
            cidx[:, d] = np.clip(cand, 0, n[d] - 2)
        hang |= valid & ~ref[cidx[:, 0], cidx[:, 1], cidx[:, 2]]
    free = verts[~hang & ~box]
    hanging = verts[hang]
    nfree = free.shape[0]
    idx = -np.ones(NF, np.int64)
    idx[free] = np.arange(nfree)

    # P: free vertices map to themselves, hanging vertices to the mean of their parents
    hc = vc[hang]
    hodd = (hc % 2) == 1
    nodd = hodd.sum(axis=1)
    rank = np.cumsum(hodd, axis=1) - 1        # order of each odd axis among the node's odd axes
    pr, pc, pv = [free], [np.arange(nfree)], [np.ones(nfree)]
    for s in range(4):
        use = s < (1 << nodd)
        bit = (s >> np.maximum(rank, 0)) & 1
        par = np.where(hodd, hc - 1 + 2 * bit, hc)
        pid = fid(par[use])
        if (idx[pid] < 0).any():
            raise AssertionError("a hanging node has a parent that is not free")
        pr.append(hanging[use])
        pc.append(idx[pid])
        pv.append(1.0 / (1 << nodd[use]))
    P = sp.coo_matrix((np.concatenate(pv), (np.concatenate(pr), np.concatenate(pc))), shape=(NF, nfree)).tocsr()

    # Dirichlet values on the box (coarse nodes)
    gcoarse = O.boundary_values(grid, mol, kD)
    gfull = np.zeros(NF)
    bv = verts[box]
    bc = vc[box]
    gfull[bv] = gcoarse[bc[:, 0] // 2, bc[:, 1] // 2, bc[:, 2] // 2]

    # load: trilinear on the corners of the cell holding each charge
    bfull = np.zeros(NF)
    for at in range(mol.n):
        x = mol.xyz[at]
        q = float(mol.charge[at])
        cidx = np.empty(3, np.int64)
        fl = np.empty(3)
        for d in range(3):
            f = (x[d] - grid.origin[d]) / H
            c0 = min(max(math.floor(f), 0), int(n[d]) - 2)
            cidx[d] = c0
        if ref[cidx[0], cidx[1], cidx[2]]:
            step, base = 1, np.empty(3, np.int64)
            t = np.empty(3)
            for d in range(3):
                f = (x[d] - grid.origin[d]) / h
                c1 = min(max(math.floor(f), 2 * int(cidx[d])), 2 * int(cidx[d]) + 1)
                base[d] = c1
                t[d] = f - c1
        else:
            step, base = 2, 2 * cidx
            t = np.empty(3)
            for d in range(3):
                f = (x[d] - grid.origin[d]) / H
                t[d] = f - cidx[d]
        for xx in (0, 1):
            for yy in (0, 1):
                for zz in (0, 1):
                    w = (t[0] if xx else 1 - t[0]) * (t[1] if yy else 1 - t[1]) * (t[2] if zz else 1 - t[2])
                    c = base + step * np.array([xx, yy, zz])
                    bfull[(c[0] * nf[1] + c[1]) * nf[2] + c[2]] += 4.0 * math.pi * q * w

    A = (P.T @ K @ P).tocsr()
    b = P.T @ (bfull - K @ gfull)
    t1 = time.perf_counter()
    if solver == "dense":
        xs = np.linalg.solve(A.toarray(), b)
        it, rr, st = 0, float(np.linalg.norm(b - A @ xs) / max(np.linalg.norm(b), 1e-300)), 0
    elif solver == "mg":
        pre = TwoLevel(A, grid, mol, free, nf)
        xs, it, rr, st = pre.pcg(b, rtol, max_iter)
    else:
        xs, it, rr, st = O.pcg(A, b, rtol, max_iter)
    t2 = time.perf_counter()
    phi = np.full(NF, np.nan)
    vals_v = P @ xs + gfull
    phi[verts] = vals_v[verts]
    phi = phi.reshape(tuple(int(v) for v in nf))
    en = O.energies(fg, mol, sol, cut, phi, lB) if want_energy else {}
    t3 = time.perf_counter()
    return RefinedRun(lB, kD, ref, fg, sol, cut, A, b, free, hanging, phi, it, rr, st, en,
                      dict(build=t1 - t0, solve=t2 - t1, energy=t3 - t2))


# ---- two-level preconditioner for the composite system ------------------------------------

def coarse_interpolation(grid, free: np.ndarray, nf) -> "object":
    """I_H: the trilinear interpolation of the coarse grid (all nodes, flat (i, j, k) order,
    box nodes excluded) to the free vertices: a free vertex at fine-lattice coordinates F takes
    coarse node F/2 with weight 1 along an even axis and nodes (F-1)/2, (F+1)/2 with weight
    1/2 each along an odd one (the product over the axes)."""
    import scipy.sparse as sp
    n = np.array([int(v) for v in grid.n], np.int64)
    nf = np.asarray(nf, np.int64)
    F = np.stack([free // (nf[1] * nf[2]), (free // nf[2]) % nf[1], free % nf[2]], axis=1)
    odd = (F % 2) == 1
    rows, cols, vals = [], [], []
    for s in range(8):
        I = np.empty_like(F)
        w = np.ones(F.shape[0])
        ok = np.ones(F.shape[0], bool)
        for d in range(3):
            bit = (s >> d) & 1
            I[:, d] = np.where(odd[:, d], (F[:, d] - 1) // 2 + bit, F[:, d] // 2)
            ok &= odd[:, d] | (bit == 0)
            w *= np.where(odd[:, d], 0.5, 1.0)
        ok &= ((I > 0) & (I < n - 1)).all(axis=1)
        rows.append(np.nonzero(ok)[0])
        cols.append((I[ok, 0] * n[1] + I[ok, 1]) * n[2] + I[ok, 2])
        vals.append(w[ok])
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(F.shape[0], int(n.prod()))).tocsr()


class TwoLevel:
    """Symmetric two-level preconditioner of the composite operator A (this implementation's,
    like the uniform multigrid; the paper preconditions CG with SSOR, Sect. 4):

        z1 = w D^-1 r,   z2 = z1 + I_H V(I_H^T (r - A z1)),   z = z2 + w D^-1 (r - A z2)

    with D = diag(A), w = 0.8, and V one V-cycle of the uniform multigrid of the coarse grid
    (its operator from the coarse-grid geometry, ``oracle.mg``; nu = grid.mg_smooth or 1,
    coarse_sweeps = grid.mg_coarse_sweeps or 4, levels as grid.mg_levels).  It is
    S + (I - S A) C (I - A S) + S (I - A S) with S = w D^-1 and C = I_H V I_H^T, symmetric,
    and positive definite while w D^-1 A has spectral radius below 2 (about 1.6 here: the
    composite operator is close to diagonally dominant, D^-1 A below 2)."""

    OMEGA = 0.8

    def __init__(self, A, grid, mol, free, nf):
        from oracle import mg as M
        self.M = M
        self.A = A
        self.dinv = 1.0 / A.diagonal()
        self.IH = coarse_interpolation(grid, free, nf)
        self.levels = M.hierarchy(M.fine_level(grid, mol), int(getattr(grid, "mg_levels", 0) or 0))
        self.nu = int(getattr(grid, "mg_smooth", 0) or 1)
        self.cs = int(getattr(grid, "mg_coarse_sweeps", 0) or 4)

    def apply(self, r: np.ndarray) -> np.ndarray:
        w = self.OMEGA
        z = w * self.dinv * r
        bc = (self.IH.T @ (r - self.A @ z)).reshape(self.levels[0].D.shape)
        e = self.M.vcycle(self.levels, bc, self.nu, self.cs)
        z = z + self.IH @ e.reshape(-1)
        return z + w * self.dinv * (r - self.A @ z)

    def pcg(self, b: np.ndarray, rtol: float, max_iter: int):
        """PCG from x = 0, stopping on the recursive residual ||r|| <= rtol ||b||; returns
        (x, iterations, relres, status 0 converged / 1 not)."""
        x = np.zeros_like(b)
        r = b.copy()
        bn = float(np.linalg.norm(b))
        if bn == 0.0:
            return x, 0, 0.0, 0
        z = self.apply(r)
        p = z.copy()
        gamma = float(r @ z)
        for it in range(1, max_iter + 1):
            q = self.A @ p
            alpha = gamma / float(p @ q)
            x += alpha * p
            r -= alpha * q
            rn = float(np.linalg.norm(r))
            if rn <= rtol * bn:
                return x, it, rn / bn, 0
            z = self.apply(r)
            g2 = float(r @ z)
            p = z + (g2 / gamma) * p
            gamma = g2
        return x, max_iter, float(np.linalg.norm(r)) / bn, 1
