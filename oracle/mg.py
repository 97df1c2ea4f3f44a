"""Multigrid-preconditioned CG for the PBE operator: the plain FP64 oracle.

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and the CPU-baseline leg of ``bench.py``.
The product path never imports it, and it imports nothing from the product package.

The paper solves its linear systems with CG and an SSOR preconditioner (Sect. 4, solver
structure).  This module defines the stronger preconditioner the GPU solver offers in its
place: one symmetric V-cycle of geometric multigrid on the uniform grid, smoothed by
red-black Gauss-Seidel.  Everything below is a definition written out plainly over
full-grid arrays (shape (nx, ny, nz), z contiguous; box nodes hold 0 in every correction):

* operator       the assembled 7-point operator as node fields: K[ax] at node (i,j,k) is the
                 weight of the edge to the next node along ax, m the lumped ionic term
                 (``oracle.edge_coeffs``); (A x)_v = sum_edges K (x_v - x_nbr) + m_v x_v at
                 interior nodes
* colours        node (i,j,k) is red when i+j+k is even, black otherwise; every neighbour
                 of a red node is black, so a half-sweep over one colour is exact
                 Gauss-Seidel
* coarse grids   node I of the coarse grid is fine node 2I (needs n-1 even on every axis);
                 a coarse edge joins two coarse nodes 2h apart: along the edge the two fine
                 edges are in series (K1 K2 / (K1 + K2)); across it the 3 x 3 fine lines
                 around it are averaged with weights (1/4, 1/2, 1/4) per axis and the sum
                 is multiplied by 4 (the coarse dual face holds four fine ones), so a
                 constant coefficient gives the 2h operator (2h eps); the coarse ionic term
                 is P^T m (the row sums of P^T M P)
* transfers      P = trilinear interpolation (weight 1, 1/2, 1/4 or 1/8 from the coarse
                 corners of the fine node's coarse cell), restriction R = P^T
* V-cycle        zero start; pre-smoothing nu times (red, black); residual; restrict;
                 recurse; add P e; post-smoothing nu times (black, red); the coarsest grid
                 takes ``coarse_sweeps`` symmetric sweeps (red, then (black, red) repeated).
                 Pre- and post-smoothing are adjoint and R = P^T, so the V-cycle is a
                 symmetric positive definite operator and CG may use it as preconditioner.
                 With one level it is red-black symmetric Gauss-Seidel, i.e. SSOR with
                 omega = 1 in red-black order.
* PCG            standard preconditioned CG (z = V-cycle(r)), stopping on the recursive
                 residual ||r|| <= rtol ||b|| like the Jacobi oracle
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

from . import oracle as O


@dataclass
class Level:
    n: tuple            # nodes per axis
    h: float
    K: list             # [Kx, Ky, Kz] full-grid edge weights
    m: np.ndarray       # lumped ionic term
    D: np.ndarray       # diagonal at interior nodes (1 elsewhere)
    interior: np.ndarray  # bool mask of the unknowns
    red: np.ndarray       # bool mask of red unknowns
    black: np.ndarray     # bool mask of black unknowns


def _masks(n):
    inner = np.zeros(n, bool)
    inner[1:-1, 1:-1, 1:-1] = True
    i, j, k = np.meshgrid(*[np.arange(v) for v in n], indexing="ij")
    even = ((i + j + k) % 2) == 0
    return inner, inner & even, inner & ~even


def make_level(n, h, K, m) -> Level:
    n = tuple(int(v) for v in n)
    inner, red, black = _masks(n)
    Kx, Ky, Kz = K
    D = np.zeros(n)
    # sum of the six edge weights of each node, then the ionic term
    D[1:-1, 1:-1, 1:-1] = (Kx[:-2, 1:-1, 1:-1] + Kx[1:-1, 1:-1, 1:-1] + Ky[1:-1, :-2, 1:-1] + Ky[1:-1, 1:-1, 1:-1]
                           + Kz[1:-1, 1:-1, :-2] + Kz[1:-1, 1:-1, 1:-1] + m[1:-1, 1:-1, 1:-1])
    D[~inner] = 1.0
    return Level(n, float(h), [Kx, Ky, Kz], m, D, inner, red, black)


def fine_level(grid, mol) -> Level:
    """The operator of the paper's discretization (the one ``oracle.run`` assembles)."""
    lB, kD = O.constants(grid.temp_K, grid.ionic_M, grid.eps_out)
    sol = O.classify(grid, mol)
    cut = O.cut_edges(grid, mol, sol)
    Kx, Ky, Kz, m = O.edge_coeffs(grid, sol, cut, grid.eps_out * kD * kD)
    return make_level(grid.n, grid.h, [Kx, Ky, Kz], m)


def neighbour_sum(L: Level, x: np.ndarray) -> np.ndarray:
    """sum over the six edges of K * x(neighbour), at interior nodes (0 elsewhere)."""
    Kx, Ky, Kz = L.K
    s = np.zeros(L.n)
    c = (slice(1, -1),) * 3
    s[c] = (Kx[:-2, 1:-1, 1:-1] * x[:-2, 1:-1, 1:-1] + Kx[1:-1, 1:-1, 1:-1] * x[2:, 1:-1, 1:-1]
            + Ky[1:-1, :-2, 1:-1] * x[1:-1, :-2, 1:-1] + Ky[1:-1, 1:-1, 1:-1] * x[1:-1, 2:, 1:-1]
            + Kz[1:-1, 1:-1, :-2] * x[1:-1, 1:-1, :-2] + Kz[1:-1, 1:-1, 1:-1] * x[1:-1, 1:-1, 2:])
    return s


def apply(L: Level, x: np.ndarray) -> np.ndarray:
    """A x at the interior nodes (x is 0 on the box); 0 on the box."""
    y = L.D * x - neighbour_sum(L, x)
    y[~L.interior] = 0.0
    return y


def half_sweep(L: Level, x: np.ndarray, b: np.ndarray, colour: np.ndarray) -> None:
    """Gauss-Seidel on the nodes of one colour: x_v = (b_v + sum K x_nbr) / D_v."""
    s = neighbour_sum(L, x)
    x[colour] = (b[colour] + s[colour]) / L.D[colour]


def can_coarsen(n) -> bool:
    return all((v - 1) % 2 == 0 and (v - 1) // 2 + 1 >= 3 for v in n)


def _series(a, b):
    t = a + b
    out = np.zeros_like(t)
    nz = t > 0
    out[nz] = a[nz] * b[nz] / t[nz]
    return out


W3 = {-1: 0.25, 0: 0.5, 1: 0.25}


def coarsen(L: Level) -> Level:
    """The coarse level: series along each coarse edge, weighted average across it (x4),
    and P^T m for the ionic term."""
    nf = L.n
    nc = tuple((v - 1) // 2 + 1 for v in nf)
    Kc = []
    for ax in range(3):
        Kf = L.K[ax]
        K = np.zeros(nc)
        # coarse edges from I to I+1 along ax, for coarse nodes with both transverse
        # indices inside the box (edges on the box faces join two box nodes: unused)
        t1, t2 = [a for a in range(3) if a != ax]
        lo = [0, 0, 0]
        hi = list(nc)
        hi[ax] = nc[ax] - 1
        lo[t1], lo[t2] = 1, 1
        hi[t1], hi[t2] = nc[t1] - 1, nc[t2] - 1
        acc = np.zeros(tuple(hi[d] - lo[d] for d in range(3)))
        for a in (-1, 0, 1):
            for b in (-1, 0, 1):
                sl1, sl2 = [], []
                for d in range(3):
                    I = np.arange(lo[d], hi[d])
                    if d == ax:
                        f1, f2 = 2 * I, 2 * I + 1
                    else:
                        off = a if d == t1 else b
                        f1 = f2 = 2 * I + off
                    sl1.append(f1)
                    sl2.append(f2)
                k1 = Kf[np.ix_(*sl1)]
                k2 = Kf[np.ix_(*sl2)]
                acc += W3[a] * W3[b] * _series(k1, k2)
        K[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]] = 4.0 * acc
        Kc.append(K)
    mc = restrict(L, nc, L.m)
    return make_level(nc, 2.0 * L.h, Kc, mc)


def restrict(Lf: Level, nc, r: np.ndarray) -> np.ndarray:
    """P^T r: coarse interior node I gathers the fine nodes 2I + (a,b,c), a,b,c in {-1,0,1},
    with weight prod (1 if a == 0 else 1/2)."""
    out = np.zeros(nc)
    I = [np.arange(1, v - 1) for v in nc]
    for a in (-1, 0, 1):
        for b in (-1, 0, 1):
            for c in (-1, 0, 1):
                w = (1.0 if a == 0 else 0.5) * (1.0 if b == 0 else 0.5) * (1.0 if c == 0 else 0.5)
                out[1:-1, 1:-1, 1:-1] += w * r[np.ix_(2 * I[0] + a, 2 * I[1] + b, 2 * I[2] + c)]
    return out


def prolong(nf, e: np.ndarray) -> np.ndarray:
    """P e: trilinear interpolation of the coarse values onto the fine grid (box: 0)."""
    out = np.zeros(nf)
    # per axis: fine index f takes coarse f/2 (even f) or the mean of (f-1)/2 and (f+1)/2
    idx = []
    for v in nf:
        f = np.arange(v)
        lo = f // 2
        hi = (f + 1) // 2
        idx.append((lo, hi))
    for sa in (0, 1):
        for sb in (0, 1):
            for sc in (0, 1):
                w = 0.125
                out += w * e[np.ix_(idx[0][sa], idx[1][sb], idx[2][sc])]
    inner = np.zeros(nf, bool)
    inner[1:-1, 1:-1, 1:-1] = True
    out[~inner] = 0.0
    return out


def hierarchy(L0: Level, max_levels: int = 0) -> list:
    levels = [L0]
    while can_coarsen(levels[-1].n) and (max_levels <= 0 or len(levels) < max_levels):
        levels.append(coarsen(levels[-1]))
    return levels


def vcycle(levels: list, b: np.ndarray, nu: int = 1, coarse_sweeps: int = 4, lev: int = 0) -> np.ndarray:
    """One symmetric V-cycle from a zero start: returns an approximation of A^-1 b."""
    L = levels[lev]
    x = np.zeros(L.n)
    if lev == len(levels) - 1:
        half_sweep(L, x, b, L.red)
        for _ in range(coarse_sweeps):
            half_sweep(L, x, b, L.black)
            half_sweep(L, x, b, L.red)
        return x
    for _ in range(nu):
        half_sweep(L, x, b, L.red)
        half_sweep(L, x, b, L.black)
    r = b - apply(L, x)
    r[~L.interior] = 0.0
    Lc = levels[lev + 1]
    e = vcycle(levels, restrict(L, Lc.n, r), nu, coarse_sweeps, lev + 1)
    x += prolong(L.n, e)
    for _ in range(nu):
        half_sweep(L, x, b, L.black)
        half_sweep(L, x, b, L.red)
    return x


def mg_pcg(levels: list, b: np.ndarray, rtol: float, max_iter: int = 10000, nu: int = 1,
           coarse_sweeps: int = 4):
    """PCG with one V-cycle as preconditioner on the full-grid right-hand side b (0 on the
    box).  Returns (x, iterations, relres, status 0 converged / 1 not)."""
    L = levels[0]
    x = np.zeros(L.n)
    r = b.copy()
    r[~L.interior] = 0.0
    bn = np.linalg.norm(r)
    if bn == 0.0:
        return x, 0, 0.0, 0
    z = vcycle(levels, r, nu, coarse_sweeps)
    p = z.copy()
    gamma = float(np.sum(r * z))
    for it in range(1, max_iter + 1):
        q = apply(L, p)
        alpha = gamma / float(np.sum(p * q))
        x += alpha * p
        r -= alpha * q
        rn = np.linalg.norm(r)
        if rn <= rtol * bn:
            return x, it, rn / bn, 0
        z = vcycle(levels, r, nu, coarse_sweeps)
        g2 = float(np.sum(r * z))
        p = z + (g2 / gamma) * p
        gamma = g2
    return x, max_iter, float(np.linalg.norm(r)) / bn, 1


def run(mol, grid, rtol: float = 1e-12, max_iter: int = 10000, nu: int = 1, coarse_sweeps: int = 4,
        max_levels: int = 0, want_energy: bool = True):
    """The oracle's pipeline (geometry, load, box values, energies) with MG-PCG in place of
    Jacobi-PCG.  Returns an ``oracle.OracleRun``."""
    t0 = time.perf_counter()
    lB, kD = O.constants(grid.temp_K, grid.ionic_M, grid.eps_out)
    sol = O.classify(grid, mol)
    cut = O.cut_edges(grid, mol, sol)
    g = O.boundary_values(grid, mol, kD)
    Kx, Ky, Kz, m = O.edge_coeffs(grid, sol, cut, grid.eps_out * kD * kD)
    L0 = make_level(grid.n, grid.h, [Kx, Ky, Kz], m)
    levels = hierarchy(L0, max_levels)
    # load and Dirichlet lift: b = deposit + sum over edges to box nodes of K g
    gb = g.copy()
    gb[L0.interior] = 0.0
    b = O.deposit(grid, mol) + neighbour_sum(L0, gb)
    b[~L0.interior] = 0.0
    t1 = time.perf_counter()
    x, it, rr, st = mg_pcg(levels, b, rtol, max_iter, nu, coarse_sweeps)
    t2 = time.perf_counter()
    phi = g.copy()
    phi[L0.interior] = x[L0.interior]
    en = O.energies(grid, mol, sol, cut, phi, lB) if want_energy else {}
    t3 = time.perf_counter()
    run = O.OracleRun(lB, kD, sol, cut, None, b, g, phi, it, rr, st, en,
                      dict(build=t1 - t0, solve=t2 - t1, energy=t3 - t2))
    run.levels = levels
    return run
