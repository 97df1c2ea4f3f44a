"""Seeded synthetic inputs for the linearized Poisson-Boltzmann grid solve.

This module only draws random molecules and grid descriptions. It holds none of
the method's arithmetic (no geometry tests, no operator, no energies), so that the
GPU path and the CPU oracle can both be fed from it without sharing any code.

Molecules follow the paper's model of a solute as a union of charged atom balls
(Sect. 2.1): centres are drawn by rejection sampling inside a ball of radius
``sphere_R`` with a minimum pair distance, radii are uniform, and partial charges
are normal and then shifted so that the net charge is an integer.

Random draws happen in a fixed order: candidate centres (batches of 4096 points,
three uniforms each, in [-R, R]^3), then radii, then charges.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Boundary-condition codes and precision codes (same values as the C header).
BC_ZERO, BC_DH, BC_USER = 0, 1, 2
FP64, MIXED = 0, 1
JACOBI, MG = 0, 1            # preconditioners


@dataclass
class Molecule:
    xyz: np.ndarray      # (N, 3) float64, Angstrom
    radius: np.ndarray   # (N,) float64, Angstrom
    charge: np.ndarray   # (N,) float64, units of e

    @property
    def n(self) -> int:
        return int(self.radius.shape[0])


@dataclass
class GridSpec:
    n: tuple             # nodes per axis (nx, ny, nz)
    h: float             # spacing, Angstrom
    origin: tuple        # coordinates of node (0, 0, 0), Angstrom
    eps_in: float = 2.0
    eps_out: float = 80.0
    ionic_M: float = 0.145
    temp_K: float = 298.0
    bc: int = BC_DH
    rtol: float = 1e-10
    max_iter: int = 20000
    tile_planes: int = 0      # planes per x-chunk of the GPU iteration tiles (0 = automatic)
    refine: int = 0           # 1: one level of 2:1 local refinement near the surface;
                              # 2: the grid is a coarse far field, refined around the solute
    refine_shell: float = 3.0 # refine coarse cells within this distance of a crossing point
                              # (refine 1) or of the solute's extent (refine 2)
    refine_brick: int = 4     # ... rounded up to aligned bricks of this many cells per edge
    precision: int = FP64
    inner_rtol: float = 1e-4
    precond: int = 0          # 0: Jacobi, 1: multigrid V-cycle (red-black Gauss-Seidel smoothing)
    mg_smooth: int = 1        # multigrid: sweeps before and after the coarse correction
    mg_coarse_sweeps: int = 4 # multigrid: symmetric sweeps on the coarsest level
    mg_levels: int = 0        # multigrid: level cap (0 = as many as the grid allows)
    bc_values: np.ndarray | None = field(default=None, repr=False)  # BC_USER: full grid

    @property
    def nodes(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])

    @property
    def unknowns(self) -> int:
        return (int(self.n[0]) - 2) * (int(self.n[1]) - 2) * (int(self.n[2]) - 2)


def random_molecule(n_atoms: int, sphere_R: float, seed: int,
                    min_dist: float = 1.0, r_lo: float = 1.2, r_hi: float = 2.0,
                    q_sigma: float = 0.4, center=(0.0, 0.0, 0.0)) -> Molecule:
    """Rejection-sampled synthetic molecule (seeded, PCG64)."""
    rng = np.random.default_rng(seed)
    cell = min_dist
    grid: dict = {}
    acc = np.empty((n_atoms, 3))
    na = 0
    md2 = min_dist * min_dist
    R2 = sphere_R * sphere_R
    while na < n_atoms:
        cand = rng.uniform(-sphere_R, sphere_R, size=(4096, 3))
        for c in cand:
            if na >= n_atoms:
                break
            if c[0] * c[0] + c[1] * c[1] + c[2] * c[2] > R2:
                continue
            key = (int(math.floor(c[0] / cell)), int(math.floor(c[1] / cell)),
                   int(math.floor(c[2] / cell)))
            ok = True
            for dx in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dz in (-1, 0, 1):
                        lst = grid.get((key[0] + dx, key[1] + dy, key[2] + dz))
                        if not lst:
                            continue
                        for idx in lst:
                            d = acc[idx] - c
                            if d[0] * d[0] + d[1] * d[1] + d[2] * d[2] < md2:
                                ok = False
                                break
                        if not ok:
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                continue
            acc[na] = c
            grid.setdefault(key, []).append(na)
            na += 1
    radius = rng.uniform(r_lo, r_hi, size=n_atoms)
    charge = rng.normal(0.0, q_sigma, size=n_atoms)
    net = charge.sum()
    charge = charge - (net - np.round(net)) / n_atoms   # np.round: half to even
    xyz = acc + np.asarray(center, dtype=np.float64)[None, :]
    return Molecule(np.ascontiguousarray(xyz), np.ascontiguousarray(radius),
                    np.ascontiguousarray(charge))


def sphere_cluster(n: int, seed: int, r_lo: float = 1.5, r_hi: float = 2.5, gap: float = 1.0,
                   q_sigma: float = 1.0, n_neutral_top: int = 3) -> Molecule:
    """Non-overlapping charged spheres grown as an aggregate without symmetry (the paper's
    many-sphere benchmark, Sect. 5: one central charge per sphere, the spheres with the
    largest z left uncharged).  Sphere 0 sits at the origin; each later sphere is placed next
    to a randomly chosen earlier one, at a centre distance of the two radii plus
    gap * U[1, 1.5] in a uniformly random direction, and is kept only if it stays at least
    ``gap`` from every other sphere.  Draw order: all radii, then per attempt (parent index,
    direction as three normals, distance factor), then the charges; the ``n_neutral_top``
    spheres of largest z then get charge 0."""
    rng = np.random.default_rng(seed)
    radius = rng.uniform(r_lo, r_hi, size=n)
    xyz = np.zeros((n, 3))
    k = 1
    while k < n:
        par = int(rng.integers(0, k))
        v = rng.normal(size=3)
        f = rng.uniform(1.0, 1.5)
        c = xyz[par] + v / np.linalg.norm(v) * (radius[par] + radius[k] + gap * f)
        d = np.linalg.norm(xyz[:k] - c, axis=1)
        if np.all(d >= radius[:k] + radius[k] + gap):
            xyz[k] = c
            k += 1
    charge = rng.normal(0.0, q_sigma, size=n)
    if n_neutral_top > 0:
        charge[np.argsort(xyz[:, 2])[-n_neutral_top:]] = 0.0
    return Molecule(np.ascontiguousarray(xyz), np.ascontiguousarray(radius), np.ascontiguousarray(charge))


def single_charge_sphere(R: float = 2.0, q: float = 1.0, center=(0.0, 0.0, 0.0)) -> Molecule:
    return Molecule(np.array([center], dtype=np.float64), np.array([R]), np.array([q]))


def cubic_grid(n: int, h: float, center=(0.0, 0.0, 0.0), **kw) -> GridSpec:
    """Cubic grid of n^3 nodes with spacing h centred on ``center``."""
    half = 0.5 * (n - 1) * h
    origin = tuple(float(c) - half for c in center)
    return GridSpec(n=(n, n, n), h=h, origin=origin, **kw)


# --- the five workloads -------------------------------------------------------

def kirkwood_c1(**kw):
    """One +1 e charge at the centre of a 2 A sphere; 65^3 nodes at 0.25 A."""
    mol = single_charge_sphere()
    g = cubic_grid(65, 0.25, **kw)
    return mol, g


def protein_c2(seed: int = 2502, **kw):
    """2,000-atom synthetic molecule in a 20 A ball; 161^3 nodes at 0.5 A."""
    mol = random_molecule(2000, 20.0, seed)
    return mol, cubic_grid(161, 0.5, **kw)


def refined_c3(seed: int = 2503, **kw):
    """20,000-atom molecule in a 45 A ball; coarse 193^3 nodes at 1.0 A, refined to 0.5 A
    within 3 A of the surface (bricks of 4^3 coarse cells)."""
    mol = random_molecule(20000, 45.0, seed)
    kw.setdefault("refine", 1)
    kw.setdefault("refine_shell", 3.0)
    kw.setdefault("refine_brick", 4)
    return mol, cubic_grid(193, 1.0, **kw)


def large_c4(seed: int = 2504, **kw):
    """60,000-atom molecule in a 65 A ball; 385^3 nodes at 0.5 A."""
    mol = random_molecule(60000, 65.0, seed)
    return mol, cubic_grid(385, 0.5, **kw)


def serving_sizes(n_atoms: int, h: float):
    """Placement-ball radius and cubic node count for a serving request."""
    Rs = 20.0 * (n_atoms / 2000.0) ** (1.0 / 3.0)
    cells = 32 * math.ceil(4.0 * Rs / (32.0 * h))
    cells = min(max(cells, 64), 256)
    return Rs, cells + 1


def serving_stream_c5(n_req: int = 512, seed: int = 2505, rate_hz: float = 1.0, **kw):
    """Request list for the serving stream: (arrival_s, molecule, grid).

    Atom counts are log-uniform in [200, 20000], spacings uniform in
    {0.5, 0.75, 1.0} A; arrivals are a Poisson process of the given rate.
    Per-request molecules use seed ``seed * 100003 + k``.
    """
    rng = np.random.default_rng(seed)
    logn = rng.uniform(math.log(200.0), math.log(20000.0), size=n_req)
    hs = rng.choice(np.array([0.5, 0.75, 1.0]), size=n_req)
    gaps = rng.exponential(1.0 / rate_hz, size=n_req)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for k in range(n_req):
        na = int(round(math.exp(logn[k])))
        Rs, n = serving_sizes(na, float(hs[k]))
        mol = random_molecule(na, Rs, seed * 100003 + k)
        out.append((float(t[k]), mol, cubic_grid(n, float(hs[k]), **kw)))
    return out


# --- binding energies (complex and parts) --------------------------------------

def binding_complex(seed: int, n_rec: int = 1500, n_lig: int = 250, R_rec: float = 18.0, R_lig: float = 8.0,
                    gap: float = 1.0):
    """A synthetic receptor-ligand pair and their complex: two molecules generated in balls
    whose centres are R_rec + R_lig + gap apart along x (atom centres of the two parts at
    least gap apart; their spheres overlap across the interface), the complex being the union
    of their atoms.  Returns (complex, receptor, ligand), centred on the complex's bounding
    box."""
    rec = random_molecule(n_rec, R_rec, 2 * seed + 1)
    lig = random_molecule(n_lig, R_lig, 2 * seed + 2, center=(R_rec + R_lig + gap, 0.0, 0.0))
    xyz = np.concatenate([rec.xyz, lig.xyz])
    rad = np.concatenate([rec.radius, lig.radius])
    lo = (xyz - rad[:, None]).min(axis=0)
    hi = (xyz + rad[:, None]).max(axis=0)
    shift = -0.5 * (lo + hi)
    rec = Molecule(rec.xyz + shift, rec.radius, rec.charge)
    lig = Molecule(lig.xyz + shift, lig.radius, lig.charge)
    cpx = Molecule(np.ascontiguousarray(np.concatenate([rec.xyz, lig.xyz])), np.ascontiguousarray(rad),
                   np.ascontiguousarray(np.concatenate([rec.charge, lig.charge])))
    return cpx, rec, lig


def shifted(mol: Molecule, d) -> Molecule:
    return Molecule(np.ascontiguousarray(mol.xyz + np.asarray(d, dtype=np.float64)[None, :]), mol.radius, mol.charge)


def binding_grid(cpx: Molecule, h: float, margin: float = 8.0, **kw) -> GridSpec:
    """One cubic grid for a complex and its parts: the complex's extent plus a margin on every
    side, cells rounded up to a multiple of 32."""
    ext = float(((cpx.xyz + cpx.radius[:, None]).max(axis=0) - (cpx.xyz - cpx.radius[:, None]).min(axis=0)).max())
    cells = 32 * math.ceil((ext + 2.0 * margin) / (32.0 * h))
    return cubic_grid(cells + 1, h, **kw)


def binding_workload(n_complex: int = 6, n_disp: int = 30, h: float = 0.5, seed: int = 2506, **kw):
    """The binding-energy protocol of the paper on synthetic complexes: for each complex, the
    solute's centroid is displaced n_disp times uniformly within a cube of half the grid
    spacing (the same displacement for the complex and its parts, the grid fixed), and each
    displacement needs three solves.  Returns a list of (complex index, displacement index,
    part 'c' | '1' | '2', molecule, grid)."""
    rng = np.random.default_rng(seed)
    out = []
    for c in range(n_complex):
        cpx, rec, lig = binding_complex(seed * 1000 + c)
        grid = binding_grid(cpx, h, **kw)
        for k in range(n_disp):
            d = rng.uniform(-0.25 * h, 0.25 * h, size=3)
            for part, mol in (("c", cpx), ("1", rec), ("2", lig)):
                out.append((c, k, part, shifted(mol, d), grid))
    return out
