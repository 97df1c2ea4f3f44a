"""Pins of the refined-grid oracle (one level of 2:1 refinement with hanging nodes).

CPU only.  Each pin fixes a different part, so that a plausible mistake fails one of them:

* refinement rule      -> brute force over every cell and crossing point on tiny grids
* hanging constraints,
  mixed-size assembly  -> patch test: with one permittivity and no ions the constrained
                          finite-element space reproduces a linear potential exactly
                          (a wrong parent weight or a missing half-cell edge breaks it)
* operator, load, CG,
  flux on the fine
  lattice              -> Born polarization energy to solver tolerance (discrete Gauss
                          law) with the charge in a coarse cell inside the molecule
* assembly in general  -> dense direct solve equals Jacobi-CG
* surface terms        -> Kirkwood ionic energy within the paper's error band; energies
                          close to the uniform fine-grid solve, surface sums identical
"""
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from oracle import refined as R
from paper_2502_09323_amd import inputs as I

GOLD = os.path.join(os.path.dirname(__file__), "golden", "kirkwood_table1.txt")


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build()


def brute_refine(grid, rp, delta, brick):
    """The refinement rule written out cell by cell."""
    n = [int(v) for v in grid.n]
    nc = [v - 1 for v in n]
    H, o = float(grid.h), grid.origin
    flag = np.zeros(nc, bool)
    for i in range(nc[0]):
        for j in range(nc[1]):
            for k in range(nc[2]):
                lo = np.array([o[0] + H * i, o[1] + H * j, o[2] + H * k])
                hi = lo + H
                d = np.maximum(0.0, np.maximum(lo - rp, rp - hi))
                if ((d * d).sum(axis=1) <= delta * delta).any():
                    flag[i, j, k] = True
    out = np.zeros(nc, bool)
    for i in range(nc[0]):
        for j in range(nc[1]):
            for k in range(nc[2]):
                bi, bj, bk = i // brick, j // brick, k // brick
                out[i, j, k] = flag[bi * brick:(bi + 1) * brick, bj * brick:(bj + 1) * brick,
                                    bk * brick:(bk + 1) * brick].any()
    return out


@pytest.mark.parametrize("delta,brick", [(0.6, 1), (1.3, 2), (0.0, 3)])
def test_refinement_rule_matches_brute_force(delta, brick):
    mol = I.random_molecule(8, 1.6, 17)
    grid = I.cubic_grid(15, 0.5)
    fg = R.fine_grid(grid)
    cut = O.cut_edges(fg, mol, O.classify(fg, mol))
    got = R.refine_cells(grid, cut.rp, delta, brick).astype(bool)
    assert got.any()
    np.testing.assert_array_equal(got, brute_refine(grid, cut.rp, delta, brick))


def test_patch_test_linear_potential_is_reproduced():
    mol = I.random_molecule(12, 2.0, 5)
    mol.charge[:] = 0.0
    n, h = 25, 0.5
    grid = I.cubic_grid(n, h, eps_in=1.0, eps_out=1.0, ionic_M=0.0, bc=I.BC_USER)
    lin = lambda X, Y, Z: 0.3 * X - 0.7 * Y + 0.45 * Z + 1.1  # noqa: E731
    ax = [grid.origin[d] + h * np.arange(n) for d in range(3)]
    grid.bc_values = lin(*np.meshgrid(*ax, indexing="ij"))
    run = R.refined_run(mol, grid, delta=0.6, brick=2, rtol=1e-14)
    assert run.hanging.size > 1000 and 0 < run.refined.sum() < run.refined.size
    fg = run.fgrid
    axf = [grid.origin[d] + fg.h * np.arange(fg.n[d]) for d in range(3)]
    want = lin(*np.meshgrid(*axf, indexing="ij"))
    m = ~np.isnan(run.phi)
    assert np.abs(run.phi[m] - want[m]).max() < 1e-11


def test_born_on_refined_grid_with_coarse_interior():
    mol = I.single_charge_sphere(R=3.0, q=1.0, center=(0.13, -0.07, 0.21))
    grid = I.cubic_grid(41, 0.5)
    run = R.refined_run(mol, grid, delta=0.75, brick=2, rtol=1e-12)
    # the charge sits in an unrefined coarse cell, inside a refined shell
    c = [int(math.floor((mol.xyz[0, d] - grid.origin[d]) / grid.h)) for d in range(3)]
    assert not run.refined[c[0], c[1], c[2]] and run.hanging.size > 0
    lB, _ = O.constants(grid.temp_K, grid.ionic_M, grid.eps_out)
    born = 0.5 * lB * (1.0 / grid.eps_out - 1.0 / grid.eps_in) / 3.0
    assert abs(run.energy["e_pol"] / born - 1.0) < 1e-10
    assert abs(run.energy["q_pol_total"] - (1.0 / grid.eps_out - 1.0 / grid.eps_in)) < 1e-10


def test_dense_direct_matches_pcg():
    mol = I.random_molecule(6, 1.5, 3)
    grid = I.cubic_grid(21, 0.5)
    a = R.refined_run(mol, grid, delta=0.5, brick=2, solver="dense")
    b = R.refined_run(mol, grid, delta=0.5, brick=2, rtol=1e-13)
    assert a.hanging.size > 0
    for k in ("e_pol", "e_ion"):
        assert abs(a.energy[k] - b.energy[k]) <= 1e-10 * abs(a.energy[k])


def test_kirkwood_refined_within_paper_band():
    gold = {}
    for line in open(GOLD):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()
            gold[k] = float(v)
    mol = I.single_charge_sphere(2.0)
    grid = I.cubic_grid(33, 0.5, temp_K=298.15)
    run = R.refined_run(mol, grid, delta=1.0, brick=2, rtol=1e-12)
    lB, kD = O.constants(298.15, 0.145, 80.0)
    e_pol = 0.5 * (1.0 / 80.0 - 1.0 / 2.0) / 2.0 * lB
    e_ion = -0.5 / 80.0 * kD / (1.0 + kD * 2.0) * lB
    assert abs(run.energy["e_pol"] / e_pol - 1.0) < 1e-10
    # fine spacing 0.25 A at the surface: better than the paper's 3.4% at 0.5 A
    err = abs(run.energy["e_ion"] / e_ion - 1.0)
    assert err < gold["ngpb_relerr_ion"] * 1.5


def test_refined_close_to_uniform_fine_grid():
    mol = I.random_molecule(40, 3.0, 11)
    grid = I.cubic_grid(33, 0.5)
    r = R.refined_run(mol, grid, delta=1.0, brick=2, rtol=1e-12)
    u = O.run(mol, R.fine_grid(grid), rtol=1e-12)
    # the same fine lattice at the surface: identical cut points and areas
    assert r.energy["n_cut"] == u.energy["n_cut"]
    assert r.energy["area_total"] == u.energy["area_total"]
    # only the far field is coarser
    assert abs(r.energy["e_pol"] / u.energy["e_pol"] - 1.0) < 3e-3
    assert abs(r.energy["e_ion"] / u.energy["e_ion"] - 1.0) < 2e-2


def test_box_rule_covers_the_widened_extent_in_aligned_bricks():
    """De-refinement toward the box: the refined cells are whole aligned bricks, they hold every
    cell that meets the solute's extent widened by delta, and every refined brick meets it."""
    mol = I.random_molecule(20, 3.0, 23, center=(0.3, -0.4, 0.2))
    grid = I.cubic_grid(33, 1.0, bc=I.BC_ZERO)
    delta, brick = 1.5, 3
    lo, hi = R.solute_extent(mol)
    ref = R.refine_cells_box(grid, lo, hi, delta, brick).astype(bool)
    nc = ref.shape
    H, o = grid.h, grid.origin
    meets = np.ones(nc, bool)
    for d in range(3):
        c = np.arange(nc[d])
        ok = (o[d] + H * (c + 1) >= lo[d] - delta) & (o[d] + H * c <= hi[d] + delta)
        sh = [1, 1, 1]
        sh[d] = nc[d]
        meets &= ok.reshape(sh)
    assert meets.any() and np.all(ref[meets])
    for bi in range(0, nc[0], brick):
        for bj in range(0, nc[1], brick):
            for bk in range(0, nc[2], brick):
                blk = ref[bi:bi + brick, bj:bj + brick, bk:bk + brick]
                assert blk.all() or not blk.any()
                if blk.any():
                    assert meets[bi:bi + brick, bj:bj + brick, bk:bk + brick].any()


def test_derefined_zero_bc_kirkwood():
    """The paper's box treatment with one level: a fine region around the sphere, a coarse far
    field and null Dirichlet values on a far box.  E_pol is exact for any box (discrete Gauss
    law); E_ion approaches the uniform fine grid on the same box and improves as the box grows."""
    gold = {}
    for line in open(GOLD):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()
            gold[k] = float(v)
    mol = I.single_charge_sphere(2.0, center=(0.13, -0.07, 0.21))
    lB, kD = O.constants(298.15, 0.145, 80.0)
    e_pol = 0.5 * (1.0 / 80.0 - 1.0 / 2.0) / 2.0 * lB
    e_ion = -0.5 / 80.0 * kD / (1.0 + kD * 2.0) * lB
    errs = []
    for n in (21, 41):
        grid = I.cubic_grid(n, 1.0, temp_K=298.15, bc=I.BC_ZERO)
        run = R.refined_run(mol, grid, delta=2.0, brick=2, rtol=1e-12, mode="box")
        assert 0 < run.refined.sum() < run.refined.size
        assert abs(run.energy["e_pol"] / e_pol - 1.0) < 1e-10
        errs.append(abs(run.energy["e_ion"] / e_ion - 1.0))
    assert errs[1] < 0.5 * errs[0] and errs[1] < 2.0 * gold["ngpb_relerr_ion"]
    # against the uniform h = 0.5 grid on the same 40 A box
    u = O.run(mol, I.cubic_grid(81, 0.5, temp_K=298.15, bc=I.BC_ZERO), rtol=1e-12)
    assert abs(run.energy["e_ion"] / u.energy["e_ion"] - 1.0) < 0.02


def test_two_level_preconditioner_is_symmetric_positive_definite():
    """The two-level preconditioner of the composite operator, as a dense matrix on a small
    refined problem: symmetric, positive definite, and w D^-1 A inside the smoother's bound."""
    mol = I.single_charge_sphere(1.5, center=(0.13, -0.07, 0.21))
    grid = I.cubic_grid(13, 1.0, temp_K=298.15)
    run = R.refined_run(mol, grid, delta=0.5, brick=2, rtol=1e-8)
    pre = R.TwoLevel(run.A, grid, mol, run.free, run.fgrid.n)
    n = run.A.shape[0]
    assert 200 < n < 3000
    Bm = np.column_stack([pre.apply(np.eye(n)[:, i]) for i in range(n)])
    assert np.abs(Bm - Bm.T).max() <= 1e-12 * np.abs(Bm).max()
    assert np.linalg.eigvalsh(0.5 * (Bm + Bm.T)).min() > 0.0
    d = run.A.diagonal()
    lam = np.linalg.eigvalsh((run.A.toarray() / np.sqrt(d)[:, None]) / np.sqrt(d)[None, :]).max()
    assert pre.OMEGA * lam < 2.0


@pytest.mark.parametrize("case", ["sphere", "molecule", "derefined"])
def test_two_level_pcg_matches_jacobi_in_fewer_iterations(case):
    if case == "sphere":
        mol, grid, mode = I.single_charge_sphere(2.0, center=(0.13, -0.07, 0.21)), I.cubic_grid(25, 1.0, temp_K=298.15), "surface"
    elif case == "molecule":
        mol, grid, mode = I.random_molecule(30, 3.0, 7), I.cubic_grid(25, 1.0), "surface"
    else:
        mol, grid, mode = I.random_molecule(30, 3.0, 7), I.cubic_grid(29, 1.0, bc=I.BC_ZERO), "box"
    a = R.refined_run(mol, grid, delta=1.5, brick=2, rtol=1e-12, mode=mode)
    b = R.refined_run(mol, grid, delta=1.5, brick=2, rtol=1e-12, mode=mode, solver="mg")
    assert b.status == 0 and 4 * b.iters <= a.iters
    for k in ("e_pol", "e_ion"):
        assert abs(b.energy[k] - a.energy[k]) <= 1e-10 * abs(a.energy[k]), k
    ok = np.isfinite(a.phi)
    assert np.abs(b.phi[ok] - a.phi[ok]).max() <= 1e-9 * np.abs(a.phi[ok]).max()
