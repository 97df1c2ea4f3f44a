"""Multigrid-preconditioned CG on the GPU against the multigrid oracle.

Element by element: one V-cycle on the same right-hand side (FP64 1e-12, FP32 1e-5 of the
largest entry) on several hierarchies -- a cubic grid with five levels, a ragged grid whose
coarsening stops at a different depth per axis, one level (red-black symmetric Gauss-Seidel),
and a large one-level grid whose coarsest solve runs over many blocks.  The solve: the
potential and energies against the oracle's (FP64 1e-10 / 1e-9, mixed 1e-6) with the
oracle's iteration count; the 161^3 molecule against the GPU's Jacobi-CG solution and the
discrete Gauss law.
"""
from dataclasses import replace

import numpy as np
import pytest

from oracle import mg as M
from oracle import oracle as O
from paper_2502_09323_amd import binding as B
from paper_2502_09323_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    B.load()
    c = B.Context(0)
    yield c
    c.close()


def _vcycle_cases():
    mol = I.random_molecule(40, 3.0, 11)
    return [
        ("cubic33", mol, I.cubic_grid(33, 0.5, precond=I.MG), 5),
        ("ragged", I.random_molecule(25, 2.5, 4),
         I.GridSpec(n=(33, 25, 41), h=0.5, origin=(-8.0, -6.0, -10.0), bc=I.BC_ZERO, precond=I.MG), 4),
        ("one_level", mol, I.cubic_grid(33, 0.5, precond=I.MG, mg_levels=1, mg_coarse_sweeps=1), 1),
        ("nu2_cs7", mol, I.cubic_grid(33, 0.5, precond=I.MG, mg_smooth=2, mg_coarse_sweeps=7, mg_levels=3), 3),
        ("large_one_level", mol, I.cubic_grid(36, 0.5, precond=I.MG, mg_coarse_sweeps=2), 1),
    ]


@pytest.mark.parametrize("name,mol,grid,nlev", _vcycle_cases(), ids=[c[0] for c in _vcycle_cases()])
@pytest.mark.parametrize("prec", [I.FP64, I.MIXED], ids=["fp64", "mixed"])
def test_vcycle_parity(ctx, name, mol, grid, nlev, prec):
    grid = replace(grid, precision=prec)
    levels = M.hierarchy(M.fine_level(grid, mol), grid.mg_levels)
    assert len(levels) == nlev
    rng = np.random.default_rng(7)
    r = np.zeros(levels[0].n)
    r[levels[0].interior] = rng.standard_normal(int(levels[0].interior.sum()))
    if prec == I.MIXED:
        r = r.astype(np.float32).astype(np.float64)
    want = M.vcycle(levels, r, nu=grid.mg_smooth, coarse_sweeps=grid.mg_coarse_sweeps)
    pb = B.Problem(ctx, mol, grid)
    try:
        z, nl = pb.mg_vcycle(r)
        assert nl == nlev
        tol = 1e-12 if prec == I.FP64 else 1e-5
        scale = np.abs(want).max()
        assert np.abs(z - want).max() <= tol * scale, (np.abs(z - want).max() / scale)
        assert not z[~levels[0].interior].any()
    finally:
        pb.close()


def _solve_cases():
    return [
        ("molecule_dh", I.random_molecule(40, 3.0, 11), I.cubic_grid(33, 0.5, precond=I.MG)),
        ("ragged_zero_bc", I.random_molecule(25, 2.5, 4),
         I.GridSpec(n=(33, 25, 41), h=0.5, origin=(-8.0, -6.0, -10.0), bc=I.BC_ZERO, precond=I.MG)),
        ("kirkwood65", I.single_charge_sphere(2.0), I.cubic_grid(65, 0.25, precond=I.MG, temp_K=298.15)),
    ]


@pytest.mark.parametrize("name,mol,grid", _solve_cases(), ids=[c[0] for c in _solve_cases()])
def test_mg_solve_parity_fp64(ctx, name, mol, grid):
    grid = replace(grid, rtol=1e-12)
    ref = M.run(mol, grid, rtol=1e-12)
    pb = B.Problem(ctx, mol, grid)
    try:
        st = pb.solve()
        assert st["status"] == 0 and st["relres"] <= 1e-12
        assert abs(st["iters"] - ref.iters) <= 1
        en = pb.energy()
        for k in ("e_pol", "e_ion", "q_pol_total", "area_total"):
            assert abs(en[k] - ref.energy[k]) <= 1e-10 * max(abs(ref.energy[k]), 1e-12), (k, en[k], ref.energy[k])
        phi = pb.potential()
        want = ref.lB * ref.phi
        assert np.abs(phi - want).max() <= 1e-9 * np.abs(want).max()
    finally:
        pb.close()


@pytest.mark.parametrize("name,mol,grid", _solve_cases()[:2], ids=[c[0] for c in _solve_cases()[:2]])
def test_mg_solve_parity_mixed(ctx, name, mol, grid):
    grid = replace(grid, precision=I.MIXED, rtol=1e-10, inner_rtol=1e-2)
    ref = M.run(mol, replace(grid, precision=I.FP64), rtol=1e-12)
    pb = B.Problem(ctx, mol, grid)
    try:
        st = pb.solve()
        assert st["status"] == 0 and st["relres"] <= 1e-10 and st["outer_iters"] >= 1
        en = pb.energy()
        for k in ("e_pol", "e_ion", "q_pol_total"):
            assert abs(en[k] - ref.energy[k]) <= 1e-6 * abs(ref.energy[k]), (k, en[k], ref.energy[k])
        want = ref.lB * ref.phi
        assert np.abs(pb.potential() - want).max() <= 1e-6 * np.abs(want).max()
    finally:
        pb.close()


def test_mg_full_size_161(ctx):
    """The 161^3 2000-atom molecule: six levels; the solution equals the Jacobi-CG one and
    satisfies the discrete Gauss law."""
    mol, grid = I.protein_c2(rtol=1e-10)
    a = B.Problem(ctx, mol, grid)
    b = B.Problem(ctx, mol, replace(grid, precond=I.MG))
    c = B.Problem(ctx, mol, replace(grid, precond=I.MG, precision=I.MIXED, inner_rtol=1e-2))
    try:
        sa, sb, sc = a.solve(), b.solve(), c.solve()
        assert sa["status"] == 0 and sb["status"] == 0 and sc["status"] == 0
        assert sb["iters"] * 8 < sa["iters"]
        ea, eb, ec = a.energy(), b.energy(), c.energy()
        for k in ("e_pol", "e_ion"):
            assert abs(eb[k] - ea[k]) <= 1e-8 * abs(ea[k]), k
            assert abs(ec[k] - ea[k]) <= 1e-6 * abs(ea[k]), k
        q = float(mol.charge.sum())
        assert abs(eb["q_pol_total"] - (1.0 / grid.eps_out - 1.0 / grid.eps_in) * q) <= 1e-8 * max(abs(q), 1.0)
        _, nl = b.mg_vcycle(np.zeros(b.shape))
        assert nl == 6
    finally:
        a.close()
        b.close()
        c.close()


def test_mg_invalid(ctx):
    mol = I.random_molecule(10, 2.0, 1)
    for g in (I.cubic_grid(33, 0.5, precond=2),
              I.cubic_grid(33, 0.5, precond=I.MG, mg_smooth=9), I.cubic_grid(33, 0.5, precond=I.MG, mg_levels=13)):
        with pytest.raises(B.PbError) as e:
            B.Problem(ctx, mol, g)
        assert e.value.code == B.PB_EINVAL
    pb = B.Problem(ctx, mol, I.cubic_grid(17, 0.5))
    try:
        with pytest.raises(B.PbError) as e:
            pb.mg_vcycle(np.zeros(pb.shape))
        assert e.value.code == B.PB_EINVAL
    finally:
        pb.close()
