"""The GPU grid energy (Sect. 3.3, electrostatic energy) against the oracle's, and the
two-run estimate of the salt contribution built on it: G(I) - G(0) over two solves of one
geometry on one grid.

- Kirkwood sphere (65^3, h = 0.25 A) with the exact box values at both ionic strengths:
  the difference equals the oracle's to the solver tolerance and the closed-form ionic
  energy to the discretization error the oracle's pin allows.
- A 60-atom molecule: both grid energies match the oracle's.
- The 2,000-atom 161^3 molecule (multigrid, mixed precision): the difference agrees with
  the change of the surface read-back's solvation energy, E_pol + E_ion at I minus E_pol at 0.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2502_09323_amd import binding as B
from paper_2502_09323_amd import inputs as I

from test_oracle_pins import born_kirkwood, kirkwood_bc

pytestmark = pytest.mark.gpu

E_TOL64 = 1e-10
E_TOL_MIXED = 1e-6


@pytest.fixture(scope="module")
def ctx():
    B.load()
    c = B.Context(0)
    yield c
    c.close()


def _gpu_grid_energy(ctx, mol, grid):
    pb = B.Problem(ctx, mol, grid)
    try:
        st = pb.solve()
        assert st["status"] == 0
        return pb.grid_energy(), pb.energy()
    finally:
        pb.close()


@pytest.mark.parametrize("prec", [I.FP64, I.MIXED], ids=["fp64", "mixed"])
def test_two_run_kirkwood(ctx, prec):
    tol = E_TOL64 if prec == I.FP64 else E_TOL_MIXED
    lB, kD = O.constants(298.15, 0.145, 80.0)
    _, e_ion = born_kirkwood(lB, kD)
    mol = I.single_charge_sphere()
    g, ref = {}, {}
    for ion in (0.145, 0.0):
        grid = I.cubic_grid(65, 0.25, temp_K=298.15, precision=prec, rtol=1e-12 if prec == I.FP64 else 1e-10,
                            inner_rtol=1e-4)
        grid.ionic_M = ion
        grid.bc = I.BC_USER
        grid.bc_values = kirkwood_bc(grid, O.constants(298.15, ion, 80.0)[1])
        run = O.run(mol, grid, rtol=1e-12)
        ref[ion] = O.grid_energy(grid, mol, run.phi, run.lB)
        g[ion], _ = _gpu_grid_energy(ctx, mol, grid)
        assert abs(g[ion] - ref[ion]) <= tol * abs(ref[ion])
    d, d_ref = g[0.145] - g[0.0], ref[0.145] - ref[0.0]
    assert abs(d - d_ref) <= tol * abs(ref[0.0])
    assert abs(d / e_ion - 1.0) < 1.5e-3


def test_molecule_grid_energy_parity(ctx):
    mol = I.random_molecule(60, 5.0, 1)
    for ion in (0.145, 0.0):
        grid = I.cubic_grid(65, 0.5, temp_K=300.0, rtol=1e-12)
        grid.ionic_M = ion
        run = O.run(mol, grid, rtol=1e-12)
        ref = O.grid_energy(grid, mol, run.phi, run.lB)
        got, _ = _gpu_grid_energy(ctx, mol, grid)
        assert abs(got - ref) <= E_TOL64 * abs(ref), (ion, got, ref)


def test_two_run_matches_the_change_of_solvation_energy_c2(ctx):
    mol = I.protein_c2()[0]
    g, solv = {}, {}
    for ion in (0.145, 0.0):
        grid = I.protein_c2(rtol=1e-10)[1]
        grid.precond, grid.precision, grid.inner_rtol = I.MG, I.MIXED, 1e-4
        grid.ionic_M = ion
        g[ion], en = _gpu_grid_energy(ctx, mol, grid)
        solv[ion] = en["e_pol"] + en["e_ion"]
    d_grid, d_surf = g[0.145] - g[0.0], solv[0.145] - solv[0.0]
    print("two-run", d_grid, "surface", d_surf, flush=True)
    assert d_grid < 0.0 and d_surf < 0.0
    assert abs(d_grid - d_surf) <= 0.03 * abs(d_surf)


def test_grid_energy_errors(ctx):
    mol = I.random_molecule(20, 3.0, 9)
    pb = B.Problem(ctx, mol, I.cubic_grid(33, 0.5))
    try:
        with pytest.raises(B.PbError) as e:
            pb.grid_energy()
        assert e.value.code == B.PB_EINVAL
    finally:
        pb.close()
    grid = I.cubic_grid(33, 0.5, refine=1, refine_shell=1.0, refine_brick=2)
    pb = B.Problem(ctx, I.random_molecule(40, 3.0, 11), grid)
    try:
        assert pb.solve()["status"] == 0
        with pytest.raises(B.PbError) as e:
            pb.grid_energy()
        assert e.value.code == B.PB_EINVAL
    finally:
        pb.close()
