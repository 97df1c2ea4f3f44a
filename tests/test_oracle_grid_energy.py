"""Pins of the oracle's grid energy (Sect. 3.3, electrostatic energy: half the sum of the
charges mapped onto the grid nodes times the potential there), and of the two-run estimate
of the salt contribution built on it.

- Trilinear deposition is a partition of unity that reproduces linear functions: on a
  constant or linear potential the grid energy is half the sum of q_i times that potential
  at the atom centres, exactly.
- A charge on a node sees only that node.
- Kirkwood sphere with the exact box values at both ionic strengths: the polarization energy
  of a central charge does not depend on the salt, so G(I) - G(0) is the closed-form ionic
  energy of Sect. 6.1.1 (the Kirkwood sphere) up to a discretization error that falls at second order in h.
- A molecule: G(I) - G(0) is the change of the solvation energy with the salt, and agrees
  with the same change from the surface read-back (E_pol + E_ion at I, minus E_pol at 0) to
  within the two methods' discretization errors.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2502_09323_amd import inputs as I

from test_oracle_pins import born_kirkwood, kirkwood_bc


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build()


def _node_coords(grid):
    axes = [grid.origin[d] + grid.h * np.arange(grid.n[d]) for d in range(3)]
    return np.meshgrid(*axes, indexing="ij")


def test_grid_energy_of_constant_and_linear_potentials():
    mol = I.random_molecule(40, 4.0, 5)
    grid = I.cubic_grid(29, 0.5)
    lB = 0.731
    X, Y, Z = _node_coords(grid)
    ref_q = 0.5 * lB * float(mol.charge.sum())
    assert abs(O.grid_energy(grid, mol, np.ones(tuple(grid.n)), lB) - ref_q) <= 1e-12 * max(1.0, abs(ref_q))
    a, c = np.array([0.3, -1.7, 0.9]), 2.5
    phi = a[0] * X + a[1] * Y + a[2] * Z + c
    ref = 0.5 * lB * float(np.dot(mol.charge, mol.xyz @ a + c))
    assert abs(O.grid_energy(grid, mol, phi, lB) - ref) <= 1e-13 * 0.5 * lB * np.abs(mol.charge).sum() * np.abs(phi).max()


def test_charge_on_a_node_sees_that_node_only():
    grid = I.cubic_grid(11, 0.5)
    mol = I.Molecule(np.array([[0.5, -1.0, 1.5]]), np.array([1.5]), np.array([-2.0]))
    phi = np.random.default_rng(3).normal(size=tuple(grid.n))
    # the node at (0.5, -1.0, 1.5) is (6, 3, 8) with the origin at -2.5
    assert O.grid_energy(grid, mol, phi, 1.0) == pytest.approx(0.5 * -2.0 * phi[6, 3, 8], rel=1e-14)


def test_two_run_kirkwood_gives_the_closed_form_ionic_energy():
    lB, kD = O.constants(298.15, 0.145, 80.0)
    _, e_ion = born_kirkwood(lB, kD)
    errs = []
    for n, h in [(33, 0.5), (65, 0.25)]:
        mol = I.single_charge_sphere()
        g = {}
        for ion in (0.145, 0.0):
            grid = I.cubic_grid(n, h, temp_K=298.15)
            grid.ionic_M = ion
            grid.bc = I.BC_USER
            grid.bc_values = kirkwood_bc(grid, O.constants(298.15, ion, 80.0)[1])
            run = O.run(mol, grid, rtol=1e-12)
            assert run.status == 0
            g[ion] = O.grid_energy(grid, mol, run.phi, run.lB)
        errs.append(abs((g[0.145] - g[0.0]) / e_ion - 1.0))
    assert errs[0] < 5e-3 and errs[1] < 1.5e-3
    assert errs[1] < errs[0] / 2.5


def test_two_run_matches_the_change_of_solvation_energy():
    mol = I.random_molecule(60, 5.0, 1)
    g, solv = {}, {}
    for ion in (0.145, 0.0):
        grid = I.cubic_grid(65, 0.5, temp_K=300.0)
        grid.ionic_M = ion
        run = O.run(mol, grid, rtol=1e-12)
        assert run.status == 0
        g[ion] = O.grid_energy(grid, mol, run.phi, run.lB)
        solv[ion] = run.energy["e_solv"]
    d_grid = g[0.145] - g[0.0]
    d_surf = solv[0.145] - solv[0.0]
    assert d_grid < 0.0 and d_surf < 0.0
    assert abs(d_grid - d_surf) <= 0.02 * abs(d_surf)
    # the self-energy that cancels in the difference is far larger than the difference
    assert abs(g[0.0]) > 100 * abs(d_grid)
    assert math.isfinite(g[0.0])
