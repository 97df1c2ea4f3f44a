"""GPU parity of a molecule far from the coordinate origin.

The method is invariant under translation: moving the molecule and the box together moves
the potential with them and leaves every energy unchanged (the energies of Sect. 3.3 depend
only on distances).  The oracle forms every distance as a difference of coordinates, so its
results shift exactly up to the rounding of the shifted inputs; the GPU's energy and box-value
kernels form squared distances in an expanded form, which stays exact to FP64 rounding only
relative to a nearby centre.  These cases check the GPU against the oracle at the FP64 and
mixed-precision tolerances with the molecule and its box moved by hundreds and thousands of
Angstrom."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2502_09323_amd import binding as B
from paper_2502_09323_amd import inputs as I

pytestmark = pytest.mark.gpu

SHIFTS = [(150.0, -90.0, 230.0), (1500.25, -900.5, 2300.75)]


@pytest.fixture(scope="module")
def ctx():
    import torch

    assert torch.cuda.is_available()
    B.load()
    c = B.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("shift", SHIFTS, ids=["shift_300A", "shift_3000A"])
def test_translated_molecule_parity(ctx, shift):
    mol = I.shifted(I.random_molecule(600, 12.0, 31), shift)
    grid = I.cubic_grid(81, 0.4, center=shift, rtol=1e-12)
    print(f"translated parity: shift {shift}, {mol.n} atoms, n {grid.n}", flush=True)
    run = O.run(mol, grid, rtol=1e-12)
    pb = B.Problem(ctx, mol, grid)
    cut = pb.cut()
    assert np.array_equal(cut["key"], run.cut.key) and np.array_equal(cut["owner"], run.cut.owner)
    st = pb.solve()
    assert st["status"] == 0
    en = pb.energy(per_atom=True)
    for k in ("e_pol", "e_ion", "e_coul"):
        r = run.energy[k]
        assert abs(en[k] - r) <= 1e-10 * abs(r), (k, en[k], r)
    pr = run.energy["phi_reac"]
    assert np.max(np.abs(en["phi_reac"] - pr)) <= 1e-9 * np.max(np.abs(pr))
    pb.close()
    # the mixed form with the multigrid preconditioner: FP32 box values from the expanded form
    g2 = I.cubic_grid(81, 0.4, center=shift, rtol=1e-9, precision=I.MIXED, inner_rtol=1e-4, precond=I.MG)
    pb = B.Problem(ctx, mol, g2)
    st = pb.solve()
    assert st["status"] == 0
    en = pb.energy()
    for k in ("e_pol", "e_ion", "e_coul"):
        r = run.energy[k]
        assert abs(en[k] - r) <= 1e-6 * abs(r), (k, en[k], r)
    pb.close()
