"""The allocation-free energy read-back (pb_energy_noalloc) against pb_energy.

Both run the same kernels on the same solved problem; the allocation-free form takes its
buffers from the library's static scratch array instead of the context allocator.  Two calls
in a row, the second on a smaller problem (the array keeps the first call's contents), must
give pb_energy's energies and reaction potentials to the FP64 bar (1e-10 relative); with
pb_energy's N-body chunking (it fits both problems) they are equal bit for bit.  A problem
whose read-back needs more than the array is rejected with PB_ENOMEM."""
from dataclasses import replace

import numpy as np
import pytest

from paper_2502_09323_amd import binding as B
from paper_2502_09323_amd import inputs as I

pytestmark = pytest.mark.gpu

KEYS = ("e_pol", "e_ion", "e_coul", "e_solv", "e_total", "q_pol_total", "area_total")


def compare(got, ref, tol=1e-10):
    assert got["n_cut"] == ref["n_cut"]
    for k in KEYS:
        assert abs(got[k] - ref[k]) <= tol * max(abs(ref[k]), 1e-300), (k, got[k], ref[k])
    pr = ref["phi_reac"]
    assert np.max(np.abs(got["phi_reac"] - pr)) <= tol * np.max(np.abs(pr))


@pytest.fixture(scope="module")
def ctx():
    import torch

    assert torch.cuda.is_available()
    B.load()
    c = B.Context(0)
    yield c
    c.close()


def test_noalloc_energy_equals_pb_energy(ctx):
    assert B.load().pb_energy_noalloc_limit() == 128 << 20
    print("no-alloc read-back: 2000 atoms, 161^3, FP64 multigrid", flush=True)
    mol, grid = I.protein_c2(rtol=1e-10, precond=I.MG)
    pb = B.Problem(ctx, mol, grid)
    assert pb.solve()["status"] == 0
    ref = pb.energy(per_atom=True)
    got = pb.energy_noalloc(per_atom=True)
    compare(got, ref)
    for k in KEYS:
        assert got[k] == ref[k], k
    assert np.array_equal(got["phi_reac"], ref["phi_reac"])
    pb.close()
    print("no-alloc read-back: 150 atoms, 49^3, mixed Jacobi", flush=True)
    mol2 = I.random_molecule(150, 6.0, 5)
    grid2 = I.cubic_grid(49, 0.4, precision=I.MIXED, rtol=1e-9, inner_rtol=1e-3)
    pb2 = B.Problem(ctx, mol2, grid2)
    assert pb2.solve()["status"] == 0
    got2 = pb2.energy_noalloc(per_atom=True)
    ref2 = pb2.energy(per_atom=True)
    compare(got2, ref2)
    for k in KEYS:
        assert got2[k] == ref2[k], k
    assert np.array_equal(got2["phi_reac"], ref2["phi_reac"])
    # the allocation-free call leaves pb_energy's per-edge fields in place
    cut = pb2.cut(fields=True)
    assert np.all(np.isfinite(cut["F"]))
    pb2.close()


def test_noalloc_energy_limits(ctx):
    mol = I.random_molecule(40, 4.0, 3)
    pb = B.Problem(ctx, mol, I.cubic_grid(33, 0.5))
    with pytest.raises(B.PbError) as e:
        pb.energy_noalloc()                 # not solved
    assert e.value.code == B.PB_EINVAL
    pb.close()
    print("no-alloc read-back: 385^3 problem beyond the scratch array", flush=True)
    mol, grid = I.large_c4()
    pb = B.Problem(ctx, mol, replace(grid, precision=I.MIXED))
    with pytest.raises(B.PbError) as e:
        pb.energy_noalloc()                 # about 4.3M cut edges
    assert e.value.code == B.PB_ENOMEM and "limit" in str(e.value)
    pb.close()
