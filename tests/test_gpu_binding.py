"""Binding energies on the GPU: the three solves of a complex and its parts served together
through the serving loop (multigrid and Jacobi requests in one mix), against the oracle's
FP64 solves of the same molecules on the same grid."""
from dataclasses import replace

import numpy as np
import pytest

from oracle import oracle as O
from paper_2502_09323_amd import binding as B
from paper_2502_09323_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctxs():
    import torch

    B.load()
    main = B.Context(0)
    side = B.Context(0, stream=torch.cuda.Stream(0))
    yield main, side
    main.close()
    side.close()


def test_served_binding_energy_matches_oracle(ctxs):
    main, side = ctxs
    cpx, rec, lig = I.binding_complex(3, n_rec=90, n_lig=25, R_rec=6.0, R_lig=3.0)
    grid = I.binding_grid(cpx, 0.6, margin=4.0, precision=I.MIXED, rtol=1e-10, inner_rtol=1e-2)
    parts = [("c", cpx), ("1", rec), ("2", lig)]
    srv = B.Server(main, side, max_resident=8)
    for i, (name, mol) in enumerate(parts):
        srv.submit(mol, replace(grid, precond=I.MG if i != 2 else I.JACOBI), i)
    got = {}
    while len(got) < 3:
        srv.step()
        for r in srv.poll():
            got[r["id"]] = r
    srv.close()
    ref = [O.run(mol, replace(grid, precision=I.FP64), rtol=1e-12).energy for _, mol in parts]
    for i in range(3):
        assert got[i]["code"] == 0
        for k in ("e_pol", "e_ion", "e_coul"):
            assert abs(got[i][k] - ref[i][k]) <= 1e-6 * abs(ref[i][k]), (i, k)
    ddg = B.binding_ddg(got[0], got[1], got[2])
    ddg_ref = B.binding_ddg(ref[0], ref[1], ref[2])
    scale = max(abs(ref[0]["e_total"]), abs(ref[1]["e_total"]))
    for k in ("ddg_total", "ddg_pol", "ddg_ion"):
        assert abs(ddg[k] - ddg_ref[k]) <= 2e-6 * scale, k
    # the Coulomb part is the sum over pairs across the two parts
    d = np.linalg.norm(rec.xyz[:, None, :] - lig.xyz[None, :, :], axis=2)
    lB, _ = O.constants(grid.temp_K, grid.ionic_M, grid.eps_out)
    cross = lB * float(np.sum(rec.charge[:, None] * lig.charge[None, :] / d)) / grid.eps_in
    assert abs(ddg["ddg_coul"] - cross) <= 1e-9 * abs(cross)
