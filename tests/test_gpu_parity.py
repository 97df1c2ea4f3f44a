"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the same seeded
inputs.  Integer and flag data must be bit-exact; FP64 coefficients agree to rounding;
FP64 energies to 1e-10 relative; the mixed FP32/FP64 path to 1e-6 relative."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2502_09323_amd import binding as B
from paper_2502_09323_amd import inputs as I

pytestmark = pytest.mark.gpu

E_TOL64 = 1e-10
E_TOL_MIXED = 1e-6


@pytest.fixture(scope="module")
def ctx():
    import torch

    assert torch.cuda.is_available()
    B.load()
    c = B.Context(0)
    yield c
    c.close()


def oracle_offdiag(grid, A):
    """Edge coefficients K (positive) between interior unknowns from the oracle's CSR."""
    nx, ny, nz = (int(v) - 2 for v in grid.n)
    coo = A.tocoo()
    r, c, v = coo.row, coo.col, coo.data
    out = {}
    for name, off in (("kz", 1), ("ky", nz), ("kx", ny * nz)):
        m = c == r + off
        arr = np.full(nx * ny * nz, np.nan)
        arr[r[m]] = -v[m]
        out[name] = arr
    return out


def compare_build(pb, run, grid):
    co = pb.coeffs()
    assert np.array_equal(co["solute"], run.solute), "solute flags differ"
    inner = (slice(1, -1),) * 3
    d_gpu = co["diag"][inner].reshape(-1)
    d_or = run.A.diagonal()
    assert np.max(np.abs(d_gpu - d_or) / d_or) <= 1e-13
    off = oracle_offdiag(grid, run.A)
    for name in ("kx", "ky", "kz"):
        g = co[name][inner].reshape(-1)
        m = ~np.isnan(off[name])
        assert np.max(np.abs(g[m] - off[name][m]) / off[name][m]) <= 1e-13, name
    b_gpu = co["rhs"][inner].reshape(-1)
    sc = max(np.max(np.abs(run.b)), 1e-300)
    assert np.max(np.abs(b_gpu - run.b)) <= 1e-13 * sc
    cut = pb.cut()
    assert np.array_equal(cut["key"], run.cut.key), "cut-edge keys differ"
    assert np.array_equal(cut["owner"], run.cut.owner)
    assert np.max(np.abs(cut["alpha"] - run.cut.alpha), initial=0) <= 1e-13
    assert np.max(np.abs(cut["rp"] - run.cut.rp), initial=0) <= 1e-12
    assert np.max(np.abs(cut["np"] - run.cut.np_), initial=0) <= 1e-12
    if run.energy:
        wp = run.energy["wp"]
        assert np.max(np.abs(cut["wp"] - wp), initial=0) <= 1e-12 * max(np.max(wp, initial=0), 1.0)


def compare_energy(got, ref, tol, keys=("e_pol", "e_ion", "e_coul")):
    for k in keys:
        r = ref[k]
        assert abs(got[k] - r) <= tol * max(abs(r), 1e-12), (k, got[k], r)


def test_kirkwood_c1_full_parity(ctx):
    mol, grid = I.kirkwood_c1(rtol=1e-12)
    run = O.run(mol, grid, rtol=1e-12)
    pb = B.Problem(ctx, mol, grid)
    compare_build(pb, run, grid)
    st = pb.solve()
    assert st["status"] == 0
    en = pb.energy(per_atom=True)
    compare_energy(en, run.energy, E_TOL64, keys=("e_pol", "e_ion"))
    assert en["n_cut"] == run.cut.m == 1158
    assert abs(en["area_total"] - run.energy["area_total"]) <= 1e-12 * run.energy["area_total"]
    phi = pb.potential()
    lB = run.lB
    assert np.max(np.abs(phi - lB * run.phi)) <= 1e-8 * np.max(np.abs(lB * run.phi))
    # the Born polarization energy holds to solver tolerance on the GPU too
    born = 0.5 * (1 / 80 - 1 / 2) / 2.0 * lB
    assert abs(en["e_pol"] - born) <= 1e-10 * abs(born)
    assert abs(en["phi_reac"][0] - 2 * (en["e_pol"] + en["e_ion"])) <= 1e-12 * abs(en["phi_reac"][0])
    ge = O.grid_energy(grid, mol, run.phi, lB)
    assert abs(pb.grid_energy() - ge) <= E_TOL64 * abs(ge)
    pb.close()


CASES = [
    # (n_atoms, sphere_R, seed, n, h, bc)
    (60, 5.0, 1, (33, 33, 33), 0.5, I.BC_DH),
    (120, 6.0, 2, (41, 47, 70), 0.45, I.BC_ZERO),
    (200, 7.0, 3, (67, 61, 131), 0.3, I.BC_DH),
    (25, 3.0, 4, (29, 17, 66), 0.6, I.BC_USER),
]


@pytest.mark.parametrize("case", CASES, ids=[f"N{c[0]}_n{'x'.join(map(str, c[3]))}_bc{c[5]}" for c in CASES])
def test_small_molecule_parity(ctx, case):
    na, R, seed, n, h, bc = case
    mol = I.random_molecule(na, R, seed)
    half = [0.5 * (v - 1) * h for v in n]
    grid = I.GridSpec(n=n, h=h, origin=tuple(-x for x in half), bc=bc, rtol=1e-12, temp_K=300.0)
    if bc == I.BC_USER:
        rng = np.random.default_rng(seed)
        grid.bc_values = rng.normal(0, 0.01, size=n)
    run = O.run(mol, grid, rtol=1e-12)
    pb = B.Problem(ctx, mol, grid)
    compare_build(pb, run, grid)
    st = pb.solve()
    assert st["status"] == 0
    en = pb.energy(per_atom=True)
    compare_energy(en, run.energy, E_TOL64)
    assert abs(en["q_pol_total"] - run.energy["q_pol_total"]) <= 1e-10 * max(1.0, abs(run.energy["q_pol_total"]))
    pr = run.energy["phi_reac"]
    assert np.max(np.abs(en["phi_reac"] - pr)) <= 1e-9 * np.max(np.abs(pr))
    cut = pb.cut(fields=True)
    assert np.max(np.abs(cut["F"] - run.energy["F"])) <= 1e-8 * np.max(np.abs(run.energy["F"]))
    ge = O.grid_energy(grid, mol, run.phi, run.lB)
    assert abs(pb.grid_energy() - ge) <= E_TOL64 * abs(ge)
    pb.close()


def test_mixed_precision_matches_fp64_oracle(ctx):
    mol = I.random_molecule(300, 8.0, 21)
    grid = I.cubic_grid(49, 0.5, precision=I.MIXED, rtol=1e-9, inner_rtol=1e-4)
    run = O.run(mol, grid, rtol=1e-12)
    pb = B.Problem(ctx, mol, grid)
    st = pb.solve()
    assert st["status"] == 0 and st["outer_iters"] >= 2
    assert st["relres"] <= 1e-9
    en = pb.energy()
    compare_energy(en, run.energy, E_TOL_MIXED)
    ge = O.grid_energy(grid, mol, run.phi, run.lB)
    assert abs(pb.grid_energy() - ge) <= E_TOL_MIXED * abs(ge)
    pb.close()


def test_solve_is_deterministic(ctx):
    mol = I.random_molecule(150, 7.0, 8)
    grid = I.cubic_grid(57, 0.4, rtol=1e-10)
    out = []
    for _ in range(2):
        pb = B.Problem(ctx, mol, grid)
        st = pb.solve()
        en = pb.energy(per_atom=True)
        out.append((st["iters"], en["e_pol"], en["e_ion"], en["phi_reac"].copy(), pb.potential()))
        pb.close()
    a, b = out
    assert a[0] == b[0] and a[1] == b[1] and a[2] == b[2]
    assert np.array_equal(a[3], b[3]) and np.array_equal(a[4], b[4])


def test_invalid_inputs_and_nonconvergence(ctx):
    mol = I.single_charge_sphere(R=2.0, center=(0.0, 0.0, 6.9))
    grid = I.cubic_grid(33, 0.5)  # half-width 8 A: the ball reaches the last interior cell
    with pytest.raises(B.PbError) as e:
        B.Problem(ctx, mol, grid)
    assert e.value.code == B.PB_EINVAL
    bad = I.single_charge_sphere()
    bad.xyz[0, 1] = float("nan")
    with pytest.raises(B.PbError) as e:
        B.Problem(ctx, bad, I.cubic_grid(33, 0.5))
    assert e.value.code == B.PB_EINVAL
    mol, grid = I.kirkwood_c1(max_iter=5)
    pb = B.Problem(ctx, mol, grid)
    st = pb.solve()
    assert st["status"] == B.PB_ENOCONV and st["iters"] == 5
    en = pb.energy()  # the last iterate is still usable
    assert math.isfinite(en["e_pol"])
    pb.close()


def test_empty_molecule(ctx):
    mol = I.Molecule(np.zeros((0, 3)), np.zeros(0), np.zeros(0))
    grid = I.cubic_grid(17, 0.5)
    pb = B.Problem(ctx, mol, grid)
    st = pb.solve()
    assert st["status"] == 0 and st["iters"] == 0
    en = pb.energy()
    assert en["n_cut"] == 0 and en["e_pol"] == 0.0 and en["e_ion"] == 0.0
    assert np.all(pb.potential() == 0.0)
    assert pb.grid_energy() == 0.0
    pb.close()


def test_c2_full_size_parity(ctx):
    """The 2,000-atom, 161^3 workload: every coefficient, every cut edge and the energies."""
    mol, grid = I.protein_c2(rtol=1e-11)
    run = O.run(mol, grid, rtol=1e-12)
    pb = B.Problem(ctx, mol, grid)
    compare_build(pb, run, grid)
    st = pb.solve()
    assert st["status"] == 0
    en = pb.energy()
    compare_energy(en, run.energy, E_TOL64)
    ge = O.grid_energy(grid, mol, run.phi, run.lB)
    assert abs(pb.grid_energy() - ge) <= E_TOL64 * abs(ge)
    pb.close()


DH_CASES = [
    # (label, ionic strength M, molecule centre)
    ("salt", 0.145, (0.0, 0.0, 0.0)),
    ("no_salt", 0.0, (0.0, 0.0, 0.0)),
    ("salt_far_from_origin", 0.145, (150.0, -90.0, 230.0)),
]


def dh_abs_scale(grid, mol, kD):
    """Full-grid array holding, at the box nodes, sum over atoms of |q| exp(-kD r) / (eps_out r):
    the scale of the rounding error of a Debye-Hueckel value (the sum itself cancels between
    charges of both signs)."""
    n = [int(v) for v in grid.n]
    idx = np.indices(n).reshape(3, -1)
    box = np.zeros(idx.shape[1], bool)
    for d in range(3):
        box |= (idx[d] == 0) | (idx[d] == n[d] - 1)
    pts = (idx[:, box].T * grid.h + np.asarray(grid.origin)).astype(np.float64)
    xyz = np.asarray(mol.xyz, np.float64)
    aq = np.abs(np.asarray(mol.charge, np.float64))
    out = np.empty(len(pts))
    for s0 in range(0, len(pts), 1024):
        r = np.linalg.norm(pts[s0:s0 + 1024, None, :] - xyz[None, :, :], axis=2)
        out[s0:s0 + 1024] = (aq[None, :] * np.exp(-kD * r) / (grid.eps_out * r)).sum(axis=1)
    full = np.zeros(idx.shape[1])
    full[box] = out
    return full.reshape(n)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_dh_all_box_nodes_non_cubic(ctx, prec):
    """Debye-Hueckel values (Sect. 2.3) at every box node, the edges and corners of the box
    included, on a grid with a different node count per axis (so that every face has ragged
    patch rows and columns): the exported potential at the box nodes is lB g, against the
    oracle's g, to 1e-13 (FP64) or 1e-6 (mixed: FP32 distance, exponential and group sums) of the
    absolute-value scale of each node."""
    mol = I.random_molecule(700, 8.0, 23, center=(3.0, -2.0, 1.0))
    n = (45, 38, 51)
    h = 0.6
    origin = tuple(c - 0.5 * (v - 1) * h for c, v in zip((3.0, -2.0, 1.0), n))
    grid = I.GridSpec(n=n, h=h, origin=origin, ionic_M=0.145,
                      precision=I.FP64 if prec == "fp64" else I.MIXED)
    lB, kD = O.constants(grid.temp_K, grid.ionic_M, grid.eps_out)
    g = O.boundary_values(grid, mol, kD)
    sabs = dh_abs_scale(grid, mol, kD)
    pb = B.Problem(ctx, mol, grid)
    try:
        phi = pb.potential()
    finally:
        pb.close()
    box = sabs > 0
    assert box.sum() == 2 * (n[0] * n[1] + n[0] * n[2] + n[1] * n[2]) - 4 * sum(n) + 8
    err = np.abs(phi[box] / lB - g[box]) / sabs[box]
    tol = 1e-13 if prec == "fp64" else 1e-6
    print(f"{prec}: {box.sum()} box nodes, max difference {err.max():.2e} of the absolute-value scale")
    assert err.max() <= tol


@pytest.mark.parametrize("label,ionic,center", DH_CASES, ids=[c[0] for c in DH_CASES])
def test_dh_box_values_parity(ctx, label, ionic, center):
    """FP64 Debye-Hueckel box values (Sect. 2.3) against the oracle's: at the interior nodes
    next to the box the right-hand side is the charge deposit plus the boundary lift K g, and
    it agrees with the oracle's node by node to 1e-13 of the lift's absolute-value scale (the
    values sum charges of both signs, so they cancel), and to 1e-13 of the largest value."""
    mol = I.random_molecule(3000, 12.0, 21, center=center)
    grid = I.cubic_grid(65, 0.5, center=center, ionic_M=ionic)
    lB, kD = O.constants(grid.temp_K, grid.ionic_M, grid.eps_out)
    assert (kD == 0.0) == (ionic == 0.0)
    sol = O.classify(grid, mol)
    cut = O.cut_edges(grid, mol, sol)
    g = O.boundary_values(grid, mol, kD)
    _, lift = O.assemble(grid, sol, cut, g, grid.eps_out * kD * kD)
    b_or = O.interior(O.deposit(grid, mol)) + lift
    pb = B.Problem(ctx, mol, grid)
    try:
        b_gpu = pb.coeffs()["rhs"][(slice(1, -1),) * 3].reshape(-1)
    finally:
        pb.close()
    ni = [int(v) - 2 for v in grid.n]
    idx = np.indices(ni).reshape(3, -1)
    next_to_box = np.zeros(idx.shape[1], bool)
    for d in range(3):
        next_to_box |= (idx[d] == 0) | (idx[d] == ni[d] - 1)
    # scale of the lift's rounding error at each node: K (h eps_out on the solvent edges to the
    # box) times the absolute-value sums of its box neighbours
    sabs = dh_abs_scale(grid, mol, kD)
    lscale = np.zeros(ni)
    inner = (slice(1, -1),) * 3
    for d in range(3):
        for sh in (-1, 1):
            lscale += np.roll(sabs, sh, axis=d)[inner]
    lscale = grid.h * grid.eps_out * lscale.reshape(-1)
    bo, bg, ls = b_or[next_to_box], b_gpu[next_to_box], lscale[next_to_box]
    assert np.all(ls > 0)
    err = np.abs(bg - bo) / ls
    print(f"{label}: {next_to_box.sum()} nodes next to the box, max difference {err.max():.2e} of the lift's "
          f"absolute-value scale, {np.max(np.abs(bg - bo)) / np.max(np.abs(bo)):.2e} of the largest value")
    assert err.max() <= 1e-13
    assert np.max(np.abs(bg - bo)) <= 1e-13 * np.max(np.abs(bo))
