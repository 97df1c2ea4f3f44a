"""Pins of the multigrid-preconditioned CG oracle (``oracle/mg.py``).

CPU only.  Each part is fixed by something other than itself:

* operator fields      -> they reproduce the cell-by-cell assembled CSR matrix
* transfers            -> P is exact for linear functions; R is exactly P^T
* coarse operator      -> a constant coefficient gives the operator of the 2h grid
* smoother ordering    -> with one level the preconditioner is the textbook red-black
                          symmetric Gauss-Seidel matrix ((D+L) D^-1 (D+U))^-1, built densely
* V-cycle as a whole   -> symmetric and positive definite; on the constant-coefficient
                          Poisson problem it contracts the error by the factor expected of
                          V(1,1) red-black Gauss-Seidel multigrid (a wrong transfer weight or
                          a one-sided smoother fails these)
* PCG                  -> the same solution as the Jacobi-CG oracle (energies), Born energy
                          to solver tolerance, and far fewer iterations
"""
import numpy as np
import pytest

from oracle import mg as M
from oracle import oracle as O
from paper_2502_09323_amd import inputs as I


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build()


def _level(mol, grid):
    return M.fine_level(grid, mol)


def test_fields_reproduce_assembled_operator():
    mol = I.random_molecule(12, 2.5, 7)
    grid = I.cubic_grid(15, 0.5)
    L = _level(mol, grid)
    lB, kD = O.constants(grid.temp_K, grid.ionic_M, grid.eps_out)
    sol = O.classify(grid, mol)
    cut = O.cut_edges(grid, mol, sol)
    A, _ = O.assemble(grid, sol, cut, np.zeros(L.n), grid.eps_out * kD * kD)
    rng = np.random.default_rng(3)
    x = np.zeros(L.n)
    x[L.interior] = rng.standard_normal(int(L.interior.sum()))
    y = M.apply(L, x)
    want = A @ O.interior(x)
    assert np.max(np.abs(O.interior(y) - want)) <= 1e-13 * np.max(np.abs(want))


def test_prolongation_linear_exact_and_restriction_is_transpose():
    nf = (17, 13, 21)
    nc = tuple((v - 1) // 2 + 1 for v in nf)
    ax = [np.arange(v) * 2.0 for v in nc]   # coarse node coordinates in fine index units
    X, Y, Z = np.meshgrid(*ax, indexing="ij")
    lin = 0.3 * X - 1.7 * Y + 0.45 * Z + 2.0
    pf = M.prolong(nf, lin)
    fx = np.meshgrid(*[np.arange(v) * 1.0 for v in nf], indexing="ij")
    want = 0.3 * fx[0] - 1.7 * fx[1] + 0.45 * fx[2] + 2.0
    inner = np.zeros(nf, bool)
    inner[1:-1, 1:-1, 1:-1] = True
    assert np.max(np.abs(pf[inner] - want[inner])) <= 1e-12
    rng = np.random.default_rng(5)
    u = np.zeros(nf)
    u[inner] = rng.standard_normal(int(inner.sum()))
    v = np.zeros(nc)
    v[1:-1, 1:-1, 1:-1] = rng.standard_normal(tuple(c - 2 for c in nc))
    L = M.make_level(nf, 1.0, [np.ones(nf)] * 3, np.zeros(nf))
    lhs = float(np.sum(M.restrict(L, nc, u) * v))
    rhs = float(np.sum(u * M.prolong(nf, v)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_coarse_operator_of_constant_coefficient_is_the_2h_operator():
    n, h, eps, kb2 = 17, 0.5, 3.0, 0.7
    K = [np.full((n, n, n), h * eps) for _ in range(3)]
    L = M.make_level((n, n, n), h, K, np.full((n, n, n), h ** 3 * kb2))
    Lc = M.coarsen(L)
    c = slice(1, -1)
    for ax in range(3):
        # every coarse edge with an interior end point
        sl = [c, c, c]
        sl[ax] = slice(0, -1)
        assert np.allclose(Lc.K[ax][tuple(sl)], 2 * h * eps, rtol=1e-15, atol=0)
    assert np.allclose(Lc.m[c, c, c], (2 * h) ** 3 * kb2, rtol=1e-15, atol=0)


def test_one_level_is_red_black_symmetric_gauss_seidel():
    mol = I.random_molecule(6, 1.5, 9)
    grid = I.cubic_grid(7, 0.5)
    L = _level(mol, grid)
    idx = np.flatnonzero(L.interior.reshape(-1))
    nu = idx.size
    A = np.zeros((nu, nu))
    for t in range(nu):
        e = np.zeros(L.n)
        e.reshape(-1)[idx[t]] = 1.0
        A[:, t] = M.apply(L, e).reshape(-1)[idx]
    red = L.red.reshape(-1)[idx]
    perm = np.concatenate([np.flatnonzero(red), np.flatnonzero(~red)])
    Ap = A[np.ix_(perm, perm)]
    nr = int(red.sum())
    D = np.diag(np.diag(Ap))
    Lo = np.zeros_like(Ap)
    Lo[nr:, :nr] = Ap[nr:, :nr]
    Up = Lo.T.copy()
    Msgs = (D + Lo) @ np.linalg.inv(D) @ (D + Up)
    rng = np.random.default_rng(11)
    r = np.zeros(L.n)
    r[L.interior] = rng.standard_normal(nu)
    z = M.vcycle([L], r, nu=1, coarse_sweeps=1)
    want = np.linalg.solve(Msgs, r.reshape(-1)[idx][perm])
    got = z.reshape(-1)[idx][perm]
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


def test_vcycle_symmetric_positive_definite():
    mol = I.random_molecule(40, 3.0, 11)
    grid = I.cubic_grid(33, 0.5)
    levels = M.hierarchy(_level(mol, grid))
    assert [L.n[0] for L in levels] == [33, 17, 9, 5, 3]
    rng = np.random.default_rng(2)
    L = levels[0]
    u = np.zeros(L.n)
    v = np.zeros(L.n)
    u[L.interior] = rng.standard_normal(int(L.interior.sum()))
    v[L.interior] = rng.standard_normal(int(L.interior.sum()))
    Bu, Bv = M.vcycle(levels, u), M.vcycle(levels, v)
    a, b = float(np.sum(u * Bv)), float(np.sum(Bu * v))
    assert abs(a - b) <= 1e-12 * abs(a)
    assert float(np.sum(u * Bu)) > 0 and float(np.sum(v * Bv)) > 0


def _contraction(levels, iters=12, nu=1):
    """Asymptotic error reduction of x <- x + B (b - A x) (power iteration with b = 0)."""
    L = levels[0]
    rng = np.random.default_rng(4)
    e = np.zeros(L.n)
    e[L.interior] = rng.standard_normal(int(L.interior.sum()))
    rho = 0.0
    for _ in range(iters):
        n0 = np.linalg.norm(e)
        e = e - M.vcycle(levels, M.apply(L, e), nu=nu)
        rho = np.linalg.norm(e) / n0
    return rho


def test_vcycle_contraction_on_poisson():
    n = 33
    h = 1.0
    K = [np.full((n, n, n), h) for _ in range(3)]
    L = M.make_level((n, n, n), h, K, np.zeros((n, n, n)))
    levels = M.hierarchy(L)
    # V(1,1) and V(2,2) with red-black Gauss-Seidel, trilinear P, R = P^T on the 7-point
    # Laplacian reduce the error by about 0.41 and 0.17 per cycle (two-grid: the same 0.41,
    # so the factor does not grow with the number of levels); a restriction scaled by 1/2 or
    # 2, or injection in place of trilinear interpolation, gives 0.8 or more
    assert _contraction(levels) < 0.45
    assert _contraction(levels, nu=2) < 0.2
    # two-level and one-level variants: the coarse-grid correction is what makes the
    # difference (one level = a smoother only, which stalls on smooth errors)
    assert _contraction(levels[:1]) > 0.85


def test_mg_pcg_same_solution_as_jacobi_oracle():
    mol = I.random_molecule(40, 3.0, 11)
    grid = I.cubic_grid(33, 0.5)
    a = O.run(mol, grid, rtol=1e-12)
    b = M.run(mol, grid, rtol=1e-12)
    assert b.status == 0
    for k in ("e_pol", "e_ion", "q_pol_total"):
        assert abs(a.energy[k] - b.energy[k]) <= 1e-9 * abs(a.energy[k]), k
    assert np.max(np.abs(a.phi - b.phi)) <= 1e-9 * np.max(np.abs(a.phi))
    assert b.iters * 5 < a.iters


def test_mg_pcg_born_exact():
    mol = I.single_charge_sphere(center=(0.11, -0.07, 0.21))
    grid = I.cubic_grid(37, 0.5, temp_K=298.15)
    run = M.run(mol, grid, rtol=1e-13)
    lB = run.lB
    born = 0.5 * lB * (1.0 / 80.0 - 1.0 / 2.0) / 2.0
    assert run.status == 0
    assert abs(run.energy["e_pol"] / born - 1.0) < 1e-10
