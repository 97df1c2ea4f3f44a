"""Pins of the analytic many-sphere reference (``oracle/spheres.py``), then the grid oracle
against it.

The reference is pinned to what does not depend on it: the addition theorem of spherical
harmonics, the Kirkwood closed forms and the paper's Table 1, the uniform-medium limit, the
classical image-charge series for two conducting spheres (the limit eps_in -> infinity), the
boundary conditions checked point by point on every sphere from the expansions themselves,
and invariance under rotation and translation.  Then the grid oracle's energies and
reaction potentials on a multi-charge cluster approach the reference as h shrinks.
"""
import math
import os

import numpy as np
import pytest
from numpy.polynomial import legendre

from oracle import oracle as O
from oracle import spheres as S
from paper_2502_09323_amd import inputs as I

GOLD = os.path.join(os.path.dirname(__file__), "golden", "kirkwood_table1.txt")


def _gold():
    g = {}
    for line in open(GOLD):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()
            g[k] = float(v)
    return g


def _sph(m):
    return S.Spheres(m.xyz, m.radius, m.charge)


def test_harmonics_orthonormal_and_addition_theorem():
    rng = np.random.default_rng(0)
    u, w = S.sphere_quadrature(24)
    Y = S.real_harmonics(12, u)
    assert np.abs((Y * w) @ Y.T - np.eye(Y.shape[0])).max() < 1e-12
    a = rng.standard_normal((20, 3))
    a /= np.linalg.norm(a, axis=1)[:, None]
    b = rng.standard_normal((20, 3))
    b /= np.linalg.norm(b, axis=1)[:, None]
    Ya, Yb = S.real_harmonics(12, a), S.real_harmonics(12, b)
    for n in range(13):
        rows = slice(n * n, (n + 1) * (n + 1))
        lhs = (Ya[rows] * Yb[rows]).sum(axis=0)
        c = np.zeros(n + 1)
        c[n] = 1.0
        rhs = (2 * n + 1) / (4 * math.pi) * legendre.legval((a * b).sum(axis=1), c)
        assert np.abs(lhs - rhs).max() < 1e-12


@pytest.mark.parametrize("ionic", [0.145, 0.0])
def test_single_sphere_is_kirkwood(ionic):
    g = _gold()
    lB, kD = O.constants(g["temp_K"], ionic, g["eps_out"])
    R, q = g["radius_A"], g["charge_e"]
    sph = S.Spheres(np.array([[0.7, -1.3, 2.2]]), np.array([R]), np.array([q]))
    e = S.energies(S.solve(sph, g["eps_in"], g["eps_out"], kD, N=6), lB)
    born = 0.5 * q * q * (1.0 / g["eps_out"] - 1.0 / g["eps_in"]) / R * lB
    ion = -0.5 * q * q / g["eps_out"] * kD / (1.0 + kD * R) * lB
    assert abs(e["e_pol"] / born - 1.0) < 1e-12
    assert abs(e["e_ion"] - ion) < 1e-12 * abs(born)
    assert e["e_coul"] == 0.0
    if ionic > 0:   # the values printed in Table 1, two decimals
        assert round(e["e_pol"], 2) == g["E_pol_kT"]
        assert round(e["e_ion"], 2) == g["E_ion_kT"]
        assert round(e["e_total"], 2) == g["E_total_kT"]


def test_uniform_medium_has_no_reaction():
    m = I.sphere_cluster(5, 3, n_neutral_top=0)
    sol = S.solve(_sph(m), 4.0, 4.0, 0.0, N=8)
    e = S.energies(sol)
    assert abs(e["e_pol"]) < 1e-12 * abs(e["e_coul"])
    assert abs(e["e_ion"]) < 1e-12 * abs(e["e_coul"])
    assert np.abs(e["phi_reac"]).max() < 1e-12 * np.abs(m.charge).max()


def _kelvin_potential_coefficient(R1, R2, d):
    """P_11 of two conducting spheres in vacuum (potential of sphere 1 per unit charge on it,
    sphere 2 uncharged), from the capacitance coefficients of the classical image series:
    sphere a held at potential 1 and sphere b grounded start from the charge R_a at centre a;
    a charge q at distance D from a grounded sphere's centre has the image -q R/D at R^2/D."""
    def images(Ra, Rb):
        qa, qb = Ra, 0.0
        q, x, side = Ra, 0.0, "a"       # x: position from centre a toward centre b
        while abs(q) > 1e-22:
            if side == "a":
                D = d - x
                q, x, side = -q * Rb / D, d - Rb * Rb / D, "b"
                qb += q
            else:
                D = x
                q, x, side = -q * Ra / D, Ra * Ra / D, "a"
                qa += q
        return qa, qb
    C11, C21 = images(R1, R2)
    C22, C12 = images(R2, R1)
    return float(np.linalg.inv(np.array([[C11, C12], [C21, C22]]))[0, 0])


@pytest.mark.parametrize("gap", [0.5, 1.0, 3.0])
def test_two_conducting_spheres_match_the_image_series(gap):
    R1, R2 = 2.0, 1.5
    d = R1 + R2 + gap
    direction = np.array([0.6, 0.8, 0.0])
    sph = S.Spheres(np.array([[0.0, 0.0, 0.0], d * direction]), np.array([R1, R2]), np.array([1.0, 0.0]))
    e = S.energies(S.solve(sph, 1e10, 1.0, 0.0, N=24))
    want = 0.5 * _kelvin_potential_coefficient(R1, R2, d)
    assert abs(e["e_total"] / want - 1.0) < 1e-8


def test_boundary_conditions_hold_pointwise():
    lB, kD = O.constants(298.15, 0.145, 80.0)
    sph = S.Spheres(np.array([[0.0, 0.0, 0.0], [5.6, 0.5, 0.3], [-0.8, 5.4, 1.0], [1.5, 1.0, -5.6]]),
                    np.array([2.0, 1.6, 1.8, 1.4]), np.array([1.0, -0.6, 0.4, 0.0]))
    rng = np.random.default_rng(3)
    res = {}
    for N in (8, 16):
        sol = S.solve(sph, 2.0, 80.0, kD, N=N)
        wv = wd = 0.0
        h = 1e-4
        for i in range(4):
            v = rng.standard_normal((40, 3))
            v /= np.linalg.norm(v, axis=1)[:, None]
            p = sph.centers[i] + sph.radii[i] * v

            def dn(f):
                return (-f(p + 2 * h * v) + 8 * f(p + h * v) - 8 * f(p - h * v) + f(p - 2 * h * v)) / (12 * h)
            fin, fout = S.interior_potential(sol, i, p), S.exterior_potential(sol, p)
            din = dn(lambda x: S.interior_potential(sol, i, x))
            dout = dn(lambda x: S.exterior_potential(sol, x))
            wv = max(wv, np.abs(fin - fout).max() / np.abs(fin).max())
            wd = max(wd, np.abs(2.0 * din - 80.0 * dout).max() / np.abs(2.0 * din).max())
        res[N] = (wv, wd)
    assert res[16][0] < 1e-7 and res[16][1] < 1e-6
    assert res[16][0] < 0.01 * res[8][0] and res[16][1] < 0.01 * res[8][1]


def test_rotation_and_translation_invariance():
    lB, kD = O.constants(298.15, 0.145, 80.0)
    m = I.sphere_cluster(5, 8, n_neutral_top=1)
    e0 = S.energies(S.solve(_sph(m), 2.0, 80.0, kD, N=12), lB)
    Q, _ = np.linalg.qr(np.random.default_rng(5).standard_normal((3, 3)))
    xyz = m.xyz @ Q.T + np.array([3.1, -7.4, 0.9])
    e1 = S.energies(S.solve(S.Spheres(xyz, m.radius, m.charge), 2.0, 80.0, kD, N=12), lB)
    for k in ("e_total", "e_pol", "e_ion", "e_coul"):
        assert abs(e1[k] - e0[k]) < 1e-9 * abs(e0["e_total"]), k
    assert np.abs(e1["phi_reac"] - e0["phi_reac"]).max() < 1e-9 * np.abs(e0["phi_reac"]).max()


def test_truncation_converges():
    lB, kD = O.constants(298.15, 0.145, 80.0)
    m = I.sphere_cluster(6, 21, n_neutral_top=1)
    e = {N: S.energies(S.solve(_sph(m), 2.0, 80.0, kD, N=N), lB) for N in (10, 14)}
    for k in ("e_total", "e_pol", "e_ion"):
        assert abs(e[14][k] - e[10][k]) < 1e-7 * abs(e[14]["e_total"]), k


def test_grid_oracle_converges_to_the_many_sphere_solution():
    """The external pin of the grid method on a multi-charge geometry: six spheres, five
    charged, Debye-Hueckel box values.  E_pol is close at h = 0.5 (the self terms are exact by
    the discrete Gauss law), E_ion and the reaction potentials at the centres converge."""
    lB, kD = O.constants(298.15, 0.145, 80.0)
    m = I.sphere_cluster(6, 21, n_neutral_top=1)
    ref = S.energies(S.solve(_sph(m), 2.0, 80.0, kD, N=14), lB)
    lo, hi = (m.xyz - m.radius[:, None]).min(0), (m.xyz + m.radius[:, None]).max(0)
    ctr = tuple(0.5 * (lo + hi))
    err = {}
    for n, h in ((61, 0.5), (121, 0.25)):
        run = O.run(m, I.cubic_grid(n, h, center=ctr, temp_K=298.15), rtol=1e-10)
        en = run.energy
        err[h] = (abs(en["e_pol"] / ref["e_pol"] - 1.0), abs(en["e_ion"] / ref["e_ion"] - 1.0),
                  np.abs(en["phi_reac"] - ref["phi_reac"]).max() / np.abs(ref["phi_reac"]).max())
        assert abs(en["e_coul"] / ref["e_coul"] - 1.0) < 1e-12
    assert err[0.5][0] < 1e-3 and err[0.25][0] < 5e-4
    assert err[0.25][1] < 0.5 * err[0.5][1] and err[0.25][1] < 0.05
    assert err[0.25][2] < 0.5 * err[0.5][2] and err[0.25][2] < 2e-3


def test_polarization_potential_by_direct_quadrature():
    """phi_pol at every centre equals the Coulomb integral of the polarization layer
    (1/eps_out - 1/eps_in) D_n/(4 pi), with D_n = -eps_in dphi_in/dn taken by finite
    differences of the interior expansion and the integral done by surface quadrature."""
    lB, kD = O.constants(298.15, 0.145, 80.0)
    sph = S.Spheres(np.array([[0.0, 0.0, 0.0], [5.6, 0.5, 0.3], [-0.8, 5.4, 1.0]]),
                    np.array([2.0, 1.6, 1.8]), np.array([1.0, -0.6, 0.4]))
    sol = S.solve(sph, 2.0, 80.0, kD, N=14)
    e = S.energies(sol)
    u, w = S.sphere_quadrature(40)
    h = 1e-4
    want = np.zeros(3)
    for i in range(3):
        R = sph.radii[i]
        p = sph.centers[i] + R * u
        f = lambda x: S.interior_potential(sol, i, x)   # noqa: E731
        dphi = (-f(p + 2 * h * u) + 8 * f(p + h * u) - 8 * f(p - h * u) + f(p - 2 * h * u)) / (12 * h)
        sigma = (1.0 / 80.0 - 1.0 / 2.0) * (-2.0 * dphi) / (4.0 * math.pi)
        for j in range(3):
            want[j] += np.sum(w * R * R * sigma / np.linalg.norm(sph.centers[j] - p, axis=1))
    assert np.abs(e["phi_pol"] - want).max() < 1e-8 * np.abs(want).max()


def test_stored_thirty_sphere_values_reproduce():
    """The stored analytic values of the 30-sphere cluster (degree 14) are those of the
    reference: recomputed at degree 8 they agree to 1e-6."""
    gold = {}
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "spheres30_analytic.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()
            gold[k] = float(v)
    m = I.sphere_cluster(30, 2506)
    lB, kD = O.constants(298.15, 0.145, 80.0)
    e = S.energies(S.solve(_sph(m), 2.0, 80.0, kD, N=8), lB)
    for k in ("e_total", "e_coul", "e_pol", "e_ion"):
        assert abs(e[k] - gold[k]) < 1e-6 * abs(gold["e_total"]), k
    pr = np.array([gold[f"phi_reac_{i}"] for i in range(30)])
    assert np.abs(e["phi_reac"] - pr).max() < 1e-6 * np.abs(pr).max()
