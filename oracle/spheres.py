"""Analytic reference for non-overlapping dielectric spheres with central point charges in a
Debye-Hueckel solvent (paper Sect. "An analytical benchmark" and its appendix).

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and by the script that writes stored
reference values under ``tests/golden/``.  The product path never imports it, and it imports
nothing from the product package.

Model (reduced Gaussian units, as the grid oracle: potentials in e/Angstrom, energies times
the Bjerrum length give kT).  Sphere i has centre c_i, radius R_i, permittivity eps_in and a
point charge q_i at its centre; outside all spheres the permittivity is eps_out and the
potential obeys the linearized PBE with inverse Debye length kappa.  As in the paper:

    inside sphere i:  phi = q_i/(eps_in rho_i) + sum_{n,m} L_{nm,i} rho_i^n Y_nm(u_i)
    outside:          phi = sum_j sum_{n,m} G_{nm,j} f_n(rho_j) Y_nm(u_j)

with rho_j, u_j the distance and direction from c_j, f_n(r) = k_n(kappa r) (modified spherical
Bessel function of the second kind; r^-(n+1) when kappa = 0), and Y_nm a real orthonormal
basis of spherical harmonics.  The unknowns follow from continuity of phi and of
eps dphi/dn on every sphere.

Re-expansion (this module's own route; the paper uses closed-form translation
coefficients): on sphere i, the field of every other sphere j is regular, so on the closed
ball of radius R_i it equals sum_{n,m} B_nm g_n(rho_i) Y_nm(u_i) with g_n(r) = i_n(kappa r)
(r^n when kappa = 0).  Its coefficients are read off by projecting its values on the surface
rho_i = R_i onto Y_nm with a product Gauss-Legendre x trapezoid quadrature; its normal
derivative is then B_nm g_n'(R_i).  With degrees up to N on every sphere, projecting both
conditions onto Y_nm (n <= N) gives, for the scaled exterior coefficients
b_nm,i = G_nm,i f_n(R_i) and the projections O_nm,i of the other spheres' fields,

    (1)  a_nm,i + q_i sqrt(4 pi)/(eps_in R_i) [n = 0] = b_nm,i + O_nm,i
    (2)  -q_i sqrt(4 pi)/R_i^2 [n = 0] + eps_in (n/R_i) a_nm,i
             = eps_out (F_n,i b_nm,i + G_n,i O_nm,i)

where a_nm,i = L_nm,i R_i^n, F_n,i = f_n'(R_i)/f_n(R_i), G_n,i = g_n'(R_i)/g_n(R_i).
Eliminating a with (1) leaves one dense linear system in b.

Energies (the paper's partition):
* E = 1/2 sum_i q_i (phi - q_i/(eps_in rho_i)) at c_i = 1/2 sum_i q_i a_00,i / sqrt(4 pi)
  (every contribution but the self-energy of each point charge);
* E_coul = 1/2 sum_{i != j} q_i q_j /(eps_in |c_i - c_j|);
* E_pol = 1/2 sum_j q_j phi_pol(c_j), phi_pol the potential of the polarization charge
  sigma = (1/eps_out - 1/eps_in) D_n/(4 pi) on all spheres, D_n = -eps_in dphi_in/drho the
  outward normal displacement; on sphere i, D_nm = q_i sqrt(4 pi)/R_i^2 [n = 0]
  - eps_in n a_nm/R_i, and the potential of the layer sum_nm s_nm Y_nm on a sphere of
  radius R is sqrt(4 pi) R s_00 at its centre and sum_nm s_nm 4 pi R^2 R^n/((2n+1) d^(n+1))
  Y_nm(u) at distance d > R in direction u (the multipole expansion of 1/|x - y|);
* E_ion = E - E_coul - E_pol.
The reaction potential at c_i (polarization plus ions) is phi - q_i/(eps_in rho_i) at c_i
minus the other charges' Coulomb potentials sum_{j != i} q_j/(eps_in |c_i - c_j|).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy import special


def nmodes(N: int) -> int:
    return (N + 1) * (N + 1)


def mode_degree(N: int) -> np.ndarray:
    """Degree n of each mode index n*n + n + m, m = -n..n."""
    return np.concatenate([np.full(2 * n + 1, n) for n in range(N + 1)])


def real_harmonics(N: int, u: np.ndarray) -> np.ndarray:
    """Real orthonormal spherical harmonics of degree <= N at unit vectors u (npts, 3):
    Y_{n,0} = pbar_n^0, Y_{n,m} = sqrt(2) pbar_n^m cos(m phi), Y_{n,-m} = sqrt(2) pbar_n^m
    sin(m phi), m > 0, with pbar_n^m the associated Legendre functions (no Condon-Shortley
    sign) normalized so that each Y has unit square integral over the sphere.  Returned as
    ((N+1)^2, npts), row n*n + n + m."""
    u = np.atleast_2d(np.asarray(u, dtype=np.float64))
    x = np.clip(u[:, 2], -1.0, 1.0)
    s = np.sqrt(np.maximum(0.0, 1.0 - x * x))
    az = np.arctan2(u[:, 1], u[:, 0])
    p = {}
    p[(0, 0)] = np.full_like(x, 1.0 / math.sqrt(4.0 * math.pi))
    for m in range(1, N + 1):
        p[(m, m)] = math.sqrt((2.0 * m + 1.0) / (2.0 * m)) * s * p[(m - 1, m - 1)]
    for m in range(0, N):
        p[(m + 1, m)] = math.sqrt(2.0 * m + 3.0) * x * p[(m, m)]
    for m in range(0, N + 1):
        for n in range(m + 2, N + 1):
            a = math.sqrt((4.0 * n * n - 1.0) / (n * n - m * m))
            b = math.sqrt(((n - 1.0) ** 2 - m * m) / (4.0 * (n - 1.0) ** 2 - 1.0))
            p[(n, m)] = a * (x * p[(n - 1, m)] - b * p[(n - 2, m)])
    Y = np.empty((nmodes(N), x.size))
    r2 = math.sqrt(2.0)
    for n in range(N + 1):
        Y[n * n + n] = p[(n, 0)]
        for m in range(1, n + 1):
            Y[n * n + n + m] = r2 * p[(n, m)] * np.cos(m * az)
            Y[n * n + n - m] = r2 * p[(n, m)] * np.sin(m * az)
    return Y


def sphere_quadrature(nt: int):
    """Product rule on the unit sphere: nt Gauss-Legendre nodes in cos(theta) times 2 nt
    equally spaced azimuths; exact for polynomials of degree < 2 nt.  Returns (u, w)."""
    xg, wg = np.polynomial.legendre.leggauss(nt)
    nphi = 2 * nt
    az = 2.0 * math.pi * np.arange(nphi) / nphi
    X, A = np.meshgrid(xg, az, indexing="ij")
    W = np.repeat(wg[:, None], nphi, axis=1) * (2.0 * math.pi / nphi)
    S = np.sqrt(1.0 - X * X)
    u = np.stack([S * np.cos(A), S * np.sin(A), X], axis=-1).reshape(-1, 3)
    return u, W.reshape(-1)


def radial_out(n: np.ndarray, r: np.ndarray, kappa: float) -> np.ndarray:
    """f_n(r): k_n(kappa r), or r^-(n+1) without ions."""
    if kappa > 0:
        return special.spherical_kn(n, kappa * r)
    return r ** (-(n + 1.0))


def log_derivative_out(n: np.ndarray, R: float, kappa: float) -> np.ndarray:
    """f_n'(R)/f_n(R)."""
    if kappa > 0:
        return kappa * special.spherical_kn(n, kappa * R, derivative=True) / special.spherical_kn(n, kappa * R)
    return -(n + 1.0) / R


def log_derivative_reg(n: np.ndarray, R: float, kappa: float) -> np.ndarray:
    """g_n'(R)/g_n(R), g_n(r) = i_n(kappa r), or r^n without ions."""
    if kappa > 0:
        return kappa * special.spherical_in(n, kappa * R, derivative=True) / special.spherical_in(n, kappa * R)
    return n / R


@dataclass
class Spheres:
    centers: np.ndarray   # (ns, 3), Angstrom
    radii: np.ndarray     # (ns,)
    charges: np.ndarray   # (ns,), e

    def check(self):
        c, R = np.asarray(self.centers, float), np.asarray(self.radii, float)
        for i in range(len(R)):
            for j in range(i + 1, len(R)):
                if np.linalg.norm(c[i] - c[j]) <= R[i] + R[j]:
                    raise ValueError(f"spheres {i} and {j} overlap")


@dataclass
class Solution:
    sph: Spheres
    eps_in: float
    eps_out: float
    kappa: float
    N: int
    a: np.ndarray         # (ns, (N+1)^2) interior coefficients a_nm,i = L_nm,i R_i^n
    b: np.ndarray         # (ns, (N+1)^2) exterior coefficients b_nm,i = G_nm,i f_n(R_i)


def radial_out_all(N: int, r: np.ndarray, kappa: float) -> np.ndarray:
    """f_n(r) for n = 0..N, shape (N+1, len(r)): k_n(kappa r) by the upward recurrence
    k_{n+1}(x) = k_{n-1}(x) + (2n+1)/x k_n(x) from k_0 = (pi/2) e^-x / x and
    k_1 = (pi/2) e^-x (1/x + 1/x^2) (stable upward, same normalization as ``radial_out``),
    or r^-(n+1) without ions."""
    r = np.asarray(r, float)
    out = np.empty((N + 1, r.size))
    if kappa > 0:
        x = kappa * r
        out[0] = 0.5 * math.pi * np.exp(-x) / x
        if N >= 1:
            out[1] = out[0] * (1.0 + 1.0 / x)
        for n in range(1, N):
            out[n + 1] = out[n - 1] + (2.0 * n + 1.0) / x * out[n]
    else:
        out[0] = 1.0 / r
        for n in range(N):
            out[n + 1] = out[n] / r
    return out


def _offsphere_values(sph, j, pts, N, kappa, deg):
    """Values at points pts (npts, 3) of the scaled exterior basis of sphere j:
    f_n(rho_j)/f_n(R_j) Y_nm(u_j), shape (npts, (N+1)^2)."""
    d = pts - sph.centers[j]
    rho = np.linalg.norm(d, axis=1)
    Y = real_harmonics(N, d / rho[:, None])
    f = radial_out_all(N, rho, kappa) / radial_out_all(N, np.array([sph.radii[j]]), kappa)
    return (f[deg] * Y).T


def solve(sph: Spheres, eps_in: float, eps_out: float, kappa: float, N: int = 12, nt: int | None = None) -> Solution:
    """Coefficients of the multi-sphere solution with degrees up to N on every sphere.  The
    projections use nt x 2nt surface points (default N + 40: the other spheres' fields are
    smooth on each surface, their degree-k content falling like (R_i/|c_i - c_j|)^k)."""
    sph = Spheres(np.asarray(sph.centers, float), np.asarray(sph.radii, float), np.asarray(sph.charges, float))
    sph.check()
    ns, K = len(sph.radii), nmodes(N)
    deg = mode_degree(N)
    u, w = sphere_quadrature(nt if nt else N + 40)
    YW = real_harmonics(N, u) * w[None, :]          # (K, npts)
    # P[iK + k, jK + k'] = projection on mode k of sphere i of mode k' of sphere j (j != i)
    P = np.zeros((ns * K, ns * K))
    alpha = np.empty(ns * K)
    beta = np.empty(ns * K)
    rhs = np.zeros(ns * K)
    for i in range(ns):
        Ri = sph.radii[i]
        alpha[i * K:(i + 1) * K] = eps_in * deg / Ri - eps_out * log_derivative_out(deg, Ri, kappa)
        beta[i * K:(i + 1) * K] = eps_in * deg / Ri - eps_out * log_derivative_reg(deg, Ri, kappa)
        pts = sph.centers[i] + Ri * u
        for j in range(ns):
            if j != i:
                P[i * K:(i + 1) * K, j * K:(j + 1) * K] = YW @ _offsphere_values(sph, j, pts, N, kappa, deg)
        rhs[i * K] = sph.charges[i] * math.sqrt(4.0 * math.pi) / Ri ** 2
    A = beta[:, None] * P
    A[np.diag_indices_from(A)] += alpha
    bv = np.linalg.solve(A, rhs)
    del A
    # interior coefficients from condition (1)
    a = (bv + P @ bv).reshape(ns, K)
    b = bv.reshape(ns, K)
    a[:, 0] -= sph.charges * math.sqrt(4.0 * math.pi) / (eps_in * sph.radii)
    return Solution(sph, eps_in, eps_out, kappa, N, a, b)


def exterior_potential(sol: Solution, x: np.ndarray) -> np.ndarray:
    """Sum of every sphere's exterior expansion at points x (npts, 3): the potential outside
    the spheres (the expansions are defined at any point but the centres)."""
    x = np.atleast_2d(np.asarray(x, float))
    deg = mode_degree(sol.N)
    out = np.zeros(len(x))
    for j in range(len(sol.sph.radii)):
        out += _offsphere_values(sol.sph, j, x, sol.N, sol.kappa, deg) @ sol.b[j]
    return out


def interior_potential(sol: Solution, i: int, x: np.ndarray) -> np.ndarray:
    """Interior expansion of sphere i at points x (npts, 3), the charge's own Coulomb term
    included: the potential inside sphere i (defined at any point but its centre)."""
    x = np.atleast_2d(np.asarray(x, float))
    sph = sol.sph
    deg = mode_degree(sol.N)
    d = x - sph.centers[i]
    rho = np.linalg.norm(d, axis=1)
    Y = real_harmonics(sol.N, d / rho[:, None])
    scale = (rho[None, :] / sph.radii[i]) ** deg[:, None]
    return (sol.a[i][:, None] * scale * Y).sum(axis=0) + sph.charges[i] / (sol.eps_in * rho)


def potential(sol: Solution, x: np.ndarray) -> np.ndarray:
    """The potential (e/Angstrom) at points x (npts, 3), none at a sphere centre: the
    interior expansion inside a sphere, the exterior sum outside."""
    x = np.atleast_2d(np.asarray(x, float))
    sph = sol.sph
    inside = np.full(len(x), -1)
    for i in range(len(sph.radii)):
        inside[np.linalg.norm(x - sph.centers[i], axis=1) < sph.radii[i]] = i
    out = np.zeros(len(x))
    m = inside < 0
    if m.any():
        out[m] = exterior_potential(sol, x[m])
    for i in range(len(sph.radii)):
        mi = inside == i
        if mi.any():
            out[mi] = interior_potential(sol, i, x[mi])
    return out


def energies(sol: Solution, lB: float = 1.0) -> dict:
    """E, E_coul, E_pol, E_ion (times lB) and the reaction potential at every centre."""
    sph, N = sol.sph, sol.N
    ns = len(sph.radii)
    deg = mode_degree(N)
    q, c, R = sph.charges, sph.centers, sph.radii
    e_tot = 0.5 * float(np.sum(q * sol.a[:, 0])) / math.sqrt(4.0 * math.pi)
    phic = np.zeros(ns)
    for i in range(ns):
        for j in range(ns):
            if j != i:
                phic[i] += q[j] / (sol.eps_in * np.linalg.norm(c[i] - c[j]))
    e_coul = 0.5 * float(np.sum(q * phic))
    # polarization layer on each sphere and its potential at every centre
    fac = (1.0 / sol.eps_out - 1.0 / sol.eps_in) / (4.0 * math.pi)
    phip = np.zeros(ns)
    for i in range(ns):
        D = -sol.eps_in * deg * sol.a[i] / R[i]
        D[0] += q[i] * math.sqrt(4.0 * math.pi) / R[i] ** 2
        s = fac * D
        phip[i] += math.sqrt(4.0 * math.pi) * R[i] * s[0]
        for j in range(ns):
            if j == i:
                continue
            d = c[j] - c[i]
            dist = np.linalg.norm(d)
            Y = real_harmonics(N, (d / dist)[None, :])[:, 0]
            phip[j] += float(np.sum(s * 4.0 * math.pi * R[i] ** 2 * R[i] ** deg / ((2 * deg + 1) * dist ** (deg + 1)) * Y))
    e_pol = 0.5 * float(np.sum(q * phip))
    phi_reac = sol.a[:, 0] / math.sqrt(4.0 * math.pi) - phic
    return dict(e_total=lB * e_tot, e_coul=lB * e_coul, e_pol=lB * e_pol, e_ion=lB * (e_tot - e_coul - e_pol),
                phi_reac=lB * phi_reac, phi_pol=lB * phip)
