"""Binding energies ddG = dG_complex - dG_1 - dG_2 (paper Sect. 6.2, binding energy calculation): CPU pins.

* the Coulomb part: the oracle's pair sum is additive, so ddG_coul is exactly the sum over
  the pairs that straddle the two parts, and for two point charges it is the closed form
  l_B q1 q2 / (eps_in r)
* the ABI's pb_binding_ddg is the component-wise difference (host arithmetic, no device)
* the synthetic complexes keep the two parts' atom centres at least the stated gap apart
"""
import ctypes as C
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2502_09323_amd import inputs as I


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build()


def test_coulomb_part_is_the_cross_pair_sum():
    cpx, rec, lig = I.binding_complex(5, n_rec=120, n_lig=30, R_rec=7.0, R_lig=3.5)
    eps_in = 2.0
    ddg = O.coulomb(cpx, eps_in) - O.coulomb(rec, eps_in) - O.coulomb(lig, eps_in)
    d = np.linalg.norm(rec.xyz[:, None, :] - lig.xyz[None, :, :], axis=2)
    cross = float(np.sum(rec.charge[:, None] * lig.charge[None, :] / d)) / eps_in
    assert abs(ddg - cross) <= 1e-12 * max(abs(cross), 1.0)
    assert d.min() >= 1.0 - 1e-12


def test_two_point_charges_closed_form():
    a = I.Molecule(np.array([[0.0, 0.0, 0.0]]), np.array([1.5]), np.array([0.7]))
    b = I.Molecule(np.array([[3.25, 0.0, 0.0]]), np.array([1.5]), np.array([-1.3]))
    ab = I.Molecule(np.concatenate([a.xyz, b.xyz]), np.concatenate([a.radius, b.radius]),
                    np.concatenate([a.charge, b.charge]))
    eps_in = 4.0
    ddg = O.coulomb(ab, eps_in) - O.coulomb(a, eps_in) - O.coulomb(b, eps_in)
    assert ddg == pytest.approx(0.7 * -1.3 / (eps_in * 3.25), rel=1e-15)


def test_abi_binding_ddg_is_the_componentwise_difference():
    lib = C.CDLL(os.path.join(os.path.dirname(__file__), "..", "paper_2502_09323_amd", "libpb.so"))

    class E(C.Structure):
        _fields_ = [("e_coul", C.c_double), ("e_pol", C.c_double), ("e_ion", C.c_double),
                    ("e_solv", C.c_double), ("e_total", C.c_double), ("q_pol_total", C.c_double),
                    ("area_total", C.c_double), ("n_cut", C.c_int64), ("t_energy_s", C.c_double)]

    class Bo(C.Structure):
        _fields_ = [("ddg_total", C.c_double), ("ddg_coul", C.c_double), ("ddg_pol", C.c_double),
                    ("ddg_ion", C.c_double)]

    def e(coul, pol, ion):
        return E(coul, pol, ion, pol + ion, coul + pol + ion, 0.0, 0.0, 0, 0.0)

    c, p1, p2, out = e(-10.0, -50.0, -2.0), e(-6.0, -40.0, -1.5), e(-1.0, -12.0, -0.25), Bo()
    lib.pb_binding_ddg.argtypes = [C.POINTER(E), C.POINTER(E), C.POINTER(E), C.POINTER(Bo)]
    assert lib.pb_binding_ddg(C.byref(c), C.byref(p1), C.byref(p2), C.byref(out)) == 0
    assert (out.ddg_coul, out.ddg_pol, out.ddg_ion) == (-3.0, 2.0, -0.25)
    assert out.ddg_total == (-62.0) - (-47.5) - (-13.25)
    assert lib.pb_binding_ddg(None, C.byref(p1), C.byref(p2), C.byref(out)) != 0


def test_workload_protocol():
    w = I.binding_workload(n_complex=2, n_disp=3, h=0.5)
    assert len(w) == 2 * 3 * 3
    for c in range(2):
        grids = {id(g) for cc, _, _, _, g in w if cc == c}
        assert len(grids) == 1   # one grid per complex, shared by every displacement and part
    # the displacement is common to the three parts and within a cube of half the spacing
    cpx0 = [m for cc, k, p, m, _ in w if cc == 0 and p == "c"]
    base, _, _ = I.binding_complex(2506 * 1000)
    for m in cpx0:
        d = m.xyz - base.xyz
        assert np.allclose(d, d[0]) and np.all(np.abs(d[0]) <= 0.125 + 1e-12)
