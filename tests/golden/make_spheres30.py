"""Write ``spheres30_analytic.txt``: the analytic energies and reaction potentials of the
30-sphere cluster used by the GPU many-sphere test (seed 2506, eps 2/80, 0.145 M, 298.15 K),
from the many-sphere reference with degrees up to 14 on every sphere (the energies change
by about 1e-10 relative from degree 10 to 14).  Calls only the oracle and the input
generator.  Run from the repository root: python tests/golden/make_spheres30.py"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O      # noqa: E402
from oracle import spheres as S     # noqa: E402
from paper_2502_09323_amd import inputs as I   # noqa: E402

SEED, N_SPH, DEGREE = 2506, 30, 14


def main():
    m = I.sphere_cluster(N_SPH, SEED)
    lB, kD = O.constants(298.15, 0.145, 80.0)
    e = S.energies(S.solve(S.Spheres(m.xyz, m.radius, m.charge), 2.0, 80.0, kD, N=DEGREE), lB)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "spheres30_analytic.txt")
    with open(out, "w") as f:
        f.write("# Analytic many-sphere solution (paper Sect. \"An analytical benchmark\"), written by\n")
        f.write("# make_spheres30.py from oracle/spheres.py: inputs.sphere_cluster(30, 2506), eps_in 2,\n")
        f.write("# eps_out 80, 0.145 M, 298.15 K, degree 14.  Energies in kT; phi_reac_i is the\n")
        f.write("# reaction potential (polarization + ions) at the centre of sphere i, in kT/e.\n")
        for k in ("e_total", "e_coul", "e_pol", "e_ion"):
            f.write(f"{k} {e[k]:.15e}\n")
        for i, v in enumerate(e["phi_reac"]):
            f.write(f"phi_reac_{i} {v:.15e}\n")
    print("wrote", out)


if __name__ == "__main__":
    main()
