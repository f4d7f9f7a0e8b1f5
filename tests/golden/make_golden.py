"""Write the oracle regression fixtures in this folder.

Calls only ``oracle`` and ``synth``.  The fixtures freeze the FP64 oracle's
output for the first sample of the two small workloads, so that any later
change to the oracle's arithmetic shows up as a failing test and has to be
justified by the passage of the paper (or the documented reading of it) that
motivates it.  Run from the repository root:  python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import wpcd  # noqa: E402
from synth import configs, potentials  # noqa: E402


def yamaguchi_case():
    k = configs.grid("yamaguchi_s")
    x, _ = wpcd.gauss_nodes(k, configs.N_GAUSS)
    lam = configs.yamaguchi_lambda(0)
    r = wpcd.solve_channel(k, configs.N_GAUSS, potentials.yamaguchi(x, x, lam, configs.YAMAGUCHI_BETA), 1)
    return np.column_stack([r["evals"], r["delta"][:, 0]])


def coupled_case():
    k = configs.grid("coupled_yukawa")
    x, _ = wpcd.gauss_nodes(k, configs.N_GAUSS)
    c = configs.yukawa_coefficients(0)
    u = sum(ci * ti for ci, ti in zip(c, configs.coupled_yukawa_terms(x)))
    r = wpcd.solve_channel(k, configs.N_GAUSS, u, 2)
    return r["evals"], np.column_stack([r["delta"], r["mix"]])


if __name__ == "__main__":
    hdr = "oracle regression fixture; written by tests/golden/make_golden.py from oracle/ only\n"
    np.savetxt(os.path.join(HERE, "yamaguchi_s_sample0.txt"), yamaguchi_case(), fmt="%.17e",
               header=hdr + "Yamaguchi S-wave, N_WP=50, sample 0: columns eigenvalue [fm^-2], delta [deg] per bin")
    ev, ph = coupled_case()
    np.savetxt(os.path.join(HERE, "coupled_yukawa_sample0_evals.txt"), ev, fmt="%.17e",
               header=hdr + "coupled Yukawa J=1, N_WP=100, sample 0: eigenvalues [fm^-2]")
    np.savetxt(os.path.join(HERE, "coupled_yukawa_sample0_phases.txt"), ph, fmt="%.17e",
               header=hdr + "coupled Yukawa J=1, N_WP=100, sample 0: delta_-, delta_+, eps_1 [deg] per bin")
