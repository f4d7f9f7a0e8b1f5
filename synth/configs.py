"""Seeded synthetic workloads standing in for the paper's chiral-potential inputs.

The paper's results use a chiral NN potential that is not available here; these
workloads reproduce its shapes instead (channel structure, N_WP range, energy
range, bound-state content).  Every draw is seeded: the base seed of workload
``idx`` is 20210601 + idx, and item streams derive from
SeedSequence([base, sample_id, channel_id]).

Workloads
---------
* ``yamaguchi_s``      : uncoupled S-wave, Yamaguchi separable potential,
                         beta = 1.4 fm^-1, lam ~ U[0.5, 2.0] fm^-3, N_WP = 50,
                         momenta on [0, 4] fm^-1 (tan^2 mesh), 8 Gauss points/bin.
* ``coupled_yukawa``   : coupled l = 0/2, J = 1, S = 1; three central Yukawa
                         terms mu = (0.7, 1.5, 3.1) fm^-1 with coefficient means
                         (-10, -600, +1500) MeV fm plus an off-diagonal
                         tensor-like term (mean -10 MeV fm, mu = 0.7 fm^-1);
                         draws ~ N(mean, 0.1 |mean|); N_WP = 100 (200 x 200 H).
"""
from __future__ import annotations

import numpy as np

from . import grids, potentials

BASE_SEED = 20210601

YAMAGUCHI_BETA = 1.4
YAMAGUCHI_LAM_RANGE = (0.5, 2.0)

YUKAWA_MU = (0.7, 1.5, 3.1)
YUKAWA_MEANS = (-10.0, -600.0, 1500.0)
TENSOR_MU = 0.7
TENSOR_MEAN = -10.0

#: index of each workload in the seed scheme
WORKLOAD_INDEX = {"yamaguchi_s": 0, "coupled_yukawa": 1}


def item_rng(workload: str, sample_id: int, channel_id: int = 0) -> np.random.Generator:
    base = BASE_SEED + WORKLOAD_INDEX[workload]
    return np.random.default_rng(np.random.SeedSequence([base, int(sample_id), int(channel_id)]))


def yamaguchi_lambda(sample_id: int) -> float:
    lo, hi = YAMAGUCHI_LAM_RANGE
    return float(item_rng("yamaguchi_s", sample_id).uniform(lo, hi))


def yukawa_coefficients(sample_id: int, channel_id: int = 0) -> np.ndarray:
    """Four coefficients in MeV fm: three central terms then the tensor term."""
    rng = item_rng("coupled_yukawa", sample_id, channel_id)
    means = np.array(YUKAWA_MEANS + (TENSOR_MEAN,))
    return rng.normal(means, 0.1 * np.abs(means))


def coupled_yukawa_terms(nodes: np.ndarray, J: int = 1) -> list:
    """Unit-coefficient (1 MeV fm) fine-mesh matrices of the four terms.

    The potential of a sample with coefficients c is sum_t c[t] * terms[t]; each
    term is a (2M x 2M) channel-major matrix for l = J-1 (rows/cols 0..M-1) and
    l = J+1 (M..2M-1) at the given momenta.
    """
    m = nodes.size
    terms = []
    for mu in YUKAWA_MU:
        u00 = potentials.yukawa_central(J - 1, nodes, nodes, 1.0, mu)
        u11 = potentials.yukawa_central(J + 1, nodes, nodes, 1.0, mu)
        terms.append(potentials.coupled_matrix(u00, np.zeros((m, m)), u11))
    t01 = potentials.tensor_block(J, nodes, nodes, 1.0, TENSOR_MU)
    terms.append(potentials.coupled_matrix(np.zeros((m, m)), t01, np.zeros((m, m))))
    return terms


def grid(workload: str) -> np.ndarray:
    if workload == "yamaguchi_s":
        return grids.tan2_bounded(50, 4.0)
    if workload == "coupled_yukawa":
        return grids.tan2_bounded(100, 4.0)
    raise KeyError(workload)


N_GAUSS = 8
