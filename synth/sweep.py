"""Batched-sweep workload: every partial wave with J <= 6 for many parameter samples.

Stands in for the paper's neutron-proton cross-section sweeps with a chiral
potential (Sec. 5.1.1: J <= 6, about 20 channels; total cross sections at
T_lab up to 350 MeV).  A parameter sample is a 7-vector of Yukawa strengths in
MeV fm: three singlet (S = 0) central terms, three triplet (S = 1) central
terms (mu = 0.7, 1.5, 3.1 fm^-1 for both) and one tensor-like coupling
(mu = 0.7 fm^-1), drawn ~ N(mean, 0.1 |mean|).  The channel set holds every
(S, l, J) with J <= 6 once:

* singlet  1S0 1P1 1D2 1F3 1G4 1H5 1I6      (l = J, S = 0; singlet terms)
* triplet  3P0 3P1 3D2 3F3 3G4 3H5 3I6      (l = 1 for 3P0, else l = J; triplet terms)
* coupled  3S1-3D1 ... 3H6-3K6              (l = J -+ 1, J = 1..6; triplet
           terms on both diagonal blocks, the tensor term off-diagonal)

Each item draws its N_WP uniformly from {50, 100, 150}; grids are the bounded
tan^2 mesh on [0, 4] fm^-1 with 8 Gauss points per bin.  Every potential is an
affine combination of fixed unit-strength terms, so a term list per
(channel, grid) plus the item's coefficients define it completely.
"""
from __future__ import annotations

import numpy as np

from . import configs, grids, potentials

WORKLOAD = "sweep"
SEED_INDEX = 2
N_WP_CHOICES = (50, 100, 150)
K_MAX = 4.0
N_GAUSS = 8
TLAB = np.linspace(1.0, 350.0, 30)

SINGLET_MEANS = (-10.0, -420.0, 1500.0)   # no 1S0 bound state at the means
TRIPLET_MEANS = configs.YUKAWA_MEANS       # one 3S1-3D1 bound state
PARAM_MEANS = np.array(SINGLET_MEANS + TRIPLET_MEANS + (configs.TENSOR_MEAN,))

#: (name, n_ch, J, S, l of the first orbital channel)
CHANNELS = (
    [(f"1{'SPDFGHI'[J]}{J}", 1, J, 0, J) for J in range(7)]
    + [("3P0", 1, 0, 1, 1)] + [(f"3{'SPDFGHI'[J]}{J}", 1, J, 1, J) for J in range(1, 7)]
    + [(f"3{'SPDFGHIK'[J - 1]}{J}-3{'SPDFGHIK'[J + 1]}{J}", 2, J, 1, J - 1) for J in range(1, 7)]
)


def _rng(sample_id: int, channel_id: int) -> np.random.Generator:
    base = configs.BASE_SEED + SEED_INDEX
    return np.random.default_rng(np.random.SeedSequence([base, int(sample_id), int(channel_id)]))


def sample_params(sample_id: int) -> np.ndarray:
    """The 7 strengths (MeV fm) of one parameter sample."""
    return _rng(sample_id, 0).normal(PARAM_MEANS, 0.1 * np.abs(PARAM_MEANS))


def item_nwp(sample_id: int, channel: int) -> int:
    """N_WP of the item (sample, channel), uniform over N_WP_CHOICES."""
    return int(_rng(sample_id, 1 + channel).choice(N_WP_CHOICES))


def grid_bounds(n_wp: int) -> np.ndarray:
    return grids.tan2_bounded(n_wp, K_MAX)


def term_index(channel: int) -> list:
    """Positions in the 7-vector of the channel's term coefficients."""
    _, n_ch, _, S, _ = CHANNELS[channel]
    if n_ch == 2:
        return [3, 4, 5, 6]
    return [0, 1, 2] if S == 0 else [3, 4, 5]


class TermCache:
    """Unit-strength fine-mesh terms per (node set, channel), built once.

    Legendre Q_l for all l <= 7 at one (node set, mu) come from a single
    downward recursion, so the central terms of every channel share it.
    """

    def __init__(self):
        self._q = {}
        self._t = {}

    def _central(self, key, nodes, l, mu):
        qk = (key, mu)
        if qk not in self._q:
            pr, pc = nodes[:, None], nodes[None, :]
            zm1 = ((pr - pc) ** 2 + mu * mu) / (2.0 * pr * pc)
            ql = potentials.legendre_q(7, zm1)
            pref = potentials.RED_PER_MEV / (np.pi * pr * pc)
            self._q[qk] = [pref * q for q in ql]
        return self._q[qk][l]

    def terms(self, key, nodes: np.ndarray, channel: int) -> list:
        """Fine-mesh matrices (M or 2M square) with unit coefficients."""
        tk = (key, channel)
        if tk in self._t:
            return self._t[tk]
        _, n_ch, J, _, l = CHANNELS[channel]
        m = nodes.size
        out = []
        if n_ch == 1:
            out = [self._central(key, nodes, l, mu) for mu in configs.YUKAWA_MU]
        else:
            z = np.zeros((m, m))
            for mu in configs.YUKAWA_MU:
                out.append(potentials.coupled_matrix(self._central(key, nodes, J - 1, mu), z,
                                                     self._central(key, nodes, J + 1, mu)))
            t01 = potentials.tensor_block(J, nodes, nodes, 1.0, configs.TENSOR_MU)
            out.append(potentials.coupled_matrix(z, t01, z))
        self._t[tk] = out
        return out


def items(n_samples: int, sample0: int = 0) -> list:
    """(sample_id, channel, n_wp) for every item of the sweep, sample-major."""
    return [(s, c, item_nwp(s, c)) for s in range(sample0, sample0 + n_samples) for c in range(len(CHANNELS))]


def coefficients(sample_id: int, channel: int) -> np.ndarray:
    return sample_params(sample_id)[term_index(channel)]
