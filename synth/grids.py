"""Momentum bin boundaries k_0 = 0 < k_1 < ... < k_N (fm^-1).

Two mesh kinds are provided:

* ``tan2_bounded`` -- k_j = k_max * tan^2(j*pi/(4N)), j = 0..N.  This is the
  sparseness-degree-2 tangent distribution of the paper's Chebyshev mesh
  (Sec. 3.2, step 1, Eq. for y_j) re-indexed so that it ends exactly at a
  finite cut-off k_N = k_max; bins are dense below 1 fm^-1.
* ``chebyshev`` -- the paper-literal distribution y_j = alpha*tan^t((2j-1)pi/(4N)),
  j = 1..N, with y_0 = 0 (Sec. 3.2, step 1).  alpha is given in MeV and
  converted to a momentum with hbar*c.
"""
import numpy as np

HBARC_MEV_FM = 197.327


def tan2_bounded(n_wp: int, k_max: float = 4.0) -> np.ndarray:
    if n_wp < 2:
        raise ValueError("n_wp must be >= 2")
    j = np.arange(n_wp + 1, dtype=np.float64)
    k = k_max * np.tan(j * np.pi / (4.0 * n_wp)) ** 2
    k[0] = 0.0
    k[-1] = k_max
    return k


def chebyshev(n_wp: int, alpha_mev: float = 100.0, t: float = 2.0) -> np.ndarray:
    if n_wp < 2:
        raise ValueError("n_wp must be >= 2")
    j = np.arange(1, n_wp + 1, dtype=np.float64)
    y = (alpha_mev / HBARC_MEV_FM) * np.tan((2.0 * j - 1.0) * np.pi / (4.0 * n_wp)) ** t
    return np.concatenate([[0.0], y])
