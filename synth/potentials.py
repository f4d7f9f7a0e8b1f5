"""Partial-wave potentials in reduced units, evaluated at caller-given momenta.

Units: momenta in fm^-1, the reduced potential U = m_N V / (hbar c)^2 in fm,
so that the partial-wave Lippmann-Schwinger kernel reads
U(p',q) q^2 dq / (p^2 - q^2 + i0) with states normalised as
<k'|k> = delta(k'-k)/(k'k) (Sec. 2, the momentum-space partial-wave LS
equation and the state normalisation stated after it).

Potentials provided (inputs only -- the wave-packet method never appears here):

* Yamaguchi separable:  U(p',p) = -lam g(p') g(p),  g(p) = 1/(p^2 + beta^2).
* Central Yukawa term V(r) = C exp(-mu r)/r, projected on orbital l:
  U_l(p',p) = (2/pi) int r^2 dr j_l(p'r) U(r) j_l(pr) = c Q_l(z) / (pi p p'),
  z = (p^2 + p'^2 + mu^2)/(2 p p'), c = m_N C/(hbar c)^2.  Q_l is the Legendre
  function of the second kind, evaluated by downward continued-fraction ratios
  normalised to Q_0 (the minimal solution of the three-term recurrence).
* Tensor-like off-diagonal block between l = J-1 and l = J+1:
  U_{J-1,J+1}(p',p) = (2/pi) * 6 sqrt(J(J+1))/(2J+1)
                      * int r^2 dr j_{J-1}(p'r) U_T(r) j_{J+1}(pr),
  U_T(r) = c_t exp(-mu r)(1 + 3/(mu r) + 3/(mu r)^2)/r, by composite
  Gauss-Legendre radial quadrature; U_{J+1,J-1}(p',p) = U_{J-1,J+1}(p,p').
"""
from __future__ import annotations

import numpy as np
from scipy.special import spherical_jn

M_N_MEV = 938.918
HBARC_MEV_FM = 197.327
#: m_N/(hbar c)^2 in MeV^-1 fm^-2: converts V [MeV] to U(r) [fm^-2].
RED_PER_MEV = M_N_MEV / HBARC_MEV_FM ** 2


def yamaguchi(p_row, p_col, lam: float, beta: float) -> np.ndarray:
    """U(p',p) = -lam g(p') g(p) with g = 1/(p^2+beta^2); lam in fm^-3."""
    g_r = 1.0 / (np.asarray(p_row, float) ** 2 + beta * beta)
    g_c = 1.0 / (np.asarray(p_col, float) ** 2 + beta * beta)
    return -lam * np.outer(g_r, g_c)


def legendre_q(lmax: int, zm1: np.ndarray) -> list:
    """Q_0..Q_lmax of the second kind at z = 1 + zm1 (zm1 > 0), any shape.

    Q_0 = 0.5*log((z+1)/(z-1)) is taken as log1p(2/zm1)/2.  Ratios
    r_l = Q_l/Q_{l-1} obey r_l = l/((2l+1) z - (l+1) r_{l+1}) and are run
    downward from r_{L+1} = 0, with L past lmax far enough that the start
    error has decayed below double precision.
    """
    zm1 = np.asarray(zm1, dtype=np.float64)
    if np.any(zm1 <= 0):
        raise ValueError("legendre_q needs z > 1")
    shape = zm1.shape
    zm1 = zm1.ravel()
    z = 1.0 + zm1
    q0 = 0.5 * np.log1p(2.0 / zm1)
    if lmax == 0:
        return [q0.reshape(shape)]
    # decay rate of the minimal solution: Q_{l+1}/Q_l -> exp(-x); points are
    # processed in groups of similar x, each started deep enough for its
    # smallest x
    x = np.arccosh(z)
    order = np.argsort(x)
    ratios = np.empty((lmax + 1, z.size))
    chunk = 65536
    for c0 in range(0, z.size, chunk):
        idx = order[c0:c0 + chunk]
        zc = z[idx]
        extra = int(np.ceil(40.0 / max(float(x[idx[0]]), 1e-3)))
        r = np.zeros_like(zc)
        for l in range(lmax + min(extra, 20000), 0, -1):
            r = l / ((2 * l + 1) * zc - (l + 1) * r)
            if l <= lmax:
                ratios[l, idx] = r
    out = [q0.reshape(shape)]
    q = q0
    for l in range(1, lmax + 1):
        q = q * ratios[l]
        out.append(q.reshape(shape))
    return out


def yukawa_central(l: int, p_row, p_col, c_mev_fm: float, mu: float) -> np.ndarray:
    """Orbital-l projection of C exp(-mu r)/r (C in MeV fm, mu in fm^-1)."""
    pr = np.asarray(p_row, float)[:, None]
    pc = np.asarray(p_col, float)[None, :]
    zm1 = ((pr - pc) ** 2 + mu * mu) / (2.0 * pr * pc)
    ql = legendre_q(l, zm1)[l]
    c = RED_PER_MEV * c_mev_fm
    return c * ql / (np.pi * pr * pc)


def _radial_rule(mu: float, panel: float = 0.5, npts: int = 16):
    r_max = 40.0 / mu
    n_panels = int(np.ceil(r_max / panel))
    x, w = np.polynomial.legendre.leggauss(npts)
    edges = np.linspace(0.0, n_panels * panel, n_panels + 1)
    a, b = edges[:-1, None], edges[1:, None]
    r = (0.5 * (b - a) * x[None, :] + 0.5 * (b + a)).ravel()
    wr = (0.5 * (b - a) * w[None, :]).ravel()
    return r, wr


def tensor_block(J: int, p_row, p_col, c_mev_fm: float, mu: float) -> np.ndarray:
    """U_{J-1,J+1}(p',p) of the tensor-like term (rows p' in l=J-1, cols p in l=J+1)."""
    if J < 1:
        raise ValueError("tensor coupling needs J >= 1")
    r, wr = _radial_rule(mu)
    x = mu * r
    c = RED_PER_MEV * c_mev_fm
    ut = c * np.exp(-x) * (1.0 + 3.0 / x + 3.0 / (x * x)) / r
    a = spherical_jn(J - 1, np.outer(np.asarray(p_row, float), r))
    b = spherical_jn(J + 1, np.outer(np.asarray(p_col, float), r))
    f = 6.0 * np.sqrt(J * (J + 1.0)) / (2.0 * J + 1.0)
    return (2.0 / np.pi) * f * (a * (wr * r * r * ut)[None, :]) @ b.T


def coupled_matrix(blocks00, blocks01, blocks11) -> np.ndarray:
    """Assemble the (2M x 2M) coupled-channel matrix, channel-major ordering.

    Row (a, alpha): a = 0 for l = J-1, a = 1 for l = J+1; alpha = node index.
    The lower-left block is the transpose of the upper-right block, which is
    U_{J+1,J-1}(p',p) = U_{J-1,J+1}(p,p').
    """
    m = blocks00.shape[0]
    u = np.empty((2 * m, 2 * m))
    u[:m, :m] = blocks00
    u[:m, m:] = blocks01
    u[m:, :m] = blocks01.T
    u[m:, m:] = blocks11
    return u
