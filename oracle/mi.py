"""Matrix-inversion (MI) solver of the partial-wave LS equation (test infrastructure only).

Sec. 2.1 of the paper, read in reduced units without the 2/pi factor:
t(p',p) = U(p',p) + int_0^Lam dq q^2 U(p',q) t(q,p)/(p^2 - q^2 + i0).
The pole is removed by principal-value subtraction; the subtracted integral is
taken with N_Q Gauss-Legendre points on [0, Lam], and the on-shell point p is
appended to the basis.  With D_j = w_j q_j^2/(p^2 - q_j^2) (j <= N_Q) and
D_{N_Q+1} = -p^2 sum_j w_j/(p^2 - q_j^2) + (p/2) ln((Lam+p)/(Lam-p)) - i pi p/2
(the log is the finite-cut-off principal value of int_0^Lam dq/(p^2-q^2)),
the wave matrix F = 1 - U diag(D) gives F t = U, solved by LU (LAPACK gesv).
The K-matrix route drops the -i pi p/2 term and yields a real K with
S = (1 - i pi p K/2)(1 + i pi p K/2)^{-1}.

Pins: the Yamaguchi closed form at finite cut-off; S-matrix unitarity and
symmetry; agreement of the T- and K-matrix routes; N_Q convergence.
"""
from __future__ import annotations

import numpy as np


def _mesh(n_q: int, cutoff: float):
    x, w = np.polynomial.legendre.leggauss(n_q)
    return 0.5 * cutoff * (x + 1.0), 0.5 * cutoff * w


def solve(u_fn, p: float, n_q: int, cutoff: float, n_ch: int, kmatrix: bool = False) -> np.ndarray:
    """On-shell t_{l'l}(p,p) (n_ch x n_ch) for U given by u_fn(rows, cols).

    u_fn(p_row, p_col) must return the (n_ch*len(p_row)) x (n_ch*len(p_col))
    channel-major matrix.  With kmatrix=True the real K-matrix is returned.
    """
    if not 0.0 < p < cutoff:
        raise ValueError("on-shell momentum must lie in (0, cutoff)")
    q, w = _mesh(n_q, cutoff)
    pts = np.append(q, p)
    d = np.empty(n_q + 1, dtype=np.complex128)
    d[:n_q] = w * q * q / (p * p - q * q)
    d[n_q] = -p * p * np.sum(w / (p * p - q * q)) + 0.5 * p * np.log((cutoff + p) / (cutoff - p))
    if not kmatrix:
        d[n_q] -= 0.5j * np.pi * p
    else:
        d = d.real
    u = np.asarray(u_fn(pts, pts))
    dd = np.tile(d, n_ch)
    f = np.eye(u.shape[0]) - u * dd[None, :]
    t = np.linalg.solve(f, u)
    idx = np.array([a * (n_q + 1) + n_q for a in range(n_ch)])
    return t[np.ix_(idx, idx)]


def s_from_k(kmat: np.ndarray, p: float) -> np.ndarray:
    n_ch = kmat.shape[0]
    a = 0.5j * np.pi * p * kmat
    return (np.eye(n_ch) - a) @ np.linalg.inv(np.eye(n_ch) + a)
