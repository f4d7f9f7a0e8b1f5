"""Closed-form on-shell T-matrix of the Yamaguchi separable potential (test infrastructure only).

For U(p',p) = -lam g(p') g(p), g(p) = 1/(p^2 + beta^2), the LS equation of
Sec. 2 (reduced units, integration over [0, Lam]) is solved by
t(p',p) = g(p') tau g(p) with tau = -lam/(1 + lam J(p)) and
J(p) = int_0^Lam dq q^2 g(q)^2/(p^2 - q^2 + i0).

J is written in closed form.  With x = q^2,
x/((x+b^2)^2 (p^2-x)) = C/(x+b^2) - b^2/((p^2+b^2)(x+b^2)^2) + C/(p^2-x),
C = p^2/(p^2+b^2)^2, so J_inf(p) = -pi/(4 b (b - i p)^2) and the finite cut-off
value subtracts the regular tail int_Lam^inf, which is elementary.

Pins: J against principal-value quadrature; the Lam -> inf effective-range
form p cot(delta) = 2(b^2+p^2)^2/(pi lam) - (b^2 - p^2)/(2b); the MI solver.
"""
from __future__ import annotations

import numpy as np


def j_integral(p, beta: float, cutoff=None):
    p = np.asarray(p, dtype=np.float64)
    b = beta
    j_inf = -np.pi / (4.0 * b * (b - 1j * p) ** 2)
    if cutoff is None:
        return j_inf
    lam_c = float(cutoff)
    s = p * p + b * b
    c = p * p / (s * s)
    at = 0.5 * np.pi - np.arctan(lam_c / b)
    tail = (c / b) * at \
        - (b * b / s) * (at / (2.0 * b ** 3) - lam_c / (2.0 * b * b * (lam_c * lam_c + b * b))) \
        - (c / (2.0 * p)) * np.log((lam_c + p) / (lam_c - p))
    return j_inf - tail


def t_onshell(p, lam: float, beta: float, cutoff=None):
    p = np.asarray(p, dtype=np.float64)
    g = 1.0 / (p * p + beta * beta)
    tau = -lam / (1.0 + lam * j_integral(p, beta, cutoff))
    return g * g * tau


def phase_shift_deg(p, lam: float, beta: float, cutoff=None):
    """Principal-value phase shift in (-90, 90] degrees from S = 1 - i pi p t."""
    p = np.asarray(p, dtype=np.float64)
    s = 1.0 - 1j * np.pi * p * t_onshell(p, lam, beta, cutoff)
    return np.degrees(0.5 * np.angle(s))
