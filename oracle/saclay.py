"""Spin-scattering matrix, Saclay amplitudes and dsigma/dOmega (test infrastructure only).

App. A of the paper, read as follows (each reading pinned in tests/test_oracle_pins.py):

* M-matrix in partial waves, for c.m. momentum p and scattering angle theta
  (phi = 0, incoming momentum along z):
    M^s_{ms,ms'}(theta) = (2 pi/(i p)) sum_{J,l,l'} w sqrt((2l+1)/(4 pi))
        Y_{l'}^{ms-ms'}(theta, 0) <l' ms-ms', s ms'|J ms> <l 0, s ms|J ms>
        (S^{sJ}_{l'l} - delta_{l'l}),
  with ms the incoming and ms' the outgoing spin projection.  The channel
  weight w = 1 counts every (s, l, J) once, as for neutron-proton scattering
  with isospin conservation; the paper's factor [1 - (-1)^(l+s+T_z)] is the
  identical-particle form (it would remove the isospin-1 states of np at
  T_z = 0).  Y and the Clebsch-Gordan coefficients use the Condon-Shortley
  phase.  S^{sJ} is the on-shell S-matrix of the channel, S = 1 - i pi p t in
  the units used everywhere here.
* Saclay amplitudes, from the spin-projected elements (with n = p x p'/|..|,
  m and l as printed; the spin-orbit term is e (sigma_1 + sigma_2).n):
    a = (M^1_{11} + M^1_{00} - M^1_{1,-1})/2
    b = (M^1_{11} + M^0_{00} + M^1_{1,-1})/2
    c = (M^1_{11} - M^0_{00} + M^1_{1,-1})/2
    d = -(M^1_{10} + M^1_{01})/(sqrt(2) sin theta)  = (M^1_{00} - a)/cos theta
    e = i (M^1_{01} - M^1_{10})/sqrt(2)
  The printed a carries +M^1_{1,-1} and the printed e half this value and the
  opposite sign; with the printed forms the identity
  (1/4) Tr(M M^+) = (1/2)(|a|^2 + ... + |e|^2) that the paper states for
  dsigma/dOmega fails, with these it holds (and the operator form of M rebuilt
  from them reproduces every M^s element).  Both forms of d are exact; the one
  with the larger denominator is used.
* dsigma/dOmega = (|a|^2 + |b|^2 + |c|^2 + |d|^2 + |e|^2)/2 and
  sigma_tot = (2 pi/p) Im(a + b) at theta = 0; 1 fm^2 = 10 mb.
"""
from __future__ import annotations

import math

import numpy as np

from . import observables


def clebsch_gordan(j1: int, m1: int, j2: int, m2: int, J: int, M: int) -> float:
    """<j1 m1, j2 m2|J M> for integer angular momenta (Racah's closed form)."""
    if m1 + m2 != M or abs(m1) > j1 or abs(m2) > j2 or abs(M) > J:
        return 0.0
    if J < abs(j1 - j2) or J > j1 + j2:
        return 0.0
    f = math.factorial
    pre = math.sqrt((2 * J + 1) * f(J + j1 - j2) * f(J - j1 + j2) * f(j1 + j2 - J) / f(j1 + j2 + J + 1))
    pre *= math.sqrt(f(J + M) * f(J - M) * f(j1 - m1) * f(j1 + m1) * f(j2 - m2) * f(j2 + m2))
    s = 0.0
    for k in range(0, j1 + j2 - J + 1):
        d = [k, j1 + j2 - J - k, j1 - m1 - k, j2 + m2 - k, J - j2 + m1 + k, J - j1 - m2 + k]
        if min(d) < 0:
            continue
        s += (-1) ** k / math.prod(f(x) for x in d)
    return pre * s


def sph_harm_theta(l: int, m: int, theta) -> np.ndarray:
    """Y_l^m(theta, phi = 0) with the Condon-Shortley phase (real at phi = 0).

    P_l^m (no phase) by the upward recurrence in l from P_m^m = (2m-1)!! sin^m;
    Y_l^m = (-1)^m sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) P_l^m(cos theta),
    Y_l^{-m} = (-1)^m Y_l^m.
    """
    am = abs(m)
    if am > l:
        return np.zeros_like(np.asarray(theta, dtype=np.float64))
    x = np.cos(np.asarray(theta, dtype=np.float64))
    sx = np.sin(np.asarray(theta, dtype=np.float64))
    pmm = np.ones_like(x)
    for k in range(1, am + 1):
        pmm = pmm * (2 * k - 1) * sx
    if l == am:
        plm = pmm
    else:
        p1 = x * (2 * am + 1) * pmm
        p0 = pmm
        for ll in range(am + 2, l + 1):
            p0, p1 = p1, ((2 * ll - 1) * x * p1 - (ll + am - 1) * p0) / (ll - am)
        plm = p1
    norm = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
    y = (-1) ** am * norm * plm
    return y if m >= 0 else (-1) ** am * y


SPIN_ELEMENTS = ((0, 0, 0), (1, 1, 1), (1, 1, 0), (1, 1, -1), (1, 0, 1), (1, 0, 0), (1, 0, -1), (1, -1, 1),
                 (1, -1, 0), (1, -1, -1))


def m_matrix(channels, p: float, theta) -> dict:
    """M^s_{ms,ms'}(theta) in fm for channels [(s, J, ls, S)] at momentum p.

    ls lists the orbital momenta of the channel (one, or J-1 and J+1) and S
    is the matching on-shell S-matrix (1 x 1 or 2 x 2, S[l'_index, l_index]).
    """
    theta = np.asarray(theta, dtype=np.float64)
    out = {}
    for (s, ms, msp) in SPIN_ELEMENTS:
        acc = np.zeros(theta.shape, dtype=np.complex128)
        for (sc, J, ls, smat) in channels:
            if sc != s:
                continue
            smat = np.atleast_2d(np.asarray(smat))
            for ia, l in enumerate(ls):
                cin = clebsch_gordan(l, 0, s, ms, J, ms)
                if cin == 0.0:
                    continue
                for ib, lp in enumerate(ls):
                    cout = clebsch_gordan(lp, ms - msp, s, msp, J, ms)
                    if cout == 0.0:
                        continue
                    amp = smat[ib, ia] - (1.0 if ia == ib else 0.0)
                    acc = acc + math.sqrt((2 * l + 1) / (4 * math.pi)) * cin * cout * amp * \
                        sph_harm_theta(lp, ms - msp, theta)
        out[(s, ms, msp)] = 2.0 * math.pi / (1j * p) * acc
    return out


def saclay_amplitudes(M: dict, theta) -> dict:
    """a, b, c, d, e (fm) from the M-matrix elements (readings in the module docstring)."""
    theta = np.asarray(theta, dtype=np.float64)
    g = lambda s, i, j: M[(s, i, j)]
    a = 0.5 * (g(1, 1, 1) + g(1, 0, 0) - g(1, 1, -1))
    b = 0.5 * (g(1, 1, 1) + g(0, 0, 0) + g(1, 1, -1))
    c = 0.5 * (g(1, 1, 1) - g(0, 0, 0) + g(1, 1, -1))
    st, ct = np.sin(theta), np.cos(theta)
    use_sin = np.abs(st) >= np.abs(ct)
    with np.errstate(divide="ignore", invalid="ignore"):
        d_sin = -(g(1, 1, 0) + g(1, 0, 1)) / (math.sqrt(2.0) * st)
        d_cos = (g(1, 0, 0) - a) / ct
    d = np.where(use_sin, d_sin, d_cos)
    e = 1j * (g(1, 0, 1) - g(1, 1, 0)) / math.sqrt(2.0)
    return {"a": a, "b": b, "c": c, "d": d, "e": e}


def dsigma_domega(amps: dict) -> np.ndarray:
    """dsigma/dOmega in mb/sr."""
    return 10.0 * 0.5 * sum(np.abs(amps[k]) ** 2 for k in "abcde")


def sigma_tot_forward(amps: dict, p: float):
    """(2 pi/p) Im(a + b) in mb, with the amplitudes at theta = 0."""
    return 10.0 * 2.0 * math.pi / p * np.imag(amps["a"] + amps["b"])


def channel_s_at(delta_deg, eps_deg, kbar, k_max, p):
    """On-shell S of one channel at momentum p from its bin phase shifts.

    The phases are unwrapped and linearly interpolated in q between bin
    midpoints exactly as for the total cross section (Sec. 5.1.1; the mixing
    angle follows the parity of the shifts), and S is rebuilt from them in the
    Stapp form (App. A).
    """
    delta_deg = np.asarray(delta_deg, dtype=np.float64)
    K = delta_deg.shape[1]
    ds, sh = [], []
    for a in range(K):
        d, s = observables.unwrap_deg(delta_deg[:, a])
        ds.append(float(observables.interpolate(kbar, d, p, k_max)[0]))
        sh.append(s)
    if K == 1:
        return np.array([[np.exp(2j * np.radians(ds[0]))]])
    sign = np.where((sh[0] + sh[1]) % 2 == 0, 1.0, -1.0)
    e = float(observables.interpolate(kbar, sign * np.asarray(eps_deg), p, k_max)[0])
    return observables.stapp_s(ds[0], ds[1], e)
