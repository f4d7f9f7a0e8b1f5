"""Pins of the oracle's spin-scattering matrix and Saclay amplitudes (CPU only).

Independent references: sympy's Clebsch-Gordan coefficients, scipy's
spherical harmonics, the optical theorem against the partial-wave total cross
section (observables.sigma_from_s), unitarity (the angle-integrated
dsigma/dOmega equals sigma_tot for a unitary S), the operator form of M
(Saclay decomposition) rebuilt from the amplitudes, and the pure 1S0 case.
"""
import math

import numpy as np
import pytest
from scipy.special import sph_harm_y
from sympy import S as Sy
from sympy.physics.quantum.cg import CG

from oracle import observables, saclay


def test_clebsch_gordan_matches_sympy():
    rng = np.random.default_rng(3)
    for _ in range(300):
        j1, j2 = int(rng.integers(0, 8)), int(rng.integers(0, 2))
        J = int(rng.integers(abs(j1 - j2), j1 + j2 + 1))
        m2 = int(rng.integers(-j2, j2 + 1))
        M = int(rng.integers(-J, J + 1))
        m1 = M - m2
        ref = float(CG(Sy(j1), Sy(m1), Sy(j2), Sy(m2), Sy(J), Sy(M)).doit()) if abs(m1) <= j1 else 0.0
        assert abs(saclay.clebsch_gordan(j1, m1, j2, m2, J, M) - ref) < 1e-13


def test_spherical_harmonics_match_scipy():
    th = np.linspace(0.0, np.pi, 37)
    for l in range(10):
        for m in range(-l, l + 1):
            ref = sph_harm_y(l, m, th, 0.0)
            assert np.abs(saclay.sph_harm_theta(l, m, th) - ref).max() < 1e-12


def _channels(seed, jmax=4):
    """Random unitary S for every (s, l, J) with J <= jmax (np-like set)."""
    rng = np.random.default_rng(seed)
    ch = []
    for J in range(jmax + 1):
        ch.append((0, J, [J], np.array([[np.exp(2j * np.radians(rng.uniform(-80, 80)))]])))
        if J == 0:
            ch.append((1, 0, [1], np.array([[np.exp(2j * np.radians(rng.uniform(-80, 80)))]])))
            continue
        ch.append((1, J, [J], np.array([[np.exp(2j * np.radians(rng.uniform(-80, 80)))]])))
        ch.append((1, J, [J - 1, J + 1], observables.stapp_s(rng.uniform(-70, 70), rng.uniform(-70, 70),
                                                              rng.uniform(-30, 30))))
    return ch


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_optical_theorem_and_unitarity(seed):
    ch = _channels(seed)
    p = 0.9
    amps0 = saclay.saclay_amplitudes(saclay.m_matrix(ch, p, np.array([0.0])), np.array([0.0]))
    want = observables.sigma_from_s([(J, s) for (_, J, _, s) in ch], p)
    assert abs(saclay.sigma_tot_forward(amps0, p)[0] - want) < 1e-10 * want
    # every amplitude is a polynomial in cos(theta) (times sin^m): Gauss-Legendre in cos is exact
    x, w = np.polynomial.legendre.leggauss(40)
    th = np.arccos(x)
    ds = saclay.dsigma_domega(saclay.saclay_amplitudes(saclay.m_matrix(ch, p, th), th))
    assert abs(2 * np.pi * np.sum(w * ds) - want) < 1e-10 * want


def test_saclay_operator_form_rebuilds_m():
    # M = (1/2)[(a+b) + (a-b)(s1.n)(s2.n) + (c+d)(s1.m)(s2.m) + (c-d)(s1.l)(s2.l) + e (s1+s2).n]
    # between |s ms> states (initial ms, final ms') must give back every M^s element
    ch = _channels(7)
    p = 0.6
    sx = np.array([[0, 1], [1, 0]])
    sy = np.array([[0, -1j], [1j, 0]])
    sz = np.array([[1, 0], [0, -1]])
    one, two = [np.kron(s, np.eye(2)) for s in (sx, sy, sz)], [np.kron(np.eye(2), s) for s in (sx, sy, sz)]
    up, dn = np.array([1.0, 0.0]), np.array([0.0, 1.0])
    st = {(1, 1): np.kron(up, up), (1, 0): (np.kron(up, dn) + np.kron(dn, up)) / math.sqrt(2),
          (1, -1): np.kron(dn, dn), (0, 0): (np.kron(up, dn) - np.kron(dn, up)) / math.sqrt(2)}
    for theta in (0.2, 0.8, math.pi / 2, 2.2, 3.0):
        t = np.array([theta])
        M = saclay.m_matrix(ch, p, t)
        am = {k: complex(v[0]) for k, v in saclay.saclay_amplitudes(M, t).items()}
        pv, pf = np.array([0, 0, 1.0]), np.array([math.sin(theta), 0, math.cos(theta)])
        l = (pv + pf) / np.linalg.norm(pv + pf)
        m = (pv - pf) / np.linalg.norm(pv - pf)
        n = np.cross(pv, pf) / np.linalg.norm(np.cross(pv, pf))
        d1 = lambda v: sum(v[i] * one[i] for i in range(3))
        d2 = lambda v: sum(v[i] * two[i] for i in range(3))
        op = 0.5 * ((am["a"] + am["b"]) * np.eye(4) + (am["a"] - am["b"]) * d1(n) @ d2(n)
                    + (am["c"] + am["d"]) * d1(m) @ d2(m) + (am["c"] - am["d"]) * d1(l) @ d2(l)
                    + am["e"] * (d1(n) + d2(n)))
        for (s, ms, msp) in saclay.SPIN_ELEMENTS:
            assert abs(st[(s, msp)].conj() @ op @ st[(s, ms)] - M[(s, ms, msp)][0]) < 1e-12 * max(
                1.0, abs(M[(s, ms, msp)][0]))
        # (1/4) Tr(M M^+) over the 4 spin states equals (1/2) sum |amplitude|^2
        tr = 0.25 * sum(abs(M[k][0]) ** 2 for k in saclay.SPIN_ELEMENTS)
        assert abs(tr - 0.5 * sum(abs(v) ** 2 for v in am.values())) < 1e-12 * tr


def test_pure_singlet_s_wave_is_isotropic():
    d = np.radians(50.0)
    p = 0.4
    th = np.linspace(0.1, 3.0, 9)
    am = saclay.saclay_amplitudes(saclay.m_matrix([(0, 0, [0], np.array([[np.exp(2j * d)]]))], p, th), th)
    # M^0_00 = exp(i d) sin d / p, b = -c = M/2, a = d = e = 0
    assert np.allclose(am["b"], np.exp(1j * d) * np.sin(d) / (2 * p)) and np.allclose(am["c"], -am["b"])
    assert np.abs(am["a"]).max() < 1e-15 and np.abs(am["d"]).max() < 1e-15 and np.abs(am["e"]).max() < 1e-15
    assert np.allclose(saclay.dsigma_domega(am), 10.0 * np.sin(d) ** 2 / (4 * p * p))


def test_channel_s_at_recovers_linear_stapp_parameters():
    kbar = np.linspace(0.05, 2.5, 40)
    dm, dp, ep = 120.0 * kbar - 20.0, -51.0 * kbar + 10.0, 12.0 * kbar - 10.0
    ph = observables.phase_shifts(observables.stapp_s(dm, dp, ep))
    for p in (0.3, 1.17, 2.3):
        s = saclay.channel_s_at(ph["delta"], ph["mix"], kbar, 4.0, p)
        want = observables.stapp_s(120.0 * p - 20.0, -51.0 * p + 10.0, 12.0 * p - 10.0)
        assert np.abs(s - want).max() < 1e-12
