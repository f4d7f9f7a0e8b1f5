"""Pins of the oracle's method variants: energy wave packets, the midpoint
projection, interpolation points and the paper's Chebyshev mesh.

Each check compares the oracle with something it does not compute itself:
numerical quadrature, exact integrals, hand-evaluated closed forms, the Born
limit and the N_WP -> infinity convergence to the Yamaguchi closed form.
CPU only.
"""
import numpy as np
import pytest
from scipy import integrate

from oracle import observables, wpcd, yamaguchi
from synth import grids, potentials

BETA = 1.4
CUT = 4.0


def _yamaguchi(k, lam, packet, n_gauss=8):
    x, _ = wpcd.gauss_nodes(k, n_gauss)
    return wpcd.solve_channel(k, n_gauss, potentials.yamaguchi(x, x, lam, BETA), 1, packet)


def _max_err_vs_closed_form(k, r, lam):
    q = r["q"]
    ok = q <= observables.tlab_to_p(350.0)
    ex = yamaguchi.phase_shift_deg(q, lam, BETA, k[-1])
    d = ((r["delta"][:, 0] - ex + 90.0) % 180.0) - 90.0
    return np.abs(d[ok]).max()


# ------------------------------------------------------------ energy packets
def test_energy_packets_are_normalised_and_h0_is_their_energy_average():
    # <x_i|x_i> = (1/N_i) int f(k)^2 dk = 1 and <x_i|k^2|x_i> = (1/N_i) int k^2 f(k)^2 dk
    k = grids.tan2_bounded(9)
    norm = wpcd.packet_norm(k, "energy")
    e = wpcd.h0_diagonal(k, "energy")
    for i in range(9):
        f2 = lambda q: wpcd.packet_weight(q, "energy") ** 2
        one, _ = integrate.quad(f2, k[i], k[i + 1], epsabs=0, epsrel=1e-13)
        avg, _ = integrate.quad(lambda q: q * q * f2(q), k[i], k[i + 1], epsabs=0, epsrel=1e-13)
        assert abs(one / norm[i] - 1.0) < 1e-12
        assert abs(e[i] - avg / norm[i]) < 1e-12 * e[i]
    # the paper's eigenvalue of an energy packet is its energy midpoint
    assert np.allclose(wpcd.onshell_momenta(k, "energy") ** 2, 0.5 * (k[1:] ** 2 + k[:-1] ** 2), rtol=1e-15)


def test_energy_packet_projection_against_quadrature():
    # U(k',k) = k'^a k^b: V_ij = int_i k'^(a+1) f dk' int_j k^(b+1) f dk / sqrt(dE_i dE_j)
    k = grids.tan2_bounded(7)
    x, _ = wpcd.gauss_nodes(k, 16)
    dE = np.diff(k * k)
    for a, b in [(0, 0), (2, 1)]:
        v = wpcd.project(k, 16, np.outer(x ** a, x ** b), 1, "energy")
        ia = [integrate.quad(lambda q: q ** (a + 1) * np.sqrt(2 * q), k[i], k[i + 1], epsabs=0, epsrel=1e-13)[0]
              for i in range(7)]
        ib = [integrate.quad(lambda q: q ** (b + 1) * np.sqrt(2 * q), k[i], k[i + 1], epsabs=0, epsrel=1e-13)[0]
              for i in range(7)]
        exact = np.outer(ia, ib) / np.sqrt(np.outer(dE, dE))
        # Gauss-Legendre is not exact for the half-integer power; the first bin
        # (integrand ~ k^1.5 at 0) limits it
        assert np.allclose(v, exact, rtol=2e-6, atol=0)


def test_energy_packets_zero_potential_and_born_limit():
    k = grids.tan2_bounded(24)
    m = 24 * 8
    r = wpcd.solve_channel(k, 8, np.zeros((m, m)), 1, "energy")
    assert np.all(r["t"] == 0) and np.all(r["delta"] == 0)
    # first order in U: S = 1 - i pi q t with t = f(q)^2 V_kk/(N_k q^2) = 2 V_kk/(dE_k q),
    # so delta -> -pi V_kk/dE_k (rad)
    x, _ = wpcd.gauss_nodes(k, 8)
    shape = potentials.yamaguchi(x, x, 1.0, BETA)
    dE = np.diff(k * k)
    errs = []
    for eta in (1e-4, 5e-5):
        r = wpcd.solve_channel(k, 8, eta * shape, 1, "energy")
        born = -np.pi * np.diag(r["v"]) / dE
        errs.append(np.abs(np.radians(r["delta"][:, 0]) - born).max() / np.abs(born).max())
    assert errs[0] < 1e-3 and 1.6 < errs[0] / errs[1] < 2.4


def test_energy_packets_converge_to_yamaguchi_at_second_order():
    errs = [_max_err_vs_closed_form(k, _yamaguchi(k, 2.0, "energy"), 2.0)
            for k in (grids.tan2_bounded(n, CUT) for n in (32, 64, 128))]
    assert errs[0] < 0.3 and errs[2] < 0.02
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0


def test_energy_and_momentum_packets_agree_in_the_limit():
    k = grids.tan2_bounded(200, CUT)
    a = _yamaguchi(k, 1.2, "momentum")
    b = _yamaguchi(k, 1.2, "energy")
    # same bins, different on-shell points: compare both with the closed form
    assert _max_err_vs_closed_form(k, a, 1.2) < 0.01
    assert _max_err_vs_closed_form(k, b, 1.2) < 0.01


def test_energy_packets_reject_unknown_kind():
    with pytest.raises(wpcd.WPCDError):
        wpcd.h0_diagonal(grids.tan2_bounded(4), "position")


# ------------------------------------------------------- midpoint projection
def test_midpoint_projection_exact_for_constant_and_second_order_otherwise():
    # one Gauss node per bin is the midpoint rule: int_i k dk = dk_i kbar_i exactly,
    # so a constant U is projected exactly
    k = grids.tan2_bounded(11)
    dk, kbar, _ = wpcd.bins(k)
    x, w = wpcd.gauss_nodes(k, 1)
    assert np.allclose(x, kbar, rtol=1e-15) and np.allclose(w, dk, rtol=1e-15)
    v = wpcd.project(k, 1, np.full((11, 11), -0.7), 1)
    exact = -0.7 * np.outer(dk * kbar, dk * kbar) / np.sqrt(np.outer(dk, dk))
    assert np.allclose(v, exact, rtol=1e-14)
    # a smooth U: the error against the 8-point projection falls as dk^2
    errs = []
    for n in (20, 40, 80):
        kk = grids.tan2_bounded(n, CUT)
        x1, _ = wpcd.gauss_nodes(kk, 1)
        x8, _ = wpcd.gauss_nodes(kk, 8)
        v1 = wpcd.project(kk, 1, potentials.yamaguchi(x1, x1, 1.0, BETA), 1)
        v8 = wpcd.project(kk, 8, potentials.yamaguchi(x8, x8, 1.0, BETA), 1)
        errs.append(np.abs(v1 - v8).max() / np.abs(v8).max())
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0


@pytest.mark.parametrize("packet", ["momentum", "energy"])
def test_midpoint_projection_converges_to_yamaguchi(packet):
    errs = [_max_err_vs_closed_form(k, _yamaguchi(k, 2.0, packet, n_gauss=1), 2.0)
            for k in (grids.tan2_bounded(n, CUT) for n in (32, 64, 128))]
    assert errs[2] < 0.02
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0


# -------------------------------------------------------- interpolation points
def test_interpolation_points_and_linear_phases():
    k = grids.tan2_bounded(30)
    _, kbar, _ = wpcd.bins(k)
    assert np.allclose(observables.interpolation_points(k, 0.5), kbar, rtol=1e-15)
    assert np.array_equal(observables.interpolation_points(k, 0.0), k[:-1])
    with pytest.raises(ValueError):
        observables.interpolation_points(k, 1.5)
    # phases linear in q, given at the interpolation points of any frac, are
    # reproduced exactly: sigma = 10 pi/p^2 sin^2 delta(p) for one S-wave channel
    p = observables.tlab_to_p(np.array([2.0, 40.0, 150.0, 300.0]))
    for frac in (0.01, 0.3, 0.5, 0.99):
        x = observables.interpolation_points(k, frac)
        d = 5.0 + 20.0 * x
        sig = observables.sigma_tot([(0, d[:, None], None, x, k[-1])], None, [2.0, 40.0, 150.0, 300.0], None)
        expect = 10.0 * np.pi / p ** 2 * np.sin(np.radians(5.0 + 20.0 * p)) ** 2
        assert np.allclose(sig, expect, rtol=1e-12)


def test_sigma_band_brackets_midpoint_and_vanishes_for_constant_phases():
    k, r = grids.tan2_bounded(40, CUT), None
    r = _yamaguchi(k, 1.5, "momentum")
    tl = np.linspace(1.0, 300.0, 12)
    fr = [0.01, 0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9, 0.99]
    lo, hi = observables.sigma_band([(0, r["delta"], None, k)], tl, fr)
    mid = observables.sigma_tot([(0, r["delta"], None)], wpcd.bins(k)[1], tl, k[-1])
    assert np.all(lo <= mid + 1e-12) and np.all(mid <= hi + 1e-12) and np.all(hi > lo)
    const = np.full((40, 1), 12.5)
    lo, hi = observables.sigma_band([(0, const, None, k)], tl, fr)
    assert np.allclose(lo, hi, rtol=1e-14)


# ------------------------------------------------------------- Chebyshev mesh
def test_chebyshev_mesh_closed_form_values():
    # tan(pi/8) = sqrt2 - 1, tan(3 pi/8) = sqrt2 + 1, so with N = 2, t = 2:
    # y = alpha (3 -/+ 2 sqrt2)
    k = grids.chebyshev(2, 100.0, 2.0)
    hc = 197.327
    assert k[0] == 0.0
    assert abs(k[1] - 100.0 * (3 - 2 * np.sqrt(2)) / hc) < 1e-15
    assert abs(k[2] - 100.0 * (3 + 2 * np.sqrt(2)) / hc) < 1e-13
    # t = 1, N = 3: tan(pi/12) = 2 - sqrt3, tan(pi/4) = 1, tan(5 pi/12) = 2 + sqrt3
    k = grids.chebyshev(3, 50.0, 1.0)
    assert np.allclose(k, [0, 50 * (2 - np.sqrt(3)) / hc, 50 / hc, 50 * (2 + np.sqrt(3)) / hc], rtol=1e-14)


@pytest.mark.parametrize("packet", ["momentum", "energy"])
def test_wpcd_on_chebyshev_mesh_converges_to_yamaguchi(packet):
    errs = [_max_err_vs_closed_form(k, _yamaguchi(k, 2.0, packet), 2.0)
            for k in (grids.chebyshev(n) for n in (32, 64, 128))]
    assert errs[2] < 0.06
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0
