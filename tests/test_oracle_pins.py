"""Pins of the FP64 oracle against results it does not compute itself.

Every check here compares the oracle with something independent: numerical
quadrature (scipy / mpmath), textbook closed forms, exact polynomial
integration, algebraic invariants, or the N_WP -> infinity limit of exactly
solvable problems.  CPU only.
"""
import numpy as np
import pytest
import mpmath
from scipy import integrate

from oracle import wpcd, mi, yamaguchi, observables
from synth import grids, potentials, configs

BETA = 1.4
CUT = 4.0


# ----------------------------------------------------------------- Yamaguchi
@pytest.mark.parametrize("p", [0.05, 0.5, 1.3, 2.5, 3.7])
def test_yamaguchi_j_integral_matches_pv_quadrature(p):
    # PV int_0^Lam q^2 g^2/(p^2-q^2) dq: write 1/(p^2-q^2) = -1/((q-p)(q+p)) and
    # let QUADPACK's Cauchy weight 1/(q - p) take the principal value.
    f = lambda q: -q * q / (q * q + BETA ** 2) ** 2 / (q + p)
    pv, _ = integrate.quad(f, 0.0, CUT, weight="cauchy", wvar=p, epsabs=1e-14, epsrel=1e-13)
    im = -np.pi * p / (p * p + BETA ** 2) ** 2 / 2.0
    j = yamaguchi.j_integral(p, BETA, CUT)
    assert abs(j.real - pv) < 1e-11
    assert abs(j.imag - im) < 1e-14


@pytest.mark.parametrize("lam", [0.5, 1.2, 2.0])
def test_yamaguchi_infinite_cutoff_effective_range_form(lam):
    # textbook: p cot(delta) = 2(b^2+p^2)^2/(pi lam) - (b^2-p^2)/(2b) for U = -lam g g
    p = np.array([0.01, 0.3, 1.0, 2.0, 3.0])
    d = np.radians(yamaguchi.phase_shift_deg(p, lam, BETA, None))
    expect = 2 * (BETA ** 2 + p ** 2) ** 2 / (np.pi * lam) - (BETA ** 2 - p ** 2) / (2 * BETA)
    assert np.allclose(p / np.tan(d), expect, rtol=1e-12)


@pytest.mark.parametrize("lam", [0.5, 2.0, 6.0])
def test_mi_reproduces_yamaguchi_closed_form(lam):
    for p in [0.02, 0.4, 1.1, 2.05, 3.5]:
        tc = yamaguchi.t_onshell(p, lam, BETA, CUT)
        tm = mi.solve(lambda r, c: potentials.yamaguchi(r, c, lam, BETA), p, 96, CUT, 1)[0, 0]
        assert abs(tm - tc) <= 1e-10 * abs(tc)


def _coupled_u(coeffs):
    def u(r, c):
        assert r is c
        return sum(ci * ti for ci, ti in zip(coeffs, configs.coupled_yukawa_terms(r)))
    return u


def test_mi_coupled_unitary_symmetric_and_k_route():
    u = _coupled_u(configs.yukawa_coefficients(0))
    for p in [0.1, 0.8, 2.0]:
        t = mi.solve(u, p, 96, CUT, 2)
        s = observables.s_from_t_continuum(t, p)
        assert np.abs(s @ s.conj().T - np.eye(2)).max() < 1e-10
        assert abs(s[0, 1] - s[1, 0]) < 1e-12
        kmat = mi.solve(u, p, 96, CUT, 2, kmatrix=True)
        assert np.abs(kmat.imag).max() == 0.0
        assert np.abs(mi.s_from_k(kmat.real, p) - s).max() < 1e-10
        t2 = mi.solve(u, p, 192, CUT, 2)
        assert np.abs(t2 - t).max() < 1e-7 * np.abs(t).max()


# ------------------------------------------------------------ bins / nodes / H0
def test_gauss_nodes_integrate_polynomials_exactly():
    k = grids.tan2_bounded(12)
    x, w = wpcd.gauss_nodes(k, 8)
    for deg in range(16):
        assert abs(np.sum(w * x ** deg) - k[-1] ** (deg + 1) / (deg + 1)) < 1e-13 * k[-1] ** (deg + 1)


def test_h0_is_bin_average_of_k2():
    k = grids.tan2_bounded(7)
    e = wpcd.h0_diagonal(k)
    for i in range(7):
        val, _ = integrate.quad(lambda q: q * q, k[i], k[i + 1], epsabs=0, epsrel=1e-13)
        assert abs(e[i] - val / (k[i + 1] - k[i])) < 1e-13 * max(e[i], 1e-300)


def test_projection_of_separable_polynomial_is_exact():
    # U(k',k) = k'^a k^b  =>  V_ij = int_i k'^(a+1) dk' int_j k^(b+1) dk / sqrt(dk_i dk_j)
    k = grids.tan2_bounded(9)
    x, _ = wpcd.gauss_nodes(k, 8)
    dk = np.diff(k)
    for a, b in [(0, 0), (2, 3), (5, 1)]:
        v = wpcd.project(k, 8, np.outer(x ** a, x ** b), 1)
        ia = (k[1:] ** (a + 2) - k[:-1] ** (a + 2)) / (a + 2)
        ib = (k[1:] ** (b + 2) - k[:-1] ** (b + 2)) / (b + 2)
        exact = np.outer(ia, ib) / np.sqrt(np.outer(dk, dk))
        assert np.allclose(v, exact, rtol=1e-12, atol=1e-300)


def test_projection_coupled_blocks_and_rank_one_yamaguchi():
    k = grids.tan2_bounded(10)
    x, _ = wpcd.gauss_nodes(k, 8)
    g = 1.0 / (x * x + BETA ** 2)
    u = -1.3 * np.outer(g, g)
    v = wpcd.project(k, 8, u, 1)
    s = np.linalg.svd(v, compute_uv=False)
    assert s[1] < 1e-14 * s[0]
    z = np.zeros_like(u)
    v2 = wpcd.project(k, 8, potentials.coupled_matrix(u, 0.5 * u, 2 * u), 2)
    assert np.allclose(v2[:10, :10], v) and np.allclose(v2[:10, 10:], 0.5 * v)
    assert np.allclose(v2[10:, :10], 0.5 * v.T) and np.allclose(v2[10:, 10:], 2 * v)
    assert np.all(wpcd.project(k, 8, potentials.coupled_matrix(z, z, z), 2) == 0)


# -------------------------------------------------------------- SWP boundaries
def test_swp_bins_hand_examples():
    lo, hi, bound = wpcd.swp_bins(np.array([-1.0, 1.0, 2.0, 4.0]), 1)
    assert list(bound) == [True, False, False, False]
    assert np.allclose(lo[1:], [0.0, 1.5, 3.0]) and np.allclose(hi[1:], [1.5, 3.0, 4.75])
    eps = np.array([-2.0, 0.5, 0.6, 1.0, 1.2, 2.0, 2.2])
    lo, hi, bound = wpcd.swp_bins(eps, 2)
    # family 1: 0.5, 1.0, 2.0 ; family 2: 0.6, 1.2, 2.2
    assert np.allclose(lo[[1, 3, 5]], [0, 0.75, 1.5]) and np.allclose(hi[[1, 3, 5]], [0.75, 1.5, 2.375])
    assert np.allclose(lo[[2, 4, 6]], [0, 0.9, 1.7]) and np.allclose(hi[[2, 4, 6]], [0.9, 1.7, 2.6])


def test_swp_bins_treat_states_above_the_continuum_as_discrete():
    lo, hi, disc = wpcd.swp_bins(np.array([-1.0, 1.0, 2.0, 4.0, 30.0]), 1, 16.0)
    assert list(disc) == [True, False, False, False, True]
    assert np.allclose(hi[1:4], [1.5, 3.0, 4.75]) and np.isnan(lo[4])


def test_swp_bins_rejects_degenerate_cases():
    with pytest.raises(wpcd.WPCDError):
        wpcd.swp_bins(np.array([-1.0, 0.0, 1.0, 2.0]), 1)
    with pytest.raises(wpcd.WPCDError):
        wpcd.swp_bins(np.array([-1.0, 3.0]), 1)
    with pytest.raises(wpcd.WPCDError):
        wpcd.swp_bins(np.array([0.5, 0.6, 1.0]), 2)


# ------------------------------------------------------------ averaged resolvent
def _gbar_numeric(a, b, c, d):
    """(1/((b-a)(d-c))) int_a^b dE PV int_c^d dE'/(E-E'), inner PV in closed form."""
    mpmath.mp.dps = 30
    inner = lambda e: mpmath.log(abs(e - c)) - mpmath.log(abs(e - d))
    pts = sorted({a, b} | {x for x in (c, d) if a < x < b})
    val = mpmath.quad(inner, pts)
    return float(val) / ((b - a) * (d - c))


@pytest.mark.parametrize("bins_", [
    ((10.0, 11.0), (0.0, 1.0)),      # far apart
    ((1.0, 2.0), (2.0, 3.5)),        # touching
    ((1.0, 2.0), (1.5, 2.5)),        # overlapping
    ((1.0, 2.0), (1.2, 1.7)),        # nested
    ((0.0, 1e-6), (0.0, 3e-6)),      # tiny low-energy bins, shared edge
    ((0.3, 0.31), (0.0, 0.02)),
])
def test_resolvent_real_part_matches_quadrature(bins_):
    (a, b), (c, d) = bins_
    k = np.array([0.0, np.sqrt(a), np.sqrt(b)]) if a > 0 else np.array([0.0, np.sqrt(b), np.sqrt(b) + 1.0])
    kb = k if a > 0 else k
    row = 1 if a > 0 else 0
    g = wpcd.resolvent_table(kb, np.array([0.5 * (c + d)]), np.array([c]), np.array([d]), np.array([False]))
    num = _gbar_numeric(a, b, c, d)
    assert abs(g[row, 0].real - num) <= 1e-10 * max(1.0, abs(num))
    ov = max(0.0, min(b, d) - max(a, c))
    assert abs(g[row, 0].imag + np.pi * ov / ((b - a) * (d - c))) <= 1e-12 * max(1.0, abs(g[row, 0].imag))


def test_resolvent_disjoint_bins_full_double_quadrature():
    # fully numerical double integral, no antiderivative at all
    val, _ = integrate.dblquad(lambda ep, e: 1.0 / (e - ep), 10.0, 11.0, 0.0, 1.0, epsabs=1e-13, epsrel=1e-12)
    assert abs(val - 0.1001673369) < 1e-9
    k = np.array([0.0, np.sqrt(10.0), np.sqrt(11.0)])
    g = wpcd.resolvent_table(k, np.array([0.5]), np.array([0.0]), np.array([1.0]), np.array([False]))
    assert abs(g[1, 0].real - val) < 1e-11 and g[1, 0].imag == 0.0


def test_resolvent_far_bin_limit_and_bound_state_average():
    k = np.array([0.0, 10.0, 10.001])
    g = wpcd.resolvent_table(k, np.array([0.2]), np.array([0.1]), np.array([0.3]), np.array([False]))
    ebar = 0.5 * (k[1] ** 2 + k[2] ** 2)
    assert abs(g[1, 0].real * (ebar - 0.2) - 1.0) < 1e-6
    gb = wpcd.resolvent_table(k, np.array([-2.0]), np.array([np.nan]), np.array([np.nan]), np.array([True]))
    val, _ = integrate.quad(lambda e: 1.0 / (e + 2.0), k[1] ** 2, k[2] ** 2, epsabs=0, epsrel=1e-13)
    assert abs(gb[1, 0].real - val / (k[2] ** 2 - k[1] ** 2)) < 1e-12 and gb[1, 0].imag == 0


# --------------------------------------------------------------- whole channel
def _yamaguchi_channel(n_wp, lam):
    k = grids.tan2_bounded(n_wp, CUT)
    x, _ = wpcd.gauss_nodes(k, 8)
    return k, wpcd.solve_channel(k, 8, potentials.yamaguchi(x, x, lam, BETA), 1)


def test_zero_potential_gives_zero_t_and_phase():
    k = grids.tan2_bounded(20)
    m = 20 * 8
    r = wpcd.solve_channel(k, 8, np.zeros((m, m)), 1)
    assert np.all(r["t"] == 0) and np.all(r["delta"] == 0)
    r2 = wpcd.solve_channel(k, 8, np.zeros((2 * m, 2 * m)), 2)
    assert np.all(r2["t"] == 0) and np.all(r2["delta"] == 0) and np.all(r2["mix"] == 0)


def test_vc_identity_holds_for_exact_eigenpairs():
    k, r = _yamaguchi_channel(40, 1.7)
    e = wpcd.h0_diagonal(k)
    vc = r["v"] @ r["evecs"]
    ident = r["evecs"] * (r["evals"][None, :] - e[:, None])
    assert np.abs(vc - ident).max() <= 1e-12 * np.abs(r["v"]).max()


def test_born_limit():
    k = grids.tan2_bounded(30)
    x, _ = wpcd.gauss_nodes(k, 8)
    dk, kbar, _ = wpcd.bins(k)
    shape = potentials.yamaguchi(x, x, 1.0, BETA)
    errs = []
    for eta in (1e-4, 5e-5):
        r = wpcd.solve_channel(k, 8, eta * shape, 1)
        born = -0.5 * np.pi * np.diag(r["v"]) / (dk * kbar)
        errs.append(np.abs(np.radians(r["delta"][:, 0]) - born).max() / np.abs(born).max())
    assert errs[0] < 1e-3 and 1.6 < errs[0] / errs[1] < 2.4   # O(eta) error


def test_wpcd_converges_to_yamaguchi_at_second_order():
    errs = []
    for n in (32, 64, 128):
        k, r = _yamaguchi_channel(n, 2.0)
        _, kbar, _ = wpcd.bins(k)
        ok = kbar <= observables.tlab_to_p(350.0)
        ex = yamaguchi.phase_shift_deg(kbar, 2.0, BETA, CUT)
        d = ((r["delta"][:, 0] - ex + 90.0) % 180.0) - 90.0
        errs.append(np.abs(d[ok]).max())
    assert errs[0] < 0.2 and errs[2] < 0.015
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0


def test_wpcd_bound_state_channel_converges():
    errs = []
    for n in (50, 100):
        k, r = _yamaguchi_channel(n, 6.0)
        assert (r["evals"] < 0).sum() == 1
        _, kbar, _ = wpcd.bins(k)
        ok = kbar <= observables.tlab_to_p(350.0)
        ex = yamaguchi.phase_shift_deg(kbar, 6.0, BETA, CUT)
        d = ((r["delta"][:, 0] - ex + 90.0) % 180.0) - 90.0
        errs.append(np.abs(d[ok]).max())
    assert errs[1] < 0.06 and errs[1] < errs[0] / 3.0


def test_coupled_wpcd_converges_to_mi():
    coeffs = configs.yukawa_coefficients(0)
    u_mi = _coupled_u(coeffs)
    worst = []
    for n in (50, 100, 200):
        k = grids.tan2_bounded(n, CUT)
        x, _ = wpcd.gauss_nodes(k, 8)
        u = sum(c * t for c, t in zip(coeffs, configs.coupled_yukawa_terms(x)))
        r = wpcd.solve_channel(k, 8, u, 2)
        _, kbar, _ = wpcd.bins(k)
        assert np.allclose(r["s"][:, 0, 1], r["s"][:, 1, 0], rtol=1e-9, atol=1e-13)
        sel = np.flatnonzero((kbar > 0.2) & (kbar < 1.6))[:: max(1, n // 25)]
        e = 0.0
        for i in sel:
            ph = observables.phase_shifts(observables.s_from_t_continuum(mi.solve(u_mi, kbar[i], 96, CUT, 2), kbar[i]))
            dd = ((r["delta"][i] - ph["delta"] + 90.0) % 180.0) - 90.0
            e = max(e, np.abs(dd).max(), abs(r["mix"][i] - ph["mix"]))
        worst.append(e)
    # second order in 1/N_WP: each doubling cuts the error about four-fold
    assert 3.0 < worst[0] / worst[1] < 5.0 and 3.0 < worst[1] / worst[2] < 5.0 and worst[2] < 0.02


# ------------------------------------------------------------ observables
def test_stapp_round_trip():
    rng = np.random.default_rng(5)
    dm, dp = rng.uniform(-89, 89, 50), rng.uniform(-89, 89, 50)
    ep = rng.uniform(-44, 44, 50)
    s = observables.stapp_s(dm, dp, ep)
    assert np.abs(np.einsum("nij,nkj->nik", s, s.conj()) - np.eye(2)).max() < 1e-14
    ph = observables.phase_shifts(s)
    assert np.allclose(ph["delta"][:, 0], dm, atol=1e-10) and np.allclose(ph["delta"][:, 1], dp, atol=1e-10)
    assert np.allclose(ph["mix"], ep, atol=1e-10)


def test_sigma_single_channel_textbook_and_coupled_reduction():
    kbar = np.linspace(0.05, 3.0, 40)
    slope = 37.0
    delta = (slope * kbar)[:, None]               # linear in q, crosses +-90 several times
    wrapped = ((delta + 90.0) % 180.0) - 90.0
    tl = np.array([1.0, 25.0, 150.0, 349.0])
    p = observables.tlab_to_p(tl)
    sig = observables.sigma_tot([(0, wrapped, None)], kbar, tl, 4.0)
    assert np.allclose(sig, 10.0 * np.pi / p ** 2 * np.sin(np.radians(slope * p)) ** 2, rtol=1e-12)
    # coupled, eps = 0: two uncoupled waves with the same J weight
    d2 = np.concatenate([wrapped, -0.5 * wrapped], axis=1)
    sig2 = observables.sigma_tot([(1, d2, np.zeros(40))], kbar, tl, 4.0)
    ref = 3 * (observables.sigma_tot([(0, wrapped, None)], kbar, tl, 4.0)
               + observables.sigma_tot([(0, -0.5 * wrapped, None)], kbar, tl, 4.0))
    assert np.allclose(sig2, ref, rtol=1e-12)


def test_sigma_coupled_mixing_branch_against_closed_form():
    # A coupled channel whose Stapp parameters are linear in q, so mid-point
    # interpolation is exact: delta_-(q), delta_+(q) cross +-90 degrees at
    # different momenta (each wrapped phase picks up its own 180-degree
    # jumps) and eps(q) != 0 moves through both signs.  S is built from the
    # parameters at the bin midpoints (App. A, Stapp form), the principal
    # values are re-extracted from it, and sigma_tot must equal the partial-
    # wave optical theorem evaluated directly from the unwrapped parameters:
    #   sigma(p) = 10 pi/(2 p^2) (2J+1) (2 - cos 2eps (cos 2d_- + cos 2d_+)).
    # A wrong sign rule for eps under odd shift parity, cos(eps) for cos(2 eps)
    # or a dropped mixing factor all move this by far more than 1e-9.
    kbar = np.linspace(0.04, 2.9, 55)
    dm_true = 120.0 * kbar - 20.0           # crosses +90 and +270 degrees
    dp_true = -51.0 * kbar + 10.0           # crosses -90 degrees
    ep_true = 24.0 * kbar - 30.0            # mixing angle from -29 to +40 degrees
    s = observables.stapp_s(dm_true, dp_true, ep_true)
    ph = observables.phase_shifts(s)
    wrapped_m, wrapped_p = ph["delta"][:, 0], ph["delta"][:, 1]
    # the extraction really wraps: some bins differ from the truth by 180 deg,
    # with odd total shift parity somewhere (so the extracted eps flips sign)
    km = np.round((dm_true - wrapped_m) / 180.0)
    kp = np.round((dp_true - wrapped_p) / 180.0)
    assert np.abs(km).max() >= 1 and np.abs(kp).max() >= 1
    odd = ((km + kp) % 2) != 0
    assert odd.any() and (~odd).any()
    assert np.allclose(ph["mix"][odd], -ep_true[odd], atol=1e-9)
    assert np.allclose(ph["mix"][~odd], ep_true[~odd], atol=1e-9)
    J = 3
    p = np.linspace(kbar[0] * 1.01, kbar[-1] * 0.999, 400)
    tl = 2.0 * (observables.HBARC_MEV_FM * p) ** 2 / observables.M_N_MEV
    got = observables.sigma_tot([(J, np.stack([wrapped_m, wrapped_p], axis=1), ph["mix"])], kbar, tl, 4.0)
    slope = lambda y: np.interp(p, kbar, y)        # exact for data linear in q
    e2, m2, p2 = (2.0 * np.radians(slope(y)) for y in (ep_true, dm_true, dp_true))
    want = 10.0 * np.pi / (2.0 * p * p) * (2 * J + 1) * (2.0 - np.cos(e2) * (np.cos(m2) + np.cos(p2)))
    assert np.abs(got - want).max() <= 1e-9 * np.abs(want).max()
    # the intervals whose end bins have opposite shift parity are where the
    # sign rule matters; the check above covers p in such intervals
    i = np.clip(np.searchsorted(kbar, p, side="right"), 1, kbar.size - 1)
    assert (odd[i] != odd[i - 1]).any()


def test_sigma_from_s_textbook_forms():
    # single wave: S = exp(2 i d) -> (pi/p^2)(2J+1) sin^2 d / 2 ... per partial wave
    # (np-like weights): 10 pi/(2 p^2) (2J+1) (1 - cos 2d) = 10 pi/p^2 (2J+1) sin^2 d
    p, d = 0.7, np.radians(37.0)
    assert abs(observables.sigma_from_s([(2, np.exp(2j * d))], p) - 10 * np.pi / p ** 2 * 5 * np.sin(d) ** 2) < 1e-12
    # coupled Stapp S: (2J+1)(2 - cos 2e (cos 2d- + cos 2d+))
    s = observables.stapp_s(20.0, -35.0, 7.0)
    want = 10 * np.pi / (2 * p * p) * 3 * (2 - np.cos(np.radians(14)) * (np.cos(np.radians(40)) + np.cos(np.radians(-70))))
    assert abs(observables.sigma_from_s([(1, s)], p) - want) < 1e-12


def test_tlab_kinematics():
    # E_cm = T_lab/2 = (hbar c p)^2/m_N for equal masses
    p = observables.tlab_to_p([1.0, 40.0, 350.0])
    assert np.allclose((197.327 * p) ** 2 / 938.918, [0.5, 20.0, 175.0], rtol=1e-14)
    assert np.allclose(p, [0.109803, 0.694452, 2.054217], atol=1e-6)


# ------------------------------------------------------------ synthetic inputs
def test_legendre_q_matches_mpmath():
    mpmath.mp.dps = 30
    for z in [1.0153, 1.3, 4.0, 1e3, 1e8]:
        q = potentials.legendre_q(7, np.array([z - 1.0]))
        for l in range(8):
            ref = float(mpmath.legenq(l, 0, mpmath.mpf(z), type=3).real)
            assert abs(q[l][0] - ref) <= 1e-12 * abs(ref)


def test_tensor_block_matches_direct_radial_integral():
    mpmath.mp.dps = 20
    mu, J = 0.7, 1
    for pp, p in [(0.3, 1.1), (2.5, 0.8), (3.9, 3.7)]:
        f = lambda r: r * r * mpmath.sqrt(mpmath.pi / (2 * pp * r)) * mpmath.besselj(J - 0.5, pp * r) \
            * potentials.RED_PER_MEV * mpmath.exp(-mu * r) * (1 + 3 / (mu * r) + 3 / (mu * r) ** 2) / r \
            * mpmath.sqrt(mpmath.pi / (2 * p * r)) * mpmath.besselj(J + 1.5, p * r)
        ref = float(mpmath.quad(f, mpmath.linspace(0, 60, 121))) * (2 / np.pi) * 6 * np.sqrt(2.0) / 3
        got = potentials.tensor_block(J, np.array([pp]), np.array([p]), 1.0, mu)[0, 0]
        assert abs(got - ref) <= 1e-9 * abs(ref)


def test_legendre_q_array_matches_mpmath_across_depth_groups():
    # > 65536 points so several depth groups (sorted by decay rate) are formed
    mpmath.mp.dps = 30
    rng = np.random.default_rng(5)
    zm1 = np.concatenate([10.0 ** rng.uniform(-3, 5, 70000), [0.0153, 1e-3]])
    q = potentials.legendre_q(7, zm1.reshape(2, -1))
    for j in rng.integers(0, zm1.size, 25).tolist() + [zm1.size - 1, zm1.size - 2]:
        z = 1 + mpmath.mpf(zm1[j])
        for l in (0, 3, 7):
            ref = float(mpmath.legenq(l, 0, z, type=3).real)
            assert abs(q[l].ravel()[j] - ref) <= 1e-12 * abs(ref)


def test_sweep_channel_set_and_sigma_with_per_channel_bins():
    from synth import sweep
    names = [c[0] for c in sweep.CHANNELS]
    assert len(names) == 20 and len(set(names)) == 20
    slj = set()
    for _, n_ch, J, S, l in sweep.CHANNELS:
        assert 0 <= J <= 6
        ls = (l,) if n_ch == 1 else (l, l + 2)
        if n_ch == 2:
            assert S == 1 and l == J - 1
        for ll in ls:
            assert abs(ll - J) <= S and (S, ll, J) not in slj
            slj.add((S, ll, J))
    assert len(slj) == 26            # 7 singlet + 7 triplet uncoupled + 6 x 2 coupled
    # per-channel bins: identical to the shared-bin form when the bins agree
    kbar = np.linspace(0.05, 3.0, 40)
    d = (20.0 * kbar)[:, None]
    tl = np.array([1.0, 100.0, 300.0])
    a = observables.sigma_tot([(0, d, None), (2, d, None)], kbar, tl, 4.0)
    b = observables.sigma_tot([(0, d, None, kbar, 4.0), (2, d, None, kbar, 4.0)], None, tl, None)
    assert np.array_equal(a, b)
