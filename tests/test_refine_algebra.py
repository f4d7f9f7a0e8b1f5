"""Algebra behind the refinement's chain blocks, checked on the CPU in FP64.

The chain kernels form the Rayleigh-Ritz matrix P^T S P of a chain (columns
C, P = I_C + E_C) without the n x n x m product S P: with
T = S_C + Lam E_C / 2 and V = P^T T,

    P^T S P = V + V^T - T_C - T_C^T + S_CC + E_C^T (S - Lam) E_C,

and the last term is dropped.  These tests hold the identity exactly (to
rounding, for arbitrary S, E and Lam) and show that the dropped term is third
order: scaling both the off-diagonal part of S - Lam and E by t shrinks it by
t^3.  (Newton-type update after Ogita & Aishima; the closeness test bounds
|E| by 1/c off the close pairs.)
"""
import numpy as np
import pytest


def _setup(rng, n, cols, e_scale, o_scale):
    lam = np.sort(rng.uniform(-50.0, 700.0, n))
    o = rng.normal(0.0, o_scale, (n, n))
    s = np.diag(lam) + 0.5 * (o + o.T)  # S = Lam + a symmetric off-diagonal part
    e = rng.normal(0.0, e_scale, (n, len(cols)))
    return s, lam, e


def _fast(s, lam, e, cols):
    """V + V^T - T_C - T_C^T + S_CC, as the kernels form it."""
    n, m = e.shape
    p = e.copy()
    p[cols, np.arange(m)] += 1.0
    t = s[:, cols] + 0.5 * lam[:, None] * e
    v = p.T @ t
    tc = t[cols, :]
    return v + v.T - tc - tc.T + s[np.ix_(cols, cols)], p


@pytest.mark.parametrize("cols", [[3, 4], [10, 11, 12, 13, 14], list(range(40, 64))])
def test_chain_block_identity_is_exact_with_the_third_order_term(cols):
    rng = np.random.default_rng(7)
    n = 96
    s, lam, e = _setup(rng, n, cols, 1e-2, 1.0)
    fast, p = _fast(s, lam, e, cols)
    exact = p.T @ s @ p
    third = e.T @ (s - np.diag(lam)) @ e
    scale = np.abs(exact).max()
    assert np.abs(fast + third - exact).max() <= 1e-13 * scale
    # the formed block is symmetric, as the Jacobi on it assumes
    assert np.abs(fast - fast.T).max() <= 1e-13 * scale


def test_dropped_term_is_third_order():
    rng = np.random.default_rng(11)
    n, cols = 80, list(range(20, 30))
    errs = []
    for t in (1e-2, 1e-3, 1e-4):
        s, lam, e = _setup(rng, n, cols, t, t)
        fast, p = _fast(s, lam, e, cols)
        errs.append(np.abs(fast - p.T @ s @ p).max())
    # each factor 10 in t shrinks the dropped term by about 10^3
    assert 300.0 < errs[0] / errs[1] < 3000.0
    assert 300.0 < errs[1] / errs[2] < 3000.0


def test_diagonal_s_needs_no_correction():
    # with S = Lam (an exact eigenbasis) the formula is exact for any E
    rng = np.random.default_rng(3)
    n, cols = 50, [7, 8, 9]
    lam = np.sort(rng.uniform(0.0, 100.0, n))
    s = np.diag(lam)
    e = rng.normal(0.0, 0.3, (n, len(cols)))
    fast, p = _fast(s, lam, e, cols)
    assert np.abs(fast - p.T @ s @ p).max() <= 1e-12 * np.abs(lam).max()
