"""The batched matrix-inversion (K-matrix) solver on the GPU against the oracle.

The same discretised LS equation (Gauss-Legendre nodes on [0, L] with the
on-shell point appended, principal-value subtraction, K-matrix route) is
solved by the library (one FP64 LU per item and energy) and by the oracle's
matrix-inversion solver (its own nodes, LAPACK gesv).  Yamaguchi items are
also checked against the closed-form T-matrix at the same cut-off.  Bars: the
K-matrix to 1e-9 of its scale, phase shifts and mixing angles within 1e-6 deg
(both sides solve the same FP64 system), the closed form within 1e-8 deg,
cross sections within 1e-6 mb of the oracle's S matrices.
"""
import numpy as np
import pytest
import torch

import paper_2106_00454_amd as wp
from oracle import mi as omi
from oracle import observables as oo
from oracle import yamaguchi
from synth import configs, potentials

pytestmark = pytest.mark.gpu

CUT = 4.0
TLAB = np.linspace(1.0, 330.0, 24)


def _pack(solver, mats):
    u = np.zeros(solver.layout["u_elems"])
    for off, m in zip(solver.u_off, mats):
        u[off:off + m.size] = m.ravel()
    return torch.tensor(u, dtype=torch.float64, device="cuda")


def _run(solver, mats):
    u = _pack(solver, mats)
    bufs = solver.alloc()
    solver.solve(u, bufs)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in bufs.items()}


def test_mi_yamaguchi_matches_closed_form_and_oracle():
    ctx = wp.Context(0)
    lams = (0.6, 1.4, 2.0, 6.0)            # 6.0: a bound state
    nq = 96
    s = wp.MiSolver(ctx, [(1, 0, i) for i in range(len(lams))], nq, CUT, TLAB)
    pts = s.points
    mats = [potentials.yamaguchi(pts, pts, lam, 1.4) for lam in lams]
    h = _run(s, mats)
    assert (h["status"] == 0).all()
    p = oo.tlab_to_p(TLAB)
    assert np.allclose(pts[nq:], p, rtol=1e-15)
    for i, lam in enumerate(lams):
        d = h["delta"][s.delta_off[i]:s.delta_off[i] + TLAB.size]
        km = h["kmat"][s.k_off[i]:s.k_off[i] + TLAB.size]
        exact = yamaguchi.phase_shift_deg(p, lam, 1.4, CUT)
        de = np.abs(((d - exact + 90.0) % 180.0) - 90.0).max()
        ko = np.array([omi.solve(lambda r, c: potentials.yamaguchi(r, c, lam, 1.4), pe, nq, CUT, 1, kmatrix=True)[0, 0]
                       for pe in p])
        dk = np.abs(km - ko.real).max() / np.abs(ko).max()
        sig_o = np.array([oo.sigma_from_s([(0, omi.s_from_k(np.array([[k]]), pe))], pe) for k, pe in zip(ko.real, p)])
        ds = np.abs(h["sigma"].reshape(len(lams), -1)[i] - sig_o).max()
        print(f"MI Yamaguchi lam={lam}: delta vs closed form {de:.2e} deg, K vs oracle {dk:.2e}, "
              f"sigma vs oracle {ds:.2e} mb", flush=True)
        assert de <= 1e-8 and dk <= 1e-9 and ds <= 1e-6


def test_mi_coupled_yukawa_matches_oracle():
    ctx = wp.Context(0)
    nq = 48
    ns = 3
    items = [(2, 1, 0), (1, 0, 0), (2, 1, 1), (2, 1, 2)]     # sample 0 holds a coupled and an uncoupled item
    s = wp.MiSolver(ctx, items, nq, CUT, TLAB)
    pts = s.points
    coeffs = [configs.yukawa_coefficients(k) for k in range(ns)]
    u_cpl = lambda c, r: sum(ci * t for ci, t in zip(c, configs.coupled_yukawa_terms(r)))
    u_unc = lambda r, cc: sum(C * potentials.yukawa_central(0, r, cc, 1.0, mu)
                              for C, mu in zip((-10.0, -420.0, 1500.0), configs.YUKAWA_MU))
    mats = [u_cpl(coeffs[0], pts), u_unc(pts, pts), u_cpl(coeffs[1], pts), u_cpl(coeffs[2], pts)]
    h = _run(s, mats)
    assert (h["status"] == 0).all()
    p = oo.tlab_to_p(TLAB)
    per_sample = {}
    for i, (K, J, sid) in enumerate(items):
        if K == 2:
            c = coeffs[[0, None, 1, 2][i]]
            fn = lambda r, cc, c=c: u_cpl(c, r)
        else:
            fn = u_unc
        kmat = h["kmat"][s.k_off[i]:s.k_off[i] + TLAB.size * K * K].reshape(-1, K, K)
        dl = h["delta"][s.delta_off[i]:s.delta_off[i] + TLAB.size * K].reshape(-1, K)
        mx = h["mix"][s.mix_off[i]:s.mix_off[i] + TLAB.size]
        worst = [0.0, 0.0, 0.0]
        for e, pe in enumerate(p):
            ko = omi.solve(fn, pe, nq, CUT, K, kmatrix=True).real
            so = omi.s_from_k(ko, pe)
            ph = oo.phase_shifts(so)
            worst[0] = max(worst[0], np.abs(kmat[e] - ko).max() / np.abs(ko).max())
            worst[1] = max(worst[1], np.abs(((dl[e] - ph["delta"] + 90.0) % 180.0) - 90.0).max())
            if K == 2:
                worst[2] = max(worst[2], abs(mx[e] - ph["mix"]))
            per_sample.setdefault(sid, {}).setdefault(e, []).append((J, so))
        print(f"MI item {i} (n_ch={K}): K rel {worst[0]:.2e}, delta {worst[1]:.2e} deg, mix {worst[2]:.2e} deg",
              flush=True)
        assert worst[0] <= 1e-9 and worst[1] <= 1e-6 and worst[2] <= 1e-6
    sig = h["sigma"].reshape(-1, TLAB.size)
    for sid, byE in per_sample.items():
        want = np.array([oo.sigma_from_s(byE[e], p[e]) for e in range(TLAB.size)])
        ds = np.abs(sig[sid] - want).max()
        print(f"MI sample {sid}: sigma vs oracle {ds:.2e} mb", flush=True)
        assert ds <= 1e-6


def test_mi_argument_errors():
    ctx = wp.Context(0)
    with pytest.raises(wp.WPCDError) as e:
        wp.MiSolver(ctx, [(2, 1, 0)], 80, CUT, TLAB)             # coupled system too large for the LDS
    assert e.value.code == wp.WPCD_ERR_UNSUPPORTED
    with pytest.raises(wp.WPCDError) as e:
        wp.MiSolver(ctx, [(1, 0, 0)], 16, 1.0, TLAB)             # p beyond the cut-off
    assert e.value.code == wp.WPCD_ERR_INVALID
