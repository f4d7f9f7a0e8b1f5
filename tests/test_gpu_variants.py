"""Method variants on the GPU against the FP64 oracle (Sec. 3.1, 3.2, 5.1.1).

* energy wave packets (f(k) = sqrt(k/mu), N_i = dE_i; H0 diagonal and
  on-shell momentum at the energy midpoint): Yamaguchi N_WP = 50 and coupled
  Yukawa N_WP = 100 items, both arithmetic modes;
* the midpoint projection (one node per bin: the bin midpoint with weight
  dk_i), momentum and energy packets;
* the paper-literal Chebyshev mesh (y_j = alpha tan^2((2j-1) pi/(4N)),
  alpha = 100 MeV, unbounded: k_N is about 1000 fm^-1 at N_WP = 32), both
  modes;
* interpolation-point bands of sigma_tot (wpcd_sigma_band) against the
  oracle's band over the same fractions.

Bars: phase shifts and mixing angles within 0.01 deg and sigma within
0.01 mb of the oracle, as for the default path; eigenpairs by residual and
orthogonality against the H the GPU diagonalised.
"""
import numpy as np
import pytest
import torch

import paper_2106_00454_amd as wp
from oracle import observables as oo
from oracle import wpcd as ow
from synth import configs, grids, potentials
from synth import device as sdev
from tests.gpu_util import DELTA_TOL, SIGMA_TOL, TLAB, dmod180, item_view

pytestmark = pytest.mark.gpu

PACKETS = {wp.PACKET_MOMENTUM: "momentum", wp.PACKET_ENERGY: "energy"}


def _run(ctx, k, n_gauss, packet, K, us, mode, tlab):
    """Items on one grid (one sample each); us: host U at the grid's nodes."""
    g = ctx.grid(k, n_gauss, packet)
    J = 1 if K == 2 else 0
    b = ctx.batch([(g, K, J, s) for s in range(len(us))])
    u = sdev.pack_host_matrices(b.layout["u_elems"], b.u_off, [f(g.nodes) for f in us], torch.float64)
    bufs = b.alloc()
    tl = torch.tensor(tlab, dtype=torch.float64, device="cuda")
    sig = torch.full((b.layout["n_samples"] * len(tlab),), np.nan, dtype=torch.float64, device="cuda")
    b.run(u, bufs, mode, tl, sig)
    torch.cuda.synchronize()
    host = {kk: v.cpu().numpy() for kk, v in bufs.items()}
    host["sigma"] = sig.cpu().numpy().reshape(b.layout["n_samples"], len(tlab))
    return b, host, bufs


def _check(tag, b, host, k, n_gauss, packet, K, us, mode, tlab):
    x, _ = ow.gauss_nodes(k, n_gauss)
    name = PACKETS[packet]
    for i, f in enumerate(us):
        ref = ow.solve_channel(k, n_gauss, f(x), K, name)
        it = item_view(b, host, i)
        n = it["v"].shape[0]
        h = it["v"] + np.diag(np.tile(ow.h0_diagonal(k, name), K))
        hmax = np.abs(h).max()
        resid = np.abs(h @ it["evecs"] - it["evecs"] * it["evals"][None, :]).max()
        orth = np.abs(it["evecs"].T @ it["evecs"] - np.eye(n)).max()
        dd = dmod180(it["delta"], ref["delta"]).max()
        dm = np.abs(it["mix"] - ref["mix"]).max() if K == 2 else 0.0
        J = 1 if K == 2 else 0
        sref = oo.sigma_tot([(J, ref["delta"], ref["mix"], ref["q"], k[-1])], None, tlab, None)
        ds = np.abs(host["sigma"][i] - sref).max()
        msg = (f"{tag} item {i}: ddelta={dd:.3e} dmix={dm:.3e} dsigma={ds:.3e} resid={resid:.3e} "
               f"orth={orth:.3e} sweeps={it['eig_status']}")
        print(msg, flush=True)
        assert it["eig_status"] > 0 and it["t_status"] == 0, msg
        assert dd <= DELTA_TOL and dm <= DELTA_TOL and ds <= SIGMA_TOL, msg
        assert resid <= 1e-9 * hmax, msg
        assert orth <= (3e-9 if mode == wp.MIXED else 1e-13), msg


def _yamaguchi_items(n):
    return [lambda x, lam=configs.yamaguchi_lambda(s): potentials.yamaguchi(x, x, lam, configs.YAMAGUCHI_BETA)
            for s in range(n)]


def _coupled_items(n):
    return [lambda x, c=configs.yukawa_coefficients(s): sum(ci * t for ci, t in zip(c, configs.coupled_yukawa_terms(x)))
            for s in range(n)]


@pytest.mark.timeout(300)
@pytest.mark.parametrize("mode", [wp.MIXED, wp.F64])
def test_energy_packets_match_oracle(mode):
    ctx = wp.Context(0)
    for K, k, us in ((1, configs.grid("yamaguchi_s"), _yamaguchi_items(6)),
                     (2, configs.grid("coupled_yukawa"), _coupled_items(3))):
        b, host, _ = _run(ctx, k, 8, wp.PACKET_ENERGY, K, us, mode, TLAB)
        _check(f"energy packets K={K} mode={mode}", b, host, k, 8, wp.PACKET_ENERGY, K, us, mode, TLAB)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("packet", [wp.PACKET_MOMENTUM, wp.PACKET_ENERGY])
def test_midpoint_projection_matches_oracle(packet):
    ctx = wp.Context(0)
    for K, k, us in ((1, configs.grid("yamaguchi_s"), _yamaguchi_items(6)),
                     (2, configs.grid("coupled_yukawa"), _coupled_items(3))):
        g = ctx.grid(k, 1, packet)
        dk, kbar, _ = ow.bins(k)
        assert np.allclose(g.nodes, kbar, rtol=1e-15) and np.allclose(g.weights, dk, rtol=1e-15)
        for mode in (wp.MIXED, wp.F64):
            b, host, _ = _run(ctx, k, 1, packet, K, us, mode, TLAB)
            _check(f"midpoint {PACKETS[packet]} K={K} mode={mode}", b, host, k, 1, packet, K, us, mode, TLAB)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("mode", [wp.MIXED, wp.F64])
def test_chebyshev_mesh_matches_oracle(mode):
    ctx = wp.Context(0)
    k = grids.chebyshev(32)
    # T_lab up to 350 MeV lies far inside this mesh (p <= 2.06 fm^-1)
    b, host, _ = _run(ctx, k, 8, wp.PACKET_MOMENTUM, 1, _yamaguchi_items(4), mode, TLAB)
    _check(f"chebyshev N=32 mode={mode}", b, host, k, 8, wp.PACKET_MOMENTUM, 1, _yamaguchi_items(4), mode, TLAB)


@pytest.mark.timeout(300)
def test_sigma_band_matches_oracle_band():
    ctx = wp.Context(0)
    fr = np.array([0.01, 0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9, 0.99])
    tl = np.linspace(1.0, 300.0, 40)
    # two samples: a Yamaguchi S-wave and a coupled channel
    gy = ctx.grid(configs.grid("yamaguchi_s"), 8)
    gc = ctx.grid(configs.grid("coupled_yukawa"), 8)
    lam = configs.yamaguchi_lambda(3)
    c = configs.yukawa_coefficients(3)
    fy = lambda x: potentials.yamaguchi(x, x, lam, configs.YAMAGUCHI_BETA)
    fc = lambda x: sum(ci * t for ci, t in zip(c, configs.coupled_yukawa_terms(x)))
    b = ctx.batch([(gy, 1, 0, 0), (gc, 2, 1, 1), (gy, 1, 0, 1)])
    u = sdev.pack_host_matrices(b.layout["u_elems"], b.u_off, [fy(gy.nodes), fc(gc.nodes), fy(gy.nodes)],
                                torch.float64)
    bufs = b.alloc()
    b.run(u, bufs, wp.MIXED)
    t_tl = torch.tensor(tl, dtype=torch.float64, device="cuda")
    t_fr = torch.tensor(fr, dtype=torch.float64, device="cuda")
    lo = torch.full((2 * tl.size,), np.nan, dtype=torch.float64, device="cuda")
    hi = torch.full((2 * tl.size,), np.nan, dtype=torch.float64, device="cuda")
    b.sigma_band(bufs["delta"], bufs["mix"], t_tl, t_fr, lo, hi)
    torch.cuda.synchronize()
    lo, hi = lo.cpu().numpy().reshape(2, -1), hi.cpu().numpy().reshape(2, -1)
    assert np.all(lo <= hi)
    ky, kc = configs.grid("yamaguchi_s"), configs.grid("coupled_yukawa")
    # the whole path against the oracle's band from its own phases
    xy, _ = ow.gauss_nodes(ky, 8)
    xc, _ = ow.gauss_nodes(kc, 8)
    ry, rc = ow.solve_channel(ky, 8, fy(xy), 1), ow.solve_channel(kc, 8, fc(xc), 2)
    och = [[(0, ry["delta"], None, ky)], [(1, rc["delta"], rc["mix"], kc), (0, ry["delta"], None, ky)]]
    for s in range(2):
        olo, ohi = oo.sigma_band(och[s], tl, fr)
        d = max(np.abs(lo[s] - olo).max(), np.abs(hi[s] - ohi).max())
        print(f"band sample {s}: max |GPU - oracle| {d:.3e} mb (band width up to {np.max(ohi - olo):.3e} mb)",
              flush=True)
        assert d <= SIGMA_TOL


def test_grid_rejects_unknown_packet_kind():
    ctx = wp.Context(0)
    with pytest.raises(wp.WPCDError) as ei:
        ctx.grid(grids.tan2_bounded(10), 8, 7)
    assert ei.value.code == wp.WPCD_ERR_INVALID
