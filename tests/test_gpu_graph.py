"""HIP graph capture of a batch's whole path (wpcd_graph_create / wpcd_graph_launch) and wpcd_run.

A mixed batch -- coupled fine-mesh items (LDS eigensolver), affine items of
the J <= 6 sweep at N_WP = 50 and a coupled N_WP = 150 item (device-memory
eigensolver, hundreds of launches) -- is captured once.  The graph is then
replayed several times; before each replay the affine coefficients are
changed in place and other eager device work runs, and each replay is
compared with an eager run (the separate library calls) of the same inputs
on separate buffers.  Both run the same kernels on the same data, so the
results must agree to rounding level (they are in fact expected to be
bitwise equal; the bar is 1e-12 relative).  wpcd_run (the whole path in one
call) is compared the same way.
"""
import numpy as np
import pytest
import torch

import paper_2106_00454_amd as wp
from synth import configs, sweep
from synth import device as sdev
from tests.gpu_util import TLAB

pytestmark = pytest.mark.gpu

KEYS = ("eval", "evec", "t", "delta", "mix", "s_dev")


def _close(tag, a, b):
    for k in KEYS + ("sigma",):
        x, y = a[k], b[k]
        assert x.shape == y.shape, (tag, k)
        scale = max(1.0, float(np.nanmax(np.abs(y))))
        d = float(np.nanmax(np.abs(x - y))) if x.size else 0.0
        assert np.array_equal(np.isnan(x), np.isnan(y)), (tag, k)
        assert d <= 1e-12 * scale, f"{tag}: {k} differs by {d:.3e}"
    for k in ("eig_status", "t_status"):
        assert np.array_equal(a[k], b[k]), (tag, k)


def _host(bufs, sig):
    h = {k: v.cpu().numpy() for k, v in bufs.items()}
    h["sigma"] = sig.cpu().numpy()
    return h


@pytest.mark.timeout(300)
def test_graph_replays_match_eager_runs():
    ctx = wp.Context(0)
    gc = ctx.grid(configs.grid("coupled_yukawa"), 8)
    cache = sweep.TermCache()
    g50 = ctx.grid(sweep.grid_bounds(50), sweep.N_GAUSS)
    g150 = ctx.grid(sweep.grid_bounds(150), sweep.N_GAUSS)
    chans = (0, 7, 14, 16)  # 1S0, 3P0, 3S1-3D1, 3D3-3G3
    bases = {c: ctx.basis(g50, sweep.CHANNELS[c][1], cache.terms(("lib", 50), g50.nodes, c)) for c in chans}
    big = ctx.basis(g150, 2, cache.terms(("lib", 150), g150.nodes, 14))
    specs, coef_of = [], []
    for s in range(4):                           # fine-mesh coupled items
        specs.append((gc, 2, 1, s))
        coef_of.append(None)
    for s in range(4):                           # affine items of four samples
        for c in chans:
            specs.append((bases[c].grid, sweep.CHANNELS[c][1], sweep.CHANNELS[c][2], 4 + s, bases[c]))
            coef_of.append((s, c))
    specs.append((g150, 2, 1, 8, big))          # device-memory eigensolver
    coef_of.append((0, 14))
    b = ctx.batch(specs)
    coeffs = np.array([configs.yukawa_coefficients(s) for s in range(4)])
    u = sdev.pack_coupled_yukawa(b.layout["u_elems"], b.u_off[:4], gc.nodes, coeffs, torch.float64,
                                 terms=configs.coupled_yukawa_terms(gc.nodes))

    def coef_host(shift):
        c = np.zeros(max(1, b.layout["coef_elems"]))
        for i, cs in enumerate(coef_of):
            if cs is not None:
                s, ch = cs
                v = sweep.coefficients(s + shift, ch)
                c[b.coef_off[i]:b.coef_off[i] + len(v)] = v
        return c

    coef = torch.tensor(coef_host(0), dtype=torch.float64, device="cuda")
    tl = torch.tensor(TLAB, dtype=torch.float64, device="cuda")
    n_sig = b.layout["n_samples"] * TLAB.size
    bufs_g, bufs_e = b.alloc(), b.alloc()
    sig_g = torch.full((n_sig,), np.nan, dtype=torch.float64, device="cuda")
    sig_e = torch.full((n_sig,), np.nan, dtype=torch.float64, device="cuda")
    b.run(u, bufs_e, wp.MIXED, tl, sig_e, coef=coef)   # first use: the second stream exists before the capture
    torch.cuda.synchronize()
    graph = b.graph(u, bufs_g, wp.MIXED, tl, sig_g, coef=coef)
    torch.cuda.synchronize()
    print(f"graph: {graph.nodes} nodes for {len(specs)} items", flush=True)
    assert graph.nodes > 10
    # capturing enqueued nothing: the graph's buffers are still untouched
    assert torch.isnan(sig_g).all()
    x = torch.randn(512, 512, device="cuda")
    for rep in range(4):
        coef.copy_(torch.tensor(coef_host(rep), dtype=torch.float64))
        y = x @ x                                  # eager work between replays
        b.run(u, bufs_e, wp.MIXED, tl, sig_e, coef=coef)
        torch.cuda.synchronize()
        graph.launch()
        torch.cuda.synchronize()
        he, hg = _host(bufs_e, sig_e), _host(bufs_g, sig_g)
        assert (he["eig_status"] > 0).all() and (he["t_status"] == 0).all()
        _close(f"replay {rep}", hg, he)
        del y
    # wpcd_run: the whole path in one call
    bufs_r = b.alloc()
    sig_r = torch.full((n_sig,), np.nan, dtype=torch.float64, device="cuda")
    b.run_path(u, bufs_r, wp.MIXED, tl, sig_r, coef=coef)
    torch.cuda.synchronize()
    _close("wpcd_run", _host(bufs_r, sig_r), he)
    graph.close()


def test_graph_refused_while_timing():
    ctx = wp.Context(0)
    g = ctx.grid(configs.grid("yamaguchi_s"), 8)
    b = ctx.batch([(g, 1, 0, 0)])
    u = torch.zeros(b.layout["u_elems"], dtype=torch.float64, device="cuda")
    bufs = b.alloc()
    ctx.profile(True)
    with pytest.raises(wp.WPCDError) as ei:
        b.graph(u, bufs, wp.MIXED)
    assert ei.value.code == wp.WPCD_ERR_INVALID
    ctx.profile(False)
    with pytest.raises(wp.WPCDError) as ei:
        b.run_path(None, bufs, wp.MIXED)         # fine-mesh items but no u
    assert ei.value.code == wp.WPCD_ERR_INVALID


@pytest.mark.timeout(300)
def test_autotune_picks_a_schedule_and_caches_it(tmp_path):
    # the autotuner times the candidate schedules on the batch, keeps the
    # fastest in the context and records it; a second call with the same
    # batch signature takes it from the cache.  The chosen schedule's results
    # agree with the default schedule's within the refinement's accuracy.
    ctx = wp.Context(0)
    gc = ctx.grid(configs.grid("coupled_yukawa"), 8)
    gy = ctx.grid(configs.grid("yamaguchi_s"), 8)
    specs = [(gc, 2, 1, s) for s in range(40)] + [(gy, 1, 0, 40 + s) for s in range(24)]
    b = ctx.batch(specs)
    from synth import potentials
    mats = [sum(ci * t for ci, t in zip(configs.yukawa_coefficients(s), configs.coupled_yukawa_terms(gc.nodes)))
            for s in range(40)]
    mats += [potentials.yamaguchi(gy.nodes, gy.nodes, configs.yamaguchi_lambda(s), configs.YAMAGUCHI_BETA)
             for s in range(24)]
    u = sdev.pack_host_matrices(b.layout["u_elems"], b.u_off, mats, torch.float64)
    tl = torch.tensor(TLAB, dtype=torch.float64, device="cuda")
    n_sig = b.layout["n_samples"] * TLAB.size
    ref_bufs = b.alloc()
    ref_sig = torch.empty(n_sig, dtype=torch.float64, device="cuda")
    b.run(u, ref_bufs, wp.MIXED, tl, ref_sig)
    bufs = b.alloc()
    sig = torch.empty(n_sig, dtype=torch.float64, device="cuda")
    cache = str(tmp_path / "tune.txt")
    r = b.autotune(u, bufs, wp.MIXED, tl, sig, reps=1, cache_path=cache)
    print(f"autotune: {r}", flush=True)
    assert not r["from_cache"] and len(r["cand_ms"]) == 4
    assert (r["jacobi_block"], r["refine_gemm"]) in {(0, 0), (5, 0), (0, 1), (5, 1)}
    assert r["best_ms"] == min(r["cand_ms"])
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and lines[0].startswith("mixed:")
    r2 = b.autotune(u, bufs, wp.MIXED, tl, sig, reps=1, cache_path=cache)
    assert r2["from_cache"] and (r2["jacobi_block"], r2["refine_gemm"]) == (r["jacobi_block"], r["refine_gemm"])
    b.run(u, bufs, wp.MIXED, tl, sig)              # with the chosen schedule
    torch.cuda.synchronize()
    h, hr = bufs["delta"].cpu().numpy(), ref_bufs["delta"].cpu().numpy()
    dd = np.abs(((h - hr + 90.0) % 180.0) - 90.0).max()
    ds = np.abs(sig.cpu().numpy() - ref_sig.cpu().numpy()).max()
    print(f"chosen vs default schedule: ddelta={dd:.3e} dsigma={ds:.3e}", flush=True)
    assert dd <= 1e-4 and ds <= 1e-4
    assert (bufs["eig_status"].cpu().numpy() > 0).all()
