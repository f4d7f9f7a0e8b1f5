"""Convergence-aware enqueueing of the device-memory Jacobi (Sec. 4.2, cyclic
Jacobi run to convergence), through the C ABI.

Outside stream capture the library enqueues the sweeps of a device-memory
Jacobi launch sequence a few at a time and stops two sweeps after the first
sweep that left every item converged; a captured sequence (HIP graph)
enqueues all max_sweeps sweeps, converged items returning at once.  Both
must give the same results bit for bit, and the eager run must enqueue
exactly max(status) + 2 sweeps (status = sweeps to convergence) per launch
sequence while that is below max_sweeps.  Covered: the plain FP64 path (every
item in device memory) and the mixed path's items above n = 200, against the
oracle as well (phase shifts within 0.01 deg, sigma within 0.01 mb).
"""
import numpy as np
import pytest
import torch

import paper_2106_00454_amd as wp
from oracle import observables as oo
from oracle import wpcd as ow
from synth import configs, grids
from synth import device as sdev
from tests.gpu_util import TLAB, check_item, item_view

pytestmark = pytest.mark.gpu

LOOKAHEAD = 2
KEYS = ("eval", "evec", "t", "delta", "mix", "s_dev", "eig_status", "t_status")


def _items(ctx):
    k1 = configs.grid("coupled_yukawa")          # n = 200
    k3 = grids.tan2_bounded(120)                  # n = 240: device memory in both modes
    g1, g3 = ctx.grid(k1, configs.N_GAUSS), ctx.grid(k3, configs.N_GAUSS)
    cs = [configs.yukawa_coefficients(s) for s in range(4)]
    items = [(g1, 2, 1, 0), (g1, 2, 1, 1), (g3, 2, 1, 2), (g3, 2, 1, 3)]
    mats = [sum(c * t for c, t in zip(cs[i], configs.coupled_yukawa_terms(g.nodes)))
            for i, (g, _, _, _) in enumerate(items)]
    return items, mats, [k1, k1, k3, k3], cs


@pytest.mark.timeout(300)
@pytest.mark.parametrize("mode", [wp.F64, wp.MIXED])
def test_sweeps_stop_after_convergence_and_match_captured_run(mode):
    # every item starts cold (jacobi_start = 1): in the mixed path the two
    # n = 240 items then form one launch sequence (with warm starts the
    # second one would run in a sequence of its own, from the first one's
    # eigenvectors)
    ctx = wp.Context(0, jacobi_start=1)
    items, mats, ks, cs = _items(ctx)
    b = ctx.batch(items)
    u = sdev.pack_host_matrices(b.layout["u_elems"], b.u_off, mats, torch.float64)
    tl = torch.tensor(TLAB, dtype=torch.float64, device="cuda")
    n_sig = b.layout["n_samples"] * TLAB.size
    bufs_e, bufs_g = b.alloc(), b.alloc()
    sig_e = torch.full((n_sig,), np.nan, dtype=torch.float64, device="cuda")
    sig_g = torch.full((n_sig,), np.nan, dtype=torch.float64, device="cuda")
    b.jacobi_launches(clear=True)
    b.run(u, bufs_e, mode, tl, sig_e)
    torch.cuda.synchronize()
    cnt = b.jacobi_launches(clear=True)
    st = bufs_e["eig_status"].cpu().numpy()
    print(f"mode={mode}: eager run {cnt}, eig status {st.tolist()}", flush=True)
    assert (st > 0).all()
    # one launch sequence: all items in F64, the n = 240 class in MIXED
    dev = st if mode == wp.F64 else st[2:]
    assert cnt["sweeps"] == min(int(dev.max()) + LOOKAHEAD, 30)
    assert cnt["launches"] > 0
    # the captured sequence enqueues every sweep and must agree bit for bit
    graph = b.graph(u, bufs_g, mode, tl, sig_g)
    graph.launch()
    torch.cuda.synchronize()
    cg = b.jacobi_launches(clear=True)
    assert cg["sweeps"] == 30, cg
    for key in KEYS:
        x, y = bufs_g[key].cpu().numpy(), bufs_e[key].cpu().numpy()
        assert np.array_equal(x, y, equal_nan=True), key
    assert np.array_equal(sig_g.cpu().numpy(), sig_e.cpu().numpy())
    graph.close()
    # and the eager results against the oracle
    host = {k: v.cpu().numpy() for k, v in bufs_e.items()}
    host["sigma"] = sig_e.cpu().numpy().reshape(b.layout["n_samples"], TLAB.size)
    for i, k in enumerate(ks):
        xo, _ = ow.gauss_nodes(k, configs.N_GAUSS)
        ref = ow.solve_channel(k, configs.N_GAUSS, sum(c * t for c, t in zip(cs[i], configs.coupled_yukawa_terms(xo))),
                               2)
        _, kbar, _ = ow.bins(k)
        sig_ref = oo.sigma_tot([(1, ref["delta"], ref["mix"])], kbar, TLAB, k[-1])
        check_item(f"feedback mode={mode} item={i}", item_view(b, host, i), ref, k, mode, 1, sig_ref,
                   host["sigma"][i])


def test_sweep_cap_still_enqueues_every_sweep():
    # max_sweeps = 3 from a cold start: no sweep leaves the items converged,
    # so all three are enqueued and the status is WPCD_ERR_NOCONV
    ctx = wp.Context(0, max_sweeps=3)
    items, mats, _, _ = _items(ctx)
    b = ctx.batch(items)
    u = sdev.pack_host_matrices(b.layout["u_elems"], b.u_off, mats, torch.float64)
    bufs = b.alloc()
    b.run(u, bufs, wp.F64)
    torch.cuda.synchronize()
    cnt = b.jacobi_launches()
    st = bufs["eig_status"].cpu().numpy()
    print(f"max_sweeps=3: {cnt}, status {st.tolist()}", flush=True)
    assert cnt["sweeps"] == 3
    assert (st == wp.WPCD_ERR_NOCONV).all()
