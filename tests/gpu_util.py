"""Helpers shared by the GPU tests: run a batch through the library and unpack per-item results."""
import numpy as np
import torch

import paper_2106_00454_amd as wp
from synth import device as sdev

TLAB = np.linspace(1.0, 350.0, 30)


def run_items(ctx, items, u, mode, tlab=TLAB):
    """items: list of (grid, n_ch, J, sample_id); u: packed device tensor (or list of host matrices)."""
    b = ctx.batch(items)
    if not isinstance(u, torch.Tensor):
        u = sdev.pack_host_matrices(b.layout["u_elems"], b.u_off, u, torch.float64)
    bufs = b.alloc()
    sig = None
    tl = None
    if tlab is not None:
        tl = torch.tensor(tlab, dtype=torch.float64, device="cuda")
        sig = torch.full((b.layout["n_samples"] * len(tlab),), np.nan, dtype=torch.float64, device="cuda")
    b.run(u, bufs, mode, tl, sig)
    torch.cuda.synchronize()
    host = {k: v.cpu().numpy() for k, v in bufs.items()}
    if sig is not None:
        host["sigma"] = sig.cpu().numpy().reshape(b.layout["n_samples"], len(tlab))
    return b, host


def item_view(b, host, i):
    g, K, J, sid = b.items[i]
    N = g.n_wp
    n = K * N
    vo, eo, to, do, mo = b.v_off[i], b.eval_off[i], b.t_off[i], b.delta_off[i], b.mix_off[i]
    t = host["t"][to:to + 2 * N * K * K].reshape(N, K, K, 2)
    return {
        "v": host["v64"][vo:vo + n * n].reshape(n, n),
        "evals": host["eval"][eo:eo + n],
        "evecs": host["evec"][vo:vo + n * n].reshape(n, n),
        "t": t[..., 0] + 1j * t[..., 1],
        "delta": host["delta"][do:do + N * K].reshape(N, K),
        "mix": host["mix"][mo:mo + N],
        "s_dev": host["s_dev"][do:do + N * K].reshape(N, K),
        "eig_status": int(host["eig_status"][i]),
        "t_status": int(host["t_status"][i]),
    }


def dmod180(a, b):
    return np.abs(((np.asarray(a) - np.asarray(b) + 90.0) % 180.0) - 90.0)
