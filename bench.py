#!/usr/bin/env python3
"""Channel-solves per second of the WPCD path on one MI355X.

Workload: coupled S-D channel (l = 0/2, J = 1) with three central Yukawa terms
and a tensor-like coupling, N_WP = 100 momentum bins on [0, 4] fm^-1 (200 x 200
H), 8 Gauss points per bin; every item is a distinct seeded potential sample.
One step = the whole path over one batch of items already resident in HBM:
projection of the FP32 fine-mesh potential, FP32 Jacobi in LDS plus FP64
refinement, T at all 100 bin energies, phase shifts / mixing angles and the
total cross section at 30 T_lab values per item.

Also reported: the plain FP64 path (one item per launch sequence, synchronised
per item) on the same GPU, per-stage times from the library's event timers,
the roofline of the dominant kernel, and the FP64 CPU oracle on the host cores.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "channel-solves/sec (coupled, N_WP=100, all bin energies) batched vs plain; p99 ms"
N_WP = 100
N_CH = 2
N_TLAB = 30
PEAK_FP32_PUBLISHED = 157.3                         # TFLOP/s, published FP32 vector peak (packed FMA)
PEAK_FP32_VALU = 256 * 4 * 16 * 2 * 2.4e9 / 1e12   # TFLOP/s, non-packed FP32 FMA (packed FP32 is off)
PEAK_FP64_MFMA = 78.6                               # TFLOP/s, published dense FP64 matrix peak


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when the kernel's sources changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_jacobi_coupled_n200.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            rec[k.strip()] = v.strip()
    if rec.get("kernel") != kernel:
        return None
    h = hashlib.sha256()
    for f in rec.get("source_files", "").split():
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest()[:16] != rec.get("source_sha256"):
        return None
    return float(rec["traffic_bytes_per_launch"]), path


# ----------------------------------------------------------------- CPU oracle
_W = {}


def _worker_init():
    from oracle import wpcd as ow
    from synth import configs
    k = configs.grid("coupled_yukawa")
    x, _ = ow.gauss_nodes(k, configs.N_GAUSS)
    _W["k"] = k
    _W["terms"] = configs.coupled_yukawa_terms(x)


def _worker_item(sid: int) -> float:
    from oracle import observables as oo
    from oracle import wpcd as ow
    from synth import configs
    k = _W["k"]
    u = sum(c * t for c, t in zip(configs.yukawa_coefficients(sid), _W["terms"]))
    t0 = time.perf_counter()
    r = ow.solve_channel(k, configs.N_GAUSS, u, N_CH)
    _, kbar, _ = ow.bins(k)
    oo.sigma_tot([(1, r["delta"], r["mix"])], kbar, np.linspace(1.0, 350.0, N_TLAB), k[-1])
    return time.perf_counter() - t0


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(seconds: float) -> dict:
    """The oracle as it stands, one item per task, on all host cores."""
    cores = os.cpu_count() or 1
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"
    ctx = mp.get_context("spawn")
    per_item = []
    with cf.ProcessPoolExecutor(max_workers=cores, mp_context=ctx, initializer=_worker_init) as ex:
        list(ex.map(_worker_item, range(cores)))          # warm every worker
        done, t0 = 0, time.perf_counter()
        chunk = 4 * cores
        while time.perf_counter() - t0 < seconds:
            per_item += list(ex.map(_worker_item, range(done, done + chunk)))
            done += chunk
        wall = time.perf_counter() - t0
    return {"value": done / wall, "unit": "channel-solves/s", "cores": cores, "kind": "oracle",
            "cpu_model": _cpu_model(), "per_item_p50_ms": float(np.percentile(per_item, 50) * 1e3),
            "sample": f"{done} coupled N_WP=100 items (a1-a9 incl. sigma_tot), FP64 NumPy/LAPACK, "
                      f"one single-threaded process per core, {wall:.1f} s wall"}


# ------------------------------------------------------- other workloads
def _jacobi_flops(ns, sweeps):
    """One-sided Jacobi work: per sweep n(n-1)/2 pair rotations of 12 n flops."""
    ns = np.asarray(ns, dtype=np.float64)
    return float(np.sum(np.asarray(sweeps, dtype=np.float64) * ns * (ns - 1) / 2 * 12 * ns))


def _register_bases(ctx, cache, n_wps, channels):
    from synth import sweep
    grids = {N: ctx.grid(sweep.grid_bounds(N), sweep.N_GAUSS) for N in n_wps}
    bases = {}
    for N in n_wps:
        for c in channels:
            bases[(c, N)] = ctx.basis(grids[N], sweep.CHANNELS[c][1], cache.terms(("lib", N), grids[N].nodes, c))
    return grids, bases


def _affine_batch_run(args, ctx, specs, coefs, tlab, label):
    """Stage an affine batch, warm up, time args.steps passes; returns the common JSON fields."""
    import torch
    import paper_2106_00454_amd as wp
    b = ctx.batch(specs)
    c = np.zeros(max(1, b.layout["coef_elems"]))
    for i, ci in enumerate(coefs):
        c[b.coef_off[i]:b.coef_off[i] + len(ci)] = ci
    coef = torch.tensor(c, dtype=torch.float64, device="cuda")
    bufs = b.alloc()
    tl = torch.tensor(tlab, dtype=torch.float64, device="cuda")
    sigma = torch.empty(b.layout["n_samples"] * len(tlab), dtype=torch.float64, device="cuda")
    for _ in range(args.warmup):
        b.run(None, bufs, wp.MIXED, tl, sigma, coef=coef)
    torch.cuda.synchronize()
    st_e = bufs["eig_status"].cpu().numpy()
    st_t = bufs["t_status"].cpu().numpy()
    if (st_e <= 0).any() or (st_t != 0).any():
        log(f"{label}: item failures: eig {int((st_e <= 0).sum())} tmatrix {int((st_t != 0).sum())}")
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.run(None, bufs, wp.MIXED, tl, sigma, coef=coef)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stages = ctx.stage_times()
    ctx.profile(False)
    ns = [sp[1] * sp[0].n_wp for sp in specs]
    value = len(specs) * args.steps / wall
    log(f"{label}: {value:.0f} channel-solves/s, {wall / args.steps * 1e3:.2f} ms/step")
    avg = {k: (ms / cnt if cnt else 0.0) for k, (ms, cnt) in stages.items()}
    jac = _jacobi_flops(ns, np.maximum(st_e, 0)) / (stages["jacobi_f32"][0] / args.steps * 1e-3) / 1e12
    roof = {"bound": "alu", "achieved": jac, "peak": PEAK_FP32_VALU, "unit": "TFLOP/s", "frac": jac / PEAK_FP32_VALU,
            "traffic": None, "kernel": "jacobi_f32 (all size classes)",
            "avg_stage_ms": stages["jacobi_f32"][0] / args.steps,
            "note": "upper bound: 12n flops per column-pair visit, every visit counted as a rotation"}
    return {"value": value, "unit": "channel-solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
            "jacobi_sweeps_mean": float(st_e[st_e > 0].mean()) if (st_e > 0).any() else None,
            "stages_ms_per_step": {k: ms / args.steps for k, (ms, cnt) in stages.items() if cnt},
            "stage_avg_launch_ms": {k: v for k, v in avg.items() if v}, "roofline": roof, "cpu_baseline": None}


_TERMS = {}


def _term_cache():
    """One host cache of the unit-strength term matrices for every workload of a run."""
    from synth import sweep
    if "cache" not in _TERMS:
        _TERMS["cache"] = sweep.TermCache()
    return _TERMS["cache"]


def run_sweep(args) -> dict:
    """J <= 6 batched sweep: args.samples x 20 channels, N_WP from {50, 100, 150}, affine bases."""
    import paper_2106_00454_amd as wp
    from synth import sweep
    ctx = wp.Context(0, jacobi_block=args.jacobi_block, jacobi_stop_f32=args.jacobi_stop,
                     jacobi_start=args.jacobi_start, refine_gemm=args.refine_gemm, refine_steps=args.refine_steps,
                     refine_close_log10=args.refine_close, refine_rr_steps=args.refine_rr)
    t0 = time.perf_counter()
    _, bases = _register_bases(ctx, _term_cache(), sweep.N_WP_CHOICES, range(len(sweep.CHANNELS)))
    log(f"sweep: registered {len(bases)} bases in {time.perf_counter() - t0:.1f} s")
    items = sweep.items(args.samples)
    specs = [(bases[(c, N)].grid, sweep.CHANNELS[c][1], sweep.CHANNELS[c][2], s, bases[(c, N)])
             for s, c, N in items]
    coefs = [sweep.coefficients(s, c) for s, c, N in items]
    out = _affine_batch_run(args, ctx, specs, coefs, sweep.TLAB, "sweep")
    out["metric"] = "channel-solves/sec (J<=6 sweep, 20 channels, N_WP in {50,100,150}, sigma_tot per sample)"
    out["config"] = {"workload": f"batched sweep: {args.samples} samples x 20 channels (J<=6), N_WP uniform in "
                                 "{50,100,150}, affine Yukawa+tensor bases, sigma_tot at 30 T_lab per sample",
                     "items_per_step": len(specs)}
    return out


def run_large(args) -> dict:
    """Large mesh: 64 samples x 6 coupled channels (J = 1..6) at N_WP = args.large_nwp."""
    import paper_2106_00454_amd as wp
    from synth import sweep
    ctx = wp.Context(0, jacobi_block=args.jacobi_block, jacobi_stop_f32=args.jacobi_stop,
                     jacobi_start=args.jacobi_start, refine_gemm=args.refine_gemm, refine_steps=args.refine_steps,
                     refine_close_log10=args.refine_close, refine_rr_steps=args.refine_rr)
    coupled = [c for c in range(len(sweep.CHANNELS)) if sweep.CHANNELS[c][1] == 2]
    N = args.large_nwp
    t0 = time.perf_counter()
    _, bases = _register_bases(ctx, sweep.TermCache(), (N,), coupled)
    log(f"large: registered {len(bases)} bases in {time.perf_counter() - t0:.1f} s")
    specs, coefs = [], []
    for s in range(64):
        for c in coupled:
            specs.append((bases[(c, N)].grid, 2, sweep.CHANNELS[c][2], s, bases[(c, N)]))
            coefs.append(sweep.coefficients(s, c))
    out = _affine_batch_run(args, ctx, specs, coefs, sweep.TLAB, "large")
    out["metric"] = f"channel-solves/sec (coupled, N_WP={N}, device-memory eigensolver)"
    out["config"] = {"workload": f"large mesh: 64 samples x 6 coupled channels (J=1..6), N_WP={N} "
                                 f"({2 * N}x{2 * N} H), affine bases", "items_per_step": len(specs)}
    return out


def run_mi(args) -> dict:
    """The matrix-inversion solver on the coupled workload: args.batch coupled
    N_WP-independent items (the same Yukawa + tensor samples), N_Q nodes on
    [0, 4] fm^-1, the 30 T_lab energies of sigma_tot, one FP64 LU per item and
    energy, phase shifts, mixing angles and sigma_tot."""
    import torch
    import paper_2106_00454_amd as wp
    from synth import configs
    ctx = wp.Context(0)
    B, nq = args.batch, args.mi_nq
    tl = np.linspace(1.0, 350.0, N_TLAB)
    s = wp.MiSolver(ctx, [(2, 1, i) for i in range(B)], nq, 4.0, tl)
    pts = s.points
    coeffs = np.array([configs.yukawa_coefficients(i) for i in range(B)])
    terms = configs.coupled_yukawa_terms(pts)
    t = torch.from_numpy(np.stack([x.ravel() for x in terms])).cuda()
    c = torch.as_tensor(coeffs, dtype=torch.float64, device="cuda")
    u = (c @ t).reshape(-1).contiguous()
    assert u.numel() == s.layout["u_elems"]
    bufs = s.alloc()
    for _ in range(args.warmup):
        s.solve(u, bufs)
    torch.cuda.synchronize()
    st = bufs["status"].cpu().numpy()
    if (st != 0).any():
        log(f"mi: {int((st != 0).sum())} items flagged")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s.solve(u, bufs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    value = B * args.steps / wall
    m = 2 * (nq + 1)
    flop = B * N_TLAB * (2.0 / 3.0 * m ** 3 + 2.0 * 2 * m * m)     # LU of [A | 2 right-hand sides]
    log(f"mi: {value:.0f} channel-solves/s ({value * N_TLAB:.0f} energy-solves/s), {wall / args.steps * 1e3:.2f} ms/step")
    return {"metric": f"channel-solves/sec (coupled, matrix inversion, N_Q={nq}, {N_TLAB} energies)",
            "value": value, "unit": "channel-solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"matrix inversion (K-matrix route): {B} coupled S-D Yukawa+tensor items, "
                                   f"N_Q={nq} Gauss nodes on [0,4] fm^-1, sigma_tot at {N_TLAB} T_lab",
                       "items_per_step": B, "energies": N_TLAB, "system_size": m},
            "roofline": {"bound": "alu", "achieved": flop * args.steps / wall / 1e12, "peak": 78.6,
                         "unit": "TFLOP/s", "frac": flop * args.steps / wall / 1e12 / 78.6,
                         "kernel": "mi_solve_kernel (FP64 VALU elimination in LDS)", "traffic": None},
            "cpu_baseline": None}


def run_serve(args) -> dict:
    """Poisson arrivals of parameter-vector requests with random channel subsets."""
    import paper_2106_00454_amd as wp
    from synth import sweep
    ctx = wp.Context(0, jacobi_block=args.jacobi_block, jacobi_stop_f32=args.jacobi_stop,
                     jacobi_start=args.jacobi_start, refine_gemm=args.refine_gemm, refine_steps=args.refine_steps,
                     refine_close_log10=args.refine_close, refine_rr_steps=args.refine_rr)
    n_wps = (50, 100, 150, 200)
    t0 = time.perf_counter()
    _, bases = _register_bases(ctx, _term_cache(), n_wps, range(len(sweep.CHANNELS)))
    log(f"serve: registered {len(bases)} bases in {time.perf_counter() - t0:.1f} s")
    srv = wp.Server(ctx, hbm_budget_bytes=16 << 30, max_inflight=4, max_batch_items=2048)
    rng = np.random.default_rng(np.random.SeedSequence([20210601 + 4, 0]))
    warm = args.serve_warmup
    n_req = int((args.duration + warm) * args.rate * 1.2) + 10
    gaps = rng.exponential(1.0 / args.rate, n_req)
    arrivals = np.cumsum(gaps)
    arrivals = arrivals[arrivals < args.duration + warm]
    reqs = []
    for r in range(arrivals.size):
        k = int(rng.integers(1, 21))
        chans = rng.choice(20, size=k, replace=False)
        N = int(rng.choice(n_wps))
        reqs.append([(bases[(int(c), N)], sweep.CHANNELS[int(c)][2], sweep.coefficients(r, int(c))) for c in chans])
    log(f"serve: {len(reqs)} requests generated")
    lat, t_done, outstanding = [], [], []
    n_items = 0
    start = time.perf_counter()
    nxt = 0
    while nxt < len(reqs) or outstanding:
        now = time.perf_counter() - start
        while nxt < len(reqs) and arrivals[nxt] <= now:
            tk = srv.submit(reqs[nxt], sweep.TLAB)
            outstanding.append((tk, arrivals[nxt], len(reqs[nxt])))
            nxt += 1
        still = []
        for tk, ta, nc in outstanding:
            if srv.poll(tk):
                tnow = time.perf_counter() - start
                if ta >= warm:
                    lat.append((tnow - ta) * 1e3)
                    t_done.append(tnow)
                    n_items += nc
                if tk.code != 0:
                    log(f"serve: request failed with code {tk.code}")
            else:
                still.append((tk, ta, nc))
        outstanding = still
    st = srv.stats()
    srv.close()
    lat = np.array(lat)
    span = max(t_done) - warm if t_done else float("nan")
    out = {
        "metric": "serving: p50/p99 latency (ms) and channel-solves/s under Poisson arrivals",
        "value": float(np.percentile(lat, 99)), "unit": "ms (p99 latency)", "n_gpus": 1, "steps": len(lat),
        "warmup": int(np.sum(arrivals < warm)), "ms_per_step": float(np.mean(lat)), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"serving: Poisson arrivals at {args.rate:.0f} req/s for {args.duration:.0f} s after "
                               f"{warm:.0f} s warm-up; each request 1-20 random channels of the J<=6 set, "
                               "N_WP uniform in {50,100,150,200}, sigma_tot at 30 T_lab"},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "max": float(lat.max())},
        "throughput": {"requests_per_s": len(lat) / span, "channel_solves_per_s": n_items / span},
        "server": st, "roofline": None, "cpu_baseline": None,
    }
    log(f"serve: p50 {out['latency_ms']['p50']:.2f} ms p99 {out['latency_ms']['p99']:.2f} ms, "
        f"{out['throughput']['channel_solves_per_s']:.0f} channel-solves/s, {st['batches']} batches")
    return out


# ----------------------------------------------------------------- GPU path
def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--plain-items", type=int, default=16)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cold", action="store_true", help="skip the cold-start comparison run")
    ap.add_argument("--jacobi-block", type=int, default=0, help="LDS Jacobi variant (wpcd_config.jacobi_block; 0: default)")
    ap.add_argument("--jacobi-start", type=int, default=0, help="LDS Jacobi start (wpcd_config.jacobi_start; 0: warm, 1: cold)")
    ap.add_argument("--refine-gemm", type=int, default=0,
                    help="refinement products (wpcd_config.refine_gemm; 0: whole-item for n 193..208, 1: tiles)")
    ap.add_argument("--refine-steps", type=int, default=2, help="FP64 refinement steps (wpcd_config.refine_steps)")
    ap.add_argument("--refine-close", type=int, default=0, help="wpcd_config.refine_close_log10 (0: default)")
    ap.add_argument("--refine-rr", type=int, default=0,
                    help="wpcd_config.refine_rr_steps: trailing refinement steps with Rayleigh-Ritz (0: every step)")
    ap.add_argument("--jacobi-stop", type=float, default=0.0, help="FP32 Jacobi stopping threshold (wpcd_config.jacobi_stop_f32; 0: default)")
    ap.add_argument("--workload", choices=("coupled", "sweep", "large", "serve", "mi"), default="coupled",
                    help="coupled: the headline line; sweep / large / serve: the other workloads")
    ap.add_argument("--samples", type=int, default=512, help="sweep: parameter samples per step")
    ap.add_argument("--large-nwp", type=int, default=300, help="large: N_WP of the coupled items")
    ap.add_argument("--mi-nq", type=int, default=48, help="mi: Gauss nodes of the matrix-inversion solver")
    ap.add_argument("--rate", type=float, default=2000.0, help="serve: Poisson arrival rate (requests/s)")
    ap.add_argument("--duration", type=float, default=20.0, help="serve: seconds of arrivals after warm-up")
    ap.add_argument("--serve-warmup", type=float, default=5.0, help="serve: seconds of arrivals before the measurement")
    ap.add_argument("--no-extras", action="store_true",
                    help="coupled workload only (by default a short J<=6 sweep and a short serving run follow)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: items are independent and the library has no multi-GPU path "
              "(batches would shard by parameter sample, one process per GPU); run with --gpus 1", flush=True)
        return 2

    if args.workload != "coupled":
        out = {"sweep": run_sweep, "large": run_large, "serve": run_serve, "mi": run_mi}[args.workload](args)
        print(json.dumps(out), flush=True)
        return 0

    import torch
    import paper_2106_00454_amd as wp
    from synth import configs
    from synth import device as sdev

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ctx = wp.Context(0, jacobi_block=args.jacobi_block, jacobi_stop_f32=args.jacobi_stop,
                     jacobi_start=args.jacobi_start, refine_gemm=args.refine_gemm, refine_steps=args.refine_steps,
                     refine_close_log10=args.refine_close, refine_rr_steps=args.refine_rr)
    k = configs.grid("coupled_yukawa")
    g = ctx.grid(k, configs.N_GAUSS)
    B = args.batch
    coeffs = np.array([configs.yukawa_coefficients(s) for s in range(B)])
    b = ctx.batch([(g, N_CH, 1, s) for s in range(B)])
    log(f"staging {B} items: {b.layout['u_elems'] * 4 / 1e9:.1f} GB of FP32 fine-mesh potentials")
    terms = configs.coupled_yukawa_terms(g.nodes)
    u = sdev.pack_coupled_yukawa(b.layout["u_elems"], b.u_off, g.nodes, coeffs, torch.float32, terms=terms)
    bufs = b.alloc()
    tlab = torch.linspace(1.0, 350.0, N_TLAB, dtype=torch.float64, device=dev)
    sigma = torch.empty(B * N_TLAB, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()

    for _ in range(args.warmup):
        b.run(u, bufs, wp.MIXED, tlab, sigma)
    torch.cuda.synchronize()
    st_e = bufs["eig_status"].cpu().numpy()
    st_t = bufs["t_status"].cpu().numpy()
    if (st_e <= 0).any() or (st_t != 0).any():
        log(f"item failures: eig {int((st_e <= 0).sum())} tmatrix {int((st_t != 0).sum())}")
    sweeps = st_e[st_e > 0].astype(np.float64)

    ctx.profile(True)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record()
    for i in range(args.steps):
        b.run(u, bufs, wp.MIXED, tlab, sigma)
        evs[i + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stages = ctx.stage_times()
    counts = ctx.jacobi_counts()
    ctx.profile(False)
    step_ms = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps)])
    value = B * args.steps / wall
    log(f"batched: {value:.0f} channel-solves/s, {wall / args.steps * 1e3:.2f} ms/step")

    # roofline of the dominant kernel group
    n = N_CH * N_WP
    avg = {s: (ms / cnt if cnt else 0.0) for s, (ms, cnt) in stages.items()}
    # algorithmic FLOPs of the LDS Jacobi per launch: a dot product (2n) per
    # column-pair visit, per applied rotation 4n (scaled rotations, the
    # default variant: one FMA per element and column) or 6n (plain
    # rotations), 2 per norm multiply-add
    rot_flops = 4.0 if args.jacobi_block in (0, 5, 6, 7) else 6.0   # scaled rotations: one FMA per element and column
    jac_flops = (2.0 * n * counts["pair_visits"] + rot_flops * n * counts["rotations"]
                 + 2.0 * counts["norm_madds"])          # over all timed launches
    jac_ms, jac_launches = stages["jacobi_f32"]          # HIP events around each launch
    ref_flops = B * 2 * 6.0 * n ** 3
    cand = {
        "jacobi_f32_lds_kernel": {"bound": "alu", "achieved": jac_flops / (jac_ms * 1e-3) / 1e12,
                       "peak": PEAK_FP32_PUBLISHED, "unit": "TFLOP/s"},
        "refine": {"bound": "mfma", "achieved": ref_flops / (avg["refine"] * 1e-3) / 1e12,
                   "peak": PEAK_FP64_MFMA, "unit": "TFLOP/s"},
    }
    # the dominant kernel is the LDS Jacobi (two launches per step: the cold
    # starts, then the warm starts); the refinement stage is six kernels per
    # step, each well below it (profiles/)
    dom = "jacobi_f32_lds_kernel"
    roof = dict(cand[dom])
    roof["frac"] = roof["achieved"] / roof["peak"]
    tr = measured_traffic(dom) if B == 4096 else None
    roof["traffic"] = tr[0] if tr else None
    roof["traffic_source"] = (f"stored rocprofv3 FETCH_SIZE/WRITE_SIZE summary of the same kernel sources "
                              f"({os.path.relpath(tr[1], ROOT)})" if tr else
                              "none: no counter summary of the current kernel sources")
    roof["peak_nonpacked"] = PEAK_FP32_VALU
    roof["frac_nonpacked"] = roof["achieved"] / PEAK_FP32_VALU
    roof["kernel"] = dom
    roof["flop_per_item"] = jac_flops / (B * args.steps)
    roof["avg_launch_ms"] = jac_ms / jac_launches
    roof["launches_per_step"] = jac_launches / args.steps
    ref_roof = dict(cand["refine"])
    ref_roof["frac"] = ref_roof["achieved"] / ref_roof["peak"]
    ref_roof["kernel"] = "refinement stage (gemm_y, gemm_sg, refine_reach, refine_chain, gemm_xm x 2 steps, finish)"

    # the paper's sequential operation count per channel (dense eigensolver
    # 8/3 n^3 + 2 n^3 - n^2, T at n_E = N energies 6 N n_E) at this rate
    paper_flop = 8.0 / 3.0 * n ** 3 + 2.0 * n ** 3 - n ** 2 + 6.0 * N_WP * N_WP
    paper_model = {"flop_per_item": paper_flop, "achieved": value * paper_flop / 1e12, "unit": "TFLOP/s",
                   "peak": PEAK_FP32_PUBLISHED, "frac": value * paper_flop / 1e12 / PEAK_FP32_PUBLISHED}

    cold = None
    if not args.no_cold:
        # the same batch with every item started cold (wpcd_config.jacobi_start = 1)
        del b, bufs
        torch.cuda.synchronize()
        cctx = wp.Context(0, jacobi_block=args.jacobi_block, jacobi_stop_f32=args.jacobi_stop, jacobi_start=1,
                          refine_gemm=args.refine_gemm, refine_steps=args.refine_steps,
                          refine_close_log10=args.refine_close, refine_rr_steps=args.refine_rr)
        cg = cctx.grid(k, configs.N_GAUSS)
        cb = cctx.batch([(cg, N_CH, 1, s) for s in range(B)])
        cbufs = cb.alloc()
        cb.run(u, cbufs, wp.MIXED, tlab, sigma)
        torch.cuda.synchronize()
        tc0 = time.perf_counter()
        for _ in range(args.steps):
            cb.run(u, cbufs, wp.MIXED, tlab, sigma)
        torch.cuda.synchronize()
        cwall = time.perf_counter() - tc0
        cst = cbufs["eig_status"].cpu().numpy()
        cold = {"value": B * args.steps / cwall, "unit": "channel-solves/s", "ms_per_step": cwall / args.steps * 1e3,
                "jacobi_sweeps_mean": float(cst[cst > 0].mean()) if (cst > 0).any() else None,
                "note": "same batch and steps, every item started cold (wpcd_config.jacobi_start = 1)"}
        log(f"cold starts: {cold['value']:.0f} channel-solves/s, {cold['ms_per_step']:.2f} ms/step")
        del cb, cbufs
        torch.cuda.synchronize()

    # plain FP64 path: one item per launch sequence, synchronised per item
    P = args.plain_items
    plain_lat = []
    pbs = []
    for s in range(P):
        pb = ctx.batch([(g, N_CH, 1, 0)])
        pu = sdev.pack_coupled_yukawa(pb.layout["u_elems"], pb.u_off, g.nodes, coeffs[s:s + 1], torch.float64,
                                      terms=terms)
        pbs.append((pb, pu, pb.alloc(), torch.empty(N_TLAB, dtype=torch.float64, device=dev)))
    pb, pu, pbuf, psig = pbs[0]
    pb.run(pu, pbuf, wp.F64, tlab, psig)          # warm-up
    torch.cuda.synchronize()
    for pb, _, _, _ in pbs:
        pb.jacobi_launches(clear=True)
    tp0 = time.perf_counter()
    for pb, pu, pbuf, psig in pbs:
        t1 = time.perf_counter()
        pb.run(pu, pbuf, wp.F64, tlab, psig)
        torch.cuda.synchronize()
        plain_lat.append((time.perf_counter() - t1) * 1e3)
    plain_wall = time.perf_counter() - tp0
    plain_lat = np.array(plain_lat)
    jl = [pb.jacobi_launches() for pb, _, _, _ in pbs]
    plain = {"value": P / plain_wall, "unit": "channel-solves/s", "items": P,
             "p50_ms": float(np.percentile(plain_lat, 50)), "p99_ms": float(np.percentile(plain_lat, 99)),
             "jacobi_launches_per_item": float(np.mean([c["launches"] for c in jl])),
             "jacobi_sweeps_enqueued_per_item": float(np.mean([c["sweeps"] for c in jl])),
             "jacobi_sweeps_per_item": float(np.mean([pbuf["eig_status"].cpu().numpy().max() for _, _, pbuf, _ in pbs]))}
    log(f"plain FP64: {plain['value']:.1f} channel-solves/s, p50 {plain['p50_ms']:.2f} ms")

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.cpu_seconds)
        log(f"cpu oracle: {cpu['value']:.1f} channel-solves/s on {cpu['cores']} cores")

    extras = None
    if not args.no_extras:
        # the other workloads, short: the J <= 6 sweep (256 samples x 20
        # channels, 3 steps) and the request loop (Poisson arrivals at
        # 2000/s, 8 s measured after 2 s)
        torch.cuda.synchronize()
        ea = argparse.Namespace(**vars(args))
        ea.samples, ea.steps, ea.warmup = 256, 3, 1
        sw = run_sweep(ea)
        ea.rate, ea.duration, ea.serve_warmup = 2000.0, 8.0, 2.0
        sv = run_serve(ea)
        extras = {
            "sweep": {"value": sw["value"], "unit": sw["unit"], "ms_per_step": sw["ms_per_step"],
                      "items_per_step": sw["config"]["items_per_step"], "jacobi_sweeps_mean": sw["jacobi_sweeps_mean"],
                      "stages_ms_per_step": sw["stages_ms_per_step"], "workload": sw["config"]["workload"]},
            "serve": {"latency_ms": sv["latency_ms"], "throughput": sv["throughput"], "requests": sv["steps"],
                      "batches": sv["server"]["batches"],
                      "device_jacobi_launches_per_batch": sv["server"]["jacobi_launches"] / max(1, sv["server"]["batches"]),
                      "device_jacobi_sweeps_per_batch": sv["server"]["jacobi_sweeps"] / max(1, sv["server"]["batches"]),
                      "workload": sv["config"]["workload"]},
        }

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "channel-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "coupled S-D Yukawa+tensor channel, N_WP=100 (200x200 H), 8 Gauss/bin, "
                               "T at all 100 bin energies, sigma_tot at 30 T_lab",
                   "items_per_step": B, "n_wp": N_WP, "n_ch": N_CH, "input_dtype": "f32"},
        "latency_ms": {"step_p50": float(np.percentile(step_ms, 50)), "step_p99": float(np.percentile(step_ms, 99))},
        "plain_f64": plain,
        "speedup_vs_plain": value / plain["value"],
        "jacobi_sweeps_mean": float(sweeps.mean()) if sweeps.size else None,
        "jacobi_rotated_fraction": counts["rotations"] / max(1, counts["pair_visits"]),
        "stages_ms_per_step": {s: ms / args.steps for s, (ms, cnt) in stages.items() if cnt},
        "cold_start": cold,
        "roofline": roof,
        "paper_model_rate": paper_model,
        "roofline_refine_stage": ref_roof,
        "cpu_baseline": cpu,
        "other_workloads": extras,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
