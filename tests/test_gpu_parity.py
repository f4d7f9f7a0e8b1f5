"""GPU path vs the FP64 oracle, element by element, through the C ABI.

Bars: phase shifts and mixing angles within 0.01 deg and
total cross sections within 0.01 mb of the oracle; intermediate quantities are
checked with bounds derived from the arithmetic (stated per check).
"""
import numpy as np
import pytest
import torch

import paper_2106_00454_amd as wp
from oracle import observables as oo
from oracle import wpcd as ow
from synth import configs, grids, potentials
from synth import device as sdev
from tests.gpu_util import DELTA_TOL, SIGMA_TOL, TLAB, check_item, dmod180, item_view, run_items

pytestmark = pytest.mark.gpu

@pytest.fixture(scope="module")
def ctx():
    return wp.Context(0)


def oracle_item(k, u_oracle_nodes, K):
    return ow.solve_channel(k, configs.N_GAUSS, u_oracle_nodes, K)


# ------------------------------------------------------------------ grid
def test_grid_nodes_match_oracle(ctx):
    k = grids.tan2_bounded(37)
    g = ctx.grid(k, 8)
    x, w = ow.gauss_nodes(k, 8)
    assert np.abs(g.nodes - x).max() <= 1e-15 * k[-1]
    assert np.abs(g.weights - w).max() <= 1e-15 * k[-1]


# ------------------------------------------------------------ Yamaguchi S-wave
@pytest.mark.parametrize("mode", [wp.MIXED, wp.F64])
def test_yamaguchi_batch_matches_oracle(ctx, mode):
    k = configs.grid("yamaguchi_s")
    g = ctx.grid(k, configs.N_GAUSS)
    xo, _ = ow.gauss_nodes(k, configs.N_GAUSS)
    lams = [configs.yamaguchi_lambda(s) for s in range(16)]
    mats = [potentials.yamaguchi(g.nodes, g.nodes, lam, configs.YAMAGUCHI_BETA) for lam in lams]
    items = [(g, 1, 0, s) for s in range(16)]
    b, host = run_items(ctx, items, mats, mode)
    _, kbar, _ = ow.bins(k)
    for s, lam in enumerate(lams):
        ref = oracle_item(k, potentials.yamaguchi(xo, xo, lam, configs.YAMAGUCHI_BETA), 1)
        it = item_view(b, host, s)
        assert np.abs(it["v"] - ref["v"]).max() <= 1e-12 * np.abs(ref["v"]).max()
        sig_ref = oo.sigma_tot([(0, ref["delta"], None)], kbar, TLAB, k[-1])
        check_item(f"yamaguchi mode={mode} s={s}", it, ref, k, mode, 0, sig_ref, host["sigma"][s])


# -------------------------------------------------------- coupled Yukawa N=100
@pytest.fixture(scope="module")
def coupled_setup(ctx):
    k = configs.grid("coupled_yukawa")
    g = ctx.grid(k, configs.N_GAUSS)
    xo, _ = ow.gauss_nodes(k, configs.N_GAUSS)
    return k, g, configs.coupled_yukawa_terms(g.nodes), configs.coupled_yukawa_terms(xo)


@pytest.mark.parametrize("mode,dtype", [(wp.MIXED, torch.float32), (wp.F64, torch.float64)])
def test_coupled_batch_matches_oracle(ctx, coupled_setup, mode, dtype):
    k, g, t_lib, t_or = coupled_setup
    ns = 6
    coeffs = np.array([configs.yukawa_coefficients(s) for s in range(ns)])
    mats = [sum(c * t for c, t in zip(cs, t_lib)) for cs in coeffs]
    if dtype == torch.float32:
        mats = [m.astype(np.float32).astype(np.float64) for m in mats]
    items = [(g, 2, 1, s) for s in range(ns)]
    b = ctx.batch(items)
    u = sdev.pack_host_matrices(b.layout["u_elems"], b.u_off, mats, dtype)
    b, host = run_items(ctx, items, u, mode)
    _, kbar, _ = ow.bins(k)
    for s in range(ns):
        uo = sum(c * t for c, t in zip(coeffs[s], t_or))
        if dtype == torch.float32:
            uo = uo.astype(np.float32).astype(np.float64)
        ref = oracle_item(k, uo, 2)
        it = item_view(b, host, s)
        vt = 1e-12 if dtype == torch.float64 else 2e-6
        assert np.abs(it["v"] - ref["v"]).max() <= vt * np.abs(ref["v"]).max()
        sig_ref = oo.sigma_tot([(1, ref["delta"], ref["mix"])], kbar, TLAB, k[-1])
        check_item(f"coupled mode={mode} s={s}", it, ref, k, mode, 1, sig_ref, host["sigma"][s])


# ------------------------------------------------ ragged mixed batch, odd n
@pytest.mark.parametrize("mode,rr", [(wp.MIXED, 0), (wp.MIXED, 1), (wp.F64, 0)])
def test_ragged_mixed_batch(ctx, mode, rr):
    # n = 37, 240, 40, 64, 233, 150, 100, 128, 200: every eigensolver size class
    # (<= 64, <= 128, <= 200 in LDS, > 200 in device memory) with its boundary
    # sizes, interleaved so each class launch works from a scattered item list
    specs = [("yam", 37, 1), ("cyuk", 120, 2), ("cyuk", 20, 2), ("yuk0", 64, 1), ("yam", 233, 1),
             ("cyuk", 75, 2), ("yam", 100, 1), ("cyuk", 64, 2), ("cyuk", 100, 2)]
    items, mats, refs = [], [], []
    rng = np.random.default_rng(7)
    for sid, (kind, N, K) in enumerate(specs):
        k = grids.tan2_bounded(N)
        g = ctx.grid(k, 8)
        xo, _ = ow.gauss_nodes(k, 8)
        if kind == "yam":
            lam = rng.uniform(0.5, 2.0)
            f = lambda x: potentials.yamaguchi(x, x, lam, 1.4)
            J = 0
        elif kind == "yuk0":
            f = lambda x: sum(C * potentials.yukawa_central(0, x, x, 1.0, mu)
                              for C, mu in zip(configs.YUKAWA_MEANS, configs.YUKAWA_MU))
            J = 0
        else:
            c = configs.yukawa_coefficients(100 + sid)
            f = lambda x, c=c: sum(ci * ti for ci, ti in zip(c, configs.coupled_yukawa_terms(x)))
            J = 1
        items.append((g, K, J, sid))
        mats.append(f(g.nodes))
        refs.append((k, ow.solve_channel(k, 8, f(xo), K), J))
    # rr = 1: Rayleigh-Ritz on clusters in the last refinement step only
    # (wpcd_config.refine_rr_steps), on a context of its own
    rctx = ctx if rr == 0 else wp.Context(0, refine_rr_steps=rr)
    if rctx is not ctx:
        items = [(rctx.grid(g.k_bounds, 8), K, J, sid) for (g, K, J, sid) in items]
    b, host = run_items(rctx, items, mats, mode)
    for i, (k, ref, J) in enumerate(refs):
        _, kbar, _ = ow.bins(k)
        it = item_view(b, host, i)
        K = it["delta"].shape[1]
        sig_ref = oo.sigma_tot([(J, ref["delta"], ref["mix"])], kbar, TLAB, k[-1])
        check_item(f"ragged mode={mode} rr={rr} item={i} n={it['v'].shape[0]}", it, ref, k, mode, J, sig_ref,
                   host["sigma"][i])


# ------------------------------------------------------------- degenerate
@pytest.mark.parametrize("mode", [wp.MIXED, wp.F64])
def test_zero_potential_gives_exact_zero(ctx, mode):
    k = grids.tan2_bounded(24)
    g = ctx.grid(k, 8)
    m = 24 * 8
    items = [(g, 1, 0, 0), (g, 2, 1, 1)]
    b, host = run_items(ctx, items, [np.zeros((m, m)), np.zeros((2 * m, 2 * m))], mode)
    for i in range(2):
        it = item_view(b, host, i)
        assert it["t_status"] == 0 and it["eig_status"] > 0
        assert np.all(it["t"] == 0) and np.all(it["delta"] == 0) and np.all(it["mix"] == 0)
    assert np.all(host["sigma"] == 0)


def test_argument_errors_are_reported_before_launch(ctx):
    k = grids.tan2_bounded(10)
    g = ctx.grid(k, 8)
    with pytest.raises(wp.WPCDError) as e:
        ctx.batch([(g, 3, 0, 0)])
    assert e.value.code == wp.WPCD_ERR_INVALID
    with pytest.raises(wp.WPCDError) as e:
        ctx.grid(np.array([0.0, 1.0, 1.0, 2.0]), 8)
    assert e.value.code == wp.WPCD_ERR_INVALID
    big = ctx.grid(grids.tan2_bounded(601), 2)
    with pytest.raises(wp.WPCDError) as e:
        ctx.batch([(big, 2, 1, 0)])          # n = 1202 > 1200
    assert e.value.code == wp.WPCD_ERR_UNSUPPORTED
    b = ctx.batch([(g, 1, 0, 0)])
    bufs = b.alloc()
    with pytest.raises(wp.WPCDError) as e:
        b.eigh(bufs["v64"], 7, bufs["eval"], bufs["evec"], bufs["eig_status"])
    assert e.value.code == wp.WPCD_ERR_INVALID


# ------------------------------------------------- LDS Jacobi variants
@pytest.mark.parametrize("variant", [1, 2, 3, 4, 5, 6, 7])
def test_lds_jacobi_variants_match_oracle(variant):
    # every variant of the in-LDS FP32 Jacobi (wpcd_config.jacobi_block), on
    # one item of each LDS size class (n = 37, 40, 128, 200), mixed precision
    vctx = wp.Context(0, jacobi_block=variant)
    specs = [("yam", 37, 1), ("cyuk", 20, 2), ("cyuk", 64, 2), ("cyuk", 100, 2)]
    items, mats, refs = [], [], []
    for sid, (kind, N, K) in enumerate(specs):
        k = configs.grid("coupled_yukawa") if N == 100 else grids.tan2_bounded(N)
        g = vctx.grid(k, 8)
        xo, _ = ow.gauss_nodes(k, 8)
        if kind == "yam":
            f = lambda x: potentials.yamaguchi(x, x, 1.7, 1.4)
            J = 0
        else:
            c = configs.yukawa_coefficients(200 + sid)
            f = lambda x, c=c: sum(ci * ti for ci, ti in zip(c, configs.coupled_yukawa_terms(x)))
            J = 1
        items.append((g, K, J, sid))
        mats.append(f(g.nodes))
        refs.append((k, ow.solve_channel(k, 8, f(xo), K), J))
    b, host = run_items(vctx, items, mats, wp.MIXED)
    for i, (k, ref, J) in enumerate(refs):
        _, kbar, _ = ow.bins(k)
        it = item_view(b, host, i)
        sig_ref = oo.sigma_tot([(J, ref["delta"], ref["mix"])], kbar, TLAB, k[-1])
        check_item(f"jacobi variant={variant} item={i} n={it['v'].shape[0]}", it, ref, k, wp.MIXED, J, sig_ref,
                   host["sigma"][i])


# ------------------------------------------- warm-started LDS Jacobi
def test_warm_started_jacobi_matches_oracle_and_cold_start():
    # more items of one channel than compute units: the first 256 (one per
    # CU) start cold, the rest warm from the first item's eigenvectors
    # (wpcd_config.jacobi_start = 0, the default); the same batch solved with
    # cold starts only (jacobi_start = 1) must agree with it and the oracle
    k = configs.grid("yamaguchi_s")
    n_items = 300
    lams = [configs.yamaguchi_lambda(s) for s in range(n_items)]
    res = {}
    for start in (0, 1):
        c = wp.Context(0, jacobi_start=start)
        g = c.grid(k, configs.N_GAUSS)
        mats = [potentials.yamaguchi(g.nodes, g.nodes, lam, configs.YAMAGUCHI_BETA) for lam in lams]
        b, host = run_items(c, [(g, 1, 0, s) for s in range(n_items)], mats, wp.MIXED)
        assert (host["eig_status"] > 0).all() and (host["t_status"] == 0).all()
        res[start] = (b, host)
    xo, _ = ow.gauss_nodes(k, configs.N_GAUSS)
    _, kbar, _ = ow.bins(k)
    bw, hw = res[0]
    bc, hc = res[1]
    assert dmod180(hw["delta"], hc["delta"]).max() <= 1e-6
    assert np.abs(hw["sigma"] - hc["sigma"]).max() <= 1e-6
    for s in (0, 1, 255, 256, 257, 280, 299):
        ref = oracle_item(k, potentials.yamaguchi(xo, xo, lams[s], configs.YAMAGUCHI_BETA), 1)
        it = item_view(bw, hw, s)
        sig_ref = oo.sigma_tot([(0, ref["delta"], None)], kbar, TLAB, k[-1])
        check_item(f"warm start s={s}", it, ref, k, wp.MIXED, 0, sig_ref, hw["sigma"][s])


# ------------------------------------ whole-item refinement products
def test_whole_item_products_match_tiles_and_oracle():
    # batches whose items all have 193..208 rows take the whole-item products
    # of the refinement (one work-group per item, persistent over the items,
    # wpcd_config.refine_gemm = 0); ragged and odd n, more items than compute
    # units so work-groups move on to items of another size; the same batch
    # with 64 x 64 tiles (refine_gemm = 1) must agree, and both the oracle
    specs = [("yam", 193, 1), ("cyuk", 100, 2), ("yam", 203, 1), ("cyuk", 104, 2), ("yam", 197, 1),
             ("cyuk", 97, 2)]
    n_items = 264
    res = {}
    for mode_g in (0, 1):
        c = wp.Context(0, refine_gemm=mode_g)
        gs = {}
        items, mats = [], []
        for s in range(n_items):
            kind, N, K = specs[s % len(specs)]
            if N not in gs:
                gs[N] = c.grid(configs.grid("coupled_yukawa") if N == 100 else grids.tan2_bounded(N), 8)
            g = gs[N]
            if kind == "yam":
                mats.append(potentials.yamaguchi(g.nodes, g.nodes, configs.yamaguchi_lambda(s), 1.4))
                items.append((g, 1, 0, s))
            else:
                cf = configs.yukawa_coefficients(300 + s)
                mats.append(sum(ci * ti for ci, ti in zip(cf, configs.coupled_yukawa_terms(g.nodes))))
                items.append((g, 2, 1, s))
        b, host = run_items(c, items, mats, wp.MIXED)
        assert (host["eig_status"] > 0).all() and (host["t_status"] == 0).all()
        res[mode_g] = (b, host)
    (bw, hw), (bt, ht) = res[0], res[1]
    assert dmod180(hw["delta"], ht["delta"]).max() <= 1e-6
    assert np.abs(hw["mix"] - ht["mix"]).max() <= 1e-6
    assert np.abs(hw["sigma"] - ht["sigma"]).max() <= 1e-6
    for s in list(range(len(specs))) + [256, 257, 263]:
        kind, N, K = specs[s % len(specs)]
        k = configs.grid("coupled_yukawa") if N == 100 else grids.tan2_bounded(N)
        xo, _ = ow.gauss_nodes(k, 8)
        if kind == "yam":
            uo, J = potentials.yamaguchi(xo, xo, configs.yamaguchi_lambda(s), 1.4), 0
        else:
            cf = configs.yukawa_coefficients(300 + s)
            uo, J = sum(ci * ti for ci, ti in zip(cf, configs.coupled_yukawa_terms(xo))), 1
        ref = oracle_item(k, uo, K)
        _, kbar, _ = ow.bins(k)
        sig_ref = oo.sigma_tot([(J, ref["delta"], ref["mix"])], kbar, TLAB, k[-1])
        for tag, (b, host) in (("whole", (bw, hw)), ("tiles", (bt, ht))):
            it = item_view(b, host, s)
            iw = item_view(bw, hw, s)
            assert np.abs(it["evals"] - iw["evals"]).max() <= 1e-10 * np.abs(iw["evals"]).max()
            check_item(f"refine products={tag} s={s} n={it['v'].shape[0]}", it, ref, k, wp.MIXED, J, sig_ref,
                       host["sigma"][s])


# ------------------------------------- warm start from the nearest cold item
def test_warm_start_picks_the_nearest_cold_item():
    # one cold item per compute unit (lambda in [0.5, 2]), then warm items
    # whose potentials equal those of cold items 7 and 150 exactly: the
    # reference choice (nearest V on a strided sample) must pick those twins,
    # whose eigenvectors already diagonalise the warm items, so the Jacobi
    # stops after its first sweep; warm items far from every cold item
    # (lambda 0.05 ... 3.3) need more; all match the oracle
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    k = configs.grid("yamaguchi_s")
    c = wp.Context(0)
    g = c.grid(k, configs.N_GAUSS)
    lams = [configs.yamaguchi_lambda(s) for s in range(n_cu)]
    twins = {n_cu: 7, n_cu + 1: 150}
    lams += [lams[7], lams[150]] + [0.05, 0.1, 0.2, 3.0, 3.3]
    mats = [potentials.yamaguchi(g.nodes, g.nodes, lam, configs.YAMAGUCHI_BETA) for lam in lams]
    b, host = run_items(c, [(g, 1, 0, s) for s in range(len(lams))], mats, wp.MIXED)
    sw = host["eig_status"]
    print("sweeps: cold mean", sw[:n_cu].mean(), "twins", [int(sw[i]) for i in twins], "others",
          [int(x) for x in sw[n_cu + 2:]], flush=True)
    assert (sw > 0).all() and (host["t_status"] == 0).all()
    for i, j in twins.items():
        assert sw[i] == 1, (i, j, sw[i])
        assert np.abs(item_view(b, host, i)["evals"] - item_view(b, host, j)["evals"]).max() <= 1e-12 * np.abs(
            item_view(b, host, j)["evals"]).max()
    assert sw[n_cu + 2:].min() >= 2
    xo, _ = ow.gauss_nodes(k, configs.N_GAUSS)
    _, kbar, _ = ow.bins(k)
    for s in list(twins) + [len(lams) - 1]:
        ref = oracle_item(k, potentials.yamaguchi(xo, xo, lams[s], configs.YAMAGUCHI_BETA), 1)
        sig_ref = oo.sigma_tot([(0, ref["delta"], None)], kbar, TLAB, k[-1])
        check_item(f"nearest-reference warm start s={s}", item_view(b, host, s), ref, k, wp.MIXED, 0, sig_ref,
                   host["sigma"][s])


@pytest.mark.timeout(300)
@pytest.mark.parametrize("variant", [0, 5, 6, 7])
def test_lds_jacobi_variants_on_a_batch(variant):
    # the LDS Jacobi variants on batches of many items per launch: 24
    # Yamaguchi n = 50 items (13 blocks of 4: an odd block count) and 12
    # coupled n = 200 items, all cold; every item against the oracle
    vctx = wp.Context(0, jacobi_block=variant)
    ky, kc = configs.grid("yamaguchi_s"), configs.grid("coupled_yukawa")
    gy, gc = vctx.grid(ky, 8), vctx.grid(kc, 8)
    xy, _ = ow.gauss_nodes(ky, 8)
    xc, _ = ow.gauss_nodes(kc, 8)
    items, mats, refs = [], [], []
    for s in range(24):
        lam = configs.yamaguchi_lambda(s)
        items.append((gy, 1, 0, s))
        mats.append(potentials.yamaguchi(gy.nodes, gy.nodes, lam, configs.YAMAGUCHI_BETA))
        refs.append((ky, 0, lambda x, lam=lam: potentials.yamaguchi(x, x, lam, configs.YAMAGUCHI_BETA), xy, 1))
    for s in range(12):
        c = configs.yukawa_coefficients(300 + s)
        f = lambda x, c=c: sum(ci * t for ci, t in zip(c, configs.coupled_yukawa_terms(x)))
        items.append((gc, 2, 1, 24 + s))
        mats.append(f(gc.nodes))
        refs.append((kc, 1, f, xc, 2))
    b, host = run_items(vctx, items, mats, wp.MIXED)
    worst = {}
    for i, (k, J, f, xo, K) in enumerate(refs):
        ref = ow.solve_channel(k, 8, f(xo), K)
        it = item_view(b, host, i)
        dd = dmod180(it["delta"], ref["delta"]).max()
        worst[K] = max(worst.get(K, 0.0), dd)
        if dd > DELTA_TOL or i in (0, 23, 24, 35):
            _, kbar, _ = ow.bins(k)
            sig_ref = oo.sigma_tot([(J, ref["delta"], ref["mix"])], kbar, TLAB, k[-1])
            check_item(f"variant={variant} batch item={i} n={K * (k.size - 1)}", it, ref, k, wp.MIXED, J, sig_ref,
                       host["sigma"][i])
    print(f"variant={variant}: worst ddelta per channel count {worst}", flush=True)
