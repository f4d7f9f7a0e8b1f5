"""The request loop (wpcd_server_create / wpcd_submit / wpcd_poll) on the GPU.

A reference request is solved alone, then again in the middle of a mix of
other requests submitted in waves while earlier ones are still on the device
(continuous batching).  Its channels span every eigensolver size class (n from
50 to 400, the device-memory Jacobi included), and so do the other requests'.
The kernels a batch takes depend on its size mix (the device-memory Jacobi's
block width on the largest n of its class, the refinement's product kernels on
the smallest and largest n of the batch), which changes the rounding order but
not the solved problem: the two runs must agree within 1e-7 deg and 1e-6 mb,
far below the oracle bars, and both must match the FP64 oracle within 0.01 deg
and 0.01 mb.
"""
import time

import numpy as np
import pytest

import paper_2106_00454_amd as wp
from oracle import observables as oo
from oracle import wpcd as ow
from synth import sweep
from tests.gpu_util import DELTA_TOL, SIGMA_TOL, dmod180

pytestmark = pytest.mark.gpu

CHANNELS = (0, 7, 14, 16)          # 1S0, 3P0, 3S1-3D1, 3D3-3G3
NWP = (50, 100, 150, 200)


@pytest.fixture(scope="module")
def setup():
    # (CHANNELS x NWP bases; the coupled N_WP = 200 terms alone are 1.3 GB)
    ctx = wp.Context(0)
    cache = sweep.TermCache()
    grids = {N: ctx.grid(sweep.grid_bounds(N), sweep.N_GAUSS) for N in NWP}
    bases = {}
    for N in NWP:
        for c in CHANNELS:
            bases[(c, N)] = ctx.basis(grids[N], sweep.CHANNELS[c][1], cache.terms(("lib", N), grids[N].nodes, c))
    srv = wp.Server(ctx, hbm_budget_bytes=1 << 30, max_inflight=3, max_batch_items=64)
    yield ctx, bases, srv
    srv.close()


def request(bases, sample, spec):
    """spec: list of (channel, N) -> submit arguments."""
    return [(bases[(c, N)], sweep.CHANNELS[c][2], sweep.coefficients(sample, c)) for c, N in spec]


def wait(srv, tickets, timeout=60.0):
    t0 = time.time()
    pending = list(tickets)
    while pending:
        pending = [t for t in pending if not srv.poll(t)]
        if time.time() - t0 > timeout:
            raise TimeoutError(f"{len(pending)} requests still pending")
        time.sleep(1e-4)


REF_SPEC = [(0, 50), (14, 100), (16, 50), (7, 150), (16, 200)]


@pytest.mark.timeout(300)
def test_request_alone_and_in_the_mix(setup):
    ctx, bases, srv = setup
    ref = srv.submit(request(bases, 0, REF_SPEC), sweep.TLAB, want_phases=True)
    wait(srv, [ref])
    assert ref.code == wp.WPCD_OK and (ref.status > 0).all()
    b0 = srv.stats()["batches"]
    rng = np.random.default_rng(11)
    mix_tickets, again = [], None
    for wave in range(4):
        for r in range(8):
            k = int(rng.integers(1, len(CHANNELS) + 1))
            spec = [(int(c), int(rng.choice(NWP))) for c in rng.choice(CHANNELS, size=k, replace=False)]
            mix_tickets.append(srv.submit(request(bases, 100 + 8 * wave + r, spec), sweep.TLAB[:int(rng.integers(1, 31))]))
            if wave == 2 and r == 3:
                again = srv.submit(request(bases, 0, REF_SPEC), sweep.TLAB, want_phases=True)
        time.sleep(0.002)          # the next wave arrives while this one runs
    wait(srv, mix_tickets + [again])
    st = srv.stats()
    print("server stats", st, flush=True)
    assert st["batches"] - b0 >= 2 and st["completed"] == st["submitted"]
    assert all(t.code == wp.WPCD_OK for t in mix_tickets) and again.code == wp.WPCD_OK
    ds = np.abs(again.sigma - ref.sigma).max()
    dd = np.abs(again.delta - ref.delta).max()
    dm = np.abs(again.mix - ref.mix).max()
    print(f"alone vs mix: dsigma={ds:.3e} ddelta={dd:.3e} dmix={dm:.3e}", flush=True)
    assert ds <= 1e-6 and dd <= 1e-7 and dm <= 1e-7
    # the reference request against the oracle
    cache = sweep.TermCache()
    chans, off, moff = [], 0, 0
    for c, N in REF_SPEC:
        _, K, J, _, _ = sweep.CHANNELS[c]
        k = sweep.grid_bounds(N)
        xo, _ = ow.gauss_nodes(k, sweep.N_GAUSS)
        u = sum(ci * t for ci, t in zip(sweep.coefficients(0, c), cache.terms(("or", N), xo, c)))
        r = ow.solve_channel(k, sweep.N_GAUSS, u, K)
        got = ref.delta[off:off + N * K].reshape(N, K)
        d = dmod180(got, r["delta"]).max()
        m = np.abs(ref.mix[moff:moff + N] - r["mix"]).max() if K == 2 else 0.0
        print(f"serve {sweep.CHANNELS[c][0]} N={N}: ddelta={d:.3e} dmix={m:.3e}", flush=True)
        assert d <= DELTA_TOL and m <= DELTA_TOL
        _, kbar, _ = ow.bins(k)
        chans.append((J, r["delta"], r["mix"], kbar, k[-1]))
        off += N * K
        moff += N
    dsig = np.abs(ref.sigma - oo.sigma_tot(chans, None, sweep.TLAB, None)).max()
    print(f"serve sigma vs oracle: {dsig:.3e} mb", flush=True)
    assert dsig <= SIGMA_TOL


def test_submit_errors(setup):
    ctx, bases, srv = setup
    with pytest.raises(wp.WPCDError) as e:
        srv.submit([], sweep.TLAB)
    assert e.value.code == wp.WPCD_ERR_INVALID
    with pytest.raises(wp.WPCDError) as e:
        srv.submit(request(bases, 0, [(0, 50)]), np.linspace(1, 300, 1025))
    assert e.value.code == wp.WPCD_ERR_INVALID
    small = wp.Server(ctx, hbm_budget_bytes=1 << 20)
    with pytest.raises(wp.WPCDError) as e:
        small.submit(request(bases, 0, [(14, 100)]), sweep.TLAB)     # n = 200 needs ~3 MB
    assert e.value.code == wp.WPCD_ERR_UNSUPPORTED
    small.close()
    t = srv.submit(request(bases, 1, [(7, 50)]), sweep.TLAB)
    wait(srv, [t])
    with pytest.raises(wp.WPCDError) as e:
        srv.poll(wp.Ticket(t.id, None, None, None, None))              # retired
    assert e.value.code == wp.WPCD_ERR_INVALID
