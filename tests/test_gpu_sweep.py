"""The J <= 6 batched sweep through the C ABI against the FP64 oracle.

Every item of two parameter samples (20 channels each, N_WP drawn from
{50, 100, 150}, so n = 50 ... 300 including the device-memory eigensolver
class) is projected from registered affine bases (wpcd_basis_register +
wpcd_project_affine); the oracle projects the same affine potential from its
fine-mesh form.  Bars: V to 1e-12 relative (linearity of the projection), phase
shifts and mixing angles within 0.01 deg, per-sample total cross sections over
all 20 channels within 0.01 mb.
"""
import numpy as np
import pytest

import paper_2106_00454_amd as wp
from oracle import observables as oo
from oracle import wpcd as ow
from synth import sweep
from tests.gpu_util import SIGMA_TOL, check_item, item_view, run_items

pytestmark = pytest.mark.gpu

N_SAMPLES = 2


@pytest.fixture(scope="module")
def setup():
    ctx = wp.Context(0)
    items = sweep.items(N_SAMPLES)
    grids = {N: ctx.grid(sweep.grid_bounds(N), sweep.N_GAUSS) for N in sweep.N_WP_CHOICES}
    lib_terms, or_terms = sweep.TermCache(), sweep.TermCache()
    bases = {}
    specs, coefs, refs = [], [], []
    for s, c, N in items:
        _, n_ch, J, _, _ = sweep.CHANNELS[c]
        g = grids[N]
        if (c, N) not in bases:
            bases[(c, N)] = ctx.basis(g, n_ch, lib_terms.terms(("lib", N), g.nodes, c))
        specs.append((g, n_ch, J, s, bases[(c, N)]))
        coefs.append(sweep.coefficients(s, c))
    for s, c, N in items:
        k = sweep.grid_bounds(N)
        xo, _ = ow.gauss_nodes(k, sweep.N_GAUSS)
        u = sum(ci * t for ci, t in zip(sweep.coefficients(s, c), or_terms.terms(("or", N), xo, c)))
        refs.append((k, ow.solve_channel(k, sweep.N_GAUSS, u, sweep.CHANNELS[c][1])))
    return ctx, items, specs, coefs, refs


@pytest.mark.parametrize("mode", [wp.MIXED, wp.F64])
def test_sweep_matches_oracle(setup, mode):
    ctx, items, specs, coefs, refs = setup
    b, host = run_items(ctx, specs, None, mode, tlab=sweep.TLAB, coef=coefs)
    assert b.layout["u_elems"] == 0 and b.layout["max_n"] == max(sp[1] * sp[0].n_wp for sp in specs)
    per_sample = {}
    for i, ((s, c, N), (k, ref)) in enumerate(zip(items, refs)):
        it = item_view(b, host, i)
        J = sweep.CHANNELS[c][2]
        assert np.abs(it["v"] - ref["v"]).max() <= 1e-12 * np.abs(ref["v"]).max()
        check_item(f"sweep mode={mode} sample={s} {sweep.CHANNELS[c][0]} N={N}", it, ref, k, mode, J)
        _, kbar, _ = ow.bins(k)
        per_sample.setdefault(s, []).append((J, ref["delta"], ref["mix"], kbar, k[-1]))
    for s, chans in per_sample.items():
        want = oo.sigma_tot(chans, None, sweep.TLAB, None)
        ds = np.abs(host["sigma"][s] - want).max()
        print(f"sweep mode={mode} sample={s}: dsigma={ds:.3e} mb (sigma at 1 MeV {want[0]:.1f} mb)", flush=True)
        assert ds <= SIGMA_TOL


def test_basis_errors(setup):
    ctx = setup[0]
    g = ctx.grid(sweep.grid_bounds(50), sweep.N_GAUSS)
    m = 50 * sweep.N_GAUSS
    bs = ctx.basis(g, 1, [np.eye(m)])
    g2 = ctx.grid(sweep.grid_bounds(60), sweep.N_GAUSS)
    with pytest.raises(wp.WPCDError) as e:
        ctx.batch([(g2, 1, 0, 0, bs)])           # basis of another grid
    assert e.value.code == wp.WPCD_ERR_INVALID
    with pytest.raises(wp.WPCDError) as e:
        ctx.batch([(g, 2, 1, 0, bs)])            # basis of another n_ch
    assert e.value.code == wp.WPCD_ERR_INVALID
