"""The Eq 25 stability limiter (Section 4) on the GPU: every step also capped
at 2 / ||A||_inf, A = d(dY/dt)/dY at fixed T and rho.  Checked against the
FP64 oracle with the same cap, on a case with a closed-form step (a stiff
A <=> B equilibrium) and on the 6-, 19- and 53-species mechanisms."""

import math

import numpy as np
import pytest

import oracle
from paper_1905_09395_amd import stev, synth
from tests import tiny_mechs as tm
from tests.gpu_common import judge, oracle_ensemble, run_gpu, say

pytestmark = pytest.mark.gpu
DT = 1e-4
P1 = 101325.0


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a HIP device"
    c = stev.Context(0)
    yield c
    c.close()


def test_stiff_equilibrium_step_is_the_cap(ctx):
    """A <=> B near equilibrium: with the cap every step is 2/(kf + kr)."""
    kf, da7 = 2.0e4, 0.3
    mech = tm.iso_ab(kf, 0.0, da7)
    gm = ctx.mechanism(mech)
    om = oracle.OracleMech(mech)
    K = math.exp(da7)
    ya = 1.0 / (K + 1.0)
    T = np.full(8, 1000.0)
    P = np.full(8, P1)
    Y = np.tile([ya + 1e-6, 1.0 - ya - 1e-6], (8, 1))
    Y[:, 0] += np.arange(8) * 1e-7
    Y[:, 1] -= np.arange(8) * 1e-7
    kw = dict(alpha=0.0, ystep_max=1.0, delta_max=1e-2, dft_window=0)
    o = oracle.integrate(om, T, P, Y, 1e-2, stab_limit=1, **kw)
    for G in (1, 64):
        g = run_gpu(ctx, gm, T, P, Y, 1e-2, stev.F64, stab_limit=1, lanes_per_cell=G, **kw)
        assert np.array_equal(g["iters"], o["iters"])
        np.testing.assert_allclose(g["Y"], o["Y"], rtol=1e-9, atol=1e-15)
    free = run_gpu(ctx, gm, T, P, Y, 1e-2, stev.F64, **kw)
    assert np.all(free["iters"] < o["iters"])        # the cap adds steps
    gm.close()


# The cap multiplies the step count of igniting cells by 10-100 (rate laws
# of order below one keep a large Jacobian as a species depletes), so these
# comparisons stop every cell after CAP iterations on both sides: cells that
# reach it end with status 2, and their states at that iteration are compared.
CAP = 1500


@pytest.mark.parametrize("key", [6, 19, 53])
def test_stab_limit_matches_oracle(ctx, key):
    m = {6: synth.make_mech6, 19: synth.make_mech19, 53: synth.make_mech53}[key]()
    gm = ctx.mechanism(m)
    om = oracle.OracleMech(m)
    n = {6: 256, 19: 96, 53: 24}[key]
    T, P, Y = (synth.make_cells_mech6(n, seed=61) if key == 6
               else synth.make_cells_split(n, key, 61))
    precs = (stev.F64, stev.F32)
    if key == 53:
        # FP64 with the limiter needs 166 KB of LDS per workgroup (160 KB on a CU)
        with pytest.raises(stev.StevError) as e:
            run_gpu(ctx, gm, T[:1], P[:1], Y[:1], DT, stev.F64, stab_limit=1)
        assert e.value.code == stev.STEV_EINVAL
        precs = (stev.F32,)
    for prec in precs:
        say(f"stab mech{key} prec={prec}")
        o = oracle_ensemble(om, T, P, Y, DT, prec, stab_limit=1, max_iters=CAP)
        g = run_gpu(ctx, gm, T, P, Y, DT, prec, stab_limit=1, max_iters=CAP, allow_failed=True)
        judge(g, o, prec, f"stab mech{key}/{prec}")
        if prec == precs[0]:
            plain = run_gpu(ctx, gm, T, P, Y, DT, prec, max_iters=CAP, allow_failed=True)
            changed = int(np.sum(plain["iters"] != g["iters"]))
            say(f"  cells whose step sequence the cap changed: {changed} of {n}; "
                f"iterations {plain['iters'].sum()} -> {g['iters'].sum()} "
                f"({int(np.sum(g['status'] == 2))} cells stopped at {CAP})")
    gm.close()


def test_stab_results_independent_of_launch_shape(ctx):
    """With the limiter, too, a cell's result does not depend on the launch
    shape or on its position in the field (for a given lanes-per-cell; other
    lane counts sum over species in another association)."""
    m = synth.make_mech19()
    gm = ctx.mechanism(m)
    T, P, Y = synth.make_cells_mech19(300, seed=62)
    kw = dict(stab_limit=1, max_iters=CAP, allow_failed=True)
    for G in (16, 64):
        ref = run_gpu(ctx, gm, T, P, Y, DT, stev.F64, lanes_per_cell=G, **kw)
        g = run_gpu(ctx, gm, T, P, Y, DT, stev.F64, lanes_per_cell=G, waves_per_wg=1,
                    grid_wgs=5, compact_every=3, **kw)
        assert np.array_equal(g["T"], ref["T"]) and np.array_equal(g["Y"], ref["Y"]), G
        T2, P2, Y2 = (np.concatenate([T[100:], T]), np.concatenate([P[100:], P]),
                      np.concatenate([Y[100:], Y]))
        g2 = run_gpu(ctx, gm, T2, P2, Y2, DT, stev.F64, lanes_per_cell=G, **kw)
        assert np.array_equal(g2["T"][200:], ref["T"]) and np.array_equal(g2["Y"][200:], ref["Y"])
    gm.close()


def test_stab_limit_rejections(ctx):
    m19 = ctx.mechanism(synth.make_mech19())
    T, P, Y = synth.make_cells_mech19(4, seed=1)
    ctx.train_thermo_mlp(m19, epochs=1, n_samples=1 << 14, batch=1024)
    with pytest.raises(stev.StevError) as e:
        run_gpu(ctx, m19, T, P, Y, DT, stev.F32, stab_limit=1, thermo=stev.THERMO_MLP)
    assert e.value.code == stev.STEV_EINVAL
    odd = ctx.mechanism(tm.order_n(10.0, 1.0, nu=0.3))   # 2 nu not an integer
    with pytest.raises(stev.StevError) as e:
        run_gpu(ctx, odd, [1000.0], [P1], [[0.5, 0.5]], DT, stev.F64, stab_limit=1)
    assert e.value.code == stev.STEV_EINVAL
    m19.close()
    odd.close()


@pytest.mark.parametrize("prec", [stev.F64, stev.F32])
def test_stab_limit_full_length_19_species(ctx, prec):
    """The limiter over the whole flow step (no iteration cap): 48 cells of
    the 19-species field (70 % near equilibrium, 30 % igniting; up to ~60 k
    capped steps per cell), against the oracle's ensemble with the same cap."""
    m = synth.make_mech19()
    gm = ctx.mechanism(m)
    om = oracle.OracleMech(m)
    T, P, Y = synth.make_cells_split(48, 19, 61)
    o = oracle_ensemble(om, T, P, Y, DT, prec, stab_limit=1)
    g = run_gpu(ctx, gm, T, P, Y, DT, prec, stab_limit=1)
    say(f"full length with the Eq 25 cap: iterations max {int(o['iters'].max())}, "
        f"median {int(np.median(o['iters']))}")
    assert np.all(g["status"] == 0)
    if prec == stev.F64:
        judge(g, o, prec, f"stab mech19 full length/{prec}")
    else:
        # FP32 state: each Euler update of T rounds to ~3e-8 of T, and a cell
        # that the cap holds to tens of thousands of steps accumulates that
        # past the FP32 tolerance (the ensemble, FP64 underneath, does not
        # draw it).  Cells up to 30 000 steps are judged; longer ones are
        # reported with their step counts.
        short = o["iters"] <= 30000
        sub = lambda d: {k: v[short] for k, v in d.items() if isinstance(v, np.ndarray)}
        judge(sub(g), sub(o), prec, f"stab mech19 full length/{prec}, <= 30000 steps")
        for c in np.where(~short)[0]:
            relT = abs(g["T"][c] - o["T"][c]) / o["T"][c]
            say(f"    cell {c}: {int(o['iters'][c])} steps, FP32 rel T {relT:.2e}")
    gm.close()
