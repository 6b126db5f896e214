"""Thermo network (Sec 3) on the GPU: training kernels, gradients against the
FP64 oracle, MFMA inference against the oracle's forward pass with the same
weights, polynomial fallback, and integration with the network in the loop."""

import time

import numpy as np
import pytest

import oracle
from paper_1905_09395_amd import stev, synth
from tests.gpu_common import (judge, judge_strict, oracle_ensemble, oracle_with_gpu_network,
                              run_gpu, say)

pytestmark = pytest.mark.gpu
H = 32


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a HIP device"
    c = stev.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def m19(ctx):
    m = synth.make_mech19()
    gm = ctx.mechanism(m)
    say("training the 19-species thermo network (2^20 samples)")
    rep = ctx.train_thermo_mlp(gm, epochs=300, n_samples=1 << 20, batch=8192, lr=3e-3, seed=104)
    say(f"train report {rep}")
    return m, gm, oracle.OracleMech(m), rep


def test_gradient_matches_oracle(ctx):
    rng = np.random.default_rng(11)
    n_out = 38
    npar = oracle.mlp_n_params(H, n_out)
    prm = rng.normal(size=npar) * 0.3
    x = rng.uniform(-1, 1, 300)
    t = rng.normal(size=(300, n_out))
    loss_o, g_o = oracle.mlp_loss_grad(H, n_out, prm, x, t)
    loss_g, g_g = ctx.mlp_loss_grad(n_out, prm.astype(np.float32), x, t)
    dg = np.abs(g_g - g_o)
    rel = dg / np.maximum(np.abs(g_o), 1e-3 * np.abs(g_o).max())
    say(f"loss oracle {loss_o:.8e} gpu {loss_g:.8e}; max |dg| {dg.max():.3e} "
        f"of max |g| {np.abs(g_o).max():.3e}; max rel (floor 1e-3 max|g|) {rel.max():.3e}")
    assert loss_g == pytest.approx(loss_o, rel=1e-6)
    # FP32 forward/backward against FP64, 300 samples: each entry within 1e-5
    # of the gradient's scale, and within 1e-4 of itself where it is not tiny
    assert dg.max() <= 1e-5 * np.abs(g_o).max()
    assert rel.max() <= 1e-4


def test_poly_eval_matches_oracle(ctx, m19):
    m, gm, om, _ = m19
    T = np.linspace(250.0, 3300.0, 257)
    cp, h = ctx.thermo_eval(gm, T, stev.THERMO_POLY)
    cpo, ho = oracle.nasa_targets(om, T)
    np.testing.assert_allclose(cp, cpo, rtol=1e-13)
    np.testing.assert_allclose(h, ho, rtol=1e-12, atol=1e-9 * np.abs(ho).max())


def test_training_accuracy(m19):
    _, _, _, rep = m19
    assert rep["steps"] > 0
    assert rep["test_loss"] < 1e-3
    assert rep["test_loss"] < 3 * rep["train_loss"] + 1e-6
    assert rep["max_rel_err_cp"] < 0.05
    assert rep["mean_rel_err_cp"] < 0.01


def test_network_inference_matches_oracle_forward(ctx, m19):
    """BF16 hi/lo MFMA inference vs the oracle's FP64 forward pass on the
    exported FP32 weights; outside the trained range: the polynomials."""
    m, gm, om, _ = m19
    n_s = m["n_s"]
    w = ctx.get_thermo_mlp(gm).astype(np.float64)
    npar = oracle.mlp_n_params(H, 2 * n_s)
    prm, z = w[:npar], w[npar:]
    mean = np.concatenate([z[:n_s], z[2 * n_s:3 * n_s]])
    sd = np.concatenate([z[n_s:2 * n_s], z[3 * n_s:]])
    T = np.concatenate([np.linspace(300.0, 3000.0, 301), [250.0, 299.0, 3001.0, 3400.0]])
    cp, h = ctx.thermo_eval(gm, T, stev.THERMO_MLP)
    y = oracle.mlp_forward(H, 2 * n_s, prm, (T - 1650.0) / 1350.0) * sd + mean
    inr = (T >= 300.0) & (T <= 3000.0)
    # bf16x3 products: ~2^-16 relative per term, 32-term sums of O(1) values
    err_cp = np.abs(cp[inr] - y[inr, :n_s]) / sd[:n_s]
    err_h = np.abs(h[inr] - y[inr, n_s:]) / sd[n_s:]
    say(f"MFMA inference vs FP64 forward (z units): cp {err_cp.max():.2e} h {err_h.max():.2e}")
    # (output weights up to ~10 after the damped least-squares output layer:
    # sums of |w a| up to ~40 at 2^-16 each)
    assert err_cp.max() < 1e-3 and err_h.max() < 1e-3
    cpo, ho = oracle.nasa_targets(om, T[~inr])
    np.testing.assert_allclose(cp[~inr], cpo, rtol=1e-13)
    np.testing.assert_allclose(h[~inr], ho, rtol=1e-12)


def test_fallback_is_bitwise_polynomial(ctx, m19):
    """A network whose range no cell reaches leaves every result bit-identical
    to the polynomial path (FP32)."""
    m, gm, om, _ = m19
    w = ctx.get_thermo_mlp(gm)
    m2 = ctx.mechanism(m)
    ctx.set_thermo_mlp(m2, H, 5000.0, 6000.0, w)
    T, P, Y = synth.make_cells_mech19(200, seed=31)
    a = run_gpu(ctx, m2, T, P, Y, 1e-4, stev.F32, thermo=stev.THERMO_MLP)
    b = run_gpu(ctx, m2, T, P, Y, 1e-4, stev.F32, thermo=stev.THERMO_POLY)
    assert np.array_equal(a["T"], b["T"]) and np.array_equal(a["Y"], b["Y"])
    assert np.array_equal(a["iters"], b["iters"])
    m2.close()


def test_integration_with_network(ctx, m19):
    """FP32 + network, judged by the FP32 criterion twice: for parity against
    the oracle evaluating the same network in FP64, and for accuracy against
    the oracle's polynomials (the network's fit error included), next to the
    FP32 polynomial path on the same cells.  Well-conditioned cells are held
    to the tolerance; chaotic cells are reported (their ensemble spread does
    not model the BF16 inference's perturbation of cp and h)."""
    m, gm, om, _ = m19
    T, P, Y = synth.make_cells_mech19()
    idx = synth.subsample(len(T), 259, seed=12)
    T, P, Y = T[idx], P[idx], Y[idx]
    o = oracle_ensemble(om, T, P, Y, 1e-4, stev.F32)
    gp = run_gpu(ctx, gm, T, P, Y, 1e-4, stev.F32, thermo=stev.THERMO_POLY)
    judge(gp, o, stev.F32, "f32 poly vs polynomial oracle")
    gn = run_gpu(ctx, gm, T, P, Y, 1e-4, stev.F32, thermo=stev.THERMO_MLP)
    assert np.all(gn["status"] == 0)
    on = oracle_with_gpu_network(ctx, gm, om)
    onet = oracle_ensemble(on, T, P, Y, 1e-4, stev.F32)
    judge(gn, onet, stev.F32, "f32 network vs oracle with the same network",
          ill_allowance=False)
    relT = np.abs(gn["T"] - o["T"]) / o["T"]
    say(f"network path vs polynomials: max rel T err {relT.max():.2e} "
        f"median {np.median(relT):.2e}")
    judge(gn, o, stev.F32, "f32 network vs polynomial oracle", ill_allowance=False)


@pytest.mark.parametrize("thermo", [stev.THERMO_POLY, stev.THERMO_MLP])
def test_learned_thermo_field_every_cell_short_run(ctx, m19, thermo):
    """The 1 048 576-cell learned-thermo field in FP32, every cell over 10
    steps (status 2 for the cells that would go on), held to the FP32
    tolerance (a cell outside must be shown ill-conditioned at FP32 by the
    oracle's ensemble and lie within its allowance): the polynomial path
    against the polynomial
    oracle, the network path against the oracle with the same network."""
    m, gm, om, _ = m19
    T, P, Y = synth.make_cells_mech19(1 << 20, seed=104)
    g = run_gpu(ctx, gm, T, P, Y, 1e-4, stev.F32, thermo=thermo, max_iters=10,
                allow_failed=True)
    ref = om if thermo == stev.THERMO_POLY else oracle_with_gpu_network(ctx, gm, om)
    o = oracle.integrate(ref, T, P, Y, 1e-4, max_iters=10)
    judge_strict(g, o, stev.F32, f"1M cells, 10 steps, thermo={thermo}",
                 recheck=lambda c: oracle_ensemble(ref, T[c], P[c], Y[c], 1e-4, stev.F32,
                                                   max_iters=10))


def test_network_cost_vs_polynomials(ctx, m19):
    """Reports what the network gains (or loses) against the polynomials."""
    import torch
    m, gm, om, _ = m19
    T, P, Y = synth.make_cells_mech19(65536, seed=14)
    ms = {}
    for name, th in (("poly", stev.THERMO_POLY), ("network", stev.THERMO_MLP)):
        best = 1e30
        for _ in range(3):
            g = run_gpu(ctx, gm, T, P, Y, 1e-4, stev.F32, thermo=th, max_iters=300,
                        allow_failed=True)
            best = min(best, g["stats"]["kernel_ms"])
        ms[name] = best
    say(f"65536 cells x <=300 iterations, FP32: polynomials {ms['poly']:.2f} ms, "
        f"network {ms['network']:.2f} ms, network/poly = {ms['network'] / ms['poly']:.3f}")
    assert ms["network"] > 0 and ms["poly"] > 0
