"""The paper's thermo network trained by Levenberg-Marquardt on the GPU
(Section 3): the GPU's structured sums for J^T J, J^T r and the loss against
the oracle's sample-by-sample Jacobian products, the damped step against
the oracle's linear solve, a short training trajectory step by step, and a
full fit of the 19-species polynomials beside the tanh / Adam network."""

import numpy as np
import pytest

from oracle import ann_lma as L
from paper_1905_09395_amd import stev, synth
from tests.gpu_common import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a HIP device"
    c = stev.Context(0)
    yield c
    c.close()


def spread_network(rng, H, n_out):
    """Sigmoid centres spread over [-1, 1], alternating slopes: a
    well-conditioned point for comparisons."""
    c = -1.0 + 2.0 * (np.arange(H) + 0.5) / H
    w1 = np.where(np.arange(H) % 2 == 0, 1.0, -1.0) * rng.uniform(2.0, 4.0, H)
    return np.concatenate([rng.normal(0.0, 0.3, n_out * H), rng.normal(0.0, 0.3, n_out),
                           w1, -w1 * c])


@pytest.mark.parametrize("H,n_out", [(12, 12), (38, 38), (7, 12)])
def test_normal_equations_match_oracle(ctx, H, n_out):
    rng = np.random.default_rng(H * 100 + n_out)
    prm = spread_network(rng, H, n_out)
    x = rng.uniform(-1.0, 1.0, 200)
    t = rng.normal(0.0, 1.0, (200, n_out))
    A, g, loss, _ = ctx.lma_normal_eq(H, n_out, prm, x, t)
    A_o, g_o, loss_o = L.normal_equations(prm, H, n_out, x, t)
    say(f"H={H} n_out={n_out}: max |dJtJ| / max|JtJ| = "
        f"{np.abs(A - A_o).max() / np.abs(A_o).max():.2e}")
    np.testing.assert_allclose(A, A_o, rtol=0, atol=1e-11 * np.abs(A_o).max())
    np.testing.assert_allclose(g, g_o, rtol=0, atol=1e-11 * np.abs(g_o).max())
    assert abs(loss - loss_o) <= 1e-11 * loss_o


@pytest.mark.parametrize("lam", [1e-2, 1.0])
def test_damped_step_matches_oracle(ctx, lam):
    rng = np.random.default_rng(21)
    H, n_out = 38, 38
    prm = spread_network(rng, H, n_out)
    x = rng.uniform(-1.0, 1.0, 400)
    t = rng.normal(0.0, 1.0, (400, n_out))
    _, _, _, d = ctx.lma_normal_eq(H, n_out, prm, x, t, lam=lam, jtj=False)
    A_o, g_o, _ = L.normal_equations(prm, H, n_out, x, t)
    d_o = L.lma_step(A_o, g_o, lam)
    say(f"lambda={lam}: max |d - d_oracle| / max |d_oracle| = "
        f"{np.abs(d - d_o).max() / np.abs(d_o).max():.2e}")
    np.testing.assert_allclose(d, d_o, rtol=0, atol=1e-7 * np.abs(d_o).max())


def test_training_trajectory_matches_oracle(ctx):
    """Five accept/reject iterations driven from the host with GPU steps and
    GPU losses, against the oracle's own loop on the same data."""
    rng = np.random.default_rng(22)
    H, n_out = 12, 12
    x = rng.uniform(-1.0, 1.0, 300)
    teacher = spread_network(rng, H, n_out)
    t = L.forward(teacher, H, n_out, x) + rng.normal(0.0, 1e-3, (300, n_out))
    p0 = spread_network(np.random.default_rng(23), H, n_out)
    p_o, hist_o, lam_o = L.train(p0, H, n_out, x, t, iters=5, lam=1e-2)
    p, lam = p0.copy(), 1e-2
    _, _, cur, _ = ctx.lma_normal_eq(H, n_out, p, x, t, jtj=False)
    for _ in range(5):
        _, _, _, d = ctx.lma_normal_eq(H, n_out, p, x, t, lam=lam, jtj=False)
        _, _, new, _ = ctx.lma_normal_eq(H, n_out, p + d, x, t, jtj=False)
        if new < cur:
            p, cur, lam = p + d, new, lam / 10.0
        else:
            lam *= 10.0
    assert lam == lam_o
    np.testing.assert_allclose(p, p_o, rtol=0, atol=1e-7 * np.abs(p_o).max())
    assert abs(cur - hist_o[-1]) <= 1e-8 * hist_o[-1]


def test_fit_of_the_polynomials_and_comparison(ctx):
    m = synth.make_mech19()
    gm = ctx.mechanism(m)
    rep, prm = ctx.train_thermo_lma(gm, iters=60, n_samples=1 << 16)
    say(f"LMA sigmoid {rep['hidden']} hidden ({rep['n_params']} params): test loss "
        f"{rep['test_loss']:.2e}, cp max/mean rel err {rep['max_rel_cp']:.2e}/"
        f"{rep['mean_rel_cp']:.2e}, {rep['accepted']} accepted / {rep['rejected']} rejected, "
        f"{rep['train_ms']:.0f} ms")
    assert rep["hidden"] == 38 and rep["n_params"] == stev.load().stev_lma_n_params(38, 38)
    assert rep["accepted"] >= 10
    assert rep["test_loss"] < 1e-4
    assert rep["max_rel_cp"] < 1e-2
    adam = ctx.train_thermo_mlp(gm, epochs=40, n_samples=1 << 16, batch=4096, seed=104)
    say(f"Adam tanh 32-32: test loss {adam['test_loss']:.2e}, cp max rel err "
        f"{adam['max_rel_err_cp']:.2e}, {adam['train_ms']:.0f} ms")
    gm.close()
