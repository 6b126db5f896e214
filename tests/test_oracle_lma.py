"""Pins of the oracle for the paper's thermo network and its
Levenberg-Marquardt training (Section 3), each against something other than
the oracle's own formulas: finite differences for the Jacobian, a QR-based
least-squares solve for the undamped step, and recovery of a known network."""

import numpy as np

from oracle import ann_lma as L


def _rand_params(rng, H, n_out, scale=1.0):
    return rng.normal(0.0, scale, L.n_params(H, n_out))


def test_jacobian_matches_central_differences():
    rng = np.random.default_rng(11)
    H, n_out = 5, 4
    prm = _rand_params(rng, H, n_out)
    x = rng.uniform(-1.0, 1.0, 7)
    J = L.jacobian(prm, H, n_out, x)
    eps = 1e-6
    for k in range(len(prm)):
        dp = np.zeros_like(prm)
        dp[k] = eps
        fd = (L.forward(prm + dp, H, n_out, x) - L.forward(prm - dp, H, n_out, x)) / (2 * eps)
        np.testing.assert_allclose(J[:, :, k], fd, rtol=1e-7, atol=1e-9)


def test_undamped_step_is_the_least_squares_step():
    # lambda = 0: (J^T J) d = -J^T r is the Gauss-Newton step, the minimiser
    # of |J d + r|, which a QR/SVD least-squares solve finds independently
    # (a network with spread sigmoid centres: cond(J) ~ 5e4, so the normal
    # equations, conditioned as cond(J)^2, still carry ~7 digits)
    rng = np.random.default_rng(12)
    H, n_out = 3, 2
    W2 = rng.normal(0.0, 1.0, (n_out, H))
    b2 = rng.normal(0.0, 1.0, n_out)
    prm = np.concatenate([W2.ravel(), b2, [2.0, -2.5, 3.0], [1.0, 0.0, -1.2]])
    x = rng.uniform(-1.0, 1.0, 60)
    t = rng.normal(0.0, 1.0, (60, n_out))
    JtJ, Jtr, loss = L.normal_equations(prm, H, n_out, x, t)
    d = L.lma_step(JtJ, Jtr, 0.0)
    J = L.jacobian(prm, H, n_out, x).reshape(-1, len(prm))
    r = (L.forward(prm, H, n_out, x) - t).reshape(-1)
    d_ls = np.linalg.lstsq(J, -r, rcond=None)[0]
    np.testing.assert_allclose(d, d_ls, rtol=1e-5, atol=1e-8 * np.abs(d_ls).max())
    assert np.isclose(loss, float(r @ r))


def test_damping_shrinks_the_step_towards_the_gradient_direction():
    # large lambda: d -> -(J^T r) / (lambda D), a scaled descent step, D the
    # diagonal of J^T J with its floor (mu times the mean diagonal)
    rng = np.random.default_rng(13)
    H, n_out = 3, 2
    prm = _rand_params(rng, H, n_out)
    x = rng.uniform(-1.0, 1.0, 40)
    t = rng.normal(0.0, 1.0, (40, n_out))
    JtJ, Jtr, _ = L.normal_equations(prm, H, n_out, x, t)
    lam = 1e9
    d = L.lma_step(JtJ, Jtr, lam)
    D = np.diag(JtJ) + 1e-6 * np.mean(np.diag(JtJ))
    np.testing.assert_allclose(d, -Jtr / (lam * D), rtol=1e-6)


def test_fits_a_known_network():
    # targets made by a network of the same shape: the fit error must fall by
    # orders of magnitude and never rise (rejected steps are discarded).  The
    # normal equations square cond(J) (~1e5 here), so progress stalls near a
    # residual of 1e-6 rather than at round-off.
    rng = np.random.default_rng(14)
    H, n_out = 4, 3
    teacher = np.concatenate([rng.normal(0.0, 1.0, n_out * H), rng.normal(0.0, 1.0, n_out),
                              [2.0, -2.5, 3.0, -1.5], [1.0, 0.0, -1.2, 0.4]])
    x = rng.uniform(-1.0, 1.0, 200)
    t = L.forward(teacher, H, n_out, x)
    student = teacher + rng.normal(0.0, 0.05, len(teacher))
    prm, hist, _ = L.train(student, H, n_out, x, t, iters=40)
    assert all(b <= a for a, b in zip(hist, hist[1:]))
    assert hist[-1] < 1e-5 * L.loss(student, H, n_out, x, t)
    np.testing.assert_allclose(L.forward(prm, H, n_out, x), t, atol=1e-4)
