"""Oracle (test infrastructure only) for the paper's thermo network and its
Levenberg-Marquardt training (Section 3).

The network maps one normalised temperature to the species properties:
one hidden layer of sigmoid units, as many as there are outputs, and a
linear output layer.  Parameters are one flat FP64 vector laid out as
[W2 (n_out x H, row-major), b2 (n_out), w1 (H), b1 (H)]:

    a = sigmoid(w1 x + b1),   y = W2 a + b2.

Training minimises the sum of squared residuals y - t over the samples by
Levenberg-Marquardt: with J the Jacobian of all residuals with respect to
the parameters, a step solves (J^T J + lam D) d = -J^T r; it is kept when
the loss falls (then lam shrinks) and discarded otherwise (lam grows).  The
paper does not give the damping matrix; D here is Marquardt's diag(J^T J)
with a floor of mu times its mean (mu = 1e-6), so that directions with a
nearly vanishing diagonal are still damped (38 sigmoids of one input give
cond(J^T J) near 1e21, and the plain diagonal lets steps blow up).

Everything here is written from those definitions: the Jacobian is formed
explicitly per sample, J^T J and J^T r are summed sample by sample, and the
step uses a library linear solve.  Plain and slow; the GPU
path shares no code with it.
"""

import numpy as np


def n_params(H, n_out):
    return n_out * H + n_out + 2 * H


def unpack(prm, H, n_out):
    prm = np.asarray(prm, dtype=np.float64)
    W2 = prm[:n_out * H].reshape(n_out, H)
    b2 = prm[n_out * H:n_out * H + n_out]
    w1 = prm[n_out * H + n_out:n_out * H + n_out + H]
    b1 = prm[n_out * H + n_out + H:]
    return W2, b2, w1, b1


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def forward(prm, H, n_out, x):
    """Network outputs for the inputs x (n,) -> (n, n_out)."""
    W2, b2, w1, b1 = unpack(prm, H, n_out)
    a = sigmoid(np.outer(x, w1) + b1)
    return a @ W2.T + b2


def jacobian(prm, H, n_out, x):
    """d y / d prm for each sample: (n, n_out, P), from the chain rule."""
    W2, b2, w1, b1 = unpack(prm, H, n_out)
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    z = np.outer(x, w1) + b1
    a = sigmoid(z)
    ds = a * (1.0 - a)                          # sigmoid'(z)
    P = n_params(H, n_out)
    J = np.zeros((n, n_out, P))
    for o in range(n_out):
        J[:, o, o * H:(o + 1) * H] = a           # d y_o / d W2[o, :]
        J[:, o, n_out * H + o] = 1.0             # d y_o / d b2[o]
        g = W2[o][None, :] * ds                  # d y_o / d z
        J[:, o, n_out * H + n_out:n_out * H + n_out + H] = g * x[:, None]   # w1
        J[:, o, n_out * H + n_out + H:] = g                                   # b1
    return J


def normal_equations(prm, H, n_out, x, target, chunk=64):
    """(J^T J, J^T r, loss) with r = y - target, loss = sum r^2."""
    P = n_params(H, n_out)
    JtJ = np.zeros((P, P))
    Jtr = np.zeros(P)
    loss = 0.0
    x = np.asarray(x, dtype=np.float64)
    target = np.asarray(target, dtype=np.float64)
    for s0 in range(0, len(x), chunk):
        xs = x[s0:s0 + chunk]
        r = forward(prm, H, n_out, xs) - target[s0:s0 + chunk]
        J = jacobian(prm, H, n_out, xs).reshape(-1, P)
        JtJ += J.T @ J
        Jtr += J.T @ r.reshape(-1)
        loss += float(np.sum(r * r))
    return JtJ, Jtr, loss


MU = 1e-6


def damping(JtJ, mu=MU):
    """Diagonal of the damping matrix: diag(J^T J) + mu * mean(diag(J^T J))."""
    dg = np.diag(JtJ)
    return dg + mu * np.mean(dg)


def lma_step(JtJ, Jtr, lam, mu=MU):
    """Step d of (J^T J + lam D) d = -J^T r."""
    A = JtJ + lam * np.diag(damping(JtJ, mu))
    return np.linalg.solve(A, -Jtr)


def loss(prm, H, n_out, x, target):
    r = forward(prm, H, n_out, x) - np.asarray(target, dtype=np.float64)
    return float(np.sum(r * r))


def train(prm, H, n_out, x, target, iters, lam=1e-3, up=10.0, down=10.0):
    """Levenberg-Marquardt iterations; returns (prm, loss history, lam)."""
    prm = np.array(prm, dtype=np.float64)
    hist = []
    JtJ, Jtr, cur = normal_equations(prm, H, n_out, x, target)
    for _ in range(iters):
        d = lma_step(JtJ, Jtr, lam)
        trial = prm + d
        new = loss(trial, H, n_out, x, target)
        if new < cur:
            prm, cur = trial, new
            lam /= down
            JtJ, Jtr, cur = normal_equations(prm, H, n_out, x, target)
        else:
            lam *= up
        hist.append(cur)
    return prm, hist, lam
