"""The paper's sigmoid thermo network (Section 3) inside the integrator: the
network fitted by Levenberg-Marquardt on the GPU is attached as a thermo
mode and the integration is compared with the oracle evaluating the same
network in FP64 (parity), with the polynomial oracle (what the network's fit
error costs in accuracy), and timed against the polynomials and the tanh
network (what it gains)."""

import numpy as np
import pytest

import oracle
from paper_1905_09395_amd import stev, synth
from tests.gpu_common import judge, judge_strict, oracle_ensemble, run_gpu, say

pytestmark = pytest.mark.gpu
T_LO, T_HI = 300.0, 3000.0


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a HIP device"
    c = stev.Context(0)
    yield c
    c.close()


def _attach(ctx, m, iters, seed):
    gm = ctx.mechanism(m)
    rep, prm = ctx.train_thermo_lma(gm, iters=iters, n_samples=1 << 16, T_lo=T_LO, T_hi=T_HI,
                                    seed=seed)
    say(f"LMA sigmoid network, {m['n_s']} species: hidden {rep['hidden']}, test loss "
        f"{rep['test_loss']:.2e}, cp max/mean rel err {rep['max_rel_cp']:.2e}/"
        f"{rep['mean_rel_cp']:.2e}, {rep['accepted']} accepted, {rep['train_ms']:.0f} ms")
    ctx.set_thermo_ann(gm, rep["hidden"], T_LO, T_HI, prm)
    om = oracle.OracleMech(m)
    return dict(m=m, gm=gm, om=om, on=om.with_ann(rep["hidden"], prm, T_LO, T_HI),
                prm=prm, H=rep["hidden"], rep=rep)


@pytest.fixture(scope="module")
def n19(ctx):
    return _attach(ctx, synth.make_mech19(), 150, 104)


@pytest.fixture(scope="module")
def n6(ctx):
    return _attach(ctx, synth.make_mech6(), 150, 105)


def test_trained_network_reproduces_the_polynomials(n19):
    """The folded output layer gives cp/R and h/R in physical units: the
    oracle's forward pass of the returned parameters stays within the fit
    error of the polynomials."""
    m, om, H = n19["m"], n19["om"], n19["H"]
    n_s = m["n_s"]
    T = np.linspace(T_LO, T_HI, 301)
    y = oracle.ann_forward(H, 2 * n_s, n19["prm"], (T - 1650.0) / 1350.0)
    cp = np.array([[oracle.thermo(om, k, t)[0] for k in range(n_s)] for t in T])
    rel = np.abs(y[:, :n_s] - cp) / np.abs(cp)
    say(f"network cp/R against the polynomials: max rel {rel.max():.2e}, "
        f"mean {rel.mean():.2e}")
    assert rel.max() < 1e-2


def test_eval_matches_oracle_forward(ctx, n19):
    """The FP64 network as the FP64 integrator evaluates it, against the
    oracle's forward pass with the same parameters; the polynomials, bit for
    bit, outside the trained range."""
    m, gm, H, prm = n19["m"], n19["gm"], n19["H"], n19["prm"]
    n_s = m["n_s"]
    T = np.concatenate([np.linspace(250.0, 3300.0, 257), [T_LO, T_HI]])
    cp, h = ctx.thermo_eval(gm, T, stev.THERMO_ANN)
    cpp, hp = ctx.thermo_eval(gm, T, stev.THERMO_POLY)
    inside = (T >= T_LO) & (T <= T_HI)
    y = oracle.ann_forward(H, 2 * n_s, prm, (T[inside] - 1650.0) / 1350.0)
    W2 = prm[:2 * n_s * H].reshape(2 * n_s, H)
    scale = np.abs(prm[2 * n_s * H:2 * n_s * H + 2 * n_s]) + np.abs(W2).sum(axis=1)
    err = np.abs(np.concatenate([cp[inside], h[inside]], axis=1) - y) / scale
    say(f"sigmoid network, FP64 GPU vs oracle: max error {err.max():.2e} of the output scale")
    assert err.max() < 1e-13
    assert np.array_equal(cp[~inside], cpp[~inside]) and np.array_equal(h[~inside], hp[~inside])


@pytest.mark.parametrize("precision", [stev.F64, stev.F32])
def test_fallback_is_bitwise_polynomial(ctx, n19, precision):
    """A network whose range no cell reaches leaves every result bit-identical
    to the polynomial path."""
    m = n19["m"]
    m2 = ctx.mechanism(m)
    ctx.set_thermo_ann(m2, n19["H"], 5000.0, 6000.0, n19["prm"])
    T, P, Y = synth.make_cells_mech19(200, seed=31)
    a = run_gpu(ctx, m2, T, P, Y, 1e-4, precision, thermo=stev.THERMO_ANN)
    b = run_gpu(ctx, m2, T, P, Y, 1e-4, precision, thermo=stev.THERMO_POLY)
    assert np.array_equal(a["T"], b["T"]) and np.array_equal(a["Y"], b["Y"])
    assert np.array_equal(a["iters"], b["iters"])
    m2.close()


@pytest.mark.parametrize("precision", [stev.F64, stev.F32])
def test_field_every_cell_short_run(ctx, n19, precision):
    """The 262 144-cell 19-species field with the network in the loop, every
    cell over 10 steps, against the oracle with the same network: FP64 to
    1e-9 with equal iteration counts, FP32 to its tolerance (a cell outside
    must be ill-conditioned at FP32 by the oracle's ensemble)."""
    gm, on = n19["gm"], n19["on"]
    T, P, Y = synth.make_cells_mech19()
    g = run_gpu(ctx, gm, T, P, Y, 1e-4, precision, thermo=stev.THERMO_ANN, max_iters=10,
                allow_failed=True)
    o = oracle.integrate(on, T, P, Y, 1e-4, max_iters=10)
    judge_strict(g, o, precision, f"262144 cells, 10 steps, sigmoid network, prec={precision}",
                 recheck=lambda c: oracle_ensemble(on, T[c], P[c], Y[c], 1e-4, stev.F32,
                                                   max_iters=10))


@pytest.mark.parametrize("precision", [stev.F64, stev.F32])
def test_full_length_sample(ctx, n19, precision):
    """259 sampled cells of the 19-species field over the whole flow step:
    parity with the oracle evaluating the same network (its ensemble), and
    the accuracy the network's fit costs against the polynomial oracle,
    reported beside the polynomial path's."""
    gm, om, on = n19["gm"], n19["om"], n19["on"]
    T, P, Y = synth.make_cells_mech19()
    idx = synth.subsample(len(T), 259, seed=12)
    T, P, Y = T[idx], P[idx], Y[idx]
    g = run_gpu(ctx, gm, T, P, Y, 1e-4, precision, thermo=stev.THERMO_ANN)
    assert np.all(g["status"] == 0)
    onet = oracle_ensemble(on, T, P, Y, 1e-4, precision)
    judge(g, onet, precision, f"sigmoid network vs oracle with the same network, prec={precision}")
    o = oracle.integrate(om, T, P, Y, 1e-4)
    relT = np.abs(g["T"] - o["T"]) / o["T"]
    m = o["Y"] > 1e-6
    relY = np.where(m, np.abs(g["Y"] - o["Y"]) / np.where(m, o["Y"], 1.0), 0.0).max(axis=1)
    say(f"sigmoid network vs the polynomial oracle (fit error included), prec={precision}: "
        f"rel T max {relT.max():.2e} median {np.median(relT):.2e}; rel Y (Y > 1e-6) max "
        f"{relY.max():.2e} median {np.median(relY):.2e}; within 1e-4 / 1e-3: "
        f"{int(np.sum((relT <= 1e-4) & (relY <= 1e-3)))} of {len(T)}")


def test_small_mechanism_full_field(ctx, n6):
    """The 1024-cell 6-species field (one cell per lane) with its own network,
    FP64, against the oracle with the same network."""
    gm, on = n6["gm"], n6["on"]
    T, P, Y = synth.make_cells_mech6()
    g = run_gpu(ctx, gm, T, P, Y, 1e-4, stev.F64, thermo=stev.THERMO_ANN)
    o = oracle_ensemble(on, T, P, Y, 1e-4, stev.F64)
    judge(g, o, stev.F64, "1024 cells mech6, sigmoid network, FP64")


def test_cost_against_polynomials_and_tanh_network(ctx, n19):
    """Reports the in-loop cost of the sigmoid network against the
    polynomials and the 32-32 tanh network (the paper reports the network
    evaluation faster than the polynomials; here both run in registers)."""
    m, gm = n19["m"], n19["gm"]
    ctx.train_thermo_mlp(gm, epochs=20, n_samples=1 << 16, batch=4096, lr=3e-3, seed=104)
    T, P, Y = synth.make_cells_mech19(65536, seed=14)
    ms = {}
    for prec in (stev.F32, stev.F64):
        for name, th in (("poly", stev.THERMO_POLY), ("sigmoid", stev.THERMO_ANN),
                         ("tanh", stev.THERMO_MLP)):
            if th == stev.THERMO_MLP and prec == stev.F64:
                continue
            best = 1e30
            for _ in range(3):
                g = run_gpu(ctx, gm, T, P, Y, 1e-4, prec, thermo=th, max_iters=300,
                            allow_failed=True)
                best = min(best, g["stats"]["kernel_ms"])
            ms[(prec, name)] = best
    for prec in (stev.F32, stev.F64):
        p = ms[(prec, "poly")]
        line = ", ".join(f"{k[1]} {v:.2f} ms ({v / p:.3f}x)" for k, v in ms.items() if k[0] == prec)
        say(f"65536 cells x <=300 iterations, {'FP32' if prec == stev.F32 else 'FP64'}: {line}")
    assert all(v > 0 for v in ms.values())


@pytest.mark.parametrize("precision", [stev.F64, stev.F32])
def test_other_entry_points_with_the_sigmoid_network(ctx, n19, precision):
    """The sigmoid thermo mode through the multi-batch launch (hottest-first
    groups), the allocation-free call and a served request gives, cell for
    cell, the bits of a plain call."""
    import time
    import torch
    gm = n19["gm"]
    T, P, Y = synth.make_cells_mech19(9000, seed=77)
    dt = torch.float64 if precision == stev.F64 else torch.float32
    prm = stev.default_params(precision=precision, thermo=stev.THERMO_ANN)

    def dev(a):
        return torch.tensor(a, dtype=dt, device="cuda").contiguous()

    ref = run_gpu(ctx, gm, T, P, Y, 1e-4, precision, thermo=stev.THERMO_ANN)
    # two batches of 4 500 and 4 500 cells in one launch
    Ts, Ps, Ys = [dev(T[:4500]), dev(T[4500:])], [dev(P[:4500]), dev(P[4500:])], \
        [dev(Y[:4500]), dev(Y[4500:])]
    ctx.integrate_batched([gm, gm], Ts, Ps, Ys, 1e-4, params=prm)
    torch.cuda.synchronize()
    bT = np.concatenate([t.cpu().double().numpy() for t in Ts])
    bY = np.concatenate([y.cpu().double().numpy() for y in Ys])
    assert np.array_equal(bT, ref["T"]) and np.array_equal(bY, ref["Y"])
    # allocation-free
    Tn, Pn, Yn = dev(T), dev(P), dev(Y)
    ctx.integrate_noalloc(gm, Tn, Pn, Yn, 1e-4, params=prm)
    torch.cuda.synchronize()
    assert np.array_equal(Tn.cpu().double().numpy(), ref["T"])
    assert np.array_equal(Yn.cpu().double().numpy(), ref["Y"])
    # served (host arrays, staged)
    Th = np.array(T, dtype=np.float64 if precision == stev.F64 else np.float32)
    Yh = np.ascontiguousarray(Y, dtype=Th.dtype)
    Ph = np.ascontiguousarray(P, dtype=Th.dtype)
    tk = ctx.submit(gm, Th, Ph, Yh, 1e-4, params=prm)
    while True:
        rc, _ = ctx.poll(tk)
        if rc != stev.STEV_EAGAIN:
            break
        time.sleep(1e-3)
    assert rc == stev.STEV_OK
    assert np.array_equal(Th.astype(np.float64), ref["T"])
    assert np.array_equal(Yh.astype(np.float64), ref["Y"])
