"""Many uneven batches in one persistent launch per mechanism (Sec 2.4 over a
set of batches), replayed from a HIP graph.  Every batch is checked against
the FP64 oracle on a seeded subsample, and every cell of every batch against
the same batch run alone through stev_integrate (bit for bit: a cell's result
depends on the cell only)."""

import numpy as np
import pytest

import oracle
from paper_1905_09395_amd import stev, synth
from tests.gpu_common import judge, oracle_ensemble, say

pytestmark = pytest.mark.gpu
DT = 1e-4


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a HIP device"
    c = stev.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def mechs(ctx):
    m6, m19 = synth.make_mech6(), synth.make_mech19()
    return {6: (m6, ctx.mechanism(m6), oracle.OracleMech(m6)),
            19: (m19, ctx.mechanism(m19), oracle.OracleMech(m19))}


def to_dev(batches, prec):
    import torch
    dt = torch.float64 if prec == stev.F64 else torch.float32
    out = []
    for key, T, P, Y in batches:
        n = len(T)
        out.append(dict(key=key, T=torch.tensor(T, dtype=dt, device="cuda"),
                        P=torch.tensor(P, dtype=dt, device="cuda"),
                        Y=torch.tensor(Y, dtype=dt, device="cuda").contiguous(),
                        it=torch.zeros(n, dtype=torch.int32, device="cuda"),
                        st=torch.zeros(n, dtype=torch.uint8, device="cuda")))
    return out


def run_batched(ctx, mechs, dev, prec, **kw):
    prm = stev.default_params(precision=prec, **kw)
    rc, stats = ctx.integrate_batched([mechs[d["key"]][1] for d in dev], [d["T"] for d in dev],
                                      [d["P"] for d in dev], [d["Y"] for d in dev], DT,
                                      params=prm, iters=[d["it"] for d in dev],
                                      status=[d["st"] for d in dev])
    return rc, stats


def host(d):
    return dict(T=d["T"].cpu().double().numpy(), Y=d["Y"].cpu().double().numpy(),
                iters=d["it"].cpu().numpy().astype(np.int64), status=d["st"].cpu().numpy())


def test_batched_64_uneven_batches(ctx, mechs):
    """64 batches, log-uniform sizes in [256, 131072], alternating 6- and
    19-species mechanisms, FP32 state, graph-recorded launch sequence."""
    import torch
    batches = synth.make_batches(64, 256, 131072, seed=103)
    prec = stev.F32
    dev = to_dev(batches, prec)
    say(f"batched: {len(dev)} batches, {sum(len(b[1]) for b in batches)} cells")
    rc, stats = run_batched(ctx, mechs, dev, prec)
    torch.cuda.synchronize()
    say(f"batched stats {stats}")
    got = [host(d) for d in dev]
    assert stats["n_cells"] == sum(len(b[1]) for b in batches)
    assert stats["total_iters"] == sum(int(g["iters"].sum()) for g in got)
    assert stats["max_cell_iters"] == max(int(g["iters"].max()) for g in got)
    assert stats["n_failed"] == 0 and all(np.all(g["status"] == 0) for g in got)

    # every cell equals the same batch integrated alone
    alone = to_dev(batches, prec)
    for d in alone:
        ctx.integrate(mechs[d["key"]][1], d["T"], d["P"], d["Y"], DT,
                      params=stev.default_params(precision=prec), iters=d["it"], status=d["st"])
    for b, (g, d) in enumerate(zip(got, alone)):
        a = host(d)
        assert np.array_equal(g["T"], a["T"]) and np.array_equal(g["Y"], a["Y"]), f"batch {b}"
        assert np.array_equal(g["iters"], a["iters"]), f"batch {b}"

    # each batch against the FP64 oracle on a seeded subsample
    for key in (6, 19):
        idx_b = [b for b in range(len(batches)) if batches[b][0] == key]
        T, P, Y, G = [], [], [], {"T": [], "Y": [], "iters": [], "status": []}
        for b in idx_b:
            sel = synth.subsample(len(batches[b][1]), 8, seed=7000 + b)
            T.append(batches[b][1][sel]); P.append(batches[b][2][sel]); Y.append(batches[b][3][sel])
            for k in G:
                G[k].append(got[b][k][sel])
        T, P, Y = np.concatenate(T), np.concatenate(P), np.concatenate(Y)
        g = {k: np.concatenate(v) for k, v in G.items()}
        o = oracle_ensemble(mechs[key][2], T, P, Y, DT, prec)
        judge(g, o, prec, f"batched mech{key} subsample")


def test_graph_replay_matches_eager(ctx, mechs):
    """Replays of the recorded sequence, with other GPU work and new input
    values in between, equal direct launches on the same inputs."""
    import torch
    batches = synth.make_batches(10, 64, 4096, seed=211)
    for prec in (stev.F64, stev.F32):
        dev = to_dev(batches, prec)
        orig = [(d["T"].clone(), d["Y"].clone()) for d in dev]
        for rep in range(4):
            shift = 7.0 * rep      # new values in the same arrays
            for d, (T0, Y0) in zip(dev, orig):
                d["T"].copy_(T0 + shift)
                d["Y"].copy_(Y0)
            ref = to_dev(batches, prec)
            for d, r in zip(dev, ref):
                r["T"].copy_(d["T"])
            say(f"graph replay {rep} prec={prec}")
            run_batched(ctx, mechs, ref, prec, use_graph=0)
            # unrelated eager work between replays
            x = torch.randn(1 << 20, device="cuda")
            (x * 2).sum().item()
            run_batched(ctx, mechs, dev, prec, use_graph=1)
            torch.cuda.synchronize()
            for b, (d, r) in enumerate(zip(dev, ref)):
                g, e = host(d), host(r)
                assert np.array_equal(g["T"], e["T"]) and np.array_equal(g["Y"], e["Y"]), \
                    f"replay {rep} batch {b}"
                assert np.array_equal(g["iters"], e["iters"])


def test_batched_edge_cases(ctx, mechs):
    import torch
    batches = synth.make_batches(6, 1, 300, seed=212)
    # empty batches at the start, middle and end; a one-cell batch
    batches = ([(6,) + synth.make_cells_mech6(0, seed=1)] + batches[:3] +
               [(19,) + synth.make_cells_mech19(0, seed=2)] + batches[3:] +
               [(19,) + synth.make_cells_mech19(1, seed=3), (6,) + synth.make_cells_mech6(0, seed=4)])
    dev = to_dev(batches, stev.F64)
    rc, stats = run_batched(ctx, mechs, dev, stev.F64)
    assert stats["n_cells"] == sum(len(b[1]) for b in batches)
    for b, d in enumerate(dev):
        if len(batches[b][1]) == 0:
            continue
        o = oracle_ensemble(mechs[batches[b][0]][2], *batches[b][1:], DT, stev.F64)
        judge(host(d), o, stev.F64, f"edge batch {b} n={len(batches[b][1])}")
    # nothing to do
    rc, stats = ctx.integrate_batched([], [], [], [], DT)
    assert rc == stev.STEV_OK and stats["n_cells"] == 0
    # host pointers are rejected before anything runs
    T, P, Y = synth.make_cells_mech6(4, seed=5)
    with pytest.raises(stev.StevError) as e:
        ctx.integrate_batched([mechs[6][1]], [np.ascontiguousarray(T)], [np.ascontiguousarray(P)],
                              [np.ascontiguousarray(Y)], DT)
    assert e.value.code == stev.STEV_EINVAL
    torch.cuda.synchronize()


def test_destroyed_mechanism_drops_recorded_sequences(ctx):
    """A recorded sequence never outlives a mechanism it launches."""
    import torch
    m6 = synth.make_mech6()
    T, P, Y = synth.make_cells_mech6(500, seed=77)
    o = oracle_ensemble(oracle.OracleMech(m6), T, P, Y, DT, stev.F64)
    first = None
    for round_ in range(3):
        gm = ctx.mechanism(m6)
        Tt = torch.tensor(T, dtype=torch.float64, device="cuda")
        Pt = torch.tensor(P, dtype=torch.float64, device="cuda")
        Yt = torch.tensor(Y, dtype=torch.float64, device="cuda")
        it = torch.zeros(500, dtype=torch.int32, device="cuda")
        stt = torch.zeros(500, dtype=torch.uint8, device="cuda")
        ctx.integrate_batched([gm], [Tt], [Pt], [Yt], DT, iters=[it], status=[stt])
        g = dict(T=Tt.cpu().numpy(), Y=Yt.cpu().numpy(), iters=it.cpu().numpy().astype(np.int64),
                 status=stt.cpu().numpy())
        if first is None:
            first = g
            judge(g, o, stev.F64, "batched, fresh mechanism")
        assert np.array_equal(g["T"], first["T"]) and np.array_equal(g["Y"], first["Y"])
        gm.close()


def test_batched_takes_each_mechanisms_tuned_shape(mechs):
    """Launch-shape fields left on auto take, per mechanism, the shape the
    context's tuner cached for that mechanism and cell count (here one fixed
    by the caller, so the outcome is known); waves and cadence change no
    result."""
    import torch
    T, P, Y = synth.make_cells_mech19(6000, seed=305)
    prec = stev.F32
    out = []
    for tune in (False, True):
        c = stev.Context(0)
        gm = c.mechanism(mechs[19][0])
        dev = to_dev([(19, T[:2500], P[:2500], Y[:2500]), (19, T[2500:], P[2500:], Y[2500:])], prec)
        if tune:
            fixed = stev.default_params(precision=prec, lanes_per_cell=64, waves_per_wg=2,
                                        compact_every=8)
            c.autotune(gm, torch.cat([d["T"] for d in dev]), torch.cat([d["P"] for d in dev]),
                       torch.cat([d["Y"] for d in dev]), DT, fixed)
        rc, st = c.integrate_batched([gm, gm], [d["T"] for d in dev], [d["P"] for d in dev],
                                     [d["Y"] for d in dev], DT,
                                     params=stev.default_params(precision=prec),
                                     iters=[d["it"] for d in dev], status=[d["st"] for d in dev])
        torch.cuda.synchronize()
        say(f"tuned cache {tune}: shape {st['lanes_per_cell']}/{st['waves_per_wg']}/"
            f"{st['compact_every']}")
        out.append(([host(d) for d in dev], st))
        gm.close()
        c.close()
    (a, sa), (b, sb) = out
    assert (sb["lanes_per_cell"], sb["waves_per_wg"], sb["compact_every"]) == (64, 2, 8)
    # auto: one cell per wave refills as soon as its cell retires, so the
    # claim attempts are spaced 64 iterations apart
    assert sa["lanes_per_cell"] == 64 and sa["compact_every"] == 64
    for x, y in zip(a, b):
        for k in ("T", "Y", "iters", "status"):
            assert np.array_equal(x[k], y[k]), k


def test_autotune(ctx, mechs):
    """The tuner returns a compiled launch shape, caches it, keeps the fields
    the caller fixed, and the tuned shape gives bit-identical results."""
    import time
    import torch
    T, P, Y = synth.make_cells_mech19(16384, seed=301)
    gm = mechs[19][1]
    for prec in (stev.F64, stev.F32):
        dt = torch.float64 if prec == stev.F64 else torch.float32
        Tt = torch.tensor(T, dtype=dt, device="cuda")
        Pt = torch.tensor(P, dtype=dt, device="cuda")
        Yt = torch.tensor(Y, dtype=dt, device="cuda")
        t0 = time.perf_counter()
        tuned = ctx.autotune(gm, Tt, Pt, Yt, DT, stev.default_params(precision=prec))
        t_tune = time.perf_counter() - t0
        say(f"autotune prec={prec}: lanes {tuned.lanes_per_cell} waves {tuned.waves_per_wg} "
            f"cadence {tuned.compact_every} ({t_tune:.2f} s)")
        assert tuned.lanes_per_cell in (8, 16, 32, 64)
        assert 1 <= tuned.waves_per_wg <= 4 and tuned.compact_every in (1, 2, 4, 8)
        # inputs untouched
        assert np.array_equal(Tt.cpu().double().numpy(), np.asarray(T, dtype=Tt.cpu().numpy().dtype))
        t0 = time.perf_counter()
        again = ctx.autotune(gm, Tt, Pt, Yt, DT, stev.default_params(precision=prec))
        assert time.perf_counter() - t0 < 0.1 * t_tune + 0.05       # cached
        assert (again.lanes_per_cell, again.waves_per_wg, again.compact_every) == \
            (tuned.lanes_per_cell, tuned.waves_per_wg, tuned.compact_every)
        fixed = ctx.autotune(gm, Tt, Pt, Yt, DT, stev.default_params(precision=prec, lanes_per_cell=16))
        assert fixed.lanes_per_cell == 16
        res = []
        for prm in (stev.default_params(precision=prec), tuned):
            T2, Y2 = Tt.clone(), Yt.clone()
            it = torch.zeros(len(T), dtype=torch.int32, device="cuda")
            _, st = ctx.integrate(gm, T2, Pt, Y2, DT, params=prm, iters=it)
            res.append((T2.cpu().numpy(), Y2.cpu().numpy(), it.cpu().numpy(), st["kernel_ms"],
                        st["lanes_per_cell"]))
        say(f"  default {res[0][3]:.2f} ms, tuned {res[1][3]:.2f} ms")
        # the same variant gives the same bits for any waves and cadence;
        # another variant orders its lane reductions differently and is held
        # to the oracle by the parity tests of every variant
        if res[0][4] == res[1][4]:
            assert all(np.array_equal(a, b) for a, b in zip(res[0][:3], res[1][:3]))
    with pytest.raises(stev.StevError):
        ctx.autotune(gm, Tt[:0], Pt[:0], Yt[:0], DT)
