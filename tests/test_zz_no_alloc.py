"""stev_integrate_noalloc (the entry point for callers that cannot allocate)
against stev_integrate: the same kernels on the same inputs, so every cell's
state, iteration count and status, and the call's statistics, must agree bit
for bit.  Two calls in a row, the second on a smaller field, then the first
again: whatever the first call left in the shared scratch array must not
reach the later ones."""

import ctypes as C

import numpy as np
import pytest

from paper_1905_09395_amd import stev, synth
from tests.gpu_common import say

pytestmark = pytest.mark.gpu

DT = 1e-4


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a HIP device"
    c = stev.Context(0)
    yield c
    c.close()


def _run(ctx, gm, T, P, Y, prec, noalloc, **kw):
    import torch
    dtype = torch.float64 if prec == stev.F64 else torch.float32
    Tt = torch.tensor(T, dtype=dtype, device="cuda")
    Pt = torch.tensor(P, dtype=dtype, device="cuda")
    Yt = torch.tensor(Y, dtype=dtype, device="cuda").contiguous()
    it = torch.full((len(T),), -1, dtype=torch.int32, device="cuda")
    st = torch.full((len(T),), 255, dtype=torch.uint8, device="cuda")
    prm = stev.default_params(precision=prec, **kw)
    f = ctx.integrate_noalloc if noalloc else ctx.integrate
    rc, stats = f(gm, Tt, Pt, Yt, DT, params=prm, iters=it, status=st, allow_failed=True)
    torch.cuda.synchronize()
    return dict(rc=rc, stats=stats, T=Tt.cpu().numpy(), Y=Yt.cpu().numpy(),
                iters=it.cpu().numpy(), status=st.cpu().numpy())


def _same(a, b, label):
    for k in ("T", "Y", "iters", "status"):
        assert np.array_equal(a[k], b[k], equal_nan=True), (label, k)
    assert a["rc"] == b["rc"], label
    for k in ("n_cells", "total_iters", "max_cell_iters", "n_failed", "lanes_per_cell",
              "waves_per_wg", "grid_wgs"):
        assert a["stats"][k] == b["stats"][k], (label, k)


def test_noalloc_matches_integrate_twice(ctx):
    m19 = synth.make_mech19()
    gm = ctx.mechanism(m19)
    T, P, Y = synth.make_cells_mech19(9001, seed=43)
    T = T.copy()
    T[77] = np.nan                       # one failing cell: status 1, reported alike
    Ts, Ps, Ys = synth.make_cells_mech19(1500, seed=44)
    cases = [("9001 cells, probe-refined order", T, P, Y, stev.F64, dict(hot_first=2)),
             ("1500 cells, array order", Ts, Ps, Ys, stev.F64, dict()),
             ("9001 cells again, FP32", T, P, Y, stev.F32, dict(hot_first=2)),
             ("1500 cells, FP32, max_iters 40", Ts, Ps, Ys, stev.F32, dict(max_iters=40))]
    for label, t, p, y, prec, kw in cases:
        say(f"noalloc vs integrate: {label}")
        ref = _run(ctx, gm, t, p, y, prec, False, **kw)
        got = _run(ctx, gm, t, p, y, prec, True, **kw)
        _same(ref, got, label)
        say(f"  rc={got['rc']} total_iters={got['stats']['total_iters']} "
            f"failed={got['stats']['n_failed']} kernel_ms={got['stats']['kernel_ms']:.2f}")
    gm.close()


def test_noalloc_rejections(ctx):
    import torch
    m6 = synth.make_mech6()
    gm = ctx.mechanism(m6)
    T, P, Y = synth.make_cells_mech6(64, seed=3)
    # host arrays would need staging buffers: refused, nothing touched
    Th = T.copy()
    with pytest.raises(stev.StevError) as e:
        ctx.integrate_noalloc(gm, Th, P.copy(), Y.copy(), DT)
    assert e.value.code == stev.STEV_EINVAL
    assert np.array_equal(Th, T)
    # a field beyond the scratch array's capacity: refused before any launch
    n_max = ctx.noalloc_max_cells()
    assert n_max == 1 << 22
    Tt = torch.tensor(T, device="cuda")
    Pt = torch.tensor(P, device="cuda")
    Yt = torch.tensor(Y, device="cuda")
    st = stev.Stats()
    rc = ctx.lib.stev_integrate_noalloc(ctx.h, gm.h, n_max + 1, Tt.data_ptr(), Pt.data_ptr(),
                                        Yt.data_ptr(), 6, 1, DT, None, None, None, C.byref(st))
    assert rc == stev.STEV_EINVAL and "exceeds" in ctx.last_error()
    assert torch.equal(Tt.cpu(), torch.tensor(T))
    gm.close()
