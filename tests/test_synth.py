"""The seeded synthetic inputs follow their stated recipe (no GPU): the
mechanisms are element-balanced with the stated sizes and reversibility, the
NASA-7 sets keep cp/R in the accepted band and are continuous at T_mid, and
the fields and batch sizes have the stated shapes and ranges."""

import numpy as np
import pytest

from paper_1905_09395_amd import synth


def _cp_R(a, T):
    return a[0] + a[1] * T + a[2] * T ** 2 + a[3] * T ** 3 + a[4] * T ** 4


@pytest.mark.parametrize("make,n_s,n_r,all_rev", [
    (synth.make_mech6, 6, 4, False), (synth.make_mech19, 19, 50, True),
    (synth.make_mech53, 53, 325, True)])
def test_mechanisms_are_element_balanced(make, n_s, n_r, all_rev):
    m = make()
    assert m["n_s"] == n_s and m["n_r"] == n_r
    elem = np.asarray(m["elem"], dtype=np.float64)
    ptr = m["rxn_ptr"]
    used = np.zeros(n_s, bool)
    for j in range(n_r):
        sl = slice(ptr[j], ptr[j + 1])
        sp, nu = np.asarray(m["sp_idx"][sl]), np.asarray(m["nu"][sl], dtype=np.float64)
        # element balance and hence mass balance (W is the element sum)
        np.testing.assert_allclose(nu @ elem[sp], 0.0, atol=1e-12)
        assert abs(float(nu @ np.asarray(m["W"])[sp])) < 1e-12
        used[sp] = True
    if all_rev:
        assert np.all(m["reversible"]) and used.all()


@pytest.mark.parametrize("make", [synth.make_mech6, synth.make_mech19, synth.make_mech53])
def test_nasa_sets_in_band_and_continuous(make):
    m = make()
    T = np.linspace(300.0, 3000.0, 271)
    for k in range(m["n_s"]):
        lo, hi, tm = m["nasa_lo"][k], m["nasa_hi"][k], m["T_mid"][k]
        cp = np.where(T < tm, _cp_R(lo, T), _cp_R(hi, T))
        assert cp.min() >= 2.0 - 1e-9 and cp.max() <= 25.0 + 1e-9, k
        assert _cp_R(lo, tm) == pytest.approx(_cp_R(hi, tm), rel=1e-9), k


def test_fields_and_batches_have_the_stated_shape():
    T, P, Y = synth.make_cells_mech19(8192)
    hot = T >= 1400.0
    assert np.all((T >= 300.0) & (T <= 2500.0)) and np.all(hot | (T <= 900.0))
    assert abs(hot.mean() - 0.3) < 0.02
    assert np.all(P == 101325.0) and Y.shape == (8192, 19)
    assert np.all(Y >= 0.0) and np.abs(Y.sum(axis=1) - 1.0).max() < 1e-12
    T6, P6, Y6 = synth.make_cells_mech6(1024, seed=101)
    assert np.all((T6 >= 1200.0) & (T6 <= 2200.0)) and Y6.shape == (1024, 6)
    # half of every cell is N2 (the last species)
    assert np.all(Y6[:, 5] >= 0.5 - 1e-12)
    sizes = synth.batch_sizes(64, 256, 131072, seed=103)
    assert len(sizes) == 64 and sizes.min() >= 256 and sizes.max() <= 131072


def test_c3m_cells_are_consistent_gas_solid_states():
    st = synth.make_c3m_cells(2048, seed=108)
    assert st.shape == (2048, 26)
    # volume fractions add to one; each phase's mass fractions add to one
    np.testing.assert_allclose(st[:, 3] + st[:, 5], 1.0, atol=1e-15)
    np.testing.assert_allclose(st[:, 8:22].sum(axis=1), 1.0, atol=1e-12)
    np.testing.assert_allclose(st[:, 22:26].sum(axis=1), 1.0, atol=1e-12)
    assert np.all(st[:, 8:26] >= 0.0) and np.all(st[:, [0, 1, 2, 4, 6, 7]] > 0.0)
