"""Tiny hand-built mechanisms whose behaviour has a closed form.

Only inputs live here (coefficients and stoichiometry); expected values are
derived in the tests from mathematics, never from the code under test.
"""

import numpy as np

from paper_1905_09395_amd.synth import pack_mechanism

# a thermally inert NASA-7 set (constant cp/R = 3.5, zero formation terms)
FLAT = [3.5, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0]


def species_sets(n, a7=None, scale=None):
    lo = np.tile(np.array(FLAT), (n, 1))
    if scale is not None:
        for k, s in enumerate(scale):
            lo[k, :6] *= s
    if a7 is not None:
        lo[:, 6] = a7
    return lo, lo.copy()


def chain_abc(k1, k2, W=0.028):
    """A -> B -> C, first order, identical inert thermo, equal W (Sec 4, Eq 18)."""
    lo, hi = species_sets(3)
    rx = [dict(reac={0: 1.0}, prod={1: 1.0}, rev=False, A=k1, b=0.0, Ea=0.0),
          dict(reac={1: 1.0}, prod={2: 1.0}, rev=False, A=k2, b=0.0, Ea=0.0)]
    elem = np.zeros((3, 4), dtype=int)
    return pack_mechanism("abc", ["A", "B", "C"], elem, lo, hi, rx, W=np.full(3, W))


def decay_ab(k, W=0.028):
    """A -> B, first order."""
    lo, hi = species_sets(2)
    rx = [dict(reac={0: 1.0}, prod={1: 1.0}, rev=False, A=k, b=0.0, Ea=0.0)]
    elem = np.zeros((2, 4), dtype=int)
    return pack_mechanism("ab", ["A", "B"], elem, lo, hi, rx, W=np.full(2, W))


def order_n(k, order, nu=1.0, W=0.028):
    """nu A -> nu B with forward order `order` (Eq 28 empirical form)."""
    lo, hi = species_sets(2)
    rx = [dict(reac={0: nu}, prod={1: nu}, rev=False, forder={0: order}, A=k, b=0.0,
               Ea=0.0)]
    elem = np.zeros((2, 4), dtype=int)
    return pack_mechanism("ordn", ["A", "B"], elem, lo, hi, rx, W=np.full(2, W))


def iso_ab(kf, a7_A, a7_B, W=0.028):
    """A <=> B, species identical except the entropy constant a7 (Eqs 29-30)."""
    lo, hi = species_sets(2, a7=[a7_A, a7_B])
    rx = [dict(reac={0: 1.0}, prod={1: 1.0}, rev=True, A=kf, b=0.0, Ea=0.0)]
    elem = np.zeros((2, 4), dtype=int)
    return pack_mechanism("isoab", ["A", "B"], elem, lo, hi, rx, W=np.full(2, W))


def dissoc_a2b(kf, a7_A, a7_B, WA=0.032):
    """A <=> 2 B with W_A = 2 W_B and B's a1..a6 exactly half of A's (dH = 0)."""
    lo = np.tile(np.array([3.5, 1e-3, 0.0, 0.0, 0.0, -2000.0, a7_A]), (2, 1))
    lo[1, :6] *= 0.5
    lo[1, 6] = a7_B
    rx = [dict(reac={0: 1.0}, prod={1: 2.0}, rev=True, A=kf, b=0.0, Ea=0.0)]
    elem = np.zeros((2, 4), dtype=int)
    return pack_mechanism("a2b", ["A", "B"], elem, lo, lo.copy(), rx,
                          W=np.array([WA, WA / 2.0]))


def bfer_table1():
    """The paper's two-step BFER methane mechanism: kinetics from the cited
    fixture (Table 1 constants, Eqs 26-29 forms; cm-mol-s units, calories),
    on the synthetic NASA-7 thermo of the 6-species set (the paper prints no
    thermo data), N2 inert."""
    import json
    import os
    from paper_1905_09395_amd import synth
    with open(os.path.join(os.path.dirname(__file__), "golden", "bfer_table1.json")) as f:
        fx = json.load(f)
    m6 = synth.make_mech6()
    names = list(m6["species"])
    ix = {s: i for i, s in enumerate(names)}
    rx = []
    for name in ("MEPOX", "COROX"):
        r = fx["reactions"][name]
        rx.append(dict(reac={ix[s]: v for s, v in r["reactants"].items()},
                       prod={ix[s]: v for s, v in r["products"].items()},
                       rev=r["reversible"],
                       forder={ix[s]: v for s, v in r["orders"].items()},
                       A=r["k"], b=r["T_exponent"], Ea=r["Ea_cal_per_mol"] * 4.184))
    return pack_mechanism("bfer", names, m6["elem"], m6["nasa_lo"], m6["nasa_hi"], rx)
