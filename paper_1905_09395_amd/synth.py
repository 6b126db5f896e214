"""Seeded synthetic inputs: chemical mechanisms and cell fields.

This module only *generates inputs*.  It contains no step of the integration
method (no rates, no step-size rule, no Euler update, no DFT).  Both the FP64
CPU oracle and the GPU library read the arrays produced here, so it must stay
free of the method's arithmetic.

A mechanism is a plain ``dict`` of numpy arrays:

``species``     list of names, length ``n_s``
``elem``        int array ``[n_s, 4]`` atoms of C, H, O, N per species
``W``           molar masses, kg/mol
``nasa_lo``     ``[n_s, 7]`` NASA-7 coefficients a1..a7 below ``T_mid``
``nasa_hi``     ``[n_s, 7]`` NASA-7 coefficients a1..a7 at/above ``T_mid``
``T_lo``, ``T_mid``, ``T_hi``  per-species ranges (K)
``rxn_ptr``     int32 ``[n_r+1]``: participants of reaction j are
                ``rxn_ptr[j]:rxn_ptr[j+1]``
``sp_idx``      int32 participant species index
``nu``          float64 signed net stoichiometric coefficient (<0 reactant)
``order``       float64 rate order: forward order for reactants, reverse
                order for products of reversible reactions (0 otherwise)
``A``           pre-exponential factor in cm-mol-s units (Table 1 units)
``b``           temperature exponent
``Ea``          activation energy, J/mol
``reversible``  uint8 per reaction

The NASA-7 coefficient sets are built from cp(T) polynomials: the low set is
drawn, the high set's a1 is chosen so cp is continuous at ``T_mid`` and the
integration constants a6/a7 are chosen (with ``numpy.polynomial``) so that
h(298.15 K) and s(298.15 K) hit drawn formation values and h, s are
continuous at ``T_mid``.  Formation enthalpies and entropies follow a crude
group-additivity rule plus noise, and every reversible reaction is oriented
exothermic at 298 K, so that reverse barriers are never negative.
"""

from __future__ import annotations

import itertools
import json
import math
import os

import numpy as np
from numpy.polynomial import Polynomial

ELEMENTS = ("C", "H", "O", "N")
ATOMIC_MASS_G = np.array([12.011, 1.008, 15.999, 14.007])  # g/mol
P_ATM = 101325.0
T_REF = 298.15
T_LO, T_MID, T_HI = 300.0, 1000.0, 3000.0

FORMULAS = {
    "CH4": (1, 4, 0, 0), "O2": (0, 0, 2, 0), "CO": (1, 0, 1, 0),
    "CO2": (1, 0, 2, 0), "H2O": (0, 2, 1, 0), "N2": (0, 0, 0, 2),
    "H2": (0, 2, 0, 0),
}


def molar_mass(elem):
    """kg/mol from atom counts (C, H, O, N)."""
    return (np.asarray(elem, dtype=np.float64) @ ATOMIC_MASS_G) / 1000.0


# ----------------------------------------------------------------------------
# thermo coefficient synthesis
# ----------------------------------------------------------------------------

def _cp_poly(a):
    return Polynomial(list(a[:5]))


def _h_R(a):
    """h/R as a polynomial in T plus the constant a6 (library integration)."""
    return _cp_poly(a).integ() + a[5]


def _s_R_nolog(a):
    """s/R minus a1*ln(T): integral of (cp/R - a1)/T, plus a7."""
    q = Polynomial(list(a[1:5]))  # (cp/R - a1)/T
    return q.integ() + a[6]


def _nasa_pair(rng, hf_R, s0_R, Tmid=T_MID):
    """Draw one species' low/high NASA-7 sets.

    cp/R stays within [1.5, 12] over [T_LO, T_HI]; cp, h and s are continuous
    at Tmid; h(298.15)/R = hf_R and s(298.15)/R = s0_R.
    """
    grid_lo = np.linspace(T_LO, Tmid, 64)
    grid_hi = np.linspace(Tmid, T_HI, 128)
    for _ in range(10000):
        lo = np.zeros(7)
        lo[0] = rng.uniform(2.5, 4.5)
        lo[1] = rng.uniform(0.0, 4e-3)
        lo[2] = rng.uniform(-1e-6, 1e-6)
        lo[3] = rng.uniform(-2e-10, 2e-10)
        lo[4] = rng.uniform(-2e-14, 2e-14)
        hi = np.zeros(7)
        hi[1] = rng.uniform(0.0, 2e-3)
        hi[2] = rng.uniform(-2e-7, 2e-7)
        hi[3] = rng.uniform(-2e-11, 2e-11)
        hi[4] = rng.uniform(-1e-15, 1e-15)
        hi[0] = _cp_poly(lo)(Tmid) - (_cp_poly(hi)(Tmid) - 0.0)
        cl = _cp_poly(lo)(grid_lo)
        ch = _cp_poly(hi)(grid_hi)
        if cl.min() >= 1.5 and ch.min() >= 1.5 and cl.max() <= 12 and ch.max() <= 12:
            break
    else:  # pragma: no cover
        raise RuntimeError("NASA-7 rejection sampling failed")
    # integration constants: h(Tref) and s(Tref) at the drawn formation values
    lo[5] = hf_R - (_h_R(lo)(T_REF) - lo[5])
    lo[6] = s0_R - (lo[0] * math.log(T_REF) + _s_R_nolog(lo)(T_REF) - lo[6])
    # continuity of h and s at Tmid
    hi[5] = 0.0
    hi[5] = _h_R(lo)(Tmid) - _h_R(hi)(Tmid)
    hi[6] = 0.0
    hi[6] = (lo[0] * math.log(Tmid) + _s_R_nolog(lo)(Tmid)) - (
        hi[0] * math.log(Tmid) + _s_R_nolog(hi)(Tmid))
    return lo, hi


def _formation(rng, elem, hf_range=(-3e4, 3e4)):
    """Formation enthalpy/R (K) and standard entropy/R for a species."""
    n_atoms = int(np.sum(elem))
    s0 = 14.0 + 2.5 * n_atoms + rng.uniform(-2.0, 2.0)
    hf = rng.uniform(*hf_range)
    return hf, s0


def _reaction_dH_R(nasa_lo, reac, prod):
    """Reaction enthalpy/R at 298.15 K from the synthesized sets."""
    h = 0.0
    for k, n in prod.items():
        h += n * _h_R(nasa_lo[k])(T_REF)
    for k, n in reac.items():
        h -= n * _h_R(nasa_lo[k])(T_REF)
    return h


def _arrhenius(rng, A_range=(1e8, 1e14), b_range=(-1.0, 1.0), Ea_kJ=(80.0, 200.0)):
    A = math.exp(rng.uniform(math.log(A_range[0]), math.log(A_range[1])))
    b = rng.uniform(*b_range)
    Ea = rng.uniform(*Ea_kJ) * 1000.0
    return A, b, Ea


# ----------------------------------------------------------------------------
# mechanism packing
# ----------------------------------------------------------------------------

def pack_mechanism(name, species, elem, nasa_lo, nasa_hi, reactions, W=None,
                   T_mid=None):
    """Pack a list of reaction dicts into the CSR mechanism dict.

    Each reaction dict has ``reac`` {k: nu}, ``prod`` {k: nu}, ``A``, ``b``,
    ``Ea``, ``rev`` and optionally ``forder`` {k: order} (forward orders of
    the reactants; default mass action).  Reversible reactions use mass-action
    reverse orders (the product coefficients).
    """
    elem = np.asarray(elem, dtype=np.int64).reshape(len(species), 4)
    n_s = len(species)
    rxn_ptr = [0]
    sp_idx, nu, order = [], [], []
    A, b, Ea, rev = [], [], [], []
    for r in reactions:
        forder = r.get("forder", None) or {k: float(v) for k, v in r["reac"].items()}
        for k, v in r["reac"].items():
            sp_idx.append(k)
            nu.append(-float(v))
            order.append(float(forder[k]))
        for k, v in r["prod"].items():
            sp_idx.append(k)
            nu.append(float(v))
            order.append(float(v) if r["rev"] else 0.0)
        rxn_ptr.append(len(sp_idx))
        A.append(r["A"])
        b.append(r["b"])
        Ea.append(r["Ea"])
        rev.append(1 if r["rev"] else 0)
    mech = {
        "name": name,
        "species": list(species),
        "elem": elem,
        "W": molar_mass(elem) if W is None else np.asarray(W, dtype=np.float64),
        "nasa_lo": np.asarray(nasa_lo, dtype=np.float64).reshape(n_s, 7),
        "nasa_hi": np.asarray(nasa_hi, dtype=np.float64).reshape(n_s, 7),
        "T_lo": np.full(n_s, T_LO),
        "T_mid": np.full(n_s, T_MID) if T_mid is None else np.asarray(T_mid, dtype=np.float64),
        "T_hi": np.full(n_s, T_HI),
        "rxn_ptr": np.asarray(rxn_ptr, dtype=np.int32),
        "sp_idx": np.asarray(sp_idx, dtype=np.int32),
        "nu": np.asarray(nu, dtype=np.float64),
        "order": np.asarray(order, dtype=np.float64),
        "A": np.asarray(A, dtype=np.float64),
        "b": np.asarray(b, dtype=np.float64),
        "Ea": np.asarray(Ea, dtype=np.float64),
        "reversible": np.asarray(rev, dtype=np.uint8),
    }
    mech["n_s"] = n_s
    mech["n_r"] = len(reactions)
    return mech


# ----------------------------------------------------------------------------
# the three synthetic mechanisms
# ----------------------------------------------------------------------------

def make_mech6(seed=11):
    """6-species / 4-reaction global methane mechanism (BFER-like forms).

    Species CH4, O2, CO, CO2, H2O, N2 (N2 inert).  R1 is the Eq 28 form with
    empirical orders 0.5/0.65; R2 the reversible CO oxidation of Eq 29;
    R3 a reversible mass-action total oxidation; R4 an irreversible
    CH4 + 3 CO2 -> 4 CO + 2 H2O.  Arrhenius data are drawn:
    A ~ logU[1e8, 1e14] (cm-mol-s), b ~ U[-1, 1], Ea ~ U[80, 200] kJ/mol.
    """
    rng = np.random.default_rng(seed)
    names = ["CH4", "O2", "CO", "CO2", "H2O", "N2"]
    elem = np.array([FORMULAS[s] for s in names])
    hf_brackets = {"CH4": (-1.2e4, -0.6e4), "CO": (-1.6e4, -1.0e4),
                   "CO2": (-5e4, -4.4e4), "H2O": (-3.2e4, -2.6e4)}
    lo, hi = [], []
    for s, e in zip(names, elem):
        hf, s0 = _formation(rng, e)
        hf = 0.0 if s in ("O2", "N2") else rng.uniform(*hf_brackets[s])
        a_lo, a_hi = _nasa_pair(rng, hf, s0)
        lo.append(a_lo)
        hi.append(a_hi)
    CH4, O2, CO, CO2, H2O, N2 = range(6)
    rx = []
    A, b, Ea = _arrhenius(rng)
    rx.append(dict(reac={CH4: 1.0, O2: 1.5}, prod={CO: 1.0, H2O: 2.0}, rev=False,
                   forder={CH4: 0.5, O2: 0.65}, A=A, b=b, Ea=Ea))
    A, b, Ea = _arrhenius(rng)
    rx.append(dict(reac={CO: 1.0, O2: 0.5}, prod={CO2: 1.0}, rev=True, A=A, b=b, Ea=Ea))
    A, b, Ea = _arrhenius(rng)
    rx.append(dict(reac={CH4: 1.0, O2: 2.0}, prod={CO2: 1.0, H2O: 2.0}, rev=True,
                   A=A, b=b, Ea=Ea))
    A, b, Ea = _arrhenius(rng)
    rx.append(dict(reac={CH4: 1.0, CO2: 3.0}, prod={CO: 4.0, H2O: 2.0}, rev=False,
                   forder={CH4: 1.0, CO2: 1.0}, A=A, b=b, Ea=Ea))
    return pack_mechanism("mech6", names, elem, lo, hi, rx)


def _random_formulas(rng, n, exclude):
    """n distinct C_cH_hO_oN_n formulas, c<=2, h<=4, o<=3, n<=1, 1..7 atoms."""
    pool = []
    for c, h, o, nn in itertools.product(range(3), range(5), range(4), range(2)):
        atoms = c + h + o + nn
        if 1 <= atoms <= 7 and (c, h, o, nn) not in exclude:
            pool.append((c, h, o, nn))
    idx = rng.choice(len(pool), size=n, replace=False)
    return [pool[i] for i in idx]


def _formula_name(f):
    s = ""
    for sym, cnt in zip(ELEMENTS, f):
        if cnt:
            s += sym + (str(cnt) if cnt > 1 else "")
    return s


C_REF_CGS = 8.0e-6  # mol/cm^3, about 1 atm at 1500 K
ETA_MOL = 3.0e4     # K, per-molecule formation-enthalpy term (random mechanisms)
ETA_C = -1.3e4      # K, extra per carbon atom


def make_random_mechanism(n_species, n_reactions, seed, name=None,
                          A_range=(1e8, 1e14), Ea_kJ=(80.0, 200.0)):
    """Random element-balanced, all-reversible mass-action mechanism.

    Species: O2, H2, N2, CO and random C/H/O/N formulas.  Reactions: pairs of
    distinct multisets (size 1-3) with equal element vectors and disjoint
    species; every species appears in at least one reaction; each reaction is
    oriented exothermic at 298 K.

    A is drawn log-uniform in ``A_range`` as a bimolecular cm-mol-s value and
    then carried to the reaction's forward order m by ``C_REF_CGS**(2-m)``, so
    that uni-, bi- and termolecular steps have comparable pseudo-first-order
    rates at about 1 atm (a unimolecular step with a bimolecular-sized A would
    be unphysically fast).
    """
    rng = np.random.default_rng(seed)
    base = ["O2", "H2", "N2", "CO"]
    fixed = [FORMULAS[s] for s in base]
    for attempt in range(200):
        forms = fixed + _random_formulas(rng, n_species - 4, set(fixed))
        elem = np.array(forms, dtype=np.int64)
        # multisets of size 1..3 grouped by element vector
        groups = {}
        for size in (1, 2, 3):
            for ms in itertools.combinations_with_replacement(range(n_species), size):
                key = tuple(elem[list(ms)].sum(axis=0))
                groups.setdefault(key, []).append(ms)
        cands = []
        for key, lst in groups.items():
            if len(lst) < 2:
                continue
            for a, c in itertools.combinations(lst, 2):
                if set(a) & set(c):
                    continue
                cands.append((a, c))
        if len(cands) < n_reactions:
            continue
        cover = set()
        for a, c in cands:
            cover |= set(a) | set(c)
        if len(cover) < n_species:
            continue
        order = rng.permutation(len(cands))
        chosen, used = [], set()
        # first pass: cover every species
        for sp in rng.permutation(n_species):
            if sp in used:
                continue
            for i in order:
                a, c = cands[i]
                if sp in a or sp in c:
                    if (a, c) not in chosen:
                        chosen.append((a, c))
                        used |= set(a) | set(c)
                    break
        for i in order:
            if len(chosen) >= n_reactions:
                break
            if cands[i] not in chosen:
                chosen.append(cands[i])
        if len(chosen) == n_reactions and len(used) == n_species:
            break
    else:  # pragma: no cover
        raise RuntimeError("mechanism generation failed")
    names = base + [_formula_name(f) for f in forms[4:]]
    lo, hi = [], []
    for s, e in zip(names, elem):
        hf, s0 = _formation(rng, e)
        # bond-count enthalpy: each molecule costs ETA_MOL, each atom returns
        # ETA_MOL/2 (so O2, H2, N2 sit at zero), carbon a bit more, plus noise;
        # association steps are then exothermic, as their entropy loss demands
        hf = ETA_MOL * (1.0 - 0.5 * float(np.sum(e))) + ETA_C * e[0] + rng.uniform(-1e4, 1e4)
        if s in ("O2", "H2", "N2"):
            hf = 0.0
        elif s == "CO":
            hf = rng.uniform(-1.6e4, -1.0e4)
        a_lo, a_hi = _nasa_pair(rng, hf, s0)
        lo.append(a_lo)
        hi.append(a_hi)
    lo = np.array(lo)
    rx = []
    for a, c in chosen:
        reac = {}
        for k in a:
            reac[k] = reac.get(k, 0.0) + 1.0
        prod = {}
        for k in c:
            prod[k] = prod.get(k, 0.0) + 1.0
        if _reaction_dH_R(lo, reac, prod) > 0.0:
            reac, prod = prod, reac
        A, b, Ea = _arrhenius(rng, A_range=A_range, Ea_kJ=Ea_kJ)
        m_f = sum(reac.values())
        A = A * C_REF_CGS ** (2.0 - m_f)
        rx.append(dict(reac=reac, prod=prod, rev=True, A=A, b=b, Ea=Ea))
    return pack_mechanism(name or f"mech{n_species}", names, elem, lo, np.array(hi), rx)


def make_mech19(seed=12):
    """19 species over C, H, O, N; 50 reversible mass-action reactions."""
    return make_random_mechanism(19, 50, seed, name="mech19")


def make_mech53(seed=13):
    """53 species; 325 reversible mass-action reactions."""
    return make_random_mechanism(53, 325, seed, name="mech53")


# ----------------------------------------------------------------------------
# cell fields
# ----------------------------------------------------------------------------

def make_cells_mech6(n=1024, seed=101):
    """T ~ U[1200, 2200] K, P = 1 atm, Y = 0.5 Dir(1^6) + 0.5 e_N2."""
    rng = np.random.default_rng(seed)
    T = rng.uniform(1200.0, 2200.0, n)
    Y = 0.5 * rng.dirichlet(np.ones(6), n)
    Y[:, 5] += 0.5
    P = np.full(n, P_ATM)
    return T, P, Y


def make_cells_split(n, n_s, seed, hot_frac=0.3, cold=(300.0, 900.0), hot=(1400.0, 2500.0)):
    """(1-hot_frac) cells with T ~ U[cold], hot_frac with T ~ U[hot]; Y ~ Dir(1)."""
    rng = np.random.default_rng(seed)
    n_hot = int(round(hot_frac * n))
    T = np.empty(n)
    perm = rng.permutation(n)
    T[perm[:n_hot]] = rng.uniform(*hot, n_hot)
    T[perm[n_hot:]] = rng.uniform(*cold, n - n_hot)
    Y = rng.dirichlet(np.ones(n_s), n)
    P = np.full(n, P_ATM)
    return T, P, Y


def make_cells_mech19(n=262144, seed=102):
    return make_cells_split(n, 19, seed)


def batch_sizes(n_batches=64, lo=256, hi=131072, seed=103):
    """Log-uniform batch sizes in [lo, hi]."""
    rng = np.random.default_rng(seed)
    return np.round(np.exp(rng.uniform(math.log(lo), math.log(hi), n_batches))).astype(np.int64)


def subsample(n, k, seed):
    """Seeded sorted subsample of k indices out of n."""
    rng = np.random.default_rng(seed)
    if k >= n:
        return np.arange(n)
    return np.sort(rng.choice(n, size=k, replace=False))


def make_batches(n_batches=64, lo=256, hi=131072, seed=103):
    """Independent cell batches of log-uniform sizes; even batches are
    6-species cells, odd batches 19-species cells.  Returns a list of
    (mechanism key 6|19, T, P, Y)."""
    sizes = batch_sizes(n_batches, lo, hi, seed)
    out = []
    for b, n in enumerate(sizes):
        s = seed * 1000 + b
        if b % 2 == 0:
            out.append((6,) + make_cells_mech6(int(n), seed=s))
        else:
            out.append((19,) + make_cells_mech19(int(n), seed=s))
    return out


# ---------------------------------------------------------------------------
# Multiphase coal gasification (Sec 7.2): the C3M description and cell fields
# ---------------------------------------------------------------------------
C3M_GAS = ("CO", "CO2", "CH4", "H2", "H2O", "H2S", "C3H6", "HCN", "C2H4", "C2H6", "Tar", "O2",
           "SO3", "N2")
C3M_SOLID = ("CV", "CC", "CM", "CA")
# element masses (kg/kmol) whose sums give the molar masses printed in
# Eqs 47-50 to their printed digits
ELEMENT_MASS = {"C": 12.011, "H": 1.00794, "O": 15.9994, "N": 14.0067, "S": 32.065}
C3M_FORMULA = {"CO": {"C": 1, "O": 1}, "CO2": {"C": 1, "O": 2}, "CH4": {"C": 1, "H": 4},
               "H2": {"H": 2}, "H2O": {"H": 2, "O": 1}, "H2S": {"H": 2, "S": 1},
               "C3H6": {"C": 3, "H": 6}, "HCN": {"H": 1, "C": 1, "N": 1},
               "C2H4": {"C": 2, "H": 4}, "C2H6": {"C": 2, "H": 6}, "O2": {"O": 2},
               "SO3": {"S": 1, "O": 3}, "N2": {"N": 2}}
# ash takes part in no reaction; its molar mass (silica's) only labels it
ASH_MOLAR_MASS = 60.0843
C3M_TABLE2 = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                          "tests", "golden", "c3m_table2.json")


def _formula_mass(f):
    return sum(ELEMENT_MASS[e] * n for e, n in f.items())


def c3m_compositions(desc):
    """Element content (kmol per kmol) of every species, the pseudo-species
    included: tar from the atom balance of Eq 37, volatile matter from that
    of Eq 31, fixed carbon C, moisture H2O, ash none."""
    comp = {k: dict(C3M_FORMULA[k]) for k in C3M_FORMULA}
    nt = dict(zip(("O2", "CO2", "H2O", "SO3", "N2"), desc["nu_tox"]))
    tar = {}
    for sp, n in nt.items():
        for e, a in C3M_FORMULA[sp].items():
            tar[e] = tar.get(e, 0.0) + n * a
    comp["Tar"] = tar
    cv = {}
    for sp, n in zip(C3M_GAS[:11], desc["nu_pyro"]):
        for e, a in comp[sp].items():
            cv[e] = cv.get(e, 0.0) + n * a
    comp["CV"] = cv
    comp["CC"] = {"C": 1}
    comp["CM"] = {"H": 2, "O": 1}
    comp["CA"] = {}
    return comp


def make_c3m(table2_path=C3M_TABLE2):
    """The C3M gasification chemistry with the paper's constants (Table 2,
    Eqs 31 and 37).  Molar masses follow from the element masses; those of
    the pseudo-species tar and volatile matter from the atom balances of
    Eqs 37 and 31, so every reaction conserves mass exactly."""
    with open(table2_path) as f:
        g = json.load(f)
    t = g["table2"]
    desc = dict(A_pyro=t["A_PYRO"], Ea_pyro=t["Ea_PYRO"],
                A_wgs=t["A_WGS"], Fp_wgs=t["F_P_WGS"], Kf_wgs=t["K_F_WGS"],
                Eaf_wgs=t["Ea_F_WGS"], Kr_wgs=t["K_R_WGS"], Ear_wgs=t["Ea_R_WGS"],
                theta_G=[t[f"theta{i}_G"] for i in range(5)],
                theta_C=[t[f"theta{i}_C"] for i in range(5)],
                A_stg=t["A_STG"], Fp_stg=t["F_P_STG"], Ea_stg=t["Ea_STG"],
                A_cg=t["A_CG"], Fp_cg=t["F_P_CG"], Ea_cg=t["Ea_CG"],
                A_meg=t["A_MEG"], Ea_meg=t["Ea_MEG"], beta_c=t["beta_c"],
                A_cox=t["A_COX"], Ea_cox=t["Ea_COX"], A_tox=t["A_TOX"], Ea_tox=t["Ea_TOX"],
                A_coox=t["A_COOX"], Ea_coox=t["Ea_COOX"], A_hox=t["A_HOX"], Ea_hox=t["Ea_HOX"],
                A_meox=t["A_MEOX"], Ea_meox=t["Ea_MEOX"], A_mr=t["A_MR"])
    py = g["eq31_pyrolysis_products_per_CV"]
    desc["nu_pyro"] = [py[k] for k in C3M_GAS[:11]]
    tx = g["eq37_tar_oxidation_per_Tar"]
    desc["nu_tox"] = [tx[k] for k in ("O2", "CO2", "H2O", "SO3", "N2")]
    comp = c3m_compositions(desc)
    W = {k: _formula_mass(comp[k]) for k in C3M_GAS}
    desc["W_g"] = [W[k] for k in C3M_GAS]
    desc["W_s"] = [_formula_mass(comp["CV"]), ELEMENT_MASS["C"], W["H2O"], ASH_MOLAR_MASS]
    return desc


R_KMOL = 8314.46261815324   # J/(kmol K)


def make_c3m_cells(n=262144, seed=108, desc=None):
    """Random gasifier states, 26 values per cell (T_g, T_s, P_g, ep_g, rho_g,
    ep_s, rho_s, d_p, X_g[14], X_s[4]; K, Pa, kg/m^3, m):
    T_g ~ U[900, 1400] K, T_s = T_g + U[-50, 50] K, P_g ~ U[1, 15] atm,
    ep_s ~ U[0.02, 0.3], ep_g = 1 - ep_s, rho_s ~ U[900, 1400] kg/m^3,
    d_p log-uniform in [50, 500] um, X_g ~ Dirichlet(1) over the 14 gas
    species, X_s = 0.1 ash + 0.9 Dirichlet(1) over the 4 solids, and rho_g
    from the ideal gas at T_g, P_g."""
    desc = desc or make_c3m()
    rng = np.random.default_rng(seed)
    st = np.zeros((n, 26))
    Tg = rng.uniform(900.0, 1400.0, n)
    st[:, 0] = Tg
    st[:, 1] = Tg + rng.uniform(-50.0, 50.0, n)
    st[:, 2] = rng.uniform(1.0, 15.0, n) * 101325.0
    eps = rng.uniform(0.02, 0.3, n)
    st[:, 5] = eps
    st[:, 3] = 1.0 - eps
    st[:, 6] = rng.uniform(900.0, 1400.0, n)
    st[:, 7] = np.exp(rng.uniform(np.log(50e-6), np.log(500e-6), n))
    Xg = rng.dirichlet(np.ones(14), n)
    Xs = 0.9 * rng.dirichlet(np.ones(4), n)
    Xs[:, 3] += 0.1
    st[:, 8:22] = Xg
    st[:, 22:26] = Xs
    mw = 1.0 / (Xg / np.asarray(desc["W_g"])).sum(axis=1)
    st[:, 4] = st[:, 2] * mw / (R_KMOL * Tg)
    return st
