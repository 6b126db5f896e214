"""FP64 CPU oracle for STEV -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  The GPU library never loads it.

The C sources (``stev_oracle.c``) implement the method literally; this module
only builds them with gcc and marshals numpy arrays through ctypes.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "stev_oracle.c")
_SRC_C3M = os.path.join(_HERE, "c3m_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# a mutated build of the same sources (tests/test_oracle_mutations.py) is
# loaded in a child process through this variable; nothing else sets it
_LIB_OVERRIDE = os.environ.get("STEV_ORACLE_LIB")
_lib = None


def build(force=True):
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra", "-o", _LIB + ".tmp",
           _SRC, _SRC_C3M, "-lm"]
    if force or not os.path.exists(_LIB):
        subprocess.check_call(cmd, cwd=_HERE)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Mech(C.Structure):
    _fields_ = [("n_s", C.c_int), ("n_r", C.c_int),
                ("W", C.c_void_p), ("nasa_lo", C.c_void_p), ("nasa_hi", C.c_void_p),
                ("T_mid", C.c_void_p), ("rxn_ptr", C.c_void_p), ("sp_idx", C.c_void_p),
                ("nu", C.c_void_p), ("order", C.c_void_p), ("A", C.c_void_p),
                ("b", C.c_void_p), ("Ea", C.c_void_p), ("rev", C.c_void_p),
                ("mlp_H", C.c_int), ("mlp_prm", C.c_void_p), ("mlp_mean", C.c_void_p),
                ("mlp_sd", C.c_void_p), ("mlp_T_lo", C.c_double), ("mlp_T_hi", C.c_double),
                ("ann_H", C.c_int), ("ann_prm", C.c_void_p), ("ann_T_lo", C.c_double),
                ("ann_T_hi", C.c_double)]


class _Params(C.Structure):
    _fields_ = [("ystep_max", C.c_double), ("delta_max", C.c_double),
                ("alpha", C.c_double), ("tol_ring", C.c_double),
                ("tol_freq", C.c_double), ("r_fac", C.c_double),
                ("rof_min", C.c_double), ("dft_window", C.c_int), ("stab_limit", C.c_int),
                ("max_iters", C.c_longlong), ("noise_eps", C.c_double),
                ("noise_seed", C.c_ulonglong)]


DEFAULT_PARAMS = dict(ystep_max=1e-3, delta_max=1e-2, alpha=1e-5, tol_ring=0.5,
                      tol_freq=1e-6, r_fac=2.0, rof_min=1e-12, dft_window=13,
                      stab_limit=0, max_iters=1_000_000, noise_eps=0.0, noise_seed=0)


C3M_NG, C3M_NS, C3M_NR, C3M_NVAR = 14, 4, 11, 26
C3M_GAS = ("CO", "CO2", "CH4", "H2", "H2O", "H2S", "C3H6", "HCN", "C2H4", "C2H6", "Tar", "O2",
           "SO3", "N2")
C3M_SOLID = ("CV", "CC", "CM", "CA")
C3M_REACTIONS = ("PYRO", "WGS", "STG", "CG", "MEG", "COX", "TOX", "COOX", "HOX", "MEOX", "MR")
C3M_VARS = ("T_g", "T_s", "P_g", "ep_g", "rho_g", "ep_s", "rho_s", "d_p")


class _C3M(C.Structure):
    _fields_ = [("A_pyro", C.c_double), ("Ea_pyro", C.c_double),
                ("A_wgs", C.c_double), ("Fp_wgs", C.c_double), ("Kf_wgs", C.c_double),
                ("Eaf_wgs", C.c_double), ("Kr_wgs", C.c_double), ("Ear_wgs", C.c_double),
                ("theta_G", C.c_double * 5), ("theta_C", C.c_double * 5),
                ("A_stg", C.c_double), ("Fp_stg", C.c_double), ("Ea_stg", C.c_double),
                ("A_cg", C.c_double), ("Fp_cg", C.c_double), ("Ea_cg", C.c_double),
                ("A_meg", C.c_double), ("Ea_meg", C.c_double), ("beta_c", C.c_double),
                ("A_cox", C.c_double), ("Ea_cox", C.c_double),
                ("A_tox", C.c_double), ("Ea_tox", C.c_double),
                ("A_coox", C.c_double), ("Ea_coox", C.c_double),
                ("A_hox", C.c_double), ("Ea_hox", C.c_double),
                ("A_meox", C.c_double), ("Ea_meox", C.c_double), ("A_mr", C.c_double),
                ("nu_pyro", C.c_double * 11), ("nu_tox", C.c_double * 5),
                ("W_g", C.c_double * 14), ("W_s", C.c_double * 4)]


class C3M:
    """C view of a C3M description (a dict as made by synth.make_c3m)."""

    def __init__(self, desc):
        self.desc = desc
        c = _C3M()
        for f, t in _C3M._fields_:
            v = desc[f]
            if hasattr(t, "_length_"):
                getattr(c, f)[:] = [float(x) for x in v]
            else:
                setattr(c, f, float(v))
        self.c = c


def lib():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            L = C.CDLL(_LIB_OVERRIDE)
        else:
            if not os.path.exists(_LIB):
                build()
            L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        L.orc_thermo.argtypes = [C.POINTER(_Mech), C.c_int, C.c_double, dp]
        L.orc_ystarstar.argtypes = [C.c_double, C.c_double]
        L.orc_ystarstar.restype = C.c_double
        L.orc_source.argtypes = [C.POINTER(_Mech), C.POINTER(_Params), C.c_double, C.c_double,
                                 dp, dp, dp, dp, dp, dp, dp]
        L.orc_jacobian_inf_norm.argtypes = [C.POINTER(_Mech), C.POINTER(_Params), C.c_double,
                                            C.c_double, dp, dp, dp]
        L.orc_jacobian_inf_norm.restype = C.c_double
        L.orc_step_size.argtypes = [C.POINTER(_Params), C.c_int, dp, dp, C.c_double, C.c_double]
        L.orc_step_size.restype = C.c_double
        L.orc_dft_mag.argtypes = [dp, C.c_int, dp]
        L.orc_ringing_eq.argtypes = [dp, C.c_int, C.POINTER(_Params), dp]
        L.orc_ringing_eq.restype = C.c_int
        L.orc_rof_next.argtypes = [C.c_double, C.c_int, C.POINTER(_Params)]
        L.orc_rof_next.restype = C.c_double
        L.orc_integrate_cell.argtypes = [C.POINTER(_Mech), C.POINTER(_Params), dp, C.c_double,
                                         dp, C.c_double, C.POINTER(C.c_longlong), dp, dp, dp,
                                         C.c_longlong]
        L.orc_integrate_cell.restype = C.c_int
        L.orc_integrate.argtypes = [C.POINTER(_Mech), C.POINTER(_Params), C.c_longlong, dp, dp,
                                    dp, C.c_longlong, C.c_double, C.POINTER(C.c_longlong),
                                    C.POINTER(C.c_ubyte), dp, dp, C.c_int, dp]
        L.orc_integrate.restype = C.c_int
        L.orc_nasa_targets.argtypes = [C.POINTER(_Mech), C.c_longlong, dp, dp, dp]
        L.orc_mlp_n_params.argtypes = [C.c_int, C.c_int]
        L.orc_mlp_n_params.restype = C.c_longlong
        L.orc_mlp_forward.argtypes = [C.c_int, C.c_int, dp, C.c_longlong, dp, dp]
        L.orc_ann_forward.argtypes = [C.c_int, C.c_int, dp, C.c_longlong, dp, dp]
        L.orc_mlp_loss_grad.argtypes = [C.c_int, C.c_int, dp, C.c_longlong, dp, dp, dp]
        L.orc_mlp_loss_grad.restype = C.c_double
        L.orc_adam_step.argtypes = [C.c_longlong, dp, dp, dp, dp, C.c_longlong, C.c_double,
                                    C.c_double, C.c_double, C.c_double]
        L.orc_c3m_anneal.argtypes = [C.POINTER(_C3M), C.c_double, C.c_double, dp, dp, dp]
        L.orc_c3m_rates.argtypes = [C.POINTER(_C3M), C.POINTER(_Params), dp, C.c_double,
                                    C.c_double, dp, dp, dp]
        L.orc_c3m_source.argtypes = [C.POINTER(_C3M), C.POINTER(_Params), dp, C.c_double,
                                     C.c_double, dp, dp, C.c_double, dp, dp, dp, dp, dp, dp]
        L.orc_c3m_integrate_cell.argtypes = [C.POINTER(_C3M), C.POINTER(_Params), dp,
                                             C.c_double, C.POINTER(C.c_longlong)]
        L.orc_c3m_integrate_cell.restype = C.c_int
        L.orc_c3m_integrate.argtypes = [C.POINTER(_C3M), C.POINTER(_Params), C.c_longlong, dp,
                                        C.c_longlong, C.c_double, C.POINTER(C.c_longlong),
                                        C.POINTER(C.c_ubyte), C.c_int]
        L.orc_c3m_integrate.restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class OracleMech:
    """Holds contiguous copies of a mechanism dict and the C view of them."""

    def __init__(self, mech):
        self.mech = mech
        self._keep = {
            "W": np.ascontiguousarray(mech["W"], dtype=np.float64),
            "nasa_lo": np.ascontiguousarray(mech["nasa_lo"], dtype=np.float64),
            "nasa_hi": np.ascontiguousarray(mech["nasa_hi"], dtype=np.float64),
            "T_mid": np.ascontiguousarray(mech["T_mid"], dtype=np.float64),
            "rxn_ptr": np.ascontiguousarray(mech["rxn_ptr"], dtype=np.int32),
            "sp_idx": np.ascontiguousarray(mech["sp_idx"], dtype=np.int32),
            "nu": np.ascontiguousarray(mech["nu"], dtype=np.float64),
            "order": np.ascontiguousarray(mech["order"], dtype=np.float64),
            "A": np.ascontiguousarray(mech["A"], dtype=np.float64),
            "b": np.ascontiguousarray(mech["b"], dtype=np.float64),
            "Ea": np.ascontiguousarray(mech["Ea"], dtype=np.float64),
            "rev": np.ascontiguousarray(mech["reversible"], dtype=np.uint8),
        }
        k = self._keep
        self.c = _Mech(int(mech["n_s"]), int(mech["n_r"]),
                       *[k[f].ctypes.data for f in ("W", "nasa_lo", "nasa_hi", "T_mid",
                                                    "rxn_ptr", "sp_idx", "nu", "order",
                                                    "A", "b", "Ea", "rev")])
        self.n_s = int(mech["n_s"])
        self.n_r = int(mech["n_r"])

    def with_network(self, H, prm, mean, sd, T_lo, T_hi):
        """A copy whose thermo (cp/R, h/R) comes from a network inside
        [T_lo, T_hi] (Sec 3): FP64 parameters in the orc_mlp_forward layout,
        z-score means and deviations [2 n_s] (cp/R first, then h/R)."""
        o = OracleMech(self.mech)
        o._keep.update(mlp_prm=np.ascontiguousarray(prm, dtype=np.float64),
                       mlp_mean=np.ascontiguousarray(mean, dtype=np.float64),
                       mlp_sd=np.ascontiguousarray(sd, dtype=np.float64))
        o.c.mlp_H = int(H)
        o.c.mlp_prm = o._keep["mlp_prm"].ctypes.data
        o.c.mlp_mean = o._keep["mlp_mean"].ctypes.data
        o.c.mlp_sd = o._keep["mlp_sd"].ctypes.data
        o.c.mlp_T_lo = float(T_lo)
        o.c.mlp_T_hi = float(T_hi)
        return o

    def with_ann(self, H, prm, T_lo, T_hi):
        """A copy whose thermo (cp/R, h/R) comes from the paper's sigmoid
        network inside [T_lo, T_hi] (Sec 3): FP64 parameters in the
        orc_ann_forward layout, outputs in physical units."""
        o = OracleMech(self.mech)
        o._keep.update(ann_prm=np.ascontiguousarray(prm, dtype=np.float64))
        o.c.ann_H = int(H)
        o.c.ann_prm = o._keep["ann_prm"].ctypes.data
        o.c.ann_T_lo = float(T_lo)
        o.c.ann_T_hi = float(T_hi)
        return o


def make_params(**kw):
    d = dict(DEFAULT_PARAMS)
    d.update(kw)
    return _Params(d["ystep_max"], d["delta_max"], d["alpha"], d["tol_ring"], d["tol_freq"],
                   d["r_fac"], d["rof_min"], int(d["dft_window"]), int(d["stab_limit"]),
                   int(d["max_iters"]),
                   float(d["noise_eps"]), int(d["noise_seed"]))


def thermo(om, k, T):
    out = np.zeros(3)
    lib().orc_thermo(C.byref(om.c), int(k), float(T), _p(out))
    return out


def ystarstar(y, alpha):
    return lib().orc_ystarstar(float(y), float(alpha))


def source(om, T, P, Y, rOF=None, **kw):
    """Returns dict(q, omega, dYdt, dTdt, rho) for one state."""
    prm = make_params(**kw)
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    rOF = np.ones(om.n_r) if rOF is None else np.ascontiguousarray(rOF, dtype=np.float64)
    q = np.zeros(om.n_r)
    om_ = np.zeros(om.n_s)
    dY = np.zeros(om.n_s)
    dT = np.zeros(1)
    rho = np.zeros(1)
    lib().orc_source(C.byref(om.c), C.byref(prm), float(T), float(P), _p(Y), _p(rOF), _p(q),
                     _p(om_), _p(dY), _p(dT), _p(rho))
    return dict(q=q, omega=om_, dYdt=dY, dTdt=float(dT[0]), rho=float(rho[0]))


def jacobian(om, T, P, Y, rOF=None, **kw):
    """(A, ||A||_inf): d(dY/dt)/dY at fixed T and rho (Section 4, Eqs 22-24)."""
    prm = make_params(**kw)
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    rOF = np.ones(om.n_r) if rOF is None else np.ascontiguousarray(rOF, dtype=np.float64)
    A = np.zeros((om.n_s, om.n_s))
    nrm = lib().orc_jacobian_inf_norm(C.byref(om.c), C.byref(prm), float(T), float(P), _p(Y),
                                      _p(rOF), _p(A))
    return A, nrm


def step_size(Y, dYdt, t, tf, **kw):
    prm = make_params(**kw)
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    dYdt = np.ascontiguousarray(dYdt, dtype=np.float64)
    return lib().orc_step_size(C.byref(prm), len(Y), _p(Y), _p(dYdt), float(t), float(tf))


def dft_mag(x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    D = np.zeros(len(x))
    lib().orc_dft_mag(_p(x), len(x), _p(D))
    return D


def ringing_eq(D, **kw):
    prm = make_params(**kw)
    D = np.ascontiguousarray(D, dtype=np.float64)
    mg = np.zeros(1)
    r = lib().orc_ringing_eq(_p(D), len(D), C.byref(prm), _p(mg))
    return bool(r), float(mg[0])


def rof_next(rof, ring_eq, **kw):
    prm = make_params(**kw)
    return lib().orc_rof_next(float(rof), int(bool(ring_eq)), C.byref(prm))


def integrate_cell(om, T, P, Y, tf, trace_cap=0, **kw):
    prm = make_params(**kw)
    Tb = np.array([float(T)])
    Yb = np.array(Y, dtype=np.float64).copy()
    it = C.c_longlong(0)
    md = np.zeros(1)
    my = np.zeros(1)
    tr = np.zeros(max(trace_cap, 1))
    st = lib().orc_integrate_cell(C.byref(om.c), C.byref(prm), _p(Tb), float(P), _p(Yb),
                                  float(tf), C.byref(it), _p(md), _p(my),
                                  _p(tr) if trace_cap else None, int(trace_cap))
    out = dict(T=float(Tb[0]), Y=Yb, iters=int(it.value), status=int(st),
               margin_dft=float(md[0]), margin_y=float(my[0]))
    if trace_cap:
        out["h"] = tr[:min(trace_cap, it.value)]
    return out


def integrate(om, T, P, Y, tf, nthreads=0, **kw):
    """Integrate all cells; returns dict(T, Y, iters, status, margin_dft, margin_y,
    margin_h) (the margins are diagnostics: see orc_integrate_cell_keyed)."""
    prm = make_params(**kw)
    T = np.array(T, dtype=np.float64).copy()
    P = np.ascontiguousarray(P, dtype=np.float64)
    Y = np.array(Y, dtype=np.float64).copy()
    n = len(T)
    iters = np.zeros(n, dtype=np.int64)
    status = np.zeros(n, dtype=np.uint8)
    md = np.zeros(n)
    my = np.zeros(n)
    mh = np.zeros(n)
    lib().orc_integrate(C.byref(om.c), C.byref(prm), n, _p(T), _p(P), _p(Y), Y.shape[1],
                        float(tf), iters.ctypes.data_as(C.POINTER(C.c_longlong)),
                        status.ctypes.data_as(C.POINTER(C.c_ubyte)), _p(md), _p(my),
                        int(nthreads), _p(mh))
    return dict(T=T, Y=Y, iters=iters, status=status, margin_dft=md, margin_y=my,
                margin_h=mh)


def nasa_targets(om, T):
    T = np.ascontiguousarray(T, dtype=np.float64)
    cp = np.zeros((len(T), om.n_s))
    h = np.zeros((len(T), om.n_s))
    lib().orc_nasa_targets(C.byref(om.c), len(T), _p(T), _p(cp), _p(h))
    return cp, h


def mlp_n_params(H, n_out):
    return int(lib().orc_mlp_n_params(H, n_out))


def mlp_forward(H, n_out, prm, x):
    prm = np.ascontiguousarray(prm, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.zeros((len(x), n_out))
    lib().orc_mlp_forward(H, n_out, _p(prm), len(x), _p(x), _p(y))
    return y


def ann_forward(H, n_out, prm, x):
    """The sigmoid network's outputs [n, n_out] at normalised inputs x."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.zeros((len(x), n_out))
    lib().orc_ann_forward(int(H), int(n_out), _p(np.ascontiguousarray(prm, dtype=np.float64)),
                          len(x), _p(x), _p(y))
    return y


def mlp_loss_grad(H, n_out, prm, x, target):
    prm = np.ascontiguousarray(prm, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    t = np.ascontiguousarray(target, dtype=np.float64)
    g = np.zeros_like(prm)
    loss = lib().orc_mlp_loss_grad(H, n_out, _p(prm), len(x), _p(x), _p(t), _p(g))
    return loss, g


def adam_step(prm, grad, m1, m2, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam update of prm, m1, m2 (float64 arrays)."""
    lib().orc_adam_step(len(prm), _p(prm), _p(np.ascontiguousarray(grad)), _p(m1), _p(m2),
                        int(step), lr, beta1, beta2, eps)


def c3m_anneal(c3, X_CC, X_CA):
    """Eqs 44-46: (vartheta, alpha_G, alpha_C)."""
    th, aG, aC = C.c_double(), C.c_double(), C.c_double()
    lib().orc_c3m_anneal(C.byref(c3.c), float(X_CC), float(X_CA), C.byref(th), C.byref(aG),
                         C.byref(aC))
    return th.value, aG.value, aC.value


def _c3m_split(cell, ROP_g=None, ROP_s=None):
    cell = np.ascontiguousarray(cell, dtype=np.float64)
    ROP_g = cell[3] * cell[4] if ROP_g is None else ROP_g
    ROP_s = cell[5] * cell[6] if ROP_s is None else ROP_s
    Xg = np.ascontiguousarray(cell[8:22])
    Xs = np.ascontiguousarray(cell[22:26])
    return cell, float(ROP_g), float(ROP_s), Xg, Xs


def c3m_rates(c3, cell, ROP_g=None, ROP_s=None, **kw):
    """Eqs 42-56 at one 26-value cell state: r[11] (kmol/m^3/s)."""
    prm = make_params(**kw)
    cell, Rg, Rs, Xg, Xs = _c3m_split(cell, ROP_g, ROP_s)
    r = np.zeros(C3M_NR)
    lib().orc_c3m_rates(C.byref(c3.c), C.byref(prm), _p(cell), Rg, Rs, _p(Xg), _p(Xs), _p(r))
    return r


def c3m_source(c3, cell, rof=1.0, ROP_g=None, ROP_s=None, **kw):
    """dict(r, dXg, dXs, dROPg, dROPs, src) at one cell state (src: the
    species mass sources W_k omega_k, gas then solids)."""
    prm = make_params(**kw)
    cell, Rg, Rs, Xg, Xs = _c3m_split(cell, ROP_g, ROP_s)
    r = np.zeros(C3M_NR)
    dXg = np.zeros(C3M_NG)
    dXs = np.zeros(C3M_NS)
    dRg = np.zeros(1)
    dRs = np.zeros(1)
    src = np.zeros(C3M_NG + C3M_NS)
    lib().orc_c3m_source(C.byref(c3.c), C.byref(prm), _p(cell), Rg, Rs, _p(Xg), _p(Xs),
                         float(rof), _p(r), _p(dXg), _p(dXs), _p(dRg), _p(dRs), _p(src))
    return dict(r=r, dXg=dXg, dXs=dXs, dROPg=float(dRg[0]), dROPs=float(dRs[0]), src=src)


def c3m_integrate(c3, state, tf, nthreads=0, **kw):
    """Integrate cells [n, 26] over tf; returns dict(state, iters, status)."""
    prm = make_params(**kw)
    st = np.array(state, dtype=np.float64).copy()
    n = st.shape[0]
    iters = np.zeros(n, dtype=np.int64)
    status = np.zeros(n, dtype=np.uint8)
    lib().orc_c3m_integrate(C.byref(c3.c), C.byref(prm), n, _p(st), st.shape[1], float(tf),
                            iters.ctypes.data_as(C.POINTER(C.c_longlong)),
                            status.ctypes.data_as(C.POINTER(C.c_ubyte)), int(nthreads))
    return dict(state=st, iters=iters, status=status)
