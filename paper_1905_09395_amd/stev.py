"""ctypes binding of libstev.so (argument marshalling only).

Every step of the integration runs in the library's HIP kernels; this module
never computes any part of the method.  If the compiled library is missing,
loading fails loudly -- there is no CPU fallback.

Arrays may be torch tensors (device or host) or numpy arrays (host); torch is
used only for device memory and streams.
"""

from __future__ import annotations

import ctypes as C
import os
import re
import sys

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstev.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "stev.h")

STEV_OK, STEV_EINVAL, STEV_ENOMEM, STEV_EAGAIN, STEV_ENOTFOUND, STEV_EDEVICE, STEV_ECELLS = range(7)
LOAD_BINS = 128


def load_bin_edges():
    """Lower edge (iteration count) of each bin of Stats.load_hist."""
    edges = []
    for b in range(LOAD_BINS):
        if b < 4:
            edges.append(b)
        else:
            e, k = b // 4 + 1, b % 4
            edges.append((1 << e) + k * (1 << (e - 2)))
    return edges


def load_curve(load_hist):
    """Sec 2.4 load from a load histogram: [(i, cells still integrating in
    their i-th step)] at every bin edge i >= 1 where the load changes."""
    edges = load_bin_edges()
    out, tail = [], 0
    for b in range(LOAD_BINS - 1, 0, -1):
        tail += int(load_hist[b])
        if load_hist[b]:
            out.append((edges[b], tail))
    return out[::-1]
F64, F32 = 0, 1
THERMO_POLY, THERMO_MLP, THERMO_ANN = 0, 1, 2
ERR_NAMES = {0: "STEV_OK", 1: "STEV_EINVAL", 2: "STEV_ENOMEM", 3: "STEV_EAGAIN",
             4: "STEV_ENOTFOUND", 5: "STEV_EDEVICE", 6: "STEV_ECELLS"}


class StevError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


class MechDesc(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("n_reactions", C.c_int32),
                ("W", C.c_void_p), ("nasa_lo", C.c_void_p), ("nasa_hi", C.c_void_p),
                ("T_mid", C.c_void_p), ("rxn_ptr", C.c_void_p), ("sp_idx", C.c_void_p),
                ("nu", C.c_void_p), ("order", C.c_void_p), ("A", C.c_void_p),
                ("b", C.c_void_p), ("Ea", C.c_void_p), ("reversible", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("precision", C.c_int32), ("thermo", C.c_int32),
                ("ystep_max", C.c_double), ("delta_max", C.c_double), ("alpha", C.c_double),
                ("tol_ring", C.c_double), ("tol_freq", C.c_double), ("r_fac", C.c_double),
                ("rof_min", C.c_double), ("dft_window", C.c_int32),
                ("lanes_per_cell", C.c_int32), ("max_iters", C.c_int64),
                ("waves_per_wg", C.c_int32), ("compact_every", C.c_int32),
                ("grid_wgs", C.c_int32), ("use_graph", C.c_int32),
                ("stab_limit", C.c_int32), ("hot_first", C.c_int32),
                ("reserved", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("total_iters", C.c_int64),
                ("max_cell_iters", C.c_int64), ("n_failed", C.c_int64),
                ("kernel_ms", C.c_double), ("total_ms", C.c_double),
                ("lanes_per_cell", C.c_int32), ("waves_per_wg", C.c_int32),
                ("grid_wgs", C.c_int32), ("compact_every", C.c_int32),
                ("latency_ms", C.c_double), ("queued_ms", C.c_double),
                ("budget_waits", C.c_int32), ("round_requests", C.c_int32),
                ("launch_ms", C.c_double), ("load_hist", C.c_int64 * 128)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["load_hist"] = list(self.load_hist)
        return d


class MlpCfg(C.Structure):
    _fields_ = [("hidden", C.c_int32), ("epochs", C.c_int32), ("n_samples", C.c_int64),
                ("batch", C.c_int32), ("seed", C.c_int32), ("lr", C.c_double),
                ("T_lo", C.c_double), ("T_hi", C.c_double), ("holdout_frac", C.c_double)]


class MlpReport(C.Structure):
    _fields_ = [("train_loss", C.c_double), ("test_loss", C.c_double),
                ("max_rel_err_cp", C.c_double), ("mean_rel_err_cp", C.c_double),
                ("max_rel_err_h", C.c_double), ("mean_rel_err_h", C.c_double),
                ("train_ms", C.c_double), ("steps", C.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class C3mDesc(C.Structure):
    """stev_c3m_desc: Table 2 constants, the Eq 31 / Eq 37 stoichiometry and
    the molar masses (a dict as made by synth.make_c3m)."""
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

    @classmethod
    def from_dict(cls, d):
        c = cls()
        for f, t in cls._fields_:
            if hasattr(t, "_length_"):
                getattr(c, f)[:] = [float(x) for x in d[f]]
            else:
                setattr(c, f, float(d[f]))
        return c


class LmaCfg(C.Structure):
    _fields_ = [("hidden", C.c_int32), ("iters", C.c_int32), ("n_samples", C.c_int64),
                ("T_lo", C.c_double), ("T_hi", C.c_double), ("holdout_frac", C.c_double),
                ("lambda0", C.c_double), ("seed", C.c_uint64)]


class LmaReport(C.Structure):
    _fields_ = [("hidden", C.c_int32), ("accepted", C.c_int32), ("rejected", C.c_int32),
                ("reserved", C.c_int32), ("n_params", C.c_int64),
                ("train_loss", C.c_double), ("test_loss", C.c_double),
                ("max_rel_cp", C.c_double), ("mean_rel_cp", C.c_double),
                ("final_lambda", C.c_double), ("train_ms", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def header_symbols():
    """Entry points declared in include/stev.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(stev_[a-z_0-9]+)\s*\(", text)))


def load():
    """Load libstev.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libstev.so not built ({LIB_PATH}); run __graft_entry__.build()")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.stev_default_params.argtypes = [C.POINTER(Params)]
    L.stev_default_params.restype = None
    L.stev_init.argtypes = [C.POINTER(vp), C.c_int, C.c_size_t]
    L.stev_set_stream.argtypes = [vp, vp]
    L.stev_create_mechanism.argtypes = [vp, C.POINTER(MechDesc), C.POINTER(vp)]
    L.stev_integrate.argtypes = [vp, vp, i64, vp, vp, vp, i64, i64, dbl, C.POINTER(Params),
                                 vp, vp, C.POINTER(Stats)]
    L.stev_integrate_noalloc.argtypes = [vp, vp, i64, vp, vp, vp, i64, i64, dbl,
                                         C.POINTER(Params), vp, vp, C.POINTER(Stats)]
    L.stev_noalloc_max_cells.argtypes = []
    L.stev_noalloc_max_cells.restype = i64
    L.stev_integrate_batched.argtypes = [vp, i32, C.POINTER(vp), C.POINTER(i64), C.POINTER(vp),
                                         C.POINTER(vp), C.POINTER(vp), C.POINTER(i64),
                                         C.POINTER(i64), dbl, C.POINTER(Params), C.POINTER(vp),
                                         C.POINTER(vp), C.POINTER(Stats)]
    L.stev_submit.argtypes = [vp, vp, i64, vp, vp, vp, i64, i64, dbl, C.POINTER(Params), vp, vp,
                              C.POINTER(C.c_uint64)]
    L.stev_poll.argtypes = [vp, C.c_uint64, C.POINTER(Stats)]
    L.stev_train_thermo_mlp.argtypes = [vp, vp, C.POINTER(MlpCfg), C.POINTER(MlpReport)]
    L.stev_get_thermo_mlp.argtypes = [vp, vp, vp, C.POINTER(i64)]
    L.stev_set_thermo_mlp.argtypes = [vp, vp, i32, dbl, dbl, vp, i64]
    L.stev_set_thermo_ann.argtypes = [vp, vp, i32, dbl, dbl, vp]
    L.stev_autotune.argtypes = [vp, vp, i64, vp, vp, vp, i64, i64, dbl, C.POINTER(Params)]
    L.stev_mlp_loss_grad.argtypes = [vp, i32, i32, vp, i64, vp, vp, vp, C.POINTER(dbl)]
    L.stev_thermo_eval.argtypes = [vp, vp, i32, i64, vp, vp, vp]
    L.stev_lma_n_params.argtypes = [i32, i32]
    L.stev_lma_n_params.restype = i64
    L.stev_train_thermo_lma.argtypes = [vp, vp, C.POINTER(LmaCfg), C.POINTER(LmaReport), vp]
    L.stev_lma_normal_eq.argtypes = [vp, i32, i32, vp, i64, vp, vp, dbl, vp, vp,
                                     C.POINTER(dbl), vp]
    L.stev_c3m_create.argtypes = [vp, C.POINTER(C3mDesc), C.POINTER(vp)]
    L.stev_c3m_destroy.argtypes = [vp, vp]
    L.stev_c3m_destroy.restype = None
    L.stev_c3m_integrate.argtypes = [vp, vp, i64, vp, i64, i64, dbl, C.POINTER(Params), vp, vp,
                                     C.POINTER(Stats)]
    L.stev_c3m_model_flops.argtypes = [C.POINTER(dbl)]
    L.stev_c3m_model_flops.restype = dbl
    L.stev_model_flops.argtypes = [vp, i32, C.POINTER(dbl)]
    L.stev_model_flops.restype = dbl
    L.stev_destroy_mechanism.argtypes = [vp, vp]
    L.stev_destroy_mechanism.restype = None
    L.stev_shutdown.argtypes = [vp]
    L.stev_shutdown.restype = None
    L.stev_last_error.argtypes = [vp]
    L.stev_last_error.restype = C.c_char_p
    _lib = L
    return L


def default_params(**kw):
    p = Params()
    load().stev_default_params(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def _after_torch():
    """Order a library call after the work torch has queued on its current
    stream (the library runs on its own stream): wait for that stream."""
    t = sys.modules.get("torch")
    if t is not None and t.cuda.is_available() and t.cuda.is_initialized():
        t.cuda.current_stream().synchronize()


def _ptr(x):
    """(address, keepalive) for a torch tensor / numpy array / None."""
    if x is None:
        return None, None
    if hasattr(x, "data_ptr"):
        return x.data_ptr(), x
    if isinstance(x, np.ndarray):
        if not x.flags["C_CONTIGUOUS"]:
            raise ValueError("numpy arrays must be C-contiguous")
        return x.ctypes.data, x
    raise TypeError(f"unsupported array type {type(x)}")


class Mechanism:
    def __init__(self, ctx, mech):
        self.ctx = ctx
        self.mech = mech
        self.n_s = int(mech["n_s"])
        self.n_r = int(mech["n_r"])
        keep = {
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
            "reversible": np.ascontiguousarray(mech["reversible"], dtype=np.uint8),
        }
        d = MechDesc(self.n_s, self.n_r, *[keep[f].ctypes.data for f in (
            "W", "nasa_lo", "nasa_hi", "T_mid", "rxn_ptr", "sp_idx", "nu", "order", "A", "b",
            "Ea", "reversible")])
        h = C.c_void_p()
        ctx._check(ctx.lib.stev_create_mechanism(ctx.h, C.byref(d), C.byref(h)))
        self.h = h

    def model_flops(self, thermo=THERMO_POLY):
        tr = C.c_double()
        f = self.ctx.lib.stev_model_flops(self.h, thermo, C.byref(tr))
        return f, tr.value

    def close(self):
        if self.h:
            self.ctx.lib.stev_destroy_mechanism(self.ctx.h, self.h)
            self.h = None


class C3m:
    """A C3M description resident on the device (stev_c3m_create)."""

    def __init__(self, ctx, desc):
        self.ctx = ctx
        self.desc = desc
        d = C3mDesc.from_dict(desc)
        h = C.c_void_p()
        ctx._check(ctx.lib.stev_c3m_create(ctx.h, C.byref(d), C.byref(h)))
        self.h = h

    def model_flops(self):
        tr = C.c_double()
        f = self.ctx.lib.stev_c3m_model_flops(C.byref(tr))
        return f, tr.value

    def close(self):
        if self.h:
            self.ctx.lib.stev_c3m_destroy(self.ctx.h, self.h)
            self.h = None


class Context:
    """One libstev context on one HIP device."""

    def __init__(self, device=0, hbm_budget=0):
        self.lib = load()
        h = C.c_void_p()
        rc = self.lib.stev_init(C.byref(h), int(device), int(hbm_budget))
        if rc != STEV_OK:
            raise StevError(rc, "stev_init failed")
        self.h = h
        self._inflight = {}

    def last_error(self):
        s = self.lib.stev_last_error(self.h)
        return s.decode() if s else ""

    def _check(self, rc, ok=(STEV_OK,)):
        if rc not in ok:
            raise StevError(rc, self.last_error())
        return rc

    def set_stream(self, stream):
        """Launch on a torch.cuda.Stream (or raw hipStream_t int); None = own stream."""
        if stream is None:
            addr = None
        elif hasattr(stream, "cuda_stream"):
            addr = stream.cuda_stream
        else:
            addr = int(stream)
        self._check(self.lib.stev_set_stream(self.h, addr))

    def mechanism(self, mech):
        return Mechanism(self, mech)

    def integrate(self, mech, T, P, Y, dt_flow, params=None, iters=None, status=None,
                  ld_cell=None, ld_species=None, allow_failed=False):
        """Integrate in place.  Y is [n_cells, n_s] unless strides are given.

        Returns (rc, stats dict).  rc is STEV_OK or STEV_ECELLS (failed cells,
        only when allow_failed).
        """
        params = params or default_params()
        n = int(T.shape[0])
        if ld_cell is None:
            ld_cell = int(Y.shape[1]) if len(Y.shape) == 2 else mech.n_s
        if ld_species is None:
            ld_species = 1
        pT, kT = _ptr(T)
        pP, kP = _ptr(P)
        pY, kY = _ptr(Y)
        pI, kI = _ptr(iters)
        pS, kS = _ptr(status)
        _after_torch()
        st = Stats()
        rc = self.lib.stev_integrate(self.h, mech.h, n, pT, pP, pY, int(ld_cell), int(ld_species),
                                     float(dt_flow), C.byref(params), pI, pS, C.byref(st))
        self._check(rc, (STEV_OK, STEV_ECELLS) if allow_failed else (STEV_OK,))
        return rc, st.as_dict()

    def integrate_noalloc(self, mech, T, P, Y, dt_flow, params=None, iters=None, status=None,
                          ld_cell=None, ld_species=None, allow_failed=False):
        """stev_integrate_noalloc: as integrate(), device tensors only; the
        library allocates nothing during the call."""
        params = params or default_params()
        n = int(T.shape[0])
        if ld_cell is None:
            ld_cell = int(Y.shape[1]) if len(Y.shape) == 2 else mech.n_s
        if ld_species is None:
            ld_species = 1
        _after_torch()
        st = Stats()
        rc = self.lib.stev_integrate_noalloc(self.h, mech.h, n, _ptr(T)[0], _ptr(P)[0],
                                             _ptr(Y)[0], int(ld_cell), int(ld_species),
                                             float(dt_flow), C.byref(params), _ptr(iters)[0],
                                             _ptr(status)[0], C.byref(st))
        self._check(rc, (STEV_OK, STEV_ECELLS) if allow_failed else (STEV_OK,))
        return rc, st.as_dict()

    def noalloc_max_cells(self):
        return int(self.lib.stev_noalloc_max_cells())

    def c3m(self, desc):
        return C3m(self, desc)

    def c3m_integrate(self, c3m, state, dt_flow, params=None, iters=None, status=None,
                      ld_cell=None, ld_var=1, n_cells=None, allow_failed=False):
        """Integrate gas-solid cells in place; state is [n_cells, 26], or any
        layout given by n_cells, ld_cell and ld_var."""
        params = params or default_params()
        n = int(state.shape[0]) if n_cells is None else int(n_cells)
        if ld_cell is None:
            ld_cell = int(state.shape[1])
        _after_torch()
        st = Stats()
        rc = self.lib.stev_c3m_integrate(self.h, c3m.h, n, _ptr(state)[0], int(ld_cell),
                                         int(ld_var), float(dt_flow), C.byref(params),
                                         _ptr(iters)[0], _ptr(status)[0], C.byref(st))
        self._check(rc, (STEV_OK, STEV_ECELLS) if allow_failed else (STEV_OK,))
        return rc, st.as_dict()

    def integrate_batched(self, mechs, Ts, Ps, Ys, dt_flow, params=None, iters=None,
                          status=None, allow_failed=False):
        params = params or default_params()
        nb = len(Ts)
        keep = []
        arr = lambda t, xs: (t * nb)(*xs)
        ph = arr(C.c_void_p, [m.h for m in mechs])
        pn = arr(C.c_int64, [int(t.shape[0]) for t in Ts])
        pT = arr(C.c_void_p, [_ptr(t)[0] for t in Ts])
        pP = arr(C.c_void_p, [_ptr(t)[0] for t in Ps])
        pY = arr(C.c_void_p, [_ptr(t)[0] for t in Ys])
        lc = arr(C.c_int64, [int(y.shape[1]) for y in Ys])
        ls = arr(C.c_int64, [1] * nb)
        pI = arr(C.c_void_p, [_ptr(x)[0] for x in iters]) if iters else None
        pS = arr(C.c_void_p, [_ptr(x)[0] for x in status]) if status else None
        keep.extend([Ts, Ps, Ys, iters, status])
        _after_torch()
        st = Stats()
        rc = self.lib.stev_integrate_batched(self.h, nb, ph, pn, pT, pP, pY, lc, ls,
                                             float(dt_flow), C.byref(params), pI, pS,
                                             C.byref(st))
        self._check(rc, (STEV_OK, STEV_ECELLS) if allow_failed else (STEV_OK,))
        return rc, st.as_dict()

    def submit(self, mech, T, P, Y, dt_flow, params=None, iters=None, status=None,
               ld_cell=None, ld_species=None):
        """Enqueue one solve (host or device arrays); returns its ticket.  The
        arrays are kept alive here until poll() reports the ticket done."""
        params = params or default_params()
        n = int(T.shape[0])
        if ld_cell is None:
            ld_cell = int(Y.shape[1]) if len(Y.shape) == 2 else mech.n_s
        if ld_species is None:
            ld_species = 1
        _after_torch()
        tk = C.c_uint64()
        rc = self.lib.stev_submit(self.h, mech.h, n, _ptr(T)[0], _ptr(P)[0], _ptr(Y)[0],
                                  int(ld_cell), int(ld_species), float(dt_flow), C.byref(params),
                                  _ptr(iters)[0], _ptr(status)[0], C.byref(tk))
        self._check(rc)
        self._inflight[tk.value] = (T, P, Y, iters, status)
        return tk.value

    def poll(self, ticket):
        """(rc, stats): rc is STEV_OK / STEV_ECELLS when done, STEV_EAGAIN while pending."""
        st = Stats()
        rc = self.lib.stev_poll(self.h, C.c_uint64(ticket), C.byref(st))
        if rc not in (STEV_OK, STEV_EAGAIN, STEV_ECELLS):
            self._inflight.pop(ticket, None)
            raise StevError(rc, self.last_error())
        if rc != STEV_EAGAIN:
            self._inflight.pop(ticket, None)
        return rc, st.as_dict()

    def train_thermo_mlp(self, mech, **cfg):
        c = MlpCfg(32, 4, 1 << 20, 4096, 104, 3e-3, 300.0, 3000.0, 0.125)
        for k, v in cfg.items():
            setattr(c, k, v)
        rep = MlpReport()
        self._check(self.lib.stev_train_thermo_mlp(self.h, mech.h, C.byref(c), C.byref(rep)))
        return rep.as_dict()

    def get_thermo_mlp(self, mech):
        n = C.c_int64(0)
        self._check(self.lib.stev_get_thermo_mlp(self.h, mech.h, None, C.byref(n)))
        buf = np.zeros(n.value, dtype=np.float32)
        self._check(self.lib.stev_get_thermo_mlp(self.h, mech.h, buf.ctypes.data, C.byref(n)))
        return buf

    def set_thermo_mlp(self, mech, hidden, T_lo, T_hi, values):
        v = np.ascontiguousarray(values, dtype=np.float32)
        self._check(self.lib.stev_set_thermo_mlp(self.h, mech.h, int(hidden), float(T_lo),
                                                 float(T_hi), v.ctypes.data, len(v)))

    def set_thermo_ann(self, mech, hidden, T_lo, T_hi, params):
        """Attach the paper's sigmoid network (FP64 parameters in the
        Levenberg-Marquardt layout, outputs cp/R then h/R) for THERMO_ANN."""
        p = np.ascontiguousarray(params, dtype=np.float64)
        if len(p) != self.lib.stev_lma_n_params(int(hidden), 2 * mech.n_s):
            raise ValueError("parameter count does not match hidden and the species count")
        self._check(self.lib.stev_set_thermo_ann(self.h, mech.h, int(hidden), float(T_lo),
                                                 float(T_hi), p.ctypes.data))

    def train_thermo_lma(self, mech, **cfg):
        """The paper's sigmoid network fitted by Levenberg-Marquardt on the
        GPU; returns (report dict, FP64 parameters with outputs cp/R and h/R,
        ready for set_thermo_ann)."""
        c = LmaCfg(0, 60, 1 << 16, 300.0, 3000.0, 0.125, 1e-2, 104)
        for k, v in cfg.items():
            setattr(c, k, v)
        rep = LmaReport()
        n_out = 2 * mech.n_s
        H = c.hidden if c.hidden > 0 else n_out
        prm = np.zeros(self.lib.stev_lma_n_params(H, n_out))
        self._check(self.lib.stev_train_thermo_lma(self.h, mech.h, C.byref(c), C.byref(rep),
                                                   prm.ctypes.data))
        return rep.as_dict(), prm

    def lma_normal_eq(self, hidden, n_out, params, x, target, lam=None, jtj=True):
        """GPU normal equations (J^T J, J^T r, loss) and, with lam, the
        Levenberg-Marquardt step; host FP64 arrays."""
        p = np.ascontiguousarray(params, dtype=np.float64)
        xx = np.ascontiguousarray(x, dtype=np.float64)
        t = np.ascontiguousarray(target, dtype=np.float64)
        P = len(p)
        A = np.zeros((P, P)) if jtj else None
        g = np.zeros(P)
        d = np.zeros(P) if lam is not None else None
        loss = C.c_double()
        self._check(self.lib.stev_lma_normal_eq(
            self.h, int(hidden), int(n_out), p.ctypes.data, len(xx), xx.ctypes.data,
            t.ctypes.data, float(lam if lam is not None else 0.0),
            A.ctypes.data if A is not None else None, g.ctypes.data, C.byref(loss),
            d.ctypes.data if d is not None else None))
        return A, g, loss.value, d

    def mlp_loss_grad(self, n_out, params, x, target, hidden=32):
        """GPU loss and gradient of a thermo network (FP32), host arrays."""
        p = np.ascontiguousarray(params, dtype=np.float32)
        xx = np.ascontiguousarray(x, dtype=np.float32)
        t = np.ascontiguousarray(target, dtype=np.float32)
        g = np.zeros_like(p)
        loss = C.c_double()
        self._check(self.lib.stev_mlp_loss_grad(self.h, hidden, n_out, p.ctypes.data, len(xx),
                                                xx.ctypes.data, t.ctypes.data, g.ctypes.data,
                                                C.byref(loss)))
        return loss.value, g

    def thermo_eval(self, mech, T, thermo=THERMO_POLY):
        """cp/R and h/R at temperatures T ([n, n_s] each), evaluated on the GPU."""
        TT = np.ascontiguousarray(T, dtype=np.float64)
        cp = np.zeros((len(TT), mech.n_s))
        h = np.zeros((len(TT), mech.n_s))
        self._check(self.lib.stev_thermo_eval(self.h, mech.h, thermo, len(TT), TT.ctypes.data,
                                              cp.ctypes.data, h.ctypes.data))
        return cp, h

    def autotune(self, mech, T, P, Y, dt_flow, params=None):
        params = params or default_params()
        _after_torch()
        self._check(self.lib.stev_autotune(self.h, mech.h, int(T.shape[0]), _ptr(T)[0],
                                           _ptr(P)[0], _ptr(Y)[0], int(Y.shape[1]), 1,
                                           float(dt_flow), C.byref(params)))
        return params

    def close(self):
        if self.h:
            self.lib.stev_shutdown(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
