"""ctypes wrapper of the plain FP64 CPU oracle (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` use this module.  It loads ``oracle/libpcpic_oracle.so`` (built by
``oracle/build_oracle.py``) and keeps every array in NumPy, owned here.

A tube is described by a plain dict with the keys
``n_cells, length, radius, dt_over_dz, q_over_m, ppc, rho_kind, rho_amp, kappa,
r_star, knots, fp_bits, flags, capacity`` (missing keys take the defaults below).
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# PCPIC_ORACLE_LIB selects another build of the same source (the planted-mistake
# tests build mutated copies of it).
LIB_PATH = os.environ.get("PCPIC_ORACLE_LIB") or os.path.join(HERE, "libpcpic_oracle.so")

RHO_UNIFORM, RHO_FRAME_DRAG, RHO_KNOTS, RHO_GR = 0, 1, 2, 3
NO_AUTO_INJECT, FREEZE_FIELDS, B_STEADY_INIT, GR_ALPHA = 1, 2, 4, 8
ST_CAPACITY, ST_NONFINITE = 1, 2

DEFAULTS = dict(n_cells=1024, length=10.0, radius=1.0, dt_over_dz=0.5, q_over_m=-1.0,
                ppc=4.0, rho_kind=RHO_UNIFORM, rho_amp=1.0, kappa=0.0, r_star=10.0,
                knots=None, fp_bits=32, flags=0, capacity=1 << 16, macro_charge=0.0, inj_rate=0.0,
                schedule=None, incl=0.0, theta_star=0.0, cos_phi=1.0, rg_over_rstar=0.0)

_pd = ctypes.POINTER(ctypes.c_double)
_pi = ctypes.POINTER(ctypes.c_int64)


class OrcCfg(ctypes.Structure):
    _fields_ = [("n_cells", ctypes.c_int64), ("length", ctypes.c_double),
                ("radius", ctypes.c_double), ("dt_over_dz", ctypes.c_double),
                ("q_over_m", ctypes.c_double), ("ppc", ctypes.c_double),
                ("rho_kind", ctypes.c_int32), ("n_knots", ctypes.c_int32),
                ("rho_amp", ctypes.c_double), ("kappa", ctypes.c_double),
                ("r_star", ctypes.c_double), ("knots", _pd),
                ("fp_bits", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("capacity", ctypes.c_int64), ("macro_charge", ctypes.c_double),
                ("inj_rate", ctypes.c_double), ("schedule", _pi), ("n_schedule", ctypes.c_int64),
                ("incl", ctypes.c_double), ("theta_star", ctypes.c_double), ("cos_phi", ctypes.c_double),
                ("rg_over_rstar", ctypes.c_double)]


class OrcState(ctypes.Structure):
    _fields_ = [("x", _pd), ("u", _pd), ("rho_gj", _pd), ("ez", _pd), ("er", _pd),
                ("b", _pd), ("j", _pi), ("k", _pd), ("phi", _pd), ("cp", _pd),
                ("dp", _pd), ("w", _pi), ("n", ctypes.c_int64), ("step", ctypes.c_int64),
                ("n_injected", ctypes.c_int64), ("n_exit", ctypes.c_int64),
                ("n_absorb", ctypes.c_int64), ("w0", ctypes.c_int64),
                ("last_ninj", ctypes.c_int64), ("status", ctypes.c_int64),
                ("exit_sum_lo", ctypes.c_uint64), ("exit_sum_hi", ctypes.c_int64),
                ("e_surf", ctypes.c_double), ("cls", ctypes.POINTER(ctypes.c_uint8)), ("j_inj", _pi)]


_lib = None


def load():
    """Load (building first if needed) the oracle library."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build_oracle  # noqa: F401  (package-relative when imported as oracle.oracle)
            build_oracle.build()
        lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        lib.orc_rho_gj.argtypes = [P(OrcCfg), _pd]
        lib.orc_weights.argtypes = [P(OrcCfg), _pd, ctypes.c_int64, _pi]
        lib.orc_init.argtypes = [P(OrcCfg), P(OrcState)]
        lib.orc_inject.argtypes = [P(OrcCfg), P(OrcState), ctypes.c_int64, _pd, _pd]
        lib.orc_step.argtypes = [P(OrcCfg), P(OrcState), ctypes.c_int64]
        lib.orc_gauss.argtypes = [P(OrcCfg), P(OrcState), _pd, _pd]
        lib.orc_profile.argtypes = [P(OrcCfg), P(OrcState), ctypes.c_int32, _pi,
                                    P(ctypes.c_uint64), _pi, _pd, _pd]
        for f in ("orc_tl_fields", "orc_ad_fields"):
            getattr(lib, f).argtypes = [P(OrcCfg), P(OrcState)] + [_pd] * 7
        for f in ("orc_tl_push", "orc_ad_push"):
            getattr(lib, f).argtypes = [P(OrcCfg), P(OrcState)] + [_pd] * 6
        lib.orc_tl_poisson.argtypes = [P(OrcCfg), P(OrcState)] + [_pd] * 3
        lib.orc_ad_poisson.argtypes = [P(OrcCfg), P(OrcState)] + [_pd] * 3
        for f in ("orc_tl_fields", "orc_ad_fields", "orc_tl_push", "orc_ad_push", "orc_tl_poisson",
                  "orc_ad_poisson"):
            getattr(lib, f).restype = ctypes.c_int
        lib.orc_step_par.argtypes = [P(OrcCfg), P(OrcState), ctypes.c_int64, ctypes.c_int32]
        lib.orc_step_par.restype = ctypes.c_int
        lib.orc_adjoint.argtypes = [P(OrcCfg), P(OrcState), ctypes.c_int64, _pd, _pd, _pd, _pi]
        lib.orc_adjoint.restype = ctypes.c_int
        for f in ("orc_rho_gj", "orc_weights", "orc_init", "orc_inject", "orc_step",
                  "orc_gauss", "orc_profile"):
            getattr(lib, f).restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a, t=_pd):
    return a.ctypes.data_as(t)


def i128_to_float(lo, hi):
    """Value of a two-word 128-bit integer (unsigned low word, signed high word)."""
    return float((int(hi) << 64) + int(lo))


class OracleTube:
    """One tube advanced by the oracle.  All arrays are NumPy, owned here."""

    def __init__(self, cfg=None, **kw):
        c = dict(DEFAULTS)
        c.update(cfg or {})
        c.update(kw)
        self.cfg = c
        self.lib = load()
        N, cap = int(c["n_cells"]), int(c["capacity"])
        self.N = N
        knots = c.get("knots")
        self._knots = None if knots is None else np.ascontiguousarray(knots, dtype=np.float64)
        sched = c.get("schedule")
        self._sched = None if sched is None else np.ascontiguousarray(sched, dtype=np.int64)
        self.ccfg = OrcCfg(N, c["length"], c["radius"], c["dt_over_dz"], c["q_over_m"], c["ppc"],
                           int(c["rho_kind"]), 0 if self._knots is None else len(self._knots),
                           c["rho_amp"], c["kappa"], c["r_star"],
                           None if self._knots is None else _ptr(self._knots),
                           int(c["fp_bits"]), int(c["flags"]), cap, float(c["macro_charge"]),
                           float(c["inj_rate"]), None if self._sched is None else _ptr(self._sched, _pi),
                           0 if self._sched is None else len(self._sched), float(c["incl"]),
                           float(c["theta_star"]), float(c["cos_phi"]), float(c["rg_over_rstar"]))
        self._x = np.zeros(cap, np.float64)
        self._u = np.zeros(cap, np.float64)
        self.rho_gj = np.zeros(N + 1)
        self.ez = np.zeros(N)
        self.er = np.zeros(N + 1)
        self.b = np.zeros(N)
        self.j = np.zeros(N, np.int64)
        self.k = np.zeros(N)
        self.phi = np.zeros(N + 1)
        self._cp = np.zeros(N + 1)
        self._dp = np.zeros(N + 1)
        self.w = np.zeros(N + 1, np.int64)
        self._cls = np.zeros(cap, np.uint8)
        self.j_inj = np.zeros(N, np.int64)
        self.st = OrcState(_ptr(self._x), _ptr(self._u), _ptr(self.rho_gj), _ptr(self.ez),
                           _ptr(self.er), _ptr(self.b), _ptr(self.j, _pi), _ptr(self.k),
                           _ptr(self.phi), _ptr(self._cp), _ptr(self._dp), _ptr(self.w, _pi))
        self.st.cls = self._cls.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        self.st.j_inj = _ptr(self.j_inj, _pi)
        rc = self.lib.orc_init(ctypes.byref(self.ccfg), ctypes.byref(self.st))
        if rc != 0:
            raise ValueError(f"orc_init rejected the configuration (rc={rc})")

    # -- operations ---------------------------------------------------------
    def inject(self, x, u):
        x = np.ascontiguousarray(x, np.float64)
        u = np.ascontiguousarray(u, np.float64)
        rc = self.lib.orc_inject(ctypes.byref(self.ccfg), ctypes.byref(self.st), len(x),
                                 _ptr(x), _ptr(u))
        if rc != 0:
            raise ValueError(f"orc_inject failed (rc={rc})")

    def step(self, n=1):
        rc = self.lib.orc_step(ctypes.byref(self.ccfg), ctypes.byref(self.st), int(n))
        if rc != 0:
            raise ValueError(f"orc_step failed (rc={rc})")

    def step_par(self, n=1, threads=0):
        """n steps with the particles split over `threads` OpenMP threads (0 = the
        default count); the same state as step(n), bit for bit."""
        rc = self.lib.orc_step_par(ctypes.byref(self.ccfg), ctypes.byref(self.st), int(n), int(threads))
        if rc != 0:
            raise ValueError(f"orc_step_par failed (rc={rc})")

    # -- linearised kernels (dot-product pins of the reverse sweep) ------------
    def _lin(self, name, ins, out_sizes):
        ins = [np.ascontiguousarray(a, np.float64) for a in ins]
        outs = [np.zeros(n) for n in out_sizes]
        rc = getattr(self.lib, name)(ctypes.byref(self.ccfg), ctypes.byref(self.st), *[_ptr(a) for a in ins + outs])
        if rc != 0:
            raise ValueError(f"{name} failed (rc={rc})")
        return outs

    def tl_fields(self, dez, der, db, dj):
        N = self.N
        return self._lin("orc_tl_fields", [dez, der, db, dj], [N, N + 1, N])

    def ad_fields(self, lez1, ler1, lb1):
        N = self.N
        return self._lin("orc_ad_fields", [lez1, ler1, lb1], [N, N + 1, N, N])

    def tl_push(self, dx, du, dk):
        n = self.n
        return self._lin("orc_tl_push", [dx, du, dk], [n, n, self.N])

    def ad_push(self, lx1, lu1, lj):
        n = self.n
        return self._lin("orc_ad_push", [lx1, lu1, lj], [n, n, self.N])

    def tl_poisson(self, drho):
        return self._lin("orc_tl_poisson", [drho], [self.N, self.N + 1])

    def ad_poisson(self, lez, ler):
        return self._lin("orc_ad_poisson", [lez, ler], [self.N + 1])

    def gauss(self):
        g = np.zeros(self.N + 1)
        gm = ctypes.c_double(0.0)
        self.lib.orc_gauss(ctypes.byref(self.ccfg), ctypes.byref(self.st), _ptr(g), ctypes.byref(gm))
        return g, gm.value

    def weights(self):
        w = np.zeros(self.N + 1, np.int64)
        self.lib.orc_weights(ctypes.byref(self.ccfg), _ptr(self._x), self.st.n, _ptr(w, _pi))
        return w

    def profile(self, nb):
        cnt = np.zeros(nb, np.int64)
        lo = np.zeros(nb, np.uint64)
        hi = np.zeros(nb, np.int64)
        mn = np.zeros(nb)
        mx = np.zeros(nb)
        self.lib.orc_profile(ctypes.byref(self.ccfg), ctypes.byref(self.st), nb, _ptr(cnt, _pi),
                             lo.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), _ptr(hi, _pi),
                             _ptr(mn), _ptr(mx))
        return cnt, lo, hi, mn, mx

    def adjoint(self, n_steps):
        """Run n_steps recording, then the reverse sweep: returns (loss, n_exit,
        dL/d rho_GJ at the nodes, dL/d inj_rate)."""
        g = np.zeros(self.N + 1)
        gr = ctypes.c_double(0.0)
        loss = ctypes.c_double(0.0)
        nex = ctypes.c_int64(0)
        rc = self.lib.orc_adjoint(ctypes.byref(self.ccfg), ctypes.byref(self.st), int(n_steps), _ptr(g),
                                  ctypes.byref(gr), ctypes.byref(loss), ctypes.byref(nex))
        if rc != 0:
            raise ValueError(f"orc_adjoint failed (rc={rc})")
        return loss.value, nex.value, g, gr.value

    @property
    def cls(self):
        return self._cls[: self.st.n]

    def rho_gj_of(self):
        r = np.zeros(self.N + 1)
        self.lib.orc_rho_gj(ctypes.byref(self.ccfg), _ptr(r))
        return r

    # -- state ----------------------------------------------------------------
    @property
    def n(self):
        return self.st.n

    @property
    def x(self):
        return self._x[: self.st.n]

    @property
    def u(self):
        return self._u[: self.st.n]

    @property
    def counters(self):
        s = self.st
        return dict(step=s.step, n_alive=s.n, n_injected=s.n_injected, n_exit=s.n_exit,
                    n_absorb=s.n_absorb, w0=s.w0, last_ninj=s.last_ninj, status=s.status,
                    exit_sum_lo=s.exit_sum_lo, exit_sum_hi=s.exit_sum_hi, e_surf=s.e_surf)

    def exit_gamma_sum(self):
        return i128_to_float(self.st.exit_sum_lo, self.st.exit_sum_hi) / 2.0 ** 32

    @property
    def dz(self):
        return self.cfg["length"] / self.N

    @property
    def macro_charge(self):
        return self.rho_gj[0] * self.dz / self.cfg["ppc"]
