"""ctypes binding of ``libpcpic.so`` (the C ABI in ``include/pcpic.h``).

Argument marshalling only: every step of the method runs in the library's
gfx950 kernels.  PyTorch supplies the device workspace (a ``uint8`` tensor)
and the HIP stream; nothing here computes on the host.

A tube is described by a dict with the keys of ``pic_params`` (see
``DEFAULTS``); the same dict drives the CPU oracle in the tests.
"""
import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libpcpic.so")

ABI_VERSION = 4
FP64, FP32_BULK = 0, 1
RHO_UNIFORM, RHO_FRAME_DRAG, RHO_KNOTS, RHO_GR = 0, 1, 2, 3
NO_AUTO_INJECT, FREEZE_FIELDS, B_STEADY_INIT, GR_ALPHA = 1, 2, 4, 8
ST_CAPACITY, ST_NONFINITE, ST_GAUSS = 1, 2, 4

STATUS_NAMES = {0: "PIC_OK", -1: "PIC_EINVAL", -2: "PIC_EWORKSPACE", -3: "PIC_ECAPACITY",
                -4: "PIC_ENONFINITE", -5: "PIC_ECFL", -6: "PIC_EDEVICE", -7: "PIC_ESTATE",
                -8: "PIC_EABI", -9: "PIC_EDEVSTATUS"}

DEFAULTS = dict(precision=FP64, n_cells=1024, length=10.0, radius=1.0, dt_over_dz=0.5,
                q_over_m=-1.0, ppc=4.0, rho_kind=RHO_UNIFORM, rho_amp=1.0, kappa=0.0,
                r_star=10.0, knots=None, fp_bits=32, sort_every=0, capacity=1 << 16, flags=0,
                max_bins=1024, gamma_fp64=0.0, macro_charge=0.0, incl=0.0, theta_star=0.0, cos_phi=1.0,
                rg_over_rstar=0.0)

_pd = ctypes.POINTER(ctypes.c_double)
_pi = ctypes.POINTER(ctypes.c_int64)
_pu = ctypes.POINTER(ctypes.c_uint64)


class PicParams(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("n_cells", ctypes.c_int64), ("length", ctypes.c_double),
                ("radius", ctypes.c_double), ("dt_over_dz", ctypes.c_double),
                ("q_over_m", ctypes.c_double), ("ppc", ctypes.c_double),
                ("rho_kind", ctypes.c_int32), ("n_knots", ctypes.c_int32),
                ("rho_amp", ctypes.c_double), ("kappa", ctypes.c_double),
                ("r_star", ctypes.c_double), ("knots", _pd),
                ("fp_bits", ctypes.c_int32), ("sort_every", ctypes.c_int32),
                ("capacity", ctypes.c_int64), ("flags", ctypes.c_uint32),
                ("max_bins", ctypes.c_int32), ("gamma_fp64", ctypes.c_double),
                ("macro_charge", ctypes.c_double), ("incl", ctypes.c_double), ("theta_star", ctypes.c_double),
                ("cos_phi", ctypes.c_double), ("rg_over_rstar", ctypes.c_double)]


class PicDiagReq(ctypes.Structure):
    _fields_ = [("n_bins", ctypes.c_int32), ("want_gauss", ctypes.c_int32), ("gauss_tol", ctypes.c_double)]


class PicDiag(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("n_alive", ctypes.c_int64), ("n_slots", ctypes.c_int64),
                ("n_injected", ctypes.c_int64), ("n_exit", ctypes.c_int64),
                ("n_absorb", ctypes.c_int64), ("last_n_inj", ctypes.c_int64),
                ("w0", ctypes.c_int64), ("status", ctypes.c_int64), ("e_surf", ctypes.c_double),
                ("exit_sum_lo", ctypes.c_uint64), ("exit_sum_hi", ctypes.c_int64),
                ("exit_gamma_sum", ctypes.c_double), ("gauss_max", ctypes.c_double),
                ("n_slots_high", ctypes.c_int64), ("gauss_l2", ctypes.c_double), ("ez", _pd), ("er", _pd), ("b_phi", _pd), ("rho_gj", _pd), ("j_last", _pi),
                ("weights", _pi), ("gauss", _pd), ("prof_count", _pi), ("prof_mean", _pd),
                ("prof_min", _pd), ("prof_max", _pd), ("prof_sum_lo", _pu), ("prof_sum_hi", _pi)]


class PicTiming(ctypes.Structure):
    _fields_ = [("push_ms", ctypes.c_double), ("field_ms", ctypes.c_double),
                ("sort_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("push_launches", ctypes.c_int64), ("field_launches", ctypes.c_int64),
                ("sort_launches", ctypes.c_int64), ("particle_steps", ctypes.c_int64)]


class PicAdjointOut(ctypes.Structure):
    _fields_ = [("loss", ctypes.c_double), ("n_exit", ctypes.c_int64), ("g_rate", ctypes.c_double),
                ("g_kappa", ctypes.c_double), ("g_amp", ctypes.c_double), ("g_rho", _pd),
                ("g_knots", _pd), ("forward_ms", ctypes.c_double), ("backward_ms", ctypes.c_double)]


# Every symbol include/pcpic.h declares, with its ctypes signature.
SIGNATURES = {
    "pic_abi_version": (ctypes.c_int32, []),
    "pic_last_error": (ctypes.c_char_p, []),
    "pic_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(PicParams)]),
    "pic_init": (ctypes.c_int32, [ctypes.POINTER(PicParams), ctypes.c_void_p, ctypes.c_size_t,
                                  ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "pic_inject": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_int32]),
    "pic_step": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int64]),
    "pic_diagnostics": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(PicDiagReq),
                                         ctypes.POINTER(PicDiag)]),
    "pic_read_particles": (ctypes.c_int32, [ctypes.c_void_p, _pd, _pd, ctypes.c_int64, _pi]),
    "pic_profile_noalloc": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pic_write_fields": (ctypes.c_int32, [ctypes.c_void_p, _pd, _pd, _pd]),
    "pic_step_timed": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(PicTiming)]),
    "pic_set_push_config": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_uint32]),
    "pic_sync": (ctypes.c_int32, [ctypes.c_void_p]),
    "pic_stream_copy": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "pic_adjoint_tape_bytes": (ctypes.c_size_t, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32]),
    "pic_run_adjoint": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p,
                                         ctypes.c_size_t, ctypes.POINTER(PicAdjointOut)]),
    "pic_adjoint_forward": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p,
                                             ctypes.c_size_t, ctypes.POINTER(PicAdjointOut)]),
    "pic_backward": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_double, ctypes.POINTER(PicAdjointOut)]),
    "pic_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(PicParams), ctypes.c_int32]),
    "pic_init_batch": (ctypes.c_int32, [ctypes.POINTER(PicParams), ctypes.c_int32, ctypes.c_void_p,
                                        ctypes.c_size_t, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "pic_batch_tube": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]),
    "pic_batch_set_config": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint32]),
    "pic_batch_get_config": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                              ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64),
                                              ctypes.POINTER(ctypes.c_int64)]),
    "pic_set_injection_schedule": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64]),
    "pic_save": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]),
    "pic_load": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]),
    "pic_destroy": (ctypes.c_int32, [ctypes.c_void_p]),
}

_lib = None


class PicError(RuntimeError):
    def __init__(self, code, where, msg):
        super().__init__(f"{where}: {STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def load():
    """Load the built library; raise if it is missing (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1011_6330_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _check(code, where):
    if code != 0:
        raise PicError(code, where, load().pic_last_error().decode())


def _ptr(a, t=_pd):
    return None if a is None else a.ctypes.data_as(t)


def make_params(cfg=None, **kw):
    """pic_params from a config dict; returns (struct, knots array kept alive)."""
    c = dict(DEFAULTS)
    c.update(cfg or {})
    c.update(kw)
    knots = c.get("knots")
    knots = None if knots is None else np.ascontiguousarray(knots, dtype=np.float64)
    p = PicParams(ABI_VERSION, int(c["precision"]), int(c["n_cells"]), float(c["length"]),
                  float(c["radius"]), float(c["dt_over_dz"]), float(c["q_over_m"]), float(c["ppc"]),
                  int(c["rho_kind"]), 0 if knots is None else len(knots), float(c["rho_amp"]),
                  float(c["kappa"]), float(c["r_star"]), _ptr(knots), int(c["fp_bits"]),
                  int(c["sort_every"]), int(c["capacity"]), int(c["flags"]), int(c["max_bins"]),
                  float(c["gamma_fp64"]), float(c["macro_charge"]), float(c["incl"]),
                  float(c["theta_star"]), float(c["cos_phi"]), float(c["rg_over_rstar"]))
    return p, knots, c


def workspace_bytes(cfg=None, **kw):
    p, _k, _c = make_params(cfg, **kw)
    n = load().pic_workspace_bytes(ctypes.byref(p))
    if n == 0:
        raise PicError(-1, "pic_workspace_bytes", load().pic_last_error().decode())
    return n


class _TubeOps:
    """Per-tube operations shared by a stand-alone Tube and a tube of a Batch."""

    # -- operations -----------------------------------------------------------
    def inject(self, x, u):
        """Append particles from NumPy (host) arrays or torch CUDA float64 tensors."""
        try:
            import torch
            if isinstance(x, torch.Tensor) and x.is_cuda:
                x = x.contiguous().to(torch.float64)
                u = u.contiguous().to(torch.float64)
                self.stream.wait_stream(torch.cuda.current_stream(self.device))
                _check(self.lib.pic_inject(self._h, x.numel(), ctypes.c_void_p(x.data_ptr()),
                                           ctypes.c_void_p(u.data_ptr()), 1), "pic_inject")
                return
        except ImportError:
            pass
        x = np.ascontiguousarray(x, np.float64)
        u = np.ascontiguousarray(u, np.float64)
        _check(self.lib.pic_inject(self._h, len(x), x.ctypes.data_as(ctypes.c_void_p),
                                   u.ctypes.data_as(ctypes.c_void_p), 0), "pic_inject")


    def save(self):
        """The tube's state as bytes (pic_save)."""
        n = ctypes.c_size_t(0)
        _check(self.lib.pic_save(self._h, None, 0, ctypes.byref(n)), "pic_save")
        buf = ctypes.create_string_buffer(n.value)
        _check(self.lib.pic_save(self._h, buf, n.value, ctypes.byref(n)), "pic_save")
        return buf.raw[:n.value]


class Tube(_TubeOps):
    """One tube on the GPU.  The workspace is a torch uint8 tensor on ``device``
    and all work is ordered on ``stream`` (a torch.cuda.Stream, created at the
    default priority when not given)."""

    def __init__(self, cfg=None, device="cuda", stream=None, **kw):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("pcpic.Tube needs a HIP GPU")
        self.lib = load()
        self.params, self._knots, self.cfg = make_params(cfg, **kw)
        self.N = int(self.cfg["n_cells"])
        self.device = torch.device(device)
        nbytes = workspace_bytes(self.cfg)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
            self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._h = ctypes.c_void_p()
        _check(self.lib.pic_init(ctypes.byref(self.params), ctypes.c_void_p(self.ws.data_ptr()), nbytes,
                                 ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self._h)), "pic_init")

    def step(self, n=1):
        _check(self.lib.pic_step(self._h, int(n)), "pic_step")

    def step_timed(self, n):
        """Step with per-kernel HIP events on the tube's stream; returns a dict."""
        t = PicTiming()
        _check(self.lib.pic_step_timed(self._h, int(n), ctypes.byref(t)), "pic_step_timed")
        return {k: getattr(t, k) for k, _ in PicTiming._fields_}

    def load(self, state):
        """Restore a state from save() into this tube (same parameters)."""
        buf = ctypes.create_string_buffer(bytes(state), len(state))
        _check(self.lib.pic_load(self._h, buf, len(state)), "pic_load")

    def set_injection_schedule(self, counts, first_step=0):
        """Replay injection counts (host or CUDA int64) from step first_step on;
        None clears the schedule."""
        import torch
        if counts is None or len(counts) == 0:
            self._sched = None
            _check(self.lib.pic_set_injection_schedule(self._h, None, 0, 0), "pic_set_injection_schedule")
            return
        d = torch.as_tensor(np.asarray(counts, np.int64) if not isinstance(counts, torch.Tensor) else counts,
                            dtype=torch.int64).to(self.device).contiguous()
        torch.cuda.synchronize(self.device)
        self._sched = d                      # keep the device array alive while it is set
        _check(self.lib.pic_set_injection_schedule(self._h, ctypes.c_void_p(d.data_ptr()), int(first_step),
                                                   d.numel()), "pic_set_injection_schedule")

    def set_push_config(self, block, per_thread, nontemporal=False):
        _check(self.lib.pic_set_push_config(self._h, int(block), int(per_thread), 1 if nontemporal else 0),
               "pic_set_push_config")

    def sync(self):
        _check(self.lib.pic_sync(self._h), "pic_sync")

    def run_adjoint(self, n_steps, checkpoint_every=50, tape=None):
        """Advance n_steps with checkpoints, then the reverse sweep: returns the loss
        (mean exit gamma), its gradient and the device times.  The tape is a torch
        uint8 tensor (allocated here when not given)."""
        import torch
        nbytes = self.lib.pic_adjoint_tape_bytes(self._h, int(n_steps), int(checkpoint_every))
        if nbytes == 0:
            raise PicError(-1, "pic_adjoint_tape_bytes", self.lib.pic_last_error().decode())
        if tape is None or tape.numel() < nbytes:
            with torch.cuda.device(self.device):
                tape = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        out = PicAdjointOut()
        g_rho = np.zeros(self.N + 1)
        nk = 0 if self.cfg.get("knots") is None else len(self.cfg["knots"])
        g_knots = np.zeros(max(nk, 1))
        out.g_rho = _ptr(g_rho)
        out.g_knots = _ptr(g_knots)
        _check(self.lib.pic_run_adjoint(self._h, int(n_steps), int(checkpoint_every),
                                        ctypes.c_void_p(tape.data_ptr()), nbytes, ctypes.byref(out)),
               "pic_run_adjoint")
        return dict(loss=out.loss, n_exit=out.n_exit, g_rate=out.g_rate, g_kappa=out.g_kappa, g_amp=out.g_amp,
                    g_rho=g_rho, g_knots=g_knots[:nk], forward_ms=out.forward_ms, backward_ms=out.backward_ms,
                    tape_bytes=nbytes)

    def adjoint_forward(self, n_steps, checkpoint_every=50, tape=None):
        """The checkpointed forward of the adjoint (pic_adjoint_forward): advances
        the tube and records the run for backward(); returns loss, n_exit and the
        forward's device time.  The tape (a torch uint8 tensor, allocated here when
        not given) is kept on the tube until the next adjoint_forward."""
        import torch
        nbytes = self.lib.pic_adjoint_tape_bytes(self._h, int(n_steps), int(checkpoint_every))
        if nbytes == 0:
            raise PicError(-1, "pic_adjoint_tape_bytes", self.lib.pic_last_error().decode())
        if tape is None or tape.numel() < nbytes:
            with torch.cuda.device(self.device):
                tape = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._tape = tape
        out = PicAdjointOut()
        _check(self.lib.pic_adjoint_forward(self._h, int(n_steps), int(checkpoint_every),
                                            ctypes.c_void_p(tape.data_ptr()), nbytes, ctypes.byref(out)),
               "pic_adjoint_forward")
        return dict(loss=out.loss, n_exit=out.n_exit, forward_ms=out.forward_ms, tape_bytes=nbytes)

    def backward(self, dloss=1.0):
        """The reverse sweep of the recorded forward (pic_backward), scaled by dloss."""
        out = PicAdjointOut()
        g_rho = np.zeros(self.N + 1)
        nk = 0 if self.cfg.get("knots") is None else len(self.cfg["knots"])
        g_knots = np.zeros(max(nk, 1))
        out.g_rho = _ptr(g_rho)
        out.g_knots = _ptr(g_knots)
        _check(self.lib.pic_backward(self._h, float(dloss), ctypes.byref(out)), "pic_backward")
        return dict(loss=out.loss, n_exit=out.n_exit, g_rate=out.g_rate, g_kappa=out.g_kappa, g_amp=out.g_amp,
                    g_rho=g_rho, g_knots=g_knots[:nk], forward_ms=out.forward_ms, backward_ms=out.backward_ms)

    def diagnostics(self, n_bins=0, gauss=False, fields=True, j=False, weights=False, rho=False,
                    raise_on_status=True, gauss_tol=0.0):
        N = self.N
        d = PicDiag()
        out = {}
        if fields:
            out["ez"], out["er"], out["b_phi"] = np.zeros(N), np.zeros(N + 1), np.zeros(N)
            d.ez, d.er, d.b_phi = _ptr(out["ez"]), _ptr(out["er"]), _ptr(out["b_phi"])
        if rho:
            out["rho_gj"] = np.zeros(N + 1)
            d.rho_gj = _ptr(out["rho_gj"])
        if j:
            out["j_last"] = np.zeros(N, np.int64)
            d.j_last = _ptr(out["j_last"], _pi)
        if weights:
            out["weights"] = np.zeros(N + 1, np.int64)
            d.weights = _ptr(out["weights"], _pi)
        if gauss:
            out["gauss"] = np.zeros(N + 1)
            d.gauss = _ptr(out["gauss"])
        if n_bins:
            for k, dt in (("prof_count", np.int64), ("prof_mean", np.float64), ("prof_min", np.float64),
                          ("prof_max", np.float64), ("prof_sum_lo", np.uint64), ("prof_sum_hi", np.int64)):
                out[k] = np.zeros(n_bins, dt)
            d.prof_count, d.prof_mean = _ptr(out["prof_count"], _pi), _ptr(out["prof_mean"])
            d.prof_min, d.prof_max = _ptr(out["prof_min"]), _ptr(out["prof_max"])
            d.prof_sum_lo, d.prof_sum_hi = _ptr(out["prof_sum_lo"], _pu), _ptr(out["prof_sum_hi"], _pi)
        req = PicDiagReq(int(n_bins), int(bool(gauss)), float(gauss_tol))
        rc = self.lib.pic_diagnostics(self._h, ctypes.byref(req), ctypes.byref(d))
        if rc != 0 and (rc != -9 or raise_on_status):
            _check(rc, "pic_diagnostics")
        for k in ("step", "n_alive", "n_slots", "n_injected", "n_exit", "n_absorb", "last_n_inj", "w0",
                  "status", "e_surf", "exit_sum_lo", "exit_sum_hi", "exit_gamma_sum", "gauss_max",
                  "gauss_l2", "n_slots_high"):
            out[k] = getattr(d, k)
        return out

    def read_particles(self):
        n = ctypes.c_int64(0)
        self.lib.pic_read_particles(self._h, None, None, 0, ctypes.byref(n))
        x, u = np.zeros(n.value), np.zeros(n.value)
        _check(self.lib.pic_read_particles(self._h, _ptr(x), _ptr(u), n.value, ctypes.byref(n)),
               "pic_read_particles")
        return x, u

    def write_fields(self, ez=None, er=None, b_phi=None):
        arrs = [None if a is None else np.ascontiguousarray(a, np.float64) for a in (ez, er, b_phi)]
        _check(self.lib.pic_write_fields(self._h, *[_ptr(a) for a in arrs]), "pic_write_fields")

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self.lib.pic_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h


class _TubeView(Tube):
    """A tube of a Batch (borrowed handle: no workspace, stepped by the batch)."""

    def __init__(self, batch, t):
        self.lib = batch.lib
        self.stream = batch.stream
        self.device = batch.device
        self.cfg = batch.cfgs[t]
        self.N = int(self.cfg["n_cells"])
        self._h = ctypes.c_void_p()
        _check(self.lib.pic_batch_tube(batch.handle, int(t), ctypes.byref(self._h)), "pic_batch_tube")
        self._batch = batch

    def step(self, n=1):
        raise PicError(-7, "step", "tubes of a batch are stepped through the batch")

    def close(self):
        self._h = ctypes.c_void_p()   # borrowed; released with the batch

    def __del__(self):
        pass


class Batch:
    """Many independent tubes of uneven size, stepped together: each round of
    steps plus the batched sort is captured once in a HIP graph and replayed."""

    def __init__(self, cfgs, device="cuda", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("pcpic.Batch needs a HIP GPU")
        self.lib = load()
        made = [make_params(c) for c in cfgs]
        self.cfgs = [m[2] for m in made]
        self._knots = [m[1] for m in made]
        arr = (PicParams * len(made))(*[m[0] for m in made])
        self._params = arr
        n = self.lib.pic_batch_workspace_bytes(arr, len(made))
        if n == 0:
            raise PicError(-1, "pic_batch_workspace_bytes", self.lib.pic_last_error().decode())
        self.device = torch.device(device)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
            self.ws = torch.empty(n, dtype=torch.uint8, device=self.device)
        self._h = ctypes.c_void_p()
        _check(self.lib.pic_init_batch(arr, len(made), ctypes.c_void_p(self.ws.data_ptr()), n,
                                       ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self._h)),
               "pic_init_batch")
        self.tubes = [_TubeView(self, t) for t in range(len(made))]

    @property
    def handle(self):
        return self._h

    def __len__(self):
        return len(self.tubes)

    def step(self, n=1):
        _check(self.lib.pic_step(self._h, int(n)), "pic_step")

    def step_timed(self, n):
        t = PicTiming()
        _check(self.lib.pic_step_timed(self._h, int(n), ctypes.byref(t)), "pic_step_timed")
        return {k: getattr(t, k) for k, _ in PicTiming._fields_}

    def sync(self):
        _check(self.lib.pic_sync(self._h), "pic_sync")

    def set_config(self, block, per_thread, graph=True):
        _check(self.lib.pic_batch_set_config(self._h, int(block), int(per_thread), 0 if graph else 1),
               "pic_batch_set_config")

    def get_config(self):
        v = [ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()]
        _check(self.lib.pic_batch_get_config(self._h, *[ctypes.byref(x) for x in v]), "pic_batch_get_config")
        return dict(block=v[0].value, per_thread=v[1].value, push_blocks=v[2].value, field_blocks=v[3].value)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            for t in self.tubes:
                t.close()
            self.lib.pic_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
