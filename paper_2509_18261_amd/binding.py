"""ctypes binding for libpmp.so (include/pmp.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of the library.  Functions keep the C names (``pmp_create``, ``pmp_deposit``
...) and take PyTorch CUDA tensors where the C side takes device pointers;
``Context`` bundles a layout with the tensors of one workload.

Importing this module loads the library and raises if it is missing: there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpmp.so")

PMP_ACC_F32, PMP_ACC_F64, PMP_ACC_FIX64, PMP_ACC_F64R = 0, 1, 2, 3
MARGIN_DEFAULT = 28  # PMP_ACC_F64R safety margin (bits) unless the workload sets margin_bits
PMP_STATE_F32, PMP_STATE_F64 = 0, 1
ACC = {"f32": PMP_ACC_F32, "f64": PMP_ACC_F64, "fix64": PMP_ACC_FIX64, "f64r": PMP_ACC_F64R}
FLAGS = {0x1: "OUTSIDE", 0x2: "REACH", 0x4: "OVERFLOW", 0x8: "NAN", 0x10: "FLOOR",
         0x20: "CAPACITY"}
ERRORS = {-1: "EINVAL", -2: "ERANGE", -3: "EDEVICE", -4: "ENOMEM", -5: "EUNSUPPORTED"}


class PmpError(RuntimeError):
    def __init__(self, code, fn, msg):
        super().__init__(f"{fn}: {ERRORS.get(code, code)}: {msg}")
        self.code = code


class pmp_layout(C.Structure):
    _fields_ = [("nbox", C.c_int32), ("lo", C.c_void_p), ("n", C.c_void_p),
                ("ghost", C.c_int32), ("domain", C.c_int32 * 3), ("dx", C.c_double),
                ("acc", C.c_int32), ("state", C.c_int32), ("with_sinks", C.c_int32),
                ("channels", C.c_int32), ("margin_bits", C.c_int32)]


# buffer channel bits (pmp_layout.channels): bit f is channel f of rho, px, py, pz, E, K
PMP_CH_RHO, PMP_CH_MOM, PMP_CH_E, PMP_CH_K = 0x1, 0xE, 0x10, 0x20


class pmp_cic(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p), ("m", C.c_void_p),
                ("n", C.c_int64), ("box_off", C.c_void_p)]


class pmp_sn(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p), ("m", C.c_void_p),
                ("e", C.c_void_p), ("r", C.c_void_p), ("n", C.c_int64), ("box_off", C.c_void_p),
                ("r_max", C.c_double)]


class pmp_snr(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p), ("m", C.c_void_p),
                ("e", C.c_void_p), ("vx", C.c_void_p), ("vy", C.c_void_p), ("vz", C.c_void_p),
                ("n", C.c_int64), ("box_off", C.c_void_p), ("r_k", C.c_double),
                ("sub", C.c_int32), ("nh_per_rho", C.c_double), ("msf_coef", C.c_double),
                ("psnr_coef", C.c_double), ("eps_k", C.c_double)]


PMP_SINK_FRACTION, PMP_SINK_BONDI = 0, 1


class pmp_sinks(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p), ("a", C.c_void_p),
                ("n", C.c_int64), ("box_off", C.c_void_p), ("r_k", C.c_double),
                ("r_gauss", C.c_double), ("rate", C.c_int32),
                ("m", C.c_void_p), ("vx", C.c_void_p), ("vy", C.c_void_p), ("vz", C.c_void_p),
                ("G", C.c_double), ("dt", C.c_double), ("gamma", C.c_double),
                ("lambda_", C.c_double)]


class pmp_limits(C.Structure):
    _fields_ = [("rho_floor", C.c_double), ("rho_tr", C.c_double), ("cap", C.c_double),
                ("eint_mode", C.c_int32), ("truelove_J", C.c_double), ("G", C.c_double),
                ("gamma", C.c_double)]


def limits_of(L, rho_tr=None):
    """pmp_limits from a workloads.Limits (rho_tr overrides its constant)."""
    return pmp_limits(float(L.rho_floor), float(L.rho_tr if rho_tr is None else rho_tr),
                      float(L.cap), int(L.eint_mode), float(getattr(L, "truelove_J", 0.0)),
                      float(getattr(L, "G", 1.0)), float(getattr(L, "gamma", 5.0 / 3.0)))


class pmp_status(C.Structure):
    _fields_ = [("flags", C.c_uint32), ("reserved", C.c_uint32), ("touched", C.c_int64),
                ("bind", C.c_int64), ("lam", C.c_int64), ("fall", C.c_int64)]

    def as_dict(self):
        d = {k: int(getattr(self, k)) for k, _ in self._fields_ if k != "reserved"}
        d["flag_names"] = [v for b, v in FLAGS.items() if self.flags & b]
        return d


class pmp_tuning(C.Structure):
    _fields_ = [("deposit_path", C.c_int32), ("tile_x", C.c_int32), ("tile_yz", C.c_int32),
                ("tile_block", C.c_int32), ("block", C.c_int32), ("grid_per_cu", C.c_int32),
                ("sn_lanes", C.c_int32), ("tile_grid_per_cu", C.c_int32),
                ("chunk_cic", C.c_int32), ("chunk_sn", C.c_int32),
                ("fuse_apply", C.c_int32), ("count_lanes", C.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


NPHASE = 10
PHASES = ["zero", "cic", "sn", "sink_deposit", "fold", "sink_update", "apply", "bin", "tile",
          "snr"]

_VP, _I = C.c_void_p, C.c_int
# (name, restype, argtypes) for every exported function of include/pmp.h
SIGNATURES = [
    ("pmp_create", _I, [C.POINTER(C.c_void_p), C.POINTER(pmp_layout)]),
    ("pmp_destroy", None, [_VP]),
    ("pmp_sizes", _I, [_VP, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    ("pmp_workspace_size", _I, [_VP, C.c_int64, C.c_int64, C.c_double, C.c_int64,
                                C.POINTER(C.c_size_t)]),
    ("pmp_set_workspace", _I, [_VP, _VP, C.c_size_t]),
    ("pmp_deposit", _I, [_VP, _VP, _VP, C.POINTER(pmp_cic), C.POINTER(pmp_sn),
                         C.POINTER(pmp_sinks), C.POINTER(pmp_limits), _VP]),
    ("pmp_deposit_snr", _I, [_VP, _VP, _VP, C.POINTER(pmp_snr), _VP, _VP]),
    ("pmp_ghost_fold", _I, [_VP, _VP, _VP]),
    ("pmp_sink_update", _I, [_VP, _VP, _VP, C.POINTER(pmp_sinks), C.POINTER(pmp_limits),
                             _VP, _VP, _VP, _VP, _VP]),
    ("pmp_apply", _I, [_VP, _VP, _VP, C.POINTER(pmp_limits), _VP, _VP]),
    ("pmp_sink_create", _I, [_VP, _VP, _VP, C.POINTER(pmp_sinks), C.c_double,
                             C.POINTER(pmp_limits), C.c_int64, _VP, _VP, _VP]),
    ("pmp_sink_create_noalloc", _I, [_VP, _VP, _VP, C.POINTER(pmp_sinks), C.c_double,
                                     C.POINTER(pmp_limits), C.c_int64, _VP, _VP, _VP]),
    ("pmp_step", _I, [_VP, _VP, _VP, C.POINTER(pmp_cic), C.POINTER(pmp_sn),
                      C.POINTER(pmp_sinks), C.POINTER(pmp_limits), _VP, _VP]),
    ("pmp_step_per_box", _I, [_VP, _VP, _VP, C.POINTER(pmp_cic), C.POINTER(pmp_sn),
                              C.POINTER(pmp_limits), _VP, _VP, _VP]),
    ("pmp_graph_build", _I, [_VP, _I, _VP, _VP, C.POINTER(pmp_cic), C.POINTER(pmp_sn),
                             C.POINTER(pmp_sinks), C.POINTER(pmp_limits), _VP, _VP]),
    ("pmp_graph_launch", _I, [_VP, _VP]),
    ("pmp_get_status", _I, [_VP, C.POINTER(pmp_status), _I]),
    ("pmp_get_tuning", _I, [_VP, C.POINTER(pmp_tuning)]),
    ("pmp_set_tuning", _I, [_VP, C.POINTER(pmp_tuning)]),
    ("pmp_autotune", _I, [_VP, _VP, _VP, C.POINTER(pmp_cic), C.POINTER(pmp_sn),
                          C.POINTER(pmp_sinks), C.POINTER(pmp_limits), _VP, _VP,
                          C.POINTER(C.c_double)]),
    ("pmp_profile_begin", _I, [_VP, _I]),
    ("pmp_profile_end", _I, [_VP, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    ("pmp_stream_copy", _I, [_VP, _VP, C.c_size_t, _VP]),
    ("pmp_copy_bench", _I, [_VP, _VP, C.c_size_t, _I, _VP]),
    ("pmp_atomic_bench", _I, [_VP, C.c_int64, _I, _I, C.c_int64, _VP]),
    ("pmp_last_error", C.c_char_p, []),
]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libpmp.so not built ({LIB_PATH}); run __graft_entry__.build()")
    lib = C.CDLL(LIB_PATH)
    for name, res, args in SIGNATURES:
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def _call(name, *args):
    rc = getattr(lib, name)(*args)
    if rc != 0:
        raise PmpError(rc, name, lib.pmp_last_error().decode())
    return rc


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


# ------------------------------------------------------------------ objects

class Context:
    """A pmp context plus the device tensors of one workload.

    ``w`` is a workload (paper_2509_18261_amd.workloads.Workload); ``acc`` is
    "f32", "f64" or "fix64".  State type follows ``w.state.dtype``.
    ``channels``: "all" (rho, p, E, and K with sinks), "auto" (only the
    channels the workload's particle kinds deposit into) or PMP_CH_* bits.
    ``fields`` lists the channels present, in buffer order, as indices
    0..5 = rho, px, py, pz, E, K."""

    def __init__(self, w, acc="fix64", device="cuda", channels="all"):
        import torch
        self.w = w
        self.acc = acc
        self.device = device
        self.lo = np.ascontiguousarray(np.asarray(w.lo, dtype=np.int32))
        self.n = np.ascontiguousarray(np.asarray(w.n, dtype=np.int32))
        st_dtype = np.dtype(w.state.dtype)
        self.state_type = PMP_STATE_F32 if st_dtype == np.float32 else PMP_STATE_F64
        with_sinks = 1 if w.nfield == 6 else 0
        ch = channel_bits(w, channels)
        full = ch if ch else (0x1F | (PMP_CH_K if with_sinks else 0))
        self.fields = [f for f in range(6) if full >> f & 1]
        self.layout = pmp_layout(w.nbox, self.lo.ctypes.data, self.n.ctypes.data, w.ghost,
                                 (C.c_int32 * 3)(*w.domain), float(w.dx), ACC[acc],
                                 self.state_type, with_sinks, ch,
                                 int(getattr(w, "margin_bits", MARGIN_DEFAULT)))
        h = C.c_void_p()
        _call("pmp_create", C.byref(h), C.byref(self.layout))
        self.h = h
        se, be, oc = C.c_int64(), C.c_int64(), C.c_int64()
        _call("pmp_sizes", self.h, C.byref(se), C.byref(be), C.byref(oc))
        self.state_elems, self.buffer_elems, self.owned_cells = se.value, be.value, oc.value
        assert self.state_elems == w.state.size, "state size does not match the layout"
        tdt = torch.float32 if self.state_type == PMP_STATE_F32 else torch.float64
        bdt = {"f32": torch.float32, "f64": torch.float64, "fix64": torch.int64,
               "f64r": torch.float64}[acc]
        self.state = torch.from_numpy(np.ascontiguousarray(w.state)).to(device)
        assert self.state.dtype == tdt
        self.buf = torch.empty(self.buffer_elems, dtype=bdt, device=device)
        self.lim = limits_of(w.limits)
        self._keep = []
        self.cic = self._kind(w.cic, ["x", "y", "z", "m"], pmp_cic)
        self.sn = self._kind(w.sn, ["x", "y", "z", "m", "e", "r"], pmp_sn)
        if self.sn is not None:
            self.sn.r_max = float(np.max(w.sn.fields["r"]))
        rate = int(getattr(w, "sink_rate", PMP_SINK_FRACTION))
        names = ["x", "y", "z", "a"] + (["m", "vx", "vy", "vz"] if rate == PMP_SINK_BONDI else [])
        self.sinks = self._kind(w.sinks, names, pmp_sinks)
        self.snr = self._kind(getattr(w, "snr", None),
                              ["x", "y", "z", "m", "e", "vx", "vy", "vz"], pmp_snr)
        if self.snr is not None:
            P = w.snr_params
            self.snr.r_k, self.snr.sub = float(P.r_k), int(P.sub)
            self.snr.nh_per_rho, self.snr.msf_coef = float(P.nh_per_rho), float(P.msf_coef)
            self.snr.psnr_coef, self.snr.eps_k = float(P.psnr_coef), float(P.eps_k)
        self.sink_out = None
        if self.sinks is not None:
            self.sinks.r_k = float(w.r_k)
            self.sinks.r_gauss = float(w.r_gauss)
            self.sinks.rate = rate
            if rate == PMP_SINK_BONDI:
                self.sinks.G, self.sinks.dt = float(w.grav_G), float(w.dt)
                self.sinks.gamma, self.sinks.lambda_ = float(w.gamma), float(w.bhl_lambda)
            self.sink_out = torch.zeros(4 * w.sinks.n, dtype=torch.float64, device=device)

    def _kind(self, P, names, struct):
        import torch
        if P is None or P.n == 0:
            return None
        ts = [torch.from_numpy(np.ascontiguousarray(P.fields[k], dtype=np.float64)).to(self.device)
              for k in names]
        off = torch.from_numpy(np.ascontiguousarray(P.box_off, dtype=np.int64)).to(self.device)
        self._keep += ts + [off]
        vals = [C.c_void_p(t.data_ptr()) for t in ts]
        s = struct()
        for k, v in zip(names, vals):
            setattr(s, k, v)
        s.n = P.n
        s.box_off = C.c_void_p(off.data_ptr())
        return s

    # ---------------------------------------------------------- workspace
    def workspace_size(self, max_cic=None, max_sn=None, max_sn_radius=None, max_sinks=None):
        """Device bytes a caller-owned workspace needs (default: this workload)."""
        w = self.w
        nc = (w.cic.n if w.cic is not None else 0) if max_cic is None else max_cic
        ns = (w.sn.n if w.sn is not None else 0) if max_sn is None else max_sn
        r = (self.sn.r_max if self.sn is not None else 0.0) if max_sn_radius is None else max_sn_radius
        nk = (w.sinks.n if w.sinks is not None else 0) if max_sinks is None else max_sinks
        out = C.c_size_t()
        _call("pmp_workspace_size", self.h, int(nc), int(ns), float(r), int(nk), C.byref(out))
        return out.value

    def set_workspace(self, ws):
        """Carve every scratch array from ``ws`` (a CUDA tensor, kept alive
        here), or return to library-owned scratch with None."""
        if ws is None:
            _call("pmp_set_workspace", self.h, None, 0)
        else:
            _call("pmp_set_workspace", self.h, _ptr(ws), ws.numel() * ws.element_size())
        self.workspace = ws

    # -------------------------------------------------------------- calls
    def _r(self, s):
        return None if s is None else C.byref(s)

    def reset_state(self):
        import torch
        self.state.copy_(torch.from_numpy(np.ascontiguousarray(self.w.state)).to(self.device))

    def deposit(self, stream=None):
        _call("pmp_deposit", self.h, _ptr(self.buf), _ptr(self.state), self._r(self.cic),
              self._r(self.sn), self._r(self.sinks), C.byref(self.lim), _stream(stream))

    def deposit_snr(self, info=None, stream=None):
        """Add the supernova remnants (TIGRESS variant) to the deposited buffer."""
        if self.snr is None:
            return
        _call("pmp_deposit_snr", self.h, _ptr(self.buf), _ptr(self.state), C.byref(self.snr),
              _ptr(info), _stream(stream))

    def ghost_fold(self, stream=None):
        _call("pmp_ghost_fold", self.h, _ptr(self.buf), _stream(stream))

    def sink_update(self, stream=None):
        if self.sinks is None:
            return
        n = self.w.sinks.n
        o = self.sink_out
        _call("pmp_sink_update", self.h, _ptr(self.state), _ptr(self.buf), C.byref(self.sinks),
              C.byref(self.lim), _ptr(o[0:n]), _ptr(o[n:2 * n]), _ptr(o[2 * n:3 * n]),
              _ptr(o[3 * n:]), _stream(stream))

    def apply(self, eta=None, stream=None):
        _call("pmp_apply", self.h, _ptr(self.state), _ptr(self.buf), C.byref(self.lim),
              _ptr(eta), _stream(stream))

    def sink_create(self, r_k, rho_tr, max_new, buf=True, limits=None, existing=None,
                    stream=None):
        """Sink creation after a step (state updated in place).  Returns the
        device arrays (out [7][max_new], work [2 max_new + 1]); work[0] is the
        number of qualifying cells.  ``buf=False`` passes no buffer.  The
        Truelove density is the constant ``rho_tr``, or comes from ``limits``
        (a workloads.Limits, per cell when its truelove_J > 0).  ``existing``:
        "workload" (this workload's sinks), a particle kind with x, y, z, or
        None."""
        import torch
        out = torch.zeros(7 * max(int(max_new), 1), dtype=torch.float64, device=self.device)
        work = torch.zeros(2 * int(max_new) + 1, dtype=torch.int64, device=self.device)
        lim = limits_of(self.w.limits, rho_tr) if limits is None else limits_of(limits)
        ex = self._positions(existing)
        _call("pmp_sink_create", self.h, _ptr(self.state), _ptr(self.buf) if buf else None,
              None if ex is None else C.byref(ex), float(r_k), C.byref(lim), int(max_new),
              _ptr(out), _ptr(work), _stream(stream))
        return out, work

    def sink_create_noalloc(self, r_k, rho_tr, max_new, buf=True, limits=None, existing=None,
                            stream=None):
        """pmp_sink_create_noalloc: as sink_create, with the library's static
        scratch; returns (out [7][max_new], count [1]) device arrays."""
        import torch
        out = torch.zeros(7 * max(int(max_new), 1), dtype=torch.float64, device=self.device)
        count = torch.zeros(1, dtype=torch.int64, device=self.device)
        lim = limits_of(self.w.limits, rho_tr) if limits is None else limits_of(limits)
        ex = self._positions(existing)
        _call("pmp_sink_create_noalloc", self.h, _ptr(self.state),
              _ptr(self.buf) if buf else None, None if ex is None else C.byref(ex), float(r_k),
              C.byref(lim), int(max_new), _ptr(out), _ptr(count), _stream(stream))
        return out, count

    def _positions(self, existing):
        """pmp_sinks holding only the positions of ``existing`` (see sink_create)."""
        import torch
        if existing is None:
            return None
        if isinstance(existing, str):
            assert existing == "workload"
            return self.sinks
        if existing.n == 0:
            return None
        ts = [torch.from_numpy(np.ascontiguousarray(existing.fields[k], dtype=np.float64))
              .to(self.device) for k in ("x", "y", "z")]
        self._keep += ts
        s = pmp_sinks()
        s.x, s.y, s.z = (C.c_void_p(t.data_ptr()) for t in ts)
        s.n = existing.n
        return s

    def step(self, stream=None):
        _call("pmp_step", self.h, _ptr(self.state), _ptr(self.buf), self._r(self.cic),
              self._r(self.sn), self._r(self.sinks), C.byref(self.lim), _ptr(self.sink_out),
              _stream(stream))

    def step_per_box(self, stream=None):
        """The per-box launch baseline (one launch per box per kernel)."""
        if not hasattr(self, "_host_off"):
            self._host_off = [None if P is None or P.n == 0 else
                              np.ascontiguousarray(P.box_off, dtype=np.int64)
                              for P in (self.w.cic, self.w.sn)]
        co, so = self._host_off
        _call("pmp_step_per_box", self.h, _ptr(self.state), _ptr(self.buf), self._r(self.cic),
              self._r(self.sn), C.byref(self.lim),
              None if co is None else C.c_void_p(co.ctypes.data),
              None if so is None else C.c_void_p(so.ctypes.data), _stream(stream))

    def graph_build(self, nsteps, stream=None):
        _call("pmp_graph_build", self.h, int(nsteps), _ptr(self.state), _ptr(self.buf),
              self._r(self.cic), self._r(self.sn), self._r(self.sinks), C.byref(self.lim),
              _ptr(self.sink_out), _stream(stream))

    def graph_launch(self, stream=None):
        _call("pmp_graph_launch", self.h, _stream(stream))

    def status(self, reset=True):
        st = pmp_status()
        _call("pmp_get_status", self.h, C.byref(st), 1 if reset else 0)
        return st.as_dict()

    def tuning(self):
        t = pmp_tuning()
        _call("pmp_get_tuning", self.h, C.byref(t))
        return t

    def set_tuning(self, **kw):
        t = self.tuning()
        for k, v in kw.items():
            setattr(t, k, int(v))
        _call("pmp_set_tuning", self.h, C.byref(t))
        return t

    def autotune(self, stream=None):
        best = C.c_double()
        _call("pmp_autotune", self.h, _ptr(self.state), _ptr(self.buf), self._r(self.cic),
              self._r(self.sn), self._r(self.sinks), C.byref(self.lim), _ptr(self.sink_out),
              _stream(stream), C.byref(best))
        return best.value

    def profile_begin(self, max_launches):
        _call("pmp_profile_begin", self.h, int(max_launches))

    def profile_end(self):
        """Summed kernel ms and launch count per phase, as a dict."""
        ms = (C.c_double * NPHASE)()
        cnt = (C.c_int64 * NPHASE)()
        _call("pmp_profile_end", self.h, ms, cnt)
        return {PHASES[p]: (ms[p], cnt[p]) for p in range(NPHASE) if cnt[p] > 0}

    def close(self):
        if getattr(self, "h", None):
            lib.pmp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def channel_bits(w, channels):
    """pmp_layout.channels for a workload: "all" -> 0, "auto" -> the channels
    its particle kinds deposit into (CIC rho; supernovae rho and E; sinks K)."""
    if channels == "all":
        return 0
    if channels != "auto":
        return int(channels)
    ch = 0
    if w.cic is not None and w.cic.n > 0:
        ch |= PMP_CH_RHO
    if w.sn is not None and w.sn.n > 0:
        ch |= PMP_CH_RHO | PMP_CH_E
    if w.nfield == 6:
        ch |= PMP_CH_K
    if getattr(w, "snr", None) is not None and w.snr.n > 0:
        ch |= PMP_CH_RHO | PMP_CH_MOM | PMP_CH_E
    return ch or PMP_CH_RHO


def stream_copy(dst, src, stream=None):
    _call("pmp_stream_copy", _ptr(dst), _ptr(src), dst.numel() * dst.element_size(),
          _stream(stream))


def copy_bench(dst, src, variant, stream=None):
    _call("pmp_copy_bench", _ptr(dst), _ptr(src), dst.numel() * dst.element_size(),
          int(variant), _stream(stream))


ATOMIC_TYPES = {"int64": 0, "f32": 1, "f64": 2}
ATOMIC_PATTERNS = {"coalesced": 0, "scattered": 1, "same_address": 2}


def atomic_bench(dst, type_name, pattern, n_ops, stream=None):
    """n_ops atomic adds into the tensor dst (its element count a power of two)."""
    _call("pmp_atomic_bench", _ptr(dst), dst.numel(), ATOMIC_TYPES[type_name],
          ATOMIC_PATTERNS[pattern], int(n_ops), _stream(stream))


def buffer_to_numpy(ctx, t=None):
    """Device buffer as a host numpy array (float64 view for float modes)."""
    return (ctx.buf if t is None else t).cpu().numpy()


INV_Q = math.ldexp(1.0, -40)
