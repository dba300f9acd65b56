"""Python access to the serial CPU oracle (``pmp_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by ``__graft_entry__.smoke``
and by the benchmark's CPU-baseline leg; never by the library.  It does not
import the HIP package either: workloads are passed in duck-typed (any object
with ``lo, n, ghost, domain, dx, state, cic, sn, sinks, limits, r_k,
r_gauss``; Bondi-Hoyle sinks as described in ``_sinks``), particle kinds as
objects with ``fields`` and ``box_off``.

Modes: ``"f64"`` (double buffer, sequential sums in array order),
``"fix64"`` (int64 buffer on the 2^-40 grid; exact and order-free) and
``"f64r"`` (double sums with the error bound of App. A.1, each buffer element
truncated after the deposit; margin ``M`` from the workload's
``margin_bits``, default 28).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pmp_oracle.c")
_LIB = os.path.join(_HERE, "libpmp_oracle.so")
CFLAGS = ["-O2", "-std=c11", "-Wall", "-ffp-contract=off", "-fno-fast-math",
          "-shared", "-fPIC"]

F64, FIX64, F64R = 0, 1, 2
MODES = {"f64": F64, "fix64": FIX64, "f64r": F64R}
MARGIN_DEFAULT = 28
FIX_INV = 2.0 ** -40

ERRORS = {-1: "EINVAL", -2: "EOUTSIDE", -3: "EREACH", -4: "EOVERFLOW", -5: "ENOMEM",
          -6: "EOVERLAP"}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Mesh(C.Structure):
    _fields_ = [("nbox", C.c_int32), ("lo", C.c_void_p), ("n", C.c_void_p),
                ("ghost", C.c_int32), ("domain", C.c_int32 * 3), ("dx", C.c_double),
                ("nfield", C.c_int32)]


class _Cic(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p), ("m", C.c_void_p),
                ("box_off", C.c_void_p)]


class _Sn(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p), ("m", C.c_void_p),
                ("e", C.c_void_p), ("r", C.c_void_p), ("box_off", C.c_void_p)]


class _Sinks(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p), ("a", C.c_void_p),
                ("box_off", C.c_void_p), ("r_k", C.c_double), ("r_gauss", C.c_double),
                ("m", C.c_void_p), ("vx", C.c_void_p), ("vy", C.c_void_p), ("vz", C.c_void_p),
                ("rate", C.c_int32), ("G", C.c_double), ("dt", C.c_double),
                ("gamma", C.c_double), ("lam", C.c_double)]


RATE_FRACTION, RATE_BONDI = 0, 1


class _Snr(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p), ("m", C.c_void_p),
                ("e", C.c_void_p), ("vx", C.c_void_p), ("vy", C.c_void_p), ("vz", C.c_void_p),
                ("box_off", C.c_void_p), ("r_k", C.c_double), ("sub", C.c_int32),
                ("nh_per_rho", C.c_double), ("msf_coef", C.c_double),
                ("psnr_coef", C.c_double), ("eps_k", C.c_double)]


def _snr(w):
    """ctypes description of a workload's supernova remnants (kind ``snr``:
    fields x, y, z, m (ejecta mass), e (energy), vx, vy, vz; parameters in
    ``snr_params``)."""
    s, keep = _kind(w.snr, ["x", "y", "z", "m", "e", "vx", "vy", "vz"], _Snr)
    P = w.snr_params
    s.r_k, s.sub = float(P.r_k), int(P.sub)
    s.nh_per_rho, s.msf_coef = float(P.nh_per_rho), float(P.msf_coef)
    s.psnr_coef, s.eps_k = float(P.psnr_coef), float(P.eps_k)
    return s, keep


def _sinks(w):
    """ctypes sink description of a workload and the arrays it points at.
    Bondi-Hoyle workloads (``sink_rate`` 1) carry the sink fields m, vx, vy,
    vz and the scalars grav_G, dt, gamma, bhl_lambda."""
    s4, keep = _kind(w.sinks, ["x", "y", "z", "a"], _Cic)
    sk = _Sinks(s4.x, s4.y, s4.z, s4.m, s4.box_off, float(w.r_k), float(w.r_gauss))
    rate = int(getattr(w, "sink_rate", RATE_FRACTION))
    sk.rate = rate
    if rate == RATE_BONDI:
        arrs = [_f64(w.sinks.fields[k]) for k in ("m", "vx", "vy", "vz")]
        keep += arrs
        sk.m, sk.vx, sk.vy, sk.vz = (_ptr(a) for a in arrs)
        sk.G, sk.dt = float(w.grav_G), float(w.dt)
        sk.gamma, sk.lam = float(w.gamma), float(w.bhl_lambda)
    return sk, keep


class _Limits(C.Structure):
    _fields_ = [("rho_floor", C.c_double), ("rho_tr", C.c_double), ("cap", C.c_double),
                ("eint_mode", C.c_int32), ("truelove_J", C.c_double), ("G", C.c_double),
                ("gamma", C.c_double)]


class Counters(C.Structure):
    _fields_ = [("touched", C.c_int64), ("bind", C.c_int64), ("lam", C.c_int64),
                ("fall", C.c_int64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        vp, i32 = C.c_void_p, C.c_int
        L.orc_exp.restype = C.c_double
        L.orc_exp.argtypes = [C.c_double]
        L.orc_log.restype = C.c_double
        L.orc_log.argtypes = [C.c_double]
        L.orc_pow.restype = C.c_double
        L.orc_pow.argtypes = [C.c_double, C.c_double]
        L.orc_deposit_snr.argtypes = [vp, i32, vp, vp, vp, vp]
        L.orc_buffer_elems.restype = C.c_int64
        L.orc_buffer_elems.argtypes = [vp]
        L.orc_state_elems.restype = C.c_int64
        L.orc_state_elems.argtypes = [vp]
        L.orc_deposit.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.orc_deposit_r.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, i32, vp, vp, vp]
        L.orc_truncate_err.restype = C.c_double
        L.orc_truncate_err.argtypes = [C.c_double, C.c_double, i32]
        L.orc_fold.argtypes = [vp, i32, vp]
        L.orc_sink_update.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.orc_apply.argtypes = [vp, i32, vp, vp, vp, vp, vp]
        L.orc_sink_create.argtypes = [vp, i32, vp, vp, vp, C.c_double, vp, C.c_int64, vp, vp]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed: {ERRORS.get(rc, rc)}")


def exp(x: float) -> float:
    return lib().orc_exp(float(x))


class Mesh:
    """Keeps the ctypes mesh and the arrays it points at alive together."""

    def __init__(self, lo, n, ghost, domain, dx, nfield):
        self.lo = np.ascontiguousarray(np.asarray(lo, dtype=np.int32).reshape(-1, 3))
        self.n = np.ascontiguousarray(np.asarray(n, dtype=np.int32).reshape(-1, 3))
        self.ghost, self.domain, self.dx, self.nfield = int(ghost), tuple(domain), float(dx), int(nfield)
        self.c = _Mesh(self.lo.shape[0], _ptr(self.lo), _ptr(self.n), self.ghost,
                       (C.c_int32 * 3)(*self.domain), self.dx, self.nfield)

    @classmethod
    def of(cls, w):
        return cls(w.lo, w.n, w.ghost, w.domain, w.dx, w.nfield)

    @property
    def buffer_elems(self):
        return lib().orc_buffer_elems(C.byref(self.c))

    @property
    def state_elems(self):
        return lib().orc_state_elems(C.byref(self.c))

    def box_buffer(self, buf, b):
        """View of box b's buffer as [F][nz+2g][ny+2g][nx+2g]."""
        g = self.ghost
        pads = [(int(nx) + 2 * g) * (int(ny) + 2 * g) * (int(nz) + 2 * g) for nx, ny, nz in self.n]
        off = sum(pads[:b]) * self.nfield
        nx, ny, nz = (int(v) + 2 * g for v in self.n[b])
        return buf[off: off + self.nfield * nx * ny * nz].reshape(self.nfield, nz, ny, nx)


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _kind(P, names, struct):
    if P is None or P.n == 0:
        return None, []
    arrs = [_f64(P.fields[k]) for k in names]
    off = np.ascontiguousarray(np.asarray(P.box_off, dtype=np.int64))
    return struct(*[_ptr(a) for a in arrs], _ptr(off)), arrs + [off]


def _limits(L):
    return _Limits(float(L.rho_floor), float(L.rho_tr), float(L.cap), int(L.eint_mode),
                   float(getattr(L, "truelove_J", 0.0)), float(getattr(L, "G", 1.0)),
                   float(getattr(L, "gamma", 5.0 / 3.0)))


def deposit(w, mode, mesh=None, state64=None, want_racc=False):
    """Step 1. Returns (buffer, sink_w, sink_mreq), and the sinks' Gaussian
    widths r_acc as a fourth item with ``want_racc``."""
    m = MODES[mode]
    mesh = mesh or Mesh.of(w)
    keep = []
    cic, a = _kind(w.cic, ["x", "y", "z", "m"], _Cic); keep += a
    sn, a = _kind(w.sn, ["x", "y", "z", "m", "e", "r"], _Sn); keep += a
    sk = None
    nsink = 0
    if w.sinks is not None and w.sinks.n > 0:
        sk, a = _sinks(w); keep += a
        nsink = w.sinks.n
    if state64 is None:
        state64 = _f64(w.state)
    lim = _limits(w.limits)
    buf = np.empty(mesh.buffer_elems, dtype=np.int64 if m == FIX64 else np.float64)
    sw = np.zeros(max(nsink, 1))
    sm = np.zeros(max(nsink, 1))
    sr = np.zeros(max(nsink, 1))
    args = (C.byref(cic) if cic else None, C.byref(sn) if sn else None,
            C.byref(sk) if sk else None, C.byref(lim), _ptr(state64), _ptr(buf))
    if m == F64R:
        err = np.empty(mesh.buffer_elems)
        rc = lib().orc_deposit_r(C.byref(mesh.c), *args, _ptr(err), margin_of(w), _ptr(sw),
                                 _ptr(sm), _ptr(sr))
    else:
        rc = lib().orc_deposit(C.byref(mesh.c), m, *args, _ptr(sw), _ptr(sm), _ptr(sr))
    _check(rc, "deposit")
    if want_racc:
        return buf, sw[:nsink], sm[:nsink], sr[:nsink]
    return buf, sw[:nsink], sm[:nsink]


def deposit_snr(w, mode, buf, mesh=None, state64=None):
    """Supernova remnants (TIGRESS variant, Sec. 3.2.1) added to the
    deposited buffer ``buf`` in place.  Returns info [4][n]: V_snr, M_snr,
    n_H and |p_rad| per supernova."""
    mesh = mesh or Mesh.of(w)
    s, keep = _snr(w)
    if state64 is None:
        state64 = _f64(w.state)
    n = w.snr.n
    info = np.zeros((4, max(n, 1)))
    rc = lib().orc_deposit_snr(C.byref(mesh.c), MODES[mode], C.byref(s), _ptr(state64),
                               _ptr(buf), _ptr(info))
    _check(rc, "deposit_snr")
    return info[:, :n]


def has_snr(w):
    return getattr(w, "snr", None) is not None and w.snr.n > 0


def margin_of(w):
    """The reproducibility mode's safety margin M (bits) of a workload."""
    return int(getattr(w, "margin_bits", MARGIN_DEFAULT))


def truncate_err(v, err, margin):
    """The oracle's App. A.1 truncation of one value (for checks)."""
    return lib().orc_truncate_err(float(v), float(err), int(margin))


def fold(w, mode, buf, mesh=None):
    """Step 2, in place."""
    mesh = mesh or Mesh.of(w)
    _check(lib().orc_fold(C.byref(mesh.c), MODES[mode], _ptr(buf)), "fold")
    return buf


def sink_update(w, mode, buf, sink_w, sink_mreq, mesh=None, state64=None, sink_racc=None):
    """Step 4. Returns (dm, dpx, dpy, dpz) per sink.  ``sink_racc`` (Step 1's
    widths) defaults to the workload's fixed r_gauss."""
    mesh = mesh or Mesh.of(w)
    n = w.sinks.n
    sk, keep = _sinks(w)
    if state64 is None:
        state64 = _f64(w.state)
    lim = _limits(w.limits)
    outs = [np.zeros(n) for _ in range(4)]
    sw, sm = _f64(sink_w), _f64(sink_mreq)
    sr = np.full(n, float(w.r_gauss)) if sink_racc is None else _f64(sink_racc)
    rc = lib().orc_sink_update(C.byref(mesh.c), MODES[mode], _ptr(state64), _ptr(buf),
                               C.byref(sk), C.byref(lim), _ptr(sw), _ptr(sm), _ptr(sr),
                               *[_ptr(o) for o in outs])
    _check(rc, "sink_update")
    return tuple(outs)


def apply(w, mode, buf, mesh=None, state64=None, want_eta=False):
    """Steps 3 + 5. Returns (new_state_f64, eta or None, counters dict)."""
    mesh = mesh or Mesh.of(w)
    st = _f64(w.state).copy() if state64 is None else state64.copy()
    eta = np.empty(st.size // 5) if want_eta else None
    lim = _limits(w.limits)
    cnt = Counters()
    rc = lib().orc_apply(C.byref(mesh.c), MODES[mode], _ptr(st), _ptr(buf), C.byref(lim),
                         _ptr(eta), C.byref(cnt))
    _check(rc, "apply")
    return st, eta, cnt.as_dict()


def sink_create(w, mode, state64, buf, r_k, rho_tr, max_new, mesh=None, limits=None,
                existing=None):
    """Sink creation (Sec. 3.1.2) on any box layout, after a step.
    ``state64`` (float64, packed) is updated in place; ``buf`` is the folded
    buffer in the mode's type, or None.  The Truelove density is the
    constant ``rho_tr``, or per cell from ``limits`` (a Limits with
    truelove_J > 0; its rho_tr is then unused).  ``existing``: a particle kind
    (fields x, y, z and box_off) of the sinks already present, or None.
    Returns (count, out[7][max_new])."""
    mesh = mesh or Mesh.of(w)
    out = np.zeros((7, max(int(max_new), 1)))
    cnt = C.c_int64(0)
    b = None if buf is None else np.ascontiguousarray(buf)
    if limits is None:
        lim = _Limits(float(w.limits.rho_floor), float(rho_tr), float(w.limits.cap),
                      int(w.limits.eint_mode), 0.0, 1.0, 5.0 / 3.0)
    else:
        lim = _limits(limits)
    ex, keep = (None, [])
    if existing is not None and existing.n > 0:
        ex, keep = _kind(existing, ["x", "y", "z", "x"], _Cic)
        sk = _Sinks(ex.x, ex.y, ex.z, ex.m, ex.box_off, float(r_k), 1.0, None, None, None,
                    None, RATE_FRACTION, 0.0, 0.0, 1.0, 0.0)
        ex = sk
    rc = lib().orc_sink_create(C.byref(mesh.c), MODES[mode], _ptr(state64), _ptr(b),
                               C.byref(ex) if ex is not None else None, float(r_k),
                               C.byref(lim), int(max_new), _ptr(out), C.byref(cnt))
    _check(rc, "sink_create")
    return int(cnt.value), out[:, :int(max_new)]


def step(w, mode, want_eta=False):
    """One full pass: deposit, fold, sink update (before the mesh changes),
    limit + apply.  Returns a dict of every intermediate."""
    mesh = Mesh.of(w)
    s64 = _f64(w.state)
    buf, sw, sm, sr = deposit(w, mode, mesh, s64, want_racc=True)
    out = {}
    if has_snr(w):
        out["snr_info"] = deposit_snr(w, mode, buf, mesh, s64)
    pre = buf.copy()
    fold(w, mode, buf, mesh)
    out.update({"buf_deposit": pre, "buf_fold": buf, "sink_w": sw, "sink_mreq": sm,
                "sink_racc": sr})
    if w.sinks is not None and w.sinks.n > 0:
        out["sink_d"] = sink_update(w, mode, buf, sw, sm, mesh, s64, sr)
    st, eta, cnt = apply(w, mode, buf, mesh, s64, want_eta)
    out.update(state=st, eta=eta, counters=cnt)
    return out


def timed_step(w, mode="f64"):
    """Wall time (seconds, single thread) of one oracle pass: deposit, fold,
    sink update (if sinks), limit + apply; without the copies step() keeps."""
    mesh = Mesh.of(w)
    s64 = _f64(w.state)
    t0 = time.perf_counter()
    buf, sw, sm, sr = deposit(w, mode, mesh, s64, want_racc=True)
    fold(w, mode, buf, mesh)
    if w.sinks is not None and w.sinks.n > 0:
        sink_update(w, mode, buf, sw, sm, mesh, s64, sr)
    lim = _limits(w.limits)
    cnt = Counters()
    rc = lib().orc_apply(C.byref(mesh.c), MODES[mode], _ptr(s64), _ptr(buf), C.byref(lim),
                         None, C.byref(cnt))
    _check(rc, "apply")
    return time.perf_counter() - t0
