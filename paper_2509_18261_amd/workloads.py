"""Seeded synthetic workloads for the particle-mesh-particle path.

This module draws inputs only: box layouts, gas states and particle lists.  It
holds none of the method's arithmetic (no deposition, folding or limiting), so
that both the HIP path and the serial oracle can be fed from it without sharing
any computation.

Units: positions are in cell units of the global index space, a particle at
``x`` lies in cell ``floor(x)``; ``dx`` is the cell edge so that ``V = dx**3``.
Memory layout (the library's interface, Sec. 2.1 "Formulation of the problem"):

* boxes are listed in order; box ``b`` owns global cells ``[lo_b, lo_b+n_b)``
  (x, y, z order in the arrays);
* the state is the concatenation over boxes of ``[5][nz][ny][nx]`` arrays
  (rho, px, py, pz, E), x fastest;
* a particle list of one kind is grouped by box, with a CSR offset array
  ``box_off`` of length ``nbox+1``.

Workloads follow the synthetic stand-ins for the paper's galaxy run
(Sec. 4.6): the paper's AGORA initial condition is not available, so each
workload is a seeded draw with the shape, sizes and clustering of its row in
the design notes (uniform, Plummer-clustered, and a batched AMR level).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

NSTATE = 5  # rho, px, py, pz, E


@dataclasses.dataclass
class Limits:
    rho_floor: float = 1e-10
    rho_tr: float = math.inf   # Truelove density; +inf disables it
    cap: float = 0.25          # largest removed fraction of a cell's mass per step
    eint_mode: int = 0         # 0: e_int >= 0, 1: specific e_int may not drop
    # truelove_J > 0: each cell's Truelove density from its own sound speed
    # (Jeans number J, gravitational constant G, adiabatic index gamma);
    # rho_tr is then unused
    truelove_J: float = 0.0
    G: float = 1.0
    gamma: float = 5.0 / 3.0


# Code units of the supernova-remnant workloads: mass 1 Msun, length one
# cell of 4 pc, velocity 10 km/s.  Then a code density of 1 is
# 1 Msun / (4 pc)^3 = 1.058e-24 g cm^-3, i.e. n_H = 0.4518 cm^-3 with
# mu_H = 1.4 m_H; 1e51 erg is 5.028e5 code energy units; the paper's
# shell-formation mass at n_H = 1 is 1679 Msun and its terminal momentum
# 2.8e5 Msun km/s = 2.8e4 code units; the ejecta mass is 10 Msun.
SNR_NH_PER_RHO = 0.4518
SNR_E_SN = 5.028e5
SNR_M_EJ = 10.0


@dataclasses.dataclass
class SnrParams:
    """Parameters of the TIGRESS-variant supernova deposit (code units)."""
    r_k: float = 3.0              # kernel radius (cells); 3 dx in the paper
    sub: int = 4                  # sample points per axis for the covered fraction
    nh_per_rho: float = SNR_NH_PER_RHO   # n_H (cm^-3) per unit code density
    msf_coef: float = 1679.0      # shell-formation mass at n_H = 1 cm^-3
    psnr_coef: float = 2.8e4      # terminal momentum at n_H = 1 cm^-3
    eps_k: float = 0.28           # kinetic fraction of the Sedov-Taylor phase


@dataclasses.dataclass
class Particles:
    """One particle kind, grouped by box.  Fields are float64 arrays."""
    fields: dict
    box_off: np.ndarray  # int64 [nbox+1]

    @property
    def n(self) -> int:
        return int(self.box_off[-1])


@dataclasses.dataclass
class Workload:
    name: str
    domain: tuple            # (nx, ny, nz)
    lo: np.ndarray           # int32 [nbox, 3]
    n: np.ndarray            # int32 [nbox, 3]
    ghost: int
    dx: float
    state: np.ndarray        # float32 or float64, packed per box
    cic: Particles | None = None
    sn: Particles | None = None
    sinks: Particles | None = None
    r_k: float = 4.0         # sink kernel radius (cells)
    r_gauss: float = 2.0     # sink Gaussian width (cells), fraction rate
    limits: Limits = dataclasses.field(default_factory=Limits)
    # sink request rate: 0 = fraction ``a`` of the kernel gas mass, 1 =
    # Bondi-Hoyle (sink fields m, vx, vy, vz and the scalars below)
    sink_rate: int = 0
    grav_G: float = 1.0      # gravitational constant, code units
    dt: float = 0.05         # time step
    gamma: float = 5.0 / 3.0  # adiabatic index of the gas
    bhl_lambda: float = math.exp(1.5) / 4.0  # isothermal value used throughout the paper
    # supernova remnants with the TIGRESS-variant deposit (fields x, y, z,
    # m (ejecta mass), e (energy), vx, vy, vz)
    snr: Particles | None = None
    snr_params: SnrParams = dataclasses.field(default_factory=SnrParams)

    @property
    def nbox(self) -> int:
        return int(self.lo.shape[0])

    @property
    def nfield(self) -> int:
        return 6 if self.sinks is not None and self.sinks.n > 0 else 5

    @property
    def owned_cells(self) -> int:
        return int(np.prod(self.n.astype(np.int64), axis=1).sum())

    def box_state(self, b: int) -> np.ndarray:
        """View of box ``b``'s state as [5][nz][ny][nx]."""
        sizes = np.prod(self.n.astype(np.int64), axis=1)
        off = int(sizes[:b].sum()) * NSTATE
        nx, ny, nz = (int(v) for v in self.n[b])
        return self.state[off: off + NSTATE * nx * ny * nz].reshape(NSTATE, nz, ny, nx)

    def with_state(self, state: np.ndarray) -> "Workload":
        return dataclasses.replace(self, state=state)


# --------------------------------------------------------------------------- draws

def _wrap(x: np.ndarray, n: float) -> np.ndarray:
    y = np.mod(x, n)
    return np.where(y >= n, 0.0, y)


def plummer(rng: np.random.Generator, count: int, a: float, centre, domain) -> np.ndarray:
    """Positions [count, 3] from a Plummer sphere of scale radius ``a``."""
    X = rng.random(count)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = a / np.sqrt(np.power(X, -2.0 / 3.0) - 1.0)
    r = np.where(np.isfinite(r), r, 0.0)
    mu = 2.0 * rng.random(count) - 1.0
    phi = 2.0 * math.pi * rng.random(count)
    s = np.sqrt(np.maximum(0.0, 1.0 - mu * mu))
    d = np.stack([s * np.cos(phi), s * np.sin(phi), mu], axis=1)
    pos = np.asarray(centre, dtype=np.float64)[None, :] + r[:, None] * d
    for ax in range(3):
        pos[:, ax] = _wrap(pos[:, ax], float(domain[ax]))
    return pos


def uniform_positions(rng: np.random.Generator, count: int, domain) -> np.ndarray:
    pos = rng.random((count, 3)) * np.asarray(domain, dtype=np.float64)[None, :]
    for ax in range(3):
        pos[:, ax] = _wrap(pos[:, ax], float(domain[ax]))
    return pos


def clumped_positions(rng, count, domain, nclump=32, a=8.0) -> np.ndarray:
    """Half uniform, half split evenly over ``nclump`` Plummer clumps."""
    nu = count // 2
    nc = count - nu
    parts = [uniform_positions(rng, nu, domain)]
    centres = rng.random((nclump, 3)) * np.asarray(domain, dtype=np.float64)[None, :]
    per = np.full(nclump, nc // nclump)
    per[: nc - per.sum()] += 1
    for c in range(nclump):
        parts.append(plummer(rng, int(per[c]), a, centres[c], domain))
    pos = np.concatenate(parts, axis=0)
    return pos[rng.permutation(pos.shape[0])]


def gas_state(rng, ncell: int, dtype, sigma_lnrho=1.0, sigma_v=0.3) -> np.ndarray:
    """[5, ncell] log-normal density, Gaussian velocity, specific e_int = 1.

    Every value is representable in ``dtype``; E is built from the rounded
    density and momentum so that it is consistent in that precision."""
    rho = np.exp(sigma_lnrho * rng.standard_normal(ncell)).astype(dtype)
    v = sigma_v * rng.standard_normal((3, ncell))
    p = (rho.astype(np.float64)[None, :] * v).astype(dtype)
    r64 = rho.astype(np.float64)
    p64 = p.astype(np.float64)
    E = (r64 + 0.5 * (p64 * p64).sum(axis=0) / r64).astype(dtype)
    return np.concatenate([rho[None], p, E[None]], axis=0)


def pack_by_box(fields: np.ndarray, n: np.ndarray) -> np.ndarray:
    """Lay a [5, ncell] draw out in the packed per-box order (each box's
    [5][nz][ny][nx] block in turn)."""
    sizes = np.prod(np.asarray(n, dtype=np.int64), axis=1)
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    return np.concatenate([fields[:, int(o): int(o + s)].reshape(-1)
                           for o, s in zip(offs, sizes)])


def uniform_state(ncell: int, dtype, rho=1.0, E=1.0) -> np.ndarray:
    s = np.zeros((5, ncell), dtype=dtype)
    s[0] = rho
    s[4] = E
    return s


# ------------------------------------------------------------------ layouts

def single_box(nx, ny=None, nz=None):
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    lo = np.zeros((1, 3), dtype=np.int32)
    n = np.array([[nx, ny, nz]], dtype=np.int32)
    return (nx, ny, nz), lo, n


def rectilinear(edges_x, edges_y, edges_z):
    """Boxes tiling the periodic domain on a rectilinear grid.

    Box index b = (kz * nby + jy) * nbx + ix.  Returns domain, lo, n and the
    per-axis cumulative edges (for locating a particle's box)."""
    ex, ey, ez = (np.asarray(e, dtype=np.int64) for e in (edges_x, edges_y, edges_z))
    cx, cy, cz = (np.concatenate([[0], np.cumsum(e)]) for e in (ex, ey, ez))
    lo, n = [], []
    for kz in range(len(ez)):
        for jy in range(len(ey)):
            for ix in range(len(ex)):
                lo.append([cx[ix], cy[jy], cz[kz]])
                n.append([ex[ix], ey[jy], ez[kz]])
    domain = (int(cx[-1]), int(cy[-1]), int(cz[-1]))
    return domain, np.asarray(lo, np.int32), np.asarray(n, np.int32), (cx, cy, cz)


def _group_by_box(pos: np.ndarray, fields: dict, cuts, nbox_axes) -> Particles:
    """Sort particles by the rectilinear box that holds floor(x)."""
    cx, cy, cz = cuts
    nbx, nby, nbz = nbox_axes
    cell = np.floor(pos).astype(np.int64)
    ix = np.searchsorted(cx, cell[:, 0], side="right") - 1
    jy = np.searchsorted(cy, cell[:, 1], side="right") - 1
    kz = np.searchsorted(cz, cell[:, 2], side="right") - 1
    box = (kz * nby + jy) * nbx + ix
    order = np.argsort(box, kind="stable")
    counts = np.bincount(box, minlength=nbx * nby * nbz)
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    out = {"x": np.ascontiguousarray(pos[order, 0]),
           "y": np.ascontiguousarray(pos[order, 1]),
           "z": np.ascontiguousarray(pos[order, 2])}
    for k, v in fields.items():
        out[k] = np.ascontiguousarray(np.asarray(v, dtype=np.float64)[order])
    return Particles(out, off)


def _one_box(pos: np.ndarray, fields: dict) -> Particles:
    out = {"x": np.ascontiguousarray(pos[:, 0]), "y": np.ascontiguousarray(pos[:, 1]),
           "z": np.ascontiguousarray(pos[:, 2])}
    for k, v in fields.items():
        out[k] = np.ascontiguousarray(np.asarray(v, dtype=np.float64))
    return Particles(out, np.array([0, pos.shape[0]], dtype=np.int64))


def cic_fields(rng, count):
    return {"m": rng.uniform(0.1, 1.0, count)}


def sn_fields(count, radius, m=1e-2, e=1.0):
    return {"m": np.full(count, m), "e": np.full(count, e), "r": np.full(count, float(radius))}


# ---------------------------------------------------------------- workloads

def c1(seed: int = 1) -> Workload:
    """32^3 periodic box, FP64 uniform gas, 8 CIC + 8 SN (r = 2), g = 2."""
    rng = np.random.default_rng(seed)
    domain, lo, n = single_box(32)
    state = uniform_state(32 ** 3, np.float64).reshape(-1)
    pc = uniform_positions(rng, 8, domain)
    cic = _one_box(pc, cic_fields(rng, 8))
    ps = uniform_positions(rng, 8, domain)
    sn = _one_box(ps, sn_fields(8, 2.0))
    return Workload("c1_32cube_fp64", domain, lo, n, 2, 1.0, state, cic=cic, sn=sn)


def c2(seed: int = 2, nx: int = 256, n_cic: int | None = None, n_sn: int | None = None,
       dtype=np.float32) -> Workload:
    """Uniform CIC + SN (r = 4) over a log-normal gas, g = 4."""
    rng = np.random.default_rng(seed)
    scale = (nx / 256.0) ** 3
    n_cic = int(round(1_000_000 * scale)) if n_cic is None else n_cic
    n_sn = int(round(100_000 * scale)) if n_sn is None else n_sn
    domain, lo, n = single_box(nx)
    state = gas_state(rng, nx ** 3, dtype).reshape(-1)
    cic = _one_box(uniform_positions(rng, n_cic, domain), cic_fields(rng, n_cic))
    sn = _one_box(uniform_positions(rng, n_sn, domain), sn_fields(n_sn, 4.0))
    return Workload(f"c2_{nx}cube_uniform_cic_sn", domain, lo, n, 4, 1.0, state, cic=cic, sn=sn)


def c3(seed: int = 3, nx: int = 256, n_cic: int | None = None, n_sink: int = 256,
       dtype=np.float32) -> Workload:
    """Plummer-clustered CIC (a = 8) plus sinks (r_K = 4, Gaussian width 2)."""
    rng = np.random.default_rng(seed)
    scale = (nx / 256.0) ** 3
    n_cic = int(round(1_000_000 * scale)) if n_cic is None else n_cic
    domain, lo, n = single_box(nx)
    state = gas_state(rng, nx ** 3, dtype).reshape(-1)
    centre = (nx / 2.0, nx / 2.0, nx / 2.0)
    cic = _one_box(plummer(rng, n_cic, 8.0, centre, domain), cic_fields(rng, n_cic))
    sk = _one_box(plummer(rng, n_sink, 8.0, centre, domain), {"a": np.full(n_sink, 0.25)})
    return Workload(f"c3_{nx}cube_plummer_sinks", domain, lo, n, 4, 1.0, state,
                    cic=cic, sinks=sk, r_k=4.0, r_gauss=2.0)


def bondi_fields(rng, count, log10_m=(-1.5, 1.5), sigma_v=0.3):
    """Sink masses log-uniform over ``log10_m`` and Gaussian velocities.
    With the gas of ``gas_state`` (c_s about 1) and G = 1 the Bondi-Hoyle
    radius G m / (v^2 + c^2) spans about 0.03 to 30 cells, so the three
    branches of the r_acc clamp all occur."""
    m = np.power(10.0, rng.uniform(log10_m[0], log10_m[1], count))
    v = sigma_v * rng.standard_normal((3, count))
    return {"a": np.zeros(count), "m": m, "vx": v[0], "vy": v[1], "vz": v[2]}


def c3bh(seed: int = 3, nx: int = 256, n_cic: int | None = None, n_sink: int = 256,
         dtype=np.float32) -> Workload:
    """c3 with Bondi-Hoyle sinks (G = 1, dt = 0.05, gamma = 5/3)."""
    w = c3(seed, nx, n_cic, n_sink, dtype)
    rng = np.random.default_rng(seed + 1000)
    pos = np.stack([w.sinks.fields[k] for k in ("x", "y", "z")], axis=1)
    sk = _one_box(pos, bondi_fields(rng, n_sink))
    return dataclasses.replace(w, name=f"c3bh_{nx}cube_plummer_bondi_sinks", sinks=sk,
                               sink_rate=1)


def c4(seed: int = 4, nx: int = 512, n_total: int | None = None,
       dtype=np.float32) -> Workload:
    """Half uniform, half in 32 Plummer clumps; CIC:SN = 10:1, SN r = 3, g = 4."""
    rng = np.random.default_rng(seed)
    scale = (nx / 512.0) ** 3
    n_total = int(round(4_000_000 * scale)) if n_total is None else n_total
    n_sn = int(round(n_total / 11))
    n_cic = n_total - n_sn
    domain, lo, n = single_box(nx)
    state = gas_state(rng, nx ** 3, dtype).reshape(-1)
    cic = _one_box(clumped_positions(rng, n_cic, domain), cic_fields(rng, n_cic))
    sn = _one_box(clumped_positions(rng, n_sn, domain), sn_fields(n_sn, 3.0))
    return Workload(f"c4_{nx}cube_mixed", domain, lo, n, 4, 1.0, state, cic=cic, sn=sn)


def c5(seed: int = 5, nb: int = 16, n_total: int | None = None, emin=8, emax=64,
       dtype=np.float32) -> Workload:
    """Batched AMR level: nb^3 boxes on a rectilinear grid with log-uniform
    edges in [emin, emax]; half uniform, half clumped particles, CIC:SN = 10:1,
    SN r = 2, g = 2."""
    rng = np.random.default_rng(seed)
    edges = []
    for _ax in range(3):
        e = np.rint(np.exp(rng.uniform(math.log(emin), math.log(emax), nb)))
        edges.append(np.clip(e, emin, emax).astype(np.int64))
    domain, lo, n, cuts = rectilinear(*edges)
    ncell = int(np.prod(np.asarray(domain, dtype=np.int64)))
    if n_total is None:
        n_total = int(round(8_000_000 * (nb / 16.0) ** 3))
    n_sn = int(round(n_total / 11))
    n_cic = n_total - n_sn
    assert int(np.prod(n.astype(np.int64), axis=1).sum()) == ncell
    state = pack_by_box(gas_state(rng, ncell, dtype), n)
    cic = _group_by_box(clumped_positions(rng, n_cic, domain), cic_fields(rng, n_cic),
                        cuts, (nb, nb, nb))
    sn = _group_by_box(clumped_positions(rng, n_sn, domain), sn_fields(n_sn, 2.0),
                       cuts, (nb, nb, nb))
    return Workload(f"c5_{nb}x{nb}x{nb}_boxes", domain, lo, n, 2, 1.0, state, cic=cic, sn=sn)


def multibox(edges_x, edges_y, edges_z, ghost, positions_cic=None, masses=None,
             positions_sn=None, sn_radius=1.0, seed=0, dtype=np.float64,
             positions_sink=None, sink_rate=0, r_k=None) -> Workload:
    """Hand-built rectilinear layout with given particle positions, for edge
    and corner tests (particles placed on box faces, edges and corners).
    Sinks (``positions_sink``) request a quarter of their kernel mass, or the
    Bondi-Hoyle rate with ``sink_rate`` 1; r_K defaults to the ghost width
    and the Gaussian width to r_K / 2."""
    rng = np.random.default_rng(seed)
    domain, lo, n, cuts = rectilinear(edges_x, edges_y, edges_z)
    nbx, nby, nbz = len(edges_x), len(edges_y), len(edges_z)
    ncell = int(np.prod(np.asarray(domain, dtype=np.int64)))
    state = pack_by_box(gas_state(rng, ncell, dtype), n)
    cic = sn = None
    if positions_cic is not None:
        pc = np.asarray(positions_cic, dtype=np.float64).reshape(-1, 3)
        m = np.asarray(masses if masses is not None else rng.uniform(0.1, 1.0, pc.shape[0]))
        cic = _group_by_box(pc, {"m": m}, cuts, (nbx, nby, nbz))
    if positions_sn is not None:
        ps = np.asarray(positions_sn, dtype=np.float64).reshape(-1, 3)
        sn = _group_by_box(ps, sn_fields(ps.shape[0], sn_radius), cuts, (nbx, nby, nbz))
    sk = None
    r_k = float(ghost) if r_k is None else float(r_k)
    if positions_sink is not None:
        pk = np.asarray(positions_sink, dtype=np.float64).reshape(-1, 3)
        fields = (bondi_fields(rng, pk.shape[0]) if sink_rate == 1
                  else {"a": np.full(pk.shape[0], 0.25)})
        sk = _group_by_box(pk, fields, cuts, (nbx, nby, nbz))
    return Workload("multibox", domain, lo, n, ghost, 1.0, state, cic=cic, sn=sn, sinks=sk,
                    r_k=r_k, r_gauss=r_k / 2.0, sink_rate=sink_rate)


def c5s(seed: int = 5, nb: int = 16, n_sink: int | None = None, bondi: bool = False,
        dtype=np.float32) -> Workload:
    """The batched AMR level of c5 with sinks drawn from the same clumps,
    grouped by box: r_K = g = 2, Gaussian width 1 (fraction a = 1/4), or the
    Bondi-Hoyle rate with r_acc clamped to [1/4, 1]."""
    w = c5(seed, nb, dtype=dtype)
    rng = np.random.default_rng(seed + 2000)
    n_sink = int(round(1024 * (nb / 16.0) ** 3)) if n_sink is None else n_sink
    cx, cy, cz = (np.concatenate([[0], np.cumsum(e)]) for e in _edges_of(w))
    pos = clumped_positions(rng, n_sink, w.domain)
    fields = bondi_fields(rng, n_sink) if bondi else {"a": np.full(n_sink, 0.25)}
    sk = _group_by_box(pos, fields, (cx, cy, cz), (nb, nb, nb))
    return dataclasses.replace(w, name=w.name + ("_bondi_sinks" if bondi else "_sinks"),
                               sinks=sk, r_k=2.0, r_gauss=1.0, sink_rate=1 if bondi else 0)


def _edges_of(w):
    """Per-axis box edges of a rectilinear layout (boxes in x-fastest order)."""
    lo = np.asarray(w.lo)
    n = np.asarray(w.n)
    out = []
    for a in range(3):
        firsts = np.unique(lo[:, a])
        out.append(np.array([n[np.flatnonzero(lo[:, a] == f)[0], a] for f in firsts]))
    return out


def snr_box(seed: int = 7, nx: int = 32, n_snr: int = 24, dtype=np.float64, sub: int = 4,
            r_k: float = 3.0, nb: int = 1) -> Workload:
    """Supernova remnants over gas whose mean density steps between three
    slabs along x (0.05, 1 and 30 code units, each with log-normal scatter of
    0.5 dex in e), so that the kernels fall in all three regimes (ejecta,
    Sedov-Taylor, momentum-conserving) and some straddle a density step;
    gas velocities N(0, 1), specific e_int = 1; remnant velocities N(0, 2).
    nb > 1: an nb^3 rectilinear tiling with uneven edges; g = 4."""
    rng = np.random.default_rng(seed)
    if nb == 1:
        domain, lo, n = single_box(nx)
        cuts, axes = None, None
    else:
        edges = [np.full(nb, nx // nb, dtype=np.int64) for _ in range(3)]
        for e in edges:
            e[0] += nx - e.sum() + 2
            e[-1] -= 2
        domain, lo, n, cuts = rectilinear(*edges)
        axes = (nb, nb, nb)
    ncell = int(np.prod(np.asarray(domain, dtype=np.int64)))
    X, _Y, _Z = domain
    ix = np.arange(ncell) % X
    level = np.where(ix < X // 3, 0.05, np.where(ix < 2 * X // 3, 1.0, 30.0))
    rho = (level * np.exp(0.5 * rng.standard_normal(ncell))).astype(dtype)
    v = rng.standard_normal((3, ncell))
    r64 = rho.astype(np.float64)
    p = (r64[None, :] * v).astype(dtype)
    p64 = p.astype(np.float64)
    E = (r64 + 0.5 * (p64 * p64).sum(axis=0) / r64).astype(dtype)
    fields = np.concatenate([rho[None], p, E[None]], axis=0)
    # the gas draw is in global x-fastest order; lay it out per box
    if nb == 1:
        state = fields.reshape(-1)
    else:
        gz, gy, gx = np.unravel_index(np.arange(ncell), (domain[2], domain[1], domain[0]))
        parts = []
        for b in range(lo.shape[0]):
            sel = ((gx >= lo[b, 0]) & (gx < lo[b, 0] + n[b, 0]) & (gy >= lo[b, 1]) &
                   (gy < lo[b, 1] + n[b, 1]) & (gz >= lo[b, 2]) & (gz < lo[b, 2] + n[b, 2]))
            parts.append(fields[:, np.flatnonzero(sel)].reshape(-1))
        state = np.concatenate(parts)
    pos = uniform_positions(rng, n_snr, domain)
    f = {"m": np.full(n_snr, SNR_M_EJ), "e": np.full(n_snr, SNR_E_SN)}
    vel = 2.0 * rng.standard_normal((3, n_snr))
    f.update({"vx": vel[0], "vy": vel[1], "vz": vel[2]})
    snr = _one_box(pos, f) if nb == 1 else _group_by_box(pos, f, cuts, axes)
    return Workload(f"snr_{nx}cube_{n_snr}_remnants" + ("" if nb == 1 else f"_{nb}boxes"),
                    domain, lo, n, 4, 1.0, state, snr=snr,
                    snr_params=SnrParams(r_k=r_k, sub=sub))


CONFIGS = {"c1": c1, "c2": c2, "c3": c3, "c4": c4, "c5": c5, "c3bh": c3bh, "c5s": c5s}
