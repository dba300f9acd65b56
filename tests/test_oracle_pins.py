"""Pins for the serial oracle: each check ties the oracle to something other
than itself (the paper's worked example, closed forms, lattice counts,
brute force over all cells and periodic images, invariants)."""
import dataclasses
import itertools
import math
import os

import numpy as np
import pytest

from paper_2509_18261_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")
Q = 2.0 ** 40


def golden(name):
    out = {}
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, v = line.split()
        out[k] = float(v)
    return out


def one_box(nx, ghost, state=None, cic=None, sn=None, sinks=None, ny=None, nz=None,
            limits=None, r_k=4.0, r_gauss=2.0, dx=1.0):
    domain, lo, n = W.single_box(nx, ny, nz)
    ncell = int(np.prod(domain))
    if state is None:
        state = W.uniform_state(ncell, np.float64).reshape(-1)

    def kind(pos, fields):
        if pos is None:
            return None
        pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
        return W._one_box(pos, fields)

    return W.Workload("t", domain, lo, n, ghost, dx, np.asarray(state, dtype=np.float64),
                      cic=kind(*cic) if cic else None, sn=kind(*sn) if sn else None,
                      sinks=kind(*sinks) if sinks else None, r_k=r_k, r_gauss=r_gauss,
                      limits=limits or W.Limits())


def owned(orc, w, buf, field):
    """Owned region of field `field` of a single-box buffer."""
    mesh = orc.Mesh.of(w)
    g = w.ghost
    B = mesh.box_buffer(buf, 0)[field]
    return B[g:B.shape[0] - g, g:B.shape[1] - g, g:B.shape[2] - g]


# ------------------------------------------------------------------ exp

def test_exp_against_libm(orc):
    xs = np.concatenate([np.linspace(-30, 30, 4001), -np.linspace(0, 4, 1001),
                         [0.0, -0.5, -1.0, -2.0, -4.0, 1e-300, -1e-300]])
    worst = 0
    for x in xs:
        a = orc.exp(float(x))
        b = math.exp(float(x))
        ulp = math.ulp(b)
        worst = max(worst, abs(a - b) / ulp)
    assert worst <= 2.0, worst
    assert orc.exp(0.0) == 1.0


# ------------------------------------------------------------------ CIC (P2)

@pytest.mark.parametrize("mode", ["f64", "fix64"])
def test_cic_cell_centre_and_corner(orc, mode):
    # particle at a cell centre: the whole mass in that cell
    w = one_box(8, 1, cic=([[3.5, 4.5, 5.5]], {"m": [0.7]}))
    buf, _, _ = orc.deposit(w, mode)
    o = owned(orc, w, buf, 0).astype(np.float64) * (1 / Q if mode == "fix64" else 1)
    assert np.count_nonzero(o) == 1
    assert o[5, 4, 3] == pytest.approx(0.7, abs=1e-12)
    # particle at a cell corner: 1/8 of the mass in each of 8 cells
    w = one_box(8, 1, cic=([[3.0, 4.0, 5.0]], {"m": [0.8]}))
    buf, _, _ = orc.deposit(w, mode)
    o = owned(orc, w, buf, 0).astype(np.float64) * (1 / Q if mode == "fix64" else 1)
    assert np.count_nonzero(o) == 8
    np.testing.assert_allclose(o[4:6, 3:5, 2:4], 0.1, atol=1e-12)


def test_cic_tensor_product(orc):
    # weights along x for x = 3.25: cells 2 and 3 with 0.25 and 0.75 (tent function)
    w = one_box(8, 1, cic=([[3.25, 4.5, 5.5]], {"m": [1.0]}))
    buf, _, _ = orc.deposit(w, "f64")
    o = owned(orc, w, buf, 0)
    assert o[5, 4, 2] == 0.25 and o[5, 4, 3] == 0.75
    assert np.count_nonzero(o) == 2


def _rint_half_even(fr):
    """Nearest integer to a Fraction, ties to even."""
    from fractions import Fraction
    f = math.floor(fr)
    d = fr - f
    if d > Fraction(1, 2) or (d == Fraction(1, 2) and f % 2 == 1):
        return f + 1
    return f


def test_fixed_point_remainder_goes_to_host_cell_at_a_tie(orc):
    """The fixed-point remainder rule, pinned to a cell: each contribution is
    rounded half-to-even on the 2^-40 grid and the particle's residue
    rint(m 2^40) - sum of the rounded contributions lands in its host cell
    floor(x).  x = 5 makes the two x weights tie at 1/2 (cells 4 and 5, host
    5, the upper of the tied cells, where a largest-weight rule with ties to
    the lowest index would pick 4); y = 4.75 gives weights 3/4 and 1/4 on
    cells 4 and 5 (host 4); z sits on a cell centre.  Expected values from exact
    rational arithmetic; the mass is chosen so that the residue is nonzero
    and every double product is exact."""
    from fractions import Fraction
    wx = {4: Fraction(1, 2), 5: Fraction(1, 2)}
    wy = {4: Fraction(3, 4), 5: Fraction(1, 4)}
    chosen = None
    for k in range(1, 64):
        m = 1.0 + k * 2.0 ** -43
        Fm = Fraction(m)
        q = {(i, j): _rint_half_even(Fm * wx[i] * wy[j] * 2 ** 40) for i in wx for j in wy}
        res = _rint_half_even(Fm * 2 ** 40) - sum(q.values())
        if res != 0:
            chosen = (m, q, res)
            break
    assert chosen is not None
    m, q, res = chosen
    w = one_box(10, 1, cic=([[5.0, 4.75, 6.5]], {"m": [m]}))
    buf, _, _ = orc.deposit(w, "fix64")
    o = owned(orc, w, buf, 0)
    assert np.count_nonzero(o) == 4
    for (i, j), v in q.items():
        expect = v + (res if (i, j) == (5, 4) else 0)
        assert int(o[6, j, i]) == expect, (i, j, int(o[6, j, i]), expect)
    assert int(o.sum()) == _rint_half_even(Fraction(m) * 2 ** 40)


# ------------------------------------------------------- SN lattice counts (P3)

def lattice_count(r2):
    """Integer points (a,b,c) with a^2+b^2+c^2 <= r2, by enumeration."""
    R = int(math.isqrt(r2)) + 1
    rng = range(-R, R + 1)
    return sum(1 for a, b, c in itertools.product(rng, rng, rng) if a * a + b * b + c * c <= r2)


@pytest.mark.parametrize("r,expected", [(2, 33), (3, 123), (4, 257)])
def test_sn_centred_lattice_count(orc, r, expected):
    assert lattice_count(r * r) == expected
    w = one_box(16, r, sn=([[8.5, 8.5, 8.5]], W.sn_fields(1, float(r), m=1.0, e=2.0)))
    buf, _, _ = orc.deposit(w, "f64")
    o = owned(orc, w, buf, 0)
    e = owned(orc, w, buf, 4)
    assert np.count_nonzero(o) == expected
    np.testing.assert_allclose(o[o != 0], 1.0 / expected, rtol=1e-15)
    np.testing.assert_allclose(e[e != 0], 2.0 / expected, rtol=1e-15)
    for f in (1, 2, 3):
        assert not owned(orc, w, buf, f).any()


# ---------------------------------------------------- brute force (P6, P2, P3)

def brute_force(w):
    """All-cells, all-periodic-images deposit straight onto the owned cells:
    CIC as the tent function prod(max(0, 1 - |x - c|)), SN as equal shares
    over every unwrapped cell index whose centre lies within r."""
    nx, ny, nz = w.domain
    out = np.zeros((5, nz, ny, nx))
    S = 2
    shifts = range(-S, S + 1)
    ci = np.arange(nx) + 0.5
    cj = np.arange(ny) + 0.5
    ck = np.arange(nz) + 0.5
    V = w.dx ** 3
    if w.cic is not None:
        f = w.cic.fields
        for p in range(w.cic.n):
            x, y, z, m = f["x"][p], f["y"][p], f["z"][p], f["m"][p]
            for sx, sy, sz in itertools.product(shifts, shifts, shifts):
                wx = np.maximum(0.0, 1.0 - np.abs(x - (ci + sx * nx)))
                wy = np.maximum(0.0, 1.0 - np.abs(y - (cj + sy * ny)))
                wz = np.maximum(0.0, 1.0 - np.abs(z - (ck + sz * nz)))
                out[0] += m / V * wz[:, None, None] * wy[None, :, None] * wx[None, None, :]
    if w.sn is not None:
        f = w.sn.fields
        I, J, K = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
        for p in range(w.sn.n):
            x, y, z, m, e, r = (f[k][p] for k in ("x", "y", "z", "m", "e", "r"))
            hits = np.zeros((nz, ny, nx))
            for sx, sy, sz in itertools.product(shifts, shifts, shifts):
                dxv = ((I + sx * nx).astype(np.float64) + 0.5) - x
                dyv = ((J + sy * ny).astype(np.float64) + 0.5) - y
                dzv = ((K + sz * nz).astype(np.float64) + 0.5) - z
                d2 = (dxv * dxv + dyv * dyv) + dzv * dzv
                hits += (d2 <= r * r).transpose(2, 1, 0)
            N = hits.sum()
            out[0] += hits * m / (N * V)
            out[4] += hits * e / (N * V)
    return out


def gather_owned(orc, w, buf, nfield=5):
    """Owned cells of every box, painted into a domain array [F][nz][ny][nx]."""
    mesh = orc.Mesh.of(w)
    nx, ny, nz = w.domain
    out = np.zeros((nfield, nz, ny, nx))
    g = w.ghost
    for b in range(w.nbox):
        B = mesh.box_buffer(buf, b).astype(np.float64)
        (lx, ly, lz), (bx, by, bz) = w.lo[b], w.n[b]
        out[:, lz:lz + bz, ly:ly + by, lx:lx + bx] = B[:nfield, g:g + bz, g:g + by, g:g + bx]
    return out


def small_workloads():
    rng = np.random.default_rng(11)
    # single box, reach equal to the ghost width, particles everywhere
    w1 = W.Workload("a", *W.single_box(7, 6, 9), 2, 1.0,
                    W.uniform_state(7 * 6 * 9, np.float64).reshape(-1),
                    cic=W._one_box(W.uniform_positions(rng, 40, (7, 6, 9)), W.cic_fields(rng, 40)),
                    sn=W._one_box(W.uniform_positions(rng, 6, (7, 6, 9)), W.sn_fields(6, 2.0, e=3.0)))
    # 2x2x2 boxes of unequal size; particles on faces, edges and corners of boxes
    edges = ([5, 7], [6, 4], [4, 6])
    pos_c = [[5.0, 6.0, 4.0], [0.0, 0.0, 0.0], [4.99, 5.99, 3.99], [11.5, 9.5, 9.5],
             [5.0, 2.5, 7.2], [0.25, 9.75, 4.0], [6.0, 6.0, 6.0]]
    pos_s = [[5.0, 6.0, 4.0], [0.1, 9.9, 9.9], [11.9, 0.2, 5.0], [3.3, 3.3, 3.3]]
    w2 = W.multibox(*edges, ghost=2, positions_cic=pos_c, positions_sn=pos_s, sn_radius=1.5,
                    seed=3)
    # box smaller than twice the ghost width (several images of one cell)
    w3 = W.Workload("c", *W.single_box(3, 4, 3), 2, 1.0,
                    W.uniform_state(36, np.float64).reshape(-1),
                    cic=W._one_box(W.uniform_positions(rng, 9, (3, 4, 3)), W.cic_fields(rng, 9)),
                    sn=W._one_box(W.uniform_positions(rng, 3, (3, 4, 3)), W.sn_fields(3, 1.7)))
    return [w1, w2, w3]


@pytest.mark.parametrize("idx", [0, 1, 2])
def test_deposit_fold_equals_brute_force(orc, idx):
    w = small_workloads()[idx]
    ref = brute_force(w)
    buf, _, _ = orc.deposit(w, "f64")
    orc.fold(w, "f64", buf)
    got = gather_owned(orc, w, buf)
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-14)
    # fixed point: within half a quantum per contribution of the same answer
    bq, _, _ = orc.deposit(w, "fix64")
    orc.fold(w, "fix64", bq)
    gq = gather_owned(orc, w, bq) / Q
    np.testing.assert_allclose(gq, ref, rtol=0, atol=1e-9)


# ------------------------------------------------------- conservation (P4, P5)

def test_fixed_point_conservation_exact(orc):
    for w in small_workloads() + [W.c2(nx=32), W.c4(nx=32)]:
        bq, _, _ = orc.deposit(w, "fix64")
        mesh = orc.Mesh.of(w)
        tot = [int(sum(int(mesh.box_buffer(bq, b)[f].sum(dtype=np.int64)) for b in range(w.nbox)))
               for f in range(5)]
        V = w.dx ** 3
        m_parts = 0
        e_parts = 0
        if w.cic is not None:
            m_parts += int(np.rint(w.cic.fields["m"] / V * Q).astype(np.int64).sum())
        if w.sn is not None:
            m_parts += int(np.rint(w.sn.fields["m"] / V * Q).astype(np.int64).sum())
            e_parts += int(np.rint(w.sn.fields["e"] / V * Q).astype(np.int64).sum())
        assert tot[0] == m_parts
        assert tot[4] == e_parts
        assert tot[1] == tot[2] == tot[3] == 0
        # the fold moves, never creates: owned total after = everything before
        orc.fold(w, "fix64", bq)
        g = w.ghost
        after = 0
        for b in range(w.nbox):
            B = mesh.box_buffer(bq, b)[0]
            after += int(B[g:B.shape[0] - g, g:B.shape[1] - g, g:B.shape[2] - g].sum(dtype=np.int64))
        assert after == m_parts


def test_f64_conservation(orc):
    w = W.c2(nx=32)
    buf, _, _ = orc.deposit(w, "f64")
    total = math.fsum(w.cic.fields["m"]) + math.fsum(w.sn.fields["m"])
    assert math.fsum(orc.Mesh.of(w).box_buffer(buf, 0)[0].ravel()) == pytest.approx(total, rel=1e-14)


# ------------------------------------------------------------ determinism (P7)

def test_fixed_point_permutation_invariant(orc):
    w = W.c4(nx=32)
    bq, _, _ = orc.deposit(w, "fix64")
    rng = np.random.default_rng(5)
    perm_c = rng.permutation(w.cic.n)
    perm_s = rng.permutation(w.sn.n)
    cic = W.Particles({k: v[perm_c] for k, v in w.cic.fields.items()}, w.cic.box_off)
    sn = W.Particles({k: v[perm_s] for k, v in w.sn.fields.items()}, w.sn.box_off)
    import dataclasses
    w2 = dataclasses.replace(w, cic=cic, sn=sn)
    b2, _, _ = orc.deposit(w2, "fix64")
    assert np.array_equal(bq, b2)


# ------------------------------------ reproducibility mode (App. A.1, error bound)

def _bits(a):
    return np.ascontiguousarray(a, dtype=np.float64).view(np.uint64)


def test_truncation_closed_forms(orc):
    """One contribution: err = eps |v| exactly, so nb = M and 52 - M mantissa
    bits stay; two same-sign contributions: err / |v| lies strictly between
    eps and 2 eps, so nb = M + 1; zero, and err = 0, pass unchanged."""
    eps = 2.0 ** -52
    for v in (1.2345678901234567, -3.75e-7, 6.02e23):
        for M in (0, 10, 28, 40):
            got = orc.truncate_err(v, eps * abs(v), M)
            want = (_bits([v]) & ~np.uint64((1 << M) - 1)).view(np.float64)[0]
            assert got == want, (v, M)
    a, b = 0.7, 0.3001
    s = a + b
    err = eps * abs(a) + eps * abs(s)
    got = orc.truncate_err(s, err, 28)
    assert got == (_bits([s]) & ~np.uint64((1 << 29) - 1)).view(np.float64)[0]
    assert orc.truncate_err(0.0, 1e-30, 28) == 0.0
    assert orc.truncate_err(5.0, 0.0, 28) == 5.0
    # nb never exceeds the 52 mantissa bits: a huge bound leaves the leading power of two
    assert orc.truncate_err(1.9999, 1.0, 28) == 1.0


def test_f64r_is_f64_with_low_bits_cleared(orc):
    """The reproducibility mode sums in the order of the plain FP64 mode, so
    every buffer element equals the FP64 one with low mantissa bits cleared,
    at least M of them wherever anything was deposited (a single-contribution
    cell exactly M)."""
    M = 28
    w = W.c2(nx=32)
    b64, _, _ = orc.deposit(w, "f64")
    br, _, _ = orc.deposit(w, "f64r")
    x, y = _bits(b64), _bits(br)
    nz = b64 != 0.0
    assert np.array_equal(br[~nz], b64[~nz])
    cleared = x[nz] ^ y[nz]
    assert np.all((y[nz] & ~x[nz]) == 0)  # only bits of x cleared, none set
    # the cleared bits are low bits: x with its low k bits cleared equals y for
    # the k of its highest cleared bit
    hi = np.where(cleared == 0, 0, np.floor(np.log2(np.maximum(cleared, 1).astype(np.float64))) + 1)
    assert np.all(hi <= 52)
    keep = x[nz] & ~((np.uint64(1) << hi.astype(np.uint64)) - np.uint64(1))
    assert np.array_equal(keep, y[nz])
    # an isolated CIC particle at a cell centre: one contribution, exactly M bits cleared
    w1 = one_box(8, 1, cic=([[4.5, 4.5, 4.5]], {"m": [0.8123456789]}))
    b1, _, _ = orc.deposit(w1, "f64")
    r1, _, _ = orc.deposit(w1, "f64r")
    i = int(np.flatnonzero(b1)[0])
    assert np.count_nonzero(b1) == 1
    assert _bits([r1[i]])[0] == _bits([b1[i]])[0] & ~np.uint64((1 << M) - 1)


def test_f64r_mostly_permutation_invariant(orc):
    """The property App. A.1 claims: re-ordering the contributions moves the
    truncated sums only where a sum lies within its error of a truncation
    boundary, or where the bound itself crosses a power of two (cells with
    three or more contributions); most cells keep their bits, and every cell
    stays within one truncation interval."""
    w = W.c2(nx=32)
    br, _, _ = orc.deposit(w, "f64r")
    rng = np.random.default_rng(7)
    perm_c = rng.permutation(w.cic.n)
    perm_s = rng.permutation(w.sn.n)
    cic = W.Particles({k: v[perm_c] for k, v in w.cic.fields.items()}, w.cic.box_off)
    sn = W.Particles({k: v[perm_s] for k, v in w.sn.fields.items()}, w.sn.box_off)
    import dataclasses
    b2, _, _ = orc.deposit(dataclasses.replace(w, cic=cic, sn=sn), "f64r")
    nz = (br != 0.0) | (b2 != 0.0)
    same = np.mean(br[nz] == b2[nz])
    assert same > 0.9, same
    rel = np.abs(br[nz] - b2[nz]) / np.maximum(np.abs(br[nz]), np.abs(b2[nz]))
    assert rel.max() <= 2.0 ** -(52 - 28 - 8), rel.max()


# ------------------------------------------------------------ limiter (P1, P8, P11)

def test_fig1_worked_example(orc):
    """Fig. 1: two sinks share one cell of density 1; cap 1/4, rho_Tr = 0.2."""
    G = golden("fig1_worked_example.txt")
    lim = W.Limits(rho_floor=1e-10, rho_tr=G["rho_tr"], cap=G["cap"])
    # limiter level: the summed request of the figure, K = 2 * 0.5
    w = one_box(1, 0, state=W.uniform_state(1, np.float64, rho=G["rho0"]).reshape(-1),
                limits=lim)
    w.sinks = W.Particles({}, np.array([0, 1]))  # six buffer fields
    buf = np.zeros(6)
    buf[5] = G["drho_per_sink"] * G["nsink"]
    assert buf[5] == G["drho_sum"]
    st, eta, cnt = orc.apply(w, "f64", buf, want_eta=True)
    assert eta[0] * buf[5] == pytest.approx(G["drho_limited"], abs=1e-15)
    assert st[0] == pytest.approx(G["rho_final"], abs=1e-15)
    assert cnt["bind"] == 1
    # full step: two sinks in a one-cell periodic domain, each asking for half
    # the kernel mass
    sinks = ([[0.5, 0.5, 0.5], [0.5, 0.5, 0.5]], {"a": [G["drho_per_sink"]] * 2})
    state = W.uniform_state(1, np.float64, rho=G["rho0"]).reshape(-1)
    w = one_box(1, 1, state=state, sinks=sinks, limits=lim, r_k=0.5, r_gauss=0.5)
    for mode in ("f64", "fix64"):
        out = orc.step(w, mode, want_eta=True)
        scale = 1 / Q if mode == "fix64" else 1.0
        K = float(owned(orc, w, out["buf_fold"], 5)[0, 0, 0]) * scale
        assert K == pytest.approx(G["drho_sum_with_truelove"], abs=1e-12)
        assert out["eta"][0] * K == pytest.approx(G["drho_limited"], abs=1e-12)
        assert out["state"][0] == pytest.approx(G["rho_final"], abs=1e-12)
        dm = out["sink_d"][0]
        np.testing.assert_allclose(dm, G["sink_gain"], atol=1e-12)
        # mass is conserved between gas and sinks (eq. "conservation")
        assert out["state"][0] + dm.sum() == pytest.approx(G["rho0"], abs=1e-12)
    # with the Truelove term off, the cap alone binds: the cell keeps 3/4
    w.limits.rho_tr = math.inf
    out = orc.step(w, "f64", want_eta=True)
    assert out["state"][0] == pytest.approx(0.75, abs=1e-15)
    np.testing.assert_allclose(out["sink_d"][0], 0.125, atol=1e-15)


def lambda_cell(orc, mode):
    w = one_box(1, 0)
    w.limits.eint_mode = mode
    buf = np.zeros(5)
    buf[1] = 3.0  # d_px
    buf[4] = 1.0  # d_E
    st, _, cnt = orc.apply(w, "f64", buf)
    return st, cnt


def test_lambda_hand_computed(orc):
    G = golden("lambda_cell.txt")
    st, cnt = lambda_cell(orc, 0)
    assert st[1] / 3.0 == pytest.approx(G["mode0_lambda"], rel=1e-15)
    assert st[4] == 2.0 and st[0] == 1.0 and cnt["lam"] == 1
    # internal energy lands exactly on the floor
    assert st[4] - st[1] ** 2 / (2 * st[0]) == pytest.approx(0.0, abs=1e-15)
    st, _ = lambda_cell(orc, 1)
    assert st[1] / 3.0 == pytest.approx(G["mode1_lambda"], rel=1e-15)
    assert st[4] - st[1] ** 2 / (2 * st[0]) == pytest.approx(1.0, rel=1e-14)


def test_limiter_invariants(orc):
    rng = np.random.default_rng(7)
    n = 4000
    w = one_box(n, 0, ny=1, nz=1)
    rho = np.exp(rng.standard_normal(n))
    v = rng.standard_normal((3, n))
    p = rho * v
    eint = rng.uniform(0.0, 2.0, n) * rho
    E = eint + 0.5 * (p * p).sum(0) / rho
    state = np.concatenate([rho, p[0], p[1], p[2], E])
    w = W.Workload("l", *W.single_box(n, 1, 1), 0, 1.0, state, limits=W.Limits())
    # 6-field buffer: random sources, removal in a third of the cells
    w.sinks = W.Particles({}, np.array([0, 1]))  # marks F = 6
    buf = np.zeros(6 * n)
    buf[0:n] = rng.uniform(0, 1, n) * (rng.random(n) < 0.5)
    buf[n:4 * n] = rng.standard_normal(3 * n) * 3.0 * (rng.random(3 * n) < 0.5)
    buf[4 * n:5 * n] = rng.uniform(0, 1, n) * (rng.random(n) < 0.5)
    sink_only = rng.random(n) < 0.3
    buf[5 * n:] = rng.uniform(0, 2, n) * rho * (rng.random(n) < 0.6)
    for f in range(5):
        buf[f * n:(f + 1) * n][sink_only] = 0.0
    for mode in (0, 1):
        w.limits.eint_mode = mode
        st, eta, cnt = orc.apply(w, "f64", buf, want_eta=True)
        r1, p1, E1 = st[:n], st[n:4 * n].reshape(3, n), st[4 * n:]
        K = buf[5 * n:]
        assert np.all((eta >= 0) & (eta <= 1))
        on = K > 0
        assert np.all(r1[on] >= np.maximum(1e-10, 0.75 * rho[on]) * (1 - 1e-15))
        # the fraction removed never exceeds the cap (rho_Tr disabled)
        Kl = eta * K
        assert np.all(Kl <= 0.25 * rho * (1 + 1e-15))
        # internal energy floor
        f = 1 - Kl / rho
        rr = f * rho + buf[:n]
        emin = np.zeros(n) if mode == 0 else rr * (E - 0.5 * (p * p).sum(0) / rho) / rho
        e1 = E1 - 0.5 * (p1 * p1).sum(0) / r1
        assert np.all(e1 >= emin - 1e-12 * np.abs(E1))
        # lambda in [0, 1]: p' = f p + lambda dp
        dp = buf[n:4 * n].reshape(3, n)
        nz = np.abs(dp) > 0
        lam = (p1 - f * p)[nz] / dp[nz]
        assert np.all((lam >= -1e-12) & (lam <= 1 + 1e-12))
        # sink-only cells keep velocity and specific energy
        so = sink_only & on
        np.testing.assert_allclose(E1[so] / r1[so], E[so] / rho[so], rtol=5e-16)
        np.testing.assert_allclose((p1 / r1)[:, so], (p / rho)[:, so], rtol=5e-16)
        if mode == 0:
            # e_int >= 0 can always be met by lambda = 0 (sources add mass and
            # energy, removal scales the cell); mode 1 can be infeasible when
            # mass arrives without energy, and then E is raised to the floor
            assert cnt["fall"] == 0


# ------------------------------------------------------------- sinks (P9, P12)

def test_sink_closed_form(orc):
    """Uniform gas rho = 1, one sink at a cell centre, r_K = 4, Gaussian width
    2, request 1/4 of the kernel mass."""
    pts = [(a, b, c) for a, b, c in itertools.product(range(-4, 5), repeat=3)
           if a * a + b * b + c * c <= 16]
    assert len(pts) == 257
    d2 = np.array([a * a + b * b + c * c for a, b, c in pts], dtype=np.float64)
    wts = np.exp(-d2 / 4.0)
    Wsum = math.fsum(wts)
    k = 0.25 * 257 * wts / Wsum
    bind = k > 0.25
    assert bind.sum() == lattice_count(7) == 81
    w = one_box(16, 4, sinks=([[8.5, 8.5, 8.5]], {"a": [0.25]}))
    for mode in ("f64", "fix64"):
        out = orc.step(w, mode, want_eta=True)
        assert out["sink_w"][0] == pytest.approx(Wsum, rel=1e-12)
        assert out["sink_mreq"][0] == pytest.approx(64.25, rel=1e-12)
        assert out["counters"]["bind"] == 81 and out["counters"]["touched"] == 257
        dm = out["sink_d"][0][0]
        # the kernel sum W is accumulated on the 2^-40 grid: |dW| <= 257 * 2^-41
        assert dm == pytest.approx(math.fsum(np.minimum(k, 0.25)), rel=1e-11)
        # P9: what the sink gains is what the gas loses
        rho1 = out["state"][: 16 ** 3]
        assert dm == pytest.approx(math.fsum(1.0 - rho1), rel=1e-12)


def test_sink_update_conservation_clustered(orc):
    w = W.c3(nx=32, n_cic=0, n_sink=40)
    w = W.Workload(w.name, w.domain, w.lo, w.n, w.ghost, w.dx, w.state, sinks=w.sinks)
    for mode in ("f64", "fix64"):
        out = orc.step(w, mode, want_eta=True)
        dm = out["sink_d"][0]
        rho0 = w.state[: 32 ** 3].astype(np.float64)
        lost = math.fsum(rho0 - out["state"][: 32 ** 3])
        assert math.fsum(dm) == pytest.approx(lost, rel=1e-10)
        assert out["counters"]["bind"] > 0
        # momentum: the sinks gain what the gas loses
        for ax in range(3):
            p0 = w.state[(1 + ax) * 32 ** 3:(2 + ax) * 32 ** 3].astype(np.float64)
            p1 = out["state"][(1 + ax) * 32 ** 3:(2 + ax) * 32 ** 3]
            assert math.fsum(out["sink_d"][1 + ax]) == pytest.approx(math.fsum(p0 - p1), rel=1e-9, abs=1e-9)


# ------------------------------------------------- Bondi-Hoyle sinks (S4, S5)

LAMBDA_ISO = math.exp(1.5) / 4.0


def kernel_offsets(x, r_k):
    """Integer cells whose centres lie within r_k of x (brute force)."""
    c = [range(int(math.floor(p - r_k)) - 1, int(math.ceil(p + r_k)) + 2) for p in x]
    return [(i, j, k) for i in c[0] for j in c[1] for k in c[2]
            if (i + 0.5 - x[0]) ** 2 + (j + 0.5 - x[1]) ** 2 + (k + 0.5 - x[2]) ** 2 <= r_k * r_k]


def bondi_box(nx, state, pos, m, v, G=1.0, dt=0.05, gamma=5.0 / 3.0, r_k=4.0, ghost=4,
              dx=1.0, limits=None):
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    v = np.asarray(v, dtype=np.float64).reshape(-1, 3)
    fields = {"a": np.zeros(len(pos)), "m": np.asarray(m, dtype=np.float64),
              "vx": v[:, 0], "vy": v[:, 1], "vz": v[:, 2]}
    w = one_box(nx, ghost, state=state, sinks=(pos, fields), r_k=r_k, dx=dx, limits=limits)
    return dataclasses.replace(w, sink_rate=1, grav_G=G, dt=dt, gamma=gamma)


def moving_gas(nx, rho, u, e_sp):
    """Uniform gas of density rho, velocity u and specific internal energy e_sp."""
    n = nx ** 3
    s = np.zeros((5, n))
    s[0] = rho
    for ax in range(3):
        s[1 + ax] = rho * u[ax]
    s[4] = rho * e_sp + 0.5 * rho * float(np.dot(u, u))
    return s.reshape(-1)


def test_bhl_lambda_is_the_isothermal_value():
    # Sec. 3.1.1 quotes lambda = e^(3/2) / 4 ~ 1.120 for isothermal gas
    lam = W.Workload("t", (1, 1, 1), None, None, 1, 1.0, None).bhl_lambda
    assert lam == LAMBDA_ISO
    assert abs(lam - 1.120) < 5e-4
    assert lam * lam * 16.0 == pytest.approx(math.exp(3.0), rel=1e-15)


@pytest.mark.parametrize("mode", ["f64", "fix64"])
def test_bondi_limit_gas_at_rest(orc, mode):
    """Sink at rest in uniform gas at rest: v_inf = 0, c_inf = c_s, rho_inf =
    rho, so eq. "mdot" is the Bondi rate 4 pi lambda G^2 m^2 rho / c^3."""
    gamma, e_sp, rho, G, dt = 5.0 / 3.0, 1.5, 2.0, 0.7, 0.05
    c2 = gamma * (gamma - 1.0) * e_sp
    c = math.sqrt(c2)
    rbh = 1.5                                  # cells, inside [1/4, r_K/2]
    m = rbh * c2 / G
    x = (8.5, 8.5, 8.5)
    w = bondi_box(16, moving_gas(16, rho, (0, 0, 0), e_sp), [x], [m], [(0, 0, 0)], G=G, dt=dt)
    out = orc.step(w, mode)
    bondi = 4.0 * math.pi * LAMBDA_ISO * G * G * m * m * rho / c ** 3 * dt
    assert out["sink_mreq"][0] == pytest.approx(bondi, rel=1e-11)
    assert out["sink_racc"][0] == pytest.approx(rbh, rel=1e-13)
    offs = kernel_offsets(x, 4.0)
    assert len(offs) == 257
    wts = [math.exp(-((i + 0.5 - x[0]) ** 2 + (j + 0.5 - x[1]) ** 2 + (k + 0.5 - x[2]) ** 2)
                    / rbh ** 2) for i, j, k in offs]
    assert out["sink_w"][0] == pytest.approx(math.fsum(wts), rel=1e-11)
    # what the buffer receives sums to the request; a cell next to the host
    # holds its Gaussian share (no Truelove term; in fixed point the host
    # cell also takes the rounding remainder of the request)
    K = owned(orc, w, out["buf_deposit"], 5)
    K = K * Q ** -1 if mode == "fix64" else K
    assert math.fsum(K.ravel()) == pytest.approx(bondi, rel=1e-11)
    share = bondi * math.exp(-1.0 / rbh ** 2) / math.fsum(wts)
    assert K[9, 8, 8] == pytest.approx(share, rel=1e-11)


@pytest.mark.parametrize("mode", ["f64", "fix64"])
def test_bondi_moving_gas_first_form_and_clamp(orc, mode):
    """Moving gas, moving sinks: eq. "mdot" in its first form
    4 pi rho G^2 m^2 [(lambda^2 c^2 + v^2) / (c^2 + v^2)^4]^(1/2), and r_acc
    on all three branches of its clamp (dx = 0.5, so cells and lengths differ)."""
    gamma, e_sp, rho, G, dt, dx = 1.4, 0.9, 0.8, 2.0, 0.01, 0.5
    u = np.array([0.8, -0.3, 0.5])
    vs = np.array([0.1, 0.2, -0.1])
    c2 = gamma * (gamma - 1.0) * e_sp
    v2 = float(np.dot(u - vs, u - vs))
    V = dx ** 3
    pos = [(8.5, 8.5, 8.5), (24.5, 8.5, 8.5), (8.5, 24.5, 8.5)]
    rbh_len = np.array([0.05, 0.7, 3.0])          # lengths: 0.1, 1.4, 6 cells
    m = rbh_len * (c2 + v2) / G
    w = bondi_box(32, moving_gas(32, rho, u, e_sp), pos, m, [vs] * 3, G=G, dt=dt, gamma=gamma,
                  dx=dx)
    out = orc.step(w, mode)
    first = [4.0 * math.pi * rho * G * G * mm * mm *
             math.sqrt((LAMBDA_ISO ** 2 * c2 + v2) / (c2 + v2) ** 4) * dt for mm in m]
    # the kernel sums sit on the 2^-40 grid: terms of about 0.1 carry a
    # relative rounding of up to 5e-12 each, and the rate goes as 1/(c^2+v^2)^2
    np.testing.assert_allclose(out["sink_mreq"], first, rtol=1e-10)
    np.testing.assert_allclose(out["sink_racc"], [0.25, 1.4, 2.0], rtol=1e-10)
    # the gas loses what the sinks gain, in mass and momentum
    n = 32 ** 3
    lost = rho * n - math.fsum(out["state"][:n])
    assert math.fsum(out["sink_d"][0]) == pytest.approx(lost * V, rel=1e-10)
    # the two lighter sinks get their whole request; the heaviest one's
    # central cells hit the removal limiter (a quarter of the cell's mass)
    x = pos[2]
    d2 = [(i + 0.5 - x[0]) ** 2 + (j + 0.5 - x[1]) ** 2 + (k + 0.5 - x[2]) ** 2
          for i, j, k in kernel_offsets(x, 4.0)]
    wts = [math.exp(-d / 4.0) for d in d2]
    got2 = math.fsum(min(first[2] * wk / (math.fsum(wts) * V), 0.25 * rho) * V for wk in wts)
    assert got2 < first[2]
    gain = np.array([first[0], first[1], got2])
    # fixed point sums 257 terms on the 2^-40 grid: at most 257 * 2^-41 apart
    tol = dict(rtol=1e-10, atol=257 * 2.0 ** -41)
    np.testing.assert_allclose(out["sink_d"][0], gain, **tol)
    for ax in range(3):
        np.testing.assert_allclose(out["sink_d"][1 + ax], gain * u[ax], **tol)


def test_bondi_hoyle_lyttleton_limit_cold_gas(orc):
    """Cold gas (c_s = 0) streaming past the sink: the Hoyle-Lyttleton rate
    4 pi G^2 m^2 rho / v^3."""
    rho, G, dt = 3.0, 1.0, 0.02
    u = np.array([0.0, 0.6, 0.0])
    m = 0.5 * 0.36                                   # r_BH = 0.5 cells
    w = bondi_box(16, moving_gas(16, rho, u, 0.0), [(8.2, 7.9, 8.6)], [m], [(0, 0, 0)], G=G,
                  dt=dt)
    out = orc.step(w, "f64")
    assert out["sink_mreq"][0] == pytest.approx(4 * math.pi * G * G * m * m * rho / 0.6 ** 3 * dt,
                                               rel=1e-12)
    assert out["sink_racc"][0] == pytest.approx(0.5, rel=1e-13)


def test_bondi_mass_weighted_means_brute_force(orc):
    """Log-normal gas: v_inf, c_inf mass-weighted over the kernel, rho_inf
    the kernel's mean density, all by brute force over the kernel cells
    (periodic images included: the sink sits next to the domain corner)."""
    nx, gamma, G, dt = 16, 5.0 / 3.0, 1.0, 0.05
    rng = np.random.default_rng(11)
    st = W.gas_state(rng, nx ** 3, np.float64)
    # a spread of temperatures, so that the mass-weighted mean sound speed
    # differs from the root-mean-square and from the volume mean
    e_sp = np.exp(0.7 * rng.standard_normal(nx ** 3))
    st[4] = st[0] * e_sp + 0.5 * (st[1] ** 2 + st[2] ** 2 + st[3] ** 2) / st[0]
    pos = [(1.3, 14.8, 0.6), (8.1, 8.9, 7.7)]
    vs = [(0.2, -0.1, 0.05), (-0.3, 0.0, 0.1)]
    m = [0.4, 1.7]
    w = bondi_box(nx, st.reshape(-1), pos, m, vs, G=G, dt=dt, gamma=gamma)
    out = orc.step(w, "f64")
    F = st.reshape(5, nx, nx, nx)                       # [f][z][y][x]
    for s in range(2):
        cells = kernel_offsets(pos[s], 4.0)
        Ms = Px = Py = Pz = Cs = 0.0
        for i, j, k in cells:
            r, px, py, pz, E = (F[f, k % nx, j % nx, i % nx] for f in range(5))
            eint = max(E - (px * px + py * py + pz * pz) / (2 * r), 0.0)
            cs = math.sqrt(gamma * (gamma - 1) * eint / r)
            Ms += r
            Px += px
            Py += py
            Pz += pz
            Cs += r * cs
        uinf = np.array([Px, Py, Pz]) / Ms - np.asarray(vs[s])
        v2 = float(np.dot(uinf, uinf))
        cinf = Cs / Ms
        rho_inf = Ms / len(cells)
        rbh = G * m[s] / (v2 + cinf ** 2)
        mdot = 4 * math.pi * rho_inf * rbh ** 2 * math.sqrt(LAMBDA_ISO ** 2 * cinf ** 2 + v2)
        assert out["sink_mreq"][s] == pytest.approx(min(mdot * dt, Ms), rel=1e-10)
        assert out["sink_racc"][s] == pytest.approx(min(max(rbh, 0.25), 2.0), rel=1e-12)
        racc = out["sink_racc"][s]
        Wb = math.fsum(math.exp(-((i + 0.5 - pos[s][0]) ** 2 + (j + 0.5 - pos[s][1]) ** 2 +
                                  (k + 0.5 - pos[s][2]) ** 2) / racc ** 2) for i, j, k in cells)
        assert out["sink_w"][s] == pytest.approx(Wb, rel=1e-11)


def test_bondi_request_capped_at_kernel_mass(orc):
    rho, e_sp = 1.25, 1.0
    x = (8.5, 8.5, 8.5)
    # a heavy sink asks for more than its kernel holds
    w = bondi_box(16, moving_gas(16, rho, (0, 0, 0), e_sp), [x], [1e4], [(0, 0, 0)])
    out = orc.step(w, "f64", want_eta=True)
    assert out["sink_mreq"][0] == pytest.approx(257 * rho, rel=1e-14)
    assert out["sink_racc"][0] == 2.0
    # the removal limiter (a quarter of a cell's mass) binds wherever the
    # Gaussian share of 257 rho exceeds rho / 4
    wts = np.array([math.exp(-((i + 0.5 - x[0]) ** 2 + (j + 0.5 - x[1]) ** 2 +
                               (k + 0.5 - x[2]) ** 2) / 4.0) for i, j, k in kernel_offsets(x, 4.0)])
    assert out["counters"]["bind"] == int((257 * wts / wts.sum() > 0.25).sum()) == 179
    # cold gas at rest with the sink: v_inf = c_inf = 0 requests the kernel mass
    w = bondi_box(16, moving_gas(16, rho, (0, 0, 0), 0.0), [x], [0.1], [(0, 0, 0)])
    out = orc.step(w, "fix64")
    assert out["sink_mreq"][0] == pytest.approx(257 * rho, rel=1e-14)
    assert out["sink_racc"][0] == 2.0
    # a massless sink asks for nothing
    w = bondi_box(16, moving_gas(16, rho, (0, 0, 0), e_sp), [x], [0.0], [(0, 0, 0)])
    out = orc.step(w, "f64")
    assert out["sink_mreq"][0] == 0.0 and out["sink_racc"][0] == 0.25
    assert not out["buf_deposit"].any()


def test_bondi_clustered_conservation_and_modes(orc):
    w = W.c3bh(nx=32, n_cic=200, n_sink=40, dtype=np.float64)
    a = orc.step(w, "f64")
    b = orc.step(w, "fix64")
    np.testing.assert_allclose(a["sink_mreq"], b["sink_mreq"], rtol=1e-15)
    np.testing.assert_array_equal(a["sink_racc"], b["sink_racc"])
    np.testing.assert_allclose(a["state"], b["state"], rtol=1e-10, atol=1e-10)
    racc = a["sink_racc"]
    # the drawn masses put sinks on all three branches of the clamp
    assert (racc == 0.25).any() and (racc == 2.0).any() and ((racc > 0.25) & (racc < 2)).any()
    n = 32 ** 3
    cic = math.fsum(w.cic.fields["m"])
    lost = math.fsum(w.state[:n]) + cic - math.fsum(b["state"][:n])
    assert math.fsum(b["sink_d"][0]) == pytest.approx(lost, rel=1e-10)


def test_bondi_parameter_errors(orc):
    x = (8.5, 8.5, 8.5)
    st = moving_gas(16, 1.0, (0, 0, 0), 1.0)
    for kw in ({"gamma": 0.9}, {"dt": -1.0}, {"G": float("nan")}, {"r_k": 0.4}):
        w = bondi_box(16, st, [x], [1.0], [(0, 0, 0)], **kw)
        with pytest.raises(RuntimeError, match="EINVAL"):
            orc.deposit(w, "f64")


def to_global(w, packed):
    """Packed per-box [5][nz][ny][nx] blocks -> one global [5][Z][Y][X] array."""
    X, Y, Z = w.domain
    out = np.zeros((5, Z, Y, X))
    off = 0
    for (x0, y0, z0), (nx, ny, nz) in zip(w.lo, w.n):
        blk = packed[off: off + 5 * nx * ny * nz].reshape(5, nz, ny, nx)
        out[:, z0:z0 + nz, y0:y0 + ny, x0:x0 + nx] = blk
        off += 5 * nx * ny * nz
    return out


@pytest.mark.parametrize("rate", [0, 1])
def test_sinks_multibox_equal_single_box(orc, rate):
    """Sinks on a 2 x 2 x 1 box tiling (kernels crossing faces, edges and the
    periodic boundary) give, in fixed point, exactly the state and sink gains
    of the same particles on one box covering the same domain."""
    pts = [(6.0, 5.0, 3.5), (5.9, 4.9, 0.2), (12.6, 13.4, 7.9), (3.5, 10.2, 4.4),
           (0.3, 0.4, 0.5)]
    cic = [(6.2, 5.1, 3.3), (1.0, 13.9, 7.5)]
    mb = W.multibox([6, 7], [5, 9], [8], ghost=2, positions_cic=cic, masses=[0.5, 0.7],
                    positions_sink=pts, sink_rate=rate, seed=3)
    assert mb.nbox == 4 and mb.sinks.n == 5
    g = to_global(mb, mb.state)
    domain, lo, n = W.single_box(13, 14, 8)
    order_s = np.lexsort((mb.sinks.fields["z"], mb.sinks.fields["y"], mb.sinks.fields["x"]))
    order_c = np.lexsort((mb.cic.fields["z"], mb.cic.fields["y"], mb.cic.fields["x"]))

    def one(P, order):
        f = {k: np.ascontiguousarray(v[order]) for k, v in P.fields.items()}
        return W.Particles(f, np.array([0, len(order)], dtype=np.int64))

    sb = dataclasses.replace(mb, lo=lo, n=n, state=g.reshape(-1),
                             sinks=one(mb.sinks, order_s), cic=one(mb.cic, order_c))
    a = orc.step(mb, "fix64")
    b = orc.step(sb, "fix64")
    assert np.array_equal(to_global(mb, a["state"]), b["state"].reshape(5, 8, 14, 13))
    for x, y in zip(a["sink_d"], b["sink_d"]):
        assert np.array_equal(x[order_s], y)
    assert a["counters"] == b["counters"] and a["counters"]["touched"] > 0
    if rate == 1:
        assert np.array_equal(a["sink_racc"][order_s], b["sink_racc"])


# ------------------------------------------------------ sink creation (S11)

def peaks_state(nx, peaks, u=(0.2, -0.1, 0.3), e_sp=1.3, rho0=1.0):
    """Uniform moving gas with single-cell density peaks {(i, j, k): rho}."""
    rho = np.full((nx, nx, nx), rho0)
    for (i, j, k), r in peaks.items():
        rho[k, j, i] = r
    st = np.zeros((5, nx, nx, nx))
    st[0] = rho
    for a in range(3):
        st[1 + a] = rho * u[a]
    st[4] = rho * (e_sp + 0.5 * float(np.dot(u, u)))
    return st.reshape(-1)


def created_cells(out, count):
    return [tuple(int(v) for v in np.floor(out[:3, s])) for s in range(count)]


def test_sink_create_single_peak(orc):
    u, e_sp, dx = np.array([0.2, -0.1, 0.3]), 1.3, 0.5
    V = dx ** 3
    st = peaks_state(16, {(5, 6, 7): 10.0}, u, e_sp)
    w = one_box(16, 3, state=st, dx=dx)
    s64 = st.copy()
    n, out = orc.sink_create(w, "f64", s64, None, 3.0, 4.0, 8)
    assert n == 1
    assert tuple(out[:3, 0]) == (5.5, 6.5, 7.5)
    assert out[3, 0] == pytest.approx(6.0 * V, rel=1e-15)
    np.testing.assert_allclose(out[4:, 0], 6.0 * V * u, rtol=1e-15)
    after = s64.reshape(5, 16, 16, 16)[:, 7, 6, 5]
    assert after[0] == 4.0
    np.testing.assert_allclose(after[1:4] / after[0], u, rtol=1e-15)
    assert after[4] / after[0] == pytest.approx(e_sp + 0.5 * float(np.dot(u, u)), rel=1e-15)
    # mass and momentum move from the cell to the sink
    assert math.fsum(s64[:16 ** 3]) * V + out[3, 0] == pytest.approx(math.fsum(st[:16 ** 3]) * V,
                                                                     rel=1e-15)
    # every other cell is untouched
    changed = np.flatnonzero(s64 != st)
    assert set(changed % 16 ** 3) == {(7 * 16 + 6) * 16 + 5}


@pytest.mark.parametrize("mode", ["f64", "fix64"])
def test_sink_create_excluded_where_sinks_remove(orc, mode):
    st = peaks_state(16, {(5, 6, 7): 10.0})
    w = one_box(16, 3, state=st, sinks=([[1.5, 1.5, 1.5]], {"a": [0.1]}), r_k=3.0)
    mesh = orc.Mesh.of(w)
    buf = np.zeros(mesh.buffer_elems, dtype=np.int64 if mode == "fix64" else np.float64)
    view = mesh.box_buffer(buf, 0)
    view[5, 7 + 3, 6 + 3, 5 + 3] = 1            # removal reaches the peak cell
    s64 = st.copy()
    n, _ = orc.sink_create(w, mode, s64, buf, 3.0, 4.0, 8)
    assert n == 0 and np.array_equal(s64, st)
    view[5, 7 + 3, 6 + 3, 5 + 3] = 0
    view[5, 7 + 3, 6 + 3, 6 + 3] = 1            # a neighbour only: creation goes ahead
    n, _ = orc.sink_create(w, mode, s64, buf, 3.0, 4.0, 8)
    assert n == 1


def test_sink_create_local_maximum_in_a_sphere(orc):
    # two peaks 2 cells apart (inside r_K = 3): only the denser
    n, out = orc.sink_create(one_box(16, 3), "f64",
                             peaks_state(16, {(5, 6, 7): 10.0, (7, 6, 7): 12.0}), None, 3.0, 4.0, 8)
    assert n == 1 and created_cells(out, n) == [(7, 6, 7)]
    # offset (2, 2, 2): inside the cube [-3, 3]^3 but |d| = sqrt(12) > 3, so both
    n, out = orc.sink_create(one_box(16, 3), "f64",
                             peaks_state(16, {(5, 6, 7): 10.0, (7, 8, 9): 12.0}), None, 3.0, 4.0, 8)
    assert n == 2 and created_cells(out, n) == [(5, 6, 7), (7, 8, 9)]
    # offset (3, 0, 0): on the sphere, |d| = r_K, so only the denser
    n, out = orc.sink_create(one_box(16, 3), "f64",
                             peaks_state(16, {(5, 6, 7): 10.0, (8, 6, 7): 12.0}), None, 3.0, 4.0, 8)
    assert n == 1
    # through the periodic boundary: (0, 0, 0) and (15, 0, 0) are neighbours
    n, out = orc.sink_create(one_box(16, 3), "f64",
                             peaks_state(16, {(0, 0, 0): 10.0, (15, 0, 0): 9.0}), None, 3.0, 4.0, 8)
    assert n == 1 and created_cells(out, n) == [(0, 0, 0)]
    # a plateau of two equal cells: one sink, in the cell of lower index
    n, out = orc.sink_create(one_box(16, 3), "f64",
                             peaks_state(16, {(5, 6, 7): 10.0, (6, 6, 7): 10.0}), None, 3.0, 4.0, 8)
    assert n == 1 and created_cells(out, n) == [(5, 6, 7)]
    # below the Truelove density: nothing
    n, _ = orc.sink_create(one_box(16, 3), "f64", peaks_state(16, {(5, 6, 7): 3.9}), None, 3.0,
                           4.0, 8)
    assert n == 0
    # r_K = 0: every cell above rho_Tr
    st = peaks_state(16, {(5, 6, 7): 10.0, (6, 6, 7): 10.0, (1, 1, 1): 5.0})
    n, out = orc.sink_create(one_box(16, 3), "f64", st, None, 0.0, 4.0, 8)
    assert n == 3 and created_cells(out, n) == [(1, 1, 1), (5, 6, 7), (6, 6, 7)]


def test_sink_create_brute_force_lognormal(orc):
    """A log-normal density field: the qualifying cells found by shifting the
    whole field over every offset of the r_K sphere."""
    nx, r_k, rho_tr = 12, 2.5, math.exp(1.2)
    rng = np.random.default_rng(21)
    st = W.gas_state(rng, nx ** 3, np.float64)
    rho = st[0].reshape(nx, nx, nx)
    idx = np.arange(nx ** 3).reshape(nx, nx, nx)
    best = rho > rho_tr
    R = int(r_k)
    for dk, dj, di in itertools.product(range(-R, R + 1), repeat=3):
        if (di, dj, dk) == (0, 0, 0) or di * di + dj * dj + dk * dk > r_k * r_k:
            continue
        ro = np.roll(rho, (-dk, -dj, -di), axis=(0, 1, 2))
        io = np.roll(idx, (-dk, -dj, -di), axis=(0, 1, 2))
        best &= (ro < rho) | ((ro == rho) & (io > idx))
    expect = np.flatnonzero(best.ravel())
    assert 5 < expect.size < 60
    w = one_box(nx, 2, state=st.reshape(-1))
    s64 = st.reshape(-1).copy()
    n, out = orc.sink_create(w, "f64", s64, None, r_k, rho_tr, 100)
    assert n == expect.size
    k, j, i = np.unravel_index(expect, (nx, nx, nx))
    np.testing.assert_array_equal(out[0, :n], i + 0.5)
    np.testing.assert_array_equal(out[1, :n], j + 0.5)
    np.testing.assert_array_equal(out[2, :n], k + 0.5)
    np.testing.assert_allclose(out[3, :n], rho.ravel()[expect] - rho_tr, rtol=1e-14)
    # too small an output list: the count is reported, nothing is created
    s2 = st.reshape(-1).copy()
    n2, _ = orc.sink_create(w, "f64", s2, None, r_k, rho_tr, expect.size - 1)
    assert n2 == expect.size and np.array_equal(s2, st.reshape(-1))


def test_sink_create_multibox_equals_single_box(orc):
    """Creation after a fixed-point step with sinks, on a 2 x 2 x 1 tiling and
    on one box covering the same domain: the same new sinks (global cell
    order) and the same state."""
    pts = [(6.0, 5.0, 3.5), (12.6, 13.4, 7.9), (0.3, 0.4, 0.5)]
    mb = W.multibox([6, 7], [5, 9], [8], ghost=2, positions_sink=pts, seed=8)
    g = to_global(mb, mb.state)
    domain, lo, n = W.single_box(13, 14, 8)
    order = np.lexsort((mb.sinks.fields["z"], mb.sinks.fields["y"], mb.sinks.fields["x"]))
    f = {k: np.ascontiguousarray(v[order]) for k, v in mb.sinks.fields.items()}
    sb = dataclasses.replace(mb, lo=lo, n=n, state=g.reshape(-1),
                             sinks=W.Particles(f, np.array([0, len(order)], dtype=np.int64)))
    rho_tr, r_k = float(np.exp(1.0)), 1.5
    res = []
    for w in (mb, sb):
        out = orc.step(w, "fix64")
        st = out["state"].copy()
        nn, rec = orc.sink_create(w, "fix64", st, out["buf_fold"], r_k, rho_tr, 256)
        # without the removal channel no cell is excluded
        nfree, _ = orc.sink_create(w, "fix64", out["state"].copy(), None, r_k, rho_tr, 256)
        res.append((nn, rec, st, nfree))
    (n1, o1, s1, f1), (n2, o2, s2, f2) = res
    assert n1 == n2 and n1 > 5
    assert np.array_equal(o1[:, :n1], o2[:, :n2])
    assert np.array_equal(to_global(mb, s1), s2.reshape(5, 8, 14, 13))
    assert f1 == f2 > n1


# ------------------------------------------------------------ C1 totals (P10)

@pytest.mark.parametrize("mode", ["f64", "fix64"])
def test_c1_closed_form_totals(orc, mode):
    w = W.c1()
    out = orc.step(w, mode)
    st = out["state"]
    n = 32 ** 3
    M = math.fsum(st[:n])
    E = math.fsum(st[4 * n:])
    assert M == pytest.approx(n + math.fsum(w.cic.fields["m"]) + 8 * 0.01, rel=1e-14)
    assert E == pytest.approx(n + 8 * 1.0, rel=1e-14)
    assert not st[n:4 * n].any()


def test_fixed_vs_f64_agree(orc):
    w = W.c4(nx=32)
    a = orc.step(w, "f64")
    b = orc.step(w, "fix64")
    np.testing.assert_allclose(a["state"], b["state"], rtol=1e-10, atol=1e-10)


def test_errors(orc):
    # particle whose host cell is not in its box
    w = W.multibox([4, 4], [4], [4], ghost=1, positions_cic=[[1.5, 1.5, 1.5]], seed=1)
    w.cic.box_off[:] = [0, 0, 1]  # claim it belongs to box 1
    with pytest.raises(RuntimeError, match="EOUTSIDE"):
        orc.deposit(w, "f64")
    # stencil reach larger than the ghost width
    w = one_box(8, 1, sn=([[0.5, 4.5, 4.5]], W.sn_fields(1, 2.0)))
    with pytest.raises(RuntimeError, match="EREACH"):
        orc.deposit(w, "f64")


# ------------------------------------- per-cell Truelove density (S6, eq. "truelove")

def two_temperature_state(nx, rho, e_cold, e_hot, u=(0.1, -0.2, 0.05)):
    """Gas with the given density field; specific internal energy e_cold in
    cells with x < nx / 2 and e_hot elsewhere (so the sound speed, and with
    it the Truelove density, differs between the halves)."""
    rho = np.asarray(rho, dtype=np.float64).reshape(nx, nx, nx)
    esp = np.where(np.arange(nx)[None, None, :] < nx // 2, e_cold, e_hot) * np.ones_like(rho)
    st = np.zeros((5, nx, nx, nx))
    st[0] = rho
    for a in range(3):
        st[1 + a] = rho * u[a]
    st[4] = rho * (esp + 0.5 * float(np.dot(u, u)))
    return st.reshape(-1)


def test_truelove_closed_form_in_uniform_gas(orc):
    """c_s^2 = gamma (gamma - 1) e_int / rho = 1 exactly (gamma = 2, specific
    e_int 1/2, gas at rest), J = 1/4, G = 1: rho_Tr = pi / 16 per cell, for
    dx = 1, and pi / 64 for dx = 2 (rho_Tr ~ 1 / dx^2).  A single peak turns
    into a sink of mass (rho - rho_Tr) V, and the cell is left at rho_Tr."""
    for dx, expect in ((1.0, math.pi / 16.0), (2.0, math.pi / 64.0)):
        st = peaks_state(12, {(4, 5, 6): 3.0}, u=(0.0, 0.0, 0.0), e_sp=0.5, rho0=0.01)
        w = one_box(12, 2, state=st, dx=dx)
        lim = W.Limits(truelove_J=0.25, G=1.0, gamma=2.0)
        s64 = st.copy()
        n, out = orc.sink_create(w, "f64", s64, None, 2.0, math.nan, 4, limits=lim)
        assert n == 1
        V = dx ** 3
        assert out[3, 0] == pytest.approx((3.0 - expect) * V, rel=1e-14)
        after = s64.reshape(5, 12, 12, 12)[:, 6, 5, 4]
        assert after[0] == pytest.approx(expect, rel=1e-14)
        assert after[4] / after[0] == pytest.approx(0.5, rel=1e-14)
        # background cells (rho 0.01 < pi / 64) never qualify; a peak below
        # the closed-form value does not either
        s2 = peaks_state(12, {(4, 5, 6): 0.99 * expect}, u=(0.0, 0.0, 0.0), e_sp=0.5,
                         rho0=0.01)
        n2, _ = orc.sink_create(w, "f64", s2.copy(), None, 2.0, math.nan, 4, limits=lim)
        assert n2 == 0


def _region_union(nx, a, b):
    """Cells with x < nx / 2 from a, the others from b (flat state arrays)."""
    ax = np.arange(nx)[None, None, None, :] < nx // 2
    return np.where(ax, a.reshape(5, nx, nx, nx), b.reshape(5, nx, nx, nx)).reshape(-1)


def test_truelove_per_cell_equals_constant_per_region(orc):
    """Two temperatures: the per-cell Truelove density is one constant in
    each half, so creation, the sink deposit and the limiter in per-cell mode
    equal, cell by cell, the constant-density runs at each half's value
    (the local-maximum test and the sink requests do not depend on it)."""
    nx = 16
    rng = np.random.default_rng(31)
    rho = np.exp(0.8 * rng.standard_normal(nx ** 3))
    # gamma = 2, gas at rest, specific e_int 1/2 and 2: c_s^2 = 2 e_int / rho is
    # exactly 1 and 4, so each half has one Truelove density, J^2 pi c_s^2 / G
    lim = W.Limits(truelove_J=0.25, G=0.1, gamma=2.0)
    st = two_temperature_state(nx, rho, 0.5, 2.0, u=(0.0, 0.0, 0.0))
    cold, hot = ((0.25 * 0.25) * math.pi) * 1.0 / 0.1, ((0.25 * 0.25) * math.pi) * 4.0 / 0.1
    per = st.reshape(5, nx, nx, nx)
    assert np.all(2.0 * per[4] / per[0] == np.where(np.arange(nx) < nx // 2, 1.0, 4.0))
    # creation
    w = one_box(nx, 3, state=st)
    s_pc = st.copy()
    n_pc, out_pc = orc.sink_create(w, "f64", s_pc, None, 2.0, math.nan, 512, limits=lim)
    s_c, s_h = st.copy(), st.copy()
    n_c, out_c = orc.sink_create(w, "f64", s_c, None, 2.0, cold, 512)
    n_h, out_h = orc.sink_create(w, "f64", s_h, None, 2.0, hot, 512)
    pick = lambda out, n, left: [tuple(out[:, s]) for s in range(n)
                                 if (out[0, s] < nx // 2) == left]
    assert 0 < len(pick(out_h, n_h, False)) and 0 < len(pick(out_c, n_c, True))
    got = [tuple(out_pc[:, s]) for s in range(n_pc)]
    want = sorted(pick(out_c, n_c, True) + pick(out_h, n_h, False),
                  key=lambda r: ((r[2] * nx) + r[1]) * nx + r[0])
    assert len(got) == len(want)
    for a, b in zip(got, want):
        assert np.allclose(a, b, rtol=0, atol=0) or a == b
    np.testing.assert_array_equal(s_pc, _region_union(nx, s_c, s_h))
    # sink deposit and limiter: sinks spread over both halves, fraction 1/4
    pos = rng.uniform(0, nx, (24, 3))
    for mode in ("f64", "fix64"):
        base = dict(state=st, sinks=(pos, {"a": np.full(24, 0.25)}), r_k=3.0, r_gauss=1.5)
        wp = one_box(nx, 3, limits=lim, **base)
        wc = one_box(nx, 3, limits=W.Limits(rho_tr=cold), **base)
        wh = one_box(nx, 3, limits=W.Limits(rho_tr=hot), **base)
        rp, rc_, rh = orc.step(wp, mode), orc.step(wc, mode), orc.step(wh, mode)
        mesh = orc.Mesh.of(wp)
        K = lambda r: owned(orc, wp, r["buf_deposit"], 5)
        xs = np.arange(nx)[None, None, :] < nx // 2
        Kp = K(rp)
        assert np.array_equal(Kp[:, :, :nx // 2], K(rc_)[:, :, :nx // 2])
        assert np.array_equal(Kp[:, :, nx // 2:], K(rh)[:, :, nx // 2:])
        assert np.array_equal(rp["state"], _region_union(nx, rc_["state"], rh["state"]))
        # Step 4 conserves mass with the per-cell limiter
        lost = (math.fsum(st[:nx ** 3]) - math.fsum(rp["state"][:nx ** 3]))
        assert math.fsum(rp["sink_d"][0]) == pytest.approx(lost, rel=1e-12)
        assert rp["counters"]["bind"] > 0 and xs.any()
        del mesh


def test_truelove_parameter_errors(orc):
    st = peaks_state(8, {(2, 2, 2): 3.0})
    w = one_box(8, 2, state=st)
    for bad in (W.Limits(truelove_J=0.25, G=0.0), W.Limits(truelove_J=0.25, gamma=0.5),
                W.Limits(truelove_J=0.25, G=math.inf)):
        with pytest.raises(RuntimeError):
            orc.sink_create(w, "f64", st.copy(), None, 2.0, 1.0, 4, limits=bad)


# --------------------------- creation: no existing sink within r_K (Sec. 3.1.2)

def test_sink_create_excluded_near_existing_sinks_by_distance(orc):
    """Criterion (3) holds by distance, whatever the buffer holds: a sink
    whose removal rounds to nothing (it requests no mass) still forbids
    creation within r_K, inclusive, also across the periodic boundary;
    just outside r_K creation goes ahead.  With only the buffer (all zero)
    the peak would become a sink."""
    from paper_2509_18261_amd.workloads import Particles
    st = peaks_state(16, {(5, 6, 7): 10.0})
    w = one_box(16, 3, state=st)
    mesh = orc.Mesh.of(dataclasses.replace(w, sinks=W._one_box(np.zeros((1, 3)),
                                                              {"a": [0.0]})))
    zero_buf = np.zeros(mesh.buffer_elems, dtype=np.int64)

    def sinks_at(*pts):
        return W._one_box(np.asarray(pts, dtype=np.float64).reshape(-1, 3),
                          {"a": np.zeros(len(pts))})

    def n_new(existing, buf=None):
        n, _ = orc.sink_create(w, "fix64", st.copy(), buf, 3.0, 4.0, 8, existing=existing)
        return n

    assert n_new(None, zero_buf) == 1
    # 2 cells away along x: excluded
    assert n_new(sinks_at((7.5, 6.5, 7.5)), zero_buf) == 0
    # exactly r_K away (centre to sink 3.0): excluded, the test is inclusive
    assert n_new(sinks_at((8.5, 6.5, 7.5))) == 0
    # just beyond r_K: allowed
    assert n_new(sinks_at((8.5 + 1e-9, 6.5, 7.5))) == 1
    # off-axis inside the cube but outside the sphere: sqrt(12) > 3
    assert n_new(sinks_at((7.5, 8.5, 9.5))) == 1
    # across the periodic boundary: peak at x = 0, sink near x = 16
    st2 = peaks_state(16, {(0, 6, 7): 10.0})
    n, _ = orc.sink_create(w, "fix64", st2.copy(), None, 3.0, 4.0, 8,
                           existing=sinks_at((15.2, 6.5, 7.5)))
    assert n == 0
    n, _ = orc.sink_create(w, "fix64", st2.copy(), None, 3.0, 4.0, 8,
                           existing=sinks_at((12.2, 6.5, 7.5)))
    assert n == 1
    assert isinstance(sinks_at((1.0, 1.0, 1.0)), Particles)


# -------------------------------------- supernova remnants, TIGRESS variant

def test_log_and_pow_against_libm(orc):
    """The power laws of Sec. 3.2.1 (M_sf, P_snr) go through the oracle's own
    log and exp: log within 4 ulp of libm, x^a within 1e-15 relative."""
    L = orc.lib()
    rng = np.random.default_rng(0)
    xs = np.concatenate([np.exp(rng.uniform(-690, 690, 4000)),
                         1.0 + rng.uniform(-1e-3, 1e-3, 1000), rng.uniform(0.5, 2.0, 1000),
                         [1.0, 2.0, 0.5, 10.0, 1e-300, 1e300]])
    for x in xs:
        a, b = L.orc_log(float(x)), math.log(x)
        assert a == b or abs(a - b) <= 4 * math.ulp(b), (x, a, b)
    for x in np.exp(rng.uniform(-20, 20, 1000)):
        for e in (-0.26, -0.17, 0.5, 2.0):
            assert abs(L.orc_pow(float(x), e) - x ** e) <= 1e-15 * x ** e


def snr_uniform(nx, rho, pos, v_s=(0.0, 0.0, 0.0), sub=1, r_k=3.0, u_gas=(0.0, 0.0, 0.0),
                e_sp=1.0, m_ej=W.SNR_M_EJ, e_sn=W.SNR_E_SN):
    """Uniform gas of density rho moving at u_gas with specific e_int e_sp,
    and supernova remnants at pos, all with velocity v_s."""
    domain, lo, n = W.single_box(nx)
    ncell = nx ** 3
    st = np.zeros((5, ncell))
    st[0] = rho
    for a in range(3):
        st[1 + a] = rho * u_gas[a]
    st[4] = rho * e_sp + 0.5 * rho * float(np.dot(u_gas, u_gas))
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    k = pos.shape[0]
    f = {"m": np.full(k, m_ej), "e": np.full(k, e_sn), "vx": np.full(k, v_s[0]),
         "vy": np.full(k, v_s[1]), "vz": np.full(k, v_s[2])}
    return W.Workload("snr_t", domain, lo, n, 4, 1.0, st.reshape(-1), snr=W._one_box(pos, f),
                      snr_params=W.SnrParams(r_k=r_k, sub=sub))


def snr_fields(orc, w, mode="f64"):
    """Deposited buffer (owned + ghost, 5 fields, float64 values) and info."""
    mesh = orc.Mesh.of(w)
    buf, _, _ = orc.deposit(w, mode, mesh)
    info = orc.deposit_snr(w, mode, buf, mesh)
    B = mesh.box_buffer(buf, 0).astype(np.float64)
    if mode == "fix64":
        B = B / Q
    return B, info


def kernel_cells(x, r_k, nx, g):
    """Centre members of the r_K sphere (sub = 1): padded-local indices and
    the offset of each centre from x (lattice enumeration)."""
    out = []
    R = int(math.ceil(r_k)) + 1
    h = [int(math.floor(c)) for c in x]
    for k in range(h[2] - R, h[2] + R + 1):
        for j in range(h[1] - R, h[1] + R + 1):
            for i in range(h[0] - R, h[0] + R + 1):
                d = np.array([i + 0.5 - x[0], j + 0.5 - x[1], k + 0.5 - x[2]])
                if (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2] <= r_k * r_k:
                    out.append(((k + g, j + g, i + g), d))
    return out


def test_snr_covered_fraction(orc):
    """sub = 1: the kernel is the 123 centre members of an r = 3 ball (a
    remnant at a cell centre), V_snr = 123; with 16^3 sample points per cell
    the covered volume approaches 4/3 pi r^3 (within 0.5%) wherever the
    remnant sits, and cells wholly inside count 1."""
    w = snr_uniform(24, 1.0, [(12.5, 12.5, 12.5)], sub=1)
    _, info = snr_fields(orc, w)
    assert info[0, 0] == 123.0
    for pos in [(12.5, 12.5, 12.5), (12.0, 12.0, 12.0), (12.31, 11.77, 12.9)]:
        w = snr_uniform(24, 1.0, [pos], sub=16)
        B, info = snr_fields(orc, w)
        assert abs(info[0, 0] - 4.0 / 3.0 * math.pi * 27.0) < 0.005 * 113.1
        # the mass share of a cell wholly inside the ball is a whole cell's
        c = [int(math.floor(p)) + 4 for p in pos]
        assert B[0, c[2], c[1], c[0]] == pytest.approx(W.SNR_M_EJ / info[0, 0], rel=1e-15)


def regime_density(target, r_k=3.0, sub=1, m_ej=W.SNR_M_EJ):
    """Uniform gas density at which R_M = M_snr / M_sf equals `target` for a
    centred remnant with sub = 1 (V_snr = 123), by bisection with libm's pow."""
    V = 123.0

    def rm(rho):
        msnr = rho * V + m_ej
        nh = msnr / V * W.SNR_NH_PER_RHO
        return msnr / (1679.0 * nh ** -0.26)
    lo, hi = 1e-8, 1e6
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        lo, hi = (mid, hi) if rm(mid) < target else (lo, mid)
    return lo


@pytest.mark.parametrize("mode", ["f64", "fix64"])
def test_snr_regimes_and_terminal_momentum(orc, mode):
    """Eqs. "dp" and "psnr" at chosen n_H: uniform gas at rest, a remnant at
    rest at a cell centre.  MC: |p_rad| = 2.8e4 n_H^-0.17 (code units);
    ST: sqrt(2 M_ej eps_K E_sn); EJ: 0.  The radial momentum per cell is
    |p_rad| / N along the cell's direction (N = 123 members, none at the
    centre cell), so sum |dp| V = |p_rad| (1 - 1/N) and sum dp = 0; the
    mass and energy totals are M_ej and E_sn (exact in fixed point); the
    thresholds 1 and 0.027 are strict from below."""
    x = (12.5, 12.5, 12.5)
    cells = kernel_cells(x, 3.0, 24, 4)
    assert len(cells) == 123
    for target, regime in ((3.0, "MC"), (1.0 + 1e-4, "MC"), (1.0 - 1e-4, "ST"), (0.2, "ST"),
                           (0.027 + 1e-5, "ST"), (0.027 - 1e-5, "EJ"), (0.005, "EJ")):
        rho = regime_density(target)
        w = snr_uniform(24, rho, [x])
        B, info = snr_fields(orc, w, mode)
        msnr = rho * 123.0 + W.SNR_M_EJ
        nh = msnr / 123.0 * W.SNR_NH_PER_RHO
        # the kernel sums lie on the 2^-40 grid: 123 roundings of at most 2^-41
        assert info[1, 0] == pytest.approx(msnr, rel=1e-12, abs=123 * 2.0 ** -41)
        assert info[2, 0] == pytest.approx(nh, rel=1e-12)
        P = {"MC": 2.8e4 * nh ** -0.17, "ST": math.sqrt(2 * W.SNR_M_EJ * 0.28 * W.SNR_E_SN),
             "EJ": 0.0}[regime]
        assert info[3, 0] == pytest.approx(P, rel=1e-12, abs=0.0), (target, regime)
        dp = np.stack([B[1 + a] for a in range(3)])
        mag = np.sqrt((dp * dp).sum(axis=0))
        tol = 1e-12 if mode == "f64" else 1e-9
        assert mag.sum() == pytest.approx(P * (1.0 - 1.0 / 123.0), rel=tol, abs=1e-9)
        for a in range(3):
            assert abs(dp[a].sum()) <= 1e-9 * max(P, 1.0)
        # each cell's momentum points away from the remnant, |p_rad| / N long
        for (k, j, i), d in cells[:20]:
            L = math.sqrt(float(d @ d))
            if L > 0:
                assert np.allclose(dp[:, k, j, i], P / 123.0 * d / L, rtol=1e-12, atol=1e-9)
        if mode == "fix64":
            assert B[0].sum() * Q == round(W.SNR_M_EJ * Q)
            assert B[4].sum() * Q == round(W.SNR_E_SN * Q)
        else:
            assert B[0].sum() == pytest.approx(W.SNR_M_EJ, rel=1e-14)
            assert B[4].sum() == pytest.approx(W.SNR_E_SN, rel=1e-14)


def test_snr_galilean_covariance(orc):
    """Boosting gas and remnant by u (sub = 1, closed forms per cell): the
    mass deposit is unchanged, the momentum deposit gains d rho u (eq. "du":
    rho_new v_COM - rho v with v_COM and v shifted by u), and the energy
    deposit gains a (E_kin' - E_kin) + u . p_rad with a = 1/N and
    p_rad = |p_rad| / N along the cell's direction."""
    x = (12.3, 11.8, 12.6)
    cells = kernel_cells(x, 3.0, 24, 4)
    N = len(cells)
    rho = regime_density(3.0)
    v_s = np.array([0.7, -0.4, 0.2])
    u = np.array([3.0, -1.5, 2.0])
    w0 = snr_uniform(24, rho, [x], v_s=tuple(v_s), u_gas=(0.2, 0.1, -0.3))
    w1 = snr_uniform(24, rho, [x], v_s=tuple(v_s + u), u_gas=tuple(np.array([0.2, 0.1, -0.3]) + u))
    B0, i0 = snr_fields(orc, w0)
    B1, i1 = snr_fields(orc, w1)
    P = i0[3, 0]
    assert P > 0 and i1[3, 0] == P
    assert np.array_equal(B0[0], B1[0])
    dEkin = 0.5 * W.SNR_M_EJ * (float((v_s + u) @ (v_s + u)) - float(v_s @ v_s))
    for (k, j, i), d in cells:
        dr = B0[0, k, j, i]
        assert dr == pytest.approx(W.SNR_M_EJ / N, rel=1e-14)
        for a in range(3):
            assert B1[1 + a, k, j, i] - B0[1 + a, k, j, i] == pytest.approx(dr * u[a], rel=1e-9,
                                                                          abs=1e-9)
        L = math.sqrt(float(d @ d))
        prad = P / N * d / L if L > 0 else np.zeros(3)
        want = dEkin / N + float(u @ prad)
        assert B1[4, k, j, i] - B0[4, k, j, i] == pytest.approx(want, rel=1e-9, abs=1e-6)


def test_snr_momentum_conservation_symmetric_kernel(orc):
    """A remnant at a cell centre in inhomogeneous, moving gas (sub = 4):
    the covered fractions and the radial directions are symmetric, so the
    radial momenta cancel and sum dp V = M_ej v_s (the gas within the kernel
    is brought to v_COM, which conserves its covered momentum)."""
    rng = np.random.default_rng(5)
    w = snr_uniform(24, 1.0, [(12.5, 12.5, 12.5)], v_s=(1.5, -2.0, 0.5), sub=4)
    st = w.state.reshape(5, -1).copy()
    st[0] = np.exp(rng.standard_normal(st.shape[1]))
    v = rng.standard_normal((3, st.shape[1]))
    st[1:4] = st[0] * v
    st[4] = st[0] * (1.0 + 0.5 * (v * v).sum(axis=0))
    w = w.with_state(st.reshape(-1))
    for rho_scale in (1.0, 30.0):
        ws = w.with_state((st * np.array([[rho_scale]] * 5)).reshape(-1))
        B, info = snr_fields(orc, ws)
        assert info[3, 0] > 0
        tot = [B[1 + a].sum() for a in range(3)]
        want = W.SNR_M_EJ * np.array([1.5, -2.0, 0.5])
        assert np.allclose(tot, want, rtol=1e-10, atol=1e-8 * max(info[3, 0], 1.0))


def test_snr_superposition_and_permutation_fixed_point(orc):
    """Each remnant reads the state before the step, so in fixed point the
    deposit of several overlapping remnants is the sum of their single
    deposits, and it does not depend on their order."""
    pts = [(10.2, 11.7, 12.1), (12.9, 12.4, 10.8), (11.1, 13.3, 12.6)]
    w = W.snr_box(nx=24, n_snr=3, seed=11)
    w = dataclasses.replace(w, snr=W._one_box(np.array(pts), {k: v[:3] for k, v in
                                                              w.snr.fields.items()
                                                              if k not in "xyz"}))
    mesh = orc.Mesh.of(w)

    def dep(ww):
        b, _, _ = orc.deposit(ww, "fix64", mesh)
        orc.deposit_snr(ww, "fix64", b, mesh)
        return b

    full = dep(w)
    parts = []
    for s in range(3):
        f = {k: v[s:s + 1] for k, v in w.snr.fields.items()}
        parts.append(dep(dataclasses.replace(w, snr=W.Particles(f, np.array([0, 1])))))
    assert np.array_equal(full, parts[0] + parts[1] + parts[2])
    perm = [2, 0, 1]
    f = {k: v[perm] for k, v in w.snr.fields.items()}
    assert np.array_equal(full, dep(dataclasses.replace(w, snr=W.Particles(f, np.array([0, 3])))))


def test_snr_limiter_binds_and_floor_holds(orc):
    """Remnants near the density steps of the slab workload: the energy
    limiter (eq. "lambda") binds on real radial momentum, and after the step
    every cell keeps e_int >= 0; the three regimes all occur."""
    w = W.snr_box()
    r = orc.step(w, "f64")
    assert r["counters"]["lam"] > 0
    info = r["snr_info"]
    rm = info[1] / (1679.0 * info[2] ** -0.26)
    assert (rm > 1).any() and ((rm > 0.027) & (rm <= 1)).any() and (rm <= 0.027).any()
    st = r["state"].reshape(5, -1)
    eint = st[4] - 0.5 * (st[1:4] ** 2).sum(axis=0) / st[0]
    assert (eint >= -1e-9 * np.abs(st[4])).all()


def test_snr_multibox_equals_single_box(orc):
    """The same gas and remnants on a 3 x 3 x 3 tiling with uneven boxes
    (kernels crossing faces, edges and the periodic boundary) give, in fixed
    point, exactly the single box's state."""
    mb = W.snr_box(nb=3)
    sb = W.snr_box(nb=1)
    a = orc.step(mb, "fix64")
    b = orc.step(sb, "fix64")
    X = mb.domain[0]
    assert np.array_equal(to_global(mb, a["state"]), b["state"].reshape(5, X, X, X))
    assert a["counters"] == b["counters"]


def test_snr_parameter_errors(orc):
    w = snr_uniform(16, 1.0, [(8.5, 8.5, 8.5)])
    for bad in (dict(sub=3), dict(sub=0), dict(r_k=-1.0), dict(nh_per_rho=0.0),
                dict(msf_coef=-1.0), dict(sub=32)):
        ww = dataclasses.replace(w, snr_params=dataclasses.replace(w.snr_params, **bad))
        with pytest.raises(RuntimeError):
            snr_fields(orc, ww)
    # a kernel reaching past the ghost zone: from x = 15.9, sample points of
    # cell 20 lie within 4.9, five cells beyond the host cell with g = 4
    ww = snr_uniform(16, 1.0, [(15.9, 8.5, 8.5)], r_k=4.9)
    with pytest.raises(RuntimeError):
        snr_fields(orc, ww)


@pytest.mark.parametrize("mode", ["f64", "fix64"])
def test_snr_radial_momentum_with_covered_fractions(orc, mode):
    """sub = 4, a remnant at rest at a cell centre in uniform gas at rest: each
    cell receives |p_rad| w / V_snr along its direction, so
    sum |dp| V = |p_rad| (V_snr - V) / V_snr (the centre cell, wholly covered,
    has no direction), and the mass shares w M_ej / V_snr sum to M_ej."""
    rho = regime_density(3.0)
    w = snr_uniform(24, rho, [(12.5, 12.5, 12.5)], sub=4)
    B, info = snr_fields(orc, w, mode)
    P, Vsnr = info[3, 0], info[0, 0]
    assert P > 0 and 110.0 < Vsnr < 116.0
    dp = np.stack([B[1 + a] for a in range(3)])
    mag = np.sqrt((dp * dp).sum(axis=0))
    tol = 1e-12 if mode == "f64" else 1e-9
    assert mag.sum() == pytest.approx(P * (Vsnr - 1.0) / Vsnr, rel=tol)
    # partially covered cells: |dp| / d rho = |p_rad| / M_ej wherever both are set
    sel = (B[0] > 0) & (mag > 0)
    assert np.allclose(mag[sel] / B[0][sel], P / W.SNR_M_EJ, rtol=1e-6)
    frac = B[0][sel] * Vsnr / W.SNR_M_EJ
    assert (frac < 0.999).sum() > 50  # fractional cells present


@pytest.mark.parametrize("mode", ["f64", "fix64"])
def test_cells_without_an_update_keep_their_state(orc, mode):
    """Step 5 adds a zero update to a cell no particle reaches, and the limiters
    act on updates: such a cell keeps its state bit for bit (eta = 1, nothing
    counted), even where that state violates the energy floor; a touched cell
    with the same violating state is lifted to the floor and counted."""
    rng = np.random.default_rng(12)
    n = 64
    rho = np.exp(rng.standard_normal(n))
    v = rng.standard_normal((3, n))
    p = rho * v
    E = 0.5 * (p * p).sum(0) / rho * np.where(np.arange(n) % 2 == 0, 0.5, 2.0)  # even: e_int < 0
    state = np.concatenate([rho, p[0], p[1], p[2], E])
    for eint_mode in (0, 1):
        w = W.Workload("u", *W.single_box(n, 1, 1), 0, 1.0, state.copy(),
                       limits=W.Limits(eint_mode=eint_mode))
        touched = np.arange(n) % 4 < 2  # every other pair: one violating, one valid
        q = np.zeros(5 * n)
        q[0:n] = np.where(touched, 0.25, 0.0)
        q[4 * n:5 * n] = np.where(touched, 0.5, 0.0)
        buf = (np.rint(q * Q).astype(np.int64) if mode == "fix64" else q)
        st, eta, cnt = orc.apply(w, mode, buf, want_eta=True)
        st = st.reshape(5, n)
        ref = state.reshape(5, n)
        assert np.array_equal(st[:, ~touched], ref[:, ~touched])
        assert np.all(eta == 1.0)
        # untouched cells that violate the floor still do; touched ones meet it
        e_old = ref[4] - 0.5 * (ref[1:4] ** 2).sum(0) / ref[0]
        assert (e_old[~touched] < 0).sum() == (~touched).sum() // 2
        if eint_mode == 0:
            e1 = st[4] - 0.5 * (st[1:4] ** 2).sum(0) / st[0]
            assert np.all(e1[touched] >= -1e-12 * st[4][touched])
            assert cnt["fall"] > 0
