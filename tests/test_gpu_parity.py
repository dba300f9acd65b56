"""Parity of the HIP path against the serial oracle, through the C-ABI.

Bar: int64 fixed point (buffers, folded buffers, sink sums, eta and the
applied state) bit-exact; FP64 accumulation within 1e-12 and FP32 within
1e-6, both as max|x - r| / max|r| per field against the FP64 oracle."""
import dataclasses
import math
import sys

import numpy as np
import pytest

from paper_2509_18261_amd import workloads as W

from buffers import expand_channels

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-6}


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_18261_amd import binding
    return binding


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_gpu(B, w, acc, want_eta=True, tuning=None, channels="all"):
    import torch
    ctx = B.Context(w, acc, channels=channels)
    if tuning:
        ctx.set_tuning(**tuning)
    ctx.deposit()
    dep = expand_channels(w, ctx.buf.cpu().numpy().copy(), ctx.fields)
    ctx.ghost_fold()
    fold = expand_channels(w, ctx.buf.cpu().numpy().copy(), ctx.fields)
    ctx.sink_update()
    eta = torch.empty(ctx.owned_cells, dtype=torch.float64, device="cuda") if want_eta else None
    ctx.apply(eta)
    torch.cuda.synchronize()
    out = {"buf_deposit": dep, "buf_fold": fold, "state": ctx.state.cpu().numpy(),
           "status": ctx.status()}
    if eta is not None:
        out["eta"] = eta.cpu().numpy()
    if ctx.sink_out is not None:
        n = w.sinks.n
        s = ctx.sink_out.cpu().numpy()
        out["sink_d"] = (s[:n], s[n:2 * n], s[2 * n:3 * n], s[3 * n:])
    ctx.close()
    return out


def field_views(w, flat, kind):
    """Split a packed array into per-field 1-D arrays (over all boxes)."""
    nf = w.nfield if kind == "buf" else 5
    g = w.ghost if kind == "buf" else 0
    sizes = [int(np.prod(n + 2 * g)) for n in w.n.astype(np.int64)]
    out = [[] for _ in range(nf)]
    off = 0
    for s in sizes:
        for f in range(nf):
            out[f].append(flat[off + f * s: off + (f + 1) * s])
        off += nf * s
    return [np.concatenate(o) for o in out]


def rel_err(x, r):
    x = x.astype(np.float64)
    r = r.astype(np.float64)
    den = np.max(np.abs(r)) if r.size else 0.0
    num = np.max(np.abs(x - r)) if r.size else 0.0
    if den == 0.0:
        return num
    return num / den


def compare(w, acc, got, ref):
    if acc == "fix64":
        assert np.array_equal(got["buf_deposit"], ref["buf_deposit"]), "deposit buffer differs"
        assert np.array_equal(got["buf_fold"], ref["buf_fold"]), "folded buffer differs"
        st_ref = ref["state"].astype(got["state"].dtype)
        bad = np.flatnonzero(got["state"] != st_ref)
        assert bad.size == 0, f"{bad.size} state values differ, first at {bad[:5]}"
        assert np.array_equal(got["eta"], ref["eta"])
        if "sink_d" in ref:
            for a, b in zip(got["sink_d"], ref["sink_d"]):
                assert np.array_equal(a, b)
        return
    tol = TOL[acc]
    for key in ("buf_deposit", "buf_fold"):
        for f, (x, r) in enumerate(zip(field_views(w, got[key], "buf"),
                                       field_views(w, ref[key], "buf"))):
            e = rel_err(x, r)
            assert e <= tol, f"{key} field {f}: {e:.3e} > {tol}"
    # the state is stored in its own type: compare with the oracle rounded to
    # that type, allowing the tolerance or one unit of the stored precision
    sdt = got["state"].dtype
    stol = max(tol, float(np.finfo(sdt).eps))
    for f, (x, r) in enumerate(zip(field_views(w, got["state"], "state"),
                                   field_views(w, ref["state"].astype(sdt), "state"))):
        e = rel_err(x, r)
        assert e <= stol, f"state field {f}: {e:.3e} > {stol}"
    if "sink_d" in ref:
        for a, b in zip(got["sink_d"], ref["sink_d"]):
            assert rel_err(a, b) <= max(tol, 1e-9)


def check(B, orc, w, acc, **kw):
    say(f"case {w.name} acc={acc} nbox={w.nbox} cic={w.cic.n if w.cic else 0} "
        f"sn={w.sn.n if w.sn else 0} sinks={w.sinks.n if w.sinks else 0}")
    got = run_gpu(B, w, acc, **kw)
    assert got["status"]["flags"] in (0, 0x10), got["status"]
    ref = orc.step(w, "fix64" if acc == "fix64" else "f64", want_eta=True)
    compare(w, acc, got, ref)
    if acc == "fix64":
        for k in ("touched", "bind", "lam", "fall"):
            assert got["status"][k] == ref["counters"][k], (k, got["status"], ref["counters"])
    return got, ref


# ------------------------------------------------------------- small configs

SMALL = {
    "c1": lambda: W.c1(),
    "c2_40": lambda: W.c2(nx=40),
    "c3_40": lambda: W.c3(nx=40, n_sink=48),
    "c3bh_40": lambda: W.c3bh(nx=40, n_sink=48),
    "c4_48": lambda: W.c4(nx=48),
    "c5_4": lambda: W.c5(nb=4),
    "c5s_4": lambda: W.c5s(nb=4),
    "c5sbh_4": lambda: W.c5s(nb=4, bondi=True),
    "c3tl_40": lambda: truelove(W.c3(nx=40, n_sink=48)),
    "c5sbhtl_4": lambda: truelove(W.c5s(nb=4, bondi=True), G=0.04),
    # wide sink kernels (r_K = 7, ghost 7): the owner-tile sink flags walk
    # 19 planes per sink, more than the 16 threads a sink gets
    "c3_40_rk7": lambda: dataclasses.replace(W.c3(nx=40, n_sink=48), ghost=7, r_k=7.0,
                                            r_gauss=3.0),
}


def truelove(w, J=0.25, G=0.05):
    """The workload with the per-cell Truelove density (eq. "truelove"): its gas
    has specific e_int = 1, so with gamma 5/3 each cell's rho_Tr is about
    J^2 pi (10/9) / G (4.4 for G = 0.05), which the densest few percent of the
    log-normal cells exceed."""
    return dataclasses.replace(w, name=w.name + "_truelove",
                               limits=dataclasses.replace(w.limits, truelove_J=J, G=G))


@pytest.mark.parametrize("path", [1, 0])
@pytest.mark.parametrize("acc", ["fix64", "f64", "f32"])
@pytest.mark.parametrize("name", list(SMALL))
def test_small_configs(B, orc, name, acc, path):
    check(B, orc, SMALL[name](), acc, tuning={"deposit_path": path})


def test_c1_fp64_state_all_modes(B, orc):
    w = W.c1()
    assert w.state.dtype == np.float64
    for acc in ("fix64", "f64", "f32"):
        check(B, orc, w, acc)


def edge_workloads():
    out = []
    edges = ([5, 7], [6, 4], [4, 6])
    pos_c = [[5.0, 6.0, 4.0], [0.0, 0.0, 0.0], [4.99, 5.99, 3.99], [11.5, 9.5, 9.5],
             [5.0, 2.5, 7.2], [0.25, 9.75, 4.0], [6.0, 6.0, 6.0], [11.999999, 9.999999, 9.999]]
    pos_s = [[5.0, 6.0, 4.0], [0.1, 9.9, 9.9], [11.9, 0.2, 5.0], [3.3, 3.3, 3.3], [0.0, 0.0, 0.0]]
    out.append(W.multibox(*edges, ghost=2, positions_cic=pos_c, positions_sn=pos_s,
                          sn_radius=1.5, seed=3, dtype=np.float32))
    # boxes smaller than twice the ghost width: several periodic images per cell
    rng = np.random.default_rng(9)
    w = W.Workload("tiny", *W.single_box(3, 4, 3), 2, 1.0,
                   W.gas_state(rng, 36, np.float64).reshape(-1),
                   cic=W._one_box(W.uniform_positions(rng, 9, (3, 4, 3)), W.cic_fields(rng, 9)),
                   sn=W._one_box(W.uniform_positions(rng, 3, (3, 4, 3)), W.sn_fields(3, 1.7)))
    out.append(w)
    # a 3x2x1 layout with many particles on box corners and an empty box
    edges = ([3, 8, 5], [6, 6], [9])
    pts = [[3.0, 6.0, 0.0], [11.0, 0.0, 4.5], [0.0, 0.0, 8.999], [3.0, 6.0, 4.5]] * 5
    out.append(W.multibox(*edges, ghost=1, positions_cic=pts, positions_sn=pts[:4],
                          sn_radius=1.0, seed=4))
    # no particles at all: the step must leave the state unchanged
    out.append(dataclasses.replace(W.c2(nx=16), cic=None, sn=None, name="empty"))
    # supernova radius 0: only the host cell (or the cell whose centre it is)
    rng = np.random.default_rng(2)
    out.append(W.Workload("r0", *W.single_box(8), 1, 1.0,
                          W.gas_state(rng, 512, np.float32).reshape(-1),
                          sn=W._one_box(W.uniform_positions(rng, 20, (8, 8, 8)),
                                        W.sn_fields(20, 0.0))))
    return out


@pytest.mark.parametrize("path", [1, 0])
@pytest.mark.parametrize("acc", ["fix64", "f64", "f32"])
@pytest.mark.parametrize("idx", range(5))
def test_edge_layouts(B, orc, idx, acc, path):
    w = edge_workloads()[idx]
    got, _ = check(B, orc, w, acc, tuning={"deposit_path": path})
    if w.name == "empty":
        assert np.array_equal(got["state"], w.state)


SINK_EDGE_PTS = [(6.0, 5.0, 3.5), (5.9, 4.9, 0.2), (12.6, 13.4, 7.9), (3.5, 10.2, 4.4),
                 (0.3, 0.4, 0.5), (6.5, 5.5, 4.0), (6.99, 13.99, 7.99)]


@pytest.mark.parametrize("rate", [0, 1])
@pytest.mark.parametrize("acc", ["fix64", "f64", "f32"])
def test_multibox_sinks_on_faces_and_corners(B, orc, acc, rate):
    """Sinks on box faces, edges and corners of a 2 x 2 x 1 tiling, with
    kernels reaching into three other boxes and across the periodic boundary."""
    w = W.multibox([6, 7], [5, 9], [8], ghost=2, positions_cic=[(6.2, 5.1, 3.3)],
                   masses=[0.5], positions_sink=SINK_EDGE_PTS, sink_rate=rate, seed=3,
                   dtype=np.float32 if acc == "f32" else np.float64)
    check(B, orc, w, acc)


SHAPES = [
    {"deposit_path": 0, "block": 64, "sn_lanes": 16},
    {"deposit_path": 0, "block": 1024, "sn_lanes": 32},
    {"deposit_path": 1, "tile_x": 16, "tile_yz": 2, "tile_block": 64},
    {"deposit_path": 1, "tile_x": 32, "tile_yz": 8, "tile_block": 1024},
    {"deposit_path": 1, "tile_x": 64, "tile_yz": 4, "tile_grid_per_cu": 1},
    {"deposit_path": 1, "tile_x": 16, "tile_yz": 4, "tile_grid_per_cu": 3, "block": 128},
    # split tiles: small chunk thresholds put most tiles through the chunked path
    {"deposit_path": 1, "chunk_cic": 64, "chunk_sn": 16},
    {"deposit_path": 1, "tile_x": 16, "tile_yz": 2, "chunk_cic": 64, "chunk_sn": 16,
     "tile_grid_per_cu": 1},
    # lanes per supernova in the member count
    {"deposit_path": 1, "count_lanes": 1},
    {"deposit_path": 1, "count_lanes": 16},
    # long x tiles
    {"deposit_path": 1, "tile_x": 128, "tile_yz": 2, "tile_block": 256},
    {"deposit_path": 1, "tile_x": 256, "tile_yz": 4, "tile_block": 512},
]


def test_launch_shape_invariance_fixed_point(B, orc):
    """Fixed point gives the same bits whatever the path, tiles or launch shape."""
    w = W.c4(nx=40)
    base = run_gpu(B, w, "fix64")
    for tun in SHAPES:
        say("tuning", tun)
        other = run_gpu(B, w, "fix64", tuning=tun)
        assert np.array_equal(base["buf_deposit"], other["buf_deposit"])
        assert np.array_equal(base["buf_fold"], other["buf_fold"])
        assert np.array_equal(base["state"], other["state"])


def test_scratch_grown_by_another_shape(B, orc):
    """One context bins with a many-tile shape first (its scratch grows to
    that shape's histograms), then with a large-tile shape: the second
    deposit's launches are sized by its own slices, and its buffer equals the
    oracle's and a fresh context's bit for bit (fixed point)."""
    import torch
    w = W.c4(nx=48)
    small = {"deposit_path": 1, "tile_x": 16, "tile_yz": 2}
    large = {"deposit_path": 1, "tile_x": 64, "tile_yz": 8}
    ctx = B.Context(w, "fix64")
    ctx.set_tuning(**small)
    ctx.deposit()
    first = ctx.buf.cpu().numpy().copy()
    ctx.set_tuning(**large)
    ctx.deposit()
    torch.cuda.synchronize()
    second = ctx.buf.cpu().numpy().copy()
    fields = ctx.fields
    st = ctx.status()
    ctx.close()
    assert st["flags"] in (0, 0x10), st
    assert np.array_equal(first, second)
    got = expand_channels(w, second, fields)
    fresh = run_gpu(B, w, "fix64", tuning=large)
    assert np.array_equal(got, fresh["buf_deposit"])
    ref = orc.step(w, "fix64", want_eta=False)
    assert np.array_equal(got, ref["buf_deposit"])


def test_tiled_paths_multibox(B, orc):
    """Tile shapes on an uneven multi-box layout, every mode against the oracle."""
    w = W.c5(nb=3, n_total=20000)
    for tun in SHAPES[2:]:
        for acc in ("fix64", "f32"):
            check(B, orc, w, acc, tuning=tun)


@pytest.mark.parametrize("acc", ["fix64", "f32", "f64"])
def test_split_tiles_clustered(B, orc, acc):
    """Clustered particles with small chunk thresholds: split tiles combine
    their chunks exactly (fixed point) or within tolerance."""
    w = W.c3(nx=48, n_sink=16)
    check(B, orc, w, acc, tuning={"deposit_path": 1, "chunk_cic": 64, "chunk_sn": 16})


def test_split_tiles_out_of_slots(B, orc):
    """More chunks than chunk slots: the tiles that find no slots stay whole,
    and the result is unchanged."""
    w = W.c3(nx=128, n_sink=16)
    assert w.cic.n / 64 > 4 * 256
    check(B, orc, w, "fix64", tuning={"deposit_path": 1, "chunk_cic": 64, "chunk_sn": 16})


def test_run_twice_bitwise(B):
    w = W.c3(nx=40, n_sink=48)
    a = run_gpu(B, w, "fix64")
    b = run_gpu(B, w, "fix64")
    for k in ("buf_fold", "state", "eta"):
        assert np.array_equal(a[k], b[k])


def test_limiter_binds_on_clustered_sinks(B, orc):
    got, ref = check(B, orc, W.c3(nx=64, n_sink=256), "fix64")
    st = got["status"]
    assert st["touched"] > 0
    assert st["bind"] / st["touched"] >= 0.10, st


def test_bondi_sink_parameter_errors(B):
    """Bondi-Hoyle sink parameters are checked on the host before any launch."""
    w = W.c3bh(nx=16, n_cic=10, n_sink=4, dtype=np.float64)
    for kw, msg in (({"gamma": 0.5}, "gamma"), ({"dt": float("inf")}, "dt"),
                    ({"r_k": 0.4}, "r_k")):
        bad = dataclasses.replace(w, **kw)
        say(f"case bondi error {kw}")
        ctx = B.Context(bad, "f64")
        with pytest.raises(B.PmpError):
            ctx.deposit()
        ctx.close()
    ctx = B.Context(w, "f64")
    ctx.sinks.rate = 7
    with pytest.raises(B.PmpError):
        ctx.deposit()
    ctx.close()


def test_outside_particle_flagged(B):
    import torch
    w = W.multibox([4, 4], [4], [4], ghost=1, positions_cic=[[1.5, 1.5, 1.5], [5.5, 1.5, 1.5]],
                   seed=1)
    w.cic.box_off[:] = [0, 0, 2]  # both claimed by box 1; the first is not in it
    ctx = B.Context(w, "fix64")
    ctx.step()
    torch.cuda.synchronize()
    st = ctx.status()
    assert "OUTSIDE" in st["flag_names"]
    ctx.close()


def test_geometry_errors(B):
    # overlapping boxes are refused at create
    w = W.multibox([4, 4], [4], [4], ghost=1, seed=1)
    w.lo[1, 0] = 2
    with pytest.raises(B.PmpError, match="ERANGE"):
        B.Context(w, "fix64")
    # supernova reach beyond the ghost width is refused before launch
    rng = np.random.default_rng(0)
    w = W.Workload("reach", *W.single_box(8), 1, 1.0, W.gas_state(rng, 512, np.float32).reshape(-1),
                   sn=W._one_box(np.array([[4.5, 4.5, 4.5]]), W.sn_fields(1, 2.0)))
    ctx = B.Context(w, "f32")
    with pytest.raises(B.PmpError, match="ERANGE"):
        ctx.deposit()
    ctx.close()


GRAPH_CASES = {
    "c2_32": lambda: W.c2(nx=32),
    "c3bh_32": lambda: W.c3bh(nx=32, n_cic=2000, n_sink=24),
    "c5s_4": lambda: W.c5s(nb=4),
}


@pytest.mark.parametrize("name", list(GRAPH_CASES))
def test_graph_replays_match_eager(B, name):
    """A captured 3-step graph equals 3 eager steps (state and, with sinks,
    the last step's sink gains), on every replay, with eager work and
    synchronisation between replays."""
    import torch
    w = GRAPH_CASES[name]()
    say(f"case graph {name}")
    eager = B.Context(w, "fix64")
    for _ in range(3):
        eager.step()
    torch.cuda.synchronize()
    ref = eager.state.cpu().numpy()
    ref_sink = None if eager.sink_out is None else eager.sink_out.cpu().numpy()
    g = B.Context(w, "fix64")
    g.graph_build(3)
    for rep in range(3):
        g.reset_state()
        torch.cuda.synchronize()
        g.graph_launch()
        torch.cuda.synchronize()
        assert np.array_equal(g.state.cpu().numpy(), ref), f"replay {rep}"
        if ref_sink is not None:
            assert np.array_equal(g.sink_out.cpu().numpy(), ref_sink), f"replay {rep} sinks"
        eager.reset_state()
        eager.step()
        torch.cuda.synchronize()
    eager.close()
    g.close()


def step_vs_oracle(B, orc, w, acc, channels="all", tuning=None):
    import torch
    ctx = B.Context(w, acc, channels=channels)
    if tuning:
        ctx.set_tuning(**tuning)
    ctx.profile_begin(16)
    ctx.step()
    torch.cuda.synchronize()
    phases = ctx.profile_end()
    got = ctx.state.cpu().numpy()
    st = ctx.status()
    ctx.close()
    assert st["flags"] in (0, 0x10), st
    ref = orc.step(w, "fix64" if acc == "fix64" else "f64", want_eta=True)
    out = {"status": st, "oracle_counters": ref["counters"], "phases": phases}
    if acc == "fix64":
        assert np.array_equal(got, ref["state"].astype(got.dtype))
        for k in ("touched", "bind", "lam", "fall"):
            assert st[k] == ref["counters"][k], (k, st, ref["counters"])
    else:
        for f, (x, r) in enumerate(zip(field_views(w, got, "state"),
                                       field_views(w, ref["state"].astype(got.dtype), "state"))):
            assert rel_err(x, r) <= max(TOL[acc], float(np.finfo(got.dtype).eps)), f
    return out


@pytest.mark.parametrize("fuse", [2, 1, 0])
@pytest.mark.parametrize("acc", ["fix64", "f64", "f32"])
@pytest.mark.parametrize("idx", range(5))
def test_step_edge_layouts(B, orc, idx, acc, fuse):
    """pmp_step on the edge layouts, with the apply fused into the tile pass
    (interior cells) and the shell folded and applied together, or not."""
    w = edge_workloads()[idx]
    say(f"step edge {w.name} acc={acc} fuse={fuse}")
    step_vs_oracle(B, orc, w, acc, tuning={"deposit_path": 1, "fuse_apply": fuse})


def owner_tiles_fit(w, tx, tyz):
    """Owner tiles fit a layout when no tile along an axis is wider than the
    domain less 2g cells (the library's own rule)."""
    t = (tx, tyz, tyz)
    n = w.n.astype(np.int64)
    return all(max(min(t[a], int(v)) for v in n[:, a]) <= int(w.domain[a]) - 2 * w.ghost
               for a in range(3))


def irregular_layout(seed=13, dtype=np.float64, kind="three"):
    """Boxes that are not a rectilinear grid, with CIC and supernovae, some
    on the faces and edges.  "three": box 0 meets three boxes across its +x
    face (and, periodically, across its -x face), so a stencil there finds its
    tiles through the owner index.  "misaligned": the box beyond the +x faces
    of boxes 0 and 1 spans both, so its tiles straddle their y faces."""
    rng = np.random.default_rng(seed)
    if kind == "three":
        domain = (24, 16, 16)
        lo = np.array([[0, 0, 0], [12, 0, 0], [12, 8, 0], [12, 8, 8]], np.int32)
        n = np.array([[12, 16, 16], [12, 8, 16], [12, 8, 8], [12, 8, 8]], np.int32)
        face_y = [7.9, 8.0, 15.95]
    else:
        domain = (24, 24, 16)
        lo = np.array([[0, 0, 0], [0, 10, 0], [12, 0, 0]], np.int32)
        n = np.array([[12, 10, 16], [12, 14, 16], [12, 24, 16]], np.int32)
        face_y = [9.6, 10.0, 10.3, 23.9]
    ncell = int(np.prod(domain))
    state = W.pack_by_box(W.gas_state(rng, ncell, dtype), n)

    def group(pos, fields):
        cell = np.floor(pos).astype(np.int64)
        box = np.full(len(pos), -1)
        for b in range(len(lo)):
            inside = np.all((cell >= lo[b]) & (cell < lo[b] + n[b]), axis=1)
            box[inside] = b
        assert (box >= 0).all()
        order = np.argsort(box, kind="stable")
        off = np.concatenate([[0], np.cumsum(np.bincount(box, minlength=len(lo)))])
        out = {"x": pos[order, 0].copy(), "y": pos[order, 1].copy(), "z": pos[order, 2].copy()}
        for k, v in fields.items():
            out[k] = np.asarray(v, np.float64)[order].copy()
        return W.Particles(out, off.astype(np.int64))

    def positions(count):
        p = rng.uniform(0, 1, (count, 3)) * np.array(domain)
        faces = rng.random(count) < 0.5
        p[faces, 0] = rng.choice([0.0, 11.7, 12.0, 23.9], faces.sum())
        edge = rng.random(count) < 0.3
        p[edge, 1] = rng.choice(face_y, edge.sum())
        return np.mod(p, np.array(domain, np.float64))

    pc, ps = positions(400), positions(60)
    return W.Workload(f"irregular_{kind}", domain, lo, n, 2, 1.0, state,
                      cic=group(pc, W.cic_fields(rng, len(pc))),
                      sn=group(ps, W.sn_fields(len(ps), 1.7)))


OWNER_CASES = {
    "irregular": irregular_layout,
    "misaligned": lambda: irregular_layout(seed=14, kind="misaligned"),
    "edge_multibox": lambda: edge_workloads()[0],
    "edge_corners": lambda: edge_workloads()[2],
    "c2_40": lambda: W.c2(nx=40),
    "c4_48": lambda: W.c4(nx=48),
    "c5_4": lambda: W.c5(nb=4),
    "c4_40": lambda: W.c4(nx=40, seed=7),
}


@pytest.mark.parametrize("split", [False, True])
@pytest.mark.parametrize("shape", [(16, 4), (32, 2)])
@pytest.mark.parametrize("acc", ["fix64", "f64", "f32"])
@pytest.mark.parametrize("name", list(OWNER_CASES))
def test_step_owner_tiles(B, orc, name, acc, shape, split):
    """The fold-free step (fuse_apply 2): tiles over owned cells only, each
    particle binned into every tile a periodic image of its stencil reaches,
    every owned cell applied from its complete LDS sum; no fold launch, and
    the oracle's step (fixed point bit for bit, with its limiter counters)."""
    w = OWNER_CASES[name]()
    tx, tyz = shape
    assert owner_tiles_fit(w, tx, tyz)
    tun = {"deposit_path": 1, "fuse_apply": 2, "tile_x": tx, "tile_yz": tyz}
    if split:
        tun.update(chunk_cic=64, chunk_sn=16)
    say(f"owner tiles {w.name} acc={acc} tile {tx}x{tyz} split={split}")
    out = step_vs_oracle(B, orc, w, acc, tuning=tun)
    assert "fold" not in out["phases"] and "tile" in out["phases"], out["phases"]


@pytest.mark.parametrize("idx", [1, 4])
def test_step_owner_tiles_fall_back(B, orc, idx):
    """Layouts the owner tiles do not fit (a domain under 2g + tile cells
    along an axis) run fuse_apply 2 as the fused step with a fold."""
    w = edge_workloads()[idx]
    assert not owner_tiles_fit(w, 16, 2)
    out = step_vs_oracle(B, orc, w, "fix64",
                         tuning={"deposit_path": 1, "fuse_apply": 2, "tile_x": 16, "tile_yz": 2})
    assert "fold" in out["phases"], out["phases"]


def test_owner_tiles_not_in_reproducibility_mode(B):
    """fuse_apply 2 in the reproducibility mode (its bounds follow the fold's
    order) runs the ghost-zone step with its fold."""
    import torch
    w = W.c2(nx=40)
    ctx = B.Context(w, "f64r", channels="all")
    ctx.set_tuning(deposit_path=1, fuse_apply=2, tile_x=16, tile_yz=4)
    assert owner_tiles_fit(w, 16, 4)
    ctx.profile_begin(16)
    ctx.step()
    torch.cuda.synchronize()
    phases = ctx.profile_end()
    ctx.close()
    assert "fold" in phases, phases


OWNER_SINK_CASES = ["c3_40", "c3bh_40", "c3tl_40", "c5s_4", "c5sbh_4", "c5sbhtl_4", "c3_40_rk7"]


@pytest.mark.parametrize("acc", ["fix64", "f64", "f32"])
@pytest.mark.parametrize("name", OWNER_SINK_CASES)
def test_step_owner_tiles_with_sinks(B, orc, name, acc):
    """Steps with sinks on owner tiles: the tile pass stores the owned cells,
    the sinks add their removal to the owning cells, no fold runs, then the
    sink update and the apply; the oracle's state and sink gains (fixed point
    bit for bit)."""
    import torch
    w = SMALL[name]()
    assert owner_tiles_fit(w, 16, 4)
    say(f"owner tiles with sinks {w.name} acc={acc}")
    ctx = B.Context(w, acc, channels="all")
    ctx.set_tuning(deposit_path=1, fuse_apply=2, tile_x=16, tile_yz=4)
    ctx.profile_begin(16)
    ctx.step()
    torch.cuda.synchronize()
    phases = ctx.profile_end()
    got = ctx.state.cpu().numpy()
    st = ctx.status()
    sink = ctx.sink_out.cpu().numpy()
    ctx.close()
    assert "fold" not in phases and "sink_deposit" in phases, phases
    assert st["flags"] in (0, 0x10), st
    ref = orc.step(w, "fix64" if acc == "fix64" else "f64", want_eta=True)
    k = w.sinks.n
    if acc == "fix64":
        assert np.array_equal(got, ref["state"].astype(got.dtype))
        for i, a in enumerate(ref["sink_d"]):
            assert np.array_equal(sink[i * k:(i + 1) * k], a)
        for key in ("touched", "bind", "lam", "fall"):
            assert st[key] == ref["counters"][key], (key, st, ref["counters"])
    else:
        for f, (x, r) in enumerate(zip(field_views(w, got, "state"),
                                       field_views(w, ref["state"].astype(got.dtype), "state"))):
            assert rel_err(x, r) <= max(TOL[acc], float(np.finfo(got.dtype).eps)), f
        for i, a in enumerate(ref["sink_d"]):
            assert rel_err(sink[i * k:(i + 1) * k], a) <= max(TOL[acc], 1e-9), i


def test_graph_owner_tiles(B):
    """A captured multi-box graph of fold-free steps replays like eager steps."""
    import torch
    w = W.c5(nb=3, n_total=30000)
    tun = {"deposit_path": 1, "fuse_apply": 2, "tile_x": 16, "tile_yz": 4}
    assert owner_tiles_fit(w, 16, 4)
    eager = B.Context(w, "fix64")
    eager.set_tuning(**tun)
    eager.step()
    eager.step()
    torch.cuda.synchronize()
    ref = eager.state.cpu().numpy()
    eager.close()
    g = B.Context(w, "fix64")
    g.set_tuning(**tun)
    g.graph_build(2)
    for _ in range(3):
        g.reset_state()
        torch.cuda.synchronize()
        g.graph_launch()
        torch.cuda.synchronize()
        assert np.array_equal(g.state.cpu().numpy(), ref)
    g.close()


@pytest.mark.parametrize("fuse", [2, 1, 0])
@pytest.mark.parametrize("eint_mode", [0, 1])
@pytest.mark.parametrize("acc", ["fix64", "f32"])
def test_step_energy_floor(B, orc, acc, eint_mode, fuse):
    """Cold gas: about a third of the cells hold less total energy than their
    kinetic part, so the energy limiter takes the floor branch (lam = 0);
    both e_int modes, with the apply fused into the tile pass or separate,
    and the deposited channels only (the source-free apply) or all."""
    rng = np.random.default_rng(21)
    w = W.c2(nx=24)
    st = w.state.reshape(5, -1).copy()
    r64 = st[0].astype(np.float64)
    ke = 0.5 * (st[1:4].astype(np.float64) ** 2).sum(axis=0) / r64
    cold = rng.random(st.shape[1]) < 0.35
    st[4, cold] = (0.3 * ke[cold]).astype(st.dtype)
    w = dataclasses.replace(w, state=st.reshape(-1), name="cold",
                            limits=dataclasses.replace(w.limits, eint_mode=eint_mode))
    for channels in ("auto", "all"):
        say(f"energy floor acc={acc} eint_mode={eint_mode} fuse={fuse} channels={channels}")
        tun = {"deposit_path": 1, "fuse_apply": fuse}
        if fuse == 2:
            tun["tile_x"] = 16  # owner tiles: at most domain - 2g cells wide
            assert owner_tiles_fit(w, 16, 4)
        out = step_vs_oracle(B, orc, w, acc, channels=channels, tuning=tun)
        assert ("fold" in out["phases"]) == (fuse != 2), out["phases"]
        assert out["oracle_counters"]["fall"] > 1000, out
        if acc == "f32":
            # decided in FP64 from FP32 deposits, cells at the limiter's edge may
            # go either way (the state is continuous there and checked above)
            ref = out["oracle_counters"]["fall"]
            assert abs(out["status"]["fall"] - ref) <= 0.05 * ref, out


@pytest.mark.parametrize("acc", ["fix64", "f32"])
def test_ghost_width_zero(B, orc, acc):
    """g = 0: supernovae of radius below 1/2 (one cell each), every owned cell
    interior; separate calls and the (fused and unfused) step."""
    rng = np.random.default_rng(11)
    dom = (70, 9, 6)
    w = W.Workload("g0", *W.single_box(*dom), 0, 1.0,
                   W.gas_state(rng, int(np.prod(dom)), np.float32).reshape(-1),
                   sn=W._one_box(W.uniform_positions(rng, 300, dom), W.sn_fields(300, 0.4)))
    for path in (1, 0):
        check(B, orc, w, acc, tuning={"deposit_path": path})
    for fuse in (1, 0):
        step_vs_oracle(B, orc, w, acc, tuning={"deposit_path": 1, "fuse_apply": fuse})


@pytest.mark.parametrize("fuse", [1, 0])
@pytest.mark.parametrize("name", list(SMALL))
def test_step_fused_split_tiles(B, orc, name, fuse):
    """Fused step with split tiles and small tiles."""
    w = SMALL[name]()
    for tun in ({"chunk_cic": 64, "chunk_sn": 16}, {"tile_x": 16, "tile_yz": 2}):
        say(f"step {w.name} fuse={fuse} {tun}")
        step_vs_oracle(B, orc, w, "fix64", tuning={"deposit_path": 1, "fuse_apply": fuse, **tun})


@pytest.mark.parametrize("channels", ["auto", "all"])
@pytest.mark.parametrize("name", ["c2_40", "c3_40", "c4_48", "c5_4"])
def test_step_matches_oracle(B, orc, name, channels):
    """pmp_step (all buffer channels, or only the deposited ones) against the
    oracle's step."""
    import torch
    w = SMALL[name]()
    say(f"step {w.name} channels={channels}")
    for acc in ("fix64", "f32"):
        ctx = B.Context(w, acc, channels=channels)
        ctx.step()
        torch.cuda.synchronize()
        got = ctx.state.cpu().numpy()
        st = ctx.status()
        ctx.close()
        assert st["flags"] in (0, 0x10), st
        ref = orc.step(w, "fix64" if acc == "fix64" else "f64")["state"].astype(got.dtype)
        if acc == "fix64":
            assert np.array_equal(got, ref)
        else:
            for f, (x, r) in enumerate(zip(field_views(w, got, "state"),
                                           field_views(w, ref, "state"))):
                assert rel_err(x, r) <= 1e-6, f


@pytest.mark.parametrize("path", [1, 0])
@pytest.mark.parametrize("acc", ["fix64", "f32"])
@pytest.mark.parametrize("name", list(SMALL))
def test_deposited_channels_only(B, orc, name, acc, path):
    """Layouts holding only the channels the particle kinds deposit into (the
    others are zero in the oracle's buffer and read as zero in the apply)."""
    check(B, orc, SMALL[name](), acc, tuning={"deposit_path": path}, channels="auto")


def test_channel_errors(B):
    w = W.c2(nx=16)
    # supernovae need rho and E
    ctx = B.Context(w, "f32", channels=B.PMP_CH_RHO)
    with pytest.raises(B.PmpError, match="EINVAL"):
        ctx.deposit()
    ctx.close()
    # momentum channels come together; unknown bits are refused
    for ch in (0x2, 0x40):
        with pytest.raises(B.PmpError, match="EINVAL"):
            B.Context(w, "f32", channels=ch | B.PMP_CH_RHO)
    # K is present exactly when the layout has sinks
    with pytest.raises(B.PmpError, match="EINVAL"):
        B.Context(w, "f32", channels=B.PMP_CH_RHO | B.PMP_CH_K)
    w3 = W.c3(nx=16, n_sink=4)
    with pytest.raises(B.PmpError, match="EINVAL"):
        B.Context(w3, "f32", channels=B.PMP_CH_RHO)


def test_per_box_launches_match_batched(B, orc):
    """The per-box launch baseline computes the same step (fixed point: same
    bits) as the batched launches and the oracle."""
    import torch
    w = W.c5(nb=3, n_total=30000)
    a = B.Context(w, "fix64")
    a.set_tuning(deposit_path=0)
    a.step_per_box()
    b = B.Context(w, "fix64")
    b.step()
    torch.cuda.synchronize()
    sa, sb = a.state.cpu().numpy(), b.state.cpu().numpy()
    a.close()
    b.close()
    ref = orc.step(w, "fix64")["state"].astype(np.float32)
    assert np.array_equal(sa, ref)
    assert np.array_equal(sb, ref)


def test_autotune_then_step(B, orc):
    """The tuner leaves the caller's state alone, picks a valid tuning, and
    the tuned step still matches the oracle bit for bit."""
    import torch
    from paper_2509_18261_amd import autotune
    w = W.c5(nb=3, n_total=30000)
    ctx = B.Context(w, "fix64")
    before = ctx.state.cpu().numpy().copy()
    res = autotune.tune(ctx, cache_path=None)
    torch.cuda.synchronize()
    assert res["best_ms"] > 0
    assert np.array_equal(ctx.state.cpu().numpy(), before)
    ctx.step()
    torch.cuda.synchronize()
    got = ctx.state.cpu().numpy()
    ctx.close()
    assert np.array_equal(got, orc.step(w, "fix64")["state"].astype(np.float32))


def test_graph_multibox(B):
    """A captured multi-box graph (binned path) replays like eager steps."""
    import torch
    w = W.c5(nb=3, n_total=30000)
    eager = B.Context(w, "fix64")
    eager.step()
    eager.step()
    torch.cuda.synchronize()
    ref = eager.state.cpu().numpy()
    eager.close()
    g = B.Context(w, "fix64")
    g.graph_build(2)
    for _ in range(3):
        g.reset_state()
        torch.cuda.synchronize()
        g.graph_launch()
        torch.cuda.synchronize()
        assert np.array_equal(g.state.cpu().numpy(), ref)
    g.close()


@pytest.mark.parametrize("name", ["c2", "c3"])
def test_workspace_caller_owned(B, name):
    """Scratch carved from a caller-owned workspace gives the results of the
    library's own scratch, bit for bit in fixed point, for the step and for a
    graph of it (CIC + supernovae fused; CIC + sinks); a workspace too small
    for the deposit is refused with PMP_ERANGE, and None returns to the
    library's own scratch."""
    import torch
    w = W.c2(nx=32) if name == "c2" else W.c3(nx=32, n_sink=16)
    say(f"workspace {name}")

    def run(ctx, graph=False):
        ctx.reset_state()
        if graph:
            ctx.graph_build(1)
            ctx.graph_launch()
        else:
            ctx.step()
        torch.cuda.synchronize()
        return ctx.state.cpu().numpy().copy(), ctx.status()

    ref = B.Context(w, "fix64", channels="auto")
    ref.set_tuning(deposit_path=1)
    want, st_ref = run(ref)
    ref.close()
    ctx = B.Context(w, "fix64", channels="auto")
    ctx.set_tuning(deposit_path=1)
    nbytes = ctx.workspace_size()
    assert nbytes >= 256 and nbytes % 256 == 0
    ws = torch.full((nbytes,), 0xAB, dtype=torch.uint8, device="cuda")
    ctx.set_workspace(ws)
    for graph in (False, True):
        got, st = run(ctx, graph)
        assert st["flags"] in (0, 0x10), st
        assert np.array_equal(got, want), graph
        for k in ("touched", "bind", "lam", "fall"):
            assert st[k] == st_ref[k], (k, st, st_ref)
    ctx.close()
    # too small: refused, nothing launched
    ctx = B.Context(w, "fix64", channels="auto")
    ctx.set_tuning(deposit_path=1)
    small = torch.empty(max(256, (nbytes // 2) // 256 * 256), dtype=torch.uint8, device="cuda")
    ctx.set_workspace(small)
    with pytest.raises(B.PmpError) as e:
        ctx.step()
    assert "workspace" in str(e.value)
    ctx.set_workspace(None)
    got, _ = run(ctx)
    assert np.array_equal(got, want)
    ctx.close()


# ------------------------------------- reproducibility mode (App. A.1, error bound)

def repro_bound(x, r, margin):
    """Elementwise, the most two truncations (App. A.1) of sums of the same
    contributions in different orders can differ by, relative to the larger
    magnitude: one truncation interval for up to 2^8 contributions."""
    return 2.0 ** -(52 - margin - 8)


@pytest.mark.parametrize("name", list(SMALL))
def test_reproducibility_mode_vs_oracle(B, orc, name):
    """PMP_ACC_F64R against the oracle's mode: the deposited and the folded
    buffers within one truncation interval of the oracle's in every element
    and bit-identical in most (the GPU sums in another order, and the bound,
    so the truncation width, follows the order from three contributions on);
    the applied state within 1e-6 of the oracle's per field."""
    w = SMALL[name]()
    margin = 28
    say(f"repro mode {w.name}")
    got = run_gpu(B, w, "f64r")
    assert got["status"]["flags"] in (0, 0x10), got["status"]
    ref = orc.step(w, "f64r", want_eta=True)
    for key in ("buf_deposit", "buf_fold"):
        x, r = got[key], ref[key]
        nz = (x != 0.0) | (r != 0.0)
        assert np.array_equal(x[~nz], r[~nz])
        if not nz.any():
            continue
        rel = np.abs(x[nz] - r[nz]) / np.maximum(np.abs(x[nz]), np.abs(r[nz]))
        assert rel.max() <= repro_bound(x, r, margin), (key, rel.max())
        same = float(np.mean(x[nz] == r[nz]))
        say(f"  {key}: {nz.sum()} elements, {same:.4f} identical")
        assert same >= 0.9, (key, same)
    for f, (x, r) in enumerate(zip(field_views(w, got["state"], "state"),
                                   field_views(w, ref["state"].astype(got["state"].dtype),
                                               "state"))):
        e = rel_err(x, r)
        assert e <= max(1e-6, float(np.finfo(got["state"].dtype).eps)), (f, e)
    if "sink_d" in ref:
        for a, b in zip(got["sink_d"], ref["sink_d"]):
            assert rel_err(a, b) <= 1e-6


def test_reproducibility_mode_fused_step_and_errors(B, orc):
    """The fused step in the reproducibility mode equals the separate calls'
    result within the state tolerance, and the mode refuses the direct path
    and the per-box launches."""
    import torch
    w = W.c2(nx=40)
    ctx = B.Context(w, "f64r", channels="auto")
    ctx.set_tuning(fuse_apply=1)
    ctx.step()
    torch.cuda.synchronize()
    st = ctx.state.cpu().numpy()
    ref = orc.step(w, "f64r")
    for f, (x, r) in enumerate(zip(field_views(w, st, "state"),
                                   field_views(w, ref["state"].astype(st.dtype), "state"))):
        assert rel_err(x, r) <= 1e-6, f
    with pytest.raises(B.PmpError):
        ctx.set_tuning(deposit_path=0)
    with pytest.raises(B.PmpError):
        ctx.step_per_box()
    ctx.close()


def test_truelove_per_cell_changes_the_limiter(B, orc):
    """The per-cell Truelove density raises removals in dense cells: the
    limiter's counters differ from the constant (disabled) density's, and the
    GPU step still matches the oracle bit for bit."""
    w = W.c3(nx=40, n_sink=48)
    base = orc.step(w, "fix64")["counters"]
    got, ref = check(B, orc, truelove(w), "fix64")
    assert ref["counters"]["touched"] > base["touched"] or ref["counters"]["bind"] != base["bind"]


# ------------------------------------------------- status flags and ties

def _add_particle(P, pos, **fields):
    """A single-box particle kind with one more particle appended."""
    f = {k: np.concatenate([v, [fields.get(k, v[0])]]) for k, v in P.fields.items()}
    for a, k in enumerate(("x", "y", "z")):
        f[k][-1] = pos[a]
    return W.Particles(f, np.array([0, P.n + 1], dtype=np.int64))


def _flags(got):
    return got["status"]["flags"]


@pytest.mark.parametrize("path", [1, 0])
def test_overflow_flag_skips_the_contribution(B, orc, path):
    """A fixed-point contribution beyond 2^62 on the 2^-40 grid (a CIC mass of
    1e7 at a cell centre: one contribution of 1e7 per unit volume) is skipped
    and raises OVERFLOW; everything else equals the oracle without it."""
    w = W.c2(nx=24)
    bad = dataclasses.replace(w, cic=_add_particle(w.cic, (12.5, 7.5, 3.5), m=1e7))
    say(f"case overflow path={path}")
    got = run_gpu(B, bad, "fix64", tuning={"deposit_path": path})
    assert _flags(got) & 0x4, got["status"]
    ref = orc.step(w, "fix64", want_eta=True)
    got["status"]["flags"] &= ~0x4
    compare(w, "fix64", got, ref)


@pytest.mark.parametrize("acc", ["fix64", "f32"])
@pytest.mark.parametrize("path", [1, 0])
def test_nan_particles_flagged_and_skipped(B, orc, path, acc):
    """A CIC particle with a NaN mass and a supernova with a NaN energy are
    skipped and raise NAN; the rest equals the oracle without them."""
    w = W.c2(nx=24)
    bad = dataclasses.replace(w, cic=_add_particle(w.cic, (3.2, 4.4, 5.6), m=float("nan")),
                              sn=_add_particle(w.sn, (10.1, 11.2, 12.3), e=float("nan")))
    say(f"case nan path={path} acc={acc}")
    got = run_gpu(B, bad, acc, tuning={"deposit_path": path})
    assert _flags(got) & 0x8, got["status"]
    ref = orc.step(w, "fix64" if acc == "fix64" else "f64", want_eta=True)
    got["status"]["flags"] &= ~0x8
    compare(w, acc, got, ref)


def test_capacity_flag_when_radius_bound_is_wrong(B):
    """The binned path sizes its supernova entry lists from pmp_sn.r_max; a
    caller that declares r_max = 0 for radius-4 supernovae overflows them:
    the entries past the capacity are skipped (never read) and CAPACITY is
    raised; the deposit completes and the deposited total falls short."""
    import torch
    w = W.c2(nx=24)
    tun = dict(deposit_path=1, tile_x=16, tile_yz=2, tile_block=64)
    sums = []
    for r_max in (4.0, 0.0):
        ctx = B.Context(w, "fix64", channels="all")
        ctx.set_tuning(**tun)
        ctx.sn.r_max = r_max
        say(f"case capacity r_max={r_max}")
        ctx.deposit()
        torch.cuda.synchronize()
        sums.append((ctx.buf.cpu().numpy().sum(), ctx.status()))
        ctx.close()
    assert sums[0][1]["flags"] == 0, sums[0][1]
    assert sums[1][1]["flags"] & 0x20, sums[1][1]
    assert sums[1][0] < sums[0][0]


@pytest.mark.parametrize("path", [1, 0])
def test_fixed_point_remainder_at_an_exact_tie(B, orc, path):
    """CIC particles on cell corners (f = 1/2 on every axis: eight equal
    weights) with masses whose eighths are not on the 2^-40 grid: the
    rounding residue goes to the host cell, as in the oracle, bit for bit."""
    rng = np.random.default_rng(4)
    pos = np.array([[5.0, 6.0, 7.0], [1.0, 1.0, 1.0], [16.0, 3.0, 9.0], [8.0, 8.0, 8.0]])
    m = np.array([0.3, 0.7, 1.0 / 3.0, 0.1])
    domain, lo, n = W.single_box(16)
    w = W.Workload("ties", domain, lo, n, 2, 1.0,
                   W.gas_state(rng, 16 ** 3, np.float64).reshape(-1),
                   cic=W._one_box(pos % 16, {"m": m}))
    say(f"case tie path={path}")
    check(B, orc, w, "fix64", tuning={"deposit_path": path})
