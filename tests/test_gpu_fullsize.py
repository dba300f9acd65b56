"""Parity at the full workload sizes, in the launch configuration the
benchmark times (buffer holding only the deposited channels): every cell
compared with the serial oracle (exact in int64 fixed
point; FP32 within 1e-6 per field, max|x - r| / max|r|)."""
import sys

import numpy as np
import pytest

from paper_2509_18261_amd import workloads as W

from buffers import expand_channels

pytestmark = pytest.mark.gpu


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


def run(B, w, acc, tuning=None, channels="auto"):
    import torch
    ctx = B.Context(w, acc, channels=channels)
    if tuning:
        ctx.set_tuning(**tuning)
    ctx.deposit()
    ctx.ghost_fold()
    torch.cuda.synchronize()
    fold = expand_channels(w, ctx.buf.cpu().numpy(), ctx.fields)
    ctx.sink_update()
    ctx.apply()
    torch.cuda.synchronize()
    out = {"buf_fold": fold, "state": ctx.state.cpu().numpy(), "status": ctx.status()}
    if ctx.sink_out is not None:
        out["sink"] = ctx.sink_out.cpu().numpy()
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    return out


def per_field_rel(w, x, r, nf, g):
    sizes = [int(np.prod(n + 2 * g)) for n in w.n.astype(np.int64)]
    worst = 0.0
    for f in range(nf):
        parts_x, parts_r = [], []
        off = 0
        for sz in sizes:
            parts_x.append(x[off + f * sz: off + (f + 1) * sz])
            parts_r.append(r[off + f * sz: off + (f + 1) * sz])
            off += nf * sz
        xx = np.concatenate(parts_x).astype(np.float64)
        rr = np.concatenate(parts_r).astype(np.float64)
        den = np.max(np.abs(rr))
        if den > 0:
            worst = max(worst, float(np.max(np.abs(xx - rr)) / den))
    return worst


CASES = {"c2": W.c2, "c3": W.c3, "c3bh": W.c3bh, "c5": W.c5}


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name", list(CASES))
def test_full_size_fixed_point_exact(B, orc, name):
    w = CASES[name]()
    say(f"full-size {w.name}: fixed point, both deposit paths")
    ref = orc.step(w, "fix64")
    for path in (1, 0):
        got = run(B, w, "fix64", {"deposit_path": path})
        assert got["status"]["flags"] in (0, 0x10), got["status"]
        assert np.array_equal(got["buf_fold"], ref["buf_fold"]), f"path {path}: folded buffer"
        st = ref["state"].astype(got["state"].dtype)
        assert np.array_equal(got["state"], st), f"path {path}: state"
        if "sink" in got:
            n = w.sinks.n
            for i, a in enumerate(ref["sink_d"]):
                assert np.array_equal(got["sink"][i * n:(i + 1) * n], a)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name", list(CASES))
def test_full_size_fp32_tolerance(B, orc, name):
    w = CASES[name]()
    say(f"full-size {w.name}: FP32 against the FP64 oracle")
    ref = orc.step(w, "f64")
    got = run(B, w, "f32", {"deposit_path": 1})
    e_buf = per_field_rel(w, got["buf_fold"], ref["buf_fold"], w.nfield, w.ghost)
    e_st = per_field_rel(w, got["state"], ref["state"].astype(np.float32), 5, 0)
    say(f"  folded buffer {e_buf:.3e}  state {e_st:.3e}")
    assert e_buf <= 1e-6
    assert e_st <= max(1e-6, float(np.finfo(np.float32).eps))


@pytest.mark.timeout(900)
def test_full_size_c4_fixed_point(B, orc):
    """512^3 mixed workload: final state and folded buffer bit-exact."""
    w = W.c4()
    say(f"full-size {w.name}: fixed point")
    got = run(B, w, "fix64")
    ref = orc.step(w, "fix64")
    assert got["status"]["flags"] in (0, 0x10), got["status"]
    assert np.array_equal(got["buf_fold"], ref["buf_fold"])
    assert np.array_equal(got["state"], ref["state"].astype(np.float32))


@pytest.mark.timeout(900)
@pytest.mark.parametrize("acc", ["f32", "f64"])
def test_full_size_c4_float_modes(B, orc, acc):
    """512^3 mixed workload in FP32 (FP32 state) and FP64 (state promoted to
    FP64) against the FP64 oracle: per-field max and RMS relative error of
    the folded buffer and of the state, and the drift of the total mass and
    energy (sum over owned cells) from the oracle's."""
    w = W.c4()
    if acc == "f64":
        w = w.with_state(w.state.astype(np.float64))
    say(f"full-size {w.name}: {acc} against the FP64 oracle")
    got = run(B, w, acc)
    assert got["status"]["flags"] in (0, 0x10), got["status"]
    ref = orc.step(w, "f64")
    sdt = got["state"].dtype
    e_buf = per_field_rel(w, got["buf_fold"], ref["buf_fold"], w.nfield, w.ghost)
    e_st = per_field_rel(w, got["state"], ref["state"].astype(sdt), 5, 0)
    x = got["state"].astype(np.float64).reshape(5, -1)
    r = ref["state"].astype(sdt).astype(np.float64).reshape(5, -1)
    rms = [float(np.linalg.norm(x[f] - r[f]) / np.linalg.norm(r[f])) for f in range(5)]
    drift = [abs(float(x[f].sum() - r[f].sum())) / abs(float(r[f].sum())) for f in (0, 4)]
    say(f"  max rel: folded buffer {e_buf:.3e}, state {e_st:.3e}; state RMS rel "
        f"{max(rms):.3e}; mass / energy drift {drift[0]:.3e} / {drift[1]:.3e}")
    tol = 1e-6 if acc == "f32" else 1e-12
    assert e_buf <= tol
    assert e_st <= max(tol, float(np.finfo(sdt).eps))
    assert max(rms) <= max(tol, float(np.finfo(sdt).eps))
    assert max(drift) <= max(tol, 1e-9 if acc == "f32" else 1e-14)


@pytest.mark.timeout(600)
def test_full_size_sink_create_after_step(B, orc):
    """256^3 with 256 sinks: a fixed-point step, then sink creation (r_K = 4,
    rho_Tr = e^3) on each side's own result, compared bit for bit."""
    import torch
    w = W.c3()
    say(f"full-size {w.name}: sink creation after a fixed-point step")
    ref = orc.step(w, "fix64")
    rho_tr, max_new = float(np.exp(3.0)), 65536
    s64 = ref["state"].astype(np.float32).astype(np.float64)
    n_ref, out_ref = orc.sink_create(w, "fix64", s64, ref["buf_fold"], w.r_k, rho_tr, max_new)
    assert 100 < n_ref < max_new
    ctx = B.Context(w, "fix64", channels="all")
    ctx.deposit()
    ctx.ghost_fold()
    ctx.sink_update()
    ctx.apply()
    out, work = ctx.sink_create(w.r_k, rho_tr, max_new)
    torch.cuda.synchronize()
    n = int(work[0].item())
    got = out.cpu().numpy().reshape(7, -1)
    st = ctx.state.cpu().numpy()
    ctx.close()
    say(f"  {n} new sinks")
    assert n == n_ref
    assert np.array_equal(got[:, :n], out_ref[:, :n])
    assert np.array_equal(st, s64.astype(np.float32))


def step_state(B, w, acc, tuning):
    import torch
    ctx = B.Context(w, acc)
    ctx.set_tuning(**tuning)
    ctx.profile_begin(4)
    ctx.step()
    torch.cuda.synchronize()
    phases = ctx.profile_end()
    out = {"state": ctx.state.cpu().numpy(), "status": ctx.status(), "phases": phases}
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    return out


OWNER_FULL = {
    # the benchmark's default workload and tile shape, FP64 state
    "c4": (lambda: (lambda w: w.with_state(w.state.astype(np.float64)))(W.c4()),
           {"tile_x": 64, "tile_yz": 4, "tile_block": 256}, ("fix64", "f64")),
    "c5": (W.c5, {"tile_x": 32, "tile_yz": 4, "tile_block": 128}, ("fix64", "f32")),
    # with 1024 sinks across the boxes: flagged tiles applied after the sink update
    "c5s": (W.c5s, {"tile_x": 32, "tile_yz": 4, "tile_block": 128}, ("fix64",)),
}


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name", list(OWNER_FULL))
def test_full_size_owner_tiles_step(B, orc, name):
    """The fold-free step (owner tiles, fuse_apply 2) at full size against the
    oracle's step: fixed point bit for bit with the limiter counters, floats
    per field within their tolerance; no fold launch."""
    make, shape, accs = OWNER_FULL[name]
    w = make()
    tun = {"deposit_path": 1, "fuse_apply": 2, "chunk_cic": 16384, "chunk_sn": 2048, **shape}
    for acc in accs:
        say(f"full-size {w.name}: owner tiles, {acc}, {shape}")
        got = step_state(B, w, acc, tun)
        assert got["status"]["flags"] in (0, 0x10), got["status"]
        assert "fold" not in got["phases"], got["phases"]
        ref = orc.step(w, "fix64" if acc == "fix64" else "f64")
        sdt = got["state"].dtype
        if acc == "fix64":
            assert np.array_equal(got["state"], ref["state"].astype(sdt))
            for k in ("touched", "bind", "lam", "fall"):
                assert got["status"][k] == ref["counters"][k], (k, got["status"])
        else:
            e = per_field_rel(w, got["state"], ref["state"].astype(sdt), 5, 0)
            say(f"  state max rel {e:.3e}")
            assert e <= max(1e-6 if acc == "f32" else 1e-12, float(np.finfo(sdt).eps))
