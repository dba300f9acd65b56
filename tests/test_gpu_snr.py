"""Supernova remnants with the TIGRESS-variant deposit (Sec. 3.2.1, eqs.
"du", "dp", "psnr") on the GPU against the serial oracle, through the C-ABI
(pmp_deposit_snr after pmp_deposit, then the fold and the apply).  Fixed
point: the deposited and folded buffers, the per-remnant scalars and the
applied state bit for bit; FP64 within 1e-12 and FP32 within 1e-6 of each
field's largest magnitude."""
import dataclasses
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


def run_gpu(B, w, acc, tuning=None):
    import torch
    ctx = B.Context(w, acc, channels="all")
    if tuning:
        ctx.set_tuning(**tuning)
    n = w.snr.n if w.snr is not None else 0
    info = torch.zeros(4 * max(n, 1), dtype=torch.float64, device="cuda")
    ctx.deposit()
    ctx.deposit_snr(info)
    dep = expand_channels(w, ctx.buf.cpu().numpy().copy(), ctx.fields)
    ctx.ghost_fold()
    fold = expand_channels(w, ctx.buf.cpu().numpy().copy(), ctx.fields)
    ctx.sink_update()
    ctx.apply()
    torch.cuda.synchronize()
    out = {"buf_deposit": dep, "buf_fold": fold, "state": ctx.state.cpu().numpy(),
           "info": info.cpu().numpy()[:4 * n].reshape(4, n), "status": ctx.status()}
    if ctx.sink_out is not None:
        k = w.sinks.n
        s = ctx.sink_out.cpu().numpy()
        out["sink_d"] = (s[:k], s[k:2 * k], s[2 * k:3 * k], s[3 * k:])
    ctx.close()
    return out


def fields(w, flat, kind):
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


def rel(x, r):
    x = x.astype(np.float64)
    r = r.astype(np.float64)
    den = np.max(np.abs(r)) if r.size else 0.0
    num = np.max(np.abs(x - r)) if r.size else 0.0
    return num if den == 0.0 else num / den


def check(B, orc, w, acc, tuning=None):
    say(f"case {w.name} acc={acc} nbox={w.nbox} snr={w.snr.n if w.snr else 0} "
        f"sub={w.snr_params.sub} r_k={w.snr_params.r_k} state={w.state.dtype}")
    got = run_gpu(B, w, acc, tuning)
    assert got["status"]["flags"] in (0, 0x10), got["status"]
    ref = orc.step(w, "fix64" if acc == "fix64" else "f64", want_eta=True)
    if acc == "fix64":
        assert np.array_equal(got["info"], ref["snr_info"]), "remnant scalars differ"
        assert np.array_equal(got["buf_deposit"], ref["buf_deposit"]), "deposit buffer differs"
        assert np.array_equal(got["buf_fold"], ref["buf_fold"]), "folded buffer differs"
        st = ref["state"].astype(got["state"].dtype)
        bad = np.flatnonzero(got["state"] != st)
        assert bad.size == 0, f"{bad.size} state values differ, first at {bad[:5]}"
        for k in ("touched", "bind", "lam", "fall"):
            assert got["status"][k] == ref["counters"][k], (k, got["status"], ref["counters"])
        if "sink_d" in ref:
            for a, b in zip(got["sink_d"], ref["sink_d"]):
                assert np.array_equal(a, b)
        return got, ref
    tol = TOL[acc]
    # the per-remnant scalars come from exact sums, so they agree to rounding
    assert np.allclose(got["info"], ref["snr_info"], rtol=1e-14, atol=0.0)
    for key in ("buf_deposit", "buf_fold"):
        for f, (x, r) in enumerate(zip(fields(w, got[key], "buf"), fields(w, ref[key], "buf"))):
            e = rel(x, r)
            assert e <= tol, f"{key} field {f}: {e:.3e} > {tol}"
    sdt = got["state"].dtype
    stol = max(tol, float(np.finfo(sdt).eps))
    for f, (x, r) in enumerate(zip(fields(w, got["state"], "state"),
                                   fields(w, ref["state"].astype(sdt), "state"))):
        e = rel(x, r)
        assert e <= stol, f"state field {f}: {e:.3e} > {stol}"
    return got, ref


CASES = {
    "slabs_sub4": lambda dt: W.snr_box(dtype=dt),
    "slabs_sub1": lambda dt: W.snr_box(dtype=dt, sub=1, seed=8),
    "slabs_sub16": lambda dt: W.snr_box(dtype=dt, sub=16, n_snr=6, seed=9),
    "multibox_sub4": lambda dt: W.snr_box(dtype=dt, nb=3, n_snr=40, seed=10),
    "dense_overlap": lambda dt: W.snr_box(dtype=dt, nx=24, n_snr=60, seed=12),
}


@pytest.mark.parametrize("dt", [np.float64, np.float32])
@pytest.mark.parametrize("acc", ["fix64", "f64", "f32"])
@pytest.mark.parametrize("name", list(CASES))
def test_snr_vs_oracle(B, orc, name, acc, dt):
    w = CASES[name](dt)
    got, ref = check(B, orc, w, acc)
    if name.startswith("slabs") and acc == "fix64":
        rm = ref["snr_info"][1] / (1679.0 * ref["snr_info"][2] ** -0.26)
        assert (rm > 1).any() and (rm <= 0.027).any()
        assert ref["counters"]["lam"] > 0


def edge_workloads():
    out = []
    w = W.snr_box(nx=16, n_snr=4, seed=3)
    pts = np.array([[0.0, 0.0, 0.0], [15.999, 15.999, 0.5], [8.0, 8.0, 8.0], [3.3, 12.7, 15.2]])
    f = {k: v for k, v in w.snr.fields.items() if k not in ("x", "y", "z")}
    # on the domain's corner and faces (periodic kernels)
    out.append(dataclasses.replace(w, name="corners", snr=W._one_box(pts, f)))
    # a kernel so small that no sample point lies within it: the host cell alone
    out.append(dataclasses.replace(w, name="tiny_kernel", snr=W._one_box(pts, f),
                                   snr_params=W.SnrParams(r_k=0.05, sub=2)))
    # radius 0 with one sample per cell: the cell whose centre is the remnant
    ctr = np.array([[4.5, 4.5, 4.5], [10.5, 3.5, 7.5], [1.2, 1.7, 1.9], [12.5, 12.5, 12.5]])
    out.append(dataclasses.replace(w, name="zero_radius", snr=W._one_box(ctr, f),
                                   snr_params=W.SnrParams(r_k=0.0, sub=1)))
    # remnants on box faces, edges and corners of a multi-box tiling
    mb = W.snr_box(nx=24, n_snr=4, nb=2, seed=4)
    fm = {k: v for k, v in mb.snr.fields.items() if k not in ("x", "y", "z")}
    cuts = np.unique(mb.lo[:, 0])
    e = float(cuts[1])
    pts = np.array([[e, e, e], [e - 0.001, 3.0, 20.0], [0.2, e, 23.9], [e, 0.0, 11.5]])
    cx = [np.concatenate([np.unique(mb.lo[:, a]), [mb.domain[a]]]) for a in range(3)]
    out.append(dataclasses.replace(mb, name="box_faces",
                                   snr=W._group_by_box(pts, fm, cx, (2, 2, 2))))
    # together with CIC, uniform supernovae and sinks in one step
    c3 = W.c3(nx=24, n_sink=12, dtype=np.float64)
    full = W.snr_box(nx=24, n_snr=10, seed=5)
    out.append(dataclasses.replace(full, name="all_kinds", cic=c3.cic, sinks=c3.sinks,
                                   r_k=2.0, r_gauss=1.0,
                                   sn=W._one_box(W.uniform_positions(np.random.default_rng(1), 8,
                                                                     full.domain),
                                                 W.sn_fields(8, 2.0))))
    return out


@pytest.mark.parametrize("path", [1, 0])
@pytest.mark.parametrize("acc", ["fix64", "f64", "f32"])
@pytest.mark.parametrize("idx", range(5))
def test_snr_edge_cases(B, orc, idx, acc, path):
    w = edge_workloads()[idx]
    check(B, orc, w, acc, tuning={"deposit_path": path})


def test_snr_errors(B):
    import torch
    w = W.snr_box(nx=16, n_snr=3)
    ctx = B.Context(w, "f64r", channels="all")
    ctx.deposit()
    with pytest.raises(B.PmpError, match="EUNSUPPORTED"):
        ctx.deposit_snr()
    ctx.close()
    # the rho, momentum and E channels are needed
    ctx = B.Context(dataclasses.replace(w, snr=None), "f64", channels=B.PMP_CH_RHO | B.PMP_CH_E)
    ctx.snr = B.Context(w, "f64").snr
    with pytest.raises(B.PmpError, match="EINVAL"):
        ctx.deposit_snr()
    ctx.close()
    for bad, code in ((dict(sub=3), "EINVAL"), (dict(r_k=-1.0), "EINVAL"),
                      (dict(nh_per_rho=0.0), "EINVAL"), (dict(r_k=4.5), "ERANGE")):
        ww = dataclasses.replace(w, snr_params=dataclasses.replace(w.snr_params, **bad))
        ctx = B.Context(ww, "f64")
        ctx.deposit()
        with pytest.raises(B.PmpError, match=code):
            ctx.deposit_snr()
        ctx.close()
    torch.cuda.synchronize()


def test_snr_full_size_fixed_point(B, orc):
    """A 128^3 slab box with 2000 remnants: fixed point bit-exact in the
    deposit, the fold and the state; FP32 within 1e-6."""
    w = W.snr_box(nx=128, n_snr=2000, seed=21, dtype=np.float32)
    check(B, orc, w, "fix64")
    check(B, orc, w, "f32")
