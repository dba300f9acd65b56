"""pmp_sink_create_noalloc (the sink-creation entry point that allocates
nothing: its scratch is a static device array of the library) against
pmp_sink_create with a caller-owned work array, through the C-ABI, on two
calls in a row, the second with a smaller input that leaves the first
call's contents in the shared array."""
import dataclasses
import sys

import numpy as np
import pytest

from paper_2509_18261_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_18261_amd import binding
    return binding


def _run(B, w, acc, buf_np, r_k, max_new, limits, existing, noalloc):
    import torch
    ctx = B.Context(w, acc, channels="all")
    if buf_np is not None:
        ctx.buf.copy_(torch.from_numpy(np.ascontiguousarray(buf_np)))
    if noalloc:
        out, cnt = ctx.sink_create_noalloc(r_k, float("nan"), max_new, buf=buf_np is not None,
                                           limits=limits, existing=existing)
        n = cnt
    else:
        out, work = ctx.sink_create(r_k, float("nan"), max_new, buf=buf_np is not None,
                                    limits=limits, existing=existing)
        n = work[0:1]
    torch.cuda.synchronize()
    res = (int(n.item()), out.cpu().numpy().reshape(7, -1)[:, :max_new], ctx.state.cpu().numpy())
    ctx.close()
    return res


def _case(orc, nx, n_sink, G):
    w = W.c3(nx=nx, n_cic=0, n_sink=n_sink)
    w = W.Workload(w.name, w.domain, w.lo, w.n, w.ghost, w.dx, w.state, sinks=w.sinks,
                   r_k=w.r_k, r_gauss=w.r_gauss)
    buf, _, _ = orc.deposit(w, "fix64")
    orc.fold(w, "fix64", buf)
    lim = dataclasses.replace(w.limits, truelove_J=0.25, G=G)
    return w, buf, lim


def test_noalloc_matches_caller_scratch_twice(B, orc):
    calls = [(_case(orc, 40, 48, 0.05), 2.0, 4096), (_case(orc, 24, 8, 0.04), 1.5, 1024)]
    counts = []
    for (w, buf, lim), r_k, max_new in calls:
        print(f"case noalloc nx={w.domain[0]} max_new={max_new}", flush=True)
        sys.stdout.flush()
        ref = _run(B, w, "fix64", buf, r_k, max_new, lim, "workload", noalloc=False)
        got = _run(B, w, "fix64", buf, r_k, max_new, lim, "workload", noalloc=True)
        assert got[0] == ref[0]
        assert np.array_equal(got[1], ref[1])
        assert np.array_equal(got[2], ref[2])
        # and both are the oracle's
        s64 = w.state.astype(np.float64).copy()
        n_o, out_o = orc.sink_create(w, "fix64", s64, buf, r_k, float("nan"), max_new,
                                     limits=lim, existing=w.sinks)
        assert n_o == got[0] and np.array_equal(out_o[:, :n_o], got[1][:, :n_o])
        assert np.array_equal(s64.astype(np.float32), got[2])
        counts.append(got[0])
    assert counts[0] > counts[1] > 0


def test_noalloc_errors(B):
    w = W.c3(nx=24, n_cic=0, n_sink=8)
    ctx = B.Context(w, "f64")
    with pytest.raises(B.PmpError, match="EINVAL"):
        ctx.sink_create_noalloc(1.5, 2.0, 65537)
    ctx.close()
