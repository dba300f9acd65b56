"""Buffer layout helpers shared by the GPU tests (host-side reshaping only)."""
import numpy as np


def expand_channels(w, flat, fields):
    """A buffer holding only the channels ``fields`` (oracle field indices, in
    buffer order), re-laid out with every field of the oracle's buffer; the
    absent channels are zero."""
    if list(fields) == list(range(w.nfield)):
        return flat
    g = w.ghost
    sizes = [int(np.prod(n + 2 * g)) for n in w.n.astype(np.int64)]
    out = np.zeros(sum(sizes) * w.nfield, dtype=flat.dtype)
    src = dst = 0
    for sz in sizes:
        for k, f in enumerate(fields):
            out[dst + f * sz: dst + (f + 1) * sz] = flat[src + k * sz: src + (k + 1) * sz]
        src += len(fields) * sz
        dst += w.nfield * sz
    assert src == flat.size
    return out
