"""Per-block comparison of iterates in the paper's layout x = [y_1..y_N | u | p_1..p_N].

The blocks differ in scale by orders of magnitude (with nu = 1e-4 the adjoint
block is ~1e-4 of the whole vector), so one relative error over the whole
vector would pin the small blocks only loosely; every block is compared on its
own scale instead."""
import numpy as np


def blocks(v, n, N):
    nn = n * n
    v = np.asarray(v)
    return {"y": v[:N * nn], "u": v[N * nn:(N + 1) * nn], "p": v[(N + 1) * nn:]}


def block_rel(a, b, n, N):
    """Relative error of a against b in each of the Y, U and P blocks; a block
    that is zero in b is measured against the whole of b."""
    whole = max(np.linalg.norm(b), 1e-300)
    ba, bb = blocks(a, n, N), blocks(b, n, N)
    out = {}
    for k in ("y", "u", "p"):
        nb = np.linalg.norm(bb[k])
        out[k] = np.linalg.norm(ba[k] - bb[k]) / (nb if nb > 0 else whole)
    return out


def assert_blocks(a, b, n, N, tol, what=""):
    e = block_rel(a, b, n, N)
    assert max(e.values()) <= tol, (what, e)
    return e
