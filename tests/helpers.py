"""Small helpers shared by the test modules (no method arithmetic here)."""
import numpy as np


def interior_index(shape):
    """Boolean mask of interior nodes for a node array of the given shape."""
    m = np.ones(shape, dtype=bool)
    for ax in range(len(shape)):
        sl = [slice(None)] * len(shape)
        sl[ax] = 0
        m[tuple(sl)] = False
        sl[ax] = -1
        m[tuple(sl)] = False
    return m


def dense_operator(H, lv=0):
    """Dense interior matrix of the oracle's operator, assembled column by column
    from unit vectors (interior unknowns in row-major node order)."""
    shape = H.shape(lv)
    mask = interior_index(shape)
    idx = np.flatnonzero(mask.ravel())
    n = idx.size
    A = np.zeros((n, n))
    for k, p in enumerate(idx):
        e = np.zeros(int(np.prod(shape)))
        e[p] = 1.0
        A[:, k] = H.apply(e.reshape(shape), lv).ravel()[idx]
    return A, mask


def rel_inf(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def rel_inf_scaled(a, b, *inputs):
    """max |a - b| relative to the largest magnitude among b and the inputs the
    computation started from: rounding errors scale with the largest values
    that enter the arithmetic, which for a cycle that cancels most of a large
    random start are the start's, not the (much smaller) result's."""
    a = np.asarray(a)
    b = np.asarray(b)
    scale = max([np.max(np.abs(b))] + [np.max(np.abs(np.asarray(x))) for x in inputs])
    return float(np.max(np.abs(a - b)) / max(scale, 1e-300))
