"""Map pruning (App. C.1, Algorithm 1 and its three criteria), in numpy.

TEST INFRASTRUCTURE ONLY: imported by the test suite, never by the product
path. Shares no code with the GPU implementation.

A Gaussian is removed when its opacity is below tau_o, or, when a scale
threshold is given, when its largest scale exceeds tau_s or exceeds tau_e
times the sum of its other two scales (the union of the three sets of
App. C.1). The survivors keep their order. Readings:
  - the comparisons are strict, as printed (opacity exactly tau_o stays);
  - "no scale threshold" is tau_s <= 0: only opacity pruning runs;
  - the criteria are integer decisions taken in binary32 on both sides, in
    one fixed order: the largest scale is found by scanning s0, s1, s2 and
    replacing on a strictly larger value (the first of equal maxima wins),
    the "other two" are the remaining two added in index order (one binary32
    addition, equal to sum(s) - max(s) up to that rounding), and tau_e times
    that sum is one binary32 product;
  - opacity and scales are the activated values the renderer takes.
"""
import numpy as np

F32 = np.float32


def prune_mask(opacity, scales, tau_o=0.005, tau_s=0.25, tau_e=10.0) -> np.ndarray:
    """Boolean [n]: True where the Gaussian is removed."""
    o = np.asarray(opacity, dtype=F32)
    s = np.asarray(scales, dtype=F32)
    m = o < F32(tau_o)
    if tau_s > 0:
        s0, s1, s2 = s[0], s[1], s[2]
        idx = np.zeros(o.shape, np.int64)
        idx = np.where(s1 > s0, 1, idx)
        big = np.where(idx == 1, s1, s0)
        idx = np.where(s2 > big, 2, idx)
        big = np.where(idx == 2, s2, big)
        other = np.where(idx == 0, (s1 + s2).astype(F32), np.where(idx == 1, (s0 + s2).astype(F32), (s0 + s1).astype(F32)))
        m = m | (big > F32(tau_s)) | (big > (F32(tau_e) * other).astype(F32))
    return m


def prune(m: dict, tau_o=0.005, tau_s=0.25, tau_e=10.0):
    """(kept map with the survivors in their original order, removal mask)."""
    mask = prune_mask(m["opacity"], m["scales"], tau_o, tau_s, tau_e)
    keep = ~mask
    out = {}
    for k, v in m.items():
        v = np.asarray(v)
        out[k] = v[..., keep]
    return out, mask
