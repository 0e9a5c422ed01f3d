"""Euclidean projection onto X = {lo <= v <= hi, 1^T v <= vmax} (oracle, FP64).

Sec. 4.2 (Efficient Implementation), Eq. piecewiseLinearEQ.  The projection
of y is the minimiser of |v - y|^2 over X.  If clamping y to the box already
satisfies the sum constraint the clamp is the projection.  Otherwise the
KKT conditions give v = clamp(y - lambda, lo, hi) with lambda > 0 solving
    phi(lambda) = vmax,   phi(t) = sum_e clamp(y_e - t, lo, hi),
a continuous, non-increasing function that is linear between consecutive
breakpoints of {y_e - lo} and {y_e - hi}.  The paper's Alg. 4 finds the
crossing by sorting those breakpoints and sweeping; here the crossing piece
is located by a binary search over the sorted breakpoints with phi
evaluated directly from its definition at each probe, and lambda is the
linear interpolation on that piece.  The paper writes the upper bound as 1;
it is a parameter `hi` here.
"""
from __future__ import annotations

import numpy as np


def box_clamp(y, lo, hi):
    return np.clip(np.asarray(y, dtype=np.float64), lo, hi)


def volume_sum(y, t, lo, hi):
    """phi(t) = sum_e clamp(y_e - t, lo, hi), summed directly."""
    return float(box_clamp(y - t, lo, hi).sum())


def project_volume_ref(y, lo, hi, vmax, return_lambda=False):
    """The projection onto X from Eq. piecewiseLinearEQ.  Where phi is flat
    at vmax every point of the flat piece is a root; the smallest is
    returned (x is the same for all of them)."""
    y = np.asarray(y, dtype=np.float64)
    E = y.size
    if vmax < E * lo:
        raise ValueError("infeasible: vmax < E * lo")
    x = box_clamp(y, lo, hi)
    if x.sum() <= vmax:
        return (x, 0.0) if return_lambda else x
    # phi(t) = E hi at the smallest breakpoint, E lo <= vmax at the largest
    t = np.unique(np.concatenate([y - lo, y - hi]))
    a, b = 0, t.size - 1            # phi(t[a]) > vmax >= phi(t[b])
    if volume_sum(y, t[b], lo, hi) > vmax:   # only when vmax < E lo, excluded above
        raise ValueError("no root of the volume equation")
    while b - a > 1:
        m = (a + b) // 2
        if volume_sum(y, t[m], lo, hi) > vmax:
            a = m
        else:
            b = m
    fa, fb = volume_sum(y, t[a], lo, hi), volume_sum(y, t[b], lo, hi)
    if fb == vmax:
        lam = float(t[b])
    else:                           # phi is linear on [t[a], t[b]]
        lam = float(t[a] + (fa - vmax) * (t[b] - t[a]) / (fa - fb))
    x = box_clamp(y - lam, lo, hi)
    return (x, lam) if return_lambda else x


def project_bisect(y, lo, hi, vmax, iters=200, return_lambda=False):
    """Same projection by FP64 bisection on lambda (cross-check)."""
    y = np.asarray(y, dtype=np.float64)
    x = box_clamp(y, lo, hi)
    if x.sum() <= vmax:
        return (x, 0.0) if return_lambda else x
    a, b = 0.0, float(y.max() - lo)
    for _ in range(iters):
        m = 0.5 * (a + b)
        if m == a or m == b:
            break
        if box_clamp(y - m, lo, hi).sum() > vmax:
            a = m
        else:
            b = m
    lam = 0.5 * (a + b)
    x = box_clamp(y - lam, lo, hi)
    return (x, lam) if return_lambda else x
