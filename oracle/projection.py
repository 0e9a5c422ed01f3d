"""Euclidean projection onto X = {lo <= v <= hi, 1^T v <= vmax} (oracle, FP64).

Sec. 4.2 (Efficient Implementation) and Alg. 4.  If clamping to the box
already satisfies the sum constraint the clamp is the projection.
Otherwise the KKT conditions give v = clamp(y - lambda 1, lo, hi) with
lambda solving the piecewise-linear equation (Eq. piecewiseLinearEQ)
    vmax = sum_e clamp(y_e - lambda, lo, hi),
whose 2E breakpoints are y_e - lo and y_e - hi.  Alg. 4 sorts them and
sweeps with a running slope and right-hand side, then solves on the linear
piece that crosses vmax.  The paper writes the upper bound as 1; it is a
parameter `hi` here.
"""
from __future__ import annotations

import numpy as np


def box_clamp(y, lo, hi):
    return np.clip(np.asarray(y, dtype=np.float64), lo, hi)


def project_alg4(y, lo, hi, vmax, return_lambda=False):
    """Projection by sorting the breakpoints (Alg. 4)."""
    y = np.asarray(y, dtype=np.float64)
    E = y.size
    if vmax < E * lo:
        raise ValueError("infeasible: vmax < E * lo")
    x = box_clamp(y, lo, hi)
    if x.sum() <= vmax:
        return (x, 0.0) if return_lambda else x
    # breakpoints: kind +1 at y_e - lo (element reaches lo, slope back up),
    #              kind -1 at y_e - hi (element leaves hi, slope down)
    pts = np.concatenate([y - lo, y - hi])
    kind = np.concatenate([np.ones(E), -np.ones(E)])
    order = np.argsort(pts, kind="stable")
    pts, kind = pts[order], kind[order]
    slope, rhs, lam_last = 0.0, E * hi, 0.0
    node_lam, node_rhs = [], []
    for lam_star, kd in zip(pts, kind):
        rhs = rhs + slope * (lam_star - lam_last)
        slope += kd
        node_lam.append(lam_star)
        node_rhs.append(rhs)
        lam_last = lam_star
    lam = None
    for a in range(len(node_lam) - 1):
        ra, rb = node_rhs[a], node_rhs[a + 1]
        if ra >= vmax >= rb:
            la, lb = node_lam[a], node_lam[a + 1]
            lam = la if ra == rb else la + (ra - vmax) * (lb - la) / (ra - rb)
            break
    if lam is None:                     # vmax == E*lo exactly: past the last node
        lam = node_lam[-1]
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
