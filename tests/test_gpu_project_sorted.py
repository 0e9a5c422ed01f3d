"""GPU parity of the sort-based projection (fbto_project_volume_sorted: Alg. 4
as a radix sort and scans) against the oracle's projection, and against the
other device projection at full size."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import DEV, EPS, dev, host, say

pytestmark = pytest.mark.gpu


def _grid(nx, ny, nz, vf=0.3):
    from paper_2204_06204_amd.grid import Grid
    p = synth.cantilever(nx, ny, nz, volfrac=vf, filter_radius=1.0, outer_iters=1, inner_steps=1)
    return p, Grid.from_problem(p)


def _values(kind, E, seed):
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        return rng.uniform(-0.4, 1.4, E)
    if kind == "ties":                       # few distinct values: long runs of equal keys
        return rng.integers(-2, 7, E) * 0.25
    if kind == "signs":                      # both signs, zeros of both signs, wide exponents
        y = rng.normal(0.0, 1.0, E) * 10.0 ** rng.integers(-6, 4, E)
        y[: min(E, 4)] = [-0.0, 0.0, -0.0, 0.0][: min(E, 4)]
        return y
    if kind == "design":                     # a gradient step from a feasible density
        return rng.uniform(0.2, 0.4, E) - 0.05 * rng.normal(0.0, 1.0, E)
    raise ValueError(kind)


def _phi(y, lam, lo, hi):
    return np.clip(y - lam, lo, hi).sum()


def _sum_bound(y, xr, lo, hi):
    """Bound on the multiplier's FP64 error from the sums (both sides form
    the volume sum as running or prefix sums of the y values, each with an
    error of a small multiple of eps * sum |y|).  Divided by the slope at
    the root (the elements strictly inside the box, at least 1 on a piece
    next to it), that is the error in lambda and so in x."""
    n_act = int(((xr > lo) & (xr < hi)).sum())
    return 16 * EPS[torch.float64] * float(np.abs(y).sum()) / max(1, n_act)


# E = 765 (one ragged tile), 6 (a partial wave), 8000 (three tiles and a
# ragged fourth), 524288 (256 whole tiles), 1 (a single element)
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("shape,kind,seed", [((17, 9, 5), "uniform", 1), ((6, 1, 1), "ties", 2),
                                             ((40, 20, 10), "ties", 3), ((40, 20, 10), "signs", 4),
                                             ((128, 64, 64), "design", 5), ((1, 1, 1), "uniform", 6)])
def test_sorted_projection_against_alg4(dtype, shape, kind, seed):
    say(f"sorted projection {shape} {kind} {dtype}")
    p, g = _grid(*shape)
    y_t = dev(_values(kind, p.E, seed), dtype)
    yd = host(y_t)
    lam = torch.zeros(1, dtype=torch.float64, device=DEV)
    for lo in (0.0, 0.1):
        s0 = float(np.clip(yd, lo, 1.0).sum())
        # the workload's bound, a middle one, and crossings near either end
        # of the node range (just above lo * E; just below sum clamp(y))
        for vmax in (p.vmax, lo * p.E + 0.37 * p.E * (1.0 - lo), lo * p.E + 1e-3 * p.E * (1.0 - lo),
                     s0 - 1e-6 * (s0 - lo * p.E)):
            if vmax < lo * p.E:
                continue
            x = host(g.project_volume(y_t, lo=lo, hi=1.0, vmax=vmax, lam=lam, method="sort"))
            xr, lr = oracle.project_volume_ref(yd, lo, 1.0, vmax, return_lambda=True)
            sb = _sum_bound(yd, xr, lo, 1.0)
            xtol = (1e-12 if dtype == torch.float64 else 2 * EPS[torch.float32]) + sb
            assert np.abs(x - xr).max() <= xtol, (lo, vmax, np.abs(x - xr).max())
            lg = float(lam[0])
            if lr == 0.0:
                assert lg == 0.0, lg            # clamp(y) is feasible
            elif kind in ("ties", "signs"):
                # gaps wider than hi - lo: the root may lie on a flat piece,
                # where every root gives the same x
                assert abs(_phi(yd, lg, lo, 1.0) - vmax) <= 1e-9 * max(1.0, vmax) + p.E * sb
            else:
                assert abs(lg - lr) <= 1e-10 * max(1.0, abs(lr)) + sb, (lg, lr)
            if lr > 0:
                assert abs(x.sum() - vmax) <= 1e-9 * vmax + p.E * xtol


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_sorted_projection_edge_cases(dtype):
    from paper_2204_06204_amd import FbtoError
    say(f"sorted projection edge cases {dtype}")
    p, g = _grid(8, 4, 4, vf=0.9)
    y = dev(np.random.default_rng(0).uniform(0, 1.2, p.E), dtype)
    yd = host(y)
    lam = torch.full((1,), -1.0, dtype=torch.float64, device=DEV)
    # clamp(y) feasible: lambda = 0 and x = clamp(y)
    x = host(g.project_volume(y, lo=0.0, hi=1.0, vmax=0.9 * p.E, lam=lam, method="sort"))
    assert np.array_equal(x, np.clip(yd, 0.0, 1.0).astype(host(y).dtype)) and float(lam[0]) == 0.0
    # vmax = lo * E: every element at lo
    x = host(g.project_volume(y, lo=0.2, hi=1.0, vmax=0.2 * p.E, lam=lam, method="sort"))
    assert np.abs(x - 0.2).max() <= 2 * EPS[dtype]
    # lo = hi: the box is a point
    x = host(g.project_volume(y, lo=0.5, hi=0.5, vmax=0.5 * p.E, lam=lam, method="sort"))
    assert np.all(x == 0.5) and float(lam[0]) == 0.0
    # empty feasible set
    with pytest.raises(FbtoError):
        g.project_volume(y, lo=0.5, hi=1.0, vmax=0.1 * p.E, method="sort")
    # in place (x aliases y)
    yy = y.clone()
    xr = oracle.project_volume_ref(yd, 0.0, 1.0, 0.3 * p.E)
    g.project_volume(yy, x=yy, lo=0.0, hi=1.0, vmax=0.3 * p.E, method="sort")
    assert np.abs(host(yy) - xr).max() <= (1e-12 if dtype == torch.float64 else 2 * EPS[torch.float32])
    # a non-finite input gives lambda = NaN and x = NaN
    yn = y.clone()
    yn[5] = float("nan")
    x = host(g.project_volume(yn, lo=0.0, hi=1.0, vmax=0.3 * p.E, lam=lam, method="sort"))
    assert np.isnan(float(lam[0])) and np.all(np.isnan(x))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_sorted_projection_deterministic_and_matches_newton(dtype):
    """Two calls agree bit for bit; the two device projections agree."""
    say(f"sorted vs newton projection 128x64x64 {dtype}")
    p, g = _grid(128, 64, 64, vf=0.25)
    y = dev(_values("design", p.E, 11), dtype)
    la = torch.zeros(1, dtype=torch.float64, device=DEV)
    lb = torch.zeros(1, dtype=torch.float64, device=DEV)
    lc = torch.zeros(1, dtype=torch.float64, device=DEV)
    xa = g.project_volume(y, lo=0.0, hi=1.0, vmax=p.vmax, lam=la, method="sort")
    xb = g.project_volume(y, lo=0.0, hi=1.0, vmax=p.vmax, lam=lb, method="sort")
    xc = g.project_volume(y, lo=0.0, hi=1.0, vmax=p.vmax, lam=lc, method="newton")
    assert torch.equal(xa, xb) and float(la[0]) == float(lb[0])
    assert abs(float(la[0]) - float(lc[0])) <= 1e-12 * max(1.0, abs(float(lc[0])))
    assert float((xa.double() - xc.double()).abs().max()) <= (1e-14 if dtype == torch.float64 else EPS[torch.float32])


def test_sorted_projection_at_14m_elements():
    """384x192x192 (14,155,776 elements, 6,912 tiles) in FP32: the root
    satisfies the volume equation in FP64, x = clamp(y - lambda) on a sample,
    and the multiplier agrees with the Newton projection."""
    say("sorted projection 384x192x192 fp32")
    p, g = _grid(384, 192, 192, vf=0.1)
    y = dev(_values("design", p.E, 12), torch.float32)
    yd = host(y)
    ls = torch.zeros(1, dtype=torch.float64, device=DEV)
    ln = torch.zeros(1, dtype=torch.float64, device=DEV)
    x = g.project_volume(y, lo=0.0, hi=1.0, vmax=p.vmax, lam=ls, method="sort")
    g.project_volume(y, lo=0.0, hi=1.0, vmax=p.vmax, lam=ln, method="newton")
    lam = float(ls[0])
    assert lam > 0.0
    assert abs(_phi(yd, lam, 0.0, 1.0) - p.vmax) <= 1e-10 * p.vmax
    assert abs(lam - float(ln[0])) <= 1e-10 * abs(lam)
    idx = np.random.default_rng(3).integers(0, p.E, 4096)
    xs = host(x)[idx]
    ref = np.clip(yd[idx] - lam, 0.0, 1.0).astype(np.float32).astype(np.float64)
    assert np.array_equal(xs, ref)
