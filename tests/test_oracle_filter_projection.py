"""Pins for the oracle's density filter and projection (CPU only)."""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle.density_filter import stencil_offsets
from oracle.grid import Grid


def brute_force_filter(g: Grid, r: float, x):
    """O(E^2) cone filter straight from its definition."""
    ex, ey, ez = g.elem_coords()
    C = np.stack([ex, ey, ez], axis=1).astype(float) + 0.5
    out = np.zeros(g.E)
    for e in range(g.E):
        d = np.sqrt(((C - C[e]) ** 2).sum(axis=1))
        w = np.maximum(0.0, r - d)
        out[e] = (w @ x) / w.sum()
    return out


@pytest.mark.parametrize("r", [1.0, 1.5, 2.0, 3.0])
def test_filter_against_brute_force(r):
    g = Grid(6, 5, 4)
    x = np.random.default_rng(3).uniform(0, 1, g.E)
    H, Hs = oracle.cone_filter_matrix(g, r)
    assert np.abs(oracle.filter_forward(H, Hs, x) - brute_force_filter(g, r, x)).max() < 1e-15


def test_filter_properties():
    g = Grid(7, 4, 5)
    rng = np.random.default_rng(4)
    for r in (1.5, 2.0, 3.0):
        H, Hs = oracle.cone_filter_matrix(g, r)
        assert np.allclose(oracle.filter_forward(H, Hs, np.full(g.E, 0.37)), 0.37, rtol=0, atol=1e-15)
        x, y = rng.standard_normal(g.E), rng.standard_normal(g.E)
        lhs = oracle.filter_forward(H, Hs, x) @ y
        rhs = x @ oracle.filter_transpose(H, Hs, y)
        assert abs(lhs - rhs) < 1e-13 * abs(lhs)
    # interior stencil sizes of the cone filter
    assert [len(stencil_offsets(r)) for r in (1.0, 1.5, 2.0, 3.0)] == [1, 19, 27, 93]


def brute_force_projection(y, lo, hi, vmax):
    """Enumerate every assignment of {at lo, at hi, free} to the elements,
    solve the free part from the active sum constraint, keep KKT-consistent
    candidates, return the closest point (E <= 7)."""
    E = y.size
    best, best_d = None, np.inf
    clamp = np.clip(y, lo, hi)
    if clamp.sum() <= vmax:
        return clamp
    for states in itertools.product((0, 1, 2), repeat=E):
        st = np.array(states)
        free = st == 2
        if not free.any():
            x = np.where(st == 0, lo, hi)
            if abs(x.sum() - vmax) > 1e-12:
                continue
            lam = None
        else:
            fixed_sum = lo * (st == 0).sum() + hi * (st == 1).sum()
            lam = (y[free].sum() + fixed_sum - vmax) / free.sum()
            x = np.where(st == 0, lo, np.where(st == 1, hi, y - lam))
            if lam < -1e-12:
                continue
            z = y - lam
            if np.any((st == 0) & (z > lo + 1e-12)) or np.any((st == 1) & (z < hi - 1e-12)):
                continue
            if np.any(free & ((z < lo - 1e-12) | (z > hi + 1e-12))):
                continue
        d = ((x - y) ** 2).sum()
        if d < best_d:
            best, best_d = x, d
    return best


def test_projection_against_brute_force_and_bisection():
    rng = np.random.default_rng(7)
    for trial in range(40):
        E = int(rng.integers(1, 7))
        y = rng.uniform(-0.5, 1.5, E)
        if trial % 5 == 0:
            y[: E // 2] = y[0]                      # ties
        lo, hi = 0.1, 1.0
        vmax = float(rng.uniform(E * lo, E * hi))
        x4 = oracle.project_volume_ref(y, lo, hi, vmax)
        xb = brute_force_projection(y, lo, hi, vmax)
        xs = oracle.project_bisect(y, lo, hi, vmax)
        assert np.abs(x4 - xb).max() < 1e-12
        assert np.abs(x4 - xs).max() < 1e-12


def test_projection_kkt_large():
    rng = np.random.default_rng(8)
    E = 20000
    y = rng.uniform(-0.3, 1.4, E)
    lo, hi, vmax = 0.0, 1.0, 0.25 * E
    x, lam = oracle.project_volume_ref(y, lo, hi, vmax, return_lambda=True)
    assert lam > 0
    assert abs(x.sum() - vmax) <= 1e-12 * vmax
    assert np.abs(x - np.clip(y - lam, lo, hi)).max() == 0.0
    xb, lamb = oracle.project_bisect(y, lo, hi, vmax, return_lambda=True)
    assert abs(lam - lamb) < 1e-13
    # inactive: clamp returned unchanged
    assert np.array_equal(oracle.project_volume_ref(y, lo, hi, 0.9 * E), np.clip(y, lo, hi))
    with pytest.raises(ValueError):
        oracle.project_volume_ref(y, 0.5, 1.0, 0.25 * E)


@pytest.mark.parametrize("r", [1.5, 2.0, 3.0])
def test_sampled_filter_equals_matrix_filter(r):
    """The per-element filter (forward, transpose, weight sums) used for
    sampled checks on large grids equals the matrix filter at every element
    of a small grid, boundary-truncated stencils included."""
    g = Grid(9, 6, 5)
    H, Hs = oracle.cone_filter_matrix(g, r)
    rng = np.random.default_rng(7)
    x = rng.uniform(0.0, 1.0, g.E)
    gr = rng.normal(0.0, 1.0, g.E)
    e = np.arange(g.E)
    assert np.allclose(oracle.filter_weight_sums_at(g, r, e), Hs, rtol=0, atol=1e-13)
    assert np.allclose(oracle.filter_forward_at(g, r, x, e), oracle.filter_forward(H, Hs, x), rtol=0, atol=1e-14)
    assert np.allclose(oracle.filter_transpose_at(g, r, gr, e), oracle.filter_transpose(H, Hs, gr), rtol=0, atol=1e-13)
