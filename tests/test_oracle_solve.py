"""Pins for the oracle's inner solvers (CPU only): pcg_ref follows SciPy's
preconditioned CG iterate for iterate, reaches the direct solution when run
long enough, and the Alg. 1 / damped-Jacobi variants are checked against
their fixed points."""
import numpy as np
import scipy.sparse.linalg as spla

import oracle
import synth
from oracle.grid import Grid


def _system(nx=6, ny=4, nz=3, seed=0):
    g = Grid(nx, ny, nz)
    p = synth.cantilever(nx, ny, nz, volfrac=0.3, filter_radius=1.5, outer_iters=1,
                         inner_steps=5, seed=seed)
    s = oracle.simp_scale(p.x0)
    K = oracle.assemble_K(g, s, p.fixed_mask)
    D = oracle.jacobi_diag(g, s, p.fixed_mask)
    return g, p, s, K, D


def test_pcg_ref_matches_scipy_cg_iterates():
    g, p, s, K, D = _system()
    f = p.loads[0]
    rng = np.random.default_rng(5)
    u0 = np.where(p.fixed_mask == 0, rng.standard_normal(g.ndof) * 1e-2, 0.0)
    m = 7
    _, _, its = oracle.pcg_ref(lambda v: K @ v, D, f, u0, m, history=True)
    seen = []
    M = spla.LinearOperator(K.shape, matvec=lambda v: v / D)
    spla.cg(K, f, x0=u0.copy(), M=M, maxiter=m, rtol=0.0, atol=0.0,
            callback=lambda xk: seen.append(xk.copy()))
    assert len(seen) == m
    for a, b in zip(its, seen):
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()


def test_pcg_ref_converges_to_direct_solution():
    g, p, s, K, D = _system(2, 2, 2)
    f = p.loads[0]
    u_ex = oracle.solve_direct(K, f)
    nfree = int((p.fixed_mask == 0).sum())
    u, r = oracle.pcg_ref(lambda v: K @ v, D, f, np.zeros(g.ndof), nfree)
    assert np.abs(u - u_ex).max() <= 1e-10 * np.abs(u_ex).max()
    # the recursive residual tracks the true residual
    assert np.abs(r - (f - K @ u)).max() <= 1e-10 * np.abs(f).max()


def test_pcg_to_tol_and_variants():
    g, p, s, K, D = _system(4, 3, 3)
    f = p.loads[0]
    u_ex = oracle.solve_direct(K, f)
    u, rel, its = oracle.pcg_to_tol(lambda v: K @ v, D, f, np.zeros(g.ndof), 1e-12)
    assert rel <= 1e-11 and np.abs(u - u_ex).max() <= 1e-9 * np.abs(u_ex).max()
    # the exact solution is a fixed point of Alg. 1's step and of damped Jacobi
    from oracle.solve import damped_jacobi_ref, richardson_ref
    u1, _ = richardson_ref(lambda v: K @ v, f, u_ex, 3, 0.5)
    u2, _ = damped_jacobi_ref(lambda v: K @ v, D, f, u_ex, 3, 0.6)
    assert np.abs(u1 - u_ex).max() <= 1e-10 * np.abs(u_ex).max()
    assert np.abs(u2 - u_ex).max() <= 1e-10 * np.abs(u_ex).max()
    # energy-norm error of PCG decreases monotonically
    errs = []
    for m in range(1, 12):
        um, _ = oracle.pcg_ref(lambda v: K @ v, D, f, np.zeros(g.ndof), m)
        e = um - u_ex
        errs.append(e @ (K @ e))
    assert all(b <= a * (1 + 1e-12) for a, b in zip(errs, errs[1:]))
