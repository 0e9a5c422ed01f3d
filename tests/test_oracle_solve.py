"""Pins for the oracle's inner solvers (CPU only): pcg_ref follows SciPy's
preconditioned CG iterate for iterate, reaches the direct solution when run
long enough, and the Alg. 1 / damped-Jacobi variants are checked against
their fixed points.  The Krylov step of Alg. 3 (Eq. LSP) is pinned against
SciPy's GMRES with one cycle of D + 1 steps, against the exact solve when
the operator has D + 1 distinct eigenvalues, and by the monotone decrease
of its residual in D."""
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


def test_relaxation_steps_on_eigenvectors():
    """Pins Alg. 1's low-level update u <- u - beta (K u - f) and the damped
    Jacobi step u <- u - omega D^-1 (K u - f) by their action on
    eigenvectors: from u0 = u* + v with K v = lam v, one Richardson step
    gives exactly u* + (1 - beta lam) v; from u0 = u* + w with K w = mu D w
    (an eigenvector of D^-1 K), one damped Jacobi step gives
    u* + (1 - omega mu) w.  A flipped sign, a missing beta, or D in place of
    D^-1 gives another factor and fails."""
    import scipy.linalg as sla
    from oracle.solve import damped_jacobi_ref, richardson_ref
    g, p, s, K, D = _system(3, 2, 2)
    f = p.loads[0]
    u_ex = oracle.solve_direct(K, f)
    Kd = K.toarray()
    lam, V = np.linalg.eigh(Kd)
    mu, W = sla.eigh(Kd, np.diag(D))
    for i in (0, len(lam) // 3, len(lam) - 1):
        v = V[:, i]
        for beta in (0.3 / lam[-1], 1.0 / lam[-1], 1.7 / lam[-1]):
            u1, r1 = richardson_ref(lambda q: K @ q, f, u_ex + v, 1, beta)
            assert np.abs(u1 - (u_ex + (1.0 - beta * lam[i]) * v)).max() <= 1e-12
            assert np.abs(r1 - (f - K @ u1)).max() <= 1e-12
            u2, _ = richardson_ref(lambda q: K @ q, f, u_ex + v, 2, beta)
            assert np.abs(u2 - (u_ex + (1.0 - beta * lam[i]) ** 2 * v)).max() <= 1e-12
        w = W[:, i] / np.abs(W[:, i]).max()
        for omega in (0.4, 0.9, 1.3):
            u1, _ = damped_jacobi_ref(lambda q: K @ q, D, f, u_ex + w, 1, omega)
            assert np.abs(u1 - (u_ex + (1.0 - omega * mu[i]) * w)).max() <= 1e-11
    # the Jacobi diagonal is not constant here, so D^-1 and D (or no D) differ
    assert D.max() / D.min() > 1.5


def test_krylov_step_is_one_gmres_cycle():
    """Eq. LSP with beta = 1 minimises the residual over u + span{delta, ...,
    K^D delta}, which is what one GMRES(D + 1) cycle from u computes (by a
    different, Arnoldi-based route)."""
    g, p, s, K, D = _system(6, 4, 3)
    f = p.loads[0]
    rng = np.random.default_rng(1)
    u0 = np.where(p.fixed_mask == 0, rng.standard_normal(g.ndof) * 1e-2, 0.0)
    for deg in (2, 5, 10):
        u1, r1 = oracle.krylov_step_ref(lambda v: K @ v, f, u0, deg)
        ug, _ = spla.gmres(K, f, x0=u0.copy(), restart=deg + 1, maxiter=1, rtol=0.0, atol=0.0)
        assert np.abs(u1 - ug).max() <= 1e-9 * np.abs(ug - u0).max(), deg
        assert np.abs(r1 - (f - K @ u1)).max() <= 1e-12 * np.abs(f).max()
    # D = 20: the monomial basis is ill-conditioned; the least-squares
    # residual it reaches is still within 1e-3 of the optimum
    u1, r1 = oracle.krylov_step_ref(lambda v: K @ v, f, u0, 20)
    ug, _ = spla.gmres(K, f, x0=u0.copy(), restart=21, maxiter=1, rtol=0.0, atol=0.0)
    rg = np.linalg.norm(f - K @ ug)
    assert rg <= np.linalg.norm(r1) <= rg * (1.0 + 1e-3)


def test_krylov_step_exact_with_few_eigenvalues():
    """An SPD operator with 4 distinct eigenvalues is solved exactly by the
    degree-3 Krylov step (its minimal polynomial has degree 4)."""
    rng = np.random.default_rng(2)
    n = 40
    Qm, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.repeat([0.5, 1.0, 2.0, 4.0], n // 4)
    Kd = (Qm * lam) @ Qm.T
    f = rng.standard_normal(n)
    u0 = rng.standard_normal(n)
    u1, r1 = oracle.krylov_step_ref(lambda v: Kd @ v, f, u0, 3)
    u_ex = np.linalg.solve(Kd, f)
    assert np.abs(u1 - u_ex).max() <= 1e-10 * np.abs(u_ex).max()
    # the damped step moves a fraction beta of the way
    uh, _ = oracle.krylov_step_ref(lambda v: Kd @ v, f, u0, 3, beta=0.25)
    assert np.abs(uh - (u0 + 0.25 * (u_ex - u0))).max() <= 1e-10 * np.abs(u_ex).max()


def test_krylov_step_residual_decreases_with_degree():
    """A larger Krylov space can only lower the minimal residual, and any
    D >= 0 lowers it below the starting one for an SPD K (the contraction
    the convergence argument of Alg. 3 relies on)."""
    g, p, s, K, D = _system(5, 3, 3)
    f = p.loads[0]
    u0 = np.zeros(g.ndof)
    prev = np.linalg.norm(f)
    for deg in (0, 1, 2, 4, 8):
        _, r = oracle.krylov_step_ref(lambda v: K @ v, f, u0, deg)
        cur = np.linalg.norm(r)
        assert cur < prev
        prev = cur
