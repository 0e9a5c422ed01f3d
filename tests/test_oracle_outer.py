"""Invariants of the oracle's outer iteration (CPU only): feasibility of
every iterate, the mean-projected gradient sums to zero, the step size
schedule, and agreement of a run with exact inner solves with plain
projected gradient descent on the exact objective."""
import numpy as np

import oracle
import synth
from oracle.outer import OuterContext, outer_step_ref, run_outer_ref, step_size


def _ctx(p, **kw):
    return OuterContext(p.nx, p.ny, p.nz, p.filter_radius, p.fixed_mask, p.springs, **kw)


def test_step_size_schedule():
    assert step_size(0.5, 1) == 0.5
    assert abs(step_size(0.5, 16) - 0.5 / 8.0) < 1e-16


def test_cfg1_run_is_feasible_and_mean_projected():
    p = synth.config("cfg1")
    ctx = _ctx(p)
    x, u, recs, xs = run_outer_ref(ctx, p.x0, p.loads, 8, 0.05, p.inner_steps, 0.0, 1.0, p.vmax)
    for xk in xs:
        assert xk.min() >= 0.0 and xk.max() <= 1.0
        assert xk.sum() <= p.vmax * (1 + 1e-12)
    assert all(np.isfinite(r.compliance) and r.compliance > 0 for r in recs)
    _, _, _, gx = outer_step_ref(ctx, xs[-1], u, p.loads, 9, 0.05, p.inner_steps, 0.0, 1.0, p.vmax)
    assert abs(gx.sum()) <= 1e-12 * np.abs(gx).sum()


def test_exact_inner_solve_gives_projected_gradient_descent():
    """With enough inner CG steps the inexact gradient is the exact one, so
    one outer step equals Proj(x - alpha/2 (g - mean g)) on the exact
    compliance gradient (built from a direct solve)."""
    p = synth.cantilever(4, 3, 3, volfrac=0.3, filter_radius=1.5, outer_iters=1,
                         inner_steps=1, seed=1)
    ctx = _ctx(p)
    x = oracle.project_volume_ref(p.x0, 0.0, 1.0, p.vmax)
    nfree = int((p.fixed_mask == 0).sum())
    x1, u1, rec, _ = outer_step_ref(ctx, x, np.zeros_like(p.loads), p.loads, 1, 0.3, 3 * nfree,
                                    0.0, 1.0, p.vmax)
    rho = oracle.filter_forward(ctx.H, ctx.Hs, x)
    s = oracle.simp_scale(rho)
    K = oracle.assemble_K(ctx.grid, s, p.fixed_mask)
    u = oracle.solve_direct(K, p.loads[0])
    g = oracle.filter_transpose(ctx.H, ctx.Hs, oracle.compliance_gradient(ctx.grid, rho, u, p.fixed_mask))
    g = g - g.mean()
    ref = oracle.project_bisect(x - 0.3 * 0.5 * g, 0.0, 1.0, p.vmax)
    assert np.abs(x1 - ref).max() < 1e-9
    assert abs(rec.compliance - p.loads[0] @ u) < 1e-9 * abs(rec.compliance)


def test_cpfbto_step_uses_one_gmres_cycle():
    """Alg. 3's outer step with the Krylov preconditioner (beta = 1) equals the
    same outer step whose low-level update is one GMRES(D + 1) cycle from u
    (SciPy), and its r_inf is that update's true residual."""
    import scipy.sparse.linalg as spla
    from oracle.density_filter import filter_forward
    p = synth.config("cfg1")
    ctx = _ctx(p)
    x = oracle.project_volume_ref(p.x0, 0.0, 1.0, p.vmax)
    rng = np.random.default_rng(3)
    u0 = np.where(p.fixed_mask == 0, rng.standard_normal(p.ndof) * 1e-2, 0.0)
    deg = 6
    x1, u1, rec, _ = outer_step_ref(ctx, x, u0, p.loads[0], 1, 0.05, 0, 0.0, 1.0, p.vmax,
                                    low_level=("krylov", deg, 1.0))
    s = oracle.simp_scale(filter_forward(ctx.H, ctx.Hs, x))
    K = oracle.assemble_K(ctx.grid, s, p.fixed_mask)
    ug, _ = spla.gmres(K, p.loads[0], x0=u0.copy(), restart=deg + 1, maxiter=1, rtol=0.0, atol=0.0)
    assert np.abs(u1 - ug).max() <= 1e-9 * np.abs(ug - u0).max()
    assert abs(rec.r_inf - np.abs(p.loads[0] - K @ ug).max()) <= 1e-9 * rec.r_inf
    assert abs(rec.compliance - p.loads[0] @ ug) <= 1e-9 * abs(rec.compliance)


def test_exact_low_level_equals_many_pcg_steps():
    """The oracle's direct low-level solve (the PGD baseline) gives the same
    outer step as Jacobi-PCG run to convergence."""
    p = synth.cantilever(4, 3, 3, volfrac=0.3, filter_radius=1.5, outer_iters=1, inner_steps=1, seed=1)
    ctx = _ctx(p)
    x = oracle.project_volume_ref(p.x0, 0.0, 1.0, p.vmax)
    u0 = np.zeros(p.ndof)
    xe, ue, re_, _ = outer_step_ref(ctx, x, u0, p.loads[0], 1, 0.05, 0, 0.0, 1.0, p.vmax, low_level=("exact",))
    xp, up, rp, _ = outer_step_ref(ctx, x, u0, p.loads[0], 1, 0.05, 150, 0.0, 1.0, p.vmax)
    assert np.abs(ue - up).max() <= 1e-9 * np.abs(ue).max()
    assert np.abs(xe - xp).max() <= 1e-10
    assert abs(re_.compliance - rp.compliance) <= 1e-10 * re_.compliance


def test_relative_projection_error_pins():
    """Delta^v (Sec. 4, after Thm. 1) is 0 at a first-order point of X;
    equals |g|^2 when the step stays inside the box and below the volume
    bound (the projection is the identity); equals |g - mean g|^2 when the
    volume bound is active and the box is not hit (the projection only
    shifts by a constant)."""
    from oracle import relative_projection_error as dv
    # a KKT point: x_0 at hi with -g_0 pushing out, x_1 at lo with -g_1
    # pushing below, interior entries with equal gradient = -(the multiplier)
    x = np.array([1.0, 0.0, 0.5, 0.5])
    g = np.array([-3.0, 2.0, -0.7, -0.7])
    for alpha in (1e-3, 0.1, 1.0, 10.0):
        assert dv(x, g, alpha, 0.0, 1.0, 2.0) * alpha ** 2 <= 1e-30   # |z - x| at rounding level
    rng = np.random.default_rng(3)
    x = rng.uniform(0.3, 0.7, 50)
    g = rng.normal(0.0, 1.0, 50)
    alpha = 1e-3
    assert abs(dv(x, g, alpha, 0.0, 1.0, x.sum() + 1.0) - (g ** 2).sum()) <= 1e-9 * (g ** 2).sum()
    gp = g - g.mean()
    assert abs(dv(x, g, alpha, 0.0, 1.0, x.sum()) - (gp ** 2).sum()) <= 1e-9 * (gp ** 2).sum()


def test_true_objective_gradient_matches_fd():
    """The exact objective's gradient (through the filter) against central
    differences of direct solves, and l = compliance / 2."""
    p = synth.cantilever(4, 3, 2, volfrac=0.3, filter_radius=1.5, outer_iters=1, inner_steps=1, seed=4)
    ctx = OuterContext(p.nx, p.ny, p.nz, p.filter_radius, p.fixed_mask, p.springs)
    x = synth.uniform_density(p.E, 9)
    l, grad, U = oracle.true_objective(ctx, x, p.loads)
    assert abs(2 * l - float(p.loads[0] @ U[0])) <= 1e-14 * abs(l)
    h = 1e-5
    for j in range(p.E):
        xp, xm = x.copy(), x.copy()
        xp[j] += h
        xm[j] -= h
        fd = (oracle.true_objective(ctx, xp, p.loads)[0] - oracle.true_objective(ctx, xm, p.loads)[0]) / (2 * h)
        assert abs(fd - grad[j]) <= 1e-6 * np.abs(grad).max()
