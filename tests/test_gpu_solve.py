"""GPU parity of the low-level solves: Jacobi-PCG iterate after m steps,
Alg. 1's gradient step and damped Jacobi against the oracle's recurrences,
the solve-to-tolerance mode, and the FP64 iterative refinement of an FP32
inner solve (checked by the oracle's own FP64 residual and exact solve)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle.grid import Grid as OGrid
from gpu_util import DEV, dev, host, say

pytestmark = pytest.mark.gpu


def _setup(p, dtype, seed=3, max_rhs=1):
    from paper_2204_06204_amd.grid import Grid
    og = OGrid(p.nx, p.ny, p.nz)
    g = Grid.from_problem(p, max_rhs=max_rhs)
    rho_t = dev(synth.uniform_density(p.E, seed), dtype)
    s = oracle.simp_scale(host(rho_t), p.penal, p.rho_min)
    K = oracle.assemble_K(og, s, p.fixed_mask, p.springs)
    D = oracle.jacobi_diag(og, s, p.fixed_mask, p.springs)
    return og, g, rho_t, s, K, D


CASES = [(24, 13, 11, 5), (37, 9, 6, 6), (5, 3, 2, 7)]


@pytest.mark.parametrize("nx,ny,nz,seed", CASES)
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_pcg_steps_match_oracle(nx, ny, nz, seed, dtype):
    say(f"pcg {nx}x{ny}x{nz} {dtype}")
    p = synth.cantilever(nx, ny, nz, volfrac=0.3, filter_radius=1.5, outer_iters=1, inner_steps=5,
                         seed=seed)
    og, g, rho_t, s, K, D = _setup(p, dtype, seed)
    f = p.loads[0]
    rng = np.random.default_rng(seed)
    u0 = np.where(p.fixed_mask == 0, rng.standard_normal(p.ndof) * 1e-1, 0.0)
    u_t = dev(u0, dtype)
    u0 = host(u_t)
    info = torch.zeros(8, dtype=torch.float64, device=DEV)
    m = 6
    g.inner_solve(rho_t, dev(f, dtype), u_t, m, info=info)
    u_ref, r_ref = oracle.pcg_ref(lambda v: K @ v, D, f, u0, m)
    u = host(u_t)
    tol = 1e-10 if dtype == torch.float64 else 2e-4
    assert np.abs(u - u_ref).max() <= tol * np.abs(u_ref).max()
    inf = host(info)
    assert inf[3] == m and inf[4] == 0
    assert abs(inf[0] - np.linalg.norm(r_ref)) <= (1e-8 if dtype == torch.float64 else 1e-2) * np.linalg.norm(r_ref)
    assert abs(inf[2] - np.linalg.norm(f)) <= 1e-12


def test_pcg_multi_rhs_independent():
    p = synth.multiload_cantilever(20, 10, 10, seed=4)
    og, g, rho_t, s, K, D = _setup(p, torch.float64, 8, max_rhs=4)
    F = p.loads
    U = torch.zeros(4 * p.ndof, dtype=torch.float64, device=DEV)
    g.inner_solve(rho_t, dev(F.ravel()), U, 7)
    Uh = host(U).reshape(4, -1)
    for r in range(4):
        ur, _ = oracle.pcg_ref(lambda v: K @ v, D, F[r], np.zeros(p.ndof), 7)
        assert np.abs(Uh[r] - ur).max() <= 1e-10 * np.abs(ur).max()


@pytest.mark.parametrize("method,omega", [("richardson", 0.5), ("jacobi", 0.6)])
def test_relaxation_variants(method, omega):
    p = synth.cantilever(10, 5, 4, volfrac=0.3, filter_radius=1.5, outer_iters=1, inner_steps=5, seed=9)
    og, g, rho_t, s, K, D = _setup(p, torch.float64, 9)
    f = p.loads[0]
    u_t = torch.zeros(p.ndof, dtype=torch.float64, device=DEV)
    g.inner_solve(rho_t, dev(f), u_t, 9, method=method, omega=omega)
    from oracle.solve import damped_jacobi_ref, richardson_ref
    if method == "richardson":
        ur, _ = richardson_ref(lambda v: K @ v, f, np.zeros(p.ndof), 9, omega)
    else:
        ur, _ = damped_jacobi_ref(lambda v: K @ v, D, f, np.zeros(p.ndof), 9, omega)
    assert np.abs(host(u_t) - ur).max() <= 1e-12 * np.abs(ur).max()


def test_residual_info_per_load_case():
    """Four load cases (the largest RHS count) on a grid of many blocks:
    after damped Jacobi steps, whose final norms come from the residual
    pass, every case's reported ||r||_2, ||r||_inf and ||f||_2 equal those
    of the oracle's residual (each case's |r|_inf is a max over blocks,
    not a sum)."""
    p = synth.multiload_cantilever(24, 12, 12, seed=4)
    og, g, rho_t, s, K, D = _setup(p, torch.float64, 8, max_rhs=4)
    F = p.loads
    U = torch.zeros(4 * p.ndof, dtype=torch.float64, device=DEV)
    info = torch.zeros(4 * 8, dtype=torch.float64, device=DEV)
    g.inner_solve(rho_t, dev(F.ravel()), U, 6, method="jacobi", omega=0.6, info=info)
    Uh = host(U).reshape(4, -1)
    inf = host(info).reshape(4, 8)
    for r in range(4):
        res = F[r] - K @ Uh[r]
        assert abs(inf[r][0] - np.linalg.norm(res)) <= 1e-12 * np.linalg.norm(F[r]), r
        assert abs(inf[r][1] - np.abs(res).max()) <= 1e-12 * np.abs(F[r]).max(), r
        assert abs(inf[r][2] - np.linalg.norm(F[r])) <= 1e-13 * np.linalg.norm(F[r]), r


def test_pcg_to_tolerance():
    p = synth.cantilever(16, 8, 8, volfrac=0.3, filter_radius=1.5, outer_iters=1, inner_steps=5, seed=2)
    og, g, rho_t, s, K, D = _setup(p, torch.float64, 2)
    f = p.loads[0]
    u_t = torch.zeros(p.ndof, dtype=torch.float64, device=DEV)
    info = torch.zeros(8, dtype=torch.float64, device=DEV)
    g.inner_solve(rho_t, dev(f), u_t, 20000, rtol=1e-10, info=info)
    u = host(u_t)
    u_ex = oracle.solve_direct(K, f)
    assert np.linalg.norm(f - K @ u) <= 2e-10 * np.linalg.norm(f)
    assert abs(f @ u - f @ u_ex) <= 1e-9 * abs(f @ u_ex)
    assert host(info)[3] < 20000


@pytest.mark.parametrize("inner", [torch.float32, torch.float64])
def test_iterative_refinement_small(inner):
    say(f"IR small {inner}")
    p = synth.cantilever(16, 8, 8, volfrac=0.3, filter_radius=1.5, outer_iters=1, inner_steps=5, seed=12)
    og, g, rho_t, s, K, D = _setup(p, torch.float64, 12)
    f = p.loads[0]
    u = torch.zeros(p.ndof, dtype=torch.float64, device=DEV)
    nref = g.solve_refined(rho_t, dev(f), u, 1e-10, 200, 60, inner_dtype=inner)
    uh = host(u)
    u_ex = oracle.solve_direct(K, f)
    assert np.linalg.norm(f - K @ uh) <= 1e-10 * np.linalg.norm(f)
    assert abs(f @ uh - f @ u_ex) <= 1e-9 * abs(f @ u_ex)
    assert 1 <= nref <= 200


def test_iterative_refinement_cfg3_residual():
    """128x64x64 cantilever: FP32 inner PCG + FP64 refinement reaches
    ||f - K u|| <= 1e-8 ||f||, with the residual recomputed by the oracle's
    FP64 element loop; the compliance agrees with the oracle's
    residual-corrected estimate  f.u + u.r  to 1e-6 (error r^T K^-1 r)."""
    say("IR cfg3")
    p = synth.config("cfg3")
    from paper_2204_06204_amd.grid import Grid
    og = OGrid(p.nx, p.ny, p.nz)
    g = Grid.from_problem(p)
    rho_t = dev(p.x0)
    f = p.loads[0]
    u = torch.zeros(p.ndof, dtype=torch.float64, device=DEV)
    nref = g.solve_refined(rho_t, dev(f), u, 1e-8, 400, 200, inner_dtype=torch.float32)
    uh = host(u)
    s = oracle.simp_scale(p.x0, p.penal, p.rho_min)
    r = f - oracle.apply_K(og, s, uh, p.fixed_mask)
    assert np.linalg.norm(r) <= 1.05e-8 * np.linalg.norm(f), (nref, np.linalg.norm(r))
    c = f @ uh
    c_corr = c + uh @ r
    assert abs(c - c_corr) <= 1e-6 * abs(c_corr)


def test_solver_state_is_reset_between_calls():
    """A converged tolerance solve must not leak its convergence flag or
    step count into later solves on the same grid handle."""
    p = synth.cantilever(16, 8, 8, volfrac=0.3, filter_radius=1.5, outer_iters=1, inner_steps=5, seed=2)
    og, g, rho_t, s, K, D = _setup(p, torch.float64, 2)
    f = p.loads[0]
    info = torch.zeros(8, dtype=torch.float64, device=DEV)
    u = torch.zeros(p.ndof, dtype=torch.float64, device=DEV)
    g.inner_solve(rho_t, dev(f), u, 20000, rtol=1e-10, info=info)
    assert host(info)[4] == 0
    # fixed-step solve from zero on the same handle: exactly the oracle iterate
    u2 = torch.zeros(p.ndof, dtype=torch.float64, device=DEV)
    g.inner_solve(rho_t, dev(f), u2, 6, info=info)
    ur, _ = oracle.pcg_ref(lambda v: K @ v, D, f, np.zeros(p.ndof), 6)
    assert np.abs(host(u2) - ur).max() <= 1e-10 * np.abs(ur).max()
    assert host(info)[3] == 6
    # refinement after a converged solve on the same handle still converges
    u3 = torch.zeros(p.ndof, dtype=torch.float64, device=DEV)
    g.solve_refined(rho_t, dev(f), u3, 1e-10, 200, 60, inner_dtype=torch.float32)
    assert np.linalg.norm(f - K @ host(u3)) <= 1e-10 * np.linalg.norm(f)


@pytest.mark.parametrize("nx,ny,nz,seed", [(24, 13, 11, 5), (5, 3, 2, 7)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_krylov_step_matches_oracle(nx, ny, nz, seed, dtype):
    """One Alg. 3 step with the Krylov preconditioner (Eq. LSP) against the
    oracle's Householder-QR solution.  For D <= 10 both are the exact
    minimiser to rounding; at D = 20 the oracle's monomial basis keeps only
    about four digits, so there the minimal residuals are compared."""
    say(f"krylov {nx}x{ny}x{nz} {dtype}")
    p = synth.cantilever(nx, ny, nz, volfrac=0.3, filter_radius=1.5, outer_iters=1, inner_steps=5,
                         seed=seed)
    og, g, rho_t, s, K, D = _setup(p, dtype, seed)
    f = p.loads[0]
    rng = np.random.default_rng(seed)
    u0 = np.where(p.fixed_mask == 0, rng.standard_normal(p.ndof) * 1e-1, 0.0)
    u0 = host(dev(u0, dtype))
    info = torch.zeros(8, dtype=torch.float64, device=DEV)
    for deg in (0, 3, 8):
        u_t = dev(u0, dtype)
        g.inner_solve(rho_t, dev(f, dtype), u_t, deg, method="krylov", omega=1.0, info=info)
        u_ref, r_ref = oracle.krylov_step_ref(lambda v: K @ v, f, u0, deg)
        u = host(u_t)
        # FP32: D + 1 Lanczos steps in FP32 arithmetic, relative to the update
        tol = 1e-9 if dtype == torch.float64 else 3e-4
        assert np.abs(u - u_ref).max() <= tol * np.abs(u_ref - u0).max(), deg
        inf = host(info)
        assert inf[3] == deg + 1 and inf[4] == 0
        rn = np.linalg.norm(f - K @ u)
        assert abs(inf[0] - rn) <= (1e-8 if dtype == torch.float64 else 1e-3) * rn
    u_t = dev(u0, dtype)
    g.inner_solve(rho_t, dev(f, dtype), u_t, 20, method="krylov", omega=1.0)
    _, r_ref = oracle.krylov_step_ref(lambda v: K @ v, f, u0, 20)
    rn, rref = np.linalg.norm(f - K @ host(u_t)), np.linalg.norm(r_ref)
    assert abs(rn - rref) <= (1e-3 if dtype == torch.float64 else 2e-3) * rref
    assert rn < np.linalg.norm(f - K @ u0)


def test_krylov_step_damping_and_multi_rhs():
    """Alg. 3's beta_k scales the step; load cases are independent (each
    equals its single-case run bitwise)."""
    p = synth.multiload_cantilever(20, 10, 10, seed=4)
    og, g, rho_t, s, K, D = _setup(p, torch.float64, 8, max_rhs=4)
    F = np.concatenate(p.loads)
    rng = np.random.default_rng(4)
    U0 = np.where(np.tile(p.fixed_mask, 4) == 0, rng.standard_normal(4 * p.ndof) * 1e-2, 0.0)
    U = dev(U0, torch.float64)
    g.inner_solve(rho_t, dev(F, torch.float64), U, 6, method="krylov", omega=1.0)
    for r in range(4):
        sl = slice(r * p.ndof, (r + 1) * p.ndof)
        u1 = dev(U0[sl], torch.float64)
        g.inner_solve(rho_t, dev(p.loads[r], torch.float64), u1, 6, method="krylov", omega=1.0)
        assert torch.equal(U[sl], u1)
        uh = dev(U0[sl], torch.float64)
        g.inner_solve(rho_t, dev(p.loads[r], torch.float64), uh, 6, method="krylov", omega=0.5)
        want = U0[sl] + 0.5 * (host(u1) - U0[sl])
        assert np.abs(host(uh) - want).max() <= 1e-12 * np.abs(want).max()


def test_krylov_step_cfg3_residual_decreases():
    """At 128x64x64 (FP32): the step's residual falls with the degree D, as
    the minimal residual over a growing Krylov space must, and the reported
    norm equals an independent f - K u by the apply."""
    say("krylov cfg3")
    p = synth.config("cfg3")
    from paper_2204_06204_amd.grid import Grid
    g = Grid.from_problem(p)
    rho = dev(p.x0, torch.float32)
    f = dev(p.loads[0], torch.float32)
    info = torch.zeros(8, dtype=torch.float64, device=DEV)
    prev = float(torch.linalg.norm(f.double()))
    for deg in (1, 5, 10, 20):
        u = torch.zeros_like(f)
        g.inner_solve(rho, f, u, deg, method="krylov", omega=1.0, info=info)
        inf = host(info)
        r = (f - g.apply_K(rho, u)).double()
        rn = float(torch.linalg.norm(r))
        assert abs(inf[0] - rn) <= 1e-3 * rn
        assert rn < prev, deg
        prev = rn


def test_krylov_step_384x192x192_fp32_against_fp64():
    """The largest workload grid (43M DOFs), degree 20 from u = 0.  The step
    minimises the residual over a space that holds f, so ||r|| <= ||f||.
    The reported norm equals f - K u by the apply.  The FP32 step (fused
    Lanczos passes) agrees with the FP64 one: residual norm to 1e-3 and u
    to 1e-3 of its largest entry."""
    say("krylov 384x192x192 fp32 vs fp64")
    p = synth.config("cfg5")
    from paper_2204_06204_amd.grid import Grid
    g = Grid.from_problem(p)
    info = torch.zeros(8, dtype=torch.float64, device=DEV)
    out = {}
    for dtype in (torch.float32, torch.float64):
        rho = dev(p.x0, dtype)
        f = dev(p.loads[0], dtype)
        u = torch.zeros_like(f)
        g.inner_solve(rho, f, u, 20, method="krylov", omega=1.0, info=info)
        inf = host(info)
        rn = float(torch.linalg.norm((f - g.apply_K(rho, u)).double()))
        fn = float(torch.linalg.norm(f.double()))
        assert inf[4] == 0 and abs(inf[0] - rn) <= 1e-3 * rn and rn < fn, (dtype, inf[0], rn, fn)
        out[dtype] = (rn, host(u))
        del rho, f, u
    (r32, u32), (r64, u64) = out[torch.float32], out[torch.float64]
    assert abs(r32 - r64) <= 1e-3 * r64, (r32, r64)
    assert np.abs(u32 - u64).max() <= 1e-3 * np.abs(u64).max()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_krylov_step_at_the_solution_is_a_fixed_point(dtype):
    """Degenerate case: from the exact solution the residual is zero, every
    Lanczos vector vanishes, and the step must leave u unchanged (no 0/0,
    no 0 * inf in FP32)."""
    p = synth.cantilever(6, 4, 3, volfrac=0.3, filter_radius=1.5, outer_iters=1, inner_steps=1, seed=2)
    og, g, rho_t, s, K, D = _setup(p, dtype, 2)
    f = np.zeros(p.ndof)                      # f = 0: u = 0 is exact, r = 0 exactly
    u_t = torch.zeros(p.ndof, dtype=dtype, device=DEV)
    info = torch.zeros(8, dtype=torch.float64, device=DEV)
    g.inner_solve(rho_t, dev(f, dtype), u_t, 5, method="krylov", omega=1.0, info=info)
    assert torch.count_nonzero(u_t) == 0
    assert host(info)[0] == 0.0 and host(info)[4] == 0


def _indefinite_case():
    """A density field whose stiffness has a positive diagonal but is
    indefinite: solid boundary layer, interior checkerboard of rho = 1 and
    rho = -0.9 (s < 0).  The oracle's PCG meets p^T K p <= 0 on its third
    step with a unit load at the centre node."""
    n = 6
    p = synth.cantilever(n, n, n, volfrac=0.3, filter_radius=1.5, outer_iters=1, inner_steps=5, seed=1)
    og = OGrid(n, n, n)
    ex, ey, ez = og.elem_coords()
    inner = (ex > 0) & (ex < n - 1) & (ey > 0) & (ey < n - 1) & (ez > 0) & (ez < n - 1)
    rho = np.where(inner & ((ex + ey + ez) % 2 == 1), -0.9, 1.0)
    f = np.zeros(p.ndof)
    f[3 * og.node(3, 3, 3) + 2] = -1.0
    return p, og, rho, f


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_pcg_reports_breakdown(dtype):
    """p^T K p <= 0 stops the solve with FBTO_ERR_BREAKDOWN; the iterate is
    the one of the last completed step (FP64: the oracle's, after two)."""
    from paper_2204_06204_amd.grid import Grid
    say(f"pcg breakdown {dtype}")
    p, og, rho, f = _indefinite_case()
    s = oracle.simp_scale(rho, p.penal, p.rho_min)
    K = oracle.assemble_K(og, s, p.fixed_mask)
    D = oracle.jacobi_diag(og, s, p.fixed_mask)
    with pytest.raises(FloatingPointError):
        oracle.pcg_ref(lambda v: K @ v, D, f, np.zeros(p.ndof), 3)
    g = Grid.from_problem(p)
    u = torch.zeros(p.ndof, dtype=dtype, device=DEV)
    info = torch.zeros(8, dtype=torch.float64, device=DEV)
    g.inner_solve(dev(rho, dtype), dev(f, dtype), u, 10, info=info)
    inf = host(info)
    assert inf[4] == 5.0, inf          # FBTO_ERR_BREAKDOWN
    # FP32 rounding may move the sign change of p^T K p by one step
    assert inf[3] == 2.0 if dtype == torch.float64 else inf[3] in (2.0, 3.0), inf
    if dtype == torch.float64:
        u_ref, _ = oracle.pcg_ref(lambda v: K @ v, D, f, np.zeros(p.ndof), 2)
        assert np.abs(host(u) - u_ref).max() <= 1e-10 * np.abs(u_ref).max()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_nonfinite_load_is_reported(dtype):
    """A NaN in the load reaches the status slot as FBTO_ERR_NONFINITE, in the
    inner solve and in the outer step's info record."""
    from paper_2204_06204_amd.grid import Grid
    say(f"nonfinite {dtype}")
    p = synth.cantilever(12, 6, 5, volfrac=0.3, filter_radius=1.5, outer_iters=1, inner_steps=5, seed=3)
    f = p.loads[0].copy()
    free = np.flatnonzero(p.fixed_mask == 0)
    f[free[len(free) // 2]] = np.nan
    g = Grid.from_problem(p)
    u = torch.zeros(p.ndof, dtype=dtype, device=DEV)
    info = torch.zeros(8, dtype=torch.float64, device=DEV)
    g.inner_solve(dev(synth.uniform_density(p.E, 1), dtype), dev(f, dtype), u, 5, info=info)
    assert host(info)[4] == 6.0
    x = dev(oracle.project_volume_ref(p.x0, 0.0, 1.0, p.vmax), dtype)
    u.zero_()
    g.outer_step(x, u, dev(f, dtype), 1, 1e-3, 5, 0.0, p.vmax, info=info)
    assert host(info)[6] == 6.0


@pytest.mark.parametrize("tile", [(11, 20, 5, 0), (32, 6, 3, 2), (16, 8, 9, 3), (50, 4, 1, 0)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_pcg_tile_override_matches_oracle(tile, dtype):
    """Tile shapes, slab depths and block caps set by fbto_set_option change
    the layout of the z-march only: the PCG iterate still follows the
    oracle's recurrence (a grid of several tiles and slabs, ragged in x, y
    and z for every shape)."""
    bx, by, dz, cap = tile
    say(f"pcg tile {tile} {dtype}")
    p = synth.cantilever(45, 14, 10, volfrac=0.3, filter_radius=1.5, outer_iters=1, inner_steps=5, seed=6)
    og, g, rho_t, s, K, D = _setup(p, dtype, 6)
    value = bx | (by << 8) | (dz << 16) | (cap << 24)
    g.set_option("cgf_tile", value)
    g.set_option("apply_tile", value)
    f = p.loads[0]
    u_t = torch.zeros(p.ndof, dtype=dtype, device=DEV)
    info = torch.zeros(8, dtype=torch.float64, device=DEV)
    m = 7
    g.inner_solve(rho_t, dev(f, dtype), u_t, m, info=info)
    u_ref, r_ref = oracle.pcg_ref(lambda v: K @ v, D, f, np.zeros(p.ndof), m)
    tol = 1e-10 if dtype == torch.float64 else 2e-4
    assert np.abs(host(u_t) - u_ref).max() <= tol * np.abs(u_ref).max()
    assert host(info)[3] == m


def test_tile_option_limits():
    from paper_2204_06204_amd._lib import FbtoError
    p = synth.cantilever(8, 4, 4, volfrac=0.3, filter_radius=1.5, outer_iters=1, inner_steps=2, seed=1)
    from paper_2204_06204_amd.grid import Grid
    g = Grid.from_problem(p)
    # (bx + 1)(by + 1) threads must lie in 128 .. 256
    for bad in (7, 65, 8 | (4 << 8), 16 | (16 << 8), 16 | (65 << 8), 15 | (15 << 8) | (65 << 16), 1 << 24,
                1 << 28, -1):
        with pytest.raises(FbtoError):
            g.set_option("cgf_tile", bad)
    g.set_option("cgf_tile", 15 | (15 << 8) | (4 << 16) | (2 << 24))
    g.close()


@pytest.mark.parametrize("tile", [(11, 20, 5), (32, 6, 3), (16, 8, 9)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_krylov_step_tile_override_matches_oracle(tile, dtype):
    """The fused MINRES steps (one thread per node column) and the residual
    kernels (one per element column) under tile overrides on a ragged grid:
    the Krylov step still equals the oracle's."""
    bx, by, dz = tile
    say(f"krylov tile {tile} {dtype}")
    p = synth.cantilever(45, 14, 10, volfrac=0.3, filter_radius=1.5, outer_iters=1, inner_steps=5, seed=6)
    og, g, rho_t, s, K, D = _setup(p, dtype, 6)
    g.set_option("apply_tile", bx | (by << 8) | (dz << 16))
    f = p.loads[0]
    u0 = np.zeros(p.ndof)
    deg = 6
    u_t = dev(u0, dtype)
    g.inner_solve(rho_t, dev(f, dtype), u_t, deg, method="krylov", omega=1.0)
    u_ref, _ = oracle.krylov_step_ref(lambda v: K @ v, f, u0, deg)
    tol = 1e-9 if dtype == torch.float64 else 3e-4
    assert np.abs(host(u_t) - u_ref).max() <= tol * np.abs(u_ref).max()
