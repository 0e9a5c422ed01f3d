"""Low-level (displacement) solves (oracle, FP64).

The low-level problem of the bilevel program (Eq. optBilevel, Sec. 4) is
u = argmin 1/2 u^T K u - f^T u, i.e. K u = f.  Alg. 1 refines u by one
gradient step per outer iteration, u <- u - beta (K u - f); Alg. 3 adds a
preconditioner commuting with K.  The inner step used here is a few steps of
Jacobi-preconditioned conjugate gradients, restarted each outer iteration
and warm-started from the previous displacement (the Jacobi preconditioner
is among the lightweight preconditioners Sec. 4.1 names).  The plain
gradient step of Alg. 1 and a damped Jacobi step are kept as variants, and
Alg. 3's step with the Krylov preconditioner of Eq. LSP (krylov_step_ref).

``operator`` arguments are callables u -> K_bc u (CSR matvec or the element
loop), so that every solver here is a textbook recurrence over a black box.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla


def solve_direct(K, f):
    """Exact u = K^{-1} f by sparse LU (SuperLU)."""
    return spla.spsolve(K.tocsc(), f)


def pcg_ref(apply, diag, f, u0, steps, *, history=False):
    """`steps` iterations of Jacobi-preconditioned CG from the warm start u0
    (no early exit).  Returns (u, r) where r is the recursively updated
    residual; with history=True also the list of iterates u_1..u_m.

        r = f - K u ; z = D^-1 r ; p = z
        repeat: q = K p ; alpha = r.z / p.q ; u += alpha p ; r -= alpha q
                z = D^-1 r ; beta = r.z(new) / r.z(old) ; p = z + beta p
    """
    u = np.array(u0, dtype=np.float64, copy=True)
    r = f - apply(u)
    z = r / diag
    p = z.copy()
    rz = float(r @ z)
    its = []
    for _ in range(steps):
        q = apply(p)
        pq = float(p @ q)
        if pq <= 0.0:
            raise FloatingPointError("CG breakdown: p^T K p <= 0")
        alpha = rz / pq
        u = u + alpha * p
        r = r - alpha * q
        z = r / diag
        rz_new = float(r @ z)
        beta = rz_new / rz if rz != 0.0 else 0.0
        p = z + beta * p
        rz = rz_new
        if history:
            its.append(u.copy())
    return (u, r, its) if history else (u, r)


def richardson_ref(apply, f, u0, steps, beta):
    """Alg. 1's low-level update u <- u - beta (K u - f), `steps` times."""
    u = np.array(u0, dtype=np.float64, copy=True)
    for _ in range(steps):
        u = u - beta * (apply(u) - f)
    return u, f - apply(u)


def damped_jacobi_ref(apply, diag, f, u0, steps, omega):
    """u <- u - omega D^-1 (K u - f), `steps` times."""
    u = np.array(u0, dtype=np.float64, copy=True)
    for _ in range(steps):
        u = u - omega * (apply(u) - f) / diag
    return u, f - apply(u)


def krylov_step_ref(apply, f, u0, D, beta=1.0):
    """One low-level step of Alg. 3 (CPFBTO) with the Krylov preconditioner
    of Eq. LSP (Sec. 4.1):

        delta = K u - f
        c*    = argmin_c || delta - sum_{i=1}^{D+1} c_{i-1} K^i delta ||
        M^-1 delta = sum_{i=0}^{D} c*_i K^i delta
        u    <- u - beta M^-1 delta

    The least-squares problem is solved as the paper does, by Householder QR
    of the monomial Krylov matrix [K delta, ..., K^(D+1) delta] (LAPACK's
    geqrf behind numpy.linalg.qr).  With beta = 1 the new residual is the
    smallest over u + span{delta, ..., K^D delta}: one GMRES(D + 1) cycle.
    Returns (u_new, f - K u_new)."""
    u = np.array(u0, dtype=np.float64, copy=True)
    delta = apply(u) - f
    cols = []
    v = delta
    for _ in range(D + 1):
        v = apply(v)
        cols.append(v)
    A = np.stack(cols, axis=1)
    Q, R = np.linalg.qr(A)
    c = np.linalg.solve(R, Q.T @ delta)
    minv = np.zeros_like(u)
    v = delta
    for i in range(D + 1):
        minv += c[i] * v
        v = apply(v)
    u = u - beta * minv
    return u, f - apply(u)


def pcg_to_tol(apply, diag, f, u0, rtol, max_steps=100000):
    """Jacobi-PCG until ||r||_2 <= rtol ||f||_2 (recursive residual), then one
    true residual.  Returns (u, true_residual_norm_ratio, steps)."""
    u = np.array(u0, dtype=np.float64, copy=True)
    r = f - apply(u)
    z = r / diag
    p = z.copy()
    rz = float(r @ z)
    fn = float(np.linalg.norm(f))
    it = 0
    while np.linalg.norm(r) > rtol * fn and it < max_steps:
        q = apply(p)
        alpha = rz / float(p @ q)
        u += alpha * p
        r -= alpha * q
        z = r / diag
        rz_new = float(r @ z)
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
    true = np.linalg.norm(f - apply(u)) / fn
    return u, true, it
