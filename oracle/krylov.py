"""Right-preconditioned Krylov solvers (oracle).

The paper names GMRES (Saad-Schultz) and BiCGStab (van der Vorst) as the
Krylov backbones that the trunk-basis preconditioner accelerates (§3.1.2,
§4).  It prints no algorithmic detail, so the following readings are fixed
here and followed identically by the GPU library:

* right preconditioning, u0 given (zero in the workloads), stopping on the
  true unpreconditioned residual ||f - A u||_2 <= tol ||f||_2; with f = 0
  the relative residual is undefined and the residual is measured in
  absolute terms (scale 1 instead of ||f||_2);
* GMRES(m): classical Gram-Schmidt, one projection (PETSc's default) or two
  (CGS2, one full re-orthogonalisation); complex Givens rotations
  G = [[c, s], [-conj(s), c]] with real c; the iteration count is the total
  number of Arnoldi steps over restarts;
* BiCGStab: shadow vector r_hat = r0, early exit on ||s||, one count per
  iteration, breakdown on an exactly zero or non-finite rho, r_hat^H v or
  omega; if the recomputed true residual misses the tolerance after the
  recursive one met it, the method restarts with r_hat = r.

Vectors are flat complex128 arrays; ``A`` and ``M`` are callables.
Inner products are <x, y> = sum conj(x_i) y_i.
"""
from __future__ import annotations

import numpy as np

CONVERGED, NOT_CONVERGED, BREAKDOWN, NONFINITE = 0, 1, -4, -5


def _identity(v):
    return v


def givens(a: complex, b: float):
    """Rotation (c, s) that maps (a, b), b real >= 0, to (nu * a/|a|, 0)."""
    if b == 0.0:
        return 1.0, 0.0 + 0.0j
    if a == 0:
        return 0.0, 1.0 + 0.0j
    nu = np.sqrt(abs(a) ** 2 + b * b)
    return abs(a) / nu, (a / abs(a)) * (b / nu)


def back_substitute(H, g, k):
    """Solve the upper-triangular k x k system H[:k, :k] y = g[:k]."""
    y = np.zeros(k, dtype=np.complex128)
    for i in range(k - 1, -1, -1):
        y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
    return y


def gmres(A, f, u0, restart, tol, max_iters, M=None, history=None, gs_passes=2):
    """Restarted, right-preconditioned GMRES(m).  The new Arnoldi vector is
    orthogonalized by classical Gram-Schmidt: gs_passes = 2 projects twice
    (CGS2, one full re-orthogonalization), gs_passes = 1 once (the default of
    PETSc's GMRES, the solver library of the paper's experiments, section 4).

    Returns (u, info) with info = dict(status, iters, rel_res, matvecs,
    precond_apps)."""
    if gs_passes not in (1, 2):
        raise ValueError("gs_passes must be 1 or 2")
    has_m = M is not None
    M = M or _identity
    f = np.asarray(f, dtype=np.complex128)
    u = np.array(u0, dtype=np.complex128)
    fn = np.linalg.norm(f)
    fs = fn if fn > 0 else 1.0  # residual scale
    count = matvecs = papps = 0
    status = NOT_CONVERGED
    while True:
        r = f - A(u)
        matvecs += 1
        beta = np.linalg.norm(r)
        if history is not None and not history:
            history.append(beta / fs)
        if not np.isfinite(beta):
            status = NONFINITE
            break
        if beta <= tol * fs:
            status = CONVERGED
            break
        if count >= max_iters:
            break
        m = restart
        V = np.zeros((m + 1, f.size), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        V[0] = r / beta
        g[0] = beta
        k = 0
        for j in range(m):
            z = M(V[j])
            w = A(z)
            papps += has_m
            matvecs += 1
            Vj = V[: j + 1]
            h = Vj.conj() @ w
            w = w - Vj.T @ h
            if gs_passes == 2:
                h2 = Vj.conj() @ w
                w = w - Vj.T @ h2
                h = h + h2
            hn = np.linalg.norm(w)
            H[: j + 1, j] = h
            H[j + 1, j] = hn
            if hn != 0.0:
                V[j + 1] = w / hn
            for i in range(j):
                a, b = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * b
                H[i + 1, j] = -np.conj(sn[i]) * a + cs[i] * b
            c, s = givens(H[j, j], float(hn))
            cs[j], sn[j] = c, s
            H[j, j] = c * H[j, j] + s * hn
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(s) * g[j]
            g[j] = c * g[j]
            count += 1
            k = j + 1
            if history is not None:
                history.append(abs(g[j + 1]) / fs)
            if abs(g[j + 1]) <= tol * fs or count >= max_iters or hn == 0.0:
                break
        y = back_substitute(H, g, k)
        u = u + M(V[:k].T @ y)
        papps += has_m
    rel = np.linalg.norm(f - A(u)) / fs
    return u, dict(status=status, iters=count, rel_res=rel, matvecs=matvecs, precond_apps=papps)


def bicgstab(A, f, u0, tol, max_iters, M=None, history=None):
    """Right-preconditioned BiCGStab (van der Vorst)."""
    has_m = M is not None
    M = M or _identity
    f = np.asarray(f, dtype=np.complex128)
    u = np.array(u0, dtype=np.complex128)
    fn = np.linalg.norm(f)
    fs = fn if fn > 0 else 1.0  # residual scale
    count = matvecs = papps = 0
    status = NOT_CONVERGED
    r = f - A(u)
    matvecs += 1
    rn = np.linalg.norm(r)
    if history is not None:
        history.append(rn / fs)
    if not np.isfinite(rn):
        return u, dict(status=NONFINITE, iters=0, rel_res=np.inf, matvecs=matvecs, precond_apps=0)
    if rn <= tol * fs:
        return u, dict(status=CONVERGED, iters=0, rel_res=rn / fs,
                       matvecs=matvecs, precond_apps=0)
    while True:
        # one restartable sweep of the recurrence
        rhat = r.copy()
        rho0 = alpha = omega = 1.0 + 0j
        v = np.zeros_like(r)
        p = np.zeros_like(r)
        stopped = False
        while count < max_iters:
            rho = np.vdot(rhat, r)
            if rho == 0 or not np.isfinite(rho):
                status = BREAKDOWN if np.isfinite(rho) else NONFINITE
                stopped = True
                break
            beta = (rho / rho0) * (alpha / omega)
            p = r + beta * (p - omega * v)
            ph = M(p)
            v = A(ph)
            papps += has_m
            matvecs += 1
            den = np.vdot(rhat, v)
            if den == 0 or not np.isfinite(den):
                status = BREAKDOWN if np.isfinite(den) else NONFINITE
                stopped = True
                break
            alpha = rho / den
            s = r - alpha * v
            count += 1
            sn = np.linalg.norm(s)
            if sn <= tol * fs:
                u = u + alpha * ph
                if history is not None:
                    history.append(sn / fs)
                break
            sh = M(s)
            t = A(sh)
            papps += has_m
            matvecs += 1
            tt = np.vdot(t, t).real
            omega = np.vdot(t, s) / tt if tt != 0 else 0.0
            if omega == 0 or not np.isfinite(omega):
                status = BREAKDOWN if np.isfinite(omega) else NONFINITE
                stopped = True
                break
            u = u + alpha * ph + omega * sh
            r = s - omega * t
            rho0 = rho
            rn = np.linalg.norm(r)
            if history is not None:
                history.append(rn / fs)
            if rn <= tol * fs:
                break
        if stopped:
            break
        r = f - A(u)
        matvecs += 1
        rn = np.linalg.norm(r)
        if not np.isfinite(rn):
            status = NONFINITE
            break
        if rn <= tol * fs:
            status = CONVERGED
            break
        if count >= max_iters:
            status = NOT_CONVERGED
            break
    rel = np.linalg.norm(f - A(u)) / fs
    return u, dict(status=status, iters=count, rel_res=rel, matvecs=matvecs, precond_apps=papps)
