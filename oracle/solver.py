"""BiCGStab for the shifted systems (D + sigma I) x = b (oracle).

The paper solves (D + s_i I) x = z and the adjoint system (Sec. 3.1, eqs.
shifted_linear_systems and conj_shifted_linear_systems) with a multigrid
solver; this build uses BiCGStab (van der Vorst, SIAM J. Sci. Stat. Comput.
13 (1992) 631) in the textbook form below, with the stop criterion taken on
the true residual ||b - A x|| / ||b|| <= tol, recomputed at exit.

The adjoint solution uses gamma_5-hermiticity of the Wilson operator
(D^dagger = g5 D g5, so (D + sigma)^-dagger z = g5 (D + sigma)^-1 g5 z).

Parity: pinned against dense LU solves (scipy) on small lattices.
"""

import numpy as np


def _dot(a, b):
    return np.vdot(a.ravel(), b.ravel())


def bicgstab(apply_A, b, tol=1e-12, max_iter=10000, x0=None):
    """Solve A x = b.  Returns (x, info) with info = dict(iters, true_rel, restarts)."""
    b = np.asarray(b, dtype=np.complex128)
    bnorm = np.sqrt(_dot(b, b).real)
    if bnorm == 0.0:
        return np.zeros_like(b), dict(iters=0, true_rel=0.0, restarts=0)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    r = b - apply_A(x)
    iters = 0
    restarts = 0
    while True:
        rhat = r.copy()
        rho = _dot(rhat, r)
        p = r.copy()
        while iters < max_iter:
            v = apply_A(p)
            rv = _dot(rhat, v)
            if rv == 0:
                break
            alpha = rho / rv
            s = r - alpha * v
            t = apply_A(s)
            tt = _dot(t, t).real
            omega = _dot(t, s) / tt if tt > 0 else 0.0
            x = x + alpha * p + omega * s
            r = s - omega * t
            iters += 1
            rr = np.sqrt(_dot(r, r).real)
            if rr <= tol * bnorm or omega == 0:
                break
            rho_new = _dot(rhat, r)
            beta = (rho_new / rho) * (alpha / omega)
            rho = rho_new
            p = r + beta * (p - omega * v)
        r = b - apply_A(x)
        true_rel = np.sqrt(_dot(r, r).real) / bnorm
        if true_rel <= tol or iters >= max_iter or restarts >= 20:
            return x, dict(iters=iters, true_rel=true_rel, restarts=restarts)
        restarts += 1
