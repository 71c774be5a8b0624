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


def bicgstab_multishift(apply_A, b, shifts, tol=1e-12, max_iter=10000, trace=None):
    """Solve (A + sigma_k) x_k = b for every sigma_k in shifts from one Krylov space.

    Multi-shift BiCGStab (the shifted-system form of van der Vorst's method, as in
    Jegerlehner's "Krylov space solvers for shifted linear systems" and Frommer's
    shifted BiCGStab).  The base iteration is the textbook one on A + sigma_0
    (sigma_0 = shifts[0], the slowest system when the shifts increase); every other
    system k, with relative shift d = sigma_k - sigma_0, reuses its vectors:

    * BiCG part: the shifted BiCG residuals are zeta_n times the base ones, with
        zeta_{n+1} = zeta_n zeta_{n-1} alpha_{n-1} /
                     (zeta_{n-1} alpha_{n-1} (1 + alpha_n d) + alpha_n beta_{n-1} (zeta_{n-1} - zeta_n)),
      alpha^d_n = alpha_n zeta_{n+1} / zeta_n, beta^d_n = (zeta_{n+1} / zeta_n)^2 beta_n
      (zeta_0 = zeta_{-1} = 1, beta_{-1} = 0);
    * stabiliser: omega^d_n = omega_n / (1 + omega_n d), so that
      1 - omega^d (A + d) = (1 - omega A) / (1 + omega d); with tau_n =
      prod_{j<n} (1 + omega_j d) the shifted residual and s-vector are
      r^d_n = (zeta_n / tau_n) r_n and s^d_n = (zeta_{n+1} / tau_n) s_n;
    * updates: x^d += alpha^d_n p^d_n + omega^d_n s^d_n and
      p^d_{n+1} = r^d_{n+1} + beta^d_n (p^d_n - (omega^d_n / alpha^d_n)(r^d_n - s^d_n)),
      where (A + d) p^d_n = (r^d_n - s^d_n) / alpha^d_n needs no operator application.

    A system stops updating once its residual estimate |zeta/tau| ||r_n|| reaches
    tol ||b||; the base stops at its own.  No restarts (they would break the
    recurrences).  Returns (xs, info) with info = dict(iters, true_rel[k]) from the
    true residuals recomputed at exit.  trace, if a list, receives per iteration
    the pairs (r_n, [r^d_n]) for the collinearity check in the tests.
    """
    b = np.asarray(b, dtype=np.complex128)
    shifts = list(shifts)
    m = len(shifts)
    s0 = shifts[0]
    d = [s - s0 for s in shifts]
    bnorm = np.sqrt(_dot(b, b).real)

    def A0(v):
        return apply_A(v) + s0 * v

    xs = [np.zeros_like(b) for _ in range(m)]
    if bnorm == 0.0:
        return xs, dict(iters=0, true_rel=[0.0] * m)
    r = b.copy()
    rhat = b.copy()
    p = b.copy()
    ps = [b.copy() for _ in range(m)]
    zeta_prev = [1.0 + 0j] * m
    zeta = [1.0 + 0j] * m
    tau = [1.0 + 0j] * m
    alpha_prev, beta_prev = 1.0 + 0j, 0.0 + 0j
    rho = _dot(rhat, r)
    done = [False] * m
    iters = 0
    while iters < max_iter and not done[0]:
        v = A0(p)
        alpha = rho / _dot(rhat, v)
        s = r - alpha * v
        t = A0(s)
        omega = _dot(t, s) / _dot(t, t).real
        r_new = s - omega * t
        rho_new = _dot(rhat, r_new)
        beta = (rho_new / rho) * (alpha / omega)
        xs[0] = xs[0] + alpha * p + omega * s
        rr = np.sqrt(_dot(r_new, r_new).real)
        shifted_r = []
        for k in range(1, m):
            if done[k]:
                shifted_r.append(None)
                continue
            dk = d[k]
            zn, zp = zeta[k], zeta_prev[k]
            z_next = zn * zp * alpha_prev / (zp * alpha_prev * (1.0 + alpha * dk) + alpha * beta_prev * (zp - zn))
            a_k = alpha * z_next / zn
            w_k = omega / (1.0 + omega * dk)
            b_k = (z_next / zn) ** 2 * beta
            tau_next = tau[k] * (1.0 + omega * dk)
            r_k = (zn / tau[k]) * r            # r^d_n
            s_k = (z_next / tau[k]) * s        # s^d_n
            xs[k] = xs[k] + a_k * ps[k] + w_k * s_k
            ps[k] = (z_next / tau_next) * r_new + b_k * (ps[k] - (w_k / a_k) * (r_k - s_k))
            shifted_r.append((zn / tau[k]) * r)
            zeta_prev[k], zeta[k], tau[k] = zn, z_next, tau_next
            if abs(z_next / tau_next) * rr <= tol * bnorm:
                done[k] = True
        if trace is not None:
            trace.append((r.copy(), shifted_r))
        p = r_new + beta * (p - omega * v)
        r = r_new
        rho = rho_new
        alpha_prev, beta_prev = alpha, beta
        iters += 1
        if rr <= tol * bnorm:
            done[0] = True
    true_rel = []
    for k in range(m):
        res = b - apply_A(xs[k]) - shifts[k] * xs[k]
        true_rel.append(float(np.sqrt(_dot(res, res).real) / bnorm))
    return xs, dict(iters=iters, true_rel=true_rel)
