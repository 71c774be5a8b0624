"""Frequency-Splitting MLMC estimator of Tr(Gamma_n Omega_p D^-1) (oracle).

Paper Sec. 2.2 (eq. tele_sum_prod_disp) splits the target into levels,
with 0 = sigma_0 < sigma_1 < ... < sigma_L:

  level l < L:  A_l = (sigma_{l+1} - sigma_l) (D + sigma_l)^-1 Gamma Omega_p (D + sigma_{l+1})^-1
  level L:      A_L = Gamma Omega_p (D + sigma_L)^-1

and Tr(Gamma Omega_p D^-1) = sum_l Tr(A_l).  Each level is estimated with
independent Z4 noise (eq. fs_trace_est):  X_s = z_s^dagger A_l z_s, i.e.

  level l < L:  x = (D + sigma_{l+1})^-1 z,  y = (D + sigma_l)^-dagger z
                  = g5 (D + sigma_l)^-1 g5 z,    X = (sigma_{l+1}-sigma_l) y^dagger Gamma Omega_p x
  level L:      x = (D + sigma_L)^-1 z,           X = z^dagger Gamma Omega_p x

Per level the mean t = (1/N) sum X_s and the variance of eq.
practical_variance, (1/N) sum |X_s|^2 - |t|^2, are reported, with the
(N-1)-normalised form beside it.

Readings (listed in the design notes): the estimator sums N_l samples
s = 1..N_l (the printed range 0..N_l has one term too many); noise for
(level l, sample s) is the Z4 vector keyed by (seed, instance, l, s); for Z4
noise the exact variance of one sample is ||A||_F^2 - sum |A_ii|^2 (the factor
2 printed in eq. test_var belongs to real +-1 noise).

Parity: the exact traces are pinned by free-field closed forms and the
telescoping identity; the variance formula by exhaustive Z4 enumeration; the
stochastic estimates by unbiasedness against the exact values.
"""

import numpy as np
import scipy.linalg as sla

from . import clover, lattice as lat
from .philox import z4_noise
from .solver import bicgstab


# ---------------------------------------------------------------------------
# Solve back-ends: dense LU (tiny lattices) or matrix-free BiCGStab.
# ---------------------------------------------------------------------------

class DenseSolver:
    """(D + sigma)^-1 via one LU factorisation per shift (scipy); with c_sw != 0
    D is the clover-improved operator of oracle.clover."""

    def __init__(self, U, dims, m0, antiperiodic=False, c_sw=0.0):
        self.U, self.dims, self.m0, self.ap, self.c_sw = U, dims, m0, antiperiodic, c_sw
        if c_sw == 0.0:
            self.D0 = lat.wilson_dense(U, m0, 0.0, dims, antiperiodic)
        else:
            self.D0 = clover.clover_dense(U, m0, 0.0, c_sw, dims, antiperiodic)
        self._lu = {}

    def _factor(self, sigma):
        if sigma not in self._lu:
            A = self.D0 + sigma * np.eye(self.D0.shape[0])
            self._lu[sigma] = sla.lu_factor(A)
        return self._lu[sigma]

    def solve(self, sigma, b):
        shape = b.shape
        return sla.lu_solve(self._factor(sigma), b.reshape(-1)).reshape(shape)

    def inverse(self, sigma):
        n = self.D0.shape[0]
        return sla.lu_solve(self._factor(sigma), np.eye(n, dtype=np.complex128))


class IterativeSolver:
    """(D + sigma)^-1 b via the oracle BiCGStab on the matrix-free operator."""

    def __init__(self, U, dims, m0, antiperiodic=False, tol=1e-13, c_sw=0.0):
        self.U, self.dims, self.m0, self.ap, self.tol, self.c_sw = U, dims, m0, antiperiodic, tol, c_sw
        self.C = clover.clover_term(U, dims, c_sw) if c_sw != 0.0 else None
        self.last_info = None

    def solve(self, sigma, b):
        def A(v):
            if self.C is not None:
                return clover.clover_apply(self.U, v, self.m0, sigma, self.c_sw, self.dims, self.ap, C=self.C)
            return lat.wilson_apply(self.U, v, self.m0, sigma, self.dims, self.ap)
        x, info = bicgstab(A, b, tol=self.tol)
        self.last_info = info
        return x


# ---------------------------------------------------------------------------
# Bilinears y^dagger Gamma_n Omega_p x
# ---------------------------------------------------------------------------

def bilinears(U, dims, y, x, gammas, p_max):
    """X[n_idx, p] = y^dagger Gamma_n Omega_p x, written from the definition."""
    out = np.zeros((len(gammas), p_max + 1), dtype=np.complex128)
    phi = np.asarray(x, dtype=np.complex128)
    for p in range(p_max + 1):
        if p > 0:
            phi = lat.displace(U, phi, 1, dims)  # Omega_p = (one hop)^p
        for i, n in enumerate(gammas):
            out[i, p] = np.vdot(y.ravel(), lat.apply_gamma(n, phi).ravel())
    return out


def level_vectors(solver, sigmas, level, z):
    """(coef, y, x) with X = coef * y^dagger Gamma Omega_p x for this level."""
    L = len(sigmas) - 1
    if level < L:
        x = solver.solve(sigmas[level + 1], z)
        y = lat.apply_gamma5(solver.solve(sigmas[level], lat.apply_gamma5(z)))
        return sigmas[level + 1] - sigmas[level], y, x
    x = solver.solve(sigmas[L], z)
    return 1.0, z, x


def fs_samples(U, dims, sigmas, n_noise, seed, gammas, p_max, solver,
               instance=0, levels=None, samples=None, shared_noise=False):
    """Per-sample estimates X[l, s, n_idx, p] with independent noise per level
    (eq. fs_trace_est), or with one noise vector z_s for every level
    (shared_noise: the key of level 0), as the sampling algorithm of Sec. 3.1
    shares its noise across shifts."""
    L = len(sigmas) - 1
    V = lat.volume(dims)
    levels = range(L + 1) if levels is None else levels
    samples = range(n_noise) if samples is None else samples
    X = np.zeros((L + 1, len(samples), len(gammas), p_max + 1), dtype=np.complex128)
    for l in levels:
        for j, s in enumerate(samples):
            z = z4_noise(V, seed, instance, 0 if shared_noise else l, s)
            coef, y, x = level_vectors(solver, sigmas, l, z)
            X[l, j] = coef * bilinears(U, dims, y, x, gammas, p_max)
    return X


def level_stats(X, axis=1):
    """Mean and variances over the sample axis (eq. practical_variance)."""
    N = X.shape[axis]
    t = X.mean(axis=axis)
    var_paper = (np.abs(X) ** 2).mean(axis=axis) - np.abs(t) ** 2
    var_unbiased = var_paper * N / (N - 1) if N > 1 else np.full_like(var_paper, np.nan)
    return t, var_paper, var_unbiased


def optimal_samples(V, C, eps2):
    """Eq. num_samples: real-valued N_l = mu sqrt(V_l / C_l) with
    mu = eps^-2 sum_l sqrt(V_l C_l) (the Lagrange solution of: least
    sum_l C_l N_l subject to sum_l V_l / N_l = eps^2).  Returns (N, mu)."""
    V = np.asarray(V, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    mu = np.sum(np.sqrt(V * C)) / eps2
    return mu * np.sqrt(V / C), mu


def fs_combine(t_levels, var_levels, n_levels):
    """Total estimate sum_l t_l, V_FS = sum_l V_l / N_l (eq. total_var), V_total = sum_l V_l (eq. tosv)."""
    t_levels = np.asarray(t_levels)
    var_levels = np.asarray(var_levels)
    n_levels = np.asarray(n_levels, dtype=np.float64)
    shape = (-1,) + (1,) * (var_levels.ndim - 1)
    return (t_levels.sum(axis=0),
            (var_levels / n_levels.reshape(shape)).sum(axis=0),
            var_levels.sum(axis=0))


# ---------------------------------------------------------------------------
# Exact level quantities (dense, tiny lattices)
# ---------------------------------------------------------------------------

def offdiag_frobenius(A):
    """||A||_F^2 - sum_i |A_ii|^2: exact one-sample variance for Z4 noise."""
    return float(np.sum(np.abs(A) ** 2) - np.sum(np.abs(np.diag(A)) ** 2))


def level_matrix(inv_lo, inv_hi, G, coef):
    """coef * inv_lo @ G @ inv_hi (inv_lo = None for the last level)."""
    B = G @ inv_hi
    return coef * (B if inv_lo is None else inv_lo @ B)


def exact_levels(solver, sigmas, gammas, p_list, with_variance=True):
    """Exact T_l and V_l per (level, Gamma_n, p): arrays of shape (L+1, nG, nP)."""
    U, dims = solver.U, solver.dims
    V = lat.volume(dims)
    L = len(sigmas) - 1
    invs = [solver.inverse(s) for s in sigmas]
    T = np.zeros((L + 1, len(gammas), len(p_list)), dtype=np.complex128)
    Var = np.zeros((L + 1, len(gammas), len(p_list)))
    for ip, p in enumerate(p_list):
        Om = lat.omega_dense(U, p, dims)
        for ig, n in enumerate(gammas):
            G = lat.gamma_dense(n, V) @ Om
            for l in range(L + 1):
                if l < L:
                    A = level_matrix(invs[l], invs[l + 1], G, sigmas[l + 1] - sigmas[l])
                else:
                    A = level_matrix(None, invs[L], G, 1.0)
                T[l, ig, ip] = np.trace(A)
                if with_variance:
                    Var[l, ig, ip] = offdiag_frobenius(A)
    return T, Var


def exact_trace(solver, sigma, n, p):
    """Tr(Gamma_n Omega_p (D + sigma)^-1) from the dense inverse."""
    V = lat.volume(solver.dims)
    G = lat.gamma_dense(n, V) @ lat.omega_dense(solver.U, p, solver.dims)
    return np.trace(G @ solver.inverse(sigma))


# ---------------------------------------------------------------------------
# Variance sampling (Sec. 3.1, subsection "Sampling the Variance")
# ---------------------------------------------------------------------------

# Level field of the noise key used by the sampling phase: one Z4 vector z_k
# per sample, shared by every sampling shift and independent of the
# estimation noise (whose level fields are 0..L).
SAMPLING_LEVEL = 0xFFFFFFFF


def sampling_slots(m):
    """Order of the sampled quantities: V_L(s_i) for i = 0..m-1, then
    Vbar_l(s_i, s_j) for i = 0..m-1, j = i..m-1."""
    return [("single", i, i) for i in range(m)] + [("pair", i, j) for i in range(m) for j in range(i, m)]


# ---------------------------------------------------------------------------
# Generalized Hopping Parameter Expansion (Sec. 3.1, closing paragraph of
# "Sampling the Variance"): with D + sigma = a - H, a = 4 + m0 + sigma and H
# the hopping term,
#   (D + sigma)^-1 = sum_{j<k} (H/a)^j / a + (H/a)^k (D + sigma)^-1,
# so the trace of Gamma Omega_p (D + sigma)^-1 is the trace of the first k
# terms (computable exactly) plus that of Gamma Omega_p (H/a)^k (D + sigma)^-1,
# whose stochastic estimate has the smaller variance when m0 + sigma is large.
# The paper samples V_L that way at order k = 4 for the shifts with
# m0 + s > 0.  With the clover term the expansion is the generalized one:
# D_sw + sigma = A - H with the site-local A = C + a, and (H/a) becomes A^-1 H.
# ---------------------------------------------------------------------------

def hopping_apply(U, psi, m0, sigma, dims, antiperiodic=False):
    """H psi with D + sigma = (4 + m0 + sigma) - H (H depends on neither m0 nor sigma)."""
    return (4.0 + m0 + sigma) * np.asarray(psi, np.complex128) - lat.wilson_apply(U, psi, m0, sigma, dims,
                                                                                  antiperiodic)


def hpe_apply(U, x, m0, sigma, k, dims, antiperiodic=False, C=None):
    """(H / a)^k x, a = 4 + m0 + sigma; with the clover term C (per site, (V, 12, 12))
    the generalized (A^-1 H)^k x, A = C + a.  H is the hopping term either way."""
    a = 4.0 + m0 + sigma
    w = np.asarray(x, np.complex128)
    if C is not None:
        A = C + a * np.eye(12)
    for _ in range(k):
        h = hopping_apply(U, w, m0, sigma, dims, antiperiodic)
        if C is None:
            w = h / a
        else:
            V = A.shape[0]
            w = np.linalg.solve(A, h.reshape(V, 12, 1)).reshape(h.shape)
    return w


def hpe_eligible(m0, s):
    """The sampling shifts the expansion is used for (m_q + s > 0 in the paper's notation)."""
    return m0 + s > 0.0


def sampling_samples(U, dims, shifts, n_samples, seed, gammas, p_max, solver, instance=0, hpe_order=0):
    """Per-sample values of the sampling algorithm, X[slot, k, n_idx, p].

    For each noise vector z_k and each sampling shift s_i: x_i = (D+s_i)^-1 z_k
    and y_i = (D+s_i)^-dagger z_k = g5 (D+s_i)^-1 g5 z_k (the second solve
    for non-diluted noise).  Then V_L(s_i) samples z_k^dagger Gamma Omega_p x_i
    (A = Gamma Omega_p (D+s_i)^-1) and Vbar_l(s_i, s_j), j >= i, samples
    y_i^dagger Gamma Omega_p x_j (A = (D+s_i)^-1 Gamma Omega_p (D+s_j)^-1),
    without the (s_j - s_i)^2 factor of V_l (eq. sampled_prod, eq. bar_vl).
    With hpe_order = k > 0 the V_L samples of the shifts with m0 + s_i > 0
    are z_k^dagger Gamma Omega_p (H/a_i)^k x_i (the expansion's remainder).
    """
    C = clover.clover_term(U, dims, solver.c_sw) if getattr(solver, "c_sw", 0.0) != 0.0 and hpe_order > 0 else None
    m = len(shifts)
    V = lat.volume(dims)
    slots = sampling_slots(m)
    X = np.zeros((len(slots), n_samples, len(gammas), p_max + 1), dtype=np.complex128)
    for k in range(n_samples):
        z = z4_noise(V, seed, instance, SAMPLING_LEVEL, k)
        xs = [solver.solve(s, z) for s in shifts]
        ys = [lat.apply_gamma5(solver.solve(s, lat.apply_gamma5(z))) for s in shifts]
        for q, (kind, i, j) in enumerate(slots):
            y = z if kind == "single" else ys[i]
            x = xs[j]
            if kind == "single" and hpe_order > 0 and hpe_eligible(solver.m0, shifts[j]):
                x = hpe_apply(U, x, solver.m0, shifts[j], hpe_order, dims, solver.ap, C=C)
            X[q, k] = bilinears(U, dims, y, x, gammas, p_max)
    return X


def exact_sampling(solver, shifts, gammas, p_list, hpe_order=0):
    """Exact traces and one-sample variances of every sampled matrix, per slot
    (with hpe_order as in sampling_samples: the singles of eligible shifts are
    Gamma Omega_p (H/a)^k (D + s)^-1)."""
    U, dims = solver.U, solver.dims
    V = lat.volume(dims)
    m = len(shifts)
    invs = [solver.inverse(s) for s in shifts]
    singles = list(invs)
    if hpe_order > 0:
        n = solver.D0.shape[0]
        Ad = (4.0 + solver.m0) * np.eye(n, dtype=np.complex128)  # A at sigma = 0
        csw = getattr(solver, "c_sw", 0.0)
        if csw != 0.0:
            Cs = clover.clover_term(U, dims, csw)
            for q in range(V):
                Ad[12 * q:12 * q + 12, 12 * q:12 * q + 12] += Cs[q]
        Hd = Ad - solver.D0  # D0 = D at sigma = 0; H is the hopping term
        for i, s in enumerate(shifts):
            if hpe_eligible(solver.m0, s):
                M = np.linalg.solve(Ad + s * np.eye(n), Hd)  # A^-1 H
                singles[i] = np.linalg.matrix_power(M, hpe_order) @ invs[i]
    slots = sampling_slots(m)
    T = np.zeros((len(slots), len(gammas), len(p_list)), dtype=np.complex128)
    Var = np.zeros((len(slots), len(gammas), len(p_list)))
    for ip, p in enumerate(p_list):
        Om = lat.omega_dense(U, p, dims)
        for ig, n in enumerate(gammas):
            G = lat.gamma_dense(n, V) @ Om
            for q, (kind, i, j) in enumerate(slots):
                A = level_matrix(None if kind == "single" else invs[i], singles[j] if kind == "single" else invs[j],
                                 G, 1.0)
                T[q, ig, ip] = np.trace(A)
                Var[q, ig, ip] = offdiag_frobenius(A)
    return T, Var
