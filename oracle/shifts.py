"""Shift selection for Frequency Splitting (oracle): interpolation and the C_FS argmin.

TEST INFRASTRUCTURE ONLY (see the package docstring).

After the sampling phase (Sec. 3.1) has estimated V_L(s^_i) and
Vbar_l(s^_i, s^_j), j >= i, and the iteration counts r(s^_i) on the m
sampling shifts s^, the paper predicts these quantities on a finer
evaluation set s (n shifts) and picks the L shifts of s that minimise
eq. ml_cost_shifts (eq. opt_shifts):

* Sec. 3.2, interpolation in log space with piecewise cubic Hermite
  polynomials that preserve monotonicity (PCHIP; Fritsch & Carlson 1980,
  with the derivative choice of Fritsch & Butland 1984), linear when only
  two points exist:
    V_L(s_k)     = exp(q(s_k)),  q through (s^_i, ln V_L(s^_i));
    Vbar_l       by the three-stage 2-D algorithm of Figure "boundary";
    V_l(s_i,s_k) = (s_k - s_i)^2 Vbar_l(s_i, s_k)   (eq. sampled_prod).
* Sec. 3.2, solver cost: r(s_i) = r(s^_j) for s^_{j-1} < s_i <= s^_j (the
  nearest sampled shift at or above s_i; C(s) = 12 c r(s), eq.
  solver_cost_shift, with 12 c = 1 for undiluted noise).
* Sec. 2.3, eq. ml_cost_shifts with eps = 1:
    C_FS = (sum_{l=0}^{L} sqrt(C_l V_l))^2,
  C_l = C(sigma_l) + C(sigma_{l+1}) for l < L (a level-l sample solves at
  both of its shifts) and C_L = C(sigma_L).
* Sec. 3.3, eq. opt_shifts: the argmin over 0 = s_0 < s_{j_1} < ... < s_{j_L}.
  `select_brute` walks every combination as the paper does;
  `select_dp` gets the same minimum from a shortest-path recursion over
  increasing indices (the objective is a sum of terms that each depend on
  two consecutive shifts).

Readings (listed in the design notes):
* the evaluation set is the paper's grid [0, logspace(-5,-2,4),
  logspace(log10(0.011), 0, 76)] (0 prepended), cut at s^_{m-1}, with the
  sampling shifts inserted where missing (the evaluation set contains the
  sampling set);
* step 3 of the 2-D algorithm at fixed s_i interpolates through the diagonal
  point (s_i, Vbar(s_i, s_i)) and the points (s^_j, Vbar(s_i, s^_j)) with
  s^_j > s_i, which the text describes (the printed "j = 0..m-1" would need
  values below the diagonal that the algorithm never forms);
* PCHIP end slopes use the one-sided three-point formula with the
  shape-preserving limits of Fritsch-Butland; two points give a line.

Parity: PCHIP against scipy's PchipInterpolator and against linear data; the
2-D scheme against separable exponential surfaces it must reproduce exactly;
the cost model by hand values; the DP against the brute force on small grids;
the grid against the optimal shifts printed in the Results section.
"""

import itertools

import numpy as np


# ---------------------------------------------------------------------------
# Evaluation set
# ---------------------------------------------------------------------------

def eval_grid(s_hat):
    """The paper's 81-point evaluation set (Sec. 3.3), cut at the largest
    sampling shift, with the sampling shifts inserted."""
    base = np.concatenate([[0.0], np.logspace(-5, -2, 4), np.logspace(np.log10(1e-2 + 1e-3), 0, 76)])
    top = s_hat[-1]
    pts = [v for v in base if v <= top]
    for v in s_hat:
        if not any(v == p for p in pts):
            pts.append(v)
    return np.array(sorted(pts))


# ---------------------------------------------------------------------------
# PCHIP (Sec. 3.2)
# ---------------------------------------------------------------------------

def _sign(v):
    return (v > 0) - (v < 0)


def pchip_slopes(x, y):
    """Node derivatives of the monotone cubic Hermite interpolant."""
    n = len(x)
    h = [x[k + 1] - x[k] for k in range(n - 1)]
    d = [(y[k + 1] - y[k]) / h[k] for k in range(n - 1)]
    if n == 2:
        return [d[0], d[0]]
    g = [0.0] * n
    for k in range(1, n - 1):
        if d[k - 1] * d[k] <= 0:
            g[k] = 0.0
        else:
            w1 = 2 * h[k] + h[k - 1]
            w2 = h[k] + 2 * h[k - 1]
            g[k] = (w1 + w2) / (w1 / d[k - 1] + w2 / d[k])

    def end(h0, h1, d0, d1):
        e = ((2 * h0 + h1) * d0 - h0 * d1) / (h0 + h1)
        if _sign(e) != _sign(d0):
            return 0.0
        if _sign(d0) != _sign(d1) and abs(e) > abs(3 * d0):
            return 3 * d0
        return e

    g[0] = end(h[0], h[1], d[0], d[1])
    g[n - 1] = end(h[n - 2], h[n - 3], d[n - 2], d[n - 3])
    return g


def pchip_eval(x, y, g, t):
    """Value at t (x[0] <= t <= x[-1]) of the cubic Hermite interpolant with
    node values y and node derivatives g."""
    n = len(x)
    k = 0
    while k < n - 2 and t > x[k + 1]:
        k += 1
    hk = x[k + 1] - x[k]
    u = (t - x[k]) / hk
    h00 = (1 + 2 * u) * (1 - u) ** 2
    h10 = u * (1 - u) ** 2
    h01 = u * u * (3 - 2 * u)
    h11 = u * u * (u - 1)
    return h00 * y[k] + h10 * hk * g[k] + h01 * y[k + 1] + h11 * hk * g[k + 1]


def interpolate(x, y, t):
    """The paper's Interpolate(x, y) evaluated at the points t: PCHIP, or the
    line through two points; a single point is a constant."""
    x = [float(v) for v in x]
    y = [float(v) for v in y]
    if len(x) == 1:
        return np.full(len(t), y[0])
    g = pchip_slopes(x, y)
    return np.array([pchip_eval(x, y, g, float(v)) for v in t])


# ---------------------------------------------------------------------------
# Predicted variances and costs on the evaluation set (Sec. 3.2)
# ---------------------------------------------------------------------------

def interp_single(s_hat, v_single, s):
    """V_L(s_k) = exp(q(s_k)), q through (s^_i, ln V_L(s^_i))."""
    return np.exp(interpolate(s_hat, np.log(v_single), s))


def interp_pairs(s_hat, v_pair, s):
    """The 2-D algorithm of Figure "boundary": V_l(s_i, s_k) for k > i (zero
    elsewhere).  v_pair[i][j], j >= i, holds the sampled Vbar_l(s^_i, s^_j)."""
    m, n = len(s_hat), len(s)
    # stage 1: along the first argument at each fixed sampled s^_j, j >= 1
    col = np.full((n, m), np.nan)  # col[k, j] = Vbar(s_k, s^_j) for s_k <= s^_j
    for j in range(1, m):
        w = [np.log(v_pair[i][j]) for i in range(j + 1)]
        ks = [k for k in range(n) if s[k] <= s_hat[j]]
        col[ks, j] = np.exp(interpolate(s_hat[:j + 1], w, s[ks]))
    # stage 2: along the diagonal
    diag = np.exp(interpolate(s_hat, [np.log(v_pair[i][i]) for i in range(m)], s))
    # stage 3: along the second argument at each fixed s_i
    out = np.zeros((n, n))
    for i in range(n - 1):
        xs = [s[i]] + [s_hat[j] for j in range(m) if s_hat[j] > s[i]]
        ws = [np.log(diag[i])] + [np.log(col[i, j]) for j in range(m) if s_hat[j] > s[i]]
        ks = list(range(i + 1, n))
        q = interpolate(xs, ws, s[ks])
        for kk, k in enumerate(ks):
            out[i, k] = (s[k] - s[i]) ** 2 * np.exp(q[kk])
    return out


def nn_cost(s_hat, r_hat, s):
    """r(s_i) = r(s^_j) with s^_{j-1} < s_i <= s^_j; r(0) = r(s^_0)."""
    out = np.zeros(len(s))
    for k, v in enumerate(s):
        j = 0
        while s_hat[j] < v:
            j += 1
        out[k] = r_hat[j]
    return out


# ---------------------------------------------------------------------------
# Multilevel cost and its argmin (Sec. 2.3, 3.3)
# ---------------------------------------------------------------------------

def level_terms(idx, v_pair_eval, v_single_eval, r_eval):
    """Per-level (V_l, C_l) for the shift indices idx = (0, j_1, ..., j_L)."""
    L = len(idx) - 1
    V = [v_pair_eval[idx[l], idx[l + 1]] for l in range(L)] + [v_single_eval[idx[L]]]
    C = [r_eval[idx[l]] + r_eval[idx[l + 1]] for l in range(L)] + [r_eval[idx[L]]]
    return np.array(V), np.array(C)


def c_fs(idx, v_pair_eval, v_single_eval, r_eval):
    """eq. ml_cost_shifts with eps = 1, summed over levels in order."""
    V, C = level_terms(idx, v_pair_eval, v_single_eval, r_eval)
    acc = 0.0
    for l in range(len(V)):
        acc += np.sqrt(C[l] * V[l])
    return acc * acc


def select_brute(L, v_pair_eval, v_single_eval, r_eval):
    """eq. opt_shifts by trying every 0 < j_1 < ... < j_L <= n-1."""
    n = len(r_eval)
    best, best_idx = np.inf, None
    for comb in itertools.combinations(range(1, n), L):
        idx = (0,) + comb
        c = c_fs(idx, v_pair_eval, v_single_eval, r_eval)
        if c < best:
            best, best_idx = c, idx
    return best_idx, best


def select_dp(L, v_pair_eval, v_single_eval, r_eval):
    """eq. opt_shifts by a shortest path: f_l(k) is the least sum of the first l
    level terms over paths 0 = j_0 < ... < j_l = k."""
    n = len(r_eval)

    def w(i, k):
        return np.sqrt((r_eval[i] + r_eval[k]) * v_pair_eval[i, k])

    if L == 0:
        return (0,), r_eval[0] * v_single_eval[0]
    f = {k: (w(0, k), (0, k)) for k in range(1, n)}
    for _ in range(1, L):
        g = {}
        for k in range(1, n):
            cand = [(f[i][0] + w(i, k), f[i][1] + (k,)) for i in f if i < k]
            if cand:
                g[k] = min(cand, key=lambda t: t[0])
        f = g
    tot = [(f[k][0] + np.sqrt(r_eval[k] * v_single_eval[k]), f[k][1]) for k in f]
    s, idx = min(tot, key=lambda t: t[0])
    return idx, s * s
