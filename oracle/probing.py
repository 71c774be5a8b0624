"""Probing with full spin-colour dilution for the FS estimator (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Background, Probing: a distance-k colouring of the graph of A leaves the trace
of A^k exact when the estimator sums z_j^dagger A z_j over the colour
indicator vectors z_j (eq. probing_vectors).  For a displacement Pi_p the
colouring is taken on the symmetric part of Pi_p A^k: two sites x != y
conflict when y lies within distance k of x + p z^ or of x - p z^
(neighbourhoods centred at the displaced sites).  On the lattice the graph
distance of the Wilson operator is the periodic taxicab distance.  A greedy
colouring suffices; it visits the sites in index order and gives each the
smallest colour that no conflicting, already coloured site holds.

Combined with Z4 noise and full spin-colour dilution (Sec. 3.1), each sample
uses the 12 c sources
    z^(j, a)(x, b) = xi(x, a) if colour(x) = j and b = a, else 0,
a = spin-colour index (spin a // 3, colour a % 3), xi the Z4 field keyed
(seed, instance, level, sample), and sums their bilinears:
    X_s = sum_{j, a} coef * y^dagger Gamma Omega_p x
For a spin-diluted source g5 z = s_a z with s_a = +1 for spins 0, 1 and -1 for
spins 2, 3 (DeGrand-Rossi g5 = diag(1, 1, -1, -1)), so the adjoint solution
is y = (D+sigma)^-dagger z = s_a g5 (D+sigma)^-1 z: a level l < L needs the
solves at sigma_l and sigma_{l+1} of the same source and no g5 solve.

Readings (listed in the design notes): the per-site noise differs per
spin-colour component (the Z4 field's own component); the colouring is the
greedy one in site order; one colouring serves every displacement p.

Parity: a valid colouring (brute-force conflict check) makes the estimate of
Tr(Gamma Omega_p M) exact for any operator M whose couplings reach at most k
sites, e.g. M = (D + sigma)^m with m <= k, against the dense trace; the
adjoint shortcut against the g5 solve; unbiasedness against the exact trace.
"""

import itertools

import numpy as np

from . import lattice as lat
from .fs import bilinears
from .philox import z4_noise


def torus_dist(a, b, dims):
    """Periodic taxicab distance between site coordinates a and b."""
    d = 0
    for u, v, L in zip(a, b, dims):
        e = abs(u - v) % L
        d += min(e, L - e)
    return d


def conflicts(s, dims, p, k):
    """Sites y != s within distance k of s + p z^ or s - p z^."""
    x = lat.site_coords(s, dims)
    up = (x[0], x[1], (x[2] + p) % dims[2], x[3])
    dn = (x[0], x[1], (x[2] - p) % dims[2], x[3])
    out = []
    for y in range(lat.volume(dims)):
        if y == s:
            continue
        c = lat.site_coords(y, dims)
        if torus_dist(up, c, dims) <= k or torus_dist(dn, c, dims) <= k:
            out.append(y)
    return out


def greedy_coloring(dims, p, k):
    """Colours in site order: the smallest colour unused by conflicting earlier sites."""
    V = lat.volume(dims)
    col = [-1] * V
    for s in range(V):
        used = {col[y] for y in conflicts(s, dims, p, k) if y < s}
        c = 0
        while c in used:
            c += 1
        col[s] = c
    return np.array(col)


def coloring_is_valid(col, dims, p, k):
    """Brute force: no two conflicting sites share a colour."""
    V = lat.volume(dims)
    for s in range(V):
        for y in conflicts(s, dims, p, k):
            if col[y] == col[s]:
                return False
    return True


def diluted_source(xi, col, j, a):
    """xi restricted to the sites of colour j and to spin-colour component a."""
    z = np.zeros_like(xi)
    sites = np.flatnonzero(col == j)
    z[sites, a // 3, a % 3] = xi[sites, a // 3, a % 3]
    return z


def g5_sign(a):
    return 1.0 if a // 3 < 2 else -1.0


def probed_level_vectors(solver, sigmas, level, z, a):
    """(coef, y, x) of one diluted source for this level."""
    L = len(sigmas) - 1
    if level < L:
        x = solver.solve(sigmas[level + 1], z)
        y = g5_sign(a) * lat.apply_gamma5(solver.solve(sigmas[level], z))
        return sigmas[level + 1] - sigmas[level], y, x
    return 1.0, z, solver.solve(sigmas[L], z)


def fs_samples_probed(U, dims, sigmas, n_noise, seed, gammas, p_max, solver, col, instance=0):
    """Per-sample estimates X[l, s, n_idx, p], each summed over the 12 c diluted sources."""
    L = len(sigmas) - 1
    V = lat.volume(dims)
    n_col = int(col.max()) + 1
    X = np.zeros((L + 1, n_noise, len(gammas), p_max + 1), dtype=np.complex128)
    for l in range(L + 1):
        for s in range(n_noise):
            xi = z4_noise(V, seed, instance, l, s)
            for j, a in itertools.product(range(n_col), range(12)):
                z = diluted_source(xi, col, j, a)
                coef, y, x = probed_level_vectors(solver, sigmas, l, z, a)
                X[l, s] += coef * bilinears(U, dims, y, x, gammas, p_max)
    return X
