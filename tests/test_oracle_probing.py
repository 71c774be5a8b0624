"""Pins of the probing / dilution oracle against facts outside it.

* The greedy colouring passes a brute-force conflict check; with p = 0, k = 1
  on an even torus it is the two-colour checkerboard (x+y+z+t) mod 2.
* With a valid (p, k) colouring, the diluted estimate of Tr(Gamma Omega_p M)
  is exact for every noise draw when M = (D + sigma)^m, m <= k (M couples
  sites at most m apart), against the trace of the dense product; with
  m = k + 1 it is not, so the check is not vacuous.
* The adjoint shortcut y = s_a g5 (D+sigma)^-1 z equals the g5 solve.
* The probed FS estimator is unbiased: per-level means within 4 standard
  errors of the exact dense-LU level traces.
"""

import numpy as np
import pytest

import synth
from oracle import fs as ofs, lattice as lat, probing as opr
from oracle.philox import z4_noise


@pytest.mark.parametrize("dims,p,k", [((4, 4, 4, 4), 1, 1), ((4, 4, 6, 4), 2, 2), ((4, 4, 8, 2), 3, 2),
                                      ((4, 4, 4, 4), 0, 2)])
def test_coloring_is_valid(dims, p, k):
    col = opr.greedy_coloring(dims, p, k)
    assert opr.coloring_is_valid(col, dims, p, k)
    assert set(col) == set(range(col.max() + 1))  # every colour used


def test_distance_one_coloring_is_checkerboard():
    dims = (4, 4, 4, 2)
    col = opr.greedy_coloring(dims, 0, 1)
    par = np.array([sum(lat.site_coords(s, dims)) % 2 for s in range(lat.volume(dims))])
    assert col.max() == 1 and np.array_equal(col, par)


class _PowerOp:
    """'solve' that applies (D + sigma)^m: an operator reaching m sites."""

    def __init__(self, U, dims, m0, m):
        self.U, self.dims, self.m0, self.m = U, dims, m0, m

    def solve(self, sigma, z):
        v = z
        for _ in range(self.m):
            v = lat.wilson_apply(self.U, v, self.m0, sigma, self.dims)
        return v


@pytest.mark.parametrize("dims,p,k", [((4, 4, 4, 4), 1, 1), ((4, 4, 6, 2), 2, 2)])
def test_probing_exact_for_short_range_operator(dims, p, k):
    U = synth.gauge_field(dims, eps=0.4, seed=2)
    V = lat.volume(dims)
    col = opr.greedy_coloring(dims, p, k)
    gam = [0, 5, 11, 15]
    sig = 0.3
    Dd = lat.wilson_dense(U, 0.1, sig, dims)
    GO = {n: lat.gamma_dense(n, V) @ lat.omega_dense(U, p, dims) for n in gam}
    M = np.eye(Dd.shape[0], dtype=complex)
    for m in range(0, k + 2):
        if m > 0:
            M = Dd @ M
        X = opr.fs_samples_probed(U, dims, [sig], 1, seed=4, gammas=gam, p_max=p, solver=_PowerOp(U, dims, 0.1, m),
                                  col=col)[0, 0]
        for ig, n in enumerate(gam):
            T = (GO[n] @ M).trace()
            err = abs(X[ig, p] - T)
            if m <= k:
                assert err <= 1e-10 * max(1.0, abs(T)), (m, n, err)
            elif n == 0:
                assert err > 1e-6, "m = k + 1 should reach beyond the colouring"


class _DenseOp:
    def __init__(self, A):
        self.A = A

    def solve(self, sigma, z):
        return (self.A @ z.reshape(-1)).reshape(z.shape)


def test_probing_exact_for_backward_displacement():
    """The colouring also covers the neighbourhood of x - p z^: the estimate of
    Tr(Gamma Omega_p^dagger M), M = (D + sigma)^k, formed as p = 0 bilinears
    with the map Omega_p^dagger M, is exact."""
    dims, p, k = (4, 4, 6, 2), 2, 2
    U = synth.gauge_field(dims, eps=0.4, seed=3)
    V = lat.volume(dims)
    col = opr.greedy_coloring(dims, p, k)
    M = np.linalg.matrix_power(lat.wilson_dense(U, 0.1, 0.3, dims), k)
    A = lat.omega_dense(U, p, dims).conj().T @ M
    gam = [0, 11]
    X = opr.fs_samples_probed(U, dims, [0.3], 1, seed=6, gammas=gam, p_max=0, solver=_DenseOp(A), col=col)[0, 0]
    for ig, n in enumerate(gam):
        T = (lat.gamma_dense(n, V) @ A).trace()
        assert abs(X[ig, 0] - T) <= 1e-10 * max(1.0, abs(T)), n


def test_adjoint_shortcut_for_diluted_sources():
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, eps=0.3, seed=1)
    dense = ofs.DenseSolver(U, dims, 0.1)
    col = opr.greedy_coloring(dims, 1, 1)
    xi = z4_noise(lat.volume(dims), 9, 0, 0, 0)
    for j, a in ((0, 0), (1, 5), (2, 7), (0, 11)):
        z = opr.diluted_source(xi, col, j, a)
        y_short = opr.g5_sign(a) * lat.apply_gamma5(dense.solve(0.4, z))
        y_full = lat.apply_gamma5(dense.solve(0.4, lat.apply_gamma5(z)))
        assert np.allclose(y_short, y_full, atol=1e-13)


def test_probed_estimator_unbiased():
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, eps=0.3, seed=0)
    dense = ofs.DenseSolver(U, dims, 0.1)
    col = opr.greedy_coloring(dims, 1, 1)
    sig = [0.0, 0.5]
    gam = [0, 11]
    N = 4
    X = opr.fs_samples_probed(U, dims, sig, N, seed=1, gammas=gam, p_max=1, solver=dense, col=col)
    T, _ = ofs.exact_levels(dense, sig, gam, [0, 1], with_variance=False)
    t, var, _ = ofs.level_stats(X, axis=1)
    se = np.sqrt(np.maximum(var, 1e-30) / (N - 1))
    assert np.all(np.abs(t - T) <= 4 * se + 1e-12 * np.abs(T).max())
