"""Pins of the oracle functions behind the per-level outputs of the boundary.

* eq. num_samples (optimal N_l): checked against a numerical constrained
  minimisation of the total cost (scipy SLSQP), which knows nothing of the
  Lagrange solution, and against eq. ml_cost_shifts for the cost it reaches;
* the lower bound on the smallest singular value of D + sigma (used by the
  a-posteriori error bound of every level): checked against dense SVD on weak,
  strong, antiperiodic and non-unitary links, and reached exactly in the free
  field (k = 0 mode);
* shared noise across levels: each level stays unbiased (deterministic seeds).
"""

import numpy as np
import pytest
from scipy.optimize import minimize

import synth
from oracle import fs as ofs, lattice as lat


def test_optimal_samples_is_the_constrained_minimum():
    rng = np.random.default_rng(3)
    for _ in range(5):
        n = int(rng.integers(2, 7))
        V = rng.uniform(0.1, 50.0, n)
        C = rng.uniform(1.0, 100.0, n)
        eps2 = 0.01
        N, mu = ofs.optimal_samples(V, C, eps2)
        # it meets the target variance (eq. total_var) exactly ...
        assert np.isclose(np.sum(V / N), eps2, rtol=1e-12)
        # ... at the cost of eq. ml_cost_shifts, eps^-2 (sum_l sqrt(C_l V_l))^2
        assert np.isclose(np.sum(C * N), np.sum(np.sqrt(C * V)) ** 2 / eps2, rtol=1e-12)
        # ... which a generic constrained optimiser cannot beat
        x0 = np.full(n, np.sum(V) / eps2)
        res = minimize(lambda x: np.dot(C, x) / 1e4, x0, method="SLSQP",
                       constraints=[{"type": "eq", "fun": lambda x: np.sum(V / x) / eps2 - 1.0}],
                       bounds=[(1e-6, None)] * n, options={"ftol": 1e-14, "maxiter": 1000})
        assert res.success
        assert np.dot(C, res.x) >= np.dot(C, N) * (1 - 1e-6)
        assert np.allclose(res.x, N, rtol=2e-2)  # the cost is flat at the minimum: x is loose


def _dense_smin(U, dims, m0, sigma, ap=False):
    A = lat.wilson_dense(U, m0, sigma, dims, ap)
    return np.linalg.svd(A, compute_uv=False)[-1]


@pytest.mark.parametrize("eps,ap,scale", [(0.3, False, 1.0), (3.0, False, 1.0), (0.5, True, 1.0), (0.3, False, 1.1)])
def test_smin_lower_bound_holds(eps, ap, scale):
    dims = (2, 2, 4, 2)
    U = synth.gauge_field(dims, eps=eps, seed=5) * scale
    for m0, sigma in ((0.1, 0.0), (0.02, 0.5), (-0.05, 1.0)):
        bound = lat.smin_lower_bound(U, m0, sigma)
        assert _dense_smin(U, dims, m0, sigma, ap) >= bound - 1e-12


def test_smin_lower_bound_is_reached_in_the_free_field():
    dims = (2, 4, 2, 4)
    U = synth.gauge_field(dims, eps=0.0)
    for m0, sigma in ((0.1, 0.0), (0.02, 0.7)):
        assert np.isclose(_dense_smin(U, dims, m0, sigma), lat.smin_lower_bound(U, m0, sigma), rtol=1e-12)


def test_shared_noise_levels_are_unbiased():
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, eps=0.3, seed=0)
    sig = [0.0, 0.5, 1.0]
    dense = ofs.DenseSolver(U, dims, 0.1)
    X = ofs.fs_samples(U, dims, sig, 48, seed=1, gammas=[0, 11], p_max=1, solver=dense, shared_noise=True)
    T, Var = ofs.exact_levels(dense, sig, [0, 11], [0, 1])
    t = X.mean(axis=1)
    assert np.all(np.abs(t - T) <= 4.0 * np.sqrt(Var / 48) + 1e-12)
    # level 0 uses the key of level 0 in both modes; the other levels differ
    Xi = ofs.fs_samples(U, dims, sig, 2, seed=1, gammas=[0], p_max=0, solver=dense)
    Xs = ofs.fs_samples(U, dims, sig, 2, seed=1, gammas=[0], p_max=0, solver=dense, shared_noise=True)
    assert np.array_equal(Xi[0], Xs[0]) and not np.allclose(Xi[1], Xs[1])
