"""Pins of the oracle's multi-shift BiCGStab (CPU).

The multi-shift solver builds every shifted solution from the base system's
Krylov space.  Checks that do not reuse its recurrences: with one shift it is
the textbook BiCGStab of oracle.solver step for step; every shifted solution
meets the tolerance on its own recomputed residual and equals the dense
solution; the shifted residuals it forms as multiples of the base residual
(as the shifted-system theory requires) equal the true residuals
b - (A + s) x of its iterates after every number of steps tried.
"""

import numpy as np

import synth
from oracle import fs as ofs, lattice as lat
from oracle.solver import bicgstab, bicgstab_multishift
from oracle.philox import z4_noise


def _op(U, dims, m0):
    return lambda v: lat.wilson_apply(U, v, m0, 0.0, dims)


def test_one_shift_is_the_textbook_method():
    dims = (4, 4, 2, 2)
    U = synth.gauge_field(dims, eps=0.3, seed=1)
    b = z4_noise(lat.volume(dims), 1, 0, 0, 0)
    A = _op(U, dims, 0.1)
    x1, i1 = bicgstab(lambda v: A(v) + 0.2 * v, b, tol=1e-12)
    xs, i2 = bicgstab_multishift(A, b, [0.2], tol=1e-12)
    assert i1["restarts"] == 0
    assert i1["iters"] == i2["iters"]
    assert np.abs(xs[0] - x1).max() <= 1e-13 * np.abs(x1).max()


def test_shifted_solutions_match_dense_solves():
    dims = (4, 4, 4, 4)
    m0 = 0.05
    U = synth.gauge_field(dims, eps=0.3, seed=0)
    b = z4_noise(lat.volume(dims), 2, 0, 0, 3)
    shifts = [0.0, 0.05, 0.25, 0.5, 1.0]
    xs, info = bicgstab_multishift(_op(U, dims, m0), b, shifts, tol=1e-12)
    dense = ofs.DenseSolver(U, dims, m0)
    for k, s in enumerate(shifts):
        assert info["true_rel"][k] <= 2e-12, (s, info["true_rel"][k])
        ref = dense.solve(s, b)
        assert np.linalg.norm(xs[k] - ref) <= 1e-9 * np.linalg.norm(ref)


def test_shifted_residuals_are_the_true_residuals_of_the_iterates():
    dims = (4, 4, 2, 2)
    m0 = 0.1
    U = synth.gauge_field(dims, eps=0.4, seed=2)
    b = z4_noise(lat.volume(dims), 3, 0, 0, 1)
    shifts = [0.0, 0.3, 0.8]
    A = _op(U, dims, m0)
    trace = []
    # run a few iterations and keep the iterates: the implied shifted residual of
    # iteration n must equal b - (A + s) x^s_n
    for n_it in (3, 7):
        trace.clear()
        xs, _ = bicgstab_multishift(A, b, shifts, tol=1e-30, max_iter=n_it, trace=trace)
        r_last, shifted = trace[-1]
        # after the last iteration the recorded r^d belong to step n_it - 1; recompute at n_it instead:
        xs_prev, _ = bicgstab_multishift(A, b, shifts, tol=1e-30, max_iter=n_it - 1)
        for k in range(1, len(shifts)):
            true_prev = b - A(xs_prev[k]) - shifts[k] * xs_prev[k]
            # the solver forms r^d_n as a multiple of the base residual r_n; that this
            # multiple is the true residual of its own iterate pins the recurrences
            assert np.linalg.norm(shifted[k - 1] - true_prev) <= 1e-10 * np.linalg.norm(b)
