"""Multi-shift BiCGStab on the GPU (fs_solve_params.multi_shift) against the oracle.

One Krylov space per right-hand side serves every shift: the smallest shift is
solved by the batched FP64 BiCGStab and the others follow as shifted systems.
Each solution is checked on its own: against the oracle's dense solution and
with the oracle's FP64 residual b - (D + sigma) x (the library's reported true
residual must agree and meet tol).
"""

import numpy as np
import pytest

import synth
from oracle import fs as ofs, lattice as lat
from oracle.philox import z4_noise

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_2212_04430_amd import _lib
    return _lib


def _check(U, dims, m0, sig, B, X, stats, tol, dense=None):
    for i, s in enumerate(sig):
        for r in range(len(B)):
            res = np.linalg.norm(B[r] - lat.wilson_apply(U, X[i, r], m0, s, dims)) / np.linalg.norm(B[r])
            st = stats[i * len(B) + r]
            assert res <= 1.5 * tol, (s, r, res)
            assert st.status == 0 and st.true_rel_residual <= tol
            assert abs(st.true_rel_residual - res) <= 0.1 * tol + 0.01 * res
            if dense is not None:
                ref = dense.solve(s, B[r])
                assert np.linalg.norm(X[i, r] - ref) <= 1e-7 * np.linalg.norm(ref)


@pytest.mark.parametrize("nr,graph,sig", [(4, 1, [0.0, 0.05, 0.25, 0.5, 1.0]), (2, 0, [0.5, 0.0, 1.0]),
                                          (1, 1, [0.3])])
def test_multishift_against_dense(L, nr, graph, sig):
    dims = (4, 4, 4, 4)
    m0 = 0.05
    U = synth.gauge_field(dims, eps=0.3, seed=0)
    V = lat.volume(dims)
    B = np.stack([z4_noise(V, 5, 0, 0, s) for s in range(6)])  # 6 rhs: a padded last block at nr = 4
    print(f"multishift nr={nr} graph={graph} shifts={sig}", flush=True)
    ctx = L.fs_create(dims, 0, 0)
    try:
        L.fs_upload_gauge(ctx, U)
        prm = L.solve_params(m0, tol=1e-10, storage="f64", batched=1, rhs_block=nr, use_graph=graph, multi_shift=1)
        X, stats, code = L.fs_solve_shifted(ctx, prm, sig, B)
        assert code == 0
        _check(U, dims, m0, sig, B, X, stats, 1e-10, ofs.DenseSolver(U, dims, m0))
        # each shift reports the Krylov steps it took: the base (smallest shift) the most
        base = int(np.argmin(sig))
        for r in range(len(B)):
            its = [stats[i * len(B) + r].iters for i in range(len(sig))]
            assert its[base] == max(its) and min(its) > 0
            for i, j in zip(np.argsort(sig)[:-1], np.argsort(sig)[1:]):
                assert its[j] <= its[i]  # larger shifts converge no later
    finally:
        L.fs_destroy(ctx)


def test_multishift_rejects_unsupported_settings(L):
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, eps=0.3, seed=0)
    B = z4_noise(lat.volume(dims), 1, 0, 0, 0)[None]
    ctx = L.fs_create(dims, 0, 0)
    try:
        L.fs_upload_gauge(ctx, U)
        for prm in (L.solve_params(0.1, storage="f32", batched=1, multi_shift=1),
                    L.solve_params(0.1, storage="f64", batched=1, even_odd=1, multi_shift=1)):
            with pytest.raises(L.FsError) as e:
                L.fs_solve_shifted(ctx, prm, [0.0, 0.5], B)
            assert e.value.code == L.FS_E_ARG
        with pytest.raises(L.FsError) as e:
            L.fs_solve_shifted(ctx, L.solve_params(0.1, batched=1, multi_shift=1), list(np.linspace(0, 1, 18)), B)
        assert e.value.code == L.FS_E_ARG
        est = L.fs_est_params(1, 2, 0, 0, L.solve_params(0.1, batched=1, multi_shift=1))
        with pytest.raises(L.FsError) as e:
            L.fs_estimate(ctx, est, [0.0, 0.5])
        assert e.value.code == L.FS_E_ARG
    finally:
        L.fs_destroy(ctx)


def test_multishift_full_size(L):
    """16^3 x 32 (eps 0.2, m0 0.02), the sampling shifts {0, .05, .25, .5, 1}, 4 rhs:
    every solution verified with the oracle's FP64 residual."""
    dims = (16, 16, 16, 32)
    m0 = 0.02
    U = synth.gauge_field(dims, eps=0.2, seed=0)
    V = lat.volume(dims)
    B = np.stack([z4_noise(V, 1, 0, 0, s) for s in range(4)])
    sig = [0.0, 0.05, 0.25, 0.5, 1.0]
    ctx = L.fs_create(dims, 0, 0)
    try:
        L.fs_upload_gauge(ctx, U)
        prm = L.solve_params(m0, tol=1e-10, storage="f64", batched=1, rhs_block=4, use_graph=1, multi_shift=1)
        print("multishift 16^3x32", flush=True)
        X, stats, code = L.fs_solve_shifted(ctx, prm, sig, B)
        assert code == 0
        _check(U, dims, m0, sig, B, X, stats, 1e-10)
    finally:
        L.fs_destroy(ctx)
