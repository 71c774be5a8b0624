"""GPU BiCGStab (FP64 and mixed precision with FP64 reliable updates) against the oracle.

The oracle pins each solution two ways: against a dense LU solve (error bound
tol * ||b|| / s_min(D + sigma)), and by recomputing the FP64 true residual
||b - (D + sigma) x|| / ||b|| of the returned x with the oracle's operator.
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


def _true_rel(U, dims, m0, sigma, x, b, ap=False):
    r = b - lat.wilson_apply(U, x, m0, sigma, dims, ap)
    return np.linalg.norm(r) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def cfg1(L):
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, eps=0.3, seed=0)
    ctx = L.fs_create(dims, 0, 0)
    L.fs_upload_gauge(ctx, U)
    dense = ofs.DenseSolver(U, dims, 0.1)
    yield ctx, U, dims, dense
    L.fs_destroy(ctx)


@pytest.mark.parametrize("batched,nr,graph", [(0, 0, 0), (1, 4, 0), (1, 2, 1), (1, 16, 1)])
def test_fp64_solve_vs_dense_lu(L, cfg1, batched, nr, graph):
    ctx, U, dims, dense = cfg1
    print(f"fp64 solve batched={batched} nr={nr} graph={graph}", flush=True)
    V = lat.volume(dims)
    B = np.stack([z4_noise(V, 1, 0, 0, s) for s in range(5)])
    sig = [0.0, 0.5, 1.0]
    tol = 1e-12
    prm = L.solve_params(0.1, tol=tol, storage="f64", batched=batched, rhs_block=nr, use_graph=graph)
    X, stats, code = L.fs_solve_shifted(ctx, prm, sig, B)
    assert code == L.FS_OK
    for i, s in enumerate(sig):
        A = dense.D0 + s * np.eye(dense.D0.shape[0])
        smin = np.linalg.svd(A, compute_uv=False)[-1] if i == 0 else None
        for r in range(B.shape[0]):
            st = stats[i * B.shape[0] + r]
            assert st.status == 0 and st.true_rel_residual <= tol
            assert _true_rel(U, dims, 0.1, s, X[i, r], B[r]) <= 1.5 * tol
            xd = dense.solve(s, B[r])
            if smin is not None:
                assert np.linalg.norm(X[i, r] - xd) <= 1.5 * tol * np.linalg.norm(B[r]) / smin


@pytest.mark.parametrize("prec", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("graph", [0, 1])
def test_mixed_precision_reaches_fp64_tolerance(L, cfg1, prec, graph):
    ctx, U, dims, dense = cfg1
    print(f"mixed solve prec={prec} graph={graph}", flush=True)
    V = lat.volume(dims)
    B = np.stack([z4_noise(V, 3, 0, 1, s) for s in range(8)])
    sig = [0.0, 0.05, 1.0]
    tol = 1e-10
    prm = L.solve_params(0.1, tol=tol, storage=prec, batched=1, rhs_block=8, use_graph=graph)
    X, stats, code = L.fs_solve_shifted(ctx, prm, sig, B)
    assert code == L.FS_OK
    for i, s in enumerate(sig):
        for r in range(B.shape[0]):
            st = stats[i * B.shape[0] + r]
            assert st.status == 0 and st.reliable_updates >= 1
            assert _true_rel(U, dims, 0.1, s, X[i, r], B[r]) <= 1.5 * tol


def test_non_convergence_reported(L, cfg1):
    ctx, U, dims, dense = cfg1
    V = lat.volume(dims)
    B = z4_noise(V, 1, 0, 0, 0)[None]
    prm = L.solve_params(0.1, tol=1e-12, max_iter=3, storage="f64")
    X, stats, code = L.fs_solve_shifted(ctx, prm, [0.0], B, allow_noconv=True)
    assert code == L.FS_E_NOCONV
    assert stats[0].status == L.FS_E_NOCONV and stats[0].iters >= 3
    assert np.isfinite(X).all()
    # the reported residual is the true one of the returned iterate
    assert abs(_true_rel(U, dims, 0.1, 0.0, X[0, 0], B[0]) - stats[0].true_rel_residual) < 1e-8


def test_solver_argument_errors(L, cfg1):
    ctx = cfg1[0]
    V = 256
    B = np.zeros((1, V, 4, 3), dtype=complex)
    with pytest.raises(L.FsError) as e:
        L.fs_solve_shifted(ctx, L.solve_params(0.1, tol=-1.0), [0.0], B)
    assert e.value.code == L.FS_E_ARG
    with pytest.raises(L.FsError) as e:
        L.fs_solve_shifted(ctx, L.solve_params(0.1, rhs_block=3, batched=1), [0.0], B)
    assert e.value.code == L.FS_E_ARG
    # zero source: converged at once with x = 0
    X, st, code = L.fs_solve_shifted(ctx, L.solve_params(0.1), [0.0], B)
    assert code == 0 and np.all(X == 0)


def test_solve_at_cfg2_shape_true_residual(L):
    """8^3 x 16 (eps 0.25, m0 0.05): every shift of cfg 2 to 1e-10, FP64 and mixed."""
    dims = (8, 8, 8, 16)
    U = synth.gauge_field(dims, eps=0.25, seed=0)
    ctx = L.fs_create(dims, 0, 0)
    try:
        L.fs_upload_gauge(ctx, U)
        V = lat.volume(dims)
        B = np.stack([z4_noise(V, 1, 0, 0, s) for s in range(4)])
        sig = [0.0, 0.1, 0.4, 1.2]
        for prec, batched in (("f64", 0), ("f32", 1), ("f16", 1)):
            print(f"cfg2 solve prec={prec}", flush=True)
            prm = L.solve_params(0.05, tol=1e-10, storage=prec, batched=batched, rhs_block=4, use_graph=batched)
            X, stats, code = L.fs_solve_shifted(ctx, prm, sig, B)
            assert code == L.FS_OK
            for i, s in enumerate(sig):
                for r in range(B.shape[0]):
                    assert _true_rel(U, dims, 0.05, s, X[i, r], B[r]) <= 1.5e-10
    finally:
        L.fs_destroy(ctx)
