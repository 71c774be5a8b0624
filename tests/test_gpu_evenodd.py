"""Even-odd preconditioned solves and estimates (GPU) against the oracle.

With even_odd = 1 the Krylov solver iterates on the even-site Schur complement
S = a - D_eo D_oe / a (a = 4 + m0 + sigma) and the odd sites follow from
x_o = (b_o - D_oe x_e) / a.  The returned x still solves (D + sigma) x = b, so
the oracle pins it exactly as for the unpreconditioned solver: against dense
LU within tol * ||b|| / s_min, and by recomputing the FP64 true residual of x
with the oracle's operator.  The estimators then match the oracle sample by
sample, and at 16^3x32 the preconditioned and plain paths agree sample by
sample on the same noise while the preconditioned one needs fewer iterations.
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


_SMIN = {}


def _smin(dense, dims, ap, s):
    """Smallest singular value of D + sigma (dense SVD), on the smaller lattices only."""
    if lat.volume(dims) > 256:
        return None
    key = (dims, ap, s)
    if key not in _SMIN:
        A = dense.D0 + s * np.eye(dense.D0.shape[0])
        _SMIN[key] = np.linalg.svd(A, compute_uv=False)[-1]
    return _SMIN[key]


@pytest.mark.parametrize("dims,ap", [((4, 4, 4, 4), False), ((4, 4, 8, 4), True), ((6, 4, 2, 4), False)])
@pytest.mark.parametrize("batched,nr,graph", [(0, 0, 0), (1, 1, 1), (1, 4, 0), (1, 16, 1)])
def test_eo_fp64_solve_vs_dense_lu(L, dims, ap, batched, nr, graph):
    print(f"eo fp64 solve dims={dims} ap={ap} batched={batched} nr={nr} graph={graph}", flush=True)
    U = synth.gauge_field(dims, eps=0.3, seed=3)
    dense = ofs.DenseSolver(U, dims, 0.1, antiperiodic=ap)
    V = lat.volume(dims)
    B = np.stack([z4_noise(V, 2, 0, 0, s) for s in range(5)])
    B[1] *= np.where(np.arange(V) % 3 == 0, 1.0, 0.0)[:, None, None]  # a sparse source
    sig = [0.0, 0.4, 1.1]
    tol = 1e-12
    ctx = L.fs_create(dims, int(ap), 0)
    try:
        L.fs_upload_gauge(ctx, U)
        prm = L.solve_params(0.1, tol=tol, storage="f64", batched=batched, rhs_block=nr, use_graph=graph,
                             even_odd=1)
        X, stats, code = L.fs_solve_shifted(ctx, prm, sig, B)
        assert code == L.FS_OK
        for i, s in enumerate(sig):
            smin = _smin(dense, dims, ap, s)
            for r in range(B.shape[0]):
                st = stats[i * B.shape[0] + r]
                assert st.status == 0 and st.true_rel_residual <= tol, (i, r, st.true_rel_residual)
                assert _true_rel(U, dims, 0.1, s, X[i, r], B[r], ap) <= 1.5 * tol, (i, r)
                if smin is not None:
                    xd = dense.solve(s, B[r])
                    assert np.linalg.norm(X[i, r] - xd) <= 1.5 * tol * np.linalg.norm(B[r]) / smin, (i, r)
    finally:
        L.fs_destroy(ctx)


@pytest.mark.parametrize("prec", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("nr", [2, 8])
def test_eo_mixed_precision_true_residual(L, prec, nr):
    dims = (4, 4, 8, 4)
    print(f"eo mixed {prec} nr={nr}", flush=True)
    U = synth.gauge_field(dims, eps=0.3, seed=4)
    V = lat.volume(dims)
    B = np.stack([z4_noise(V, 3, 0, 0, s) for s in range(6)])
    sig = [0.0, 0.3]
    ctx = L.fs_create(dims, 0, 0)
    try:
        L.fs_upload_gauge(ctx, U)
        prm = L.solve_params(0.05, tol=1e-10, storage=prec, batched=1, rhs_block=nr, use_graph=1, even_odd=1)
        X, stats, code = L.fs_solve_shifted(ctx, prm, sig, B)
        assert code == L.FS_OK
        for i, s in enumerate(sig):
            for r in range(B.shape[0]):
                assert stats[i * B.shape[0] + r].true_rel_residual <= 1e-10
                assert _true_rel(U, dims, 0.05, s, X[i, r], B[r]) <= 1.5e-10, (i, r)
    finally:
        L.fs_destroy(ctx)


def test_eo_needs_even_extents(L):
    ctx = L.fs_create((4, 4, 4, 3), 0, 0)
    try:
        L.fs_upload_gauge(ctx, synth.gauge_field((4, 4, 4, 3), eps=0.3, seed=0))
        b = z4_noise(192, 1, 0, 0, 0)[None]
        with pytest.raises(L.FsError) as e:
            L.fs_solve_shifted(ctx, L.solve_params(0.1, even_odd=1), [0.0], b)
        assert e.value.code == L.FS_E_ARG
        prm = L.fs_est_params(1, 2, 0, 1, L.solve_params(0.1, batched=1, even_odd=1))
        with pytest.raises(L.FsError) as e:
            L.fs_estimate(ctx, prm, [0.0, 0.5])
        assert e.value.code == L.FS_E_ARG
    finally:
        L.fs_destroy(ctx)


@pytest.fixture(scope="module")
def cfg1_ref():
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, eps=0.3, seed=0)
    sig = [0.0, 0.5, 1.0]
    X = ofs.fs_samples(U, dims, sig, 16, seed=1, gammas=list(range(16)), p_max=3,
                       solver=ofs.DenseSolver(U, dims, 0.1))
    return dims, U, sig, X


@pytest.mark.parametrize("storage,tol,ts,batched", [("f64", 1e-12, 1e-9, 0), ("f64", 1e-12, 1e-9, 1),
                                                    ("f32", 1e-10, 1e-7, 1)])
def test_eo_estimate_matches_oracle(L, cfg1_ref, storage, tol, ts, batched):
    dims, U, sig, X_ref = cfg1_ref
    print(f"eo estimate {storage} batched={batched}", flush=True)
    ctx = L.fs_create(dims, 0, 0)
    try:
        L.fs_upload_gauge(ctx, U)
        sp = L.solve_params(0.1, tol=tol, storage=storage, batched=batched, use_graph=batched, even_odd=1)
        stats, X, rep = L.fs_estimate(ctx, L.fs_est_params(1, 16, 0, 3, sp), sig, want_samples=True)
        assert rep.max_rel_residual <= tol
        scale = np.abs(X_ref).mean(axis=1)
        scale = np.where(scale > 0, scale, 1.0)
        assert (np.abs(X - X_ref).max(axis=1) / scale).max() <= ts
        # level means: 1e-10 of mean |X| on the FP64 paths, the stated tolerance otherwise
        t_ref, vp_ref, _ = ofs.level_stats(X_ref, axis=1)
        t_gpu = stats[..., 0] + 1j * stats[..., 1]
        assert (np.abs(t_gpu - t_ref) / scale).max() <= (1e-10 if storage == "f64" else ts)
        assert np.allclose(stats[..., 2], vp_ref, rtol=1e-6, atol=1e-12 * scale.max() ** 2)
    finally:
        L.fs_destroy(ctx)


def test_eo_sampling_and_probing_match_oracle(L):
    from oracle import probing as opr
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, eps=0.3, seed=5)
    dense = ofs.DenseSolver(U, dims, 0.1)
    shifts = [0.0, 0.3, 1.0]
    Xs_ref = ofs.sampling_samples(U, dims, shifts, 4, seed=3, gammas=list(range(16)), p_max=1, solver=dense)
    col = opr.greedy_coloring(dims, 1, 1)
    Xp_ref = opr.fs_samples_probed(U, dims, [0.0, 0.5], 2, seed=2, gammas=list(range(16)), p_max=1, solver=dense,
                                   col=col)
    ctx = L.fs_create(dims, 0, 0)
    try:
        L.fs_upload_gauge(ctx, U)
        sp = L.solve_params(0.1, tol=1e-12, storage="f64", batched=1, rhs_block=4, use_graph=1, even_odd=1)
        print("eo sampling", flush=True)
        _, _, Xs, _, _ = L.fs_sample_variances(ctx, L.fs_est_params(3, 4, 0, 1, sp), shifts, want_samples=True)
        print("eo probed", flush=True)
        _, Xp, _ = L.fs_estimate_probed(ctx, L.fs_est_params(2, 2, 0, 1, sp), [0.0, 0.5], col, want_samples=True)
        for X, Xr in ((Xs, Xs_ref), (Xp, Xp_ref)):
            scale = np.abs(Xr).mean(axis=1)
            scale = np.where(scale > 0, scale, 1.0)
            assert (np.abs(X - Xr).max(axis=1) / scale).max() <= 1e-9
    finally:
        L.fs_destroy(ctx)


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_eo_full_size_agrees_with_plain(L, prec):
    """16^3x32 workload lattice, shifts {0, .05, .25, .5, 1}, 4 Z4 vectors, all
    Gamma, p <= 8: per-sample estimates of the preconditioned and plain batched
    paths agree to 1e-7 of mean |X|, both at the FP64 residual 1e-10, and the
    preconditioned path needs fewer iterations."""
    dims = (16, 16, 16, 32)
    sig = [0.0, 0.05, 0.25, 0.5, 1.0]
    ctx = L.fs_create(dims, 0, 0)
    try:
        L.fs_upload_gauge(ctx, synth.gauge_field(dims, eps=0.2, seed=0))
        out = {}
        for eo in (0, 1):
            print(f"full size {prec} even_odd={eo}", flush=True)
            sp = L.solve_params(0.02, tol=1e-10, storage=prec, batched=1, use_graph=1, even_odd=eo,
                                max_iter=20000)
            stats, X, rep = L.fs_estimate(ctx, L.fs_est_params(1, 4, 0, 8, sp), sig, want_samples=True)
            assert rep.max_rel_residual <= 1e-10
            out[eo] = (X, rep.iterations / rep.systems)
        X0, it0 = out[0]
        X1, it1 = out[1]
        scale = np.abs(X0).mean(axis=1)
        scale = np.where(scale > 0, scale, 1.0)
        assert (np.abs(X1 - X0).max(axis=1) / scale).max() <= 1e-7
        print(f"iterations per system: plain {it0:.1f}, even-odd {it1:.1f}", flush=True)
        assert it1 < it0
    finally:
        L.fs_destroy(ctx)
