"""The clover-improved operator on the GPU against the CPU oracle.

fs_set_clover builds C from the links on the device; the operator, the
even-odd solves (Schur complement with per-shift inverses of C_o + a) and the
Frequency-Splitting estimates are compared with oracle.clover on the same
links and noise.  FP64: the operator to 1e-13 relative, per-sample estimates to
1e-9 and level means to 1e-10 of mean |X_s| (as for the plain operator);
FP32 storage: the operator to 2e-6 relative (inputs and links rounded to FP32),
mixed-precision estimates to 1e-7 after FP64 reliable updates.
"""

import numpy as np
import pytest

import synth
from oracle import clover as cl, fs as ofs, lattice as lat
from oracle.philox import z4_noise

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_2212_04430_amd import _lib
    return _lib


def _rand_spinors(n, V, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, V, 4, 3)) + 1j * rng.standard_normal((n, V, 4, 3))


@pytest.mark.parametrize("dims,csw", [((4, 4, 4, 4), 1.3), ((8, 4, 4, 6), 1.0), ((4, 6, 2, 4), 1.9)])
def test_operator_parity(L, dims, csw):
    print(f"clover operator dims={dims} csw={csw}", flush=True)
    U = synth.gauge_field(dims, eps=0.4, seed=1)
    V = lat.volume(dims)
    psi = _rand_spinors(5, V, 2)
    C = cl.clover_term(U, dims, csw)
    ctx = L.fs_create(dims, 0, 0)
    try:
        L.fs_upload_gauge(ctx, U)
        L.fs_set_clover(ctx, csw)
        for sigma in (0.0, 0.37):
            ref = np.stack([cl.clover_apply(U, p, 0.05, sigma, csw, dims, C=C) for p in psi])
            scale = np.abs(ref).max()
            got = L.fs_apply_dirac(ctx, 0.05, sigma, "f64", psi)
            assert np.abs(got - ref).max() <= 1e-13 * scale
            got32 = L.fs_apply_dirac(ctx, 0.05, sigma, "f32", psi)
            assert np.abs(got32 - ref).max() <= 2e-6 * scale
        # back to the plain operator
        L.fs_set_clover(ctx, 0.0)
        got = L.fs_apply_dirac(ctx, 0.05, 0.0, "f64", psi[0])
        assert np.abs(got - lat.wilson_apply(U, psi[0], 0.05, 0.0, dims)).max() <= 1e-13 * np.abs(got).max()
    finally:
        L.fs_destroy(ctx)


def test_term_follows_a_new_gauge_upload(L):
    dims = (4, 4, 4, 4)
    U0 = synth.gauge_field(dims, eps=0.4, seed=3)
    U1 = synth.gauge_field(dims, eps=0.4, seed=4)
    psi = _rand_spinors(1, lat.volume(dims), 5)[0]
    ctx = L.fs_create(dims, 0, 0)
    try:
        L.fs_upload_gauge(ctx, U0)
        L.fs_set_clover(ctx, 1.1)
        L.fs_upload_gauge(ctx, U1)
        got = L.fs_apply_dirac(ctx, 0.1, 0.0, "f64", psi)
        ref = cl.clover_apply(U1, psi, 0.1, 0.0, 1.1, dims)
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    finally:
        L.fs_destroy(ctx)


@pytest.mark.parametrize("storage,batched,nr,graph", [("f64", 0, 0, 0), ("f64", 1, 4, 1), ("f32", 1, 4, 1),
                                                       ("f32", 1, 2, 0)])
def test_even_odd_solves(L, storage, batched, nr, graph):
    dims = (4, 4, 4, 4)
    csw = 1.4
    U = synth.gauge_field(dims, eps=0.3, seed=0)
    V = lat.volume(dims)
    B = np.stack([z4_noise(V, 7, 0, 0, s) for s in range(4)])
    sig = [0.0, 0.2, 0.9]
    print(f"clover solves storage={storage} batched={batched} nr={nr} graph={graph}", flush=True)
    ctx = L.fs_create(dims, 0, 0)
    try:
        L.fs_upload_gauge(ctx, U)
        L.fs_set_clover(ctx, csw)
        prm = L.solve_params(0.05, tol=1e-10, storage=storage, batched=batched, rhs_block=nr, use_graph=graph,
                             even_odd=1)
        X, stats, code = L.fs_solve_shifted(ctx, prm, sig, B)
        assert code == 0
        dense = ofs.DenseSolver(U, dims, 0.05, c_sw=csw)
        C = cl.clover_term(U, dims, csw)
        for i, s in enumerate(sig):
            for r in range(len(B)):
                res = np.linalg.norm(B[r] - cl.clover_apply(U, X[i, r], 0.05, s, csw, dims, C=C)) / np.linalg.norm(B[r])
                assert res <= 1.5e-10, (s, r, res)
                assert stats[i * len(B) + r].true_rel_residual <= 1e-10
                x_ref = dense.solve(s, B[r])
                assert np.linalg.norm(X[i, r] - x_ref) <= 1e-8 * np.linalg.norm(x_ref)
    finally:
        L.fs_destroy(ctx)


@pytest.fixture(scope="module")
def cfg1_clover_ref():
    """cfg 1 with the clover term: 4^4, eps 0.3, m0 0.1, c_sw 1.2, shifts {0, 0.5, 1.0},
    32 Z4 vectors, all Gamma, p <= 2."""
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, eps=0.3, seed=0)
    csw = 1.2
    sig = [0.0, 0.5, 1.0]
    dense = ofs.DenseSolver(U, dims, 0.1, c_sw=csw)
    X = ofs.fs_samples(U, dims, sig, 32, seed=1, gammas=list(range(16)), p_max=2, solver=dense)
    return dims, U, csw, sig, X


@pytest.mark.parametrize("storage,tol,ts,tm", [("f64", 1e-12, 1e-9, 1e-10), ("f32", 1e-10, 1e-7, 1e-7)])
def test_estimate_parity(L, cfg1_clover_ref, storage, tol, ts, tm):
    dims, U, csw, sig, X_ref = cfg1_clover_ref
    print(f"clover estimate {storage}", flush=True)
    ctx = L.fs_create(dims, 0, 0)
    try:
        L.fs_upload_gauge(ctx, U)
        L.fs_set_clover(ctx, csw)
        sp = L.solve_params(0.1, tol=tol, storage=storage, batched=1, rhs_block=4, use_graph=1, even_odd=1)
        prm = L.fs_est_params(1, 32, 0, 2, sp)
        prm.report_fp64_error = 1
        stats, X, rep = L.fs_estimate(ctx, prm, sig, want_samples=True)
        assert rep.max_rel_residual <= tol
        scale = np.abs(X_ref).mean(axis=1)
        scale = np.where(scale > 0, scale, 1.0)
        assert (np.abs(X - X_ref).max(axis=1) / scale).max() <= ts
        t_ref, vp_ref, _ = ofs.level_stats(X_ref, axis=1)
        t_gpu = stats[..., 0] + 1j * stats[..., 1]
        assert (np.abs(t_gpu - t_ref) / scale).max() <= tm
        assert np.allclose(stats[..., 2], vp_ref, rtol=1e-6, atol=1e-12 * scale.max() ** 2)
        # the reported FP64 deviation stays within the reported bound (infinite
        # here: 4 + m0 - 4 max||U|| - max||C|| < 0 for this field, so the s_min
        # bound gives nothing)
        assert cl.smin_lower_bound(U, 0.1, 0.0, csw, dims) < 0
        assert np.all(stats[..., 6] <= stats[..., 7])
    finally:
        L.fs_destroy(ctx)


def test_unsupported_settings_are_rejected(L):
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, eps=0.3, seed=0)
    V = lat.volume(dims)
    B = z4_noise(V, 1, 0, 0, 0)[None]
    ctx = L.fs_create(dims, 0, 0)
    try:
        L.fs_upload_gauge(ctx, U)
        with pytest.raises(L.FsError) as e:
            L.fs_set_clover(ctx, float("nan"))
        assert e.value.code == L.FS_E_ARG
        L.fs_set_clover(ctx, 1.0)
        for prm in (L.solve_params(0.1, storage="f64", even_odd=0),
                    L.solve_params(0.1, storage="f16", batched=1, rhs_block=4, even_odd=1),
                    L.solve_params(0.1, storage="bf16", batched=1, rhs_block=4, even_odd=1)):
            with pytest.raises(L.FsError) as e:
                L.fs_solve_shifted(ctx, prm, [0.0], B)
            assert e.value.code == L.FS_E_ARG
        with pytest.raises(L.FsError) as e:
            L.fs_apply_dirac(ctx, 0.1, 0.0, "f16", B[0])
        assert e.value.code == L.FS_E_ARG
    finally:
        L.fs_destroy(ctx)


def test_full_size_solves_at_the_benchmark_configuration(L):
    """16^3 x 32 (eps 0.2, m0 0.02, c_sw 1.0), FP32 storage, batched, graph, even-odd at
    rhs block 4: sampled solutions verified by the oracle's FP64 clover residual."""
    dims = (16, 16, 16, 32)
    csw = 1.0
    V = lat.volume(dims)
    U = synth.gauge_field(dims, eps=0.2, seed=0)
    B = np.stack([z4_noise(V, 1, 0, 0, s) for s in range(2)])
    sig = [0.0, 1.0]
    ctx = L.fs_create(dims, 0, 0)
    try:
        L.fs_upload_gauge(ctx, U)
        L.fs_set_clover(ctx, csw)
        prm = L.solve_params(0.02, tol=1e-10, storage="f32", batched=1, rhs_block=4, use_graph=1, even_odd=1)
        print("clover cfg4-size solve", flush=True)
        X, _, code = L.fs_solve_shifted(ctx, prm, sig, B)
        assert code == 0
        C = cl.clover_term(U, dims, csw)
        for i, s in enumerate(sig):
            for r in range(2):
                res = np.linalg.norm(B[r] - cl.clover_apply(U, X[i, r], 0.02, s, csw, dims, C=C)) / np.linalg.norm(B[r])
                assert res <= 1.5e-10, (s, r, res)
        # the operator at full size, FP64, on one vector
        got = L.fs_apply_dirac(ctx, 0.02, 0.3, "f64", B[0])
        ref = cl.clover_apply(U, B[0], 0.02, 0.3, csw, dims, C=C)
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    finally:
        L.fs_destroy(ctx)


@pytest.mark.parametrize("storage,tol,ts", [("f64", 1e-12, 1e-9), ("f32", 1e-10, 1e-7)])
def test_sampling_generalized_expansion(L, storage, tol, ts):
    """The variance-sampling singles through the generalized hopping parameter
    expansion (A^-1 H)^4, A = C + a (Sec. 3.1), on the clover operator, against
    the oracle per sample."""
    dims = (4, 4, 4, 4)
    m0, csw = 0.1, 1.2
    U = synth.gauge_field(dims, eps=0.3, seed=0)
    shifts = [0.0, 0.3, 1.0]
    dense = ofs.DenseSolver(U, dims, m0, c_sw=csw)
    X_ref = ofs.sampling_samples(U, dims, shifts, 8, seed=3, gammas=list(range(16)), p_max=1, solver=dense,
                                 hpe_order=4)
    print(f"clover sampling hpe {storage}", flush=True)
    ctx = L.fs_create(dims, 0, 0)
    try:
        L.fs_upload_gauge(ctx, U)
        L.fs_set_clover(ctx, csw)
        sp = L.solve_params(m0, tol=tol, storage=storage, batched=1, rhs_block=4, use_graph=1, even_odd=1)
        prm = L.fs_est_params(3, 8, 0, 1, sp)
        prm.hpe_order = 4
        single, pair, X, _, rep = L.fs_sample_variances(ctx, prm, shifts, want_samples=True)
        assert rep.max_rel_residual <= tol
        scale = np.abs(X_ref).mean(axis=1)
        scale = np.where(scale > 0, scale, 1.0)
        assert (np.abs(X - X_ref).max(axis=1) / scale).max() <= ts
    finally:
        L.fs_destroy(ctx)
