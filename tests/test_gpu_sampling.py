"""GPU variance-sampling phase (Sec. 3.1) against the CPU oracle.

fs_sample_variances draws one Z4 vector per sample (shared by every sampling
shift) and returns, per sample, z^dagger Gamma Omega_p x_i (V_L(s_i)) and
y_i^dagger Gamma Omega_p x_j for j >= i (Vbar_l(s_i, s_j)), together with the
mean and eq. practical_variance of each.  On small lattices the samples are
compared one by one with the dense-LU oracle, per sample at 1e-9 of mean
|X_s| for FP64 solves to 1e-12 and at 1e-7 for reduced storage solved to the
FP64 residual 1e-10.  At the 16^3x32 workload size, where the oracle cannot
solve, two properties that hold sample by sample are checked instead:
* the resolvent identity (D+s_i)^-1 - (D+s_j)^-1 = (s_j - s_i)(D+s_i)^-1(D+s_j)^-1
  at Gamma = 1, p = 0 links the singles of s_i and s_j to the pair (i, j);
* gamma5 (D+s)^-1 is Hermitian, so z^dagger gamma5 (D+s)^-1 z (Gamma_15, p = 0)
  is real.
"""

import numpy as np
import pytest

import synth
from oracle import fs as ofs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_2212_04430_amd import _lib
    return _lib


def _params(L, m0, n_noise, p_max, storage="f64", tol=1e-12, nr=0, seed=3):
    sp = L.solve_params(m0, tol=tol, storage=storage, batched=1, rhs_block=nr, use_graph=1)
    return L.fs_est_params(seed, n_noise, 0, p_max, sp)


def _slot_of(m, i, j):
    return ofs.sampling_slots(m).index(("pair", i, j))


def _check(L, single, pair, X, X_ref, m, tol):
    scale = np.abs(X_ref).mean(axis=1)
    scale = np.where(scale > 0, scale, 1.0)
    dev = np.abs(X - X_ref).max(axis=1) / scale
    assert dev.max() <= tol, dev.max()
    t_ref, vp_ref, vu_ref = ofs.level_stats(X_ref, axis=1)
    for q, (kind, i, j) in enumerate(ofs.sampling_slots(m)):
        st = single[i] if kind == "single" else pair[i, j]
        assert (np.abs(st[..., 0] + 1j * st[..., 1] - t_ref[q]) / scale[q]).max() <= tol, (kind, i, j)
        assert np.allclose(st[..., 2], vp_ref[q], rtol=1e-6, atol=1e-12 * scale[q].max() ** 2)
        assert np.allclose(st[..., 3], vu_ref[q], rtol=1e-6, atol=1e-12 * scale[q].max() ** 2)
    for i in range(m):
        for j in range(i):
            assert np.all(pair[i, j] == 0)


@pytest.fixture(scope="module")
def ref_4444():
    """4^4, eps 0.3, m0 0.1, sampling shifts {0, 0.3, 1.0}, 12 Z4 vectors, all Gamma, p <= 2."""
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, eps=0.3, seed=5)
    shifts = [0.0, 0.3, 1.0]
    dense = ofs.DenseSolver(U, dims, 0.1)
    X = ofs.sampling_samples(U, dims, shifts, 12, seed=3, gammas=list(range(16)), p_max=2, solver=dense)
    return dims, U, shifts, X


@pytest.mark.parametrize("nr", [4, 8, 16])  # 3 full blocks; a padded last block; one block, 4 idle
def test_sampling_fp64_per_sample_parity(L, ref_4444, nr):
    dims, U, shifts, X_ref = ref_4444
    print(f"sampling fp64 nr={nr}", flush=True)
    ctx = L.fs_create(dims, 0, 0)
    try:
        L.fs_upload_gauge(ctx, U)
        single, pair, X, iters, rep = L.fs_sample_variances(ctx, _params(L, 0.1, 12, 2, nr=nr), shifts,
                                                     want_samples=True)
        assert rep.systems == 2 * 3 * 12 and rep.max_rel_residual <= 1e-12
        assert np.all(iters > 0) and abs(iters.sum() * 24 - rep.iterations) < 1e-6 * rep.iterations
        assert np.all(np.diff(iters) <= 0.5)  # larger shifts converge no slower (within rounding)
        _check(L, single, pair, X, X_ref, 3, 1e-9)
        assert np.all(single[..., 4] == 12)
    finally:
        L.fs_destroy(ctx)


@pytest.mark.parametrize("prec", ["f32", "f16", "bf16"])
def test_sampling_mixed_precision_parity(L, ref_4444, prec):
    dims, U, shifts, X_ref = ref_4444
    print(f"sampling {prec}", flush=True)
    ctx = L.fs_create(dims, 0, 0)
    try:
        L.fs_upload_gauge(ctx, U)
        single, pair, X, iters, rep = L.fs_sample_variances(ctx, _params(L, 0.1, 12, 2, storage=prec, tol=1e-10, nr=4),
                                                     shifts, want_samples=True)
        assert rep.max_rel_residual <= 1e-10
        _check(L, single, pair, X, X_ref, 3, 1e-7)
    finally:
        L.fs_destroy(ctx)


def test_sampling_paper_shift_count_mini(L):
    """Seven sampling shifts (as many as the paper's shift set has values) on
    4x4x8x4 with the tiled stencil: 7 singles and 28 pairs."""
    dims = (4, 4, 8, 4)
    U = synth.gauge_field(dims, eps=0.25, seed=0)
    shifts = [0.0, 1e-5, 0.053, 0.146, 0.360, 0.618, 1.0]
    X_ref = ofs.sampling_samples(U, dims, shifts, 4, seed=3, gammas=list(range(16)), p_max=3,
                                 solver=ofs.DenseSolver(U, dims, 0.05))
    ctx = L.fs_create(dims, 0, 0)
    try:
        L.fs_upload_gauge(ctx, U)
        L.fs_set_tuning(ctx, "f32", 4, 64, 2, 0)
        print("sampling 7 shifts f32 tiled", flush=True)
        single, pair, X, iters, rep = L.fs_sample_variances(ctx, _params(L, 0.05, 4, 3, storage="f32", tol=1e-10),
                                                     shifts, want_samples=True)
        assert X.shape[0] == 7 + 28
        _check(L, single, pair, X, X_ref, 7, 1e-7)
    finally:
        L.fs_destroy(ctx)


def test_sampling_argument_errors(L):
    dims = (4, 4, 4, 4)
    ctx = L.fs_create(dims, 0, 0)
    try:
        L.fs_upload_gauge(ctx, synth.gauge_field(dims, eps=0.3, seed=0))
        prm = _params(L, 0.1, 4, 1)
        for bad in ([0.1, 0.5], [0.0, 0.5, 0.5], [0.0, 1.0, 0.5], [], list(np.linspace(0, 1, 17))):
            with pytest.raises(L.FsError) as e:
                L.fs_sample_variances(ctx, prm, bad)
            assert e.value.code == L.FS_E_ARG, bad
        prm.n_noise = 1
        with pytest.raises(L.FsError) as e:
            L.fs_sample_variances(ctx, prm, [0.0, 0.5])
        assert e.value.code == L.FS_E_ARG
        prm.n_noise = 4
        prm.p_max = 4  # Lz = 4
        with pytest.raises(L.FsError) as e:
            L.fs_sample_variances(ctx, prm, [0.0, 0.5])
        assert e.value.code == L.FS_E_ARG
    finally:
        L.fs_destroy(ctx)


def test_sampling_full_size_identities(L):
    """16^3x32, eps 0.2, m0 0.02, shifts {0, 0.1, 0.5}, 8 Z4 vectors, FP16 storage
    with FP64 reliable updates to the FP64 residual 1e-10."""
    dims = (16, 16, 16, 32)
    shifts = [0.0, 0.1, 0.5]
    ctx = L.fs_create(dims, 0, 0)
    try:
        L.fs_upload_gauge(ctx, synth.gauge_field(dims, eps=0.2, seed=0))
        print("sampling full size f16", flush=True)
        prm = _params(L, 0.02, 8, 2, storage="f16", tol=1e-10)
        prm.solve.max_iter = 20000
        single, pair, X, iters, rep = L.fs_sample_variances(ctx, prm, shifts, want_samples=True)
        assert rep.systems == 2 * 3 * 8 and rep.max_rel_residual <= 1e-10
        m = len(shifts)
        for i in range(m):
            for j in range(i + 1, m):
                lhs = X[i, :, 0, 0] - X[j, :, 0, 0]
                rhs = (shifts[j] - shifts[i]) * X[_slot_of(m, i, j), :, 0, 0]
                assert np.abs(lhs - rhs).max() <= 1e-6 * np.abs(X[i, :, 0, 0]).max(), (i, j)
            g5 = X[i, :, 15, 0]
            assert np.abs(g5.imag).max() <= 1e-5 * np.abs(g5.real).max(), i
    finally:
        L.fs_destroy(ctx)


@pytest.mark.parametrize("m0,storage,tol,ts", [(-0.1, "f64", 1e-12, 1e-9), (0.2, "f64", 1e-12, 1e-9),
                                                (0.2, "f32", 1e-10, 1e-7)])
def test_hopping_expansion_singles(L, m0, storage, tol, ts):
    """Order-4 expansion of the V_L samples (Sec. 3.1): the singles of shifts with
    m0 + s > 0 are z^+ Gamma Omega_p (H/a)^4 x, the others and the pairs unchanged.
    At m0 = -0.1 only the shifts 0.25 and 0.5 qualify."""
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, eps=0.3, seed=5)
    shifts = [0.0, 0.05, 0.25, 0.5]
    dense = ofs.DenseSolver(U, dims, m0)
    X_ref = ofs.sampling_samples(U, dims, shifts, 8, seed=3, gammas=list(range(16)), p_max=2, solver=dense,
                                 hpe_order=4)
    print(f"sampling hpe m0={m0} {storage}", flush=True)
    ctx = L.fs_create(dims, 0, 0)
    try:
        L.fs_upload_gauge(ctx, U)
        prm = _params(L, m0, 8, 2, storage=storage, tol=tol, nr=4)
        prm.hpe_order = 4
        single, pair, X, _, rep = L.fs_sample_variances(ctx, prm, shifts, want_samples=True)
        assert rep.max_rel_residual <= tol
        _check(L, single, pair, X, X_ref, len(shifts), ts)
        prm.hpe_order = 0
        _, _, X0, _, _ = L.fs_sample_variances(ctx, prm, shifts, want_samples=True)
        for i, s in enumerate(shifts):
            same = np.array_equal(X[i], X0[i])
            assert same == (not ofs.hpe_eligible(m0, s)), (i, s)
        assert np.array_equal(X[len(shifts):], X0[len(shifts):])
        # the order is rejected where it does not apply
        prm.hpe_order = 4
        with pytest.raises(L.FsError) as e:
            L.fs_estimate(ctx, prm, [0.0, 0.5])
        assert e.value.code == L.FS_E_ARG
        prm.hpe_order = 17
        with pytest.raises(L.FsError) as e:
            L.fs_sample_variances(ctx, prm, shifts)
        assert e.value.code == L.FS_E_ARG
    finally:
        L.fs_destroy(ctx)


@pytest.mark.parametrize("nr", [4, 16])
def test_sampling_multishift_per_sample_parity(L, ref_4444, nr):
    """The sampling solves by multi-shift BiCGStab (one Krylov space per sample and
    family for every sampling shift): the same per-sample parity as independent solves."""
    dims, U, shifts, X_ref = ref_4444
    print(f"sampling multishift nr={nr}", flush=True)
    ctx = L.fs_create(dims, 0, 0)
    try:
        L.fs_upload_gauge(ctx, U)
        prm = _params(L, 0.1, 12, 2, nr=nr)
        prm.solve.multi_shift = 1
        single, pair, X, iters, rep = L.fs_sample_variances(ctx, prm, shifts, want_samples=True)
        assert rep.systems == 2 * 3 * 12 and rep.max_rel_residual <= 1e-12
        assert iters[0] == max(iters) and np.all(np.diff(iters) <= 0)  # each shift's own Krylov steps
        _check(L, single, pair, X, X_ref, 3, 1e-9)
        prm.solve.storage = 2  # FP16: rejected
        with pytest.raises(L.FsError) as e:
            L.fs_sample_variances(ctx, prm, shifts)
        assert e.value.code == L.FS_E_ARG
    finally:
        L.fs_destroy(ctx)
