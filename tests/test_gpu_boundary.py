"""Per-level outputs of the estimate boundary against the oracle (GPU).

* per-level sample counts N_l (eq. fs_trace_est with N_l of eq. num_samples),
  shared noise across levels, level totals (eqs. fs_trace_est, total_var,
  tosv) and eq. num_samples itself, each against the oracle;
* the a-posteriori error bound of every level holds sample by sample against
  dense-LU samples (FP64 and mixed-precision paths), and the reported
  deviation from the FP64 path equals the one measured by two separate calls.
"""

import numpy as np
import pytest

import synth
from oracle import fs as ofs

pytestmark = pytest.mark.gpu

DIMS = (4, 4, 4, 4)
SIG = [0.0, 0.5, 1.0]
M0 = 0.1


@pytest.fixture(scope="module")
def L():
    from paper_2212_04430_amd import _lib
    return _lib


@pytest.fixture(scope="module")
def cfg1():
    U = synth.gauge_field(DIMS, eps=0.3, seed=0)
    return U, ofs.DenseSolver(U, DIMS, M0)


def _ctx(L, U):
    ctx = L.fs_create(DIMS, 0, 0)
    L.fs_upload_gauge(ctx, U)
    return ctx


def _prm(L, n_noise, p_max, storage="f64", tol=1e-12, nr=4, eo=0, **kw):
    sp = L.solve_params(M0, tol=tol, storage=storage, batched=1, rhs_block=nr, use_graph=1, even_odd=eo)
    prm = L.fs_est_params(1, n_noise, 0, p_max, sp)
    for k, v in kw.items():
        setattr(prm, k, v)
    return prm


@pytest.mark.parametrize("eo", [0, 1])
def test_per_level_sample_counts(L, cfg1, eo):
    U, dense = cfg1
    nl = [7, 3, 5]
    print(f"per-level counts {nl} even_odd={eo}", flush=True)
    ctx = _ctx(L, U)
    try:
        prm = _prm(L, 99, 2, eo=eo).set_n_level(nl)
        stats, X, rep = L.fs_estimate(ctx, prm, SIG, want_samples=True)
        assert rep.systems == 2 * 7 + 2 * 3 + 5
        assert X.shape[1] == 7
        for l, n in enumerate(nl):
            Xr = ofs.fs_samples(U, DIMS, SIG, n, seed=1, gammas=list(range(16)), p_max=2, solver=dense,
                                levels=[l])[l]
            scale = np.abs(Xr).mean(axis=0)
            scale = np.where(scale > 0, scale, 1.0)
            assert (np.abs(X[l, :n] - Xr).max(axis=0) / scale).max() <= 1e-9
            assert np.all(X[l, n:] == 0)
            t, vp, vu = ofs.level_stats(Xr[None], axis=1)
            assert (np.abs(stats[l, ..., 0] + 1j * stats[l, ..., 1] - t[0]) / scale).max() <= 1e-10
            assert np.allclose(stats[l, ..., 2], vp[0], rtol=1e-6, atol=1e-12 * scale.max() ** 2)
            assert np.allclose(stats[l, ..., 3], vu[0], rtol=1e-6, atol=1e-12 * scale.max() ** 2)
            assert np.all(stats[l, ..., 4] == n)
        with pytest.raises(L.FsError) as e:
            L.fs_estimate(ctx, _prm(L, 4, 2).set_n_level([4, 0, 4]), SIG)
        assert e.value.code == L.FS_E_ARG
    finally:
        L.fs_destroy(ctx)


def test_shared_noise(L, cfg1):
    U, dense = cfg1
    ctx = _ctx(L, U)
    try:
        stats, X, _ = L.fs_estimate(ctx, _prm(L, 6, 1, shared_noise=1), SIG, want_samples=True)
    finally:
        L.fs_destroy(ctx)
    Xr = ofs.fs_samples(U, DIMS, SIG, 6, seed=1, gammas=list(range(16)), p_max=1, solver=dense, shared_noise=True)
    scale = np.abs(Xr).mean(axis=1)
    scale = np.where(scale > 0, scale, 1.0)
    assert (np.abs(X - Xr).max(axis=1) / scale).max() <= 1e-9


def test_level_totals_match_oracle_combination(L, cfg1):
    U, dense = cfg1
    nl = [6, 4, 9]
    ctx = _ctx(L, U)
    try:
        prm = _prm(L, 0, 1).set_n_level(nl)
        prm.gamma_mask = 0x0801  # Gamma_0 and Gamma_11
        stats, X, _, raw = L.fs_estimate(ctx, prm, SIG, want_samples=True, raw=True)
        tot = L.fs_level_totals(raw, len(SIG) - 1, 1)
    finally:
        L.fs_destroy(ctx)
    t_l = [X[l, :n].mean(axis=0) for l, n in enumerate(nl)]
    vp_l = [(np.abs(X[l, :n]) ** 2).mean(axis=0) - np.abs(t_l[l]) ** 2 for l, n in enumerate(nl)]
    vu_l = [vp_l[l] * n / (n - 1) for l, n in enumerate(nl)]
    t, v_fs, v_tot = ofs.fs_combine(np.array(t_l), np.array(vp_l), nl)
    _, v_fs_u, v_tot_u = ofs.fs_combine(np.array(t_l), np.array(vu_l), nl)
    for g in (0, 11):
        sc = np.abs(X[:, :, g]).mean() + 1e-300
        assert np.allclose(tot["tr"][g], t[g], rtol=0, atol=1e-12 * sc)
        assert np.allclose(tot["v_fs"][g], v_fs[g], rtol=1e-9, atol=1e-12 * sc ** 2)
        assert np.allclose(tot["v_total"][g], v_tot[g], rtol=1e-9, atol=1e-12 * sc ** 2)
        assert np.allclose(tot["v_fs_unbiased"][g], v_fs_u[g], rtol=1e-9, atol=1e-12 * sc ** 2)
        assert np.allclose(tot["v_total_unbiased"][g], v_tot_u[g], rtol=1e-9, atol=1e-12 * sc ** 2)
    off = [n for n in range(16) if n not in (0, 11)]
    assert np.all(tot["tr"][off] == 0) and np.all(tot["v_fs"][off] == 0)


def test_optimal_samples_match_oracle(L):
    rng = np.random.default_rng(7)
    for _ in range(6):
        n = int(rng.integers(1, 8))
        V = rng.uniform(0.01, 100.0, n)
        C = rng.uniform(1.0, 200.0, n)
        eps2 = float(rng.uniform(0.01, 1.0))
        N, mu = L.fs_optimal_samples(V, C, eps2, n_min=2)
        Nr, mur = ofs.optimal_samples(V, C, eps2)
        assert np.isclose(mu, mur, rtol=1e-12)
        assert np.array_equal(N, np.maximum(2, np.ceil(Nr)).astype(np.int32))
        assert np.sum(V / N) <= eps2 * (1 + 1e-12)
    with pytest.raises(L.FsError) as e:
        L.fs_optimal_samples([1.0, 2.0], [1.0, 0.0], 0.1)
    assert e.value.code == L.FS_E_ARG


@pytest.mark.parametrize("storage,tol", [("f64", 1e-10), ("f32", 1e-10), ("f16", 1e-10)])
def test_error_bound_holds_sample_by_sample(L, cfg1, storage, tol):
    """err_bound bounds |X_s - X_s^exact| for every sample of its level; X^exact
    from dense LU (its own error ~1e-14 relative is allowed on top)."""
    U, dense = cfg1
    n = 12
    print(f"error bound {storage}", flush=True)
    ctx = _ctx(L, U)
    try:
        prm = _prm(L, n, 3, storage=storage, tol=tol, report_fp64_error=1)
        stats, X, rep = L.fs_estimate(ctx, prm, SIG, want_samples=True)
        prm64 = _prm(L, n, 3, storage="f64", tol=tol)
        stats64, X64, _ = L.fs_estimate(ctx, prm64, SIG, want_samples=True)
    finally:
        L.fs_destroy(ctx)
    Xr = ofs.fs_samples(U, DIMS, SIG, n, seed=1, gammas=list(range(16)), p_max=3, solver=dense)
    bound = stats[..., 7]  # [L+1, 16, P1]
    assert np.all(np.isfinite(bound)) and np.all(bound > 0)
    dev = np.abs(X - Xr)  # [L+1, N, 16, P1]
    slack = 1e-12 * np.abs(Xr).max(axis=1)
    assert np.all(dev <= bound[:, None] + slack[:, None])
    ratio = (dev.max(axis=1) / bound).max()
    print(f"largest deviation / bound: {ratio:.2e}", flush=True)
    # the reported deviation from the FP64 path
    scale64 = np.abs(X64).mean(axis=1)
    t = stats[..., 0] + 1j * stats[..., 1]
    t64 = stats64[..., 0] + 1j * stats64[..., 1]
    want = np.abs(t - t64) / np.where(scale64 > 0, scale64, 1.0)
    if storage == "f64":
        assert np.all(stats[..., 6] == 0)
    else:
        assert np.allclose(stats[..., 6], want, rtol=1e-6, atol=1e-15)
        assert stats[..., 6].max() <= 1e-7


def test_last_error_per_context(L, cfg1):
    """fs_last_error(ctx) keeps the message of the last failing call on each
    context; fs_last_error(NULL) that of the last failing call on the thread."""
    U, _ = cfg1
    a = L.fs_create(DIMS, 0, 0)
    b = _ctx(L, U)
    try:
        assert L.fs_last_error(a) == "no error" and L.fs_last_error(b) == "no error"
        psi = synth.random_spinor(DIMS, seed=3)
        with pytest.raises(L.FsError) as e:
            L.fs_apply_dirac(a, M0, 0.0, "f64", psi)  # no gauge field on a
        assert e.value.code == L.FS_E_STATE
        msg_a = L.fs_last_error(a)
        assert "gauge" in msg_a and L.fs_last_error(None) == msg_a
        assert L.fs_last_error(b) == "no error"
        with pytest.raises(L.FsError) as e:
            L.fs_displace(b, -1, psi)
        assert e.value.code == L.FS_E_ARG
        msg_b = L.fs_last_error(b)
        assert "p must be" in msg_b and L.fs_last_error(None) == msg_b
        assert L.fs_last_error(a) == msg_a  # a keeps its own message
        L.fs_apply_dirac(b, M0, 0.0, "f64", psi)  # a call that succeeds leaves it
        assert L.fs_last_error(b) == msg_b
    finally:
        L.fs_destroy(a)
        L.fs_destroy(b)
