"""Uneven-lattice batches at full size, reproducibility and failure handling (GPU).

* Uneven batch with the lattice sizes 8^3x16, 12^3x24, 16^3x32 and 24^3x48 and the
  paper's six-shift set (Results section: sigma = [0, 1e-5, 0.053, 0.146,
  0.360, 0.618, 1.0]), FP16 storage with FP64 reliable updates: every level
  meets the FP64 residual bound and each instance's statistics equal those of
  the same instance estimated alone (both solved to 1e-10, so they agree to
  ~kappa * 1e-10 of the sample scale; asserted at 1e-6).
* Passes: a batch split into several passes (pass_bytes) gives the samples of
  the one-pass estimate to the solver tolerance, every system solved once.
* Reproducibility: reductions are summed in a fixed order, so two estimates
  of the same inputs are bit-identical, in every storage precision.
* Failure handling, forced from the host: a source orthogonal to the solver's
  shadow residual (BiCGStab breakdown, restart from a fresh shadow residual)
  and a NaN link (no hang, FS_E_NOCONV with the status set).
"""

import numpy as np
import pytest

import synth
from oracle import lattice as lat
from oracle.philox import z4_noise

pytestmark = pytest.mark.gpu

SIGMA_PAPER = [0.0, 1e-5, 0.053, 0.146, 0.360, 0.618, 1.0]


@pytest.fixture(scope="module")
def L():
    from paper_2212_04430_amd import _lib
    return _lib


def test_uneven_batch_full_size_half_precision(L):
    shapes = [(8, 8, 8, 16), (12, 12, 12, 24), (16, 16, 16, 32), (24, 24, 24, 48)]
    ctxs = []
    try:
        for k, d in enumerate(shapes):
            print(f"instance {k}: {d}", flush=True)
            c = L.fs_create(d, 0, 0)
            L.fs_set_instance(c, k)
            L.fs_upload_gauge(c, synth.gauge_field(d, eps=0.2, seed=k))
            ctxs.append(c)
        sp = L.solve_params(0.02, tol=1e-10, storage="f16", batched=1, use_graph=1, max_iter=20000)
        prm = L.fs_est_params(1, 4, 0, 2, sp)
        batch = L.fs_batch_create(ctxs)
        try:
            print("batch estimate", flush=True)
            stats, rep = L.fs_batch_estimate(batch, len(ctxs), prm, SIGMA_PAPER)
        finally:
            L.fs_batch_destroy(batch)
        assert rep.systems == 4 * len(ctxs) * (2 * 6 + 1)
        assert rep.max_rel_residual <= 1e-10
        assert np.all(stats[..., 5] <= 1e-10)
        for k, c in enumerate(ctxs):
            print(f"single estimate {k}", flush=True)
            single, _, _ = L.fs_estimate(c, prm, SIGMA_PAPER)
            scale = np.sqrt(single[..., 2] + single[..., 0] ** 2 + single[..., 1] ** 2)
            scale = np.where(scale > 0, scale, 1.0)
            dev = np.abs((stats[k][..., 0] - single[..., 0]) + 1j * (stats[k][..., 1] - single[..., 1])) / scale
            assert dev.max() <= 1e-6, (k, dev.max())
    finally:
        for c in ctxs:
            L.fs_destroy(c)


@pytest.mark.parametrize("storage,tol", [("f64", 1e-8), ("f32", 1e-6)])
def test_batch_estimate_in_passes_matches_one_pass(L, storage, tol):
    """A pass bound (pass_bytes) below the batch's need splits the systems into
    passes: rhs-block chunks of every (instance, level) dealt by chunk index
    (two passes here), or one chunk per pass (a bound of one byte).  Every
    sample must agree with the one-pass estimate to the solver tolerance (the
    passes change only the workgroup split of the FP64 dot products), and every
    system is solved exactly once."""
    shapes = [(4, 4, 4, 4), (4, 4, 8, 4), (6, 4, 4, 4)]
    sigma = [0.0, 0.3, 1.0]
    nr, n = 2, 8
    ctxs = []
    try:
        for k, d in enumerate(shapes):
            c = L.fs_create(d, 0, 0)
            L.fs_set_instance(c, k)
            L.fs_upload_gauge(c, synth.gauge_field(d, eps=0.3, seed=10 + k))
            ctxs.append(c)
        batch = L.fs_batch_create(ctxs)
        try:
            sp = L.solve_params(0.1, tol=1e-10, storage=storage, batched=1, use_graph=1, rhs_block=nr,
                                even_odd=1)
            prm = L.fs_est_params(1, n, 0, 2, sp)
            st1, X1, rep1 = L.fs_batch_estimate(batch, len(ctxs), prm, sigma, want_samples=True)
            # the library's estimate of a pass's device memory: per site and system
            # 4 FP64 spinors and 6 in the storage precision (+ FP16 scales)
            low = {"f64": 192, "f32": 96}[storage]
            per_site = 4 * 192 + 6 * low
            Lv = len(sigma) - 1
            need = sum(int(np.prod(d)) * per_site * nr * (2 if l < Lv else 1) * ((n + nr - 1) // nr)
                       for d in shapes for l in range(Lv + 1))
            for pb in (need // 2 + 1, 1):
                print(f"{storage}: pass_bytes {pb} (one-pass need {need})", flush=True)
                prm.pass_bytes = pb
                st2, X2, rep2 = L.fs_batch_estimate(batch, len(ctxs), prm, sigma, want_samples=True)
                assert rep2.systems == rep1.systems == len(shapes) * n * (2 * Lv + 1)
                assert rep2.max_rel_residual <= 1e-10
                scale = np.abs(X1).mean(axis=2, keepdims=True)
                scale = np.where(scale > 0, scale, 1.0)
                dev = (np.abs(X2 - X1) / scale).max()
                assert dev <= tol, (pb, dev)
                assert np.allclose(st2[..., 4], st1[..., 4])  # sample counts
        finally:
            L.fs_batch_destroy(batch)
    finally:
        for c in ctxs:
            L.fs_destroy(c)


def test_estimates_are_bit_reproducible(L):
    dims = (8, 8, 8, 16)
    c = L.fs_create(dims, 0, 0)
    try:
        L.fs_upload_gauge(c, synth.gauge_field(dims, eps=0.25, seed=0))
        for storage in ("f64", "f32", "f16", "bf16"):
            sp = L.solve_params(0.05, tol=1e-10, storage=storage, batched=1, use_graph=1)
            prm = L.fs_est_params(3, 8, 0, 4, sp)
            s1, X1, _ = L.fs_estimate(c, prm, [0.0, 0.1, 0.4, 1.2], want_samples=True)
            s2, X2, _ = L.fs_estimate(c, prm, [0.0, 0.1, 0.4, 1.2], want_samples=True)
            assert np.array_equal(X1, X2) and np.array_equal(s1, s2), storage
    finally:
        L.fs_destroy(c)


def test_breakdown_restart_source_orthogonal_to_shadow_residual(L):
    """b is orthogonalised against the shadow residual of system 0 of
    fs_solve_shifted (the Z4 stream with seed 0x5A4E4F4953452121, instance
    0x40000000, level 0, sample 0): rho_0 = 0, BiCGStab breaks down at once
    and must restart from a fresh shadow residual."""
    dims = (4, 4, 4, 4)
    V = lat.volume(dims)
    U = synth.gauge_field(dims, eps=0.3, seed=0)
    c = L.fs_create(dims, 0, 0)
    try:
        L.fs_upload_gauge(c, U)
        rhat = z4_noise(V, 0x5A4E4F4953452121, 0x40000000, 0, 0)
        b = synth.random_spinor(dims, seed=21)
        b = b - np.vdot(rhat.ravel(), b.ravel()) / np.vdot(rhat.ravel(), rhat.ravel()) * rhat
        assert abs(np.vdot(rhat.ravel(), b.ravel())) < 1e-12 * np.linalg.norm(b) * np.linalg.norm(rhat)
        for storage in ("f64", "f32"):
            prm = L.solve_params(0.1, tol=1e-10, storage=storage, batched=1, rhs_block=1)
            X, st, code = L.fs_solve_shifted(c, prm, [0.0], b[None])
            assert code == L.FS_OK
            if storage == "f64":  # FP32 rounding of b leaves a small projection on rhat
                assert st[0].restarts >= 1, st[0].restarts
            r = b - lat.wilson_apply(U, X[0, 0], 0.1, 0.0, dims)
            assert np.linalg.norm(r) / np.linalg.norm(b) <= 1.5e-10
    finally:
        L.fs_destroy(c)


def test_nan_link_reports_failure_without_hanging(L):
    dims = (4, 4, 4, 4)
    V = lat.volume(dims)
    U = synth.gauge_field(dims, eps=0.3, seed=0)
    U[1, 17, 0, 2] = np.nan
    c = L.fs_create(dims, 0, 0)
    try:
        L.fs_upload_gauge(c, U)
        b = z4_noise(V, 1, 0, 0, 0)[None]
        for storage, batched in (("f64", 0), ("f32", 1)):
            prm = L.solve_params(0.1, tol=1e-10, storage=storage, batched=batched, max_iter=200)
            X, st, code = L.fs_solve_shifted(c, prm, [0.0], b, allow_noconv=True)
            assert code == L.FS_E_NOCONV and st[0].status == L.FS_E_NOCONV
            assert not (st[0].true_rel_residual <= 1e-10)
    finally:
        L.fs_destroy(c)
