"""GPU parity of the LDS-tiled stencil (variant 2) against the CPU oracle.

The tiled variant stages each t-slice of a TX x TY x TZ tile in LDS and loads
only the tile faces' outside neighbours from memory.  The cases below force
it through fs_set_tuning on tiles with faces in every axis (T < L), tiles
spanning an axis (wrap-around inside LDS), several rhs blocks with a padded
last block, antiperiodic t, every storage precision, and a shape with no
valid tile (the column variant runs instead).  Tolerances are those of the
column variant: FP64 1e-13, FP32 2e-6, FP16 4e-3, BF16 3e-2 relative to
max |reference|.
"""

import numpy as np
import pytest

import synth
from oracle import fs as ofs, lattice as lat

pytestmark = pytest.mark.gpu

DSLASH_TOL = {"f64": 1e-13, "f32": 2e-6, "f16": 4e-3, "bf16": 3e-2}

# (dims, antiperiodic t, rhs_block, wg): tile chosen by the library
CASES = [
    ((8, 8, 8, 4), True, 1, 64),      # 4x4x4: faces in x, y, z
    ((8, 8, 8, 4), False, 4, 256),    # 4x4x4 x 4 rhs
    ((4, 8, 16, 6), True, 2, 128),    # 4x4x4: x spans the lattice, faces in y, z
    ((16, 4, 4, 2), False, 16, 256),  # 4x2x2 x 16 rhs
    ((4, 4, 8, 4), False, 8, 64),     # 2x2x2 x 8 rhs
    ((6, 4, 2, 6), True, 1, 64),      # no tile of 64 sites divides 6x4x2: column variant
]


@pytest.fixture(scope="module")
def L():
    from paper_2212_04430_amd import _lib
    return _lib


@pytest.mark.parametrize("dims,ap,nr,wg", CASES)
@pytest.mark.parametrize("prec", ["f64", "f32", "f16", "bf16"])
def test_tiled_dslash_parity(L, dims, ap, nr, wg, prec):
    n_rhs = 2 * nr + 1 if nr > 1 else 2  # several blocks, the last one padded
    print(f"tiled dslash dims={dims} ap={ap} nr={nr} wg={wg} prec={prec} n_rhs={n_rhs}", flush=True)
    ctx = L.fs_create(dims, int(ap), 0)
    try:
        U = synth.gauge_field(dims, eps=0.3, seed=11)
        L.fs_upload_gauge(ctx, U)
        L.fs_set_tuning(ctx, prec, nr, wg, 2, 0)
        psi = synth.random_spinor(dims, seed=12, n=n_rhs)
        got = L.fs_apply_dirac(ctx, 0.1, 0.27, prec, psi)
        for r in range(n_rhs):
            ref = lat.wilson_apply(U, psi[r], 0.1, 0.27, dims, ap)
            err = np.abs(got[r] - ref).max() / np.abs(ref).max()
            assert err <= DSLASH_TOL[prec], (r, err)
    finally:
        L.fs_destroy(ctx)


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_tiled_batched_solve_true_residual(L, prec):
    """Batched BiCGStab with the tiled stencil (FP64 reliable updates for the
    reduced precisions) reaches the FP64 true residual 1e-10 on every system."""
    dims = (8, 8, 8, 4)
    ctx = L.fs_create(dims, 1, 0)
    try:
        U = synth.gauge_field(dims, eps=0.3, seed=13)
        L.fs_upload_gauge(ctx, U)
        L.fs_set_tuning(ctx, prec, 4, 256, 2, 0)
        b = synth.random_spinor(dims, seed=14, n=6)
        sig = [0.0, 0.4]
        print(f"tiled solve prec={prec}", flush=True)
        prm = L.solve_params(0.05, tol=1e-10, storage=prec, batched=1, use_graph=1)
        X, st, code = L.fs_solve_shifted(ctx, prm, sig, b)
        assert code == L.FS_OK
        for i, s in enumerate(sig):
            for r in range(b.shape[0]):
                res = b[r] - lat.wilson_apply(U, X[i, r], 0.05, s, dims, True)
                assert np.linalg.norm(res) / np.linalg.norm(b[r]) <= 1.5e-10, (i, r)
    finally:
        L.fs_destroy(ctx)


def test_tiled_estimate_matches_dense_oracle(L):
    """The FS estimate of the 4x4x8x4 reduction of the 8^3x16 workload (eps 0.25,
    m0 0.05, shifts {0, .1, .4, 1.2}, all Gamma, p = 0..4, 8 Z4 vectors) with the
    2x2x2-tile stencil, against the dense-LU oracle sample by sample."""
    dims = (4, 4, 8, 4)
    U = synth.gauge_field(dims, eps=0.25, seed=0)
    sig = [0.0, 0.1, 0.4, 1.2]
    X_ref = ofs.fs_samples(U, dims, sig, 8, seed=1, gammas=list(range(16)), p_max=4,
                           solver=ofs.DenseSolver(U, dims, 0.05))
    scale = np.abs(X_ref).mean(axis=1)
    scale = np.where(scale > 0, scale, 1.0)
    ctx = L.fs_create(dims, 0, 0)
    try:
        L.fs_upload_gauge(ctx, U)
        for storage, tol, ts in (("f64", 1e-12, 1e-9), ("f32", 1e-10, 1e-7)):
            print(f"tiled estimate {storage}", flush=True)
            L.fs_set_tuning(ctx, storage, 8, 64, 2, 0)
            sp = L.solve_params(0.05, tol=tol, storage=storage, batched=1, rhs_block=8, use_graph=1)
            stats, X, _ = L.fs_estimate(ctx, L.fs_est_params(1, 8, 0, 4, sp), sig, want_samples=True)
            dev = np.abs(X - X_ref).max(axis=1) / scale
            assert dev.max() <= ts, (storage, dev.max())
    finally:
        L.fs_destroy(ctx)


@pytest.mark.parametrize("prec", ["f32", "f16", "bf16"])
def test_variants_converge_alike_at_full_size(L, prec):
    """On the 16^3x32 workload lattice every stencil variant gives the same
    solver: each system reaches the FP64 true residual 1e-10 and the mean
    iteration count stays within 25% of the register-rich column variant's
    (reduced-precision rounding differs by variant, the operator does not)."""
    dims = (16, 16, 16, 32)
    ctx = L.fs_create(dims, 0, 0)
    try:
        U = synth.gauge_field(dims, eps=0.2, seed=0)
        L.fs_upload_gauge(ctx, U)
        b = synth.random_spinor(dims, seed=15, n=4)
        sig = [0.0, 0.25]
        iters = {}
        for var in (1, 0, 2):
            print(f"full-size solve prec={prec} variant={var}", flush=True)
            L.fs_set_tuning(ctx, prec, 4, 256, var, 0)
            prm = L.solve_params(0.02, tol=1e-10, storage=prec, batched=1, use_graph=1, max_iter=2000)
            X, st, code = L.fs_solve_shifted(ctx, prm, sig, b)
            assert code == L.FS_OK, var
            assert max(s.true_rel_residual for s in st) <= 1e-10, var
            iters[var] = np.mean([s.iters for s in st])
            res = b[1] - lat.wilson_apply(U, X[1, 1], 0.02, sig[1], dims)
            assert np.linalg.norm(res) / np.linalg.norm(b[1]) <= 1.5e-10, var
        for var in (0, 2):
            assert iters[var] <= 1.25 * iters[1], iters
    finally:
        L.fs_destroy(ctx)
