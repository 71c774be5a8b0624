"""GPU parity of the individual HIP kernels against the CPU oracle (via the C-ABI).

Tolerances (relative to max |reference|):
  FP64 dslash  1e-13   (rounding of ~100 flops per component)
  FP32 dslash  2e-6    (inputs and links rounded to FP32, FP32 accumulation)
  FP16 dslash  4e-3    (10-bit mantissa with a per-site scale on spinors)
  BF16 dslash  3e-2    (8-bit mantissa)
Noise and displacement indexing: bit-exact.
"""

import numpy as np
import pytest

import synth
from oracle import fs as ofs, lattice as lat
from oracle.philox import z4_noise

pytestmark = pytest.mark.gpu

DSLASH_TOL = {"f64": 1e-13, "f32": 2e-6, "f16": 4e-3, "bf16": 3e-2}


@pytest.fixture(scope="module")
def L():
    from paper_2212_04430_amd import _lib
    return _lib


def _ctx(L, dims, eps, seed=0, ap=False):
    ctx = L.fs_create(dims, int(ap), 0)
    U = synth.gauge_field(dims, eps=eps, seed=seed)
    L.fs_upload_gauge(ctx, U)
    return ctx, U


@pytest.mark.parametrize("dims,ap", [((4, 4, 4, 4), False), ((4, 4, 4, 4), True), ((6, 4, 2, 6), False),
                                     ((3, 5, 4, 2), True)])
@pytest.mark.parametrize("prec", ["f64", "f32", "f16", "bf16"])
def test_dslash_parity(L, dims, ap, prec):
    print(f"dslash parity dims={dims} ap={ap} prec={prec}", flush=True)
    ctx, U = _ctx(L, dims, 0.3, seed=1, ap=ap)
    try:
        psi = synth.random_spinor(dims, seed=2)
        ref = lat.wilson_apply(U, psi, 0.1, 0.35, dims, ap)
        got = L.fs_apply_dirac(ctx, 0.1, 0.35, prec, psi)
        err = np.abs(got - ref).max() / np.abs(ref).max()
        assert err <= DSLASH_TOL[prec], err
    finally:
        L.fs_destroy(ctx)


@pytest.mark.parametrize("n_rhs", [2, 4, 16, 48, 6])
def test_dslash_multi_rhs(L, n_rhs):
    """Blocks of right-hand sides sharing link loads (default block 4 for FP64, 8
    otherwise, halved down to n_rhs; a last partial block is zero-padded)."""
    dims = (4, 2, 6, 4)
    print(f"dslash multi-rhs n_rhs={n_rhs}", flush=True)
    ctx, U = _ctx(L, dims, 0.4, seed=3)
    try:
        psi = synth.random_spinor(dims, seed=4, n=n_rhs)
        for prec in ("f64", "f32"):
            got = L.fs_apply_dirac(ctx, 0.05, 0.2, prec, psi)
            for r in range(n_rhs):
                ref = lat.wilson_apply(U, psi[r], 0.05, 0.2, dims)
                assert np.abs(got[r] - ref).max() <= DSLASH_TOL[prec] * np.abs(ref).max()
    finally:
        L.fs_destroy(ctx)


def test_dslash_gamma5_hermiticity_on_device(L):
    dims = (8, 4, 4, 8)
    ctx, U = _ctx(L, dims, 0.5, seed=5, ap=True)
    try:
        u = synth.random_spinor(dims, seed=6)
        v = synth.random_spinor(dims, seed=7)
        Du = L.fs_apply_dirac(ctx, 0.1, 0.4, "f64", u)
        Dv = L.fs_apply_dirac(ctx, 0.1, 0.4, "f64", v)
        lhs = np.vdot(u.ravel(), lat.apply_gamma5(Dv).ravel())
        rhs = np.conj(np.vdot(v.ravel(), lat.apply_gamma5(Du).ravel()))
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    finally:
        L.fs_destroy(ctx)


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (5, 3, 7, 2), (16, 16, 16, 32)])
def test_z4_noise_bit_exact(L, dims):
    V = lat.volume(dims)
    ctx = L.fs_create(dims, 0, 0)
    try:
        for (seed, inst, level, sample) in [(1, 0, 0, 0), (1, 0, 3, 17), (2 ** 63 + 5, 7, 1, 2 ** 40)]:
            got = L.fs_z4_noise(ctx, V, seed, inst, level, sample)
            ref = z4_noise(V, seed, inst, level, sample)
            assert np.array_equal(got, ref), (seed, inst, level, sample)
    finally:
        L.fs_destroy(ctx)


def test_displacement_bit_exact_unit_links(L):
    dims = (3, 2, 5, 2)
    V = lat.volume(dims)
    ctx, U = _ctx(L, dims, 0.0)
    try:
        labels = np.arange(V * 12, dtype=np.float64).reshape(V, 4, 3) * (1 + 1j)
        for p in range(0, 7):
            got = L.fs_displace(ctx, p, labels)
            assert np.array_equal(got, lat.displace(U, labels, p, dims)), p
    finally:
        L.fs_destroy(ctx)


def test_displacement_random_links(L):
    dims = (4, 4, 6, 4)
    ctx, U = _ctx(L, dims, 0.6, seed=8)
    try:
        psi = synth.random_spinor(dims, seed=9)
        for p in (1, 3, 6):
            got = L.fs_displace(ctx, p, psi)
            ref = lat.displace(U, psi, p, dims)
            assert np.abs(got - ref).max() < 1e-14 * np.abs(ref).max()
    finally:
        L.fs_destroy(ctx)


def test_bilinear_all_gamma_and_p(L):
    dims = (4, 4, 8, 4)
    ctx, U = _ctx(L, dims, 0.5, seed=10)
    try:
        y = synth.random_spinor(dims, seed=11)
        x = synth.random_spinor(dims, seed=12)
        p_max = 7
        got = L.fs_bilinear(ctx, p_max, y, x)  # [p, n]
        ref = ofs.bilinears(U, dims, y, x, list(range(16)), p_max)  # [n, p]
        scale = np.abs(ref).max()
        assert np.abs(got.T - ref).max() <= 1e-13 * scale
    finally:
        L.fs_destroy(ctx)


def test_device_pointers_roundtrip(L):
    torch = pytest.importorskip("torch")
    dims = (4, 4, 4, 4)
    ctx, U = _ctx(L, dims, 0.3, seed=13)
    try:
        psi = synth.random_spinor(dims, seed=14)
        t = torch.from_numpy(psi).to("cuda")
        got = L.fs_apply_dirac(ctx, 0.1, 0.0, "f64", t).cpu().numpy()
        ref = lat.wilson_apply(U, psi, 0.1, 0.0, dims)
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    finally:
        L.fs_destroy(ctx)
