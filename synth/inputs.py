"""Synthetic, deterministic inputs with the shapes of the paper's workloads.

The paper runs on a 32^3 x 64 clover ensemble (Results section) that is not
available; weak random SU(3) fields stand in for it.  Each link is

    U = exp(i * eps * H),   H = sum_{a=1..8} h_a * lambda_a / 2,   h_a ~ N(0, 1)

with lambda_a the Gell-Mann matrices.  H is Hermitian and traceless, so U is
unitary with det U = 1 up to rounding.  The exponential is taken through the
eigendecomposition of H: U = V diag(exp(i eps e_k)) V^dagger.

Random numbers come from numpy's Philox bit generator keyed by the seed and a
stream tag, so every array is reproducible on any machine.
"""

import numpy as np

_TAG_GAUGE = 1
_TAG_SPINOR = 2
_TAG_GTRANS = 3


def volume(dims):
    """Number of lattice sites for dims = (Lx, Ly, Lz, Lt)."""
    v = 1
    for d in dims:
        v *= int(d)
    return v


def _rng(seed, tag, stream=0):
    key = np.array([int(seed) & 0xFFFFFFFFFFFFFFFF, (int(tag) << 32) | int(stream)],
                   dtype=np.uint64)
    return np.random.Generator(np.random.Philox(key=key))


def gell_mann():
    """The eight Gell-Mann matrices lambda_1..lambda_8, shape (8, 3, 3)."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1] = -1j
    lam[1][1, 0] = 1j
    lam[2][0, 0] = 1
    lam[2][1, 1] = -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2] = -1j
    lam[4][2, 0] = 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2] = -1j
    lam[6][2, 1] = 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3)
    lam[7][2, 2] = -2 / np.sqrt(3)
    return lam


def su3_exp_field(n, eps, rng, chunk=1 << 20):
    """n matrices exp(i eps H) with H = sum h_a lambda_a / 2, h_a ~ N(0,1)."""
    lam = gell_mann() / 2.0
    out = np.empty((n, 3, 3), dtype=np.complex128)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        h = rng.standard_normal((hi - lo, 8))
        H = np.einsum('na,aij->nij', h, lam)
        # Symmetrise away rounding so eigh sees an exactly Hermitian matrix.
        H = 0.5 * (H + np.conj(np.swapaxes(H, 1, 2)))
        w, v = np.linalg.eigh(H)
        ph = np.exp(1j * eps * w)
        out[lo:hi] = (v * ph[:, None, :]) @ np.conj(np.swapaxes(v, 1, 2))
    return out


def gauge_field(dims, eps, seed=0):
    """Gauge links in canonical layout (4, V, 3, 3); eps = 0 gives unit links."""
    V = volume(dims)
    if eps == 0.0:
        U = np.zeros((4, V, 3, 3), dtype=np.complex128)
        U[:, :, 0, 0] = U[:, :, 1, 1] = U[:, :, 2, 2] = 1.0
        return U
    rng = _rng(seed, _TAG_GAUGE)
    return su3_exp_field(4 * V, eps, rng).reshape(4, V, 3, 3)


def random_spinor(dims, seed=0, n=None, stream=0):
    """Gaussian complex spinor field(s): (V, 4, 3), or (n, V, 4, 3) if n given."""
    V = volume(dims)
    rng = _rng(seed, _TAG_SPINOR, stream)
    shape = (V, 4, 3) if n is None else (n, V, 4, 3)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) / np.sqrt(2.0)


def gauge_transform(dims, seed=0, eps=3.0):
    """Random per-site SU(3) matrices g(x), shape (V, 3, 3)."""
    V = volume(dims)
    rng = _rng(seed, _TAG_GTRANS)
    return su3_exp_field(V, eps, rng)
