"""Pins of the oracle's clover term (CPU).

The clover-improved operator is the one of the Results section; its
conventions are a reading (see oracle/clover.py).  These checks tie the
oracle to facts that do not depend on its own formulas: c_sw = 0 is the Wilson
operator, a pure-gauge field has no field strength, a constant abelian field
has the closed-form field strength of its plaquette angle, the clover leaves
equal products of links along walked paths, and the sign of the term is the
one that cancels the O(a) shift that the Wilson term gives the would-be zero
modes of a constant abelian field (tree-level improvement).
"""

import numpy as np
import pytest

import synth
from oracle import clover as cl, lattice as lat


def _random_su3(rng, n):
    z = (rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))) / np.sqrt(2)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=1, axis2=2)
    q = q * (d / np.abs(d))[:, None, :]
    return q / np.linalg.det(q)[:, None, None] ** (1.0 / 3.0)


def _gauge_transform(U, g, dims):
    """U_mu(x) -> g(x) U_mu(x) g(x + mu)^dagger."""
    V = lat.volume(dims)
    out = np.empty_like(U)
    for s in range(V):
        c = list(lat.site_coords(s, dims))
        for mu in range(4):
            cf = list(c)
            cf[mu] = (cf[mu] + 1) % dims[mu]
            out[mu, s] = g[s] @ U[mu, s] @ np.conj(g[lat.site_index(*cf, dims)]).T
    return out


def _abelian_field(dims, k, charges):
    """Constant field in the x-y plane: every x-y plaquette equals diag(exp(i q_c theta)),
    theta = 2 pi k / (Lx Ly) (the flux through the periodic plane is quantised)."""
    Lx, Ly = dims[0], dims[1]
    th = 2 * np.pi * k / (Lx * Ly)
    q = np.asarray(charges, float)
    V = lat.volume(dims)
    U = np.tile(np.eye(3, dtype=np.complex128), (4, V, 1, 1))
    for s in range(V):
        x, y, _, _ = lat.site_coords(s, dims)
        U[1, s] = np.diag(np.exp(1j * q * th * x))
        if x == Lx - 1:
            U[0, s] = np.diag(np.exp(-1j * q * th * Lx * y))
    return U, th


def _walk(U, dims, s, path):
    """Ordered link product along a path of steps (+/-(mu + 1)) starting at site s."""
    c = list(lat.site_coords(s, dims))
    m = np.eye(3, dtype=np.complex128)
    for step in path:
        mu = abs(step) - 1
        if step > 0:
            m = m @ U[mu, lat.site_index(*c, dims)]
            c[mu] = (c[mu] + 1) % dims[mu]
        else:
            c[mu] = (c[mu] - 1) % dims[mu]
            m = m @ np.conj(U[mu, lat.site_index(*c, dims)]).T
    return m


def test_csw_zero_is_wilson():
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, eps=0.3, seed=0)
    rng = np.random.default_rng(1)
    psi = rng.standard_normal((lat.volume(dims), 4, 3)) + 1j * rng.standard_normal((lat.volume(dims), 4, 3))
    a = cl.clover_apply(U, psi, 0.1, 0.3, 0.0, dims)
    b = lat.wilson_apply(U, psi, 0.1, 0.3, dims)
    assert np.array_equal(a, b)


def test_leaves_match_walked_paths():
    dims = (4, 2, 4, 2)
    U = synth.gauge_field(dims, eps=0.6, seed=3)
    for mu, nu in cl.plane_pairs():
        Q = cl.clover_leaves(U, dims, mu, nu).reshape(-1, 3, 3)
        a, b = mu + 1, nu + 1
        for s in (0, 5, 17, lat.volume(dims) - 1):
            ref = sum(_walk(U, dims, s, p) for p in ([a, b, -a, -b], [b, -a, -b, a],
                                                      [-a, -b, a, b], [-b, a, b, -a]))
            assert np.abs(Q[s] - ref).max() < 1e-13, (mu, nu, s)


def test_pure_gauge_has_no_field_strength():
    dims = (4, 4, 2, 4)
    rng = np.random.default_rng(7)
    one = np.tile(np.eye(3, dtype=np.complex128), (4, lat.volume(dims), 1, 1))
    U = _gauge_transform(one, _random_su3(rng, lat.volume(dims)), dims)
    assert np.abs(cl.field_strength(U, dims)).max() < 1e-13
    psi = rng.standard_normal((lat.volume(dims), 4, 3)) + 0j
    assert np.allclose(cl.clover_apply(U, psi, 0.1, 0.0, 1.7, dims), lat.wilson_apply(U, psi, 0.1, 0.0, dims),
                       atol=1e-13, rtol=0)


@pytest.mark.parametrize("charges", [(1, -1, 0), (1, 1, -2)])
def test_constant_abelian_field_closed_form(charges):
    dims = (4, 4, 2, 2)
    U, th = _abelian_field(dims, 1, charges)
    F = cl.field_strength(U, dims).reshape(6, -1, 3, 3)
    f = np.sin(np.asarray(charges) * th)
    f = f - f.mean()  # traceless part
    assert np.abs(F[0] - np.diag(f)).max() < 1e-14  # the x-y plane
    assert np.abs(F[1:]).max() < 1e-14
    C = cl.clover_term(U, dims, 1.3)
    ref = -0.65 * np.kron(cl.sigma_munu(0, 1), np.diag(f))
    assert np.abs(C - ref).max() < 1e-14


def test_sigma_and_clover_symmetries():
    _, g5 = lat.gammas()
    for mu, nu in cl.plane_pairs():
        s = cl.sigma_munu(mu, nu)
        assert np.allclose(s, s.conj().T) and np.allclose(s @ s, np.eye(4)) and np.allclose(s @ g5, g5 @ s)
    dims = (4, 4, 4, 2)
    U = synth.gauge_field(dims, eps=0.5, seed=2)
    F = cl.field_strength(U, dims)
    assert np.abs(F - np.conj(np.swapaxes(F, -1, -2))).max() < 1e-14
    assert np.abs(np.trace(F, axis1=-2, axis2=-1)).max() < 1e-14
    C = cl.clover_term(U, dims, 1.1)
    assert np.abs(C - np.conj(np.swapaxes(C, 1, 2))).max() < 1e-14
    blocks = cl.chiral_blocks(C)
    assert blocks.shape == (lat.volume(dims), 2, 6, 6)


def test_gamma5_hermiticity_and_gauge_covariance():
    dims = (4, 4, 2, 4)
    V = lat.volume(dims)
    U = synth.gauge_field(dims, eps=0.4, seed=5)
    rng = np.random.default_rng(11)
    u = rng.standard_normal((V, 4, 3)) + 1j * rng.standard_normal((V, 4, 3))
    v = rng.standard_normal((V, 4, 3)) + 1j * rng.standard_normal((V, 4, 3))
    m0, sig, csw = 0.05, 0.2, 1.4
    lhs = np.vdot(u, lat.apply_gamma5(cl.clover_apply(U, v, m0, sig, csw, dims)))
    rhs = np.conj(np.vdot(v, lat.apply_gamma5(cl.clover_apply(U, u, m0, sig, csw, dims))))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    g = _random_su3(rng, V)
    Ug = _gauge_transform(U, g, dims)
    gv = np.einsum('vab,vsb->vsa', g, v)
    out = cl.clover_apply(Ug, gv, m0, sig, csw, dims)
    ref = np.einsum('vab,vsb->vsa', g, cl.clover_apply(U, v, m0, sig, csw, dims))
    assert np.abs(out - ref).max() < 1e-12
    Fg = cl.field_strength(Ug, dims).reshape(6, V, 3, 3)
    F = cl.field_strength(U, dims).reshape(6, V, 3, 3)
    assert np.abs(Fg - np.einsum('vab,kvbc,vdc->kvad', g, F, np.conj(g))).max() < 1e-13


def test_dense_matches_matrix_free():
    dims = (4, 2, 2, 4)
    U = synth.gauge_field(dims, eps=0.5, seed=9)
    D = cl.clover_dense(U, 0.1, 0.25, 1.2, dims)
    rng = np.random.default_rng(4)
    psi = rng.standard_normal((lat.volume(dims), 4, 3)) + 1j * rng.standard_normal((lat.volume(dims), 4, 3))
    assert np.abs(D @ psi.ravel() - cl.clover_apply(U, psi, 0.1, 0.25, 1.2, dims).ravel()).max() < 1e-13


def test_sign_cancels_the_wilson_shift_of_zero_modes():
    """Constant abelian field (charges +1, -1 on two colours, flux 2 pi): the
    continuum operator has exact zero modes; the Wilson term moves their
    eigenvalues to about m0 + theta/2, and the clover term with c_sw = 1 (the
    tree-level coefficient) must cancel that to O(theta^2); the opposite sign
    doubles it."""
    dims = (8, 8, 1, 1)
    m0 = 0.05
    U, th = _abelian_field(dims, 1, (1, -1, 0))

    def lowest_charged(csw):
        ev = np.linalg.eigvals(cl.clover_dense(U, m0, 0.0, csw, dims))
        near = np.sort(ev[np.abs(ev.imag) < 1e-8].real)
        near = near[np.abs(near - m0) > 1e-12]  # the neutral colour's constant modes sit at m0
        return near[0] - m0

    w, c, anti = lowest_charged(0.0), lowest_charged(1.0), lowest_charged(-1.0)
    assert abs(w - th / 2) < 0.05 * th
    assert abs(c) < 0.02 * abs(w)
    assert abs(anti - 2 * w) < 0.05 * th


@pytest.mark.parametrize("eps,csw", [(0.3, 1.0), (0.8, 1.9)])
def test_smin_lower_bound_holds(eps, csw):
    dims = (4, 2, 2, 4)
    U = synth.gauge_field(dims, eps=eps, seed=6)
    for sigma in (0.0, 0.5):
        D = cl.clover_dense(U, 0.3, sigma, csw, dims)
        smin = np.linalg.svd(D, compute_uv=False).min()
        bound = cl.smin_lower_bound(U, 0.3, sigma, csw, dims)
        assert bound <= smin + 1e-12, (bound, smin)
    # the row-sum bound is at least the exact spectral norm of every site block
    C = cl.clover_term(U, dims, csw)
    assert cl.norm_bound(C) >= np.linalg.norm(C, ord=2, axis=(1, 2)).max() - 1e-14
