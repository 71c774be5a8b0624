"""Lattice, gamma matrices, Wilson-Dirac operator and Omega_p (oracle).

Conventions (readings of the paper where it is silent; each is listed with its
reason in the design notes):

* site = x + Lx*(y + Ly*(z + Lz*t)); numpy arrays are shaped (Lt, Lz, Ly, Lx,
  ...) so a C-order flatten gives exactly that site order.  Direction mu = 0,
  1, 2, 3 is x, y, z, t, i.e. numpy axis 3, 2, 1, 0.
* gamma matrices in the DeGrand-Rossi basis (the basis of the Chroma library
  that the paper's Results section names); gamma_5 = g1 g2 g3 g4 =
  diag(1, 1, -1, -1).
* Wilson-Dirac operator with shift sigma:
      ((D + sigma) psi)(x) = (4 + m0 + sigma) psi(x)
          - 1/2 sum_mu [ (1 - g_mu) U_mu(x) psi(x + mu)
                       + (1 + g_mu) U_mu(x - mu)^dagger psi(x - mu) ]
  periodic in every direction, optionally antiperiodic in t.
* Gamma_n = g1^b0 g2^b1 g3^b2 g4^b3 for n = sum_k b_k 2^k; this 4-bit order is
  the row order of the paper's appendix speedup table (I, g1, g2, g1g2, g3, ...).
* Omega_p = W Pi_p along z (Introduction): (Omega_p psi)(x) =
  U_z(x) U_z(x+z) ... U_z(x+(p-1)z) psi(x + p z).
"""

import numpy as np

AXIS = {0: 3, 1: 2, 2: 1, 3: 0}  # direction mu -> numpy axis of a (t,z,y,x,...) array


def volume(dims):
    v = 1
    for d in dims:
        v *= int(d)
    return v


def site_index(x, y, z, t, dims):
    Lx, Ly, Lz, _ = dims
    return x + Lx * (y + Ly * (z + Lz * t))


def site_coords(s, dims):
    Lx, Ly, Lz, _ = dims
    x = s % Lx
    s //= Lx
    y = s % Ly
    s //= Ly
    z = s % Lz
    t = s // Lz
    return x, y, z, t


def gammas():
    """DeGrand-Rossi gamma_1..gamma_4 (index 0..3) and gamma_5."""
    i = 1j
    g1 = np.array([[0, 0, 0, i], [0, 0, i, 0], [0, -i, 0, 0], [-i, 0, 0, 0]], dtype=np.complex128)
    g2 = np.array([[0, 0, 0, -1], [0, 0, 1, 0], [0, 1, 0, 0], [-1, 0, 0, 0]], dtype=np.complex128)
    g3 = np.array([[0, 0, i, 0], [0, 0, 0, -i], [-i, 0, 0, 0], [0, i, 0, 0]], dtype=np.complex128)
    g4 = np.array([[0, 0, 1, 0], [0, 0, 0, 1], [1, 0, 0, 0], [0, 1, 0, 0]], dtype=np.complex128)
    g5 = g1 @ g2 @ g3 @ g4
    return [g1, g2, g3, g4], g5


def gamma_n(n):
    """Gamma_n = g1^b0 g2^b1 g3^b2 g4^b3 (4x4)."""
    g, _ = gammas()
    out = np.eye(4, dtype=np.complex128)
    for k in range(4):
        if (n >> k) & 1:
            out = out @ g[k]
    return out


def all_gamma_n():
    return np.stack([gamma_n(n) for n in range(16)])


def _field(psi, dims):
    Lx, Ly, Lz, Lt = dims
    return psi.reshape(Lt, Lz, Ly, Lx, 4, 3)


def _links(U, dims):
    Lx, Ly, Lz, Lt = dims
    return U.reshape(4, Lt, Lz, Ly, Lx, 3, 3)


def _shift_fwd(f, mu, dims, antiperiodic):
    """g(x) = f(x + mu) with the boundary sign (f is (t,z,y,x,...))."""
    g = np.roll(f, -1, axis=AXIS[mu])
    if antiperiodic and mu == 3:
        g[dims[3] - 1] *= -1.0
    return g


def _shift_bwd(f, mu, dims, antiperiodic):
    """g(x) = f(x - mu) with the boundary sign."""
    g = np.roll(f, 1, axis=AXIS[mu])
    if antiperiodic and mu == 3:
        g[0] *= -1.0
    return g


def wilson_apply(U, psi, m0, sigma, dims, antiperiodic=False):
    """((D + sigma) psi), psi canonical (V,4,3) complex128; returns (V,4,3)."""
    g, _ = gammas()
    f = _field(np.asarray(psi, dtype=np.complex128), dims)
    L = _links(U, dims)
    out = (4.0 + m0 + sigma) * f
    one = np.eye(4, dtype=np.complex128)
    for mu in range(4):
        fwd = _shift_fwd(f, mu, dims, antiperiodic)
        # U_mu(x) psi(x + mu), colour index contracted.
        hop_f = np.einsum('tzyxab,tzyxsb->tzyxsa', L[mu], fwd)
        out -= 0.5 * np.einsum('rs,tzyxsa->tzyxra', one - g[mu], hop_f)
        # U_mu(x - mu)^dagger psi(x - mu): form U^dagger psi at x, then shift.
        udag_psi = np.einsum('tzyxba,tzyxsb->tzyxsa', np.conj(L[mu]), f)
        hop_b = _shift_bwd(udag_psi, mu, dims, antiperiodic)
        out -= 0.5 * np.einsum('rs,tzyxsa->tzyxra', one + g[mu], hop_b)
    return out.reshape(-1, 4, 3)


def wilson_dense(U, m0, sigma, dims, antiperiodic=False):
    """Dense N x N matrix of (D + sigma), N = 12 V, index (site*4+spin)*3+colour.

    Built site by site from the definition, independent of `wilson_apply`.
    """
    g, _ = gammas()
    V = volume(dims)
    N = 12 * V
    D = np.zeros((N, N), dtype=np.complex128)
    one = np.eye(4, dtype=np.complex128)
    for s in range(V):
        D[12 * s:12 * s + 12, 12 * s:12 * s + 12] += (4.0 + m0 + sigma) * np.eye(12)
        x = list(site_coords(s, dims))
        for mu in range(4):
            # forward neighbour
            xf = list(x)
            xf[mu] += 1
            sign_f = 1.0
            if xf[mu] == dims[mu]:
                xf[mu] = 0
                if antiperiodic and mu == 3:
                    sign_f = -1.0
            sf = site_index(*xf, dims)
            D[12 * s:12 * s + 12, 12 * sf:12 * sf + 12] += -0.5 * sign_f * np.kron(one - g[mu], U[mu, s])
            # backward neighbour
            xb = list(x)
            xb[mu] -= 1
            sign_b = 1.0
            if xb[mu] < 0:
                xb[mu] = dims[mu] - 1
                if antiperiodic and mu == 3:
                    sign_b = -1.0
            sb = site_index(*xb, dims)
            D[12 * s:12 * s + 12, 12 * sb:12 * sb + 12] += -0.5 * sign_b * np.kron(one + g[mu], np.conj(U[mu, sb]).T)
    return D


def apply_gamma(n, psi):
    """(Gamma_n psi) on a canonical (..., 4, 3) field (spin index contracted)."""
    return np.einsum('rs,...sc->...rc', gamma_n(n), psi)


def apply_gamma5(psi):
    _, g5 = gammas()
    return np.einsum('rs,...sc->...rc', g5, psi)


def displace(U, psi, p, dims):
    """(Omega_p psi)(x) = U_z(x) ... U_z(x+(p-1)z) psi(x+pz), by p single hops.

    One hop: phi_k(x) = U_z(x) phi_{k-1}(x + z); z is periodic.
    """
    f = _field(np.asarray(psi, dtype=np.complex128), dims)
    Uz = _links(U, dims)[2]
    for _ in range(p):
        nb = np.roll(f, -1, axis=AXIS[2])
        f = np.einsum('tzyxab,tzyxsb->tzyxsa', Uz, nb)
    return f.reshape(-1, 4, 3)


def omega_dense(U, p, dims):
    """Dense matrix of Omega_p built from the explicit Wilson-line product."""
    V = volume(dims)
    N = 12 * V
    Om = np.zeros((N, N), dtype=np.complex128)
    Lz = dims[2]
    for s in range(V):
        x, y, z, t = site_coords(s, dims)
        W = np.eye(3, dtype=np.complex128)
        for k in range(p):
            W = W @ U[2, site_index(x, y, (z + k) % Lz, t, dims)]
        sp = site_index(x, y, (z + p) % Lz, t, dims)
        Om[12 * s:12 * s + 12, 12 * sp:12 * sp + 12] = np.kron(np.eye(4), W)
    return Om


def gamma_dense(n, V):
    """Dense matrix of Gamma_n acting on every site (spin x colour)."""
    import scipy.sparse as sp
    blk = np.kron(gamma_n(n), np.eye(3))
    return sp.kron(sp.identity(V, format='csr'), sp.csr_matrix(blk), format='csr')


def link_norm_bound(U):
    """Largest spectral norm of the links, max_x,mu ||U_mu(x)||_2 (from numpy's SVD)."""
    U = np.asarray(U).reshape(-1, 3, 3)
    return float(np.linalg.norm(U, ord=2, axis=(1, 2)).max())


def smin_lower_bound(U, m0, sigma):
    """Lower bound on the smallest singular value of D + sigma.

    D + sigma = (4 + m0 + sigma) - sum_mu H_mu with H_mu = P-_mu (U_mu shift_+mu)
    + P+_mu (shift_-mu U_mu^dagger), P-+_mu = (1 -+ g_mu)/2 complementary
    orthogonal spin projectors that commute with the colour/site maps, so
    ||H_mu psi||^2 = ||A P- psi||^2 + ||B P+ psi||^2 <= u^2 ||psi||^2 with u the
    largest link norm (antiperiodic signs do not change norms).  Hence
    s_min >= 4 + m0 + sigma - 4 u.  Parity: pinned against dense SVD (tests).
    """
    return 4.0 + m0 + sigma - 4.0 * link_norm_bound(U)
