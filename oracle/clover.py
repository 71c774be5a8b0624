"""Clover (Sheikholeslami-Wohlert) term of the Wilson-Dirac operator (oracle).

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this module; the library never does.

The Results section runs the estimator on the clover-improved Wilson operator
of the Chroma library; the paper prints neither the term nor its conventions.
Reading used here (listed with its reasons in the design notes), in the
normalisation of lattice.wilson_apply (forward hop with (1 - g_mu), diagonal
4 + m0 + sigma):

    ((D_sw + sigma) psi)(x) = ((D + sigma) psi)(x) + (C psi)(x)
    C(x) = -(c_sw / 2) sum_{mu < nu} sigma_{mu nu} (x) F_{mu nu}(x)
    sigma_{mu nu} = (i / 2) [g_mu, g_nu]
    F_{mu nu}(x) = traceless part of (Q_{mu nu}(x) - Q_{mu nu}(x)^dagger) / (8 i)

with Q_{mu nu}(x) the sum of the four plaquettes of the (mu, nu) plane that
start and end at x, each taken counter-clockwise (a step along +mu turned
towards +nu).  sigma_{mu nu} and F_{mu nu} are Hermitian, so C(x) is a
Hermitian 12 x 12 matrix per site; sigma_{mu nu} commutes with g_5, so in the
DeGrand-Rossi basis C(x) is block diagonal: one 6 x 6 block on spins 0-1 and
one on spins 2-3.  The term is site-local, so a shift still enters only the
scalar diagonal, and D_sw keeps g_5-hermiticity.

Parity pins (tests, CPU): c_sw = 0 gives the Wilson operator; a pure-gauge
field has F = 0; a constant abelian field has the closed-form F of its
plaquette angle; the clover leaves agree with a path-walking product;
F and C are Hermitian, C commutes with g_5, D_sw is g_5-Hermitian and gauge
covariant.
"""

import numpy as np

from . import lattice as lat


def _roll(f, mu, step):
    """g(x) = f(x + step * mu) for a (t, z, y, x, ...) array (links are periodic)."""
    return np.roll(f, -step, axis=lat.AXIS[mu])


def _dag(m):
    return np.conj(np.swapaxes(m, -1, -2))


def plane_pairs():
    """The six planes (mu, nu), mu < nu, in the order used by field_strength."""
    return [(mu, nu) for mu in range(4) for nu in range(mu + 1, 4)]


def clover_leaves(U, dims, mu, nu):
    """Q_{mu nu}(x): the four plaquettes of the (mu, nu) plane at x, summed.

    Each leaf is the ordered product of the links along a closed path that
    leaves x and returns to it: +mu +nu -mu -nu, +nu -mu -nu +mu, -mu -nu +mu +nu
    and -nu +mu +nu -mu (a step along -mu uses U_mu(x - mu)^dagger).
    Returns a (Lt, Lz, Ly, Lx, 3, 3) array.
    """
    L = lat._links(U, dims)
    Um, Un = L[mu], L[nu]
    mm = np.matmul
    # leaf 1: U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
    q = mm(mm(Um, _roll(Un, mu, 1)), mm(_dag(_roll(Um, nu, 1)), _dag(Un)))
    # leaf 2: U_nu(x) U_mu(x+nu-mu)^+ U_nu(x-mu)^+ U_mu(x-mu)
    Um_m = _roll(Um, mu, -1)                      # U_mu(x - mu)
    Un_m = _roll(Un, mu, -1)                      # U_nu(x - mu)
    q = q + mm(mm(Un, _dag(_roll(Um_m, nu, 1))), mm(_dag(Un_m), Um_m))
    # leaf 3: U_mu(x-mu)^+ U_nu(x-mu-nu)^+ U_mu(x-mu-nu) U_nu(x-nu)
    Un_mn = _roll(Un_m, nu, -1)                   # U_nu(x - mu - nu)
    Um_mn = _roll(Um_m, nu, -1)                   # U_mu(x - mu - nu)
    Un_n = _roll(Un, nu, -1)                      # U_nu(x - nu)
    q = q + mm(mm(_dag(Um_m), _dag(Un_mn)), mm(Um_mn, Un_n))
    # leaf 4: U_nu(x-nu)^+ U_mu(x-nu) U_nu(x+mu-nu) U_mu(x)^+
    Um_n = _roll(Um, nu, -1)                      # U_mu(x - nu)
    q = q + mm(mm(_dag(Un_n), Um_n), mm(_roll(Un_n, mu, 1), _dag(Um)))
    return q


def field_strength(U, dims):
    """F[k] for the planes of plane_pairs(): (6, Lt, Lz, Ly, Lx, 3, 3), Hermitian, traceless."""
    out = []
    eye = np.eye(3)
    for mu, nu in plane_pairs():
        q = clover_leaves(U, dims, mu, nu)
        f = (q - _dag(q)) / 8j
        tr = np.trace(f, axis1=-2, axis2=-1)
        out.append(f - tr[..., None, None] * eye / 3.0)
    return np.stack(out)


def sigma_munu(mu, nu):
    """sigma_{mu nu} = (i/2) [g_mu, g_nu] (4 x 4, Hermitian)."""
    g, _ = lat.gammas()
    return 0.5j * (g[mu] @ g[nu] - g[nu] @ g[mu])


def clover_term(U, dims, c_sw):
    """C(x) per site as (V, 12, 12), index spin * 3 + colour (Hermitian)."""
    F = field_strength(U, dims).reshape(6, -1, 3, 3)
    V = F.shape[1]
    C = np.zeros((V, 12, 12), dtype=np.complex128)
    for k, (mu, nu) in enumerate(plane_pairs()):
        s = sigma_munu(mu, nu)
        C -= 0.5 * c_sw * np.einsum('ab,vij->vaibj', s, F[k]).reshape(V, 12, 12)
    return C


def clover_apply(U, psi, m0, sigma, c_sw, dims, antiperiodic=False, C=None):
    """((D_sw + sigma) psi) for canonical psi (V, 4, 3); C may be passed precomputed."""
    out = lat.wilson_apply(U, psi, m0, sigma, dims, antiperiodic)
    if c_sw == 0.0 and C is None:
        return out
    if C is None:
        C = clover_term(U, dims, c_sw)
    V = C.shape[0]
    return out + np.einsum('vij,vj->vi', C, np.asarray(psi, np.complex128).reshape(V, 12)).reshape(V, 4, 3)


def clover_dense(U, m0, sigma, c_sw, dims, antiperiodic=False):
    """Dense matrix of (D_sw + sigma): the Wilson matrix plus the block-diagonal C."""
    D = lat.wilson_dense(U, m0, sigma, dims, antiperiodic)
    if c_sw == 0.0:
        return D
    C = clover_term(U, dims, c_sw)
    for s in range(C.shape[0]):
        D[12 * s:12 * s + 12, 12 * s:12 * s + 12] += C[s]
    return D


def chiral_blocks(C):
    """The two 6 x 6 blocks of each site's C (spins 0-1, spins 2-3): (V, 2, 6, 6).

    Raises if C has entries between the chiralities (it cannot, as sigma_{mu nu}
    commutes with g_5; a nonzero entry there means a wrong sigma)."""
    off = max(np.abs(C[:, :6, 6:]).max(), np.abs(C[:, 6:, :6]).max())
    if off > 1e-13 * max(1.0, np.abs(C).max()):
        raise ValueError("clover term mixes chiralities")
    return np.stack([C[:, :6, :6], C[:, 6:, 6:]], axis=1)


def norm_bound(C):
    """Upper bound on max_x ||C(x)||_2: the largest absolute row sum of the site
    matrices (for a Hermitian matrix the spectral norm is at most any induced norm)."""
    return float(np.abs(np.asarray(C)).sum(axis=-1).max())


def smin_lower_bound(U, m0, sigma, c_sw, dims):
    """Lower bound on the smallest singular value of D_sw + sigma:
    D_sw + sigma = (4 + m0 + sigma) + C - H with ||H|| <= 4 u (lattice.smin_lower_bound)
    and ||C|| <= norm_bound(C), so s_min >= 4 + m0 + sigma - 4 u - norm_bound(C)
    (Weyl's inequality).  Parity: pinned against dense SVD (tests)."""
    return lat.smin_lower_bound(U, m0, sigma) - norm_bound(clover_term(U, dims, c_sw))
