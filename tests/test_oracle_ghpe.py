"""Pins of the oracle's hopping parameter expansion (CPU).

D + sigma = a - H with a = 4 + m0 + sigma; the expansion used for V_L
sampling (Sec. 3.1) estimates Gamma Omega_p (H/a)^k (D + sigma)^-1.  Checks:
the expansion identity with the dense inverse; the hopping term's low powers
are traceless (odd powers cannot close a loop on the bipartite lattice, and
the square's back-and-forth terms vanish because (1 - g_mu)(1 + g_mu) = 0);
the free-field trace of H^4 equals its momentum-space closed form; the exact
traces split into the low-order terms plus the remainder; the sampled values
are the bilinears of the dense remainder.
"""

import itertools

import numpy as np
import pytest

import synth
from oracle import fs as ofs, lattice as lat
from oracle.philox import z4_noise


def _dense_h(U, dims):
    """H as a dense matrix, column by column from hopping_apply (matrix-free)."""
    V = lat.volume(dims)
    N = 12 * V
    H = np.zeros((N, N), dtype=np.complex128)
    e = np.zeros(N, dtype=np.complex128)
    for c in range(N):
        e[c] = 1.0
        H[:, c] = ofs.hopping_apply(U, e.reshape(V, 4, 3), 0.3, 0.1, dims).ravel()
        e[c] = 0.0
    return H


@pytest.fixture(scope="module")
def small():
    dims = (4, 4, 2, 2)
    U = synth.gauge_field(dims, eps=0.5, seed=4)
    return dims, U, _dense_h(U, dims)


def test_expansion_identity(small):
    dims, U, H = small
    m0, sigma, k = 0.1, 0.3, 4
    a = 4.0 + m0 + sigma
    inv = ofs.DenseSolver(U, dims, m0).inverse(sigma)
    lhs = sum(np.linalg.matrix_power(H / a, j) / a for j in range(k)) + np.linalg.matrix_power(H / a, k) @ inv
    assert np.abs(lhs - inv).max() < 1e-12 * np.abs(inv).max()


def test_low_powers_of_the_hopping_term_are_traceless():
    """Every extent 4, so no closed path shorter than 4 hops wraps the lattice."""
    import scipy.sparse as sp
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, eps=0.5, seed=4)
    H = sp.csr_matrix((4.0 + 0.2) * np.eye(12 * lat.volume(dims)) - lat.wilson_dense(U, 0.2, 0.0, dims))
    Hj = sp.identity(H.shape[0], dtype=np.complex128, format="csr")
    tr = []
    for j in range(1, 5):
        Hj = Hj @ H
        tr.append(Hj.diagonal().sum())
    assert max(abs(t) for t in tr[:3]) < 1e-10
    assert abs(tr[3]) > 1.0  # plaquette loops first appear at order 4


def test_free_field_trace_of_h4():
    dims = (4, 2, 2, 4)
    V = lat.volume(dims)
    one = np.tile(np.eye(3, dtype=np.complex128), (4, V, 1, 1))
    H = _dense_h(one, dims)
    tr = np.trace(np.linalg.matrix_power(H, 4)).real
    # H(k) = sum_mu cos k_mu - i g.sin k: tr_spin H(k)^4 = 4 [(c^2 - s^2)^2 - 4 c^2 s^2]
    ref = 0.0
    for n in itertools.product(*[range(L) for L in dims]):
        kk = [2 * np.pi * n[m] / dims[m] for m in range(4)]
        c = sum(np.cos(x) for x in kk)
        s2 = sum(np.sin(x) ** 2 for x in kk)
        ref += 12 * ((c * c - s2) ** 2 - 4 * c * c * s2)
    assert abs(tr - ref) < 1e-9 * abs(ref)


def test_exact_traces_split_into_low_orders_and_remainder():
    dims = (4, 4, 2, 2)
    U = synth.gauge_field(dims, eps=0.3, seed=1)
    m0 = 0.4
    solver = ofs.DenseSolver(U, dims, m0)
    shifts = [0.0, 0.5]
    gammas, p_list = [0, 4, 11], [0, 1]
    T, Var = ofs.exact_sampling(solver, shifts, gammas, p_list)
    Th, Varh = ofs.exact_sampling(solver, shifts, gammas, p_list, hpe_order=4)
    V = lat.volume(dims)
    Hd = (4.0 + m0) * np.eye(12 * V) - solver.D0
    for i, s in enumerate(shifts):
        a = 4.0 + m0 + s
        for ip, p in enumerate(p_list):
            Om = lat.omega_dense(U, p, dims)
            for ig, n in enumerate(gammas):
                G = lat.gamma_dense(n, V) @ Om
                low = sum(np.trace(G @ np.linalg.matrix_power(Hd / a, j)) / a for j in range(4))
                assert abs(low + Th[i, ig, ip] - T[i, ig, ip]) < 1e-10 * max(1.0, abs(T[i, ig, ip]))
        # the pairs are untouched
    assert np.allclose(Th[len(shifts):], T[len(shifts):]) and np.allclose(Varh[len(shifts):], Var[len(shifts):])
    # at this mass the remainder's one-sample variance is the smaller one for the unit operator
    assert np.all(Varh[:2, 0, 0] < Var[:2, 0, 0])


def test_samples_are_bilinears_of_the_dense_remainder():
    dims = (4, 4, 2, 2)
    U = synth.gauge_field(dims, eps=0.3, seed=2)
    m0 = -0.1
    shifts = [0.0, 0.05, 0.25]
    solver = ofs.DenseSolver(U, dims, m0)
    X = ofs.sampling_samples(U, dims, shifts, 2, 3, [0, 7], 1, solver, hpe_order=4)
    X0 = ofs.sampling_samples(U, dims, shifts, 2, 3, [0, 7], 1, solver)
    V = lat.volume(dims)
    Hd = (4.0 + m0) * np.eye(12 * V) - solver.D0
    for i, s in enumerate(shifts):
        if not ofs.hpe_eligible(m0, s):  # m0 + s <= 0: plain samples
            assert np.array_equal(X[i], X0[i])
            continue
        R = np.linalg.matrix_power(Hd / (4.0 + m0 + s), 4) @ solver.inverse(s)
        for k in range(2):
            z = z4_noise(V, 3, 0, ofs.SAMPLING_LEVEL, k).ravel()
            for ig, n in enumerate([0, 7]):
                for p in range(2):
                    G = lat.gamma_dense(n, V) @ lat.omega_dense(U, p, dims)
                    ref = np.vdot(z, G @ (R @ z))
                    assert abs(X[i, k, ig, p] - ref) < 1e-10 * max(1.0, abs(ref))
    assert np.array_equal(X[len(shifts):], X0[len(shifts):])


def test_generalized_expansion_with_the_clover_term():
    """D_sw + sigma = A - H with A = C + a: the identity
    (D_sw + sigma)^-1 = sum_{j<k} (A^-1 H)^j A^-1 + (A^-1 H)^k (D_sw + sigma)^-1
    with the dense clover inverse; H is the Wilson hopping term; the sampled
    remainder equals the bilinears of the dense remainder."""
    from oracle import clover as cl
    dims = (4, 4, 2, 2)
    U = synth.gauge_field(dims, eps=0.4, seed=3)
    m0, sigma, csw, k = 0.2, 0.1, 1.3, 4
    V = lat.volume(dims)
    C = cl.clover_term(U, dims, csw)
    A = (4.0 + m0 + sigma) * np.eye(12 * V, dtype=np.complex128)
    for q in range(V):
        A[12 * q:12 * q + 12, 12 * q:12 * q + 12] += C[q]
    D = cl.clover_dense(U, m0, sigma, csw, dims)
    H = A - D
    assert np.abs(H - _dense_h(U, dims)).max() < 1e-13  # the hopping term does not change
    inv = np.linalg.inv(D)
    M = np.linalg.solve(A, H)
    lhs = sum(np.linalg.matrix_power(M, j) @ np.linalg.inv(A) for j in range(k)) + np.linalg.matrix_power(M, k) @ inv
    assert np.abs(lhs - inv).max() < 1e-12 * np.abs(inv).max()
    solver = ofs.DenseSolver(U, dims, m0, c_sw=csw)
    X = ofs.sampling_samples(U, dims, [0.0, sigma], 2, 5, [0, 11], 1, solver, hpe_order=k)
    z = z4_noise(V, 5, 0, ofs.SAMPLING_LEVEL, 1).ravel()
    R = np.linalg.matrix_power(M, k) @ inv
    for ig, n in enumerate([0, 11]):
        for p in range(2):
            G = lat.gamma_dense(n, V) @ lat.omega_dense(U, p, dims)
            ref = np.vdot(z, G @ (R @ z))
            assert abs(X[1, 1, ig, p] - ref) < 1e-10 * max(1.0, abs(ref))
