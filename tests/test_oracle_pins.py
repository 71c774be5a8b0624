"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test checks one oracle function against a closed form, a symmetry, an
exhaustive enumeration, an independent library routine or a value printed in
the paper, so that a dropped term, a wrong sign or index or a transposed
operand in the oracle fails at least one of them.
"""

import itertools
import os

import numpy as np
import pytest

import synth
from oracle import fs, lattice as lat
from oracle.philox import philox4x64, philox4x64_scalar, z4_codes, z4_noise
from oracle.solver import bicgstab

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- gamma algebra

def test_gamma_clifford_hermitian_g5():
    g, g5 = lat.gammas()
    I4 = np.eye(4)
    for m in range(4):
        assert np.allclose(g[m], g[m].conj().T)
        for n in range(4):
            assert np.allclose(g[m] @ g[n] + g[n] @ g[m], 2 * (m == n) * I4)
    assert np.allclose(g5, np.diag([1, 1, -1, -1]))


def _label_matrix(label):
    g, g5 = lat.gammas()
    table = {"1": g[0], "2": g[1], "3": g[2], "4": g[3], "5": g5}
    M = np.eye(4, dtype=complex)
    if label == "I":
        return M
    for tok in label.split("g")[1:]:
        M = M @ table[tok]
    return M


def test_gamma_n_matches_paper_table_order():
    labels = [l.strip() for l in open(os.path.join(GOLDEN, "gamma_order.txt"))
              if l.strip() and not l.startswith("#")]
    assert len(labels) == 16
    signs = []
    for n, label in enumerate(labels):
        G = lat.gamma_n(n)
        M = _label_matrix(label)
        # equal up to an overall sign (the table names the matrix, not its phase)
        if np.allclose(G, M):
            signs.append(1)
        else:
            assert np.allclose(G, -M), (n, label)
            signs.append(-1)
    assert signs[13] == -1 and signs.count(-1) == 1  # Gamma_13 = -g2 g5


# ---------------------------------------------------------------- SU(3) inputs

def test_links_are_su3():
    U = synth.gauge_field((2, 2, 2, 4), eps=0.3, seed=0)
    I3 = np.eye(3)
    uu = np.einsum('mvji,mvjk->mvik', U.conj(), U)
    assert np.abs(uu - I3).max() < 1e-14
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-14
    U0 = synth.gauge_field((2, 2, 2, 4), eps=0.0)
    assert np.array_equal(U0, np.broadcast_to(I3, U0.shape))


# ---------------------------------------------------------------- free field

def _free_symbol(dims, m0, sigma, antiperiodic):
    """All (a, |s|) for the free Wilson operator in momentum space."""
    ks = []
    for mu, L in enumerate(dims):
        n = np.arange(L)
        k = (2 * n + 1) * np.pi / L if (antiperiodic and mu == 3) else 2 * np.pi * n / L
        ks.append(k)
    kx, ky, kz, kt = np.meshgrid(*ks, indexing='ij')
    K = [kx, ky, kz, kt]
    a = m0 + sigma + sum(1 - np.cos(k) for k in K)
    s2 = sum(np.sin(k) ** 2 for k in K)
    return a, s2, K


@pytest.mark.parametrize("antiperiodic", [False, True])
def test_free_field_spectrum(antiperiodic):
    dims = (4, 2, 2, 4)
    m0, sigma = 0.1, 0.3
    U = synth.gauge_field(dims, eps=0.0)
    D = lat.wilson_dense(U, m0, sigma, dims, antiperiodic)
    ev = np.linalg.eigvals(D)
    a, s2, _ = _free_symbol(dims, m0, sigma, antiperiodic)
    a, s = a.ravel(), np.sqrt(s2.ravel())
    expect = np.concatenate([np.repeat(a + 1j * s, 6), np.repeat(a - 1j * s, 6)])
    key = lambda z: np.lexsort((np.round(z.imag, 9), np.round(z.real, 9)))
    assert np.allclose(np.sort_complex(np.round(ev, 9)), np.sort_complex(np.round(expect, 9)), atol=1e-9)
    assert np.abs(ev[key(ev)] - expect[key(expect)]).max() < 1e-10


def test_free_field_plane_wave_matrix_free():
    dims = (4, 4, 4, 4)
    m0, sigma = 0.05, 0.2
    U = synth.gauge_field(dims, eps=0.0)
    g, _ = lat.gammas()
    n = (1, 3, 2, 1)
    k = [2 * np.pi * n[mu] / dims[mu] for mu in range(4)]
    rng = np.random.default_rng(3)
    chi = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    V = lat.volume(dims)
    phase = np.empty(V, dtype=complex)
    for s in range(V):
        x = lat.site_coords(s, dims)
        phase[s] = np.exp(1j * sum(k[m] * x[m] for m in range(4)))
    psi = phase[:, None, None] * chi
    a = m0 + sigma + sum(1 - np.cos(km) for km in k)
    Dk = a * np.eye(4) + 1j * sum(g[m] * np.sin(k[m]) for m in range(4))
    expect = phase[:, None, None] * (Dk @ chi)[None]
    got = lat.wilson_apply(U, psi, m0, sigma, dims)
    assert np.abs(got - expect).max() < 1e-13


@pytest.mark.parametrize("antiperiodic", [False, True])
def test_free_field_traces_closed_form(antiperiodic):
    """Tr(Pi_p G), Tr(g3 Pi_p G) from the momentum-space propagator."""
    dims = (2, 2, 6, 2)
    m0, sigma = 0.1, 0.25
    U = synth.gauge_field(dims, eps=0.0)
    solver = fs.DenseSolver(U, dims, m0, antiperiodic)
    a, s2, K = _free_symbol(dims, m0, 0.0, antiperiodic)
    a = a + sigma
    kz = K[2]
    for p in range(0, 6):
        t_id = 12 * np.sum(np.cos(kz * p) * a / (a ** 2 + s2))
        t_g3 = 12 * np.sum(np.sin(kz * p) * np.sin(kz) / (a ** 2 + s2))
        got_id = fs.exact_trace(solver, sigma, 0, p)
        got_g3 = fs.exact_trace(solver, sigma, 4, p)  # Gamma_4 = g3
        assert abs(got_id - t_id) < 1e-11 * max(1, abs(t_id))
        assert abs(got_g3 - t_g3) < 1e-11 * max(1, abs(t_g3))
        if p in (1, 2):
            assert abs(t_g3) > 1e-3  # the g3 pin is not vacuous


# ---------------------------------------------------------------- symmetries

def test_dense_equals_matrix_free_random_links():
    dims = (2, 4, 2, 4)
    U = synth.gauge_field(dims, eps=0.4, seed=5)
    psi = synth.random_spinor(dims, seed=1)
    for ap in (False, True):
        D = lat.wilson_dense(U, 0.07, 0.3, dims, ap)
        assert np.abs(D @ psi.ravel() - lat.wilson_apply(U, psi, 0.07, 0.3, dims, ap).ravel()).max() < 1e-13


def test_gamma5_hermiticity():
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, eps=0.5, seed=2)
    u = synth.random_spinor(dims, seed=3)
    v = synth.random_spinor(dims, seed=4)
    for ap in (False, True):
        Dv = lat.wilson_apply(U, v, 0.1, 0.4, dims, ap)
        Du = lat.wilson_apply(U, u, 0.1, 0.4, dims, ap)
        lhs = np.vdot(u.ravel(), lat.apply_gamma5(Dv).ravel())
        rhs = np.conj(np.vdot(v.ravel(), lat.apply_gamma5(Du).ravel()))
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def _gauge_rotate(U, g, dims):
    V = lat.volume(dims)
    Up = np.empty_like(U)
    for mu in range(4):
        fwd = np.empty(V, dtype=np.int64)
        for s in range(V):
            x = list(lat.site_coords(s, dims))
            x[mu] = (x[mu] + 1) % dims[mu]
            fwd[s] = lat.site_index(*x, dims)
        Up[mu] = g @ U[mu] @ np.conj(np.swapaxes(g[fwd], 1, 2))
    return Up


def test_gauge_covariance_operator_and_displacement():
    dims = (2, 2, 4, 4)
    U = synth.gauge_field(dims, eps=0.5, seed=7)
    g = synth.gauge_transform(dims, seed=8)
    Up = _gauge_rotate(U, g, dims)
    psi = synth.random_spinor(dims, seed=9)
    gpsi = np.einsum('vab,vsb->vsa', g, psi)
    lhs = lat.wilson_apply(Up, gpsi, 0.1, 0.2, dims, True)
    rhs = np.einsum('vab,vsb->vsa', g, lat.wilson_apply(U, psi, 0.1, 0.2, dims, True))
    assert np.abs(lhs - rhs).max() < 1e-13
    for p in range(5):
        lhs = lat.displace(Up, gpsi, p, dims)
        rhs = np.einsum('vab,vsb->vsa', g, lat.displace(U, psi, p, dims))
        assert np.abs(lhs - rhs).max() < 1e-13


def test_exact_trace_gauge_invariant():
    dims = (2, 2, 4, 2)
    U = synth.gauge_field(dims, eps=0.5, seed=11)
    g = synth.gauge_transform(dims, seed=12)
    Up = _gauge_rotate(U, g, dims)
    s1 = fs.DenseSolver(U, dims, 0.1)
    s2 = fs.DenseSolver(Up, dims, 0.1)
    for n, p in [(0, 0), (4, 1), (11, 2), (15, 3)]:
        t1 = fs.exact_trace(s1, 0.2, n, p)
        t2 = fs.exact_trace(s2, 0.2, n, p)
        assert abs(t1 - t2) < 1e-12 * max(1.0, abs(t1))


# ---------------------------------------------------------------- displacement

def test_displacement_unit_links_is_exact_shift():
    dims = (2, 3, 5, 2)
    V = lat.volume(dims)
    U = synth.gauge_field(dims, eps=0.0)
    labels = np.arange(V * 12, dtype=np.float64).reshape(V, 4, 3).astype(np.complex128)
    for p in range(0, 7):
        out = lat.displace(U, labels, p, dims)
        for s in range(V):
            x, y, z, t = lat.site_coords(s, dims)
            sp = lat.site_index(x, y, (z + p) % dims[2], t, dims)
            assert np.array_equal(out[s], labels[sp])


def test_displacement_composition_dense_and_polyakov():
    dims = (2, 2, 4, 2)
    U = synth.gauge_field(dims, eps=0.6, seed=13)
    psi = synth.random_spinor(dims, seed=14)
    for a, b in [(1, 2), (2, 2), (0, 3)]:
        lhs = lat.displace(U, lat.displace(U, psi, b, dims), a, dims)
        assert np.abs(lhs - lat.displace(U, psi, a + b, dims)).max() < 1e-13
    for p in range(4):
        Om = lat.omega_dense(U, p, dims)
        assert np.abs(Om @ psi.ravel() - lat.displace(U, psi, p, dims).ravel()).max() < 1e-13
    # Omega_{Lz}: colour trace of the Polyakov line in z is gauge invariant
    g = synth.gauge_transform(dims, seed=15)
    Up = _gauge_rotate(U, g, dims)
    Lz = dims[2]
    tr1 = np.trace(lat.omega_dense(U, Lz, dims).reshape(lat.volume(dims), 12, -1, 12)[np.arange(lat.volume(dims)), :, np.arange(lat.volume(dims)), :], axis1=1, axis2=2)
    tr2 = np.trace(lat.omega_dense(Up, Lz, dims).reshape(lat.volume(dims), 12, -1, 12)[np.arange(lat.volume(dims)), :, np.arange(lat.volume(dims)), :], axis1=1, axis2=2)
    assert np.abs(tr1 - tr2).max() < 1e-12


# ---------------------------------------------------------------- telescoping

def test_telescoping_and_one_end_trick():
    dims = (2, 2, 4, 2)
    U = synth.gauge_field(dims, eps=0.3, seed=0)
    solver = fs.DenseSolver(U, dims, 0.1)
    sig = [0.0, 0.5, 1.0]
    gam = [0, 4, 11]
    T, _ = fs.exact_levels(solver, sig, gam, [0, 1, 2], with_variance=False)
    for ig, n in enumerate(gam):
        for ip, p in enumerate([0, 1, 2]):
            full = fs.exact_trace(solver, 0.0, n, p)
            assert abs(T[:, ig, ip].sum() - full) < 1e-12 * max(1, abs(full))
            for l in range(len(sig) - 1):
                diff = fs.exact_trace(solver, sig[l], n, p) - fs.exact_trace(solver, sig[l + 1], n, p)
                assert abs(T[l, ig, ip] - diff) < 1e-12 * max(1, abs(diff))


def test_adjoint_via_gamma5():
    dims = (2, 2, 2, 4)
    U = synth.gauge_field(dims, eps=0.4, seed=3)
    solver = fs.DenseSolver(U, dims, 0.1)
    z = z4_noise(lat.volume(dims), 1, 0, 0, 0)
    D = solver.D0 + 0.3 * np.eye(solver.D0.shape[0])
    y_direct = np.linalg.solve(D.conj().T, z.ravel())
    y_g5 = lat.apply_gamma5(solver.solve(0.3, lat.apply_gamma5(z))).ravel()
    assert np.abs(y_direct - y_g5).max() < 1e-12


# ---------------------------------------------------------------- variance

def test_z4_variance_exhaustive_enumeration():
    """Over all 4^n Z4 vectors the population variance of z^H A z is exactly
    ||A||_F^2 - sum |A_ii|^2 (factor 1, not the 2 of real +-1 noise)."""
    n = 6
    rng = np.random.default_rng(0)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    vals = np.array([1, 1j, -1, -1j])
    Z = np.array([vals[list(c)] for c in itertools.product(range(4), repeat=n)])
    X = np.einsum('ki,ij,kj->k', Z.conj(), A, Z)
    t, var_paper, _ = fs.level_stats(X[None, :], axis=1)
    # brute-force closed form, written independently of fs.offdiag_frobenius
    closed = sum(abs(A[i, j]) ** 2 for i in range(n) for j in range(n) if i != j)
    assert abs(t[0] - np.trace(A)) < 1e-12
    assert abs(var_paper[0] - closed) < 1e-10 * closed
    assert abs(fs.offdiag_frobenius(A) - closed) < 1e-10 * closed
    # real +-1 noise on a real symmetric matrix: factor 2 (Hutchinson's setting)
    S = rng.standard_normal((n, n))
    S = S + S.T
    R = np.array(list(itertools.product([1.0, -1.0], repeat=n)))
    Xr = np.einsum('ki,ij,kj->k', R, S, R)
    closed_r = sum(S[i, j] ** 2 for i in range(n) for j in range(n) if i != j)
    assert abs(Xr.var() - 2 * closed_r) < 1e-9 * closed_r


def test_level_stats_unbiased_form():
    X = np.array([[1.0 + 1j, 2.0, -1.0j, 0.5]])
    t, vp, vu = fs.level_stats(X, axis=1)
    m = X[0].mean()
    assert abs(t[0] - m) < 1e-15
    assert abs(vp[0] - np.mean(np.abs(X[0] - m) ** 2)) < 1e-14
    assert abs(vu[0] - np.sum(np.abs(X[0] - m) ** 2) / 3) < 1e-14


# ---------------------------------------------------------------- RNG

def test_philox_matches_numpy():
    for key in ([0, 0], [1, 0], [0xDEADBEEF, 123456789], [2 ** 64 - 1, 7]):
        for ctr0 in (0, 5, 2 ** 63):
            bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                                  counter=np.array([ctr0, 3, 0, 9], dtype=np.uint64))
            raw = bg.random_raw(4)
            # numpy pre-increments the 256-bit counter before each block
            c = ctr0 + 1
            assert philox4x64_scalar([c & (2 ** 64 - 1), 3 + (c >> 64), 0, 9], key) == [int(v) for v in raw]
            vec = philox4x64(np.uint64(c & (2 ** 64 - 1)), np.uint64(3 + (c >> 64)), 0, 9, key[0], key[1])
            assert [int(v) for v in vec] == [int(v) for v in raw]


def test_z4_codes_layout_and_uniformity():
    V = 256
    k = z4_codes(V, seed=1, instance=0, level=2, sample=5)
    flat = k.reshape(-1)
    # component c uses bits 2*(c%32) of word (c%128)//32 of block c//128
    for c in (0, 1, 31, 32, 127, 128, 1000, 12 * V - 1):
        w = philox4x64_scalar([c // 128, 5, 2, 0], [1, 0])[(c % 128) // 32]
        assert flat[c] == (w >> (2 * (c % 32))) & 3
    counts = np.bincount(flat, minlength=4) / flat.size
    assert np.all(np.abs(counts - 0.25) < 0.02)
    z = z4_noise(V, 1, 0, 2, 5)
    assert set(np.unique(z)) <= {1, 1j, -1, -1j}
    assert not np.array_equal(z, z4_noise(V, 1, 0, 2, 6))
    assert not np.array_equal(z, z4_noise(V, 1, 0, 3, 5))
    assert not np.array_equal(z, z4_noise(V, 1, 1, 2, 5))


# ---------------------------------------------------------------- solver

def test_bicgstab_matches_dense_lu():
    dims = (2, 2, 4, 4)
    U = synth.gauge_field(dims, eps=0.3, seed=0)
    dense = fs.DenseSolver(U, dims, 0.05)
    b = z4_noise(lat.volume(dims), 1, 0, 0, 0)
    for sigma in (0.0, 0.4):
        x, info = bicgstab(lambda v: lat.wilson_apply(U, v, 0.05, sigma, dims), b, tol=1e-12)
        assert info['true_rel'] <= 1e-12
        xd = dense.solve(sigma, b)
        smin = np.linalg.svd(dense.D0 + sigma * np.eye(dense.D0.shape[0]), compute_uv=False)[-1]
        bound = 1e-12 * np.linalg.norm(b) / smin
        assert np.linalg.norm(x - xd) <= 1.01 * bound


# ---------------------------------------------------------------- estimator

def _tiny_setup():
    dims = (2, 2, 4, 2)
    U = synth.gauge_field(dims, eps=0.3, seed=0)
    solver = fs.DenseSolver(U, dims, 0.1)
    return dims, U, solver


def test_estimator_unbiased_within_4_sigma():
    dims, U, solver = _tiny_setup()
    sig = [0.0, 0.5, 1.0]
    gam = [0, 4, 11]
    p_max = 2
    N = 64
    X = fs.fs_samples(U, dims, sig, N, seed=1, gammas=gam, p_max=p_max, solver=solver)
    t, vp, vu = fs.level_stats(X, axis=1)
    T, Var = fs.exact_levels(solver, sig, gam, list(range(p_max + 1)))
    assert np.all(np.abs(t - T) <= 4 * np.sqrt(Var / N) + 1e-12)
    # the per-level exact variances are what the samples estimate (loose: N=64)
    big = Var > 1e-6
    assert np.all(np.abs(vu[big] - Var[big]) <= 0.8 * Var[big])


def test_sample_variance_matches_closed_form():
    dims = (2, 2, 2, 2)
    U = synth.gauge_field(dims, eps=0.3, seed=4)
    solver = fs.DenseSolver(U, dims, 0.1)
    sig = [0.0, 0.4]
    N = 4096
    V = lat.volume(dims)
    invs = [solver.inverse(s) for s in sig]
    g5 = np.kron(np.eye(V), np.kron(np.diag([1.0, 1, -1, -1]), np.eye(3)))
    Z = np.stack([z4_noise(V, 2, 0, 0, s).ravel() for s in range(N)], axis=1)
    G = lat.gamma_dense(4, V) @ lat.omega_dense(U, 1, dims)
    # batched form of the level-0 estimator: X_s = (s1-s0) (g5 inv0 g5 z)^H G inv1 z
    x = invs[1] @ Z
    y = g5 @ (invs[0] @ (g5 @ Z))
    X = (sig[1] - sig[0]) * np.einsum('is,is->s', y.conj(), G @ x)
    t, vp, vu = fs.level_stats(X[None, :], axis=1)
    A = (sig[1] - sig[0]) * invs[0] @ G @ invs[1]
    closed = fs.offdiag_frobenius(A)
    dev = np.abs(X - t[0]) ** 2
    se = dev.std() / np.sqrt(N)
    assert abs(vu[0] - closed) <= 4 * se
    # and the per-sample values agree with the general estimator path
    Xs = fs.fs_samples(U, dims, sig, 3, seed=2, gammas=[4], p_max=1, solver=solver, levels=[0])
    assert np.allclose(Xs[0, :, 0, 1], X[:3], rtol=1e-12, atol=1e-14)


def test_fs_combine():
    t = np.array([1.0, 2.0, 3.0])
    v = np.array([4.0, 2.0, 1.0])
    n = np.array([4, 2, 1])
    tot, vfs, vtot = fs.fs_combine(t, v, n)
    assert tot == 6.0 and vfs == 3.0 and vtot == 7.0


# ---------------------------------------------------------------- variance sampling

def test_sampling_samples_match_dense_matrices():
    """Every sampled value is z_k^H A z_k with the dense matrix of its slot:
    A = G (D+s_i)^-1 for V_L(s_i) and A = (D+s_i)^-1 G (D+s_j)^-1 for
    Vbar_l(s_i, s_j), with one noise vector shared by all shifts.  The
    oracle's path solves with g5 (D+s)^-1 g5 instead of using the inverse on
    the left, so a transposed product, a lost g5 or per-shift noise fails."""
    dims = (2, 2, 4, 2)
    U = synth.gauge_field(dims, eps=0.3, seed=0)
    solver = fs.DenseSolver(U, dims, 0.1)
    shifts = [0.0, 0.3, 1.0]
    gam = [4, 11]
    X = fs.sampling_samples(U, dims, shifts, 3, seed=5, gammas=gam, p_max=2, solver=solver)
    V = lat.volume(dims)
    invs = [solver.inverse(s) for s in shifts]
    for k in range(3):
        z = z4_noise(V, 5, 0, fs.SAMPLING_LEVEL, k).ravel()
        for ip in range(3):
            Om = lat.omega_dense(U, ip, dims)
            for ig, n in enumerate(gam):
                G = lat.gamma_dense(n, V) @ Om
                for q, (kind, i, j) in enumerate(fs.sampling_slots(len(shifts))):
                    A = G @ invs[j] if kind == "single" else invs[i] @ G @ invs[j]
                    assert abs(X[q, k, ig, ip] - np.vdot(z, A @ z)) <= 1e-11 * max(1.0, abs(X[q, k, ig, ip]))


def test_sampling_variance_matches_closed_form():
    """The practical variance of the sampled pair (s_0, s_1) and single s_1
    estimates ||A||_F^2 - sum |A_ii|^2 within 4 standard errors (4096 Z4
    vectors), and exact_sampling reports that closed form."""
    dims = (2, 2, 2, 2)
    U = synth.gauge_field(dims, eps=0.3, seed=4)
    solver = fs.DenseSolver(U, dims, 0.1)
    shifts = [0.0, 0.4]
    N = 4096
    V = lat.volume(dims)
    invs = [solver.inverse(s) for s in shifts]
    Z = np.stack([z4_noise(V, 3, 0, fs.SAMPLING_LEVEL, s).ravel() for s in range(N)], axis=1)
    G = lat.gamma_dense(2, V) @ lat.omega_dense(U, 1, dims)
    _, Var = fs.exact_sampling(solver, shifts, [2], [1])
    slots = fs.sampling_slots(2)
    for q, (kind, i, j) in enumerate(slots):
        A = G @ invs[j] if kind == "single" else invs[i] @ G @ invs[j]
        X = np.einsum('is,is->s', Z.conj(), A @ Z)
        t, vp, vu = fs.level_stats(X[None, :], axis=1)
        se = (np.abs(X - t[0]) ** 2).std() / np.sqrt(N)
        assert abs(vu[0] - Var[q, 0, 0]) <= 4 * se, (kind, i, j)


def test_sampling_exact_traces_resolvent_identity():
    """(s_j - s_i) Tr((D+s_i)^-1 G (D+s_j)^-1) = Tr(G (D+s_i)^-1) - Tr(G (D+s_j)^-1)
    (resolvent identity and cyclicity of the trace) for every pair."""
    dims = (2, 2, 4, 2)
    U = synth.gauge_field(dims, eps=0.3, seed=2)
    solver = fs.DenseSolver(U, dims, 0.05)
    shifts = [0.0, 0.1, 0.4, 1.2]
    T, _ = fs.exact_sampling(solver, shifts, [0, 11], [0, 2])
    slots = fs.sampling_slots(len(shifts))
    single = {i: q for q, (kind, i, j) in enumerate(slots) if kind == "single"}
    for q, (kind, i, j) in enumerate(slots):
        if kind == "pair" and i < j:
            lhs = (shifts[j] - shifts[i]) * T[q]
            rhs = T[single[i]] - T[single[j]]
            assert np.allclose(lhs, rhs, rtol=1e-10, atol=1e-10)
