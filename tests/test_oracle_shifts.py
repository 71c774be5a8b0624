"""Pins of the shift-selection oracle (Sec. 3.2-3.3) against facts outside it.

* PCHIP equals scipy's PchipInterpolator (the same published method), keeps
  monotone data monotone and reproduces lines exactly.
* The 2-D scheme passes through every sampled pair (with the (s_j - s_i)^2
  prefactor restored) for arbitrary data, and reproduces separable
  exponential surfaces exactly everywhere (ln of such a surface is linear in
  each argument, and both PCHIP and the line reproduce linear data).
* The iteration-count model on hand-worked values.
* The shortest-path argmin equals the brute-force sweep over every
  combination on small grids.
* The evaluation grid holds the optimal shifts printed in the Results section
  (to their printed three decimals) and the sampling set.
"""

import os

import numpy as np
import pytest
from scipy.interpolate import PchipInterpolator

from oracle import shifts as osh

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_shifts():
    out = {}
    with open(os.path.join(GOLDEN, "shifts.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, *v = line.split()
                out[k] = [float(x) for x in v]
    return out


@pytest.mark.parametrize("seed", range(6))
def test_pchip_matches_scipy(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(3, 9))
    x = np.sort(rng.uniform(0, 2, n))
    y = rng.normal(size=n) if seed % 2 else np.cumsum(rng.uniform(-1, 0.3, n))
    t = np.concatenate([x, rng.uniform(x[0], x[-1], 200)])
    ref = PchipInterpolator(x, y)(t)
    got = osh.interpolate(x, y, t)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_pchip_monotone_and_linear():
    rng = np.random.default_rng(7)
    x = np.sort(rng.uniform(0, 1, 7))
    y = -np.cumsum(rng.uniform(0, 1, 7) ** 3)  # decreasing, uneven steps
    t = np.linspace(x[0], x[-1], 2001)
    q = osh.interpolate(x, y, t)
    assert np.all(np.diff(q) <= 1e-15)
    lin = 0.3 - 2.5 * x
    assert np.allclose(osh.interpolate(x, lin, t), 0.3 - 2.5 * t, atol=1e-13)
    assert np.allclose(osh.interpolate(x[:2], lin[:2], t[t <= x[1]]), 0.3 - 2.5 * t[t <= x[1]], atol=1e-13)


def test_single_reproduces_exponential():
    s_hat = np.array([0.0, 0.05, 0.25, 0.5, 1.0])
    s = osh.eval_grid(s_hat)
    got = osh.interp_single(s_hat, np.exp(1.5 - 3.0 * s_hat), s)
    assert np.allclose(got, np.exp(1.5 - 3.0 * s), rtol=1e-12)


def test_pairs_reproduce_separable_exponential():
    """Vbar(a, b) = exp(al + be a + ga b) with be != ga, so a transposed
    argument changes the result."""
    s_hat = np.array([0.0, 0.05, 0.25, 0.5, 1.0])
    s = osh.eval_grid(s_hat)
    al, be, ga = 2.0, -1.3, -4.1
    vb = np.exp(al + be * s_hat[:, None] + ga * s_hat[None, :])
    got = osh.interp_pairs(s_hat, vb, s)
    n = len(s)
    for i in range(n):
        for k in range(n):
            want = (s[k] - s[i]) ** 2 * np.exp(al + be * s[i] + ga * s[k]) if k > i else 0.0
            assert got[i, k] == pytest.approx(want, rel=1e-11, abs=0), (i, k)


@pytest.mark.parametrize("seed", range(4))
def test_pairs_pass_through_samples(seed):
    """Arbitrary positive samples: the prediction at every sampled pair
    (s^_i, s^_j), j > i, is (s^_j - s^_i)^2 times the sample."""
    rng = np.random.default_rng(seed)
    s_hat = np.array([0.0, 0.05, 0.25, 0.5, 1.0])
    vb = np.exp(rng.normal(size=(5, 5)) * 2)
    s = osh.eval_grid(s_hat)
    got = osh.interp_pairs(s_hat, vb, s)
    pos = [int(np.flatnonzero(s == v)[0]) for v in s_hat]
    for i in range(5):
        for j in range(i + 1, 5):
            want = (s_hat[j] - s_hat[i]) ** 2 * vb[i, j]
            assert got[pos[i], pos[j]] == pytest.approx(want, rel=1e-12)


def test_nn_cost_hand_values():
    s_hat = [0.0, 0.05, 0.25, 0.5, 1.0]
    r_hat = [50.0, 40.0, 30.0, 20.0, 10.0]
    s = [0.0, 0.01, 0.05, 0.06, 0.25, 0.3, 0.999, 1.0]
    assert list(osh.nn_cost(s_hat, r_hat, s)) == [50, 40, 40, 30, 30, 20, 10, 10]


def _random_tables(rng, n):
    r = np.sort(rng.uniform(5, 50, n))[::-1].copy()
    vp = np.triu(np.exp(rng.normal(size=(n, n))), 1)
    vs = np.exp(rng.normal(size=n))
    return vp, vs, r


@pytest.mark.parametrize("L", [0, 1, 2, 3, 4])
def test_dp_equals_brute_force(L):
    rng = np.random.default_rng(100 + L)
    for _ in range(3):
        vp, vs, r = _random_tables(rng, 11)
        i_b, c_b = osh.select_brute(L, vp, vs, r)
        i_d, c_d = osh.select_dp(L, vp, vs, r)
        assert c_d == pytest.approx(c_b, rel=1e-13)
        assert i_d[0] == 0 and all(a < b for a, b in zip(i_d, i_d[1:])) and len(i_d) == L + 1
        assert osh.c_fs(i_d, vp, vs, r) == pytest.approx(c_d, rel=1e-13)


def test_single_level_cost():
    vp, vs, r = _random_tables(np.random.default_rng(3), 6)
    assert osh.c_fs((0,), vp, vs, r) == pytest.approx(r[0] * vs[0], rel=1e-15)
    V, C = osh.level_terms((0, 2, 5), vp, vs, r)
    assert list(V) == [vp[0, 2], vp[2, 5], vs[5]] and list(C) == [r[0] + r[2], r[2] + r[5], r[5]]


def test_grid_holds_printed_shifts():
    g = _golden_shifts()
    s = osh.eval_grid(np.array(g["sampling"]))
    assert len(s) == 81 + 3  # 0.05, 0.25, 0.5 are inserted; 0 and 1 are grid points
    assert s[0] == 0.0 and s[-1] == 1.0 and np.all(np.diff(s) > 0)
    for v in g["sampling"]:
        assert v in s
    for v in g["optimal"]:  # printed to three decimals (1e-5 exactly)
        assert np.any(np.round(s, 3) == v) or np.any(np.abs(s - v) <= 1e-12 * v), v
