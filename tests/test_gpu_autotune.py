"""The autotuner and its on-disk cache (GPU).

fs_autotune times the stencil configurations and, on lattices with even
extents, the even-odd operator (variant and residency cap), appends the
winners to the cache file and stores them in the context.  A second context
reading the same file takes the cached choice without re-timing (the file does
not grow) and gets the same configuration; solves on a tuned context still
meet the FP64 residual checked with the oracle's operator.
"""

import numpy as np
import pytest

import synth
from oracle import lattice as lat
from oracle.philox import z4_noise

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_2212_04430_amd import _lib
    return _lib


def test_autotune_cache_round_trip(L, tmp_path):
    dims = (8, 8, 8, 8)
    U = synth.gauge_field(dims, eps=0.25, seed=2)
    cache = str(tmp_path / "tune.txt")
    c1 = L.fs_create(dims, 0, 0)
    c2 = L.fs_create(dims, 0, 0)
    try:
        L.fs_upload_gauge(c1, U)
        L.fs_upload_gauge(c2, U)
        print("autotune (timing)", flush=True)
        nr1, wg1 = L.fs_autotune(c1, "f32", 16, cache)
        lines = open(cache).read().splitlines()
        assert len(lines) == 2, lines
        assert lines[1].startswith("eo ")
        var, occ = int(lines[1].split()[-3]), int(lines[1].split()[-2])  # ... variant occ ms_per_system
        assert var in (0, 2) and -1 <= occ <= 8
        print("autotune (cached)", flush=True)
        nr2, wg2 = L.fs_autotune(c2, "f32", 16, cache)
        assert (nr1, wg1) == (nr2, wg2)
        assert open(cache).read().splitlines() == lines
        # a solve on the tuned context, checked with the oracle's operator
        V = lat.volume(dims)
        B = np.stack([z4_noise(V, 4, 0, 0, s) for s in range(4)])
        for eo in (0, 1):
            sp = L.solve_params(0.05, tol=1e-10, storage="f32", batched=1, use_graph=1, even_odd=eo)
            X, st, code = L.fs_solve_shifted(c2, sp, [0.2], B)
            assert code == 0
            for r in range(4):
                res = np.linalg.norm(B[r] - lat.wilson_apply(U, X[0, r], 0.05, 0.2, dims)) / np.linalg.norm(B[r])
                assert res <= 1.5e-10
        with pytest.raises(L.FsError) as e:
            L.fs_set_eo_tuning(c2, "f32", 1, 0)
        assert e.value.code == L.FS_E_ARG
        with pytest.raises(L.FsError) as e:
            L.fs_set_eo_tuning(c2, "f32", 2, 9)
        assert e.value.code == L.FS_E_ARG
    finally:
        L.fs_destroy(c1)
        L.fs_destroy(c2)
