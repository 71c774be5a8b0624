"""ctypes binding of libfsmlmc.so: the C-ABI entry points under the same names.

Argument marshalling only: every computation runs in the HIP library.  Arrays
may be numpy arrays (host, complex128/float64, C-contiguous) or torch tensors
on the GPU (device pointers are passed straight through); outputs are returned
as the same kind of array.  If the library is not built or cannot be loaded
this module raises at import time -- there is no fallback.
"""

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("FSMLMC_LIB") or os.path.join(HERE, "libfsmlmc.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2212_04430_amd.build`")
# One HIP runtime per process: when torch is present its runtime is loaded
# first and the library binds to it (same soname), so torch tensors and
# streams are valid handles for the library.
try:
    import torch  # noqa: F401
except ImportError:
    torch = None
_lib = C.CDLL(LIB_PATH)

FS_OK, FS_E_ARG, FS_E_HIP, FS_E_OOM, FS_E_NOCONV, FS_E_BREAKDOWN, FS_E_STATE = 0, -1, -2, -3, -4, -5, -6
FS_F64, FS_F32, FS_F16, FS_BF16 = 0, 1, 2, 3
PREC = {"f64": FS_F64, "f32": FS_F32, "f16": FS_F16, "bf16": FS_BF16}
STATUS_NAME = {0: "FS_OK", -1: "FS_E_ARG", -2: "FS_E_HIP", -3: "FS_E_OOM", -4: "FS_E_NOCONV",
               -5: "FS_E_BREAKDOWN", -6: "FS_E_STATE"}


class FsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAME.get(code, code)}: {msg}")
        self.code = code


_DP = C.POINTER(C.c_double)


class fs_solve_params(C.Structure):
    _fields_ = [("m0", C.c_double), ("tol", C.c_double), ("max_iter", C.c_int32),
                ("storage", C.c_int32), ("rhs_block", C.c_int32), ("use_graph", C.c_int32),
                ("reliable_delta", C.c_double), ("check_every", C.c_int32), ("batched", C.c_int32),
                ("even_odd", C.c_int32), ("multi_shift", C.c_int32)]


class fs_solve_stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("reliable_updates", C.c_int32), ("status", C.c_int32),
                ("restarts", C.c_int32), ("true_rel_residual", C.c_double)]


class fs_est_params(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("n_noise", C.c_int32), ("gamma_mask", C.c_uint16),
                ("p_max", C.c_int32), ("solve", fs_solve_params), ("n_level", C.POINTER(C.c_int32)),
                ("shared_noise", C.c_int32), ("report_fp64_error", C.c_int32), ("hpe_order", C.c_int32),
                ("pad_", C.c_int32), ("pass_bytes", C.c_int64)]

    def set_n_level(self, counts):
        """Per-level sample counts N_l (None: n_noise on every level); the array is kept alive here."""
        if counts is None:
            self._n_level = None
            self.n_level = C.POINTER(C.c_int32)()
        else:
            self._n_level = np.ascontiguousarray(counts, dtype=np.int32)
            self.n_level = self._n_level.ctypes.data_as(C.POINTER(C.c_int32))
        return self

    def n_slots(self, n_levels):
        """Sample slots per level of the samples array (max N_l)."""
        nl = getattr(self, "_n_level", None)
        return int(max(nl)) if nl is not None else int(self.n_noise)


class fs_level_stat(C.Structure):
    _fields_ = [("tr_re", C.c_double), ("tr_im", C.c_double), ("var_paper", C.c_double),
                ("var_unbiased", C.c_double), ("n", C.c_int64), ("max_rel_residual", C.c_double),
                ("fp64_rel_err", C.c_double), ("err_bound", C.c_double)]


class fs_total_stat(C.Structure):
    _fields_ = [("tr_re", C.c_double), ("tr_im", C.c_double), ("v_fs", C.c_double), ("v_fs_unbiased", C.c_double),
                ("v_total", C.c_double), ("v_total_unbiased", C.c_double), ("err_bound", C.c_double)]


class fs_est_report(C.Structure):
    _fields_ = [("systems", C.c_int64), ("iterations", C.c_int64), ("reliable_updates", C.c_int64),
                ("dslash_calls", C.c_int64), ("max_rel_residual", C.c_double), ("seconds", C.c_double)]


class fs_shift_model(C.Structure):
    _fields_ = [("m", C.c_int32), ("s_hat", _DP), ("v_single", _DP), ("v_pair", _DP), ("iters", _DP),
                ("n", C.c_int32), ("s", _DP)]


_P = C.c_void_p
_sig = {
    "fs_version": (C.c_char_p, []),
    "fs_struct_sizes": (C.c_int32, [_P, C.c_int32]),
    "fs_last_error": (C.c_char_p, [_P]),
    "fs_create": (C.c_int, [C.POINTER(_P), C.POINTER(C.c_int32), C.c_int32, C.c_int32, _P]),
    "fs_destroy": (C.c_int, [_P]),
    "fs_set_instance": (C.c_int, [_P, C.c_uint32]),
    "fs_upload_gauge": (C.c_int, [_P, _P, C.c_int32]),
    "fs_gauge_info": (C.c_int, [_P, C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    "fs_set_clover": (C.c_int, [_P, C.c_double]),
    "fs_apply_dirac": (C.c_int, [_P, C.c_double, C.c_double, C.c_int32, _P, _P, C.c_int32, C.c_int32]),
    "fs_apply_dirac_noalloc": (C.c_int, [_P, C.c_double, C.c_double, C.c_int32, _P, _P, C.c_int32]),
    "fs_z4_noise": (C.c_int, [_P, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64, _P, C.c_int32]),
    "fs_displace": (C.c_int, [_P, C.c_int32, _P, _P, C.c_int32]),
    "fs_bilinear": (C.c_int, [_P, C.c_int32, _P, _P, _P, C.c_int32]),
    "fs_solve_shifted": (C.c_int, [_P, C.POINTER(fs_solve_params), _P, C.c_int32, _P, C.c_int32, _P,
                                   C.c_int32, C.POINTER(fs_solve_stats)]),
    "fs_estimate": (C.c_int, [_P, C.POINTER(fs_est_params), _P, C.c_int32, C.POINTER(fs_level_stat), _P,
                              C.POINTER(fs_est_report)]),
    "fs_sample_variances": (C.c_int, [_P, C.POINTER(fs_est_params), _P, C.c_int32, C.POINTER(fs_level_stat),
                                      C.POINTER(fs_level_stat), _P, _P, C.POINTER(fs_est_report)]),
    "fs_batch_create": (C.c_int, [C.POINTER(_P), C.POINTER(_P), C.c_int32]),
    "fs_batch_estimate": (C.c_int, [_P, C.POINTER(fs_est_params), _P, C.c_int32, C.POINTER(fs_level_stat), _P,
                                    C.POINTER(fs_est_report)]),
    "fs_level_totals": (C.c_int, [C.POINTER(fs_level_stat), C.c_int32, C.c_int32, C.POINTER(fs_total_stat)]),
    "fs_optimal_samples": (C.c_int, [_DP, _DP, C.c_int32, C.c_double, C.c_int32, C.POINTER(C.c_int32), _DP]),
    "fs_batch_destroy": (C.c_int, [_P]),
    "fs_autotune": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_char_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "fs_set_tuning": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "fs_time_dslash": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                 C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "fs_time_copy": (C.c_int, [_P, C.c_uint64, C.c_int32, C.POINTER(C.c_double)]),
    "fs_time_dslash_eo_each": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_float),
                                         C.POINTER(C.c_double)]),
    "fs_set_eo_tuning": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int32]),
    "fs_time_dslash_eo": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                    C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "fs_probing_colours": (C.c_int, [C.POINTER(C.c_int32), C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                                     C.POINTER(C.c_int32)]),
    "fs_estimate_probed": (C.c_int, [_P, C.POINTER(fs_est_params), _P, C.c_int32, C.POINTER(C.c_int32), C.c_int32,
                                     C.POINTER(fs_level_stat), _P, C.POINTER(fs_est_report)]),
    "fs_eval_grid": (C.c_int, [_DP, C.c_int32, _DP, C.c_int32, C.POINTER(C.c_int32)]),
    "fs_shift_tables": (C.c_int, [C.POINTER(fs_shift_model), _DP, _DP, _DP]),
    "fs_select_shifts": (C.c_int, [C.POINTER(fs_shift_model), C.c_int32, C.POINTER(C.c_int32), _DP, _DP, _DP]),
    "fs_sweep_shifts": (C.c_int, [_P, C.POINTER(fs_shift_model), C.c_int32, C.POINTER(C.c_int32), _DP, _DP]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sig)


def _check(code, allow=()):
    if code != FS_OK and code not in allow:
        raise FsError(code, _lib.fs_last_error(None).decode())
    return code


def _is_torch(a):
    return type(a).__module__.startswith("torch")


def _ptr(a):
    """(pointer, is_device) of a numpy array or a CUDA/HIP torch tensor."""
    if _is_torch(a):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return C.c_void_p(a.data_ptr()), 1 if a.is_cuda else 0
    if not a.flags.c_contiguous:
        raise ValueError("array must be C-contiguous")
    return C.c_void_p(a.ctypes.data), 0


def _host_c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _like(a, shape):
    if _is_torch(a):
        import torch
        return torch.empty(shape, dtype=torch.complex128, device=a.device)
    return np.empty(shape, dtype=np.complex128)


def _prec(p):
    return PREC[p] if isinstance(p, str) else int(p)


def solve_params(m0, tol=1e-10, max_iter=10000, storage="f64", rhs_block=0, use_graph=0,
                 reliable_delta=0.0, check_every=0, batched=0, even_odd=0, multi_shift=0):
    return fs_solve_params(m0, tol, max_iter, _prec(storage), rhs_block, int(use_graph), reliable_delta,
                           check_every, int(batched), int(even_odd), int(multi_shift))


# ------------------------------------------------------------------ entry points

def fs_version():
    return _lib.fs_version().decode()


STRUCTS = (fs_solve_params, fs_solve_stats, fs_est_params, fs_level_stat, fs_total_stat, fs_est_report,
           fs_shift_model)


def fs_struct_sizes():
    """sizeof of the header's structs, in the order of STRUCTS."""
    n = _lib.fs_struct_sizes(None, 0)
    out = (C.c_int64 * n)()
    _lib.fs_struct_sizes(C.cast(out, _P), n)
    return list(out)


def fs_last_error(ctx=None):
    """Message of the last failing call on ctx, or on this thread (ctx None)."""
    return _lib.fs_last_error(ctx).decode()


def fs_create(dims, t_antiperiodic=0, device=0, stream=None):
    h = C.c_void_p()
    d = (C.c_int32 * 4)(*[int(x) for x in dims])
    _check(_lib.fs_create(C.byref(h), d, int(t_antiperiodic), int(device),
                          C.c_void_p(stream) if stream else None))
    return h


def fs_destroy(ctx):
    _check(_lib.fs_destroy(ctx))


def fs_set_instance(ctx, instance):
    _check(_lib.fs_set_instance(ctx, int(instance)))


def fs_upload_gauge(ctx, links):
    if not _is_torch(links):
        links = _host_c128(links)
    p, dev = _ptr(links)
    _check(_lib.fs_upload_gauge(ctx, p, dev))


def fs_set_clover(ctx, c_sw):
    """Use the clover-improved operator with coefficient c_sw (0: plain Wilson)."""
    _check(_lib.fs_set_clover(ctx, float(c_sw)))


def fs_gauge_info(ctx):
    """(two_rows, su3_defect): whether the FP32 stencils rebuild row 2 of the links."""
    tr = C.c_int32(0)
    d = C.c_double(0.0)
    _check(_lib.fs_gauge_info(ctx, C.byref(tr), C.byref(d)))
    return bool(tr.value), d.value


def fs_apply_dirac(ctx, m0, sigma, storage, psi):
    """(D + sigma) psi for one spinor (V,4,3) or a stack (n,V,4,3)."""
    if not _is_torch(psi):
        psi = _host_c128(psi)
    n = 1 if psi.ndim == 3 else psi.shape[0]
    out = _like(psi, tuple(psi.shape))
    pi, dev = _ptr(psi)
    po, _ = _ptr(out)
    _check(_lib.fs_apply_dirac(ctx, float(m0), float(sigma), _prec(storage), pi, po, n, dev))
    return out


def fs_apply_dirac_noalloc(ctx, m0, sigma, storage, psi, out):
    """(D + sigma) psi into out, both CUDA/HIP torch tensors (V,4,3) or (n,V,4,3) complex128,
    through the allocation-free entry point."""
    if not (_is_torch(psi) and psi.is_cuda and _is_torch(out) and out.is_cuda):
        raise ValueError("fs_apply_dirac_noalloc takes device tensors")
    if psi.shape != out.shape:
        raise ValueError("in and out must have the same shape")
    n = 1 if psi.ndim == 3 else psi.shape[0]
    pi, _ = _ptr(psi)
    po, _ = _ptr(out)
    _check(_lib.fs_apply_dirac_noalloc(ctx, float(m0), float(sigma), _prec(storage), pi, po, n))
    return out


def fs_z4_noise(ctx, V, seed, instance, level, sample, device=None):
    out = _like(device, (V, 4, 3)) if device is not None else np.empty((V, 4, 3), dtype=np.complex128)
    po, dev = _ptr(out)
    _check(_lib.fs_z4_noise(ctx, int(seed), int(instance), int(level), int(sample), po, dev))
    return out


def fs_displace(ctx, p, psi):
    if not _is_torch(psi):
        psi = _host_c128(psi)
    out = _like(psi, tuple(psi.shape))
    pi, dev = _ptr(psi)
    po, _ = _ptr(out)
    _check(_lib.fs_displace(ctx, int(p), pi, po, dev))
    return out


def fs_bilinear(ctx, p_max, y, x):
    """out[p, n] = y^+ Gamma_n Omega_p x (host complex128 array (p_max+1, 16))."""
    if not _is_torch(y):
        y = _host_c128(y)
        x = _host_c128(x)
    out = np.empty((p_max + 1, 16), dtype=np.complex128)
    py, dev = _ptr(y)
    px, _ = _ptr(x)
    _check(_lib.fs_bilinear(ctx, int(p_max), py, px, C.c_void_p(out.ctypes.data), 0))
    return out


def fs_solve_shifted(ctx, params, sigma, B, allow_noconv=False):
    """X[s, r] = (D + sigma_s)^-1 B[r]; returns (X, stats list, status)."""
    if not _is_torch(B):
        B = _host_c128(B)
    if B.ndim == 3:
        B = B.reshape((1,) + tuple(B.shape))
    n_rhs = B.shape[0]
    sig = np.ascontiguousarray(sigma, dtype=np.float64)
    X = _like(B, (len(sig),) + tuple(B.shape))
    st = (fs_solve_stats * (len(sig) * n_rhs))()
    pb, dev = _ptr(B)
    px, _ = _ptr(X)
    code = _lib.fs_solve_shifted(ctx, C.byref(params), C.c_void_p(sig.ctypes.data), len(sig), pb, n_rhs, px,
                                 dev, st)
    _check(code, allow=(FS_E_NOCONV,) if allow_noconv else ())
    return X, [st[i] for i in range(len(st))], code


STAT_FIELDS = ("tr_re", "tr_im", "var_paper", "var_unbiased", "n", "max_rel_residual", "fp64_rel_err", "err_bound")


_STAT_DTYPE = np.dtype([(f, np.int64 if t is C.c_int64 else np.float64) for f, t in fs_level_stat._fields_])


def _stats_array(stats, shape):
    """fs_level_stat array (ctypes) -> float array shape + (len(STAT_FIELDS),)."""
    assert _STAT_DTYPE.itemsize == C.sizeof(fs_level_stat)
    rec = np.frombuffer(stats, dtype=_STAT_DTYPE, count=len(stats))
    a = np.stack([rec[f].astype(np.float64) for f in STAT_FIELDS], axis=-1)
    return a.reshape(shape + (len(STAT_FIELDS),))


def fs_estimate(ctx, params, sigma, want_samples=False, allow_noconv=False, raw=False):
    """Per-level stats as an array [L+1, 16, p_max+1, 8] (STAT_FIELDS: tr_re, tr_im,
    var_paper, var_unbiased, n, max_rel_residual, fp64_rel_err, err_bound), the
    per-sample X [L+1, N, 16, p_max+1] (N = max_l N_l; or None) and the report.
    raw=True also returns the fs_level_stat array (for fs_level_totals)."""
    sig = np.ascontiguousarray(sigma, dtype=np.float64)
    L = len(sig) - 1
    P1 = params.p_max + 1
    out = (fs_level_stat * ((L + 1) * 16 * P1))()
    N = params.n_slots(L + 1)
    samples = np.zeros((L + 1, N, 16, P1), dtype=np.complex128) if want_samples else None
    rep = fs_est_report()
    code = _lib.fs_estimate(ctx, C.byref(params), C.c_void_p(sig.ctypes.data), L, out,
                            C.c_void_p(samples.ctypes.data) if want_samples else None, C.byref(rep))
    _check(code, allow=(FS_E_NOCONV,) if allow_noconv else ())
    st = _stats_array(out, (L + 1, 16, P1))
    return (st, samples, rep, out) if raw else (st, samples, rep)


def fs_level_totals(levels, L, p_max):
    """Totals per (Gamma_n, p) from an fs_level_stat array: dict of [16, p_max+1] arrays
    (tr (complex), v_fs, v_fs_unbiased, v_total, v_total_unbiased, err_bound)."""
    P1 = p_max + 1
    out = (fs_total_stat * (16 * P1))()
    _check(_lib.fs_level_totals(levels, int(L), int(p_max), out))
    g = lambda f: np.array([getattr(o, f) for o in out]).reshape(16, P1)
    return {"tr": g("tr_re") + 1j * g("tr_im"), "v_fs": g("v_fs"), "v_fs_unbiased": g("v_fs_unbiased"),
            "v_total": g("v_total"), "v_total_unbiased": g("v_total_unbiased"), "err_bound": g("err_bound")}


def fs_optimal_samples(v_levels, c_levels, eps2, n_min=2):
    """(N_l [L+1] int array, mu) of eq. num_samples."""
    v = np.ascontiguousarray(v_levels, dtype=np.float64)
    c = np.ascontiguousarray(c_levels, dtype=np.float64)
    n = np.zeros(len(v), dtype=np.int32)
    mu = C.c_double()
    _check(_lib.fs_optimal_samples(_dp(v), _dp(c), len(v) - 1, float(eps2), int(n_min),
                                   n.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(mu)))
    return n, mu.value


def fs_sample_variances(ctx, params, shifts, want_samples=False, allow_noconv=False):
    """Variance-sampling phase.  Returns the single-shift stats [m, 16, p_max+1, 6],
    the pair stats [m, m, 16, p_max+1, 6] (zero for j < i), the samples
    [m + m(m+1)/2, N, 16, p_max+1] (singles, then pairs (i, j >= i); or None),
    the mean iterations per shift [m] and the report."""
    sh = np.ascontiguousarray(shifts, dtype=np.float64)
    m = len(sh)
    P1 = params.p_max + 1
    single = (fs_level_stat * (m * 16 * P1))()
    pair = (fs_level_stat * (m * m * 16 * P1))()
    n_slot = m + m * (m + 1) // 2
    samples = np.zeros((n_slot, params.n_noise, 16, P1), dtype=np.complex128) if want_samples else None
    iters = np.zeros(m)
    rep = fs_est_report()
    code = _lib.fs_sample_variances(ctx, C.byref(params), C.c_void_p(sh.ctypes.data), m, single, pair,
                                    C.c_void_p(samples.ctypes.data) if want_samples else None,
                                    C.c_void_p(iters.ctypes.data), C.byref(rep))
    _check(code, allow=(FS_E_NOCONV,) if allow_noconv else ())
    return (_stats_array(single, (m, 16, P1)), _stats_array(pair, (m, m, 16, P1)), samples, iters,
            rep)


def fs_batch_create(ctxs):
    h = C.c_void_p()
    arr = (C.c_void_p * len(ctxs))(*[c.value for c in ctxs])
    _check(_lib.fs_batch_create(C.byref(h), arr, len(ctxs)))
    return h


def fs_batch_estimate(batch, n_inst, params, sigma, allow_noconv=False, want_samples=False):
    """Stats [n_inst, L+1, 16, p_max+1, 8] and the report; with want_samples also the
    per-sample X [n_inst, L+1, N, 16, p_max+1] (returned between them)."""
    sig = np.ascontiguousarray(sigma, dtype=np.float64)
    L = len(sig) - 1
    P1 = params.p_max + 1
    out = (fs_level_stat * (n_inst * (L + 1) * 16 * P1))()
    N = params.n_slots(L + 1)
    samples = np.zeros((n_inst, L + 1, N, 16, P1), dtype=np.complex128) if want_samples else None
    rep = fs_est_report()
    code = _lib.fs_batch_estimate(batch, C.byref(params), C.c_void_p(sig.ctypes.data), L, out,
                                  C.c_void_p(samples.ctypes.data) if want_samples else None, C.byref(rep))
    _check(code, allow=(FS_E_NOCONV,) if allow_noconv else ())
    st = _stats_array(out, (n_inst, L + 1, 16, P1))
    return (st, samples, rep) if want_samples else (st, rep)


def fs_batch_destroy(batch):
    _check(_lib.fs_batch_destroy(batch))


def fs_autotune(ctx, storage, n_sys, cache_path=None):
    nr = C.c_int32()
    wg = C.c_int32()
    _check(_lib.fs_autotune(ctx, _prec(storage), int(n_sys), cache_path.encode() if cache_path else None,
                            C.byref(nr), C.byref(wg)))
    return nr.value, wg.value


def fs_set_tuning(ctx, storage, rhs_block, wg, variant, occ=0):
    _check(_lib.fs_set_tuning(ctx, _prec(storage), int(rhs_block), int(wg), int(variant), int(occ)))


def fs_time_dslash_eo(ctx, storage, n_sys, rhs_block=0, n_launch=20, occ=-1):
    ms = C.c_double()
    b = C.c_double()
    _check(_lib.fs_time_dslash_eo(ctx, _prec(storage), int(n_sys), int(rhs_block), int(occ), int(n_launch),
                                  C.byref(ms), C.byref(b)))
    return ms.value, b.value


def fs_time_dslash(ctx, storage, n_sys, rhs_block=0, wg=0, n_launch=20, ilp=-1, occ=-1):
    ms = C.c_double()
    b = C.c_double()
    _check(_lib.fs_time_dslash(ctx, _prec(storage), int(n_sys), int(rhs_block), int(wg), int(ilp), int(occ),
                               int(n_launch), C.byref(ms), C.byref(b)))
    return ms.value, b.value


def fs_time_dslash_eo_each(ctx, storage, n_sys, rhs_block=0, n_launch=100):
    """(per-launch ms array, algorithmic bytes per launch) of the context's even-odd hop."""
    ms = np.zeros(n_launch, dtype=np.float32)
    b = C.c_double()
    _check(_lib.fs_time_dslash_eo_each(ctx, _prec(storage), int(n_sys), int(rhs_block), int(n_launch),
                                       ms.ctypes.data_as(C.POINTER(C.c_float)), C.byref(b)))
    return ms.astype(np.float64), b.value


def fs_set_eo_tuning(ctx, storage, variant, occ=-1):
    _check(_lib.fs_set_eo_tuning(ctx, _prec(storage), int(variant), int(occ)))


def fs_time_copy(ctx, nbytes, n_launch=20):
    ms = C.c_double()
    _check(_lib.fs_time_copy(ctx, int(nbytes), int(n_launch), C.byref(ms)))
    return ms.value


# ---------------------------------------------------------------- shift selection

def _dp(a):
    return a.ctypes.data_as(_DP)


class ShiftModel:
    """Host arrays of an fs_shift_model, kept alive with the struct."""

    def __init__(self, s_hat, v_single, v_pair, iters, s):
        self.arrays = [np.ascontiguousarray(a, dtype=np.float64) for a in (s_hat, v_single, v_pair, iters, s)]
        sh, vs, vp, it, ev = self.arrays
        m = len(sh)
        if vs.shape != (m,) or vp.shape != (m, m) or it.shape != (m,):
            raise ValueError("shift model arrays must be [m], [m], [m][m], [m]")
        self.n = len(ev)
        self.c = fs_shift_model(m, _dp(sh), _dp(vs), _dp(vp), _dp(it), self.n, _dp(ev))


def fs_eval_grid(s_hat):
    sh = np.ascontiguousarray(s_hat, dtype=np.float64)
    out = np.zeros(256)
    n = C.c_int32()
    _check(_lib.fs_eval_grid(_dp(sh), len(sh), _dp(out), len(out), C.byref(n)))
    return out[:n.value].copy()


def fs_shift_tables(model):
    """(V_l(s_i, s_k) [n][n], V_L(s_k) [n], r(s_k) [n]) on the evaluation set."""
    n = model.n
    vp, vs, r = np.zeros((n, n)), np.zeros(n), np.zeros(n)
    _check(_lib.fs_shift_tables(C.byref(model.c), _dp(vp), _dp(vs), _dp(r)))
    return vp, vs, r


def fs_select_shifts(model, L):
    """(idx [L+1], C_FS, V_l [L+1], C_l [L+1]) of the optimal shifts."""
    idx = (C.c_int32 * (L + 1))()
    c = C.c_double()
    v, cl = np.zeros(L + 1), np.zeros(L + 1)
    _check(_lib.fs_select_shifts(C.byref(model.c), int(L), idx, C.byref(c), _dp(v), _dp(cl)))
    return tuple(idx), c.value, v, cl


def fs_sweep_shifts(ctx, model, L):
    """(idx [L+1], C_FS, GPU ms) from the exhaustive sweep on the GPU."""
    idx = (C.c_int32 * (L + 1))()
    c = C.c_double()
    ms = C.c_double()
    _check(_lib.fs_sweep_shifts(ctx, C.byref(model.c), int(L), idx, C.byref(c), C.byref(ms)))
    return tuple(idx), c.value, ms.value


# ---------------------------------------------------------------- probing and dilution

def fs_probing_colours(dims, p, k):
    """(colour per site [V] int32, number of colours)."""
    d = (C.c_int32 * 4)(*[int(v) for v in dims])
    V = int(np.prod(dims))
    col = np.zeros(V, dtype=np.int32)
    nc = C.c_int32()
    _check(_lib.fs_probing_colours(d, int(p), int(k), col.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(nc)))
    return col, nc.value


def fs_estimate_probed(ctx, params, sigma, colours, want_samples=False, allow_noconv=False):
    """As fs_estimate, with probing colours [V] and full spin-colour dilution."""
    sig = np.ascontiguousarray(sigma, dtype=np.float64)
    col = np.ascontiguousarray(colours, dtype=np.int32)
    L = len(sig) - 1
    P1 = params.p_max + 1
    out = (fs_level_stat * ((L + 1) * 16 * P1))()
    samples = np.zeros((L + 1, params.n_noise, 16, P1), dtype=np.complex128) if want_samples else None
    rep = fs_est_report()
    n_col = int(col.max()) + 1 if col.size else 0
    code = _lib.fs_estimate_probed(ctx, C.byref(params), C.c_void_p(sig.ctypes.data), L,
                                   col.ctypes.data_as(C.POINTER(C.c_int32)), n_col, out,
                                   C.c_void_p(samples.ctypes.data) if want_samples else None, C.byref(rep))
    _check(code, allow=(FS_E_NOCONV,) if allow_noconv else ())
    return _stats_array(out, (L + 1, 16, P1)), samples, rep
