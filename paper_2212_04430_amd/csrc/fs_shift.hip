// Shift selection (paper Sec. 3.2-3.3).
//
// Host side: the sampled V_L(s^_i), Vbar_l(s^_i, s^_j) and iteration counts
// r(s^_i) are carried to the evaluation set by monotone cubic Hermite
// interpolation in log space (PCHIP: Fritsch & Carlson 1980, slopes of
// Fritsch & Butland 1984; a line through two points), the 2-D scheme of the
// paper's interpolation algorithm for Vbar_l, and the solver-cost rule
// r(s) = r(s^_j) for s^_{j-1} < s <= s^_j (eq. solver_cost_shift).  The
// multilevel cost of eq. ml_cost_shifts (eps = 1) is
//   C_FS = (sum_l sqrt(C_l V_l))^2,  C_l = r(sigma_l) + r(sigma_{l+1}) (l < L),
//   C_L = r(sigma_L),
// so the sum is a path cost over increasing indices and eq. opt_shifts is a
// shortest path with L edges, found by dynamic programming in O(L n^2).
//
// GPU side: the paper's own method, an exhaustive sweep over every
// combination 0 < j_1 < ... < j_L <= n-1.  Each thread takes a run of
// consecutive prefixes (j_1..j_{L-1}) in lexicographic order (unranked once,
// then advanced by the lexicographic successor) and scans every last index
// j_L.  The level terms sit in LDS.  Costs are summed left to right, as in the
// dynamic program, so both give bit-identical sums for the same path.
#include "fs_shift.h"

#include <algorithm>
#include <cmath>
#include <string>

namespace fs {

namespace {

[[noreturn]] void bad(const std::string& m) { throw ShiftArgError(m); }

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Monotone piecewise cubic Hermite interpolant through (x_k, y_k).
class Pchip {
public:
    Pchip(std::vector<double> x, std::vector<double> y) : x_(std::move(x)), y_(std::move(y)), g_(x_.size(), 0.0) {
        const int n = (int)x_.size();
        if (n < 2) return;
        std::vector<double> h(n - 1), d(n - 1);
        for (int k = 0; k + 1 < n; ++k) {
            h[k] = x_[k + 1] - x_[k];
            d[k] = (y_[k + 1] - y_[k]) / h[k];
        }
        if (n == 2) {
            g_[0] = g_[1] = d[0];
            return;
        }
        for (int k = 1; k + 1 < n; ++k) {
            if (d[k - 1] * d[k] <= 0.0) continue;  // local extremum or flat: zero slope
            const double a = 2.0 * h[k] + h[k - 1], b = h[k] + 2.0 * h[k - 1];
            g_[k] = (a + b) / (a / d[k - 1] + b / d[k]);  // weighted harmonic mean
        }
        g_[0] = end_slope(h[0], h[1], d[0], d[1]);
        g_[n - 1] = end_slope(h[n - 2], h[n - 3], d[n - 2], d[n - 3]);
    }

    double operator()(double t) const {
        const int n = (int)x_.size();
        if (n == 1) return y_[0];
        int k = 0;
        while (k < n - 2 && t > x_[k + 1]) ++k;
        const double hk = x_[k + 1] - x_[k];
        const double v = (t - x_[k]) / hk, w = 1.0 - v;
        return (1.0 + 2.0 * v) * w * w * y_[k] + v * w * w * hk * g_[k] + v * v * (3.0 - 2.0 * v) * y_[k + 1] -
               v * v * w * hk * g_[k + 1];
    }

private:
    static int sgn(double v) { return (v > 0) - (v < 0); }
    // One-sided three-point slope, limited so the end interval stays shape preserving.
    static double end_slope(double h0, double h1, double d0, double d1) {
        const double e = ((2.0 * h0 + h1) * d0 - h0 * d1) / (h0 + h1);
        if (sgn(e) != sgn(d0)) return 0.0;
        if (sgn(d0) != sgn(d1) && std::fabs(e) > std::fabs(3.0 * d0)) return 3.0 * d0;
        return e;
    }
    std::vector<double> x_, y_, g_;
};

void check_model(const fs_shift_model& M) {
    if (M.m < 2 || M.m > 16) bad("m must be in 2..16");
    if (!M.s_hat || !M.v_single || !M.v_pair || !M.iters || !M.s) bad("null array in the shift model");
    if (M.s_hat[0] != 0.0) bad("s_hat[0] must be 0");
    for (int i = 0; i + 1 < M.m; ++i)
        if (!(M.s_hat[i + 1] > M.s_hat[i]) || !std::isfinite(M.s_hat[i + 1])) bad("s_hat must be strictly increasing");
    for (int i = 0; i < M.m; ++i) {
        if (!finite_pos(M.v_single[i])) bad("v_single must be finite and > 0");
        if (!finite_pos(M.iters[i])) bad("iters must be finite and > 0");
        for (int j = i; j < M.m; ++j)
            if (!finite_pos(M.v_pair[i * M.m + j])) bad("v_pair[i][j], j >= i, must be finite and > 0");
    }
    if (M.n < 2 || M.n > 4096) bad("n must be in 2..4096");
    if (M.s[0] != 0.0) bad("s[0] must be 0");
    for (int k = 0; k + 1 < M.n; ++k)
        if (!(M.s[k + 1] > M.s[k])) bad("s must be strictly increasing");
    if (M.s[M.n - 1] > M.s_hat[M.m - 1]) bad("s must end at or below the largest sampling shift");
    for (int i = 0, k = 0; i < M.m; ++i) {
        while (k < M.n && M.s[k] < M.s_hat[i]) ++k;
        if (k == M.n || M.s[k] != M.s_hat[i]) bad("s must contain every sampling shift");
    }
}

}  // namespace

std::vector<double> paper_eval_grid(const double* s_hat, int m) {
    if (!s_hat || m < 2 || m > 16) bad("m must be in 2..16");
    const double top = s_hat[m - 1];
    std::vector<double> g{0.0};
    // 4 points from 1e-5 to 1e-2, then 76 from 0.011 to 1, log-spaced
    for (int k = 0; k < 4; ++k) g.push_back(std::pow(10.0, -5.0 + k));
    const double a = std::log10(1e-2 + 1e-3);
    const double step = (0.0 - a) / 75.0;
    for (int k = 0; k < 76; ++k) g.push_back(k == 75 ? 1.0 : std::pow(10.0, k * step + a));
    std::vector<double> out;
    for (double v : g)
        if (v <= top) out.push_back(v);
    for (int i = 0; i < m; ++i)
        if (std::find(out.begin(), out.end(), s_hat[i]) == out.end()) out.push_back(s_hat[i]);
    std::sort(out.begin(), out.end());
    return out;
}

ShiftTables shift_tables(const fs_shift_model& M) {
    check_model(M);
    const int m = M.m, n = M.n;
    const std::vector<double> sh(M.s_hat, M.s_hat + m), s(M.s, M.s + n);
    auto vbar = [&](int i, int j) { return M.v_pair[i * m + j]; };
    ShiftTables T;
    T.n = n;
    T.s = s;
    T.vp.assign((size_t)n * n, 0.0);
    T.vs.resize(n);
    T.r.resize(n);
    // V_L along the sampling shifts
    {
        std::vector<double> ly(m);
        for (int i = 0; i < m; ++i) ly[i] = std::log(M.v_single[i]);
        Pchip q(sh, ly);
        for (int k = 0; k < n; ++k) T.vs[k] = std::exp(q(s[k]));
    }
    // Vbar_l, first argument at each sampled second argument s^_j (j >= 1): only
    // evaluation shifts s_k <= s^_j are needed
    std::vector<double> col((size_t)n * m, 0.0);
    for (int j = 1; j < m; ++j) {
        std::vector<double> x(sh.begin(), sh.begin() + j + 1), y(j + 1);
        for (int i = 0; i <= j; ++i) y[i] = std::log(vbar(i, j));
        Pchip q(x, y);
        for (int k = 0; k < n && s[k] <= sh[j]; ++k) col[(size_t)k * m + j] = std::exp(q(s[k]));
    }
    // ... along the diagonal
    std::vector<double> diag(n);
    {
        std::vector<double> y(m);
        for (int i = 0; i < m; ++i) y[i] = std::log(vbar(i, i));
        Pchip q(sh, y);
        for (int k = 0; k < n; ++k) diag[k] = std::exp(q(s[k]));
    }
    // ... and along the second argument at each evaluation shift s_i, through
    // the diagonal point and the sampled second arguments above s_i
    for (int i = 0; i + 1 < n; ++i) {
        std::vector<double> x{s[i]}, y{std::log(diag[i])};
        for (int j = 0; j < m; ++j)
            if (sh[j] > s[i]) {
                x.push_back(sh[j]);
                y.push_back(std::log(col[(size_t)i * m + j]));
            }
        Pchip q(x, y);
        for (int k = i + 1; k < n; ++k) {
            const double ds = s[k] - s[i];
            T.vp[(size_t)i * n + k] = ds * ds * std::exp(q(s[k]));
        }
    }
    // iteration counts: the nearest sampled shift at or above s_k
    for (int k = 0, j = 0; k < n; ++k) {
        while (sh[j] < s[k]) ++j;
        T.r[k] = M.iters[j];
    }
    T.w.assign((size_t)n * n, 0.0);
    T.u.resize(n);
    for (int i = 0; i < n; ++i) {
        T.u[i] = std::sqrt(T.r[i] * T.vs[i]);
        for (int k = i + 1; k < n; ++k) T.w[(size_t)i * n + k] = std::sqrt((T.r[i] + T.r[k]) * T.vp[(size_t)i * n + k]);
    }
    return T;
}

double shift_select_dp(const ShiftTables& T, int L, int* idx) {
    const int n = T.n;
    if (L < 0 || L > n - 1) bad("L must be in 0..n-1");
    idx[0] = 0;
    if (L == 0) return T.u[0] * T.u[0];
    // f[k]: least sum of the first l level terms over 0 = j_0 < ... < j_l = k
    std::vector<double> f(n, INFINITY), g(n);
    std::vector<int> pred((size_t)(L + 1) * n, -1);
    for (int k = 1; k < n; ++k) f[k] = T.w[k];  // w[0][k]
    for (int l = 2; l <= L; ++l) {
        std::fill(g.begin(), g.end(), INFINITY);
        for (int k = l; k < n; ++k)
            for (int i = l - 1; i < k; ++i) {
                const double c = f[i] + T.w[(size_t)i * n + k];
                if (c < g[k]) {
                    g[k] = c;
                    pred[(size_t)l * n + k] = i;
                }
            }
        f.swap(g);
    }
    double best = INFINITY;
    int kb = -1;
    for (int k = L; k < n; ++k) {
        const double c = f[k] + T.u[k];
        if (c < best) {
            best = c;
            kb = k;
        }
    }
    for (int l = L; l >= 1; --l) {
        idx[l] = kb;
        kb = l >= 2 ? pred[(size_t)l * n + kb] : 0;
    }
    return best * best;
}

// ------------------------------------------------------------------ GPU sweep

namespace {

__device__ inline void keep_min(double& c, uint64_t& k, double c2, uint64_t k2) {
    if (c2 < c || (c2 == c && k2 < k)) {
        c = c2;
        k = k2;
    }
}

__device__ inline void wave_min(double& c, uint64_t& k) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double c2 = __shfl_xor(c, off, 64);
        const uint64_t k2 = __shfl_xor(k, off, 64);
        keep_min(c, k, c2, k2);
    }
}

// Block of 256: (c, k) of thread 0 is the block's least (ties: smaller key).
__device__ inline void block_min(double& c, uint64_t& k) {
    __shared__ double sc[4];
    __shared__ uint64_t sk[4];
    wave_min(c, k);
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sc[wv] = c;
        sk[wv] = k;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int i = 1; i < 4; ++i) keep_min(c, k, sc[i], sk[i]);
}

// K = L - 1 prefix indices from {1, ..., n-2}; the last index runs over
// (j_{L-1}, n-1].  Prefix ranks are lexicographic.
template <int K>
__global__ void __launch_bounds__(256) k_shift_sweep(const double* __restrict__ w, const double* __restrict__ u,
                                                     const uint64_t* __restrict__ binom, int n, uint64_t n_prefix,
                                                     uint64_t per_thread, double* __restrict__ pc,
                                                     uint64_t* __restrict__ pk) {
    extern __shared__ double lds[];  // w [n][n], then u [n]
    for (int i = threadIdx.x; i < n * n; i += 256) lds[i] = w[i];
    for (int i = threadIdx.x; i < n; i += 256) lds[n * n + i] = u[i];
    __syncthreads();
    const double* lu = lds + n * n;
    const int M = n - 2;  // prefix values 1..M
    double best = INFINITY;
    uint64_t bkey = ~0ull;
    const uint64_t r0 = ((uint64_t)blockIdx.x * 256 + threadIdx.x) * per_thread;
    if (r0 < n_prefix) {
        const uint64_t cnt = (n_prefix - r0 < per_thread) ? n_prefix - r0 : per_thread;
        int c[K > 0 ? K : 1];
        {
            uint64_t r = r0;
            int x = 1;
#pragma unroll
            for (int p = 0; p < K; ++p) {
                // prefixes whose position p holds x: choose the rest from the M - x values above x
                while (x < M) {  // x never passes M for r0 < n_prefix; the bound keeps the table read in range
                    const uint64_t b = binom[(M - x) * (kSweepMaxL + 1) + (K - 1 - p)];
                    if (r < b) break;
                    r -= b;
                    ++x;
                }
                c[p] = x++;
            }
        }
        for (uint64_t q = 0; q < cnt; ++q) {
            double pre = 0.0;
            int last = 0;
            if (K > 0) {
                pre = lds[c[0]];  // w[0][j_1]
#pragma unroll
                for (int p = 1; p < K; ++p) pre = pre + lds[c[p - 1] * n + c[p]];
                last = c[K - 1];
            }
            const double* wr = lds + last * n;
            const uint64_t kb = (r0 + q) << 7;
            for (int j = last + 1; j < n; ++j) {
                const double cost = (pre + wr[j]) + lu[j];
                if (cost < best) {
                    best = cost;
                    bkey = kb | (uint64_t)j;
                }
            }
            // lexicographic successor of the prefix
            bool done = false;
#pragma unroll
            for (int p = K - 1; p >= 0; --p) {
                if (!done && c[p] < M - (K - 1 - p)) {
                    c[p] += 1;
#pragma unroll
                    for (int q2 = p + 1; q2 < K; ++q2) c[q2] = c[q2 - 1] + 1;
                    done = true;
                }
            }
        }
    }
    block_min(best, bkey);
    if (threadIdx.x == 0) {
        pc[blockIdx.x] = best;
        pk[blockIdx.x] = bkey;
    }
}

__global__ void __launch_bounds__(256) k_sweep_reduce(const double* __restrict__ pc, const uint64_t* __restrict__ pk,
                                                      int nb, double* out_c, uint64_t* out_k) {
    double c = INFINITY;
    uint64_t k = ~0ull;
    for (int i = threadIdx.x; i < nb; i += 256) keep_min(c, k, pc[i], pk[i]);
    block_min(c, k);
    if (threadIdx.x == 0) {
        out_c[0] = c;
        out_k[0] = k;
    }
}

}  // namespace

void launch_shift_sweep(int L, const double* w, const double* u, const uint64_t* binom, int n, uint64_t n_prefix,
                        uint64_t per_thread, int grid, double* pc, uint64_t* pk, hipStream_t s) {
    const size_t lds = sizeof(double) * ((size_t)n * n + n);
#define FS_SWEEP(K)                                                                                              \
    case K + 1:                                                                                                  \
        hipLaunchKernelGGL(k_shift_sweep<K>, dim3(grid), dim3(256), lds, s, w, u, binom, n, n_prefix, per_thread, \
                           pc, pk);                                                                              \
        break;
    switch (L) {
        FS_SWEEP(0)
        FS_SWEEP(1)
        FS_SWEEP(2)
        FS_SWEEP(3)
        FS_SWEEP(4)
        FS_SWEEP(5)
        FS_SWEEP(6)
        FS_SWEEP(7)
        default:
            bad("sweep L must be in 1..8");
    }
#undef FS_SWEEP
}

void launch_sweep_reduce(const double* pc, const uint64_t* pk, int nb, double* out_c, uint64_t* out_k,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_sweep_reduce, dim3(1), dim3(256), 0, s, pc, pk, nb, out_c, out_k);
}

}  // namespace fs
