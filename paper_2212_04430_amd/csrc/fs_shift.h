// Shift selection for Frequency Splitting (paper Sec. 3.2-3.3): predicted
// variances and solver costs on an evaluation set, and the argmin of the
// multilevel cost (eqs. ml_cost_shifts, opt_shifts).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <vector>

#include "../../include/fsmlmc.h"

namespace fs {

// Argument errors of this module (mapped to FS_E_ARG at the boundary).
struct ShiftArgError : std::invalid_argument {
    using std::invalid_argument::invalid_argument;
};

constexpr int kSweepMaxN = 88;  // w and u of the sweep fit in 64 KiB of LDS
constexpr int kSweepMaxL = 8;

// Predicted quantities on the n evaluation shifts.
struct ShiftTables {
    int n = 0;
    std::vector<double> s;   // [n]
    std::vector<double> vp;  // [n][n], V_l(s_i, s_k) for k > i, zero elsewhere
    std::vector<double> vs;  // [n], V_L(s_k)
    std::vector<double> r;   // [n], r(s_k)
    // level terms sqrt(C_l V_l): w[i][k] = sqrt((r_i + r_k) vp[i][k]), u[k] = sqrt(r_k vs[k])
    std::vector<double> w, u;
};

std::vector<double> paper_eval_grid(const double* s_hat, int m);
ShiftTables shift_tables(const fs_shift_model& mdl);
// Least sum of level terms over 0 = j_0 < j_1 < ... < j_L <= n-1; idx[0..L].
double shift_select_dp(const ShiftTables& t, int L, int* idx);

// Exhaustive sweep on the GPU.  w: [n][n], u: [n], binom: [(kSweepMaxN+1)][kSweepMaxL+1].
// Per workgroup b: least cost pc[b] and its key pk[b] = prefix_rank * 128 + j_L.
void launch_shift_sweep(int L, const double* w, const double* u, const uint64_t* binom, int n, uint64_t n_prefix,
                        uint64_t per_thread, int grid, double* pc, uint64_t* pk, hipStream_t s);
// Reduces nb per-workgroup results to out_c[0], out_k[0] (ties: smaller key).
void launch_sweep_reduce(const double* pc, const uint64_t* pk, int nb, double* out_c, uint64_t* out_k,
                         hipStream_t s);

}  // namespace fs
