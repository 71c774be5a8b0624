// Host-visible launchers of the FS-MLMC HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fs_device.h"

namespace fs {

// Per-system solver state (device).  Codes of `state`:
enum SysCode : int {
    S_RUN = 0,     // iterating
    S_REL = 1,     // reliable update due (residual fell by delta)
    S_CHK = 2,     // iterated residual below tol: verify in FP64
    S_DONE = 3,    // converged (FP64 true residual <= tol)
    S_BRK = 4,     // breakdown: restart from the FP64 residual
    S_MAXIT = 5,   // iteration limit: fold x and measure the true residual
    S_CONV = 8,    // transient: copy FP64 residual to the Krylov residual, resume
    S_RST = 9,     // transient: as S_CONV and restart the Krylov space
    S_FAIL = 10,   // gave up (max_iter); x holds the last iterate
    S_IDLE = 11    // padding slot of a partially filled block (never runs)
};

struct SysState {
    double rho[2], alpha[2], omega[2], beta[2];
    double rr, bb, rr_max, rr_true;
    double tol2;      // tol^2 (relative)
    double delta2;    // reliable-update trigger (0 = only at convergence)
    double rhat2;     // |rhat|^2 (breakdown test)
    double bnorm2;    // even-odd: |b|^2 of the full system (0 otherwise); the tolerance is relative to it
    int state, iters, upd_p, n_rel;
    int restarts, max_iter;
    int upd_x;        // the system iterated: the vector update applies to its x and r
    int pad_;
};

// One batched launch: a set of blocks of NR systems on possibly different lattices.
struct Work {
    const LatDesc* lats;      // device table (gauge pointer in the launch precision)
    const BlockDesc* blocks;  // device table
    const int* wg_start;      // device [nblk+1], first workgroup of each block
    int nblk;
    int total_wg;
    int tpw;                  // tiles (of wg threads) per workgroup
    int wg;                   // threads per workgroup
    int nr, lognr;            // systems per block
    const int* blk_on;        // device [nblk]: 0 => workgroups of the block exit (may be null)
    int tc;                   // stencil launches: t-slices per workgroup column (0 = tile mapping)
    int ilp;                  // stencil variant: 0 default, 1 register-rich (one wave per SIMD), 2 LDS tiles
    int tl[3];                // stencil variant 2: log2 of the tile extent in x, y, z
    int occ;                  // stencil: cap on resident waves per SIMD (0 = none)
    int two_rows;             // FP32 gauge_q of every lattice holds rows 0-1 only
    int prow;                 // finish stages: partial-sum rows per workgroup of the mapping (<= 1: one)
    // Persistent launches: when vlist is set, a fixed grid walks the virtual
    // workgroups of the blocks listed there (vlist[0..*vcount)), vstart being
    // their prefix sums in this launch's mapping (tile or stencil table).
    const int* vlist;
    const int* vstart;
    const int* vcount;
};

// Device-side list of active blocks with virtual-workgroup prefix sums for
// both mappings (built by launch_vlist from a block flag array).
struct VList {
    int* list = nullptr;         // [nblk]
    int* vstart_tile = nullptr;  // [nblk + 1]
    int* vstart_sten = nullptr;  // [nblk + 1]
    int* count = nullptr;        // [1]
};

// Walk the virtual workgroups of a launch: body(wg_id, b) once per workgroup
// of every listed block (or of every block with its flag set when the launch
// has no list).  Each XCD walks a contiguous range of virtual workgroups.
template <typename F>
__device__ __forceinline__ void for_each_vwg(const Work& w, F&& body) {
    // The block and workgroup indices are uniform over the workgroup; saying
    // so (readfirstlane) lets the block and lattice descriptors and the buffer
    // resources built from them live in scalar registers.
    if (!w.vlist) {
        const int wg_id = xcd_remap(blockIdx.x, gridDim.x);
        if (wg_id >= w.total_wg) return;
        const int b = __builtin_amdgcn_readfirstlane(find_block(w.wg_start, w.nblk, wg_id));
        if (w.blk_on && !w.blk_on[b]) return;
        body(wg_id, b);
        return;
    }
    const int n = *w.vcount;
    if (n <= 0) return;
    const int T = w.vstart[n];
    const int nx = 8;
    const int xcd = (int)(blockIdx.x % nx), slot = (int)(blockIdx.x / nx), nper = (int)(gridDim.x / nx);
    const int lo = (int)((long long)T * xcd / nx), hi = (int)((long long)T * (xcd + 1) / nx);
    for (int v = lo + slot; v < hi; v += nper) {
        const int k = __builtin_amdgcn_readfirstlane(find_block(w.vstart, n, v));
        const int b = __builtin_amdgcn_readfirstlane(w.vlist[k]);
        body(__builtin_amdgcn_readfirstlane(w.wg_start[b] + (v - w.vstart[k])), b);
    }
}


// Common prologue: for every virtual workgroup of this launch, bind the block
// and its geometry; the body runs once per virtual workgroup (FS_WG_EPILOGUE
// closes it).
#define FS_WG_PROLOGUE(w)                                                   \
    for_each_vwg((w), [&](const int wg_id, const int b) {                   \
    (void)b;                                                                \
    const BlockDesc bd = (w).blocks[b];                                     \
    const LatDesc ld = (w).lats[bd.lat];                                    \
    const int wgb = wg_id - (w).wg_start[b];                                \
    const size_t gs = (size_t)ld.Vf << (w).lognr;

#define FS_WG_EPILOGUE });

#define FS_SLOT_LOOP(w)                                                     \
    for (int it = 0; it < (w).tpw; ++it) {                                  \
        const size_t slot = ((size_t)wgb * (w).tpw + it) * (w).wg + threadIdx.x; \
        if (slot >= gs) break;                                              \
        const int rhs = (int)(slot & (size_t)((w).nr - 1));                 \
        const int sys = bd.sys0 + rhs;

#define FS_SLOT_LOOP_END }

struct Fld {
    uint4* v = nullptr;    // block-layout field (16-byte groups)
    float* n = nullptr;    // FP16 scales (per slot) or null
};

// Clover term of the even-odd operator.  Per site the term is two Hermitian
// 6 x 6 blocks (spins 0-1 and 2-3, index spin * 3 + colour within the block),
// each packed as 36 reals: the 6 diagonal entries, then the 15 entries above
// the diagonal row by row as (re, im).  A field of such sites is stored
// [chunk][half-lattice site] in 16-byte chunks: 36 chunks per site in FP64, 18
// in FP32.  `inv` holds, per (lattice, shift), the inverses of C + 4 + m0 +
// sigma at the odd sites; off[sys] is the chunk offset of system sys's field.
constexpr int CLV_REALS = 72;  // two packed blocks
struct Clv {
    const uint4* inv = nullptr;
    const long long* off = nullptr;
};

// Z4 noise.  Block layout (FP64) for systems with noise keys, or canonical.
// The same keys generate the BiCGStab shadow residual rhat on the fly.
struct NoiseKey {
    uint64_t seed;
    uint32_t instance, level;
    uint64_t sample;
    int g5;        // apply gamma_5 to the vector
    int pad;       // padding system: the zero vector
    int dil;       // 0: the whole Z4 vector; 1 + 12 j + a: only the sites of probing colour j,
                   // only spin-colour component a (spin a / 3, colour a % 3)
    int resv;
};

// The 12 components of `site` for key k: z_c = i^code(c), optionally times g5
// (spins 2, 3 negated).  Component c = site*12 + j draws 2 bits of Philox block
// c/128 (counter (c/128, sample, level, instance), key (seed, 0)).
__device__ __forceinline__ void z4_site(const NoiseKey& k, long long site, double v[24]) {
    const long long c0 = site * 12;
    const long long b0 = c0 >> 7, b1 = (c0 + 11) >> 7;
    U64x4 o0 = philox4x64_10((uint64_t)b0, k.sample, k.level, k.instance, k.seed, 0ull);
    U64x4 o1 = o0;
    if (b1 != b0) o1 = philox4x64_10((uint64_t)b1, k.sample, k.level, k.instance, k.seed, 0ull);
#pragma unroll
    for (int j = 0; j < 12; ++j) {
        const long long c = c0 + j;
        const int e = (int)(c & 127);
        // value selects (an indexed or address-taken array would live in private memory)
        const bool first = (c >> 7) == b0;
        const int wi = e >> 5;
        const uint64_t w01 = wi == 0 ? (first ? o0.v[0] : o1.v[0]) : (first ? o0.v[1] : o1.v[1]);
        const uint64_t w23 = wi == 2 ? (first ? o0.v[2] : o1.v[2]) : (first ? o0.v[3] : o1.v[3]);
        const uint64_t word = wi < 2 ? w01 : w23;
        const int code = (int)((word >> (2 * (e & 31))) & 3ull);
        double re = code == 0 ? 1.0 : code == 2 ? -1.0 : 0.0;
        double im = code == 1 ? 1.0 : code == 3 ? -1.0 : 0.0;
        if (k.g5 && j >= 6) {
            re = -re;
            im = -im;
        }
        v[2 * j] = re;
        v[2 * j + 1] = im;
    }
}

// BiCGStab shadow residual of a system: its Z4 source stream (rhat = r0 = b
// for estimator systems, x0 = 0); after the n-th breakdown restart a fresh Z4
// stream (instance bit 31 set, level + n).  Padding systems: zero.
//
// The solver keeps rhat as one 32-bit code word per slot: bits 2j, 2j + 1 hold
// k_j of component j (rhat_j = i^k_j, the key's gamma_5 folded in as k_j + 2),
// bit 31 marks the zero vector.  rhat_code forms the word of one site from the
// Philox words of z4_site (same components, same values).
__device__ __forceinline__ uint32_t rhat_code(const NoiseKey& k0, int restarts, long long site) {
    if (k0.pad) return 0x80000000u;
    NoiseKey k = k0;
    if (restarts > 0) {
        k.instance ^= 0x80000000u;
        k.level += (uint32_t)restarts;
    }
    const long long c0 = site * 12;
    const long long b0 = c0 >> 7, b1 = (c0 + 11) >> 7;
    U64x4 o0 = philox4x64_10((uint64_t)b0, k.sample, k.level, k.instance, k.seed, 0ull);
    U64x4 o1 = o0;
    if (b1 != b0) o1 = philox4x64_10((uint64_t)b1, k.sample, k.level, k.instance, k.seed, 0ull);
    uint32_t word = 0;
#pragma unroll
    for (int j = 0; j < 12; ++j) {
        const long long c = c0 + j;
        const int e = (int)(c & 127);
        const bool first = (c >> 7) == b0;
        const int wi = e >> 5;
        const uint64_t w01 = wi == 0 ? (first ? o0.v[0] : o1.v[0]) : (first ? o0.v[1] : o1.v[1]);
        const uint64_t w23 = wi == 2 ? (first ? o0.v[2] : o1.v[2]) : (first ? o0.v[3] : o1.v[3]);
        uint32_t code = (uint32_t)(((wi < 2 ? w01 : w23) >> (2 * (e & 31))) & 3ull);
        if (k.g5 && j >= 6) code = (code + 2u) & 3u;
        word |= code << (2 * j);
    }
    return word;
}

// sum_j conj(rhat_j) v_j and sum_j conj(rhat_j) w_j over the 12 components of
// one site (NW = 1: v only), rhat given by its code word.  conj(i^k) v is v
// with its parts swapped and negated (k = 1: (vi, -vr); 2: -v; 3: (-vi, vr)),
// so no complex product is formed.  The 12 terms are summed in A, then added
// to the FP64 sums.  The zero vector adds nothing.
template <int NW, typename A>
__device__ __forceinline__ void rhat_code_dots(uint32_t code, const A v[24], const A w[24], double acc_v[2],
                                               double acc_w[2]) {
    if (code >> 31) return;
    A fv0 = A(0), fv1 = A(0), fw0 = A(0), fw1 = A(0);
#pragma unroll
    for (int j = 0; j < 12; ++j) {
        const uint32_t k = (code >> (2 * j)) & 3u;
        const bool sw = k & 1u;                 // parts swapped (odd powers)
        const bool nre = k & 2u;                // new real part negated (k = 2, 3)
        const bool nim = (k ^ (k >> 1)) & 1u;   // new imaginary part negated (k = 1, 2)
        {
            const A re = sw ? v[2 * j + 1] : v[2 * j], im = sw ? v[2 * j] : v[2 * j + 1];
            fv0 += nre ? -re : re;
            fv1 += nim ? -im : im;
        }
        if constexpr (NW == 2) {
            const A re = sw ? w[2 * j + 1] : w[2 * j], im = sw ? w[2 * j] : w[2 * j + 1];
            fw0 += nre ? -re : re;
            fw1 += nim ? -im : im;
        }
    }
    acc_v[0] += (double)fv0;
    acc_v[1] += (double)fv1;
    if constexpr (NW == 2) {
        acc_w[0] += (double)fw0;
        acc_w[1] += (double)fw1;
    }
}
enum Mask : int { M_ALL = 0, M_RUN = 1, M_PEND = 2, M_CONVERT = 3, M_UPDP = 4 };

// dslash modes
enum DMode : int {
    D_PLAIN = 0,   // out = (D + sigma) in
    D_RHAT = 1,    // + partial (rhat, out)             [2 doubles]
    D_TS = 2,      // + partials (out, in), (out, out), (in, in), (rhat, in), (rhat, out)  [8 doubles]
    D_RESID = 3,   // out = b - (D + sigma) in (b FP64 in aux) + |out|^2 [1 double]
    D_HOP = 4,     // even-odd only: out = D_{par_out, other} in, the off-diagonal block
    D_PREP = 5,    // even-odd, FP64: out_e = b_e - D_eo b_o / a from b in full layout, + |b|^2
    D_POST = 6     // even-odd, FP64: x (full layout) = (x_e, (b_o - D_oe x_e) / a)
};

// Even-odd preconditioning.  Fields hold one parity (field site = site >> 1 with
// Lx even).  With a = 4 + m0 + sigma, D = [[a, D_eo], [D_oe, a]] and the Schur
// operator on even sites is S = a - D_eo D_oe / a.  launch_dslash_eo:
//   D_HOP:    out = D_{par_out, 1-par_out} in
//   other modes (par_out = even): out = a cen - D_eo in / a with in = D_oe cen,
//   and the partial sums of launch_dslash (D_RESID: out = b - S cen, b in aux;
//   D_RHAT and D_TS: rhat from rc).
// With the stencil mapping of a one-parity plan (w.tc > 0) the kernel streams
// over t; with the tile mapping it takes one slot per lane.  The finish that
// follows takes the same mapping.
void launch_dslash_eo(int prec, int mode, const Work& w, Fld out, Fld in, Fld cen, Fld aux, const double* diag,
                      const SysState* st, int mask, double* part, hipStream_t s, const uint32_t* rc, int par_out);
// Over a one-parity plan whose blocks match fblocks (full-lattice layout) one
// for one, FP64: bh = b_e - D_eo b_o / a, plus partial |b|^2 of both parities
// (finished by F_BNORM); and x = (x_e, (b_o - D_oe x_e) / a) in full layout.
void launch_eo_prep(const Work& wh, const BlockDesc* fblocks, Fld bfull, Fld bh, const double* diag, double* part,
                    hipStream_t s);
void launch_eo_post(const Work& wh, const BlockDesc* fblocks, Fld bfull, Fld xh, Fld xfull, const double* diag,
                    hipStream_t s);

// D_RHAT and D_TS take the shadow residual from rc (one rhat_code word per slot
// of the plan's fields); D_RESID reads b from aux.
void launch_dslash(int prec, int mode, const Work& w, Fld out, Fld in, Fld aux, const double* diag,
                   const SysState* st, int mask, double* part, hipStream_t s, const uint32_t* rc = nullptr);

// BiCGStab vector kernels (precision of the Krylov fields)
void launch_axpy_s(int prec, const Work& w, Fld r, Fld v, const SysState* st, hipStream_t s);
// x += alpha p + omega s, r = s - omega t for the systems that iterated (s held
// in r), then p = r + beta (p - omega v) for those that continue
// Multi-shift BiCGStab: the systems (A + d_k) x_k = b, k < nm, carried along the
// base system A x = b of each (system) slot without operator applications of
// their own.  Per (system, member): the recurrence state and this iteration's
// update coefficients (complex, (re, im)).
constexpr int MS_MAX = 16;
struct MsState {
    double zp[2], z[2], tau[2], ap[2], bp[2];  // zeta_{n-1}, zeta_n, tau_n, alpha_{n-1}, beta_{n-1}
    int done, iters;                           // iters: Krylov steps the member took
};
struct MsCoef {
    double cxp[2], cxs[2];                     // x += cxp p + cxs s
    double cpp[2], cps[2], cpv[2], cpt[2];     // p = cpp p + cps s + cpv v + cpt t
    int on, pad_;
};
struct MsFields {
    uint4* x[MS_MAX];
    uint4* p[MS_MAX];
};
// After the F_OMEGA finish: the members' scalars from the base's alpha, omega,
// beta (systems that iterated, before any reliable update or restart); a member
// stops once |zeta/tau| |r| <= tol |b| / 2 (its residual estimate, with a margin).
void launch_ms_scalars(int nsys, int nm, const double* d, const SysState* st, MsState* ms, MsCoef* co,
                       hipStream_t s);
// Before the base's vector update (s held in r): every active member's x and p (FP64).
void launch_ms_update(const Work& w, int nm, Fld s_, Fld v, Fld t, const MsFields& f, const MsCoef* co,
                      hipStream_t s);
void launch_update_xrp(int prec, const Work& w, Fld x, Fld p, Fld r, Fld t, Fld v, const SysState* st,
                       hipStream_t s);

// finish kernels: one workgroup per block, reduce partials, update state
enum FStage : int { F_INIT = 0, F_ALPHA = 1, F_OMEGA = 2, F_TRUE = 4, F_RESUME = 5, F_BNORM = 6 };
// w.blk_on: flags of the launch being completed (blocks with 0 are skipped);
// out: flags for the next launch; out2 (F_OMEGA only): blocks with systems
// pending a reliable update.
void launch_finish(int stage, const Work& w, SysState* st, const double* part, int* out, int* out2, hipStream_t s);

// reliable update / init
void launch_fold(int prec, const Work& w, Fld xhi, Fld xlo, const SysState* st, hipStream_t s);
// rc: the shadow residual's code words (one per slot).  launch_init writes
// them from rk (restart count 0); launch_convert rewrites those of restarting
// systems (their restart count) and reads the others.
void launch_convert(int prec, const Work& w, Fld rhi, Fld r, const NoiseKey* rk, uint32_t* rc, Fld p,
                    const SysState* st, double* part, hipStream_t s);
void launch_init(int prec, const Work& w, Fld b, Fld xhi, Fld xlo, Fld rhi, Fld r, const NoiseKey* rk, uint32_t* rc,
                 Fld p, double* part, hipStream_t s);
// rc = the code words of rk's shadow residuals (restart count 0) over plan w.
void launch_rhat_codes(const Work& w, const NoiseKey* rk, uint32_t* rc, hipStream_t s);

// layout conversion between canonical complex128 [sys][site][spin][col] and block layout;
// sys_map[sys] = canonical index, -1 = write zeros (pack) / skip (unpack), < -1 = skip
void launch_pack(int prec, const Work& w, Fld dst, const double* src, long long sys_stride,
                 const int* sys_map, hipStream_t s);
void launch_unpack(int prec, const Work& w, double* dst, Fld src, long long sys_stride,
                   const int* sys_map, hipStream_t s);

// gauge: canonical complex128 [mu][site][3][3] -> [mu][9][site] in precision prec
void launch_gauge_convert(int prec, void* dst, const double* src, int V, hipStream_t s);
void launch_gauge_convert_q(int prec, void* dst, const double* src, int V, bool two_rows, hipStream_t s);

// colour: per-site probing colour (only read for diluted keys; may be null otherwise)
void launch_noise_block(int prec, const Work& w, Fld dst, const NoiseKey* keys /* per system */, hipStream_t s,
                        const uint16_t* colour = nullptr);
void launch_noise_canonical(double* dst, int V, NoiseKey key, hipStream_t s);

// Displacement + bilinear (FP64).  For each block b (the "x" block) with
// partner yb[b] (or -1: y is the field `ysrc` of block b itself):
//   phi_out = hop(phi_in) (p > 0) or phi_in (p == 0),  M_ab += conj(y_a) phi_b
void launch_hop_reduce(const Work& w, int p, Fld phi_out, Fld phi_in, Fld yfld, Fld ysrc,
                       const int* yb, double* part, hipStream_t s);
// reduce hop partials to M[sys][16 complex] for one p
void launch_hop_finish(const Work& w, const double* part, double* M, int M_stride, int p, hipStream_t s);

// plain single-lattice displacement (canonical in/out, FP64) used by fs_displace
void launch_displace_canonical(double* out, const double* in, const double* gauge64, LatDesc ld,
                               hipStream_t s);

// Gamma contraction of the spin correlations and per-level statistics.
struct XMap {          // per x-system of a hop launch
    int level;         // -1: not an estimator system
    int sample;
    int g5;            // y carries gamma_5
    int pad;
    double coef;       // sigma_{l+1} - sigma_l, or 1 on the last level
};
struct GammaTab {      // Gamma_n row a: single nonzero i^ph[n][a] at column perm[n][a]
    int8_t perm[16][4];
    int8_t ph[16][4];
};
void launch_gamma_contract(const double* M, int P1, int nsys, const XMap* xm, const GammaTab& gt, double* X,
                           int n_noise, hipStream_t s);
// n_level: NULL or device [L1] sample counts per level (each <= n_noise, the slot stride)
void launch_level_stats(const double* X, int L1, int n_noise, int P1, double* out, hipStream_t s,
                        const int* n_level = nullptr);
// X[g][16][P1] = sum_{d < D} Y[g0[g] + d][16][P1] (complex), summed in order d = 0..D-1
void launch_dilution_sum(const double* Y, int P1, const int* g0, int G, int D, double* X, hipStream_t s);
void launch_blk_mask(const Work& w, const SysState* st, int mask, int* blk_on, hipStream_t s);
// list of blocks with flags[b] != 0; wg_tile / wg_sten: the two workgroup tables of the plan
void launch_vlist(const int* flags, int nblk, const int* wg_tile, const int* wg_sten, VList out, hipStream_t s);
// physical grid of persistent launches
inline int persistent_grid(int wg) { return 2048 * (256 / wg); }

// copy kernel of known size (bandwidth calibration)
void launch_copy(uint4* dst, const uint4* src, size_t n16, hipStream_t s);
// out = coef[sys] * in over the slots of w (FP64 fields)
void launch_scale_sys(const Work& w, Fld out, Fld in, const double* coef, hipStream_t s);

}  // namespace fs
