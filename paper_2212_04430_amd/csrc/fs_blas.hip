// Vector, reduction, noise and displacement kernels of the FS-MLMC hot path.
//
//  * BiCGStab (van der Vorst 1992) updates, one lane per (site, rhs), fused
//    with the dot products each step needs; partial sums are FP64 and reduced
//    in a fixed order, so results are run-to-run reproducible.
//  * Per-system scalar updates and the convergence / reliable-update state
//    machine (one workgroup per block of NR systems).
//  * Z4 noise from Philox4x64-10 (paper Introduction, eq. test: entries in
//    {1,-1,i,-i}), written straight into the solver's block layout.
//  * The Wilson-line displacement Omega_p (Introduction: Omega_p = W Pi_p along
//    z) fused with the 4x4 spin-correlation M_ab = sum_{x,c} conj(y_ac) phi_bc,
//    from which every bilinear y^+ Gamma_n Omega_p x of eq. fs_trace_est is a
//    16-term contraction.
#include <algorithm>

#include "fs_kernels.h"

namespace fs {

namespace {

__device__ __forceinline__ bool mask_ok(int mask, const SysState* __restrict__ st, int sys) {
    if (mask == M_ALL) return true;
    const int s = st[sys].state;
    if (mask == M_RUN) return s == S_RUN;
    if (mask == M_PEND) return s == S_REL || s == S_CHK || s == S_BRK || s == S_MAXIT;
    if (mask == M_CONVERT) return s == S_CONV || s == S_RST;
    return st[sys].upd_p != 0;
}


template <int P>
__device__ __forceinline__ const uint4* fbase(const Fld& f, const BlockDesc& bd) {
    return f.v + (size_t)bd.slot_off * Tr<P>::G;
}
template <int P>
__device__ __forceinline__ uint4* fbase_w(const Fld& f, const BlockDesc& bd) {
    return f.v + (size_t)bd.slot_off * Tr<P>::G;
}
__device__ __forceinline__ float* nbase(const Fld& f, const BlockDesc& bd) {
    return f.n ? f.n + bd.slot_off : nullptr;
}

// ------------------------------------------------------------------ BiCGStab

// s = r - alpha v  (stored in r)
template <int P>
__global__ void __launch_bounds__(256) k_axpy_s(Work w, Fld r, Fld v, const SysState* __restrict__ st) {
    using A = typename Tr<P>::acc;
    FS_WG_PROLOGUE(w)
    uint4* rb = fbase_w<P>(r, bd);
    float* rn = nbase(r, bd);
    const uint4* vb = fbase<P>(v, bd);
    const float* vn = nbase(v, bd);
    FS_SLOT_LOOP(w)
        if (st[sys].state != S_RUN) continue;
        const A ar = (A)st[sys].alpha[0], ai = (A)st[sys].alpha[1];
        A x[24], y[24];
        load_sp<P, A>(rb, rn, gs, slot, x);
        load_sp<P, A>(vb, vn, gs, slot, y);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            x[2 * k] -= ar * y[2 * k] - ai * y[2 * k + 1];
            x[2 * k + 1] -= ar * y[2 * k + 1] + ai * y[2 * k];
        }
        store_sp<P, A>(rb, rn, gs, slot, x);
    FS_SLOT_LOOP_END
    FS_WG_EPILOGUE
}

// The vector update of one BiCGStab iteration, once its last reduction (the
// F_OMEGA finish of the t = A s stencil) is done: for the systems that
// iterated, x += alpha p + omega s and r = s - omega t (s is held in r), and
// for those that continue, p = r + beta (p - omega v).  Five fields in (x, p,
// s, t, v), three out; every field is touched once: non-temporal accesses.
template <int P>
__global__ void __launch_bounds__(256) k_update_xrp(Work w, Fld x, Fld p, Fld r, Fld t, Fld v,
                                                    const SysState* __restrict__ st) {
    using A = typename Tr<P>::acc;
    FS_WG_PROLOGUE(w)
    uint4* xb = fbase_w<P>(x, bd);
    float* xn = nbase(x, bd);
    uint4* rb = fbase_w<P>(r, bd);
    float* rn = nbase(r, bd);
    uint4* pb = fbase_w<P>(p, bd);
    float* pn = nbase(p, bd);
    FS_SLOT_LOOP(w)
        if (!st[sys].upd_x) continue;
        const A ar = (A)st[sys].alpha[0], ai = (A)st[sys].alpha[1];
        const A wr = (A)st[sys].omega[0], wi = (A)st[sys].omega[1];
        A pv[24], sv[24];
        {
            A xv[24];
            load_sp<P, A, true>(xb, xn, gs, slot, xv);
            load_sp<P, A, true>(pb, pn, gs, slot, pv);
            load_sp<P, A, true>(rb, rn, gs, slot, sv);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                xv[2 * k] += ar * pv[2 * k] - ai * pv[2 * k + 1] + wr * sv[2 * k] - wi * sv[2 * k + 1];
                xv[2 * k + 1] += ar * pv[2 * k + 1] + ai * pv[2 * k] + wr * sv[2 * k + 1] + wi * sv[2 * k];
            }
            store_sp<P, A, true>(xb, xn, gs, slot, xv);
        }
        {
            A tv[24];
            load_sp<P, A, true>(fbase<P>(t, bd), nbase(t, bd), gs, slot, tv);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                sv[2 * k] -= wr * tv[2 * k] - wi * tv[2 * k + 1];
                sv[2 * k + 1] -= wr * tv[2 * k + 1] + wi * tv[2 * k];
            }
        }
        round_sp<P, A>(sv);  // the residual as stored, which p is built from
        store_sp<P, A, true>(rb, rn, gs, slot, sv);
        if (st[sys].upd_p) {
            const A br = (A)st[sys].beta[0], bi = (A)st[sys].beta[1];
            A vv[24];
            load_sp<P, A, true>(fbase<P>(v, bd), nbase(v, bd), gs, slot, vv);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                const A qr = pv[2 * k] - (wr * vv[2 * k] - wi * vv[2 * k + 1]);
                const A qi = pv[2 * k + 1] - (wr * vv[2 * k + 1] + wi * vv[2 * k]);
                pv[2 * k] = sv[2 * k] + br * qr - bi * qi;
                pv[2 * k + 1] = sv[2 * k + 1] + br * qi + bi * qr;
            }
            store_sp<P, A, true>(pb, pn, gs, slot, pv);
        }
    FS_SLOT_LOOP_END
    FS_WG_EPILOGUE
}

// ------------------------------------------------ FP32, one thread per group
//
// The element-wise FP32 updates without reductions run one thread per 16-byte
// group of a slot (two complex numbers) instead of one per slot.  The launch
// holds 6 x (tile-mapping workgroups of the plan) x tpw workgroups, ordered
// group-major: while one group of every listed block streams through, all
// resident waves read and write narrow windows of the same few arrays.  With
// a device list (persistent mapping of the other kernels) the workgroups past
// the listed blocks' share exit at once.  Loads and stores are non-temporal:
// each field is touched once per launch.

typedef float f32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4_t ld_nt(const f32x4_t* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void st_nt(f32x4_t v, f32x4_t* p) { __builtin_nontemporal_store(v, p); }

// body(block, group, workgroup in the block, tile in the workgroup, slot) for
// this workgroup's tile, if it has one.  PER_TILE: one workgroup per tile
// (6 x workgroups x tpw); otherwise one per (group, tile-mapping workgroup),
// walking its tpw tiles (6 x workgroups).
template <bool PER_TILE = true, typename F>
__device__ __forceinline__ void for_group_tile(const Work& w, F&& body) {
    constexpr int G = Tr<P32>::G;
    int n = 0, T;
    if (w.vlist) {
        n = *w.vcount;
        if (n <= 0) return;
        T = w.vstart[n];
    } else {
        T = w.total_wg;
    }
    const int tpu = PER_TILE ? w.tpw : 1;  // units per tile-mapping workgroup
    const long long per_g = (long long)T * tpu;
    const long long u = blockIdx.x;
    if (u >= per_g * G) return;
    const int g = (int)(u / per_g);
    const long long rem = u - (long long)g * per_g;
    const int v = (int)(rem / tpu), it0 = (int)(rem - (long long)v * tpu);
    int b, wgb;
    if (w.vlist) {
        const int k = __builtin_amdgcn_readfirstlane(find_block(w.vstart, n, v));
        b = __builtin_amdgcn_readfirstlane(w.vlist[k]);
        wgb = v - w.vstart[k];
    } else {
        b = __builtin_amdgcn_readfirstlane(find_block(w.wg_start, w.nblk, v));
        if (w.blk_on && !w.blk_on[b]) return;
        wgb = v - w.wg_start[b];
    }
    if constexpr (PER_TILE) {
        body(b, g, wgb, it0, ((size_t)wgb * w.tpw + it0) * w.wg + threadIdx.x);
    } else {
        for (int it = 0; it < w.tpw; ++it) body(b, g, wgb, it, ((size_t)wgb * w.tpw + it) * w.wg + threadIdx.x);
    }
}

// s = r - alpha v  (stored in r), FP32 storage
__global__ void __launch_bounds__(256) k_axpy_s_g(Work w, Fld r, Fld v, const SysState* __restrict__ st) {
    for_group_tile(w, [&](const int b, const int g, const int, const int, const size_t slot) {
        const BlockDesc bd = w.blocks[b];
        const size_t gs = (size_t)w.lats[bd.lat].Vf << w.lognr;
        if (slot >= gs) return;
        const int sys = bd.sys0 + (int)(slot & (size_t)(w.nr - 1));
        if (st[sys].state != S_RUN) return;
        const float ar = (float)st[sys].alpha[0], ai = (float)st[sys].alpha[1];
        const size_t e = (size_t)g * gs + slot;
        f32x4_t* rp = reinterpret_cast<f32x4_t*>(fbase_w<P32>(r, bd)) + e;
        const f32x4_t y = ld_nt(reinterpret_cast<const f32x4_t*>(fbase<P32>(v, bd)) + e);
        f32x4_t x = ld_nt(rp);
        x.x -= ar * y.x - ai * y.y;
        x.y -= ar * y.y + ai * y.x;
        x.z -= ar * y.z - ai * y.w;
        x.w -= ar * y.w + ai * y.z;
        st_nt(x, rp);
    });
}

// The fused vector update of k_update_xrp, FP32 storage, one thread per group.
__global__ void __launch_bounds__(256) k_update_xrp_g(Work w, Fld x, Fld p, Fld r, Fld t, Fld v,
                                                      const SysState* __restrict__ st) {
    for_group_tile(w, [&](const int b, const int g, const int, const int, const size_t slot) {
        const BlockDesc bd = w.blocks[b];
        const size_t gs = (size_t)w.lats[bd.lat].Vf << w.lognr;
        if (slot >= gs) return;
        const int sys = bd.sys0 + (int)(slot & (size_t)(w.nr - 1));
        if (!st[sys].upd_x) return;
        const float ar = (float)st[sys].alpha[0], ai = (float)st[sys].alpha[1];
        const float wr = (float)st[sys].omega[0], wi = (float)st[sys].omega[1];
        const size_t e = (size_t)g * gs + slot;
        f32x4_t* xp = reinterpret_cast<f32x4_t*>(fbase_w<P32>(x, bd)) + e;
        f32x4_t* rp = reinterpret_cast<f32x4_t*>(fbase_w<P32>(r, bd)) + e;
        f32x4_t* pp = reinterpret_cast<f32x4_t*>(fbase_w<P32>(p, bd)) + e;
        f32x4_t pv = ld_nt(pp);
        const f32x4_t tv = ld_nt(reinterpret_cast<const f32x4_t*>(fbase<P32>(t, bd)) + e);
        f32x4_t xv = ld_nt(xp), sv = ld_nt(rp);
        xv.x += ar * pv.x - ai * pv.y + wr * sv.x - wi * sv.y;
        xv.y += ar * pv.y + ai * pv.x + wr * sv.y + wi * sv.x;
        xv.z += ar * pv.z - ai * pv.w + wr * sv.z - wi * sv.w;
        xv.w += ar * pv.w + ai * pv.z + wr * sv.w + wi * sv.z;
        st_nt(xv, xp);
        sv.x -= wr * tv.x - wi * tv.y;
        sv.y -= wr * tv.y + wi * tv.x;
        sv.z -= wr * tv.z - wi * tv.w;
        sv.w -= wr * tv.w + wi * tv.z;
        st_nt(sv, rp);
        if (!st[sys].upd_p) return;
        const float br = (float)st[sys].beta[0], bi = (float)st[sys].beta[1];
        const f32x4_t vv = ld_nt(reinterpret_cast<const f32x4_t*>(fbase<P32>(v, bd)) + e);
        const float q0 = pv.x - (wr * vv.x - wi * vv.y), q1 = pv.y - (wr * vv.y + wi * vv.x);
        const float q2 = pv.z - (wr * vv.z - wi * vv.w), q3 = pv.w - (wr * vv.w + wi * vv.z);
        pv.x = sv.x + br * q0 - bi * q1;
        pv.y = sv.y + br * q1 + bi * q0;
        pv.z = sv.z + br * q2 - bi * q3;
        pv.w = sv.w + br * q3 + bi * q2;
        st_nt(pv, pp);
    });
}

// x_hi += x_lo; x_lo = 0  (systems pending a reliable update)
template <int P>
__global__ void __launch_bounds__(256) k_fold(Work w, Fld xhi, Fld xlo, const SysState* __restrict__ st) {
    using A = typename Tr<P>::acc;
    FS_WG_PROLOGUE(w)
    uint4* hb = xhi.v + (size_t)bd.slot_off * 12;
    uint4* lb = fbase_w<P>(xlo, bd);
    float* ln = nbase(xlo, bd);
    FS_SLOT_LOOP(w)
        if (!mask_ok(M_PEND, st, sys)) continue;
        double h[24];
        A l[24];
        load_sp<P64, double>(hb, nullptr, gs, slot, h);
        load_sp<P, A>(lb, ln, gs, slot, l);
#pragma unroll
        for (int k = 0; k < 24; ++k) {
            h[k] += (double)l[k];
            l[k] = A(0);
        }
        store_sp<P64, double>(hb, nullptr, gs, slot, h);
        store_sp<P, A>(lb, ln, gs, slot, l);
    FS_SLOT_LOOP_END
    FS_WG_EPILOGUE
}

// r = round(r_hi); restart systems also set p = r and write the code words of
// their fresh shadow residual.  Partials (rhat, r), |r|^2
template <int P>
__global__ void __launch_bounds__(256) k_convert(Work w, Fld rhi, Fld r, const NoiseKey* __restrict__ rk,
                                                 uint32_t* __restrict__ rc, Fld p, const SysState* __restrict__ st,
                                                 double* __restrict__ part) {
    using A = typename Tr<P>::acc;
    FS_WG_PROLOGUE(w)
    double acc[3] = {0.0, 0.0, 0.0};
    const uint4* hb = rhi.v + (size_t)bd.slot_off * 12;
    uint4* rb = fbase_w<P>(r, bd);
    float* rn = nbase(r, bd);
    FS_SLOT_LOOP(w)
        const int s = st[sys].state;
        if (s != S_CONV && s != S_RST) continue;
        double h[24];
        A q[24];
        load_sp<P64, double>(hb, nullptr, gs, slot, h);
#pragma unroll
        for (int k = 0; k < 24; ++k) q[k] = (A)h[k];
        store_sp<P, A>(rb, rn, gs, slot, q);
        if (s == S_RST) store_sp<P, A>(fbase_w<P>(p, bd), nbase(p, bd), gs, slot, q);
        round_sp<P, A>(q);  // the stored value the iteration will see
        uint32_t code;
        if (s == S_RST) {
            code = rhat_code(rk[sys], st[sys].restarts, (long long)(slot >> w.lognr));
            rc[bd.slot_off + slot] = code;
        } else {
            code = rc[bd.slot_off + slot];
        }
        rhat_code_dots<1, A>(code, q, q, acc, acc);
#pragma unroll
        for (int k = 0; k < 24; ++k) acc[2] += (double)q[k] * (double)q[k];
    FS_SLOT_LOOP_END
    block_partials<3, 4>(acc, w.nr, part, wg_id);
    FS_WG_EPILOGUE
}

// The shadow residual's code words of every slot of the plan (restart count 0).
__global__ void __launch_bounds__(256) k_rhat_codes(Work w, const NoiseKey* __restrict__ rk,
                                                    uint32_t* __restrict__ rc) {
    FS_WG_PROLOGUE(w)
    FS_SLOT_LOOP(w)
        rc[bd.slot_off + slot] = rhat_code(rk[sys], 0, (long long)(slot >> w.lognr));
    FS_SLOT_LOOP_END
    FS_WG_EPILOGUE
}

// x_hi = x_lo = 0, r_hi = b, r = p = round(b), the shadow residual's code
// words.  Partials |b|^2, (rhat, r), |r|^2
template <int P>
__global__ void __launch_bounds__(256) k_init(Work w, Fld bf, Fld xhi, Fld xlo, Fld rhi, Fld r,
                                              const NoiseKey* __restrict__ rk, uint32_t* __restrict__ rc, Fld p,
                                              double* __restrict__ part) {
    using A = typename Tr<P>::acc;
    FS_WG_PROLOGUE(w)
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const uint4* bb = bf.v + (size_t)bd.slot_off * 12;
    FS_SLOT_LOOP(w)
        double h[24], z[24];
        A q[24];
        load_sp<P64, double>(bb, nullptr, gs, slot, h);
#pragma unroll
        for (int k = 0; k < 24; ++k) {
            z[k] = 0.0;
            q[k] = (A)h[k];
            acc[0] += h[k] * h[k];
        }
        store_sp<P64, double>(xhi.v + (size_t)bd.slot_off * 12, nullptr, gs, slot, z);
        store_sp<P64, double>(rhi.v + (size_t)bd.slot_off * 12, nullptr, gs, slot, h);
        A zl[24];
#pragma unroll
        for (int k = 0; k < 24; ++k) zl[k] = A(0);
        store_sp<P, A>(fbase_w<P>(xlo, bd), nbase(xlo, bd), gs, slot, zl);
        store_sp<P, A>(fbase_w<P>(r, bd), nbase(r, bd), gs, slot, q);
        store_sp<P, A>(fbase_w<P>(p, bd), nbase(p, bd), gs, slot, q);
        round_sp<P, A>(q);  // the stored value
        const uint32_t code = rhat_code(rk[sys], 0, (long long)(slot >> w.lognr));
        rc[bd.slot_off + slot] = code;
        rhat_code_dots<1, A>(code, q, q, acc + 1, acc + 1);
#pragma unroll
        for (int k = 0; k < 24; ++k) acc[3] += (double)q[k] * (double)q[k];
    FS_SLOT_LOOP_END
    block_partials<4, 4>(acc, w.nr, part, wg_id);
    FS_WG_EPILOGUE
}

// ------------------------------------------------------------------ finish

__device__ __forceinline__ bool finite_d(double x) { return x == x && fabs(x) <= 1.7976931348623157e308; }

// Per-system scalar update after a reduction; one thread per system of the block.
template <int STAGE>
__device__ __forceinline__ void finish_system(SysState& S, const double* q, int nr, int r, double V) {
    auto Q = [&](int k) { return q[k * nr + r]; };
    if constexpr (STAGE == F_INIT) {
        if (S.state != S_IDLE) {
            S.bb = Q(0);
            S.rho[0] = Q(1);
            S.rho[1] = Q(2);
            S.rr = Q(3);
            S.rr_max = S.rr;
            S.rhat2 = 12.0 * V;  // |rhat|^2 of a Z4 vector
            S.rr_true = S.bb;
            // even-odd: the Schur residual equals the full residual, so measure it
            // against the full source
            if (S.bnorm2 > 0.0 && S.bb > 0.0) S.tol2 *= S.bnorm2 / S.bb;
            S.iters = 0;
            S.n_rel = 0;
            S.restarts = 0;
            S.upd_p = 0;
            S.alpha[0] = S.omega[0] = 1.0;
            S.alpha[1] = S.omega[1] = 0.0;
            S.beta[0] = S.beta[1] = 0.0;
            S.state = (S.bb == 0.0) ? S_DONE : S_RUN;
        }
    } else if constexpr (STAGE == F_ALPHA) {
        if (S.state == S_RUN) {
            const double vr = Q(0), vi = Q(1);
            const double d = vr * vr + vi * vi;
            const double rho2 = S.rho[0] * S.rho[0] + S.rho[1] * S.rho[1];
            if (!(d > 0.0) || !finite_d(d) || rho2 <= 1e-28 * S.rhat2 * S.rr) {
                // (rhat, v) = 0 or (rhat, r) = 0: the Lanczos recurrence breaks down
                S.state = S_BRK;
            } else {
                // alpha = rho / (rhat, v)
                S.alpha[0] = (S.rho[0] * vr + S.rho[1] * vi) / d;
                S.alpha[1] = (S.rho[1] * vr - S.rho[0] * vi) / d;
            }
        }
    } else if constexpr (STAGE == F_OMEGA) {
        // t = A s is done: omega = (t, s) / (t, t), and for r = s - omega t
        // rho_new = (rhat, r) = (rhat, s) - omega (rhat, t) and
        // |r|^2 = |s|^2 - |(t, s)|^2 / (t, t), all from the stencil's partial sums
        // (a |r|^2 lost to cancellation can only ask early for the FP64 check);
        // then the state, and beta = (rho_new / rho) (alpha / omega)
        S.upd_x = 0;
        S.upd_p = 0;
        if (S.state == S_RUN) {
            const double tsr = Q(0), tsi = Q(1), tt = Q(2), ss = Q(3);
            const double hsr = Q(4), hsi = Q(5), htr = Q(6), hti = Q(7);
            if (!finite_d(tt) || !finite_d(tsr) || !finite_d(tsi) || !finite_d(ss) || !finite_d(hsr) ||
                !finite_d(hsi) || !finite_d(htr) || !finite_d(hti)) {
                S.state = S_BRK;
            } else {
                if (tt > 0.0) {
                    S.omega[0] = tsr / tt;
                    S.omega[1] = tsi / tt;
                } else {
                    S.omega[0] = S.omega[1] = 0.0;
                }
                const double wr = S.omega[0], wi = S.omega[1];
                const double nr_ = hsr - (wr * htr - wi * hti), ni = hsi - (wr * hti + wi * htr);
                const double rr = std::max(0.0, tt > 0.0 ? ss - (tsr * tsr + tsi * tsi) / tt : ss);
                S.upd_x = 1;
                S.iters += 1;
                S.rr = rr;
                const double om2 = wr * wr + wi * wi;
                const double rho2 = S.rho[0] * S.rho[0] + S.rho[1] * S.rho[1];
                int ns = S_RUN;
                if (rr <= S.tol2 * S.bb) ns = S_CHK;
                else if (S.delta2 > 0.0 && rr < S.delta2 * S.rr_max) ns = S_REL;
                else if (S.iters >= S.max_iter) ns = S_MAXIT;
                const double nn2 = nr_ * nr_ + ni * ni;
                if (om2 > 0.0 && rho2 > 0.0) {
                    const double ar = (nr_ * S.rho[0] + ni * S.rho[1]) / rho2;
                    const double ai = (ni * S.rho[0] - nr_ * S.rho[1]) / rho2;
                    const double cr = (S.alpha[0] * wr + S.alpha[1] * wi) / om2;
                    const double ci = (S.alpha[1] * wr - S.alpha[0] * wi) / om2;
                    S.beta[0] = ar * cr - ai * ci;
                    S.beta[1] = ar * ci + ai * cr;
                    S.upd_p = 1;
                } else if (ns == S_RUN) {
                    ns = S_BRK;
                }
                if (ns == S_RUN && nn2 <= 1e-28 * rr * S.rhat2) ns = S_BRK;  // rho ~ 0
                S.rho[0] = nr_;
                S.rho[1] = ni;
                if (ns == S_BRK) S.upd_p = 0;
                if (rr > S.rr_max) S.rr_max = rr;
                S.state = ns;
            }
        }
    } else if constexpr (STAGE == F_TRUE) {
        const int s = S.state;
        if (s == S_REL || s == S_CHK || s == S_BRK || s == S_MAXIT) {
            S.rr_true = Q(0);
            S.n_rel += 1;
            if (S.rr_true <= S.tol2 * S.bb) S.state = S_DONE;
            else if (s == S_MAXIT || !finite_d(S.rr_true)) S.state = S_FAIL;
            else if (s == S_BRK) {
                S.restarts += 1;
                S.state = S.restarts > 64 ? S_FAIL : S_RST;
            } else S.state = S_CONV;
        }
    } else if constexpr (STAGE == F_BNORM) {
        if (S.state != S_IDLE) S.bnorm2 = Q(0);
    } else {  // F_RESUME
        const int s = S.state;
        if (s == S_CONV || s == S_RST) {
            S.rho[0] = Q(0);
            S.rho[1] = Q(1);
            S.rr = Q(2);
            S.rr_max = S.rr;
            S.state = S_RUN;
        }
    }
}

// One workgroup per block: reduce the partial sums of the launch it completes
// (fixed order), update the per-system scalars and state, and write the block
// flags of the next launches.  blk_on (out): blocks that have work in the
// next kernels (F_OMEGA: the vector update; F_TRUE: blocks to convert);
// blk_pend (out2): after F_OMEGA, blocks with systems that need an FP64
// reliable update (the other stages write 0 there, clearing the flags they
// consumed).
template <int STAGE>
__global__ void __launch_bounds__(256) k_finish(Work w, SysState* __restrict__ st, const double* __restrict__ part,
                                                int* __restrict__ blk_on, int* __restrict__ blk_pend) {
    constexpr int ND = STAGE == F_INIT ? 4 : STAGE == F_ALPHA ? 2 : STAGE == F_OMEGA ? 8
                     : (STAGE == F_TRUE || STAGE == F_BNORM) ? 1 : 3;
    __shared__ double q[ND * 16];
    __shared__ int any_on, any_rel, any_pend;
    const int nr = w.nr;
    // blocks of the launch being completed: its list (persistent launches), or
    // one workgroup per block skipping those whose launch was skipped
    const int nlist = w.vlist ? *w.vcount : 1;
    for (int kk = w.vlist ? (int)blockIdx.x : 0; kk < nlist; kk += w.vlist ? (int)gridDim.x : 1) {
    const int b = w.vlist ? w.vlist[kk] : (int)blockIdx.x;
    const BlockDesc bd = w.blocks[b];
    if (!w.vlist && w.blk_on && !w.blk_on[b] && STAGE != F_INIT) return;
    const int M = w.prow > 1 ? w.prow : 1;  // partial rows per workgroup of the mapping
    reduce_rows(part, ND * nr, w.wg_start[b] * M, w.wg_start[b + 1] * M, q);
    if (threadIdx.x == 0) {
        any_on = 0;
        any_rel = 0;
        any_pend = 0;
    }
    __syncthreads();
    const bool mine = threadIdx.x < nr;
    if (mine) {
        SysState& S = st[bd.sys0 + threadIdx.x];
        finish_system<STAGE>(S, q, nr, threadIdx.x, (double)w.lats[bd.lat].Vf);
        if (STAGE == F_OMEGA && S.state == S_REL) atomicOr(&any_rel, 1);
    }
    __syncthreads();
    if (mine) {
        SysState& S = st[bd.sys0 + threadIdx.x];
        // Reliable updates are taken block by block: when one system of the
        // block asks for one, every running system of the block joins it, so
        // the FP64 stencil of the update does useful work on all its lanes.
        if (STAGE == F_OMEGA && any_rel && S.state == S_RUN) S.state = S_REL;
        bool on;
        if (STAGE == F_OMEGA) on = S.upd_x;
        else if (STAGE == F_TRUE) on = S.state == S_CONV || S.state == S_RST;
        else on = S.state == S_RUN;
        const bool pend = STAGE == F_OMEGA &&
                          (S.state == S_REL || S.state == S_CHK || S.state == S_BRK || S.state == S_MAXIT);
        if (on) atomicOr(&any_on, 1);
        if (pend) atomicOr(&any_pend, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (blk_on) blk_on[b] = any_on;
        if (blk_pend) blk_pend[b] = any_pend;
    }
    }
}

// Per-block mask "has systems in the given class" (sets blk_on for eager launches).
__global__ void k_blk_mask(Work w, const SysState* __restrict__ st, int mask, int* __restrict__ blk_on) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= w.nblk) return;
    const int s0 = w.blocks[b].sys0;
    int any = 0;
    for (int r = 0; r < w.nr; ++r) any |= mask_ok(mask, st, s0 + r) ? 1 : 0;
    blk_on[b] = any;
}

// Compact the blocks with flags[b] != 0 into a list (block order) with the
// prefix sums of their workgroup counts in both mappings.  One workgroup.
__global__ void __launch_bounds__(256) k_vlist(const int* __restrict__ flags, int nblk, const int* __restrict__ wg_tile,
                                               const int* __restrict__ wg_sten, VList out) {
    __shared__ int sc[256], st[256], ss[256];
    __shared__ int base_n, base_t, base_s;
    if (threadIdx.x == 0) {
        base_n = 0;
        base_t = 0;
        base_s = 0;
    }
    __syncthreads();
    for (int c0 = 0; c0 < nblk; c0 += 256) {
        const int b = c0 + threadIdx.x;
        const int on = (b < nblk && flags[b]) ? 1 : 0;
        const int ct = on ? wg_tile[b + 1] - wg_tile[b] : 0;
        const int cs = on ? wg_sten[b + 1] - wg_sten[b] : 0;
        sc[threadIdx.x] = on;
        st[threadIdx.x] = ct;
        ss[threadIdx.x] = cs;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {  // inclusive scan (Hillis-Steele)
            const int a0 = threadIdx.x >= off ? sc[threadIdx.x - off] : 0;
            const int a1 = threadIdx.x >= off ? st[threadIdx.x - off] : 0;
            const int a2 = threadIdx.x >= off ? ss[threadIdx.x - off] : 0;
            __syncthreads();
            sc[threadIdx.x] += a0;
            st[threadIdx.x] += a1;
            ss[threadIdx.x] += a2;
            __syncthreads();
        }
        if (on) {
            const int k = base_n + sc[threadIdx.x] - 1;
            out.list[k] = b;
            out.vstart_tile[k] = base_t + st[threadIdx.x] - ct;
            out.vstart_sten[k] = base_s + ss[threadIdx.x] - cs;
        }
        __syncthreads();
        if (threadIdx.x == 255) {
            base_n += sc[255];
            base_t += st[255];
            base_s += ss[255];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out.vstart_tile[base_n] = base_t;
        out.vstart_sten[base_n] = base_s;
        *out.count = base_n;
    }
}

// ------------------------------------------------------------------ layout conversion

template <int P>
__global__ void __launch_bounds__(256) k_pack(Work w, Fld dst, const double* __restrict__ src, long long sys_stride,
                                              const int* __restrict__ sys_map) {
    using A = typename Tr<P>::acc;
    FS_WG_PROLOGUE(w)
    FS_SLOT_LOOP(w)
        const int site = (int)(slot >> w.lognr);
        const int ci = sys_map ? sys_map[sys] : sys;
        if (ci < -1) continue;  // leave this system untouched
        A v[24];
        if (ci < 0) {
#pragma unroll
            for (int k = 0; k < 24; ++k) v[k] = A(0);
        } else {
            const double* s = src + (size_t)ci * (size_t)sys_stride + (size_t)site * 24;
#pragma unroll
            for (int k = 0; k < 24; ++k) v[k] = (A)s[k];
        }
        store_sp<P, A>(fbase_w<P>(dst, bd), nbase(dst, bd), gs, slot, v);
    FS_SLOT_LOOP_END
    FS_WG_EPILOGUE
}

template <int P>
__global__ void __launch_bounds__(256) k_unpack(Work w, double* __restrict__ dst, Fld src, long long sys_stride,
                                                const int* __restrict__ sys_map) {
    using A = typename Tr<P>::acc;
    FS_WG_PROLOGUE(w)
    FS_SLOT_LOOP(w)
        const int site = (int)(slot >> w.lognr);
        const int ci = sys_map ? sys_map[sys] : sys;
        if (ci < 0) continue;
        A v[24];
        load_sp<P, A>(fbase<P>(src, bd), nbase(src, bd), gs, slot, v);
        double* d = dst + (size_t)ci * (size_t)sys_stride + (size_t)site * 24;
#pragma unroll
        for (int k = 0; k < 24; ++k) d[k] = (double)v[k];
    FS_SLOT_LOOP_END
    FS_WG_EPILOGUE
}

template <int P>
__global__ void k_gauge_convert(void* __restrict__ dst, const double* __restrict__ src, int V) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)4 * V) return;
    const int mu = (int)(i / V);
    const int site = (int)(i % V);
    const double* s = src + i * 18;
    for (int k = 0; k < 9; ++k) {
        const size_t o = ((size_t)mu * 9 + k) * V + site;
        const double re = s[2 * k], im = s[2 * k + 1];
        if constexpr (P == P64) {
            reinterpret_cast<double2*>(dst)[o] = make_double2(re, im);
        } else if constexpr (P == P32) {
            reinterpret_cast<float2*>(dst)[o] = make_float2((float)re, (float)im);
        } else if constexpr (P == P16) {
            reinterpret_cast<uint32_t*>(dst)[o] = (uint32_t)f_to_h((float)re) | ((uint32_t)f_to_h((float)im) << 16);
        } else {
            reinterpret_cast<uint32_t*>(dst)[o] =
                (uint32_t)f_to_bf16((float)re) | ((uint32_t)f_to_bf16((float)im) << 16);
        }
    }
}

// Site-major copy of the links for quad-shared loads: link (mu, site) is NW
// 32-bit words at ((mu * V + site) * NW), the complex entries packed row-major
// in the storage precision.  The full form (R = false) keeps all 9 entries in
// link_q_bytes<P>() (FP64 and FP32 in 16-byte chunks, the tail padded with
// zeros; FP16 and BF16 as nine words); the two-row form (R = true, FP32 only,
// Tr<P32>::QCR chunks) keeps rows 0 and 1, whose cross product gives row 2 of a
// special unitary link.
template <int P, bool R>
__global__ void k_gauge_convert_q(uint4* __restrict__ dst, const double* __restrict__ src, int V) {
    static_assert(!R || P == P32, "only FP32 links are kept in the two-row form");
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)4 * V) return;
    constexpr int NW = R ? 4 * Tr<P32>::QCR : (int)(link_q_bytes<P>() / 4u);
    constexpr int NE = R ? 6 : 9;
    uint32_t w[NW];
#pragma unroll
    for (int k = 0; k < NW; ++k) w[k] = 0u;
    const double* s = src + i * 18;
#pragma unroll
    for (int k = 0; k < NE; ++k) {
        const double re = s[2 * k], im = s[2 * k + 1];
        if constexpr (P == P64) {
            w[4 * k] = (uint32_t)__double2loint(re);
            w[4 * k + 1] = (uint32_t)__double2hiint(re);
            w[4 * k + 2] = (uint32_t)__double2loint(im);
            w[4 * k + 3] = (uint32_t)__double2hiint(im);
        } else if constexpr (P == P32) {
            w[2 * k] = __float_as_uint((float)re);
            w[2 * k + 1] = __float_as_uint((float)im);
        } else if constexpr (P == P16) {
            w[k] = (uint32_t)f_to_h((float)re) | ((uint32_t)f_to_h((float)im) << 16);
        } else {
            w[k] = (uint32_t)f_to_bf16((float)re) | ((uint32_t)f_to_bf16((float)im) << 16);
        }
    }
    if constexpr (NW % 4 == 0) {
        uint4* d = dst + i * (NW / 4);  // i = mu * V + site
#pragma unroll
        for (int c = 0; c < NW / 4; ++c) d[c] = make_uint4(w[4 * c], w[4 * c + 1], w[4 * c + 2], w[4 * c + 3]);
    } else {
        uint32_t* d = reinterpret_cast<uint32_t*>(dst) + i * NW;
#pragma unroll
        for (int k = 0; k < NW; ++k) d[k] = w[k];
    }
}

// ------------------------------------------------------------------ Z4 noise

template <int P>
__global__ void __launch_bounds__(256) k_noise_block(Work w, Fld dst, const NoiseKey* __restrict__ keys,
                                                     const uint16_t* __restrict__ colour) {
    using A = typename Tr<P>::acc;
    FS_WG_PROLOGUE(w)
    FS_SLOT_LOOP(w)
        const int site = (int)(slot >> w.lognr);
        const NoiseKey k = keys[sys];
        double v[24];
        if (k.pad) {  // padding system: zero source
#pragma unroll
            for (int j = 0; j < 24; ++j) v[j] = 0.0;
        } else {
            z4_site(k, site, v);
            if (k.dil > 0) {  // diluted: one probing colour, one spin-colour component
                const int d = k.dil - 1;
                const bool on = (int)colour[site] == d / 12;
#pragma unroll
                for (int j = 0; j < 12; ++j)
                    if (!on || j != d % 12) v[2 * j] = v[2 * j + 1] = 0.0;
            }
        }
        A q[24];
#pragma unroll
        for (int j = 0; j < 24; ++j) q[j] = (A)v[j];
        store_sp<P, A>(fbase_w<P>(dst, bd), nbase(dst, bd), gs, slot, q);
    FS_SLOT_LOOP_END
    FS_WG_EPILOGUE
}

__global__ void k_noise_canonical(double* __restrict__ dst, int V, NoiseKey k) {
    const int site = blockIdx.x * blockDim.x + threadIdx.x;
    if (site >= V) return;
    double v[24];
    z4_site(k, site, v);
    double2* d = reinterpret_cast<double2*>(dst) + (size_t)site * 12;
#pragma unroll
    for (int j = 0; j < 12; ++j) d[j] = make_double2(v[2 * j], v[2 * j + 1]);
}

// out = coef[sys] * in (FP64), e.g. one factor 1/a of a hopping expansion.
__global__ void __launch_bounds__(256) k_scale_sys(Work w, Fld out, Fld in, const double* __restrict__ coef) {
    FS_WG_PROLOGUE(w)
    const uint4* ib = fbase<P64>(in, bd);
    uint4* ob = fbase_w<P64>(out, bd);
    FS_SLOT_LOOP(w)
        const double c = coef[sys];
        double v[24];
        load_sp<P64, double>(ib, nullptr, gs, slot, v);
#pragma unroll
        for (int k = 0; k < 24; ++k) v[k] *= c;
        store_sp<P64, double>(ob, nullptr, gs, slot, v);
    FS_SLOT_LOOP_END
    FS_WG_EPILOGUE
}

// ------------------------------------------------------------------ multi-shift BiCGStab

struct Cx {
    double r, i;
};
__device__ __forceinline__ Cx cx(const double* a) { return {a[0], a[1]}; }
__device__ __forceinline__ Cx operator+(Cx a, Cx b) { return {a.r + b.r, a.i + b.i}; }
__device__ __forceinline__ Cx operator-(Cx a, Cx b) { return {a.r - b.r, a.i - b.i}; }
__device__ __forceinline__ Cx operator*(Cx a, Cx b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ __forceinline__ Cx operator/(Cx a, Cx b) {
    const double d = b.r * b.r + b.i * b.i;
    return {(a.r * b.r + a.i * b.i) / d, (a.i * b.r - a.r * b.i) / d};
}
__device__ __forceinline__ void put(double* o, Cx a) {
    o[0] = a.r;
    o[1] = a.i;
}

// Per (system, member) with relative shift d: the shifted BiCG factor
//   zeta_{n+1} = zeta_n zeta_{n-1} alpha_{n-1} /
//                (zeta_{n-1} alpha_{n-1} (1 + alpha_n d) + alpha_n beta_{n-1} (zeta_{n-1} - zeta_n)),
// alpha^d = alpha zeta_{n+1} / zeta_n, beta^d = (zeta_{n+1} / zeta_n)^2 beta,
// omega^d = omega / (1 + omega d), tau_{n+1} = tau_n (1 + omega d); with
// r^d_n = (zeta_n / tau_n) r_n, s^d_n = (zeta_{n+1} / tau_n) s_n and
// r_n = s_n + alpha v_n the member's update is
//   x^d += alpha^d p^d + omega^d s^d_n,
//   p^d = (zeta_{n+1} / tau_{n+1}) (s - omega t) + beta^d (p^d - (omega^d / alpha^d)(r^d_n - s^d_n)).
__global__ void k_ms_scalars(int nsys, int nm, const double* __restrict__ dsh, const SysState* __restrict__ st,
                             MsState* __restrict__ ms, MsCoef* __restrict__ co) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nsys * nm) return;
    const int sys = i / nm, k = i - sys * nm;
    const SysState& S = st[sys];
    MsState M = ms[i];
    MsCoef C;
    memset(&C, 0, sizeof(C));
    if (S.upd_x && !M.done) {
        if (S.n_rel != 0 || S.restarts != 0 || !S.upd_p) {
            M.done = 1;  // the base restarted: the members' recurrences no longer hold
        } else {
            const Cx one = {1.0, 0.0}, d = {dsh[k], 0.0};
            const Cx al = cx(S.alpha), om = cx(S.omega), be = cx(S.beta);
            const Cx zn = cx(M.z), zp = cx(M.zp), tau = cx(M.tau), ap = cx(M.ap), bp = cx(M.bp);
            const Cx zn1 = zn * zp * ap / (zp * ap * (one + al * d) + al * bp * (zp - zn));
            const Cx ak = al * zn1 / zn;
            const Cx wk = om / (one + om * d);
            const Cx bk = (zn1 / zn) * (zn1 / zn) * be;
            const Cx tau1 = tau * (one + om * d);
            const Cx q = bk * wk / ak;
            put(C.cxp, ak);
            put(C.cxs, wk * zn1 / tau);
            put(C.cpp, bk);
            put(C.cps, zn1 / tau1 - q * (zn - zn1) / tau);
            put(C.cpv, Cx{0.0, 0.0} - q * zn * al / tau);
            put(C.cpt, Cx{0.0, 0.0} - zn1 / tau1 * om);
            C.on = 1;
            M.iters += 1;
            put(M.zp, zn);
            put(M.z, zn1);
            put(M.tau, tau1);
            put(M.ap, al);
            put(M.bp, be);
            const Cx e = zn1 / tau1;
            // a margin of 2 in the residual norm for the drift of the recurrences
            if ((e.r * e.r + e.i * e.i) * S.rr <= 0.25 * S.tol2 * S.bb) M.done = 1;
            if (!isfinite(e.r) || !isfinite(e.i)) {
                M.done = 1;
                C.on = 0;
            }
        }
    }
    ms[i] = M;
    co[i] = C;
}

__global__ void __launch_bounds__(256) k_ms_update(Work w, int nm, Fld sf, Fld vf, Fld tf, MsFields f,
                                                   const MsCoef* __restrict__ co) {
    FS_WG_PROLOGUE(w)
    const uint4* sb = fbase<P64>(sf, bd);
    const uint4* vb = fbase<P64>(vf, bd);
    const uint4* tb = fbase<P64>(tf, bd);
    FS_SLOT_LOOP(w)
        bool any = false;
        for (int k = 0; k < nm; ++k) any |= co[sys * nm + k].on != 0;
        if (!any) continue;
        double sv[24], vv[24], tv[24];
        load_sp<P64, double>(sb, nullptr, gs, slot, sv);
        load_sp<P64, double>(vb, nullptr, gs, slot, vv);
        load_sp<P64, double>(tb, nullptr, gs, slot, tv);
        for (int k = 0; k < nm; ++k) {
            const MsCoef C = co[sys * nm + k];
            if (!C.on) continue;
            uint4* xb = f.x[k] + (size_t)bd.slot_off * Tr<P64>::G;
            uint4* pb = f.p[k] + (size_t)bd.slot_off * Tr<P64>::G;
            double xv[24], pv[24];
            load_sp<P64, double>(xb, nullptr, gs, slot, xv);
            load_sp<P64, double>(pb, nullptr, gs, slot, pv);
#pragma unroll
            for (int j = 0; j < 12; ++j) {
                const Cx p = {pv[2 * j], pv[2 * j + 1]}, s = {sv[2 * j], sv[2 * j + 1]};
                const Cx v = {vv[2 * j], vv[2 * j + 1]}, t = {tv[2 * j], tv[2 * j + 1]};
                const Cx x = Cx{xv[2 * j], xv[2 * j + 1]} + cx(C.cxp) * p + cx(C.cxs) * s;
                const Cx pn = cx(C.cpp) * p + cx(C.cps) * s + cx(C.cpv) * v + cx(C.cpt) * t;
                xv[2 * j] = x.r;
                xv[2 * j + 1] = x.i;
                pv[2 * j] = pn.r;
                pv[2 * j + 1] = pn.i;
            }
            store_sp<P64, double>(xb, nullptr, gs, slot, xv);
            store_sp<P64, double>(pb, nullptr, gs, slot, pv);
        }
    FS_SLOT_LOOP_END
    FS_WG_EPILOGUE
}

// ------------------------------------------------------------------ displacement + bilinear

// phi(x) = U_z(x) phi_in(x + z) per spin (colour product), or phi_in(x) at p = 0;
// M_ab += conj(y_a(x)) . phi_b(x) (colour dot), 16 complex per rhs.
__global__ void __launch_bounds__(256) k_hop_reduce(Work w, int p, Fld phi_out, Fld phi_in, Fld yfld, Fld ysrc,
                                                    const int* __restrict__ yb, double* __restrict__ part) {
    FS_WG_PROLOGUE(w)
    double acc[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) acc[k] = 0.0;
    const int pb = yb[2 * b];
    const uint4* ybase = pb >= 0 ? yfld.v + (size_t)w.blocks[pb].slot_off * 12 : ysrc.v + (size_t)bd.slot_off * 12;
    const uint4* ib = phi_in.v + (size_t)bd.slot_off * 12;
    uint4* ob = phi_out.v + (size_t)bd.slot_off * 12;
    const int Lz = ld.L[2];
    const int sz = ld.L[0] * ld.L[1];
    FS_SLOT_LOOP(w)
        (void)sys;
        const int site = (int)(slot >> w.lognr);
        double f[24];
        if (p == 0) {
            load_sp<P64, double>(ib, nullptr, gs, slot, f);
        } else {
            const int z = (site / sz) % Lz;
            const int sn = (z == Lz - 1) ? site - (Lz - 1) * sz : site + sz;
            double v[24], u[18];
            load_sp<P64, double>(ib, nullptr, gs, ((size_t)sn << w.lognr) + rhs, v);
            load_link<P64, double>(ld.gauge, ld.V, 2, site, u);
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    double re = 0.0, im = 0.0;
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        const double ur = u[2 * (3 * i + j)], ui = u[2 * (3 * i + j) + 1];
                        const double hr = v[2 * (3 * s + j)], hi = v[2 * (3 * s + j) + 1];
                        re = fma_(ur, hr, re);
                        re = fma_(-ui, hi, re);
                        im = fma_(ur, hi, im);
                        im = fma_(ui, hr, im);
                    }
                    f[2 * (3 * s + i)] = re;
                    f[2 * (3 * s + i) + 1] = im;
                }
            store_sp<P64, double>(ob, nullptr, gs, slot, f);
        }
        double y[24];
        load_sp<P64, double>(ybase, nullptr, gs, slot, y);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int bb = 0; bb < 4; ++bb) {
                double re = acc[2 * (4 * a + bb)], im = acc[2 * (4 * a + bb) + 1];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double yr = y[2 * (3 * a + c)], yi = y[2 * (3 * a + c) + 1];
                    const double fr = f[2 * (3 * bb + c)], fi = f[2 * (3 * bb + c) + 1];
                    re = fma_(yr, fr, re);
                    re = fma_(yi, fi, re);
                    im = fma_(yr, fi, im);
                    im = fma_(-yi, fr, im);
                }
                acc[2 * (4 * a + bb)] = re;
                acc[2 * (4 * a + bb) + 1] = im;
            }
    FS_SLOT_LOOP_END
    block_partials<32, 4>(acc, w.nr, part, wg_id);
    FS_WG_EPILOGUE
}

// M[(sys * M_stride + p) * 32 + k] = reduced partial k of system sys.
__global__ void __launch_bounds__(256) k_hop_finish(Work w, const double* __restrict__ part, double* __restrict__ M,
                                                    int M_stride, int p) {
    __shared__ double q[32 * 16];
    const int b = blockIdx.x;
    const int nr = w.nr;
    const BlockDesc bd = w.blocks[b];
    if (w.blk_on && !w.blk_on[b]) return;
    reduce_rows(part, 32 * nr, w.wg_start[b], w.wg_start[b + 1], q);
    for (int i = threadIdx.x; i < 32 * nr; i += blockDim.x) {
        const int k = i / nr, r = i % nr;
        M[((size_t)(bd.sys0 + r) * M_stride + p) * 32 + k] = q[i];
    }
}

__global__ void k_displace1(double* __restrict__ out, const double* __restrict__ in, const double* __restrict__ g,
                            LatDesc ld) {
    const int site = blockIdx.x * blockDim.x + threadIdx.x;
    if (site >= ld.V) return;
    const int sz = ld.L[0] * ld.L[1];
    const int Lz = ld.L[2];
    const int z = (site / sz) % Lz;
    const int sn = (z == Lz - 1) ? site - (Lz - 1) * sz : site + sz;
    const double2* U = reinterpret_cast<const double2*>(g) + (size_t)2 * 9 * ld.V + site;
    const double2* v = reinterpret_cast<const double2*>(in) + (size_t)sn * 12;
    double2* o = reinterpret_cast<double2*>(out) + (size_t)site * 12;
    for (int s = 0; s < 4; ++s)
        for (int i = 0; i < 3; ++i) {
            double re = 0.0, im = 0.0;
            for (int j = 0; j < 3; ++j) {
                const double2 u = U[(size_t)(3 * i + j) * ld.V];
                const double2 h = v[3 * s + j];
                re += u.x * h.x - u.y * h.y;
                im += u.x * h.y + u.y * h.x;
            }
            o[3 * s + i] = make_double2(re, im);
        }
}


// X[level][sample][n][p] = coef * sum_a Gamma_n[a, perm_n(a)] * sy_a * M_{a, perm_n(a)}:
// every Gamma_n of the DeGrand-Rossi basis has one nonzero (a power of i) per row.
// sy_a = -1 for a >= 2 when y carries a gamma_5 (y = g5 (D+sigma)^-1 g5 z).
__global__ void k_gamma_contract(const double* __restrict__ M, int P1, int nsys, const XMap* __restrict__ xm,
                                 GammaTab gt, double* __restrict__ X, int n_noise) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nsys * P1 * 16) return;
    const int n = i % 16;
    const int p = (i / 16) % P1;
    const int sys = i / (16 * P1);
    const XMap m = xm[sys];
    if (m.level < 0) return;
    const double* Mp = M + ((size_t)sys * P1 + p) * 32;
    double re = 0.0, im = 0.0;
    for (int a = 0; a < 4; ++a) {
        const int c = gt.perm[n][a];
        double mr = Mp[2 * (4 * a + c)], mi = Mp[2 * (4 * a + c) + 1];
        if (m.g5 && a >= 2) {
            mr = -mr;
            mi = -mi;
        }
        const int ph = gt.ph[n][a];
        const double gr = ph == 0 ? 1.0 : ph == 2 ? -1.0 : 0.0;
        const double gi = ph == 1 ? 1.0 : ph == 3 ? -1.0 : 0.0;
        re += gr * mr - gi * mi;
        im += gr * mi + gi * mr;
    }
    const size_t o = (((size_t)m.level * n_noise + m.sample) * 16 + n) * P1 + p;
    X[2 * o] = m.coef * re;
    X[2 * o + 1] = m.coef * im;
}

// Per (level, n, p): mean and the variance of eq. practical_variance over the
// samples, summed in sample order (FP64).
// Sum of the per-system estimates of the D diluted sources of each sample.
__global__ void k_dilution_sum(const double* __restrict__ Y, int P1, const int* __restrict__ g0, int G, int D,
                               double* __restrict__ X) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int per = 16 * P1;
    if (i >= G * per) return;
    const int g = i / per, np = i % per;
    const double* y = Y + 2 * ((size_t)g0[g] * per + np);
    double re = 0.0, im = 0.0;
    for (int d = 0; d < D; ++d) {
        re += y[2 * (size_t)d * per];
        im += y[2 * (size_t)d * per + 1];
    }
    X[2 * (size_t)i] = re;
    X[2 * (size_t)i + 1] = im;
}

// Samples s < N_l of level l (N_l = n_level[l], or n_noise without a table);
// X holds n_noise sample slots per level.
__global__ void k_level_stats(const double* __restrict__ X, int L1, int n_noise, int P1,
                              const int* __restrict__ n_level, double* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L1 * 16 * P1) return;
    const int p = i % P1;
    const int n = (i / P1) % 16;
    const int l = i / (16 * P1);
    const int nl = n_level ? n_level[l] : n_noise;
    double sr = 0.0, si = 0.0, s2 = 0.0;
    for (int s = 0; s < nl; ++s) {
        const size_t o = (((size_t)l * n_noise + s) * 16 + n) * P1 + p;
        const double xr = X[2 * o], xi = X[2 * o + 1];
        sr += xr;
        si += xi;
        s2 += xr * xr + xi * xi;
    }
    const double N = (double)nl;
    const double tr = nl > 0 ? sr / N : 0.0, ti = nl > 0 ? si / N : 0.0;
    const double vp = nl > 0 ? s2 / N - (tr * tr + ti * ti) : 0.0;
    double* d = out + (size_t)i * 4;
    d[0] = tr;
    d[1] = ti;
    d[2] = vp;
    d[3] = nl > 1 ? vp * N / (N - 1.0) : 0.0;
}

// Streaming copy: each lane moves 4 x 16 bytes with all loads issued first.
// Streaming copy: one 16-byte element per lane, non-temporal loads and
// stores (the fastest of the copy forms measured on the MI355X: 6.5 TB/s for
// 1 GiB, against 5.5 with four elements per lane and cached accesses).
__global__ void __launch_bounds__(256) k_copy(uint4* __restrict__ dst, const uint4* __restrict__ src, size_t n) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) st16<true>(dst + i, ld16<true>(src + i));
}

}  // namespace

// ------------------------------------------------------------------ launchers

static int grid_of(const Work& w) { return w.vlist ? persistent_grid(w.wg) : (w.total_wg + 7) / 8 * 8; }

#define FS_DISPATCH_P(prec, CALL)          \
    switch (prec) {                         \
        case P64: { constexpr int PP = P64; CALL; } break; \
        case P32: { constexpr int PP = P32; CALL; } break; \
        case P16: { constexpr int PP = P16; CALL; } break; \
        case PBF: { constexpr int PP = PBF; CALL; } break; \
        default: break;                     \
    }

// Workgroups of a one-thread-per-group FP32 launch (every block of the plan).
static unsigned grid_groups(const Work& w) { return (unsigned)((long long)Tr<P32>::G * w.total_wg * w.tpw); }

void launch_axpy_s(int prec, const Work& w, Fld r, Fld v, const SysState* st, hipStream_t s) {
    if (prec == P32 && w.wg == 256) {
        hipLaunchKernelGGL(k_axpy_s_g, dim3(grid_groups(w)), dim3(256), 0, s, w, r, v, st);
        return;
    }
    FS_DISPATCH_P(prec, hipLaunchKernelGGL(k_axpy_s<PP>, dim3(grid_of(w)), dim3(w.wg), 0, s, w, r, v, st))
}
void launch_update_xrp(int prec, const Work& w, Fld x, Fld p, Fld r, Fld t, Fld v, const SysState* st,
                       hipStream_t s) {
    if (prec == P32 && w.wg == 256) {
        hipLaunchKernelGGL(k_update_xrp_g, dim3(grid_groups(w)), dim3(256), 0, s, w, x, p, r, t, v, st);
        return;
    }
    FS_DISPATCH_P(prec, hipLaunchKernelGGL(k_update_xrp<PP>, dim3(grid_of(w)), dim3(w.wg), 0, s, w, x, p, r, t, v, st))
}
void launch_fold(int prec, const Work& w, Fld xhi, Fld xlo, const SysState* st, hipStream_t s) {
    FS_DISPATCH_P(prec, hipLaunchKernelGGL(k_fold<PP>, dim3(grid_of(w)), dim3(w.wg), 0, s, w, xhi, xlo, st))
}
void launch_convert(int prec, const Work& w, Fld rhi, Fld r, const NoiseKey* rk, uint32_t* rc, Fld p,
                    const SysState* st, double* part, hipStream_t s) {
    FS_DISPATCH_P(prec, hipLaunchKernelGGL(k_convert<PP>, dim3(grid_of(w)), dim3(w.wg), 0, s, w, rhi, r, rk, rc, p,
                                           st, part))
}
void launch_rhat_codes(const Work& w, const NoiseKey* rk, uint32_t* rc, hipStream_t s) {
    hipLaunchKernelGGL(k_rhat_codes, dim3(grid_of(w)), dim3(w.wg), 0, s, w, rk, rc);
}
void launch_init(int prec, const Work& w, Fld b, Fld xhi, Fld xlo, Fld rhi, Fld r, const NoiseKey* rk, uint32_t* rc,
                 Fld p, double* part, hipStream_t s) {
    FS_DISPATCH_P(prec, hipLaunchKernelGGL(k_init<PP>, dim3(grid_of(w)), dim3(w.wg), 0, s, w, b, xhi, xlo, rhi, r,
                                           rk, rc, p, part))
}
void launch_finish(int stage, const Work& w, SysState* st, const double* part, int* out, int* out2, hipStream_t s) {
    Work wf = w;
    const int grid = w.vlist ? std::min(w.nblk, 1024) : w.nblk;
    switch (stage) {
        case F_INIT: wf.blk_on = nullptr; wf.vlist = nullptr; hipLaunchKernelGGL(k_finish<F_INIT>, dim3(grid), dim3(256), 0, s, wf, st, part, out, out2); break;
        case F_ALPHA: hipLaunchKernelGGL(k_finish<F_ALPHA>, dim3(grid), dim3(256), 0, s, wf, st, part, out, out2); break;
        case F_OMEGA: hipLaunchKernelGGL(k_finish<F_OMEGA>, dim3(grid), dim3(256), 0, s, wf, st, part, out, out2); break;
        case F_TRUE: hipLaunchKernelGGL(k_finish<F_TRUE>, dim3(grid), dim3(256), 0, s, wf, st, part, out, out2); break;
        case F_RESUME: hipLaunchKernelGGL(k_finish<F_RESUME>, dim3(grid), dim3(256), 0, s, wf, st, part, out, out2); break;
        case F_BNORM: wf.blk_on = nullptr; wf.vlist = nullptr; hipLaunchKernelGGL(k_finish<F_BNORM>, dim3(grid), dim3(256), 0, s, wf, st, part, out, out2); break;
        default: break;
    }
}
void launch_blk_mask(const Work& w, const SysState* st, int mask, int* blk_on, hipStream_t s) {
    hipLaunchKernelGGL(k_blk_mask, dim3((w.nblk + 255) / 256), dim3(256), 0, s, w, st, mask, blk_on);
}
void launch_vlist(const int* flags, int nblk, const int* wg_tile, const int* wg_sten, VList out, hipStream_t s) {
    hipLaunchKernelGGL(k_vlist, dim3(1), dim3(256), 0, s, flags, nblk, wg_tile, wg_sten, out);
}
void launch_pack(int prec, const Work& w, Fld dst, const double* src, long long sys_stride, const int* sys_map,
                 hipStream_t s) {
    FS_DISPATCH_P(prec, hipLaunchKernelGGL(k_pack<PP>, dim3(grid_of(w)), dim3(w.wg), 0, s, w, dst, src, sys_stride,
                                           sys_map))
}
void launch_unpack(int prec, const Work& w, double* dst, Fld src, long long sys_stride, const int* sys_map,
                   hipStream_t s) {
    FS_DISPATCH_P(prec, hipLaunchKernelGGL(k_unpack<PP>, dim3(grid_of(w)), dim3(w.wg), 0, s, w, dst, src, sys_stride,
                                           sys_map))
}
void launch_ms_scalars(int nsys, int nm, const double* d, const SysState* st, MsState* ms, MsCoef* co,
                       hipStream_t s) {
    const int n = nsys * nm;
    if (n > 0) hipLaunchKernelGGL(k_ms_scalars, dim3((n + 255) / 256), dim3(256), 0, s, nsys, nm, d, st, ms, co);
}
void launch_ms_update(const Work& w, int nm, Fld s_, Fld v, Fld t, const MsFields& f, const MsCoef* co,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_ms_update, dim3(grid_of(w)), dim3(w.wg), 0, s, w, nm, s_, v, t, f, co);
}
void launch_scale_sys(const Work& w, Fld out, Fld in, const double* coef, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_sys, dim3(grid_of(w)), dim3(w.wg), 0, s, w, out, in, coef);
}
void launch_gauge_convert(int prec, void* dst, const double* src, int V, hipStream_t s) {
    const int n = 4 * V;
    FS_DISPATCH_P(prec, hipLaunchKernelGGL(k_gauge_convert<PP>, dim3((n + 255) / 256), dim3(256), 0, s, dst, src, V))
}
void launch_gauge_convert_q(int prec, void* dst, const double* src, int V, bool two_rows, hipStream_t s) {
    const int n = 4 * V;
    if (two_rows && prec == P32)
        hipLaunchKernelGGL((k_gauge_convert_q<P32, true>), dim3((n + 255) / 256), dim3(256), 0, s,
                           static_cast<uint4*>(dst), src, V);
    else
        FS_DISPATCH_P(prec, hipLaunchKernelGGL((k_gauge_convert_q<PP, false>), dim3((n + 255) / 256), dim3(256), 0,
                                               s, static_cast<uint4*>(dst), src, V))
}
void launch_noise_block(int prec, const Work& w, Fld dst, const NoiseKey* keys, hipStream_t s,
                        const uint16_t* colour) {
    FS_DISPATCH_P(prec,
                  hipLaunchKernelGGL(k_noise_block<PP>, dim3(grid_of(w)), dim3(w.wg), 0, s, w, dst, keys, colour))
}
void launch_noise_canonical(double* dst, int V, NoiseKey key, hipStream_t s) {
    hipLaunchKernelGGL(k_noise_canonical, dim3((V + 255) / 256), dim3(256), 0, s, dst, V, key);
}
void launch_hop_reduce(const Work& w, int p, Fld phi_out, Fld phi_in, Fld yfld, Fld ysrc, const int* yb,
                       double* part, hipStream_t s) {
    hipLaunchKernelGGL(k_hop_reduce, dim3(grid_of(w)), dim3(w.wg), 0, s, w, p, phi_out, phi_in, yfld, ysrc, yb, part);
}
void launch_hop_finish(const Work& w, const double* part, double* M, int M_stride, int p, hipStream_t s) {
    hipLaunchKernelGGL(k_hop_finish, dim3(w.nblk), dim3(256), 0, s, w, part, M, M_stride, p);
}
void launch_displace_canonical(double* out, const double* in, const double* gauge64, LatDesc ld, hipStream_t s) {
    hipLaunchKernelGGL(k_displace1, dim3((ld.V + 127) / 128), dim3(128), 0, s, out, in, gauge64, ld);
}
void launch_gamma_contract(const double* M, int P1, int nsys, const XMap* xm, const GammaTab& gt, double* X,
                           int n_noise, hipStream_t s) {
    const int n = nsys * P1 * 16;
    hipLaunchKernelGGL(k_gamma_contract, dim3((n + 255) / 256), dim3(256), 0, s, M, P1, nsys, xm, gt, X, n_noise);
}
void launch_dilution_sum(const double* Y, int P1, const int* g0, int G, int D, double* X, hipStream_t s) {
    const int n = G * 16 * P1;
    hipLaunchKernelGGL(k_dilution_sum, dim3((n + 255) / 256), dim3(256), 0, s, Y, P1, g0, G, D, X);
}
void launch_level_stats(const double* X, int L1, int n_noise, int P1, double* out, hipStream_t s,
                        const int* n_level) {
    const int n = L1 * 16 * P1;
    hipLaunchKernelGGL(k_level_stats, dim3((n + 255) / 256), dim3(256), 0, s, X, L1, n_noise, P1, n_level, out);
}
void launch_copy(uint4* dst, const uint4* src, size_t n16, hipStream_t s) {
    const size_t blocks = (n16 + 255) / 256;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, s, dst, src, n16);
}

}  // namespace fs
