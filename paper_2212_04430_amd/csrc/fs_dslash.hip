// Shifted Wilson dslash for gfx950:
//   ((D + sigma) psi)(x) = (4 + m0 + sigma) psi(x)
//       - 1/2 sum_mu [(1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^+ psi(x-mu)]
// (DeGrand-Rossi gamma basis).  The operator is the one whose shifted inverses
// the Frequency-Splitting levels are built from (paper Sec. 2.2, eq.
// tele_sum_prod_disp; Sec. 3.1, eq. shifted_linear_systems).
//
// One lane computes one (site, rhs) of a block of NR right-hand sides stored
// [group][site][NR]; the NR lanes of one site share each link load (the
// hardware merges equal addresses within a wave), so link traffic per rhs is
// divided by NR.  Each hop is spin-projected to a half spinor before the SU(3)
// product, halving the colour arithmetic.  Fused epilogues produce the
// per-workgroup partial sums that BiCGStab needs (FP64).
#include <algorithm>

#include "fs_kernels.h"

namespace fs {

namespace {

template <typename A>
__device__ __forceinline__ void ph(int code, A re, A im, A& ore, A& oim) {
    // multiply (re + i im) by i^code
    if (code == 0) { ore = re; oim = im; }
    else if (code == 1) { ore = -im; oim = re; }
    else if (code == 2) { ore = -re; oim = -im; }
    else { ore = im; oim = -re; }
}

// Spin projection (1 -/+ g_mu) psi -> half spinor h[2][3] and reconstruction.
// Each row of a projector is h0 = psi0 + i^A0 psi_J0, h1 = psi1 + i^A1 psi_J1;
// the lower two spins of the result are i^B2 h_K2 and i^B3 h_K3.
template <int J0, int A0, int J1, int A1, int K2, int B2, int K3, int B3>
struct Proj {
    template <typename A>
    __device__ __forceinline__ static void project(const A v[24], A h[12]) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            A re, im;
            ph<A>(A0, v[2 * (J0 * 3 + c)], v[2 * (J0 * 3 + c) + 1], re, im);
            h[2 * c] = v[2 * c] + re;
            h[2 * c + 1] = v[2 * c + 1] + im;
            ph<A>(A1, v[2 * (J1 * 3 + c)], v[2 * (J1 * 3 + c) + 1], re, im);
            h[6 + 2 * c] = v[2 * (3 + c)] + re;
            h[6 + 2 * c + 1] = v[2 * (3 + c) + 1] + im;
        }
    }
    template <typename A>
    __device__ __forceinline__ static void accum(A o[24], const A w[12], A cf) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            o[2 * c] += cf * w[2 * c];
            o[2 * c + 1] += cf * w[2 * c + 1];
            o[2 * (3 + c)] += cf * w[6 + 2 * c];
            o[2 * (3 + c) + 1] += cf * w[6 + 2 * c + 1];
            A re, im;
            ph<A>(B2, w[6 * K2 + 2 * c], w[6 * K2 + 2 * c + 1], re, im);
            o[2 * (6 + c)] += cf * re;
            o[2 * (6 + c) + 1] += cf * im;
            ph<A>(B3, w[6 * K3 + 2 * c], w[6 * K3 + 2 * c + 1], re, im);
            o[2 * (9 + c)] += cf * re;
            o[2 * (9 + c) + 1] += cf * im;
        }
    }
};

// phase codes: 0 -> +1, 1 -> +i, 2 -> -1, 3 -> -i
using PxM = Proj<3, 3, 2, 3, 1, 1, 0, 1>;  // 1 - g1
using PxP = Proj<3, 1, 2, 1, 1, 3, 0, 3>;  // 1 + g1
using PyM = Proj<3, 0, 2, 2, 1, 2, 0, 0>;  // 1 - g2
using PyP = Proj<3, 2, 2, 0, 1, 0, 0, 2>;  // 1 + g2
using PzM = Proj<2, 3, 3, 1, 0, 1, 1, 3>;  // 1 - g3
using PzP = Proj<2, 1, 3, 3, 0, 3, 1, 1>;  // 1 + g3
using PtM = Proj<2, 2, 3, 2, 0, 2, 1, 2>;  // 1 - g4
using PtP = Proj<2, 0, 3, 0, 0, 0, 1, 0>;  // 1 + g4

template <typename A>
__device__ __forceinline__ void mul_u(const A u[18], const A h[12], A w[12]) {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            A re = 0, im = 0;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                A ur = u[2 * (3 * i + j)], ui = u[2 * (3 * i + j) + 1];
                A hr = h[6 * s + 2 * j], hi = h[6 * s + 2 * j + 1];
                re += ur * hr - ui * hi;
                im += ur * hi + ui * hr;
            }
            w[6 * s + 2 * i] = re;
            w[6 * s + 2 * i + 1] = im;
        }
}

template <typename A>
__device__ __forceinline__ void mul_udag(const A u[18], const A h[12], A w[12]) {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            A re = 0, im = 0;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                A ur = u[2 * (3 * j + i)], ui = -u[2 * (3 * j + i) + 1];
                A hr = h[6 * s + 2 * j], hi = h[6 * s + 2 * j + 1];
                re += ur * hr - ui * hi;
                im += ur * hi + ui * hr;
            }
            w[6 * s + 2 * i] = re;
            w[6 * s + 2 * i + 1] = im;
        }
}

template <int P, int MU, typename PF, typename PB>
__device__ __forceinline__ void hop_dir(const LatDesc& ld, const uint4* __restrict__ ib,
                                        const float* __restrict__ inn, size_t gs, int site, int coord,
                                        int stride, int r, int lognr, typename Tr<P>::acc o[24]) {
    using A = typename Tr<P>::acc;
    const int Lm = ld.L[MU];
    const int sf = (coord == Lm - 1) ? site - (Lm - 1) * stride : site + stride;
    const int sb = (coord == 0) ? site + (Lm - 1) * stride : site - stride;
    A cf = A(-0.5), cb = A(-0.5);
    if (MU == 3 && ld.tsign < 0) {
        if (coord == Lm - 1) cf = A(0.5);
        if (coord == 0) cb = A(0.5);
    }
    {
        A v[24], h[12], u[18], w[12];
        load_sp<P, A>(ib, inn, gs, ((size_t)sf << lognr) + r, v);
        PF::project(v, h);
        load_link<P, A>(ld.gauge, ld.V, MU, site, u);
        mul_u(u, h, w);
        PF::accum(o, w, cf);
    }
    {
        A v[24], h[12], u[18], w[12];
        load_sp<P, A>(ib, inn, gs, ((size_t)sb << lognr) + r, v);
        PB::project(v, h);
        load_link<P, A>(ld.gauge, ld.V, MU, sb, u);
        mul_udag(u, h, w);
        PB::accum(o, w, cb);
    }
}

__device__ __forceinline__ bool mask_ok(int mask, const SysState* __restrict__ st, int sys) {
    if (mask == M_ALL) return true;
    const int s = st[sys].state;
    if (mask == M_RUN) return s == S_RUN;
    if (mask == M_PEND) return s == S_REL || s == S_CHK || s == S_BRK || s == S_MAXIT;
    if (mask == M_CONVERT) return s == S_CONV || s == S_RST;
    return st[sys].upd_p != 0;
}

template <int MODE> struct NDots { static constexpr int v = 1; };
template <> struct NDots<D_RHAT> { static constexpr int v = 2; };
template <> struct NDots<D_TS> { static constexpr int v = 3; };
template <> struct NDots<D_RESID> { static constexpr int v = 1; };

// Stencil over t-columns.  A workgroup owns `wg` consecutive (xyz, rhs) slots
// of one block and walks t through a chunk of `tc` slices; each lane carries
// the backward-t half spinor U_t(x,t-1)^+ (1+g4) psi(x,t-1) in registers from
// one slice to the next, so the t-direction needs no cache reuse, while the
// x/y/z neighbours of slice t are loaded by neighbouring lanes and concurrently
// running workgroups at the same t (L1/L2 hits).
// Two register budgets per precision.  ILP = 0 lets the compiler size the
// allocation for several resident waves; ILP = 1 allows one wave per SIMD the
// whole register file, so a site's neighbour and link loads are all in flight
// at once.  Which one wins depends on how much of the stencil's footprint the
// per-XCD L2 holds, so the autotuner measures both, together with a cap on
// resident waves (dynamic LDS per workgroup, see launch_dslash).
template <int P, int ILP> struct Wpe {
    static constexpr int lo = 1;
    static constexpr int hi = ILP ? 1 : 8;
};

template <int P, int MODE, int ILP>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(Wpe<P, ILP>::lo, Wpe<P, ILP>::hi)))
k_dslash(Work w, Fld out, Fld in, Fld aux,
                                                const double* __restrict__ diag,
                                                const SysState* __restrict__ st, int mask,
                                                double* __restrict__ part, const NoiseKey* __restrict__ rk) {
    using A = typename Tr<P>::acc;
    constexpr int G = Tr<P>::G;
    constexpr int ND = NDots<MODE>::v;
    for_each_vwg(w, [&](const int wg_id, const int b) {
    const BlockDesc bd = w.blocks[b];
    const LatDesc ld = w.lats[bd.lat];
    const int wgb = wg_id - w.wg_start[b];
    const size_t gs = (size_t)ld.V << w.lognr;
    const uint4* ib = in.v + (size_t)bd.slot_off * G;
    const float* inn = in.n ? in.n + bd.slot_off : nullptr;
    uint4* ob = out.v + (size_t)bd.slot_off * G;
    float* on = out.n ? out.n + bd.slot_off : nullptr;
    const int sy = ld.L[0], sz = ld.L[0] * ld.L[1], vxyz = sz * ld.L[2];
    const int Lt = ld.L[3];
    const int n3 = vxyz << w.lognr;             // (xyz, rhs) slots of one t-slice
    const int ntile3 = (n3 + w.wg - 1) / w.wg;
    const int j = wgb % ntile3, ch = wgb / ntile3;
    const int s3 = j * w.wg + threadIdx.x;
    const int t0 = ch * w.tc, t1 = min(Lt, t0 + w.tc);

    double acc[ND];
#pragma unroll
    for (int k = 0; k < ND; ++k) acc[k] = 0.0;

    const int xyz = s3 >> w.lognr;
    const int r = s3 & (w.nr - 1);
    const int sys = bd.sys0 + r;
    if (s3 < n3 && mask_ok(mask, st, sys)) {
        const A dg = (A)diag[sys];
        Coord c;
        {
            int q = xyz;
            c.x = q % ld.L[0];
            q /= ld.L[0];
            c.y = q % ld.L[1];
            c.z = q / ld.L[1];
        }
        // backward-t contribution entering slice t0: from (x, t0-1)
        A bw[12];
        {
            const int tb = (t0 == 0) ? Lt - 1 : t0 - 1;
            const int sb = xyz + vxyz * tb;
            A v[24], h[12], u[18];
            load_sp<P, A>(ib, inn, gs, ((size_t)sb << w.lognr) + r, v);
            PtP::project(v, h);
            load_link<P, A>(ld.gauge, ld.V, 3, sb, u);
            mul_udag(u, h, bw);
            if (t0 == 0 && ld.tsign < 0) {
#pragma unroll
                for (int k = 0; k < 12; ++k) bw[k] = -bw[k];
            }
        }
        // centre spinor of the current slice, carried in registers: the
        // forward-t neighbour loaded at slice t is the centre of slice t+1
        A cv[24];
        load_sp<P, A>(ib, inn, gs, ((size_t)(xyz + vxyz * t0) << w.lognr) + r, cv);
#pragma unroll 1
        for (int t = t0; t < t1; ++t) {
            const int site = xyz + vxyz * t;
            const size_t slot = ((size_t)site << w.lognr) + r;
            A o[24];
            A bn[12];  // backward-t term of slice t+1
            {
                // centre: diagonal term, and with U_t(x,t) the next slice's backward term
                A h[12], u[18];
#pragma unroll
                for (int k = 0; k < 24; ++k) o[k] = dg * cv[k];
                load_link<P, A>(ld.gauge, ld.V, 3, site, u);
                PtP::project(cv, h);
                mul_udag(u, h, bn);
                // forward t hop with the same link
                const bool wrap = (t == Lt - 1);
                const int sf = wrap ? xyz : site + vxyz;
                A ww[12], v[24];
                load_sp<P, A>(ib, inn, gs, ((size_t)sf << w.lognr) + r, v);
                PtM::project(v, h);
                mul_u(u, h, ww);
                PtM::accum(o, ww, (wrap && ld.tsign < 0) ? A(0.5) : A(-0.5));
#pragma unroll
                for (int k = 0; k < 24; ++k) {
                    const A c0 = cv[k];
                    cv[k] = v[k];      // next slice's centre
                    v[k] = c0;         // this slice's centre, for the dot below
                }
                PtP::accum(o, bw, A(-0.5));
                hop_dir<P, 0, PxM, PxP>(ld, ib, inn, gs, site, c.x, 1, r, w.lognr, o);
                hop_dir<P, 1, PyM, PyP>(ld, ib, inn, gs, site, c.y, sy, r, w.lognr, o);
                hop_dir<P, 2, PzM, PzP>(ld, ib, inn, gs, site, c.z, sz, r, w.lognr, o);
#pragma unroll
                for (int k = 0; k < 12; ++k) bw[k] = bn[k];
                if constexpr (MODE == D_TS) {
#pragma unroll
                    for (int k = 0; k < 12; ++k) {
                        const double tr = o[2 * k], ti = o[2 * k + 1], sr = v[2 * k], si = v[2 * k + 1];
                        acc[0] += tr * sr + ti * si;
                        acc[1] += tr * si - ti * sr;
                        acc[2] += tr * tr + ti * ti;
                    }
                }
            }
            if constexpr (MODE == D_RESID) {
                A bv[24];
                load_sp<P, A>(aux.v + (size_t)bd.slot_off * G, nullptr, gs, slot, bv);
#pragma unroll
                for (int k = 0; k < 24; ++k) o[k] = bv[k] - o[k];
            }
            store_sp<P, A>(ob, on, gs, slot, o);
            if constexpr (MODE == D_RHAT) {
                A rh[24];
                rhat_site<A>(rk[sys], st[sys].restarts, site, rh);
#pragma unroll
                for (int k = 0; k < 12; ++k) {
                    acc[0] += (double)rh[2 * k] * (double)o[2 * k] + (double)rh[2 * k + 1] * (double)o[2 * k + 1];
                    acc[1] += (double)rh[2 * k] * (double)o[2 * k + 1] - (double)rh[2 * k + 1] * (double)o[2 * k];
                }
            } else if constexpr (MODE == D_RESID) {
#pragma unroll
                for (int k = 0; k < 24; ++k) acc[0] += (double)o[k] * (double)o[k];
            }
        }
    }
    if constexpr (MODE != D_PLAIN) block_partials<ND, 4>(acc, w.nr, part, wg_id);
    });
}

}  // namespace

static int grid_of(const Work& w) { return w.vlist ? persistent_grid(w.wg) : (w.total_wg + 7) / 8 * 8; }

// Dynamic LDS that caps resident workgroups per CU (160 KiB of LDS per CU):
// waves = target waves per SIMD (0 = no cap).
static size_t lds_cap(int wg, int waves) {
    if (waves <= 0) return 0;
    const int waves_per_wg = (wg + 63) / 64;
    int wg_per_cu = std::max(1, (waves * 4) / waves_per_wg);
    size_t bytes = (size_t)(160 * 1024) / (size_t)wg_per_cu;
    bytes = bytes > 4096 ? bytes - 4096 : 0;  // leave room for the static partial-sum buffer
    return std::min<size_t>(bytes, 64 * 1024);
}

template <int P, int MODE, int ILP>
static void launch_t(const Work& w, Fld out, Fld in, Fld aux, const double* diag, const SysState* st,
                     int mask, double* part, hipStream_t s, const NoiseKey* rk) {
    hipLaunchKernelGGL((k_dslash<P, MODE, ILP>), dim3(grid_of(w)), dim3(w.wg), lds_cap(w.wg, w.occ), s, w, out, in,
                       aux, diag, st, mask, part, rk);
}

template <int P, int MODE>
static void launch_v(const Work& w, Fld out, Fld in, Fld aux, const double* diag, const SysState* st,
                     int mask, double* part, hipStream_t s, const NoiseKey* rk) {
    if (w.ilp) launch_t<P, MODE, 1>(w, out, in, aux, diag, st, mask, part, s, rk);
    else launch_t<P, MODE, 0>(w, out, in, aux, diag, st, mask, part, s, rk);
}

template <int P>
static void launch_p(int mode, const Work& w, Fld out, Fld in, Fld aux, const double* diag,
                     const SysState* st, int mask, double* part, hipStream_t s, const NoiseKey* rk) {
    switch (mode) {
        case D_PLAIN: launch_v<P, D_PLAIN>(w, out, in, aux, diag, st, mask, part, s, rk); break;
        case D_RHAT: launch_v<P, D_RHAT>(w, out, in, aux, diag, st, mask, part, s, rk); break;
        case D_TS: launch_v<P, D_TS>(w, out, in, aux, diag, st, mask, part, s, rk); break;
        default: break;
    }
}

void launch_dslash(int prec, int mode, const Work& w, Fld out, Fld in, Fld aux, const double* diag,
                   const SysState* st, int mask, double* part, hipStream_t s, const NoiseKey* rk) {
    if (mode == D_RESID) {
        launch_v<P64, D_RESID>(w, out, in, aux, diag, st, mask, part, s, rk);
        return;
    }
    switch (prec) {
        case P64: launch_p<P64>(mode, w, out, in, aux, diag, st, mask, part, s, rk); break;
        case P32: launch_p<P32>(mode, w, out, in, aux, diag, st, mask, part, s, rk); break;
        case P16: launch_p<P16>(mode, w, out, in, aux, diag, st, mask, part, s, rk); break;
        case PBF: launch_p<PBF>(mode, w, out, in, aux, diag, st, mask, part, s, rk); break;
        default: break;
    }
}

}  // namespace fs
