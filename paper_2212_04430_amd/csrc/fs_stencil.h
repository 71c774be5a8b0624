// Stencil kernels of the shifted Wilson-Dirac operator (device templates shared
// by the launch files of the plain and the clover-improved operator).
//
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
#pragma once

#include <algorithm>

#include "fs_kernels.h"

namespace fs {

namespace {

// Packed FP16 complex (re, im): the FP16 x-pair stencil works on stored
// spinors in this form (see PairIn).
typedef _Float16 h2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ h2 as_h2(uint32_t w) { return __builtin_bit_cast(h2, w); }
template <int K>
__device__ __forceinline__ h2 ph_h(h2 b) {  // i^K b
    if constexpr (K == 0) return b;
    else if constexpr (K == 1) return (h2){-b.y, b.x};
    else if constexpr (K == 2) return -b;
    else return (h2){b.y, -b.x};
}
__device__ __forceinline__ h2 conj_h(h2 z) { return (h2){z.x, -z.y}; }
// a.x b.x + a.y b.y in FP32 (the first term of a chain): the three-operand
// encoding with an inline zero; the builtin with a zero accumulator compiles to
// the two-operand accumulate-in-place form plus a copy of the zero.
__device__ __forceinline__ float dot2_first(h2 a, h2 b) {
    float r;
    asm("v_dot2_f32_f16 %0, %1, %2, 0" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ h2 swap_h(h2 z) { return (h2){z.y, z.x}; }

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
    // The same projection of a stored FP16 spinor (12 packed complex), in the
    // two operand forms its link product takes: for U h, conj(h) and swap(h)
    // = (Im h, Re h); for U^+ h, h and -i h.  Each form is one packed FP16 add
    // per complex (the phases become operand swaps and negations).
    __device__ __forceinline__ static void project_fwd_h(const uint32_t v[12], h2 hc[6], h2 hs[6]) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const h2 a0 = as_h2(v[c]), b0 = ph_h<A0>(as_h2(v[J0 * 3 + c]));
            const h2 a1 = as_h2(v[3 + c]), b1 = ph_h<A1>(as_h2(v[J1 * 3 + c]));
            hc[c] = conj_h(a0) + conj_h(b0);
            hs[c] = swap_h(a0) + swap_h(b0);
            hc[3 + c] = conj_h(a1) + conj_h(b1);
            hs[3 + c] = swap_h(a1) + swap_h(b1);
        }
    }
    __device__ __forceinline__ static void project_bwd_h(const uint32_t v[12], h2 hh[6], h2 hn[6]) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const h2 a0 = as_h2(v[c]), b0 = ph_h<A0>(as_h2(v[J0 * 3 + c]));
            const h2 a1 = as_h2(v[3 + c]), b1 = ph_h<A1>(as_h2(v[J1 * 3 + c]));
            hh[c] = a0 + b0;
            hn[c] = ph_h<3>(a0) + ph_h<3>(b0);
            hh[3 + c] = a1 + b1;
            hn[3 + c] = ph_h<3>(a1) + ph_h<3>(b1);
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

// Complex 3x3 matrix times the two colour vectors of a half spinor, as chains
// of fused multiply-adds: 4 operations per complex product, the first of each
// sum a plain product.  (Written as re += ur*hr - ui*hi the compiler keeps the
// difference as its own rounding step and spends 6.)
template <typename A>
__device__ __forceinline__ void mul_u(const A u[18], const A h[12], A w[12]) {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const A* hs = h + 6 * s;
            const A* ur = u + 6 * i;  // row i
            A re = ur[0] * hs[0], im = ur[0] * hs[1];
            re = fma_(-ur[1], hs[1], re);
            im = fma_(ur[1], hs[0], im);
#pragma unroll
            for (int j = 1; j < 3; ++j) {
                re = fma_(ur[2 * j], hs[2 * j], re);
                re = fma_(-ur[2 * j + 1], hs[2 * j + 1], re);
                im = fma_(ur[2 * j], hs[2 * j + 1], im);
                im = fma_(ur[2 * j + 1], hs[2 * j], im);
            }
            w[6 * s + 2 * i] = re;
            w[6 * s + 2 * i + 1] = im;
        }
}

// The same with the Hermitian conjugate U^dagger (column i of U, conjugated).
template <typename A>
__device__ __forceinline__ void mul_udag(const A u[18], const A h[12], A w[12]) {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const A* hs = h + 6 * s;
            A re = u[2 * i] * hs[0], im = u[2 * i] * hs[1];
            re = fma_(u[2 * i + 1], hs[1], re);
            im = fma_(-u[2 * i + 1], hs[0], im);
#pragma unroll
            for (int j = 1; j < 3; ++j) {
                const A cr = u[2 * (3 * j + i)], ci = u[2 * (3 * j + i) + 1];
                re = fma_(cr, hs[2 * j], re);
                re = fma_(ci, hs[2 * j + 1], re);
                im = fma_(cr, hs[2 * j + 1], im);
                im = fma_(-ci, hs[2 * j], im);
            }
            w[6 * s + 2 * i] = re;
            w[6 * s + 2 * i + 1] = im;
        }
}

// U h for a half spinor in its packed forms hc = conj(h), hs = swap(h): each
// complex product is two v_dot2_f32_f16 (Re: u . conj(h), Im: u . swap(h)),
// summed in FP32.  u: 9 packed FP16 complex, row-major.
__device__ __forceinline__ void mul_u_h(const uint32_t u[9], const h2 hc[6], const h2 hs[6], float w[12]) {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            float re = dot2_first(as_h2(u[3 * i]), hc[3 * s]);
            float im = dot2_first(as_h2(u[3 * i]), hs[3 * s]);
#pragma unroll
            for (int j = 1; j < 3; ++j) {
                re = __builtin_amdgcn_fdot2(as_h2(u[3 * i + j]), hc[3 * s + j], re, false);
                im = __builtin_amdgcn_fdot2(as_h2(u[3 * i + j]), hs[3 * s + j], im, false);
            }
            w[6 * s + 2 * i] = re;
            w[6 * s + 2 * i + 1] = im;
        }
}

// U^+ h with hh = h, hn = -i h: Re conj(u) h = u . h, Im conj(u) h = u . (-i h).
__device__ __forceinline__ void mul_udag_h(const uint32_t u[9], const h2 hh[6], const h2 hn[6], float w[12]) {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            float re = dot2_first(as_h2(u[i]), hh[3 * s]);
            float im = dot2_first(as_h2(u[i]), hn[3 * s]);
#pragma unroll
            for (int j = 1; j < 3; ++j) {
                re = __builtin_amdgcn_fdot2(as_h2(u[3 * j + i]), hh[3 * s + j], re, false);
                im = __builtin_amdgcn_fdot2(as_h2(u[3 * j + i]), hn[3 * s + j], im, false);
            }
            w[6 * s + 2 * i] = re;
            w[6 * s + 2 * i + 1] = im;
        }
}

// FP16 link U_mu(site) as 9 packed complex, by link variant Q (see link()).
template <int Q>
__device__ __forceinline__ void link_h(const LatDesc& ld, int mu, int site, uint32_t u[9]) {
    if constexpr (Q == 0) {
        const uint32_t plane = uni((uint32_t)ld.V * 4u);
        const auto rs = buf_rsrc(reinterpret_cast<const char*>(ld.gauge) + (size_t)mu * 9 * plane, 9 * plane);
        const uint32_t off = (uint32_t)site * 4u;
#pragma unroll
        for (int k = 0; k < 9; ++k) u[k] = __builtin_amdgcn_raw_buffer_load_b32(rs, off, k * plane, 0);
    } else {
        // quad-shared: nine packed words per site, lanes 0-2 load three each
        constexpr uint32_t QB = link_q_bytes<P16>();
        const uint32_t plane = uni((uint32_t)ld.V * QB);
        const auto rs = buf_rsrc(reinterpret_cast<const char*>(ld.gauge_q) + (size_t)mu * plane, plane);
        load_words9_q(rs, (uint32_t)site * QB, threadIdx.x & 3, u);
    }
}

// LDS entries of a spinor in the tiled stencils: [16-byte group][lane].
template <typename A> struct LdsVec;
template <> struct LdsVec<float> { using T = float4; };
template <> struct LdsVec<double> { using T = double2; };

template <typename A>
__device__ __forceinline__ void lds_put(typename LdsVec<A>::T* sh, int wg, int lane, const A v[24]) {
    constexpr int K = 16 / sizeof(A);
#pragma unroll
    for (int g = 0; g < 24 / K; ++g) {
        typename LdsVec<A>::T q;
        if constexpr (K == 4) q = make_float4(v[4 * g], v[4 * g + 1], v[4 * g + 2], v[4 * g + 3]);
        else q = make_double2(v[2 * g], v[2 * g + 1]);
        sh[g * wg + lane] = q;
    }
}

template <typename A>
__device__ __forceinline__ void lds_get(const typename LdsVec<A>::T* sh, int wg, int lane, A v[24]) {
    constexpr int K = 16 / sizeof(A);
#pragma unroll
    for (int g = 0; g < 24 / K; ++g) {
        const typename LdsVec<A>::T q = sh[g * wg + lane];
        if constexpr (K == 4) {
            v[4 * g] = q.x; v[4 * g + 1] = q.y; v[4 * g + 2] = q.z; v[4 * g + 3] = q.w;
        } else {
            v[2 * g] = q.x; v[2 * g + 1] = q.y;
        }
    }
}

// Input spinors of the hop stencils as loaded, exchanged through LDS and
// selected.  FP64, FP32 and BF16: the 24 reals in the arithmetic type.  FP16:
// the stored form, 12 packed complex and the slot's scale, so the projection
// adds in FP16 and every link product is a v_dot2_f32_f16 (two FP16 products
// summed in FP32); the hop results are scaled and accumulated in FP32.  The
// projection rounds once more than storage does, by at most half an FP16 ulp
// of the normalised sum.  (The x-pair stencil takes every hop in this form;
// the streaming stencils their x, y and z hops.)
struct SpH {
    uint32_t w[12];  // component spin * 3 + colour as a (re, im) FP16 pair
    float s;         // scale: the spinor is s * w
};
template <int P> struct PairIn {
    struct T {
        typename Tr<P>::acc v[24];
    };
};
template <> struct PairIn<P16> { using T = SpH; };

// LDS bytes per lane of one slice buffer: [groups][lanes] 16-byte groups (FP16:
// then [lanes] scales).
template <int P> constexpr int in_lds_bytes() { return P == P16 ? 52 : 24 * (int)sizeof(typename Tr<P>::acc); }

template <int P>
__device__ __forceinline__ void in_load(const uint4* __restrict__ ib, const float* __restrict__ inn, size_t gs,
                                        size_t slot, typename PairIn<P>::T& x) {
    if constexpr (P == P16) {
#pragma unroll
        for (int g = 0; g < 3; ++g) {
            const uint4 d = ld16<false>(ib + g * gs + slot);
            x.w[4 * g] = d.x;
            x.w[4 * g + 1] = d.y;
            x.w[4 * g + 2] = d.z;
            x.w[4 * g + 3] = d.w;
        }
        x.s = inn[slot];
    } else {
        load_sp<P, typename Tr<P>::acc>(ib, inn, gs, slot, x.v);
    }
}

template <int P>
__device__ __forceinline__ void in_put(char* sh, int wg, int lane, const typename PairIn<P>::T& x) {
    if constexpr (P == P16) {
        uint4* q = reinterpret_cast<uint4*>(sh);
#pragma unroll
        for (int g = 0; g < 3; ++g)
            q[g * wg + lane] = make_uint4(x.w[4 * g], x.w[4 * g + 1], x.w[4 * g + 2], x.w[4 * g + 3]);
        reinterpret_cast<float*>(q + 3 * wg)[lane] = x.s;
    } else {
        using A = typename Tr<P>::acc;
        lds_put<A>(reinterpret_cast<typename LdsVec<A>::T*>(sh), wg, lane, x.v);
    }
}

template <int P>
__device__ __forceinline__ void in_get(const char* sh, int wg, int lane, typename PairIn<P>::T& x) {
    if constexpr (P == P16) {
        const uint4* q = reinterpret_cast<const uint4*>(sh);
#pragma unroll
        for (int g = 0; g < 3; ++g) {
            const uint4 d = q[g * wg + lane];
            x.w[4 * g] = d.x;
            x.w[4 * g + 1] = d.y;
            x.w[4 * g + 2] = d.z;
            x.w[4 * g + 3] = d.w;
        }
        x.s = reinterpret_cast<const float*>(q + 3 * wg)[lane];
    } else {
        using A = typename Tr<P>::acc;
        lds_get<A>(reinterpret_cast<const typename LdsVec<A>::T*>(sh), wg, lane, x.v);
    }
}

// o = c ? a : b, without a branch
template <int P>
__device__ __forceinline__ void in_sel(bool c, const typename PairIn<P>::T& a, const typename PairIn<P>::T& b,
                                       typename PairIn<P>::T& o) {
    if constexpr (P == P16) {
#pragma unroll
        for (int k = 0; k < 12; ++k) o.w[k] = c ? a.w[k] : b.w[k];
        o.s = c ? a.s : b.s;
    } else {
#pragma unroll
        for (int k = 0; k < 24; ++k) o.v[k] = c ? a.v[k] : b.v[k];
    }
}

// o += cf (1 -/+ g_mu) U_mu(lsite) x: the hop from the forward neighbour x
template <int P, int Q, typename PF>
__device__ __forceinline__ void hop_fwd(const LatDesc& ld, int mu, int lsite, const typename PairIn<P>::T& x,
                                        typename Tr<P>::acc o[24], typename Tr<P>::acc cf) {
    using A = typename Tr<P>::acc;
    if constexpr (P == P16) {
        uint32_t u[9];
        h2 hc[6], hs[6];
        float w[12];
        PF::project_fwd_h(x.w, hc, hs);
        link_h<Q>(ld, mu, lsite, u);
        mul_u_h(u, hc, hs, w);
        PF::accum(o, w, cf * x.s);
    } else {
        A h[12], u[18], w[12];
        PF::project(x.v, h);
        link<P, Q, A>(ld, mu, lsite, u);
        mul_u(u, h, w);
        PF::accum(o, w, cf);
    }
}

// w = U_mu(lsite)^+ (1 +/- g_mu) x without x's scale, which goes to ws (1
// except for FP16): the hop from the backward neighbour before accumulation.
template <int P, int Q, typename PB>
__device__ __forceinline__ void half_bwd(const LatDesc& ld, int mu, int lsite, const typename PairIn<P>::T& x,
                                         typename Tr<P>::acc w[12], typename Tr<P>::acc& ws) {
    using A = typename Tr<P>::acc;
    if constexpr (P == P16) {
        uint32_t u[9];
        h2 hh[6], hn[6];
        PB::project_bwd_h(x.w, hh, hn);
        link_h<Q>(ld, mu, lsite, u);
        mul_udag_h(u, hh, hn, w);
        ws = x.s;
    } else {
        A h[12], u[18];
        PB::project(x.v, h);
        link<P, Q, A>(ld, mu, lsite, u);
        mul_udag(u, h, w);
        ws = A(1);
    }
}

template <int P, int Q, typename PB>
__device__ __forceinline__ void hop_bwd(const LatDesc& ld, int mu, int lsite, const typename PairIn<P>::T& x,
                                        typename Tr<P>::acc o[24], typename Tr<P>::acc cf) {
    using A = typename Tr<P>::acc;
    A w[12], ws;
    half_bwd<P, Q, PB>(ld, mu, lsite, x, w, ws);
    PB::accum(o, w, cf * ws);
}

template <int P, int Q, int MU, typename PF, typename PB>
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
        typename PairIn<P>::T v;
        in_load<P>(ib, inn, gs, ((size_t)sf << lognr) + r, v);
        hop_fwd<P, Q, PF>(ld, MU, site, v, o, cf);
    }
    {
        typename PairIn<P>::T v;
        in_load<P>(ib, inn, gs, ((size_t)sb << lognr) + r, v);
        hop_bwd<P, Q, PB>(ld, MU, sb, v, o, cb);
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
template <> struct NDots<D_TS> { static constexpr int v = 8; };

// Partial sums of a D_TS launch (t = out, s = the input at the output site):
// (t, s), (t, t), (s, s), (rhat, s) and (rhat, t), from which the omega finish
// forms omega and, for r = s - omega t, (rhat, r) and |r|^2 (so the vector
// update needs no reduction of its own).  rcode: the system's shadow residual
// at this slot (rhat_code).  Each site's 12 terms are summed in A, then added
// to the FP64 sums.
template <typename A>
__device__ __forceinline__ void ts_dots(const A o[24], const A s[24], uint32_t rcode, double acc[8]) {
    A f0 = A(0), f1 = A(0), f2 = A(0), f3 = A(0);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        const A tr = o[2 * k], ti = o[2 * k + 1], sr = s[2 * k], si = s[2 * k + 1];
        f0 = fma_(tr, sr, fma_(ti, si, f0));
        f1 = fma_(tr, si, fma_(-ti, sr, f1));
        f2 = fma_(tr, tr, fma_(ti, ti, f2));
        f3 = fma_(sr, sr, fma_(si, si, f3));
    }
    acc[0] += (double)f0;
    acc[1] += (double)f1;
    acc[2] += (double)f2;
    acc[3] += (double)f3;
    rhat_code_dots<2, A>(rcode, s, o, acc + 4, acc + 6);
}
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

template <int P, int MODE, int ILP, int Q>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(Wpe<P, ILP>::lo, Wpe<P, ILP>::hi)))
k_dslash(Work w, Fld out, Fld in, Fld aux,
                                                const double* __restrict__ diag,
                                                const SysState* __restrict__ st, int mask,
                                                double* __restrict__ part, const uint32_t* __restrict__ rc) {
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
    // With quad-shared links every lane of a valid site runs (the quad must be
    // complete); the system mask then only gates stores and partial sums.
    const bool act = s3 < n3 && mask_ok(mask, st, sys);
    if (Q ? s3 < n3 : act) {
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
            link<P, Q, A>(ld, 3, sb, u);
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
                link<P, Q, A>(ld, 3, site, u);
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
                hop_dir<P, Q, 0, PxM, PxP>(ld, ib, inn, gs, site, c.x, 1, r, w.lognr, o);
                hop_dir<P, Q, 1, PyM, PyP>(ld, ib, inn, gs, site, c.y, sy, r, w.lognr, o);
                hop_dir<P, Q, 2, PzM, PzP>(ld, ib, inn, gs, site, c.z, sz, r, w.lognr, o);
#pragma unroll
                for (int k = 0; k < 12; ++k) bw[k] = bn[k];
                if constexpr (MODE == D_TS) {
                    if (act) ts_dots<A>(o, v, rc[bd.slot_off + slot], acc);
                }
            }
            // A lane whose system is not running (possible only with quad-shared
            // links) computes and stores its own system's result from that
            // system's own fields; those outputs (v, t, r_hi) are recomputed
            // before the system uses them again, so only partial sums are masked.
            if constexpr (MODE == D_RESID) {
                A bv[24];
                load_sp<P, A>(aux.v + (size_t)bd.slot_off * G, nullptr, gs, slot, bv);
#pragma unroll
                for (int k = 0; k < 24; ++k) o[k] = bv[k] - o[k];
            }
            store_sp<P, A, true>(ob, on, gs, slot, o);
            if (act) {
                if constexpr (MODE == D_RHAT) {
                    rhat_code_dots<1, A>(rc[bd.slot_off + slot], o, o, acc, acc);
                } else if constexpr (MODE == D_RESID) {
#pragma unroll
                    for (int k = 0; k < 24; ++k) acc[0] += (double)o[k] * (double)o[k];
                }
            }
        }
    }
    if constexpr (MODE != D_PLAIN) block_partials<ND, 4>(acc, w.nr, part, wg_id);
    });
}

// LDS-staged variant.  A workgroup owns a TX x TY x TZ tile of sites times the
// NR systems of one block (lane = r + NR*(ix + TX*(iy + TY*iz))) and walks t
// as above.  At every slice the lanes publish their centre spinor in LDS, so
// a neighbour inside the tile is read from LDS and only the lanes on a tile
// face load their outside neighbour from memory: per site ~sum_mu 2/T_mu of
// the six spatial neighbour spinors instead of all six.

// One spatial direction of the tiled stencil: forward and backward hop of
// slice-t site `site` (tile coordinate i of extent T = 1 << lt, lattice
// coordinate coord of extent Lm, site stride `stride`, lane stride `ls`).
// Every lane reads its neighbour's LDS entry and issues the memory load; a
// lane whose neighbour is inside the tile points that load at slot 0 of the
// block instead (one address for the whole wave: a broadcast, no traffic),
// and the projected half spinors are selected without branching.
template <int P, typename PR>
__device__ __forceinline__ void fetch_half(bool in_tile, const uint4* __restrict__ ib,
                                           const float* __restrict__ inn, size_t gs, size_t gslot,
                                           const typename LdsVec<typename Tr<P>::acc>::T* sh, int wg, int nl,
                                           typename Tr<P>::acc h[12]) {
    using A = typename Tr<P>::acc;
    A hg[12];
    {
        A g[24];
        load_sp<P, A>(ib, inn, gs, in_tile ? (size_t)0 : gslot, g);
        PR::project(g, hg);
    }
    {
        A l[24];
        lds_get<A>(sh, wg, nl, l);
        PR::project(l, h);
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) h[k] = in_tile ? h[k] : hg[k];
}

template <int P, int Q, int MU, typename PF, typename PB>
__device__ __forceinline__ void hop_tile(const LatDesc& ld, const uint4* __restrict__ ib,
                                         const float* __restrict__ inn, size_t gs,
                                         const typename LdsVec<typename Tr<P>::acc>::T* sh, int wg, int lane,
                                         int site, int coord, int stride, int i, int lt, int ls, int r, int lognr,
                                         typename Tr<P>::acc o[24]) {
    using A = typename Tr<P>::acc;
    const int Lm = ld.L[MU];
    const int T = 1 << lt;
    const bool whole = (T == Lm);  // the tile spans the lattice: wrap-around inside it
    {
        const int sf = (coord == Lm - 1) ? site - (Lm - 1) * stride : site + stride;
        A h[12], u[18], w[12];
        fetch_half<P, PF>(whole || i < T - 1, ib, inn, gs, ((size_t)sf << lognr) + r, sh, wg,
                          (i < T - 1) ? lane + ls : lane - (T - 1) * ls, h);
        link<P, Q, A>(ld, MU, site, u);
        mul_u(u, h, w);
        PF::accum(o, w, A(-0.5));
    }
    {
        const int sb = (coord == 0) ? site + (Lm - 1) * stride : site - stride;
        A h[12], u[18], w[12];
        fetch_half<P, PB>(whole || i > 0, ib, inn, gs, ((size_t)sb << lognr) + r, sh, wg,
                          (i > 0) ? lane - ls : lane + (T - 1) * ls, h);
        link<P, Q, A>(ld, MU, sb, u);
        mul_udag(u, h, w);
        PB::accum(o, w, A(-0.5));
    }
}

// LDS buffers of the tiled stencil: two for 4-byte arithmetic (one barrier
// per slice), one for FP64 (two barriers per slice), 16-byte groups.
// Minimum resident waves per SIMD the tiled stencil is compiled for: 3
// matches the three 48 KiB workgroups that fit a CU's LDS; variants whose
// live state does not fit take fewer rather than spill (FP64 arithmetic
// doubles every register, BF16 needs its rounding temporaries).
template <int P, int MODE> struct TileW {
    // FP32 D_TS keeps eight FP64 partial sums and 24 FP32 centre values live
    // through the slice loop: at three waves it spills 112-144 B per lane and
    // measured no faster, so it takes two; D_RHAT (two partial sums) spills
    // 36-64 B at three and gains 1%.  The packed FP16 forms hold half the input
    // state and take three throughout.
    static constexpr int v = P == P16 ? 3 : P == P32 ? (MODE != D_TS ? 3 : 2) : 1;
};

template <int P> constexpr int tile_nbuf() { return sizeof(typename Tr<P>::acc) == 4 ? 2 : 1; }

template <int P, int MODE, int Q>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(TileW<P, MODE>::v, 8))) k_dslash_tile(Work w, Fld out, Fld in, Fld aux,
                                                     const double* __restrict__ diag,
                                                     const SysState* __restrict__ st, int mask,
                                                     double* __restrict__ part, const uint32_t* __restrict__ rc) {
    using A = typename Tr<P>::acc;
    using V16 = typename LdsVec<A>::T;
    constexpr int G = Tr<P>::G;
    constexpr int ND = NDots<MODE>::v;
    constexpr int NBUF = tile_nbuf<P>();
    constexpr int NG = 24 * (int)sizeof(A) / 16;
    extern __shared__ uint4 lds_dyn[];
    V16* const shb = reinterpret_cast<V16*>(lds_dyn);
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
    const int tx = w.tl[0], ty = w.tl[1], tz = w.tl[2];
    const int ntx = ld.L[0] >> tx, nty = ld.L[1] >> ty, ntz = ld.L[2] >> tz;
    const int ntile3 = ntx * nty * ntz;
    const int j = wgb % ntile3, ch = wgb / ntile3;
    const int t0 = ch * w.tc, t1 = min(Lt, t0 + w.tc);
    const int lane = threadIdx.x;
    const int r = lane & (w.nr - 1);
    int q = lane >> w.lognr;
    const int ix = q & ((1 << tx) - 1);
    q >>= tx;
    const int iy = q & ((1 << ty) - 1);
    const int iz = q >> ty;
    Coord c;
    {
        int jq = j;
        c.x = ((jq % ntx) << tx) + ix;
        jq /= ntx;
        c.y = ((jq % nty) << ty) + iy;
        c.z = ((jq / nty) << tz) + iz;
    }
    const int xyz = c.x + ld.L[0] * (c.y + ld.L[1] * c.z);
    const int sys = bd.sys0 + r;
    const bool act = mask_ok(mask, st, sys);
    const bool run = Q || act;  // quad-shared links need every lane of the quad
    const int lsx = w.nr, lsy = w.nr << tx, lsz = w.nr << (tx + ty);

    double acc[ND];
#pragma unroll
    for (int k = 0; k < ND; ++k) acc[k] = 0.0;
    const A dg = act ? (A)diag[sys] : A(0);

    A bw[12], cv[24];
#pragma unroll
    for (int k = 0; k < 12; ++k) bw[k] = A(0);
#pragma unroll
    for (int k = 0; k < 24; ++k) cv[k] = A(0);
    if (run) {
        const int tb = (t0 == 0) ? Lt - 1 : t0 - 1;
        const int sb = xyz + vxyz * tb;
        A v[24], h[12], u[18];
        load_sp<P, A>(ib, inn, gs, ((size_t)sb << w.lognr) + r, v);
        PtP::project(v, h);
        link<P, Q, A>(ld, 3, sb, u);
        mul_udag(u, h, bw);
        if (t0 == 0 && ld.tsign < 0) {
#pragma unroll
            for (int k = 0; k < 12; ++k) bw[k] = -bw[k];
        }
        load_sp<P, A>(ib, inn, gs, ((size_t)(xyz + vxyz * t0) << w.lognr) + r, cv);
    }
#pragma unroll 1
    for (int t = t0; t < t1; ++t) {
        V16* const sh = shb + (NBUF == 2 ? ((t - t0) & 1) : 0) * NG * w.wg;
        const int site = xyz + vxyz * t;
        const size_t slot = ((size_t)site << w.lognr) + r;
        const bool wrap = (t == Lt - 1);
        // forward-t neighbour (the next slice's centre), in flight during the
        // LDS exchange and the spatial hops
        A nv[24];
        if (run) load_sp<P, A>(ib, inn, gs, ((size_t)(wrap ? xyz : site + vxyz) << w.lognr) + r, nv);
        if (NBUF == 1 && t > t0) __syncthreads();  // the previous slice's LDS reads are done
        lds_put<A>(sh, w.wg, lane, cv);
        __syncthreads();
        if (run) {
            A o[24];
#pragma unroll
            for (int k = 0; k < 24; ++k) o[k] = A(0);
            hop_tile<P, Q, 0, PxM, PxP>(ld, ib, inn, gs, sh, w.wg, lane, site, c.x, 1, ix, tx, lsx, r, w.lognr, o);
            hop_tile<P, Q, 1, PyM, PyP>(ld, ib, inn, gs, sh, w.wg, lane, site, c.y, sy, iy, ty, lsy, r, w.lognr, o);
            hop_tile<P, Q, 2, PzM, PzP>(ld, ib, inn, gs, sh, w.wg, lane, site, c.z, sz, iz, tz, lsz, r, w.lognr, o);
            PtP::accum(o, bw, A(-0.5));
            {
                // centre (re-read from LDS): diagonal term, the next slice's
                // backward term with U_t(x,t), and the forward t hop
                A v[24], h[12], u[18], ww[12];
                lds_get<A>(sh, w.wg, lane, v);
#pragma unroll
                for (int k = 0; k < 24; ++k) o[k] += dg * v[k];
                link<P, Q, A>(ld, 3, site, u);
                PtP::project(v, h);
                mul_udag(u, h, bw);
                PtM::project(nv, h);
                mul_u(u, h, ww);
                PtM::accum(o, ww, (wrap && ld.tsign < 0) ? A(0.5) : A(-0.5));
                if constexpr (MODE == D_TS) {
                    if (act) ts_dots<A>(o, v, rc[bd.slot_off + slot], acc);
                }
            }
#pragma unroll
            for (int k = 0; k < 24; ++k) cv[k] = nv[k];
            // A lane whose system is not running (possible only with quad-shared
            // links) computes and stores its own system's result from that
            // system's own fields; those outputs (v, t, r_hi) are recomputed
            // before the system uses them again, so only partial sums are masked.
            if constexpr (MODE == D_RESID) {
                A bv[24];
                load_sp<P, A>(aux.v + (size_t)bd.slot_off * G, nullptr, gs, slot, bv);
#pragma unroll
                for (int k = 0; k < 24; ++k) o[k] = bv[k] - o[k];
            }
            store_sp<P, A, true>(ob, on, gs, slot, o);
            if (act) {
                if constexpr (MODE == D_RHAT) {
                    rhat_code_dots<1, A>(rc[bd.slot_off + slot], o, o, acc, acc);
                } else if constexpr (MODE == D_RESID) {
#pragma unroll
                    for (int k = 0; k < 24; ++k) acc[0] += (double)o[k] * (double)o[k];
                }
            }
        }
    }
    if constexpr (MODE != D_PLAIN) block_partials<ND, 4>(acc, w.nr, part, wg_id);
    else __syncthreads();  // LDS is reused by the next virtual workgroup
    });
}

// ------------------------------------------------------------------ even-odd

// One hop direction as in hop_dir, reading a one-parity field (HALF: neighbour
// slot = (site >> 1) * NR + r) or a full-layout field.
template <int P, int Q, bool HALF, int MU, typename PF, typename PB>
__device__ __forceinline__ void hop_dir_h(const LatDesc& ld, const uint4* __restrict__ ib,
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
        typename PairIn<P>::T v;
        in_load<P>(ib, inn, gs, ((size_t)(HALF ? (sf >> 1) : sf) << lognr) + r, v);
        hop_fwd<P, Q, PF>(ld, MU, site, v, o, cf);
    }
    {
        typename PairIn<P>::T v;
        in_load<P>(ib, inn, gs, ((size_t)(HALF ? (sb >> 1) : sb) << lognr) + r, v);
        hop_bwd<P, Q, PB>(ld, MU, sb, v, o, cb);
    }
}

// o += hopping term of D at `site`: -1/2 sum_mu [(1-g_mu) U psi(x+mu) + (1+g_mu) U^+ psi(x-mu)]
template <int P, int Q, bool HALF>
__device__ __forceinline__ void hop_all(const LatDesc& ld, const uint4* __restrict__ ib,
                                        const float* __restrict__ inn, size_t gs, int site, const Coord& c, int r,
                                        int lognr, typename Tr<P>::acc o[24]) {
    const int sy = ld.L[0], sz = ld.L[0] * ld.L[1], stt = sz * ld.L[2];
    hop_dir_h<P, Q, HALF, 0, PxM, PxP>(ld, ib, inn, gs, site, c.x, 1, r, lognr, o);
    hop_dir_h<P, Q, HALF, 1, PyM, PyP>(ld, ib, inn, gs, site, c.y, sy, r, lognr, o);
    hop_dir_h<P, Q, HALF, 2, PzM, PzP>(ld, ib, inn, gs, site, c.z, sz, r, lognr, o);
    hop_dir_h<P, Q, HALF, 3, PtM, PtP>(ld, ib, inn, gs, site, c.t, stt, r, lognr, o);
}

// Site of parity `par` ((x+y+z+t) mod 2) with field index cb = site >> 1 (Lx even).
__device__ __forceinline__ int eo_site(const LatDesc& ld, int cb, int par, Coord& c) {
    const int Lxh = ld.L[0] >> 1;
    int q = cb / Lxh;
    const int xh = cb - q * Lxh;
    c.y = q % ld.L[1];
    q /= ld.L[1];
    c.z = q % ld.L[2];
    c.t = q / ld.L[2];
    c.x = 2 * xh + ((c.y + c.z + c.t + par) & 1);
    return c.x + ld.L[0] * (c.y + ld.L[1] * (c.z + ld.L[2] * c.t));
}

template <int MODE> struct NDotsEo { static constexpr int v = NDots<MODE>::v; };

// ------------------------------------------------------------ clover term
// (layout in fs_kernels.h, struct Clv)

// Packed Hermitian 6 x 6 block: entry (i, j), i < j, starts at real 6 + 2 k,
// k its row-major index among the entries above the diagonal.
__host__ __device__ constexpr int herm_off(int i, int j) { return 6 + 2 * (5 * i - i * (i - 1) / 2 + (j - i - 1)); }

// Block blk (0: spins 0-1, 1: spins 2-3) of the packed site idx of a clover
// field starting at base, with plane half-lattice sites per chunk row.
template <int P, typename A>
__device__ __forceinline__ void load_herm(const uint4* __restrict__ base, size_t plane, size_t idx, int blk, A h[36]) {
    if constexpr (P == P64) {
#pragma unroll
        for (int k = 0; k < 18; ++k) {
            const uint4 q = base[(size_t)(18 * blk + k) * plane + idx];
            h[2 * k] = (A)__hiloint2double((int)q.y, (int)q.x);
            h[2 * k + 1] = (A)__hiloint2double((int)q.w, (int)q.z);
        }
    } else {
        static_assert(P == P32, "clover fields are kept in FP64 and FP32");
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const uint4 q = base[(size_t)(9 * blk + k) * plane + idx];
            h[4 * k] = (A)__uint_as_float(q.x);
            h[4 * k + 1] = (A)__uint_as_float(q.y);
            h[4 * k + 2] = (A)__uint_as_float(q.z);
            h[4 * k + 3] = (A)__uint_as_float(q.w);
        }
    }
}

// w = H v for one packed Hermitian block; v and w are 6 complex numbers as (re, im).
template <typename A>
__device__ __forceinline__ void herm6_mul(const A h[36], const A* v, A* w) {
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        A re = h[i] * v[2 * i], im = h[i] * v[2 * i + 1];
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            if (j == i) continue;
            const int o = j > i ? herm_off(i, j) : herm_off(j, i);
            const A hr = h[o], hi = j > i ? h[o + 1] : -h[o + 1];  // H_ij = conj(H_ji)
            re = fma_(hr, v[2 * j], re);
            re = fma_(-hi, v[2 * j + 1], re);
            im = fma_(hr, v[2 * j + 1], im);
            im = fma_(hi, v[2 * j], im);
        }
        w[2 * i] = re;
        w[2 * i + 1] = im;
    }
}

// o <- M o with M the packed site idx of the clover-type field at base.
template <int P, typename A>
__device__ __forceinline__ void clv_mul(const uint4* __restrict__ base, size_t plane, size_t idx, A o[24]) {
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
        A h[36], w[12];
        load_herm<P, A>(base, plane, idx, blk, h);
        herm6_mul(h, o + 12 * blk, w);
#pragma unroll
        for (int k = 0; k < 12; ++k) o[12 * blk + k] = w[k];
    }
}

// Schur operator at an even site idx: o <- (C_e + a) cv - o.
template <int P, typename A>
__device__ __forceinline__ void clv_schur(const LatDesc& ld, size_t idx, A a, const A cv[24], A o[24]) {
    const uint4* base = reinterpret_cast<const uint4*>(ld.clv);  // parity 0 first
    const size_t plane = (size_t)ld.V >> 1;
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
        A h[36], w[12];
        load_herm<P, A>(base, plane, idx, blk, h);
        herm6_mul(h, cv + 12 * blk, w);
#pragma unroll
        for (int k = 0; k < 12; ++k) o[12 * blk + k] = fma_(a, cv[12 * blk + k], w[k]) - o[12 * blk + k];
    }
}

// o <- (C_o + a_sys)^-1 o at an odd site idx.
template <int P, typename A>
__device__ __forceinline__ void clv_inv(const Clv& cl, const LatDesc& ld, int sys, size_t idx, A o[24]) {
    clv_mul<P, A>(cl.inv + cl.off[sys], (size_t)ld.V >> 1, idx, o);
}

// One lane per (field site, rhs) slot of one parity; see launch_dslash_eo.
template <int P, int MODE, int Q>
__global__ void __launch_bounds__(256) k_dslash_eo(Work w, Fld out, Fld in, Fld cen, Fld aux,
                                                   const double* __restrict__ diag,
                                                   const SysState* __restrict__ st, int mask,
                                                   double* __restrict__ part, const uint32_t* __restrict__ rc,
                                                   int par_out) {
    using A = typename Tr<P>::acc;
    constexpr int G = Tr<P>::G;
    constexpr int ND = NDotsEo<MODE>::v;
    for_each_vwg(w, [&](const int wg_id, const int b) {
    const BlockDesc bd = w.blocks[b];
    const LatDesc ld = w.lats[bd.lat];
    const int wgb = wg_id - w.wg_start[b];
    const size_t gs = (size_t)ld.Vf << w.lognr;
    const uint4* ib = in.v + (size_t)bd.slot_off * G;
    const float* inn = in.n ? in.n + bd.slot_off : nullptr;
    uint4* ob = out.v + (size_t)bd.slot_off * G;
    float* on = out.n ? out.n + bd.slot_off : nullptr;
    double acc[ND];
#pragma unroll
    for (int k = 0; k < ND; ++k) acc[k] = 0.0;
    for (int it = 0; it < w.tpw; ++it) {
        const size_t slot = ((size_t)wgb * w.tpw + it) * w.wg + threadIdx.x;
        if (slot >= gs) break;
        const int r = (int)(slot & (size_t)(w.nr - 1));
        const int sys = bd.sys0 + r;
        // quad-shared links need the whole quad; then the mask gates only the dots
        const bool act = mask_ok(mask, st, sys);
        if (!(Q || act)) continue;
        const int cb = (int)(slot >> w.lognr);
        Coord c;
        const int site = eo_site(ld, cb, par_out, c);
        A o[24];
#pragma unroll
        for (int k = 0; k < 24; ++k) o[k] = A(0);
        hop_all<P, Q, true>(ld, ib, inn, gs, site, c, r, w.lognr, o);
        A cv[24];
        if constexpr (MODE != D_HOP) {
            load_sp<P, A>(cen.v + (size_t)bd.slot_off * G, cen.n ? cen.n + bd.slot_off : nullptr, gs, slot, cv);
            const A a = (A)diag[sys];
            const A ia = A(1) / a;
#pragma unroll
            for (int k = 0; k < 24; ++k) o[k] = a * cv[k] - ia * o[k];
        }
        if constexpr (MODE == D_RESID) {
            A bv[24];
            load_sp<P, A>(aux.v + (size_t)bd.slot_off * G, nullptr, gs, slot, bv);
#pragma unroll
            for (int k = 0; k < 24; ++k) o[k] = bv[k] - o[k];
        }
        store_sp<P, A, true>(ob, on, gs, slot, o);
        if (act) {
            if constexpr (MODE == D_RHAT) {
                rhat_code_dots<1, A>(rc[bd.slot_off + slot], o, o, acc, acc);
            } else if constexpr (MODE == D_TS) {
                ts_dots<A>(o, cv, rc[bd.slot_off + slot], acc);
            } else if constexpr (MODE == D_RESID) {
#pragma unroll
                for (int k = 0; k < 24; ++k) acc[0] += (double)o[k] * (double)o[k];
            }
        }
    }
    if constexpr (MODE == D_RHAT || MODE == D_TS || MODE == D_RESID) block_partials<ND, 4>(acc, w.nr, part, wg_id);
    });
}

// The same operator streaming over t.  A workgroup owns wg consecutive
// (column, rhs) slots of one parity class q = (x+y+z) mod 2 of one block and
// walks the output sites of those columns, t = tq, tq+2, ... with
// tq = par_out xor q, through a chunk of tc steps.  All its lanes sit on one
// t-slice at a time, and the forward-t neighbour psi(x, t+1) loaded for output t
// gives, with U_t(x, t+1), the backward-t term of output t+2, carried in
// registers.  Workgroup index within a block: (q, chunk, column tile).
// D_PREP and D_POST (FP64) read or write full-layout fields, whose block
// descriptors are fblocks (the same blocks over V sites): D_PREP reads the
// hop input b and its centres from there, D_POST writes both parities of x
// there and reads b_o from aux.
template <int P, int MODE, int Q, int CLV = 0>
__global__ void __launch_bounds__(256) k_dslash_eo_t(Work w, Fld out, Fld in, Fld cen, Fld aux,
                                                     const double* __restrict__ diag,
                                                     const SysState* __restrict__ st, int mask,
                                                     double* __restrict__ part, const uint32_t* __restrict__ rc,
                                                     int par_out, const BlockDesc* __restrict__ fblocks, Clv cl) {
    using A = typename Tr<P>::acc;
    constexpr int G = Tr<P>::G;
    constexpr int ND = NDotsEo<MODE>::v;
    // D_PREP reads the hop input from the full-layout source, or with the
    // clover term from a one-parity field holding (C_o + a)^-1 b_o
    constexpr bool FULL_IN = MODE == D_PREP && !CLV;
    constexpr bool FULL_OUT = MODE == D_POST;
    static_assert(!(MODE == D_PREP || FULL_OUT) || P == P64, "the even-odd source and reconstruction are FP64");
    static_assert(!CLV || P == P64 || P == P32, "the clover term is kept in FP64 and FP32");
    for_each_vwg(w, [&](const int wg_id, const int b) {
    const BlockDesc bd = w.blocks[b];
    const LatDesc ld = w.lats[bd.lat];
    const int wgb = wg_id - w.wg_start[b];
    const size_t gs = (size_t)ld.Vf << w.lognr;
    const size_t gsf = (size_t)ld.V << w.lognr;   // full-layout fields
    const size_t gsi = FULL_IN ? gsf : gs;         // the hop input
    const long long foff = (MODE == D_PREP || FULL_OUT) ? fblocks[b].slot_off : 0;
    const uint4* ib = in.v + (size_t)(FULL_IN ? foff : bd.slot_off) * G;
    const float* inn = in.n ? in.n + bd.slot_off : nullptr;
    uint4* ob = out.v + (size_t)(FULL_OUT ? foff : bd.slot_off) * G;
    float* on = out.n ? out.n + bd.slot_off : nullptr;
    const int Lx = ld.L[0], Ly = ld.L[1], Lt = ld.L[3];
    const int Lxh = Lx >> 1;
    const int sy = Lx, sz = Lx * Ly, vxyz = sz * ld.L[2];
    const int n3 = (vxyz >> 1) << w.lognr;  // (column, rhs) slots of one class
    const int ntile3 = (n3 + w.wg - 1) / w.wg;
    const int nsteps = Lt >> 1;
    const int nchunk = (nsteps + w.tc - 1) / w.tc;
    const int q = wgb / (ntile3 * nchunk);
    const int rem = wgb - q * (ntile3 * nchunk);
    const int ch = rem / ntile3, jt = rem - ch * ntile3;
    const int s3 = jt * w.wg + threadIdx.x;
    const int k0 = ch * w.tc, k1 = min(nsteps, k0 + w.tc);
    double acc[ND];
#pragma unroll
    for (int k = 0; k < ND; ++k) acc[k] = 0.0;
    const int col = s3 >> w.lognr;
    const int r = s3 & (w.nr - 1);
    const int sys = bd.sys0 + r;
    const bool valid = s3 < n3;
    const bool act = valid && mask_ok(mask, st, sys);
    if (Q ? valid : act) {
        Coord c;
        {
            int qq = col / Lxh;
            const int xh = col - qq * Lxh;
            c.y = qq % Ly;
            c.z = qq / Ly;
            c.x = 2 * xh + ((c.y + c.z + q) & 1);
        }
        const int xyz = c.x + Lx * (c.y + Ly * c.z);
        const int tq = (par_out ^ q) & 1;
        // backward-t term of the first output
        A bw[12];
        {
            const int tf = tq + 2 * k0;
            const int tb = (tf == 0) ? Lt - 1 : tf - 1;
            const int sb = xyz + vxyz * tb;
            A v[24], h[12], u[18];
            load_sp<P, A>(ib, inn, gsi, ((size_t)(FULL_IN ? sb : sb >> 1) << w.lognr) + r, v);
            PtP::project(v, h);
            link<P, Q, A>(ld, 3, sb, u);
            mul_udag(u, h, bw);
            if (tf == 0 && ld.tsign < 0) {
#pragma unroll
                for (int k = 0; k < 12; ++k) bw[k] = -bw[k];
            }
        }
#pragma unroll 1
        for (int k = k0; k < k1; ++k) {
            const int t = tq + 2 * k;
            const int site = xyz + vxyz * t;
            c.t = t;
            const size_t slot = ((size_t)(site >> 1) << w.lognr) + r;
            A o[24];
#pragma unroll
            for (int j = 0; j < 24; ++j) o[j] = A(0);
            A bn[12];  // backward-t term of output t + 2
            {
                const bool wrap = (t == Lt - 1);
                const int sf = wrap ? xyz : site + vxyz;
                A v[24], h[12], u[18], ww[12];
                load_sp<P, A>(ib, inn, gsi, ((size_t)(FULL_IN ? sf : sf >> 1) << w.lognr) + r, v);
                PtM::project(v, h);
                link<P, Q, A>(ld, 3, site, u);
                mul_u(u, h, ww);
                PtM::accum(o, ww, (wrap && ld.tsign < 0) ? A(0.5) : A(-0.5));
                PtP::project(v, h);
                link<P, Q, A>(ld, 3, sf, u);
                mul_udag(u, h, bn);
            }
            PtP::accum(o, bw, A(-0.5));
#pragma unroll
            for (int j = 0; j < 12; ++j) bw[j] = bn[j];
            hop_dir_h<P, Q, !FULL_IN, 0, PxM, PxP>(ld, ib, inn, gsi, site, c.x, 1, r, w.lognr, o);
            hop_dir_h<P, Q, !FULL_IN, 1, PyM, PyP>(ld, ib, inn, gsi, site, c.y, sy, r, w.lognr, o);
            hop_dir_h<P, Q, !FULL_IN, 2, PzM, PzP>(ld, ib, inn, gsi, site, c.z, sz, r, w.lognr, o);
            if constexpr (MODE == D_PREP) {
                // out_e = b_e - D_eo b_o / a; partial |b_e|^2 + |b_o|^2 (b_o at the odd
                // site of the same field index).  The scheduling barriers keep the
                // centre loads after the hop: hoisted above it they overflow the
                // register file.
                const A ia = CLV ? A(1) : A(1) / (A)diag[sys];
                const uint4* bsrc = CLV ? aux.v + (size_t)foff * G : ib;  // the full-layout source
                __builtin_amdgcn_sched_barrier(0);
                {
                    A be[24];
                    load_sp<P, A>(bsrc, nullptr, gsf, ((size_t)site << w.lognr) + r, be);
#pragma unroll
                    for (int j = 0; j < 24; ++j) {
                        if (act) acc[0] += (double)be[j] * (double)be[j];
                        o[j] = be[j] - ia * o[j];
                    }
                }
                store_sp<P, A, true>(ob, on, gs, slot, o);
                __builtin_amdgcn_sched_barrier(0);
                {
                    A bo[24];
                    load_sp<P, A>(bsrc, nullptr, gsf, ((size_t)(site ^ 1) << w.lognr) + r, bo);
#pragma unroll
                    for (int j = 0; j < 24; ++j)
                        if (act) acc[0] += (double)bo[j] * (double)bo[j];
                }
                continue;
            } else if constexpr (MODE == D_POST) {
                // x_o = (b_o - D_oe x_e) / a at this odd site; x_e copied to the even
                // site of the same field index
                const A ia = CLV ? A(1) : A(1) / (A)diag[sys];
                __builtin_amdgcn_sched_barrier(0);
                {
                    A bo[24];
                    load_sp<P, A>(aux.v + (size_t)foff * G, nullptr, gsf, ((size_t)site << w.lognr) + r, bo);
#pragma unroll
                    for (int j = 0; j < 24; ++j) o[j] = ia * (bo[j] - o[j]);
                }
                if constexpr (CLV) clv_inv<P, A>(cl, ld, sys, (size_t)(site >> 1), o);
                store_sp<P, A, true>(ob, nullptr, gsf, ((size_t)site << w.lognr) + r, o);
                __builtin_amdgcn_sched_barrier(0);
                {
                    A xe[24];
                    load_sp<P, A>(ib, inn, gs, slot, xe);
                    store_sp<P, A, true>(ob, nullptr, gsf, ((size_t)(site ^ 1) << w.lognr) + r, xe);
                }
                continue;
            }
            A cv[24];
            if constexpr (MODE != D_HOP) {
                load_sp<P, A>(cen.v + (size_t)bd.slot_off * G, cen.n ? cen.n + bd.slot_off : nullptr, gs, slot, cv);
                const A a = (A)diag[sys];
                if constexpr (CLV) {
                    clv_schur<P, A>(ld, (size_t)(site >> 1), a, cv, o);
                } else {
                    const A ia = A(1) / a;
#pragma unroll
                    for (int j = 0; j < 24; ++j) o[j] = a * cv[j] - ia * o[j];
                }
            } else if constexpr (CLV) {
                clv_inv<P, A>(cl, ld, sys, (size_t)(site >> 1), o);
            }
            if constexpr (MODE == D_RESID) {
                A bv[24];
                load_sp<P, A>(aux.v + (size_t)bd.slot_off * G, nullptr, gs, slot, bv);
#pragma unroll
                for (int j = 0; j < 24; ++j) o[j] = bv[j] - o[j];
            }
            // written once and read by the next launch: non-temporal, so the
            // output stream does not evict the neighbours other lanes still read
            store_sp<P, A, true>(ob, on, gs, slot, o);
            if (act) {
                if constexpr (MODE == D_RHAT) {
                    rhat_code_dots<1, A>(rc[bd.slot_off + slot], o, o, acc, acc);
                } else if constexpr (MODE == D_TS) {
                    ts_dots<A>(o, cv, rc[bd.slot_off + slot], acc);
                } else if constexpr (MODE == D_RESID) {
#pragma unroll
                    for (int j = 0; j < 24; ++j) acc[0] += (double)o[j] * (double)o[j];
                }
            }
        }
    }
    if constexpr (MODE == D_RHAT || MODE == D_TS || MODE == D_RESID || MODE == D_PREP)
        block_partials<ND, 4>(acc, w.nr, part, wg_id);
    });
}

// The even-odd operator over x-pairs with LDS sharing (variant 2 of the
// one-parity plans).  Lane (r, xh, iy, iz) of a workgroup owns the pair of
// columns x = 2 xh, 2 xh + 1 at (y, z) = tile origin + (iy, iz) for system r,
// and walks every t-slice of its chunk.  At slice t one column of the pair
// holds an output site (parity par_out) and the other an input site: the lane
// computes the output, while the input site's spinor sits in LDS, where the
// x/y/z neighbours of the other lanes' outputs read it.  That spinor is the
// lane's forward-t neighbour of slice t-1: loaded once from memory, used for
// the forward-t hop and written to the other LDS buffer for the next slice.
// So every input spinor is read from memory once, plus, for the lanes on a
// y/z face of the tile (TY x TZ pairs; the tile spans all of x), the
// neighbour beyond the face.  The backward-t term of the next slice's output
// (the lane's other column) is formed from the pair's input site and carried
// in registers.  Modes as k_dslash_eo_t (D_HOP, and with par_out = 0 the
// Schur modes).
// One neighbour of the x-pair stencil: from LDS when it is inside the tile,
// else from memory; every lane issues the memory load (interior lanes load
// slot 0, a broadcast) and the value is selected, so the code has no branch.
template <int P>
__device__ __forceinline__ void pair_fetch(bool inside, const uint4* __restrict__ ib, const float* __restrict__ inn,
                                           size_t gs, size_t gslot, const char* sh, int wg, int nl,
                                           typename PairIn<P>::T& v) {
    typename PairIn<P>::T g, l;
    in_load<P>(ib, inn, gs, inside ? (size_t)0 : gslot, g);
    in_get<P>(sh, wg, nl, l);
    in_sel<P>(inside, l, g, v);
}

// One spatial axis of the x-pair stencil: forward and backward hops of the
// output site so (pair field index cb, lattice coordinate c of extent Lm,
// tile coordinate i of extent T, LDS lane stride ls).
template <int P, int Q, int MU, typename PF, typename PB>
__device__ __forceinline__ void pair_hop(const LatDesc& ld, const uint4* __restrict__ ib,
                                         const float* __restrict__ inn, size_t gs, const char* sh, int wg, int lane,
                                         int i, int T, int Lm, int ls, int c, int cb, int cstride, int so,
                                         int sstride, int r, int lognr, typename Tr<P>::acc o[24]) {
    using A = typename Tr<P>::acc;
    const bool whole = T == Lm;  // the tile spans the axis: wrap-around inside it
    {
        const int cbf = (c == Lm - 1) ? cb - (Lm - 1) * cstride : cb + cstride;
        typename PairIn<P>::T v;
        pair_fetch<P>(whole || i < T - 1, ib, inn, gs, ((size_t)cbf << lognr) + r, sh, wg,
                      (i < T - 1) ? lane + ls : lane - (T - 1) * ls, v);
        hop_fwd<P, Q, PF>(ld, MU, so, v, o, A(-0.5));
    }
    {
        const int cbb = (c == 0) ? cb + (Lm - 1) * cstride : cb - cstride;
        const int sb = (c == 0) ? so + (Lm - 1) * sstride : so - sstride;
        typename PairIn<P>::T v;
        pair_fetch<P>(whole || i > 0, ib, inn, gs, ((size_t)cbb << lognr) + r, sh, wg,
                      (i > 0) ? lane - ls : lane + (T - 1) * ls, v);
        hop_bwd<P, Q, PB>(ld, MU, sb, v, o, A(-0.5));
    }
}

template <int P, int MODE, int Q, int CLV = 0>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(TileW<P, MODE>::v, 8)))
k_dslash_eo_pair(Work w, Fld out, Fld in, Fld cen, Fld aux, const double* __restrict__ diag,
                 const SysState* __restrict__ st, int mask, double* __restrict__ part,
                 const uint32_t* __restrict__ rc, int par_out, Clv cl) {
    static_assert(!CLV || P == P64 || P == P32, "the clover term is kept in FP64 and FP32");
    using A = typename Tr<P>::acc;
    using In = typename PairIn<P>::T;
    constexpr int G = Tr<P>::G;
    constexpr int ND = NDotsEo<MODE>::v;
    constexpr int NBUF = tile_nbuf<P>();
    constexpr int LB = in_lds_bytes<P>();
    extern __shared__ uint4 lds_dyn[];
    char* const shb = reinterpret_cast<char*>(lds_dyn);
    for_each_vwg(w, [&](const int wg_id, const int b) {
    const BlockDesc bd = w.blocks[b];
    const LatDesc ld = w.lats[bd.lat];
    const int wgb = wg_id - w.wg_start[b];
    const size_t gs = (size_t)ld.Vf << w.lognr;
    const uint4* ib = in.v + (size_t)bd.slot_off * G;
    const float* inn = in.n ? in.n + bd.slot_off : nullptr;
    uint4* ob = out.v + (size_t)bd.slot_off * G;
    float* on = out.n ? out.n + bd.slot_off : nullptr;
    const int Lx = ld.L[0], Ly = ld.L[1], Lz = ld.L[2], Lt = ld.L[3];
    const int Lxh = Lx >> 1;
    const int TY = ld.pty, TZ = ld.ptz;
    const int nty = Ly / TY;
    const int ntile = nty * (Lz / TZ);
    const int ch = wgb / ntile, jt = wgb - ch * ntile;
    const int t0 = ch * w.tc, t1 = min(Lt, t0 + w.tc);
    const int lane = threadIdx.x;
    const int r = lane & (w.nr - 1);
    int q = lane >> w.lognr;
    const int xh = q % Lxh;
    q /= Lxh;
    const int iy = q % TY, iz = q / TY;
    const bool valid = iz < TZ;  // lanes beyond the tile only join the barriers
    const int y = (jt % nty) * TY + iy, z = (jt / nty) * TZ + iz;
    const int sys = bd.sys0 + r;
    const bool act = valid && mask_ok(mask, st, sys);
    const int vxyzh = Lxh * Ly * Lz;          // field sites of one t-slice
    const int cb0 = xh + Lxh * (y + Ly * z);  // field index at t = 0
    const int ls_y = w.nr * Lxh, ls_z = ls_y * TY;
    const int sy = Lx, sz = Lx * Ly, stt = sz * Lz;
    // x neighbour across the pair boundary: pair xh - 1 when the output column
    // is even, xh + 1 when it is odd (periodic in x; the tile spans all of x)
    const int lxm = xh == 0 ? lane + (Lxh - 1) * w.nr : lane - w.nr;
    const int lxp = xh == Lxh - 1 ? lane - (Lxh - 1) * w.nr : lane + w.nr;

    double acc[ND];
#pragma unroll
    for (int k = 0; k < ND; ++k) acc[k] = 0.0;
    // backward-t term of the next output, U^+ (1 + g4) psi, and its scale
    A bw[12], bws = A(0);
#pragma unroll
    for (int k = 0; k < 12; ++k) bw[k] = A(0);
    if (valid) {
        {
            In e;
            in_load<P>(ib, inn, gs, ((size_t)(cb0 + t0 * vxyzh) << w.lognr) + r, e);
            in_put<P>(shb, w.wg, lane, e);
        }
        // backward-t term of the first output: its column at t0 - 1 is this
        // pair's input site there
        const int tb = t0 == 0 ? Lt - 1 : t0 - 1;
        const int xo0 = 2 * xh + ((y + z + t0 + par_out) & 1);
        In v;
        in_load<P>(ib, inn, gs, ((size_t)(cb0 + tb * vxyzh) << w.lognr) + r, v);
        half_bwd<P, Q, PtP>(ld, 3, xo0 + sy * y + sz * z + stt * tb, v, bw, bws);
        if (t0 == 0 && ld.tsign < 0) bws = -bws;
    }
    __syncthreads();
#pragma unroll 1
    for (int t = t0; t < t1; ++t) {
        const char* const sh = shb + (NBUF == 2 ? ((t - t0) & 1) : 0) * LB * w.wg;   // slice t
        char* const shn = shb + (NBUF == 2 ? ((t - t0 + 1) & 1) : 0) * LB * w.wg;    // slice t + 1
        const bool wrap = t == Lt - 1;
        const int cb = cb0 + t * vxyzh;
        In nxt;
        if (valid) {
            const int par = (y + z + t + par_out) & 1;  // output column 2 xh + par
            const int so = 2 * xh + par + sy * y + sz * z + stt * t;
            const size_t slot = ((size_t)cb << w.lognr) + r;
            A o[24];
#pragma unroll
            for (int k = 0; k < 24; ++k) o[k] = A(0);
            PtP::accum(o, bw, A(-0.5) * bws);
            {  // x: one neighbour is the pair's own input site, the other the next pair's;
               // the own site also gives the next output's backward-t term
                In e, l, v;
                in_get<P>(sh, w.wg, lane, e);
                half_bwd<P, Q, PtP>(ld, 3, so ^ 1, e, bw, bws);
                in_get<P>(sh, w.wg, par ? lxp : lxm, l);
                in_sel<P>(par, l, e, v);
                hop_fwd<P, Q, PxM>(ld, 0, so, v, o, A(-0.5));
                in_sel<P>(par, e, l, v);
                const int xo = 2 * xh + par;
                hop_bwd<P, Q, PxP>(ld, 0, xo == 0 ? so + Lx - 1 : so - 1, v, o, A(-0.5));
            }
            // scheduling barriers keep each axis's loads in its own phase: hoisted
            // together they overflow the register file
            __builtin_amdgcn_sched_barrier(0);
            pair_hop<P, Q, 1, PyM, PyP>(ld, ib, inn, gs, sh, w.wg, lane, iy, TY, Ly, ls_y, y, cb, Lxh, so, sy, r,
                                        w.lognr, o);
            __builtin_amdgcn_sched_barrier(0);
            pair_hop<P, Q, 2, PzM, PzP>(ld, ib, inn, gs, sh, w.wg, lane, iz, TZ, Lz, ls_z, z, cb, Lxh * Ly, so, sz,
                                        r, w.lognr, o);
            __builtin_amdgcn_sched_barrier(0);
            {  // t: forward hop from the pair's input site at t + 1 (the next slice's LDS entry)
                in_load<P>(ib, inn, gs, ((size_t)(wrap ? cb0 : cb + vxyzh) << w.lognr) + r, nxt);
                hop_fwd<P, Q, PtM>(ld, 3, so, nxt, o, (wrap && ld.tsign < 0) ? A(0.5) : A(-0.5));
            }
            if (NBUF == 2) in_put<P>(shn, w.wg, lane, nxt);
            A cv[24];
            if constexpr (MODE != D_HOP) {
                load_sp<P, A>(cen.v + (size_t)bd.slot_off * G, cen.n ? cen.n + bd.slot_off : nullptr, gs, slot, cv);
                const A a = (A)diag[sys];
                if constexpr (CLV) {
                    clv_schur<P, A>(ld, (size_t)cb, a, cv, o);
                } else {
                    const A ia = A(1) / a;
#pragma unroll
                    for (int k = 0; k < 24; ++k) o[k] = a * cv[k] - ia * o[k];
                }
            } else if constexpr (CLV) {
                clv_inv<P, A>(cl, ld, sys, (size_t)cb, o);
            }
            if constexpr (MODE == D_RESID) {
                A bv[24];
                load_sp<P, A>(aux.v + (size_t)bd.slot_off * G, nullptr, gs, slot, bv);
#pragma unroll
                for (int k = 0; k < 24; ++k) o[k] = bv[k] - o[k];
            }
            store_sp<P, A, true>(ob, on, gs, slot, o);
            if (act) {
                if constexpr (MODE == D_RHAT) {
                    rhat_code_dots<1, A>(rc[bd.slot_off + slot], o, o, acc, acc);
                } else if constexpr (MODE == D_TS) {
                    ts_dots<A>(o, cv, rc[bd.slot_off + slot], acc);
                } else if constexpr (MODE == D_RESID) {
#pragma unroll
                    for (int k = 0; k < 24; ++k) acc[0] += (double)o[k] * (double)o[k];
                }
            }
        }
        if (NBUF == 1) {  // one buffer: every read of slice t ends before slice t + 1 is written
            __syncthreads();
            if (valid) in_put<P>(shn, w.wg, lane, nxt);
        }
        __syncthreads();
    }
    if constexpr (MODE == D_RHAT || MODE == D_TS || MODE == D_RESID) block_partials<ND, 4>(acc, w.nr, part, wg_id);
    });
}

// FP64, over a one-parity plan: bh = b_e - D_eo b_o / a; partials |b_e|^2 + |b_o|^2.
// Q: quad-shared links (rhs blocks of 4 or more; the quads of a slot range are whole).
template <int Q>
__global__ void __launch_bounds__(256) k_eo_prep(Work w, const BlockDesc* __restrict__ fblocks, Fld bfull, Fld bh,
                                                 const double* __restrict__ diag, double* __restrict__ part) {
    for_each_vwg(w, [&](const int wg_id, const int b) {
    const BlockDesc bd = w.blocks[b];
    const LatDesc ld = w.lats[bd.lat];
    const int wgb = wg_id - w.wg_start[b];
    const size_t gsh = (size_t)ld.Vf << w.lognr, gsf = (size_t)ld.V << w.lognr;
    const uint4* fb = bfull.v + (size_t)fblocks[b].slot_off * 12;
    uint4* hb = bh.v + (size_t)bd.slot_off * 12;
    double acc[1] = {0.0};
    for (int it = 0; it < w.tpw; ++it) {
        const size_t slot = ((size_t)wgb * w.tpw + it) * w.wg + threadIdx.x;
        if (slot >= gsh) break;
        const int r = (int)(slot & (size_t)(w.nr - 1));
        const int sys = bd.sys0 + r;
        const int cb = (int)(slot >> w.lognr);
        Coord c;
        const int se = eo_site(ld, cb, 0, c);
        const int so = se ^ 1;  // the odd site of the same field index (Lx even)
        double h[24], be[24], bo[24];
#pragma unroll
        for (int k = 0; k < 24; ++k) h[k] = 0.0;
        hop_all<P64, Q, false>(ld, fb, nullptr, gsf, se, c, r, w.lognr, h);
        load_sp<P64, double>(fb, nullptr, gsf, ((size_t)se << w.lognr) + r, be);
        load_sp<P64, double>(fb, nullptr, gsf, ((size_t)so << w.lognr) + r, bo);
        const double ia = 1.0 / diag[sys];
#pragma unroll
        for (int k = 0; k < 24; ++k) {
            acc[0] += be[k] * be[k] + bo[k] * bo[k];
            be[k] -= ia * h[k];
        }
        store_sp<P64, double>(hb, nullptr, gsh, slot, be);
    }
    block_partials<1, 4>(acc, w.nr, part, wg_id);
    });
}

// FP64: x (full layout) = x_e at even sites, (b_o - D_oe x_e) / a at odd sites.
template <int Q>
__global__ void __launch_bounds__(256) k_eo_post(Work w, const BlockDesc* __restrict__ fblocks, Fld bfull, Fld xh,
                                                 Fld xfull, const double* __restrict__ diag) {
    for_each_vwg(w, [&](const int wg_id, const int b) {
    (void)wg_id;
    const BlockDesc bd = w.blocks[b];
    const LatDesc ld = w.lats[bd.lat];
    const int wgb = wg_id - w.wg_start[b];
    const size_t gsh = (size_t)ld.Vf << w.lognr, gsf = (size_t)ld.V << w.lognr;
    const uint4* fb = bfull.v + (size_t)fblocks[b].slot_off * 12;
    uint4* fx = xfull.v + (size_t)fblocks[b].slot_off * 12;
    const uint4* hx = xh.v + (size_t)bd.slot_off * 12;
    for (int it = 0; it < w.tpw; ++it) {
        const size_t slot = ((size_t)wgb * w.tpw + it) * w.wg + threadIdx.x;
        if (slot >= gsh) break;
        const int r = (int)(slot & (size_t)(w.nr - 1));
        const int sys = bd.sys0 + r;
        const int cb = (int)(slot >> w.lognr);
        Coord c;
        const int so = eo_site(ld, cb, 1, c);
        const int se = so ^ 1;
        double h[24], bo[24], xe[24];
#pragma unroll
        for (int k = 0; k < 24; ++k) h[k] = 0.0;
        hop_all<P64, Q, true>(ld, hx, nullptr, gsh, so, c, r, w.lognr, h);
        load_sp<P64, double>(fb, nullptr, gsf, ((size_t)so << w.lognr) + r, bo);
        load_sp<P64, double>(hx, nullptr, gsh, slot, xe);
        const double ia = 1.0 / diag[sys];
#pragma unroll
        for (int k = 0; k < 24; ++k) bo[k] = ia * (bo[k] - h[k]);
        store_sp<P64, double>(fx, nullptr, gsf, ((size_t)se << w.lognr) + r, xe);
        store_sp<P64, double>(fx, nullptr, gsf, ((size_t)so << w.lognr) + r, bo);
    }
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

// Link-load variant of a launch (the Q of link()): 0 for rhs blocks of 1 or
// 2, else 1, or 2 where the plan's FP32 links keep two rows.
template <int P>
static int qmode(const Work& w) { return w.nr < 4 ? 0 : (P == P32 && w.two_rows) ? 2 : 1; }

template <int P, int MODE, int CLV = 0>
static void launch_eo_q(const Work& w, Fld out, Fld in, Fld cen, Fld aux, const double* diag, const SysState* st,
                        int mask, double* part, hipStream_t s, const uint32_t* rc, int par_out,
                        Clv cl = Clv()) {
    const int q = qmode<P>(w);
    if (w.tc > 0 && w.ilp == 2) {  // x-pair stencil mapping with LDS sharing
        const size_t need = (size_t)tile_nbuf<P>() * in_lds_bytes<P>() * w.wg;
        const size_t lds = std::max(need, lds_cap(w.wg, w.occ));
        switch (q) {
            case 2:
                if constexpr (P == P32)
                    hipLaunchKernelGGL((k_dslash_eo_pair<P, MODE, 2, CLV>), dim3(grid_of(w)), dim3(w.wg), lds, s, w, out,
                                       in, cen, aux, diag, st, mask, part, rc, par_out, cl);
                break;
            case 1:
                hipLaunchKernelGGL((k_dslash_eo_pair<P, MODE, 1, CLV>), dim3(grid_of(w)), dim3(w.wg), lds, s, w, out, in,
                                   cen, aux, diag, st, mask, part, rc, par_out, cl);
                break;
            default:
                hipLaunchKernelGGL((k_dslash_eo_pair<P, MODE, 0, CLV>), dim3(grid_of(w)), dim3(w.wg), lds, s, w, out, in,
                                   cen, aux, diag, st, mask, part, rc, par_out, cl);
        }
        return;
    }
    if (w.tc > 0) {  // stencil mapping: t-streaming, with the plan's residency cap
        const size_t lds = lds_cap(w.wg, w.occ);
        switch (q) {
            case 2:
                if constexpr (P == P32)
                    hipLaunchKernelGGL((k_dslash_eo_t<P, MODE, 2, CLV>), dim3(grid_of(w)), dim3(w.wg), lds, s, w, out, in,
                                       cen, aux, diag, st, mask, part, rc, par_out, nullptr, cl);
                break;
            case 1:
                hipLaunchKernelGGL((k_dslash_eo_t<P, MODE, 1, CLV>), dim3(grid_of(w)), dim3(w.wg), lds, s, w, out, in, cen,
                                   aux, diag, st, mask, part, rc, par_out, nullptr, cl);
                break;
            default:
                hipLaunchKernelGGL((k_dslash_eo_t<P, MODE, 0, CLV>), dim3(grid_of(w)), dim3(w.wg), lds, s, w, out, in, cen,
                                   aux, diag, st, mask, part, rc, par_out, nullptr, cl);
        }
        return;
    }
    if constexpr (!CLV) {  // one-parity stencil work with the clover term always walks t (tc > 0)
        switch (q) {
            case 2:
                if constexpr (P == P32)
                    hipLaunchKernelGGL((k_dslash_eo<P, MODE, 2>), dim3(grid_of(w)), dim3(w.wg), 0, s, w, out, in, cen,
                                       aux, diag, st, mask, part, rc, par_out);
                break;
            case 1:
                hipLaunchKernelGGL((k_dslash_eo<P, MODE, 1>), dim3(grid_of(w)), dim3(w.wg), 0, s, w, out, in, cen, aux,
                                   diag, st, mask, part, rc, par_out);
                break;
            default:
                hipLaunchKernelGGL((k_dslash_eo<P, MODE, 0>), dim3(grid_of(w)), dim3(w.wg), 0, s, w, out, in, cen, aux,
                                   diag, st, mask, part, rc, par_out);
        }
    }
}

}  // namespace fs
