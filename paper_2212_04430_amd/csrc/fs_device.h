// Device-side building blocks for the FS-MLMC kernels (gfx950, wave64).
//
// Field layout in HBM ("block" AoSoA).  A block holds NR systems (right-hand
// sides) on one lattice of V sites.  A spinor field of a block is
//     [group g][site][r]          r = 0..NR-1 fastest
// where a group is 16 bytes of the spinor's 24 reals (component order
// c = spin*3 + colour, re/im interleaved):
//     FP64: 1 complex per group, 12 groups
//     FP32: 2 complex per group,  6 groups
//     FP16: 4 complex per group,  3 groups  + one float scale per (site, r)
//     BF16: 4 complex per group,  3 groups
// so lane (site, r) issues 16-byte loads and a wave reads contiguous memory.
// Gauge links of one lattice: [mu][k = row*3 + col][site] complex in the
// storage precision (16, 8, 4, 4 bytes per complex).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fs {

enum Prec : int { P64 = 0, P32 = 1, P16 = 2, PBF = 3 };

// ----------------------------------------------------------- descriptors

struct LatDesc {
    int L[4];          // Lx, Ly, Lz, Lt
    int V;             // sites (links are indexed by site)
    int Vf;            // sites of a field: V, or V/2 for even-odd (one-parity) fields
    int eo;            // 1: fields hold one parity, field site = site >> 1
    int tsign;         // +1 periodic, -1 antiperiodic in t
    const void* gauge; // links in the launch's storage precision, [mu][9][site]
    const void* gauge_q; // the same links site-major, [mu][site][link_q_bytes], or
                         // rows 0-1 only ([mu][site][QCR], FP32) in plans that rebuild row 2
    int pty, ptz;        // one-parity plans with the x-pair stencil: tile of TY x TZ pairs
                         // (dividing Ly, Lz) per workgroup; 0 otherwise
    const void* clv;     // clover term C of the lattice in the launch precision (FP64 or
                         // FP32), [parity][chunk][V/2] packed Hermitian blocks; null: none
};

struct BlockDesc {
    int lat;            // index into the lattice table
    int sys0;           // first system id (per-system arrays are indexed sys0 + r)
    long long slot_off; // offset of this block in slot units (site*NR + r)
};

// ----------------------------------------------------------- scalars

__device__ __forceinline__ float bf16_to_f(uint16_t h) {
    return __uint_as_float(((uint32_t)h) << 16);
}
__device__ __forceinline__ uint16_t f_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);  // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float h_to_f(uint16_t h) {
    _Float16 v;
    __builtin_memcpy(&v, &h, 2);
    return (float)v;
}
__device__ __forceinline__ uint16_t f_to_h(float f) {
    _Float16 v = (_Float16)f;
    uint16_t h;
    __builtin_memcpy(&h, &v, 2);
    return h;
}

// ----------------------------------------------------------- precision traits

template <int P> struct Tr;
template <> struct Tr<P64> {
    using acc = double;
    static constexpr int G = 12;   // 16-byte groups per spinor
    static constexpr int GB = 16;  // bytes per stored link complex
    static constexpr int SB = 192; // spinor bytes (without scale)
    static constexpr int QC = 9;   // 16-byte chunks per site-major link (144 B)
};
template <> struct Tr<P32> {
    using acc = float;
    static constexpr int G = 6;
    static constexpr int GB = 8;
    static constexpr int SB = 96;
    static constexpr int QC = 5;   // 72 B padded to 80 B
    static constexpr int QCR = 3;  // rows 0-1 only: 48 B
};
template <> struct Tr<P16> {
    using acc = float;
    static constexpr int G = 3;
    static constexpr int GB = 4;
    static constexpr int SB = 48;
};
template <> struct Tr<PBF> {
    using acc = float;
    static constexpr int G = 3;
    static constexpr int GB = 4;
    static constexpr int SB = 48;
};

// Bytes per site-major link (gauge_q): FP64 and FP32 as 16-byte chunks (the
// FP32 tail padded), FP16 and BF16 as nine packed complex words, unpadded.
template <int P> constexpr uint32_t link_q_bytes() {
    if constexpr (P == P64 || P == P32) return 16u * Tr<P>::QC;
    else return 36u;
}

// Link loads go through raw buffer instructions: a 128-bit resource holds a
// wave-uniform base address and extent (scalar registers), each lane supplies
// a 32-bit byte offset and a uniform offset selects the link component, so the
// addressing costs no per-lane 64-bit arithmetic and the loads are not
// generic (flat) accesses.  A lattice's links of one direction (nine complex
// planes) must stay below 4 GiB, which fs_create checks.  Spinor fields, which
// the vector kernels update in place, use plain global pointers.
constexpr int kBufFlags = 0x00020000;  // raw 32-bit data format (gfx9 family)

// Bases and extents come from per-block tables in ordinary memory, which the
// compiler cannot prove uniform; they are uniform over the workgroup by
// construction, so they are moved to scalar registers explicitly.
__device__ __forceinline__ uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// a * b + c with one rounding (an explicit multiply-add, so a chain of them
// is not split into products and separate additions)
__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, uint32_t bytes) {
    const uint64_t p = reinterpret_cast<uint64_t>(base);
    const uint64_t q = ((uint64_t)uni((uint32_t)(p >> 32)) << 32) | uni((uint32_t)p);
    return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(q), (short)0, (int)uni(bytes), kBufFlags);
}

// 16-byte group load / store, optionally with the non-temporal hint (data
// touched once by the launch: it streams through the caches instead of
// displacing lines that other lanes will read again).
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ __forceinline__ uint4 ld16(const uint4* p) {
    if constexpr (NT) {
        const u32x4_t v = __builtin_nontemporal_load(reinterpret_cast<const u32x4_t*>(p));
        return make_uint4(v.x, v.y, v.z, v.w);
    } else {
        return *p;
    }
}

template <bool NT>
__device__ __forceinline__ void st16(uint4* p, uint4 v) {
    if constexpr (NT) {
        const u32x4_t u = {v.x, v.y, v.z, v.w};
        __builtin_nontemporal_store(u, reinterpret_cast<u32x4_t*>(p));
    } else {
        *p = v;
    }
}

__device__ __forceinline__ uint4 pack_d(double re, double im) {
    return make_uint4((uint32_t)__double2loint(re), (uint32_t)__double2hiint(re), (uint32_t)__double2loint(im),
                      (uint32_t)__double2hiint(im));
}

// Load / store the 24 reals of spinor (slot) from a block base.  gs = group
// stride in 16-byte units (= V * NR).  `nrm` is the FP16 per-slot scale array.
// NT: non-temporal accesses (see ld16).
template <int P, typename A, bool NT = false>
__device__ __forceinline__ void load_sp(const uint4* __restrict__ base, const float* __restrict__ nrm,
                                        size_t gs, size_t slot, A v[24]) {
    if constexpr (P == P64) {
#pragma unroll
        for (int g = 0; g < 12; ++g) {
            const uint4 d = ld16<NT>(base + g * gs + slot);
            v[2 * g] = (A)__hiloint2double((int)d.y, (int)d.x);
            v[2 * g + 1] = (A)__hiloint2double((int)d.w, (int)d.z);
        }
    } else if constexpr (P == P32) {
#pragma unroll
        for (int g = 0; g < 6; ++g) {
            const uint4 d = ld16<NT>(base + g * gs + slot);
            v[4 * g] = (A)__uint_as_float(d.x);
            v[4 * g + 1] = (A)__uint_as_float(d.y);
            v[4 * g + 2] = (A)__uint_as_float(d.z);
            v[4 * g + 3] = (A)__uint_as_float(d.w);
        }
    } else {
        float s = 1.0f;
        if constexpr (P == P16) s = nrm[slot];
#pragma unroll
        for (int g = 0; g < 3; ++g) {
            uint4 d = ld16<NT>(base + g * gs + slot);
            uint32_t w[4] = {d.x, d.y, d.z, d.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                float lo, hi;
                if constexpr (P == P16) {
                    lo = h_to_f((uint16_t)(w[k] & 0xffff)) * s;
                    hi = h_to_f((uint16_t)(w[k] >> 16)) * s;
                } else {
                    lo = bf16_to_f((uint16_t)(w[k] & 0xffff));
                    hi = bf16_to_f((uint16_t)(w[k] >> 16));
                }
                v[8 * g + 2 * k] = (A)lo;
                v[8 * g + 2 * k + 1] = (A)hi;
            }
        }
    }
}

template <int P, typename A, bool NT = false>
__device__ __forceinline__ void store_sp(uint4* __restrict__ base, float* __restrict__ nrm,
                                         size_t gs, size_t slot, const A v[24]) {
    if constexpr (P == P64) {
#pragma unroll
        for (int g = 0; g < 12; ++g) st16<NT>(base + g * gs + slot, pack_d((double)v[2 * g], (double)v[2 * g + 1]));
    } else if constexpr (P == P32) {
#pragma unroll
        for (int g = 0; g < 6; ++g)
            st16<NT>(base + g * gs + slot,
                     make_uint4(__float_as_uint((float)v[4 * g]), __float_as_uint((float)v[4 * g + 1]),
                                __float_as_uint((float)v[4 * g + 2]), __float_as_uint((float)v[4 * g + 3])));
    } else {
        float inv = 1.0f;
        if constexpr (P == P16) {
            float m = 0.0f;
#pragma unroll
            for (int k = 0; k < 24; ++k) m = fmaxf(m, fabsf((float)v[k]));
            nrm[slot] = m;
            inv = m > 0.0f ? 1.0f / m : 0.0f;
        }
#pragma unroll
        for (int g = 0; g < 3; ++g) {
            uint32_t w[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                float lo = (float)v[8 * g + 2 * k], hi = (float)v[8 * g + 2 * k + 1];
                if constexpr (P == P16) {
                    w[k] = (uint32_t)f_to_h(lo * inv) | ((uint32_t)f_to_h(hi * inv) << 16);
                } else {
                    w[k] = (uint32_t)f_to_bf16(lo) | ((uint32_t)f_to_bf16(hi) << 16);
                }
            }
            st16<NT>(base + g * gs + slot, make_uint4(w[0], w[1], w[2], w[3]));
        }
    }
}

// The value a spinor takes after store_sp followed by load_sp, computed in
// registers (the same conversions, no memory round trip).
template <int P, typename A>
__device__ __forceinline__ void round_sp(A v[24]) {
    if constexpr (P == P64) {
        return;
    } else if constexpr (P == P32) {
#pragma unroll
        for (int k = 0; k < 24; ++k) v[k] = (A)(float)v[k];
    } else if constexpr (P == P16) {
        float m = 0.0f;
#pragma unroll
        for (int k = 0; k < 24; ++k) m = fmaxf(m, fabsf((float)v[k]));
        const float inv = m > 0.0f ? 1.0f / m : 0.0f;
#pragma unroll
        for (int k = 0; k < 24; ++k) v[k] = (A)(h_to_f(f_to_h((float)v[k] * inv)) * m);
    } else {
#pragma unroll
        for (int k = 0; k < 24; ++k) v[k] = (A)bf16_to_f(f_to_bf16((float)v[k]));
    }
}

// Load link U_mu(site) as 18 reals (row-major complex).  Links are stored
// [mu][k = row*3+col][site], one complex per (k, site).
template <int P, typename A>
__device__ __forceinline__ void load_link(const void* __restrict__ gauge, int V, int mu, int site, A u[18]) {
    constexpr uint32_t ES = P == P64 ? 16u : (P == P32 ? 8u : 4u);  // bytes per complex
    const uint32_t plane = uni((uint32_t)V * ES);
    const auto rs = buf_rsrc(reinterpret_cast<const char*>(gauge) + (size_t)mu * 9 * plane, 9 * plane);
    const uint32_t off = (uint32_t)site * ES;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        if constexpr (P == P64) {
            const auto q = __builtin_amdgcn_raw_buffer_load_b128(rs, off, k * plane, 0);
            u[2 * k] = (A)__hiloint2double((int)q[1], (int)q[0]);
            u[2 * k + 1] = (A)__hiloint2double((int)q[3], (int)q[2]);
        } else if constexpr (P == P32) {
            const auto q = __builtin_amdgcn_raw_buffer_load_b64(rs, off, k * plane, 0);
            u[2 * k] = (A)__uint_as_float(q[0]);
            u[2 * k + 1] = (A)__uint_as_float(q[1]);
        } else {
            const uint32_t w = __builtin_amdgcn_raw_buffer_load_b32(rs, off, k * plane, 0);
            if constexpr (P == P16) {
                u[2 * k] = (A)h_to_f((uint16_t)(w & 0xffff));
                u[2 * k + 1] = (A)h_to_f((uint16_t)(w >> 16));
            } else {
                u[2 * k] = (A)bf16_to_f((uint16_t)(w & 0xffff));
                u[2 * k + 1] = (A)bf16_to_f((uint16_t)(w >> 16));
            }
        }
    }
}

// Quad-shared link load.  When the four lanes of a quad hold four systems of
// the same site (rhs blocks of 4 or more), each lane loads one 16-byte chunk of
// the site-major link, so a quad reads one contiguous window per instruction,
// and the chunks are exchanged inside the quad with DPP broadcasts.  All four
// lanes of the quad must be active.  (With the [mu][9][site] layout every link
// costs the cache one access per quad for each of its nine components.)  One
// direction's site-major links must stay below 4 GiB (fs_create's limit).
template <int J>
__device__ __forceinline__ uint32_t quad_bcast(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, J * 0x55, 0xF, 0xF, false);
}

template <int J>
__device__ __forceinline__ void chunk_bcast(const uint4& c, uint32_t o[4]) {
    o[0] = quad_bcast<J>(c.x);
    o[1] = quad_bcast<J>(c.y);
    o[2] = quad_bcast<J>(c.z);
    o[3] = quad_bcast<J>(c.w);
}

// Nine 32-bit words at byte offset off of rs, shared by a quad: lanes 0-2 load
// three each (lane 3 repeats lane 2's), every lane receives all nine.
__device__ __forceinline__ void load_words9_q(__amdgpu_buffer_rsrc_t rs, uint32_t off, int qd, uint32_t w[9]) {
    const auto q = __builtin_amdgcn_raw_buffer_load_b96(rs, off + 12u * (uint32_t)(qd < 2 ? qd : 2), 0, 0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        w[k] = quad_bcast<0>(q[k]);
        w[3 + k] = quad_bcast<1>(q[k]);
        w[6 + k] = quad_bcast<2>(q[k]);
    }
}

// Row 2 of a special unitary 3x3 matrix from rows 0 and 1: the complex
// conjugate of their cross product, U_2j = conj(U_0k U_1l - U_0l U_1k) with
// (j, k, l) a cyclic permutation of (0, 1, 2).  u holds the matrix row-major
// as (re, im) pairs; u[12..17] is overwritten.
template <typename A>
__device__ __forceinline__ void su3_third_row(A u[18]) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int k = (j + 1) % 3, l = (j + 2) % 3;
        const A akr = u[2 * k], aki = u[2 * k + 1], alr = u[2 * l], ali = u[2 * l + 1];
        const A bkr = u[6 + 2 * k], bki = u[7 + 2 * k], blr = u[6 + 2 * l], bli = u[7 + 2 * l];
        // re = akr blr - aki bli - alr bkr + ali bki, -im = -(akr bli + aki blr - alr bki - ali bkr),
        // each one multiply-add chain
        A re = akr * blr;
        re = fma_(-aki, bli, re);
        re = fma_(-alr, bkr, re);
        re = fma_(ali, bki, re);
        A nim = -akr * bli;
        nim = fma_(-aki, blr, nim);
        nim = fma_(alr, bki, nim);
        nim = fma_(ali, bkr, nim);
        u[12 + 2 * j] = re;
        u[13 + 2 * j] = nim;
    }
}

// Two-row form of the quad-shared load (FP32 storage): rows 0 and 1 are
// three 16-byte chunks per site, lanes 0-2 of the quad load one each (lane 3
// repeats chunk 2), and row 2 is rebuilt with su3_third_row.  This trades 24
// bytes of link traffic per load for about 40 FP32 operations per lane; the
// FP16 and BF16 stencils, whose links are smaller and whose lanes already
// spend more instructions on conversions, read whole links.
template <int P, typename A>
__device__ __forceinline__ void load_link_q2(const void* __restrict__ gauge_q, int V, int mu, int site, A u[18]) {
    static_assert(P == P32, "only FP32 links are kept in the two-row form");
    constexpr uint32_t QB = 16u * Tr<P>::QCR;  // bytes per site
    const int qd = threadIdx.x & 3;
    const uint32_t plane = uni((uint32_t)V * QB);
    const auto rs = buf_rsrc(reinterpret_cast<const char*>(gauge_q) + (size_t)mu * plane, plane);
    const uint32_t off = (uint32_t)site * QB;
    const auto q = __builtin_amdgcn_raw_buffer_load_b128(rs, off + 16u * (qd < 2 ? qd : 2), 0, 0);
    const uint4 c = make_uint4(q[0], q[1], q[2], q[3]);
    uint32_t w[12];
    chunk_bcast<0>(c, w + 0);
    chunk_bcast<1>(c, w + 4);
    chunk_bcast<2>(c, w + 8);
#pragma unroll
    for (int k = 0; k < 12; ++k) u[k] = (A)__uint_as_float(w[k]);
    su3_third_row<A>(u);
}

template <int P, typename A>
__device__ __forceinline__ void load_link_q(const void* __restrict__ gauge_q, int V, int mu, int site, A u[18]) {
    constexpr uint32_t QB = link_q_bytes<P>();  // bytes per site
    const int qd = threadIdx.x & 3;
    const uint32_t plane = uni((uint32_t)V * QB);
    const auto rs = buf_rsrc(reinterpret_cast<const char*>(gauge_q) + (size_t)mu * plane, plane);
    const uint32_t off = (uint32_t)site * QB;
    if constexpr (P == P64) {
        // chunks 0-7 shared (two rounds), chunk 8 loaded by every lane
        const auto q0 = __builtin_amdgcn_raw_buffer_load_b128(rs, off + 16u * qd, 0, 0);
        const auto q1 = __builtin_amdgcn_raw_buffer_load_b128(rs, off + 16u * (4 + qd), 0, 0);
        const auto q8 = __builtin_amdgcn_raw_buffer_load_b128(rs, off + 128u, 0, 0);
        const uint4 c0 = make_uint4(q0[0], q0[1], q0[2], q0[3]);
        const uint4 c1 = make_uint4(q1[0], q1[1], q1[2], q1[3]);
        uint32_t w[36];
        chunk_bcast<0>(c0, w + 0);
        chunk_bcast<1>(c0, w + 4);
        chunk_bcast<2>(c0, w + 8);
        chunk_bcast<3>(c0, w + 12);
        chunk_bcast<0>(c1, w + 16);
        chunk_bcast<1>(c1, w + 20);
        chunk_bcast<2>(c1, w + 24);
        chunk_bcast<3>(c1, w + 28);
        w[32] = q8[0]; w[33] = q8[1]; w[34] = q8[2]; w[35] = q8[3];
#pragma unroll
        for (int k = 0; k < 18; ++k) u[k] = (A)__hiloint2double((int)w[2 * k + 1], (int)w[2 * k]);
    } else if constexpr (P == P32) {
        // chunks 0-3 shared, the last complex (chunk 4) loaded by every lane
        const auto q = __builtin_amdgcn_raw_buffer_load_b128(rs, off + 16u * qd, 0, 0);
        const auto t = __builtin_amdgcn_raw_buffer_load_b64(rs, off + 64u, 0, 0);
        const uint4 c = make_uint4(q[0], q[1], q[2], q[3]);
        uint32_t w[18];
        chunk_bcast<0>(c, w + 0);
        chunk_bcast<1>(c, w + 4);
        chunk_bcast<2>(c, w + 8);
        chunk_bcast<3>(c, w + 12);
        w[16] = t[0]; w[17] = t[1];
#pragma unroll
        for (int k = 0; k < 18; ++k) u[k] = (A)__uint_as_float(w[k]);
    } else {
        uint32_t w[9];
        load_words9_q(rs, off, qd, w);
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            if constexpr (P == P16) {
                u[2 * k] = (A)h_to_f((uint16_t)(w[k] & 0xffff));
                u[2 * k + 1] = (A)h_to_f((uint16_t)(w[k] >> 16));
            } else {
                u[2 * k] = (A)bf16_to_f((uint16_t)(w[k] & 0xffff));
                u[2 * k + 1] = (A)bf16_to_f((uint16_t)(w[k] >> 16));
            }
        }
    }
}

// Link load of the stencil, by variant Q: 0 one component per load (rhs
// blocks of 1 or 2), 1 quad-shared whole links, 2 quad-shared rows 0-1 with
// row 2 rebuilt (FP32; every lattice of the plan holds special unitary links).
template <int P, int Q, typename A>
__device__ __forceinline__ void link(const LatDesc& ld, int mu, int site, A u[18]) {
    if constexpr (Q == 2) load_link_q2<P, A>(ld.gauge_q, ld.V, mu, site, u);
    else if constexpr (Q == 1) load_link_q<P, A>(ld.gauge_q, ld.V, mu, site, u);
    else load_link<P, A>(ld.gauge, ld.V, mu, site, u);
}

// ----------------------------------------------------------- lattice geometry

struct Coord {
    int x, y, z, t;
};

__device__ __forceinline__ Coord coords(int site, const LatDesc& ld) {
    Coord c;
    int s = site;
    c.x = s % ld.L[0];
    s /= ld.L[0];
    c.y = s % ld.L[1];
    s /= ld.L[1];
    c.z = s % ld.L[2];
    c.t = s / ld.L[2];
    return c;
}

// ----------------------------------------------------------- work mapping

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2);
// remap so that XCD k receives a contiguous range of logical workgroups and
// neighbouring tiles of the stencil share one L2.
__device__ __forceinline__ int xcd_remap(int wg, int n_wg) {
    const int nx = 8;
    int per = (n_wg + nx - 1) / nx;
    return (wg % nx) * per + wg / nx;
}

// First index b with start[b+1] > w (start is non-decreasing, start[0] = 0).
__device__ __forceinline__ int find_block(const int* __restrict__ start, int nblk, int w) {
    int lo = 0, hi = nblk - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= w) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// ----------------------------------------------------------- reductions

// Sum `ND` doubles per rhs over the workgroup (lanes with equal r = lane % NR)
// in a fixed order and write them to part[(wg*ND + k)*NR + r].  At most MAXW
// waves per workgroup and NR <= 16.
template <int ND, int MAXW>
__device__ __forceinline__ void block_partials(double (&v)[ND], int nr, double* __restrict__ part, int wg) {
    __shared__ double red[MAXW][ND * 16];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nwave = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < ND; ++k) {
        double x = v[k];
        for (int off = 32; off >= nr; off >>= 1) x += __shfl_xor(x, off, 64);
        v[k] = x;
    }
    if (lane < nr) {
#pragma unroll
        for (int k = 0; k < ND; ++k) red[wave][k * nr + lane] = v[k];
    }
    __syncthreads();
    const int nq = ND * nr;
    for (int q = threadIdx.x; q < nq; q += blockDim.x) {
        double s = 0.0;
        for (int w = 0; w < nwave; ++w) s += red[w][q];
        part[(size_t)wg * nq + q] = s;
    }
    __syncthreads();  // red[] is reused by the next virtual workgroup of a persistent launch
}

// Reduce part rows [w0, w1) of width nq into out[q] (shared), fixed order.
// Must be called by all threads of a 256-thread workgroup.
__device__ __forceinline__ void reduce_rows(const double* __restrict__ part, int nq, int w0, int w1,
                                            double* __restrict__ out /* shared, nq */) {
    __shared__ double tmp[256];
    const int T = blockDim.x;
    for (int q0 = 0; q0 < nq; q0 += T) {
        int nqc = min(T, nq - q0);
        int nqp = 1;
        while (nqp < nqc) nqp <<= 1;
        int C = T / nqp;
        int q = threadIdx.x % nqp;
        int c = threadIdx.x / nqp;
        int cnt = w1 - w0;
        double s = 0.0;
        if (q < nqc && c < C) {
            int a = w0 + (int)((long long)cnt * c / C);
            int b = w0 + (int)((long long)cnt * (c + 1) / C);
            for (int w = a; w < b; ++w) s += part[(size_t)w * nq + q0 + q];
        }
        tmp[threadIdx.x] = s;
        __syncthreads();
        if (threadIdx.x < nqc) {
            double t = 0.0;
            for (int cc = 0; cc < C; ++cc) t += tmp[cc * nqp + threadIdx.x];
            out[q0 + threadIdx.x] = t;
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------- Philox4x64-10

struct U64x4 {
    uint64_t v[4];
};

__device__ __forceinline__ U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    U64x4 o;
    o.v[0] = c0;
    o.v[1] = c1;
    o.v[2] = c2;
    o.v[3] = c3;
    return o;
}

}  // namespace fs
