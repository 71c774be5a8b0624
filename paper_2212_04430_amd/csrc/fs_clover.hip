// Clover term: construction of C from the links, the per-shift inverses of
// C + a at the odd sites, and the even-odd launches that apply them
// (conventions in fs_clover.h).
#include <stdexcept>

#include "fs_clover.h"
#include "fs_stencil.h"

namespace fs {

namespace {

// 3 x 3 complex matrices as 18 reals, row-major (re, im).
__device__ __forceinline__ void m3_mul(const double* a, const double* b, double* c, bool dag_a, bool dag_b) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double re = 0.0, im = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                // (a)_ik or conj(a_ki); (b)_kj or conj(b_jk)
                const int ia = dag_a ? 2 * (3 * k + i) : 2 * (3 * i + k);
                const int ib = dag_b ? 2 * (3 * j + k) : 2 * (3 * k + j);
                const double ar = a[ia], ai = dag_a ? -a[ia + 1] : a[ia + 1];
                const double br = b[ib], bi = dag_b ? -b[ib + 1] : b[ib + 1];
                re = fma_(ar, br, re);
                re = fma_(-ai, bi, re);
                im = fma_(ar, bi, im);
                im = fma_(ai, br, im);
            }
            c[2 * (3 * i + j)] = re;
            c[2 * (3 * i + j) + 1] = im;
        }
}

struct Geo {
    int L[4];
    __device__ int step(int site, int mu, int d) const {  // site + d * mu, periodic
        int c[4];
        int s = site;
        for (int k = 0; k < 4; ++k) {
            c[k] = s % L[k];
            s /= L[k];
        }
        c[mu] = (c[mu] + d + L[mu]) % L[mu];
        return c[0] + L[0] * (c[1] + L[1] * (c[2] + L[2] * c[3]));
    }
};

// F_{mu nu}(x) (traceless Hermitian, 18 reals) from the four leaves at x.
__device__ void field_strength(const LatDesc& ld, const Geo& g, int x, int mu, int nu, double F[18]) {
    double Q[18], u1[18], u2[18], t1[18], t2[18], l[18];
#pragma unroll
    for (int k = 0; k < 18; ++k) Q[k] = 0.0;
    auto link = [&](int m, int site, double* u) { load_link<P64, double>(ld.gauge, ld.V, m, site, u); };
    auto add = [&]() {
#pragma unroll
        for (int k = 0; k < 18; ++k) Q[k] += l[k];
    };
    const int xm = g.step(x, mu, 1), xn = g.step(x, nu, 1);
    const int xmm = g.step(x, mu, -1), xnm = g.step(x, nu, -1);
    // +mu +nu -mu -nu: U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
    link(mu, x, u1);
    link(nu, xm, u2);
    m3_mul(u1, u2, t1, false, false);
    link(mu, xn, u1);
    m3_mul(t1, u1, t2, false, true);
    link(nu, x, u1);
    m3_mul(t2, u1, l, false, true);
    add();
    // +nu -mu -nu +mu: U_nu(x) U_mu(x+nu-mu)^+ U_nu(x-mu)^+ U_mu(x-mu)
    link(nu, x, u1);
    link(mu, g.step(xn, mu, -1), u2);
    m3_mul(u1, u2, t1, false, true);
    link(nu, xmm, u1);
    m3_mul(t1, u1, t2, false, true);
    link(mu, xmm, u1);
    m3_mul(t2, u1, l, false, false);
    add();
    // -mu -nu +mu +nu: U_mu(x-mu)^+ U_nu(x-mu-nu)^+ U_mu(x-mu-nu) U_nu(x-nu)
    const int xmn = g.step(xmm, nu, -1);
    link(mu, xmm, u1);
    link(nu, xmn, u2);
    m3_mul(u1, u2, t1, true, true);
    link(mu, xmn, u1);
    m3_mul(t1, u1, t2, false, false);
    link(nu, xnm, u1);
    m3_mul(t2, u1, l, false, false);
    add();
    // -nu +mu +nu -mu: U_nu(x-nu)^+ U_mu(x-nu) U_nu(x+mu-nu) U_mu(x)^+
    link(nu, xnm, u1);
    link(mu, xnm, u2);
    m3_mul(u1, u2, t1, true, false);
    link(nu, g.step(xnm, mu, 1), u1);
    m3_mul(t1, u1, t2, false, false);
    link(mu, x, u1);
    m3_mul(t2, u1, l, false, true);
    add();
    // F = (Q - Q^+) / (8 i): F_ij = (Im Q_ij + Im Q_ji, Re Q_ji - Re Q_ij) / 8
    double tr = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int a = 2 * (3 * i + j), b = 2 * (3 * j + i);
            F[a] = (Q[a + 1] + Q[b + 1]) * 0.125;
            F[a + 1] = (Q[b] - Q[a]) * 0.125;
        }
#pragma unroll
    for (int i = 0; i < 3; ++i) tr += F[2 * (4 * i)];
#pragma unroll
    for (int i = 0; i < 3; ++i) F[2 * (4 * i)] -= tr / 3.0;
}

__global__ void __launch_bounds__(256) k_clover_build(LatDesc ld, double c_sw, SigmaTab tab, uint4* __restrict__ c64,
                                                      uint4* __restrict__ c32, unsigned long long* __restrict__ nbits) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= ld.V) return;
    Geo g;
    for (int k = 0; k < 4; ++k) g.L[k] = ld.L[k];
    // blocks[half][(s a), (s' b)] accumulated as -(c_sw / 2) sum_k sigma_k[s][s'] F_k[a][b]
    double H[2][72];
#pragma unroll
    for (int k = 0; k < 72; ++k) H[0][k] = H[1][k] = 0.0;
    int plane = 0;
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = mu + 1; nu < 4; ++nu, ++plane) {
            double F[18];
            field_strength(ld, g, x, mu, nu, F);
            for (int h = 0; h < 2; ++h)
                for (int s = 0; s < 2; ++s)
                    for (int sp = 0; sp < 2; ++sp) {
                        const double sr = -0.5 * c_sw * tab.re[plane][h][s][sp];
                        const double si = -0.5 * c_sw * tab.im[plane][h][s][sp];
                        if (sr == 0.0 && si == 0.0) continue;
                        for (int a = 0; a < 3; ++a)
                            for (int b = 0; b < 3; ++b) {
                                const double fr = F[2 * (3 * a + b)], fi = F[2 * (3 * a + b) + 1];
                                const int e = 2 * (6 * (3 * s + a) + (3 * sp + b));
                                H[h][e] += sr * fr - si * fi;
                                H[h][e + 1] += sr * fi + si * fr;
                            }
                    }
        }
    // pack, bound the norm, store
    int c[4];
    {
        int s = x;
        for (int k = 0; k < 4; ++k) {
            c[k] = s % ld.L[k];
            s /= ld.L[k];
        }
    }
    const int par = (c[0] + c[1] + c[2] + c[3]) & 1;
    const size_t vh = (size_t)ld.V >> 1, hidx = (size_t)(x >> 1);
    double nrm = 0.0;
    for (int h = 0; h < 2; ++h) {
        double p[36];
        for (int i = 0; i < 6; ++i) {
            p[i] = H[h][2 * (6 * i + i)];
            double row = 0.0;
            for (int j = 0; j < 6; ++j) row += sqrt(H[h][2 * (6 * i + j)] * H[h][2 * (6 * i + j)] +
                                                    H[h][2 * (6 * i + j) + 1] * H[h][2 * (6 * i + j) + 1]);
            nrm = fmax(nrm, row);
            for (int j = i + 1; j < 6; ++j) {
                p[herm_off(i, j)] = H[h][2 * (6 * i + j)];
                p[herm_off(i, j) + 1] = H[h][2 * (6 * i + j) + 1];
            }
        }
        for (int k = 0; k < 18; ++k) {
            const unsigned long long lo = (unsigned long long)__double_as_longlong(p[2 * k]);
            const unsigned long long hi = (unsigned long long)__double_as_longlong(p[2 * k + 1]);
            c64[(size_t)(par * 36 + 18 * h + k) * vh + hidx] =
                make_uint4((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32));
        }
        for (int k = 0; k < 9; ++k)
            c32[(size_t)(par * 18 + 9 * h + k) * vh + hidx] =
                make_uint4(__float_as_uint((float)p[4 * k]), __float_as_uint((float)p[4 * k + 1]),
                           __float_as_uint((float)p[4 * k + 2]), __float_as_uint((float)p[4 * k + 3]));
    }
    atomicMax(nbits, (unsigned long long)__double_as_longlong(nrm));
}

// One thread per (odd site, chiral block): Gauss-Jordan elimination with
// partial pivoting of C + a, then the upper triangle of the inverse packed.
__global__ void __launch_bounds__(256) k_clover_invert(const uint4* __restrict__ c64_odd, int vh, double a,
                                                       uint4* __restrict__ inv64, uint4* __restrict__ inv32,
                                                       int* __restrict__ bad) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= 2 * vh) return;
    const int h = tid & 1, idx = tid >> 1;
    double p[36];
    load_herm<P64, double>(c64_odd, (size_t)vh, (size_t)idx, h, p);
    double M[6][6][2], R[6][6][2];
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            double re, im;
            if (i == j) {
                re = p[i] + a;
                im = 0.0;
            } else if (i < j) {
                re = p[herm_off(i, j)];
                im = p[herm_off(i, j) + 1];
            } else {
                re = p[herm_off(j, i)];
                im = -p[herm_off(j, i) + 1];
            }
            M[i][j][0] = re;
            M[i][j][1] = im;
            R[i][j][0] = i == j ? 1.0 : 0.0;
            R[i][j][1] = 0.0;
        }
    bool ok = true;
    for (int col = 0; col < 6; ++col) {
        int piv = col;
        double best = -1.0;
        for (int i = col; i < 6; ++i) {
            const double m = M[i][col][0] * M[i][col][0] + M[i][col][1] * M[i][col][1];
            if (m > best) {
                best = m;
                piv = i;
            }
        }
        if (!(best > 1e-280) || !isfinite(best)) {
            ok = false;
            break;
        }
        if (piv != col)
            for (int j = 0; j < 6; ++j)
                for (int q = 0; q < 2; ++q) {
                    double t = M[col][j][q];
                    M[col][j][q] = M[piv][j][q];
                    M[piv][j][q] = t;
                    t = R[col][j][q];
                    R[col][j][q] = R[piv][j][q];
                    R[piv][j][q] = t;
                }
        // scale the pivot row by 1 / pivot
        const double pr = M[col][col][0], pi = M[col][col][1];
        const double ir = pr / best, ii = -pi / best;
        for (int j = 0; j < 6; ++j) {
            double re = M[col][j][0] * ir - M[col][j][1] * ii, im = M[col][j][0] * ii + M[col][j][1] * ir;
            M[col][j][0] = re;
            M[col][j][1] = im;
            re = R[col][j][0] * ir - R[col][j][1] * ii;
            im = R[col][j][0] * ii + R[col][j][1] * ir;
            R[col][j][0] = re;
            R[col][j][1] = im;
        }
        for (int i = 0; i < 6; ++i) {
            if (i == col) continue;
            const double fr = M[i][col][0], fi = M[i][col][1];
            for (int j = 0; j < 6; ++j) {
                M[i][j][0] -= fr * M[col][j][0] - fi * M[col][j][1];
                M[i][j][1] -= fr * M[col][j][1] + fi * M[col][j][0];
                R[i][j][0] -= fr * R[col][j][0] - fi * R[col][j][1];
                R[i][j][1] -= fr * R[col][j][1] + fi * R[col][j][0];
            }
        }
    }
    if (!ok) {
        atomicOr(bad, 1);
        for (int k = 0; k < 36; ++k) p[k] = 0.0;
    } else {
        // the inverse of a Hermitian matrix is Hermitian: average the two triangles
        for (int i = 0; i < 6; ++i) {
            p[i] = R[i][i][0];
            for (int j = i + 1; j < 6; ++j) {
                p[herm_off(i, j)] = 0.5 * (R[i][j][0] + R[j][i][0]);
                p[herm_off(i, j) + 1] = 0.5 * (R[i][j][1] - R[j][i][1]);
            }
        }
    }
    for (int k = 0; k < 18; ++k) {
        const unsigned long long lo = (unsigned long long)__double_as_longlong(p[2 * k]);
        const unsigned long long hi = (unsigned long long)__double_as_longlong(p[2 * k + 1]);
        inv64[(size_t)(18 * h + k) * vh + idx] =
            make_uint4((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32));
    }
    if (inv32)
        for (int k = 0; k < 9; ++k)
            inv32[(size_t)(9 * h + k) * vh + idx] =
                make_uint4(__float_as_uint((float)p[4 * k]), __float_as_uint((float)p[4 * k + 1]),
                           __float_as_uint((float)p[4 * k + 2]), __float_as_uint((float)p[4 * k + 3]));
}

// The odd site of one-parity field index hidx (sites 2 hidx and 2 hidx + 1
// differ in x only, so one of them is odd).
__device__ __forceinline__ int odd_site(const LatDesc& ld, int hidx) {
    const int s = 2 * hidx;
    const int x = s % ld.L[0];
    int r = s / ld.L[0];
    const int y = r % ld.L[1];
    r /= ld.L[1];
    const int z = r % ld.L[2];
    const int t = r / ld.L[2];
    return ((x + y + z + t) & 1) ? s : s + 1;
}

__global__ void __launch_bounds__(256) k_clover_bo_inv(Work w, const BlockDesc* __restrict__ fblocks, Fld bfull,
                                                       Fld out, Clv cl) {
    FS_WG_PROLOGUE(w)
    const size_t gsf = (size_t)ld.V << w.lognr;
    const uint4* fb = bfull.v + (size_t)fblocks[b].slot_off * Tr<P64>::G;
    uint4* ob = out.v + (size_t)bd.slot_off * Tr<P64>::G;
    FS_SLOT_LOOP(w)
        const int hidx = (int)(slot >> w.lognr);
        const int site = odd_site(ld, hidx);
        double v[24];
        load_sp<P64, double>(fb, nullptr, gsf, ((size_t)site << w.lognr) + rhs, v);
        clv_mul<P64, double>(cl.inv + cl.off[sys], (size_t)ld.V >> 1, (size_t)hidx, v);
        store_sp<P64, double>(ob, nullptr, gs, slot, v);
    FS_SLOT_LOOP_END
    FS_WG_EPILOGUE
}

// out = -(C + a_sys)^-1 in at every site of a full-lattice plan (FP64): cl.inv +
// cl.off[sys] holds the system's inverse blocks for both parities, [2][36][V/2].
__global__ void __launch_bounds__(256) k_clover_inv_full(Work w, Fld out, Fld in, Clv cl) {
    FS_WG_PROLOGUE(w)
    const uint4* ib = in.v + (size_t)bd.slot_off * Tr<P64>::G;
    uint4* ob = out.v + (size_t)bd.slot_off * Tr<P64>::G;
    const size_t vh = (size_t)ld.V >> 1;
    FS_SLOT_LOOP(w)
        const int site = (int)(slot >> w.lognr);
        int c = site, par = 0;
        for (int k = 0; k < 4; ++k) {
            par += c % ld.L[k];
            c /= ld.L[k];
        }
        par &= 1;
        double v[24];
        load_sp<P64, double>(ib, nullptr, gs, slot, v);
        clv_mul<P64, double>(cl.inv + cl.off[sys] + (size_t)par * 36 * vh, vh, (size_t)(site >> 1), v);
#pragma unroll
        for (int k = 0; k < 24; ++k) v[k] = -v[k];
        store_sp<P64, double>(ob, nullptr, gs, slot, v);
    FS_SLOT_LOOP_END
    FS_WG_EPILOGUE
}

template <int P>
__global__ void __launch_bounds__(256) k_clover_add(Work w, Fld out, Fld in) {
    using A = typename Tr<P>::acc;
    constexpr int NCH = P == P64 ? 36 : 18;
    FS_WG_PROLOGUE(w)
    const uint4* ib = in.v + (size_t)bd.slot_off * Tr<P>::G;
    uint4* ob = out.v + (size_t)bd.slot_off * Tr<P>::G;
    const size_t vh = (size_t)ld.V >> 1;
    FS_SLOT_LOOP(w)
        (void)sys;
        const int site = (int)(slot >> w.lognr);
        int c = site, par = 0;
        for (int k = 0; k < 4; ++k) {
            par += c % ld.L[k];
            c /= ld.L[k];
        }
        par &= 1;
        A v[24], o[24];
        load_sp<P, A>(ib, nullptr, gs, slot, v);
        clv_mul<P, A>(reinterpret_cast<const uint4*>(ld.clv) + (size_t)par * NCH * vh, vh, (size_t)(site >> 1), v);
        load_sp<P, A>(ob, nullptr, gs, slot, o);
#pragma unroll
        for (int k = 0; k < 24; ++k) o[k] += v[k];
        store_sp<P, A>(ob, nullptr, gs, slot, o);
    FS_SLOT_LOOP_END
    FS_WG_EPILOGUE
}

template <int P>
void launch_eo_clv_p(int mode, const Work& w, Fld out, Fld in, Fld cen, Fld aux, const double* diag,
                     const SysState* st, int mask, double* part, hipStream_t s, const uint32_t* rc, int par_out,
                     const Clv& cl) {
    switch (mode) {
        case D_HOP: launch_eo_q<P, D_HOP, 1>(w, out, in, cen, aux, diag, st, mask, part, s, rc, par_out, cl); break;
        case D_PLAIN: launch_eo_q<P, D_PLAIN, 1>(w, out, in, cen, aux, diag, st, mask, part, s, rc, par_out, cl); break;
        case D_RHAT: launch_eo_q<P, D_RHAT, 1>(w, out, in, cen, aux, diag, st, mask, part, s, rc, par_out, cl); break;
        case D_TS: launch_eo_q<P, D_TS, 1>(w, out, in, cen, aux, diag, st, mask, part, s, rc, par_out, cl); break;
        default: break;
    }
}

}  // namespace

SigmaTab make_sigma_tab() {
    using C = std::complex<double>;
    C g[4][4][4];
    dr_gammas(g);
    SigmaTab t{};
    int plane = 0;
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = mu + 1; nu < 4; ++nu, ++plane) {
            C sg[4][4];
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) {
                    C comm = 0;
                    for (int k = 0; k < 4; ++k) comm += g[mu][i][k] * g[nu][k][j] - g[nu][i][k] * g[mu][k][j];
                    sg[i][j] = C(0, 0.5) * comm;
                }
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j)
                    if ((i < 2) != (j < 2) && std::abs(sg[i][j]) > 1e-12)
                        throw std::runtime_error("sigma_{mu nu} mixes the chiral halves");
            for (int h = 0; h < 2; ++h)
                for (int i = 0; i < 2; ++i)
                    for (int j = 0; j < 2; ++j) {
                        t.re[plane][h][i][j] = sg[2 * h + i][2 * h + j].real();
                        t.im[plane][h][i][j] = sg[2 * h + i][2 * h + j].imag();
                    }
        }
    return t;
}

void launch_clover_build(const LatDesc& ld, double c_sw, const SigmaTab& tab, uint4* c64, uint4* c32,
                         unsigned long long* norm_bits, hipStream_t s) {
    hipLaunchKernelGGL(k_clover_build, dim3((ld.V + 255) / 256), dim3(256), 0, s, ld, c_sw, tab, c64, c32, norm_bits);
}

void launch_clover_invert(const uint4* c64_odd, int vh, double a, uint4* inv64, uint4* inv32, int* bad,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_clover_invert, dim3((2 * vh + 255) / 256), dim3(256), 0, s, c64_odd, vh, a, inv64, inv32,
                       bad);
}

void launch_clover_bo_inv(const Work& wh, const BlockDesc* fblocks, Fld bfull, Fld out, const Clv& cl64,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_clover_bo_inv, dim3(grid_of(wh)), dim3(wh.wg), 0, s, wh, fblocks, bfull, out, cl64);
}

void launch_clover_inv_full(const Work& w, Fld out, Fld in, const Clv& cl64, hipStream_t s) {
    hipLaunchKernelGGL(k_clover_inv_full, dim3(grid_of(w)), dim3(w.wg), 0, s, w, out, in, cl64);
}

void launch_clover_add(int prec, const Work& w, Fld out, Fld in, hipStream_t s) {
    if (prec == P64) hipLaunchKernelGGL(k_clover_add<P64>, dim3(grid_of(w)), dim3(w.wg), 0, s, w, out, in);
    else if (prec == P32) hipLaunchKernelGGL(k_clover_add<P32>, dim3(grid_of(w)), dim3(w.wg), 0, s, w, out, in);
}

void launch_dslash_eo_clv(int prec, int mode, const Work& w, Fld out, Fld in, Fld cen, Fld aux, const double* diag,
                          const SysState* st, int mask, double* part, hipStream_t s, const uint32_t* rc, int par_out,
                          const Clv& cl) {
    if (mode == D_RESID) {
        launch_eo_q<P64, D_RESID, 1>(w, out, in, cen, aux, diag, st, mask, part, s, rc, par_out, cl);
        return;
    }
    if (prec == P64) launch_eo_clv_p<P64>(mode, w, out, in, cen, aux, diag, st, mask, part, s, rc, par_out, cl);
    else if (prec == P32) launch_eo_clv_p<P32>(mode, w, out, in, cen, aux, diag, st, mask, part, s, rc, par_out, cl);
}

void launch_eo_prep_clv(const Work& wh, const BlockDesc* fblocks, Fld bfull, Fld bo_inv, Fld bh, const double* diag,
                        double* part, hipStream_t s) {
    const size_t lds = lds_cap(wh.wg, wh.occ);
    if (wh.nr >= 4)
        hipLaunchKernelGGL((k_dslash_eo_t<P64, D_PREP, 1, 1>), dim3(grid_of(wh)), dim3(wh.wg), lds, s, wh, bh, bo_inv,
                           Fld(), bfull, diag, nullptr, (int)M_ALL, part, nullptr, 0, fblocks, Clv());
    else
        hipLaunchKernelGGL((k_dslash_eo_t<P64, D_PREP, 0, 1>), dim3(grid_of(wh)), dim3(wh.wg), lds, s, wh, bh, bo_inv,
                           Fld(), bfull, diag, nullptr, (int)M_ALL, part, nullptr, 0, fblocks, Clv());
}

void launch_eo_post_clv(const Work& wh, const BlockDesc* fblocks, Fld bfull, Fld xh, Fld xfull, const double* diag,
                        const Clv& cl64, hipStream_t s) {
    const size_t lds = lds_cap(wh.wg, wh.occ);
    if (wh.nr >= 4)
        hipLaunchKernelGGL((k_dslash_eo_t<P64, D_POST, 1, 1>), dim3(grid_of(wh)), dim3(wh.wg), lds, s, wh, xfull, xh,
                           Fld(), bfull, diag, nullptr, (int)M_ALL, nullptr, nullptr, 1, fblocks, cl64);
    else
        hipLaunchKernelGGL((k_dslash_eo_t<P64, D_POST, 0, 1>), dim3(grid_of(wh)), dim3(wh.wg), lds, s, wh, xfull, xh,
                           Fld(), bfull, diag, nullptr, (int)M_ALL, nullptr, nullptr, 1, fblocks, cl64);
}

}  // namespace fs
