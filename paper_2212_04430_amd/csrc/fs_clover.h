// Clover term of the improved Wilson-Dirac operator (host declarations).
//
// The Results section runs the estimator on the clover-improved Wilson
// operator; the term is site-local, so a shift still enters only the scalar
// diagonal.  Convention (the paper does not print one), in the normalisation
// of the plain operator (forward hop with 1 - g_mu, diagonal 4 + m0 + sigma):
//   C(x) = -(c_sw / 2) sum_{mu<nu} sigma_{mu nu} F_{mu nu}(x),
//   sigma_{mu nu} = (i/2) [g_mu, g_nu],
//   F_{mu nu}(x) = traceless part of (Q_{mu nu}(x) - Q_{mu nu}(x)^+) / (8 i),
// Q_{mu nu}(x) the four plaquettes of the (mu, nu) plane at x, each taken
// counter-clockwise.  With this sign c_sw = 1 is the tree-level improvement
// coefficient.  sigma_{mu nu} commutes with g_5, so C(x) is two Hermitian 6 x 6
// blocks (spins 0-1 and 2-3); their packed layout is described at struct Clv.
#pragma once

#include <complex>

#include "fs_kernels.h"

namespace fs {

// sigma_{mu nu} on the two chiral halves: s[plane][half][row][col] (2 x 2
// complex each), planes (0,1), (0,2), (0,3), (1,2), (1,3), (2,3).
struct SigmaTab {
    double re[6][2][2][2];
    double im[6][2][2][2];
};

// The DeGrand-Rossi gamma_1..gamma_4 of the library (g[mu][row][col]).
void dr_gammas(std::complex<double> g[4][4][4]);

// sigma_{mu nu} from dr_gammas; throws std::runtime_error if a sigma mixes the
// chiral halves (it cannot for a basis with diagonal gamma_5).
SigmaTab make_sigma_tab();

// C of one lattice from its FP64 links ([mu][9][site] complex): FP64 packed
// sites into c64 ([parity][36][V/2] chunks) and their FP32 copy into c32
// ([parity][18][V/2]); *norm_bits receives (as the bit pattern of a
// non-negative double, atomic max) an upper bound on the spectral norm of every
// block (largest absolute row sum).  *norm_bits must hold 0 before the launch.
void launch_clover_build(const LatDesc& ld, double c_sw, const SigmaTab& tab, uint4* c64, uint4* c32,
                         unsigned long long* norm_bits, hipStream_t s);

// (C + a)^-1 at the odd sites: from the parity-1 half of c64, into inv64
// ([36][V/2]) and, if not null, inv32 ([18][V/2]).  *bad is set nonzero where a
// block is numerically singular.
void launch_clover_invert(const uint4* c64_odd, int vh, double a, uint4* inv64, uint4* inv32, int* bad,
                          hipStream_t s);

// out_o = (C_o + a_sys)^-1 b_o: b in the full layout of fblocks, out one-parity
// (odd) over the blocks of wh (FP64).
void launch_clover_bo_inv(const Work& wh, const BlockDesc* fblocks, Fld bfull, Fld out, const Clv& cl64,
                          hipStream_t s);

// out = -(C + a_sys)^-1 in over every site of a full-lattice plan (FP64), with
// cl64.inv + cl64.off[sys] the system's inverse blocks of both parities
// ([2][36][V/2], e.g. from launch_clover_invert on each parity).
void launch_clover_inv_full(const Work& w, Fld out, Fld in, const Clv& cl64, hipStream_t s);

// out += C in over every site of a full-lattice plan (FP64 or FP32 storage;
// the lattices' ld.clv in that precision).
void launch_clover_add(int prec, const Work& w, Fld out, Fld in, hipStream_t s);

// The even-odd launches of launch_dslash_eo with the clover term (FP64 and
// FP32): D_HOP (odd output) is followed by (C_o + a)^-1, the Schur modes form
// (C_e + a) in - D_eo (hop input).
void launch_dslash_eo_clv(int prec, int mode, const Work& w, Fld out, Fld in, Fld cen, Fld aux, const double* diag,
                          const SysState* st, int mask, double* part, hipStream_t s, const uint32_t* rc, int par_out,
                          const Clv& cl);

// Even-odd source with the clover term: bh = b_e - D_eo bo_inv (bo_inv from
// launch_clover_bo_inv), partial sums |b_e|^2 + |b_o|^2 of the full source.
void launch_eo_prep_clv(const Work& wh, const BlockDesc* fblocks, Fld bfull, Fld bo_inv, Fld bh, const double* diag,
                        double* part, hipStream_t s);

// Reconstruction: x_o = (C_o + a)^-1 (b_o - D_oe x_e), x_e copied, into xfull.
void launch_eo_post_clv(const Work& wh, const BlockDesc* fblocks, Fld bfull, Fld xh, Fld xfull, const double* diag,
                        const Clv& cl64, hipStream_t s);

}  // namespace fs
