// Launches of the shifted Wilson-Dirac stencils (kernels in fs_stencil.h).
#include "fs_stencil.h"

namespace fs {

template <int P, int MODE, int ILP>
static void launch_t(const Work& w, Fld out, Fld in, Fld aux, const double* diag, const SysState* st,
                     int mask, double* part, hipStream_t s, const uint32_t* rc) {
    const size_t lds = lds_cap(w.wg, w.occ);
    switch (qmode<P>(w)) {
        case 2:
            if constexpr (P == P32)
                hipLaunchKernelGGL((k_dslash<P, MODE, ILP, 2>), dim3(grid_of(w)), dim3(w.wg), lds, s, w, out, in, aux,
                                   diag, st, mask, part, rc);
            break;
        case 1:
            hipLaunchKernelGGL((k_dslash<P, MODE, ILP, 1>), dim3(grid_of(w)), dim3(w.wg), lds, s, w, out, in, aux,
                               diag, st, mask, part, rc);
            break;
        default:
            hipLaunchKernelGGL((k_dslash<P, MODE, ILP, 0>), dim3(grid_of(w)), dim3(w.wg), lds, s, w, out, in, aux,
                               diag, st, mask, part, rc);
    }
}

template <int P, int MODE>
static void launch_tile(const Work& w, Fld out, Fld in, Fld aux, const double* diag, const SysState* st,
                        int mask, double* part, hipStream_t s, const uint32_t* rc) {
    const size_t need = (size_t)tile_nbuf<P>() * 24 * sizeof(typename Tr<P>::acc) * w.wg;
    const size_t lds = std::max(need, lds_cap(w.wg, w.occ));
    switch (qmode<P>(w)) {
        case 2:
            if constexpr (P == P32)
                hipLaunchKernelGGL((k_dslash_tile<P, MODE, 2>), dim3(grid_of(w)), dim3(w.wg), lds, s, w, out, in, aux,
                                   diag, st, mask, part, rc);
            break;
        case 1:
            hipLaunchKernelGGL((k_dslash_tile<P, MODE, 1>), dim3(grid_of(w)), dim3(w.wg), lds, s, w, out, in, aux,
                               diag, st, mask, part, rc);
            break;
        default:
            hipLaunchKernelGGL((k_dslash_tile<P, MODE, 0>), dim3(grid_of(w)), dim3(w.wg), lds, s, w, out, in, aux,
                               diag, st, mask, part, rc);
    }
}

template <int P, int MODE>
static void launch_v(const Work& w, Fld out, Fld in, Fld aux, const double* diag, const SysState* st,
                     int mask, double* part, hipStream_t s, const uint32_t* rc) {
    if (w.ilp == 2) launch_tile<P, MODE>(w, out, in, aux, diag, st, mask, part, s, rc);
    else if (w.ilp) launch_t<P, MODE, 1>(w, out, in, aux, diag, st, mask, part, s, rc);
    else launch_t<P, MODE, 0>(w, out, in, aux, diag, st, mask, part, s, rc);
}

template <int P>
static void launch_p(int mode, const Work& w, Fld out, Fld in, Fld aux, const double* diag,
                     const SysState* st, int mask, double* part, hipStream_t s, const uint32_t* rc) {
    switch (mode) {
        case D_PLAIN: launch_v<P, D_PLAIN>(w, out, in, aux, diag, st, mask, part, s, rc); break;
        case D_RHAT: launch_v<P, D_RHAT>(w, out, in, aux, diag, st, mask, part, s, rc); break;
        case D_TS: launch_v<P, D_TS>(w, out, in, aux, diag, st, mask, part, s, rc); break;
        default: break;
    }
}

void launch_dslash(int prec, int mode, const Work& w, Fld out, Fld in, Fld aux, const double* diag,
                   const SysState* st, int mask, double* part, hipStream_t s, const uint32_t* rc) {
    if (mode == D_RESID) {
        launch_v<P64, D_RESID>(w, out, in, aux, diag, st, mask, part, s, rc);
        return;
    }
    switch (prec) {
        case P64: launch_p<P64>(mode, w, out, in, aux, diag, st, mask, part, s, rc); break;
        case P32: launch_p<P32>(mode, w, out, in, aux, diag, st, mask, part, s, rc); break;
        case P16: launch_p<P16>(mode, w, out, in, aux, diag, st, mask, part, s, rc); break;
        case PBF: launch_p<PBF>(mode, w, out, in, aux, diag, st, mask, part, s, rc); break;
        default: break;
    }
}


template <int P>
static void launch_eo_p(int mode, const Work& w, Fld out, Fld in, Fld cen, Fld aux, const double* diag,
                        const SysState* st, int mask, double* part, hipStream_t s, const uint32_t* rc, int par_out) {
    switch (mode) {
        case D_HOP: launch_eo_q<P, D_HOP>(w, out, in, cen, aux, diag, st, mask, part, s, rc, par_out); break;
        case D_PLAIN: launch_eo_q<P, D_PLAIN>(w, out, in, cen, aux, diag, st, mask, part, s, rc, par_out); break;
        case D_RHAT: launch_eo_q<P, D_RHAT>(w, out, in, cen, aux, diag, st, mask, part, s, rc, par_out); break;
        case D_TS: launch_eo_q<P, D_TS>(w, out, in, cen, aux, diag, st, mask, part, s, rc, par_out); break;
        default: break;
    }
}

void launch_dslash_eo(int prec, int mode, const Work& w, Fld out, Fld in, Fld cen, Fld aux, const double* diag,
                      const SysState* st, int mask, double* part, hipStream_t s, const uint32_t* rc, int par_out) {
    if (mode == D_RESID) {
        launch_eo_q<P64, D_RESID>(w, out, in, cen, aux, diag, st, mask, part, s, rc, par_out);
        return;
    }
    switch (prec) {
        case P64: launch_eo_p<P64>(mode, w, out, in, cen, aux, diag, st, mask, part, s, rc, par_out); break;
        case P32: launch_eo_p<P32>(mode, w, out, in, cen, aux, diag, st, mask, part, s, rc, par_out); break;
        case P16: launch_eo_p<P16>(mode, w, out, in, cen, aux, diag, st, mask, part, s, rc, par_out); break;
        case PBF: launch_eo_p<PBF>(mode, w, out, in, cen, aux, diag, st, mask, part, s, rc, par_out); break;
        default: break;
    }
}

void launch_eo_prep(const Work& wh, const BlockDesc* fblocks, Fld bfull, Fld bh, const double* diag, double* part,
                    hipStream_t s) {
    if (wh.tc > 0) {  // stencil mapping: stream over t
        const size_t lds = lds_cap(wh.wg, wh.occ);
        if (wh.nr >= 4)
            hipLaunchKernelGGL((k_dslash_eo_t<P64, D_PREP, 1>), dim3(grid_of(wh)), dim3(wh.wg), lds, s, wh, bh, bfull,
                               Fld(), Fld(), diag, nullptr, (int)M_ALL, part, nullptr, 0, fblocks, Clv());
        else
            hipLaunchKernelGGL((k_dslash_eo_t<P64, D_PREP, 0>), dim3(grid_of(wh)), dim3(wh.wg), lds, s, wh, bh, bfull,
                               Fld(), Fld(), diag, nullptr, (int)M_ALL, part, nullptr, 0, fblocks, Clv());
        return;
    }
    if (wh.nr >= 4)
        hipLaunchKernelGGL(k_eo_prep<1>, dim3(grid_of(wh)), dim3(wh.wg), 0, s, wh, fblocks, bfull, bh, diag, part);
    else
        hipLaunchKernelGGL(k_eo_prep<0>, dim3(grid_of(wh)), dim3(wh.wg), 0, s, wh, fblocks, bfull, bh, diag, part);
}

void launch_eo_post(const Work& wh, const BlockDesc* fblocks, Fld bfull, Fld xh, Fld xfull, const double* diag,
                    hipStream_t s) {
    if (wh.tc > 0) {  // stencil mapping: stream over t
        const size_t lds = lds_cap(wh.wg, wh.occ);
        if (wh.nr >= 4)
            hipLaunchKernelGGL((k_dslash_eo_t<P64, D_POST, 1>), dim3(grid_of(wh)), dim3(wh.wg), lds, s, wh, xfull, xh,
                               Fld(), bfull, diag, nullptr, (int)M_ALL, nullptr, nullptr, 1, fblocks, Clv());
        else
            hipLaunchKernelGGL((k_dslash_eo_t<P64, D_POST, 0>), dim3(grid_of(wh)), dim3(wh.wg), lds, s, wh, xfull, xh,
                               Fld(), bfull, diag, nullptr, (int)M_ALL, nullptr, nullptr, 1, fblocks, Clv());
        return;
    }
    if (wh.nr >= 4)
        hipLaunchKernelGGL(k_eo_post<1>, dim3(grid_of(wh)), dim3(wh.wg), 0, s, wh, fblocks, bfull, xh, xfull, diag);
    else
        hipLaunchKernelGGL(k_eo_post<0>, dim3(grid_of(wh)), dim3(wh.wg), 0, s, wh, fblocks, bfull, xh, xfull, diag);
}

}  // namespace fs
