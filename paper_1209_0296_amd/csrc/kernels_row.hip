// kernels_row.hip -- whole-row streaming checkerboard kernels for gfx950
// (the device code, and what it computes, is described in row_device.hpp).
#include <utility>

#include "row_device.hpp"

namespace spinlat {

using namespace rowk;

namespace {

template <int KIND, int DIM, int D, bool XW>
__global__ void __launch_bounds__(1024) k_row_half(SweepArgs a, RowGeom rg)
{
    __shared__ RowLuts lut;
    __shared__ uint32_t xch[2][16][2];
    uint64_t thr_up, thr_down;
    build_row_luts<KIND, DIM>(lut, a.lut, thr_up, thr_down);
    __syncthreads();

    Obs o = {0, 0, 0, 0, 0};
    const Lanes ln = lanes_of(rg, XW);
    const uint32_t item = row_item(rg, XW, ln);
    half_item<KIND, DIM, D, XW>(a, rg, item, ln, lut, xch, thr_up, thr_down, o);
    int32_t bond, mag, acc, unfl;
    finish_obs<KIND, DIM>(o, bond, mag, acc, unfl);
    block_accumulate(bond, mag, acc, unfl, a.acc);
}

// Rows y0 + 1 .. y0 + HT - 1 of an unrolled walk (K = 0 .. HT - 2): row
// y0 + 1 + K has parity (K + 1) & 1 because y0 is even.
template <int KIND, int D, bool XW, int... K>
__device__ __forceinline__ void fused_inner_rows(std::integer_sequence<int, K...>, int y0, FusedState<KIND, D>& st,
                                                 const RowGeom& rg, const Lanes& ln, const uint8_t* S0,
                                                 const uint8_t* S1, uint8_t* D0, uint8_t* D1,
                                                 uint32_t (&xch)[2][16][4], uint32_t& buf, const SweepArgs& a,
                                                 const PhiloxKey& ks, const RowLuts& lut, uint64_t thr_up,
                                                 uint64_t thr_down, Obs& o)
{
    // the scheduling barrier keeps the compiler from interleaving rows, which
    // would keep several rows' state live at once (register spills)
    ((fused_step<KIND, D, XW, (K + 1) & 1, true, true, true>(y0 + 1 + K, st, rg, ln, S0, S1, D0, D1, xch, buf, a,
                                                             ks, lut, thr_up, thr_down, o),
      __builtin_amdgcn_sched_barrier(0)),
     ...);
}

// HT > 0: the strip height is the compile-time HT (even, dividing L), so the
// walk is unrolled: every row's parity is known (y0 = item * HT is even) and
// the rotating row state needs no register moves.  HT = 0: runtime strip
// height rg.H (any H >= 1, ragged last strip).
template <int KIND, int D, bool XW, int HT>
__global__ void __launch_bounds__(1024) k_row_fused(SweepArgs a, RowGeom rg, const uint8_t* S0,
                                                    const uint8_t* S1, uint8_t* D0, uint8_t* D1)
{
    __shared__ RowLuts lut;
    __shared__ uint32_t xch[2][16][4];
    uint64_t thr_up, thr_down;
    build_row_luts<KIND, 2>(lut, a.lut, thr_up, thr_down);
    __syncthreads();

    Obs o = {0, 0, 0, 0, 0};
    const Lanes ln = lanes_of(rg, XW);
    const uint32_t item = row_item(rg, XW, ln);
    if (item < rg.nitems) {
        const uint32_t L = rg.L;
        const uint64_t rowb = rg.Lh;
        const uint64_t cb = 4ull * D * ln.pos;
        const int H = HT > 0 ? HT : (int)rg.H;
        const int y0 = (int)(item * (uint32_t)H);
        const int y1 = min(y0 + H, (int)L);
        const PhiloxKey ks = philox_schedule(a.key0, a.key1);
        FusedState<KIND, D> st;
        st.c1a = ldv<D>(S1, (uint64_t)wrap1(y0 - 2, L) * rowb + cb);
        st.c1b = ldv<D>(S1, (uint64_t)wrap1(y0 - 1, L) * rowb + cb);
        st.c1d = ldv<D>(S1, (uint64_t)wrap1(y0, L) * rowb + cb);
        st.q1a = prepv<KIND, D>(st.c1a);
        st.q1b = prepv<KIND, D>(st.c1b);
        st.q1d = prepv<KIND, D>(st.c1d);
        st.own0 = ldv<D>(S0, (uint64_t)wrap1(y0 - 1, L) * rowb + cb);
#pragma unroll
        for (int d = 0; d < D; ++d) st.q0a.w[d] = st.q0b.w[d] = 0u;
        uint32_t buf = 0;
        // halo row y0-1 (colour 0 only, not stored), first row y0 (colour 0
        // only), rows y0+1 .. y1-1, halo row y1 (colour 1 of row y1-1 only)
        if constexpr (HT > 0) {
            // y0 is even, so row y0 + k has parity k & 1
            fused_step<KIND, D, XW, 1, false, false, true>(y0 - 1, st, rg, ln, S0, S1, D0, D1, xch, buf, a,
                                                           ks, lut, thr_up, thr_down, o);
            fused_step<KIND, D, XW, 0, false, true, true>(y0, st, rg, ln, S0, S1, D0, D1, xch, buf, a, ks,
                                                          lut, thr_up, thr_down, o);
            // rows y0 + 1 .. y0 + HT - 1 in pairs of parity (1, 0), then row y0 + HT - 1
#pragma nounroll
            for (int k = 1; k + 1 < HT; k += 2) {
                fused_step<KIND, D, XW, 1, true, true, true>(y0 + k, st, rg, ln, S0, S1, D0, D1, xch, buf, a, ks,
                                                             lut, thr_up, thr_down, o);
                fused_step<KIND, D, XW, 0, true, true, true>(y0 + k + 1, st, rg, ln, S0, S1, D0, D1, xch, buf, a,
                                                             ks, lut, thr_up, thr_down, o);
            }
            fused_step<KIND, D, XW, 1, true, true, true>(y0 + HT - 1, st, rg, ln, S0, S1, D0, D1, xch, buf, a, ks,
                                                         lut, thr_up, thr_down, o);
            fused_step<KIND, D, XW, 0, true, false, false>(y0 + HT, st, rg, ln, S0, S1, D0, D1, xch, buf, a,
                                                           ks, lut, thr_up, thr_down, o);
        } else {
            fused_step_p<KIND, D, XW, false, false, true>(y0 - 1, st, rg, ln, S0, S1, D0, D1, xch, buf, a, ks,
                                                          lut, thr_up, thr_down, o);
            fused_step_p<KIND, D, XW, false, true, true>(y0, st, rg, ln, S0, S1, D0, D1, xch, buf, a, ks, lut,
                                                         thr_up, thr_down, o);
            for (int i = y0 + 1; i < y1; ++i)
                fused_step_p<KIND, D, XW, true, true, true>(i, st, rg, ln, S0, S1, D0, D1, xch, buf, a, ks, lut,
                                                            thr_up, thr_down, o);
            fused_step_p<KIND, D, XW, true, false, false>(y1, st, rg, ln, S0, S1, D0, D1, xch, buf, a, ks, lut,
                                                          thr_up, thr_down, o);
        }
    }
    int32_t bond, mag, acc, unfl;
    finish_obs<KIND, 2>(o, bond, mag, acc, unfl);
    block_accumulate(bond, mag, acc, unfl, a.acc);
}

// ---- host side ----------------------------------------------------------------
unsigned row_blocks(const RowGeom& rg)
{
    if (rg.R > 64) return rg.nitems;
    return cdiv(rg.nitems, (rg.block / 64) * rg.slots);
}

template <int KIND, int DIM, int D>
void launch_half_d(const SweepArgs& a, const RowGeom& rg, hipStream_t s)
{
    if (rg.R > 64)
        hipLaunchKernelGGL((k_row_half<KIND, DIM, D, true>), dim3(row_blocks(rg)), dim3(rg.block), 0, s, a, rg);
    else
        hipLaunchKernelGGL((k_row_half<KIND, DIM, D, false>), dim3(row_blocks(rg)), dim3(rg.block), 0, s, a, rg);
}

template <int KIND, int DIM>
void launch_half_k(const SweepArgs& a, const RowGeom& rg, hipStream_t s)
{
    if (rg.D == 4) launch_half_d<KIND, DIM, 4>(a, rg, s);
    else if (rg.D == 2) launch_half_d<KIND, DIM, 2>(a, rg, s);
    else launch_half_d<KIND, DIM, 1>(a, rg, s);
}

template <int KIND, int D, int HT>
void launch_fused_h(const SweepArgs& a, const RowGeom& rg, const uint8_t* s0, const uint8_t* s1, uint8_t* d0,
                    uint8_t* d1, hipStream_t s)
{
    if (rg.R > 64)
        hipLaunchKernelGGL((k_row_fused<KIND, D, true, HT>), dim3(row_blocks(rg)), dim3(rg.block), 0, s, a, rg,
                           s0, s1, d0, d1);
    else
        hipLaunchKernelGGL((k_row_fused<KIND, D, false, HT>), dim3(row_blocks(rg)), dim3(rg.block), 0, s, a, rg,
                           s0, s1, d0, d1);
}

// Strip heights of the default schedules (2, 4, 8) run the unrolled walk
// when they divide L; any other height runs the runtime-height kernel.
template <int KIND, int D>
void launch_fused_d(const SweepArgs& a, const RowGeom& rg, const uint8_t* s0, const uint8_t* s1, uint8_t* d0,
                    uint8_t* d1, hipStream_t s)
{
    const bool whole = rg.L % rg.H == 0;
    if (whole && rg.H == 8) launch_fused_h<KIND, D, 8>(a, rg, s0, s1, d0, d1, s);
    else if (whole && rg.H == 4) launch_fused_h<KIND, D, 4>(a, rg, s0, s1, d0, d1, s);
    else if (whole && rg.H == 2) launch_fused_h<KIND, D, 2>(a, rg, s0, s1, d0, d1, s);
    else launch_fused_h<KIND, D, 0>(a, rg, s0, s1, d0, d1, s);
}

template <int KIND>
void launch_fused_k(const SweepArgs& a, const RowGeom& rg, const uint8_t* s0, const uint8_t* s1, uint8_t* d0,
                    uint8_t* d1, hipStream_t s)
{
    if (rg.D == 4) launch_fused_d<KIND, 4>(a, rg, s0, s1, d0, d1, s);
    else if (rg.D == 2) launch_fused_d<KIND, 2>(a, rg, s0, s1, d0, d1, s);
    else launch_fused_d<KIND, 1>(a, rg, s0, s1, d0, d1, s);
}

}  // namespace

bool row_supported(const Geom& g, int kind, int tile_rows, int tile_words, bool fused, bool lut32_ok)
{
    if (kind == KIND_ISING_HALF && !lut32_ok) return false;
    RowGeom rg;
    return tile_rows >= 1 && make_row_geom(g, tile_rows, tile_words, fused, rg);
}

hipError_t launch_row_half(const SweepArgs& a, int kind, int H, int D, hipStream_t s)
{
    RowGeom rg;
    if (!make_row_geom(a.g, H, D, false, rg)) return hipErrorInvalidValue;
    if (a.g.dim == 2) {
        if (kind == KIND_ISING_HALF) launch_half_k<KIND_ISING_HALF, 2>(a, rg, s);
        else if (kind == KIND_ISING_ONE) launch_half_k<KIND_ISING_ONE, 2>(a, rg, s);
        else if (a.lut_n > 2) launch_half_k<KIND_NE_COUPLED, 2>(a, rg, s);
        else launch_half_k<KIND_NE, 2>(a, rg, s);
    } else {
        if (kind == KIND_ISING_HALF) launch_half_k<KIND_ISING_HALF, 3>(a, rg, s);
        else launch_half_k<KIND_ISING_ONE, 3>(a, rg, s);
    }
    return hipGetLastError();
}

hipError_t launch_row_fused(const SweepArgs& a, int kind, int H, int D, const uint8_t* src0,
                            const uint8_t* src1, uint8_t* dst0, uint8_t* dst1, hipStream_t s)
{
    RowGeom rg;
    if (!make_row_geom(a.g, H, D, true, rg)) return hipErrorInvalidValue;
    if (kind == KIND_ISING_HALF) launch_fused_k<KIND_ISING_HALF>(a, rg, src0, src1, dst0, dst1, s);
    else if (kind == KIND_ISING_ONE) launch_fused_k<KIND_ISING_ONE>(a, rg, src0, src1, dst0, dst1, s);
    else if (a.lut_n > 2) launch_fused_k<KIND_NE_COUPLED>(a, rg, src0, src1, dst0, dst1, s);
    else launch_fused_k<KIND_NE>(a, rg, src0, src1, dst0, dst1, s);
    return hipGetLastError();
}

}  // namespace spinlat
