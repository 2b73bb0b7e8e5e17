// kernels_row.hip -- whole-row streaming checkerboard kernels for gfx950
// (the device code, and what it computes, is described in row_device.hpp).
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

// Fused sweep of the strip `item` of every row group (see fused_item).
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
    fused_item<KIND, D, XW, HT>(a, rg, item, ln, lut, xch, thr_up, thr_down, S0, S1, D0, D1, o);
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

// Strip heights of the default schedules (2, 4, 8, 16, 32) run the unrolled walk
// when they divide L; any other height runs the runtime-height kernel.
template <int KIND, int D>
void launch_fused_d(const SweepArgs& a, const RowGeom& rg, const uint8_t* s0, const uint8_t* s1, uint8_t* d0,
                    uint8_t* d1, hipStream_t s)
{
    const bool whole = rg.L % rg.H == 0;
    if (whole && rg.H == 32) launch_fused_h<KIND, D, 32>(a, rg, s0, s1, d0, d1, s);
    else if (whole && rg.H == 16) launch_fused_h<KIND, D, 16>(a, rg, s0, s1, d0, d1, s);
    else if (whole && rg.H == 8) launch_fused_h<KIND, D, 8>(a, rg, s0, s1, d0, d1, s);
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
