// kernels_rows.hip -- the half-sweep by independent row groups
// (SL_MODE_HALF_ROWS) for single lattices; the device code and what it
// computes are described in rows_device.hpp.
#include "rows_device.hpp"

namespace spinlat {

using namespace rowk;

namespace {

// rg.nstrips holds the row sets (waves' worth of rows) of one plane, both
// parities; rg.nitems those of the launch.  rg.K row sets per wave; the block
// has blockDim.x / 64 waves.
template <int KIND, int DIM, int D, int RAGS>
__global__ void __launch_bounds__(1024) k_rows_half(SweepArgs a, RowGeom rg)
{
    __shared__ RowLuts lut;
    Obs o = {0, 0, 0, 0, 0};
    const Lanes ln = lanes_of(rg, false);
    const uint32_t it0 = (remap_block() * (blockDim.x >> 6) + ln.wave) * rg.K;
    rows_run<KIND, DIM, D, RAGS>(a, rg, it0, ln, a.lut, lut, o);
    int32_t bond, mag, acc, unfl;
    finish_obs<KIND, DIM>(o, bond, mag, acc, unfl);
    block_accumulate(bond, mag, acc, unfl, a.acc);
}

// Ragged rows get kernels of their own, so that the others carry no code for
// them (a runtime branch between the two updates cost 8% at 3D L = 256).
template <int KIND, int DIM>
void launch_rows_k(const SweepArgs& a, const RowGeom& rg, hipStream_t s)
{
    const dim3 grid(cdiv(rg.nitems, rg.block / 64 * rg.K)), block(rg.block);
    constexpr bool ising = KIND == KIND_ISING_HALF || KIND == KIND_ISING_ONE;
    // NE kinds never get ragged geometry (rows_supported)
    constexpr int kRag = ising ? kRagAll : kRagNone;
    if (rg.D == 4) {
        if (rg.rag) hipLaunchKernelGGL((k_rows_half<KIND, DIM, 4, kRag>), grid, block, 0, s, a, rg);
        else hipLaunchKernelGGL((k_rows_half<KIND, DIM, 4, kRagNone>), grid, block, 0, s, a, rg);
    } else if (rg.D == 2) {
        if (rg.rag) hipLaunchKernelGGL((k_rows_half<KIND, DIM, 2, kRag>), grid, block, 0, s, a, rg);
        else hipLaunchKernelGGL((k_rows_half<KIND, DIM, 2, kRagNone>), grid, block, 0, s, a, rg);
    } else {
        hipLaunchKernelGGL((k_rows_half<KIND, DIM, 1, kRagNone>), grid, block, 0, s, a, rg);
    }
}

}  // namespace

// Ising rows may be ragged (D need not divide the row's word count); the NE
// kinds' observables are not masked for it.
bool rows_supported(const Geom& g, int kind, int waves, int tile_words, bool lut32_ok)
{
    if (kind == KIND_ISING_HALF && !lut32_ok) return false;
    RowGeom rg;
    return make_rows_geom(g, tile_words, waves, rg, kind == KIND_ISING_HALF || kind == KIND_ISING_ONE);
}

hipError_t launch_rows_half(const SweepArgs& a, int kind, int waves, int D, hipStream_t s)
{
    RowGeom rg;
    if (!make_rows_geom(a.g, D, waves, rg, kind == KIND_ISING_HALF || kind == KIND_ISING_ONE))
        return hipErrorInvalidValue;
    if (a.g.dim == 2) {
        if (kind == KIND_ISING_HALF) launch_rows_k<KIND_ISING_HALF, 2>(a, rg, s);
        else if (kind == KIND_ISING_ONE) launch_rows_k<KIND_ISING_ONE, 2>(a, rg, s);
        else if (a.lut_n > 2) launch_rows_k<KIND_NE_COUPLED, 2>(a, rg, s);
        else launch_rows_k<KIND_NE, 2>(a, rg, s);
    } else {
        if (kind == KIND_ISING_HALF) launch_rows_k<KIND_ISING_HALF, 3>(a, rg, s);
        else launch_rows_k<KIND_ISING_ONE, 3>(a, rg, s);
    }
    return hipGetLastError();
}

}  // namespace spinlat
