// kernels_stream.hip -- window-streaming checkerboard kernels for gfx950
// (the device code, and what it computes, is described in stream_device.hpp).
#include "stream_device.hpp"

namespace spinlat {

using namespace streamk;

namespace {

// -------------------------------------------------------------------------
// HALF: colour c in place.
template <int KIND, int DIM>
__global__ void __launch_bounds__(kBlock) k_stream_half(SweepArgs a, StreamGeom sg)
{
    __shared__ Luts lut;
    uint64_t thr_up, thr_down;
    build_luts<KIND, DIM>(lut, a.lut, thr_up, thr_down);
    __syncthreads();

    Obs o = {0, 0, 0, 0};
    stream_half_item<KIND, DIM>(a, sg, item_of_lane(sg), lut, thr_up, thr_down, o);
    block_accumulate(o.bond, o.mag, o.acc, o.unfl, a.acc);
}

// -------------------------------------------------------------------------
// FUSED (2D): both colours of a strip, source copy -> destination copy.
template <int KIND>
__global__ void __launch_bounds__(kBlock) k_stream_fused(SweepArgs a, StreamGeom sg,
                                                         const uint8_t* S0, const uint8_t* S1,
                                                         uint8_t* D0, uint8_t* D1)
{
    __shared__ Luts lut;
    uint64_t thr_up, thr_down;
    build_luts<KIND, 2>(lut, a.lut, thr_up, thr_down);
    __syncthreads();

    Obs o = {0, 0, 0, 0};
    const uint32_t item = item_of_lane(sg);
    if (item < sg.nitems) {
        const uint32_t lane = threadIdx.x & 63u;
        const uint32_t li = lane % sg.W;
        const uint32_t gbase = lane - li;
        const uint32_t win = item % sg.nwin;
        const uint32_t strip = item / sg.nwin;
        const uint32_t J = win * sg.win_cols;
        // window mode: lanes 1..62 own columns J..J+61, lanes 0 and 63 are halo
        const uint32_t col = sg.wrap ? li : (J + sg.ncols - 1 + li) % sg.ncols;
        const bool owned = sg.wrap || (li >= 1 && li <= 62 && J + li - 1 < sg.ncols);
        const uint32_t src_l = gbase + ((li + sg.W - 1) & (sg.W - 1));
        const uint32_t src_r = gbase + ((li + 1) & (sg.W - 1));
        uint32_t colE = col;
        if (!sg.wrap) {
            if (li == 0) colE = (J + 2 * sg.ncols - 2) % sg.ncols;
            if (li == 63) colE = (J + 63) % sg.ncols;
        }
        const uint32_t L = sg.L;
        const uint64_t rowb = sg.Lh;
        const uint32_t y0 = strip * sg.H;
        const uint32_t y1 = min(y0 + sg.H, L);
        const PhiloxKey ks = philox_schedule(a.key0, a.key1);
        const uint64_t c4 = 4ull * col;

        // window of old colour-1 rows (i-1, i) and new colour-0 rows (i-2, i-1)
        uint32_t c1a = ld(S1, wrap_row((int)y0 - 2, L) * rowb + c4);
        uint32_t c1b = ld(S1, wrap_row((int)y0 - 1, L) * rowb + c4);
        uint32_t n0a = 0, n0b = 0;
        for (int i = (int)y0 - 1; i <= (int)y1; ++i) {
            const uint32_t yi = wrap_row(i, L);
            const uint32_t c1d = ld(S1, wrap_row(i + 1, L) * rowb + c4);
            const uint32_t own0 = ld(S0, (uint64_t)yi * rowb + c4);
            // colour 0 at row i (p = i & 1): neighbours c1 rows i-1, i, i+1
            const uint32_t p0 = yi & 1u;
            uint32_t adj = __shfl(c1b, p0 ? src_r : src_l, 64);
            if (!sg.wrap) {
                const uint32_t E = ld(S1, (uint64_t)yi * rowb + 4ull * colE);
                if (p0 ? li == 63 : li == 0) adj = E;
            }
            uint32_t nb0[4] = {c1b, side_word(c1b, adj, p0), c1a, c1d};
            const bool own_row0 = i >= (int)y0 && i < (int)y1;
            const uint32_t new0 = word_update<KIND, 2>(own0, nb0, p0, yi * sg.ncols + col, 0u, a.t,
                                                       ks, lut, thr_up, thr_down,
                                                       owned && own_row0, false, o);
            if (owned && own_row0) st(D0, (uint64_t)yi * rowb + c4, new0);
            // colour 1 at row i-1 (p = i & 1): neighbours new c0 rows i-2, i-1, i
            if (i - 1 >= (int)y0) {
                const uint32_t ym = wrap_row(i - 1, L);
                const uint32_t p1 = p0;
                const uint32_t adj1 = __shfl(n0b, p1 ? src_r : src_l, 64);
                uint32_t nb1[4] = {n0b, side_word(n0b, adj1, p1), n0a, new0};
                const uint32_t new1 = word_update<KIND, 2>(c1a, nb1, p1, ym * sg.ncols + col, 1u,
                                                           a.t, ks, lut, thr_up, thr_down, owned,
                                                           true, o);
                if (owned) st(D1, (uint64_t)ym * rowb + c4, new1);
            }
            c1a = c1b;
            c1b = c1d;
            n0a = n0b;
            n0b = new0;
        }
    }
    block_accumulate(o.bond, o.mag, o.acc, o.unfl, a.acc);
}

inline unsigned blocks_for_items(const StreamGeom& sg)
{
    const uint32_t groups_per_block = kWaves * sg.G;
    return (unsigned)ceil_div(sg.nitems, groups_per_block);
}

int default_rows(const Geom& g, bool fused) { return fused ? 32 : (g.dim == 3 ? 16 : 32); }

}  // namespace

bool tiled_supported(const Geom& g, int kind, int tile_rows, int tile_words, bool fused)
{
    if (tile_words != 0) return false;
    if (tile_rows < 0 || tile_rows > (int)g.L) return false;
    if (fused && g.dim != 2) return false;
    (void)kind;
    return (g.Lh % 4) == 0;
}

hipError_t launch_tiled_half(const SweepArgs& a, int kind, hipStream_t s)
{
    const int H = a.tile_rows > 0 ? a.tile_rows : default_rows(a.g, false);
    const StreamGeom sg = make_geom(a.g, H, false);
    const dim3 grid(blocks_for_items(sg)), block(kBlock);
    if (a.g.dim == 2) {
        if (kind == KIND_ISING_HALF)
            hipLaunchKernelGGL((k_stream_half<KIND_ISING_HALF, 2>), grid, block, 0, s, a, sg);
        else if (kind == KIND_ISING_ONE)
            hipLaunchKernelGGL((k_stream_half<KIND_ISING_ONE, 2>), grid, block, 0, s, a, sg);
        else
            hipLaunchKernelGGL((k_stream_half<KIND_NE, 2>), grid, block, 0, s, a, sg);
    } else {
        if (kind == KIND_ISING_HALF)
            hipLaunchKernelGGL((k_stream_half<KIND_ISING_HALF, 3>), grid, block, 0, s, a, sg);
        else
            hipLaunchKernelGGL((k_stream_half<KIND_ISING_ONE, 3>), grid, block, 0, s, a, sg);
    }
    return hipGetLastError();
}

hipError_t launch_fused_sweep(const SweepArgs& a, int kind, const uint8_t* src0,
                              const uint8_t* src1, uint8_t* dst0, uint8_t* dst1, hipStream_t s)
{
    const int H = a.tile_rows > 0 ? a.tile_rows : default_rows(a.g, true);
    const StreamGeom sg = make_geom(a.g, H, true);
    const dim3 grid(blocks_for_items(sg)), block(kBlock);
    if (kind == KIND_ISING_HALF)
        hipLaunchKernelGGL(k_stream_fused<KIND_ISING_HALF>, grid, block, 0, s, a, sg, src0, src1,
                           dst0, dst1);
    else if (kind == KIND_ISING_ONE)
        hipLaunchKernelGGL(k_stream_fused<KIND_ISING_ONE>, grid, block, 0, s, a, sg, src0, src1,
                           dst0, dst1);
    else
        hipLaunchKernelGGL(k_stream_fused<KIND_NE>, grid, block, 0, s, a, sg, src0, src1, dst0,
                           dst1);
    return hipGetLastError();
}

}  // namespace spinlat
