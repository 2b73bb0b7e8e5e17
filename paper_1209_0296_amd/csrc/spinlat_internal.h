// spinlat_internal.h -- shared between the host runtime and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "host_logic.h"

namespace spinlat {

// Record accumulator layout (kSub, kQ, kSubStride, kSlotWords, kRecordWords),
// kMaxLut and the kernel kinds come from host_logic.h.

// Geometry of the colour-split layout.  Natural site (x, y, z) has colour
// (x+y+z)&1 and in-colour index k = ((z*L + y)*L + x) >> 1; the colour array
// holds row r = z*L + y at bytes [r*Lh, (r+1)*Lh), Lh = L/2, and row r of
// colour c holds x = 2*kk + ((y+z+c)&1).
struct Geom {
    uint32_t L;
    uint32_t Lh;
    uint32_t dim;
    uint32_t rows;  // L (2D) or L*L (3D)
    uint64_t nh;    // sites per colour = rows * Lh
};

struct SweepArgs {
    uint8_t* col[2];          // colour arrays (device)
    Geom g;
    uint32_t key0, key1;      // Philox key = seed
    uint32_t t;               // sweep index
    uint32_t colour;          // half-sweep colour (SIMPLE/HALF modes)
    int32_t update;           // 0: only accumulate observables (record r_0)
    int32_t lut_n;
    unsigned long long* acc;  // record slot [kSub][kQ]
    const uint64_t* lut;      // threshold table (device), lut_n entries
    // LDS-tiled modes
    int32_t tile_rows;
    int32_t tile_words;
};

// Colour array c of a sweep's lattice, by select rather than array index: the
// batched kernels build SweepArgs in registers, where a runtime index would
// put the array in scratch memory.
__device__ __forceinline__ uint8_t* colour_array(const SweepArgs& a, uint32_t c)
{
    return c ? a.col[1] : a.col[0];
}

hipError_t launch_fill_u64(unsigned long long* p, uint64_t n, hipStream_t s);
hipError_t launch_init(const SweepArgs& a, int kind, int init_mode, uint32_t bern_thr_lo,
                       uint32_t bern_thr_hi, hipStream_t s);
hipError_t launch_from_natural(const SweepArgs& a, const int8_t* nat, hipStream_t s);
hipError_t launch_to_natural(const SweepArgs& a, int8_t* nat, hipStream_t s);
hipError_t launch_clear_flags(const SweepArgs& a, hipStream_t s);
// Small lattices: both colour arrays in the LDS of one workgroup, nsweeps
// sweeps per launch, record s into a.acc + s slots, sweep index a.t + s.
constexpr int kResidentLds = 48 * 1024;  // bytes of lattice one workgroup holds
bool resident_supported(const Geom& g);
hipError_t launch_resident(const SweepArgs& a, int kind, uint32_t nsweeps, hipStream_t s);
// out (one int64, zeroed by the caller) += sum_i v_i v_i^ref; ne: v = 2n - 1
hipError_t launch_overlap(const SweepArgs& a, const int8_t* ref, int ne, unsigned long long* out,
                          hipStream_t s);
hipError_t launch_simple_half(const SweepArgs& a, int kind, hipStream_t s);
hipError_t launch_tiled_half(const SweepArgs& a, int kind, hipStream_t s);
hipError_t launch_fused_sweep(const SweepArgs& a, int kind, const uint8_t* src0, const uint8_t* src1,
                              uint8_t* dst0, uint8_t* dst1, hipStream_t s);
hipError_t launch_fold(unsigned long long* acc, int64_t* out, uint64_t n, uint64_t t_first,
                       int ising, hipStream_t s);

// Shape limits of the window-streaming kernels (checked by the runtime before launch).
bool tiled_supported(const Geom& g, int kind, int tile_rows, int tile_words, bool fused);

// Whole-row kernels: tile_rows = strip height H >= 1, tile_words = words per
// lane D in {1, 2, 4}; spin-1/2 needs every threshold >= 1 (lut32_ok).
bool row_supported(const Geom& g, int kind, int tile_rows, int tile_words, bool fused, bool lut32_ok);
hipError_t launch_row_half(const SweepArgs& a, int kind, int H, int D, hipStream_t s);
// Half-sweep by independent row groups (no walk): workgroups of `waves`
// waves (1..16), D in {1, 2, 4} words per lane, a colour row within one wave;
// spin-1/2 needs every threshold >= 1.
bool rows_supported(const Geom& g, int kind, int waves, int tile_words, bool lut32_ok);
hipError_t launch_rows_half(const SweepArgs& a, int kind, int waves, int D, hipStream_t s);
hipError_t launch_row_fused(const SweepArgs& a, int kind, int H, int D, const uint8_t* src0,
                            const uint8_t* src1, uint8_t* dst0, uint8_t* dst1, hipStream_t s);

// North-East model by random sub-lattices: one launch processes every B x B
// sub-lattice once (q = B^2 / (2 lambda) iterations of lambda random sites),
// reading `src` and writing `dst`.
struct NeSubArgs {
    const uint8_t* src[2];      // colour arrays at launch start
    uint8_t* dst[2];            // colour arrays after the launch
    uint32_t L, Lh, tiles_x, ntiles;
    uint32_t key0, key1;        // Philox key = seed
    uint32_t launch;            // launch index: 2 t, 2 t + 1 (balanced: 4 t .. 4 t + 3)
    uint32_t thr_m1_up;         // NE up-flip threshold minus one (accept iff word <= it)
    uint32_t thr_m1_down;       // NE down-flip threshold minus one
    uint32_t never;             // bit 0: up-flip threshold is 0; bit 1: down-flip threshold is 0
    unsigned long long* acc;    // record slot [kSub][kQ] of this sweep (accepted)
    unsigned long long* obs;    // if set: record slot that receives bond_sum, mag and
                                // unflipped of the launch-start lattice
};

// Shapes: host::ne_sub_supported.
// balanced: colour 0 then colour 1 per iteration, P/(8 lambda) iterations
// (four launches per sweep); else q = P/(2 lambda) iterations (two launches)
hipError_t launch_ne_sub(const NeSubArgs& a, int B, int lambda, bool balanced, hipStream_t s);

}  // namespace spinlat
