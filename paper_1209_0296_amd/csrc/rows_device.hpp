// rows_device.hpp -- device code of the half-sweep by independent row groups
// (SL_MODE_HALF_ROWS), shared by the single-lattice kernel (kernels_rows.hip)
// and the batched kernel (kernels_batch.hip).
//
// One colour is updated per launch (Alg. I steps 5-7: the kernel end separates
// the colours).  Every row group of R lanes owns one colour row outright: it
// loads its own D words per lane and the other colour's rows y-1, y, y+1 (and,
// in 3D, the rows of planes z-1 and z+1) with one vector load each, updates,
// stores, and is done.  There is no walk along y, so no prologue whose latency
// a short walk cannot hide; instead many short waves keep every SIMD busy
// while others wait on memory.  The neighbour rows a wave loads overlap those
// of the adjacent waves and come from the caches.
//
// A row set is 64 / R row groups' worth of rows, all of one row parity: row set
// w of plane z holds rows y = q + 2 (j * slots + slot) with q = w & 1,
// j = w >> 1, so the side the same-row neighbour sits on (p = (y + z + c) & 1)
// is uniform across a wave.  A wave takes K = 4 / D consecutive row sets one
// after the other, so every lane updates four words per launch whatever the
// row width.  (Measured and dropped: waves that load the next row set while
// updating the current one were slower at every depth, and so was issuing the
// first set's loads before the threshold table is built: the loaded words
// live across the table build and the registers cut the waves per SIMD.)
#pragma once
#include "row_device.hpp"

namespace spinlat {
namespace rowk {

// The neighbour words one row group needs for one row, raw.
template <int DIM, int D>
struct RowsIn {
    Vec<D> own, o0, om, op, zm, zp;
};

// Row set `it` of the launch (wave-uniform) and this lane's row in it.
struct RowsAt {
    uint32_t z, y;
    bool ok;  // this lane's row group has a row here
};

__device__ __forceinline__ RowsAt rows_at(const RowGeom& rg, uint32_t it, uint32_t slot)
{
    RowsAt r;
    r.z = it / rg.nstrips;
    const uint32_t rem = it - r.z * rg.nstrips;
    r.y = (rem & 1u) + 2u * ((rem >> 1) * rg.slots + slot);
    r.ok = it < rg.nitems && slot < rg.slots && r.y < rg.L;
    return r;
}

template <int DIM, int D>
__device__ __forceinline__ void rows_load(RowsIn<DIM, D>& in, const SweepArgs& a, const RowGeom& rg, const RowsAt& at,
                                          const Lanes& ln)
{
    if (!at.ok) return;
    const uint32_t L = rg.L, z = at.z, y = at.y;
    const uint32_t c = a.colour;
    const uint8_t* O = colour_array(a, c ^ 1u);
    const uint64_t rowb = rg.Lh;
    // one byte offset for the row, the neighbour rows as signed steps from it
    // (the periodic wrap as a select); the plane steps are wave-uniform
    const int64_t base = (int64_t)(((uint64_t)z * L + y) * rowb + 4ull * ln.col0);
    const int64_t ystep = (int64_t)rowb, ywrap = (int64_t)(L - 1) * (int64_t)rowb;
    in.own = ldv<D>(colour_array(a, c), (uint64_t)base);
    in.o0 = ldv<D>(O, (uint64_t)base);
    in.om = ldv<D>(O, (uint64_t)(base + (y == 0 ? ywrap : -ystep)));
    in.op = ldv<D>(O, (uint64_t)(base + (y + 1 == L ? -ywrap : ystep)));
    if constexpr (DIM == 3) {
        const int64_t zstep = (int64_t)L * ystep, zwrap = (int64_t)(L - 1) * zstep;
        in.zm = ldv<D>(O, (uint64_t)(base + (z == 0 ? zwrap : -zstep)));
        in.zp = ldv<D>(O, (uint64_t)(base + (z + 1 == L ? -zwrap : zstep)));
    }
}

// RAG: a ragged row (edge_words).
template <int KIND, int DIM, int D, int P, bool RAG>
__device__ __forceinline__ void rows_update(const RowsIn<DIM, D>& in, const SweepArgs& a, const RowGeom& rg,
                                            const RowsAt& at, const Lanes& ln, const PhiloxKey& ks,
                                            const RowLuts& lut, uint64_t thr_up, uint64_t thr_down, Obs& o,
                                            const Words4* pre)
{
    const uint64_t row = (uint64_t)at.z * rg.L + at.y;
    const uint64_t cb = 4ull * ln.col0;
    const Vec<D> q0 = prepv<KIND, D>(in.o0);
    uint32_t last, first;
    const uint32_t uncounted = edge_words<D, P, RAG>(q0, rg, ln, last, first);
    const uint32_t x = shift_in<false, P>(last, first, ln, 0u);
    uint32_t side[D];
    side_words<D, P>(q0, x, side);
    const Vec<D> qm = prepv<KIND, D>(in.om);
    const Vec<D> qp = prepv<KIND, D>(in.op);
    Vec<D> qzm, qzp;
    if constexpr (DIM == 3) {
        qzm = prepv<KIND, D>(in.zm);
        qzp = prepv<KIND, D>(in.zp);
    }
    const uint32_t g0 = (uint32_t)(row * rg.ncols + ln.col0);
    const Vec<D> nw = row_update<KIND, DIM, D, P, RAG>(in.own, q0, side, qm, qp, &qzm, &qzp, g0, a.colour, a.t, ks,
                                                       lut, thr_up, thr_down, true, o, pre, uncounted);
    stv<D>(colour_array(a, a.colour), row * rg.Lh + cb, nw);
}

// Ragged-row handling of a kernel: none, or every row (rg.rag != 0).  Each
// gets kernels of its own: a runtime branch between the two updates slowed
// the plain rows.
enum RagMode { kRagNone = 0, kRagAll = 1 };

template <int KIND, int DIM, int D, int RAGS>
__device__ __forceinline__ void rows_step(const RowsIn<DIM, D>& in, const SweepArgs& a, const RowGeom& rg,
                                          const RowsAt& at, const Lanes& ln, const PhiloxKey& ks, const RowLuts& lut,
                                          uint64_t thr_up, uint64_t thr_down, Obs& o)
{
    if (!at.ok) return;
    // Ising: the words' random numbers do not depend on the lattice, so they
    // are drawn here, before the first use of the loaded rows, while the loads
    // are still in flight (the scheduling barrier keeps that order).  Spin-1
    // with four words per lane would hold 32 words and spill: it draws late.
    constexpr bool kPre = KIND == KIND_ISING_HALF || (KIND == KIND_ISING_ONE && D <= 2);
    constexpr int kCalls = KIND == KIND_ISING_ONE ? 2 : 1;  // Philox calls per word
    Words4 pre[kPre ? kCalls * D : 1];
    if constexpr (kPre) {
        const uint32_t g0 = (uint32_t)(((uint64_t)at.z * rg.L + at.y) * rg.ncols + ln.col0);
#pragma unroll
        for (int i = 0; i < kCalls * D; ++i) pre[i] = philox4x32_10(kCalls * g0 + i, a.colour, a.t, 0u, ks);
        __builtin_amdgcn_sched_barrier(0);
    }
    const Words4* const pw = kPre ? pre : nullptr;
    // the row parity is uniform across the wave: every row of a row set has
    // the parity of rem & 1
    const bool p1 = ((at.y + at.z + a.colour) & 1u) != 0;
    constexpr bool kRag = D > 1 && (KIND == KIND_ISING_HALF || KIND == KIND_ISING_ONE) && RAGS == kRagAll;
    if constexpr (kRag) {
        if (!p1) rows_update<KIND, DIM, D, 0, kRag>(in, a, rg, at, ln, ks, lut, thr_up, thr_down, o, pw);
        else rows_update<KIND, DIM, D, 1, kRag>(in, a, rg, at, ln, ks, lut, thr_up, thr_down, o, pw);
    } else {
        if (!p1) rows_update<KIND, DIM, D, 0, false>(in, a, rg, at, ln, ks, lut, thr_up, thr_down, o, pw);
        else rows_update<KIND, DIM, D, 1, false>(in, a, rg, at, ln, ks, lut, thr_up, thr_down, o, pw);
    }
}

// Row groups of one wave at most; the row sets per plane go to nstrips, the
// launch's to nitems, the threads per block (waves >= 1 waves of 64, at most
// 16) to block.  `ragged`: rows whose word count D does not divide are
// accepted (Ising kinds only).
inline bool make_rows_geom(const Geom& g, int D, int waves, RowGeom& rg, bool ragged)
{
    if (waves < 1 || waves > 16 || !make_row_geom(g, 1, D, false, rg, ragged) || rg.R > 64) return false;
    rg.nstrips = 2 * cdiv(g.L, 2 * rg.slots);
    rg.nitems = rg.nstrips * rg.nplanes;
    rg.block = 64u * (uint32_t)waves;
    rg.K = 4u / rg.D;
    return true;
}

// Row sets it0 .. it0 + K - 1 of one wave (it0 wave-uniform, K = 4 / D).  Every thread of
// the block calls this: the table build inside ends in a workgroup barrier.
template <int KIND, int DIM, int D, int RAGS>
__device__ __forceinline__ void rows_run(const SweepArgs& a, const RowGeom& rg, uint32_t it0, const Lanes& ln,
                                         const uint64_t* table, RowLuts& lut, Obs& o)
{
    uint64_t thr_up, thr_down;
    build_row_luts<KIND, DIM>(lut, table, thr_up, thr_down);
    lds_barrier();
    const PhiloxKey ks = philox_schedule(a.key0, a.key1);
    constexpr uint32_t K = 4 / D;  // rg.K
    if constexpr (D == 1) {
        // one word per lane leaves registers to spare: both row sets of a
        // pair are loaded before either is updated, so the second set's loads
        // overlap the first set's work
#pragma nounroll
        for (uint32_t k = 0; k < K; k += 2) {
            const RowsAt at0 = rows_at(rg, it0 + k, ln.slot), at1 = rows_at(rg, it0 + k + 1, ln.slot);
            RowsIn<DIM, D> in0, in1;
            rows_load<DIM, D>(in0, a, rg, at0, ln);
            rows_load<DIM, D>(in1, a, rg, at1, ln);
            rows_step<KIND, DIM, D, RAGS>(in0, a, rg, at0, ln, ks, lut, thr_up, thr_down, o);
            rows_step<KIND, DIM, D, RAGS>(in1, a, rg, at1, ln, ks, lut, thr_up, thr_down, o);
        }
    } else {
#pragma nounroll
        for (uint32_t k = 0; k < K; ++k) {
            const RowsAt at = rows_at(rg, it0 + k, ln.slot);
            RowsIn<DIM, D> in;
            rows_load<DIM, D>(in, a, rg, at, ln);
            rows_step<KIND, DIM, D, RAGS>(in, a, rg, at, ln, ks, lut, thr_up, thr_down, o);
        }
    }
}

}  // namespace rowk
}  // namespace spinlat
