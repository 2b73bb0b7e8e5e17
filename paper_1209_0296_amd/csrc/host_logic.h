// host_logic.h -- the pure host logic of the library: parameter validation,
// device-buffer layout, the double-precision Metropolis threshold table, the
// checks on sweep counts, and the first-fit allocator of a batch arena.
//
// Nothing here calls the HIP runtime or includes its headers, so the same
// source also builds with a plain host compiler under AddressSanitizer and
// UndefinedBehaviorSanitizer (tests/host_checks.cpp).
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <map>

#include "../../include/spinlat.h"

namespace spinlat {

// Per-record accumulators: kSub sub-slots spread the workgroups' atomics, each
// on a 128-byte line of its own (atomics on one line serialise: with the four
// sub-slots of a line shared by 2048 workgroups a launch took 7.4 us instead
// of 2.3 us); a sub-slot holds kQ int64 quantities.
constexpr int kSub = 16;
constexpr int kQ = 4;           // bond_sum, mag, accepted, unflipped
constexpr int kSubStride = 16;  // int64 words per sub-slot (one 128-byte line)
constexpr int kSlotWords = kSub * kSubStride;
constexpr int kRecordWords = 5;  // t, bond_sum, mag, accepted, unflipped
constexpr int kMaxLut = 64;      // >= 4*(4*3+1) = 52 Ising entries

enum Kind : int { KIND_ISING_HALF = 0, KIND_ISING_ONE = 1, KIND_NE = 2 };

namespace host {

constexpr size_t kAlign = 256;
inline size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Layout {
    uint64_t nsites;   // L^dim
    uint64_t nh;       // per colour
    size_t col_bytes;  // one colour array, rounded to kAlign
    size_t off_col[2][2];  // [copy][colour]: two copies of the lattice (fused sweeps
                           // read one and write the other)
    size_t off_acc;    // accumulators [capacity][kSub][kQ] int64
    size_t off_out;    // folded records [capacity][5] int64
    size_t off_lut;    // threshold table, kMaxLut u64
    size_t total;
};

const char* last_error();
sl_status fail(sl_status st, const char* fmt, ...);
int kind_of(const sl_params* p);
bool is_sub_lattice(int model);  // SL_NE_SUBLATTICE or its balanced variant
uint64_t sweep_limit(int model);  // sweep indices stay below this
// Shapes the NE sub-lattice kernels take: B in {8, 16, 32, 64}, L % B == 0,
// lambda a power of two in [2, 128], 2 lambda <= B^2 (balanced: 8 lambda).
bool ne_sub_supported(uint32_t L, int B, int lambda, bool balanced);
sl_status validate(const sl_params* p);  // full validation of a lattice's parameters
Layout layout_of(const sl_params* p);
uint64_t thr_from_prob(double pr);
uint64_t thr_from_energy(double dE, double T);
size_t build_table(const sl_params* p, uint64_t* out);  // FP64 Metropolis thresholds

// May n more sweeps be enqueued?  pending <= capacity unread records are
// held, and the next sweep index is next_t <= t_end.  SL_E_STATE when the
// records would not fit, SL_E_OVERFLOW when a sweep index would reach t_end;
// written so that no sum can wrap, whatever n is.
sl_status check_sweep_count(uint64_t pending, uint64_t capacity, uint64_t next_t, uint64_t t_end,
                            uint64_t n);

// First-fit allocator of a batch arena's heap: free ranges keyed by offset,
// coalesced with their neighbours on release.  All sizes are multiples of
// kAlign.
class FreeList {
public:
    void reset(size_t start, size_t bytes);  // one free range [start, start + bytes)
    bool alloc(size_t bytes, size_t* off);   // lowest-offset range that fits
    void release(size_t off, size_t bytes);
    size_t free_bytes() const;
    size_t ranges() const { return free_.size(); }
    const std::map<size_t, size_t>& map() const { return free_; }

private:
    std::map<size_t, size_t> free_;  // offset -> size
};

}  // namespace host
}  // namespace spinlat
