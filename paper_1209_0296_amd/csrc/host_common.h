// host_common.h -- host helpers shared by the lattice and batch runtimes.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/spinlat.h"

namespace spinlat {
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
sl_status hip_fail(hipError_t e, const char* what);
int kind_of(const sl_params* p);
bool is_sub_lattice(int model);  // SL_NE_SUBLATTICE or its balanced variant
uint64_t sweep_limit(int model);  // sweep indices stay below this
sl_status validate(const sl_params* p);  // full validation of a lattice's parameters
Layout layout_of(const sl_params* p);
uint64_t thr_from_prob(double pr);
uint64_t thr_from_energy(double dE, double T);
size_t build_table(const sl_params* p, uint64_t* out);  // FP64 Metropolis thresholds

}  // namespace host
}  // namespace spinlat
