// host_logic.cpp -- pure host logic of the library (declared in
// host_logic.h): validation of a lattice's parameters, the layout of the
// caller's device buffer, the Metropolis threshold table in double precision
// (paper Sec. 3.1: P_acc = min[1, exp(-dE/T)]; Sec. 3.2 for the NE model), the
// overflow-safe checks on sweep counts and the first-fit allocator of a batch
// arena.  No HIP call: this file also builds with g++ under sanitizers.
#include "host_logic.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <iterator>

namespace spinlat {
namespace host {

thread_local char g_err[512] = "";

const char* last_error() { return g_err; }

sl_status fail(sl_status st, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return st;
}

bool is_sub_lattice(int model) { return model == SL_NE_SUBLATTICE || model == SL_NE_SUBLATTICE_BALANCED; }

// Sweep indices stay below this: the launch index (2 or 4 per sweep) is 32-bit.
uint64_t sweep_limit(int model)
{
    if (model == SL_NE_SUBLATTICE) return 1ull << 31;
    if (model == SL_NE_SUBLATTICE_BALANCED) return 1ull << 30;
    return 1ull << 32;
}

int kind_of(const sl_params* p)
{
    if (p->model != SL_ISING) return KIND_NE;
    return p->two_s == 1 ? KIND_ISING_HALF : KIND_ISING_ONE;
}

sl_status validate(const sl_params* p)
{
    if (!p) return fail(SL_E_INVALID, "params is NULL");
    if (p->abi_version != SL_ABI_VERSION)
        return fail(SL_E_INVALID, "abi_version %u != %u", p->abi_version, SL_ABI_VERSION);
    if (p->model != SL_ISING && p->model != SL_NORTH_EAST && p->model != SL_NE_SUBLATTICE &&
        p->model != SL_NE_SUBLATTICE_BALANCED && p->model != SL_NE_COUPLED)
        return fail(SL_E_INVALID, "unknown model %d", p->model);
    if (p->dim != 2 && p->dim != 3) return fail(SL_E_INVALID, "dim must be 2 or 3 (got %d)", p->dim);
    if (p->L < 2 || (p->L & 1))
        return fail(SL_E_INVALID, "L must be even and >= 2 (got %d): the checkerboard needs a "
                                  "bipartite periodic lattice", p->L);
    if (p->two_s != 1 && p->two_s != 2)
        return fail(SL_E_INVALID, "two_s must be 1 (spin-1/2) or 2 (spin-1), got %d", p->two_s);
    if (p->init != SL_INIT_COLD && p->init != SL_INIT_RANDOM && p->init != SL_INIT_BUFFER)
        return fail(SL_E_INVALID, "unknown init %d", p->init);
    if (p->init == SL_INIT_BUFFER && !p->init_spins)
        return fail(SL_E_INVALID, "SL_INIT_BUFFER needs init_spins");
    if (p->model == SL_ISING || p->model == SL_NE_COUPLED) {
        if (!(p->T > 0.0)) return fail(SL_E_INVALID, "T must be > 0 (got %g)", p->T);
        if (std::isnan(p->J) || std::isnan(p->h) || std::isinf(p->J) || std::isinf(p->h))
            return fail(SL_E_INVALID, "J and h must be finite");
    }
    if (p->model != SL_ISING) {
        if (p->dim != 2) return fail(SL_E_INVALID, "the North-East model is two-dimensional");
        if (p->two_s != 1) return fail(SL_E_INVALID, "the North-East model has binary sites");
        if (!(p->c > 0.0 && p->c < 1.0))
            return fail(SL_E_INVALID, "c must lie in (0, 1) (got %g)", p->c);
        if (p->init == SL_INIT_COLD)
            return fail(SL_E_INVALID, "NE lattices start from Bernoulli(c) or a buffer");
    }
    if (is_sub_lattice(p->model)) {
        const bool bal = p->model == SL_NE_SUBLATTICE_BALANCED;
        const int B = p->ne_side, lam = p->ne_lambda, per = bal ? 8 : 2;
        if (B < 2 || (B & 1) || lam < 1 || p->L % B != 0 || (B * B) % (per * lam) != 0)
            return fail(SL_E_INVALID, "sub-lattices need an even B with L %% B == 0 and "
                                      "B^2 %% (%d lambda) == 0 (L %d, B %d, lambda %d)",
                        per, p->L, B, lam);
        if (!ne_sub_supported((uint32_t)p->L, B, lam, bal))
            return fail(SL_E_UNSUPPORTED, "the sub-lattice kernels take B in {8,16,32,64} and "
                                          "lambda a power of two in [2,128] (B %d, lambda %d)",
                        B, lam);
        if (p->t0 >= sweep_limit(p->model))
            return fail(SL_E_OVERFLOW, "t0 must be < %llu (launch indices are 32-bit)",
                        (unsigned long long)sweep_limit(p->model));
    }
    if (p->t0 >= (1ull << 32)) return fail(SL_E_OVERFLOW, "t0 must be < 2^32");
    if (p->record_capacity < 1 || p->record_capacity > (1ull << 32))
        return fail(SL_E_INVALID, "record_capacity must be in [1, 2^32]");
    if (p->L % 8 != 0)
        return fail(SL_E_UNSUPPORTED, "kernels need L %% 8 == 0 (got %d)", p->L);
    // the first counter word holds the Philox group index (k / G) in 32 bits
    const uint64_t nsites = p->dim == 2 ? (uint64_t)p->L * p->L : (uint64_t)p->L * p->L * p->L;
    const uint64_t groups = (nsites / 2) / (p->two_s == 1 ? 4 : 2);
    if (groups > (1ull << 32))
        return fail(SL_E_UNSUPPORTED, "lattice too large for the 32-bit Philox group index");
    return SL_OK;
}

Layout layout_of(const sl_params* p)
{
    Layout l{};
    l.nsites = p->dim == 2 ? (uint64_t)p->L * p->L : (uint64_t)p->L * p->L * p->L;
    l.nh = l.nsites / 2;
    l.col_bytes = round_up(l.nh, kAlign);
    for (int b = 0; b < 2; ++b)
        for (int c = 0; c < 2; ++c) l.off_col[b][c] = (size_t)(2 * b + c) * l.col_bytes;
    l.off_acc = 4 * l.col_bytes;
    l.off_out = l.off_acc + round_up(p->record_capacity * kSlotWords * sizeof(int64_t), kAlign);
    l.off_lut = l.off_out + round_up(p->record_capacity * kRecordWords * sizeof(int64_t), kAlign);
    l.total = l.off_lut + round_up(kMaxLut * sizeof(uint64_t), kAlign);
    return l;
}

// ---- Metropolis thresholds (double precision, host) ------------------------

uint64_t thr_from_prob(double pr)
{
    if (!(pr < 1.0)) return 1ull << 32;
    if (!(pr > 0.0)) return 0;
    return (uint64_t)std::floor(pr * 4294967296.0);
}

uint64_t thr_from_energy(double dE, double T)
{
    if (dE <= 0.0) return 1ull << 32;
    return thr_from_prob(std::exp(-dE / T));
}

size_t build_table(const sl_params* p, uint64_t* out)
{
    if (p->model != SL_ISING && p->model != SL_NE_COUPLED) {
        out[0] = thr_from_prob(p->c / (1.0 - p->c));  // up-flip: energy +1
        out[1] = thr_from_prob((1.0 - p->c) / p->c);  // down-flip
        return 2;
    }
    const int z = 2 * p->dim;
    const int ds_of[4] = {-2, -1, 1, 2};
    size_t n = 0;
    for (int di = 0; di < 4; ++di)
        for (int nsum = -z; nsum <= z; ++nsum) {
            const double dE = -(double)ds_of[di] * (p->J * (double)nsum + p->h);
            out[n++] = thr_from_energy(dE, p->T);
        }
    return n;
}


bool ne_sub_supported(uint32_t L, int B, int lambda, bool balanced)
{
    if (B != 8 && B != 16 && B != 32 && B != 64) return false;
    if (L % (uint32_t)B != 0) return false;
    if (lambda < 2 || lambda > 128 || (lambda & (lambda - 1)) != 0) return false;
    return (balanced ? 8 : 2) * lambda <= B * B;
}

sl_status check_sweep_count(uint64_t pending, uint64_t capacity, uint64_t next_t, uint64_t t_end,
                            uint64_t n)
{
    const uint64_t room = capacity > pending ? capacity - pending : 0;
    if (n > room)
        return fail(SL_E_STATE, "%llu unread records + %llu sweeps exceed record_capacity %llu; "
                                "call sl_measure first", (unsigned long long)pending,
                    (unsigned long long)n, (unsigned long long)capacity);
    const uint64_t left = t_end > next_t ? t_end - next_t : 0;
    if (n > left)
        return fail(SL_E_OVERFLOW, "sweep index would reach %llu", (unsigned long long)t_end);
    return SL_OK;
}

void FreeList::reset(size_t start, size_t bytes)
{
    free_.clear();
    if (bytes) free_[start] = bytes;
}

bool FreeList::alloc(size_t bytes, size_t* off)
{
    for (auto it = free_.begin(); it != free_.end(); ++it) {
        if (it->second >= bytes) {
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t roff = it->first + bytes;
            free_.erase(it);
            if (rest) free_[roff] = rest;
            return true;
        }
    }
    return false;
}

void FreeList::release(size_t off, size_t bytes)
{
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
        it->second += next->second;
        free_.erase(next);
    }
    if (it != free_.begin()) {
        auto prev = std::prev(it);
        if (prev->first + prev->second == it->first) {
            prev->second += it->second;
            free_.erase(it);
        }
    }
}

size_t FreeList::free_bytes() const
{
    size_t s = 0;
    for (const auto& kv : free_) s += kv.second;
    return s;
}

}  // namespace host
}  // namespace spinlat
