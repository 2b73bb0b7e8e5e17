// runtime.cpp -- host side of the C ABI declared in include/spinlat.h.
//
// Responsibilities: validate parameters, lay out the caller's device buffer,
// build the Metropolis threshold table in double precision (paper Sec. 3.1:
// P_acc = min[1, exp(-dE/T)]; Sec. 3.2 for the NE model), enqueue the
// kernels on the caller's stream (one sweep = colour 0 then colour 1, Alg. I
// steps 5-7; a kernel boundary, or a workgroup barrier in the resident mode,
// separates the colours; the NE sub-lattice algorithms of Sec. 3.2 take two or
// four launches per sweep), drain the per-sweep record ring, and evaluate the
// observables of records and lattices.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "../../include/spinlat.h"
#include "host_common.h"
#include "runtime_internal.h"
#include "spinlat_internal.h"

using namespace spinlat;

namespace spinlat {
namespace host {

sl_status hip_fail(hipError_t e, const char* what)
{
    return fail(SL_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace host
}  // namespace spinlat

using namespace spinlat::host;

namespace {

// NE records count over the occupations n = (s + 1) / 2.  On a 2D lattice of
// N sites and 2N forward bonds, each site in four of them:
// sum s_i s_j = 4 bond - 8 mag + 2N and sum s_i = 2 mag - N.
void spin_sums(const sl_record& r, double nsites, double& bond, double& mag)
{
    bond = 4.0 * (double)r.bond_sum - 8.0 * (double)r.mag + 2.0 * nsites;
    mag = 2.0 * (double)r.mag - nsites;
}

// (bond, mag) in spin variables for the statistics of either energy model.
void stat_sums(const sl_params* p, const sl_record& r, double nsites, double& bond, double& mag)
{
    if (p->model == SL_NE_COUPLED) {
        spin_sums(r, nsites, bond, mag);
    } else {
        bond = (double)r.bond_sum;
        mag = (double)r.mag;
    }
}

}  // namespace


namespace spinlat {
namespace rt {

void release(sl_lattice* h)
{
    if (h->stage) (void)hipHostFree(h->stage);
    delete h;
}

SweepArgs args_of(const sl_lattice* h)
{
    SweepArgs a{};
    a.col[0] = h->base + h->lay.off_col[h->cur][0];
    a.col[1] = h->base + h->lay.off_col[h->cur][1];
    a.g.L = (uint32_t)h->params.L;
    a.g.Lh = (uint32_t)(h->params.L / 2);
    a.g.dim = (uint32_t)h->params.dim;
    a.g.rows = h->params.dim == 2 ? a.g.L : a.g.L * a.g.L;
    a.g.nh = h->lay.nh;
    a.key0 = (uint32_t)h->params.seed;
    a.key1 = (uint32_t)(h->params.seed >> 32);
    a.lut = reinterpret_cast<const uint64_t*>(h->base + h->lay.off_lut);
    a.lut_n = (int32_t)h->table_n;
    a.update = 1;
    a.tile_rows = h->launch.tile_rows;
    a.tile_words = h->launch.tile_words;
    return a;
}

unsigned long long* slot_ptr(const sl_lattice* h, uint64_t idx)
{
    return reinterpret_cast<unsigned long long*>(h->base + h->lay.off_acc) + idx * kSlotWords;
}

bool lut32_ok(const sl_lattice* h)
{
    for (size_t i = 0; i < h->table_n; ++i)
        if (h->table[i] == 0) return false;
    return true;
}

// Default schedule for a shape, from the schedule autotuner's timings on
// MI355X (us per sweep):
//   - lattices of at most 16 KiB run resident in LDS (2D L = 64: 2.4);
//   - 2D up to L = 1024: fused with 2-row strips, 1 word per lane (L = 1024:
//     4.9 against 6.1 with 2 words); L = 2048: fused, 2-row strips, 2 words;
//   - 2D L = 4096: fused, 4-row strips, 2 words (spin-1/2: 14.6 against 17.7
//     with 4 words); L = 8192 spin-1/2 takes 16-row strips with 2 words per
//     lane (38.3 against 39.8 with 8-row strips and 4 words, 40.5 with 16
//     rows and 4 words, 42.2 with 32 rows and 1 word), and from L = 16384
//     32-row strips with 4 words (16384: 133.7 against 141.4 with 16 rows;
//     32768: 538 against 569); spin-1 takes 16-row strips with 2 words from
//     L = 8192 (68.3 against 80.7 with 4-row strips); NE takes 8-row strips
//     with 1 word at L = 4096 (17.1 against 17.6 with 4 rows and 2 words)
//     and 4-row strips with 2 words from 8192; coupled NE keeps 4-row strips
//     with 2 words;
//   - 3D: half-sweeps by independent row groups with 4 words per lane (L =
//     256: 18.4 against 19.2 for the walk with 4-row strips; L = 64: 7.4
//     against 8.8 with 2 words and 9.8 with 1; L = 128: 7.7 against 10.0 with
//     1), also when 4 does not divide the row (Ising rows may be ragged: L =
//     136: 8.7 against 13.0 with 1 word; L = 200: 13.1 against 22.1; spin-1
//     at 200: 18.2 against 25.6); spin-1/2 takes blocks of 8 waves from L =
//     256 (17.3 against 17.6 with 4), else 4 (L = 128: 7.7 against 8.6;
//     spin-1 at 256: 24.7 against 24.9).
// A fused 3D sweep would recompute a halo in two directions, so 3D uses
// half-sweeps.  Other widths are tried in order when a row does not fit, and
// shapes the whole-row kernels cannot take fall back to the window kernels.
constexpr uint64_t kResidentAuto = 16 * 1024;

sl_launch auto_launch(const sl_lattice* h)
{
    const Geom g = {(uint32_t)h->params.L, (uint32_t)(h->params.L / 2), (uint32_t)h->params.dim,
                    0u, h->lay.nh};
    if (2 * h->lay.nh <= kResidentAuto) {  // launch-bound sizes: all sweeps in one launch
        sl_launch r{};
        r.mode = SL_MODE_RESIDENT;
        return r;
    }
    const bool coupled = h->params.model == SL_NE_COUPLED;
    if (coupled && !lut32_ok(h)) {  // the row kernels keep "word <= thr - 1" in 32 bits
        sl_launch r{};
        r.mode = SL_MODE_SIMPLE;
        return r;
    }
    const int L = h->params.L;
    const bool half_spin = h->kind == KIND_ISING_HALF;
    sl_launch l{};
    if (h->params.dim == 3) {
        const int Ds[3] = {4, 2, 1};
        const int waves = L >= 256 && half_spin ? 8 : 4;
        for (int D : Ds)
            if (rows_supported(g, h->kind, waves, D, lut32_ok(h))) {
                l.mode = SL_MODE_HALF_ROWS;
                l.tile_rows = waves;
                l.tile_words = D;
                return l;
            }
    }
    const bool fused = h->params.dim == 2;
    int H = 4, Ds[3] = {4, 2, 1};
    if (h->params.dim == 3) {
        if (L <= 160) {
            H = 2;
            Ds[0] = 1, Ds[1] = 2, Ds[2] = 4;
        }
    } else if (L <= 1024) {
        H = 2;
        Ds[0] = 1, Ds[1] = 2, Ds[2] = 4;
    } else if (L <= 2048) {
        H = 2;
        Ds[0] = 2, Ds[1] = 1, Ds[2] = 4;
    } else if (h->params.model == SL_NORTH_EAST && L < 8192) {
        H = 8;
        Ds[0] = 1, Ds[1] = 2, Ds[2] = 4;
    } else if (L < 8192 || !(half_spin || h->kind == KIND_ISING_ONE)) {
        H = 4;
        Ds[0] = 2, Ds[1] = 4, Ds[2] = 1;
    } else if (L >= 16384 && half_spin) {
        H = 32;
    } else {
        H = 16;
        Ds[0] = 2, Ds[1] = 4, Ds[2] = 1;
    }
    for (int D : Ds)
        if (row_supported(g, h->kind, H, D, fused, lut32_ok(h))) {
            l.mode = fused ? SL_MODE_FUSED : SL_MODE_HALF;
            l.tile_rows = H;
            l.tile_words = D;
            return l;
        }
    l.mode = coupled ? SL_MODE_SIMPLE : fused ? SL_MODE_FUSED_WINDOW : SL_MODE_HALF_WINDOW;
    l.tile_rows = 0;
    l.tile_words = 0;
    return l;
}

sl_status check_launch(const sl_lattice* h, sl_launch* l)
{
    if (is_sub_lattice(h->params.model)) {
        if (l->mode != SL_MODE_AUTO)
            return fail(SL_E_UNSUPPORTED, "NE sub-lattice lattices have one schedule (SL_MODE_AUTO)");
        return SL_OK;
    }
    const Geom g = {(uint32_t)h->params.L, (uint32_t)(h->params.L / 2), (uint32_t)h->params.dim,
                    0u, h->lay.nh};
    if (h->params.model == SL_NE_COUPLED) {
        const bool row = l->mode == SL_MODE_HALF || l->mode == SL_MODE_FUSED || l->mode == SL_MODE_HALF_ROWS;
        if (!(l->mode == SL_MODE_SIMPLE || l->mode == SL_MODE_RESIDENT || (row && lut32_ok(h))))
            return fail(SL_E_UNSUPPORTED, "coupled NE lattices run SL_MODE_SIMPLE, SL_MODE_RESIDENT, "
                                          "or SL_MODE_HALF / SL_MODE_FUSED / SL_MODE_HALF_ROWS when every "
                                          "threshold is >= 1");
    }
    switch (l->mode) {
        case SL_MODE_SIMPLE:
            return SL_OK;
        case SL_MODE_RESIDENT:
            if (!resident_supported(g) || l->tile_rows != 0 || l->tile_words != 0)
                return fail(SL_E_UNSUPPORTED, "the resident mode holds at most %d bytes of lattice "
                            "(this one has %llu) and takes no tile sizes", kResidentLds,
                            (unsigned long long)(2 * h->lay.nh));
            return SL_OK;
        case SL_MODE_HALF:
        case SL_MODE_FUSED: {
            const bool fused = l->mode == SL_MODE_FUSED;
            if (l->tile_rows == 0) l->tile_rows = 8;
            if (l->tile_words == 0) {  // first width that fits
                l->tile_words = 2;
                for (int D : {2, 4, 1})
                    if (row_supported(g, h->kind, l->tile_rows, D, fused, lut32_ok(h))) {
                        l->tile_words = D;
                        break;
                    }
            }
            if (!row_supported(g, h->kind, l->tile_rows, l->tile_words, fused, lut32_ok(h)))
                return fail(SL_E_UNSUPPORTED, "mode %d with %d rows x %d words per lane does not fit "
                            "this lattice", l->mode, l->tile_rows, l->tile_words);
            return SL_OK;
        }
        case SL_MODE_HALF_ROWS:
            if (l->tile_rows == 0) l->tile_rows = 4;
            if (l->tile_words == 0)
                for (int D : {4, 2, 1})
                    if (rows_supported(g, h->kind, l->tile_rows, D, lut32_ok(h))) {
                        l->tile_words = D;
                        break;
                    }
            if (!rows_supported(g, h->kind, l->tile_rows, l->tile_words, lut32_ok(h)))
                return fail(SL_E_UNSUPPORTED, "SL_MODE_HALF_ROWS with %d waves per workgroup and %d words "
                            "per lane does not fit this lattice", l->tile_rows, l->tile_words);
            return SL_OK;
        case SL_MODE_HALF_WINDOW:
        case SL_MODE_FUSED_WINDOW:
            if (!tiled_supported(g, h->kind, l->tile_rows, l->tile_words,
                                 l->mode == SL_MODE_FUSED_WINDOW))
                return fail(SL_E_UNSUPPORTED, "window mode %d with %d rows x %d words does not fit "
                            "this lattice", l->mode, l->tile_rows, l->tile_words);
            return SL_OK;
    }
    return fail(SL_E_INVALID, "unknown launch mode %d", l->mode);
}

// Record of the current state without any update (r_0): both colours with
// update = 0 through the direct kernel.
sl_status enqueue_observe(sl_lattice* h, uint64_t slot)
{
    SweepArgs a = args_of(h);
    a.update = 0;
    a.acc = slot_ptr(h, slot);
    for (uint32_t c = 0; c < 2; ++c) {
        a.colour = c;
        hipError_t e = launch_simple_half(a, h->kind, h->stream);
        if (e != hipSuccess) return hip_fail(e, "observe kernel");
    }
    return SL_OK;
}

// Paper Sec. 3.2, NE algorithm with random sub-lattices: per sweep, launch
// 2t reads the current copy and writes the other, launch 2t+1 reads that and
// writes the current copy back (balanced variant: launches 4t .. 4t+3,
// alternating the copies the same way).  All add their accepted counts to
// the sweep's record slot.  The lattice part of a sweep's record is measured by
// the first launch of the next sweep from the state it loads; after the last
// sweep of the call a separate pass (both colours, no update) measures it.
sl_status sweep_ne_sub(sl_lattice* h, uint64_t n)
{
    const int B = h->params.ne_side, lam = h->params.ne_lambda;
    const bool bal = h->params.model == SL_NE_SUBLATTICE_BALANCED;
    const int per = bal ? 4 : 2;  // launches per sweep
    const uint32_t L = (uint32_t)h->params.L;
    NeSubArgs na{};
    na.L = L;
    na.Lh = L / 2;
    na.tiles_x = L / (uint32_t)B;
    na.ntiles = na.tiles_x * na.tiles_x;
    na.key0 = (uint32_t)h->params.seed;
    na.key1 = (uint32_t)(h->params.seed >> 32);
    // thresholds in [0, 2^32] as 32-bit "word <= thr - 1" with a flag for 0
    na.thr_m1_up = h->table[0] ? (uint32_t)(h->table[0] - 1) : 0u;
    na.thr_m1_down = h->table[1] ? (uint32_t)(h->table[1] - 1) : 0u;
    na.never = (h->table[0] == 0 ? 1u : 0u) | (h->table[1] == 0 ? 2u : 0u);
    uint8_t* cur[2] = {h->base + h->lay.off_col[h->cur][0], h->base + h->lay.off_col[h->cur][1]};
    uint8_t* oth[2] = {h->base + h->lay.off_col[h->cur ^ 1][0],
                       h->base + h->lay.off_col[h->cur ^ 1][1]};
    for (uint64_t i = 0; i < n; ++i) {
        const uint64_t t = h->next_t + i;
        na.acc = slot_ptr(h, h->pending + i);
        hipError_t e = hipSuccess;
        for (int k = 0; k < per && e == hipSuccess; ++k) {
            uint8_t** from = (k & 1) == 0 ? cur : oth;
            uint8_t** to = (k & 1) == 0 ? oth : cur;
            na.src[0] = from[0];
            na.src[1] = from[1];
            na.dst[0] = to[0];
            na.dst[1] = to[1];
            na.launch = (uint32_t)((uint64_t)per * t + (uint64_t)k);
            na.obs = (k == 0 && i > 0) ? slot_ptr(h, h->pending + i - 1) : nullptr;
            e = launch_ne_sub(na, B, lam, bal, h->stream);
        }
        sl_status st = SL_OK;
        if (e != hipSuccess) {
            st = hip_fail(e, "sub-lattice launch");
            if (i > 0) (void)enqueue_observe(h, h->pending + i - 1);
        } else if (i + 1 == n) {
            st = enqueue_observe(h, h->pending + i);
        }
        if (st != SL_OK) {
            h->next_t += i;
            h->pending += i;
            return st;
        }
    }
    h->next_t += n;
    h->pending += n;
    return SL_OK;
}

// Enqueue n sweeps (the caller has checked the count): the launches of the
// lattice's schedule, records into ring slots pending .. pending + n - 1.
sl_status enqueue_sweeps(sl_lattice* h, uint64_t n)
{
    if (is_sub_lattice(h->params.model)) return sweep_ne_sub(h, n);
    SweepArgs a = args_of(h);
    if (h->launch.mode == SL_MODE_RESIDENT) {
        for (uint64_t i = 0; i < n;) {
            const uint32_t k = (uint32_t)std::min<uint64_t>(n - i, kResidentChunk);
            a.t = (uint32_t)(h->next_t + i);
            a.acc = slot_ptr(h, h->pending + i);
            hipError_t e = launch_resident(a, h->kind, k, h->stream);
            if (e != hipSuccess) {
                h->next_t += i;
                h->pending += i;
                return hip_fail(e, "resident sweep launch");
            }
            i += k;
        }
        h->next_t += n;
        h->pending += n;
        return SL_OK;
    }
    for (uint64_t i = 0; i < n; ++i) {
        a.t = (uint32_t)(h->next_t + i);
        a.acc = slot_ptr(h, h->pending + i);
        hipError_t e = hipSuccess;
        const int H = h->launch.tile_rows, D = h->launch.tile_words;
        switch (h->launch.mode) {
            case SL_MODE_FUSED:
            case SL_MODE_FUSED_WINDOW: {
                const int nxt = h->cur ^ 1;
                uint8_t* d0 = h->base + h->lay.off_col[nxt][0];
                uint8_t* d1 = h->base + h->lay.off_col[nxt][1];
                if (h->launch.mode == SL_MODE_FUSED)
                    e = launch_row_fused(a, h->kind, H, D, a.col[0], a.col[1], d0, d1, h->stream);
                else
                    e = launch_fused_sweep(a, h->kind, a.col[0], a.col[1], d0, d1, h->stream);
                if (e == hipSuccess) {
                    h->cur = nxt;
                    a.col[0] = d0;
                    a.col[1] = d1;
                }
                break;
            }
            case SL_MODE_HALF:
            case SL_MODE_HALF_WINDOW:
            case SL_MODE_HALF_ROWS:
                for (uint32_t c = 0; c < 2 && e == hipSuccess; ++c) {
                    a.colour = c;
                    if (h->launch.mode == SL_MODE_HALF) e = launch_row_half(a, h->kind, H, D, h->stream);
                    else if (h->launch.mode == SL_MODE_HALF_ROWS) e = launch_rows_half(a, h->kind, H, D, h->stream);
                    else e = launch_tiled_half(a, h->kind, h->stream);
                }
                break;
            default:
                for (uint32_t c = 0; c < 2 && e == hipSuccess; ++c) {
                    a.colour = c;
                    e = launch_simple_half(a, h->kind, h->stream);
                }
                break;
        }
        if (e != hipSuccess) {
            // sweeps before i were enqueued and will produce their records
            h->next_t += i;
            h->pending += i;
            return hip_fail(e, "sweep launch");
        }
    }
    h->next_t += n;
    h->pending += n;
    return SL_OK;
}

}  // namespace rt
}  // namespace spinlat

using namespace spinlat::rt;

extern "C" {

sl_status sl_query_bytes(const sl_params* params, size_t* device_bytes)
{
    sl_status st = validate(params);
    if (st != SL_OK) return st;
    if (!device_bytes) return fail(SL_E_INVALID, "device_bytes is NULL");
    *device_bytes = layout_of(params).total;
    return SL_OK;
}

sl_status sl_threshold_table(const sl_params* params, uint64_t* out, size_t cap, size_t* n_out)
{
    sl_status st = validate(params);
    if (st != SL_OK) return st;
    uint64_t tmp[kMaxLut];
    const size_t n = build_table(params, tmp);
    if (n_out) *n_out = n;
    if (!out || cap < n) return fail(SL_E_BUFFER, "table needs %zu entries", n);
    std::memcpy(out, tmp, n * sizeof(uint64_t));
    return SL_OK;
}

sl_status sl_create_lattice(const sl_params* params, void* device_buf, size_t bytes,
                            void* hip_stream, sl_lattice** out)
{
    sl_status st = validate(params);
    if (st != SL_OK) return st;
    if (!out) return fail(SL_E_INVALID, "out is NULL");
    *out = nullptr;
    const Layout lay = layout_of(params);
    if (!device_buf) return fail(SL_E_BUFFER, "device buffer is NULL");
    if (reinterpret_cast<uintptr_t>(device_buf) % kAlign != 0)
        return fail(SL_E_BUFFER, "device buffer must be %zu-byte aligned", kAlign);
    if (bytes < lay.total)
        return fail(SL_E_BUFFER, "device buffer has %zu bytes, needs %zu", bytes, lay.total);

    sl_lattice* h = new (std::nothrow) sl_lattice();
    if (!h) return fail(SL_E_STATE, "out of host memory");
    h->params = *params;
    h->lay = lay;
    h->base = static_cast<uint8_t*>(device_buf);
    h->stream = static_cast<hipStream_t>(hip_stream);
    h->kind = kind_of(params);
    h->next_t = params->t0;
    h->pending = 0;
    h->first_t = params->t0;
    h->cur = 0;
    h->table_n = build_table(params, h->table);
    h->launch = auto_launch(h);
    if (is_sub_lattice(params->model)) h->launch = sl_launch{};
    h->stage = nullptr;
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&h->stage),
                                 params->record_capacity * sizeof(sl_record), hipHostMallocDefault);
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e, "create: pinned record staging");
    }
    e = hipMemcpyAsync(h->base + lay.off_lut, h->table, h->table_n * sizeof(uint64_t),
                                  hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess)
        e = launch_fill_u64(slot_ptr(h, 0), params->record_capacity * kSlotWords, h->stream);
    if (e != hipSuccess) {
        release(h);
        return hip_fail(e, "create: table upload / ring clear");
    }
    SweepArgs a = args_of(h);
    if (params->init == SL_INIT_BUFFER) {
        e = launch_from_natural(a, params->init_spins, h->stream);
    } else {
        const uint64_t bern = thr_from_prob(params->c);
        e = launch_init(a, h->kind, params->init == SL_INIT_COLD ? 0 : 1, (uint32_t)bern,
                        (uint32_t)(bern >> 32), h->stream);
    }
    if (e != hipSuccess) {
        release(h);
        return hip_fail(e, "create: initial state");
    }
    st = enqueue_observe(h, 0);
    if (st != SL_OK) {
        release(h);
        return st;
    }
    h->pending = 1;
    // the table upload reads h->table; keep it alive until the copy is done
    e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        release(h);
        return hip_fail(e, "create: synchronise");
    }
    *out = h;
    return SL_OK;
}

sl_status sl_set_launch(sl_lattice* h, const sl_launch* launch)
{
    if (!h || !launch) return fail(SL_E_INVALID, "NULL argument");
    sl_launch l = *launch;
    if (l.mode == SL_MODE_AUTO && !is_sub_lattice(h->params.model)) l = auto_launch(h);
    sl_status st = check_launch(h, &l);
    if (st != SL_OK) return st;
    h->launch = l;
    return SL_OK;
}

sl_status sl_get_launch(const sl_lattice* h, sl_launch* launch)
{
    if (!h || !launch) return fail(SL_E_INVALID, "NULL argument");
    *launch = h->launch;
    return SL_OK;
}

sl_status sl_sweep(sl_lattice* h, uint64_t n)
{
    const TraceRange range("sl_sweep");
    if (!h) return fail(SL_E_INVALID, "NULL lattice");
    if (n == 0) return SL_OK;
    sl_status st = check_sweep_count(h->pending, h->params.record_capacity, h->next_t,
                                     sweep_limit(h->params.model), n);
    if (st != SL_OK) return st;
    return enqueue_sweeps(h, n);
}

sl_status sl_measure(sl_lattice* h, sl_record* out, size_t cap, size_t* n_out)
{
    const TraceRange range("sl_measure");
    if (!h) return fail(SL_E_INVALID, "NULL lattice");
    if (n_out) *n_out = 0;
    const uint64_t n = h->pending;
    if (n == 0) return SL_OK;
    if (!out || cap < n)
        return fail(SL_E_BUFFER, "%llu records pending, buffer holds %zu", (unsigned long long)n,
                    cap);
    int64_t* dev_out = reinterpret_cast<int64_t*>(h->base + h->lay.off_out);
    hipError_t e = launch_fold(slot_ptr(h, 0), dev_out, n, h->first_t,
                               h->params.model == SL_ISING ? 1 : 0, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->stage, dev_out, n * sizeof(sl_record), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "measure");
    std::memcpy(out, h->stage, n * sizeof(sl_record));
    static_assert(sizeof(sl_record) == kRecordWords * sizeof(int64_t), "record layout");
    h->first_t += n;
    h->pending = 0;
    if (n_out) *n_out = n;
    return SL_OK;
}

sl_status sl_status_counts(const sl_lattice* h, uint64_t* pending, uint64_t* next_t)
{
    if (!h) return fail(SL_E_INVALID, "NULL lattice");
    if (pending) *pending = h->pending;
    if (next_t) *next_t = h->next_t;
    return SL_OK;
}

sl_status sl_copy_spins(sl_lattice* h, int8_t* device_out, size_t n)
{
    if (!h) return fail(SL_E_INVALID, "NULL lattice");
    if (!device_out || n < h->lay.nsites)
        return fail(SL_E_BUFFER, "copy_spins needs %llu bytes", (unsigned long long)h->lay.nsites);
    hipError_t e = launch_to_natural(args_of(h), device_out, h->stream);
    if (e != hipSuccess) return hip_fail(e, "copy_spins");
    return SL_OK;
}

sl_status sl_reset_persistence(sl_lattice* h)
{
    if (!h) return fail(SL_E_INVALID, "NULL lattice");
    if (h->params.model == SL_ISING)
        return fail(SL_E_STATE, "persistence is tracked for the North-East model only");
    hipError_t e = launch_clear_flags(args_of(h), h->stream);
    if (e != hipSuccess) return hip_fail(e, "reset_persistence");
    return SL_OK;
}

sl_status sl_destroy(sl_lattice* h)
{
    if (!h) return fail(SL_E_INVALID, "NULL lattice");
    hipError_t e = hipStreamSynchronize(h->stream);
    release(h);
    if (e != hipSuccess) return hip_fail(e, "destroy: synchronise");
    return SL_OK;
}

sl_status sl_record_observables(const sl_params* params, const sl_record* records, size_t n,
                                double* E, double* M, double* P)
{
    sl_status st = validate(params);
    if (st != SL_OK && st != SL_E_UNSUPPORTED) return st;
    if (n && !records) return fail(SL_E_INVALID, "records is NULL");
    const double nsites = (double)layout_of(params).nsites;
    for (size_t i = 0; i < n; ++i) {
        const sl_record& r = records[i];
        if (params->model == SL_ISING) {
            if (E) E[i] = -params->J * (double)r.bond_sum - params->h * (double)r.mag;
            if (P) P[i] = std::nan("");
        } else if (params->model == SL_NE_COUPLED) {
            double bond, mag;
            spin_sums(r, nsites, bond, mag);
            if (E) E[i] = -params->J * bond - params->h * mag;
            if (P) P[i] = (double)r.unflipped / nsites;
        } else {
            if (E) E[i] = (double)r.mag;
            if (P) P[i] = (double)r.unflipped / nsites;
        }
        if (M) M[i] = (double)r.mag;
    }
    return SL_OK;
}

sl_status sl_record_statistics(const sl_params* params, const sl_record* records, size_t n,
                               sl_stats* out)
{
    sl_status st = validate(params);
    if (st != SL_OK && st != SL_E_UNSUPPORTED) return st;
    if (params->model != SL_ISING && params->model != SL_NE_COUPLED)
        return fail(SL_E_INVALID, "thermodynamic statistics are defined for the Ising energy");
    if (n == 0 || !records || !out) return fail(SL_E_INVALID, "need n >= 1 records and an output");
    const double N = (double)layout_of(params).nsites;
    const double inv_n = 1.0 / (double)n;
    double se = 0.0, sm = 0.0, sma = 0.0, sm2 = 0.0, sm4 = 0.0;
    for (size_t i = 0; i < n; ++i) {
        double bond, mag;
        stat_sums(params, records[i], N, bond, mag);
        const double e = (-params->J * bond - params->h * mag) / N;
        const double m = mag / N;
        se += e;
        sm += m;
        sma += std::fabs(m);
        sm2 += m * m;
        sm4 += (m * m) * (m * m);
    }
    const double mean_e = se * inv_n;
    double sv = 0.0;  // second pass: variance of e
    for (size_t i = 0; i < n; ++i) {
        double bond, mag;
        stat_sums(params, records[i], N, bond, mag);
        const double e = (-params->J * bond - params->h * mag) / N;
        sv += (e - mean_e) * (e - mean_e);
    }
    sl_stats r{};
    r.n = n;
    r.e = mean_e;
    r.e_var = sv * inv_n;
    r.m = sm * inv_n;
    r.m_abs = sma * inv_n;
    r.m2 = sm2 * inv_n;
    r.m4 = sm4 * inv_n;
    r.heat_capacity = N * r.e_var / (params->T * params->T);
    r.susceptibility = N * (r.m2 - r.m_abs * r.m_abs) / params->T;
    r.binder = r.m2 > 0.0 ? 1.0 - r.m4 / (3.0 * r.m2 * r.m2) : std::nan("");
    *out = r;
    return SL_OK;
}

sl_status sl_overlap(sl_lattice* h, const int8_t* reference, int64_t* overlap)
{
    if (!h || !reference || !overlap) return fail(SL_E_INVALID, "NULL argument");
    // the first folded-record slot serves as the accumulator: sl_measure
    // rewrites that area from the ring before it reads it
    unsigned long long* acc = reinterpret_cast<unsigned long long*>(h->base + h->lay.off_out);
    hipError_t e = launch_fill_u64(acc, 1, h->stream);
    if (e == hipSuccess) e = launch_overlap(args_of(h), reference, h->kind == KIND_NE ? 1 : 0, acc, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->stage, acc, sizeof(int64_t), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "overlap");
    std::memcpy(overlap, h->stage, sizeof(int64_t));
    return SL_OK;
}

sl_status sl_autocorrelation(const sl_params* params, int64_t overlap, double* phi)
{
    sl_status st = validate(params);
    if (st != SL_OK && st != SL_E_UNSUPPORTED) return st;
    if (params->model == SL_ISING)
        return fail(SL_E_INVALID, "Phi(t) of Eq. 4 is defined for the North-East model");
    if (!phi) return fail(SL_E_INVALID, "phi is NULL");
    const double N = (double)layout_of(params).nsites;
    const double m0 = 2.0 * params->c - 1.0;
    *phi = ((double)overlap / N - m0 * m0) / (1.0 - m0 * m0);
    return SL_OK;
}

const char* sl_status_str(sl_status s)
{
    switch (s) {
        case SL_OK: return "SL_OK";
        case SL_E_INVALID: return "SL_E_INVALID";
        case SL_E_UNSUPPORTED: return "SL_E_UNSUPPORTED";
        case SL_E_BUFFER: return "SL_E_BUFFER";
        case SL_E_HIP: return "SL_E_HIP";
        case SL_E_STATE: return "SL_E_STATE";
        case SL_E_OVERFLOW: return "SL_E_OVERFLOW";
    }
    return "SL_E_UNKNOWN";
}

const char* sl_last_error(void) { return last_error(); }

}  // extern "C"
