// ne_sub_device.hpp -- device code of the North-East model by the paper's
// random sub-lattice algorithm (Sec. 3.2) for gfx950; kernels_ne_sub_b*.hip
// instantiate it for one sub-lattice side each (separate translation units
// compile in parallel).
//
// The lattice is cut into Q square sub-lattices of B x B sites.  One launch
// processes every sub-lattice once: q = B^2 / (2 lambda) iterations, each of
// which draws lambda random sites of the sub-lattice and updates them
// together; two launches make a sweep.  Neighbours in other sub-lattices (the
// north row and east column) are read as they were when the launch started:
// the launch reads one copy of the lattice and writes the other.  Neighbours
// in the same sub-lattice are read as they were at the start of the iteration.
//
// Mapping: a sub-lattice belongs to one wavefront, lambda/2 lanes of it, each
// lane making two attempts per iteration from one Philox4x32-10 call
// (counter (tau, a/2, launch, 2) for attempts a, a+1).  Because a whole
// sub-lattice lives in one wavefront, the iteration needs no barrier: the
// wavefront's LDS instructions execute in program order, so every read of an
// iteration precedes every write of it.  A workgroup is one wavefront holding
// up to 64/(lambda/2) sub-lattices in LDS.
//
// LDS holds each sub-lattice in natural order: B+1 rows of stride S = B + 8
// (row 0 = the north row, rows 1..B = the sub-lattice), with the east column
// in column B.  A site's north and east neighbours are then at fixed offsets
// (-S, +1) from it, so an attempt costs three byte reads from one address.
// The colour-split rows of HBM are interleaved on the way in and split on the
// way out.
//
// Accepted moves: the move sets n to 1-n and raises the "has flipped" flag
// with LDS atomics on the containing 32-bit word (AND clears n for a
// down-flip, OR sets n for an up-flip and sets the flag).  Attempts of one
// iteration on one site all see the same iteration-start n, so the value an
// atomic returns tells whether another attempt already changed the site: each
// changed site is counted once, and a site drawn twice flips once.  The four
// atomics of a lane's two attempts are issued back to back (no-op masks for an
// attempt that was not accepted).
//
// Latency: the Philox words of iteration j+1 do not depend on the lattice, so
// they are computed while iteration j's LDS traffic is in flight.
//
// Records: the first launch of a sweep also measures the lattice it starts
// from -- the state after the previous sweep -- from the sub-lattices it has
// just loaded (bonds to the north and east neighbours, which tile the lattice's
// bonds exactly once), so no separate pass reads the lattice for that record.
//
// The balanced variant (k_ne_bal, end of Sec. 3.2) shares the loads, stores and
// records; its iterations alternate the two colours of the sub-lattice and
// four launches make a sweep (see the comment above the kernel).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "philox.hpp"
#include "spinlat_internal.h"

namespace spinlat {

namespace nesub {

constexpr int kLdsBudget = 32768;  // bytes of LDS per one-wavefront workgroup
constexpr uint32_t kTagNeSub = 2u;
constexpr uint32_t kTagNeBal = 3u;

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }

template <int B>
struct SubLayout {
    static constexpr int half = B / 2;                  // bytes of a colour row
    static constexpr int stride = B + 8;                // LDS row stride (8-byte aligned)
    static constexpr int bytes = (B + 1) * stride;      // one sub-lattice with its boundary
    static constexpr int unit = half < 16 ? half : 16;  // bytes of a colour vector copy
    static constexpr int units_per_row = half / unit;
};

template <int B, int LPT>
constexpr int tiles_per_wave()
{
    return (64 / LPT) < (kLdsBudget / SubLayout<B>::bytes) ? (64 / LPT)
                                                           : (kLdsBudget / SubLayout<B>::bytes);
}

template <int N>
struct ColourVec {
    uint32_t w[N / 4];
};

// Natural order from colour order: e holds the sites at even x, o those at
// odd x (4 each); the result is the 8 sites in x order.
__device__ __forceinline__ uint2 interleave(uint32_t e, uint32_t o)
{
    uint2 r;
    r.x = (e & 0xFFu) | ((o & 0xFFu) << 8) | ((e & 0xFF00u) << 8) | ((o & 0xFF00u) << 16);
    r.y = ((e >> 16) & 0xFFu) | ((o >> 8) & 0xFF00u) | ((e >> 8) & 0xFF0000u) | (o & 0xFF000000u);
    return r;
}

__device__ __forceinline__ void split(uint2 v, uint32_t& e, uint32_t& o)
{
    e = (v.x & 0xFFu) | ((v.x >> 8) & 0xFF00u) | ((v.y & 0xFFu) << 16) | ((v.y << 8) & 0xFF000000u);
    o = ((v.x >> 8) & 0xFFu) | ((v.x >> 16) & 0xFF00u) | ((v.y << 8) & 0xFF0000u) | (v.y & 0xFF000000u);
}

template <int N>
__device__ __forceinline__ ColourVec<N> load_vec(const uint8_t* p)
{
    ColourVec<N> v;
    if constexpr (N == 16) {
        const uint4 q = *reinterpret_cast<const uint4*>(p);
        v.w[0] = q.x; v.w[1] = q.y; v.w[2] = q.z; v.w[3] = q.w;
    } else if constexpr (N == 8) {
        const uint2 q = *reinterpret_cast<const uint2*>(p);
        v.w[0] = q.x; v.w[1] = q.y;
    } else {
        v.w[0] = *reinterpret_cast<const uint32_t*>(p);
    }
    return v;
}

template <int N>
__device__ __forceinline__ void store_vec(uint8_t* p, const ColourVec<N>& v)
{
    if constexpr (N == 16) {
        *reinterpret_cast<uint4*>(p) = make_uint4(v.w[0], v.w[1], v.w[2], v.w[3]);
    } else if constexpr (N == 8) {
        *reinterpret_cast<uint2*>(p) = make_uint2(v.w[0], v.w[1]);
    } else {
        *reinterpret_cast<uint32_t*>(p) = v.w[0];
    }
}

// Measurement of the sub-lattice as loaded (launch-start state): occupation,
// bonds to the north and east neighbours, sites with the flag clear.
template <int B, int LPT>
__device__ __forceinline__ void observe_tile(const uint8_t* t, uint32_t l, int& mag, int& bond,
                                             int& fresh)
{
    using Lay = SubLayout<B>;
    constexpr int WPR = B / 4;  // 4-byte words per row
    constexpr int NWORD = B * WPR;
#pragma unroll
    for (int i = 0; i < (NWORD + LPT - 1) / LPT; ++i) {
        const int u = (int)l + i * LPT;
        if (u < NWORD) {
            const uint8_t* p = t + (1 + u / WPR) * Lay::stride + 4 * (u % WPR);
            const uint32_t v = *reinterpret_cast<const uint32_t*>(p);
            const uint32_t north = *reinterpret_cast<const uint32_t*>(p - Lay::stride);
            const uint32_t next = *reinterpret_cast<const uint32_t*>(p + 4);
            const uint32_t east = __builtin_amdgcn_alignbyte(next, v, 1);
            const uint32_t nv = v & 0x01010101u;
            mag += __builtin_popcount(nv);
            bond += __builtin_popcount(nv & north) + __builtin_popcount(nv & east);
            fresh += 4 - __builtin_popcount(v & 0x02020202u);
        }
    }
}

// LDS offsets of a site and of its north and east neighbours.
template <int B, bool WRAP>
__device__ __forceinline__ void site_offsets(uint32_t site, uint32_t& own, uint32_t& north,
                                             uint32_t& east)
{
    constexpr int S = SubLayout<B>::stride;
    constexpr int LOGB = ilog2(B);
    const uint32_t r = site >> LOGB;
    if constexpr (!WRAP) {
        north = site + r * (S - B);  // r * S + c
        own = north + S;
        east = own + 1;
    } else {  // one sub-lattice: the periodic neighbours are inside it
        const uint32_t c = site & (B - 1);
        own = (r + 1) * S + c;
        north = (r == 0 ? (uint32_t)B : r) * S + c;
        east = (r + 1) * S + (c == B - 1 ? 0u : c + 1);
    }
}

// Copy sub-lattice tau with its north row and east column from the colour
// arrays into LDS (natural order, see SubLayout); lanes l of LPT share it.
template <int B, int LPT>
__device__ __forceinline__ void load_tile(const NeSubArgs& a, uint8_t* t, uint32_t l, uint32_t x0,
                                          uint32_t y0)
{
    using Lay = SubLayout<B>;
    constexpr int S = Lay::stride;
    constexpr int UNIT = Lay::unit;
    constexpr int NU = (B + 1) * Lay::units_per_row;  // colour-vector pairs
    const uint32_t ynorth = y0 == 0 ? a.L - 1 : y0 - 1;
    const size_t kx = x0 >> 1;
    // north row and sub-lattice rows: both colours, interleaved
#pragma unroll
    for (int i = 0; i < (NU + LPT - 1) / LPT; ++i) {
        const int u = (int)l + i * LPT;
        if (u < NU) {
            const int pr = u / Lay::units_per_row, part = u % Lay::units_per_row;
            const uint32_t y = pr == 0 ? ynorth : y0 + pr - 1;
            const size_t off = (size_t)y * a.Lh + kx + part * UNIT;
            const ColourVec<UNIT> c0 = load_vec<UNIT>(a.src[0] + off);
            const ColourVec<UNIT> c1 = load_vec<UNIT>(a.src[1] + off);
            const bool odd = (y & 1u) != 0;  // colour 1 holds the even x of odd rows
            uint2* dstp = reinterpret_cast<uint2*>(t + pr * S + part * 2 * UNIT);
#pragma unroll
            for (int k = 0; k < UNIT / 4; ++k)
                dstp[k] = odd ? interleave(c1.w[k], c0.w[k]) : interleave(c0.w[k], c1.w[k]);
        }
    }
    // east column: site (x0 + B, y) has colour (x0 + B + y) & 1
    const uint32_t xe = x0 + B == a.L ? 0u : x0 + B;
#pragma unroll
    for (int i = 0; i < (B + LPT - 1) / LPT; ++i) {
        const int r = (int)l + i * LPT;
        if (r < B) {
            const uint32_t y = y0 + r;
            t[(r + 1) * S + B] = a.src[(xe + y) & 1u][(size_t)y * a.Lh + (xe >> 1)];
        }
    }
}

// The sub-lattice rows back to the colour arrays of the destination copy.
template <int B, int LPT>
__device__ __forceinline__ void store_tile(const NeSubArgs& a, const uint8_t* t, uint32_t l,
                                           uint32_t x0, uint32_t y0)
{
    using Lay = SubLayout<B>;
    constexpr int S = Lay::stride;
    constexpr int UNIT = Lay::unit;
    constexpr int NW = B * Lay::units_per_row;
    const size_t kx = x0 >> 1;
#pragma unroll
    for (int i = 0; i < (NW + LPT - 1) / LPT; ++i) {
        const int u = (int)l + i * LPT;
        if (u < NW) {
            const int r = u / Lay::units_per_row, part = u % Lay::units_per_row;
            const uint32_t y = y0 + r;
            const uint2* srcp = reinterpret_cast<const uint2*>(t + (r + 1) * S + part * 2 * UNIT);
            ColourVec<UNIT> c0, c1;
            const bool odd = (y & 1u) != 0;
#pragma unroll
            for (int k = 0; k < UNIT / 4; ++k) {
                uint32_t e, o;
                split(srcp[k], e, o);
                c0.w[k] = odd ? o : e;
                c1.w[k] = odd ? e : o;
            }
            const size_t off = (size_t)y * a.Lh + kx + part * UNIT;
            store_vec<UNIT>(a.dst[0] + off, c0);
            store_vec<UNIT>(a.dst[1] + off, c1);
        }
    }
}

// Wavefront sums of the per-lane counts into the records.
__device__ __forceinline__ void add_counts(const NeSubArgs& a, uint32_t lane, int changed, int mag,
                                           int bond, int fresh)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) changed += __shfl_xor(changed, off, 64);
    if (lane == 0 && changed != 0)
        atomicAdd(&a.acc[(blockIdx.x % kSub) * kSubStride + 2], (unsigned long long)changed);
    if (a.obs) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            mag += __shfl_xor(mag, off, 64);
            bond += __shfl_xor(bond, off, 64);
            fresh += __shfl_xor(fresh, off, 64);
        }
        unsigned long long* o = a.obs + (blockIdx.x % kSub) * kSubStride;
        if (lane == 0 && bond != 0) atomicAdd(&o[0], (unsigned long long)bond);
        if (lane == 1 && mag != 0) atomicAdd(&o[1], (unsigned long long)mag);
        if (lane == 2 && fresh != 0) atomicAdd(&o[3], (unsigned long long)fresh);
    }
}

template <int B, int LPT, bool WRAP>
__global__ void __launch_bounds__(64) k_ne_sub(NeSubArgs a)
{
    using Lay = SubLayout<B>;
    constexpr int TPW = tiles_per_wave<B, LPT>();
    constexpr int LOGB = ilog2(B);
    constexpr int QIT = B * B / (4 * LPT);  // q = P / (2 lambda), lambda = 2 LPT
    __shared__ __align__(16) uint8_t lds[TPW * Lay::bytes];

    const uint32_t lane = threadIdx.x;
    const uint32_t g = lane / LPT;
    const uint32_t l = lane % LPT;
    const uint32_t tau = blockIdx.x * TPW + g;
    int changed = 0, mag = 0, bond = 0, fresh = 0;
    if (g < (uint32_t)TPW && tau < a.ntiles) {
        uint8_t* t = lds + g * Lay::bytes;
        const uint32_t tx = tau % a.tiles_x, ty = tau / a.tiles_x;
        const uint32_t x0 = tx * B, y0 = ty * B;
        load_tile<B, LPT>(a, t, l, x0, y0);

        if (a.obs) observe_tile<B, LPT>(t, l, mag, bond, fresh);

        const PhiloxKey ks = philox_schedule(a.key0, a.key1);
        uint32_t* w32 = reinterpret_cast<uint32_t*>(t);
        Words4 w = philox4x32_10(tau, l, a.launch, kTagNeSub, ks);
        for (int j = 0; j < QIT; ++j) {
            uint32_t own[2], nocc[2], vs[2], vn[2], ve[2], acc_word[2];
            bool ok[2];
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                uint32_t north, east;
                site_offsets<B, WRAP>(w.w[2 * m] >> (32 - 2 * LOGB), own[m], north, east);
                vs[m] = t[own[m]];
                vn[m] = t[north];
                ve[m] = t[east];
                acc_word[m] = w.w[2 * m + 1];
            }
            // next iteration's words while the reads are in flight; the empty
            // asm pins them here (the compiler would otherwise sink them past
            // the atomics, where they would wait for the atomics' results)
            w = philox4x32_10(tau, (uint32_t)(j + 1) * LPT + l, a.launch, kTagNeSub, ks);
            asm volatile("" : "+v"(w.w[0]), "+v"(w.w[1]), "+v"(w.w[2]), "+v"(w.w[3]));
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                const uint32_t n = vs[m] & 1u;
                const uint32_t allow = vn[m] & ve[m] & 1u;
                // accept iff word < thr, thr in [0, 2^32]: word <= thr - 1 unless thr = 0
                const uint32_t thr_m1 = n ? a.thr_m1_down : a.thr_m1_up;
                const uint32_t never = (a.never >> n) & 1u;
                ok[m] = (allow & (acc_word[m] <= thr_m1 ? 1u : 0u) & (never ^ 1u)) != 0u;
                nocc[m] = n;
            }
            if (ok[0] | ok[1]) {
                uint32_t sh[2], old_and[2], old_or[2];
#pragma unroll
                for (int m = 0; m < 2; ++m) {
                    sh[m] = (own[m] & 3u) * 8u;
                    const bool dn = ok[m] & (nocc[m] != 0u);
                    old_and[m] = atomicAnd(w32 + (own[m] >> 2), dn ? ~(1u << sh[m]) : ~0u);
                }
#pragma unroll
                for (int m = 0; m < 2; ++m) {
                    const uint32_t set = ok[m] ? (nocc[m] ? 2u : 3u) : 0u;
                    old_or[m] = atomicOr(w32 + (own[m] >> 2), set << sh[m]);
                }
#pragma unroll
                for (int m = 0; m < 2; ++m) {
                    // first change of the site in this iteration: n still as at its start
                    const uint32_t before = nocc[m] ? old_and[m] : old_or[m];
                    changed += (int)(ok[m] & (((before >> sh[m]) & 1u) == nocc[m]));
                }
            }
        }

        store_tile<B, LPT>(a, t, l, x0, y0);
    }
    add_counts(a, lane, changed, mag, bond, fresh);
}

// Balanced variant: each iteration draws lambda sites of colour 0, then lambda
// sites of colour 1 (half h); P/(8 lambda) iterations per launch, four
// launches per sweep.  Sites of one colour are not neighbours, so the
// attempts of a half only read frozen neighbours; when attempts of a half
// draw the same site only the lowest-numbered one applies.  Each sub-lattice
// keeps an owner word per site of the half's colour: attempts post their
// number with an LDS atomic minimum, read it back, and only the owner
// evaluates the move and resets the word.  The winner's site is unique, so
// its store needs no atomic.
template <int B, int LPT>
constexpr int bal_tile_bytes()
{
    return SubLayout<B>::bytes + 4 * (B * B / 2);
}

template <int B, int LPT>
constexpr int bal_tiles_per_wave()
{
    return (64 / LPT) < (kLdsBudget / bal_tile_bytes<B, LPT>()) ? (64 / LPT)
                                                                : (kLdsBudget / bal_tile_bytes<B, LPT>());
}

template <int B, int LPT, bool WRAP>
__global__ void __launch_bounds__(64) k_ne_bal(NeSubArgs a)
{
    using Lay = SubLayout<B>;
    constexpr int TB = bal_tile_bytes<B, LPT>();
    constexpr int TPW = bal_tiles_per_wave<B, LPT>();
    constexpr int HS = B * B / 2;  // sites of one colour
    constexpr int LOGHS = ilog2(HS), LOGBH = ilog2(B / 2);
    constexpr int QIT = B * B / (16 * LPT);  // P / (8 lambda), lambda = 2 LPT
    static_assert(Lay::bytes % 4 == 0, "owner words must be aligned");
    __shared__ __align__(16) uint8_t lds[TPW * TB];

    const uint32_t lane = threadIdx.x;
    const uint32_t g = lane / LPT;
    const uint32_t l = lane % LPT;
    const uint32_t tau = blockIdx.x * TPW + g;
    int changed = 0, mag = 0, bond = 0, fresh = 0;
    if (g < (uint32_t)TPW && tau < a.ntiles) {
        uint8_t* t = lds + g * TB;
        uint32_t* owner = reinterpret_cast<uint32_t*>(t + Lay::bytes);
        const uint32_t x0 = (tau % a.tiles_x) * B, y0 = (tau / a.tiles_x) * B;
        load_tile<B, LPT>(a, t, l, x0, y0);
        for (int i = (int)l; i < HS; i += LPT) owner[i] = 0xFFFFFFFFu;
        if (a.obs) observe_tile<B, LPT>(t, l, mag, bond, fresh);

        const PhiloxKey ks = philox_schedule(a.key0, a.key1);
        for (int j = 0; j < QIT; ++j) {
#pragma unroll
            for (uint32_t h = 0; h < 2; ++h) {
                const Words4 w =
                    philox4x32_10(tau, (2u * j + h) * LPT + l, a.launch, kTagNeBal, ks);
                uint32_t idx[2], own[2], vs[2], vn[2], ve[2];
#pragma unroll
                for (int m = 0; m < 2; ++m) {
                    idx[m] = w.w[2 * m] >> (32 - LOGHS);  // floor(word (P/2) / 2^32)
                    const uint32_t r = idx[m] >> LOGBH;
                    const uint32_t cc = 2u * (idx[m] & (B / 2 - 1)) + ((r + h) & 1u);
                    uint32_t north, east;
                    site_offsets<B, WRAP>((r << ilog2(B)) + cc, own[m], north, east);
                    vs[m] = t[own[m]];
                    vn[m] = t[north];
                    ve[m] = t[east];
                    atomicMin(owner + idx[m], 2u * l + (uint32_t)m);
                }
                uint32_t win[2];
#pragma unroll
                for (int m = 0; m < 2; ++m)
                    win[m] = __hip_atomic_load(owner + idx[m], __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP) == 2u * l + (uint32_t)m;
#pragma unroll
                for (int m = 0; m < 2; ++m) {
                    const uint32_t n = vs[m] & 1u;
                    const uint32_t allow = vn[m] & ve[m] & 1u;
                    const uint32_t thr_m1 = n ? a.thr_m1_down : a.thr_m1_up;
                    const uint32_t never = (a.never >> n) & 1u;
                    const bool ok = (win[m] & allow & (w.w[2 * m + 1] <= thr_m1 ? 1u : 0u) &
                                     (never ^ 1u)) != 0u;
                    if (ok) {
                        t[own[m]] = (uint8_t)((n ^ 1u) | 2u);
                        changed += 1;
                    }
                    if (win[m]) owner[idx[m]] = 0xFFFFFFFFu;
                }
            }
        }
        store_tile<B, LPT>(a, t, l, x0, y0);
    }
    add_counts(a, lane, changed, mag, bond, fresh);
}

template <int B, int LPT>
hipError_t launch_one(const NeSubArgs& a, bool balanced, hipStream_t s)
{
    if (balanced) {
        constexpr int TPW = bal_tiles_per_wave<B, LPT>();
        static_assert(TPW >= 1, "a sub-lattice must fit the LDS budget");
        const uint32_t blocks = (a.ntiles + TPW - 1) / TPW;
        if (a.ntiles == 1)
            hipLaunchKernelGGL((k_ne_bal<B, LPT, true>), dim3(blocks), dim3(64), 0, s, a);
        else
            hipLaunchKernelGGL((k_ne_bal<B, LPT, false>), dim3(blocks), dim3(64), 0, s, a);
        return hipGetLastError();
    }
    constexpr int TPW = tiles_per_wave<B, LPT>();
    static_assert(TPW >= 1, "a sub-lattice must fit the LDS budget");
    const uint32_t blocks = (a.ntiles + TPW - 1) / TPW;
    if (a.ntiles == 1)
        hipLaunchKernelGGL((k_ne_sub<B, LPT, true>), dim3(blocks), dim3(64), 0, s, a);
    else
        hipLaunchKernelGGL((k_ne_sub<B, LPT, false>), dim3(blocks), dim3(64), 0, s, a);
    return hipGetLastError();
}

template <int B>
hipError_t launch_side(const NeSubArgs& a, int lambda, bool balanced, hipStream_t s)
{
    switch (lambda) {
        case 2: return launch_one<B, 1>(a, balanced, s);
        case 4: return launch_one<B, 2>(a, balanced, s);
        case 8: return launch_one<B, 4>(a, balanced, s);
        case 16: return launch_one<B, 8>(a, balanced, s);
        case 32: return launch_one<B, 16>(a, balanced, s);
        case 64: return launch_one<B, 32>(a, balanced, s);
        case 128: return launch_one<B, 64>(a, balanced, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace nesub

}  // namespace spinlat
