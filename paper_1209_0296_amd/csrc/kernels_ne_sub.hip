// kernels_ne_sub.hip -- the North-East model by the paper's random
// sub-lattice algorithm (Sec. 3.2) for gfx950.
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
// LDS holds each sub-lattice in the colour-split form of the global layout:
// for colour c, B+1 rows (row 0 = the north row, rows 1..B = the sub-lattice)
// of B/2 bytes, plus one byte at index B/2 that holds the east column for the
// sites whose east neighbour has colour c.  Rows then copy to and from HBM as
// plain vectors, and a site's neighbours are found by index arithmetic.
//
// Accepted moves: the move sets n to 1-n and raises the "has flipped" flag
// with LDS atomics on the containing 32-bit word (OR for an up-flip, AND then
// OR for a down-flip).  The returned old value tells whether another attempt
// of the same iteration already changed the site, so each changed site is
// counted once, and a site drawn twice flips once.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "philox.hpp"
#include "spinlat_internal.h"

namespace spinlat {

namespace {

constexpr int kLdsBudget = 32768;  // bytes of LDS per one-wavefront workgroup
constexpr uint32_t kTagNeSub = 2u;

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }

template <int B>
struct SubLayout {
    static constexpr int half = B / 2;                          // bytes of a colour row
    static constexpr int stride = ((half + 1 + 15) / 16) * 16;  // LDS row stride
    static constexpr int plane = (B + 1) * stride;              // one colour
    static constexpr int bytes = 2 * plane;                     // one sub-lattice
    static constexpr int unit = half < 16 ? half : 16;          // bytes per vector copy
    static constexpr int units_per_row = half / unit;
};

template <int B, int LPT>
constexpr int tiles_per_wave()
{
    return (64 / LPT) < (kLdsBudget / SubLayout<B>::bytes) ? (64 / LPT)
                                                           : (kLdsBudget / SubLayout<B>::bytes);
}

template <int N>
struct VecOf;
template <>
struct VecOf<4> {
    using T = uint32_t;
};
template <>
struct VecOf<8> {
    using T = uint2;
};
template <>
struct VecOf<16> {
    using T = uint4;
};

// Accepted move at LDS byte `idx` (word array w32) whose iteration-start
// occupation is n: returns 1 if this call changed the site.
__device__ __forceinline__ int flip_site(uint32_t* w32, uint32_t idx, uint32_t n)
{
    const uint32_t sh = (idx & 3u) * 8u;
    uint32_t* p = w32 + (idx >> 2);
    if (n == 0u) {
        const uint32_t old = atomicOr(p, 3u << sh);  // n = 1, flag
        return ((old >> sh) & 1u) == 0u ? 1 : 0;
    }
    const uint32_t old = atomicAnd(p, ~(1u << sh));  // n = 0
    atomicOr(p, 2u << sh);                           // flag
    return (int)((old >> sh) & 1u);
}

template <int B, int LPT>
__global__ void __launch_bounds__(64) k_ne_sub(NeSubArgs a)
{
    using Lay = SubLayout<B>;
    using V = typename VecOf<Lay::unit>::T;
    constexpr int TPW = tiles_per_wave<B, LPT>();
    constexpr int LOGB = ilog2(B);
    constexpr int QIT = B * B / (4 * LPT);  // q = P / (2 lambda), lambda = 2 LPT
    constexpr int NU = 2 * (B + 1) * Lay::units_per_row;  // vector copies per load
    constexpr int NW = 2 * B * Lay::units_per_row;        // vector copies per store
    __shared__ __align__(16) uint8_t lds[TPW * Lay::bytes];

    const uint32_t lane = threadIdx.x;
    const uint32_t g = lane / LPT;
    const uint32_t l = lane % LPT;
    const uint32_t tau = blockIdx.x * TPW + g;
    int changed = 0;
    if (g < (uint32_t)TPW && tau < a.ntiles) {
        uint8_t* t = lds + g * Lay::bytes;
        const uint32_t tx = tau % a.tiles_x, ty = tau / a.tiles_x;
        const uint32_t x0 = tx * B, y0 = ty * B;
        const uint32_t ynorth = y0 == 0 ? a.L - 1 : y0 - 1;
        const size_t kx = x0 >> 1;

        // north row and sub-lattice rows of both colours
#pragma unroll
        for (int i = 0; i < (NU + LPT - 1) / LPT; ++i) {
            const int u = (int)l + i * LPT;
            if (u < NU) {
                const int c = u / ((B + 1) * Lay::units_per_row);
                const int rem = u % ((B + 1) * Lay::units_per_row);
                const int pr = rem / Lay::units_per_row, part = rem % Lay::units_per_row;
                const uint32_t y = pr == 0 ? ynorth : y0 + pr - 1;
                const V v = *reinterpret_cast<const V*>(a.src[c] + (size_t)y * a.Lh + kx +
                                                        part * Lay::unit);
                *reinterpret_cast<V*>(t + c * Lay::plane + pr * Lay::stride + part * Lay::unit) = v;
            }
        }
        // east column: site (x0 + B, y) has colour (x0 + B + y) & 1
        const uint32_t xe = x0 + B == a.L ? 0u : x0 + B;
#pragma unroll
        for (int i = 0; i < (B + LPT - 1) / LPT; ++i) {
            const int r = (int)l + i * LPT;
            if (r < B) {
                const uint32_t y = y0 + r;
                const uint32_t c = (xe + y) & 1u;
                t[c * Lay::plane + (r + 1) * Lay::stride + Lay::half] =
                    a.src[c][(size_t)y * a.Lh + (xe >> 1)];
            }
        }

        const PhiloxKey ks = philox_schedule(a.key0, a.key1);
        uint32_t* w32 = reinterpret_cast<uint32_t*>(t);
        const bool wrap = a.wrap != 0;
        for (int j = 0; j < QIT; ++j) {
            const Words4 w = philox4x32_10(tau, (uint32_t)j * LPT + l, a.launch, kTagNeSub, ks);
            uint32_t idx[2], nv[2];
            bool ok[2];
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                const uint32_t site = w.w[2 * m] >> (32 - 2 * LOGB);  // floor(word P / 2^32)
                const uint32_t r = site >> LOGB, cc = site & (B - 1);
                const uint32_t cs = (cc ^ r) & 1u;  // colour of (x0+cc, y0+r)
                const uint32_t own = cs * Lay::plane, oth = (cs ^ 1u) * Lay::plane;
                idx[m] = own + (r + 1) * Lay::stride + (cc >> 1);
                const uint32_t rn = (wrap && r == 0) ? (uint32_t)B : r;
                const uint32_t ce = (wrap && cc == B - 1) ? 0u : cc + 1;
                const uint32_t n = t[idx[m]] & 1u;
                const uint32_t north = t[oth + rn * Lay::stride + (cc >> 1)];
                const uint32_t east = t[oth + (r + 1) * Lay::stride + (ce >> 1)];
                const uint64_t thr = n ? a.thr_down : a.thr_up;
                ok[m] = ((north & east & 1u) != 0u) && ((uint64_t)w.w[2 * m + 1] < thr);
                nv[m] = n;
            }
#pragma unroll
            for (int m = 0; m < 2; ++m)
                if (ok[m]) changed += flip_site(w32, idx[m], nv[m]);
        }

        // the sub-lattice rows of both colours back to HBM
#pragma unroll
        for (int i = 0; i < (NW + LPT - 1) / LPT; ++i) {
            const int u = (int)l + i * LPT;
            if (u < NW) {
                const int c = u / (B * Lay::units_per_row);
                const int rem = u % (B * Lay::units_per_row);
                const int r = rem / Lay::units_per_row, part = rem % Lay::units_per_row;
                const V v = *reinterpret_cast<const V*>(t + c * Lay::plane + (r + 1) * Lay::stride +
                                                        part * Lay::unit);
                *reinterpret_cast<V*>(a.dst[c] + (size_t)(y0 + r) * a.Lh + kx + part * Lay::unit) = v;
            }
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) changed += __shfl_xor(changed, off, 64);
    if (lane == 0 && changed != 0)
        atomicAdd(&a.acc[(blockIdx.x % kSub) * kQ + 2], (unsigned long long)changed);
}

template <int B, int LPT>
hipError_t launch_one(const NeSubArgs& a, hipStream_t s)
{
    constexpr int TPW = tiles_per_wave<B, LPT>();
    static_assert(TPW >= 1, "a sub-lattice must fit the LDS budget");
    const uint32_t blocks = (a.ntiles + TPW - 1) / TPW;
    hipLaunchKernelGGL((k_ne_sub<B, LPT>), dim3(blocks), dim3(64), 0, s, a);
    return hipGetLastError();
}

template <int B>
hipError_t launch_side(const NeSubArgs& a, int lambda, hipStream_t s)
{
    switch (lambda) {
        case 2: return launch_one<B, 1>(a, s);
        case 4: return launch_one<B, 2>(a, s);
        case 8: return launch_one<B, 4>(a, s);
        case 16: return launch_one<B, 8>(a, s);
        case 32: return launch_one<B, 16>(a, s);
        case 64: return launch_one<B, 32>(a, s);
        case 128: return launch_one<B, 64>(a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

bool ne_sub_supported(uint32_t L, int B, int lambda)
{
    if (B != 8 && B != 16 && B != 32 && B != 64) return false;
    if (L % (uint32_t)B != 0) return false;
    if (lambda < 2 || lambda > 128 || (lambda & (lambda - 1)) != 0) return false;
    return 2 * lambda <= B * B;
}

hipError_t launch_ne_sub(const NeSubArgs& a, int B, int lambda, hipStream_t s)
{
    switch (B) {
        case 8: return launch_side<8>(a, lambda, s);
        case 16: return launch_side<16>(a, lambda, s);
        case 32: return launch_side<32>(a, lambda, s);
        case 64: return launch_side<64>(a, lambda, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace spinlat
