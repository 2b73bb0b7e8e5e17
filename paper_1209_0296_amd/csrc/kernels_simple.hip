// kernels_simple.hip -- initial state, layout conversion, record folding, the
// overlap reduction, the direct (no LDS) half-sweep kernel and the resident
// kernel that runs many sweeps of a small lattice held in LDS, for gfx950.
//
// Layout: two colour arrays of L^dim/2 int8 sites (see spinlat_internal.h).
// One thread owns one 4-byte word = 4 consecutive same-colour sites of one row
// (Lh % 4 == 0), which is exactly the set of sites one Philox4x32-10 call
// serves for one-word moves (spin-1/2, NE) and two calls serve for spin-1.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "philox.hpp"
#include "site_update.hpp"
#include "simple_device.hpp"
#include "spinlat_internal.h"

namespace spinlat {

using namespace simplek;

namespace {

constexpr int kBlock = 256;

// ---------------------------------------------------------------------------
// Initial state (Alg. I step 1; NE: up with probability c, Sec. 3.2), drawn
// from Philox with tag 1 at sweep 0.  mode: 0 cold (+1), 1 random.
template <int KIND>
__global__ void __launch_bounds__(kBlock) k_init(SweepArgs a, int mode, uint32_t thr_lo,
                                                 uint32_t thr_hi)
{
    const uint64_t ngroups = a.g.nh >> 2;
    const uint64_t gi = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (gi >= 2 * ngroups) return;
    const uint32_t c = gi >= ngroups ? 1u : 0u;
    const uint64_t g = gi - (c ? ngroups : 0);
    const PhiloxKey ks = philox_schedule(a.key0, a.key1);
    const Words4 r = philox4x32_10((uint32_t)g, c, 0u, 1u, ks);
    const uint64_t thr = ((uint64_t)thr_hi << 32) | thr_lo;
    uint32_t word = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const uint32_t u = r.w[b];
        int v;
        if (KIND == KIND_NE) {
            v = ((uint64_t)u < thr) ? 1 : 0;
        } else if (mode == 0) {
            v = 1;
        } else if (KIND == KIND_ISING_HALF) {
            v = (u < 0x80000000u) ? 1 : -1;
        } else {
            v = (int)(((uint64_t)u * 3u) >> 32) - 1;
        }
        word |= ((uint32_t)(uint8_t)(int8_t)v) << (8 * b);
    }
    *reinterpret_cast<uint32_t*>(a.col[c] + 4 * g) = word;
}

// Natural row-major bytes <-> colour arrays.
__device__ __forceinline__ uint64_t natural_index(const Geom& g, uint32_t c, uint64_t k)
{
    const uint64_t row = k / g.Lh;
    const uint32_t kk = (uint32_t)(k - row * g.Lh);
    const uint32_t y = (uint32_t)(row % g.L);
    const uint32_t z = (uint32_t)(row / g.L);
    const uint32_t x = 2 * kk + ((y + z + c) & 1u);
    return row * g.L + x;
}

__global__ void __launch_bounds__(kBlock) k_from_natural(SweepArgs a, const int8_t* nat)
{
    const uint64_t ngroups = a.g.nh >> 2;
    const uint64_t gi = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (gi >= 2 * ngroups) return;
    const uint32_t c = gi >= ngroups ? 1u : 0u;
    const uint64_t g = gi - (c ? ngroups : 0);
    uint32_t word = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b)
        word |= (uint32_t)(uint8_t)nat[natural_index(a.g, c, 4 * g + b)] << (8 * b);
    *reinterpret_cast<uint32_t*>(a.col[c] + 4 * g) = word;
}

__global__ void __launch_bounds__(kBlock) k_to_natural(SweepArgs a, int8_t* nat)
{
    const uint64_t ngroups = a.g.nh >> 2;
    const uint64_t gi = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (gi >= 2 * ngroups) return;
    const uint32_t c = gi >= ngroups ? 1u : 0u;
    const uint64_t g = gi - (c ? ngroups : 0);
    const uint32_t word = *reinterpret_cast<const uint32_t*>(a.col[c] + 4 * g);
#pragma unroll
    for (int b = 0; b < 4; ++b)
        nat[natural_index(a.g, c, 4 * g + b)] = (int8_t)(uint8_t)(word >> (8 * b));
}

// Overlap sum_i v_i v_i^ref with a natural-order reference lattice (v = s for
// Ising, 2n - 1 for an NE occupation n), accumulated into one int64.
__global__ void __launch_bounds__(kBlock) k_overlap(SweepArgs a, const int8_t* ref, int ne,
                                                    unsigned long long* out)
{
    const uint64_t ngroups = a.g.nh >> 2;
    const uint64_t gi = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    int32_t sum = 0;
    if (gi < 2 * ngroups) {
        const uint32_t c = gi >= ngroups ? 1u : 0u;
        const uint64_t g = gi - (c ? ngroups : 0);
        const uint32_t word = *reinterpret_cast<const uint32_t*>(a.col[c] + 4 * g);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int v = (int)(int8_t)(uint8_t)(word >> (8 * b));
            const int r = (int)ref[natural_index(a.g, c, 4 * g + b)];
            sum += ne ? (2 * (v & 1) - 1) * (2 * (r & 1) - 1) : v * r;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
    __shared__ int32_t part[kBlock / 64];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int w = 0; w < kBlock / 64; ++w) t += part[w];
        if (t != 0) atomicAdd(out, (unsigned long long)t);
    }
}

__global__ void __launch_bounds__(kBlock) k_clear_flags(SweepArgs a)
{
    const uint64_t ngroups = a.g.nh >> 2;
    const uint64_t gi = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (gi >= 2 * ngroups) return;
    const uint32_t c = gi >= ngroups ? 1u : 0u;
    const uint64_t g = gi - (c ? ngroups : 0);
    uint32_t* p = reinterpret_cast<uint32_t*>(a.col[c] + 4 * g);
    *p = *p & 0x01010101u;
}

__global__ void __launch_bounds__(kBlock) k_fill_u64(unsigned long long* p, uint64_t n)
{
    const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// Sum the kSub sub-slots of each pending record, write {t, q0..q3} and clear
// the accumulators for reuse.
__global__ void __launch_bounds__(kBlock) k_fold(unsigned long long* acc, int64_t* out, uint64_t n,
                                                 uint64_t t_first, int ising)
{
    const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    unsigned long long* slot = acc + i * kSlotWords;
    int64_t sum[kQ] = {0, 0, 0, 0};
    for (int s = 0; s < kSub; ++s)
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            sum[q] += (int64_t)slot[s * kSubStride + q];
            slot[s * kSubStride + q] = 0ull;
        }
    int64_t* o = out + i * kRecordWords;
    o[0] = (int64_t)(t_first + i);
    o[1] = sum[0];
    o[2] = sum[1];
    o[3] = sum[2];
    o[4] = ising ? -1 : sum[3];
}

// Direct half-sweep: one thread per 4-site word of colour a.colour.
template <int KIND, int DIM>
__global__ void __launch_bounds__(kBlock) k_simple_half(SweepArgs a)
{
    __shared__ uint64_t lut[kMaxLut];
    for (int i = threadIdx.x; i < a.lut_n; i += kBlock) lut[i] = a.lut[i];
    __syncthreads();

    const uint64_t ngroups = a.g.nh >> 2;
    const uint64_t gi = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    int32_t q_bond = 0, q_mag = 0, q_acc = 0, q_unfl = 0;
    if (gi < ngroups) {
        const PhiloxKey ks = philox_schedule(a.key0, a.key1);
        simple_word<KIND, DIM>(a.col[a.colour], reinterpret_cast<const int8_t*>(a.col[a.colour ^ 1u]),
                               a.g, a.colour, gi, a.t, a.update, ks, lut, KIND == KIND_NE && a.lut_n > 2,
                               q_bond, q_mag, q_acc, q_unfl);
    }
    block_accumulate(q_bond, q_mag, q_acc, q_unfl, a.acc);
}

template <int KIND, int DIM>
__global__ void __launch_bounds__(kResidentBlock) k_resident(SweepArgs a, uint32_t nsweeps)
{
    extern __shared__ __align__(16) uint8_t sm[];
    __shared__ uint64_t lut[kMaxLut];
    resident_run<KIND, DIM>(a, nsweeps, sm, lut);
}

inline unsigned blocks_for(uint64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

hipError_t launch_fill_u64(unsigned long long* p, uint64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3(blocks_for(n)), dim3(kBlock), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_init(const SweepArgs& a, int kind, int init_mode, uint32_t thr_lo,
                       uint32_t thr_hi, hipStream_t s)
{
    const unsigned nb = blocks_for(2 * (a.g.nh >> 2));
    switch (kind) {
        case KIND_ISING_HALF:
            hipLaunchKernelGGL(k_init<KIND_ISING_HALF>, dim3(nb), dim3(kBlock), 0, s, a, init_mode,
                               thr_lo, thr_hi);
            break;
        case KIND_ISING_ONE:
            hipLaunchKernelGGL(k_init<KIND_ISING_ONE>, dim3(nb), dim3(kBlock), 0, s, a, init_mode,
                               thr_lo, thr_hi);
            break;
        default:
            hipLaunchKernelGGL(k_init<KIND_NE>, dim3(nb), dim3(kBlock), 0, s, a, init_mode, thr_lo,
                               thr_hi);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_from_natural(const SweepArgs& a, const int8_t* nat, hipStream_t s)
{
    hipLaunchKernelGGL(k_from_natural, dim3(blocks_for(2 * (a.g.nh >> 2))), dim3(kBlock), 0, s, a,
                       nat);
    return hipGetLastError();
}

hipError_t launch_to_natural(const SweepArgs& a, int8_t* nat, hipStream_t s)
{
    hipLaunchKernelGGL(k_to_natural, dim3(blocks_for(2 * (a.g.nh >> 2))), dim3(kBlock), 0, s, a,
                       nat);
    return hipGetLastError();
}

hipError_t launch_overlap(const SweepArgs& a, const int8_t* ref, int ne, unsigned long long* out,
                          hipStream_t s)
{
    hipLaunchKernelGGL(k_overlap, dim3(blocks_for(2 * (a.g.nh >> 2))), dim3(kBlock), 0, s, a, ref,
                       ne, out);
    return hipGetLastError();
}

bool resident_supported(const Geom& g) { return 2 * g.nh <= (uint64_t)kResidentLds; }

hipError_t launch_resident(const SweepArgs& a, int kind, uint32_t nsweeps, hipStream_t s)
{
    const size_t lds = (size_t)(2 * a.g.nh);
    if (lds > (size_t)kResidentLds) return hipErrorInvalidValue;
    const dim3 grid(1), block(kResidentBlock);
    if (kind == KIND_NE) {
        hipLaunchKernelGGL((k_resident<KIND_NE, 2>), grid, block, lds, s, a, nsweeps);
    } else if (a.g.dim == 2) {
        if (kind == KIND_ISING_HALF)
            hipLaunchKernelGGL((k_resident<KIND_ISING_HALF, 2>), grid, block, lds, s, a, nsweeps);
        else
            hipLaunchKernelGGL((k_resident<KIND_ISING_ONE, 2>), grid, block, lds, s, a, nsweeps);
    } else {
        if (kind == KIND_ISING_HALF)
            hipLaunchKernelGGL((k_resident<KIND_ISING_HALF, 3>), grid, block, lds, s, a, nsweeps);
        else
            hipLaunchKernelGGL((k_resident<KIND_ISING_ONE, 3>), grid, block, lds, s, a, nsweeps);
    }
    return hipGetLastError();
}

hipError_t launch_clear_flags(const SweepArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(k_clear_flags, dim3(blocks_for(2 * (a.g.nh >> 2))), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fold(unsigned long long* acc, int64_t* out, uint64_t n, uint64_t t_first,
                       int ising, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fold, dim3(blocks_for(n)), dim3(kBlock), 0, s, acc, out, n, t_first,
                       ising);
    return hipGetLastError();
}

hipError_t launch_simple_half(const SweepArgs& a, int kind, hipStream_t s)
{
    const dim3 grid(blocks_for(a.g.nh >> 2));
    const dim3 block(kBlock);
    if (kind == KIND_NE) {
        hipLaunchKernelGGL((k_simple_half<KIND_NE, 2>), grid, block, 0, s, a);
    } else if (a.g.dim == 2) {
        if (kind == KIND_ISING_HALF)
            hipLaunchKernelGGL((k_simple_half<KIND_ISING_HALF, 2>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((k_simple_half<KIND_ISING_ONE, 2>), grid, block, 0, s, a);
    } else {
        if (kind == KIND_ISING_HALF)
            hipLaunchKernelGGL((k_simple_half<KIND_ISING_HALF, 3>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((k_simple_half<KIND_ISING_ONE, 3>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace spinlat
