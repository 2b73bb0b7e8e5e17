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
#include "spinlat_internal.h"

namespace spinlat {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ uint32_t wrap_inc(uint32_t v, uint32_t n) { return v + 1 == n ? 0 : v + 1; }
__device__ __forceinline__ uint32_t wrap_dec(uint32_t v, uint32_t n) { return v == 0 ? n - 1 : v - 1; }

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

// North-East constraint on the Ising energy (Sec. 3.2 with J != 0): an
// allowed move n -> 1 - n is the spin-1/2 move s -> -s of s = 2n - 1, with
// nsum over the four neighbours' 2n - 1 (spin-1/2 table, z = 4).
__device__ __forceinline__ int move_ne_coupled(int byte, int north, int east, int south, int west,
                                               uint32_t u, const uint64_t* lut)
{
    if (!((north & east) & 1)) return byte;
    const int n = byte & 1;
    const int s = 2 * n - 1;
    const int nsum = 2 * ((north & 1) + (east & 1) + (south & 1) + (west & 1)) - 4;
    return move_ising_half(s, nsum, u, lut, 4) != s ? ((n ^ 1) | 2) : byte;
}

// ---------------------------------------------------------------------------
// Direct update of one 4-site word gi of colour c: the neighbours are read
// straight from the other colour array (global memory, or LDS in the resident
// kernel).  With update == 0 only the observables of the current state are
// accumulated (record r_0).  `coupled` (NE only) takes the Ising rates of the
// spin-1/2 table instead of the two J = 0 thresholds.
template <int KIND, int DIM>
__device__ __forceinline__ void simple_word(uint8_t* own, const int8_t* oth, const Geom& g, uint32_t c,
                                            uint64_t gi, uint32_t t, int update, const PhiloxKey& ks,
                                            const uint64_t* lut, bool coupled, int32_t& q_bond,
                                            int32_t& q_mag, int32_t& q_acc, int32_t& q_unfl)
{
    {
        const bool upd = update != 0;
        const uint64_t k0 = gi * 4;
        const uint64_t row = k0 / g.Lh;
        const uint32_t kk0 = (uint32_t)(k0 - row * g.Lh);
        const uint32_t y = (uint32_t)(row % g.L);
        const uint32_t zc = DIM == 3 ? (uint32_t)(row / g.L) : 0u;
        const uint32_t p = (y + zc + c) & 1u;
        const uint64_t r_ym = (uint64_t)zc * g.L + wrap_dec(y, g.L);
        const uint64_t r_yp = (uint64_t)zc * g.L + wrap_inc(y, g.L);
        const uint64_t r_zm = (uint64_t)wrap_dec(zc, g.L) * g.L + y;
        const uint64_t r_zp = (uint64_t)wrap_inc(zc, g.L) * g.L + y;

        const uint32_t cur = *reinterpret_cast<const uint32_t*>(own + k0);
        Words4 wa = {{0, 0, 0, 0}}, wb = {{0, 0, 0, 0}};
        if (upd) {
            if (KIND == KIND_ISING_ONE) {
                wa = philox4x32_10((uint32_t)(2 * gi), c, t, 0u, ks);
                wb = philox4x32_10((uint32_t)(2 * gi + 1), c, t, 0u, ks);
            } else {
                wa = philox4x32_10((uint32_t)gi, c, t, 0u, ks);
            }
        }
        constexpr int z = 2 * DIM;
        uint32_t out = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const uint32_t kk = kk0 + b;
            const uint32_t kside = p ? wrap_inc(kk, g.Lh) : wrap_dec(kk, g.Lh);
            const int sv = (int)(int8_t)(uint8_t)(cur >> (8 * b));
            int nv;
            if (KIND == KIND_NE) {
                const int north = oth[r_ym * g.Lh + kk];
                const int east = oth[row * g.Lh + (p ? kside : kk)];
                int south = 0, west = 0;
                if (c == 1 || coupled) {
                    south = oth[r_yp * g.Lh + kk];
                    west = oth[row * g.Lh + (p ? kk : kside)];
                }
                if (!upd) nv = sv;
                else if (coupled) nv = move_ne_coupled(sv, north, east, south, west, wa.w[b], lut);
                else nv = move_ne(sv, north, east, wa.w[b], lut[0], lut[1]);
                q_mag += nv & 1;
                q_unfl += (nv & 2) ? 0 : 1;
                if (c == 1) q_bond += (nv & 1) * ((north & 1) + (east & 1) + (south & 1) + (west & 1));
            } else {
                int nsum = oth[row * g.Lh + kk] + oth[row * g.Lh + kside] + oth[r_ym * g.Lh + kk] +
                           oth[r_yp * g.Lh + kk];
                if (DIM == 3) nsum += oth[r_zm * g.Lh + kk] + oth[r_zp * g.Lh + kk];
                if (!upd) {
                    nv = sv;
                } else if (KIND == KIND_ISING_HALF) {
                    nv = move_ising_half(sv, nsum, wa.w[b], lut, z);
                } else {
                    const Words4& w = (b < 2) ? wa : wb;
                    nv = move_ising_one(sv, nsum, w.w[(b & 1) * 2], w.w[(b & 1) * 2 + 1], lut, z);
                }
                q_mag += nv;
                if (c == 1) q_bond += nv * nsum;
            }
            q_acc += (nv != sv) ? 1 : 0;
            out |= (uint32_t)(uint8_t)(int8_t)nv << (8 * b);
        }
        if (upd) *reinterpret_cast<uint32_t*>(own + k0) = out;
    }
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

// Small lattices: one workgroup holds both colour arrays in LDS and runs
// `nsweeps` whole sweeps in one launch (colour 0, barrier, colour 1, barrier,
// record), so the sweep costs no launch.  Record s goes to acc + s slots; the
// sweep index of sweep s is a.t + s.  The lattice is written back at the end.
constexpr int kResidentBlock = 512;

template <int KIND, int DIM>
__global__ void __launch_bounds__(kResidentBlock) k_resident(SweepArgs a, uint32_t nsweeps)
{
    extern __shared__ __align__(16) uint8_t sm[];
    __shared__ uint64_t lut[kMaxLut];
    const uint64_t nh = a.g.nh;
    const uint32_t nwords = (uint32_t)(nh >> 2);
    for (uint32_t i = threadIdx.x; i < nwords; i += kResidentBlock) {
        reinterpret_cast<uint32_t*>(sm)[i] = reinterpret_cast<const uint32_t*>(a.col[0])[i];
        reinterpret_cast<uint32_t*>(sm + nh)[i] = reinterpret_cast<const uint32_t*>(a.col[1])[i];
    }
    for (int i = threadIdx.x; i < a.lut_n; i += kResidentBlock) lut[i] = a.lut[i];
    __syncthreads();
    const PhiloxKey ks = philox_schedule(a.key0, a.key1);
    const bool coupled = KIND == KIND_NE && a.lut_n > 2;
    for (uint32_t s = 0; s < nsweeps; ++s) {
        int32_t q_bond = 0, q_mag = 0, q_acc = 0, q_unfl = 0;
#pragma unroll
        for (uint32_t c = 0; c < 2; ++c) {
            uint8_t* own = sm + c * nh;
            const int8_t* oth = reinterpret_cast<const int8_t*>(sm + (c ^ 1u) * nh);
            for (uint32_t gi = threadIdx.x; gi < nwords; gi += kResidentBlock)
                simple_word<KIND, DIM>(own, oth, a.g, c, gi, a.t + s, 1, ks, lut, coupled, q_bond, q_mag,
                                       q_acc, q_unfl);
            __syncthreads();
        }
        block_accumulate(q_bond, q_mag, q_acc, q_unfl, a.acc + (uint64_t)s * kSlotWords);
    }
    for (uint32_t i = threadIdx.x; i < nwords; i += kResidentBlock) {
        reinterpret_cast<uint32_t*>(a.col[0])[i] = reinterpret_cast<const uint32_t*>(sm)[i];
        reinterpret_cast<uint32_t*>(a.col[1])[i] = reinterpret_cast<const uint32_t*>(sm + nh)[i];
    }
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
