// site_update.hpp -- the single-site moves of the checkerboard sweep and the
// workgroup reduction of the per-sweep observables (device code).
//
// Ising (paper Sec. 3.1, Eq. 2 with field h): the move s -> s' is accepted
// with probability min[1, exp(-dE/T)], here as "word < thr[s'-s][nsum]" where
// thr is the host-built threshold table.  Spin-1/2 proposes s' = -s; spin-1
// proposes one of the two other values, chosen by a second word.
// North-East model (Sec. 3.2, Eq. 3, J = 0): the site may change only if its
// north and east neighbours are both up; an up-flip uses thr_up, a down-flip
// thr_down (table entries 0 and 1); bit 1 of the byte records "has flipped".
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spinlat_internal.h"

namespace spinlat {

// Table column of the spin change ds = s' - s in {-2,-1,+1,+2}.
__device__ __forceinline__ int ds_index(int ds) { return ds < 0 ? ds + 2 : ds + 1; }

// Spin-1/2: returns the new spin.
__device__ __forceinline__ int move_ising_half(int s, int nsum, uint32_t u, const uint64_t* lut,
                                               int z)
{
    const int di = s > 0 ? 0 : 3;  // ds = -2s
    const uint64_t thr = lut[di * (2 * z + 1) + nsum + z];
    return ((uint64_t)u < thr) ? -s : s;
}

// Spin-1: ua decides acceptance, up picks the lower other value iff < 2^31.
__device__ __forceinline__ int move_ising_one(int s, int nsum, uint32_t ua, uint32_t up,
                                              const uint64_t* lut, int z)
{
    // the two values other than s, a < b
    const int a = (s == -1) ? 0 : -1;
    const int b = (s == 1) ? 0 : 1;
    const int sp = (up < 0x80000000u) ? a : b;
    const uint64_t thr = lut[ds_index(sp - s) * (2 * z + 1) + nsum + z];
    return ((uint64_t)ua < thr) ? sp : s;
}

// North-East: byte = n | flag << 1; returns the new byte.
__device__ __forceinline__ int move_ne(int byte, int north, int east, uint32_t u,
                                       uint64_t thr_up, uint64_t thr_down)
{
    const int n = byte & 1;
    if (!((north & east) & 1)) return byte;
    const uint64_t thr = n ? thr_down : thr_up;
    return ((uint64_t)u < thr) ? ((n ^ 1) | 2) : byte;
}

// Workgroup barrier that orders LDS accesses only: global loads and stores in
// flight stay in flight across it (a full barrier also waits for them).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Sum of v over the 64 lanes of a wave whose lanes are all active, as a
// wave-uniform value: DPP butterflies inside each row of 16 lanes (quad
// permutes [1,0,3,2] and [2,3,0,1], then the half-row and row mirrors leave
// every lane holding its row's sum), then the four row sums read out.
__device__ __forceinline__ int32_t wave_sum(int32_t v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, false);
    return __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16) + __builtin_amdgcn_readlane(v, 32) +
           __builtin_amdgcn_readlane(v, 48);
}

// Sum four per-thread int32 partials over the workgroup and add them to one
// of the kSub sub-slots of the record (integer atomics: the result does not
// depend on the order).  blockDim.x must be a multiple of 64, <= 1024, and
// every thread of the block calls this.
__device__ __forceinline__ void block_accumulate(int32_t v0, int32_t v1, int32_t v2, int32_t v3,
                                                 unsigned long long* acc)
{
    __shared__ int32_t part[16][kQ];
    v0 = wave_sum(v0);
    v1 = wave_sum(v1);
    v2 = wave_sum(v2);
    v3 = wave_sum(v3);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    if (lane == 0) {
        part[wave][0] = v0;
        part[wave][1] = v1;
        part[wave][2] = v2;
        part[wave][3] = v3;
    }
    lds_barrier();
    if (threadIdx.x < kQ) {
        const int nw = blockDim.x >> 6;
        int64_t sum = 0;
        for (int w = 0; w < nw; ++w) sum += part[w][threadIdx.x];
        if (sum != 0)
            atomicAdd(&acc[(blockIdx.x % kSub) * kSubStride + threadIdx.x], (unsigned long long)sum);
    }
}

}  // namespace spinlat
