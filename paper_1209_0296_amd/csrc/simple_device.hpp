// simple_device.hpp -- the direct per-word site update (neighbours read
// straight from the other colour array, in global memory or LDS) and the
// resident multi-sweep body built on it; shared by kernels_simple.hip and the
// batched kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "philox.hpp"
#include "site_update.hpp"
#include "spinlat_internal.h"

namespace spinlat {
namespace simplek {

__device__ __forceinline__ uint32_t wrap_inc(uint32_t v, uint32_t n) { return v + 1 == n ? 0 : v + 1; }
__device__ __forceinline__ uint32_t wrap_dec(uint32_t v, uint32_t n) { return v == 0 ? n - 1 : v - 1; }

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

// Small lattices: one workgroup of kResidentBlock threads holds both colour
// arrays in LDS (`sm`, 2 nh bytes) and runs `nsweeps` whole sweeps (colour 0,
// barrier, colour 1, barrier, record), so a sweep costs no launch.  Record s
// goes to a.acc + s slots; the sweep index of sweep s is a.t + s.  The lattice
// is written back at the end.  `lut` is the threshold table in LDS.
constexpr int kResidentBlock = 512;

template <int KIND, int DIM>
__device__ __forceinline__ void resident_run(const SweepArgs& a, uint32_t nsweeps, uint8_t* sm, uint64_t* lut)
{
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

}  // namespace simplek
}  // namespace spinlat
