// row_device.hpp -- device code of the whole-row streaming checkerboard kernels (gfx950).
//
// A row group of R lanes covers one whole colour row (ncols = L/8 four-byte
// words): each lane holds D consecutive words (D*4 same-colour sites) and
// loads them with one 4*D-byte access.  Because the group spans the row, the
// periodic same-row neighbours never leave it: inside a lane they come from
// the lane's own words, across lanes from a lane shift (DPP within a wave,
// LDS between the waves of a group when R > 64).  The group walks down a
// strip of rows keeping the other colour's rows y-1, y, y+1 in registers and
// prefetching the next row's words while it computes the current one.
//
// HALF (2D and 3D): one colour in place per launch (reads only the other
// colour and its own words), two launches per sweep.
// FUSED (2D): both colours of a strip per launch; the colour-0 rows just
// above and below the strip are recomputed (bit-identical, counter-based
// random numbers) and the sweep reads one copy of the lattice and writes the
// other, since neighbouring strips read those rows.
//
// Spin-1/2 acceptance uses a 32-bit table of thr-1 (requires every threshold
// >= 1; the runtime sends other tables to the generic kernels).
//
// Neighbour words are "prepared" once per row and reused by the three rows
// that read them: spin-1/2 keeps bit 2 of each byte (4 per -1 spin), so the
// sum of prepared neighbours is 4 x (number of -1 neighbours) per byte;
// spin-1 keeps s+1; NE keeps n.  The row parity p (which side the same-row
// neighbour sits on) is a template parameter chosen by a uniform branch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "philox.hpp"
#include "site_update.hpp"
#include "spinlat_internal.h"

namespace spinlat {

namespace rowk {

constexpr uint32_t M4 = 0x04040404u;

struct RowGeom {
    uint32_t L, Lh, ncols;
    uint32_t D;       // words per lane
    uint32_t R;       // lanes per row group
    uint32_t slots;   // row groups per wave (R <= 64)
    uint32_t nw;      // waves per row group (R > 64)
    uint32_t nplanes, H, nstrips, nitems;
    uint32_t block;   // threads per block
    uint32_t rdiv;    // ceil(2^16 / R): lane / R == (lane * rdiv) >> 16 for every lane < 64
    uint32_t K;       // row sets per wave (row-group kernels)
    uint32_t rag;     // row-group kernels: words of the row in the last lane when D does not
                      // divide ncols (then 1 .. D-1), else 0
};

__host__ __device__ inline uint32_t cdiv(uint32_t a, uint32_t b) { return (a + b - 1) / b; }

__device__ __forceinline__ uint32_t wrapr(int y, uint32_t L)
{
    int r = y % (int)L;
    return (uint32_t)(r < 0 ? r + (int)L : r);
}

// Periodic row index for y in [-L, 2L): the walks step at most a few rows
// past an edge, so two compares replace the integer division of wrapr.
__device__ __forceinline__ uint32_t wrap1(int y, uint32_t L)
{
    return (uint32_t)(y < 0 ? y + (int)L : (y >= (int)L ? y - (int)L : y));
}

__device__ __forceinline__ uint32_t remap_block()
{
    const uint32_t nb = gridDim.x;
    uint32_t b = blockIdx.x;
    if ((nb & 7u) == 0) b = (b & 7u) * (nb >> 3) + (b >> 3);
    return b;
}

template <int D>
struct Vec {
    uint32_t w[D];
};

template <int D>
__device__ __forceinline__ Vec<D> ldv(const uint8_t* base, uint64_t off)
{
    Vec<D> v;
    if constexpr (D == 4) {
        const uint4 q = *reinterpret_cast<const uint4*>(base + off);
        v.w[0] = q.x; v.w[1] = q.y; v.w[2] = q.z; v.w[3] = q.w;
    } else if constexpr (D == 2) {
        const uint2 q = *reinterpret_cast<const uint2*>(base + off);
        v.w[0] = q.x; v.w[1] = q.y;
    } else {
        v.w[0] = *reinterpret_cast<const uint32_t*>(base + off);
    }
    return v;
}

template <int D>
__device__ __forceinline__ void stv(uint8_t* base, uint64_t off, const Vec<D>& v)
{
    if constexpr (D == 4) {
        *reinterpret_cast<uint4*>(base + off) = make_uint4(v.w[0], v.w[1], v.w[2], v.w[3]);
    } else if constexpr (D == 2) {
        *reinterpret_cast<uint2*>(base + off) = make_uint2(v.w[0], v.w[1]);
    } else {
        *reinterpret_cast<uint32_t*>(base + off) = v.w[0];
    }
}

// Cross-lane neighbour word.  For row parity p = 0 a lane needs the last word
// of the lane to its left, for p = 1 the first word of the lane to its right
// (periodic within the row group).
struct Lanes {
    uint32_t lane, wave, slot, pos, src_l, src_r;  // wave is wave-uniform
    uint32_t col0;  // first word of the row this lane holds (D * pos but in a ragged last lane)
};

template <bool XW, int P>
__device__ __forceinline__ uint32_t shift_in(uint32_t last, uint32_t first, const Lanes& ln, uint32_t e)
{
    // e: value the wave-edge lane takes (from LDS) when XW
    if constexpr (XW) {
        if constexpr (P == 0) return (uint32_t)__builtin_amdgcn_update_dpp((int)e, (int)last, 0x138, 0xF, 0xF, false);
        else return (uint32_t)__builtin_amdgcn_update_dpp((int)e, (int)first, 0x130, 0xF, 0xF, false);
    } else {
        if constexpr (P == 0) return (uint32_t)__shfl((int)last, (int)ln.src_l, 64);
        else return (uint32_t)__shfl((int)first, (int)ln.src_r, 64);
    }
}

// Aligned neighbour words of the D words of a lane in the same row (P = row
// parity): P = 0 takes the site to the left (k-1), P = 1 to the right (k+1);
// x is the adjacent lane's edge word.
template <int D, int P>
__device__ __forceinline__ void side_words(const Vec<D>& o, uint32_t x, uint32_t (&s)[D])
{
#pragma unroll
    for (int d = 0; d < D; ++d) {
        if constexpr (P == 0) {
            const uint32_t prev = d > 0 ? o.w[d > 0 ? d - 1 : 0] : x;
            s[d] = __builtin_amdgcn_alignbyte(o.w[d], prev, 3);
        } else {
            const uint32_t next = d < D - 1 ? o.w[d < D - 1 ? d + 1 : 0] : x;
            s[d] = __builtin_amdgcn_alignbyte(next, o.w[d], 1);
        }
    }
}

// Edge words a lane passes to its neighbours for shift_in, and how many of
// its first words another lane also holds and counts.  Ragged rows (RAG):
// ncols = (R - 1) D + rag and the last lane holds words ncols - D .. ncols - 1,
// so its first D - rag words are also lane R-2's last ones.  Both copies of
// such a word see the same neighbours and random numbers, so they store the
// same value; only lane R-2's copy is counted.  For that, for p = 0 lane R-2
// passes word rag - 1 (the one before the last lane's first word), for p = 1
// the last lane passes word D - rag (the one after lane R-2's last word).
template <int D, int P, bool RAG>
__device__ __forceinline__ uint32_t edge_words(const Vec<D>& q, const RowGeom& rg, const Lanes& ln, uint32_t& last,
                                               uint32_t& first)
{
    last = q.w[D - 1];
    first = q.w[0];
    if constexpr (RAG) {
        static_assert(D > 1, "one word per lane divides every row");
        const uint32_t r = rg.rag;  // 1 .. D-1, wave-uniform
        if constexpr (P == 0) {
            const uint32_t w = D == 2 ? q.w[0] : (r == 1 ? q.w[0] : r == 2 ? q.w[1 % D] : q.w[2 % D]);
            if (ln.pos + 2 == rg.R) last = w;
        } else {
            const uint32_t w = D == 2 ? q.w[1 % D] : (r == 1 ? q.w[3 % D] : r == 2 ? q.w[2 % D] : q.w[1 % D]);
            if (ln.pos + 1 == rg.R) first = w;
        }
        return ln.pos + 1 == rg.R ? D - r : 0u;
    }
    return 0u;
}

// ---- tables ---------------------------------------------------------------
struct RowLuts {
    uint64_t e[3 * 2 * 13];  // spin-1 entries; spin-1/2 uses the first words as u32
};

// Kernel kind of NE lattices with the Ising coupling: the NE code paths (every
// kind other than the two Ising ones), with the spin-1/2 table and move.
constexpr int KIND_NE_COUPLED = 3;

template <int KIND, int DIM>
__device__ __forceinline__ void build_row_luts(RowLuts& lut, const uint64_t* table, uint64_t& thr_up,
                                               uint64_t& thr_down)
{
    constexpr int z = 2 * DIM;
    // entries each kind reads: spin-1/2 tables 2 (z + 1), spin-1 6 (2z + 1), NE none
    constexpr int n = (KIND == KIND_ISING_HALF || KIND == KIND_NE_COUPLED) ? 2 * (z + 1)
                      : KIND == KIND_ISING_ONE                             ? 6 * (2 * z + 1)
                                                                           : 0;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        if (KIND == KIND_ISING_HALF || KIND == KIND_NE_COUPLED) {
            if (t < 2 * (z + 1)) {
                // entry nd + sneg*(z+1): nd neighbours at -1, sneg = (s == -1)
                const int sneg = t / (z + 1), nd = t % (z + 1);
                const int s = sneg ? -1 : 1;
                const int nsum = z - 2 * nd;
                const int di = s > 0 ? 0 : 3;
                // thr >= 1 here: accept iff word <= thr - 1
                reinterpret_cast<uint32_t*>(lut.e)[t] =
                    (uint32_t)(table[di * (2 * z + 1) + nsum + z] - 1ull);
            }
        } else if (KIND == KIND_ISING_ONE) {
            const int nz = t % (2 * z + 1);
            const int ch = (t / (2 * z + 1)) & 1;
            const int s = t / (2 * (2 * z + 1)) - 1;
            const int av = (s == -1) ? 0 : -1;
            const int bv = (s == 1) ? 0 : 1;
            const int sp = ch ? bv : av;
            const uint64_t thr = table[ds_index(sp - s) * (2 * z + 1) + nz];
            lut.e[t] = thr | ((uint64_t)(uint32_t)(sp + 1) << 40);
        }
    }
    thr_up = table[0];
    thr_down = table[1];
}

struct Obs {
    int32_t acc;   // spin-1/2: 7 x accepted moves; others: accepted moves
    int32_t mag0;  // sum of s (NE: n) over colour-0 words
    int32_t mag1;  // same over colour-1 words
    int32_t dd;    // spin-1/2: sum s' * 4 nd; spin-1: sum s' * (nsum + z); NE: bond
    int32_t unfl;  // NE: sites with the flip flag clear
};

// prepared form of an other-colour word
template <int KIND>
__device__ __forceinline__ uint32_t prep(uint32_t w)
{
    if constexpr (KIND == KIND_ISING_HALF) return w & M4;
    else if constexpr (KIND == KIND_ISING_ONE) return (w ^ 0x80808080u) + 0x80808081u;  // s+1, no carries
    else return w & 0x01010101u;
}

template <int KIND, int D>
__device__ __forceinline__ Vec<D> prepv(const Vec<D>& v)
{
    Vec<D> o;
#pragma unroll
    for (int d = 0; d < D; ++d) o.w[d] = prep<KIND>(v.w[d]);
    return o;
}

__device__ __forceinline__ int dot4(uint32_t a, uint32_t b, int c)
{
    return __builtin_amdgcn_sdot4((int)a, (int)b, c, false);
}

// spin-1/2: nd4 = 4 x (number of -1 neighbours) per byte
__device__ __forceinline__ uint32_t half_word(uint32_t own, uint32_t nd4, const Words4& w,
                                              const uint8_t* lut_bytes, int z)
{
    const uint32_t idx4 = nd4 + (own & M4) * (uint32_t)(z + 1);
    uint32_t flip = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const uint32_t off = (idx4 >> (8 * b)) & 0xFFu;
        const uint32_t t = *reinterpret_cast<const uint32_t*>(lut_bytes + off);
        flip |= (w.w[b] <= t) ? (0xFEu << (8 * b)) : 0u;
    }
    return own ^ flip;
}

// spin-1: S = per-byte nsum + z
template <int DIM>
__device__ __forceinline__ uint32_t one_word(uint32_t own, uint32_t S, const Words4& wa, const Words4& wb,
                                             const RowLuts& lut, int& nacc)
{
    constexpr int z = 2 * DIM;
    const uint32_t ob = prep<KIND_ISING_ONE>(own);
    uint32_t out = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const Words4& w = b < 2 ? wa : wb;
        const uint32_t ua = w.w[(b & 1) * 2];
        const uint32_t up = w.w[(b & 1) * 2 + 1];
        const uint32_t s1 = (ob >> (8 * b)) & 0xFFu;
        const uint32_t nz = (S >> (8 * b)) & 0xFFu;
        const uint64_t ent = lut.e[(s1 * 2 + (up >> 31)) * (2 * z + 1) + nz];
        const bool acc = (uint64_t)ua < (ent & 0x1FFFFFFFFull);
        const uint32_t n1 = acc ? (uint32_t)(ent >> 40) : s1;
        nacc += acc ? 1 : 0;
        out |= ((n1 - 1u) & 0xFFu) << (8 * b);
    }
    return out;
}

// NE constraint on the Ising energy (Sec. 3.2 with J != 0): a site whose north
// and east neighbours are up takes the spin-1/2 move of s = 2n - 1.  S holds
// the number of up neighbours per byte, so the table entry nd + sneg*5 (nd
// neighbours down, sneg = 1 - n) is 9 - S - 5n, with no borrow between bytes.
__device__ __forceinline__ uint32_t ne_coupled_word(uint32_t own, uint32_t north, uint32_t east, uint32_t S,
                                                    uint32_t g, uint32_t colour, uint32_t t,
                                                    const PhiloxKey& ks, const RowLuts& lut)
{
    const uint32_t n = own & 0x01010101u;
    const uint32_t allowed = north & east;
    uint32_t f = 0;
    if (__builtin_amdgcn_ballot_w64(allowed != 0u) != 0ull) {
        const Words4 w = philox4x32_10(g, colour, t, 0u, ks);
        const uint32_t idx = 0x09090909u - S - n * 5u;
        const uint32_t* thr_m1 = reinterpret_cast<const uint32_t*>(lut.e);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const uint32_t bit = 1u << (8 * b);
            if ((allowed & bit) && w.w[b] <= thr_m1[(idx >> (8 * b)) & 0xFFu]) f |= bit;
        }
    }
    return (own ^ f) | (f << 1);
}

__device__ __forceinline__ uint32_t ne_word(uint32_t own, uint32_t north, uint32_t east, uint32_t g,
                                            uint32_t colour, uint32_t t, const PhiloxKey& ks,
                                            uint64_t thr_up, uint64_t thr_down)
{
    // north, east: prepared (n bits)
    const uint32_t n = own & 0x01010101u;
    const uint32_t allowed = north & east;
    const uint32_t up = allowed & ~n;
    const uint32_t down = allowed & n;
    const bool up_rand = thr_up < (1ull << 32);
    const bool down_rand = thr_down < (1ull << 32);
    const uint32_t need = (up_rand ? up : 0u) | (down_rand ? down : 0u);
    uint32_t f = (up_rand ? 0u : up) | (down_rand ? 0u : down);
    if (__builtin_amdgcn_ballot_w64(need != 0u) != 0ull) {
        const Words4 w = philox4x32_10(g, colour, t, 0u, ks);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const uint32_t bit = 1u << (8 * b);
            const uint32_t thr = (uint32_t)((n & bit) ? thr_down : thr_up);
            if ((need & bit) && w.w[b] < thr) f |= bit;
        }
    }
    return (own ^ f) | (f << 1);
}

// Update the D words of one lane in one row.  Neighbour words are prepared;
// `side` are the prepared same-row neighbours aligned to the words.
// RAG (Ising kinds): the first `uncounted` words of this lane are also held,
// and counted, by another lane; they are updated and stored alike but left
// out of the observables.
template <int KIND, int DIM, int D, int P, bool RAG = false>
__device__ __forceinline__ Vec<D> row_update(const Vec<D>& own, const Vec<D>& same, const uint32_t (&side)[D],
                                             const Vec<D>& up, const Vec<D>& down, const Vec<D>* zm,
                                             const Vec<D>* zp, uint32_t g0, uint32_t colour, uint32_t t,
                                             const PhiloxKey& ks, const RowLuts& lut, uint64_t thr_up,
                                             uint64_t thr_down, bool count, Obs& o, const Words4* pre = nullptr,
                                             uint32_t uncounted = 0)
{
    // pre: the words' Philox outputs (spin-1: two per word), when the caller drew them
    static_assert(!RAG || KIND == KIND_ISING_HALF || KIND == KIND_ISING_ONE, "ragged rows: Ising kinds");
    constexpr int z = 2 * DIM;
    Vec<D> out;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const uint32_t g = g0 + d;
        if constexpr (KIND == KIND_ISING_HALF || KIND == KIND_ISING_ONE) {
            uint32_t S = same.w[d] + side[d] + up.w[d] + down.w[d];
            if constexpr (DIM == 3) S += zm->w[d] + zp->w[d];
            if constexpr (KIND == KIND_ISING_HALF) {
                const Words4 w = pre ? pre[d] : philox4x32_10(g, colour, t, 0u, ks);
                out.w[d] = half_word(own.w[d], S, w, reinterpret_cast<const uint8_t*>(lut.e), z);
                if (count) {
                    uint32_t ow = out.w[d], iw = own.w[d];
                    if constexpr (RAG) {
                        const uint32_t m = (uint32_t)d < uncounted ? 0u : ~0u;
                        ow &= m;
                        iw &= m;
                    }
                    o.acc += __builtin_popcount(iw ^ ow);
                    if (colour == 0) {
                        o.mag0 = dot4(ow, 0x01010101u, o.mag0);
                    } else {
                        o.mag1 = dot4(ow, 0x01010101u, o.mag1);
                        o.dd = dot4(ow, S, o.dd);
                    }
                }
            } else {
                const Words4 wa = pre ? pre[2 * d] : philox4x32_10(2 * g, colour, t, 0u, ks);
                const Words4 wb = pre ? pre[2 * d + 1] : philox4x32_10(2 * g + 1, colour, t, 0u, ks);
                int nacc = 0;
                out.w[d] = one_word<DIM>(own.w[d], S, wa, wb, lut, nacc);
                if (count) {
                    uint32_t ow = out.w[d];
                    if constexpr (RAG) {
                        const uint32_t m = (uint32_t)d < uncounted ? 0u : ~0u;
                        ow &= m;
                        nacc &= (int)m;
                    }
                    o.acc += nacc;
                    if (colour == 0) {
                        o.mag0 = dot4(ow, 0x01010101u, o.mag0);
                    } else {
                        o.mag1 = dot4(ow, 0x01010101u, o.mag1);
                        o.dd = dot4(ow, S, o.dd);
                    }
                }
            }
        } else {
            // north = row y-1; east = site x+1 (side word when p = 1)
            const uint32_t east = P ? side[d] : same.w[d];
            const uint32_t west = P ? same.w[d] : side[d];
            if constexpr (KIND == KIND_NE_COUPLED)
                out.w[d] = ne_coupled_word(own.w[d], up.w[d], east, up.w[d] + down.w[d] + east + west, g,
                                           colour, t, ks, lut);
            else
                out.w[d] = ne_word(own.w[d], up.w[d], east, g, colour, t, ks, thr_up, thr_down);
            if (count) {
                const uint32_t n = out.w[d] & 0x01010101u;
                o.acc += __builtin_popcount((own.w[d] ^ out.w[d]) & 0x01010101u);
                o.mag0 += __builtin_popcount(n);
                o.unfl += 4 - __builtin_popcount(out.w[d] & 0x02020202u);
                if (colour == 1) o.dd = dot4(n, up.w[d] + down.w[d] + east + west, o.dd);
            }
        }
    }
    return out;
}

// Record units per lane: {bond_sum, mag, accepted, unflipped}.
template <int KIND, int DIM>
__device__ __forceinline__ void finish_obs(const Obs& o, int32_t& bond, int32_t& mag, int32_t& acc,
                                           int32_t& unfl)
{
    constexpr int z = 2 * DIM;
    if constexpr (KIND == KIND_ISING_HALF) {
        // sum_b s'_b nsum_b = z sum s' - 2 sum s' nd, and dd = sum s' * 4 nd
        bond = z * o.mag1 - o.dd / 2;
        mag = o.mag0 + o.mag1;
        acc = o.acc / 7;
        unfl = 0;
    } else if constexpr (KIND == KIND_ISING_ONE) {
        bond = o.dd - z * o.mag1;  // dd = sum s' (nsum + z)
        mag = o.mag0 + o.mag1;
        acc = o.acc;
        unfl = 0;
    } else {
        bond = o.dd;
        mag = o.mag0;
        acc = o.acc;
        unfl = o.unfl;
    }
}

__device__ __forceinline__ Lanes lanes_of(const RowGeom& rg, bool xw)
{
    Lanes ln;
    ln.lane = threadIdx.x & 63u;
    // uniform across the wave: what depends only on it stays on the scalar unit
    ln.wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (xw) {
        ln.slot = 0;
        ln.pos = threadIdx.x;
        ln.src_l = ln.src_r = 0;
        ln.col0 = rg.D * ln.pos;
    } else {
        const uint32_t slot = __umul24(ln.lane, rg.rdiv) >> 16;  // ln.lane / rg.R
        ln.slot = slot;
        ln.pos = ln.lane - slot * rg.R;
        const uint32_t base = slot * rg.R;
        ln.src_l = base + (ln.pos == 0 ? rg.R - 1 : ln.pos - 1);
        ln.src_r = base + (ln.pos + 1 == rg.R ? 0 : ln.pos + 1);
        // a ragged row's last lane holds the row's last D words, rag of them its own
        ln.col0 = rg.D * ln.pos - (rg.rag != 0 && ln.pos + 1 == rg.R ? rg.D - rg.rag : 0u);
    }
    return ln;
}

// Item (strip, plane) of this lane, or >= nitems if idle.
__device__ __forceinline__ uint32_t row_item(const RowGeom& rg, bool xw, const Lanes& ln)
{
    const uint32_t b = remap_block();
    if (xw) return b;
    if (ln.slot >= rg.slots) return 0xFFFFFFFFu;
    return (b * (blockDim.x >> 6) + ln.wave) * rg.slots + ln.slot;
}

// ---- HALF -----------------------------------------------------------------
template <int KIND, int DIM, int D>
struct HalfState {
    Vec<D> Om, O0, Op;    // prepared other-colour rows y-1, y, y+1
    Vec<D> own;           // own words of row y
    Vec<D> Opn, ownn;     // prefetched: other row y+2 (raw), own row y+1
    Vec<D> zm, zp;        // prepared planes z-1, z+1 at row y (3D)
    Vec<D> zmn, zpn;      // prefetched (raw)
};

template <int KIND, int DIM, int D, bool XW, int P>
__device__ __forceinline__ void half_step(uint32_t y, HalfState<KIND, DIM, D>& st, const RowGeom& rg,
                                          const Lanes& ln, const uint8_t* O, uint8_t* A, uint64_t plane,
                                          uint64_t planem, uint64_t planep, uint32_t (&xch)[2][16][2],
                                          uint32_t& buf, const SweepArgs& a, const PhiloxKey& ks,
                                          const RowLuts& lut, uint64_t thr_up, uint64_t thr_down, Obs& o)
{
    const uint32_t L = rg.L;
    const uint64_t rowb = rg.Lh;
    const uint64_t cb = 4ull * D * ln.pos;
    const uint32_t yn = y + 1 == L ? 0 : y + 1;
    const uint32_t ynn = yn + 1 == L ? 0 : yn + 1;
    st.Opn = ldv<D>(O, (plane + ynn) * rowb + cb);
    st.ownn = ldv<D>(A, (plane + yn) * rowb + cb);
    if constexpr (DIM == 3) {
        st.zmn = ldv<D>(O, (planem + yn) * rowb + cb);
        st.zpn = ldv<D>(O, (planep + yn) * rowb + cb);
    }
    uint32_t e = 0;
    if constexpr (XW) {
        const uint32_t nwv = rg.nw;
        if (ln.lane == 63) xch[buf][ln.wave][1] = st.O0.w[D - 1];
        if (ln.lane == 0) xch[buf][ln.wave][0] = st.O0.w[0];
        __syncthreads();
        if constexpr (P == 0) {
            if (ln.lane == 0) e = xch[buf][ln.wave == 0 ? nwv - 1 : ln.wave - 1][1];
        } else {
            if (ln.lane == 63) e = xch[buf][ln.wave + 1 == nwv ? 0 : ln.wave + 1][0];
        }
        buf ^= 1u;
    }
    const uint32_t x = shift_in<XW, P>(st.O0.w[D - 1], st.O0.w[0], ln, e);
    uint32_t side[D];
    side_words<D, P>(st.O0, x, side);
    const uint32_t c = a.colour;
    const uint32_t g0 = (uint32_t)((plane + y) * rg.ncols + (uint64_t)D * ln.pos);
    const Vec<D> nw = row_update<KIND, DIM, D, P>(st.own, st.O0, side, st.Om, st.Op, &st.zm, &st.zp, g0, c,
                                                  a.t, ks, lut, thr_up, thr_down, true, o);
    stv<D>(A, (plane + y) * rowb + cb, nw);
    st.Om = st.O0;
    st.O0 = st.Op;
    st.Op = prepv<KIND, D>(st.Opn);
    st.own = st.ownn;
    if constexpr (DIM == 3) {
        st.zm = prepv<KIND, D>(st.zmn);
        st.zp = prepv<KIND, D>(st.zpn);
    }
}

// One item (strip of rows of one plane) of a half-sweep, for this lane.
template <int KIND, int DIM, int D, bool XW>
__device__ __forceinline__ void half_item(const SweepArgs& a, const RowGeom& rg, uint32_t item, const Lanes& ln,
                                          const RowLuts& lut, uint32_t (&xch)[2][16][2], uint64_t thr_up,
                                          uint64_t thr_down, Obs& o)
{
    if (item < rg.nitems) {  // block-uniform when XW
        const uint32_t strip = item % rg.nstrips;
        const uint32_t zp = item / rg.nstrips;
        const uint32_t L = rg.L;
        const uint32_t c = a.colour;
        const uint8_t* O = colour_array(a, c ^ 1u);
        uint8_t* A = colour_array(a, c);
        const uint64_t rowb = rg.Lh;
        const uint64_t cb = 4ull * D * ln.pos;
        const uint64_t plane = (uint64_t)zp * L;
        const uint64_t planem = (uint64_t)wrapr((int)zp - 1, L) * L;
        const uint64_t planep = (uint64_t)wrapr((int)zp + 1, L) * L;
        const uint32_t y0 = strip * rg.H;
        const uint32_t y1 = min(y0 + rg.H, L);
        const PhiloxKey ks = philox_schedule(a.key0, a.key1);

        HalfState<KIND, DIM, D> st;
        st.Om = prepv<KIND, D>(ldv<D>(O, (plane + wrapr((int)y0 - 1, L)) * rowb + cb));
        st.O0 = prepv<KIND, D>(ldv<D>(O, (plane + y0) * rowb + cb));
        st.Op = prepv<KIND, D>(ldv<D>(O, (plane + wrapr((int)y0 + 1, L)) * rowb + cb));
        st.own = ldv<D>(A, (plane + y0) * rowb + cb);
        if constexpr (DIM == 3) {
            st.zm = prepv<KIND, D>(ldv<D>(O, (planem + y0) * rowb + cb));
            st.zp = prepv<KIND, D>(ldv<D>(O, (planep + y0) * rowb + cb));
        }
        uint32_t buf = 0;
        for (uint32_t y = y0; y < y1; ++y) {
            if (((y + zp + c) & 1u) == 0)
                half_step<KIND, DIM, D, XW, 0>(y, st, rg, ln, O, A, plane, planem, planep, xch, buf, a, ks,
                                               lut, thr_up, thr_down, o);
            else
                half_step<KIND, DIM, D, XW, 1>(y, st, rg, ln, O, A, plane, planem, planep, xch, buf, a, ks,
                                               lut, thr_up, thr_down, o);
        }
    }
}

// ---- FUSED (2D) -------------------------------------------------------------
template <int KIND, int D>
struct FusedState {
    Vec<D> c1a, c1b;          // old colour-1 rows i-1, i (raw: c1a is updated at i-1)
    Vec<D> q1a, q1b, q1d;     // the same rows i-1, i, i+1 prepared
    Vec<D> c1d, c1n;          // raw row i+1, prefetched raw row i+2
    Vec<D> own0, own0n;       // old colour-0 row i, prefetched row i+1
    Vec<D> q0a, q0b;          // new colour-0 rows i-2, i-1 prepared
};

template <int KIND, int D, bool XW, int P, bool DO_C1, bool STORE0, bool PREF>
__device__ __forceinline__ void fused_step(int i, FusedState<KIND, D>& st, const RowGeom& rg, const Lanes& ln,
                                           const uint8_t* S0, const uint8_t* S1, uint8_t* D0, uint8_t* D1,
                                           uint32_t (&xch)[2][16][4], uint32_t& buf, const SweepArgs& a,
                                           const PhiloxKey& ks, const RowLuts& lut, uint64_t thr_up,
                                           uint64_t thr_down, Obs& o)
{
    const uint32_t L = rg.L;
    const uint64_t rowb = rg.Lh;
    const uint64_t cb = 4ull * D * ln.pos;
    const uint32_t yi = wrap1(i, L);
    if constexpr (PREF) {
        // for step i+1: old colour-1 row i+2, old colour-0 row i+1
        st.c1n = ldv<D>(S1, (uint64_t)wrap1(i + 2, L) * rowb + cb);
        st.own0n = ldv<D>(S0, (uint64_t)wrap1(i + 1, L) * rowb + cb);
    }
    uint32_t e0 = 0, e1 = 0;
    if constexpr (XW) {
        const uint32_t nwv = rg.nw;
        if (ln.lane == 63) {
            xch[buf][ln.wave][1] = st.q1b.w[D - 1];
            xch[buf][ln.wave][3] = st.q0b.w[D - 1];
        }
        if (ln.lane == 0) {
            xch[buf][ln.wave][0] = st.q1b.w[0];
            xch[buf][ln.wave][2] = st.q0b.w[0];
        }
        __syncthreads();
        if constexpr (P == 0) {
            if (ln.lane == 0) {
                const uint32_t wl = ln.wave == 0 ? nwv - 1 : ln.wave - 1;
                e0 = xch[buf][wl][1];
                e1 = xch[buf][wl][3];
            }
        } else {
            if (ln.lane == 63) {
                const uint32_t wr = ln.wave + 1 == nwv ? 0 : ln.wave + 1;
                e0 = xch[buf][wr][0];
                e1 = xch[buf][wr][2];
            }
        }
        buf ^= 1u;
    }
    // colour 0, row i (parity P): neighbours old colour-1 rows i-1, i, i+1
    const uint32_t x0 = shift_in<XW, P>(st.q1b.w[D - 1], st.q1b.w[0], ln, e0);
    uint32_t side0[D];
    side_words<D, P>(st.q1b, x0, side0);
    const uint32_t g0 = yi * rg.ncols + D * ln.pos;
    const Vec<D> new0 = row_update<KIND, 2, D, P>(st.own0, st.q1b, side0, st.q1a, st.q1d, nullptr, nullptr,
                                                  g0, 0u, a.t, ks, lut, thr_up, thr_down, STORE0, o);
    if constexpr (STORE0) stv<D>(D0, (uint64_t)yi * rowb + cb, new0);
    const Vec<D> q0 = prepv<KIND, D>(new0);
    if constexpr (DO_C1) {
        // colour 1, row i-1 (parity of i as well): neighbours new colour-0 rows i-2, i-1, i
        const uint32_t ym = wrap1(i - 1, L);
        const uint32_t x1 = shift_in<XW, P>(st.q0b.w[D - 1], st.q0b.w[0], ln, e1);
        uint32_t side1[D];
        side_words<D, P>(st.q0b, x1, side1);
        const uint32_t g1 = ym * rg.ncols + D * ln.pos;
        const Vec<D> new1 = row_update<KIND, 2, D, P>(st.c1a, st.q0b, side1, st.q0a, q0, nullptr, nullptr, g1,
                                                      1u, a.t, ks, lut, thr_up, thr_down, true, o);
        stv<D>(D1, (uint64_t)ym * rowb + cb, new1);
    }
    st.c1a = st.c1b;
    st.c1b = st.c1d;
    st.q1a = st.q1b;
    st.q1b = st.q1d;
    if constexpr (PREF) {
        st.c1d = st.c1n;
        st.q1d = prepv<KIND, D>(st.c1n);
        st.own0 = st.own0n;
    }
    st.q0a = st.q0b;
    st.q0b = q0;
}

template <int KIND, int D, bool XW, bool DO_C1, bool STORE0, bool PREF>
__device__ __forceinline__ void fused_step_p(int i, FusedState<KIND, D>& st, const RowGeom& rg,
                                             const Lanes& ln, const uint8_t* S0, const uint8_t* S1,
                                             uint8_t* D0, uint8_t* D1, uint32_t (&xch)[2][16][4],
                                             uint32_t& buf, const SweepArgs& a, const PhiloxKey& ks,
                                             const RowLuts& lut, uint64_t thr_up, uint64_t thr_down, Obs& o)
{
    // row parity of i (L is even, so wrapping keeps it)
    if ((i & 1) == 0)
        fused_step<KIND, D, XW, 0, DO_C1, STORE0, PREF>(i, st, rg, ln, S0, S1, D0, D1, xch, buf, a, ks, lut,
                                                         thr_up, thr_down, o);
    else
        fused_step<KIND, D, XW, 1, DO_C1, STORE0, PREF>(i, st, rg, ln, S0, S1, D0, D1, xch, buf, a, ks, lut,
                                                         thr_up, thr_down, o);
}

// Fused sweep (both colours) of strip `item` (rows item*H .. item*H + H - 1)
// for this lane's row group, reading copy (S0, S1) and writing (D0, D1).
// HT > 0: the strip height is the compile-time HT (even, dividing L), so every
// row's parity is known (y0 = item * HT is even) and the rows run in parity
// pairs with no per-row branch.  HT = 0: runtime strip height rg.H (any
// H >= 1, ragged last strip).
template <int KIND, int D, bool XW, int HT>
__device__ __forceinline__ void fused_item(const SweepArgs& a, const RowGeom& rg, uint32_t item, const Lanes& ln,
                                           const RowLuts& lut, uint32_t (&xch)[2][16][4], uint64_t thr_up,
                                           uint64_t thr_down, const uint8_t* S0, const uint8_t* S1, uint8_t* D0,
                                           uint8_t* D1, Obs& o)
{
    if (item < rg.nitems) {
        const uint32_t L = rg.L;
        const uint64_t rowb = rg.Lh;
        const uint64_t cb = 4ull * D * ln.pos;
        const int H = HT > 0 ? HT : (int)rg.H;
        const int y0 = (int)(item * (uint32_t)H);
        const int y1 = min(y0 + H, (int)L);
        const PhiloxKey ks = philox_schedule(a.key0, a.key1);
        FusedState<KIND, D> st;
        st.c1a = ldv<D>(S1, (uint64_t)wrap1(y0 - 2, L) * rowb + cb);
        st.c1b = ldv<D>(S1, (uint64_t)wrap1(y0 - 1, L) * rowb + cb);
        st.c1d = ldv<D>(S1, (uint64_t)wrap1(y0, L) * rowb + cb);
        st.q1a = prepv<KIND, D>(st.c1a);
        st.q1b = prepv<KIND, D>(st.c1b);
        st.q1d = prepv<KIND, D>(st.c1d);
        st.own0 = ldv<D>(S0, (uint64_t)wrap1(y0 - 1, L) * rowb + cb);
#pragma unroll
        for (int d = 0; d < D; ++d) st.q0a.w[d] = st.q0b.w[d] = 0u;
        uint32_t buf = 0;
        // halo row y0-1 (colour 0 only, not stored), first row y0 (colour 0
        // only), rows y0+1 .. y1-1, halo row y1 (colour 1 of row y1-1 only)
        if constexpr (HT > 0) {
            // y0 is even, so row y0 + k has parity k & 1
            fused_step<KIND, D, XW, 1, false, false, true>(y0 - 1, st, rg, ln, S0, S1, D0, D1, xch, buf, a,
                                                           ks, lut, thr_up, thr_down, o);
            fused_step<KIND, D, XW, 0, false, true, true>(y0, st, rg, ln, S0, S1, D0, D1, xch, buf, a, ks,
                                                          lut, thr_up, thr_down, o);
            // rows y0 + 1 .. y0 + HT - 1 in pairs of parity (1, 0), then row y0 + HT - 1
#pragma nounroll
            for (int k = 1; k + 1 < HT; k += 2) {
                fused_step<KIND, D, XW, 1, true, true, true>(y0 + k, st, rg, ln, S0, S1, D0, D1, xch, buf, a, ks,
                                                             lut, thr_up, thr_down, o);
                fused_step<KIND, D, XW, 0, true, true, true>(y0 + k + 1, st, rg, ln, S0, S1, D0, D1, xch, buf, a,
                                                             ks, lut, thr_up, thr_down, o);
            }
            fused_step<KIND, D, XW, 1, true, true, true>(y0 + HT - 1, st, rg, ln, S0, S1, D0, D1, xch, buf, a, ks,
                                                         lut, thr_up, thr_down, o);
            fused_step<KIND, D, XW, 0, true, false, false>(y0 + HT, st, rg, ln, S0, S1, D0, D1, xch, buf, a,
                                                           ks, lut, thr_up, thr_down, o);
        } else {
            fused_step_p<KIND, D, XW, false, false, true>(y0 - 1, st, rg, ln, S0, S1, D0, D1, xch, buf, a, ks,
                                                          lut, thr_up, thr_down, o);
            fused_step_p<KIND, D, XW, false, true, true>(y0, st, rg, ln, S0, S1, D0, D1, xch, buf, a, ks, lut,
                                                         thr_up, thr_down, o);
            for (int i = y0 + 1; i < y1; ++i)
                fused_step_p<KIND, D, XW, true, true, true>(i, st, rg, ln, S0, S1, D0, D1, xch, buf, a, ks, lut,
                                                            thr_up, thr_down, o);
            fused_step_p<KIND, D, XW, true, false, false>(y1, st, rg, ln, S0, S1, D0, D1, xch, buf, a, ks, lut,
                                                          thr_up, thr_down, o);
        }
    }
}

// Host: whole-row geometry for strip height H and D words per lane.  With
// `ragged` (row-group kernels only) D need not divide the row: the group has
// ceil(ncols / D) >= 2 lanes, at most one wave, and its last lane holds the
// row's last D words, of which rg.rag are its own.
inline bool make_row_geom(const Geom& g, int H, int D, bool fused, RowGeom& rg, bool ragged = false)
{
    rg = RowGeom{};
    rg.L = g.L;
    rg.Lh = g.Lh;
    rg.ncols = g.Lh / 4;
    if (D != 1 && D != 2 && D != 4) return false;
    rg.D = (uint32_t)D;
    rg.rag = rg.ncols % rg.D;
    if (rg.rag && !ragged) return false;
    rg.R = cdiv(rg.ncols, rg.D);
    if (rg.R == 0 || (rg.rag && (rg.R < 2 || rg.R > 64))) return false;
    rg.rdiv = (65536u + rg.R - 1u) / rg.R;
    if (rg.R <= 64) {
        rg.slots = 64 / rg.R;
        rg.nw = 1;
        rg.block = 256;
    } else {
        if (rg.R % 64 || rg.R > 1024) return false;
        rg.slots = 1;
        rg.nw = rg.R / 64;
        rg.block = rg.R;
    }
    if (fused && g.dim != 2) return false;
    rg.nplanes = g.dim == 3 ? g.L : 1;
    rg.H = (uint32_t)H;
    rg.K = 1;
    rg.nstrips = cdiv(g.L, rg.H);
    rg.nitems = rg.nstrips * rg.nplanes;
    return true;
}

}  // namespace rowk

}  // namespace spinlat
