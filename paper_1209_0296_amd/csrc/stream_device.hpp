// stream_device.hpp -- device code of the window-streaming checkerboard kernels (gfx950).
//
// Work decomposition.  A colour row holds ncols = L/8 four-byte words (4
// same-colour sites each, one Philox4x32-10 call per word for one-word moves).
// A group of W lanes (W = ncols when ncols is a power of two <= 64, else 64)
// owns a window of columns and walks down a strip of rows of one plane,
// keeping the three other-colour rows it needs (y-1, y, y+1) in registers, so
// every byte is loaded from memory about once per half-sweep.  The same-row
// neighbour that lies one byte outside a lane's word comes from the adjacent
// lane (cross-lane permute); lanes at a window edge load it instead.
//
// HALF mode (2D and 3D) updates one colour in place per launch: colour c is
// written, only colour 1-c is read (plus each lane's own word), so the launch
// has no read-after-write hazard (the kernel end is the global barrier of
// Alg. I steps 6-7).
//
// FUSED mode (2D) updates both colours of a strip in one launch.  A strip's
// colour-1 rows need the new colour-0 values of one row above and below and
// of one column left and right, so those halo words are recomputed (the
// counter-based random numbers make the recomputation bit-identical to the
// owner's); window edges use two halo lanes.  Halo rows of the old lattice are
// read by neighbouring strips while this strip writes, so the sweep reads one
// copy of the lattice and writes the other (ping-pong).
//
// Per-sweep observables are accumulated per lane and reduced per workgroup
// into the record slot (see site_update.hpp).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "philox.hpp"
#include "site_update.hpp"
#include "spinlat_internal.h"

namespace spinlat {

namespace streamk {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr uint32_t M8 = 0x08080808u;

// -------------------------------------------------------------------------
// geometry of one launch
struct StreamGeom {
    uint32_t L, Lh, ncols, rows_per_plane, nplanes;
    uint32_t W, G;        // group width, groups per wave
    uint32_t wrap;        // group covers a whole row (W == ncols)
    uint32_t win_cols;    // owned columns per window
    uint32_t nwin, H, nstrips;
    uint32_t nitems;
};

__host__ __device__ inline uint32_t ceil_div(uint32_t a, uint32_t b) { return (a + b - 1) / b; }

__host__ inline StreamGeom make_geom(const Geom& g, int H, bool fused)
{
    StreamGeom s{};
    s.L = g.L;
    s.Lh = g.Lh;
    s.ncols = g.Lh / 4;
    s.rows_per_plane = g.L;
    s.nplanes = g.dim == 3 ? g.L : 1;
    const bool pow2 = (s.ncols & (s.ncols - 1)) == 0;
    if (s.ncols <= 64 && pow2) {
        s.W = s.ncols;
        s.wrap = 1;
        s.win_cols = s.ncols;
    } else {
        s.W = 64;
        s.wrap = 0;
        s.win_cols = fused ? 62 : 64;
    }
    s.G = 64 / s.W;
    s.nwin = ceil_div(s.ncols, s.win_cols);
    s.H = (uint32_t)H;
    s.nstrips = ceil_div(s.L, s.H);
    s.nitems = s.nwin * s.nstrips * s.nplanes;
    return s;
}

__device__ __forceinline__ uint32_t wrap_row(int y, uint32_t L)
{
    int r = y % (int)L;
    return (uint32_t)(r < 0 ? r + (int)L : r);
}

// Item of this lane group; consecutive items run along a row of windows, then
// down the strips, then through the planes.  Blocks are dealt round-robin to
// the 8 XCDs; remapping gives each XCD a contiguous band of items, so the
// halo rows two strips share are mostly fetched into one XCD's L2.
__device__ __forceinline__ uint32_t item_of_lane(const StreamGeom& sg)
{
    const uint32_t nb = gridDim.x;
    uint32_t b = blockIdx.x;
    if ((nb & 7u) == 0) b = (b & 7u) * (nb >> 3) + (b >> 3);
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = threadIdx.x >> 6;
    return (b * kWaves + wave) * sg.G + lane / sg.W;
}

// Same-row neighbour word aligned to this lane's four sites.  In row y of
// colour c the other colour's sites k and k-1 (p = 0) or k and k+1 (p = 1)
// neighbour in-colour site k, p = (y + z + c) & 1; `cur` is the other
// colour's word at this lane's column and `adj` the word one column to the
// left (p = 0) or right (p = 1).
__device__ __forceinline__ uint32_t side_word(uint32_t cur, uint32_t adj, uint32_t p)
{
    return p ? __builtin_amdgcn_alignbyte(adj, cur, 1) : __builtin_amdgcn_alignbyte(cur, adj, 3);
}

// -------------------------------------------------------------------------
// Threshold tables in LDS.  Ising spin-1/2: entry m + sneg*(z+1) for m
// neighbours anti-aligned with the spin and sneg = (s == -1); spin-1: entry
// ((s+1)*2 + ch)*(2z+1) + nsum + z holding thr | (s'+1) << 40.
struct Luts {
    uint64_t e[3 * 2 * 13];
};

template <int KIND, int DIM>
__device__ __forceinline__ void build_luts(Luts& lut, const uint64_t* table, uint64_t& thr_up,
                                           uint64_t& thr_down)
{
    constexpr int z = 2 * DIM;
    const int t = threadIdx.x;
    if (KIND == KIND_ISING_HALF) {
        if (t < 2 * (z + 1)) {
            const int sneg = t / (z + 1), m = t % (z + 1);
            const int s = sneg ? -1 : 1;
            const int nsum = s * (z - 2 * m);
            const int di = s > 0 ? 0 : 3;
            lut.e[t] = table[di * (2 * z + 1) + nsum + z];
        }
    } else if (KIND == KIND_ISING_ONE) {
        if (t < 6 * (2 * z + 1)) {
            const int nz = t % (2 * z + 1);
            const int ch = (t / (2 * z + 1)) & 1;
            const int s = t / (2 * (2 * z + 1)) - 1;
            const int a = (s == -1) ? 0 : -1;
            const int b = (s == 1) ? 0 : 1;
            const int sp = ch ? b : a;
            const int ds = sp - s;
            const uint64_t thr = table[ds_index(ds) * (2 * z + 1) + nz];
            lut.e[t] = thr | ((uint64_t)(uint32_t)(sp + 1) << 40);
        }
    }
    thr_up = table[0];
    thr_down = table[1];
}

// -------------------------------------------------------------------------
// Per-word moves.  `nb` are the other-colour neighbour words aligned to the
// four sites; `w`/`w2` the Philox words.

struct Obs {
    int32_t bond, mag, acc, unfl;
};

template <int DIM>
__device__ __forceinline__ uint32_t ising_half_word(uint32_t own, const uint32_t (&nb)[2 * DIM],
                                                    const Words4& w, const uint8_t* lut_bytes)
{
    constexpr int z = 2 * DIM;
    uint32_t mis = 0;
#pragma unroll
    for (int j = 0; j < z; ++j) mis += (nb[j] ^ own) & M8;  // 8 per anti-aligned neighbour
    const uint32_t idx8 = mis + (own & M8) * (uint32_t)(z + 1);
    uint32_t flip = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const uint32_t off = (idx8 >> (8 * b)) & 0xFFu;
        const uint64_t thr = *reinterpret_cast<const uint64_t*>(lut_bytes + off);
        flip |= ((uint64_t)w.w[b] < thr) ? (0xFEu << (8 * b)) : 0u;
    }
    return own ^ flip;
}

template <int DIM>
__device__ __forceinline__ void ising_half_obs(uint32_t own, uint32_t nw, const uint32_t (&nb)[2 * DIM],
                                               bool bond, Obs& o)
{
    constexpr int z = 2 * DIM;
    const int nflip = __builtin_popcount(own ^ nw) / 7;
    const int nneg = __builtin_popcount(nw & 0x02020202u);
    o.acc += nflip;
    o.mag += 4 - 2 * nneg;
    if (bond) {
        uint32_t mis = 0;
#pragma unroll
        for (int j = 0; j < z; ++j) mis += (nb[j] ^ nw) & M8;
        const uint32_t sum8 = __builtin_amdgcn_sad_u8(mis, 0u, 0u);  // 8 * anti-aligned bonds
        o.bond += 4 * z - (int)(sum8 >> 2);
    }
}

// biased value v+1 of each spin-1 byte (0xFF, 0, 1 -> 0, 1, 2), no carries
__device__ __forceinline__ uint32_t bias1(uint32_t v) { return (v ^ 0x80808080u) + 0x80808081u; }

template <int DIM>
__device__ __forceinline__ uint32_t ising_one_word(uint32_t own, const uint32_t (&nb)[2 * DIM],
                                                   const Words4& wa, const Words4& wb,
                                                   const Luts& lut, bool bond, bool count, Obs& o)
{
    constexpr int z = 2 * DIM;
    uint32_t S = 0;
#pragma unroll
    for (int j = 0; j < z; ++j) S += bias1(nb[j]);  // per byte nsum + z
    const uint32_t ob = bias1(own);
    uint32_t out = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const Words4& w = b < 2 ? wa : wb;
        const uint32_t ua = w.w[(b & 1) * 2];
        const uint32_t up = w.w[(b & 1) * 2 + 1];
        const uint32_t s1 = (ob >> (8 * b)) & 0xFFu;
        const uint32_t nz = (S >> (8 * b)) & 0xFFu;
        const uint32_t e = (s1 * 2 + (up >> 31)) * (2 * z + 1) + nz;
        const uint64_t ent = lut.e[e];
        const uint32_t nb1 = ((uint64_t)ua < (ent & 0x1FFFFFFFFull)) ? (uint32_t)(ent >> 40) : s1;
        out |= ((nb1 - 1u) & 0xFFu) << (8 * b);
        if (count) {
            o.acc += nb1 != s1;
            o.mag += (int)nb1 - 1;
            if (bond) o.bond += ((int)nb1 - 1) * ((int)nz - z);
        }
    }
    return out;
}

// North-East: north/east words aligned; returns the new word.  Random words
// are only drawn when some lane of the wave has a move that needs one.
__device__ __forceinline__ uint32_t ne_word(uint32_t own, uint32_t north, uint32_t east,
                                            uint32_t g, uint32_t colour, uint32_t t,
                                            const PhiloxKey& ks, uint64_t thr_up, uint64_t thr_down)
{
    const uint32_t n = own & 0x01010101u;
    const uint32_t allowed = north & east & 0x01010101u;
    const uint32_t up = allowed & ~n;
    const uint32_t down = allowed & n;
    const bool up_rand = thr_up < (1ull << 32);
    const bool down_rand = thr_down < (1ull << 32);
    const uint32_t need = (up_rand ? up : 0u) | (down_rand ? down : 0u);
    uint32_t f = (up_rand ? 0u : up) | (down_rand ? 0u : down);  // moves taken surely
    if (__builtin_amdgcn_ballot_w64(need != 0u) != 0ull) {
        const Words4 w = philox4x32_10(g, colour, t, 0u, ks);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const uint32_t bit = 1u << (8 * b);
            const uint64_t thr = (n & bit) ? thr_down : thr_up;
            if ((need & bit) && (uint64_t)w.w[b] < thr) f |= bit;
        }
    }
    return (own ^ f) | (f << 1);
}

__device__ __forceinline__ void ne_obs(uint32_t own, uint32_t nw, uint32_t north, uint32_t south,
                                       uint32_t east, uint32_t west, bool bond, Obs& o)
{
    o.acc += __builtin_popcount((own ^ nw) & 0x01010101u);
    o.mag += __builtin_popcount(nw & 0x01010101u);
    o.unfl += 4 - __builtin_popcount(nw & 0x02020202u);
    if (bond) {
        const uint32_t m = 0x01010101u;
        const uint32_t s = (north & m) + (south & m) + (east & m) + (west & m);  // <= 4 per byte
        const uint32_t sel = (nw & m) * 0xFFu;                                   // 0xFF where up
        o.bond += (int)__builtin_amdgcn_sad_u8(s & sel, 0u, 0u);
    }
}

// One word update for any kind, given the neighbour words.
template <int KIND, int DIM>
__device__ __forceinline__ uint32_t word_update(uint32_t own, const uint32_t (&nb)[2 * DIM], uint32_t p,
                                                uint32_t g, uint32_t colour, uint32_t t,
                                                const PhiloxKey& ks, const Luts& lut,
                                                uint64_t thr_up, uint64_t thr_down, bool count,
                                                bool bond, Obs& o)
{
    // nb[0] same row same column, nb[1] same row side word, nb[2] row above
    // (y-1), nb[3] row below (y+1), nb[4], nb[5] planes z-1, z+1
    if (KIND == KIND_ISING_HALF) {
        const Words4 w = philox4x32_10(g, colour, t, 0u, ks);
        const uint32_t nw = ising_half_word<DIM>(own, nb, w, reinterpret_cast<const uint8_t*>(lut.e));
        if (count) ising_half_obs<DIM>(own, nw, nb, bond, o);
        return nw;
    } else if (KIND == KIND_ISING_ONE) {
        const Words4 wa = philox4x32_10(2 * g, colour, t, 0u, ks);
        const Words4 wb = philox4x32_10(2 * g + 1, colour, t, 0u, ks);
        return ising_one_word<DIM>(own, nb, wa, wb, lut, bond, count, o);
    } else {
        // north = row y-1; east = site x+1: side word when p = 1, else same word
        const uint32_t east = p ? nb[1] : nb[0];
        const uint32_t west = p ? nb[0] : nb[1];
        const uint32_t nw = ne_word(own, nb[2], east, g, colour, t, ks, thr_up, thr_down);
        if (count) ne_obs(own, nw, nb[2], nb[3], east, west, bond, o);
        return nw;
    }
}

__device__ __forceinline__ uint32_t ld(const uint8_t* base, uint64_t off)
{
    return *reinterpret_cast<const uint32_t*>(base + off);
}
__device__ __forceinline__ void st(uint8_t* base, uint64_t off, uint32_t v)
{
    *reinterpret_cast<uint32_t*>(base + off) = v;
}

// One item (window, strip, plane) of a half-sweep, for this lane group.
template <int KIND, int DIM>
__device__ __forceinline__ void stream_half_item(const SweepArgs& a, const StreamGeom& sg, uint32_t item,
                                                 const Luts& lut, uint64_t thr_up, uint64_t thr_down, Obs& o)
{
    if (item < sg.nitems) {
        const uint32_t lane = threadIdx.x & 63u;
        const uint32_t li = lane % sg.W;
        const uint32_t gbase = lane - li;
        const uint32_t win = item % sg.nwin;
        const uint32_t strip = (item / sg.nwin) % sg.nstrips;
        const uint32_t zp = item / (sg.nwin * sg.nstrips);
        const uint32_t J = win * sg.win_cols;
        const uint32_t col = (J + li) % sg.ncols;
        const bool owned = sg.wrap || (J + li < sg.ncols);
        const uint32_t src_l = gbase + ((li + sg.W - 1) & (sg.W - 1));
        const uint32_t src_r = gbase + ((li + 1) & (sg.W - 1));
        // window edges: lane 0 needs column J-1, lane 63 column J+64
        uint32_t colE = col;
        if (!sg.wrap) {
            if (li == 0) colE = (J + sg.ncols - 1) % sg.ncols;
            if (li == 63) colE = (J + 64) % sg.ncols;
        }
        const uint32_t c = a.colour;
        const uint8_t* O = colour_array(a, c ^ 1u);
        uint8_t* A = colour_array(a, c);
        const uint32_t L = sg.L;
        const uint64_t plane = (uint64_t)zp * L;
        const uint64_t rowb = sg.Lh;  // bytes per colour row
        const uint32_t y0 = strip * sg.H;
        const uint32_t y1 = min(y0 + sg.H, L);
        const PhiloxKey ks = philox_schedule(a.key0, a.key1);
        const uint64_t planem = (uint64_t)wrap_row((int)zp - 1, L) * L;
        const uint64_t planep = (uint64_t)wrap_row((int)zp + 1, L) * L;

        uint32_t Om = ld(O, (plane + wrap_row((int)y0 - 1, L)) * rowb + 4 * col);
        uint32_t O0 = ld(O, (plane + y0) * rowb + 4 * col);
        for (uint32_t y = y0; y < y1; ++y) {
            const uint32_t yp = y + 1 == L ? 0 : y + 1;
            const uint32_t Op = ld(O, (plane + yp) * rowb + 4 * col);
            const uint64_t off = (plane + y) * rowb + 4 * col;
            const uint32_t own = ld(A, off);
            const uint32_t p = (y + zp + c) & 1u;
            uint32_t adj = __shfl(O0, p ? src_r : src_l, 64);
            if (!sg.wrap) {
                const uint32_t E = ld(O, (plane + y) * rowb + 4 * colE);
                if (p ? li == 63 : li == 0) adj = E;
            }
            uint32_t nb[2 * DIM];
            nb[0] = O0;
            nb[1] = side_word(O0, adj, p);
            nb[2] = Om;
            nb[3] = Op;
            if constexpr (DIM == 3) {
                nb[2 * DIM - 2] = ld(O, (planem + y) * rowb + 4 * col);
                nb[2 * DIM - 1] = ld(O, (planep + y) * rowb + 4 * col);
            }
            const uint32_t g = (uint32_t)((plane + y) * sg.ncols + col);
            const uint32_t nw = word_update<KIND, DIM>(own, nb, p, g, c, a.t, ks, lut, thr_up,
                                                       thr_down, owned, c == 1, o);
            if (owned) st(A, off, nw);
            Om = O0;
            O0 = Op;
        }
    }
}

}  // namespace streamk

}  // namespace spinlat
