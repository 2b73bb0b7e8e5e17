// host_checks.cpp -- the library's pure host logic (host_logic.cpp) under
// AddressSanitizer and UndefinedBehaviorSanitizer: parameter validation over
// fixed and random inputs, the device-buffer layout, the threshold table's
// range and size, the overflow-safe sweep-count checks, and the first-fit
// arena allocator against a byte-map model over random alloc/release
// sequences.  Built and run by tests/test_host_sanitizers.py with g++ (no HIP).
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <random>
#include <vector>

#include "host_logic.h"

using namespace spinlat;
using namespace spinlat::host;

static int g_fail = 0;

#define CHECK(cond)                                                       \
    do {                                                                  \
        if (!(cond)) {                                                    \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__,   \
                         __LINE__, #cond);                                \
            ++g_fail;                                                     \
        }                                                                 \
    } while (0)

static sl_params base_params()
{
    sl_params p{};
    p.abi_version = SL_ABI_VERSION;
    p.model = SL_ISING;
    p.dim = 2;
    p.L = 64;
    p.two_s = 1;
    p.init = SL_INIT_RANDOM;
    p.J = 1.0;
    p.h = 0.0;
    p.T = 2.269;
    p.c = 0.1;
    p.seed = 1;
    p.t0 = 0;
    p.record_capacity = 16;
    p.init_spins = nullptr;
    p.ne_side = 32;
    p.ne_lambda = 16;
    return p;
}

static void check_validate_fixed()
{
    sl_params p = base_params();
    CHECK(validate(&p) == SL_OK);
    CHECK(validate(nullptr) == SL_E_INVALID);
    p.L = 63;
    CHECK(validate(&p) == SL_E_INVALID);
    p.L = 12;
    CHECK(validate(&p) == SL_E_UNSUPPORTED);
    p = base_params();
    p.T = std::nan("");
    CHECK(validate(&p) == SL_E_INVALID);
    p.T = std::numeric_limits<double>::infinity();
    CHECK(validate(&p) == SL_OK);
    p = base_params();
    p.t0 = 1ull << 32;
    CHECK(validate(&p) == SL_E_OVERFLOW);
    p = base_params();
    p.model = SL_NE_SUBLATTICE;
    p.t0 = 1ull << 31;
    CHECK(validate(&p) == SL_E_OVERFLOW);
    p = base_params();
    p.record_capacity = 0;
    CHECK(validate(&p) == SL_E_INVALID);
    p = base_params();
    p.init = SL_INIT_BUFFER;
    CHECK(validate(&p) == SL_E_INVALID);  // no init_spins
    p = base_params();
    p.dim = 3;
    p.L = 1 << 12;  // 2^36 sites: the 32-bit Philox group index overflows
    CHECK(validate(&p) == SL_E_UNSUPPORTED);
    CHECK(last_error()[0] != '\0');
}

// Random parameters: validate never misbehaves, and every accepted set has a
// consistent layout and a table in range.
static void check_validate_random()
{
    std::mt19937_64 rng(12345);
    const double specials[] = {0.0, -0.0, 1.0, -1.0, 0.5, 2.269, 1e-300, 1e300,
                               std::numeric_limits<double>::infinity(),
                               -std::numeric_limits<double>::infinity(), std::nan("")};
    int accepted = 0;
    for (int it = 0; it < 200000; ++it) {
        sl_params p = base_params();
        auto pick_int = [&](int lo, int hi) { return (int)(lo + (int64_t)(rng() % (uint64_t)(hi - lo + 1))); };
        auto pick_d = [&]() {
            return (rng() & 1) ? specials[rng() % (sizeof specials / sizeof specials[0])]
                               : std::ldexp((double)(int64_t)rng(), -60);
        };
        // each field keeps its valid base value or, one time in three, takes a
        // random one
        auto r3 = [&]() { return rng() % 3 == 0; };
        if (rng() % 8 == 0) p.abi_version = (uint32_t)rng();
        if (r3()) p.model = pick_int(-2, 6);
        if (r3()) p.dim = pick_int(0, 4);
        if (r3()) p.L = (rng() % 3 == 0) ? (int32_t)(uint32_t)rng() : pick_int(-4, 600);
        if (r3()) p.two_s = pick_int(0, 3);
        if (r3()) p.init = pick_int(-1, 3);
        if (r3()) p.J = pick_d();
        if (r3()) p.h = pick_d();
        if (r3()) p.T = pick_d();
        if (r3()) p.c = pick_d();
        p.seed = rng();
        if (r3()) p.t0 = (rng() % 2) ? rng() : rng() % 8;
        if (r3()) p.record_capacity = (rng() % 2) ? rng() : rng() % 64;
        if (r3()) p.ne_side = pick_int(-2, 130);
        if (r3()) p.ne_lambda = pick_int(-2, 260);
        if (p.init == SL_INIT_BUFFER && (rng() & 1)) p.init_spins = reinterpret_cast<const int8_t*>(&p);
        const sl_status st = validate(&p);
        CHECK(st == SL_OK || st == SL_E_INVALID || st == SL_E_UNSUPPORTED || st == SL_E_OVERFLOW);
        if (st != SL_OK) continue;
        ++accepted;
        CHECK(p.L >= 8 && p.L % 8 == 0);
        CHECK(p.t0 < (1ull << 32));
        CHECK(p.record_capacity >= 1 && p.record_capacity <= (1ull << 32));
        if (p.L > 512) continue;  // keep the layout arithmetic of the check itself small
        const Layout l = layout_of(&p);
        const uint64_t N = p.dim == 2 ? (uint64_t)p.L * p.L : (uint64_t)p.L * p.L * p.L;
        CHECK(l.nsites == N && l.nh * 2 == N);
        CHECK(l.col_bytes >= l.nh && l.col_bytes % kAlign == 0);
        CHECK(l.off_col[1][1] + l.col_bytes <= l.off_acc);
        CHECK(l.off_acc % kAlign == 0 && l.off_out % kAlign == 0 && l.off_lut % kAlign == 0);
        CHECK(l.off_out - l.off_acc >= p.record_capacity * kSlotWords * sizeof(int64_t));
        CHECK(l.off_lut - l.off_out >= p.record_capacity * kRecordWords * sizeof(int64_t));
        CHECK(l.total >= l.off_lut + kMaxLut * sizeof(uint64_t));
        uint64_t tab[kMaxLut + 8];
        const size_t n = build_table(&p, tab);
        if (p.model == SL_ISING || p.model == SL_NE_COUPLED) CHECK(n == (size_t)(4 * (4 * p.dim + 1)));
        else CHECK(n == 2);
        CHECK(n <= (size_t)kMaxLut);
        for (size_t i = 0; i < n; ++i) CHECK(tab[i] <= (1ull << 32));
    }
    CHECK(accepted > 1000);
}

static void check_sweep_counts()
{
    const uint64_t M = std::numeric_limits<uint64_t>::max();
    const uint64_t T32 = 1ull << 32;
    CHECK(check_sweep_count(0, 16, 0, T32, 0) == SL_OK);
    CHECK(check_sweep_count(1, 16, 0, T32, 15) == SL_OK);
    CHECK(check_sweep_count(1, 16, 0, T32, 16) == SL_E_STATE);
    CHECK(check_sweep_count(16, 16, 0, T32, 1) == SL_E_STATE);
    CHECK(check_sweep_count(1, 16, 0, T32, M) == SL_E_STATE);      // n = 2^64 - 1 (sweep(-1))
    CHECK(check_sweep_count(1, M, 0, T32, M - 1) == SL_E_OVERFLOW);  // no wrap of pending + n
    CHECK(check_sweep_count(0, M, T32 - 1, T32, 1) == SL_OK);
    CHECK(check_sweep_count(0, M, T32 - 1, T32, 2) == SL_E_OVERFLOW);
    CHECK(check_sweep_count(0, M, T32 - 8, T32, M - 2) == SL_E_OVERFLOW);  // next_t + n would wrap
    CHECK(check_sweep_count(0, 1ull << 32, 0, 1ull << 31, 1ull << 31) == SL_OK);
    CHECK(check_sweep_count(0, 1ull << 32, 1, 1ull << 31, 1ull << 31) == SL_E_OVERFLOW);
}

// First-fit allocator against a byte-map model (one entry per kAlign unit).
static void check_free_list()
{
    std::mt19937_64 rng(777);
    for (int round = 0; round < 20; ++round) {
        const size_t units = 64 + rng() % 512;
        const size_t start = kAlign * (rng() % 16);
        FreeList fl;
        fl.reset(start, units * kAlign);
        std::vector<int> owner(units, -1);
        struct Block { size_t off, bytes; };
        std::vector<Block> live;
        for (int op = 0; op < 3000; ++op) {
            if (live.empty() || rng() % 3 != 0) {
                const size_t want = kAlign * (1 + rng() % 24);
                size_t off = 0;
                // model: lowest offset with `want` free bytes in a free run
                size_t model_off = (size_t)-1, run = 0;
                for (size_t u = 0; u < units; ++u) {
                    run = owner[u] < 0 ? run + 1 : 0;
                    if (run * kAlign >= want) {
                        // first-fit is by free range, not by run: the range
                        // containing this run starts at its first free unit
                        size_t s = u + 1 - run;
                        while (s > 0 && owner[s - 1] < 0) --s;
                        model_off = start + s * kAlign;
                        break;
                    }
                }
                const bool ok = fl.alloc(want, &off);
                CHECK(ok == (model_off != (size_t)-1));
                if (!ok) continue;
                CHECK(off == model_off);
                CHECK(off >= start && off + want <= start + units * kAlign && off % kAlign == 0);
                for (size_t u = (off - start) / kAlign; u < (off - start + want) / kAlign; ++u) {
                    CHECK(owner[u] < 0);
                    owner[u] = 1;
                }
                live.push_back({off, want});
            } else {
                const size_t k = rng() % live.size();
                const Block b = live[k];
                fl.release(b.off, b.bytes);
                for (size_t u = (b.off - start) / kAlign; u < (b.off - start + b.bytes) / kAlign; ++u)
                    owner[u] = -1;
                live[k] = live.back();
                live.pop_back();
            }
            // free ranges are coalesced: no two touch
            size_t prev_end = (size_t)-1;
            size_t free_units = 0;
            for (const auto& kv : fl.map()) {
                CHECK(kv.first != prev_end);
                prev_end = kv.first + kv.second;
                free_units += kv.second / kAlign;
            }
            size_t model_free = 0;
            for (size_t u = 0; u < units; ++u) model_free += owner[u] < 0;
            CHECK(free_units == model_free);
        }
        for (const Block& b : live) fl.release(b.off, b.bytes);
        CHECK(fl.ranges() == 1 && fl.free_bytes() == units * kAlign);
        CHECK(fl.map().begin()->first == start);
    }
}

int main()
{
    check_validate_fixed();
    check_validate_random();
    check_sweep_counts();
    check_free_list();
    if (g_fail) {
        std::fprintf(stderr, "host_checks: %d failures\n", g_fail);
        return 1;
    }
    std::printf("host_checks: ok\n");
    return 0;
}
