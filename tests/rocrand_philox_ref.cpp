// Host-only probe of rocRAND's Philox4x32-10 engine, used by the CPU test
// suite to pin the oracle's Philox against an independent implementation.
// It only calls rocRAND's public device/host API (rocrand_init, skipahead,
// skipahead_subsequence, rocrand); no HIP runtime call is made.
//
// stdin : lines "ctr0 ctr1 ctr2 ctr3 key0 key1" (decimal u32)
// stdout: lines "w0 w1 w2 w3" = Philox4x32-10(ctr, key)
//
// rocRAND's state for (seed, subsequence, offset) holds key = (seed lo, seed
// hi) and counter = (offset/4 as a 64-bit number in words 0-1) +
// (subsequence in words 2-3); the four words of one counter are returned in
// order by successive rocrand() calls.
#include <cstdio>
#include <rocrand/rocrand_kernel.h>

int main() {
    unsigned long long c0, c1, c2, c3, k0, k1;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        rocrand_state_philox4x32_10 st;
        const unsigned long long seed = k0 | (k1 << 32);
        rocrand_init(seed, 0ull, 0ull, &st);
        skipahead_subsequence(c2 | (c3 << 32), &st);
        skipahead(4ull * c0, &st);
        // counter word 1 = c1: advance by c1 * 2^32 counters in four steps of
        // c1 * 2^30 counters (offset c1 * 2^32 numbers each), so that no
        // 64-bit offset overflows.
        for (int i = 0; i < 4; ++i) skipahead(c1 << 32, &st);
        unsigned int w[4];
        for (int i = 0; i < 4; ++i) w[i] = rocrand(&st);
        std::printf("%u %u %u %u\n", w[0], w[1], w[2], w[3]);
    }
    return 0;
}
