// Prints rocRAND's Philox4x32-10 output for counters/keys read from stdin.
// Input lines: c0 c1 c2 c3 k0 k1 (decimal).  The engine is seeded with
// seed = k0 | k1<<32, subsequence = c2 | c3<<32, offset = 4*(c0 | c1<<32), so
// its first four outputs are the block for counter (c0,c1,c2,c3) under key (k0,k1).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
    unsigned long long c0, c1, c2, c3, k0, k1;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        rocrand_device::philox4x32_10_engine e(k0 | (k1 << 32), c2 | (c3 << 32),
                                               4ull * (c0 | (c1 << 32)));
        unsigned a = e(), b = e(), c = e(), d = e();
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
