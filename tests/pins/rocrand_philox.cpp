// Independent Philox4x32-10 reference for the oracle's pin test: rocRAND's
// host-callable engine, compiled from the installed header.  Reads lines
// "k0 k1 c0 c1 c2 c3" (decimal) and prints the four output words.
// rocRAND's engine keeps a 128-bit counter whose low 64 bits advance with
// discard(4*m) and whose high 64 bits are the subsequence number.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned long long k0, k1, c0, c1, c2, c3;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        unsigned long long seed = k0 | (k1 << 32);
        unsigned long long sub = c2 | (c3 << 32);
        rocrand_device::philox4x32_10_engine e(seed, sub, 0ull);
        unsigned long long low = c0 | (c1 << 32);
        const unsigned long long chunk = 1ull << 60;
        while (low > 0) {
            unsigned long long m = low < chunk ? low : chunk;
            e.discard(4ull * m);
            low -= m;
        }
        unsigned a = e.next(), b = e.next(), c = e.next(), d = e.next();
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
