// Independent reference for the oracle's Philox4x32-10: rocRAND's engine,
// compiled for the host.  Reads lines "seed c0 c1 c2 c3" and prints the four
// output words of the counter (c0, c1, c2, c3) under key (seed lo, seed hi).
// rocRAND places the subsequence in counter words 2-3 and offset/4 in words
// 0-1, which is how the counter is set here (c1 < 2^30 keeps offset in range).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
    unsigned long long seed, c0, c1, c2, c3;
    while (std::scanf("%llu %llu %llu %llu %llu", &seed, &c0, &c1, &c2, &c3) == 5) {
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, c2 | (c3 << 32), 4ull * (c0 | (c1 << 32)), &st);
        unsigned a = rocrand(&st), b = rocrand(&st), c = rocrand(&st), d = rocrand(&st);
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
