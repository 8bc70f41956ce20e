// Host-only probe: evaluates rocRAND's Philox4x32-10 engine (a library built
// from the same published algorithm) on counters read from stdin, so that
// the oracle's transcription can be checked against an independent one.
// Input lines: c0 c1 c2 c3 k0 k1 (decimal).  Output lines: four hex words.
// rocRAND's engine(seed, subsequence, offset) starts at the counter
// (offset/4 as 64 bits in c0:c1, subsequence as 64 bits in c2:c3) with
// key (seed low, seed high).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned long long c0, c1, c2, c3, k0, k1;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = (k1 << 32) | k0;
        unsigned long long sub = (c3 << 32) | c2;
        unsigned long long blk = (c1 << 32) | c0;
        rocrand_device::philox4x32_10_engine e(seed, sub, blk * 4);
        for (int i = 0; i < 4; i++) std::printf("%08x%c", e(), i == 3 ? '\n' : ' ');
    }
    return 0;
}
