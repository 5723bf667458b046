// A third-party reference for the oracle's Philox4x32-10 (Salmon et al., SC'11):
// rocRAND's engine (header-only source from the ROCm installation), run on the
// host.  Reads lines "seed c0 c1 c2 c3" (c1 < 2^30) and prints the four words of
// Philox4x32-10 with key (seed & 0xffffffff, seed >> 32) and counter
// (c0, c1, c2, c3).  rocRAND's engine starts its counter at (offset / 4) in the
// low 64 bits and the subsequence in the high 64 bits, so the counter is
// reached with subsequence = c2 + 2^32 c3 and offset = 4 (c0 + 2^32 c1).
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main()
{
    unsigned long long seed;
    unsigned int c0, c1, c2, c3;
    while (std::scanf("%llu %u %u %u %u", &seed, &c0, &c1, &c2, &c3) == 5) {
        if (c1 >= (1u << 30)) return 2;
        const unsigned long long sub = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        const unsigned long long off = 4ull * ((unsigned long long)c0 | ((unsigned long long)c1 << 32));
        rocrand_device::philox4x32_10_engine e(seed, sub, off);
        const unsigned int x0 = e(), x1 = e(), x2 = e(), x3 = e();
        std::printf("%u %u %u %u\n", x0, x1, x2, x3);
    }
    return 0;
}
