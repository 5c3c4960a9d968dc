// Prints rocRAND's Philox4x32-10 block for each (counter, key) read from
// stdin, one "c0 c1 c2 c3 k0 k1" line (hex) per case.  Built as host code;
// rocRAND is an implementation independent of the oracle's.
#include <rocrand/rocrand_kernel.h>
#include <cstdio>

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        // rocRAND's state: key = (lo, hi) of the seed; subsequence adds to
        // counter words 2-3, offset/4 to counter words 0-1.
        unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
        unsigned long long sub = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        unsigned long long low = (unsigned long long)c0 | ((unsigned long long)c1 << 32);
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, sub, 0ULL, &st);
        // add the low 64 counter bits in five pieces, each small enough that
        // the offset argument (4 per counter step) does not overflow
        unsigned long long piece = low / 5ULL;
        for (int i = 0; i < 4; ++i) skipahead(4ULL * piece, &st);
        skipahead(4ULL * (low - 4ULL * piece), &st);
        uint4 r = rocrand4(&st);
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
