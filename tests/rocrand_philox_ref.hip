// Reference Philox4x32-10 words from rocRAND's header-only engine, evaluated on the host.
// Reads lines "c0 c1 c2 c3 k0 k1" (hex) on stdin and prints the four output words per line.
// rocrand_init(seed, subsequence, offset): key = seed, counter words 2,3 = subsequence,
// counter words 0,1 = offset / 4, first output = Philox(counter, key).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
        unsigned long long sub = ((unsigned long long)c3 << 32) | c2;
        unsigned long long off = 4ull * (((unsigned long long)c1 << 32) | c0);
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, sub, off, &st);
        uint4 r = rocrand4(&st);
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
