// Host-only reference words from rocRAND's Philox4x32-10 engine, used to pin
// the oracle's own Philox implementation.  Reads lines "c0 c1 c2 c3 k0 k1"
// (hex) on stdin and prints the four output words of each counter/key.
// The engine's (seed, subsequence, offset) arguments are chosen so that its
// internal counter equals {c0, c1, c2, c3} and its key equals {k0, k1}:
// the offset advances the low 64 counter bits by offset/4 (in units of 32-bit
// outputs), the subsequence sets the high 64 bits.
#include <cstdio>
#include <rocrand/rocrand_kernel.h>

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
        unsigned long long sub = ((unsigned long long)c3 << 32) | c2;
        unsigned long long low = ((unsigned long long)c1 << 32) | c0;
        rocrand_state_philox4x32_10 st;
        // offset counts 32-bit outputs: 4 per counter value
        rocrand_init(seed, sub, 0, &st);
        // advance by 4*low outputs in four calls of `low` each, so that no
        // offset overflows 64 bits (the sub-counter carries add up exactly)
        for (int r = 0; r < 4; ++r) skipahead(low, &st);
        uint4 w = rocrand4(&st);
        std::printf("%08x %08x %08x %08x\n", w.x, w.y, w.z, w.w);
    }
    return 0;
}
