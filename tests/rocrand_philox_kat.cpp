// Host-only driver that runs rocRAND's philox4x32_10 engine on a given
// (counter, key) and prints the four output words.  Used by the Philox pin
// of the oracle: it is an independent, installed implementation, run as is.
#include <cstdio>
#include <cstdint>
#include <rocrand/rocrand_philox4x32_10.h>

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        const unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
        const unsigned long long sub = ((unsigned long long)c3 << 32) | c2;
        const unsigned long long X = ((unsigned long long)c1 << 32) | c0;
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, sub, 0, &st);
        // advance counter words 0..1 by X (four outputs per counter value)
        const unsigned long long Y = X / 4, r = X % 4;
        for (int i = 0; i < 4; ++i) skipahead(4ull * Y, &st);
        skipahead(4ull * r, &st);
        unsigned o[4];
        for (int i = 0; i < 4; ++i) o[i] = rocrand(&st);
        std::printf("%08x %08x %08x %08x\n", o[0], o[1], o[2], o[3]);
    }
    return 0;
}
