// Host-side reference for Philox4x32-10 taken from rocRAND's header-only
// engine (a library routine, independent of the oracle).  Reads lines
// "key ctr0 ctr1 ctr2 ctr3" (hex) on stdin and prints the four output words.
// The engine's counter starts at (offset / 4) in its low 64 bits and the
// subsequence number in its high 64 bits; the first four words it returns
// are the Philox block of that counter.
#include <cstdio>
#include <cstdint>
#include <rocrand/rocrand_philox4x32_10.h>

int main()
{
    unsigned long long key;
    unsigned int c0, c1, c2, c3;
    while (std::scanf("%llx %x %x %x %x", &key, &c0, &c1, &c2, &c3) == 5) {
        const unsigned long long low = (static_cast<unsigned long long>(c1) << 32) | c0;
        const unsigned long long high = (static_cast<unsigned long long>(c3) << 32) | c2;
        rocrand_device::philox4x32_10_engine eng(key, high, low * 4ull);
        unsigned int w0 = eng(), w1 = eng(), w2 = eng(), w3 = eng();
        std::printf("%08x %08x %08x %08x\n", w0, w1, w2, w3);
    }
    return 0;
}
