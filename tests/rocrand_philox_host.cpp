// Host-side driver of rocRAND's Philox4x32-10 engine, used only as an
// independent cross-check of the CPU oracle's Philox implementation.
// Reads lines "seed subsequence offset" from stdin and prints the four 32-bit
// words that rocrand4() returns for a state initialised with rocrand_init().
#include <cstdio>
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>

int main()
{
    unsigned long long seed, subsequence, offset;
    while (std::scanf("%llu %llu %llu", &seed, &subsequence, &offset) == 3) {
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, subsequence, offset, &st);
        uint4 w = rocrand4(&st);
        std::printf("%u %u %u %u\n", w.x, w.y, w.z, w.w);
    }
    return 0;
}
