// Third-party reference for the Philox4x32-10 pin: rocRAND's open-source
// engine (header only, run on the host).  Reads lines "seed x y z w" and
// prints the four output words of Philox4x32-10 at counter (x, y, z, w).
// rocRAND places the subsequence in counter words z, w and offset/4 in x, y.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main()
{
    unsigned long long seed;
    unsigned int x, y, z, w;
    while (std::scanf("%llu %u %u %u %u", &seed, &x, &y, &z, &w) == 5) {
        unsigned long long subsequence = ((unsigned long long)w << 32) | z;
        unsigned long long offset = 4ull * (((unsigned long long)y << 32) | x);
        rocrand_device::philox4x32_10_engine eng(seed, subsequence, offset);
        unsigned int o0 = eng(), o1 = eng(), o2 = eng(), o3 = eng();
        std::printf("%u %u %u %u\n", o0, o1, o2, o3);
    }
    return 0;
}
