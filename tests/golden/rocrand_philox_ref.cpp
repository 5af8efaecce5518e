// Independent reference for the oracle's Philox4x32-10: rocRAND's host-callable
// philox4x32_10 engine.  Reads "c0 c1 c2 c3 k0 k1" per line from stdin and
// prints the 4 output words of one Philox block for counter (c0,c1,c2,c3) and
// key (k0,k1).  rocRAND maps seed -> key, subsequence -> counter words 2..3
// and offset/4 -> counter words 0..1, so c1 must stay below 2^30.
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        rocrand_state_philox4x32_10 st;
        unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
        unsigned long long subseq = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        unsigned long long offset = 4ull * ((unsigned long long)c0 | ((unsigned long long)c1 << 32));
        rocrand_init(seed, subseq, offset, &st);
        uint4 r = rocrand4(&st);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
