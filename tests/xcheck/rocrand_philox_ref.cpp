// Independent Philox4x32-10 reference for the oracle's pin: calls rocRAND's
// device-API generator (host-callable inline functions) and prints the block
// it returns for each requested (key, counter).
//
// Input (stdin), one request per line:  key0 key1 c0 c1 c2 c3  (decimal u32)
// Output (stdout), one line per request: r0 r1 r2 r3           (decimal u32)
//
// rocRAND is driven only through its public API: rocrand_init(seed,
// subsequence, offset) followed by rocrand4().  The request is mapped as
//   seed        = key1:key0
//   subsequence = c3:c2
//   offset      = 4 * (c1:c0)        (elements; 4 per block)
// and the test that uses this program checks that this mapping makes the
// two implementations agree.
#include <rocrand/rocrand_kernel.h>
#include <cstdio>
#include <cstdint>

int main()
{
    unsigned long long k0, k1, c0, c1, c2, c3;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        const unsigned long long seed = (k1 << 32) | k0;
        const unsigned long long subseq = (c3 << 32) | c2;
        const unsigned long long block = (c1 << 32) | c0;
        rocrand_state_philox4x32_10 st;
        // offset is in elements; 4 elements per counter block.  block < 2^64 / 4
        // is enforced by the caller.
        rocrand_init(seed, subseq, block * 4ull, &st);
        const uint4 r = rocrand4(&st);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
