// Independent Philox4x32-10 for pinning the oracle: rocRAND's host-callable
// engine (header only, no GPU needed).  Reads lines "c0 c1 c2 c3 k0 k1"
// (decimal) and prints the four output words of one block per line.
//
// rocrand_init(seed, subsequence, offset) sets key = (seed lo, seed hi),
// adds `subsequence` to counter words 2..3 and offset/4 to words 0..1, so
// the first rocrand4() returns the block for counter (c0, c1, c2, c3) when
// seed = k1:k0, subsequence = c3:c2 and offset = 4 * (c1:c0) (c1 < 2^30).
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main() {
    unsigned long long c[4], k[2];
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
        rocrand_state_philox4x32_10 st;
        const unsigned long long seed = (k[1] << 32) | k[0];
        const unsigned long long sub = (c[3] << 32) | c[2];
        const unsigned long long off = 4ull * ((c[1] << 32) | c[0]);
        rocrand_init(seed, sub, off, &st);
        const uint4 r = rocrand4(&st);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
