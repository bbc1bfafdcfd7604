// Test helper: Philox4x32-10 words from rocRAND's header-only engine, run on
// the host.  Reads (key0 key1 c0 c1 c2 c3) lines on stdin (c1 < 2^30), writes
// the four output words of each counter.  rocRAND's engine is seeded with the
// 64-bit key, its subsequence selects counter words 2-3 and its offset (in
// 32-bit outputs) selects words 0-1.
#include <rocrand/rocrand_kernel.h>

#include <cstdio>

int main() {
    unsigned k0, k1, c0, c1, c2, c3;
    while (std::scanf("%u %u %u %u %u %u", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        rocrand_state_philox4x32_10 st;
        const unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
        const unsigned long long sub = ((unsigned long long)c3 << 32) | c2;
        const unsigned long long off = 4ull * (((unsigned long long)c1 << 32) | c0);
        rocrand_init(seed, sub, off, &st);
        uint4 r = rocrand4(&st);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
