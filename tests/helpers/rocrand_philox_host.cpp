// Host-side driver that exposes the ROCm random-number library's Philox4x32-10
// bijection (ten rounds of a counter under a key) so that the CPU oracle's
// Philox can be checked against an independent library implementation.
// Reads lines "c0 c1 c2 c3 k0 k1" (decimal) on stdin and prints the four output
// words, one line per counter.  Host code only; no GPU is touched.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

struct philox_probe : rocrand_device::philox4x32_10_engine {
    uint4 bijection(uint4 ctr, uint2 key) { return this->ten_rounds(ctr, key); }
};

int main() {
    unsigned long long c0, c1, c2, c3, k0, k1;
    philox_probe p;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 ctr = {(unsigned)c0, (unsigned)c1, (unsigned)c2, (unsigned)c3};
        uint2 key = {(unsigned)k0, (unsigned)k1};
        uint4 r = p.bijection(ctr, key);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
