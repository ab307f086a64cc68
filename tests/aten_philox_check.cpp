// Reads "key0 key1 ctr0 ctr1 ctr2 ctr3" lines and prints the four 32-bit
// outputs of PyTorch's own Philox4x32-10 engine (ATen, header-only) for that
// key and counter: an implementation independent of the oracle's.
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
int main() {
    unsigned long long k0, k1, c0, c1, c2, c3;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        uint64_t seed = (uint64_t)k0 | ((uint64_t)k1 << 32);
        uint64_t subseq = (uint64_t)c2 | ((uint64_t)c3 << 32);
        uint64_t offset = (uint64_t)c0 | ((uint64_t)c1 << 32);
        at::philox_engine e(seed, subseq, offset);
        uint32_t a = e(), b = e(), c = e(), d = e();
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
