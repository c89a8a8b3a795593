// Philox-4x32-10 blocks from third-party library implementations, used only
// as an independent reference for the oracle's Philox in the CPU tests.
// Build with -DUSE_ATEN (g++, PyTorch's ATen header) or -DUSE_ROCRAND
// (hipcc host compile, rocRAND's header).  Reads lines "k0 k1 c0 c1 c2 c3"
// (decimal u32) on stdin and prints the four output words of each block.
#include <cstdio>
#include <cstdint>
#if defined(USE_ATEN)
#include <ATen/core/PhiloxRNGEngine.h>
#elif defined(USE_ROCRAND)
#include <rocrand/rocrand_kernel.h>
#else
#error "define USE_ATEN or USE_ROCRAND"
#endif

int main() {
    unsigned k0, k1, c0, c1, c2, c3;
    while (std::scanf("%u %u %u %u %u %u", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        uint64_t seed = (uint64_t)k0 | ((uint64_t)k1 << 32);
        uint64_t sub = (uint64_t)c2 | ((uint64_t)c3 << 32);
        uint64_t blk = (uint64_t)c0 | ((uint64_t)c1 << 32);
        uint32_t w[4];
#if defined(USE_ATEN)
        // ATen: counter = (offset lo, offset hi, subsequence lo, subsequence hi)
        at::philox_engine e(seed, sub, blk);
        for (int i = 0; i < 4; ++i) w[i] = e();
#else
        // rocRAND: subsequence adds to counter words 2-3, offset counts 32-bit
        // outputs (4 per block) into words 0-1
        rocrand_state_philox4x32_10 s;
        rocrand_init(seed, sub, blk * 4ull, &s);
        for (int i = 0; i < 4; ++i) w[i] = rocrand(&s);
#endif
        std::printf("%u %u %u %u\n", w[0], w[1], w[2], w[3]);
    }
    return 0;
}
