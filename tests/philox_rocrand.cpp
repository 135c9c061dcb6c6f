// Reference outputs of Philox4x32-10 from an implementation that is not this
// project's: the rocRAND engine (rocrand_philox4x32_10.h, a source header of
// the ROCm image).  Test infrastructure only: the Philox pin compiles this with
// the host compiler and compares its words with the CPU oracle's generator.
//
// stdin: lines "seed block table_id" (decimal).  stdout: the four output
// words of the counter (block lo, block hi, table_id, 0) under key seed, in
// hex, one line per input line.
//
// The engine is driven only through its public interface:
//   key     = (seed low word, seed high word)         -- engine(seed, ...)
//   counter = (0, 0, subsequence lo, subsequence hi)  -- subsequence = table_id
//             + offset / 4 added to words (x, y)      -- offset = 4 * block
// so its first four draws are the block of the counter (block lo, block hi,
// table_id, 0), word x first.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main() {
    unsigned long long seed, block;
    unsigned int tid;
    while (std::scanf("%llu %llu %u", &seed, &block, &tid) == 3) {
        rocrand_device::philox4x32_10_engine e(seed, tid, 4ull * block);
        const unsigned int w0 = e.next(), w1 = e.next(), w2 = e.next(), w3 = e.next();
        std::printf("%08x %08x %08x %08x\n", w0, w1, w2, w3);
    }
    return 0;
}
