// Host-only check of the pipeline's copy pool: every byte of every copy
// arrives, for part counts 1-8 and sizes around the splits where a share
// is a multiple of 64 bytes with a remainder left over.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "copy_pool.h"

int main() {
    std::vector<size_t> sizes = {0, 1, 63, 64, 1000, (size_t)1 << 20, ((size_t)1 << 20) + 1,
                                 ((size_t)1 << 20) + 63, ((size_t)1 << 20) + 64,
                                 ((size_t)32 << 20) - 1, (size_t)32 << 20};
    // share a multiple of 64 with a remainder: parts * 64 * k + r, 0 < r < parts
    for (size_t parts = 2; parts <= 8; parts++)
        for (size_t r = 1; r < parts; r++) sizes.push_back(parts * 64 * 4100 + r);
    unsigned seed = 12345;
    for (int i = 0; i < 40; i++) {
        seed = seed * 1103515245u + 12345u;
        sizes.push_back(((size_t)1 << 20) + (seed >> 8) % ((size_t)7 << 20));
    }
    size_t maxb = 0;
    for (size_t b : sizes) maxb = b > maxb ? b : maxb;
    std::vector<unsigned char> src(maxb + 64), dst(maxb + 64);
    for (size_t i = 0; i < src.size(); i++) src[i] = (unsigned char)(i * 131 + 7);
    int bad = 0;
    for (unsigned workers = 0; workers <= 7; workers++) {
        wfa::CopyPool pool(workers);
        for (int round = 0; round < 2; round++) {
            for (size_t b : sizes) {
                const size_t off = (size_t)(round * 3 + workers) % 17;  // unaligned starts too
                if (off + b > src.size()) continue;
                std::memset(dst.data(), 0xEE, dst.size());
                pool.copy(dst.data() + off, src.data() + off, b);
                if (std::memcmp(dst.data() + off, src.data() + off, b) != 0) {
                    size_t k = 0;
                    while (dst[off + k] == src[off + k]) k++;
                    std::printf("workers %u size %zu: first wrong byte %zu\n", workers, b, k);
                    bad++;
                }
                for (size_t k = off + b; k < dst.size(); k++)
                    if (dst[k] != 0xEE) {
                        std::printf("workers %u size %zu: wrote past the end at %zu\n", workers, b, k);
                        bad++;
                        break;
                    }
            }
        }
    }
    std::printf(bad ? "copy pool: %d failures\n" : "copy pool ok\n", bad);
    return bad ? 1 : 0;
}
