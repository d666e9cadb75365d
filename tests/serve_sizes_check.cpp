// CPU check of the serving chunk layout (serve_sizes.hpp): for every tile
// shape in the list and every N from 3 to 4096, the bytes the (i, j) table
// kernel writes - computed by enumerating the blocks its launch fills -
// stay inside the table region of the request's chunk, for either tile
// type, and the parts of the chunk do not overlap.  Built and run by
// test_serve_sizes.py with the host compiler.
#include "serve_sizes.hpp"

#include <cstdio>
#include <cstdlib>

using namespace mb::serve;

int main() {
    // I blocks of the two tile types (waves x points per wave) that the tile
    // shapes allow, J blocks of 64
    const int64_t ib32[] = {16, 32, 48, 64, 96, 128, 192};
    const int64_t ib64[] = {16, 32, 48, 64, 96};
    long checked = 0;
    for (int64_t v : {2, 3})  // numbers per pair: (a, w), or (a, q, w)
    for (int64_t a : ib32)
        for (int64_t b : ib64) {
            const TableShape t32{a, 64, 4, v}, t64{b, 64, 8, v};
            for (int64_t n = 3; n <= 4096; ++n) {
                const ChunkLayout c = chunk_layout(n, t32, t64);
                // the launch's own grid (what the kernel indexes)
                for (const TableShape *t : {&t32, &t64}) {
                    const int64_t e = table_extent(n, *t);
                    if (e > c.tab_bytes) {
                        std::printf("FAIL n=%lld ib=%lld elem=%lld extent %lld > region %lld\n",
                                    (long long)n, (long long)t->ib, (long long)t->elem,
                                    (long long)e, (long long)c.tab_bytes);
                        return 1;
                    }
                }
                if (!(c.phi >= 24 * n && c.mag >= c.phi + 8 * n && c.tab >= c.mag + 8 * n &&
                      c.total >= c.tab + c.tab_bytes && c.tab % 256 == 0)) {
                    std::printf("FAIL n=%lld: overlapping chunk parts\n", (long long)n);
                    return 1;
                }
                ++checked;
            }
        }
    std::printf("OK %ld\n", checked);
    return 0;
}
