// Device-memory layout of one serving request (host arithmetic only, so a
// CPU test can check it for any tile shape).
//
// A request's chunk holds, in order: its points (24 N bytes), Phi (8 N), the
// near-field magnitudes of the binary32 refinement (8 N) and the (i, j)
// pair-term table of the exhaustive sum; each part starts on a 256-byte
// boundary.  The table's tile type is known only after validation, so the
// table region is sized for the larger of the binary32 and binary64 tables.
#pragma once

#include <algorithm>
#include <cstdint>

namespace mb {
namespace serve {

inline int64_t align256(int64_t b) { return (b + 255) & ~(int64_t)255; }

// Shape of the exhaustive sum's (i, j) table: I blocks of `ib` points, J
// blocks of `jb`, `elem` bytes per number, `vals` numbers per pair.
struct TableShape {
    int64_t ib, jb, elem, vals;
};

// I blocks that J block b needs: those holding an i < 64 b + 63, the last j
// of the block (the same rule as the unit enumeration).
inline int64_t table_blocks_a(int64_t b, int64_t ib, int64_t jb, int64_t na) {
    return std::min(na, (jb * b + jb - 2) / ib + 1);
}

// Bytes the table kernel writes for N points, from its launch: block (a, b)
// with a < table_blocks_a(b) fills [(b na + a) S, (b na + a + 1) S) with
// S = ib jb vals elem bytes.  The largest end over all blocks it writes.
inline int64_t table_extent(int64_t n, const TableShape &t) {
    const int64_t na = (n + t.ib - 1) / t.ib, nb = (n + t.jb - 1) / t.jb;
    const int64_t blk = t.ib * t.jb * t.vals * t.elem;
    int64_t end = 0;
    for (int64_t b = 0; b < nb; ++b) {
        const int64_t ka = table_blocks_a(b, t.ib, t.jb, na);
        if (ka > 0) end = std::max(end, (b * na + ka) * blk);
    }
    return end;
}

// Bytes reserved for the table: the whole na x nb block grid.
inline int64_t table_region(int64_t n, const TableShape &t) {
    const int64_t na = (n + t.ib - 1) / t.ib, nb = (n + t.jb - 1) / t.jb;
    return na * nb * t.ib * t.jb * t.vals * t.elem;
}

// Offsets of the parts of a chunk and its total size; the table region
// takes the larger of the two tile types' tables.
struct ChunkLayout {
    int64_t phi, mag, tab, tab_bytes, total;
};

inline ChunkLayout chunk_layout(int64_t n, const TableShape &t32, const TableShape &t64) {
    ChunkLayout c;
    c.phi = align256(24 * n);
    c.mag = c.phi + align256(8 * n);
    c.tab = c.mag + align256(8 * n);
    c.tab_bytes = align256(std::max(table_region(n, t32), table_region(n, t64)));
    c.total = c.tab + c.tab_bytes;
    return c;
}

}  // namespace serve
}  // namespace mb
