// Host-side construction of the q-derivative tiles (plain C++, no device
// code): a partition of the points into tiles of at most `tile` points, the
// sorted union of each tile's neighbours, and every CSR entry's neighbour as
// a position in its point's tile list.  The LDS-tiled q-derivative kernels
// stage a tile's list once and read every neighbour from LDS through these
// positions; a point's neighbours are still visited in CSR order, so the
// partition changes which data are staged, never the arithmetic.
//
// Two partitions are formed and the one that stages fewer points is kept:
//  * runs of `tile` consecutive points;
//  * for components stored row by row (a structured grid's natural order,
//    detected from the connectivity), blocks of tj points by tk rows, whose
//    neighbour union is much smaller than a run's: for a 5 x 5 stencil a run
//    of 64 points along a row stages (64 + 4) x 5 points, a 16 x 4 block
//    (16 + 4) x (4 + 4).
#pragma once

#include <algorithm>
#include <cstdint>
#include <map>
#include <vector>

namespace lskum {

struct TileSet {
    int64_t ntile = 0;
    int32_t hmax = 0;            // longest tile list
    int64_t staged = 0;          // sum of the tile list lengths
    std::vector<int32_t> pts;    // ntile * tile: the tile's points, -1 past its end
    std::vector<int32_t> off;    // ntile + 1: tile list offsets
    std::vector<int32_t> list;   // the tile lists (sorted point indices)
    std::vector<uint16_t> lnbr;  // nnz: entry e's neighbour as a position in its tile list
};

// Row length W of the points [c0, c1) when they are stored row by row: for
// each point the smallest forward index jump beyond two (the first point of
// the stencil's part in the next row, p + W - 2 for a 5 x 5 stencil, and the
// same for the first points of a row through the periodic seam), its most
// frequent value (the smallest on a tie), plus two.  0 when no point has such
// a jump.  Only the tiles' shape depends on it: any value gives a valid
// partition.
inline int64_t tile_row_length(const int32_t* off, const int32_t* idx, int64_t c0, int64_t c1) {
    std::map<int64_t, int64_t> count;
    for (int64_t p = c0; p < c1; ++p) {
        int64_t m = -1;
        for (int32_t e = off[p]; e < off[p + 1]; ++e) {
            const int64_t d = (int64_t)idx[e] - p;
            if (d > 2 && (m < 0 || d < m)) m = d;
        }
        if (m > 0) ++count[m];
    }
    int64_t best = -1, best_count = 0;
    for (const auto& kv : count)
        if (kv.second > best_count) {
            best = kv.first;
            best_count = kv.second;
        }
    return best > 0 ? best + 2 : 0;
}

// Tile points, -1 padded to `tile` per tile.  blocked = false: runs of `tile`
// consecutive points over the whole cloud.  blocked = true: per component
// [comp_off[k], comp_off[k+1]), blocks of tj points by tk rows of the
// component's row length (tj x tk <= tile), in row-band order; a component
// without a row length of at least tj points gets runs instead.
inline std::vector<int32_t> tile_points(int64_t n, const int32_t* off, const int32_t* idx,
                                        const std::vector<int64_t>& comp_off, int tile, int tj,
                                        int tk, bool blocked) {
    std::vector<int32_t> pts;
    auto runs = [&](int64_t a, int64_t b) {
        for (int64_t p0 = a; p0 < b; p0 += tile) {
            for (int64_t s = 0; s < tile; ++s) pts.push_back(p0 + s < b ? (int32_t)(p0 + s) : -1);
        }
    };
    if (!blocked) {
        runs(0, n);
        return pts;
    }
    for (size_t k = 0; k + 1 < comp_off.size(); ++k) {
        const int64_t c0 = comp_off[k], c1 = comp_off[k + 1], m = c1 - c0;
        const int64_t W = tile_row_length(off, idx, c0, c1);
        if (W < tj || W > m) {
            runs(c0, c1);
            continue;
        }
        const int64_t rows = (m + W - 1) / W;
        for (int64_t r0 = 0; r0 < rows; r0 += tk)
            for (int64_t j0 = 0; j0 < W; j0 += tj) {
                const size_t start = pts.size();
                for (int64_t r = r0; r < std::min(rows, r0 + tk); ++r)
                    for (int64_t j = j0; j < std::min(W, j0 + tj); ++j) {
                        const int64_t p = c0 + r * W + j;
                        if (p < c1) pts.push_back((int32_t)p);
                    }
                if (pts.size() == start) continue;
                pts.resize(start + tile, -1);
            }
    }
    return pts;
}

// Lists and positions of the partition `pts` (tile entries per tile, -1
// padded).  Returns false (and leaves ts empty) when the partition does not
// hold every point exactly once, some list is longer than max_list, or a
// position fails to name its entry's neighbour.
inline bool tile_lists(int64_t n, const int32_t* off, const int32_t* idx, std::vector<int32_t> pts,
                       int tile, int max_list, TileSet& ts) {
    ts = TileSet{};
    if (pts.size() % tile != 0) return false;
    const int64_t nt = (int64_t)(pts.size() / tile);
    std::vector<uint8_t> seen(n, 0);
    for (int32_t p : pts) {
        if (p < 0) continue;
        if (p >= n || seen[p]) return false;
        seen[p] = 1;
    }
    for (int64_t p = 0; p < n; ++p)
        if (!seen[p]) return false;
    const int64_t nnz = off[n];
    std::vector<int32_t> stamp(n, -1), pos(n, 0), list;
    ts.off.reserve(nt + 1);
    ts.off.push_back(0);
    ts.lnbr.assign(nnz, 0);
    for (int64_t b = 0; b < nt; ++b) {
        list.clear();
        for (int s = 0; s < tile; ++s) {
            const int32_t p = pts[b * tile + s];
            if (p < 0) continue;
            for (int32_t e = off[p]; e < off[p + 1]; ++e) {
                const int32_t i = idx[e];
                if (stamp[i] != (int32_t)b) {
                    stamp[i] = (int32_t)b;
                    list.push_back(i);
                }
            }
        }
        if ((int64_t)list.size() > max_list) {
            ts = TileSet{};
            return false;
        }
        std::sort(list.begin(), list.end());
        for (size_t k = 0; k < list.size(); ++k) pos[list[k]] = (int32_t)k;
        for (int s = 0; s < tile; ++s) {
            const int32_t p = pts[b * tile + s];
            if (p < 0) continue;
            for (int32_t e = off[p]; e < off[p + 1]; ++e) ts.lnbr[e] = (uint16_t)pos[idx[e]];
        }
        ts.list.insert(ts.list.end(), list.begin(), list.end());
        ts.off.push_back((int32_t)ts.list.size());
        ts.hmax = std::max(ts.hmax, (int32_t)list.size());
    }
    // every entry's position must name its own neighbour
    for (int64_t b = 0; b < nt; ++b)
        for (int s = 0; s < tile; ++s) {
            const int32_t p = pts[b * tile + s];
            if (p < 0) continue;
            for (int32_t e = off[p]; e < off[p + 1]; ++e)
                if (!(ts.lnbr[e] < ts.off[b + 1] - ts.off[b] &&
                      ts.list[ts.off[b] + ts.lnbr[e]] == idx[e])) {
                    ts = TileSet{};
                    return false;
                }
        }
    ts.ntile = nt;
    ts.staged = (int64_t)ts.list.size();
    ts.pts = std::move(pts);
    return true;
}

// The partition that stages fewer points (runs on a tie), or an empty set
// (ntile 0) when neither has every list within max_list.
inline TileSet build_tiles(int64_t n, const int32_t* off, const int32_t* idx,
                           const std::vector<int64_t>& comp_off, int tile, int tj, int tk,
                           int max_list) {
    TileSet runs, blocks;
    const bool ok_r = tile_lists(n, off, idx, tile_points(n, off, idx, comp_off, tile, tj, tk, false),
                                 tile, max_list, runs);
    const bool ok_b = tile_lists(n, off, idx, tile_points(n, off, idx, comp_off, tile, tj, tk, true),
                                 tile, max_list, blocks);
    if (ok_b && (!ok_r || blocks.staged < runs.staged)) return blocks;
    if (ok_r) return runs;
    return TileSet{};
}

}  // namespace lskum
