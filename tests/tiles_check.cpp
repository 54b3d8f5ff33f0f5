// Host check of the q-derivative tile builder (paper_2406_07441_amd/csrc/lskum_tiles.h):
// reads a CSR cloud and its component offsets, builds the tiles with the
// library's constants and writes the result for the Python test to verify
// independently.
//
// input  (little-endian): int64 n, int64 ncomp, int64 comp_off[ncomp+1],
//                         int32 off[n+1], int32 idx[off[n]]
// output: int64 ntile, hmax, staged, row length of each component,
//         int32 pts[ntile*64], int32 off[ntile+1], int32 list[staged],
//         uint16 lnbr[nnz]
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../paper_2406_07441_amd/csrc/lskum_tiles.h"

template <class T>
static void rd(FILE* f, T* p, size_t n) {
    if (n && fread(p, sizeof(T), n, f) != n) {
        fprintf(stderr, "short read\n");
        exit(2);
    }
}
template <class T>
static void wr(FILE* f, const T* p, size_t n) {
    if (n) fwrite(p, sizeof(T), n, f);
}

int main(int argc, char** argv) {
    if (argc != 3) return 2;
    FILE* f = fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t n, ncomp;
    rd(f, &n, 1);
    rd(f, &ncomp, 1);
    std::vector<int64_t> comp_off(ncomp + 1);
    rd(f, comp_off.data(), comp_off.size());
    std::vector<int32_t> off(n + 1);
    rd(f, off.data(), off.size());
    std::vector<int32_t> idx(off[n]);
    rd(f, idx.data(), idx.size());
    fclose(f);
    // the library's tile shape (lskum_internal.h): 64 points, 16 x 4 blocks, lists <= 512
    const lskum::TileSet ts =
        lskum::build_tiles(n, off.data(), idx.data(), comp_off, 64, 16, 4, 512);
    FILE* g = fopen(argv[2], "wb");
    if (!g) return 2;
    const int64_t head[3] = {ts.ntile, ts.hmax, ts.staged};
    wr(g, head, 3);
    for (int64_t k = 0; k < ncomp; ++k) {
        const int64_t w = lskum::tile_row_length(off.data(), idx.data(), comp_off[k], comp_off[k + 1]);
        wr(g, &w, 1);
    }
    wr(g, ts.pts.data(), ts.pts.size());
    wr(g, ts.off.data(), ts.off.size());
    wr(g, ts.list.data(), ts.list.size());
    wr(g, ts.lnbr.data(), ts.lnbr.size());
    fclose(g);
    return 0;
}
