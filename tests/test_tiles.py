"""Host check of the q-derivative tiles (csrc/lskum_tiles.h), no GPU.

The LDS-tiled q-derivative kernels take a tile's points from tile_pts and
read every neighbour through a 2-byte position into the tile's staged list,
so the builder must give a partition of the points, lists no longer than the
LDS allocation allows, and positions that name each entry's own neighbour.
The builder is compiled here with g++ from the library's header and its
output is checked independently of its own checks, on O-grids (stored row by
row: blocks of rows expected), a jittered O-grid, a box, a two-component
cloud like a batch, and a randomly renumbered O-grid (no row structure)."""
import os
import re
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from paper_2406_07441_amd import cloudgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TILE, TJ, TK, MAXLIST = 64, 16, 4, 512


def test_harness_constants_match_library():
    """The harness builds tiles with the library's shape constants."""
    src = open(os.path.join(ROOT, "paper_2406_07441_amd", "csrc", "lskum_internal.h")).read()
    got = {k: int(v) for k, v in re.findall(r"constexpr int (kQTile\w*) = (\d+);", src)}
    assert got == {"kQTile": TILE, "kQTileJ": TJ, "kQTileK": TK, "kQTileMax": MAXLIST}


@pytest.fixture(scope="module")
def harness():
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    d = tempfile.mkdtemp(prefix="tiles_check_")
    exe = os.path.join(d, "tiles_check")
    subprocess.run([gxx, "-O2", "-std=c++17", os.path.join(ROOT, "tests", "tiles_check.cpp"),
                    "-o", exe], check=True)
    yield exe, d
    shutil.rmtree(d, ignore_errors=True)


def build(harness, off, idx, comp_off):
    exe, d = harness
    n = len(off) - 1
    fin, fout = os.path.join(d, "in.bin"), os.path.join(d, "out.bin")
    with open(fin, "wb") as f:
        np.array([n, len(comp_off) - 1], np.int64).tofile(f)
        np.asarray(comp_off, np.int64).tofile(f)
        np.asarray(off, np.int32).tofile(f)
        np.asarray(idx, np.int32).tofile(f)
    subprocess.run([exe, fin, fout], check=True)
    raw = open(fout, "rb").read()
    ntile, hmax, staged = np.frombuffer(raw, np.int64, 3)
    pos = 24
    rowlen = np.frombuffer(raw, np.int64, len(comp_off) - 1, pos)
    pos += 8 * (len(comp_off) - 1)
    pts = np.frombuffer(raw, np.int32, ntile * TILE, pos)
    pos += 4 * ntile * TILE
    toff = np.frombuffer(raw, np.int32, ntile + 1 if ntile else 0, pos)
    pos += 4 * len(toff)
    lst = np.frombuffer(raw, np.int32, staged, pos)
    pos += 4 * staged
    lnbr = np.frombuffer(raw, np.uint16, len(idx) if ntile else 0, pos)
    assert pos + 2 * len(lnbr) == len(raw)
    return dict(ntile=int(ntile), hmax=int(hmax), staged=int(staged), rowlen=rowlen, pts=pts,
                off=toff, list=lst, lnbr=lnbr)


def verify(t, off, idx):
    """Partition, list bounds, sorted unions and positions, checked here."""
    n = len(off) - 1
    pts = t["pts"].reshape(t["ntile"], TILE)
    real = pts[pts >= 0]
    assert np.all(pts[pts >= 0] < n)
    assert np.array_equal(np.sort(real), np.arange(n)), "not a partition of the points"
    sizes = np.diff(t["off"])
    assert sizes.max() == t["hmax"] <= MAXLIST and t["off"][-1] == t["staged"]
    for b in range(t["ntile"]):
        tp = pts[b][pts[b] >= 0]
        lst = t["list"][t["off"][b]:t["off"][b + 1]]
        union = np.unique(np.concatenate([idx[off[p]:off[p + 1]] for p in tp]))
        assert np.array_equal(lst, union)
        for p in tp:
            e = np.arange(off[p], off[p + 1])
            assert np.all(t["lnbr"][e] < len(lst))
            assert np.array_equal(lst[t["lnbr"][e]], idx[e])


def runs_staged(off, idx):
    n = len(off) - 1
    return sum(np.unique(idx[off[p0]:off[min(n, p0 + TILE)]]).size for p0 in range(0, n, TILE))


def test_ogrid_blocks_of_rows(harness):
    cl = cloudgen.ogrid(160, 40)
    off, idx = cl.nbr_off, cl.nbr_idx
    t = build(harness, off, idx, [0, cl.n])
    assert t["rowlen"][0] == 160
    verify(t, off, idx)
    # 16 x 4 blocks: (16 + 4) x (4 + 4) listed points at most, about 2.4 per point
    assert t["hmax"] <= 160 and t["staged"] < 0.5 * runs_staged(off, idx)
    assert t["ntile"] == (160 // TJ) * (40 // TK)


def test_jittered_ogrid_and_box(harness):
    for cl in (cloudgen.ogrid(128, 36, jitter_p=0.04, seed=7), cloudgen.box(11, 11)):
        off, idx = cl.nbr_off, cl.nbr_idx
        t = build(harness, off, idx, [0, cl.n])
        verify(t, off, idx)
        assert t["staged"] <= runs_staged(off, idx)


def test_two_components_like_a_batch(harness):
    """Two O-grids of different row length stored one after the other: each
    component gets its own row length; the row ends are partial blocks."""
    a, b = cloudgen.ogrid(96, 24), cloudgen.ogrid(70, 21)
    off = np.concatenate([a.nbr_off, b.nbr_off[1:] + a.nbr_off[-1]])
    idx = np.concatenate([a.nbr_idx, b.nbr_idx + a.n])
    t = build(harness, off, idx, [0, a.n, a.n + b.n])
    assert list(t["rowlen"]) == [96, 70]
    verify(t, off, idx)
    assert t["staged"] < runs_staged(off, idx)


def test_renumbered_cloud_without_rows(harness):
    """A random numbering has no rows: whichever partition the builder keeps
    is still valid (runs when blocks stage more or overflow the lists)."""
    cl = cloudgen.ogrid(64, 16)
    rng = np.random.default_rng(3)
    perm = rng.permutation(cl.n)          # new index of each old point
    inv = np.argsort(perm)                # old point of each new index
    deg = np.diff(cl.nbr_off)[inv]
    off = np.concatenate([[0], np.cumsum(deg)]).astype(np.int32)
    idx = np.concatenate([perm[cl.nbr_idx[cl.nbr_off[p]:cl.nbr_off[p + 1]]] for p in inv])
    t = build(harness, off, idx.astype(np.int32), [0, cl.n])
    if t["ntile"]:
        verify(t, off, idx)
        assert t["staged"] <= runs_staged(off, idx)
