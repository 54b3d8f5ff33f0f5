"""Seeded synthetic point clouds and flow conditions.

This module only builds inputs: point coordinates, point types, the wall
frame, CSR connectivity and flow conditions.  It holds none of the method's
arithmetic (no fluxes, no least squares, no colouring), so both the HIP
library's callers and the CPU oracle's tests draw their inputs from here.

Cloud recipe (a stand-in for the paper's NACA 0012 point distributions of the
subsonic/transonic test cases, Section 5 and Table 5, whose files are not
published):

* profile: symmetric NACA 4-digit thickness with the closed trailing-edge
  coefficient -0.1036, thickness ratio ``t``;
* wall points j = 0..Nw-1 at x_j = 1 - cos(psi_j), psi_j = pi/2 |1 - 2j/Nw|
  (clustered at the leading edge, linear at the trailing edge), y = +thickness
  for j <= Nw/2 and -thickness otherwise (j = 0 is the trailing edge, j = Nw/2
  the leading edge, (j, Nw-j) are mirror pairs).  The alternative
  ``spacing="cosine"`` (x = (1 + cos 2 pi j/Nw)/2) also clusters at the
  trailing edge; on the finer clouds its trailing-edge points (spacing
  ~1e-5 chord against ~1e-3 normal) drive the implicit iteration unstable;
* far field F_j = (0.5, 0) + 15 (cos phi_j, sin phi_j);
* layers k = 0..K-1 at P_jk = W_j + s_k (F_j - W_j), s_k = (r^k - 1)/(r^(K-1) - 1);
* point index p = k*Nw + j; k = 0 wall, k = K-1 outer (free stream), else interior;
* connectivity: every (j', k') with cyclic |dj| <= 2 and |dk| <= 2 except the
  point itself, in (dk, dj) lexicographic order -- the 8 grid neighbours plus
  the second ring, symmetric by construction;
* wall frame: unit tangent t_j = (W_{j-1} - W_{j+1}) / |.|, so that the normal
  n = (-t_y, t_x) points into the fluid; the outer ring's frame by the same
  rule, its normal pointing out of the domain; interior points get t = (1, 0);
* optional jitter: each interior point independently with probability
  ``jitter_p`` is displaced by xi1*0.2*h_j*e_j + xi2*0.2*h_k*e_k, xi ~ U(-1, 1),
  where e_j, h_j (e_k, h_k) are the unit direction and half-length of the
  grid-line chord between the point's j-neighbours (k-neighbours).

Random numbers come from splitmix64 used as a counter-based generator: draw n
of stream ``seed`` is mix(seed + (n + 1) * 0x9E3779B97F4A7C15) with the
published splitmix64 finaliser; a uniform in [0, 1) is (z >> 11) * 2^-53.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

WALL, INTERIOR, OUTER = 0, 1, 2

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, counters: np.ndarray) -> np.ndarray:
    """splitmix64 output for draws ``counters`` (uint64 array) of stream ``seed``."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (counters.astype(np.uint64) + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, counters: np.ndarray) -> np.ndarray:
    """Uniform doubles in [0, 1): top 53 bits of splitmix64 times 2^-53."""
    z = splitmix64(seed, counters)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


@dataclasses.dataclass
class Cloud:
    """A point cloud in structure-of-arrays form (all arrays C-contiguous)."""

    x: np.ndarray          # float64 [n]
    y: np.ndarray          # float64 [n]
    type: np.ndarray       # int8 [n]: 0 wall, 1 interior, 2 outer
    tx: np.ndarray         # float64 [n]: unit wall tangent, n = (-ty, tx) into the fluid
    ty: np.ndarray         # float64 [n]
    nbr_off: np.ndarray    # int32 [n+1] CSR offsets
    nbr_idx: np.ndarray    # int32 [nnz] CSR neighbour indices
    nw: int = 0            # wall points per ring (O-grid only)
    nk: int = 0            # rings (O-grid only)
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def nnz(self) -> int:
        return int(self.nbr_idx.shape[0])


def naca_thickness(x: np.ndarray, t: float) -> np.ndarray:
    """Half thickness of a symmetric NACA 4-digit section, closed trailing edge."""
    return 5.0 * t * (0.2969 * np.sqrt(x) - 0.1260 * x - 0.3516 * x ** 2
                      + 0.2843 * x ** 3 - 0.1036 * x ** 4)


def wall_points(nw: int, t: float, spacing: str = "le") -> tuple[np.ndarray, np.ndarray]:
    """Wall points: ``cosine`` x = (1 + cos phi)/2 clusters at both edges;
    ``le`` x = 1 - cos(psi), psi = pi/2 |1 - 2 j/nw|, clusters at the leading
    edge only and is linear near the trailing edge."""
    if nw < 8 or nw % 2:
        raise ValueError("nw must be even and >= 8")
    j = np.arange(nw)
    phi = 2.0 * np.pi * j / nw
    if spacing == "cosine":
        xw = 0.5 * (1.0 + np.cos(phi))
    elif spacing == "le":
        psi = 0.5 * np.pi * np.abs(1.0 - 2.0 * j / nw)
        xw = 1.0 - np.cos(psi)
    else:
        raise ValueError(spacing)
    yt = naca_thickness(np.clip(xw, 0.0, 1.0), t)
    yw = np.where(j <= nw // 2, yt, -yt)
    yw[0] = 0.0
    yw[nw // 2] = 0.0
    # exact mirror symmetry of the pairs (j, nw - j)
    jj = np.arange(1, nw // 2)
    xw[nw - jj] = xw[jj]
    yw[nw - jj] = -yw[jj]
    return xw, yw


def far_field_points(nw: int) -> tuple[np.ndarray, np.ndarray]:
    """Far-field circle of radius 15 about (0.5, 0), exactly mirror symmetric."""
    phi = 2.0 * np.pi * np.arange(nw) / nw
    fx, fy = 0.5 + 15.0 * np.cos(phi), 15.0 * np.sin(phi)
    fy[0] = 0.0
    fy[nw // 2] = 0.0
    jj = np.arange(1, nw // 2)
    fx[nw - jj] = fx[jj]
    fy[nw - jj] = -fy[jj]
    return fx, fy


def stretch_for_first_spacing(nw: int, nk: int, t: float, spacing: str = "le") -> float:
    """Ratio r whose first normal spacing equals the mean wall spacing."""
    xw, yw = wall_points(nw, t, spacing)
    per = np.hypot(np.roll(xw, -1) - xw, np.roll(yw, -1) - yw).sum()
    fx, fy = far_field_points(nw)
    length = np.hypot(fx - xw, fy - yw).mean()
    target = (per / nw) / length          # wanted s_1
    lo, hi = 1.0 + 1e-12, 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        s1 = (mid - 1.0) / (mid ** (nk - 1) - 1.0)
        if s1 > target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def ogrid(nw: int, nk: int, r: float | None = None, t: float = 0.12,
          jitter_p: float = 0.0, seed: int = 2406, name: str = "",
          spacing: str = "le") -> Cloud:
    """O-grid point cloud around a NACA 00tt profile (see module docstring)."""
    if nk < 5:
        raise ValueError("need at least 5 rings")
    if r is None:
        r = stretch_for_first_spacing(nw, nk, t, spacing)
    xw, yw = wall_points(nw, t, spacing)
    fx, fy = far_field_points(nw)
    k = np.arange(nk, dtype=np.float64)
    s = (r ** k - 1.0) / (r ** (nk - 1) - 1.0)
    s[0], s[-1] = 0.0, 1.0
    X = xw[None, :] + s[:, None] * (fx - xw)[None, :]
    Y = yw[None, :] + s[:, None] * (fy - yw)[None, :]

    if jitter_p > 0.0:
        X, Y = _jitter(X, Y, jitter_p, seed)

    n = nw * nk
    typ = np.full((nk, nw), INTERIOR, dtype=np.int8)
    typ[0, :] = WALL
    typ[-1, :] = OUTER
    tx = np.ones((nk, nw))
    ty = np.zeros((nk, nw))
    dxw = np.roll(xw, 1) - np.roll(xw, -1)     # W_{j-1} - W_{j+1}
    dyw = np.roll(yw, 1) - np.roll(yw, -1)
    ln = np.hypot(dxw, dyw)
    tx[0, :] = dxw / ln
    ty[0, :] = dyw / ln
    # outer ring: the same rule, so that n = (-t_y, t_x) points out of the domain
    xo, yo = X[-1], Y[-1]
    dxo = np.roll(xo, 1) - np.roll(xo, -1)
    dyo = np.roll(yo, 1) - np.roll(yo, -1)
    lo = np.hypot(dxo, dyo)
    tx[-1, :] = dxo / lo
    ty[-1, :] = dyo / lo

    off, idx = _ring_csr(nw, nk)
    return Cloud(x=np.ascontiguousarray(X.reshape(n)), y=np.ascontiguousarray(Y.reshape(n)),
                 type=typ.reshape(n).copy(), tx=tx.reshape(n).copy(), ty=ty.reshape(n).copy(),
                 nbr_off=off, nbr_idx=idx, nw=nw, nk=nk, name=name or f"ogrid{nw}x{nk}")


def _jitter(X, Y, p, seed):
    nk, nw = X.shape
    X = X.copy()
    Y = Y.copy()
    k = np.arange(1, nk - 1)
    j = np.arange(nw)
    kk, jj = np.meshgrid(k, j, indexing="ij")
    pid = (kk * nw + jj).astype(np.uint64)
    u_sel = uniform01(seed, 3 * pid)
    xi1 = 2.0 * uniform01(seed, 3 * pid + 1) - 1.0
    xi2 = 2.0 * uniform01(seed, 3 * pid + 2) - 1.0
    jp, jm = (jj + 1) % nw, (jj - 1) % nw
    ejx = X[kk, jp] - X[kk, jm]
    ejy = Y[kk, jp] - Y[kk, jm]
    ekx = X[kk + 1, jj] - X[kk - 1, jj]
    eky = Y[kk + 1, jj] - Y[kk - 1, jj]
    # 0.2 * half chord * unit vector = 0.1 * chord vector
    dx = xi1 * 0.1 * ejx + xi2 * 0.1 * ekx
    dy = xi1 * 0.1 * ejy + xi2 * 0.1 * eky
    sel = u_sel < p
    X[kk[sel], jj[sel]] += dx[sel]
    Y[kk[sel], jj[sel]] += dy[sel]
    return X, Y


def _ring_csr(nw: int, nk: int) -> tuple[np.ndarray, np.ndarray]:
    k = np.repeat(np.arange(nk), nw)
    j = np.tile(np.arange(nw), nk)
    cols = []
    for dk in range(-2, 3):
        for dj in range(-2, 3):
            if dk == 0 and dj == 0:
                continue
            kn = k + dk
            ok = (kn >= 0) & (kn < nk)
            cols.append(np.where(ok, kn * nw + (j + dj) % nw, -1))
    nb = np.stack(cols, axis=1)
    mask = nb >= 0
    cnt = mask.sum(axis=1)
    off = np.zeros(nw * nk + 1, dtype=np.int64)
    np.cumsum(cnt, out=off[1:])
    if off[-1] >= 2 ** 31:
        raise ValueError("too many edges for int32 CSR")
    return off.astype(np.int32), nb[mask].astype(np.int32)


def box(nx: int, ny: int, h: float = 0.1, wall_bottom: bool = False) -> Cloud:
    """Cartesian box cloud with the same 5x5 ring connectivity (no wrap).

    Boundary rows/columns are outer points; with ``wall_bottom`` the bottom
    row is a flat wall (tangent (1, 0), normal (0, 1) into the fluid).
    """
    jj, kk = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    X = (jj * h).astype(np.float64)
    Y = (kk * h).astype(np.float64)
    typ = np.full((ny, nx), INTERIOR, dtype=np.int8)
    typ[:, 0] = typ[:, -1] = typ[-1, :] = OUTER
    typ[0, :] = WALL if wall_bottom else OUTER
    if wall_bottom:
        typ[0, 0] = typ[0, -1] = OUTER
    n = nx * ny
    k = kk.reshape(n)
    j = jj.reshape(n)
    cols = []
    for dk in range(-2, 3):
        for dj in range(-2, 3):
            if dk == 0 and dj == 0:
                continue
            kn, jn = k + dk, j + dj
            ok = (kn >= 0) & (kn < ny) & (jn >= 0) & (jn < nx)
            cols.append(np.where(ok, kn * nx + jn, -1))
    nb = np.stack(cols, axis=1)
    mask = nb >= 0
    off = np.zeros(n + 1, dtype=np.int32)
    np.cumsum(mask.sum(axis=1), out=off[1:])
    return Cloud(x=X.reshape(n).copy(), y=Y.reshape(n).copy(), type=typ.reshape(n).copy(),
                 tx=np.ones(n), ty=np.zeros(n), nbr_off=off,
                 nbr_idx=nb[mask].astype(np.int32), nw=nx, nk=ny, name=f"box{nx}x{ny}")


# ---------------------------------------------------------------------------
# Named workloads.  Sizes follow the paper's 2D inviscid NACA 0012 cases
# (Mach 0.63 / 2 deg subsonic, 0.85 / 1 deg transonic) at O-grid resolutions.
# ---------------------------------------------------------------------------

def cloud_6400() -> Cloud:
    """160 x 40 O-grid, stretching 1.1, 12% thick."""
    return ogrid(160, 40, r=1.1, t=0.12, name="ogrid160x40")


def cloud_163840(seed: int = 2406) -> Cloud:
    """640 x 256 O-grid, first spacing = mean wall spacing, 4% jittered."""
    return ogrid(640, 256, r=None, t=0.12, jitter_p=0.04, seed=seed, name="ogrid640x256j")


def cloud_2621440() -> Cloud:
    """2560 x 1024 O-grid, first spacing = mean wall spacing, no jitter."""
    return ogrid(2560, 1024, r=None, t=0.12, name="ogrid2560x1024")


def batch_clouds(seed: int = 4, count: int = 8, nmin: int = 40_000, nmax: int = 640_000):
    """Uneven clouds: N ~ U(nmin, nmax), thickness ~ U(0.09, 0.15)."""
    u = uniform01(seed, np.arange(2 * count, dtype=np.uint64))
    out = []
    for c in range(count):
        n_target = nmin + u[2 * c] * (nmax - nmin)
        t = 0.09 + u[2 * c + 1] * 0.06
        nw = 2 * int(round(math.sqrt(2.5 * n_target) / 2.0))
        nk = int(round(n_target / nw))
        out.append(ogrid(nw, nk, r=None, t=t, name=f"batch{c}_{nw}x{nk}"))
    return out


def batch_conditions(seed: int = 5, count: int = 64):
    """Mach ~ U(0.3, 0.85), AoA ~ U(-4, 8) degrees."""
    u = uniform01(seed, np.arange(2 * count, dtype=np.uint64))
    mach = 0.3 + u[0::2] * 0.55
    aoa = -4.0 + u[1::2] * 12.0
    return mach, aoa
