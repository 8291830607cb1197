"""Seeded synthetic inputs: conductivity models, Dirichlet boundary tables,
interface-node sets and request streams.

This module holds problem *data* only -- none of the walk, the phase
integral or the estimator.  Both the GPU library (through its binding) and
the CPU oracle consume the same :class:`Problem` objects built here.

Boundary data (Sec. 2.1, the Dirichlet conditions): every wall value is the
1-D layered-earth TE solution of the vertical column through that point,
normalised to E = 1 at the top of the domain, linear in air (alpha = 0) and
decaying in the bottom half-space.  For the homogeneous unit-square toy the
analytic plane wave exp(-sqrt(i alpha) z) is used directly.

Lengths are in skin depths delta1 of sigma1 = 0.01 S/m at f1 = 1 Hz
(delta1 = sqrt(2 / (omega1 mu0 sigma1)) = 5032.9 m), so alpha = 2 (sigma /
sigma1) (f / f1) for a region of conductivity sigma at frequency f.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

MU0 = 4.0e-7 * math.pi
SIGMA1 = 0.01
F1 = 1.0
DELTA1 = math.sqrt(2.0 / (2.0 * math.pi * F1 * MU0 * SIGMA1))

HALF_Z_LT, HALF_Y_LT, BOX, TRIANGLE = 0, 1, 2, 3
FP64, FP32_MIXED = 0, 1
WALL_TOP, WALL_RIGHT, WALL_BOTTOM, WALL_LEFT = 0, 1, 2, 3


@dataclasses.dataclass
class Region:
    kind: int
    params: Tuple[float, ...]          # up to 6 numbers, see the kind
    sigma: float

    def param6(self) -> List[float]:
        p = list(self.params) + [0.0] * (6 - len(self.params))
        return p[:6]


@dataclasses.dataclass
class Problem:
    """One interface-solve request: model, boundary data, nodes, paths."""
    y_lo: float
    y_hi: float
    z_lo: float
    z_hi: float
    regions: List[Region]
    sigma_background: float
    length_unit_m: float
    freq_hz: float                     # > 0: alpha = omega mu0 sigma L^2
    alpha_direct: float                # freq_hz == 0: alpha = alpha_direct sigma
    g: np.ndarray                      # complex128 (4, M+1): top, right, bottom, left
    nodes: np.ndarray                  # float64 (n, 2): (y, z)
    path_begin: np.ndarray             # uint32 (n,)
    path_count: np.ndarray             # uint32 (n,)
    dt: float
    seed: int = 0
    stream: int = 0
    max_steps: int = 2_000_000_000
    precision: int = FP64
    name: str = ""
    naive_exit: bool = False           # exit only on a crossing (no Brownian-bridge test)

    @property
    def n_nodes(self) -> int:
        return int(self.nodes.shape[0])

    @property
    def total_paths(self) -> int:
        return int(np.asarray(self.path_count, dtype=np.uint64).sum())

    @property
    def g_norm(self) -> float:
        return float(np.abs(self.g).max()) if self.g.size else 0.0

    def alphas(self) -> np.ndarray:
        """alpha per region (regions first, background last)."""
        sig = np.array([r.sigma for r in self.regions] + [self.sigma_background])
        if self.freq_hz > 0:
            return 2.0 * math.pi * self.freq_hz * MU0 * sig * self.length_unit_m ** 2
        return self.alpha_direct * sig

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)

    def subset(self, idx: Sequence[int]) -> "Problem":
        idx = np.asarray(idx, dtype=np.int64)
        return self.replace(nodes=self.nodes[idx].copy(),
                            path_begin=self.path_begin[idx].copy(),
                            path_count=self.path_count[idx].copy())

    def with_paths(self, count: int, begin: int = 0) -> "Problem":
        n = self.n_nodes
        return self.replace(path_begin=np.full(n, begin, np.uint32),
                            path_count=np.full(n, count, np.uint32))


# --------------------------------------------------------------------------
# Region predicate (used here only to lay out 1-D columns for the boundary
# tables): first primitive in list order wins, else the background.
# --------------------------------------------------------------------------

def _inside(kind: int, v: Sequence[float], y: float, z: float) -> bool:
    if kind == HALF_Z_LT:
        return z < v[0]
    if kind == HALF_Y_LT:
        return y < v[0]
    if kind == BOX:
        return v[0] <= y < v[1] and v[2] <= z < v[3]
    if kind == TRIANGLE:
        e0 = (v[2] - v[0]) * (z - v[1]) - (v[3] - v[1]) * (y - v[0])
        e1 = (v[4] - v[2]) * (z - v[3]) - (v[5] - v[3]) * (y - v[2])
        e2 = (v[0] - v[4]) * (z - v[5]) - (v[1] - v[5]) * (y - v[4])
        return (e0 >= 0 and e1 >= 0 and e2 >= 0) or (e0 <= 0 and e1 <= 0 and e2 <= 0)
    raise ValueError(kind)


def sigma_at(regions: Sequence[Region], sigma_bg: float, y: float, z: float) -> float:
    for r in regions:
        if _inside(r.kind, r.param6(), y, z):
            return r.sigma
    return sigma_bg


def _column_breaks(regions: Sequence[Region], y: float) -> List[float]:
    zs: List[float] = []
    for r in regions:
        v = r.param6()
        if r.kind == HALF_Z_LT:
            zs.append(v[0])
        elif r.kind == BOX and v[0] <= y < v[1]:
            zs += [v[2], v[3]]
        elif r.kind == TRIANGLE:
            pts = [(v[0], v[1]), (v[2], v[3]), (v[4], v[5])]
            for a in range(3):
                (ya, za), (yb, zb) = pts[a], pts[(a + 1) % 3]
                if ya == yb:
                    if y == ya:
                        zs += [za, zb]
                    continue
                t = (y - ya) / (yb - ya)
                if 0.0 <= t <= 1.0:
                    zs.append(za + t * (zb - za))
    return sorted(set(zs))


def column_layers(regions: Sequence[Region], sigma_bg: float, y: float,
                  z_top: float) -> Tuple[np.ndarray, np.ndarray]:
    """Layer tops (ascending, first = z_top) and conductivities of the
    vertical column at y below z_top; the last layer extends to +infinity."""
    cuts = [z for z in _column_breaks(regions, y) if z > z_top]
    tops = [z_top] + cuts
    sig = []
    for i, zt in enumerate(tops):
        zb = tops[i + 1] if i + 1 < len(tops) else zt + 1.0
        sig.append(sigma_at(regions, sigma_bg, y, 0.5 * (zt + zb)))
    # merge equal neighbours
    mt, ms = [tops[0]], [sig[0]]
    for zt, s in zip(tops[1:], sig[1:]):
        if s != ms[-1]:
            mt.append(zt)
            ms.append(s)
    return np.array(mt, dtype=np.float64), np.array(ms, dtype=np.float64)


def layered_1d(tops: np.ndarray, alphas: np.ndarray, z: np.ndarray) -> np.ndarray:
    """1-D TE solution of E'' = i alpha(z) E on layers [tops[i], tops[i+1])
    with the last layer a half-space (alpha > 0: decaying wave), alpha = 0
    layers linear, normalised to E(tops[0]) = 1.  Evaluated at z >= tops[0].

    Propagates the log-amplitude and the ratio zeta = E'/E upward, which is
    stable for any layer thickness."""
    tops = np.asarray(tops, dtype=np.float64)
    alphas = np.asarray(alphas, dtype=np.float64)
    K = len(tops)
    if alphas[-1] <= 0:
        raise ValueError("bottom half-space must be conducting")
    k = np.sqrt(1j * alphas.astype(np.complex128))
    logE = np.zeros(K, dtype=np.complex128)   # log E at each layer top
    zeta = np.zeros(K, dtype=np.complex128)   # E'/E just below each layer top
    zeta[K - 1] = -k[K - 1]
    logE[K - 1] = 0.0

    def up(i: int, zeta_b: complex, h: float) -> Tuple[complex, complex]:
        """Move up by h >= 0 from a point at the bottom side within layer i:
        returns (log(E_top / E_bottom), zeta at the top)."""
        if alphas[i] == 0.0:
            fac = 1.0 - zeta_b * h
            return np.log(fac), zeta_b / fac
        kk = k[i]
        rho = zeta_b / kk
        e = np.exp(-2.0 * kk * h)
        num = (1.0 - rho) + (1.0 + rho) * e
        return kk * h + np.log(0.5 * num), kk * ((rho - 1.0) + (rho + 1.0) * e) / num

    for i in range(K - 2, -1, -1):
        h = tops[i + 1] - tops[i]
        dlog, zt = up(i, zeta[i + 1], h)
        logE[i] = logE[i + 1] + dlog
        zeta[i] = zt

    z = np.asarray(z, dtype=np.float64)
    out = np.empty(z.shape, dtype=np.complex128)
    for idx, zz in np.ndenumerate(z):
        i = int(np.searchsorted(tops, zz, side="right") - 1)
        i = max(i, 0)
        if i == K - 1:
            lg = logE[i] - k[i] * (zz - tops[i])
        else:
            h = tops[i + 1] - zz
            dlog, _ = up(i, zeta[i + 1], h)
            lg = logE[i + 1] + dlog
        out[idx] = np.exp(lg - logE[0])
    return out


def _alpha_of(sig: np.ndarray, freq_hz: float, L: float, alpha_direct: float) -> np.ndarray:
    if freq_hz > 0:
        return 2.0 * math.pi * freq_hz * MU0 * sig * L * L
    return alpha_direct * sig


def column_tables(regions: Sequence[Region], sigma_bg: float, walls: Tuple[float, float, float, float],
                  freq_hz: float, L: float, alpha_direct: float, M: int) -> np.ndarray:
    """Dirichlet tables (4, M+1) from the 1-D solution of each column."""
    y_lo, y_hi, z_lo, z_hi = walls
    g = np.empty((4, M + 1), dtype=np.complex128)
    ys = y_lo + np.arange(M + 1) * ((y_hi - y_lo) / M)
    zs = z_lo + np.arange(M + 1) * ((z_hi - z_lo) / M)
    cache = {}

    def col(y: float):
        tops, sig = column_layers(regions, sigma_bg, y, z_lo)
        key = (tuple(tops), tuple(sig))
        if key not in cache:
            cache[key] = (tops, _alpha_of(sig, freq_hz, L, alpha_direct))
        return cache[key]

    for i, y in enumerate(ys):
        tops, al = col(float(y))
        g[WALL_TOP, i] = layered_1d(tops, al, np.array([z_lo]))[0]
        g[WALL_BOTTOM, i] = layered_1d(tops, al, np.array([z_hi]))[0]
    tops, al = col(float(y_lo))
    g[WALL_LEFT] = layered_1d(tops, al, zs)
    tops, al = col(float(y_hi))
    g[WALL_RIGHT] = layered_1d(tops, al, zs)
    return g


def column_field(regions: Sequence[Region], sigma_bg: float, y: np.ndarray, z: np.ndarray, z_top: float,
                 freq_hz: float, L: float, alpha_direct: float = 0.0, boundary_only: bool = False) -> np.ndarray:
    """The layered 1-D solution of each vertical column y[i] at depths z
    (normalised to 1 at z_top), as a complex (nz, ny) array; with
    boundary_only, only the first and last rows and columns are filled (the
    outer Dirichlet values of a grid) and the rest is zero."""
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    F = np.zeros((z.size, y.size), dtype=np.complex128)
    cols = range(y.size) if not boundary_only else sorted({0, y.size - 1} | set(range(y.size)))
    for i in cols:
        tops, sig = column_layers(regions, sigma_bg, float(y[i]), z_top)
        col = layered_1d(tops, _alpha_of(sig, freq_hz, L, alpha_direct), z)
        if boundary_only and 0 < i < y.size - 1:
            F[0, i], F[-1, i] = col[0], col[-1]
        else:
            F[:, i] = col
    return F


def wall_coords(y_lo: float, y_hi: float, z_lo: float, z_hi: float, M: int):
    """Sample coordinates of the tables: (points (4, M+1, 2))."""
    ys = y_lo + np.arange(M + 1) * ((y_hi - y_lo) / M)
    zs = z_lo + np.arange(M + 1) * ((z_hi - z_lo) / M)
    P = np.empty((4, M + 1, 2))
    P[WALL_TOP, :, 0], P[WALL_TOP, :, 1] = ys, z_lo
    P[WALL_BOTTOM, :, 0], P[WALL_BOTTOM, :, 1] = ys, z_hi
    P[WALL_LEFT, :, 0], P[WALL_LEFT, :, 1] = y_lo, zs
    P[WALL_RIGHT, :, 0], P[WALL_RIGHT, :, 1] = y_hi, zs
    return P


def tables_from_function(fn, walls, M: int) -> np.ndarray:
    P = wall_coords(*walls, M)
    return np.asarray(fn(P[..., 0], P[..., 1]), dtype=np.complex128).reshape(4, M + 1)


# --------------------------------------------------------------------------
# The five workload families.
# --------------------------------------------------------------------------

def unit_square(alpha: float = 20.0, g_fn=None, M: int = 4096, n_nodes: int = 8,
                paths: int = 4096, dt: float = 1e-4, seed: int = 0, stream: int = 0,
                precision: int = FP64, nodes: Optional[np.ndarray] = None) -> Problem:
    """Homogeneous toy: Omega = [0,1]^2, Laplace E = i alpha E, g on the whole
    boundary (default: the plane wave exp(-sqrt(i alpha) z)), nodes at
    ((j + 1/2)/n, 1/2)."""
    if g_fn is None:
        k = np.sqrt(1j * alpha)
        g_fn = lambda y, z: np.exp(-k * z)  # noqa: E731
    walls = (0.0, 1.0, 0.0, 1.0)
    g = tables_from_function(g_fn, walls, M)
    if nodes is None:
        nodes = np.stack([(np.arange(n_nodes) + 0.5) / n_nodes, np.full(n_nodes, 0.5)], axis=1)
    n = nodes.shape[0]
    return Problem(*walls, regions=[], sigma_background=1.0, length_unit_m=1.0,
                   freq_hz=0.0, alpha_direct=float(alpha), g=g, nodes=np.asarray(nodes, np.float64),
                   path_begin=np.zeros(n, np.uint32), path_count=np.full(n, paths, np.uint32),
                   dt=dt, seed=seed, stream=stream, precision=precision, name="unit_square")


QS_WALLS = (-8.0, 8.0, -6.0, 8.0)


def quarter_space(paths: int = 65536, dt: float = 4e-4, M: int = 16384, seed: int = 0,
                  stream: int = 0, precision: int = FP32_MIXED, freq_hz: float = 1.0,
                  sigma_left: float = 0.01, sigma_right: float = 0.1) -> Problem:
    """Quarter-space TE: sigma_left for y < 0, sigma_right for y >= 0, air for
    z < 0; 256 nodes on the vertical interface y = 0, z in (0, 8) and 256 on
    the surface z = 0, y in (-8, 8)."""
    regions = [Region(HALF_Z_LT, (0.0,), 0.0), Region(HALF_Y_LT, (0.0,), sigma_left)]
    g = column_tables(regions, sigma_right, QS_WALLS, freq_hz, DELTA1, 0.0, M)
    j = np.arange(256)
    n1 = np.stack([np.zeros(256), (j + 0.5) / 32.0], axis=1)
    n2 = np.stack([-8.0 + (j + 0.5) / 16.0, np.zeros(256)], axis=1)
    nodes = np.concatenate([n1, n2])
    n = nodes.shape[0]
    return Problem(*QS_WALLS, regions=regions, sigma_background=sigma_right,
                   length_unit_m=DELTA1, freq_hz=freq_hz, alpha_direct=0.0, g=g, nodes=nodes,
                   path_begin=np.zeros(n, np.uint32), path_count=np.full(n, paths, np.uint32),
                   dt=dt, seed=seed, stream=stream, precision=precision, name="quarter_space")


def block_in_half_space(freq_hz: float, paths: int = 32768, dt: float = 4e-4, M: int = 16384,
                        seed: int = 0, stream: int = 0, precision: int = FP32_MIXED) -> Problem:
    """Block sigma = 1 S/m on y in [-1, 1], z in [0.5, 1.5] in a 0.01 S/m
    half-space under air; 4 x 128 nodes at the midpoints of equal segments of
    the block edges plus 512 on the surface."""
    regions = [Region(HALF_Z_LT, (0.0,), 0.0), Region(BOX, (-1.0, 1.0, 0.5, 1.5), 1.0)]
    g = column_tables(regions, 0.01, QS_WALLS, freq_hz, DELTA1, 0.0, M)
    k = (np.arange(128) + 0.5) / 128.0
    top = np.stack([-1.0 + 2.0 * k, np.full(128, 0.5)], axis=1)
    bot = np.stack([-1.0 + 2.0 * k, np.full(128, 1.5)], axis=1)
    left = np.stack([np.full(128, -1.0), 0.5 + k], axis=1)
    right = np.stack([np.full(128, 1.0), 0.5 + k], axis=1)
    s = np.arange(512)
    surf = np.stack([-8.0 + (s + 0.5) * 16.0 / 512.0, np.zeros(512)], axis=1)
    nodes = np.concatenate([top, bot, left, right, surf])
    n = nodes.shape[0]
    return Problem(*QS_WALLS, regions=regions, sigma_background=0.01, length_unit_m=DELTA1,
                   freq_hz=freq_hz, alpha_direct=0.0, g=g, nodes=nodes,
                   path_begin=np.zeros(n, np.uint32), path_count=np.full(n, paths, np.uint32),
                   dt=dt, seed=seed, stream=stream, precision=precision,
                   name=f"block_f{freq_hz:g}")


def multi_body(seed: int = 0, n_boxes: int = 4, n_triangles: int = 2, freq_hz: float = 1.0, paths: int = 16384,
               dt: float = 4e-4, M: int = 4096, precision: int = FP32_MIXED) -> Problem:
    """A seeded model of several bodies under air (the walker's generic
    signature): n_boxes boxes and n_triangles triangles with corners uniform
    in y in [-5, 5], z in [0.2, 5] skin depths (boxes 0.5-3 wide, 0.3-2 tall),
    conductivities log-uniform in [0.1, 10] S/m, in a 0.01 S/m half-space; the
    first body listed wins where bodies overlap.  Nodes: the 128 surface
    nodes y = -8 + (j + 1/2) / 8, z = 0 (the same as block_in_half_space's
    surface subset), `paths` paths each."""
    rng = np.random.default_rng(7_000_003 + seed)
    regions = [Region(HALF_Z_LT, (0.0,), 0.0)]
    for _ in range(n_boxes):
        y0, z0 = rng.uniform(-5, 4), rng.uniform(0.2, 4)
        regions.append(Region(BOX, (y0, y0 + rng.uniform(0.5, 3), z0, z0 + rng.uniform(0.3, 2)),
                              float(10 ** rng.uniform(-1, 1))))
    for _ in range(n_triangles):
        v = np.stack([rng.uniform(-5, 5, 3), rng.uniform(0.2, 5, 3)], axis=1)
        regions.append(Region(TRIANGLE, tuple(float(x) for x in v.reshape(-1)), float(10 ** rng.uniform(-1, 1))))
    g = column_tables(regions, 0.01, QS_WALLS, freq_hz, DELTA1, 0.0, M)
    j = np.arange(128)
    nodes = np.stack([-8.0 + (j + 0.5) / 8.0, np.zeros(128)], axis=1)
    return Problem(*QS_WALLS, regions=regions, sigma_background=0.01, length_unit_m=DELTA1, freq_hz=freq_hz,
                   alpha_direct=0.0, g=g, nodes=nodes, path_begin=np.zeros(128, np.uint32),
                   path_count=np.full(128, paths, np.uint32), dt=dt, seed=seed, precision=precision,
                   name=f"multi_body_{seed}")


# COMMEMI 2D-1 geometry of Sec. 4.3, in kilometres: a 2 S/m block 1 km wide
# and 2 km tall, its top 0.25 km below the surface, in a 0.01 S/m half-space
# under air; response sites on the surface.
COMMEMI_SITES_KM = (0.0, 0.5, 1.0, 2.0, 4.0)
COMMEMI_WALLS = (-10.0, 10.0, -5.0, 10.0)
# point spacing h per site for the surface-jump-corrected difference: below
# the block's top (0.25 km) over the block, wider away from it
COMMEMI_H_KM = (0.1, 0.1, 0.2, 0.4, 0.4)


def commemi_te_points(freq_hz: float = 10.0, paths: int = 65536, h=0.01, dt: float = 1e-4,
                      sites=COMMEMI_SITES_KM, walls=COMMEMI_WALLS, M: int = 16384, seed: int = 0,
                      precision: int = FP32_MIXED, block: bool = True) -> List[Problem]:
    """Three problems whose node j is site j at depth -h_j, 0 and +h_j (z
    down; h one spacing for all sites or one per site): the field there gives
    the TE response of the site by a centred difference.  The three share
    seed, stream and node order, so the three points of a site walk on the
    same random numbers.  block=False gives the plain half-space (apparent
    resistivity 100 ohm m, phase 45 degrees)."""
    regions = [Region(HALF_Z_LT, (0.0,), 0.0)]
    if block:
        regions.append(Region(BOX, (-0.5, 0.5, 0.25, 2.25), 2.0))
    g = column_tables(regions, 0.01, walls, freq_hz, 1000.0, 0.0, M)
    ys = np.asarray(sites, dtype=np.float64)
    hs = np.broadcast_to(np.asarray(h, dtype=np.float64), ys.shape)
    out = []
    for sgn, tag in ((-1.0, "minus"), (0.0, "mid"), (1.0, "plus")):
        nodes = np.stack([ys, sgn * hs], axis=1)
        n = nodes.shape[0]
        out.append(Problem(*walls, regions=regions, sigma_background=0.01, length_unit_m=1000.0,
                           freq_hz=freq_hz, alpha_direct=0.0, g=g, nodes=nodes,
                           path_begin=np.zeros(n, np.uint32), path_count=np.full(n, paths, np.uint32),
                           dt=dt, seed=seed, stream=0, precision=precision,
                           name=f"commemi_te_{tag}" if block else f"halfspace_te_{tag}"))
    return out


TRIANGLE_FREQS = tuple(float(x) for x in np.logspace(-2, 2, 8))


def _perimeter_points(poly: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Points at arc-length fractions u of a closed polyline."""
    seg = np.roll(poly, -1, axis=0) - poly
    ln = np.hypot(seg[:, 0], seg[:, 1])
    cum = np.concatenate([[0.0], np.cumsum(ln)])
    s = u * cum[-1]
    i = np.clip(np.searchsorted(cum, s, side="right") - 1, 0, len(ln) - 1)
    t = (s - cum[i]) / ln[i]
    return poly[i] + t[:, None] * seg[i]


def triangle_request(m: int, precision: int = FP32_MIXED, dt: float = 4e-4, M: int = 16384,
                     paths_scale: float = 1.0) -> Problem:
    """Request m of the triangle family (seed m): a triangle with vertices
    uniform in y in [-3, 3], z in [0.2, 3], sigma log-uniform in [0.1, 10]
    S/m, in a 0.01 S/m half-space under air; one of 8 log-spaced frequencies
    in [0.01, 100] Hz; 32..1024 nodes spread by arc length over the triangle
    perimeter and the surface segment [-8, 8]; paths log-uniform in
    [4096, 262144], a multiple of 64."""
    rng = np.random.default_rng(1_000_003 + m)
    while True:
        V = np.stack([rng.uniform(-3, 3, 3), rng.uniform(0.2, 3, 3)], axis=1)
        area = 0.5 * abs((V[1, 0] - V[0, 0]) * (V[2, 1] - V[0, 1]) - (V[2, 0] - V[0, 0]) * (V[1, 1] - V[0, 1]))
        if area > 0.05:
            break
    sig = float(10 ** rng.uniform(-1, 1))
    f = TRIANGLE_FREQS[int(rng.integers(0, 8))]
    n = int(rng.integers(32, 1025))
    paths = int(round(math.exp(rng.uniform(math.log(4096), math.log(262144))) / 64.0)) * 64
    paths = max(64, int(paths * paths_scale) // 64 * 64)
    regions = [Region(HALF_Z_LT, (0.0,), 0.0), Region(TRIANGLE, tuple(V.reshape(-1)), sig)]
    g = column_tables(regions, 0.01, QS_WALLS, f, DELTA1, 0.0, M)
    # arc-length positions over triangle perimeter + surface segment, in
    # proportion to their lengths
    per = float(np.sum(np.hypot(*(np.roll(V, -1, axis=0) - V).T)))
    n_tri = int(round(n * per / (per + 16.0)))
    pts_tri = _perimeter_points(V, np.sort(rng.uniform(0, 1, n_tri)))
    ys = np.sort(rng.uniform(-8, 8, n - n_tri))
    ys = np.clip(ys, -8 + 1e-6, 8 - 1e-6)
    pts_surf = np.stack([ys, np.zeros(n - n_tri)], axis=1)
    nodes = np.concatenate([pts_tri, pts_surf]).astype(np.float64)
    return Problem(*QS_WALLS, regions=regions, sigma_background=0.01, length_unit_m=DELTA1,
                   freq_hz=f, alpha_direct=0.0, g=g, nodes=nodes,
                   path_begin=np.zeros(n, np.uint32), path_count=np.full(n, paths, np.uint32),
                   dt=dt, seed=m, stream=0, precision=precision, name=f"triangle_{m}")


def layered_check(alpha_ground: float = 2.0, walls=(-2.0, 2.0, -1.0, 3.0), M: int = 4096,
                  n_nodes: int = 8, paths: int = 4096, dt: float = 4e-4, seed: int = 7,
                  precision: int = FP64) -> Problem:
    """Air over a uniform half-space (alpha_ground), g from the same 1-D
    solution on all four walls, so the 2-D solution is the 1-D one."""
    regions = [Region(HALF_Z_LT, (0.0,), 0.0)]
    g = column_tables(regions, 1.0, walls, 0.0, 1.0, alpha_ground, M)
    zs = walls[2] + (np.arange(n_nodes) + 0.5) * (walls[3] - walls[2]) / n_nodes
    nodes = np.stack([np.full(n_nodes, 0.3), zs], axis=1)
    return Problem(*walls, regions=regions, sigma_background=1.0, length_unit_m=1.0,
                   freq_hz=0.0, alpha_direct=alpha_ground, g=g, nodes=nodes,
                   path_begin=np.zeros(n_nodes, np.uint32),
                   path_count=np.full(n_nodes, paths, np.uint32), dt=dt, seed=seed,
                   precision=precision, name="layered_check")


def served_trace(n_requests: int, rate_hz: float, seed: int = 1, paths_cap: int = 1 << 20,
                 node_range=(16, 64), paths_override: Optional[int] = None,
                 precision: int = FP32_MIXED) -> List[Tuple[float, Problem]]:
    """Poisson arrivals of requests drawn uniformly from the unit-square,
    quarter-space and block families; node subsets seeded per request.
    Returns (arrival_time_s, problem) pairs.  Paths per node are either
    `paths_override` or left for the caller's target-SE rule."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    base_qs = quarter_space(paths=4096, precision=precision)
    base_blk = {f: block_in_half_space(f, paths=4096, precision=precision) for f in (0.1, 1.0, 10.0, 100.0)}
    base_us = unit_square(paths=4096, precision=precision)
    for i in range(n_requests):
        t += float(rng.exponential(1.0 / rate_hz))
        kind = int(rng.integers(0, 3))
        if kind == 0:
            p = base_us
            idx = np.arange(p.n_nodes)
        elif kind == 1:
            p = base_qs
            idx = np.sort(rng.choice(p.n_nodes, int(rng.integers(node_range[0], node_range[1] + 1)), replace=False))
        else:
            p = base_blk[float(rng.choice([0.1, 1.0, 10.0, 100.0]))]
            idx = np.sort(rng.choice(p.n_nodes, int(rng.integers(node_range[0], node_range[1] + 1)), replace=False))
        q = p.subset(idx).replace(seed=1000 + i, name=f"{p.name}#{i}")
        if paths_override is not None:
            q = q.with_paths(paths_override)
        out.append((t, q))
    return out


# ---------------------------------------------------------------------------
# Discontinuous kappa (the interface scheme of Secs. 2.2, 3.1): one vertical
# interface, (1/2) div(kappa grad u) - lambda u = 0 with kappa, lambda constant
# on each side.
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class KappaProblem:
    y_lo: float
    y_hi: float
    z_lo: float
    z_hi: float
    y_if: float
    kappa: Tuple[float, float]            # y < y_if, y >= y_if
    lam: Tuple[complex, complex]          # killing rate per side
    g: np.ndarray                         # (4, M+1) complex, walls top, right, bottom, left
    nodes: np.ndarray
    path_begin: np.ndarray
    path_count: np.ndarray
    dt: float
    seed: int = 0
    stream: int = 0
    max_steps: int = 2_000_000_000
    name: str = ""

    @property
    def n_nodes(self) -> int:
        return int(self.nodes.shape[0])

    @property
    def total_paths(self) -> int:
        return int(np.sum(self.path_count, dtype=np.int64))

    def replace(self, **kw) -> "KappaProblem":
        return dataclasses.replace(self, **kw)

    def with_paths(self, paths: int) -> "KappaProblem":
        n = self.n_nodes
        return self.replace(path_begin=np.zeros(n, np.uint32), path_count=np.full(n, paths, np.uint32))


def kappa_model_field(y, z, lam: complex = 10j, kappa=(1.0, 10.0)):
    """The analytic test model of Sec. 4.1 (reading: div(kappa grad u) =
    lambda u, principal roots): (z + 1) cosh(sqrt(lambda / kappa_i) y) on side
    i of y = 0."""
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    k = np.where(y < 0.0, kappa[0], kappa[1])
    return (z + 1.0) * np.cosh(np.sqrt(lam / k) * y)


def kappa_analytic(paths: int = 10000, dt: float = 1e-4, M: int = 4096, seed: int = 0,
                   nodes: Optional[np.ndarray] = None, lam: complex = 10j, kappa=(1.0, 10.0)) -> KappaProblem:
    """Sec. 4.1: Omega = [-1, 1]^2, kappa 1 (y < 0) and 10 (y >= 0),
    div(kappa grad u) = lambda u with lambda = 10 i, i.e. the Eq. (9) form
    with killing rate lambda / 2 on both sides; g = the exact solution.
    Default node: (0.6, 0.6), the point of Table 1."""
    walls = (-1.0, 1.0, -1.0, 1.0)
    g = tables_from_function(lambda yy, zz: kappa_model_field(yy, zz, lam, kappa), walls, M)
    if nodes is None:
        nodes = np.array([[0.6, 0.6]])
    n = nodes.shape[0]
    return KappaProblem(*walls, y_if=0.0, kappa=tuple(kappa), lam=(lam / 2.0, lam / 2.0), g=g, nodes=nodes,
                        path_begin=np.zeros(n, np.uint32), path_count=np.full(n, paths, np.uint32),
                        dt=dt, seed=seed, name="kappa_analytic")


def kappa_analytic_grid(n: int = 51, paths: int = 10000, dt: float = 1e-4, seed: int = 0, M: int = 4096,
                        lam: complex = 10j, kappa=(1.0, 10.0)) -> KappaProblem:
    """Sec. 4.1 at every interior point of the uniform n x n mesh of
    [-1, 1]^2 (the paper: 51 x 51 points, N = 10000 paths per point);
    nodes y fastest."""
    y = np.linspace(-1.0, 1.0, n)[1:-1]
    yy, zz = np.meshgrid(y, y)
    nodes = np.stack([yy.ravel(), zz.ravel()], axis=1)
    return kappa_analytic(paths=paths, dt=dt, M=M, seed=seed, nodes=nodes, lam=lam, kappa=kappa).replace(
        name=f"kappa_analytic_grid_{n}x{n}")
