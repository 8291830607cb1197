"""Stochastic domain decomposition over rectangular sub-domains (Secs. 3.1
and 3.2): the field at the grid nodes on the interfaces between sub-domains
comes from the walks (the persistent walker through the C ABI), then every
sub-domain is solved by RBF-FD (the library's host solver) with those values
and the outer Dirichlet data as its boundary values.

A sub-domain is a rectangle of grid nodes (i0..i1, j0..j1) with one phase
rate alpha; rectangles share their edges (the interfaces).  This module only
routes values between the two library stages.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np

from . import sdd


@dataclasses.dataclass
class SubDomain:
    i0: int
    i1: int
    j0: int
    j1: int
    alpha: float


def interface_nodes(ny: int, nz: int, subs: Sequence[SubDomain]) -> np.ndarray:
    """(k, 2) integer (i, j) of the nodes on sub-domain edges that are not on
    the outer boundary, in a fixed order (j, then i)."""
    mark = np.zeros((nz, ny), dtype=bool)
    for s in subs:
        mark[s.j0, s.i0:s.i1 + 1] = True
        mark[s.j1, s.i0:s.i1 + 1] = True
        mark[s.j0:s.j1 + 1, s.i0] = True
        mark[s.j0:s.j1 + 1, s.i1] = True
    mark[0, :] = mark[-1, :] = False
    mark[:, 0] = mark[:, -1] = False
    jj, ii = np.nonzero(mark)
    return np.stack([ii, jj], axis=1)


def solve_subdomains(y, z, subs: Sequence[SubDomain], field: np.ndarray, eps: float) -> np.ndarray:
    """RBF-FD solve of every sub-domain; `field` (nz, ny) holds the outer
    Dirichlet values and the interface values.  Returns the completed grid."""
    F = np.array(field, dtype=np.complex128)
    for s in subs:
        part = sdd.rbffd_solve(y[s.i0:s.i1 + 1], z[s.j0:s.j1 + 1], s.alpha, eps,
                               F[s.j0:s.j1 + 1, s.i0:s.i1 + 1])
        F[s.j0 + 1:s.j1, s.i0 + 1:s.i1] = part[1:-1, 1:-1]
    return F


def decompose(ctx, p, y, z, subs: Sequence[SubDomain], outer: np.ndarray, eps: float,
              precision: Optional[int] = None) -> Tuple[np.ndarray, dict]:
    """Walk at the interface nodes (model, tables, paths, time step and
    streams of problem p, one node per interface grid node), then solve the
    sub-domains.  outer: (nz, ny) complex array whose first and last rows and
    columns are the outer Dirichlet values.  Returns the grid and the walk
    result at the interface nodes."""
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    ij = interface_nodes(y.size, z.size, subs)
    nodes = np.stack([y[ij[:, 0]], z[ij[:, 1]]], axis=1)
    paths = int(p.path_count[0])
    q = p.replace(nodes=nodes, path_begin=np.zeros(len(nodes), np.uint32),
                  path_count=np.full(len(nodes), paths, np.uint32))
    r = ctx.solve(q, precision=precision)
    F = np.array(outer, dtype=np.complex128)
    F[ij[:, 1], ij[:, 0]] = r["mean"]
    r["ij"] = ij
    return solve_subdomains(y, z, subs, F, eps), r


def graded_axis(lo: float, hi: float, h0: float, growth: float, hmax: float) -> np.ndarray:
    """Grid points from lo to hi through 0: spacing h0 at 0, growing by
    `growth` per cell up to hmax (symmetric on both sides of 0; the end cells
    absorb the remainder)."""
    def side(length):
        pts, x, h = [0.0], 0.0, h0
        while x + h < length - 0.5 * min(h, hmax):
            x += h
            pts.append(x)
            h = min(h * growth, hmax)
        pts.append(length)
        return np.array(pts)
    neg = -side(-lo)[::-1] if lo < 0 else np.array([])
    pos = side(hi) if hi > 0 else np.array([])
    return np.unique(np.concatenate([neg, pos]))
