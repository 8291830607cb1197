"""The exact expectation of the discontinuous-kappa walk's discrete scheme on a
strip, by a deterministic evaluation of its Markov chain (no Monte Carlo).

Geometry: |y| < a, interface y = 0 (side 0: y < 0, kappa_0 and lambda_0;
side 1: y >= 0), the walls z = +-Z far enough that a walk never reaches them,
and Dirichlet data g_left at y = -a and g_right at y = a.  Then the walk's
y-coordinate is a Markov chain of its own and the weight of a path is the
product of one factor per step, so the scheme's expectation u (as a function
of the starting y) solves the linear equation u = K u + b, K and b being the
expectations over one step.  One step from y (si its side, s = sqrt(kappa_si dt)),
as the scheme of Secs. 2.2 and 3.1 prescribes in the reading this build takes:

* the proposal y' = y + s N;
* the outer boundary: the wall nearer to y (the upper one iff y > 0) is left
  if y' lies beyond it (fraction d0 / (d0 - d1) of the step) or, if not, with
  the Brownian bridge's probability exp(-2 d0 d1 / (kappa dt)), at the fraction
  e / E of the step, E ~ e + Exp(1), e = 2 d0 d1 / (kappa dt) (Eq. 14); the
  weight of the exit is exp(-lambda_si fr dt) g_wall;
* otherwise the interface: reached when y' lies on the other side (at the
  fraction t_g / dt = |y| / |y' - y|) or, on the same side, with the bridge's
  probability exp(-2 |y| |y'| / (kappa dt)) at t_g = dt e / E; not reached:
  the walk moves to y' with the factor exp(-lambda_si dt);
* reached: with p_i = kappa_si / (kappa_0 + kappa_1) the walk resumes on its
  own side i, else on the other side j, at a uniform point of the disc of
  radius h = s touching the interface from the chosen side (Eqs. 11-12); the
  step's time is split between the sides by `split` (the default is the
  reading of the build: resume on i: i gets dt - (dt - t_g) p_i / 2, j gets
  (dt - t_g) p_i / 2; resume on j: i gets t_g + (dt - t_g) p_j / 2, j gets
  (dt - t_g)(2 - p_j) / 2).

u is piecewise linear on a grid of each side (the scheme's u jumps at the
interface, the step size changing there); the one-step expectations are
Gauss-Legendre sums over the proposal between grid nodes, Gauss-Laguerre
sums over the bridges' exponential variables and Gauss-Chebyshev sums over
the disc's y-marginal (2 / (pi h^2)) sqrt(h^2 - x^2).  Test infrastructure:
it computes no part of the walk the library runs."""
import math

import numpy as np

_XL, _WL = np.polynomial.laguerre.laggauss(40)      # int_0^inf e^-x f(x) dx
_XG, _WG = np.polynomial.legendre.leggauss(6)       # per sub-interval


def split_reading(dt, tg, pi_, pj, resume_own):
    """Time of an interface step on (own side, other side)."""
    if resume_own:
        return dt - 0.5 * (dt - tg) * pi_, 0.5 * (dt - tg) * pi_
    return tg + 0.5 * (dt - tg) * pj, 0.5 * (dt - tg) * (2.0 - pj)


class StripChain:
    def __init__(self, a, kappa, lam, g_left, g_right, dt, n_side=600, split=split_reading, swap_p=False,
                 own_radius_each_side=False):
        """swap_p and own_radius_each_side evaluate two other readings of
        Eqs. 11-12 (for comparison): the resume probabilities exchanged, and
        each disc with the radius sqrt(kappa dt) of its own side."""
        self.a, self.kappa, self.lam, self.dt = float(a), tuple(map(float, kappa)), tuple(map(complex, lam)), float(dt)
        self.gl, self.gr = complex(g_left), complex(g_right)
        self.split = split
        self.swap_p, self.own_radius = swap_p, own_radius_each_side
        # grid: side 0 nodes in [-a, 0], side 1 in [0, a]; unknowns at every node
        # (the end nodes carry values only through the interpolation)
        self.y0 = np.linspace(-a, 0.0, n_side + 1)
        self.y1 = np.linspace(0.0, a, n_side + 1)
        self.n = 2 * (n_side + 1)

    # ------------------------------------------------------------------
    # interpolation: sum_i w_i u(x_i) as a row of weights on the grid values
    # (points x inside (-a, a); piecewise linear on each side's grid)
    def _interp(self, x, w):
        x = np.asarray(x, dtype=np.float64)
        w = np.asarray(w)
        row = np.zeros(self.n, dtype=np.complex128)
        m = self.y0.size
        for side, grid, off in ((0, self.y0, 0), (1, self.y1, m)):
            sel = (x < 0.0) if side == 0 else (x >= 0.0)
            if not np.any(sel):
                continue
            xs, ws = x[sel], w[sel]
            k = np.clip(np.searchsorted(grid, xs, side="right") - 1, 0, m - 2)
            t = (xs - grid[k]) / (grid[k + 1] - grid[k])
            for part, wt in ((off + k, ws * (1.0 - t)), (off + k + 1, ws * t)):
                row += np.bincount(part, weights=wt.real, minlength=self.n)
                if np.iscomplexobj(wt):
                    row += 1j * np.bincount(part, weights=wt.imag, minlength=self.n)
        return row

    def _disc_rows(self, centre, h, nq=64):
        # y-marginal of a uniform point of the disc: (2/(pi h^2)) sqrt(h^2 - x^2)
        # on [-h, h]; Gauss-Chebyshev of the second kind
        j = np.arange(1, nq + 1)
        th = j * math.pi / (nq + 1)
        x = h * np.cos(th)
        w = (2.0 / (nq + 1)) * np.sin(th) ** 2
        pts = centre + x
        inside = (pts > -self.a) & (pts < self.a)
        row = self._interp(pts[inside], w[inside])
        bnd = np.sum(w[~inside & (pts <= -self.a)]) * self.gl + np.sum(w[~inside & (pts >= self.a)]) * self.gr
        return row, bnd

    # ------------------------------------------------------------------
    def _row(self, y):
        """(row of K, entry of b) for a walk starting at y."""
        a, dt = self.a, self.dt
        si = 0 if y < 0.0 else 1
        sj = 1 - si
        ki, kj = self.kappa[si], self.kappa[sj]
        li, lj = self.lam[si], self.lam[sj]
        s = math.sqrt(ki * dt)
        upper = y > 0.0
        d0 = (a - y) if upper else (y + a)
        gw = self.gr if upper else self.gl
        # proposals: Gauss-Legendre on sub-intervals of [y - 9 s, y + 9 s]
        # split at the walls, the interface and the grid nodes near y
        lo, hi = y - 9.0 * s, y + 9.0 * s
        cuts = [lo, hi, -a, a, 0.0] + list(np.linspace(lo, hi, 73))   # sub-intervals of at most s / 4
        for grid in (self.y0, self.y1):
            cuts.extend(grid[(grid > lo) & (grid < hi)])
        cuts = np.unique(np.clip(np.asarray(cuts), lo, hi))
        L, R = cuts[:-1], cuts[1:]
        yn = (0.5 * (R - L))[:, None] * _XG[None, :] + (0.5 * (R + L))[:, None]
        wq = (0.5 * (R - L))[:, None] * _WG[None, :]
        yn, wq = yn.ravel(), wq.ravel()
        phi = np.exp(-0.5 * ((yn - y) / s) ** 2) / (s * math.sqrt(2.0 * math.pi))
        wq = wq * phi
        row = np.zeros(self.n, dtype=np.complex128)
        b = 0.0 + 0.0j
        d1 = (a - yn) if upper else (yn + a)
        cross = d1 <= 0.0
        # crossings of the nearer wall
        fr = d0 / (d0 - d1[cross])
        b += np.sum(wq[cross] * np.exp(-li * fr * dt)) * gw
        # the far wall is never within 9 s (7 s < a is required)
        keep = ~cross
        yn, wq, d1 = yn[keep], wq[keep], d1[keep]
        e = 2.0 * d0 * d1 / (ki * dt)
        pb = np.exp(-e)
        # bridge exits: fr = e / (e + x), x ~ Exp(1)
        fb = e[:, None] / (e[:, None] + _XL[None, :])
        eb = np.exp(-li * fb * dt) @ _WL
        b += np.sum(wq * pb * eb) * gw
        wq = wq * (1.0 - pb)
        # the interface
        sn = np.where(yn < 0.0, 0, 1)
        di = abs(y)
        h = s
        hj = math.sqrt(kj * dt) if self.own_radius else h
        pi_ = (kj if self.swap_p else ki) / (ki + kj)
        pj = 1.0 - pi_
        towards = 1.0 if si == 0 else -1.0
        own_row, own_b = self._disc_rows(-towards * h, h)
        oth_row, oth_b = self._disc_rows(towards * hj, hj)

        def resume(tg):
            """Expected factor of each resume side for interface times tg (array)."""
            ti, tj = self.split(dt, tg, pi_, pj, True)
            fo = pi_ * np.exp(-li * ti - lj * tj)
            ti, tj = self.split(dt, tg, pi_, pj, False)
            fx = pj * np.exp(-li * ti - lj * tj)
            return fo, fx

        crossed = sn != si
        if np.any(crossed):
            tg = dt * di / np.abs(yn[crossed] - y)
            fo, fx = resume(tg)
            co, cx = np.sum(wq[crossed] * fo), np.sum(wq[crossed] * fx)
            row += co * own_row + cx * oth_row
            b += co * own_b + cx * oth_b
        same = ~crossed
        ys, ws = yn[same], wq[same]
        er = 2.0 * di * np.abs(ys) / (ki * dt)
        pr = np.exp(-er)
        # not reached: move to y'
        row += self._interp(ys, ws * (1.0 - pr) * np.exp(-li * dt))
        # reached: tg = dt er / (er + x), x ~ Exp(1)
        tg = dt * er[:, None] / (er[:, None] + _XL[None, :])
        fo, fx = resume(tg)
        co = np.sum(ws * pr * (fo @ _WL))
        cx = np.sum(ws * pr * (fx @ _WL))
        row += co * own_row + cx * oth_row
        b += co * own_b + cx * oth_b
        return row, b

    def solve(self):
        ys = np.concatenate([self.y0, self.y1])
        # the end nodes -a and a are walls: a start there is not a walk; give
        # them the wall values so that interpolation next to them is consistent
        K = np.zeros((self.n, self.n), dtype=np.complex128)
        bvec = np.zeros(self.n, dtype=np.complex128)
        m = self.y0.size
        for k, y in enumerate(ys):
            if k == 0:
                K[k, :] = 0.0
                bvec[k] = self.gl
                continue
            if k == self.n - 1:
                K[k, :] = 0.0
                bvec[k] = self.gr
                continue
            if k == m - 1:
                # the side-0 node at 0 stands for y -> 0-: a start just left of the interface
                y = -1e-12 * self.a
            K[k, :], bvec[k] = self._row(y)
        self.u = np.linalg.solve(np.eye(self.n) - K, bvec)
        return self

    def value(self, y):
        return complex(self._interp(np.array([y]), np.array([1.0])) @ self.u)
