"""A second, pure-Python implementation of one realisation of the walk, for
tiny brute-force comparisons with the C oracle (path by path, bit for bit).

Written from the paper (Sec. 3.1, Eqs. 13-14 and the MC estimator), not from
the oracle's source: Philox4x32-10 from its published definition, Box-Muller,
the nearer-wall Brownian-bridge exit test, right-point occupation rule.
Pure-Python loops: only for a handful of short paths.
"""
import math

MASK = 0xFFFFFFFF


def philox(ctr, key):
    x = list(ctr)
    k0, k1 = key
    for _ in range(10):
        a = 0xD2511F53 * x[0]
        b = 0xCD9E8D57 * x[2]
        x = [((b >> 32) ^ x[1] ^ k0) & MASK, b & MASK, ((a >> 32) ^ x[3] ^ k1) & MASK, a & MASK]
        k0 = (k0 + 0x9E3779B9) & MASK
        k1 = (k1 + 0xBB67AE85) & MASK
    return x


def unif(w):
    return (w + 0.5) * 2.0 ** -32


def inside(kind, v, y, z):
    if kind == 0:
        return z < v[0]
    if kind == 1:
        return y < v[0]
    if kind == 2:
        return v[0] <= y < v[1] and v[2] <= z < v[3]
    e = [(v[2] - v[0]) * (z - v[1]) - (v[3] - v[1]) * (y - v[0]),
         (v[4] - v[2]) * (z - v[3]) - (v[5] - v[3]) * (y - v[2]),
         (v[0] - v[4]) * (z - v[5]) - (v[1] - v[5]) * (y - v[4])]
    return all(t >= 0 for t in e) or all(t <= 0 for t in e)


def walk(p, j, path):
    """Returns dict(w_re, w_im, S, tau, exit_t, steps, wall)."""
    key = (p.seed & MASK, p.seed >> 32)
    alph = list(p.alphas())
    c = [a * p.dt / 2.0 for a in alph]

    def reg(y, z):
        for r, R in enumerate(p.regions):
            if inside(R.kind, R.param6(), y, z):
                return r
        return len(p.regions)

    s = math.sqrt(p.dt)
    y, z = float(p.nodes[j, 0]), float(p.nodes[j, 1])
    S = 0.0
    lo = (p.y_lo, p.z_lo)
    hi = (p.y_hi, p.z_hi)
    n = 0
    while n < p.max_steps:
        w = philox((n >> 1, path, j, 2 * p.stream), key)
        a, b = (w[0], w[1]) if n % 2 == 0 else (w[2], w[3])
        r = math.sqrt(-2.0 * math.log(unif(a)))
        th = 6.283185307179586 * unif(b)
        yn = y + s * (r * math.cos(th))
        zn = z + s * (r * math.sin(th))
        ub = philox((n, path, j, 2 * p.stream + 1), key)
        hits = []
        for ax, (x0, x1) in enumerate(((y, yn), (z, zn))):
            dlo, dhi = x0 - lo[ax], hi[ax] - x0
            up = not (dlo <= dhi)
            d0 = dhi if up else dlo
            d1 = (hi[ax] - x1) if up else (x1 - lo[ax])
            if d1 <= 0.0:
                hits.append((d0 / (d0 - d1), ax, up))
            else:
                q = (2.0 * d0) * d1
                L = -math.log(unif(ub[ax]))
                if q <= p.dt * L:
                    hits.append((q / (p.dt * L), ax, up))
        if hits:
            f, ax, up = hits[0] if len(hits) == 1 or hits[0][0] <= hits[1][0] else hits[1]
            if ax == 0:
                wall = 1 if up else 3
                t = min(max(z + f * (zn - z), p.z_lo), p.z_hi)
                t0, t1 = p.z_lo, p.z_hi
            else:
                wall = 2 if up else 0
                t = min(max(y + f * (yn - y), p.y_lo), p.y_hi)
                t0, t1 = p.y_lo, p.y_hi
            S += c[reg(y, z)] * f
            M = p.g.shape[1] - 1
            h = (t1 - t0) / M
            u = (t - t0) / h
            i = min(max(int(math.floor(u)), 0), M - 1)
            lam = u - i
            g0, g1 = p.g[wall, i], p.g[wall, i + 1]
            gre = (1.0 - lam) * g0.real + lam * g1.real
            gim = (1.0 - lam) * g0.imag + lam * g1.imag
            cs, sn = math.cos(S), math.sin(S)
            return dict(w_re=gre * cs + gim * sn, w_im=gim * cs - gre * sn, S=S,
                        tau=(n + f) * p.dt, exit_t=t, steps=n + 1, wall=wall)
        S += c[reg(yn, zn)]
        y, z = yn, zn
        n += 1
    return dict(w_re=0.0, w_im=0.0, S=S, tau=-1.0, exit_t=0.0, steps=p.max_steps, wall=-1)
