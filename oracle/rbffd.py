"""Test infrastructure: plain numpy/scipy RBF-FD sub-domain solver, written
from Sec. 3.2 of the paper, used only to check the library's host solver.

For each interior node x0 of a rectangular grid the stencil is x0 and its 8
grid neighbours; the weights w of an operator L solve A w = b with
A_kl = phi(|x_k - x_l|), b_k = (L phi(|x - x_k|))(x0), phi the multiquadric
sqrt(1 + (eps r)^2).  Separate weights for d2/dy2 and d2/dz2; the rows of
(D_yy + D_zz - i alpha I) E = 0 over the interior with the boundary values
moved to the right-hand side give a sparse system solved by scipy.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def phi(eps, r2):
    return np.sqrt(1.0 + eps * eps * r2)


def phi_yy(eps, dy, dz):
    """Second derivative in the first coordinate of sqrt(1 + eps^2 (dy^2 + dz^2))."""
    q = 1.0 + eps * eps * (dy * dy + dz * dz)
    return eps * eps / np.sqrt(q) - eps ** 4 * dy * dy / q ** 1.5


def stencil(y, z, i, j):
    pts = [(y[i + di], z[j + dj]) for dj in (-1, 0, 1) for di in (-1, 0, 1)]
    return np.array(pts)


def weights(y, z, eps):
    """((nz-2)(ny-2), 9) weights of d2/dy2 and d2/dz2, rows y fastest."""
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    wy, wz = [], []
    e0 = eps
    for j in range(1, z.size - 1):
        for i in range(1, y.size - 1):
            # eps < 0: eps h = |eps| with h the largest spacing next to the node
            if e0 < 0:
                h = max(y[i + 1] - y[i], y[i] - y[i - 1], z[j + 1] - z[j], z[j] - z[j - 1])
                eps = -e0 / h
            P = stencil(y, z, i, j)
            d = P[:, None, :] - P[None, :, :]
            A = phi(eps, (d ** 2).sum(-1))
            dy = y[i] - P[:, 0]
            dz = z[j] - P[:, 1]
            b = np.stack([phi_yy(eps, dy, dz), phi_yy(eps, dz, dy)], axis=1)
            w = np.linalg.solve(A, b)
            wy.append(w[:, 0])
            wz.append(w[:, 1])
    return np.array(wy), np.array(wz)


def solve(y, z, alpha, eps, field):
    """field: complex (nz, ny), boundary rows/columns given; alpha a scalar or
    an (nz, ny) array (the phase rate at each node); returns the solved
    field."""
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    F = np.array(field, dtype=np.complex128)
    ny, nz = y.size, z.size
    m = ny - 2
    n = m * (nz - 2)
    wy, wz = weights(y, z, eps)
    al = np.broadcast_to(np.asarray(alpha, dtype=np.float64), (nz, ny))
    rows, cols, vals = [], [], []
    rhs = np.zeros(n, dtype=np.complex128)
    for j in range(1, nz - 1):
        for i in range(1, ny - 1):
            r = (j - 1) * m + (i - 1)
            k = 0
            for dj in (-1, 0, 1):
                for di in (-1, 0, 1):
                    w = wy[r, k] + wz[r, k] - (1j * al[j, i] if (di == 0 and dj == 0) else 0.0)
                    ii, jj = i + di, j + dj
                    if ii in (0, ny - 1) or jj in (0, nz - 1):
                        rhs[r] -= w * F[jj, ii]
                    else:
                        rows.append(r)
                        cols.append((jj - 1) * m + (ii - 1))
                        vals.append(w)
                    k += 1
    M = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    x = spla.spsolve(M.tocsc(), rhs)
    F[1:-1, 1:-1] = x.reshape(nz - 2, m)
    return F
