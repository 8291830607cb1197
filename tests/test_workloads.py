"""The seeded input generators: 1-D layered boundary data against a closed
form and an independent finite-difference solve; node sets; sizes."""
import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from paper_1603_09311_amd import workloads as W


def test_delta1():
    assert abs(W.DELTA1 - 5032.92) < 0.01


def test_halfspace_closed_form():
    for alpha in (2.0, 20.0, 0.37):
        k = np.sqrt(1j * alpha)
        e0 = 1.0 / (1.0 + 6.0 * k)
        z = np.array([-6.0, -3.0, -1e-9, 0.0, 0.5, 2.0, 8.0])
        got = W.layered_1d(np.array([-6.0, 0.0]), np.array([0.0, alpha]), z)
        want = np.where(z < 0, e0 * (1 - k * z), e0 * np.exp(-k * z))
        assert np.allclose(got, want, rtol=1e-12, atol=1e-15)
    e = W.layered_1d(np.array([-6.0, 0.0]), np.array([0.0, 2.0]), np.array([0.0]))[0]
    assert abs(e - (0.0824 - 0.0706j)) < 1e-4
    e = W.layered_1d(np.array([-6.0, 0.0]), np.array([0.0, 20.0]), np.array([0.0]))[0]
    assert abs(e - (0.0263 - 0.0250j)) < 1e-4


def _fd_column(tops, al, zb, n):
    """Second-order FD for E'' = i alpha E, E(top) = 1, decaying Robin
    condition E' = -k E at z = zb; returns (z, E)."""
    z = np.linspace(tops[0], zb, n + 1)
    h = z[1] - z[0]
    a = al[np.searchsorted(tops, z, side="right") - 1]
    kb = np.sqrt(1j * al[-1])
    main = (-2.0 / h ** 2 - 1j * a).astype(np.complex128)
    A = sp.diags([np.full(n, 1 / h ** 2), main, np.full(n, 1 / h ** 2)], [-1, 0, 1], format="lil")
    rhs = np.zeros(n + 1, dtype=np.complex128)
    A[0, :] = 0
    A[0, 0] = 1.0
    rhs[0] = 1.0
    # ghost point E_{n+1} = E_{n-1} - 2 h k E_n
    A[n, n - 1] = 2 / h ** 2
    A[n, n] = -2.0 / h ** 2 - 1j * a[-1] - 2 * kb / h
    return z, spla.spsolve(A.tocsc(), rhs)


def test_layered_matches_finite_differences():
    """Air / 2 / 30 / 5 layers: FD on two fine grids converges to the transfer
    solution (first order, from the coefficient jumps); the Richardson
    extrapolation of the two agrees to 2e-6."""
    tops = np.array([-2.0, 0.0, 0.7, 1.3])
    al = np.array([0.0, 2.0, 30.0, 5.0])
    z1, e1 = _fd_column(tops, al, 6.0, 20000)
    z2, e2 = _fd_column(tops, al, 6.0, 40000)
    got = W.layered_1d(tops, al, z1)
    err1 = np.max(np.abs(got - e1))
    err2 = np.max(np.abs(got - e2[::2]))
    assert err2 < 0.6 * err1 and err1 < 2e-4
    assert np.max(np.abs(got - (2 * e2[::2] - e1))) < 2e-6


def test_continuity_across_layers():
    tops = np.array([-6.0, 0.0, 0.5, 1.5])
    al = np.array([0.0, 2.0, 200.0, 2.0])
    for zc in tops[1:]:
        e = 1e-7
        l, c, r = W.layered_1d(tops, al, np.array([zc - e, zc, zc + e]))
        assert abs(l - c) < 1e-5 and abs(r - c) < 1e-5
        dl = (c - W.layered_1d(tops, al, np.array([zc - 2e-5]))[0]) / 2e-5
        dr = (W.layered_1d(tops, al, np.array([zc + 2e-5]))[0] - c) / 2e-5
        assert abs(dl - dr) < 1e-3 * max(1.0, abs(dl))


def test_quarter_space_tables_and_nodes():
    p = W.quarter_space(paths=16, M=1024)
    assert p.nodes.shape == (512, 2) and p.g.shape == (4, 1025)
    assert np.allclose(p.g[W.WALL_TOP], 1.0)
    zs = p.z_lo + np.arange(1025) * (14.0 / 1024)
    k2, k20 = np.sqrt(2j), np.sqrt(20j)
    want_l = np.where(zs < 0, (1 - k2 * zs) / (1 + 6 * k2), np.exp(-k2 * zs) / (1 + 6 * k2))
    want_r = np.where(zs < 0, (1 - k20 * zs) / (1 + 6 * k20), np.exp(-k20 * zs) / (1 + 6 * k20))
    assert np.allclose(p.g[W.WALL_LEFT], want_l, atol=1e-13)
    assert np.allclose(p.g[W.WALL_RIGHT], want_r, atol=1e-13)
    alphas = p.alphas()
    assert np.allclose(alphas, [0.0, 2.0, 20.0])
    assert np.all((p.nodes[:, 0] > p.y_lo) & (p.nodes[:, 0] < p.y_hi))
    assert np.all((p.nodes[:, 1] > p.z_lo) & (p.nodes[:, 1] < p.z_hi))


def test_block_and_triangle_families():
    p = W.block_in_half_space(10.0, paths=64, M=256)
    assert p.nodes.shape == (1024, 2)
    assert np.allclose(p.alphas(), [0.0, 2000.0, 20.0])
    for m in range(4):
        q = W.triangle_request(m, M=256)
        assert 32 <= q.n_nodes <= 1024
        assert 4096 <= int(q.path_count[0]) <= 262144 and int(q.path_count[0]) % 64 == 0
        assert q.freq_hz in W.TRIANGLE_FREQS
        assert np.all(np.isfinite(q.g))
        assert np.all((q.nodes[:, 1] >= 0) & (q.nodes[:, 1] < 8))
    # seeded: same request twice is the same
    a, b = W.triangle_request(3, M=64), W.triangle_request(3, M=64)
    assert np.array_equal(a.nodes, b.nodes) and a.regions == b.regions
