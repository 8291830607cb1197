"""Pointwise TE responses (apparent resistivity and phase) from the field at
three points per site: the library's host arithmetic against Eqs. 2-3 written
out in numpy, and against exact 1-D fields (a uniform half-space: rho_a =
1/sigma, phase 45 degrees; a half-space under air; two layers under air),
with and without the correction for a jump of sigma between the points.
CPU only."""
import ctypes as C

import numpy as np
import pytest

import closed_forms as CF
from paper_1603_09311_amd import sdd
from paper_1603_09311_amd import workloads as W


def test_matches_equations_on_random_fields():
    rng = np.random.default_rng(5)
    n = 200
    e = [rng.normal(size=n) + 1j * rng.normal(size=n) for _ in range(3)]
    h, L, f = 0.013, 734.0, 3.7
    rho, phi = sdd.mt_te_response(*e, h, L, f)
    rho_x, phi_x = CF.mt_te_response(*e, h, L, f)
    assert np.allclose(rho, rho_x, rtol=1e-13, atol=0)
    assert np.allclose(phi, phi_x, rtol=0, atol=1e-11)


@pytest.mark.parametrize("sigma,freq", [(0.01, 10.0), (0.1, 1.0), (2.0, 100.0)])
def test_uniform_half_space_exact(sigma, freq):
    """Inside a uniform conductor the centred difference of exp(-k z) has a
    relative error (k h)^2 / 6: rho_a = 1/sigma and 45 degrees to that order."""
    L, h = 1000.0, 0.002
    z = 0.5
    e = [CF.halfspace_field(sigma, freq, (z + d) * L) for d in (-h, 0.0, h)]
    rho, phi = sdd.mt_te_response(*[np.atleast_1d(x) for x in e], h, L, freq)
    k = abs(np.sqrt(2j * np.pi * freq * CF.MU0 * sigma)) * h * L
    assert rho[0] == pytest.approx(1.0 / sigma, rel=max(1e-9, k ** 2))
    assert phi[0] == pytest.approx(45.0, abs=max(1e-7, np.degrees(k ** 2)))


def test_surface_under_air_first_order():
    """At the surface the field is linear above and exp(-k z) below; its
    second derivative jumps, so the centred difference is first order in
    k h: rho_a and phase within a few k h of the half-space values."""
    regions = [W.Region(W.HALF_Z_LT, (0.0,), 0.0)]
    tops, sig = W.column_layers(regions, 0.01, 0.0, -5.0)
    f, L, h = 10.0, 1000.0, 0.01
    al = W._alpha_of(np.asarray(sig), f, L, 0.0)
    e = W.layered_1d(np.asarray(tops), al, np.array([-h, 0.0, h]))
    rho, phi = sdd.mt_te_response(*[np.atleast_1d(x) for x in e], h, L, f)
    kh = abs(np.sqrt(2j * np.pi * f * CF.MU0 * 0.01)) * h * L
    assert abs(rho[0] / 100.0 - 1.0) < 2 * kh
    assert abs(phi[0] - 45.0) < np.degrees(2 * kh)


def _column(tops, sigmas, f, L, z):
    al = W._alpha_of(np.asarray(sigmas, dtype=np.float64), f, L, 0.0)
    return W.layered_1d(np.asarray(tops, dtype=np.float64), al, np.atleast_1d(np.asarray(z, dtype=np.float64)))


def test_jump_matches_equations_and_zero_jump_is_plain():
    rng = np.random.default_rng(6)
    n = 200
    e = [rng.normal(size=n) + 1j * rng.normal(size=n) for _ in range(3)]
    h, L, f, sj = 0.013, 734.0, 3.7, 0.37
    rho, phi = sdd.mt_te_response(*e, h, L, f, sigma_jump=sj)
    rho_x, phi_x = CF.mt_te_response_jump(*e, h, L, f, sj)
    assert np.allclose(rho, rho_x, rtol=1e-12, atol=0)
    assert np.allclose(phi, phi_x, rtol=0, atol=1e-10)
    # sigma_jump = 0 through the jump entry point: the plain results bit for bit
    arrs = [np.ascontiguousarray(np.stack([x.real, x.imag], axis=-1)) for x in e]
    ptr = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))  # noqa: E731
    r0, p0 = np.zeros(n), np.zeros(n)
    assert sdd.lib().sdd_mt_te_response_jump(n, *[ptr(a) for a in arrs], h, L, f, 0.0, ptr(r0), ptr(p0)) == 0
    r1, p1 = sdd.mt_te_response(*e, h, L, f)
    assert np.array_equal(r0, r1) and np.array_equal(p0, p1)
    with pytest.raises(sdd.SddError):
        sdd.mt_te_response(*e, h, L, f, sigma_jump=float("nan"))


@pytest.mark.parametrize("h", [0.1, 0.2, 0.4])
def test_jump_at_surface_is_second_order(h):
    """Half-space (0.01 S/m, 10 Hz) under air, site on the surface: with the
    jump term removed rho_a and phase are within (k h)^2 / 6 of 100 ohm m and
    45 degrees (measured: -0.13% and -0.57 degrees at h = 400 m); without it
    the first-order error is several times that bound."""
    f, L = 10.0, 1000.0
    e = _column([-5.0, 0.0], [0.0, 0.01], f, L, [-h, 0.0, h])
    kh = abs(np.sqrt(2j * np.pi * f * CF.MU0 * 0.01)) * h * L
    rho, phi = sdd.mt_te_response(*[np.atleast_1d(x) for x in e], h, L, f, sigma_jump=0.01)
    assert abs(rho[0] / 100.0 - 1.0) < kh ** 2 / 6
    assert abs(np.radians(phi[0] - 45.0)) < kh ** 2 / 6
    rho_p, phi_p = sdd.mt_te_response(*[np.atleast_1d(x) for x in e], h, L, f)
    assert abs(rho_p[0] / 100.0 - 1.0) > 3 * kh ** 2 / 6
    # the correction's sign and size: a jump taken with the wrong sign or
    # twice its size misses the bound as well
    for sj in (-0.01, 0.02):
        r, _ = sdd.mt_te_response(*[np.atleast_1d(x) for x in e], h, L, f, sigma_jump=sj)
        assert abs(r[0] / 100.0 - 1.0) > 3 * kh ** 2 / 6


def test_jump_between_two_layers():
    """Air, 0.1 S/m to 1 km, then 1 S/m (1 Hz); a site on the 1 km interface:
    the jump-corrected difference is second order (error under (k h)^2 / 6 of
    the 1 S/m layer against the exact derivative, which is continuous), the
    plain one first order."""
    f, L, h, zs = 1.0, 1000.0, 0.05, 1.0
    tops, sig = [-5.0, 0.0, zs], [0.0, 0.1, 1.0]
    e = _column(tops, sig, f, L, [zs - h, zs, zs + h])
    eps = 1e-6
    d_exact = (_column(tops, sig, f, L, zs)[0] - _column(tops, sig, f, L, zs - eps)[0]) / eps   # from above
    e0 = e[1]
    rho_x, phi_x = sdd.mt_te_response(np.atleast_1d(e0 - h * d_exact), np.atleast_1d(e0),
                                      np.atleast_1d(e0 + h * d_exact), h, L, f)
    kh = abs(np.sqrt(2j * np.pi * f * CF.MU0 * 1.0)) * h * L
    rho, phi = sdd.mt_te_response(*[np.atleast_1d(x) for x in e], h, L, f, sigma_jump=0.9)
    assert abs(rho[0] / rho_x[0] - 1.0) < kh ** 2 / 6
    assert abs(np.radians(phi[0] - phi_x[0])) < kh ** 2 / 6
    rho_p, _ = sdd.mt_te_response(*[np.atleast_1d(x) for x in e], h, L, f)
    assert abs(rho_p[0] / rho_x[0] - 1.0) > 3 * kh ** 2 / 6


def test_rejects_bad_arguments():
    e = np.ones(3, dtype=complex)
    for h, L, f in ((0.0, 1.0, 1.0), (1.0, -1.0, 1.0), (1.0, 1.0, 0.0)):
        with pytest.raises(sdd.SddError) as ex:
            sdd.mt_te_response(e, e, e, h, L, f)
        assert ex.value.status == sdd.SDD_E_INVALID
    rho, phi = sdd.mt_te_response(e, e, e, 0.1, 1.0, 1.0)   # zero difference
    assert np.all(np.isinf(rho)) and np.all(np.isnan(phi))


def test_commemi_points_share_streams():
    ps = W.commemi_te_points(paths=8, M=256)
    assert [p.n_nodes for p in ps] == [5, 5, 5]
    assert all(p.seed == ps[0].seed and p.stream == ps[0].stream for p in ps)
    assert np.allclose(ps[2].nodes[:, 1] - ps[0].nodes[:, 1], 0.02)
    assert np.array_equal(ps[0].nodes[:, 0], ps[1].nodes[:, 0])
