"""Closed-form solutions that pin the walk (not from any implementation).

All on the unit square [0,1]^2 unless stated; standard Brownian motion with
generator Laplace/2, so E solves Laplace E = i alpha E (TE mode).
"""
import numpy as np


def plane_wave(alpha, z):
    """exp(-sqrt(i alpha) z): the 1-D decaying TE wave; principal root."""
    return np.exp(-np.sqrt(1j * alpha) * np.asarray(z))


def cosh_model(alpha, y, z):
    """(z + 1) cosh(sqrt(i alpha) (y - 1/2)): the analytic test model of
    Sec. 4.1 (Eq. 15b) with equal kappa on both sides, shifted to the unit
    square; Laplace u = i alpha u."""
    return (np.asarray(z) + 1.0) * np.cosh(np.sqrt(1j * alpha) * (np.asarray(y) - 0.5))


def _odd(K):
    return np.arange(1, K + 1, 2, dtype=np.float64)


def g1_const_alpha(alpha, y, z, K=801):
    """u = 1 on the boundary, Laplace u = i alpha u inside:
    u = 1 - sum_{m,n odd} 16 i alpha / (pi^2 m n (pi^2 (m^2+n^2) + i alpha))
              sin(m pi y) sin(n pi z)."""
    m = _odd(K)[:, None]
    n = _odd(K)[None, :]
    coef = 16j * alpha / (np.pi ** 2 * m * n * (np.pi ** 2 * (m ** 2 + n ** 2) + 1j * alpha))
    y = np.atleast_1d(np.asarray(y, dtype=np.float64))
    z = np.atleast_1d(np.asarray(z, dtype=np.float64))
    out = np.empty(y.shape, dtype=np.complex128)
    for i in range(y.size):
        out.flat[i] = 1.0 - np.sum(coef * np.sin(m * np.pi * y.flat[i]) * np.sin(n * np.pi * z.flat[i]))
    return out


def mean_exit_time(y, z, K=801):
    """E[tau] for standard BM leaving the unit square: (1/2) Laplace u = -1,
    u = sum_{m,n odd} 32 / (pi^4 m n (m^2 + n^2)) sin(m pi y) sin(n pi z)."""
    m = _odd(K)[:, None]
    n = _odd(K)[None, :]
    coef = 32.0 / (np.pi ** 4 * m * n * (m ** 2 + n ** 2))
    y = np.atleast_1d(np.asarray(y, dtype=np.float64))
    z = np.atleast_1d(np.asarray(z, dtype=np.float64))
    out = np.empty(y.shape)
    for i in range(y.size):
        out.flat[i] = np.sum(coef * np.sin(m * np.pi * y.flat[i]) * np.sin(n * np.pi * z.flat[i]))
    return out


def halfspace_e0(alpha, z_top):
    """Air (linear) over a uniform half-space (exp(-k z)), normalised to 1 at
    z_top < 0: E(z) = E0 exp(-k z) below 0, E0 (1 - k z) above, E0 = 1/(1 - k z_top)."""
    k = np.sqrt(1j * alpha)
    return 1.0 / (1.0 - k * z_top)


def skin_depth_m(rho_ohm_m, freq_hz):
    """Plane-wave skin depth in metres by the textbook magnetotelluric rule
    delta = 503.29 sqrt(rho / f) (rho in ohm m, f in Hz).  The constant is
    the published one, not derived here from mu0, so a pin built on it does
    not repeat the oracle's own conversion of a frequency into a phase
    rate."""
    return 503.29 * np.sqrt(rho_ohm_m / freq_hz)


def air_over_halfspace(k, z, z_top):
    """Air (alpha = 0, linear field) over a uniform half-space with wave
    number k (field exp(-k z) below z = 0), normalised to 1 at z_top < 0:
    E = E0 (1 - k z) for z < 0 and E0 exp(-k z) below, E0 = 1 / (1 - k z_top)."""
    z = np.asarray(z, dtype=np.float64)
    e0 = 1.0 / (1.0 - k * z_top)
    return np.where(z < 0.0, e0 * (1.0 - k * z), e0 * np.exp(-k * z))


def zscores(mean, exact, se_re, se_im, bias=0.0):
    """Component z-scores with a stated bias allowance subtracted first."""
    d = np.asarray(mean) - np.asarray(exact)
    zr = np.maximum(np.abs(d.real) - bias, 0.0) / np.asarray(se_re)
    zi = np.maximum(np.abs(d.imag) - bias, 0.0) / np.asarray(se_im)
    return np.concatenate([np.atleast_1d(zr), np.atleast_1d(zi)])


MU0 = 4e-7 * np.pi


def halfspace_field(sigma, freq_hz, z_m):
    """The TE field of a uniform half-space, exp(-k z), k = sqrt(i omega mu0
    sigma) (principal root), z in metres positive down."""
    k = np.sqrt(1j * 2.0 * np.pi * freq_hz * MU0 * sigma)
    return np.exp(-k * np.asarray(z_m, dtype=np.float64))


def mt_te_response(e_minus, e_mid, e_plus, h, length_unit_m, freq_hz):
    """Eqs. 2-3 of Sec. 2.1 with a centred difference: H = -(1/(i omega mu0))
    dE/dz, rho_a = |E/H|^2 / (omega mu0), phi = arg(E/H) in degrees."""
    w = 2.0 * np.pi * freq_hz
    dedz = (np.asarray(e_plus) - np.asarray(e_minus)) / (2.0 * h * length_unit_m)
    hx = -dedz / (1j * w * MU0)
    z = np.asarray(e_mid) / hx
    return np.abs(z) ** 2 / (w * MU0), np.degrees(np.angle(z))


def mt_te_response_jump(e_minus, e_mid, e_plus, h, length_unit_m, freq_hz, sigma_jump):
    """mt_te_response across a horizontal jump of sigma (below minus above)
    between the outer points: d2E/dz2 jumps by i omega mu0 sigma_jump E
    there, which puts (h L / 4) i omega mu0 sigma_jump E(z) into the centred
    difference; that term is taken out of dE/dz."""
    w = 2.0 * np.pi * freq_hz
    hm = h * length_unit_m
    e0 = np.asarray(e_mid)
    dedz = (np.asarray(e_plus) - np.asarray(e_minus)) / (2.0 * hm) - 0.25 * hm * 1j * w * MU0 * sigma_jump * e0
    hx = -dedz / (1j * w * MU0)
    z = e0 / hx
    return np.abs(z) ** 2 / (w * MU0), np.degrees(np.angle(z))


def kappa_strip(lam, kappa, a, g_left, g_right, y):
    """(1/2)(kappa u')' - lam u = 0 on -a < y < a with kappa_i, lam_i
    constant on y < 0 (i = 0) and y >= 0 (i = 1), u(-a) = g_left,
    u(a) = g_right, u and the flux kappa u' continuous at 0: on each side
    u = A_i cosh(k_i y) + B_i sinh(k_i y) / k_i, k_i = sqrt(2 lam_i / kappa_i)
    (B_i y when lam_i = 0)."""
    k = [np.sqrt(2.0 * complex(lam[i]) / kappa[i]) for i in range(2)]

    def S(kk, yy):
        return yy if kk == 0 else np.sinh(kk * yy) / kk
    M = np.array([[np.cosh(-k[0] * a), S(k[0], -a), 0, 0],
                  [0, 0, np.cosh(k[1] * a), S(k[1], a)],
                  [1, 0, -1, 0],
                  [0, kappa[0], 0, -kappa[1]]], dtype=complex)
    A0, B0, A1, B1 = np.linalg.solve(M, np.array([g_left, g_right, 0, 0], dtype=complex))
    y = np.asarray(y, dtype=np.float64)
    return np.where(y < 0, A0 * np.cosh(k[0] * y) + B0 * S(k[0], y), A1 * np.cosh(k[1] * y) + B1 * S(k[1], y))


def kappa_two_sided(lam, kappa, y, z, y_if=0.0):
    """(1/2) div(kappa grad u) - lam_i u = 0 with kappa_i, lam_i constant on
    the sides y < y_if (i = 0) and y >= y_if (i = 1): u = (z + 1) f(y) with
    f = cosh(k_i (y - y_if)) + B_i sinh(k_i (y - y_if)), k_i = sqrt(2 lam_i /
    kappa_i), B_0 = 1 and B_1 = kappa_0 k_0 / (kappa_1 k_1) (u and the flux
    kappa du/dy continuous at the interface).  lam = 0 on both sides gives the
    piecewise-linear f = 1 + (y - y_if) / kappa_i."""
    y = np.asarray(y, dtype=np.float64) - y_if
    z = np.asarray(z, dtype=np.float64)
    lam = [complex(v) for v in lam]
    if lam[0] == 0 and lam[1] == 0:
        f = np.where(y < 0, 1.0 + y / kappa[0], 1.0 + y / kappa[1]) + 0j
    else:
        k = [np.sqrt(2.0 * lam[i] / kappa[i]) for i in range(2)]
        b1 = kappa[0] * k[0] / (kappa[1] * k[1])
        f = np.where(y < 0, np.cosh(k[0] * y) + np.sinh(k[0] * y), np.cosh(k[1] * y) + b1 * np.sinh(k[1] * y))
    return (z + 1.0) * f
