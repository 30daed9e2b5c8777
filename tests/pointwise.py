"""Test-side pointwise evaluation of contracted real solid-harmonic Gaussians.

Independent of the oracle's Cartesian machinery: the angular part is evaluated
from the recursion for the regular scaled solid harmonics R^{c/s}_{l,m}
(Sec. II.F, eq. regular_scaled_harmonics_recursion) times the prefactor A_{l,m}
(eq. A), and the normalisation uses N_l (eq. N_l). Integrals are then done by
brute-force Gauss-Hermite quadrature."""
from math import factorial, pi, sqrt

import numpy as np


def regular_solid(lmax, x, y, z):
    """Rc[l][m], Rs[l][m] for 0 <= m <= l <= lmax, evaluated pointwise."""
    r2 = x * x + y * y + z * z
    Rc = [[None] * (lmax + 1) for _ in range(lmax + 1)]
    Rs = [[None] * (lmax + 1) for _ in range(lmax + 1)]
    one = np.ones_like(x)
    Rc[0][0], Rs[0][0] = one, 0 * one
    for l in range(lmax):
        Rc[l + 1][l + 1] = -(x * Rc[l][l] - y * Rs[l][l]) / (2 * l + 2)
        Rs[l + 1][l + 1] = -(y * Rc[l][l] + x * Rs[l][l]) / (2 * l + 2)
        for m in range(0, l + 1):
            prev_c = Rc[l - 1][m] if (l >= 1 and m <= l - 1) else 0 * one
            prev_s = Rs[l - 1][m] if (l >= 1 and m <= l - 1) else 0 * one
            den = (l + m + 1) * (l - m + 1)
            Rc[l + 1][m] = ((2 * l + 1) * z * Rc[l][m] - r2 * prev_c) / den
            Rs[l + 1][m] = ((2 * l + 1) * z * Rs[l][m] - r2 * prev_s) / den
    return Rc, Rs


def A_lm(l, m):
    mu = abs(m)
    return (-1) ** mu * sqrt((2 - (mu == 0)) * factorial(l + mu) * factorial(l - mu))


def real_solid(l, x, y, z):
    """S_{l,m}(r) for m = -l..l (list), m < 0 sine parts: A_{l,|m|} R^{c/s}_{l,|m|}."""
    Rc, Rs = regular_solid(l, x, y, z)
    out = []
    for m in range(-l, l + 1):
        mu = abs(m)
        out.append(A_lm(l, mu) * (Rs[l][mu] if m < 0 else Rc[l][mu]))
    return out


def norm_l(l, exps, coefs):
    Kl = sqrt((2 * l + 1) / (4 * pi))
    s = 0.0
    for a, ca in zip(exps, coefs):
        for b, cb in zip(exps, coefs):
            s += sqrt(pi) * factorial(2 * l + 2) * ca * cb / (2 ** (2 * l + 3) * factorial(l + 1)
                                                               * (a + b) ** (l + 1.5))
    return Kl / sqrt(s)


def shell_values(l, exps, coefs, center, pts):
    """phi_{l,m}(pts) for m=-l..l, shape (2l+1, npts)."""
    d = pts - np.asarray(center)[None, :]
    r2 = (d * d).sum(1)
    radial = sum(c * np.exp(-a * r2) for a, c in zip(exps, coefs))
    S = real_solid(l, d[:, 0], d[:, 1], d[:, 2])
    N = norm_l(l, exps, coefs)
    return np.array([N * s * radial for s in S])


def gh_grid(center, alpha, n):
    """3-D Gauss-Hermite nodes and weights for the weight exp(-alpha |r-center|^2)."""
    t, w = np.polynomial.hermite.hermgauss(n)
    t = t / sqrt(alpha)
    w = w / sqrt(alpha)
    X, Y, Z = np.meshgrid(t, t, t, indexing="ij")
    W = (w[:, None, None] * w[None, :, None] * w[None, None, :]).ravel()
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1) + np.asarray(center)[None, :]
    return pts, W


def potential_s(op, omega, beta, d):
    """Potential at distance d of the s Gaussian exp(-beta r^2) under the kernel O."""
    from scipy.special import erf
    d = np.maximum(d, 1e-300)
    if op == "coulomb":
        return (pi / beta) ** 1.5 * erf(sqrt(beta) * d) / d
    if op == "erf":
        g = beta * omega ** 2 / (beta + omega ** 2)
        return (pi / beta) ** 1.5 * erf(sqrt(g) * d) / d
    if op == "erfc":
        return potential_s("coulomb", omega, beta, d) - potential_s("erf", omega, beta, d)
    if op == "gauss":
        return (pi / (beta + omega)) ** 1.5 * np.exp(-beta * omega * d * d / (beta + omega))
    if op == "gcoulomb":
        # exp(-w s^2)/s = (2/sqrt(pi)) int_0^inf exp(-(t^2 + w) s^2) dt; the Gaussian convolution
        # under the integral and t = sqrt(beta + w) tan(phi), sin(phi) = u, give
        # 2 pi / (beta + w) exp(-beta w d^2 / (beta + w)) int_0^1 exp(-x u^2) du,
        # x = beta^2 d^2 / (beta + w), and int_0^1 exp(-x u^2) du = sqrt(pi) erf(sqrt x) / (2 sqrt x)
        x = beta * beta * d * d / (beta + omega)
        sx = np.sqrt(np.maximum(x, 1e-300))
        f0 = np.where(x < 1e-12, 1.0 - x / 3, sqrt(pi) * erf(sx) / (2 * sx))
        return 2 * pi / (beta + omega) * np.exp(-beta * omega * d * d / (beta + omega)) * f0
    raise ValueError(op)
