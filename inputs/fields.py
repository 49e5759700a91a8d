"""Initial velocity fields and seeded random test data.

All functions take physical coordinates ``x, y`` (NumPy arrays of any matching
shape) and return the two velocity components.  They are plain closed forms of
the synthetic workloads; nothing here discretises anything.
"""
import numpy as np

TWO_PI = 2.0 * np.pi


def taylor_green_2d(x, y, t=0.0, nu=0.0):
    """Taylor-Green vortex on the unit torus, an exact Navier-Stokes solution.

    u = (sin 2pi x cos 2pi y, -cos 2pi x sin 2pi y) * exp(-8 pi^2 nu t);
    its pressure is (cos 4pi x + cos 4pi y)/4 * exp(-16 pi^2 nu t).
    """
    d = np.exp(-2.0 * TWO_PI ** 2 * nu * t)
    u1 = np.sin(TWO_PI * x) * np.cos(TWO_PI * y) * d
    u2 = -np.cos(TWO_PI * x) * np.sin(TWO_PI * y) * d
    return u1, u2


def double_shear_layer(x, y, sharpness=80.0, delta=0.05):
    """Double shear layer on the unit torus (exactly divergence free).

    u1 = tanh(s (y - 1/4)) for y <= 1/2, tanh(s (3/4 - y)) for y > 1/2;
    u2 = delta sin(2 pi x).
    """
    y = np.asarray(y, dtype=float)
    x = np.asarray(x, dtype=float)
    yy = np.mod(y, 1.0)
    u1 = np.where(yy <= 0.5, np.tanh(sharpness * (yy - 0.25)), np.tanh(sharpness * (0.75 - yy)))
    u2 = delta * np.sin(TWO_PI * x)
    return u1, u2


def channel_shear_layer(x, y, sharpness=80.0, delta=0.05):
    """Double shear layer in the channel [0, 1) x [0, 1] with walls at y = 0 and 1:
    exactly divergence free and tangent to the walls.

    u1 = tanh profile of ``double_shear_layer`` + (delta/2) cos(2 pi x) sin(2 pi y);
    u2 = delta sin(2 pi x) sin^2(pi y), which vanishes on both walls.
    """
    x, y = np.asarray(x) * 1.0, np.asarray(y) * 1.0  # complex arguments pass through
    base = np.where(np.real(y) <= 0.5, np.tanh(sharpness * (y - 0.25)), np.tanh(sharpness * (0.75 - y)))
    u1 = base + 0.5 * delta * np.cos(TWO_PI * x) * np.sin(TWO_PI * y)
    u2 = delta * np.sin(TWO_PI * x) * np.sin(np.pi * y) ** 2
    return u1, u2


class RandomStreamField:
    """u0 = (d psi/dy, -d psi/dx) for a seeded random trigonometric stream function.

    psi = sum_k a_k cos(2 pi k.x) + b_k sin(2 pi k.x) over the half plane of
    integer wave vectors 0 < |k| <= kmax, a, b ~ N(0, 1) from
    ``numpy.random.default_rng(seed)``; the field is scaled so that its L2 norm
    over the unit torus is exactly ``norm``.
    """

    def __init__(self, seed=0, kmax=8, norm=1.0):
        ks = []
        for k1 in range(0, kmax + 1):
            for k2 in range(-kmax, kmax + 1):
                if k1 == 0 and k2 <= 0:
                    continue
                if k1 * k1 + k2 * k2 <= kmax * kmax:
                    ks.append((k1, k2))
        self.k = np.array(ks, dtype=float)
        rng = np.random.default_rng(seed)
        self.a = rng.standard_normal(len(ks))
        self.b = rng.standard_normal(len(ks))
        k2sum = (self.k ** 2).sum(axis=1)
        energy = (TWO_PI ** 2 * k2sum * (self.a ** 2 + self.b ** 2) / 2.0).sum()
        self.scale = norm / np.sqrt(energy)

    def __call__(self, x, y):
        x = np.asarray(x, dtype=float)
        y = np.asarray(y, dtype=float)
        u1 = np.zeros(np.broadcast(x, y).shape)
        u2 = np.zeros_like(u1)
        for (k1, k2), a, b in zip(self.k, self.a, self.b):
            th = TWO_PI * (k1 * x + k2 * y)
            amp = TWO_PI * (-a * np.sin(th) + b * np.cos(th))
            u1 += amp * k2
            u2 -= amp * k1
        return self.scale * u1, self.scale * u2


def n_monomials(k):
    return (k + 1) * (k + 2) // 2


def random_broken_poly(T, k, seed=0):
    """Seeded coefficients c[T, 2, n] of a random broken vector polynomial of degree k.

    The field on element t is sum_a c[t, comp, a] xi^p eta^q in the element's
    reference coordinates (see ``eval_broken_poly`` for the monomial order).
    """
    return np.random.default_rng(seed).standard_normal((T, 2, n_monomials(k)))


def eval_broken_poly(coef, ref_pts):
    """Evaluate the field of ``random_broken_poly`` at reference points.

    ref_pts[P, 2] are (xi, eta) with x = v0 + xi (v1 - v0) + eta (v2 - v0);
    monomials are ordered by total degree d = 0..k, then q = 0..d: xi^(d-q) eta^q.
    Returns values[T, 2, P].
    """
    n = coef.shape[-1]
    k = int(round((np.sqrt(8 * n + 1) - 3) / 2))
    xi = ref_pts[:, 0]
    eta = ref_pts[:, 1]
    mono = []
    for d in range(k + 1):
        for q in range(d + 1):
            mono.append(xi ** (d - q) * eta ** q)
    mono = np.array(mono)  # [n, P]
    return np.einsum("tca,ap->tcp", coef, mono)


def taylor_green_3d(x, y, z):
    """Three-dimensional Taylor-Green vortex on the unit torus (divergence free):
    u = (sin 2pi x cos 2pi y cos 2pi z, -cos 2pi x sin 2pi y cos 2pi z, 0)."""
    cz = np.cos(TWO_PI * z)
    u1 = np.sin(TWO_PI * x) * np.cos(TWO_PI * y) * cz
    u2 = -np.cos(TWO_PI * x) * np.sin(TWO_PI * y) * cz
    return u1, u2, np.zeros_like(u1)


def abc_flow(x, y, z, t=0.0, nu=0.0, a=1.0, b=0.7, c=0.4):
    """Arnold-Beltrami-Childress flow on the unit torus, an exact Navier-Stokes solution:
    u = (a sin 2pi z + c cos 2pi y, b sin 2pi x + a cos 2pi z, c sin 2pi y + b cos 2pi x)
    * exp(-4 pi^2 nu t).  curl u = 2 pi u, so the convective term is a gradient that the
    pressure balances, and the viscous term decays the field."""
    d = np.exp(-(TWO_PI ** 2) * nu * t)
    u1 = (a * np.sin(TWO_PI * z) + c * np.cos(TWO_PI * y)) * d
    u2 = (b * np.sin(TWO_PI * x) + a * np.cos(TWO_PI * z)) * d
    u3 = (c * np.sin(TWO_PI * y) + b * np.cos(TWO_PI * x)) * d
    return u1, u2, u3


class RandomVectorPotentialField:
    """u0 = curl A for a seeded random trigonometric vector potential on the unit torus:
    A = sum_k a_k cos(2 pi k.x) + b_k sin(2 pi k.x) over integer wave vectors 0 < |k| <= kmax
    in a half space, a_k, b_k in R^3 ~ N(0, 1) from ``numpy.random.default_rng(seed)``,
    scaled to unit L2 norm over the torus."""

    def __init__(self, seed=0, kmax=3, norm=1.0):
        ks = []
        for k1 in range(-kmax, kmax + 1):
            for k2 in range(-kmax, kmax + 1):
                for k3 in range(-kmax, kmax + 1):
                    if (k1, k2, k3) <= (0, 0, 0):
                        continue
                    if k1 * k1 + k2 * k2 + k3 * k3 <= kmax * kmax:
                        ks.append((k1, k2, k3))
        self.k = np.array(ks, dtype=float)
        rng = np.random.default_rng(seed)
        self.a = rng.standard_normal((len(ks), 3))
        self.b = rng.standard_normal((len(ks), 3))
        # curl of a cos(th) is -2pi sin(th) k x a, of b sin(th) 2pi cos(th) k x b: mean square
        # of each term is (2 pi)^2 |k x a|^2 / 2
        ka = np.cross(self.k, self.a)
        kb = np.cross(self.k, self.b)
        energy = (TWO_PI ** 2 * ((ka ** 2).sum(1) + (kb ** 2).sum(1)) / 2.0).sum()
        self.scale = norm / np.sqrt(energy)

    def __call__(self, x, y, z):
        x, y, z = (np.asarray(v, dtype=float) for v in (x, y, z))
        u = np.zeros((3,) + np.broadcast(x, y, z).shape)
        for kv, a, b in zip(self.k, self.a, self.b):
            th = TWO_PI * (kv[0] * x + kv[1] * y + kv[2] * z)
            ka = np.cross(kv, a)
            kb = np.cross(kv, b)
            for c in range(3):
                u[c] += TWO_PI * (-np.sin(th) * ka[c] + np.cos(th) * kb[c])
        return tuple(self.scale * u[c] for c in range(3))


def n_monomials_3d(k):
    return (k + 1) * (k + 2) * (k + 3) // 6


def random_broken_poly_3d(T, k, seed=0):
    """Seeded coefficients c[T, 3, n] of a random broken vector polynomial of degree k on
    tetrahedra (monomial order of ``eval_broken_poly_3d``)."""
    return np.random.default_rng(seed).standard_normal((T, 3, n_monomials_3d(k)))


def eval_broken_poly_3d(coef, ref_pts):
    """Evaluate ``random_broken_poly_3d`` data at reference points ref_pts[P, 3] = (xi, eta,
    zeta) with x = v0 + xi (v1 - v0) + eta (v2 - v0) + zeta (v3 - v0); monomials
    xi^p eta^q zeta^r ordered by total degree d, then q + r, then r.  Returns [T, 3, P]."""
    n = coef.shape[-1]
    k = 0
    while n_monomials_3d(k) < n:
        k += 1
    xi, eta, zeta = ref_pts[:, 0], ref_pts[:, 1], ref_pts[:, 2]
    mono = []
    for d in range(k + 1):
        for qr in range(d + 1):
            for r in range(qr + 1):
                mono.append(xi ** (d - qr) * eta ** (qr - r) * zeta ** r)
    return np.einsum("tca,ap->tcp", coef, np.array(mono))
