"""Seeded synthetic inputs: grids, immersed-body level sets, Dirichlet data and sources.

This module is shared by the CPU oracle tests and the GPU path.  It holds none of the
discretisation or solver arithmetic: it only produces the problem statement of the
paper's Eq. (poisson) -- grid coordinates (Sec. 2, first paragraph), a nodal level set
whose sign marks the fluid region (phi > 0) and the solid region (phi <= 0), nodal
Dirichlet data g (a smooth field whose values at boundary nodes and, interpolated, at
the interface intersections are the boundary values) and the nodal source f.

Arrays are float64 with shape (nz, ny, nx), i.e. node (i, j, k) sits at flat index
i + nx*(j + ny*k).  Coordinates are the points x_1 < ... < x_nx including both walls.

Workloads (N = interior points per direction, n = N + 2 stored points):
  uniform_sine      unit cube, uniform, no body, u = sin(pi x) sin(pi y) sin(pi z)
  sphere_exp        tanh-stretched, one sphere r=0.25 at the centre, u = exp(x+y+z)
  spheres8          tanh-stretched, 8 seeded spheres, u = sin(2 pi x) cos(pi y) exp(z)
  star_fourier      tanh-stretched, star-shaped body, f = seeded random Fourier series, g = 0
  bodies16_fourier  tanh-stretched, 8 spheres + 8 rotated ellipsoids, Fourier f, g = 0
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

PI = math.pi


# ----------------------------------------------------------------------------------------
# grids
# ----------------------------------------------------------------------------------------
def uniform_grid(n: int) -> np.ndarray:
    """n points 0 = x_1 < ... < x_n = 1, equally spaced."""
    return np.arange(n, dtype=np.float64) / (n - 1)


def tanh_grid(n: int, beta: float) -> np.ndarray:
    """Wall-clustered points x(eta) = (1 + tanh(beta (2 eta - 1)) / tanh(beta)) / 2 on [0, 1].

    beta = 0 gives the uniform grid.  Both walls are hit exactly.
    """
    if beta == 0.0:
        return uniform_grid(n)
    eta = np.arange(n, dtype=np.float64) / (n - 1)
    x = 0.5 * (1.0 + np.tanh(beta * (2.0 * eta - 1.0)) / math.tanh(beta))
    x[0], x[-1] = 0.0, 1.0
    return x


def sinh_grid(n: int, beta: float, L: float, H: float, y0: float = 0.0) -> np.ndarray:
    """Interior clustering (Eqs. p2_y, p4_y, p4_z): n points on [y0, y0 + H], densest at
    y0 + L, y(eta) = y0 + L (1 + sinh(beta (eta - s)) / sinh(beta s)) with s of Eq. p2_s,
    which makes y(1) = y0 + H.  Both ends are set exactly."""
    s = math.log((1.0 + (math.exp(beta) - 1.0) * (L / H)) / (1.0 + (math.exp(-beta) - 1.0) * (L / H))) / (2.0 * beta)
    eta = np.arange(n, dtype=np.float64) / (n - 1)
    y = y0 + L * (1.0 + np.sinh(beta * (eta - s)) / math.sinh(beta * s))
    y[0], y[-1] = y0, y0 + H
    return y


def random_grid(n: int, rng: np.random.Generator, jitter: float = 0.35) -> np.ndarray:
    """A strictly increasing irregular grid on [0,1] (spacings vary by up to +-jitter)."""
    h = 1.0 + jitter * (2.0 * rng.random(n - 1) - 1.0)
    x = np.concatenate([[0.0], np.cumsum(h)])
    x /= x[-1]
    x[-1] = 1.0
    return x


def mesh(x, y, z):
    """Broadcastable coordinate arrays of shape (nz,1,1), (1,ny,1), (1,1,nx)."""
    return (np.asarray(z)[:, None, None], np.asarray(y)[None, :, None], np.asarray(x)[None, None, :])


# ----------------------------------------------------------------------------------------
# bodies (level sets: > 0 outside = fluid, <= 0 inside = solid)
# ----------------------------------------------------------------------------------------
@dataclass
class Sphere:
    c: tuple
    r: float

    def level(self, Z, Y, X):
        return np.sqrt((X - self.c[0]) ** 2 + (Y - self.c[1]) ** 2 + (Z - self.c[2]) ** 2) - self.r

    @property
    def bound(self):
        return self.r


@dataclass
class Ellipsoid:
    c: tuple
    semi: tuple
    rot: np.ndarray  # 3x3 rotation, columns = body axes in world frame

    def level(self, Z, Y, X):
        d = [X - self.c[0], Y - self.c[1], Z - self.c[2]]
        acc = 0.0
        for a in range(3):
            q = self.rot[0, a] * d[0] + self.rot[1, a] * d[1] + self.rot[2, a] * d[2]
            acc = acc + (q / self.semi[a]) ** 2
        return (np.sqrt(acc) - 1.0) * min(self.semi)

    @property
    def bound(self):
        return max(self.semi)


@dataclass
class Star:
    c: tuple = (0.5, 0.5, 0.5)
    r0: float = 0.3
    amp: float = 0.2

    def level(self, Z, Y, X):
        dx, dy, dz = X - self.c[0], Y - self.c[1], Z - self.c[2]
        rho = np.sqrt(dx * dx + dy * dy + dz * dz)
        cos_t = np.where(rho > 0, dz / np.where(rho > 0, rho, 1.0), 1.0)
        theta = np.arccos(np.clip(cos_t, -1.0, 1.0))
        az = np.arctan2(dy, dx)
        return rho - self.r0 * (1.0 + self.amp * np.sin(5.0 * theta) * np.cos(3.0 * az))

    @property
    def bound(self):
        return self.r0 * (1.0 + self.amp)


def union_level(bodies, x, y, z):
    Z, Y, X = mesh(x, y, z)
    phi = np.full((len(z), len(y), len(x)), np.inf)
    for b in bodies:
        phi = np.minimum(phi, b.level(Z, Y, X))
    return phi


def _random_rotation(rng):
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, a, b, c = q
    return np.array([
        [1 - 2 * (b * b + c * c), 2 * (a * b - c * w), 2 * (a * c + b * w)],
        [2 * (a * b + c * w), 1 - 2 * (a * a + c * c), 2 * (b * c - a * w)],
        [2 * (a * c - b * w), 2 * (b * c + a * w), 1 - 2 * (a * a + b * b)],
    ])


def sample_bodies(seed, n_sph, n_ell, r_sph, semi_rng, gap, lo=0.15, hi=0.85, wall=0.0, max_tries=100000):
    """Rejection-sample non-overlapping bodies (bounding spheres + a surface gap).

    Centres are uniform in [lo, hi]^3.  Spheres first, then ellipsoids.  A candidate is
    rejected if its bounding sphere comes closer than `gap` to an accepted one or closer than
    `wall` to a wall of the unit cube.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    bodies = []
    kinds = ["s"] * n_sph + ["e"] * n_ell
    for kind in kinds:
        for _ in range(max_tries):
            c = tuple(rng.uniform(lo, hi, 3))
            if kind == "s":
                b = Sphere(c, float(rng.uniform(*r_sph)))
            else:
                semi = tuple(rng.uniform(*semi_rng, 3))
                b = Ellipsoid(c, semi, _random_rotation(rng))
            R = b.bound
            if min(min(c) - R, min(1.0 - ci for ci in c) - R) < wall:
                continue
            ok = all(np.linalg.norm(np.subtract(c, o.c)) >= R + o.bound + gap for o in bodies)
            if ok:
                bodies.append(b)
                break
        else:
            raise RuntimeError("could not place body")
    return bodies


# ----------------------------------------------------------------------------------------
# sources
# ----------------------------------------------------------------------------------------
def fourier_modes(seed: int, K: int):
    """Seeded random Fourier modes: k in {0..K}^3, 0 < |k| <= K, lexicographic order.

    Amplitudes N(0,1)/|k|^2 (all normals drawn first), phases U[0, 2 pi) (3 per mode, drawn after).
    """
    ks = [(a, b, c) for a in range(K + 1) for b in range(K + 1) for c in range(K + 1)
          if 0 < a * a + b * b + c * c <= K * K]
    ks = np.array(ks, dtype=np.float64)
    rng = np.random.Generator(np.random.PCG64(seed))
    amp = rng.standard_normal(len(ks)) / np.sum(ks * ks, axis=1)
    ph = rng.uniform(0.0, 2.0 * PI, (len(ks), 3))
    return ks, amp, ph


def fourier_field(seed, K, x, y, z):
    """f = sum_k A_k prod_d cos(pi k_d x_d + theta_{k,d}), evaluated plane by plane."""
    ks, amp, ph = fourier_modes(seed, K)
    X = np.cos(PI * ks[:, 0:1] * x[None, :] + ph[:, 0:1])     # (M, nx)
    Y = np.cos(PI * ks[:, 1:2] * y[None, :] + ph[:, 1:2])     # (M, ny)
    Zs = np.cos(PI * ks[:, 2:3] * z[None, :] + ph[:, 2:3])    # (M, nz)
    out = np.empty((len(z), len(y), len(x)))
    for k in range(len(z)):
        out[k] = (Y * (amp * Zs[:, k])[:, None]).T @ X
    return out


# ----------------------------------------------------------------------------------------
# the same level sets and sources on the GPU (torch, FP64), for grids too large for the
# CPU generators (512^3: 136 M nodes)
# ----------------------------------------------------------------------------------------
def union_level_torch(bodies, x, y, z, device="cuda"):
    """union_level evaluated with torch on `device`; same formulas, shape (nz, ny, nx)."""
    import torch
    Z = torch.as_tensor(np.asarray(z, dtype=np.float64), device=device)[:, None, None]
    Y = torch.as_tensor(np.asarray(y, dtype=np.float64), device=device)[None, :, None]
    X = torch.as_tensor(np.asarray(x, dtype=np.float64), device=device)[None, None, :]
    phi = torch.full((len(z), len(y), len(x)), float("inf"), dtype=torch.float64, device=device)
    for b in bodies:
        if isinstance(b, Sphere):
            lv = torch.sqrt((X - b.c[0]) ** 2 + (Y - b.c[1]) ** 2 + (Z - b.c[2]) ** 2) - b.r
        elif isinstance(b, Ellipsoid):
            d = [X - b.c[0], Y - b.c[1], Z - b.c[2]]
            acc = 0.0
            for a in range(3):
                q = float(b.rot[0, a]) * d[0] + float(b.rot[1, a]) * d[1] + float(b.rot[2, a]) * d[2]
                acc = acc + (q / b.semi[a]) ** 2
            lv = (torch.sqrt(acc) - 1.0) * min(b.semi)
        elif isinstance(b, Star):
            dx, dy, dz = X - b.c[0], Y - b.c[1], Z - b.c[2]
            rho = torch.sqrt(dx * dx + dy * dy + dz * dz)
            cos_t = torch.where(rho > 0, dz / torch.where(rho > 0, rho, torch.ones_like(rho)), torch.ones_like(rho))
            theta = torch.arccos(torch.clamp(cos_t, -1.0, 1.0))
            az = torch.atan2(dy, dx)
            lv = rho - b.r0 * (1.0 + b.amp * torch.sin(5.0 * theta) * torch.cos(3.0 * az))
        else:
            raise TypeError(type(b))
        phi = torch.minimum(phi, lv)
    return phi


def fourier_field_torch(seed, K, x, y, z, device="cuda"):
    """fourier_field evaluated with torch on `device`, plane by plane."""
    import torch
    ks, amp, ph = fourier_modes(seed, K)
    kt, at, pt = (torch.as_tensor(a, device=device) for a in (ks, amp, ph))
    xt, yt, zt = (torch.as_tensor(np.asarray(a, dtype=np.float64), device=device) for a in (x, y, z))
    Xc = torch.cos(PI * kt[:, 0:1] * xt[None, :] + pt[:, 0:1])
    Yc = torch.cos(PI * kt[:, 1:2] * yt[None, :] + pt[:, 1:2])
    Zc = torch.cos(PI * kt[:, 2:3] * zt[None, :] + pt[:, 2:3])
    out = torch.empty((len(z), len(y), len(x)), dtype=torch.float64, device=device)
    for k in range(len(z)):
        out[k] = (Yc * (at * Zc[:, k])[:, None]).T @ Xc
    return out


def bodies16_fourier_torch(N: int = 512, beta: float = 2.0, seed: int = 1, K: int = 16, device="cuda"):
    """The inputs of bodies16_fourier generated on the GPU: (x, bodies, phi, g, f), the last
    three torch tensors on `device`."""
    import torch
    x = tanh_grid(N + 2, beta)
    hc = float(np.max(np.diff(x)))
    bodies = sample_bodies(seed, 8, 8, (0.04, 0.1), (0.04, 0.12), gap=6 * hc)
    phi = union_level_torch(bodies, x, x, x, device)
    f = fourier_field_torch(seed, K, x, x, x, device)
    return x, bodies, phi, torch.zeros_like(f), f


# ----------------------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    phi: np.ndarray
    g: np.ndarray
    f: np.ndarray
    u_exact: np.ndarray | None = None
    bodies: list = field(default_factory=list)
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        return (len(self.z), len(self.y), len(self.x))


def _manufactured(name, x, y, z, bodies, u_fn, f_fn, meta):
    Z, Y, X = mesh(x, y, z)
    u = np.broadcast_to(u_fn(X, Y, Z), (len(z), len(y), len(x))).astype(np.float64).copy()
    f = np.broadcast_to(f_fn(X, Y, Z), u.shape).astype(np.float64).copy()
    phi = union_level(bodies, x, y, z) if bodies else np.ones(u.shape)
    return Workload(name, x, y, z, phi, u.copy(), f, u, bodies, meta)


def uniform_sine(N: int) -> Workload:
    """Unit cube, uniform grid, no body; u = sin(pi x) sin(pi y) sin(pi z), f = -3 pi^2 u."""
    x = uniform_grid(N + 2)
    return _manufactured(
        f"uniform_sine_{N}", x, x, x, [],
        lambda X, Y, Z: np.sin(PI * X) * np.sin(PI * Y) * np.sin(PI * Z),
        lambda X, Y, Z: -3 * PI * PI * np.sin(PI * X) * np.sin(PI * Y) * np.sin(PI * Z),
        {"N": N})


def sphere_exp(N: int = 128, beta: float = 2.0, r: float = 0.25) -> Workload:
    """tanh-stretched unit cube, one sphere (radius r) at the centre; u = exp(x+y+z), f = 3u."""
    x = tanh_grid(N + 2, beta)
    return _manufactured(
        f"sphere_exp_{N}", x, x, x, [Sphere((0.5, 0.5, 0.5), r)],
        lambda X, Y, Z: np.exp(X + Y + Z), lambda X, Y, Z: 3.0 * np.exp(X + Y + Z),
        {"N": N, "beta": beta, "r": r})


def spheres8_bodies(N: int = 256, beta: float = 1.5, seed: int = 0):
    x = tanh_grid(N + 2, beta)
    hc = float(np.max(np.diff(x)))
    return sample_bodies(seed, 8, 0, (0.06, 0.14), None, gap=6 * hc, wall=0.0)


def spheres8(N: int = 256, beta: float = 1.5, seed: int = 0) -> Workload:
    """8 seeded spheres (centres U[0.15,0.85]^3, radii U[0.06,0.14], gap 6 central cells);
    u = sin(2 pi x) cos(pi y) exp(z), f = (1 - 5 pi^2) u, g = u."""
    x = tanh_grid(N + 2, beta)
    bodies = spheres8_bodies(N, beta, seed)
    return _manufactured(
        f"spheres8_{N}", x, x, x, bodies,
        lambda X, Y, Z: np.sin(2 * PI * X) * np.cos(PI * Y) * np.exp(Z),
        lambda X, Y, Z: (1.0 - 5.0 * PI * PI) * np.sin(2 * PI * X) * np.cos(PI * Y) * np.exp(Z),
        {"N": N, "beta": beta, "seed": seed})


def star_fourier(N: int = 128, beta: float = 2.0, seed: int = 0, K: int = 8) -> Workload:
    """Star-shaped body r = 0.3 (1 + 0.2 sin 5theta cos 3phi) at the centre; random Fourier f; g = 0."""
    x = tanh_grid(N + 2, beta)
    body = Star()
    phi = union_level([body], x, x, x)
    f = fourier_field(seed, K, x, x, x)
    return Workload(f"star_fourier_{N}_s{seed}", x, x, x, phi, np.zeros_like(f), f, None, [body],
                    {"N": N, "beta": beta, "seed": seed, "K": K})


def bodies16_fourier(N: int = 512, beta: float = 2.0, seed: int = 1, K: int = 16) -> Workload:
    """8 spheres (r in [0.04,0.1]) + 8 rotated ellipsoids (semi-axes in [0.04,0.12]); Fourier f; g = 0."""
    x = tanh_grid(N + 2, beta)
    hc = float(np.max(np.diff(x)))
    bodies = sample_bodies(seed, 8, 8, (0.04, 0.1), (0.04, 0.12), gap=6 * hc)
    phi = union_level(bodies, x, x, x)
    f = fourier_field(seed, K, x, x, x)
    return Workload(f"bodies16_fourier_{N}", x, x, x, phi, np.zeros_like(f), f, None, bodies,
                    {"N": N, "beta": beta, "seed": seed, "K": K})


def polynomial_case(N: int, bodies, rng_seed: int = 7, deg: int = 4, beta: float = 0.0,
                    grids=None) -> Workload:
    """u = sum of random tensor monomials x^a y^b z^c with a, b, c <= deg; f = Laplacian(u).

    Polynomials of degree <= 4 in each variable separately are reproduced exactly by the
    fourth-order compact scheme on any tensor grid, with or without modified lines.
    """
    rng = np.random.Generator(np.random.PCG64(rng_seed))
    if grids is None:
        x = tanh_grid(N + 2, beta)
        grids = (x, x, x)
    x, y, z = grids
    terms = [(int(rng.integers(0, deg + 1)), int(rng.integers(0, deg + 1)), int(rng.integers(0, deg + 1)),
              float(rng.standard_normal())) for _ in range(6)]

    def u_fn(X, Y, Z):
        return sum(c * X ** a * Y ** b * Z ** e for a, b, e, c in terms)

    def d2(p, t):
        return p * (p - 1) * t ** (p - 2) if p >= 2 else 0.0 * t

    def f_fn(X, Y, Z):
        return sum(c * (d2(a, X) * Y ** b * Z ** e + X ** a * d2(b, Y) * Z ** e + X ** a * Y ** b * d2(e, Z))
                   for a, b, e, c in terms)

    w = _manufactured(f"poly_{N}", x, y, z, bodies, u_fn, f_fn, {"N": N, "terms": terms})
    return w


def sphere_sin(N: int, beta: float = 0.0, r: float = 0.2, c=(0.5, 0.5, 0.5)) -> Workload:
    """A sphere with the smooth manufactured solution u = sin(2 pi x) cos(pi y) exp(z)."""
    x = tanh_grid(N + 2, beta)
    return _manufactured(
        f"sphere_sin_{N}", x, x, x, [Sphere(tuple(c), r)],
        lambda X, Y, Z: np.sin(2 * PI * X) * np.cos(PI * Y) * np.exp(Z),
        lambda X, Y, Z: (1.0 - 5.0 * PI * PI) * np.sin(2 * PI * X) * np.cos(PI * Y) * np.exp(Z),
        {"N": N, "beta": beta, "r": r})


def interior_exp(n: int, sigma: float = -10.0, semi=(0.4, 0.1, 0.1)) -> Workload:
    """An interior problem in the setting of the paper's Problem 4 (Eq. p4): the fluid region
    is the inside of a closed body and the box walls lie outside it.  Grid of Eqs. p4_y /
    p4_z: x uniform on [0, 1], y on [0, 0.5] clustered at 0.14 (beta = 2), z on [0.35, 0.65]
    clustered at 0.5 (beta = 4), n points each.  The paper's stenosed pipe is given only by
    a figure; an ellipsoid around the clustering line (centre (0.5, 0.14, 0.5), semi-axes
    `semi`) stands in for it.  u = exp(sigma r), r = |x - (0.5, 0.5, 0.5)|^2, f =
    2 sigma exp(sigma r)(3 + 2 sigma r), g = u."""
    x = uniform_grid(n)
    y = sinh_grid(n, 2.0, 0.14, 0.5)
    z = sinh_grid(n, 4.0, 0.15, 0.3, 0.35)
    body = Ellipsoid((0.5, 0.14, 0.5), tuple(semi), np.eye(3))
    Z, Y, X = mesh(x, y, z)
    r = (X - 0.5) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2
    shape = (len(z), len(y), len(x))
    u = np.broadcast_to(np.exp(sigma * r), shape).astype(np.float64).copy()
    f = np.broadcast_to(2.0 * sigma * np.exp(sigma * r) * (3.0 + 2.0 * sigma * r), shape).astype(np.float64).copy()
    phi = -union_level([body], x, y, z)            # positive inside the body
    return Workload(f"interior_exp_{n}", x, y, z, phi, u.copy(), f, u, [body],
                    {"n": n, "sigma": sigma, "semi": tuple(semi)})


WORKLOADS = {
    "uniform_sine": uniform_sine,
    "sphere_exp": sphere_exp,
    "spheres8": spheres8,
    "star_fourier": star_fourier,
    "bodies16_fourier": bodies16_fourier,
    "interior_exp": interior_exp,
}
