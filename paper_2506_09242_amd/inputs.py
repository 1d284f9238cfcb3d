"""Seeded synthetic inputs shared by the HIP path's tests/bench and the oracle.

This module holds geometry, initial fields and random streams only -- none of
the lattice Boltzmann arithmetic (no equilibria, no collision, no streaming).
Both sides receive exactly the same arrays from here.

Shapes follow the paper's workloads: the Taylor-Green vortex initial field
(Sec. 3.1, Eqs. 1-4), the lid-driven cubic cavity (Sec. 3.2), a porous solid
standing in for the Berea micro-CT sample (Sec. 3.3, porosity ~0.2), plus
plane channels for the analytic Poiseuille / Couette checks.

Random numbers: SplitMix64 (Steele, Lea & Flood 2014; Vigna's reference
constants), Box-Muller for normals, Fisher-Yates for permutations.
"""
from __future__ import annotations

import numpy as np

TAG_SOLID, TAG_BGK, TAG_TRT, TAG_SMAG, TAG_MLP, TAG_REG, TAG_WALL0 = 0, 1, 2, 3, 4, 5, 16
TAG_VIN, TAG_POUT, TAG_PIN, TAG_VOUT = 6, 7, 8, 9  # open boundaries on the x planes
TAG_RR = 10

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, n: int, offset: int = 0) -> np.ndarray:
    """n outputs of SplitMix64 started at state `seed` (outputs offset..offset+n-1)."""
    k = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + k * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, n: int, offset: int = 0) -> np.ndarray:
    """Uniform doubles in (0, 1] from the top 53 bits."""
    return ((splitmix64(seed, n, offset) >> np.uint64(11)).astype(np.float64) + 1.0) * (1.0 / 9007199254740992.0)


def normal(seed: int, n: int) -> np.ndarray:
    """Standard normals by Box-Muller from pairs of SplitMix64 uniforms."""
    m = (n + 1) // 2
    u1 = uniform01(seed, m, 0)
    u2 = uniform01(seed, m, m)
    r = np.sqrt(-2.0 * np.log(u1))
    z = np.concatenate([r * np.cos(2 * np.pi * u2), r * np.sin(2 * np.pi * u2)])
    return z[:n]


def permutation(n: int, seed: int) -> np.ndarray:
    """Fisher-Yates shuffle of 0..n-1 driven by SplitMix64 (j = r mod (i+1))."""
    r = splitmix64(seed, max(n - 1, 0))
    p = np.arange(n, dtype=np.int64)
    for idx, i in enumerate(range(n - 1, 0, -1)):
        j = int(r[idx] % np.uint64(i + 1))
        p[i], p[j] = p[j], p[i]
    return p


# ------------------------------------------------------------------ geometry
def all_fluid(nx, ny, nz, tag=TAG_BGK) -> np.ndarray:
    return np.full((nz, ny, nx), tag, dtype=np.uint8)


def cavity_tags(n: int, fluid_tag=TAG_BGK, lid_tag=TAG_WALL0) -> np.ndarray:
    """Cubic cavity n^3: one-cell solid shell, the whole top layer z=n-1 is the lid.

    Fluid occupies (n-2)^3 cells; with half-way walls the cavity length is n-2.
    """
    t = np.full((n, n, n), TAG_SOLID, dtype=np.uint8)
    t[1:-1, 1:-1, 1:-1] = fluid_tag
    t[n - 1, :, :] = lid_tag
    return t


def channel_tags(nx, ny, nz, fluid_tag=TAG_BGK, bottom=TAG_SOLID, top=TAG_SOLID) -> np.ndarray:
    """Plane channel: walls at z=0 and z=nz-1, periodic in x and y (width nz-2)."""
    t = np.full((nz, ny, nx), fluid_tag, dtype=np.uint8)
    t[0] = bottom
    t[nz - 1] = top
    return t


def random_tags(nx, ny, nz, seed, solid_frac=0.2, wall_frac=0.05, fluid_tags=(TAG_BGK,),
                n_walls=2) -> np.ndarray:
    """Random mix of fluid / solid / moving-wall tags (race-freedom and parity edge cases)."""
    u = uniform01(seed, nx * ny * nz).reshape(nz, ny, nx)
    v = splitmix64(seed + 1, nx * ny * nz).reshape(nz, ny, nx)
    t = np.array(fluid_tags, dtype=np.uint8)[(v % np.uint64(len(fluid_tags))).astype(np.int64)]
    t = t.astype(np.uint8)
    t[u < solid_frac + wall_frac] = (TAG_WALL0 + (v[u < solid_frac + wall_frac] % np.uint64(n_walls))).astype(np.uint8)
    t[u < solid_frac] = TAG_SOLID
    return t


def gaussian_random_field(n: int, ell: float, seed: int) -> np.ndarray:
    """Periodic Gaussian random field, covariance ~ exp(-r^2/(2 ell^2)).

    White noise (SplitMix64 + Box-Muller) filtered in Fourier space by the
    amplitude exp(-|k|^2 ell^2 / 4) (square root of the covariance spectrum).
    """
    w = normal(seed, n ** 3).reshape(n, n, n).astype(np.float32)
    W = np.fft.rfftn(w)
    k = 2 * np.pi * np.fft.fftfreq(n)
    kr = 2 * np.pi * np.fft.rfftfreq(n)
    k2 = k[:, None, None] ** 2 + k[None, :, None] ** 2 + kr[None, None, :] ** 2
    W *= np.exp(-k2 * ell * ell / 4.0).astype(np.float32)
    return np.fft.irfftn(W, s=(n, n, n)).astype(np.float32)


def porous_tags(n: int, porosity=0.20, ell=8.0, seed=42, fluid_tag=TAG_TRT) -> np.ndarray:
    """Solid mask from a thresholded Gaussian random field: the lowest `porosity`
    fraction of values is fluid (ties broken by linear index), the rest solid."""
    g = gaussian_random_field(n, ell, seed).ravel()
    order = np.argsort(g, kind="stable")
    nf = int(round(porosity * g.size))
    t = np.full(g.size, TAG_SOLID, dtype=np.uint8)
    t[order[:nf]] = fluid_tag
    return t.reshape(n, n, n)


def percolates_x(tags: np.ndarray) -> bool:
    """6-connected fluid path from the x=0 face to the x=nx-1 face."""
    from scipy import ndimage
    fluid = (tags >= 1) & (tags <= 10)
    lab, _ = ndimage.label(fluid)
    a = set(np.unique(lab[:, :, 0])) - {0}
    b = set(np.unique(lab[:, :, -1])) - {0}
    return len(a & b) > 0


# ------------------------------------------------------------- initial fields
def tgv3d_fields(n: int, u0: float, rho0: float = 1.0):
    """Taylor-Green vortex of Sec. 3.1, Eqs. (1)-(4), on an n^3 node-centred grid
    x_i = 2 pi i / n.  Pressure term read as rho0 u0^2/16 (dimensionally
    required); density from the lattice equation of state p = rho / 3."""
    s = 2 * np.pi * np.arange(n) / n
    # separable factors broadcast over (z, y, x); products in the same order as
    # the formulas, so the values do not depend on this arrangement
    x, y, z = s[None, None, :], s[None, :, None], s[:, None, None]
    u = np.empty((3, n, n, n))
    u[0] = u0 * np.sin(x) * np.cos(y) * np.cos(z)
    u[1] = -u0 * np.cos(x) * np.sin(y) * np.cos(z)
    u[2] = 0.0
    dp = rho0 * u0 * u0 / 16.0 * (np.cos(2 * z) + 2.0) * (np.cos(2 * x) + np.cos(2 * y))
    rho = rho0 + 3.0 * dp
    return rho, u


def tgv2d_fields(n: int, nz: int, u0: float, rho0: float = 1.0):
    """z-invariant Taylor-Green vortex: u = u0 (sin kx cos ky, -cos kx sin ky, 0),
    p - p0 = (rho0 u0^2 / 4)(cos 2kx + cos 2ky), k = 2 pi / n."""
    s = 2 * np.pi * np.arange(n) / n
    z = np.arange(nz)
    Z, Y, X = np.meshgrid(z, s, s, indexing="ij")
    ux = u0 * np.sin(X) * np.cos(Y)
    uy = -u0 * np.cos(X) * np.sin(Y)
    uz = np.zeros_like(ux)
    rho = rho0 + 3.0 * rho0 * u0 * u0 / 4.0 * (np.cos(2 * X) + np.cos(2 * Y))
    return rho, np.stack([ux, uy, uz])


def random_fields(nx, ny, nz, seed, du=0.02, drho=0.01):
    """Smooth-free random perturbation around rest (parity tests)."""
    N = nx * ny * nz
    r = 1.0 + drho * (2.0 * uniform01(seed, N) - 1.0)
    u = du * (2.0 * uniform01(seed + 7, 3 * N) - 1.0)
    return r.reshape(nz, ny, nx), u.reshape(3, nz, ny, nx)


# ------------------------------------------------------------- MLP parameters
def mlp_he_init(seed: int) -> np.ndarray:
    """He-normal initial weights for the 7->32->32->1 closure network, zero biases,
    identity normalisation; packed W1,b1,W2,b2,W3,b3,mean,std (1359 floats)."""
    z = normal(seed, 224 + 1024 + 32)
    W1 = z[:224] * np.sqrt(2.0 / 7.0)
    W2 = z[224:1248] * np.sqrt(2.0 / 32.0)
    W3 = z[1248:1280] * np.sqrt(2.0 / 32.0)
    p = np.concatenate([W1, np.zeros(32), W2, np.zeros(32), W3, np.zeros(1), np.zeros(7), np.ones(7)])
    return p.astype(np.float32)


def permutation_by_keys(n: int, seed: int) -> np.ndarray:
    """Random permutation of 0..n-1 by sorting SplitMix64 keys (ties by index).
    Used where a Python-level Fisher-Yates loop over millions of items is too slow."""
    return np.argsort(splitmix64(seed, n), kind="stable").astype(np.int64)


def sample_without_replacement(pool: int, k: int, seed: int) -> np.ndarray:
    """k distinct indices of range(pool): the k smallest SplitMix64 keys, in key order."""
    keys = splitmix64(seed, pool)
    idx = np.argpartition(keys, k - 1)[:k]
    return idx[np.argsort(keys[idx], kind="stable")].astype(np.int64)
