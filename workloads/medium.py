"""Seeded material models, evaluated per element at the element centroid.

Layered model on [0, 10]^3 with depth measured from the top face z = 10:
layer index Lz = min(3, floor((10 - z) / 2.5)), so the interfaces sit at
z = 7.5, 5 and 2.5 and align with meshes of 16 and 24 cells per side.

* P-wave speed of the layer: 1.5 + 2.5 * Lz / 3  (1.5, 2.333, 3.167, 4.0).
* 5 % noise: a 48^3 standard-normal field (seed 2205, indexed [iz, iy, ix],
  samples at cell centres of a 48^3 grid on [0, 10]^3) smoothed by a separable
  Gaussian of width 0.5 length units (truncated at 4 widths, reflecting
  edges), divided by its largest magnitude and sampled trilinearly:
  cp = cp_layer * (1 + 0.05 * noise).
* cs = cp / sqrt(3); rho = 1 + 2 * Lz / 3 (1.0 ... 3.0, no noise).
* Lame parameters: mu = rho * cs^2, lambda = rho * cp^2 - 2 * mu.
"""

import numpy as np
from scipy import ndimage

MEDIUM_SEED = 2205
NOISE_GRID = 48
NOISE_SIGMA = 0.5
NOISE_AMPLITUDE = 0.05
BOX = 10.0


def lame_from_velocities(cp, cs, rho):
    """(rho, lambda, mu) from wave speeds and density."""
    cp = np.asarray(cp, dtype=np.float64)
    cs = np.asarray(cs, dtype=np.float64)
    rho = np.asarray(rho, dtype=np.float64)
    mu = rho * cs * cs
    lam = rho * cp * cp - 2.0 * mu
    return rho, lam, mu


def homogeneous_medium(K, rho=1.0, cp=np.sqrt(3.0), cs=1.0):
    """Constant material on K elements; default rho = 1, lambda = mu = 1."""
    return lame_from_velocities(np.full(K, cp), np.full(K, cs),
                                np.full(K, rho))


def _layer(z):
    return np.minimum(3, np.floor((BOX - z) / 2.5)).astype(np.float64)


def _noise(points):
    rng = np.random.default_rng(MEDIUM_SEED)
    g = rng.standard_normal((NOISE_GRID, NOISE_GRID, NOISE_GRID))
    hcell = BOX / NOISE_GRID
    sm = ndimage.gaussian_filter(g, sigma=NOISE_SIGMA / hcell, mode="reflect",
                                 truncate=4.0)
    sm /= np.max(np.abs(sm))
    # grid index of a point: x / hcell - 0.5 (samples at cell centres)
    coords = np.stack([points[:, 2], points[:, 1], points[:, 0]]) / hcell - 0.5
    return ndimage.map_coordinates(sm, coords, order=1, mode="nearest")


def layered_medium(centroids):
    """Returns (rho, lam, mu, cp) at the given [K, 3] centroids."""
    z = centroids[:, 2]
    Lz = _layer(z)
    cp_layer = 1.5 + 2.5 * Lz / 3.0
    cp = cp_layer * (1.0 + NOISE_AMPLITUDE * _noise(centroids))
    cs = cp / np.sqrt(3.0)
    rho = 1.0 + 2.0 * Lz / 3.0
    r, lam, mu = lame_from_velocities(cp, cs, rho)
    return r, lam, mu, cp


def blob_start_medium(centroids, centre=(5.0, 5.0, 8.5), width=1.0,
                      depth=0.10):
    """Starting model for the gradient test: the layered model with cp lowered
    by a Gaussian blob (10 % at its centre), cs = cp / sqrt(3), rho unchanged."""
    rho, _, _, cp = layered_medium(centroids)
    d2 = np.sum((centroids - np.asarray(centre)) ** 2, axis=1)
    cp = cp * (1.0 - depth * np.exp(-d2 / (2.0 * width * width)))
    r, lam, mu = lame_from_velocities(cp, cp / np.sqrt(3.0), rho)
    return r, lam, mu, cp


def sponge_profile(centroids, lo=(0.0, 0.0, 0.0), hi=(BOX, BOX, BOX), width=1.0,
                   sigma_max=1.0, faces=("x-", "x+", "y-", "y+", "z-")):
    """Per-element damping rate of an absorbing sponge layer inside the box
    [lo, hi]: sigma = sigma_max (1 - d / width)^2 where d < width is the
    centroid's distance to the nearest listed face ("x-" is x = lo[0], "z+"
    is z = hi[2], ...), 0 elsewhere.  The default lists every face but the
    top (free surface)."""
    c = np.asarray(centroids, dtype=np.float64)
    d = np.full(c.shape[0], np.inf)
    for f in faces:
        a = "xyz".index(f[0])
        d = np.minimum(d, c[:, a] - lo[a] if f[1] == "-" else hi[a] - c[:, a])
    s = np.clip(1.0 - d / width, 0.0, None)
    return sigma_max * s * s


def pml_profile(points, lo=(0.0, 0.0, 0.0), hi=(BOX, BOX, BOX), width=1.0,
                cp_max=4.2, reflection=1e-3, f0=1.0,
                faces=("x-", "x+", "y-", "y+", "z-")):
    """Per-axis damping profiles of a convolutional perfectly matched layer
    of the given width inside the box [lo, hi] along the listed faces, at
    points [..., 3] (element centroids or nodes): for axis b,
    r_b = (depth into the layer along b) / width in [0, 1], d_b = d0 r_b^2 with
    d0 = 3 cp_max ln(1 / reflection) / (2 width) (the quadratic profile's
    nominal normal-incidence reflection), and the frequency shift
    alpha_b = pi f0 (1 - r_b) inside the layer, 0 outside.  Returns
    (d [..., 3], alpha [..., 3])."""
    c = np.asarray(points, dtype=np.float64)
    r = np.zeros_like(c)
    for f in faces:
        a = "xyz".index(f[0])
        depth = width - (c[..., a] - lo[a] if f[1] == "-" else hi[a] - c[..., a])
        r[..., a] = np.maximum(r[..., a], np.clip(depth / width, 0.0, 1.0))
    d0 = 3.0 * cp_max * np.log(1.0 / reflection) / (2.0 * width)
    d = d0 * r * r
    alpha = np.where(r > 0, np.pi * f0 * (1.0 - r), 0.0)
    return d, alpha


def pml_layer(mesh, N, **kw):
    """The perfectly matched layer of ``pml_profile`` (same keywords) at the
    nodes of an order-N mesh, in the two forms the solvers take: per node for
    every element, d [K, 3, Np] and alpha [K, 3, Np], and restricted to the
    layer, the strictly increasing ids of the elements with d > 0 at some
    node and their profile [n, 6, Np] (d_x, d_y, d_z, alpha_x, alpha_y,
    alpha_z).  Returns (elements, profile, d, alpha)."""
    from .mesh import lattice_node_coords
    X = lattice_node_coords(mesh, N)                               # [K, Np, 3]
    d, a = pml_profile(X, **kw)
    d = np.ascontiguousarray(np.moveaxis(d, 2, 1))
    a = np.ascontiguousarray(np.moveaxis(a, 2, 1))
    elems = np.nonzero((d > 0).any(axis=(1, 2)))[0].astype(np.int32)
    prof = np.ascontiguousarray(np.concatenate([d[elems], a[elems]], axis=1))
    return elems, prof, d, a


def isotropic_stiffness(lam, mu):
    """Voigt stiffness [K, 6, 6] (order xx, yy, zz, yz, xz, xy; engineering
    shear strains) of isotropic elements."""
    lam = np.atleast_1d(np.asarray(lam, dtype=np.float64))
    mu = np.atleast_1d(np.asarray(mu, dtype=np.float64))
    C = np.zeros(lam.shape + (6, 6))
    C[:, :3, :3] = lam[:, None, None]
    for i in range(3):
        C[:, i, i] += 2.0 * mu
        C[:, 3 + i, 3 + i] = mu
    return C


def random_stiffness(K, seed, strength=0.5):
    """Seeded fully anisotropic stiffness [K, 6, 6]: a random isotropic
    background (cp in [1.5, 3], cp/cs in [1.5, 2.2], rho in [1, 3]) plus
    strength * mu * G G^T / 6 with G a 6x6 standard-normal matrix per
    element (symmetric positive definite, every one of the 21 entries
    nonzero).  Returns (rho, C)."""
    rng = np.random.default_rng(seed)
    cp = rng.uniform(1.5, 3.0, K)
    cs = cp / rng.uniform(1.5, 2.2, K)
    rho = rng.uniform(1.0, 3.0, K)
    rho, lam, mu = lame_from_velocities(cp, cs, rho)
    G = rng.standard_normal((K, 6, 6))
    C = isotropic_stiffness(lam, mu) + strength * mu[:, None, None] * (G @ G.transpose(0, 2, 1)) / 6.0
    return rho, C


def stiffness_upper(C):
    """The 21 upper-triangle entries of each Voigt stiffness, row by row
    (C11 C12 ... C16 C22 ... C66): [K, 21]."""
    iu = np.triu_indices(6)
    return np.ascontiguousarray(np.asarray(C, dtype=np.float64)[:, iu[0], iu[1]])
