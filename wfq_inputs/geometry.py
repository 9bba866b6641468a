"""Lattice geometries (positions in Angstrom) for the structure families the paper studies.

Families: graphene disks (the GD series of the geometry study), graphene
sheets and ribbons, (n,m) carbon nanotubes (the CNT series, with the
diameter rule printed under the CNT table), and FCC metal spheres standing in
for the sodium nanorod of the large-systems section. Positions are plain
float64 arrays of shape (N, 3); nothing here knows about charges or matrices.
"""

import math

import numpy as np

from .rng import gaussian

A_CC = 1.42                      # graphene C-C bond length, Angstrom
A_GRAPHENE = math.sqrt(3.0) * A_CC   # graphene lattice constant (2.4595 Angstrom)
A_FCC = 4.09                     # cubic FCC lattice constant used for metal spheres

# Primitive vectors of the honeycomb lattice (A sublattice) and the A->B offset.
_A1 = np.array([A_GRAPHENE, 0.0])
_A2 = np.array([0.5 * A_GRAPHENE, 0.5 * math.sqrt(3.0) * A_GRAPHENE])
_DELTA = (_A1 + _A2) / 3.0       # |_DELTA| == A_CC


def _honeycomb_points(radius: float, center: np.ndarray) -> np.ndarray:
    """All A and B honeycomb sites within `radius` of `center` (2D)."""
    nmax = int(math.ceil(radius / (0.5 * A_GRAPHENE))) + 3
    i, j = np.meshgrid(np.arange(-nmax, nmax + 1), np.arange(-nmax, nmax + 1), indexing="ij")
    lat = i.reshape(-1, 1) * _A1 + j.reshape(-1, 1) * _A2
    pts = np.concatenate([lat, lat + _DELTA], axis=0)
    keep = np.sum((pts - center) ** 2, axis=1) <= radius * radius
    return pts[keep] - center


def graphene_disk(radius: float) -> np.ndarray:
    """Disk cut from a flat graphene sheet, centred on a hexagon centre, edge atoms kept.

    Atoms with |r - c| <= radius are kept, c being a hexagon centre (the third
    sublattice point 2*delta); dangling edge atoms are retained as the paper
    does for its disks.
    """
    center = 2.0 * _DELTA
    p = _honeycomb_points(radius, center)
    order = np.lexsort((p[:, 0], p[:, 1]))
    p = p[order]
    return np.column_stack([p, np.zeros(len(p))])


def _orthogonal_cells(nx: int, ny: int) -> np.ndarray:
    """nx x ny orthogonal 4-atom graphene cells (a along x, 3*a_cc along y), z = 0."""
    a, b = A_GRAPHENE, A_CC
    basis = np.array([[0.0, 0.0], [0.5 * a, 0.5 * b], [0.5 * a, 1.5 * b], [0.0, 2.0 * b]])
    ix, iy = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    origin = np.column_stack([ix.ravel() * a, iy.ravel() * 3.0 * b])
    p = (origin[:, None, :] + basis[None, :, :]).reshape(-1, 2)
    return np.column_stack([p, np.zeros(len(p))])


def graphene_sheet(nx: int, ny: int) -> np.ndarray:
    """Rectangular sheet of nx x ny orthogonal cells (4*nx*ny atoms)."""
    return _orthogonal_cells(nx, ny)


def graphene_ribbon(width_A: float, n_atoms: int) -> np.ndarray:
    """Ribbon of the given width (along y); its length (along x) is chosen from the atom count."""
    ny = max(1, int(round(width_A / (3.0 * A_CC))))
    nx = max(1, int(round(n_atoms / (4.0 * ny))))
    return _orthogonal_cells(nx, ny)


def nanotube_diameter(n: int, m: int) -> float:
    """Tube diameter d = (a/pi) sqrt(n^2 + m^2 + n m) in Angstrom (rule under the CNT table)."""
    return A_GRAPHENE / math.pi * math.sqrt(n * n + m * m + n * m)


def _tube_vectors(n: int, m: int):
    dr = math.gcd(2 * m + n, 2 * n + m)
    t1 = (2 * m + n) // dr
    t2 = -(2 * n + m) // dr
    return dr, t1, t2


def nanotube_atoms_per_cell(n: int, m: int) -> int:
    """Atoms in one translational unit cell of an (n,m) tube: 4 (n^2 + n m + m^2) / gcd(2m+n, 2n+m)."""
    dr, _, _ = _tube_vectors(n, m)
    return 4 * (n * n + n * m + m * m) // dr


def nanotube(n: int, m: int, n_cells: int) -> np.ndarray:
    """(n,m) carbon nanotube of `n_cells` translational unit cells, axis along z.

    The graphene strip spanned by the chiral vector C = n a1 + m a2 and
    n_cells times the translation vector T is selected with exact integer
    coordinates, then rolled onto a cylinder of circumference |C|.
    """
    if n < 1 or m < 0:
        raise ValueError("need n >= 1, m >= 0")
    dr, t1, t2 = _tube_vectors(n, m)
    den_u = 2 * (n * n + n * m + m * m)          # 2 |C|^2 / a^2
    den_v = 2 * (t1 * t1 + t1 * t2 + t2 * t2)    # 2 |T|^2 / a^2
    corners_i = [0, n, n_cells * t1, n + n_cells * t1]
    corners_j = [0, m, n_cells * t2, m + n_cells * t2]
    i, j = np.meshgrid(np.arange(min(corners_i) - 1, max(corners_i) + 2),
                       np.arange(min(corners_j) - 1, max(corners_j) + 2), indexing="ij")
    i = i.ravel().astype(np.int64)
    j = j.ravel().astype(np.int64)
    num_u = i * (2 * n + m) + j * (n + 2 * m)
    num_v = i * (2 * t1 + t2) + j * (t1 + 2 * t2)
    inside = (num_u >= 0) & (num_u < den_u) & (num_v >= 0) & (num_v < n_cells * den_v)
    i, j = i[inside], j[inside]
    lat = i[:, None] * _A1 + j[:, None] * _A2
    pts = np.concatenate([lat, lat + _DELTA], axis=0)
    cvec = n * _A1 + m * _A2
    tvec = t1 * _A1 + t2 * _A2
    u = pts @ cvec / (cvec @ cvec)
    v = pts @ tvec / (tvec @ tvec)
    radius = math.sqrt(cvec @ cvec) / (2.0 * math.pi)
    theta = 2.0 * math.pi * u
    xyz = np.column_stack([radius * np.cos(theta), radius * np.sin(theta),
                           v * math.sqrt(tvec @ tvec)])
    order = np.lexsort((theta, xyz[:, 2]))
    return xyz[order]


def fcc_sphere(radius: float, a: float = A_FCC) -> np.ndarray:
    """Atoms of a cubic FCC lattice (constant a) within `radius` of a lattice site."""
    nmax = int(math.ceil(radius / a)) + 1
    r = np.arange(-nmax, nmax + 1)
    ix, iy, iz = np.meshgrid(r, r, r, indexing="ij")
    cells = np.column_stack([ix.ravel(), iy.ravel(), iz.ravel()]).astype(np.float64) * a
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]]) * a
    p = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3)
    p = p[np.sum(p * p, axis=1) <= radius * radius]
    order = np.lexsort((p[:, 0], p[:, 1], p[:, 2]))
    return p[order]


def jitter(xyz: np.ndarray, sigma: float, seed: int) -> np.ndarray:
    """Add i.i.d. N(0, sigma^2) displacements to every Cartesian coordinate (seeded SplitMix64)."""
    if sigma == 0.0:
        return np.array(xyz, dtype=np.float64, copy=True)
    g = gaussian(seed, xyz.size).reshape(xyz.shape)
    return np.asarray(xyz, dtype=np.float64) + sigma * g
