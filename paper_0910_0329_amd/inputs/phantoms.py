"""Seeded synthetic voxel phantoms.

The paper's phantoms are rectangular boxes of voxels made of slabs along z
(water-lung-water and water-bone-water, Sec. 3).  A phantom here is a grid plus
two arrays in x-fastest order: a material index per voxel (u8, indexing the
table blob's materials) and a mass density per voxel (f32, g/cm^3).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .tables import MAT_AIR, MAT_BONE, MAT_LUNG, MAT_WATER


@dataclass
class Phantom:
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    x0: float = 0.0
    y0: float = 0.0
    z0: float = 0.0
    mat: np.ndarray = None       # uint8 [nz, ny, nx]
    rho: np.ndarray = None       # float32 [nz, ny, nx]

    @property
    def n_vox(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def voxel_volume(self) -> float:
        return self.dx * self.dy * self.dz

    def centre_xy(self):
        return (self.x0 + 0.5 * self.nx * self.dx, self.y0 + 0.5 * self.ny * self.dy)

    def grid_tuple(self):
        return (self.nx, self.ny, self.nz, self.dx, self.dy, self.dz, self.x0, self.y0, self.z0)


def slab_phantom(nx, ny, dx, dy, layers, dz, x0=0.0, y0=0.0, z0=0.0) -> Phantom:
    """Layers along z: a list of (n_slices, material index, density)."""
    nz = sum(n for n, _, _ in layers)
    mat = np.empty((nz, ny, nx), dtype=np.uint8)
    rho = np.empty((nz, ny, nx), dtype=np.float32)
    k = 0
    for n, m, r in layers:
        mat[k:k + n] = m
        rho[k:k + n] = r
        k += n
    return Phantom(nx, ny, nz, dx, dy, dz, x0, y0, z0, mat, rho)


def homogeneous(nx, ny, nz, d, material=MAT_WATER, density=1.0, dz=None) -> Phantom:
    return slab_phantom(nx, ny, d, d, [(nz, material, density)], d if dz is None else dz)


def water_lung_water_32() -> Phantom:
    """32x32x30 voxels of 0.5 cm: water 0-3 cm, lung (0.26) 3-10 cm, water 10-15 cm."""
    return slab_phantom(32, 32, 0.5, 0.5,
                        [(6, MAT_WATER, 1.0), (14, MAT_LUNG, 0.26), (10, MAT_WATER, 1.0)], 0.5)


def water_bone_water_61() -> Phantom:
    """61x61x60 voxels of 0.5 cm: water 0-3 cm, bone (1.85) 3-7 cm, water 7-30 cm."""
    return slab_phantom(61, 61, 0.5, 0.5,
                        [(6, MAT_WATER, 1.0), (8, MAT_BONE, 1.85), (46, MAT_WATER, 1.0)], 0.5)


def paper_slab_phantom(middle: str = "lung") -> Phantom:
    """The paper's own geometry (Sec. 3): 61x61x150 voxels of 0.5x0.5x0.2 cm,
    5 cm water, 5 cm lung or bone, 20 cm water."""
    m, r = (MAT_LUNG, 0.26) if middle == "lung" else (MAT_BONE, 1.85)
    return slab_phantom(61, 61, 0.5, 0.5, [(25, MAT_WATER, 1.0), (25, m, r), (100, MAT_WATER, 1.0)], 0.2)


def material_from_density(rho: np.ndarray) -> np.ndarray:
    """Thresholds 0.1 / 0.5 / 1.3 g/cm^3 -> air / lung / water / bone."""
    mat = np.full(rho.shape, MAT_BONE, dtype=np.uint8)
    mat[rho < 1.3] = MAT_WATER
    mat[rho < 0.5] = MAT_LUNG
    mat[rho < 0.1] = MAT_AIR
    return mat


# upper density bounds (g/cm^3) of the eight tissue classes, in the order
# air, lung, adipose, water, muscle, cartilage, spongiosa (bone above)
TISSUE_BOUNDS = (0.1, 0.5, 0.97, 1.02, 1.08, 1.14, 1.3)


def tissue_from_density(rho: np.ndarray) -> np.ndarray:
    """Eight-class material map for the TISSUES8 table set (material indices
    0-3 air, lung, water, bone; 4-7 adipose, muscle, cartilage, spongiosa)."""
    order = np.array([0, 1, 4, 2, 5, 6, 7, 3], dtype=np.uint8)
    return order[np.digitize(rho, TISSUE_BOUNDS)]


def random_field_phantom(n, d, seed, nz=None, sigma_cm=1.0) -> Phantom:
    """CT-like heterogeneous phantom from a Gaussian-smoothed random field.

    White N(0,1) noise (numpy PCG64, `seed`) is smoothed by a periodic Gaussian
    filter of standard deviation `sigma_cm` applied in Fourier space, renormalised
    to zero mean and unit variance (g), mapped to rho = clip(0.9 + 0.45 g, 0.0012,
    2.0) and thresholded into materials.  The density stays continuous per voxel.
    """
    nx = ny = n
    nz = n if nz is None else nz
    rng = np.random.default_rng(seed)
    white = rng.standard_normal((nz, ny, nx), dtype=np.float32)
    spec = np.fft.rfftn(white)
    del white
    s = sigma_cm / d                       # filter width in voxels
    kz = np.fft.fftfreq(nz)[:, None, None]
    ky = np.fft.fftfreq(ny)[None, :, None]
    kx = np.fft.rfftfreq(nx)[None, None, :]
    filt = np.exp(-2.0 * (np.pi * s) ** 2 * (kx * kx + ky * ky + kz * kz))
    spec *= filt
    g = np.fft.irfftn(spec, s=(nz, ny, nx), axes=(0, 1, 2)).astype(np.float64)
    del spec
    g -= g.mean()
    g /= g.std()
    rho = np.clip(0.9 + 0.45 * g, 0.0012, 2.0).astype(np.float32)
    return Phantom(nx, ny, nz, d, d, d, 0.0, 0.0, 0.0, material_from_density(rho), rho)
