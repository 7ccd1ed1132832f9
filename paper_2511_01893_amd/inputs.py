"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module only draws random numbers and evaluates simple test objects
(Gaussian blobs, a layer of cubes, Gaussian noise).  It holds none of the
laminography method's arithmetic, and it imports neither the HIP library nor
the oracle, so both sides can be fed the same arrays without sharing code.

Recipe (the paper's datasets are not available, so phantoms of the paper's
cubic shapes stand in for them):

* Blob phantom: ``rng = numpy.random.default_rng(seed)`` draws the centres
  ``uniform(-0.3, 0.3, (nblobs, 3))`` as (x, y, z), then the widths
  ``uniform(0.03, 0.1, nblobs)``, then the amplitudes ``uniform(0.5, 1,
  nblobs)``.  A blob is ``A * exp(-|r - c|^2 / (2 sigma^2))`` with the voxel
  at centred index ``j`` sitting at ``r = j / n`` along each axis.
* Cube layer (optional): voxels with ``|z| < 1/8`` are split into cubes of
  edge ``n / 16`` voxels whose values are drawn i.i.d. from {0, 0.5, 1} by
  the same generator, after the blob parameters, and added to the blobs.
* Random detector data: real and imaginary parts i.i.d. N(0, 1) from
  ``default_rng(seed + 200)``.
* Measurement noise: real N(0, (level * max|Re d|)^2) from
  ``default_rng(seed + 100)``.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class BlobSet:
    centres: np.ndarray   # (nb, 3) as (x, y, z), unit-cube coordinates
    sigmas: np.ndarray    # (nb,)
    amps: np.ndarray      # (nb,)
    cube_values: np.ndarray | None  # (nzc, nyc, nxc) values of the cube layer, or None


def draw_blobs(seed: int, nblobs: int, cube_layer: bool = False, n: int | None = None) -> BlobSet:
    """Draw the blob (and optional cube-layer) parameters from ``seed``."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-0.3, 0.3, (nblobs, 3))
    sigmas = rng.uniform(0.03, 0.1, nblobs)
    amps = rng.uniform(0.5, 1.0, nblobs)
    cubes = None
    if cube_layer:
        if n is None or n % 16:
            raise ValueError("cube layer needs a volume edge divisible by 16")
        edge = n // 16
        nzc = max(1, (n // 4) // edge)   # |z| < 1/8 spans n/4 voxels
        cubes = rng.choice(np.array([0.0, 0.5, 1.0]), size=(nzc, 16, 16))
    return BlobSet(centres, sigmas, amps, cubes)


def _axis(n: int) -> np.ndarray:
    return (np.arange(n) - n // 2) / n


def blob_phantom(shape, blobs: BlobSet) -> np.ndarray:
    """Evaluate the phantom on a (n0, n1, n2) = (z, y, x) grid in float64 (NumPy)."""
    n0, n1, n2 = shape
    z, y, x = _axis(n0), _axis(n1), _axis(n2)
    u = np.zeros(shape, dtype=np.float64)
    for c, s, a in zip(blobs.centres, blobs.sigmas, blobs.amps):
        gx = np.exp(-((x - c[0]) ** 2) / (2 * s * s))
        gy = np.exp(-((y - c[1]) ** 2) / (2 * s * s))
        gz = a * np.exp(-((z - c[2]) ** 2) / (2 * s * s))
        u += gz[:, None, None] * (gy[:, None] * gx[None, :])[None, :, :]
    if blobs.cube_values is not None:
        u += _cube_layer(shape, blobs.cube_values)
    return u


def _cube_layer(shape, cube_values: np.ndarray) -> np.ndarray:
    n0, n1, n2 = shape
    edge = n0 // 16
    lay = np.zeros(shape, dtype=np.float64)
    nzc = cube_values.shape[0]
    z0 = n0 // 2 - (nzc * edge) // 2
    block = np.repeat(np.repeat(np.repeat(cube_values, edge, 0), n1 // 16, 1), n2 // 16, 2)
    lay[z0:z0 + nzc * edge] = block
    return lay


def blob_phantom_torch(shape, blobs: BlobSet, device, dtype, z_range=None):
    """Same phantom evaluated with torch on ``device`` (float64 math, cast to ``dtype``).

    Used for large volumes, where the NumPy loop would take minutes.  The
    arithmetic is the blob formula only.  ``z_range=(z0, z1)`` returns only the
    planes z0 <= z < z1 of the volume (for volumes that are built slab by slab)."""
    import torch

    n0, n1, n2 = shape
    z0, z1 = (0, n0) if z_range is None else z_range
    ax = [torch.as_tensor(_axis(k), dtype=torch.float64, device=device) for k in (n0, n1, n2)]
    z, y, x = ax
    z = z[z0:z1]
    u = torch.zeros((z1 - z0, n1, n2), dtype=torch.float64, device=device)
    for c, s, a in zip(blobs.centres, blobs.sigmas, blobs.amps):
        gx = torch.exp(-((x - float(c[0])) ** 2) / (2 * s * s))
        gy = torch.exp(-((y - float(c[1])) ** 2) / (2 * s * s))
        gz = float(a) * torch.exp(-((z - float(c[2])) ** 2) / (2 * s * s))
        u += gz[:, None, None] * (gy[:, None] * gx[None, :])[None, :, :]
    if blobs.cube_values is not None:
        u += torch.as_tensor(_cube_layer(shape, blobs.cube_values)[z0:z1], device=device)
    return u.to(dtype)


def random_complex_torch(shape, seed: int, device, dtype):
    """Seeded i.i.d. N(0,1) real and imaginary parts drawn on ``device`` (torch generator)."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed)
    rdt = torch.float32 if dtype == torch.complex64 else torch.float64
    re = torch.randn(shape, generator=g, device=device, dtype=rdt)
    im = torch.randn(shape, generator=g, device=device, dtype=rdt)
    return torch.complex(re, im)


def random_complex(shape, seed: int) -> np.ndarray:
    """i.i.d. N(0,1) real and imaginary parts, complex128."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def random_detector_data(shape, seed: int) -> np.ndarray:
    """Random complex detector data for the adjoint test (seed + 200 by convention)."""
    return random_complex(shape, seed + 200)


def gaussian_noise(shape, seed: int, scale: float) -> np.ndarray:
    """Real Gaussian noise with standard deviation ``scale`` (seed + 100 by convention)."""
    rng = np.random.default_rng(seed + 100)
    return rng.standard_normal(shape) * scale


# The five workloads of the study, by name: volume edge, angles, tilt (deg),
# detector (h = w), blob count, cube layer, seed.  R = 2 and m = 4 throughout.
WORKLOADS = {
    "tiny32": dict(n=32, ntheta=32, phi_deg=20.0, det=32, nblobs=8, cubes=False, seed=1),
    "lam256": dict(n=256, ntheta=256, phi_deg=20.0, det=256, nblobs=32, cubes=False, seed=2),
    "lam512": dict(n=512, ntheta=512, phi_deg=30.0, det=512, nblobs=64, cubes=True, seed=3),
    "lam1024": dict(n=1024, ntheta=1024, phi_deg=20.0, det=1024, nblobs=256, cubes=False, seed=4),
    "lam2048": dict(n=2048, ntheta=2048, phi_deg=20.0, det=2048, nblobs=1024, cubes=False, seed=5),
    # the paper's 1.5K^3 shape (Section 6.1): transforms of 3 2^k points
    "lam1536": dict(n=1536, ntheta=1536, phi_deg=20.0, det=1536, nblobs=512, cubes=False, seed=6),
}
