"""Closed-form detector data of a Gaussian-blob phantom (test helper, pure mathematics).

The laminography data at detector point (p, v) of angle theta is the line integral of the
volume along the beam direction a x b through the point p a + v b (a, b the detector axes of
the Fourier-slice geometry, in units of the volume side), times N for voxel units.  For a blob
A exp(-|r - c|^2 / (2 s^2)) the integral over the beam's segment inside the volume's cube
[-1/2, 1/2)^3 is A exp(-d^2 / (2 s^2)) s sqrt(pi/2) [erf((t1 - tc) / (s sqrt 2)) - erf((t0 - tc) / (s sqrt 2))],
with d the distance of the centre from the beam, tc the centre's position along it and
[t0, t1] the segment.  The discrete operator's detector is periodic with the volume's period
(w / N = 1 in these units), and the cube's shadow is wider than that, so the data sum the
neighbouring images of the detector point.  Against the FP64 oracle the residual is the
voxel sampling of the truncated blobs, falling as 1/N.
"""
import numpy as np
from scipy.special import erf


def _axes(theta, phi):
    a = np.stack([np.cos(theta), np.sin(theta), np.zeros_like(theta)], -1)             # (x, y, z)
    b = np.stack([np.sin(phi) * np.sin(theta), -np.sin(phi) * np.cos(theta),
                  np.full_like(theta, np.cos(phi))], -1)
    return a, b, np.cross(a, b)


def _segment(o, d):
    """Parameter interval [t0, t1] of the lines o + t d inside [-1/2, 1/2)^3 (empty: t0 = t1)."""
    lo = np.full(len(o), -np.inf)
    hi = np.full(len(o), np.inf)
    empty = np.zeros(len(o), bool)
    for k in range(3):
        dk = d[:, k]
        par = np.abs(dk) <= 1e-12
        safe = np.where(par, 1.0, dk)
        t1 = (-0.5 - o[:, k]) / safe
        t2 = (0.5 - o[:, k]) / safe
        lo = np.where(par, lo, np.maximum(lo, np.minimum(t1, t2)))
        hi = np.where(par, hi, np.minimum(hi, np.maximum(t1, t2)))
        empty |= par & ((o[:, k] < -0.5) | (o[:, k] >= 0.5))   # parallel to the faces, outside
    empty |= hi <= lo
    return np.where(empty, 0.0, lo), np.where(empty, 0.0, hi)


def blob_data(blobs, n, thetas, phi, p, v):
    """Data at points (thetas[i], p[i], v[i]) (p, v in units of the volume side, centred) of an
    n^3 volume holding `blobs` (centres as (x, y, z) in [-1/2, 1/2)), in voxel units."""
    a, b, d = _axes(np.asarray(thetas, float), phi)
    out = np.zeros(len(p))
    for iv in (-1, 0, 1):
        for iu in (-1, 0, 1):
            o = (p + iu)[:, None] * a + (v + iv)[:, None] * b
            t0, t1 = _segment(o, d)
            for c, s, amp in zip(blobs.centres, blobs.sigmas, blobs.amps):
                rel = np.asarray(c)[None, :] - o
                tc = (rel * d).sum(-1)
                dist2 = (rel * rel).sum(-1) - tc * tc
                out += amp * np.exp(-dist2 / (2 * s * s)) * s * np.sqrt(np.pi / 2) * (
                    erf((t1 - tc) / (s * np.sqrt(2))) - erf((t0 - tc) / (s * np.sqrt(2))))
    return n * out
