"""Seeded synthetic inputs for the 3D SIFT-Rank hot path.

This module only draws random numbers and renders test volumes. It holds
none of the extraction method's arithmetic (no scale-space taps, no
difference of Gaussians, no extremum test, no descriptor): both the CPU
oracle and the GPU path receive the same bytes from here.

The paper evaluates on OASIS1 T1 brain MRI volumes of 145x174x145 voxels at
1 mm with about 2896 keypoints per volume (Materials & Methods, Experiments
and Data, dataset table). That dataset is not available here; the phantoms
below stand in for it with the same shape and a comparable keypoint count.

Volumes are float32 arrays indexed [z, y, x] (x fastest), shape (nz, ny, nx).

Recipes (all draws from numpy Generator(PCG64(seed))):

* ``noise_blob_volume`` (the "config-1 generator"): white noise N(0,1)
  smoothed by scipy's Gaussian filter (sigma 3, periodic edges), rescaled
  to standard deviation 0.05, plus isotropic Gaussian blobs with centres
  uniform in [margin, n-margin] per axis, sigma U[2,5] and amplitude
  +/-U[0.5,1.0] (sign 50/50).
* ``brain_phantom``: an ellipsoid with semi-axes (60, 75, 62) voxels in
  (x, y, z), three nested shells at ellipsoidal radius 1.0 / 0.8 / 0.55 with
  intensity 0.2 / 0.6 / 0.9, edges smoothed with sigma 1.5, a multiplicative
  bias field 1 + 0.15 f / max|f| (f = sum of three random cosines whose
  wavelength is at least the volume extent), 600 blobs inside the ellipsoid
  (sigma U[1.5,5], amplitude +/-U[0.1,0.4]) and additive N(0, 0.02^2) noise.
* ``pair_draws``: the standard-normal draws that the BRIEF/RRIEF point-pair
  selection consumes, shape (n, 2, 3) float64. How they are turned into
  point offsets is part of the method and is done by each side.
* ``similarity_copy``: a volume resampled under a known similarity
  transform T(x) = s R x + t (input voxel coordinates, x = (x, y, z)),
  B(y) = A(T^-1(y)) by scipy's cubic-spline affine_transform (outside A:
  0), optionally with fresh N(0, noise^2) noise and a smooth random
  displacement field (white noise smoothed with scipy's Gaussian filter,
  scaled to a given largest displacement). R comes from scipy's
  Rotation.from_rotvec(axis * angle); t keeps A's centre at B's centre.
  The stand-in for the paper's pairs of brain volumes: the true
  correspondences are known.
* ``hough_scene``: oriented keypoint geometry rows (x, y, z, sigma, R[9])
  for two point sets, the first n_true of A mapped into B by a planted
  similarity with small position, scale and frame noise, the rest random;
  frames from scipy's Rotation.random.
"""
from __future__ import annotations

import numpy as np
import scipy.ndimage as ndi

__all__ = [
    "noise_blob_volume",
    "brain_phantom",
    "pair_draws",
    "config1",
    "config2",
    "config3",
    "config4",
    "config5_requests",
    "similarity_copy",
    "hough_scene",
    "PAIR_SEED",
]

# Seed of the BRIEF/RRIEF point-pair draws used by every workload.
PAIR_SEED = 10258


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _add_blobs(vol: np.ndarray, centres: np.ndarray, sigmas: np.ndarray,
               amps: np.ndarray) -> None:
    """Add amp * exp(-|p - c|^2 / (2 s^2)) for each blob, in place (float64)."""
    nz, ny, nx = vol.shape
    for (cx, cy, cz), s, a in zip(centres, sigmas, amps):
        h = int(np.ceil(4.0 * s))
        x0, x1 = max(0, int(np.floor(cx)) - h), min(nx, int(np.floor(cx)) + h + 2)
        y0, y1 = max(0, int(np.floor(cy)) - h), min(ny, int(np.floor(cy)) + h + 2)
        z0, z1 = max(0, int(np.floor(cz)) - h), min(nz, int(np.floor(cz)) + h + 2)
        if x0 >= x1 or y0 >= y1 or z0 >= z1:
            continue
        gx = np.exp(-((np.arange(x0, x1) - cx) ** 2) / (2.0 * s * s))
        gy = np.exp(-((np.arange(y0, y1) - cy) ** 2) / (2.0 * s * s))
        gz = np.exp(-((np.arange(z0, z1) - cz) ** 2) / (2.0 * s * s))
        vol[z0:z1, y0:y1, x0:x1] += a * gz[:, None, None] * gy[None, :, None] * gx[None, None, :]


def noise_blob_volume(shape_xyz, seed: int, n_blobs: int | None = None,
                      margin: float = 12.0, blobs_per_voxel: float = 1.0 / 25000.0,
                      centre_range=None) -> np.ndarray:
    """Smoothed-noise volume with planted Gaussian blobs, float32 [z,y,x].

    ``shape_xyz`` is (nx, ny, nz). When ``n_blobs`` is None the count is
    ``round(nx*ny*nz*blobs_per_voxel)``. ``centre_range`` (lo, hi) overrides
    the per-axis centre interval [margin, n - margin].
    """
    nx, ny, nz = (int(v) for v in shape_xyz)
    rng = _rng(seed)
    noise = rng.standard_normal((nz, ny, nx), dtype=np.float32)
    noise = ndi.gaussian_filter(noise, 3.0, mode="wrap", truncate=4.0)
    noise *= np.float32(0.05 / max(float(noise.std(dtype=np.float64)), 1e-30))
    vol = noise.astype(np.float64)
    del noise
    if n_blobs is None:
        n_blobs = int(round(nx * ny * nz * blobs_per_voxel))
    if n_blobs > 0:
        dims = np.array([nx, ny, nz], dtype=np.float64)
        if centre_range is not None:
            lo = np.full(3, float(centre_range[0]))
            hi = np.full(3, float(centre_range[1]))
        else:
            lo = np.full(3, margin)
            hi = dims - margin
        centres = lo + (hi - lo) * rng.random((n_blobs, 3))
        sigmas = rng.uniform(2.0, 5.0, n_blobs)
        amps = rng.uniform(0.5, 1.0, n_blobs) * np.where(rng.random(n_blobs) < 0.5, -1.0, 1.0)
        _add_blobs(vol, centres, sigmas, amps)
    return np.ascontiguousarray(vol.astype(np.float32))


def brain_phantom(seed: int, shape_xyz=(145, 174, 145), semi_axes=(60.0, 75.0, 62.0),
                  n_blobs: int = 600) -> np.ndarray:
    """Brain-like ellipsoidal phantom, float32 [z,y,x] (recipe in module doc)."""
    nx, ny, nz = shape_xyz
    rng = _rng(seed)
    c = np.array([(nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0])
    ax, ay, az = semi_axes
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    rho = np.sqrt(((x - c[0]) / ax) ** 2 + ((y - c[1]) / ay) ** 2 + ((z - c[2]) / az) ** 2)
    lab = np.zeros((nz, ny, nx), dtype=np.float64)
    lab[rho < 1.0] = 0.2
    lab[rho < 0.8] = 0.6
    lab[rho < 0.55] = 0.9
    vol = ndi.gaussian_filter(lab, 1.5, mode="nearest", truncate=4.0)
    # low-frequency multiplicative bias field
    f = np.zeros_like(vol)
    ext = np.array([nx, ny, nz], dtype=np.float64)
    for _ in range(3):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        lam = ext.max() * rng.uniform(1.0, 2.0)
        ph = rng.uniform(0.0, 2.0 * np.pi)
        f += np.cos(2.0 * np.pi * (d[0] * x + d[1] * y + d[2] * z) / lam + ph)
    vol *= 1.0 + 0.15 * f / max(np.abs(f).max(), 1e-30)
    # blobs inside the ellipsoid (rejection sampling of centres)
    centres = []
    while len(centres) < n_blobs:
        p = rng.uniform(-1.0, 1.0, 3)
        if p @ p < 0.9 ** 2:
            centres.append(c + p * np.array([ax, ay, az]))
    centres = np.array(centres)
    sigmas = rng.uniform(1.5, 5.0, n_blobs)
    amps = rng.uniform(0.1, 0.4, n_blobs) * np.where(rng.random(n_blobs) < 0.5, -1.0, 1.0)
    _add_blobs(vol, centres, sigmas, amps)
    vol += rng.normal(0.0, 0.02, vol.shape)
    return np.ascontiguousarray(vol.astype(np.float32))


def pair_draws(seed: int = PAIR_SEED, n: int = 256) -> np.ndarray:
    """Standard-normal draws for n point pairs, float64 of shape (n, 2, 3).

    Entry [i, 0] and [i, 1] are two independent N(0, I3) vectors; the
    point-pair selection methods build their pair offsets from them.
    """
    return _rng(seed).standard_normal((int(n), 2, 3))


# --- the named workloads -------------------------------------------------

def config1(seed: int = 1) -> np.ndarray:
    """64^3 smoothed noise + 24 blobs with centres U[12,52]^3."""
    return noise_blob_volume((64, 64, 64), seed, n_blobs=24, centre_range=(12.0, 52.0))


def config2(seed: int = 2) -> np.ndarray:
    """145x174x145 brain-like phantom."""
    return brain_phantom(seed)


def config3(n: int = 32, seed0: int = 3000):
    """n volumes with each axis length drawn from U{96..192}."""
    vols = []
    for i in range(n):
        rng = _rng(seed0 + i)
        shape = tuple(int(v) for v in rng.integers(96, 193, 3))
        vols.append(noise_blob_volume(shape, seed0 + i))
    return vols


def config4(seed: int = 4) -> np.ndarray:
    """512x512x384 smoothed noise with about 4000 blobs."""
    return noise_blob_volume((512, 512, 384), seed, n_blobs=4000)


CONFIG5_SIZES = ((64, 64, 64), (145, 174, 145), (192, 224, 192), (256, 256, 256))
CONFIG5_PROBS = (0.2, 0.5, 0.2, 0.1)


def config5_requests(n: int = 2000, rate: float = 200.0, seed: int = 5000):
    """Arrival times (s) and sizes of a Poisson request stream.

    Returns a list of (arrival_s, shape_xyz, volume_seed); the volume for a
    request is ``noise_blob_volume(shape_xyz, volume_seed)``.
    """
    rng = _rng(seed)
    gaps = rng.exponential(1.0 / rate, n)
    t = np.cumsum(gaps) - gaps[0]
    idx = rng.choice(len(CONFIG5_SIZES), size=n, p=CONFIG5_PROBS)
    return [(float(t[i]), CONFIG5_SIZES[int(idx[i])], seed + i) for i in range(n)]


# --- pairs with known correspondences -------------------------------------

def _rotation(axis, angle):
    from scipy.spatial.transform import Rotation
    a = np.asarray(axis, dtype=np.float64)
    return Rotation.from_rotvec(a / np.linalg.norm(a) * float(angle)).as_matrix()


def similarity_copy(vol: np.ndarray, scale: float = 1.0, axis=(0.3, -0.5, 0.8), angle_deg: float = 20.0,
                    noise: float = 0.0, seed: int = 7, warp: float = 0.0, warp_sigma: float = 12.0):
    """(vol_b, s, R, t): vol resampled under T(x) = s R x + t (recipe in the
    module doc). Shape unchanged; t = c - s R c with c the volume centre.
    warp > 0 adds a smooth random displacement u (white noise smoothed with
    sigma warp_sigma voxels, each component scaled to a largest magnitude of
    warp voxels): B(y) = A(T^-1(y) + u(y)), a stand-in for the anatomical
    differences between two subjects on top of the global similarity."""
    nz, ny, nx = vol.shape
    R = _rotation(axis, np.deg2rad(angle_deg))
    s = float(scale)
    c = np.array([(nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0])
    t = c - s * (R @ c)
    # output index o (z, y, x) reads input T^-1: x_a = R^T (x_b - t) / s
    P = np.array([[0, 0, 1], [0, 1, 0], [1, 0, 0]], dtype=np.float64)
    M = P @ (R.T / s) @ P
    off = P @ (-(R.T @ t) / s)
    if warp > 0.0:
        rng = _rng(seed + 1)
        z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        coords = np.stack([z, y, x]).reshape(3, -1).astype(np.float64)
        src = M @ coords + off[:, None]
        for k in range(3):
            u = ndi.gaussian_filter(rng.standard_normal((nz, ny, nx)), warp_sigma, mode="wrap")
            src[k] += warp * u.reshape(-1) / max(np.abs(u).max(), 1e-30)
        out = ndi.map_coordinates(vol.astype(np.float64), src, order=3, mode="constant", cval=0.0).reshape(nz, ny, nx)
    else:
        out = ndi.affine_transform(vol.astype(np.float64), M, offset=off, order=3, mode="constant", cval=0.0)
    if noise > 0.0:
        out = out + _rng(seed).normal(0.0, noise, out.shape)
    return np.ascontiguousarray(out.astype(np.float32)), s, R, t


def hough_scene(n_true: int, n_false: int, seed: int, scale: float = 1.3, axis=(1.0, 2.0, -0.5),
                angle_deg: float = 35.0, shift=(12.0, -7.0, 5.0), extent=(145.0, 174.0, 145.0),
                pos_noise: float = 0.3, frame_noise_deg: float = 3.0):
    """Synthetic matched geometry for the Hough vote.

    Returns (geo_a [n][13] float32, geo_b [n][13] float32, match [n] int32,
    truth dict(s, R, t)). Row i of A matches row match[i] of B (a random
    permutation). A's positions are uniform in the extent, sigma is
    1.6 * 2^U[0, 3], frames are random rotations. For i < n_true the B row
    is (s R x + t + N(0, pos_noise^2) per axis, s sigma, R_noise R R_a) with
    R_noise a rotation of N(0, frame_noise_deg^2) degrees about a random
    axis; the other B rows are independent random keypoints.
    """
    from scipy.spatial.transform import Rotation
    rng = _rng(seed)
    n = int(n_true) + int(n_false)
    R = _rotation(axis, np.deg2rad(angle_deg))
    s = float(scale)
    ext = np.asarray(extent, dtype=np.float64)
    xa = rng.random((n, 3)) * ext
    sa = 1.6 * 2.0 ** rng.uniform(0.0, 3.0, n)
    Ra = Rotation.random(n, random_state=rng).as_matrix()
    c = (ext - 1.0) / 2.0
    t = c - s * (R @ c) + np.asarray(shift, dtype=np.float64)
    xb = rng.random((n, 3)) * ext
    sb = 1.6 * 2.0 ** rng.uniform(0.0, 3.0, n)
    Rb = Rotation.random(n, random_state=rng).as_matrix()
    for i in range(int(n_true)):
        ax = rng.standard_normal(3)
        Rn = _rotation(ax, np.deg2rad(frame_noise_deg * rng.standard_normal()))
        xb[i] = s * (R @ xa[i]) + t + rng.normal(0.0, pos_noise, 3)
        sb[i] = s * sa[i]
        Rb[i] = Rn @ R @ Ra[i]
    perm = rng.permutation(n)          # B row of pair i is perm[i]
    geo_a = np.zeros((n, 13), dtype=np.float32)
    geo_b = np.zeros((n, 13), dtype=np.float32)
    geo_a[:, :3], geo_a[:, 3], geo_a[:, 4:] = xa, sa, Ra.reshape(n, 9)
    geo_b[perm, :3], geo_b[perm, 3], geo_b[perm, 4:] = xb, sb, Rb.reshape(n, 9)
    return geo_a, geo_b, perm.astype(np.int32), {"s": s, "R": R, "t": t}
