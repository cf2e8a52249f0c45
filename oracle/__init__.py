"""FP64 CPU oracle of the 3D SIFT-Rank hot path -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package. The product library never calls it and shares no code
with it. The arithmetic lives in ``sift3d_oracle.c`` (plain loops, double
precision); this module is the orchestration, written step by step in the
order of the paper (Carluer et al., arXiv 2112.10258):

1. Gaussian scale space by incremental separable blurring (Related Work:
   recursive Gaussian filtering by separable 1D filters; Section 3.2.2,
   Gaussian Convolution).
2. Difference of Gaussians between consecutive levels (Section 3.2.2,
   Difference-of-Gaussian).
3. 2x sub-sampling by the mean of 2x2x2 blocks into the next octave
   (Section 3.2.2, Sub-sampling).
4. 4D extremum detection by the sum of signs over 80 neighbours with the
   peak/valley values +/-80 (Section 3.2.2, 4D Peak Detection).
5. Descriptors: upright SIFT-Rank (Related Work: 2x2x2 spatial x 8
   orientation bins, ranked), BRIEF and RRIEF with any of the five point-pair
   methods and a Gaussian patch pre-blur (Section 3.2.3); dominant
   orientations from a discrete spherical gradient histogram and SIFT-Rank
   after reorientation (Related Work, 3D SIFT-Rank).
6. Beside the path: nearest-neighbour matching of descriptors (Section 3.3)
   and the uniform-filter approximation of the Gaussian blur (Related Work).

Readings where the paper is silent are listed in the design notes; each is
named here where it is applied (R-numbers).

Parity status: every function here is pinned by tests/test_oracle_pins.py
(closed forms, brute force on tiny inputs, invariants, planted blobs).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sift3d_oracle.c")
_LIB = os.path.join(_HERE, "libsift3d_oracle.so")

KEYPOINT_DTYPE = np.dtype([
    ("x", "<i4"), ("y", "<i4"), ("z", "<i4"),
    ("octave", "<i2"), ("scale", "<i2"), ("polarity", "i1"), ("pad", "i1", (3,)),
    ("dog", "<f4"), ("xf", "<f4"), ("yf", "<f4"), ("zf", "<f4"), ("sigma", "<f4"),
])


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (strict IEEE double, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-shared", "-fPIC", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def _L():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.orc_gauss_taps.restype = ctypes.c_int
        lib.orc_gauss_taps.argtypes = [ctypes.c_double, ctypes.c_double, dp, ctypes.c_int]
        lib.orc_blur_axis.argtypes = [dp, dp] + [ctypes.c_int] * 4 + [dp, ctypes.c_int]
        lib.orc_blur.restype = ctypes.c_int
        lib.orc_blur.argtypes = [dp, dp, dp] + [ctypes.c_int] * 3 + [ctypes.c_double] * 2
        lib.orc_dog.argtypes = [dp, dp, dp, ctypes.c_size_t]
        lib.orc_subsample.argtypes = [dp] + [ctypes.c_int] * 3 + [dp]
        lib.orc_sum_of_signs.restype = ctypes.c_int
        lib.orc_sum_of_signs.argtypes = [dp, dp, dp] + [ctypes.c_int] * 6
        lib.orc_detect.restype = ctypes.c_long
        lib.orc_detect.argtypes = [dp, dp, dp] + [ctypes.c_int] * 3 + [ctypes.c_double, ctypes.c_int,
                                                                       ip, ctypes.c_long]
        lib.orc_rank.argtypes = [dp, ctypes.c_int, ip]
        lib.orc_siftrank.argtypes = [dp] + [ctypes.c_int] * 3 + [ip, ctypes.c_long, ctypes.c_int,
                                                                 dp, ctypes.c_void_p]
        lib.orc_brief_rrief.argtypes = [dp] + [ctypes.c_int] * 3 + [ip, ctypes.c_long, ip, ctypes.c_int,
                                                                    dp, ctypes.c_int, dp,
                                                                    ctypes.c_void_p, ctypes.c_void_p]
        lib.orc_orient.argtypes = [dp] + [ctypes.c_int] * 3 + [ip, ctypes.c_long, ctypes.c_int, ctypes.c_double,
                                                               ctypes.c_int, ip, dp, dp, ctypes.c_void_p, dp]
        lib.orc_siftrank_frames.argtypes = [dp] + [ctypes.c_int] * 3 + [ip, ctypes.c_long, ctypes.c_int, dp, dp,
                                                                        ctypes.c_void_p, dp]
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        lib.orc_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def set_threads(n: int) -> None:
    _L().orc_set_threads(int(n))


def max_threads() -> int:
    return int(_L().orc_max_threads())


@dataclass
class Params:
    """Method parameters; defaults are the readings used on the hot path."""
    n_octaves: int = 0          # 0: keep octave o while min(dims_o) >= min_dim (R7)
    min_dim: int = 16
    scales: int = 3             # S; S+3 Gaussian and S+2 DoG levels per octave (R1)
    sigma0: float = 1.6
    sigma_in: float = 0.0       # blur already present in the input (R5)
    trunc: float = 3.0          # tap radius = ceil(trunc * sigma) (R2)
    dog_threshold: float = 0.01  # strict |D| > t
    votes: int = 80             # sum-of-signs acceptance |f| >= votes (R9)
    brief_n: int = 256          # pairs per BRIEF/RRIEF descriptor (R14)
    brief_blur: float = 0.95    # patch pre-blur sigma_b, octave voxels (R16)
    siftrank_factor: float = 2.0  # SIFT-Rank window half-width R = ceil(f * sigma_s) (R11)
    brief_method: int = 3       # point-pair selection method 1..5 (Section 3.2.3; R15, R21-R23)


# ---------------------------------------------------------------- primitives

def gauss_taps(sigma: float, trunc: float = 3.0) -> np.ndarray:
    """Normalised sampled Gaussian, length 2*ceil(trunc*sigma)+1 (R2)."""
    w = np.zeros(127)
    r = _L().orc_gauss_taps(float(sigma), float(trunc), _dp(w), 127)
    if r < 0:
        raise ValueError("filter too long")
    return w[: 2 * r + 1].copy()


def blur_axis(vol: np.ndarray, w: np.ndarray, axis: int) -> np.ndarray:
    """One clamp-to-edge 1D pass; axis 0 = x, 1 = y, 2 = z of a [z,y,x] array."""
    v = _f64(vol)
    out = np.empty_like(v)
    w = _f64(w)
    r = (len(w) - 1) // 2
    nz, ny, nx = v.shape
    _L().orc_blur_axis(_dp(v), _dp(out), nx, ny, nz, int(axis), _dp(w), r)
    return out


def blur(vol: np.ndarray, sigma: float, trunc: float = 3.0) -> np.ndarray:
    """Separable Gaussian blur x -> y -> z with clamp-to-edge (R3)."""
    v = _f64(vol)
    out = np.empty_like(v)
    tmp = np.empty_like(v)
    nz, ny, nx = v.shape
    if _L().orc_blur(_dp(v), _dp(out), _dp(tmp), nx, ny, nz, float(sigma), float(trunc)) < 0:
        raise ValueError("filter too long")
    return out


def dog(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """D = a - b, a the finer level (R4)."""
    a = _f64(a)
    b = _f64(b)
    d = np.empty_like(a)
    _L().orc_dog(_dp(a), _dp(b), _dp(d), a.size)
    return d


def subsample(vol: np.ndarray) -> np.ndarray:
    """Mean of each 2x2x2 block; output dims floor(n/2) (R6)."""
    v = _f64(vol)
    nz, ny, nx = v.shape
    out = np.empty((nz // 2, ny // 2, nx // 2))
    _L().orc_subsample(_dp(v), nx, ny, nz, _dp(out))
    return out


def sum_of_signs(dm, d0, dp, x: int, y: int, z: int) -> int:
    dm, d0, dp = _f64(dm), _f64(d0), _f64(dp)
    nz, ny, nx = d0.shape
    return int(_L().orc_sum_of_signs(_dp(dm), _dp(d0), _dp(dp), nx, ny, nz, x, y, z))


def detect_triple(dm, d0, dp, thr: float, votes: int) -> np.ndarray:
    """Rows (x, y, z, polarity) of extrema of the middle level, z-y-x order."""
    dm, d0, dp = _f64(dm), _f64(d0), _f64(dp)
    nz, ny, nx = d0.shape
    cap = 1 << 16
    while True:
        out = np.zeros((cap, 4), dtype=np.int32)
        n = _L().orc_detect(_dp(dm), _dp(d0), _dp(dp), nx, ny, nz, float(thr), int(votes), _ip(out), cap)
        if n <= cap:
            return out[:n].copy()
        cap = int(n)


def rank(v: np.ndarray) -> np.ndarray:
    v = _f64(v)
    r = np.zeros(len(v), dtype=np.int32)
    _L().orc_rank(_dp(v), len(v), _ip(r))
    return r


def siftrank(G: np.ndarray, kp_xyz: np.ndarray, R: int):
    """(hist [K,64] float64, rank [K,64] uint8) for keypoints on level G."""
    G = _f64(G)
    kp = np.ascontiguousarray(kp_xyz, dtype=np.int32).reshape(-1, 3)
    K = len(kp)
    hist = np.zeros((K, 64))
    rk = np.zeros((K, 64), dtype=np.uint8)
    nz, ny, nx = G.shape
    if K:
        _L().orc_siftrank(_dp(G), nx, ny, nz, _ip(kp), K, int(R), _dp(hist), rk.ctypes.data)
    return hist, rk


ORIENT_TAU = 0.8      # peak threshold relative to the histogram maximum (reading R25)
ORIENT_KMAX = 4       # frames kept per keypoint


def orient(G: np.ndarray, kp_xyz: np.ndarray, R: int, tau: float = ORIENT_TAU, kmax: int = ORIENT_KMAX):
    """Dominant orientations and oriented SIFT-Rank (Related Work, 3D
    SIFT-Rank; reading R25, see orc_orient). Returns a dict: nframes [K],
    frames [K, kmax, 3, 3] (columns e1, e2, e3), hist [K, kmax, 64],
    rank [K, kmax, 64] uint8, margin [K]."""
    G = _f64(G)
    kp = np.ascontiguousarray(kp_xyz, dtype=np.int32).reshape(-1, 3)
    K = len(kp)
    nf = np.zeros(K, dtype=np.int32)
    fr = np.zeros((K, kmax, 3, 3))
    hist = np.zeros((K, kmax, 64))
    rk = np.zeros((K, kmax, 64), dtype=np.uint8)
    mg = np.zeros(K)
    nz, ny, nx = G.shape
    if K:
        _L().orc_orient(_dp(G), nx, ny, nz, _ip(kp), K, int(R), float(tau), int(kmax), _ip(nf), _dp(fr),
                        _dp(hist), rk.ctypes.data, _dp(mg))
    return {"nframes": nf, "frames": fr, "hist": hist, "rank": rk, "margin": mg}


def siftrank_frames(G: np.ndarray, kp_xyz: np.ndarray, R: int, frames: np.ndarray):
    """SIFT-Rank of keypoints in given frames [K, 3, 3] (columns = axes):
    (hist [K,64], rank [K,64] uint8, margin [K]); the identity frame gives
    the upright descriptor."""
    G = _f64(G)
    kp = np.ascontiguousarray(kp_xyz, dtype=np.int32).reshape(-1, 3)
    K = len(kp)
    F = np.ascontiguousarray(frames, dtype=np.float64).reshape(K, 9)
    hist = np.zeros((K, 64))
    rk = np.zeros((K, 64), dtype=np.uint8)
    mg = np.zeros(K)
    nz, ny, nx = G.shape
    if K:
        _L().orc_siftrank_frames(_dp(G), nx, ny, nz, _ip(kp), K, int(R), _dp(F), _dp(hist), rk.ctypes.data, _dp(mg))
    return hist, rk, mg


def orientations(G_levels, kps: np.ndarray, p: "Params", tau: float = ORIENT_TAU, kmax: int = ORIENT_KMAX):
    """orient() for every keypoint on G_s of its octave with the SIFT-Rank
    window half-width of its scale."""
    K = len(kps)
    out = {"nframes": np.zeros(K, dtype=np.int32), "frames": np.zeros((K, kmax, 3, 3)),
           "hist": np.zeros((K, kmax, 64)), "rank": np.zeros((K, kmax, 64), dtype=np.uint8),
           "margin": np.zeros(K)}
    for o, G in enumerate(G_levels):
        for s in range(1, p.scales + 1):
            sel = np.nonzero((kps["octave"] == o) & (kps["scale"] == s))[0]
            if len(sel) == 0:
                continue
            xyz = np.stack([kps["x"][sel], kps["y"][sel], kps["z"][sel]], axis=1)
            r = orient(G[s], xyz, siftrank_radius(p, s), tau, kmax)
            for k in out:
                out[k][sel] = r[k]
    return out


def brief_rrief(G: np.ndarray, kp_xyz: np.ndarray, offsets: np.ndarray, wb: np.ndarray):
    """(d [K,n] float64, bits [K,n/64] uint64, ranks [K,n] uint16)."""
    G = _f64(G)
    kp = np.ascontiguousarray(kp_xyz, dtype=np.int32).reshape(-1, 3)
    off = np.ascontiguousarray(offsets, dtype=np.int32).reshape(-1, 2, 3)
    n = len(off)
    wb = _f64(wb)
    rb = (len(wb) - 1) // 2
    K = len(kp)
    nw = (n + 63) // 64
    d = np.zeros((K, n))
    bits = np.zeros((K, nw), dtype=np.uint64)
    rk = np.zeros((K, n), dtype=np.uint16)
    nz, ny, nx = G.shape
    if K:
        _L().orc_brief_rrief(_dp(G), nx, ny, nz, _ip(kp), K, _ip(off), n, _dp(wb), rb,
                             _dp(d), bits.ctypes.data, rk.ctypes.data)
    return d, bits, rk


# ---------------------------------------------------------------- schedule

def scale_sigma(p: Params, s: float) -> float:
    """Blur of level s of an octave, in that octave's voxels: sigma0 * 2^(s/S)."""
    return p.sigma0 * 2.0 ** (s / p.scales)


def level_increments(p: Params):
    """(sigma of the first blur of octave 0, [incremental sigma of G_1..G_{S+2}]).

    Level i of an octave has total blur sigma0 * kappa^i, kappa = 2^(1/S);
    G_i is G_{i-1} blurred by sqrt(total_i^2 - total_{i-1}^2) (R1, R5).
    """
    base = math.sqrt(p.sigma0 ** 2 - p.sigma_in ** 2)
    inc = []
    for i in range(1, p.scales + 3):
        a, b = scale_sigma(p, i), scale_sigma(p, i - 1)
        inc.append(math.sqrt(a * a - b * b))
    return base, inc


def octave_dims(shape_xyz, p: Params):
    """Dims (nx, ny, nz) of each octave: halve (floor) while min >= min_dim (R7)."""
    nx, ny, nz = (int(v) for v in shape_xyz)
    dims = []
    while min(nx, ny, nz) >= p.min_dim:
        if p.n_octaves > 0 and len(dims) == p.n_octaves:
            break
        dims.append((nx, ny, nz))
        nx, ny, nz = nx // 2, ny // 2, nz // 2
    return dims


def siftrank_radius(p: Params, s: int) -> int:
    return int(math.ceil(p.siftrank_factor * scale_sigma(p, s)))


def _chi3_cdf(x: float) -> float:
    """P(|z|^2 <= x) for z ~ N(0, I_3): the chi-square CDF with 3 degrees of freedom."""
    return math.erf(math.sqrt(x / 2.0)) - math.sqrt(2.0 * x / math.pi) * math.exp(-x / 2.0)


def pair_points(draws: np.ndarray, p: Params, s: int) -> np.ndarray:
    """Real-valued (x,y,z) points (p1, p2) of the n pairs at scale s, [n][2][3].

    The five selection methods of Section 3.2.3, with sigma the keypoint
    scale in octave voxels (R13) and the pair draws (z1, z2), two
    standard-normal 3-vectors per pair, as the only randomness (R15):
      1: p1, p2 uniform in the ball of radius 2 sigma (R21). A point is
         direction z/|z| times radius 2 sigma F(|w|^2)^(1/3), F the
         chi-square(3) CDF, so F(|w|^2) is uniform; p1 takes z1's direction
         and z2's norm, p2 the reverse (direction and norm of a normal
         vector are independent, so p1 and p2 are independent);
      2: p1 = sigma z1, p2 = sigma z2;
      3: p1 = sigma z1, p2 = p1 + sigma z2;
      4: p1 = 0, p2 = sigma z2 (R22);
      5: p1 = 0, p2 on a regular spherical grid: n/64 radii
         2 sigma (k+1)/(n/64), 8 polar angles pi (j + 1/2)/8, 8 azimuths
         2 pi (i + (j mod 2)/2)/8, pair 64 k + 8 j + i (R23).
    """
    z = np.asarray(draws, dtype=np.float64).reshape(-1, 2, 3)[: p.brief_n]
    n = len(z)
    sig = scale_sigma(p, s)
    out = np.zeros((n, 2, 3))
    m = p.brief_method
    if m == 1:
        for i in range(n):
            a, b = z[i, 0], z[i, 1]
            na, nb = float(np.sqrt(a @ a)), float(np.sqrt(b @ b))
            if na > 0:
                out[i, 0] = a / na * (2.0 * sig * np.cbrt(_chi3_cdf(nb * nb)))
            if nb > 0:
                out[i, 1] = b / nb * (2.0 * sig * np.cbrt(_chi3_cdf(na * na)))
    elif m == 2:
        out[:, 0] = sig * z[:, 0]
        out[:, 1] = sig * z[:, 1]
    elif m == 3:
        out[:, 0] = sig * z[:, 0]
        out[:, 1] = sig * (z[:, 0] + z[:, 1])
    elif m == 4:
        out[:, 1] = sig * z[:, 1]
    elif m == 5:
        nr = max(1, p.brief_n // 64)
        for q in range(n):
            k, j, i = q // 64, (q // 8) % 8, q % 8
            r = 2.0 * sig * (k + 1) / nr
            th = math.pi * (j + 0.5) / 8.0
            ph = 2.0 * math.pi * (i + 0.5 * (j % 2)) / 8.0
            out[q, 1] = (r * math.sin(th) * math.cos(ph), r * math.sin(th) * math.sin(ph), r * math.cos(th))
    else:
        raise ValueError("brief_method must be 1..5")
    return out


def pair_offsets(draws: np.ndarray, p: Params, s: int) -> np.ndarray:
    """Integer (x,y,z) offsets of the pairs at scale s, [n][2][3]: each point
    of pair_points rounded to the nearest voxel, floor(c + 0.5)."""
    return np.floor(pair_points(draws, p, s) + 0.5).astype(np.int32)


# ---------------------------------------------------------------- matching

def match_nn(A: np.ndarray, B: np.ndarray, kind: int):
    """Nearest neighbour in B of every descriptor of A, by brute force.

    The descriptors' consumer (Section 3.3: keypoints are matched by their
    descriptors). kind 0: binary BRIEF words [n][w] (uint64), distance =
    Hamming distance; kind 1 / 2: rank vectors [n][m] (uint8, SIFT-Rank /
    RRIEF), distance = squared Euclidean distance of the rank vectors (rank
    vectors all have the same norm, so this orders neighbours exactly as
    the distance of the unit-length normalised vectors does). Returns
    (idx, d1, d2): the index of the nearest element of B (the lowest index
    among equal distances; -1 when B is empty), its distance, and the
    second-smallest distance over the other elements of B (2^31 - 1 when B
    has fewer than two elements).
    """
    A = np.asarray(A)
    B = np.asarray(B)
    na, nb = len(A), len(B)
    big = 2 ** 31 - 1
    idx = np.full(na, -1, dtype=np.int64)
    d1 = np.full(na, big, dtype=np.int64)
    d2 = np.full(na, big, dtype=np.int64)
    for i in range(na):
        if kind == 0:
            x = np.bitwise_xor(A[i].astype(np.uint64)[None, :], B.astype(np.uint64))
            d = np.array([sum(bin(int(w)).count("1") for w in row) for row in x], dtype=np.int64)
        else:
            diff = A[i].astype(np.int64)[None, :] - B.astype(np.int64)
            d = (diff * diff).sum(axis=1)
        if nb == 0:
            continue
        j = int(np.argmin(d))            # first occurrence: the lowest index
        idx[i], d1[i] = j, d[j]
        if nb > 1:
            d2[i] = np.min(np.delete(d, j))
    return idx, d1, d2


def box_half_width(sigma: float, passes: int) -> int:
    """Half-width h of the uniform filter (width 2h+1) whose `passes`-fold
    repetition stands in for a Gaussian of standard deviation sigma (Related
    Work: the scale space can also be built from uniform 1D filters; R24).
    A width-w uniform filter has variance (w^2 - 1)/12, so the ideal width
    of one of m equal passes is sqrt(12 sigma^2 / m + 1); h is the nearest
    integer to (that width - 1) / 2."""
    if sigma < 0 or passes < 1:
        raise ValueError("sigma >= 0 and passes >= 1")
    return int(math.floor((math.sqrt(12.0 * sigma * sigma / passes + 1.0) - 1.0) / 2.0 + 0.5))


def box_axis(vol: np.ndarray, h: int, axis: int) -> np.ndarray:
    """One clamp-to-edge uniform pass along axis (0 = x, 1 = y, 2 = z of a
    [z,y,x] array): each output is the mean of the 2h+1 samples centred on
    it, indices outside the volume clamped to the nearest edge (R24)."""
    v = _f64(vol)
    a = {0: 2, 1: 1, 2: 0}[axis]
    n = v.shape[a]
    acc = np.zeros_like(v)
    for j in range(-h, h + 1):
        acc += np.take(v, np.clip(np.arange(n) + j, 0, n - 1), axis=a)
    return acc / (2 * h + 1)


def box_blur(vol: np.ndarray, h: int, passes: int) -> np.ndarray:
    """Uniform-filter approximation of a separable Gaussian blur (R24):
    `passes` uniform passes of half-width h along x, then along y, then
    along z."""
    v = _f64(vol)
    for axis in (0, 1, 2):
        for _ in range(passes):
            v = box_axis(v, h, axis)
    return v


# ---------------------------------------------------------------- pipeline

@dataclass
class Octave:
    dims: tuple
    G: list = field(default_factory=list)   # S+3 arrays [z,y,x] float64
    D: list = field(default_factory=list)   # S+2 arrays


def pyramid(vol: np.ndarray, p: Params):
    """Gaussian and DoG levels of every octave (steps 1-3)."""
    nz, ny, nx = vol.shape
    dims = octave_dims((nx, ny, nz), p)
    if not dims:
        raise ValueError("volume smaller than min_dim: no octave")
    base, inc = level_increments(p)
    octs = []
    for o, d in enumerate(dims):
        oc = Octave(d)
        if o == 0:
            oc.G.append(blur(vol, base, p.trunc))
        else:
            oc.G.append(subsample(octs[o - 1].G[p.scales]))
            assert oc.G[0].shape == (d[2], d[1], d[0])
        for i in range(1, p.scales + 3):
            oc.G.append(blur(oc.G[i - 1], inc[i - 1], p.trunc))
        for i in range(p.scales + 2):
            oc.D.append(dog(oc.G[i], oc.G[i + 1]))
        octs.append(oc)
    return octs


def detect(D_levels, p: Params) -> np.ndarray:
    """Keypoints of every octave in canonical (octave, scale, z, y, x) order.

    ``D_levels[o]`` is the list of S+2 DoG arrays of octave o. Input-space
    position x_in = 2^o x + (2^o - 1)/2 (centre of the 2x2x2 means) and
    sigma_in = sigma0 * 2^(s/S) * 2^o (R10).
    """
    rows = []
    for o, D in enumerate(D_levels):
        for s in range(1, p.scales + 1):
            r = detect_triple(D[s - 1], D[s], D[s + 1], p.dog_threshold, p.votes)
            if len(r) == 0:
                continue
            kp = np.zeros(len(r), dtype=KEYPOINT_DTYPE)
            kp["x"], kp["y"], kp["z"] = r[:, 0], r[:, 1], r[:, 2]
            kp["octave"], kp["scale"], kp["polarity"] = o, s, r[:, 3]
            Ds = _f64(D[s])
            kp["dog"] = Ds[r[:, 2], r[:, 1], r[:, 0]]
            f = 2.0 ** o
            kp["xf"] = f * r[:, 0] + (f - 1) / 2
            kp["yf"] = f * r[:, 1] + (f - 1) / 2
            kp["zf"] = f * r[:, 2] + (f - 1) / 2
            kp["sigma"] = scale_sigma(p, s) * f
            rows.append(kp)
    if not rows:
        return np.zeros(0, dtype=KEYPOINT_DTYPE)
    return np.concatenate(rows)


def describe(G_levels, kps: np.ndarray, draws: np.ndarray, p: Params):
    """SIFT-Rank ranks [K,64] u8, BRIEF words [K,n/64] u64, RRIEF ranks [K,n] u8.

    Also returns the raw SIFT-Rank histograms and BRIEF differences so that
    tests can apply the near-tie margins.
    """
    K = len(kps)
    n = p.brief_n
    nw = (n + 63) // 64
    sr = np.zeros((K, 64), dtype=np.uint8)
    hist = np.zeros((K, 64))
    br = np.zeros((K, nw), dtype=np.uint64)
    rr = np.zeros((K, n), dtype=np.uint8)
    dd = np.zeros((K, n))
    wb = gauss_taps(p.brief_blur, p.trunc)
    for o, G in enumerate(G_levels):
        for s in range(1, p.scales + 1):
            sel = np.nonzero((kps["octave"] == o) & (kps["scale"] == s))[0]
            if len(sel) == 0:
                continue
            xyz = np.stack([kps["x"][sel], kps["y"][sel], kps["z"][sel]], axis=1)
            h, r = siftrank(G[s], xyz, siftrank_radius(p, s))
            hist[sel], sr[sel] = h, r
            d, b, q = brief_rrief(G[s], xyz, pair_offsets(draws, p, s), wb)
            dd[sel], br[sel], rr[sel] = d, b, q.astype(np.uint8)
    return {"siftrank": sr, "hist": hist, "brief": br, "rrief": rr, "diff": dd}


def extract(vol: np.ndarray, p: Params, draws: np.ndarray):
    """Whole hot path: pyramid, keypoints, descriptors."""
    octs = pyramid(vol, p)
    kps = detect([oc.D for oc in octs], p)
    desc = describe([oc.G for oc in octs], kps, draws, p)
    return octs, kps, desc


# ------------------------------------------- matching: normalisation, Hough
from .hough import (HoughParams, geometry, hough, hough_default_params, hypothesis, pack_key,  # noqa: E402
                    rotation_vector, similarity_fit, unit_normalize, unpack_key)
