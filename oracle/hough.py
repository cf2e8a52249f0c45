"""FP64 CPU oracle of the matching stage beside the hot path -- TEST
INFRASTRUCTURE ONLY (imported by the tests, the smoke check and the
benchmark's CPU-baseline leg; the product library never calls it).

What it computes (Carluer et al., arXiv 2112.10258):

* Unit-length normalisation of descriptors (Section 3.1, step e): the
  stored descriptor f is scaled to |f| = 1, so that the nearest neighbour
  under the Euclidean distance is also the largest scalar product.
* The accuracy measure of Section 3.3 (Experiments and Data): descriptor
  matches between two volumes count when they are inliers to a global
  similarity transform (3D rotation, translation, isotropic scale: 7 degrees
  of freedom) found by a Hough transform. The paper gives no vote layout;
  reading R26 fixes one, written out step by step in ``hough``.

Plain numpy in float64, loops over matches; nothing here is blocked or
reordered beyond the definitions below.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# --- unit-length normalisation (Section 3.1 e) ---------------------------


def unit_normalize(desc: np.ndarray, kind: int, n_bits: int | None = None) -> np.ndarray:
    """Descriptors scaled to unit length, float64 rows.

    kind 0: BRIEF words [n][w] uint64; bit i (least significant first of
    word i // 64) becomes the entry +1 (set) or -1 (clear), so every row has
    norm sqrt(n_bits) before scaling (n_bits = 64 w unless given: only the
    first n_bits bits are entries). Squared distances of the results are then
    4 * Hamming / n_bits.
    kind 1: rank vectors [n][m] uint8, f = r / |r|; an all-zero row (an
    unused descriptor slot) stays zero.
    """
    desc = np.asarray(desc)
    if kind == 0:
        w = desc.shape[1]
        nb = 64 * w if n_bits is None else int(n_bits)
        out = np.empty((len(desc), nb))
        for i, row in enumerate(desc):
            for b in range(nb):
                bit = (int(row[b // 64]) >> (b % 64)) & 1
                out[i, b] = 1.0 if bit else -1.0
        return out / math.sqrt(nb)
    f = desc.astype(np.float64)
    out = np.zeros_like(f)
    for i, row in enumerate(f):
        nrm = math.sqrt(float(row @ row))
        if nrm > 0.0:
            out[i] = row / nrm
    return out


# --- the 7-DoF Hough vote (Section 3.3; reading R26) ---------------------

FIELD_BITS = 9           # bits per bin coordinate in a packed bin key
FIELD_BIAS = 256         # a coordinate c is stored as c + 256, 0 <= c + 256 <= 511
N_DIMS = 7               # log2 scale, rotation vector (3), predicted centre (3)


@dataclass
class HoughParams:
    """Bin widths and inlier rule (reading R26)."""
    scale_bin: float = 1.0                  # width of a log2(scale) bin
    angle_bin: float = math.pi / 6.0        # width of a rotation-vector component bin, radians
    trans_bin: float = 36.25                # width of a predicted-centre bin, input voxels
    centre: tuple = (72.0, 86.5, 72.0)      # reference point c of volume A (input voxels)
    inlier_sigmas: float = 2.0              # inlier: |T(x_a) - x_b| <= inlier_sigmas * sigma_b
    inlier_log2s: float = 0.5               # and |log2(s sigma_a / sigma_b)| <= inlier_log2s
    iterations: int = 2                     # fit / inlier rounds (>= 1)


def hough_default_params(shape_xyz) -> HoughParams:
    """Defaults for a volume A of dims (nx, ny, nz): the reference point is
    its centre and a translation bin is a quarter of its largest dimension."""
    nx, ny, nz = (int(v) for v in shape_xyz)
    return HoughParams(trans_bin=0.25 * max(nx, ny, nz),
                       centre=((nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0))


def rotation_vector(R: np.ndarray):
    """Rotation vector w = theta * a of a 3x3 matrix (the inverse of
    Rodrigues' formula), evaluated as written for any R, orthonormal or not:

      cos t = clamp((trace R - 1) / 2, -1, 1), t = arccos(cos t);
      v = (R[2,1] - R[1,2], R[0,2] - R[2,0], R[1,0] - R[0,1]) (= 2 sin t a);
      cos t >= -0.99: w = v * t / (2 sin t), with t / (2 sin t) taken as
        (1 + t^2 / 6) / 2 for t < 1e-4;
      cos t < -0.99 (t near pi, where v vanishes): from the symmetric part
        B = (R + R^T) / 2 - cos t I = (1 - cos t) a a^T, with i the index of
        the largest diagonal entry B[i,i] (the lowest among equal ones),
        a = B[:, i] / sqrt(B[i,i] (1 - cos t)); a is negated if a . v < 0;
        w = t a.
    Returns (w, margin): margin is the distance of cos t to the branch point
    -0.99 (a decision both implementations must take alike)."""
    R = np.asarray(R, dtype=np.float64).reshape(3, 3)
    c = min(1.0, max(-1.0, (R[0, 0] + R[1, 1] + R[2, 2] - 1.0) / 2.0))
    t = math.acos(c)
    v = np.array([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]])
    margin = abs(c + 0.99)
    if c >= -0.99:
        f = 0.5 * (1.0 + t * t / 6.0) if t < 1e-4 else t / (2.0 * math.sin(t))
        return v * f, margin
    B = 0.5 * (R + R.T) - c * np.eye(3)
    i = int(np.argmax(np.diag(B)))
    a = B[:, i] / math.sqrt(B[i, i] * (1.0 - c))
    if float(a @ v) < 0.0:
        a = -a
    margin = min(margin, abs(float(a @ v)))
    return t * a, margin


def similarity_fit(xa: np.ndarray, xb: np.ndarray):
    """Least-squares similarity x_b ~ s R x_a + t over point pairs (the
    closed form of Umeyama 1991): with means ma, mb, centred sets
    A = xa - ma, B = xb - mb, covariance S = B^T A / n = U D V^T,
    E = diag(1, 1, det(U) det(V)): R = U E V^T, s = trace(D E) / var_a with
    var_a = sum |A|^2 / n, t = mb - s R ma. Returns (s, R, t); s = 0 when
    var_a = 0."""
    xa = np.asarray(xa, dtype=np.float64).reshape(-1, 3)
    xb = np.asarray(xb, dtype=np.float64).reshape(-1, 3)
    n = len(xa)
    ma, mb = xa.mean(axis=0), xb.mean(axis=0)
    A, B = xa - ma, xb - mb
    var_a = float((A * A).sum()) / n
    S = B.T @ A / n
    U, D, Vt = np.linalg.svd(S)
    E = np.diag([1.0, 1.0, 1.0 if np.linalg.det(U) * np.linalg.det(Vt) >= 0.0 else -1.0])
    R = U @ E @ Vt
    s = float(np.trace(np.diag(D) @ E)) / var_a if var_a > 0.0 else 0.0
    t = mb - s * (R @ ma)
    return s, R, t


def pack_key(c) -> int:
    """Packed bin key: coordinate d (0 = log2 scale, 1..3 = rotation vector
    x, y, z, 4..6 = predicted centre x, y, z) in bits 9d .. 9d+8 as c + 256."""
    k = 0
    for d in range(N_DIMS):
        k |= (int(c[d]) + FIELD_BIAS) << (FIELD_BITS * d)
    return k


def unpack_key(k: int):
    return [((int(k) >> (FIELD_BITS * d)) & ((1 << FIELD_BITS) - 1)) - FIELD_BIAS for d in range(N_DIMS)]


def geometry(kp_xyz_sigma: np.ndarray, frames: np.ndarray) -> np.ndarray:
    """Rows of the geometry array the Hough vote reads: [n][13] float32 =
    (x, y, z, sigma, R[9]) with R[3 i + j] = component i of frame axis j."""
    g = np.zeros((len(kp_xyz_sigma), 13), dtype=np.float32)
    g[:, :4] = np.asarray(kp_xyz_sigma, dtype=np.float32).reshape(-1, 4)
    g[:, 4:] = np.asarray(frames, dtype=np.float32).reshape(-1, 9)
    return g


def hypothesis(ga: np.ndarray, gb: np.ndarray, hp: HoughParams):
    """The similarity one match of oriented keypoints implies, and its bin
    coordinates (reading R26):

      s = sigma_b / sigma_a, R = R_b R_a^T (A's frame turned onto B's),
      p = x_b + s R (c - x_a) (where the transform takes A's reference
      point c); the vote vector v = (log2 s, w(R), p) with w the rotation
      vector; q = v / width per coordinate, bin b = floor(q), and the
      neighbouring bin on the nearer side, b + 1 if q - b >= 0.5 else b - 1;
      lo = min of the two. The match votes for the 2^7 bins lo + {0, 1}^7.

    Inputs are geometry rows (float32, taken exactly; both sigmas > 0).
    Returns (lo [7] int, or None if a coordinate is not finite, s, R,
    margin): margin is the smallest distance, in bin units, of any q
    to a multiple of 1/2 (where floor or the side would change), or of the
    rotation-vector branch decision."""
    ga = np.asarray(ga, dtype=np.float64)
    gb = np.asarray(gb, dtype=np.float64)
    xa, sa, Ra = ga[:3], ga[3], ga[4:].reshape(3, 3)
    xb, sb, Rb = gb[:3], gb[3], gb[4:].reshape(3, 3)
    s = sb / sa
    R = Rb @ Ra.T
    w, mg = rotation_vector(R)
    p = xb + s * (R @ (np.asarray(hp.centre, dtype=np.float64) - xa))
    v = np.concatenate([[math.log2(s)], w, p])
    width = np.array([hp.scale_bin] + [hp.angle_bin] * 3 + [hp.trans_bin] * 3)
    lo = np.zeros(N_DIMS, dtype=np.int64)
    if not np.all(np.isfinite(v)):
        return None, s, R, mg
    for d in range(N_DIMS):
        q = v[d] / width[d]
        b = math.floor(q)
        nb = b + 1 if q - b >= 0.5 else b - 1
        lo[d] = min(b, nb)
        # a scale ratio that is a power of two (keypoints of the same level,
        # or levels whole octaves apart) has an exact log2: its decision is
        # exact in any implementation, so it sets no margin
        if d == 0 and math.frexp(s)[0] == 0.5:
            continue
        mg = min(mg, abs(q - round(2.0 * q) / 2.0))
    return lo, s, R, mg


def _inliers(ga, gb, match, valid, s, R, t, hp):
    """Inlier rule: |s R x_a + t - x_b| <= k sigma_b and
    |log2(s sigma_a / sigma_b)| <= l; also the smallest distance of either
    test to its threshold (relative), for near-tie accounting."""
    n = len(ga)
    inl = np.zeros(n, dtype=bool)
    mg = np.full(n, np.inf)
    for i in range(n):
        if not valid[i]:
            continue
        a, b = ga[i].astype(np.float64), gb[match[i]].astype(np.float64)
        e = np.linalg.norm(s * (R @ a[:3]) + t - b[:3])
        lim = hp.inlier_sigmas * b[3]
        ds = abs(math.log2(s * a[3] / b[3]))
        inl[i] = e <= lim and ds <= hp.inlier_log2s
        mg[i] = min(abs(e - lim) / max(lim, 1.0), abs(ds - hp.inlier_log2s))
    return inl, mg


def hough(geo_a: np.ndarray, geo_b: np.ndarray, match: np.ndarray, hp: HoughParams):
    """Global 7-DoF similarity by a Hough vote over matches, then its
    inliers (Section 3.3; reading R26).

    geo_a [n_a][13], geo_b [n_b][13]: geometry rows; match [n_a]: index of
    A row i's match in B, or -1. A match is valid when its index is in
    [0, n_b) and both rows have sigma > 0; only valid matches vote and can
    be inliers.

      1. every valid match votes once for each of its 2^7 bins (hypothesis);
         a match with a bin coordinate outside -256 .. 254 (or a vote
         coordinate that is not finite) does not vote;
      2. the winning bin has the most votes; among equal counts, the
         smallest packed key (pack_key);
      3. the fit set is the matches voting for the winning bin;
      4. per round (hp.iterations rounds): if the fit set has at least 3
         matches, the least-squares similarity of their positions
         (similarity_fit, x_a -> x_b) is the transform and the inliers are
         the valid matches passing the inlier rule; the next round's fit set
         is those inliers. With fewer than 3 (or var_a = 0) the rounds stop;
         in the first round that leaves no transform.

    Returns a dict: status (1 = transform found), bin (packed key, -1 if
    no vote), votes, scale, R [3,3], t [3], n_fit (size of the last fit
    set), inlier [n_a] bool, n_inliers, lo [n_a][7] (-1 rows for
    non-voting matches), voted [n_a] bool, margin [n_a] (near-tie distance
    of each match's bin and inlier decisions)."""
    ga = np.asarray(geo_a, dtype=np.float32)
    gb = np.asarray(geo_b, dtype=np.float32)
    match = np.asarray(match, dtype=np.int64)
    n_a, n_b = len(ga), len(gb)
    # a match counts when its index is in range and both scales are positive
    valid = (match >= 0) & (match < n_b)
    for i in np.nonzero(valid)[0]:
        valid[i] = bool(ga[i, 3] > 0.0) and bool(gb[match[i], 3] > 0.0)
    lo = np.full((n_a, N_DIMS), -1, dtype=np.int64)
    voted = np.zeros(n_a, dtype=bool)
    margin = np.full(n_a, np.inf)
    votes = {}
    for i in range(n_a):
        if not valid[i]:
            continue
        l, _, _, mg = hypothesis(ga[i], gb[match[i]], hp)
        margin[i] = mg
        if l is None or np.any(l < -FIELD_BIAS) or np.any(l + 1 > (1 << FIELD_BITS) - 1 - FIELD_BIAS):
            continue
        lo[i], voted[i] = l, True
        for corner in range(1 << N_DIMS):
            k = pack_key([l[d] + ((corner >> d) & 1) for d in range(N_DIMS)])
            votes[k] = votes.get(k, 0) + 1
    out = {"status": 0, "bin": -1, "votes": 0, "scale": 0.0, "R": np.zeros((3, 3)), "t": np.zeros(3),
           "n_fit": 0, "inlier": np.zeros(n_a, dtype=bool), "n_inliers": 0, "lo": lo, "voted": voted,
           "margin": margin}
    if not votes:
        return out
    best = max(votes.values())
    win = min(k for k, c in votes.items() if c == best)
    out["bin"], out["votes"] = win, best
    W = np.array(unpack_key(win))
    fit_set = np.array([voted[i] and bool(np.all((lo[i] <= W) & (W <= lo[i] + 1))) for i in range(n_a)])
    inl_mg = np.full(n_a, np.inf)
    for _ in range(max(1, int(hp.iterations))):
        idx = np.nonzero(fit_set)[0]
        if len(idx) < 3:
            break
        xa = ga[idx, :3].astype(np.float64)
        xb = gb[match[idx], :3].astype(np.float64)
        s, R, t = similarity_fit(xa, xb)
        if s <= 0.0:
            break
        inl, mg = _inliers(ga, gb, match, valid, s, R, t, hp)
        inl_mg = np.minimum(inl_mg, mg)
        out.update(status=1, scale=s, R=R, t=t, n_fit=len(idx), inlier=inl, n_inliers=int(inl.sum()))
        fit_set = inl
    out["margin"] = np.minimum(margin, inl_mg)
    return out
