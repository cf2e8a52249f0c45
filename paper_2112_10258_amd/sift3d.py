"""ctypes binding of libsift3d.so: argument marshalling only.

Every step of the hot path runs in the HIP kernels of libsift3d.so; this
module converts torch tensors (device memory) and streams into the raw
pointers the C ABI takes. There is no fallback: if the library is missing
or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsift3d.so")

KEYPOINT_DTYPE = np.dtype([
    ("x", "<i4"), ("y", "<i4"), ("z", "<i4"),
    ("octave", "<i2"), ("scale", "<i2"), ("polarity", "i1"), ("pad", "i1", (3,)),
    ("dog", "<f4"), ("xf", "<f4"), ("yf", "<f4"), ("zf", "<f4"), ("sigma", "<f4"),
])
KEYPOINT_BYTES = 40
assert KEYPOINT_DTYPE.itemsize == KEYPOINT_BYTES

OK, E_ARG, E_TOO_SMALL, E_WORKSPACE, E_HIP, E_UNSUPPORTED, E_SCRATCH, E_TIMEOUT = 0, -1, -2, -3, -5, -6, -7, -8
DETECT_STATIC_SCRATCH = 64 << 20     # SIFT3D_DETECT_STATIC_SCRATCH
MAX_ORIENTATIONS = 4                 # SIFT3D_MAX_ORIENTATIONS
PENDING = 1


class Params(ctypes.Structure):
    _fields_ = [
        ("n_octaves", ctypes.c_int),
        ("min_dim", ctypes.c_int),
        ("scales", ctypes.c_int),
        ("sigma0", ctypes.c_double),
        ("sigma_in", ctypes.c_double),
        ("trunc", ctypes.c_double),
        ("dog_threshold", ctypes.c_float),
        ("votes", ctypes.c_int),
        ("brief_n", ctypes.c_int),
        ("brief_blur", ctypes.c_double),
        ("siftrank_factor", ctypes.c_double),
        ("pyramid_mode", ctypes.c_int),
        ("brief_method", ctypes.c_int),
    ]


class ServerConfig(ctypes.Structure):
    _fields_ = [
        ("hbm_budget", ctypes.c_size_t),
        ("n_streams", ctypes.c_int),
        ("max_inflight", ctypes.c_int),
        ("kp_capacity", ctypes.c_int),
        ("max_batch", ctypes.c_int),
        ("admit_timeout_s", ctypes.c_double),
    ]


class Result(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int),
        ("hip_error", ctypes.c_int),
        ("count", ctypes.c_int),
        ("capacity", ctypes.c_int),
        ("d_kp", ctypes.c_void_p),
        ("d_siftrank", ctypes.c_void_p),
        ("d_brief", ctypes.c_void_p),
        ("d_rrief", ctypes.c_void_p),
        ("stream", ctypes.c_int),
        ("t_submit", ctypes.c_double),
        ("t_start", ctypes.c_double),
        ("t_done", ctypes.c_double),
    ]


class ServerCounters(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_int64),
        ("completed", ctypes.c_int64),
        ("failed", ctypes.c_int64),
        ("in_flight", ctypes.c_int),
        ("pending", ctypes.c_int),
        ("allocated", ctypes.c_size_t),
        ("peak_allocated", ctypes.c_size_t),
        ("hbm_budget", ctypes.c_size_t),
        ("slot_allocations", ctypes.c_int64),
        ("slot_evictions", ctypes.c_int64),
        ("groups", ctypes.c_int64),
        ("grouped_requests", ctypes.c_int64),
    ]


class HoughParams(ctypes.Structure):
    _fields_ = [
        ("scale_bin", ctypes.c_double),
        ("angle_bin", ctypes.c_double),
        ("trans_bin", ctypes.c_double),
        ("centre", ctypes.c_double * 3),
        ("inlier_sigmas", ctypes.c_double),
        ("inlier_log2s", ctypes.c_double),
        ("iterations", ctypes.c_int),
    ]


class Similarity(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("votes", ctypes.c_int32),
        ("bin", ctypes.c_int64),
        ("n_fit", ctypes.c_int32),
        ("n_inliers", ctypes.c_int32),
        ("scale", ctypes.c_double),
        ("rot", ctypes.c_double * 9),
        ("trans", ctypes.c_double * 3),
    ]


SIMILARITY_BYTES = 128
assert ctypes.sizeof(Similarity) == SIMILARITY_BYTES


class Sift3dError(RuntimeError):
    def __init__(self, code: int, what: str):
        lib = _load()
        msg = lib.sift3d_error_string(code).decode()
        if code == E_HIP:
            msg += f" (hipError {lib.sift3d_last_hip_error()})"
        super().__init__(f"{what}: {msg} [{code}]")
        self.code = code


_lib = None
_vp = ctypes.c_void_p


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libsift3d.so not built ({LIB_PATH}); run python -m paper_2112_10258_amd.build")
    # torch's HIP and HSA runtimes first: torch's libraries ask for them by
    # unversioned file names, the library by soname (libamdhip64.so.7), so
    # loading the library first would bring a second copy of each runtime
    # into the process, and torch's copy then finds no GPU. Loaded the other
    # way round, the library's soname lookup resolves to torch's copy.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    i, sz = ctypes.c_int, ctypes.c_size_t
    P = ctypes.POINTER
    sig = {
        "sift3d_default_params": (i, [P(Params)]),
        "sift3d_create": (i, [P(Params), P(ctypes.c_double), i, P(_vp)]),
        "sift3d_destroy": (i, [_vp]),
        "sift3d_pair_offsets": (i, [P(Params), P(ctypes.c_double), i, i, P(ctypes.c_int32)]),
        "sift3d_plan_create": (i, [_vp, i, i, i, i, P(_vp)]),
        "sift3d_plan_create_batch": (i, [_vp, i, P(i), i, P(_vp)]),
        "sift3d_plan_destroy": (i, [_vp]),
        "sift3d_plan_info": (i, [_vp, P(sz), P(i), P(sz)]),
        "sift3d_plan_volume": (i, [_vp, i, P(i), P(sz), P(i)]),
        "sift3d_plan_octave_dims": (i, [_vp, i, i, P(i)]),
        "sift3d_level": (i, [_vp, _vp, i, i, i, i, P(_vp)]),
        "sift3d_build_pyramid": (i, [_vp, _vp, _vp, sz, _vp]),
        "sift3d_detect": (i, [_vp, _vp, sz, _vp, i, _vp, _vp]),
        "sift3d_detect_static": (i, [_vp, _vp, sz, _vp, i, _vp, _vp]),
        "sift3d_plan_tune": (i, [_vp, _vp, _vp, sz, i, _vp]),
        "sift3d_plan_tuning_count": (i, [_vp, P(i)]),
        "sift3d_plan_tuning": (i, [_vp, i, P(i), P(ctypes.c_float)]),
        "sift3d_plan_detect_scratch": (i, [_vp, P(sz)]),
        "sift3d_describe": (i, [_vp, _vp, sz, _vp, _vp, i, _vp, _vp, _vp, _vp]),
        "sift3d_orient": (i, [_vp, _vp, sz, _vp, _vp, i, ctypes.c_double, _vp, _vp, _vp, _vp]),
        "sift3d_extract": (i, [_vp, _vp, _vp, sz, _vp, i, _vp, _vp, _vp, _vp, _vp]),
        "sift3d_pyramid_pass_count": (i, [_vp, P(i)]),
        "sift3d_pyramid_pass_info": (i, [_vp, i, P(i), P(sz)]),
        "sift3d_pyramid_pass": (i, [_vp, i, _vp, _vp, sz, _vp]),
        "sift3d_pyramid_step_count": (i, [_vp, P(i)]),
        "sift3d_pyramid_step_info": (i, [_vp, i, P(i), P(sz)]),
        "sift3d_pyramid_step": (i, [_vp, i, _vp, _vp, sz, _vp]),
        "sift3d_ctx_params": (i, [_vp, P(Params)]),
        "sift3d_server_create": (i, [_vp, P(ServerConfig), P(_vp)]),
        "sift3d_server_footprint": (i, [_vp, i, i, i, P(sz)]),
        "sift3d_server_submit": (i, [_vp, _vp, i, i, i, P(ctypes.c_int64)]),
        "sift3d_server_result": (i, [_vp, ctypes.c_int64, i, P(Result)]),
        "sift3d_server_fetch": (i, [_vp, ctypes.c_int64, _vp, _vp, _vp, _vp]),
        "sift3d_server_release": (i, [_vp, ctypes.c_int64]),
        "sift3d_server_stats": (i, [_vp, P(ServerCounters)]),
        "sift3d_server_clock": (ctypes.c_double, []),
        "sift3d_server_destroy": (i, [_vp]),
        "sift3d_match": (i, [i, _vp, i, _vp, i, i, _vp, _vp, _vp, _vp]),
        "sift3d_normalize": (i, [i, _vp, i, i, _vp, _vp]),
        "sift3d_units": (i, [_vp, _vp, i, _vp, _vp, _vp, i, _vp, _vp, _vp, _vp, _vp]),
        "sift3d_hough_default_params": (i, [i, i, i, P(HoughParams)]),
        "sift3d_hough_workspace": (i, [i, P(sz)]),
        "sift3d_hough": (i, [_vp, i, _vp, i, _vp, P(HoughParams), _vp, sz, _vp, _vp, _vp]),
        "sift3d_box_blur": (i, [_vp, _vp, _vp, i, i, i, i, i, _vp]),
        "sift3d_box_half_width": (i, [ctypes.c_double, i, P(i)]),
        "sift3d_error_string": (ctypes.c_char_p, [i]),
        "sift3d_last_hip_error": (i, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    """Names the binding resolves in libsift3d.so (all C ABI entry points)."""
    lib = _load()
    return [n for n in dir(lib) if n.startswith("sift3d_")]


def _check(code: int, what: str):
    if code != OK:
        raise Sift3dError(code, what)


def _ptr(t) -> int:
    if t is None:
        return None
    return t.data_ptr()


def _stream(stream) -> int:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


MATCH_BRIEF = 0
MATCH_RANKS = 1


def match(a, b, kind: int, stream=None):
    """Nearest row of b for every row of a (sift3d_match): device tensors
    [n][words] int64 (BRIEF, kind MATCH_BRIEF) or [n][m] uint8 (ranks, kind
    MATCH_RANKS). Returns (idx, d1, d2) int32 device tensors of length n_a."""
    import torch
    assert a.is_cuda and b.is_cuda and a.dim() == 2 and b.dim() == 2 and a.shape[1] == b.shape[1]
    a = a.contiguous()
    b = b.contiguous()
    n_a, n_b = a.shape[0], b.shape[0]
    idx = torch.empty(n_a, dtype=torch.int32, device=a.device)
    d1 = torch.empty(n_a, dtype=torch.int32, device=a.device)
    d2 = torch.empty(n_a, dtype=torch.int32, device=a.device)
    _check(_load().sift3d_match(int(kind), _vp(a.data_ptr()), n_a, _vp(b.data_ptr() if n_b else None), n_b,
                                int(a.shape[1]), _vp(idx.data_ptr()), _vp(d1.data_ptr()), _vp(d2.data_ptr()),
                                _vp(_stream(stream))), "sift3d_match")
    return idx, d1, d2


def normalize(desc, kind: int, stream=None):
    """Unit-length descriptors (sift3d_normalize): [n][words] int64 BRIEF
    rows (kind MATCH_BRIEF) give [n][64 words] float32 of +-1/sqrt(64 words);
    [n][m] uint8 rank rows (kind MATCH_RANKS) give [n][m] float32 r/|r|."""
    import torch
    assert desc.is_cuda and desc.dim() == 2
    desc = desc.contiguous()
    n, w = desc.shape
    cols = 64 * w if kind == MATCH_BRIEF else w
    out = torch.empty((n, cols), dtype=torch.float32, device=desc.device)
    _check(_load().sift3d_normalize(int(kind), _vp(desc.data_ptr() if n else None), n, int(w),
                                    _vp(out.data_ptr() if n else None), _vp(_stream(stream))), "sift3d_normalize")
    return out


def units(kp, count, capacity: int, nframes=None, frames=None, desc=None, stream=None):
    """Matching units of one volume (sift3d_units). kp: keypoint rows
    (uint8 [cap][40] device tensor or any device tensor of that size),
    count: int32 device tensor whose first element is the keypoint count.
    nframes/frames: sift3d_orient outputs for oriented units (None: upright,
    one unit per keypoint with the identity frame). desc: device tensor of
    descriptor rows ([cap*4][row] oriented, [cap][row] upright) to copy, or
    None. Returns (unit int32 [n], geo float32 [n][13], desc_out or None),
    cut to the unit count (read back to the host)."""
    import torch
    dev = count.device
    rows = capacity * (MAX_ORIENTATIONS if nframes is not None else 1)
    unit = torch.empty(max(rows, 1), dtype=torch.int32, device=dev)
    geo = torch.empty((max(rows, 1), 13), dtype=torch.float32, device=dev)
    n = torch.empty(1, dtype=torch.int32, device=dev)
    dout, rb = None, 0
    if desc is not None:
        if not desc.is_contiguous() or rows == 0 or desc.numel() % rows:
            raise ValueError("units: desc must be contiguous with one row per keypoint (per frame if oriented)")
        per_row = desc.numel() // rows
        rb = per_row * desc.element_size()
        dout = torch.empty((max(rows, 1), per_row), dtype=desc.dtype, device=dev)
    _check(_load().sift3d_units(_vp(kp.data_ptr()), _vp(count.data_ptr()), int(capacity),
                                _vp(_ptr(nframes)), _vp(_ptr(frames)), _vp(_ptr(desc)), int(rb),
                                _vp(unit.data_ptr()), _vp(geo.data_ptr()), _vp(_ptr(dout)), _vp(n.data_ptr()),
                                _vp(_stream(stream))), "sift3d_units")
    k = int(n.item())
    return unit[:k], geo[:k], (dout[:k] if dout is not None else None)


def hough_default_params(shape_xyz) -> HoughParams:
    hp = HoughParams()
    nx, ny, nz = (int(v) for v in shape_xyz)
    _check(_load().sift3d_hough_default_params(nx, ny, nz, ctypes.byref(hp)), "sift3d_hough_default_params")
    return hp


def hough_workspace_bytes(n_a: int) -> int:
    b = ctypes.c_size_t()
    _check(_load().sift3d_hough_workspace(int(n_a), ctypes.byref(b)), "sift3d_hough_workspace")
    return b.value


def hough(geo_a, geo_b, match_idx, hp: HoughParams, ws=None, stream=None, sync=True):
    """7-DoF similarity Hough vote and inliers (sift3d_hough). geo_a [n_a][13],
    geo_b [n_b][13] float32 and match_idx [n_a] int32 device tensors.
    Returns (result, inlier): result is a dict read from the device (when
    sync) or the raw uint8 [128] device tensor; inlier is uint8 [n_a]."""
    import torch
    dev = match_idx.device
    n_a, n_b = int(geo_a.shape[0]), int(geo_b.shape[0])
    if ws is None:
        ws = torch.empty(hough_workspace_bytes(n_a), dtype=torch.uint8, device=dev)
    out = torch.zeros(SIMILARITY_BYTES, dtype=torch.uint8, device=dev)
    inl = torch.empty(max(n_a, 1), dtype=torch.uint8, device=dev)
    _check(_load().sift3d_hough(_vp(geo_a.data_ptr() if n_a else None), n_a,
                                _vp(geo_b.data_ptr() if n_b else None), n_b,
                                _vp(match_idx.data_ptr() if n_a else None), ctypes.byref(hp),
                                _vp(ws.data_ptr()), ws.numel(), _vp(out.data_ptr()), _vp(inl.data_ptr()),
                                _vp(_stream(stream))), "sift3d_hough")
    if not sync:
        return out, inl[:n_a]
    return similarity_dict(out), inl[:n_a]


def similarity_dict(raw) -> dict:
    """The sift3d_similarity in a uint8 [128] tensor as a dict of numpy values."""
    r = Similarity.from_buffer_copy(bytes(raw.cpu().numpy().tobytes()))
    return {"status": r.status, "votes": r.votes, "bin": r.bin, "n_fit": r.n_fit, "n_inliers": r.n_inliers,
            "scale": r.scale, "R": np.array(r.rot[:]).reshape(3, 3), "t": np.array(r.trans[:])}


def box_half_width(sigma: float, passes: int) -> int:
    """Half-width of the uniform filter whose `passes`-fold repetition stands
    in for a Gaussian of standard deviation sigma (sift3d_box_half_width)."""
    h = ctypes.c_int()
    _check(_load().sift3d_box_half_width(float(sigma), int(passes), ctypes.byref(h)), "sift3d_box_half_width")
    return h.value


def box_blur(vol, half_width: int, passes: int, out=None, tmp=None, stream=None):
    """Uniform-filter blur of a float32 [z,y,x] device tensor (sift3d_box_blur):
    `passes` clamp-to-edge passes of width 2*half_width+1 along x, y, then z.
    Returns `out` (allocated when None); `tmp` is scratch of the same size."""
    import torch
    if not (vol.is_cuda and vol.dtype == torch.float32 and vol.dim() == 3 and vol.is_contiguous()):
        raise ValueError("box_blur: vol must be a contiguous float32 [z,y,x] device tensor")
    nz, ny, nx = vol.shape
    if out is None:
        out = torch.empty_like(vol)
    if tmp is None:
        tmp = torch.empty_like(vol)
    for name, t in (("out", out), ("tmp", tmp)):
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.numel() == vol.numel()):
            raise ValueError(f"box_blur: {name} must be a contiguous float32 device tensor of vol's size")
    if len({vol.data_ptr(), out.data_ptr(), tmp.data_ptr()}) != 3:
        raise ValueError("box_blur: vol, out and tmp must be distinct buffers")
    _check(_load().sift3d_box_blur(_vp(vol.data_ptr()), _vp(out.data_ptr()), _vp(tmp.data_ptr()), nx, ny, nz,
                                   int(half_width), int(passes), _vp(_stream(stream))), "sift3d_box_blur")
    return out


def default_params(**overrides) -> Params:
    p = Params()
    _check(_load().sift3d_default_params(ctypes.byref(p)), "sift3d_default_params")
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def pair_offsets(params: Params, pair_draws: np.ndarray, scale: int) -> np.ndarray:
    """Integer (x,y,z) pair offsets [brief_n][2][3] of one scale (host only)."""
    draws = np.ascontiguousarray(pair_draws, dtype=np.float64).reshape(-1, 2, 3)
    out = np.zeros((params.brief_n, 2, 3), dtype=np.int32)
    _check(_load().sift3d_pair_offsets(ctypes.byref(params), draws.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       len(draws), scale, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))),
           "sift3d_pair_offsets")
    return out


class Context:
    """Method parameters plus the pair draws; owns a small device table."""

    def __init__(self, params: Params | None = None, pair_draws: np.ndarray | None = None, **overrides):
        lib = _load()
        self.params = params if params is not None else default_params(**overrides)
        draws = None
        n = 0
        if pair_draws is not None:
            draws = np.ascontiguousarray(pair_draws, dtype=np.float64).reshape(-1, 2, 3)
            n = len(draws)
        self._draws = draws
        h = _vp()
        dp = draws.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if draws is not None else None
        _check(lib.sift3d_create(ctypes.byref(self.params), dp, n, ctypes.byref(h)), "sift3d_create")
        self.handle = h

    def pair_offsets(self, scale: int) -> np.ndarray:
        return pair_offsets(self.params, self._draws, scale)

    def close(self):
        if getattr(self, "handle", None):
            _load().sift3d_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """Extraction plan for one volume shape, or for a batch of volumes.

    Plan(ctx, (nx, ny, nz), cap) plans one volume; Plan(ctx, [(nx, ny, nz), ...],
    cap, batch=True) plans a batch processed together (inputs packed with
    ``pack_volumes``).
    """

    def __init__(self, ctx: Context, shape_xyz, kp_capacity: int, batch: bool = False):
        lib = _load()
        self.ctx = ctx
        self.capacity = int(kp_capacity)
        h = _vp()
        if batch:
            shapes = [tuple(int(v) for v in s) for s in shape_xyz]
            dims = (ctypes.c_int * (3 * len(shapes)))(*[v for s in shapes for v in s])
            _check(lib.sift3d_plan_create_batch(ctx.handle, len(shapes), dims, self.capacity, ctypes.byref(h)),
                   "sift3d_plan_create_batch")
        else:
            nx, ny, nz = (int(v) for v in shape_xyz)
            _check(lib.sift3d_plan_create(ctx.handle, nx, ny, nz, self.capacity, ctypes.byref(h)),
                   "sift3d_plan_create")
        self.handle = h
        ws = ctypes.c_size_t()
        nv = ctypes.c_int()
        ne = ctypes.c_size_t()
        _check(lib.sift3d_plan_info(h, ctypes.byref(ws), ctypes.byref(nv), ctypes.byref(ne)), "sift3d_plan_info")
        self.workspace_bytes = ws.value
        self.n_volumes = nv.value
        self.input_elems = ne.value
        self.volumes = []
        for v in range(self.n_volumes):
            d = (ctypes.c_int * 3)()
            off = ctypes.c_size_t()
            no = ctypes.c_int()
            _check(lib.sift3d_plan_volume(h, v, d, ctypes.byref(off), ctypes.byref(no)), "sift3d_plan_volume")
            self.volumes.append({"shape_xyz": tuple(d), "offset": off.value, "n_octaves": no.value})
        self.shape_xyz = self.volumes[0]["shape_xyz"]
        self.n_octaves = self.volumes[0]["n_octaves"]

    def octave_dims(self, o: int, volume: int = 0):
        d = (ctypes.c_int * 3)()
        _check(_load().sift3d_plan_octave_dims(self.handle, volume, o, d), "sift3d_plan_octave_dims")
        return tuple(d)

    def level(self, ws, octave: int, kind: int, idx: int, volume: int = 0):
        """torch view [nz, ny, nx] float32 of a level inside the workspace tensor."""
        import torch
        p = _vp()
        _check(_load().sift3d_level(self.handle, _vp(ws.data_ptr()), volume, octave, kind, idx, ctypes.byref(p)),
               "sift3d_level")
        nx, ny, nz = self.octave_dims(octave, volume)
        off = p.value - ws.data_ptr()
        n = nx * ny * nz
        return ws[off:off + 4 * n].view(torch.float32).view(nz, ny, nx)

    def pack_volumes(self, vols, device="cuda"):
        """One device buffer holding the volumes at the plan's input offsets."""
        import torch
        buf = torch.zeros(max(self.input_elems, 1), dtype=torch.float32, device=device)
        for v, vol in enumerate(vols):
            info = self.volumes[v]
            nx, ny, nz = info["shape_xyz"]
            t = torch.as_tensor(np.ascontiguousarray(vol, dtype=np.float32)).reshape(-1)
            assert t.numel() == nx * ny * nz
            buf[info["offset"]:info["offset"] + t.numel()].copy_(t)
        return buf

    def alloc_workspace(self, device="cuda"):
        import torch
        return torch.empty(self.workspace_bytes, dtype=torch.uint8, device=device)

    def build_pyramid(self, vol, ws, stream=None):
        _check(_load().sift3d_build_pyramid(self.handle, _vp(vol.data_ptr()), _vp(ws.data_ptr()), ws.numel(),
                                            _vp(_stream(stream))), "sift3d_build_pyramid")

    def pyramid_passes(self):
        """[(octave, level, radius, writes_sub, algorithmic_bytes, path, volume)] in dependency order;
        path: 1 = fused streaming launch, 2 = compact launch, 0 = xy + z launches."""
        lib = _load()
        n = ctypes.c_int()
        _check(lib.sift3d_pyramid_pass_count(self.handle, ctypes.byref(n)), "sift3d_pyramid_pass_count")
        out = []
        for i in range(n.value):
            info = (ctypes.c_int * 6)()
            b = ctypes.c_size_t()
            _check(lib.sift3d_pyramid_pass_info(self.handle, i, info, ctypes.byref(b)), "sift3d_pyramid_pass_info")
            out.append((info[0], info[1], info[2], info[3], b.value, info[4], info[5]))
        return out

    def pyramid_pass(self, i, vol, ws, stream=None):
        _check(_load().sift3d_pyramid_pass(self.handle, i, _vp(_ptr(vol)), _vp(ws.data_ptr()), ws.numel(),
                                           _vp(_stream(stream))), "sift3d_pyramid_pass")

    def pyramid_steps(self):
        """Launches of build_pyramid, in order: dicts with kind (0 fused, 1 xy, 2 z,
        3 compact), level passes, pre-blurs, max radius, octave and level ranges,
        pb flag and the algorithmic bytes of the levels it completes."""
        lib = _load()
        n = ctypes.c_int()
        _check(lib.sift3d_pyramid_step_count(self.handle, ctypes.byref(n)), "sift3d_pyramid_step_count")
        out = []
        for i in range(n.value):
            info = (ctypes.c_int * 9)()
            b = ctypes.c_size_t()
            _check(lib.sift3d_pyramid_step_info(self.handle, i, info, ctypes.byref(b)), "sift3d_pyramid_step_info")
            out.append({"kind": info[0], "level_passes": info[1], "preblurs": info[2], "max_r": info[3],
                        "octaves": (info[4], info[5]), "levels": (info[6], info[7]), "pb": info[8],
                        "bytes": b.value})
        return out

    def pyramid_step(self, i, vol, ws, stream=None):
        _check(_load().sift3d_pyramid_step(self.handle, i, _vp(_ptr(vol)), _vp(ws.data_ptr()), ws.numel(),
                                           _vp(_stream(stream))), "sift3d_pyramid_step")

    def detect(self, ws, kp, count, stream=None):
        _check(_load().sift3d_detect(self.handle, _vp(ws.data_ptr()), ws.numel(), _vp(_ptr(kp)), self.capacity,
                                     _vp(count.data_ptr()), _vp(_stream(stream))), "sift3d_detect")

    def tune(self, vol, ws, reps=3, stream=None):
        """sift3d_plan_tune: time tile height and slab candidates of every fused
        launch and keep the fastest (plan-time, synchronises). Returns the records."""
        _check(_load().sift3d_plan_tune(self.handle, _vp(_ptr(vol)), _vp(ws.data_ptr()), ws.numel(), int(reps),
                                        _vp(_stream(stream))), "sift3d_plan_tune")
        return self.tuning()

    def tuning(self):
        lib = _load()
        n = ctypes.c_int()
        _check(lib.sift3d_plan_tuning_count(self.handle, ctypes.byref(n)), "sift3d_plan_tuning_count")
        out = []
        for i in range(n.value):
            info = (ctypes.c_int * 6)()
            ms = (ctypes.c_float * 2)()
            _check(lib.sift3d_plan_tuning(self.handle, i, info, ms), "sift3d_plan_tuning")
            out.append({"step": info[0], "default": {"ty": info[1], "slabs": info[2], "ms": round(ms[0], 5)},
                        "tuned": {"ty": info[3], "slabs": info[4], "ms": round(ms[1], 5)}, "candidates": info[5]})
        return out

    def detect_static(self, ws, kp, count, stream=None):
        """sift3d_detect with the library's static scratch (allocates nothing)."""
        _check(_load().sift3d_detect_static(self.handle, _vp(ws.data_ptr()), ws.numel(), _vp(_ptr(kp)),
                                            self.capacity, _vp(count.data_ptr()), _vp(_stream(stream))),
               "sift3d_detect_static")

    def detect_scratch_bytes(self):
        b = ctypes.c_size_t()
        _check(_load().sift3d_plan_detect_scratch(self.handle, ctypes.byref(b)), "sift3d_plan_detect_scratch")
        return b.value

    def describe(self, ws, kp, count, siftrank=None, brief=None, rrief=None, stream=None):
        _check(_load().sift3d_describe(self.handle, _vp(ws.data_ptr()), ws.numel(), _vp(_ptr(kp)),
                                       _vp(count.data_ptr()), self.capacity, _vp(_ptr(siftrank)),
                                       _vp(_ptr(brief)), _vp(_ptr(rrief)), _vp(_stream(stream))),
               "sift3d_describe")

    def orient(self, ws, kp, count, nframes, frames, siftrank, peak_ratio=0.8, stream=None):
        """sift3d_orient: nframes [cap*n_volumes] int32, frames [.., 4, 9] float32,
        siftrank [.., 4, 64] uint8 (torch device tensors)."""
        _check(_load().sift3d_orient(self.handle, _vp(ws.data_ptr()), ws.numel(), _vp(_ptr(kp)),
                                     _vp(count.data_ptr()), self.capacity, float(peak_ratio),
                                     _vp(_ptr(nframes)), _vp(_ptr(frames)), _vp(_ptr(siftrank)),
                                     _vp(_stream(stream))), "sift3d_orient")

    def extract(self, vol, ws, kp, count, siftrank=None, brief=None, rrief=None, stream=None):
        _check(_load().sift3d_extract(self.handle, _vp(vol.data_ptr()), _vp(ws.data_ptr()), ws.numel(),
                                      _vp(_ptr(kp)), self.capacity, _vp(count.data_ptr()), _vp(_ptr(siftrank)),
                                      _vp(_ptr(brief)), _vp(_ptr(rrief)), _vp(_stream(stream))),
               "sift3d_extract")

    def close(self):
        if getattr(self, "handle", None):
            _load().sift3d_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Buffers:
    """Device buffers (torch) for one plan: workspace, keypoints, counts, descriptors."""

    def __init__(self, plan: Plan, device="cuda"):
        import torch
        cap = max(plan.capacity, 1)
        nv = plan.n_volumes
        n = plan.ctx.params.brief_n
        self.ws = plan.alloc_workspace(device)
        self.kp = torch.zeros(nv * cap * KEYPOINT_BYTES, dtype=torch.uint8, device=device)
        self.count = torch.zeros(nv, dtype=torch.int32, device=device)
        self.siftrank = torch.zeros(nv * cap, 64, dtype=torch.uint8, device=device)
        self.brief = torch.zeros(nv * cap, max(n // 64, 1), dtype=torch.int64, device=device)
        self.rrief = torch.zeros(nv * cap, max(n, 1), dtype=torch.uint8, device=device)


def run_extract(plan: Plan, vol, buf: Buffers, stream=None):
    plan.extract(vol, buf.ws, buf.kp, buf.count, buf.siftrank, buf.brief, buf.rrief, stream=stream)


def fetch_results(plan: Plan, buf: Buffers, volume: int = 0):
    """Copy one volume's keypoints and descriptors to host numpy (synchronises)."""
    cap = max(plan.capacity, 1)
    count = int(buf.count[volume].item())
    k = min(count, plan.capacity)
    base = volume * cap
    kp = buf.kp[base * KEYPOINT_BYTES:(base + k) * KEYPOINT_BYTES].cpu().numpy().view(KEYPOINT_DTYPE)
    n = plan.ctx.params.brief_n
    return {
        "count": count,
        "keypoints": kp,
        "siftrank": buf.siftrank[base:base + k].cpu().numpy(),
        "brief": buf.brief[base:base + k].cpu().numpy().view(np.uint64)[:, : n // 64],
        "rrief": buf.rrief[base:base + k].cpu().numpy()[:, :n],
    }


class Server:
    """Continuous-batching request server (sift3d_server_*): submit device
    volumes as they arrive, poll or wait for results, release their slots."""

    def __init__(self, ctx: Context, hbm_budget: int, n_streams: int = 4, max_inflight: int = 8,
                 kp_capacity: int = 1 << 14, max_batch: int = 8, admit_timeout_s: float = 0.0):
        lib = _load()
        self.ctx = ctx
        self.capacity = int(kp_capacity)
        cfg = ServerConfig(int(hbm_budget), int(n_streams), int(max_inflight), int(kp_capacity), int(max_batch),
                           float(admit_timeout_s))
        h = ctypes.c_void_p()
        _check(lib.sift3d_server_create(ctx.handle, ctypes.byref(cfg), ctypes.byref(h)), "sift3d_server_create")
        self.handle = h
        self._inputs = {}

    @staticmethod
    def clock() -> float:
        return _load().sift3d_server_clock()

    def footprint(self, shape_xyz) -> int:
        b = ctypes.c_size_t()
        nx, ny, nz = (int(v) for v in shape_xyz)
        _check(_load().sift3d_server_footprint(self.handle, nx, ny, nz, ctypes.byref(b)), "sift3d_server_footprint")
        return b.value

    def submit(self, vol) -> int:
        """Queue one volume (a contiguous float32 [nz, ny, nx] CUDA tensor whose
        producing work has completed); returns the ticket."""
        nz, ny, nx = vol.shape
        t = ctypes.c_int64()
        _check(_load().sift3d_server_submit(self.handle, _ptr(vol), nx, ny, nz, ctypes.byref(t)),
               "sift3d_server_submit")
        self._inputs[t.value] = vol
        return t.value

    def result(self, ticket: int, wait: bool = True):
        """Result struct of a ticket, or None if wait is False and it is not finished."""
        r = Result()
        rc = _load().sift3d_server_result(self.handle, int(ticket), 1 if wait else 0, ctypes.byref(r))
        if rc == PENDING:
            return None
        _check(rc, "sift3d_server_result")
        return r

    def fetch(self, ticket: int):
        """Host copies of a finished request's keypoints and descriptors."""
        r = self.result(ticket, wait=True)
        _check(r.status, "server request")
        k = min(r.count, r.capacity)
        n = self.ctx.params.brief_n
        kp = np.zeros(k, dtype=KEYPOINT_DTYPE)
        sr = np.zeros((k, 64), dtype=np.uint8)
        br = np.zeros((k, max(n // 64, 1)), dtype=np.uint64)
        rr = np.zeros((k, max(n, 1)), dtype=np.uint8)
        _check(_load().sift3d_server_fetch(self.handle, int(ticket), kp.ctypes.data, sr.ctypes.data,
                                           br.ctypes.data if n else None, rr.ctypes.data if n else None),
               "sift3d_server_fetch")
        return {"count": r.count, "keypoints": kp, "siftrank": sr, "brief": br[:, : n // 64], "rrief": rr[:, :n]}

    def release(self, ticket: int):
        _check(_load().sift3d_server_release(self.handle, int(ticket)), "sift3d_server_release")
        self._inputs.pop(int(ticket), None)

    def stats(self) -> dict:
        c = ServerCounters()
        _check(_load().sift3d_server_stats(self.handle, ctypes.byref(c)), "sift3d_server_stats")
        return {f: getattr(c, f) for f, _ in ServerCounters._fields_}

    def close(self):
        if getattr(self, "handle", None):
            _load().sift3d_server_destroy(self.handle)
            self.handle = None
            self._inputs.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
