"""MI355X (gfx950) 3D SIFT-Rank hot path: HIP kernels behind a C ABI.

The compute lives in libsift3d.so (built from csrc/ by ``build.py``); the
Python side only marshals torch tensors and streams into the C ABI
declared in include/sift3d.h.
"""
from .sift3d import (  # noqa: F401
    DETECT_STATIC_SCRATCH,
    E_ARG,
    E_HIP,
    E_SCRATCH,
    E_TIMEOUT,
    E_TOO_SMALL,
    E_UNSUPPORTED,
    E_WORKSPACE,
    KEYPOINT_BYTES,
    MAX_ORIENTATIONS,
    KEYPOINT_DTYPE,
    MATCH_BRIEF,
    MATCH_RANKS,
    Buffers,
    Context,
    HoughParams,
    Params,
    Plan,
    Server,
    Sift3dError,
    box_blur,
    box_half_width,
    default_params,
    pair_offsets,
    exported_symbols,
    fetch_results,
    hough,
    hough_default_params,
    hough_workspace_bytes,
    match,
    normalize,
    run_extract,
    similarity_dict,
    units,
)
