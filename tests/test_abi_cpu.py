"""CPU checks of the C ABI: the library loads, exports every declared entry
point, and its host-only functions behave (no compute calls)."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle as O
from gen import phantoms as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sift3d.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sift3d_[a-z_]+)\s*\(", src)))


def test_header_declares_the_hot_path_calls():
    names = _declared()
    for n in ("sift3d_build_pyramid", "sift3d_detect", "sift3d_describe", "sift3d_extract"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2112_10258_amd.sift3d as S
    lib = ctypes.CDLL(S.LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n), n


def test_default_params_and_error_strings():
    import paper_2112_10258_amd as S
    p = S.default_params()
    assert (p.scales, p.sigma0, p.votes, p.brief_n, p.min_dim) == (3, 1.6, 80, 256, 16)
    assert p.brief_blur == pytest.approx(0.95)
    lib = S.sift3d._load()
    for code in (0, -1, -2, -3, -5, -6):
        assert lib.sift3d_error_string(code)
    assert ctypes.sizeof(S.Params) == 80


def test_pair_offsets_host_function_matches_oracle():
    import paper_2112_10258_amd as S
    for m in range(1, 6):
        for n in (64, 128, 256):
            p = S.default_params(brief_n=n, brief_method=m)
            draws = P.pair_draws(3 + m, n)
            for s in (1, 2, 3):
                want = O.pair_offsets(draws, O.Params(brief_n=n, brief_method=m), s)
                assert np.array_equal(S.pair_offsets(p, draws, s), want), (m, n, s)


def test_bad_params_rejected():
    import paper_2112_10258_amd as S
    draws = P.pair_draws()
    for kw in (dict(brief_n=100), dict(votes=0), dict(votes=81), dict(scales=0), dict(min_dim=2),
               dict(pyramid_mode=4), dict(pyramid_mode=-1), dict(brief_method=0), dict(brief_method=6)):
        with pytest.raises(S.Sift3dError) as ei:
            S.pair_offsets(S.default_params(**kw), draws, 1)
        assert ei.value.code == -1
    with pytest.raises(S.Sift3dError) as ei:
        S.pair_offsets(S.default_params(siftrank_factor=5.0), draws, 1)
    assert ei.value.code == -6
    # the paper's sigma_b sweep reaches 3.05 (pre-blur radius 10); past radius 10 is refused
    S.pair_offsets(S.default_params(brief_blur=3.05), draws, 1)
    with pytest.raises(S.Sift3dError) as ei:
        S.pair_offsets(S.default_params(brief_blur=3.4), draws, 1)
    assert ei.value.code == -6
    with pytest.raises(S.Sift3dError):
        S.pair_offsets(S.default_params(), draws[:10], 1)


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors have the sizes and field offsets the C compiler
    gives the header's structs."""
    import shutil
    import subprocess

    import paper_2112_10258_amd.sift3d as S
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    mirrors = {"sift3d_params": S.Params, "sift3d_server_config": S.ServerConfig,
               "sift3d_result": S.Result, "sift3d_server_counters": S.ServerCounters,
               "sift3d_hough_params": S.HoughParams, "sift3d_similarity": S.Similarity}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "sift3d.h"', "int main(void) {"]
    for cname, py in mirrors.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append('printf("sift3d_keypoint %zu\\n", sizeof(sift3d_keypoint));')
    for f in S.KEYPOINT_DTYPE.names:
        lines.append(f'printf("sift3d_keypoint.{f} %zu\\n", offsetof(sift3d_keypoint, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True, check=True)
               .stdout.splitlines())
    for cname, py in mirrors.items():
        assert int(got[cname]) == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(py, f).offset, (cname, f)
    assert int(got["sift3d_keypoint"]) == S.KEYPOINT_DTYPE.itemsize
    for f in S.KEYPOINT_DTYPE.names:
        assert int(got[f"sift3d_keypoint.{f}"]) == S.KEYPOINT_DTYPE.fields[f][1], f


def test_match_argument_checks():
    """sift3d_match validates kind, row length and sizes on the host (no launch)."""
    import paper_2112_10258_amd as S
    lib = S.sift3d._load()
    null = None
    assert lib.sift3d_match(0, null, 0, null, 5, 4, null, null, null, null) == 0     # n_a = 0: nothing to do
    assert lib.sift3d_match(2, null, 1, null, 1, 4, null, null, null, null) == -1    # kind
    assert lib.sift3d_match(0, null, 1, null, 1, 5, null, null, null, null) == -1    # 5 BRIEF words
    assert lib.sift3d_match(1, null, 1, null, 1, 100, null, null, null, null) == -1  # ranks not a multiple of 64
    assert lib.sift3d_match(1, null, 1, null, 1, 64, null, null, null, null) == -1   # null pointers
    assert lib.sift3d_match(1, null, -1, null, 1, 64, null, null, null, null) == -1  # negative size


def test_box_half_width_host_function_matches_oracle():
    import paper_2112_10258_amd as S
    for m in (1, 2, 3, 4):
        for sigma in (0.0, 0.5, 0.95, 1.2263, 1.6, 2.0, 2.4525, 3.09, 5.0, 8.0):
            assert S.box_half_width(sigma, m) == O.box_half_width(sigma, m), (sigma, m)
    for sigma, m in ((-1.0, 3), (1.0, 0)):
        with pytest.raises(S.Sift3dError) as ei:
            S.box_half_width(sigma, m)
        assert ei.value.code == -1


def test_box_blur_argument_checks():
    """Refused before any device call: null or aliased buffers, empty or
    oversized dims,
    pass counts outside 1..4, half-widths outside 0..8, reach above 28."""
    import paper_2112_10258_amd.sift3d as S
    lib = S._load()
    a, b, c = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000), ctypes.c_void_p(0x3000)
    bad = [
        (None, b, c, 8, 8, 8, 1, 3), (a, None, c, 8, 8, 8, 1, 3), (a, b, None, 8, 8, 8, 1, 3),
        (a, a, c, 8, 8, 8, 1, 3), (a, b, b, 8, 8, 8, 1, 3), (a, b, a, 8, 8, 8, 1, 3),
        (a, b, c, 0, 8, 8, 1, 3), (a, b, c, 8, -1, 8, 1, 3), (a, b, c, 8, 8, 0, 1, 3),
        (a, b, c, 8, 8, 8, 1, 0), (a, b, c, 8, 8, 8, 1, 5), (a, b, c, 8, 8, 8, -1, 3),
        (a, b, c, 8, 8, 8, 8, 4), (a, b, c, 8, 8, 8, 15, 2), (a, b, c, 8, 8, 8, 9, 1), (a, b, c, 1 << 16, 1 << 15, 1, 1, 1), (a, b, c, 1, 1, (1 << 30) + 1, 1, 1),
    ]
    for args in bad:
        assert lib.sift3d_box_blur(*args, None) == -1, args


def test_box_blur_binding_rejects_host_tensors():
    import torch

    import paper_2112_10258_amd as S
    with pytest.raises(ValueError):
        S.box_blur(torch.zeros(4, 5, 6), 1, 3)


def test_matching_entry_points_validate_on_host():
    """sift3d_normalize, sift3d_units and sift3d_hough check their
    arguments before any launch; the Hough defaults and workspace sizes are
    host computations."""
    import ctypes

    import paper_2112_10258_amd.sift3d as S
    lib = S._load()
    null = None
    # normalize: n = 0 is a no-op; bad kind, row length or null pointers fail
    assert lib.sift3d_normalize(1, null, 0, 64, null, null) == 0
    assert lib.sift3d_normalize(2, null, 1, 64, null, null) == -1
    assert lib.sift3d_normalize(0, null, 1, 5, null, null) == -1
    assert lib.sift3d_normalize(1, null, 1, 100, null, null) == -1
    assert lib.sift3d_normalize(1, null, 1, 64, null, null) == -1
    assert lib.sift3d_normalize(1, null, -1, 64, null, null) == -1
    # units: null outputs, negative capacity, frames missing, half a copy
    fake = ctypes.c_void_p(4096)
    assert lib.sift3d_units(null, fake, 4, null, null, null, 0, fake, fake, null, fake, null) == -1
    assert lib.sift3d_units(fake, fake, -1, null, null, null, 0, fake, fake, null, fake, null) == -1
    assert lib.sift3d_units(fake, fake, 4, fake, null, null, 0, fake, fake, null, fake, null) == -1
    assert lib.sift3d_units(fake, fake, 4, null, null, fake, 64, fake, fake, null, fake, null) == -1
    assert lib.sift3d_units(fake, fake, 4, null, null, fake, 6, fake, fake, fake, fake, null) == -1
    # Hough defaults and workspace
    hp = S.HoughParams()
    assert lib.sift3d_hough_default_params(145, 174, 145, ctypes.byref(hp)) == 0
    assert hp.trans_bin == 43.5 and tuple(hp.centre) == (72.0, 86.5, 72.0) and hp.iterations == 2
    assert abs(hp.angle_bin - math.pi / 6) < 1e-15 and hp.scale_bin == 1.0
    assert hp.inlier_sigmas == 2.0 and hp.inlier_log2s == 0.5
    assert lib.sift3d_hough_default_params(0, 1, 1, ctypes.byref(hp)) == -1
    b = ctypes.c_size_t()
    assert lib.sift3d_hough_workspace(1000, ctypes.byref(b)) == 0
    assert b.value >= 2 * 128 * 1000 * 12 + 8 * 1000
    assert lib.sift3d_hough_workspace(-1, ctypes.byref(b)) == -1
    assert lib.sift3d_hough_workspace((1 << 21) + 1, ctypes.byref(b)) == -1
    ws = ctypes.c_void_p(1 << 20)
    good = S.HoughParams()
    lib.sift3d_hough_default_params(64, 64, 64, ctypes.byref(good))
    for field, bad in (("scale_bin", 0.0), ("angle_bin", -1.0), ("trans_bin", float("nan")),
                       ("inlier_sigmas", -0.5), ("inlier_log2s", float("inf")), ("iterations", 0),
                       ("iterations", 17)):
        hp = S.HoughParams.from_buffer_copy(good)
        setattr(hp, field, bad)
        assert lib.sift3d_hough(fake, 4, fake, 4, fake, ctypes.byref(hp), ws, 1 << 30, fake, fake, null) == -1, field
    # short workspace
    assert lib.sift3d_hough(fake, 4, fake, 4, fake, ctypes.byref(good), ws, 16, fake, fake, null) == -3
    # null pointers with work to do
    assert lib.sift3d_hough(null, 4, fake, 4, fake, ctypes.byref(good), ws, 1 << 30, fake, fake, null) == -1
    assert lib.sift3d_hough(fake, 4, fake, 4, fake, ctypes.byref(good), null, 1 << 30, fake, fake, null) == -1
