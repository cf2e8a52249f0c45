"""CPU checks of the C ABI: the library loads, exports every declared entry
point, and its host-only functions behave (no compute calls)."""
import ctypes
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
    for n in (64, 256):
        p = S.default_params(brief_n=n)
        draws = P.pair_draws(3, n)
        for s in (1, 2, 3):
            assert np.array_equal(S.pair_offsets(p, draws, s), O.pair_offsets(draws, O.Params(brief_n=n), s))


def test_bad_params_rejected():
    import paper_2112_10258_amd as S
    draws = P.pair_draws()
    for kw in (dict(brief_n=100), dict(votes=0), dict(votes=81), dict(scales=0), dict(min_dim=2),
               dict(pyramid_mode=3)):
        with pytest.raises(S.Sift3dError) as ei:
            S.pair_offsets(S.default_params(**kw), draws, 1)
        assert ei.value.code == -1
    with pytest.raises(S.Sift3dError) as ei:
        S.pair_offsets(S.default_params(siftrank_factor=5.0), draws, 1)
    assert ei.value.code == -6
    with pytest.raises(S.Sift3dError):
        S.pair_offsets(S.default_params(), draws[:10], 1)
