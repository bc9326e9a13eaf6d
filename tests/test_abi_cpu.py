"""The C ABI library loads and exports every symbol include/artemis.h declares
(no compute calls: this runs without a GPU)."""
import os
import re
import ctypes

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "artemis.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(art_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["art_create", "art_destroy", "art_load_octree", "art_set_skin", "art_set_skeleton",
              "art_set_poses", "art_set_cameras", "art_render", "art_backward"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2202_05628_amd import _lib
    lib = _lib.load()
    for n in _declared():
        assert hasattr(lib, n), n
    # the binding's signature table covers the header exactly
    assert sorted(s[0] for s in _lib.SIGNATURES) == _declared()
    assert lib.art_version() == 10000


def test_null_context_is_rejected_without_device_work():
    from paper_2202_05628_amd import _lib
    lib = _lib.load()
    assert lib.art_create(0, None, None) == _lib.ART_EINVAL
    assert lib.art_last_error(None) == b""
    lib.art_destroy(None)
    for fn, args in [("art_load_octree", (None, 3, 1, None)), ("art_set_skin", (None, None, None)),
                     ("art_render", (None, 8, 0, None, None, 0.0, 0, None, None, None)),
                     ("art_proposal_init", (None, 1)),
                     ("art_render_ckpt", (None, 8, 0, None, None, 0.0, 0, None, None, None, 6, 3, None, None)),
                     ("art_backward_ckpt", (None, 8, 0, None, None, 0.0, 0, None, None, None, None, None, None, 6, 3,
                                            None, None))]:
        assert getattr(lib, fn)(*args) == _lib.ART_EINVAL


def test_binding_constants_match_the_header():
    """Every integer constant the header defines has the same value in the
    binding (flags, sizes and the length of the statistics record)."""
    from paper_2202_05628_amd import _lib
    src = open(os.path.join(ROOT, "include", "artemis.h")).read()
    consts = {m.group(1): int(m.group(2)) for m in re.finditer(r"^#define (ART_[A-Z0-9_]+) (\d+)u?\b", src, re.M)}
    assert {"ART_GEOM_FP32", "ART_TIMING", "ART_ASYNC", "ART_NUM_STATS"} <= set(consts)
    for name, value in consts.items():
        assert getattr(_lib, name) == value, name
