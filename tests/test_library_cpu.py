"""Host-side checks of the HIP library that need no GPU: the shared library loads,
exports every entry point declared in include/pic.h, and validates its inputs."""
import ctypes as C
import os
import re

import pytest

from paper_2602_15130_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pic.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|int64_t|void|const char\*)\s+(pic_\w+)\s*\(", src, re.M)))


def test_header_declares_the_four_core_calls():
    names = _declared()
    for n in ("pic_init_manufactured", "pic_step", "pic_collide", "pic_errors"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2602_15130_amd import pic

    for n in _declared():
        assert hasattr(pic.lib, n), n
        assert n in pic.EXPORTED


def test_workspace_size_and_validation():
    from paper_2602_15130_amd import pic

    c = W.get("cfg2")
    b = pic.pic_workspace_size(c["problem"], c["disc"], "fp64")
    # x, v, id double-buffered (104 B), sort keys/slots (16 B), collision output and
    # scratch (48 B): at least 168 B per particle
    assert b >= 168 * c["disc"]["np"]
    bad = dict(c["disc"])
    bad["nc"] = (2, 64, 64)
    with pytest.raises(pic.PicError) as e:
        pic.pic_workspace_size(c["problem"], bad, "fp64")
    assert e.value.code == pic.PIC_EINVAL
    bad = dict(c["disc"])
    bad["np"] = 0
    with pytest.raises(pic.PicError):
        pic.pic_workspace_size(c["problem"], bad, "fp64")
    p = dict(c["problem"])
    p["omega"] = 0.7
    with pytest.raises(pic.PicError):
        pic.pic_workspace_size(p, c["disc"], "fp64")
    p = W.paper_problem()
    p["sigma_model"] = "vhs"
    p["omega"] = 0.5
    with pytest.raises(pic.PicError):  # hard sphere has no closed-form source for the paper f_v
        pic.pic_workspace_size(p, c["disc"], "fp64")


def test_init_without_gpu_or_workspace_fails_cleanly():
    from paper_2602_15130_amd import pic

    c = W.get("cfg0")
    with pytest.raises(pic.PicError) as e:
        pic.pic_init_manufactured(c["problem"], c["disc"], 1, 0, "fp64", 0, 0, 0)
    assert e.value.code in (pic.PIC_ESPACE, pic.PIC_EINVAL)
