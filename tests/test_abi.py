"""The C library loads and exports every entry point of include/stereo.h (no GPU)."""

import ctypes
import os
import re

import pytest

import paper_2212_00488_amd as sm
from paper_2212_00488_amd.build import LIB, ROOT

HEADER = os.path.join(ROOT, "include", "stereo.h")
HEADERS = sorted(os.path.join(ROOT, "include", n) for n in os.listdir(os.path.join(ROOT, "include"))
                 if n.endswith(".h"))


def declared_functions():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names.update(re.findall(r"\b(stereo_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("stereo_create", "stereo_disparity", "stereo_destroy", "stereo_default_params",
              "stereo_disparity_batch", "stereo_get_intermediate", "stereo_last_error",
              "stereo_disparity_noalloc", "stereo_calib_lds_read", "stereo_calib_valu",
              "stereo_calib_copy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    L = ctypes.CDLL(LIB)
    for n in declared_functions():
        assert hasattr(L, n), n


def test_default_params_are_the_papers():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    p = sm.default_params()
    assert p.size == ctypes.sizeof(sm.Params) == 44
    assert abs(p.lambda_ad - 0.3) < 1e-6 and abs(p.lambda_mc - 2.3) < 1e-6
    assert (p.cost_scale, p.color_delta, p.arm_x, p.arm_y, p.fill_T, p.flags, p.arm_x_r,
            p.fill_mode) == (1024, 13, 21, 31, 3, 0, -1, 0)


def test_struct_layouts_match_header():
    """The ctypes mirrors list the header's struct members in order."""
    from paper_2212_00488_amd import binding as b
    text = open(HEADER).read()
    for cname, cls in (("stereo_params", b.Params), ("stereo_soft_params", b.SoftParams),
                       ("stereo_server_config", b.ServerConfig),
                       ("stereo_server_result", b.ServerResult)):
        body = re.search(r"typedef struct " + cname + r" \{(.*?)\} " + cname + ";", text, re.S)
        assert body, cname
        members = re.findall(r"^\s*[A-Za-z_0-9]+\s+([A-Za-z_0-9]+(?:\s*,\s*[A-Za-z_0-9]+)*);",
                             body.group(1), re.M)
        names = [n.strip() for m in members for n in m.split(",")]
        assert names == [f[0] for f in cls._fields_], (cname, names)


def test_intermediate_ids_match_header():
    text = open(HEADER).read()
    ids = dict((k.lower(), int(v)) for k, v in re.findall(r"STEREO_I_([A-Z_]+)\s*=\s*(\d+)", text))
    from paper_2212_00488_amd.binding import INTERMEDIATES, I_LUT
    for name, (which, _, _) in INTERMEDIATES.items():
        assert ids[name] == which, name
    assert ids["lut"] == I_LUT
