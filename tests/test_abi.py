"""CPU checks of the C-ABI library: it loads, exports every entry point that
include/pic.h declares, the Python binding covers exactly those, and the
host-side argument validation of pic_create works without a GPU."""
import ctypes as C
import math
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pic.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2208_08038_amd import pic
    if not os.path.exists(pic.LIB_PATH):
        from paper_2208_08038_amd.build import build
        build()
    return pic.load_library()


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pic_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ["pic_create", "pic_load_particles", "pic_step", "pic_diagnostics",
                 "pic_destroy", "pic_last_error"]:
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    from paper_2208_08038_amd import pic
    out = subprocess.run(["nm", "-D", "--defined-only", pic.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (pic_[a-z_]+)", out))
    for name in _declared():
        assert name in exported, name
        assert hasattr(lib, name)


def test_binding_covers_the_header():
    from paper_2208_08038_amd import pic
    assert sorted(n for n, _, _ in pic.SIGNATURES) == _declared()


def _cfg(pic, **kw):
    c = pic.PicConfig()
    c.ndim = kw.get("ndim", 1)
    c.precision = kw.get("precision", 64)
    c.pad = 3
    for d in range(3):
        c.n[d] = kw.get("n", 64)
        c.dx[d] = 0.1
        c.bc_lo[d] = c.bc_hi[d] = 0
    c.dt = kw.get("dt", 0.05)
    return c


@pytest.mark.parametrize("bad", [
    {"dt": 0.2},                       # CFL violated in 1D (dt >= dx)
    {"ndim": 3, "dt": 0.06},           # CFL violated in 3D (0.1/sqrt(3) = 0.0577)
    {"ndim": 4},
    {"precision": 16},
    {"ndim": 3, "n": 2048, "dt": 0.05},  # 3 x 11 bits > 31 for the packed cell
])
def test_create_rejects_invalid_config_on_host(lib, bad):
    from paper_2208_08038_amd import pic
    cfg = _cfg(pic, **bad)
    ctx = C.c_void_p()
    rc = lib.pic_create(C.byref(cfg), None, None, C.byref(ctx))
    assert rc == pic.PIC_EINVAL
    assert not ctx.value
    assert len(lib.pic_last_error(None)) > 0


def test_create_requires_an_allocator(lib):
    """The library allocates device memory only through the caller's
    allocator: a valid configuration with no allocator is refused on the host,
    before any HIP call."""
    from paper_2208_08038_amd import pic
    cfg = _cfg(pic)
    ctx = C.c_void_p()
    rc = lib.pic_create(C.byref(cfg), None, None, C.byref(ctx))
    assert rc == pic.PIC_EINVAL
    assert not ctx.value
    assert b"allocator" in lib.pic_last_error(None)
    half = pic.PicAllocator()  # alloc and free left NULL
    rc = lib.pic_create(C.byref(cfg), C.byref(half), None, C.byref(ctx))
    assert rc == pic.PIC_EINVAL and b"allocator" in lib.pic_last_error(None)


def test_version_string(lib):
    assert b"gfx950" in lib.pic_version()
