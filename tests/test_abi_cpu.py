"""CPU checks of the C ABI: the library loads, exports every entry point that
include/smr.h declares, and rejects bad descriptors on the host before any device call."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import paper_2201_10062_amd as pkg
from paper_2201_10062_amd import smr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "smr.h")).read()
    return sorted(set(re.findall(r"^\s*(?:smr_status|const char \*)\s*(smr_\w+)\s*\(", text, flags=re.M)))


def test_header_and_binding_agree():
    assert sorted(smr.EXPORTS) == _header_functions()


def test_library_exports_every_declared_symbol():
    lib = pkg.load()
    out = subprocess.run(["nm", "-D", "--defined-only", smr.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (smr_\w+)", out))
    for name in _header_functions():
        assert name in exported, name
        assert getattr(lib, name) is not None
    assert lib.smr_version().startswith(b"smr")


@pytest.mark.parametrize("kw,status", [
    (dict(dim=4, N=7, n=4), smr.SMR_EINVAL),
    (dict(dim=0, N=7, n=4), smr.SMR_EINVAL),
    (dict(dim=3, N=255, n=4), smr.SMR_EINVAL),          # 3D: N + 1 <= 128
    (dict(dim=3, N=7, n=4, ax=np.ones((7, 7, 8)), ay=np.ones((7, 8, 7))), smr.SMR_EINVAL),   # az missing
    (dict(dim=2, N=7, n=4, ax=np.ones((7, 8)), ay=np.ones((8, 7)), az=np.ones(1)), smr.SMR_EINVAL),
    (dict(dim=3, N=7, n=4, a_nodal=np.ones((9, 9, 9))), smr.SMR_EINVAL),   # 3D takes face values
    (dict(dim=2, N=7, n=4, pinv="f32"), smr.SMR_EINVAL),               # float32 intermediates: float32 plans only
    (dict(dim=2, N=6, n=4), smr.SMR_EINVAL),           # N + 1 not a power of two
    (dict(dim=2, N=1023, n=4), smr.SMR_EINVAL),        # N too large
    (dict(dim=2, N=7, n=0), smr.SMR_EINVAL),
    (dict(dim=2, N=7, n=1, scheme="bdf2"), smr.SMR_EINVAL),
    (dict(dim=2, N=7, n=3, scheme="bdf4"), smr.SMR_EINVAL),         # BDF-l needs n >= l
    (dict(dim=2, N=7, n=8, scheme="bdf3", precond="PTHETA_CHEB"), smr.SMR_EINVAL),
    (dict(dim=2, N=7, n=4, theta=1.5), smr.SMR_EINVAL),
    (dict(dim=2, N=7, n=4, T=-1.0), smr.SMR_EINVAL),
    (dict(dim=2, N=7, n=4, precond="PTHETA_CHEB", cheb_k=0), smr.SMR_EINVAL),
    (dict(dim=2, N=7, n=4, precond="PTHETA_CHEB", scheme="bdf2"), smr.SMR_EINVAL),
    (dict(dim=2, N=7, n=257, tile_cols=32), smr.SMR_EUNSUPPORTED),   # ceil(n/2) > 128
])
def test_invalid_descriptors_rejected_on_host(kw, status):
    with pytest.raises(smr.SmrError) as ei:
        smr.workspace_size(**kw)
    assert ei.value.status == status


def test_tile_width_flags_checked_on_host():
    assert smr.workspace_size(dim=2, N=7, n=256, tile_cols=32) == smr.workspace_size(dim=2, N=7, n=256)
    assert smr.workspace_size(dim=2, N=7, n=512, tile_cols=16) > 0
    lib = pkg.load()
    d, keep = smr.make_desc(2, 7, 4)
    d.flags = smr.FLAG_TILE16 | smr.FLAG_TILE32
    out = ctypes.c_size_t(0)
    assert lib.smr_workspace_size(ctypes.byref(d), ctypes.byref(out)) == smr.SMR_EINVAL
    assert b"exclude" in lib.smr_last_error()
    d.flags = 1024                    # no such flag
    assert lib.smr_workspace_size(ctypes.byref(d), ctypes.byref(out)) == smr.SMR_EINVAL
    with pytest.raises(ValueError):
        smr.make_desc(2, 7, 4, tile_cols=24)
    cols = ctypes.c_int32(-1)
    assert lib.smr_tile_cols(None, ctypes.byref(cols)) == smr.SMR_EINVAL


def test_setup_rejects_bad_workspace_before_device_work():
    lib = pkg.load()
    d, keep = smr.make_desc(2, 7, 4)
    h = ctypes.c_void_p(0)
    st = lib.smr_setup(ctypes.byref(d), None, 0, None, ctypes.byref(h))
    assert st == smr.SMR_EWORKSPACE
    st = lib.smr_setup(ctypes.byref(d), ctypes.c_void_p(256), 16, None, ctypes.byref(h))
    assert st == smr.SMR_EWORKSPACE and b"too small" in lib.smr_last_error()
    st = lib.smr_setup(ctypes.byref(d), ctypes.c_void_p(8), 1 << 30, None, ctypes.byref(h))
    assert st == smr.SMR_EWORKSPACE and b"aligned" in lib.smr_last_error()


def test_null_plan_rejected():
    lib = pkg.load()
    assert lib.smr_apply_A(None, None, None, None) == smr.SMR_EINVAL
    assert lib.smr_minres_solve(None, None, None, None, 1e-8, 10, None, None) == smr.SMR_EINVAL


def test_pinv_flags_checked_on_host():
    assert smr.workspace_size(dim=2, N=7, n=4, pprec="fp32", pinv="f32c16") > 0
    assert smr.workspace_size(dim=2, N=7, n=4, pinv="f64c16") > 0
    d, keep = smr.make_desc(2, 7, 4, pprec="fp32")
    d.flags = smr.PINV_FLAGS["f32"] | smr.PINV_FLAGS["f64"]
    out = ctypes.c_size_t(0)
    assert pkg.load().smr_workspace_size(ctypes.byref(d), ctypes.byref(out)) == smr.SMR_EINVAL
    with pytest.raises(ValueError):
        smr.make_desc(2, 7, 4, pinv="bf16")


def test_matvec_flags_checked_on_host():
    """The N = 127 variable-coefficient sine-basis plan holds four more level-sized vectors (for
    the tiled per-level matvec); the two forms exclude each other; other plans are unchanged."""
    ax, ay = np.full((127, 128), 1.3), np.full((128, 127), 1.3)
    ax[3, 4] = 1.7
    base = smr.workspace_size(dim=2, N=127, n=16, scheme="bdf2", ax=ax, ay=ay)
    const = smr.workspace_size(dim=2, N=127, n=16, scheme="bdf2")
    assert base > const
    assert smr.workspace_size(dim=2, N=127, n=16, scheme="bdf2", ax=ax, ay=ay, matvec="level") == base
    assert smr.workspace_size(dim=2, N=127, n=16, scheme="bdf2", ax=ax, ay=ay, matvec="tiles") == base
    assert smr.workspace_size(dim=2, N=63, n=16, matvec="tiles") == smr.workspace_size(dim=2, N=63, n=16)
    d, keep = smr.make_desc(2, 127, 16, ax=ax, ay=ay)
    d.flags = smr.MATVEC_FLAGS["level"] | smr.MATVEC_FLAGS["tiles"]
    out = ctypes.c_size_t(0)
    lib = pkg.load()
    assert lib.smr_workspace_size(ctypes.byref(d), ctypes.byref(out)) == smr.SMR_EINVAL
    assert b"exclude" in lib.smr_last_error()
    with pytest.raises(ValueError):
        smr.make_desc(2, 7, 4, matvec="fft")
    t = ctypes.c_int32(-1)
    assert lib.smr_matvec_tiles(None, ctypes.byref(t)) == smr.SMR_EINVAL


def test_tune_stats_on_host():
    smr.tune_reset()
    assert smr.tune_stats() == (0, 0, 0)


def test_desc_fields_match_header():
    """The binding's smr_desc mirrors the C struct field by field (names and order)."""
    text = open(os.path.join(ROOT, "include", "smr.h")).read()
    body = re.search(r"typedef struct \{(.*?)\} smr_desc;", text, flags=re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = re.findall(r"(\w+)\s*;", body)
    assert names == [f[0] for f in smr.SmrDesc._fields_]


def test_3d_workspace_sizes():
    a = smr.workspace_size(dim=3, N=63, n=64)
    assert a > 10 * 8 * 63 ** 3 * 64          # the ten work vectors alone
    assert smr.workspace_size(dim=3, N=127, n=8) > a / 2
    faces = dict(ax=np.ones((7, 7, 8)), ay=np.ones((7, 8, 7)), az=np.ones((8, 7, 7)))
    assert smr.workspace_size(dim=3, N=7, n=4, **faces) == smr.workspace_size(dim=3, N=7, n=4)


def test_workspace_size_grows_with_problem():
    a = smr.workspace_size(dim=2, N=31, n=64)
    b = smr.workspace_size(dim=2, N=127, n=256)
    assert b > 16 * a * 0.9
    c = smr.workspace_size(dim=2, N=127, n=256, precond="PTHETA_CHEB")
    assert c > b
