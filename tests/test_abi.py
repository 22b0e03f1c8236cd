"""The C interface: the built library loads on the host and exports every
function that include/*.h declares (no compute call is made here)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1703_06680_amd", "libddm.so")


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b(ddm_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1703_06680_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_entry_points():
    names = declared_functions()
    assert {"ddm_match", "ddm_workspace_bytes", "ddm_strerror"} <= set(names)


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_host_only_queries(lib):
    lib.ddm_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_int64]
    lib.ddm_workspace_bytes.restype = ctypes.c_size_t
    assert lib.ddm_workspace_bytes(1000, 1000, 2, 0, 0) > 0
    assert lib.ddm_workspace_bytes(-1, 10, 2, 0, 0) == 0
    assert lib.ddm_workspace_bytes(10, 10, 0, 0, 0) == 0
    assert lib.ddm_workspace_bytes(10, 10, 17, 0, 0) == 0
    assert lib.ddm_workspace_bytes(10, 10, 2, 7, 0) == 0
    assert lib.ddm_workspace_bytes(2**30, 2**30, 1, 0, 0) == 0
    # pair capacity grows the pair workspace only in pair mode
    assert lib.ddm_workspace_bytes(10, 10, 2, 2, 10**6) > lib.ddm_workspace_bytes(10, 10, 2, 2, 0)
    assert lib.ddm_workspace_bytes(10, 10, 2, 0, 10**6) == lib.ddm_workspace_bytes(10, 10, 2, 0, 0)
    # the closed-interval flag (16) changes no buffer size; other bits are rejected
    for mode in (0, 1, 2):
        assert lib.ddm_workspace_bytes(500, 700, 3, mode | 16, 1000) == \
            lib.ddm_workspace_bytes(500, 700, 3, mode, 1000)
    assert lib.ddm_workspace_bytes(10, 10, 2, 32, 0) == 0
    assert lib.ddm_workspace_bytes(10, 10, 2, 16 | 3, 0) == 0
    lib.ddm_strerror.restype = ctypes.c_char_p
    assert b"workspace" in lib.ddm_strerror(-3)


def test_host_side_argument_errors_return_before_any_launch(lib):
    """Calls that fail host-side checks never touch the device, so they can
    run without a GPU."""
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    lib.ddm_match.argtypes = [vp, vp, i64, vp, vp, i64, ctypes.c_int, ctypes.c_int, vp,
                              ctypes.c_size_t, vp, ctypes.POINTER(ctypes.c_uint64), vp, vp, i64]
    lib.ddm_match.restype = ctypes.c_int
    cnt = ctypes.c_uint64(7)
    fake = ctypes.c_void_p(0x1000)
    # negative n, bad d, bad mode, missing count pointer, NULL data
    assert lib.ddm_match(fake, fake, -1, fake, fake, 1, 1, 0, fake, 1 << 30, None, ctypes.byref(cnt), None, None, 0) == -1
    assert lib.ddm_match(fake, fake, 1, fake, fake, 1, 0, 0, fake, 1 << 30, None, ctypes.byref(cnt), None, None, 0) == -1
    assert lib.ddm_match(fake, fake, 1, fake, fake, 1, 1, 9, fake, 1 << 30, None, ctypes.byref(cnt), None, None, 0) == -1
    assert lib.ddm_match(fake, fake, 1, fake, fake, 1, 1, 16 | 3, fake, 1 << 30, None, ctypes.byref(cnt), None, None, 0) == -1
    assert lib.ddm_match(fake, fake, 1, fake, fake, 1, 1, 0, fake, 1 << 30, None, None, None, None, 0) == -1
    assert lib.ddm_match(None, fake, 1, fake, fake, 1, 1, 0, fake, 1 << 30, None, ctypes.byref(cnt), None, None, 0) == -1
    # per-update mode without the output, pair mode without the pair buffer
    assert lib.ddm_match(fake, fake, 1, fake, fake, 1, 1, 1, fake, 1 << 30, None, ctypes.byref(cnt), None, None, 0) == -1
    assert lib.ddm_match(fake, fake, 1, fake, fake, 1, 1, 2, fake, 1 << 30, None, ctypes.byref(cnt), None, None, 5) == -1
    # workspace one byte short
    need = lib.ddm_workspace_bytes(5, 5, 2, 0, 0)
    assert lib.ddm_match(fake, fake, 5, fake, fake, 5, 2, 0, fake, need - 1, None, ctypes.byref(cnt), None, None, 0) == -3
    assert lib.ddm_match(fake, fake, 5, fake, fake, 5, 2, 0, None, need, None, ctypes.byref(cnt), None, None, 0) == -3


def test_resident_sizes_and_argument_errors(lib):
    """Resident-simulation entry points: state sizes and the checks that
    return before any device call."""
    vp, i64, f32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_float
    lib.ddm_resident_bytes.argtypes = [i64, i64, ctypes.c_int]
    lib.ddm_resident_bytes.restype = ctypes.c_size_t
    small = lib.ddm_resident_bytes(1000, 1000, 2)
    assert small > 0 and small % 256 == 0
    assert lib.ddm_resident_bytes(100000, 100000, 2) > small
    # one slab per bucket of about 1536 regions: at least a slab of 2048
    # records (16 bytes) and coordinates per region slot
    assert lib.ddm_resident_bytes(100000, 100000, 2) >= (200000 // 1536) * 2048 * (16 + 4 + 16)
    assert lib.ddm_resident_bytes(10, 10, 7) > 0      # d > 3: matched by the full call
    assert lib.ddm_resident_bytes(0, 0, 2) > 0        # nothing to match, still a state
    assert lib.ddm_resident_bytes(-1, 10, 2) == 0
    assert lib.ddm_resident_bytes(10, 10, 0) == 0
    assert lib.ddm_resident_bytes(10, 10, 17) == 0
    assert lib.ddm_resident_bytes(2**30, 2**30, 1) == 0
    lib.ddm_resident_create.argtypes = [vp, ctypes.c_size_t, vp, vp, i64, vp, vp, i64,
                                        ctypes.c_int, f32, f32, ctypes.c_uint64, vp,
                                        ctypes.POINTER(vp)]
    lib.ddm_resident_create.restype = ctypes.c_int
    fake, state = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x100000)
    out = ctypes.c_void_p(None)
    need = lib.ddm_resident_bytes(5, 5, 2)

    def create(**kw):
        a = dict(state=state, size=need, n=5, m=5, d=2, side=1.0, sigma=0.1, out=ctypes.byref(out))
        a.update(kw)
        return lib.ddm_resident_create(a["state"], a["size"], fake, fake, a["n"], fake, fake,
                                       a["m"], a["d"], a["side"], a["sigma"], 1, None, a["out"])

    assert create(out=None) == -1
    assert create(n=-1) == -1
    assert create(d=0) == -1
    assert create(side=float("nan")) == -1
    assert create(side=-1.0) == -1
    assert create(side=float("inf")) == -1
    assert create(sigma=float("nan")) == -1
    assert create(sigma=1e31) == -1
    assert create(state=ctypes.c_void_p(0x100010)) == -1  # not 256-byte aligned
    assert create(state=None) == -1
    assert create(size=need - 1) == -3
    assert out.value is None
    for name in ("ddm_resident_step", "ddm_resident_finish", "ddm_resident_export",
                 "ddm_resident_get_info"):
        getattr(lib, name).restype = ctypes.c_int
    lib.ddm_resident_step.argtypes = [vp, ctypes.c_uint32, vp]
    assert lib.ddm_resident_step(None, 1, None) == -1
    lib.ddm_resident_finish.argtypes = [vp, vp]
    assert lib.ddm_resident_finish(None, None) == -1
    lib.ddm_resident_export.argtypes = [vp, vp, vp, vp, vp, vp]
    assert lib.ddm_resident_export(None, fake, fake, fake, fake, None) == -1
    lib.ddm_resident_get_info.argtypes = [vp, vp]
    assert lib.ddm_resident_get_info(None, None) == -1
    lib.ddm_resident_destroy.argtypes = [vp]
    lib.ddm_resident_destroy.restype = ctypes.c_int
    assert lib.ddm_resident_destroy(None) == 0


def test_noalloc_refuses_oversize_requests_before_touching_the_gpu(lib):
    """ddm_match_noalloc checks the sizes against its static array first, so
    these calls return without any HIP call (no GPU is needed here)."""
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    f = lib.ddm_match_noalloc
    f.argtypes = [vp, vp, i64, vp, vp, i64, ctypes.c_int, ctypes.c_int, vp,
                  ctypes.POINTER(ctypes.c_uint64), vp, vp, i64]
    f.restype = ctypes.c_int
    lib.ddm_workspace_bytes.argtypes = [i64, i64, ctypes.c_int, ctypes.c_int, i64]
    lib.ddm_workspace_bytes.restype = ctypes.c_size_t
    scratch = 64 << 20
    fake = vp(256)  # never dereferenced: the calls below end on the host
    cnt = ctypes.c_uint64(0)
    for d, n in ((1, 1_400_000), (2, 1_100_000), (3, 900_000)):
        assert lib.ddm_workspace_bytes(n, n, d, 0, 0) > scratch
        assert f(fake, fake, n, fake, fake, n, d, 0, None, ctypes.byref(cnt), None, None, 0) == -6
        assert f(fake, fake, n, fake, fake, n, d, 1, None, ctypes.byref(cnt), fake, None, 0) == -6
    # a pair capacity beyond the array is refused the same way
    assert lib.ddm_workspace_bytes(1000, 1000, 2, 2, 10**7) > scratch
    assert f(fake, fake, 1000, fake, fake, 1000, 2, 2, None, ctypes.byref(cnt), None, fake,
             10**7) == -6
    # argument errors come first
    assert f(fake, fake, -1, fake, fake, 10, 2, 0, None, ctypes.byref(cnt), None, None, 0) == -1
    assert f(fake, fake, 10, fake, fake, 10, 2, 0, None, None, None, None, 0) == -1
    assert f(fake, fake, 10, fake, fake, 10, 2, 7, None, ctypes.byref(cnt), None, None, 0) == -1
    lib.ddm_strerror.argtypes = [ctypes.c_int]
    lib.ddm_strerror.restype = ctypes.c_char_p
    assert b"scratch" in lib.ddm_strerror(-6)


def test_copy_probe_rejects_bad_arguments_before_touching_the_gpu(lib):
    """ddm_copy_probe checks pointers, alignment, size and repeat count on the
    host first (no GPU is needed for these calls)."""
    vp = ctypes.c_void_p
    f = lib.ddm_copy_probe
    f.argtypes = [vp, vp, ctypes.c_size_t, ctypes.c_int, vp, ctypes.POINTER(ctypes.c_double)]
    f.restype = ctypes.c_int
    ms = ctypes.c_double(0.0)
    a, b = vp(256), vp(512)  # never dereferenced
    assert f(None, b, 64, 1, None, ctypes.byref(ms)) == -1
    assert f(a, None, 64, 1, None, ctypes.byref(ms)) == -1
    assert f(a, b, 64, 1, None, None) == -1
    assert f(a, b, 64, 0, None, ctypes.byref(ms)) == -1
    assert f(a, b, 60, 1, None, ctypes.byref(ms)) == -1
    assert f(vp(264), b, 64, 1, None, ctypes.byref(ms)) == -1
