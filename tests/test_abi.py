"""The C ABI without a GPU: the library loads, exports every function that
include/rfsr.h declares, and rejects invalid arguments before touching the
device (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rfsr.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(\w+)\s*\(", src, flags=re.M)
    return sorted({n for n in names if n.startswith(("rfsr_", "fsr_"))})


@pytest.fixture(scope="module")
def R():
    import paper_2203_09200_amd as R
    return R


def test_header_declares_the_three_entry_points():
    names = declared_functions()
    for n in ("rfsr_reconstruct_frame", "rfsr_motion_check", "fsr_blocks", "rfsr_workspace_bytes"):
        assert n in names


def test_library_exports_every_declared_symbol(R):
    lib = R.lib()
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert lib.rfsr_version() == 10000
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.rfsr_status_string(code).startswith(b"RFSR_")


def test_workspace_bytes_validation(R):
    me, fsr = R.MEParams(), R.FSRParams()
    n = R.workspace_bytes(1080, 1920, 3, me, fsr)
    assert n > 1080 * 1920 * 20
    assert R.workspace_bytes(8, 8, 0) > 0
    lib = R.lib()
    for H, W, nref in ((0, 8, 0), (6, 8, 0), (8, 10, 0), (8, 8, 4), (20000, 8, 0)):
        assert lib.rfsr_workspace_bytes(H, W, nref, None, None) == 0


def _me(R, **kw):
    p = R.MEParams(**kw).c()
    return ctypes.byref(p), p


def test_motion_check_rejects_bad_arguments(R):
    lib = R.lib()
    P = ctypes.c_void_p
    fake = P(4096)   # never dereferenced: validation fails first
    me, _ = _me(R)
    # null inputs / outputs
    assert lib.rfsr_motion_check(None, fake, fake, 8, 8, 8, me, fake, fake, None, None, fake, 1 << 20, None) == -1
    # shapes
    assert lib.rfsr_motion_check(fake, fake, fake, 6, 8, 8, me, fake, fake, None, None, fake, 1 << 20, None) == -2
    assert lib.rfsr_motion_check(fake, fake, fake, 8, 8, 4, me, fake, fake, None, None, fake, 1 << 20, None) == -2
    # parameters
    for kw, code in (({"search": 16}, -1), ({"search": -1}, -1), ({"rmc_radius": 99}, -1),
                     ({"tmpl": 3}, -5), ({"tmpl": 0}, -1)):
        bad, _ = _me(R, **kw)
        assert lib.rfsr_motion_check(fake, fake, fake, 8, 8, 8, bad, fake, fake, None, None, fake,
                                     1 << 20, None) == code, kw
    # workspace: null, misaligned, too small
    assert lib.rfsr_motion_check(fake, fake, fake, 8, 8, 8, me, fake, fake, None, None, None, 1 << 20, None) == -3
    assert lib.rfsr_motion_check(fake, fake, fake, 8, 8, 8, me, fake, fake, None, None, P(4097), 1 << 20, None) == -3
    assert lib.rfsr_motion_check(fake, fake, fake, 8, 8, 8, me, fake, fake, None, None, fake, 16, None) == -3


def test_fsr_blocks_rejects_bad_arguments(R):
    lib = R.lib()
    fake = ctypes.c_void_p(4096)
    for kw, code in (({"iters": -1}, -1), ({"iters": 5000}, -1), ({"rho": 0.0}, -1), ({"rho": 1.5}, -1),
                     ({"gamma": 0.0}, -1), ({"gamma": 2.0}, -1), ({"proj_weight": -1.0}, -1),
                     ({"block": 8}, -5), ({"support": 16}, -5)):
        p = R.FSRParams(**kw)
        c = p.c()
        assert lib.fsr_blocks(fake, fake, 8, 8, 8, ctypes.byref(c), fake, None, fake, 1 << 20, None) == code, kw
    c = R.FSRParams().c()
    c.overwrite = 7
    assert lib.fsr_blocks(fake, fake, 8, 8, 8, ctypes.byref(c), fake, None, fake, 1 << 20, None) == -1
    c = R.FSRParams().c()
    assert lib.fsr_blocks(None, fake, 8, 8, 8, ctypes.byref(c), fake, None, fake, 1 << 20, None) == -1
    assert lib.fsr_blocks(fake, fake, 8, 8, 8, ctypes.byref(c), fake, None, fake, 8, None) == -3


def test_reconstruct_frame_rejects_bad_arguments(R):
    lib = R.lib()
    P = ctypes.c_void_p
    fake = P(4096)
    me = R.MEParams().c()
    fsr = R.FSRParams().c()
    arr = (P * 3)(4096, 4096, None)
    ok = (P * 3)(4096, 4096, 4096)
    # nref out of range, null reference entries, null out
    assert lib.rfsr_reconstruct_frame(fake, fake, 4, ok, ok, ok, 8, 8, 8, ctypes.byref(me), ctypes.byref(fsr),
                                      fake, None, None, fake, 1 << 20, None) == -1
    assert lib.rfsr_reconstruct_frame(fake, fake, 3, arr, ok, ok, 8, 8, 8, ctypes.byref(me), ctypes.byref(fsr),
                                      fake, None, None, fake, 1 << 20, None) == -1
    assert lib.rfsr_reconstruct_frame(fake, fake, 0, None, None, None, 8, 8, 8, ctypes.byref(me),
                                      ctypes.byref(fsr), None, None, None, fake, 1 << 20, None) == -1
    ev = (P * 4)(4096, None, 4096, 4096)
    assert lib.rfsr_reconstruct_frame(fake, fake, 0, None, None, None, 8, 8, 8, ctypes.byref(me),
                                      ctypes.byref(fsr), fake, None, ev, fake, 1 << 20, None) == -1
    assert lib.rfsr_reconstruct_frame(fake, fake, 0, None, None, None, 8, 8, 8, ctypes.byref(me),
                                      ctypes.byref(fsr), fake, None, None, fake, 64, None) == -3


def test_binding_refuses_host_tensors(R):
    import torch
    x = torch.zeros((8, 8), dtype=torch.uint8)
    with pytest.raises(R.RfsrError):
        R.motion_check(x, x, x)
    with pytest.raises(R.RfsrError):
        R.fsr_blocks(torch.zeros((8, 8)), x)
