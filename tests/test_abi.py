"""The C ABI without a GPU: the library loads, exports every function that
include/rfsr.h declares, and rejects invalid arguments before touching the
device (no compute calls here)."""
import ctypes
import os
import re
import struct

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
    assert lib.rfsr_version() == 10800
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
                     ({"block": 8}, -5), ({"support": 16}, -5),
                     ({"prior_sigma": -0.1}, -1), ({"prior_sigma": 1.5}, -1), ({"stop_ratio": -1.0}, -1),
                     ({"stop_ratio": 1.0}, -1), ({"prior_sigma": 0.8, "pairs": True}, -5),
                     ({"stop_ratio": 0.01, "precision": "bf16x3"}, -5),
                     ({"prior_sigma": 0.8, "concealed_weight": 0.5}, -5),
                     ({"precision": "fp32", "pairs": True}, -5),
                     ({"precision": "fp32", "concealed_weight": 0.5}, -5),
                     ({"precision": "fp32", "prior_sigma": 0.8}, -5),
                     ({"precision": "fp32", "stop_ratio": 0.01}, -5)):
        p = R.FSRParams(**kw)
        c = p.c()
        assert lib.fsr_blocks(fake, fake, 8, 8, 8, ctypes.byref(c), fake, None, fake, 1 << 20, None) == code, kw
    c = R.FSRParams().c()
    c.precision = 5
    assert lib.fsr_blocks(fake, fake, 8, 8, 8, ctypes.byref(c), fake, None, fake, 1 << 20, None) == -1
    for bound in (0.0, -1.0, float("nan"), float("inf")):
        c = R.FSRParams(precision="mixed").c()
        c.mixed_bound = bound
        assert lib.fsr_blocks(fake, fake, 8, 8, 8, ctypes.byref(c), fake, None, fake, 1 << 20, None) == -1, bound
    for kw in ({"pairs": True}, {"concealed_weight": 0.5}, {"prior_sigma": 0.8}, {"stop_ratio": 0.01}):
        c = R.FSRParams(precision="mixed", **kw).c()
        assert lib.fsr_blocks(fake, fake, 8, 8, 8, ctypes.byref(c), fake, None, fake, 1 << 20, None) == -5, kw
    # the mixed form's recomputation lists (4 bytes per block) are part of the workspace
    n32 = lib.rfsr_workspace_bytes(1080, 1920, 0, None, ctypes.byref(R.FSRParams().c()))
    assert n32 >= 16896 + 256 + 4 * 270 * 480
    c = R.FSRParams().c()
    c.overwrite = 7
    assert lib.fsr_blocks(fake, fake, 8, 8, 8, ctypes.byref(c), fake, None, fake, 1 << 20, None) == -1
    c = R.FSRParams().c()
    assert lib.fsr_blocks(None, fake, 8, 8, 8, ctypes.byref(c), fake, None, fake, 1 << 20, None) == -1
    assert lib.fsr_blocks(fake, fake, 8, 8, 8, ctypes.byref(c), fake, None, fake, 8, None) == -3


def test_fsr_blocks_noalloc_rejects_bad_arguments(R):
    """Argument validation of the entry point that allocates nothing runs
    before it touches the device (its scratch array is looked up only for a
    valid request)."""
    lib = R.lib()
    fake = ctypes.c_void_p(4096)
    for kw, code in (({"iters": -1}, -1), ({"rho": 0.0}, -1), ({"gamma": 2.0}, -1), ({"block": 8}, -5),
                     ({"precision": "fp32", "pairs": True}, -5)):
        c = R.FSRParams(**kw).c()
        assert lib.fsr_blocks_noalloc(fake, fake, 8, 8, 8, ctypes.byref(c), fake, None, None) == code, kw
    c = R.FSRParams().c()
    assert lib.fsr_blocks_noalloc(None, fake, 8, 8, 8, ctypes.byref(c), fake, None, None) == -1
    assert lib.fsr_blocks_noalloc(fake, fake, 8, 8, 8, ctypes.byref(c), None, None, None) == -1
    assert lib.fsr_blocks_noalloc(fake, fake, 8, 8, 8, None, fake, None, None) == -1
    for H, W, pitch in ((6, 8, 8), (8, 10, 10), (8, 8, 4), (20000, 8, 8)):
        assert lib.fsr_blocks_noalloc(fake, fake, H, W, pitch, ctypes.byref(c), fake, None, None) == -2
    # mixed frames whose recomputation lists (4 bytes per block + 256) do not fit
    # next to the 16,896-byte tables in the 4 MB array: RFSR_EWORKSPACE before
    # any device access
    c = R.FSRParams(precision="mixed").c()
    for H, W in ((16384, 16384), (8192, 8192), (4096, 4096), (4096, 4088)):
        assert 16896 + 256 + 4 * (H // 4) * (W // 4) > 4194304
        assert lib.fsr_blocks_noalloc(fake, fake, H, W, W, ctypes.byref(c), fake, None, None) == -3, (H, W)


def test_me_params_options_validation(R):
    """The FRMC offset set, cost_norm and nnc_center are validated before any
    device work (rfsr_workspace_bytes returns 0 for invalid parameters)."""
    lib = R.lib()

    def ws(**kw):
        p = R.MEParams(**kw).c()
        return lib.rfsr_workspace_bytes(64, 64, 1, ctypes.byref(p), None)

    assert ws() > 0
    assert ws(frmc=(-2, -1, 0, 1, 2)) > 0
    assert ws(frmc=tuple(range(-14, 1))) > 0                 # 15 offsets, reach 14
    assert ws(frmc=(0,)) > 0
    assert ws(cost_norm=False, nnc_center="raw") > 0
    for bad in ((-2, -1, 1, 2), (-1, 0, 0, 1), (1, 0, -1), (-15, 0), (0, 15), tuple(range(-15, 1))):
        assert ws(frmc=bad) == 0, bad
    p = R.MEParams().c()
    p.cost_norm = 2
    assert lib.rfsr_workspace_bytes(64, 64, 1, ctypes.byref(p), None) == 0
    p = R.MEParams().c()
    p.nnc_center = 2
    assert lib.rfsr_workspace_bytes(64, 64, 1, ctypes.byref(p), None) == 0
    p = R.MEParams().c()
    p.n_frmc = 16
    assert lib.rfsr_workspace_bytes(64, 64, 1, ctypes.byref(p), None) == 0
    # the same validation guards the calls themselves
    fake = ctypes.c_void_p(4096)
    p = R.MEParams(frmc=(-2, 2)).c()
    assert lib.rfsr_motion_check(fake, fake, fake, 8, 8, 8, ctypes.byref(p), fake, fake, None, None,
                                 fake, 1 << 20, None) == -1


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


def test_frame_split_rejects_bad_arguments(R):
    """rfsr_frame_motion / rfsr_frame_finish: `first` outside 0..nref, a null
    output, a too small workspace; first == nref leaves nothing for the
    early part, which returns OK without any device work."""
    lib = R.lib()
    P = ctypes.c_void_p
    fake = P(4096)   # never dereferenced
    me = R.MEParams().c()
    fsr = R.FSRParams().c()
    ok = (P * 3)(4096, 4096, 4096)
    big = 1 << 20
    for first, nref in ((-1, 2), (3, 2), (1, 0)):
        assert lib.rfsr_frame_motion(fake, fake, nref, ok, ok, ok, 8, 8, 8, ctypes.byref(me), first,
                                     fake, big, None) == -1, (first, nref)
        assert lib.rfsr_frame_finish(fake, fake, nref, ok, ok, ok, 8, 8, 8, ctypes.byref(me), ctypes.byref(fsr),
                                     first, fake, None, None, fake, big, None) == -1, (first, nref)
    assert lib.rfsr_frame_finish(fake, fake, 2, ok, ok, ok, 8, 8, 8, ctypes.byref(me), ctypes.byref(fsr), 1,
                                 None, None, None, fake, big, None) == -1
    assert lib.rfsr_frame_motion(fake, fake, 2, ok, ok, ok, 6, 8, 8, ctypes.byref(me), 1, fake, big, None) == -2
    assert lib.rfsr_frame_motion(fake, fake, 2, ok, ok, ok, 8, 8, 8, ctypes.byref(me), 1, fake, 16, None) == -3
    assert lib.rfsr_frame_finish(fake, fake, 2, ok, ok, ok, 8, 8, 8, ctypes.byref(me), ctypes.byref(fsr), 1,
                                 fake, None, None, fake, 16, None) == -3
    # the early part needs the second table slot: the workspace of one slot is too small
    one_slot = R.workspace_bytes(8, 8, 2) - 1024
    assert lib.rfsr_frame_motion(fake, fake, 2, ok, ok, ok, 8, 8, 8, ctypes.byref(me), 1, fake, one_slot,
                                 None) == -3
    assert lib.rfsr_frame_motion(fake, fake, 2, ok, ok, ok, 8, 8, 8, ctypes.byref(me), 2, fake, big, None) == 0


def test_binding_refuses_host_tensors(R):
    import torch
    x = torch.zeros((8, 8), dtype=torch.uint8)
    with pytest.raises(R.RfsrError):
        R.motion_check(x, x, x)
    with pytest.raises(R.RfsrError):
        R.fsr_blocks(torch.zeros((8, 8)), x)


def _descs(R, shapes, nrefs, base=1 << 20):
    """Descriptors with fake (never dereferenced) device addresses."""
    ds = (R.FrameDesc * len(shapes))()
    a = base
    for d, (H, W), nref in zip(ds, shapes, nrefs):
        d.cur, d.cur_mask, d.out = a, a + 0x1000, a + 0x2000
        for k in range(nref):
            d.ref_recon[k], d.ref_meas[k], d.ref_mask[k] = a + 0x3000 + k, a + 0x4000 + k, a + 0x5000 + k
        d.nref, d.H, d.W, d.pitch = nref, H, W, W
        a += 1 << 24
    return ds


def test_batch_sizes_and_validation(R):
    lib = R.lib()
    me, fsr = R.MEParams().c(), R.FSRParams().c()
    shapes, nrefs = [(64, 64), (96, 128), (1080, 1920)], [3, 0, 2]
    ds = _descs(R, shapes, nrefs)
    ws = lib.rfsr_batch_workspace_bytes(ds, 3, ctypes.byref(me), ctypes.byref(fsr))
    singles = sum(R.workspace_bytes(H, W, max(n, 1)) for (H, W), n in zip(shapes, nrefs))
    # per-frame scratch plus one set of FSR tables; a frame without references
    # needs no reference planes
    assert 0 < ws <= singles
    tb = lib.rfsr_batch_table_bytes(ds, 3)
    assert tb % 256 == 0 and tb > 256
    # invalid descriptors: bad shape, nref, null planes, n out of range
    for mut in (lambda d: setattr(d, "H", 6), lambda d: setattr(d, "nref", 4),
                lambda d: setattr(d, "cur", None), lambda d: setattr(d, "pitch", 8)):
        bad = _descs(R, shapes, nrefs)
        mut(bad[2])
        assert lib.rfsr_batch_workspace_bytes(bad, 3, ctypes.byref(me), ctypes.byref(fsr)) == 0
        assert lib.rfsr_batch_table_bytes(bad, 3) == 0
    assert lib.rfsr_batch_table_bytes(ds, 0) == 0
    assert lib.rfsr_batch_table_bytes(None, 1) == 0
    bad = _descs(R, shapes, nrefs)
    bad[0].ref_meas[2] = None
    assert lib.rfsr_batch_table_bytes(bad, 3) == 0


def test_batch_tables_are_keyed_to_their_descriptors(R):
    """The job-table image is built on the host: its header counts the jobs and
    carries a key that changes with any descriptor, the check or the
    workspace address."""
    lib = R.lib()
    me = R.MEParams().c()
    shapes, nrefs = [(64, 64), (96, 128)], [3, 1]
    ds = _descs(R, shapes, nrefs)
    tb = lib.rfsr_batch_table_bytes(ds, 2)
    img = ctypes.create_string_buffer(tb)

    def key(descs, mc, ws):
        assert lib.rfsr_batch_write_tables(descs, 2, ctypes.byref(mc), ctypes.c_void_p(ws), img, tb) == 0
        k, nf, nr = struct.unpack_from("<Qii", img.raw, 0)
        assert (nf, nr) == (2, 4)
        return k

    k0 = key(ds, me, 1 << 30)
    assert key(ds, me, 1 << 30) == k0
    assert key(ds, me, (1 << 30) + 256) != k0
    other = R.MEParams(check="rmc").c()
    assert key(ds, other, 1 << 30) != k0
    ds2 = _descs(R, shapes, nrefs)
    ds2[1].out = ds2[1].out + 256
    assert key(ds2, me, 1 << 30) != k0
    ds3 = _descs(R, shapes, nrefs)
    ds3[0].reserved = 7           # not part of the key
    assert key(ds3, me, 1 << 30) == k0
    # errors: image too small, misaligned workspace
    assert lib.rfsr_batch_write_tables(ds, 2, ctypes.byref(me), ctypes.c_void_p(1 << 30), img, tb - 1) == -1
    assert lib.rfsr_batch_write_tables(ds, 2, ctypes.byref(me), ctypes.c_void_p((1 << 30) + 8), img, tb) == -3


def test_batch_part_tables(R):
    """Job-table images of a batch split at reference index `first`: the
    early part holds the references >= first of every frame, the finish the
    others, each under its own key; unknown parts and first outside 0..3 are
    rejected."""
    lib = R.lib()
    me = R.MEParams().c()
    fsr = R.FSRParams().c()
    shapes, nrefs = [(64, 64), (96, 128), (32, 32)], [3, 1, 2]
    ds = _descs(R, shapes, nrefs)
    tb = lib.rfsr_batch_table_bytes(ds, 3)
    ws = ctypes.c_void_p(1 << 30)

    def header(part, first):
        img = ctypes.create_string_buffer(tb)
        assert lib.rfsr_batch_write_tables_part(ds, 3, ctypes.byref(me), part, first, ws, img, tb) == 0
        return struct.unpack_from("<Qii", img.raw, 0)

    k_all, nf, nr = header(0, 0)
    assert (nf, nr) == (3, 6)
    k_mot, _, nr_mot = header(1, 1)
    k_fin, _, nr_fin = header(2, 1)
    assert (nr_mot, nr_fin) == (2 + 0 + 1, 1 + 1 + 1)
    assert len({k_all, k_mot, k_fin}) == 3
    assert header(0, 2)[0] == k_all          # `first` is ignored for whole frames
    assert header(1, 0)[2] == 6 and header(2, 0)[2] == 0 and header(1, 3)[2] == 0
    img = ctypes.create_string_buffer(tb)
    for part, first in ((3, 1), (-1, 1), (1, -1), (2, 4)):
        assert lib.rfsr_batch_write_tables_part(ds, 3, ctypes.byref(me), part, first, ws, img, tb) == -1
        assert lib.rfsr_reconstruct_batch_part(ds, 3, ctypes.byref(me), ctypes.byref(fsr), part, first, ws, None,
                                               ws, 1 << 40, None) == -1


def test_reconstruct_batch_rejects_bad_arguments(R):
    lib = R.lib()
    P = ctypes.c_void_p
    me, fsr = R.MEParams().c(), R.FSRParams().c()
    ds = _descs(R, [(64, 64)], [2])
    need = lib.rfsr_batch_workspace_bytes(ds, 1, ctypes.byref(me), ctypes.byref(fsr))
    ws, tab = P(1 << 32), P(1 << 33)
    call = lambda d=ds, n=1, t=tab, w=ws, nb=need, ev=None, m=me, f=fsr: lib.rfsr_reconstruct_batch(
        d, n, ctypes.byref(m), ctypes.byref(f), t, ev, w, nb, None)
    assert call(t=None) == -1
    assert call(t=P((1 << 33) + 64)) == -1
    assert call(w=None) == -3
    assert call(nb=need - 1) == -3
    assert call(w=P((1 << 32) + 16)) == -3
    assert call(n=0) == -1
    assert call(ev=(P * 4)(1, 2, None, 4)) == -1
    bad_me = R.MEParams(search=16).c()
    assert call(m=bad_me) == -1
    bad_fsr = R.FSRParams(iters=-1).c()
    assert call(f=bad_fsr) == -1


def test_quality_validation(R):
    lib = R.lib()
    P = ctypes.c_void_p
    fake = P(4096)
    assert lib.rfsr_quality_workspace_bytes(100, 100, 40) > 0
    assert lib.rfsr_quality_workspace_bytes(90, 100, 40) == 0        # 10 rows left < 11
    assert lib.rfsr_quality_workspace_bytes(11, 11, 0) > 0
    assert lib.rfsr_quality_workspace_bytes(100, 100, -1) == 0
    n = lib.rfsr_quality_workspace_bytes(100, 100, 40)
    call = lambda ref=fake, H=100, W=100, pitch=100, border=40, res=fake, ws=fake, nb=n: lib.rfsr_quality(
        ref, fake, H, W, pitch, border, res, ws, nb, None)
    assert call(ref=None) == -1
    assert call(res=None) == -1
    assert call(border=-2) == -1
    assert call(H=90) == -2
    assert call(pitch=99) == -2
    assert call(ws=None) == -3
    assert call(nb=n - 1) == -3
