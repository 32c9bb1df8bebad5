"""ctypes binding of librfsr.so.

Argument marshalling only: every step of the reconstruction runs in the HIP
kernels behind the C ABI declared in include/rfsr.h.  Torch tensors provide
device memory and the current stream.  There is no fallback: if the library
is missing or a call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librfsr.so")

CHECKS = {"none": 0, "rme": 1, "rmc": 2, "frmc": 3, "nnc": 4, "nnc_frmc": 5}
OVERWRITE = {"dfsr": 0, "rfsr": 1}
PRECISION = {"fp64": 0, "bf16x3": 1, "fp16x3": 2, "fp32": 3, "mixed": 4}
MIXED_BOUND = 1.0   # RFSR_MIXED_BOUND
NCOUNTERS = 4
COUNTER_NAMES = ("forward_costs", "check_costs", "checked_pixels", "accepted")


class RfsrError(RuntimeError):
    pass


class _MEParams(ctypes.Structure):
    _fields_ = [("tmpl", ctypes.c_int32), ("search", ctypes.c_int32),
                ("check", ctypes.c_int32), ("rmc_radius", ctypes.c_int32),
                ("n_frmc", ctypes.c_int32), ("frmc", ctypes.c_int8 * 16),
                ("cost_norm", ctypes.c_int32), ("nnc_center", ctypes.c_int32)]


class _FSRParams(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("support", ctypes.c_int32),
                ("iters", ctypes.c_int32), ("overwrite", ctypes.c_int32),
                ("rho", ctypes.c_double), ("gamma", ctypes.c_double),
                ("proj_weight", ctypes.c_double), ("precision", ctypes.c_int32),
                ("pairs", ctypes.c_int32), ("concealed_weight", ctypes.c_double),
                ("prior_sigma", ctypes.c_double), ("stop_ratio", ctypes.c_double),
                ("mixed_bound", ctypes.c_double), ("block_margin", ctypes.c_void_p),
                ("rerun_blocks", ctypes.c_void_p)]


NNC_CENTER = {"filtered": 0, "raw": 1}


@dataclass
class MEParams:
    """Motion estimation and consistency check (Sec. 2.2, Sec. 3.1).
    frmc: FRMC per-axis offsets (None: the paper's {-7,-3,-1,0,1,3,7});
    cost_norm: compare reverse costs as S/n (False: raw S); nnc_center:
    "filtered" or "raw" vector at p in NNC."""
    search: int = 9
    check: str = "nnc_frmc"
    rmc_radius: int = 0
    tmpl: int = 4
    frmc: tuple | None = None
    cost_norm: bool = True
    nnc_center: str = "filtered"

    def c(self) -> _MEParams:
        offs = () if self.frmc is None else tuple(int(d) for d in self.frmc)
        if len(offs) > 16:
            raise RfsrError("frmc: at most 15 offsets")
        arr = (ctypes.c_int8 * 16)(*offs)
        return _MEParams(self.tmpl, self.search, CHECKS[self.check], self.rmc_radius, len(offs), arr,
                         int(bool(self.cost_norm)), NNC_CENTER[self.nnc_center])


@dataclass
class FSRParams:
    """Block-wise FSR (Sec. 2.1, Sec. 3.2)."""
    iters: int = 100
    rho: float = 0.7
    gamma: float = 0.5
    proj_weight: float = 1.0
    overwrite: str = "dfsr"
    block: int = 4
    support: int = 32
    precision: str = "fp64"     # "fp64"; block DFT "bf16x3" or "fp16x3" (matrix cores); "fp32" (all float32);
                                # "mixed" (float32 with a near-tie test, float64 for the blocks that fail it)
    concealed_weight: float = 0.0   # delta > 0: raster-order blocks (wavefront), single frames only
    pairs: bool = False             # real-valued FSR: conjugate pairs per iteration
    prior_sigma: float = 0.0        # frequency-weighting prior (0: off)
    stop_ratio: float = 0.0         # residual-energy early stop (0: off)
    mixed_bound: float = MIXED_BOUND    # "mixed": near-tie bound a
    block_margin: object = None     # "fp32": float32 device tensor, one margin per block (diagnostic)
    rerun_blocks: object = None     # "mixed": int64 device tensor (1 element) the call adds its recomputed blocks to

    def c(self) -> _FSRParams:
        for t, dt, nm in ((self.block_margin, torch.float32, "block_margin"),
                          (self.rerun_blocks, torch.int64, "rerun_blocks")):
            if t is not None and (not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dt
                                  or not t.is_contiguous()):
                raise RfsrError(f"{nm}: expected a contiguous {dt} device tensor")
        return _FSRParams(self.block, self.support, self.iters, OVERWRITE[self.overwrite],
                          self.rho, self.gamma, self.proj_weight, PRECISION[self.precision],
                          int(self.pairs), self.concealed_weight, self.prior_sigma, self.stop_ratio,
                          self.mixed_bound,
                          None if self.block_margin is None else self.block_margin.data_ptr(),
                          None if self.rerun_blocks is None else self.rerun_blocks.data_ptr())


class FrameDesc(ctypes.Structure):
    """rfsr_frame_desc: one frame of a batch (device pointers)."""
    _fields_ = [("cur", ctypes.c_void_p), ("cur_mask", ctypes.c_void_p),
                ("ref_recon", ctypes.c_void_p * 3), ("ref_meas", ctypes.c_void_p * 3),
                ("ref_mask", ctypes.c_void_p * 3), ("out", ctypes.c_void_p), ("out_u8", ctypes.c_void_p),
                ("nref", ctypes.c_int32), ("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("pitch", ctypes.c_int64)]


_lib = None

_P = ctypes.c_void_p
_STATUS = ctypes.c_int32


def lib():
    """Load librfsr.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RfsrError(f"{LIB_PATH} not built; run `python -m paper_2203_09200_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    L.rfsr_workspace_bytes.restype = ctypes.c_size_t
    L.rfsr_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.POINTER(_MEParams), ctypes.POINTER(_FSRParams)]
    L.rfsr_motion_check.restype = _STATUS
    L.rfsr_motion_check.argtypes = [_P, _P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                    ctypes.POINTER(_MEParams), _P, _P, _P, _P, _P, ctypes.c_size_t, _P]
    L.fsr_blocks_noalloc.restype = _STATUS
    L.fsr_blocks_noalloc.argtypes = [_P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                     ctypes.POINTER(_FSRParams), _P, _P, _P]
    L.fsr_blocks.restype = _STATUS
    L.fsr_blocks.argtypes = [_P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                             ctypes.POINTER(_FSRParams), _P, _P, _P, ctypes.c_size_t, _P]
    L.rfsr_reconstruct_frame.restype = _STATUS
    L.rfsr_reconstruct_frame.argtypes = [_P, _P, ctypes.c_int32, ctypes.POINTER(_P), ctypes.POINTER(_P),
                                         ctypes.POINTER(_P), ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int64, ctypes.POINTER(_MEParams),
                                         ctypes.POINTER(_FSRParams), _P, _P, ctypes.POINTER(_P),
                                         _P, ctypes.c_size_t, _P]
    L.rfsr_frame_motion.restype = _STATUS
    L.rfsr_frame_motion.argtypes = [_P, _P, ctypes.c_int32, ctypes.POINTER(_P), ctypes.POINTER(_P),
                                    ctypes.POINTER(_P), ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                    ctypes.POINTER(_MEParams), ctypes.c_int32, _P, ctypes.c_size_t, _P]
    L.rfsr_frame_finish.restype = _STATUS
    L.rfsr_frame_finish.argtypes = [_P, _P, ctypes.c_int32, ctypes.POINTER(_P), ctypes.POINTER(_P),
                                    ctypes.POINTER(_P), ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                    ctypes.POINTER(_MEParams), ctypes.POINTER(_FSRParams), ctypes.c_int32,
                                    _P, _P, ctypes.POINTER(_P), _P, ctypes.c_size_t, _P]
    L.rfsr_batch_workspace_bytes.restype = ctypes.c_size_t
    L.rfsr_batch_workspace_bytes.argtypes = [ctypes.POINTER(FrameDesc), ctypes.c_int32,
                                             ctypes.POINTER(_MEParams), ctypes.POINTER(_FSRParams)]
    L.rfsr_batch_table_bytes.restype = ctypes.c_size_t
    L.rfsr_batch_table_bytes.argtypes = [ctypes.POINTER(FrameDesc), ctypes.c_int32]
    L.rfsr_batch_write_tables.restype = _STATUS
    L.rfsr_batch_write_tables.argtypes = [ctypes.POINTER(FrameDesc), ctypes.c_int32,
                                          ctypes.POINTER(_MEParams), _P, _P, ctypes.c_size_t]
    L.rfsr_batch_write_tables_part.restype = _STATUS
    L.rfsr_batch_write_tables_part.argtypes = [ctypes.POINTER(FrameDesc), ctypes.c_int32,
                                               ctypes.POINTER(_MEParams), ctypes.c_int32, ctypes.c_int32, _P,
                                               _P, ctypes.c_size_t]
    L.rfsr_reconstruct_batch_part.restype = _STATUS
    L.rfsr_reconstruct_batch_part.argtypes = [ctypes.POINTER(FrameDesc), ctypes.c_int32,
                                              ctypes.POINTER(_MEParams), ctypes.POINTER(_FSRParams),
                                              ctypes.c_int32, ctypes.c_int32, _P, ctypes.POINTER(_P), _P,
                                              ctypes.c_size_t, _P]
    L.rfsr_reconstruct_batch.restype = _STATUS
    L.rfsr_reconstruct_batch.argtypes = [ctypes.POINTER(FrameDesc), ctypes.c_int32,
                                         ctypes.POINTER(_MEParams), ctypes.POINTER(_FSRParams), _P,
                                         ctypes.POINTER(_P), _P, ctypes.c_size_t, _P]
    L.rfsr_quality_workspace_bytes.restype = ctypes.c_size_t
    L.rfsr_quality_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    L.rfsr_quality.restype = _STATUS
    L.rfsr_quality.argtypes = [_P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, _P, _P,
                               ctypes.c_size_t, _P]
    L.rfsr_event_create.restype = _STATUS
    L.rfsr_event_create.argtypes = [ctypes.POINTER(_P)]
    L.rfsr_event_destroy.restype = _STATUS
    L.rfsr_event_destroy.argtypes = [_P]
    L.rfsr_event_record.restype = _STATUS
    L.rfsr_event_record.argtypes = [_P, _P]
    L.rfsr_event_wait.restype = _STATUS
    L.rfsr_event_wait.argtypes = [_P, _P]
    L.rfsr_event_elapsed_ms.restype = _STATUS
    L.rfsr_event_elapsed_ms.argtypes = [_P, _P, ctypes.POINTER(ctypes.c_float)]
    L.rfsr_status_string.restype = ctypes.c_char_p
    L.rfsr_status_string.argtypes = [ctypes.c_int32]
    L.rfsr_version.restype = ctypes.c_int32
    L.rfsr_version.argtypes = []
    _lib = L
    return L


def _check(status: int, what: str):
    if status != 0:
        msg = lib().rfsr_status_string(status).decode()
        raise RfsrError(f"{what} failed: {msg} ({status})")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _plane(t, dtype, name, shape=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise RfsrError(f"{name}: expected a device tensor")
    if t.dtype != dtype:
        raise RfsrError(f"{name}: expected {dtype}, got {t.dtype}")
    if t.dim() != 2 or t.stride(1) != 1:
        raise RfsrError(f"{name}: expected a 2-D row-major plane")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise RfsrError(f"{name}: expected shape {shape}, got {tuple(t.shape)}")
    return t


def workspace_bytes(H, W, nref=3, me: MEParams | None = None, fsr: FSRParams | None = None) -> int:
    mc = me.c() if me else None
    fc = fsr.c() if fsr else None
    n = lib().rfsr_workspace_bytes(H, W, nref, ctypes.byref(mc) if mc else None,
                                   ctypes.byref(fc) if fc else None)
    if n == 0:
        raise RfsrError("invalid arguments for rfsr_workspace_bytes")
    return int(n)


class Workspace:
    """Device scratch buffer reused across calls (grown on demand)."""

    def __init__(self, device=None):
        self.device = device or torch.device("cuda")
        self.buf = None

    def get(self, nbytes: int) -> torch.Tensor:
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
            if self.buf.data_ptr() % 256:
                raise RfsrError("workspace allocation is not 256-byte aligned")
        return self.buf


_default_ws = {}


def _ws(workspace, device, nbytes):
    if workspace is None:
        key = str(device)
        workspace = _default_ws.setdefault(key, Workspace(device))
    return workspace.get(nbytes)


def motion_check(cur, cur_mask, ref_recon, me: MEParams | None = None, counters=None,
                 want_cost=True, workspace: Workspace | None = None, stream=None):
    """Forward ME of `cur` against `ref_recon` plus the consistency check.

    Returns (mv int8 (2,H,W), accept uint8 (H,W), cost int16 (H,W) or None).
    `counters`: optional int64 device tensor of 4 entries, added to.
    """
    me = me or MEParams()
    _plane(cur, torch.uint8, "cur")
    H, W = cur.shape
    _plane(cur_mask, torch.uint8, "cur_mask", (H, W))
    _plane(ref_recon, torch.uint8, "ref_recon", (H, W))
    if not (cur.stride(0) == cur_mask.stride(0) == ref_recon.stride(0) == W):
        raise RfsrError("motion_check: inputs must be contiguous")
    dev = cur.device
    mv = torch.empty((2, H, W), dtype=torch.int8, device=dev)
    acc = torch.empty((H, W), dtype=torch.uint8, device=dev)
    cost = torch.empty((H, W), dtype=torch.int16, device=dev) if want_cost else None
    if counters is not None and (counters.dtype != torch.int64 or counters.numel() < NCOUNTERS
                                 or not counters.is_cuda):
        raise RfsrError("counters: expected int64 device tensor with 4 entries")
    mc = me.c()
    nbytes = workspace_bytes(H, W, 0, me, None)
    ws = _ws(workspace, dev, nbytes)
    st = lib().rfsr_motion_check(_ptr(cur), _ptr(cur_mask), _ptr(ref_recon), H, W, W,
                                 ctypes.byref(mc), _ptr(mv), _ptr(acc), _ptr(cost), _ptr(counters),
                                 _ptr(ws), ws.numel(), _stream(stream))
    _check(st, "rfsr_motion_check")
    return mv, acc, cost


def fsr_blocks(values, cls, fsr: FSRParams | None = None, want_u8=True,
               workspace: Workspace | None = None, stream=None):
    """Block-parallel FSR.  Returns (out float32 (H,W), out_u8 uint8 or None)."""
    fsr = fsr or FSRParams()
    _plane(values, torch.float32, "values")
    H, W = values.shape
    _plane(cls, torch.uint8, "cls", (H, W))
    if values.stride(0) != cls.stride(0):
        raise RfsrError("fsr_blocks: values and cls must share the row pitch")
    pitch = values.stride(0)
    out = torch.empty_strided((H, W), (pitch, 1), dtype=torch.float32, device=values.device)
    out_u8 = torch.empty_strided((H, W), (pitch, 1), dtype=torch.uint8, device=values.device) if want_u8 else None
    fc = fsr.c()
    ws = _ws(workspace, values.device, workspace_bytes(H, W, 0, None, fsr))
    st = lib().fsr_blocks(_ptr(values), _ptr(cls), H, W, pitch, ctypes.byref(fc), _ptr(out),
                          _ptr(out_u8), _ptr(ws), ws.numel(), _stream(stream))
    _check(st, "fsr_blocks")
    return out, out_u8


def fsr_blocks_noalloc(values, cls, fsr: FSRParams | None = None, out=None, out_u8=None, stream=None):
    """fsr_blocks through the entry point that allocates nothing: its scratch
    is the library's own device array.  `out` (float32) and `out_u8` (uint8,
    optional) may be given with the pitch of `values`; missing `out` is
    allocated here by torch, before the call.  Returns (out, out_u8)."""
    fsr = fsr or FSRParams()
    _plane(values, torch.float32, "values")
    H, W = values.shape
    _plane(cls, torch.uint8, "cls", (H, W))
    pitch = values.stride(0)
    if cls.stride(0) != pitch:
        raise RfsrError("fsr_blocks_noalloc: values and cls must share the row pitch")
    if out is None:
        out = torch.empty_strided((H, W), (pitch, 1), dtype=torch.float32, device=values.device)
    for t, dt, nm in ((out, torch.float32, "out"), (out_u8, torch.uint8, "out_u8")):
        if t is not None:
            _plane(t, dt, nm, (H, W))
            if t.stride(0) != pitch:
                raise RfsrError(f"fsr_blocks_noalloc: {nm} must have the pitch of values")
    fc = fsr.c()
    st = lib().fsr_blocks_noalloc(_ptr(values), _ptr(cls), H, W, pitch, ctypes.byref(fc), _ptr(out),
                                  _ptr(out_u8), _stream(stream))
    _check(st, "fsr_blocks_noalloc")
    return out, out_u8


def _frame_args(cur, cur_mask, refs, name):
    """Validated planes of one frame: (H, W, pitch, nref, rr, rm, rk, planes)."""
    _plane(cur, torch.uint8, "cur")
    H, W = cur.shape
    _plane(cur_mask, torch.uint8, "cur_mask", (H, W))
    pitch = cur.stride(0)
    planes = [cur, cur_mask]
    nref = len(refs)
    if nref > 3:
        raise RfsrError("at most 3 references")
    for k, (r, m, b) in enumerate(refs):
        for t, nm in ((r, "recon"), (m, "meas"), (b, "mask")):
            _plane(t, torch.uint8, f"ref{k}.{nm}", (H, W))
            planes.append(t)
    arr = ctypes.c_void_p * 3
    rr = arr(*[r[0].data_ptr() for r in refs])
    rm = arr(*[r[1].data_ptr() for r in refs])
    rk = arr(*[r[2].data_ptr() for r in refs])
    return H, W, pitch, nref, rr, rm, rk, planes


def reconstruct_frame(cur, cur_mask, refs=(), me: MEParams | None = None,
                      fsr: FSRParams | None = None, out=None, out_u8=None, stage_events=None,
                      workspace: Workspace | None = None, stream=None, first=None):
    """One recursive frame (Fig. 1 order).  refs: sequence of
    (recon uint8, meas uint8, mask uint8) device planes for lags 1..len(refs).
    Returns (out float32 (H,W), out_u8 uint8 (H,W)).

    first: None for the whole frame (rfsr_reconstruct_frame); otherwise the
    frame's second part (rfsr_frame_finish): references of index < first,
    projection and FSR, after `frame_motion(..., first)` ran the others into
    the same workspace."""
    me = me or MEParams()
    fsr = fsr or FSRParams()
    H, W, pitch, nref, rr, rm, rk, planes = _frame_args(cur, cur_mask, refs, "reconstruct_frame")
    dev = cur.device
    if out is None:
        out = torch.empty_strided((H, W), (pitch, 1), dtype=torch.float32, device=dev)
    if out_u8 is None:
        out_u8 = torch.empty_strided((H, W), (pitch, 1), dtype=torch.uint8, device=dev)
    planes += [_plane(out, torch.float32, "out", (H, W)), _plane(out_u8, torch.uint8, "out_u8", (H, W))]
    if any(p.stride(0) != pitch for p in planes):
        raise RfsrError("reconstruct_frame: all planes must share the row pitch")
    ev = None
    if stage_events is not None:
        ev = (ctypes.c_void_p * 4)(*[e.handle for e in stage_events])
    mc, fc = me.c(), fsr.c()
    ws = _ws(workspace, dev, workspace_bytes(H, W, nref, me, fsr))
    if first is None:
        st = lib().rfsr_reconstruct_frame(_ptr(cur), _ptr(cur_mask), nref, rr, rm, rk, H, W, pitch,
                                          ctypes.byref(mc), ctypes.byref(fc), _ptr(out), _ptr(out_u8), ev,
                                          _ptr(ws), ws.numel(), _stream(stream))
        _check(st, "rfsr_reconstruct_frame")
    else:
        st = lib().rfsr_frame_finish(_ptr(cur), _ptr(cur_mask), nref, rr, rm, rk, H, W, pitch,
                                     ctypes.byref(mc), ctypes.byref(fc), int(first), _ptr(out), _ptr(out_u8),
                                     ev, _ptr(ws), ws.numel(), _stream(stream))
        _check(st, "rfsr_frame_finish")
    return out, out_u8


def frame_motion(cur, cur_mask, refs=(), me: MEParams | None = None, first: int = 1,
                 workspace: Workspace | None = None, stream=None):
    """First part of a frame split for pipelining (rfsr_frame_motion): the
    window plane and the forward ME + check of the references of index
    >= first (lags first+1..len(refs)) into `workspace`; complete the frame
    with reconstruct_frame(..., first=first) on the same workspace."""
    me = me or MEParams()
    H, W, pitch, nref, rr, rm, rk, planes = _frame_args(cur, cur_mask, refs, "frame_motion")
    if any(p.stride(0) != pitch for p in planes):
        raise RfsrError("frame_motion: all planes must share the row pitch")
    mc = me.c()
    ws = _ws(workspace, cur.device, workspace_bytes(H, W, nref, me, None))
    st = lib().rfsr_frame_motion(_ptr(cur), _ptr(cur_mask), nref, rr, rm, rk, H, W, pitch, ctypes.byref(mc),
                                 int(first), _ptr(ws), ws.numel(), _stream(stream))
    _check(st, "rfsr_frame_motion")


def quality_async(ref, test, border: int = 40, result=None, workspace: Workspace | None = None, stream=None):
    """PSNR and mean SSIM (Sec. 4) of `test` (float32 device plane) against
    `ref` (uint8 device plane), computed on the device.  Returns a float64
    device tensor (psnr, ssim); nothing is synchronised."""
    _plane(ref, torch.uint8, "ref")
    H, W = ref.shape
    _plane(test, torch.float32, "test", (H, W))
    if ref.stride(0) != test.stride(0):
        raise RfsrError("quality: ref and test must share the row pitch")
    n = lib().rfsr_quality_workspace_bytes(H, W, border)
    if n == 0:
        raise RfsrError(f"quality: {H}x{W} with border {border} leaves less than one 11x11 window")
    ws = _ws(workspace, ref.device, n)
    if result is None:
        result = torch.empty(2, dtype=torch.float64, device=ref.device)
    st = lib().rfsr_quality(_ptr(ref), _ptr(test), H, W, ref.stride(0), border, _ptr(result), _ptr(ws),
                            ws.numel(), _stream(stream))
    _check(st, "rfsr_quality")
    return result


def quality(ref, test, border: int = 40, workspace: Workspace | None = None, stream=None):
    """(psnr, mean ssim) as Python floats (waits for the device)."""
    r = quality_async(ref, test, border, workspace=workspace, stream=stream).cpu()
    return float(r[0]), float(r[1])


class Event:
    """HIP event created by the library (for stage timing)."""

    def __init__(self):
        h = ctypes.c_void_p()
        _check(lib().rfsr_event_create(ctypes.byref(h)), "rfsr_event_create")
        self.handle = h.value

    def record(self, stream=None):
        _check(lib().rfsr_event_record(ctypes.c_void_p(self.handle), _stream(stream)), "rfsr_event_record")

    def wait(self, stream=None):
        """Make work enqueued on `stream` after this call wait for the
        event's last record."""
        _check(lib().rfsr_event_wait(ctypes.c_void_p(self.handle), _stream(stream)), "rfsr_event_wait")

    def elapsed_ms(self, end: "Event") -> float:
        ms = ctypes.c_float()
        _check(lib().rfsr_event_elapsed_ms(ctypes.c_void_p(self.handle), ctypes.c_void_p(end.handle),
                                           ctypes.byref(ms)), "rfsr_event_elapsed_ms")
        return float(ms.value)

    def __del__(self):
        try:
            if self.handle and _lib is not None:
                _lib.rfsr_event_destroy(ctypes.c_void_p(self.handle))
        except Exception:
            pass


class Sequence:
    """Causal recursion over a stream of frames: keeps the last three
    (reconstruction, measured frame, mask) planes resident on the device and
    reconstructs each new frame against them (Sec. 2.2, three previous
    frames as in Sec. 4).

    pipelined=True overlaps consecutive frames (same results): frame t's
    references of lag >= 2 are final once frame t-2 is, so their motion
    path (rfsr_frame_motion) runs on a side stream while frame t-1's FSR
    runs (it starts once frame t-1's projection is done, so that it does
    not compete with frame t-1's own motion path), and only the lag-1
    reference, the projection and FSR (rfsr_frame_finish) wait for frame
    t-1.  Two workspaces alternate between frames.  The inputs of push()
    must be complete on the device when push() is called (pass `ready`, a
    torch event, if they are still being produced).

    The ring holds the pushed tensors themselves (no copies): the measured
    frame, the mask and the uint8 reconstruction of the last `nref` frames
    are the next frames' references.  Their contents must not change while
    they are (passing one unchanged tensor for every frame, e.g. a fixed
    mask, is fine), and an out_u8 that is one of them raises RfsrError: the
    call would overwrite a reference it reads (pass a fresh tensor, or
    out_u8=None to allocate)."""

    def __init__(self, H, W, me: MEParams | None = None, fsr: FSRParams | None = None,
                 nref=3, device=None, pipelined=False):
        self.H, self.W = H, W
        self.me = me or MEParams()
        self.fsr = fsr or FSRParams()
        self.nref = nref
        self.device = device or torch.device("cuda")
        self.ring = []
        self.workspace = Workspace(self.device)
        self.pipelined = pipelined
        if pipelined:
            nbytes = workspace_bytes(H, W, nref, self.me, self.fsr)
            self._ws = [Workspace(self.device), Workspace(self.device)]
            for w in self._ws:
                w.get(nbytes)
            self._side = torch.cuda.Stream(device=self.device)   # default priority
            self._done = [None, None]
            self._stage = [[Event() for _ in range(4)] for _ in range(2)]
            self._fsr_start = None   # stage event [2] of the last frame: its FSR is next
            self._n = 0

    def reset(self):
        """Start a new recursion (the next frame has no references)."""
        self.ring = []
        if self.pipelined:
            self._fsr_start = None

    def push(self, meas, mask, stage_events=None, stream=None, out=None, out_u8=None, ready=None):
        if out_u8 is not None and any(out_u8.data_ptr() == t.data_ptr() for r in self.ring for t in r):
            raise RfsrError("Sequence.push: out_u8 is a plane the ring still holds as a reference; "
                            "pass a fresh tensor or out_u8=None")
        refs = [(r[0], r[1], r[2]) for r in reversed(self.ring[-self.nref:])] if self.nref else []
        if not self.pipelined:
            out, out_u8 = reconstruct_frame(meas, mask, refs, self.me, self.fsr, out=out, out_u8=out_u8,
                                            stage_events=stage_events, workspace=self.workspace, stream=stream)
        else:
            main = stream or torch.cuda.current_stream(self.device)
            k = self._n % 2
            ws = self._ws[k]
            stage = stage_events if stage_events is not None else self._stage[k]
            first = min(1, len(refs))
            if len(refs) > first:
                side = self._side
                if self._done[k] is not None:   # frame t-2: its workspace and the lag >= 2 references
                    side.wait_event(self._done[k])
                if self._fsr_start is not None:   # frame t-1 has reached its FSR
                    self._fsr_start.wait(side)
                if ready is not None:
                    side.wait_event(ready)
                for t in [meas, mask] + [p for r in refs[first:] for p in r]:
                    t.record_stream(side)
                frame_motion(meas, mask, refs, self.me, first, workspace=ws, stream=side)
                ev = torch.cuda.Event()
                ev.record(side)
                main.wait_event(ev)
            elif ready is not None:
                main.wait_event(ready)
            out, out_u8 = reconstruct_frame(meas, mask, refs, self.me, self.fsr, out=out, out_u8=out_u8,
                                            stage_events=stage, workspace=ws, stream=main, first=first)
            done = torch.cuda.Event()
            done.record(main)
            self._done[k] = done
            self._fsr_start = stage[2]
            self._n += 1
        self.ring.append((out_u8, meas, mask))
        if len(self.ring) > self.nref:
            self.ring.pop(0)
        return out, out_u8


# ----------------------------------------------------------------- batches --
@dataclass
class BatchFrame:
    """One frame of a batch: measured frame and mask, up to three references
    (recon, meas, mask) for lags 1..3, and the output planes.  All planes of a
    frame are uint8 (out: float32) device tensors sharing one row pitch."""
    cur: torch.Tensor
    mask: torch.Tensor
    refs: tuple = ()
    out: torch.Tensor | None = None
    out_u8: torch.Tensor | None = None


def _frame_desc(f: BatchFrame, i: int) -> FrameDesc:
    _plane(f.cur, torch.uint8, f"frames[{i}].cur")
    H, W = f.cur.shape
    pitch = f.cur.stride(0)
    planes = [f.cur, _plane(f.mask, torch.uint8, f"frames[{i}].mask", (H, W))]
    if len(f.refs) > 3:
        raise RfsrError(f"frames[{i}]: at most 3 references")
    d = FrameDesc()
    d.cur, d.cur_mask = f.cur.data_ptr(), f.mask.data_ptr()
    for k, (r, m, b) in enumerate(f.refs):
        for t, nm in ((r, "recon"), (m, "meas"), (b, "mask")):
            planes.append(_plane(t, torch.uint8, f"frames[{i}].ref{k}.{nm}", (H, W)))
        d.ref_recon[k], d.ref_meas[k], d.ref_mask[k] = r.data_ptr(), m.data_ptr(), b.data_ptr()
    if f.out is None:
        f.out = torch.empty_strided((H, W), (pitch, 1), dtype=torch.float32, device=f.cur.device)
    planes.append(_plane(f.out, torch.float32, f"frames[{i}].out", (H, W)))
    d.out = f.out.data_ptr()
    if f.out_u8 is not None:
        planes.append(_plane(f.out_u8, torch.uint8, f"frames[{i}].out_u8", (H, W)))
        d.out_u8 = f.out_u8.data_ptr()
    if any(p.stride(0) != pitch for p in planes):
        raise RfsrError(f"frames[{i}]: all planes must share the row pitch")
    if any(p.device != f.cur.device for p in planes):
        raise RfsrError(f"frames[{i}]: planes on different devices")
    d.nref, d.H, d.W, d.pitch = len(f.refs), H, W, pitch
    return d


class Batch:
    """A fixed set of frames reconstructed together by rfsr_reconstruct_batch
    (one launch chain for all frames).  The job tables are written once at
    construction; `run()` enqueues the chain, `capture()` records it in a
    CUDA/HIP graph whose replays recompute the same frames from whatever the
    input planes hold at replay time.

    workspace: optional uint8 device tensor (256-byte aligned, at least
    `Batch.workspace_bytes(frames)`), which batches that never run at the
    same time may share.
    stream: if given, the job tables are uploaded asynchronously on it (from
    pinned memory) and the host does not wait; run the batch on the same
    stream.  Otherwise the upload completes before the constructor returns.
    part / first: "all" (whole frames), or one part of the frames split at
    reference index `first` for pipelining ("motion": the motion path of
    references first.., "finish": the rest; rfsr_reconstruct_batch_part).
    """

    PARTS = {"all": 0, "motion": 1, "finish": 2}

    def __init__(self, frames, me: MEParams | None = None, fsr: FSRParams | None = None,
                 workspace: torch.Tensor | None = None, stream=None, part: str = "all", first: int = 0):
        if not frames:
            raise RfsrError("Batch: no frames")
        if part not in self.PARTS:
            raise RfsrError(f"Batch: part must be one of {sorted(self.PARTS)}")
        self.part, self.first = self.PARTS[part], int(first)
        self.frames = list(frames)
        self.me = me or MEParams()
        self.fsr = fsr or FSRParams()
        self.n = len(self.frames)
        self.device = self.frames[0].cur.device
        self.descs = (FrameDesc * self.n)(*[_frame_desc(f, i) for i, f in enumerate(self.frames)])
        self._mc, self._fc = self.me.c(), self.fsr.c()
        L = lib()
        need = L.rfsr_batch_workspace_bytes(self.descs, self.n, ctypes.byref(self._mc), ctypes.byref(self._fc))
        if need == 0:
            raise RfsrError("Batch: invalid frame descriptors")
        if workspace is None:
            workspace = torch.empty(int(need), dtype=torch.uint8, device=self.device)
        if workspace.numel() < need or workspace.data_ptr() % 256 or workspace.device != self.device:
            raise RfsrError(f"Batch: workspace needs {need} bytes on {self.device}, 256-byte aligned")
        self.workspace = workspace
        tb = int(L.rfsr_batch_table_bytes(self.descs, self.n))
        image = torch.empty(tb, dtype=torch.uint8, pin_memory=True)
        _check(L.rfsr_batch_write_tables_part(self.descs, self.n, ctypes.byref(self._mc), self.part, self.first,
                                              _ptr(workspace), _ptr(image), tb), "rfsr_batch_write_tables_part")
        if stream is None:
            self.tables = torch.empty(tb, dtype=torch.uint8, device=self.device)
            self.tables.copy_(image)
            torch.cuda.current_stream(self.device).synchronize()
        else:
            with torch.cuda.stream(stream):
                self.tables = torch.empty(tb, dtype=torch.uint8, device=self.device)
                self.tables.copy_(image, non_blocking=True)
            self._image = image     # keep the pinned source alive with the batch
        if self.tables.data_ptr() % 256:
            raise RfsrError("Batch: job-table allocation is not 256-byte aligned")

    @staticmethod
    def workspace_bytes(frames, me: MEParams | None = None, fsr: FSRParams | None = None) -> int:
        descs = (FrameDesc * len(frames))(*[_frame_desc(f, i) for i, f in enumerate(frames)])
        mc, fc = (me or MEParams()).c(), (fsr or FSRParams()).c()
        n = lib().rfsr_batch_workspace_bytes(descs, len(frames), ctypes.byref(mc), ctypes.byref(fc))
        if n == 0:
            raise RfsrError("invalid frame descriptors")
        return int(n)

    def run(self, stage_events=None, stream=None):
        ev = None
        if stage_events is not None:
            ev = (ctypes.c_void_p * 4)(*[e.handle for e in stage_events])
        st = lib().rfsr_reconstruct_batch_part(self.descs, self.n, ctypes.byref(self._mc), ctypes.byref(self._fc),
                                               self.part, self.first, _ptr(self.tables), ev, _ptr(self.workspace),
                                               self.workspace.numel(), _stream(stream))
        _check(st, "rfsr_reconstruct_batch_part")
        return [(f.out, f.out_u8) for f in self.frames]

    def capture(self):
        """Record the chain in a graph (torch.cuda.CUDAGraph); replay() reruns it."""
        g = torch.cuda.CUDAGraph()
        torch.cuda.synchronize(self.device)
        with torch.cuda.graph(g):
            self.run()
        torch.cuda.synchronize(self.device)
        return g


class StreamSet:
    """Many independent quarter-sampled streams, each its own causal
    recursion with up to three references (Sec. 2.2), advanced one time step
    at a time as ONE batch.  Frame sizes may differ between streams.

    Each stream keeps a ring of four slots (measured frame, mask, outputs);
    time step t writes slot t mod 4 and references slots t-1..t-3.  The
    buffer pattern repeats every four steps, so from t = 3 on the chain of
    each phase is captured once in a graph and replayed (graphs=True).

    pipelined=True overlaps consecutive time steps as Sequence does (same
    results; eager launches, no graphs): the motion path of every stream's
    lag-2/3 references runs on a side stream beside the previous step's
    FSR, with two workspaces alternating between steps.  The inputs of
    step() must be complete on the device when step() is called.
    """

    SLOTS = 4

    def __init__(self, sizes, me: MEParams | None = None, fsr: FSRParams | None = None,
                 nref: int = 3, graphs: bool = True, device=None, pipelined: bool = False):
        if not 0 <= nref <= 3:
            raise RfsrError("nref must be in 0..3")
        self.sizes = [tuple(map(int, s)) for s in sizes]
        self.me = me or MEParams()
        self.fsr = fsr or FSRParams()
        self.nref = nref
        self.pipelined = pipelined
        self.graphs = graphs and not pipelined
        self.device = device or torch.device("cuda")
        dev = self.device
        mk = lambda H, W, dt: [torch.empty((H, W), dtype=dt, device=dev) for _ in range(self.SLOTS)]
        self.meas = [mk(H, W, torch.uint8) for H, W in self.sizes]
        self.mask = [mk(H, W, torch.uint8) for H, W in self.sizes]
        self.out = [mk(H, W, torch.float32) for H, W in self.sizes]
        self.out_u8 = [mk(H, W, torch.uint8) for H, W in self.sizes]
        self.t = 0
        self._batches = {}
        self._graphs = {}
        # one workspace for every phase (phases never overlap); pipelined:
        # two, alternating between time steps (slot parity)
        need = max(Batch.workspace_bytes(self._frames(slot, self.nref), self.me, self.fsr)
                   for slot in range(self.SLOTS))
        self.workspace = torch.empty(need, dtype=torch.uint8, device=dev)
        if pipelined:
            self._wss = [self.workspace, torch.empty(need, dtype=torch.uint8, device=dev)]
            self._side = torch.cuda.Stream(device=dev)   # default priority
            self._done = [None, None]
            self._stage = [[Event() for _ in range(4)] for _ in range(2)]
            self._fsr_start = None

    def _frames(self, slot, nref):
        fr = []
        for s in range(len(self.sizes)):
            refs = tuple((self.out_u8[s][(slot - k) % self.SLOTS], self.meas[s][(slot - k) % self.SLOTS],
                          self.mask[s][(slot - k) % self.SLOTS]) for k in range(1, nref + 1))
            fr.append(BatchFrame(self.meas[s][slot], self.mask[s][slot], refs, self.out[s][slot],
                                 self.out_u8[s][slot]))
        return fr

    def step(self, meas, masks, stage_events=None):
        """Reconstruct one frame of every stream.  meas/masks: sequences of
        uint8 (H, W) device tensors, one per stream.  Returns the list of
        (out float32, out_u8 uint8) planes (valid until the same slot is
        written again, four steps later)."""
        if len(meas) != len(self.sizes) or len(masks) != len(self.sizes):
            raise RfsrError("StreamSet.step: one frame and mask per stream")
        slot = self.t % self.SLOTS
        nref = min(self.t, self.nref)
        if self.pipelined:
            return self._step_pipelined(meas, masks, slot, nref, stage_events)
        for s in range(len(self.sizes)):
            self.meas[s][slot].copy_(meas[s], non_blocking=True)
            self.mask[s][slot].copy_(masks[s], non_blocking=True)
        key = (slot, nref)
        b = self._batches.get(key)
        if b is None:
            b = self._batches[key] = Batch(self._frames(slot, nref), self.me, self.fsr, self.workspace)
        if self.graphs and nref == self.nref and stage_events is None:
            g = self._graphs.get(key)
            if g is None:
                g = self._graphs[key] = b.capture()
            g.replay()
        else:
            b.run(stage_events=stage_events)
        self.t += 1
        return [(self.out[s][slot], self.out_u8[s][slot]) for s in range(len(self.sizes))]

    def _batch(self, slot, nref, part, first):
        key = (slot, nref, part)
        b = self._batches.get(key)
        if b is None:
            b = self._batches[key] = Batch(self._frames(slot, nref), self.me, self.fsr, self._wss[slot % 2],
                                           part=part, first=first)
        return b

    def _step_pipelined(self, meas, masks, slot, nref, stage_events):
        main = torch.cuda.current_stream(self.device)
        k = slot % 2
        stage = stage_events if stage_events is not None else self._stage[k]
        first = min(1, nref)

        def copy_inputs():
            for s in range(len(self.sizes)):
                self.meas[s][slot].copy_(meas[s], non_blocking=True)
                self.mask[s][slot].copy_(masks[s], non_blocking=True)

        if nref > first:
            side = self._side
            if self._done[k] is not None:   # step t-2: its workspace, the lag >= 2 references, slot t-4
                side.wait_event(self._done[k])
            if self._fsr_start is not None:   # step t-1 has reached its FSR
                self._fsr_start.wait(side)
            for t in list(meas) + list(masks):
                t.record_stream(side)
            with torch.cuda.stream(side):
                copy_inputs()
            self._batch(slot, nref, "motion", first).run(stream=side)
            ev = torch.cuda.Event()
            ev.record(side)
            main.wait_event(ev)
            fin = self._batch(slot, nref, "finish", first)
        else:
            if self._done[k] is not None:
                main.wait_event(self._done[k])
            copy_inputs()
            fin = self._batch(slot, nref, "all", 0)
        fin.run(stage_events=stage, stream=main)
        done = torch.cuda.Event()
        done.record(main)
        self._done[k] = done
        self._fsr_start = stage[2]
        self.t += 1
        return [(self.out[s][slot], self.out_u8[s][slot]) for s in range(len(self.sizes))]
