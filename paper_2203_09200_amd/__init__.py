"""MI355X (gfx950) implementation of recursive frequency selective
reconstruction of quarter-sampled video with fast motion consistency checks
(Grosche, Seiler, Kaup, ICIP 2021).

The computation lives in librfsr.so (HIP kernels behind the C ABI of
include/rfsr.h); this package is its Python binding.
"""
from ._lib import (CHECKS, COUNTER_NAMES, MIXED_BOUND, Batch, BatchFrame, Event, FrameDesc, FSRParams, MEParams,
                   RfsrError, Sequence, StreamSet, Workspace, frame_motion, fsr_blocks, fsr_blocks_noalloc,
                   lib, motion_check, quality, quality_async, reconstruct_frame, workspace_bytes, LIB_PATH)

__all__ = ["CHECKS", "COUNTER_NAMES", "MIXED_BOUND", "Batch", "BatchFrame", "Event", "FrameDesc", "FSRParams",
           "MEParams", "RfsrError", "Sequence", "StreamSet", "Workspace", "frame_motion", "fsr_blocks",
           "fsr_blocks_noalloc", "lib",
           "motion_check", "quality", "quality_async", "reconstruct_frame", "workspace_bytes",
           "LIB_PATH"]
