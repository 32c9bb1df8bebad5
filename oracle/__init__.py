"""CPU oracle for recursive frequency selective reconstruction (FSR) of
quarter-sampled video with consistency-checked motion projection
(Grosche, Seiler, Kaup, "Novel Consistency Check for Fast Recursive
Reconstruction of Non-Regularly Sampled Video Data", ICIP 2021).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously-correct
statement of what the GPU path computes: integer arithmetic for motion
estimation and the consistency checks, float64 for FSR.  Only the test suite,
the smoke check and the CPU-baseline leg of the benchmark may import it.  The
product path (the HIP library and its Python binding) never imports, calls or
links anything here, and this package shares no code with it.

Modules
  me          Sec. 2.2: pixel-wise template-matching motion estimation.
  checks      Sec. 2.2 (RME), Sec. 3.1.1 (RMC, FRMC), Sec. 3.1.2 / Eq. (1) (NNC).
  projection  Sec. 2.2: projection of measured past pixels, averaged.
  fsr         Sec. 2.1 / Sec. 3.2: block-wise FSR with concealed weighting 0
              (Sec. 4), and the FSR-literature variants the GPU also offers:
              non-zero concealed weighting, conjugate pairs, frequency prior,
              residual-energy early stop.
  frame       Fig. 1 order (ME -> check -> projection -> FSR) for one frame,
              the causal recursion over a sequence, PSNR (Sec. 4).
  quality     mean SSIM reported beside PSNR (Sec. 4).

Readings of points the paper leaves open are listed in each module header.
"""
from .me import (template_offsets, cost_at, reverse_cost_at, n_map, forward_me,
                 forward_me_at)
from .checks import (frmc_offsets, rmc_offsets, reverse_me, rme_accept, rmc_accept, rmc_accept_at,
                     median3x3, nnc_accept, motion_check, CHECKS)
from .projection import project
from .fsr import (rho_table, prior_table, fsr_spatial, fsr_spectral, gather_supports, fsr_frame,
                  fsr_frame_concealed, fsr_pairs_spatial, fsr_pairs_spectral, fsr_pairs_blocks_out)
from .frame import (MEParams, FSRParams, reconstruct_frame, reconstruct_sequence,
                    quantize, psnr)
from .quality import gaussian_window, ssim, ssim_map, ssim_bruteforce

__all__ = [
    "template_offsets", "cost_at", "reverse_cost_at", "n_map", "forward_me",
    "forward_me_at", "frmc_offsets", "rmc_offsets", "reverse_me", "rme_accept",
    "rmc_accept", "rmc_accept_at", "median3x3", "nnc_accept", "motion_check", "CHECKS", "project",
    "rho_table", "prior_table", "fsr_spatial", "fsr_spectral", "gather_supports", "fsr_frame", "fsr_frame_concealed",
    "fsr_pairs_spatial", "fsr_pairs_spectral", "fsr_pairs_blocks_out",
    "MEParams", "FSRParams", "reconstruct_frame", "reconstruct_sequence",
    "quantize", "psnr", "gaussian_window", "ssim", "ssim_map", "ssim_bruteforce",
]
