"""fsr_blocks_noalloc (the entry point that allocates nothing; its scratch is
an array inside the library) against fsr_blocks (caller's workspace) on two
calls in a row, the second with a smaller frame and other parameters, so
that it runs on the array the first call left behind.  Both entry points run
the same kernels on the same inputs, so their outputs must be identical; the
first frame is also held to the float64 oracle's tolerance."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from _gpu import AMB_MAX, FSR_TOL, compare_fsr, dev, host, need_gpu

pytestmark = pytest.mark.gpu

CASES = [  # (H, W, seed, FSR parameters)
    (192, 256, 11, dict(iters=100, rho=0.7)),
    (64, 96, 12, dict(iters=40, rho=0.8, gamma=0.4, overwrite="rfsr")),
]


def test_noalloc_equals_fsr_blocks_on_two_calls():
    R = need_gpu()
    for H, W, seed, kw in CASES:
        print(f"fsr_blocks_noalloc {H}x{W} seed={seed} {kw}", flush=True)
        f, m = synth.workload_c2(n=1, h=H, w=W, seed=seed)
        meas = synth.measured(f, m)[0]
        v, c = dev(meas, torch.float32), dev(m[0])
        prm = R.FSRParams(**kw)
        ref, ref_u8 = R.fsr_blocks(v, c, prm)
        out = torch.full((H, W), float("nan"), dtype=torch.float32, device=v.device)
        out_u8 = torch.zeros((H, W), dtype=torch.uint8, device=v.device)
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        got, got_u8 = R.fsr_blocks_noalloc(v, c, prm, out=out, out_u8=out_u8)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before
        assert got is out and got_u8 is out_u8
        assert torch.equal(got, ref) and torch.equal(got_u8, ref_u8)
        if seed == 11:
            ora, gaps = O.fsr_frame(meas.astype(np.float64), m[0], K=kw["iters"], rho=kw["rho"])
            worst, namb, nb = compare_fsr(host(got), ora, gaps)
            print(f"  max |noalloc - oracle| {worst:.2e}, ambiguous {namb}/{nb}")
            assert worst <= FSR_TOL and namb <= AMB_MAX * nb
        # release this case's tensors before the next measures the allocator
        del v, c, ref, ref_u8, out, out_u8, got, got_u8


def test_noalloc_fp32_form_and_output_without_u8():
    R = need_gpu()
    f, m = synth.workload_c2(n=1, h=96, w=128, seed=13)
    meas = synth.measured(f, m)[0]
    v, c = dev(meas, torch.float32), dev(m[0])
    prm = R.FSRParams(iters=60, precision="fp32")
    ref, _ = R.fsr_blocks(v, c, prm, want_u8=False)
    got, got_u8 = R.fsr_blocks_noalloc(v, c, prm)
    torch.cuda.synchronize()
    assert got_u8 is None
    assert torch.equal(got, ref)
