"""GPU parity of the consistency-check options of rfsr_me_params against the
integer oracle, bit-exact: an FRMC offset set given as data (Sec. 3.1.1; the
small range {-2,-1,0,1,2} of the Fig. 2 caption, asymmetric sets, 15 offsets
reaching 14), raw instead of normalised reverse costs (an ablation of the
S/n reading) in RME, RMC and FRMC, and the raw vector at p in NNC (the other
reading of Sec. 3.1.2).  Each case also changes decisions against the
default setting on these inputs, so the option is exercised."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from _gpu import dev, host, need_gpu
from test_gpu_frame import teacher_forced_case

pytestmark = pytest.mark.gpu

CASES = [("frmc", dict(frmc=(-2, -1, 0, 1, 2))),
         ("frmc", dict(frmc=(-5, -2, 0, 4))),
         ("nnc_frmc", dict(frmc=(-3, 0, 3))),
         ("frmc", dict(frmc=tuple(range(-14, 1)))),
         ("rme", dict(cost_norm=False)),
         ("rmc", dict(cost_norm=False)),
         ("frmc", dict(cost_norm=False)),
         ("nnc_frmc", dict(cost_norm=False, frmc=(-7, -2, 0, 2, 7))),
         ("nnc", dict(nnc_center="raw")),
         ("nnc_frmc", dict(nnc_center="raw"))]


@pytest.mark.parametrize("check,opts", CASES)
def test_check_options_bit_exact(check, opts):
    R = need_gpu()
    frames, masks = synth.workload_c1()
    meas = synth.measured(frames, masks)
    cur, mask, ref = meas[1], masks[1], frames[0]
    noisy = np.clip(ref.astype(int) + np.random.default_rng(0).integers(-8, 9, ref.shape), 0, 255).astype(np.uint8)
    changed = 0
    for r in (ref, noisy):
        cnt = torch.zeros(4, dtype=torch.int64, device="cuda")
        mv, acc, _ = R.motion_check(dev(cur), dev(mask), dev(r), R.MEParams(search=8, check=check, **opts),
                                    counters=cnt)
        mv, acc, cnt = host(mv).astype(np.int64), host(acc).astype(bool), host(cnt)
        a, b, S, n = O.forward_me(cur, mask, r, 8)
        assert (mv[0] == a).all() and (mv[1] == b).all()
        oacc, oev = O.motion_check(check, cur, mask, r, a, b, 8, **opts)
        print(f"{check} {opts}: accept {acc.mean():.3f}, check costs {cnt[1]} (oracle, no early exit, {oev})")
        assert (acc == oacc).all()
        assert cnt[3] == oacc.sum()
        if check == "rme":
            assert cnt[1] == oev
        else:
            assert cnt[1] <= oev
        dflt, _ = O.motion_check(check, cur, mask, r, a, b, 8)
        changed += int((oacc != dflt).sum())
    assert changed > 0


@pytest.mark.parametrize("check,opts", [("nnc_frmc", dict(frmc=(-2, -1, 0, 1, 2), nnc_center="raw")),
                                        ("frmc", dict(cost_norm=False, frmc=(-9, -4, 0, 4, 9))),
                                        ("rme", dict(cost_norm=False))])
def test_frame_path_with_check_options(check, opts):
    """The frame entry point (checks on projectable pixels only, projection,
    FSR) with the options, teacher-forced against the oracle's frame."""
    teacher_forced_case(64, 80, check, "dynamic", 3, seed=21, me_opts=opts)
