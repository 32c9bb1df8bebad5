"""Host logic of bench.py (CPU): the algorithmic flop count of an FSR block,
percentiles, the PSNR report, the refusal of more than one GPU, and the
gating of the committed counter record by the hash of the FSR kernel's
sources."""
import json
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2203_09200_amd import profiling  # noqa: E402


def test_fsr_flops_per_block():
    # 1024 complex bins x 11 flops per iteration, one 32x32 complex FFT
    # (5 N log2 N), 16 pixels x 4 flops per synthesised coefficient
    assert bench.fsr_flops_per_block(100) == 11 * 1024 * 100 + 5 * 1024 * 10 + 64 * 100 == 1_184_000
    assert bench.fsr_flops_per_block(0) == 51_200
    assert bench.fsr_flops_per_block(50, pairs=True) == 19 * 513 * 50 + 51_200 + 64 * 50


def test_percentile():
    xs = [5.0, 1.0, 3.0, 2.0, 4.0]
    assert bench.percentile(xs, 50) == 3.0
    assert bench.percentile(xs, 0) == 1.0 and bench.percentile(xs, 100) == 5.0
    assert bench.percentile([1.0, 2.0], 50) == 1.5
    assert bench.percentile([], 50) is None


def test_psnr_report():
    rng = np.random.default_rng(0)
    ref = rng.integers(0, 256, (100, 120)).astype(np.uint8)
    assert bench.psnr(ref, ref.astype(np.float32), border=10) == float("inf")
    test = ref.astype(np.float64) + 2.0          # MSE 4 away from the clamp at 255
    test[ref > 250] -= 4.0
    mse = np.mean((ref[10:-10, 10:-10] - np.clip(test, 0, 255)[10:-10, 10:-10]) ** 2)
    assert bench.psnr(ref, test, border=10) == pytest.approx(10 * np.log10(255.0 ** 2 / mse))


def test_more_than_one_gpu_is_refused(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    assert "one GPU" in capsys.readouterr().err


def test_counter_record_is_used_only_for_the_measured_sources(tmp_path, monkeypatch):
    rec = {"kernel": "fsr_block_kernel", "bytes_per_launch": 123.0, "valu_insts_per_dispatch": 4.0}
    (tmp_path / "profiles").mkdir()
    path = tmp_path / "profiles" / "fsr_block_kernel_1080p_traffic.json"
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.counters_from_profile() == {}                     # no record
    path.write_text(json.dumps({**rec, "kernel_sha256": "0" * 64}))
    assert bench.counters_from_profile() == {}                     # other sources
    path.write_text(json.dumps({**rec, "kernel_sha256": profiling.kernel_digest()}))
    assert bench.counters_from_profile()["bytes_per_launch"] == 123.0


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_kernel_digest_covers_every_source(tmp_path, monkeypatch, precision):
    csrc = tmp_path / "csrc"
    csrc.mkdir()
    names = profiling.FORMS[precision]["sources"]
    for name in names:
        (csrc / name).write_text(name)
    monkeypatch.setattr(profiling, "HERE", str(tmp_path))
    d0 = profiling.kernel_digest(precision)
    for name in names:
        (csrc / name).write_text(name + " changed")
        assert profiling.kernel_digest(precision) != d0, name
        (csrc / name).write_text(name)
    assert profiling.kernel_digest(precision) == d0
    assert "fsr32.hip" in profiling.FORMS["mixed"]["sources"]   # the float32 pass is part of a mixed launch


def test_traffic_record_scales_counters_by_the_copy(tmp_path, monkeypatch):
    """record(): the FSR kernel's FETCH_SIZE / WRITE_SIZE per dispatch, each
    scaled by what the same counter reads for a copy of known size."""
    def csv_file(name, rows):
        p = tmp_path / name
        lines = ["Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value"]
        lines += [f'{d},"{k}",{c},{v}' for d, k, c, v in rows]
        p.write_text("\n".join(lines) + "\n")
        return str(p)
    kern = "void rfsr::fsr_block_kernel<0, false, false, 0>(args)"
    ff = csv_file("ff.csv", [(1, kern, "FETCH_SIZE", 600.0), (2, kern, "FETCH_SIZE", 800.0),
                             (3, "other_kernel", "FETCH_SIZE", 5.0)])
    fw = csv_file("fw.csv", [(1, kern, "WRITE_SIZE", 1000.0), (2, kern, "WRITE_SIZE", 1000.0)])
    cf = csv_file("cf.csv", [(1, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 512.0)])
    cw = csv_file("cw.csv", [(1, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 1024.0)])
    sq = csv_file("sq.csv", [(1, kern, "SQ_INSTS_VALU", 10.0), (2, kern, "SQ_INSTS_VALU", 14.0)])
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(profiling, "ROOT", str(tmp_path))
    profiling.record(ff, fw, cf, cw, 1, "copyBuffer", sq_csv=sq)
    rec = json.loads((tmp_path / "profiles" / "fsr_block_kernel_1080p_traffic.json").read_text())
    # 1 MiB copied: FETCH_SIZE unit = 2^20 / 512 bytes, WRITE_SIZE unit = 2^20 / 1024 bytes
    assert rec["fetch_scale_bytes_per_unit"] == 2048.0 and rec["write_scale_bytes_per_unit"] == 1024.0
    assert rec["bytes_per_launch"] == 700.0 * 2048.0 + 1000.0 * 1024.0
    assert rec["valu_insts_per_dispatch"] == 12.0
    assert rec["kernel_sha256"] == profiling.kernel_digest()


def test_banded_oracle_equals_whole_frame_oracle():
    """The CPU baseline's decomposition (motion path on column strips of the
    band with halos, projection, FSR on block tiles, as pool tasks) gives
    exactly the whole-frame oracle's rows: at the bench's setting (R = 9,
    NNC -> FRMC, the default halo) on a frame large enough for crops whose
    edges lie inside it, and for RME (the widest reach, 2R + 2) with a halo
    just above that reach."""
    import multiprocessing as mp
    import oracle as O
    import synth
    rng = np.random.default_rng(4)
    fsr = O.FSRParams(iters=8)
    with mp.get_context("spawn").Pool(2) as pool:
        for H, W, R, check, y0, y1, strips, halo in ((120, 96, 9, "nnc_frmc", 52, 68, 3, None),
                                                    (64, 48, 4, "rme", 24, 40, 3, 12)):
            frames, _ = synth.video_translate_edges(4, H, W, rng, max_step=3, n_edges=3)
            masks = synth.mask_sequence("dynamic", 4, H, W, rng)
            meas = synth.measured(frames, masks)
            recon = [np.clip(frames[t].astype(int) + rng.integers(-4, 5, (H, W)), 0, 255).astype(np.uint8)
                     for t in range(3)]
            refs = [(recon[2 - k], meas[2 - k], masks[2 - k]) for k in range(3)]
            me = O.MEParams(search=R, check=check)
            if halo is None:
                assert bench.oracle_halo(me) == 22
            whole = O.reconstruct_frame(meas[3], masks[3], refs, me, fsr, track_gaps=False)["out"]
            got = bench.oracle_frame_rows(pool, meas[3], masks[3], refs, me, fsr, y0, y1, strips=strips,
                                          halo=halo)
            assert np.array_equal(got, whole[y0:y1]), (check, y0, y1)


def test_cpu_cores_is_one_gpu_share():
    assert 1 <= bench.cpu_cores() <= 16


def test_mixed_record_adds_the_float32_pass_and_the_recomputation(tmp_path, monkeypatch):
    """A mixed launch is two dispatches; its record adds their per-dispatch
    averages, and the float64 kernel's name does not also match the float32
    pass's."""
    def csv_file(name, rows):
        p = tmp_path / name
        lines = ["Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value"]
        lines += [f'{d},"{k}",{c},{v}' for d, k, c, v in rows]
        p.write_text("\n".join(lines) + "\n")
        return str(p)
    k32 = "void rfsr::fsr_block_kernel_f32<1>(args)"
    k64 = "void rfsr::fsr_block_kernel<0, false, false, 0, true>(args)"
    ff = csv_file("ff.csv", [(1, k32, "FETCH_SIZE", 100.0), (2, k64, "FETCH_SIZE", 10.0),
                             (3, k32, "FETCH_SIZE", 300.0), (4, k64, "FETCH_SIZE", 30.0)])
    fw = csv_file("fw.csv", [(1, k32, "WRITE_SIZE", 50.0), (2, k64, "WRITE_SIZE", 5.0)])
    cf = csv_file("cf.csv", [(1, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 1024.0)])
    cw = csv_file("cw.csv", [(1, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 1024.0)])
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(profiling, "ROOT", str(tmp_path))
    profiling.record(ff, fw, cf, cw, 1, "copyBuffer", precision="mixed")
    rec = json.loads((tmp_path / "profiles" / "fsr_mixed_1080p_traffic.json").read_text())
    assert rec["fetch_kib_per_dispatch"] == 200.0 + 20.0 and rec["write_kib_per_dispatch"] == 55.0
    assert rec["bytes_per_launch"] == (220.0 + 55.0) * 1024.0
    assert rec["kernel_sha256"] == profiling.kernel_digest("mixed")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.counters_from_profile("mixed")["bytes_per_launch"] == rec["bytes_per_launch"]
    assert bench.counters_from_profile("fp64") == {} and bench.counters_from_profile("fp32") == {}
