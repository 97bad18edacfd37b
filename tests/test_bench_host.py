"""Host arithmetic of bench.py's roofline object (no GPU): units, peaks and the HBM view."""
import os
import sys
from types import SimpleNamespace

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def wl2d():
    return SimpleNamespace(name="tgv2d_64k_f32", ckpt_every=8, steps=16, adjoint=True, dtype="f32")


def test_sweep_roofline_against_the_published_fp32_peak():
    wl = wl2d()
    per_state = [1e6] * wl.steps
    # 16 forward sweeps + 14 recomputed ones per job, 2 jobs, 30 us each
    n = 2 * (16 + 14)
    prof = {"sweep": (n * 0.030, n)}
    r = bench.roofline(prof, "sweep", wl, per_state, 2, 2, 4096, (4, 4, 1))
    pairs = (16 + 14) * 1e6 * 2
    flops = bench.FLOPS_PER_PAIR[("sweep", 2)] * pairs / n
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s"
    # the published FP32 vector peak counts packed FP32 (two operations per lane)
    assert r["peak"] == pytest.approx(2 * 256 * 4 * 16 * 2 * 2.4e9 / 1e12, rel=1e-3)
    assert r["achieved"] == pytest.approx(flops / 30e-6 / 1e12, rel=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"], abs=1e-4)
    assert r["frac_of_unpacked_fp32_peak"] == pytest.approx(r["achieved"] / 78.6, abs=1e-4)
    assert r["mean_launch_us"] == pytest.approx(30.0)
    assert r["pairs_per_launch"] == int(pairs / n)


def test_hbm_view_uses_the_counted_bytes(monkeypatch):
    wl = wl2d()
    monkeypatch.setattr(bench, "measured_traffic", lambda w, k: 48_000_000)
    prof = {"adjoint": (16 * 0.020, 16)}
    r = bench.roofline(prof, "adjoint", wl, [500.0] * wl.steps, 1, 2, 4096, (4, 8, 1))
    assert r["traffic"] == 48_000_000
    assert r["hbm_gbs"] == pytest.approx(48e6 / 20e-6 / 1e9, rel=1e-3)
    assert r["hbm_frac"] == pytest.approx(r["hbm_gbs"] / 8000.0, rel=1e-3)


def test_traffic_is_null_once_the_sources_change(tmp_path, monkeypatch):
    prof_dir = tmp_path / "profiles"
    prof_dir.mkdir()
    (prof_dir / "hbm_traffic_and_counters.md").write_text(
        "traffic tgv2d_64k_f32 sph::k_sweep<float,2,0,4> %s 123\n"
        "traffic tgv2d_64k_f32 sph::k_sweep<float,2,0,8> 0000000000000000 456\n" % bench.source_hash())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # the hash is of the sources under ROOT: copy them so it is unchanged
    src = tmp_path / "paper_2507_21684_amd" / "csrc"
    src.mkdir(parents=True)
    for f in ("sph_device.hpp", "sph_api.hip"):
        (src / f).write_bytes(open(os.path.join(ROOT, "paper_2507_21684_amd", "csrc", f), "rb").read())
    assert bench.measured_traffic("tgv2d_64k_f32", "sph::k_sweep<float,2,0,4>") == 123
    assert bench.measured_traffic("tgv2d_64k_f32", "sph::k_sweep<float,2,0,8>") is None
    (src / "sph_api.hip").write_bytes(b"changed")
    assert bench.measured_traffic("tgv2d_64k_f32", "sph::k_sweep<float,2,0,4>") is None


def test_build_roofline_is_hbm_bound():
    wl = wl2d()
    per_state = [1000.0] * wl.steps
    prof = {"build": (4 * 0.010, 4)}
    r = bench.roofline(prof, "build", wl, per_state, 1, 2, 4096, (4, 4, 8))
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    # builds at steps 0 and 8, forward and again in the recomputation
    entries = 4 * (1000 + 4096)
    expect = (4 * entries + 4 * 4096 * (4 + 16)) / 4
    assert r["algorithmic_bytes_per_launch"] == int(expect)
    assert r["achieved"] == pytest.approx(expect / 10e-6 / 1e9, abs=0.1)


def test_cpu_samples_are_bounded_and_spread():
    from paper_2507_21684_amd import inputs as I
    wl = I.batched_512_f32()
    pick, steps, pick1, steps1 = bench.cpu_samples(wl)
    assert len(pick) == 20 and len(set(pick)) == 20 and pick1 == pick and steps == steps1 == wl.steps
    assert min(pick) < 26 and max(pick) > 486
    # the 3D box: two steps of the full state, no single-thread run
    assert bench.cpu_samples(I.tgv3d_262k_f32())[1:] == (2, None, None)


def test_host_info_names_the_cpu():
    info = bench.host_info()
    assert info["nproc"] >= 1 and 1 <= info["usable_cpus"] <= info["nproc"]
    assert isinstance(info["cpu_model"], str)


def test_taped_backward_counts_no_recomputed_sweeps():
    wl = wl2d()
    per_state = [1e6] * wl.steps
    prof = {"sweep": (16 * 0.030, 16)}
    r = bench.roofline(prof, "sweep", wl, per_state, 1, 2, 4096, (4, 4, 1), taped=True)
    assert r["pairs_per_launch"] == int(1e6)
