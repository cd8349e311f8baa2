"""Host-side logic of bench.py (no GPU): the one-GPU refusal, the HBM-traffic
figure locked to the kernel source it was measured on, and the run's
evaluation counts that weight the oracle's sampled times."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from synth import workload  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr or "single" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_figure_is_locked_to_the_kernel_source(tmp_path, monkeypatch):
    """The committed counter summary holds HBM bytes per launch and the hash
    of the kernel source it was taken on; the bench reports the figure only
    while that source is unchanged."""
    got = bench._traffic_from_profile()
    assert got is not None and got > 0
    changed = tmp_path / "k.hip"
    with open(bench.KERNEL_SRC, "rb") as f:
        changed.write_bytes(f.read() + b"\n// changed\n")
    monkeypatch.setattr(bench, "KERNEL_SRC", str(changed))
    assert bench._traffic_from_profile() is None
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(tmp_path / "missing.txt"))
    assert bench._traffic_from_profile() is None


def test_full_run_counts():
    """Evaluations of a whole 450x375 run: every pixel once (initial costs),
    then per level every clipped 3x3-cell region once per candidate step and
    iteration; checked against a direct count of pixels covered by regions."""
    wl = workload("lowres-450x375")
    n_init, full = bench._full_counts(450, 375, wl)
    assert n_init == 450 * 375
    for cell, kp, kr in wl["grids"]:
        cover = 0
        for v in range(375):
            # regions (i, j) whose clipped rect holds row v, times those holding column u, summed over pixels
            nj = sum(1 for j in range(-(-375 // cell)) if max((j - 1) * cell, 0) <= v < min((j + 2) * cell, 375))
            cover += nj
        per_col = sum(sum(1 for i in range(-(-450 // cell)) if max((i - 1) * cell, 0) <= u < min((i + 2) * cell, 450))
                      for u in range(450))
        assert full[cell] == cover * per_col * (kp + kr) * wl["iterations"]


def test_weighted_rate_of_a_uniform_sample():
    """With the same time per evaluation everywhere, the weighted rate is the
    reciprocal of that time whatever the sample's mix."""
    wl = workload("lowres-450x375")
    per = 2e-7
    sample = (per * 1000, 1000, {c: per * 300 * (k + 1) for k, (c, _, _) in enumerate(wl["grids"])},
              {c: 300 * (k + 1) for k, (c, _, _) in enumerate(wl["grids"])})
    rate = bench._weighted(sample, 450, 375, wl)[0]
    assert rate == pytest.approx(1.0 / per / 1e9, rel=1e-12)


def test_committed_profiles_name_the_current_kernel_sources():
    """Every committed profile summary that records the hash of the kernel
    source it was taken on names the source as it stands (a profile of an
    older kernel would describe code that is no longer built)."""
    import glob
    import hashlib
    import re

    def h16(rel):
        with open(os.path.join(ROOT, "paper_1603_08328_amd", "csrc", rel), "rb") as fh:
            return hashlib.sha256(fh.read()).hexdigest()[:16]

    fused, cut = h16("lexp_kernels.hip"), h16("lexp_cut.hip")
    seen = 0
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*"))):
        with open(path) as fh:
            text = fh.read()
        for m in re.finditer(r"Kernel source( \(lexp_cut\.hip\))? sha256\[:16\] ([0-9a-f]{16})", text):
            assert m.group(2) == (cut if m.group(1) else fused), os.path.basename(path)
            seen += 1
        for m in re.finditer(r"kernel_source_sha256_16: ([0-9a-f]{16})", text):
            assert m.group(1) == fused, os.path.basename(path)
            seen += 1
    assert seen >= 5
