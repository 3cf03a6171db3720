"""Host logic of bench.py (no GPU): the one-GPU guard, the algorithmic byte
model of each phase, and the reading of measured traffic from a counter
summary keyed by the kernel-source hash."""
import hashlib
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_phase_bytes_model():
    N, S, n, esz = 128, 5, 8_500_000, 4
    cells = N ** 3
    X = (N + 1) * N * N * 8
    C = (N + 1) * 2 * N * N * 8
    H = (N + 1) ** 3 * 4
    assert bench.phase_bytes("fwd_x", N, S, n, esz) == S * (cells * 4 + X)
    assert bench.phase_bytes("zpass", N, S, n, esz) == S * (2 * C + H)
    assert bench.phase_bytes("inv_y", N, S, n, esz) == bench.phase_bytes("fwd_y", N, S, n, esz)
    # one 128^3 solve moves 228 MB in FP32 (the five passes)
    one = sum(bench.phase_bytes(p, N, 1, n, esz) for p in bench.FFT_PASSES)
    assert 227e6 < one < 229e6
    # force: x, v read and written (12 esz), galaxy and flag bytes, fields once
    assert bench.phase_bytes("force", N, S, n, esz) == n * (12 * esz + 2) + S * cells * esz
    assert bench.phase_bytes("unknown", N, S, n, esz) == 0


def _summary(tmp_path, digest, force_total):
    text = "\n".join([
        "# test summary", "", f"Kernel-source hash: {digest}", "",
        "| kernel | dispatches | read MB/dispatch | written MB/dispatch | total MB/dispatch |",
        "|---|---|---|---|---|",
        f"| k_force<float, 1> | 9 | 300.00 | 200.00 | {force_total:.2f} |",
        "| k_deposit<float, false> | 11 | 150.00 | 50.00 | 200.00 |",
    ])
    p = tmp_path / "summary.md"
    p.write_text(text + "\n")
    return str(p)


def _hash(paths):
    h = hashlib.sha256()
    for f in paths:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def test_measured_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("kernel source\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "KERNEL_SOURCES", ["k.hip"])
    monkeypatch.setattr(bench, "PROFILE", _summary(tmp_path, _hash([src]), 500.0))
    assert bench.measured_traffic("force") == pytest.approx(500.0e6)
    assert bench.measured_traffic("deposit") == pytest.approx(200.0e6)
    assert bench.measured_traffic("zpass") is None        # no kernel mapped to the phase
    src.write_text("kernel source, changed\n")              # counters no longer describe it
    assert bench.measured_traffic("force") is None


def test_phase_kernels_named_in_the_committed_profile():
    """Every kernel the bench maps a phase to has a row (5 cells) in the
    committed counter summary, under the name the profiler gives it."""
    import os
    text = open(os.path.join(bench.ROOT, bench.PROFILE)).read()
    rows = {[c.strip() for c in l.strip("|").split("|")][0] for l in text.splitlines()
            if l.startswith("|") and len(l.strip("|").split("|")) == 5}
    for phase, name in bench.PHASE_KERNEL.items():
        assert name in rows, (phase, name)


def test_measured_traffic_missing_files(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "KERNEL_SOURCES", ["absent.hip"])
    assert bench.measured_traffic("force") is None


def test_cpu_baseline_step_equals_oracle_step():
    """The CPU baseline's step (System.step's phases with the per-particle
    Eq. 8 phase over forked workers) gives the oracle's System.step exactly."""
    import bench
    import synth
    from tests import common as T
    w = T.small_galaxy(scale=0.002, N=32, q=1.0)
    sysm = T.oracle_system(w)
    lost = np.zeros(w.n, bool)
    a = sysm.step(w.x, w.v, w.m, w.gal, lost, w.dt)
    b = bench.oracle_parallel_step(sysm, w.x, w.v, w.m, w.gal, lost, w.dt, 2)
    for p, q in zip(a, b):
        assert np.array_equal(p, q)


def test_cpu_threads_respects_budget(monkeypatch):
    import bench
    monkeypatch.setenv("OMP_NUM_THREADS", "3")
    assert bench.cpu_threads() == 3
    monkeypatch.delenv("OMP_NUM_THREADS")
    assert 1 <= bench.cpu_threads() <= 16


def test_plane_form_bytes_and_form_parsing():
    """The plane-fused form's algorithmic bytes (no x-transformed planes in
    memory) and the form read from a tuning report."""
    import bench
    N, S, esz = 128, 5, 4
    cells = N ** 3
    C = (N + 1) * 2 * N * N * 8
    X = (N + 1) * N * N * 8
    H = (N + 1) ** 3 * esz
    three = sum(bench.phase_bytes(p, N, S, 0, esz, 3) for p in bench.FFT_PASSES)
    five = sum(bench.phase_bytes(p, N, S, 0, esz, 5) for p in bench.FFT_PASSES)
    assert three == S * (2 * cells * esz + 4 * C + H)
    assert five - three == S * 4 * X
    rep = ("fp32 N=128 x5 form=3 plane_fwd nt=1024\nfp32 N=128 x5 form=3 zpass nt=256 grid=tiles v=16\n"
           "fp64 N=128 x5 form=5 fwd_x nt=256 grid=tiles v=16\n")
    assert bench.fft_form(rep, 4, 128, 5) == 3
    assert bench.fft_form(rep, 8, 128, 5) == 5
    assert bench.fft_form(rep, 4, 64, 5) == 5
