"""Host-side logic of the benchmark and the seeded input recipes (no GPU): the
steps-to-thermalize definition, the counter-record check, the one-GPU guard, and the
workloads' shapes and coupling laws."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2102_05613_amd import inputs  # noqa: E402


def test_t_within_definition():
    """t_1%: the first t after which every window mean stays within 1% of the
    reference; None when the tail never settles."""
    ref = -1.0
    e = np.concatenate([np.linspace(0.0, -1.0, 50), np.full(200, -1.0)])
    t = bench._t_within(e, ref, window=10)
    # windows starting at t' >= t have means within 1% of -1; the one before does not
    assert t is not None
    win = lambda s: e[s:s + 10].mean()
    assert abs(win(t) - ref) <= 0.01 and abs(win(t - 1) - ref) > 0.01
    assert bench._t_within(np.full(100, -0.5), ref, window=10) is None
    assert bench._t_within(np.full(100, -1.0), ref, window=10) == 0
    assert bench._t_within(np.full(5, -1.0), ref, window=10) is None   # shorter than a window


def test_traffic_record_is_tied_to_the_kernel_sources(tmp_path, monkeypatch):
    """The committed counter record is used only while the split kernel's sources hash
    to its source_sha256."""
    h = bench.kernel_source_hash()
    rec = {"kernel": "k_score_split", "fetch_bytes": 1.0, "write_bytes": 2.0, "source_sha256": h}
    f = tmp_path / "traffic.md"
    f.write_text("# notes\n\n" + json.dumps(rec) + "\n")
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(f))
    got, status = bench._traffic_from_profile()
    assert status == "measured" and got["fetch_bytes"] == 1.0
    rec["source_sha256"] = "0" * 64
    f.write_text(json.dumps(rec) + "\n")
    got, status = bench._traffic_from_profile()
    assert got is None and "changed" in status
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(tmp_path / "missing.md"))
    assert bench._traffic_from_profile()[0] is None


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU" in out.stderr


def test_workload_recipes():
    names = [w.name for w in inputs.workloads()]
    assert names[0] == "sk_n32_pm1_m4" and "sk_n1024_m128_split" in names
    w = inputs.workload("sk_n1024_m128_split")
    assert (w.N, w.M, w.chains, w.kmin, w.kmax) == (1024, 128, 256, 1, 128)
    J, scale = w.couplings_matrix()
    assert J.shape == (1024, 1024) and scale == 1.0
    assert np.array_equal(J, J.T) and not np.any(np.diag(J))
    iu = np.triu_indices(1024, 1)
    assert np.var(J[iu]) == pytest.approx(1.0 / 1024, rel=0.02)   # J ~ N(0, 1/N)
    J2, _ = w.couplings_matrix()
    assert np.array_equal(J, J2)                                   # seeded
    P, sp = inputs.couplings_pm1(32, 0x5EED0001)
    assert sp == pytest.approx(1.0 / np.sqrt(32)) and set(np.unique(P[np.triu_indices(32, 1)])) == {-1.0, 1.0}


def test_batch_recipe():
    d = inputs.batch_descs(200)
    N = np.array([x[0] for x in d])
    M = np.array([x[1] for x in d])
    assert np.all(N % 64 == 0) and N.min() >= 64 and N.max() <= 2048
    assert M.min() >= 8 and M.max() <= 256
    assert all(x[2] == inputs.BATCH_CHAINS and x[3] == 1 and 1 <= x[4] <= max(1, x[0] // 16) for x in d)
    assert d == inputs.batch_descs(200)


def test_beta_schedule():
    b = inputs.beta_schedule(0.1, 3.0, 1000, 0, 1000)
    assert b[0] == 0.1 and b[-1] == pytest.approx(3.0, rel=1e-15)
    assert np.all(np.diff(b) > 0)
    np.testing.assert_array_equal(inputs.beta_schedule(0.1, 3.0, 1000, 500, 10), b[500:510])


def test_source_hash_ignores_comments():
    """The counter record's source hash covers code only: a comment or blank-line edit
    keeps it, a code edit changes it."""
    a = "int x = 1;  // one\n\n// note\nint y;\n"
    b = "int x = 1;\n// another note\nint y;   \n"
    c = "int x = 2;\nint y;\n"
    assert bench.code_lines(a) == bench.code_lines(b) == ["int x = 1;", "int y;"]
    assert bench.code_lines(c) != bench.code_lines(a)
