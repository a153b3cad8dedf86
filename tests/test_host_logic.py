"""Host-side logic without a GPU: the benchmark's byte counts, its traffic
record and its one-GPU rule; the workload generators of the paper's
set-ups; the sweep drivers' case lists and comparison."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1906_03065_amd import taylor as T  # noqa: E402
from paper_1906_03065_amd import workloads as W  # noqa: E402


def test_bytes_per_lattice_update():
    # algorithmic: the three population sets read and written once
    assert bench.alg_bytes_per_lup("fp32", 9) == 216
    assert bench.alg_bytes_per_lup("fp32", 19) == 456
    assert bench.alg_bytes_per_lup("fp64", 9) == 432
    assert bench.alg_bytes_per_lup("fp16", 9) == 120
    # stored: FP32 keeps g_0, h_0 in FP64; 16-bit keeps f_0 in FP32, g_0, h_0 in FP64
    assert bench.stored_bytes_per_lup("fp32", 9) == 232
    assert bench.stored_bytes_per_lup("fp32", 19) == 2 * (55 * 4 + 16)
    assert bench.stored_bytes_per_lup("fp16", 9) == 136
    assert bench.stored_bytes_per_lup("bf16", 19) == 2 * (54 * 2 + 4 + 16)


def test_traffic_record_only_for_its_workload():
    t = bench.measured_traffic("fp32", 2048, 1)
    assert t is None or 0.9e9 < t < 2e9
    assert bench.measured_traffic("fp16", 2048, 1) is None
    assert bench.measured_traffic("fp32", 1024, 1) is None


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_taylor_setup_geometry():
    for sym in (True, False):
        w = W.taylor2d(5e-4, 1e-2, 1e-4, symmetric=sym)
        p = w["params"]
        assert (p["nx"], p["ny"], p["wall_y"]) == (240, 120, 0)
        assert p["kappa"][:2] == ([8e-3, 8e-3] if sym else [8e-3, 2e-3])
        assert p["alpha"] == 2.0 and p["kappa_c"] == 1e-2 and p["r_cut"] == 24.0
        X = w["membranes"][0]["X"]
        assert X.shape == (160, 2)
        np.testing.assert_allclose(np.linalg.norm(X - (120.0, 59.5), axis=1), 20.0, rtol=1e-12)
    assert len(W.TAYLOR_KAPPA3_SYM) == 20 and len(W.TAYLOR_KAPPA3_ASYM) == 16
    assert W.TAYLOR_KAPPA3_SYM[-1] == pytest.approx(1e-2) and W.TAYLOR_KAPPA3_ASYM[-1] == pytest.approx(8e-3)
    w = W.taylor2d(1e-3, 1e-2, 1e-4, u0=1e-3)
    np.testing.assert_allclose(w["fields"]["u"][0], 1e-3)


def test_taylor_case_list_and_compare():
    cases = T.case_list()
    assert len(cases) == (20 + 16) * 6
    assert len(T.case_list(stride=2, which="sym")) == 10 * 6
    sweep = {"runs": [dict(symmetric=True, kappa3=5e-4, kappa_s=0.1, kappa_b=1e-4, D=0.23),
                      dict(symmetric=False, kappa3=1e-3, kappa_s=0.01, kappa_b=1e-2, D=0.18)]}
    ref = {"runs": [dict(symmetric=True, kappa3=5e-4, kappa_s=0.1, kappa_b=1e-4, D=0.20),
                    dict(symmetric=False, kappa3=1e-3, kappa_s=0.01, kappa_b=1e-2, D=0.20)]}
    rows, summ = T.compare(sweep, ref)
    assert [round(r[6], 12) for r in rows] == [0.15, -0.1]
    assert summ["sym"]["within_10pct"] == 0 and summ["asym"]["max"] == pytest.approx(0.1)


def test_prestressed_mesh_rest_lengths():
    w = W.prestressed_mesh(2, lam0=1.25)
    m = w["membranes"][0]
    X, F = m["X"], np.asarray(m["tris"])
    keys = sorted({(min(int(t[k]), int(t[(k + 1) % 3])), max(int(t[k]), int(t[(k + 1) % 3])))
                   for t in F for k in range(3)})
    assert len(keys) == len(m["rest"]) == 3 * len(F) // 2
    lens = np.array([np.linalg.norm(X[a] - X[b]) for a, b in keys])
    np.testing.assert_allclose(lens / m["rest"], 1.25, rtol=1e-12)
    assert m["law"] == 2 and w["params"]["kappa_c"] == 0.0


def test_mode_decay_fields():
    for mode in ("phi", "psi"):
        w = W.mode_decay(mode, mobility=(0.3, 0.1))
        p, f = w["params"], w["fields"]
        assert p["gamma_phi"] * (p["tau_phi"] - 0.5) == pytest.approx(0.3)
        assert p["gamma_psi"] * (p["tau_psi"] - 0.5) == pytest.approx(0.1)
        q = f["phi"] if mode == "phi" else f["psi"]
        assert np.abs(q).max() <= 1.0e-5 * (1 + 1e-12)
        np.testing.assert_allclose(f["rho"], 1.0)
