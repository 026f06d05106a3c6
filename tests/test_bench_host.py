"""bench.py's host-side arithmetic and contract, on the CPU: the
precision-weighted factor roofline, the measured-traffic figures that are
valid only for the sources they were taken on, and the one-GPU limit."""
import os
import shutil
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _stats(qr=0.0, diag=0.0, vs=0.0, schur=0.0, pair=0.0, far=0.0, root=0.0):
    fl = [0.0] * len(bench.PHASES)
    fl[0], fl[1], fl[3], fl[4], fl[5], fl[7] = qr, diag, vs, pair, far, root
    return {"flops_factor_phase": fl, "flops_schur": schur}


def test_factor_roofline_weights_each_phase_by_its_instruction_peak():
    f64, f32, bf = 78.6e12, 157.3e12, 2500e12
    # split BF16 (prec 3): transforms at a third of the BF16 peak, the Schur
    # update on FP32, V, QR and root on FP64; one second each
    st = _stats(qr=f64, vs=f64 + f32, schur=f32, pair=bf / 3, root=f64)
    t = [0.0] * len(bench.PHASES)
    t[0], t[3], t[4], t[7] = 2.0, 4.0, 1.0, 0.5
    r = bench.factor_roofline(st, t, 10.0, 3)
    assert r["bound"] == "mfma"
    assert r["ideal_s"] == pytest.approx(5.0)
    assert r["frac"] == pytest.approx(0.5)
    ph = r["phases"]
    assert set(ph) == {"basis_qr", "v_schur", "near_pair_transform", "root"}
    assert ph["basis_qr"]["frac"] == pytest.approx(0.5)
    assert ph["v_schur"]["frac"] == pytest.approx(0.5)
    assert ph["near_pair_transform"]["frac"] == pytest.approx(1.0)
    assert ph["near_pair_transform"]["tflops"] == pytest.approx(bf / 3 / 1e12)
    assert ph["root"]["frac"] == pytest.approx(2.0)
    # the plain FP64 path: every phase on FP64
    r0 = bench.factor_roofline(_stats(pair=f64, vs=f64, schur=f64 / 2), [1.0] * len(bench.PHASES),
                               4.0, 0)
    assert r0["ideal_s"] == pytest.approx(2.0) and r0["frac"] == pytest.approx(0.5)
    # FP32 and plain BF16 transforms
    assert bench.factor_roofline(_stats(diag=f32), [1.0] * 9, 1.0, 1)["ideal_s"] == pytest.approx(1.0)
    assert bench.factor_roofline(_stats(far=bf), [1.0] * 9, 1.0, 2)["ideal_s"] == pytest.approx(1.0)


def test_measured_traffic_is_tied_to_its_sources(tmp_path, monkeypatch):
    for k, m in bench.MEASURED_TRAFFIC.items():
        assert bench.measured_traffic(k) == m["bytes_per_launch"], k
    assert bench.measured_traffic("no_such_kernel") is None
    # a copy of the sources with one byte changed no longer matches
    for src in bench.GATHER_SRC:
        dst = tmp_path / src
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(ROOT, src), dst)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    k = next(iter(bench.MEASURED_TRAFFIC))
    assert bench.measured_traffic(k) == bench.MEASURED_TRAFFIC[k]["bytes_per_launch"]
    with open(tmp_path / bench.GATHER_SRC[0], "ab") as f:
        f.write(b"\n")
    assert bench.measured_traffic(k) is None


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
