"""Host logic of bench.py (no GPU): the one-GPU contract, the algorithmic byte counts behind every
roofline figure, and the CPU-baseline record of the oracle solve."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1802_03061_amd import inputs  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_padded_size():
    # the smallest power of two >= 2n - 1, at least 16
    for n, P in ((2, 16), (8, 16), (9, 32), (33, 128), (64, 128), (65, 256), (512, 1024)):
        assert bench.padded(n) == P


def test_apply_bytes_512_L8():
    """The per-pass algorithmic bytes at 512^2, L = 8, written out term by term: 17 channels of
    512^2 FP64 values (x, y), the FP32 x-spectrum of 512 packed columns by 512 rows, and the quarter
    kernel spectra of 17 mode differences on 513 x 513 frequencies."""
    vec = 17 * 512 * 512 * 8
    spec = 17 * 512 * 512 * 8
    kern = 17 * 513 * 513 * 8
    b = bench.apply_pass_bytes(512, 8)
    assert b == {"A": vec + spec, "B": 2 * spec + kern, "C": spec + 2 * vec}
    assert b == {"A": 71303168, "B": 107094152, "C": 106954752}
    # FP64 apply: 16-byte complex spectra
    b64 = bench.apply_pass_bytes(512, 8, cbytes=16)
    assert b64["B"] == 2 * 2 * spec + 2 * kern


def test_cpu_baseline_record_small():
    """The CPU baseline and the error record on a 16^2, L = 2 problem: an oracle solve timed to the
    tolerance, a reference to 1e-13, and the error of a given solution against it."""
    w = inputs.workload("hg512", seed=0, mu_s=2.0, n=16)
    w["L"] = 2
    w["sigma_hat"] = inputs.hg_sigma_hat(0.5, 2)
    u = np.zeros((5, 16, 16), dtype=complex)
    cpu, err = bench.oracle_2d(w, 1e-8, {"zero": u})
    assert cpu["kind"] == "oracle" and cpu["unit"] == "solves/s" and cpu["value"] > 0
    assert cpu["cores"] >= 1 and cpu["relres_true"] <= 1e-8
    assert err["reference"]["relres_true"] <= 1e-12
    assert err["seed0_cpu_solve"] <= 1e-6
    assert abs(err["zero"] - 1.0) < 1e-12   # a zero solution is off by 100 %
