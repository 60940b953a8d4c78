"""Host-side checks of the benchmark's arithmetic (no device): the complex-CSR bytes per restart
against the figures derived from the same formula for the L = 20 ring and the Bose chain, the
roofline entry and the sparse-product + orthogonalisation rates from synthetic kernel totals,
and the refusal of more than one GPU."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_survey_bytes_per_restart():
    # the Krylov build's bytes plus the recombination's 16 d (m + 1) give the per-restart totals
    # derived for the configurations: XXZ L = 20 (d = 2^20, nnz = 11,534,336, m = 40) 40.95 GB,
    # Bose chain K = N = 12 (d = 1,352,078, nnz = 16,871,582, m = 60) 107.6 GB
    for d, nnz, m, total in [(1 << 20, 11534336, 40, 40.95e9), (1352078, 16871582, 60, 107.6e9)]:
        assert bench.survey_bytes_per_restart(d, nnz, m) + 16.0 * d * (m + 1) == pytest.approx(total, rel=1e-3)
    # one iteration by hand: 20 nnz + 4 (d + 1) + 16 d (2 j + 5) at j = 1
    d, nnz = 1000, 5000
    assert bench.survey_bytes_per_restart(d, nnz, 1) == 20 * nnz + 4 * (d + 1) + 16 * d * 7


def _totals(**seconds_bytes_launches):
    t = {k: {"launches": 0, "seconds": 0.0, "bytes": 0.0} for k in ("project", "update", "step", "combine", "fold")}
    for k, (sec, byt, n) in seconds_bytes_launches.items():
        t[k] = {"launches": n, "seconds": sec, "bytes": byt}
    return t


def test_roofline_entry_from_totals():
    t = _totals(project=(2.0, 8.0e12, 100), update=(1.0, 6.0e12, 100), step=(0.1, 0.0, 4), fold=(0.05, 0.0, 100))
    r = bench.roofline_of(t)
    assert r["kernel"] == "project" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["achieved"] == pytest.approx(4000.0) and r["frac"] == pytest.approx(0.5)
    assert r["algorithmic_bytes_per_launch"] == pytest.approx(8.0e10)
    s = bench.spmv_orth_rates(t, 1 << 20, 11534336, 40, 10)
    assert s["gbs"] == pytest.approx(14.0e12 / 3.05 / 1e9)
    assert s["gbs_on_complex_csr_bytes"] == pytest.approx(10 * bench.survey_bytes_per_restart(1 << 20, 11534336, 40)
                                                          / 3.05 / 1e9)


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert p.returncode == 2 and "one GPU" in p.stderr and p.stdout == ""
