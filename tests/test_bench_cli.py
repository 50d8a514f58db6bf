"""Host-side checks of bench.py: the one-GPU contract, the VALU slot count
of the inner-product roofline and the choice of value generation per
operand precision.  No GPU is touched."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_slots_per_draw_inner():
    # 1.25 Philox calls x 60 slots + a 1-slot power-of-two index map + two
    # 4-slot values + 2 for the product and sum
    assert bench.slots_per_draw_inner(1 << 20, word32=True) == 86
    assert bench.slots_per_draw_inner(1 << 20, word32=False) == 101
    # any other n: high multiply + multiply-add for the index map
    assert bench.slots_per_draw_inner(1000, word32=False) == 104


def test_peaks_are_the_published_ones():
    assert bench.PEAK_VALU_SLOTS == pytest.approx(78.6e12, rel=1e-3)
    assert bench.PEAK_MFMA == {"fp64": 78.6e12, "fp32": 157.3e12, "bf16": 2.5e15, "fp8": 5.0e15}
    assert bench.PEAK_HBM == 8.0e12


@pytest.mark.parametrize("bits, expect", [
    ("auto", {"fp64": False, "fp32": False, "bf16": True, "fp8": True}),
    ("23", {"fp64": False, "fp32": False, "bf16": False, "fp8": False}),
    ("16", {"fp64": True, "fp32": True, "bf16": True, "fp8": True}),
])
def test_value_bits_choice(monkeypatch, bits, expect):
    monkeypatch.setitem(bench._OPTS, "value_bits", bits)
    assert {p: bench._value16(p) for p in expect} == expect


def test_host_threads_and_cpu_model():
    assert 1 <= bench.host_threads() <= 16
    assert isinstance(bench.cpu_model(), str) and bench.cpu_model()
