"""Pins of the oracle's random-number layer (Philox4x32-10 and conversions).

Philox is checked against PyTorch's independent header-only implementation;
the conversions against exact closed forms and distribution tests.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))


def _torch_include():
    try:
        import torch
    except Exception:
        return None
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    return inc if os.path.exists(os.path.join(inc, "ATen", "core", "PhiloxRNGEngine.h")) else None


def test_philox_matches_aten_engine(orc, tmp_path):
    inc = _torch_include()
    if inc is None or shutil.which("g++") is None:
        pytest.skip("ATen Philox header or g++ not available")
    exe = tmp_path / "aten_philox"
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", inc, "-o", str(exe),
                    os.path.join(HERE, "aten_philox_check.cpp")], check=True)
    rng = np.random.default_rng(1234)
    rows = rng.integers(0, 2**32, size=(300, 6), dtype=np.uint64)
    rows[0] = 0
    rows[1] = 2**32 - 1
    text = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
    out = subprocess.run([str(exe)], input=text, capture_output=True, text=True, check=True)
    ref = np.array([[int(v) for v in line.split()] for line in out.stdout.strip().splitlines()],
                   dtype=np.uint64)
    for r, want in zip(rows, ref):
        got = orc.philox([r[2], r[3], r[4], r[5]], [r[0], r[1]])
        assert np.array_equal(got.astype(np.uint64), want), (r, got, want)


def test_u01_exact_cells(orc):
    # u = (2k + 1) / 2^53 with k the 52-bit integer built from the top 26 bits
    # of each word: the extremes and one interior cell are exact.
    assert orc.u01(0, 0) == 2.0 ** -53
    assert orc.u01(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    assert orc.u01(1 << 6, 0) == (2 * (1 << 26) + 1) * 2.0 ** -53
    assert orc.u01(0, 1 << 6) == 3 * 2.0 ** -53
    # the low 6 bits of each word are discarded
    assert orc.u01(0x3F, 0x3F) == orc.u01(0, 0)


def test_move_draw_distributions(orc):
    d = np.array([orc.move_draws(99, 3, s, r, j) for s in range(4) for r in range(50)
                  for j in range(40)])
    assert d.shape == (8000, 8)
    for c in range(4):
        assert stats.kstest(d[:, c], "uniform").pvalue > 1e-3
        assert 0.0 < d[:, c].min() and d[:, c].max() < 1.0
    assert stats.kstest(d[:, 4], "expon").pvalue > 1e-3
    assert stats.kstest(d[:, 5], "norm").pvalue > 1e-3
    assert stats.kstest(d[:, 6], "norm").pvalue > 1e-3
    assert abs(np.corrcoef(d[:, 5], d[:, 6])[0, 1]) < 0.05
    assert stats.kstest(np.exp(d[:, 7]), "uniform").pvalue > 1e-3
    # different counters give different streams; same counter gives the same
    assert not np.array_equal(orc.move_draws(1, 0, 0, 0, 0), orc.move_draws(1, 0, 0, 0, 1))
    assert np.array_equal(orc.move_draws(1, 0, 5, 7, 9), orc.move_draws(1, 0, 5, 7, 9))


def test_offset_uniform_on_region_width(orc):
    offs = np.array([orc.offset(5, 0, s, 0.2, 0.25) for s in range(4000)])
    assert (offs[:, 0] >= 0).all() and (offs[:, 0] < 0.2).all()
    assert (offs[:, 1] >= 0).all() and (offs[:, 1] < 0.25).all()
    assert stats.kstest(offs[:, 0] / 0.2, "uniform").pvalue > 1e-3
    assert stats.kstest(offs[:, 1] / 0.25, "uniform").pvalue > 1e-3
