"""The FP32/FP64 distance-marginalization rule's node table (the kernel
header's 24-point Gauss-Legendre rule) against numpy's, CPU only."""
import os
import re

import numpy as np

HDR = os.path.join(os.path.dirname(__file__), "..", "paper_2210_07912_amd", "csrc", "dmarg.h")


def _table(name):
    src = open(HDR).read()
    m = re.search(r"constexpr double " + name + r"\[\d+\] = \{([^}]*)\}", src)
    assert m, name
    return np.array([float(v) for v in m.group(1).replace("\n", " ").split(",")])


def test_gauss_legendre_table_matches_numpy():
    x, w = np.polynomial.legendre.leggauss(24)
    half_x, half_w = _table("kDmNode"), _table("kDmWeight")
    assert np.abs(np.r_[-half_x[::-1], half_x] - x).max() < 1e-15
    assert np.abs(np.r_[half_w[::-1], half_w] - w).max() < 1e-15
    assert abs(w.sum() - 2.0) < 1e-14
