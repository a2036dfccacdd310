"""The measurement model of bench.py, on the CPU: the algorithmic bytes per
pass launch and the column pass's flop count, against values worked out by
hand from their definitions (each vector read or written once; 5 m log2 m
flops per complex m-point FFT)."""
import math
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


@pytest.mark.parametrize("p,prec,cu,cn", [
    (0, 0, 32, 1),         # z, p_old read; p_new, q written (8 B each) at U; 1-byte mask
    (1, 0, 48, 9),         # F, p, q, r read; F, r written at U; mask; t written (8 B)
    (2, 0, 0, 16),         # t read and written
    (3, 0, 16, 9),         # r read, z written at U; mask; t read
    (1, 1, 48, 5),         # FP32 transforms: 4-byte t
    (2, 1, 0, 8),
])
def test_pass_bytes_per_node(p, prec, cu, cn):
    assert bench.pass_coeffs(p, prec) == (cu, cn)
    assert bench.pass_bytes(p, 1000, 5000, prec) == cu * 1000 + cn * 5000


def test_column_pass_flops():
    # power-of-two side: one forward and one inverse 1024-point FFT per pair
    assert bench.column_pass_flops(1024) == 512 * 2 * 5 * 1024 * 10
    # chirp-z sides: the core is the power of two at least 2n - 1, two FFTs
    # per transform
    assert bench.column_pass_flops(1429) == 715 * 4 * 5 * 4096 * 12
    assert bench.column_pass_flops(1025) == 513 * 4 * 5 * 4096 * 12     # 2n - 1 = 2049
    assert bench.column_pass_flops(153) == 77 * 4 * 5 * 512 * 9
    # a core of exactly 2n - 1 points is never possible (2n - 1 is odd), so
    # the core is always strictly longer than 2n - 2
    for n in range(5, 3000, 37):
        if n & (n - 1):
            m = 1 << (2 * n - 2).bit_length()
            assert m >= 2 * n - 1 and m // 2 < 2 * n - 1
            assert bench.column_pass_flops(n) == (n + 1) // 2 * 4 * 5 * m * math.log2(m)
