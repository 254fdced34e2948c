"""Pins for the sphere T-matrix: an independent textbook Mie implementation
(logarithmic-derivative method), the lossless unitarity relation, the
index-matched limit and the Rayleigh limit."""
import numpy as np
import pytest

from oracle.mie import bohren_huffman_ab, mie_Q


@pytest.mark.parametrize("x,m", [(0.3, 1.5), (1.142, 1.5 + 0.01j), (1.714, 1.52), (5.0, 1.33 + 0.1j),
                                 (12.0, 2.0 + 0.5j), (0.8, 0.6 + 0.2j)])
def test_paper_formula_matches_textbook_series(x, m):
    L = 12
    k = 2 * np.pi / 550
    R = x / k
    Q = mie_Q(L, k, R, m)
    a, b = bohren_huffman_ab(L, x, m)
    # a_l = -Q_2l, b_l = -Q_1l
    assert np.allclose(-Q[1], a, rtol=1e-10, atol=1e-15)
    assert np.allclose(-Q[0], b, rtol=1e-10, atol=1e-15)


def test_lossless_unitarity_and_matched_index():
    k = 1.0
    for x in (0.4, 1.7, 4.0):
        Q = mie_Q(8, k, x, 1.52)
        assert np.allclose(np.real(Q), -np.abs(Q) ** 2, atol=1e-14)
        Q0 = mie_Q(8, k, x, 1.0)
        assert np.abs(Q0).max() < 1e-14


def test_rayleigh_limit():
    m = 1.5 + 0.1j
    for x in (1e-3, 1e-2):
        Q = mie_Q(3, 1.0, x, m)
        want = 2j / 3 * x ** 3 * (m * m - 1) / (m * m + 2)
        assert abs(Q[1, 0] - want) <= 1e-2 * x * x * abs(want) * 100
        assert abs(Q[0, 0]) < 10 * x ** 5
