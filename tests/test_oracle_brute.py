"""The FP64 oracle against a 50-digit mpmath brute force on tiny inputs (no GPU).

Covers L < T (no products), L = T (one product), rational and non-dyadic
cycle frequencies, and |alpha| > 1.  The bound is the a-priori FP64 rounding
of a length-N complex dot product, a few units of N * 2^-53 times the scale.
"""
import numpy as np
import pytest

from oracle.brute import brute_tables
from oracle.cyclic import cyclic_tables, scale_per_lag


@pytest.mark.parametrize("L,T", [(3, 4), (4, 4), (9, 1), (16, 4), (11, 3)])
def test_against_mpmath(L, T):
    rng = np.random.default_rng(100 + L * 7 + T)
    x = (rng.standard_normal(L) + 1j * rng.standard_normal(L)).astype(np.complex64)
    alphas = [0.0, 0.125, -0.5, 1 / 3, 0.7123456789, 2.25, -0.0001, 0.4999]
    R, Rc, n = cyclic_tables(x, alphas, T, chunk=5)
    Rb, Rcb, nb = brute_tables(x, alphas, T)
    assert n == nb == max(0, L - T + 1)
    if n == 0:
        assert not R.any() and not Rc.any()
        return
    s = scale_per_lag(x, T)
    for t in range(T):
        for j in range(len(alphas)):
            bound = 8 * n * 2.0 ** -53 * max(s[t], 1e-300)
            assert abs(R[t, j] - complex(Rb[t][j])) <= bound
            assert abs(Rc[t, j] - complex(Rcb[t][j])) <= bound
