"""The oracle reproduces the cycle-frequency locations the paper states (no GPU).

Sec. 3: a CPM signal is cyclostationary at alpha = k/T; for h = 1/2 (GMSK) it
is also conjugate-cyclostationary at beta = 1/(2T) + k/T, and for
h != 1/2 + k the conjugate statistics vanish.  Sec. 5, Table 1 and
experiments #1/#2: at 8 samples/symbol these are the normalised values
0.125 (cyclic ACF) and 0.0625 (cyclic CCF).  Sec. 5 also notes that a
carrier offset leaves the cyclic ACF alone but moves the conjugate cycle
frequency.  Magnitudes are not pinned: the paper's theoretical curves
(Figs. 1-2) are images only ("parity unpinned" for magnitudes).
"""
import json
import os

import numpy as np
import pytest

from oracle.cyclic import cyclic_tables
from paper_2405_16911_amd import siggen

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_table1.json")))
SPS = GOLDEN["samples_per_symbol"]
BT = GOLDEN["bt"]
A = 256
ALPHAS = np.arange(A) / A - 0.5


def _gmsk(h, f0, seed, n=1 << 16, snr=10.0):
    rng = siggen.rng_for(seed, 0)
    x = siggen.gmsk(n, sps=SPS, bt=BT, h=h, rng=rng)
    return siggen.apply_cfo(siggen.add_awgn(x, snr, rng), f0)


def _z(tab):
    m = np.abs(tab)
    return m / (np.median(m, axis=1, keepdims=True) / 1.1774)


def _bin(a):
    return int(round((a + 0.5) * A)) % A


def test_table1_values_follow_from_symbol_rate():
    assert GOLDEN["sample_rate_hz"] == GOLDEN["baud_rate_hz"] * SPS
    assert GOLDEN["exp1_acf_alpha_normalised"] == 1.0 / SPS
    assert GOLDEN["exp2_ccf_beta_normalised"] == 1.0 / (2 * SPS)


def test_exp2_conjugate_feature_at_half_symbol_rate():
    beta = GOLDEN["exp2_ccf_beta_normalised"]
    _, Rc, _ = cyclic_tables(_gmsk(0.5, 0.0, seed=21), ALPHAS, 16, chunk=8192)
    z = _z(Rc)
    for b in (beta, -beta):
        assert np.all(z[:10, _bin(b)] > 50) and np.all(z[:, _bin(b)] > 20)
    mask = np.ones(A, bool)
    mask[[_bin(beta), _bin(-beta)]] = False
    assert z[:10, _bin(beta)].min() > 4 * z[:10, mask].max()


def test_exp1_acf_feature_at_symbol_rate():
    alpha = GOLDEN["exp1_acf_alpha_normalised"]
    x = _gmsk(0.5, 0.0, seed=22, n=1 << 17)
    feat = [alpha, -alpha]
    off = [0.0625, 0.1, 0.3, 0.25, -0.2, 0.4375]
    R, _, _ = cyclic_tables(x, feat + off, 16, chunk=1 << 15)
    m = np.abs(R)
    lags = slice(6, 15)
    assert m[lags, 0].max() > 2.5 * m[lags, 2:].max()
    assert m[lags, 1].max() > 2.5 * m[lags, 2:].max()
    # constant envelope: no feature at lag 0 beyond the noise level
    assert m[0, 0] < 0.3 * m[lags, 0].max()


def test_proper_cpm_has_no_conjugate_feature():
    _, Rc_half, _ = cyclic_tables(_gmsk(0.5, 0.0, seed=23), ALPHAS, 8, chunk=8192)
    _, Rc_07, _ = cyclic_tables(_gmsk(0.7, 0.0, seed=23), ALPHAS, 8, chunk=8192)
    assert _z(Rc_half).max() > 100
    assert _z(Rc_07).max() < 25


def test_carrier_offset_shifts_conjugate_but_not_acf():
    f0 = 3.0 / A                    # 2 f0 on the grid
    beta = GOLDEN["exp2_ccf_beta_normalised"]
    R0, Rc0, _ = cyclic_tables(_gmsk(0.5, 0.0, seed=24), ALPHAS, 8, chunk=8192)
    R1, Rc1, _ = cyclic_tables(_gmsk(0.5, f0, seed=24), ALPHAS, 8, chunk=8192)
    assert np.max(np.abs(np.abs(R1) - np.abs(R0))) < 1e-9
    z1 = _z(Rc1)
    for b in (2 * f0 + beta, 2 * f0 - beta):
        assert np.all(z1[:, _bin(b)] > 50)
    assert _z(Rc1)[:, _bin(beta)].max() < 25
