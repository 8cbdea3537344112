"""Pins of the FP64 oracle against closed forms (no GPU).

Each expected value below is derived by hand from the estimator's definition
(Sec. 4, Eq. (11) with x = y and lag t >= 0; conjugate form per Sec. 2,
Eq. (9)) for signals whose cyclic statistics are known exactly, and evaluated
independently of the oracle (mpmath Dirichlet kernels, textbook sums):

* sums of complex tones: every (i, k) tone pair contributes a Dirichlet kernel
  at alpha = f_i - f_k (non-conjugate) or alpha = f_i + f_k (conjugate); a
  dropped cross term, a wrong sign of the exponent, a lag on the wrong sample,
  a wrong phase origin or a wrong normalisation count each changes the value;
* rectangular-pulse BPSK: the expected cyclic ACF/CCF at alpha = k/P (and
  2 f0 + k/P) is a finite geometric sum; the estimator is consistent (Sec. 2),
  so the estimate lies within a few standard deviations of it.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle.cyclic import cyclic_tables
from paper_2405_16911_amd import siggen


def dirichlet(nu: float, N: int) -> complex:
    """D_N(nu) = (1/N) sum_{n<N} exp(-j 2 pi nu n), closed form, 40 digits.

    D_N(nu) = exp(-j pi nu (N-1)) sin(pi nu N) / (N sin(pi nu)), and 1 when
    nu is an integer (every term equals 1).
    """
    with mp.workdps(40):
        v = mp.mpf(nu)
        if abs(v - mp.nint(v)) < mp.mpf(10) ** -25:
            return 1.0 + 0j
        val = mp.expjpi(-v * (N - 1)) * mp.sin(mp.pi * v * N) / (N * mp.sin(mp.pi * v))
        return complex(val)


def tone_signal(n, freqs, amps):
    """Tone sum evaluated at 40 digits, then rounded once to complex128."""
    out = np.empty(n, dtype=np.complex128)
    with mp.workdps(40):
        fs = [mp.mpf(f) for f in freqs]
        for i in range(n):
            acc = mp.mpc(0)
            for f, a in zip(fs, amps):
                acc += mp.mpc(a.real, a.imag) * mp.expjpi(2 * f * i)
            out[i] = complex(acc)
    return out


def expected_tone_tables(freqs, amps, alphas, T, N):
    R = np.zeros((T, len(alphas)), dtype=np.complex128)
    Rc = np.zeros_like(R)
    for t in range(T):
        for j, a in enumerate(alphas):
            s = 0j
            sc = 0j
            for fi, ai in zip(freqs, amps):
                lagph = complex(mp.expjpi(2 * mp.mpf(fi) * t))
                for fk, ak in zip(freqs, amps):
                    s += ai * np.conj(ak) * lagph * dirichlet(float(mp.mpf(a) - (mp.mpf(fi) - mp.mpf(fk))), N)
                    sc += ai * ak * lagph * dirichlet(float(mp.mpf(a) - (mp.mpf(fi) + mp.mpf(fk))), N)
            R[t, j] = s
            Rc[t, j] = sc
    return R, Rc


def test_single_tone_closed_form():
    f = 0.0371
    a = 0.8 * np.exp(0.3j)
    T, L = 5, 700
    N = L - T + 1
    alphas = [0.0, 2 * f, f, -0.25, 0.5, 2 * f + 1.0 / N, 0.3333]
    x = tone_signal(L, [f], [a])
    R, Rc, n_used = cyclic_tables(x, alphas, T)
    assert n_used == N
    Re, Rce = expected_tone_tables([f], [a], alphas, T, N)
    assert np.max(np.abs(R - Re)) < 1e-12
    assert np.max(np.abs(Rc - Rce)) < 1e-12
    # alpha = 0: |a|^2 exp(j 2 pi f t) exactly; conjugate feature at alpha = 2f.
    t = np.arange(T)
    assert np.allclose(R[:, 0], abs(a) ** 2 * np.exp(2j * np.pi * f * t), atol=1e-12)
    assert np.allclose(Rc[:, 1], a * a * np.exp(2j * np.pi * f * t), atol=1e-12)


def test_three_tones_cross_terms():
    freqs = [0.05, -0.1234, 0.31]
    amps = [1.0 + 0j, 0.5 * np.exp(1.1j), 0.25 * np.exp(-2.0j)]
    T, L = 6, 517
    N = L - T + 1
    # Non-conjugate features at f_i - f_k, conjugate at f_i + f_k, plus off-feature cells.
    alphas = sorted({round(fi - fk, 12) for fi in freqs for fk in freqs}
                    | {round(fi + fk, 12) for fi in freqs for fk in freqs} | {0.0117, -0.4})
    x = tone_signal(L, freqs, amps)
    R, Rc, n_used = cyclic_tables(x, alphas, T, chunk=128)
    Re, Rce = expected_tone_tables(freqs, amps, alphas, T, N)
    assert np.max(np.abs(R - Re)) < 1e-12
    assert np.max(np.abs(Rc - Rce)) < 1e-12


def test_tone_distinguishes_conventions():
    """A lag on the trailing sample or a +j exponent gives a different value."""
    f = 0.1
    T, L = 4, 300
    x = tone_signal(L, [f], [1.0 + 0j])
    R, Rc, _ = cyclic_tables(x, [0.0, 0.2], T)
    t = np.arange(T)
    # lag on the leading sample: exp(+j 2 pi f t); the other convention would be exp(-j 2 pi f t)
    assert np.allclose(R[:, 0], np.exp(2j * np.pi * f * t), atol=1e-12)
    assert not np.allclose(R[1:, 0], np.exp(-2j * np.pi * f * t[1:]), atol=1e-3)
    # conjugate feature at +2f with exp(-j 2 pi alpha n) sign convention
    assert np.allclose(Rc[:, 1], np.exp(2j * np.pi * f * t), atol=1e-12)
    _, Rc_neg, _ = cyclic_tables(x, [-0.2], T)
    assert np.max(np.abs(Rc_neg)) < 0.05


@pytest.mark.parametrize("f0", [0.0, 0.0125])
def test_rect_bpsk_expected_value(f0):
    """E[R^{k/P}(t)] = exp(j 2 pi f0 t) (1/P) sum_{r=0}^{P-1-t} exp(-j 2 pi k r / P)."""
    P, L, T = 8, 1 << 20, 8
    rng = siggen.rng_for(1234, 0)
    theta = float(rng.uniform(0, 2 * np.pi))
    x = siggen.rect_bpsk(L, P, rng) * np.exp(1j * (2 * np.pi * f0 * np.arange(L) + theta))
    ks = [0, 1, 2, 3]
    acf_alphas = [k / P for k in ks] + [0.5 / P, 2.5 / P]
    ccf_alphas = [2 * f0 + k / P for k in ks] + [2 * f0 + 1.5 / P]
    R, _, N = cyclic_tables(x, acf_alphas, T, chunk=1 << 16)
    _, Rc, _ = cyclic_tables(x, ccf_alphas, T, chunk=1 << 16)
    for t in range(T):
        sigma = min(t, P) / math.sqrt(N * P)
        tol = 6 * sigma + 2 * P / N
        lagph = np.exp(2j * np.pi * f0 * t)
        for j, k in enumerate(ks):
            geo = sum(np.exp(-2j * np.pi * k * r / P) for r in range(P - t)) / P
            assert abs(R[t, j] - lagph * geo) < tol, (t, k)
            assert abs(Rc[t, j] - np.exp(2j * theta) * lagph * geo) < tol, (t, k)
        # off the cycle-frequency set the expected value is zero
        assert abs(R[t, len(ks)]) < tol and abs(R[t, len(ks) + 1]) < tol
        assert abs(Rc[t, len(ks)]) < tol
