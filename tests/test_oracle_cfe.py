"""Pins of the cycle-frequency estimator oracle (oracle/cfe.py), no GPU.

Closed-form locations:
* a complex tone a exp(j2pi f n) has |R_conj^alpha| = |a|^2 |D_N(alpha - 2f)|,
  whose only peak is alpha = 2f, and |R^alpha| = |a|^2 |D_N(alpha)| (the power
  term at alpha = 0, which the non-conjugate table never reports);
* two tones f1, f2 add non-conjugate features at +-(f1 - f2) and conjugate
  ones at 2 f1, 2 f2 and f1 + f2;
* rectangular-pulse BPSK with P samples per symbol on a carrier f0 has
  non-conjugate features at k/P and conjugate ones at 2 f0 + k/P (its
  expected cyclic autocorrelation, nonzero at lag 1 for every k);
* a carrier offset moves the conjugate features by twice the offset and
  leaves the non-conjugate ones in place (Sec. 5);
* complex Gaussian noise alone gives no detection.
Each estimate must sit within three zoom steps (1/(Z A) each) of its closed
form; a planted mistake (no leakage masking) fails the pin of a tone on a
grid twice as fine as 1/N.
"""
import numpy as np
import pytest

from oracle import cfe

N, A, T, Z = 4096, 4096, 4, 16
STEP = 1.0 / (Z * A)


def _wrap(a):
    return (np.asarray(a) + 0.5) % 1.0 - 0.5


def _noise(rng, n, var):
    return (rng.standard_normal(n) + 1j * rng.standard_normal(n)) * np.sqrt(var / 2)


def _match(est, expected, tol=3 * STEP):
    got = sorted(_wrap([a for _, a, _ in est]).tolist())
    exp = sorted(_wrap(expected).tolist())
    assert len(got) == len(exp), (got, exp)
    for g, e in zip(got, exp):
        assert abs(_wrap(g - e)) <= tol, (got, exp)


def test_tone():
    rng = np.random.default_rng(1)
    f = 0.0873
    x = np.exp(2j * np.pi * f * np.arange(N)) + _noise(rng, N, 0.1)
    _match(cfe.estimate(x, T, -0.5, A, Z=Z, which="Rc"), [2 * f])
    assert cfe.estimate(x, T, -0.5, A, Z=Z, which="R") == []


def test_tone_on_an_oversampled_grid():
    # A = 2N samples the Dirichlet kernel's sidelobes: only leakage masking
    # keeps them from being reported as features
    rng = np.random.default_rng(11)
    f = 0.0873
    x = np.exp(2j * np.pi * f * np.arange(N)) + _noise(rng, N, 0.01)
    _match(cfe.estimate(x, T, -0.5, 2 * A, Z=Z, which="Rc"), [2 * f], tol=3 / (Z * 2 * A))


def test_two_tones():
    rng = np.random.default_rng(2)
    f1, f2 = 0.0873, -0.1311
    n = np.arange(N)
    x = np.exp(2j * np.pi * f1 * n) + 0.7 * np.exp(2j * np.pi * f2 * n) + _noise(rng, N, 0.1)
    _match(cfe.estimate(x, T, -0.5, A, Z=Z, which="R"), [f1 - f2, f2 - f1])
    _match(cfe.estimate(x, T, -0.5, A, Z=Z, which="Rc"), [2 * f1, 2 * f2, f1 + f2])


def _rect_bpsk(rng, n, P, f0):
    bits = rng.choice([-1.0, 1.0], size=n // P + 1)
    return np.repeat(bits, P)[:n] * np.exp(2j * np.pi * f0 * np.arange(n))


def test_rect_bpsk_features():
    rng = np.random.default_rng(3)
    P, f0 = 4, 0.0311
    x = _rect_bpsk(rng, N, P, f0) + _noise(rng, N, 0.05)
    _match(cfe.estimate(x, T, -0.5, A, Z=Z, which="R"), [k / P for k in range(1, P)])
    _match(cfe.estimate(x, T, -0.5, A, Z=Z, which="Rc"), [2 * f0 + k / P for k in range(P)])


def test_carrier_offset_moves_only_the_conjugate_features():
    rng = np.random.default_rng(4)
    P, f0 = 4, 0.0311
    x = _rect_bpsk(rng, N, P, f0) + _noise(rng, N, 0.05)
    k0 = 37                                   # offset of k0 / (2A): conjugate features move k0 bins
    y = x * np.exp(2j * np.pi * (k0 / (2 * A)) * np.arange(N))
    rx, ry = cfe.estimate(x, T, -0.5, A, Z=Z, which="R"), cfe.estimate(y, T, -0.5, A, Z=Z, which="R")
    assert [k for k, _, _ in rx] == [k for k, _, _ in ry]
    assert np.allclose([a for _, a, _ in rx], [a for _, a, _ in ry], rtol=0, atol=1e-12)
    cx, cy = cfe.estimate(x, T, -0.5, A, Z=Z, which="Rc"), cfe.estimate(y, T, -0.5, A, Z=Z, which="Rc")
    assert [(k + k0) % A for k, _, _ in cx] == sorted(k for k, _, _ in cy)
    shifted = sorted(_wrap([a + k0 / A for _, a, _ in cx]).tolist())
    assert np.allclose(shifted, sorted(_wrap([a for _, a, _ in cy]).tolist()), rtol=0, atol=1e-12)


@pytest.mark.parametrize("seed", [5, 6, 7])
def test_noise_alone_gives_nothing(seed):
    rng = np.random.default_rng(seed)
    x = _noise(rng, N, 1.0)
    assert cfe.estimate(x, T, -0.5, A, Z=Z, which="R") == []
    assert cfe.estimate(x, T, -0.5, A, Z=Z, which="Rc") == []


def test_scales_and_statistic_by_hand():
    # one lag, 192 bins = three blocks of 64: each block's window is the whole row
    R = np.zeros((1, 192), dtype=np.complex128)
    R[0, :] = np.arange(192) + 1.0
    R[0, 10] = 3 + 4j                           # |.| = 5
    m = np.abs(R[0])
    med = np.median(m)                          # even count: mean of the middle two
    sigma = cfe.scales(R)
    assert sigma.shape == (1, 3) and np.all(sigma == med / np.sqrt(2 * np.log(2)))
    q = cfe.ratios(R, sigma)
    assert q[0, 10] == 5 / sigma[0, 0]
    # candidates: circular local maxima above kappa, first of a plateau
    qq = np.array([0.0, 8.0, 8.0, 1.0, 9.0, 0.5])
    assert cfe.candidates(qq, 7.0).tolist() == [1, 4]
    assert cfe.zero_bin(-0.5, 8) == 4 and cfe.zero_bin(0.25 / 8, 8) is None


def test_leak_factor_bounds_the_dirichlet_kernel():
    # half the factor must cover the kernel's leakage for any feature offset
    # within half a bin of the peak bin, relative to the peak bin's value
    Nn, Aa = 1000, 1024
    nu = np.linspace(-0.5, 0.5, 201) / Aa

    def dk(v):
        v = np.asarray(v, dtype=np.float64)
        out = np.ones_like(v)
        nz = np.abs(np.sin(np.pi * v)) > 0
        out[nz] = np.abs(np.sin(np.pi * v[nz] * Nn) / (Nn * np.sin(np.pi * v[nz])))
        return out

    peak = dk(nu)
    for d in (1, 2, 5, 40, 512):
        leak = np.maximum(dk(d / Aa - nu), dk(-d / Aa - nu))
        assert np.all(leak <= cfe.leak_factor(d, Aa, Nn) / 2 * peak + 1e-15), d


def test_planted_mistake_no_masking_fails_the_tone_pin(monkeypatch):
    monkeypatch.setattr(cfe, "leak_factor", lambda d, A_, N_: 0.0)
    with pytest.raises(AssertionError):
        test_tone_on_an_oversampled_grid()
