"""Pins of the cyclic-spectrum oracle (cyclic Wiener-Khinchin over a lag table).

* closed form: a complex exponential x = a exp(j2pi f0 n) has R[m, alpha] =
  |a|^2 exp(j2pi f0 m) D_N(alpha); with the rectangular window over lags
  -M..M the spectrum is |a|^2 D_N(alpha) K(alpha/2 + f - f0), where
  K(theta) = sum_{|m|<=M} exp(-j2pi theta m) = sin(pi theta (2M+1)) / sin(pi theta),
  so at alpha = 0 it peaks at f = f0 with height (2M+1) |a|^2;
* alpha = 0 with symmetric lags is the Blackman-Tukey spectrum: a real,
  even-in-m Hermitian autocorrelation gives a real spectrum;
* the Hann window of a one-lag table (m = 0) is 1.
"""
import numpy as np

from oracle.cyclic import cross_tables, cyclic_spectrum, lag_window


def _K(theta, M):
    theta = np.asarray(theta, dtype=np.float64)
    s = np.sin(np.pi * theta)
    out = np.full(theta.shape, 2.0 * M + 1.0)
    nz = np.abs(s) > 1e-12
    out[nz] = np.sin(np.pi * theta[nz] * (2 * M + 1)) / s[nz]
    return out


def test_tone_closed_form():
    L, M, F = 3000, 12, 64
    f0 = 5 / 64 + 0.003
    a = 0.8 + 0.3j
    n = np.arange(L)
    x = a * np.exp(2j * np.pi * f0 * n)
    alphas = np.array([0.0, 0.02, -0.11])
    R, _, N = cross_tables(x, x, alphas, -M, 2 * M + 1)
    S = cyclic_spectrum(R, alphas, -M, F, "rect")
    f = -0.5 + np.arange(F) / F
    dy = M
    for j, al in enumerate(alphas):
        nu = al
        D = np.exp(-2j * np.pi * nu * dy) * np.mean(np.exp(-2j * np.pi * nu * np.arange(N)))
        ref = abs(a) ** 2 * D * _K(al / 2 + f - f0, M)
        assert np.max(np.abs(S[:, j] - ref)) < 1e-10
    k0 = int(np.argmax(np.abs(S[:, 0])))
    assert abs(f[k0] - f0) <= 0.5 / F
    assert abs(np.max(np.abs(S[:, 0])) - (2 * M + 1) * abs(a) ** 2) < 0.2 * (2 * M + 1) * abs(a) ** 2


def test_alpha_zero_symmetric_lags_is_real():
    rng = np.random.default_rng(3)
    x = rng.standard_normal(5000) + 1j * rng.standard_normal(5000)
    M = 20
    R, _, _ = cross_tables(x, x, [0.0], -M, 2 * M + 1)
    # over a matched index range R(-m) = conj(R(m)) only up to edge terms; symmetrise
    Rh = 0.5 * (R[:, 0] + np.conj(R[::-1, 0]))
    S = cyclic_spectrum(Rh[:, None], [0.0], -M, 128, "hann")
    assert np.max(np.abs(S.imag)) < 1e-12 * np.max(np.abs(S))


def test_hann_window():
    assert lag_window([0], "hann")[0] == 1.0
    w = lag_window(np.arange(-4, 5), "hann")
    assert np.allclose(w, w[::-1]) and w[4] == 1.0 and np.all(w > 0)
