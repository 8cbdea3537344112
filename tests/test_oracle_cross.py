"""Pins of the two-input (cross) oracle, Sec. 4 Eq. (11) with lags of either sign.

* closed form: for x = a exp(j2pi f n), y = b exp(j2pi g n) and the y-referenced
  phase, R[m, alpha] = a conj(b) exp(j2pi f m) exp(-j2pi nu dy) D_N(nu) with
  nu = alpha - f + g, and Rc = a b exp(j2pi f m) exp(-j2pi nu' dy) D_N(nu') with
  nu' = alpha - f - g, where D_N(nu) = (1/N) sum_{n<N} exp(-j2pi nu n) =
  exp(-j pi nu (N-1)) sin(pi nu N) / (N sin(pi nu)) and dy = max(0, -lag_min);
* a delayed copy: y[k] = x[k - d] and lags -d .. -d+T-1 give
  exp(-j2pi alpha d) times the single-input tables of x (lags 0 .. T-1);
* y = x with lag_min = 0 reduces to the single-input oracle.
"""
import numpy as np

from oracle.cyclic import cross_tables, cyclic_tables


def _dirichlet(nu, N):
    nu = np.asarray(nu, dtype=np.float64)
    out = np.empty(nu.shape, dtype=np.complex128)
    s = np.sin(np.pi * nu)
    near = np.abs(s) < 1e-12
    out[near] = np.exp(-1j * np.pi * nu[near] * (N - 1)) * np.cos(np.pi * nu[near] * (N - 1))
    out[~near] = np.exp(-1j * np.pi * nu[~near] * (N - 1)) * np.sin(np.pi * nu[~near] * N) / (N * s[~near])
    return out


def test_two_tones_closed_form_any_lag_range():
    L = 777
    n = np.arange(L)
    a, b = 0.7 - 0.2j, -0.4 + 0.9j
    f, g = 0.0831, -0.2113
    x = a * np.exp(2j * np.pi * f * n)
    y = b * np.exp(2j * np.pi * g * n)
    alphas = np.array([0.0, f - g, f + g, 0.3, -0.41, f - g + 1.0 / 512])
    for lag_min, T in ((-5, 11), (0, 4), (3, 6), (-9, 3)):
        R, Rc, N = cross_tables(x, y, alphas, lag_min, T)
        dy = max(0, -lag_min)
        assert N == L - (T - 1) - abs(lag_min)
        for t in range(T):
            m = t + lag_min
            nu = alphas - f + g
            nuc = alphas - f - g
            ref = a * np.conj(b) * np.exp(2j * np.pi * f * m) * np.exp(-2j * np.pi * nu * dy) * _dirichlet(nu, N)
            refc = a * b * np.exp(2j * np.pi * f * m) * np.exp(-2j * np.pi * nuc * dy) * _dirichlet(nuc, N)
            assert np.max(np.abs(R[t] - ref)) < 1e-12
            assert np.max(np.abs(Rc[t] - refc)) < 1e-12


def test_delayed_copy_equals_phase_shifted_autocorrelation():
    rng = np.random.default_rng(4)
    L, d, T = 900, 7, 9
    x = rng.standard_normal(L) + 1j * rng.standard_normal(L)
    y = np.concatenate([np.zeros(d), x[:L - d]])          # y[k] = x[k - d]
    alphas = np.array([0.0, 0.125, -0.3, 0.49, 1.0 / 3.0])
    R, Rc, N = cross_tables(x, y, alphas, -d, T)
    Rs, Rcs, Ns = cyclic_tables(x[:L - d], alphas, T)
    assert N == Ns
    ph = np.exp(-2j * np.pi * alphas * d)[None, :]
    assert np.max(np.abs(R - ph * Rs)) < 1e-12
    assert np.max(np.abs(Rc - ph * Rcs)) < 1e-12


def test_reduces_to_the_single_input_oracle():
    rng = np.random.default_rng(5)
    x = rng.standard_normal(500) + 1j * rng.standard_normal(500)
    alphas = np.linspace(-0.5, 0.5, 17)
    R, Rc, N = cross_tables(x, x, alphas, 0, 6)
    Rs, Rcs, Ns = cyclic_tables(x, alphas, 6)
    assert N == Ns
    assert np.max(np.abs(R - Rs)) < 1e-13 and np.max(np.abs(Rc - Rcs)) < 1e-13


def test_too_short_gives_zero_tables():
    x = np.ones(5, dtype=complex)
    R, Rc, N = cross_tables(x, x, [0.0, 0.1], -3, 4)
    assert N == 0 and not R.any() and not Rc.any()
