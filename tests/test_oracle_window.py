"""Pins of the sliding-window oracle.

For a tone x = a exp(j2pi f n) and the window-start phase reference, the
conjugate table over the window n_w .. n_w + N_w - 1 is
  Rc[t, alpha] = a^2 exp(j2pi f t) exp(j4pi f n_w) D_{N_w}(alpha - 2f),
so it pins both the window's position and the re-referencing; the
non-conjugate table |a|^2 exp(j2pi f t) D_{N_w}(alpha) does not depend on n_w.
"""
import numpy as np

from oracle.cyclic import window_tables


def _D(nu, N):
    return np.mean(np.exp(-2j * np.pi * np.asarray(nu)[..., None] * np.arange(N)), axis=-1)


def test_tone_window_position_and_phase_reference():
    a, f = 0.9 - 0.4j, 0.0371
    T, hop, W = 5, 64, 3
    alphas = np.array([0.0, 2 * f, 2 * f + 1 / 192, 0.3])
    for L in (60, 64 + T - 1, 5 * 64 + 17 + T - 1, 9 * 64 + T - 1):
        x = a * np.exp(2j * np.pi * f * np.arange(L))
        R, Rc, Nw = window_tables(x, alphas, T, hop, W)
        c = max(0, L - T + 1) // hop
        Wn = min(W, c)
        assert Nw == Wn * hop
        if Wn == 0:
            assert not R.any() and not Rc.any()
            continue
        n_w = (c - Wn) * hop
        for t in range(T):
            ref = abs(a) ** 2 * np.exp(2j * np.pi * f * t) * _D(alphas, Nw)
            refc = a * a * np.exp(2j * np.pi * f * t) * np.exp(4j * np.pi * f * n_w) * _D(alphas - 2 * f, Nw)
            assert np.max(np.abs(R[t] - ref)) < 1e-12
            assert np.max(np.abs(Rc[t] - refc)) < 1e-12
