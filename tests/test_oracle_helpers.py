"""Pins of the oracle's helper functions (no GPU).

Each helper is checked against something other than itself: hand-summed
values, a closed form, or an independent library routine (SciPy, PyTorch).
A planted mistake in the oracle (monkeypatched on the CPU) shows that each
pin actually bites.

* ``scale_per_lag`` (the denominator of every scaled-error bound):
  s_t = (1/N_used) sum_n |x[n+t]| |x[n]| is exactly 1 for any unit-modulus
  signal, matches a hand-summed four-sample case, and bounds |R^0(t)|.
* ``welch_log_spectra`` (the proposal's features): equals
  ``scipy.signal.welch`` (periodic Hann window, non-overlapping segments of
  1024, no detrending, two-sided) after the same shift, log and
  standardisation, on noise, on tones and on a constant-modulus signal whose
  empty bins pin the log offset.
* ``lag_window('hann')`` (the cyclic spectrum's lag window): hand values at
  M = 3 and SciPy's symmetric Hann window of length 2M + 3 without its zero
  end points.
* ``roundoff_ratio_per_lag`` (the random-walk factor of the reduced-precision
  bounds): 1/sqrt(N_used) for constant modulus, a hand-summed case, and the
  root-mean-square error of simulated independent roundings.
* ``adamw_step``: ``torch.optim.AdamW`` in float64 over several steps (bias
  correction at t >= 2, decoupled weight decay).
* ``bce_loss``: ``torch.nn.functional.binary_cross_entropy_with_logits``.
"""
import numpy as np
import pytest
import scipy.signal
import torch

from oracle import cyclic as C
from oracle import proposal as P

# ----------------------------------------------------------------------------- roundoff_ratio_per_lag


def test_roundoff_ratio_constant_modulus_is_inverse_sqrt_n():
    rng = np.random.default_rng(13)
    x = 2.5 * np.exp(2j * np.pi * rng.random(1000))
    r = C.roundoff_ratio_per_lag(x, 7)
    assert np.max(np.abs(r * np.sqrt(1000 - 7 + 1) - 1.0)) < 1e-14


def test_roundoff_ratio_hand_summed():
    # |x| = 1, 2, 3, 4; T = 2 -> N_used = 3
    x = np.array([1.0, 2j, -3.0, 4.0 + 0j])
    r = C.roundoff_ratio_per_lag(x, 2)
    assert r[0] == pytest.approx(np.sqrt(1 + 16 + 81) / (1 + 4 + 9), rel=1e-15)
    assert r[1] == pytest.approx(np.sqrt(4 + 36 + 144) / (2 + 6 + 12), rel=1e-15)
    assert C.roundoff_ratio_per_lag(x, 5).tolist() == [0.0] * 5


def test_roundoff_ratio_predicts_a_simulated_random_rounding():
    # relative errors uniform in +-u on each component of each product: the
    # scaled error of the sum has root mean square u * sqrt(2/3) * r_t
    rng = np.random.default_rng(14)
    x = (rng.standard_normal(4000) + 1j * rng.standard_normal(4000)) * (0.5 + rng.random(4000))
    T, u = 3, 2.0 ** -8
    r = C.roundoff_ratio_per_lag(x, T)
    N = x.size - T + 1
    for t in range(T):
        p = x[t: t + N] * np.conj(x[:N])
        w = np.exp(-2j * np.pi * 0.137 * np.arange(N))
        q = p * w
        errs = []
        for _ in range(400):
            d = q.real * rng.uniform(-u, u, N) + 1j * q.imag * rng.uniform(-u, u, N)
            errs.append(abs(d.sum()) / np.abs(p).sum())
        rms = np.sqrt(np.mean(np.square(errs)))
        # uniform relative errors: E d^2 = u^2 |q|^2 / 3, i.e. sqrt(1/3) per rounding
        assert rms == pytest.approx(u * np.sqrt(1 / 3) * r[t], rel=0.15)


# ----------------------------------------------------------------------------- scale_per_lag


def test_scale_per_lag_unit_modulus_is_one():
    rng = np.random.default_rng(11)
    x = np.exp(2j * np.pi * rng.random(777))
    s = C.scale_per_lag(x, 9)
    assert np.max(np.abs(s - 1.0)) < 1e-15


def test_scale_per_lag_hand_summed():
    # |x| = 1, 2, 3, 4; T = 2 -> N_used = 3
    x = np.array([1.0, 2j, -3.0, 4.0 + 0j])
    s = C.scale_per_lag(x, 2)
    assert s[0] == pytest.approx((1 + 4 + 9) / 3, rel=1e-15)            # |x0|^2 + |x1|^2 + |x2|^2
    assert s[1] == pytest.approx((2 * 1 + 3 * 2 + 4 * 3) / 3, rel=1e-15)  # |x1||x0| + |x2||x1| + |x3||x2|
    s3 = C.scale_per_lag(x, 3)                                           # N_used = 2
    assert s3.tolist() == pytest.approx([(1 + 4) / 2, (2 + 6) / 2, (3 + 8) / 2], rel=1e-15)
    assert C.scale_per_lag(x, 5).tolist() == [0.0] * 5                   # N_used = 0


def test_scale_per_lag_bounds_the_alpha_zero_row():
    rng = np.random.default_rng(12)
    x = (rng.standard_normal(3000) + 1j * rng.standard_normal(3000)) * (1 + rng.random(3000))
    T = 6
    R, Rc, _ = C.cyclic_tables(x, [0.0, 0.21], T)
    s = C.scale_per_lag(x, T)
    assert np.all(np.abs(R) <= s[:, None] * (1 + 1e-12))
    assert np.all(np.abs(Rc) <= s[:, None] * (1 + 1e-12))
    # lag 0 of the alpha = 0 row is the mean power, which is exactly s_0
    assert abs(R[0, 0] - s[0]) < 1e-12 * s[0]


def test_scale_per_lag_planted_mistakes_fail():
    x = np.array([1.0, 2j, -3.0, 4.0 + 0j])

    def no_normalisation(x, T):
        a = np.abs(np.asarray(x).astype(np.complex128))
        N = max(0, a.size - T + 1)
        return np.array([np.dot(a[t: t + N], a[:N]) for t in range(T)])

    def lag_on_both(x, T):
        a = np.abs(np.asarray(x).astype(np.complex128))
        N = max(0, a.size - T + 1)
        return np.array([np.dot(a[t: t + N], a[t: t + N]) / N for t in range(T)])

    for bad in (no_normalisation, lag_on_both):
        s = bad(x, 2)
        assert not (abs(s[0] - 14 / 3) < 1e-12 and abs(s[1] - 20 / 3) < 1e-12)


# ----------------------------------------------------------------------------- Welch spectra


def _scipy_features(x, nseg=64, nfft=1024, eps=1e-12):
    x = np.asarray(x).astype(np.complex128)[: nseg * nfft]
    out = np.empty((3, nfft))
    for c, v in enumerate((x, x * x, (np.abs(x) ** 2).astype(np.complex128))):
        _, Pw = scipy.signal.welch(v, fs=1.0, window="hann", nperseg=nfft, noverlap=0, nfft=nfft,
                                   detrend=False, return_onesided=False, scaling="spectrum",
                                   average="mean")
        # 'spectrum' scaling divides the averaged |FFT|^2 by (sum of the window)^2
        w = scipy.signal.get_window("hann", nfft)
        Pw = Pw * np.sum(w) ** 2
        L = np.log(np.fft.fftshift(Pw) + eps)
        out[c] = (L - L.mean()) / L.std()
    return out


def _signals():
    rng = np.random.default_rng(21)
    n = np.arange(64 * 1024)
    noise = (rng.standard_normal(n.size) + 1j * rng.standard_normal(n.size)) / np.sqrt(2)
    tones = 0.7 * np.exp(2j * np.pi * 0.1234 * n) + 0.2 * np.exp(2j * np.pi * (-0.31) * n) + 0.1 * noise
    unit = np.exp(2j * np.pi * (37 / 1024) * n)    # |x|^2 = 1: only the DC bins are non-zero
    return {"noise": noise, "tones": tones, "unit_modulus": unit}


@pytest.mark.parametrize("name", ["noise", "tones", "unit_modulus"])
def test_welch_log_spectra_match_scipy(name):
    x = _signals()[name]
    ours = P.welch_log_spectra(x)
    ref = _scipy_features(x)
    assert np.max(np.abs(ours - ref)) < 1e-9


def test_welch_planted_mistakes_fail(monkeypatch):
    x = _signals()["tones"]
    ref = _scipy_features(x)
    # a symmetric instead of periodic window
    monkeypatch.setattr(P, "hann", lambda n: 0.5 - 0.5 * np.cos(2.0 * np.pi * np.arange(n) / (n - 1)))
    assert np.max(np.abs(P.welch_log_spectra(x) - ref)) > 1e-6
    monkeypatch.undo()
    # another log offset shows in the empty bins of a constant-modulus signal
    u = _signals()["unit_modulus"]
    assert np.max(np.abs(P.welch_log_spectra(u, eps=1e-9) - _scipy_features(u))) > 1e-3
    # segments overlapped by half instead of disjoint
    xs = x[: 64 * 1024]
    _, Pw = scipy.signal.welch(xs, window="hann", nperseg=1024, noverlap=512, detrend=False,
                               return_onesided=False, scaling="spectrum")
    Lh = np.log(np.fft.fftshift(Pw) * np.sum(scipy.signal.get_window("hann", 1024)) ** 2 + 1e-12)
    assert np.max(np.abs((Lh - Lh.mean()) / Lh.std() - P.welch_log_spectra(x)[0])) > 1e-6


# ----------------------------------------------------------------------------- lag window


def test_hann_lag_window_hand_values():
    w = C.lag_window(np.arange(-3, 4), "hann")     # M = 3: w(m) = (1 + cos(pi m / 4)) / 2
    r2 = np.sqrt(2.0) / 2
    ref = [(1 - r2) / 2, 0.5, (1 + r2) / 2, 1.0, (1 + r2) / 2, 0.5, (1 - r2) / 2]
    assert np.max(np.abs(w - np.array(ref))) < 1e-15


@pytest.mark.parametrize("lag_min,T", [(-3, 7), (-5, 11), (-2, 7), (0, 9)])
def test_hann_lag_window_is_scipy_symmetric_hann(lag_min, T):
    m = lag_min + np.arange(T)
    M = int(np.max(np.abs(m)))
    full = scipy.signal.windows.hann(2 * M + 3, sym=True)[1:-1]   # lags -M-1 .. M+1 without the zeros
    ref = full[m + M]
    assert np.max(np.abs(C.lag_window(m, "hann") - ref)) < 1e-15
    assert np.all(C.lag_window(m, "rect") == 1.0)


# ----------------------------------------------------------------------------- AdamW and BCE


def test_adamw_matches_torch_over_several_steps():
    rng = np.random.default_rng(31)
    shapes = {"a": (5,), "b": (3, 4)}
    p = {k: rng.standard_normal(s) for k, s in shapes.items()}
    m = {k: np.zeros(s) for k, s in shapes.items()}
    v = {k: np.zeros(s) for k, s in shapes.items()}
    tp = [torch.tensor(p[k].copy(), dtype=torch.float64, requires_grad=True) for k in shapes]
    lr, wd = 3e-2, 0.1
    opt = torch.optim.AdamW(tp, lr=lr, betas=(0.9, 0.999), eps=1e-8, weight_decay=wd)
    for t in range(1, 8):
        g = {k: rng.standard_normal(s) * (0.1 + t) for k, s in shapes.items()}
        P.adamw_step(p, g, m, v, t, lr=lr, wd=wd)
        for tt, k in zip(tp, shapes):
            tt.grad = torch.tensor(g[k], dtype=torch.float64)
        opt.step()
        for tt, k in zip(tp, shapes):
            assert np.max(np.abs(tt.detach().numpy() - p[k])) < 1e-13 * (1 + np.max(np.abs(p[k])))


def test_adamw_planted_mistake_fails():
    # bias correction dropped from the second moment: identical at t = 1 for
    # equal gradients only through the first step, different afterwards
    rng = np.random.default_rng(32)
    p0 = rng.standard_normal(4)
    tp = torch.tensor(p0.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.AdamW([tp], lr=1e-2, weight_decay=0.01)
    p, m, v = p0.copy(), np.zeros(4), np.zeros(4)
    for t in range(1, 4):
        g = rng.standard_normal(4)
        m = 0.9 * m + 0.1 * g
        v = 0.999 * v + 0.001 * g * g
        p = p - 1e-2 * (m / (1 - 0.9 ** t) / (np.sqrt(v) + 1e-8) + 0.01 * p)
        tp.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
    assert np.max(np.abs(tp.detach().numpy() - p)) > 1e-6


def test_bce_loss_matches_torch():
    rng = np.random.default_rng(41)
    z = rng.standard_normal((5, 37)) * 6.0
    z[0, :4] = [40.0, -40.0, 0.0, 700.0]
    y = (rng.random((5, 37)) < 0.3).astype(np.float64)
    ref = torch.nn.functional.binary_cross_entropy_with_logits(
        torch.tensor(z, dtype=torch.float64), torch.tensor(y, dtype=torch.float64)).item()
    assert abs(P.bce_loss(z, y) - ref) < 1e-14 * max(1.0, abs(ref))
