"""Properties of the seeded signal generators (no GPU)."""
import math

import numpy as np

from paper_2405_16911_amd import siggen


def test_gmsk_constant_envelope_and_phase_accumulation():
    rng = siggen.rng_for(3, 0)
    sps, L, h = 8, 4, 0.5
    bits = rng.integers(0, 2, size=200)
    n = 150 * sps
    x = siggen.gmsk(n, sps=sps, bt=0.3, h=h, L=L, bits=bits)
    assert np.allclose(np.abs(x), 1.0, atol=1e-12)
    # g(LT) = 1/2: once symbol k's pulse has ended, it has added pi*h*a_k of phase.
    ph = np.unwrap(np.angle(x))
    a = 2.0 * bits - 1.0
    k = 100
    # total phase after sample k*sps - 1 includes complete pulses of symbols 0..k-L
    f = siggen.gaussian_frequency_pulse(0.3, sps, L)
    assert abs(f.sum() - 0.5) < 1e-15
    full = math.pi * h * a[: k - L + 1].sum()
    partial = 2 * math.pi * h * sum(a[j] * f[: k * sps - j * sps].sum() for j in range(k - L + 1, k))
    assert abs(ph[k * sps - 1] - ph[0] + (2 * math.pi * h * a[0] * f[0]) - (full + partial)) < 1e-9


def test_rrc_unit_energy_and_nyquist():
    sps, b = 4, 0.35
    h = siggen.rrc_taps(b, sps)
    assert abs(np.sum(h * h) - 1.0) < 1e-12
    rc = np.convolve(h, h)
    c = rc.size // 2
    # raised cosine: zero crossings at non-zero multiples of the symbol period
    assert np.max(np.abs(rc[c + sps: c + 6 * sps + 1: sps])) < 2e-3


def test_ofdm_cyclic_prefix():
    rng = siggen.rng_for(4, 0)
    U = 3
    x = siggen.ofdm(5 * 80 * U, U, rng)
    nfft, ncp = 64 * U, 16 * U
    for s in range(4):
        blk = x[s * (nfft + ncp): (s + 1) * (nfft + ncp)]
        assert np.allclose(blk[:ncp], blk[-ncp:])


def test_awgn_power_and_unit_power_workloads():
    rng = siggen.rng_for(5, 0)
    x = np.zeros(1 << 18, dtype=np.complex128)
    y = siggen.add_awgn(x, 10.0, rng)
    assert abs(np.mean(np.abs(y) ** 2) - 0.1) < 0.002
    q = siggen.qpsk_rrc_stream(n=1 << 16)
    assert q.dtype == np.complex64
    assert abs(np.mean(np.abs(q.astype(np.complex128)) ** 2) - (1 + 10 ** -0.5)) < 0.03


def test_seeded_reproducibility():
    a = siggen.gmsk_stream(n=4096, seed=1)
    b = siggen.gmsk_stream(n=4096, seed=1)
    c = siggen.gmsk_stream(n=4096, seed=2)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    x1, m1 = siggen.mixed_stream(4, 17, n=5000)
    x2, m2 = siggen.mixed_stream(4, 17, n=5000)
    assert np.array_equal(x1, x2) and m1 == m2
    assert 64 <= m1["n_alpha"] <= 2048 and 2 <= m1["sps"] <= 16
