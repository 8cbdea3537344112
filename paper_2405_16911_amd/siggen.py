"""Seeded synthetic baseband signal generators (NumPy, host only).

This module only draws test signals; it contains none of the cyclic-statistics
arithmetic.  It is the one piece of code shared by the CPU oracle tests and the
GPU path's tests and benchmark, so both sides see identical samples.

Signal models
-------------
* GMSK: the CPM complex envelope of Sec. 3, Eq. (10), with modulation index h,
  binary symbols and a Gaussian-filtered rectangular frequency pulse of
  bandwidth B (Sec. 3 names the pulse but not its formula; the standard one is
  used, truncated to L symbols and renormalised so that g(LT) = 1/2, which is
  condition (c) of Sec. 3).
* BPSK/QPSK with a root-raised-cosine pulse (span 16 symbols, unit energy).
* OFDM with 64 QPSK subcarriers, oversampling U and a cyclic prefix of 16*U.
* Rectangular-pulse BPSK and sums of complex tones (closed-form test signals).
* Complex AWGN at a given SNR and a carrier-frequency offset (Sec. 5 discusses
  the offset's effect on the conjugate statistics).

Every random draw comes from ``numpy.random.default_rng`` seeded with
``SeedSequence(entropy=seed, spawn_key=(stream,))``.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc


def rng_for(seed: int, stream: int = 0) -> np.random.Generator:
    """Generator for (seed, stream); streams of one seed are independent."""
    return np.random.default_rng(np.random.SeedSequence(entropy=int(seed), spawn_key=(int(stream),)))


# ----------------------------------------------------------------------------- pulses

def gaussian_frequency_pulse(bt: float, sps: int, L: int = 4) -> np.ndarray:
    """Samples of the GMSK frequency pulse f(t) times Ts, on [0, L*T).

    f(t) = (1/2T) [Q(2 pi B (t - T/2)/sqrt(ln 2)) - Q(2 pi B (t + T/2)/sqrt(ln 2))]
    centred on L*T/2, sampled at the midpoints of the sps*L sample intervals and
    renormalised so the samples sum to exactly 1/2 (g(LT) = 1/2).
    Units: T = 1 symbol, so B = bt.
    """
    n = sps * L
    t = (np.arange(n, dtype=np.float64) + 0.5) / sps - L / 2.0
    k = 2.0 * math.pi * bt / math.sqrt(math.log(2.0))
    q = lambda v: 0.5 * erfc(v / math.sqrt(2.0))
    f = q(k * (t - 0.5)) - q(k * (t + 0.5))
    return f * (0.5 / f.sum())


def rrc_taps(rolloff: float, sps: int, span: int = 16) -> np.ndarray:
    """Root-raised-cosine impulse response, span symbols long, unit energy."""
    n = span * sps
    t = (np.arange(n + 1, dtype=np.float64) - n / 2.0) / sps
    b = float(rolloff)
    h = np.empty_like(t)
    for i, ti in enumerate(t):
        if abs(ti) < 1e-12:
            h[i] = 1.0 + b * (4.0 / math.pi - 1.0)
        elif b > 0 and abs(abs(ti) - 1.0 / (4.0 * b)) < 1e-9:
            h[i] = (b / math.sqrt(2.0)) * ((1 + 2 / math.pi) * math.sin(math.pi / (4 * b))
                                           + (1 - 2 / math.pi) * math.cos(math.pi / (4 * b)))
        else:
            num = math.sin(math.pi * ti * (1 - b)) + 4 * b * ti * math.cos(math.pi * ti * (1 + b))
            den = math.pi * ti * (1 - (4 * b * ti) ** 2)
            h[i] = num / den
    return h / math.sqrt(np.sum(h * h))


# ----------------------------------------------------------------------------- modulations

def gmsk(n: int, sps: int = 8, bt: float = 0.3, h: float = 0.5, L: int = 4,
         rng: np.random.Generator | None = None, bits: np.ndarray | None = None) -> np.ndarray:
    """Binary CPM/GMSK complex envelope, |x| = 1, complex128.

    phase[n] = 2 pi h * sum_k a_k g(n Ts - k T), a_k = +-1, g = running sum of f.
    """
    nsym = n // sps + L + 2
    if bits is None:
        bits = rng.integers(0, 2, size=nsym)
    a = 2.0 * np.asarray(bits[:nsym], dtype=np.float64) - 1.0
    f = gaussian_frequency_pulse(bt, sps, L)
    up = np.zeros(nsym * sps, dtype=np.float64)
    up[::sps] = a
    freq = np.convolve(up, f)[: nsym * sps]
    phase = 2.0 * math.pi * h * np.cumsum(freq)
    return np.exp(1j * phase[:n])


def psk_rrc(n: int, sps: int, rolloff: float, order: int, rng: np.random.Generator,
            span: int = 16) -> np.ndarray:
    """BPSK (order 2) or QPSK (order 4) symbols shaped by an RRC pulse, unit power."""
    nsym = n // sps + span + 2
    if order == 2:
        s = 2.0 * rng.integers(0, 2, size=nsym) - 1.0 + 0j
    elif order == 4:
        s = ((2.0 * rng.integers(0, 2, size=nsym) - 1.0)
             + 1j * (2.0 * rng.integers(0, 2, size=nsym) - 1.0)) / math.sqrt(2.0)
    else:
        raise ValueError("order must be 2 or 4")
    up = np.zeros(nsym * sps, dtype=np.complex128)
    up[::sps] = s
    y = np.convolve(up, rrc_taps(rolloff, sps, span))
    y = y[span * sps // 2: span * sps // 2 + n]
    return y / math.sqrt(np.mean(np.abs(y) ** 2))


def ofdm(n: int, oversample: int, rng: np.random.Generator, nsc: int = 64, cp: int = 16) -> np.ndarray:
    """CP-OFDM, nsc QPSK subcarriers, IFFT size nsc*U (zero-padded centre), CP cp*U."""
    U = int(oversample)
    nfft, ncp = nsc * U, cp * U
    nblk = n // (nfft + ncp) + 1
    out = []
    for _ in range(nblk):
        d = ((2.0 * rng.integers(0, 2, size=nsc) - 1.0)
             + 1j * (2.0 * rng.integers(0, 2, size=nsc) - 1.0)) / math.sqrt(2.0)
        spec = np.zeros(nfft, dtype=np.complex128)
        spec[: nsc // 2] = d[nsc // 2:]          # subcarriers 0..nsc/2-1
        spec[nfft - nsc // 2:] = d[: nsc // 2]   # subcarriers -nsc/2..-1
        sym = np.fft.ifft(spec)
        out.append(np.concatenate([sym[nfft - ncp:], sym]))
    y = np.concatenate(out)[:n]
    return y / math.sqrt(np.mean(np.abs(y) ** 2))


def rect_bpsk(n: int, period: int, rng: np.random.Generator) -> np.ndarray:
    """Rectangular-pulse BPSK: x[n] = a_{floor(n/P)}, a i.i.d. +-1 (complex128)."""
    a = 2.0 * rng.integers(0, 2, size=n // period + 1) - 1.0
    return np.repeat(a, period)[:n].astype(np.complex128)


def tones(n: int, freqs, amps) -> np.ndarray:
    """sum_i amps[i] * exp(j 2 pi freqs[i] n), n = 0..n-1, complex128."""
    idx = np.arange(n, dtype=np.float64)
    x = np.zeros(n, dtype=np.complex128)
    for f, a in zip(freqs, amps):
        x += complex(a) * np.exp(2j * math.pi * float(f) * idx)
    return x


# ----------------------------------------------------------------------------- channel

def add_awgn(x: np.ndarray, snr_db: float, rng: np.random.Generator) -> np.ndarray:
    """Adds circular complex Gaussian noise of variance 10^(-snr/10) (unit signal power)."""
    var = 10.0 ** (-snr_db / 10.0)
    w = rng.standard_normal(x.size) + 1j * rng.standard_normal(x.size)
    return x + math.sqrt(var / 2.0) * w


def apply_cfo(x: np.ndarray, f0: float) -> np.ndarray:
    """Multiplies by exp(j 2 pi f0 n) (carrier offset in cycles/sample)."""
    return x * np.exp(2j * math.pi * f0 * np.arange(x.size, dtype=np.float64))


# ----------------------------------------------------------------------------- workloads

def gmsk_stream(n=32768, sps=8, bt=0.3, snr_db=10.0, cfo=0.05, seed=1, stream=0) -> np.ndarray:
    """GMSK, i.i.d. bits, unit power, complex AWGN, carrier offset; complex64."""
    rng = rng_for(seed, stream)
    x = gmsk(n, sps=sps, bt=bt, rng=rng)
    x = add_awgn(x, snr_db, rng)
    return apply_cfo(x, cfo).astype(np.complex64)


def qpsk_rrc_stream(n=1 << 24, sps=4, rolloff=0.35, snr_db=5.0, cfo=0.1, seed=2, stream=0) -> np.ndarray:
    """QPSK with RRC pulse, unit power, complex AWGN, carrier offset; complex64."""
    rng = rng_for(seed, stream)
    x = psk_rrc(n, sps, rolloff, 4, rng)
    x = add_awgn(x, snr_db, rng)
    return apply_cfo(x, cfo).astype(np.complex64)


def uniform_grid(n_alpha: int, start: float) -> np.ndarray:
    """alpha_k = start + k/n_alpha (exact in FP64 for power-of-two n_alpha)."""
    return start + np.arange(n_alpha, dtype=np.float64) / n_alpha


def mixed_stream(seed: int, stream: int, n: int | None = None):
    """One stream of the mixed-modulation batch workload.

    Returns (x complex64, meta dict).  Modulation drawn with equal weights from
    GMSK (BT 0.3), BPSK-RRC, QPSK-RRC (rolloff U[0.25,0.5]) and OFDM (64
    subcarriers, CP 16); samples/symbol (or OFDM oversampling) U{2..16};
    carrier offset U[-0.25,0.25]; SNR U[0,20] dB; length log-uniform in
    [2^12, 2^20] unless n is given; alpha-set size log-uniform in [64, 2048].
    """
    rng = rng_for(seed, stream)
    kind = int(rng.integers(0, 4))
    sps = int(rng.integers(2, 17))
    cfo = float(rng.uniform(-0.25, 0.25))
    snr = float(rng.uniform(0.0, 20.0))
    rolloff = float(rng.uniform(0.25, 0.5))
    length = int(2.0 ** rng.uniform(12.0, 20.0)) if n is None else int(n)
    n_alpha = int(2.0 ** rng.uniform(6.0, 11.0))
    if kind == 0:
        x = gmsk(length, sps=sps, bt=0.3, rng=rng)
        name = "gmsk"
    elif kind == 1:
        x = psk_rrc(length, sps, rolloff, 2, rng)
        name = "bpsk_rrc"
    elif kind == 2:
        x = psk_rrc(length, sps, rolloff, 4, rng)
        name = "qpsk_rrc"
    else:
        x = ofdm(length, sps, rng)
        name = "ofdm"
    x = apply_cfo(add_awgn(x, snr, rng), cfo).astype(np.complex64)
    meta = dict(kind=name, sps=sps, cfo=cfo, snr_db=snr, rolloff=rolloff, length=length, n_alpha=n_alpha)
    return x, meta
