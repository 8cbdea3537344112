"""Pins of the FP64 oracle against exact invariants and library routines (no GPU).

* alpha = 0 row equals the ordinary sample autocorrelation (numpy.vdot);
* uniform grids: the fold identity turns the table into numpy.fft.fft of the
  folded, pre-rotated lag products (the FFT evaluation behind the paper's
  Full mode, Sec. 4);
* 1-periodicity in alpha, rational vs FP64 phase reduction;
* Hermitian symmetry at lag 0, conjugation of the input, scaling;
* carrier offset (Sec. 5): the cyclic ACF only picks up a lag phase while the
  conjugate cycle frequency moves by twice the offset;
* Sec. 2 vs Sec. 4 lag conventions (Eqs. (8) and (11)) differ by an exact phase;
* streaming: any segmentation of the pushes gives a bit-identical result.
"""
import numpy as np
import pytest

from oracle.cyclic import (OracleStream, cyclic_tables, cyclic_tables_sec2, cyclic_cell,
                           phase_frac, phase_frac_rational, scale_per_lag)
from paper_2405_16911_amd import siggen


def _noise(n, seed=0):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(n) + 1j * rng.standard_normal(n)).astype(np.complex64)


def test_alpha_zero_is_autocorrelation():
    x = _noise(3001).astype(np.complex128)
    T = 9
    R, _, N = cyclic_tables(x, [0.0], T, chunk=256)
    for t in range(T):
        ref = np.vdot(x[:N], x[t:t + N]) / N   # sum conj(x[n]) x[n+t]
        assert abs(R[t, 0] - ref) < 1e-13 * max(1.0, abs(ref))


@pytest.mark.parametrize("A,a0", [(64, 0.0), (48, -0.5), (16, 0.1234)])
def test_fold_identity_fft(A, a0):
    """alpha_k = a0 + k/A: S[t,k] = sum_r exp(-j2pi k r/A) q_t[r],
    q_t[r] = sum_{n = r mod A} p_t[n] exp(-j 2 pi a0 n)."""
    x = siggen.gmsk_stream(n=2500, seed=7).astype(np.complex128)
    T = 5
    alphas = a0 + np.arange(A) / A
    R, Rc, N = cyclic_tables(x, alphas, T, chunk=512)
    n = np.arange(N)
    rot = np.exp(-2j * np.pi * a0 * n)
    for t in range(T):
        for table, prod in ((R, x[t:t + N] * np.conj(x[:N])), (Rc, x[t:t + N] * x[:N])):
            q = np.zeros(A, dtype=np.complex128)
            np.add.at(q, n % A, prod * rot)
            ref = np.fft.fft(q) / N
            assert np.max(np.abs(table[t] - ref)) < 1e-12


def test_alpha_periodicity_and_rational_path():
    x = _noise(2000, 3)
    A = 128
    k = np.arange(A)
    alphas = k / A
    R1, Rc1, _ = cyclic_tables(x, alphas, 4)
    R2, Rc2, _ = cyclic_tables(x, alphas + 3.0, 4)
    R3, Rc3, _ = cyclic_tables(x, alphas - 7.0, 4)
    Rq, Rcq, _ = cyclic_tables(x, T=4, rational=(k, A))
    s = scale_per_lag(x, 4)[:, None]
    for a, b in ((R1, R2), (R1, R3), (R1, Rq), (Rc1, Rc2), (Rc1, Rcq)):
        assert np.max(np.abs(a - b) / s) <= 1e-15 * 8


def test_phase_reduction_large_n():
    """Rational vs TwoProduct agree to ~1e-16 at n ~ 2^24..2^40; FP32 alpha*n does not."""
    k = np.array([1, 3, 4095, 2047, 1234])
    A = 4096
    n = np.array([(1 << 24) - 1, 1 << 24, (1 << 24) + 12345, (1 << 33) + 7, (1 << 40) + 99])
    for kk in k:
        exact = phase_frac_rational(kk, A, n)
        fp64 = phase_frac(kk / A, n)
        d = np.abs(exact - fp64)
        d = np.minimum(d, 1 - d)
        assert np.max(d) < 1e-15
    # Negative check: a single-precision product alpha*n keeps no fractional bits near 2^24.
    a32 = np.float32(1234 / 4096)
    n32 = (np.arange(1 << 24, (1 << 24) + 64)).astype(np.float32)
    p32 = a32 * n32
    phi32 = (p32 - np.floor(p32)).astype(np.float64)
    exact = phase_frac_rational(1234, A, np.arange(1 << 24, (1 << 24) + 64))
    err = np.abs(phi32 - exact)
    err = np.minimum(err, 1 - err)
    assert np.max(err) > 0.1


def test_phase_reduction_non_dyadic_exact():
    """frac(alpha*n) for non-dyadic FP64 alpha equals the exact rational value.

    An FP64 alpha is an exact binary fraction, so Fraction(alpha)*n mod 1 is
    the exact phase; the error-free product must reproduce it to ~2^-53 even
    where alpha*n itself has no fractional bits left in FP64.
    """
    from fractions import Fraction
    alphas = [1 / 3, 0.7123456789, -0.4999999, 2.0 ** -30 + 0.1, 123.456]
    ns = [1, 12345, (1 << 24) + 3, (1 << 37) + 11, (1 << 50) + 1]
    for a in alphas:
        got = phase_frac(a, np.array(ns, dtype=np.int64))
        for g, n in zip(got, ns):
            ex = float((Fraction(a) * n) % 1)
            d = abs(g - ex)
            assert min(d, 1 - d) < 2.0 ** -50, (a, n, g, ex)


def test_lag0_hermitian_and_input_conjugation():
    x = _noise(1500, 5)
    alphas = np.array([0.013, 0.25, -0.4, 0.111])
    T = 6
    R, Rc, _ = cyclic_tables(x, alphas, T)
    Rn, Rcn, _ = cyclic_tables(x, -alphas, T)
    assert np.max(np.abs(Rn[0] - np.conj(R[0]))) < 1e-14
    Rx, Rcx, _ = cyclic_tables(np.conj(x), alphas, T)
    assert np.max(np.abs(Rx - np.conj(Rn))) < 1e-14
    assert np.max(np.abs(Rcx - np.conj(Rcn))) < 1e-14


def test_scaling():
    x = _noise(900, 6).astype(np.complex128)
    c = 0.7 - 1.3j
    alphas = [0.0, 0.2, -0.37]
    R, Rc, _ = cyclic_tables(x, alphas, 5)
    Rs, Rcs, _ = cyclic_tables(c * x, alphas, 5)
    assert np.max(np.abs(Rs - abs(c) ** 2 * R)) < 1e-13
    assert np.max(np.abs(Rcs - c * c * Rc)) < 1e-13


def test_carrier_offset_moves_conjugate_cycle_frequency():
    """y = x exp(j2pi f n): R_y^a(t) = e^{j2pi f t} R_x^a(t); Rc_y^a(t) = e^{j2pi f t} Rc_x^{a-2f}(t)."""
    A = 64
    f = 3 / (2 * A)                      # 2f is on the grid
    x = siggen.gmsk_stream(n=4000, seed=11, cfo=0.0).astype(np.complex128)
    y = x * np.exp(2j * np.pi * f * np.arange(x.size))
    alphas = np.arange(A) / A
    T = 7
    Rx, Rcx, _ = cyclic_tables(x, alphas, T)
    Ry, Rcy, _ = cyclic_tables(y, alphas, T)
    lag = np.exp(2j * np.pi * f * np.arange(T))[:, None]
    assert np.max(np.abs(Ry - lag * Rx)) < 1e-12
    shift = int(round(2 * f * A))
    assert np.max(np.abs(Rcy - lag * np.roll(Rcx, shift, axis=1))) < 1e-12


def test_sec2_and_sec4_conventions_differ_by_exact_phase():
    x = _noise(700, 8)
    alphas = np.array([0.0, 0.125, -0.2, 0.333])
    T = 5
    R, Rc, _ = cyclic_tables(x, alphas, T)
    R2, Rc2 = cyclic_tables_sec2(x, alphas, T)
    ph = np.exp(-2j * np.pi * np.outer(np.arange(T), alphas))
    assert np.max(np.abs(R2 - ph * R)) < 1e-13
    assert np.max(np.abs(Rc2 - ph * Rc)) < 1e-13


def test_cell_matches_table():
    x = _noise(5000, 9)
    alphas = [0.0, 0.3, -0.125]
    T = 6
    R, Rc, _ = cyclic_tables(x, alphas, T)
    for j, a in enumerate(alphas):
        for t in (0, 3, 5):
            r, rc = cyclic_cell(x, a, t, T, n_block=777)
            assert abs(r - R[t, j]) < 1e-13 and abs(rc - Rc[t, j]) < 1e-13


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_streaming_segmentation_bitwise(seed):
    x = _noise(5000, 20 + seed)
    alphas = np.array([0.0, 0.0625, -0.31, 0.5])
    T = 13
    ref = cyclic_tables(x, alphas, T, chunk=1000)
    rng = np.random.default_rng(seed)
    st = OracleStream(alphas, T, chunk=1000)
    pos = 0
    while pos < x.size:
        n = int(rng.integers(0, 40 if seed == 0 else 3000))
        st.push(x[pos:pos + n])
        pos += n
    got = st.read()
    assert got[2] == ref[2]
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])


def test_one_sample_pushes_reset_and_empty():
    x = _noise(300, 30)
    alphas = [0.1, 0.2]
    T = 17
    st = OracleStream(alphas, T, chunk=64)
    for i in range(T - 1):
        st.push(x[i:i + 1])
        R, Rc, n = st.read()
        assert n == 0 and not R.any() and not Rc.any()
    for i in range(T - 1, x.size):
        st.push(x[i:i + 1])
    ref = cyclic_tables(x, alphas, T, chunk=64)
    got = st.read()
    assert np.array_equal(got[0], ref[0]) and got[2] == x.size - T + 1
    st.reset()
    st.push(x[:T])
    R, _, n = st.read()
    assert n == 1
    assert np.allclose(R[:, 0], x[:T].astype(complex) * np.conj(complex(x[0])))
    st.push(np.zeros(0, np.complex64))
    assert st.read()[2] == 1
