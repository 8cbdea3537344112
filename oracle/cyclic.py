"""FP64 CPU oracle for the cyclic autocorrelation and its conjugate form.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call or execute this module; only the tests, the
graft entry's smoke check and the benchmark's CPU-baseline leg do.  It shares
no code with the GPU path.

What it computes (the estimator of Sec. 4, Eq. (11), applied to one signal,
x = y, non-negative lags; normalisation and conjugate form as in Sec. 2,
Eqs. (8)-(9)):

    N_used      = max(0, L - T + 1)                      (one count for all lags)
    E(a, n)     = exp(-j 2 pi frac(a * n))              (absolute sample index n)
    S[t, a]     = sum_{n=0}^{N_used-1} x[n+t] * conj(x[n]) * E(a, n)
    Sc[t, a]    = sum_{n=0}^{N_used-1} x[n+t] * x[n]       * E(a, n)
    R  = S  / N_used,   Rc = Sc / N_used   (all-zero tables when N_used = 0)

for lags t = 0..T-1 and an arbitrary list of cycle frequencies a (cycles per
sample, the normalised frequency of Sec. 2).  The result is the plain
definition written out; the only library primitives are a complex matrix
product (step "O2") or a dot product (step "O1") used as the sum over n.

Phase reduction frac(a*n):
  * general FP64 a: error-free product p + e = a*n (Dekker/Veltkamp
    TwoProduct, no FMA needed), frac = (p - floor(p)) + e, wrapped to [0, 1);
  * rational a = k/A (exact integers): (k*n mod A)/A in integer arithmetic.
The twiddle is then cos(2 pi phi) - j sin(2 pi phi) from FP64 libm.

Streaming: ``OracleStream`` keeps (tail, S, L) and adds products in fixed
absolute chunks of ``chunk`` products, so any segmentation of the pushes
gives a bit-identical result, and ``cyclic_tables`` is a single push.
"""
from __future__ import annotations

import numpy as np

_SPLIT = 134217729.0  # 2^27 + 1, Veltkamp splitter for FP64


def _split(a: np.ndarray):
    c = _SPLIT * a
    hi = c - (c - a)
    return hi, a - hi


def two_product(a: np.ndarray, b: np.ndarray):
    """Error-free product: returns (p, e) with p = fl(a*b) and p + e = a*b exactly."""
    p = a * b
    ah, al = _split(a)
    bh, bl = _split(b)
    e = ((ah * bh - p) + ah * bl + al * bh) + al * bl
    return p, e


def phase_frac(alpha, n) -> np.ndarray:
    """frac(alpha * n) in [0, 1) for FP64 alpha and integer n (broadcasting)."""
    a = np.asarray(alpha, dtype=np.float64)
    nn = np.asarray(n, dtype=np.int64).astype(np.float64)  # exact for |n| < 2^53
    p, e = two_product(a, nn)
    phi = (p - np.floor(p)) + e
    phi = phi - np.floor(phi)
    return np.where(phi >= 1.0, 0.0, phi)


def phase_frac_rational(k, A, n) -> np.ndarray:
    """frac((k/A) * n) = ((k*n) mod A) / A with exact integer arithmetic."""
    k = np.asarray(k, dtype=np.int64)
    n = np.asarray(n, dtype=np.int64)
    A = int(A)
    r = np.mod(np.mod(k, A) * np.mod(n, A), A)
    return r.astype(np.float64) / A


def twiddle(phi: np.ndarray) -> np.ndarray:
    """exp(-j 2 pi phi) from FP64 cos/sin."""
    ang = 2.0 * np.pi * phi
    return np.cos(ang) - 1j * np.sin(ang)


class _Alphas:
    """Either a list of FP64 cycle frequencies or an exact rational grid."""

    def __init__(self, alphas=None, rational=None):
        if rational is not None:
            k, A = rational
            self.k = np.asarray(k, dtype=np.int64)
            self.A = int(A)
            self.values = self.k.astype(np.float64) / self.A
        else:
            self.k = None
            self.values = np.asarray(alphas, dtype=np.float64).reshape(-1)

    def __len__(self):
        return self.values.size

    def E(self, n: np.ndarray) -> np.ndarray:
        """Twiddle matrix E[i, a] = E(alpha_a, n_i), shape (len(n), A)."""
        n = np.asarray(n, dtype=np.int64)[:, None]
        if self.k is not None:
            phi = phase_frac_rational(self.k[None, :], self.A, n)
        else:
            phi = phase_frac(self.values[None, :], n)
        return twiddle(phi)


def lag_products(x: np.ndarray, n0: int, n1: int, T: int):
    """P[t, i] = x[n0+i+t] conj(x[n0+i]) and Pc[t, i] = x[n0+i+t] x[n0+i], i < n1-n0."""
    m = n1 - n0
    base = x[n0:n1]
    shifted = np.stack([x[n0 + t: n0 + t + m] for t in range(T)]) if T > 0 else np.zeros((0, m), complex)
    return shifted * np.conj(base)[None, :], shifted * base[None, :]


class OracleStream:
    """Streaming form of the oracle: push blocks, read tables at any time."""

    def __init__(self, alphas=None, T: int = 1, rational=None, chunk: int = 4096):
        if T <= 0:
            raise ValueError("T must be positive")
        self.al = _Alphas(alphas, rational)
        if len(self.al) == 0:
            raise ValueError("empty alpha list")
        self.T = int(T)
        self.chunk = int(chunk)
        self.reset()

    def reset(self):
        A = len(self.al)
        self.S = np.zeros((self.T, A), dtype=np.complex128)
        self.Sc = np.zeros((self.T, A), dtype=np.complex128)
        self.L = 0            # samples pushed
        self.nc = 0           # products committed (multiple of chunk)
        self.tail = np.zeros(0, dtype=np.complex128)  # samples nc .. L-1

    def _sum(self, x, n0, n1):
        """Products n0..n1-1 (absolute), x holds samples from absolute index self.nc."""
        off = self.nc
        P, Pc = lag_products(x, n0 - off, n1 - off, self.T)
        E = self.al.E(np.arange(n0, n1, dtype=np.int64))
        return P @ E, Pc @ E

    def push(self, xb):
        xb = np.asarray(xb).astype(np.complex128).reshape(-1)
        if xb.size == 0:
            return
        buf = np.concatenate([self.tail, xb])
        self.L += xb.size
        n_used = max(0, self.L - self.T + 1)
        while self.nc + self.chunk <= n_used:
            s, sc = self._sum(buf, self.nc, self.nc + self.chunk)
            self.S += s
            self.Sc += sc
            buf = buf[self.chunk:]
            self.nc += self.chunk
        self.tail = buf

    @property
    def n_used(self) -> int:
        return max(0, self.L - self.T + 1)

    def read(self):
        """Returns (R, Rc, n_used): complex128 [T, A] tables; state unchanged."""
        n_used = self.n_used
        A = len(self.al)
        if n_used == 0:
            z = np.zeros((self.T, A), dtype=np.complex128)
            return z, z.copy(), 0
        S, Sc = self.S.copy(), self.Sc.copy()
        if n_used > self.nc:
            s, sc = self._sum(self.tail, self.nc, n_used)
            S += s
            Sc += sc
        return S / n_used, Sc / n_used, n_used


def cyclic_tables(x, alphas=None, T: int = 1, rational=None, chunk: int = 4096):
    """Batch oracle (O2): (R, Rc, n_used) for the whole record x."""
    st = OracleStream(alphas, T, rational=rational, chunk=chunk)
    st.push(x)
    return st.read()


def cross_tables(x, y, alphas, lag_min: int, T: int):
    """Two-input form of Sec. 4, Eq. (11), lags m = lag_min .. lag_min + T - 1.

    Lag m pairs x[k + m] with y[k]; the phase is referenced to y's index k:
      R [t, a] = (1/N) sum_{n<N} x[n + dx + t] conj(y[n + dy]) E(a, n + dy),
      Rc[t, a] = (1/N) sum_{n<N} x[n + dx + t]      y[n + dy]  E(a, n + dy),
    dx = max(0, lag_min), dy = max(0, -lag_min), so every product of every lag
    has both samples; N = max(0, L - (T - 1) - |lag_min|), L = min(len x, len y)
    (one count for all lags).  With y = x and lag_min = 0 this is cyclic_tables.
    Returns (R, Rc, N).
    """
    x = np.asarray(x).astype(np.complex128).reshape(-1)
    y = np.asarray(y).astype(np.complex128).reshape(-1)
    al = _Alphas(alphas, None)
    L = min(x.size, y.size)
    dx, dy = max(0, lag_min), max(0, -lag_min)
    N = max(0, L - (T - 1) - abs(lag_min))
    A = len(al)
    if N == 0:
        z = np.zeros((T, A), dtype=np.complex128)
        return z, z.copy(), 0
    yb = y[dy:dy + N]
    X = np.stack([x[dx + t: dx + t + N] for t in range(T)])
    E = al.E(np.arange(dy, dy + N, dtype=np.int64))
    return (X * np.conj(yb)[None, :]) @ E / N, (X * yb[None, :]) @ E / N, N


def window_tables(x, alphas, T: int, hop: int, n_hops: int):
    """Sliding-window form: the estimate over the last n_hops complete hops.

    Products are grouped in hops of `hop` (aligned to the first product); with
    c complete hops among the N = L - T + 1 products, the window holds the
    last W = min(n_hops, c) of them, products n_w .. n_w + W hop - 1 with
    n_w = (c - W) hop, and the phase is referenced to the window's first
    product (as the block's `state` re-references it, Sec. 4):
      R[t, a] = (1/(W hop)) sum_{n in window} x[n+t] conj(x[n]) E(a, n - n_w),
    i.e. the cumulative tables of the slice x[n_w : n_w + W hop + T - 1].
    Returns (R, Rc, W hop) (zero tables and 0 before the first complete hop).
    """
    x = np.asarray(x).astype(np.complex128).reshape(-1)
    N = max(0, x.size - T + 1)
    c = N // hop
    W = min(n_hops, c)
    if W == 0:
        A = len(_Alphas(alphas, None))
        z = np.zeros((T, A), dtype=np.complex128)
        return z, z.copy(), 0
    n_w = (c - W) * hop
    R, Rc, n = cyclic_tables(x[n_w: n_w + W * hop + T - 1], alphas, T)
    assert n == W * hop
    return R, Rc, n


def lag_window(lags, window: str):
    """Lag window: 'rect' (ones) or 'hann', w(m) = (1 + cos(pi m / (M + 1))) / 2 with M = max |m|."""
    lags = np.asarray(lags, dtype=np.float64)
    if window == "rect":
        return np.ones_like(lags)
    M = np.max(np.abs(lags))
    return 0.5 * (1.0 + np.cos(np.pi * lags / (M + 1.0)))


def cyclic_spectrum(R, alphas, lag_min: int, n_freq: int, window: str = "rect"):
    """Cyclic spectrum by the cyclic Wiener-Khinchin relation, from a table R[t, a]
    with lags m_t = lag_min + t (as cross_tables or the single-input tables):

      S[k, a] = sum_t w(m_t) exp(-j pi alpha_a m_t) R[t, a] exp(-j2pi f_k m_t),
      f_k = -1/2 + k / n_freq.

    exp(-j pi alpha m) R(m) is the symmetric form sum x[k + m/2] conj(y[k - m/2])
    exp(-j2pi alpha k) of the leading-lag table.  Plain definition in FP64.
    """
    R = np.asarray(R, dtype=np.complex128)
    T, A = R.shape
    m = lag_min + np.arange(T)
    al = np.asarray(alphas, dtype=np.float64).reshape(-1)
    f = -0.5 + np.arange(n_freq) / n_freq
    w = lag_window(m, window)
    P = w[:, None] * np.exp(-1j * np.pi * al[None, :] * m[:, None]) * R
    return np.exp(-2j * np.pi * f[:, None] * m[None, :]) @ P


def cyclic_cell(x, alpha: float, tau: int, T: int, n_block: int = 1 << 20):
    """O1: one (alpha, tau) cell of (R, Rc) by a direct dot product over n.

    Uses the same common count N_used = L - T + 1 as the tables, so a cell of
    the full table can be checked on its own at any record length.
    """
    x = np.asarray(x).reshape(-1)
    L = x.size
    n_used = max(0, L - T + 1)
    if n_used == 0:
        return 0j, 0j
    s = 0j
    sc = 0j
    a = np.float64(alpha)
    for n0 in range(0, n_used, n_block):
        n1 = min(n_used, n0 + n_block)
        n = np.arange(n0, n1, dtype=np.int64)
        e = twiddle(phase_frac(a, n))
        xt = x[n0 + tau: n1 + tau].astype(np.complex128)
        xb = x[n0:n1].astype(np.complex128)
        s += np.dot(xt * np.conj(xb), e)
        sc += np.dot(xt * xb, e)
    return s / n_used, sc / n_used


def cyclic_tables_sec2(x, alphas, T: int):
    """Sec. 2 form (Eqs. (8)-(9)) over a matched index range.

    R2[m, a] = (1/N) sum_{n=m}^{m+N-1} x[n] conj(x[n-m]) E(a, n),
    Rc2[m, a] = (1/N) sum_{n=m}^{m+N-1} x[n] x[n-m] E(a, n),  N = L - T + 1.
    The lag sits on the trailing sample and the phase on the leading one; over
    this range R2 = exp(-j 2 pi a m) * R (Sec. 4 form).
    """
    x = np.asarray(x).astype(np.complex128).reshape(-1)
    al = _Alphas(alphas)
    N = max(0, x.size - T + 1)
    R = np.zeros((T, len(al)), dtype=np.complex128)
    Rc = np.zeros_like(R)
    if N == 0:
        return R, Rc
    for m in range(T):
        n = np.arange(m, m + N, dtype=np.int64)
        E = al.E(n)
        lead = x[m: m + N]
        trail = x[0:N]
        R[m] = (lead * np.conj(trail)) @ E / N
        Rc[m] = (lead * trail) @ E / N
    return R, Rc


def scale_per_lag(x, T: int) -> np.ndarray:
    """s_t = (1/N_used) sum_n |x[n+t]| |x[n]|, the dot-product condition scale.

    The GPU results are compared with ``|Rhat - R| / s_t`` (the scaled error).
    """
    x = np.abs(np.asarray(x).astype(np.complex128).reshape(-1))
    N = max(0, x.size - T + 1)
    if N == 0:
        return np.zeros(T)
    return np.array([np.dot(x[t: t + N], x[:N]) / N for t in range(T)])


def roundoff_ratio_per_lag(x, T: int) -> np.ndarray:
    """r_t = sqrt(sum_n |x[n+t]|^2 |x[n]|^2) / sum_n |x[n+t]| |x[n]|, n < N_used.

    Ratio of the root-sum-square of the lag products' magnitudes to their sum:
    independent roundings of relative size u in each product give a scaled
    error of about u * r_t (a random walk), against u for roundings that all
    push the same way.  Equals 1/sqrt(N_used) for a constant-modulus signal.
    Test infrastructure for the reduced-precision tolerances; zeros when
    N_used = 0.
    """
    x = np.abs(np.asarray(x).astype(np.complex128).reshape(-1))
    N = max(0, x.size - T + 1)
    if N == 0:
        return np.zeros(T)
    out = np.empty(T)
    for t in range(T):
        m = x[t: t + N] * x[:N]
        out[t] = np.sqrt(np.dot(m, m)) / m.sum()
    return out
