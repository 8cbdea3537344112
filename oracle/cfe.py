"""FP64 CPU oracle for cycle-frequency estimation from the cyclic tables.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): nothing in the product
path imports it; it shares no code with the GPU path.

The paper names estimation of the cycle frequencies themselves as future work
(Sec. 6) and, among related estimators, describes a coarse-to-fine search
(Sec. 1).  The estimator here is a reading of that idea on the tables of
Sec. 4, Eq. (11), on a coarse grid fine enough to hold every feature's main
lobe (spacing 1/A <= 1/N_used, as the grid of the Full mode in Sec. 4 is):

1. Coarse table R[t, k] (either table) on the uniform grid
   alpha_k = alpha0 + k / A, k < A, A a multiple of B = 64.
2. Local noise scale sigma[t, c] per lag and block c of B bins: the median of
   |R[t, .]| over blocks c-1, c, c+1 (circular) divided by sqrt(2 ln 2), the
   Rayleigh scale of cells without a feature (oracle.proposal.local_sigma, the
   rule of the proposal's labels; local because a modulated signal's
   self-noise is strong near its features and weak elsewhere).
3. Statistic per cycle frequency: q_k = max_t |R[t, k]| / sigma[t, k div B].
4. Candidates: bins with q_k > kappa that are circular local maxima,
   q_k > q_{k-1} and q_k >= q_{k+1} (of a run of equal values the first wins).
5. Leakage masking.  A feature between grid points leaks into every bin
   through the Dirichlet kernel of the N products,
   |D_N(nu)| = |sin(pi nu N) / (N sin(pi nu))|.  With spacing 1/A <= 1/N the
   feature is within half a bin of its peak bin p, where |D_N| >= 2/pi, and a
   bin d bins away (circular distance, 1 <= d <= A/2) is at least (d - 1/2)/A
   from it; with sin(x) >= 2x/pi on [0, pi/2] the leaked magnitude at any lag
   is at most |R[t, p]| (pi/2) / (N sin(pi (d - 1/2)/A)) <= |R[t, p]| (pi/4) r,
   r = A / (N (d - 1/2)).  Candidates are taken in descending q (ties ->
   lower k); one is kept if at some lag t it exceeds kappa sigma[t, .] and
   |R[t, k]| > ((pi/2) r) |R[t, p]| for every kept p (twice the leakage bound:
   the noise allowance).  `exclude` (the alpha = 0 bin of the non-conjugate
   table, where the power term always sits) is never reported, but it is a
   candidate like any other and masks its own leakage.
6. Refinement of each detection: the same table on the zoom grid
   alpha_k + (j - Z) / (Z A), j = 0..2Z (one coarse spacing either side),
   and alpha_hat = the zoom point with the largest max_t |R| / sigma[t, k div B]
   (the detection's coarse scale; ties -> lower j).  Resolution 1 / (Z A).

Magnitudes sqrt(Re^2 + Im^2), scales and every comparison are FP64.
"""
from __future__ import annotations

import numpy as np

from oracle.cyclic import cyclic_tables
from oracle.proposal import local_sigma

BLOCK = 64
HALF_PI = np.pi / 2.0


def magnitudes(R) -> np.ndarray:
    """|R| = sqrt(Re^2 + Im^2) in FP64 (one rounding of the sum, then the square root)."""
    R = np.asarray(R).astype(np.complex128)
    return np.sqrt(R.real * R.real + R.imag * R.imag)


def scales(R) -> np.ndarray:
    """sigma[t, c] for the blocks of B bins of a [T, A] table."""
    m = magnitudes(R)
    return local_sigma(m, m.shape[1] // BLOCK)


def ratios(R, sigma) -> np.ndarray:
    """|R[t, k]| / sigma[t, k div B] (inf where sigma is 0 and |R| > 0, 0 for 0/0)."""
    m = magnitudes(R)
    s = np.repeat(sigma, BLOCK, axis=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        q = m / s
    return np.where(np.isnan(q), 0.0, q)


def candidates(q: np.ndarray, kappa: float) -> np.ndarray:
    """Bins k with q_k > kappa that are circular local maxima (q_k > left, >= right)."""
    A = q.size
    out = []
    for k in range(A):
        if not q[k] > kappa:
            continue
        if A > 1 and not (q[k] > q[(k - 1) % A] and q[k] >= q[(k + 1) % A]):
            continue
        out.append(k)
    return np.array(out, dtype=np.int64)


def leak_factor(d: int, A: int, N: int) -> float:
    """(pi/2) r with r = A / (N (d - 1/2)): twice the most a feature's magnitude
    can leak, relative to its peak bin, into a bin at circular distance d >= 1."""
    return HALF_PI * (A / (N * (d - 0.5)))


def detect(R, kappa: float, N: int, exclude: int | None = None):
    """Detected bins of a table, ascending, and the scales sigma."""
    m = magnitudes(R)
    A = m.shape[1]
    sigma = scales(R)
    r = ratios(R, sigma)
    q = r.max(axis=0)
    cand = candidates(q, kappa)
    kept = []
    for k in sorted(cand.tolist(), key=lambda k: (-q[k], k)):
        ok = False
        for t in range(m.shape[0]):
            if not r[t, k] > kappa:
                continue
            clear = True
            for p in kept:
                d = abs(k - p)
                d = min(d, A - d)
                if not m[t, k] > leak_factor(d, A, N) * m[t, p]:
                    clear = False
                    break
            if clear:
                ok = True
                break
        if ok:
            kept.append(k)
    return np.array(sorted(k for k in kept if k != exclude), dtype=np.int64), sigma


def zero_bin(alpha0: float, A: int) -> int | None:
    """The bin k with alpha0 + k/A an integer, if there is one."""
    k = int(np.rint(-alpha0 * A)) % A
    a = alpha0 + k / A
    return k if abs(a - np.rint(a)) < 1e-12 else None


def zoom_grid(alpha_k: float, A: int, Z: int) -> np.ndarray:
    """alpha_k + (j - Z) / (Z A), j = 0..2Z."""
    return np.array([alpha_k + (j - Z) / (Z * A) for j in range(2 * Z + 1)])


def refine(Rz, sigma_col):
    """(j, q_j): the zoom column with the largest max_t |R[t, j]| / sigma_col[t]
    (ties -> lower j)."""
    m = magnitudes(Rz)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = m / sigma_col[:, None]
    q = np.where(np.isnan(r), 0.0, r).max(axis=0)
    j = int(np.argmax(q))
    return j, float(q[j])


def estimate(x, T: int, alpha0: float, A: int, kappa: float = 7.0, Z: int = 16, which: str = "R",
             exclude_zero: bool = True):
    """Cycle-frequency estimates from one table ('R' or 'Rc') of the samples x.

    Returns a list of (coarse bin k, alpha_hat, statistic at alpha_hat),
    ascending in k.
    """
    if A % BLOCK:
        raise ValueError("A must be a multiple of 64")
    alphas = np.array([alpha0 + k / A for k in range(A)])
    R, Rc, N = cyclic_tables(x, alphas, T)
    if N > A:
        raise ValueError("the coarse grid must be at least as fine as 1/N_used")
    tab = R if which == "R" else Rc
    excl = zero_bin(alpha0, A) if (exclude_zero and which == "R") else None
    bins, sigma = detect(tab, kappa, N, excl)
    out = []
    for k in bins:
        zg = zoom_grid(alphas[k], A, Z)
        Rz, Rcz, _ = cyclic_tables(x, zg, T)
        j, qj = refine(Rz if which == "R" else Rcz, sigma[:, k // BLOCK])
        out.append((int(k), float(zg[j]), qj))
    return out
