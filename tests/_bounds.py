"""Scaled-error bounds of the GPU tables against the FP64 oracle.

FP32 operands: 1e-5 for every cell (the stated FP32 target; it also covers
FP32 accumulation within a chunk, the FP32 twiddle tables and the FP64 chunk
phase, which every precision shares).

BF16 / FP16 operands, per cell (tau, alpha), from the rounding model: every
product rounds m operands independently (the Hankel sample and the modulated
operand, which is formed in FP32 and rounded once; relative error uniform
within half an ulp, mean square <= u^2/3 each), so the cell's error is a random
walk of standard deviation u * sqrt(m/3) * r_tau in scaled units, with r_tau
from oracle.cyclic.roundoff_ratio_per_lag; the bound takes six of them.
  BF16: u = 2^-8, FP16: u = 2^-11; m = 2, or 1 with the split modulated operand
"""
import numpy as np

from oracle.cyclic import roundoff_ratio_per_lag, scale_per_lag

FP32_TOL = 1e-5


def bound(flags, chunk, r, rho):
    """The bound for cells with lag factor r = r_tau and rho = |R| / s_tau
    (numpy arrays broadcast), for operand flags `flags` and chunk length
    `chunk` (the model has no term in rho or chunk: the 16-bit roundings are
    independent of the cell's value, and FP32 accumulation over a chunk is
    inside the FP32 tolerance)."""
    prec, split = flags & 3, bool(flags & 4)
    shape = np.broadcast(np.asarray(r), np.asarray(rho)).shape
    if prec == 0:
        return np.full(shape, FP32_TOL)
    u = 2.0 ** -8 if prec == 1 else 2.0 ** -11
    m = 1 if split else 2
    return 6 * u * np.sqrt(m / 3) * np.asarray(r) + np.zeros(shape) + FP32_TOL


def cell_bounds(x, T, flags, chunk, R_ref, Rc_ref):
    """Bound arrays (same shape as R_ref / Rc_ref, whose rows are the lags
    0..T-1) for the scaled error |Rhat - R| / s_tau of a state with operand
    flags `flags` and chunk length `chunk`."""
    r = roundoff_ratio_per_lag(x, T)[:, None]
    s = scale_per_lag(x, T)[:, None]
    s = np.where(s > 0, s, 1.0)
    return tuple(bound(flags, chunk, r, np.abs(ref) / s) for ref in (R_ref, Rc_ref))


def scaled_errors(x, T, R, Rc, R_ref, Rc_ref):
    s = scale_per_lag(x, T)[:, None]
    s = np.where(s > 0, s, 1.0)
    eR = np.abs(np.asarray(R).astype(np.complex128) - R_ref) / s
    eRc = np.abs(np.asarray(Rc).astype(np.complex128) - Rc_ref) / s
    return eR, eRc


def check_cells(x, T, flags, chunk, R, Rc, R_ref, Rc_ref, label=""):
    """Asserts every cell within its bound; returns (max error, max error / bound,
    median error)."""
    eR, eRc = scaled_errors(x, T, R, Rc, R_ref, Rc_ref)
    bR, bRc = cell_bounds(x, T, flags, chunk, R_ref, Rc_ref)
    worst = max(eR.max(), eRc.max())
    ratio = max((eR / bR).max(), (eRc / bRc).max())
    med = float(np.median(np.concatenate([eR.ravel(), eRc.ravel()])))
    print(f"  {label} max scaled error {worst:.3e}, median {med:.3e}, max error/bound {ratio:.3f}", flush=True)
    assert ratio <= 1.0, (label, worst, ratio)
    return worst, ratio, med
