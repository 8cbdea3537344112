"""mpmath brute force of the cyclic-statistics definition, for tiny inputs.

TEST INFRASTRUCTURE ONLY (see ``oracle/cyclic.py``).  Evaluates the same sums
as the FP64 oracle (Sec. 4, Eq. (11) with x = y, conjugate form per Sec. 2,
Eq. (9)) term by term at ``dps`` decimal digits, so the FP64 oracle's rounding
can be bounded against it.  FP64 inputs are exact binary fractions and are
converted to mpmath without rounding.
"""
from __future__ import annotations

import mpmath as mp


def brute_tables(x, alphas, T: int, dps: int = 50):
    """Returns (R, Rc, n_used) as nested lists of mpmath complex numbers."""
    with mp.workdps(dps):
        xs = [mp.mpc(mp.mpf(float(v.real)), mp.mpf(float(v.imag))) for v in x]
        L = len(xs)
        n_used = max(0, L - T + 1)
        R = [[mp.mpc(0) for _ in alphas] for _ in range(T)]
        Rc = [[mp.mpc(0) for _ in alphas] for _ in range(T)]
        if n_used == 0:
            return R, Rc, 0
        for ai, a in enumerate(alphas):
            am = mp.mpf(float(a))
            for t in range(T):
                s = mp.mpc(0)
                sc = mp.mpc(0)
                for n in range(n_used):
                    prod = am * n
                    phi = prod - mp.floor(prod)
                    e = mp.expjpi(-2 * phi)
                    s += xs[n + t] * mp.conj(xs[n]) * e
                    sc += xs[n + t] * xs[n] * e
                R[t][ai] = s / n_used
                Rc[t][ai] = sc / n_used
        return R, Rc, n_used
