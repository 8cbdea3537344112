"""cyc_scf_noalloc (no device allocation, fixed per-GPU workspace) against
cyc_scf through the C ABI: two calls in a row, the second on a smaller table,
each bit-identical to cyc_scf on the same input (same kernels, same order) and
within the spectrum's tolerance of the FP64 oracle; sizes beyond the fixed
workspace are rejected before any work is enqueued.
"""
import ctypes

import numpy as np
import pytest

from oracle.cyclic import cross_tables, cyclic_spectrum, lag_window
from paper_2405_16911_amd import siggen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cy():
    from paper_2405_16911_amd import cyclo
    assert torch.cuda.is_available()
    cyclo.lib()
    return cyclo


def _table(seed, lag_min, T, A):
    x = siggen.mixed_stream(6, seed, n=9000)[0]
    alphas = np.linspace(-0.5, 0.5, A, endpoint=False)
    R, _, _ = cross_tables(x, x, alphas, lag_min, T)
    return R.astype(np.complex64), alphas


def test_noalloc_matches_allocating_call_twice(cy):
    cases = [(-40, 81, 700, 512, "hann", 1), (-5, 11, 130, 96, "rect", 2)]  # second call smaller
    for lag_min, T, A, F, window, seed in cases:
        print(f"  case lag_min={lag_min} T={T} A={A} F={F} {window}", flush=True)
        t32, alphas = _table(seed, lag_min, T, A)
        R = torch.from_numpy(t32).to("cuda")
        ref = cy.cyc_scf(R, alphas, lag_min, F, window)
        # fill the output with garbage first: every entry must be written
        out = torch.full((F, A), float("nan"), dtype=torch.complex64, device="cuda")
        got = cy.cyc_scf(R, alphas, lag_min, F, window, noalloc=True, out=out)
        torch.cuda.synchronize()
        assert torch.equal(got, ref)
        oracle = cyclic_spectrum(t32.astype(np.complex128), alphas, lag_min, F, window)
        w = lag_window(lag_min + np.arange(T), window)
        scale = (np.abs(w)[:, None] * np.abs(t32)).sum(0)[None, :]
        assert np.max(np.abs(got.cpu().numpy() - oracle) / scale) <= 1e-5


def test_noalloc_rejects_tables_beyond_the_workspace(cy):
    L = cy.lib()
    R = torch.zeros(1, dtype=torch.complex64, device="cuda")
    al = torch.zeros(1, dtype=torch.float64, device="cuda")
    S = torch.zeros(1, dtype=torch.complex64, device="cuda")
    p = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    # 4096 lags x 513 cycle frequencies > 2^21 entries: refused on the host, nothing launched
    assert L.cyc_scf_noalloc(p(R), p(al), 513, 0, 4096, 1, 0, p(S), None) == cy.CYC_EUNSUPPORTED
    assert L.cyc_scf_noalloc(None, p(al), 1, 0, 1, 1, 0, p(S), None) == cy.CYC_EINVAL
