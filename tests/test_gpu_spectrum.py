"""GPU cyclic spectrum (cyc_scf) against the FP64 oracle on the same lag table.

The table is the oracle's own (rounded to complex64), so the comparison isolates
the spectrum: FP64 phases, FP32 lag sums of at most n_lag terms, held to
1e-5 of sum_t |w R| per cycle frequency.
"""
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


@pytest.mark.parametrize("lag_min,T,F,window", [(-32, 65, 128, "hann"), (0, 40, 64, "rect"), (-7, 9, 1000, "hann")])
def test_spectrum_matches_oracle(cy, lag_min, T, F, window):
    x = siggen.mixed_stream(5, 11, n=12000)[0]
    alphas = np.concatenate([np.linspace(-0.5, 0.5, 300, endpoint=False), [0.0, 0.125, 1 / 3]])
    R, Rc, _ = cross_tables(x, x, alphas, lag_min, T)
    for tab in (R, Rc):
        t32 = tab.astype(np.complex64)
        ref = cyclic_spectrum(t32.astype(np.complex128), alphas, lag_min, F, window)
        got = cy.cyc_scf(torch.from_numpy(t32).to("cuda"), alphas, lag_min, F, window).cpu().numpy()
        w = lag_window(lag_min + np.arange(T), window)
        scale = (np.abs(w)[:, None] * np.abs(t32)).sum(0)[None, :]
        e = np.max(np.abs(got - ref) / scale)
        print(f"  lag_min={lag_min} T={T} F={F} {window}: max relative error {e:.2e}", flush=True)
        assert e <= 1e-5


def test_spectrum_of_a_tone_peaks_at_its_frequency(cy):
    # end to end: two-input state with symmetric lags -> cyclic spectrum at alpha = 0
    L, M, F = 20000, 16, 256
    f0 = 37 / 256
    x = (np.exp(2j * np.pi * f0 * np.arange(L)) + 0.1 * siggen.gmsk_stream(n=L, seed=3)).astype(np.complex64)
    st = cy.CrossStream(np.array([0.0, 0.01]), -M, 2 * M + 1, 0)
    d = torch.from_numpy(x).to("cuda")
    st.push2(d, d)
    R, Rc, n = st.read()
    S = cy.cyc_scf(R, np.array([0.0, 0.01]), -M, F, "hann").cpu().numpy()
    st.close()
    f = -0.5 + np.arange(F) / F
    assert abs(f[int(np.argmax(np.abs(S[:, 0])))] - f0) < 1e-12
