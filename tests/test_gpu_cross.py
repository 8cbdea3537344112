"""GPU parity of the two-input form (lags of either sign) against the FP64 oracle.

Tolerances as the single-input tables (tests/_bounds.py), per cell, on the
scaled error with s_t = (1/N) sum_n |x[n + dx + t]| |y[n + dy]| and the
random-walk factor r_t = sqrt(sum |x[n+dx+t]|^2 |y[n+dy]|^2) / sum |x||y|
over the same products.  Segmentations are bitwise equal; a two-input state fed one input
with lag_min = 0 equals a single-input state bitwise.
"""
import numpy as np
import pytest

from _bounds import FP32_TOL, bound
from oracle.cyclic import cross_tables
from paper_2405_16911_amd import siggen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

@pytest.fixture(scope="module")
def cy():
    from paper_2405_16911_amd import cyclo
    assert torch.cuda.is_available()
    cyclo.lib()
    return cyclo


def _products(x, y, lag_min, T):
    x = np.abs(x.astype(np.complex128))
    y = np.abs(y.astype(np.complex128))
    L = min(x.size, y.size)
    dx, dy = max(0, lag_min), max(0, -lag_min)
    N = L - (T - 1) - abs(lag_min)
    return [x[dx + t: dx + t + N] * y[dy: dy + N] for t in range(T)]


def _scale(x, y, lag_min, T):
    return np.array([np.mean(p) for p in _products(x, y, lag_min, T)])


def _rratio(x, y, lag_min, T):
    return np.array([np.sqrt(np.dot(p, p)) / p.sum() for p in _products(x, y, lag_min, T)])


def _signals(L, seed):
    x = siggen.qpsk_rrc_stream(n=L, seed=seed)
    y = (np.roll(x, 9) * np.exp(2j * np.pi * 0.01 * np.arange(L)) + 0.3 * siggen.gmsk_stream(n=L, seed=seed)
         ).astype(np.complex64)
    return x, y


def _run(cy, x, y, alphas, lag_min, T, flags=0, splits=()):
    st = cy.CrossStream(alphas, lag_min, T, flags)
    dx, dy = torch.from_numpy(x).to("cuda"), torch.from_numpy(y).to("cuda")
    cuts = [0] + sorted(splits) + [x.size]
    for a, b in zip(cuts[:-1], cuts[1:]):
        if b > a:
            st.push2(dx[a:b], dy[a:b])
    R, Rc, n = st.read()
    torch.cuda.synchronize()
    st.close()
    return R.cpu().numpy(), Rc.cpu().numpy(), n


@pytest.mark.parametrize("lag_min,T", [(-7, 16), (0, 37), (5, 8), (-40, 81)])
@pytest.mark.parametrize("flags", [0, 1, 2])
def test_cross_tables_match_oracle(cy, lag_min, T, flags):
    L = 3 * 4096 + 123 + T + abs(lag_min)
    x, y = _signals(L, 12)
    alphas = np.concatenate([np.linspace(-0.5, 0.5, 61, endpoint=False), [0.0, 0.01, 0.25, -0.125, 1 / 3]])
    Ro, Rco, no = cross_tables(x, y, alphas, lag_min, T)
    R, Rc, n = _run(cy, x, y, alphas, lag_min, T, flags)
    assert n == no
    sc = _scale(x, y, lag_min, T)[:, None]
    r = _rratio(x, y, lag_min, T)[:, None]
    e = max(np.max(np.abs(R - Ro) / sc), np.max(np.abs(Rc - Rco) / sc))
    ratio = max(np.max(np.abs(R - Ro) / sc / bound(flags, 4096, r, np.abs(Ro) / sc)),
                np.max(np.abs(Rc - Rco) / sc / bound(flags, 4096, r, np.abs(Rco) / sc)))
    print(f"  lag_min={lag_min} T={T} flags={flags}: max scaled error {e:.2e}, error/bound {ratio:.3f}",
          flush=True)
    assert ratio <= 1.0


@pytest.mark.parametrize("flags", [0, 1])
def test_cross_segmentation_bitwise(cy, flags):
    lag_min, T = -13, 24
    L = 2 * 4096 + 777
    x, y = _signals(L, 13)
    alphas = np.linspace(-0.5, 0.5, 130, endpoint=False)
    R, Rc, n = _run(cy, x, y, alphas, lag_min, T, flags)
    rng = np.random.default_rng(flags)
    cuts = list(rng.integers(0, L, size=11)) + [1, 5, 12, 13, 14, 36, 37, 4096, 4096 + 37]
    R2, Rc2, n2 = _run(cy, x, y, alphas, lag_min, T, flags, splits=cuts)
    assert n2 == n and np.array_equal(R2, R) and np.array_equal(Rc2, Rc)


def test_delayed_copy_is_a_phase_shifted_autocorrelation(cy):
    # y[k] = x[k - d]: lags -d .. -d + T - 1 of (x, y) equal exp(-j2pi alpha d) times
    # lags 0 .. T-1 of x alone over the same products, up to FP32 rounding
    d, T, L = 11, 32, 20000
    x = siggen.gmsk_stream(n=L)
    y = np.concatenate([np.zeros(d, np.complex64), x[:L - d]]).astype(np.complex64)
    alphas = np.arange(128) / 128.0
    Rxy, Rcxy, n = _run(cy, x, y, alphas, -d, T)
    st = cy.CyclicStream(alphas, T, 0)
    st.push(torch.from_numpy(np.ascontiguousarray(x[:n + T - 1])).to("cuda"))
    Rs, Rcs, ns = st.read()
    torch.cuda.synchronize()
    st.close()
    assert ns == n == L - (T - 1) - d
    ph = np.exp(-2j * np.pi * alphas * d)[None, :]
    sc = _scale(x[:n + T - 1], x[:n + T - 1], 0, T)[:, None]
    e = max(np.max(np.abs(Rxy - ph * Rs.cpu().numpy()) / sc), np.max(np.abs(Rcxy - ph * Rcs.cpu().numpy()) / sc))
    print(f"  delayed copy: max scaled difference {e:.2e}", flush=True)
    assert e <= 2e-5


def test_one_input_lag0_equals_single_state_bitwise(cy):
    x = siggen.qpsk_rrc_stream(n=9000, seed=14)
    alphas = np.linspace(-0.5, 0.5, 70, endpoint=False)
    T = 20
    d = torch.from_numpy(x).to("cuda")
    a = cy.CrossStream(alphas, 0, T, 1)
    a.push(d[:3000])
    a.push2(d[3000:], d[3000:])
    Ra, Rca, na = a.read()
    b = cy.CyclicStream(alphas, T, 1)
    b.push(d)
    Rb, Rcb, nb = b.read()
    torch.cuda.synchronize()
    a.close()
    b.close()
    assert na == nb and torch.equal(Ra, Rb) and torch.equal(Rca, Rcb)


def test_cross_edge_cases(cy):
    alphas = np.array([0.0, 0.1, -0.3])
    x, y = _signals(300, 15)
    # lag range longer than the record: nothing to sum
    R, Rc, n = _run(cy, x, y, alphas, -250, 60)
    assert n == 0 and not np.abs(R).any() and not np.abs(Rc).any()
    # one-sample pushes
    R1, Rc1, n1 = _run(cy, x, y, alphas, -3, 5, splits=list(range(1, 300)))
    R2, Rc2, n2 = _run(cy, x, y, alphas, -3, 5)
    assert n1 == n2 == 300 - 4 - 3 and np.array_equal(R1, R2) and np.array_equal(Rc1, Rc2)
    Ro, Rco, _ = cross_tables(x, y, alphas, -3, 5)
    sc = _scale(x, y, -3, 5)[:, None]
    assert max(np.max(np.abs(R1 - Ro) / sc), np.max(np.abs(Rc1 - Rco) / sc)) <= FP32_TOL
    # two-input push on a one-input state is rejected
    st = cy.CyclicStream(alphas, 4, 0)
    d = torch.from_numpy(x).to("cuda")
    with pytest.raises(cy.CycloError):
        cy._check(cy.lib().cyc_push2(st._s, cy.ctypes.c_void_p(d.data_ptr()), cy.ctypes.c_void_p(d.data_ptr()),
                                     10, None), "cyc_push2")
    st.close()


@pytest.mark.parametrize("flags", [1, 2])
def test_cross_push_coalescing_bitwise(cy, flags, monkeypatch):
    """Two inputs with lags of either sign: pushes that coalesce until five
    1024-product chunks are pending (both inputs' pending buffers then hold
    more than a chunk) give the bits of committing at every push, and match
    the oracle."""
    lag_min, T = -19, 40
    L = 30000
    x, y = _signals(L, 14)
    alphas = np.linspace(-0.5, 0.5, 150, endpoint=False)
    monkeypatch.setenv("CYC_CHUNK", "1024")
    monkeypatch.setenv("CYC_COALESCE", "0")
    ref = _run(cy, x, y, alphas, lag_min, T, flags)
    monkeypatch.setenv("CYC_COALESCE", "5000")
    rng = np.random.default_rng(20 + flags)
    for trial in range(2):
        cuts = list(rng.integers(1, L, size=6 + 10 * trial)) + [4000, 5200, 9000]
        got = _run(cy, x, y, alphas, lag_min, T, flags, splits=cuts)
        assert got[2] == ref[2] and np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), trial
    Ro, Rco, no = cross_tables(x, y, alphas, lag_min, T)
    assert ref[2] == no
    sc = _scale(x, y, lag_min, T)[:, None]
    r = _rratio(x, y, lag_min, T)[:, None]
    ratio = max(np.max(np.abs(ref[0] - Ro) / sc / bound(flags, 1024, r, np.abs(Ro) / sc)),
                np.max(np.abs(ref[1] - Rco) / sc / bound(flags, 1024, r, np.abs(Rco) / sc)))
    assert ratio <= 1.0
