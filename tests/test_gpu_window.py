"""GPU parity of the sliding-window form against the FP64 oracle.

Tolerances as the cumulative tables (tests/_bounds.py), per cell, with the
scale and random-walk factor over the window's products.  Any segmentation of the record gives the
same bits; the window slides hop by hop and wraps its ring many times.
"""
import numpy as np
import pytest

from _bounds import bound
from oracle.cyclic import roundoff_ratio_per_lag, scale_per_lag, window_tables
from paper_2405_16911_amd import siggen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

@pytest.fixture(scope="module")
def cy():
    from paper_2405_16911_amd import cyclo
    assert torch.cuda.is_available()
    cyclo.lib()
    return cyclo


def _window_samples(x, T, hop, n_hops):
    N = max(0, x.size - T + 1)
    c = N // hop
    W = min(n_hops, c)
    n_w = (c - W) * hop
    return x[n_w: n_w + W * hop + T - 1]


def _window_scale(x, T, hop, n_hops):
    return scale_per_lag(_window_samples(x, T, hop, n_hops), T)


@pytest.mark.parametrize("flags", [0, 1])
@pytest.mark.parametrize("hop,n_hops,T", [(512, 4, 16), (4096, 2, 37), (64, 9, 5)])
def test_window_matches_oracle_as_it_slides(cy, flags, hop, n_hops, T):
    x = siggen.qpsk_rrc_stream(n=6 * 4096 + 777, seed=31)
    alphas = np.concatenate([np.linspace(-0.5, 0.5, 67, endpoint=False), [0.0, 0.25, 1 / 3]])
    st = cy.WindowStream(alphas, T, hop, n_hops, flags)
    d = torch.from_numpy(x).to("cuda")
    rng = np.random.default_rng(hop + T)
    cuts = sorted(set([0, x.size] + list(rng.integers(1, x.size, size=7)) + [hop - 1, hop + T - 1]))
    worst = 0.0
    for a, b in zip(cuts[:-1], cuts[1:]):
        st.push(d[a:b])
        R, Rc, n = st.read()
        torch.cuda.synchronize()
        Ro, Rco, no = window_tables(x[:b], alphas, T, hop, n_hops)
        assert n == no
        if no == 0:
            assert not R.abs().any() and not Rc.abs().any()
            continue
        sc = _window_scale(x[:b], T, hop, n_hops)[:, None]
        r = roundoff_ratio_per_lag(_window_samples(x[:b], T, hop, n_hops), T)[:, None]
        eR = np.abs(R.cpu().numpy() - Ro) / sc
        eRc = np.abs(Rc.cpu().numpy() - Rco) / sc
        e = max(eR.max(), eRc.max())
        worst = max(worst, e)
        ratio = max(np.max(eR / bound(flags, 4096, r, np.abs(Ro) / sc)),
                    np.max(eRc / bound(flags, 4096, r, np.abs(Rco) / sc)))
        assert ratio <= 1.0, (b, e, ratio)
    print(f"  hop={hop} n_hops={n_hops} T={T} flags={flags}: max scaled error {worst:.2e}", flush=True)
    # one push of the whole record gives the same bits
    R1, Rc1, n1 = R, Rc, n
    st2 = cy.WindowStream(alphas, T, hop, n_hops, flags)
    st2.push(d)
    R2, Rc2, n2 = st2.read()
    torch.cuda.synchronize()
    st.close()
    st2.close()
    assert n2 == n1 and torch.equal(R1, R2) and torch.equal(Rc1, Rc2)


def test_window_reset_and_short_records(cy):
    x = siggen.gmsk_stream(n=3000)
    alphas = np.arange(32) / 32.0
    st = cy.WindowStream(alphas, 8, 1024, 2)
    d = torch.from_numpy(x).to("cuda")
    st.push(d[:1000])
    R, Rc, n = st.read()
    assert n == 0 and not R.abs().any()
    st.push(d[1000:])
    _, _, n = st.read()
    assert n == 2 * 1024
    st.reset()
    st.push(d[:1031])           # exactly one hop of products (1024 + T - 1 samples)
    R, Rc, n = st.read()
    torch.cuda.synchronize()
    st.close()
    Ro, Rco, no = window_tables(x[:1031], alphas, 8, 1024, 2)
    assert n == no == 1024
    sc = scale_per_lag(x[:1031], 8)[:, None]
    assert np.max(np.abs(R.cpu().numpy() - Ro) / sc) <= 1e-5
