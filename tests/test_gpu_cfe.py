"""GPU cycle-frequency estimation against the FP64 oracle (oracle/cfe.py).

* Detection (scales, statistic, candidates, leakage masking) on a table the
  oracle made, rounded to complex64 and fed to both sides: the scales must be
  bitwise equal and the detected bins identical (every decision is FP64 on
  the same values).
* Refinement on an oracle zoom table: identical zoom indices.
* The whole estimator from samples: the same detected bins as the oracle's
  estimate, and each alpha_hat within one zoom step of the oracle's (the GPU
  zoom table is FP32, so near-equal zoom columns may swap) and within three
  of the closed-form location.
"""
import ctypes

import numpy as np
import pytest

from oracle import cfe
from oracle.cyclic import cyclic_tables

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N, T, Z = 4096, 4, 16


@pytest.fixture(scope="module")
def cy():
    from paper_2405_16911_amd import cyclo
    assert torch.cuda.is_available()
    cyclo.lib()
    return cyclo


def _noise(rng, n, var):
    return (rng.standard_normal(n) + 1j * rng.standard_normal(n)) * np.sqrt(var / 2)


def _signals():
    rng = np.random.default_rng(21)
    n = np.arange(N)
    tone = np.exp(2j * np.pi * 0.0873 * n) + _noise(rng, N, 0.1)
    two = np.exp(2j * np.pi * 0.0873 * n) + 0.7 * np.exp(2j * np.pi * -0.1311 * n) + _noise(rng, N, 0.1)
    bits = rng.choice([-1.0, 1.0], size=N // 4 + 1)
    bpsk = np.repeat(bits, 4)[:N] * np.exp(2j * np.pi * 0.0311 * n) + _noise(rng, N, 0.05)
    strong = np.exp(2j * np.pi * 0.0873 * n) + _noise(rng, N, 0.01)
    noise = _noise(rng, N, 1.0)
    return {"tone": (tone, [], [2 * 0.0873]),
            "two_tones": (two, [0.0873 + 0.1311, -0.0873 - 0.1311], [2 * 0.0873, -2 * 0.1311, 0.0873 - 0.1311]),
            "bpsk": (bpsk, [0.25, 0.5, 0.75], [0.0622 + k / 4 for k in range(4)]),
            "strong_tone": (strong, [], [2 * 0.0873]),
            "noise": (noise, [], [])}


SIG = _signals()
CASES = [(name, which, A) for name in SIG for which in ("R", "Rc") for A in (4096,)] + \
        [("strong_tone", "Rc", 8192), ("bpsk", "R", 4160)]


@pytest.mark.parametrize("name,which,A", CASES)
def test_detection_on_the_same_table(cy, name, which, A):
    x = SIG[name][0].astype(np.complex64)
    alphas = np.array([-0.5 + k / A for k in range(A)])
    R, Rc, n_used = cyclic_tables(x, alphas, T)
    tab = (R if which == "R" else Rc).astype(np.complex64)
    excl = cfe.zero_bin(-0.5, A) if which == "R" else None
    ref, ref_sigma = cfe.detect(tab, 7.0, n_used, excl)
    bins, sigma, n = cy.cyc_cfe_detect(torch.from_numpy(tab).to("cuda"), n_used, 7.0,
                                       -1 if excl is None else excl, 256)
    print(f"  {name} {which} A={A}: {n} detections {bins.tolist()}", flush=True)
    assert np.array_equal(sigma.cpu().numpy(), ref_sigma)
    assert n == ref.size and bins.tolist() == ref.tolist()


def test_refinement_on_the_same_zoom_table(cy):
    x = SIG["two_tones"][0].astype(np.complex64)
    A = 4096
    alphas = np.array([-0.5 + k / A for k in range(A)])
    R, Rc, n_used = cyclic_tables(x, alphas, T)
    tab = Rc.astype(np.complex64)
    bins, sigma_ref = cfe.detect(tab, 7.0, n_used)
    zg = np.concatenate([cfe.zoom_grid(alphas[k], A, Z) for k in bins])
    _, Rcz, _ = cyclic_tables(x, zg, T)
    Rcz = Rcz.astype(np.complex64)
    W = 2 * Z + 1
    d_bins = torch.from_numpy(bins.astype(np.int32)).to("cuda")
    d_sigma = torch.from_numpy(sigma_ref).to("cuda")
    dj = torch.empty(bins.size, dtype=torch.int32, device="cuda")
    dq = torch.empty(bins.size, dtype=torch.float64, device="cuda")
    p = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    Rz_d = torch.from_numpy(Rcz).to("cuda")
    assert cy.lib().cyc_cfe_refine(p(Rz_d), T, int(bins.size), Z, p(d_bins), p(d_sigma), A, p(dj), p(dq), None) == 0
    torch.cuda.synchronize()
    for i, k in enumerate(bins):
        j, q = cfe.refine(Rcz[:, i * W:(i + 1) * W], sigma_ref[:, k // 64])
        assert int(dj[i]) == j and float(dq[i]) == q, (k, int(dj[i]), j)


def _wrap(a):
    return (np.asarray(a, dtype=np.float64) + 0.5) % 1.0 - 0.5


@pytest.mark.parametrize("name,which,A", CASES)
def test_estimator_from_samples(cy, name, which, A):
    x = SIG[name][0].astype(np.complex64)
    got, n = cy.cyc_estimate_cycle_freqs(torch.from_numpy(x).to("cuda"), -0.5, A, T, which, 7.0, Z)
    ref = cfe.estimate(x, T, -0.5, A, Z=Z, which=which)
    print(f"  {name} {which} A={A}: {[(k, round(a, 6)) for k, a, _ in got]}", flush=True)
    assert n == len(ref) == len(got)
    assert [k for k, _, _ in got] == [k for k, _, _ in ref]
    step = 1.0 / (Z * A)
    for (_, a, _), (_, b, _) in zip(got, ref):
        assert abs(_wrap(a - b)) <= step * (1 + 1e-9)
    closed = SIG[name][1] if which == "R" else SIG[name][2]
    assert len(closed) == len(got)
    for a, e in zip(sorted(_wrap([a for _, a, _ in got]).tolist()), sorted(_wrap(closed).tolist())):
        assert abs(_wrap(a - e)) <= 3 * step


def test_estimator_limits_and_errors(cy):
    x = torch.from_numpy(SIG["bpsk"][0].astype(np.complex64)).to("cuda")
    got, n = cy.cyc_estimate_cycle_freqs(x, -0.5, 4096, T, "Rc", 7.0, Z, max_out=2)
    assert n == 4 and len(got) == 2
    full, _ = cy.cyc_estimate_cycle_freqs(x, -0.5, 4096, T, "Rc", 7.0, Z)
    assert got == full[:2]
    L = cy.lib()
    cnt = ctypes.c_int32(0)
    # a grid coarser than 1/N_used is refused
    assert L.cyc_estimate_cycle_freqs(ctypes.c_void_p(x.data_ptr()), N, -0.5, 2048, T, 0, 7.0, Z, 1, 0, None, None,
                                      None, ctypes.byref(cnt), None) == cy.CYC_EINVAL
    assert L.cyc_estimate_cycle_freqs(ctypes.c_void_p(x.data_ptr()), N, -0.5, 4100, T, 0, 7.0, Z, 1, 0, None, None,
                                      None, ctypes.byref(cnt), None) == cy.CYC_EINVAL
