"""GPU parity of the uniform-grid form (fold + FFT) against the FP64 oracle.

Tolerance: both sides are FP64 (the GPU folds FP32 samples in FP64 and takes
FP64 FFTs); the a-priori bound of an N-term FP64 sum is N u = 2^24 * 2^-53 ~
1.9e-9 of the scaled error, so parity is held to 1e-9 (measured values are
printed).  Segmentations of the same record are bitwise equal.
"""
import numpy as np
import pytest

from oracle.cyclic import cyclic_cell, cyclic_tables, scale_per_lag
from paper_2405_16911_amd import siggen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-9


@pytest.fixture(scope="module")
def cy():
    from paper_2405_16911_amd import cyclo
    assert torch.cuda.is_available()
    cyclo.lib()
    return cyclo


def _run(cy, x, alpha0, A, T, splits=(), flags=0):
    g = cy.GridStream(alpha0, A, T, flags)
    d = torch.from_numpy(np.ascontiguousarray(x)).to("cuda")
    cuts = [0] + sorted(splits) + [x.size]
    for a, b in zip(cuts[:-1], cuts[1:]):
        if b > a:
            g.push(d[a:b])
    R, Rc, n = g.read()
    torch.cuda.synchronize()
    out = (R.cpu().numpy(), Rc.cpu().numpy(), n)
    g.close()
    return out


def _err(x, T, R, Rc, Ro, Rco):
    sc = scale_per_lag(x, T)[:, None]
    return max(np.max(np.abs(R - Ro) / sc), np.max(np.abs(Rc - Rco) / sc))


def test_gmsk_grid_128_full_table(cy):
    x = siggen.gmsk_stream()
    T, A = 32, 128
    Ro, Rco, no = cyclic_tables(x, np.arange(A) / A, T)
    R, Rc, n = _run(cy, x, 0.0, A, T, flags=cy.CYC_OUT_C128)
    assert n == no
    e = _err(x, T, R, Rc, Ro, Rco)
    print(f"  A=128 max scaled error {e:.2e}", flush=True)
    assert e <= TOL


@pytest.mark.parametrize("A,T,alpha0", [(4096, 37, -0.5), (256, 5, 0.3125), (2, 1, 0.0), (8192, 16, 0.123456789)])
def test_ragged_full_tables_and_segmentation(cy, A, T, alpha0):
    x = siggen.qpsk_rrc_stream(n=3 * 4096 + 123 + T, seed=11)
    alphas = alpha0 + np.arange(A) / A
    Ro, Rco, no = cyclic_tables(x, alphas, T)
    R, Rc, n = _run(cy, x, alpha0, A, T, flags=cy.CYC_OUT_C128)
    assert n == no
    e = _err(x, T, R, Rc, Ro, Rco)
    print(f"  A={A} T={T} max scaled error {e:.2e}", flush=True)
    assert e <= TOL
    rng = np.random.default_rng(A + T)
    cuts = list(rng.integers(0, x.size, size=9)) + [1, 2, T - 1, T, T + 1]
    R2, Rc2, n2 = _run(cy, x, alpha0, A, T, splits=cuts, flags=cy.CYC_OUT_C128)
    assert n2 == n and np.array_equal(R2, R) and np.array_equal(Rc2, Rc)


@pytest.mark.parametrize("A", [16384, 65536])
def test_large_grids_two_stage_fft_sampled_cells(cy, A):
    # A > 8192: 8192-point LDS FFTs plus a radix-A/8192 combining pass
    T = 4
    x = siggen.mixed_stream(5, 7, n=70000)[0]
    R, Rc, n = _run(cy, x, -0.5, A, T, flags=cy.CYC_OUT_C128)
    sc = scale_per_lag(x, T)
    rng = np.random.default_rng(A)
    ks = sorted(set([0, 1, A // 2, A - 1, A // 3] + list(rng.integers(0, A, size=19))))
    worst = 0.0
    for k in ks:
        a = -0.5 + k / A
        for t in (0, T - 1):
            r, rc = cyclic_cell(x, a, t, T)
            worst = max(worst, abs(R[t, k] - r) / sc[t], abs(Rc[t, k] - rc) / sc[t])
    print(f"  A={A} sampled max scaled error {worst:.2e}", flush=True)
    assert worst <= TOL
    # the alpha = 0 cell at lag 0 is the mean power
    assert abs(R[0, A // 2] - np.mean(np.abs(x[:n].astype(np.complex128)) ** 2)) <= TOL * sc[0]


def test_agrees_with_the_dense_path(cy):
    x = siggen.qpsk_rrc_stream(n=50000, seed=3)
    T, A = 64, 1024
    alphas = -0.5 + np.arange(A) / A
    Rg, Rcg, n = _run(cy, x, -0.5, A, T)
    st = cy.CyclicStream(alphas, T, cy.CYC_OP_FP32)
    st.push(torch.from_numpy(x).to("cuda"))
    Rd, Rcd, nd = st.read()
    torch.cuda.synchronize()
    st.close()
    assert nd == n
    sc = scale_per_lag(x, T)[:, None]
    e = max(np.max(np.abs(Rd.cpu().numpy() - Rg) / sc), np.max(np.abs(Rcd.cpu().numpy() - Rcg) / sc))
    print(f"  dense FP32 vs grid: max scaled difference {e:.2e}", flush=True)
    assert e <= 1e-5


def test_edge_cases(cy):
    T, A = 8, 64
    x = siggen.gmsk_stream()[:5]          # fewer samples than lags: nothing to sum
    R, Rc, n = _run(cy, x, 0.0, A, T)
    assert n == 0 and not np.abs(R).any() and not np.abs(Rc).any()
    # one-sample pushes, then reset equals a fresh state
    x = siggen.gmsk_stream()[:300]
    g = cy.GridStream(0.25, A, T, cy.CYC_OUT_C128)
    d = torch.from_numpy(x).to("cuda")
    for i in range(x.size):
        g.push(d[i:i + 1])
    R1, Rc1, n1 = g.read()
    g.reset()
    g.push(d)
    R2, Rc2, n2 = g.read()
    # the fold bins are cleared by the first push after a reset, whatever it holds:
    # two resets, a read of the empty state, a push too short to complete a product
    g.reset()
    g.reset()
    R0, Rc0, n0 = g.read()
    g.push(d[:3])
    g.push(d[3:])
    R3, Rc3, n3 = g.read()
    torch.cuda.synchronize()
    g.close()
    assert n0 == 0 and not R0.abs().any() and not Rc0.abs().any()
    assert n1 == n2 == n3 == x.size - T + 1
    assert torch.equal(R1, R2) and torch.equal(Rc1, Rc2)
    assert torch.equal(R1, R3) and torch.equal(Rc1, Rc3)
    Ro, Rco, _ = cyclic_tables(x, 0.25 + np.arange(A) / A, T)
    assert _err(x, T, R1.cpu().numpy(), Rc1.cpu().numpy(), Ro, Rco) <= TOL


def test_invalid_arguments(cy):
    with pytest.raises(cy.CycloError):
        cy.GridStream(0.0, 100, 4)       # not a power of two
    with pytest.raises(cy.CycloError):
        cy.GridStream(0.0, 1 << 17, 4)   # too large
    with pytest.raises(cy.CycloError):
        cy.GridStream(float("nan"), 64, 4)


@pytest.mark.parametrize("lag_min,T,A", [(-9, 20, 512), (4, 6, 128), (-300, 8, 16384)])
def test_two_inputs_match_the_cross_oracle(cy, lag_min, T, A):
    from oracle.cyclic import cross_tables
    L = 9000 + abs(lag_min)
    x = siggen.qpsk_rrc_stream(n=L, seed=21)
    y = (np.roll(x, 5) + 0.5 * siggen.gmsk_stream(n=L, seed=22)).astype(np.complex64)
    alpha0 = -0.5
    ks = np.arange(A) if A <= 512 else np.unique(np.concatenate([[0, A // 2, A - 1],
                                                                  np.random.default_rng(A).integers(0, A, 30)]))
    Ro, Rco, no = cross_tables(x, y, alpha0 + ks / A, lag_min, T)
    g = cy.GridStream(alpha0, A, T, cy.CYC_OUT_C128, lag_min=lag_min)
    dx, dy = torch.from_numpy(x).to("cuda"), torch.from_numpy(y).to("cuda")
    for a, b in ((0, 1), (1, 333), (333, 4000), (4000, L)):
        g.push2(dx[a:b], dy[a:b])
    R, Rc, n = g.read()
    torch.cuda.synchronize()
    g.close()
    assert n == no
    R, Rc = R.cpu().numpy()[:, ks], Rc.cpu().numpy()[:, ks]
    ax, ay = np.abs(x.astype(np.complex128)), np.abs(y.astype(np.complex128))
    dxo, dyo = max(0, lag_min), max(0, -lag_min)
    sc = np.array([np.mean(ax[dxo + t: dxo + t + n] * ay[dyo: dyo + n]) for t in range(T)])[:, None]
    e = max(np.max(np.abs(R - Ro) / sc), np.max(np.abs(Rc - Rco) / sc))
    print(f"  two inputs lag_min={lag_min} A={A}: max scaled error {e:.2e}", flush=True)
    assert e <= TOL
