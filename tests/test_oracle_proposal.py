"""Pins of the proposal oracle (no GPU): finite differences for every gradient,
the convolution against a direct loop, AdamW against a hand-stepped scalar,
spectra against a tone's known line, and selection corner cases."""
import numpy as np
import pytest

from oracle import proposal as P


def _tiny(seed=0, N=3, C_in=3, C=4, K=7, L=16, n_out=16, n_conv=2):
    rng = np.random.default_rng(seed)
    p = P.init_params(rng, C_in=C_in, C=C, K=K, L=L, n_out=n_out, n_conv=n_conv)
    for k in p:
        if k.startswith("b"):
            p[k] = rng.standard_normal(p[k].shape) * 0.1
    X = rng.standard_normal((N, C_in, L))
    y = (rng.random((N, n_out)) < 0.3).astype(float)
    return p, X, y


def test_conv_against_direct_loop():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 3, 9))
    W = rng.standard_normal((4, 3, 5))
    b = rng.standard_normal(4)
    y = P.conv_circ(x, W, b)
    for n in range(2):
        for o in range(4):
            for t in range(9):
                ref = b[o] + sum(W[o, i, k] * x[n, i, (t + k - 2) % 9] for i in range(3) for k in range(5))
                assert abs(y[n, o, t] - ref) < 1e-12


def test_gradients_by_central_differences():
    n_conv = 2
    p, X, y = _tiny(n_conv=n_conv)
    z, cache = P.forward(p, X, n_conv)
    g = P.backward(p, cache, z, y, n_conv)
    h = 1e-6
    rng = np.random.default_rng(2)
    for k in p:
        flat = p[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = P.bce_loss(P.forward(p, X, n_conv)[0], y)
            flat[idx] = old - h
            lm = P.bce_loss(P.forward(p, X, n_conv)[0], y)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = g[k].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1e-4, abs(fd)) + 1e-9, (k, idx, fd, an)


def test_local_layer_reads_the_bins_own_position():
    # with the dense layer zeroed, logit j is b_j + sum_c Wl[c] * relu(last conv)[c, j]
    p, X, _ = _tiny(n_conv=2)
    p["Wh"][:] = 0.0
    z, cache = P.forward(p, X, 2)
    a = cache["acts"][-1]
    for n in range(X.shape[0]):
        for j in range(16):
            ref = p["bh"][j] + sum(p["Wl"][c] * a[n, c, j] for c in range(4))
            assert abs(z[n, j] - ref) < 1e-12


def test_adamw_first_steps_scalar():
    p = {"w": np.array([0.5])}
    g = {"w": np.array([0.2])}
    m = {"w": np.zeros(1)}
    v = {"w": np.zeros(1)}
    P.adamw_step(p, g, m, v, 1, lr=0.1, wd=0.01)
    # bias-corrected first step: m_hat = g, v_hat = g^2 -> step lr * (sign(g) + wd * w)
    assert abs(p["w"][0] - (0.5 - 0.1 * (0.2 / (0.2 + 1e-8) + 0.01 * 0.5))) < 1e-12


def test_spectra_of_a_tone():
    f = 37 / 1024                       # on a bin
    n = np.arange(64 * 1024)
    x = np.exp(2j * np.pi * f * n)
    S = P.welch_log_spectra(x)
    assert np.argmax(S[0]) == 512 + 37       # x: line at f
    assert np.argmax(S[1]) == 512 + 74       # x^2: line at 2f
    assert np.argmax(S[2]) == 512            # |x|^2 = 1: line at 0
    for c in range(3):
        assert abs(S[c].mean()) < 1e-9 and abs(S[c].std() - 1) < 1e-6


def test_selection_ties_wrap_and_zero_bin():
    p = np.zeros(32)
    p[[0, 5, 31]] = 0.9                       # tie: lower indices first
    p[10] = 0.95
    sel, conf = P.select(p, k=3, width=1, zero_bin=16)
    assert list(sel) == [0, 1, 4, 5, 6, 9, 10, 11, 16, 31]   # 31 is 0's circular neighbour
    assert conf == 1.0
    sel1, conf1 = P.select(p, k=3, width=0, zero_bin=16)
    assert list(sel1) == [0, 5, 10, 16]
    assert abs(conf1 - (1 - 0.9)) < 1e-12     # bin 31 (0.9) was left out
    sel2, conf2 = P.select(p, k=4, width=1)
    assert 30 in sel2 and 31 in sel2 and conf2 == 1.0


def test_selection_non_finite_probabilities_fall_back():
    p = np.zeros(32)
    p[[3, 20]] = 0.8
    p[7] = np.nan
    sel, conf = P.select(p, k=2, width=0)
    assert list(sel) == [3, 20] and conf == 0.0   # NaN never chosen; no confidence
    sel, conf = P.select(np.full(8, np.nan), k=2, width=1, zero_bin=4)
    assert list(sel) == [4] and conf == 0.0
    q = p.copy()
    q[7] = np.inf
    sel, conf = P.select(q, k=1, width=0)
    assert list(sel) == [7] and conf == 0.0
    q[7] = 0.1
    assert P.select(q, k=2, width=0)[1] == pytest.approx(0.9)


def test_labels_exclude_power_bin():
    rng = np.random.default_rng(3)
    A, n_coarse = 256, 16
    R = (rng.standard_normal((4, A)) + 1j * rng.standard_normal((4, A))) * 0.01
    Rc = R.copy() * 0.5
    R[:, 128] = 5.0          # power term at alpha = 0 (coarse bin 8)
    R[2, 40] = 1.0           # a feature in coarse bin 2
    Rc[0, 250] = 1.0         # a conjugate feature in coarse bin 15
    lab = P.coarse_labels(R, Rc, n_coarse, zero_bin=8)
    assert list(np.nonzero(lab)[0]) == [2, 15]


def test_peak_rule_uses_the_rayleigh_median():
    # sigma = median / sqrt(2 ln 2); threshold 7 sigma.  With 3 coarse bins every
    # window holds the whole row.
    c = np.sqrt(2 * np.log(2))
    # 11 ones and an 8: median 1 -> threshold 7/c = 5.95 flags the 8
    # (the mean 1.58 would give 9.4 and flag nothing).
    row = np.array([1.0] * 11 + [8.0])
    assert list(np.nonzero(P.peak_cells(row[None, :], 3)[0])[0]) == [11]
    # even count: the mean of the two middle values (1.5) -> threshold 8.92;
    # the upper middle (2) would miss the 10, the lower middle (1) would flag the 7.
    base = [0.5] * 5 + [1.0, 2.0] + [3.0] * 4
    pk = P.peak_cells(np.array([base + [10.0], base + [7.0]]), 3)
    assert pk[0].tolist() == [False] * 11 + [True]
    assert not pk[1].any()
    assert abs(7 * 1.5 / c - 8.9177) < 1e-3


def test_peak_rule_noise_scale_is_local():
    # 8 coarse bins of 4: a pedestal of 10 over bins 0..3, 1 elsewhere.  The
    # window of bin c is bins c-1..c+1 (circular).
    row = np.ones(32)
    row[:16] = 10.0
    row[5] = 30.0      # bin 1: local median 10 -> threshold 59 -> no peak
    row[26] = 6.0      # bin 6: local median 1 -> threshold 5.95 -> peak
    pk = P.peak_cells(row[None, :], 8)[0]
    assert list(np.nonzero(pk)[0]) == [26]
    # a global median (5.5 -> threshold 32.7) would flag neither; the window
    # edges (bins 3, 4 and 7, 0) raise no peak at the pedestal's steps
    sig = P.local_sigma(row[None, :], 8)[0] * np.sqrt(2 * np.log(2))
    assert sig.tolist() == [10, 10, 10, 10, 1, 1, 1, 1]


def test_peak_rule_noise_scale_is_rayleigh():
    # complex Gaussian noise of scale s: |R| is Rayleigh(s); the estimate recovers s,
    # so the false-alarm rate at 3 sigma is exp(-9/2)
    rng = np.random.default_rng(7)
    s = 0.37
    R = s * (rng.standard_normal((2, 200000)) + 1j * rng.standard_normal((2, 200000)))
    frac = P.peak_cells(R, 1000, thresh=3.0).mean()
    assert abs(frac - np.exp(-4.5)) < 0.1 * np.exp(-4.5)


# ----------------------------------------------------------------------------- running-error bound of the network


def _bf16(v):
    """Round to BF16 (nearest, ties to even) from the FP32 value the GPU holds."""
    b = np.asarray(v, dtype=np.float64).astype(np.float32).view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def _f32(v):
    return np.asarray(v, dtype=np.float64).astype(np.float32).astype(np.float64)


def _emulated_bf16_gradients(p, X, y, n_conv=4):
    """The network with BF16 operands at every matrix product and FP32 results,
    in the GPU's order of steps (a NumPy emulation, for pinning the bound)."""
    B, L = X.shape[0], X.shape[2]
    q = {k: _bf16(v) for k, v in p.items()}
    acts, pre = [X], []
    a = X
    for i in range(n_conv):
        u = _f32(P.conv_circ(_bf16(a), q[f"W{i}"], np.zeros(p[f"W{i}"].shape[0])))
        u = _f32(u + p[f"b{i}"][None, :, None])
        pre.append(u)
        a = np.maximum(u, 0.0)
        acts.append(a)
    h = a.reshape(B, -1)
    z = _f32(_bf16(h) @ q["Wh"].T)
    z = _f32(z + _f32(np.einsum("c,ncj->nj", p["Wl"], a)))
    z = _f32(z + p["bh"][None, :])
    prob = _f32(1.0 / (1.0 + np.exp(-z)))
    dz = _f32(_f32(prob - y) / z.size)
    g = {"Wh": _f32(_bf16(dz).T @ _bf16(h)), "bh": _f32(dz.sum(axis=0)),
         "Wl": _f32(np.einsum("nj,ncj->c", dz, a))}
    dh = _f32(_bf16(dz) @ q["Wh"])
    da = _f32(dh.reshape(a.shape) + p["Wl"][None, :, None] * dz[:, None, :])
    for i in reversed(range(n_conv)):
        du = da * (pre[i] > 0)
        g[f"W{i}"] = _f32(P.conv_circ_backward(_bf16(acts[i]), q[f"W{i}"], _bf16(du))[1])
        g[f"b{i}"] = _f32(du.sum(axis=(0, 2)))
        if i > 0:
            da = _f32(P.conv_circ_backward(acts[i], q[f"W{i}"], _bf16(du))[0])
    return prob, g


def _small_net(seed):
    rng = np.random.default_rng(seed)
    p = P.init_params(rng, C_in=3, C=8, K=7, L=64, n_out=64)
    for k in p:
        if k.startswith("b"):
            p[k] = rng.standard_normal(p[k].shape) * 0.05
        p[k] = _f32(p[k])
    X = _f32(rng.standard_normal((3, 3, 64)))
    y = (rng.random((3, 64)) < 0.1).astype(np.float64)
    return p, X, y


def _noise_check(p, X, y, prob_e, g_e, u, trials=24, seed=0):
    """Per-tensor energy ratio Q = |err|^2 / |model rms|^2 and the worst
    per-element ratio err / (10 model rms + FP32 floor) of an emulated run."""
    z, cache = P.forward(p, X)
    g = P.backward(p, cache, z, y)
    sp, sg = P.rounding_noise_scale(p, X, y, u, trials, seed)
    mz, mg = P.gradient_magnitude_sums(p, X, y)
    out = {}
    for k, got, ref, s, m in [("prob", prob_e, P.sigmoid(z), sp, mz)] + [(k, g_e[k], g[k], sg[k], mg[k]) for k in g]:
        err = np.abs(got - ref)
        q = float(np.sum(err ** 2) / max(np.sum(s ** 2), 1e-300))
        worst = float(np.max(err / (10 * s + 1e-4 * m + 1e-300)))
        out[k] = (q, worst)
    return out


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_rounding_noise_model_covers_emulated_bf16_arithmetic(seed):
    """The GPU test holds each BF16 tensor to |err|^2 <= 4 |model rms|^2 and each
    element to 10 model rms (plus an FP32 floor); a NumPy emulation of the
    BF16 arithmetic (round-to-nearest-even operands at every product, FP32
    results) meets both, and a model with an eighth of the rounding does not."""
    p, X, y = _small_net(seed)
    prob_e, g_e = _emulated_bf16_gradients(p, X, y)
    res = _noise_check(p, X, y, prob_e, g_e, 2.0 ** -8)
    for k, (q, worst) in res.items():
        assert q <= 4.0 and worst <= 1.0, (k, q, worst)
    assert max(q for q, _ in res.values()) > 0.05      # the model is not vacuous
    small = _noise_check(p, X, y, prob_e, g_e, 2.0 ** -11)
    assert max(q for q, _ in small.values()) > 4.0


def test_rounding_noise_model_vanishes_without_rounding():
    p, X, y = _small_net(4)
    sp, sg = P.rounding_noise_scale(p, X, y, 0.0, 2, 0)
    assert np.all(sp == 0) and all(np.all(v == 0) for v in sg.values())
