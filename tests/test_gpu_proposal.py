"""GPU parity of the learned-proposal kernels against the FP64 oracle.

Tolerances: spectra (standardised log, FP32 FFT) <= 5e-3 absolute; network
probabilities, gradients and one AdamW step with FP32 operands: relative L2
error per tensor <= 1e-5 (probabilities) / 2e-5 (gradients) / 1e-3 (the step).
BF16 operands: the oracle's rounding-noise model (oracle.proposal.
perturbed_pass: every operand of every matrix product perturbed by a relative
error uniform in +-2^-8, as often as the GPU rounds it) gives each probability
and gradient element a root-mean-square deviation s over 24 draws; each tensor
must satisfy |err|^2 <= 4 |s|^2 and each element |err| <= 10 s + 1e-4 M (M: the
sum of |terms| of its last sum, an FP32 accumulation floor).  Uniform errors
overstate round-to-nearest's mean square, so the expected energy ratio is
about 0.5 (pinned on the CPU against an emulated BF16 network).
Selection and labels are bit-exact (the label kernel is fed the oracle's own
tables, rounded to complex64).
"""
import numpy as np
import pytest

from oracle import proposal as P
from oracle.cyclic import cyclic_tables
from paper_2405_16911_amd import siggen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KEYS = ["W0", "b0", "W1", "b1", "W2", "b2", "W3", "b3", "Wh", "bh", "Wl"]


@pytest.fixture(scope="module")
def cy():
    from paper_2405_16911_amd import cyclo
    assert torch.cuda.is_available()
    cyclo.lib()
    return cyclo


def _flat(p):
    return np.concatenate([p[k].reshape(-1) for k in KEYS])


def _unflat(v, like):
    out, o = {}, 0
    for k in KEYS:
        n = like[k].size
        out[k] = v[o:o + n].reshape(like[k].shape)
        o += n
    return out


def _params(seed):
    rng = np.random.default_rng(seed)
    p = P.init_params(rng)
    for k in KEYS:
        if k.startswith("b"):
            p[k] = rng.standard_normal(p[k].shape) * 0.05
        p[k] = p[k].astype(np.float32).astype(np.float64)   # the values the GPU holds
    return p


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_spectra_match_oracle(cy):
    n = 3
    xs = [siggen.mixed_stream(5, i, n=65536)[0] for i in range(n)]
    m = cy.ProposalModel(4, cy.CYC_OP_FP32)
    feat = m.spectra(torch.from_numpy(np.concatenate(xs)).to("cuda")).cpu().numpy()
    m.close()
    for i, x in enumerate(xs):
        ref = P.welch_log_spectra(x)
        err = np.abs(feat[:, i, :] - ref)
        print(f"  window {i}: max {err.max():.2e} median {np.median(err):.2e}", flush=True)
        assert err.max() < 5e-3


@pytest.mark.parametrize("flags", [0, 1])
def test_forward_and_gradients(cy, flags):
    p = _params(1)
    rng = np.random.default_rng(2)
    B = 2
    X = rng.standard_normal((B, 3, 1024)).astype(np.float32).astype(np.float64)
    y = (rng.random((B, 1024)) < 0.05).astype(np.float64)
    z, cache = P.forward(p, X)
    g = P.backward(p, cache, z, y)
    loss = P.bce_loss(z, y)
    m = cy.ProposalModel(B, flags)
    m.set_params(_flat(p))
    feat = torch.from_numpy(np.ascontiguousarray(X.transpose(1, 0, 2)).astype(np.float32)).to("cuda")
    lab = torch.from_numpy(y.astype(np.float32)).to("cuda")
    prob = m.forward(feat).cpu().numpy().astype(np.float64)
    gg, gl = m.gradients(feat, lab)
    gg = _unflat(gg.cpu().numpy().astype(np.float64), p)
    m.close()
    got = dict(gg, prob=prob)
    ref = dict(g, prob=P.sigmoid(z))
    if flags == 0:
        assert abs(gl - loss) <= 1e-5 * abs(loss)
        for k in ["prob"] + KEYS:
            e = _rel(got[k], ref[k])
            print(f"  {k}: rel {e:.2e}", flush=True)
            assert e <= (1e-5 if k == "prob" else 2e-5), k
        return
    sp, sg = P.rounding_noise_scale(p, X, y, 2.0 ** -8, trials=24, seed=7)
    mz, mg = P.gradient_magnitude_sums(p, X, y)
    sg["prob"], mg["prob"] = sp, mz
    for k in ["prob"] + KEYS:
        err = np.abs(got[k] - ref[k])
        q = float(np.sum(err ** 2) / np.sum(sg[k] ** 2))
        worst = float(np.max(err / (10 * sg[k] + 1e-4 * mg[k] + 1e-300)))
        print(f"  {k}: rel {_rel(got[k], ref[k]):.2e} energy ratio {q:.3f} worst element {worst:.3f}", flush=True)
        assert q <= 4.0 and worst <= 1.0, k
    # the loss moves by (p - y) dz / n per logit, dz = dp / (p (1 - p)): ten times
    # the noise that the probabilities' model spread implies
    pr = P.sigmoid(z)
    s_loss = np.sqrt(np.sum(((pr - y) / (pr * (1 - pr)) * sp) ** 2)) / pr.size
    print(f"  loss: error {abs(gl - loss):.2e}, model scale {s_loss:.2e}", flush=True)
    assert abs(gl - loss) <= 10 * s_loss + 1e-6 * abs(loss)


def test_adamw_step_fp32(cy):
    p = _params(3)
    rng = np.random.default_rng(4)
    B = 2
    X = rng.standard_normal((B, 3, 1024)).astype(np.float32).astype(np.float64)
    y = (rng.random((B, 1024)) < 0.05).astype(np.float64)
    z, cache = P.forward(p, X)
    g = P.backward(p, cache, z, y)
    m0 = {k: np.zeros_like(v) for k, v in p.items()}
    v0 = {k: np.zeros_like(v) for k, v in p.items()}
    ref = {k: v.copy() for k, v in p.items()}
    P.adamw_step(ref, g, m0, v0, 1, lr=1e-3, wd=1e-2)
    m = cy.ProposalModel(B, cy.CYC_OP_FP32)
    m.set_params(_flat(p))
    feat = torch.from_numpy(np.ascontiguousarray(X.transpose(1, 0, 2)).astype(np.float32)).to("cuda")
    m.train_step(feat, torch.from_numpy(y.astype(np.float32)).to("cuda"), 1e-3, 1e-2)
    got = _unflat(m.get_params().astype(np.float64), p)
    m.close()
    for k in KEYS:
        # the step itself (first AdamW step moves each weight by about lr)
        e = _rel(got[k] - p[k], ref[k] - p[k])
        assert e <= 1e-3, (k, e)


def test_selection_matches_oracle(cy):
    rng = np.random.default_rng(5)
    n = 6
    prob = rng.random((n, 1024)).astype(np.float32)
    prob[0, [3, 700, 1023]] = 0.999          # ties
    prob[1, :] = 0.5                         # all equal
    prob[2, 1020:] = 0.9999                  # wrap-around neighbourhood
    sel, conf = cy.cyc_select(torch.from_numpy(prob).to("cuda"), topk=16, width=2, zero_bin=512)
    sel, conf = sel.cpu().numpy(), conf.cpu().numpy()
    for i in range(n):
        s_ref, c_ref = P.select(prob[i].astype(np.float64), k=16, width=2, zero_bin=512)
        assert list(np.nonzero(sel[i])[0]) == list(s_ref), i
        assert abs(conf[i] - c_ref) < 1e-6


def test_selection_falls_back_on_non_finite_probabilities(cy):
    # a diverged network (NaN outputs) must not look confident
    rng = np.random.default_rng(6)
    prob = rng.random((4, 1024)).astype(np.float32) * 0.5
    prob[0, :] = np.nan                      # every bin NaN
    prob[1, 17] = np.nan                     # one NaN bin
    prob[2, [5, 900]] = np.inf               # infinite bins
    sel, conf = cy.cyc_select(torch.from_numpy(prob).to("cuda"), topk=16, width=2, zero_bin=512)
    sel, conf = sel.cpu().numpy(), conf.cpu().numpy()
    for i in range(4):
        s_ref, c_ref = P.select(prob[i].astype(np.float64), k=16, width=2, zero_bin=512)
        assert list(np.nonzero(sel[i])[0]) == list(s_ref), i
        assert abs(conf[i] - c_ref) < 1e-6, i
    assert conf[0] == 0 and conf[1] == 0 and conf[2] == 0 and conf[3] > 0
    m = cy.ProposalModel(4)
    try:
        x = torch.zeros(2 * cy.WINDOW, dtype=torch.complex64, device="cuda")
        x[5] = float("nan")                  # a non-finite sample in the first window
        bins, nb, conf, fb = m.propose(x, theta=0.5)
        assert fb.cpu().tolist()[0] == 1 and conf.cpu().tolist()[0] == 0.0
    finally:
        m.close()


@pytest.mark.parametrize("A,n_coarse,zero_bin", [(4096, 64, 32), (4095, 63, 31)])
def test_labels_match_oracle(cy, A, n_coarse, zero_bin):
    # even A: the median is the mean of the two middle magnitudes; odd A: the middle one
    T = 8
    x = siggen.mixed_stream(6, 1, n=20000)[0]
    alphas = -0.5 + np.arange(A) / A
    R, Rc, _ = cyclic_tables(x, alphas, T)
    R32, Rc32 = R.astype(np.complex64), Rc.astype(np.complex64)
    ref = P.coarse_labels(R32.astype(np.complex128), Rc32.astype(np.complex128), n_coarse, zero_bin=zero_bin)
    lab = cy.cyc_peak_labels(torch.from_numpy(R32).to("cuda"), torch.from_numpy(Rc32).to("cuda"),
                             n_coarse=n_coarse, zero_bin=zero_bin).cpu().numpy()
    print(f"  A={A}: {int(ref.sum())} positive coarse bins", flush=True)
    assert ref.sum() > 0
    assert np.array_equal(lab, ref.astype(np.float32))


@pytest.mark.parametrize("A,n_coarse,thresh", [(1023, 3, 4.0), (50, 50, 3.0), (96, 4, 3.0), (6400, 100, 3.0),
                                               (8192, 1024, 3.0)])
def test_labels_random_tables_match_oracle(cy, A, n_coarse, thresh):
    # Rayleigh-like tables whose scale changes from coarse bin to coarse bin,
    # rounded to quarter steps so that many magnitudes tie; 341, 1, 24, 64 and
    # 8 fine bins per coarse bin (one or several workgroups, a partial last one,
    # windows that wrap around the circle)
    rng = np.random.default_rng(A + n_coarse)
    T = 3
    scale = np.repeat(rng.uniform(0.5, 2.0, size=n_coarse), A // n_coarse)[None, :]

    def table():
        z = (rng.standard_normal((T, A)) + 1j * rng.standard_normal((T, A))) * scale
        return (np.round(z * 4) / 4).astype(np.complex64)

    R, Rc = table(), table()
    zb = n_coarse // 2
    ref = P.coarse_labels(R.astype(np.complex128), Rc.astype(np.complex128), n_coarse, zero_bin=zb, thresh=thresh)
    lab = cy.cyc_peak_labels(torch.from_numpy(R).to("cuda"), torch.from_numpy(Rc).to("cuda"),
                             n_coarse=n_coarse, zero_bin=zb, thresh=thresh).cpu().numpy()
    print(f"  A={A} n_coarse={n_coarse}: {int(ref.sum())} positive", flush=True)
    assert 0 < ref.sum() < n_coarse
    assert np.array_equal(lab, ref.astype(np.float32))


def test_label_noise_scale_matches_oracle_median(cy):
    # 8 coarse bins of 8: each window holds 24 magnitudes, the median is the mean
    # of the 12th and 13th.  Both rows put 12 values of 0.25 and 12 larger ones
    # in a window, so the median is 0.625 and the threshold 7 * 0.625 / c = 3.72.
    T, A, n_coarse = 2, 64, 8
    R = np.ones((T, A), np.complex64)
    R[0, 8:20] = 0.25
    R[0, 22] = 3.0          # bin 2: below 3.72 (a lower-middle median, 0.25, would flag it)
    R[1, 32:44] = 0.25
    R[1, 46] = 5.0          # bin 5: above 3.72 (an upper-middle median, 1, would miss it)
    R[1, 47] = 3.0
    Rc = np.full((T, A), 0.1 + 0.1j, np.complex64)
    Rc[1, 60] = 0.8         # 7 * 0.1414 / c = 0.84 -> no peak
    ref = P.coarse_labels(R.astype(np.complex128), Rc.astype(np.complex128), n_coarse, zero_bin=-1)
    lab = cy.cyc_peak_labels(torch.from_numpy(R).to("cuda"), torch.from_numpy(Rc).to("cuda"),
                             n_coarse=n_coarse, zero_bin=-1).cpu().numpy()
    assert ref.tolist() == [0, 0, 0, 0, 0, 1, 0, 0]
    assert np.array_equal(lab, ref.astype(np.float32))


def test_labels_with_one_table(cy):
    # a NULL table contributes no peaks: one-table labels equal the oracle's with
    # a zero table, and their union the two-table labels
    T, A, n_coarse = 6, 4096, 64
    x = siggen.mixed_stream(6, 4, n=20000)[0]
    alphas = -0.5 + np.arange(A) / A
    R, Rc, _ = cyclic_tables(x, alphas, T)
    R32, Rc32 = R.astype(np.complex64), Rc.astype(np.complex64)
    z = np.zeros_like(R)
    want_a = P.coarse_labels(R32.astype(np.complex128), z, n_coarse, zero_bin=32)
    want_c = P.coarse_labels(z, Rc32.astype(np.complex128), n_coarse, zero_bin=32)
    dR, dRc = torch.from_numpy(R32).to("cuda"), torch.from_numpy(Rc32).to("cuda")
    la = cy.cyc_peak_labels(dR, None, n_coarse=n_coarse, zero_bin=32).cpu().numpy()
    lc = cy.cyc_peak_labels(None, dRc, n_coarse=n_coarse, zero_bin=32).cpu().numpy()
    both = cy.cyc_peak_labels(dR, dRc, n_coarse=n_coarse, zero_bin=32).cpu().numpy()
    assert want_a.sum() > 0 and want_c.sum() > 0
    assert np.array_equal(la, want_a.astype(np.float32)) and np.array_equal(lc, want_c.astype(np.float32))
    assert np.array_equal(both, np.maximum(la, lc))


def test_propose_equals_its_steps_and_the_oracle_selection(cy):
    # cyc_propose (spectra -> network -> selection -> compaction) against the
    # separate calls on the same windows, and its bins against the oracle's
    # selection of the same probabilities
    n = 3
    x = torch.from_numpy(np.concatenate([siggen.mixed_stream(5, 100 + i, n=65536)[0] for i in range(n)])).to("cuda")
    m = cy.ProposalModel(4, cy.CYC_OP_FP32)
    m.set_params(_flat(_params(7)))
    bins, nbins, conf, fb = m.propose(x, topk=16, width=2, zero_bin=512, theta=0.5)
    prob = m.forward(m.spectra(x))
    sel, conf2 = cy.cyc_select(prob, topk=16, width=2, zero_bin=512)
    bins, nbins, conf, fb = bins.cpu().numpy(), nbins.cpu().numpy(), conf.cpu().numpy(), fb.cpu().numpy()
    prob, sel, conf2 = prob.cpu().numpy(), sel.cpu().numpy(), conf2.cpu().numpy()
    m.close()
    for i in range(n):
        want = np.nonzero(sel[i])[0]
        assert nbins[i] == want.size
        assert list(bins[i, :nbins[i]]) == list(want)
        assert (bins[i, nbins[i]:] == -1).all()
        assert conf[i] == conf2[i] and fb[i] == (1 if conf[i] < 0.5 else 0)
        s_ref, c_ref = P.select(prob[i].astype(np.float64), k=16, width=2, zero_bin=512)
        assert list(want) == list(s_ref)
        assert abs(conf[i] - c_ref) < 1e-6


def test_network_without_local_layer(cy):
    """CYC_NN_NO_LOCAL: the four convolutions and the dense head alone (the
    oracle's network with Wl = 0); Wl is ignored and gets a zero gradient."""
    p = _params(8)
    rng = np.random.default_rng(9)
    B = 2
    X = rng.standard_normal((B, 3, 1024)).astype(np.float32).astype(np.float64)
    y = (rng.random((B, 1024)) < 0.05).astype(np.float64)
    p0 = dict(p, Wl=np.zeros_like(p["Wl"]))
    z, cache = P.forward(p0, X)
    g = P.backward(p0, cache, z, y)
    m = cy.ProposalModel(B, cy.CYC_OP_FP32 | cy.CYC_NN_NO_LOCAL)
    m.set_params(_flat(p))                   # Wl nonzero on the GPU: must be ignored
    feat = torch.from_numpy(np.ascontiguousarray(X.transpose(1, 0, 2)).astype(np.float32)).to("cuda")
    prob = m.forward(feat).cpu().numpy().astype(np.float64)
    gg, _ = m.gradients(feat, torch.from_numpy(y.astype(np.float32)).to("cuda"))
    gg = _unflat(gg.cpu().numpy().astype(np.float64), p)
    m.close()
    assert _rel(prob, P.sigmoid(z)) <= 1e-5
    assert not np.any(gg["Wl"])
    for k in KEYS:
        if k != "Wl":
            assert _rel(gg[k], g[k]) <= 2e-5, k
