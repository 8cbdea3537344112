"""FP64 CPU oracle for the learned cycle-frequency proposal.

TEST INFRASTRUCTURE ONLY (see ``oracle/cyclic.py``); shares no code with the
HIP path.

The paper's related-work discussion (Sec. 1) describes a two-stage estimator:
a coarse stage locates cyclic features and a fine stage evaluates the
estimator only near them; cycle-frequency estimation is named as future work
(Sec. 6).  This module holds the plain definitions of every step of the
learned form of that coarse stage:

* features: Welch spectra (Hann window, non-overlapping segments, averaged
  squared magnitude) of x, x^2 and |x|^2, shifted to [-1/2, 1/2), log, then
  standardised per channel;
* the network: circular 1-D convolutions with ReLU, then per coarse bin the
  sum of a dense layer over the flattened channels x positions and a local
  layer (one weight per channel, shared by all bins) over the channels at
  that bin's position, and a sigmoid;
* binary cross-entropy loss (mean over windows and bins), its gradients by
  the chain rule, and one AdamW step;
* labels: coarse bins holding a peak of the full-grid tables;
* selection: top-k coarse bins, each widened by +-w bins circularly, the
  coarse bin of alpha = 0 always included, and the confidence rule.
"""
from __future__ import annotations

import numpy as np

# ----------------------------------------------------------------------------- features


def hann(n: int) -> np.ndarray:
    """Periodic Hann window w[i] = 1/2 - 1/2 cos(2 pi i / n)."""
    return 0.5 - 0.5 * np.cos(2.0 * np.pi * np.arange(n) / n)


def welch_log_spectra(x, nseg: int = 64, nfft: int = 1024, eps: float = 1e-12) -> np.ndarray:
    """(3, nfft) standardised log spectra of x, x^2, |x|^2 (bins f = -1/2 + m/nfft)."""
    x = np.asarray(x).astype(np.complex128).reshape(-1)[: nseg * nfft]
    w = hann(nfft)
    out = np.empty((3, nfft))
    for c, v in enumerate((x, x * x, (np.abs(x) ** 2).astype(np.complex128))):
        segs = v.reshape(nseg, nfft) * w[None, :]
        P = np.mean(np.abs(np.fft.fft(segs, axis=1)) ** 2, axis=0)
        L = np.log(np.fft.fftshift(P) + eps)
        out[c] = (L - L.mean()) / (L.std() + 1e-12)
    return out


# ----------------------------------------------------------------------------- network


def init_params(rng, C_in=3, C=64, K=7, L=1024, n_out=1024, n_conv=4):
    """He-style initial weights (FP64)."""
    p = {}
    cin = C_in
    for i in range(n_conv):
        p[f"W{i}"] = rng.standard_normal((C, cin, K)) * np.sqrt(2.0 / (cin * K))
        p[f"b{i}"] = np.zeros(C)
        cin = C
    p["Wh"] = rng.standard_normal((n_out, C * L)) * np.sqrt(1.0 / (C * L))
    p["bh"] = np.zeros(n_out)
    p["Wl"] = rng.standard_normal(C) * np.sqrt(1.0 / C)
    return p


def conv_circ(x, W, b):
    """y[n, o, t] = b[o] + sum_{i,k} W[o, i, k] x[n, i, (t + k - K//2) mod L]."""
    K = W.shape[2]
    L = x.shape[2]
    y = np.broadcast_to(b[None, :, None], (x.shape[0], W.shape[0], L)).copy()
    for k in range(K):
        xs = np.roll(x, -(k - K // 2), axis=2)   # xs[..., t] = x[..., t + k - K//2]
        y += np.einsum("oi,nit->not", W[:, :, k], xs)
    return y


def conv_circ_backward(x, W, dy):
    """Gradients of conv_circ w.r.t. x, W and b for upstream gradient dy."""
    K = W.shape[2]
    dW = np.empty_like(W)
    dx = np.zeros_like(x)
    for k in range(K):
        xs = np.roll(x, -(k - K // 2), axis=2)
        dW[:, :, k] = np.einsum("not,nit->oi", dy, xs)
        # y[t] gets x[t + s], s = k - K//2, so x[u] feeds y[u - s]
        dx += np.roll(np.einsum("oi,not->nit", W[:, :, k], dy), (k - K // 2), axis=2)
    db = dy.sum(axis=(0, 2))
    return dx, dW, db


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def forward(p, X, n_conv=4):
    """Returns (logits z (N, n_out), cache)."""
    acts = [X]
    pre = []
    a = X
    for i in range(n_conv):
        u = conv_circ(a, p[f"W{i}"], p[f"b{i}"])
        pre.append(u)
        a = np.maximum(u, 0.0)
        acts.append(a)
    h = a.reshape(a.shape[0], -1)           # h[n, c*L + t] = a[n, c, t]
    z = h @ p["Wh"].T + p["bh"][None, :]
    # local layer: output bin j reads position j (requires n_out == L)
    z = z + np.einsum("c,ncj->nj", p["Wl"], a)
    return z, dict(acts=acts, pre=pre, h=h)


def bce_loss(z, y):
    """Mean binary cross-entropy of sigmoid(z) against labels y, computed stably."""
    return float(np.mean(np.maximum(z, 0) - z * y + np.log1p(np.exp(-np.abs(z)))))


def backward(p, cache, z, y, n_conv=4):
    """Gradients of bce_loss(forward(p, X)) with respect to every parameter."""
    g = {}
    dz = (sigmoid(z) - y) / z.size
    g["Wh"] = dz.T @ cache["h"]
    g["bh"] = dz.sum(axis=0)
    g["Wl"] = np.einsum("nj,ncj->c", dz, cache["acts"][-1])
    dh = dz @ p["Wh"]
    da = dh.reshape(cache["acts"][-1].shape) + p["Wl"][None, :, None] * dz[:, None, :]
    for i in reversed(range(n_conv)):
        du = da * (cache["pre"][i] > 0)
        dx, g[f"W{i}"], g[f"b{i}"] = conv_circ_backward(cache["acts"][i], p[f"W{i}"], du)
        da = dx
    return g


def adamw_step(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, wd=1e-2):
    """One AdamW update (decoupled weight decay) in place; t is the 1-based step."""
    for k in p:
        m[k] = b1 * m[k] + (1 - b1) * g[k]
        v[k] = b2 * v[k] + (1 - b2) * g[k] * g[k]
        mh = m[k] / (1 - b1 ** t)
        vh = v[k] / (1 - b2 ** t)
        p[k] = p[k] - lr * (mh / (np.sqrt(vh) + eps) + wd * p[k])


# ----------------------------------------------------------------------------- rounding-noise model of the GPU network


def perturbed_pass(p, X, y, u, rng, n_conv=4):
    """One draw of the rounding-noise model of the reduced-precision network
    (test infrastructure).

    The GPU rounds both operands of every matrix product (convolutions, head,
    backward products) to the operand precision and keeps everything else in
    FP32.  This pass is the FP64 network with each such operand value v
    replaced by v (1 + d), d uniform in [-u, u] and drawn once per value per
    pass (a value that feeds several products is rounded the same way in each,
    as on the GPU); the backward ReLU masks with the pass's own
    pre-activations.  Uniform relative errors in [-u, u] have mean square u^2/3,
    which is at least that of round-to-nearest (half an ulp uniform, at most
    u^2/3 relative).  Returns (probabilities, gradient dict).
    """
    def rnd(v):
        return v * (1.0 + rng.uniform(-u, u, size=v.shape)) if u > 0 else v

    B = X.shape[0]
    Wq = {i: rnd(p[f"W{i}"]) for i in range(n_conv)}
    Whq = rnd(p["Wh"])
    acts, aq, pre = [X], [rnd(X)], []
    for i in range(n_conv):
        u_ = conv_circ(aq[i], Wq[i], p[f"b{i}"])
        pre.append(u_)
        a = np.maximum(u_, 0.0)
        acts.append(a)
        aq.append(rnd(a))
    a4 = acts[-1]
    hq = aq[-1].reshape(B, -1)
    z = hq @ Whq.T + p["bh"][None, :] + np.einsum("c,ncj->nj", p["Wl"], a4)
    prob = sigmoid(z)
    dz = (prob - y) / z.size
    dzq = rnd(dz)
    g = {"Wh": dzq.T @ hq, "bh": dz.sum(axis=0), "Wl": np.einsum("nj,ncj->c", dz, a4)}
    da = (dzq @ Whq).reshape(a4.shape) + p["Wl"][None, :, None] * dz[:, None, :]
    for i in reversed(range(n_conv)):
        du = da * (pre[i] > 0)
        duq = rnd(du)
        dx, g[f"W{i}"], _ = conv_circ_backward(aq[i], Wq[i], duq)
        g[f"b{i}"] = du.sum(axis=(0, 2))
        if i > 0:
            da = dx
    return prob, g


def rounding_noise_scale(p, X, y, u, trials, seed, n_conv=4):
    """Root-mean-square deviation from the exact FP64 values, per element, of
    the probabilities and gradients over `trials` draws of perturbed_pass."""
    rng = np.random.default_rng(seed)
    z, cache = forward(p, X, n_conv)
    prob0 = sigmoid(z)
    g0 = backward(p, cache, z, y, n_conv)
    sp = np.zeros_like(prob0)
    sg = {k: np.zeros_like(v) for k, v in g0.items()}
    for _ in range(trials):
        prob, g = perturbed_pass(p, X, y, u, rng, n_conv)
        sp += (prob - prob0) ** 2
        for k in sg:
            sg[k] += (g[k] - g0[k]) ** 2
    return np.sqrt(sp / trials), {k: np.sqrt(v / trials) for k, v in sg.items()}


def gradient_magnitude_sums(p, X, y, n_conv=4):
    """Sum of |terms| of the last sum behind each gradient element (and of the
    logit behind each probability): the scale of FP32 accumulation error."""
    B = X.shape[0]
    z, cache = forward(p, X, n_conv)
    acts, pre = cache["acts"], cache["pre"]
    a4 = np.abs(acts[-1])
    h = a4.reshape(B, -1)
    mz = h @ np.abs(p["Wh"]).T + np.abs(p["bh"])[None, :] + np.einsum("c,ncj->nj", np.abs(p["Wl"]), a4)
    prob = sigmoid(z)
    dz = (prob - y) / z.size
    m = {"Wh": np.abs(dz).T @ h, "bh": np.abs(dz).sum(axis=0), "Wl": np.einsum("nj,ncj->c", np.abs(dz), a4)}
    da = (dz @ p["Wh"]).reshape(acts[-1].shape) + p["Wl"][None, :, None] * dz[:, None, :]
    for i in reversed(range(n_conv)):
        du = da * (pre[i] > 0)
        m[f"W{i}"] = conv_circ_backward(np.abs(acts[i]), np.abs(p[f"W{i}"]), np.abs(du))[1]
        m[f"b{i}"] = np.abs(du).sum(axis=(0, 2))
        if i > 0:
            da = conv_circ_backward(acts[i], p[f"W{i}"], du)[0]
    return mz, m


# ----------------------------------------------------------------------------- labels and selection


def local_sigma(m, n_coarse: int):
    """Noise scale per (lag, coarse bin) from magnitudes m [T, A].

    sigma[t, c] = median of m[t, a] over the fine bins a of coarse bins c-1, c
    and c+1 (circular, since alpha is 1-periodic) divided by sqrt(2 ln 2): for
    noise-only cells |R| is Rayleigh distributed with scale sigma, whose median
    is sigma * sqrt(2 ln 2) (about 1.1774 sigma).  The estimate is local
    because the self-noise of a modulated signal is strong in band and weak
    out of band; a line feature occupies a few of the 3 * A / n_coarse cells
    and does not move the median.  An even count takes the mean of the two
    middle values.
    """
    T, A = m.shape
    per = A // n_coarse
    blocks = m.reshape(T, n_coarse, per)
    win = np.concatenate([np.roll(blocks, 1, axis=1), blocks, np.roll(blocks, -1, axis=1)], axis=2)
    return np.median(win, axis=2) / np.sqrt(2.0 * np.log(2.0))


def peak_cells(R, n_coarse: int, thresh: float = 7.0):
    """|R[t, a]| > thresh * sigma[t, coarse bin of a] (a local median CFAR test)."""
    m = np.abs(R)
    per = R.shape[1] // n_coarse
    sigma = np.repeat(local_sigma(m, n_coarse), per, axis=1)
    return m > thresh * sigma


def coarse_labels(R, Rc, n_coarse: int, zero_bin: int, thresh: float = 7.0) -> np.ndarray:
    """Coarse bin positive if any of its fine bins peaks at any lag in either table.

    The coarse bin holding alpha = 0 is excluded for the non-conjugate table
    (the power term is always there; that bin is always evaluated).
    """
    A = R.shape[1]
    per = A // n_coarse
    pk = peak_cells(R, n_coarse, thresh).any(axis=0).reshape(n_coarse, per).any(axis=1)
    pkc = peak_cells(Rc, n_coarse, thresh).any(axis=0).reshape(n_coarse, per).any(axis=1)
    if zero_bin is not None and zero_bin >= 0:   # a negative bin means none is excluded
        pk[zero_bin] = False
    return (pk | pkc).astype(np.float64)


def select(prob, k: int = 16, width: int = 2, zero_bin: int | None = None):
    """Top-k bins (ties -> lower index), each widened by +-width circularly, sorted.

    Returns (selected bins, confidence = 1 - max probability outside the set).
    NaN bins are never among the top k, and a window with any non-finite
    probability has confidence 0 (it always falls back to the full grid): the
    confidence rule is defined for probabilities only.
    """
    prob = np.asarray(prob, dtype=np.float64)
    n = prob.size
    order = np.lexsort((np.arange(n), -prob))   # descending prob, then ascending index
    order = [i for i in order if not np.isnan(prob[i])]
    sel = set()
    for i in order[:k]:
        for d in range(-width, width + 1):
            sel.add(int((i + d) % n))
    if zero_bin is not None:
        sel.add(int(zero_bin))
    sel = np.array(sorted(sel), dtype=np.int64)
    mask = np.ones(n, bool)
    mask[sel] = False
    conf = 1.0 - (prob[mask].max() if mask.any() else 0.0)
    if not np.all(np.isfinite(prob)):
        conf = 0.0
    return sel, conf
