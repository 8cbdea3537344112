"""Learned cycle-frequency proposal: data, labels, training and evaluation.

Orchestration over the C ABI only (every numeric step runs in the HIP
library):

* windows: 65536-sample records of the mixed-modulation workload;
* labels: the full-grid tables (fine grid alpha_j = -1/2 + j/65536, lags
  0..63; the uniform-grid form, FP64) of each window, reduced by
  ``cyc_peak_labels`` to 1024 coarse bins;
* features: ``cyc_model_spectra``; training: ``cyc_model_train_step``;
* proposal: network probabilities -> ``cyc_select`` (top-16 coarse bins +-2,
  the alpha = 0 bin always) -> the exact estimator on the 64 fine bins of each
  selected coarse bin, or the full fine grid when the confidence is below
  theta.

Reported: miss rate (labelled coarse bins not evaluated / labelled coarse
bins), fallback rate, and the speedup of the proposal path over the dense full
grid, next to a spectral-peak heuristic and an untrained network.
"""
from __future__ import annotations

import json
import time
from multiprocessing import Pool

import numpy as np

from . import cyclo, siggen

WINDOW = cyclo.WINDOW
N_COARSE = cyclo.N_COARSE
VAL_FIRST = 1 << 24   # first index of the validation windows (training windows start at 0)
TEST_FIRST = 1 << 25  # first index of the test windows
FINE = 65536
PER = FINE // N_COARSE
ZERO_BIN = N_COARSE // 2
T_LAG = 64
FINE_GRID = -0.5 + np.arange(FINE) / FINE


def _window(args):
    seed, i = args
    return siggen.mixed_stream(seed, i, n=WINDOW)[0]


def make_windows(seed: int, first: int, n: int, pool=None) -> np.ndarray:
    """n windows (complex64, [n, 65536]) of the mixed workload, seeded per window.

    pool: an optional process pool, forked before the process first touches
    the GPU; without one the windows are generated in this process.
    """
    args = [(seed, first + i) for i in range(n)]
    xs = pool.map(_window, args, chunksize=16) if pool is not None else [_window(a) for a in args]
    return np.stack(xs)


def init_params(seed: int, prior_logit: float = -6.0) -> np.ndarray:
    """He-initialised FP32 parameter vector in the ABI's order.

    The output bias starts at the logit of the label prior (a few positive
    coarse bins in 1024), so the first steps do not spend themselves on it.
    """
    rng = np.random.default_rng(seed)
    parts = []
    cin = 3
    for _ in range(4):
        parts.append(rng.standard_normal(64 * cin * 7) * np.sqrt(2.0 / (cin * 7)))
        parts.append(np.zeros(64))
        cin = 64
    parts.append(rng.standard_normal(N_COARSE * 64 * 1024) * np.sqrt(1.0 / (64 * 1024)))
    parts.append(np.full(N_COARSE, prior_logit))
    parts.append(rng.standard_normal(64) * np.sqrt(1.0 / 64))
    v = np.concatenate(parts).astype(np.float32)
    assert v.size == cyclo.ProposalModel.num_params()
    return v


class FullGrid:
    """The full fine grid (65536 alphas, lags 0..63) of one window at a time.

    mode "dense": the dense contraction on the alpha list (BF16 operands,
    autotuned kernel configuration), the baseline the proposal is timed
    against.  mode "fft": the uniform-grid form (fold + FP64 FFT), used for the
    labels.
    """

    def __init__(self, mode: str = "dense", flags=cyclo.CYC_OP_BF16):
        import torch
        self.mode = mode
        if mode == "dense":
            cyclo.cyc_autotune(FINE, T_LAG, flags)
            self.st = cyclo.CyclicStream(FINE_GRID, T_LAG, flags)
        elif mode == "fft":
            self.st = cyclo.GridStream(-0.5, FINE, T_LAG)
        else:
            raise ValueError(mode)
        self.R = torch.empty((T_LAG, FINE), dtype=torch.complex64, device="cuda")
        self.Rc = torch.empty_like(self.R)

    def tables(self, x):
        self.st.reset()
        self.st.push(x)
        if self.mode == "dense":
            cyclo.cyc_read(self.st._s, self.R, self.Rc)
        else:
            self.st.read_into(self.R, self.Rc)
        return self.R, self.Rc

    def close(self):
        self.st.close()


def label_windows(xd, fg: FullGrid, thresh: float = 7.0):
    """Labels of device windows xd [n, 65536]: (non-conjugate, conjugate), each [n, 1024] on the GPU.

    Each label call is given one table; the other is NULL and contributes no peaks.
    """
    import torch
    acf = torch.empty((xd.shape[0], N_COARSE), dtype=torch.float32, device="cuda")
    conj = torch.empty_like(acf)
    for i in range(xd.shape[0]):
        R, Rc = fg.tables(xd[i])
        acf[i] = cyclo.cyc_peak_labels(R, None, N_COARSE, ZERO_BIN, thresh)
        conj[i] = cyclo.cyc_peak_labels(None, Rc, N_COARSE, ZERO_BIN, thresh)
    return acf, conj


def heuristic_scores(feat):
    """Coarse-stage heuristic: spectral lines of |x|^2 (ACF) and x^2 (conjugate)."""
    import torch
    s = torch.maximum(feat[1], feat[2]).clone()   # [n, 1024] standardised log spectra
    s[:, ZERO_BIN] = -1e9                          # DC of |x|^2 is the power term
    return torch.sigmoid(s)


def miss_rate(sel, labels, fell_back):
    """Labelled coarse bins (alpha = 0 bin excluded by the labels) left unevaluated."""
    lab = labels.bool()
    covered = sel.bool() | fell_back[:, None]
    missed = (lab & ~covered).sum().item()
    total = lab.sum().item()
    return missed / max(total, 1), int(missed), int(total)


def shifted_batch(feat, acf, conj, idx, shifts):
    """Features and labels of windows idx as if each had been shifted in frequency.

    A carrier shift x[n] exp(j2pi k n / 1024) moves the Welch spectrum of x by
    k bins and that of x^2 by 2k bins (each segment is 1024 samples long, so the
    shift is a whole number of bins and only the segment phases change), leaves
    |x|^2 unchanged, moves every conjugate cycle frequency by 2k / 1024 (2k
    coarse bins) and leaves the non-conjugate ones in place.  shifts: int64 [B]
    on the GPU.  Returns ([3, B, 1024] features, [B, 1024] labels).
    """
    import torch
    pos = torch.arange(N_COARSE, device=feat.device)
    src1 = (pos[None, :] - shifts[:, None]) % N_COARSE
    src2 = (pos[None, :] - 2 * shifts[:, None]) % N_COARSE
    f0 = torch.gather(feat[0, idx], 1, src1)
    f1 = torch.gather(feat[1, idx], 1, src2)
    f2 = feat[2, idx]
    lab = torch.maximum(acf[idx], torch.gather(conj[idx], 1, src2))
    return torch.stack([f0, f1, f2]).contiguous(), lab.contiguous()


def train(model, feat, labels, epochs: int, batch: int, lr: float, wd: float, seed: int = 0, log=None,
          val=None, augment: bool = True):
    """AdamW epochs over shuffled batches (cosine learning-rate decay).

    labels = (non-conjugate, conjugate) label tensors; with augment every
    window of a batch is seen at a random carrier shift (shifted_batch).  With
    val = (features, labels) the validation loss is taken after every epoch
    and the parameters of the best epoch are kept.
    """
    import torch
    acf, conj = labels
    n = feat.shape[1]
    rng = np.random.default_rng(seed)
    losses, val_losses = [], []
    steps, step_s = 0, 0.0
    best = (np.inf, None, -1)
    for ep in range(epochs):
        order = rng.permutation(n)
        ep_loss = []
        lr_ep = lr * 0.5 * (1 + np.cos(np.pi * ep / max(epochs, 1)))
        torch.cuda.synchronize()
        t = time.perf_counter()
        for s in range(0, n - batch + 1, batch):
            idx = torch.from_numpy(order[s:s + batch]).to("cuda")
            k = rng.integers(0, N_COARSE, size=batch) if augment else np.zeros(batch, dtype=np.int64)
            fb, lb = shifted_batch(feat, acf, conj, idx, torch.from_numpy(k).to("cuda"))
            ep_loss.append(model.train_step(fb, lb, lr_ep, wd))
            steps += 1
        torch.cuda.synchronize()
        step_s += time.perf_counter() - t
        losses.append(float(np.mean(ep_loss)))
        msg = f"epoch {ep}: loss {losses[-1]:.5f}"
        if val is not None:
            vf, vl = val
            B = model.max_batch
            v = float(np.mean([model.loss(vf[:, s:s + B].contiguous(), vl[s:s + B].contiguous())
                               for s in range(0, vf.shape[1], B)]))
            val_losses.append(v)
            msg += f" val {v:.5f}"
            if v < best[0]:
                best = (v, model.get_params(), ep)
        if log:
            log(msg)
    if best[1] is not None:
        model.set_params(best[1])
    return dict(losses=losses, val_losses=val_losses, steps=steps, ms_per_step=1e3 * step_s / max(steps, 1),
                best_epoch=best[2])


def probabilities(model, feat, batch: int):
    import torch
    outs = []
    for s in range(0, feat.shape[1], batch):
        outs.append(model.forward(feat[:, s:s + batch, :].contiguous()))
    return torch.cat(outs)


def choose_theta(conf, sel, labels, target: float):
    """Smallest fallback threshold whose miss rate is at or below the target.

    Candidates are 0 and just above each window's confidence (a window falls
    back when its confidence is below the threshold).
    """
    c = conf.cpu().numpy().astype(np.float32)   # thresholds are compared in FP32
    missed = (labels.bool() & ~sel.bool()).sum(1).cpu().numpy()
    total = max(int(labels.sum().item()), 1)
    order = np.argsort(c)
    cum = np.concatenate([[0], np.cumsum(missed[order])])   # misses recovered by the k least confident
    for k in range(len(c) + 1):
        if (missed.sum() - cum[k]) / total <= target:
            return 0.0 if k == 0 else float(np.nextafter(c[order[k - 1]], np.float32(np.inf)))
    return 1.0


def dataset(model, fg: FullGrid, seed: int, first: int, n: int, keep_windows: bool = False, chunk: int = 512,
            log=None, pool=None):
    """Features [3, n, 1024] and labels [n, 1024] (GPU) of n windows, made chunk by chunk."""
    import torch
    feats, acfs, conjs, wins = [], [], [], []
    starts = list(range(0, n, chunk))

    def submit(s):  # the pool makes the next chunk's windows while this one is labelled
        m = min(chunk, n - s)
        args = [(seed, first + s + i) for i in range(m)]
        return pool.map_async(_window, args, chunksize=16) if pool is not None else None

    pending = submit(starts[0]) if starts else None
    for k, s in enumerate(starts):
        m = min(chunk, n - s)
        if pool is not None:
            xs = np.stack(pending.get())
            if k + 1 < len(starts):
                pending = submit(starts[k + 1])
        else:
            xs = make_windows(seed, first + s, m)
        xd = torch.from_numpy(xs).to("cuda")
        a, c = label_windows(xd, fg)
        acfs.append(a)
        conjs.append(c)
        feats.append(model.spectra(xd.reshape(-1)))
        if keep_windows:
            wins.append(xd)
        if log:
            log(f"  windows {first + s}..{first + s + m - 1} labelled")
    feat = torch.cat(feats, dim=1)
    acf, conj = torch.cat(acfs), torch.cat(conjs)
    return feat, (acf, conj), (torch.cat(wins) if keep_windows else None)


def run(n_train=4096, n_val=512, n_test=512, epochs=30, batch=128, lr=2e-3, wd=0.1, seed=5,
        target_miss=0.01, log=print, pool=None, augment=True, compare_no_local=False):
    """Labels, trains and evaluates the proposal network (see the module docstring).

    compare_no_local: also train the network without its local layer
    (CYC_NN_NO_LOCAL: the four convolutions and the dense head alone) on the
    same windows, and report its miss rates at its own validated threshold.
    """
    import torch
    t0 = time.time()
    res = {"config": dict(n_train=n_train, n_val=n_val, n_test=n_test, epochs=epochs, batch=batch, lr=lr,
                          weight_decay=wd, seed=seed, window=WINDOW, fine_bins=FINE, coarse_bins=N_COARSE,
                          lags=T_LAG, select="top16+-2 and the alpha=0 bin", label_threshold=7.0,
                          target_miss=target_miss, augment=augment)}
    fg = FullGrid("fft")
    model = cyclo.ProposalModel(max(batch, 512), cyclo.CYC_OP_BF16)
    torch.cuda.synchronize()
    t1 = time.time()
    # held-out windows come from fixed index ranges, so every training size is
    # validated and tested on the same windows
    f_tr, ls_tr, _ = dataset(model, fg, seed, 0, n_train, log=log, pool=pool)
    f_va, ls_va, _ = dataset(model, fg, seed, VAL_FIRST, n_val, log=log, pool=pool)
    f_te, ls_te, x_te = dataset(model, fg, seed, TEST_FIRST, n_test, keep_windows=True, log=log, pool=pool)
    l_tr, l_va, l_te = (torch.maximum(*ls) for ls in (ls_tr, ls_va, ls_te))
    torch.cuda.synchronize()
    res["labelling_s"] = time.time() - t1
    res["positives_per_window"] = float(torch.cat([l_tr, l_va, l_te]).sum(1).mean().item())
    log(f"labels: {res['labelling_s']:.1f} s, {res['positives_per_window']:.2f} positive coarse bins/window")
    # untrained network
    model.set_params(init_params(seed))
    p_untrained = probabilities(model, f_te, 512)
    # training
    t2 = time.time()
    tr = train(model, f_tr, ls_tr, epochs, batch, lr, wd, seed, log, val=(f_va, l_va), augment=augment)
    torch.cuda.synchronize()
    res["train"] = dict(seconds=time.time() - t2, steps=tr["steps"], ms_per_step=tr["ms_per_step"],
                        loss_first_epoch=tr["losses"][0], loss_last_epoch=tr["losses"][-1],
                        val_loss_best=min(tr["val_losses"]), best_epoch=tr["best_epoch"])
    p_val = probabilities(model, f_va, 512)
    sel_v, conf_v = cyclo.cyc_select(p_val, 16, 2, ZERO_BIN)
    theta = choose_theta(conf_v, sel_v, l_va, target_miss)
    res["theta"] = theta
    # evaluation on the test windows
    evals = {}
    for name, prob, th in (("trained", probabilities(model, f_te, 512), theta), ("untrained", p_untrained, None),
                           ("heuristic", heuristic_scores(f_te), None)):
        sel, conf = cyclo.cyc_select(prob.contiguous(), 16, 2, ZERO_BIN)
        fb = conf < th if th is not None else torch.zeros_like(conf, dtype=torch.bool)
        mr, missed, total = miss_rate(sel, l_te, fb)
        mr0, _, _ = miss_rate(sel, l_te, torch.zeros_like(fb))
        evals[name] = dict(miss_rate=mr, miss_rate_without_fallback=mr0, missed=missed, labelled=total,
                           fallback_rate=float(fb.float().mean().item()),
                           selected_bins_per_window=float(sel.float().sum(1).mean().item()))
        log(f"{name}: miss {mr:.4f} (no fallback {mr0:.4f}), fallback {evals[name]['fallback_rate']:.3f}")
    res["eval"] = evals
    if compare_no_local:
        m2 = cyclo.ProposalModel(max(batch, 512), cyclo.CYC_OP_BF16 | cyclo.CYC_NN_NO_LOCAL)
        m2.set_params(init_params(seed))
        t3 = time.time()
        tr2 = train(m2, f_tr, ls_tr, epochs, batch, lr, wd, seed, log, val=(f_va, l_va), augment=augment)
        sel_v2, conf_v2 = cyclo.cyc_select(probabilities(m2, f_va, 512), 16, 2, ZERO_BIN)
        theta2 = choose_theta(conf_v2, sel_v2, l_va, target_miss)
        sel2, conf2 = cyclo.cyc_select(probabilities(m2, f_te, 512).contiguous(), 16, 2, ZERO_BIN)
        fb2 = conf2 < theta2
        mr2, _, _ = miss_rate(sel2, l_te, fb2)
        mr20, _, _ = miss_rate(sel2, l_te, torch.zeros_like(fb2))
        res["no_local_head"] = dict(theta=theta2, miss_rate=mr2, miss_rate_without_fallback=mr20,
                                    fallback_rate=float(fb2.float().mean().item()),
                                    train_s=time.time() - t3, val_loss_best=min(tr2["val_losses"]))
        log(f"without the local layer: miss {mr2:.4f} (no fallback {mr20:.4f}), "
            f"fallback {res['no_local_head']['fallback_rate']:.3f}")
        m2.close()
    prob = probabilities(model, f_te, 512)
    sel, conf = cyclo.cyc_select(prob.contiguous(), 16, 2, ZERO_BIN)
    thetas = [0.0, 0.5, 0.8, 0.9, 0.95, 0.98, 0.99, 0.995, 0.999, 1.0]
    curve = theta_curve(conf, sel, l_te, thetas)
    fd = FullGrid("dense")
    res["speed"] = speed(model, x_te, fd, theta, conf_curve=[c[2] for c in curve], fft=fg)
    fd.close()
    res["theta_curve"] = [dict(theta=c[0], miss_rate=c[1], fallback_rate=c[2], predicted_speedup=p)
                          for c, p in zip(curve, res["speed"].pop("predicted_speedup"))]
    log(f"speed: {res['speed']}")
    for c in res["theta_curve"]:
        log(f"  theta {c['theta']:.3f}: miss {c['miss_rate']:.4f} fallback {c['fallback_rate']:.3f} "
            f"speedup {c['predicted_speedup']:.2f}")
    fg.close()
    model.close()
    res["total_s"] = time.time() - t0
    return res


def _contract_selected(xt, sel_h, idx, chunk: int = 512):
    """Exact estimator on the fine bins of the selected coarse bins of windows idx.

    One batch per chunk of windows; returns the tables of the first chunk.
    """
    first = None
    for s in range(0, len(idx), chunk):
        part = idx[s:s + chunk]
        lists = [FINE_GRID.reshape(N_COARSE, PER)[np.nonzero(sel_h[i])[0]].reshape(-1) for i in part]
        b = cyclo.CyclicBatch(lists, T_LAG, cyclo.CYC_OP_BF16)
        b.push([xt[i] for i in part])
        out = b.read()
        b.close()
        if first is None:
            first = out
    return first


def speed(model, xt, fg: FullGrid, theta: float, conf_curve=None, fft: FullGrid = None):
    """Dense full grid vs. spectra + network + selection + proposal contraction (+ fallbacks).

    Measured: the full grid over every window; the front end; the proposal
    contraction with no fallback; and the whole proposal path at theta.
    conf_curve = (thetas, fallback fractions) adds the speedup predicted from
    the measured per-window costs at each threshold.
    """
    import torch
    n = xt.shape[0]
    torch.cuda.synchronize()
    t = time.perf_counter()
    for i in range(n):
        fg.tables(xt[i])
    torch.cuda.synchronize()
    t_full = time.perf_counter() - t
    # kernel-only rate of the dense full grid: HIP events around its contraction
    # launches over a few more windows
    fg.st.profile(True)
    for i in range(min(n, 16)):
        fg.tables(xt[i])
    kp = fg.st.profile_read()
    fg.st.profile(False)
    k_tflops = 16.0 * kp["work"] / (kp["total_ms"] * 1e-3) / 1e12 if kp["total_ms"] > 0 else None
    t_fft = None
    if fft is not None:
        t = time.perf_counter()
        for i in range(n):
            fft.tables(xt[i])
        torch.cuda.synchronize()
        t_fft = time.perf_counter() - t
    t = time.perf_counter()
    feat = model.spectra(xt.reshape(-1))
    prob = probabilities(model, feat, 512)   # the network takes at most 512 windows per call
    sel, conf = cyclo.cyc_select(prob, 16, 2, ZERO_BIN)
    torch.cuda.synchronize()
    t_front = time.perf_counter() - t
    sel_h = sel.cpu().numpy().astype(bool)
    conf_h = conf.cpu().numpy()
    # proposal contraction on every window (no fallback)
    torch.cuda.synchronize()
    t = time.perf_counter()
    _contract_selected(xt, sel_h, np.arange(n))
    torch.cuda.synchronize()
    t_sel = time.perf_counter() - t
    # the whole path at theta
    fb = conf_h < theta
    keep = np.nonzero(~fb)[0]
    torch.cuda.synchronize()
    t = time.perf_counter()
    out = _contract_selected(xt, sel_h, keep)
    for i in np.nonzero(fb)[0]:
        fg.tables(xt[i])
    torch.cuda.synchronize()
    t_path = time.perf_counter() - t
    # the proposal tables equal the full-grid tables at the evaluated alphas (same estimator)
    diff = 0.0
    if out is not None:
        Rs, Rcs, _ = out
        for j, i in enumerate(keep[:4]):
            R, Rc = fg.tables(xt[i])
            cols = torch.from_numpy(np.nonzero(np.repeat(sel_h[i], PER))[0]).to("cuda")
            scale = R[0].abs().max().item()
            diff = max(diff, (Rs[j] - R[:, cols]).abs().max().item() / scale,
                       (Rcs[j] - Rc[:, cols]).abs().max().item() / scale)
    res = dict(windows=n, full_grid_s=t_full, full_grid_fft_s=t_fft, front_end_s=t_front,
               proposal_contract_no_fallback_s=t_sel,
               proposal_path_s=t_front + t_path, fallback_windows=int(fb.sum()),
               speedup=t_full / (t_front + t_path), speedup_no_fallback=t_full / (t_front + t_sel),
               evaluated_alphas_per_window=float(sel_h.sum(1).mean() * PER),
               ideal_speedup_no_fallback=float(FINE / (sel_h.sum(1).mean() * PER)),
               max_rel_diff_vs_full_grid=diff, full_grid_kernel_tflops=k_tflops)
    if conf_curve is not None:
        res["predicted_speedup"] = [float(t_full / (t_front + (1 - f) * t_sel + f * t_full)) for f in conf_curve]
    return res


def theta_curve(conf, sel, labels, thetas):
    """Miss rate and fallback fraction for each threshold."""
    out = []
    for th in thetas:
        fb = conf < float(th)
        out.append((float(th), miss_rate(sel, labels, fb)[0], float(fb.float().mean().item())))
    return out


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-train", type=int, default=4096)
    ap.add_argument("--n-val", type=int, default=512)
    ap.add_argument("--n-test", type=int, default=512)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=128)
    ap.add_argument("--out", default="")
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--wd", type=float, default=0.1)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--target-miss", type=float, default=0.01)
    ap.add_argument("--no-augment", action="store_true")
    a = ap.parse_args()
    import os
    # forked before anything touches the GPU
    with Pool(max(1, min(a.workers, os.cpu_count() or 1))) as pool:
        r = run(a.n_train, a.n_val, a.n_test, a.epochs, batch=a.batch, lr=a.lr, wd=a.wd,
                target_miss=a.target_miss, pool=pool, augment=not a.no_augment)
    s = json.dumps(r, indent=1)
    print(s)
    if a.out:
        open(a.out, "w").write(s)
