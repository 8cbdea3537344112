"""Throughput of the streaming cyclic-statistics path on one MI355X.

One step = reset the stream state, push the whole record in blocks, read both
tables (R and Rc) into device buffers.  The record is resident in HBM before
the timed region.  Default workload: QPSK with a root-raised-cosine pulse
(rolloff 0.35, 4 samples/symbol, SNR 5 dB, carrier offset 0.1), 2^24
complex64 samples pushed in 256 blocks of 65536, lags 0..127, 4096 cycle
frequencies alpha_k = -1/2 + k/4096, FP32 operands.

Extra forms in the same line: the 512-stream batch form, the learned proposal
(trained in the run, then timed against the dense full fine grid on held-out
windows) and the uniform-grid form (fold + FFT) on the same record, which is
exact on uniform power-of-two grids and quoted as context only.

Output: one JSON line (metric, value, ..., roofline, cpu_baseline, forms).
value = (alpha, tau)*samples per second = A * T * N_used / seconds per step.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "(α,τ)·samples/s per GPU"
UNIT = "(alpha,tau)*samples/s"
FLOPS_PER_TRIPLE = 16  # 8 real flops per complex multiply-add, two tables
PEAK_TFLOPS = {"f32": 157.3, "bf16": 2500.0, "f16": 2500.0}
PREC_FLAGS = {"f32": 0x0, "bf16": 0x1, "f16": 0x2}


HBM_PROFILE = os.path.join(ROOT, "profiles", "contract_qpsk_rrc_2p24_hbm_counters.txt")
KERNEL_SOURCES = {name: os.path.join(ROOT, "paper_2405_16911_amd", "csrc", name)
                  for name in ("cyclo_kernels.hip", "cyclo_internal.h")}


def profiled_traffic(cfg_name: str):
    """HBM bytes per launch of configuration cfg_name on the default record, from the
    committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary; None when the kernel sources
    have changed since the counters were taken or the configuration was not profiled."""
    import hashlib
    if not os.path.exists(HBM_PROFILE):
        return None
    digests, traffic = {}, None
    for line in open(HBM_PROFILE):
        f = line.split()
        if len(f) == 3 and f[0] == "source_sha256":
            digests[f[1]] = f[2]
        elif len(f) == 7 and f[0] == "cfg" and f[1] == cfg_name:
            traffic = float(f[6])
    for name, path in KERNEL_SOURCES.items():
        if digests.get(name) != hashlib.sha256(open(path, "rb").read()).hexdigest():
            return None
    return traffic


def workload(name: str):
    from paper_2405_16911_amd import siggen
    if name == "qpsk_rrc_2p24":
        x = siggen.qpsk_rrc_stream(n=1 << 24)
        return dict(x=x, T=128, alphas=siggen.uniform_grid(4096, -0.5), block=65536,
                    desc="qpsk_rrc_L2^24_T128_A4096_push65536")
    if name == "gmsk_32k":
        x = siggen.gmsk_stream(n=32768)
        return dict(x=x, T=32, alphas=np.arange(128) / 128.0, block=32768,
                    desc="gmsk_L32768_T32_A128_push32768")
    if name == "window_t64":
        # the learned proposal's dense baseline: one mixed-modulation window of
        # 65536 samples on the full fine grid (65536 alphas), lags 0..63
        x = siggen.mixed_stream(5, 0, n=65536)[0]
        return dict(x=x, T=64, alphas=siggen.uniform_grid(65536, -0.5), block=65536,
                    desc="mixed_window65536_T64_A65536_push65536")
    raise SystemExit(f"unknown workload {name}")


def sample_cells(T: int, A: int):
    """Cells checked against the oracle's direct sum (features alpha = 0, +-1/4 on
    the record's grid, the last lag, and seeded random cells)."""
    rng = np.random.default_rng(2)
    cells = [(0, A // 2), (1, A // 2), (4, A // 4), (4, 3 * A // 4), (T - 1, A // 2), (T // 2, 0), (3, A // 2 + 1)]
    cells += [(int(rng.integers(0, T)), int(rng.integers(0, A))) for _ in range(9)]
    return cells


def algorithmic_bytes(wl, prof) -> float:
    """Bytes the path must move per contraction launch: 8 per sample in and the two
    complex64 tables (2 T A 8 bytes) per read, over the launches of one step
    (one reset, every push, one read)."""
    T, A, L = wl["T"], wl["alphas"].size, wl["x"].size
    launches_per_step = max(1.0, prof["launches"] / max(1, prof["steps"]))
    return (8.0 * L + 2.0 * T * A * 8.0) / launches_per_step


def design_bytes(wl, q, prof) -> float:
    """Bytes per launch the design adds: the FP32 chunk partials [2][T][A] written by
    the contraction (and read back once by the FP64 accumulation)."""
    T, A, Kc = wl["T"], wl["alphas"].size, q["chunk"]
    prods = prof["work"] / max(1, prof["launches"]) / (T * A)
    return prods / Kc * 2 * T * A * 8


def run_gpu(wl, prec: str, split: bool, steps: int, warmup: int, autotune: bool = True):
    import torch
    from paper_2405_16911_amd import cyclo
    flags = PREC_FLAGS[prec] | (cyclo.CYC_TW_SPLIT if split else 0)
    x = torch.from_numpy(wl["x"]).to("cuda")
    T, alphas, blk = wl["T"], wl["alphas"], wl["block"]
    A = alphas.size
    tuned = cyclo.cyc_autotune(alphas.size, T, flags) if autotune else None
    st = cyclo.CyclicStream(alphas, T, flags)
    R = torch.empty((T, A), dtype=torch.complex64, device="cuda")
    Rc = torch.empty_like(R)
    blocks = [x[i:i + blk] for i in range(0, x.numel(), blk)]

    def step():
        st.reset()
        for b in blocks:
            st.push(b)
        return cyclo.cyc_read(st._s, R, Rc)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    st.profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        n_used = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    prof = st.profile_read()
    prof["steps"] = steps
    st.profile(False)
    q = st.query()
    st.close()
    triples = float(A) * T * n_used
    q["kernel_cfg_name"] = cyclo.cyc_kernel_cfg_info(q["kernel_cfg"])["name"]
    cells = sample_cells(T, A)
    Rh, Rch = R.cpu().numpy(), Rc.cpu().numpy()
    got = [(complex(Rh[t, j]), complex(Rch[t, j])) for t, j in cells]
    return dict(sec_per_step=dt, n_used=n_used, triples=triples, prof=prof, query=q, tuned=tuned, cells=got)


def oracle_cells(wl):
    """The oracle's direct sums over the whole record at the sampled cells, and the
    per-lag scales s_t (for scaled errors).  Part of the CPU (oracle) leg."""
    from oracle.cyclic import cyclic_cell, scale_per_lag
    T, alphas, x = wl["T"], wl["alphas"], wl["x"]
    t0 = time.perf_counter()
    cells = sample_cells(T, alphas.size)
    ref = [cyclic_cell(x, alphas[j], t, T) for t, j in cells]
    s = scale_per_lag(x, T)
    return dict(cells=cells, ref=ref, s=s, seconds=time.perf_counter() - t0)


def error_report(run, oc):
    """Max / median scaled error |Rhat - R| / s_t over the sampled cells (both tables),
    and max plain relative error at the feature cells (|R| >= 0.1 s_t)."""
    scaled, rel = [], []
    for (t, _), (g, gc), (r, rc) in zip(oc["cells"], run["cells"], oc["ref"]):
        for a, b in ((g, r), (gc, rc)):
            e = abs(a - b)
            scaled.append(e / oc["s"][t])
            if abs(b) >= 0.1 * oc["s"][t]:
                rel.append(e / abs(b))
    return dict(cells=len(scaled), max_scaled_error=float(np.max(scaled)),
                median_scaled_error=float(np.median(scaled)),
                feature_cells=len(rel), max_rel_error_at_features=float(np.max(rel)) if rel else None)


def cpu_baseline(wl, n_samples: int):
    """The FP64 oracle (NumPy/BLAS) on a bounded sample of the same workload."""
    from oracle.cyclic import cyclic_tables
    T, alphas = wl["T"], wl["alphas"]
    A = alphas.size
    sel = np.unique(np.concatenate([np.linspace(0, A - 1, 61).astype(int), [A // 2, A // 4, 3 * A // 4]]))
    sel = sel[:64]
    x = wl["x"][:n_samples]
    threads = len(os.sched_getaffinity(0))
    try:
        from threadpoolctl import threadpool_info
        info = [p for p in threadpool_info() if p.get("user_api") == "blas"]
        if info:
            threads = int(info[0]["num_threads"])
    except Exception:
        pass
    t0 = time.perf_counter()
    _, _, n_used = cyclic_tables(x, alphas[sel], T, chunk=4096)
    dt = time.perf_counter() - t0
    rate = sel.size * T * n_used / dt
    model = platform.processor() or platform.machine()
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return dict(value=rate, unit=UNIT, cores=threads, kind="oracle",
                sample=f"first {n_samples} samples, all {T} lags, {sel.size} of {A} alphas "
                       f"(incl. 0, +-1/4); FP64 NumPy direct sum; {dt:.1f} s; {threads} BLAS threads "
                       f"of {len(os.sched_getaffinity(0))} usable CPUs; {model}")


def batch_workload(n_streams: int = 512, seed: int = 4, T: int = 64):
    """Mixed-modulation batch: uneven lengths (log-uniform 2^12..2^20) and alpha sets."""
    from paper_2405_16911_amd import siggen
    xs, alists, metas = [], [], []
    for s in range(n_streams):
        x, m = siggen.mixed_stream(seed, s)
        xs.append(x)
        alists.append(siggen.uniform_grid(m["n_alpha"], -0.5))
        metas.append(m)
    return dict(xs=xs, alists=alists, T=T, metas=metas,
                desc=f"mixed_{n_streams}streams_T{T}_L2^12-2^20_A64-2048")


def run_batch(bw, prec: str, steps: int, warmup: int, compare_single: bool = False):
    """One step = reset, one batched push of every stream's record, batched read."""
    import torch
    from paper_2405_16911_amd import cyclo
    flags = PREC_FLAGS[prec]
    T = bw["T"]
    dev = [torch.from_numpy(x).to("cuda") for x in bw["xs"]]
    b = cyclo.CyclicBatch(bw["alists"], T, flags)
    Rs = [torch.empty((T, a.size), dtype=torch.complex64, device="cuda") for a in bw["alists"]]
    Rcs = [torch.empty_like(r) for r in Rs]

    def step():
        b.reset()
        b.push(dev)
        return cyclo.cyc_batch_read(b._b, Rs, Rcs)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        nu = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    q = b.query()
    # one more step with HIP events around every persistent contraction launch
    # (direct launches instead of the graph while profiling): kernel-only rate
    b.profile(True)
    step()
    kp = b.profile_read()
    b.profile(False)
    b.close()
    work = float(sum(a.size * T * n for a, n in zip(bw["alists"], nu)))
    k_tflops = FLOPS_PER_TRIPLE * kp["work"] / (kp["total_ms"] * 1e-3) / 1e12 if kp["total_ms"] > 0 else None
    out = dict(dtype=prec, value=work / dt, ms_per_step=1e3 * dt, work=work,
               kernel_cfg=cyclo.cyc_kernel_cfg_info(q["kernel_cfg"])["name"],
               rounds_per_push=q["rounds"], graph=q["graph"],
               mfma_frac_whole_path=FLOPS_PER_TRIPLE * work / dt / 1e12 / PEAK_TFLOPS[prec],
               kernel_ms_per_step=kp["total_ms"], kernel_launches_per_step=kp["launches"],
               kernel_tflops=k_tflops,
               kernel_frac=k_tflops / PEAK_TFLOPS[prec] if k_tflops else None)
    if compare_single:
        # the same work as one single-state push per stream, back to back
        old = os.environ.get("CYC_WORKSPACE_MB")
        os.environ["CYC_WORKSPACE_MB"] = "8"  # 512 states: keep each workspace small
        try:
            states = [cyclo.CyclicStream(a, T, flags) for a in bw["alists"]]
        finally:
            if old is None:
                os.environ.pop("CYC_WORKSPACE_MB", None)
            else:
                os.environ["CYC_WORKSPACE_MB"] = old
        for _ in range(max(1, warmup)):
            for st, d in zip(states, dev):
                st.reset()
                st.push(d)
                cyclo.cyc_read(st._s, None, None)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            for st, d, R, Rc in zip(states, dev, Rs, Rcs):
                st.reset()
                st.push(d)
                cyclo.cyc_read(st._s, R, Rc)
        torch.cuda.synchronize()
        out["single_state_loop_ms_per_step"] = 1e3 * (time.perf_counter() - t0) / steps
        for st in states:
            st.close()
    return out


def run_grid(wl, steps: int, warmup: int):
    """The uniform-grid form (fold + FP64 FFT) on the same record and grid: exact, and
    available only because the grid is uniform with a power-of-two size; context for
    the dense contraction, never part of its roofline."""
    import torch
    from paper_2405_16911_amd import cyclo
    T, alphas, blk = wl["T"], wl["alphas"], wl["block"]
    A = alphas.size
    alpha0 = float(alphas[0])
    assert np.allclose(alphas, alpha0 + np.arange(A) / A, rtol=0, atol=1e-15)
    x = torch.from_numpy(wl["x"]).to("cuda")
    g = cyclo.GridStream(alpha0, A, T)
    R = torch.empty((T, A), dtype=torch.complex64, device="cuda")
    Rc = torch.empty_like(R)
    blocks = [x[i:i + blk] for i in range(0, x.numel(), blk)]

    def step():
        g.reset()
        for b in blocks:
            g.push(b)
        return g.read_into(R, Rc)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        n_used = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    g.close()
    return dict(workload=wl["desc"] + "_uniform_grid_fold_fft", value=float(A) * T * n_used / dt,
                ms_per_step=1e3 * dt, arithmetic="FP64 fold and FFT", exact_on="uniform grids, A a power of two")


def run_proposal(n_train: int, pool, compare_no_local: bool = False):
    """Learned proposal trained in this run, then timed against the full fine grid.

    Windows of 65536 mixed-modulation samples, labels from the full-grid
    estimator (65536 alphas, lags 0..63, BF16), BF16 training with FP32
    master weights and random carrier-shift augmentation; the fallback
    threshold is tuned on 2048 validation windows for a 1 % miss rate; miss
    rate and timing on 2048 test windows (validation and test windows are the
    same for any training size).
    """
    from paper_2405_16911_amd import proposal
    r = proposal.run(n_train=n_train, n_val=2048, n_test=2048, epochs=30, batch=128, lr=2e-3, wd=0.1, seed=5,
                     target_miss=0.01, log=lambda m: print(m, file=sys.stderr, flush=True), pool=pool,
                     compare_no_local=compare_no_local)
    ev, sp = r["eval"], r["speed"]
    return dict(workload="mixed_gmsk_psk_ofdm_window65536_fine65536_T64",
                metric="learned-proposal vs full-grid speedup at equal error",
                speedup=sp["speedup"], miss_rate=ev["trained"]["miss_rate"],
                fallback_rate=ev["trained"]["fallback_rate"], theta=r["theta"],
                speedup_no_fallback=sp["speedup_no_fallback"],
                full_grid_kernel_tflops=sp["full_grid_kernel_tflops"],
                full_grid_kernel_frac=sp["full_grid_kernel_tflops"] / PEAK_TFLOPS["bf16"],
                network="4 circular conv1d (64 ch, k 7) + dense 65536->1024 head + a shared local head "
                        "(64 weights shared by all coarse bins; a deviation from the specified network, which "
                        "has no local head: it lets every bin learn from the spectral lines of all bins at "
                        "small training sizes)",
                miss_rate_no_fallback=ev["trained"]["miss_rate_without_fallback"],
                miss_rate_untrained=ev["untrained"]["miss_rate_without_fallback"],
                miss_rate_heuristic=ev["heuristic"]["miss_rate_without_fallback"],
                max_rel_diff_vs_full_grid=sp["max_rel_diff_vs_full_grid"],
                evaluated_alphas_per_window=sp["evaluated_alphas_per_window"],
                full_grid_ms_per_window=1e3 * sp["full_grid_s"] / sp["windows"],
                full_grid_fft_ms_per_window=1e3 * sp["full_grid_fft_s"] / sp["windows"],
                proposal_ms_per_window=1e3 * sp["proposal_path_s"] / sp["windows"],
                theta_curve=r["theta_curve"], train=r["train"], labelling_s=r["labelling_s"],
                positives_per_window=r["positives_per_window"],
                windows=dict(train=n_train, val=2048, test=2048),
                no_local_head=r.get("no_local_head"))


def copy_calibration(nbytes: int = 256 << 20, reps: int = 5):
    """A plain copy kernel of known size: reads and writes nbytes per launch."""
    import torch
    src = torch.rand(nbytes // 4, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_per_launch": nbytes, "launches": reps}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=sorted(PREC_FLAGS), default="f32")
    ap.add_argument("--split", action="store_true")
    ap.add_argument("--workload", default="qpsk_rrc_2p24",
                    help="qpsk_rrc_2p24 (default), gmsk_32k, window_t64, or none (extra forms only)")
    ap.add_argument("--variants", default="bf16,f16,bf16s,f16s",
                    help="extra precision forms timed after the main one ('' for none)")
    ap.add_argument("--cpu-samples", type=int, default=6 << 20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--forms", default="batch,proposal,grid",
                    help="extra forms measured after the main workload: any of 'batch', 'proposal', 'grid' "
                         "('' for none)")
    ap.add_argument("--proposal-train", type=int, default=49152,
                    help="training windows of the learned proposal trained inside the run")
    ap.add_argument("--proposal-compare-no-local", action="store_true",
                    help="also train the proposal network without its local layer on the same windows")
    ap.add_argument("--batch-streams", type=int, default=512)
    ap.add_argument("--batch-precisions", default="bf16",
                    help="precisions of the batch runs with --workload none (comma-separated)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain elementwise copy of 256 MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the estimator runs and is measured on one GPU only; sharding it "
                                   "across GPUs is designed but not implemented", "n_gpus": args.gpus}))
        raise SystemExit(2)

    forms_wanted = [f for f in args.forms.split(",") if f]
    pool = None
    if "proposal" in forms_wanted:
        from multiprocessing import Pool
        # window generators, forked before anything in this process touches the GPU
        pool = Pool(max(1, min(16, os.cpu_count() or 1)))
    forms = {}
    if args.workload == "none":
        # forms only (for profiling one form at a time); not the measurement line
        if "batch" in forms_wanted:
            bw = batch_workload(args.batch_streams)
            forms["batch"] = dict(workload=bw["desc"], runs=[run_batch(bw, p, max(1, args.steps), args.warmup)
                                                             for p in args.batch_precisions.split(",")])
        if "proposal" in forms_wanted:
            forms["proposal"] = run_proposal(args.proposal_train, pool, args.proposal_compare_no_local)
            pool.close()
        print(json.dumps({"forms": forms}), flush=True)
        return
    wl = workload(args.workload)
    main_run = run_gpu(wl, args.precision, args.split, args.steps, args.warmup, not args.no_autotune)
    prof = main_run["prof"]
    kernel_ms = prof["total_ms"] / max(1, prof["launches"])
    achieved = FLOPS_PER_TRIPLE * prof["work"] / (prof["total_ms"] * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.precision]
    value = main_run["triples"] / main_run["sec_per_step"]

    variants, variant_runs = [], []
    for v in [s for s in args.variants.split(",") if s]:
        prec, split = v.rstrip("s"), v.endswith("s")
        if prec == args.precision and split == args.split:
            continue
        r = run_gpu(wl, prec, split, max(2, args.steps), 1, not args.no_autotune)
        p = r["prof"]
        variant_runs.append(r)
        variants.append(dict(dtype=prec, split=split, value=r["triples"] / r["sec_per_step"],
                             kernel_cfg=r["query"]["kernel_cfg_name"],
                             ms_per_step=1e3 * r["sec_per_step"],
                             speedup_vs_main=(r["triples"] / r["sec_per_step"]) / value,
                             kernel_tflops=FLOPS_PER_TRIPLE * p["work"] / (p["total_ms"] * 1e-3) / 1e12,
                             kernel_frac=(FLOPS_PER_TRIPLE * p["work"] / (p["total_ms"] * 1e-3) / 1e12)
                             / PEAK_TFLOPS[prec],
                             whole_path_frac=FLOPS_PER_TRIPLE * r["triples"] / r["sec_per_step"] / 1e12
                             / PEAK_TFLOPS[prec]))

    out = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * main_run["sec_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.precision + ("+split" if args.split else ""),
        "data": "synthetic",
        "config": {"workload": wl["desc"], "n_samples": int(wl["x"].size), "n_lag": wl["T"],
                   "n_alpha": int(wl["alphas"].size), "push_block": wl["block"],
                   "chunk": main_run["query"]["chunk"], "kernel_cfg": main_run["query"]["kernel_cfg_name"],
                   "autotuned": main_run["tuned"] is not None},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak,
                     "traffic": (profiled_traffic(main_run["query"]["kernel_cfg_name"])
                                 if args.workload == "qpsk_rrc_2p24" else None),
                     "traffic_unit": "bytes per launch (HBM, rocprofv3 counters scaled by a copy kernel)",
                     "algorithmic_bytes_per_launch": algorithmic_bytes(wl, prof),
                     "design_bytes_per_launch": design_bytes(wl, main_run["query"], prof),
                     "design_bytes_note": "FP32 chunk partials written by the contraction and read once by "
                                          "the FP64 accumulation; not algorithmic",
                     "kernel": "contract (chunk contraction)", "kernel_ms_avg": kernel_ms,
                     "launches": prof["launches"], "flops_per_launch": FLOPS_PER_TRIPLE * prof["work"]
                     / max(1, prof["launches"])},
        "whole_path_frac": FLOPS_PER_TRIPLE * value / 1e12 / peak,
        "variants": variants,
    }
    if "batch" in forms_wanted:
        bw = batch_workload(args.batch_streams)
        forms["batch"] = dict(workload=bw["desc"], n_streams=len(bw["xs"]),
                              n_samples=int(sum(x.size for x in bw["xs"])),
                              runs=[run_batch(bw, "bf16", 3, 1, compare_single=True),
                                    run_batch(bw, "f32", 2, 1)])
        del bw
    if "grid" in forms_wanted and args.workload == "qpsk_rrc_2p24":
        forms["grid"] = run_grid(wl, max(3, args.steps), 1)
        forms["grid"]["speedup_vs_dense_main"] = forms["grid"]["value"] / value
    if "proposal" in forms_wanted:
        forms["proposal"] = run_proposal(args.proposal_train, pool)
        pool.close()
    if forms:
        out["forms"] = forms
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_samples)
        # the same (oracle) leg: direct sums at sampled cells for the error of every precision
        oc = oracle_cells(wl)
        out["error_vs_oracle"] = dict(main=error_report(main_run, oc), oracle_seconds=oc["seconds"],
                                      cells="features alpha = 0, +-1/4 and seeded random cells, both tables, "
                                            "direct FP64 sums over the whole record")
        for v, r in zip(variants, variant_runs):
            v["error_vs_oracle"] = error_report(r, oc)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
