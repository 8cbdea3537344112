"""The learned proposal trained on the GPU by the library's own kernels.

Windows of the mixed-modulation workload are labelled by the full-grid
estimator; the network is trained with BF16 operands and FP32 master weights
(AdamW).  On held-out windows the trained network must miss fewer labelled
coarse bins than the same network untrained and than the spectral-peak
heuristic, and the proposal path (spectra, network, selection, contraction on
the selected alphas, fallbacks below the confidence threshold tuned on
validation windows) must be faster than the full grid at a bounded miss rate,
while returning the full grid's values at the alphas it evaluates.

The training script (paper_2405_16911_amd/proposal.py) runs as a child
process so that its window generators (a process pool) start before anything
in that process touches the GPU.
"""
import json
import math
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TARGET = 0.01   # the miss rate the confidence threshold is tuned for
N_VAL, N_TEST = 512, 256


def test_trained_proposal_gains_over_untrained_and_heuristic(tmp_path):
    out = tmp_path / "proposal.json"
    cmd = [sys.executable, "-u", "-m", "paper_2405_16911_amd.proposal", "--n-train", "4096", "--n-val", str(N_VAL),
           "--n-test", str(N_TEST), "--epochs", "20", "--batch", "128", "--lr", "2e-3", "--wd", "0.1",
           "--target-miss", str(TARGET), "--out", str(out)]
    print("  " + " ".join(cmd[3:]), flush=True)
    p = subprocess.run(cmd, cwd=ROOT, capture_output=True, text=True, timeout=400)
    print(p.stdout[-3000:], p.stderr[-2000:], flush=True)
    assert p.returncode == 0
    r = json.loads(out.read_text())
    ev, sp = r["eval"], r["speed"]
    assert r["positives_per_window"] > 1.0
    assert r["train"]["val_loss_best"] < r["train"]["loss_first_epoch"]
    tr = ev["trained"]["miss_rate_without_fallback"]
    assert tr < 0.5 * ev["untrained"]["miss_rate_without_fallback"]
    assert tr < ev["heuristic"]["miss_rate_without_fallback"]
    # theta is tuned on the validation windows for the target miss rate; on the
    # test windows the rate may differ from it by sampling alone: three standard
    # deviations of a binomial proportion over the labelled bins of both sets
    pos = r["positives_per_window"]
    allow = 3.0 * math.sqrt(TARGET * (1.0 - TARGET) * (1.0 / (pos * N_TEST) + 1.0 / (pos * N_VAL)))
    assert ev["trained"]["miss_rate"] <= TARGET + allow
    assert sp["max_rel_diff_vs_full_grid"] < 1e-3
    assert sp["speedup_no_fallback"] > 4.0
    assert sp["speedup"] > 1.5
