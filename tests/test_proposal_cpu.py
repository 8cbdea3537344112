"""Host-side pieces of the learned-proposal driver (no GPU).

The training augmentation claims that a carrier shift of k/1024 cycles per
sample moves the three feature channels by k, 2k and 0 bins and the conjugate
labels by 2k coarse bins; it is checked against the oracle's spectra of the
shifted window itself.  The threshold choice is checked against a direct count.
"""
import numpy as np
import pytest

from oracle import proposal as P
from paper_2405_16911_amd import siggen

torch = pytest.importorskip("torch")


def test_shift_augmentation_matches_a_shifted_window():
    from paper_2405_16911_amd.proposal import shifted_batch
    x = siggen.mixed_stream(5, 3, n=65536)[0].astype(np.complex128)
    k = 37
    y = x * np.exp(2j * np.pi * k * np.arange(x.size) / 1024)
    fx, fy = P.welch_log_spectra(x), P.welch_log_spectra(y)
    feat = torch.from_numpy(fx[:, None, :].copy())
    acf = torch.zeros((1, 1024), dtype=torch.float64)
    acf[0, 100] = 1
    conj = torch.zeros((1, 1024), dtype=torch.float64)
    conj[0, 1000] = 1
    f, lab = shifted_batch(feat, acf, conj, torch.tensor([0]), torch.tensor([k]))
    assert np.abs(f[:, 0, :].numpy() - fy).max() < 1e-8
    assert list(np.nonzero(lab[0].numpy())[0]) == sorted([100, (1000 + 2 * k) % 1024])


def test_conjugate_features_move_by_twice_the_shift():
    # the label shift rests on R_conj of the shifted signal at alpha + 2f equalling
    # R_conj of the original at alpha (up to a phase): a tone at f0 has its
    # conjugate line at 2 f0, the shifted tone at 2 (f0 + k/1024)
    from oracle.cyclic import cyclic_tables
    n = 4096
    f0, k = 5 / 1024, 3
    x = np.exp(2j * np.pi * f0 * np.arange(n))
    y = x * np.exp(2j * np.pi * k * np.arange(n) / 1024)
    al = np.arange(1024) / 1024 - 0.5
    _, Rcx, _ = cyclic_tables(x, al, 2)
    _, Rcy, _ = cyclic_tables(y, al, 2)
    assert np.argmax(np.abs(Rcy[0])) - np.argmax(np.abs(Rcx[0])) == 2 * k


def test_theta_choice_meets_the_target_with_fewest_fallbacks():
    from paper_2405_16911_amd.proposal import choose_theta, miss_rate
    rng = np.random.default_rng(0)
    n = 60
    conf = torch.from_numpy(rng.random(n).astype(np.float32))
    sel = torch.from_numpy((rng.random((n, 1024)) < 0.08).astype(np.uint8))
    lab = torch.from_numpy((rng.random((n, 1024)) < 0.003).astype(np.float32))
    for target in (0.0, 0.2, 0.5, 0.9):
        th = choose_theta(conf, sel, lab, target)
        fb = conf < th
        assert miss_rate(sel, lab, fb)[0] <= target + 1e-12
        # one fewer fallback (the most confident window that falls back) misses the target
        if fb.any():
            drop = int(torch.argmax(torch.where(fb, conf, torch.tensor(-1.0))))
            fb2 = fb.clone()
            fb2[drop] = False
            assert miss_rate(sel, lab, fb2)[0] > target
