"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Error measure (per table entry): scaled error |Rhat - R| / s_t with
s_t = (1/N_used) sum_n |x[n+t]| |x[n]|, the condition scale of the length-N
dot product behind each entry (so entries where R is near zero are judged
against what rounding can actually do there).  Bounds (tests/_bounds.py):
  FP32 operands                   <= 1e-5 per cell
  BF16 / FP16 operands (+ split)  per cell, six standard deviations of the
                                  random-walk rounding model plus 1e-5
"""
import os

import numpy as np
import pytest

from _bounds import bound, check_cells, scaled_errors
from oracle.cyclic import cyclic_cell, cyclic_tables, roundoff_ratio_per_lag, scale_per_lag
from paper_2405_16911_amd import siggen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cy():
    from paper_2405_16911_amd import cyclo
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cyclo.lib()
    return cyclo


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _run(cy, x, alphas, T, flags=0, splits=None, env=None):
    old = {}
    for k, v in (env or {}).items():
        old[k] = os.environ.get(k)
        os.environ[k] = str(v)
    try:
        st = cy.CyclicStream(alphas, T, flags)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    xd = _dev(x)
    pos = 0
    for n in (splits or [x.size]):
        st.push(xd[pos:pos + n])
        pos += n
    assert pos == x.size
    R, Rc, n = st.read()
    torch.cuda.synchronize()
    q = st.query()
    st.close()
    return R.cpu().numpy(), Rc.cpu().numpy(), n, q


def _scaled_err(got, ref, s):
    return np.abs(got.astype(np.complex128) - ref) / s[:, None]


def _check(x, alphas, T, R, Rc, n, flags, chunk, label=""):
    Ro, Rco, no = cyclic_tables(x, alphas, T)
    assert n == no
    return check_cells(x, T, flags, chunk, R, Rc, Ro, Rco, label)


def test_config1_gmsk_fp32(cy):
    """GMSK 32768 samples, T = 32, alpha = k/128 (the small single-stream workload)."""
    x = siggen.gmsk_stream(n=32768, seed=1)
    alphas = np.arange(128) / 128
    R, Rc, n, q = _run(cy, x, alphas, 32)
    _check(x, alphas, 32, R, Rc, n, 0, q["chunk"])


@pytest.mark.parametrize("flags", [1, 2, 1 | 4, 2 | 4])
def test_config1_low_precision(cy, flags):
    x = siggen.gmsk_stream(n=32768, seed=1)
    alphas = np.arange(128) / 128
    R, Rc, n, q = _run(cy, x, alphas, 32, flags=flags)
    _check(x, alphas, 32, R, Rc, n, flags, q["chunk"], f"flags {flags}")


@pytest.mark.parametrize("prec", [1, 2])
def test_split_lowers_the_error(cy, prec):
    """The split modulated operand removes one of the two operand roundings, so
    on the same input the median scaled error over all cells must fall (by
    about sqrt(2) for BF16; more for FP16, whose unsplit operand is formed in
    FP16 arithmetic)."""
    T, A = 37, 150
    x = siggen.qpsk_rrc_stream(n=3 * 4096 + 123 + T, seed=3)
    alphas = np.random.default_rng(5).uniform(-0.5, 0.5, size=A)
    Ro, Rco, _ = cyclic_tables(x, alphas, T)
    med = {}
    for split in (0, 4):
        R, Rc, n, q = _run(cy, x, alphas, T, flags=prec | split)
        eR, eRc = scaled_errors(x, T, R, Rc, Ro, Rco)
        med[split] = float(np.median(np.concatenate([eR.ravel(), eRc.ravel()])))
    print(f"  prec {prec}: median scaled error {med[0]:.3e} unsplit, {med[4]:.3e} split", flush=True)
    assert med[4] < 0.85 * med[0], med


@pytest.mark.parametrize("flags", [0, 1, 2, 5])
@pytest.mark.parametrize("T,A", [(37, 150), (128, 70), (5, 1), (257, 66)])
def test_ragged_shapes(cy, flags, T, A):
    """Lag/alpha counts that are not tile multiples; several chunks plus a ragged tail."""
    rng = np.random.default_rng(T * 1000 + A)
    L = 3 * 4096 + 123 + T
    x = siggen.qpsk_rrc_stream(n=L, seed=3)
    alphas = rng.uniform(-2.0, 2.0, size=A)
    alphas[0] = 0.0
    R, Rc, n, q = _run(cy, x, alphas, T, flags=flags, splits=[1000, 5000, 1, 7000, L - 13001])
    assert q["n_committed"] == ((L - T + 1) // q["chunk"]) * q["chunk"]
    _check(x, alphas, T, R, Rc, n, flags, q["chunk"], f"T={T} A={A} flags {flags}")
    # run-to-run bitwise reproducibility (fixed reduction order, no races)
    R2, Rc2, _, _ = _run(cy, x, alphas, T, flags=flags)
    assert np.array_equal(R, R2) and np.array_equal(Rc, Rc2)


@pytest.mark.parametrize("flags", [0, 1])
def test_maximum_lag_count(cy, flags):
    """T = 4096, the largest lag count: 32 lag tiles, two full chunks and a
    partial one, five cycle frequencies (one alpha tile, ragged)."""
    T = 4096
    x = siggen.qpsk_rrc_stream(n=T - 1 + 2 * 4096 + 905, seed=31)
    alphas = np.array([0.0, 0.1, -0.25, 1 / 3, 0.4999])
    R, Rc, n, q = _run(cy, x, alphas, T, flags=flags, splits=[5000, x.size - 5000])
    _check(x, alphas, T, R, Rc, n, flags, q["chunk"], f"T={T} flags {flags}")


@pytest.mark.parametrize("flags", [0, 1])
def test_many_cycle_frequencies_sampled(cy, flags):
    """65536 cycle frequencies (1024 alpha tiles, the proposal's fine grid):
    sampled columns, including the first and last tiles, against the oracle
    evaluated on those cycle frequencies alone."""
    T, A = 8, 65536
    x = siggen.mixed_stream(4, 2, n=2 * 4096 + 300 + T)[0]
    alphas = -0.5 + np.arange(A) / A
    R, Rc, n, q = _run(cy, x, alphas, T, flags=flags)
    rng = np.random.default_rng(flags)
    cols = np.unique(np.concatenate([np.arange(64), np.arange(A - 64, A), rng.integers(0, A, size=256)]))
    Ro, Rco, no = cyclic_tables(x, alphas[cols], T)
    assert n == no
    check_cells(x, T, flags, q["chunk"], R[:, cols], Rc[:, cols], Ro, Rco, f"{cols.size} sampled columns")


def test_every_kernel_configuration(cy):
    """Each tile configuration against the oracle; within one precision/split mode
    all configurations give bit-identical tables (same operands, same order)."""
    T, A = 70, 150
    x = siggen.qpsk_rrc_stream(n=2 * 4096 + 555, seed=9)
    alphas = np.random.default_rng(1).uniform(-0.5, 0.5, size=A)
    by_mode = {}
    tbl_bits = cy.CYC_TBL_R | cy.CYC_TBL_RCONJ
    infos = [cy.cyc_kernel_cfg_info(i) for i in range(cy.cyc_kernel_cfg_count())]
    # two-table configurations first, so every one-table configuration has its reference
    for info in sorted(infos, key=lambda i: bool(i["flags"] & tbl_bits)):
        idx = info["index"]
        st = cy.CyclicStream(alphas, T, info["flags"])
        st.set_kernel_cfg(idx)
        xd = _dev(x)
        st.push(xd[:5000])
        st.push(xd[5000:])
        R, Rc, n = st.read()
        torch.cuda.synchronize()
        st.close()
        print(f"  cfg {idx} {info['name']}", flush=True)
        mode = info["flags"] & ~tbl_bits
        if info["flags"] & tbl_bits:
            # one table: bitwise the two-table configurations' table
            ref = by_mode[mode]
            if info["flags"] & cy.CYC_TBL_R:
                assert Rc is None and np.array_equal(R.cpu().numpy(), ref[0]), info["name"]
            else:
                assert R is None and np.array_equal(Rc.cpu().numpy(), ref[1]), info["name"]
            continue
        R, Rc = R.cpu().numpy(), Rc.cpu().numpy()
        _check(x, alphas, T, R, Rc, n, info["flags"], 4096, info["name"])
        ref = by_mode.setdefault(mode, (R, Rc))
        assert np.array_equal(ref[0], R) and np.array_equal(ref[1], Rc), info["name"]


def test_default_chunk_length_by_shape(cy, monkeypatch):
    """FP32 states commit 4096-product chunks.  A 16-bit state takes 16384 or
    8192 when one launch (the 2^18-product coalescing target, else a
    2^16-sample push) still gives two workgroups per CU over its lag-by-alpha
    tiles (the default tiles: 128 lags x 64 alphas above 64 lags, 64 x 128 at
    33..64); CYC_CHUNK overrides."""
    monkeypatch.delenv("CYC_CHUNK", raising=False)
    monkeypatch.delenv("CYC_KERNEL_CFG", raising=False)
    monkeypatch.delenv("CYC_COALESCE", raising=False)
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    bf16 = cy.CYC_OP_BF16

    def chunk(T, A, flags):
        st = cy.CyclicStream(siggen.uniform_grid(A, -0.5), T, flags)
        info = cy.cyc_kernel_cfg_info(st.query()["kernel_cfg"])
        k = st.query()["chunk"]
        st.close()
        tiles = -(-A // info["alpha_tile"]) * -(-T // info["lag_tile"])
        return k, tiles

    def rule(tiles, launch):
        return 16384 if tiles * (launch // 16384) >= 2 * ncu else 8192 if tiles * (launch // 8192) >= 2 * ncu else 4096

    assert chunk(128, 4096, cy.CYC_OP_FP32)[0] == 4096
    assert chunk(64, 65536, cy.CYC_OP_FP32)[0] == 4096
    shapes = [(128, 4096), (64, 65536), (32, 128), (64, 2048), (64, 512)]
    for T, A in shapes:
        k, tiles = chunk(T, A, bf16)
        assert k == rule(tiles, 1 << 18), (T, A, tiles, k)
    monkeypatch.setenv("CYC_COALESCE", "0")
    for T, A in shapes:
        k, tiles = chunk(T, A, bf16)
        assert k == rule(tiles, 1 << 16), (T, A, tiles, k)
    monkeypatch.setenv("CYC_CHUNK", "4096")
    assert chunk(64, 65536, bf16)[0] == 4096


@pytest.mark.parametrize("flags", [1, 2, 5])
def test_push_coalescing(cy, flags, monkeypatch):
    """16-bit pushes wait until the coalescing target is pending; the results are
    bit for bit those of committing at every push, whatever the segmentation and
    with reads in between, and match the oracle."""
    x = siggen.qpsk_rrc_stream(n=40000, seed=9)
    alphas = np.random.default_rng(11).uniform(-0.5, 0.5, size=200)
    T = 40
    env0 = {"CYC_CHUNK": 1024, "CYC_COALESCE": 0}
    envc = {"CYC_CHUNK": 1024, "CYC_COALESCE": 5000}  # 5 chunks
    ref = _run(cy, x, alphas, T, flags=flags, env=env0)
    rng = np.random.default_rng(flags)
    for trial in range(3):
        cuts = np.sort(rng.choice(np.arange(1, x.size), size=5 + 15 * trial, replace=False))
        splits = np.diff(np.concatenate([[0], cuts, [x.size]])).tolist()
        got = _run(cy, x, alphas, T, flags=flags, splits=splits, env=envc)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), trial
        assert got[3]["n_committed"] == ref[3]["n_committed"] == ((x.size - T + 1) // 1024) * 1024
    # a push below the target commits nothing; one that reaches it commits every
    # complete chunk; a read in between commits the rest and changes nothing later
    for k, v in envc.items():
        monkeypatch.setenv(k, str(v))
    st = cy.CyclicStream(alphas, T, flags)
    for k in envc:
        monkeypatch.delenv(k)
    xd = _dev(x)
    st.push(xd[:4000])
    assert st.query()["n_committed"] == 0
    st.push(xd[4000:5150])                   # 5111 products: below 5 chunks
    assert st.query()["n_committed"] == 0
    st.push(xd[5150:5200])                   # 5161 products
    assert st.query()["n_committed"] == 5 * 1024
    st.push(xd[5200:9000])
    assert st.query()["n_committed"] == 5 * 1024
    R1, Rc1, n1 = st.read()
    assert n1 == 9000 - T + 1 and st.query()["n_committed"] == 8 * 1024
    mid = _run(cy, x[:9000], alphas, T, flags=flags, env=env0)
    assert np.array_equal(R1.cpu().numpy(), mid[0]) and np.array_equal(Rc1.cpu().numpy(), mid[1])
    st.push(xd[9000:])
    R2, Rc2, n2 = st.read()
    torch.cuda.synchronize()
    st.close()
    assert n2 == ref[2]
    assert np.array_equal(R2.cpu().numpy(), ref[0]) and np.array_equal(Rc2.cpu().numpy(), ref[1])
    _check(x, alphas, T, ref[0], ref[1], ref[2], flags, 1024, f"flags {flags}")


def test_autotune_picks_a_configuration(cy, tmp_path):
    cache = tmp_path / "tune.txt"
    os.environ["CYC_TUNE_CACHE"] = str(cache)
    try:
        res = cy.cyc_autotune(300, 40, cy.CYC_OP_BF16)
        assert res["cfg"] >= 0 and res["ms_per_push"] > 0
        info = cy.cyc_kernel_cfg_info(res["cfg"])
        assert info["flags"] == cy.CYC_OP_BF16
        st = cy.CyclicStream(np.arange(300) / 300, 40, cy.CYC_OP_BF16)
        assert st.query()["kernel_cfg"] == res["cfg"]
        st.close()
        line = cache.read_text().split()
        assert line[-1] == info["name"] and line[3] == "40"
    finally:
        os.environ.pop("CYC_TUNE_CACHE", None)


def test_segmentation_bitwise_and_determinism(cy):
    x = siggen.gmsk_stream(n=20000, seed=5)
    alphas = np.arange(96) / 96 - 0.5
    T = 24
    ref = _run(cy, x, alphas, T)
    again = _run(cy, x, alphas, T)
    assert np.array_equal(ref[0], again[0]) and np.array_equal(ref[1], again[1])
    rng = np.random.default_rng(0)
    for trial in range(3):
        cuts = np.sort(rng.choice(np.arange(1, x.size), size=10 + trial * 20, replace=False))
        splits = np.diff(np.concatenate([[0], cuts, [x.size]])).tolist()
        got = _run(cy, x, alphas, T, splits=splits)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), trial
    # pushes shorter than T, one sample at a time for the first 3*T samples
    splits = [1] * (3 * T) + [x.size - 3 * T]
    got = _run(cy, x, alphas, T, splits=splits)
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])


def test_small_chunks_many_commits(cy):
    x = siggen.gmsk_stream(n=5000, seed=6)
    alphas = np.arange(40) / 40
    T = 9
    R, Rc, n, q = _run(cy, x, alphas, T, env={"CYC_CHUNK": 64}, splits=[100, 1, 2000, 2899])
    assert q["chunk"] == 64
    _check(x, alphas, T, R, Rc, n, 0, 64)
    # workspace limited to one chunk per launch
    R2, Rc2, n2, _ = _run(cy, x, alphas, T, env={"CYC_CHUNK": 64, "CYC_WORKSPACE_MB": 0})
    assert np.array_equal(R, R2) and np.array_equal(Rc, Rc2)


def test_edge_cases(cy):
    alphas = np.array([0.0, 0.25, -0.125])
    T = 8
    x = siggen.gmsk_stream(n=64, seed=7)
    st = cy.CyclicStream(alphas, T)
    R, Rc, n = st.read()
    assert n == 0 and not R.abs().sum().item() and not Rc.abs().sum().item()
    xd = _dev(x)
    st.push(xd[:0])
    st.push(xd[:T - 1])
    R, Rc, n = st.read()
    assert n == 0 and not R.abs().sum().item()
    st.push(xd[T - 1:T])
    R, Rc, n = st.read()
    torch.cuda.synchronize()
    assert n == 1
    Ro, Rco, _ = cyclic_tables(x[:T], alphas, T)
    assert np.max(np.abs(R.cpu().numpy() - Ro)) < 1e-5 * np.max(np.abs(Ro))
    # reset == fresh state
    st.push(xd[T:])
    st.reset()
    st.push(xd)
    R1, Rc1, n1 = st.read()
    fresh = cy.CyclicStream(alphas, T)
    fresh.push(xd)
    R2, Rc2, n2 = fresh.read()
    torch.cuda.synchronize()
    assert n1 == n2 == x.size - T + 1
    assert torch.equal(R1, R2) and torch.equal(Rc1, Rc2)
    # read one table only
    Ronly, none, _ = st.read(which=(True, False))
    assert none is None and torch.equal(Ronly, R1)
    st.close()
    fresh.close()


def test_complex128_output(cy):
    x = siggen.gmsk_stream(n=9000, seed=8)
    alphas = np.arange(32) / 32
    R, Rc, n, q = _run(cy, x, alphas, 16, flags=8)
    assert R.dtype == np.complex128
    _check(x, alphas, 16, R, Rc, n, 0, q["chunk"])


def test_abi_errors_on_device(cy):
    import ctypes
    st = cy.CyclicStream([0.1], 4)
    L = cy.lib()
    assert L.cyc_push(st._s, None, 5, None) == cy.CYC_EINVAL
    assert L.cyc_push(st._s, None, -1, None) == cy.CYC_EINVAL
    assert L.cyc_push(st._s, None, 0, None) == cy.CYC_OK
    n = ctypes.c_int64(-1)
    assert L.cyc_read(st._s, None, None, ctypes.byref(n), None) == cy.CYC_OK and n.value == 0
    st.close()


_CFG2 = {}


def _config2_reference():
    """The 2^24-sample QPSK-RRC record, its sampled cells from the oracle's direct
    sum over the whole record, and the per-lag scales (computed once)."""
    if not _CFG2:
        L, T, A = 1 << 24, 128, 4096
        x = siggen.qpsk_rrc_stream(n=L)
        alphas = siggen.uniform_grid(A, -0.5)
        rng = np.random.default_rng(2)
        cells = [(0, 2048), (1, 2048), (4, 1024), (4, 3072), (127, 2048), (64, 0), (3, 2049)]
        cells += [(int(rng.integers(0, T)), int(rng.integers(0, A))) for _ in range(9)]
        ref = [cyclic_cell(x, alphas[j], t, T) for t, j in cells]
        _CFG2.update(x=x, alphas=alphas, cells=cells, ref=ref, T=T, A=A,
                     s=scale_per_lag(x, T), r=roundoff_ratio_per_lag(x, T))
    return _CFG2


@pytest.mark.parametrize("flags", [0, 1, 2, 1 | 4, 2 | 4])
def test_config2_full_size_sampled_cells(cy, flags):
    """QPSK-RRC 2^24 samples, T = 128, 4096 alphas in [-1/2, 1/2), 256 pushes of
    65536, in every operand precision (the precision forms run on this record).

    Sampled cells (features at alpha = 0, +-1/4 and random cells) are checked
    one by one against the oracle's direct sum over the whole record, each
    within its per-cell bound; max and median scaled errors are printed.
    """
    c = _config2_reference()
    x, alphas, T, A = c["x"], c["alphas"], c["T"], c["A"]
    L, blk = x.size, 65536
    R, Rc, n, q = _run(cy, x, alphas, T, flags=flags, splits=[blk] * (L // blk))
    assert n == L - T + 1
    errs, ratios = [], []
    for (t, j), (r, rc) in zip(c["cells"], c["ref"]):
        s = c["s"][t]
        for got, ref in ((R[t, j], r), (Rc[t, j], rc)):
            e = abs(complex(got) - ref) / s
            errs.append(e)
            ratios.append(e / float(bound(flags, q["chunk"], c["r"][t], abs(ref) / s)))
    print(f"  config-2 flags {flags}: {len(errs)} sampled cells, max scaled error {max(errs):.3e}, "
          f"median {np.median(errs):.3e}, max error/bound {max(ratios):.3f}", flush=True)
    assert max(ratios) <= 1.0
    # the strongest features of QPSK-RRC at 4 samples/symbol: alpha = 0 and +-1/4
    m = np.abs(R[2])
    assert set(np.argsort(-m)[:3]) == {2048, 1024, 3072}


@pytest.mark.parametrize("flags", [0, 1, 2, 2 | 4])
@pytest.mark.parametrize("T,A", [(128, 150), (40, 200), (9, 65)])
def test_one_table_states(cy, flags, T, A):
    """CYC_TBL_R / CYC_TBL_RCONJ: a state that keeps one table contracts only
    that table; its table matches the oracle within the bound and equals the
    two-table state's bit for bit (same operands, same summation order), and
    reading the table it does not keep is refused."""
    x = siggen.qpsk_rrc_stream(n=3 * 4096 + 321 + T, seed=17)
    alphas = np.random.default_rng(T + A).uniform(-0.5, 0.5, size=A)
    both = _run(cy, x, alphas, T, flags=flags, splits=[5000, x.size - 5000])
    Ro, Rco, no = cyclic_tables(x, alphas, T)
    for which, tflag in ((0, cy.CYC_TBL_R), (1, cy.CYC_TBL_RCONJ)):
        st = cy.CyclicStream(alphas, T, flags | tflag)
        xd = _dev(x)
        st.push(xd[:5000])
        st.push(xd[5000:])
        got, other, n = st.read()
        torch.cuda.synchronize()
        if which == 1:
            got, other = other, got
        assert other is None and n == no
        got = got.cpu().numpy()
        assert np.array_equal(got, both[which]), (which, tflag)
        ref = Ro if which == 0 else Rco
        check_cells(x, T, flags, both[3]["chunk"], got, got, ref, ref, f"table {which} flags {flags}")
        # the other table is not kept
        import ctypes
        d = torch.empty((T, A), dtype=torch.complex64, device="cuda")
        n_used = ctypes.c_int64(0)
        args = (None, ctypes.c_void_p(d.data_ptr())) if which == 0 else (ctypes.c_void_p(d.data_ptr()), None)
        assert cy.lib().cyc_read(st._s, *args, ctypes.byref(n_used), None) == cy.CYC_EINVAL
        st.close()


def test_one_table_flags_are_refused_where_unsupported(cy):
    import ctypes
    al = np.array([0.1, 0.2])
    out = ctypes.c_void_p()
    L = cy.lib()
    ap = al.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert L.cyc_create_window(ctypes.byref(out), al.ctypes.data_as(ctypes.c_void_p), 2, 4, 64, 2,
                               cy.CYC_TBL_R, None) == cy.CYC_EUNSUPPORTED
    offs = (ctypes.c_int64 * 2)(0, 2)
    assert L.cyc_batch_create(ctypes.byref(out), 1, offs, ap, 4, cy.CYC_TBL_RCONJ, None) == cy.CYC_EUNSUPPORTED
    # both flags = both tables
    st = cy.CyclicStream(al, 4, cy.CYC_TBL_R | cy.CYC_TBL_RCONJ)
    assert st.tables() == (True, True)
    st.close()
