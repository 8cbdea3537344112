"""GPU parity of batched stream states (one persistent launch per round,
replayed from a HIP graph) against the FP64 oracle and against single states.

Per stream the batch must give exactly the single-state tables (same operands,
same order), whatever the round split, and graph replays must equal direct
launches.  Workload: a scaled-down mixed-modulation batch (GMSK, BPSK/QPSK-RRC,
OFDM; random samples/symbol, carrier offset and SNR) with uneven lengths,
including streams shorter than the lag count and empty pushes.
"""
import os

import numpy as np
import pytest

from _bounds import check_cells
from oracle.cyclic import cyclic_tables
from paper_2405_16911_amd import siggen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

@pytest.fixture(scope="module")
def cy():
    from paper_2405_16911_amd import cyclo
    assert torch.cuda.is_available()
    cyclo.lib()
    return cyclo


def _workload(n_streams, seed, T, lmax=1 << 14):
    xs, alists = [], []
    for s in range(n_streams):
        rng = np.random.default_rng(seed * 1000 + s)
        L = int(rng.integers(1, lmax)) if s % 5 else int(rng.integers(0, T))  # some shorter than T
        x, meta = siggen.mixed_stream(seed, s, n=max(L, 1))
        xs.append(x[:L])
        A = int(rng.integers(1, 200))
        alists.append(-0.5 + np.arange(A) / A)
    return xs, alists


def _with_env(env, fn):
    old = {k: os.environ.get(k) for k in env}
    os.environ.update({k: str(v) for k, v in env.items()})
    try:
        return fn()
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def _run_batch(cy, xs, alists, T, flags=0, splits=1, env=None):
    b = _with_env(env or {}, lambda: cy.CyclicBatch(alists, T, flags))
    dev = [torch.from_numpy(np.ascontiguousarray(x)).to("cuda") for x in xs]
    qs = []
    for k in range(splits):
        part = []
        for d in dev:
            n = d.numel()
            a, c = n * k // splits, n * (k + 1) // splits
            part.append(d[a:c] if c > a else None)
        b.push(part)
        qs.append(b.query())
    Rs, Rcs, nu = b.read()
    torch.cuda.synchronize()
    out = ([r.cpu().numpy() for r in Rs], [r.cpu().numpy() for r in Rcs], nu, qs)
    b.close()
    return out


@pytest.mark.parametrize("flags", [0, 1, 2])
def test_batch_matches_oracle_and_single_states(cy, flags):
    T = 64
    xs, alists = _workload(13, 7, T)
    Rs, Rcs, nu, qs = _run_batch(cy, xs, alists, T, flags, splits=3)
    assert qs[-1]["graph"] in (True, False)
    for s, (x, al) in enumerate(zip(xs, alists)):
        Ro, Rco, no = cyclic_tables(x, al, T)
        assert nu[s] == no
        if no == 0:
            assert not np.abs(Rs[s]).any() and not np.abs(Rcs[s]).any()
            continue
        # 16-bit operands: 16384 products per chunk in a batch, 4096 in a single
        # state by default
        chunk = 4096 if flags == 0 else 16384
        check_cells(x, T, flags, chunk, Rs[s], Rcs[s], Ro, Rco, f"stream {s} L={x.size} A={al.size}")
        # single state, same samples, the batch's kernel configuration and chunk
        # length
        st = _with_env({"CYC_CHUNK": chunk}, lambda: cy.CyclicStream(al, T, flags))
        assert st.query()["chunk"] == chunk
        st.set_kernel_cfg(qs[-1]["kernel_cfg"])
        st.push(torch.from_numpy(np.ascontiguousarray(x)).to("cuda"))
        R1, Rc1, n1 = st.read()
        torch.cuda.synchronize()
        st.close()
        assert np.array_equal(R1.cpu().numpy(), Rs[s]) and np.array_equal(Rc1.cpu().numpy(), Rcs[s]), s


def test_batch_rounds_graph_and_segmentation_bitwise(cy):
    T = 40
    xs, alists = _workload(9, 11, T, lmax=20000)
    ref = _run_batch(cy, xs, alists, T, splits=1)
    # tiny workspace: many rounds per push; several pushes (graph replayed each round)
    many = _run_batch(cy, xs, alists, T, splits=4, env={"CYC_WORKSPACE_MB": 0})
    assert max(q["rounds"] for q in many[3]) > 1
    direct = _run_batch(cy, xs, alists, T, splits=4, env={"CYC_NO_GRAPH": 1, "CYC_WORKSPACE_MB": 0})
    assert not any(q["graph"] for q in direct[3])
    for s in range(len(xs)):
        for other in (many, direct):
            assert np.array_equal(ref[0][s], other[0][s]) and np.array_equal(ref[1][s], other[1][s]), s


def test_batch_reset_and_reuse(cy):
    T = 16
    xs, alists = _workload(5, 3, T, lmax=9000)
    b = cy.CyclicBatch(alists, T)
    dev = [torch.from_numpy(np.ascontiguousarray(x)).to("cuda") for x in xs]
    b.push([d if d.numel() else None for d in dev])
    R1, Rc1, n1 = b.read()
    b.reset()
    b.push([d if d.numel() else None for d in dev])
    R2, Rc2, n2 = b.read()
    torch.cuda.synchronize()
    assert n1 == n2
    for a, c in zip(R1 + Rc1, R2 + Rc2):
        assert torch.equal(a, c)
    b.close()


def _long_workload(seed, T):
    """Streams of 2^15..2^18 samples (several 16384-product chunks each) with
    alpha sets up to 2048 bins, most of them not powers of two."""
    xs, alists = [], []
    rng = np.random.default_rng(seed)
    for s, A in enumerate([2048, 1500, 777, 64, 1234, 333]):
        L = int(2 ** rng.uniform(15, 18))
        xs.append(siggen.mixed_stream(seed, s, n=L)[0])
        alists.append(-0.5 + np.arange(A) / A)
    return xs, alists


@pytest.mark.parametrize("flags", [1, 2, 1 | 4, 2 | 4])
def test_batch_16bit_committed_chunks(cy, flags):
    """16-bit batches whose pushes commit whole 16384-product chunks: against the
    oracle on sampled columns (every cell within its bound), bitwise against
    single states with the same chunk length and kernel configuration, and
    bitwise across round splits (a 16 MiB workspace: several rounds per push)
    and graph replay vs direct launches."""
    T = 64
    xs, alists = _long_workload(21, T)
    Rs, Rcs, nu, qs = _run_batch(cy, xs, alists, T, flags, splits=3, env={"CYC_WORKSPACE_MB": 16})
    print(f"  rounds per push {[q['rounds'] for q in qs]}, graph {qs[-1]['graph']}", flush=True)
    assert max(q["rounds"] for q in qs) > 1
    direct = _run_batch(cy, xs, alists, T, flags, splits=3, env={"CYC_WORKSPACE_MB": 16, "CYC_NO_GRAPH": 1})
    one = _run_batch(cy, xs, alists, T, flags, splits=1)
    for s in range(len(xs)):
        for other in (direct, one):
            assert np.array_equal(Rs[s], other[0][s]) and np.array_equal(Rcs[s], other[1][s]), s
    rng = np.random.default_rng(flags)
    for s, (x, al) in enumerate(zip(xs, alists)):
        A = al.size
        assert (x.size - T + 1) // 16384 >= 1
        cols = np.unique(np.concatenate([np.arange(min(8, A)), np.arange(max(0, A - 8), A),
                                         rng.integers(0, A, size=32), [A // 2, A // 4, (3 * A) // 4]]))
        Ro, Rco, no = cyclic_tables(x, al[cols], T)
        assert nu[s] == no
        check_cells(x, T, flags, 16384, Rs[s][:, cols], Rcs[s][:, cols], Ro, Rco,
                    f"stream {s} L={x.size} A={A} ({cols.size} columns)")
        st = _with_env({"CYC_CHUNK": 16384}, lambda: cy.CyclicStream(al, T, flags))
        st.set_kernel_cfg(qs[-1]["kernel_cfg"])
        d = torch.from_numpy(np.ascontiguousarray(x)).to("cuda")
        st.push(d[:x.size // 3])
        st.push(d[x.size // 3:])
        R1, Rc1, n1 = st.read()
        torch.cuda.synchronize()
        st.close()
        assert n1 == nu[s]
        assert np.array_equal(R1.cpu().numpy(), Rs[s]) and np.array_equal(Rc1.cpu().numpy(), Rcs[s]), s
