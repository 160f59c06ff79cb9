"""Fold-in (new rows solved against resident factors) and the serving loop,
on the GPU through the C ABI, against the FP64 oracle.

Tolerances: FP64 within 1e-10 of the oracle (max-abs relative); FP32 within
1e-4 (FP32 Gram accumulation of at most a few thousand terms).  Serving must
give every request the same bits alone, in a mix, and through tf_foldin."""
import numpy as np
import pytest

import synth
from gpu_util import note, pair, problem, rel_max

pytestmark = pytest.mark.gpu


def _requests(dims, mode, sizes, seed):
    N = len(dims)
    other = [d for l, d in enumerate(dims) if l != mode]
    ptr = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    total = int(ptr[-1])
    oidx = np.stack([synth.uniform_ints(seed, 60 + t, total, other[t]) for t in range(N - 1)],
                    axis=1).astype(np.int32) if total else np.zeros((0, N - 1), np.int32)
    vals = synth.values(seed, [max(o, 1) for o in other], oidx, 2, 0, 0.1) if total else \
        np.zeros(0)
    return ptr, oidx.reshape(total, N - 1), vals


def _gpu_foldin(g, mode, ptr, oidx, vals, method, sweeps=3):
    import torch
    from paper_1410_5209_amd import tf
    nreq = len(ptr) - 1
    d_idx = torch.from_numpy(np.ascontiguousarray(oidx)).cuda()
    d_vals = torch.from_numpy(np.ascontiguousarray(vals)).cuda()
    d_rows = torch.empty((nreq, g.K), dtype=torch.float64, device="cuda")
    tf.tf_foldin(g.ctx, mode, ptr, d_idx, d_vals, method, sweeps, d_rows)
    return d_rows.cpu().numpy()


SIZES = [0, 1, 3, 17, 64, 65, 300, 1200]


@pytest.mark.parametrize("mode,reg", [(0, 0), (1, 0), (2, 1)])
@pytest.mark.parametrize("method", [0, 1])
def test_foldin_parity_f64(mode, reg, method):
    from paper_1410_5209_amd import tf
    dims, K = [40, 30, 20], 6
    note(f"foldin f64 mode={mode} reg={reg} method={method}")
    idx, x, A = problem(31, dims, 3000, K, first_zero=False)
    g, o = pair(dims, idx, x, A, K, 0.3, "f64", reg)
    ptr, oidx, vals = _requests(dims, mode, SIZES, 5)
    rows = _gpu_foldin(g, mode, ptr, oidx, vals, method)
    for q in range(len(SIZES)):
        sl = slice(ptr[q], ptr[q + 1])
        want = o.foldin_full(mode, oidx[sl], vals[sl]) if method == tf.TF_FOLDIN_FULL else \
            o.foldin_cdtf(mode, oidx[sl], vals[sl], 3)
        if SIZES[q] == 0:
            assert np.all(rows[q] == 0.0)
        else:
            assert rel_max(rows[q], want) < 1e-10, q
    g.close()


@pytest.mark.parametrize("method", [0, 1])
def test_foldin_k100_f32(method):
    dims, K = [2000, 1500, 1000], 100
    note(f"foldin f32 K=100 method={method}")
    idx, x, A = problem(32, dims, 50000, K, first_zero=False)
    g, o = pair(dims, idx, x, A, K, 1.0, "f32")
    sizes = [1, 20, 375, 4300, 5000]
    ptr, oidx, vals = _requests(dims, 0, sizes, 6)
    rows = _gpu_foldin(g, 0, ptr, oidx, vals, method)
    for q in range(len(sizes)):
        sl = slice(ptr[q], ptr[q + 1])
        want = o.foldin_full(0, oidx[sl], vals[sl]) if method == 0 else \
            o.foldin_cdtf(0, oidx[sl], vals[sl], 3)
        assert rel_max(rows[q], want) < 1e-4, q
    g.close()


def test_foldin_rejects_bad_index_and_large_k():
    from paper_1410_5209_amd import tf
    dims, K = [10, 10, 10], 4
    note("foldin validation")
    idx, x, A = problem(33, dims, 300, K, first_zero=False)
    g, _ = pair(dims, idx, x, A, K, 0.3, "f64")
    ptr, oidx, vals = _requests(dims, 0, [5, 5], 7)
    oidx[7, 1] = 10
    with pytest.raises(tf.TFError, match="entry 7"):
        _gpu_foldin(g, 0, ptr, oidx, vals, 0)
    g.close()
    dims, K = [10, 10, 10], 130
    idx, x, A = problem(34, dims, 300, K, first_zero=False)
    g, o = pair(dims, idx, x, A, K, 0.3, "f64")
    ptr, oidx, vals = _requests(dims, 0, [4], 8)
    with pytest.raises(tf.TFError) as e:
        _gpu_foldin(g, 0, ptr, oidx, vals, 0)
    assert e.value.status == tf.TF_E_UNSUPPORTED
    rows = _gpu_foldin(g, 0, ptr, oidx, vals, 1)          # CDTF has no K limit
    assert rel_max(rows[0], o.foldin_cdtf(0, oidx, vals, 3)) < 1e-10
    g.close()


# ------------------------------------------------------------------ serving

def _serve_setup(prec="f32", K=24):
    dims = [3000, 2000, 1500]
    idx, x, A = problem(35, dims, 60000, K, first_zero=False)
    g, o = pair(dims, idx, x, A, K, 1.0, prec)
    sizes = list(synth.zipf_ints(9, 500, 60, 1.1, 2000))
    ptr, oidx, vals = _requests(dims, 0, sizes, 10)
    return g, o, ptr, oidx, vals


def _slot_bytes_full_rank(N, K, ta, nreq, total):
    """Device bytes of a full-rank serving batch, as the library lays out its
    slot arena: request offsets, chunk tables, indices, values, P, partial
    Gram records (one per 256-entry chunk), rows, per-request status words,
    flags; 256-byte aligned."""
    a = lambda b: (b + 255) & ~255
    nc = nreq + total // 256
    gs = (K * (K + 1) // 2 + K + 3) & ~3
    return (a((nreq + 1) * 8) + a((nreq + 1) * 4) + a(nc * 4) + a(total * (N - 1) * 4) +
            a(total * 8) + a(total * K * ta) + a(nc * gs * ta) + a(nreq * K * 8) + a(nreq * 4) +
            256)


def _submit_all(tf, srv, ptr, oidx, vals, order):
    keep, tickets = [], {}
    for q in order:
        sl = slice(ptr[q], ptr[q + 1])
        oi = np.ascontiguousarray(oidx[sl])
        va = np.ascontiguousarray(vals[sl])
        keep.append((oi, va))
        tickets[q] = tf.tf_serve_submit(srv, tf.make_request(oi, va))
    return keep, tickets


@pytest.mark.parametrize("method", [0, 1])
def test_serving_alone_and_mixed_are_bit_identical(method):
    from paper_1410_5209_amd import tf
    note(f"serving alone vs mix method={method}")
    g, o, ptr, oidx, vals = _serve_setup()
    nreq = len(ptr) - 1
    batch_rows = _gpu_foldin(g, 0, ptr, oidx, vals, method)
    srv = tf.tf_serve_open(g.ctx, tf.tf_serve_default_options(method=method, streams=3))
    alone = np.empty((nreq, g.K))
    for q in range(nreq):                      # one at a time
        sl = slice(ptr[q], ptr[q + 1])
        oi, va = np.ascontiguousarray(oidx[sl]), np.ascontiguousarray(vals[sl])
        t = tf.tf_serve_submit(srv, tf.make_request(oi, va))
        alone[q], st = tf.tf_serve_wait(srv, t, g.K)
        assert st.batch_size >= 1
    for order in (list(range(nreq)), list(reversed(range(nreq)))):   # bursts
        keep, tickets = _submit_all(tf, srv, ptr, oidx, vals, order)
        mixed = np.empty((nreq, g.K))
        sizes = []
        for q in order:
            mixed[q], st = tf.tf_serve_wait(srv, tickets[q], g.K)
            sizes.append(st.batch_size)
        assert np.array_equal(mixed, alone)
        assert max(sizes) > 1                  # the burst was batched
    assert np.array_equal(alone, batch_rows)
    rep = tf.tf_serve_report(srv)
    assert rep.completed == 3 * nreq and rep.p99_us >= rep.p50_us > 0
    tf.tf_serve_close(srv)
    for q in range(nreq):
        sl = slice(ptr[q], ptr[q + 1])
        want = o.foldin_full(0, oidx[sl], vals[sl]) if method == 0 else \
            o.foldin_cdtf(0, oidx[sl], vals[sl], 3)
        assert rel_max(alone[q], want) < 1e-4
    g.close()


def test_serving_device_failures_are_reported_per_request():
    """A batch whose launch fails (forced from the host through the
    tf_serve_inject_fault hook: no kernel runs) completes every one of its
    requests with TF_E_DEVICE and a NaN row, never TF_OK; the server keeps
    serving, and later requests get the rows tf_foldin gives."""
    from paper_1410_5209_amd import tf
    note("serving injected launch failures")
    g, o, ptr, oidx, vals = _serve_setup()
    nreq = len(ptr) - 1
    want = _gpu_foldin(g, 0, ptr, oidx, vals, 0)
    srv = tf.tf_serve_open(g.ctx, tf.tf_serve_default_options(streams=2))
    tf.tf_serve_inject_fault(srv, 3)
    keep = []
    for q in range(nreq):                      # one at a time: one request per batch
        sl = slice(ptr[q], ptr[q + 1])
        oi, va = np.ascontiguousarray(oidx[sl]), np.ascontiguousarray(vals[sl])
        keep.append((oi, va))
        t = tf.tf_serve_submit(srv, tf.make_request(oi, va))
        rc, row, st = tf.tf_serve_wait_status(srv, t, g.K)
        if q < 3:
            assert rc == tf.TF_E_DEVICE and st.status == tf.TF_E_DEVICE
            assert np.all(np.isnan(row))
        else:
            assert rc == tf.TF_OK and st.status == tf.TF_OK
            assert np.array_equal(row, want[q])
    assert "fold-in launch" in tf.tf_serve_last_error(srv)
    rep = tf.tf_serve_report(srv)
    assert rep.failed == 3 and rep.completed == nreq
    # a failed batch in a burst: its requests fail together, the others do not
    tf.tf_serve_inject_fault(srv, 1)
    keep2, tickets = _submit_all(tf, srv, ptr, oidx, vals, list(range(nreq)))
    nfail = 0
    for q in range(nreq):
        rc, row, st = tf.tf_serve_wait_status(srv, tickets[q], g.K)
        if rc == tf.TF_E_DEVICE:
            nfail += 1
            assert np.all(np.isnan(row))
        else:
            assert rc == tf.TF_OK and np.array_equal(row, want[q])
    assert 1 <= nfail < nreq
    tf.tf_serve_close(srv)
    g.close()


def test_serving_numeric_failure_is_per_request():
    """A request whose Gram matrix overflows (it meets a factor row of 1e200,
    so a Cholesky pivot is NaN) completes with TF_E_NUMERIC and a zero row,
    alone and inside a batch; the other requests of its batch complete with
    TF_OK and the same rows as alone (the status is the request's own, not
    the batch's)."""
    from paper_1410_5209_amd import tf
    note("serving per-request numeric status")
    dims, K = [400, 300, 200], 12
    idx, x, A = problem(36, dims, 20000, K, first_zero=False)
    A[1][5, :] = 1e200
    g, o = pair(dims, idx, x, A, K, 1.0, "f64")
    sizes = [30, 8, 50, 3, 40, 12, 25, 9]
    ptr, oidx, vals = _requests(dims, 0, sizes, 12)
    oidx = oidx.copy()
    oidx[ptr[1], 0] = 5                          # requests 1 and 5 meet row 5 of mode 1
    oidx[ptr[5] + 2, 0] = 5
    oidx[np.setdiff1d(np.arange(len(vals)), [ptr[1], ptr[5] + 2]), 0] %= 5
    srv = tf.tf_serve_open(g.ctx, tf.tf_serve_default_options(streams=2))
    alone = []
    for q in range(len(sizes)):
        sl = slice(ptr[q], ptr[q + 1])
        oi, va = np.ascontiguousarray(oidx[sl]), np.ascontiguousarray(vals[sl])
        t = tf.tf_serve_submit(srv, tf.make_request(oi, va))
        alone.append(tf.tf_serve_wait_status(srv, t, K))
    for q, (rc, row, st) in enumerate(alone):
        if q in (1, 5):
            assert rc == tf.TF_E_NUMERIC and np.all(row == 0.0)
        else:
            assert rc == tf.TF_OK
            sl = slice(ptr[q], ptr[q + 1])
            assert rel_max(row, o.foldin_full(0, oidx[sl], vals[sl])) < 1e-10
    keep, tickets = _submit_all(tf, srv, ptr, oidx, vals, list(range(len(sizes))))
    sizes_seen = []
    for q in range(len(sizes)):
        rc, row, st = tf.tf_serve_wait_status(srv, tickets[q], K)
        sizes_seen.append(st.batch_size)
        assert rc == alone[q][0] and np.array_equal(row, alone[q][1])
    assert max(sizes_seen) > 1
    tf.tf_serve_close(srv)
    g.close()


def test_serving_memory_admission_and_busy_queue():
    from paper_1410_5209_amd import tf
    note("serving admission")
    g, o, ptr, oidx, vals = _serve_setup()
    nreq = len(ptr) - 1
    want = _gpu_foldin(g, 0, ptr, oidx, vals, 0)
    biggest = int(np.max(np.diff(ptr)))
    # a budget that holds one largest request per slot forces small batches
    budget = 2 * (_slot_bytes_full_rank(3, g.K, 4, 1, biggest) + 4096)
    srv = tf.tf_serve_open(g.ctx, tf.tf_serve_default_options(streams=2, mem_budget=budget,
                                                              queue_cap=8))
    keep, tickets, busy = [], {}, 0
    for q in range(nreq):
        sl = slice(ptr[q], ptr[q + 1])
        oi, va = np.ascontiguousarray(oidx[sl]), np.ascontiguousarray(vals[sl])
        keep.append((oi, va))
        while True:
            try:
                tickets[q] = tf.tf_serve_submit(srv, tf.make_request(oi, va))
                break
            except tf.TFError as e:
                assert e.status == tf.TF_E_BUSY
                busy += 1
    for q in range(nreq):
        row, st = tf.tf_serve_wait(srv, tickets[q], g.K)
        assert np.array_equal(row, want[q])
    rep = tf.tf_serve_report(srv)
    assert rep.busy_rejects == busy and rep.max_queue <= 8
    assert rep.mean_batch < nreq
    # a request larger than a slot's share is refused
    big = 4 * biggest
    oi = np.zeros((big, 2), dtype=np.int32)
    va = np.ones(big)
    with pytest.raises(tf.TFError) as e:
        tf.tf_serve_submit(srv, tf.make_request(oi, va))
    assert e.value.status == tf.TF_E_INVALID
    tf.tf_serve_close(srv)
    g.close()


def test_serving_replay_poisson_and_close_with_work_in_flight():
    from paper_1410_5209_amd import tf
    note("serving replay")
    g, o, ptr, oidx, vals = _serve_setup()
    nreq = len(ptr) - 1
    want = _gpu_foldin(g, 0, ptr, oidx, vals, 0)
    srv = tf.tf_serve_open(g.ctx, tf.tf_serve_default_options(streams=2))
    gaps = synth.exponential(11, 1, nreq, 2000.0)
    arrival = np.cumsum(gaps)
    keep = [(np.ascontiguousarray(oidx[ptr[q]:ptr[q + 1]]),
             np.ascontiguousarray(vals[ptr[q]:ptr[q + 1]])) for q in range(nreq)]
    reqs = [tf.make_request(oi, va) for oi, va in keep]
    tickets = tf.tf_serve_replay(srv, arrival, reqs)
    for q in range(nreq):
        row, st = tf.tf_serve_wait(srv, int(tickets[q]), g.K)
        assert np.array_equal(row, want[q]) and st.latency_us > 0
    rep = tf.tf_serve_report(srv)
    assert rep.completed == nreq and rep.solves_per_s > 0
    # close while requests are queued / running: it drains and returns
    for oi, va in keep:
        tf.tf_serve_submit(srv, tf.make_request(oi, va))
    tf.tf_serve_close(srv)
    g.close()


@pytest.mark.parametrize("method", [0, 1])
def test_foldin_bf16_factors_and_k_above_the_full_rank_limit(method):
    """BF16 factor storage (the oracle holds the same BF16 values), K = 48, plus
    CDTF fold-in at K = 160, where it walks the entries instead of a Gram."""
    from oracle import oracle as orc
    from paper_1410_5209_amd.model import SparseCP
    for prec, K in (("bf16", 48), ("f32", 160)):
        if method == 0 and K > 128:
            continue        # full rank stops at K = 128 (tested elsewhere)
        dims = [300, 200, 150]
        note(f"foldin {prec} K={K} method={method}")
        idx, x, A = problem(36, dims, 20000, K, first_zero=False)
        g = SparseCP(dims, idx, x, K, 0.5, precision=prec)
        g.set_factors(A)
        o = orc.Oracle(dims, idx, x, K, 0.5)
        for n in range(3):
            o.set_factor(n, g.factor(n))     # the values the GPU holds
        sizes = [1, 7, 64, 900, 3000]
        ptr, oidx, vals = _requests(dims, 1, sizes, 8)
        rows = _gpu_foldin(g, 1, ptr, oidx, vals, method)
        for q in range(len(sizes)):
            sl = slice(ptr[q], ptr[q + 1])
            want = o.foldin_full(1, oidx[sl], vals[sl]) if method == 0 else \
                o.foldin_cdtf(1, oidx[sl], vals[sl], 3)
            assert rel_max(rows[q], want) < 1e-4, (prec, K, q)
        g.close()


def test_serving_through_torch_allocator_and_context_budget():
    """Serving slots come from the context's allocator: with torch's caching
    allocator as the hook the served rows equal tf_foldin's, and a context
    memory budget too small for the slots makes tf_serve_open fail with
    TF_E_NOMEM and leaves the context usable."""
    import torch
    from paper_1410_5209_amd import tf
    from paper_1410_5209_amd.model import SparseCP
    note("serving through the torch allocator")
    dims, K = [3000, 2000, 1500], 24
    idx, x, A = problem(37, dims, 60000, K, first_zero=False)
    sizes = list(synth.zipf_ints(11, 500, 40, 1.1, 2000))
    ptr, oidx, vals = _requests(dims, 0, sizes, 12)
    g = SparseCP(dims, idx, x, K, 1.0, torch_alloc=True)
    g.set_factors(A)
    want = _gpu_foldin(g, 0, ptr, oidx, vals, 0)
    before = torch.cuda.memory_allocated()
    srv = tf.tf_serve_open(g.ctx, tf.tf_serve_default_options(streams=2, mem_budget=64 << 20))
    assert torch.cuda.memory_allocated() >= before + (64 << 20)   # slots in torch's pool
    keep, tickets = [], []
    for q in range(len(sizes)):
        sl = slice(ptr[q], ptr[q + 1])
        oi, va = np.ascontiguousarray(oidx[sl]), np.ascontiguousarray(vals[sl])
        keep.append((oi, va))
        tickets.append(tf.tf_serve_submit(srv, tf.make_request(oi, va)))
    for q, t in enumerate(tickets):
        row, _ = tf.tf_serve_wait(srv, t, K)
        assert np.array_equal(row, want[q])
    tf.tf_serve_close(srv)
    assert torch.cuda.memory_allocated() <= before
    g.close()

    g = SparseCP(dims, idx, x, K, 1.0, mem_budget=48 << 20)
    g.set_factors(A)
    with pytest.raises(tf.TFError) as e:
        tf.tf_serve_open(g.ctx, tf.tf_serve_default_options(streams=2, mem_budget=64 << 20))
    assert e.value.status == tf.TF_E_NOMEM
    got = _gpu_foldin(g, 0, ptr, oidx, vals, 0)
    assert np.array_equal(got, want)
    g.close()
