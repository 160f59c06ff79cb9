"""The tf_options the boundary carries beyond the method's inputs: the random
column order (Algorithm 1 draws each split's columns without replacement), the
self-tuning strategy, the device-memory hooks and the memory budget.  GPU runs
against the FP64 oracle through the C ABI."""
import numpy as np
import pytest

from gpu_util import note, pair, problem, rel_max
from oracle import oracle as orc

pytestmark = pytest.mark.gpu


def test_random_column_order_matches_the_oracle_rule_f64():
    from paper_1410_5209_amd import tf
    dims, K, C, seed = [50, 40, 30], 12, 5, 77
    note("random column order f64")
    idx, x, A = problem(310, dims, 4000, K)
    g, o = pair(dims, idx, x, A, K, 0.3, "f64", col_order=tf.TF_ORDER_RANDOM, seed=seed)
    for t in range(3):
        g.sweep(C, 1)
        order = orc.column_order(seed, t, K)
        assert np.array_equal(g.col_order(), order), t
        o.sweep(C, 1, order=order)
        for n in range(3):
            assert rel_max(g.factor(n), o.get_factor(n)) < 1e-10, (t, n)
    gl, _ = g.loss()
    ol, _ = o.loss()
    assert abs(gl - ol) <= 1e-9 * ol
    g.close()


@pytest.mark.parametrize("precision,C", [("f64", 4), ("f32", 32)])
def test_self_tuning_strategy_matches_the_oracle(precision, C):
    from paper_1410_5209_amd import tf
    dims, K = [400, 300, 200], 40 if C == 32 else 8
    note(f"strategy auto {precision} C={C}")
    idx, x, A = problem(311, dims, 30000, K, dist="zipf", dedupe="drop")
    g, o = pair(dims, idx, x, A, K, 0.5, precision, strategy=tf.TF_STRATEGY_AUTO)
    g.sweep(C, 1)
    o.sweep(C, 1)
    tol = 1e-10 if precision == "f64" else 1e-3
    for n in range(3):
        assert rel_max(g.factor(n), o.get_factor(n)) < tol, n
    g.split(list(range(3)), 2)      # a narrower split (tuned again when its compute width differs)
    o.split(list(range(3)), 2)
    for n in range(3):
        assert rel_max(g.factor(n), o.get_factor(n)) < tol, n
    g.close()


def test_torch_allocator_hooks_give_identical_results_and_free_everything():
    import torch
    from paper_1410_5209_amd import tf
    from test_gpu_foldin import _gpu_foldin, _requests
    dims, K = [300, 200, 100], 16
    note("device memory hooks")
    idx, x, A = problem(312, dims, 20000, K)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    runs = []
    for hooks in (False, True):
        g, _ = pair(dims, idx, x, A, K, 0.4, "f32", torch_alloc=hooks)
        if hooks:
            assert torch.cuda.memory_allocated() > base + 20000 * 4   # the model lives in torch's pool
        g.sweep(8, 2)
        ptr, oidx, vals = _requests(dims, 0, [1, 30, 700], 9)
        rows = _gpu_foldin(g, 0, ptr, oidx, vals, tf.TF_FOLDIN_FULL)
        runs.append((g.factors(), g.residual(), rows))
        g.close()
        torch.cuda.synchronize()
    for a, b in zip(runs[0][0], runs[1][0]):
        assert np.array_equal(a, b)
    assert np.array_equal(runs[0][1], runs[1][1]) and np.array_equal(runs[0][2], runs[1][2])
    assert torch.cuda.memory_allocated() <= base + 4096   # tensors of this test aside


def test_memory_budget_refuses_what_does_not_fit():
    from paper_1410_5209_amd import tf
    from paper_1410_5209_amd.model import SparseCP
    dims, K = [300, 200, 100], 16
    note("memory budget")
    idx, x, _ = problem(313, dims, 20000, K)
    with pytest.raises(tf.TFError) as e:
        SparseCP(dims, idx, x, K, 0.4, mem_budget=1 << 20)
    assert e.value.status == tf.TF_E_NOMEM
    g = SparseCP(dims, idx, x, K, 0.4, mem_budget=64 << 20)
    g.sweep(8, 1)
    g.close()


@pytest.mark.parametrize("C", [10, 32])
def test_persistent_launch_gives_the_skew_results_bit_for_bit(C):
    """TF_STRATEGY_PERSISTENT runs the same plan with workgroups that take
    tasks from a counter: every task is the same work in the same order, so
    factors and residual equal the grid launch's bit for bit."""
    from paper_1410_5209_amd import tf
    dims, K = [900, 700, 500], 40
    note(f"persistent launch C={C}")
    idx, x, A = problem(370 + C, dims, 60000, K, dist="zipf", dedupe="drop")
    runs = []
    for strat in (tf.TF_STRATEGY_SKEW, tf.TF_STRATEGY_PERSISTENT):
        g, _ = pair(dims, idx, x, A, K, 0.5, "f32", strategy=strat, split_threshold=512,
                    chunk_nnz=128)
        g.sweep(C, 2)
        runs.append((g.factors(), g.residual()))
        g.close()
    for a, b in zip(runs[0][0], runs[1][0]):
        assert np.array_equal(a, b)
    assert np.array_equal(runs[0][1], runs[1][1])


GRAPH_CASES = {
    # precision, dims, nnz, K, C per sweep, T_in, options
    "f64-cdtf": ("f64", [300, 200, 100], 20000, 10, [1] * 5, 1, {}),
    "f32-random-order": ("f32", [400, 300, 200], 30000, 20,
                         [4, 4, 4, 4, 3, 3, 3, 3, 4, 4, 4], 2, {"col_order": 1}),
    "f32-wide-persistent": ("f32", [300, 250, 200, 150], 30000, 40, [32] * 5, 1,
                            {"strategy": 3}),
    "bf16-shared": ("bf16", [400, 300, 200], 30000, 40, [16] * 5, 2, {"resid_share": 2}),
}


@pytest.mark.parametrize("case", sorted(GRAPH_CASES))
def test_sweep_graph_replays_equal_eager_sweeps_bit_for_bit(case):
    """tf_options.graph: a sweep whose starting state repeats the previous
    sweep's is captured as one HIP graph, and later sweeps with that state
    replay it.  After every sweep (loss, factors and residual read eagerly
    between the replays), factors, residual and loss equal those of a
    context that launches every kernel, bit for bit, also when C changes (a
    new capture) and changes back, with a random column order per sweep."""
    prec, dims, nnz, K, Cs, T_in, opts = GRAPH_CASES[case]
    note(f"sweep graph {case}")
    idx, x, A = problem(390 + len(dims) + K, dims, nnz, K, dist="zipf", dedupe="drop")
    ge, _ = pair(dims, idx, x, A, K, 0.5, prec, split_threshold=512, chunk_nnz=128, **opts)
    gg, _ = pair(dims, idx, x, A, K, 0.5, prec, split_threshold=512, chunk_nnz=128, graph=True,
                 **opts)
    for s, C in enumerate(Cs):
        ge.sweep(C, T_in)
        gg.sweep(C, T_in)
        for n in range(len(dims)):
            assert np.array_equal(ge.factor(n), gg.factor(n)), (s, n)
        assert np.array_equal(ge.residual(), gg.residual()), s
        assert ge.loss() == gg.loss(), s
    # the graph path was taken (captured, then replayed) for the repeated states
    assert gg.profile_read().graph_sweeps >= 2
    assert ge.profile_read().graph_sweeps == 0
    ge.close()
    gg.close()
