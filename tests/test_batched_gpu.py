"""Batched persistent launches (one-shot and hipGraph handle) on the GPU."""
import numpy as np
import pytest

import oracle
import synth
import paper_1908_09606_amd as cm
from gpu_util import device_matrix, log

pytestmark = pytest.mark.gpu

DIMS = [(1, 1, 1), (64, 64, 64), (65, 130, 33), (300, 17, 250), (17, 300, 1000),
        (128, 128, 128), (257, 255, 129), (3, 500, 70), (500, 3, 70), (1000, 900, 600),
        (0, 5, 5), (5, 0, 5), (40, 50, 0), (33, 44, 55)]


def make_batch(dims, dtype_dist, seed0, int_range=0):
    import torch
    mats = []
    for i, (m, n, k) in enumerate(dims):
        s = seed0 + i
        _, A = device_matrix(m, k, s, synth.STREAM_A, dtype_dist, int_range, ld=k + (i % 3))
        _, B = device_matrix(k, n, s, synth.STREAM_B, dtype_dist, int_range, ld=n + (i % 2))
        _, C = device_matrix(m, n, s, synth.STREAM_C, dtype_dist, int_range, ld=n + 1)
        mats.append((A, B, C))
    return mats


def args_of(dims, mats, alpha, beta):
    ms = [d[0] for d in dims]; ns = [d[1] for d in dims]; ks = [d[2] for d in dims]
    lda = [max(1, A.stride(0)) if A.dim() == 2 else 1 for A, _, _ in mats]
    ldb = [max(1, B.stride(0)) for _, B, _ in mats]
    ldc = [max(1, C.stride(0)) for _, _, C in mats]
    lda = [max(l, max(1, d[2])) for l, d in zip(lda, dims)]
    ldb = [max(l, max(1, d[1])) for l, d in zip(ldb, dims)]
    ldc = [max(l, max(1, d[1])) for l, d in zip(ldc, dims)]
    return (len(dims), ms, ns, ks, alpha, [A for A, _, _ in mats], lda, [B for _, B, _ in mats], ldb,
            beta, [C for _, _, C in mats], ldc)


@pytest.mark.parametrize("dtype,dist,rng_int", [(cm.COSMA_F32, synth.INT_F32, 8),
                                                (cm.COSMA_F64, synth.INT_F64, 8)])
def test_oneshot_integer_exact(gpu, dtype, dist, rng_int):
    import torch
    mats = make_batch(DIMS, dist, 100, rng_int)
    a = args_of(DIMS, mats, [1.0] * len(DIMS), [0.0] * len(DIMS))
    assert cm.gemm_batched(*a, dtype) == 0
    torch.cuda.synchronize()
    for i, (m, n, k) in enumerate(DIMS):
        if m == 0 or n == 0:
            continue
        C = mats[i][2].cpu().numpy().astype(np.float64)
        Ah = synth.gen(m, k, 100 + i, synth.STREAM_A, dist, rng_int).astype(np.int64)
        Bh = synth.gen(k, n, 100 + i, synth.STREAM_B, dist, rng_int).astype(np.int64)
        assert np.array_equal(C, (Ah @ Bh).astype(np.float64)), (i, m, n, k)


@pytest.mark.parametrize("dtype,dist", [(cm.COSMA_F32, synth.UNIFORM_F32),
                                        (cm.COSMA_F64, synth.UNIFORM_F64)])
def test_graph_handle_bit_equal_to_single_launches(gpu, dtype, dist):
    """Every problem of a batch equals, bit for bit, the single-launch result
    under the tile and split the batch's policy gave it; replays after the
    inputs change (with eager work between) are checked one by one."""
    import torch
    dims = [d for d in DIMS if d[2] > 0]
    mats = make_batch(dims, dist, 200)
    a = args_of(dims, mats, [1.0] * len(dims), [0.0] * len(dims))
    rc, h = cm.cosma_batch_create(*a, dtype)
    assert rc == 0 and h
    try:
        rc, policy, groups, items, ms = cm.cosma_batch_info(h)
        log(f"batch policy {policy} groups {groups} items {items} tuned ms {ms}")
        # the refinement starts from the fastest policy and keeps only gains
        rc, trials, seed_ms, tuned_ms = cm.cosma_batch_tuning(h)
        log(f"  refinement: {trials} trials, {seed_ms:.4f} -> {tuned_ms:.4f} ms")
        assert rc == 0 and trials >= 0
        assert seed_ms == min(ms) and ms[policy] == seed_ms and 0.0 < tuned_ms <= seed_ms
        rc, tiles = cm.cosma_batch_tiles(h, len(dims))
        assert rc == 0 and all(t >= 0 for t, d in zip(tiles, dims) if d[0] and d[1] and d[2])
        rc, splits = cm.cosma_batch_splits(h, len(dims))
        assert rc == 0 and all(s >= 1 for s, d in zip(splits, dims) if d[0] and d[1] and d[2])
        for rep in range(3):
            for i, (m, n, k) in enumerate(dims):  # new inputs each replay
                if m and k:
                    synth.fill_device(mats[i][0][:m, :k], 300 + rep * 50 + i, synth.STREAM_A, dist)
            torch.cuda.synchronize()
            assert cm.cosma_batch_run(h) == 0
            torch.cuda.synchronize()
            for i, (m, n, k) in enumerate(dims):
                if m == 0 or n == 0:
                    continue
                A, B, C = mats[i]
                ref = torch.empty((m, n), dtype=C.dtype, device=C.device)
                t = tiles[i]
                rc, plan = cm.cosma_plan_make(m, n, k, dtype, t, splits[i])
                cm.ensure_workspace(plan.workspace_bytes)
                assert rc == 0
                assert cm.cosma_gemm_planned(plan, 1.0, A, a[6][i], B, a[8][i], 0.0, ref,
                                             max(1, n)) == 0
                torch.cuda.synchronize()
                assert torch.equal(C[:m, :n], ref[:m, :n]), (rep, i, m, n, k, t)
    finally:
        assert cm.cosma_batch_destroy(h) == 0


def test_f32_batch_uses_tiles_with_a_batched_form(gpu):
    """The 256 x 256 FP32 tile (menu index 3) has no persistent batched form:
    the batch cost model never gives it a problem, large ones included."""
    import torch
    dims = [(2048, 2048, 512), (1024, 4096, 256), (300, 200, 100)]
    mats = make_batch(dims, synth.UNIFORM_F32, 400)
    a = args_of(dims, mats, [1.0] * len(dims), [0.0] * len(dims))
    rc, h = cm.cosma_batch_create(*a, cm.COSMA_F32)
    assert rc == 0 and h
    try:
        rc, tiles = cm.cosma_batch_tiles(h, len(dims))
        log(f"f32 batch tiles {tiles}")
        assert rc == 0 and all(0 <= t <= 2 for t in tiles)
        assert cm.cosma_batch_run(h) == 0
        torch.cuda.synchronize()
    finally:
        assert cm.cosma_batch_destroy(h) == 0


def test_graph_handle_beta_nonzero_against_oracle(gpu):
    import torch
    dims = [(130, 70, 300), (64, 200, 129), (5, 5, 5), (40, 50, 0)]
    mats = make_batch(dims, synth.UNIFORM_F64, 400)
    C0 = [mats[i][2].cpu().numpy().copy() for i in range(len(dims))]
    alpha = [0.5, -1.0, 2.0, 1.0]
    beta = [1.5, 0.25, -1.0, 3.0]
    a = args_of(dims, mats, alpha, beta)
    rc, h = cm.cosma_batch_create(*a, cm.COSMA_F64)
    assert rc == 0
    rc, policy, groups, items, ms = cm.cosma_batch_info(h)
    assert policy == cm.BATCH_POLICY_DEFAULT and ms == [0.0] * cm.BATCH_POLICIES  # no tuning when some beta != 0
    assert cm.cosma_batch_run(h) == 0
    torch.cuda.synchronize()
    for i, (m, n, k) in enumerate(dims):
        Ah = synth.gen(m, k, 400 + i, synth.STREAM_A, synth.UNIFORM_F64)
        Bh = synth.gen(k, n, 400 + i, synth.STREAM_B, synth.UNIFORM_F64)
        ref, D = oracle.gemm(Ah, Bh, alpha[i], beta[i], C0[i][:m, :n])
        err = oracle.normalised_err(mats[i][2][:m, :n].cpu().numpy(), ref, D)
        assert err <= oracle.fp64_bound(k), (i, err)
    assert cm.cosma_batch_destroy(h) == 0


def test_invalid_batches(gpu):
    dims = [(10, 10, 10)]
    mats = make_batch(dims, synth.UNIFORM_F32, 1)
    a = list(args_of(dims, mats, [1.0], [0.0]))
    a[6] = [5]  # lda < k
    assert cm.cosma_gemm_batched(*a, cm.COSMA_F32) == cm.COSMA_ERR_INVALID_ARG
    rc, h = cm.cosma_batch_create(*a, cm.COSMA_F32)
    assert rc == cm.COSMA_ERR_INVALID_ARG and not h
    a = list(args_of(dims, mats, [1.0], [0.0]))
    assert cm.cosma_gemm_batched(*a, cm.COSMA_F32_BF16X3) == cm.COSMA_ERR_UNSUPPORTED
    assert cm.cosma_batch_run(None) == cm.COSMA_ERR_INVALID_ARG
    # a workspace smaller than the batch needs: nothing is launched
    rc, need = cm.cosma_workspace_size_batched(1, [10], [10], [10], [1.0], cm.COSMA_F32)
    assert rc == 0 and need > 0
    import torch
    small = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    saved = cm._workspace.get(torch.cuda.current_device())
    try:
        assert cm.cosma_set_workspace(small, small.numel()) == 0
        assert cm.cosma_gemm_batched(*a, cm.COSMA_F32) == cm.COSMA_ERR_WORKSPACE
    finally:
        if saved is not None:
            assert cm.cosma_set_workspace(saved, saved.numel()) == 0
        else:
            assert cm.cosma_set_workspace(None, 0) == 0


def test_config_512_problems_sampled(gpu):
    """512 FP32 problems, dims log-uniform in [64, 4096], seeded per problem:
    graph handle; two sampled rows x two sampled columns per problem against
    the oracle."""
    import torch
    dims = [tuple(int(x) for x in d) for d in synth.batch_dims(512, seed=5)]
    log(f"512 problems, sum 2mnk = {sum(2.0 * m * n * k for m, n, k in dims):.3e}")
    mats = []
    for i, (m, n, k) in enumerate(dims):
        A = torch.empty((m, k), dtype=torch.float32, device="cuda")
        B = torch.empty((k, n), dtype=torch.float32, device="cuda")
        C = torch.empty((m, n), dtype=torch.float32, device="cuda")
        synth.fill_device(A, 1000 + i, synth.STREAM_A, synth.UNIFORM_F32)
        synth.fill_device(B, 1000 + i, synth.STREAM_B, synth.UNIFORM_F32)
        mats.append((A, B, C))
    a = (512, [d[0] for d in dims], [d[1] for d in dims], [d[2] for d in dims], [1.0] * 512,
         [x[0] for x in mats], [d[2] for d in dims], [x[1] for x in mats], [d[1] for d in dims],
         [0.0] * 512, [x[2] for x in mats], [d[1] for d in dims])
    rc, h = cm.cosma_batch_create(*a, cm.COSMA_F32)
    assert rc == 0
    rc, policy, groups, items, ms = cm.cosma_batch_info(h)
    log(f"  policy {policy} groups {groups} items {items} candidate ms {ms}")
    for C in (x[2] for x in mats):
        C.fill_(float("nan"))
    assert cm.cosma_batch_run(h) == 0
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    worst = 0.0
    for i, (m, n, k) in enumerate(dims):
        rows = np.unique(np.concatenate([[m - 1], rng.integers(0, m, 1)]))
        cols = np.unique(np.concatenate([[n - 1], rng.integers(0, n, 1)]))
        Ar = synth.gen(m, k, 1000 + i, synth.STREAM_A, synth.UNIFORM_F32, row_idx=rows)
        Bc = synth.gen(k, n, 1000 + i, synth.STREAM_B, synth.UNIFORM_F32, col_idx=cols)
        ref, D = oracle.gemm(Ar, Bc)
        got = mats[i][2].cpu().numpy()[np.ix_(rows, cols)]
        err = oracle.normalised_err(got, ref, D)
        worst = max(worst, err / oracle.fp32_bound(k))
        assert err <= oracle.fp32_bound(k), (i, m, n, k, err)
    log(f"  worst err / bound = {worst:.3e}")
    assert cm.cosma_batch_destroy(h) == 0


# Few tiles and long k next to many small problems: the batch model cuts k
# for the long ones (section 6.2's rule inside a batch).
SPLIT_DIMS = [(128, 128, 16384), (200, 130, 12000), (64, 300, 9000)] + \
             [(96 + 7 * i, 80 + 5 * i, 64 + 3 * i) for i in range(40)]


def model_plan(dims, mats, dtype):
    """Tiles and splits of the planner's batch policy (what the one-shot
    call runs): a handle with one beta != 0 skips the autotuner."""
    beta = [0.0] * len(dims)
    beta[-1] = 1.0
    a = args_of(dims, mats, [1.0] * len(dims), beta)
    rc, h = cm.cosma_batch_create(*a, dtype)
    assert rc == 0
    try:
        assert cm.cosma_batch_info(h)[1] == cm.BATCH_POLICY_DEFAULT
        rc, tiles = cm.cosma_batch_tiles(h, len(dims))
        rc2, splits = cm.cosma_batch_splits(h, len(dims))
        assert rc == 0 and rc2 == 0
    finally:
        assert cm.cosma_batch_destroy(h) == 0
    return tiles, splits


@pytest.mark.parametrize("dtype,dist", [(cm.COSMA_F32, synth.UNIFORM_F32),
                                        (cm.COSMA_F64, synth.UNIFORM_F64)])
def test_oneshot_split_k_bit_equal_to_planned_launches(gpu, dtype, dist):
    """The one-shot call cuts k for the long problems; every problem equals,
    bit for bit, cosma_gemm_planned under the same tile and split, and is
    within the stated bound of the oracle."""
    import torch
    dims = SPLIT_DIMS
    mats = make_batch(dims, dist, 500)
    tiles, splits = model_plan(dims, mats, dtype)
    log(f"split batch: splits {splits[:3]} ... tiles {tiles[:3]}")
    assert max(splits[:3]) > 1 and max(splits[3:]) == 1
    alpha = [1.0 + 0.01 * i for i in range(len(dims))]
    beta = [0.0] * len(dims)
    a = args_of(dims, mats, alpha, beta)
    assert cm.gemm_batched(*a, dtype) == 0
    torch.cuda.synchronize()
    for i, (m, n, k) in enumerate(dims):
        A, B, C = mats[i]
        rc, plan = cm.cosma_plan_make(m, n, k, dtype, tiles[i], splits[i])
        assert rc == 0 and plan.p_k == splits[i]
        ref = torch.empty((m, n), dtype=C.dtype, device=C.device)
        cm.ensure_workspace(plan.workspace_bytes)
        assert cm.cosma_gemm_planned(plan, alpha[i], A, a[6][i], B, a[8][i], 0.0, ref, n) == 0
        torch.cuda.synchronize()
        assert torch.equal(C[:m, :n], ref), (i, m, n, k, tiles[i], splits[i])
        if i < 3:
            rows = np.array([0, m // 2, m - 1])
            Ar = synth.gen(m, k, 500 + i, synth.STREAM_A, dist, row_idx=rows)
            Bh = synth.gen(k, n, 500 + i, synth.STREAM_B, dist)
            r, D = oracle.gemm(Ar, Bh, alpha[i])
            err = oracle.normalised_err(C[rows].double().cpu().numpy(), r, D)
            bound = oracle.fp64_bound(k) if dtype == cm.COSMA_F64 else oracle.fp32_bound(k)
            assert err <= bound, (i, err)


@pytest.mark.parametrize("dtype,dist", [(cm.COSMA_F32, synth.UNIFORM_F32),
                                        (cm.COSMA_F64, synth.UNIFORM_F64)])
def test_oneshot_under_graph_capture(gpu, dtype, dist):
    """cosma_gemm_batched recorded into a HIP graph: every replay (inputs
    refilled and eager one-shot calls on the same workspace between
    replays) equals the eager call's result bit for bit, split problems and
    beta != 0 included."""
    import torch
    dims = SPLIT_DIMS[:3] + [(70, 90, 33), (5, 5, 5), (40, 50, 0)] + SPLIT_DIMS[3:12]
    mats = make_batch(dims, dist, 600)
    C0 = [x[2].clone() for x in mats]
    alpha = [0.5 + 0.1 * i for i in range(len(dims))]
    beta = [(-0.5 if i % 3 == 0 else 0.0) for i in range(len(dims))]
    a = args_of(dims, mats, alpha, beta)
    rc, need = cm.cosma_workspace_size_batched(len(dims), a[1], a[2], a[3], alpha, dtype)
    assert rc == 0 and need > 0
    cm.ensure_workspace(need)          # before capture: nothing is allocated inside

    def reset():
        for x, c0 in zip(mats, C0):
            x[2].copy_(c0)

    def refill(rep):
        for i, (m, n, k) in enumerate(dims):
            if m and k:
                synth.fill_device(mats[i][0][:m, :k], 700 + 10 * rep + i, synth.STREAM_A, dist)

    stream = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    reset()
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=stream):
        assert cm.cosma_gemm_batched(*a, dtype, stream) == 0
    for rep in range(3):
        refill(rep)
        reset()
        torch.cuda.synchronize()
        assert cm.cosma_gemm_batched(*a, dtype) == 0     # eager, same workspace
        torch.cuda.synchronize()
        eager = [x[2].clone() for x in mats]
        reset()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for i in range(len(dims)):
            assert torch.equal(mats[i][2], eager[i]), (rep, i, dims[i])
    del graph
