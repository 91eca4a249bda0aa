"""Helpers for the GPU parity tests: seeded device inputs and sampled oracle
checks.  Inputs come from synth (host and device fill implement the same
generator); expected values come only from the oracle."""
import sys

import numpy as np

import oracle
import synth


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def device_matrix(rows, cols, seed, stream, dist, param=0, ld=None, torch_dtype=None):
    """A rows x cols device matrix (leading dimension ld) filled by synth."""
    import torch
    dt = torch.float32 if dist in (synth.UNIFORM_F32, synth.INT_F32) else torch.float64
    ld = cols if ld is None else ld
    buf = torch.empty((max(rows, 1), max(ld, 1)), dtype=dt, device="cuda")
    view = buf[:rows, :cols]
    if rows and cols:
        synth.fill_device(view, seed, stream, dist, param)
    return buf, view


def sample_indices(total, count, rng, tile=128):
    """Indices for sampled verification: random ones plus the first and last
    rows/columns of the first and last tiles (edge tiles)."""
    edge = set(range(min(total, 4))) | set(range(max(0, total - 4), total))
    last_tile = (total - 1) // tile * tile
    edge |= {last_tile, min(total - 1, last_tile + 1)}
    rnd = rng.choice(total, size=min(total, count), replace=False) if total else []
    return np.array(sorted(edge | set(int(x) for x in rnd)), dtype=np.int64)


def sampled_check(C_dev_view, m, n, k, seed, dist, alpha=1.0, beta=0.0, C0_host=None,
                  rows=None, cols=None, bound=None):
    """Compare sampled entries of the device result with the oracle computed
    from regenerated rows of A and columns of B.  Returns the normalised error."""
    import torch
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    Ar = synth.gen(m, k, seed, synth.STREAM_A, dist, row_idx=rows)
    Bc = synth.gen(k, n, seed, synth.STREAM_B, dist, col_idx=cols)
    c0 = None if C0_host is None else C0_host[np.ix_(rows, cols)]
    ref, D = oracle.gemm(Ar, Bc, alpha, beta, c0)
    ri = torch.as_tensor(rows, device=C_dev_view.device)
    ci = torch.as_tensor(cols, device=C_dev_view.device)
    got = C_dev_view.index_select(0, ri).index_select(1, ci).double().cpu().numpy()
    err = oracle.normalised_err(got, ref, D)
    if bound is not None:
        assert err <= bound, f"normalised error {err:.3e} > bound {bound:.3e}"
    return err


def run_gemm(cm, m, n, k, A, lda, B, ldb, C, ldc, alpha=1.0, beta=0.0, plan=None, dtype=0):
    """cosma_gemm / cosma_gemm_planned through the C ABI with the workspace
    the plan needs registered; synchronises and returns the status."""
    import torch
    if plan is None:
        rc, ws = cm.cosma_workspace_size(m, n, k, dtype)
        assert rc == 0
    else:
        ws = plan.workspace_bytes
    if ws:
        cm.ensure_workspace(ws)
    if plan is None:
        rc = cm.cosma_gemm(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, dtype)
    else:
        rc = cm.cosma_gemm_planned(plan, alpha, A, lda, B, ldb, beta, C, ldc)
    torch.cuda.synchronize()
    return rc


def contract_check(got, Ah, Bh, plan, alpha, beta, C0):
    """Assert the plan's contract entry by entry; returns (worst ratio to the
    absolute bound, covered fraction, worst normalised error on covered
    entries)."""
    m, k = Ah.shape
    ref, D = oracle.gemm(Ah, Bh, alpha, beta, C0)
    _, e = np.frexp(np.abs(Ah).max(axis=1))
    _, f = np.frexp(np.abs(Bh).max(axis=0))
    scale = abs(alpha) * k * np.ldexp(np.ones(ref.shape), e[:, None] + f[None, :])
    g_ref = (1.01 * k + 3) * 2.0 ** -53
    bound = plan.err_scaled * scale + (plan.err_rounding + g_ref) * D
    diff = np.abs(got - ref)
    assert np.all(np.isfinite(got))
    zero = D == 0.0  # all-zero row or column: the result must be exact
    assert np.all(diff[zero] == 0.0)
    D1 = np.where(zero, 1.0, D)
    ratio = float(np.max(np.where(zero, 0.0, diff / np.where(zero, 1.0, bound))))
    assert ratio <= 1.0, f"absolute contract broken: {ratio:.3g} of the bound"
    rho = scale / D1
    covered = zero | (rho <= plan.spread_limit)
    norm = np.where(zero, 0.0, diff / D1)
    worst = float(norm[covered].max()) if covered.any() else 0.0
    assert worst <= oracle.fp64_bound(k), (worst, oracle.fp64_bound(k))
    return ratio, float(covered.mean()), worst


def _gen_threaded(rows, cols, seed, stream, dist, row_idx=None, col_idx=None, threads=16):
    """synth.gen of a sub-block, cut into row chunks generated in parallel."""
    from concurrent.futures import ThreadPoolExecutor
    r = np.arange(rows) if row_idx is None else np.asarray(row_idx)
    chunks = [r[i:i + max(1, len(r) // threads + 1)] for i in range(0, len(r), max(1, len(r) // threads + 1))]
    with ThreadPoolExecutor(max_workers=threads) as ex:
        parts = list(ex.map(lambda rr: synth.gen(rows, cols, seed, stream, dist, row_idx=rr,
                                                 col_idx=col_idx), chunks))
    return np.concatenate(parts, axis=0) if parts else np.empty((0, 0))


def fullsize_check(C_dev, m, n, k, seed, dist, plan, bound, budget_fma=3.2e11, nsamp=256):
    """Full-size verification against the oracle:
      - 65,536 entries: nsamp x nsamp uniformly drawn rows and columns;
      - the edge tiles: every entry of the first and last tile row and tile
        column of C when that costs at most budget_fma multiply-adds on the
        host, else every entry of the four corner tiles.
    Returns (worst normalised error, number of entries checked)."""
    import torch
    rng = np.random.default_rng(m * 7 + n * 3 + k)
    tm, tn = plan.tile_m, plan.tile_n
    er = np.unique(np.concatenate([np.arange(min(tm, m)), np.arange((m - 1) // tm * tm, m)]))
    ec = np.unique(np.concatenate([np.arange(min(tn, n)), np.arange((n - 1) // tn * tn, n)]))
    rows = np.sort(rng.choice(m, size=min(m, nsamp), replace=False))
    cols = np.sort(rng.choice(n, size=min(n, nsamp), replace=False))
    worst, count = 0.0, 0

    def check(ri, ci, Ar, Bc):
        nonlocal worst, count
        ref, D = oracle.gemm(Ar, Bc)
        got = C_dev.index_select(0, torch.as_tensor(ri, device=C_dev.device)) \
                   .index_select(1, torch.as_tensor(ci, device=C_dev.device)).double().cpu().numpy()
        err = oracle.normalised_err(got, ref, D)
        assert err <= bound, f"normalised error {err:.3e} > bound {bound:.3e}"
        worst = max(worst, err)
        count += got.size

    Bs = _gen_threaded(k, n, seed, synth.STREAM_B, dist, col_idx=cols)
    check(rows, cols, _gen_threaded(m, k, seed, synth.STREAM_A, dist, row_idx=rows), Bs)
    del Bs
    full = (len(er) * n + len(ec) * m) * float(k) <= budget_fma
    if full:
        Bf = _gen_threaded(k, n, seed, synth.STREAM_B, dist)
        check(er, np.arange(n), _gen_threaded(m, k, seed, synth.STREAM_A, dist, row_idx=er), Bf)
        del Bf
        Af = _gen_threaded(m, k, seed, synth.STREAM_A, dist)
        check(np.arange(m), ec, Af, _gen_threaded(k, n, seed, synth.STREAM_B, dist, col_idx=ec))
        del Af
    else:
        check(er, ec, _gen_threaded(m, k, seed, synth.STREAM_A, dist, row_idx=er),
              _gen_threaded(k, n, seed, synth.STREAM_B, dist, col_idx=ec))
    log(f"  checked {count} entries ({'edge tile rows and columns' if full else 'corner tiles'}"
        f" + {len(rows) * len(cols)} sampled): worst {worst:.3e}, bound {bound:.3e}")
    return worst, count
