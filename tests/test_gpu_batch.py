"""GPU parity of the batched forms: all products in one launch per class,
one readback for the whole count pass, and the reusable numeric plan (bins
once, HIP graph replay, autotuned lanes per row). Every product must equal
the oracle bit for bit; graph replays are checked one by one with eager
work and synchronisations between them."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu
mls = pytest.importorskip("paper_1804_00695_amd")


def mixed_batch():
    prods = []
    for n in (4, 5, 7, 9, 12):
        A, P, R = synth.amg_instance(n)
        prods.append((A, P))
        prods.append((R, synth.amg_instance(n)[0]))            # R * A, rectangular
    prods.append((synth.poisson_csr(700, 500, 6.0, 1), synth.poisson_csr(500, 900, 9.0, 2)))
    prods.append((synth.Csr(30, 20, np.zeros(31, np.int32), np.zeros(0, np.int32), np.zeros(0)),
                  synth.poisson_csr(20, 25, 3.0, 3)))          # empty product
    prods.append((synth.stencil27_3d(7, amp=0.1), synth.stencil27_3d(7, amp=0.1, seed=9)))
    return prods


def to_dev(prods):
    return [mls.DeviceCsr.from_host(a) for a, _ in prods], [mls.DeviceCsr.from_host(b) for _, b in prods]


def check_all(prods, Cs):
    torch.cuda.synchronize()
    for (A, B), C in zip(prods, Cs):
        R, _ = oracle.spgemm(A, B)
        rp, ci, v = C.numpy()
        assert np.array_equal(rp, R.row_ptr) and np.array_equal(ci[:R.nnz], R.col_idx)
        assert np.array_equal(v[:R.nnz], R.values)


def test_batch_symbolic_numeric():
    prods = mixed_batch()
    As, Bs = to_dev(prods)
    Cs = mls.batch_symbolic(As, Bs)
    mls.batch_numeric(As, Bs, Cs)
    check_all(prods, Cs)


@pytest.mark.parametrize("use_graph,group", [(True, 0), (False, 0), (True, 16)])
def many_products(count, seed):
    """Small products of varied shape (some empty), so that waves straddle
    product boundaries and the product lookup searches more than 64 products."""
    g = np.random.default_rng(seed)
    prods = []
    for t in range(count):
        m, k, n = (int(x) for x in g.integers(1, 60, 3))
        if t % 17 == 5:
            A = synth.Csr(m, k, np.zeros(m + 1, np.int32), np.zeros(0, np.int32), np.zeros(0))
        else:
            A = synth.poisson_csr(m, k, float(g.uniform(0.5, 6.0)), 1000 + 2 * t)
        prods.append((A, synth.poisson_csr(k, n, float(g.uniform(0.5, 8.0)), 1001 + 2 * t)))
    return prods


@pytest.mark.parametrize("count", [65, 300])
def test_batch_many_products(count):
    prods = many_products(count, count)
    As, Bs = to_dev(prods)
    Cs = mls.batch_symbolic(As, Bs)
    mls.batch_numeric(As, Bs, Cs)
    check_all(prods, Cs)
    plan = mls.BatchPlan(As, Bs, Cs, group_size=8, use_graph=False)
    for C in Cs:
        C.values.fill_(float("nan"))
    plan.run()
    check_all(prods, Cs)


@pytest.mark.parametrize("use_graph,group", [(True, 0), (False, 0), (True, 16)])
def test_batch_plan_replays(use_graph, group):
    prods = mixed_batch()
    As, Bs = to_dev(prods)
    Cs = mls.batch_symbolic(As, Bs)
    plan = mls.BatchPlan(As, Bs, Cs, group_size=group, use_graph=use_graph)
    assert plan.group_size in (8, 16, 32, 64)
    for rep in range(3):
        for C in Cs:
            C.values.fill_(float("nan"))          # eager work between replays
        torch.cuda.synchronize()
        plan.run()
        check_all(prods, Cs)
    # new values on the same structure: the replay reads them in place
    for (A, B), dA in zip(prods, As):
        dA.values.mul_(2.0)
    plan.run()
    torch.cuda.synchronize()
    for (A, B), C in zip(prods, Cs):
        A2 = synth.Csr(A.nrows, A.ncols, A.row_ptr, A.col_idx, None if A.values is None else A.values * 2.0)
        R, _ = oracle.spgemm(A2, B)
        assert np.array_equal(C.values.cpu().numpy()[:R.nnz], R.values)


def test_galerkin_two_stages_symmetric():
    n = 9
    A, P, R = synth.amg_instance(n)
    dA, dP, dR = (mls.DeviceCsr.from_host(x) for x in (A, P, R))
    [AP] = mls.batch_symbolic([dA], [dP])
    mls.batch_numeric([dA], [dP], [AP])
    [Ac] = mls.batch_symbolic([dR], [AP])
    mls.batch_numeric([dR], [AP], [Ac])
    torch.cuda.synchronize()
    rp, ci, v = Ac.numpy()
    M = synth.to_dense(synth.Csr(Ac.nrows, Ac.ncols, rp, ci, v))
    # Ac = P^T A P is symmetric; entries are sums of a few products of values in {-1, 6} x {1/9..}
    assert np.allclose(M, M.T, rtol=0, atol=1e-12 * np.abs(M).max())
    APo, _ = oracle.spgemm(A, P)
    Aco, _ = oracle.spgemm(R, APo)
    assert np.array_equal(v, Aco.values)


def test_batch_with_spill_rows():
    # a batch whose products include rows of C past the LDS classes (a power-
    # law square and wide rows): the batched symbolic bitmaps and the batched
    # numeric windows, next to small multigrid products; also as a graph plan
    G = synth.rmat_graph(12, 8, seed=5)
    Rm = synth.Csr(G.nrows, G.ncols, G.row_ptr, G.col_idx, synth.normal_values(len(G.col_idx), 8))
    g = synth.rng(21)
    rows = [np.sort(g.choice(6000, 1500, replace=False)) for _ in range(6)]
    rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
    W = synth.Csr(6, 6000, rp, np.concatenate(rows).astype(np.int32), g.standard_normal(int(rp[-1])))
    prods = [synth.amg_instance(5)[:2], (Rm, Rm), (W, synth.poisson_csr(6000, 20000, 8.0, 22)),
             synth.amg_instance(6)[:2]]
    As, Bs = to_dev(prods)
    Cs = mls.batch_symbolic(As, Bs)
    mls.batch_numeric(As, Bs, Cs)
    check_all(prods, Cs)
    plan = mls.BatchPlan(As, Bs, Cs, use_graph=True)
    for rep in range(2):
        for C in Cs:
            C.values.fill_(float("nan"))
        torch.cuda.synchronize()
        plan.run()
        check_all(prods, Cs)


def test_tuned_schedule_persisted_and_reused(tmp_path):
    """The autotuner writes its choice to the cache file; a plan for another
    batch shape whose line is already in the file takes that schedule without
    searching (the crafted schedule moves the smallest class's rows up and
    uses 64 lanes in both classes), and its results stay bit-exact."""
    cache = tmp_path / "tune.txt"
    prods = mixed_batch()
    As, Bs = to_dev(prods)
    Cs = mls.batch_symbolic(As, Bs)
    plan = mls.BatchPlan(As, Bs, Cs, use_graph=True, tune_cache=cache)
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and lines[0].startswith("batch ")
    f = lines[0].split()
    g1, g2, fl = plan.schedule
    assert (int(f[7]), int(f[8]), int(f[9])) == (g1, g2, fl)
    plan.run()
    check_all(prods, Cs)
    # a second shape: its line is written by hand with the first line's device
    prods2 = prods[:-2]
    As2, Bs2 = to_dev(prods2)
    Cs2 = mls.batch_symbolic(As2, Bs2)
    na = sum(a.nrows for a, _ in prods2)
    nb = sum(b.nrows for _, b in prods2)
    za = sum(a.nnz for a, _ in prods2)
    zc = sum(c.nnz for c in Cs2)
    with open(cache, "a") as fh:
        fh.write("not a schedule line\n")
        fh.write(f"batch {len(prods2)} {na} {nb} {za} {zc} {f[6]} 64 64 1\n")
    plan2 = mls.BatchPlan(As2, Bs2, Cs2, use_graph=True, tune_cache=cache)
    assert plan2.schedule == (64, 64, 1)
    assert len(cache.read_text().splitlines()) == 3      # nothing appended: no search
    for C in Cs2:
        C.values.fill_(float("nan"))
    plan2.run()
    check_all(prods2, Cs2)
