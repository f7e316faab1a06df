"""GPU parity of the batched path (C ABI ipt_solve_batched) against the FP64 oracle."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import dev, say, t
from parity import check

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ipt():
    from paper_2012_14702_amd import ipt as mod
    mod.load_library()
    dev()
    return mod


def _run(ipt, ns, th_pool, de_pool, **kw):
    r = ipt.ipt_solve_batched(ns, t(th_pool), t(de_pool), **kw)
    return r.z.cpu().numpy(), r.lam.cpu().numpy(), r.status.cpu().numpy(), r.info


def _per_problem(ns, th_off, de_off, z, lam, st, b):
    n = int(ns[b])
    return (z[de_off[b]:de_off[b] + n * n].reshape(n, n), lam[th_off[b]:th_off[b] + n], st[th_off[b]:th_off[b] + n])


@pytest.mark.parametrize("prec", ["fp64", "ladder"])
def test_batched_small_batch_parity(ipt, prec):
    """48 problems with n ~ U{32..512} (both tile sizes and ragged edges), theta sorted
    uniform, eps = 0.02: every problem matches the oracle column by column."""
    say("batched B=48 %s" % prec)
    ns, th, de, th_off, de_off = W.batched_sym_gaussian(48, 32, 512, 0.02, seed=3)
    p = ipt.PREC_LADDER if prec == "ladder" else ipt.PREC_FP64
    z, lam, st, info = _run(ipt, ns, th, de, tol=1e-10, precision=p, max_iter=64)
    ref = oracle.ipt_batched(ns, th, de, th_off, de_off, tol=1e-10, max_iter=64)
    compared = 0
    for b in range(48):
        gz, gl, gs = _per_problem(ns, th_off, de_off, z, lam, st, b)
        rz, rl, rs = _per_problem(ns, th_off, de_off, ref.z, ref.lam, ref.status, b)
        n = int(ns[b])
        thb, deb = th[th_off[b]:th_off[b] + n], de[de_off[b]:de_off[b] + n * n].reshape(n, n)
        rr = oracle.ipt_dense(thb, deb, tol=1e-10, max_iter=64)   # per-column steps for the status rule
        np.testing.assert_array_equal(rr.status, rs)
        out = check(gz, gl, gs, rr, oracle.norm1(thb, deb), 1e-10, max_iter=64)
        compared += out["compared"]
    assert compared >= 0.95 * int(ns.sum())
    assert info["converged"] == int((st == 0).sum())


def test_batched_edge_sizes(ipt):
    """Sizes 1, 2, 63, 64, 65, 127, 128, 129, 192, 193, 256 and 300 in one batch."""
    sizes = [1, 2, 63, 64, 65, 127, 128, 129, 192, 193, 256, 300]
    say("batched edge sizes")
    th_parts, de_parts = [], []
    for q, n in enumerate(sizes):
        thb, deb = W.dense_sym_gaussian(n, 0.01, 100 + q)
        th_parts.append(thb)
        de_parts.append(deb.ravel())
    ns = np.array(sizes, dtype=np.int32)
    th = np.concatenate(th_parts)
    de = np.concatenate(de_parts)
    th_off = np.concatenate([[0], np.cumsum(ns)[:-1]]).astype(np.int64)
    de_off = np.concatenate([[0], np.cumsum(ns.astype(np.int64) ** 2)[:-1]]).astype(np.int64)
    z, lam, st, info = _run(ipt, ns, th, de, tol=1e-12)
    assert np.all(st == 0)
    for b, n in enumerate(sizes):
        gz, gl, gs = _per_problem(ns, th_off, de_off, z, lam, st, b)
        thb, deb = th_parts[b], de_parts[b].reshape(n, n)
        rr = oracle.ipt_dense(thb, deb, tol=1e-12)
        check(gz, gl, gs, rr, oracle.norm1(thb, deb), 1e-12)


def test_batched_invalid(ipt):
    say("batched invalid")
    ns, th, de, th_off, de_off = W.batched_sym_gaussian(4, 32, 64, 0.02, seed=1)
    th2 = th.copy()
    th2[th_off[2] + 3] = th2[th_off[2] + 4]
    with pytest.raises(ipt.IPTError) as e:
        _run(ipt, ns, th2, de)
    assert e.value.status == ipt.IPT_EDEGENERATE
    bad = ns.copy()
    bad[1] = 5000
    with pytest.raises(ipt.IPTError) as e:
        _run(ipt, bad, th, de)
    assert e.value.status == ipt.IPT_EINVAL


def _edge_batch(sizes, seed0):
    th_parts, de_parts = [], []
    for q, n in enumerate(sizes):
        thb, deb = W.dense_sym_gaussian(n, 0.01, seed0 + q)
        th_parts.append(thb)
        de_parts.append(deb.ravel())
    ns = np.array(sizes, dtype=np.int32)
    th_off = np.concatenate([[0], np.cumsum(ns)[:-1]]).astype(np.int64)
    de_off = np.concatenate([[0], np.cumsum(ns.astype(np.int64) ** 2)[:-1]]).astype(np.int64)
    return ns, np.concatenate(th_parts), np.concatenate(de_parts), th_off, de_off


def _same(a, b):
    for x, y in zip(a[:3], b[:3]):
        np.testing.assert_array_equal(x, y)
    for key in ("sweeps", "converged", "diverged", "not_converged", "matvecs", "max_step", "max_resid",
                "sweep_prec", "sweep_active", "sweep_max_step"):
        assert a[3][key] == b[3][key], key


def test_batched_graph_replays_match_eager(ipt):
    """The captured chunk of sweeps, replayed many times per solve and reused across
    solves, gives the same bits as launching every sweep from the host; a second
    batch in between forces a new capture."""
    say("batched graph vs eager")
    ns, th, de, th_off, de_off = W.batched_sym_gaussian(40, 1, 300, 0.02, seed=5)
    kw = dict(tol=1e-10, precision=ipt.PREC_LADDER, max_iter=60)
    eager = _run(ipt, ns, th, de, flags=ipt.FLAG_NO_GRAPH, **kw)
    g1 = _run(ipt, ns, th, de, **kw)
    g2 = _run(ipt, ns, th, de, **kw)
    ns2, th2, de2, _, _ = W.batched_sym_gaussian(7, 100, 200, 0.02, seed=6)
    _run(ipt, ns2, th2, de2, **kw)
    g3 = _run(ipt, ns, th, de, **kw)
    g4 = _run(ipt, ns, th, de, sync_every=3, **kw)
    e4 = _run(ipt, ns, th, de, sync_every=3, flags=ipt.FLAG_NO_GRAPH, **kw)
    for g in (g1, g2, g3, g4, e4):
        _same(eager, g)
    assert eager[3]["sweeps"] > 4  # several chunks were replayed


@pytest.mark.parametrize("tile", [32, 64, 128])
def test_batched_tile_sizes_parity(ipt, tile):
    """Every problem forced to one tile size (ragged edges at each) matches the oracle."""
    say("batched tile %d" % tile)
    sizes = [1, 3, 31, 32, 33, 64, 65, 96, 129, 200, 257, 333]
    ns, th, de, th_off, de_off = _edge_batch(sizes, 300)
    saved = ipt.ipt_batched_get_tiles()
    try:
        ipt.ipt_batched_set_tiles([tile] * ipt.TILE_BUCKETS)
        assert ipt.ipt_batched_get_tiles() == [tile] * ipt.TILE_BUCKETS
        for prec in (ipt.PREC_LADDER, ipt.PREC_FP64):
            z, lam, st, info = _run(ipt, ns, th, de, tol=1e-11, precision=prec)
            assert np.all(st == 0)
            for b, n in enumerate(sizes):
                gz, gl, gs = _per_problem(ns, th_off, de_off, z, lam, st, b)
                thb = th[th_off[b]:th_off[b] + n]
                deb = de[de_off[b]:de_off[b] + n * n].reshape(n, n)
                rr = oracle.ipt_dense(thb, deb, tol=1e-11)
                check(gz, gl, gs, rr, oracle.norm1(thb, deb), 1e-11)
    finally:
        ipt.ipt_batched_set_tiles(saved)


def test_batched_max_iter_outputs(ipt):
    """max_iter = 3: the undecided columns are NOT_CONVERGED and return the last
    iterate F(Z) with lambda from the input Z of the last sweep, as the oracle does."""
    say("batched max_iter 3")
    sizes = [5, 40, 70, 130]
    ns, th, de, th_off, de_off = _edge_batch(sizes, 400)
    z, lam, st, info = _run(ipt, ns, th, de, tol=1e-14, max_iter=3)
    assert info["sweeps"] == 3
    for b, n in enumerate(sizes):
        gz, gl, gs = _per_problem(ns, th_off, de_off, z, lam, st, b)
        thb = th[th_off[b]:th_off[b] + n]
        deb = de[de_off[b]:de_off[b] + n * n].reshape(n, n)
        rr = oracle.ipt_dense(thb, deb, tol=1e-14, max_iter=3)
        np.testing.assert_array_equal(gs, rr.status)
        nc = rr.status == 1
        if nc.any():
            np.testing.assert_allclose(gz[:, nc], rr.z[:, nc], rtol=0, atol=1e-13)
            np.testing.assert_allclose(gl[nc], rr.lam[nc], rtol=0, atol=1e-13)


def test_batched_tune_table(ipt):
    """The autotuner returns one of 32/64/128 per bucket, installs it, and a solve
    with the tuned table matches the oracle."""
    say("batched tune")
    ns, th, de, th_off, de_off = W.batched_sym_gaussian(24, 1, 400, 0.02, seed=8)
    saved = ipt.ipt_batched_get_tiles()
    try:
        tiles = ipt.ipt_batched_tune(ns, t(th), t(de))
        assert len(tiles) == ipt.TILE_BUCKETS and set(tiles) <= {32, 64, 128}
        assert ipt.ipt_batched_get_tiles() == tiles
        z, lam, st, info = _run(ipt, ns, th, de, tol=1e-10)
        for b in range(len(ns)):
            n = int(ns[b])
            gz, gl, gs = _per_problem(ns, th_off, de_off, z, lam, st, b)
            thb = th[th_off[b]:th_off[b] + n]
            deb = de[de_off[b]:de_off[b] + n * n].reshape(n, n)
            rr = oracle.ipt_dense(thb, deb, tol=1e-10, max_iter=100)
            check(gz, gl, gs, rr, oracle.norm1(thb, deb), 1e-10, max_iter=100)
        with pytest.raises(ipt.IPTError):
            ipt.ipt_batched_set_tiles([48] * ipt.TILE_BUCKETS)
    finally:
        ipt.ipt_batched_set_tiles(saved)


def test_batched_acx_parity_and_graph(ipt):
    """IPT-ACX over a batch (sizes 1..400, three tile sizes by the default table):
    every problem matches the ACX oracle, and the captured graph replays give the
    same bits as host-launched sweeps."""
    say("batched acx")
    ns, th, de, th_off, de_off = W.batched_sym_gaussian(32, 1, 400, 0.02, seed=9)
    kw = dict(tol=1e-10, max_iter=64, flags=ipt.FLAG_ACX)
    g = _run(ipt, ns, th, de, **kw)
    e = _run(ipt, ns, th, de, tol=1e-10, max_iter=64, flags=ipt.FLAG_ACX | ipt.FLAG_NO_GRAPH)
    _same(g, e)
    z, lam, st, info = g
    for b in range(len(ns)):
        n = int(ns[b])
        gz, gl, gs = _per_problem(ns, th_off, de_off, z, lam, st, b)
        thb = th[th_off[b]:th_off[b] + n]
        deb = de[de_off[b]:de_off[b] + n * n].reshape(n, n)
        rr = oracle.ipt_dense(thb, deb, tol=1e-10, max_iter=64, accel="acx")
        check(gz, gl, gs, rr, oracle.norm1(thb, deb), 1e-10, max_iter=64)
    assert info["converged"] == int((st == 0).sum())


@pytest.mark.parametrize("tile", [32, 128])
def test_batched_acx_tiles(ipt, tile):
    """ACX with every problem on one tile size, ragged sizes."""
    say("batched acx tile %d" % tile)
    sizes = [1, 3, 33, 64, 100, 129, 250]
    ns, th, de, th_off, de_off = _edge_batch(sizes, 500)
    saved = ipt.ipt_batched_get_tiles()
    try:
        ipt.ipt_batched_set_tiles([tile] * ipt.TILE_BUCKETS)
        z, lam, st, info = _run(ipt, ns, th, de, tol=1e-11, flags=ipt.FLAG_ACX)
        for b, n in enumerate(sizes):
            gz, gl, gs = _per_problem(ns, th_off, de_off, z, lam, st, b)
            thb = th[th_off[b]:th_off[b] + n]
            deb = de[de_off[b]:de_off[b] + n * n].reshape(n, n)
            rr = oracle.ipt_dense(thb, deb, tol=1e-11, accel="acx")
            check(gz, gl, gs, rr, oracle.norm1(thb, deb), 1e-11, max_iter=100)
        assert np.all(st == 0)
    finally:
        ipt.ipt_batched_set_tiles(saved)


@pytest.mark.parametrize("flags", [0, 8])
def test_batched_nonsymmetric(ipt, flags):
    """Non-symmetric problems (the paper's diag(1..n) + eps R, R iid U[0,1], Sec. 6.2)
    next to symmetric ones in one batch: the next sweep's d uses Delta_cj, which the
    solve reads as Delta_jc only for exactly symmetric problems."""
    say("batched nonsym flags=%d" % flags)
    sizes = [5, 70, 130, 200, 64]
    th_parts, de_parts = [], []
    for q, n in enumerate(sizes):
        thb, deb = (W.dense_uniform_nonsym(n, 1e-3, 700 + q) if q % 2 == 0 else W.dense_sym_gaussian(n, 0.01, 700 + q))
        th_parts.append(thb)
        de_parts.append(deb.ravel())
    ns = np.array(sizes, dtype=np.int32)
    th, de = np.concatenate(th_parts), np.concatenate(de_parts)
    th_off = np.concatenate([[0], np.cumsum(ns)[:-1]]).astype(np.int64)
    de_off = np.concatenate([[0], np.cumsum(ns.astype(np.int64) ** 2)[:-1]]).astype(np.int64)
    z, lam, st, info = _run(ipt, ns, th, de, tol=1e-11, flags=flags)
    for b, n in enumerate(sizes):
        gz, gl, gs = _per_problem(ns, th_off, de_off, z, lam, st, b)
        thb, deb = th_parts[b], de_parts[b].reshape(n, n)
        rr = oracle.ipt_dense(thb, deb, tol=1e-11, accel="acx" if flags else "picard")
        check(gz, gl, gs, rr, oracle.norm1(thb, deb), 1e-11, max_iter=100)
    assert np.all(st == 0)


def _planted_pairs(n, pairs, seed, strength=1.5):
    """theta = 1..n, a small symmetric background, and pairs (i, j) moved to a gap of
    0.02 with coupling strength * gap (beyond the 2x2 convergence bound for 1.5)."""
    rng = np.random.default_rng(seed)
    th = np.arange(1.0, n + 1.0)
    r = rng.standard_normal((n, n)) * 0.01 / np.sqrt(n)
    de = (r + r.T) / 2.0
    for i, j in pairs:
        th[j] = th[i] + 0.02
        de[i, j] = de[j, i] = strength * 0.02
    return th, de


@pytest.mark.parametrize("prec", ["fp64", "ladder"])
def test_batched_pair_rotation_parity(ipt, prec):
    """IPT_FLAG_CHOOSE_D: 20 problems of the batched workload plus three with pairs
    planted beyond the 2x2 bound (one at a 64-row tile edge, one at the end of a ragged
    size), every problem against the oracle's rotated solve column by column (the same
    pairing, rotation and chart); the planted problems converge on every column, which
    the plain solve does not."""
    say("batched pair rotation %s" % prec)
    ns0, th0, de0, _, _ = W.batched_sym_gaussian(20, 32, 384, 0.02, seed=5)
    parts_th, parts_de = [], []
    o0 = np.concatenate([[0], np.cumsum(ns0)[:-1]])
    p0 = np.concatenate([[0], np.cumsum(ns0.astype(np.int64) ** 2)[:-1]])
    for b in range(20):
        n = int(ns0[b])
        parts_th.append(th0[o0[b]:o0[b] + n])
        parts_de.append(de0[p0[b]:p0[b] + n * n])
    planted = [(96, [(10, 11), (63, 64)]), (131, [(5, 6), (129, 130)]), (40, [(0, 1), (20, 21), (38, 39)])]
    for q, (n, pairs) in enumerate(planted):
        thb, deb = _planted_pairs(n, pairs, 50 + q)
        parts_th.append(thb)
        parts_de.append(deb.ravel())
    ns = np.array([len(x) for x in parts_th], dtype=np.int32)
    th = np.concatenate(parts_th)
    de = np.concatenate(parts_de)
    th_off = np.concatenate([[0], np.cumsum(ns)[:-1]]).astype(np.int64)
    de_off = np.concatenate([[0], np.cumsum(ns.astype(np.int64) ** 2)[:-1]]).astype(np.int64)
    p = ipt.PREC_LADDER if prec == "ladder" else ipt.PREC_FP64
    z, lam, st, info = _run(ipt, ns, th, de, tol=1e-10, precision=p, max_iter=64, flags=ipt.FLAG_CHOOSE_D)
    _, _, st_plain, _ = _run(ipt, ns, th, de, tol=1e-10, precision=p, max_iter=64)
    compared = 0
    for b in range(len(ns)):
        n = int(ns[b])
        gz, gl, gs = _per_problem(ns, th_off, de_off, z, lam, st, b)
        thb, deb = th[th_off[b]:th_off[b] + n], de[de_off[b]:de_off[b] + n * n].reshape(n, n)
        th2, de2, partner, cs = oracle.choose_d(thb, deb, ipt.PAIR_TAU)
        rr = oracle.ipt_dense(th2, de2, tol=1e-10, max_iter=64)
        rr["z"] = oracle.pair_back_rotate(rr.z, partner, cs)
        out = check(gz, gl, gs, rr, oracle.norm1(thb, deb), 1e-10, max_iter=64)
        compared += out["compared"]
    assert compared >= 0.95 * int(ns.sum())
    for q in range(3):
        b = 20 + q
        s_rot = st[th_off[b]:th_off[b] + ns[b]]
        s_pl = st_plain[th_off[b]:th_off[b] + ns[b]]
        assert np.all(s_rot == 0)
        assert np.any(s_pl != 0)
    assert info["converged"] == int((st == 0).sum())
