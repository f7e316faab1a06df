"""GPU tests of the learned warm start: HIP loss, gradients and outputs within the
bounds of the BF16 network reference, the series terms against the oracle's
Rayleigh-Schroedinger recursion, training, and warm-started solves that keep the
oracle's answers."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import dev, say, t
from oracle import mlp as ref_mlp
from parity import angles, check

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ipt():
    from paper_2012_14702_amd import ipt as mod
    mod.load_library()
    dev()
    return mod


def _random_net(ipt, dims, batch, seed, scale=0.3):
    rng = np.random.default_rng(seed)
    net = ipt.MLP(*dims, seed=seed)
    p = (rng.standard_normal(net.num_params) * scale).astype(np.float32)
    net.set_params(t(p))
    x = rng.standard_normal((batch, dims[0])).astype(np.float32)
    tg = rng.standard_normal((batch, dims[-1])).astype(np.float32)
    return net, p.astype(np.float64), x, tg


@pytest.mark.parametrize("dims,batch,weighted", [((2, 64, 2, 300), 37, False), ((2, 64, 2, 300), 37, True),
                                                 ((2, 48, 3, 130), 64, False), ((3, 128, 2, 257), 200, True),
                                                 ((2, 256, 2, 32768), 512, True)])
def test_gradients_within_the_bf16_network_bounds(ipt, dims, batch, weighted):
    """ipt_mlp_loss_grad and ipt_mlp_forward against the network at the kernels' BF16
    rounding points with exact arithmetic in between (oracle.mlp.network_bf16): loss,
    every gradient element and every output within the bounds of what FP32 arithmetic
    may change; padded sizes (48, 130, 257, batch 37), per-example loss weights, and the
    benchmarked network (2 -> 256 -> 256 -> 32768 at batch 512, split-K products)."""
    say("mlp gradients dims=%s batch=%d weighted=%s" % (dims, batch, weighted))
    net, p, x, tg = _random_net(ipt, dims, batch, 3)
    w = np.random.default_rng(4).uniform(0.0, 1.0, batch).astype(np.float32) if weighted else None
    loss, g = net.loss_grad(t(x), t(tg), weights=None if w is None else t(w))
    y = net.forward(t(x)).cpu().numpy().astype(np.float64)
    g = g.cpu().numpy().astype(np.float64)
    rloss, rg, ry, lb, gb, yb = ref_mlp.network_bf16(p, x, tg, dims, row_weights=w)
    assert abs(loss - rloss) <= lb, (loss, rloss, lb)
    bad = np.abs(g - rg) > gb
    assert not bad.any(), "%d gradient entries outside the bounds, first %s: %r vs %r (bound %r)" % (
        bad.sum(), np.where(bad)[0][:5], g[bad][:5], rg[bad][:5], gb[bad][:5])
    assert np.all(np.abs(y - ry) <= yb)


def test_series_terms_and_start_match_the_oracle(ipt):
    """ipt_rs_terms against the oracle's Rayleigh-Schroedinger recursion (App. B) on 17
    scattered columns of a ragged n = 300 matrix, order 5; ipt_rs_start against the
    partial sums of those terms; an index out of range and a degenerate theta are
    refused."""
    say("rs terms n=300 k=17 order 5")
    th, de = W.dense_sym_gaussian(300, 1.0, 4)
    idx = np.random.default_rng(2).permutation(300)[:17].astype(np.int32)
    terms = ipt.ipt_rs_terms(t(th), t(de), t(idx), 5).cpu().numpy()
    ref = oracle.rs_series(th, de, 5)
    for l in range(1, 6):
        rt = ref[l][:, idx]
        assert np.max(np.abs(terms[l - 1] - rt)) <= 1e-12 * np.abs(rt).max(), l
    eps = np.array([0.0, 0.01, 0.03, 0.05])
    z0 = ipt.ipt_rs_start(t(np.ascontiguousarray(terms[:3])), t(eps), t(idx)).cpu().numpy()
    for p_, e in enumerate(eps):
        want = ref[0][:, idx] + sum(e ** l * ref[l][:, idx] for l in range(1, 4))
        assert np.max(np.abs(z0[p_] - want)) <= 1e-13
    bad = idx.copy()
    bad[3] = 300
    with pytest.raises(ipt.IPTError) as e:
        ipt.ipt_rs_terms(t(th), t(de), t(bad), 2)
    assert e.value.status == ipt.IPT_EINVAL
    th2 = th.copy()
    th2[7] = th2[idx[0]]
    with pytest.raises(ipt.IPTError) as e:
        ipt.ipt_rs_terms(t(th2), t(de), t(idx), 2)
    assert e.value.status == ipt.IPT_EDEGENERATE


@pytest.mark.parametrize("hidden", [32, 384])
def test_targets_and_prediction_definitions(ipt, hidden):
    """ipt_mlp_targets and ipt_mlp_predict_z0 on synthetic inputs against their
    definitions: targets are the remainders (Z - E - sum_l eps^l T_l) / eps^(order+1)
    standardised with weighted mean and spread, and a prediction is E + sum_l eps^l T_l + eps^(order+1) (mu + sigma y)
    with y the network output (within its BF16-network bounds). Hidden width 32: the
    one-launch hidden layers reading x itself; 384: the packed input and the per-layer
    products."""
    import torch
    say("mlp targets and prediction n=64 k=5")
    n, k, order, b = 64, 5, 2, 9
    th, de = W.dense_sym_gaussian(n, 1.0, 6)
    idx = np.array([0, 7, 19, 40, 63], dtype=np.int32)
    ref = oracle.rs_series(th, de, order)
    terms = np.stack([ref[l][:, idx] for l in range(1, order + 1)])
    rng = np.random.default_rng(8)
    eps = rng.uniform(0.01, 0.08, b)
    z = rng.standard_normal((b, n, k)) * 1e-3
    z[:, idx, np.arange(k)] = 1.0
    wts = rng.uniform(0.1, 1.0, b)
    tg, mu, sd = ipt.ipt_mlp_targets(t(z), t(idx), t(eps), t(terms), weights=t(wts))
    e0 = np.zeros((n, k))
    e0[idx, np.arange(k)] = 1.0
    rem = np.stack([(z[p_] - e0 - sum(eps[p_] ** l * terms[l - 1] for l in range(1, order + 1))) / eps[p_] ** (order + 1)
                    for p_ in range(b)]).reshape(b, n * k)
    w2 = (wts ** 2)[:, None]
    m_ = (w2 * rem).sum(axis=0) / w2.sum()
    s_ = np.sqrt((w2 * (rem - m_) ** 2).sum(axis=0) / w2.sum())
    s_ = np.where(s_ >= 1e-300, s_, 1.0)  # entries with no spread (the unit entries) keep sigma = 1
    np.testing.assert_allclose(mu.cpu().numpy(), m_, rtol=1e-6, atol=1e-30)
    np.testing.assert_allclose(sd.cpu().numpy(), s_, rtol=1e-6)
    np.testing.assert_allclose(tg.cpu().numpy(), (rem - m_) / s_, rtol=1e-5, atol=1e-5)
    dims = (2, hidden, 2, n * k)
    net, p, _, _ = _random_net(ipt, dims, b, 11)
    x = np.stack([eps / 0.08, (eps / 0.08) ** 2], axis=1).astype(np.float32)
    mu_h = rng.standard_normal(n * k).astype(np.float32)
    sd_h = rng.uniform(0.5, 2.0, n * k).astype(np.float32)
    z0 = net.predict_z0(t(x), t(mu_h), t(sd_h), t(eps), n, k, t(idx), terms=t(terms)).cpu().numpy()
    _, _, ry, _, _, yb = ref_mlp.network_bf16(p, x, np.zeros((b, n * k)), dims)
    for p_ in range(b):
        sc = eps[p_] ** (order + 1)
        base = e0 + sum(eps[p_] ** l * terms[l - 1] for l in range(1, order + 1))
        want = base + sc * (mu_h + sd_h * ry[p_]).reshape(n, k)
        want[idx, np.arange(k)] = 1.0
        tol = sc * (sd_h * yb[p_]).reshape(n, k) + 1e-15
        assert np.all(np.abs(z0[p_] - want) <= tol + 1e-12 * sc)


@pytest.mark.parametrize("n,k,hidden,depth,order", [(1024, 32, 256, 2, 2), (97, 5, 128, 3, 3), (64, 8, 32, 1, 0),
                                                     (40, 4, 256, 2, 6), (50, 4, 384, 1, 1)])
def test_prediction_rows_do_not_depend_on_the_batch(ipt, n, k, hidden, depth, order):
    """A member's warm start does not depend on the other members or on the batch's
    padding: the first 100 members of a 200-member prediction (two 128-row tiles) equal
    a 100-member prediction bit for bit, and so does a repeat and a 7-member call. Hidden
    layers of width <= 256 run as one launch reading x itself; 384 takes the packed
    input and the per-layer products. Vector stores of the epilogue (k a multiple of 4,
    order <= 4) and scalar ones (k = 5; order 6)."""
    say("mlp prediction rows n=%d k=%d hidden=%d depth=%d order=%d" % (n, k, hidden, depth, order))
    dims = (2, hidden, depth, n * k)
    net, _, _, _ = _random_net(ipt, dims, 8, 21, scale=0.1)
    rng = np.random.default_rng(22)
    b = 200
    eps = rng.uniform(0.005, 0.02, b)
    x = np.stack([eps / 0.02, (eps / 0.02) ** 2], axis=1).astype(np.float32)
    idx = np.sort(rng.choice(n, k, replace=False)).astype(np.int32)
    mu = rng.standard_normal(n * k).astype(np.float32)
    sd = rng.uniform(0.5, 2.0, n * k).astype(np.float32)
    terms = rng.standard_normal((order, n, k)) if order else None
    kw = dict(terms=None if terms is None else t(terms))
    z_all = net.predict_z0(t(x), t(mu), t(sd), t(eps), n, k, t(idx), **kw).cpu().numpy()
    z_few = net.predict_z0(t(x[:100]), t(mu), t(sd), t(eps[:100]), n, k, t(idx), **kw).cpu().numpy()
    assert np.array_equal(z_all[:100], z_few)
    assert np.array_equal(net.predict_z0(t(x[:100]), t(mu), t(sd), t(eps[:100]), n, k, t(idx), **kw).cpu().numpy(), z_few)
    assert np.array_equal(net.predict_z0(t(x[:7]), t(mu), t(sd), t(eps[:7]), n, k, t(idx), **kw).cpu().numpy(), z_few[:7])
    assert np.all(z_few[:, idx, np.arange(k)] == 1.0)
    assert np.all(np.isfinite(z_few))


def test_training_reduces_loss(ipt):
    import torch
    say("mlp training")
    dims = (2, 64, 2, 50)
    net = ipt.MLP(*dims, seed=0)
    e = np.linspace(0, 1, 64)
    x = np.stack([e, e * e], 1).astype(np.float32)
    tg = np.sin(3 * e[:, None] + np.arange(50)[None, :] * 0.1).astype(np.float32)
    l0, _ = net.loss_grad(t(x), t(tg))
    l1 = net.train(t(x), t(tg), 400, 3e-3)
    assert l1 < 0.05 * l0


def test_warm_start_keeps_answers_and_saves_sweeps(ipt):
    """Family diag(1..256) + eps R, k = 16 lowest: a network trained on 96 solutions
    warm-starts 12 new eps; every column matches the oracle and the cold solve, and the
    mean sweep count drops."""
    import torch
    from paper_2012_14702_amd import warmstart
    say("mlp warm start n=256")
    n, k = 256, 16
    th, base = W.family_base(n, 0)
    thd, based = t(th), t(base)
    idx = t(W.lowest_indices(th, k))
    eps_tr = W.family_eps(96, 0.0, 0.08, seed=1)
    eps_te = W.family_eps(12, 0.0, 0.08, seed=2)
    ztr, _, st_tr, _, _ = warmstart.solve_family(thd, based, eps_tr, idx, tol=1e-12)
    assert int((st_tr != 0).sum()) == 0
    ws = warmstart.WarmStarter(n, k, hidden=128, depth=2, seed=0)
    ws.set_family(thd, based, idx)
    # the targets are standardised remainders after the series, so the loss measures the
    # fit in units of each entry's spread over eps; what counts is the start it gives
    loss, _ = ws.fit(ztr, eps_tr, idx, steps=600, lr=2e-3)
    assert np.isfinite(loss)
    z0 = ws.predict(eps_te, idx)
    zc, lc, sc, swc, _ = warmstart.solve_family(thd, based, eps_te, idx, tol=1e-10)
    zw, lw, sw, sww, _ = warmstart.solve_family(thd, based, eps_te, idx, z0=z0, tol=1e-10)
    assert np.all(sc.cpu().numpy() == 0) and np.all(sw.cpu().numpy() == 0)
    assert sww.mean() < swc.mean()
    for p, e in enumerate(eps_te):
        de = e * base
        ref = oracle.ipt_dense(th, de, idx=W.lowest_indices(th, k), tol=1e-10)
        check(zw[p].cpu().numpy(), lw[p].cpu().numpy(), sw[p].cpu().numpy(), ref, oracle.norm1(th, de), 1e-10)
        assert np.max(angles(zw[p].cpu().numpy(), zc[p].cpu().numpy())) <= 1e-8


@pytest.mark.timeout(600)
def test_warm_start_benchmark_size(ipt):
    """The benchmarked learned configuration: family diag(1..1024) + eps R, k = 32
    lowest, the 2 -> 256 -> 256 -> 32768 network trained on 512 eps ~ U[0, 0.08]
    (seed 1) for the benchmark's 3000 Adam steps; 8 of the 128 test eps (seed 2),
    warm-started, each column against the oracle's cold solve (the start must not
    change the answer), with fewer sweeps than the cold start on average."""
    from paper_2012_14702_amd import warmstart
    say("mlp warm start n=1024 k=32 (benchmark size)")
    n, k = 1024, 32
    th, base = W.family_base(n, 0)
    thd, based = t(th), t(base)
    idx_h = W.lowest_indices(th, k)
    idx = t(idx_h)
    eps_tr = W.family_eps(512, 0.0, 0.08, seed=1)
    eps_te = W.family_eps(128, 0.0, 0.08, seed=2)[::16]
    ztr, _, st_tr, _, _ = warmstart.solve_family(thd, based, eps_tr, idx, tol=1e-12)
    assert int((st_tr != 0).sum()) == 0
    ws = warmstart.WarmStarter(n, k, hidden=256, depth=2, seed=0)
    ws.set_family(thd, based, idx)
    ws.fit(ztr, eps_tr, idx, steps=3000, lr=1e-3)
    z0 = ws.predict(eps_te, idx)
    _, _, sc, swc, _ = warmstart.solve_family(thd, based, eps_te, idx, tol=1e-10)
    zw, lw, sw, sww, _ = warmstart.solve_family(thd, based, eps_te, idx, z0=z0, tol=1e-10)
    assert np.all(sc.cpu().numpy() == 0) and np.all(sw.cpu().numpy() == 0)
    assert sww.mean() < swc.mean()
    for p, e in enumerate(eps_te):
        de = e * base
        ref = oracle.ipt_dense(th, de, idx=idx_h, tol=1e-10, resid=False)
        check(zw[p].cpu().numpy(), lw[p].cpu().numpy(), sw[p].cpu().numpy(), ref, oracle.norm1(th, de), 1e-10)
