"""GPU parity of the dense IPT path (C ABI ipt_solve_dense) against the FP64 oracle."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import dev, host, say, t
from parity import check

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ipt():
    from paper_2012_14702_amd import ipt as mod
    mod.load_library()
    dev()
    return mod


def _solve(ipt, theta, delta, idx=None, z0=None, **kw):
    r = ipt.ipt_solve_dense(t(theta), t(delta), idx=None if idx is None else t(idx.astype(np.int32)),
                            z0=None if z0 is None else t(z0), **kw)
    return host(r)


def test_small_full_spectrum_parity(ipt):
    """n = 256, eps = 0.01, full spectrum, stop at max column step 1e-12."""
    say("dense n=256 eps=0.01 fp64")
    th, de = W.dense_sym_gaussian(256, 0.01, 0)
    g = _solve(ipt, th, de, tol=1e-12)
    ref = oracle.ipt_dense(th, de, tol=1e-12)
    out = check(g.z, g.lam, g.status, ref, oracle.norm1(th, de), 1e-12, gpu_sweeps=g.sweeps)
    assert out["compared"] == 256
    assert np.all(np.diag(g.z) == 1.0)
    assert abs(g.info["norm1"] - oracle.norm1(th, de)) <= 1e-13 * oracle.norm1(th, de)


@pytest.mark.parametrize("n,k,kind,eps", [(1, 1, "full", 0.1), (2, 2, "full", 0.2), (3, 2, "rand", 0.2),
                                          (129, 129, "full", 0.02), (300, 37, "rand", 0.03),
                                          (257, 200, "low", 0.02), (640, 640, "full", 0.05),
                                          (500, 130, "rand", 0.01)])
def test_ragged_shapes(ipt, n, k, kind, eps):
    """Sizes that are not tile multiples, subsets of columns in any order."""
    say("dense ragged n=%d k=%d %s" % (n, k, kind))
    th, de = W.dense_sym_gaussian(n, eps, 3)
    rng = np.random.default_rng(n)
    idx = {"full": None, "rand": rng.permutation(n)[:k], "low": np.arange(k)}[kind]
    g = _solve(ipt, th, de, idx=idx, tol=1e-12)
    ref = oracle.ipt_dense(th, de, idx=idx, tol=1e-12)
    check(g.z, g.lam, g.status, ref, oracle.norm1(th, de), 1e-12, gpu_sweeps=g.sweeps)
    cols = np.arange(k) if idx is None else idx
    assert np.all(g.z[cols, np.arange(k)] == 1.0)


def test_nonsymmetric_paper_family(ipt):
    """The paper's non-symmetric dense family diag(i) + 0.01 R, R ~ U[0,1]."""
    say("dense nonsym n=384")
    th, de = W.dense_uniform_nonsym(384, 0.01, 1)
    g = _solve(ipt, th, de, tol=1e-12)
    ref = oracle.ipt_dense(th, de, tol=1e-12)
    check(g.z, g.lam, g.status, ref, oracle.norm1(th, de), 1e-12, gpu_sweeps=g.sweeps)


@pytest.mark.parametrize("n,pair", [(300, (299, 298)), (256, (64, 63)), (129, (128, 127))])
def test_nearly_symmetric(ipt, n, pair):
    """A symmetric Delta with one entry Delta_ab (b = a - 1) changed by 2e-3: the
    exact-symmetry check must see it, else the reported lambda_a = theta_a + d_a would
    use Delta_ba for Delta_ab and be off by about 2e-3 |z_b| ~ 3e-6, far above the
    bound.  The pairs sit in a diagonal 64 x 64 tile at the ragged edge, across two
    tiles, and in a last row tile of one row."""
    say("dense nearly symmetric n=%d pair=%s" % (n, pair))
    th, de = W.dense_sym_gaussian(n, 0.03, 4)
    de = de.copy()
    de[pair] += 2e-3
    for prec in ("fp64", "ladder"):
        p = ipt.PREC_LADDER if prec == "ladder" else ipt.PREC_FP64
        g = _solve(ipt, th, de, tol=1e-11, precision=p)
        ref = oracle.ipt_dense(th, de, tol=1e-11)
        check(g.z, g.lam, g.status, ref, oracle.norm1(th, de), 1e-11)


@pytest.mark.parametrize("eps,want", [(0.3, 0), (0.9, 1), (2.0, 2)])
def test_two_by_two_statuses(ipt, eps, want):
    """2x2 example: converges below sqrt(3)/2, cycles at 0.9, diverges at 2."""
    say("dense 2x2 eps=%g" % eps)
    th, de = W.two_by_two(eps)
    g = _solve(ipt, th, de, tol=1e-12, max_iter=300)
    ref = oracle.ipt_dense(th, de, tol=1e-12, max_iter=300)
    assert np.all(ref.status == want)
    assert np.all(g.status == want)
    if want == 0:
        check(g.z, g.lam, g.status, ref, oracle.norm1(th, de), 1e-12)


@pytest.mark.parametrize("stop", [1, 2])
@pytest.mark.parametrize("kind", ["sym", "nonsym"])
def test_warm_start_resume_and_determinism(ipt, kind, stop):
    """Stopping after 1 or 2 sweeps and resuming from the returned iterate equals the
    uninterrupted solve bit for bit (the resumed first sweep computes d from Delta and
    Z in the order in which the uninterrupted solve's previous sweep formed it); two
    identical solves are bitwise equal."""
    say("dense resume n=384 %s stop=%d" % (kind, stop))
    if kind == "sym":
        th, de = W.dense_sym_gaussian(384, 0.03, 2)
    else:
        th, de = W.dense_uniform_nonsym(384, 0.03, 2)
    full = _solve(ipt, th, de, tol=1e-12)
    again = _solve(ipt, th, de, tol=1e-12)
    np.testing.assert_array_equal(full.z, again.z)
    np.testing.assert_array_equal(full.lam, again.lam)
    part = _solve(ipt, th, de, tol=1e-12, max_iter=stop)
    assert np.all(part.status == 1)
    res = _solve(ipt, th, de, z0=part.z, tol=1e-12)
    np.testing.assert_array_equal(res.z, full.z)
    np.testing.assert_array_equal(res.lam, full.lam)
    np.testing.assert_array_equal(res.sweeps + stop, full.sweeps)
    ref = oracle.ipt_dense(th, de, z0=part.z, tol=1e-12)
    check(res.z, res.lam, res.status, ref, oracle.norm1(th, de), 1e-12)


def test_invalid_arguments(ipt):
    say("dense invalid args")
    th, de = W.dense_sym_gaussian(64, 0.01, 0)
    with pytest.raises(ipt.IPTError) as e:
        _solve(ipt, th, de, idx=np.array([1, 5, 1]))
    assert e.value.status == ipt.IPT_EINVAL
    with pytest.raises(ipt.IPTError) as e:
        _solve(ipt, th, de, idx=np.array([0, 64]))
    assert e.value.status == ipt.IPT_EINVAL
    bad = th.copy()
    bad[7] = np.nan
    with pytest.raises(ipt.IPTError) as e:
        _solve(ipt, bad, de)
    assert e.value.status == ipt.IPT_EINVAL
    deg = th.copy()
    deg[9] = deg[3]
    with pytest.raises(ipt.IPTError) as e:
        _solve(ipt, deg, de, idx=np.array([3, 20]))
    assert e.value.status == ipt.IPT_EDEGENERATE
    # a repeated theta outside the requested columns' gaps is fine
    deg2 = th.copy()
    deg2[40] = deg2[41] = 100.5
    r = _solve(ipt, deg2, de, idx=np.array([3, 20]), tol=1e-12)
    assert np.all(r.status == 0)
    with pytest.raises(ipt.IPTError) as e:
        _solve(ipt, th, de, tol=-1.0)
    assert e.value.status == ipt.IPT_EINVAL


@pytest.mark.parametrize("eps", [0.005, 0.01, 0.05])
@pytest.mark.parametrize("low", ["bf16", "fp16", "none"])
def test_ladder_parity(ipt, eps, low):
    """Precision ladder: low -> FP32 -> FP64; only FP64 sweeps certify, so the
    answer matches the FP64 oracle to the same bounds."""
    say("dense ladder n=1024 eps=%g low=%s" % (eps, low))
    th, de = W.dense_sym_gaussian(1024, eps, 0)
    lt = {"bf16": ipt.LOW_BF16, "fp16": ipt.LOW_FP16, "none": ipt.LOW_NONE}[low]
    g = _solve(ipt, th, de, tol=1e-10, precision=ipt.PREC_LADDER, low_type=lt)
    ref = oracle.ipt_dense(th, de, tol=1e-10)
    check(g.z, g.lam, g.status, ref, oracle.norm1(th, de), 1e-10)
    assert g.info["sweep_prec"][-1] == "fp64"
    # the rung after the exact first sweep follows its step s1 (~ the contraction
    # ratio of a cold start): the low rung unless s1^3 predicts certification within
    # the slack (eps = 0.005 here), or the FP32-class rung first when there is none
    s1 = g.info["sweep_max_step"][0]
    slack_tol = ipt.CERTIFY_SLACK * 1e-10
    skip_low = low == "none" or s1 ** 3 <= slack_tol or s1 <= 1e-5
    assert ("low" in g.info["sweep_prec"]) == (not skip_low), (s1, g.info["sweep_prec"])
    assert skip_low == (eps == 0.005 or low == "none")
    if skip_low and s1 ** 2 > slack_tol:
        assert g.info["sweep_prec"][1] == "fp32"


@pytest.mark.parametrize("n,low", [(1024, "none"), (1024, "fp16"), (300, "none"), (300, "fp16")])
def test_ladder_without_norm(ipt, n, low):
    """IPT_FLAG_NO_NORM with the rungs that multiply FP16 shadows of Delta (the
    three-product rung, the FP16 low rung), tile-aligned and padded: |M|_1 only
    normalises the reported residual, so iterates, eigenvalues, statuses and sweep
    counts equal the normed solve's bit for bit, and both match the oracle."""
    say("dense ladder no-norm n=%d low=%s" % (n, low))
    th, de = W.dense_sym_gaussian(n, 0.01, 3)
    lt = {"fp16": ipt.LOW_FP16, "none": ipt.LOW_NONE}[low]
    a = _solve(ipt, th, de, tol=1e-10, precision=ipt.PREC_LADDER, low_type=lt)
    b = _solve(ipt, th, de, tol=1e-10, precision=ipt.PREC_LADDER, low_type=lt, flags=ipt.FLAG_NO_NORM)
    for x, y in ((a.z, b.z), (a.lam, b.lam), (a.status, b.status), (a.sweeps, b.sweeps)):
        np.testing.assert_array_equal(x, y)
    assert list(a.info["sweep_prec"]) == list(b.info["sweep_prec"])
    assert "fp32" in b.info["sweep_prec"] and b.info["norm1"] == 0.0
    assert abs(a.info["norm1"] - oracle.norm1(th, de)) <= 1e-13 * oracle.norm1(th, de)
    ref = oracle.ipt_dense(th, de, tol=1e-10)
    check(b.z, b.lam, b.status, ref, oracle.norm1(th, de), 1e-10)


@pytest.mark.parametrize("eps", [0.01, 0.05])
def test_ladder_mid_rung_three_fp16_vs_fp32(ipt, eps):
    """The FP32-class rung from three FP16 products (default) against FP32 matrix
    cores (FLAG_MID_FP32): both certify at FP64 parity, and the three-product rung
    needs no more sweeps."""
    say("dense ladder mid rung n=1024 eps=%g" % eps)
    th, de = W.dense_sym_gaussian(1024, eps, 1)
    ref = oracle.ipt_dense(th, de, tol=1e-10)
    x3 = _solve(ipt, th, de, tol=1e-10, precision=ipt.PREC_LADDER)
    f32 = _solve(ipt, th, de, tol=1e-10, precision=ipt.PREC_LADDER, flags=ipt.FLAG_MID_FP32)
    for g in (x3, f32):
        check(g.z, g.lam, g.status, ref, oracle.norm1(th, de), 1e-10)
        assert "fp32" in g.info["sweep_prec"]
    assert x3.info["sweeps"] <= f32.info["sweeps"]


@pytest.mark.parametrize("n,k", [(640, 40), (1000, 1000)])
def test_ladder_warm_start_and_narrow(ipt, n, k):
    """A warm-started ladder begins on the FP32-class rung (its FP16 shadow of Z - E is
    scaled from the loaded iterate); k = 40 columns make every product narrow (split
    K); both against the oracle from the same start."""
    say("dense ladder warm n=%d k=%d" % (n, k))
    th, de = W.dense_sym_gaussian(n, 0.03, 5)
    idx = None if k == n else np.arange(k, dtype=np.int32)
    part = _solve(ipt, th, de, idx=idx, tol=1e-12, max_iter=2)
    g = _solve(ipt, th, de, idx=idx, z0=part.z, tol=1e-10, precision=ipt.PREC_LADDER)
    assert g.info["sweep_prec"][0] == "fp32"
    ref = oracle.ipt_dense(th, de, idx=idx, z0=part.z, tol=1e-10)
    check(g.z, g.lam, g.status, ref, oracle.norm1(th, de), 1e-10)
    # a start far from tol (the first-order start F(I)): its first FP32-class step
    # gives no contraction ratio yet, so the rung is kept for a second sweep
    far = _solve(ipt, th, de, idx=idx, tol=1e-12, max_iter=1)
    g = _solve(ipt, th, de, idx=idx, z0=far.z, tol=1e-10, precision=ipt.PREC_LADDER)
    assert g.info["sweep_max_step"][0] > 1e-7
    assert g.info["sweep_prec"][:2] == ["fp32", "fp32"], g.info["sweep_prec"]
    ref = oracle.ipt_dense(th, de, idx=idx, z0=far.z, tol=1e-10)
    check(g.z, g.lam, g.status, ref, oracle.norm1(th, de), 1e-10)
    c = _solve(ipt, th, de, idx=idx, tol=1e-10, precision=ipt.PREC_LADDER)
    ref = oracle.ipt_dense(th, de, idx=idx, tol=1e-10)
    check(c.z, c.lam, c.status, ref, oracle.norm1(th, de), 1e-10)


@pytest.mark.parametrize("low", ["bf16", "none"])
def test_ladder_parity_nonsymmetric(ipt, low):
    """The ladder on the paper's non-symmetric family (the epilogue's d of the next
    sweep then reads Delta_ij itself, beside the Delta_ji of the split product)."""
    say("dense ladder nonsym n=640 low=%s" % low)
    th, de = W.dense_uniform_nonsym(640, 0.02, 3)
    lt = {"bf16": ipt.LOW_BF16, "none": ipt.LOW_NONE}[low]
    g = _solve(ipt, th, de, tol=1e-10, precision=ipt.PREC_LADDER, low_type=lt)
    ref = oracle.ipt_dense(th, de, tol=1e-10)
    check(g.z, g.lam, g.status, ref, oracle.norm1(th, de), 1e-10)
    assert g.info["sweep_prec"][-1] == "fp64"


@pytest.mark.parametrize("eps", [0.01, 0.05])
@pytest.mark.parametrize("prec", ["fp64", "ladder"])
def test_large_full_spectrum_sampled(ipt, eps, prec):
    """n = 4096 full spectrum in the benchmarked configuration; the oracle solves a
    sample of columns (each column is an independent fixed-point problem)."""
    say("dense n=4096 eps=%g %s" % (eps, prec))
    th, de = W.dense_sym_gaussian(4096, eps, 0)
    p = ipt.PREC_LADDER if prec == "ladder" else ipt.PREC_FP64
    g = _solve(ipt, th, de, tol=1e-10, precision=p)
    assert np.all(g.status == 0)
    cols = np.unique(np.concatenate([[0, 1, 127, 128, 2047, 2048, 4094, 4095],
                                     np.random.default_rng(5).integers(0, 4096, 24)])).astype(np.int32)
    ref = oracle.ipt_dense(th, de, idx=cols, tol=1e-10, resid=False)
    check(g.z[:, cols], g.lam[cols], g.status[cols], ref, oracle.norm1(th, de), 1e-10,
          gpu_sweeps=g.sweeps[cols] if prec == "fp64" else None)
    assert np.all(g.z[np.arange(4096), np.arange(4096)] == 1.0)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec", ["fp64", "ladder"])
def test_paper_family_benchmarked_size_sampled(ipt, prec):
    """The paper's non-symmetric dense family diag(i) + 0.01 U[0,1] (Sec. 6.2) at the
    benchmarked n = 16384, full spectrum, plain FP64 and the ladder; the oracle solves a
    sample of 40 columns (first, last, tile edges, random)."""
    say("dense nonsym n=16384 %s" % prec)
    n = 16384
    th, de = W.dense_uniform_nonsym(n, 0.01, 0)
    p = ipt.PREC_LADDER if prec == "ladder" else ipt.PREC_FP64
    r = ipt.ipt_solve_dense(t(th), t(de), tol=1e-10, precision=p, colinfo=False)
    cols = np.unique(np.concatenate([[0, 1, 127, 128, 8191, 8192, n - 2, n - 1],
                                     np.random.default_rng(9).integers(0, n, 32)])).astype(np.int32)
    st = r.status.cpu().numpy()
    assert np.all(st == 0)
    gz = r.z[:, torch_index(cols)].cpu().numpy()
    gl = r.lam.cpu().numpy()[cols]
    del r
    ref = oracle.ipt_dense(th, de, idx=cols, tol=1e-10, resid=False)
    check(gz, gl, st[cols], ref, oracle.norm1(th, de), 1e-10)
    assert np.all(gz[cols, np.arange(cols.shape[0])] == 1.0)


def torch_index(a):
    import torch
    return torch.from_numpy(np.asarray(a, dtype=np.int64)).to(dev())


def test_ipt_log_lines(ipt, capfd, monkeypatch):
    """IPT_LOG=1: one summary line and one line per sweep on stderr, matching ipt_info;
    nothing without it."""
    say("dense IPT_LOG n=256 ladder")
    th, de = W.dense_sym_gaussian(256, 0.01, 0)
    monkeypatch.setenv("IPT_LOG", "1")
    capfd.readouterr()
    g = _solve(ipt, th, de, tol=1e-10, precision=ipt.PREC_LADDER, flags=ipt.FLAG_TIME_KERNELS)
    err = capfd.readouterr().err
    lines = [x for x in err.splitlines() if x.startswith("[ipt] dense")]
    inf = g.info
    assert len(lines) == 1 + inf["sweeps"], err
    head = dict(f.split("=") for f in lines[0].split(": ", 1)[1].split())
    assert int(head["sweeps"]) == inf["sweeps"] and int(head["converged"]) == inf["converged"] == 256
    assert head["status"] == "IPT_OK"
    for q, ln in enumerate(lines[1:]):
        assert ln.startswith("[ipt] dense sweep %d: " % (q + 1)), ln
        f = dict(x.split("=") for x in ln.split(": ", 1)[1].split()[1:])
        assert int(f["active"]) == inf["sweep_active"][q]
        assert float(f["max_step"]) == pytest.approx(inf["sweep_max_step"][q], rel=1e-3)
        assert "product_ms" in f
    monkeypatch.setenv("IPT_LOG", "0")
    _solve(ipt, th, de, tol=1e-10)
    assert "[ipt]" not in capfd.readouterr().err


@pytest.mark.parametrize("prec", ["fp64", "ladder"])
def test_dense_choice_of_d_parity(ipt, prec):
    """IPT_FLAG_CHOOSE_D on a dense full-spectrum solve (n = 300, pairs planted beyond the
    2x2 bound, one at a 64-row tile edge): every column against the oracle's rotated
    solve (the same pairing, rotation and chart); all converge, which the plain solve
    does not; column info and the norm of the re-partitioned matrix are filled."""
    say("dense choice of D n=300 %s" % prec)
    rng = np.random.default_rng(21)
    n = 300
    th = np.arange(1.0, n + 1.0)
    r = rng.standard_normal((n, n)) * 0.01 / np.sqrt(n)
    de = (r + r.T) / 2.0
    for i, j in [(10, 11), (63, 64), (200, 201)]:
        th[j] = th[i] + 0.02
        de[i, j] = de[j, i] = 1.5 * 0.02
    p = ipt.PREC_LADDER if prec == "ladder" else ipt.PREC_FP64
    g = _solve(ipt, th, de, tol=1e-10, precision=p, max_iter=64, flags=ipt.FLAG_CHOOSE_D)
    plain = _solve(ipt, th, de, tol=1e-10, precision=p, max_iter=64)
    th2, de2, partner, cs = oracle.choose_d(th, de, ipt.PAIR_TAU)
    rr = oracle.ipt_dense(th2, de2, tol=1e-10, max_iter=64)
    rr["z"] = oracle.pair_back_rotate(rr.z, partner, cs)
    out = check(g.z, g.lam, g.status, rr, oracle.norm1(th, de), 1e-10, max_iter=64)
    assert out["compared"] == n
    assert np.all(g.status == 0) and np.any(plain.status != 0)
    # |M'|_1 of the re-partitioned matrix the sweeps ran on (M' = R^T M R)
    assert abs(g.info["norm1"] - oracle.norm1(th2, de2)) <= 1e-12 * oracle.norm1(th2, de2)
    assert np.all(g.sweeps >= 1) and np.all(g.resid[g.status == 0] <= 1e-9)
    with pytest.raises(ipt.IPTError):   # a subset of columns cannot be re-partitioned
        ipt.ipt_solve_dense(t(th), t(de), idx=t(np.arange(5, dtype=np.int32)), flags=ipt.FLAG_CHOOSE_D)
