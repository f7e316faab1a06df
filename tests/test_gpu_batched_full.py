"""GPU parity of the batched path on the whole benchmarked batch: 4096 problems with
n_b ~ U{32..512} (1 121 466 eigenpairs, 3.1 GB of Delta pools, so the pool offsets of
the later problems pass 2^31 bytes), theta_b = sort(U(0, n_b)), Delta_b = 0.02 (R+R^T)/2,
R iid N(0, 1/n_b), seed 0, tol 1e-10, 64 sweeps; the ladder, and the ladder with the
choice of D.  The batch is solved whole, as the benchmark does; the oracle solves a
sample of 64 problems (Alg. 2 per problem) that includes the last ones."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import dev, say
from parity import check

pytestmark = pytest.mark.gpu

B = 4096


@pytest.fixture(scope="module")
def ipt():
    from paper_2012_14702_amd import ipt as mod
    mod.load_library()
    dev()
    return mod


@pytest.fixture(scope="module")
def batch():
    import torch
    say("batched full batch: generating %d problems" % B)
    ns, th, de, th_off, de_off = W.batched_sym_gaussian(B, 32, 512, 0.02, seed=0)
    d = dev()
    thd = torch.from_numpy(th).to(d)
    ded = torch.from_numpy(de).to(d)
    del de
    return ns, th, th_off, de_off, thd, ded


def _sample(ns, de_off):
    """64 problems: the last 16 (offsets beyond 2^31 bytes), the first ones past that
    boundary, the first problem, and 44 drawn at random."""
    beyond = np.where(de_off * 8 >= 2 ** 31)[0]
    picks = set(range(B - 16, B)) | {0, int(beyond[0]), int(beyond[0]) - 1, int(beyond[0]) + 1}
    rng = np.random.default_rng(2024)
    while len(picks) < 64:
        picks.add(int(rng.integers(0, B)))
    return sorted(picks)


def _problem(ns, th, th_off, b):
    n = int(ns[b])
    _, de_b = W.batched_problem(b, n, 0.02, 0)
    return th[th_off[b]:th_off[b] + n], de_b


@pytest.mark.timeout(600)
@pytest.mark.parametrize("mode", ["ladder", "ladder_choose_d"])
def test_full_batch_sampled_parity(ipt, batch, mode):
    import torch
    ns, th, th_off, de_off, thd, ded = batch
    flags = ipt.FLAG_CHOOSE_D if mode == "ladder_choose_d" else 0
    say("batched full batch %s: solving" % mode)
    z = torch.empty_like(ded)
    lam = torch.empty_like(thd)
    st = torch.empty(thd.shape[0], dtype=torch.int32, device=thd.device)
    r = ipt.ipt_solve_batched(ns, thd, ded, th_off, de_off, tol=1e-10, precision=ipt.PREC_LADDER, max_iter=64,
                              flags=flags, z_out=z, lam_out=lam, status_out=st)
    torch.cuda.synchronize()
    st_all = st.cpu().numpy()
    assert r.info["converged"] == int((st_all == 0).sum())
    assert r.info["converged"] >= (0.9999 if flags else 0.995) * int(ns.sum())
    picks = _sample(ns, de_off)
    say("batched full batch %s: oracle on %d problems" % (mode, len(picks)))
    compared = total = 0
    for b in picks:
        n = int(ns[b])
        thb, deb = _problem(ns, th, th_off, b)
        gz = z[int(de_off[b]):int(de_off[b]) + n * n].cpu().numpy().reshape(n, n)
        gl = lam[int(th_off[b]):int(th_off[b]) + n].cpu().numpy()
        gs = st_all[th_off[b]:th_off[b] + n]
        if flags:
            th2, de2, partner, cs = oracle.choose_d(thb, deb, ipt.PAIR_TAU)
            ref = oracle.ipt_dense(th2, de2, tol=1e-10, max_iter=64, resid=False)
            ref["z"] = oracle.pair_back_rotate(ref.z, partner, cs)
        else:
            ref = oracle.ipt_dense(thb, deb, tol=1e-10, max_iter=64, resid=False)
        say("batched full batch %s: problem %d (n=%d)" % (mode, b, n))
        out = check(gz, gl, gs, ref, oracle.norm1(thb, deb), 1e-10, max_iter=64, ladder=True)
        compared += out["compared"]
        total += n
    say("batched full batch %s: %d of %d sampled columns compared" % (mode, compared, total))
    assert compared >= 0.99 * total
