"""GPU (HIP, gfx950) vs the CPU FP64 oracle on the same seeded inputs, through
the C ABI.  Sizes span several tiles and a ragged tail."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests._parity import assert_operator_close, iteration_tolerance, shadow_horizon, shadow_runs

pytestmark = pytest.mark.gpu

fc = pytest.importorskip("paper_2402_05598_amd")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _to(dev, *arrs):
    return [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in arrs]


def _batch(seeds, N, contrast=(10.0, 1000.0)):
    ks, fs, us = [], [], []
    for s in seeds:
        k, f, u0, _ = synth.system(s, N, contrast)
        ks.append(k); fs.append(f); us.append(u0)
    return np.stack(ks), np.stack(fs), np.stack(us)


# ------------------------------------------------------------- operator ----

@pytest.mark.parametrize("N,C,M", [(32, 16, 8), (40, 16, 8), (50, 32, 12), (64, 32, 12), (24, 16, 12)])
def test_precond_apply_matches_oracle(dev, N, C, M):
    print(f"precond N={N} C={C} M={M}", flush=True)
    k, f, _ = _batch([N * 7 + 1, N * 7 + 2], N)
    wb = synth.init_weights(N + C + M, C, M)
    w = oracle.unpack_weights(wb, C, M)
    ref = oracle.no_apply(w, torch.from_numpy(k), torch.from_numpy(f)).numpy()
    model = fc.Model(wb, C, M)
    kt, ft = _to(dev, k, f)
    for op in ("fp64", "fp32", "bf16"):
        got = fc.precond_apply(model, kt, ft, op=op).cpu().numpy()
        for b in range(2):
            assert_operator_close(got[b], ref[b], op, f"b={b}")
    model.close()


def test_precond_zero_and_homogeneity(dev):
    N, C, M = 32, 16, 8
    k, f, _ = _batch([5], N)
    model = fc.Model(synth.init_weights(3, C, M), C, M)
    kt, ft = _to(dev, k, f)
    z = fc.precond_apply(model, kt, torch.zeros_like(ft), op="fp64")
    assert torch.count_nonzero(z) == 0
    a = fc.precond_apply(model, kt, ft, op="fp64")
    b = fc.precond_apply(model, kt, ft * 8.0, op="fp64")
    assert torch.equal(b, a * 8.0)


# ------------------------------------------------------ FCG with B = I -----

@pytest.mark.parametrize("N", [32, 50, 64])
def test_identity_fcg_matches_oracle(dev, N):
    print(f"identity N={N}", flush=True)
    k, f, u0 = _batch([100 + N, 200 + N], N)
    kt, ft, ut = _to(dev, k, f, u0)
    out = fc.solve(None, kt, ft, ut, op="identity", m_max=5, max_iter=2000, rtol=1e-6)
    for b in range(2):
        ref, H, its = shadow_runs(k[b], f[b], u0[b], None, 5, 2000, 1e-6)
        got = out["hist"][b, :ref.iters + 1]
        n = min(H, ref.iters) + 1
        rel = np.max(np.abs(got[:n] - np.array(ref.hist[:n])) / np.array(ref.hist[:n]))
        tol_it = iteration_tolerance(ref.iters, its)
        print(f"  b={b} iters gpu={out['iters'][b]} oracle={ref.iters} shadows={its} H={H} rel={rel:.2e}",
              flush=True)
        assert rel < 1e-10
        assert out["status"][b] == ref.status == oracle.SYS_OK
        assert abs(int(out["iters"][b]) - ref.iters) <= tol_it
        assert out["true_rel_res"][b] < 2e-6


# ------------------------------------------------------ FCG-NO, FP64 op ----

def test_fcgno_fp64_config0_matches_oracle(dev):
    """32x32, one solve, C=16, M=8, seeded random-init operator, m_max=5."""
    N, C, M = 32, 16, 8
    k, f, u0, _ = synth.system(0, N)
    wb = synth.init_weights(0, C, M)
    w = oracle.unpack_weights(wb, C, M)
    B = lambda r: oracle.no_apply(w, torch.from_numpy(k), r)
    ref, H = shadow_horizon(k, f, u0, B, 5, 300, 1e-6)
    model = fc.Model(wb, C, M)
    kt, ft, ut = _to(dev, k[None], f[None], u0[None])
    out = fc.solve(model, kt, ft, ut, op="fp64", m_max=5, max_iter=300, rtol=1e-6)
    n = min(H, ref.iters) + 1
    got = out["hist"][0, :n]
    rel = np.max(np.abs(got - np.array(ref.hist[:n])) / np.array(ref.hist[:n]))
    print(f"config0 iters gpu={out['iters'][0]} oracle={ref.iters} status {out['status'][0]}/{ref.status} "
          f"H={H} rel={rel:.2e}", flush=True)
    assert H >= 5
    assert rel < 1e-10
    assert out["status"][0] == ref.status
    assert int(out["iters"][0]) == ref.iters


def test_batch_invariance_and_determinism(dev):
    """A system gives the same bits alone and inside a batch, and twice."""
    N, C, M = 40, 16, 8
    k, f, u0 = _batch([11, 12, 13], N)
    model = fc.Model(synth.init_weights(9, C, M), C, M)
    kt, ft, ut = _to(dev, k, f, u0)
    u_all = ut.clone()
    a = fc.solve(model, kt, ft, u_all, op="bf16", m_max=5, max_iter=40, rtol=1e-9)
    u_one = ut[1:2].clone()
    b = fc.solve(model, kt[1:2].contiguous(), ft[1:2].contiguous(), u_one, op="bf16", m_max=5, max_iter=40,
                 rtol=1e-9)
    assert np.array_equal(a["hist"][1], b["hist"][0], equal_nan=True)
    assert torch.equal(u_all[1], u_one[0])
    u_again = ut.clone()
    c = fc.solve(model, kt, ft, u_again, op="bf16", m_max=5, max_iter=40, rtol=1e-9)
    assert np.array_equal(a["hist"], c["hist"], equal_nan=True)
    assert torch.equal(u_all, u_again)


def test_status_cases(dev):
    N = 16
    k, f, u0 = _batch([1, 2, 3, 4], N)
    k[0, 3, 4] = np.nan
    k[1, 0, 5] = -1.0          # a boundary node
    f[2] = 0.0
    u0[2] = 0.0
    kt, ft, ut = _to(dev, k, f, u0)
    out = fc.solve(None, kt, ft, ut, op="identity", m_max=5, max_iter=1, rtol=1e-6)
    assert list(out["status"]) == [fc.SYS_NONFINITE, fc.SYS_NONFINITE, fc.SYS_OK, fc.SYS_NOT_CONVERGED]
    assert list(out["iters"]) == [0, 0, 0, 1]
    assert out["rc"] == 1


@pytest.mark.parametrize("op", ["bf16", "identity", "sgs_rb"])
def test_stopped_systems_leave_the_launches(dev, op):
    """Systems stop at different iterations (two with f = 0 at once, the rest
    as they converge); once the polled count drops, the launches run on a
    compacted table of the active systems.  Every system gives the same bits
    as when it is solved alone."""
    N, C, M = 40, 16, 8
    seeds = [31, 32, 33, 34, 35, 36]
    k, f, u0 = _batch(seeds, N, contrast=(1.0, 100.0))
    f[1] = 0.0
    u0[1] = 0.0
    f[4] = 0.0
    u0[4] = 0.0
    model = fc.Model(synth.init_weights(5, C, M), C, M) if op == "bf16" else None
    kt, ft, ut = _to(dev, k, f, u0)
    u_all = ut.clone()
    kw = dict(op=op, m_max=5, max_iter=300, rtol=1e-6, check_every=4)
    if op == "sgs_rb":
        kw["precond_steps"] = 1
    a = fc.solve(model, kt, ft, u_all, **kw)
    print(f"  {op}: iters {list(a['iters'])} status {list(a['status'])}", flush=True)
    assert a["iters"][1] == 0 and a["iters"][4] == 0
    assert len(set(int(v) for v in a["iters"])) >= 2
    for b in range(len(seeds)):
        u1 = ut[b:b + 1].clone()
        one = fc.solve(model, kt[b:b + 1].contiguous(), ft[b:b + 1].contiguous(), u1, **kw)
        assert one["iters"][0] == a["iters"][b] and one["status"][0] == a["status"][b], b
        assert np.array_equal(one["hist"][0], a["hist"][b], equal_nan=True), b
        assert torch.equal(u1[0], u_all[b]), b
