"""Form 1 (precision) against the FP64 oracle at a preconditioner that
converges: an operator trained on the CPU with the oracle
(tests/golden/make_trained_no.py) preconditions FCG on seeded systems; the
GPU solves with the FP64, FP32 and BF16 operator must reach the same 1e-6
relative-residual stopping point as the oracle (checked on the CPU from the
returned iterate), with the iteration count reported: equal for FP64 (whose
residual history follows the oracle's to 1e-10 up to the rounding horizon),
within 20% for FP32, bounded for BF16."""
import os

import numpy as np
import pytest
import torch

import oracle
import synth
from _parity import shadow_horizon

pytestmark = pytest.mark.gpu

fc = pytest.importorskip("paper_2402_05598_amd")

C, M, L = 16, 4, 2
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "no_trained_c16_m4_l2.npy")
# seeded systems on which the oracle's FCG-NO converges in tens of iterations
CASES = [(24, 9101), (32, 9100), (32, 9101), (48, 9100)]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def blob():
    return np.load(GOLD)


@pytest.mark.parametrize("N,seed", CASES)
def test_stopping_point_matches_oracle(dev, blob, N, seed):
    print(f"precision N={N} seed={seed}", flush=True)
    k, f, u0, _ = synth.system(seed, N, (10.0, 100.0))
    w = oracle.unpack_weights(blob, C, M, L)
    kt = torch.from_numpy(k)
    pre = lambda r: oracle.no_apply(w, kt, r)
    ref, H = shadow_horizon(k, f, u0, pre, 5, 400, 1e-6)
    assert ref.status == oracle.SYS_OK
    ref_iters = int(ref.iters)
    model = fc.Model(blob, C, M, L)
    kd, fd = torch.from_numpy(k)[None].to(dev), torch.from_numpy(f)[None].to(dev)
    r0 = np.linalg.norm(f - oracle.stencil_apply(k, u0).numpy())
    for op in ("fp64", "fp32", "bf16"):
        u = torch.from_numpy(u0)[None].to(dev).contiguous()
        out = fc.solve(model, kd, fd, u, op=op, m_max=5, max_iter=400, rtol=1e-6)
        it, st, tres = int(out["iters"][0]), int(out["status"][0]), float(out["true_rel_res"][0])
        ug = u[0].cpu().numpy()
        true_cpu = np.linalg.norm(f - oracle.stencil_apply(k, ug).numpy()) / r0
        print(f"  {op}: iters {it} (oracle {ref_iters}), true residual {tres:.3e}", flush=True)
        assert st == fc.SYS_OK
        assert abs(tres - true_cpu) <= 1e-8 * max(true_cpu, 1e-300) + 1e-15
        assert true_cpu <= 2e-6
        if op == "fp64":
            assert abs(it - ref_iters) <= 1
        elif op == "fp32":
            assert abs(it - ref_iters) <= max(2, int(0.2 * ref_iters))
        else:
            # BF16 rounding changes the directions: same tolerance reached,
            # iteration count reported (bounded to catch a broken operator)
            assert it <= 2 * ref_iters + 10
        if op == "fp64":
            # the residual history up to the rounding horizon H of the oracle
            # against its own shadow run (1e-16 relative noise on w)
            h = out["hist"][0, :it + 1]
            hr = np.asarray(ref.hist)
            n = min(len(h), len(hr), H + 1)
            rel = np.max(np.abs(h[:n] - hr[:n]) / hr[:n])
            print(f"  fp64 history to the horizon H={H} of {ref_iters}: rel {rel:.2e}", flush=True)
            assert n >= min(ref_iters, 10)
            assert rel <= 1e-10
    model.close()


@pytest.mark.parametrize("m_max", [8, 12])
def test_window_sizes_match_oracle(dev, blob, m_max):
    """Windows of up to 8 vectors (the projection layer forms the window sums
    (w_i, s_k), two window vectors per lane group) and of 12 (the separate
    window-sum kernel): the FP64 residual history follows the oracle's to its
    rounding horizon, past the first full window, and stops at the same
    iteration."""
    N, seed = 32, 9100
    print(f"window m_max={m_max}", flush=True)
    k, f, u0, _ = synth.system(seed, N, (10.0, 100.0))
    w = oracle.unpack_weights(blob, C, M, L)
    kt = torch.from_numpy(k)
    pre = lambda r: oracle.no_apply(w, kt, r)
    ref, H = shadow_horizon(k, f, u0, pre, m_max, 400, 1e-6)
    assert ref.status == oracle.SYS_OK
    model = fc.Model(blob, C, M, L)
    kd, fd = torch.from_numpy(k)[None].to(dev), torch.from_numpy(f)[None].to(dev)
    u = torch.from_numpy(u0)[None].to(dev).contiguous()
    out = fc.solve(model, kd, fd, u, op="fp64", m_max=m_max, max_iter=400, rtol=1e-6)
    it = int(out["iters"][0])
    h = out["hist"][0, :it + 1]
    hr = np.asarray(ref.hist)
    n = min(len(h), len(hr), H + 1)
    rel = np.max(np.abs(h[:n] - hr[:n]) / hr[:n])
    print(f"  iters {it} (oracle {ref.iters}), history to H={H}: rel {rel:.2e}", flush=True)
    assert n >= m_max + 2
    assert rel < 1e-10
    assert abs(it - int(ref.iters)) <= 1
    model.close()


@pytest.mark.parametrize("N", [45, 300])
def test_window_sums_odd_and_ragged_rows(dev, blob, N):
    """The projection layer's window-sum partials on row counts that leave a
    block's last waves without rows (N = 45: 45 one-segment rows, four per
    block) and on ragged two-segment rows (N = 300): 12 FP64 iterations of
    two systems against the oracle's histories up to the rounding horizon."""
    its = 12
    print(f"window sums N={N}", flush=True)
    w = oracle.unpack_weights(blob, C, M, L)
    ks, fs, us = [], [], []
    for seed in (9100, 9101):
        k, f, u0, _ = synth.system(seed, N, (10.0, 100.0))
        ks.append(k); fs.append(f); us.append(u0)
    model = fc.Model(blob, C, M, L)
    kd = torch.from_numpy(np.stack(ks)).to(dev)
    fd = torch.from_numpy(np.stack(fs)).to(dev)
    u = torch.from_numpy(np.stack(us)).to(dev)
    out = fc.solve(model, kd, fd, u, op="fp64", m_max=5, max_iter=its, rtol=1e-300, check_every=4)
    assert np.all(out["iters"] == its)
    for b in range(2):
        kt = torch.from_numpy(ks[b])
        ref, H = shadow_horizon(ks[b], fs[b], us[b], lambda r, kt=kt: oracle.no_apply(w, kt, r), 5, its, 1e-300)
        n = min(H, its) + 1
        rel = np.max(np.abs(out["hist"][b, :n] - np.asarray(ref.hist[:n])) / np.asarray(ref.hist[:n]))
        print(f"  b={b} horizon {H}: rel {rel:.2e}", flush=True)
        assert n >= 8
        assert rel < 1e-10
    model.close()
