"""Classical preconditioners of Table 1 inside the GPU FCG, against the CPU
oracle: Jacobi(k) and symmetric Gauss-Seidel(k) in red-black order (Sec. 3.3.1),
each k sweeps from x_0 = 0 on A x = r_i.  The first iterate checks the
application itself element by element; full solves compare residual histories
up to the rounding horizon and the stopping iteration within the oracle's own
shadow spread.  Grids cover several 256-point blocks, odd sizes (ragged rows of
the red-black pairing) and batches of distinct systems."""
import numpy as np
import pytest
import torch

import oracle
import synth
from _parity import iteration_tolerance, shadow_runs

pytestmark = pytest.mark.gpu

fc = pytest.importorskip("paper_2402_05598_amd")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _oracle_precond(k, op, steps):
    return oracle.jacobi_precond(k, steps) if op == "jacobi" else oracle.rb_sgs_precond(k, steps)


def _batch(seeds, N, dev):
    ks, fs, us = zip(*[synth.diffusion_system(s, N) for s in seeds])
    return ks, fs, us, [torch.from_numpy(np.stack(a)).to(dev).contiguous() for a in (ks, fs, us)]


@pytest.mark.parametrize("op", ["jacobi", "sgs_rb"])
@pytest.mark.parametrize("N,steps", [(1, 1), (2, 3), (17, 1), (24, 2), (33, 4), (64, 1)])
def test_first_iterate_matches_oracle(dev, op, N, steps):
    """u_1 = u_0 + alpha_0 B(r_0): checks B element by element (and alpha)."""
    print(f"classical first iterate op={op} N={N} steps={steps}", flush=True)
    seeds = [300 + N, 301 + N, 302 + N]
    ks, fs, us, (kd, fd, ud) = _batch(seeds, N, dev)
    out = fc.solve(None, kd, fd, ud, op=op, m_max=5, max_iter=1, rtol=1e-300, precond_steps=steps)
    got = ud.cpu().numpy()
    for b in range(len(seeds)):
        ref = oracle.fcg(ks[b], fs[b], us[b], _oracle_precond(ks[b], op, steps), m_max=5, max_iter=1, tol=1e-300)
        assert int(out["iters"][b]) == ref.iters == 1
        du_ref = np.asarray(ref.u) - us[b]
        du_got = got[b] - us[b]
        err = np.max(np.abs(du_got - du_ref)) / np.max(np.abs(du_ref))
        assert err <= 1e-11, (b, err)


@pytest.mark.parametrize("op,steps", [("jacobi", 4), ("sgs_rb", 1), ("sgs_rb", 4)])
@pytest.mark.parametrize("N", [32, 45])
def test_solve_matches_oracle(dev, op, steps, N):
    """Table 1's setting (m_max = 20, stop at 1e-6): the GPU history follows
    the oracle's up to the rounding horizon and stops within its shadow spread."""
    print(f"classical solve op={op} steps={steps} N={N}", flush=True)
    seeds = [400 + N, 401 + N]
    ks, fs, us, (kd, fd, ud) = _batch(seeds, N, dev)
    out = fc.solve(None, kd, fd, ud, op=op, m_max=20, max_iter=1000, rtol=1e-6, precond_steps=steps)
    for b in range(len(seeds)):
        B = _oracle_precond(ks[b], op, steps)
        ref, H, its = shadow_runs(ks[b], fs[b], us[b], B, 20, 1000, 1e-6, n_shadow=3)
        assert ref.status == oracle.SYS_OK
        it = int(out["iters"][b])
        print(f"  system {b}: iters gpu {it} oracle {ref.iters} shadows {its} horizon {H}", flush=True)
        assert int(out["status"][b]) == fc.SYS_OK
        assert abs(it - ref.iters) <= iteration_tolerance(ref.iters, its)
        h = out["hist"][b, :min(it, ref.iters) + 1]
        hr = np.asarray(ref.hist)[:len(h)]
        n = max(2, min(H + 1, len(h)))
        assert np.max(np.abs(h[:n] - hr[:n]) / hr[:n]) <= 1e-9
        assert float(out["true_rel_res"][b]) <= 2e-6


def test_batch_members_are_independent(dev):
    """A system's solve does not depend on the other systems of the batch."""
    N = 40
    ks, fs, us, (kd, fd, ud) = _batch([510, 511, 512], N, dev)
    out = fc.solve(None, kd, fd, ud, op="sgs_rb", m_max=20, max_iter=500, rtol=1e-6, precond_steps=2)
    k1, f1, u1 = kd[1:2].contiguous(), fd[1:2].contiguous(), torch.from_numpy(us[1])[None].to(dev).contiguous()
    one = fc.solve(None, k1, f1, u1, op="sgs_rb", m_max=20, max_iter=500, rtol=1e-6, precond_steps=2)
    assert int(one["iters"][0]) == int(out["iters"][1])
    assert torch.equal(u1[0], ud[1])


def test_table1_counts_on_a_poisson_system(dev):
    """Table 1's columns on one Poisson system at grid 64 (m_max = 20): the GPU
    counts equal the oracle's, more sweeps give fewer iterations, and red-black
    SGS(1) needs more iterations than the lexicographic GS(1) of the paper (the
    price of the parallel ordering) while SGS(4) still beats Jacobi(4)."""
    N = 64
    k, f, u0 = synth.poisson_system(6401, N)
    kd, fd = torch.from_numpy(k)[None].to(dev), torch.from_numpy(f)[None].to(dev)
    methods = [("CG", "identity", 1, None), ("Jacobi(4)", "jacobi", 4, oracle.jacobi_precond(k, 4)),
               ("RB-SGS(1)", "sgs_rb", 1, oracle.rb_sgs_precond(k, 1)),
               ("RB-SGS(4)", "sgs_rb", 4, oracle.rb_sgs_precond(k, 4))]
    gpu, ref = {}, {}
    for name, op, steps, B in methods:
        u = torch.from_numpy(u0)[None].to(dev).contiguous()
        out = fc.solve(None, kd, fd, u, op=op, m_max=20, max_iter=2000, rtol=1e-6, precond_steps=steps, hist=False)
        assert int(out["status"][0]) == fc.SYS_OK
        gpu[name] = int(out["iters"][0])
        ref[name] = oracle.fcg(k, f, u0, B, m_max=20, max_iter=2000, tol=1e-6).iters
    lex1 = oracle.fcg(k, f, u0, oracle.sgs_precond(k, 1), m_max=20, max_iter=2000, tol=1e-6).iters
    print(f"gpu {gpu} oracle {ref} lexicographic GS(1) {lex1}", flush=True)
    for name in gpu:
        assert abs(gpu[name] - ref[name]) <= 2, name
    assert gpu["CG"] > gpu["RB-SGS(1)"] > gpu["RB-SGS(4)"]
    assert gpu["CG"] > gpu["Jacobi(4)"] > gpu["RB-SGS(4)"]
    assert ref["RB-SGS(1)"] > lex1
