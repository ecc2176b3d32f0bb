"""Serving engine (continuous batching) through the C ABI: every request's
result is the same alone and in a mix of grid sizes and arrival times, equals
the batched solve of the same system and the oracle's Algorithm 1 on the same
request (first iterations point by point, up to 1024x1024; converged BF16
requests by the oracle's own residual), and admission respects the pool,
including a large request that is refused for now between small ones."""
import os

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

fc = pytest.importorskip("paper_2402_05598_amd")

C, M = 16, 6


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def model(dev):
    m = fc.Model(synth.init_weights(17, C, M), C, M)
    yield m
    m.close()


def _system(seed, N, dev):
    k, f, u0, _ = synth.system(seed, N, (10.0, 300.0))
    return [torch.from_numpy(a).to(dev) for a in (k, f, u0)]


def _run(engine, jobs, arrivals):
    """jobs: list of (k, f, u); arrivals[i] = engine step before which job i is
    submitted.  Returns {job index: result} and the largest active count."""
    return _run_rtol(engine, jobs, arrivals, 1e-6, 400)


def _run_rtol(engine, jobs, arrivals, rtol, max_iter):
    ids, res, step, peak = {}, {}, 0, 0
    while len(res) < len(jobs):
        for i, a in enumerate(arrivals):
            if a == step and i not in ids.values():
                ids[engine.submit(*jobs[i], rtol=rtol, max_iter=max_iter)] = i
        active, _ = engine.step()
        peak = max(peak, active)
        for r in engine.poll():
            res[ids[r["id"]]] = r
        step += 1
        assert step < 10000
    return res, peak


@pytest.mark.parametrize("op", ["fp64", "bf16", "identity"])
def test_alone_equals_mix_equals_batched_solve(dev, model, op):
    print(f"serving op={op}", flush=True)
    sizes = [32, 48, 64, 40, 64, 96, 32, 128, 48, 64]
    systems = [_system(600 + i, N, dev) for i, N in enumerate(sizes)]
    probe = [0, 5, 7]   # requests compared alone vs in the mix
    alone = {}
    for i in probe:
        k, f, u0 = systems[i]
        eng = fc.Engine(model, op=op, m_max=5, check_every=4, max_slots=8, budget_bytes=1 << 28)
        u = u0.clone()
        res, _ = _run(eng, [(k, f, u)], [0])
        alone[i] = (u.clone(), res[0])
        eng.close()
    eng = fc.Engine(model, op=op, m_max=5, check_every=4, max_slots=6, budget_bytes=1 << 28)
    us = [s[2].clone() for s in systems]
    jobs = [(s[0], s[1], us[i]) for i, s in enumerate(systems)]
    arrivals = [0, 0, 1, 1, 2, 3, 5, 5, 8, 13]
    res, peak = _run(eng, jobs, arrivals)
    eng.close()
    assert peak <= 6
    for i in probe:
        ua, ra = alone[i]
        assert res[i]["status"] == ra["status"] and res[i]["iters"] == ra["iters"]
        assert torch.equal(us[i], ua), f"request {i} differs alone vs in the mix"
        assert res[i]["true_rel_res"] == ra["true_rel_res"]
    # and equal to fcgno_solve on the same system
    for i in range(len(sizes)):
        k, f, u0 = systems[i]
        u = u0.clone()[None].contiguous()
        out = fc.solve(model if op != "identity" else None, k[None].contiguous(), f[None].contiguous(), u,
                       op=op, m_max=5, max_iter=400, rtol=1e-6, hist=False)
        assert int(out["iters"][0]) == res[i]["iters"] and int(out["status"][0]) == res[i]["status"]
        assert torch.equal(u[0], us[i]), f"request {i} differs from the batched solve"
        if res[i]["status"] == 0:
            assert res[i]["true_rel_res"] < 1e-5


def test_admission_by_footprint(dev, model):
    """A pool that holds two 64x64 requests at a time: all complete, never
    more than two active; a request larger than the pool is refused."""
    probe = fc.Engine(model, op="bf16", m_max=5, check_every=4, max_slots=16, budget_bytes=1 << 30)
    per = probe.request_bytes(64, 300)
    probe.close()
    assert per > 0
    budget = int(2.5 * per)
    eng = fc.Engine(model, op="bf16", m_max=5, check_every=4, max_slots=16, budget_bytes=budget)
    systems = [_system(700 + i, 64, dev) for i in range(5)]
    us = [s[2].clone() for s in systems]
    res, peak = _run(eng, [(s[0], s[1], us[i]) for i, s in enumerate(systems)], [0] * 5)
    assert len(res) == 5 and peak == 2
    big = _system(800, 256, dev)
    with pytest.raises(fc.FcgnoError):
        eng.submit(big[0], big[1], big[2].clone())
    eng.close()


def test_refused_admission_leaves_others_intact(dev, model):
    """A pool that holds a 160x160 request alone but not beside a 64x64 one:
    the large request, queued first while a 64x64 one runs, is refused for now
    and hands its group's block back before any work is queued there; the 64x64
    requests behind it are admitted into that space and give the same bits as
    alone; the large request runs once the small ones have left."""
    probe = fc.Engine(model, op="fp64", m_max=5, check_every=4, max_slots=4, budget_bytes=1 << 30)
    r64, r160 = probe.request_bytes(64, 400), probe.request_bytes(160, 400)
    probe.close()
    assert r160 > 4 * r64
    # the large request fits alone (with its group's tables, far below r64 / 4),
    # not beside a 64x64 one, while three 64x64 ones fit together
    budget = r160 + (3 * r64) // 4
    small = [_system(900 + i, 64, dev) for i in range(3)]
    big = _system(950, 160, dev)
    alone = []
    for s_ in small:
        eng = fc.Engine(model, op="fp64", m_max=5, check_every=4, max_slots=4, budget_bytes=budget)
        u = s_[2].clone()
        res, _ = _run(eng, [(s_[0], s_[1], u)], [0])
        alone.append((u, res[0]))
        eng.close()
    eng = fc.Engine(model, op="fp64", m_max=5, check_every=4, max_slots=4, budget_bytes=budget)
    us = [s_[2].clone() for s_ in small]
    ub = big[2].clone()
    # step 0: the first small request occupies the pool; step 1: the big one
    # (refused while the first is active) is queued ahead of the other two
    jobs = [(small[0][0], small[0][1], us[0]), (big[0], big[1], ub),
            (small[1][0], small[1][1], us[1]), (small[2][0], small[2][1], us[2])]
    res, peak = _run(eng, jobs, [0, 1, 1, 1])
    eng.close()
    for j, i in ((0, 0), (2, 1), (3, 2)):
        assert torch.equal(us[i], alone[i][0]), f"small request {i} differs from its alone run"
        assert res[j]["iters"] == alone[i][1]["iters"]
    eng1 = fc.Engine(model, op="fp64", m_max=5, check_every=4, max_slots=4, budget_bytes=budget)
    ub1 = big[2].clone()
    rb, _ = _run(eng1, [(big[0], big[1], ub1)], [0])
    eng1.close()
    assert torch.equal(ub, ub1) and res[1]["iters"] == rb[0]["iters"]


@pytest.mark.parametrize("N", [64, 130, 1024])
def test_engine_first_iterations_match_oracle(dev, model, N):
    """FP64 engine requests stopped after six iterations (rtol below reach):
    the returned iterate's increment u - u0 against the oracle's Algorithm 1
    with the same operator, point by point, and the reported true residual
    against the oracle's.  1024x1024 runs the layer kernel's two-segment rows."""
    print(f"engine vs oracle N={N}", flush=True)
    its = 6
    k, f, u0 = _system(1000 + N, N, dev)
    kn, fn, un = (a.cpu().numpy() for a in (k, f, u0))
    w = oracle.unpack_weights(synth.init_weights(17, C, M), C, M)
    kt = torch.from_numpy(kn)
    ref = oracle.fcg(kn, fn, un, lambda r: oracle.no_apply(w, kt, r), m_max=5, max_iter=its, tol=1e-300)
    eng = fc.Engine(model, op="fp64", m_max=5, check_every=4, max_slots=4, budget_bytes=3 << 30)
    u = u0.clone()
    res, _ = _run_rtol(eng, [(k, f, u)], [0], 1e-300, its)
    eng.close()
    assert res[0]["iters"] == its and res[0]["status"] == fc.SYS_NOT_CONVERGED
    du_g = u.cpu().numpy() - un
    du_o = ref.u.numpy() - un
    mx = np.max(np.abs(du_g - du_o)) / np.max(np.abs(du_o))
    tr = abs(res[0]["true_rel_res"] - ref.true_rel_res) / ref.true_rel_res
    print(f"  increment max diff {mx:.2e}, true residual diff {tr:.2e}", flush=True)
    assert mx < 1e-9
    assert tr < 1e-9


TRAINED = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "weights",
                       "bench_operator_c32_m12_l4.npy")


@pytest.mark.skipif(not os.path.exists(TRAINED), reason="trained operator blob not present")
def test_engine_bf16_converged_requests_by_oracle_residual(dev):
    """Converged BF16 requests of several grid sizes, with the trained operator
    (width 32, 12 modes; a random-initial operator does not converge): the
    oracle's stencil gives ||f - A u|| / ||f - A u0|| <= 1e-6 (up to rounding)
    on the returned iterate, equal to the reported true residual."""
    sizes = [32, 64, 96, 128]
    systems = [_system(1100 + i, N, dev) for i, N in enumerate(sizes)]
    model = fc.Model(np.load(TRAINED).astype(np.float64), 32, 12)
    eng = fc.Engine(model, op="bf16", m_max=5, check_every=4, max_slots=8, budget_bytes=1 << 29)
    us = [s_[2].clone() for s_ in systems]
    res, _ = _run(eng, [(s_[0], s_[1], us[i]) for i, s_ in enumerate(systems)], [0, 0, 1, 2])
    eng.close()
    model.close()
    n_ok = 0
    for i, (k, f, u0) in enumerate(systems):
        kn, fn, un = (a.cpu().numpy() for a in (k, f, u0))
        r0 = np.linalg.norm(fn - oracle.stencil_apply(kn, un).numpy())
        true = np.linalg.norm(fn - oracle.stencil_apply(kn, us[i].cpu().numpy()).numpy()) / r0
        print(f"  N={sizes[i]} status {res[i]['status']} iters {res[i]['iters']} true {true:.3e}", flush=True)
        assert abs(res[i]["true_rel_res"] - true) <= 1e-8 * true
        if res[i]["status"] == fc.SYS_OK:
            n_ok += 1
            assert true <= 1.5e-6
    assert n_ok >= 2
