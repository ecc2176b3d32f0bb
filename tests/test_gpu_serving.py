"""Serving engine (continuous batching) through the C ABI: every request's
result is the same alone and in a mix of grid sizes and arrival times, equals
the batched solve of the same system, and admission respects the pool."""
import numpy as np
import pytest
import torch

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
    ids, res, step, peak = {}, {}, 0, 0
    while len(res) < len(jobs):
        for i, a in enumerate(arrivals):
            if a == step and i not in ids.values():
                ids[engine.submit(*jobs[i], rtol=1e-6, max_iter=400)] = i
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
