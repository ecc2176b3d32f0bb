"""Sub-batched solves (the solve descriptor's streams field): the batch split
over library-owned streams gives the same bits as one stream -- iterate,
iteration counts, statuses, histories and true residuals -- for the neural
operator in BF16 and FP64, CG and red-black SGS, with uneven sub-batches, a
system stopped at the start (zero right-hand side) and more streams asked
for than systems."""
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
    m = fc.Model(synth.init_weights(23, C, M), C, M)
    yield m
    m.close()


@pytest.mark.parametrize("op", ["bf16", "fp64", "identity", "sgs_rb"])
@pytest.mark.parametrize("N,B", [(48, 7), (128, 12)])
def test_streams_give_identical_results(dev, model, op, N, B):
    print(f"streams op={op} N={N} B={B}", flush=True)
    k, f, u0, _ = synth.batch(7, B, N, (10.0, 300.0))
    f[2] = 0.0   # with u0 = 0: r0 = 0, stops before the first iteration
    u0[2] = 0.0
    kd, fd = torch.from_numpy(k).to(dev), torch.from_numpy(f).to(dev)
    mdl = model if op in ("bf16", "fp64") else None
    runs = {}
    for streams in (0, 3, 4, 8):
        u = torch.from_numpy(u0).to(dev)
        out = fc.solve(mdl, kd, fd, u, op=op, m_max=5, max_iter=300, rtol=1e-6, streams=streams,
                       precond_steps=2, check_every=4)
        runs[streams] = (u.cpu().numpy(), out)
    u_ref, ref = runs[0]
    assert ref["status"][2] == fc.SYS_OK and ref["iters"][2] == 0
    for streams, (u, out) in runs.items():
        assert np.array_equal(u, u_ref), streams
        assert np.array_equal(out["iters"], ref["iters"]), streams
        assert np.array_equal(out["status"], ref["status"]), streams
        assert np.array_equal(out["true_rel_res"], ref["true_rel_res"]), streams
        assert np.array_equal(np.nan_to_num(out["hist"], nan=-1.0), np.nan_to_num(ref["hist"], nan=-1.0)), streams
