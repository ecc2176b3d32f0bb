"""The scratch-free operator application (fcgno_precond_apply_noalloc) against
fcgno_precond_apply on the same inputs, through the C ABI: the same kernels
run on the library's static scratch array, so the outputs must agree bit for
bit.  Two calls in a row, the second smaller, check that what an earlier call
left in the shared array does not leak into a later one; a size beyond the
array is refused before any launch."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests._parity import assert_operator_close

pytestmark = pytest.mark.gpu

fc = pytest.importorskip("paper_2402_05598_amd")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _inputs(dev, seed, N, B):
    k, f, _, _ = synth.batch(seed, B, N, (10.0, 1000.0))
    return [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (k, f)]


def test_noalloc_matches_workspace_entry_point(dev):
    C, M = 32, 12
    wb = synth.init_weights(77, C, M)
    model = fc.Model(wb, C, M)
    # larger call first, then a smaller one over the same scratch array
    for N, B, op in ((250, 4, "bf16"), (250, 4, "fp32"), (96, 2, "bf16"), (70, 3, "fp64"), (40, 1, "fp32")):
        print(f"noalloc N={N} B={B} op={op}", flush=True)
        k, r = _inputs(dev, 900 + N, N, B)
        ref = fc.precond_apply(model, k, r, op=op)
        got = fc.precond_apply_noalloc(model, k, r, op=op)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (N, B, op, (got - ref).abs().max().item())
        got2 = fc.precond_apply_noalloc(model, k, r, op=op)
        torch.cuda.synchronize()
        assert torch.equal(got2, ref), (N, B, op, "second call")
    # the oracle on one system of the last, smallest call
    wo = oracle.unpack_weights(wb, C, M)
    want = oracle.no_apply(wo, k[0].cpu(), r[0].cpu()).numpy()
    assert_operator_close(got[0].cpu().numpy(), want, "fp32", "noalloc N=40")
    model.close()


def test_noalloc_refuses_sizes_beyond_the_array(dev):
    C, M = 32, 12
    model = fc.Model(synth.init_weights(78, C, M), C, M)
    N = 1024
    need = fc.lib().fcgno_precond_workspace_bytes(model.handle, N, 1, fc.OP["fp64"])
    assert need > fc._binding.NOALLOC_SCRATCH_BYTES
    k = torch.ones(1, N + 2, N + 2, dtype=torch.float64, device=dev)
    r = torch.ones(1, N, N, dtype=torch.float64, device=dev)
    w = torch.full_like(r, 7.0)
    with pytest.raises(fc.FcgnoError, match="static array"):
        fc.precond_apply_noalloc(model, k, r, op="fp64", w=w)
    assert bool((w == 7.0).all())   # nothing was launched
    with pytest.raises(fc.FcgnoError, match="batch"):
        kb = torch.ones(65, 34, 34, dtype=torch.float64, device=dev)
        fc.precond_apply_noalloc(model, kb, torch.ones(65, 32, 32, dtype=torch.float64, device=dev), op="bf16")
    model.close()
