"""The Python binding refuses mis-shaped arguments before any pointer reaches
the library (host-only: the checks run ahead of every device call, so CPU
tensors suffice)."""
import pytest
import torch

import paper_2402_05598_amd._binding as b


class _NoModel:
    handle = None
    n_weights = 1


def _f(*shape):
    return torch.zeros(shape, dtype=torch.float64)


B, N = 2, 16
GOOD_K, GOOD_F = _f(B, N + 2, N + 2), _f(B, N, N)

CASES = [
    ("solve f not square", lambda: b.solve(None, GOOD_K, _f(B, N, N + 1), GOOD_F, op="identity")),
    ("solve f 2-d", lambda: b.solve(None, GOOD_K, _f(N, N), GOOD_F, op="identity")),
    ("solve k", lambda: b.solve(None, _f(B, N, N), GOOD_F, GOOD_F, op="identity")),
    ("solve u", lambda: b.solve(None, GOOD_K, GOOD_F, _f(B + 1, N, N), op="identity")),
    ("solve r_out", lambda: b.solve(None, GOOD_K, GOOD_F, GOOD_F, op="identity", r_out=_f(B, N, N - 1))),
    ("precond r", lambda: b.precond_apply(_NoModel(), GOOD_K, _f(B, N, 3))),
    ("precond k", lambda: b.precond_apply(_NoModel(), _f(B, N + 1, N + 2), GOOD_F)),
    ("precond w", lambda: b.precond_apply(_NoModel(), GOOD_K, GOOD_F, w=_f(B, N, N + 2))),
    ("op_forward k", lambda: b.op_forward(_NoModel(), _f(B, N, N), GOOD_F)),
    ("op_forward r", lambda: b.op_forward(_NoModel(), GOOD_K, _f(B, N))),
    ("op_backward k", lambda: b.op_backward(_NoModel(), _f(1, N + 2, N + 2), GOOD_F, GOOD_F, None)),
    ("op_backward grad_w", lambda: b.op_backward(_NoModel(), GOOD_K, GOOD_F, _f(B, N * N), None)),
    ("energy_loss k", lambda: b.energy_loss(_f(B, N, N), GOOD_F, GOOD_F)),
    ("energy_loss e", lambda: b.energy_loss(GOOD_K, GOOD_F, _f(B, N, N + 1))),
    ("train_step k", lambda: b.train_step(_NoModel(), None, _f(B, N + 2, N + 3), GOOD_F, GOOD_F)),
    ("train_step e", lambda: b.train_step(_NoModel(), None, GOOD_K, GOOD_F, _f(B + 1, N, N))),
    ("residual_samples u", lambda: b.residual_samples(GOOD_K, GOOD_F, _f(B, N - 1, N - 1))),
    ("krylov_samples k", lambda: b.krylov_samples(_f(B + 1, N + 2, N + 2), GOOD_F, GOOD_F)),
    ("krylov_samples f", lambda: b.krylov_samples(GOOD_K, _f(B, N, N, 1), GOOD_F)),
]


@pytest.mark.parametrize("name,call", CASES, ids=[c[0] for c in CASES])
def test_misshaped_arguments_are_refused(name, call):
    with pytest.raises(b.FcgnoError, match="shape"):
        call()


def test_correct_shapes_reach_the_device_check():
    """With every shape right, host tensors are refused as host tensors (the
    next check), so the shape checks above are not over-strict."""
    with pytest.raises(b.FcgnoError, match="device tensor"):
        b.energy_loss(GOOD_K, GOOD_F, GOOD_F, grad=False)
