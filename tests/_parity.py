"""Helpers for GPU-vs-oracle parity: the rounding horizon of a solve.

Rounding differences in FCG grow chaotically once the preconditioner is poor,
so two correct implementations that sum in different orders agree only up to
a horizon, and their stopping iterations scatter.  Both are measured on the
oracle itself: shadows of the oracle run with w_i perturbed by 1e-16 relative
seeded noise."""
import numpy as np
import torch

import oracle


def shadow_runs(k, f, u0, precond, m_max, max_iter, tol, n_shadow=4, agree=1e-12, ref=None):
    """Returns (reference result, H, shadow iteration counts).  H is the last
    iteration at which the first shadow's residual history agrees with the
    reference to ``agree`` relative."""
    if ref is None:
        ref = oracle.fcg(k, f, u0, precond, m_max=m_max, max_iter=max_iter, tol=tol)
    H = None
    its = []
    for s in range(n_shadow):
        g = np.random.default_rng(1234 + s)

        def hook(i, w, g=g):
            return w * (1.0 + 1e-16 * torch.from_numpy(g.standard_normal(tuple(w.shape))))
        sh = oracle.fcg(k, f, u0, precond, m_max=m_max, max_iter=max_iter, tol=tol, w_hook=hook)
        its.append(sh.iters)
        if H is None:
            a, b = np.array(ref.hist), np.array(sh.hist)
            n = min(len(a), len(b))
            rel = np.abs(a[:n] - b[:n]) / np.maximum(np.abs(a[:n]), 1e-300)
            bad = np.nonzero(rel > agree)[0]
            H = int(bad[0] - 1) if bad.size else n - 1
    return ref, H, its


def shadow_horizon(k, f, u0, precond, m_max, max_iter, tol, agree=1e-12, ref=None):
    ref, H, _ = shadow_runs(k, f, u0, precond, m_max, max_iter, tol, n_shadow=1, agree=agree, ref=ref)
    return ref, H


def iteration_tolerance(ref_iters, shadow_iters):
    """Allowed |gpu - oracle| stopping-iteration difference: 1.5x the spread of
    the oracle's own shadows, at least 2."""
    allits = list(shadow_iters) + [ref_iters]
    return max(2.0, 1.5 * (max(allits) - min(allits)))


# Operator parity bounds per precision.  FP64: about ten times the measured
# ~1e-16 error against the oracle.  FP32: 16 unit roundoffs of float32
# (u = 6e-8), 1e-6 in the norm and 3e-6 point by point; the measured errors
# are 3e-8 (Fourier basis) to 3e-7 (sine basis, whose twiddles carry more
# float32 rounding).  BF16: about ten times the measured 1.5e-4..8e-4.  Each
# system is checked in the relative 2-norm and point by point, the largest
# absolute difference against the largest value, so that one bad tile or a
# wrong ragged-edge row cannot hide in the norm.
NORM_TOL = {"fp64": 1e-13, "fp32": 1e-6, "bf16": 3e-3}
MAX_TOL = {"fp64": 1e-13, "fp32": 3e-6, "bf16": 5e-3}


def assert_operator_close(got, ref, op, label="", scale=1.0):
    """got, ref: numpy [N][N] (one system).  Prints and asserts both measures;
    ``scale`` widens both bounds for a case whose weights amplify rounding."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    assert np.all(np.isfinite(got)), f"{label} {op}: non-finite output"
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    mx = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    # worst row, to name a bad tile or edge
    row = int(np.argmax(np.max(np.abs(got - ref), axis=1)))
    print(f"  {label} {op}: rel2 {rel:.2e} max {mx:.2e} (worst row {row})", flush=True)
    assert rel < scale * NORM_TOL[op], (label, op, "rel2", rel)
    assert mx < scale * MAX_TOL[op], (label, op, "max", mx, row)
