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
