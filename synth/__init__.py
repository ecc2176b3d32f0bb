"""Seeded synthetic inputs for FCG-NO solves.

This module is the only code shared by the HIP product path and the CPU
oracle.  It draws random fields and random weights and nothing else: it holds
none of the method's arithmetic (no stencil, no Krylov step, no operator).

Grid convention (read of the problem statement in Sec. 2.1, eq. for the
general elliptic equation): ``N`` interior points per side of the unit square,
mesh width ``h = 1/(N+1)``.  Interior arrays are ``[N][N]`` indexed ``[i][j]``
with ``i`` along x1 and ``j`` along x2 (``j`` contiguous).  Coefficient fields
are nodal, ``[N+2][N+2]``, boundary nodes included, node ``(i+1, j+1)`` being
interior point ``(i, j)``.

Workload recipe (the paper's own experiments use random trigonometric
polynomials, Sec. 3.2; the solver workloads here use Gaussian random fields):

* ``k = exp(g)`` with ``g`` a Gaussian random field with squared-exponential
  covariance (length scale 0.1, variance 1) sampled on the nodes;  with a
  contrast ``c`` the exponent is rescaled so that ``k`` spans ``[1, c]``.
* ``f`` is an independent GRF on the interior nodes.
* ``u0 ~ N(0, I)`` as in Algorithm 1's initialisation.
* draw order per system: g_k, g_f, u0, contrast.
* seed of system ``s`` in workload ``w``: ``1000 * w + s`` (numpy PCG64).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "grf", "coefficient_field", "rhs_field", "initial_guess", "system",
    "batch", "init_weights", "weight_count", "trig_poly", "poisson_system",
    "diffusion_system", "rng",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def grf(g: np.random.Generator, n: int, h: float, ell: float = 0.1,
        var: float = 1.0) -> np.ndarray:
    """One sample of a stationary Gaussian field on an ``n x n`` lattice of
    spacing ``h`` with covariance ``var * exp(-d^2 / (2 ell^2))``.

    Circulant embedding on a ``2n x 2n`` torus; tiny negative embedding
    eigenvalues are clipped to zero.  Returns float64 ``[n][n]``.
    """
    m = 2 * n
    idx = np.arange(m)
    d = np.minimum(idx, m - idx) * h
    cov = var * np.exp(-(d[:, None] ** 2 + d[None, :] ** 2) / (2.0 * ell * ell))
    lam = np.maximum(np.fft.fft2(cov).real, 0.0)
    xi = g.standard_normal((m, m)) + 1j * g.standard_normal((m, m))
    z = np.fft.fft2(np.sqrt(lam / (m * m)) * xi)
    return np.ascontiguousarray(z.real[:n, :n])


def coefficient_field(g: np.random.Generator, N: int, contrast: float | None = None,
                      ell: float = 0.1) -> np.ndarray:
    """Nodal coefficient ``[N+2][N+2]``: ``exp(GRF)``, or with ``contrast`` the
    exponent rescaled to ``[-ln(contrast)/2, ln(contrast)/2]``."""
    h = 1.0 / (N + 1)
    gk = grf(g, N + 2, h, ell)
    if contrast is None:
        return np.exp(gk)
    lo, hi = gk.min(), gk.max()
    t = (gk - lo) / (hi - lo)
    return np.exp(np.log(contrast) * (t - 0.5))


def rhs_field(g: np.random.Generator, N: int, ell: float = 0.1) -> np.ndarray:
    h = 1.0 / (N + 1)
    return grf(g, N, h, ell)


def initial_guess(g: np.random.Generator, N: int) -> np.ndarray:
    return g.standard_normal((N, N))


def system(seed: int, N: int, contrast_range: tuple[float, float] | None = None):
    """One seeded system ``(k, f, u0, contrast)``.

    With ``contrast_range=(lo, hi)`` the contrast c is log-uniform in it and is
    drawn after u0 (so ``k`` is built last from the stored GRF sample); the
    GRF exponent is rescaled so that k spans [c^-1/2, c^1/2] (ratio c,
    geometric midpoint 1)."""
    g = rng(seed)
    h = 1.0 / (N + 1)
    gk = grf(g, N + 2, h)
    f = grf(g, N, h)
    u0 = g.standard_normal((N, N))
    if contrast_range is None:
        return np.exp(gk), f, u0, None
    lo, hi = contrast_range
    c = float(np.exp(g.uniform(np.log(lo), np.log(hi))))
    t = (gk - gk.min()) / (gk.max() - gk.min())
    return np.exp(np.log(c) * (t - 0.5)), f, u0, c


def batch(workload: int, B: int, N: int, contrast_range=None, first: int = 0):
    """``B`` systems with seeds ``1000*workload + first + s``; returns stacked
    float64 arrays ``k [B][N+2][N+2]``, ``f [B][N][N]``, ``u0 [B][N][N]`` and
    the list of contrasts."""
    ks, fs, us, cs = [], [], [], []
    for s in range(B):
        k, f, u0, c = system(1000 * workload + first + s, N, contrast_range)
        ks.append(k); fs.append(f); us.append(u0); cs.append(c)
    return (np.ascontiguousarray(np.stack(ks)), np.ascontiguousarray(np.stack(fs)),
            np.ascontiguousarray(np.stack(us)), cs)


# ---------------------------------------------------------------------------
# Operator weights.  Blob order (float64): W_L[C][Cin], b_L[C], then for each
# layer Re R[C][C][2M][M], Im R[C][C][2M][M], W[C][C], b[C], then W_P[C], b_P[1].
# ---------------------------------------------------------------------------

def weight_count(C: int, M: int, L: int = 4, Cin: int = 4) -> int:
    per_layer = 2 * C * C * 2 * M * M + C * C + C
    return C * Cin + C + L * per_layer + C + 1


def init_weights(seed: int, C: int, M: int, L: int = 4, Cin: int = 4) -> np.ndarray:
    """Seeded random initialisation, drawn in blob order:
    lift ~ U(+-1/sqrt(Cin)); spectral Re/Im ~ U[0,1)/C^2; bypass, biases and
    projection ~ U(+-1/sqrt(C))."""
    g = rng(seed)
    out = []
    a = 1.0 / np.sqrt(Cin)
    out.append(g.uniform(-a, a, C * Cin))
    out.append(g.uniform(-a, a, C))
    a = 1.0 / np.sqrt(C)
    nR = C * C * 2 * M * M
    for _ in range(L):
        out.append(g.random(nR) / (C * C))
        out.append(g.random(nR) / (C * C))
        out.append(g.uniform(-a, a, C * C))
        out.append(g.uniform(-a, a, C))
    out.append(g.uniform(-a, a, C))
    out.append(g.uniform(-a, a, 1))
    blob = np.concatenate(out)
    assert blob.size == weight_count(C, M, L, Cin)
    return blob


# ---------------------------------------------------------------------------
# The paper's data sets (Sec. 3.2): random trigonometric polynomials.
# ---------------------------------------------------------------------------

def trig_poly(g: np.random.Generator, x1: np.ndarray, x2: np.ndarray,
              N1: int = 5, N2: int = 5, alpha: float = 2.0) -> np.ndarray:
    """Real part of sum_{m<=N1, n<=N2} c_mn exp(2 pi i (m x1 + n x2)) / (1+m+n)^alpha
    with c_mn i.i.d. complex standard normal, evaluated on the mesh x1 (x) x2."""
    c = g.standard_normal((N1 + 1, N2 + 1)) + 1j * g.standard_normal((N1 + 1, N2 + 1))
    m = np.arange(N1 + 1)[:, None]
    n = np.arange(N2 + 1)[None, :]
    c = c / (1.0 + m + n) ** alpha
    e1 = np.exp(2j * np.pi * np.outer(x1, np.arange(N1 + 1)))  # [X1][m]
    e2 = np.exp(2j * np.pi * np.outer(x2, np.arange(N2 + 1)))  # [X2][n]
    return np.real(e1 @ c @ e2.T)


def poisson_system(seed: int, N: int):
    """Poisson data set: a = 1, f ~ P(5,5,2); u0 ~ N(0,I)."""
    g = rng(seed)
    h = 1.0 / (N + 1)
    xi = (np.arange(N) + 1) * h
    f = trig_poly(g, xi, xi)
    k = np.ones((N + 2, N + 2))
    u0 = g.standard_normal((N, N))
    return k, f, u0


def diffusion_system(seed: int, N: int):
    """Diffusion data set: a ~ P(5,5,2) + 10 on the nodes, f ~ P(5,5,2); u0 ~ N(0,I)."""
    g = rng(seed)
    h = 1.0 / (N + 1)
    xn = np.arange(N + 2) * h
    k = trig_poly(g, xn, xn) + 10.0
    xi = (np.arange(N) + 1) * h
    f = trig_poly(g, xi, xi)
    u0 = g.standard_normal((N, N))
    return k, f, u0
