"""FP64 CPU oracle of the FCG-NO hot path.  TEST INFRASTRUCTURE ONLY: it may be
imported by tests, by the smoke check and by the CPU-baseline leg of the bench,
never by the product path.

Readings of the paper where it is silent (each is also listed in the design
notes of the repository):
  * grid: N interior points per side, h = 1/(N+1), nodal coefficient k on the
    (N+2)^2 nodes including the boundary;
  * 5-point finite differences with arithmetic-mean face coefficients, scaled
    by 1/h^2 (the problem statement of Sec. 2.1 allows FD or FEM);
  * the operator sees k: features [r/s, log k, x1, x2] with s = ||r||_2/sqrt(n),
    and its output is multiplied back by s, so B(c r) = c B(r) for c > 0;
  * Fourier layers keep kx in {0..M-1} U {N-M..N-1} and ky in {0..M-1}, with an
    unnormalised forward DFT and a 1/N^2 inverse; exact-erf GELU after every
    layer; single linear lift (4 -> C) and projection (C -> 1);
  * stop at the first i with ||r_i||/||r_0|| <= tol on the recurrence residual;
    (p, s) <= 0 or non-finite is a breakdown that freezes the system.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
import torch

__all__ = [
    "SYS_OK", "SYS_NOT_CONVERGED", "SYS_BREAKDOWN", "SYS_NONFINITE",
    "stencil_apply", "assemble", "window_size", "fcg", "FCGResult",
    "NOWeights", "unpack_weights", "pack_weights", "no_apply", "no_features",
    "energy_norm", "notay_loss", "l2_loss", "krylov_samples", "exact_solve",
    "jacobi_precond", "sgs_precond", "red_black_order", "rb_sgs_precond", "adamw_step", "gelu",
    "sine_matrix",
]

SYS_OK, SYS_NOT_CONVERGED, SYS_BREAKDOWN, SYS_NONFINITE = 0, 1, 2, 3

_f64 = torch.float64


def _t(x):
    if isinstance(x, torch.Tensor):
        return x.to(_f64)
    return torch.as_tensor(np.asarray(x), dtype=_f64)


# ---------------------------------------------------------------------------
# The discrete operator A (Sec. 2.1, the general elliptic equation and the
# linear system it yields).  Reading: 5-point finite differences, nodal k,
# arithmetic-mean faces, zero Dirichlet values outside the interior, 1/h^2.
# ---------------------------------------------------------------------------

def stencil_apply(k, u):
    """(A u)_ij = h^-2 [ (kE+kW+kN+kS) u_ij - kE u_{i+1,j} - kW u_{i-1,j}
                          - kN u_{i,j+1} - kS u_{i,j-1} ]
    with kE = (k_node(i,j) + k_node(i+1,j)) / 2 etc. and u = 0 off the interior.
    ``k``: [..., N+2, N+2] nodal; ``u``: [..., N, N]."""
    k = _t(k)
    u = _t(u)
    N = u.shape[-1]
    h2 = 1.0 / float(N + 1) ** 2
    kc = k[..., 1:-1, 1:-1]
    kE = 0.5 * (kc + k[..., 2:, 1:-1])
    kW = 0.5 * (kc + k[..., :-2, 1:-1])
    kN = 0.5 * (kc + k[..., 1:-1, 2:])
    kS = 0.5 * (kc + k[..., 1:-1, :-2])
    up = torch.nn.functional.pad(u, (1, 1, 1, 1))
    uE = up[..., 2:, 1:-1]
    uW = up[..., :-2, 1:-1]
    uN = up[..., 1:-1, 2:]
    uS = up[..., 1:-1, :-2]
    return ((kE + kW + kN + kS) * u - kE * uE - kW * uW - kN * uN - kS * uS) / h2


def assemble(k) -> sp.csr_matrix:
    """Explicit sparse matrix of the same operator, row (i*N + j)."""
    k = np.asarray(k, dtype=np.float64)
    N = k.shape[-1] - 2
    h2 = 1.0 / float(N + 1) ** 2
    rows, cols, vals = [], [], []
    for i in range(N):
        for j in range(N):
            c = k[i + 1, j + 1]
            nb = [((i + 1, j), 0.5 * (c + k[i + 2, j + 1])),
                  ((i - 1, j), 0.5 * (c + k[i, j + 1])),
                  ((i, j + 1), 0.5 * (c + k[i + 1, j + 2])),
                  ((i, j - 1), 0.5 * (c + k[i + 1, j]))]
            diag = 0.0
            for (a, b), kf in nb:
                diag += kf
                if 0 <= a < N and 0 <= b < N:
                    rows.append(i * N + j); cols.append(a * N + b); vals.append(-kf / h2)
            rows.append(i * N + j); cols.append(i * N + j); vals.append(diag / h2)
    return sp.csr_matrix((vals, (rows, cols)), shape=(N * N, N * N))


def exact_solve(k, f):
    """u* = A^-1 f by a sparse direct solve (library primitive)."""
    A = assemble(k)
    f = np.asarray(f, dtype=np.float64)
    N = f.shape[-1]
    return spla.spsolve(A.tocsc(), f.reshape(-1)).reshape(N, N)


# ---------------------------------------------------------------------------
# Flexible conjugate gradients, Algorithm 1.
# ---------------------------------------------------------------------------

def window_size(i: int, m_max: int) -> int:
    """m_i = min(i, max(1, i mod (m_max + 1)))  (Algorithm 1)."""
    return min(i, max(1, i % (m_max + 1)))


@dataclass
class FCGResult:
    u: torch.Tensor
    r: torch.Tensor
    iters: int
    status: int
    hist: list = field(default_factory=list)     # ||r_i|| / ||r_0||, i = 0..iters
    true_rel_res: float = float("nan")           # ||f - A u|| / ||r_0||
    P: list = field(default_factory=list)        # search directions (if kept)
    S: list = field(default_factory=list)        # A p_i (if kept)
    W: list = field(default_factory=list)        # w_i = B(r_i) (if kept)
    alphas: list = field(default_factory=list)
    iterates: list = field(default_factory=list)  # (r_{i+1}, u_{i+1}) if kept


def fcg(k, f, u0, precond, m_max: int = 5, max_iter: int = 300, tol: float = 1e-6,
        keep: bool = False, apply_A=None, w_hook=None,
        keep_iterates: bool = False) -> FCGResult:
    """Algorithm 1 step by step, in the paper's order and notation.

    ``precond(r) -> w`` is the (possibly nonlinear) preconditioner B; ``None``
    means B = I.  Stops at the first i with ||r_i||/||r_0|| <= tol (the
    criterion of Table 1); ``iters`` is that i.  ``w_hook(i, w) -> w`` lets a
    test perturb w (shadow runs for the rounding horizon)."""
    A = apply_A if apply_A is not None else (lambda v: stencil_apply(k, v))
    f = _t(f)
    u = _t(u0).clone()
    kt = _t(k)
    if (not torch.isfinite(kt).all()) or (kt <= 0).any() or (not torch.isfinite(f).all()) \
            or (not torch.isfinite(u).all()):
        return FCGResult(u, f - A(u) if torch.isfinite(u).all() else u.clone(), 0,
                         SYS_NONFINITE, [float("nan")])
    r = f - A(u)                                        # r_0 = f - A u_0
    rho0 = torch.linalg.vector_norm(r).item()
    hist = [1.0]
    res = FCGResult(u, r, 0, SYS_NOT_CONVERGED, hist)
    if rho0 == 0.0:
        res.status = SYS_OK
        res.true_rel_res = 0.0
        return res
    P, S, PS = {}, {}, {}
    for i in range(max_iter):
        w = r.clone() if precond is None else precond(r)          # w_i = B(r_i)
        if w_hook is not None:
            w = w_hook(i, w)
        m = window_size(i, m_max)
        p = w.clone()
        for kk in range(i - m, i):                                # classical Gram-Schmidt
            p = p - (torch.sum(w * S[kk]) / PS[kk]) * P[kk]       # against the original w_i
        s = A(p)                                                  # s_i = A p_i
        ps = torch.sum(p * s).item()
        pr = torch.sum(p * r).item()
        if not (math.isfinite(ps) and math.isfinite(pr)) or ps <= 0.0:
            res.status = SYS_BREAKDOWN
            res.iters = i
            break
        alpha = pr / ps
        u = u + alpha * p                                         # u_{i+1}
        r = r - alpha * s                                         # r_{i+1}
        P[i], S[i], PS[i] = p, s, ps
        for old in [j for j in P if j < i - m_max]:
            del P[old], S[old], PS[old]
        if keep:
            res.P.append(p); res.S.append(s); res.W.append(w)
        if keep_iterates:
            res.iterates.append((r.clone(), u.clone()))
        res.alphas.append(alpha)
        rho = torch.linalg.vector_norm(r).item() / rho0
        hist.append(rho)
        res.iters = i + 1
        if rho <= tol:
            res.status = SYS_OK
            break
    res.u, res.r = u, r
    res.true_rel_res = torch.linalg.vector_norm(f - A(u)).item() / rho0
    return res


# ---------------------------------------------------------------------------
# Classical preconditioners used in Table 1 (Sec. 3.3.1): Jacobi(k) and
# symmetric Gauss-Seidel(k), each applied for k steps from x^0 = 0 with b = z.
# ---------------------------------------------------------------------------

def jacobi_precond(k, steps: int):
    """x^{n+1} = x^n + D(A)^{-1} (b - A x^n), ``steps`` times from x^0 = 0."""
    kt = _t(k)
    N = kt.shape[-1] - 2
    h2 = 1.0 / float(N + 1) ** 2
    kc = kt[1:-1, 1:-1]
    diag = (0.5 * (kc + kt[2:, 1:-1]) + 0.5 * (kc + kt[:-2, 1:-1])
            + 0.5 * (kc + kt[1:-1, 2:]) + 0.5 * (kc + kt[1:-1, :-2])) / h2

    def apply(z):
        x = torch.zeros_like(z)
        for _ in range(steps):
            x = x + (z - stencil_apply(kt, x)) / diag
        return x
    return apply


def sgs_precond(k, steps: int):
    """x^{n+1/2} = x^n + L(A)^{-1}(b - A x^n); x^{n+1} = x^{n+1/2} + U(A)^{-1}(b - A x^{n+1/2}),
    L and U the lower and upper triangles of A including the diagonal."""
    A = assemble(k)
    Lo = sp.tril(A, format="csr")
    Up = sp.triu(A, format="csr")

    def apply(z):
        b = z.numpy().reshape(-1)
        x = np.zeros_like(b)
        for _ in range(steps):
            x = x + spla.spsolve_triangular(Lo, b - A @ x, lower=True)
            x = x + spla.spsolve_triangular(Up, b - A @ x, lower=False)
        return torch.from_numpy(x.reshape(z.shape))
    return apply


def red_black_order(N: int) -> np.ndarray:
    """Unknowns of the N x N grid (row-major index i*N + j) reordered red first:
    red = i + j even, black = i + j odd, each colour in row-major order."""
    i, j = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    idx = (i * N + j).reshape(-1)
    colour = ((i + j) % 2).reshape(-1)
    return np.concatenate([idx[colour == 0], idx[colour == 1]])


def rb_sgs_precond(k, steps: int):
    """Symmetric Gauss-Seidel(k) of Sec. 3.3.1 applied to the red-black reordered
    matrix P A P^T (red points first): the same two half steps with the lower
    and upper triangles of the reordered matrix, mapped back to grid order."""
    A = assemble(k)
    N = _t(k).shape[-1] - 2
    perm = red_black_order(N)
    Ap = A[perm][:, perm].tocsr()
    Lo = sp.tril(Ap, format="csr")
    Up = sp.triu(Ap, format="csr")

    def apply(z):
        b = z.numpy().reshape(-1)[perm]
        x = np.zeros_like(b)
        for _ in range(steps):
            x = x + spla.spsolve_triangular(Lo, b - Ap @ x, lower=True)
            x = x + spla.spsolve_triangular(Up, b - Ap @ x, lower=False)
        out = np.empty_like(x)
        out[perm] = x
        return torch.from_numpy(out.reshape(z.shape))
    return apply


# ---------------------------------------------------------------------------
# The neural-operator preconditioner B(r; theta) (Sec. 2.4.2): a pointwise lift,
# L spectral layers u <- S L A u realised with the FFT (analysis = truncated
# forward DFT, L = per-mode complex channel mixing, synthesis = inverse DFT)
# plus a 1x1 bypass and GELU, and a pointwise projection.
# ---------------------------------------------------------------------------

@dataclass
class NOWeights:
    C: int
    M: int
    L: int
    Cin: int
    W_L: torch.Tensor          # [C][Cin]
    b_L: torch.Tensor          # [C]
    R: list                    # L x complex [C][C][2M][M]  (c_in, c_out, kx, ky)
    W: list                    # L x [C][C]                 (c_out, c_in)
    b: list                    # L x [C]
    W_P: torch.Tensor          # [C]
    b_P: torch.Tensor          # [1]
    basis: str = "fourier"     # "fourier" or "sine" (the spectral layers' basis)

    def params(self):
        out = [self.W_L, self.b_L]
        for l in range(self.L):
            out += [self.R[l], self.W[l], self.b[l]]
        return out + [self.W_P, self.b_P]


def unpack_weights(blob, C: int, M: int, L: int = 4, Cin: int = 4,
                   requires_grad: bool = False, basis: str = "fourier") -> NOWeights:
    """Blob order (float64): W_L, b_L, then per layer Re R, Im R, W, b, then W_P, b_P.
    basis "sine": the layers use the sine basis (only Re R takes part)."""
    if basis not in ("fourier", "sine"):
        raise ValueError("basis must be 'fourier' or 'sine'")
    v = _t(blob).clone()
    o = 0

    def take(n, shape):
        nonlocal o
        t = v[o:o + n].reshape(shape)
        o += n
        return t

    W_L = take(C * Cin, (C, Cin)); b_L = take(C, (C,))
    R, W, b = [], [], []
    nR = C * C * 2 * M * M
    for _ in range(L):
        re = take(nR, (C, C, 2 * M, M)); im = take(nR, (C, C, 2 * M, M))
        R.append(torch.complex(re, im))
        W.append(take(C * C, (C, C))); b.append(take(C, (C,)))
    W_P = take(C, (C,)); b_P = take(1, (1,))
    assert o == v.numel(), "weight blob size does not match the architecture"
    w = NOWeights(C, M, L, Cin, W_L, b_L, R, W, b, W_P, b_P, basis)
    if requires_grad:
        for p in w.params():
            p.requires_grad_(True)
    return w


def pack_weights(w: NOWeights) -> np.ndarray:
    parts = [w.W_L.reshape(-1), w.b_L]
    for l in range(w.L):
        parts += [w.R[l].real.reshape(-1), w.R[l].imag.reshape(-1), w.W[l].reshape(-1), w.b[l]]
    parts += [w.W_P, w.b_P]
    return torch.cat([p.detach().reshape(-1) for p in parts]).numpy().copy()


def gelu(z):
    """Exact GELU: z/2 * (1 + erf(z / sqrt 2))."""
    return 0.5 * z * (1.0 + torch.erf(z / math.sqrt(2.0)))


def no_features(k, r, s):
    """phi = [r/s, log k_interior, x1, x2] at the interior nodes x = (i+1) h."""
    N = r.shape[-1]
    h = 1.0 / (N + 1)
    xs = (torch.arange(N, dtype=_f64) + 1.0) * h
    X1 = xs[:, None].expand(N, N)
    X2 = xs[None, :].expand(N, N)
    kt = _t(k)
    lead = r.shape[:-2]
    return torch.stack([r / s[..., None, None], torch.log(kt[..., 1:-1, 1:-1]),
                        X1.expand(*lead, N, N), X2.expand(*lead, N, N)], dim=-3)


def _spectral(v, Rl, M):
    """Fourier layer: truncated forward DFT (kx in {0..M-1} U {N-M..N-1},
    ky in {0..M-1}), per-mode mixing W^[o] = sum_c V^[c] R[c][o], inverse DFT
    with the 1/N^2 normalisation.  ``v``: [..., C, N, N]."""
    N = v.shape[-1]
    vh = torch.fft.rfft2(v)                                    # [..., C, N, N/2+1]
    modes = torch.cat([vh[..., :M, :M], vh[..., N - M:, :M]], dim=-2)   # [..., C, 2M, M]
    wh = torch.einsum("...ckq,cokq->...okq", modes, Rl)
    out = torch.zeros(wh.shape[:-2] + (N, N // 2 + 1), dtype=wh.dtype)
    out[..., :M, :M] = wh[..., :M, :]
    out[..., N - M:, :M] = wh[..., M:, :]
    return torch.fft.irfft2(out, s=(N, N))


def sine_matrix(P: int, N: int) -> torch.Tensor:
    """S[p][x] = sin(pi (p+1)(x+1) / (N+1)), p < P: the first P discrete sine
    (DST-I) modes on the N interior points, which vanish on the boundary."""
    p = torch.arange(P, dtype=_f64)[:, None] + 1.0
    x = torch.arange(N, dtype=_f64)[None, :] + 1.0
    return torch.sin(math.pi * p * x / (N + 1))


def _spectral_sine(v, Rl, M):
    """Sine-basis layer (the Dirichlet-matched alternative to the FFT named in
    Sec. 2.4.2 and Sec. 5): truncated DST-I analysis with 2M modes along x and
    M along y, per-mode real mixing W^[o] = sum_c V^[c] Re R[c][o], synthesis
    with the inverse DST-I normalisation (2/(N+1))^2.  ``v``: [..., C, N, N]."""
    N = v.shape[-1]
    Sx, Sy = sine_matrix(2 * M, N), sine_matrix(M, N)
    vh = torch.einsum("ax,...cxy,qy->...caq", Sx, v, Sy)
    wh = torch.einsum("...caq,coaq->...oaq", vh, Rl.real)
    return (2.0 / (N + 1)) ** 2 * torch.einsum("ax,...oaq,qy->...oxy", Sx, wh, Sy)


def no_apply(w: NOWeights, k, r, return_acts: bool = False):
    """B(r; theta) = s * NO(phi(r / s, k)), s = ||r||_2 / sqrt(n); B(0) = 0.
    ``r``: [..., N, N], ``k``: [..., N+2, N+2]."""
    r = _t(r) if not isinstance(r, torch.Tensor) else r
    N = r.shape[-1]
    if 2 * w.M > N:
        raise ValueError("need 2*modes <= N")
    s = torch.linalg.vector_norm(r, dim=(-2, -1)) / math.sqrt(N * N)
    safe = torch.where(s > 0, s, torch.ones_like(s))
    phi = no_features(k, r, safe)                                       # [..., 4, N, N]
    v = torch.einsum("cf,...fxy->...cxy", w.W_L, phi) + w.b_L[:, None, None]
    acts = [v]
    for l in range(w.L):
        y = _spectral(v, w.R[l], w.M) if w.basis == "fourier" else _spectral_sine(v, w.R[l], w.M)
        z = y + torch.einsum("oc,...cxy->...oxy", w.W[l], v) + w.b[l][:, None, None]
        v = gelu(z)
        acts.append(v)
    out = torch.einsum("o,...oxy->...xy", w.W_P, v) + w.b_P[0]
    out = out * s[..., None, None]
    out = torch.where((s > 0)[..., None, None], out, torch.zeros_like(out))
    return (out, acts) if return_acts else out


# ---------------------------------------------------------------------------
# Losses (Sec. 2.4.1 and Sec. 3.1): the Notay loss in its error form
# ||B(r) - e||_A / ||e||_A with e = A^-1 r, and the L2 variant.
# ---------------------------------------------------------------------------

def energy_norm(k, x):
    """||x||_A = sqrt((x, A x)) over the last two axes."""
    return torch.sqrt(torch.sum(x * stencil_apply(k, x), dim=(-2, -1)))


def notay_loss(k, w, e):
    """mean over the batch of ||w - e||_A / ||e||_A."""
    return torch.mean(energy_norm(k, w - e) / energy_norm(k, e))


def l2_loss(w, e):
    """mean over the batch of ||w - e||_2 / ||e||_2."""
    return torch.mean(torch.linalg.vector_norm(w - e, dim=(-2, -1))
                      / torch.linalg.vector_norm(e, dim=(-2, -1)))


def krylov_samples(k, f, u0, m: int, u_star=None, m_max: int = 1):
    """Residuals drawn from Krylov subspaces (the training scheme of Sec. 3.1,
    the sampling distribution p_Km): run CG -- FCG with B = I -- from u0 for m
    iterations and keep (r_i, e_i), i = 1..m, with e_i = u* - u_i, u* = A^-1 f."""
    if u_star is None:
        u_star = torch.from_numpy(exact_solve(k, f))
    res = fcg(k, f, u0, None, m_max=m_max, max_iter=m, tol=0.0, keep_iterates=True)
    us = torch.stack([it[1] for it in res.iterates])
    rs = torch.stack([it[0] for it in res.iterates])
    return rs, _t(u_star) - us


# ---------------------------------------------------------------------------
# AdamW (decoupled weight decay), the optimiser of the training table.
# ---------------------------------------------------------------------------

def adamw_step(theta, grad, m, v, t: int, lr=1e-3, wd=1e-2, beta1=0.9, beta2=0.999,
               eps=1e-8):
    """One AdamW step on flat float64 arrays; ``t`` is the 1-based step count.
    theta <- theta (1 - lr wd); m, v moment updates; theta -= lr mhat/(sqrt(vhat)+eps)."""
    theta = theta * (1.0 - lr * wd)
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    theta = theta - lr * mhat / (np.sqrt(vhat) + eps)
    return theta, m, v
