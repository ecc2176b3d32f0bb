"""Pins of the CPU oracle against what the paper and mathematics fix, each
independent of the oracle's own code (closed forms, textbook algorithms written
here, brute-force sums, the paper's printed numbers)."""
import json
import math
import os

import numpy as np
import pytest
import scipy.fft
import torch

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _sine_mode(N, p, q):
    x = np.arange(1, N + 1) / (N + 1)
    return np.outer(np.sin(p * np.pi * x), np.sin(q * np.pi * x))


# ---------------------------------------------------------------- stencil ---

@pytest.mark.parametrize("N,p,q,kappa", [(8, 1, 1, 1.0), (8, 2, 5, 3.5), (13, 7, 2, 0.25)])
def test_stencil_sine_eigenpairs(N, p, q, kappa):
    """Constant k: sin(p pi x) sin(q pi y) is an eigenvector with
    lambda = 4 k h^-2 (sin^2(p pi h/2) + sin^2(q pi h/2))."""
    h = 1.0 / (N + 1)
    v = _sine_mode(N, p, q)
    lam = 4 * kappa / h**2 * (np.sin(p * np.pi * h / 2) ** 2 + np.sin(q * np.pi * h / 2) ** 2)
    Av = oracle.stencil_apply(np.full((N + 2, N + 2), kappa), v).numpy()
    assert np.max(np.abs(Av - lam * v)) <= 1e-12 * lam * np.max(np.abs(v))


def test_stencil_dirichlet_energy():
    """(u, A u) = h^-2 sum over grid edges of k_face (u_a - u_b)^2, with u = 0 on
    boundary nodes and k_face the mean of the two nodal values (brute force)."""
    N = 7
    g = synth.rng(3)
    k = np.exp(g.standard_normal((N + 2, N + 2)))
    u = g.standard_normal((N, N))
    U = np.zeros((N + 2, N + 2)); U[1:-1, 1:-1] = u
    e = 0.0
    for a in range(N + 2):
        for b in range(N + 2):
            for da, db in ((1, 0), (0, 1)):
                a2, b2 = a + da, b + db
                if a2 > N + 1 or b2 > N + 1:
                    continue
                inner = lambda i, j: 1 <= i <= N and 1 <= j <= N
                if not (inner(a, b) or inner(a2, b2)):
                    continue
                e += 0.5 * (k[a, b] + k[a2, b2]) * (U[a, b] - U[a2, b2]) ** 2
    e *= (N + 1) ** 2
    Au = oracle.stencil_apply(k, u).numpy()
    assert abs(np.sum(u * Au) - e) <= 1e-12 * e


def test_stencil_symmetric_and_assembled():
    N = 6
    g = synth.rng(4)
    k = np.exp(g.standard_normal((N + 2, N + 2)))
    A = oracle.assemble(k).toarray()
    assert np.allclose(A, A.T, rtol=0, atol=1e-12 * np.abs(A).max())
    assert np.all(np.linalg.eigvalsh(A) > 0)
    u = g.standard_normal((N, N)); v = g.standard_normal((N, N))
    Au = oracle.stencil_apply(k, u).numpy(); Av = oracle.stencil_apply(k, v).numpy()
    assert abs(np.sum(v * Au) - np.sum(u * Av)) < 1e-10 * np.abs(A).max()
    assert np.allclose((A @ u.reshape(-1)).reshape(N, N), Au, rtol=1e-13, atol=1e-10)


# --------------------------------------------------------------- schedule ---

def test_window_schedule_values():
    """m_i for m_max = 5 and 20, the sequence Algorithm 1 produces (by hand)."""
    assert [oracle.window_size(i, 5) for i in range(16)] == \
        [0, 1, 2, 3, 4, 5, 1, 1, 2, 3, 4, 5, 1, 1, 2, 3]
    assert [oracle.window_size(i, 20) for i in range(18, 27)] == [18, 19, 20, 1, 1, 2, 3, 4, 5]


# ------------------------------------------------------------------- FCG ---

def _textbook_cg(A, f, u0, iters):
    """Hestenes-Stiefel CG, written here independently of Algorithm 1."""
    u = u0.copy(); r = f - A(u); p = r.copy(); rr = np.sum(r * r)
    hist = [1.0]; r0 = math.sqrt(rr)
    for _ in range(iters):
        Ap = A(p); a = rr / np.sum(p * Ap)
        u += a * p; r -= a * Ap
        rr_new = np.sum(r * r)
        p = r + (rr_new / rr) * p; rr = rr_new
        hist.append(math.sqrt(rr) / r0)
    return np.array(hist)


def test_fcg_identity_is_cg():
    k, f, u0 = synth.poisson_system(11, 32)
    A = lambda v: oracle.stencil_apply(k, v).numpy()
    ref = _textbook_cg(A, f, u0, 30)
    for m_max in (1, 5, 20):
        res = oracle.fcg(k, f, u0, None, m_max=m_max, max_iter=30, tol=0.0)
        assert np.max(np.abs(np.array(res.hist) - ref) / ref) < 1e-11


def test_fcg_finite_termination():
    """Constant k, u0 = 0 and f a sum of 3 eigenvectors with distinct eigenvalues:
    CG (FCG with B = I) reaches the solution in exactly 3 iterations."""
    N = 12
    k = np.full((N + 2, N + 2), 2.0)
    f = _sine_mode(N, 1, 1) + 0.5 * _sine_mode(N, 2, 3) - 0.25 * _sine_mode(N, 4, 4)
    res = oracle.fcg(k, f, np.zeros((N, N)), None, m_max=5, max_iter=10, tol=1e-12)
    assert res.iters == 3
    assert res.hist[2] > 1e-3 and res.hist[3] < 1e-12


def test_fcg_jacobi_is_pcg():
    """Any SPD linear B: FCG equals textbook preconditioned CG (written here)."""
    k, f, u0 = synth.diffusion_system(5, 24)
    A = lambda v: oracle.stencil_apply(k, v).numpy()
    Bj = oracle.jacobi_precond(k, 4)
    B = lambda v: Bj(torch.from_numpy(v)).numpy()
    u = u0.copy(); r = f - A(u); z = B(r); p = z.copy(); rz = np.sum(r * z)
    r0 = np.linalg.norm(r); ref = [1.0]
    for _ in range(20):
        Ap = A(p); a = rz / np.sum(p * Ap)
        u += a * p; r -= a * Ap; z = B(r)
        rz_new = np.sum(r * z); p = z + (rz_new / rz) * p; rz = rz_new
        ref.append(np.linalg.norm(r) / r0)
    res = oracle.fcg(k, f, u0, Bj, m_max=5, max_iter=20, tol=0.0)
    assert np.max(np.abs(np.array(res.hist) - ref) / np.array(ref)) < 1e-10


@pytest.mark.parametrize("steps", [1, 2, 4])
def test_jacobi_is_truncated_neumann_series(steps):
    """Sec. 3.3.1: k Jacobi steps x <- x + D^-1 (z - A x) from x = 0 give
    x_k = sum_{j<k} (I - D^-1 A)^j D^-1 z.  Dense matrices on a 6x6 grid from
    the assembled matrix (not the stencil the oracle sweeps with)."""
    N = 6
    k, _, _ = synth.diffusion_system(45, N)
    A = oracle.assemble(k).toarray()
    Dinv = np.diag(1.0 / np.diag(A))
    E = np.eye(N * N) - Dinv @ A
    Bmat = sum(np.linalg.matrix_power(E, j) for j in range(steps)) @ Dinv
    B = oracle.jacobi_precond(k, steps)
    cols = np.stack([B(torch.from_numpy(e.reshape(N, N))).numpy().reshape(-1) for e in np.eye(N * N)], axis=1)
    assert np.max(np.abs(cols - Bmat)) <= 1e-12 * np.max(np.abs(Bmat))
    if steps == 1:   # one step is D^-1: the diagonal by hand at one point
        h2 = 1.0 / (N + 1) ** 2
        i, j = 2, 3
        c = k[i + 1, j + 1]
        d = 0.5 * (4 * c + k[i + 2, j + 1] + k[i, j + 1] + k[i + 1, j + 2] + k[i + 1, j]) / h2
        assert abs(cols[i * N + j, i * N + j] - 1.0 / d) <= 1e-14 / d


def _red_black_by_hand(N):
    reds = [i * N + j for i in range(N) for j in range(N) if (i + j) % 2 == 0]
    blacks = [i * N + j for i in range(N) for j in range(N) if (i + j) % 2 == 1]
    return np.array(reds + blacks)


@pytest.mark.parametrize("ordering", ["lexicographic", "red-black"])
@pytest.mark.parametrize("steps", [1, 3])
def test_sgs_is_textbook_symmetric_gauss_seidel(ordering, steps):
    """Saad, Sec. 4.1: one SGS step from x = 0 applies M^-1 with
    M = (D + L) D^-1 (D + U) in the ordering used (L, U strict triangles), and
    k steps leave the error propagator (I - M^-1 A)^k, so
    B_k = (I - (I - M^-1 A)^k) A^-1.  Dense matrices on a small grid."""
    N = 6
    k, _, _ = synth.diffusion_system(41, N)
    A = oracle.assemble(k).toarray()
    n = N * N
    perm = np.arange(n) if ordering == "lexicographic" else _red_black_by_hand(N)
    Ap = A[np.ix_(perm, perm)]
    D = np.diag(np.diag(Ap))
    Lo, Up = np.tril(Ap, -1), np.triu(Ap, 1)
    Mp = (D + Lo) @ np.linalg.inv(D) @ (D + Up)
    E = np.eye(n) - np.linalg.solve(Mp, Ap)
    Bp = (np.eye(n) - np.linalg.matrix_power(E, steps)) @ np.linalg.inv(Ap)
    Bmat = np.empty_like(Bp)
    Bmat[np.ix_(perm, perm)] = Bp
    B = (oracle.sgs_precond if ordering == "lexicographic" else oracle.rb_sgs_precond)(k, steps)
    rng = np.random.default_rng(3)
    for _ in range(3):
        z = rng.standard_normal((N, N))
        got = B(torch.from_numpy(z)).numpy().reshape(-1)
        want = Bmat @ z.reshape(-1)
        assert np.max(np.abs(got - want)) <= 1e-10 * np.max(np.abs(want))
    assert np.max(np.abs(Bmat - Bmat.T)) <= 1e-9 * np.max(np.abs(Bmat))


@pytest.mark.parametrize("steps", [1, 2, 4])
def test_rb_sgs_is_alternating_colour_sweeps(steps):
    """In red-black order points of one colour couple only to the other, so a
    symmetric step red, black, black, red repeats its black half sweep and the
    next step's red one repeats the last: k steps are 2k + 1 point sweeps
    alternating red, black, ..., red, each setting x_p = (z_p - sum_q a_pq x_q) / a_pp."""
    N = 7
    k, _, _ = synth.diffusion_system(43, N)
    A = oracle.assemble(k).toarray()
    z = np.random.default_rng(5).standard_normal((N, N))
    x = np.zeros(N * N)
    zf = z.reshape(-1)
    for h in range(2 * steps + 1):
        colour = h % 2
        for i in range(N):
            for j in range(N):
                if (i + j) % 2 != colour:
                    continue
                p = i * N + j
                acc = zf[p]
                for q in range(N * N):
                    if q != p:
                        acc -= A[p, q] * x[q]
                x[p] = acc / A[p, p]
    got = oracle.rb_sgs_precond(k, steps)(torch.from_numpy(z)).numpy().reshape(-1)
    assert np.max(np.abs(got - x)) <= 1e-12 * np.max(np.abs(x))


def test_fcg_rb_sgs_is_pcg():
    """Red-black SGS is SPD and linear: FCG equals textbook preconditioned CG."""
    k, f, u0 = synth.diffusion_system(7, 20)
    A = lambda v: oracle.stencil_apply(k, v).numpy()
    Bs = oracle.rb_sgs_precond(k, 2)
    B = lambda v: Bs(torch.from_numpy(v)).numpy()
    u = u0.copy(); r = f - A(u); z = B(r); p = z.copy(); rz = np.sum(r * z)
    r0 = np.linalg.norm(r); ref = [1.0]
    for _ in range(12):
        Ap = A(p); a = rz / np.sum(p * Ap)
        u += a * p; r -= a * Ap; z = B(r)
        rz_new = np.sum(r * z); p = z + (rz_new / rz) * p; rz = rz_new
        ref.append(np.linalg.norm(r) / r0)
    res = oracle.fcg(k, f, u0, Bs, m_max=5, max_iter=12, tol=0.0)
    assert np.max(np.abs(np.array(res.hist) - ref) / np.array(ref)) < 1e-8


def _dst_poisson_inverse(N, kappa):
    """A^-1 for constant k via the type-I sine transform (closed-form eigenbasis)."""
    h = 1.0 / (N + 1)
    p = np.arange(1, N + 1)
    lam = 4 * kappa / h**2 * (np.sin(p[:, None] * np.pi * h / 2) ** 2
                              + np.sin(p[None, :] * np.pi * h / 2) ** 2)
    return lambda r: torch.from_numpy(
        scipy.fft.idstn(scipy.fft.dstn(r.numpy(), type=1) / lam, type=1))


def test_fcg_one_step_with_exact_inverse():
    N = 20
    k = np.ones((N + 2, N + 2))
    g = synth.rng(9)
    f = g.standard_normal((N, N)); u0 = g.standard_normal((N, N))
    res = oracle.fcg(k, f, u0, _dst_poisson_inverse(N, 1.0), m_max=5, max_iter=5, tol=1e-12)
    assert res.iters == 1 and res.hist[1] < 1e-13


def _random_no(seed=1, C=8, M=3):
    return oracle.unpack_weights(synth.init_weights(seed, C, M), C, M)


def test_fcg_window_orthogonality_and_energy_identity():
    """For any (here nonlinear) B: (p_i, A p_k) = 0 over the window, (p_i, r_{i+1}) = 0,
    and ||e_i||_A^2 - ||e_{i+1}||_A^2 = (p_i, r_i)^2 / (p_i, s_i)."""
    N = 16
    k, f, u0, _ = synth.system(21, N, (10.0, 100.0))
    w = _random_no()
    kt = torch.from_numpy(k)
    ustar = oracle.exact_solve(k, f)
    iters = []
    res = oracle.fcg(k, f, u0, lambda r: oracle.no_apply(w, kt, r), m_max=4, max_iter=14,
                     tol=0.0, keep=True, keep_iterates=True)
    P = [p.numpy() for p in res.P]; S = [s.numpy() for s in res.S]
    Wv = [x.numpy() for x in res.W]
    A = lambda v: oracle.stencil_apply(k, v).numpy()
    en = lambda v: math.sqrt(np.sum(v * A(v)))
    for i in range(1, len(P)):
        m = oracle.window_size(i, 4)
        for kk in range(i - m, i):
            c = abs(np.sum(P[i] * S[kk])) / (en(Wv[i]) * en(P[kk]))
            assert c < 1e-8, (i, kk, c)       # classical Gram-Schmidt rounding only
    outside = [abs(np.sum(P[i] * S[kk])) / (en(P[i]) * en(P[kk]))
               for i in range(5, len(P)) for kk in range(0, i - oracle.window_size(i, 4))]
    assert max(outside) > 1e-2               # truncation really drops older directions
    us = [u0] + [it[1].numpy() for it in res.iterates]
    rs = [f - A(u0)] + [it[0].numpy() for it in res.iterates]
    for i in range(len(P)):
        assert abs(np.sum(P[i] * rs[i + 1])) <= 1e-11 * np.linalg.norm(P[i]) * np.linalg.norm(rs[i])
        e0 = ustar - us[i]; e1 = ustar - us[i + 1]
        lhs = np.sum(e0 * A(e0)) - np.sum(e1 * A(e1))
        rhs = np.sum(P[i] * rs[i]) ** 2 / np.sum(P[i] * S[i])
        assert lhs >= -1e-12 * np.sum(e0 * A(e0))
        assert abs(lhs - rhs) <= 1e-9 * np.sum(e0 * A(e0))


def test_fcg_status_cases():
    N = 8
    g = synth.rng(2)
    f = g.standard_normal((N, N)); u0 = g.standard_normal((N, N))
    k = np.ones((N + 2, N + 2))
    knan = k.copy(); knan[3, 3] = np.nan
    assert oracle.fcg(knan, f, u0, None).status == oracle.SYS_NONFINITE
    kneg = k.copy(); kneg[2, 5] = -1.0
    assert oracle.fcg(kneg, f, u0, None).status == oracle.SYS_NONFINITE
    res = oracle.fcg(k, np.zeros((N, N)), np.zeros((N, N)), None)
    assert res.status == oracle.SYS_OK and res.iters == 0
    res = oracle.fcg(k, f, u0, lambda r: torch.zeros_like(r))
    assert res.status == oracle.SYS_BREAKDOWN and res.iters == 0
    res = oracle.fcg(k, f, u0, None, max_iter=1)
    assert res.status == oracle.SYS_NOT_CONVERGED and res.iters == 1


@pytest.mark.slow
def test_table1_classical_columns():
    """Table 1's CG, Jacobi(4), GS(1) and GS(4) columns, reproduced on freshly drawn
    Poisson and Diffusion data (3 samples; the paper's exact samples are not
    published), m_max = 20, within 12% of the printed counts."""
    gold = json.load(open(os.path.join(GOLD, "table1_classical.json")))
    cases = [("Poisson", 32, "CG"), ("Poisson", 64, "CG"), ("Poisson", 128, "CG"),
             ("Diffusion", 32, "CG"), ("Diffusion", 64, "CG"),
             ("Poisson", 32, "Jacobi(4)"), ("Poisson", 64, "Jacobi(4)"),
             ("Diffusion", 32, "Jacobi(4)"),
             ("Poisson", 32, "GS(1)"), ("Poisson", 32, "GS(4)"), ("Diffusion", 32, "GS(4)")]
    for data, N, method in cases:
        counts = []
        for s in range(3):
            gen = synth.poisson_system if data == "Poisson" else synth.diffusion_system
            k, f, u0 = gen(100 * N + s, N)
            B = {"CG": None,
                 "Jacobi(4)": oracle.jacobi_precond(k, 4),
                 "GS(1)": oracle.sgs_precond(k, 1),
                 "GS(4)": oracle.sgs_precond(k, 4)}[method]
            res = oracle.fcg(k, f, u0, B, m_max=20, max_iter=1000, tol=1e-6)
            assert res.status == oracle.SYS_OK
            counts.append(res.iters)
        paper = gold[data][str(N)][method]
        assert abs(np.mean(counts) - paper) <= 0.12 * paper + 1, (data, N, method, counts, paper)


# ------------------------------------------------------ neural operator ---

def _brute_force_no(wb, k, r, C, M, L):
    """The operator written with explicit DFT sums over every point and kept mode."""
    N = r.shape[0]
    h = 1.0 / (N + 1)
    s = np.linalg.norm(r) / N
    xs = (np.arange(N) + 1) * h
    phi = np.stack([r / s, np.log(k[1:-1, 1:-1]), np.repeat(xs[:, None], N, 1),
                    np.repeat(xs[None, :], N, 0)])
    o = 0

    def take(n, shape):
        nonlocal o
        t = wb[o:o + n].reshape(shape); o += n
        return t
    WL = take(4 * C, (C, 4)); bL = take(C, (C,))
    v = np.einsum("cf,fxy->cxy", WL, phi) + bL[:, None, None]
    KX = list(range(M)) + list(range(N - M, N))
    xg, yg = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    for _ in range(L):
        nR = C * C * 2 * M * M
        R = take(nR, (C, C, 2 * M, M)) + 1j * take(nR, (C, C, 2 * M, M))
        W = take(C * C, (C, C)); b = take(C, (C,))
        Vh = np.zeros((C, 2 * M, M), complex)
        for c in range(C):
            for a, kx in enumerate(KX):
                for ky in range(M):
                    Vh[c, a, ky] = np.sum(v[c] * np.exp(-2j * np.pi * (kx * xg + ky * yg) / N))
        Wh = np.einsum("cak,coak->oak", Vh, R)
        y = np.zeros((C, N, N))
        for oc in range(C):
            for a, kx in enumerate(KX):
                for ky in range(M):
                    gam = 1.0 if ky == 0 else 2.0
                    y[oc] += gam * np.real(Wh[oc, a, ky] * np.exp(2j * np.pi * (kx * xg + ky * yg) / N))
        y /= N * N
        z = y + np.einsum("oc,cxy->oxy", W, v) + b[:, None, None]
        from scipy.special import erf
        v = 0.5 * z * (1 + erf(z / np.sqrt(2)))
    WP = take(C, (C,)); bP = take(1, (1,))
    return s * (np.einsum("o,oxy->xy", WP, v) + bP[0])


@pytest.mark.parametrize("N,C,M", [(6, 2, 2), (7, 3, 3), (8, 2, 4)])
def test_no_matches_explicit_dft_sums(N, C, M):
    g = synth.rng(N)
    k = np.exp(0.5 * g.standard_normal((N + 2, N + 2)))
    r = g.standard_normal((N, N))
    wb = synth.init_weights(N + 100, C, M, L=2)
    wb[C * 4 + C:] *= 3.0   # larger spectral part so that every mode matters
    w = oracle.unpack_weights(wb, C, M, L=2)
    got = oracle.no_apply(w, torch.from_numpy(k), torch.from_numpy(r)).numpy()
    ref = _brute_force_no(wb, k, r, C, M, 2)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_sine_matrix_is_scipy_dst1():
    """scipy's DST-I: y_k = 2 sum_n x_n sin(pi (k+1)(n+1) / (N+1))."""
    for N, P in [(7, 4), (16, 16), (33, 10)]:
        x = synth.rng(N).standard_normal(N)
        want = scipy.fft.dst(x, type=1)[:P] / 2.0
        got = oracle.sine_matrix(P, N).numpy() @ x
        assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))


@pytest.mark.parametrize("N,M,kappa", [(12, 3, 1.0), (17, 4, 2.5)])
def test_sine_layer_inverts_constant_k_poisson_on_kept_modes(N, M, kappa):
    """With one channel and weights 1/lambda_pq (the eigenvalues of constant-k
    A on sin(p pi x) sin(q pi y)), the sine-basis layer maps a combination of
    the kept modes (p <= 2M along x, q <= M along y) to A^-1 of it, and drops
    modes outside the kept set."""
    h = 1.0 / (N + 1)
    lam = lambda p, q: 4 * kappa / h**2 * (np.sin(p * np.pi * h / 2)**2 + np.sin(q * np.pi * h / 2)**2)
    R = np.zeros((1, 1, 2 * M, M))
    for a in range(2 * M):
        for q in range(M):
            R[0, 0, a, q] = 1.0 / lam(a + 1, q + 1)
    Rc = torch.complex(torch.from_numpy(R), torch.from_numpy(np.random.default_rng(1).standard_normal(R.shape)))
    g = synth.rng(N + M)
    r = np.zeros((N, N)); want = np.zeros((N, N))
    for p, q in [(1, 1), (2 * M, 1), (1, M), (3, 2), (2 * M, M)]:
        c = g.standard_normal()
        r += c * _sine_mode(N, p, q); want += c / lam(p, q) * _sine_mode(N, p, q)
    got = oracle.fcgno_ref._spectral_sine(torch.from_numpy(r)[None], Rc, M)[0].numpy()
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
    k = np.full((N + 2, N + 2), kappa)
    assert np.max(np.abs(oracle.stencil_apply(k, got).numpy() - r)) <= 1e-10 * np.max(np.abs(r))
    for p, q in [(2 * M + 1, 1), (1, M + 1)]:
        out = oracle.fcgno_ref._spectral_sine(torch.from_numpy(_sine_mode(N, p, q))[None], Rc, M)[0]
        assert torch.max(torch.abs(out)) <= 1e-12


def test_no_homogeneity_and_zero():
    N = 16
    w = _random_no(C=8, M=4)
    k, f, _, _ = synth.system(5, N)
    kt = torch.from_numpy(k); r = torch.from_numpy(f)
    a = oracle.no_apply(w, kt, r)
    for e in (-3, 5):
        b = oracle.no_apply(w, kt, r * 2.0**e)
        assert torch.equal(b, a * 2.0**e)
    assert torch.count_nonzero(oracle.no_apply(w, kt, torch.zeros_like(r))) == 0


def test_gelu_values():
    z = torch.tensor([0.0, 1.0, -1.0, 2.0], dtype=torch.float64)
    ref = [0.0, 0.8413447460685429, -0.15865525393145707, 1.9544997361036416]
    assert torch.allclose(oracle.gelu(z), torch.tensor(ref, dtype=torch.float64), rtol=1e-15, atol=1e-16)


# ------------------------------------------------------------- losses -----

def test_notay_loss_on_eigenvectors():
    """Constant k, e = v_pq, w = e + eps v_rs: the loss is eps sqrt(lambda_rs/lambda_pq)."""
    N = 10
    h = 1.0 / (N + 1)
    k = np.full((N + 2, N + 2), 1.5)
    lam = lambda p, q: 4 * 1.5 / h**2 * (np.sin(p * np.pi * h / 2)**2 + np.sin(q * np.pi * h / 2)**2)
    e = _sine_mode(N, 1, 2); d = _sine_mode(N, 3, 5)
    for eps in (0.5, 2.0):
        L = oracle.notay_loss(k, torch.from_numpy(e + eps * d)[None], torch.from_numpy(e)[None]).item()
        assert abs(L - eps * math.sqrt(lam(3, 5) / lam(1, 2))) < 1e-12
        L2 = oracle.l2_loss(torch.from_numpy(e + eps * d)[None], torch.from_numpy(e)[None]).item()
        assert abs(L2 - eps) < 1e-12
    assert abs(oracle.notay_loss(k, torch.zeros(1, N, N, dtype=torch.float64),
                                 torch.from_numpy(e)[None]).item() - 1.0) < 1e-14


def test_loss_gradient_finite_differences():
    """Autograd gradient of the Notay loss through the operator vs central
    differences (torch.autograd.gradcheck)."""
    N, C, M = 8, 2, 2
    g = synth.rng(17)
    k = torch.from_numpy(np.exp(0.3 * g.standard_normal((2, N + 2, N + 2))))
    r = torch.from_numpy(g.standard_normal((2, N, N)))
    e = torch.from_numpy(g.standard_normal((2, N, N)))
    wb = synth.init_weights(3, C, M, L=2)
    base = oracle.unpack_weights(wb, C, M, L=2)
    names = ["W_L", "b_L", "W_P", "b_P"]

    def loss_of(*params):
        w = oracle.unpack_weights(wb, C, M, L=2)
        w.W_L, w.b_L, w.W_P, w.b_P = params[:4]
        w.R[0], w.W[1], w.b[0] = params[4:]
        return oracle.notay_loss(k, oracle.no_apply(w, k, r), e)
    params = [getattr(base, n).clone().requires_grad_(True) for n in names]
    params += [base.R[0].clone().requires_grad_(True), base.W[1].clone().requires_grad_(True),
               base.b[0].clone().requires_grad_(True)]
    assert torch.autograd.gradcheck(loss_of, params, eps=1e-6, atol=1e-8, rtol=1e-6)


def test_operator_input_gradient_finite_differences():
    """The oracle's gradient of B(r) = s NO(r/s) with respect to r, through
    s = ||r||/N as well, against central differences (gradcheck), and Euler's
    identity sum_p r_p d<g, B(r)>/dr_p = <g, B(r)> of a degree-1 positively
    homogeneous map: the reference for the library's input gradient."""
    N, C, M = 8, 2, 2
    g = synth.rng(23)
    k = torch.from_numpy(np.exp(0.3 * g.standard_normal((2, N + 2, N + 2))))
    r = torch.from_numpy(g.standard_normal((2, N, N))).requires_grad_(True)
    wb = synth.init_weights(5, C, M, L=2)
    wb[C * 4 + C:] *= 2.0
    w = oracle.unpack_weights(wb, C, M, L=2)
    assert torch.autograd.gradcheck(lambda x: oracle.no_apply(w, k, x), (r,), eps=1e-6, atol=1e-8, rtol=1e-6)
    gw = torch.from_numpy(g.standard_normal((2, N, N)))
    val = torch.sum(gw * oracle.no_apply(w, k, r))
    (grad,) = torch.autograd.grad(val, r)
    with torch.no_grad():
        lhs = torch.sum(r * grad, dim=(1, 2))
        rhs = torch.sum(gw * oracle.no_apply(w, k, r), dim=(1, 2))
    assert torch.allclose(lhs, rhs, rtol=1e-12, atol=0)


def test_krylov_samples_are_cg_iterates_one_to_m():
    """The kept pairs are iterates i = 1..m of conjugate gradients from u0
    (Sec. 3.1, Fig. 2a): r_i equal to textbook Hestenes-Stiefel CG's residual
    after i steps (written in this file) and e_i = u* - u_i for the same u_i."""
    N, m = 12, 9
    k, f, u0, _ = synth.system(18, N, (10.0, 100.0))
    A = lambda v: oracle.stencil_apply(k, v).numpy()
    ustar = np.linalg.solve(oracle.assemble(k).toarray(), f.reshape(-1)).reshape(N, N)
    u = u0.copy(); r = f - A(u); p = r.copy(); rr = np.sum(r * r)
    want_r, want_e = [], []
    for _ in range(m):
        Ap = A(p); a = rr / np.sum(p * Ap)
        u = u + a * p; r = r - a * Ap
        rr_new = np.sum(r * r); p = r + (rr_new / rr) * p; rr = rr_new
        want_r.append(r.copy()); want_e.append(ustar - u)
    rs, es = oracle.krylov_samples(k, f, u0, m, u_star=torch.from_numpy(ustar))
    assert rs.shape == (m, N, N) and es.shape == (m, N, N)
    for i in range(m):
        sc = np.max(np.abs(want_r[i]))
        assert np.max(np.abs(rs[i].numpy() - want_r[i])) <= 1e-9 * sc, i
        assert np.max(np.abs(es[i].numpy() - want_e[i])) <= 1e-9 * np.max(np.abs(want_e[i])), i
    # i = 0 (the initial residual) is not among them
    assert np.max(np.abs(rs[0].numpy() - (f - A(u0)))) > 1e-3 * np.max(np.abs(f - A(u0)))


def test_pack_weights_layout_and_round_trip():
    """pack_weights writes the blob order of the header: W_L[C][4], b_L[C],
    per layer Re R[C][C][2M][M], Im R, W[C][C], b[C], then W_P[C], b_P.  A blob
    holding its own indices unpacks to those positions and packs back."""
    C, M, L = 4, 2, 3
    n = synth.weight_count(C, M, L)
    blob = np.arange(n, dtype=np.float64)
    w = oracle.unpack_weights(blob, C, M, L)
    nR = C * C * 2 * M * M
    assert w.W_L[1, 2].item() == 1 * 4 + 2 and w.b_L[3].item() == 4 * C + 3
    o = 5 * C
    for l in range(L):
        c, oc, a, q = 1, 3, 2, 1
        assert w.R[l][c, oc, a, q].real.item() == o + ((c * C + oc) * 2 * M + a) * M + q
        assert w.R[l][c, oc, a, q].imag.item() == o + nR + ((c * C + oc) * 2 * M + a) * M + q
        assert w.W[l][2, 1].item() == o + 2 * nR + 2 * C + 1
        assert w.b[l][2].item() == o + 2 * nR + C * C + 2
        o += 2 * nR + C * C + C
    assert w.W_P[1].item() == o + 1 and w.b_P[0].item() == o + C == n - 1
    assert np.array_equal(oracle.pack_weights(w), blob)
    wb = synth.init_weights(5, C, M, L)
    assert np.array_equal(oracle.pack_weights(oracle.unpack_weights(wb, C, M, L)), wb)


def test_krylov_samples_consistent():
    """e_i = u* - u_i satisfies A e_i = r_i for every kept CG iterate."""
    N = 16
    k, f, u0, _ = synth.system(8, N, (10.0, 1000.0))
    rs, es = oracle.krylov_samples(k, f, u0, 12)
    assert rs.shape == (12, N, N)
    Ae = oracle.stencil_apply(k, es)
    assert torch.max(torch.abs(Ae - rs)) <= 1e-8 * torch.max(torch.abs(rs[0]))
    n = torch.linalg.vector_norm(rs, dim=(1, 2))
    assert n[-1] < n[0]


def test_adamw_first_steps():
    """First AdamW step: mhat = g and vhat = g^2, so theta1 = theta0 (1 - lr wd)
    - lr g / (|g| + eps); values checked by hand."""
    th = np.array([1.0, -2.0, 0.5]); g = np.array([0.3, -4.0, 0.0])
    t1, m, v = oracle.adamw_step(th, g, np.zeros(3), np.zeros(3), 1)
    ref = th * (1 - 1e-5) - 1e-3 * np.array([0.3 / (0.3 + 1e-8), -4.0 / (4.0 + 1e-8), 0.0])
    assert np.allclose(t1, ref, rtol=0, atol=1e-15)
    assert np.allclose(m, [0.03, -0.4, 0.0]) and np.allclose(v, [0.09e-3, 16e-3, 0.0])
