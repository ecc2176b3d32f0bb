"""Training path on the GPU (hand-written backward through the C ABI) against
the CPU oracle's float64 autograd gradient, finite differences and the
oracle's AdamW step."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

fc = pytest.importorskip("paper_2402_05598_amd")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _oracle_params(blob, C, M, L):
    """Leaf tensors in blob order (R split into real and imaginary parts)."""
    t = torch.from_numpy(np.asarray(blob, dtype=np.float64)).clone()
    o = 0
    leaves = []

    def take(n, shape):
        nonlocal o
        x = t[o:o + n].reshape(shape).clone().requires_grad_(True)
        o += n
        leaves.append(x)
        return x
    WL = take(C * 4, (C, 4)); bL = take(C, (C,))
    R, W, b = [], [], []
    nR = C * C * 2 * M * M
    for _ in range(L):
        re = take(nR, (C, C, 2 * M, M)); im = take(nR, (C, C, 2 * M, M))
        R.append(torch.complex(re, im)); W.append(take(C * C, (C, C))); b.append(take(C, (C,)))
    WP = take(C, (C,)); bP = take(1, (1,))
    w = oracle.NOWeights(C, M, L, 4, WL, bL, R, W, b, WP, bP)
    return w, leaves


def _oracle_grad(blob, C, M, L, fn):
    w, leaves = _oracle_params(blob, C, M, L)
    val = fn(w)
    val.backward()
    return val.item(), torch.cat([x.grad.reshape(-1) for x in leaves]).numpy()


def _data(N, B, seed):
    k, f, u0 = [], [], []
    for s in range(B):
        kk, ff, uu, _ = synth.system(seed + s, N, (10.0, 200.0))
        k.append(kk); f.append(ff); u0.append(uu)
    return np.stack(k), np.stack(f), np.stack(u0)


# (72, ...) and (130, ...) take the segmented-row path of the backward (more
# points per row than a block holds), with ragged last segments
@pytest.mark.parametrize("N,C,M,L", [(16, 16, 4, 2), (24, 16, 3, 4), (20, 32, 5, 1), (72, 16, 4, 2),
                                     (130, 16, 5, 2)])
def test_op_backward_matches_oracle_fp64(dev, N, C, M, L):
    print(f"backward N={N} C={C} M={M} L={L}", flush=True)
    B = 2
    k, r, _ = _data(N, B, 40 + N)
    g = synth.rng(7).standard_normal((B, N, N))
    blob = synth.init_weights(N + L, C, M, L)
    blob[C * 4 + C:] *= 2.0
    kt = torch.from_numpy(k)
    val, gref = _oracle_grad(blob, C, M, L,
                             lambda w: torch.sum(torch.from_numpy(g) * oracle.no_apply(w, kt, torch.from_numpy(r))))
    model = fc.Model(blob, C, M, L)
    kd, rd, gd = [torch.from_numpy(a).to(dev) for a in (k, r, g)]
    wgpu, ws = fc.op_forward(model, kd, rd, "fp64")
    ggpu = fc.op_backward(model, kd, rd, gd, ws, "fp64").cpu().numpy()
    wref = oracle.no_apply(oracle.unpack_weights(blob, C, M, L), kt, torch.from_numpy(r)).numpy()
    assert np.max(np.abs(wgpu.cpu().numpy() - wref)) <= 1e-12 * np.max(np.abs(wref))
    rel = np.linalg.norm(ggpu - gref) / np.linalg.norm(gref)
    print(f"  grad rel err {rel:.2e}", flush=True)
    assert rel < 1e-11
    model.close()


def test_energy_loss_and_gradient(dev):
    N, B = 24, 3
    k, w, e = _data(N, B, 90)
    wt = torch.from_numpy(w).requires_grad_(True)
    L = oracle.notay_loss(torch.from_numpy(k), wt, torch.from_numpy(e))
    L.backward()
    kd, wd, ed = [torch.from_numpy(a).to(dev) for a in (k, w, e)]
    loss, gw = fc.energy_loss(kd, wd, ed)
    assert abs(loss.mean().item() - L.item()) <= 1e-13 * L.item()
    rel = torch.linalg.vector_norm(gw.cpu() - wt.grad) / torch.linalg.vector_norm(wt.grad)
    assert rel < 1e-12


def test_directional_finite_difference_fp64(dev):
    """(L(theta + h d) - L(theta - h d)) / 2h against grad . d, all on the GPU."""
    N, B, C, M, L = 16, 2, 16, 4, 2
    k, r, _ = _data(N, B, 300)
    e = synth.rng(3).standard_normal((B, N, N))
    blob = synth.init_weights(11, C, M, L)
    model = fc.Model(blob, C, M, L)
    kd, rd, ed = [torch.from_numpy(a).to(dev) for a in (k, r, e)]

    def loss_of(th):
        model.set_weights(th)
        w = fc.precond_apply(model, kd, rd, op="fp64")
        return fc.energy_loss(kd, w, ed, grad=False)[0].mean().item()
    model.set_weights(blob)
    w, ws = fc.op_forward(model, kd, rd, "fp64")
    _, gw = fc.energy_loss(kd, w, ed)
    grad = fc.op_backward(model, kd, rd, gw, ws, "fp64").cpu().numpy()
    g = synth.rng(5)
    for _ in range(3):
        d = g.standard_normal(blob.size)
        d /= np.linalg.norm(d)
        h = 1e-5
        fd = (loss_of(blob + h * d) - loss_of(blob - h * d)) / (2 * h)
        an = float(grad @ d)
        print(f"  fd {fd:.10e} analytic {an:.10e}", flush=True)
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3)
    model.close()


def test_train_step_matches_oracle_adamw(dev):
    N, B, C, M, L = 16, 4, 16, 3, 2
    k, f, u0 = _data(N, B, 500)
    rs, es = [], []
    for b in range(B):
        rr, ee = oracle.krylov_samples(k[b], f[b], u0[b], 3)
        rs.append(rr[-1].numpy()); es.append(ee[-1].numpy())
    r, e = np.stack(rs), np.stack(es)
    blob = synth.init_weights(21, C, M, L)
    kt = torch.from_numpy(k)
    val, gref = _oracle_grad(blob, C, M, L, lambda w: oracle.notay_loss(
        kt, oracle.no_apply(w, kt, torch.from_numpy(r)), torch.from_numpy(e)))
    th1, _, _ = oracle.adamw_step(blob, gref, np.zeros_like(blob), np.zeros_like(blob), 1, lr=1e-3, wd=1e-2)
    model = fc.Model(blob, C, M, L)
    opt = fc.Optim(model, lr=1e-3, weight_decay=1e-2)
    kd, rd, ed = [torch.from_numpy(a).to(dev) for a in (k, r, e)]
    loss = fc.train_step(model, opt, kd, rd, ed, op="fp64")
    assert abs(loss - val) <= 1e-12 * val
    got = model.get_weights()
    # AdamW's first step is lr * sign(g) except where |g| ~ eps: compare where the oracle gradient is resolved
    ok = np.abs(gref) > 1e-6
    assert np.max(np.abs(got[ok] - th1[ok])) < 1e-12
    assert np.max(np.abs(got - th1)) < 2e-3
    opt.close()
    model.close()


# width 16 guards the pre-activation store of the float32 training forward
@pytest.mark.parametrize("N,C", [(32, 32), (136, 32), (24, 16), (40, 16)])
def test_fp32_gradient_close_to_fp64(dev, N, C):
    print(f"fp32 vs fp64 gradient N={N} C={C}", flush=True)
    B, M, L = 2, 6, 4
    k, r, _ = _data(N, B, 700)
    g = synth.rng(8).standard_normal((B, N, N))
    blob = synth.init_weights(31, C, M, L)
    model = fc.Model(blob, C, M, L)
    kd, rd, gd = [torch.from_numpy(a).to(dev) for a in (k, r, g)]
    _, ws64 = fc.op_forward(model, kd, rd, "fp64")
    g64 = fc.op_backward(model, kd, rd, gd, ws64, "fp64").cpu().numpy()
    _, ws32 = fc.op_forward(model, kd, rd, "fp32")
    g32 = fc.op_backward(model, kd, rd, gd, ws32, "fp32").cpu().numpy()
    rel = np.linalg.norm(g32 - g64) / np.linalg.norm(g64)
    cos = float(g32 @ g64 / (np.linalg.norm(g32) * np.linalg.norm(g64)))
    print(f"  fp32 vs fp64 gradient: rel {rel:.2e} cos {cos:.8f}", flush=True)
    assert rel < 1e-4 and cos > 1 - 1e-8
    model.close()


def test_autograd_function(dev):
    N, B, C, M, L = 16, 2, 16, 3, 2
    k, r, _ = _data(N, B, 800)
    blob = synth.init_weights(41, C, M, L)
    model = fc.Model(blob, C, M, L)
    kd, rd = [torch.from_numpy(a).to(dev) for a in (k, r)]
    wts = torch.from_numpy(blob).to(dev).requires_grad_(True)
    w = fc.OperatorFunction.apply(wts, model, kd, rd, "fp64")
    (w * w).sum().backward()
    kt = torch.from_numpy(k)
    _, gref = _oracle_grad(blob, C, M, L, lambda ww: torch.sum(oracle.no_apply(ww, kt, torch.from_numpy(r)) ** 2))
    rel = np.linalg.norm(wts.grad.cpu().numpy() - gref) / np.linalg.norm(gref)
    assert rel < 1e-11
    model.close()


def test_autograd_function_interleaved_weights(dev):
    """Two forwards with different weights on one model, then the first one's
    backward: its gradient is the oracle's for the first weights (the model is
    reloaded when its weights changed after the forward); a train step in
    between invalidates the cached blob too."""
    N, B, C, M, L = 16, 2, 16, 3, 2
    k, r, _ = _data(N, B, 810)
    blob_a = synth.init_weights(42, C, M, L)
    blob_b = synth.init_weights(43, C, M, L)
    model = fc.Model(blob_a, C, M, L)
    kd, rd = [torch.from_numpy(a).to(dev) for a in (k, r)]
    wa = torch.from_numpy(blob_a).to(dev).requires_grad_(True)
    wb = torch.from_numpy(blob_b).to(dev).requires_grad_(True)
    ya = fc.OperatorFunction.apply(wa, model, kd, rd, "fp64")
    yb = fc.OperatorFunction.apply(wb, model, kd, rd, "fp64")
    (ya * ya).sum().backward()
    kt, rt = torch.from_numpy(k), torch.from_numpy(r)
    _, ga = _oracle_grad(blob_a, C, M, L, lambda ww: torch.sum(oracle.no_apply(ww, kt, rt) ** 2))
    rel = np.linalg.norm(wa.grad.cpu().numpy() - ga) / np.linalg.norm(ga)
    print(f"  interleaved backward rel {rel:.2e}", flush=True)
    assert rel < 1e-11
    (yb * yb).sum().backward()
    _, gb = _oracle_grad(blob_b, C, M, L, lambda ww: torch.sum(oracle.no_apply(ww, kt, rt) ** 2))
    assert np.linalg.norm(wb.grad.cpu().numpy() - gb) / np.linalg.norm(gb) < 1e-11
    # a train step changes the device weights: the same blob must be reloaded
    opt = fc.Optim(model, lr=1e-2)
    e = torch.randn_like(rd)
    fc.train_step(model, opt, kd, rd, e, op="fp64")
    opt.close()
    y2 = fc.OperatorFunction.apply(wa.detach(), model, kd, rd, "fp64")
    ref = oracle.no_apply(oracle.unpack_weights(blob_a, C, M, L), kt, rt).numpy()
    assert np.max(np.abs(y2.cpu().numpy() - ref)) <= 1e-12 * np.max(np.abs(ref))
    model.close()


def test_krylov_samples_match_oracle(dev):
    """GPU conjugate-gradient samples (r_i, u* - u_i) against the oracle's CG
    with u* from a sparse direct solve.  CG amplifies rounding differences
    from one iteration to the next, so the tolerance on r_i follows the spread
    of a shadow oracle run whose u0 is perturbed at the 1e-15 level."""
    N, B, m = 32, 3, 24
    k, f, u0 = _data(N, B, 900)
    kd, fd, ud = [torch.from_numpy(a).to(dev) for a in (k, f, u0)]
    r, e = fc.krylov_samples(kd, fd, ud, m_iter=m)
    r, e = r.cpu().numpy(), e.cpu().numpy()
    for b in range(B):
        rr, ee = oracle.krylov_samples(k[b], f[b], u0[b], m)
        rr, ee = rr.numpy(), ee.numpy()
        pert = u0[b] * (1.0 + 1e-15 * synth.rng(b).standard_normal(u0[b].shape))
        rs, _ = oracle.krylov_samples(k[b], f[b], pert, m)
        rs = rs.numpy()
        for i in range(m):
            spread = np.linalg.norm(rs[i] - rr[i]) / np.linalg.norm(rr[i])
            dr = np.linalg.norm(r[b, i] - rr[i]) / np.linalg.norm(rr[i])
            de = np.linalg.norm(e[b, i] - ee[i]) / np.linalg.norm(ee[i])
            assert dr < max(1e-10, 100 * spread) and de < max(1e-8, 100 * spread), (b, i, dr, spread, de)
        # A e_i = r_i up to the tight solve's residual
        Ae = oracle.stencil_apply(k[b], e[b]).numpy()
        rel = np.linalg.norm(Ae - r[b]) / np.linalg.norm(r[b, -1])
        assert rel < 1e-7


def test_l2_loss_and_gradient(dev):
    N, B = 24, 3
    k, w, e = _data(N, B, 95)
    wt = torch.from_numpy(w).requires_grad_(True)
    L = oracle.l2_loss(wt, torch.from_numpy(e))
    L.backward()
    kd, wd, ed = [torch.from_numpy(a).to(dev) for a in (k, w, e)]
    loss, gw = fc.energy_loss(kd, wd, ed, kind="l2")
    assert abs(loss.mean().item() - L.item()) <= 1e-13 * L.item()
    rel = torch.linalg.vector_norm(gw.cpu() - wt.grad) / torch.linalg.vector_norm(wt.grad)
    assert rel < 1e-12


def test_train_step_l2_matches_oracle_adamw(dev):
    N, B, C, M, L = 16, 4, 16, 3, 2
    k, f, u0 = _data(N, B, 510)
    rs, es = [], []
    for b in range(B):
        rr, ee = oracle.krylov_samples(k[b], f[b], u0[b], 3)
        rs.append(rr[-1].numpy()); es.append(ee[-1].numpy())
    r, e = np.stack(rs), np.stack(es)
    blob = synth.init_weights(23, C, M, L)
    kt = torch.from_numpy(k)
    val, gref = _oracle_grad(blob, C, M, L, lambda w: oracle.l2_loss(
        oracle.no_apply(w, kt, torch.from_numpy(r)), torch.from_numpy(e)))
    th1, _, _ = oracle.adamw_step(blob, gref, np.zeros_like(blob), np.zeros_like(blob), 1, lr=1e-3, wd=1e-2)
    model = fc.Model(blob, C, M, L)
    opt = fc.Optim(model, lr=1e-3, weight_decay=1e-2)
    kd, rd, ed = [torch.from_numpy(a).to(dev) for a in (k, r, e)]
    loss = fc.train_step(model, opt, kd, rd, ed, op="fp64", loss="l2")
    assert abs(loss - val) <= 1e-12 * val
    got = model.get_weights()
    ok = np.abs(gref) > 1e-6
    assert np.max(np.abs(got[ok] - th1[ok])) < 1e-12
    opt.close()
    model.close()


def test_residual_samples_match_oracle(dev):
    """Random right-hand sides: r = f - A u exactly, e = A^-1 f - u against a
    sparse direct solve."""
    N, B = 24, 3
    k, f, _ = _data(N, B, 930)
    u = synth.rng(12).standard_normal((B, N, N))
    kd, fd, ud = [torch.from_numpy(a).to(dev) for a in (k, f, u)]
    r, e = fc.residual_samples(kd, fd, ud)
    r, e = r.cpu().numpy(), e.cpu().numpy()
    for b in range(B):
        rr = f[b] - oracle.stencil_apply(k[b], u[b]).numpy()
        ee = oracle.exact_solve(k[b], f[b]) - u[b]
        assert np.linalg.norm(r[b] - rr) <= 1e-13 * np.linalg.norm(rr)
        assert np.linalg.norm(e[b] - ee) <= 1e-8 * np.linalg.norm(ee)


@pytest.mark.parametrize("N,C,M,L", [(24, 16, 3, 2), (72, 16, 4, 2)])
def test_op_backward_input_gradient(dev, N, C, M, L):
    """d/dr of sum <g, B(r)> (B(r) = s NO(r/s), through s too) against the
    oracle's autograd; Euler's identity for the degree-1 homogeneous operator,
    sum_p r_p dL/dr_p = sum_p g_p B(r)_p; FP32 against FP64; and the
    autograd Function delivers the same input gradient."""
    print(f"input gradient N={N}", flush=True)
    B = 2
    k, r, _ = _data(N, B, 60 + N)
    g = synth.rng(11).standard_normal((B, N, N))
    blob = synth.init_weights(N + 5, C, M, L)
    blob[C * 4 + C:] *= 2.0
    w_o = oracle.unpack_weights(blob, C, M, L)
    rt = torch.from_numpy(r).clone().requires_grad_(True)
    val = torch.sum(torch.from_numpy(g) * oracle.no_apply(w_o, torch.from_numpy(k), rt))
    val.backward()
    gr_ref = rt.grad.numpy()
    model = fc.Model(blob, C, M, L)
    kd, rd, gd = [torch.from_numpy(a).to(dev) for a in (k, r, g)]
    w64, ws = fc.op_forward(model, kd, rd, "fp64")
    _, gr = fc.op_backward(model, kd, rd, gd, ws, "fp64", input_grad=True)
    gr = gr.cpu().numpy()
    rel = np.linalg.norm(gr - gr_ref) / np.linalg.norm(gr_ref)
    print(f"  input grad rel err {rel:.2e}", flush=True)
    assert rel < 1e-10
    lhs = np.sum(r * gr, axis=(1, 2))
    rhs = np.sum(g * w64.cpu().numpy(), axis=(1, 2))
    assert np.max(np.abs(lhs - rhs) / np.abs(rhs)) < 1e-10
    _, ws32 = fc.op_forward(model, kd, rd, "fp32")
    _, gr32 = fc.op_backward(model, kd, rd, gd, ws32, "fp32", input_grad=True)
    assert np.linalg.norm(gr32.cpu().numpy() - gr) / np.linalg.norm(gr) < 1e-4
    # through the autograd Function
    wts = torch.from_numpy(blob).to(dev)
    ra = rd.clone().requires_grad_(True)
    out = fc.OperatorFunction.apply(wts, model, kd, ra, "fp64")
    torch.sum(gd * out).backward()
    assert np.linalg.norm(ra.grad.cpu().numpy() - gr) / np.linalg.norm(gr) < 1e-12
    model.close()
