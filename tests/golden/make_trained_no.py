"""Write tests/golden/no_trained_c16_m4_l2.npy: a small neural operator
trained on the CPU with the oracle (energy-norm loss of Sec. 2.4 on CG Krylov
samples of Sec. 3.1, AdamW), so that the GPU solves with every operator
precision can be checked against the FP64 oracle at a preconditioner that
converges.  Calls only the oracle and the seeded input generators.

    python tests/golden/make_trained_no.py
"""
import os
import sys

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle  # noqa: E402
import synth  # noqa: E402

C, M, L, N = 16, 4, 2, 24
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "no_trained_c16_m4_l2.npy")


def leaves_of(blob):
    t = torch.from_numpy(blob).clone()
    o, leaves = 0, []

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
    return oracle.NOWeights(C, M, L, 4, WL, bL, R, W, b, WP, bP), leaves


def main():
    torch.manual_seed(0)
    ks, rs, es = [], [], []
    for s in range(24):
        k, f, u0, _ = synth.system(9000 + s, N, (10.0, 100.0))
        r, e = oracle.krylov_samples(k, f, u0, 80)
        ks.append(np.repeat(k[None], r.shape[0], 0)); rs.append(r.numpy()); es.append(e.numpy())
    K, R, E = np.concatenate(ks), np.concatenate(rs), np.concatenate(es)
    blob = synth.init_weights(9, C, M, L)
    blob[blob.size - C - 1:] *= 1e-3
    m = np.zeros_like(blob); v = np.zeros_like(blob)
    g = np.random.default_rng(1)
    lr = 3e-3
    steps = 600
    for step in range(1, steps + 1):
        if step % 200 == 0:
            lr *= 0.5
        idx = g.integers(0, K.shape[0], 32)
        w, leaves = leaves_of(blob)
        kt = torch.from_numpy(K[idx])
        loss = oracle.notay_loss(kt, oracle.no_apply(w, kt, torch.from_numpy(R[idx])), torch.from_numpy(E[idx]))
        loss.backward()
        grad = torch.cat([x.grad.reshape(-1) for x in leaves]).numpy()
        blob, m, v = oracle.adamw_step(blob, grad, m, v, step, lr=lr, wd=1e-2)
        if step % 100 == 0:
            print(f"step {step}: loss {loss.item():.4f}", flush=True)
    np.save(OUT, blob)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
