"""Write the benchmark's operator: bench_operator_c32_m12_l4.npy.

Trains the neural operator (4 layers, width 32, 12 modes, Fourier basis) on
the GPU through the library, exactly as bench.py's set-up training does
(bench.train_operator: 1024 seeded 64 x 64 systems, k = exp(GRF) with
contrast 10..1e3, conjugate-gradient Krylov samples of iterations 1..400,
energy-norm loss, AdamW with lr 6e-4 halved every quarter of the 48000
steps, mini-batch 64, FP32 operator), and stores the float64 master weights
rounded to float32.  bench.py loads this file, so its figures compare
kernels across changes rather than training runs.

Run on a GPU:  python weights/make_bench_operator.py [out.npy]
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def main():
    import numpy as np
    import torch

    import bench
    import paper_2402_05598_amd as fc
    out = sys.argv[1] if len(sys.argv) > 1 else os.path.join(ROOT, "weights", "bench_operator_c32_m12_l4.npy")
    dev = torch.device("cuda:0")
    model, info = bench.train_operator(fc, torch, dev, 32, 12, 4, 48000, None, Bs=1024, lr=6e-4)
    np.save(out, model.get_weights().astype(np.float32))
    print(f"wrote {out}: {info}", flush=True)
    model.close()


if __name__ == "__main__":
    main()
