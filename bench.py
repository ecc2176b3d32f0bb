"""FCG-NO solve throughput on one MI355X.

Workload: 16 systems on a 512 x 512 interior grid (k = exp(GRF) rescaled to a
contrast drawn log-uniformly from [10, 1e3], f ~ GRF, u0 ~ N(0, I)), solved to
1e-6 relative residual by flexible conjugate gradients (window m = 5) with the
neural-operator preconditioner (4 layers, width 32, 12 modes) in BF16 on the
matrix cores with FP32 accumulation; Krylov vectors, stencil, dot products and
the final true-residual check in FP64.  The operator is the committed blob
weights/bench_operator_c32_m12_l4.npy, trained on 64 x 64 systems with the
energy-norm loss on conjugate-gradient Krylov samples, all on the GPU through
the library (weights/make_bench_operator.py writes it), so that the measured
figures compare kernels, not training runs.

One step = one batched solve of the 16 systems.  The same solves with the FP32
and FP64 operator are timed afterwards for comparison, then the other
workloads: the 32 x 32 single solve (FP64 operator, seeded initial weights),
64 solves at 128 x 128 and 256 x 256 (FP32 operator), training throughput
(64 x 64, batch 256) and a serving run (Poisson arrivals, grids 64..1024).
Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "layer_bf16_512x512x16_traffic.json")
BENCH_WEIGHTS = os.path.join(ROOT, "weights", "bench_operator_c32_m12_l4.npy")
KERNEL_SOURCES = ("paper_2402_05598_amd/csrc/no_fwd.hip", "paper_2402_05598_amd/csrc/common.h",
                  "paper_2402_05598_amd/csrc/mfma.h")


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--n", type=int, default=512)
    p.add_argument("--batch", type=int, default=16)
    p.add_argument("--train-steps", type=int, default=48000, help="with --train-operator")
    p.add_argument("--weights", default=BENCH_WEIGHTS, help="trained weights (.npy) of the benchmark's operator")
    p.add_argument("--train-operator", action="store_true",
                   help="train the operator at set-up (1024 systems, lr 6e-4) instead of loading --weights")
    p.add_argument("--save-weights", default=None)
    p.add_argument("--ops", default="bf16,fp32,fp64", help="first one is the reported value")
    p.add_argument("--max-iter", type=int, default=0, help="default max(2N, 300)")
    p.add_argument("--rtol", type=float, default=1e-6)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--serve-requests", type=int, default=200,
                   help="requests per serving run through the continuous-batching engine (0: no serving leg); "
                        "it runs after the timed and roofline legs")
    p.add_argument("--train-bench-steps", type=int, default=100,
                   help="timed steps of the training-throughput leg (64x64, batch 256; 0: skip)")
    p.add_argument("--cpu-seconds", type=float, default=20.0)
    p.add_argument("--calibrate-copy", action="store_true",
                   help="run one 1 GiB device copy first (HBM counter calibration under rocprofv3)")
    p.add_argument("--ablation", action="store_true",
                   help="also train with the Euclidean loss and with random-residual samples (Sec. 3.3) "
                        "and compare FCG iteration counts")
    p.add_argument("--ablation-steps", type=int, default=6000)
    p.add_argument("--classical", default="",
                   help="comma-separated grids: time FCG with CG, Jacobi(4), red-black SGS(1) and SGS(4) "
                        "next to the neural operator on the workload's systems at those sizes (Table 1)")
    p.add_argument("--cross-res", action="store_true",
                   help="Table 4: train at 32^2 and 64^2 (and fine-tune the 64^2 operator at 128^2), count "
                        "iterations to 1e-3, 1e-6 and 1e-12 at grids 64..1024")
    p.add_argument("--sine", action="store_true",
                   help="with --cross-res: also train sine-basis operators at 32^2 and 64^2")
    p.add_argument("--streams", type=int, default=0,
                   help="also time the main operator with the batch split over this many streams "
                        "(reported under comparison; kept out of the default run, whose kernel "
                        "statistics the roofline quotes)")
    p.add_argument("--main-only", action="store_true",
                   help="only the timed solves and their kernel figures (for profiler runs): no batched, "
                        "single-solve, training, serving or CPU legs")
    p.add_argument("--log", default=None, help="progress log file (default: stderr)")
    return p.parse_args()


def log(msg, f=None):
    print(msg, file=f or sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def layer_bytes_per_launch(N, B, C, M, esize, asize, S):
    """Algorithmic HBM bytes of one inner-layer kernel launch: read the layer
    input v_l and write v_{l+1} ([point][C], op precision), read the per-row
    synthesis operand [N][C][MP] and write the per-row partial spectra,
    S segments x C channels x the kept mode slots (accumulate precision: the
    bfloat16 operator stores the 2M kept slots, the others all MP), for B
    systems."""
    MP = (2 * M + 15) // 16 * 16
    kept = 2 * M if esize == 2 else MP
    per_point = 2 * C * esize
    per_row = C * MP * esize + S * kept * C * asize
    return B * (N * N * per_point + N * per_row)


def train_operator(fc, torch, dev, C, M, L, steps, logf, loss="energy", sampling="krylov", Nt=64, Bs=256,
                   m_iter=400, init=None, lr=3e-4, basis="fourier"):
    """Energy-norm training on conjugate-gradient Krylov samples of Nt x Nt
    systems (default 64, 256 systems, CG iterations 1..400; AdamW, lr halved
    every quarter of the run, weight decay 1e-2).  loss="l2" and
    sampling="random" give the two alternatives of the ablation in Sec. 3.3
    (random samples: u ~ N(0, I), f ~ GRF per sample, r = f - A u,
    e = A^-1 f - u).  init: a weight blob to start from (fine-tuning).
    basis: the spectral layers' basis ("fourier" or "sine").
    Returns the model and a summary."""
    import synth
    mb = 64
    if init is None:
        blob = synth.init_weights(3, C, M, L)
        blob[blob.size - C - 1:] *= 1e-3   # start the projection near zero: w ~ 0 has loss 1
    else:
        blob = np.array(init, dtype=np.float64)
    model = fc.Model(blob, C, M, L, basis=basis)
    if steps <= 0:
        return model, None
    k, f, u0, _ = synth.batch(3, Bs, Nt, (10.0, 1000.0))
    kd, fd, ud = [torch.from_numpy(a).to(dev) for a in (k, f, u0)]
    t0 = time.perf_counter()
    if sampling == "krylov":
        r, e = fc.krylov_samples(kd, fd, ud, m_iter=m_iter)
    else:
        per = 32
        g = synth.rng(77)
        fs = np.stack([synth.rhs_field(g, Nt) for _ in range(Bs * per)])
        us = g.standard_normal((Bs * per, Nt, Nt))
        kr = kd.repeat_interleave(per, dim=0).contiguous()
        rr, ee = fc.residual_samples(kr, torch.from_numpy(fs).to(dev), torch.from_numpy(us).to(dev))
        r, e = rr.view(Bs, per, Nt, Nt), ee.view(Bs, per, Nt, Nt)
        m_iter = per
    torch.cuda.synchronize()
    log(f"{sampling} samples {tuple(r.shape)} in {time.perf_counter() - t0:.2f}s", logf)
    lr_first = lr
    opt = fc.Optim(model, lr=lr, weight_decay=1e-2)
    ws = fc.train_workspace(model, Nt, mb, "fp32", dev)
    g = torch.Generator(device=dev)
    g.manual_seed(1234)
    sys_i = torch.randint(0, Bs, (steps, mb), generator=g, device=dev)
    it_i = torch.randint(0, m_iter, (steps, mb), generator=g, device=dev)
    t0 = time.perf_counter()
    losses = []
    for s in range(steps):
        if s and s % max(1, steps // 4) == 0:
            lr *= 0.5
            opt.set_lr(lr)
        si, ii = sys_i[s], it_i[s]
        want = s % 200 == 0 or s >= steps - 50
        val = fc.train_step(model, opt, kd[si], r[si, ii], e[si, ii], op="fp32", workspace=ws, return_loss=want,
                            loss=loss)
        if want:
            losses.append(val)
        if s % 2000 == 0:
            log(f"train step {s}: {loss} loss {val:.4f} ({time.perf_counter() - t0:.1f}s)", logf)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    opt.close()
    return model, {"grid": Nt, "systems": Bs, "lr": lr_first, "sampling": sampling, "loss": loss, "basis": basis,
                   "samples_per_system": m_iter, "batch": mb, "steps": steps,
                   "seconds": round(dt, 2), "steps_per_sec": round(steps / dt, 1), "loss_first": round(losses[0], 4),
                   "loss_last50": round(float(np.mean(losses[-50:])), 4)}


def ablation(fc, torch, dev, C, M, L, steps, logf):
    """Sec. 3.3: the energy-norm loss against the Euclidean loss, and Krylov
    samples against random residuals; FCG (m = 5, FP32 operator, tol 1e-6)
    iteration counts on 16 held-out systems per grid, next to CG."""
    import synth
    out = {}
    tests = {}
    for N in (64, 128):
        k, f, u0, _ = synth.batch(5, 16, N, (10.0, 1000.0))
        tests[N] = [torch.from_numpy(a).to(dev) for a in (k, f, u0)]

    def evaluate(model, op):
        res = {}
        for N, (kd, fd, ud) in tests.items():
            u = ud.clone()
            o = fc.solve(model, kd, fd, u, op=op, m_max=5, max_iter=1000, rtol=1e-6, hist=False)
            ok = o["status"] == 0
            res[str(N)] = {"converged": int(ok.sum()), "of": int(ok.size),
                           "iters_median": float(np.median(o["iters"])),
                           "iters_median_converged": float(np.median(o["iters"][ok])) if ok.any() else None}
        return res
    out["cg"] = evaluate(None, "identity")
    for name, loss, sampling in (("energy_krylov", "energy", "krylov"), ("l2_krylov", "l2", "krylov"),
                                 ("energy_random", "energy", "random")):
        model, info = train_operator(fc, torch, dev, C, M, L, steps, logf, loss=loss, sampling=sampling)
        out[name] = {"training": info, "fcg": evaluate(model, "fp32")}
        log(f"ablation {name}: {out[name]['fcg']}", logf)
        model.close()
    return out


def classical(fc, torch, dev, model, grids, B, main_op, logf):
    """Table 1 on the GPU with wall clock: FCG (m = 5, tol 1e-6) preconditioned
    by nothing (CG), Jacobi(4), red-black symmetric Gauss-Seidel(1) and (4),
    and the neural operator, on the benchmark's systems (k = exp(GRF),
    contrast 10..1e3) at each grid; one warm-up solve then two timed ones."""
    import synth
    out = {}
    methods = [("CG", "identity", 1), ("Jacobi(4)", "jacobi", 4), ("SGS-RB(1)", "sgs_rb", 1),
               ("SGS-RB(4)", "sgs_rb", 4), (f"NO({main_op})", main_op, 1)]
    for N in grids:
        k, f, u0, _ = synth.batch(2, B, N, (10.0, 1000.0))
        kd, fd, u0d = [torch.from_numpy(a).to(dev) for a in (k, f, u0)]
        row = {}
        for name, op, steps in methods:
            mdl = model if op in ("fp64", "fp32", "bf16") else None
            max_iter = 40 * N
            ws = torch.empty(fc.solve_workspace_bytes(mdl, N, B, op, 5, max_iter, 1e-6, steps),
                             dtype=torch.uint8, device=dev)
            u = u0d.clone()
            fc.solve(mdl, kd, fd, u, op=op, m_max=5, max_iter=max_iter, rtol=1e-6, hist=False,
                     workspace=ws, precond_steps=steps)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(2):
                u = u0d.clone()
                o = fc.solve(mdl, kd, fd, u, op=op, m_max=5, max_iter=max_iter, rtol=1e-6, hist=False,
                             workspace=ws, precond_steps=steps)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / 2
            ok = o["status"] == 0
            row[name] = {"iters_median": float(np.median(o["iters"])), "iters_max": int(o["iters"].max()),
                         "converged": int(ok.sum()), "of": B, "ms_per_batch": round(dt * 1e3, 2),
                         "ms_per_iteration": round(dt * 1e3 / max(int(o["iters"].max()), 1), 4)}
            log(f"classical N={N} {name}: {row[name]}", logf)
        out[str(N)] = row
    return out


def cross_resolution(fc, torch, dev, C, M, L, main_op, logf, model64=None, info64=None, sine=False):
    """Sec. 3.4 (Table 4): an operator trained on a coarse grid preconditions
    FCG on finer ones.  Operators trained at 32^2 and 64^2 (16000 steps each,
    the 64^2 one reused when given) and the 64^2 one fine-tuned at 128^2
    (4000 steps, lr 1e-4); 16 held-out systems per test grid (k = exp(GRF),
    contrast 10..1e3), m = 5, at most max(2N, 300) iterations; the first
    iteration reaching each relative residual (median over the systems, those
    that never reach it counted at the limit) and how many reach it."""
    import synth
    grids = (64, 128, 256, 512, 1024)
    tests = {}
    for N in grids:
        k, f, u0, _ = synth.batch(5, 16, N, (10.0, 1000.0))
        tests[N] = [torch.from_numpy(a).to(dev) for a in (k, f, u0)]

    def evaluate(model, op):
        res = {}
        for N, (kd, fd, ud) in tests.items():
            u = ud.clone()
            mi = max(2 * N, 300)
            o = fc.solve(model, kd, fd, u, op=op, m_max=5, max_iter=mi, rtol=1e-12)
            row = {"max_iter": mi}
            for tol in (1e-3, 1e-6, 1e-12):
                first = []
                for b in range(o["hist"].shape[0]):
                    idx = np.nonzero(o["hist"][b] <= tol)[0]
                    first.append(int(idx[0]) if idx.size else -1)
                first = np.array(first)
                ok = first >= 0
                row[f"{tol:g}"] = {"reached": int(ok.sum()), "of": int(ok.size),
                                   "median": float(np.median(np.where(ok, first, mi)))}
            res[str(N)] = row
        return res
    out = {"cg": evaluate(None, "identity")}
    log(f"cross-res cg: {out['cg']}", logf)
    m32, i32 = train_operator(fc, torch, dev, C, M, L, 16000, logf, Nt=32)
    out["train32"] = {"training": i32, "fcg": evaluate(m32, main_op)}
    m32.close()
    own = model64 is None
    if own:
        model64, i64 = train_operator(fc, torch, dev, C, M, L, 16000, logf, Nt=64)
    else:
        i64 = info64
    out["train64"] = {"training": i64, "fcg": evaluate(model64, main_op)}
    mft, ift = train_operator(fc, torch, dev, C, M, L, 4000, logf, Nt=128, Bs=128, init=model64.get_weights(),
                              lr=1e-4)
    out["train64_finetune128"] = {"training": ift, "fcg": evaluate(mft, main_op)}
    mft.close()
    if own:
        model64.close()
    names = ["train32", "train64", "train64_finetune128"]
    if sine:
        # the same recipe with sine-basis (DST-I) spectral layers
        for Nt in (32, 64):
            ms, inf = train_operator(fc, torch, dev, C, M, L, 16000, logf, Nt=Nt, basis="sine")
            out[f"train{Nt}_sine"] = {"training": inf, "fcg": evaluate(ms, main_op)}
            ms.close()
            names.append(f"train{Nt}_sine")
    for name in names:
        log(f"cross-res {name}: {out[name]['fcg']}", logf)
    return out


def batched(fc, torch, dev, model, C, M, L, logf, steps=3):
    """The batched configuration: 64 solves at 128^2 and at 256^2 (k = exp(GRF),
    contrast 10..1e3), FP32 operator, FP64 Krylov, tol 1e-6, at most
    max(2N, 300) iterations; one warm-up batch, then the timed batches."""
    import synth
    out = {}
    for N in (128, 256):
        k, f, u0, _ = synth.batch(1, 64, N, (10.0, 1000.0))
        kd, fd, u0d = [torch.from_numpy(a).to(dev) for a in (k, f, u0)]
        mi = max(2 * N, 300)
        ws = torch.empty(fc.solve_workspace_bytes(model, N, 64, "fp32", 5, mi, 1e-6), dtype=torch.uint8, device=dev)
        fc.solve(model, kd, fd, u0d.clone(), op="fp32", m_max=5, max_iter=mi, rtol=1e-6, hist=False, workspace=ws)
        torch.cuda.synchronize()
        fc.profile_reset()
        fc.profile_enable(True, ["layer"])
        lat, its, st = [], [], []
        t0 = time.perf_counter()
        for _ in range(steps):
            ts = time.perf_counter()
            o = fc.solve(model, kd, fd, u0d.clone(), op="fp32", m_max=5, max_iter=mi, rtol=1e-6, hist=False,
                         workspace=ws)
            lat.append((time.perf_counter() - ts) * 1e3)
            its.append(o["iters"])
            st.append(o["status"])
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        fc.profile_enable(False)
        n_l, ms_l = fc.profile_read("layer")
        its, st = np.concatenate(its), np.concatenate(st)
        act = (L - 2) * int(its.sum()) / max(n_l, 1)
        us = ms_l / max(n_l, 1) * 1e3
        tf = (8 * M * C + 2 * C * C) * N * N * act / (us * 1e-6) / 1e12
        out[f"{N}x{N}x64"] = {"solves_per_sec": round(64 * steps / total, 2),
                              "converged_per_sec": round(float((st == 0).sum()) / total, 2),
                              "converged": int((st == 0).sum()), "of": int(st.size),
                              "p50_ms": round(float(np.percentile(lat, 50)), 1),
                              "p99_ms": round(float(np.percentile(lat, 99)), 1),
                              "iters_median": float(np.median(its)), "iters_max": int(its.max()),
                              "inner_layer_avg_us": round(us, 2), "inner_layer_TFLOPs": round(tf, 1),
                              "inner_layer_mfma_frac": round(tf / 157.3, 4)}
        log(f"batched {N}: {out[f'{N}x{N}x64']}", logf)
    return out


def config0(fc, torch, dev, logf, solves=10):
    """The single-solve parity configuration: 32 x 32, k = exp(GRF) (no
    contrast rescaling), f ~ GRF, u0 ~ N(0, I), operator with 4 layers, width
    16 and 8 modes at its seeded initial weights in FP64, m = 5, tol 1e-6, at
    most 300 iterations.  Latency-bound: reported per iteration and per solve."""
    import synth
    N, C, M, L = 32, 16, 8, 4
    k, f, u0, _ = synth.system(0, N)
    model = fc.Model(synth.init_weights(0, C, M, L), C, M, L)
    kd, fd, ud = [torch.from_numpy(a)[None].to(dev).contiguous() for a in (k, f, u0)]
    ws = torch.empty(fc.solve_workspace_bytes(model, N, 1, "fp64", 5, 300, 1e-6), dtype=torch.uint8, device=dev)
    for _ in range(2):
        fc.solve(model, kd, fd, ud.clone(), op="fp64", m_max=5, max_iter=300, rtol=1e-6, hist=False, workspace=ws)
    torch.cuda.synchronize()
    lat, its = [], []
    for _ in range(solves):
        u = ud.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        o = fc.solve(model, kd, fd, u, op="fp64", m_max=5, max_iter=300, rtol=1e-6, hist=False, workspace=ws)
        lat.append(time.perf_counter() - t0)
        its.append(int(o["iters"][0]))
    model.close()
    lat = np.array(lat)
    out = {"grid": N, "width": C, "modes": M, "layers": L, "op": "fp64", "weights": "seeded initial",
           "iters": its[-1], "status": int(o["status"][0]),
           "true_rel_res": float(o["true_rel_res"][0]), "true_rel_res_f": float(o["true_rel_res_f"][0]),
           "us_per_iteration": round(float(np.median(lat)) / max(its[-1], 1) * 1e6, 2),
           "solves_per_sec": round(1.0 / float(np.median(lat)), 3),
           "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
           "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3)}
    log(f"config0: {out}", logf)
    return out


def training_throughput(fc, torch, dev, C, M, L, steps, logf, N=64, B=256, m_iter=100):
    """The training configuration: 256 seeded 64 x 64 systems (k = exp(GRF)
    rescaled to contrast 10..1e3), Krylov samples of 100 conjugate-gradient
    iterations each (Sec. 3.1), train steps at batch 256 (one sample per
    system, the iteration drawn at random) with the FP32 operator: forward,
    energy-norm loss, hand-written backward and AdamW.  The operator starts
    from the seeded initial weights (projection scaled by 1e-3)."""
    import synth
    blob = synth.init_weights(3, C, M, L)
    blob[blob.size - C - 1:] *= 1e-3
    model = fc.Model(blob, C, M, L)
    k, f, u0, _ = synth.batch(3, B, N, (10.0, 1000.0))
    kd, fd, ud = [torch.from_numpy(a).to(dev) for a in (k, f, u0)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r, e = fc.krylov_samples(kd, fd, ud, m_iter=m_iter)
    torch.cuda.synchronize()
    t_samples = time.perf_counter() - t0
    opt = fc.Optim(model, lr=3e-4, weight_decay=1e-2)
    ws = fc.train_workspace(model, N, B, "fp32", dev)
    g = torch.Generator(device=dev)
    g.manual_seed(99)
    ar = torch.arange(B, device=dev)
    pick = torch.randint(0, m_iter, (steps + 10, B), generator=g, device=dev)
    batches = [(r[ar, pick[s]].contiguous(), e[ar, pick[s]].contiguous()) for s in range(steps + 10)]
    losses = []
    for s in range(10):
        fc.train_step(model, opt, kd, batches[s][0], batches[s][1], op="fp32", workspace=ws, return_loss=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        rb, eb = batches[10 + s]
        want = s == 0 or s == steps - 1
        v = fc.train_step(model, opt, kd, rb, eb, op="fp32", workspace=ws, return_loss=want)
        if want:
            losses.append(v)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    opt.close()
    model.close()
    out = {"grid": N, "batch": B, "op": "fp32", "samples": f"CG iterations 1..{m_iter} of {B} systems",
           "sample_seconds": round(t_samples, 3), "steps": steps, "seconds": round(dt, 3),
           "steps_per_sec": round(steps / dt, 2), "ms_per_step": round(dt / steps * 1e3, 3),
           "loss_first_timed": round(losses[0], 4), "loss_last_timed": round(losses[-1], 4)}
    log(f"training throughput: {out}", logf)
    return out


def krylov_bytes_per_point(i, m_max=5):
    """Algorithmic HBM bytes per grid point of the three Krylov kernels at
    iteration i (Algorithm 1, window m_i): (w, s_k) reads w and the m_i
    s-vectors; the direction kernel reads w, the m_i p-vectors, r and k and
    writes p_i and s_i; the update reads u, p_i, r, s_i and writes u and r."""
    mi = min(i, max(1, i % (m_max + 1)))
    return {"wdots": 8 * (mi + 1) if mi > 0 else 0, "dir": 8 * (mi + 5), "update": 48}


def all_active_kernels(fc, torch, model, kd, fd, u0d, op, C, M, L, S, logf, iters=24):
    """Per-kernel averages over a solve of the whole batch stopped after
    ``iters`` iterations, before any system can reach the tolerance, so every
    launch carries every system (events around each kernel family)."""
    B, N = fd.shape[0], fd.shape[-1]
    kinds = ["layer", "layer_feat", "layer_proj", "spectral", "rowdft", "wdots", "dir", "update"]
    fc.profile_reset()
    fc.profile_enable(True, kinds)
    o = fc.solve(model, kd, fd, u0d.clone(), op=op, m_max=5, max_iter=iters, rtol=1e-300, hist=False)
    torch.cuda.synchronize()
    fc.profile_enable(False)
    if not all(int(x) == iters for x in o["iters"]):
        log(f"all-active solve: iteration counts {o['iters']}", logf)
    out = {"iterations": iters, "systems": B}
    tot = {"wdots": 0, "dir": 0, "update": 0}
    for i in range(iters):
        for kname, v in krylov_bytes_per_point(i).items():
            tot[kname] += v * N * N * B
    esize = {"bf16": 2, "fp32": 4, "fp64": 8}[op]
    lb = layer_bytes_per_launch(N, B, C, M, esize, 8 if op == "fp64" else 4, S)
    it_us = 0.0
    for name in kinds:
        n_, ms_ = fc.profile_read(name)
        avg = ms_ / max(n_, 1) * 1e3
        it_us += ms_ * 1e3 / iters
        d = {"launches": n_, "avg_us": round(avg, 2)}
        if name in tot and n_ == 0:
            d["note"] = "no launches: formed in the projection layer's epilogue"
        elif name in tot:
            gbs = tot[name] / max(ms_ * 1e-3, 1e-30) / 1e9
            d.update({"GBs": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
                      "bytes_per_launch": round(tot[name] / max(n_, 1))})
        if name == "layer":
            gbs = lb / (avg * 1e-6) / 1e9
            d.update({"GBs": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_launch": lb})
        out[name] = d
    out["sum_of_kernel_us_per_iteration"] = round(it_us, 1)
    log(f"all-active ({iters} iterations x {B} systems): " +
        ", ".join(f"{k} {v['avg_us']} us" for k, v in out.items() if isinstance(v, dict)), logf)
    return out


def time_solves(fc, torch, model, kd, fd, u0d, op, steps, warmup, args, prof_kernels=None, streams=0):
    B = fd.shape[0]
    N = fd.shape[-1]
    ws = torch.empty(fc.solve_workspace_bytes(model, N, B, op, 5, args.max_iter, args.rtol),
                     dtype=torch.uint8, device=fd.device)
    us = [u0d.clone() for _ in range(steps + warmup)]
    outs = []
    for w in range(warmup):
        fc.solve(model, kd, fd, us[w], op=op, m_max=5, max_iter=args.max_iter, rtol=args.rtol,
                 hist=False, workspace=ws, streams=streams)
    torch.cuda.synchronize()
    if prof_kernels:
        fc.profile_reset()
        fc.profile_enable(True, prof_kernels)
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        ts = time.perf_counter()
        outs.append(fc.solve(model, kd, fd, us[warmup + s], op=op, m_max=5, max_iter=args.max_iter,
                             rtol=args.rtol, hist=False, workspace=ws, streams=streams))
        lat.append(time.perf_counter() - ts)   # the call returns after the batch completed
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    prof = {}
    if prof_kernels:
        fc.profile_enable(False)
        for name in prof_kernels:
            prof[name] = fc.profile_read(name)
    return total, lat, outs, us[-1], prof


def serving(fc, torch, dev, model, n_req, logf):
    """Serving leg: requests with grids uniform over {64,...,1024}^2 (k
    contrast log-uniform in [10, 1e3], f ~ GRF, u0 ~ N(0, I)), BF16 operator,
    tol 1e-6, through the continuous-batching engine.  A closed-loop run (all
    requests at t = 0) measures the saturation rate mu; open-loop runs with
    Poisson arrivals at 0.5 mu and 0.9 mu measure latency under load."""
    import synth
    sizes = [64, 128, 256, 512, 1024]
    g = np.random.default_rng(4242)
    grids = [int(sizes[i]) for i in g.integers(0, len(sizes), n_req)]
    reqs = []
    for i, N in enumerate(grids):
        k, f, u0, _ = synth.system(4000 + i, N, (10.0, 1000.0))
        reqs.append([torch.from_numpy(a).to(dev) for a in (k, f, u0)])
    torch.cuda.synchronize()

    def run(arrivals):
        eng = fc.Engine(model, op="bf16", m_max=5, check_every=8, max_slots=64, budget_bytes=24 << 30)
        us = [r[2].clone() for r in reqs]
        torch.cuda.synchronize()
        ids, t_arr, t_sub, t_done, res = {}, {}, {}, {}, {}
        order = np.argsort(arrivals, kind="stable")
        nxt = 0
        t0 = time.perf_counter()
        while len(res) < n_req:
            now = time.perf_counter() - t0
            while nxt < n_req and arrivals[order[nxt]] <= now:
                i = int(order[nxt])
                k, f, _ = reqs[i]
                ids[eng.submit(k, f, us[i], rtol=1e-6, max_iter=max(2 * grids[i], 300))] = i
                # latency counts from the arrival, including the wait for the
                # engine step that was running when the request arrived
                t_arr[i] = float(arrivals[i])
                t_sub[i] = time.perf_counter() - t0
                nxt += 1
            active, queued = eng.step()
            for r in eng.poll():
                i = ids[r["id"]]
                t_done[i] = time.perf_counter() - t0
                res[i] = r
            if active == 0 and queued == 0 and nxt < n_req:
                time.sleep(max(0.0, arrivals[order[nxt]] - (time.perf_counter() - t0)))
        total = time.perf_counter() - t0
        eng.close()
        lat = np.array([t_done[i] - t_arr[i] for i in range(n_req)]) * 1e3
        wait = np.array([t_sub[i] - t_arr[i] for i in range(n_req)]) * 1e3
        conv = np.array([res[i]["status"] == 0 for i in range(n_req)])
        return total, lat, conv, res, wait

    t_closed, lat_c, conv_c, res_c, _ = run(np.zeros(n_req))
    mu = n_req / t_closed
    open_loop = {}
    for load in (0.5, 0.9):
        lam = load * mu
        arr = np.cumsum(np.random.default_rng(4343).exponential(1.0 / lam, n_req))
        arr -= arr[0]
        t_open, lat_o, conv_o, _, wait_o = run(arr)
        open_loop[f"{load:g}_mu"] = {"arrival_rate_per_sec": round(lam, 3), "seconds": round(t_open, 3),
                                     "solves_per_sec": round(n_req / t_open, 3),
                                     "converged_per_sec": round(float(conv_o.sum()) / t_open, 3),
                                     "p50_ms": round(float(np.percentile(lat_o, 50)), 1),
                                     "p99_ms": round(float(np.percentile(lat_o, 99)), 1),
                                     "submit_wait_p50_ms": round(float(np.percentile(wait_o, 50)), 1),
                                     "submit_wait_p99_ms": round(float(np.percentile(wait_o, 99)), 1)}
        log(f"serving: open-loop at {lam:.2f}/s: {t_open:.2f}s p50 {np.percentile(lat_o, 50):.0f} ms "
            f"p99 {np.percentile(lat_o, 99):.0f} ms", logf)
    by_n = {}
    for N in sizes:
        it = [res_c[i]["iters"] for i in range(n_req) if grids[i] == N]
        ok = [res_c[i]["status"] == 0 for i in range(n_req) if grids[i] == N]
        if it:
            by_n[str(N)] = {"requests": len(it), "converged": int(sum(ok)), "iters_median": float(np.median(it))}
    log(f"serving: closed {t_closed:.2f}s mu={mu:.2f}/s", logf)
    return {"requests": n_req, "grids": sizes, "op": "bf16", "tol": 1e-6,
            "latency": "from the request's arrival (closed loop: t = 0) to its result being polled",
            "closed_loop": {"seconds": round(t_closed, 3), "solves_per_sec": round(mu, 3),
                            "converged_per_sec": round(float(conv_c.sum()) / t_closed, 3),
                            "p50_ms": round(float(np.percentile(lat_c, 50)), 1),
                            "p99_ms": round(float(np.percentile(lat_c, 99)), 1)},
            "open_loop": open_loop,
            "by_grid": by_n}


def copy_bandwidth(torch, dev):
    """Device-to-device copy of 1 GiB (read + write), GB/s: the bandwidth a
    plain streaming kernel with a 1:1 read/write mix reaches on this GPU."""
    a = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(5):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    bw = 5 * 2 * a.numel() * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    return bw


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(k, f, u0, blob, C, M, L, iters_needed, conv_frac, seconds, logf, kb=None, fb=None,
                 solutions=None):
    """The oracle (FP64 FCG with the FP64 operator) on system 0 of the batch,
    for as many iterations as fit in about ``seconds``; scaled to solves/sec
    with the iteration count the solve needs.  The oracle's time per
    iteration does not depend on the weight values; it runs with the seeded
    initial weights.  With ``solutions`` ({op: (u [B][N][N] device, status
    [B])}), also the oracle's exact solution A^-1 f of two sampled systems
    (those converged under every op, if any) and each op's relative error
    against it, in the 2-norm and the energy norm."""
    import torch
    import oracle
    w = oracle.unpack_weights(blob, C, M, L)
    kt = torch.from_numpy(k)

    def pre(r):
        return oracle.no_apply(w, kt, r)
    # probe one iteration, then size the sample to the time budget
    t0 = time.perf_counter()
    oracle.fcg(k, f, u0, pre, m_max=5, max_iter=1, tol=0.0)
    t1 = time.perf_counter() - t0
    n_it = int(max(2, min(iters_needed, seconds / max(t1, 1e-6))))
    t0 = time.perf_counter()
    oracle.fcg(k, f, u0, pre, m_max=5, max_iter=n_it, tol=0.0)
    dt = time.perf_counter() - t0
    per_iter = dt / n_it
    log(f"cpu oracle: {n_it} iterations in {dt:.1f}s ({per_iter:.3f}s/iter)", logf)
    accuracy = None
    if solutions:
        B = next(iter(solutions.values()))[1].shape[0]
        ok_all = np.ones(B, dtype=bool)
        for _, st in solutions.values():
            ok_all &= st == 0
        picks = [int(b) for b in np.nonzero(ok_all)[0][:2]] or [0, 1]
        accuracy = {"systems": picks, "reference": "oracle exact solve A^-1 f (sparse direct, FP64)"}
        for b in picks:
            ustar = oracle.exact_solve(kb[b], fb[b])
            kt_b = torch.from_numpy(kb[b])
            en_star = float(oracle.energy_norm(kt_b, torch.from_numpy(ustar)))
            for op, (u, st) in solutions.items():
                ub = u[b].cpu().numpy()
                d = ub - ustar
                accuracy.setdefault(op, {})[str(b)] = {
                    "status": int(st[b]),
                    "rel_err_2": float(np.linalg.norm(d) / np.linalg.norm(ustar)),
                    "rel_err_A": float(oracle.energy_norm(kt_b, torch.from_numpy(d))) / en_star}
        log(f"accuracy vs oracle: {accuracy}", logf)
    return {"value": conv_frac / (per_iter * iters_needed), "unit": "solves/sec", "cores": torch.get_num_threads(),
            "host_cpus": os.cpu_count(), "host_cpu_model": cpu_model(),
            "kind": "oracle", "accuracy_vs_oracle": accuracy,
            "sample": f"first {n_it} FCG iterations (FP64 operator, m=5) of system 0 of the batch, "
                      f"{per_iter:.3f} s/iteration, scaled by the {iters_needed} iterations the batch's "
                      f"FP64-operator solves took on average and by the fraction {conv_frac:.3f} of them "
                      f"that reached the tolerance"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported (the library has no "
              "multi-GPU path; the batch of independent solves would shard by system).", file=sys.stderr)
        sys.exit(2)
    logf = open(args.log, "a") if args.log else None
    import torch
    import paper_2402_05598_amd as fc
    import synth
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    N, B, C, M, L = args.n, args.batch, 32, 12, 4
    ops = args.ops.split(",")
    if args.max_iter <= 0:
        args.max_iter = max(2 * N, 300)

    if args.calibrate_copy:
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev)
        a.fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB written", logf)
        del a, b

    if not args.train_operator:
        wb = np.load(args.weights).astype(np.float64)
        model = fc.Model(wb, C, M, L)
        train_info = {"loaded": os.path.relpath(args.weights, ROOT),
                      "sha256_16": hashlib.sha256(wb.tobytes()).hexdigest()[:16]}
    else:
        # the benchmark's operator: 1024 training systems, lr 6e-4 (measured
        # best on the 512^2 batch among 256/1024 systems, lr 3e-4 .. 1e-3)
        model, train_info = train_operator(fc, torch, dev, C, M, L, args.train_steps, logf, Bs=1024, lr=6e-4)
        if args.save_weights:
            np.save(args.save_weights, model.get_weights())
    k, f, u0, contrasts = synth.batch(2, B, N, (10.0, 1000.0))
    kd, fd, u0d = [torch.from_numpy(a).to(dev) for a in (k, f, u0)]
    torch.cuda.synchronize()
    log(f"workload N={N} B={B} contrasts {min(contrasts):.1f}..{max(contrasts):.1f}", logf)

    results = {}
    prof = None
    for j, op in enumerate(ops):
        steps = args.steps if j == 0 else max(1, min(args.steps, 2))
        # only the layer kernel carries events in the timed region (events
        # around every kernel family cost about 8% of an iteration)
        pk = ["layer"]
        total, lat, outs, ulast, pr = time_solves(fc, torch, model, kd, fd, u0d, op, steps,
                                                  args.warmup if j == 0 else 0, args, pk)
        if j == 0:
            prof = pr
        iters = np.concatenate([o["iters"] for o in outs])
        status = np.concatenate([o["status"] for o in outs])
        tres = np.concatenate([o["true_rel_res"] for o in outs])
        tresf = np.concatenate([o["true_rel_res_f"] for o in outs])
        results[op] = {"seconds": total, "steps": steps, "lat": lat, "iters": iters, "status": status,
                       "tres": tres, "tresf": tresf, "u": ulast, "prof": pr}
        log(f"op={op}: {steps} solves in {total:.3f}s, iters mean {iters.mean():.1f} max {iters.max()}, "
            f"status {np.bincount(status, minlength=4).tolist()}, true rel res max {tres.max():.2e}", logf)

    main_op = ops[0]
    R = results[main_op]
    if args.streams > 1:
        # the same solves with the batch split over several streams (identical bits)
        total, lat, outs, ulast, _ = time_solves(fc, torch, model, kd, fd, u0d, main_op, max(1, min(args.steps, 3)),
                                                 1, args, None, streams=args.streams)
        iters = np.concatenate([o["iters"] for o in outs])
        status = np.concatenate([o["status"] for o in outs])
        results[f"{main_op}_streams{args.streams}"] = {"seconds": total, "steps": len(outs), "lat": lat, "iters": iters,
                                                       "status": status,
                                                       "tres": np.concatenate([o["true_rel_res"] for o in outs]),
                                                       "tresf": np.concatenate([o["true_rel_res_f"] for o in outs]),
                                                       "u": ulast}
        assert np.array_equal(iters[-B:], R["iters"][-B:]) and torch.equal(ulast, R["u"]), \
            "sub-batched solve differs from the single-stream solve"
        log(f"op={main_op} streams={args.streams}: {len(outs)} solves in {total:.3f}s", logf)
    ms_per_step = R["seconds"] / R["steps"] * 1e3
    # solves that reached the tolerance, per second of the timed steps
    value = float((R["status"] == 0).sum()) / R["seconds"]
    lat_ms = np.array(R["lat"]) * 1e3

    # Roofline of the inner layer kernel.  Systems that have stopped leave
    # their blocks at once, so a launch moves the bytes of its active systems
    # only: (L - 2) inner-layer launches per iteration of each system, i.e.
    # (L - 2) * sum(iters) active system-launches over the timed solves.
    esize = {"bf16": 2, "fp32": 4, "fp64": 8}[main_op]
    asize = 8 if main_op == "fp64" else 4
    # one partial spectrum per row: the bytes the layer's job needs (a wave
    # that holds a whole row writes just that; the tail's one-segment-per-wave
    # launches write a partial per segment, which counts as overhead here)
    S = 1
    per_sys = layer_bytes_per_launch(N, 1, C, M, esize, asize, S)
    n_l, ms_l = prof["layer"]
    sys_launches = (L - 2) * int(R["iters"].sum())
    act_avg = sys_launches / max(n_l, 1)
    nb = per_sys * act_avg
    avg_us = ms_l / max(n_l, 1) * 1e3
    achieved = nb / (avg_us * 1e-6) / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as fh:
            tr = json.load(fh)
        if tr.get("kernel_hash") == kernel_hash() and tr.get("grid") == N and tr.get("batch") == B \
                and tr.get("op") == main_op:
            # counters were taken on launches with every system active
            traffic = round(tr["bytes_per_launch_all_active"] * act_avg / B)
    copy_bw = copy_bandwidth(torch, dev)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "copy_GBs": round(copy_bw, 1), "frac_of_copy": round(achieved / copy_bw, 4),
                "kernel": f"k_layer<{main_op}, C={C}, MP=32> inner layer", "launches": n_l,
                "avg_us": round(avg_us, 2), "active_systems_per_launch": round(act_avg, 3),
                "algorithmic_bytes_per_system": per_sys, "algorithmic_bytes_per_launch": round(nb)}

    # per-kernel breakdown from one more (untimed) solve of the same batch
    kinds = ["layer", "layer_feat", "layer_proj", "spectral", "rowdft", "wdots", "dir", "update"]
    fc.profile_reset()
    fc.profile_enable(True, kinds)
    ob = fc.solve(model, kd, fd, u0d.clone(), op=main_op, m_max=5, max_iter=args.max_iter, rtol=args.rtol,
                  hist=False)
    torch.cuda.synchronize()
    fc.profile_enable(False)
    per_kernel = {}
    for name in kinds:
        n_, ms_ = fc.profile_read(name)
        per_kernel[name] = {"launches": n_, "avg_us": round(ms_ / max(n_, 1) * 1e3, 2)}
    per_kernel["note"] = "one untimed solve of the batch with events around every kernel family"
    # Krylov kernels against HBM: algorithmic bytes per point of each
    # iteration (krylov_bytes_per_point) summed over every system's iterations
    kry_bytes = {"wdots": 0, "dir": 0, "update": 0}
    for itb in ob["iters"]:
        for i in range(int(itb)):
            for kname, v in krylov_bytes_per_point(i).items():
                kry_bytes[kname] += v
    krylov = {}
    for name, bpp in kry_bytes.items():
        n_, avg = per_kernel[name]["launches"], per_kernel[name]["avg_us"]
        if n_ == 0:
            krylov[name] = {"note": "no launches: formed in the projection layer's epilogue"}
            continue
        gbs = bpp * N * N / max(n_ * avg * 1e-6, 1e-30) / 1e9
        krylov[name] = {"GBs": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4)}
    per_kernel["krylov_hbm"] = krylov
    per_kernel["all_active"] = all_active_kernels(fc, torch, model, kd, fd, u0d, main_op, C, M, L, S, logf)
    # the operator against the matrix cores: algorithmic flops of an inner
    # layer per point, y-synthesis 2(2M)C + bypass 2C^2 + next y-analysis 2(2M)C
    flops_pt = 8 * M * C + 2 * C * C
    mfma_peak = {"bf16": 2500.0, "fp32": 157.3, "fp64": 78.6}
    operator_util = {}
    for op, Rr in results.items():
        if op not in mfma_peak or "prof" not in Rr:
            continue
        n_l, ms_l = Rr["prof"]["layer"]
        act = (L - 2) * int(Rr["iters"].sum()) / max(n_l, 1)
        us = ms_l / max(n_l, 1) * 1e3
        tf = flops_pt * N * N * act / (us * 1e-6) / 1e12
        esz = {"bf16": 2, "fp32": 4, "fp64": 8}[op]
        gbs = layer_bytes_per_launch(N, 1, C, M, esz, 8 if op == "fp64" else 4, S) * act / (us * 1e-6) / 1e9
        operator_util[op] = {"inner_layer_avg_us": round(us, 2), "TFLOPs": round(tf, 1),
                             "mfma_frac": round(tf / mfma_peak[op], 4), "GBs": round(gbs, 1),
                             "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "flops_per_point": flops_pt}
    comparison = {}
    ref = results.get("fp64")
    for op, Rr in results.items():
        conv = Rr["status"] == 0
        d = {"solves_per_sec": round(B * Rr["steps"] / Rr["seconds"], 3),
             "converged_per_sec": round(float(conv.sum()) / Rr["seconds"], 3),
             "ms_per_solve_batch": round(Rr["seconds"] / Rr["steps"] * 1e3, 2),
             # FCG iterations of all systems per second: the kernels' throughput,
             # far less sensitive than converged solves/s to how well the
             # operator trained at set-up transfers to this grid
             "system_iters_per_sec": round(float(Rr["iters"].sum()) / Rr["seconds"], 1),
             "iters_mean": round(float(Rr["iters"].mean()), 2), "iters_max": int(Rr["iters"].max()),
             "status_counts": {"ok": int(conv.sum()), "not_converged": int((Rr["status"] == 1).sum()),
                               "breakdown": int((Rr["status"] == 2).sum())},
             "true_rel_res_max_converged": float(Rr["tres"][conv].max()) if conv.any() else None,
             "true_rel_res_f_max_converged": float(Rr["tresf"][conv].max()) if conv.any() else None}
        if ref is not None and op != "fp64":
            # same systems, last timed step of each; compare where both converged
            lo, lr_ = Rr["status"][-B:] == 0, ref["status"][-B:] == 0
            both = torch.from_numpy(lo & lr_).to(Rr["u"].device)
            du = torch.linalg.vector_norm(Rr["u"] - ref["u"], dim=(1, 2)) / torch.linalg.vector_norm(ref["u"], dim=(1, 2))
            d["u_rel_diff_vs_fp64_op_max"] = float(du[both].max()) if bool(both.any()) else None
            d["iters_diff_vs_fp64_op"] = (Rr["iters"][-B:] - ref["iters"][-B:]).tolist()
        comparison[op] = d

    if args.main_only:
        args.train_bench_steps = args.serve_requests = 0
        args.no_cpu_baseline = True
    batch_cfg = None if args.main_only else batched(fc, torch, dev, model, C, M, L, logf)
    cfg0 = None if args.main_only else config0(fc, torch, dev, logf)
    train_tp = None
    if args.train_bench_steps > 0:
        train_tp = training_throughput(fc, torch, dev, C, M, L, args.train_bench_steps, logf)

    abl = None
    if args.ablation:
        abl = ablation(fc, torch, dev, C, M, L, args.ablation_steps, logf)

    xres = None
    if args.cross_res:
        xres = cross_resolution(fc, torch, dev, C, M, L, main_op, logf,
                                model64=model if train_info and train_info.get("grid") == 64
                                and train_info.get("steps") == 16000 and train_info.get("systems") == 256
                                and train_info.get("lr") == 3e-4 else None,
                                info64=train_info, sine=args.sine)

    classic = None
    if args.classical:
        classic = classical(fc, torch, dev, model, [int(g) for g in args.classical.split(",")], B, main_op, logf)

    serve = None
    if args.serve_requests > 0:
        serve = serving(fc, torch, dev, model, args.serve_requests, logf)

    cpu = None
    if not args.no_cpu_baseline:
        Rb = results.get("fp64", R)
        iters_needed = int(round(float(Rb["iters"].mean())))
        conv_frac = float((Rb["status"] == 0).mean())
        sols = {op: (Rr["u"], Rr["status"][-B:]) for op, Rr in results.items() if op in ("bf16", "fp32", "fp64")}
        cpu = cpu_baseline(k[0], f[0], u0[0], synth.init_weights(3, C, M, L), C, M, L, iters_needed, conv_frac,
                           args.cpu_seconds, logf, kb=k, fb=f, solutions=sols)

    line = {
        "metric": "solves/sec to 1e-6 rel. residual, BF16-NO vs FP64 FCG-NO; p50/p99 latency",
        "value": round(value, 3), "unit": "solves/sec", "n_gpus": 1, "steps": R["steps"],
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": main_op, "data": "synthetic",
        "config": {"workload": f"FCG-NO solve, {N}x{N} grid, batch {B}, k=exp(GRF) contrast 10..1e3, "
                               f"NO L={L} C={C} M={M} trained on 64x64 systems (committed weights), "
                               f"op {main_op} (FP32 accumulate), "
                               f"FP64 Krylov, m=5, tol {args.rtol:g}",
                   "grid": N, "batch": B, "parallelism": "single GPU"},
        "latency_ms": {"p50": round(float(np.percentile(lat_ms, 50)), 2),
                       "p99": round(float(np.percentile(lat_ms, 99)), 2),
                       "per": "batched solve of all systems (each system's result is returned with the batch)"},
        "comparison": comparison,
        "kernels": per_kernel,
        "operator_utilisation": operator_util,
        "batched_fp32": batch_cfg,
        "single_solve_32x32_fp64": cfg0,
        "training_throughput": train_tp,
        "operator": train_info,
        "serving": serve,
        "ablation": abl,
        "classical": classic,
        "cross_resolution": xres,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    model.close()


if __name__ == "__main__":
    main()
