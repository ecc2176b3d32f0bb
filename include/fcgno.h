/*
 * fcgno.h -- C ABI of the FCG-NO hot path on AMD Instinct MI355X (gfx950).
 *
 * The library solves the linear systems A u = f that the 5-point finite
 * difference discretisation of -div(k grad u) = f on the unit square with zero
 * Dirichlet boundary values produces (Sec. 2.1, the general elliptic equation
 * and the linear system it yields), by flexible conjugate gradients
 * (Algorithm 1) preconditioned by a Fourier neural operator B(r; theta)
 * (Sec. 2.4.2), and trains that operator on the energy-norm loss (Sec. 3.1,
 * the error form of the Notay loss).
 *
 * Conventions shared by every entry point
 *   - N interior points per side, h = 1/(N+1).  Interior fields (f, u, r, w,
 *     e) are float64 [batch][N][N], row-major, index [i][j] with j (x2)
 *     contiguous.  Coefficients k are nodal float64 [batch][N+2][N+2]
 *     including the boundary nodes; node (i+1, j+1) is interior point (i, j).
 *   - A is applied as h^-2 [(kE+kW+kN+kS) u_ij - kE u_{i+1,j} - kW u_{i-1,j}
 *     - kN u_{i,j+1} - kS u_{i,j-1}] with face values the mean of the two
 *     nodal values and u = 0 off the interior.
 *   - "device" pointers are HIP device memory of the current device, 8-byte
 *     aligned at least; "host" pointers are ordinary host memory.  The caller
 *     owns every buffer it passes.  Workspaces are caller-allocated device
 *     memory of at least the queried size, 256-byte aligned; the library does
 *     not allocate per call.
 *   - stream is a hipStream_t passed as void* (NULL = the null stream).
 *   - Sizes: N in 1..32768 and batch (or the engine's max_slots) in 1..65535
 *     at every entry point; a solve also needs N^2 * batch <= 4e9.  Outside
 *     these, workspace queries return 0 and calls return FCGNO_E_INVALID.
 *   - Nothing throws across the ABI and nothing aborts.  A negative status
 *     means the call did nothing useful and outputs are undefined; the text of
 *     the last error is available from fcgno_last_error().
 *
 * Operator weight blob (float64, the order every entry point uses):
 *   W_L[C][Cin], b_L[C],
 *   for each of the L layers: Re R[C][C][2M][M], Im R[C][C][2M][M], W[C][C], b[C],
 *   W_P[C], b_P[1].
 * R[c][o][a][ky] mixes input channel c into output channel o at mode
 * (kx, ky) with kx = a for a < M and kx = N - 2M + a otherwise; W[o][c] is the
 * 1x1 bypass.  The operator is B(r) = s * P(layers(lift(phi))) with
 * s = ||r||_2 / N, features phi = [r/s, log k, x1, x2], GELU(z) = z/2
 * (1 + erf(z/sqrt 2)) after every layer; B(0) = 0.
 */
#ifndef FCGNO_H
#define FCGNO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FCGNO_OK = 0,
    FCGNO_NOT_CONVERGED = 1,   /* non-fatal: some system stopped at max_iter or broke down */
    FCGNO_E_INVALID = -1,      /* null pointer, bad size, unsupported architecture */
    FCGNO_E_NOMEM = -2,        /* workspace smaller than required, or device allocation failed */
    FCGNO_E_HIP = -3,          /* a HIP runtime call failed */
} fcgno_status;

/* per-system status of a solve */
enum {
    FCGNO_SYS_OK = 0,            /* ||r_i|| / ||r_0|| <= rtol reached at iteration iters */
    FCGNO_SYS_NOT_CONVERGED = 1, /* max_iter reached */
    FCGNO_SYS_BREAKDOWN = 2,     /* (p_i, A p_i) <= 0 or not finite; the system froze at u_i */
    FCGNO_SYS_NONFINITE = 3,     /* NaN/Inf in k, f or u0, or k <= 0 at a node; nothing done */
};

/* arithmetic precision of the operator B; the Krylov part is always float64 */
enum {
    FCGNO_OP_FP64 = 0,      /* float64 matrix cores */
    FCGNO_OP_FP32 = 1,      /* float32 matrix cores */
    FCGNO_OP_BF16 = 2,      /* bfloat16 inputs on matrix cores, float32 accumulation */
    FCGNO_OP_IDENTITY = 3,  /* B = I: FCG is then conjugate gradients (Fig. 2a) */
    /* classical preconditioners of the comparison in Table 1 (no model):
     * precond_steps sweeps from x_0 = 0 on A x = r */
    FCGNO_OP_JACOBI = 4,    /* x <- x + D^-1 (r - A x) */
    FCGNO_OP_SGS_RB = 5,    /* symmetric Gauss-Seidel in red-black order: red, black, black, red */
};

/* training loss: the energy-norm (Notay) loss of Sec. 2.4, or the Euclidean
 * loss the ablation of Sec. 3.3 compares it with */
enum {
    FCGNO_LOSS_ENERGY = 0,  /* ||w - e||_A / ||e||_A */
    FCGNO_LOSS_L2 = 1,      /* ||w - e||_2 / ||e||_2 */
};

typedef struct {
    int32_t layers;       /* L >= 1 */
    int32_t width;        /* C in {16, 32} */
    int32_t modes;        /* M, 1 <= M <= 16; every solve needs 2M <= N */
    int32_t in_channels;  /* must be 4: [r/s, log k, x1, x2] */
    int32_t basis;        /* FCGNO_BASIS_*: the spectral layers' analysis/synthesis basis */
} fcgno_arch;

/* Basis of the spectral layers (Sec. 2.4.2 leaves the basis open; Sec. 5 names
 * other bases).  FOURIER: the FFT modes kx in {0..M-1} U {N-M..N-1},
 * ky in {0..M-1}, complex mixing.  SINE: the discrete sine (DST-I) modes
 * sin(pi p (x+1)/(N+1)), p = 1..2M along x and 1..M along y, which vanish on
 * the Dirichlet boundary; the mixing uses the real parts of the same weights
 * (the imaginary parts take no part and receive zero gradient). */
enum {
    FCGNO_BASIS_FOURIER = 0,
    FCGNO_BASIS_SINE = 1,
};

typedef struct fcgno_model fcgno_model;

/* Number of float64 values in a weight blob of this architecture. */
size_t fcgno_weight_count(const fcgno_arch* arch);

/* Create a model from a host float64 blob (Sec. 2.4.2, the spectral layers
 * u <- S L A u).  The library copies the weights to the current device in
 * float64, float32 and bfloat16 and owns those copies.  Errors: E_INVALID
 * (null pointer, n_weights mismatch, unsupported width, modes or basis), E_HIP. */
fcgno_status fcgno_model_create(const fcgno_arch* arch, const double* weights_host,
                                size_t n_weights, fcgno_model** out);

/* Copy the current float64 weights (updated by training) to a host blob. */
fcgno_status fcgno_model_get_weights(const fcgno_model* m, double* weights_host, size_t n);

/* Replace the weights from a host blob (same layout); not concurrent with use. */
fcgno_status fcgno_model_set_weights(fcgno_model* m, const double* weights_host, size_t n);

void fcgno_model_destroy(fcgno_model* m);

/* ------------------------------------------------------------------------ */
/* fcgno_solve: Algorithm 1 ("Input: A, B, f, m_max, iter.  Ensure: u_iter,   */
/* r_iter") for a batch of independent systems of the same size.              */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t n;          /* N, interior points per side, >= 1 (>= 2*modes unless IDENTITY) */
    int32_t batch;      /* number of systems, >= 1 */
    int32_t m_max;      /* truncation parameter of Algorithm 1, 1..32 */
    int32_t max_iter;   /* iteration limit ("iter"), >= 1 */
    double rtol;        /* stop at the first i with ||r_i||_2/||r_0||_2 <= rtol, > 0 */
    int32_t op;         /* FCGNO_OP_* */
    int32_t check_every;/* host polls convergence every this many iterations (0 = auto) */
    int32_t precond_steps; /* JACOBI / SGS_RB: sweeps per application, 1..1000 (ignored otherwise) */
    int32_t streams;    /* 0 or 1: every launch on the caller's stream.  2..8: the batch is split
                         * into that many contiguous sub-batches (at most one per system) that run
                         * on library-owned streams forked from and joined back to the caller's
                         * stream, so that one sub-batch's latency-bound kernels overlap another's
                         * bandwidth-bound ones; results are bit-identical to one stream */
} fcgno_solve_desc;

/* Workspace bytes fcgno_solve needs for this model and descriptor
 * (model may be NULL when op is IDENTITY, JACOBI or SGS_RB); 0 on invalid input. */
size_t fcgno_solve_workspace_bytes(const fcgno_model* m, const fcgno_solve_desc* d);

/* Solve, per system b, A_b u_b = f_b from u_b = u0_b.
 *   k       device [batch][N+2][N+2] float64, nodal coefficients (> 0)
 *   f       device [batch][N][N] float64, right-hand sides
 *   u       device [batch][N][N] float64, in: u_0, out: u at the stopping iteration
 *   r_out   device [batch][N][N] float64 or NULL; out: the recurrence residual r_iter
 *   iters   host [batch] int32 out: the stopping iteration i (0 if ||r_0|| = 0)
 *   sys_status host [batch] int32 out: FCGNO_SYS_*
 *   rel_hist host [batch][max_iter+1] float64 or NULL; out: ||r_i||/||r_0||,
 *           i = 0..iters, the rest of each row untouched
 *   true_rel_res host [batch] float64 or NULL; out: ||f - A u||_2 / ||r_0||_2
 *           recomputed from the returned u (the quantity the stopping test of
 *           Table 1 bounds, here for the true rather than the recurrence residual)
 *   true_rel_res_f host [batch] float64 or NULL; out: ||f - A u||_2 / ||f||_2
 *           from the same u (0 if f = 0 and A u = 0; +inf if f = 0 otherwise);
 *           with a random u_0 (Algorithm 1's initialisation) ||r_0|| can
 *           exceed ||f|| by orders of magnitude, so this is the stricter figure
 * The call enqueues on stream, polls convergence from the host and returns
 * when every system has stopped; the outputs are then final.  Returns
 * FCGNO_OK if every system converged, FCGNO_NOT_CONVERGED otherwise. */
fcgno_status fcgno_solve(const fcgno_model* m, const fcgno_solve_desc* d,
                         const double* k, const double* f, double* u, double* r_out,
                         int32_t* iters, int32_t* sys_status, double* rel_hist,
                         double* true_rel_res, double* true_rel_res_f, void* ws, size_t ws_bytes,
                         void* stream);

/* ------------------------------------------------------------------------ */
/* fcgno_precond_apply: w = B(r; theta) (the preconditioner of Sec. 2.4.2).   */
/* ------------------------------------------------------------------------ */

size_t fcgno_precond_workspace_bytes(const fcgno_model* m, int32_t n, int32_t batch, int32_t op);

/* k device [batch][N+2][N+2], r device [batch][N][N] (read only), w device
 * [batch][N][N] out.  op is FP64, FP32 or BF16.  Asynchronous on stream. */
fcgno_status fcgno_precond_apply(const fcgno_model* m, int32_t n, int32_t batch, int32_t op,
                                 const double* k, const double* r, double* w,
                                 void* ws, size_t ws_bytes, void* stream);

/* Scratch-free operator application, for callers that cannot allocate device
 * memory (tight serving loops, harnesses that forbid allocation): w = B(r)
 * exactly as fcgno_precond_apply computes it (the same kernels and bits), with
 * the workspace taken from a static device array of the library of
 * FCGNO_NOALLOC_SCRATCH_BYTES per device, which each device holds from its
 * first call until the process ends.  k, r, w, op and stream as for
 * fcgno_precond_apply; batch <= 64.  Every call on one device shares that
 * device's array and leaves its contents behind (the call clears what must
 * start at zero itself): calls that overlap on one device, on different
 * streams or from different host threads, race and give undefined results;
 * calls ordered on one stream are safe.  The call allocates nothing, but it
 * copies a per-system pointer table from host memory, so it is not meant for
 * stream capture.  Errors: E_INVALID as for fcgno_precond_apply, or batch >
 * 64; E_NOMEM when fcgno_precond_workspace_bytes(m, n, batch, op) exceeds
 * FCGNO_NOALLOC_SCRATCH_BYTES (nothing is launched); E_HIP. */
#define FCGNO_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
fcgno_status fcgno_precond_apply_noalloc(const fcgno_model* m, int32_t n, int32_t batch, int32_t op,
                                         const double* k, const double* r, double* w, void* stream);

/* ------------------------------------------------------------------------ */
/* Training (Sec. 3.1): the operator is trained on the error form of the      */
/* Notay loss, mean_b ||B(r_b) - e_b||_A / ||e_b||_A with e_b = A^-1 r_b, on  */
/* residuals drawn from Krylov subspaces; the backward pass is hand-written.  */
/* Training precisions: FCGNO_OP_FP64 or FCGNO_OP_FP32.  The model's float64  */
/* master weights live on the device and are updated in place.               */
/* ------------------------------------------------------------------------ */
typedef struct fcgno_optim fcgno_optim;

/* AdamW with decoupled weight decay (the optimiser of the training table):
 * theta <- theta (1 - lr wd), then the Adam step with bias-corrected moments.
 * Errors: E_INVALID (lr <= 0, wd < 0, betas outside [0,1), eps <= 0), E_HIP. */
fcgno_status fcgno_optim_create(const fcgno_model* m, double lr, double weight_decay, double beta1,
                                double beta2, double eps, fcgno_optim** out);
fcgno_status fcgno_optim_set_lr(fcgno_optim* o, double lr);
void fcgno_optim_destroy(fcgno_optim* o);

/* Training data drawn from Krylov subspaces (Sec. 3.1, the distribution
 * p_Km; Fig. 2a): u* = A^-1 f by conjugate gradients to 1e-13 relative
 * residual (at most max_iter iterations), then conjugate gradients (FCG with
 * B = I) from u0 for m_iter iterations, keeping after iteration i = 1..m_iter
 * r_out[b][i-1] = r_i and e_out[b][i-1] = u* - u_i (device
 * [batch][m_iter][N][N] each).  k, f, u0 device as for fcgno_solve.  Returns
 * FCGNO_NOT_CONVERGED if some u* missed 1e-13 (the samples are still written);
 * synchronises the stream. */
size_t fcgno_krylov_samples_workspace_bytes(int32_t n, int32_t batch, int32_t max_iter);
fcgno_status fcgno_krylov_samples(int32_t n, int32_t batch, int32_t m_iter, int32_t max_iter,
                                  const double* k, const double* f, const double* u0,
                                  double* r_out, double* e_out, void* ws, size_t ws_bytes, void* stream);

/* Residuals from random right-hand sides (the alternative sampling of the
 * ablation in Sec. 3.3): for device [batch] triples (k, f, u), r_out = f - A u
 * and e_out = A^-1 f - u (device [batch][N][N] each), A^-1 f by conjugate
 * gradients to 1e-13 from u (at most max_iter iterations).  Workspace as for
 * fcgno_krylov_samples; returns FCGNO_NOT_CONVERGED if some A^-1 f missed
 * 1e-13 (the samples are still written); synchronises the stream. */
fcgno_status fcgno_residual_samples(int32_t n, int32_t batch, int32_t max_iter, const double* k,
                                    const double* f, const double* u, double* r_out, double* e_out,
                                    void* ws, size_t ws_bytes, void* stream);

/* Workspace of fcgno_op_forward / fcgno_op_backward / fcgno_train_step. */
size_t fcgno_train_workspace_bytes(const fcgno_model* m, int32_t n, int32_t batch, int32_t op);

/* w = B(r) (device [batch][N][N]) keeping the activations the backward pass
 * needs in ws.  k, r as for fcgno_precond_apply.  Asynchronous. */
fcgno_status fcgno_op_forward(const fcgno_model* m, int32_t n, int32_t batch, int32_t op,
                              const double* k, const double* r, double* w,
                              void* ws, size_t ws_bytes, void* stream);

/* Gradient of L = sum_b <grad_w_b, B(r_b)> with respect to the weights,
 * written to grad_params (device float64, blob order, every entry
 * overwritten), and, if grad_r is not NULL, with respect to the input
 * residuals: grad_r device [batch][N][N] float64 (B(r) = s NO(r/s),
 * s = ||r||_2 / N, differentiated through s too; zero for r = 0, where B is
 * not differentiable).  Must follow fcgno_op_forward with the same model, k,
 * r and ws. */
fcgno_status fcgno_op_backward(const fcgno_model* m, int32_t n, int32_t batch, int32_t op,
                               const double* k, const double* r, const double* grad_w,
                               double* grad_params, double* grad_r, void* ws, size_t ws_bytes,
                               void* stream);

/* Energy-norm loss per system, loss_dev[b] = ||w_b - e_b||_A / ||e_b||_A
 * (device [batch]), and if grad_w is not NULL the gradient of the batch mean,
 * grad_w[b] = A (w_b - e_b) / (batch ||w_b - e_b||_A ||e_b||_A).  Async. */
size_t fcgno_energy_loss_workspace_bytes(int32_t n, int32_t batch);
fcgno_status fcgno_energy_loss(int32_t n, int32_t batch, const double* k, const double* w,
                               const double* e, double* loss_dev, double* grad_w,
                               void* ws, size_t ws_bytes, void* stream);
/* The same for either loss (FCGNO_LOSS_*); the Euclidean gradient is
 * (w_b - e_b) / (batch ||w_b - e_b||_2 ||e_b||_2).  Same workspace. */
fcgno_status fcgno_loss(int32_t loss_kind, int32_t n, int32_t batch, const double* k, const double* w,
                        const double* e, double* loss_dev, double* grad_w, void* ws, size_t ws_bytes,
                        void* stream);

/* One step: forward, loss on (r, e) pairs (device [batch][N][N] each),
 * backward, AdamW update of the model.  loss_host (nullable) receives the
 * batch-mean loss before the update; the call then synchronises the stream. */
fcgno_status fcgno_train_step(fcgno_model* m, fcgno_optim* opt, int32_t n, int32_t batch, int32_t op,
                              const double* k, const double* r, const double* e, double* loss_host,
                              void* ws, size_t ws_bytes, void* stream);
/* The same step with the loss chosen (FCGNO_LOSS_*); fcgno_train_step is
 * this with FCGNO_LOSS_ENERGY. */
fcgno_status fcgno_train_step_loss(fcgno_model* m, fcgno_optim* opt, int32_t n, int32_t batch, int32_t op,
                                   int32_t loss_kind, const double* k, const double* r, const double* e,
                                   double* loss_host, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------ */
/* Serving engine: continuous batching of solves (one system per request, any */
/* grid size).  A request waits in a FIFO queue until a slot and a block of   */
/* the engine's device pool (allocated once, budget_bytes) hold its state;     */
/* admitted requests of one N advance together, check_every iterations of      */
/* Algorithm 1 per fcgno_engine_step, with the kernels of fcgno_solve; systems */
/* at different iterations share launches.  A request's result depends only on */
/* its own inputs and N: it is the same alone and in any mix.  k, f and u      */
/* (in: u0, out: u_iter) are device buffers owned by the caller until the      */
/* request is reported by fcgno_engine_poll.  All work runs on the engine's     */
/* stream; fcgno_engine_step synchronises it.  One thread at a time.           */
/* ------------------------------------------------------------------------ */
typedef struct fcgno_engine fcgno_engine;
typedef struct {
  int32_t op;            /* FCGNO_OP_*, as for fcgno_solve */
  int32_t m_max;         /* truncation window, 1..32 */
  int32_t check_every;   /* iterations per step (<= 0: 8) */
  int32_t max_slots;     /* admitted requests at most */
  size_t budget_bytes;   /* device pool for request state and per-N tables */
} fcgno_engine_desc;
typedef struct {
  int64_t id;
  int32_t status;        /* FCGNO_SYS_* */
  int32_t iters;
  double true_rel_res;   /* ||f - A u|| / ||r0|| */
  double true_rel_res_f; /* ||f - A u|| / ||f|| (as for fcgno_solve) */
} fcgno_engine_result;

/* Device bytes one request of grid n takes from the pool (0 if invalid). */
size_t fcgno_engine_request_bytes(const fcgno_model* m, const fcgno_engine_desc* d, int32_t n, int32_t max_iter);
fcgno_status fcgno_engine_create(const fcgno_model* m, const fcgno_engine_desc* d, void* stream,
                                 fcgno_engine** out);
/* Queue a request; FCGNO_E_NOMEM if it can never fit the budget. */
fcgno_status fcgno_engine_submit(fcgno_engine* e, int32_t n, const double* k, const double* f, double* u,
                                 double rtol, int32_t max_iter, int64_t* id_out);
/* Admit what fits, advance every group, report and release stopped requests.
 * A negative status (a failed HIP call) leaves the queue and the slots in an
 * unspecified state: the engine can only be destroyed, after which the
 * buffers of unreported requests belong to the caller again. */
fcgno_status fcgno_engine_step(fcgno_engine* e, int32_t* n_active, int32_t* n_queued);
/* Move up to max_results finished requests into out; returns the count. */
int32_t fcgno_engine_poll(fcgno_engine* e, fcgno_engine_result* out, int32_t max_results);
/* Waits for the engine's work, then frees its streams and pool. */
void fcgno_engine_destroy(fcgno_engine* e);

/* ------------------------------------------------------------------------ */
/* Kernel timing: HIP event pairs recorded on the launch stream around each   */
/* launch of a kernel family while enabled; read after the work completed.    */
/* fcgno_profile_enable takes a bit mask of families (bit k = id k; 0 = off). */
/* kernel ids: 0 operator inner-layer kernel (matrix cores), 1 operator      */
/* spectral kernels (forward DFT, mixing, synthesis), 2 direction+stencil,    */
/* 3 window dots, 4 update, 5 row DFT of r, 6 training forward, 7 training    */
/* backward, 8 first layer kernel (lift fused), 9 last layer kernel           */
/* (projection fused).                                                        */
/* ------------------------------------------------------------------------ */
void fcgno_profile_enable(int32_t mask);
void fcgno_profile_reset(void);
fcgno_status fcgno_profile_read(int32_t kernel, int64_t* launches, double* total_ms);

/* Text of the last error on the calling thread ("" if none). */
const char* fcgno_last_error(void);
const char* fcgno_status_string(fcgno_status s);

#ifdef __cplusplus
}
#endif
#endif /* FCGNO_H */
