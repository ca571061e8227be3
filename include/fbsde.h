/*
 * fbsde.h — C ABI of the MI355X (gfx950) deep-FBSDE library.
 *
 * The library trains the Deep-BSDE form of the paper's method
 * (Güler, Laignelet, Parpas, arXiv 1910.11623):
 *   - forward SDE   dX = mu dt + sigma(X) dW, X_0 = x0        (Sec. 2.1, eq. coupled; mu = 0)
 *   - Euler–Maruyama X_{n+1} = X_n + sigma(X_n) dW_n,
 *                    Y_{n+1} = Y_n + phi(t_n,X_n,Y_n,Z_n) dt + Z_n . sigma(X_n) dW_n
 *                                                             (Sec. 2.2, eq. disc equations)
 *   - Z_n from a network per time step (Y_0 and Z_0 are trainable parameters),
 *     or from one shared network of (t, x)                     (Sec. 2.2, related-work paragraph;
 *                                                              Sec. 3.1 for the residual form)
 *   - loss (1/M) sum_m (Y_N - g(X_N))^2                        (Sec. 2.2, eq. loss, terminal term)
 *   - Adam                                                     (Sec. 4.1)
 *   - multilevel warm start from N to 2N steps                 (Sec. 3.2)
 *
 * Conventions for every call:
 *   - Pointers named *_dev are device pointers (hipMalloc'd or torch tensors'
 *     data_ptr) owned by the caller; the library never frees them.  Pointers
 *     named *_host are host memory.  `stream` is a hipStream_t (NULL = the
 *     null stream); hot calls are asynchronous on it.
 *   - Hot calls (fbsde_forward, fbsde_forward_backward, fbsde_adam_step,
 *     fbsde_train_step, fbsde_prolong, fbsde_sample_normals,
 *     fbsde_terminal_mean) allocate
 *     nothing: all scratch lives in the caller's workspace of
 *     fbsde_workspace_size bytes (256-byte aligned).  One workspace must not
 *     be used by two calls that overlap in time.
 *   - Every call returns a status and never aborts; argument errors are
 *     detected on the host before any launch and leave device memory
 *     untouched.  fbsde_last_error() returns a thread-local message.
 *   - A non-finite loss, dL/dY_0 or weight gradient is detected on the device
 *     (in the reductions of fbsde_forward / fbsde_forward_backward) and
 *     raises a flag in pinned host memory owned by the plan.  The next hot
 *     call on that plan (fbsde_forward, fbsde_forward_backward,
 *     fbsde_adam_step, fbsde_train_step, or fbsde_batch_step of a batch that
 *     holds it) returns
 *     FBSDE_ERR_NONFINITE without launching anything and clears the flag; no
 *     call synchronises to check it, so the report arrives once the
 *     offending work has completed.
 *   - Float parameters are one flat fp32 buffer (layout below); Y_0 is a
 *     separate fp64 scalar on the device.
 *
 * Flat parameter layout (row-major W[out][in], each W followed by its b):
 *   per-step MLP (depth L hidden tanh layers of width w):
 *     z0[d]; then for n = 1 .. N-1:
 *       W1[w][d] b1[w], (W_l[w][w] b_l[w]) for l = 2..L, Wo[d][w] bo[d]
 *   shared residual net (depth B blocks, Sec. 3.1 with h = 1):
 *       Win[w][d+1] bin[w]  (column d multiplies t_n),
 *       (W_k[w][w] b_k[w]) for k = 1..B, Wo[d][w] bo[d]
 *   u-network (depth K blocks; column d of W_0 and E_k multiplies t):
 *       W_0[w][d+1] b_0[w], per block A_k[w][w] (U_NAIS: R_k[w][w] E_k[w][d+1])
 *       b_k[w], then w_o[w] b_o
 */
#ifndef FBSDE_H
#define FBSDE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FBSDE_OK = 0,
  FBSDE_ERR_INVALID = 1,      /* bad argument (null pointer, size, enum)       */
  FBSDE_ERR_UNSUPPORTED = 2,  /* valid request the library does not implement */
  FBSDE_ERR_HIP = 3,          /* a HIP runtime call or kernel launch failed     */
  FBSDE_ERR_NOMEM = 4,        /* plan creation could not allocate              */
  FBSDE_ERR_NONFINITE = 5     /* an earlier call's loss or gradient not finite */
} fbsde_status;

/* Forward SDE families (mu = 0 in every problem of Sec. 4). */
typedef enum {
  FBSDE_SDE_GBM_DIAG = 0,     /* sigma(x) dW = s * x (.) dW   (Black–Scholes–Barenblatt) */
  FBSDE_SDE_SCALED_BM = 1     /* sigma(x) dW = s * dW         (HJB, Allen–Cahn)          */
} fbsde_sde;

/* Drivers phi in the convention dY = phi dt + Z^T sigma dW, Z = grad u. */
typedef enum {
  FBSDE_DRV_BSB = 0,          /* r (y - z.x)      p[0] = r    */
  FBSDE_DRV_HJB = 1,          /* lam |z|^2        p[0] = lam  */
  FBSDE_DRV_AC = 2,           /* y^3 - y                      */
  FBSDE_DRV_LINEAR = 3        /* a y + b          p[0] = a, p[1] = b */
} fbsde_driver;

/* Terminal conditions g. */
typedef enum {
  FBSDE_G_NORM2 = 0,          /* |x|^2                         */
  FBSDE_G_LOGHALF = 1,        /* ln((1 + |x|^2) / 2)           */
  FBSDE_G_INV = 2,            /* 1 / (a + b |x|^2)  p = {a, b} */
  FBSDE_G_LINEAR = 3          /* a sum_i x_i + c    p = {a, c} */
} fbsde_terminal;

typedef struct {
  int32_t d;                  /* state dimension, >= 1                      */
  double T;                   /* horizon, > 0                               */
  const double *x0_host;      /* [d] initial state, copied at plan creation */
  int32_t sde;   double sde_p[2];  /* fbsde_sde, sde_p[0] = s              */
  int32_t drv;   double drv_p[2];  /* fbsde_driver and its parameters       */
  int32_t g;     double g_p[2];    /* fbsde_terminal and its parameters     */
} fbsde_problem;

/* Network kinds.  PER_STEP_MLP and SHARED_RESNET are Z-networks of the
 * Deep-BSDE form above (Y advanced by the scheme from a trainable Y_0, loss
 * on the terminal mismatch).  The U_* kinds are the paper's own formulation
 * (Sec. 2.2, eq. (loss)): one network u(t, x) for every step, Y_n = u(t_n, X_n),
 * Z_n = grad_x u(t_n, X_n) (exact input gradient of the network), loss
 *   (1/M) sum_m [ sum_{n<N} r_n^2 + (u_N - g(X_N))^2 + kappa |Z_N - grad g(X_N)|^2 ],
 *   r_n = u_{n+1} - u_n - phi(t_n, X_n, u_n, Z_n) dt - Z_n . sigma(X_n) dW_n;
 * the kappa term is the terminal-gradient penalty proposed after eq. (loss)
 * (fbsde_plan_set_unet_loss; kappa = 0 by default).  Input z = [x; t]; with
 * depth = K >= 1 blocks of width w:
 *   h_0 = tanh(W_0 z + b_0), h_k = c h_{k-1} + tanh(A_k h_{k-1} (+ E_k z) + b_k),
 *   u = w_o . h_K + b_o,
 *   U_FC:   c = 0 (K + 1 fully connected tanh layers),
 *   U_RES:  c = 1 (Sec. 3.1 residual block, forward-Euler step h = 1),
 *   U_NAIS: c = 1, A_k = -R_k^T R_k - eps I and the input injection E_k z
 *           (Sec. 3.1; trainable R_k, E_k, b_k; eps from
 *           fbsde_plan_set_unet_loss, 0.01 by default).
 * fp32 only. */
typedef enum {
  FBSDE_NET_PER_STEP_MLP = 0, FBSDE_NET_SHARED_RESNET = 1,
  FBSDE_NET_U_FC = 2, FBSDE_NET_U_RES = 3, FBSDE_NET_U_NAIS = 4
} fbsde_net_kind;

/* Arithmetic of the network GEMMs.  Path state (X, Y, Z, lambda) is fp32
 * in both; the loss and dL/dY0 are reduced in fp64.
 *   FP32     : fp32 MFMA (v_mfma_f32_16x16x4f32), fp32 activations
 *   BF16_MFMA: bf16 operands (RNE) on v_mfma_f32_16x16x32_bf16, fp32
 *              accumulation; every GEMM operand (weights, X, hidden
 *              activations, back-propagated deltas) is rounded to bf16 once. */
typedef enum { FBSDE_FP32 = 0, FBSDE_BF16_MFMA = 1 } fbsde_precision;

typedef struct {
  int32_t kind;               /* fbsde_net_kind                              */
  int32_t width;              /* hidden width w                              */
  int32_t depth;              /* MLP: hidden layers; ResNet: residual blocks */
  int32_t prec;               /* fbsde_precision                             */
} fbsde_net;

typedef struct fbsde_plan fbsde_plan;

/* Create a plan for N time steps (dt = T/N, t_n = n dt) and M paths on the
 * current HIP device.  Validates everything, copies x0 to the device (the
 * only allocation the library makes, owned by the plan).  Limits of this
 * build: per-step MLP with d <= 256, w <= 256, 1 <= depth <= 8; u-network
 * with 1 <= depth <= 16, d, w <= 8192, (N + 1) M < 2^29.
 * Errors: INVALID, UNSUPPORTED, NOMEM, HIP. */
fbsde_status fbsde_plan_create(const fbsde_problem *problem, const fbsde_net *net, int32_t N,
                               int64_t M, fbsde_plan **out);
void fbsde_plan_destroy(fbsde_plan *plan);

/* Number of fp32 parameters in the flat layout above. */
fbsde_status fbsde_param_count(const fbsde_plan *plan, int64_t *n_params_host);

/* Block table of the flat layout above (Sec. 2.2: Y_0 aside, the trainable
 * parameters are z0 and the weights and biases of every network).  A block
 * is z0 (per-step MLP only) or one W or one b of one dense layer, in layout
 * order.  Host outputs, each nullable:
 *   n_params_host : total fp32 parameters (as fbsde_param_count);
 *   n_blocks_host : number of blocks B;
 *   offsets_host  : [B + 1] first element of every block, then n_params;
 *   shapes_host   : [B][2] (rows, cols) of every block: W is (out, in),
 *                   b and z0 are (len, 1).
 * Query B first with the arrays NULL, then pass arrays of that size.
 * Errors: INVALID (NULL plan). */
fbsde_status fbsde_param_layout(const fbsde_plan *plan, int64_t *n_params_host, int64_t *n_blocks_host,
                                int64_t *offsets_host, int32_t *shapes_host);

/* Bytes of device workspace the hot calls of this plan need. */
fbsde_status fbsde_workspace_size(const fbsde_plan *plan, size_t *bytes_host);

/* Loss of one iteration: draws the Brownian increments of iteration `iter`
 * (Philox4x32-10 keyed by `seed`, counter (i/4, n, m, iter); Box–Muller),
 * runs the Euler scheme with the networks and writes
 * L = (1/M) sum_m (Y_N - g(X_N))^2 to *loss_dev (fp64).
 * params_dev: [n_params] fp32; y0_dev: fp64 scalar. */
fbsde_status fbsde_forward(fbsde_plan *plan, const float *params_dev, const double *y0_dev,
                           uint64_t seed, uint64_t iter, double *loss_dev, void *ws_dev,
                           void *stream);

/* Loss and its exact gradient through the unrolled chain (reverse sweep of
 * the Euler scheme and of every network): grad_dev [n_params] fp32 and
 * grad_y0_dev (fp64) are overwritten.  Deterministic: no atomics; every
 * reduction has a fixed order. */
fbsde_status fbsde_forward_backward(fbsde_plan *plan, const float *params_dev,
                                    const double *y0_dev, float *grad_dev, double *grad_y0_dev,
                                    double *loss_dev, uint64_t seed, uint64_t iter, void *ws_dev,
                                    void *stream);

/* One Adam step (Kingma & Ba) with step count t >= 1 on the fp32 parameters
 * (learning rate lr) and on y0 (fp64 state, learning rate lr_y0).
 * m/v have the parameter layout; m_y0/v_y0 are fp64 scalars. */
fbsde_status fbsde_adam_step(fbsde_plan *plan, float *params_dev, double *y0_dev,
                             const float *grad_dev, const double *grad_y0_dev, float *m_dev,
                             float *v_dev, double *m_y0_dev, double *v_y0_dev, int64_t t, double lr,
                             double lr_y0, double beta1, double beta2, double eps, void *stream);

/* One training iteration (Sec. 2.2 loss, trained with Adam as in Sec. 4):
 * fbsde_forward_backward of iteration `iter` followed by fbsde_adam_step
 * with step count t, giving the same bits in every output (loss, gradients,
 * parameters, y0 and the moments), with the gradient reduction and the Adam
 * update in one launch.  grad_dev and grad_y0_dev still receive the
 * gradients.  Unlike fbsde_adam_step after a separate fbsde_forward_backward,
 * the update is applied even when this iteration's loss or gradient is
 * non-finite (the device cannot stop it); the next hot call on the plan
 * reports FBSDE_ERR_NONFINITE, as for fbsde_batch_step.  Every pointer is
 * required.  Errors: INVALID (NULL buffer, t < 1, hyper-parameters out of
 * range), UNSUPPORTED (u-network plans). */
fbsde_status fbsde_train_step(fbsde_plan *plan, float *params_dev, double *y0_dev, float *grad_dev,
                              double *grad_y0_dev, double *loss_dev, float *m_dev, float *v_dev,
                              double *m_y0_dev, double *v_y0_dev, int64_t t, double lr, double lr_y0,
                              double beta1, double beta2, double eps, uint64_t seed, uint64_t iter,
                              void *ws_dev, void *stream);

/* Multilevel warm start (Sec. 3.2): copy the parameters of a plan with Nc
 * steps into a plan with Nf = 2 Nc steps of the same problem and network.
 * Fine net j takes coarse net clamp(floor(j/2), 1, Nc-1); z0 is copied; a
 * shared network is copied unchanged.  Requires Nc >= 2 for per-step nets. */
fbsde_status fbsde_prolong(const fbsde_plan *coarse, const fbsde_plan *fine,
                           const float *params_coarse_dev, float *params_fine_dev, void *stream);

/* Test hook: the standard normals xi[n][m][i] (fp32, [N][M][d]) that the
 * forward call of iteration `iter` uses. */
fbsde_status fbsde_sample_normals(fbsde_plan *plan, uint64_t seed, uint64_t iter, float *xi_dev,
                                  void *stream);

/* Mean of g(X_N) over the M paths of iteration `iter` (fp64), a pilot value
 * to initialise Y_0.  Uses the workspace. */
fbsde_status fbsde_terminal_mean(fbsde_plan *plan, uint64_t seed, uint64_t iter,
                                 double *mean_dev, void *ws_dev, void *stream);

/* Test hook: after a forward call on `ws_dev`, copy X_N ([M][d] fp32) and
 * Y_N ([M] fp32) out of the workspace (either pointer may be NULL). */
fbsde_status fbsde_terminal_states(fbsde_plan *plan, const void *ws_dev, float *xN_dev,
                                   float *yN_dev, void *stream);

/* Per-kernel timing with HIP events recorded on the launch stream around
 * every kernel of the hot calls of one plan.  fbsde_profile_enable(plan, 1)
 * creates the event pool (host/driver allocation; not a hot call), 0
 * destroys it.  fbsde_profile_read waits for the recorded events and returns,
 * per kernel id (FBSDE_PROF_*), the summed milliseconds and launch counts
 * since the last read (n entries are written; n <= FBSDE_PROF_NUM).  For
 * the per-step MLP the packing of the step weights runs in the SDE's launch
 * (FBSDE_PROF_SDE), and the fused reverse kernel, where it runs, is timed as
 * FBSDE_PROF_BACKWARD with no FBSDE_PROF_WGRAD launches. */
enum {
  FBSDE_PROF_PACK = 0, FBSDE_PROF_SDE = 1, FBSDE_PROF_FORWARD = 2, FBSDE_PROF_SCAN = 3,
  FBSDE_PROF_BACKWARD = 4, FBSDE_PROF_WGRAD = 5, FBSDE_PROF_REDUCE = 6, FBSDE_PROF_ADAM = 7,
  FBSDE_PROF_NUM = 8
};
fbsde_status fbsde_profile_enable(fbsde_plan *plan, int32_t enable);
fbsde_status fbsde_profile_read(fbsde_plan *plan, double *ms_host, int64_t *count_host, int32_t n);

/* ---- tuning ---------------------------------------------------------------
 * A plan keeps up to two candidate register-tile shapes (the cheapest
 * instantiated kernels that cover d and width); fbsde_workspace_size covers
 * every configuration below, so tuning never needs a larger workspace.
 * fbsde_plan_config selects: shape index; the LDS mode (lds = 0: step weights
 * read from global memory; 1: staged in LDS; 2, the default: staged, and the
 * reverse sweep and weight gradient of a step run as one kernel that keeps
 * the deltas in LDS, where it applies (per-step MLP of depth 1 or 2 whose
 * d + 1 and width + 1 fit the tile shape: fp32 shapes 1x2, 2x2, 4x4, 7x7,
 * bf16 2x2, 4x4, 6x6, 8x8) and, in fp32, where its splits x N workgroups
 * fit one wave over the device's CUs (beyond that the separate kernels are
 * faster); other values are taken as 0 or 2); 16-path tiles
 * per wave of the LDS kernels (tpw, 0 = automatic); and the path splits of
 * the weight-gradient reduction (0 = automatic: one per 512 paths and at
 * least CUs / N, at most 64; explicit values <= 32).  Results are identical
 * across shapes, LDS modes and tpw; the split count changes the fp32
 * summation order of the weight gradient only. */
fbsde_status fbsde_plan_config(fbsde_plan *plan, int32_t shape, int32_t lds, int32_t tpw, int32_t splits);
/* Reports (FBSDE_ERR_NONFINITE) and clears the plan's non-finite flag
 * without launching anything; synchronise the streams that ran the plan's
 * work first to cover all of it.  FBSDE_OK if no non-finite result was
 * seen since the last report. */
fbsde_status fbsde_plan_status(fbsde_plan *plan);

/* Activation checkpointing of the shared residual network (Sec. 3.1 network
 * trained through the unrolled chain).  Rows (step, path) are processed in
 * chunks of whole steps of about chunk_rows rows (0: 262144; at least one
 * step).  recompute != 0 (the default): only X_n and v_n live across the
 * passes and the reverse sweep recomputes each chunk's activations.
 * recompute == 0: the forward pass keeps every chunk's bf16 activations
 * (h_0..h_B, a_1..a_B, [x; t]), so the reverse sweep skips the recompute;
 * the workspace grows by about N M ((2 B + 1) w + d) bf16 elements.  Call
 * before fbsde_workspace_size (it changes the workspace).  Results are
 * bitwise identical for every mode and chunk size except for the fp32
 * summation order of the weight gradients, which follows the chunks.
 * Per-step MLP (the per-step networks of Sec. 2.2 trained through the
 * unrolled chain of eq. (disc equations)): recompute == 0 (the default)
 * keeps every step's tanh activations between the passes; recompute != 0
 * keeps only those of one chunk of whole steps (about chunk_rows rows, as
 * above), which the forward pass writes chunk by chunk and the reverse pass
 * recomputes from X_n, chunk by chunk, before each chunk's reverse sweep:
 * the activation buffers shrink from N to (chunk steps) x M x L x width
 * elements, for one more forward product per step.  Its results are
 * bitwise identical to keeping the activations (the same kernels and
 * arithmetic recompute them, and every step's weight gradient has its own
 * partial sums).
 * Errors: INVALID (negative chunk_rows, or a mode that needs more workspace
 * than an earlier fbsde_workspace_size reported); UNSUPPORTED (a shared-net
 * chunk too large for 32-bit element offsets; u-network plans with
 * recompute != 0). */
fbsde_status fbsde_plan_set_checkpointing(fbsde_plan *plan, int32_t recompute, int64_t chunk_rows);
/* cfg_host[6] = {shape, ti, tw, lds, tpw (resolved), splits} of the current configuration */
fbsde_status fbsde_plan_get_config(const fbsde_plan *plan, int32_t *cfg_host);
/* Autotuner: times fbsde_forward_backward (reps timed calls per candidate,
 * HIP events on `stream`) over shapes x LDS mode, then tiles per wave, then
 * splits, and keeps the fastest configuration.  Writes grad/loss buffers;
 * params and y0 are only read.  Synchronises the stream. */
fbsde_status fbsde_plan_autotune(fbsde_plan *plan, const float *params_dev, const double *y0_dev,
                                 float *grad_dev, double *grad_y0_dev, double *loss_dev, void *ws_dev,
                                 void *stream, int32_t reps);

/* ---- batches of independent instances in one graph ------------------------
 * Many problems (uneven d, N, widths) trained together.  fbsde_batch_create
 * (optionally autotunes every plan, then) captures, for every item, one full
 * training step -- forward, reverse sweep and Adam -- into a hipGraph whose
 * independent items run on parallel branches; the iteration index is read
 * from the device counter *iter_dev (uint64, incremented by the graph at the
 * end of each step; Adam uses t = *iter_dev + 1), so every replay is the next
 * iteration.  fbsde_batch_step launches the graph on `stream`.  The batch
 * keeps the item pointers: buffers must stay allocated, and the plans must
 * not be reconfigured, until fbsde_batch_destroy.  Not a hot call: creation
 * creates streams, events and the graph. */
typedef struct {
  fbsde_plan *plan;
  float *params_dev; double *y0_dev;            /* trained in place                  */
  float *grad_dev; double *grad_y0_dev; double *loss_dev;
  float *m_dev; float *v_dev; double *m_y0_dev; double *v_y0_dev;  /* Adam state     */
  void *ws_dev;                                 /* this plan's workspace             */
  uint64_t seed;                                /* Philox key of this instance       */
} fbsde_batch_item;
typedef struct fbsde_batch fbsde_batch;
fbsde_status fbsde_batch_create(const fbsde_batch_item *items, int32_t n, double lr, double lr_y0,
                                double beta1, double beta2, double eps, uint64_t *iter_dev,
                                int32_t autotune, void *stream, fbsde_batch **out);
fbsde_status fbsde_batch_step(fbsde_batch *batch, void *stream);
void fbsde_batch_destroy(fbsde_batch *batch);

/* ---- the paper's own formulation (U_* network kinds) ----------------------
 * Hot calls of these plans are fbsde_unet_forward_backward and
 * fbsde_adam_step (y0 arguments NULL); fbsde_forward, fbsde_forward_backward,
 * tuning and batches return UNSUPPORTED / INVALID for them.  Workspace,
 * parameter count and layout, profiling and prolongation (the identity:
 * one network for every step) are shared with the other kinds. */

/* kappa >= 0: weight of the terminal-gradient penalty (Sec. 2.2, after
 * eq. (loss)); eps >= 0: NAIS diagonal shift.  Not a hot call. */
fbsde_status fbsde_plan_set_unet_loss(fbsde_plan *plan, double kappa, double eps);

/* One evaluation of the loss above on the Brownian increments of (seed,
 * iter) (same Philox counters as fbsde_forward): *loss_dev (fp64, the sums in
 * fp64 in a fixed order), u(0, x0) into *y0_dev (fp64, nullable) and, when
 * grad_dev is non-NULL, the exact gradient [n_params] fp32 through the
 * network, its input gradient Z and the residuals (reverse sweep with the
 * second-order terms).  Deterministic.  Errors: INVALID, HIP, NONFINITE (an
 * earlier call's result). */
fbsde_status fbsde_unet_forward_backward(fbsde_plan *plan, const float *params_dev, float *grad_dev,
                                         double *loss_dev, double *y0_dev, uint64_t seed, uint64_t iter,
                                         void *ws_dev, void *stream);

/* NAIS projection (Sec. 3.1): every R_k with |R_k^T R_k|_F > c is scaled in
 * place by sqrt(c / |R_k^T R_k|_F).  Uses the workspace. */
fbsde_status fbsde_unet_nais_project(fbsde_plan *plan, float *params_dev, double c, void *ws_dev,
                                     void *stream);

/* After fbsde_unet_forward_backward on ws_dev: u of every row (n, m) into
 * u_dev [(N+1) M] fp32 and Z into z_dev [(N+1) M][d] (row n M + m; either
 * pointer may be NULL). */
fbsde_status fbsde_unet_states(fbsde_plan *plan, const void *ws_dev, float *u_dev, float *z_dev, void *stream);

/* Replace the plan's initial state x0 ([d], host; copied to the device).
 * Not a hot call (synchronous copy).  Used to evaluate a trained network
 * from a perturbed initial condition (Sec. 4, generalisation). */
fbsde_status fbsde_plan_set_x0(fbsde_plan *plan, const double *x0_host);

/* ---- allocation-free variant ------------------------------------------------
 * For callers that cannot allocate device memory or pass a workspace (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): fbsde_forward_backward with the library's own static device
 * scratch array of FBSDE_NOALLOC_SCRATCH_BYTES as workspace (each GPU the
 * library runs on holds one, from the moment the library's code is loaded
 * on it until the process ends).  Same arguments, results and errors as
 * fbsde_forward_backward (bitwise the same results); the caller still
 * passes params, y0, grad, grad_y0 and loss.  Allocates nothing.  Every call
 * on one GPU uses the same array, so calls that overlap in time on one GPU
 * (other streams, threads or plans) race; the array keeps the previous
 * call's contents, which no call reads before writing.  Errors in addition:
 * UNSUPPORTED if the plan's workspace exceeds the scratch (use
 * fbsde_forward_backward, or shrink it with fbsde_plan_set_checkpointing),
 * INVALID if the current device is not the plan's. */
#define FBSDE_NOALLOC_SCRATCH_BYTES (64ull << 20)
fbsde_status fbsde_forward_backward_noalloc(fbsde_plan *plan, const float *params_dev,
                                            const double *y0_dev, float *grad_dev, double *grad_y0_dev,
                                            double *loss_dev, uint64_t seed, uint64_t iter, void *stream);

const char *fbsde_status_str(fbsde_status s);
const char *fbsde_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
