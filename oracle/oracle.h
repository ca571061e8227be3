/*
 * FP64 CPU oracle for the deep-FBSDE hot path (TEST INFRASTRUCTURE ONLY).
 *
 * Plain, slow, obviously-correct reference of what the GPU library computes:
 * Euler–Maruyama paths of the forward SDE, a Z-network per time step, the
 * Euler step of the BSDE driven by the driver phi, the terminal-mismatch
 * loss and its exact gradient by a hand-written reverse sweep.
 *
 *   Güler, Laignelet, Parpas, "Towards Robust and Stable Deep Learning
 *   Algorithms for FBSDEs" (arXiv 1910.11623):
 *     Sec. 2.1 eq. (coupled)            : the FBSDE system and Y=u, Z=grad u
 *     Sec. 2.2 eq. (disc equations)     : Euler–Maruyama for X and Y
 *     Sec. 2.2 eq. (loss), terminal term: sum_m |Y_N - g(X_N)|^2
 *     Sec. 2.2, related-work paragraph  : one network per step, Y0 and Z0
 *                                         trainable parameters
 *     Sec. 3.1 eq. (ode)                : residual block = forward Euler step
 *     Sec. 3.2                          : multilevel time grids h_l = h_0 2^-l
 *     Sec. 4.1                          : Adam optimiser
 *
 * Only tests/, the smoke check and the bench's cpu_baseline leg may load this
 * library; the product path never does.  It shares no code with the GPU
 * library: its Philox generator, layouts and arithmetic are written here
 * independently from their published definitions.
 */
#ifndef FBSDE_ORACLE_H
#define FBSDE_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* forward SDE families (mu = 0 in every problem of Sec. 4) */
enum { ORC_SDE_GBM_DIAG = 0,   /* sigma(x) dW = s * x (.) dW          */
       ORC_SDE_SCALED_BM = 1 };/* sigma(x) dW = s * dW                */
/* drivers phi(t,x,y,z), convention dY = phi dt + Z^T sigma dW          */
enum { ORC_DRV_BSB = 0,        /* r (y - z.x)            p0 = r        */
       ORC_DRV_HJB = 1,        /* lam |z|^2              p0 = lam      */
       ORC_DRV_AC = 2,         /* y^3 - y                              */
       ORC_DRV_LINEAR = 3 };   /* a y + b                p0 = a, p1 = b */
/* terminal conditions g(x) */
enum { ORC_G_NORM2 = 0,        /* |x|^2                                */
       ORC_G_LOGHALF = 1,      /* ln((1 + |x|^2) / 2)                  */
       ORC_G_INV = 2,          /* 1 / (a + b |x|^2)      p0 = a, p1 = b */
       ORC_G_LINEAR = 3 };     /* a * sum_i x_i + c      p0 = a, p1 = c */

typedef struct {
  int d;
  double T;
  const double *x0;            /* [d] */
  int sde;  double sde_s;
  int drv;  double drv_p[2];
  int g;    double g_p[2];
} orc_problem;

enum { ORC_NET_PER_STEP_MLP = 0, ORC_NET_SHARED_RESNET = 1 };

typedef struct {
  int kind;
  int width;
  int depth;   /* MLP: number of hidden tanh layers; ResNet: residual blocks */
  int bf16;    /* 1: round every GEMM operand to bfloat16 (RNE via fp32)    */
} orc_net;

/* Flat parameter layout (row-major W[out][in]):
 *   per-step MLP : z0[d], then for n = 1..N-1:
 *                  W1[w][d] b1[w] (W_l[w][w] b_l[w]) x (depth-1) Wo[d][w] bo[d]
 *   shared ResNet: Win[w][d+1] (column d multiplies t) bin[w],
 *                  (W_k[w][w] b_k[w]) x depth, Wo[d][w] bo[d]
 * y0 is a separate scalar. */
int64_t orc_param_count(const orc_problem *p, const orc_net *net, int N);

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Standard normals xi[n][m][i] (n<N, m<M, i<d) for one iteration.
 * Counter (j, n, m, iter) with j = i/4, key = (seed lo, seed hi); the four
 * words feed two Box–Muller pairs: u0,u1 -> xi[4j], xi[4j+1];
 * u2,u3 -> xi[4j+2], xi[4j+3], with U = ((u >> 8) + 1) 2^-24 in (0,1] under
 * the log and V = (u >> 8) 2^-24 in [0,1) under the angle. */
void orc_normals(uint64_t seed, uint64_t iter, int N, int64_t M, int d, double *xi);

/* Sums over paths (the batch mean of Sec. 2.2 eq. (loss), dL/dY0 and the
 * weight gradients) are formed per chunk of ORC_PATH_CHUNK consecutive paths,
 * each chunk summed from zero in path order, and the chunk partials are added
 * in chunk order.  The association is fixed by this constant alone, so the
 * result does not depend on how many OpenMP threads evaluate the chunks. */
#define ORC_PATH_CHUNK 64

/* One loss evaluation and (optionally) its gradient.
 *   xi      : [N][M][d] normals, or NULL to draw them with orc_normals
 *   grad    : [param_count] or NULL ; grad_y0 : or NULL
 *   XN, YN  : optional outputs [M][d], [M] (terminal states)
 *   Ypath   : optional output [N+1][M]
 * Returns 0 on success, nonzero on invalid arguments. */
int orc_loss_grad(const orc_problem *p, const orc_net *net, int N, int64_t M,
                  const double *params, double y0, const double *xi,
                  uint64_t seed, uint64_t iter,
                  double *loss, double *grad, double *grad_y0,
                  double *XN, double *YN, double *Ypath);

/* Forward sweep of the selected paths idx[0..k) only (same normals as path
 * idx[i] of a full batch): terminal Y_N (YN[k]) and X_N (XN[k][d]), either
 * may be NULL.  Lets a full-size GPU run be checked on sampled paths. */
int orc_paths(const orc_problem *p, const orc_net *net, int N, const double *params, double y0,
              uint64_t seed, uint64_t iter, const int64_t *idx, int64_t k, double *YN, double *XN);

/* Loss of the Euler scheme driven by the exact solution instead of a
 * network: Y_0 = y0 and Z_n = grad u(t_n, X_n) of the Black–Scholes–
 * Barenblatt closed form u = exp((r + s^2)(T - t)) |x|^2 (Sec. 4).  With
 * flip = 1 the driver is used with the opposite sign.  Used to pin the driver
 * convention: the mean terminal mismatch must vanish like O(dt). */
int orc_loss_exact_bsb(const orc_problem *p, int N, int64_t M, double y0,
                       const double *xi, uint64_t seed, uint64_t iter,
                       int flip, double *loss);

/* The Euler scheme of eq. (disc equations) driven by a given Z process
 * instead of a network: Z is [N][M][d] (Z_n of path m), Y_0 = y0, the same
 * normals, diffusion, driver phi and terminal g as orc_loss_grad.  phi enters
 * multiplied by drv_sign (1 for the convention dY = phi dt + Z^T sigma dW).
 * Writes the loss (1/M) sum_m (Y_N - g(X_N))^2.  Fed with Y_0 = u(0, x0) and
 * Z_n = grad u(t_n, X_n) of a problem's exact solution, the mean loss must
 * vanish like O(dt): this pins the driver and terminal branches. */
int orc_loss_given_z(const orc_problem *p, int N, int64_t M, double y0, const double *xi,
                     uint64_t seed, uint64_t iter, const double *Z, double drv_sign, double *loss);

/* Adam (Kingma & Ba 2015), one step t >= 1 on n parameters. */
void orc_adam(int64_t n, double *theta, const double *g, double *m, double *v,
              int64_t t, double lr, double b1, double b2, double eps);

/* Multilevel warm start (Sec. 3.2): per-step nets of a coarse grid with Nc
 * steps copied to a fine grid with Nf = 2 Nc steps; fine net j takes coarse
 * net clamp(floor(j/2), 1, Nc-1); z0 copied.  For the shared ResNet the map
 * is the identity.  Returns 0, or nonzero if Nf != 2 Nc.  The paper gives
 * the level sequence but not this map, so the map itself is a reading:
 * parity unpinned beyond the exact copy it performs. */
int orc_prolong(const orc_problem *p, const orc_net *net, int Nc, int Nf,
                const double *pc, double *pf);

/* Round-to-nearest-even fp64 -> fp32 -> bfloat16 -> fp64 (bf16 emulation). */
double orc_round_bf16(double x);

/* ======================================================================== */
/* The paper's own formulation (Sec. 2.2, eq. (loss); Sec. 3.1)              */
/* ======================================================================== */
/* One network u(t, x; Theta) for every time step; Y_n = u(t_n, X_n) and
 * Z_n = grad_x u(t_n, X_n) (the exact input gradient of the network).  The
 * network takes z = [x; t] (t appended as input d+1) and is
 *   h_0 = tanh(W_0 z + b_0),
 *   h_k = c h_{k-1} + tanh(A_k h_{k-1} (+ E_k z) + b_k),   k = 1..K,
 *   u   = w_o . h_K + b_o,
 * with
 *   FC  : c = 0 (K + 1 fully connected tanh layers of width w),
 *   RES : c = 1 (residual blocks, a forward-Euler step with h = 1, Sec. 3.1),
 *   NAIS: c = 1, A_k = -R_k^T R_k - eps I and the input injection E_k z
 *         (Sec. 3.1, the non-autonomous input-output stable block; the
 *         trainable parameters are R_k, E_k, b_k).
 * Flat layout: W_0[w][d+1] b_0[w]; per block FC/RES: A_k[w][w] b_k[w],
 * NAIS: R_k[w][w] E_k[w][d+1] b_k[w]; then w_o[w] b_o. */
enum { ORC_U_FC = 0, ORC_U_RES = 1, ORC_U_NAIS = 2 };

typedef struct {
  int arch;     /* ORC_U_*                                      */
  int width;    /* w                                            */
  int depth;    /* K blocks after the input layer               */
  double eps;   /* NAIS: A_k = -R_k^T R_k - eps I               */
} orc_unet;

int64_t orc_unet_param_count(const orc_problem *p, const orc_unet *net);

/* Loss of eq. (loss) as a batch mean,
 *   L = (1/M) sum_m [ sum_{n<N} r_n^2 + (u_N - g(X_N))^2 + kappa |Z_N - grad g(X_N)|^2 ],
 *   r_n = u_{n+1} - u_n - phi(t_n, X_n, u_n, Z_n) dt - Z_n . sigma(X_n) dW_n,
 * (the kappa term is the terminal-gradient penalty the paper proposes after
 * eq. (loss); kappa = 0 leaves it out), and its exact gradient with respect
 * to the flat parameters by a hand-written reverse sweep that includes the
 * second-order terms of Z = grad u.  Paths use the same Philox normals as
 * orc_loss_grad (xi NULL) or the given xi [N][M][d].  Optional outputs:
 * U [N+1][M] (u_n of every path), Zout [N+1][M][d].  Returns 0 on success. */
int orc_unet_loss_grad(const orc_problem *p, const orc_unet *net, int N, int64_t M,
                       const double *params, const double *xi, uint64_t seed, uint64_t iter,
                       double kappa, double *loss, double *grad, double *U, double *Zout);

/* The residual loss above with u_n and Z_n given per row instead of a
 * network: U [N+1][M], Z [N+1][M][d].  Fed with the exact solution of a
 * problem, the mean loss must vanish like O(dt) (pins the residual, the
 * driver and the penalty term). */
int orc_unet_loss_given_uz(const orc_problem *p, int N, int64_t M, const double *xi, uint64_t seed,
                           uint64_t iter, const double *U, const double *Z, double kappa, double *loss);

/* u(t, x) and grad_x u(t, x) of the network at given rows: T [R], X [R][d]
 * -> u [R], Z [R][d] (either output may be NULL). */
int orc_unet_eval(const orc_problem *p, const orc_unet *net, const double *params, int64_t R,
                  const double *T, const double *X, double *u, double *Z);

/* NAIS projection (Sec. 3.1): every R_k with |R_k^T R_k|_F > c is scaled by
 * sqrt(c / |R_k^T R_k|_F), so that |R_k^T R_k|_F <= c afterwards. */
int orc_unet_nais_project(const orc_problem *p, const orc_unet *net, double *params, double c);

#ifdef __cplusplus
}
#endif
#endif
