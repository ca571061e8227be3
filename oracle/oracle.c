/*
 * FP64 CPU oracle for the deep-FBSDE hot path.  TEST INFRASTRUCTURE ONLY:
 * loaded by tests/, the smoke check and the bench's cpu_baseline leg, never
 * by the product path.  See oracle.h for the paper passages each routine
 * follows.  Paths are processed one at a time in index order; every sum over
 * paths is accumulated in that fixed order.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from Salmon et al., "Parallel random numbers: as easy as   */
/* 1, 2, 3" (SC'11): ten rounds of two 32x32->64 multiplies, with the key    */
/* advanced by the Weyl constants between rounds.                           */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static const double TWO_PI = 6.283185307179586476925286766559;

/* Box–Muller pair from two 32-bit words (definition in oracle.h) */
static void box_muller(uint32_t ua, uint32_t ub, double *z0, double *z1) {
  double U = ((double)(ua >> 8) + 1.0) * (1.0 / 16777216.0);
  double V = (double)(ub >> 8) * (1.0 / 16777216.0);
  double r = sqrt(-2.0 * log(U));
  *z0 = r * cos(TWO_PI * V);
  *z1 = r * sin(TWO_PI * V);
}

static void normals_one(uint64_t seed, uint64_t iter, int n, int64_t m, int d, double *out) {
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  for (int j = 0; 4 * j < d; ++j) {
    uint32_t ctr[4] = {(uint32_t)j, (uint32_t)n, (uint32_t)m, (uint32_t)iter};
    uint32_t u[4];
    orc_philox4x32_10(ctr, key, u);
    double z[4];
    box_muller(u[0], u[1], &z[0], &z[1]);
    box_muller(u[2], u[3], &z[2], &z[3]);
    for (int k = 0; k < 4 && 4 * j + k < d; ++k) out[4 * j + k] = z[k];
  }
}

void orc_normals(uint64_t seed, uint64_t iter, int N, int64_t M, int d, double *xi) {
  for (int n = 0; n < N; ++n)
    for (int64_t m = 0; m < M; ++m)
      normals_one(seed, iter, n, m, d, xi + ((int64_t)n * M + m) * d);
}

/* ------------------------------------------------------------------------ */
/* bfloat16 emulation: fp64 -> fp32 (RNE) -> bf16 (RNE)                      */
/* ------------------------------------------------------------------------ */
double orc_round_bf16(double x) {
  float f = (float)x;
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (double)f;  /* inf / nan */
  u += 0x7fffu + ((u >> 16) & 1u);
  u &= 0xffff0000u;
  memcpy(&f, &u, 4);
  return (double)f;
}

static double R(const orc_net *net, double x) { return net->bf16 ? orc_round_bf16(x) : x; }

/* ------------------------------------------------------------------------ */
/* Problem pieces: diffusion, driver, its partial derivatives, terminal g   */
/* (Sec. 4 benchmark problems, written in the dY = phi dt + Z^T sigma dW    */
/* convention of eq. (disc equations))                                      */
/* ------------------------------------------------------------------------ */
static void diffusion(const orc_problem *p, const double *x, const double *dw, double *s) {
  for (int i = 0; i < p->d; ++i)
    s[i] = (p->sde == ORC_SDE_GBM_DIAG) ? p->sde_s * x[i] * dw[i] : p->sde_s * dw[i];
}

static double dot(int d, const double *a, const double *b) {
  double s = 0.0;
  for (int i = 0; i < d; ++i) s += a[i] * b[i];
  return s;
}

static double driver(const orc_problem *p, const double *x, double y, const double *z) {
  switch (p->drv) {
    case ORC_DRV_BSB: return p->drv_p[0] * (y - dot(p->d, z, x));
    case ORC_DRV_HJB: return p->drv_p[0] * dot(p->d, z, z);
    case ORC_DRV_AC: return y * y * y - y;
    default: return p->drv_p[0] * y + p->drv_p[1];
  }
}

static double driver_dy(const orc_problem *p, double y) {
  switch (p->drv) {
    case ORC_DRV_BSB: return p->drv_p[0];
    case ORC_DRV_HJB: return 0.0;
    case ORC_DRV_AC: return 3.0 * y * y - 1.0;
    default: return p->drv_p[0];
  }
}

static void driver_dz(const orc_problem *p, const double *x, const double *z, double *out) {
  for (int i = 0; i < p->d; ++i) {
    switch (p->drv) {
      case ORC_DRV_BSB: out[i] = -p->drv_p[0] * x[i]; break;
      case ORC_DRV_HJB: out[i] = 2.0 * p->drv_p[0] * z[i]; break;
      default: out[i] = 0.0; break;
    }
  }
}

static double terminal(const orc_problem *p, const double *x) {
  double q = dot(p->d, x, x);
  switch (p->g) {
    case ORC_G_NORM2: return q;
    case ORC_G_LOGHALF: return log(0.5 * (1.0 + q));
    case ORC_G_INV: return 1.0 / (p->g_p[0] + p->g_p[1] * q);
    default: {
      double s = 0.0;
      for (int i = 0; i < p->d; ++i) s += x[i];
      return p->g_p[0] * s + p->g_p[1];
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Network parameter layout                                                  */
/* ------------------------------------------------------------------------ */
static int64_t mlp_step_count(int d, int w, int L) {
  return (int64_t)w * d + w + (int64_t)(L - 1) * ((int64_t)w * w + w) + (int64_t)d * w + d;
}
static int64_t resnet_count(int d, int w, int B) {
  return (int64_t)w * (d + 1) + w + (int64_t)B * ((int64_t)w * w + w) + (int64_t)d * w + d;
}

int64_t orc_param_count(const orc_problem *p, const orc_net *net, int N) {
  if (net->kind == ORC_NET_PER_STEP_MLP)
    return p->d + (int64_t)(N - 1) * mlp_step_count(p->d, net->width, net->depth);
  return resnet_count(p->d, net->width, net->depth);
}

/* In bf16 mode every GEMM operand is rounded once (R).  The weight blocks
 * arrive already rounded (see rounded_weights); a vector operand is rounded
 * into `buf` once per product instead of once per multiply (same values). */
static const double *rvec(const orc_net *net, int n, const double *v, double *buf) {
  if (!net->bf16) return v;
  for (int i = 0; i < n; ++i) buf[i] = orc_round_bf16(v[i]);
  return buf;
}

/* dense layer: out[o] = sum_i R(W[o][i]) R(in[i]) + b[o] */
static void dense(const orc_net *net, int nout, int nin, const double *W, const double *b,
                  const double *in, double *out, double *buf) {
  const double *x = rvec(net, nin, in, buf);
  for (int o = 0; o < nout; ++o) {
    double s = 0.0;
    for (int i = 0; i < nin; ++i) s += W[(int64_t)o * nin + i] * x[i];
    out[o] = s + b[o];
  }
}

/* transposed product and outer-product accumulation for the reverse sweep */
static void dense_t(const orc_net *net, int nout, int nin, const double *W, const double *delta,
                    double *out_in, double *buf) {
  const double *dl = rvec(net, nout, delta, buf);
  for (int i = 0; i < nin; ++i) {
    double s = 0.0;
    for (int o = 0; o < nout; ++o) s += W[(int64_t)o * nin + i] * dl[o];
    out_in[i] = s;
  }
}
static void outer_acc(const orc_net *net, int nout, int nin, const double *delta, const double *in,
                      double *gW, double *gb, double *buf) {
  const double *x = rvec(net, nin, in, buf);
  for (int o = 0; o < nout; ++o) {
    double dl = R(net, delta[o]);
    for (int i = 0; i < nin; ++i) gW[(int64_t)o * nin + i] += dl * x[i];
    gb[o] += dl;
  }
}

/* Weight blocks of the flat layout rounded to bf16 (biases and z0 are not
 * GEMM operands and stay as they are).  Returns params itself in fp64 mode,
 * else a malloc'd copy the caller frees. */
static double *rounded_weights(const orc_problem *p, const orc_net *net, int N, const double *params) {
  if (!net->bf16) return (double *)params;
  const int d = p->d, w = net->width, L = net->depth;
  const int64_t npar = orc_param_count(p, net, N);
  double *q = (double *)malloc(sizeof(double) * (size_t)(npar > 0 ? npar : 1));
  memcpy(q, params, sizeof(double) * (size_t)npar);
  /* (out, in) of every dense layer of one network */
  int lo[36], li[36], nl = 0;
  if (net->kind == ORC_NET_PER_STEP_MLP) {
    lo[nl] = w; li[nl++] = d;
    for (int l = 1; l < L; ++l) { lo[nl] = w; li[nl++] = w; }
  } else {
    lo[nl] = w; li[nl++] = d + 1;
    for (int k = 0; k < L; ++k) { lo[nl] = w; li[nl++] = w; }
  }
  lo[nl] = d; li[nl++] = w;
  const int nets = net->kind == ORC_NET_PER_STEP_MLP ? N - 1 : 1;
  int64_t off = net->kind == ORC_NET_PER_STEP_MLP ? d : 0;
  for (int n = 0; n < nets; ++n)
    for (int k = 0; k < nl; ++k) {
      for (int64_t e = 0; e < (int64_t)lo[k] * li[k]; ++e) q[off + e] = orc_round_bf16(q[off + e]);
      off += (int64_t)lo[k] * li[k] + lo[k];
    }
  return q;
}

/* Per-step MLP (Sec. 2.2, one network per time step): d -> w tanh
 * (-> w tanh) x (L-1) -> d linear.  acts[l] holds hidden layer l (w values),
 * after the bf16 rounding that the later layers see. */
static void mlp_forward(const orc_problem *p, const orc_net *net, const double *P,
                        const double *x, double *acts, double *z, double *rb) {
  const int d = p->d, w = net->width, L = net->depth;
  const double *W = P, *b = P + (int64_t)w * d;
  dense(net, w, d, W, b, x, acts, rb);
  for (int o = 0; o < w; ++o) acts[o] = R(net, tanh(acts[o]));
  const double *q = b + w;
  for (int l = 1; l < L; ++l) {
    const double *Wl = q, *bl = q + (int64_t)w * w;
    dense(net, w, w, Wl, bl, acts + (int64_t)(l - 1) * w, acts + (int64_t)l * w, rb);
    for (int o = 0; o < w; ++o) acts[(int64_t)l * w + o] = R(net, tanh(acts[(int64_t)l * w + o]));
    q = bl + w;
  }
  dense(net, d, w, q, q + (int64_t)d * w, acts + (int64_t)(L - 1) * w, z, rb);
}

static void mlp_backward(const orc_problem *p, const orc_net *net, const double *P, double *G,
                         const double *x, const double *acts, const double *zeta,
                         double *work /* 2w */, double *rb) {
  const int d = p->d, w = net->width, L = net->depth;
  /* offsets of every layer */
  const int64_t off1 = 0, offb1 = (int64_t)w * d;
  int64_t offh = offb1 + w;  /* first hidden-to-hidden layer */
  int64_t offo = offh + (int64_t)(L - 1) * ((int64_t)w * w + w);
  double *dcur = work, *dnext = work + w;
  /* output layer */
  outer_acc(net, d, w, zeta, acts + (int64_t)(L - 1) * w, G + offo, G + offo + (int64_t)d * w, rb);
  dense_t(net, d, w, P + offo, zeta, dcur, rb);
  for (int l = L - 1; l >= 0; --l) {
    const double *h = acts + (int64_t)l * w;
    for (int o = 0; o < w; ++o) dcur[o] *= (1.0 - h[o] * h[o]);
    if (l == 0) {
      outer_acc(net, w, d, dcur, x, G + off1, G + offb1, rb);
    } else {
      int64_t ow = offh + (int64_t)(l - 1) * ((int64_t)w * w + w);
      outer_acc(net, w, w, dcur, acts + (int64_t)(l - 1) * w, G + ow, G + ow + (int64_t)w * w, rb);
      dense_t(net, w, w, P + ow, dcur, dnext, rb);
      double *t = dcur; dcur = dnext; dnext = t;
    }
  }
}

/* Shared residual network with t as input (Sec. 3.1, residual block as a
 * forward-Euler step of eq. (ode) with h = 1):
 *   h_0 = tanh(Win [x; t] + bin),  h_k = h_{k-1} + tanh(W_k h_{k-1} + b_k),
 *   Z = Wo h_B + bo.
 * acts holds h_0..h_B (fp64, the residual stream) and a_1..a_B; u is d + 1
 * scratch values. */
static void resnet_forward(const orc_problem *p, const orc_net *net, const double *P,
                           const double *x, double t, double *acts, double *z, double *u, double *rb) {
  const int d = p->d, w = net->width, B = net->depth;
  memcpy(u, x, sizeof(double) * d);
  u[d] = t;
  const double *Win = P, *bin = P + (int64_t)w * (d + 1);
  double *h = acts;
  dense(net, w, d + 1, Win, bin, u, h, rb);
  for (int o = 0; o < w; ++o) h[o] = tanh(h[o]);
  const double *q = bin + w;
  double *a = acts + (int64_t)(B + 1) * w;
  for (int k = 1; k <= B; ++k) {
    const double *Wk = q, *bk = q + (int64_t)w * w;
    double *ak = a + (int64_t)(k - 1) * w;
    dense(net, w, w, Wk, bk, h + (int64_t)(k - 1) * w, ak, rb);
    for (int o = 0; o < w; ++o) {
      ak[o] = tanh(ak[o]);
      h[(int64_t)k * w + o] = h[(int64_t)(k - 1) * w + o] + ak[o];
    }
    q = bk + w;
  }
  dense(net, d, w, q, q + (int64_t)d * w, h + (int64_t)B * w, z, rb);
}

static void resnet_backward(const orc_problem *p, const orc_net *net, const double *P, double *G,
                            const double *x, double t, const double *acts, const double *zeta,
                            double *work /* 3w + d + 1 */, double *rb) {
  const int d = p->d, w = net->width, B = net->depth;
  const int64_t offin = 0, offbin = (int64_t)w * (d + 1);
  const int64_t offk = offbin + w;
  const int64_t offo = offk + (int64_t)B * ((int64_t)w * w + w);
  const double *h = acts, *a = acts + (int64_t)(B + 1) * w;
  double *dh = work, *dpre = work + w, *tmp = work + 2 * w, *u = work + 3 * w;
  outer_acc(net, d, w, zeta, h + (int64_t)B * w, G + offo, G + offo + (int64_t)d * w, rb);
  dense_t(net, d, w, P + offo, zeta, dh, rb);
  for (int k = B; k >= 1; --k) {
    const double *ak = a + (int64_t)(k - 1) * w;
    int64_t ow = offk + (int64_t)(k - 1) * ((int64_t)w * w + w);
    /* bf16 form: the derivative reads the bf16-stored activation */
    for (int o = 0; o < w; ++o) dpre[o] = dh[o] * (1.0 - R(net, ak[o]) * R(net, ak[o]));
    outer_acc(net, w, w, dpre, h + (int64_t)(k - 1) * w, G + ow, G + ow + (int64_t)w * w, rb);
    dense_t(net, w, w, P + ow, dpre, tmp, rb);
    for (int o = 0; o < w; ++o) dh[o] += tmp[o];
  }
  for (int o = 0; o < w; ++o) dpre[o] = dh[o] * (1.0 - R(net, h[o]) * R(net, h[o]));
  memcpy(u, x, sizeof(double) * d);
  u[d] = t;
  outer_acc(net, w, d + 1, dpre, u, G + offin, G + offbin, rb);
}

/* Per-path scratch of one thread: the whole history of one path. */
typedef struct {
  double *X, *Zs, *S, *Y, *A, *xim, *dw, *zeta, *pz, *work, *u, *rb;
} path_buf;

static int path_buf_alloc(path_buf *b, const orc_problem *p, const orc_net *net, int N) {
  const int d = p->d, w = net->width;
  const int mlp = (net->kind == ORC_NET_PER_STEP_MLP);
  const int64_t nacts = mlp ? (int64_t)net->depth * w : (int64_t)(2 * net->depth + 1) * w;
  const int nr = (d + 1 > w ? d + 1 : w);
  b->X = (double *)calloc((size_t)(N + 1) * d, sizeof(double));
  b->Zs = (double *)calloc((size_t)N * d, sizeof(double));
  b->S = (double *)calloc((size_t)N * d, sizeof(double));
  b->Y = (double *)calloc((size_t)(N + 1), sizeof(double));
  b->A = (double *)calloc((size_t)N * nacts + 1, sizeof(double));
  b->xim = (double *)calloc((size_t)d, sizeof(double));
  b->dw = (double *)calloc((size_t)d, sizeof(double));
  b->zeta = (double *)calloc((size_t)d, sizeof(double));
  b->pz = (double *)calloc((size_t)d, sizeof(double));
  b->work = (double *)calloc((size_t)(3 * w + d + 1), sizeof(double));
  b->u = (double *)calloc((size_t)(d + 1), sizeof(double));
  b->rb = (double *)calloc((size_t)nr, sizeof(double));
  return b->X && b->Zs && b->S && b->Y && b->A && b->xim && b->dw && b->zeta && b->pz && b->work && b->u &&
         b->rb;
}

static void path_buf_free(path_buf *b) {
  free(b->X); free(b->Zs); free(b->S); free(b->Y); free(b->A); free(b->xim); free(b->dw);
  free(b->zeta); free(b->pz); free(b->work); free(b->u); free(b->rb);
}

/* Forward Euler–Maruyama sweep of one path m, eq. (disc equations) with
 * mu = 0; stores X_n, Z_n, s_n = sigma(X_n) dW_n, Y_n and the network
 * activations of every step.  xi: [N][Mx][d] normals or NULL for Philox.
 * P holds the parameters with bf16-rounded weights in bf16 mode. */
static void path_forward(const orc_problem *p, const orc_net *net, int N, const double *P,
                         double y0, const double *xi, int64_t Mx, uint64_t seed, uint64_t iter,
                         int64_t m, path_buf *b) {
  const int d = p->d, w = net->width;
  const int mlp = (net->kind == ORC_NET_PER_STEP_MLP);
  const int64_t nacts = mlp ? (int64_t)net->depth * w : (int64_t)(2 * net->depth + 1) * w;
  const int64_t pstep = mlp ? mlp_step_count(d, w, net->depth) : 0;
  const double dt = p->T / N, sdt = sqrt(dt);
  memcpy(b->X, p->x0, sizeof(double) * d);
  b->Y[0] = y0;
  for (int n = 0; n < N; ++n) {
    const double *xn = b->X + (int64_t)n * d;
    double *zn = b->Zs + (int64_t)n * d, *sn = b->S + (int64_t)n * d;
    if (mlp && n == 0) {
      memcpy(zn, P, sizeof(double) * d);                      /* Z_0 = z0 */
    } else if (mlp) {
      mlp_forward(p, net, P + d + (int64_t)(n - 1) * pstep, xn, b->A + (int64_t)n * nacts, zn, b->rb);
    } else {
      resnet_forward(p, net, P, xn, n * dt, b->A + (int64_t)n * nacts, zn, b->u, b->rb);
    }
    if (xi) memcpy(b->xim, xi + ((int64_t)n * Mx + m) * d, sizeof(double) * d);
    else normals_one(seed, iter, n, m, d, b->xim);
    for (int i = 0; i < d; ++i) b->dw[i] = sdt * b->xim[i];
    diffusion(p, xn, b->dw, sn);
    b->Y[n + 1] = b->Y[n] + driver(p, xn, b->Y[n], zn) * dt + dot(d, zn, sn);
    for (int i = 0; i < d; ++i) b->X[(int64_t)(n + 1) * d + i] = xn[i] + sn[i];
  }
}

/* ------------------------------------------------------------------------ */
/* Loss and gradient                                                         */
/* ------------------------------------------------------------------------ */
static int check_args(const orc_problem *p, const orc_net *net, int N, int64_t M) {
  if (!p || !net || p->d < 1 || N < 1 || M < 1 || !(p->T > 0.0) || !p->x0) return 1;
  if (net->width < 1 || net->depth < 1) return 1;
  if (net->kind != ORC_NET_PER_STEP_MLP && net->kind != ORC_NET_SHARED_RESNET) return 1;
  if (net->kind == ORC_NET_PER_STEP_MLP && net->depth > 34) return 1;
  if (net->kind == ORC_NET_SHARED_RESNET && net->depth > 34) return 1;
  return 0;
}

int orc_loss_grad(const orc_problem *p, const orc_net *net, int N, int64_t M,
                  const double *params, double y0, const double *xi,
                  uint64_t seed, uint64_t iter,
                  double *loss, double *grad, double *grad_y0,
                  double *XN, double *YN, double *Ypath) {
  if (check_args(p, net, N, M) || !params || !loss) return 1;
  const int d = p->d, w = net->width;
  const int mlp = (net->kind == ORC_NET_PER_STEP_MLP);
  const int64_t nacts = mlp ? (int64_t)net->depth * w : (int64_t)(2 * net->depth + 1) * w;
  const int64_t pstep = mlp ? mlp_step_count(d, w, net->depth) : 0;
  const int64_t npar = orc_param_count(p, net, N);
  const double dt = p->T / N;
  const int want_adj = grad || grad_y0;
  const int64_t nch = (M + ORC_PATH_CHUNK - 1) / ORC_PATH_CHUNK;
  double *P = rounded_weights(p, net, N, params);
  if (grad) memset(grad, 0, sizeof(double) * (size_t)npar);
  double gy0 = 0.0, lsum = 0.0;
  int fail = 0;

#pragma omp parallel
  {
    path_buf b;
    int ok = path_buf_alloc(&b, p, net, N);
    double *gpart = grad ? (double *)calloc((size_t)npar, sizeof(double)) : NULL;
    if (grad && !gpart) ok = 0;
#pragma omp for ordered schedule(dynamic, 1)
    for (int64_t c = 0; c < nch; ++c) {
      /* chunk c: paths [c K, (c+1) K), summed from zero in path order */
      double lc = 0.0, gc = 0.0;
      if (ok) {
        if (gpart) memset(gpart, 0, sizeof(double) * (size_t)npar);
        const int64_t m1 = (c + 1) * ORC_PATH_CHUNK < M ? (c + 1) * ORC_PATH_CHUNK : M;
        for (int64_t m = c * ORC_PATH_CHUNK; m < m1; ++m) {
          path_forward(p, net, N, P, y0, xi, M, seed, iter, m, &b);
          const double *xN = b.X + (int64_t)N * d;
          double e = b.Y[N] - terminal(p, xN);
          lc += e * e;
          if (XN) memcpy(XN + m * d, xN, sizeof(double) * d);
          if (YN) YN[m] = b.Y[N];
          if (Ypath) for (int n = 0; n <= N; ++n) Ypath[(int64_t)n * M + m] = b.Y[n];
          if (!want_adj) continue;
          /* reverse sweep: lambda_n = dL/dY_n, zeta_n = dL/dZ_n */
          double lam = 2.0 * e / (double)M;
          for (int n = N - 1; n >= 0; --n) {
            const double *xn = b.X + (int64_t)n * d, *zn = b.Zs + (int64_t)n * d, *sn = b.S + (int64_t)n * d;
            driver_dz(p, xn, zn, b.pz);
            for (int i = 0; i < d; ++i) b.zeta[i] = lam * (b.pz[i] * dt + sn[i]);
            double lam_prev = lam * (1.0 + driver_dy(p, b.Y[n]) * dt);
            if (gpart) {
              if (mlp && n == 0) {
                for (int i = 0; i < d; ++i) gpart[i] += R(net, b.zeta[i]);
              } else if (mlp) {
                int64_t off = d + (int64_t)(n - 1) * pstep;
                mlp_backward(p, net, P + off, gpart + off, xn, b.A + (int64_t)n * nacts, b.zeta, b.work, b.rb);
              } else {
                resnet_backward(p, net, P, gpart, xn, n * dt, b.A + (int64_t)n * nacts, b.zeta, b.work, b.rb);
              }
            }
            lam = lam_prev;
          }
          gc += lam;
        }
      }
#pragma omp ordered
      {
        /* chunk partials enter the totals in chunk order */
        if (!ok) fail = 1;
        lsum += lc;
        gy0 += gc;
        if (grad && gpart && ok)
          for (int64_t k = 0; k < npar; ++k) grad[k] += gpart[k];
      }
    }
    free(gpart);
    path_buf_free(&b);
  }
  if (P != params) free(P);
  if (fail) return 2;
  *loss = lsum / (double)M;
  if (grad_y0) *grad_y0 = gy0;
  return 0;
}

int orc_loss_given_z(const orc_problem *p, int N, int64_t M, double y0, const double *xi,
                     uint64_t seed, uint64_t iter, const double *Z, double drv_sign, double *loss) {
  if (!p || p->d < 1 || N < 1 || M < 1 || !(p->T > 0.0) || !p->x0 || !Z || !loss) return 1;
  const int d = p->d;
  const double dt = p->T / N, sdt = sqrt(dt);
  double *x = (double *)malloc(sizeof(double) * d), *dw = (double *)malloc(sizeof(double) * d);
  double *sn = (double *)malloc(sizeof(double) * d), *xim = (double *)malloc(sizeof(double) * d);
  double lsum = 0.0;
  for (int64_t m = 0; m < M; ++m) {
    memcpy(x, p->x0, sizeof(double) * d);
    double y = y0;
    for (int n = 0; n < N; ++n) {
      const double *z = Z + ((int64_t)n * M + m) * d;
      if (xi) memcpy(xim, xi + ((int64_t)n * M + m) * d, sizeof(double) * d);
      else normals_one(seed, iter, n, m, d, xim);
      for (int i = 0; i < d; ++i) dw[i] = sdt * xim[i];
      diffusion(p, x, dw, sn);
      y = y + drv_sign * driver(p, x, y, z) * dt + dot(d, z, sn);
      for (int i = 0; i < d; ++i) x[i] += sn[i];
    }
    double e = y - terminal(p, x);
    lsum += e * e;
  }
  *loss = lsum / (double)M;
  free(x); free(dw); free(sn); free(xim);
  return 0;
}

int orc_loss_exact_bsb(const orc_problem *p, int N, int64_t M, double y0,
                       const double *xi, uint64_t seed, uint64_t iter,
                       int flip, double *loss) {
  if (!p || p->d < 1 || N < 1 || M < 1 || !loss) return 1;
  const int d = p->d;
  const double dt = p->T / N, sdt = sqrt(dt);
  const double r = p->drv_p[0], s = p->sde_s;
  double *x = (double *)malloc(sizeof(double) * d), *z = (double *)malloc(sizeof(double) * d);
  double *dw = (double *)malloc(sizeof(double) * d), *sn = (double *)malloc(sizeof(double) * d);
  double *xim = (double *)malloc(sizeof(double) * d);
  double lsum = 0.0;
  for (int64_t m = 0; m < M; ++m) {
    memcpy(x, p->x0, sizeof(double) * d);
    double y = y0;
    for (int n = 0; n < N; ++n) {
      double t = n * dt, c = 2.0 * exp((r + s * s) * (p->T - t));
      for (int i = 0; i < d; ++i) z[i] = c * x[i];              /* grad u(t, x) */
      if (xi) memcpy(xim, xi + ((int64_t)n * M + m) * d, sizeof(double) * d);
      else normals_one(seed, iter, n, m, d, xim);
      for (int i = 0; i < d; ++i) dw[i] = sdt * xim[i];
      diffusion(p, x, dw, sn);
      double phi = driver(p, x, y, z);
      y = y + (flip ? -phi : phi) * dt + dot(d, z, sn);
      for (int i = 0; i < d; ++i) x[i] += sn[i];
    }
    double e = y - terminal(p, x);
    lsum += e * e;
  }
  *loss = lsum / (double)M;
  free(x); free(z); free(dw); free(sn); free(xim);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Adam and multilevel prolongation                                          */
/* ------------------------------------------------------------------------ */
void orc_adam(int64_t n, double *theta, const double *g, double *m, double *v,
              int64_t t, double lr, double b1, double b2, double eps) {
  double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
  for (int64_t i = 0; i < n; ++i) {
    m[i] = b1 * m[i] + (1.0 - b1) * g[i];
    v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
    double mh = m[i] / c1, vh = v[i] / c2;
    theta[i] -= lr * mh / (sqrt(vh) + eps);
  }
}

int orc_prolong(const orc_problem *p, const orc_net *net, int Nc, int Nf,
                const double *pc, double *pf) {
  if (!p || !net || Nc < 1 || Nf != 2 * Nc) return 1;
  if (net->kind == ORC_NET_SHARED_RESNET) {
    memcpy(pf, pc, sizeof(double) * (size_t)orc_param_count(p, net, Nc));
    return 0;
  }
  if (Nc == 1) return 1;  /* a one-step grid has no network to copy from */
  const int d = p->d;
  const int64_t ps = mlp_step_count(d, net->width, net->depth);
  memcpy(pf, pc, sizeof(double) * d);
  for (int j = 1; j < Nf; ++j) {
    int c = j / 2;
    if (c < 1) c = 1;
    if (c > Nc - 1) c = Nc - 1;
    memcpy(pf + d + (int64_t)(j - 1) * ps, pc + d + (int64_t)(c - 1) * ps, sizeof(double) * (size_t)ps);
  }
  return 0;
}

int orc_paths(const orc_problem *p, const orc_net *net, int N, const double *params, double y0,
              uint64_t seed, uint64_t iter, const int64_t *idx, int64_t k, double *YN, double *XN) {
  if (check_args(p, net, N, 1) || !params || !idx || k < 0) return 1;
  const int d = p->d;
  double *P = rounded_weights(p, net, N, params);
  int fail = 0;
#pragma omp parallel
  {
    path_buf b;
    int ok = path_buf_alloc(&b, p, net, N);
#pragma omp for schedule(dynamic, 1)
    for (int64_t i = 0; i < k; ++i) {
      if (!ok) { fail = 1; continue; }
      path_forward(p, net, N, P, y0, NULL, 0, seed, iter, idx[i], &b);
      if (YN) YN[i] = b.Y[N];
      if (XN) memcpy(XN + i * d, b.X + (int64_t)N * d, sizeof(double) * d);
    }
    path_buf_free(&b);
  }
  if (P != params) free(P);
  return fail ? 2 : 0;
}

/* ======================================================================== */
/* The paper's own formulation: one u-network, Z = grad u, residual loss     */
/* (Sec. 2.2 eq. (loss); blocks of Sec. 3.1).  Plain fp64 throughout.        */
/* ======================================================================== */
static int unet_check(const orc_problem *p, const orc_unet *net, int N, int64_t M) {
  if (!p || !net || p->d < 1 || N < 1 || M < 1 || !(p->T > 0.0) || !p->x0) return 1;
  if (net->width < 1 || net->depth < 0 || net->depth > 64) return 1;
  if (net->arch != ORC_U_FC && net->arch != ORC_U_RES && net->arch != ORC_U_NAIS) return 1;
  return 0;
}

static int64_t unet_block_count(int d, int w, int arch) {
  int64_t c = (int64_t)w * w + w;
  if (arch == ORC_U_NAIS) c += (int64_t)w * (d + 1);
  return c;
}

int64_t orc_unet_param_count(const orc_problem *p, const orc_unet *net) {
  const int d = p->d, w = net->width;
  return (int64_t)w * (d + 1) + w + (int64_t)net->depth * unet_block_count(d, w, net->arch) + w + 1;
}

/* Pointers into the flat layout (and, for NAIS, the block matrices A_k
 * formed from R_k once per call). */
typedef struct {
  const double *W0, *b0, *wo, *bo;
  const double *A[64], *E[64], *b[64];  /* E[k] NULL unless NAIS */
  int64_t oW0, ob0, owo, obo, oA[64], oE[64], ob[64];
  double *Abuf;                          /* NAIS: K w x w matrices */
} unet_view;

static int unet_view_make(const orc_problem *p, const orc_unet *net, const double *P, unet_view *v) {
  const int d = p->d, w = net->width, K = net->depth;
  int64_t off = 0;
  v->oW0 = off; off += (int64_t)w * (d + 1);
  v->ob0 = off; off += w;
  v->Abuf = NULL;
  if (net->arch == ORC_U_NAIS) {
    v->Abuf = (double *)malloc(sizeof(double) * (size_t)((int64_t)K * w * w + 1));
    if (!v->Abuf) return 1;
  }
  for (int k = 0; k < K; ++k) {
    v->oA[k] = off; off += (int64_t)w * w;
    if (net->arch == ORC_U_NAIS) { v->oE[k] = off; off += (int64_t)w * (d + 1); } else v->oE[k] = -1;
    v->ob[k] = off; off += w;
  }
  v->owo = off; off += w;
  v->obo = off;
  v->W0 = P + v->oW0; v->b0 = P + v->ob0; v->wo = P + v->owo; v->bo = P + v->obo;
  for (int k = 0; k < K; ++k) {
    v->b[k] = P + v->ob[k];
    v->E[k] = net->arch == ORC_U_NAIS ? P + v->oE[k] : NULL;
    if (net->arch == ORC_U_NAIS) {
      /* A_k = -R_k^T R_k - eps I */
      const double *Rk = P + v->oA[k];
      double *Ak = v->Abuf + (int64_t)k * w * w;
      for (int a = 0; a < w; ++a)
        for (int c = 0; c < w; ++c) {
          double s = 0.0;
          for (int q = 0; q < w; ++q) s += Rk[(int64_t)q * w + a] * Rk[(int64_t)q * w + c];
          Ak[(int64_t)a * w + c] = -s - (a == c ? net->eps : 0.0);
        }
      v->A[k] = Ak;
    } else {
      v->A[k] = P + v->oA[k];
    }
  }
  return 0;
}

/* Per-row state of one network evaluation: h_k (k = 0..K), alpha_k
 * (k = 1..K, index k-1), the input-gradient sweep hh_k = du/dh_k and
 * g_k = the pre-activation gradients (k = 0..K). */
typedef struct { double *h, *al, *hh, *g, *zb; } unet_row;

static void unet_forward_row(const orc_problem *p, const orc_unet *net, const unet_view *v,
                             const double *z, unet_row *r, double *u) {
  const int d = p->d, w = net->width, K = net->depth;
  const double c = net->arch == ORC_U_FC ? 0.0 : 1.0;
  double *h0 = r->h;
  for (int a = 0; a < w; ++a) {
    double s = v->b0[a];
    for (int i = 0; i <= d; ++i) s += v->W0[(int64_t)a * (d + 1) + i] * z[i];
    h0[a] = tanh(s);
  }
  for (int k = 1; k <= K; ++k) {
    const double *hp = r->h + (int64_t)(k - 1) * w;
    double *hk = r->h + (int64_t)k * w, *ak = r->al + (int64_t)(k - 1) * w;
    const double *A = v->A[k - 1], *E = v->E[k - 1], *b = v->b[k - 1];
    for (int a = 0; a < w; ++a) {
      double s = b[a];
      for (int q = 0; q < w; ++q) s += A[(int64_t)a * w + q] * hp[q];
      if (E)
        for (int i = 0; i <= d; ++i) s += E[(int64_t)a * (d + 1) + i] * z[i];
      ak[a] = tanh(s);
      hk[a] = c * hp[a] + ak[a];
    }
  }
  const double *hK = r->h + (int64_t)K * w;
  double s = v->bo[0];
  for (int a = 0; a < w; ++a) s += v->wo[a] * hK[a];
  *u = s;
}

/* Z = grad_x u by the reverse sweep of the network for its scalar output:
 * hh_K = w_o; g_k = hh_k (1 - alpha_k^2); hh_{k-1} = c hh_k + A_k^T g_k;
 * g_0 = hh_0 (1 - h_0^2); grad_z u = W_0^T g_0 + sum_k E_k^T g_k. */
static void unet_zgrad_row(const orc_problem *p, const orc_unet *net, const unet_view *v, unet_row *r,
                           double *Z) {
  const int d = p->d, w = net->width, K = net->depth;
  const double c = net->arch == ORC_U_FC ? 0.0 : 1.0;
  memcpy(r->hh + (int64_t)K * w, v->wo, sizeof(double) * w);
  double *zg = r->zb;  /* d + 1 */
  for (int i = 0; i <= d; ++i) zg[i] = 0.0;
  for (int k = K; k >= 1; --k) {
    const double *hk = r->hh + (int64_t)k * w, *ak = r->al + (int64_t)(k - 1) * w;
    double *gk = r->g + (int64_t)k * w, *hp = r->hh + (int64_t)(k - 1) * w;
    const double *A = v->A[k - 1], *E = v->E[k - 1];
    for (int a = 0; a < w; ++a) gk[a] = hk[a] * (1.0 - ak[a] * ak[a]);
    for (int q = 0; q < w; ++q) {
      double s = 0.0;
      for (int a = 0; a < w; ++a) s += A[(int64_t)a * w + q] * gk[a];
      hp[q] = c * hk[q] + s;
    }
    if (E)
      for (int i = 0; i <= d; ++i) {
        double s = 0.0;
        for (int a = 0; a < w; ++a) s += E[(int64_t)a * (d + 1) + i] * gk[a];
        zg[i] += s;
      }
  }
  double *g0 = r->g;
  for (int a = 0; a < w; ++a) g0[a] = r->hh[a] * (1.0 - r->h[a] * r->h[a]);
  for (int i = 0; i < d; ++i) {
    double s = 0.0;
    for (int a = 0; a < w; ++a) s += v->W0[(int64_t)a * (d + 1) + i] * g0[a];
    Z[i] = zg[i] + s;
  }
}

/* Reverse sweep of one row for the seeds ub = dL/du and Zb = dL/dZ
 * (accumulates into G in the flat layout; the gradient of A_k goes to G at
 * A_k's offset also for NAIS, converted to R_k by the caller).  work: 4w. */
static void unet_adjoint_row(const orc_problem *p, const orc_unet *net, const unet_view *v, const double *z,
                             const unet_row *r, double ub, const double *Zb, double *G, double *work) {
  const int d = p->d, w = net->width, K = net->depth;
  const double c = net->arch == ORC_U_FC ? 0.0 : 1.0;
  double *gb = work, *hhb = work + w, *hb = work + 2 * w, *alb = work + 3 * w;
  /* alb holds alpha-bar partials of every block: K w values after work + 3w */
  /* ---- second-order part, k = 0..K in forward order ---- */
  /* g_0 = hh_0 (1 - h_0^2), Z = W_0x^T g_0 */
  const double *h0 = r->h, *hh0 = r->hh, *g0 = r->g;
  for (int a = 0; a < w; ++a) {
    double s = 0.0;
    for (int i = 0; i < d; ++i) s += v->W0[(int64_t)a * (d + 1) + i] * Zb[i];
    gb[a] = s;
    for (int i = 0; i < d; ++i) G[v->oW0 + (int64_t)a * (d + 1) + i] += g0[a] * Zb[i];
  }
  for (int a = 0; a < w; ++a) {
    hhb[a] = gb[a] * (1.0 - h0[a] * h0[a]);
    hb[a] = gb[a] * hh0[a] * (-2.0 * h0[a]);  /* h_0-bar partial */
  }
  for (int k = 1; k <= K; ++k) {
    const double *A = v->A[k - 1], *E = v->E[k - 1];
    const double *gk = r->g + (int64_t)k * w, *hhk = r->hh + (int64_t)k * w, *ak = r->al + (int64_t)(k - 1) * w;
    double *albk = alb + (int64_t)(k - 1) * w;
    double *gA = G + v->oA[k - 1];
    /* gamma-bar_k = A_k hh-bar_{k-1} (+ E_k zb); A-bar_k += g_k hh-bar_{k-1}^T */
    for (int a = 0; a < w; ++a) {
      double s = 0.0;
      for (int q = 0; q < w; ++q) s += A[(int64_t)a * w + q] * hhb[q];
      if (E) {
        double *gE = G + v->oE[k - 1];
        for (int i = 0; i < d; ++i) {
          s += E[(int64_t)a * (d + 1) + i] * Zb[i];
          gE[(int64_t)a * (d + 1) + i] += gk[a] * Zb[i];
        }
      }
      for (int q = 0; q < w; ++q) gA[(int64_t)a * w + q] += gk[a] * hhb[q];
      gb[a] = s;
    }
    for (int a = 0; a < w; ++a) {
      hhb[a] = c * hhb[a] + gb[a] * (1.0 - ak[a] * ak[a]);
      albk[a] = gb[a] * hhk[a] * (-2.0 * ak[a]);
    }
  }
  /* hh_K = w_o */
  for (int a = 0; a < w; ++a) G[v->owo + a] += hhb[a];
  /* ---- first-order part: u = w_o . h_K + b_o, then the blocks backwards ---- */
  const double *hK = r->h + (int64_t)K * w;
  double *hbar = gb;  /* reuse: h-bar_k */
  for (int a = 0; a < w; ++a) {
    hbar[a] = ub * v->wo[a];
    G[v->owo + a] += ub * hK[a];
  }
  G[v->obo] += ub;
  for (int k = K; k >= 1; --k) {
    const double *A = v->A[k - 1], *E = v->E[k - 1];
    const double *ak = r->al + (int64_t)(k - 1) * w, *hp = r->h + (int64_t)(k - 1) * w;
    const double *albk = alb + (int64_t)(k - 1) * w;
    double *abar = hhb;  /* reuse */
    for (int a = 0; a < w; ++a) abar[a] = (albk[a] + hbar[a]) * (1.0 - ak[a] * ak[a]);
    double *gA = G + v->oA[k - 1], *gbk = G + v->ob[k - 1];
    for (int a = 0; a < w; ++a) {
      for (int q = 0; q < w; ++q) gA[(int64_t)a * w + q] += abar[a] * hp[q];
      gbk[a] += abar[a];
      if (E) {
        double *gE = G + v->oE[k - 1];
        for (int i = 0; i <= d; ++i) gE[(int64_t)a * (d + 1) + i] += abar[a] * z[i];
      }
    }
    for (int q = 0; q < w; ++q) {
      double s = 0.0;
      for (int a = 0; a < w; ++a) s += A[(int64_t)a * w + q] * abar[a];
      hbar[q] = c * hbar[q] + s;
    }
  }
  for (int a = 0; a < w; ++a) {
    double ab0 = (hbar[a] + hb[a]) * (1.0 - h0[a] * h0[a]);
    for (int i = 0; i <= d; ++i) G[v->oW0 + (int64_t)a * (d + 1) + i] += ab0 * z[i];
    G[v->ob0 + a] += ab0;
  }
}

static void terminal_grad(const orc_problem *p, const double *x, double *out) {
  double q = dot(p->d, x, x);
  for (int i = 0; i < p->d; ++i) {
    switch (p->g) {
      case ORC_G_NORM2: out[i] = 2.0 * x[i]; break;
      case ORC_G_LOGHALF: out[i] = 2.0 * x[i] / (1.0 + q); break;
      case ORC_G_INV: {
        double den = p->g_p[0] + p->g_p[1] * q;
        out[i] = -2.0 * p->g_p[1] * x[i] / (den * den);
        break;
      }
      default: out[i] = p->g_p[0]; break;
    }
  }
}

/* Euler–Maruyama path of X (mu = 0) for path m: X [N+1][d], S [N][d] */
static void unet_path_x(const orc_problem *p, int N, const double *xi, int64_t Mx, uint64_t seed, uint64_t iter,
                        int64_t m, double *X, double *S, double *xim) {
  const int d = p->d;
  const double sdt = sqrt(p->T / N);
  memcpy(X, p->x0, sizeof(double) * d);
  for (int n = 0; n < N; ++n) {
    if (xi) memcpy(xim, xi + ((int64_t)n * Mx + m) * d, sizeof(double) * d);
    else normals_one(seed, iter, n, m, d, xim);
    for (int i = 0; i < d; ++i) xim[i] *= sdt;
    diffusion(p, X + (int64_t)n * d, xim, S + (int64_t)n * d);
    for (int i = 0; i < d; ++i) X[(int64_t)(n + 1) * d + i] = X[(int64_t)n * d + i] + S[(int64_t)n * d + i];
  }
}

/* Residuals of one path and their seeds: r [N], e, pen [d]; ub [N+1],
 * Zb [N+1][d] (dL/du_n and dL/dZ_n with the 1/M of the batch mean). */
static double unet_path_residuals(const orc_problem *p, int N, int64_t M, const double *X, const double *S,
                                  const double *u, const double *Z, double kappa, double *ub, double *Zb,
                                  double *pz, double *gx) {
  const int d = p->d;
  const double dt = p->T / N;
  double l = 0.0;
  for (int n = 0; n <= N; ++n) ub[n] = 0.0;
  for (int64_t k = 0; k < (int64_t)(N + 1) * d; ++k) Zb[k] = 0.0;
  for (int n = 0; n < N; ++n) {
    const double *xn = X + (int64_t)n * d, *zn = Z + (int64_t)n * d, *sn = S + (int64_t)n * d;
    const double rn = u[n + 1] - u[n] - driver(p, xn, u[n], zn) * dt - dot(d, zn, sn);
    l += rn * rn;
    const double c = 2.0 * rn / (double)M;
    ub[n + 1] += c;
    ub[n] -= c * (1.0 + driver_dy(p, u[n]) * dt);
    driver_dz(p, xn, zn, pz);
    for (int i = 0; i < d; ++i) Zb[(int64_t)n * d + i] -= c * (pz[i] * dt + sn[i]);
  }
  const double *xN = X + (int64_t)N * d, *zN = Z + (int64_t)N * d;
  const double e = u[N] - terminal(p, xN);
  l += e * e;
  ub[N] += 2.0 * e / (double)M;
  if (kappa != 0.0) {
    terminal_grad(p, xN, gx);
    for (int i = 0; i < d; ++i) {
      const double q = zN[i] - gx[i];
      l += kappa * q * q;
      Zb[(int64_t)N * d + i] += 2.0 * kappa * q / (double)M;
    }
  }
  return l;
}

int orc_unet_loss_grad(const orc_problem *p, const orc_unet *net, int N, int64_t M,
                       const double *params, const double *xi, uint64_t seed, uint64_t iter,
                       double kappa, double *loss, double *grad, double *U, double *Zout) {
  if (unet_check(p, net, N, M) || !params || !loss) return 1;
  const int d = p->d, w = net->width, K = net->depth;
  const int64_t npar = orc_unet_param_count(p, net);
  const double dt = p->T / N;
  const int64_t nch = (M + ORC_PATH_CHUNK - 1) / ORC_PATH_CHUNK;
  unet_view v;
  if (unet_view_make(p, net, params, &v)) return 2;
  /* gradient with respect to A_k (NAIS: converted to R_k at the end) */
  double *GA = grad ? (double *)calloc((size_t)npar, sizeof(double)) : NULL;
  if (grad && !GA) { free(v.Abuf); return 2; }
  double lsum = 0.0;
  int fail = 0;
#pragma omp parallel
  {
    const int64_t rows = N + 1;
    double *X = (double *)malloc(sizeof(double) * (size_t)(rows * d));
    double *S = (double *)malloc(sizeof(double) * (size_t)(N * d));
    double *xim = (double *)malloc(sizeof(double) * d);
    double *u = (double *)malloc(sizeof(double) * (size_t)rows);
    double *Z = (double *)malloc(sizeof(double) * (size_t)(rows * d));
    double *ub = (double *)malloc(sizeof(double) * (size_t)rows);
    double *Zb = (double *)malloc(sizeof(double) * (size_t)(rows * d));
    double *pz = (double *)malloc(sizeof(double) * d), *gx = (double *)malloc(sizeof(double) * d);
    double *zin = (double *)malloc(sizeof(double) * (size_t)(rows * (d + 1)));
    /* per-row network state of the whole path */
    const int64_t hs = (int64_t)(K + 1) * w;
    double *H = (double *)malloc(sizeof(double) * (size_t)(rows * hs));
    double *AL = (double *)malloc(sizeof(double) * (size_t)(rows * (K > 0 ? K * w : 1)));
    double *HH = (double *)malloc(sizeof(double) * (size_t)(rows * hs));
    double *GG = (double *)malloc(sizeof(double) * (size_t)(rows * hs));
    double *zb = (double *)malloc(sizeof(double) * (size_t)(d + 1));
    double *work = (double *)malloc(sizeof(double) * (size_t)((3 + K) * w + 1));
    double *gpart = grad ? (double *)calloc((size_t)npar, sizeof(double)) : NULL;
    int ok = X && S && xim && u && Z && ub && Zb && pz && gx && zin && H && AL && HH && GG && zb && work &&
             (!grad || gpart);
#pragma omp for ordered schedule(dynamic, 1)
    for (int64_t ch = 0; ch < nch; ++ch) {
      double lc = 0.0;
      if (ok) {
        if (gpart) memset(gpart, 0, sizeof(double) * (size_t)npar);
        const int64_t m1 = (ch + 1) * ORC_PATH_CHUNK < M ? (ch + 1) * ORC_PATH_CHUNK : M;
        for (int64_t m = ch * ORC_PATH_CHUNK; m < m1; ++m) {
          unet_path_x(p, N, xi, M, seed, iter, m, X, S, xim);
          for (int n = 0; n <= N; ++n) {
            double *z = zin + (int64_t)n * (d + 1);
            memcpy(z, X + (int64_t)n * d, sizeof(double) * d);
            z[d] = n * dt;
            unet_row r = {H + n * hs, AL + (int64_t)n * K * w, HH + n * hs, GG + n * hs, zb};
            unet_forward_row(p, net, &v, z, &r, &u[n]);
            unet_zgrad_row(p, net, &v, &r, Z + (int64_t)n * d);
          }
          if (U) for (int n = 0; n <= N; ++n) U[(int64_t)n * M + m] = u[n];
          if (Zout)
            for (int n = 0; n <= N; ++n) memcpy(Zout + ((int64_t)n * M + m) * d, Z + (int64_t)n * d, sizeof(double) * d);
          lc += unet_path_residuals(p, N, M, X, S, u, Z, kappa, ub, Zb, pz, gx);
          if (!gpart) continue;
          for (int n = 0; n <= N; ++n) {
            unet_row r = {H + n * hs, AL + (int64_t)n * K * w, HH + n * hs, GG + n * hs, zb};
            unet_adjoint_row(p, net, &v, zin + (int64_t)n * (d + 1), &r, ub[n], Zb + (int64_t)n * d, gpart,
                             work);
          }
        }
      }
#pragma omp ordered
      {
        if (!ok) fail = 1;
        lsum += lc;
        if (GA && gpart && ok)
          for (int64_t k = 0; k < npar; ++k) GA[k] += gpart[k];
      }
    }
    free(X); free(S); free(xim); free(u); free(Z); free(ub); free(Zb); free(pz); free(gx); free(zin);
    free(H); free(AL); free(HH); free(GG); free(zb); free(work); free(gpart);
  }
  if (!fail && grad) {
    memcpy(grad, GA, sizeof(double) * (size_t)npar);
    if (net->arch == ORC_U_NAIS) {
      /* A = -R^T R - eps I  =>  R-bar = -R (A-bar + A-bar^T) */
      for (int k = 0; k < K; ++k) {
        const double *Rk = params + v.oA[k], *Ab = GA + v.oA[k];
        double *gR = grad + v.oA[k];
        for (int q = 0; q < w; ++q)
          for (int c2 = 0; c2 < w; ++c2) {
            double s = 0.0;
            for (int a = 0; a < w; ++a)
              s += Rk[(int64_t)q * w + a] * (Ab[(int64_t)a * w + c2] + Ab[(int64_t)c2 * w + a]);
            gR[(int64_t)q * w + c2] = -s;
          }
      }
    }
  }
  free(GA);
  free(v.Abuf);
  if (fail) return 2;
  *loss = lsum / (double)M;
  return 0;
}

int orc_unet_loss_given_uz(const orc_problem *p, int N, int64_t M, const double *xi, uint64_t seed,
                           uint64_t iter, const double *U, const double *Z, double kappa, double *loss) {
  if (!p || p->d < 1 || N < 1 || M < 1 || !(p->T > 0.0) || !p->x0 || !U || !Z || !loss) return 1;
  const int d = p->d;
  double *X = (double *)malloc(sizeof(double) * (size_t)((N + 1) * d));
  double *S = (double *)malloc(sizeof(double) * (size_t)(N * d));
  double *xim = (double *)malloc(sizeof(double) * d);
  double *u = (double *)malloc(sizeof(double) * (size_t)(N + 1));
  double *Zp = (double *)malloc(sizeof(double) * (size_t)((N + 1) * d));
  double *ub = (double *)malloc(sizeof(double) * (size_t)(N + 1));
  double *Zb = (double *)malloc(sizeof(double) * (size_t)((N + 1) * d));
  double *pz = (double *)malloc(sizeof(double) * d), *gx = (double *)malloc(sizeof(double) * d);
  double lsum = 0.0;
  for (int64_t m = 0; m < M; ++m) {
    unet_path_x(p, N, xi, M, seed, iter, m, X, S, xim);
    for (int n = 0; n <= N; ++n) {
      u[n] = U[(int64_t)n * M + m];
      memcpy(Zp + (int64_t)n * d, Z + ((int64_t)n * M + m) * d, sizeof(double) * d);
    }
    lsum += unet_path_residuals(p, N, M, X, S, u, Zp, kappa, ub, Zb, pz, gx);
  }
  *loss = lsum / (double)M;
  free(X); free(S); free(xim); free(u); free(Zp); free(ub); free(Zb); free(pz); free(gx);
  return 0;
}

int orc_unet_eval(const orc_problem *p, const orc_unet *net, const double *params, int64_t R,
                  const double *T, const double *X, double *u, double *Z) {
  if (unet_check(p, net, 1, 1) || !params || R < 0 || (R > 0 && (!T || !X))) return 1;
  const int d = p->d, w = net->width, K = net->depth;
  unet_view v;
  if (unet_view_make(p, net, params, &v)) return 2;
  const int64_t hs = (int64_t)(K + 1) * w;
  double *H = (double *)malloc(sizeof(double) * (size_t)hs), *AL = (double *)malloc(sizeof(double) * (size_t)(K * w + 1));
  double *HH = (double *)malloc(sizeof(double) * (size_t)hs), *GG = (double *)malloc(sizeof(double) * (size_t)hs);
  double *zb = (double *)malloc(sizeof(double) * (size_t)(d + 1)), *z = (double *)malloc(sizeof(double) * (size_t)(d + 1));
  double *Zr = (double *)malloc(sizeof(double) * d);
  for (int64_t i = 0; i < R; ++i) {
    memcpy(z, X + i * d, sizeof(double) * d);
    z[d] = T[i];
    unet_row r = {H, AL, HH, GG, zb};
    double ui;
    unet_forward_row(p, net, &v, z, &r, &ui);
    if (u) u[i] = ui;
    if (Z) {
      unet_zgrad_row(p, net, &v, &r, Zr);
      memcpy(Z + i * d, Zr, sizeof(double) * d);
    }
  }
  free(H); free(AL); free(HH); free(GG); free(zb); free(z); free(Zr);
  free(v.Abuf);
  return 0;
}

int orc_unet_nais_project(const orc_problem *p, const orc_unet *net, double *params, double c) {
  if (!p || !net || !params || net->arch != ORC_U_NAIS || !(c > 0.0)) return 1;
  const int d = p->d, w = net->width, K = net->depth;
  int64_t off = (int64_t)w * (d + 1) + w;
  for (int k = 0; k < K; ++k) {
    double *Rk = params + off;
    double f2 = 0.0;  /* |R^T R|_F^2 */
    for (int a = 0; a < w; ++a)
      for (int b = 0; b < w; ++b) {
        double s = 0.0;
        for (int q = 0; q < w; ++q) s += Rk[(int64_t)q * w + a] * Rk[(int64_t)q * w + b];
        f2 += s * s;
      }
    const double f = sqrt(f2);
    if (f > c) {
      const double sc = sqrt(c / f);
      for (int64_t e = 0; e < (int64_t)w * w; ++e) Rk[e] *= sc;
    }
    off += unet_block_count(d, w, net->arch);
  }
  return 0;
}
