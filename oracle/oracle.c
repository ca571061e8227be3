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

/* dense layer: out[o] = sum_i R(W[o][i]) R(in[i]) + b[o] */
static void dense(const orc_net *net, int nout, int nin, const double *W, const double *b,
                  const double *in, double *out) {
  for (int o = 0; o < nout; ++o) {
    double s = 0.0;
    for (int i = 0; i < nin; ++i) s += R(net, W[(int64_t)o * nin + i]) * R(net, in[i]);
    out[o] = s + b[o];
  }
}

/* transposed product and outer-product accumulation for the reverse sweep */
static void dense_t(const orc_net *net, int nout, int nin, const double *W, const double *delta,
                    double *out_in) {
  for (int i = 0; i < nin; ++i) {
    double s = 0.0;
    for (int o = 0; o < nout; ++o) s += R(net, W[(int64_t)o * nin + i]) * R(net, delta[o]);
    out_in[i] = s;
  }
}
static void outer_acc(const orc_net *net, int nout, int nin, const double *delta, const double *in,
                      double *gW, double *gb) {
  for (int o = 0; o < nout; ++o) {
    double dl = R(net, delta[o]);
    for (int i = 0; i < nin; ++i) gW[(int64_t)o * nin + i] += dl * R(net, in[i]);
    gb[o] += dl;
  }
}

/* Per-step MLP (Sec. 2.2, one network per time step): d -> w tanh
 * (-> w tanh) x (L-1) -> d linear.  acts[l] holds hidden layer l (w values),
 * after the bf16 rounding that the later layers see. */
static void mlp_forward(const orc_problem *p, const orc_net *net, const double *P,
                        const double *x, double *acts, double *z) {
  const int d = p->d, w = net->width, L = net->depth;
  const double *W = P, *b = P + (int64_t)w * d;
  dense(net, w, d, W, b, x, acts);
  for (int o = 0; o < w; ++o) acts[o] = R(net, tanh(acts[o]));
  const double *q = b + w;
  for (int l = 1; l < L; ++l) {
    const double *Wl = q, *bl = q + (int64_t)w * w;
    dense(net, w, w, Wl, bl, acts + (int64_t)(l - 1) * w, acts + (int64_t)l * w);
    for (int o = 0; o < w; ++o) acts[(int64_t)l * w + o] = R(net, tanh(acts[(int64_t)l * w + o]));
    q = bl + w;
  }
  dense(net, d, w, q, q + (int64_t)d * w, acts + (int64_t)(L - 1) * w, z);
}

static void mlp_backward(const orc_problem *p, const orc_net *net, const double *P, double *G,
                         const double *x, const double *acts, const double *zeta,
                         double *work /* 2w */) {
  const int d = p->d, w = net->width, L = net->depth;
  /* offsets of every layer */
  const int64_t off1 = 0, offb1 = (int64_t)w * d;
  int64_t offh = offb1 + w;  /* first hidden-to-hidden layer */
  int64_t offo = offh + (int64_t)(L - 1) * ((int64_t)w * w + w);
  double *dcur = work, *dnext = work + w;
  /* output layer */
  outer_acc(net, d, w, zeta, acts + (int64_t)(L - 1) * w, G + offo, G + offo + (int64_t)d * w);
  dense_t(net, d, w, P + offo, zeta, dcur);
  for (int l = L - 1; l >= 0; --l) {
    const double *h = acts + (int64_t)l * w;
    for (int o = 0; o < w; ++o) dcur[o] *= (1.0 - h[o] * h[o]);
    if (l == 0) {
      outer_acc(net, w, d, dcur, x, G + off1, G + offb1);
    } else {
      int64_t ow = offh + (int64_t)(l - 1) * ((int64_t)w * w + w);
      outer_acc(net, w, w, dcur, acts + (int64_t)(l - 1) * w, G + ow, G + ow + (int64_t)w * w);
      dense_t(net, w, w, P + ow, dcur, dnext);
      double *t = dcur; dcur = dnext; dnext = t;
    }
  }
}

/* Shared residual network with t as input (Sec. 3.1, residual block as a
 * forward-Euler step of eq. (ode) with h = 1):
 *   h_0 = tanh(Win [x; t] + bin),  h_k = h_{k-1} + tanh(W_k h_{k-1} + b_k),
 *   Z = Wo h_B + bo.
 * acts holds h_0..h_B (fp64, the residual stream) and a_1..a_B. */
static void resnet_forward(const orc_problem *p, const orc_net *net, const double *P,
                           const double *x, double t, double *acts, double *z) {
  const int d = p->d, w = net->width, B = net->depth;
  double *u = (double *)malloc(sizeof(double) * (d + 1));
  memcpy(u, x, sizeof(double) * d);
  u[d] = t;
  const double *Win = P, *bin = P + (int64_t)w * (d + 1);
  double *h = acts;
  dense(net, w, d + 1, Win, bin, u, h);
  for (int o = 0; o < w; ++o) h[o] = tanh(h[o]);
  const double *q = bin + w;
  double *a = acts + (int64_t)(B + 1) * w;
  for (int k = 1; k <= B; ++k) {
    const double *Wk = q, *bk = q + (int64_t)w * w;
    double *ak = a + (int64_t)(k - 1) * w;
    dense(net, w, w, Wk, bk, h + (int64_t)(k - 1) * w, ak);
    for (int o = 0; o < w; ++o) {
      ak[o] = tanh(ak[o]);
      h[(int64_t)k * w + o] = h[(int64_t)(k - 1) * w + o] + ak[o];
    }
    q = bk + w;
  }
  dense(net, d, w, q, q + (int64_t)d * w, h + (int64_t)B * w, z);
  free(u);
}

static void resnet_backward(const orc_problem *p, const orc_net *net, const double *P, double *G,
                            const double *x, double t, const double *acts, const double *zeta,
                            double *work /* 3w + d + 1 */) {
  const int d = p->d, w = net->width, B = net->depth;
  const int64_t offin = 0, offbin = (int64_t)w * (d + 1);
  const int64_t offk = offbin + w;
  const int64_t offo = offk + (int64_t)B * ((int64_t)w * w + w);
  const double *h = acts, *a = acts + (int64_t)(B + 1) * w;
  double *dh = work, *dpre = work + w, *tmp = work + 2 * w, *u = work + 3 * w;
  outer_acc(net, d, w, zeta, h + (int64_t)B * w, G + offo, G + offo + (int64_t)d * w);
  dense_t(net, d, w, P + offo, zeta, dh);
  for (int k = B; k >= 1; --k) {
    const double *ak = a + (int64_t)(k - 1) * w;
    int64_t ow = offk + (int64_t)(k - 1) * ((int64_t)w * w + w);
    /* bf16 form: the derivative reads the bf16-stored activation */
    for (int o = 0; o < w; ++o) dpre[o] = dh[o] * (1.0 - R(net, ak[o]) * R(net, ak[o]));
    outer_acc(net, w, w, dpre, h + (int64_t)(k - 1) * w, G + ow, G + ow + (int64_t)w * w);
    dense_t(net, w, w, P + ow, dpre, tmp);
    for (int o = 0; o < w; ++o) dh[o] += tmp[o];
  }
  for (int o = 0; o < w; ++o) dpre[o] = dh[o] * (1.0 - R(net, h[o]) * R(net, h[o]));
  memcpy(u, x, sizeof(double) * d);
  u[d] = t;
  outer_acc(net, w, d + 1, dpre, u, G + offin, G + offbin);
}

/* Forward Euler–Maruyama sweep of one path m, eq. (disc equations) with
 * mu = 0; stores X_n, Z_n, s_n = sigma(X_n) dW_n, Y_n and the network
 * activations of every step.  xi: [N][Mx][d] normals or NULL for Philox. */
static void path_forward(const orc_problem *p, const orc_net *net, int N, const double *params,
                         double y0, const double *xi, int64_t Mx, uint64_t seed, uint64_t iter,
                         int64_t m, double *X, double *Zs, double *S, double *Y, double *A,
                         double *xim, double *dw) {
  const int d = p->d, w = net->width;
  const int mlp = (net->kind == ORC_NET_PER_STEP_MLP);
  const int64_t nacts = mlp ? (int64_t)net->depth * w : (int64_t)(2 * net->depth + 1) * w;
  const int64_t pstep = mlp ? mlp_step_count(d, w, net->depth) : 0;
  const double dt = p->T / N, sdt = sqrt(dt);
  memcpy(X, p->x0, sizeof(double) * d);
  Y[0] = y0;
  for (int n = 0; n < N; ++n) {
    const double *xn = X + (int64_t)n * d;
    double *zn = Zs + (int64_t)n * d, *sn = S + (int64_t)n * d;
    if (mlp && n == 0) {
      memcpy(zn, params, sizeof(double) * d);                 /* Z_0 = z0 */
    } else if (mlp) {
      mlp_forward(p, net, params + d + (int64_t)(n - 1) * pstep, xn, A + (int64_t)n * nacts, zn);
    } else {
      resnet_forward(p, net, params, xn, n * dt, A + (int64_t)n * nacts, zn);
    }
    if (xi) memcpy(xim, xi + ((int64_t)n * Mx + m) * d, sizeof(double) * d);
    else normals_one(seed, iter, n, m, d, xim);
    for (int i = 0; i < d; ++i) dw[i] = sdt * xim[i];
    diffusion(p, xn, dw, sn);
    Y[n + 1] = Y[n] + driver(p, xn, Y[n], zn) * dt + dot(d, zn, sn);
    for (int i = 0; i < d; ++i) X[(int64_t)(n + 1) * d + i] = xn[i] + sn[i];
  }
}

/* ------------------------------------------------------------------------ */
/* Loss and gradient                                                         */
/* ------------------------------------------------------------------------ */
static int check_args(const orc_problem *p, const orc_net *net, int N, int64_t M) {
  if (!p || !net || p->d < 1 || N < 1 || M < 1 || !(p->T > 0.0) || !p->x0) return 1;
  if (net->width < 1 || net->depth < 1) return 1;
  if (net->kind != ORC_NET_PER_STEP_MLP && net->kind != ORC_NET_SHARED_RESNET) return 1;
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

  double *X = (double *)calloc((size_t)(N + 1) * d, sizeof(double));
  double *Zs = (double *)calloc((size_t)N * d, sizeof(double));
  double *S = (double *)calloc((size_t)N * d, sizeof(double));
  double *Y = (double *)calloc((size_t)(N + 1), sizeof(double));
  double *A = (double *)calloc((size_t)N * nacts + 1, sizeof(double));
  double *xim = (double *)calloc((size_t)d, sizeof(double));
  double *dw = (double *)calloc((size_t)d, sizeof(double));
  double *zeta = (double *)calloc((size_t)d, sizeof(double));
  double *pz = (double *)calloc((size_t)d, sizeof(double));
  double *work = (double *)calloc((size_t)(3 * w + d + 1), sizeof(double));
  if (grad) memset(grad, 0, sizeof(double) * (size_t)npar);
  double gy0 = 0.0, lsum = 0.0;

  for (int64_t m = 0; m < M; ++m) {
    path_forward(p, net, N, params, y0, xi ? xi : NULL, M, seed, iter, m, X, Zs, S, Y, A, xim, dw);
    const double *xN = X + (int64_t)N * d;
    double e = Y[N] - terminal(p, xN);
    lsum += e * e;
    if (XN) memcpy(XN + m * d, xN, sizeof(double) * d);
    if (YN) YN[m] = Y[N];
    if (Ypath) for (int n = 0; n <= N; ++n) Ypath[(int64_t)n * M + m] = Y[n];

    if (grad || grad_y0) {
      /* reverse sweep: lambda_n = dL/dY_n, zeta_n = dL/dZ_n */
      double lam = 2.0 * e / (double)M;
      for (int n = N - 1; n >= 0; --n) {
        const double *xn = X + (int64_t)n * d, *zn = Zs + (int64_t)n * d, *sn = S + (int64_t)n * d;
        driver_dz(p, xn, zn, pz);
        for (int i = 0; i < d; ++i) zeta[i] = lam * (pz[i] * dt + sn[i]);
        double lam_prev = lam * (1.0 + driver_dy(p, Y[n]) * dt);
        if (grad) {
          if (mlp && n == 0) {
            for (int i = 0; i < d; ++i) grad[i] += R(net, zeta[i]);
          } else if (mlp) {
            int64_t off = d + (int64_t)(n - 1) * pstep;
            mlp_backward(p, net, params + off, grad + off, xn, A + (int64_t)n * nacts, zeta, work);
          } else {
            resnet_backward(p, net, params, grad, xn, n * dt, A + (int64_t)n * nacts, zeta, work);
          }
        }
        lam = lam_prev;
      }
      gy0 += lam;
    }
  }
  *loss = lsum / (double)M;
  if (grad_y0) *grad_y0 = gy0;
  free(X); free(Zs); free(S); free(Y); free(A); free(xim); free(dw); free(zeta); free(pz); free(work);
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
  const int d = p->d, w = net->width;
  const int mlp = (net->kind == ORC_NET_PER_STEP_MLP);
  const int64_t nacts = mlp ? (int64_t)net->depth * w : (int64_t)(2 * net->depth + 1) * w;
  double *X = (double *)calloc((size_t)(N + 1) * d, sizeof(double));
  double *Zs = (double *)calloc((size_t)N * d, sizeof(double));
  double *S = (double *)calloc((size_t)N * d, sizeof(double));
  double *Y = (double *)calloc((size_t)(N + 1), sizeof(double));
  double *A = (double *)calloc((size_t)N * nacts + 1, sizeof(double));
  double *xim = (double *)calloc((size_t)d, sizeof(double));
  double *dw = (double *)calloc((size_t)d, sizeof(double));
  for (int64_t i = 0; i < k; ++i) {
    path_forward(p, net, N, params, y0, NULL, 0, seed, iter, idx[i], X, Zs, S, Y, A, xim, dw);
    if (YN) YN[i] = Y[N];
    if (XN) memcpy(XN + i * d, X + (int64_t)N * d, sizeof(double) * d);
  }
  free(X); free(Zs); free(S); free(Y); free(A); free(xim); free(dw);
  return 0;
}
