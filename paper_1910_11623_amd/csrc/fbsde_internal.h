// Internal declarations of the gfx950 deep-FBSDE library (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/fbsde.h"

namespace fbsde {

// ABI helpers shared by the translation units that implement entry points:
// set the thread-local error message and return the status; the bytes of
// workspace the plan's current configuration uses and the plan's device.
fbsde_status api_fail(fbsde_status s, const char* msg);
fbsde_status api_active_workspace(const fbsde_plan* plan, size_t* bytes, int* device);

// Plan geometry, passed to every kernel by value.
struct Geo {
  int d;      // state dimension
  int dp;     // row stride of X and V buffers: d rounded up to 4
  int w;      // hidden width
  int L;      // hidden layers (MLP)
  int N;      // time steps
  int M;      // paths
  int ti;     // 16-wide register tiles over d (kernel instantiation; even in bf16 mode)
  int tw;     // 16-wide register tiles over w (kernel instantiation; even in bf16 mode)
  int zp;     // row stride of zeta buffer  = 16 * ti
  int wp;     // row stride of hidden buffers = 16 * tw
  int bf16;   // 1: bf16 MFMA operands
  int sde;    float sde_s;
  int drv;    float drv_p0, drv_p1;
  int g;      float g_p0, g_p1;
  float dt, sqdt;
  long long pstep;        // fp32 parameters per time step (per-step MLP)
  long long nparams;      // total fp32 parameters
  long long pstride;      // floats between two gradient-split partial copies: nparams rounded up to 4
  long long packf_step;   // packed forward fragments per step (elements)
  long long packb_step;   // packed backward fragments per step (elements)
  long long pbias_step;   // padded fp32 biases per step: L * 16 tw + 16 ti
  int lds;                // 1: step weights may be staged in LDS (when they fit); 2: also the fused reverse kernel
  int tpw;                // 16-path tiles per wave of the LDS kernels (0: automatic)
  int kind;               // 0: per-step MLP, 1: shared residual network (L = blocks), 2: u-network
  int uarch;              // u-network blocks: 0 fully connected, 1 residual, 2 NAIS
  float kappa;            // u-network: weight of the terminal-gradient penalty
  float ueps;             // u-network NAIS: A_k = -R_k^T R_k - ueps I
  int rn_chunk;           // residual network: time steps per row chunk; per-step MLP: time steps
                          // per recompute chunk (0: every step's activations are kept)
  int rn_store;           // residual network: 1 = keep every chunk's activations (no recompute)
  // per-step MLP launches over a range of steps: blockIdx.y (or the weight
  // gradient's job) counts from step n0, over ns steps (0: all N); the
  // activation buffers H, DZ, DH hold steps n0 .. n0 + ns - 1 from their row 0
  int n0, ns;
  int recomp;             // forward launch that only recomputes the activations (no Z, c_n, v_n)
};

// steps covered by one per-step-MLP launch
inline int launch_steps(const Geo& g) { return g.ns > 0 ? g.ns : g.N; }

// Shared residual network: packed weights and the per-chunk activation buffers.
struct ResnetLayout {
  int dq;                 // d rounded up to 8
  int ldx;                // row stride of bf16 [x; t]: d + 1 rounded up to 8
  long long pk_elems;     // bf16 packed weights (forward + transposed)
  long long pf_elems;     // fp32 time column and biases
  long long rows;         // rows per chunk = rn_chunk * M
  int ntj;                // column tiles of the output GEMM (its per-row partial sums)
  int nchunks;            // row chunks per pass
  int kept;               // chunks whose activations have their own copy (1, or nchunks if stored)
};
struct ResnetBufs {
  uint16_t* pk;           // packed bf16 weights
  float* pf;              // w_t | b_in | b_k | b_o
  float* h32;             // [rows][w] fp32 residual stream
  uint16_t* hb;           // [kept][B+1][rows][w] bf16 h_0..h_B
  uint16_t* ab;           // [kept][B][rows][w] bf16 a_1..a_B
  float* d32;             // [rows][w] fp32 delta
  uint16_t* gb;           // [2][rows][w] bf16 pre-activation gradients (ping-pong)
  float* rp;              // [ntj][2][rows] fp32 per-tile row sums of the output GEMM
  uint16_t* xb;           // [kept][rows][ldx] bf16 [x; t]
  uint16_t* vb;           // [rows][dq] bf16 zeta = lambda v
};
ResnetLayout resnet_layout(const Geo& g);
hipError_t resnet_pack(const Geo& g, const float* params, uint16_t* pk, float* pf, hipStream_t s);
hipError_t resnet_forward(const Geo& g, const ResnetBufs& R, const float* X, float* V, float* C, hipStream_t s);
hipError_t resnet_backward(const Geo& g, const ResnetBufs& R, const float* X, const float* V, const float* LAM,
                           float* part, int splits, hipStream_t s);

// The paper's own formulation (u-network over all rows r = n M + m,
// n = 0..N): offsets of the flat parameter blocks and the partial-sum rows.
struct UnetLayout {
  long long R;            // rows (N + 1) M
  long long wq;           // row stride of the width-w buffers: w rounded up to 4
  int K;                  // blocks after the input layer
  long long blk;          // parameters per block
  long long off_W0, off_b0, off_blk0, off_wo, off_bo;
  int slots;              // partial sums per parameter
  long long off_abar;     // NAIS: dA_k scratch inside a partial row
  long long pstride;      // floats per partial row
};
struct UnetBufs {
  const float* X;         // [N+1][M][dp] path states (the SDE kernel's X)
  const float* S;         // [N][M][dp] sigma(X_n) dW_n (the SDE kernel's V)
  float* U;               // [R] u
  float* Z;               // [R][dp] grad_x u
  float* UB;              // [R] dL/du
  float* ZB;              // [R][dp] dL/dZ
  float* CB;              // [R] residual weights
  float* H;               // [K+1][R][wq] h_0..h_K
  float* AL;              // [K][R][wq] alpha_1..alpha_K (residual and NAIS; fully connected reads H)
  float* HH;              // [K][R][wq] du/dh_0..du/dh_{K-1}
  float* G;               // [K+1][R][wq] pre-activation gradients of u
  float* HHB;             // [K+1][R][wq] adjoints of HH (HHB_K: of w_o)
  float* HB0;             // [R][wq] h_0-adjoint part from the input-gradient sweep
  float* ALB;             // [K][R][wq] alpha-adjoint parts from the input-gradient sweep
  float* HBAR;            // [R][wq] running h-adjoint of the reverse sweep
  float* ABAR;            // [K+1][R][wq] pre-activation adjoints
  float* W0x;             // [w][dp] x columns of W_0
  float* w0t;             // [w] t column of W_0
  float* Ak;              // [K][w][wq] block matrices A_k
  float* Rk;              // NAIS [K][w][wq] R_k
  float* Ex;              // NAIS [K][w][dp] x columns of E_k
  float* et;              // NAIS [K][w] t column of E_k
  float* P;               // NAIS [R][wq] injection products
  float* Abar;            // NAIS [K][w][w] summed dA_k
  float* part;            // [slots][pstride] weight-gradient partial sums
  double* lpart;          // fp64 loss partials (one per residual workgroup), then an int flag
};
UnetLayout unet_layout(const Geo& g);
// One training evaluation: forward, Z = grad u, residual loss (fp64) and,
// with want_grad, the parameter gradient; u(0, x0) into *y0 (fp64, nullable).
hipError_t unet_forward_backward(const Geo& g, const UnetBufs& B, const float* params, float* grad, double* loss,
                                 double* y0, int* nf, int* host_flag, bool want_grad, hipStream_t s);
// NAIS projection of every R_k (|R_k^T R_k|_F <= c) in place.
hipError_t unet_nais_project(const Geo& g, const UnetBufs& B, float* params, float c, hipStream_t s);

// Offsets (bytes) of the sub-buffers of one workspace.
struct WsLayout {
  size_t X, V, C, Y, LAM, QN, LN, H, DZ, DH, PF, PB, PBIAS, PART, RED, total;
  size_t RPK, RPF, RH32, RHB, RAB, RD32, RGB, RRP, RXB, RVB;  // residual-network buffers
  size_t UU, UZ, UUB, UZB, UH, UAL, UHH, UG, UHHB, UHB0, UALB, UHBAR, UABAR, UW0X, UW0T, UAK, URK, UEX, UET, UP,
      UABARW, UPART, ULP, UCB;  // u-network buffers
  int scan_blocks;
  int splits;
  long long chunk;
};

// launchers (kernels.hip); all return hipError_t of the launch
// the per-iteration weight packing and the SDE in one launch (independent work, one grid)
hipError_t launch_pack_sde(const Geo& g, const float* params, void* packF, void* packB, float* pbias,
                           const float* x0, uint64_t seed, uint64_t iter, const uint64_t* iter_dev, float* X,
                           float* V, float* QN, float* LN, hipStream_t s);
hipError_t launch_sde(const Geo& g, const float* x0, uint64_t seed, uint64_t iter, const uint64_t* iter_dev,
                      float* X, float* V, float* QN, float* LN, hipStream_t s);
hipError_t launch_forward(const Geo& g, const float* params, const void* packF, const float* pbias,
                          const float* X, float* V, float* C, void* H, hipStream_t s);
hipError_t launch_scan(const Geo& g, const double* y0, const float* C, const float* QN, const float* LN,
                       float* Y, float* LAM, double* part, int blocks, hipStream_t s);
hipError_t launch_backward(const Geo& g, const void* packB, const float* V, const float* LAM,
                           const void* H, void* DZ, void* DH, hipStream_t s);
hipError_t launch_wgrad(const Geo& g, const float* X, const void* H, const void* DZ, const void* DH,
                        float* part, int splits, long long chunk, hipStream_t s);
// Reverse sweep and weight gradient in one kernel (fp32 per-step MLP with
// g.lds == 2, depth <= 2, d + 1 <= 16 ti, w + 1 <= 16 tw, fitting LDS); the
// same partials as launch_backward + launch_wgrad with the same splits.
bool reverse_fused_fits(const Geo& g);
// reverse_fused_fits and, for fp32, splits x N within one wave of workgroups over the CUs
bool reverse_fused_preferred(const Geo& g, int splits);
// compute units of the current device (256 if the query fails)
int device_cus();
hipError_t launch_reverse(const Geo& g, const void* packB, const float* X, const float* V, const float* LAM,
                          const void* H, float* part, int splits, long long chunk, hipStream_t s);
// The scan's partials are followed by an int flag: cleared by the scan, set
// by the reduction on a non-finite gradient; the finalize step folds it (and
// the loss, dL/dY0) into *host_flag (pinned host memory) and clears it.
hipError_t launch_reduce(const Geo& g, const float* part, int splits, float* grad, double* scan_part,
                         int scan_blocks, double* loss, double* grad_y0, int* host_flag, hipStream_t s);
// Adam state and hyper-parameters of one step (y0, my0, vy0 may be null
// together: no scalar y0 to train).
struct AdamArgs {
  float *p, *m, *v;
  double *y0, *my0, *vy0;
  double lr, t;
  const uint64_t* t_dev;  // step read on the device (t_dev[0] + 1) when non-null
  double lr_y0, b1, b2, eps;
};
// launch_reduce followed by Adam on params and y0, in one launch
hipError_t launch_reduce_adam(const Geo& g, const float* part, int splits, float* grad, double* scan_part,
                              int scan_blocks, double* loss, double* grad_y0, int* host_flag, const AdamArgs& a,
                              hipStream_t s);
hipError_t launch_loss_only(const Geo& g, double* scan_part, int scan_blocks, double* loss, int* host_flag,
                            hipStream_t s);
hipError_t launch_adam(long long n, float* p, const float* gr, float* m, float* v, double* y0,
                       const double* gy0, double* my0, double* vy0, float lr, double t, const uint64_t* t_dev,
                       double lr_y0, double b1, double b2, double eps, hipStream_t s);
hipError_t launch_count(uint64_t* c, hipStream_t s);
hipError_t launch_prolong(const Geo& coarse, const Geo& fine, const float* pc, float* pf, hipStream_t s);
hipError_t launch_normals(const Geo& g, uint64_t seed, uint64_t iter, float* xi, hipStream_t s);
hipError_t launch_gmean(const Geo& g, const float* QN, const float* LN, double* out, hipStream_t s);
hipError_t launch_terminal_copy(const Geo& g, const float* X, const float* Y, float* xN, float* yN,
                                hipStream_t s);

// Register-tile shape of the fused MLP kernels: the smallest instantiated
// (ti, tw) with ti >= ti_min, tw >= tw_min.  Returns false if none exists.
bool choose_tiles(int bf16, int ti_min, int tw_min, int* ti, int* tw);
// All instantiated shapes covering (ti_min, tw_min), cheapest first; returns the count (<= cap).
int tile_candidates(int bf16, int ti_min, int tw_min, int* ti, int* tw, int cap);
// Whether the forward / backward step weights of this geometry fit in LDS.
bool lds_fits(const Geo& g);
int auto_tiles_per_wave(const Geo& g);

}  // namespace fbsde
