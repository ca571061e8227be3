// gfx950 kernels of the deep-FBSDE hot path.
//
// One training iteration (Deep-BSDE form of Sec. 2.2 of Güler, Laignelet,
// Parpas, arXiv 1910.11623) is, in launch order:
//   pack      flat fp32 parameters -> MFMA A-fragments (forward W, backward W^T)
//   sde       Philox + Box–Muller increments, Euler–Maruyama X_n, s_n = sigma(X_n) dW_n
//             (eq. disc equations; mu = 0), and |X_N|^2, sum X_N per path
//   forward   per (step n, tile of 16 paths per wave): Z_n = NN_n(X_n) on MFMA, the Z-dependent part
//             c_n of the Y update and v_n = phi_z dt + s_n
//   scan      per path: Y_{n+1} = Y_n + dt phi_y(Y_n) + c_n, terminal mismatch,
//             fp64 loss partials, lambda_n = dL/dY_n, fp64 dL/dY0 partials
//   backward  per (step n, tile of 16 paths per wave): zeta_n = lambda_{n+1} v_n, deltas through
//             NN_n on MFMA
//   wgrad     dW = sum over paths of delta (x) activation, split over path ranges
//   reduce    fixed-order sum of the split partials into the flat gradient
//
// Because mu and sigma never depend on (Y, Z), X_n does not depend on the
// network parameters: every network evaluation of every step runs in
// parallel; only the scalar Y and lambda recursions are sequential.
//
// MFMA operand layouts (16x16 output tiles, wave64): lane l holds
//   A[row l%16][k-slot l/16], B[k-slot l/16][col l%16], D[4*(l/16)+r][l%16].
// Activations are kept feature-major ("transposed"): output rows are
// features, columns are 16 paths, so a layer's D registers serve directly as
// the next layer's B operand once the K order of the next weight matrix is
// permuted to match (done once per iteration by the pack kernel).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>

#include "fbsde_internal.h"

namespace fbsde {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

enum { SDE_GBM = 0, SDE_BM = 1 };
enum { DRV_BSB = 0, DRV_HJB = 1, DRV_AC = 2, DRV_LIN = 3 };
enum { G_NORM2 = 0, G_LOGHALF = 1, G_INV = 2, G_LIN = 3 };

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ uint32_t bf16_bits(float f) {  // round to nearest even
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ __forceinline__ float rbf(float f) { return __uint_as_float(bf16_bits(f) << 16); }
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16x8 pack8(f32x4 lo, f32x4 hi) {
  u32x4 u;
  u[0] = bf16_bits(lo[0]) | (bf16_bits(lo[1]) << 16);
  u[1] = bf16_bits(lo[2]) | (bf16_bits(lo[3]) << 16);
  u[2] = bf16_bits(hi[0]) | (bf16_bits(hi[1]) << 16);
  u[3] = bf16_bits(hi[2]) | (bf16_bits(hi[3]) << 16);
  return __builtin_bit_cast(bf16x8, u);
}

__device__ __forceinline__ f32x4 mfma_f32(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma_bf16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// tanh without a division: for |x| >= 0.4, sign(x) (1 - 2 / (exp(2|x|) + 1))
// with the hardware base-2 exponential and reciprocal (saturates to +-1);
// below 0.4 the odd Taylor series through x^13 (truncation < 4e-9
// relative), which keeps the relative error at a few ulp near zero.
__device__ __forceinline__ float fast_tanh(float x) {
  const float ax = fabsf(x);
  const float e = __builtin_amdgcn_exp2f(2.8853900817779268f * ax);  // exp(2|x|)
  const float big = fmaf(-2.0f, __builtin_amdgcn_rcpf(e + 1.0f), 1.0f);
  const float x2 = ax * ax;
  float q = 21844.0f / 6081075.0f;
  q = fmaf(q, x2, -1382.0f / 155925.0f);
  q = fmaf(q, x2, 62.0f / 2835.0f);
  q = fmaf(q, x2, -17.0f / 315.0f);
  q = fmaf(q, x2, 2.0f / 15.0f);
  q = fmaf(q, x2, -1.0f / 3.0f);
  const float small = fmaf(ax * x2, q, ax);
  return copysignf(ax < 0.4f ? small : big, x);
}

__device__ __forceinline__ f32x4 zero4() { return f32x4{0.f, 0.f, 0.f, 0.f}; }

__device__ __forceinline__ f32x4 ld4(const float* p) { return *reinterpret_cast<const f32x4*>(p); }
__device__ __forceinline__ void st4(float* p, f32x4 v) { *reinterpret_cast<f32x4*>(p) = v; }

// 4 activations of one lane, fp32 or bf16 storage
__device__ __forceinline__ f32x4 ld_act(const void* base, size_t idx, bool bf) {
  if (!bf) return ld4(reinterpret_cast<const float*>(base) + idx);
  uint2 u = *reinterpret_cast<const uint2*>(reinterpret_cast<const uint16_t*>(base) + idx);
  return f32x4{__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xffff0000u),
               __uint_as_float(u.y << 16), __uint_as_float(u.y & 0xffff0000u)};
}
__device__ __forceinline__ void st_act(void* base, size_t idx, f32x4 v, bool bf) {
  if (!bf) { st4(reinterpret_cast<float*>(base) + idx, v); return; }
  uint2 u;
  u.x = bf16_bits(v[0]) | (bf16_bits(v[1]) << 16);
  u.y = bf16_bits(v[2]) | (bf16_bits(v[3]) << 16);
  *reinterpret_cast<uint2*>(reinterpret_cast<uint16_t*>(base) + idx) = u;
}
__device__ __forceinline__ f32x4 round4(f32x4 v, bool bf) {
  if (!bf) return v;
  return f32x4{rbf(v[0]), rbf(v[1]), rbf(v[2]), rbf(v[3])};
}

// ------------------------------------------------------------ Philox4x32-10
// Salmon, Moraes, Dror, Shaw (SC'11): 10 rounds, multipliers 0xD2511F53 and
// 0xCD9E8D57, Weyl key increments 0x9E3779B9 and 0xBB67AE85.
__device__ __forceinline__ void philox10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                         uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // one 32 x 32 -> 64-bit product per multiplier (v_mad_u64_u32) gives
    // both halves, instead of separate high and low multiplies
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
  }
}

// Box–Muller: U = ((a >> 8) + 1) 2^-24 in (0,1], V = (b >> 8) 2^-24 in [0,1).
// The transcendentals are the hardware ones: log2 (-2 ln U = -2 ln2 log2 U)
// and sin/cos of 2 pi V with V in revolutions; against fp64 libm the
// normals differ by at most 1.6e-7 (1 + |z|).
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, float& z0, float& z1) {
  const float U = (float)((a >> 8) + 1u) * 5.9604644775390625e-8f;
  const float V = (float)(b >> 8) * 5.9604644775390625e-8f;
  const float r = sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(U));
  const float sn = __builtin_amdgcn_sinf(V), cs = __builtin_amdgcn_cosf(V);
  z0 = r * cs;
  z1 = r * sn;
}

// four normals for dims 4j..4j+3 of path m at step n
__device__ __forceinline__ f32x4 normals4(uint64_t seed, uint64_t iter, int j, int n, int m) {
  uint32_t c0 = (uint32_t)j, c1 = (uint32_t)n, c2 = (uint32_t)m, c3 = (uint32_t)iter;
  philox10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
  float a0, a1, a2, a3;
  box_muller(c0, c1, a0, a1);
  box_muller(c2, c3, a2, a3);
  return f32x4{a0, a1, a2, a3};
}

// Row block of step n in the activation buffers (H, DZ, DH) of a per-step
// MLP launch: they hold the launch's steps n0 .. n0 + ns - 1 (all N steps
// unless activations are recomputed in chunks of steps).
__device__ __forceinline__ size_t act_step(const Geo& g, int n) { return (size_t)(n - g.n0); }

// -------------------------------------------------------------- pack kernel
// Packed A-fragment of a (R x K) matrix A with 16-row tiles T and K tiles t:
//   fp32: elem ((T*Ti + t)*64 + lane)*4 + r   <- A[16T + lane%16][16t + 4(lane/16) + r]
//   bf16: elem ((T*Ti/2 + kb)*64 + lane)*8 + j <- A[16T + lane%16][32kb + 16(j/4) + 4(lane/16) + j%4]
// (A = W for the forward, A = W^T for the backward.)
__device__ __forceinline__ float packed_value(const float* W, int rows, int cols, bool trans, int To,
                                              int Ti, int e, bool bf) {
  int row, col;
  if (!bf) {
    const int r = e & 3;
    const int q = e >> 2;
    const int lane = q & 63;
    const int tt = q >> 6;
    const int t = tt % Ti, T = tt / Ti;
    row = 16 * T + (lane & 15);
    col = 16 * t + 4 * (lane >> 4) + r;
  } else {
    const int j = e & 7;
    const int q = e >> 3;
    const int lane = q & 63;
    const int tt = q >> 6;
    const int nkb = Ti / 2;
    const int kb = tt % nkb, T = tt / nkb;
    row = 16 * T + (lane & 15);
    col = 32 * kb + 16 * (j >> 2) + 4 * (lane >> 4) + (j & 3);
  }
  (void)To;
  const int R = trans ? cols : rows, K = trans ? rows : cols;
  if (row >= R || col >= K) return 0.f;
  return trans ? W[(long long)col * cols + row] : W[(long long)row * cols + col];
}

// One row of workgroups per step (blockIdx.y = n - 1); 32-bit indices
// inside a step's packed block.  A thread produces one packed group (4 fp32
// or 8 bf16 elements: the register fragment of one lane) and stores it as
// one vector.
template <bool BF>
__device__ __forceinline__ void pack_group(const float* W, int rows, int cols, bool trans, int To, int Ti,
                                           int e0, void* dst) {
  constexpr int G = BF ? 8 : 4;
  float v[G];
#pragma unroll
  for (int k = 0; k < G; ++k) v[k] = packed_value(W, rows, cols, trans, To, Ti, e0 + k, BF);
  if constexpr (BF) {
    uint4 u;
    u.x = bf16_bits(v[0]) | (bf16_bits(v[1]) << 16);
    u.y = bf16_bits(v[2]) | (bf16_bits(v[3]) << 16);
    u.z = bf16_bits(v[4]) | (bf16_bits(v[5]) << 16);
    u.w = bf16_bits(v[6]) | (bf16_bits(v[7]) << 16);
    *reinterpret_cast<uint4*>(dst) = u;
  } else {
    *reinterpret_cast<f32x4*>(dst) = f32x4{v[0], v[1], v[2], v[3]};
  }
}

// Block bx of gx packing step n's fragments.
template <bool BF>
__device__ __forceinline__ void pack_block(const Geo& g, const float* __restrict__ params, void* __restrict__ packF,
                                           void* __restrict__ packB, float* __restrict__ pbias, int bx, int gx,
                                           int n) {
  constexpr int G = BF ? 8 : 4;          // elements per packed group
  constexpr int ESZ = BF ? 2 : 4;
  const int pf = (int)g.packf_step / G, pb = (int)g.packb_step / G;  // groups (every block is whole groups)
  const int nb = (int)g.pbias_step;
  const int per = pf + pb + nb;
  const float* base = params + g.d + (long long)(n - 1) * g.pstep;
  const int lw1 = g.w * g.d + g.w, lwh = g.w * g.w + g.w;
  const int sz_in = 256 * g.tw * g.ti, sz_h = 256 * g.tw * g.tw, sz_o = 256 * g.ti * g.tw;
  char* F = reinterpret_cast<char*>(packF) + (size_t)(n - 1) * g.packf_step * ESZ;
  char* Bk = reinterpret_cast<char*>(packB) + (size_t)(n - 1) * g.packb_step * ESZ;
  for (int q = bx * 256 + threadIdx.x; q < per; q += gx * 256) {
    if (q >= pf + pb) {  // biases, zero padded: b_1..b_L (16 tw each), b_o (16 ti)
      const int qb = q - pf - pb;
      const int hb = 16 * g.tw;
      float val = 0.f;
      if (qb < g.L * hb) {
        const int l = 1 + qb / hb, i = qb % hb;
        const float* bl = base + (l == 1 ? g.w * g.d : lw1 + (l - 2) * lwh + g.w * g.w);
        if (i < g.w) val = bl[i];
      } else {
        const int i = qb - g.L * hb;
        if (i < g.d) val = base[lw1 + (g.L - 1) * lwh + g.d * g.w + i];
      }
      pbias[(long long)(n - 1) * g.pbias_step + qb] = val;
      continue;
    }
    if (q < pf) {  // forward: W1, W2..WL, Wo
      const int e = q * G;
      char* dst = F + (size_t)e * ESZ;
      if (e < sz_in) {
        pack_group<BF>(base, g.w, g.d, false, g.tw, g.ti, e, dst);
      } else if (e < sz_in + (g.L - 1) * sz_h) {
        const int qq = e - sz_in;
        const int l = 2 + qq / sz_h;
        pack_group<BF>(base + lw1 + (l - 2) * lwh, g.w, g.w, false, g.tw, g.tw, qq % sz_h, dst);
      } else {
        const int qq = e - sz_in - (g.L - 1) * sz_h;
        pack_group<BF>(base + lw1 + (g.L - 1) * lwh, g.d, g.w, false, g.ti, g.tw, qq, dst);
      }
    } else {  // backward: Wo^T (for delta_L), then W_{l+1}^T for delta_l, l = 1..L-1
      const int e = (q - pf) * G;
      char* dst = Bk + (size_t)e * ESZ;
      if (e < sz_o) {
        pack_group<BF>(base + lw1 + (g.L - 1) * lwh, g.d, g.w, true, g.tw, g.ti, e, dst);
      } else {
        const int qq = e - sz_o;
        const int l = 1 + qq / sz_h;  // delta_l uses W_{l+1}
        pack_group<BF>(base + lw1 + (l - 1) * lwh, g.w, g.w, true, g.tw, g.tw, qq % sz_h, dst);
      }
    }
  }
}

// --------------------------------------------------------------- SDE kernel
// A path's G = dp / 4 groups of 4 dims are spread over T = min(G, 256)
// consecutive threads of a block (thread j takes groups j, j + T, ...); a
// block holds floor(256 / T) whole paths, so |X_N|^2 and sum X_N reduce in
// LDS in a fixed order: per thread over its groups, then over the path's T
// threads.
__device__ __forceinline__ int sde_threads_per_path(int dp) { return min(dp / 4, 256); }

// Block bx of the SDE grid.
__device__ __forceinline__ void sde_block(const Geo& g, const float* __restrict__ x0, uint64_t seed,
                                          uint64_t iter_imm, const uint64_t* __restrict__ iter_dev,
                                          float* __restrict__ X, float* __restrict__ V, float* __restrict__ QN,
                                          float* __restrict__ LN, int bx) {
  const uint64_t iter = iter_dev ? iter_dev[0] : iter_imm;
  __shared__ float sq[256], sl[256];
  const int G = g.dp / 4;
  const int T = sde_threads_per_path(g.dp);
  const int ppb = 256 / T;
  const int lp = threadIdx.x / T, j0 = threadIdx.x % T;
  const int m = bx * ppb + lp;
  const bool active = lp < ppb && m < g.M;
  float q = 0.f, lin = 0.f;
  if (active) {
    const size_t rowM = (size_t)g.M * g.dp;
    for (int j = j0; j < G; j += T) {
      f32x4 x = ld4(x0 + 4 * j);
      const size_t off = (size_t)m * g.dp + 4 * j;
      for (int n = 0; n < g.N; ++n) {
        const f32x4 z = normals4(seed, iter, j, n, m);
        f32x4 s;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float dw = g.sqdt * z[r];
          s[r] = (4 * j + r < g.d) ? (g.sde == SDE_GBM ? g.sde_s * x[r] * dw : g.sde_s * dw) : 0.f;
        }
        st4(X + n * rowM + off, x);
        st4(V + n * rowM + off, s);
        x += s;
      }
      st4(X + (size_t)g.N * rowM + off, x);
      q += x[0] * x[0] + x[1] * x[1] + x[2] * x[2] + x[3] * x[3];
      lin += x[0] + x[1] + x[2] + x[3];
    }
  }
  sq[threadIdx.x] = q;
  sl[threadIdx.x] = lin;
  __syncthreads();
  if (active && j0 == 0) {
    // the path's T threads are threadIdx.x .. threadIdx.x + T - 1 < 256
    float a = 0.f, b = 0.f;
    for (int k = 0; k < T; ++k) { a += sq[threadIdx.x + k]; b += sl[threadIdx.x + k]; }
    QN[m] = a;
    LN[m] = b;
  }
}

__global__ __launch_bounds__(256) void k_sde(Geo g, const float* __restrict__ x0, uint64_t seed,
                                             uint64_t iter_imm, const uint64_t* __restrict__ iter_dev,
                                             float* __restrict__ X, float* __restrict__ V,
                                             float* __restrict__ QN, float* __restrict__ LN) {
  sde_block(g, x0, seed, iter_imm, iter_dev, X, V, QN, LN, blockIdx.x);
}

// The per-iteration packing of the step weights and the SDE are independent:
// one launch runs both.  Blocks [0, sde_blocks) simulate (each runs a long
// serial chain over the steps, so they are dispatched first), the rest pack
// (pack_gx per step) on the CU slots the SDE leaves free.
template <bool BF>
__global__ __launch_bounds__(256) void k_pack_sde(Geo g, const float* __restrict__ params, void* __restrict__ packF,
                                                  void* __restrict__ packB, float* __restrict__ pbias, int pack_gx,
                                                  int sde_blocks, const float* __restrict__ x0, uint64_t seed,
                                                  uint64_t iter_imm, const uint64_t* __restrict__ iter_dev,
                                                  float* __restrict__ X, float* __restrict__ V,
                                                  float* __restrict__ QN, float* __restrict__ LN) {
  const int b = blockIdx.x;
  if (b < sde_blocks) {
    sde_block(g, x0, seed, iter_imm, iter_dev, X, V, QN, LN, b);
  } else {
    const int q = b - sde_blocks;
    pack_block<BF>(g, params, packF, packB, pbias, q % pack_gx, pack_gx, 1 + q / pack_gx);
  }
}

// -------------------------------------------------------- MFMA layer product
// acc[T] = sum_k A_T,k * in_k over all TIN K tiles of `in` (registers, D
// layout).  Tile counts are compile-time: padded tiles carry zero weights,
// so there is no runtime guard inside the unrolled MFMA chains.
template <bool BF, int TO, int TIN>
__device__ __forceinline__ void layer_mm(f32x4 (&acc)[TO], const f32x4 (&in)[TIN], const void* pack,
                                         int lane) {
#pragma unroll
  for (int T = 0; T < TO; ++T) acc[T] = zero4();
  if constexpr (!BF) {
    // one 16-byte fragment (4 K steps of one output tile) at a time: the
    // four MFMAs on it accumulate back to back into the same tile, and only
    // a few fragments are live, which leaves registers for the callers'
    // early loads
    const f32x4* A = reinterpret_cast<const f32x4*>(pack);
#pragma unroll
    for (int t = 0; t < TIN; ++t)
#pragma unroll
      for (int T = 0; T < TO; ++T) {
        const f32x4 a = A[((size_t)T * TIN + t) * 64 + lane];
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[T] = mfma_f32(a[r], in[t][r], acc[T]);
      }
  } else {
    static_assert(TIN % 2 == 0, "bf16 K blocks span two tiles");
    const bf16x8* A = reinterpret_cast<const bf16x8*>(pack);
#pragma unroll
    for (int kb = 0; kb < TIN / 2; ++kb) {
      const bf16x8 b = pack8(in[2 * kb], in[2 * kb + 1]);
#pragma unroll
      for (int T = 0; T < TO; ++T) acc[T] = mfma_bf16(A[((size_t)T * (TIN / 2) + kb) * 64 + lane], b, acc[T]);
    }
  }
}

__device__ __forceinline__ f32x4 bias4(const float* b, int base, int n) {
  f32x4 v;
#pragma unroll
  for (int r = 0; r < 4; ++r) v[r] = (base + r < n) ? b[base + r] : 0.f;
  return v;
}

// Path tiles (16 paths each) of one step are split evenly over the
// workgroups of that step (blockIdx.x); inside a workgroup, wave w takes
// tiles t0 + w, t0 + w + waves, ... so the per-wave counts differ by at most
// one and consecutive waves read consecutive paths.
struct TileRange { int t0, t1; };
__device__ __forceinline__ TileRange tile_range(int M) {
  const int tiles = (M + 15) / 16;
  const int per = (tiles + (int)gridDim.x - 1) / (int)gridDim.x;
  const int t0 = (int)blockIdx.x * per;
  return TileRange{t0, min(tiles, t0 + per)};
}

// ----------------------------------------------------------- forward kernel
// Copy `bytes` (a multiple of 16) from global memory into LDS without the
// barrier.  Each thread issues up to 16 loads of 16 bytes before its first
// LDS write, so a step's fragments (~150 KB over 768 threads) arrive after
// one memory latency instead of one per 16-byte row.  Indices past the end
// are clamped to the last row (those lanes write the same value to the same
// LDS row), so loads and writes are unconditional and all loads are in
// flight together.
__device__ __forceinline__ void copy_to_lds(unsigned char* dst, const void* src, size_t bytes) {
  constexpr int B = 16;
  const uint4* s = reinterpret_cast<const uint4*>(src);
  uint4* d = reinterpret_cast<uint4*>(dst);
  const int n = (int)(bytes / 16), stride = (int)blockDim.x;
  if (n <= 0) return;
  for (int base = (int)threadIdx.x; base < n; base += B * stride) {
    uint4 r[B];
#pragma unroll
    for (int k = 0; k < B; ++k) r[k] = s[min(base + k * stride, n - 1)];
#pragma unroll
    for (int k = 0; k < B; ++k) d[min(base + k * stride, n - 1)] = r[k];
  }
}

// Copy one step's packed fragments (bytes, multiple of 16) into LDS.
__device__ __forceinline__ void stage_weights(unsigned char* dst, const void* src, size_t bytes) {
  copy_to_lds(dst, src, bytes);
  __syncthreads();
}

// LDSW = false: one 16-path tile per wave, fragments read from global memory.
// LDSW = true : the workgroup stages step n's fragments in LDS once, then its
//               waves stream its share of the step's 16-path tiles (at most
//               `tpw` each, see tile_range) through them.
// Waves per workgroup of the LDS-staged forward kernel (one workgroup per
// CU): 3 per SIMD for shapes up to 8 x 8 tiles (<= 170 VGPRs), else 2.
constexpr int fwd_waves(int ti, int tw) { return (ti <= 8 && tw <= 8) ? 12 : 8; }

// RC: recompute launch (activations only).  A compile-time switch: as a
// run-time test inside the tile loop it cost the ordinary forward its
// register budget (spills; bf16 51 -> 70 us at d = 100).
template <bool BF, int TI, int TW, bool LDSW, bool RC = false>
__global__ __launch_bounds__(LDSW ? 64 * fwd_waves(TI, TW) : 256) void k_forward(Geo g, const float* __restrict__ params,
                                                               const void* __restrict__ packF,
                                                               const float* __restrict__ pbias,
                                                               const float* __restrict__ X,
                                                               float* __restrict__ V, float* __restrict__ C,
                                                               void* __restrict__ H, int tpw) {
  extern __shared__ __attribute__((aligned(16))) unsigned char wsm[];
  const int n = g.n0 + (int)blockIdx.y;
  if (RC && n == 0) return;  // step 0 has no network
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nwv = blockDim.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const size_t rowM = (size_t)g.M * g.dp;
  const size_t esz = BF ? 2 : 4;
  const char* pk;
  const float* bp;
  if constexpr (LDSW) {
    if (n > 0) {
      const size_t wbytes = (size_t)g.packf_step * esz;
      copy_to_lds(wsm + wbytes, pbias + (size_t)(n - 1) * g.pbias_step, (size_t)g.pbias_step * 4);
      stage_weights(wsm, reinterpret_cast<const char*>(packF) + (size_t)(n - 1) * wbytes, wbytes);
    }
    pk = reinterpret_cast<const char*>(wsm);
    bp = reinterpret_cast<const float*>(wsm + (size_t)g.packf_step * esz);
  } else {
    pk = reinterpret_cast<const char*>(packF) + (size_t)(n > 0 ? n - 1 : 0) * g.packf_step * esz;
    bp = pbias + (size_t)(n > 0 ? n - 1 : 0) * g.pbias_step;
  }
  // rows of X_n and (up to 8 tiles of d) s_n are loaded at the start of
  // their tile, before the tile's activation stores: vector-memory operations
  // complete in order, so a load issued after those stores would also wait
  // for their writes.  Wider s rows are loaded in the epilogue (registers).
  const float* Xn = X + n * rowM;
  float* Vn = V + n * rowM;
  const TileRange tr = tile_range(g.M);
  for (int it = 0; it < tpw; ++it) {
  const int tile = tr.t0 + it * nwv + wv;
  if (tile >= tr.t1) break;
  const int p = tile * 16 + col;
  const bool valid = p < g.M;
  f32x4 xv[TI];
#pragma unroll
  for (int t = 0; t < TI; ++t) {
    const int c0 = 16 * t + 4 * grp;
    xv[t] = (valid && c0 < g.dp) ? ld4(Xn + (size_t)p * g.dp + c0) : zero4();
  }
  constexpr bool SE = TI <= 8;
  f32x4 sv[SE ? TI : 1];
  if constexpr (SE) {
#pragma unroll
    for (int t = 0; t < TI; ++t) {
      const int c0 = 16 * t + 4 * grp;
      sv[t] = (valid && c0 < g.dp) ? ld4(Vn + (size_t)p * g.dp + c0) : zero4();
    }
  }
  f32x4 Z[TI];
  if (n == 0) {
#pragma unroll
    for (int t = 0; t < TI; ++t) Z[t] = bias4(params, 16 * t + 4 * grp, g.d);  // Z_0 = z0
  } else {
    f32x4 h[TW], acc[TW];
    layer_mm<BF, TW, TI>(acc, xv, pk, lane);  // bf16: pack8 rounds X to nearest even
    const size_t hM = (size_t)g.M * g.wp;
#pragma unroll
    for (int T = 0; T < TW; ++T) {
      const f32x4 bb = ld4(bp + 16 * T + 4 * grp);
#pragma unroll
      for (int r = 0; r < 4; ++r) h[T][r] = fast_tanh(acc[T][r] + bb[r]);
      h[T] = round4(h[T], BF);
      if (valid)
        st_act(H, (act_step(g, n) * g.L) * hM + (size_t)p * g.wp + 16 * T + 4 * grp, h[T], BF);
    }
    const char* pkl = pk + 256ULL * TW * TI * esz;
    for (int l = 2; l <= g.L; ++l) {
      layer_mm<BF, TW, TW>(acc, h, pkl, lane);
      const float* bl = bp + (size_t)(l - 1) * 16 * TW;
#pragma unroll
      for (int T = 0; T < TW; ++T) {
        const f32x4 bb = ld4(bl + 16 * T + 4 * grp);
#pragma unroll
        for (int r = 0; r < 4; ++r) h[T][r] = fast_tanh(acc[T][r] + bb[r]);
        h[T] = round4(h[T], BF);
        if (valid)
          st_act(H, (act_step(g, n) * g.L + (l - 1)) * hM + (size_t)p * g.wp + 16 * T + 4 * grp, h[T], BF);
      }
      pkl += 256ULL * TW * TW * esz;
    }
    if constexpr (RC) continue;  // the activations were all that was asked for
    layer_mm<BF, TI, TW>(Z, h, pkl, lane);
    const float* bo = bp + (size_t)g.L * 16 * TW;
#pragma unroll
    for (int t = 0; t < TI; ++t) Z[t] += ld4(bo + 16 * t + 4 * grp);
  }
  // epilogue: c_n = Z.s + dt * (Z-part of phi), v_n = s + dt * phi_z
  float cz = 0.f, cx = 0.f;
#pragma unroll
  for (int t = 0; t < TI; ++t) {
    const int c0 = 16 * t + 4 * grp;
    if (valid && c0 < g.dp) {
      float* vp = Vn + (size_t)p * g.dp + c0;
      f32x4 s;
      if constexpr (SE) s = sv[t];
      else s = ld4(vp);
      f32x4 v = s;
      if (g.drv == DRV_BSB) {
        const f32x4 x = xv[t];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          cz += Z[t][r] * s[r];
          cx += Z[t][r] * x[r];
          v[r] = s[r] - g.drv_p0 * g.dt * x[r];
        }
      } else if (g.drv == DRV_HJB) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          cz += Z[t][r] * s[r];
          cx += Z[t][r] * Z[t][r];
          v[r] = s[r] + 2.f * g.drv_p0 * g.dt * Z[t][r];
        }
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) cz += Z[t][r] * s[r];
      }
      st4(vp, v);
    }
  }
  float c = cz;
  if (g.drv == DRV_BSB) c -= g.dt * g.drv_p0 * cx;
  else if (g.drv == DRV_HJB) c += g.dt * g.drv_p0 * cx;
  c += __shfl_xor(c, 16);
  c += __shfl_xor(c, 32);
  if (valid && grp == 0) C[(size_t)n * g.M + p] = c;
  }
}

// ------------------------------------------------ layer-streamed forward
// For step networks whose packed weights do not fit LDS at once (fp32 8 x 8,
// bf16 12 x 12 .. 16 x 16 tiles): the workgroup stages one layer's fragments
// at a time and runs that layer over all of its tiles, the tanh activations
// going through H (which the reverse sweep reads anyway) from one layer to
// the next.  Each step's weights cross from L2 into LDS once per workgroup,
// instead of once per 16-path tile from L2 into registers.  Layer products,
// rounding and epilogues are those of k_forward, so both give bitwise equal
// results.
constexpr int LS_WAVES = 8;

template <bool BF>
__device__ __forceinline__ void ls_stage(unsigned char* lds, const void* src, size_t bytes) {
  __syncthreads();  // every wave is done with the previous layer's fragments
  copy_to_lds(lds, src, bytes);
  __syncthreads();
}

template <bool BF, int TI, int TW>
__global__ __launch_bounds__(64 * LS_WAVES) void k_forward_ls(Geo g, const float* __restrict__ params,
                                                              const void* __restrict__ packF,
                                                              const float* __restrict__ pbias,
                                                              const float* __restrict__ X, float* __restrict__ V,
                                                              float* __restrict__ C, void* __restrict__ H, int tpw) {
  extern __shared__ __attribute__((aligned(16))) unsigned char wsm[];
  const int n = g.n0 + (int)blockIdx.y;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nwv = LS_WAVES;
  const int col = lane & 15, grp = lane >> 4;
  const size_t rowM = (size_t)g.M * g.dp, hM = (size_t)g.M * g.wp;
  const size_t esz = BF ? 2 : 4;
  const float* Xn = X + n * rowM;
  float* Vn = V + n * rowM;
  const TileRange tr = tile_range(g.M);
  // c_n = Z.s + dt * (Z-part of phi), v_n = s + dt * phi_z (as k_forward)
  auto epilogue = [&](int p, bool valid, const f32x4 (&Z)[TI]) {
    float cz = 0.f, cx = 0.f;
#pragma unroll
    for (int t = 0; t < TI; ++t) {
      const int c0 = 16 * t + 4 * grp;
      if (valid && c0 < g.dp) {
        float* vp = Vn + (size_t)p * g.dp + c0;
        const f32x4 s = ld4(vp);
        f32x4 v = s;
        if (g.drv == DRV_BSB) {
          const f32x4 x = ld4(Xn + (size_t)p * g.dp + c0);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            cz += Z[t][r] * s[r];
            cx += Z[t][r] * x[r];
            v[r] = s[r] - g.drv_p0 * g.dt * x[r];
          }
        } else if (g.drv == DRV_HJB) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            cz += Z[t][r] * s[r];
            cx += Z[t][r] * Z[t][r];
            v[r] = s[r] + 2.f * g.drv_p0 * g.dt * Z[t][r];
          }
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r) cz += Z[t][r] * s[r];
        }
        st4(vp, v);
      }
    }
    float c = cz;
    if (g.drv == DRV_BSB) c -= g.dt * g.drv_p0 * cx;
    else if (g.drv == DRV_HJB) c += g.dt * g.drv_p0 * cx;
    c += __shfl_xor(c, 16);
    c += __shfl_xor(c, 32);
    if (valid && grp == 0) C[(size_t)n * g.M + p] = c;
  };
  if (n == 0) {  // Z_0 = z0
    if (g.recomp) return;
    for (int it = 0; it < tpw; ++it) {
      const int tile = tr.t0 + it * nwv + wv;
      if (tile >= tr.t1) break;
      const int p = tile * 16 + col;
      f32x4 Z[TI];
#pragma unroll
      for (int t = 0; t < TI; ++t) Z[t] = bias4(params, 16 * t + 4 * grp, g.d);
      epilogue(p, p < g.M, Z);
    }
    return;
  }
  const char* F = reinterpret_cast<const char*>(packF) + (size_t)(n - 1) * g.packf_step * esz;
  const float* bp = pbias + (size_t)(n - 1) * g.pbias_step;
  // layer 1: x -> h_1
  ls_stage<BF>(wsm, F, 256ULL * TW * TI * esz);
  for (int it = 0; it < tpw; ++it) {
    const int tile = tr.t0 + it * nwv + wv;
    if (tile >= tr.t1) break;
    const int p = tile * 16 + col;
    const bool valid = p < g.M;
    f32x4 xv[TI], acc[TW];
#pragma unroll
    for (int t = 0; t < TI; ++t) {
      const int c0 = 16 * t + 4 * grp;
      xv[t] = (valid && c0 < g.dp) ? ld4(Xn + (size_t)p * g.dp + c0) : zero4();
    }
    layer_mm<BF, TW, TI>(acc, xv, wsm, lane);
#pragma unroll
    for (int T = 0; T < TW; ++T) {
      const f32x4 bb = ld4(bp + 16 * T + 4 * grp);
      f32x4 h;
#pragma unroll
      for (int r = 0; r < 4; ++r) h[r] = fast_tanh(acc[T][r] + bb[r]);
      h = round4(h, BF);
      if (valid) st_act(H, (act_step(g, n) * g.L) * hM + (size_t)p * g.wp + 16 * T + 4 * grp, h, BF);
    }
  }
  size_t foff = 256ULL * TW * TI;
  // hidden layers l = 2..L: h_{l-1} -> h_l (h_{l-1} read back from H)
  for (int l = 2; l <= g.L; ++l) {
    ls_stage<BF>(wsm, F + foff * esz, 256ULL * TW * TW * esz);
    const float* bl = bp + (size_t)(l - 1) * 16 * TW;
    for (int it = 0; it < tpw; ++it) {
      const int tile = tr.t0 + it * nwv + wv;
      if (tile >= tr.t1) break;
      const int p = tile * 16 + col;
      const bool valid = p < g.M;
      f32x4 hin[TW], acc[TW];
#pragma unroll
      for (int T = 0; T < TW; ++T)
        hin[T] = valid ? ld_act(H, (act_step(g, n) * g.L + (l - 2)) * hM + (size_t)p * g.wp + 16 * T + 4 * grp, BF)
                       : zero4();
      layer_mm<BF, TW, TW>(acc, hin, wsm, lane);
#pragma unroll
      for (int T = 0; T < TW; ++T) {
        const f32x4 bb = ld4(bl + 16 * T + 4 * grp);
        f32x4 h;
#pragma unroll
        for (int r = 0; r < 4; ++r) h[r] = fast_tanh(acc[T][r] + bb[r]);
        h = round4(h, BF);
        if (valid) st_act(H, (act_step(g, n) * g.L + (l - 1)) * hM + (size_t)p * g.wp + 16 * T + 4 * grp, h, BF);
      }
    }
    foff += 256ULL * TW * TW;
  }
  if (g.recomp) return;  // the activations were all that was asked for
  // output layer: Z = W_o h_L + b_o, then the c_n / v_n epilogue
  ls_stage<BF>(wsm, F + foff * esz, 256ULL * TI * TW * esz);
  const float* bo = bp + (size_t)g.L * 16 * TW;
  for (int it = 0; it < tpw; ++it) {
    const int tile = tr.t0 + it * nwv + wv;
    if (tile >= tr.t1) break;
    const int p = tile * 16 + col;
    const bool valid = p < g.M;
    f32x4 hin[TW], Z[TI];
#pragma unroll
    for (int T = 0; T < TW; ++T)
      hin[T] = valid ? ld_act(H, (act_step(g, n) * g.L + (g.L - 1)) * hM + (size_t)p * g.wp + 16 * T + 4 * grp, BF)
                     : zero4();
    layer_mm<BF, TI, TW>(Z, hin, wsm, lane);
#pragma unroll
    for (int t = 0; t < TI; ++t) Z[t] += ld4(bo + 16 * t + 4 * grp);
    epilogue(p, valid, Z);
  }
}

// -------------------------------------------------------------- scan kernel
__device__ __forceinline__ float phi_y(const Geo& g, float y) {
  switch (g.drv) {
    case DRV_BSB: return g.drv_p0 * y;
    case DRV_HJB: return 0.f;
    case DRV_AC: return y * y * y - y;
    default: return g.drv_p0 * y + g.drv_p1;
  }
}
__device__ __forceinline__ float phi_yy(const Geo& g, float y) {
  switch (g.drv) {
    case DRV_BSB: return g.drv_p0;
    case DRV_HJB: return 0.f;
    case DRV_AC: return 3.f * y * y - 1.f;
    default: return g.drv_p0;
  }
}
__device__ __forceinline__ float terminal_g(const Geo& g, float q, float lin) {
  switch (g.g) {
    case G_NORM2: return q;
    case G_LOGHALF: return logf(0.5f * (1.f + q));
    case G_INV: return 1.f / (g.g_p0 + g.g_p1 * q);
    default: return g.g_p0 * lin + g.g_p1;
  }
}

// fixed-order fp64 block sum of 256 values (result valid in thread 0)
__device__ __forceinline__ double block_sum_256(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  return sh[0];
}

// fixed-order fp64 sum over one wave (xor butterfly; every lane gets the
// same total, since each pairwise add sees the same two operands)
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// One wave per workgroup: the paths' serial recursions leave the SIMDs idle,
// so spreading the waves over as many CUs as possible shortens the latency
// chain each CU's memory pipeline serves.  NR > 0: time grids of at most NR
// steps keep c_n and Y_n in registers (NR is the smallest of 16, 32, 64 that
// holds N: the unrolled loops and loads stop there, 13 -> 10 us at N = 32);
// NR = 0: longer grids stream them.
template <int NR>
__global__ __launch_bounds__(64) void k_scan(Geo g, const double* __restrict__ y0,
                                             const float* __restrict__ C, const float* __restrict__ QN,
                                             const float* __restrict__ LN, float* __restrict__ Y,
                                             float* __restrict__ LAM, double* __restrict__ part) {
  const int m = blockIdx.x * 64 + threadIdx.x;
  double l2 = 0.0, lam0 = 0.0;
  if constexpr (NR > 0) {
    if (m < g.M) {
      // every c_n load is issued up front (indices clamped, so unconditional),
      // Y_n stays in registers for the reverse recursion: two memory latencies
      // per path instead of one per batch of steps in each direction
      float cv[NR], yv[NR + 1];
      const float qn = QN[m], ln = LN[m];  // terminal inputs, fetched with the c_n
#pragma unroll
      for (int n = 0; n < NR; ++n) cv[n] = C[(size_t)min(n, g.N - 1) * g.M + m];
      float y = (float)y0[0];
      yv[0] = y;
      Y[m] = y;
#pragma unroll
      for (int n = 0; n < NR; ++n) {
        if (n < g.N) {
          y = y + g.dt * phi_y(g, y) + cv[n];
          yv[n + 1] = y;
          Y[(size_t)(n + 1) * g.M + m] = y;
        }
      }
      const float e = y - terminal_g(g, qn, ln);
      l2 = (double)e * (double)e;
      float lam = 2.f * e / (float)g.M;
#pragma unroll
      for (int n = NR - 1; n >= 0; --n) {
        if (n < g.N) {
          LAM[(size_t)n * g.M + m] = lam;
          lam = lam * (1.f + g.dt * phi_yy(g, yv[n]));
        }
      }
      lam0 = (double)lam;
    }
  } else if (m < g.M) {
    // both recursions are serial in n; the loads they need are not, so
    // they are issued SB steps at a time ahead of the arithmetic
    constexpr int SB = 8;
    float y = (float)y0[0];
    Y[m] = y;
    for (int n0 = 0; n0 < g.N; n0 += SB) {
      float c[SB];
#pragma unroll
      for (int q = 0; q < SB; ++q) c[q] = (n0 + q < g.N) ? C[(size_t)(n0 + q) * g.M + m] : 0.f;
#pragma unroll
      for (int q = 0; q < SB; ++q) {
        if (n0 + q >= g.N) break;
        y = y + g.dt * phi_y(g, y) + c[q];
        Y[(size_t)(n0 + q + 1) * g.M + m] = y;
      }
    }
    const float e = y - terminal_g(g, QN[m], LN[m]);
    l2 = (double)e * (double)e;
    float lam = 2.f * e / (float)g.M;
    for (int n1 = g.N - 1; n1 >= 0; n1 -= SB) {
      float yv[SB];
#pragma unroll
      for (int q = 0; q < SB; ++q) yv[q] = (n1 - q >= 0) ? Y[(size_t)(n1 - q) * g.M + m] : 0.f;
#pragma unroll
      for (int q = 0; q < SB; ++q) {
        if (n1 - q < 0) break;
        LAM[(size_t)(n1 - q) * g.M + m] = lam;
        lam = lam * (1.f + g.dt * phi_yy(g, yv[q]));
      }
    }
    lam0 = (double)lam;
  }
  const double a = wave_sum(l2);
  const double b = wave_sum(lam0);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = a;
    part[2 * blockIdx.x + 1] = b;
  }
}

// ---------------------------------------------------------- backward kernel
// Waves per workgroup of the LDS-staged reverse sweep: one workgroup per CU
// (the step's weights fill the LDS), so the wave count sets the waves per
// SIMD: 3 for shapes up to 8 x 8 tiles (<= 170 VGPRs), else 2.
constexpr int bwd_waves(int ti, int tw) { return (ti <= 8 && tw <= 8) ? 12 : 8; }

template <bool BF, int TI, int TW, bool LDSW>
__global__ __launch_bounds__(LDSW ? 64 * bwd_waves(TI, TW) : 256) void k_backward(Geo g, const void* __restrict__ packB,
                                                                const float* __restrict__ V,
                                                                const float* __restrict__ LAM,
                                                                const void* __restrict__ H,
                                                                void* __restrict__ DZ, void* __restrict__ DH,
                                                                int tpw) {
  extern __shared__ __attribute__((aligned(16))) unsigned char wsm[];
  const int n = g.n0 + (int)blockIdx.y;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nwv = blockDim.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const size_t rowM = (size_t)g.M * g.dp;
  const size_t esz = BF ? 2 : 4;
  const char* pk;
  if constexpr (LDSW) {
    if (n > 0)
      stage_weights(wsm, reinterpret_cast<const char*>(packB) + (size_t)(n - 1) * g.packb_step * esz,
                    (size_t)g.packb_step * esz);
    pk = reinterpret_cast<const char*>(wsm);
  } else {
    pk = reinterpret_cast<const char*>(packB) + (size_t)(n > 0 ? n - 1 : 0) * g.packb_step * esz;
  }
  const float* Vn = V + n * rowM;
  const size_t hM = (size_t)g.M * g.wp;
  // v_n rows and lambda_{n+1} of the next tile are fetched one tile ahead.
  // With PF the tanh activations each epilogue needs are fetched one epilogue
  // ahead too, issued after the current epilogue's arithmetic and before its
  // stores: loads and stores retire in issue order, so waiting for them then
  // does not wait for the stores' completion; the last epilogue fetches the
  // next tile's first. Where the extra live registers would spill (fp32 8 x 8
  // tiles and the variant that reads its weights from global memory, !XT)
  // each layer's activations are fetched just before its product.
  constexpr bool PF = TI <= 8 && TW <= 8;
  constexpr bool XT = PF && LDSW && (BF || TI + TW < 16);
  f32x4 vnx[TI], hv[TW];
  float lnx = 0.f;
  const TileRange tr = tile_range(g.M);
  auto load_h = [&](int pp, bool ok, int li) {
#pragma unroll
    for (int T = 0; T < TW; ++T) {
      const size_t idx = (act_step(g, n) * g.L + li) * hM + (size_t)pp * g.wp + 16 * T + 4 * grp;
      hv[T] = ok ? ld_act(H, idx, BF) : zero4();
    }
  };
  if constexpr (PF) {
    const int p0 = (tr.t0 + wv) * 16 + col;
    const bool ok = tr.t0 + wv < tr.t1 && p0 < g.M;
    lnx = ok ? LAM[(size_t)n * g.M + p0] : 0.f;
#pragma unroll
    for (int t = 0; t < TI; ++t) {
      const int c0 = 16 * t + 4 * grp;
      vnx[t] = (ok && c0 < g.dp) ? ld4(Vn + (size_t)p0 * g.dp + c0) : zero4();
    }
    if (XT && n > 0) load_h(p0, ok, g.L - 1);
  }
  for (int it = 0; it < tpw; ++it) {
  const int tile = tr.t0 + it * nwv + wv;
  if (tile >= tr.t1) break;
  const int p = tile * 16 + col;
  const bool valid = p < g.M;
  const float lam = PF ? lnx : (valid ? LAM[(size_t)n * g.M + p] : 0.f);
  const int pn = p + 16 * nwv;
  const bool nxt = it + 1 < tpw && tile + nwv < tr.t1 && pn < g.M;
  f32x4 zeta[TI];
  if constexpr (!PF) {
#pragma unroll
    for (int t = 0; t < TI; ++t) {
      const int c0 = 16 * t + 4 * grp;
      vnx[t] = (valid && c0 < g.dp) ? ld4(Vn + (size_t)p * g.dp + c0) : zero4();
    }
  }
#pragma unroll
  for (int t = 0; t < TI; ++t) zeta[t] = round4(lam * vnx[t], BF);
  if constexpr (PF) {
    lnx = nxt ? LAM[(size_t)n * g.M + pn] : 0.f;
#pragma unroll
    for (int t = 0; t < TI; ++t) {
      const int c0 = 16 * t + 4 * grp;
      vnx[t] = (nxt && c0 < g.dp) ? ld4(Vn + (size_t)pn * g.dp + c0) : zero4();
    }
  }
#pragma unroll
  for (int t = 0; t < TI; ++t)
    if (valid) st_act(DZ, (act_step(g, n) * g.M + p) * g.zp + 16 * t + 4 * grp, zeta[t], BF);
  if (n == 0) continue;
  f32x4 dl[TW], acc[TW];
  // delta_l = (acc) * (1 - h^2) for layer l, then the next epilogue's loads,
  // then the stores of delta_l
  auto epilogue = [&](int l) {
    if constexpr (!PF) load_h(p, valid, l - 1);
#pragma unroll
    for (int T = 0; T < TW; ++T) {
#pragma unroll
      for (int r = 0; r < 4; ++r) dl[T][r] = acc[T][r] * (1.f - hv[T][r] * hv[T][r]);
      dl[T] = round4(dl[T], BF);
    }
    if constexpr (XT) {
      if (l > 1) load_h(p, valid, l - 2);
      else load_h(pn, nxt, g.L - 1);
    }
#pragma unroll
    for (int T = 0; T < TW; ++T) {
      const size_t idx = (act_step(g, n) * g.L + (l - 1)) * hM + (size_t)p * g.wp + 16 * T + 4 * grp;
      if (valid) st_act(DH, idx, dl[T], BF);
    }
  };
  if constexpr (PF && !XT) load_h(p, valid, g.L - 1);
  layer_mm<BF, TW, TI>(acc, zeta, pk, lane);
  epilogue(g.L);
  const char* pkl = pk + 256ULL * TW * TI * esz;
  for (int l = g.L - 1; l >= 1; --l) {
    if constexpr (PF && !XT) load_h(p, valid, l - 1);
    layer_mm<BF, TW, TW>(acc, dl, pkl + (size_t)(l - 1) * 256ULL * TW * TW * esz, lane);
    epilogue(l);
  }
  }
}

// ----------------------------------------------- layer-streamed reverse sweep
// The reverse sweep for step networks whose transposed weights do not fit
// LDS at once: one layer's fragments at a time, run over all of the
// workgroup's tiles; delta_{l+1} comes back from DH (which the weight
// gradient reads anyway).  Products, rounding and epilogues are those of
// k_backward, so both give bitwise equal results.
template <bool BF, int TI, int TW>
__global__ __launch_bounds__(64 * LS_WAVES) void k_backward_ls(Geo g, const void* __restrict__ packB,
                                                               const float* __restrict__ V,
                                                               const float* __restrict__ LAM,
                                                               const void* __restrict__ H, void* __restrict__ DZ,
                                                               void* __restrict__ DH, int tpw) {
  extern __shared__ __attribute__((aligned(16))) unsigned char wsm[];
  const int n = g.n0 + (int)blockIdx.y;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nwv = LS_WAVES;
  const int col = lane & 15, grp = lane >> 4;
  const size_t rowM = (size_t)g.M * g.dp, hM = (size_t)g.M * g.wp;
  const size_t esz = BF ? 2 : 4;
  const float* Vn = V + n * rowM;
  const TileRange tr = tile_range(g.M);
  const char* Bk = reinterpret_cast<const char*>(packB) + (size_t)(n > 0 ? n - 1 : 0) * g.packb_step * esz;
  // layer L: zeta = lambda_{n+1} v_n (stored in DZ), delta_L = (W_o^T zeta) (1 - h_L^2)
  if (n > 0) ls_stage<BF>(wsm, Bk, 256ULL * TW * TI * esz);
  for (int it = 0; it < tpw; ++it) {
    const int tile = tr.t0 + it * nwv + wv;
    if (tile >= tr.t1) break;
    const int p = tile * 16 + col;
    const bool valid = p < g.M;
    const float lam = valid ? LAM[(size_t)n * g.M + p] : 0.f;
    f32x4 zeta[TI];
#pragma unroll
    for (int t = 0; t < TI; ++t) {
      const int c0 = 16 * t + 4 * grp;
      const f32x4 v = (valid && c0 < g.dp) ? ld4(Vn + (size_t)p * g.dp + c0) : zero4();
      zeta[t] = round4(lam * v, BF);
      if (valid) st_act(DZ, (act_step(g, n) * g.M + p) * g.zp + 16 * t + 4 * grp, zeta[t], BF);
    }
    if (n == 0) continue;
    f32x4 acc[TW];
    layer_mm<BF, TW, TI>(acc, zeta, wsm, lane);
#pragma unroll
    for (int T = 0; T < TW; ++T) {
      const size_t idx = (act_step(g, n) * g.L + (g.L - 1)) * hM + (size_t)p * g.wp + 16 * T + 4 * grp;
      const f32x4 h = valid ? ld_act(H, idx, BF) : zero4();
      f32x4 dl;
#pragma unroll
      for (int r = 0; r < 4; ++r) dl[r] = acc[T][r] * (1.f - h[r] * h[r]);
      dl = round4(dl, BF);
      if (valid) st_act(DH, idx, dl, BF);
    }
  }
  if (n == 0) return;
  // delta_l = (W_{l+1}^T delta_{l+1}) (1 - h_l^2), l = L-1..1
  for (int l = g.L - 1; l >= 1; --l) {
    ls_stage<BF>(wsm, Bk + (256ULL * TW * TI + (size_t)(l - 1) * 256ULL * TW * TW) * esz, 256ULL * TW * TW * esz);
    for (int it = 0; it < tpw; ++it) {
      const int tile = tr.t0 + it * nwv + wv;
      if (tile >= tr.t1) break;
      const int p = tile * 16 + col;
      const bool valid = p < g.M;
      f32x4 din[TW], acc[TW];
#pragma unroll
      for (int T = 0; T < TW; ++T)
        din[T] = valid ? ld_act(DH, (act_step(g, n) * g.L + l) * hM + (size_t)p * g.wp + 16 * T + 4 * grp, BF) : zero4();
      layer_mm<BF, TW, TW>(acc, din, wsm, lane);
#pragma unroll
      for (int T = 0; T < TW; ++T) {
        const size_t idx = (act_step(g, n) * g.L + (l - 1)) * hM + (size_t)p * g.wp + 16 * T + 4 * grp;
        const f32x4 h = valid ? ld_act(H, idx, BF) : zero4();
        f32x4 dl;
#pragma unroll
        for (int r = 0; r < 4; ++r) dl[r] = acc[T][r] * (1.f - h[r] * h[r]);
        dl = round4(dl, BF);
        if (valid) st_act(DH, idx, dl, BF);
      }
    }
  }
}

// ------------------------------------------------------------- wgrad kernel
// Job 0: dz0 = sum_m zeta_0 (a d x 0 "matrix" with only its bias column).
// Job 1 + (n-1)(L+1) + (l-1), l = 1..L+1: dW_l of step n (bias as column cols).
// A launch over steps n0 .. n0 + ns - 1 numbers its jobs the same way from
// its first step (job 0 is step 0's only when n0 = 0).
struct Job {
  int rows, cols;
  long long base;          // flat offset of W_l (b_l follows at base + rows*cols)
  const void* A; int sA;   // deltas, row stride (per path)
  const void* B; int sB;   // activations (nullptr: none)
  bool Bf32;               // B is fp32 path state (X) rather than an activation
};

__device__ __forceinline__ Job job_info(const Geo& g, int job, const float* X, const void* H,
                                        const void* DZ, const void* DH) {
  Job J;
  const size_t esz = g.bf16 ? 2 : 4;
  if (g.n0 == 0 && job == 0) {
    J.rows = g.d; J.cols = 0; J.base = 0;
    J.A = DZ; J.sA = g.zp; J.B = nullptr; J.sB = 0; J.Bf32 = false;
    return J;
  }
  // jobs of the launch's steps with a network, from max(n0, 1)
  const int jj = job - (g.n0 == 0 ? 1 : 0);
  const int n = (g.n0 > 1 ? g.n0 : 1) + jj / (g.L + 1), l = 1 + jj % (g.L + 1);
  const size_t hM = (size_t)g.M * g.wp;
  const long long step = g.d + (long long)(n - 1) * g.pstep;
  const long long lw1 = (long long)g.w * g.d + g.w, lwh = (long long)g.w * g.w + g.w;
  J.rows = (l == g.L + 1) ? g.d : g.w;
  J.cols = (l == 1) ? g.d : g.w;
  J.base = step + (l == 1 ? 0 : lw1 + (long long)(l - 2) * lwh);
  if (l == g.L + 1) {
    J.A = reinterpret_cast<const char*>(DZ) + act_step(g, n) * g.M * g.zp * esz; J.sA = g.zp;
  } else {
    J.A = reinterpret_cast<const char*>(DH) + (act_step(g, n) * g.L + (l - 1)) * hM * esz; J.sA = g.wp;
  }
  if (l == 1) {
    J.B = X + (size_t)n * g.M * g.dp; J.sB = g.dp; J.Bf32 = true;
  } else {
    J.B = reinterpret_cast<const char*>(H) + (act_step(g, n) * g.L + (l - 2)) * hM * esz; J.sB = g.wp;
    J.Bf32 = false;
  }
  return J;
}

// LDS-staged weight-gradient GEMM.  Workgroup = (job, output block group,
// path split); it owns a T x T block of 16x16 output tiles and walks its path
// range in chunks staged in LDS.  Wave w accumulates tile column w over all T
// tile rows (with T < 8 the waves past T only stage), except for T = 7, where
// waves 0..6 take tile rows 0..5 of their column and wave 7 takes tile row 6
// of every column (see k_wgrad).  Bias gradients ride along as an extra input
// column of ones (column `cols`).
//
// Chunk length: the bf16 MFMA takes K = 32 paths per instruction, so the bf16
// form stages 32 paths (transposed to k-contiguous rows); the fp32 form
// (K = 4 per MFMA) stages 16, which halves its staging registers and keeps
// more chunks in flight per CU.
#ifndef FBSDE_WG_KC_F32
#define FBSDE_WG_KC_F32 16
#endif
template <bool BF>
constexpr int wg_kc() { return BF ? 32 : FBSDE_WG_KC_F32; }
// The fp32 form loads the next chunk into registers while the MFMAs run on
// the current one.  The bf16 form is bound by the HBM reads and the 2-byte
// transposing LDS writes; prefetching there costs registers (two workgroups
// per CU instead of three) and was slower, so it loads just before staging.
template <bool BF>
constexpr bool wg_prefetch() { return !BF; }
// tile columns per wave of the weight-gradient kernel (its workgroup has
// ceil(T / WG_CPW) <= 8 waves: 4 waves x 2 columns or 8 waves x 1 column)
#ifndef FBSDE_WG_CPW
#define FBSDE_WG_CPW 1
#endif
constexpr int WG_CPW = FBSDE_WG_CPW;
constexpr int WG_THREADS = 64 * (8 / WG_CPW);

template <bool BF, int T>
struct WgradLds {
  static constexpr int KC = wg_kc<BF>();
  static constexpr int LDA = 16 * T + ((T % 2 == 0) ? 16 : 0);  // fp32 row stride (floats), == 16 mod 32
  static constexpr int LDB = 128;                                // bf16 [path][feature] row (T <= 8 tiles)
  static constexpr size_t BYTES = BF ? 2ull * KC * LDB * 2 : 2ull * KC * LDA * 4;
  static_assert(!BF || T <= 8, "bf16 rows hold at most 8 tiles");
};

// bf16 staging keeps each path's features as one LDS row; the MFMA fragment
// (8 consecutive paths of one feature per lane) comes from two transposed
// reads (ds_read_b64_tr_b16): in each 16-lane group, lanes 4e..4e+3 point at
// row 8g + 4h + e, columns 4q..4q+3 of the tile (q = lane % 4), and lane j
// receives column j of those four rows.  The 16-feature blocks of row k are
// XOR-swizzled by (k mod 4) + 4 (floor(k / 8) mod 2), which rows k and k + 4
// share, so the 8 rows one read instruction touches per 32 lanes fall into
// distinct banks.
__device__ __forceinline__ int wg_swz(int k) { return ((k & 3) | (((k >> 3) & 1) << 2)) * 16; }
typedef short wg_v4s __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) wg_v4s wg_lds_v4s;
__device__ __forceinline__ bf16x8 wg_frag(const uint16_t* rows, int col0, int lane) {
  const int g = lane >> 4, j = lane & 15, k = 8 * g + (j >> 2);
  uint16_t* p = const_cast<uint16_t*>(rows) + k * 128 + (col0 ^ wg_swz(k)) + 4 * (j & 3);
  const wg_v4s lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((wg_lds_v4s*)p);
  const wg_v4s hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((wg_lds_v4s*)(p + 4 * 128));
  const uint2 l = __builtin_bit_cast(uint2, lo), h = __builtin_bit_cast(uint2, hi);
  return __builtin_bit_cast(bf16x8, u32x4{l.x, l.y, h.x, h.y});
}

// 4 consecutive fp32 input columns c..c+3 of one path, with the bias column
// of ones at `cols` and zeros beyond (src row holds `stride` valid entries)
__device__ __forceinline__ f32x4 load_cols4(const float* base, size_t rowoff, int c, int cols, int stride) {
  f32x4 v = zero4();
  if (c < stride) v = ld4(base + rowoff + c);
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    if (c + e == cols) v[e] = 1.f;
    else if (c + e > cols) v[e] = 0.f;
  }
  return v;
}

// Staging of one chunk: KC paths of the deltas (A, rows R0..R0+16T) and
// of the layer inputs (B, columns C0..C0+16T, bias column of ones), as
// 4-element slots; slot s < NV is A, the rest B.  Each thread owns NS slots,
// held as fp32 (f32x4) or, in the bf16 form, as packed bf16 bits (uint2).
template <bool BF, int T>
struct WgradStage {
  static constexpr int NV = wg_kc<BF>() * 4 * T;
  static constexpr int NS = (2 * NV + WG_THREADS - 1) / WG_THREADS;
};
template <bool BF> struct StageSlot { using type = f32x4; };
template <> struct StageSlot<true> { using type = uint2; };

// bf16 bits of 4 consecutive input columns c..c+3 of one path (bias column of
// ones at `cols`, zeros beyond), from bf16 activations or the fp32 state X
__device__ __forceinline__ uint2 load_cols4_bf(const void* base, bool f32src, size_t rowoff, int c, int cols,
                                               int stride) {
  uint32_t e[4] = {0u, 0u, 0u, 0u};
  if (c < stride) {
    if (f32src) {
      const f32x4 v = ld4(reinterpret_cast<const float*>(base) + rowoff + c);
#pragma unroll
      for (int i = 0; i < 4; ++i) e[i] = bf16_bits(v[i]);
    } else {
      const uint2 u = *reinterpret_cast<const uint2*>(reinterpret_cast<const uint16_t*>(base) + rowoff + c);
      e[0] = u.x & 0xffffu; e[1] = u.x >> 16; e[2] = u.y & 0xffffu; e[3] = u.y >> 16;
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (c + i == cols) e[i] = 0x3f80u;  // 1.0
    else if (c + i > cols) e[i] = 0u;
  }
  return uint2{e[0] | (e[1] << 16), e[2] | (e[3] << 16)};
}

template <bool BF, int T>
__device__ __forceinline__ void wgrad_fetch(const Job& J, int R0, int C0, long long pc, long long p1, int tid,
                                            typename StageSlot<BF>::type (&v)[WgradStage<BF, T>::NS]) {
  constexpr int NV = WgradStage<BF, T>::NV;
#pragma unroll
  for (int k = 0; k < WgradStage<BF, T>::NS; ++k) {
    const int s = tid + k * WG_THREADS;
    if constexpr (BF) v[k] = uint2{0u, 0u};
    else v[k] = zero4();
    if (s >= 2 * NV) continue;
    const bool isA = s < NV;
    const int q = isA ? s : s - NV;
    const int kp = q / (4 * T), c4 = q % (4 * T);
    const long long p = pc + kp;
    if (p >= p1) continue;
    if (isA) {
      const int r = R0 + 4 * c4;
      if (r >= J.rows) continue;
      if constexpr (BF) v[k] = *reinterpret_cast<const uint2*>(reinterpret_cast<const uint16_t*>(J.A) + (size_t)p * J.sA + r);
      else v[k] = ld4(reinterpret_cast<const float*>(J.A) + (size_t)p * J.sA + r);
    } else {
      // deltas and activations are stored in the GEMM precision; X is fp32 state
      if constexpr (BF) v[k] = load_cols4_bf(J.B, J.Bf32, (size_t)p * J.sB, C0 + 4 * c4, J.cols, J.B ? J.sB : 0);
      else v[k] = load_cols4(reinterpret_cast<const float*>(J.B), (size_t)p * J.sB, C0 + 4 * c4, J.cols, J.B ? J.sB : 0);
    }
  }
}

template <bool BF, int T>
__device__ __forceinline__ void wgrad_put(unsigned char* smem, int tid,
                                          const typename StageSlot<BF>::type (&v)[WgradStage<BF, T>::NS]) {
  using L = WgradLds<BF, T>;
  constexpr int NV = WgradStage<BF, T>::NV;
#pragma unroll
  for (int k = 0; k < WgradStage<BF, T>::NS; ++k) {
    const int s = tid + k * WG_THREADS;
    if (s >= 2 * NV) continue;
    const bool isA = s < NV;
    const int q = isA ? s : s - NV;
    const int kp = q / (4 * T), c4 = q % (4 * T);
    if constexpr (!BF) {
      float* dst = reinterpret_cast<float*>(smem) + (isA ? 0 : L::KC * L::LDA) + kp * L::LDA + 4 * c4;
      st4(dst, v[k]);
    } else {
      // features 4 c4 .. 4 c4 + 3 of path kp, one 8-byte write into its row
      uint16_t* dst = reinterpret_cast<uint16_t*>(smem) + (isA ? 0 : L::KC * L::LDB) + kp * L::LDB +
                      ((16 * (c4 >> 2)) ^ wg_swz(kp)) + 4 * (c4 & 3);
      *reinterpret_cast<uint2*>(dst) = v[k];
    }
  }
}

// fp32 staging with the loads in flight across the MFMAs: the loads are
// unconditional (rows and columns clamped into their buffers, a missing
// input read from the delta buffer) and their values are consumed only when
// wgrad_put_f32 writes them to LDS, which applies the path range, the row
// extent, the bias column and the zero padding (the semantics of
// wgrad_fetch).
template <int T>
__device__ __forceinline__ void wgrad_fetch_raw(const Job& J, int R0, int C0, long long pc, long long p1, int tid,
                                                f32x4 (&v)[WgradStage<false, T>::NS]) {
  constexpr int NV = WgradStage<false, T>::NV;
#pragma unroll
  for (int k = 0; k < WgradStage<false, T>::NS; ++k) {
    const int s = min(tid + k * WG_THREADS, 2 * NV - 1);
    const bool isA = s < NV;
    const int q = isA ? s : s - NV;
    const int kp = q / (4 * T), c4 = q % (4 * T);
    const size_t p = (size_t)min(pc + kp, p1 - 1);
    const float* src;
    if (isA || J.B == nullptr) {
      src = reinterpret_cast<const float*>(J.A) + p * J.sA + min(R0 + 4 * c4, J.sA - 4);
    } else {
      src = reinterpret_cast<const float*>(J.B) + p * J.sB + min(C0 + 4 * c4, J.sB - 4);
    }
    v[k] = ld4(src);
  }
}

template <int T>
__device__ __forceinline__ void wgrad_put_f32(const Job& J, int R0, int C0, long long pc, long long p1,
                                              unsigned char* smem, int tid,
                                              const f32x4 (&v)[WgradStage<false, T>::NS]) {
  using L = WgradLds<false, T>;
  constexpr int NV = WgradStage<false, T>::NV;
#pragma unroll
  for (int k = 0; k < WgradStage<false, T>::NS; ++k) {
    const int s = tid + k * WG_THREADS;
    if (s >= 2 * NV) continue;
    const bool isA = s < NV;
    const int q = isA ? s : s - NV;
    const int kp = q / (4 * T), c4 = q % (4 * T);
    const bool ok = pc + kp < p1;
    f32x4 x = zero4();
    if (isA) {
      if (ok && R0 + 4 * c4 < J.rows) x = v[k];
    } else if (ok) {
      const int c = C0 + 4 * c4, stride = J.B ? J.sB : 0;
      if (c < stride) x = v[k];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (c + e == J.cols) x[e] = 1.f;
        else if (c + e > J.cols) x[e] = 0.f;
      }
    }
    float* dst = reinterpret_cast<float*>(smem) + (isA ? 0 : L::KC * L::LDA) + kp * L::LDA + 4 * c4;
    st4(dst, x);
  }
}

// One wave's share of the T x T tile block: NR tile rows from rt0 times NC
// tile columns from ct0 (NR = NC = 0: the wave only stages).
template <bool BF, int T, int NR, int NC>
__device__ __forceinline__ void wgrad_tiles(const Geo& g, const Job& J, int R0, int C0, long long p0,
                                            long long p1, unsigned char* smem, float* out_split, int rt0,
                                            int ct0) {
  using L = WgradLds<BF, T>;
  const int tid = threadIdx.x, lane = tid & 63;
  const int c16 = lane & 15, grp = lane >> 4;
  constexpr bool MM = NR > 0 && NC > 0;
  constexpr int NRA = NR > 0 ? NR : 1, NCA = NC > 0 ? NC : 1;  // storage sizes
  f32x4 acc[NRA][NCA];
#pragma unroll
  for (int i = 0; i < NRA; ++i)
#pragma unroll
    for (int j = 0; j < NCA; ++j) acc[i][j] = zero4();

  typename StageSlot<BF>::type pre[WgradStage<BF, T>::NS];
  if constexpr (wg_prefetch<BF>()) wgrad_fetch_raw<T>(J, R0, C0, p0, p1, tid, pre);
  for (long long pc = p0; pc < p1; pc += L::KC) {
    __syncthreads();
    if constexpr (!wg_prefetch<BF>()) {
      wgrad_fetch<BF, T>(J, R0, C0, pc, p1, tid, pre);
      wgrad_put<BF, T>(smem, tid, pre);
    } else {
      wgrad_put_f32<T>(J, R0, C0, pc, p1, smem, tid, pre);
    }
    __syncthreads();
    // the next chunk's loads are in flight during this chunk's MFMAs
    if constexpr (wg_prefetch<BF>())
      if (pc + L::KC < p1) wgrad_fetch_raw<T>(J, R0, C0, pc + L::KC, p1, tid, pre);
    if constexpr (!MM) continue;
    // ---- MFMA over the chunk
    if constexpr (!BF) {
      const float* As = reinterpret_cast<const float*>(smem) + 16 * rt0 + c16;
      const float* Bs = reinterpret_cast<const float*>(smem) + L::KC * L::LDA + 16 * ct0 + c16;
#pragma unroll
      for (int kb = 0; kb < L::KC / 4; ++kb) {
        const int kr = 4 * kb + grp;
        float a[NRA], b[NCA];
#pragma unroll
        for (int i = 0; i < NR; ++i) a[i] = As[kr * L::LDA + 16 * i];
#pragma unroll
        for (int j = 0; j < NC; ++j) b[j] = Bs[kr * L::LDA + 16 * j];
#pragma unroll
        for (int i = 0; i < NR; ++i)
#pragma unroll
          for (int j = 0; j < NC; ++j) acc[i][j] = mfma_f32(a[i], b[j], acc[i][j]);
      }
    } else {
      const uint16_t* As = reinterpret_cast<const uint16_t*>(smem);
      const uint16_t* Bs = As + L::KC * L::LDB;
      bf16x8 a[NRA], b[NCA];
#pragma unroll
      for (int i = 0; i < NR; ++i) a[i] = wg_frag(As, 16 * (rt0 + i), lane);
#pragma unroll
      for (int j = 0; j < NC; ++j) b[j] = wg_frag(Bs, 16 * (ct0 + j), lane);
#pragma unroll
      for (int i = 0; i < NR; ++i)
#pragma unroll
        for (int j = 0; j < NC; ++j) acc[i][j] = mfma_bf16(a[i], b[j], acc[i][j]);
    }
  }
  // ---- partial sums of this path split, scattered to the flat layout
#pragma unroll
  for (int i = 0; i < NR; ++i)
#pragma unroll
    for (int j = 0; j < NC; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = R0 + 16 * (rt0 + i) + 4 * grp + r, c = C0 + 16 * (ct0 + j) + c16;
        if (row < J.rows && c <= J.cols) {
          const long long off = (c < J.cols) ? J.base + (long long)row * J.cols + c
                                             : J.base + (long long)J.rows * J.cols + row;
          out_split[off] = acc[i][j][r];
        }
      }
}

template <bool BF, int T>
__global__ __launch_bounds__(WG_THREADS) __attribute__((amdgpu_waves_per_eu(BF ? 6 : 1))) void k_wgrad(
    Geo g, const float* __restrict__ X, const void* __restrict__ H,
                                               const void* __restrict__ DZ, const void* __restrict__ DH,
                                               float* __restrict__ part, long long chunk) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[WgradLds<BF, T>::BYTES];
  const Job J = job_info(g, blockIdx.x, X, H, DZ, DH);
  const int ngc = (J.cols + 1 + 16 * T - 1) / (16 * T), ngr = (J.rows + 16 * T - 1) / (16 * T);
  if ((int)blockIdx.y >= ngc * ngr) return;  // uniform over the workgroup
  const int R0 = (blockIdx.y / ngc) * 16 * T, C0 = (blockIdx.y % ngc) * 16 * T;
  const long long p0 = (long long)blockIdx.z * chunk;
  const long long p1 = min((long long)g.M, p0 + chunk);
  float* out = part + (size_t)blockIdx.z * g.pstride;
  const int wv = threadIdx.x >> 6;
  if constexpr (WG_CPW == 1 && T == 7) {
    // 7 x 7 tiles over 8 waves: waves 0..6 take tile rows 0..5 of column wv,
    // wave 7 takes tile row 6 of every column, so every wave multiplies (6
    // or 7 tiles) and each SIMD's pair of waves carries 12 or 13 tiles
    if (wv < T) wgrad_tiles<BF, T, T - 1, 1>(g, J, R0, C0, p0, p1, smem, out, 0, wv);
    else wgrad_tiles<BF, T, 1, T>(g, J, R0, C0, p0, p1, smem, out, T - 1, 0);
  } else {
    // tile columns of this wave inside the block: WG_CPW per wave (fewer at the edge)
    const int ncol = min(WG_CPW, max(0, T - WG_CPW * wv));
    if (WG_CPW == 2 && ncol == 2) wgrad_tiles<BF, T, T, WG_CPW>(g, J, R0, C0, p0, p1, smem, out, 0, WG_CPW * wv);
    else if (ncol == 1) wgrad_tiles<BF, T, T, 1>(g, J, R0, C0, p0, p1, smem, out, 0, WG_CPW * wv);
    else wgrad_tiles<BF, T, 0, 0>(g, J, R0, C0, p0, p1, smem, out, 0, 0);
  }
}

// ---------------------------------------------------- fused reverse kernel
// fp32 reverse sweep and weight gradient of one step in one kernel, so the
// deltas never leave the CU.  Workgroup = (path split, step n), 8 waves.  It
// stages step n's transposed weights (the backward fragments) in LDS once and
// walks the split's paths in rounds of 16.  A round stages [path][feature]
// rows of zeta = lambda_{n+1} v_n and of the layer inputs x, h_1..h_L (with
// the bias column of ones); waves 0..TW-1 then form delta_L, ..., delta_1, one
// 16-feature output tile each (D registers back to LDS rows), and every wave
// accumulates its share of the step's weight-gradient tiles in registers.
// Tile ownership follows k_wgrad: with 7 x 7 tile blocks, waves 0..6 take
// tile rows 0..5 of tile column wv and wave 7 takes tile row 6 of every
// column; with T <= 4 tiles, wave wv < T takes tile column wv.  Step 0 has no
// network: its workgroups sum zeta_0 (the z0 gradient).  Paths, 16-path
// chunks, the path-to-MFMA-slot assignment and the per-tile accumulation
// order are those of k_backward + k_wgrad with the same split count, so the
// two forms give bitwise equal gradients.
//
// Staged rows are 16-byte-group swizzled (rv_at): rows 0..7 (and 8..15) take
// distinct swizzles, so the 16-byte reads and writes of 8 lanes on 8
// consecutive rows hit 8 distinct bank groups; rows 2k and 2k + 1 differ in
// bit 2 of the swizzle, so the 4-byte operand reads of one column over rows
// 4k + {0, 1} (lanes 0..31) fall in disjoint bank halves.
constexpr int RV_WAVES = 8, RV_THREADS = 64 * RV_WAVES, RV_KC = 16;

__host__ __device__ constexpr int rv_lda(int ti, int tw) { return (16 * (ti > tw ? ti : tw) + 31) / 32 * 32; }
__host__ __device__ constexpr int rv_arrays(int L) { return 2 * L + 2; }
__host__ __device__ constexpr int NRA_(int nr) { return nr > 0 ? nr : 1; }
__host__ __device__ constexpr int NCA_(int nc) { return nc > 0 ? nc : 1; }

__device__ __forceinline__ int rv_swz(int row) { return ((row & 1) << 2) | ((row >> 1) & 3); }
template <int LDA>
__device__ __forceinline__ int rv_at(int row, int col) {
  return row * LDA + 4 * ((col >> 2) ^ rv_swz(row)) + (col & 3);
}

// Weight-gradient matrix m of step n: staged arrays 0 = zeta, l = delta_l
// (l = 1..L), L + 1 = x (step 0: a column of ones), L + 1 + l = h_l.
struct RvMat { int rows, cols, rt, ct, da, aa; long long base; };
__device__ __forceinline__ RvMat rv_mat(const Geo& g, int n, int m) {
  RvMat R;
  const int d = g.d, w = g.w, L = g.L;
  if (n == 0) {  // dz0 = sum over paths of zeta_0: rows d, bias column only
    R.rows = d; R.cols = 0; R.base = 0; R.da = 0; R.aa = L + 1;
  } else {
    const long long step = d + (long long)(n - 1) * g.pstep;
    const long long lw1 = (long long)w * d + w, lwh = (long long)w * w + w;
    if (m == 0) {  // W_1 += delta_1 x^T
      R.rows = w; R.cols = d; R.base = step; R.da = 1; R.aa = L + 1;
    } else if (m < L) {  // W_{m+1} += delta_{m+1} h_m^T
      R.rows = w; R.cols = w; R.base = step + lw1 + (long long)(m - 1) * lwh; R.da = m + 1; R.aa = L + 1 + m;
    } else {  // W_o += zeta h_L^T
      R.rows = d; R.cols = w; R.base = step + lw1 + (long long)(L - 1) * lwh; R.da = 0; R.aa = 2 * L + 1;
    }
  }
  R.rt = (R.rows + 15) / 16;
  R.ct = (R.cols + 16) / 16;  // + the bias column
  return R;
}

// The whole round loop for one wave role: NR tile rows from R0 times NC tile
// columns from C0 of every weight-gradient matrix (NR = NC = 0: no tiles).
// Tiles past a matrix's extent multiply zero-padded staged columns and are
// dropped at the scatter.
template <int TI, int TW, int L, int NR, int NC>
__device__ __forceinline__ void rv_body(const Geo& g, const void* __restrict__ packB, const float* __restrict__ X,
                                        const float* __restrict__ V, const float* __restrict__ LAM,
                                        const float* __restrict__ H, float* __restrict__ part, long long p0,
                                        long long p1, unsigned char* wsm, int R0, int C0) {
  constexpr int LDA = rv_lda(TI, TW), ASZ = RV_KC * LDA, NSL = L + 2;
  static_assert(RV_KC * 4 * (TI > TW ? TI : TW) <= RV_THREADS, "one staging item per thread and array");
  const int n = g.n0 + (int)blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int c16 = lane & 15, grp = lane >> 4;
  float* arr = reinterpret_cast<float*>(wsm + (size_t)g.packb_step * 4);
  const size_t rowM = (size_t)g.M * g.dp, hM = (size_t)g.M * g.wp;
  const int nmat = n == 0 ? 1 : L + 1;

  // ---- staging: slot a of every thread serves input a (0: v, scaled to
  // zeta; 1: x, or the column of ones at step 0; 1 + l: h_l); item tid is
  // (row p, columns c..c+3) of the round (c = -1: no item)
  int sp[NSL], sc[NSL], sofs[NSL];
#pragma unroll
  for (int a = 0; a < NSL; ++a) {
    const int gq = a == 0 ? g.dp / 4 : (a == 1 ? (n == 0 ? 1 : (g.d + 4) / 4) : (g.w + 4) / 4);
    const int p = tid / gq;
    sp[a] = p < RV_KC ? p : 0;
    sc[a] = p < RV_KC ? 4 * (tid - p * gq) : -1;
    sofs[a] = (a == 0 ? 0 : L + a) * ASZ + rv_at<LDA>(sp[a], sc[a] < 0 ? 0 : sc[a]);
  }
  const float* Vn = V + n * rowM;
  const float* Ln = LAM + (size_t)n * g.M;
  const float* Xn = X + n * rowM;
  // Raw loads only: every load is unconditional (row and column clamped into
  // the buffer), so a round's loads are all in flight while the previous
  // round computes; validity, the bias column and zero padding are applied
  // when the values are written to LDS.
  f32x4 sv[NSL];
#pragma unroll
  for (int a = 0; a < NSL; ++a) sv[a] = zero4();
  float sl = 0.f;
  auto fetch = [&](long long pc) {
#pragma unroll
    for (int a = 0; a < NSL; ++a) {
      const size_t p = (size_t)min(pc + sp[a], p1 - 1);
      if (a == 0) {
        sv[a] = ld4(Vn + p * g.dp + max(sc[a], 0));
        sl = Ln[p];
      } else if (a == 1) {
        if (n > 0) sv[a] = ld4(Xn + p * g.dp + min(max(sc[a], 0), g.dp - 4));
      } else {
        sv[a] = ld4(H + (act_step(g, n) * L + (a - 2)) * hM + p * g.wp + min(max(sc[a], 0), g.wp - 4));
      }
    }
  };
  // the staged value of slot a for round pc (the semantics of load_cols4)
  auto staged = [&](int a, long long pc) -> f32x4 {
    const bool ok = sc[a] >= 0 && pc + sp[a] < p1;
    const int c = sc[a];
    if (a == 0) return ok ? sl * sv[0] : zero4();
    const int cols = a == 1 ? (n == 0 ? 0 : g.d) : g.w;
    const int stride = a == 1 ? (n == 0 ? 0 : g.dp) : g.wp;
    f32x4 v = c < stride ? sv[a] : zero4();
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if (c + e == cols) v[e] = 1.f;
      else if (c + e > cols) v[e] = 0.f;
    }
    return ok ? v : zero4();
  };

  f32x4 acc[L + 1][NRA_(NR)][NCA_(NC)];
#pragma unroll
  for (int m = 0; m < L + 1; ++m)
#pragma unroll
    for (int i = 0; i < NRA_(NR); ++i)
#pragma unroll
      for (int j = 0; j < NCA_(NC); ++j) acc[m][i][j] = zero4();

  fetch(p0);
  if (n > 0) copy_to_lds(wsm, reinterpret_cast<const char*>(packB) + (size_t)(n - 1) * g.packb_step * 4,
                         (size_t)g.packb_step * 4);
  // columns no round writes stay zero
  for (int e = tid; e < rv_arrays(L) * ASZ / 4; e += RV_THREADS) st4(arr + 4 * e, zero4());
  const f32x4* W4 = reinterpret_cast<const f32x4*>(wsm);
  for (long long pc = p0; pc < p1; pc += RV_KC) {
    __syncthreads();  // weights and zero fill (first round), or the previous round's reads, are done
#pragma unroll
    for (int a = 0; a < NSL; ++a)
      if (sc[a] >= 0) st4(arr + sofs[a], staged(a, pc));
    __syncthreads();
    if (pc + RV_KC < p1) fetch(pc + RV_KC);  // in flight during this round's MFMAs
    if (n > 0) {
      // delta_L = (W_o^T zeta) (1 - h_L^2), then delta_l = (W_{l+1}^T delta_{l+1}) (1 - h_l^2)
#pragma unroll
      for (int l = L; l >= 1; --l) {
        if (wv < TW) {
          const int kt = l == L ? TI : TW;
          const f32x4* A = W4 + (l == L ? 0 : 64 * (TW * TI + (l - 1) * TW * TW));
          const float* in = arr + (l == L ? 0 : (l + 1) * ASZ);
          f32x4 a4 = zero4();
#pragma unroll
          for (int t = 0; t < (l == L ? TI : TW); ++t) {
            const f32x4 a = A[(wv * kt + t) * 64 + lane];
            const f32x4 b = ld4(in + rv_at<LDA>(c16, 16 * t + 4 * grp));
#pragma unroll
            for (int r = 0; r < 4; ++r) a4 = mfma_f32(a[r], b[r], a4);
          }
          const int o = rv_at<LDA>(c16, 16 * wv + 4 * grp);
          const f32x4 h = ld4(arr + (L + 1 + l) * ASZ + o);
          f32x4 dl;
#pragma unroll
          for (int r = 0; r < 4; ++r) dl[r] = a4[r] * (1.f - h[r] * h[r]);
          st4(arr + l * ASZ + o, dl);
        }
        __syncthreads();
      }
    }
    if constexpr (NR > 0 && NC > 0) {
      // weight-gradient tiles: the k slot of MFMA kb is path 4 kb + (lane / 16)
#pragma unroll
      for (int m = 0; m < L + 1; ++m) {
        if (m >= nmat) break;
        // staged operands of matrix m: (delta_1, x), (delta_{m+1}, h_m), (zeta, h_L); step 0 (zeta_0, ones)
        const float* As = arr + (m == L || n == 0 ? 0 : m + 1) * ASZ;
        const float* Bs = arr + (m == 0 ? L + 1 : L + 1 + m) * ASZ;
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
          const int row = 4 * kb + grp;
          float a[NR], b[NC];
#pragma unroll
          for (int i = 0; i < NR; ++i) a[i] = As[rv_at<LDA>(row, 16 * (R0 + i) + c16)];
#pragma unroll
          for (int j = 0; j < NC; ++j) b[j] = Bs[rv_at<LDA>(row, 16 * (C0 + j) + c16)];
#pragma unroll
          for (int i = 0; i < NR; ++i)
#pragma unroll
            for (int j = 0; j < NC; ++j) acc[m][i][j] = mfma_f32(a[i], b[j], acc[m][i][j]);
        }
      }
    }
  }
  // ---- this split's partial sums, scattered to the flat layout
  if constexpr (NR > 0 && NC > 0) {
    float* out = part + (size_t)blockIdx.x * g.pstride;
#pragma unroll
    for (int m = 0; m < L + 1; ++m) {
      if (m >= nmat) break;
      const RvMat T = rv_mat(g, n, m);
#pragma unroll
      for (int i = 0; i < NR; ++i)
#pragma unroll
        for (int j = 0; j < NC; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = 16 * (R0 + i) + 4 * grp + r, c = 16 * (C0 + j) + c16;
            if (row < T.rows && c <= T.cols) {
              const long long off = (c < T.cols) ? T.base + (long long)row * T.cols + c
                                                 : T.base + (long long)T.rows * T.cols + row;
              out[off] = acc[m][i][j][r];
            }
          }
    }
  }
}

template <int TI, int TW, int L>
__global__ __launch_bounds__(RV_THREADS) void k_reverse(Geo g, const void* __restrict__ packB,
                                                        const float* __restrict__ X, const float* __restrict__ V,
                                                        const float* __restrict__ LAM, const void* __restrict__ Hv,
                                                        float* __restrict__ part, long long chunk) {
  extern __shared__ __attribute__((aligned(16))) unsigned char wsm[];
  const long long p0 = (long long)blockIdx.x * chunk;
  const long long p1 = min((long long)g.M, p0 + chunk);
  const float* H = reinterpret_cast<const float*>(Hv);
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  constexpr int T = TI > TW ? TI : TW;
  if constexpr (T == 7) {
    if (wv < 7) rv_body<TI, TW, L, 6, 1>(g, packB, X, V, LAM, H, part, p0, p1, wsm, 0, wv);
    else rv_body<TI, TW, L, 1, 7>(g, packB, X, V, LAM, H, part, p0, p1, wsm, 6, 0);
  } else {
    static_assert(T <= RV_WAVES, "one tile column per wave");
    if (wv < T) rv_body<TI, TW, L, T, 1>(g, packB, X, V, LAM, H, part, p0, p1, wsm, 0, wv);
    else rv_body<TI, TW, L, 0, 0>(g, packB, X, V, LAM, H, part, p0, p1, wsm, 0, 0);
  }
}

// ------------------------------------------- fused reverse kernel, bf16 form
// The same scheme on the bf16 MFMA (16x16x32, fp32 accumulation) in rounds
// of 32 paths, the MFMA's K for the weight gradient.  Staged operands are
// bf16 in two layouts: P rows [path][feature] hold the reverse sweep's B
// operands (zeta, delta_2..delta_L) and the activations its epilogues read
// (h_l), F rows [feature][path] hold every weight-gradient operand (zeta,
// deltas, x, h_l with the bias row of ones), 8 consecutive paths per lane.
// Rounding points are those of the separate bf16 kernels: zeta and each
// delta are rounded to bf16 once, x when it is staged; the path-to-slot
// assignment (lane group g takes paths 8g..8g+7 of a 32-path chunk) is
// theirs too, so the two forms agree bitwise.  A staging item is a pair of
// paths times 4 features, consecutive lanes taking consecutive pairs: its F
// writes are 4-byte words (both paths of one feature) that 16 lanes lay
// side by side in one row; F rows are 80 bytes apart, so the 16-byte
// fragment reads of 8 lanes on 8 consecutive rows land in 8 distinct bank
// groups; P rows are 264 bytes apart (66 words), which spreads the 8-byte
// runs of 16 lanes on consecutive rows over distinct banks.
constexpr int RB_KC = 32, RB_LDF = RB_KC + 8;
__host__ __device__ constexpr int rb_ldp(int ti, int tw) { return 16 * (ti > tw ? ti : tw) + 4; }
__host__ __device__ constexpr size_t rb_array_bytes(int ti, int tw, int L) {
  return (size_t)2 * L * RB_KC * rb_ldp(ti, tw) * 2 + (size_t)(2 * L + 2) * 16 * (ti > tw ? ti : tw) * RB_LDF * 2;
}

__device__ __forceinline__ uint2 bf4_bits(f32x4 v) {
  return uint2{bf16_bits(v[0]) | (bf16_bits(v[1]) << 16), bf16_bits(v[2]) | (bf16_bits(v[3]) << 16)};
}
// four bf16 values of one path into column `col` of F rows row0..row0+3
__device__ __forceinline__ void rb_fput(uint16_t* F, int row0, int col, uint2 b) {
  F[(row0 + 0) * RB_LDF + col] = (uint16_t)(b.x & 0xffffu);
  F[(row0 + 1) * RB_LDF + col] = (uint16_t)(b.x >> 16);
  F[(row0 + 2) * RB_LDF + col] = (uint16_t)(b.y & 0xffffu);
  F[(row0 + 3) * RB_LDF + col] = (uint16_t)(b.y >> 16);
}
// the same for two paths (columns col, col + 1: one 4-byte word per row; col even)
__device__ __forceinline__ void rb_fput2(uint16_t* F, int row0, int col, uint2 b0, uint2 b1) {
  uint32_t* w = reinterpret_cast<uint32_t*>(F + row0 * RB_LDF + col);
  constexpr int R = RB_LDF / 2;
  w[0] = (b0.x & 0xffffu) | (b1.x << 16);
  w[R] = (b0.x >> 16) | (b1.x & 0xffff0000u);
  w[2 * R] = (b0.y & 0xffffu) | (b1.y << 16);
  w[3 * R] = (b0.y >> 16) | (b1.y & 0xffff0000u);
}
// bias row `cols` of ones and zeros past it, on a run of 4 rows starting at c
__device__ __forceinline__ uint2 rb_patch(uint2 b, int c, int cols) {
  uint32_t e[4] = {b.x & 0xffffu, b.x >> 16, b.y & 0xffffu, b.y >> 16};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (c + i == cols) e[i] = 0x3f80u;
    else if (c + i > cols) e[i] = 0u;
  }
  return uint2{e[0] | (e[1] << 16), e[2] | (e[3] << 16)};
}

// P arrays: 0 zeta, l - 1 delta_l (l = 2..L), L - 1 + l h_l.
// F arrays: 0 zeta, l delta_l (l = 1..L), L + 1 x (step 0: ones), L + 1 + l h_l.
template <int TI, int TW, int L, int NR, int NC>
__device__ __forceinline__ void rb_body(const Geo& g, const void* __restrict__ packB, const float* __restrict__ X,
                                        const float* __restrict__ V, const float* __restrict__ LAM,
                                        const uint16_t* __restrict__ H, float* __restrict__ part, long long p0,
                                        long long p1, unsigned char* wsm, int R0, int C0) {
  constexpr int TM = TI > TW ? TI : TW;
  constexpr int LDP = rb_ldp(TI, TW), PSZ = RB_KC * LDP, FSZ = 16 * TM * RB_LDF;
  static_assert(RB_KC / 2 * 4 * TM <= RV_THREADS, "one staging item per thread and input");
  const int n = g.n0 + (int)blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int c16 = lane & 15, grp = lane >> 4;
  uint16_t* Pa = reinterpret_cast<uint16_t*>(wsm + (size_t)g.packb_step * 2);
  uint16_t* Fa = Pa + 2 * L * PSZ;
  const size_t rowM = (size_t)g.M * g.dp, hM = (size_t)g.M * g.wp;
  const int nmat = n == 0 ? 1 : L + 1;

  // ---- staging items: input a (0 v, 1 x or ones, 1 + l h_l); item tid is
  // paths 2 pp, 2 pp + 1 of the round times columns c..c+3 (c = -1: none)
  constexpr int NA = L + 2;
  int spp[NA], sc[NA];
#pragma unroll
  for (int a = 0; a < NA; ++a) {
    const int gq = a == 0 ? g.dp / 4 : (a == 1 ? (n == 0 ? 1 : (g.d + 4) / 4) : (g.w + 4) / 4);
    const int j = tid / (RB_KC / 2);
    spp[a] = tid % (RB_KC / 2);
    sc[a] = j < gq ? 4 * j : -1;
  }
  const float* Vn = V + n * rowM;
  const float* Ln = LAM + (size_t)n * g.M;
  const float* Xn = X + n * rowM;
  f32x4 rv[2], rx[2];
  uint2 rh[L][2];
  float rl[2];
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    rv[e] = zero4(); rx[e] = zero4(); rl[e] = 0.f;
#pragma unroll
    for (int l = 0; l < L; ++l) rh[l][e] = uint2{0u, 0u};
  }
  // raw loads, unconditional (rows and columns clamped into their buffers)
  auto fetch = [&](long long pc) {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const size_t p = (size_t)min(pc + 2 * spp[0] + e, p1 - 1);
      rv[e] = ld4(Vn + p * g.dp + max(sc[0], 0));
      rl[e] = Ln[p];
      if (n > 0) {
        rx[e] = ld4(Xn + p * g.dp + min(max(sc[1], 0), g.dp - 4));
#pragma unroll
        for (int l = 0; l < L; ++l)
          rh[l][e] = *reinterpret_cast<const uint2*>(H + (act_step(g, n) * L + l) * hM + p * g.wp +
                                                     min(max(sc[2 + l], 0), g.wp - 4));
      }
    }
  };
  // validity, rounding, the bias row and the padding; P and F writes
  auto put = [&](long long pc) {
    const int pp = spp[0];
    const bool ok0 = pc + 2 * pp < p1, ok1 = pc + 2 * pp + 1 < p1;
    {  // zeta = bf16(lambda v)
      const int c = sc[0];
      if (c >= 0) {
        const uint2 b0 = ok0 ? bf4_bits(rl[0] * rv[0]) : uint2{0u, 0u};
        const uint2 b1 = ok1 ? bf4_bits(rl[1] * rv[1]) : uint2{0u, 0u};
        *reinterpret_cast<uint2*>(Pa + (2 * pp) * LDP + c) = b0;
        *reinterpret_cast<uint2*>(Pa + (2 * pp + 1) * LDP + c) = b1;
        rb_fput2(Fa, c, 2 * pp, b0, b1);
      }
    }
    {  // x in bf16 (step 0: the column of ones)
      const int c = sc[1];
      if (c >= 0) {
        const int cols = n == 0 ? 0 : g.d;
        const bool have = n > 0 && c < g.dp;
        const uint2 b0 = ok0 ? rb_patch(have ? bf4_bits(rx[0]) : uint2{0u, 0u}, c, cols) : uint2{0u, 0u};
        const uint2 b1 = ok1 ? rb_patch(have ? bf4_bits(rx[1]) : uint2{0u, 0u}, c, cols) : uint2{0u, 0u};
        rb_fput2(Fa + (L + 1) * FSZ, c, 2 * pp, b0, b1);
      }
    }
    if (n > 0) {
#pragma unroll
      for (int l = 0; l < L; ++l) {  // h_{l+1}: P raw, F with the bias row
        const int c = sc[2 + l];
        if (c >= 0) {
          const uint2 b0 = ok0 ? rh[l][0] : uint2{0u, 0u}, b1 = ok1 ? rh[l][1] : uint2{0u, 0u};
          *reinterpret_cast<uint2*>(Pa + (L + l) * PSZ + (2 * pp) * LDP + c) = b0;
          *reinterpret_cast<uint2*>(Pa + (L + l) * PSZ + (2 * pp + 1) * LDP + c) = b1;
          rb_fput2(Fa + (L + 2 + l) * FSZ, c, 2 * pp, ok0 ? rb_patch(b0, c, g.w) : b0,
                   ok1 ? rb_patch(b1, c, g.w) : b1);
        }
      }
    }
  };

  f32x4 acc[L + 1][NRA_(NR)][NCA_(NC)];
#pragma unroll
  for (int m = 0; m < L + 1; ++m)
#pragma unroll
    for (int i = 0; i < NRA_(NR); ++i)
#pragma unroll
      for (int j = 0; j < NCA_(NC); ++j) acc[m][i][j] = zero4();

  fetch(p0);
  if (n > 0) copy_to_lds(wsm, reinterpret_cast<const char*>(packB) + (size_t)(n - 1) * g.packb_step * 2,
                         (size_t)g.packb_step * 2);
  // rows and columns no round writes stay zero
  for (int e = tid; e < (int)(rb_array_bytes(TI, TW, L) / 16); e += RV_THREADS)
    reinterpret_cast<uint4*>(Pa)[e] = uint4{0u, 0u, 0u, 0u};
  const bf16x8* W8 = reinterpret_cast<const bf16x8*>(wsm);
  for (long long pc = p0; pc < p1; pc += RB_KC) {
    __syncthreads();  // weights and zero fill (first round), or the previous round's reads, are done
    put(pc);
    __syncthreads();
    if (pc + RB_KC < p1) fetch(pc + RB_KC);  // in flight during this round's MFMAs
    if (n > 0) {
      // delta_L = bf16((W_o^T zeta) (1 - h_L^2)), delta_l = bf16((W_{l+1}^T delta_{l+1}) (1 - h_l^2))
#pragma unroll
      for (int l = L; l >= 1; --l) {
        if (wv < TW) {
          const int kt = l == L ? TI : TW;
          const bf16x8* A = W8 + (l == L ? 0 : 32 * (TW * TI + (l - 1) * TW * TW));
          const uint16_t* in = Pa + (l == L ? 0 : l) * PSZ;
          f32x4 a4[2] = {zero4(), zero4()};
#pragma unroll
          for (int kb = 0; kb < (l == L ? TI : TW) / 2; ++kb) {
            const bf16x8 a = A[(wv * (kt / 2) + kb) * 64 + lane];
#pragma unroll
            for (int pt = 0; pt < 2; ++pt) {
              const uint16_t* r = in + (16 * pt + c16) * LDP + 32 * kb + 4 * grp;
              const uint2 lo = *reinterpret_cast<const uint2*>(r), hi = *reinterpret_cast<const uint2*>(r + 16);
              a4[pt] = mfma_bf16(a, __builtin_bit_cast(bf16x8, u32x4{lo.x, lo.y, hi.x, hi.y}), a4[pt]);
            }
          }
#pragma unroll
          for (int pt = 0; pt < 2; ++pt) {
            const int row = 16 * pt + c16, col = 16 * wv + 4 * grp;
            const uint2 hb = *reinterpret_cast<const uint2*>(Pa + (L - 1 + l) * PSZ + row * LDP + col);
            const float h[4] = {__uint_as_float(hb.x << 16), __uint_as_float(hb.x & 0xffff0000u),
                                __uint_as_float(hb.y << 16), __uint_as_float(hb.y & 0xffff0000u)};
            f32x4 dl;
#pragma unroll
            for (int r = 0; r < 4; ++r) dl[r] = a4[pt][r] * (1.f - h[r] * h[r]);
            const uint2 db = bf4_bits(dl);
            if (l >= 2) *reinterpret_cast<uint2*>(Pa + (l - 1) * PSZ + row * LDP + col) = db;
            rb_fput(Fa + l * FSZ, col, row, db);
          }
        }
        __syncthreads();
      }
    }
    if constexpr (NR > 0 && NC > 0) {
      // weight-gradient tiles, K = the round's 32 paths (lane group g: paths 8g..8g+7)
#pragma unroll
      for (int m = 0; m < L + 1; ++m) {
        if (m >= nmat) break;
        const uint16_t* As = Fa + (m == L || n == 0 ? 0 : m + 1) * FSZ;
        const uint16_t* Bs = Fa + (m == 0 ? L + 1 : L + 1 + m) * FSZ;
        bf16x8 a[NR], b[NC];
#pragma unroll
        for (int i = 0; i < NR; ++i)
          a[i] = *reinterpret_cast<const bf16x8*>(As + (16 * (R0 + i) + c16) * RB_LDF + 8 * grp);
#pragma unroll
        for (int j = 0; j < NC; ++j)
          b[j] = *reinterpret_cast<const bf16x8*>(Bs + (16 * (C0 + j) + c16) * RB_LDF + 8 * grp);
#pragma unroll
        for (int i = 0; i < NR; ++i)
#pragma unroll
          for (int j = 0; j < NC; ++j) acc[m][i][j] = mfma_bf16(a[i], b[j], acc[m][i][j]);
      }
    }
  }
  // ---- this split's partial sums, scattered to the flat layout
  if constexpr (NR > 0 && NC > 0) {
    float* out = part + (size_t)blockIdx.x * g.pstride;
#pragma unroll
    for (int m = 0; m < L + 1; ++m) {
      if (m >= nmat) break;
      const RvMat T = rv_mat(g, n, m);
#pragma unroll
      for (int i = 0; i < NR; ++i)
#pragma unroll
        for (int j = 0; j < NC; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = 16 * (R0 + i) + 4 * grp + r, c = 16 * (C0 + j) + c16;
            if (row < T.rows && c <= T.cols) {
              const long long off = (c < T.cols) ? T.base + (long long)row * T.cols + c
                                                 : T.base + (long long)T.rows * T.cols + row;
              out[off] = acc[m][i][j][r];
            }
          }
    }
  }
}

template <int TI, int TW, int L>
__global__ __launch_bounds__(RV_THREADS) void k_reverse_bf(Geo g, const void* __restrict__ packB,
                                                           const float* __restrict__ X, const float* __restrict__ V,
                                                           const float* __restrict__ LAM, const void* __restrict__ Hv,
                                                           float* __restrict__ part, long long chunk) {
  extern __shared__ __attribute__((aligned(16))) unsigned char wsm[];
  const long long p0 = (long long)blockIdx.x * chunk;
  const long long p1 = min((long long)g.M, p0 + chunk);
  const uint16_t* H = reinterpret_cast<const uint16_t*>(Hv);
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  constexpr int T = TI > TW ? TI : TW;
  static_assert(T <= RV_WAVES, "one tile column per wave");
  if (wv < T) rb_body<TI, TW, L, T, 1>(g, packB, X, V, LAM, H, part, p0, p1, wsm, 0, wv);
  else rb_body<TI, TW, L, 0, 0>(g, packB, X, V, LAM, H, part, p0, p1, wsm, 0, 0);
}

// ------------------------------------------------------------ reduce kernel
// grad[e] = sum over splits k (in order) of part[k * stride + e]; 4 elements
// per thread when grad is 16-byte aligned (the partial copies always are).
// fp64 loss and dY0 from the scan's per-block partials (one wave; strided
// per-lane sums, then a fixed xor butterfly, so the result is deterministic).
// A non-finite loss or dY0 raises the host flag.
__device__ __forceinline__ void finalize_wave(int M, const double* __restrict__ sp, int nb, double* loss,
                                              double* gy0, int* host_flag) {
  double a = 0.0, b = 0.0;
  // each lane adds partials k, k + 64, k + 128, ... in that order; the loads
  // of eight of them are issued before their adds (missing ones add 0)
  for (int k0 = threadIdx.x; k0 < nb; k0 += 64 * 8) {
    double av[8], bv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int k = k0 + 64 * q;
      av[q] = k < nb ? sp[2 * k] : 0.0;
      bv[q] = k < nb ? sp[2 * k + 1] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) { a += av[q]; b += bv[q]; }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o);
    b += __shfl_xor(b, o);
  }
  if (threadIdx.x == 0) {
    if (loss) loss[0] = a / (double)M;
    if (gy0) gy0[0] = b;
    const bool bad = !isfinite(a) || (gy0 != nullptr && !isfinite(b));
    if (bad && host_flag) host_flag[0] = 1;
  }
}

// grad[e] = sum over splits k (in order) of part[k * stride + e], 4 elements
// per thread over the first nred workgroups; a non-finite sum raises the host
// flag.  Workgroup nred (the last one) finalizes the loss and dY0 from the
// scan's partials, which the reduction does not touch, so both run in one
// launch.
// Sum over the split partials of one float4 group (or one element), in split
// order from zero.  The loads go out eight at a time, so a thread waits for
// one memory latency per eight splits instead of one per split; the
// additions keep their order, so the sum is the same bits.
constexpr int RED_BATCH = 8;
__device__ __forceinline__ f32x4 sum_splits4(const float* __restrict__ part, long long stride, int splits,
                                             long long e4) {
  f32x4 s = zero4();
  for (int k0 = 0; k0 < splits; k0 += RED_BATCH) {
    f32x4 t[RED_BATCH];
#pragma unroll
    for (int q = 0; q < RED_BATCH; ++q)
      t[q] = k0 + q < splits ? ld4(part + (size_t)(k0 + q) * stride + 4 * e4) : zero4();
#pragma unroll
    for (int q = 0; q < RED_BATCH; ++q)
      if (k0 + q < splits) s += t[q];
  }
  return s;
}
__device__ __forceinline__ float sum_splits1(const float* __restrict__ part, long long stride, int splits,
                                             long long e) {
  float s = 0.f;
  for (int k0 = 0; k0 < splits; k0 += RED_BATCH) {
    float t[RED_BATCH];
#pragma unroll
    for (int q = 0; q < RED_BATCH; ++q) t[q] = k0 + q < splits ? part[(size_t)(k0 + q) * stride + e] : 0.f;
#pragma unroll
    for (int q = 0; q < RED_BATCH; ++q)
      if (k0 + q < splits) s += t[q];
  }
  return s;
}

__global__ __launch_bounds__(256) void k_reduce(long long P, long long stride, const float* __restrict__ part,
                                                int splits, float* __restrict__ grad, int nred, int M,
                                                const double* __restrict__ sp, int nb, double* __restrict__ loss,
                                                double* __restrict__ gy0, int* __restrict__ host_flag) {
  if ((int)blockIdx.x == nred) {
    if (threadIdx.x < 64) finalize_wave(M, sp, nb, loss, gy0, host_flag);
    return;
  }
  bool bad = false;
  const long long t0 = blockIdx.x * 256LL + threadIdx.x, step = (long long)nred * 256;
  const long long P4 = (reinterpret_cast<uintptr_t>(grad) & 15) == 0 ? P / 4 : 0;
  for (long long e4 = t0; e4 < P4; e4 += step) {
    const f32x4 s = sum_splits4(part, stride, splits, e4);
    st4(grad + 4 * e4, s);
    bad |= !(isfinite(s[0]) && isfinite(s[1]) && isfinite(s[2]) && isfinite(s[3]));
  }
  for (long long e = 4 * P4 + t0; e < P; e += step) {
    const float s = sum_splits1(part, stride, splits, e);
    grad[e] = s;
    bad |= !isfinite(s);
  }
  if (bad && host_flag) host_flag[0] = 1;  // every writer stores the same value
}

__global__ __launch_bounds__(64) void k_finalize(int M, const double* __restrict__ sp, int nb,
                                                 double* __restrict__ loss, int* __restrict__ host_flag) {
  finalize_wave(M, sp, nb, loss, nullptr, host_flag);
}

// -------------------------------------------------------------- Adam kernel
// Adam step t (bias corrections c1 = 1 - b1^t, c2 = 1 - b2^t).  With t_dev
// non-null, t = t_dev[0] + 1 is read on the device (graph replays).
// Adam arithmetic shared by k_adam and the fused reduction + Adam kernel, so
// that both give the same bits: bias corrections c1 = 1 - b1^t and
// c2 = 1 - b2^t (t = t_dev[0] + 1 on the device for graph replays), the
// fp32 parameter update and the fp64 update of y0.
__device__ __forceinline__ void adam_corr(double t_imm, const uint64_t* t_dev, double b1d, double b2d, double* corr) {
  const double t = t_dev ? (double)(t_dev[0] + 1) : t_imm;
  corr[0] = 1.0 - pow(b1d, t);
  corr[1] = 1.0 - pow(b2d, t);
}
// The moment updates are written as explicit fused multiply-adds: left to
// the compiler, which product it fuses can differ between two kernels that
// inline the same expression.
__device__ __forceinline__ float adam_upd(float pi, float gi, float& mi, float& vi, float lr, float b1, float b2,
                                          float eps, float c1, float c2) {
  mi = fmaf(b1, mi, (1.f - b1) * gi);
  vi = fmaf(b2, vi, ((1.f - b2) * gi) * gi);
  return pi - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}
__device__ __forceinline__ void adam_y0(double gi, double* y0, double* my0, double* vy0, double lr_y0, double b1d,
                                        double b2d, double epsd, double c1d, double c2d) {
  const double mi = fma(b1d, my0[0], (1.0 - b1d) * gi);
  const double vi = fma(b2d, vy0[0], ((1.0 - b2d) * gi) * gi);
  my0[0] = mi;
  vy0[0] = vi;
  y0[0] -= lr_y0 * (mi / c1d) / (sqrt(vi / c2d) + epsd);
}

__global__ __launch_bounds__(256) void k_adam(long long n, float* __restrict__ p, const float* __restrict__ gr,
                                              float* __restrict__ m, float* __restrict__ v,
                                              double* __restrict__ y0, const double* __restrict__ gy0,
                                              double* __restrict__ my0, double* __restrict__ vy0, float lr,
                                              double t_imm, const uint64_t* __restrict__ t_dev, double lr_y0,
                                              double b1d, double b2d, double epsd) {
  const float b1 = (float)b1d, b2 = (float)b2d, eps = (float)epsd;
  const long long i0 = blockIdx.x * 256LL + threadIdx.x;
  // 4 elements per thread when the four arrays are 16-byte aligned, then the tail
  const bool vec = ((reinterpret_cast<uintptr_t>(p) | reinterpret_cast<uintptr_t>(gr) |
                     reinterpret_cast<uintptr_t>(m) | reinterpret_cast<uintptr_t>(v)) & 15) == 0;
  const long long n4 = vec ? n / 4 : 0;
  // the first element's loads are issued before the bias corrections are
  // known, so their latency overlaps the workgroup's pow evaluations
  f32x4 P4 = zero4(), G4 = zero4(), M4 = zero4(), V4 = zero4();
  if (i0 < n4) {
    P4 = reinterpret_cast<const f32x4*>(p)[i0];
    G4 = reinterpret_cast<const f32x4*>(gr)[i0];
    M4 = reinterpret_cast<const f32x4*>(m)[i0];
    V4 = reinterpret_cast<const f32x4*>(v)[i0];
  }
  // bias corrections: one evaluation per workgroup, shared through LDS (the
  // same device code for an immediate step count and a device-side counter)
  __shared__ double corr[2];
  if (threadIdx.x == 0) adam_corr(t_imm, t_dev, b1d, b2d, corr);
  __syncthreads();
  const double c1d = corr[0], c2d = corr[1];
  const float c1 = (float)c1d, c2 = (float)c2d;
  auto upd = [&](float pi, float gi, float& mi, float& vi) { return adam_upd(pi, gi, mi, vi, lr, b1, b2, eps, c1, c2); };
  for (long long i = i0; i < n4; i += (long long)gridDim.x * 256) {
    if (i != i0) {
      P4 = reinterpret_cast<const f32x4*>(p)[i];
      G4 = reinterpret_cast<const f32x4*>(gr)[i];
      M4 = reinterpret_cast<const f32x4*>(m)[i];
      V4 = reinterpret_cast<const f32x4*>(v)[i];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float mi = M4[r], vi = V4[r];
      P4[r] = upd(P4[r], G4[r], mi, vi);
      M4[r] = mi;
      V4[r] = vi;
    }
    reinterpret_cast<f32x4*>(m)[i] = M4;
    reinterpret_cast<f32x4*>(v)[i] = V4;
    reinterpret_cast<f32x4*>(p)[i] = P4;
  }
  for (long long i = 4 * n4 + i0; i < n; i += (long long)gridDim.x * 256) {
    float mi = m[i], vi = v[i];
    p[i] = upd(p[i], gr[i], mi, vi);
    m[i] = mi;
    v[i] = vi;
  }
  if (i0 == 0 && y0) adam_y0(gy0[0], y0, my0, vy0, lr_y0, b1d, b2d, epsd, c1d, c2d);
}

// One training step's tail in one launch: workgroups [0, nred) sum the
// split partials of 4 elements per thread into grad (as k_reduce) and apply
// Adam to those elements at once (as k_adam); workgroup nred forms the loss
// and dY0 (as k_reduce's last workgroup) and applies Adam to y0.  Non-finite
// sums raise the host flag; the update is applied regardless.
__global__ __launch_bounds__(256) void k_reduce_adam(long long P, long long stride, const float* __restrict__ part,
                                                     int splits, float* __restrict__ grad, int nred, int M,
                                                     const double* __restrict__ sp, int nb, double* __restrict__ loss,
                                                     double* __restrict__ gy0, int* __restrict__ host_flag,
                                                     float* __restrict__ p, float* __restrict__ m,
                                                     float* __restrict__ v, double* __restrict__ y0,
                                                     double* __restrict__ my0, double* __restrict__ vy0, float lr,
                                                     double t_imm, const uint64_t* __restrict__ t_dev, double lr_y0,
                                                     double b1d, double b2d, double epsd) {
  __shared__ double corr[2];
  if ((int)blockIdx.x == nred) {
    if (threadIdx.x == 0) adam_corr(t_imm, t_dev, b1d, b2d, corr);
    __syncthreads();
    if (threadIdx.x < 64) {
      finalize_wave(M, sp, nb, loss, gy0, host_flag);
      if (threadIdx.x == 0 && y0) adam_y0(gy0[0], y0, my0, vy0, lr_y0, b1d, b2d, epsd, corr[0], corr[1]);
    }
    return;
  }
  bool bad = false;
  const long long t0 = blockIdx.x * 256LL + threadIdx.x, step = (long long)nred * 256;
  const bool vec = ((reinterpret_cast<uintptr_t>(grad) | reinterpret_cast<uintptr_t>(p) |
                     reinterpret_cast<uintptr_t>(m) | reinterpret_cast<uintptr_t>(v)) & 15) == 0;
  const long long P4 = vec ? P / 4 : 0;
  // the first element's sum is formed before the bias corrections are known,
  // so the partial loads overlap the workgroup's pow evaluations
  f32x4 s0 = zero4();
  if (t0 < P4) s0 = sum_splits4(part, stride, splits, t0);
  if (threadIdx.x == 0) adam_corr(t_imm, t_dev, b1d, b2d, corr);
  __syncthreads();
  const double c1d = corr[0], c2d = corr[1];
  const float b1 = (float)b1d, b2 = (float)b2d, eps = (float)epsd, c1 = (float)c1d, c2 = (float)c2d;
  for (long long e4 = t0; e4 < P4; e4 += step) {
    const f32x4 s = e4 == t0 ? s0 : sum_splits4(part, stride, splits, e4);
    st4(grad + 4 * e4, s);
    bad |= !(isfinite(s[0]) && isfinite(s[1]) && isfinite(s[2]) && isfinite(s[3]));
    f32x4 P4v = reinterpret_cast<const f32x4*>(p)[e4], M4 = reinterpret_cast<const f32x4*>(m)[e4],
          V4 = reinterpret_cast<const f32x4*>(v)[e4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float mi = M4[r], vi = V4[r];
      P4v[r] = adam_upd(P4v[r], s[r], mi, vi, lr, b1, b2, eps, c1, c2);
      M4[r] = mi;
      V4[r] = vi;
    }
    reinterpret_cast<f32x4*>(m)[e4] = M4;
    reinterpret_cast<f32x4*>(v)[e4] = V4;
    reinterpret_cast<f32x4*>(p)[e4] = P4v;
  }
  for (long long e = 4 * P4 + t0; e < P; e += step) {
    const float s = sum_splits1(part, stride, splits, e);
    grad[e] = s;
    bad |= !isfinite(s);
    float mi = m[e], vi = v[e];
    p[e] = adam_upd(p[e], s, mi, vi, lr, b1, b2, eps, c1, c2);
    m[e] = mi;
    v[e] = vi;
  }
  if (bad && host_flag) host_flag[0] = 1;  // every writer stores the same value
}

__global__ void k_count(uint64_t* __restrict__ c) {
  if (threadIdx.x == 0 && blockIdx.x == 0) c[0] += 1;
}

// --------------------------------------------------------- prolong kernel
__global__ __launch_bounds__(256) void k_prolong(int d, long long pstep, int Nc, long long Pf,
                                                 const float* __restrict__ pc, float* __restrict__ pf) {
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < Pf; e += (long long)gridDim.x * 256) {
    if (e < d) { pf[e] = pc[e]; continue; }
    const long long q = e - d;
    const int j = 1 + (int)(q / pstep);
    int c = j / 2;
    c = c < 1 ? 1 : (c > Nc - 1 ? Nc - 1 : c);
    pf[e] = pc[d + (long long)(c - 1) * pstep + q % pstep];
  }
}

// ---------------------------------------------------------- test hooks
__global__ __launch_bounds__(256) void k_normals(Geo g, uint64_t seed, uint64_t iter, float* __restrict__ xi) {
  const int G = g.dp / 4;
  const long long total = (long long)g.N * g.M * G;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < total; e += (long long)gridDim.x * 256) {
    const int j = (int)(e % G);
    const long long q = e / G;
    const int m = (int)(q % g.M), n = (int)(q / g.M);
    const f32x4 z = normals4(seed, iter, j, n, m);
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (4 * j + r < g.d) xi[((size_t)n * g.M + m) * g.d + 4 * j + r] = z[r];
  }
}

__global__ __launch_bounds__(256) void k_gmean(Geo g, const float* __restrict__ QN, const float* __restrict__ LN,
                                               double* __restrict__ out) {
  __shared__ double sh[256];
  double a = 0.0;
  for (int m = threadIdx.x; m < g.M; m += 256) a += (double)terminal_g(g, QN[m], LN[m]);
  const double A = block_sum_256(a, sh);
  if (threadIdx.x == 0) out[0] = A / (double)g.M;
}

__global__ __launch_bounds__(256) void k_terminal_copy(Geo g, const float* __restrict__ X,
                                                       const float* __restrict__ Y, float* __restrict__ xN,
                                                       float* __restrict__ yN) {
  const long long total = (long long)g.M * g.d;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < total; e += (long long)gridDim.x * 256) {
    const int m = (int)(e / g.d), i = (int)(e % g.d);
    if (xN) xN[e] = X[((size_t)g.N * g.M + m) * g.dp + i];
    if (yN && i == 0) yN[m] = Y[(size_t)g.N * g.M + m];
  }
}

// ================================================================ launchers
static inline unsigned grid1(long long n, long long cap = 65536) {
  long long b = (n + 255) / 256;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}


hipError_t launch_pack_sde(const Geo& g, const float* params, void* packF, void* packB, float* pbias,
                           const float* x0, uint64_t seed, uint64_t iter, const uint64_t* iter_dev, float* X,
                           float* V, float* QN, float* LN, hipStream_t s) {
  const int G = g.bf16 ? 8 : 4;
  const long long per = (g.packf_step + g.packb_step) / G + g.pbias_step;
  const int pack_gx = (int)grid1(per, 1024);
  const int pack_blocks = g.N >= 2 ? pack_gx * (g.N - 1) : 0;
  const int T = g.dp / 4 < 256 ? g.dp / 4 : 256;  // threads per path, as in sde_block
  const int ppb = 256 / T;
  const int sde_blocks = (int)((g.M + ppb - 1) / ppb);
  const unsigned blocks = (unsigned)(pack_blocks + sde_blocks);
  if (g.bf16)
    k_pack_sde<true><<<blocks, 256, 0, s>>>(g, params, packF, packB, pbias, pack_gx, sde_blocks, x0, seed, iter,
                                            iter_dev, X, V, QN, LN);
  else
    k_pack_sde<false><<<blocks, 256, 0, s>>>(g, params, packF, packB, pbias, pack_gx, sde_blocks, x0, seed, iter,
                                             iter_dev, X, V, QN, LN);
  return hipGetLastError();
}

hipError_t launch_sde(const Geo& g, const float* x0, uint64_t seed, uint64_t iter, const uint64_t* iter_dev,
                      float* X, float* V, float* QN, float* LN, hipStream_t s) {
  const int T = g.dp / 4 < 256 ? g.dp / 4 : 256;  // threads per path, as in k_sde
  const int ppb = 256 / T;
  const unsigned blocks = (unsigned)((g.M + ppb - 1) / ppb);
  k_sde<<<blocks, 256, 0, s>>>(g, x0, seed, iter, iter_dev, X, V, QN, LN);
  return hipGetLastError();
}

// Tiles of 16 paths per wave for the LDS-resident kernels: the count that
// minimises the makespan ceil(workgroups / CUs) * (work per SIMD + staging),
// one workgroup per CU.  A workgroup of `waves` waves gets ceil(tiles / gx)
// tiles of its step, dealt to its waves in turn, so each of the 4 SIMDs runs
// about a quarter of them; staging the step's weights in LDS costs about a
// quarter of one wave's tile.  In units of 1 / (4 * waves) of a wave-tile:
// span = rounds * (16 * ceil(per_wg / 4) + waves).
static int tiles_per_wave(const Geo& g, int waves, int cus) {
  const long long tiles = (g.M + 15) / 16;
  int best = 1;
  long long best_span = -1;
  for (int t = 1; t <= 64; ++t) {
    const long long gx = (tiles + (long long)waves * t - 1) / ((long long)waves * t);
    const long long per_wg = (tiles + gx - 1) / gx;
    const long long wgs = gx * launch_steps(g);  // a launch over a chunk of steps has fewer rows of workgroups
    const long long span = ((wgs + cus - 1) / cus) * (16LL * ((per_wg + 3) / 4) + waves);
    if (best_span < 0 || span < best_span) { best_span = span; best = t; }
  }
  return best;
}

static int num_cus() {
  static int cus = [] {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1)
      n = 256;
    return n;
  }();
  return cus;
}

int device_cus() { return num_cus(); }

static const size_t kLdsLimit = 160 * 1024;

bool lds_fits(const Geo& g) {
  const size_t esz = g.bf16 ? 2 : 4;
  return (size_t)g.packf_step * esz + (size_t)g.pbias_step * 4 <= kLdsLimit &&
         (size_t)g.packb_step * esz <= kLdsLimit;
}

// LDS bytes of the largest single layer (the layer-streamed kernels stage one at a time)
static constexpr size_t ls_layer_bytes(bool bf, int ti, int tw) {
  return 256ull * (size_t)tw * (size_t)(ti > tw ? ti : tw) * (bf ? 2 : 4);
}

int auto_tiles_per_wave(const Geo& g) { return tiles_per_wave(g, fwd_waves(g.ti, g.tw), num_cus()); }

template <bool BF, int TI, int TW>
static void fwd_inst(const Geo& g, const float* params, const void* packF, const float* pbias, const float* X,
                     float* V, float* C, void* H, hipStream_t s) {
  const size_t bytes = (size_t)g.packf_step * (BF ? 2 : 4) + (size_t)g.pbias_step * 4;
  if (g.lds && bytes <= kLdsLimit && g.N > 1) {
    static bool attr = [] {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_forward<BF, TI, TW, true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit);
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_forward<BF, TI, TW, true, true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit);
      return true;
    }();
    (void)attr;
    constexpr int NW = fwd_waves(TI, TW);
    const int tpw = g.tpw > 0 ? g.tpw : tiles_per_wave(g, NW, num_cus());
    dim3 grid((unsigned)(((g.M + 15) / 16 + NW * tpw - 1) / (NW * tpw)), launch_steps(g));
    if (g.recomp)
      k_forward<BF, TI, TW, true, true><<<grid, 64 * NW, bytes, s>>>(g, params, packF, pbias, X, V, C, H, tpw);
    else
      k_forward<BF, TI, TW, true><<<grid, 64 * NW, bytes, s>>>(g, params, packF, pbias, X, V, C, H, tpw);
  } else if (g.lds && ls_layer_bytes(BF, TI, TW) <= kLdsLimit && g.N > 1) {
    static bool attr = [] {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_forward_ls<BF, TI, TW>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit);
      return true;
    }();
    (void)attr;
    const int tpw = g.tpw > 0 ? g.tpw : tiles_per_wave(g, LS_WAVES, num_cus());
    dim3 grid((unsigned)(((g.M + 15) / 16 + LS_WAVES * tpw - 1) / (LS_WAVES * tpw)), launch_steps(g));
    k_forward_ls<BF, TI, TW><<<grid, 64 * LS_WAVES, ls_layer_bytes(BF, TI, TW), s>>>(g, params, packF, pbias, X, V, C,
                                                                                     H, tpw);
  } else {
    dim3 grid((g.M + 63) / 64, launch_steps(g));
    if (g.recomp)
      k_forward<BF, TI, TW, false, true><<<grid, 256, 0, s>>>(g, params, packF, pbias, X, V, C, H, 1);
    else
      k_forward<BF, TI, TW, false><<<grid, 256, 0, s>>>(g, params, packF, pbias, X, V, C, H, 1);
  }
}
template <bool BF, int TI, int TW>
static void bwd_inst(const Geo& g, const void* packB, const float* V, const float* LAM, const void* H,
                     void* DZ, void* DH, hipStream_t s) {
  const size_t bytes = (size_t)g.packb_step * (BF ? 2 : 4);
  if (g.lds && bytes <= kLdsLimit && g.N > 1) {
    static bool attr = [] {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_backward<BF, TI, TW, true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit);
      return true;
    }();
    (void)attr;
    constexpr int NW = bwd_waves(TI, TW);
    const int tpw = g.tpw > 0 ? g.tpw : tiles_per_wave(g, NW, num_cus());
    dim3 grid((unsigned)(((g.M + 15) / 16 + NW * tpw - 1) / (NW * tpw)), launch_steps(g));
    k_backward<BF, TI, TW, true><<<grid, 64 * NW, bytes, s>>>(g, packB, V, LAM, H, DZ, DH, tpw);
  } else if (g.lds && ls_layer_bytes(BF, TI, TW) <= kLdsLimit && g.N > 1) {
    static bool attr = [] {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_backward_ls<BF, TI, TW>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit);
      return true;
    }();
    (void)attr;
    const int tpw = g.tpw > 0 ? g.tpw : tiles_per_wave(g, LS_WAVES, num_cus());
    dim3 grid((unsigned)(((g.M + 15) / 16 + LS_WAVES * tpw - 1) / (LS_WAVES * tpw)), launch_steps(g));
    k_backward_ls<BF, TI, TW><<<grid, 64 * LS_WAVES, ls_layer_bytes(BF, TI, TW), s>>>(g, packB, V, LAM, H, DZ, DH,
                                                                                      tpw);
  } else {
    dim3 grid((g.M + 63) / 64, launch_steps(g));
    k_backward<BF, TI, TW, false><<<grid, 256, 0, s>>>(g, packB, V, LAM, H, DZ, DH, 1);
  }
}

// Instantiated register-tile shapes (TI tiles over d, TW tiles over w).
// The plan picks the one with the least padded MFMA work that covers the
// problem; FBSDE_MIN_TILES=k forces both counts to at least k (tests of the
// padded path).
struct TileShape { int bf, ti, tw; };
static const TileShape kShapes[] = {
    {0, 1, 2}, {0, 2, 2}, {0, 4, 4}, {0, 7, 7}, {0, 8, 8}, {0, 16, 16},
    {1, 2, 2}, {1, 4, 4}, {1, 6, 6}, {1, 8, 8}, {1, 10, 10}, {1, 12, 12}, {1, 14, 14}, {1, 16, 16},
};

int tile_candidates(int bf16, int ti_min, int tw_min, int* ti, int* tw, int cap) {
  int n = 0;
  // insertion by cost (ti * tw), ties by order of kShapes
  for (const TileShape& s : kShapes) {
    if (s.bf != bf16 || s.ti < ti_min || s.tw < tw_min) continue;
    int pos = n;
    while (pos > 0 && (long long)ti[pos - 1] * tw[pos - 1] > (long long)s.ti * s.tw) --pos;
    if (pos >= cap) continue;
    for (int q = (n < cap ? n : cap - 1); q > pos; --q) { ti[q] = ti[q - 1]; tw[q] = tw[q - 1]; }
    ti[pos] = s.ti;
    tw[pos] = s.tw;
    if (n < cap) ++n;
  }
  return n;
}

bool choose_tiles(int bf16, int ti_min, int tw_min, int* ti, int* tw) {
  static const int forced = [] {
    const char* e = getenv("FBSDE_MIN_TILES");
    return e ? atoi(e) : 0;
  }();
  if (forced > ti_min) ti_min = forced;
  if (forced > tw_min) tw_min = forced;
  long long best = -1;
  for (const TileShape& s : kShapes) {
    if (s.bf != bf16 || s.ti < ti_min || s.tw < tw_min) continue;
    const long long cost = (long long)s.ti * s.tw;
    if (best < 0 || cost < best) { best = cost; *ti = s.ti; *tw = s.tw; }
  }
  return best >= 0;
}

#define FBSDE_DISPATCH(FN, ...)                                                   \
  do {                                                                            \
    if (g.bf16) {                                                                 \
      if (g.ti == 2 && g.tw == 2) FN<true, 2, 2>(__VA_ARGS__);                    \
      else if (g.ti == 4 && g.tw == 4) FN<true, 4, 4>(__VA_ARGS__);               \
      else if (g.ti == 6 && g.tw == 6) FN<true, 6, 6>(__VA_ARGS__);               \
      else if (g.ti == 8 && g.tw == 8) FN<true, 8, 8>(__VA_ARGS__);               \
      else if (g.ti == 10 && g.tw == 10) FN<true, 10, 10>(__VA_ARGS__);           \
      else if (g.ti == 12 && g.tw == 12) FN<true, 12, 12>(__VA_ARGS__);           \
      else if (g.ti == 14 && g.tw == 14) FN<true, 14, 14>(__VA_ARGS__);           \
      else if (g.ti == 16 && g.tw == 16) FN<true, 16, 16>(__VA_ARGS__);           \
      else return hipErrorInvalidValue;                                           \
    } else {                                                                      \
      if (g.ti == 1 && g.tw == 2) FN<false, 1, 2>(__VA_ARGS__);                   \
      else if (g.ti == 2 && g.tw == 2) FN<false, 2, 2>(__VA_ARGS__);              \
      else if (g.ti == 4 && g.tw == 4) FN<false, 4, 4>(__VA_ARGS__);              \
      else if (g.ti == 7 && g.tw == 7) FN<false, 7, 7>(__VA_ARGS__);              \
      else if (g.ti == 8 && g.tw == 8) FN<false, 8, 8>(__VA_ARGS__);              \
      else if (g.ti == 16 && g.tw == 16) FN<false, 16, 16>(__VA_ARGS__);          \
      else return hipErrorInvalidValue;                                           \
    }                                                                             \
  } while (0)

hipError_t launch_forward(const Geo& g, const float* params, const void* packF, const float* pbias,
                          const float* X, float* V, float* C, void* H, hipStream_t s) {
  FBSDE_DISPATCH(fwd_inst, g, params, packF, pbias, X, V, C, H, s);
  return hipGetLastError();
}

hipError_t launch_scan(const Geo& g, const double* y0, const float* C, const float* QN, const float* LN,
                       float* Y, float* LAM, double* part, int blocks, hipStream_t s) {
  if (g.N <= 16) k_scan<16><<<blocks, 64, 0, s>>>(g, y0, C, QN, LN, Y, LAM, part);
  else if (g.N <= 32) k_scan<32><<<blocks, 64, 0, s>>>(g, y0, C, QN, LN, Y, LAM, part);
  else if (g.N <= 64) k_scan<64><<<blocks, 64, 0, s>>>(g, y0, C, QN, LN, Y, LAM, part);
  else k_scan<0><<<blocks, 64, 0, s>>>(g, y0, C, QN, LN, Y, LAM, part);
  return hipGetLastError();
}

hipError_t launch_backward(const Geo& g, const void* packB, const float* V, const float* LAM,
                           const void* H, void* DZ, void* DH, hipStream_t s) {
  FBSDE_DISPATCH(bwd_inst, g, packB, V, LAM, H, DZ, DH, s);
  return hipGetLastError();
}

// Output tiles per side of a weight-gradient workgroup's block.  Past 8
// tiles a matrix spans several blocks, whose tile loops always run the full
// block: 7 or 8, whichever covers the (rows x cols + 1) matrix with fewer
// tile slots (d = 188, w = 198: 4 blocks of 7 x 7 instead of 4 of 8 x 8).
// Each tile's accumulation order does not depend on the block, so neither
// do the results.
int wgrad_block_tiles(const Geo& g) {
  const int rmax = g.d > g.w ? g.d : g.w;
  const int cmax = (g.d > g.w ? g.d : g.w) + 1;
  const int t = ((rmax > cmax ? rmax : cmax) + 15) / 16;
  if (t <= 8) return t <= 1 ? 1 : (t <= 2 ? 2 : (t <= 4 ? 4 : (t <= 7 ? 7 : 8)));
  auto slots = [&](int T) { return ((rmax + 16 * T - 1) / (16 * T)) * ((cmax + 16 * T - 1) / (16 * T)) * T * T; };
  return slots(7) < slots(8) ? 7 : 8;
}

template <bool BF, int T>
static void wgrad_inst(const Geo& g, const float* X, const void* H, const void* DZ, const void* DH, float* part,
                       int splits, long long chunk, hipStream_t s) {
  const int rmax = g.d > g.w ? g.d : g.w, cmax = rmax + 1;
  const unsigned groups = (unsigned)(((rmax + 16 * T - 1) / (16 * T)) * ((cmax + 16 * T - 1) / (16 * T)));
  const int n1 = g.n0 + launch_steps(g), nf = g.n0 > 1 ? g.n0 : 1;  // steps with a network: nf .. n1 - 1
  const unsigned jobs = (g.n0 == 0 ? 1u : 0u) + (unsigned)(n1 > nf ? n1 - nf : 0) * (unsigned)(g.L + 1);
  dim3 grid(jobs, groups, splits);
  k_wgrad<BF, T><<<grid, WG_THREADS, 0, s>>>(g, X, H, DZ, DH, part, chunk);
}

hipError_t launch_wgrad(const Geo& g, const float* X, const void* H, const void* DZ, const void* DH,
                        float* part, int splits, long long chunk, hipStream_t s) {
  const int T = wgrad_block_tiles(g);
#define WG_CASE(TT)                                                                  \
  if (T == TT) {                                                                     \
    if (g.bf16) wgrad_inst<true, TT>(g, X, H, DZ, DH, part, splits, chunk, s);       \
    else wgrad_inst<false, TT>(g, X, H, DZ, DH, part, splits, chunk, s);             \
    return hipGetLastError();                                                        \
  }
  WG_CASE(1) WG_CASE(2) WG_CASE(4) WG_CASE(7) WG_CASE(8)
#undef WG_CASE
  return hipErrorInvalidValue;
}

// The fused reverse kernels serve per-step MLPs of depth 1 or 2 whose bias
// columns fit the tiles (d + 1 <= 16 ti, w + 1 <= 16 tw) and whose
// transposed weights plus staged rows fit in LDS: fp32 tile shapes (1, 2),
// (2, 2), (4, 4), (7, 7); bf16 shapes (2, 2), (4, 4), (6, 6), (8, 8).
static bool rv_shape(int bf, int ti, int tw) {
  if (bf) return ti == tw && (ti == 2 || ti == 4 || ti == 6 || ti == 8);
  return (ti == 1 && tw == 2) || (ti == 2 && tw == 2) || (ti == 4 && tw == 4) || (ti == 7 && tw == 7);
}
static size_t reverse_lds_bytes(const Geo& g) {
  if (g.bf16) return (size_t)g.packb_step * 2 + rb_array_bytes(g.ti, g.tw, g.L);
  return (size_t)g.packb_step * 4 + (size_t)rv_arrays(g.L) * RV_KC * rv_lda(g.ti, g.tw) * 4;
}
bool reverse_fused_fits(const Geo& g) {
  return g.kind == 0 && g.lds == 2 && g.L >= 1 && g.L <= 2 && rv_shape(g.bf16, g.ti, g.tw) &&
         g.d + 1 <= 16 * g.ti && g.w + 1 <= 16 * g.tw && reverse_lds_bytes(g) <= kLdsLimit;
}

// Whether the fused kernel is the faster form: bf16 always (it moves half the
// bytes of the separate pair); fp32 when its (split, step) workgroups fit one
// wave over the CUs -- beyond that the pair's larger grids keep more of the
// chip busy (BSB d = 100: fused 188 vs 197 us at M = 4096, 381 vs 369 us at
// M = 8192, 2.96 vs 2.69 ms at M = 65536).
bool reverse_fused_preferred(const Geo& g, int splits) {
  return reverse_fused_fits(g) && (g.bf16 || (long long)splits * g.N <= num_cus());
}

template <bool BF, int TI, int TW, int L>
static void rev_inst(const Geo& g, const void* packB, const float* X, const float* V, const float* LAM,
                     const void* H, float* part, int splits, long long chunk, hipStream_t s) {
  const void* fn;
  if constexpr (BF) fn = reinterpret_cast<const void*>(k_reverse_bf<TI, TW, L>);
  else fn = reinterpret_cast<const void*>(k_reverse<TI, TW, L>);
  static bool attr = [fn] {
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit);
    return true;
  }();
  (void)attr;
  dim3 grid((unsigned)splits, (unsigned)launch_steps(g));
  if constexpr (BF)
    k_reverse_bf<TI, TW, L><<<grid, RV_THREADS, reverse_lds_bytes(g), s>>>(g, packB, X, V, LAM, H, part, chunk);
  else
    k_reverse<TI, TW, L><<<grid, RV_THREADS, reverse_lds_bytes(g), s>>>(g, packB, X, V, LAM, H, part, chunk);
}

hipError_t launch_reverse(const Geo& g, const void* packB, const float* X, const float* V, const float* LAM,
                          const void* H, float* part, int splits, long long chunk, hipStream_t s) {
  const long long kc = g.bf16 ? RB_KC : RV_KC;
  if (!reverse_fused_fits(g) || splits < 1 || chunk < kc || chunk % kc != 0 ||
      (long long)splits * chunk < g.M || (long long)(splits - 1) * chunk >= g.M)
    return hipErrorInvalidValue;
#define RV_CASE(BF_, TI_, TW_)                                                                    \
  if (g.bf16 == BF_ && g.ti == TI_ && g.tw == TW_) {                                              \
    if (g.L == 1) rev_inst<BF_, TI_, TW_, 1>(g, packB, X, V, LAM, H, part, splits, chunk, s);      \
    else rev_inst<BF_, TI_, TW_, 2>(g, packB, X, V, LAM, H, part, splits, chunk, s);               \
    return hipGetLastError();                                                                     \
  }
  RV_CASE(0, 1, 2) RV_CASE(0, 2, 2) RV_CASE(0, 4, 4) RV_CASE(0, 7, 7)
  RV_CASE(1, 2, 2) RV_CASE(1, 4, 4) RV_CASE(1, 6, 6) RV_CASE(1, 8, 8)
#undef RV_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_reduce(const Geo& g, const float* part, int splits, float* grad, double* scan_part,
                         int scan_blocks, double* loss, double* grad_y0, int* host_flag, hipStream_t s) {
  const unsigned nred = grid1((g.nparams + 3) / 4, 4096);
  k_reduce<<<nred + 1, 256, 0, s>>>(g.nparams, g.pstride, part, splits, grad, (int)nred, g.M, scan_part,
                                    scan_blocks, loss, grad_y0, host_flag);
  return hipGetLastError();
}

hipError_t launch_reduce_adam(const Geo& g, const float* part, int splits, float* grad, double* scan_part,
                              int scan_blocks, double* loss, double* grad_y0, int* host_flag, const AdamArgs& a,
                              hipStream_t s) {
  const unsigned nred = grid1((g.nparams + 3) / 4, 4096);
  k_reduce_adam<<<nred + 1, 256, 0, s>>>(g.nparams, g.pstride, part, splits, grad, (int)nred, g.M, scan_part,
                                         scan_blocks, loss, grad_y0, host_flag, a.p, a.m, a.v, a.y0, a.my0, a.vy0,
                                         (float)a.lr, a.t, a.t_dev, a.lr_y0, a.b1, a.b2, a.eps);
  return hipGetLastError();
}

hipError_t launch_loss_only(const Geo& g, double* scan_part, int scan_blocks, double* loss, int* host_flag,
                            hipStream_t s) {
  k_finalize<<<1, 64, 0, s>>>(g.M, scan_part, scan_blocks, loss, host_flag);
  return hipGetLastError();
}

hipError_t launch_adam(long long n, float* p, const float* gr, float* m, float* v, double* y0,
                       const double* gy0, double* my0, double* vy0, float lr, double t, const uint64_t* t_dev,
                       double lr_y0, double b1, double b2, double eps, hipStream_t s) {
  // one thread per 4 elements, so that no thread takes a second serial pass
  k_adam<<<grid1((n + 3) / 4, 8192), 256, 0, s>>>(n, p, gr, m, v, y0, gy0, my0, vy0, lr, t, t_dev, lr_y0, b1, b2,
                                                  eps);
  return hipGetLastError();
}

hipError_t launch_count(uint64_t* c, hipStream_t s) {
  k_count<<<1, 64, 0, s>>>(c);
  return hipGetLastError();
}

hipError_t launch_prolong(const Geo& coarse, const Geo& fine, const float* pc, float* pf, hipStream_t s) {
  k_prolong<<<grid1(fine.nparams, 8192), 256, 0, s>>>(fine.d, fine.pstep, coarse.N, fine.nparams, pc, pf);
  return hipGetLastError();
}

hipError_t launch_normals(const Geo& g, uint64_t seed, uint64_t iter, float* xi, hipStream_t s) {
  const long long total = (long long)g.N * g.M * (g.dp / 4);
  k_normals<<<grid1(total), 256, 0, s>>>(g, seed, iter, xi);
  return hipGetLastError();
}

hipError_t launch_gmean(const Geo& g, const float* QN, const float* LN, double* out, hipStream_t s) {
  k_gmean<<<1, 256, 0, s>>>(g, QN, LN, out);
  return hipGetLastError();
}

hipError_t launch_terminal_copy(const Geo& g, const float* X, const float* Y, float* xN, float* yN,
                                hipStream_t s) {
  k_terminal_copy<<<grid1((long long)g.M * g.d), 256, 0, s>>>(g, X, Y, xN, yN);
  return hipGetLastError();
}

}  // namespace fbsde
