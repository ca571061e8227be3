// Shared time-conditioned residual network (Sec. 3.1, residual block as a
// forward-Euler step with h = 1), evaluated on every (step, path) row:
//   h_0 = tanh(W_in [x; t] + b_in),  a_k = tanh(W_k h_{k-1} + b_k),
//   h_k = h_{k-1} + a_k (k = 1..B),  Z = W_o h_B + b_o.
// All products are bf16 MFMA GEMMs (v_mfma_f32_16x16x32_bf16) with fp32
// accumulation; the residual stream and the back-propagated delta are fp32,
// every GEMM operand is rounded to bf16 once.  Rows are processed in chunks
// of whole time steps; the reverse sweep recomputes the chunk's activations
// (activation checkpointing: only X_n and v_n are kept across the pass).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fbsde_internal.h"

namespace fbsde {
namespace rn {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int BM = 128, BN = 128, BK = 32;
constexpr int LDK = BK + 8;  // LDS row of 40 bf16 = 80 B: conflict-free 16-byte fragment reads

__device__ __forceinline__ uint32_t bfbits(float f) {  // round to nearest even
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ __forceinline__ float rbf(float f) { return __uint_as_float(bfbits(f) << 16); }
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ float fast_tanh(float x) {
  const float ax = fabsf(x);
  const float e = __builtin_amdgcn_exp2f(2.8853900817779268f * ax);
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

// ------------------------------------------------------------- operands
// Element (i, k) of a GEMM operand; i runs over the operand's rows (the
// output dimension it contributes), k over the reduction.
enum { ROWS = 0, TRANS = 1 };
struct Opnd {
  const void* base;
  long long ld;      // row stride of the stored matrix (elements)
  int rows;          // valid i
  int kmax;          // valid k
  int mode;          // ROWS: base[i*ld + k];  TRANS: base[k*ld + i]
  int f32;           // 1: fp32 storage (rounded to bf16 when staged)
  const float* scale;  // optional scale: per row i (ROWS) or per k (TRANS)
  int tcol;          // TRANS only: i == tcol -> t_n of row k (the time input), -1 none
  int onescol;       // TRANS only: i == onescol -> 1 (bias column), -1 none
  int n0, mp;        // row k of a chunk is (step n0 + k / mp, path k % mp)
  float dt;
};

__device__ __forceinline__ float ld_elem(const Opnd& o, long long idx) {
  return o.f32 ? reinterpret_cast<const float*>(o.base)[idx]
               : bf2f(reinterpret_cast<const uint16_t*>(o.base)[idx]);
}

// 8 consecutive k of row i (ROWS), as bf16 bits packed in a uint4
__device__ __forceinline__ uint4 load_row8(const Opnd& o, int i, int k) {
  float v[8];
  if (i < o.rows && k + 8 <= o.kmax) {
    const long long idx = (long long)i * o.ld + k;
    if (o.f32) {
      const f32x4 a = *reinterpret_cast<const f32x4*>(reinterpret_cast<const float*>(o.base) + idx);
      const f32x4 b = *reinterpret_cast<const f32x4*>(reinterpret_cast<const float*>(o.base) + idx + 4);
      v[0] = a[0]; v[1] = a[1]; v[2] = a[2]; v[3] = a[3]; v[4] = b[0]; v[5] = b[1]; v[6] = b[2]; v[7] = b[3];
    } else {
      return *reinterpret_cast<const uint4*>(reinterpret_cast<const uint16_t*>(o.base) + idx);
    }
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e)
      v[e] = (i < o.rows && k + e < o.kmax) ? ld_elem(o, (long long)i * o.ld + k + e) : 0.f;
  }
  if (o.scale && i < o.rows) {
    const float s = o.scale[i];
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] *= s;
  }
  uint4 u;
  u.x = bfbits(v[0]) | (bfbits(v[1]) << 16);
  u.y = bfbits(v[2]) | (bfbits(v[3]) << 16);
  u.z = bfbits(v[4]) | (bfbits(v[5]) << 16);
  u.w = bfbits(v[6]) | (bfbits(v[7]) << 16);
  return u;
}

// 8 consecutive i at reduction index k (TRANS), as floats
__device__ __forceinline__ void load_col8(const Opnd& o, int i, int k, float v[8]) {
  const bool kok = k < o.kmax;
  if (kok && i + 8 <= o.rows && i + 8 <= (o.tcol >= 0 ? o.tcol : o.rows)) {
    const long long idx = (long long)k * o.ld + i;
    if (o.f32) {
      const f32x4 a = *reinterpret_cast<const f32x4*>(reinterpret_cast<const float*>(o.base) + idx);
      const f32x4 b = *reinterpret_cast<const f32x4*>(reinterpret_cast<const float*>(o.base) + idx + 4);
      v[0] = a[0]; v[1] = a[1]; v[2] = a[2]; v[3] = a[3]; v[4] = b[0]; v[5] = b[1]; v[6] = b[2]; v[7] = b[3];
    } else {
      const uint4 u = *reinterpret_cast<const uint4*>(reinterpret_cast<const uint16_t*>(o.base) + idx);
      v[0] = __uint_as_float(u.x << 16); v[1] = __uint_as_float(u.x & 0xffff0000u);
      v[2] = __uint_as_float(u.y << 16); v[3] = __uint_as_float(u.y & 0xffff0000u);
      v[4] = __uint_as_float(u.z << 16); v[5] = __uint_as_float(u.z & 0xffff0000u);
      v[6] = __uint_as_float(u.w << 16); v[7] = __uint_as_float(u.w & 0xffff0000u);
    }
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int ii = i + e;
      float x = 0.f;
      if (kok) {
        if (ii == o.tcol) x = (float)(o.n0 + k / o.mp) * o.dt;
        else if (ii == o.onescol) x = 1.f;
        else if (ii < o.rows && (o.tcol < 0 || ii < o.tcol)) x = ld_elem(o, (long long)k * o.ld + ii);
      }
      v[e] = x;
    }
  }
  if (o.scale && kok) {
    const float s = o.scale[k];
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] *= s;
  }
}

// ------------------------------------------------------------- epilogues
enum { EPI_STORE = 0,      // out32[i][j] = acc + bias[j]
       EPI_TANH_IN = 1,    // h0 = tanh(acc + bias[j] + t(i) w_t[j]): h32, hb
       EPI_TANH_RES = 2,   // a = tanh(acc + bias[j]), h += a: h32 (in place), hb, ab
       EPI_BWD_FIRST = 3,  // delta = acc, g = delta (1 - a^2): d32, gb
       EPI_BWD_RES = 4,    // delta += acc, g = delta (1 - a^2): d32 (in place), gb
       EPI_ACC = 5 };      // weight-gradient partials: part[off(i, j)] += acc

struct Epi {
  int rows, cols;          // valid output extent (i < rows, j < cols)
  const float* bias;       // [cols]
  const float* wt;         // [cols] time-column weights (EPI_TANH_IN)
  int n0, mp;
  float dt;
  float* h32; long long ldh;      // fp32 residual stream / delta
  uint16_t* ob; long long ldb;    // bf16 output (hb or gb)
  uint16_t* ab; long long lda;    // bf16 activation out (EPI_TANH_RES) or in (EPI_BWD_*)
  float* out32; long long ldo;    // EPI_STORE
  float* part; long long base; int wcols;  // EPI_ACC: flat W[rows][wcols] then b[rows]; column wcols is the bias
};

template <int EPI>
__device__ __forceinline__ void epilogue(const Epi& E, int i, int j, float acc) {
  if (i >= E.rows || j >= E.cols) return;
  if constexpr (EPI == EPI_STORE) {
    E.out32[(long long)i * E.ldo + j] = acc + (E.bias ? E.bias[j] : 0.f);
  } else if constexpr (EPI == EPI_TANH_IN) {
    const float t = rbf((float)(E.n0 + i / E.mp) * E.dt);
    const float a = fast_tanh(acc + E.bias[j] + t * E.wt[j]);
    E.h32[(long long)i * E.ldh + j] = a;
    E.ob[(long long)i * E.ldb + j] = (uint16_t)bfbits(a);
  } else if constexpr (EPI == EPI_TANH_RES) {
    const float a = fast_tanh(acc + E.bias[j]);
    const long long p = (long long)i * E.ldh + j;
    const float h = E.h32[p] + a;
    E.h32[p] = h;
    E.ob[(long long)i * E.ldb + j] = (uint16_t)bfbits(h);
    E.ab[(long long)i * E.lda + j] = (uint16_t)bfbits(a);
  } else if constexpr (EPI == EPI_BWD_FIRST || EPI == EPI_BWD_RES) {
    const long long p = (long long)i * E.ldh + j;
    const float dlt = (EPI == EPI_BWD_RES) ? E.h32[p] + acc : acc;
    E.h32[p] = dlt;
    const float a = bf2f(E.ab[(long long)i * E.lda + j]);
    E.ob[(long long)i * E.ldb + j] = (uint16_t)bfbits(dlt * (1.f - a * a));
  } else {  // EPI_ACC
    const long long off = (j < E.wcols) ? E.base + (long long)i * E.wcols + j
                                        : E.base + (long long)E.rows * E.wcols + i;
    E.part[off] += acc;
  }
}

// ------------------------------------------------------------------ GEMM
// C[i][j] = sum_k A(i, k) B(j, k), i < M, j < N, k in [k0, k1); 128x128 tile per
// workgroup, 4 waves of 64x64 (4 x 4 MFMA tiles), K staged 32 at a time in
// double-buffered LDS ([row][k], 80-byte rows).  blockIdx.z selects a K
// split: split s covers [s*kchunk, (s+1)*kchunk) and adds into part + s*pstride.
template <int EPI>
__global__ __launch_bounds__(256) void k_gemm(Opnd A, Opnd B, Epi E, int Kdim, long long kchunk,
                                              long long pstride) {
  __shared__ __attribute__((aligned(16))) uint16_t sA[2][BM * LDK];
  __shared__ __attribute__((aligned(16))) uint16_t sB[2][BN * LDK];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wr = wv >> 1, wc = wv & 1;
  const int i0 = blockIdx.y * BM, j0 = blockIdx.x * BN;
  const long long ks = (long long)blockIdx.z * kchunk;
  const long long ke = min((long long)Kdim, ks + kchunk);
  Epi Ez = E;
  if constexpr (EPI == EPI_ACC) Ez.part = E.part + (long long)blockIdx.z * pstride;

  f32x4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

  // staging: 512 units of 8 elements per operand tile, two per thread
  auto stage = [&](int buf, long long kt) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int unit = tid + 256 * u;
      // A
      if (A.mode == ROWS) {
        const int r = unit >> 2, kk = (unit & 3) * 8;
        const uint4 v = load_row8(A, i0 + r, (int)(kt + kk));
        *reinterpret_cast<uint4*>(&sA[buf][r * LDK + kk]) = v;
      } else {
        const int kk = unit >> 4, r = (unit & 15) * 8;
        float v[8];
        load_col8(A, i0 + r, (int)(kt + kk), v);
#pragma unroll
        for (int e = 0; e < 8; ++e) sA[buf][(r + e) * LDK + kk] = (uint16_t)bfbits(v[e]);
      }
      // B
      if (B.mode == ROWS) {
        const int r = unit >> 2, kk = (unit & 3) * 8;
        const uint4 v = load_row8(B, j0 + r, (int)(kt + kk));
        *reinterpret_cast<uint4*>(&sB[buf][r * LDK + kk]) = v;
      } else {
        const int kk = unit >> 4, r = (unit & 15) * 8;
        float v[8];
        load_col8(B, j0 + r, (int)(kt + kk), v);
#pragma unroll
        for (int e = 0; e < 8; ++e) sB[buf][(r + e) * LDK + kk] = (uint16_t)bfbits(v[e]);
      }
    }
  };

  int buf = 0;
  if (ks < ke) stage(0, ks);
  __syncthreads();
  for (long long kt = ks; kt < ke; kt += BK) {
    if (kt + BK < ke) stage(buf ^ 1, kt + BK);  // next tile into the other buffer
    bf16x8 fa[4], fb[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const uint4 u = *reinterpret_cast<const uint4*>(&sA[buf][(wr * 64 + 16 * a + (lane & 15)) * LDK + 8 * (lane >> 4)]);
      fa[a] = __builtin_bit_cast(bf16x8, u32x4{u.x, u.y, u.z, u.w});
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const uint4 u = *reinterpret_cast<const uint4*>(&sB[buf][(wc * 64 + 16 * b + (lane & 15)) * LDK + 8 * (lane >> 4)]);
      fb[b] = __builtin_bit_cast(bf16x8, u32x4{u.x, u.y, u.z, u.w});
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a], fb[b], acc[a][b], 0, 0, 0);
    __syncthreads();
    buf ^= 1;
  }
  // D layout: lane holds rows 4*(lane/16)+r, column lane%16 of each 16x16 tile
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wr * 64 + 16 * a + 4 * (lane >> 4) + r;
        const int j = j0 + wc * 64 + 16 * b + (lane & 15);
        epilogue<EPI>(Ez, i, j, acc[a][b][r]);
      }
}

// ------------------------------------------------------ row epilogue
// Per row r = (n, m) of a chunk: c_n = Z.s + dt (Z-part of phi), v_n = s + dt phi_z,
// with one wave per row (lanes stride over the d columns, fixed-order reduction).
__global__ __launch_bounds__(256) void k_row_epilogue(Geo g, int n0, int rows, const float* __restrict__ Z,
                                                      long long ldz, const float* __restrict__ X,
                                                      float* __restrict__ V, float* __restrict__ C) {
  const int lane = threadIdx.x & 63;
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= rows) return;
  const int n = n0 + r / g.M, m = r % g.M;
  const size_t row = ((size_t)n * g.M + m) * g.dp;
  float cz = 0.f, cx = 0.f;
  for (int i = lane; i < g.d; i += 64) {
    const float z = Z[(long long)r * ldz + i];
    const float s = V[row + i];
    const float x = X[row + i];
    cz += z * s;
    float v = s;
    if (g.drv == 0) {  // BSB: phi = r (y - z.x)
      cx += z * x;
      v = s - g.drv_p0 * g.dt * x;
    } else if (g.drv == 1) {  // HJB: phi = lam |z|^2
      cx += z * z;
      v = s + 2.f * g.drv_p0 * g.dt * z;
    }
    V[row + i] = v;
  }
  float c = cz;
  if (g.drv == 0) c -= g.dt * g.drv_p0 * cx;
  else if (g.drv == 1) c += g.dt * g.drv_p0 * cx;
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
  if (lane == 0) C[(size_t)n * g.M + m] = c;
}

// ------------------------------------------------------------ packing
// bf16 copies of the weights (and transposes for the reverse sweep), fp32
// biases and the time column.  Layout of `pk` (bf16, element offsets):
//   Win[w][dq] | W_k[w][w] (k = 1..B) | Wo[d][w] | W_k^T[w][w] (k = 1..B) | Wo^T[w][dq]
// with dq = d rounded up to 8; `pf` (fp32): w_t[w] | b_in[w] | b_k[w] (k=1..B) | b_o[d]
__global__ __launch_bounds__(256) void k_pack_resnet(Geo g, const float* __restrict__ P, uint16_t* __restrict__ pk,
                                                     float* __restrict__ pf) {
  const int d = g.d, w = g.w, B = g.L, dq = (d + 7) / 8 * 8;
  const long long szin = (long long)w * dq, szh = (long long)w * w, szo = (long long)d * w, szot = (long long)w * dq;
  const long long total = szin + B * szh + szo + B * szh + szot;
  const long long offin = 0, offbin = (long long)w * (d + 1), offk = offbin + w;
  const long long offo = offk + (long long)B * ((long long)w * w + w);
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < total; e += (long long)gridDim.x * 256) {
    float v = 0.f;
    long long q = e;
    if (q < szin) {
      const int o = (int)(q / dq), i = (int)(q % dq);
      v = i < d ? P[offin + (long long)o * (d + 1) + i] : 0.f;
    } else if ((q -= szin) < B * szh) {
      const int k = (int)(q / szh);
      v = P[offk + (long long)k * ((long long)w * w + w) + q % szh];
    } else if ((q -= B * szh) < szo) {
      v = P[offo + q];
    } else if ((q -= szo) < B * szh) {
      const int k = (int)(q / szh);
      const long long r = q % szh;
      const int row = (int)(r / w), col = (int)(r % w);  // W_k^T[row][col] = W_k[col][row]
      v = P[offk + (long long)k * ((long long)w * w + w) + (long long)col * w + row];
    } else {
      q -= B * szh;
      const int row = (int)(q / dq), col = (int)(q % dq);  // Wo^T[row < w][col < d] = Wo[col][row]
      v = col < d ? P[offo + (long long)col * w + row] : 0.f;
    }
    pk[e] = (uint16_t)bfbits(v);
  }
  const long long nf = 2LL * w + (long long)B * w + d;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < nf; e += (long long)gridDim.x * 256) {
    float v;
    if (e < w) v = rbf(P[offin + e * (d + 1) + d]);           // time column, bf16 like every W entry
    else if (e < 2LL * w) v = P[offbin + (e - w)];
    else if (e < 2LL * w + (long long)B * w) {
      const long long q = e - 2LL * w;
      v = P[offk + (q / w) * ((long long)w * w + w) + (long long)w * w + q % w];
    } else {
      v = P[offo + (long long)d * w + (e - 2LL * w - (long long)B * w)];
    }
    pf[e] = v;
  }
}

__global__ __launch_bounds__(256) void k_fill(float* __restrict__ p, long long n) {
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < n; e += (long long)gridDim.x * 256) p[e] = 0.f;
}

static unsigned grid1(long long n, long long cap = 65536) {
  long long b = (n + 255) / 256;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

template <int EPI>
static hipError_t gemm(const Opnd& A, const Opnd& B, const Epi& E, int Mrows, int Ncols, int Kdim, int splits,
                       long long pstride, hipStream_t s) {
  long long kchunk = Kdim;
  if (splits > 1) kchunk = ((long long)Kdim + splits - 1) / splits, kchunk = (kchunk + BK - 1) / BK * BK;
  const int z = (int)(((long long)Kdim + kchunk - 1) / kchunk);
  dim3 grid((unsigned)((Ncols + BN - 1) / BN), (unsigned)((Mrows + BM - 1) / BM), (unsigned)z);
  k_gemm<EPI><<<grid, 256, 0, s>>>(A, B, E, Kdim, kchunk, pstride);
  return hipGetLastError();
}

}  // namespace rn

// ===================================================== host sequencing
using namespace rn;

static Opnd opnd(const void* base, long long ld, int rows, int kmax, int mode, int f32) {
  Opnd o;
  o.base = base; o.ld = ld; o.rows = rows; o.kmax = kmax; o.mode = mode; o.f32 = f32;
  o.scale = nullptr; o.tcol = -1; o.onescol = -1; o.n0 = 0; o.mp = 1; o.dt = 0.f;
  return o;
}
static Epi epi0(int rows, int cols) {
  Epi e = {};
  e.rows = rows; e.cols = cols;
  return e;
}

ResnetLayout resnet_layout(const Geo& g) {
  ResnetLayout L;
  const long long d = g.d, w = g.w, B = g.L, dq = (d + 7) / 8 * 8;
  L.dq = (int)dq;
  L.pk_elems = w * dq + B * w * w + d * w + B * w * w + w * dq;
  L.pf_elems = 2 * w + B * w + d;
  L.rows = (long long)g.rn_chunk * g.M;
  return L;
}

// offsets inside the packed bf16 buffer
static inline const uint16_t* pk_win(const Geo&, const ResnetLayout&, const uint16_t* pk) { return pk; }
static inline const uint16_t* pk_wk(const Geo& g, const ResnetLayout& L, const uint16_t* pk, int k) {
  return pk + (long long)g.w * L.dq + (long long)(k - 1) * g.w * g.w;
}
static inline const uint16_t* pk_wo(const Geo& g, const ResnetLayout& L, const uint16_t* pk) {
  return pk + (long long)g.w * L.dq + (long long)g.L * g.w * g.w;
}
static inline const uint16_t* pk_wkt(const Geo& g, const ResnetLayout& L, const uint16_t* pk, int k) {
  return pk_wo(g, L, pk) + (long long)g.d * g.w + (long long)(k - 1) * g.w * g.w;
}
static inline const uint16_t* pk_wot(const Geo& g, const ResnetLayout& L, const uint16_t* pk) {
  return pk_wkt(g, L, pk, g.L + 1);
}

hipError_t resnet_pack(const Geo& g, const float* params, uint16_t* pk, float* pf, hipStream_t s) {
  const ResnetLayout L = resnet_layout(g);
  k_pack_resnet<<<grid1(L.pk_elems, 16384), 256, 0, s>>>(g, params, pk, pf);
  return hipGetLastError();
}

// forward of the rows of steps [n0, n0 + ns): activations into the chunk buffers
static hipError_t chunk_forward(const Geo& g, const ResnetLayout& L, const ResnetBufs& R, int n0, int ns,
                                const float* X, bool with_output, hipStream_t s) {
  const int rows = ns * g.M, w = g.w, d = g.d, B = g.L;
  const float* wt = R.pf;
  const float* bin = R.pf + w;
  hipError_t e;
  {  // h0 = tanh(W_in [x; t] + b_in)
    Opnd A = opnd(X + (size_t)n0 * g.M * g.dp, g.dp, rows, d, ROWS, 1);
    Opnd Bw = opnd(pk_win(g, L, R.pk), L.dq, w, d, ROWS, 0);
    Epi E = epi0(rows, w);
    E.bias = bin; E.wt = wt; E.n0 = n0; E.mp = g.M; E.dt = g.dt;
    E.h32 = R.h32; E.ldh = w; E.ob = R.hb; E.ldb = w;
    if ((e = gemm<EPI_TANH_IN>(A, Bw, E, rows, w, d, 1, 0, s)) != hipSuccess) return e;
  }
  for (int k = 1; k <= B; ++k) {  // a_k = tanh(W_k h_{k-1} + b_k), h_k = h_{k-1} + a_k
    Opnd A = opnd(R.hb + (size_t)(k - 1) * L.rows * w, w, rows, w, ROWS, 0);
    Opnd Bw = opnd(pk_wk(g, L, R.pk, k), w, w, w, ROWS, 0);
    Epi E = epi0(rows, w);
    E.bias = R.pf + 2 * w + (size_t)(k - 1) * w;
    E.h32 = R.h32; E.ldh = w;
    E.ob = R.hb + (size_t)k * L.rows * w; E.ldb = w;
    E.ab = R.ab + (size_t)(k - 1) * L.rows * w; E.lda = w;
    if ((e = gemm<EPI_TANH_RES>(A, Bw, E, rows, w, w, 1, 0, s)) != hipSuccess) return e;
  }
  if (with_output) {  // Z = W_o h_B + b_o
    Opnd A = opnd(R.hb + (size_t)B * L.rows * w, w, rows, w, ROWS, 0);
    Opnd Bw = opnd(pk_wo(g, L, R.pk), w, d, w, ROWS, 0);
    Epi E = epi0(rows, d);
    E.bias = R.pf + 2 * w + (size_t)B * w;
    E.out32 = R.z; E.ldo = L.dq;
    if ((e = gemm<EPI_STORE>(A, Bw, E, rows, d, w, 1, 0, s)) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t resnet_forward(const Geo& g, const ResnetBufs& R, const float* X, float* V, float* C, hipStream_t s) {
  const ResnetLayout L = resnet_layout(g);
  hipError_t e;
  for (int n0 = 0; n0 < g.N; n0 += g.rn_chunk) {
    const int ns = min(g.rn_chunk, g.N - n0);
    if ((e = chunk_forward(g, L, R, n0, ns, X, true, s)) != hipSuccess) return e;
    const int rows = ns * g.M;
    k_row_epilogue<<<(unsigned)((rows + 3) / 4), 256, 0, s>>>(g, n0, rows, R.z, L.dq, X, V, C);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

// Reverse sweep of every chunk (recomputing its activations); weight
// gradients accumulate over chunks into `splits` partial buffers of the flat
// parameter layout (each owned by one K split of each GEMM: deterministic).
hipError_t resnet_backward(const Geo& g, const ResnetBufs& R, const float* X, const float* V, const float* LAM,
                           float* part, int splits, hipStream_t s) {
  const ResnetLayout L = resnet_layout(g);
  const int w = g.w, d = g.d, B = g.L;
  const long long offbin = (long long)w * (d + 1), offk = offbin + w;
  const long long offo = offk + (long long)B * ((long long)w * w + w);
  hipError_t e;
  k_fill<<<grid1((long long)splits * g.nparams, 16384), 256, 0, s>>>(part, (long long)splits * g.nparams);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  for (int n0 = 0; n0 < g.N; n0 += g.rn_chunk) {
    const int ns = min(g.rn_chunk, g.N - n0);
    const int rows = ns * g.M;
    if ((e = chunk_forward(g, L, R, n0, ns, X, false, s)) != hipSuccess) return e;
    const float* Vc = V + (size_t)n0 * g.M * g.dp;
    const float* lam = LAM + (size_t)n0 * g.M;  // lambda_{n+1} of every row
    uint16_t* gcur = R.gb;
    uint16_t* gnext = R.gb + (size_t)L.rows * w;
    {  // delta_B = W_o^T zeta, zeta = lambda v;  g_B = delta_B (1 - a_B^2)
      Opnd A = opnd(Vc, g.dp, rows, d, ROWS, 1);
      A.scale = lam;
      Opnd Bw = opnd(pk_wot(g, L, R.pk), L.dq, w, d, ROWS, 0);
      Epi E = epi0(rows, w);
      E.h32 = R.d32; E.ldh = w; E.ob = gcur; E.ldb = w;
      E.ab = R.ab + (size_t)(B - 1) * L.rows * w; E.lda = w;
      if ((e = gemm<EPI_BWD_FIRST>(A, Bw, E, rows, w, d, 1, 0, s)) != hipSuccess) return e;
    }
    {  // dW_o += zeta^T h_B, db_o += sum zeta
      Opnd A = opnd(Vc, g.dp, d, rows, TRANS, 1);
      A.scale = lam;
      Opnd Bw = opnd(R.hb + (size_t)B * L.rows * w, w, w, rows, TRANS, 0);
      Bw.onescol = w;
      Epi E = epi0(d, w + 1);
      E.part = part; E.base = offo; E.wcols = w;
      if ((e = gemm<EPI_ACC>(A, Bw, E, d, w + 1, rows, splits, g.nparams, s)) != hipSuccess) return e;
    }
    for (int k = B; k >= 1; --k) {
      {  // dW_k += g_k^T h_{k-1}, db_k += sum g_k
        Opnd A = opnd(gcur, w, w, rows, TRANS, 0);
        Opnd Bw = opnd(R.hb + (size_t)(k - 1) * L.rows * w, w, w, rows, TRANS, 0);
        Bw.onescol = w;
        Epi E = epi0(w, w + 1);
        E.part = part; E.base = offk + (long long)(k - 1) * ((long long)w * w + w); E.wcols = w;
        if ((e = gemm<EPI_ACC>(A, Bw, E, w, w + 1, rows, splits, g.nparams, s)) != hipSuccess) return e;
      }
      {  // delta_{k-1} = delta_k + W_k^T g_k;  g_{k-1} = delta_{k-1} (1 - a_{k-1}^2), a_0 := h_0
        Opnd A = opnd(gcur, w, rows, w, ROWS, 0);
        Opnd Bw = opnd(pk_wkt(g, L, R.pk, k), w, w, w, ROWS, 0);
        Epi E = epi0(rows, w);
        E.h32 = R.d32; E.ldh = w; E.ob = gnext; E.ldb = w;
        E.ab = (k >= 2) ? R.ab + (size_t)(k - 2) * L.rows * w : R.hb;
        E.lda = w;
        if ((e = gemm<EPI_BWD_RES>(A, Bw, E, rows, w, w, 1, 0, s)) != hipSuccess) return e;
        uint16_t* t = gcur; gcur = gnext; gnext = t;
      }
    }
    {  // dW_in += g_0^T [x; t], db_in += sum g_0
      Opnd A = opnd(gcur, w, w, rows, TRANS, 0);
      Opnd Bx = opnd(X + (size_t)n0 * g.M * g.dp, g.dp, d, rows, TRANS, 1);
      Bx.tcol = d; Bx.onescol = d + 1; Bx.n0 = n0; Bx.mp = g.M; Bx.dt = g.dt;
      Epi E = epi0(w, d + 2);
      E.part = part; E.base = 0; E.wcols = d + 1;
      if ((e = gemm<EPI_ACC>(A, Bx, E, w, d + 2, rows, splits, g.nparams, s)) != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

}  // namespace fbsde
