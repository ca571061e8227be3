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

#include <type_traits>

#include "fbsde_internal.h"

namespace fbsde {
namespace rn {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int BK = 32;
constexpr int LDK = BK;  // 64-byte slab rows, 16-byte groups XOR-swizzled (slab_off)

// Element offset of the 16-byte group g (k = 8g .. 8g + 7) of slab row `row`:
// the group index is XORed with bits 1-2 of the row, so that both the
// staging writes (2 rows x 4 groups per 8 lanes) and the fragment reads (8
// consecutive rows, one group per 8 lanes) touch 8 distinct 16-byte bank
// groups: no LDS bank conflicts on either side.
__device__ __forceinline__ int slab_off(int row, int g) { return row * LDK + 8 * (g ^ ((row >> 1) & 3)); }
// wave tile of the row-streaming GEMMs (16 RN_TM x 16 RN_TN) and waves per SIMD
#ifndef RN_TM
#define RN_TM 8
#endif
#ifndef RN_TN
#define RN_TN 4
#endif
#ifndef RN_WPE
#define RN_WPE 2
#endif
// waves of a workgroup along j (2 along i)
#ifndef RN_WJ
#define RN_WJ 4
#endif
// register sets of slabs in flight (1 or 2)
#ifndef RN_PF
#define RN_PF 2
#endif  // LDS row of 40 bf16 = 80 B: conflict-free 16-byte fragment reads

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

// ------------------------------------------------------------------ GEMM
// C[i][j] = sum_k A[i][k] B[j][k], both operands bf16 and k-contiguous (row
// i of A and row j of B are runs of the reduction index).
struct Gm {
  const uint16_t* a; long long lda; int arows;
  const uint16_t* b; long long ldb; int brows;
  int K;                 // valid reduction length
  long long kchunk;      // reduction range of one split (multiple of BK)
  int ti, tj, ts;        // tiles over i, over j, and reduction splits
  long long pstride;     // EPI_ACC: floats between the partial buffers of two splits
};

// ------------------------------------------------------------- epilogues
enum { EPI_ROW = 0,        // Z = acc + bias[j] consumed at once: v (in place of s) and per-row partial sums
       EPI_TANH_IN = 1,    // h0 = tanh(acc + bias[j] + t(i) w_t[j]): h32, hb (+ hT)
       EPI_TANH_RES = 2,   // a = tanh(acc + bias[j]), h += a: h32 (in place), hb (+ ab, hT)
       EPI_BWD_FIRST = 3,  // delta = acc, g = delta (1 - a^2): d32, gb, gT
       EPI_BWD_RES = 4,    // delta += acc, g = delta (1 - a^2): d32 (in place), gb, gT
       EPI_ACC = 5 };      // weight-gradient partials: part[base + i*wcols + j] += acc, bias from A's rows

struct Epi {
  int rows, cols;          // valid output extent (i < rows, j < cols)
  const float* bias;       // [cols]
  const float* wt;         // [cols] time-column weights (EPI_TANH_IN)
  int n0, mp;              // row i of a chunk is (step n0 + i / mp, path i % mp)
  float dt;
  float* h32; long long ldh;      // fp32 residual stream / delta [i][j]
  uint16_t* ob; long long ldb;    // bf16 output [i][j] (hb or gb)
  uint16_t* ab; long long lda;    // bf16 activation, out (EPI_TANH_RES, optional) or in (EPI_BWD_*)
  float* part; long long base; int wcols;  // EPI_ACC: W[rows][wcols] at base, then the bias b[rows]
  // EPI_ROW: row i of the chunk is row i of sv (s_n in, v_n out) and of x (row stride ldv); its two
  // partial sums over the tile's columns go to rp[(j-tile) * 2 * rows + {0, rows} + i]
  float* sv; const float* x; long long ldv; float* rp;
  int drv; float p0;
};

__device__ __forceinline__ uint2 pack4(float a, float b, float c, float d) {
  return uint2{bfbits(a) | (bfbits(b) << 16), bfbits(c) | (bfbits(d) << 16)};
}

// Epilogue of a wave's (16 TM) x (16 TN) tile: lane l holds, for each MFMA
// tile (a, b), row i = i0w + 16 a + l % 16 and columns j = j0w + 16 b +
// 4 (l / 16) + 0..3.  Everything a row block a reads from memory (residual
// stream or delta, activations, weight-gradient partials) is loaded one block
// ahead, so that its latency overlaps the arithmetic and stores of block
// a - 1 instead of being waited for once per 4 columns; biases are loaded
// once.  The residual-stream epilogues (EPI_TANH_*, EPI_BWD_*) have cols = w,
// a multiple of 8, so a run of 4 columns is either wholly valid or wholly
// past cols.  Loads of rows past `rows` and of columns past `cols` read a
// clamped valid element; nothing is stored for them.
template <int EPI, int TM, int TN>
__device__ __forceinline__ void epilogue_tile(const Epi& E, const f32x4 (&acc)[TM][TN], int i0w, int j0w, int lane,
                                              float* red) {
  const int jl = 4 * (lane >> 4);
  if constexpr (EPI == EPI_ACC) {
    // partial[i][j] += acc: 4 TN scalar read-modify-writes per row block
    float pv[2][TN][4];
    auto ld = [&](int a, float (&v)[TN][4]) {
      const int i = min(i0w + 16 * a + (lane & 15), E.rows - 1);
      const float* p = E.part + E.base + (long long)i * E.wcols;
#pragma unroll
      for (int b = 0; b < TN; ++b)
#pragma unroll
        for (int e = 0; e < 4; ++e) v[b][e] = p[min(j0w + 16 * b + jl + e, E.cols - 1)];
    };
    ld(0, pv[0]);
#pragma unroll
    for (int a = 0; a < TM; ++a) {
      if (a + 1 < TM) ld(a + 1, pv[(a + 1) & 1]);
      const int i = i0w + 16 * a + (lane & 15);
      if (i < E.rows) {
        float* p = E.part + E.base + (long long)i * E.wcols;
#pragma unroll
        for (int b = 0; b < TN; ++b)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int j = j0w + 16 * b + jl + e;
            if (j < E.cols) p[j] = pv[a & 1][b][e] + acc[a][b][e];
          }
      }
    }
  } else if constexpr (EPI == EPI_ROW) {
    // Z = acc + b_o, then per (row, column) of the chunk the driver's Z-dependent terms: v = s + dt phi_z
    // and the row sums of z s and of z x (BSB: phi = r (y - z.x)) or z z (HJB: phi = lam |z|^2).  The
    // wave's sums over its 16 columns of each row go to `red` (LDS) for the workgroup's reduction.
    float bz[TN][4];
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) bz[b][e] = E.bias[min(j0w + 16 * b + jl + e, E.cols - 1)];
    f32x4 sv[2][TN], xv[2][TN];
    auto ld = [&](int a, f32x4 (&sr)[TN], f32x4 (&xr)[TN]) {
      const int i = min(i0w + 16 * a + (lane & 15), E.rows - 1);
#pragma unroll
      for (int b = 0; b < TN; ++b) {
        const int jc = min(j0w + 16 * b + jl, (int)E.ldv - 4);
        sr[b] = *reinterpret_cast<const f32x4*>(E.sv + (long long)i * E.ldv + jc);
        xr[b] = *reinterpret_cast<const f32x4*>(E.x + (long long)i * E.ldv + jc);
      }
    };
    ld(0, sv[0], xv[0]);
    const float hz = E.p0 * E.dt, hz2 = 2.f * E.p0 * E.dt;
#pragma unroll
    for (int a = 0; a < TM; ++a) {
      if (a + 1 < TM) ld(a + 1, sv[(a + 1) & 1], xv[(a + 1) & 1]);
      const int i = i0w + 16 * a + (lane & 15);
      float cz = 0.f, cx = 0.f;
#pragma unroll
      for (int b = 0; b < TN; ++b) {
        const int j = j0w + 16 * b + jl;
        const f32x4 sr = sv[a & 1][b], xr = xv[a & 1][b];
        float v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const bool ok = j + e < E.cols;
          const float z = acc[a][b][e] + bz[b][e];
          v[e] = sr[e];
          if (E.drv == 0) v[e] = sr[e] - hz * xr[e];
          else if (E.drv == 1) v[e] = sr[e] + hz2 * z;
          if (!ok) v[e] = sr[e];
          cz += ok ? z * sr[e] : 0.f;
          cx += ok ? (E.drv == 1 ? z * z : z * xr[e]) : 0.f;
        }
        if (i < E.rows && j < E.cols)
          *reinterpret_cast<f32x4*>(E.sv + (long long)i * E.ldv + j) = f32x4{v[0], v[1], v[2], v[3]};
      }
      // the 4 lanes of row i (lane % 16) sum their columns; lane < 16 keeps the wave's row sums
      cz += __shfl_xor(cz, 16);
      cx += __shfl_xor(cx, 16);
      cz += __shfl_xor(cz, 32);
      cx += __shfl_xor(cx, 32);
      if (lane < 16) {
        red[2 * (16 * a + lane)] = cz;
        red[2 * (16 * a + lane) + 1] = cx;
      }
    }
  } else {
    constexpr bool HIN = (EPI == EPI_TANH_RES || EPI == EPI_BWD_RES);   // reads the stream / delta
    constexpr bool AIN = (EPI == EPI_BWD_FIRST || EPI == EPI_BWD_RES);  // reads the activation
    constexpr bool BIAS = (EPI == EPI_TANH_IN || EPI == EPI_TANH_RES);
    f32x4 bz[TN], wz[TN];
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      const int jc = min(j0w + 16 * b + jl, E.cols - 4);
      if constexpr (BIAS) bz[b] = *reinterpret_cast<const f32x4*>(E.bias + jc);
      if constexpr (EPI == EPI_TANH_IN) wz[b] = *reinterpret_cast<const f32x4*>(E.wt + jc);
    }
    f32x4 hv[2][TN];
    uint2 av[2][TN];
    auto ld = [&](int a, f32x4 (&h)[TN], uint2 (&v)[TN]) {
      const int i = min(i0w + 16 * a + (lane & 15), E.rows - 1);
#pragma unroll
      for (int b = 0; b < TN; ++b) {
        const int jc = min(j0w + 16 * b + jl, E.cols - 4);
        if constexpr (HIN) h[b] = *reinterpret_cast<const f32x4*>(E.h32 + (long long)i * E.ldh + jc);
        if constexpr (AIN) v[b] = *reinterpret_cast<const uint2*>(E.ab + (long long)i * E.lda + jc);
      }
    };
    ld(0, hv[0], av[0]);
#pragma unroll
    for (int a = 0; a < TM; ++a) {
      if (a + 1 < TM) ld(a + 1, hv[(a + 1) & 1], av[(a + 1) & 1]);
      const int i = i0w + 16 * a + (lane & 15);
      float t = 0.f;
      if constexpr (EPI == EPI_TANH_IN) t = rbf((float)(E.n0 + i / E.mp) * E.dt);
#pragma unroll
      for (int b = 0; b < TN; ++b) {
        const int j = j0w + 16 * b + jl;
        const f32x4 h = hv[a & 1][b];
        const uint2 u = av[a & 1][b];
        const float avf[4] = {__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xffff0000u),
                              __uint_as_float(u.y << 16), __uint_as_float(u.y & 0xffff0000u)};
        float hout[4], gout[4], aout[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if constexpr (EPI == EPI_TANH_IN) {
            const float x = fast_tanh(acc[a][b][e] + bz[b][e] + t * wz[b][e]);
            hout[e] = x; gout[e] = x;
          } else if constexpr (EPI == EPI_TANH_RES) {
            const float x = fast_tanh(acc[a][b][e] + bz[b][e]);
            aout[e] = x;
            hout[e] = h[e] + x; gout[e] = hout[e];
          } else {  // EPI_BWD_FIRST / EPI_BWD_RES
            const float dl = HIN ? h[e] + acc[a][b][e] : acc[a][b][e];
            hout[e] = dl;
            gout[e] = dl * (1.f - avf[e] * avf[e]);
          }
        }
        if (i < E.rows && j < E.cols) {
          *reinterpret_cast<f32x4*>(E.h32 + (long long)i * E.ldh + j) = f32x4{hout[0], hout[1], hout[2], hout[3]};
          *reinterpret_cast<uint2*>(E.ob + (long long)i * E.ldb + j) = pack4(gout[0], gout[1], gout[2], gout[3]);
          if constexpr (EPI == EPI_TANH_RES)
            if (E.ab) *reinterpret_cast<uint2*>(E.ab + (long long)i * E.lda + j) = pack4(aout[0], aout[1], aout[2], aout[3]);
        }
      }
    }
  }
}

// ------------------------------------------------------------------ GEMM
// Workgroup tile (32 TM) x (16 TN WJ): 2 x WJ waves, each (16 TM) x (16 TN)
// as TM x TN MFMA 16x16x32 tiles.  The reduction is staged BK at a time in
// two LDS buffers: the global loads of slab s + 2 are in flight while slab s
// is multiplied.  The MFMA takes the B fragment as its first operand, so
// every lane ends up holding four consecutive output columns of one row
// (vector epilogue stores).  Tiles are ordered so that the j-tiles of one
// (split, i-tile) are dispatched to the same XCD and share the A slab in its
// L2.
//
// Operand forms.  KT = false: A[i][k] and B[j][k] are k-contiguous (row i of
// A is a run of the reduction index); slab rows of 64 bytes, swizzled.
// KT = true (the weight gradients, whose reduction runs over the rows of a
// chunk): A[k][i] and B[k][j] are the row-major activations themselves, and
// the slab keeps that [k][i] layout; the MFMA fragments (8 consecutive k of
// one i per lane) come from two transposed LDS reads (ds_read_b64_tr_b16):
// within each 16-lane group, lanes 4e..4e+3 point at slab row 8g + 4h + e,
// columns 4q..4q+3 (q = lane % 4), and lane j of the group receives column j
// of those four rows.
#ifndef RN_KT_SWZ
#define RN_KT_SWZ 1
#endif
// [k][i] slab rows: unpadded with the 16-element blocks of row k XOR-swizzled
// by kt_swz(k), or padded by KT_PAD elements
constexpr int KT_PAD = RN_KT_SWZ ? 0 : 16;
__device__ __forceinline__ int kt_swz(int k) { return RN_KT_SWZ ? 16 * ((k & 3) | (((k >> 3) & 1) << 2)) : 0; }

typedef short v4s __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) v4s lds_v4s;
__device__ __forceinline__ u32x4 tr_frag(const uint16_t* slab, int ld, int col0, int lane) {
  const int g = lane >> 4, j = lane & 15;
  const int k = 8 * g + (j >> 2);  // rows k and k + 4 share their swizzle
  uint16_t* p = const_cast<uint16_t*>(slab) + k * ld + (col0 ^ kt_swz(k)) + 4 * (j & 3);
  const v4s lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s*)p);
  const v4s hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s*)(p + 4 * ld));
  const uint2 l = __builtin_bit_cast(uint2, lo), h = __builtin_bit_cast(uint2, hi);
  return u32x4{l.x, l.y, h.x, h.y};
}

template <int EPI, int TM, int TN, int WJ, bool KT>
__global__ __launch_bounds__(128 * WJ) __attribute__((amdgpu_waves_per_eu(RN_WPE))) void k_gemm(Gm G, Epi E) {
  static_assert(!KT || EPI == EPI_ACC, "k-major operands are the weight-gradient form");
  static_assert(!KT || !RN_KT_SWZ || (16 * TM * 2 >= 128 && 16 * TN * WJ >= 128),
                "the [k][i] slab swizzle permutes 8 blocks of 16 columns");
  constexpr int WI = 2, NT = 64 * WI * WJ;  // waves along i and j, threads
  constexpr int BM = 16 * TM * WI, BN = 16 * TN * WJ;
  constexpr int UA = BM * 4 / NT, UB = BN * 4 / NT;  // 16-byte staging units per thread
  // slab row strides (elements) and sizes of the double-buffered A and B slabs
  constexpr int LA = KT ? BM + KT_PAD : LDK, LB = KT ? BN + KT_PAD : LDK;
  constexpr int SA = KT ? BK * LA : BM * LDK, SB = KT ? BK * LB : BN * LDK;
  __shared__ __attribute__((aligned(16))) uint16_t smem[2 * (SA + SB)];
  uint16_t (*sA)[SA] = reinterpret_cast<uint16_t (*)[SA]>(smem);
  uint16_t (*sB)[SB] = reinterpret_cast<uint16_t (*)[SB]>(smem + 2 * SA);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
  const int wi = wv / WJ, wj = wv % WJ;

  const int per_split = G.ti * G.tj;
  const int nt = per_split * G.ts;
  int T = blockIdx.x;
  if ((nt & 7) == 0) T = (T & 7) * (nt >> 3) + (T >> 3);
  const int sp = T / per_split;
  const int rem = T - sp * per_split;
  const int it = rem / G.tj, jt = rem - it * G.tj;
  const int i0 = it * BM, j0 = jt * BN;
  const long long ks = (long long)sp * G.kchunk;
  const long long ke = min((long long)G.K, ks + G.kchunk);
  const int nk = ke > ks ? (int)((ke - ks + BK - 1) / BK) : 0;  // slabs of this split
  Epi Ez = E;
  if constexpr (EPI == EPI_ACC) Ez.part = E.part + (long long)sp * G.pstride;

  // Staging unit u = tid + NT q.  Loads are unconditional so that the wait
  // before each LDS write counts exactly the loads it needs, and slabs past
  // the split's end re-read its first slab.
  // KT = false: row u / 4, k offset 8 (u % 4); rows past the operand clamp to
  // its last row (they only feed outputs that are never stored).  Only the
  // split's last slab can hold k >= ke; its runs are masked at the LDS write.
  // A run of 8 starting below round_up(K, 32) lies inside the operand's
  // allocation: every row stride is a multiple of 8 and every buffer carries
  // 64 bytes of slack.
  // KT = true: slab row (k) u / (BM / 8), columns 8 (u % (BM / 8)) .. + 7; a
  // run past the operand's columns is moved back inside its row (it only
  // feeds outputs that are never stored), rows k >= ke read row K - 1 and are
  // stored as zeros.
  int aoff[UA], boff[UB];
#pragma unroll
  for (int q = 0; q < UA; ++q) {
    const int u = tid + NT * q;
    if constexpr (KT) {
      aoff[q] = min(i0 + 8 * (u % (BM / 8)), (int)G.lda - 8);
    } else {
      const int r = min(i0 + (u >> 2), G.arows - 1);
      aoff[q] = r * (int)G.lda + (u & 3) * 8;
    }
  }
#pragma unroll
  for (int q = 0; q < UB; ++q) {
    const int u = tid + NT * q;
    if constexpr (KT) {
      boff[q] = min(j0 + 8 * (u % (BN / 8)), (int)G.ldb - 8);
    } else {
      const int r = min(j0 + (u >> 2), G.brows - 1);
      boff[q] = r * (int)G.ldb + (u & 3) * 8;
    }
  }
  const int kofs = (tid & 3) * 8;  // KT = false: this thread's k offset inside a slab (same for every unit)
  auto load = [&](int slab, uint4 (&ra)[UA], uint4 (&rb)[UB]) {
    const long long kt = (slab < nk) ? ks + (long long)slab * BK : ks;
    if constexpr (KT) {
#pragma unroll
      for (int q = 0; q < UA; ++q) {
        const int r = (int)min(kt + (tid + NT * q) / (BM / 8), (long long)G.K - 1);
        ra[q] = *reinterpret_cast<const uint4*>(G.a + r * (int)G.lda + aoff[q]);
      }
#pragma unroll
      for (int q = 0; q < UB; ++q) {
        const int r = (int)min(kt + (tid + NT * q) / (BN / 8), (long long)G.K - 1);
        rb[q] = *reinterpret_cast<const uint4*>(G.b + r * (int)G.ldb + boff[q]);
      }
    } else {
      const uint16_t* pa = G.a + kt;
      const uint16_t* pb = G.b + kt;
#pragma unroll
      for (int q = 0; q < UA; ++q) ra[q] = *reinterpret_cast<const uint4*>(pa + aoff[q]);
#pragma unroll
      for (int q = 0; q < UB; ++q) rb[q] = *reinterpret_cast<const uint4*>(pb + boff[q]);
    }
  };
  auto store = [&](int slab, int buf, const uint4 (&ra)[UA], const uint4 (&rb)[UB]) {
    const long long kt = ks + (long long)slab * BK;
    if constexpr (KT) {
      const bool full = kt + BK <= ke;  // uniform
#pragma unroll
      for (int q = 0; q < UA; ++q) {
        const int u = tid + NT * q, kr = u / (BM / 8);
        const bool ok = full || kt + kr < ke;
        *reinterpret_cast<uint4*>(&sA[buf][kr * LA + ((8 * (u % (BM / 8))) ^ kt_swz(kr))]) =
            ok ? ra[q] : uint4{0u, 0u, 0u, 0u};
      }
#pragma unroll
      for (int q = 0; q < UB; ++q) {
        const int u = tid + NT * q, kr = u / (BN / 8);
        const bool ok = full || kt + kr < ke;
        *reinterpret_cast<uint4*>(&sB[buf][kr * LB + ((8 * (u % (BN / 8))) ^ kt_swz(kr))]) =
            ok ? rb[q] : uint4{0u, 0u, 0u, 0u};
      }
    } else if (kt + BK <= ke) {  // uniform: a full slab
#pragma unroll
      for (int q = 0; q < UA; ++q) {
        const int u = tid + NT * q;
        *reinterpret_cast<uint4*>(&sA[buf][slab_off(u >> 2, u & 3)]) = ra[q];
      }
#pragma unroll
      for (int q = 0; q < UB; ++q) {
        const int u = tid + NT * q;
        *reinterpret_cast<uint4*>(&sB[buf][slab_off(u >> 2, u & 3)]) = rb[q];
      }
    } else {  // the split's last slab (or a padding slab): keep k < ke only
      const long long nv = ke - (kt + kofs);  // valid elements of this thread's runs (may be <= 0)
      uint32_t m[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) m[e] = (2 * e + 1 < nv) ? 0xffffffffu : (2 * e < nv ? 0xffffu : 0u);
#pragma unroll
      for (int q = 0; q < UA; ++q) {
        const int u = tid + NT * q;
        *reinterpret_cast<uint4*>(&sA[buf][slab_off(u >> 2, u & 3)]) =
            uint4{ra[q].x & m[0], ra[q].y & m[1], ra[q].z & m[2], ra[q].w & m[3]};
      }
#pragma unroll
      for (int q = 0; q < UB; ++q) {
        const int u = tid + NT * q;
        *reinterpret_cast<uint4*>(&sB[buf][slab_off(u >> 2, u & 3)]) =
            uint4{rb[q].x & m[0], rb[q].y & m[1], rb[q].z & m[2], rb[q].w & m[3]};
      }
    }
  };

  f32x4 acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  // EPI_ACC, first j-tile, left waves: row sums of A (the bias gradient)
  const bool rowsum = (EPI == EPI_ACC) && jt == 0 && wj == 0;
  float bsum[TM];
#pragma unroll
  for (int a = 0; a < TM; ++a) bsum[a] = 0.f;

  auto compute = [&](int buf) {
    bf16x8 fa[TM], fb[TN];
#pragma unroll
    for (int a = 0; a < TM; ++a) {
      u32x4 u;
      if constexpr (KT) {
        u = tr_frag(sA[buf], LA, wi * 16 * TM + 16 * a, lane);
      } else {
        const uint4 v = *reinterpret_cast<const uint4*>(&sA[buf][slab_off(wi * 16 * TM + 16 * a + (lane & 15), lane >> 4)]);
        u = u32x4{v.x, v.y, v.z, v.w};
      }
      fa[a] = __builtin_bit_cast(bf16x8, u);
    }
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      u32x4 u;
      if constexpr (KT) {
        u = tr_frag(sB[buf], LB, wj * 16 * TN + 16 * b, lane);
      } else {
        const uint4 v = *reinterpret_cast<const uint4*>(&sB[buf][slab_off(wj * 16 * TN + 16 * b + (lane & 15), lane >> 4)]);
        u = u32x4{v.x, v.y, v.z, v.w};
      }
      fb[b] = __builtin_bit_cast(bf16x8, u);
    }
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int b = 0; b < TN; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fb[b], fa[a], acc[a][b], 0, 0, 0);
    if constexpr (EPI == EPI_ACC) {
      if (rowsum) {  // wave-uniform
#pragma unroll
        for (int a = 0; a < TM; ++a) {
          const u32x4 u = __builtin_bit_cast(u32x4, fa[a]);
          bsum[a] += (__uint_as_float(u.x << 16) + __uint_as_float(u.x & 0xffff0000u)) +
                     (__uint_as_float(u.y << 16) + __uint_as_float(u.y & 0xffff0000u)) +
                     (__uint_as_float(u.z << 16) + __uint_as_float(u.z & 0xffff0000u)) +
                     (__uint_as_float(u.w << 16) + __uint_as_float(u.w & 0xffff0000u));
        }
      }
    }
  };

#if RN_PF == 2
  // two register sets: slab s + 2 is loaded while slab s is multiplied and
  // slab s + 1 is written to LDS; an odd slab count gets a zero padding slab
  uint4 ra0[UA], rb0[UB], ra1[UA], rb1[UB];
  const int nk2 = (nk + 1) & ~1;
  if (nk > 0) {
    load(0, ra0, rb0);
    load(1, ra1, rb1);
    store(0, 0, ra0, rb0);
  }
  __syncthreads();
  for (int s = 0; s < nk2; s += 2) {
    load(s + 2, ra0, rb0);
    compute(0);
    store(s + 1, 1, ra1, rb1);
    __syncthreads();
    load(s + 3, ra1, rb1);
    compute(1);
    if (s + 2 < nk2) store(s + 2, 0, ra0, rb0);
    __syncthreads();
  }
#else
  uint4 ra[UA], rb[UB];
  if (nk > 0) {
    load(0, ra, rb);
    store(0, 0, ra, rb);
  }
  __syncthreads();
  for (int s = 0; s < nk; ++s) {
    load(s + 1, ra, rb);  // past the last slab: a harmless re-read
    compute(s & 1);
    if (s + 1 < nk) store(s + 1, (s + 1) & 1, ra, rb);
    __syncthreads();
  }
#endif
  // lane: row i = 16a + lane % 16, columns j = 16b + 4 (lane / 16) + 0..3
  // EPI_ROW: the LDS (free after the loop's last barrier) holds each wave's row sums [wj][row][2]
  static_assert(EPI != EPI_ROW || 2 * WJ * BM * 4 <= (int)sizeof(smem), "row sums must fit the staging LDS");
  float* red = reinterpret_cast<float*>(smem) + 2 * (wj * BM + wi * 16 * TM);
  epilogue_tile<EPI, TM, TN>(Ez, acc, i0 + wi * 16 * TM, j0 + wj * 16 * TN, lane, red);
  if constexpr (EPI == EPI_ROW) {
    __syncthreads();
    if (tid < BM && i0 + tid < E.rows) {  // the workgroup's sums over its BN columns, waves in order
      const float* r = reinterpret_cast<const float*>(smem) + 2 * tid;
      float cz = 0.f, cx = 0.f;
#pragma unroll
      for (int q = 0; q < WJ; ++q) {
        cz += r[2 * q * BM];
        cx += r[2 * q * BM + 1];
      }
      E.rp[(long long)jt * 2 * E.rows + i0 + tid] = cz;
      E.rp[(long long)jt * 2 * E.rows + E.rows + i0 + tid] = cx;
    }
  }
  if constexpr (EPI == EPI_ACC) {
    if (rowsum) {
#pragma unroll
      for (int a = 0; a < TM; ++a) {
        float v = bsum[a];
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        const int i = i0 + wi * 16 * TM + 16 * a + (lane & 15);
        if (lane < 16 && i < Ez.rows) Ez.part[Ez.base + (long long)Ez.rows * Ez.wcols + i] += v;
      }
    }
  }
}

// ------------------------------------------------------------- convert
// rowm[r][c] = bf16(src[r][c] * scale[r]) (scale optional) for r < rows,
// c < cols; with tcol >= 0 also rowm[r][tcol] = bf16(t of row r), t = (n0 +
// r / mp) dt (the time input of the network, next to x).  Columns between
// cols and the next multiple of 4 are written as zeros.  Each thread converts
// float4 runs of one row and stores 4-element bf16 runs; the src row stride
// is a multiple of 4.
__global__ __launch_bounds__(256) void k_convert(const float* __restrict__ src, long long lds, int rows, int cols,
                                                 const float* __restrict__ scale, uint16_t* __restrict__ rowm,
                                                 long long ldr, int tcol, int n0, int mp, float dt) {
  const int c4 = (cols + 3) / 4;                                  // runs per row
  const long long e = blockIdx.x * 256LL + threadIdx.x;
  if (e >= (long long)rows * c4) return;
  const int r = (int)(e / c4), c = 4 * (int)(e % c4);
  f32x4 v = *reinterpret_cast<const f32x4*>(src + (long long)r * lds + c);
  if (scale) v = v * scale[r];
  float o[4] = {v[0], v[1], v[2], v[3]};
  const float t = rbf((float)(n0 + r / mp) * dt);
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (c + q >= cols) o[q] = (c + q == tcol) ? t : 0.f;
  *reinterpret_cast<uint2*>(rowm + (long long)r * ldr + c) = pack4(o[0], o[1], o[2], o[3]);
  if (tcol >= 0 && (cols & 3) == 0 && c + 4 == cols) rowm[(long long)r * ldr + tcol] = (uint16_t)bfbits(t);
}

// ------------------------------------------------------ row sums
// c_n of row r of a chunk from the output GEMM's per-tile partial sums (in
// j-tile order): c = sum z.s - dt r sum z.x (BSB), sum z.s + dt lam sum z.z
// (HJB), sum z.s otherwise; C is indexed by the chunk's first row.
__global__ __launch_bounds__(256) void k_csum(Geo g, int rows, int ntj, const float* __restrict__ rp,
                                              float* __restrict__ C) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= rows) return;
  float cz = 0.f, cx = 0.f;
  for (int q = 0; q < ntj; ++q) {
    cz += rp[(long long)q * 2 * rows + r];
    cx += rp[(long long)q * 2 * rows + rows + r];
  }
  float c = cz;
  if (g.drv == 0) c -= g.dt * g.drv_p0 * cx;
  else if (g.drv == 1) c += g.dt * g.drv_p0 * cx;
  C[r] = c;
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

// Launch with TM x TN wave tiles; `splits` > 1 splits the reduction (EPI_ACC
// only); KT: k-major operands (EPI_ACC only).
template <int EPI, int TM, int TN, bool KT = false, int WJ = RN_WJ>
static hipError_t gemm(Gm G, const Epi& E, int Mrows, int Ncols, int splits, hipStream_t s) {
  constexpr int BM = 32 * TM, BN = 16 * TN * WJ;
  G.kchunk = G.K;
  if (splits > 1) G.kchunk = (((long long)G.K + splits - 1) / splits + BK - 1) / BK * BK;
  if (G.kchunk < BK) G.kchunk = BK;
  G.ts = (int)(((long long)G.K + G.kchunk - 1) / G.kchunk);
  if (G.ts < 1) G.ts = 1;
  G.ti = (Mrows + BM - 1) / BM;
  G.tj = (Ncols + BN - 1) / BN;
  const long long nt = (long long)G.ti * G.tj * G.ts;
  if (nt <= 0) return hipSuccess;
  k_gemm<EPI, TM, TN, WJ, KT><<<(unsigned)nt, 128 * WJ, 0, s>>>(G, E);
  return hipGetLastError();
}

}  // namespace rn

// ===================================================== host sequencing
using namespace rn;

static Gm gm(const uint16_t* a, long long lda, int arows, const uint16_t* b, long long ldb, int brows, int K) {
  Gm G = {};
  G.a = a; G.lda = lda; G.arows = arows;
  G.b = b; G.ldb = ldb; G.brows = brows; G.K = K;
  return G;
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
  L.ldx = (int)((d + 1 + 7) / 8 * 8);
  L.rows = (long long)g.rn_chunk * g.M;
  L.ntj = (int)((d + 16 * RN_TN * RN_WJ - 1) / (16 * RN_TN * RN_WJ));
  L.nchunks = (g.N + g.rn_chunk - 1) / g.rn_chunk;
  L.kept = g.rn_store ? L.nchunks : 1;
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

static hipError_t convert(const float* src, long long lds, int rows, int cols, const float* scale, uint16_t* rowm,
                          long long ldr, int tcol, int n0, int mp, float dt, hipStream_t s) {
  const long long n = (long long)rows * ((cols + 3) / 4);
  if (n <= 0) return hipSuccess;
  k_convert<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(src, lds, rows, cols, scale, rowm, ldr, tcol, n0, mp, dt);
  return hipGetLastError();
}

// Forward of the rows of steps [n0, n0 + ns).  With `recompute` (reverse
// sweep) it also keeps a_1..a_B and the time column of [x; t] that the
// weight gradients read; with `with_output` it forms Z and from it v_n
// (over s_n in V) and c_n (C).
static hipError_t chunk_forward(const Geo& g, const ResnetLayout& L, const ResnetBufs& R, int n0, int ns,
                                const float* X, float* V, float* C, bool with_output, bool recompute,
                                hipStream_t s) {
  const int rows = ns * g.M, w = g.w, d = g.d, B = g.L;
  const float* wt = R.pf;
  const float* bin = R.pf + w;
  hipError_t e;
  // bf16 [x; t] (the GEMM below reads the first d columns)
  if ((e = convert(X + (size_t)n0 * g.M * g.dp, g.dp, rows, d, nullptr, R.xb, L.ldx, recompute ? d : -1, n0, g.M,
                   g.dt, s)) != hipSuccess)
    return e;
  {  // h0 = tanh(W_in [x; t] + b_in)
    Gm G = gm(R.xb, L.ldx, rows, pk_win(g, L, R.pk), L.dq, w, d);
    Epi E = epi0(rows, w);
    E.bias = bin; E.wt = wt; E.n0 = n0; E.mp = g.M; E.dt = g.dt;
    E.h32 = R.h32; E.ldh = w; E.ob = R.hb; E.ldb = w;
    if ((e = gemm<EPI_TANH_IN, RN_TM, RN_TN>(G, E, rows, w, 1, s)) != hipSuccess) return e;
  }
  for (int k = 1; k <= B; ++k) {  // a_k = tanh(W_k h_{k-1} + b_k), h_k = h_{k-1} + a_k
    Gm G = gm(R.hb + (size_t)(k - 1) * L.rows * w, w, rows, pk_wk(g, L, R.pk, k), w, w, w);
    Epi E = epi0(rows, w);
    E.bias = R.pf + 2 * w + (size_t)(k - 1) * w;
    E.h32 = R.h32; E.ldh = w;
    E.ob = R.hb + (size_t)k * L.rows * w; E.ldb = w;
    if (recompute) E.ab = R.ab + (size_t)(k - 1) * L.rows * w, E.lda = w;
    if ((e = gemm<EPI_TANH_RES, RN_TM, RN_TN>(G, E, rows, w, 1, s)) != hipSuccess) return e;
  }
  if (with_output) {  // Z = W_o h_B + b_o, consumed at once: v_n (over s_n in V) and c_n (C)
    const size_t r0 = (size_t)n0 * g.M;
    Gm G = gm(R.hb + (size_t)B * L.rows * w, w, rows, pk_wo(g, L, R.pk), w, d, w);
    Epi E = epi0(rows, d);
    E.bias = R.pf + 2 * w + (size_t)B * w;
    E.sv = V + r0 * g.dp; E.x = X + r0 * g.dp; E.ldv = g.dp; E.rp = R.rp;
    E.drv = g.drv; E.p0 = g.drv_p0; E.dt = g.dt;
    if ((e = gemm<EPI_ROW, RN_TM, RN_TN>(G, E, rows, d, 1, s)) != hipSuccess) return e;
    k_csum<<<(unsigned)((rows + 255) / 256), 256, 0, s>>>(g, rows, L.ntj, R.rp, C + r0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

// The buffers of chunk c: its own activation copies when they are kept
// across the passes, else the single shared set.
static ResnetBufs chunk_view(const Geo& g, const ResnetLayout& L, const ResnetBufs& R, int c) {
  ResnetBufs V = R;
  if (L.kept > 1) {
    const size_t w = (size_t)g.w, rows = (size_t)L.rows;
    V.hb += (size_t)c * (g.L + 1) * rows * w;
    V.ab += (size_t)c * g.L * rows * w;
    V.xb += (size_t)c * rows * L.ldx;
  }
  return V;
}

hipError_t resnet_forward(const Geo& g, const ResnetBufs& R, const float* X, float* V, float* C, hipStream_t s) {
  const ResnetLayout L = resnet_layout(g);
  hipError_t e;
  for (int n0 = 0; n0 < g.N; n0 += g.rn_chunk) {
    const int ns = min(g.rn_chunk, g.N - n0);
    // when activations are kept, the forward pass also writes what the
    // reverse sweep reads (a_k, [x; t]) into the chunk's own copy
    const ResnetBufs Rc = chunk_view(g, L, R, n0 / g.rn_chunk);
    if ((e = chunk_forward(g, L, Rc, n0, ns, X, V, C, true, g.rn_store != 0, s)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// Reverse sweep of every chunk (recomputing its activations unless the
// forward pass kept them).  Weight gradients are products over the chunk's
// rows of the row-major bf16 activations read k-major (g_k, h_k, zeta,
// [x; t]) and accumulate over chunks into `splits` partial buffers of the
// flat parameter layout, one per reduction split of each GEMM (fixed order:
// deterministic).
hipError_t resnet_backward(const Geo& g, const ResnetBufs& R0, const float* X, const float* V, const float* LAM,
                           float* part, int splits, hipStream_t s) {
  const ResnetLayout L = resnet_layout(g);
  const int w = g.w, d = g.d, B = g.L;
  const long long offbin = (long long)w * (d + 1), offk = offbin + w;
  const long long offo = offk + (long long)B * ((long long)w * w + w);
  hipError_t e;
  k_fill<<<grid1((long long)splits * g.pstride, 16384), 256, 0, s>>>(part, (long long)splits * g.pstride);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  for (int n0 = 0; n0 < g.N; n0 += g.rn_chunk) {
    const int ns = min(g.rn_chunk, g.N - n0);
    const int rows = ns * g.M;
    const ResnetBufs R = chunk_view(g, L, R0, n0 / g.rn_chunk);
    if (!g.rn_store)  // checkpointed: recompute the chunk's activations
      if ((e = chunk_forward(g, L, R, n0, ns, X, nullptr, nullptr, false, true, s)) != hipSuccess) return e;
    const float* Vc = V + (size_t)n0 * g.M * g.dp;
    const float* lam = LAM + (size_t)n0 * g.M;  // lambda_{n+1} of every row
    // zeta = lambda v in bf16
    if ((e = convert(Vc, g.dp, rows, d, lam, R.vb, L.dq, -1, 0, 1, 0.f, s)) != hipSuccess) return e;
    int cur = 0;
    uint16_t* gb[2] = {R.gb, R.gb + (size_t)L.rows * w};
    {  // delta_B = W_o^T zeta, zeta = lambda v;  g_B = delta_B (1 - a_B^2)
      Gm G = gm(R.vb, L.dq, rows, pk_wot(g, L, R.pk), L.dq, w, d);
      Epi E = epi0(rows, w);
      E.h32 = R.d32; E.ldh = w; E.ob = gb[cur]; E.ldb = w;
      E.ab = R.ab + (size_t)(B - 1) * L.rows * w; E.lda = w;
      if ((e = gemm<EPI_BWD_FIRST, RN_TM, RN_TN>(G, E, rows, w, 1, s)) != hipSuccess) return e;
    }
    {  // dW_o += zeta^T h_B, db_o += sum zeta
      Gm G = gm(R.vb, L.dq, d, R.hb + (size_t)B * L.rows * w, w, w, rows);
      G.pstride = g.pstride;
      Epi E = epi0(d, w);
      E.part = part; E.base = offo; E.wcols = w;
      if ((e = gemm<EPI_ACC, RN_TM, RN_TN, true>(G, E, d, w, splits, s)) != hipSuccess) return e;
    }
    for (int k = B; k >= 1; --k) {
      {  // dW_k += g_k^T h_{k-1}, db_k += sum g_k
        Gm G = gm(gb[cur], w, w, R.hb + (size_t)(k - 1) * L.rows * w, w, w, rows);
        G.pstride = g.pstride;
        Epi E = epi0(w, w);
        E.part = part; E.base = offk + (long long)(k - 1) * ((long long)w * w + w); E.wcols = w;
        if ((e = gemm<EPI_ACC, RN_TM, RN_TN, true>(G, E, w, w, splits, s)) != hipSuccess) return e;
      }
      {  // delta_{k-1} = delta_k + W_k^T g_k;  g_{k-1} = delta_{k-1} (1 - a_{k-1}^2), a_0 := h_0
        Gm G = gm(gb[cur], w, rows, pk_wkt(g, L, R.pk, k), w, w, w);
        Epi E = epi0(rows, w);
        E.h32 = R.d32; E.ldh = w; E.ob = gb[cur ^ 1]; E.ldb = w;
        E.ab = (k >= 2) ? R.ab + (size_t)(k - 2) * L.rows * w : R.hb;
        E.lda = w;
        if ((e = gemm<EPI_BWD_RES, RN_TM, RN_TN>(G, E, rows, w, 1, s)) != hipSuccess) return e;
        cur ^= 1;
      }
    }
    {  // dW_in += g_0^T [x; t], db_in += sum g_0
      Gm G = gm(gb[cur], w, w, R.xb, L.ldx, d + 1, rows);
      G.pstride = g.pstride;
      Epi E = epi0(w, d + 1);
      E.part = part; E.base = 0; E.wcols = d + 1;
      if ((e = gemm<EPI_ACC, RN_TM, RN_TN, true>(G, E, w, d + 1, splits, s)) != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

}  // namespace fbsde
