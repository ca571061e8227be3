// C ABI of the gfx950 deep-FBSDE library: validation, plan, workspace
// layout and the launch sequence of each hot call (declared in fbsde.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/fbsde.h"
#include "fbsde_internal.h"

using fbsde::Geo;
using fbsde::WsLayout;

// Ring of event pairs per kernel id for live per-kernel timing.
struct ProfRing {
  static constexpr int R = 64;
  std::vector<hipEvent_t> start, stop;
  std::vector<char> used;
  int head = 0;
  double ms = 0.0;
  long long count = 0;
};

struct fbsde_plan {
  fbsde_problem prob;
  fbsde_net net;
  int32_t N;
  int64_t M;
  Geo geo;
  WsLayout ws;
  float* x0_dev;  // [dp] zero-padded, owned
  int* nf_host = nullptr;  // pinned host flag: a non-finite loss or gradient was produced
  int device;
  bool prof = false;
  ProfRing ring[FBSDE_PROF_NUM];
  // tuning: candidate register-tile shapes and the workspace reserved for all of them
  int ncand = 0;
  int cand_ti[4], cand_tw[4];
  size_t reserve = 0;
  bool ws_queried = false;  // fbsde_workspace_size was called: the reserve may not grow
};

namespace {

thread_local std::string g_last_error;

fbsde_status fail(fbsde_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

fbsde_status hip_fail(hipError_t e, const char* where) {
  return fail(FBSDE_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

constexpr int kMaxTuneSplits = 32;

int tiles(int n, bool bf16) {
  // 16-wide tiles; bf16 K-blocks are 32 wide, so bf16 tile counts are even
  return bf16 ? 2 * ((n + 31) / 32) : (n + 15) / 16;
}

void make_layout(fbsde_plan* P) {
  const Geo& g = P->geo;
  WsLayout& w = P->ws;
  const size_t M = (size_t)g.M, N = (size_t)g.N, esz = g.bf16 ? 2 : 4;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align256(bytes);
    return o;
  };
  w.X = take((N + 1) * M * g.dp * 4);
  w.V = take(N * M * g.dp * 4);
  w.C = take(N * M * 4);
  w.Y = take((N + 1) * M * 4);
  w.LAM = take(N * M * 4);
  w.QN = take(M * 4);
  w.LN = take(M * 4);
  if (g.kind == 2) {
    // u-network: every buffer carries 256 bytes of slack past its end (the
    // GEMMs' 16-byte staging loads may run up to 15 floats past a row's
    // last valid k)
    const fbsde::UnetLayout U = fbsde::unet_layout(g);
    const size_t R = (size_t)U.R, wq = (size_t)U.wq, K = (size_t)U.K, wd = (size_t)g.w, dp = (size_t)g.dp;
    const bool nais = g.uarch == 2;
    auto tk = [&](size_t floats) { return take(floats * 4 + 256); };
    w.UU = tk(R);
    w.UZ = tk(R * dp);
    w.UUB = tk(R);
    w.UZB = tk(R * dp);
    w.UH = tk((K + 1) * R * wq);
    w.UAL = tk(g.uarch == 0 ? 0 : K * R * wq);
    w.UHH = tk(K * R * wq);
    w.UG = tk((K + 1) * R * wq);
    w.UHHB = tk((K + 1) * R * wq);
    w.UHB0 = tk(R * wq);
    w.UALB = tk(K * R * wq);
    w.UHBAR = tk(R * wq);
    w.UABAR = tk((K + 1) * R * wq);
    w.UW0X = tk(wd * dp);
    w.UW0T = tk(wd);
    w.UAK = tk(K * wd * wq);
    w.URK = tk(nais ? K * wd * wq : 0);
    w.UEX = tk(nais ? K * wd * dp : 0);
    w.UET = tk(nais ? K * wd : 0);
    w.UP = tk(nais ? R * wq : 0);
    w.UABARW = tk(nais ? K * wd * wd : 0);
    w.UPART = tk((size_t)U.slots * (size_t)U.pstride);
    w.UCB = tk(R);
    w.ULP = take(((R + 31) / 32) * 8 + 64);  // one fp64 partial per 32-row residual workgroup, then the flag
  } else if (g.kind == 0) {
    // activations of every step, or of one recompute chunk of steps
    const size_t NA = g.rn_chunk > 0 ? (size_t)g.rn_chunk : N;
    w.H = take(NA * g.L * M * g.wp * esz);
    w.DZ = take(NA * M * g.zp * esz);
    w.DH = take(NA * g.L * M * g.wp * esz);
    w.PF = take((N > 1 ? N - 1 : 0) * (size_t)g.packf_step * esz);
    w.PB = take((N > 1 ? N - 1 : 0) * (size_t)g.packb_step * esz);
    w.PBIAS = take((N > 1 ? N - 1 : 0) * (size_t)g.pbias_step * 4);
  } else {
    const fbsde::ResnetLayout R = fbsde::resnet_layout(g);
    const size_t rows = (size_t)R.rows, wd = (size_t)g.w;
    // bf16 GEMM operands carry 64 bytes of slack: a staged run of 8 may start
    // up to 24 elements past the last row's valid k (its values are masked)
    const size_t slack = 64;
    w.RPK = take((size_t)R.pk_elems * 2 + slack);
    w.RPF = take((size_t)R.pf_elems * 4);
    w.RH32 = take(rows * wd * 4);
    const size_t kept = (size_t)R.kept;
    w.RHB = take(kept * (g.L + 1) * rows * wd * 2 + slack);
    w.RAB = take(kept * g.L * rows * wd * 2 + slack);
    w.RD32 = take(rows * wd * 4);
    w.RGB = take(2 * rows * wd * 2 + slack);
    w.RRP = take((size_t)R.ntj * 2 * rows * 4);
    w.RXB = take(kept * rows * (size_t)R.ldx * 2 + slack);
    w.RVB = take(rows * (size_t)R.dq * 2 + slack);
  }
  // weight-gradient splits over paths (per-step MLP) or over chunk rows
  // (residual network): preset by the caller, 0 = automatic.  The per-step
  // MLP takes one split per 512 paths, and at least enough that the
  // (split, step) workgroups of the fused reverse kernel cover the CUs.
  int splits = w.splits;
  if (splits <= 0) {
    if (g.kind == 0) {
      const long long fill = (fbsde::device_cus() + (long long)N - 1) / (long long)N;
      splits = (int)std::max<long long>((long long)((M + 511) / 512), std::min<long long>(fill, (long long)M / 32));
    } else {
      splits = 16;
    }
  }
  if (w.splits <= 0)
    if (const char* e = getenv("FBSDE_WGRAD_SPLITS")) splits = atoi(e);
  if (splits < 1) splits = 1;
  if (splits > 64) splits = 64;
  long long chunk = ((long long)M + splits - 1) / splits;
  chunk = (chunk + 31) / 32 * 32;
  splits = (int)(((long long)M + chunk - 1) / chunk);
  w.splits = splits;
  w.chunk = chunk;
  // (the u-network keeps its partial sums in its own buffer)
  w.PART = take(g.kind == 2 ? 0 : (size_t)splits * (size_t)g.pstride * 4);
  w.scan_blocks = (int)((M + 63) / 64);  // one wave per scan workgroup
  w.RED = take((size_t)w.scan_blocks * 2 * 8);
  w.total = off;
}

void set_tiles(Geo& g, int ti, int tw) {
  g.ti = ti;
  g.tw = tw;
  g.zp = 16 * ti;
  g.wp = 16 * tw;
  const long long L = g.L;
  g.packf_step = 256LL * (g.tw * g.ti + (L - 1) * g.tw * g.tw + g.ti * g.tw);
  g.packb_step = 256LL * (g.tw * g.ti + (L - 1) * g.tw * g.tw);
  g.pbias_step = 16LL * (L * g.tw + g.ti);
}

// Shared residual network: rows per chunk of whole steps (about `rows`, at
// least one step), and whether a chunk's activations can be addressed with
// the GEMMs' 32-bit element offsets.
constexpr int64_t kDefaultChunkRows = 262144;
int rn_chunk_steps(int64_t N, int64_t M, int64_t rows) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(N, rows / std::max<int64_t>(1, M)));
}
bool rn_offsets_fit(int64_t M, int64_t chunk_steps, int64_t width, int64_t d) {
  const int64_t rows = chunk_steps * M, ldx = (d + 1 + 7) / 8 * 8;
  const int64_t wide = std::max<int64_t>(width, ldx);
  return (rows + 32) * wide < 0x7fffffffLL;
}

// Largest workspace over the candidate tile shapes, at the largest split count
// the tuner may pick and at the automatic one, so that any tuned
// configuration fits the caller's buffer.
size_t reserve_bytes(fbsde_plan* P) {
  const Geo keep_g = P->geo;
  const WsLayout keep_w = P->ws;
  size_t mx = 0;
  for (int c = 0; c < P->ncand; ++c) {
    if (P->geo.kind == 0) set_tiles(P->geo, P->cand_ti[c], P->cand_tw[c]);
    for (int sp : {kMaxTuneSplits, 0}) {  // the tuner's largest split count and the automatic one
      P->ws.splits = sp;
      make_layout(P);
      mx = P->ws.total > mx ? P->ws.total : mx;
    }
  }
  P->geo = keep_g;
  P->ws = keep_w;
  return mx;
}

bool finite_all(const double* v, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

template <class T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(ws) + off);
}
template <class T>
const T* at(const void* ws, size_t off) {
  return reinterpret_cast<const T*>(reinterpret_cast<const char*>(ws) + off);
}

fbsde::ResnetBufs resnet_bufs(const fbsde_plan* P, void* ws) {
  const WsLayout& L = P->ws;
  fbsde::ResnetBufs R;
  R.pk = at<uint16_t>(ws, L.RPK);
  R.pf = at<float>(ws, L.RPF);
  R.h32 = at<float>(ws, L.RH32);
  R.hb = at<uint16_t>(ws, L.RHB);
  R.ab = at<uint16_t>(ws, L.RAB);
  R.d32 = at<float>(ws, L.RD32);
  R.gb = at<uint16_t>(ws, L.RGB);
  R.rp = at<float>(ws, L.RRP);
  R.xb = at<uint16_t>(ws, L.RXB);
  R.vb = at<uint16_t>(ws, L.RVB);
  return R;
}

fbsde::UnetBufs unet_bufs(const fbsde_plan* P, void* ws) {
  const WsLayout& L = P->ws;
  fbsde::UnetBufs B;
  B.X = at<float>(ws, L.X);
  B.S = at<float>(ws, L.V);
  B.U = at<float>(ws, L.UU);
  B.Z = at<float>(ws, L.UZ);
  B.UB = at<float>(ws, L.UUB);
  B.ZB = at<float>(ws, L.UZB);
  B.H = at<float>(ws, L.UH);
  B.AL = at<float>(ws, L.UAL);
  B.HH = at<float>(ws, L.UHH);
  B.G = at<float>(ws, L.UG);
  B.HHB = at<float>(ws, L.UHHB);
  B.HB0 = at<float>(ws, L.UHB0);
  B.ALB = at<float>(ws, L.UALB);
  B.HBAR = at<float>(ws, L.UHBAR);
  B.ABAR = at<float>(ws, L.UABAR);
  B.W0x = at<float>(ws, L.UW0X);
  B.w0t = at<float>(ws, L.UW0T);
  B.Ak = at<float>(ws, L.UAK);
  B.Rk = at<float>(ws, L.URK);
  B.Ex = at<float>(ws, L.UEX);
  B.et = at<float>(ws, L.UET);
  B.P = at<float>(ws, L.UP);
  B.Abar = at<float>(ws, L.UABARW);
  B.part = at<float>(ws, L.UPART);
  B.CB = at<float>(ws, L.UCB);
  B.lpart = at<double>(ws, L.ULP);
  return B;
}

// A non-finite result of an earlier call on the plan (raised on the device
// into pinned host memory): reported once, then cleared.
fbsde_status take_nonfinite(const fbsde_plan* P) {
  volatile int* f = P->nf_host;
  if (f && *f) {
    *f = 0;
    return fail(FBSDE_ERR_NONFINITE, "an earlier call on this plan produced a non-finite loss or gradient");
  }
  return FBSDE_OK;
}

fbsde_status check_hot(const fbsde_plan* P, const void* ws) {
  if (!P) return fail(FBSDE_ERR_INVALID, "plan is NULL");
  if (!ws) return fail(FBSDE_ERR_INVALID, "workspace is NULL");
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0)
    return fail(FBSDE_ERR_INVALID, "workspace must be 256-byte aligned");
  return take_nonfinite(P);
}

// Event pair around one launch (no-op unless profiling is enabled).  A ring
// slot is reused only after its previous pair has completed.
struct ProfScope {
  fbsde_plan* P;
  int id;
  hipStream_t s;
  int slot = -1;
  ProfScope(fbsde_plan* p, int i, hipStream_t st) : P(p), id(i), s(st) {
    if (!P->prof) return;
    ProfRing& r = P->ring[id];
    slot = r.head;
    r.head = (r.head + 1) % ProfRing::R;
    if (r.used[slot]) {
      float ms = 0.f;
      if (hipEventSynchronize(r.stop[slot]) == hipSuccess &&
          hipEventElapsedTime(&ms, r.start[slot], r.stop[slot]) == hipSuccess) {
        r.ms += ms;
        r.count += 1;
      }
      r.used[slot] = 0;
    }
    (void)hipEventRecord(r.start[slot], s);
  }
  ~ProfScope() {
    if (slot < 0) return;
    ProfRing& r = P->ring[id];
    (void)hipEventRecord(r.stop[slot], s);
    r.used[slot] = 1;
  }
};

fbsde_status run_forward(fbsde_plan* P, const float* params, const double* y0, uint64_t seed,
                         uint64_t iter, const uint64_t* iter_dev, void* ws, hipStream_t s) {
  const Geo& g = P->geo;
  const WsLayout& L = P->ws;
  hipError_t e;
  if (g.kind == 1) {
    const fbsde::ResnetBufs R = resnet_bufs(P, ws);
    {
      ProfScope ps(P, FBSDE_PROF_PACK, s);
      if ((e = fbsde::resnet_pack(g, params, R.pk, R.pf, s)) != hipSuccess) return hip_fail(e, "pack");
    }
    {
      ProfScope ps(P, FBSDE_PROF_SDE, s);
      if ((e = fbsde::launch_sde(g, P->x0_dev, seed, iter, iter_dev, at<float>(ws, L.X), at<float>(ws, L.V),
                                 at<float>(ws, L.QN), at<float>(ws, L.LN), s)) != hipSuccess)
        return hip_fail(e, "sde");
    }
    {
      ProfScope ps(P, FBSDE_PROF_FORWARD, s);
      if ((e = fbsde::resnet_forward(g, R, at<float>(ws, L.X), at<float>(ws, L.V), at<float>(ws, L.C), s)) !=
          hipSuccess)
        return hip_fail(e, "forward");
    }
    {
      ProfScope ps(P, FBSDE_PROF_SCAN, s);
      if ((e = fbsde::launch_scan(g, y0, at<float>(ws, L.C), at<float>(ws, L.QN), at<float>(ws, L.LN),
                                  at<float>(ws, L.Y), at<float>(ws, L.LAM), at<double>(ws, L.RED),
                                  L.scan_blocks, s)) != hipSuccess)
        return hip_fail(e, "scan");
    }
    return FBSDE_OK;
  }
  {
    // the step weights' packing and the SDE in one launch (timed as the SDE)
    ProfScope ps(P, FBSDE_PROF_SDE, s);
    if ((e = fbsde::launch_pack_sde(g, params, at<void>(ws, L.PF), at<void>(ws, L.PB), at<float>(ws, L.PBIAS),
                                    P->x0_dev, seed, iter, iter_dev, at<float>(ws, L.X), at<float>(ws, L.V),
                                    at<float>(ws, L.QN), at<float>(ws, L.LN), s)) != hipSuccess)
      return hip_fail(e, "pack and sde");
  }
  {
    // with checkpointing the activations of each chunk of steps are written
    // over the previous chunk's (the reverse pass recomputes them)
    ProfScope ps(P, FBSDE_PROF_FORWARD, s);
    const int cs = g.rn_chunk > 0 ? g.rn_chunk : g.N;
    for (int n0 = 0; n0 < g.N; n0 += cs) {
      Geo gc = g;
      gc.n0 = n0;
      gc.ns = std::min(cs, g.N - n0);
      if ((e = fbsde::launch_forward(gc, params, at<void>(ws, L.PF), at<float>(ws, L.PBIAS), at<float>(ws, L.X),
                                     at<float>(ws, L.V), at<float>(ws, L.C), at<void>(ws, L.H), s)) != hipSuccess)
        return hip_fail(e, "forward");
    }
  }
  {
    ProfScope ps(P, FBSDE_PROF_SCAN, s);
    if ((e = fbsde::launch_scan(g, y0, at<float>(ws, L.C), at<float>(ws, L.QN), at<float>(ws, L.LN),
                                at<float>(ws, L.Y), at<float>(ws, L.LAM), at<double>(ws, L.RED),
                                L.scan_blocks, s)) != hipSuccess)
      return hip_fail(e, "scan");
  }
  return FBSDE_OK;
}

// Sum of the split partials into grad, loss and dL/dY0 (and the Adam step
// when `adam` is given).
hipError_t reduce_tail(fbsde_plan* plan, float* grad, double* grad_y0, double* loss, void* ws, hipStream_t s,
                       const fbsde::AdamArgs* adam) {
  const WsLayout& L = plan->ws;
  if (adam)
    return fbsde::launch_reduce_adam(plan->geo, at<float>(ws, L.PART), L.splits, grad, at<double>(ws, L.RED),
                                     L.scan_blocks, loss, grad_y0, plan->nf_host, *adam, s);
  return fbsde::launch_reduce(plan->geo, at<float>(ws, L.PART), L.splits, grad, at<double>(ws, L.RED),
                              L.scan_blocks, loss, grad_y0, plan->nf_host, s);
}

// The reverse sweep and the gradient reduction; with `adam` the reduction
// also applies the Adam step (one launch).
fbsde_status run_backward(fbsde_plan* plan, float* grad, double* grad_y0, double* loss, void* ws, hipStream_t s,
                          const fbsde::AdamArgs* adam = nullptr) {
  const Geo& g = plan->geo;
  const WsLayout& L = plan->ws;
  hipError_t e;
  if (g.kind == 1) {
    {
      ProfScope ps(plan, FBSDE_PROF_BACKWARD, s);
      if ((e = fbsde::resnet_backward(g, resnet_bufs(plan, ws), at<float>(ws, L.X), at<float>(ws, L.V),
                                      at<float>(ws, L.LAM), at<float>(ws, L.PART), L.splits, s)) != hipSuccess)
        return hip_fail(e, "backward");
    }
    ProfScope ps(plan, FBSDE_PROF_REDUCE, s);
    if ((e = reduce_tail(plan, grad, grad_y0, loss, ws, s, adam)) != hipSuccess) return hip_fail(e, "reduce");
    return FBSDE_OK;
  }
  // Checkpointing: chunks of steps, last first; each chunk's activations are
  // recomputed from X_n (same kernel and arithmetic as the forward pass, so
  // the same bits) just before its reverse sweep.  Every step's weight
  // gradient has its own partial slots, so the chunk order does not matter.
  const int cs = g.rn_chunk > 0 ? g.rn_chunk : g.N;
  // The fused kernel's grid is (split, step): over a chunk of steps it fills
  // the chip only with enough splits; otherwise the separate pair, whose
  // grids do not shrink with the chunk, is the faster form (same bits; BSB
  // d = 100, M = 4096, chunks of 8 steps: 1.05 -> 0.62 ms fp32, 0.50 -> 0.39
  // ms bf16 per training step).
  const bool fused = fbsde::reverse_fused_preferred(g, L.splits) &&
                     (cs >= g.N || (long long)L.splits * cs >= fbsde::device_cus());
  for (int n0 = (g.N - 1) / cs * cs; n0 >= 0; n0 -= cs) {
    Geo gc = g;
    gc.n0 = n0;
    gc.ns = std::min(cs, g.N - n0);
    if (g.rn_chunk > 0) {
      ProfScope ps(plan, FBSDE_PROF_FORWARD, s);
      gc.recomp = 1;  // step 0 has no network, so the parameters themselves are not read
      if ((e = fbsde::launch_forward(gc, nullptr, at<void>(ws, L.PF), at<float>(ws, L.PBIAS), at<float>(ws, L.X),
                                     at<float>(ws, L.V), at<float>(ws, L.C), at<void>(ws, L.H), s)) != hipSuccess)
        return hip_fail(e, "recompute");
      gc.recomp = 0;
    }
    if (fused) {
      // the reverse sweep and the weight gradient in one kernel (timed as the backward)
      ProfScope ps(plan, FBSDE_PROF_BACKWARD, s);
      if ((e = fbsde::launch_reverse(gc, at<void>(ws, L.PB), at<float>(ws, L.X), at<float>(ws, L.V),
                                     at<float>(ws, L.LAM), at<void>(ws, L.H), at<float>(ws, L.PART), L.splits,
                                     L.chunk, s)) != hipSuccess)
        return hip_fail(e, "reverse");
    } else {
      {
        ProfScope ps(plan, FBSDE_PROF_BACKWARD, s);
        if ((e = fbsde::launch_backward(gc, at<void>(ws, L.PB), at<float>(ws, L.V), at<float>(ws, L.LAM),
                                        at<void>(ws, L.H), at<void>(ws, L.DZ), at<void>(ws, L.DH), s)) !=
            hipSuccess)
          return hip_fail(e, "backward");
      }
      ProfScope ps(plan, FBSDE_PROF_WGRAD, s);
      if ((e = fbsde::launch_wgrad(gc, at<float>(ws, L.X), at<void>(ws, L.H), at<void>(ws, L.DZ),
                                   at<void>(ws, L.DH), at<float>(ws, L.PART), L.splits, L.chunk, s)) != hipSuccess)
        return hip_fail(e, "wgrad");
    }
  }
  {
    ProfScope ps(plan, FBSDE_PROF_REDUCE, s);
    if ((e = reduce_tail(plan, grad, grad_y0, loss, ws, s, adam)) != hipSuccess) return hip_fail(e, "reduce");
  }
  return FBSDE_OK;
}

}  // namespace

namespace fbsde {
fbsde_status api_fail(fbsde_status s, const char* msg) { return fail(s, msg); }
fbsde_status api_active_workspace(const fbsde_plan* plan, size_t* bytes, int* device) {
  if (!plan || !bytes || !device) return fail(FBSDE_ERR_INVALID, "NULL argument");
  *bytes = plan->ws.total;
  *device = plan->device;
  return FBSDE_OK;
}
}  // namespace fbsde

extern "C" {

const char* fbsde_status_str(fbsde_status s) {
  switch (s) {
    case FBSDE_OK: return "ok";
    case FBSDE_ERR_INVALID: return "invalid argument";
    case FBSDE_ERR_UNSUPPORTED: return "unsupported";
    case FBSDE_ERR_HIP: return "HIP error";
    case FBSDE_ERR_NOMEM: return "out of memory";
    case FBSDE_ERR_NONFINITE: return "non-finite value";
  }
  return "unknown status";
}

const char* fbsde_last_error(void) { return g_last_error.c_str(); }

fbsde_status fbsde_plan_create(const fbsde_problem* problem, const fbsde_net* net, int32_t N, int64_t M,
                               fbsde_plan** out) {
  if (!out) return fail(FBSDE_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!problem || !net) return fail(FBSDE_ERR_INVALID, "problem or net is NULL");
  const fbsde_problem& p = *problem;
  if (p.d < 1) return fail(FBSDE_ERR_INVALID, "d must be >= 1");
  if (!(p.T > 0.0) || !std::isfinite(p.T)) return fail(FBSDE_ERR_INVALID, "T must be finite and > 0");
  if (!p.x0_host) return fail(FBSDE_ERR_INVALID, "x0_host is NULL");
  if (!finite_all(p.x0_host, p.d)) return fail(FBSDE_ERR_INVALID, "x0 is not finite");
  if (p.sde < 0 || p.sde > 1) return fail(FBSDE_ERR_INVALID, "unknown sde");
  if (p.drv < 0 || p.drv > 3) return fail(FBSDE_ERR_INVALID, "unknown driver");
  if (p.g < 0 || p.g > 3) return fail(FBSDE_ERR_INVALID, "unknown terminal condition");
  if (!finite_all(p.sde_p, 2) || !finite_all(p.drv_p, 2) || !finite_all(p.g_p, 2))
    return fail(FBSDE_ERR_INVALID, "problem parameters are not finite");
  if (N < 1) return fail(FBSDE_ERR_INVALID, "N must be >= 1");
  if (M < 1 || M > 0x7fffffffLL) return fail(FBSDE_ERR_INVALID, "M must be in [1, 2^31)");
  if (net->kind != FBSDE_NET_PER_STEP_MLP && net->kind != FBSDE_NET_SHARED_RESNET && net->kind != FBSDE_NET_U_FC &&
      net->kind != FBSDE_NET_U_RES && net->kind != FBSDE_NET_U_NAIS)
    return fail(FBSDE_ERR_INVALID, "unknown network kind");
  if (net->prec != FBSDE_FP32 && net->prec != FBSDE_BF16_MFMA) return fail(FBSDE_ERR_INVALID, "unknown precision");
  if (net->width < 1 || net->depth < 1) return fail(FBSDE_ERR_INVALID, "width and depth must be >= 1");
  const bool resnet = net->kind == FBSDE_NET_SHARED_RESNET;
  const bool unet = net->kind >= FBSDE_NET_U_FC;
  if (unet) {
    if (net->prec != FBSDE_FP32) return fail(FBSDE_ERR_UNSUPPORTED, "the u-network runs in fp32 only");
    if (net->depth > 16 || p.d > 8192 || net->width > 8192)
      return fail(FBSDE_ERR_UNSUPPORTED, "u-network: depth (blocks after the input layer) <= 16, d <= 8192, width <= 8192");
    if ((long long)(N + 1) * M > 0x7fffffffLL / 4)
      return fail(FBSDE_ERR_UNSUPPORTED, "u-network: (N + 1) M must stay below 2^29 rows");
  } else if (resnet) {
    if (net->prec != FBSDE_BF16_MFMA)
      return fail(FBSDE_ERR_UNSUPPORTED, "the shared residual network runs in bf16 only");
    if (net->width % 8 != 0 || net->width > 8192 || net->depth > 32 || p.d > 8192)
      return fail(FBSDE_ERR_UNSUPPORTED, "shared residual network: width a multiple of 8, <= 8192; depth <= 32; d <= 8192");
  } else if (p.d > 256 || net->width > 256 || net->depth > 8) {
    return fail(FBSDE_ERR_UNSUPPORTED, "per-step MLP kernels support d <= 256, width <= 256, depth <= 8");
  }

  fbsde_plan* P = new (std::nothrow) fbsde_plan();
  if (!P) return fail(FBSDE_ERR_NOMEM, "host allocation failed");
  P->prob = p;
  P->prob.x0_host = nullptr;
  P->net = *net;
  P->N = N;
  P->M = M;
  Geo& g = P->geo;
  const bool bf = net->prec == FBSDE_BF16_MFMA;
  g.d = p.d;
  g.dp = (p.d + 3) / 4 * 4;
  g.w = net->width;
  g.L = net->depth;
  g.N = N;
  g.M = (int)M;
  g.kind = unet ? 2 : resnet ? 1 : 0;
  g.L = net->depth;
  g.lds = 2;  // LDS staging, and the fused reverse kernel where it applies
  g.tpw = 0;
  g.uarch = unet ? net->kind - FBSDE_NET_U_FC : 0;
  g.kappa = 0.f;
  g.ueps = 0.01f;
  if (unet) {
    P->ncand = 1;
    P->cand_ti[0] = P->cand_tw[0] = 0;
    g.ti = g.tw = 0;
    g.zp = g.wp = 0;
    g.packf_step = g.packb_step = g.pbias_step = 0;
    g.rn_chunk = 0;
    g.rn_store = 0;
  } else if (resnet) {
    // chunks of whole steps, about 64k rows each
    g.rn_chunk = rn_chunk_steps(N, M, kDefaultChunkRows);
    g.rn_store = 0;
    if (!rn_offsets_fit(M, g.rn_chunk, net->width, p.d)) {
      delete P;
      return fail(FBSDE_ERR_UNSUPPORTED, "shared residual network: M x max(width, d) must stay below 2^31");
    }
    P->ncand = 1;
    P->cand_ti[0] = P->cand_tw[0] = 0;
    g.ti = g.tw = 0;
    g.zp = g.wp = 0;
    g.packf_step = g.packb_step = g.pbias_step = 0;
  } else {
    int ti0 = 0, tw0 = 0;
    if (!fbsde::choose_tiles(bf ? 1 : 0, tiles(p.d, bf), tiles(net->width, bf), &ti0, &tw0)) {
      delete P;
      return fail(FBSDE_ERR_UNSUPPORTED, "no fused-MLP tile shape covers this d and width");
    }
    P->ncand = fbsde::tile_candidates(bf ? 1 : 0, ti0, tw0, P->cand_ti, P->cand_tw, 2);
    g.rn_chunk = 0;
    g.rn_store = 0;
    set_tiles(g, ti0, tw0);
  }
  g.bf16 = bf ? 1 : 0;
  g.sde = p.sde;
  g.sde_s = (float)p.sde_p[0];
  g.drv = p.drv;
  g.drv_p0 = (float)p.drv_p[0];
  g.drv_p1 = (float)p.drv_p[1];
  g.g = p.g;
  g.g_p0 = (float)p.g_p[0];
  g.g_p1 = (float)p.g_p[1];
  g.dt = (float)(p.T / N);
  g.sqdt = (float)std::sqrt(p.T / N);
  const long long d = p.d, w = net->width, L = net->depth;
  if (unet) {
    const long long blk = w * w + (g.uarch == 2 ? w * (d + 1) : 0) + w;
    g.pstep = 0;
    g.nparams = w * (d + 1) + w + L * blk + w + 1;
    g.pstride = (g.nparams + 3) / 4 * 4;
  } else if (resnet) {
    g.pstep = 0;
    g.nparams = w * (d + 1) + w + L * (w * w + w) + d * w + d;
    g.pstride = (g.nparams + 3) / 4 * 4;
  } else {
    g.pstep = w * d + w + (L - 1) * (w * w + w) + d * w + d;
    g.nparams = d + (long long)(N - 1) * g.pstep;
    g.pstride = (g.nparams + 3) / 4 * 4;
  }
  P->ws.splits = 0;
  make_layout(P);
  P->reserve = reserve_bytes(P);
  if (P->reserve < P->ws.total) P->reserve = P->ws.total;

  hipError_t e = hipGetDevice(&P->device);
  if (e != hipSuccess) {
    delete P;
    return hip_fail(e, "hipGetDevice");
  }
  e = hipMalloc(&P->x0_dev, (size_t)g.dp * sizeof(float));
  if (e != hipSuccess) {
    delete P;
    return fail(FBSDE_ERR_NOMEM, std::string("hipMalloc x0: ") + hipGetErrorString(e));
  }
  float* tmp = new float[g.dp];
  for (int i = 0; i < g.dp; ++i) tmp[i] = i < p.d ? (float)problem->x0_host[i] : 0.f;
  e = hipMemcpy(P->x0_dev, tmp, (size_t)g.dp * sizeof(float), hipMemcpyHostToDevice);
  delete[] tmp;
  if (e != hipSuccess) {
    (void)hipFree(P->x0_dev);
    delete P;
    return hip_fail(e, "hipMemcpy x0");
  }
  void* flag = nullptr;
  e = hipHostMalloc(&flag, 64, hipHostMallocDefault);
  if (e != hipSuccess) {
    (void)hipFree(P->x0_dev);
    delete P;
    return fail(FBSDE_ERR_NOMEM, std::string("hipHostMalloc flag: ") + hipGetErrorString(e));
  }
  P->nf_host = static_cast<int*>(flag);
  *P->nf_host = 0;
  *out = P;
  return FBSDE_OK;
}

void fbsde_plan_destroy(fbsde_plan* plan) {
  if (!plan) return;
  (void)fbsde_profile_enable(plan, 0);
  if (plan->x0_dev) (void)hipFree(plan->x0_dev);
  if (plan->nf_host) (void)hipHostFree(plan->nf_host);
  delete plan;
}

fbsde_status fbsde_param_count(const fbsde_plan* plan, int64_t* n) {
  if (!plan || !n) return fail(FBSDE_ERR_INVALID, "plan or output is NULL");
  *n = plan->geo.nparams;
  return FBSDE_OK;
}

fbsde_status fbsde_param_layout(const fbsde_plan* plan, int64_t* n_params, int64_t* n_blocks, int64_t* offsets,
                                int32_t* shapes) {
  if (!plan) return fail(FBSDE_ERR_INVALID, "plan is NULL");
  const Geo& g = plan->geo;
  // dense layers of one network as (out, in)
  std::vector<std::pair<int, int>> layers;
  if (g.kind == 2) {  // W_0, b_0, per block (A_k | R_k, [E_k], b_k), w_o, b_o
    int64_t blk = 0, off = 0;
    auto add = [&](int rows, int cols) {
      if (offsets) offsets[blk] = off;
      if (shapes) { shapes[2 * blk] = rows; shapes[2 * blk + 1] = cols; }
      off += (int64_t)rows * cols;
      ++blk;
    };
    add(g.w, g.d + 1);
    add(g.w, 1);
    for (int k = 0; k < g.L; ++k) {
      add(g.w, g.w);
      if (g.uarch == 2) add(g.w, g.d + 1);
      add(g.w, 1);
    }
    add(1, g.w);
    add(1, 1);
    if (offsets) offsets[blk] = off;
    if (off != g.nparams) return fail(FBSDE_ERR_INVALID, "internal: block table does not cover the parameters");
    if (n_params) *n_params = g.nparams;
    if (n_blocks) *n_blocks = blk;
    return FBSDE_OK;
  }
  if (g.kind == 0) {
    layers.push_back({g.w, g.d});
    for (int l = 2; l <= g.L; ++l) layers.push_back({g.w, g.w});
  } else {
    layers.push_back({g.w, g.d + 1});
    for (int k = 1; k <= g.L; ++k) layers.push_back({g.w, g.w});
  }
  layers.push_back({g.d, g.w});
  int64_t blk = 0, off = 0;
  auto add = [&](int rows, int cols) {
    if (offsets) offsets[blk] = off;
    if (shapes) { shapes[2 * blk] = rows; shapes[2 * blk + 1] = cols; }
    off += (int64_t)rows * cols;
    ++blk;
  };
  const int nets = g.kind == 0 ? g.N - 1 : 1;
  if (g.kind == 0) add(g.d, 1);  // z0
  for (int n = 0; n < nets; ++n)
    for (const auto& lo : layers) {
      add(lo.first, lo.second);  // W
      add(lo.first, 1);          // b
    }
  if (offsets) offsets[blk] = off;
  if (off != g.nparams) return fail(FBSDE_ERR_INVALID, "internal: block table does not cover the parameters");
  if (n_params) *n_params = g.nparams;
  if (n_blocks) *n_blocks = blk;
  return FBSDE_OK;
}

fbsde_status fbsde_workspace_size(const fbsde_plan* plan, size_t* bytes) {
  if (!plan || !bytes) return fail(FBSDE_ERR_INVALID, "plan or output is NULL");
  const_cast<fbsde_plan*>(plan)->ws_queried = true;
  *bytes = plan->reserve;
  return FBSDE_OK;
}

fbsde_status fbsde_forward(fbsde_plan* plan, const float* params, const double* y0, uint64_t seed,
                           uint64_t iter, double* loss, void* ws, void* stream) {
  fbsde_status st = check_hot(plan, ws);
  if (st != FBSDE_OK) return st;
  if (plan->geo.kind == 2) return fail(FBSDE_ERR_UNSUPPORTED, "u-network plans use fbsde_unet_forward_backward");
  if (!params || !y0 || !loss) return fail(FBSDE_ERR_INVALID, "params, y0 and loss must be non-NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  st = run_forward(plan, params, y0, seed, iter, nullptr, ws, s);
  if (st != FBSDE_OK) return st;
  hipError_t e = fbsde::launch_loss_only(plan->geo, at<double>(ws, plan->ws.RED), plan->ws.scan_blocks, loss,
                                         plan->nf_host, s);
  if (e != hipSuccess) return hip_fail(e, "finalize");
  return FBSDE_OK;
}

fbsde_status fbsde_forward_backward(fbsde_plan* plan, const float* params, const double* y0, float* grad,
                                    double* grad_y0, double* loss, uint64_t seed, uint64_t iter, void* ws,
                                    void* stream) {
  fbsde_status st = check_hot(plan, ws);
  if (st != FBSDE_OK) return st;
  if (plan->geo.kind == 2) return fail(FBSDE_ERR_UNSUPPORTED, "u-network plans use fbsde_unet_forward_backward");
  if (!params || !y0 || !grad || !grad_y0 || !loss)
    return fail(FBSDE_ERR_INVALID, "params, y0, grad, grad_y0 and loss must be non-NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  st = run_forward(plan, params, y0, seed, iter, nullptr, ws, s);
  if (st != FBSDE_OK) return st;
  return run_backward(plan, grad, grad_y0, loss, ws, s);
}

fbsde_status fbsde_adam_step(fbsde_plan* plan, float* params, double* y0, const float* grad,
                             const double* grad_y0, float* m, float* v, double* m_y0, double* v_y0, int64_t t,
                             double lr, double lr_y0, double b1, double b2, double eps, void* stream) {
  if (!plan) return fail(FBSDE_ERR_INVALID, "plan is NULL");
  if (!params || !grad || !m || !v) return fail(FBSDE_ERR_INVALID, "params, grad, m, v must be non-NULL");
  const bool with_y0 = y0 != nullptr;
  if (with_y0 && (!grad_y0 || !m_y0 || !v_y0))
    return fail(FBSDE_ERR_INVALID, "y0 given without grad_y0, m_y0, v_y0");
  if (t < 1) return fail(FBSDE_ERR_INVALID, "Adam step count must be >= 1");
  if (fbsde_status st = take_nonfinite(plan); st != FBSDE_OK) return st;
  if (!(lr >= 0) || !(lr_y0 >= 0) || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1) || !(eps > 0))
    return fail(FBSDE_ERR_INVALID, "Adam hyper-parameters out of range");
  ProfScope ps(plan, FBSDE_PROF_ADAM, reinterpret_cast<hipStream_t>(stream));
  hipError_t e = fbsde::launch_adam(plan->geo.nparams, params, grad, m, v, y0, grad_y0, m_y0, v_y0, (float)lr,
                                    (double)t, nullptr, lr_y0, b1, b2, eps, reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "adam");
  return FBSDE_OK;
}

fbsde_status fbsde_train_step(fbsde_plan* plan, float* params, double* y0, float* grad, double* grad_y0,
                              double* loss, float* m, float* v, double* m_y0, double* v_y0, int64_t t, double lr,
                              double lr_y0, double b1, double b2, double eps, uint64_t seed, uint64_t iter, void* ws,
                              void* stream) {
  fbsde_status st = check_hot(plan, ws);
  if (st != FBSDE_OK) return st;
  if (plan->geo.kind == 2) return fail(FBSDE_ERR_UNSUPPORTED, "u-network plans use fbsde_unet_forward_backward");
  if (!params || !y0 || !grad || !grad_y0 || !loss || !m || !v || !m_y0 || !v_y0)
    return fail(FBSDE_ERR_INVALID, "every buffer must be non-NULL");
  if (t < 1) return fail(FBSDE_ERR_INVALID, "Adam step count must be >= 1");
  if (!(lr >= 0) || !(lr_y0 >= 0) || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1) || !(eps > 0))
    return fail(FBSDE_ERR_INVALID, "Adam hyper-parameters out of range");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  st = run_forward(plan, params, y0, seed, iter, nullptr, ws, s);
  if (st != FBSDE_OK) return st;
  const fbsde::AdamArgs a = {params, m, v, y0, m_y0, v_y0, lr, (double)t, nullptr, lr_y0, b1, b2, eps};
  return run_backward(plan, grad, grad_y0, loss, ws, s, &a);
}

fbsde_status fbsde_plan_set_unet_loss(fbsde_plan* plan, double kappa, double eps) {
  if (!plan) return fail(FBSDE_ERR_INVALID, "plan is NULL");
  if (plan->geo.kind != 2) return fail(FBSDE_ERR_INVALID, "not a u-network plan");
  if (!(kappa >= 0) || !std::isfinite(kappa) || !(eps >= 0) || !std::isfinite(eps))
    return fail(FBSDE_ERR_INVALID, "kappa and eps must be finite and >= 0");
  plan->geo.kappa = (float)kappa;
  plan->geo.ueps = (float)eps;
  return FBSDE_OK;
}

fbsde_status fbsde_unet_forward_backward(fbsde_plan* plan, const float* params, float* grad, double* loss,
                                         double* y0, uint64_t seed, uint64_t iter, void* ws, void* stream) {
  fbsde_status st = check_hot(plan, ws);
  if (st != FBSDE_OK) return st;
  if (plan->geo.kind != 2) return fail(FBSDE_ERR_INVALID, "not a u-network plan");
  if (!params || !loss) return fail(FBSDE_ERR_INVALID, "params and loss must be non-NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const Geo& g = plan->geo;
  const WsLayout& L = plan->ws;
  hipError_t e;
  {
    ProfScope ps(plan, FBSDE_PROF_SDE, s);
    if ((e = fbsde::launch_sde(g, plan->x0_dev, seed, iter, nullptr, at<float>(ws, L.X), at<float>(ws, L.V),
                               at<float>(ws, L.QN), at<float>(ws, L.LN), s)) != hipSuccess)
      return hip_fail(e, "sde");
  }
  const fbsde::UnetBufs B = unet_bufs(plan, ws);
  const long long rows = (long long)(g.N + 1) * g.M;
  int* nf = reinterpret_cast<int*>(B.lpart + (rows + 31) / 32);
  {
    ProfScope ps(plan, FBSDE_PROF_FORWARD, s);
    if ((e = fbsde::unet_forward_backward(g, B, params, grad, loss, y0, nf, plan->nf_host, grad != nullptr, s)) !=
        hipSuccess)
      return hip_fail(e, "u-network");
  }
  return FBSDE_OK;
}

fbsde_status fbsde_unet_nais_project(fbsde_plan* plan, float* params, double c, void* ws, void* stream) {
  fbsde_status st = check_hot(plan, ws);
  if (st != FBSDE_OK) return st;
  if (plan->geo.kind != 2 || plan->geo.uarch != 2) return fail(FBSDE_ERR_INVALID, "not a NAIS u-network plan");
  if (!params || !(c > 0) || !std::isfinite(c)) return fail(FBSDE_ERR_INVALID, "params NULL or c not > 0");
  hipError_t e = fbsde::unet_nais_project(plan->geo, unet_bufs(plan, ws), params, (float)c,
                                          reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "nais projection");
  return FBSDE_OK;
}

fbsde_status fbsde_unet_states(fbsde_plan* plan, const void* ws, float* u, float* z, void* stream) {
  fbsde_status st = check_hot(plan, ws);
  if (st != FBSDE_OK) return st;
  if (plan->geo.kind != 2) return fail(FBSDE_ERR_INVALID, "not a u-network plan");
  const Geo& g = plan->geo;
  const long long R = (long long)(g.N + 1) * g.M;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e;
  if (u && (e = hipMemcpyAsync(u, at<float>(ws, plan->ws.UU), (size_t)R * 4, hipMemcpyDeviceToDevice, s)) !=
               hipSuccess)
    return hip_fail(e, "copy u");
  if (z && (e = hipMemcpy2DAsync(z, (size_t)g.d * 4, at<float>(ws, plan->ws.UZ), (size_t)g.dp * 4, (size_t)g.d * 4,
                                 (size_t)R, hipMemcpyDeviceToDevice, s)) != hipSuccess)
    return hip_fail(e, "copy Z");
  return FBSDE_OK;
}

fbsde_status fbsde_plan_set_x0(fbsde_plan* plan, const double* x0_host) {
  if (!plan || !x0_host) return fail(FBSDE_ERR_INVALID, "NULL argument");
  if (!finite_all(x0_host, plan->geo.d)) return fail(FBSDE_ERR_INVALID, "x0 is not finite");
  std::vector<float> tmp((size_t)plan->geo.dp, 0.f);
  for (int i = 0; i < plan->geo.d; ++i) tmp[(size_t)i] = (float)x0_host[i];
  hipError_t e = hipMemcpy(plan->x0_dev, tmp.data(), tmp.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy x0");
  return FBSDE_OK;
}

fbsde_status fbsde_prolong(const fbsde_plan* coarse, const fbsde_plan* fine, const float* pc, float* pf,
                           void* stream) {
  if (!coarse || !fine || !pc || !pf) return fail(FBSDE_ERR_INVALID, "NULL argument");
  const Geo &a = coarse->geo, &b = fine->geo;
  if (b.N != 2 * a.N) return fail(FBSDE_ERR_INVALID, "fine plan must have twice the steps of the coarse plan");
  if (a.d != b.d || a.w != b.w || a.L != b.L || coarse->net.kind != fine->net.kind)
    return fail(FBSDE_ERR_INVALID, "coarse and fine plans must share the problem dimension and network");
  if (a.kind != 0) {  // one network shared by all steps: the fine grid keeps it unchanged
    hipError_t e = hipMemcpyAsync(pf, pc, (size_t)a.nparams * sizeof(float), hipMemcpyDeviceToDevice,
                                  reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "prolong copy");
    return FBSDE_OK;
  }
  if (a.N < 2) return fail(FBSDE_ERR_INVALID, "coarse grid needs at least 2 steps to hold a network");
  hipError_t e = fbsde::launch_prolong(a, b, pc, pf, reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "prolong");
  return FBSDE_OK;
}

fbsde_status fbsde_sample_normals(fbsde_plan* plan, uint64_t seed, uint64_t iter, float* xi, void* stream) {
  if (!plan || !xi) return fail(FBSDE_ERR_INVALID, "plan or xi is NULL");
  hipError_t e = fbsde::launch_normals(plan->geo, seed, iter, xi, reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "normals");
  return FBSDE_OK;
}

fbsde_status fbsde_terminal_mean(fbsde_plan* plan, uint64_t seed, uint64_t iter, double* mean, void* ws,
                                 void* stream) {
  fbsde_status st = check_hot(plan, ws);
  if (st != FBSDE_OK) return st;
  if (!mean) return fail(FBSDE_ERR_INVALID, "mean is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const Geo& g = plan->geo;
  const WsLayout& L = plan->ws;
  hipError_t e = fbsde::launch_sde(g, plan->x0_dev, seed, iter, nullptr, at<float>(ws, L.X), at<float>(ws, L.V),
                                   at<float>(ws, L.QN), at<float>(ws, L.LN), s);
  if (e != hipSuccess) return hip_fail(e, "sde");
  e = fbsde::launch_gmean(g, at<float>(ws, L.QN), at<float>(ws, L.LN), mean, s);
  if (e != hipSuccess) return hip_fail(e, "gmean");
  return FBSDE_OK;
}

fbsde_status fbsde_terminal_states(fbsde_plan* plan, const void* ws, float* xN, float* yN, void* stream) {
  fbsde_status st = check_hot(plan, ws);
  if (st != FBSDE_OK) return st;
  if (!xN && !yN) return FBSDE_OK;
  hipError_t e = fbsde::launch_terminal_copy(plan->geo, at<float>(ws, plan->ws.X), at<float>(ws, plan->ws.Y), xN,
                                             yN, reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "terminal copy");
  return FBSDE_OK;
}

fbsde_status fbsde_profile_enable(fbsde_plan* plan, int32_t enable) {
  if (!plan) return fail(FBSDE_ERR_INVALID, "plan is NULL");
  if (enable && !plan->prof) {
    for (int k = 0; k < FBSDE_PROF_NUM; ++k) {
      ProfRing& r = plan->ring[k];
      r.start.assign(ProfRing::R, nullptr);
      r.stop.assign(ProfRing::R, nullptr);
      r.used.assign(ProfRing::R, 0);
      r.head = 0;
      r.ms = 0.0;
      r.count = 0;
      for (int i = 0; i < ProfRing::R; ++i) {
        hipError_t e1 = hipEventCreate(&r.start[i]);
        hipError_t e2 = hipEventCreate(&r.stop[i]);
        if (e1 != hipSuccess || e2 != hipSuccess) return hip_fail(e1 != hipSuccess ? e1 : e2, "hipEventCreate");
      }
    }
    plan->prof = true;
  } else if (!enable && plan->prof) {
    for (int k = 0; k < FBSDE_PROF_NUM; ++k) {
      ProfRing& r = plan->ring[k];
      for (int i = 0; i < ProfRing::R; ++i) {
        if (r.used[i]) (void)hipEventSynchronize(r.stop[i]);
        if (r.start[i]) (void)hipEventDestroy(r.start[i]);
        if (r.stop[i]) (void)hipEventDestroy(r.stop[i]);
      }
      r.start.clear();
      r.stop.clear();
      r.used.clear();
    }
    plan->prof = false;
  }
  return FBSDE_OK;
}

fbsde_status fbsde_profile_read(fbsde_plan* plan, double* ms, int64_t* count, int32_t n) {
  if (!plan || !ms || !count) return fail(FBSDE_ERR_INVALID, "NULL argument");
  if (n < 0 || n > FBSDE_PROF_NUM) return fail(FBSDE_ERR_INVALID, "n out of range");
  if (!plan->prof) return fail(FBSDE_ERR_INVALID, "profiling is not enabled on this plan");
  for (int k = 0; k < FBSDE_PROF_NUM; ++k) {
    ProfRing& r = plan->ring[k];
    for (int i = 0; i < ProfRing::R; ++i) {
      if (!r.used[i]) continue;
      float t = 0.f;
      hipError_t e = hipEventSynchronize(r.stop[i]);
      if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
      e = hipEventElapsedTime(&t, r.start[i], r.stop[i]);
      if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
      r.ms += t;
      r.count += 1;
      r.used[i] = 0;
    }
    if (k < n) {
      ms[k] = r.ms;
      count[k] = r.count;
    }
    r.ms = 0.0;
    r.count = 0;
  }
  return FBSDE_OK;
}

// ------------------------------------------------------------------ tuning
fbsde_status fbsde_plan_config(fbsde_plan* plan, int32_t shape, int32_t lds, int32_t tpw, int32_t splits) {
  if (!plan) return fail(FBSDE_ERR_INVALID, "plan is NULL");
  if (plan->geo.kind == 2) return fail(FBSDE_ERR_UNSUPPORTED, "u-network plans have no tuning configurations");
  if (shape < 0 || shape >= plan->ncand) return fail(FBSDE_ERR_INVALID, "shape index out of range");
  if (tpw < 0 || tpw > 64 || splits < 0 || splits > kMaxTuneSplits)
    return fail(FBSDE_ERR_INVALID, "tiles per wave must be in [0, 64] and splits in [0, 32]");
  const Geo keep_g = plan->geo;
  const WsLayout keep_w = plan->ws;
  if (plan->geo.kind == 0) set_tiles(plan->geo, plan->cand_ti[shape], plan->cand_tw[shape]);
  plan->geo.lds = lds <= 0 ? 0 : (lds >= 2 ? 2 : 1);
  plan->geo.tpw = tpw;
  plan->ws.splits = splits;
  make_layout(plan);
  if (plan->ws.total > plan->reserve) {
    plan->geo = keep_g;
    plan->ws = keep_w;
    return fail(FBSDE_ERR_INVALID, "configuration does not fit the reserved workspace");
  }
  return FBSDE_OK;
}

fbsde_status fbsde_plan_status(fbsde_plan* plan) {
  if (!plan) return fail(FBSDE_ERR_INVALID, "plan is NULL");
  return take_nonfinite(plan);
}

fbsde_status fbsde_plan_set_checkpointing(fbsde_plan* plan, int32_t recompute, int64_t chunk_rows) {
  if (!plan) return fail(FBSDE_ERR_INVALID, "plan is NULL");
  if (chunk_rows < 0) return fail(FBSDE_ERR_INVALID, "chunk_rows must be >= 0");
  if (plan->geo.kind == 2) {
    if (recompute) return fail(FBSDE_ERR_UNSUPPORTED, "the u-network does not recompute activations");
    return FBSDE_OK;
  }
  const int steps = rn_chunk_steps(plan->N, plan->M, chunk_rows > 0 ? chunk_rows : kDefaultChunkRows);
  if (plan->geo.kind == 1 && !rn_offsets_fit(plan->M, steps, plan->geo.w, plan->geo.d))
    return fail(FBSDE_ERR_UNSUPPORTED, "chunk too large for 32-bit element offsets");
  const Geo keep_g = plan->geo;
  const WsLayout keep_w = plan->ws;
  const size_t keep_r = plan->reserve;
  if (plan->geo.kind == 1) {
    plan->geo.rn_chunk = steps;
    plan->geo.rn_store = recompute ? 0 : 1;
  } else {
    plan->geo.rn_chunk = recompute ? steps : 0;  // per-step MLP: 0 keeps every step's activations
  }
  make_layout(plan);
  size_t r = reserve_bytes(plan);
  if (r < plan->ws.total) r = plan->ws.total;
  if (plan->ws_queried && r > keep_r) {  // a caller's buffer sized earlier would be too small
    plan->geo = keep_g;
    plan->ws = keep_w;
    return fail(FBSDE_ERR_INVALID, "checkpointing mode needs a larger workspace: set it before fbsde_workspace_size");
  }
  plan->reserve = r > keep_r || !plan->ws_queried ? r : keep_r;
  return FBSDE_OK;
}

fbsde_status fbsde_plan_get_config(const fbsde_plan* plan, int32_t* cfg_host /* [6] */) {
  if (!plan || !cfg_host) return fail(FBSDE_ERR_INVALID, "NULL argument");
  int shape = 0;
  for (int c = 0; c < plan->ncand; ++c)
    if (plan->cand_ti[c] == plan->geo.ti && plan->cand_tw[c] == plan->geo.tw) shape = c;
  cfg_host[0] = shape;
  cfg_host[1] = plan->geo.ti;
  cfg_host[2] = plan->geo.tw;
  cfg_host[3] = plan->geo.lds;
  cfg_host[4] = plan->geo.tpw > 0 ? plan->geo.tpw : fbsde::auto_tiles_per_wave(plan->geo);
  cfg_host[5] = plan->ws.splits;
  return FBSDE_OK;
}

fbsde_status fbsde_plan_autotune(fbsde_plan* plan, const float* params, const double* y0, float* grad,
                                 double* grad_y0, double* loss, void* ws, void* stream, int32_t reps) {
  fbsde_status st = check_hot(plan, ws);
  if (st != FBSDE_OK) return st;
  if (!params || !y0 || !grad || !grad_y0 || !loss) return fail(FBSDE_ERR_INVALID, "NULL buffer");
  if (reps < 1) reps = 1;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const bool prof = plan->prof;
  plan->prof = false;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    plan->prof = prof;
    return fail(FBSDE_ERR_HIP, "hipEventCreate");
  }
  auto timed = [&](float* ms) -> fbsde_status {
    fbsde_status r = fbsde_forward_backward(plan, params, y0, grad, grad_y0, loss, 0, 0, ws, stream);  // warm
    if (r != FBSDE_OK) return r;
    (void)hipEventRecord(e0, s);
    for (int k = 0; k < reps; ++k) {
      r = fbsde_forward_backward(plan, params, y0, grad, grad_y0, loss, 0, (uint64_t)k, ws, stream);
      if (r != FBSDE_OK) return r;
    }
    (void)hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess) return fail(FBSDE_ERR_HIP, "hipEventSynchronize");
    (void)hipEventElapsedTime(ms, e0, e1);
    return FBSDE_OK;
  };
  int best[4] = {0, 2, 0, 0};  // shape, lds, tpw, splits
  float best_ms = 1e30f;
  auto trial = [&](int sh, int l, int tp, int sp) -> fbsde_status {
    if (fbsde_plan_config(plan, sh, l, tp, sp) != FBSDE_OK) return FBSDE_OK;  // skip what does not fit
    float ms = 0.f;
    fbsde_status r = timed(&ms);
    if (r != FBSDE_OK) return r;
    if (ms < best_ms) {
      best_ms = ms;
      best[0] = sh; best[1] = l; best[2] = tp; best[3] = sp;
    }
    return FBSDE_OK;
  };
  fbsde_status r = FBSDE_OK;
  // 1. register-tile shape and LDS mode (2 = fused reverse where it applies, 1, 0)
  for (int sh = 0; sh < plan->ncand && r == FBSDE_OK; ++sh)
    for (int l = 2; l >= 0 && r == FBSDE_OK; --l) r = trial(sh, l, 0, 0);
  // 2. tiles per wave of the LDS kernels
  if (r == FBSDE_OK && best[1]) {
    fbsde_plan_config(plan, best[0], best[1], 0, 0);
    const int a = fbsde::auto_tiles_per_wave(plan->geo);
    const int cand[3] = {a > 1 ? a / 2 : 0, a * 2 <= 64 ? a * 2 : 0, a > 2 ? a - 1 : 0};
    for (int c = 0; c < 3 && r == FBSDE_OK; ++c)
      if (cand[c] > 0) r = trial(best[0], best[1], cand[c], 0);
  }
  // 3. weight-gradient path splits
  for (int sp : {4, 8, 16, 32}) {
    if (r != FBSDE_OK) break;
    if ((long long)sp * 64 > plan->M) continue;
    r = trial(best[0], best[1], best[2], sp);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  plan->prof = prof;
  if (r != FBSDE_OK) return r;
  return fbsde_plan_config(plan, best[0], best[1], best[2], best[3]);
}

}  // extern "C"

// ------------------------------------------------------------------ batches
struct fbsde_batch {
  std::vector<fbsde_batch_item> items;
  double lr, lr_y0, b1, b2, eps;
  uint64_t* iter_dev;
  hipStream_t cap = nullptr;
  std::vector<hipStream_t> branch;
  std::vector<hipEvent_t> events;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

void batch_free(fbsde_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (hipEvent_t e : b->events) (void)hipEventDestroy(e);
  for (hipStream_t s : b->branch) (void)hipStreamDestroy(s);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
}

// One training step of instance `it` on stream s, with the iteration read
// from the device counter.
fbsde_status batch_item_step(fbsde_batch* b, const fbsde_batch_item& it, hipStream_t s) {
  fbsde_status st = run_forward(it.plan, it.params_dev, it.y0_dev, it.seed, 0, b->iter_dev, it.ws_dev, s);
  if (st != FBSDE_OK) return st;
  // the reduction applies Adam (step iter_dev[0] + 1) in the same launch
  const fbsde::AdamArgs a = {it.params_dev, it.m_dev, it.v_dev, it.y0_dev, it.m_y0_dev, it.v_y0_dev,
                             b->lr, 1.0, b->iter_dev, b->lr_y0, b->b1, b->b2, b->eps};
  return run_backward(it.plan, it.grad_dev, it.grad_y0_dev, it.loss_dev, it.ws_dev, s, &a);
}

}  // namespace

extern "C" {

fbsde_status fbsde_batch_create(const fbsde_batch_item* items, int32_t n, double lr, double lr_y0, double b1,
                                double b2, double eps, uint64_t* iter_dev, int32_t autotune, void* stream,
                                fbsde_batch** out) {
  if (!out) return fail(FBSDE_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!items || n < 1) return fail(FBSDE_ERR_INVALID, "need at least one item");
  if (!iter_dev) return fail(FBSDE_ERR_INVALID, "iter_dev is NULL");
  if (!(lr >= 0) || !(lr_y0 >= 0) || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1) || !(eps > 0))
    return fail(FBSDE_ERR_INVALID, "Adam hyper-parameters out of range");
  for (int i = 0; i < n; ++i) {
    const fbsde_batch_item& it = items[i];
    fbsde_status st = check_hot(it.plan, it.ws_dev);
    if (st != FBSDE_OK) return st;
    if (it.plan->geo.kind == 2) return fail(FBSDE_ERR_UNSUPPORTED, "batches hold Deep-BSDE plans only");
    if (!it.params_dev || !it.y0_dev || !it.grad_dev || !it.grad_y0_dev || !it.loss_dev || !it.m_dev ||
        !it.v_dev || !it.m_y0_dev || !it.v_y0_dev)
      return fail(FBSDE_ERR_INVALID, "batch item " + std::to_string(i) + " has a NULL buffer");
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  for (int i = 0; i < n && autotune; ++i) {
    const fbsde_batch_item& it = items[i];
    fbsde_status st = fbsde_plan_autotune(it.plan, it.params_dev, it.y0_dev, it.grad_dev, it.grad_y0_dev,
                                          it.loss_dev, it.ws_dev, stream, 3);
    if (st != FBSDE_OK) return st;
  }
  // eager pass: first launches of every kernel happen outside the capture
  for (int i = 0; i < n; ++i) {
    const fbsde_batch_item& it = items[i];
    fbsde_status st = fbsde_forward_backward(it.plan, it.params_dev, it.y0_dev, it.grad_dev, it.grad_y0_dev,
                                             it.loss_dev, it.seed, 0, it.ws_dev, stream);
    if (st != FBSDE_OK) return st;
  }
  if (hipStreamSynchronize(s) != hipSuccess) return fail(FBSDE_ERR_HIP, "hipStreamSynchronize");

  fbsde_batch* b = new (std::nothrow) fbsde_batch();
  if (!b) return fail(FBSDE_ERR_NOMEM, "host allocation failed");
  b->items.assign(items, items + n);
  b->lr = lr; b->lr_y0 = lr_y0; b->b1 = b1; b->b2 = b2; b->eps = eps;
  b->iter_dev = iter_dev;
  const int nb = n < 4 ? n : 4;  // independent instances run on parallel graph branches
  hipError_t e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  for (int k = 0; k < nb && e == hipSuccess; ++k) {
    hipStream_t bs = nullptr;
    e = hipStreamCreateWithFlags(&bs, hipStreamNonBlocking);
    if (e == hipSuccess) b->branch.push_back(bs);
  }
  for (int k = 0; k < nb + 1 && e == hipSuccess; ++k) {
    hipEvent_t ev = nullptr;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) b->events.push_back(ev);
  }
  if (e != hipSuccess) {
    batch_free(b);
    return hip_fail(e, "batch streams/events");
  }
  std::vector<char> prof(n);
  for (int i = 0; i < n; ++i) {
    prof[i] = items[i].plan->prof;
    items[i].plan->prof = false;
  }
  fbsde_status st = FBSDE_OK;
  e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    // fork: every branch waits for the start of the capture stream
    (void)hipEventRecord(b->events[nb], b->cap);
    for (int k = 0; k < nb; ++k) (void)hipStreamWaitEvent(b->branch[k], b->events[nb], 0);
    for (int i = 0; i < n && st == FBSDE_OK; ++i) st = batch_item_step(b, b->items[i], b->branch[i % nb]);
    // join, then advance the device iteration counter
    for (int k = 0; k < nb; ++k) {
      (void)hipEventRecord(b->events[k], b->branch[k]);
      (void)hipStreamWaitEvent(b->cap, b->events[k], 0);
    }
    if (st == FBSDE_OK) {
      hipError_t ec = fbsde::launch_count(iter_dev, b->cap);
      if (ec != hipSuccess) st = hip_fail(ec, "count");
    }
    hipError_t ee = hipStreamEndCapture(b->cap, &b->graph);
    if (ee != hipSuccess && st == FBSDE_OK) st = hip_fail(ee, "hipStreamEndCapture");
  } else {
    st = hip_fail(e, "hipStreamBeginCapture");
  }
  for (int i = 0; i < n; ++i) items[i].plan->prof = prof[i];
  if (st == FBSDE_OK) {
    e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) st = hip_fail(e, "hipGraphInstantiate");
  }
  if (st != FBSDE_OK) {
    batch_free(b);
    return st;
  }
  *out = b;
  return FBSDE_OK;
}

fbsde_status fbsde_batch_step(fbsde_batch* b, void* stream) {
  if (!b || !b->exec) return fail(FBSDE_ERR_INVALID, "batch is NULL");
  // a non-finite result of an earlier step of any instance (see the plans' flags)
  for (const fbsde_batch_item& it : b->items)
    if (fbsde_status st = take_nonfinite(it.plan); st != FBSDE_OK) return st;
  hipError_t e = hipGraphLaunch(b->exec, reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return FBSDE_OK;
}

void fbsde_batch_destroy(fbsde_batch* b) { batch_free(b); }

}  // extern "C"
