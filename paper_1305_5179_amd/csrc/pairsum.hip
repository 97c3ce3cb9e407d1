// Gaussian pair sums y_t = sum_j w_j phi(|x_t - x_j|) over the source list of
// every target group: the operator of Sec. II.B eq. RBFsys (targets =
// centres) and the evaluation of eq. matxvet (targets = grid nodes or
// points), truncated as in Sec. III.A.
//
// float32 path.  Coordinates are scaled by sqrt(log2(e) / (2 sigma^2)) so that
// phi = exp2(-d) with d the scaled squared distance, and taken relative to
// the group's anchor before rounding to float32 (the rounding error then
// scales with the distance to the anchor, not with the cloud's extent).
// Per pair: 3 subtractions (source broadcast by DPP), 1 multiply, 2 FMAs,
// one v_exp_f32 and one FMA of the broadcast weight.  "Inner" chunks (every
// pair inside the cutoff) skip the truncation test; "outer" chunks add it:
// v = H (T - d) with H = 2^30 has the exact sign of T - d, min(-d, v) keeps
// -d inside the cutoff and sends the exponent to a huge negative value
// outside.  When |T - d| is within the float32 error bound of d the lane
// recomputes r^2 in float64 from the unscaled coordinates and takes the
// float64 decision, so the truncation is the float64 one everywhere.
//
// float64 path: the same lists; sources broadcast through LDS; r^2 and the
// cutoff test exactly as the float64 definition; exp from the device library.
#include "common.h"

namespace rbf {

namespace {

constexpr float kH = 1073741824.0f;  // 2^30

struct PairArgs {
  const double4* tpts;
  const GroupInfo* groups;
  const uint32_t* list;
  int64_t G;
  const double4* xk;   // scaled sources (float32 path)
  const double4* xs;   // unscaled sources
  const double* w;
  int64_t m;
  double sqrt_k;
  double inv_two_s2;
  double rc2;
  double Tk;           // scaled cutoff^2, k r_c^2 (float64)
  float TH;            // T * H, T = scaled cutoff^2 in float32
  int dense;
  int out_f32;
  void* out;
  const int64_t* out_index;
  const int* skip;
};

// Block b of the launch runs on XCD b % 8; give every XCD a contiguous range
// of groups so that neighbouring groups (which share sources) share an L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb) {
  const int64_t q = nb / 8, r = nb % 8, x = b % 8;
  const int64_t first = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
  return first + b / 8;
}

template <int K>
__device__ __forceinline__ float bcast(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x150 + K, 0xf, 0xf, true));
}

// acc += (weight held by lane K of this row) * e as one v_fmac_f32 with a
// DPP row_newbcast source.  The compiler does not look inside inline asm for
// hazards, so the asm carries its own wait states:
//   * a VALU reading the result of a transcendental (the v_exp_f32 that made
//     e) needs one wait state on gfx950: s_nop 0 before every use;
//   * a DPP source register needs two wait states after a VALU write; the
//     weight is written once per chunk, before its first use, which gets
//     s_nop 1 (covering both).
template <int K>
__device__ __forceinline__ void fmac_bcast(float& acc, float wt, float e) {
  if constexpr (K == 0) {
    asm volatile("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 row_newbcast:0 row_mask:0xf bank_mask:0xf bound_ctrl:1"
                 : "+v"(acc) : "v"(wt), "v"(e));
  } else {
    asm volatile("s_nop 0\n\tv_fmac_f32_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf bound_ctrl:1"
                 : "+v"(acc) : "v"(wt), "v"(e), "i"(K));
  }
}

template <int K>
__device__ __forceinline__ float sqdist_bcast(float tx, float ty, float tz, float sx, float sy, float sz) {
  const float dx = bcast<K>(sx) - tx;
  const float dy = bcast<K>(sy) - ty;
  const float dz = bcast<K>(sz) - tz;
  float d = dx * dx;
  d = __builtin_fmaf(dy, dy, d);
  d = __builtin_fmaf(dz, dz, d);
  return d;
}

template <int K>
__device__ __forceinline__ void step_inner(float& acc, float tx, float ty, float tz, float sx, float sy, float sz,
                                           float sw) {
  const float d = sqdist_bcast<K>(tx, ty, tz, sx, sy, sz);
  const float e = __builtin_amdgcn_exp2f(-d);
  fmac_bcast<K>(acc, sw, e);
}

// float64 decision for the lanes whose float32 distance is too close to the
// cutoff to decide.
__device__ __forceinline__ float resolve_f64(const PairArgs& a, int64_t tid, uint32_t idx, int row, int K,
                                                       float d) {
  const uint32_t i0 = __builtin_amdgcn_readlane(idx, K);
  const uint32_t i1 = __builtin_amdgcn_readlane(idx, 16 + K);
  const uint32_t i2 = __builtin_amdgcn_readlane(idx, 32 + K);
  const uint32_t i3 = __builtin_amdgcn_readlane(idx, 48 + K);
  const uint32_t src = row == 0 ? i0 : row == 1 ? i1 : row == 2 ? i2 : i3;
  const double4 t = a.tpts[tid];
  const double4 s = a.xs[src];
  const double dx = t.x - s.x, dy = t.y - s.y, dz = t.z - s.z;
  const double r2 = (dx * dx + dy * dy) + dz * dz;
  return r2 <= a.rc2 ? -d : -INFINITY;
}

// Outer chunk without risky sources: every pair is farther than the band
// from the cutoff, so the float32 test decides as float64 does.
template <int K>
__device__ __forceinline__ void step_outer(float& acc, float tx, float ty, float tz, float sx, float sy, float sz,
                                           float sw, float th) {
  const float d = sqdist_bcast<K>(tx, ty, tz, sx, sy, sz);
  const float v = __builtin_fmaf(d, -kH, th);
  const float e = __builtin_amdgcn_exp2f(__builtin_fminf(-d, v));
  fmac_bcast<K>(acc, sw, e);
}

template <int K>
__device__ __forceinline__ void step_risky(float& acc, float tx, float ty, float tz, float sx, float sy, float sz,
                                           float sw, float th, float gh, const PairArgs& a, int64_t tid, uint32_t idx,
                                           int row) {
  const float d = sqdist_bcast<K>(tx, ty, tz, sx, sy, sz);
  const float v = __builtin_fmaf(d, -kH, th);
  float arg = __builtin_fminf(-d, v);
  const bool amb = __builtin_fabsf(v) <= gh;
  if (__builtin_expect(__builtin_amdgcn_ballot_w64(amb) != 0, 0)) {
    if (amb) arg = resolve_f64(a, tid, idx, row, K, d);
  }
  const float e = __builtin_amdgcn_exp2f(arg);
  fmac_bcast<K>(acc, sw, e);
}

#define RBF_STEPS(F, ...) \
  F<0>(__VA_ARGS__); F<1>(__VA_ARGS__); F<2>(__VA_ARGS__); F<3>(__VA_ARGS__); \
  F<4>(__VA_ARGS__); F<5>(__VA_ARGS__); F<6>(__VA_ARGS__); F<7>(__VA_ARGS__); \
  F<8>(__VA_ARGS__); F<9>(__VA_ARGS__); F<10>(__VA_ARGS__); F<11>(__VA_ARGS__); \
  F<12>(__VA_ARGS__); F<13>(__VA_ARGS__); F<14>(__VA_ARGS__); F<15>(__VA_ARGS__)

__device__ __forceinline__ void store_result(const PairArgs& a, int64_t tid, double v) {
  if (a.out_f32)
    static_cast<float*>(a.out)[a.out_index[tid]] = (float)v;
  else
    static_cast<double*>(a.out)[a.out_index[tid]] = v;
}

__device__ __forceinline__ uint32_t list_entry(const PairArgs& a, const GroupInfo& gi, int c, int lane) {
  if (a.dense) {
    const int64_t e = (int64_t)c * kChunk + lane;
    return e < a.m ? (uint32_t)e : (uint32_t)a.m;
  }
  return a.list[gi.off + (int64_t)c * kChunk + lane];
}

__global__ __launch_bounds__(kBlock) void k_pairsum_f32(PairArgs a) {
  // the wave index is uniform across the wave: keep it (and all group data) scalar
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63, row = lane >> 4, tl = lane & 15;
  const int64_t g = xcd_remap(blockIdx.x, gridDim.x) * 4 + wave;
  if (g >= a.G) return;
  if (a.skip && *a.skip) return;
  const GroupInfo gi = a.groups[g];
  const int64_t tid = g * kGroup + tl;
  const double4 tp = a.tpts[tid];
  const float tx = (float)((tp.x - gi.ax) * a.sqrt_k);
  const float ty = (float)((tp.y - gi.ay) * a.sqrt_k);
  const float tz = (float)((tp.z - gi.az) * a.sqrt_k);
  const double akx = gi.ax * a.sqrt_k, aky = gi.ay * a.sqrt_k, akz = gi.az * a.sqrt_k;
  // the truncation threshold T*H held in a VGPR (v_fma_f32 takes it as its addend)
  float th;
  asm volatile("v_mov_b32 %0, %1" : "=v"(th) : "s"(a.TH));
  // ambiguity half-width of this group, times H
  const float gh = (float)(f32_cutoff_band(a.Tk, gi.radius * a.sqrt_k) * (double)kH);
  float acc = 0.0f;
  const int nch = gi.n_chunks, nin = gi.n_inner, nrisk = gi.first_risky;
  // Software pipeline over the chunks: the list index two chunks ahead and
  // the source gather one chunk ahead are in flight while a chunk computes.
  uint32_t idx_next = nch > 0 ? list_entry(a, gi, 0, lane) : (uint32_t)a.m;
  double4 s_next = a.xk[idx_next];
  double w_next = a.w[idx_next];
  uint32_t idx_after = nch > 1 ? list_entry(a, gi, 1, lane) : (uint32_t)a.m;
  for (int c = 0; c < nch; ++c) {
    const uint32_t idx = idx_next;
    const float sx = (float)(s_next.x - akx), sy = (float)(s_next.y - aky), sz = (float)(s_next.z - akz);
    const float sw = (float)w_next;
    if (c + 1 < nch) {
      idx_next = idx_after;
      s_next = a.xk[idx_next];
      w_next = a.w[idx_next];
    }
    if (c + 2 < nch) idx_after = list_entry(a, gi, c + 2, lane);
    if (c < nin) {
      RBF_STEPS(step_inner, acc, tx, ty, tz, sx, sy, sz, sw);
    } else if (c < nrisk) {
      RBF_STEPS(step_outer, acc, tx, ty, tz, sx, sy, sz, sw, th);
    } else {
      RBF_STEPS(step_risky, acc, tx, ty, tz, sx, sy, sz, sw, th, gh, a, tid, idx, row);
    }
  }
  acc += __shfl_xor(acc, 16);
  acc += __shfl_xor(acc, 32);
  if (row == 0 && tp.w != 0.0) store_result(a, tid, (double)acc);
}

__global__ __launch_bounds__(kBlock) void k_pairsum_f64(PairArgs a) {
  __shared__ double4 sh[kBlock / kWave][kWave];
  // the wave index is uniform across the wave: keep it (and all group data) scalar
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63, row = lane >> 4, tl = lane & 15;
  const int64_t g = xcd_remap(blockIdx.x, gridDim.x) * 4 + wave;
  if (g >= a.G) return;
  if (a.skip && *a.skip) return;
  const GroupInfo gi = a.groups[g];
  const int64_t tid = g * kGroup + tl;
  const double4 tp = a.tpts[tid];
  double acc = 0.0;
  const int nch = gi.n_chunks, nin = gi.n_inner;
  const double c2 = a.inv_two_s2;
  for (int c = 0; c < nch; ++c) {
    const uint32_t idx = list_entry(a, gi, c, lane);
    const double4 s = a.xs[idx];
    sh[wave][lane] = make_double4(s.x, s.y, s.z, a.w[idx]);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const double4* q = &sh[wave][row * kGroup];
    if (c < nin) {
#pragma unroll 4
      for (int k = 0; k < kGroup; ++k) {
        const double4 p = q[k];
        const double dx = tp.x - p.x, dy = tp.y - p.y, dz = tp.z - p.z;
        const double r2 = (dx * dx + dy * dy) + dz * dz;
        acc = fma(p.w, exp(-r2 * c2), acc);
      }
    } else {
#pragma unroll 4
      for (int k = 0; k < kGroup; ++k) {
        const double4 p = q[k];
        const double dx = tp.x - p.x, dy = tp.y - p.y, dz = tp.z - p.z;
        const double r2 = (dx * dx + dy * dy) + dz * dz;
        const double e = r2 <= a.rc2 ? exp(-r2 * c2) : 0.0;
        acc = fma(p.w, e, acc);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  acc += __shfl_xor(acc, 16);
  acc += __shfl_xor(acc, 32);
  if (row == 0 && tp.w != 0.0) store_result(a, tid, acc);
}

PairArgs make_args(const Ctx& c, const TargetSet& ts, const double* w, bool out_f32, void* out,
                   const int* skip) {
  PairArgs a;
  a.tpts = ts.pts;
  a.groups = ts.groups;
  a.list = ts.list;
  a.G = ts.n_groups;
  a.xk = c.xk;
  a.xs = c.xs;
  a.w = w;
  a.m = c.m;
  a.sqrt_k = c.sqrt_k;
  a.inv_two_s2 = c.inv_two_s2;
  a.rc2 = c.rc2;
  a.dense = ts.dense ? 1 : 0;
  a.out_f32 = out_f32 ? 1 : 0;
  a.out = out;
  a.out_index = ts.index;
  a.skip = skip;
  // Scaled cutoff T = k r_c^2 (the per-group ambiguity band is
  // f32_cutoff_band(T, scaled group radius)).
  if (std::isfinite(c.rc2)) {
    a.Tk = c.rc2 * c.sqrt_k * c.sqrt_k;
    a.TH = (float)(a.Tk) * kH;
  } else {
    a.Tk = INFINITY;
    a.TH = INFINITY;
  }
  return a;
}

// Launch timing (rbf_profile_begin / rbf_profile_end).
struct ProfRec {
  hipEvent_t a, b;
  int kind, prec;
  int64_t useful, examined;
};
struct Profiler {
  bool on = false;
  std::vector<ProfRec> recs;
};
Profiler& profiler() {
  static Profiler p;
  return p;
}

struct ProfScope {
  ProfRec rec{};
  bool on;
  hipStream_t s;
  ProfScope(int prec, const TargetSet& ts, hipStream_t st) : on(profiler().on), s(st) {
    if (!on) return;
    rec.prec = prec;
    rec.kind = ts.kind;
    rec.useful = ts.useful;
    rec.examined = ts.list_entries * kGroup;
    RBF_HIP(hipEventCreate(&rec.a));
    RBF_HIP(hipEventCreate(&rec.b));
    RBF_HIP(hipEventRecord(rec.a, s));
  }
  void done() {
    if (!on) return;
    RBF_HIP(hipEventRecord(rec.b, s));
    profiler().recs.push_back(rec);
  }
};

}  // namespace

int profile_begin() {
  Profiler& p = profiler();
  for (auto& r : p.recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  p.recs.clear();
  p.on = true;
  return RBF_OK;
}

int profile_end(rbf_profile* out) {
  Profiler& p = profiler();
  p.on = false;
  rbf_profile r{};
  for (auto& q : p.recs) {
    RBF_HIP(hipEventSynchronize(q.b));
    float ms = 0.f;
    RBF_HIP(hipEventElapsedTime(&ms, q.a, q.b));
    r.launches[q.kind][q.prec] += 1;
    r.kernel_ms[q.kind][q.prec] += ms;
    r.useful_pairs[q.kind][q.prec] += q.useful;
    r.examined_pairs[q.kind][q.prec] += q.examined;
    (void)hipEventDestroy(q.a);
    (void)hipEventDestroy(q.b);
  }
  p.recs.clear();
  if (out) *out = r;
  return RBF_OK;
}

void pairsum_f32(const Ctx& c, const TargetSet& ts, const double* w, bool out_f32, void* out, hipStream_t s,
                 const int* skip) {
  if (ts.n_groups == 0) return;
  PairArgs a = make_args(c, ts, w, out_f32, out, skip);
  const int64_t nb = ceil_div(ts.n_groups, kBlock / kWave);
  ProfScope prof(RBF_FP32, ts, s);
  hipLaunchKernelGGL(k_pairsum_f32, dim3((unsigned)nb), dim3(kBlock), 0, s, a);
  RBF_HIP(hipGetLastError());
  prof.done();
}

void pairsum_f64(const Ctx& c, const TargetSet& ts, const double* w, bool out_f32, void* out, hipStream_t s,
                 const int* skip) {
  if (ts.n_groups == 0) return;
  PairArgs a = make_args(c, ts, w, out_f32, out, skip);
  const int64_t nb = ceil_div(ts.n_groups, kBlock / kWave);
  ProfScope prof(RBF_FP64, ts, s);
  hipLaunchKernelGGL(k_pairsum_f64, dim3((unsigned)nb), dim3(kBlock), 0, s, a);
  RBF_HIP(hipGetLastError());
  prof.done();
}

}  // namespace rbf
