// Gaussian pair sums y_t = sum_j w_j phi(|x_t - x_j|) over the source list of
// every target group: the operator of Sec. II.B eq. RBFsys (targets =
// centres) and the evaluation of eq. matxvet (targets = grid nodes or
// points), truncated as in Sec. III.A.
//
// float32 path.  Coordinates are scaled by sqrt(log2(e) / (2 sigma^2)) so that
// phi = exp2(-d) with d the scaled squared distance, and taken relative to
// the group's anchor before rounding to float32 (the rounding error then
// scales with the distance to the anchor, not with the cloud's extent).
// A wave holds the 16 targets of a group in each of its four 16-lane rows;
// every lane loads one source of a 64-entry chunk of the group's list and a
// DPP row_newbcast hands source k of each row to all 16 lanes at step k.
//
// Expanded form (lists of bounded extent): d = |t|^2 + |s|^2 - 2 t.s, so
// phi = 2^{-|t|^2} 2^{2 t.s} 2^{-|s|^2}; the source factor is folded into the
// weight once per chunk, the target factor into the result, and a pair costs
// one DPP multiply and two DPP FMAs (2 t.s), one v_exp_f32 and the DPP FMA of
// the weight.
// Direct form (dense lists, and groups too wide for the expanded form's
// exponent range): three DPP subtractions, a multiply and two FMAs, the
// exponential and the weight FMA.
// Truncation: chunks of inner sources (inside the cutoff for every target)
// need no test; in every other chunk a v_cndmask with the 64-bit lane mask
// of the step (the float64 decisions of the list builder, loaded by scalar
// loads) zeroes the terms of the pairs outside the cutoff.
//
// float64 path: the same lists; sources broadcast through LDS.  Groups in
// the expanded form's range take it in float64 with the same lane masks and
// a Taylor-series exp2 (one FMA chain per pair); dense lists and wide groups
// form r^2 and the cutoff test exactly as the float64 definition, with exp
// from the device library.
#include "cells.h"

namespace rbf {

namespace {

struct PairArgs {
  const double4* tpts;
  const GroupInfo* groups;
  const uint32_t* list;
  const uint64_t* mask;  // per-step lane masks of the non-inner chunks
  const int32_t* order;  // launch order of the groups, or null (identity)
  int64_t G;
  const double4* xk;     // scaled sources (float32 path)
  const double4* xs;     // unscaled sources
  const double* w;
  const float* w32;      // float32 weights instead of w (float32 path), or null
  int64_t m;
  double sqrt_k;
  double inv_two_s2;
  double rc2;
  double Tk;             // scaled cutoff^2, k r_c^2
  double sqrt_T;         // scaled cutoff (as the list builder computes it)
  int dense;
  int out_f32;
  void* out;
  const int64_t* out_index;
  const int* skip;
};

// Word 3 of a raw buffer descriptor on gfx9 (32-bit data format, no swizzle).
constexpr int kBufferDword3 = 0x00020000;

template <int K>
__device__ __forceinline__ float bcast(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x150 + K, 0xf, 0xf, true));
}

// acc += (src held by lane K of this row) * other as one v_fmac_f32 with a
// DPP row_newbcast source.  The compiler does not look inside inline asm for
// hazards, so the asm carries its own wait states:
//   * a DPP source register needs two wait states after a VALU write; the
//     per-chunk source values are written once per chunk, before their first
//     use at K = 0, which gets s_nop 1;
//   * a VALU reading the result of a transcendental (`other` may come
//     straight from v_exp_f32) needs one wait state on gfx950: s_nop 0.
template <int K>
__device__ __forceinline__ void fmac_bcast(float& acc, float src, float other) {
  if constexpr (K == 0) {
    asm volatile("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 row_newbcast:0 row_mask:0xf bank_mask:0xf bound_ctrl:1"
                 : "+v"(acc) : "v"(src), "v"(other));
  } else {
    asm volatile("s_nop 0\n\tv_fmac_f32_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf bound_ctrl:1"
                 : "+v"(acc) : "v"(src), "v"(other), "i"(K));
  }
}

// Direct form: a lane's target and the source it contributes to the chunk
// (anchor-relative, scaled, float32).
struct Tgt {
  float x, y, z;
};
struct Src {
  float x, y, z;
  float w;
};

// ---- direct form ----------------------------------------------------------
template <int K>
__device__ __forceinline__ float sqdist_bcast(const Tgt& t, const Src& s) {
  const float dx = bcast<K>(s.x) - t.x;
  const float dy = bcast<K>(s.y) - t.y;
  const float dz = bcast<K>(s.z) - t.z;
  float d = dx * dx;
  d = __builtin_fmaf(dy, dy, d);
  d = __builtin_fmaf(dz, dz, d);
  return d;
}

template <int K>
__device__ __forceinline__ void direct_inner(float& acc, const Tgt& t, const Src& s) {
  const float d = sqdist_bcast<K>(t, s);
  fmac_bcast<K>(acc, s.w, __builtin_amdgcn_exp2f(-d));
}

// The 16 lane masks of a chunk in scalar registers.  They are read through
// the constant address space (the list builder wrote them in an earlier
// launch; nothing writes them during this one), which lets the compiler use
// scalar loads for the uniform address.
struct StepMasks {
  uint64_t m[16];
};
typedef const __attribute__((address_space(4))) uint64_t* ConstU64;
__device__ __forceinline__ StepMasks load_masks(const uint64_t* mk) {
  // the address is uniform; read-first-lane states it, so that the loads are
  // scalar whatever the compiler proves about where the pointer came from
  // (read-first-lane returns int: go through uint32_t, or bit 31 of the low
  // word would be sign-extended into the high word)
  const uint64_t u = (uint64_t)mk;
  const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)u);
  const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
  const ConstU64 p = (ConstU64)((hi << 32) | lo);
  StepMasks r;
#pragma unroll
  for (int k = 0; k < 16; ++k) r.m[k] = p[k];
  return r;
}

template <int K>
__device__ __forceinline__ void direct_masked(float& acc, const Tgt& t, const Src& s, const StepMasks& mk) {
  const float d = sqdist_bcast<K>(t, s);
  float e = __builtin_amdgcn_exp2f(-d);
  asm volatile("s_nop 0\n\tv_cndmask_b32_e64 %0, 0, %0, %1" : "+v"(e) : "s"(mk.m[K]));
  fmac_bcast<K>(acc, s.w, e);
}

#define RBF_STEPS(F, ...) \
  F<0>(__VA_ARGS__); F<1>(__VA_ARGS__); F<2>(__VA_ARGS__); F<3>(__VA_ARGS__); \
  F<4>(__VA_ARGS__); F<5>(__VA_ARGS__); F<6>(__VA_ARGS__); F<7>(__VA_ARGS__); \
  F<8>(__VA_ARGS__); F<9>(__VA_ARGS__); F<10>(__VA_ARGS__); F<11>(__VA_ARGS__); \
  F<12>(__VA_ARGS__); F<13>(__VA_ARGS__); F<14>(__VA_ARGS__); F<15>(__VA_ARGS__)

// ---- expanded form --------------------------------------------------------
// The 16 steps of a chunk as one asm block, software pipelined: the next
// pair's dot product separates each v_exp_f32 from the instruction that
// reads its result (one wait state needed), and a single s_nop 1 at the
// start covers the DPP sources written by the chunk set-up (two wait
// states).  No other hazard applies inside: DPP reads only the per-chunk
// source values, and the lane masks are scalar loads the compiler waits for.
#define RBF_DPP(K) " row_newbcast:" #K " row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
#define RBF_DOT(K)                                  \
  "v_mul_f32_dpp %[va], %[sx], %[tx]" RBF_DPP(K)    \
  "v_fmac_f32_dpp %[va], %[sy], %[ty]" RBF_DPP(K)   \
  "v_fmac_f32_dpp %[va], %[sz], %[tz]" RBF_DPP(K)
#define RBF_ACC(K) "v_fmac_f32_dpp %[acc], %[sw], %[ve]" RBF_DPP(K)
#define RBF_EXP "v_exp_f32 %[ve], %[va]\n\t"
#define RBF_SEL(K) "v_cndmask_b32_e64 %[ve], 0, %[ve], %[m" #K "]\n\t"
#define RBF_IN_STEP(K, KP) RBF_DOT(K) RBF_ACC(KP) RBF_EXP
#define RBF_MASKED_STEP(K, KP) RBF_DOT(K) RBF_SEL(KP) RBF_ACC(KP) RBF_EXP

__device__ __forceinline__ void expanded_inner_chunk(float& acc, const Tgt& t, const Src& s) {
  float va, ve;
  asm volatile(
      "s_nop 1\n\t"
      RBF_DOT(0) RBF_EXP
      RBF_IN_STEP(1, 0) RBF_IN_STEP(2, 1) RBF_IN_STEP(3, 2) RBF_IN_STEP(4, 3)
      RBF_IN_STEP(5, 4) RBF_IN_STEP(6, 5) RBF_IN_STEP(7, 6) RBF_IN_STEP(8, 7)
      RBF_IN_STEP(9, 8) RBF_IN_STEP(10, 9) RBF_IN_STEP(11, 10) RBF_IN_STEP(12, 11)
      RBF_IN_STEP(13, 12) RBF_IN_STEP(14, 13) RBF_IN_STEP(15, 14)
      "s_nop 0\n\t"
      RBF_ACC(15)
      : [acc] "+v"(acc), [va] "=&v"(va), [ve] "=&v"(ve)
      : [sx] "v"(s.x), [sy] "v"(s.y), [sz] "v"(s.z), [sw] "v"(s.w), [tx] "v"(t.x), [ty] "v"(t.y),
        [tz] "v"(t.z));
}

__device__ __forceinline__ void expanded_masked_chunk(float& acc, const Tgt& t, const Src& s,
                                                      const StepMasks& mk) {
  float va, ve;
  asm volatile(
      "s_nop 1\n\t"
      RBF_DOT(0) RBF_EXP
      RBF_MASKED_STEP(1, 0) RBF_MASKED_STEP(2, 1) RBF_MASKED_STEP(3, 2) RBF_MASKED_STEP(4, 3)
      RBF_MASKED_STEP(5, 4) RBF_MASKED_STEP(6, 5) RBF_MASKED_STEP(7, 6) RBF_MASKED_STEP(8, 7)
      RBF_MASKED_STEP(9, 8) RBF_MASKED_STEP(10, 9) RBF_MASKED_STEP(11, 10) RBF_MASKED_STEP(12, 11)
      RBF_MASKED_STEP(13, 12) RBF_MASKED_STEP(14, 13) RBF_MASKED_STEP(15, 14)
      "s_nop 0\n\t"
      RBF_SEL(15) RBF_ACC(15)
      : [acc] "+v"(acc), [va] "=&v"(va), [ve] "=&v"(ve)
      : [sx] "v"(s.x), [sy] "v"(s.y), [sz] "v"(s.z), [sw] "v"(s.w), [tx] "v"(t.x), [ty] "v"(t.y),
        [tz] "v"(t.z), [m0] "s"(mk.m[0]), [m1] "s"(mk.m[1]), [m2] "s"(mk.m[2]), [m3] "s"(mk.m[3]),
        [m4] "s"(mk.m[4]), [m5] "s"(mk.m[5]), [m6] "s"(mk.m[6]), [m7] "s"(mk.m[7]), [m8] "s"(mk.m[8]),
        [m9] "s"(mk.m[9]), [m10] "s"(mk.m[10]), [m11] "s"(mk.m[11]), [m12] "s"(mk.m[12]), [m13] "s"(mk.m[13]),
        [m14] "s"(mk.m[14]), [m15] "s"(mk.m[15]));
}

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

// The pair loop of one group, unrolled by two with fixed double buffers:
// the source gather of chunk c + 1 and the list index of chunk c + 2 are in
// flight while chunk c computes.  The loads are unconditional (the list
// array ends with kListTail padding entries, so the indices read past a
// group's last chunk are valid sources), which keeps every wait for a load
// one chunk of work after its issue.  The inner chunks (an even count) run
// in one straight loop, the masked ones in a second loop on the same
// pipeline, so neither body branches on the chunk kind.
template <bool W32>
__device__ __forceinline__ double weight(const PairArgs& a, uint32_t i) {
  if constexpr (W32)
    return (double)a.w32[i];
  else
    return a.w[i];
}

// A source (scaled coordinates) and its weight.  BUF: by buffer loads at
// 32-bit byte offsets from descriptors of the two arrays (one shift per
// offset instead of 64-bit address arithmetic; the host takes this path
// when the arrays span less than 4 GiB); else by flat 64-bit addresses.
template <bool W32, bool BUF>
struct SourceLoader {
  __amdgpu_buffer_rsrc_t xk, w;
  const PairArgs* a;
  __device__ __forceinline__ explicit SourceLoader(const PairArgs& args) : a(&args) {
    if constexpr (BUF) {
      const int n = (int)(uint32_t)((args.m + 1) * (int64_t)sizeof(double4));
      xk = __builtin_amdgcn_make_buffer_rsrc((void*)args.xk, 0, n, kBufferDword3);
      const void* wp = W32 ? (const void*)args.w32 : (const void*)args.w;
      const int nw = (int)(uint32_t)((args.m + 1) * (int64_t)(W32 ? sizeof(float) : sizeof(double)));
      w = __builtin_amdgcn_make_buffer_rsrc((void*)wp, 0, nw, kBufferDword3);
    }
  }
  __device__ __forceinline__ void operator()(uint32_t i, double4& s, double& wt) const {
    if constexpr (BUF) {
      const uint32_t off = i * (uint32_t)sizeof(double4);
      const auto xy = __builtin_amdgcn_raw_buffer_load_b128(xk, off, 0, 0);
      const auto z = __builtin_amdgcn_raw_buffer_load_b64(xk, off + 16u, 0, 0);
      s.x = __builtin_bit_cast(double, ((uint64_t)xy[1] << 32) | xy[0]);
      s.y = __builtin_bit_cast(double, ((uint64_t)xy[3] << 32) | xy[2]);
      s.z = __builtin_bit_cast(double, ((uint64_t)z[1] << 32) | z[0]);
      s.w = 0.0;
      if constexpr (W32)
        wt = (double)__builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(w, i * 4u, 0, 0));
      else
      {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(w, i * 8u, 0, 0);
        wt = __builtin_bit_cast(double, ((uint64_t)v[1] << 32) | v[0]);
      }
    } else {
      s = a->xk[i];
      wt = weight<W32>(*a, i);
    }
  }
};

template <bool W32, bool BUF, class Inner, class Masked>
__device__ __forceinline__ void chunk_loop(const PairArgs& a, const GroupInfo& gi, int lane, Inner&& inner,
                                           Masked&& masked) {
  const SourceLoader<W32, BUF> load(a);
  const int nch = gi.n_chunks, nin = gi.n_inner;
  const uint32_t i0 = list_entry(a, gi, 0, lane);
  uint32_t i1 = list_entry(a, gi, 1, lane);
  double4 sA;
  double wA;
  load(i0, sA, wA);
  int c = 0;
  for (; c < nin; c += 2) {
    double4 sB;
    double wB;
    load(i1, sB, wB);
    const uint32_t i2 = list_entry(a, gi, c + 2, lane);
    inner(c, sA, wA);
    load(i2, sA, wA);
    i1 = list_entry(a, gi, c + 3, lane);
    inner(c + 1, sB, wB);
  }
  for (; c < nch; c += 2) {
    double4 sB;
    double wB;
    load(i1, sB, wB);
    const uint32_t i2 = list_entry(a, gi, c + 2, lane);
    masked(c, sA, wA);
    if (c + 1 >= nch) break;
    load(i2, sA, wA);
    i1 = list_entry(a, gi, c + 3, lane);
    masked(c + 1, sB, wB);
  }
}

// ---- direct form ----------------------------------------------------------
template <bool MASKED>
__device__ __forceinline__ void direct_chunk(float& acc, const Tgt& t, const double4& sk, double wk, double akx,
                                             double aky, double akz, const uint64_t* mk) {
  Src s;
  s.x = (float)(sk.x - akx);
  s.y = (float)(sk.y - aky);
  s.z = (float)(sk.z - akz);
  s.w = (float)wk;
  if constexpr (MASKED) {
    const StepMasks m = load_masks(mk);
    RBF_STEPS(direct_masked, acc, t, s, m);
  } else {
    RBF_STEPS(direct_inner, acc, t, s);
  }
}

template <bool W32, bool BUF>
__device__ __forceinline__ void direct_group(const PairArgs& a, const GroupInfo& gi, int64_t g, int lane) {
  const int row = lane >> 4, tl = lane & 15;
  const int64_t tid = g * kGroup + tl;
  const double4 tp = a.tpts[tid];
  const Tgt t{(float)((tp.x - gi.ax) * a.sqrt_k), (float)((tp.y - gi.ay) * a.sqrt_k),
              (float)((tp.z - gi.az) * a.sqrt_k)};
  const double akx = gi.ax * a.sqrt_k, aky = gi.ay * a.sqrt_k, akz = gi.az * a.sqrt_k;
  const uint64_t* masks = a.mask + (gi.off >> 2);
  float acc = 0.0f;
  chunk_loop<W32, BUF>(
      a, gi, lane,
      [&](int, const double4& sk, double wk) { direct_chunk<false>(acc, t, sk, wk, akx, aky, akz, nullptr); },
      [&](int c, const double4& sk, double wk) {
        direct_chunk<true>(acc, t, sk, wk, akx, aky, akz, masks + (int64_t)c * 16);
      });
  acc += __shfl_xor(acc, 16);
  acc += __shfl_xor(acc, 32);
  if (row == 0 && tp.w != 0.0) store_result(a, tid, (double)acc);
}

// ---- expanded form --------------------------------------------------------
__device__ __forceinline__ Src expanded_source(const double4& sk, double wk, double akx, double aky, double akz) {
  Src s;
  const double dx = sk.x - akx, dy = sk.y - aky, dz = sk.z - akz;
  s.x = (float)dx;
  s.y = (float)dy;
  s.z = (float)dz;
  // |s|^2 from the float64 differences: it differs from the squared norm of
  // the rounded coordinates by at most u |s|^2, the size of the rounding of
  // the dot product itself
  const double q = fma(dx, dx, fma(dy, dy, dz * dz));
  s.w = (float)wk * __builtin_amdgcn_exp2f(-(float)q);
  return s;
}

template <bool W32, bool BUF>
__device__ __forceinline__ void expanded_group(const PairArgs& a, const GroupInfo& gi, int64_t g, int lane) {
  const int row = lane >> 4, tl = lane & 15;
  const int64_t tid = g * kGroup + tl;
  const double4 tp = a.tpts[tid];
  const float tx = (float)((tp.x - gi.ax) * a.sqrt_k);
  const float ty = (float)((tp.y - gi.ay) * a.sqrt_k);
  const float tz = (float)((tp.z - gi.az) * a.sqrt_k);
  const Tgt t{2.0f * tx, 2.0f * ty, 2.0f * tz};
  const double akx = gi.ax * a.sqrt_k, aky = gi.ay * a.sqrt_k, akz = gi.az * a.sqrt_k;
  const uint64_t* masks = a.mask + (gi.off >> 2);
  float acc = 0.0f;
  chunk_loop<W32, BUF>(
      a, gi, lane,
      [&](int, const double4& sk, double wk) {
        expanded_inner_chunk(acc, t, expanded_source(sk, wk, akx, aky, akz));
      },
      [&](int c, const double4& sk, double wk) {
        const Src s = expanded_source(sk, wk, akx, aky, akz);
        expanded_masked_chunk(acc, t, s, load_masks(masks + (int64_t)c * 16));
      });
  acc += __shfl_xor(acc, 16);
  acc += __shfl_xor(acc, 32);
  // |t|^2 of the rounded coordinates the steps used
  const double tq = ((double)tx * tx + (double)ty * ty) + (double)tz * tz;
  if (row == 0 && tp.w != 0.0) store_result(a, tid, (double)acc * exp2(-tq));
}

// A group record read field by field through the constant address space
// (nothing writes it during the launch): scalar loads, so every field is
// uniform for the compiler too.
__device__ __forceinline__ GroupInfo load_group(const GroupInfo* gp) {
  typedef const __attribute__((address_space(4))) GroupInfo* ConstGroup;
  const ConstGroup p = (ConstGroup)gp;
  GroupInfo gi;
  gi.off = p->off;
  gi.n_chunks = p->n_chunks;
  gi.n_inner = p->n_inner;
  gi.ax = p->ax;
  gi.ay = p->ay;
  gi.az = p->az;
  gi.radius = p->radius;
  return gi;
}

// Waves (groups) per workgroup.  One wave per workgroup lets the dispatcher
// balance the uneven group costs wave by wave (occupancy 87 % against 82 %)
// but measured 3 % slower: the kernel is bound by VALU issue, not by the
// tail.
constexpr int kPairWaves = 4;
static_assert(kPairWaves == kGroupsPerLaunchBlock, "the group launch order assumes four groups per workgroup");

// The group a wave runs: its launch slot (each XCD a contiguous range of
// slots), through the set's launch order when it has one.  Uniform, so the
// order is read by a scalar load.
__device__ __forceinline__ int64_t slot_group(const PairArgs& a, int64_t slot) {
  if (!a.order) return slot;
  typedef const __attribute__((address_space(4))) int32_t* ConstI32;
  return ((ConstI32)a.order)[slot];
}

template <bool W32, bool BUF>
__global__ __launch_bounds__(kPairWaves * kWave) void k_pairsum_f32(PairArgs a) {
  // the wave index is uniform across the wave: keep it (and all group data) scalar
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t slot = xcd_remap(blockIdx.x, gridDim.x) * kPairWaves + wave;
  if (slot >= a.G) return;
  if (a.skip && *a.skip) return;
  const int64_t g = slot_group(a, slot);
  const GroupInfo gi = load_group(a.groups + g);
  if (expanded_form(a.dense != 0, gi.radius * a.sqrt_k, a.sqrt_T))
    expanded_group<W32, BUF>(a, gi, g, lane);
  else
    direct_group<W32, BUF>(a, gi, g, lane);
}

// ---- float64 ---------------------------------------------------------------
// 2^y for |y| <= 1000: y = n + f with n the nearest integer (exact) and
// |f| <= 1/2; 2^f = exp(f ln 2) by its Taylor series to degree 13 (the
// first omitted term is below 2^-57 of the value), coefficients
// (ln 2)^k / k! rounded to float64; then 2^n by ldexp.  Within 2 ulp.
__device__ __forceinline__ double exp2_f64(double y) {
  constexpr double C[14] = {
      0x1.0000000000000p+0,  0x1.62e42fefa39efp-1, 0x1.ebfbdff82c58fp-3, 0x1.c6b08d704a0c0p-5,
      0x1.3b2ab6fba4e77p-7,  0x1.5d87fe78a6731p-10, 0x1.430912f86c787p-13, 0x1.ffcbfc588b0c7p-17,
      0x1.62c0223a5c824p-20, 0x1.b5253d395e7c4p-24, 0x1.e4cf5158b8ecap-28, 0x1.e8cac7351bb25p-32,
      0x1.c3bd650fc2986p-36, 0x1.816193166d0f9p-40};
  const double n = rint(y);
  const double f = y - n;
  double p = C[13];
#pragma unroll
  for (int k = 12; k >= 0; --k) p = fma(p, f, C[k]);
  return ldexp(p, (int)n);
}

// e where the step's lane mask has this lane's bit, else 0 (the mask in
// scalar registers, as the float32 kernel applies it).
__device__ __forceinline__ double mask_lane(double e, uint64_t m) {
  uint32_t lo = (uint32_t)__builtin_bit_cast(uint64_t, e), hi = (uint32_t)(__builtin_bit_cast(uint64_t, e) >> 32);
  asm volatile("v_cndmask_b32_e64 %0, 0, %0, %2\n\tv_cndmask_b32_e64 %1, 0, %1, %2"
               : "+v"(lo), "+v"(hi) : "s"(m));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Expanded form in float64, with the list builder's lane masks: per chunk
// every lane stages its source relative to the anchor (scaled) with the
// weight folded with 2^{-|s|^2}; each pair then costs the dot product 2 t.s,
// exp2_f64 and one FMA; the target factor 2^{-|t|^2} multiplies the sum.
// (Within the expanded form's range |s|^2 <= 100 and 2 t.s <= 100; the
// padding source, far away with weight 0 and always masked, is staged as 0.)
__device__ __forceinline__ void expanded_group_f64(const PairArgs& a, const GroupInfo& gi, int64_t g, int wave,
                                                   int lane, double4 (*sh)[kWave]) {
  const int row = lane >> 4, tl = lane & 15;
  const int64_t tid = g * kGroup + tl;
  const double4 tp = a.tpts[tid];
  const double tx = (tp.x - gi.ax) * a.sqrt_k, ty = (tp.y - gi.ay) * a.sqrt_k, tz = (tp.z - gi.az) * a.sqrt_k;
  const double t2x = 2.0 * tx, t2y = 2.0 * ty, t2z = 2.0 * tz;
  const double akx = gi.ax * a.sqrt_k, aky = gi.ay * a.sqrt_k, akz = gi.az * a.sqrt_k;
  const uint64_t* masks = a.mask + (gi.off >> 2);
  const int nch = gi.n_chunks, nin = gi.n_inner;
  double acc = 0.0;
  for (int c = 0; c < nch; ++c) {
    const uint32_t idx = list_entry(a, gi, c, lane);
    const double4 sk = a.xk[idx];
    const double sx = sk.x - akx, sy = sk.y - aky, sz = sk.z - akz;
    const double q = fma(sx, sx, fma(sy, sy, sz * sz));
    double4 st = make_double4(0.0, 0.0, 0.0, 0.0);
    if (q <= 1000.0) st = make_double4(sx, sy, sz, a.w[idx] * exp2_f64(-q));
    sh[wave][lane] = st;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const double4* src = &sh[wave][row * kGroup];
    if (c < nin) {
#pragma unroll 4
      for (int k = 0; k < kGroup; ++k) {
        const double4 s = src[k];
        acc = fma(s.w, exp2_f64(fma(t2x, s.x, fma(t2y, s.y, t2z * s.z))), acc);
      }
    } else {
      const StepMasks mk = load_masks(masks + (int64_t)c * 16);
#pragma unroll
      for (int k = 0; k < kGroup; ++k) {
        const double4 s = src[k];
        const double e = exp2_f64(fma(t2x, s.x, fma(t2y, s.y, t2z * s.z)));
        acc = fma(s.w, mask_lane(e, mk.m[k]), acc);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  acc += __shfl_xor(acc, 16);
  acc += __shfl_xor(acc, 32);
  const double tq = fma(tx, tx, fma(ty, ty, tz * tz));
  if (row == 0 && tp.w != 0.0) store_result(a, tid, acc * exp2_f64(-tq));
}

// Direct form in float64 (dense lists and groups too wide for the expanded
// form): r^2 and the cutoff test exactly as the float64 definition, exp from
// the device library.
__device__ __forceinline__ void direct_group_f64(const PairArgs& a, const GroupInfo& gi, int64_t g, int wave,
                                                 int lane, double4 (*sh)[kWave]) {
  const int row = lane >> 4, tl = lane & 15;
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

// Six waves per SIMD (76 VGPRs, no spills): the LDS broadcasts of the
// sources wait less with more waves in flight (102 VGPRs and four waves
// took 6 % longer; seven or eight waves spill).
__global__ __launch_bounds__(kBlock, 6) void k_pairsum_f64(PairArgs a) {
  __shared__ double4 sh[kBlock / kWave][kWave];
  // the wave index is uniform across the wave: keep it (and all group data) scalar
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t slot = xcd_remap(blockIdx.x, gridDim.x) * kGroupsPerLaunchBlock + wave;
  if (slot >= a.G) return;
  if (a.skip && *a.skip) return;
  const int64_t g = slot_group(a, slot);
  const GroupInfo gi = load_group(a.groups + g);
  if (expanded_form(a.dense != 0, gi.radius * a.sqrt_k, a.sqrt_T))
    expanded_group_f64(a, gi, g, wave, lane, sh);
  else
    direct_group_f64(a, gi, g, wave, lane, sh);
}

// Register-resident rate of the float32 pair steps (rbf_measure_rates): the
// kernel's own 16-step chunk bodies, inner and masked, on operands held in
// registers (no list, gather or set-up), one accumulator per lane as in the
// kernel.  Lane masks alternate bits.
template <bool MASKED>
__global__ __launch_bounds__(256) void k_step_rate(float* __restrict__ out, int iters) {
  const int lane = threadIdx.x & 63;
  const Tgt t{0.01f * (float)(lane & 15), 0.02f, -0.01f};
  Src s{0.1f, 0.05f * (float)((lane >> 4) + 1), 0.02f, 0.5f};
  StepMasks mk;
#pragma unroll
  for (int k = 0; k < kGroup; ++k) mk.m[k] = 0x5555555555555555ull << (k & 1);
  float acc = 0.0f;
  for (int it = 0; it < iters; ++it) {
    // opaque to the compiler: the chunk body is not hoisted out of the loop
    asm volatile("" : "+v"(s.x), "+v"(s.y), "+v"(s.z), "+v"(s.w));
    if constexpr (MASKED)
      expanded_masked_chunk(acc, t, s, mk);
    else
      expanded_inner_chunk(acc, t, s);
  }
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

PairArgs make_args(const Ctx& c, const TargetSet& ts, const double* w, bool out_f32, void* out,
                   const int* skip) {
  PairArgs a;
  a.tpts = ts.pts;
  a.groups = ts.groups;
  a.list = ts.list;
  a.mask = reinterpret_cast<const uint64_t*>(ts.mask);
  a.order = ts.order;
  a.G = ts.n_groups;
  a.xk = c.xk;
  a.xs = c.xs;
  a.w = w;
  a.w32 = nullptr;
  a.m = c.m;
  a.sqrt_k = c.sqrt_k;
  a.inv_two_s2 = c.inv_two_s2;
  a.rc2 = c.rc2;
  a.dense = ts.dense ? 1 : 0;
  a.out_f32 = out_f32 ? 1 : 0;
  a.out = out;
  a.out_index = ts.index;
  a.skip = skip;
  a.Tk = std::isfinite(c.rc2) ? c.rc2 * c.sqrt_k * c.sqrt_k : INFINITY;
  a.sqrt_T = scaled_cutoff(c);
  return a;
}

}  // namespace

void pairsum_f32(const Ctx& c, const TargetSet& ts, const double* w, bool out_f32, void* out, hipStream_t s,
                 const int* skip, const float* w32) {
  if (ts.n_groups == 0) return;
  PairArgs a = make_args(c, ts, w, out_f32, out, skip);
  a.w32 = w32;
  const int64_t nb = ceil_div(ts.n_groups, kPairWaves);
  ProfScope prof(RBF_FP32, ts.kind, ts.useful, ts.list_entries * kGroup, s);
  // buffer loads when the sources (32 B each) span less than 4 GiB
  const bool buf = (c.m + 1) * (int64_t)sizeof(double4) < ((int64_t)1 << 32);
  auto kernel = w32 ? (buf ? k_pairsum_f32<true, true> : k_pairsum_f32<true, false>)
                    : (buf ? k_pairsum_f32<false, true> : k_pairsum_f32<false, false>);
  // a timed launch carries its events in the dispatch; an untimed one is a
  // plain launch (which a stream capture can record)
  if (prof.start())
    hipExtLaunchKernelGGL(kernel, dim3((unsigned)nb), dim3(kPairWaves * kWave), 0, s, prof.start(), prof.stop(), 0,
                          a);
  else
    hipLaunchKernelGGL(kernel, dim3((unsigned)nb), dim3(kPairWaves * kWave), 0, s, a);
  RBF_HIP(hipGetLastError());
  prof.done();
}

void launch_step_rate(bool masked, float* out, int blocks, int iters, hipStream_t s) {
  if (masked)
    hipLaunchKernelGGL(k_step_rate<true>, dim3(blocks), dim3(256), 0, s, out, iters);
  else
    hipLaunchKernelGGL(k_step_rate<false>, dim3(blocks), dim3(256), 0, s, out, iters);
  RBF_HIP(hipGetLastError());
}

void pairsum_f64(const Ctx& c, const TargetSet& ts, const double* w, bool out_f32, void* out, hipStream_t s,
                 const int* skip) {
  if (ts.n_groups == 0) return;
  PairArgs a = make_args(c, ts, w, out_f32, out, skip);
  const int64_t nb = ceil_div(ts.n_groups, kBlock / kWave);
  ProfScope prof(RBF_FP64, ts.kind, ts.useful, ts.list_entries * kGroup, s);
  if (prof.start())
    hipExtLaunchKernelGGL(k_pairsum_f64, dim3((unsigned)nb), dim3(kBlock), 0, s, prof.start(), prof.stop(), 0, a);
  else
    hipLaunchKernelGGL(k_pairsum_f64, dim3((unsigned)nb), dim3(kBlock), 0, s, a);
  RBF_HIP(hipGetLastError());
  prof.done();
}

}  // namespace rbf
