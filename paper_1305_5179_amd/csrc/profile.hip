// Launch timing of the pair kernels (rbf_profile_begin / rbf_profile_end):
// while profiling is on, a timed launch carries a start and a stop event in
// its own dispatch (hipExtLaunchKernel: the timestamps of the kernel
// itself); rbf_profile_end waits for them and sums the elapsed times, the
// launches timed and their pair counts per kind (operator / evaluation) and
// precision.  The events come from a pool kept for the life of the process.
#include "common.h"

namespace rbf {

namespace {
struct ProfRec {
  hipEvent_t a, b;
  int kind, prec;
  int64_t useful, examined;
  bool ended;   // the end event was recorded
};
// The float32 operator runs thirty times per refinement step: one launch in
// kSample carries the events (every launch costs the same work; events on
// all of them slowed the step by about 4 %).
constexpr int kSample = 3;

struct Profiler {
  bool on = false;
  int64_t seen = 0;   // float32 operator launches since rbf_profile_begin
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;   // created events not in use
};
Profiler& profiler() {
  static Profiler p;
  return p;
}
hipEvent_t take_event() {
  Profiler& p = profiler();
  if (!p.pool.empty()) {
    hipEvent_t e = p.pool.back();
    p.pool.pop_back();
    return e;
  }
  hipEvent_t e;
  RBF_HIP(hipEventCreate(&e));
  return e;
}
void give_back(const ProfRec& r) {
  profiler().pool.push_back(r.a);
  profiler().pool.push_back(r.b);
}
}  // namespace

ProfScope::ProfScope(int prec, int kind, int64_t useful, int64_t examined, hipStream_t st)
    : on(profiler().on), s(st) {
  if (!on) return;
  if (kind == 0 && prec == RBF_FP32 && (profiler().seen++ % kSample) != 0) {
    on = false;   // not sampled: a plain launch
    return;
  }
  ProfRec r{};
  r.prec = prec;
  r.kind = kind;
  r.useful = useful;
  r.examined = examined;
  r.a = take_event();
  r.b = take_event();
  profiler().recs.push_back(r);
  rec = (int)profiler().recs.size() - 1;
}

hipEvent_t ProfScope::start() const { return on && rec >= 0 ? profiler().recs[rec].a : nullptr; }
hipEvent_t ProfScope::stop() const { return on && rec >= 0 ? profiler().recs[rec].b : nullptr; }

void ProfScope::done() {
  if (!on || rec < 0) return;
  profiler().recs[rec].ended = true;
}

void ProfScope::set_pairs(int64_t useful, int64_t examined) {
  if (!on || rec < 0 || rec >= (int)profiler().recs.size()) return;
  profiler().recs[rec].useful = useful;
  profiler().recs[rec].examined = examined;
}

bool profiling() { return profiler().on; }

int profile_begin() {
  Profiler& p = profiler();
  for (auto& r : p.recs) {
    if (r.ended) (void)hipEventSynchronize(r.b);
    give_back(r);
  }
  p.recs.clear();
  p.seen = 0;
  p.on = true;
  return RBF_OK;
}

int profile_end(rbf_profile* out) {
  Profiler& p = profiler();
  p.on = false;
  rbf_profile r{};
  for (auto& q : p.recs) {
    if (!q.ended) {   // a launch that failed: its events were never used
      give_back(q);
      continue;
    }
    RBF_HIP(hipEventSynchronize(q.b));
    float ms = 0.f;
    RBF_HIP(hipEventElapsedTime(&ms, q.a, q.b));
    r.launches[q.kind][q.prec] += 1;
    r.kernel_ms[q.kind][q.prec] += ms;
    r.useful_pairs[q.kind][q.prec] += q.useful;
    r.examined_pairs[q.kind][q.prec] += q.examined;
    give_back(q);
  }
  p.recs.clear();
  if (out) *out = r;
  return RBF_OK;
}

// ---- issue rates of the vector ALU ----------------------------------------
// Register-resident loops, eight independent chains per lane, every wave slot
// of the device filled: float32 FMAs (VOP2 v_fmamk_f32: this library is
// built without packed float32 arithmetic), the same FMA in its DPP form
// (v_fmac_f32_dpp row_newbcast, as the pair kernel issues it), v_exp_f32,
// and chains of one v_exp_f32 followed by three or seven FMAs.  The chains
// stay finite and normal: x <- 2^-x has its fixed point near 0.64,
// x <- 0.999 x + 0.001 its fixed point at 1, x <- x + 0.001 * 0.999 grows
// by 0.001 per step.  Then the float32 pair kernel's own chunk bodies.
namespace {
constexpr int kRateChains = 8;
constexpr int kRateIters = 16384;

template <int MODE>   // 0: FMA, 1: exp, 2: exp + 3 FMA, 3: exp + 7 FMA, 4: DPP FMA
__global__ __launch_bounds__(256) void k_rates(float* __restrict__ out, float seed) {
  float x[kRateChains];
#pragma unroll
  for (int c = 0; c < kRateChains; ++c) x[c] = seed + 0.01f * c + 1e-6f * (float)threadIdx.x;
  float ca = 0.999f, cb = 0.001f;
  asm volatile("s_nop 1" : "+v"(ca), "+v"(cb));   // (DPP reads ca: two wait states after its write)
  for (int it = 0; it < kRateIters; ++it) {
#pragma unroll
    for (int c = 0; c < kRateChains; ++c) {
      if constexpr (MODE == 0) {
        x[c] = __builtin_fmaf(x[c], 0.999f, 0.001f);
      } else if constexpr (MODE == 4) {
        asm volatile("v_fmac_f32_dpp %0, %1, %2 row_newbcast:3 row_mask:0xf bank_mask:0xf bound_ctrl:1"
                     : "+v"(x[c]) : "v"(ca), "v"(cb));
      } else {
        x[c] = __builtin_amdgcn_exp2f(-x[c]);
        constexpr int nf = MODE == 1 ? 0 : MODE == 2 ? 3 : 7;
#pragma unroll
        for (int f = 0; f < nf; ++f) x[c] = __builtin_fmaf(x[c], 0.999f, 0.001f);
      }
    }
  }
  float a = 0.0f;
#pragma unroll
  for (int c = 0; c < kRateChains; ++c) a += x[c];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = a;
}
}  // namespace

void measure_rates(rbf_rates* r, hipStream_t s) {
  int dev = 0, cus = 0;
  RBF_HIP(hipGetDevice(&dev));
  RBF_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  // eight waves on each of a CU's four SIMDs
  const int blocks = cus * 8, threads = 256;
  float* out = dalloc<float>((int64_t)blocks * threads);
  hipEvent_t a, b;
  RBF_HIP(hipEventCreate(&a));
  RBF_HIP(hipEventCreate(&b));
  const double lanes_iters = (double)blocks * threads * kRateIters * kRateChains;
  auto timed = [&](auto&& launch) {
    launch();   // warm-up
    RBF_HIP(hipEventRecord(a, s));
    launch();
    RBF_HIP(hipEventRecord(b, s));
    RBF_HIP(hipEventSynchronize(b));
    float ms = 0.f;
    RBF_HIP(hipEventElapsedTime(&ms, a, b));
    return 1e-3 * (double)ms;
  };
  auto rate = [&](auto kernel) {
    return lanes_iters / timed([&] {
             hipLaunchKernelGGL(kernel, dim3(blocks), dim3(threads), 0, s, out, 0.5f);
             RBF_HIP(hipGetLastError());
           });
  };
  r->compute_units = cus;
  r->fma_per_s = rate(k_rates<0>);
  r->exp_per_s = rate(k_rates<1>);
  r->exp_3fma_per_s = rate(k_rates<2>);
  r->exp_7fma_per_s = rate(k_rates<3>);
  r->dpp_fma_per_s = rate(k_rates<4>);
  constexpr int kStepIters = 2048;
  const double steps = (double)blocks * threads * kStepIters * kGroup;
  r->inner_pair_steps_per_s = steps / timed([&] { launch_step_rate(false, out, blocks, kStepIters, s); });
  r->masked_pair_steps_per_s = steps / timed([&] { launch_step_rate(true, out, blocks, kStepIters, s); });
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  dfree(out);
}

}  // namespace rbf
