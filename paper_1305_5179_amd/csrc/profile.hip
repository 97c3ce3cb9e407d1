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

}  // namespace rbf
