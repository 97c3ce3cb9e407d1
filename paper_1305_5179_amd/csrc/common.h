// Internal declarations shared by the librbf sources (gfx950, wave64).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "rbf.h"

namespace rbf {

// ---------------------------------------------------------------------------
// Work decomposition of the pair sums.
//   A wave (64 lanes) owns one group of kGroup = 16 targets.  Its four DPP
//   rows (lanes 16r .. 16r+15) all hold the same 16 targets and walk four
//   interleaved streams of the group's source list; a chunk is 64 list
//   entries, one per lane, and inside a chunk every row broadcasts its 16
//   sources to its lanes one by one (DPP row_newbcast), so each lane
//   evaluates 16 pairs per chunk with its own target.
// ---------------------------------------------------------------------------
constexpr int kGroup = 16;
constexpr int kWave = 64;
constexpr int kChunk = 64;
constexpr int kBlock = 256;          // threads per block of the pair kernels (4 independent waves)
constexpr int kGroupsPerLaunchBlock = kBlock / kWave;   // groups (one per wave) per workgroup of the pair kernels
// Padding entries after the last group's list: the pair kernels read the
// list indices up to three chunks ahead without bounds tests.
constexpr int kListTail = 3 * kChunk;
// The Krylov basis is allocated with its column count rounded up to this
// (extra columns zero): the dot-product kernels read columns in blocks of it.
constexpr int kKrylovColPad = 8;

// Curve keys (Hilbert order): 10 bits per axis on the fine lattice.
constexpr int kCurveBits = 10;
constexpr int kFineMax = 1 << kCurveBits;

// Far-away coordinate of the padding source/target (index M of the sorted
// arrays): every pair with it underflows to exactly 0 and its weight is 0.
constexpr double kFar = 1.0e6;

// Per-group metadata of a target set.
// The list of a group is [inner | outer], padded to whole chunks: inner
// sources are inside the cutoff for every target of the group, outer ones
// for some (float64 decisions).  Every chunk from n_inner on carries, per
// entry, the 16-bit mask of the targets it is inside for (see mask_slot).
struct GroupInfo {
  int64_t off;          // first list entry of the group (a multiple of 64)
  int32_t n_chunks;     // list length / 64
  int32_t n_inner;      // chunks [0, n_inner) hold inner sources only (an even count)
  double ax, ay, az;    // anchor (unscaled float64); float32 coordinates are taken relative to it
  double radius;        // max distance of a valid target from the anchor
};

// Number of leading chunks of a group's list that the pair kernels treat as
// inner (no test): the whole chunks of inner sources, rounded down to an even
// count (the kernels' chunk loop is unrolled by two; a chunk beyond it
// carries masks like the outer chunks).
__host__ __device__ inline int64_t inner_chunks(int64_t n_inner_sources) {
  return (n_inner_sources / kChunk) & ~int64_t(1);
}

// Position in the mask array of list entry e of a group starting at `off`.
// Entry e = 64 c + 16 r + k is the source that row r of a wave broadcasts at
// step k of chunk c; its mask is stored at off + 64 c + 4 k + r, so that the
// four masks of step k form one 64-bit lane mask (bit 16 r + t = target t).
__host__ __device__ inline int64_t mask_slot(int64_t off, int64_t e) {
  return off + (e & ~int64_t(63)) + ((e & 15) << 2) + ((e >> 4) & 3);
}

// Form of a group's float32 pair sums.  The expanded form writes the scaled
// squared distance as |t|^2 + |s|^2 - 2 t.s (anchor-relative coordinates); it
// applies when every listed source is within rk + sqrt(T) of the anchor with
// (rk + sqrt(T))^2 <= 100 and 2 rk (rk + sqrt(T)) <= 100 (scaled units),
// which keeps every exponent in range and the rounding of |s|^2 and 2 t.s at
// a few float32 units of the term.  Other groups, and dense lists, take the
// direct differences.
__host__ __device__ inline bool expanded_form(bool dense, double rk, double sqrt_T) {
  const double smax = rk + sqrt_T;
  return !dense && smax * smax <= 100.0 && 2.0 * rk * smax <= 100.0;
}

// The overlapping Schwarz preconditioner (schwarz.hip).  Subdomain i has
// members mem[mem_off[i] .. mem_off[i+1]) (sorted positions), its ncore[i]
// core centres first; its local inverse is W[woff[i] ..], float32, or with
// `half` W16[woff[i] ..], float16, n x n in column quads (schwarz.hip:
// columns 4q .. 4q+3 of a row together; float16 rows padded to an even
// count).
constexpr int kSchwarzMaxBlock = 1024;   // largest subdomain (core + overlap centres)
constexpr int kSchwarzDefaultBlock = 192;
struct SchwarzData {
  int64_t nsub = 0, nmem = 0, w_total = 0;
  int restricted = 0, max_block = 0, pct = 0, retries = 0;
  bool half = false;
  double shift = 0, max_shift = 0, factor_ms = 0;
  // the apply's persistent launch: tasks (subdomain, first row) of
  // apply_threads rows each (twice as many with `half`), largest first, taken
  // cyclically by apply_blocks workgroups
  int apply_threads = 256, apply_blocks = 0;
  int64_t ntask = 0;
  int2* tasks = nullptr;
  int64_t* mem_off = nullptr;
  int32_t* ncore = nullptr;
  uint32_t* mem = nullptr;
  int64_t* woff = nullptr;
  float* W = nullptr;
  _Float16* W16 = nullptr;
  double* Y = nullptr;          // additive form: the local solutions, by member slot
  int64_t* occ_off = nullptr;   // additive form: the member slots of every centre
  int64_t* occ_slot = nullptr;
  double* z = nullptr;          // work vectors of the preconditioned solve (length mpad)
  double* t = nullptr;
  float* z32 = nullptr;         // the preconditioned vector for the float32 operator (length mpad)
  std::vector<int64_t> h_mem_off;
  std::vector<int32_t> h_ncore;
  std::vector<uint32_t> h_mem_paper;   // members as paper indices
};

// The network of the learned narrow-band cull (mlp.hip): float32 parameters
// (layout of RBF_NET_PARAMS in rbf.h), Adam moments, bf16 copies of the
// three wide layers and of their transposes, and the input normalisation.
struct NetData {
  float* P = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  __bf16* Wb = nullptr;
  __bf16* WbT = nullptr;
  double centre[3] = {0, 0, 0};
  double scale = 1.0, tau = 1.0;
  int64_t step = 0;
};
struct NetCullStats {
  int64_t support_bricks = 0, kept_bricks = 0, useful_pairs = 0, examined_pairs = 0;
};

// A set of targets grouped by 16 (centres, grid nodes or evaluation points)
// together with the source list of every group.
struct TargetSet {
  int64_t n_targets = 0;    // valid targets
  int64_t n_groups = 0;
  double4* pts = nullptr;   // n_groups*16 targets, unscaled; .w = 1 valid, 0 padding
  int64_t* index = nullptr; // output position of every target slot
  GroupInfo* groups = nullptr;
  uint32_t* list = nullptr; // sorted-source indices (M = padding source)
  uint16_t* mask = nullptr; // per-entry target masks of the non-inner chunks (mask_slot)
  int64_t list_entries = 0;
  int64_t useful = 0;       // pairs with r^2 <= cutoff^2 (float64 decision)
  int64_t inner_entries = 0; // list entries in the groups' leading inner chunks (no cutoff test)
  bool dense = false;       // no cutoff: every group's list is 0..M-1 (implicit)
  bool temp = false;        // arrays are stream-ordered temporaries (per-call sets)
  int kind = 0;             // 0: the centres (operator), 1: evaluation targets
  bool lattice = false;     // groups are bricks of grid nodes (4 x 2 x 2, node order of k_brick_targets)
  int32_t* order = nullptr; // launch order of the groups for the pair kernels (operator sets), or null
                            // (identity): group order[slot] runs in launch slot `slot`
  std::vector<void*> owned; // device allocations to free with the set
};

// Neighbour lattice.  Fine cells (side f) order the centres along a Hilbert
// curve; a coarse cell is an aligned block of 2^shift fine cells per axis
// and therefore a contiguous run of the sorted centres.
struct Lattice {
  double origin[3];
  double fine;              // side of a fine cell
  int shift;                // coarse = fine << shift
  double coarse;            // side of a coarse cell
  int fdims[3];             // fine cells per axis (<= 1024)
  int cdims[3];             // coarse cells per axis
};

struct Ctx {
  int device = 0;
  int64_t n = 0;            // points
  int64_t m = 0;            // centres = 3n
  int64_t mpad = 0;         // padded vector length (>= m + 1, multiple of 256)
  double eps = 0, sigma = 0, cutoff = 0;
  double rc2 = 0;           // cutoff^2 (float64), +inf without cutoff
  double sqrt_k = 0;        // coordinates scaled by sqrt(log2(e) / (2 sigma^2)): phi = exp2(-|x'|^2)
  double inv_two_s2 = 0;    // 1 / (2 sigma^2)
  Lattice lat{};
  // Sorted centres (Hilbert order); index m is the far padding source.
  uint32_t* perm = nullptr;     // sorted position -> paper index
  uint32_t* keys = nullptr;     // curve keys of the sorted centres
  double4* xs = nullptr;        // unscaled coordinates, m+1
  double4* xk = nullptr;        // scaled coordinates, m+1
  double* xpaper = nullptr;     // paper-order centres, m x 3 (for rbf_centres)
  // Coarse cells: start/count in the sorted order; dense map coarse cell -> id.
  int32_t* cell_start = nullptr;
  int32_t* cell_count = nullptr;
  int32_t* cell_map = nullptr;  // product of cdims entries, -1 = empty
  int32_t* cell_xyz = nullptr;  // coarse coordinates of every cell, x | y << 10 | z << 20
  int64_t n_cells = 0;
  int64_t* cell_sat = nullptr;  // summed source counts of the coarse cells (null when too many cells)
  TargetSet centres;            // the centres as targets of the operator
  SchwarzData* schwarz = nullptr;
  NetData* net = nullptr;
  // Work vectors (sorted order, length mpad, entry m kept 0).
  double* vin = nullptr;
  double* vout = nullptr;
  // Solver storage, allocated on first use.
  int krylov_m = 0;
  int krylov_f32 = -1;          // element type the basis was last used with (1 float32, 0 float64;
                                // -1: all zero since its allocation, either type)
  double* V = nullptr;          // (m+1) basis vectors of length mpad (float64, or float32 in the same space)
  double* w = nullptr;
  double* r = nullptr;
  double* csol = nullptr;
  double* bsort = nullptr;
  double* partial = nullptr;    // block partial sums
  int64_t partial_cap = 0;
  void* state = nullptr;        // device GMRES state
  // The Arnoldi steps of one full GMRES cycle, captured (on a stream of the
  // context's own) into a graph, with the buffers and options it was
  // captured for.
  hipGraphExec_t cycle_exec = nullptr;
  hipStream_t capture_stream = nullptr;
  std::vector<intptr_t> cycle_key;
  std::vector<double> history;
  std::vector<double> history_ms;
  std::string err;
};

// ---------------------------------------------------------------------------
// Error plumbing.
// ---------------------------------------------------------------------------
struct Error {
  int code;
  std::string msg;
};

void set_thread_error(const std::string& msg);
const char* thread_error();

#define RBF_HIP(call)                                                             \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess)                                                         \
      throw ::rbf::Error{e_ == hipErrorOutOfMemory ? RBF_ENOMEM : RBF_EDEVICE,    \
                         std::string(#call) + ": " + hipGetErrorString(e_)};      \
  } while (0)

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
__host__ __device__ inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }
__host__ __device__ inline int64_t round_down(int64_t a, int64_t b) { return (a / b) * b; }


// Temporaries: stream-ordered allocations on the stream of the current API
// call (set by TempStream), served by the library's caching allocator
// (alloc.hip) without a device-wide synchronisation.
hipStream_t& temp_stream();
struct TempStream {
  hipStream_t prev;
  explicit TempStream(hipStream_t s) : prev(temp_stream()) { temp_stream() = s; }
  ~TempStream() { temp_stream() = prev; }
};
// While one of these is alive on a thread, freed blocks may be reused by any
// stream: only for code that has synchronised the device first.
struct SyncedRelease {
  bool prev;
  SyncedRelease();
  ~SyncedRelease();
};
void* temp_alloc_bytes(size_t bytes);
void temp_free(void* p);
template <class T>
T* talloc(int64_t count) {
  if (count <= 0) count = 1;
  return static_cast<T*>(temp_alloc_bytes(sizeof(T) * (size_t)count));
}
// Context arrays come from the same allocator (allocated on the stream of
// the call that creates them; rbf_setup returns only after that stream is
// idle, and rbf_destroy waits for the device before releasing them).
template <class T>
T* dalloc(int64_t count) {
  return talloc<T>(count);
}
inline void dfree(void* p) { temp_free(p); }
// Arrays of a target set: persistent or stream-ordered as the set asks.
template <class T>
T* set_alloc(const TargetSet& ts, int64_t count) {
  return ts.temp ? talloc<T>(count) : dalloc<T>(count);
}

// sqrt(T), the scaled cutoff r_c sqrt(k), as the pair kernels give it to
// expanded_form.
inline double scaled_cutoff(const Ctx& c) { return std::isfinite(c.rc2) ? std::sqrt(c.rc2) * c.sqrt_k : INFINITY; }

// ---------------------------------------------------------------------------
// Launchers (defined in the .hip files).
// ---------------------------------------------------------------------------
// setup.hip
void check_inputs(const double* points, const double* normals, int64_t n, int* flags, hipStream_t s);
void build_centres(const double* points, const double* normals, int64_t n, double eps, double* xpaper,
                   hipStream_t s);
void bounding_box(const double* xpaper, int64_t m, double* box6, double* scratch, hipStream_t s);
void sort_points(const double* pts3, int64_t m, const Lattice& lat, uint32_t* perm, uint32_t* keys_out,
                 hipStream_t s);
void gather_sorted(const double* pts3, const uint32_t* perm, int64_t m, double sqrt_k, double4* xs,
                   double4* xk, hipStream_t s);
// The occupied cells' arrays (sized by the bound m); their count arrives
// in ncell_parts[0] + ncell_parts[1] (pinned host memory) once the stream
// has been synchronised.
void build_cells(const uint32_t* keys, const double4* xs, int64_t m, const Lattice& lat, int32_t** cell_start,
                 int32_t** cell_count, int32_t** cell_map, int32_t** cell_xyz, int64_t* ncell_parts, hipStream_t s);
// Pinned host slots of the calling thread for small read-backs.  A copy into
// pinned memory is queued without a wait of its own (a copy into pageable
// memory waits for the stream), so several values cost one wait; they are
// there once the stream has been synchronised.  Slots come from a
// per-thread stack of kPinnedSlots and go back when the holder ends
// (holders nest, last in first out).
constexpr int kPinnedSlots = 64;
struct PinnedSlots {
  explicit PinnedSlots(int count);
  ~PinnedSlots();
  PinnedSlots(const PinnedSlots&) = delete;
  PinnedSlots& operator=(const PinnedSlots&) = delete;
  int64_t* p;
  int n;
};
// The source lists of a target set.  inner_slot (pinned, or null): where
// the count of inner-chunk entries is queued for the caller to read after
// its own synchronisation; null: read here, with a wait.
void build_lists(const Ctx& c, TargetSet& ts, hipStream_t s, int64_t* inner_slot = nullptr);
constexpr int64_t kCellSatMax = int64_t(1) << 26;   // entries of the summed cell counts (512 MB)
int64_t* build_cell_sat(const Ctx& c, hipStream_t s);
void group_targets(const Ctx& c, const double4* sp, const uint32_t* orig, int64_t M, TargetSet& ts, hipStream_t s);
void centre_targets(const Ctx& c, TargetSet& ts, hipStream_t s);
void scan_exclusive_i64(const int64_t* in, int64_t* out, int64_t n, hipStream_t s);
void sum_i64(const int64_t* in, int64_t n, int64_t* out, hipStream_t s);   // *out = sum (device)
void fill_f64(double* p, double v, int64_t n, hipStream_t s);
void fill_f32(float* p, float v, int64_t n, hipStream_t s);
void fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);

// pairsum.hip
// out[ts.index[t]] = sum over the source list of target t (float output when
// out_f32, else double).  `skip`: optional device flag; when it is nonzero the
// kernel returns at once.  w32: float32 weights used instead of w.
void pairsum_f32(const Ctx& c, const TargetSet& ts, const double* w, bool out_f32, void* out, hipStream_t s,
                 const int* skip = nullptr, const float* w32 = nullptr);
void pairsum_f64(const Ctx& c, const TargetSet& ts, const double* w, bool out_f32, void* out, hipStream_t s,
                 const int* skip = nullptr);

// gridsum.hip: float32 grid sums without source lists, by tiles of bricks
// (a wave per tile of 1 x 2 x 1 bricks of 4 x 2 x 2 nodes; a tile's mask
// selects the bricks it evaluates; nodes of other bricks are not written, out
// is not cleared).
//   support_tiles: the tiles of the support and their masks, carved from a
//   workspace of support_tiles_ws_elems(g) int64 entries; returns the count
//   (waits for it; pinned = false: read without the pinned slots, which a
//   thread's first use allocates).  Needs a cutoff.
//   brick_sum_tiles: the sums over such a tile list; t0, t1: start/stop
//   events the launch carries (optional).  useful/examined: optional HOST
//   totals of the pairs inside the cutoff and of the pairs computed (then the
//   call waits for them).
//   brick_sum_f32: the same over a list of brick ids (nact of them).
bool brick_sum_applies(const Ctx& c, const rbf_grid& g);
int64_t support_tiles_ws_elems(const rbf_grid& g);
int64_t support_tiles(const Ctx& c, const rbf_grid& g, int64_t* ws, const int64_t** tiles, const int64_t** masks,
                      hipStream_t s, bool pinned = true);
void brick_sum_tiles(const Ctx& c, const rbf_grid& g, const int64_t* tiles, const int64_t* masks, int64_t nt,
                     const double* w_sorted, float* out, int64_t* useful, int64_t* examined, hipStream_t s,
                     hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
void brick_sum_f32(const Ctx& c, const rbf_grid& g, const int64_t* ids, int64_t nact, const double* w_sorted,
                   float* out, int64_t* useful, int64_t* examined, hipStream_t s);

// density.hip
void density_measures(const double* P, int64_t n, const double* samples, int64_t ns, double* q, double* hmax,
                      double* hfill, hipStream_t s);

// Launch timing (rbf_profile_begin / rbf_profile_end): while profiling is
// on, a ProfScope holds the start and stop events one launch carries
// (hipExtLaunchKernelGGL with start() and stop(), both null when profiling
// is off); done() after the launch.  Pair counts known only later (read back
// from the device) are given by set_pairs before rbf_profile_end.
struct ProfScope {
  ProfScope(int prec, int kind, int64_t useful, int64_t examined, hipStream_t s);
  hipEvent_t start() const;
  hipEvent_t stop() const;
  void done();
  void set_pairs(int64_t useful, int64_t examined);
  bool on;
  hipStream_t s;
  int rec = -1;
};
int profile_begin();
int profile_end(rbf_profile* out);
bool profiling();
// Issue rates of the vector ALU on the current device (rbf_measure_rates).
void measure_rates(rbf_rates* r, hipStream_t s);
// The float32 pair kernel's chunk bodies on register operands (pairsum.hip):
// blocks x 256 lanes x iters x 16 pair steps.
void launch_step_rate(bool masked, float* out, int blocks, int iters, hipStream_t s);

// schwarz.hip
int schwarz_overlap_count(int ncore, int pct);
int schwarz_core_cap(int max_block, int pct);
SchwarzData* schwarz_setup(const Ctx& c, int max_block, int pct, int restricted, int min_block, double shift,
                           int tune, bool half, hipStream_t s);
void schwarz_apply(const Ctx& c, const SchwarzData& d, const double* r, double* z, hipStream_t s,
                   const int* skip = nullptr);
void schwarz_apply_f32(const Ctx& c, const SchwarzData& d, const float* r, float* z, hipStream_t s,
                       const int* skip = nullptr);
void free_schwarz(SchwarzData* d);

// mlp.hip
int net_param_count();
NetData* net_create(const float* host_params, const double centre[3], double scale, double tau, hipStream_t s);
void free_net(NetData* d);
void net_get(const NetData& d, float* host_params, hipStream_t s);
void net_forward(const NetData& d, const double* X, int64_t B, float* y, hipStream_t s);
double net_step(NetData& d, const double* X, const double* f, int64_t B, float* grad, bool adam, double lr,
                hipStream_t s);
void net_eval_grid_culled(const Ctx& c, const NetData& d, const double* w_sorted, const rbf_grid& g, float* out,
                          double e_val, int reach, NetCullStats* st, hipStream_t s);

// krylov.hip
void vec_add(double* x, const double* y, int64_t n, hipStream_t s);
void gather_to_sorted(const double* src, const uint32_t* perm, int64_t m, double* dst_sorted, hipStream_t s);
// 0 / +eps / -eps of the paper-order centres (n points each), in sorted order
void rhs_sorted(const uint32_t* perm, int64_t m, int64_t n, double eps, double* dst_sorted, hipStream_t s);
void scatter_from_sorted(const double* src_sorted, const uint32_t* perm, int64_t m, double* dst, hipStream_t s);

// setup.hip: targets of the evaluation entry points.  Grid nodes go by
// bricks of 4 x 2 x 2 (x fastest), brick b = bx + nb[0] (by + nb[1] bz).
struct GridDesc {
  double o[3], h[3];
  int64_t n[3];
  int64_t nb[3];
};
GridDesc grid_desc(const rbf_grid& g);
// Ids of the bricks with a centre within the cutoff of one of their nodes
// (*ids = null and every brick without a cutoff); *ids is a temporary.
int64_t support_bricks(const Ctx& c, const rbf_grid& g, int64_t** ids, hipStream_t s);
// mark[b] = 1 for the bricks of the support (those support_bricks lists).
void mark_support(const Ctx& c, const GridDesc& gd, int64_t* mark, int64_t nbricks, hipStream_t s);
void brick_targets(const Ctx& c, const rbf_grid& g, const int64_t* ids, int64_t nact, TargetSet& ts,
                   hipStream_t s);
void grid_targets(const Ctx& c, const rbf_grid& g, TargetSet& ts, hipStream_t s);
void free_targets(TargetSet& ts);
void point_targets(const Ctx& c, const double* pts, int64_t npts, TargetSet& ts, hipStream_t s);

}  // namespace rbf
