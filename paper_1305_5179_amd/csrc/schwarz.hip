// Overlapping Schwarz preconditioner (Sec. III.A: the domain is split into
// overlapping subdomains, the local systems are solved independently and
// their solutions combined, added up everywhere (additive Schwarz) or kept
// only on the non-overlapping parts (restricted additive Schwarz), as the
// preconditioner of GMRES).
//
// Subdomains.  Cores (the non-overlapping parts) are the leaves of an octree
// over the surface points: root cube at the points' componentwise minimum,
// side = their largest extent, 1024 finest cells per axis; a cell is split
// while it holds more than `cap` points, and a core holds the three centres
// of each of its points.  The points are sorted (stably) by the Hilbert
// index of their finest cell; the cells of every level are then contiguous
// ranges sharing a key prefix, and the host splits the ranges by key digits.
// Optionally, consecutive leaves of the octree's depth-first order are
// joined up to a minimum block size.  The overlap of a core is the
// k = ceil(pct |core| / 100) centres outside it nearest to it (float64
// squared distance to the nearest core centre, ties by index), searched on
// the device one workgroup per subdomain.
//
// Local inverses.  The untruncated Gaussian of a subdomain plus shift I is
// assembled and inverted in float64 by symmetric Gauss-Jordan sweeps:
// sweeping every pivot of a symmetric positive definite matrix leaves
// -A^{-1}, and every pivot is a Schur complement, so a pivot <= 0 means the
// shift is too small and the subdomain is redone with ten times the shift.
// The sweep runs 64 pivots at a time on the block's lower triangle in a
// global work space of its workgroup, its products on the FP64 matrix
// cores.  One persistent launch takes the subdomains from a queue, largest
// first.  The inverses are kept in float32, full n x n.
//
// Apply.  One persistent launch takes strips of rows of the blocks; a task
// gathers the vector on its block's members into LDS and forms its rows of
// W r, a lane per row (W is symmetric, so lane p reads column p of each row
// b: consecutive lanes, consecutive addresses).  The restricted form
// scatters the core rows (the cores partition the centres); the additive
// form stores every row, and a second kernel sums, for every centre, the
// rows of the subdomains that hold it, in subdomain order.
#include <algorithm>
#include <functional>
#include <type_traits>
#include <vector>

#include "common.h"

namespace rbf {

namespace {

constexpr int kOvThreads = 256;
// The overlap search's LDS is sized for blocks of up to MAXB centres (cores
// and overlaps): 256 for the usual block sizes (several workgroups per
// compute unit), kSchwarzMaxBlock otherwise.  Its candidate buffer holds the
// best k and at least one round of candidates.
constexpr int kOvSmall = 256;
template <int MAXB>
constexpr int ov_cand_cap() {
  return MAXB <= kOvSmall ? 4 * MAXB : 2 * MAXB;
}
static_assert(ov_cand_cap<kOvSmall>() >= kOvSmall + kOvThreads, "the best k and one round of candidates fit");
static_assert(ov_cand_cap<kSchwarzMaxBlock>() >= kSchwarzMaxBlock + kOvThreads,
              "the best k and one round of candidates fit");
constexpr int kFacThreads = 512;
constexpr int kPanel = 64;   // pivots per panel of the sweep
// LDS of the factor kernel: coordinates, pivot block, P of a tile, two Q buffers, a column
constexpr int kFacWords = 3 * kSchwarzMaxBlock + 4 * kPanel * kPanel + 3 * kPanel;
static_assert(kFacWords * 8 + 64 <= 160 * 1024, "the factor kernel's LDS fits a compute unit");
static_assert(kFacThreads == 512 && kPanel == 64,
              "the eight waves of a workgroup own two 16 x 16 blocks each of a 64 x 64 tile");

// ---------------------------------------------------------------------------
// Bounding box of every core (one wave per subdomain).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_schwarz_box(const double* __restrict__ X, const int64_t* __restrict__ core_off,
                                                    const uint32_t* __restrict__ core_mem, double* __restrict__ box) {
  const int64_t sub = blockIdx.x;
  const int64_t a = core_off[sub], b = core_off[sub + 1];
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t e = a + threadIdx.x; e < b; e += 64) {
    const uint32_t j = core_mem[e];
    for (int d = 0; d < 3; ++d) {
      const double v = X[3 * (int64_t)j + d];
      lo[d] = fmin(lo[d], v);
      hi[d] = fmax(hi[d], v);
    }
  }
  for (int off = 32; off > 0; off >>= 1)
    for (int d = 0; d < 3; ++d) {
      lo[d] = fmin(lo[d], __shfl_xor(lo[d], off));
      hi[d] = fmax(hi[d], __shfl_xor(hi[d], off));
    }
  if (threadIdx.x == 0)
    for (int d = 0; d < 3; ++d) {
      box[6 * sub + d] = lo[d];
      box[6 * sub + 3 + d] = hi[d];
    }
}

// Squared distance from a point to a box (0 inside).
__device__ __forceinline__ double box_dist2(double x, double y, double z, const double* bx) {
  const double gx = fmax(0.0, fmax(bx[0] - x, x - bx[3]));
  const double gy = fmax(0.0, fmax(bx[1] - y, y - bx[4]));
  const double gz = fmax(0.0, fmax(bx[2] - z, z - bx[5]));
  return (gx * gx + gy * gy) + gz * gz;
}
__device__ __forceinline__ double box_box_dist2(const double* a, const double* b) {
  double s = 0.0;
  for (int d = 0; d < 3; ++d) {
    const double g = fmax(0.0, fmax(a[d] - b[3 + d], b[d] - a[3 + d]));
    s += g * g;
  }
  return s;
}

__device__ __forceinline__ bool lex_less(double da, uint32_t ia, double db, uint32_t ib) {
  return da < db || (da == db && ia < ib);
}

struct OvArgs {
  const double* X;          // paper-order centres, m x 3
  int64_t nsub;
  const int64_t* core_off;  // nsub + 1
  const uint32_t* core_mem; // paper indices of the core centres
  const double* box;        // 6 per subdomain
  const int32_t* kcount;    // overlap size per subdomain
  const int64_t* ov_off;    // nsub + 1
  const double* rho;        // search radius per subdomain
  const int32_t* list;      // subdomains to process (null: blockIdx.x)
  int unbounded;            // 1: every centre is a candidate
  uint32_t* ov_mem;         // out: paper indices, nearest first
  int32_t* short_of;        // out: 1 where fewer than k centres lie within rho
};

// The k nearest centres outside one core.  Candidates (leaves whose box is
// within rho of the core box, then centres within rho of it, then an exact
// set distance <= rho^2) collect in an LDS buffer that also holds, at its
// front, the best k found so far; when it fills, k rounds of a block-wide
// lexicographic argmin keep the best k.  The selection depends only on the
// (distance, index) pairs, not on the order in which candidates arrive.
template <int MAXB>
__global__ __launch_bounds__(kOvThreads) void k_schwarz_overlap(OvArgs a) {
  constexpr int kCandCap = ov_cand_cap<MAXB>();
  __shared__ double cx[MAXB], cy[MAXB], cz[MAXB];
  __shared__ double cd[kCandCap];
  __shared__ uint32_t ci[kCandCap];
  __shared__ double bd[MAXB];
  __shared__ uint32_t bi[MAXB];
  __shared__ int32_t leaves[kOvThreads];
  __shared__ double wd[kOvThreads / 64];
  __shared__ uint32_t wi[kOvThreads / 64];
  __shared__ int32_t wp[kOvThreads / 64];
  __shared__ double mybox[6];
  __shared__ int s_nc, s_nl, s_found;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t sub = a.list ? a.list[blockIdx.x] : (int64_t)blockIdx.x;
  const int64_t c0 = a.core_off[sub];
  const int ncore = (int)(a.core_off[sub + 1] - c0);
  const int k = a.kcount[sub];
  const double rho = a.rho[sub];
  const double rho2 = rho * rho;
  const double margin = rho2 * (1.0 + 1e-9) + 1e-300;   // prefilters never drop a centre within rho
  for (int p = tid; p < ncore; p += kOvThreads) {
    const uint32_t j = a.core_mem[c0 + p];
    cx[p] = a.X[3 * (int64_t)j];
    cy[p] = a.X[3 * (int64_t)j + 1];
    cz[p] = a.X[3 * (int64_t)j + 2];
  }
  if (tid < 6) mybox[tid] = a.box[6 * sub + tid];
  if (tid == 0) s_nc = 0;
  __syncthreads();

  // keep the best k of cd/ci[0, nc) at its front, in increasing order
  auto merge = [&]() {
    const int nc = s_nc;
    int taken = 0;
    for (int r = 0; r < k; ++r) {
      double d = INFINITY;
      uint32_t id = 0xffffffffu;
      int pos = -1;
      for (int e = tid; e < nc; e += kOvThreads)
        if (cd[e] != INFINITY && lex_less(cd[e], ci[e], d, id)) {
          d = cd[e];
          id = ci[e];
          pos = e;
        }
      for (int off = 32; off > 0; off >>= 1) {
        const double d2 = __shfl_xor(d, off);
        const uint32_t i2 = __shfl_xor(id, off);
        const int p2 = __shfl_xor(pos, off);
        if (lex_less(d2, i2, d, id)) {
          d = d2;
          id = i2;
          pos = p2;
        }
      }
      if (lane == 0) {
        wd[wave] = d;
        wi[wave] = id;
        wp[wave] = pos;
      }
      __syncthreads();
      if (tid == 0) {
        double bdv = wd[0];
        uint32_t biv = wi[0];
        int bp = wp[0];
        for (int w = 1; w < kOvThreads / 64; ++w)
          if (lex_less(wd[w], wi[w], bdv, biv)) {
            bdv = wd[w];
            biv = wi[w];
            bp = wp[w];
          }
        s_found = bp >= 0 ? 1 : 0;
        if (bp >= 0) {
          bd[r] = bdv;
          bi[r] = biv;
          cd[bp] = INFINITY;
        }
      }
      __syncthreads();
      if (!s_found) break;
      ++taken;
    }
    for (int r = tid; r < taken; r += kOvThreads) {
      cd[r] = bd[r];
      ci[r] = bi[r];
    }
    if (tid == 0) s_nc = taken;
    __syncthreads();
  };

  for (int64_t l0 = 0; l0 < a.nsub; l0 += kOvThreads) {
    if (tid == 0) s_nl = 0;
    __syncthreads();
    const int64_t L = l0 + tid;
    if (L < a.nsub && L != sub && (a.unbounded || box_box_dist2(a.box + 6 * L, mybox) <= margin))
      leaves[atomicAdd(&s_nl, 1)] = (int32_t)L;
    __syncthreads();
    const int nl = s_nl;
    for (int q = 0; q < nl; ++q) {
      const int64_t L2 = leaves[q];
      const int64_t b0 = a.core_off[L2];
      const int cnt = (int)(a.core_off[L2 + 1] - b0);
      for (int c0 = 0; c0 < cnt; c0 += kOvThreads) {
        if (c0 + tid < cnt) {
          const uint32_t j = a.core_mem[b0 + c0 + tid];
          const double x = a.X[3 * (int64_t)j], y = a.X[3 * (int64_t)j + 1], z = a.X[3 * (int64_t)j + 2];
          if (a.unbounded || box_dist2(x, y, z, mybox) <= margin) {
            double best = INFINITY;
            for (int p = 0; p < ncore; ++p) {
              const double dx = x - cx[p], dy = y - cy[p], dz = z - cz[p];
              best = fmin(best, (dx * dx + dy * dy) + dz * dz);
            }
            if (a.unbounded || best <= rho2) {
              const int slot = atomicAdd(&s_nc, 1);
              cd[slot] = best;
              ci[slot] = j;
            }
          }
        }
        __syncthreads();
        if (s_nc > kCandCap - kOvThreads) merge();
      }
    }
  }
  merge();
  const int found = s_nc;
  for (int r = tid; r < found && r < k; r += kOvThreads) a.ov_mem[a.ov_off[sub] + r] = ci[r];
  if (tid == 0) a.short_of[sub] = found < k ? 1 : 0;
}

// ---------------------------------------------------------------------------
// Local inverses: one persistent launch, a subdomain per workgroup at a time.
// ---------------------------------------------------------------------------
// Storage of a block's inverse W (n x n, symmetric) in column quads: columns
// 4q .. 4q+3 of every row r lie together at (q * ld + r) * 4 + (c & 3),
// with ld rows (n, or with float16 entries n rounded up to even) and
// ceil(n / 4) quads (the pad columns hold 0).  A lane that forms row r of
// W x (rows r, r + 1 with float16 entries) reads its four (eight) entries of
// a quad as one 16-byte load.
__host__ __device__ inline int quad_rows(int n, bool half) { return half ? (n + 1) & ~1 : n; }
__host__ __device__ inline int64_t quad_elems(int n, bool half) {
  return (int64_t)((n + 3) >> 2) * 4 * quad_rows(n, half);
}
__host__ __device__ inline int64_t quad_at(int col, int row, int ld) {
  return ((int64_t)(col >> 2) * ld + row) * 4 + (col & 3);
}

struct FacArgs {
  const double4* xs;        // sorted centres
  const int64_t* mem_off;   // nsub + 1
  const uint32_t* mem;      // sorted positions
  const int32_t* order;     // subdomains, largest first
  int64_t nsub;
  const int64_t* woff;
  double two_s2;            // 2 sigma^2
  double shift;
  int max_retry;
  float* W;                 // float32 inverses (column quads), or null
  _Float16* W16;            // float16 inverses (column quads), or null
  double* shift_used;
  int32_t* retries;
  int* failed;
  int* queue;
  double* big;              // float64 work space per workgroup
  int64_t big_ld;           // its leading dimension (the largest block)
  int64_t big_stride;       // doubles per workgroup: big_ld^2 + 2 kPanel big_ld
};

typedef double v4d __attribute__((ext_vector_type(4)));

// The replay of a panel's pivot steps (see sweep_global) on R rows at
// once: lane j of a row's 16 lanes holds its entries j, j + 16, j + 32,
// j + 48 in sv[r], and collects E of the steps it owns (k % 16 == j) in
// ev[r]; the rows' chains of dependent steps interleave, and share the
// step table's loads.
template <int R>
__device__ __forceinline__ void replay_steps(double (&sv)[R][4], double (&ev)[R][4], int lane, const double* H,
                                             const double* dd) {
  const int j = lane & 15;
  for (int k = 0; k < kPanel; ++k) {
    const int ku = k >> 4;
    const int src = (lane & ~15) | (k & 15);
    const bool own = j == (k & 15);
    const double dk = dd[k], rk = dd[kPanel + k];
    double h[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) h[u] = H[k * kPanel + j + 16 * u];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double own_v = ku == 0 ? sv[r][0] : ku == 1 ? sv[r][1] : ku == 2 ? sv[r][2] : sv[r][3];
      const double c = __shfl(own_v, src);
      const double t = c * dk;
      const double e = c * rk;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double upd = fma(-t, h[u], sv[r][u]);
        sv[r][u] = own && u == ku ? t : upd;
        ev[r][u] = own && u == ku ? e : ev[r][u];
      }
    }
  }
}

__device__ __forceinline__ double gauss_entry(const double* px, const double* py, const double* pz, int i, int j,
                                              double shift, double two_s2) {
  if (i == j) return 1.0 + shift;
  const double dx = px[i] - px[j], dy = py[i] - py[j], dz = pz[i] - pz[j];
  return exp(-((dx * dx + dy * dy) + dz * dz) / two_s2);
}

// Every row outside the panel [K, K + kb): its panel entries (left of the
// panel read along the panel's rows, below it along the row itself) replay
// the panel's pivot steps; the final entries go to Pg, the factors E of the
// trailing update to Qg (both by panel column, leading dimension ld).
template <int R>
__device__ __forceinline__ void replay_rows(const double* G, double* Pg, double* Qg, int64_t ld, const double* H,
                                            const double* dd, int n, int K, int kb) {
  const int tid = threadIdx.x, lane = tid & 63, j = lane & 15;
  for (int i0 = (tid >> 4) * R; i0 < n; i0 += (kFacThreads / 16) * R) {
    // (rows in the panel or past the end ride along with zeros and are not
    // stored; a group with none to do skips the steps; the same for the 16
    // lanes of a row)
    bool any = false;
#pragma unroll
    for (int r = 0; r < R; ++r) any |= i0 + r < n && (i0 + r < K || i0 + r >= K + kb);
    if (!any) continue;
    double sv[R][4], ev[R][4];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = i0 + r;
      const bool row_ok = i < n && (i < K || i >= K + kb);
      const double* src = i < K ? G + (int64_t)K * n + i : G + (int64_t)i * n + K;
      const int64_t step = i < K ? n : 1;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int M = j + 16 * t;
        sv[r][t] = row_ok && M < kb ? src[M * step] : 0.0;
        ev[r][t] = 0.0;
      }
    }
    replay_steps<R>(sv, ev, lane, H, dd);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = i0 + r;
      if (!(i < n && (i < K || i >= K + kb))) continue;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int M = j + 16 * t;
        if (M < kb) {
          Pg[(int64_t)M * ld + i] = sv[r][t];
          Qg[(int64_t)M * ld + i] = ev[r][t];
        }
      }
    }
  }
}

// Every block: the matrix G in global memory, of which only the lower
// triangle (i >= j) is kept (the swept matrix stays symmetric), swept kPanel
// pivots at a time with the arithmetic of the one-pivot sweep reordered:
//   * the panel's pivot block D is swept in LDS pivot by pivot, recording
//     at each step k its pivot d_k and its row H[k] as they were then;
//   * every row outside the panel replays those steps on its own panel
//     entries in registers (what the one-pivot sweep does to them), giving the row's
//     final panel entries P and, from the entry c of column k at step k,
//     E_k = c / sqrt(d_k);
//   * the entries outside the panel, which the one-pivot sweep updates by
//     -c_i c_j / d_k at each step, take the whole panel at once:
//     G_ij -= E_i . E_j, over 64 x 64 tiles on or below the diagonal, on the
//     FP64 matrix cores, the next tile's entries and E rows loaded while the
//     current one computes;
//   * P goes into the panel's row and column, the swept D into its diagonal
//     block.
// (Forming P = Q D^{-1} with the explicit inverse of the pivot block instead
// loses accuracy when D is ill conditioned: small shifts.)
__device__ bool sweep_global(double* G, double* Pg, double* Qg, int64_t ld, double* lds, const double* px,
                             const double* py, const double* pz, int n, double shift, double two_s2) {
  constexpr int kT = kPanel * kPanel;
  const int tid = threadIdx.x;
  double* D = lds;                        // kPanel x kPanel, row-major (symmetric)
  double* PT = D + kT;                    // PT[l][r]: E of a tile's rows, by panel column
  double* QB = PT + kT;                   // two buffers QB[b][l][r]: E of a tile's columns
  double* colv = QB + 2 * kT;             // kPanel
  double* dd = colv + kPanel;             // 1 / d_k, then 1 / sqrt(d_k), of the panel's pivots
  double* H = PT;                         // H[k][m]: row k of the pivot block when pivot k is swept
  __syncthreads();
  for (int64_t e = tid; e < (int64_t)n * n; e += kFacThreads) {
    const int i = (int)(e / n), j = (int)(e - (int64_t)i * n);
    if (i >= j) G[e] = gauss_entry(px, py, pz, i, j, shift, two_s2);
  }
  const int nt = (n + kPanel - 1) / kPanel;
  const int wave = tid >> 6, lane = tid & 63;
  for (int p = 0; p < nt; ++p) {
    const int K = p * kPanel, kb = min(kPanel, n - K);
    __syncthreads();
    for (int e = tid; e < kT; e += kFacThreads) {
      const int r = e / kPanel, c = e % kPanel;
      D[e] = r < kb && c < kb ? G[(int64_t)(K + max(r, c)) * n + K + min(r, c)] : 0.0;
      H[e] = 0.0;   // (steps beyond kb stay zero: no-ops in the replay)
    }
    if (tid < 2 * kPanel) dd[tid] = 0.0;
    __syncthreads();
    for (int k = 0; k < kb; ++k) {
      const double d = D[k * kPanel + k];
      if (!(d > 0.0) || !isfinite(d)) return false;
      if (tid < kPanel) {
        const double v = tid < kb ? D[tid * kPanel + k] : 0.0;
        colv[tid] = v;
        H[k * kPanel + tid] = v;
      }
      const double inv = 1.0 / d;
      if (tid == 0) {
        dd[k] = inv;
        dd[kPanel + k] = 1.0 / sqrt(d);
      }
      __syncthreads();
      for (int e = tid; e < kT; e += kFacThreads) {
        const int r = e / kPanel, c = e % kPanel;
        if (r >= kb || c >= kb) continue;
        if (r != k && c != k)
          D[e] = fma(-(colv[r] * inv), colv[c], D[e]);
        else if (r == k && c == k)
          D[e] = -inv;
        else
          D[e] = (r == k ? colv[c] : colv[r]) * inv;
      }
      __syncthreads();
    }
    // every row outside the panel, one per 16-lane row of a wave (each lane
    // holding 4 of its panel entries, m = lane % 16 + 16 t; left of the
    // panel they are read along the panel's rows, below it along the row
    // itself), replays the panel's pivot steps exactly as the one-pivot
    // sweep would apply them to it: at step k the entry c of column k is
    // the pivot column's, every other panel entry m takes
    // -(c / d_k) H[k][m], and the entry k becomes c / d_k.  E = c / sqrt(d_k)
    // of every step is the row's factor of the trailing update; the final
    // entries are P.  Every step runs (the steps beyond kb have zero H rows
    // and pivot factors and change nothing).
    // (four rows per 16 lanes for large blocks, whose rows are many; one for
    // small blocks, where more rows per lane would be mostly padding)
    if (n > 4 * (kFacThreads / 16))
      replay_rows<4>(G, Pg, Qg, ld, H, dd, n, K, kb);
    else
      replay_rows<1>(G, Pg, Qg, ld, H, dd, n, K, kb);
    __syncthreads();
    // the update of the lower tiles outside the panel's row and column
    for (int ti = 0; ti < nt; ++ti) {
      if (ti == p) continue;
      const int i0 = ti * kPanel, ri = min(kPanel, n - i0);
      const int nj = ti + 1;   // tiles tj = 0 .. ti, the panel's skipped
      __syncthreads();
      for (int e = tid; e < kT; e += kFacThreads) {
        const int l = e / kPanel, r = e % kPanel;
        PT[e] = l < kb && r < ri ? Qg[(int64_t)l * ld + i0 + r] : 0.0;
      }
      // tile tj on the matrix cores: wave w owns the 16 x 16 blocks (bi,
      // bj) and (bi, bj + 1) of the tile, its accumulators in the result
      // layout of v_mfma_f64_16x16x4f64 (lane l, value v: row l / 16 + 4 v,
      // column l % 16 of the block); the next tile's entries and E rows (8
      // per thread) are loaded while the current one computes
      const int bi = wave >> 1, bj = 2 * (wave & 1);
      v4d g0, g1, gn0, gn1;
      double qn[kT / kFacThreads];
      auto load_tile = [&](int tj, v4d& x0, v4d& x1, double (&qv)[kT / kFacThreads]) {
        const int j0 = tj * kPanel, rj = min(kPanel, n - j0);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 16 * bi + (lane >> 4) + 4 * v, c0 = 16 * bj + (lane & 15), c1 = c0 + 16;
          x0[v] = r < ri && c0 < rj ? G[(int64_t)(i0 + r) * n + j0 + c0] : 0.0;
          x1[v] = r < ri && c1 < rj ? G[(int64_t)(i0 + r) * n + j0 + c1] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < kT / kFacThreads; ++k) {
          const int e = tid + k * kFacThreads, l = e / kPanel, r = e % kPanel;
          qv[k] = l < kb && r < rj ? Qg[(int64_t)l * ld + j0 + r] : 0.0;
        }
      };
      auto next_tile = [&](int tj) { return tj + 1 == p ? tj + 2 : tj + 1; };
      int tj = p == 0 ? 1 : 0;
      if (tj >= nj) continue;
      load_tile(tj, g0, g1, qn);
#pragma unroll
      for (int k = 0; k < kT / kFacThreads; ++k) QB[tid + k * kFacThreads] = qn[k];
      __syncthreads();
      for (int b = 0; tj < nj; b ^= 1) {
        const int tn = next_tile(tj);
        if (tn < nj) load_tile(tn, gn0, gn1, qn);
        // G_ij -= sum_l E_il E_jl: A = -E (rows of the tile), B = E^T
        const double* Q = QB + b * kT;
#pragma unroll 4
        for (int kk = 0; kk < kPanel / 4; ++kk) {
          const int l = 4 * kk + (lane >> 4);
          const double a = -PT[l * kPanel + 16 * bi + (lane & 15)];
          g0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Q[l * kPanel + 16 * bj + (lane & 15)], g0, 0, 0, 0);
          g1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Q[l * kPanel + 16 * (bj + 1) + (lane & 15)], g1, 0, 0, 0);
        }
        const int j0 = tj * kPanel, rj = min(kPanel, n - j0);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 16 * bi + (lane >> 4) + 4 * v, c0 = 16 * bj + (lane & 15), c1 = c0 + 16;
          if (r < ri && c0 < rj) G[(int64_t)(i0 + r) * n + j0 + c0] = g0[v];
          if (r < ri && c1 < rj) G[(int64_t)(i0 + r) * n + j0 + c1] = g1[v];
        }
        if (tn < nj) {
#pragma unroll
          for (int k = 0; k < kT / kFacThreads; ++k) QB[(b ^ 1) * kT + tid + k * kFacThreads] = qn[k];
          g0 = gn0;
          g1 = gn1;
        }
        __syncthreads();
        tj = tn;
      }
    }
    // the panel's row (left of the diagonal block), column (below it) and
    // diagonal block
    for (int64_t e = tid; e < (int64_t)kb * K; e += kFacThreads) {
      const int r = (int)(e / K), j = (int)(e - (int64_t)r * K);
      G[(int64_t)(K + r) * n + j] = Pg[(int64_t)r * ld + j];
    }
    // (by panel column, so that the reads are contiguous; the stores wait
    // for nothing)
    const int below = n - K - kb;
    for (int64_t e = tid; e < (int64_t)below * kb; e += kFacThreads) {
      const int c = (int)(e / below), i = K + kb + (int)(e % below);
      G[(int64_t)i * n + K + c] = Pg[(int64_t)c * ld + i];
    }
    for (int e = tid; e < kT; e += kFacThreads) {
      const int r = e / kPanel, c = e % kPanel;
      if (r < kb && c <= r) G[(int64_t)(K + r) * n + K + c] = D[e];
    }
  }
  __syncthreads();
  return true;
}

__global__ __launch_bounds__(kFacThreads) void k_schwarz_factor(FacArgs a) {
  __shared__ double lds[kFacWords];
  __shared__ int s_task;
  const int tid = threadIdx.x;
  double* const big = a.big + (int64_t)blockIdx.x * a.big_stride;
  for (;;) {
    __syncthreads();
    if (tid == 0) s_task = atomicAdd(a.queue, 1);
    __syncthreads();
    const int64_t task = s_task;
    if (task >= a.nsub) break;   // every workgroup reaches this once the queue is drained
    const int64_t sub = a.order[task];
    const int64_t off = a.mem_off[sub];
    const int n = (int)(a.mem_off[sub + 1] - off);
    // coordinates at the front of the LDS, before the panel buffers
    double* px = lds;
    double* py = px + kSchwarzMaxBlock;
    double* pz = py + kSchwarzMaxBlock;
    __syncthreads();
    for (int p = tid; p < n; p += kFacThreads) {
      const double4 x = a.xs[a.mem[off + p]];
      px[p] = x.x;
      py[p] = x.y;
      pz[p] = x.z;
    }
    double shift = a.shift;
    int tries = 0;
    bool ok = false;
    for (;;) {
      if (sweep_global(big, big + a.big_ld * a.big_ld, big + a.big_ld * (a.big_ld + kPanel), a.big_ld,
                       pz + kSchwarzMaxBlock, px, py, pz, n, shift, a.two_s2)) {
        ok = true;
        break;
      }
      if (++tries > a.max_retry) break;
      shift = shift > 0.0 ? 10.0 * shift : 1e-10;
    }
    __syncthreads();
    // W = -(swept matrix), full n x n in column quads; the lower triangle
    // holds the result: read along its rows, each entry stored at (i, j) and
    // (j, i); then the pad columns of the last quad, 0 in every row
    const int npad = 4 * ((n + 3) >> 2) - n;
    if (a.W16) {
      _Float16* W = a.W16 + a.woff[sub];
      const int ld = quad_rows(n, true);
      for (int64_t e = tid; e < (int64_t)n * n; e += kFacThreads) {
        const int i = (int)(e / n), j = (int)(e - (int64_t)i * n);
        if (j > i) continue;
        const _Float16 v = ok ? (_Float16)(float)(-big[e]) : (_Float16)0.0f;
        W[quad_at(j, i, ld)] = v;
        W[quad_at(i, j, ld)] = v;
      }
      for (int e = tid; e < npad * ld; e += kFacThreads) W[quad_at(n + e / ld, e % ld, ld)] = (_Float16)0.0f;
    } else {
      float* W = a.W + a.woff[sub];
      const int ld = quad_rows(n, false);
      for (int64_t e = tid; e < (int64_t)n * n; e += kFacThreads) {
        const int i = (int)(e / n), j = (int)(e - (int64_t)i * n);
        if (j > i) continue;
        const float v = ok ? (float)(-big[e]) : 0.0f;
        W[quad_at(j, i, ld)] = v;
        W[quad_at(i, j, ld)] = v;
      }
      for (int e = tid; e < npad * ld; e += kFacThreads) W[quad_at(n + e / ld, e % ld, ld)] = 0.0f;
    }
    if (tid == 0) {
      a.shift_used[sub] = shift;
      a.retries[sub] = tries;
      if (!ok) atomicOr(a.failed, 1);
    }
  }
}

// ---------------------------------------------------------------------------
// Apply.
// ---------------------------------------------------------------------------
struct ApplyArgs {
  const int2* tasks;        // (subdomain, first row), largest first
  int64_t ntask;
  const int64_t* mem_off;
  const int32_t* ncore;
  const uint32_t* mem;
  const int64_t* woff;
  const float* W;           // float32 inverses (column quads), or
  const _Float16* W16;      // float16 inverses (column quads)
  const void* r;            // float64, or float32 with F32
  void* out;                // restricted: z (sorted order; float32 with F32); additive: the local solutions
                            // by member slot (float64)
  const int* skip;
};

// One persistent launch: workgroup b takes tasks b, b + gridDim.x, ...; a
// task gathers its block's vector into LDS (0 in the last quad's pad) and
// forms T rows of W r, a lane per row, or two with float16 entries (W is
// symmetric and stored in column quads: lane p reads its row's entries of a
// quad, consecutive lanes at consecutive addresses, 16 bytes each).  The
// restricted form scatters the core rows (the cores partition the
// centres); the additive form stores every row by member slot.
template <bool RESTRICTED, int T, bool F32, bool HALF>
__global__ __launch_bounds__(T) void k_schwarz_local(ApplyArgs a) {
  if (a.skip && *a.skip) return;
  __shared__ __align__(16) double rl[kSchwarzMaxBlock];
  float* rlf = reinterpret_cast<float*>(rl);   // the float32 copy of the HALF form
  const int tid = threadIdx.x;
  // quads' loads in flight per wave before the first is used
  constexpr int kQ = 8;
  // a lane's entries of one quad: rows (row, row + 1) in float16, or row in float32
  using Quad = typename std::conditional<HALF, uint4, float4>::type;
  for (int64_t t = blockIdx.x; t < a.ntask; t += gridDim.x) {
    const int2 task = a.tasks[t];
    const int64_t sub = task.x;
    const int64_t off = a.mem_off[sub];
    const int n = (int)(a.mem_off[sub + 1] - off);
    const int nq = (n + 3) >> 2;
    const int rows = RESTRICTED ? a.ncore[sub] : n;
    // this lane's rows (row is even in the HALF form, so the eight entries
    // of a quad are one aligned 16-byte load; the pad row of an odd block
    // feeds a row that is not stored) and the stride of its quads
    const int row = task.y + (HALF ? 2 : 1) * tid;
    const bool active = row < rows;
    const int64_t qs = HALF ? quad_rows(n, true) >> 1 : quad_rows(n, false);
    const Quad* w = HALF ? reinterpret_cast<const Quad*>(a.W16 + a.woff[sub]) + (row >> 1)
                         : reinterpret_cast<const Quad*>(a.W + a.woff[sub]) + row;
    __syncthreads();   // the previous task is done with rl
    for (int p = tid; p < 4 * nq; p += T) {
      double x = 0.0;
      if (p < n)
        x = F32 ? (double)static_cast<const float*>(a.r)[a.mem[off + p]]
                : static_cast<const double*>(a.r)[a.mem[off + p]];
      if (HALF)
        rlf[p] = (float)x;
      else
        rl[p] = x;
    }
    __syncthreads();
    if (!active) continue;
    auto store = [&](int rr, double y) {
      if (RESTRICTED && F32)
        static_cast<float*>(a.out)[a.mem[off + rr]] = (float)y;
      else if (RESTRICTED)
        static_cast<double*>(a.out)[a.mem[off + rr]] = y;
      else
        static_cast<double*>(a.out)[off + rr] = y;
    };
    if constexpr (HALF) {
      // float32 products and sums (their rounding, at most n u32 <= 2^-14, is
      // below the float16 entries' own), each a mixed-precision FMA on the
      // float16 entry
      const float4* r4 = reinterpret_cast<const float4*>(rlf);
      auto h = [](uint32_t x, int k) { return (float)__builtin_bit_cast(_Float16, (uint16_t)(x >> (16 * k))); };
      auto quad = [&](const uint4& e8, const float4& r, float& ea, float& oa) {
        ea = __builtin_fmaf(h(e8.x, 0), r.x, ea);
        oa = __builtin_fmaf(h(e8.z, 0), r.x, oa);
        ea = __builtin_fmaf(h(e8.x, 1), r.y, ea);
        oa = __builtin_fmaf(h(e8.z, 1), r.y, oa);
        ea = __builtin_fmaf(h(e8.y, 0), r.z, ea);
        oa = __builtin_fmaf(h(e8.w, 0), r.z, oa);
        ea = __builtin_fmaf(h(e8.y, 1), r.w, ea);
        oa = __builtin_fmaf(h(e8.w, 1), r.w, oa);
      };
      float e[2] = {0.f, 0.f}, o[2] = {0.f, 0.f};
      int q = 0;
      for (; q + kQ <= nq; q += kQ) {
        Quad v[kQ];
#pragma unroll
        for (int u = 0; u < kQ; ++u) v[u] = w[(int64_t)(q + u) * qs];
#pragma unroll
        for (int u = 0; u < kQ; ++u) quad(v[u], r4[q + u], e[u & 1], o[u & 1]);
      }
      for (; q < nq; ++q) quad(w[(int64_t)q * qs], r4[q], e[0], o[0]);
      store(row, (double)(e[0] + e[1]));
      if (row + 1 < rows) store(row + 1, (double)(o[0] + o[1]));
    } else {
      // float64 products and sums of the float32 entries
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      auto quad = [&](const float4& e4, int qq, double& ac) {
        ac = fma((double)e4.x, rl[4 * qq], ac);
        ac = fma((double)e4.y, rl[4 * qq + 1], ac);
        ac = fma((double)e4.z, rl[4 * qq + 2], ac);
        ac = fma((double)e4.w, rl[4 * qq + 3], ac);
      };
      int q = 0;
      for (; q + kQ <= nq; q += kQ) {
        Quad v[kQ];
#pragma unroll
        for (int u = 0; u < kQ; ++u) v[u] = w[(int64_t)(q + u) * qs];
#pragma unroll
        for (int u = 0; u < kQ; ++u) quad(v[u], q + u, acc[u & 3]);
      }
      for (; q < nq; ++q) quad(w[(int64_t)q * qs], q, acc[0]);
      store(row, (acc[0] + acc[1]) + (acc[2] + acc[3]));
    }
  }
}

// Occurrences of the centres among the member slots (additive form): the
// slots of centre j are occ_slot[occ_off[j] .. occ_off[j + 1]), increasing
// (subdomain order).  Counted, scanned, filled in any order, then each
// centre's few slots sorted by one thread.
__global__ void k_occ_count(const uint32_t* __restrict__ mem, int64_t nmem, unsigned long long* __restrict__ cnt) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < nmem) atomicAdd(cnt + mem[e], 1ull);
}
__global__ void k_occ_fill(const uint32_t* __restrict__ mem, int64_t nmem, const int64_t* __restrict__ occ_off,
                           unsigned long long* __restrict__ fill, int64_t* __restrict__ occ_slot) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= nmem) return;
  const uint32_t j = mem[e];
  occ_slot[occ_off[j] + (int64_t)atomicAdd(fill + j, 1ull)] = e;
}
__global__ void k_occ_sort(const int64_t* __restrict__ occ_off, int64_t m, int64_t* __restrict__ occ_slot) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= m) return;
  const int64_t a = occ_off[j], b = occ_off[j + 1];
  for (int64_t x = a + 1; x < b; ++x) {
    const int64_t v = occ_slot[x];
    int64_t y = x - 1;
    while (y >= a && occ_slot[y] > v) {
      occ_slot[y + 1] = occ_slot[y];
      --y;
    }
    occ_slot[y + 1] = v;
  }
}

template <class TO>
__global__ void k_schwarz_sum(const int64_t* __restrict__ occ_off, const int64_t* __restrict__ occ_slot,
                              const double* __restrict__ Y, int64_t m, TO* __restrict__ z, const int* skip) {
  if (skip && *skip) return;
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= m) return;
  double s = 0.0;
  for (int64_t e = occ_off[j]; e < occ_off[j + 1]; ++e) s += Y[occ_slot[e]];
  z[j] = (TO)s;
}

template <class T>
T* upload(const std::vector<T>& h, hipStream_t s) {
  T* d = dalloc<T>((int64_t)std::max<size_t>(h.size(), 1));
  if (!h.empty()) RBF_HIP(hipMemcpyAsync(d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice, s));
  return d;
}
template <class T>
std::vector<T> download(const T* d, int64_t count, hipStream_t s) {
  std::vector<T> h((size_t)std::max<int64_t>(count, 0));
  if (count > 0) RBF_HIP(hipMemcpyAsync(h.data(), d, sizeof(T) * (size_t)count, hipMemcpyDeviceToHost, s));
  return h;
}

}  // namespace

int schwarz_overlap_count(int ncore, int pct) { return (ncore * pct + 99) / 100; }

int schwarz_core_cap(int max_block, int pct) {
  int p = max_block / 3;
  while (p > 1 && 3 * p + schwarz_overlap_count(3 * p, pct) > max_block) --p;
  return std::max(p, 1);
}

void free_schwarz(SchwarzData* d) {
  if (!d) return;
  for (void* p : {(void*)d->mem_off, (void*)d->ncore, (void*)d->mem, (void*)d->woff, (void*)d->W, (void*)d->W16,
                  (void*)d->Y,
                  (void*)d->occ_off, (void*)d->occ_slot, (void*)d->z, (void*)d->t, (void*)d->z32})
    dfree(p);
  dfree(d->tasks);
  delete d;
}

namespace {

// The tasks of the apply for strips of T rows: (subdomain, first row), by
// decreasing work (rows x block size), ties by subdomain and row.
std::vector<int2> apply_tasks(const SchwarzData& d, int threads) {
  // rows per task: one per thread, two with float16 inverses
  const int T = d.half ? 2 * threads : threads;
  std::vector<std::pair<int64_t, int2>> t;
  for (int64_t i = 0; i < d.nsub; ++i) {
    const int n = (int)(d.h_mem_off[i + 1] - d.h_mem_off[i]);
    const int rows = d.restricted ? d.h_ncore[i] : n;
    for (int r0 = 0; r0 < rows; r0 += T) t.push_back({(int64_t)n * std::min(T, rows - r0), make_int2((int)i, r0)});
  }
  std::stable_sort(t.begin(), t.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
  std::vector<int2> out(t.size());
  for (size_t k = 0; k < t.size(); ++k) out[k] = t[k].second;
  return out;
}

template <bool RESTRICTED, bool F32, bool HALF>
void launch_local_t(int T, const dim3& g, const ApplyArgs& aa, hipStream_t s) {
  if (T == 512)
    hipLaunchKernelGGL((k_schwarz_local<RESTRICTED, 512, F32, HALF>), g, dim3(512), 0, s, aa);
  else if (T == 256)
    hipLaunchKernelGGL((k_schwarz_local<RESTRICTED, 256, F32, HALF>), g, dim3(256), 0, s, aa);
  else
    hipLaunchKernelGGL((k_schwarz_local<RESTRICTED, 128, F32, HALF>), g, dim3(128), 0, s, aa);
  RBF_HIP(hipGetLastError());
}
template <bool RESTRICTED, bool F32>
void launch_local_h(const SchwarzData& d, int T, const dim3& g, const ApplyArgs& aa, hipStream_t s) {
  if (d.half)
    launch_local_t<RESTRICTED, F32, true>(T, g, aa, s);
  else
    launch_local_t<RESTRICTED, F32, false>(T, g, aa, s);
}

// f32: r is float32, and the restricted form writes out in float32.
void launch_local(const SchwarzData& d, int T, int blocks, const int2* tasks, int64_t ntask, const void* r,
                  void* out, hipStream_t s, const int* skip, bool f32 = false) {
  const ApplyArgs aa{tasks, ntask, d.mem_off, d.ncore, d.mem, d.woff, d.W, d.W16, r, out, skip};
  const dim3 g((unsigned)std::max(blocks, 1));
  if (d.restricted) {
    if (f32)
      launch_local_h<true, true>(d, T, g, aa, s);
    else
      launch_local_h<true, false>(d, T, g, aa, s);
  } else {
    if (f32)
      launch_local_h<false, true>(d, T, g, aa, s);
    else
      launch_local_h<false, false>(d, T, g, aa, s);
  }
}

// The workgroup size whose task (a strip of as many rows, twice as many with
// float16 inverses) covers the largest block's rows in one task: 128, 256
// or 512 threads.
int covering_threads(const SchwarzData& d) {
  int64_t rows = 0;
  for (int64_t i = 0; i < d.nsub; ++i)
    rows = std::max<int64_t>(rows, d.restricted ? d.h_ncore[i] : d.h_mem_off[i + 1] - d.h_mem_off[i]);
  const int64_t lanes = d.half ? (rows + 1) / 2 : rows;
  return lanes <= 128 ? 128 : lanes <= 256 ? 256 : 512;
}

// The apply's launch shape.  Candidates: the covering workgroup size and
// the next smaller one (two tasks for the largest blocks), each taken by 8
// workgroups per compute unit or by one workgroup per task (on the torus
// workloads these always won; 2 and 4 per compute unit and a larger size
// never did).  The task lists are built and uploaded once; after one untimed
// apply every candidate runs once between its own pair of events, all back
// to back (the work and the result do not depend on the values), and the
// host waits once; the fastest is kept.
void tune_apply(SchwarzData& d, int cus, hipStream_t s) {
  struct Cand {
    int T, mult, blocks;
    hipEvent_t e0, e1;
  };
  const int top = covering_threads(d);
  std::vector<int> Ts;
  if (top > 128) Ts.push_back(top / 2);
  Ts.push_back(top);
  const int nshape = (int)Ts.size();
  std::vector<int2*> dt(nshape);
  std::vector<int64_t> nt(nshape);
  for (int k = 0; k < nshape; ++k) {
    std::vector<int2> ht = apply_tasks(d, Ts[k]);
    dt[k] = upload(ht, s);
    nt[k] = (int64_t)ht.size();
  }
  auto shape = [&](int T) { return T == Ts[0] ? 0 : 1; };
  std::vector<Cand> cands;
  for (int k = 0; k < nshape; ++k)
    for (int mult : {8, 0}) {
      Cand c{Ts[k], mult, 0, nullptr, nullptr};
      c.blocks = mult > 0 ? (int)std::min<int64_t>((int64_t)mult * cus, nt[k]) : (int)nt[k];
      cands.push_back(c);
    }
  double* out = d.restricted ? d.z : d.Y;
  launch_local(d, cands[0].T, cands[0].blocks, dt[0], nt[0], d.t, out, s, nullptr);   // warm-up
  for (Cand& c : cands) {
    const int k = shape(c.T);
    RBF_HIP(hipEventCreate(&c.e0));
    RBF_HIP(hipEventCreate(&c.e1));
    RBF_HIP(hipEventRecord(c.e0, s));
    launch_local(d, c.T, c.blocks, dt[k], nt[k], d.t, out, s, nullptr);
    RBF_HIP(hipEventRecord(c.e1, s));
  }
  RBF_HIP(hipEventSynchronize(cands.back().e1));
  float best = INFINITY;
  int pick = 0;
  for (size_t i = 0; i < cands.size(); ++i) {
    float ms = 0.f;
    RBF_HIP(hipEventElapsedTime(&ms, cands[i].e0, cands[i].e1));
    if (ms < best) {
      best = ms;
      pick = (int)i;
    }
    RBF_HIP(hipEventDestroy(cands[i].e0));
    RBF_HIP(hipEventDestroy(cands[i].e1));
  }
  const int k = shape(cands[pick].T);
  dfree(d.tasks);
  d.tasks = dt[k];
  d.ntask = nt[k];
  for (int j = 0; j < nshape; ++j)
    if (j != k) dfree(dt[j]);
  d.apply_threads = cands[pick].T;
  d.apply_blocks = cands[pick].blocks;
}

// Depth-first (Morton) position of a cell at `level` of the 10-level
// octree, padded to the finest level: the coordinates' bits interleaved,
// x lowest.
__host__ __device__ inline uint32_t morton_full_depth(const uint32_t q[3], int level) {
  uint32_t key = 0;
  for (int b = level - 1; b >= 0; --b)
    key = (key << 3) | ((q[0] >> b) & 1u) | (((q[1] >> b) & 1u) << 1) | (((q[2] >> b) & 1u) << 2);
  return key << (3 * (kCurveBits - level));
}

// Depth-first key of every octree leaf: the cell, at the leaf's level, of
// the leaf's first point (fine-cell index of each coordinate, clamped to the
// lattice, shifted to the level).
__global__ void k_leaf_keys(const double* __restrict__ xp, const uint32_t* __restrict__ first_pt,
                            const int32_t* __restrict__ level, int64_t nleaf, Lattice L, uint32_t* __restrict__ key) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nleaf) return;
  const uint32_t pt = first_pt[i];
  const int lev = level[i];
  uint32_t q[3];
  for (int d = 0; d < 3; ++d) {
    double v = floor((xp[3 * (int64_t)pt + d] - L.origin[d]) / L.fine);
    if (!(v >= 0.0)) v = 0.0;
    if (v > (double)(kFineMax - 1)) v = (double)(kFineMax - 1);
    q[d] = (uint32_t)v >> (kCurveBits - lev);
  }
  key[i] = morton_full_depth(q, lev);
}

// Members in sorted positions: mem[e] = the sorted position of paper index
// mem_paper[e] (inv = the inverse of the sorting permutation).
__global__ void k_sorted_inverse(const uint32_t* __restrict__ perm, int64_t m, uint32_t* __restrict__ inv) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < m) inv[perm[k]] = (uint32_t)k;
}
__global__ void k_members_sorted(const uint32_t* __restrict__ mem_paper, int64_t nmem,
                                 const uint32_t* __restrict__ inv, uint32_t* __restrict__ mem) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < nmem) mem[e] = inv[mem_paper[e]];
}

}  // namespace

SchwarzData* schwarz_setup(const Ctx& c, int max_block, int pct, int restricted, int min_block, double shift,
                           int tune, bool half, hipStream_t s) {
  const int64_t n = c.n, m = c.m;
  const int cap = schwarz_core_cap(max_block, pct);
  // 1. root cube of the surface points and their Hilbert order on it
  double* box = talloc<double>(6);
  double* scratch = talloc<double>(6 * 1024);
  bounding_box(c.xpaper, n, box, scratch, s);
  std::vector<double> hbox = download(box, 6, s);
  RBF_HIP(hipStreamSynchronize(s));
  temp_free(box);
  temp_free(scratch);
  double side = 0.0;
  for (int d = 0; d < 3; ++d) side = std::max(side, hbox[3 + d] - hbox[d]);
  if (!(side > 0.0)) side = 1.0;
  Lattice L{};
  for (int d = 0; d < 3; ++d) {
    L.origin[d] = hbox[d];
    L.fdims[d] = kFineMax;
    L.cdims[d] = kFineMax;
  }
  L.fine = side / (double)kFineMax;
  L.shift = 0;
  L.coarse = L.fine;
  uint32_t* sperm = talloc<uint32_t>(n);
  uint32_t* skeys = talloc<uint32_t>(n);
  sort_points(c.xpaper, n, L, sperm, skeys, s);
  std::vector<uint32_t> hk = download(skeys, n, s), hp = download(sperm, n, s);
  RBF_HIP(hipStreamSynchronize(s));
  temp_free(sperm);
  temp_free(skeys);

  // 2. octree leaves: ranges of the sorted points
  struct Leaf {
    int64_t a, b;
    int level;
  };
  std::vector<Leaf> leaves;
  std::function<void(int64_t, int64_t, int)> visit = [&](int64_t a, int64_t b, int level) {
    if (b - a <= cap || level == kCurveBits) {
      for (int64_t q = a; q < b; q += cap) leaves.push_back({q, std::min<int64_t>(b, q + cap), level});
      return;
    }
    const int sh = 3 * (kCurveBits - 1 - level);
    int64_t q = a;
    while (q < b) {
      const uint32_t dig = (hk[q] >> sh) & 7u;
      int64_t e = q;
      while (e < b && ((hk[e] >> sh) & 7u) == dig) ++e;
      visit(q, e, level + 1);
      q = e;
    }
  };
  if (n > 0) visit(0, n, 0);

  // the leaves in depth-first order (cell key of the first point at the
  // leaf's level, then position: the runs of one finest cell in index order),
  // then consecutive leaves joined while the block is below min_block and
  // the cap allows
  const int64_t nleaf = (int64_t)leaves.size();
  std::vector<uint32_t> lfirst(nleaf);
  std::vector<int32_t> llevel(nleaf);
  for (int64_t i = 0; i < nleaf; ++i) {
    lfirst[i] = hp[leaves[i].a];
    llevel[i] = leaves[i].level;
  }
  std::vector<uint32_t> lkey;
  if (nleaf > 0) {
    uint32_t* d_first = upload(lfirst, s);
    int32_t* d_level = upload(llevel, s);
    uint32_t* d_key = dalloc<uint32_t>(nleaf);
    hipLaunchKernelGGL(k_leaf_keys, dim3((unsigned)ceil_div(nleaf, 256)), dim3(256), 0, s, c.xpaper, d_first, d_level,
                       nleaf, L, d_key);
    RBF_HIP(hipGetLastError());
    lkey = download(d_key, nleaf, s);
    RBF_HIP(hipStreamSynchronize(s));
    for (void* p : {(void*)d_first, (void*)d_level, (void*)d_key}) dfree(p);
  }
  std::vector<std::pair<uint32_t, int64_t>> dfo(nleaf);
  for (int64_t i = 0; i < nleaf; ++i) dfo[i] = {lkey[i], leaves[i].a};
  std::vector<int64_t> lorder(leaves.size());
  for (size_t i = 0; i < leaves.size(); ++i) lorder[i] = (int64_t)i;
  std::sort(lorder.begin(), lorder.end(), [&](int64_t x, int64_t y) { return dfo[x] < dfo[y]; });
  auto block_of = [&](int64_t pts) { return 3 * pts + schwarz_overlap_count((int)(3 * pts), pct); };
  std::vector<std::vector<int64_t>> groups;   // leaves of every core
  int64_t npts = 0;
  for (int64_t li : lorder) {
    const int64_t sz = leaves[li].b - leaves[li].a;
    const bool close = !groups.empty() && (min_block <= 0 || block_of(npts) >= min_block || npts + sz > cap);
    if (groups.empty() || close) {
      groups.emplace_back();
      npts = 0;
    }
    groups.back().push_back(li);
    npts += sz;
  }
  const int64_t nsub = (int64_t)groups.size();

  // 3. cores (paper indices: the points in increasing order, then their +, - offsets)
  std::vector<int64_t> core_off(nsub + 1, 0), ov_off(nsub + 1, 0);
  std::vector<uint32_t> core_mem;
  std::vector<int32_t> kcount(nsub);
  std::vector<double> rho(nsub);
  core_mem.reserve((size_t)m);
  // every point's core, then the points of every core in increasing index
  // order by one pass over the indices (a counting sort by core)
  std::vector<int32_t> core_of(n);
  std::vector<int64_t> pt_off(nsub + 1, 0);
  for (int64_t i = 0; i < nsub; ++i) {
    int64_t cnt = 0;
    for (int64_t li : groups[i]) {
      for (int64_t q = leaves[li].a; q < leaves[li].b; ++q) core_of[hp[q]] = (int32_t)i;
      cnt += leaves[li].b - leaves[li].a;
    }
    pt_off[i + 1] = pt_off[i] + cnt;
  }
  std::vector<uint32_t> pt_sorted(n);
  {
    std::vector<int64_t> at(pt_off.begin(), pt_off.end() - 1);
    for (int64_t p = 0; p < n; ++p) pt_sorted[at[core_of[p]]++] = (uint32_t)p;
  }
  for (int64_t i = 0; i < nsub; ++i) {
    double r = 0.0;
    for (int64_t li : groups[i]) r = std::max(r, std::ldexp(side, -leaves[li].level));   // the side of the leaf's cell
    for (int t = 0; t < 3; ++t)
      for (int64_t q = pt_off[i]; q < pt_off[i + 1]; ++q) core_mem.push_back((uint32_t)(pt_sorted[q] + t * n));
    const int nc = (int)(3 * (pt_off[i + 1] - pt_off[i]));
    core_off[i + 1] = core_off[i] + nc;
    kcount[i] = (int32_t)std::min<int64_t>(schwarz_overlap_count(nc, pct), m - nc);
    ov_off[i + 1] = ov_off[i] + kcount[i];
    rho[i] = r;
  }

  // 4. overlaps on the device
  int64_t* d_core_off = upload(core_off, s);
  uint32_t* d_core_mem = upload(core_mem, s);
  int32_t* d_k = upload(kcount, s);
  int64_t* d_ov_off = upload(ov_off, s);
  // the search radius: an eighth of the leaf side first (the overlap of a
  // core is a thin shell around it, about 1/40 of the side of a full leaf at
  // 10 %), then the side, then everything, for the cores still short of k
  std::vector<double> rho8(rho);
  for (double& r : rho8) r *= 0.125;
  double* d_rho = upload(rho8, s);
  double* d_rho_full = upload(rho, s);
  double* d_box = talloc<double>(6 * std::max<int64_t>(nsub, 1));
  uint32_t* d_ov = talloc<uint32_t>(std::max<int64_t>(ov_off[nsub], 1));
  int32_t* d_short = talloc<int32_t>(std::max<int64_t>(nsub, 1));
  std::vector<uint32_t> ov;
  if (nsub > 0) {
    hipLaunchKernelGGL(k_schwarz_box, dim3((unsigned)nsub), dim3(64), 0, s, c.xpaper, d_core_off, d_core_mem, d_box);
    RBF_HIP(hipGetLastError());
    OvArgs oa{c.xpaper, nsub, d_core_off, d_core_mem, d_box, d_k, d_ov_off, d_rho, nullptr, 0, d_ov, d_short};
    auto overlap = [&](unsigned blocks) {
      if (max_block <= kOvSmall)
        hipLaunchKernelGGL(k_schwarz_overlap<kOvSmall>, dim3(blocks), dim3(kOvThreads), 0, s, oa);
      else
        hipLaunchKernelGGL(k_schwarz_overlap<kSchwarzMaxBlock>, dim3(blocks), dim3(kOvThreads), 0, s, oa);
    };
    overlap((unsigned)nsub);
    RBF_HIP(hipGetLastError());
    std::vector<int32_t> short_of = download(d_short, nsub, s);
    RBF_HIP(hipStreamSynchronize(s));
    std::vector<int32_t> again;
    for (int64_t i = 0; i < nsub; ++i)
      if (short_of[i]) again.push_back((int32_t)i);
    for (int pass = 0; pass < 2 && !again.empty(); ++pass) {
      // too few centres within the radius: the leaf side, then every centre
      int32_t* d_list = upload(again, s);
      oa.list = d_list;
      oa.rho = d_rho_full;
      oa.unbounded = pass;
      overlap((unsigned)again.size());
      RBF_HIP(hipGetLastError());
      short_of = download(d_short, nsub, s);
      RBF_HIP(hipStreamSynchronize(s));
      dfree(d_list);
      std::vector<int32_t> still;
      for (int32_t i : again)
        if (short_of[i]) still.push_back(i);
      again.swap(still);
    }
    ov = download(d_ov, ov_off[nsub], s);
    RBF_HIP(hipStreamSynchronize(s));
  }
  for (void* p : {(void*)d_core_off, (void*)d_core_mem, (void*)d_k, (void*)d_ov_off, (void*)d_rho, (void*)d_rho_full,
                  (void*)d_box, (void*)d_ov, (void*)d_short})
    dfree(p);

  // 5. members in sorted positions, layout of the inverses, occurrences
  SchwarzData* d = new SchwarzData();
  d->nsub = nsub;
  d->restricted = restricted;
  d->half = half;
  d->shift = shift;
  d->max_block = max_block;
  d->pct = pct;
  d->h_mem_off.assign(nsub + 1, 0);
  d->h_ncore.resize(nsub);
  d->h_mem_paper.reserve((size_t)(core_off[nsub] + ov_off[nsub]));
  std::vector<int64_t> woff(nsub, 0);
  std::vector<int32_t> order(nsub);
  int64_t wtotal = 0;
  for (int64_t i = 0; i < nsub; ++i) {
    const int nc = (int)(core_off[i + 1] - core_off[i]);
    for (int64_t e = core_off[i]; e < core_off[i + 1]; ++e) d->h_mem_paper.push_back(core_mem[e]);
    for (int64_t e = ov_off[i]; e < ov_off[i + 1]; ++e) d->h_mem_paper.push_back(ov[e]);
    const int64_t nb = nc + (ov_off[i + 1] - ov_off[i]);
    d->h_mem_off[i + 1] = d->h_mem_off[i] + nb;
    d->h_ncore[i] = nc;
    woff[i] = wtotal;
    wtotal += quad_elems((int)nb, half);
    order[i] = (int32_t)i;
  }
  d->nmem = d->h_mem_off[nsub];
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    return d->h_mem_off[x + 1] - d->h_mem_off[x] > d->h_mem_off[y + 1] - d->h_mem_off[y];
  });
  d->mem_off = upload(d->h_mem_off, s);
  d->ncore = upload(d->h_ncore, s);
  d->mem = dalloc<uint32_t>(std::max<int64_t>(d->nmem, 1));
  if (d->nmem > 0) {
    uint32_t* d_paper = upload(d->h_mem_paper, s);
    uint32_t* d_inv = talloc<uint32_t>(m);
    hipLaunchKernelGGL(k_sorted_inverse, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, s, c.perm, m, d_inv);
    hipLaunchKernelGGL(k_members_sorted, dim3((unsigned)ceil_div(d->nmem, 256)), dim3(256), 0, s, d_paper, d->nmem,
                       d_inv, d->mem);
    RBF_HIP(hipGetLastError());
    temp_free(d_inv);
    dfree(d_paper);
  }
  d->woff = upload(woff, s);
  if (half)
    d->W16 = dalloc<_Float16>(std::max<int64_t>(wtotal, 2));
  else
    d->W = dalloc<float>(std::max<int64_t>(wtotal, 1));
  d->w_total = wtotal;
  if (!restricted) {
    // counts (m + 1 entries, the last 0), their exclusive scan, the fill
    int64_t* cnt = talloc<int64_t>(2 * (m + 1));
    int64_t* fill = cnt + (m + 1);
    fill_u32(reinterpret_cast<uint32_t*>(cnt), 0u, 4 * (m + 1), s);
    d->occ_off = dalloc<int64_t>(m + 1);
    d->occ_slot = dalloc<int64_t>(std::max<int64_t>(d->nmem, 1));
    const unsigned eb = (unsigned)ceil_div(std::max<int64_t>(d->nmem, 1), 256);
    hipLaunchKernelGGL(k_occ_count, dim3(eb), dim3(256), 0, s, d->mem, d->nmem,
                       reinterpret_cast<unsigned long long*>(cnt));
    RBF_HIP(hipGetLastError());
    scan_exclusive_i64(cnt, d->occ_off, m + 1, s);
    hipLaunchKernelGGL(k_occ_fill, dim3(eb), dim3(256), 0, s, d->mem, d->nmem, d->occ_off,
                       reinterpret_cast<unsigned long long*>(fill), d->occ_slot);
    hipLaunchKernelGGL(k_occ_sort, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, s, d->occ_off, m, d->occ_slot);
    RBF_HIP(hipGetLastError());
    temp_free(cnt);
    d->Y = dalloc<double>(std::max<int64_t>(d->nmem, 1));
  }
  d->z = dalloc<double>(c.mpad);
  d->t = dalloc<double>(c.mpad);
  d->z32 = dalloc<float>(c.mpad);
  fill_f64(d->z, 0.0, c.mpad, s);
  fill_f64(d->t, 0.0, c.mpad, s);
  fill_u32(reinterpret_cast<uint32_t*>(d->z32), 0u, c.mpad, s);

  // 6. local inverses
  if (nsub > 0) {
    int32_t* d_order = upload(order, s);
    double* d_shift = talloc<double>(nsub);
    int32_t* d_retries = talloc<int32_t>(nsub);
    int* d_flags = talloc<int>(2);   // [0] queue, [1] failed
    fill_u32(reinterpret_cast<uint32_t*>(d_flags), 0u, 2, s);
    int cus = 0;
    RBF_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c.device));
    cus = std::max(cus, 1);
    const unsigned grid = (unsigned)std::min<int64_t>(nsub, cus);
    // the blocks are swept in global memory: one work space (the block, and
    // the P and Q of a panel) per workgroup
    int64_t maxn = 0;
    for (int64_t i = 0; i < nsub; ++i) maxn = std::max(maxn, d->h_mem_off[i + 1] - d->h_mem_off[i]);
    const int64_t big_stride = maxn * maxn + 2 * kPanel * maxn;
    double* big = talloc<double>(big_stride * grid);
    FacArgs fa{c.xs, d->mem_off, d->mem, d_order, nsub, d->woff, 2.0 * c.sigma * c.sigma, shift, 8,
               d->W, d->W16, d_shift, d_retries, d_flags + 1, d_flags, big, maxn, big_stride};
    hipEvent_t e0, e1;
    RBF_HIP(hipEventCreate(&e0));
    RBF_HIP(hipEventCreate(&e1));
    RBF_HIP(hipEventRecord(e0, s));
    hipLaunchKernelGGL(k_schwarz_factor, dim3(grid), dim3(kFacThreads), 0, s, fa);
    RBF_HIP(hipGetLastError());
    RBF_HIP(hipEventRecord(e1, s));
    std::vector<double> hs = download(d_shift, nsub, s);
    std::vector<int32_t> hr = download(d_retries, nsub, s);
    std::vector<int> hf = download(d_flags, 2, s);
    RBF_HIP(hipStreamSynchronize(s));
    float fms = 0.f;
    RBF_HIP(hipEventElapsedTime(&fms, e0, e1));
    RBF_HIP(hipEventDestroy(e0));
    RBF_HIP(hipEventDestroy(e1));
    d->factor_ms = fms;
    for (void* p : {(void*)d_order, (void*)d_shift, (void*)d_retries, (void*)d_flags}) temp_free(p);
    temp_free(big);
    d->max_shift = 0.0;
    d->retries = 0;
    for (int64_t i = 0; i < nsub; ++i) {
      d->max_shift = std::max(d->max_shift, hs[i]);
      d->retries += hr[i];
    }
    if (hf[1]) {
      free_schwarz(d);
      throw Error{RBF_EBREAKDOWN, "a subdomain block stayed indefinite after the shift retries"};
    }
    // 7. the apply's launch shape
    if (tune) {
      tune_apply(*d, cus, s);
    } else {
      // the covering workgroup size, one workgroup per task
      const int T = covering_threads(*d);
      std::vector<int2> ht = apply_tasks(*d, T);
      d->tasks = upload(ht, s);
      d->ntask = (int64_t)ht.size();
      d->apply_threads = T;
      d->apply_blocks = (int)std::max<int64_t>(d->ntask, 1);
      RBF_HIP(hipStreamSynchronize(s));
    }
  }
  return d;
}

// z = M^{-1} r (sorted order; z must not alias r; entries >= m untouched).
void schwarz_apply(const Ctx& c, const SchwarzData& d, const double* r, double* z, hipStream_t s, const int* skip) {
  if (d.nsub == 0) return;
  launch_local(d, d.apply_threads, d.apply_blocks, d.tasks, d.ntask, r, d.restricted ? (void*)z : (void*)d.Y, s, skip);
  if (!d.restricted) {
    hipLaunchKernelGGL(k_schwarz_sum<double>, dim3((unsigned)ceil_div(c.m, 256)), dim3(256), 0, s, d.occ_off,
                       d.occ_slot, d.Y, c.m, z, skip);
    RBF_HIP(hipGetLastError());
  }
}

// The same from a float32 vector to a float32 result: the float64 products
// and sums of schwarz_apply, the input widened and the result rounded once
// (what the float32 operator does to a float64 input).
void schwarz_apply_f32(const Ctx& c, const SchwarzData& d, const float* r, float* z, hipStream_t s,
                       const int* skip) {
  if (d.nsub == 0) return;
  launch_local(d, d.apply_threads, d.apply_blocks, d.tasks, d.ntask, r, d.restricted ? (void*)z : (void*)d.Y, s, skip,
               true);
  if (!d.restricted) {
    hipLaunchKernelGGL(k_schwarz_sum<float>, dim3((unsigned)ceil_div(c.m, 256)), dim3(256), 0, s, d.occ_off,
                       d.occ_slot, d.Y, c.m, z, skip);
    RBF_HIP(hipGetLastError());
  }
}

}  // namespace rbf
