// Setup kernels: input checks, the extended centre set, Hilbert ordering
// (wave-ballot LSD radix sort), coarse cells and per-group source lists.
#include "cells.h"

namespace rbf {

namespace {

constexpr int kThreads = 256;

int grid_for(int64_t n, int threads = kThreads) {
  int64_t b = ceil_div(n, threads);
  if (b < 1) b = 1;
  if (b > (int64_t)1 << 30) b = (int64_t)1 << 30;
  return (int)b;
}

// ---------------------------------------------------------------------------
// Input checks: flags[0] = a non-finite coordinate, flags[1] = a normal
// shorter than 1e-12.
// ---------------------------------------------------------------------------
__global__ void k_check_inputs(const double* __restrict__ p, const double* __restrict__ nrm, int64_t n,
                               int* __restrict__ flags) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double x = p[3 * i], y = p[3 * i + 1], z = p[3 * i + 2];
  double a = nrm[3 * i], b = nrm[3 * i + 1], c = nrm[3 * i + 2];
  bool fin = isfinite(x) && isfinite(y) && isfinite(z) && isfinite(a) && isfinite(b) && isfinite(c);
  if (!fin) {
    flags[0] = 1;
    return;
  }
  double s = (a * a + b * b) + c * c;
  if (!(sqrt(s) >= 1e-12)) flags[1] = 1;
}

// ---------------------------------------------------------------------------
// Extended set (Sec. II.A.1): centre i = x_i, N+i = x_i + eps n_i,
// 2N+i = x_i - eps n_i with n_i normalised.  Paper order, m x 3 rows.
// ---------------------------------------------------------------------------
__global__ void k_build_centres(const double* __restrict__ p, const double* __restrict__ nrm, int64_t n,
                                double eps, double* __restrict__ X) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double x = p[3 * i], y = p[3 * i + 1], z = p[3 * i + 2];
  double a = nrm[3 * i], b = nrm[3 * i + 1], c = nrm[3 * i + 2];
  double len = sqrt((a * a + b * b) + c * c);
  double nx = a / len, ny = b / len, nz = c / len;
  double ox = eps * nx, oy = eps * ny, oz = eps * nz;
  X[3 * i] = x;
  X[3 * i + 1] = y;
  X[3 * i + 2] = z;
  X[3 * (n + i)] = x + ox;
  X[3 * (n + i) + 1] = y + oy;
  X[3 * (n + i) + 2] = z + oz;
  X[3 * (2 * n + i)] = x - ox;
  X[3 * (2 * n + i) + 1] = y - oy;
  X[3 * (2 * n + i) + 2] = z - oz;
}

// ---------------------------------------------------------------------------
// Bounding box: per-block min/max, then one block folds the partials.
// ---------------------------------------------------------------------------
__global__ void k_bbox_partial(const double* __restrict__ X, int64_t m, double* __restrict__ part) {
  __shared__ double s[6][kThreads];
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    for (int d = 0; d < 3; ++d) {
      double v = X[3 * i + d];
      lo[d] = fmin(lo[d], v);
      hi[d] = fmax(hi[d], v);
    }
  }
  for (int d = 0; d < 3; ++d) {
    s[d][threadIdx.x] = lo[d];
    s[3 + d][threadIdx.x] = hi[d];
  }
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int d = 0; d < 3; ++d) {
        s[d][threadIdx.x] = fmin(s[d][threadIdx.x], s[d][threadIdx.x + w]);
        s[3 + d][threadIdx.x] = fmax(s[3 + d][threadIdx.x], s[3 + d][threadIdx.x + w]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = s[threadIdx.x][0];
}

__global__ __launch_bounds__(kThreads) void k_bbox_final(const double* __restrict__ part, int nb,
                                                          double* __restrict__ box) {
  __shared__ double s[6][kThreads];
  double r[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  for (int b = threadIdx.x; b < nb; b += kThreads)
    for (int d = 0; d < 3; ++d) {
      r[d] = fmin(r[d], part[b * 6 + d]);
      r[3 + d] = fmax(r[3 + d], part[b * 6 + 3 + d]);
    }
  for (int d = 0; d < 6; ++d) s[d][threadIdx.x] = r[d];
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int d = 0; d < 3; ++d) {
        s[d][threadIdx.x] = fmin(s[d][threadIdx.x], s[d][threadIdx.x + w]);
        s[3 + d][threadIdx.x] = fmax(s[3 + d][threadIdx.x], s[3 + d][threadIdx.x + w]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) box[threadIdx.x] = s[threadIdx.x][0];
}

// ---------------------------------------------------------------------------
// Space-filling-curve keys on the fine lattice (10 bits per axis).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t fine_coord(double x, double o, double f, int dim) {
  double q = floor((x - o) / f);
  if (!(q >= 0.0)) q = 0.0;
  if (q > (double)(dim - 1)) q = (double)(dim - 1);
  return (uint32_t)q;
}

// Hilbert index of a fine cell (Skilling's transpose algorithm: undo the
// per-level rotations and reflections, Gray-decode, then interleave the bits
// with the most significant level first).  Like Morton order it keeps every
// aligned block of 2^s fine cells contiguous, with fewer long jumps.
__device__ __forceinline__ uint32_t hilbert3(uint32_t x, uint32_t y, uint32_t z) {
  uint32_t X[3] = {x, y, z};
  const uint32_t M = 1u << (kCurveBits - 1);
  for (uint32_t Q = M; Q > 1; Q >>= 1) {
    const uint32_t P = Q - 1;
    for (int i = 0; i < 3; ++i) {
      if (X[i] & Q) {
        X[0] ^= P;
      } else {
        const uint32_t t = (X[0] ^ X[i]) & P;
        X[0] ^= t;
        X[i] ^= t;
      }
    }
  }
  X[1] ^= X[0];
  X[2] ^= X[1];
  uint32_t t = 0;
  for (uint32_t Q = M; Q > 1; Q >>= 1)
    if (X[2] & Q) t ^= Q - 1;
  X[0] ^= t;
  X[1] ^= t;
  X[2] ^= t;
  uint32_t key = 0;
  for (int b = kCurveBits - 1; b >= 0; --b)
    for (int i = 0; i < 3; ++i) key = (key << 1) | ((X[i] >> b) & 1u);
  return key;
}

__global__ void k_curve_keys(const double* __restrict__ X, int64_t m, Lattice lat, uint32_t* __restrict__ keys,
                             uint32_t* __restrict__ idx) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= m) return;
  uint32_t cx = fine_coord(X[3 * i], lat.origin[0], lat.fine, lat.fdims[0]);
  uint32_t cy = fine_coord(X[3 * i + 1], lat.origin[1], lat.fine, lat.fdims[1]);
  uint32_t cz = fine_coord(X[3 * i + 2], lat.origin[2], lat.fine, lat.fdims[2]);
  keys[i] = hilbert3(cx, cy, cz);
  idx[i] = (uint32_t)i;
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort of (key, value) pairs, 8-bit digits.
//   hist:    per-block digit counts, stored digit-major [256][nb].
//   scan:    exclusive prefix over that array = global start of every
//            (digit, block) bucket.
//   scatter: every wave ranks its lanes among equal digits with eight
//            ballots (the peers of a lane share all eight digit bits) and
//            mbcnt; waves of a block are offset by a per-digit prefix in LDS,
//            blocks by the scanned histogram, so the order of equal keys is
//            the input order.
// ---------------------------------------------------------------------------
constexpr int kRsItems = 16;
constexpr int kRsTile = kThreads * kRsItems;

__global__ void k_rs_hist(const uint32_t* __restrict__ keys, int64_t m, int shift, int64_t* __restrict__ hist,
                          int nb) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * kRsTile;
  for (int r = 0; r < kRsItems; ++r) {
    int64_t i = base + r * kThreads + threadIdx.x;
    if (i < m) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

__global__ void k_rs_scatter(const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                             uint32_t* __restrict__ kout, uint32_t* __restrict__ vout, int64_t m, int shift,
                             const int64_t* __restrict__ offs, int nb) {
  __shared__ int64_t base[256];
  __shared__ uint32_t tot[256];
  __shared__ uint32_t wcnt[4][256];
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  base[t] = offs[(int64_t)t * nb + blockIdx.x];
  const int64_t tile = (int64_t)blockIdx.x * kRsTile;
  for (int r = 0; r < kRsItems; ++r) {
    for (int d = lane; d < 256; d += 64) wcnt[wave][d] = 0;
    __syncthreads();
    int64_t i = tile + r * kThreads + t;
    bool valid = i < m;
    uint32_t key = valid ? kin[i] : 0u, val = valid ? vin[i] : 0u;
    uint32_t dig = (key >> shift) & 255u;
    uint64_t peers = ballot(valid);
    for (int b = 0; b < 8; ++b) {
      bool bit = (dig >> b) & 1u;
      uint64_t s = ballot(bit);
      peers &= bit ? s : ~s;
    }
    uint32_t rank = lanes_below(peers);
    if (valid && rank == 0) wcnt[wave][dig] = (uint32_t)__popcll(peers);
    __syncthreads();
    {
      uint32_t c0 = wcnt[0][t], c1 = wcnt[1][t], c2 = wcnt[2][t], c3 = wcnt[3][t];
      wcnt[0][t] = 0;
      wcnt[1][t] = c0;
      wcnt[2][t] = c0 + c1;
      wcnt[3][t] = c0 + c1 + c2;
      tot[t] = c0 + c1 + c2 + c3;
    }
    __syncthreads();
    if (valid) {
      int64_t pos = base[dig] + wcnt[wave][dig] + rank;
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    base[t] += tot[t];
  }
}

// ---------------------------------------------------------------------------
// Exclusive prefix sum of int64 values (three phases, recursive on the
// block sums).
// ---------------------------------------------------------------------------
constexpr int kScanItems = 8;
constexpr int kScanTile = kThreads * kScanItems;

__device__ int64_t block_exclusive_scan(int64_t v, int64_t* total) {
  __shared__ int64_t s[kThreads];
  const int t = threadIdx.x;
  s[t] = v;
  __syncthreads();
  for (int off = 1; off < kThreads; off <<= 1) {
    int64_t add = t >= off ? s[t - off] : 0;
    __syncthreads();
    s[t] += add;
    __syncthreads();
  }
  int64_t incl = s[t];
  *total = s[kThreads - 1];
  __syncthreads();
  return incl - v;
}

__global__ void k_scan_tiles(const int64_t* __restrict__ in, int64_t* __restrict__ out, int64_t n,
                             int64_t* __restrict__ sums) {
  int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int64_t loc[kScanItems];
  int64_t run = 0;
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + k;
    int64_t v = i < n ? in[i] : 0;
    loc[k] = run;
    run += v;
  }
  int64_t total;
  int64_t pre = block_exclusive_scan(run, &total);
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + k;
    if (i < n) out[i] = pre + loc[k];
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ void k_scan_add(int64_t* __restrict__ out, int64_t n, const int64_t* __restrict__ sums_scanned) {
  int64_t base = (int64_t)blockIdx.x * kScanTile;
  int64_t add = sums_scanned[blockIdx.x];
  for (int k = threadIdx.x; k < kScanTile; k += kThreads) {
    int64_t i = base + k;
    if (i < n) out[i] += add;
  }
}

// ---------------------------------------------------------------------------
// Sorted copies of the centres, with the far padding source at index m.
// ---------------------------------------------------------------------------
__global__ void k_gather_sorted(const double* __restrict__ X, const uint32_t* __restrict__ perm, int64_t m,
                                double sk, double4* __restrict__ xs, double4* __restrict__ xk) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k > m) return;
  double x, y, z;
  if (k < m) {
    int64_t i = perm[k];
    x = X[3 * i];
    y = X[3 * i + 1];
    z = X[3 * i + 2];
  } else {
    x = y = z = kFar;
  }
  xs[k] = make_double4(x, y, z, 0.0);
  xk[k] = make_double4(x * sk, y * sk, z * sk, 0.0);
}

// Coarse cells of the sorted centres.
__global__ void k_cell_flags(const uint32_t* __restrict__ keys, int64_t m, int cshift, int64_t* __restrict__ flag) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= m) return;
  flag[k] = (k == 0 || (keys[k] >> cshift) != (keys[k - 1] >> cshift)) ? 1 : 0;
}

__global__ void k_cell_fill(const double4* __restrict__ xs, int64_t m, const int64_t* __restrict__ flag,
                            const int64_t* __restrict__ cid, Lattice lat, int32_t* __restrict__ start,
                            int32_t* __restrict__ count, int32_t* __restrict__ map, int32_t* __restrict__ xyz) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= m) return;
  if (!flag[k]) return;
  int64_t c = cid[k];
  // the run ends where the next run starts (or at m)
  int64_t e = k + 1;
  while (e < m && !flag[e]) ++e;
  start[c] = (int32_t)k;
  count[c] = (int32_t)(e - k);
  const double4 p = xs[k];
  const uint32_t cx = fine_coord(p.x, lat.origin[0], lat.fine, lat.fdims[0]) >> lat.shift;
  const uint32_t cy = fine_coord(p.y, lat.origin[1], lat.fine, lat.fdims[1]) >> lat.shift;
  const uint32_t cz = fine_coord(p.z, lat.origin[2], lat.fine, lat.fdims[2]) >> lat.shift;
  int64_t lin = (int64_t)cx + (int64_t)lat.cdims[0] * ((int64_t)cy + (int64_t)lat.cdims[1] * cz);
  map[lin] = (int32_t)c;
  xyz[c] = (int32_t)(cx | (cy << 10) | (cz << 20));
}

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_f64(double* p, double v, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_f32(float* p, float v, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// Source lists.  One wave per group of 16 targets, anchor a (centre of their
// bounding box) and radius R (largest distance of a target from a).  Every
// source s of a coarse cell near the group is classified against the exact
// float64 truncation test r^2 <= r_c^2 of every valid target:
//   inside for all targets  -> "inner" (the pair kernels apply no test)
//   inside for some targets -> "outer", with the mask of those targets
//   inside for none         -> dropped.
// By the triangle inequality |s - a| + R <= r_c (1 - 1e-12) makes s inner
// and |s - a| - R > r_c (1 + 1e-12) drops it, without looking at the
// targets (the relative margin covers the float64 rounding of the distances
// and of the exact test), whole cells at a time when the cell box allows.
// The cells near the anchor are examined one per lane (with their source
// ranges); the sources of the cells that remain are then classified 64 at a
// time, one per lane, across cell boundaries (a lane finds its cell from
// ballots over the cells' starts, cells.h); the remaining "shell"
// sources are queued in LDS and tested exactly against the 16 targets, 64
// at a time (targets in scalar registers).
// Pass 1 counts, pass 2 writes; both enumerate in the same order, so the
// list order is deterministic.  Lists are padded to whole chunks with the
// padding source m (mask 0).  Pass 2 also writes the masks of every entry
// of the chunks from the first one that is not purely inner.
// ---------------------------------------------------------------------------
struct ListCounts {
  int64_t n_in, n_out, use;
};

// Where the classifying pass writes a group's entries: its staging region
// [base, base + bound) holds the inner entries from the bottom up and the
// outer entries, with their target masks, from the top down (both come from
// the group's candidate sources, so they never meet).
struct ListOut {
  uint32_t* list;
  uint16_t* mask;
  int64_t base;
  int64_t top;      // base + bound - 1
  int64_t bound;
};

// (The two passes enumerate the same candidates, so e < bound always; the
// tests keep a broken invariant from writing outside the region, and the
// pass reports it.)
__device__ __forceinline__ void put_inner(const ListOut& o, int64_t e, uint32_t k) {
  if (e < o.bound) o.list[o.base + e] = k;
}
__device__ __forceinline__ void put_outer(const ListOut& o, int64_t e, uint32_t k, uint32_t bits) {
  if (e < o.bound) {
    o.list[o.top - e] = k;
    o.mask[o.top - e] = (uint16_t)bits;
  }
}

// Exact test of `cnt` (<= 64) queued shell sources, one per lane, against
// the group's 16 targets (uniform loads: scalar registers).  For a brick of
// grid nodes (lattice), node l = (l & 3, (l >> 2) & 1, l >> 3) shares its x
// with nodes l & 3, its y with node 4 ((l >> 2) & 1) and its z with node
// 8 (l >> 3): the eight squared axis differences give all sixteen
// r^2 = (dx dx + dy dy) + dz dz, bit for bit the same sums.
template <bool WRITE, bool LATTICE>
__device__ __forceinline__ void process_shell(const uint32_t* q, int cnt, const double4* __restrict__ tg,
                                              const double4* __restrict__ xs, uint32_t vmask, double rc2,
                                              const ListOut& o, ListCounts& n) {
  const int lane = threadIdx.x & 63;
  const bool valid = lane < cnt;
  const uint32_t k = valid ? q[lane] : 0u;
  uint32_t bits = 0;
  if (valid) {
    const double4 s = xs[k];
    if constexpr (LATTICE) {
      double dx2[4], dy2[2], dz2[2];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const double dx = tg[i].x - s.x;
        dx2[i] = dx * dx;
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const double dy = tg[4 * j].y - s.y, dz = tg[8 * j].z - s.z;
        dy2[j] = dy * dy;
        dz2[j] = dz * dz;
      }
#pragma unroll
      for (int l = 0; l < kGroup; ++l) {
        const double r2 = (dx2[l & 3] + dy2[(l >> 2) & 1]) + dz2[l >> 3];
        bits |= r2 <= rc2 ? (1u << l) : 0u;
      }
      bits &= vmask;
    } else {
#pragma unroll
      for (int l = 0; l < kGroup; ++l) {
        const double4 t = tg[l];
        const double dx = t.x - s.x, dy = t.y - s.y, dz = t.z - s.z;
        const double r2 = (dx * dx + dy * dy) + dz * dz;
        bits |= (t.w != 0.0 && r2 <= rc2) ? (1u << l) : 0u;
      }
    }
  }
  const bool is_in = valid && bits == vmask;
  const bool is_out = valid && bits != 0u && !is_in;
  const uint64_t mi = ballot(is_in), mo = ballot(is_out);
  if (WRITE) {
    if (is_in) put_inner(o, n.n_in + lanes_below(mi), k);
    if (is_out) put_outer(o, n.n_out + lanes_below(mo), k, bits);
  }
  n.n_in += __popcll(mi);
  n.n_out += __popcll(mo);
  int64_t u = __popc(bits);
  for (int off = 32; off > 0; off >>= 1) u += __shfl_xor(u, off);
  n.use += u;
}

// A group's valid targets (mask), the centre of their bounding box (the
// anchor) and their largest distance from it.
struct Frame {
  int nvalid;
  uint32_t vmask;
  double ax, ay, az, rad;
};
__device__ __forceinline__ Frame group_frame(const double4* __restrict__ tg) {
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  Frame f{0, 0u, 0.0, 0.0, 0.0, 0.0};
  for (int l = 0; l < kGroup; ++l) {
    const double4 t = tg[l];
    if (t.w != 0.0) {
      ++f.nvalid;
      f.vmask |= 1u << l;
      lo[0] = fmin(lo[0], t.x); hi[0] = fmax(hi[0], t.x);
      lo[1] = fmin(lo[1], t.y); hi[1] = fmax(hi[1], t.y);
      lo[2] = fmin(lo[2], t.z); hi[2] = fmax(hi[2], t.z);
    }
  }
  if (f.nvalid == 0) return f;
  f.ax = 0.5 * (lo[0] + hi[0]);
  f.ay = 0.5 * (lo[1] + hi[1]);
  f.az = 0.5 * (lo[2] + hi[2]);
  for (int l = 0; l < kGroup; ++l) {
    const double4 t = tg[l];
    if (t.w != 0.0) {
      const double dx = t.x - f.ax, dy = t.y - f.ay, dz = t.z - f.az;
      f.rad = fmax(f.rad, sqrt((dx * dx + dy * dy) + dz * dz));
    }
  }
  return f;
}

// Summed counts of the coarse cells: sat[(z * (ny + 1) + y) * (nx + 1) + x]
// = the sources in the cells [0, x) x [0, y) x [0, z).
__global__ void k_sat_counts(const int32_t* __restrict__ cmap, const int32_t* __restrict__ ccount, Lattice lat,
                             int64_t* __restrict__ sat) {
  const int64_t nx = lat.cdims[0] + 1, ny = lat.cdims[1] + 1, nz = lat.cdims[2] + 1;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nx * ny * nz) return;
  const int64_t x = i % nx, y = (i / nx) % ny, z = i / (nx * ny);
  int64_t v = 0;
  if (x > 0 && y > 0 && z > 0) {
    const int32_t cid = cmap[(x - 1) + (int64_t)lat.cdims[0] * ((y - 1) + (int64_t)lat.cdims[1] * (z - 1))];
    v = cid >= 0 ? ccount[cid] : 0;
  }
  sat[i] = v;
}
// Prefix sums along one axis (0, 1, 2): one thread per line.
__global__ void k_sat_scan(Lattice lat, int axis, int64_t* __restrict__ sat) {
  const int64_t n[3] = {lat.cdims[0] + 1, lat.cdims[1] + 1, lat.cdims[2] + 1};
  const int64_t stride[3] = {1, n[0], n[0] * n[1]};
  const int a1 = axis == 0 ? 1 : 0, a2 = axis == 2 ? 1 : 2;
  const int64_t line = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (line >= n[a1] * n[a2]) return;
  const int64_t base = (line % n[a1]) * stride[a1] + (line / n[a1]) * stride[a2];
  const int64_t st = stride[axis], len = n[axis];
  int64_t acc = 0;
  // eight entries at a time: their loads are in flight together
  int64_t q = 0;
  for (; q + 8 <= len; q += 8) {
    int64_t v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = sat[base + (q + u) * st];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      acc += v[u];
      sat[base + (q + u) * st] = acc;
    }
  }
  for (; q < len; ++q) {
    acc += sat[base + q * st];
    sat[base + q * st] = acc;
  }
}

// Candidate bound of every group from the summed counts: the sources of its
// whole cell cube (one thread per group).
__global__ void k_list_bound_sat(const double4* __restrict__ tpts, int64_t G, const int64_t* __restrict__ sat, Lattice lat,
                                 double rc, int64_t* __restrict__ bound) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= G) return;
  const Frame f = group_frame(tpts + g * kGroup);
  if (f.nvalid == 0) {
    bound[g] = 0;
    return;
  }
  const double r_out = rc * (1.0 + 1e-12) + f.rad;
  const double ac[3] = {f.ax, f.ay, f.az};
  int cl[3], cn[3];
  cell_cube(ac, r_out, lat, cl, cn);
  const int64_t nx = lat.cdims[0] + 1, ny = lat.cdims[1] + 1;
  auto S = [&](int64_t x, int64_t y, int64_t z) { return sat[(z * ny + y) * nx + x]; };
  const int64_t x0 = cl[0], y0 = cl[1], z0 = cl[2], x1 = cl[0] + cn[0], y1 = cl[1] + cn[1], z1 = cl[2] + cn[2];
  bound[g] = S(x1, y1, z1) - S(x0, y1, z1) - S(x1, y0, z1) - S(x1, y1, z0) + S(x0, y0, z1) + S(x0, y1, z0) +
             S(x1, y0, z0) - S(x0, y0, z0);
}

// MODE kBound: the cell phase only; bound[g] = the number of candidate
// sources (those of the cells within r_out of the anchor), an upper bound of
// the group's list.  MODE kStage: the classification, into the staging
// region at soff[g] of size bound[g]; counts, useful pairs, the valid-target
// mask and the group record (offset set later by k_list_compact).
constexpr int kBound = 0, kStage = 1;
// The centres' classification fits 64 VGPRs, eight waves per SIMD for the
// walk's latency; the lattice form (grid nodes) keeps its registers.
template <int MODE, bool LATTICE>
__global__ __launch_bounds__(kThreads, LATTICE ? 1 : 8) void k_lists(const double4* __restrict__ tpts, int64_t G, GroupInfo* __restrict__ groups,
                                                    const double4* __restrict__ xs,
                                                    const int32_t* __restrict__ cstart, const int32_t* __restrict__ ccount,
                                                    const int32_t* __restrict__ cmap, Lattice lat, double rc, double rc2,
                                                    int64_t* __restrict__ bound, const int64_t* __restrict__ soff,
                                                    int32_t* __restrict__ cnt_in, int32_t* __restrict__ cnt_out,
                                                    int64_t* __restrict__ useful, uint32_t* __restrict__ vmasks,
                                                    uint32_t* __restrict__ slist, uint16_t* __restrict__ smask,
                                                    int* __restrict__ overflow) {
  constexpr bool WRITE = MODE == kStage;
  __shared__ uint32_t qbuf[kThreads / kWave][2 * kWave];
  __shared__ int32_t cpre_s[kThreads / kWave][kWave], cst_s[kThreads / kWave][kWave];
  __shared__ uint8_t cwhole_s[kThreads / kWave][kWave];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  // neighbouring groups (which share candidate sources) on one XCD's L2
  const int64_t g = xcd_remap(blockIdx.x, gridDim.x) * 4 + wave;
  if (g >= G) return;
  uint32_t* q = qbuf[wave];
  const double4* tg = tpts + g * kGroup;
  // the group's valid targets, anchor and radius (uniform)
  const Frame fr = group_frame(tg);
  const int nvalid = fr.nvalid;
  const uint32_t vmask = fr.vmask;
  ListOut o{slist, smask, 0, 0, 0};
  if (WRITE) {
    o.base = soff[g];
    o.bound = bound[g];
    o.top = o.base + o.bound - 1;
  }
  if (nvalid == 0) {
    if (lane == 0) {
      if (MODE == kBound) {
        bound[g] = 0;
      } else {
        cnt_in[g] = 0;
        cnt_out[g] = 0;
        useful[g] = 0;
        vmasks[g] = 0;
        GroupInfo gi;
        gi.off = 0; gi.n_chunks = 0; gi.n_inner = 0;
        gi.ax = gi.ay = gi.az = 0.0;
        gi.radius = 0.0;
        groups[g] = gi;
      }
    }
    return;
  }
  const double ax = fr.ax, ay = fr.ay, az = fr.az, rad = fr.rad;
  const double r_in = rc * (1.0 - 1e-12) - rad;   // |s - a| <= r_in: inside for every target
  const double r_out = rc * (1.0 + 1e-12) + rad;  // |s - a| >  r_out: inside for none
  const double r_in2 = r_in > 0.0 ? r_in * r_in : -1.0;
  const double r_out2 = r_out * r_out;

  // candidate cube of coarse cells around the anchor
  int cl[3], cn[3];
  const double ac[3] = {ax, ay, az};
  cell_cube(ac, r_out, lat, cl, cn);
  ListCounts n{0, 0, 0};
  int qn = 0;
  const int64_t cand = walk_candidates<MODE == kBound>(
      ac, r_in2, r_out2, cl, cn, xs, cstart, ccount, cmap, lat, cpre_s[wave], cst_s[wave], cwhole_s[wave],
      [&](bool, uint32_t k, bool is_in, bool is_shell, bool, const double4&) {
        const uint64_t mi = ballot(is_in), ms = ballot(is_shell);
        if (WRITE && is_in) put_inner(o, n.n_in + lanes_below(mi), k);
        n.n_in += __popcll(mi);
        n.use += (int64_t)__popcll(mi) * nvalid;
        if (is_shell) q[qn + lanes_below(ms)] = k;
        qn += __popcll(ms);
        if (qn >= kWave) {
          wave_sync_lds();
          process_shell<WRITE, LATTICE>(q, kWave, tg, xs, vmask, rc2, o, n);
          const uint32_t rest = lane + kWave < qn ? q[kWave + lane] : 0u;
          wave_sync_lds();
          if (lane + kWave < qn) q[lane] = rest;
          qn -= kWave;
          wave_sync_lds();
        }
      });
  if (MODE == kBound) {
    if (lane == 0) bound[g] = cand;
    return;
  }
  wave_sync_lds();
  if (qn > 0) process_shell<WRITE, LATTICE>(q, qn, tg, xs, vmask, rc2, o, n);
  if (lane == 0) {
    if (n.n_in + n.n_out > o.bound) {
      atomicOr(overflow, 1);
      n.n_in = n.n_out = 0;
    }
    cnt_in[g] = (int32_t)n.n_in;
    cnt_out[g] = (int32_t)n.n_out;
    useful[g] = n.use;
    vmasks[g] = vmask;
    GroupInfo gi;
    gi.off = 0;
    gi.n_chunks = (int32_t)ceil_div(n.n_in + n.n_out, kChunk);
    gi.n_inner = (int32_t)inner_chunks(n.n_in);
    gi.ax = ax; gi.ay = ay; gi.az = az;
    gi.radius = rad;
    groups[g] = gi;
  }
}

// Final layout of a group's list at off[g] (one wave per group): the inner
// entries in order, then the outer ones (read back from the top of the
// staging region, restoring their order), padded to whole chunks with the
// padding source m; the target masks of every chunk from n_inner on
// (inner entries there: every valid target; padding: none).
__global__ __launch_bounds__(kThreads) void k_list_compact(GroupInfo* __restrict__ groups, int64_t G,
                                                           const int64_t* __restrict__ off,
                                                           const int64_t* __restrict__ soff,
                                                           const int64_t* __restrict__ bound,
                                                           const int32_t* __restrict__ cnt_in,
                                                           const int32_t* __restrict__ cnt_out,
                                                           const uint32_t* __restrict__ vmasks,
                                                           const uint32_t* __restrict__ slist,
                                                           const uint16_t* __restrict__ smask, uint32_t m,
                                                           uint32_t* __restrict__ list, uint16_t* __restrict__ mask) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t g = (int64_t)blockIdx.x * 4 + wave;
  if (g >= G) return;
  const int64_t base = off[g], sb = soff[g], top = soff[g] + bound[g] - 1;
  const int64_t nin = cnt_in[g], nout = cnt_out[g];
  const int64_t len = round_up(nin + nout, kChunk);
  const int64_t in_full = inner_chunks(nin) * kChunk;
  const uint32_t vm = vmasks[g];
  if (lane == 0) groups[g].off = base;
  // four entries per lane per pass, their loads issued together
  constexpr int kU = 4;
  for (int64_t e0 = lane; e0 < len; e0 += kU * kWave) {
    uint32_t k[kU], bits[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t e = e0 + (int64_t)u * kWave;
      k[u] = m;
      bits[u] = 0;
      if (e < nin) {
        k[u] = slist[sb + e];
        bits[u] = vm;
      } else if (e < nin + nout) {
        k[u] = slist[top - (e - nin)];
        bits[u] = smask[top - (e - nin)];
      }
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t e = e0 + (int64_t)u * kWave;
      if (e < len) {
        list[base + e] = k[u];
        if (e >= in_full) mask[mask_slot(base, e)] = (uint16_t)bits[u];
      }
    }
  }
}

// Launch order of an operator set's groups for the pair kernels.  A launch
// of nb workgroups of four groups runs the workgroups of XCD x on a
// contiguous range of slots (xcd_remap), in slot order; within each XCD's
// range the longest eighth of the groups (whole classes of 16 classes of
// chunk count) takes the first slots, so that a launch does not end on a
// long group, and every group keeps its spatial order otherwise
// (neighbouring groups, which share most candidate sources, stay close in
// time).  The order only moves whole groups between slots: every group's
// sums stay the same.  One workgroup per XCD.
constexpr int kOrderClasses = 16;
constexpr int kLongShare = 8;
__global__ __launch_bounds__(kThreads) void k_group_order(const GroupInfo* __restrict__ groups, int64_t G,
                                                          int64_t nb, int32_t* __restrict__ order) {
  __shared__ int32_t cnt[kOrderClasses], base[kOrderClasses], smax[kThreads / kWave];
  __shared__ int32_t wcnt[kThreads / kWave][kOrderClasses];
  __shared__ int32_t s_cut;
  const int x = blockIdx.x, t = threadIdx.x;
  const int64_t q = nb / 8, r = nb % 8;
  const int64_t first = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
  const int64_t count = q + (x < r ? 1 : 0);
  const int64_t g0 = min(G, first * kGroupsPerLaunchBlock), g1 = min(G, (first + count) * kGroupsPerLaunchBlock);
  // the largest chunk count of the range sets the class width
  int32_t m = 0;
  for (int64_t g = g0 + t; g < g1; g += kThreads) m = max(m, groups[g].n_chunks);
  for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o));
  if ((t & 63) == 0) smax[t >> 6] = m;
  if (t < kOrderClasses) cnt[t] = 0;
  __syncthreads();
  m = 0;
  for (int w = 0; w < kThreads / kWave; ++w) m = max(m, smax[w]);
  const int32_t width = m / kOrderClasses + 1;
  auto cls = [&](int64_t g) { return kOrderClasses - 1 - min(kOrderClasses - 1, groups[g].n_chunks / width); };
  for (int64_t g = g0 + t; g < g1; g += kThreads) atomicAdd(&cnt[cls(g)], 1);
  __syncthreads();
  if (t == 0) {
    // the longest classes holding at least 1/kLongShare of the range go
    // first; every other group keeps its place in the spatial order
    const int32_t want = (int32_t)((g1 - g0 + kLongShare - 1) / kLongShare);
    int32_t acc = 0, cut = kOrderClasses - 1;
    for (int k = 0; k < kOrderClasses; ++k) {
      acc += cnt[k];
      if (acc >= want) {
        cut = k;
        break;
      }
    }
    s_cut = cut;
    base[0] = 0;
    base[1] = acc;
  }
  __syncthreads();
  // a stable split, a tile of kThreads groups at a time: a group's slot is
  // its class's base, plus the groups of its class in the earlier waves of
  // the tile, plus those in its own wave below it
  const int wave = t >> 6, lane = t & 63;
  const int cut = s_cut;
  for (int64_t t0 = g0; t0 < g1; t0 += kThreads) {
    const int64_t g = t0 + t;
    const int c = g < g1 ? (cls(g) <= cut ? 0 : 1) : -1;
    int rank = 0;
    for (int k = 0; k < 2; ++k) {
      const uint64_t b = ballot(c == k);
      if (c == k) rank = (int)lanes_below(b);
      if (lane == 0) wcnt[wave][k] = __popcll(b);
    }
    __syncthreads();
    if (c >= 0) {
      int32_t at = base[c] + rank;
      for (int w = 0; w < wave; ++w) at += wcnt[w][c];
      order[g0 + at] = (int32_t)g;
    }
    __syncthreads();
    if (t < 2)
      for (int w = 0; w < kThreads / kWave; ++w) base[t] += wcnt[w][t];
    __syncthreads();
  }
}

__global__ void k_list_lengths(const GroupInfo* __restrict__ groups, int64_t G, int64_t* __restrict__ len) {
  int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g < G) len[g] = (int64_t)groups[g].n_chunks * kChunk;
}
__global__ void k_inner_lengths(const GroupInfo* __restrict__ groups, int64_t G, int64_t* __restrict__ len) {
  int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g < G) len[g] = (int64_t)groups[g].n_inner * kChunk;
}
// Dense sets: every group sees all m centres (padded to whole chunks).
__global__ void k_dense_groups(const double4* __restrict__ tpts, int64_t G, int64_t m, GroupInfo* __restrict__ groups) {
  int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= G) return;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  int nv = 0;
  for (int l = 0; l < kGroup; ++l) {
    double4 t = tpts[g * kGroup + l];
    if (t.w != 0.0) {
      ++nv;
      lo[0] = fmin(lo[0], t.x); hi[0] = fmax(hi[0], t.x);
      lo[1] = fmin(lo[1], t.y); hi[1] = fmax(hi[1], t.y);
      lo[2] = fmin(lo[2], t.z); hi[2] = fmax(hi[2], t.z);
    }
  }
  GroupInfo gi;
  gi.off = 0;
  gi.n_chunks = nv ? (int32_t)ceil_div(m, kChunk) : 0;
  gi.n_inner = gi.n_chunks;
  if (nv) {
    gi.ax = 0.5 * (lo[0] + hi[0]); gi.ay = 0.5 * (lo[1] + hi[1]); gi.az = 0.5 * (lo[2] + hi[2]);
    double rad = 0.0;
    for (int l = 0; l < kGroup; ++l) {
      double4 t = tpts[g * kGroup + l];
      if (t.w != 0.0) {
        double dx = t.x - gi.ax, dy = t.y - gi.ay, dz = t.z - gi.az;
        rad = fmax(rad, sqrt((dx * dx + dy * dy) + dz * dz));
      }
    }
    gi.radius = rad;
  } else {
    gi.ax = gi.ay = gi.az = 0.0;
    gi.radius = 0.0;
  }
  groups[g] = gi;
}

// Integer sum (out must start at 0): block sums added with atomics, exact and
// independent of the order.
__global__ void k_sum_i64(const int64_t* __restrict__ in, int64_t n, int64_t* __restrict__ out) {
  __shared__ int64_t s[kThreads];
  int64_t acc = 0;
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
    acc += in[i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd((unsigned long long*)out, (unsigned long long)s[0]);
}



// ---------------------------------------------------------------------------
// Grid targets.  The grid is cut into bricks of 4 x 2 x 2 nodes (16 nodes, one
// group); a brick is active when some occupied coarse cell, grown by the
// cutoff, reaches one of its nodes.  Nodes of inactive bricks have no centre
// within the cutoff and keep the zero written beforehand.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool node_range(double lo, double hi, double o, double h, int64_t n, int64_t* a, int64_t* b) {
  if (h == 0.0) {
    if (o < lo || o > hi) return false;
    *a = 0;
    *b = n - 1;
    return true;
  }
  double fa = ceil((lo - o) / h), fb = floor((hi - o) / h);
  fa = fmax(fa, 0.0);
  fb = fmin(fb, (double)(n - 1));
  if (fa > fb) return false;
  *a = (int64_t)fa;
  *b = (int64_t)fb;
  return true;
}

__global__ void k_mark_bricks(const int32_t* __restrict__ xyz, int64_t ncell, Lattice lat, double rc, GridDesc gd,
                              int64_t* __restrict__ mark) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  const int32_t v = xyz[c];
  const int cc[3] = {v & 1023, (v >> 10) & 1023, (v >> 20) & 1023};
  const int bs[3] = {4, 2, 2};
  int64_t blo[3], bhi[3];
  for (int d = 0; d < 3; ++d) {
    const double lo = lat.origin[d] + cc[d] * lat.coarse - rc;
    const double hi = lat.origin[d] + (cc[d] + 1) * lat.coarse + rc;
    int64_t a, b;
    // one node of slack on each side keeps rounding from dropping a node
    if (!node_range(lo - gd.h[d], hi + gd.h[d], gd.o[d], gd.h[d], gd.n[d], &a, &b)) return;
    blo[d] = a / bs[d];
    bhi[d] = b / bs[d];
  }
  for (int64_t bz = blo[2]; bz <= bhi[2]; ++bz)
    for (int64_t by = blo[1]; by <= bhi[1]; ++by)
      for (int64_t bx = blo[0]; bx <= bhi[0]; ++bx) mark[bx + gd.nb[0] * (by + gd.nb[1] * bz)] = 1;
}

__global__ void k_fill_i64(int64_t* p, int64_t v, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_compact(const int64_t* __restrict__ mark, const int64_t* __restrict__ pos, int64_t n,
                          int64_t* __restrict__ ids) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n && mark[i]) ids[pos[i]] = i;
}

__global__ void k_brick_targets(const int64_t* __restrict__ ids, int64_t nact, GridDesc gd, double4* __restrict__ pts,
                                int64_t* __restrict__ oidx) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= nact * kGroup) return;
  const int64_t g = t / kGroup;
  const int l = (int)(t % kGroup);
  const int64_t b = ids ? ids[g] : g;
  const int64_t bx = b % gd.nb[0], by = (b / gd.nb[0]) % gd.nb[1], bz = b / (gd.nb[0] * gd.nb[1]);
  const int64_t i = bx * 4 + (l & 3), j = by * 2 + ((l >> 2) & 1), k = bz * 2 + (l >> 3);
  if (i < gd.n[0] && j < gd.n[1] && k < gd.n[2]) {
    pts[t] = make_double4(gd.o[0] + (double)i * gd.h[0], gd.o[1] + (double)j * gd.h[1], gd.o[2] + (double)k * gd.h[2], 1.0);
    oidx[t] = i + gd.n[0] * (j + gd.n[1] * k);
  } else {
    pts[t] = make_double4(kFar, kFar, kFar, 0.0);
    oidx[t] = 0;
  }
}

__global__ void k_count_valid(const double4* __restrict__ pts, int64_t n, int64_t* __restrict__ out) {
  __shared__ int64_t s[kThreads];
  int64_t acc = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    acc += pts[i].w != 0.0 ? 1 : 0;
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd((unsigned long long*)out, (unsigned long long)s[0]);
}


// ---------------------------------------------------------------------------
// Target groups.  Consecutive targets of the curve order are packed into
// groups of at most 16 whose bounding box has a diagonal of at most E (the
// float32 coordinates of a group are taken relative to its centre, so their
// rounding error scales with E).  The packing is greedy inside segments of
// kGroupSeg targets, one wave per segment (the segment staged in LDS, one
// lane packing), which counts the groups of every segment and records each
// target's slot within its segment; after a scan of the counts a parallel
// pass gives every target its global slot.
// ---------------------------------------------------------------------------
constexpr int kGroupSeg = 256;

__global__ __launch_bounds__(kThreads) void k_group_greedy(const double4* __restrict__ sp, int64_t M, double E2,
                                                           int64_t* __restrict__ gcount,
                                                           int32_t* __restrict__ local_slot) {
  // one wave per segment: the wave stages the segment in LDS, one lane runs
  // the (sequential) greedy packing from there and records every target's
  // slot relative to the segment's first group
  __shared__ double4 seg_s[kThreads / kWave][kGroupSeg];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t s = (int64_t)blockIdx.x * (kThreads / kWave) + wave;
  const int64_t nseg = ceil_div(M, kGroupSeg);
  if (s >= nseg) return;
  const int64_t k0 = s * kGroupSeg, k1 = min(M, k0 + kGroupSeg);
  double4* seg = seg_s[wave];
  for (int64_t i = lane; i < k1 - k0; i += kWave) seg[i] = sp[k0 + i];
  wave_sync_lds();
  if (lane != 0) return;
  int32_t g = 0;
  int64_t k = k0;
  while (k < k1) {
    const double4 p = seg[k - k0];
    double lx = p.x, ly = p.y, lz = p.z, hx = p.x, hy = p.y, hz = p.z;
    local_slot[k] = g * kGroup;
    int64_t j = k + 1;
    for (; j < k1 && j - k < kGroup; ++j) {
      const double4 q = seg[j - k0];
      const double nlx = fmin(lx, q.x), nly = fmin(ly, q.y), nlz = fmin(lz, q.z);
      const double nhx = fmax(hx, q.x), nhy = fmax(hy, q.y), nhz = fmax(hz, q.z);
      const double dx = nhx - nlx, dy = nhy - nly, dz = nhz - nlz;
      if ((dx * dx + dy * dy) + dz * dz > E2) break;
      lx = nlx; ly = nly; lz = nlz; hx = nhx; hy = nhy; hz = nhz;
      local_slot[j] = g * kGroup + (int32_t)(j - k);
    }
    k = j;
    ++g;
  }
  gcount[s] = g;
}

// slot of every target: its segment's first group (scanned counts) plus its
// slot within the segment
__global__ void k_group_slots(const int32_t* __restrict__ local_slot, const int64_t* __restrict__ goff, int64_t M,
                              int64_t* __restrict__ slot_of) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < M) slot_of[k] = goff[k / kGroupSeg] * kGroup + local_slot[k];
}

__global__ void k_pad_targets(double4* __restrict__ pts, int64_t* __restrict__ oidx, int64_t total) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= total) return;
  pts[t] = make_double4(kFar, kFar, kFar, 0.0);
  oidx[t] = 0;
}

__global__ void k_place_targets(const double4* __restrict__ sp, const uint32_t* __restrict__ orig, int64_t M,
                                const int64_t* __restrict__ slot_of, double4* __restrict__ pts,
                                int64_t* __restrict__ oidx) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= M) return;
  const double4 p = sp[k];
  const int64_t t = slot_of[k];
  pts[t] = make_double4(p.x, p.y, p.z, 1.0);
  oidx[t] = orig ? (int64_t)orig[k] : k;
}

// Target order of the centres: the surface points in curve order (their
// on-surface centre, paper index i < n, in sorted order), each followed by
// its two off-surface centres i + n and i + 2n, which lie within the offset
// of it.  Groups of whole triples cover fewer surface points than groups of
// centres in their own curve order, so their source lists are shorter.
__global__ void k_invert_perm(const uint32_t* __restrict__ perm, int64_t m, uint32_t* __restrict__ inv) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < m) inv[perm[k]] = (uint32_t)k;
}
__global__ void k_surface_flags(const uint32_t* __restrict__ perm, int64_t m, int64_t n, int64_t* __restrict__ f) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < m) f[k] = perm[k] < (uint32_t)n ? 1 : 0;
}
__global__ void k_triple_order(const uint32_t* __restrict__ perm, const uint32_t* __restrict__ inv,
                               const int64_t* __restrict__ rank, int64_t m, int64_t n, const double4* __restrict__ xs,
                               uint32_t* __restrict__ order, double4* __restrict__ sp) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= m) return;
  const uint32_t i = perm[k];
  if (i >= (uint32_t)n) return;
  const int64_t r = rank[k];
  const uint32_t k1 = inv[i + n], k2 = inv[i + 2 * n];
  order[3 * r] = (uint32_t)k;
  order[3 * r + 1] = k1;
  order[3 * r + 2] = k2;
  sp[3 * r] = xs[k];
  sp[3 * r + 1] = xs[k1];
  sp[3 * r + 2] = xs[k2];
}

// Points of an evaluation set in a given order, as double4.
__global__ void k_gather_points(const double* __restrict__ P, const uint32_t* __restrict__ perm, int64_t n,
                                double4* __restrict__ sp) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int64_t i = perm[k];
  sp[k] = make_double4(P[3 * i], P[3 * i + 1], P[3 * i + 2], 0.0);
}

}  // namespace

// ===========================================================================
// Launchers
// ===========================================================================
void check_inputs(const double* points, const double* normals, int64_t n, int* flags, hipStream_t s) {
  hipLaunchKernelGGL(k_check_inputs, dim3(grid_for(n)), dim3(kThreads), 0, s, points, normals, n, flags);
  RBF_HIP(hipGetLastError());
}

void build_centres(const double* points, const double* normals, int64_t n, double eps, double* xpaper,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_build_centres, dim3(grid_for(n)), dim3(kThreads), 0, s, points, normals, n, eps, xpaper);
  RBF_HIP(hipGetLastError());
}

void bounding_box(const double* X, int64_t m, double* box6, double* scratch, hipStream_t s) {
  int nb = (int)std::min<int64_t>(1024, ceil_div(m, kThreads));
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_bbox_partial, dim3(nb), dim3(kThreads), 0, s, X, m, scratch);
  hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(kThreads), 0, s, scratch, nb, box6);
  RBF_HIP(hipGetLastError());
}

// Workspace of scan_exclusive_i64_ws for n entries: the tile sums and their
// scan, two entries per tile at every level of the recursion.
int64_t scan_ws_elems(int64_t n) {
  int64_t total = 0;
  while (n > 0) {
    const int64_t nb = ceil_div(n, kScanTile);
    total += 2 * nb;
    if (nb <= 1) break;
    n = nb;
  }
  return total;
}

void scan_exclusive_i64_ws(const int64_t* in, int64_t* out, int64_t n, int64_t* ws, hipStream_t s) {
  if (n <= 0) return;
  const int64_t nb = ceil_div(n, kScanTile);
  int64_t* sums = ws;
  int64_t* sums_scanned = ws + nb;
  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nb), dim3(kThreads), 0, s, in, out, n, sums);
  RBF_HIP(hipGetLastError());
  if (nb > 1) {
    scan_exclusive_i64_ws(sums, sums_scanned, nb, ws + 2 * nb, s);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(kThreads), 0, s, out, n, sums_scanned);
    RBF_HIP(hipGetLastError());
  }
}

void scan_exclusive_i64(const int64_t* in, int64_t* out, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  int64_t* ws = talloc<int64_t>(scan_ws_elems(n));
  scan_exclusive_i64_ws(in, out, n, ws, s);
  temp_free(ws);
}

// Stable LSD radix sort of (key, value) pairs on the low `bits` key bits,
// 8 bits per pass; on return ki/vi point at the sorted arrays (the buffers
// swap roles every pass).  hist/offs hold 256 entries per tile.
static void radix_passes(uint32_t*& ki, uint32_t*& vi, uint32_t*& ko, uint32_t*& vo, int64_t m, int bits,
                         int64_t* hist, int64_t* offs, hipStream_t s) {
  const int nb = (int)ceil_div(m, kRsTile);
  for (int shift = 0; shift < bits; shift += 8) {
    hipLaunchKernelGGL(k_rs_hist, dim3(nb), dim3(kThreads), 0, s, ki, m, shift, hist, nb);
    RBF_HIP(hipGetLastError());
    scan_exclusive_i64(hist, offs, (int64_t)256 * nb, s);
    hipLaunchKernelGGL(k_rs_scatter, dim3(nb), dim3(kThreads), 0, s, ki, vi, ko, vo, m, shift, offs, nb);
    RBF_HIP(hipGetLastError());
    std::swap(ki, ko);
    std::swap(vi, vo);
  }
}

void sort_points(const double* pts3, int64_t m, const Lattice& lat, uint32_t* perm, uint32_t* keys_out,
                 hipStream_t s) {
  const int nb = (int)ceil_div(m, kRsTile);
  uint32_t* k0 = talloc<uint32_t>(m);
  uint32_t* v0 = talloc<uint32_t>(m);
  uint32_t* k1 = talloc<uint32_t>(m);
  uint32_t* v1 = talloc<uint32_t>(m);
  int64_t* hist = talloc<int64_t>((int64_t)256 * nb);
  int64_t* offs = talloc<int64_t>((int64_t)256 * nb);
  hipLaunchKernelGGL(k_curve_keys, dim3(grid_for(m)), dim3(kThreads), 0, s, pts3, m, lat, k0, v0);
  RBF_HIP(hipGetLastError());
  uint32_t *ki = k0, *vi = v0, *ko = k1, *vo = v1;
  radix_passes(ki, vi, ko, vo, m, 3 * kCurveBits, hist, offs, s);
  RBF_HIP(hipMemcpyAsync(perm, vi, sizeof(uint32_t) * m, hipMemcpyDeviceToDevice, s));
  if (keys_out) RBF_HIP(hipMemcpyAsync(keys_out, ki, sizeof(uint32_t) * m, hipMemcpyDeviceToDevice, s));
  temp_free(k0); temp_free(v0); temp_free(k1); temp_free(v1); temp_free(hist); temp_free(offs);
}

void gather_sorted(const double* pts3, const uint32_t* perm, int64_t m, double sqrt_k, double4* xs, double4* xk,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_gather_sorted, dim3(grid_for(m + 1)), dim3(kThreads), 0, s, pts3, perm, m, sqrt_k, xs, xk);
  RBF_HIP(hipGetLastError());
}

namespace {
struct PinnedStack {
  int64_t* base = nullptr;   // kPinnedSlots slots, kept until the thread ends
  int top = 0;
};
PinnedStack& pinned_stack() {
  static thread_local PinnedStack st;
  if (!st.base) RBF_HIP(hipHostMalloc((void**)&st.base, kPinnedSlots * sizeof(int64_t), hipHostMallocDefault));
  return st;
}
}  // namespace

PinnedSlots::PinnedSlots(int count) : p(nullptr), n(0) {
  PinnedStack& st = pinned_stack();
  if (count < 0 || st.top + count > kPinnedSlots)
    throw Error{RBF_EDEVICE, "pinned read-back slots exhausted (internal error)"};
  p = st.base + st.top;
  n = count;
  st.top += count;
}
PinnedSlots::~PinnedSlots() { pinned_stack().top -= n; }

void build_cells(const uint32_t* keys, const double4* xs, int64_t m, const Lattice& lat, int32_t** cell_start,
                 int32_t** cell_count, int32_t** cell_map, int32_t** cell_xyz, int64_t* ncell_parts, hipStream_t s) {
  const int cshift = 3 * lat.shift;
  int64_t* flag = talloc<int64_t>(m);
  int64_t* cid = talloc<int64_t>(m);
  hipLaunchKernelGGL(k_cell_flags, dim3(grid_for(m)), dim3(kThreads), 0, s, keys, m, cshift, flag);
  RBF_HIP(hipGetLastError());
  scan_exclusive_i64(flag, cid, m, s);
  // the number of occupied cells is cid[m-1] + flag[m-1]: queued into the
  // caller's pinned slots, not waited for (the arrays take the bound m)
  RBF_HIP(hipMemcpyAsync(ncell_parts, cid + (m - 1), sizeof(int64_t), hipMemcpyDeviceToHost, s));
  RBF_HIP(hipMemcpyAsync(ncell_parts + 1, flag + (m - 1), sizeof(int64_t), hipMemcpyDeviceToHost, s));
  const int64_t nmap = (int64_t)lat.cdims[0] * lat.cdims[1] * lat.cdims[2];
  *cell_start = dalloc<int32_t>(m);
  *cell_count = dalloc<int32_t>(m);
  *cell_map = dalloc<int32_t>(nmap);
  *cell_xyz = dalloc<int32_t>(m);
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(nmap)), dim3(kThreads), 0, s, *cell_map, -1, nmap);
  hipLaunchKernelGGL(k_cell_fill, dim3(grid_for(m)), dim3(kThreads), 0, s, xs, m, flag, cid, lat,
                     *cell_start, *cell_count, *cell_map, *cell_xyz);
  RBF_HIP(hipGetLastError());
  temp_free(flag);
  temp_free(cid);
}

void group_targets(const Ctx& c, const double4* sp, const uint32_t* orig, int64_t M, TargetSet& ts,
                   hipStream_t s) {
  const double E = 8.0 * c.sigma;
  const int64_t nseg = ceil_div(M, kGroupSeg);
  int64_t* gcount = talloc<int64_t>(nseg);
  int64_t* goff = talloc<int64_t>(nseg);
  int64_t* slot_of = talloc<int64_t>(M);
  int32_t* local_slot = talloc<int32_t>(M);
  const unsigned gblocks = (unsigned)ceil_div(nseg, kThreads / kWave);
  hipLaunchKernelGGL(k_group_greedy, dim3(gblocks), dim3(kThreads), 0, s, sp, M, E * E, gcount, local_slot);
  RBF_HIP(hipGetLastError());
  scan_exclusive_i64(gcount, goff, nseg, s);
  PinnedSlots last(2);
  RBF_HIP(hipMemcpyAsync(last.p, goff + (nseg - 1), sizeof(int64_t), hipMemcpyDeviceToHost, s));
  RBF_HIP(hipMemcpyAsync(last.p + 1, gcount + (nseg - 1), sizeof(int64_t), hipMemcpyDeviceToHost, s));
  RBF_HIP(hipStreamSynchronize(s));
  ts.n_targets = M;
  ts.n_groups = last.p[0] + last.p[1];
  const int64_t total = ts.n_groups * kGroup;
  ts.pts = set_alloc<double4>(ts, total);
  ts.index = set_alloc<int64_t>(ts, total);
  ts.owned.push_back(ts.index);
  hipLaunchKernelGGL(k_group_slots, dim3(grid_for(M)), dim3(kThreads), 0, s, local_slot, goff, M, slot_of);
  hipLaunchKernelGGL(k_pad_targets, dim3(grid_for(total)), dim3(kThreads), 0, s, ts.pts, ts.index, total);
  hipLaunchKernelGGL(k_place_targets, dim3(grid_for(M)), dim3(kThreads), 0, s, sp, orig, M, slot_of, ts.pts,
                     ts.index);
  RBF_HIP(hipGetLastError());
  temp_free(gcount);
  temp_free(goff);
  temp_free(slot_of);
  temp_free(local_slot);
}

// The centres as the operator's targets, grouped by surface-point triples
// (m = 3 n centres, sorted by `perm`).
void centre_targets(const Ctx& c, TargetSet& ts, hipStream_t s) {
  const int64_t m = c.m, n = c.n;
  uint32_t* inv = talloc<uint32_t>(m);
  int64_t* flag = talloc<int64_t>(m);
  int64_t* rank = talloc<int64_t>(m);
  uint32_t* order = talloc<uint32_t>(m);
  double4* sp = talloc<double4>(m);
  hipLaunchKernelGGL(k_invert_perm, dim3(grid_for(m)), dim3(kThreads), 0, s, c.perm, m, inv);
  hipLaunchKernelGGL(k_surface_flags, dim3(grid_for(m)), dim3(kThreads), 0, s, c.perm, m, n, flag);
  RBF_HIP(hipGetLastError());
  scan_exclusive_i64(flag, rank, m, s);
  hipLaunchKernelGGL(k_triple_order, dim3(grid_for(m)), dim3(kThreads), 0, s, c.perm, inv, rank, m, n, c.xs, order,
                     sp);
  RBF_HIP(hipGetLastError());
  group_targets(c, sp, order, m, ts, s);
  temp_free(inv);
  temp_free(flag);
  temp_free(rank);
  temp_free(order);
  temp_free(sp);
}

void sum_i64(const int64_t* in, int64_t n, int64_t* out, hipStream_t s) {
  RBF_HIP(hipMemsetAsync(out, 0, sizeof(int64_t), s));
  if (n <= 0) return;
  hipLaunchKernelGGL(k_sum_i64, dim3((unsigned)std::min<int64_t>(256, ceil_div(n, kThreads))), dim3(kThreads), 0, s,
                     in, n, out);
  RBF_HIP(hipGetLastError());
}

void fill_f64(double* p, double v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(n)), dim3(kThreads), 0, s, p, v, n);
  RBF_HIP(hipGetLastError());
}
void fill_f32(float* p, float v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_f32, dim3(grid_for(n)), dim3(kThreads), 0, s, p, v, n);
  RBF_HIP(hipGetLastError());
}
void fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n)), dim3(kThreads), 0, s, p, v, n);
  RBF_HIP(hipGetLastError());
}

// Builds ts.groups / ts.list for the targets in ts.pts (n_groups*16 points).
void build_lists(const Ctx& c, TargetSet& ts, hipStream_t s, int64_t* inner_slot) {
  const int64_t G = ts.n_groups;
  ts.groups = set_alloc<GroupInfo>(ts, G);
  ts.owned.push_back(ts.groups);
  int64_t* tmp = talloc<int64_t>(1);
  if (ts.dense) {
    hipLaunchKernelGGL(k_dense_groups, dim3(grid_for(G)), dim3(kThreads), 0, s, ts.pts, G, c.m, ts.groups);
    RBF_HIP(hipGetLastError());
    ts.list = nullptr;
    ts.mask = nullptr;
    ts.list_entries = G * round_up(c.m, kChunk);
    ts.inner_entries = ts.list_entries;
    ts.useful = ts.n_targets * c.m;
  } else {
    int64_t* bnd = talloc<int64_t>(G);
    int64_t* soff = talloc<int64_t>(G);
    int32_t* cin = talloc<int32_t>(G);
    int32_t* cout = talloc<int32_t>(G);
    int64_t* use = talloc<int64_t>(G);
    uint32_t* vm = talloc<uint32_t>(G);
    int64_t* len = talloc<int64_t>(G);
    int64_t* off = talloc<int64_t>(G);
    const unsigned nblk = (unsigned)ceil_div(G, 4);
    // 1. candidate bounds: staging regions (the sources of each group's
    // cell cube from the summed cell counts; without them, the cells of the
    // cube within reach, one wave per group)
    if (c.cell_sat)
      hipLaunchKernelGGL(k_list_bound_sat, dim3(grid_for(G)), dim3(kThreads), 0, s, ts.pts, G, c.cell_sat, c.lat,
                         c.cutoff, bnd);
    else
      hipLaunchKernelGGL((k_lists<kBound, false>), dim3(nblk), dim3(kThreads), 0, s, ts.pts, G, ts.groups, c.xs,
                         c.cell_start, c.cell_count, c.cell_map, c.lat, c.cutoff, c.rc2, bnd,
                         (const int64_t*)nullptr, (int32_t*)nullptr, (int32_t*)nullptr, (int64_t*)nullptr,
                         (uint32_t*)nullptr, (uint32_t*)nullptr, (uint16_t*)nullptr, (int*)nullptr);
    RBF_HIP(hipGetLastError());
    scan_exclusive_i64(bnd, soff, G, s);
    int64_t staged = 0;
    {
      PinnedSlots last(2);
      RBF_HIP(hipMemcpyAsync(last.p, soff + (G - 1), sizeof(int64_t), hipMemcpyDeviceToHost, s));
      RBF_HIP(hipMemcpyAsync(last.p + 1, bnd + (G - 1), sizeof(int64_t), hipMemcpyDeviceToHost, s));
      RBF_HIP(hipStreamSynchronize(s));
      staged = last.p[0] + last.p[1];
    }
    uint32_t* slist = talloc<uint32_t>(staged);
    uint16_t* smask = talloc<uint16_t>(staged);
    int* overflow = talloc<int>(1);
    RBF_HIP(hipMemsetAsync(overflow, 0, sizeof(int), s));
    // 2. the classification, once, into the staging regions
    if (ts.lattice)
      hipLaunchKernelGGL((k_lists<kStage, true>), dim3(nblk), dim3(kThreads), 0, s, ts.pts, G, ts.groups, c.xs,
                         c.cell_start, c.cell_count, c.cell_map, c.lat, c.cutoff, c.rc2, bnd, soff, cin, cout, use, vm,
                         slist, smask, overflow);
    else
      hipLaunchKernelGGL((k_lists<kStage, false>), dim3(nblk), dim3(kThreads), 0, s, ts.pts, G, ts.groups, c.xs,
                         c.cell_start, c.cell_count, c.cell_map, c.lat, c.cutoff, c.rc2, bnd, soff, cin, cout, use, vm,
                         slist, smask, overflow);
    RBF_HIP(hipGetLastError());
    // 3. final offsets and the compact layout
    hipLaunchKernelGGL(k_list_lengths, dim3(grid_for(G)), dim3(kThreads), 0, s, ts.groups, G, len);
    RBF_HIP(hipGetLastError());
    scan_exclusive_i64(len, off, G, s);
    sum_i64(use, G, tmp, s);
    int64_t last_off = 0, last_len = 0, overflowed = 0;
    {
      PinnedSlots v(4);
      v.p[3] = 0;
      RBF_HIP(hipMemcpyAsync(v.p, off + (G - 1), sizeof(int64_t), hipMemcpyDeviceToHost, s));
      RBF_HIP(hipMemcpyAsync(v.p + 1, len + (G - 1), sizeof(int64_t), hipMemcpyDeviceToHost, s));
      RBF_HIP(hipMemcpyAsync(v.p + 2, tmp, sizeof(int64_t), hipMemcpyDeviceToHost, s));
      RBF_HIP(hipMemcpyAsync(v.p + 3, overflow, sizeof(int), hipMemcpyDeviceToHost, s));
      RBF_HIP(hipStreamSynchronize(s));
      last_off = v.p[0];
      last_len = v.p[1];
      ts.useful = v.p[2];
      overflowed = (int)(uint32_t)v.p[3];
    }
    temp_free(overflow);
    if (overflowed) throw Error{RBF_EDEVICE, "source list larger than its candidate bound (internal error)"};
    ts.list_entries = last_off + last_len;
    ts.list = set_alloc<uint32_t>(ts, ts.list_entries + kListTail);
    ts.owned.push_back(ts.list);
    fill_u32(ts.list + ts.list_entries, (uint32_t)c.m, kListTail, s);
    ts.mask = set_alloc<uint16_t>(ts, ts.list_entries);
    ts.owned.push_back(ts.mask);
    hipLaunchKernelGGL(k_list_compact, dim3(nblk), dim3(kThreads), 0, s, ts.groups, G, off, soff, bnd, cin, cout, vm,
                       slist, smask, (uint32_t)c.m, ts.list, ts.mask);
    RBF_HIP(hipGetLastError());
    temp_free(slist); temp_free(smask); temp_free(bnd); temp_free(soff); temp_free(cin); temp_free(cout);
    // entries of the inner chunks (the pair kernels' unmasked loop), for the statistics
    hipLaunchKernelGGL(k_inner_lengths, dim3(grid_for(G)), dim3(kThreads), 0, s, ts.groups, G, len);
    RBF_HIP(hipGetLastError());
    sum_i64(len, G, tmp, s);
    temp_free(use); temp_free(vm); temp_free(len); temp_free(off);
    if (inner_slot) {
      RBF_HIP(hipMemcpyAsync(inner_slot, tmp, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    } else {
      PinnedSlots v(1);
      RBF_HIP(hipMemcpyAsync(v.p, tmp, sizeof(int64_t), hipMemcpyDeviceToHost, s));
      RBF_HIP(hipStreamSynchronize(s));
      ts.inner_entries = v.p[0];
    }
  }
  if (ts.dense && inner_slot) *inner_slot = ts.inner_entries;
  // the operator's groups run many times: longest first within each XCD's slots
  if (!ts.dense && ts.kind == 0 && G > 0 && G < ((int64_t)1 << 31)) {
    ts.order = set_alloc<int32_t>(ts, G);
    ts.owned.push_back(ts.order);
    hipLaunchKernelGGL(k_group_order, dim3(8), dim3(kThreads), 0, s, ts.groups, G,
                       ceil_div(G, (int64_t)kGroupsPerLaunchBlock), ts.order);
    RBF_HIP(hipGetLastError());
  }
  temp_free(tmp);
}

// Releases every array of a target set (stream-ordered for temporaries).
void free_targets(TargetSet& ts) {
  auto release = [&](void* p) {
    if (ts.temp)
      temp_free(p);
    else
      dfree(p);
  };
  for (void* p : ts.owned) release(p);
  ts.owned.clear();
  release(ts.pts);
  ts.pts = nullptr;
  ts.groups = nullptr;
  ts.list = nullptr;
  ts.mask = nullptr;
  ts.order = nullptr;
}

int64_t* build_cell_sat(const Ctx& c, hipStream_t s) {
  const int64_t n = (int64_t)(c.lat.cdims[0] + 1) * (c.lat.cdims[1] + 1) * (c.lat.cdims[2] + 1);
  if (n > kCellSatMax) return nullptr;
  int64_t* sat = dalloc<int64_t>(n);
  hipLaunchKernelGGL(k_sat_counts, dim3(grid_for(n)), dim3(kThreads), 0, s, c.cell_map, c.cell_count, c.lat, sat);
  for (int axis = 0; axis < 3; ++axis) {
    const int64_t lines = n / (c.lat.cdims[axis] + 1);
    hipLaunchKernelGGL(k_sat_scan, dim3(grid_for(lines)), dim3(kThreads), 0, s, c.lat, axis, sat);
  }
  RBF_HIP(hipGetLastError());
  return sat;
}

GridDesc grid_desc(const rbf_grid& g) {
  GridDesc gd;
  const int bs[3] = {4, 2, 2};
  for (int d = 0; d < 3; ++d) {
    gd.o[d] = g.origin[d];
    gd.h[d] = g.h[d];
    gd.n[d] = g.dims[d];
    gd.nb[d] = ceil_div(g.dims[d], bs[d]);
  }
  return gd;
}

// mark[b] = 1 for the bricks with an occupied cell within the cutoff (plus a
// node of slack), 0 for the others.
void mark_support(const Ctx& c, const GridDesc& gd, int64_t* mark, int64_t nbricks, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_i64, dim3(grid_for(nbricks)), dim3(kThreads), 0, s, mark, (int64_t)0, nbricks);
  hipLaunchKernelGGL(k_mark_bricks, dim3(grid_for(c.n_cells)), dim3(kThreads), 0, s, c.cell_xyz, c.n_cells, c.lat,
                     c.cutoff, gd, mark);
  RBF_HIP(hipGetLastError());
}

// Marks the bricks with a centre in reach (mark, 0/1) and scans the marks
// (pos); returns their count.  scan_ws: scan_ws_elems(nbricks) entries.
static int64_t mark_support_bricks(const Ctx& c, const GridDesc& gd, int64_t nbricks, int64_t* mark, int64_t* pos,
                                   int64_t* scan_ws, hipStream_t s) {
  mark_support(c, gd, mark, nbricks, s);
  scan_exclusive_i64_ws(mark, pos, nbricks, scan_ws, s);
  PinnedSlots last(2);
  RBF_HIP(hipMemcpyAsync(last.p, pos + (nbricks - 1), sizeof(int64_t), hipMemcpyDeviceToHost, s));
  RBF_HIP(hipMemcpyAsync(last.p + 1, mark + (nbricks - 1), sizeof(int64_t), hipMemcpyDeviceToHost, s));
  RBF_HIP(hipStreamSynchronize(s));
  return last.p[0] + last.p[1];
}

int64_t support_bricks(const Ctx& c, const rbf_grid& g, int64_t** ids_out, hipStream_t s) {
  const GridDesc gd = grid_desc(g);
  const int64_t nbricks = gd.nb[0] * gd.nb[1] * gd.nb[2];
  *ids_out = nullptr;
  if (!std::isfinite(c.cutoff)) return nbricks;
  int64_t* mark = talloc<int64_t>(nbricks);
  int64_t* pos = talloc<int64_t>(nbricks);
  int64_t* ws = talloc<int64_t>(scan_ws_elems(nbricks));
  const int64_t nact = mark_support_bricks(c, gd, nbricks, mark, pos, ws, s);
  int64_t* ids = talloc<int64_t>(nact);
  hipLaunchKernelGGL(k_compact, dim3(grid_for(nbricks)), dim3(kThreads), 0, s, mark, pos, nbricks, ids);
  RBF_HIP(hipGetLastError());
  temp_free(mark);
  temp_free(pos);
  temp_free(ws);
  *ids_out = ids;
  return nact;
}

void brick_targets(const Ctx& c, const rbf_grid& g, const int64_t* ids, int64_t nact, TargetSet& ts,
                   hipStream_t s) {
  const GridDesc gd = grid_desc(g);
  ts.temp = true;
  ts.kind = 1;
  ts.lattice = true;
  ts.dense = !std::isfinite(c.cutoff);
  ts.n_groups = nact;
  ts.pts = set_alloc<double4>(ts, nact * kGroup);
  ts.index = set_alloc<int64_t>(ts, nact * kGroup);
  ts.owned.push_back(ts.index);
  if (nact > 0) {
    hipLaunchKernelGGL(k_brick_targets, dim3(grid_for(nact * kGroup)), dim3(kThreads), 0, s, ids, nact, gd, ts.pts,
                       ts.index);
    RBF_HIP(hipGetLastError());
    int64_t* cnt = talloc<int64_t>(1);
    RBF_HIP(hipMemsetAsync(cnt, 0, sizeof(int64_t), s));
    const int nbk = (int)std::min<int64_t>(1024, ceil_div(nact * kGroup, kThreads));
    hipLaunchKernelGGL(k_count_valid, dim3(nbk), dim3(kThreads), 0, s, ts.pts, nact * kGroup, cnt);
    RBF_HIP(hipGetLastError());
    RBF_HIP(hipMemcpyAsync(&ts.n_targets, cnt, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    RBF_HIP(hipStreamSynchronize(s));
    temp_free(cnt);
    build_lists(c, ts, s);
  }
}

void grid_targets(const Ctx& c, const rbf_grid& g, TargetSet& ts, hipStream_t s) {
  int64_t* ids = nullptr;
  const int64_t nact = support_bricks(c, g, &ids, s);
  brick_targets(c, g, ids, nact, ts, s);
  temp_free(ids);
}

void point_targets(const Ctx& c, const double* pts, int64_t npts, TargetSet& ts, hipStream_t s) {
  ts.temp = true;
  ts.kind = 1;
  uint32_t* perm = talloc<uint32_t>(npts);
  double4* sp = talloc<double4>(npts);
  sort_points(pts, npts, c.lat, perm, nullptr, s);
  hipLaunchKernelGGL(k_gather_points, dim3(grid_for(npts)), dim3(kThreads), 0, s, pts, perm, npts, sp);
  RBF_HIP(hipGetLastError());
  ts.dense = !std::isfinite(c.cutoff);
  group_targets(c, sp, perm, npts, ts, s);
  build_lists(c, ts, s);
  temp_free(perm);
  temp_free(sp);
}

}  // namespace rbf
