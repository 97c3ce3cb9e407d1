// Restarted GMRES on the device, float64 throughout (Sec. III.A: the
// interpolation system is solved by GMRES; the paper relies on PETSc's
// KSPSolve).  One Arnoldi step after the operator has produced w = A v_j:
//   pass 1  h1 = V^T w                       (block partial dot products)
//   pass 2  w <- w - V h1,  h2 = V^T w,      (one sweep: update, then dots;
//           |w|^2                             classical Gram-Schmidt applied
//                                             twice, "twice is enough")
//   pass 3  beta = |w - V h2| = sqrt(|w|^2 - |h2|^2), H(:,j) = h1 + h2,
//           H(j+1,j) = beta, Givens rotations, |g_{j+1}|, and
//           v_{j+1} = (w - V h2) / beta in one sweep
// (the second pass's coefficients h2 are of the order of the basis' rounding
// times |w|, so the norm of the corrected vector follows from |w|^2 - |h2|^2
// to float64 precision unless the step is at a breakdown, which ends the
// cycle anyway; every block forms beta from the same folded values).
// Every kernel of a step first reads the device flag `done`, set when the
// residual estimate |g_{j+1}| reaches the tolerance (or on breakdown), so the
// host can enqueue a whole cycle without waiting on it.
// The basis (and the operator's output w) is stored as T: float64, or
// float32 for the inner solve of the refinement, whose operator is float32
// anyway (half the traffic of these memory-bound passes); dot products,
// norms and updates are formed in float64 either way, and the rounding to T
// happens once per stored element.
#include <cstddef>

#include "common.h"

namespace rbf {

constexpr int kMaxRestart = 64;
constexpr int kVecThreads = 256;
constexpr int kRowsPerThread = 2;
constexpr int kRowsPerBlock = kVecThreads * kRowsPerThread;

struct GmState {
  int m;
  int k;
  int done;
  int breakdown;
  double tol_abs;
  double beta0;
  double inv_beta;
  double g[kMaxRestart + 1];
  // (the host reads the fields above after every cycle; those below stay on the device)
  double h1[kMaxRestart + 1];
  double h2[kMaxRestart + 1];
  double H[(kMaxRestart + 1) * kMaxRestart];     // column j at H[j*(kMaxRestart+1) + i], rotated
  double Hraw[(kMaxRestart + 1) * kMaxRestart];  // the same columns before the rotations
  double cs[kMaxRestart], sn[kMaxRestart];
  double y[kMaxRestart];
};

namespace {

// v plus lane `ctrl` of the DPP pattern (a double moved as two 32-bit halves);
// lanes the row mask leaves out add 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_add(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, ROW_MASK, 0xf, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, ROW_MASK, 0xf, false);
  return v + __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Sum over the wave's 64 lanes, the same in every lane, in a fixed order:
// quads, half-rows and rows by DPP (quad_perm, row_half_mirror, row_mirror),
// then rows 0+1 and 2+3 (row_bcast:15), then all (row_bcast:31) into lane
// 63, read back as a uniform value.
__device__ __forceinline__ double wave_sum(double v) {
  v = dpp_add<0xB1, 0xf>(v);    // quad_perm [1,0,3,2]
  v = dpp_add<0x4E, 0xf>(v);    // quad_perm [2,3,0,1]
  v = dpp_add<0x141, 0xf>(v);   // row_half_mirror
  v = dpp_add<0x140, 0xf>(v);   // row_mirror
  v = dpp_add<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
  v = dpp_add<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, 63);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), 63);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Block sums: every wave folds its lanes (fixed butterfly order) into
// s[wave][i]; thread i then adds the four waves in order.  The partials are
// stored column by column (partial[i * nb + b] for block b of nb), so that
// the fold of one column reads contiguous memory.
__device__ __forceinline__ void wave_partial(double v, int i, double (*s)[kMaxRestart + 1]) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6][i] = v;
}
__device__ __forceinline__ void block_store(double (*s)[kMaxRestart + 1], int ncols, double* partial) {
  __syncthreads();
  for (int i = threadIdx.x; i < ncols; i += kVecThreads)
    partial[(int64_t)i * gridDim.x + blockIdx.x] = ((s[0][i] + s[1][i]) + s[2][i]) + s[3][i];
}

// Dot products of the block's rows of x with columns 0..ncols-1 of V, into
// s[wave][i].  Columns go eight at a time with eight independent sums, so the
// loads of a block of columns are all in flight together and the eight wave
// reductions interleave.  The basis holds round_up(ncols, 8) finite columns
// (kKrylovColPad; zeroed at allocation), so the block reads them unguarded
// and keeps only the first ncols sums.
constexpr int kColPad = kKrylovColPad;
template <class T>
__device__ __forceinline__ void block_dots(const T* __restrict__ V, int64_t ldv, int ncols,
                                           const double (&x)[kRowsPerThread], int64_t base, int64_t n,
                                           double (*s)[kMaxRestart + 1]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int i0 = 0; i0 < ncols; i0 += kColPad) {
    double a[kColPad];
#pragma unroll
    for (int c = 0; c < kColPad; ++c) a[c] = 0.0;
#pragma unroll
    for (int q = 0; q < kRowsPerThread; ++q) {
      const int64_t r = base + (int64_t)q * kVecThreads;
      if (r < n) {
#pragma unroll
        for (int c = 0; c < kColPad; ++c) a[c] = fma((double)V[(int64_t)(i0 + c) * ldv + r], x[q], a[c]);
      }
    }
#pragma unroll
    for (int c = 0; c < kColPad; ++c) a[c] = wave_sum(a[c]);
    if (lane == 0) {
#pragma unroll
      for (int c = 0; c < kColPad; ++c)
        if (i0 + c < ncols) s[wave][i0 + c] = a[c];
    }
  }
}

// pass 1: partial[b][i] = sum_{r in block b} V_i[r] w[r]
template <class T>
__global__ __launch_bounds__(kVecThreads) void k_dots(const T* __restrict__ V, int64_t ldv, int ncols,
                                                      const T* __restrict__ w, int64_t n,
                                                      const GmState* __restrict__ st, double* __restrict__ partial) {
  if (st->done) return;
  __shared__ double s[kVecThreads / 64][kMaxRestart + 1];
  const int64_t base = (int64_t)blockIdx.x * kRowsPerBlock + threadIdx.x;
  double wr[kRowsPerThread];
#pragma unroll
  for (int q = 0; q < kRowsPerThread; ++q) {
    const int64_t r = base + (int64_t)q * kVecThreads;
    wr[q] = r < n ? (double)w[r] : 0.0;
  }
  block_dots(V, ldv, ncols, wr, base, n, s);
  block_store(s, ncols, partial);
}

// pass 2: w <- w - V h1 ; partial = V^T w, and |w|^2 as column ncols
template <class T>
__global__ __launch_bounds__(kVecThreads) void k_update_dots(const T* __restrict__ V, int64_t ldv, int ncols,
                                                             T* __restrict__ w, int64_t n,
                                                             const GmState* __restrict__ st,
                                                             double* __restrict__ partial) {
  if (st->done) return;
  __shared__ double h[kMaxRestart + 1];
  for (int i = threadIdx.x; i < ncols; i += kVecThreads) h[i] = st->h1[i];
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRowsPerBlock + threadIdx.x;
  double wr[kRowsPerThread];
  double nrm = 0.0;
  for (int q = 0; q < kRowsPerThread; ++q) {
    const int64_t r = base + (int64_t)q * kVecThreads;
    if (r < n) {
      double v = (double)w[r];
      for (int i = 0; i < ncols; ++i) v = fma(-h[i], (double)V[(int64_t)i * ldv + r], v);
      const T vt = (T)v;
      w[r] = vt;
      wr[q] = (double)vt;
      nrm = fma(wr[q], wr[q], nrm);
    } else {
      wr[q] = 0.0;
    }
  }
  __shared__ double s[kVecThreads / 64][kMaxRestart + 1];
  block_dots(V, ldv, ncols, wr, base, n, s);
  wave_partial(nrm, ncols, s);
  block_store(s, ncols + 1, partial);
}

// pass 2 with the basis values of the thread's rows kept in registers
// between the update and the dot products (one read of V instead of two):
// ncols <= 8 NB columns, float32 basis.
template <int NB>
__global__ __launch_bounds__(kVecThreads) void k_update_dots_reg(const float* __restrict__ V, int64_t ldv, int ncols,
                                                                 float* __restrict__ w, int64_t n,
                                                                 const GmState* __restrict__ st,
                                                                 double* __restrict__ partial) {
  if (st->done) return;
  constexpr int NC = NB * kColPad;
  __shared__ double h[kMaxRestart + 1];
  for (int i = threadIdx.x; i < ncols; i += kVecThreads) h[i] = st->h1[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t base = (int64_t)blockIdx.x * kRowsPerBlock + threadIdx.x;
  float vc[NC][kRowsPerThread];
  double wr[kRowsPerThread];
#pragma unroll
  for (int q = 0; q < kRowsPerThread; ++q) {
    const int64_t r = base + (int64_t)q * kVecThreads;
    if (r < n) {
      // columns ncols .. NC-1 exist (the basis is padded to whole blocks of
      // eight) but are not part of this step
#pragma unroll
      for (int i = 0; i < NC; ++i) vc[i][q] = V[(int64_t)i * ldv + r];
      double v = (double)w[r];
#pragma unroll
      for (int i = 0; i < NC; ++i)
        if (i < ncols) v = fma(-h[i], (double)vc[i][q], v);
      const float vt = (float)v;
      w[r] = vt;
      wr[q] = (double)vt;
    } else {
#pragma unroll
      for (int i = 0; i < NC; ++i) vc[i][q] = 0.0f;
      wr[q] = 0.0;
    }
  }
  double nrm = 0.0;
#pragma unroll
  for (int q = 0; q < kRowsPerThread; ++q) nrm = fma(wr[q], wr[q], nrm);
  __shared__ double s[kVecThreads / 64][kMaxRestart + 1];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    double a[kColPad];
#pragma unroll
    for (int c = 0; c < kColPad; ++c) {
      a[c] = 0.0;
#pragma unroll
      for (int q = 0; q < kRowsPerThread; ++q) a[c] = fma((double)vc[b * kColPad + c][q], wr[q], a[c]);
      a[c] = wave_sum(a[c]);
    }
    if (lane == 0) {
#pragma unroll
      for (int c = 0; c < kColPad; ++c)
        if (b * kColPad + c < ncols) s[wave][b * kColPad + c] = a[c];
    }
  }
  wave_partial(nrm, ncols, s);
  block_store(s, ncols + 1, partial);
}

// Sum of the block partials of one column by a whole block: thread t adds
// partials t, t+256, ... in order, each wave adds its lanes (wave_sum), and
// the four wave sums are added in order, so the result does not depend on
// scheduling.  Every thread gets the sum.
__device__ double block_fold(const double* __restrict__ partial, int nb, int col) {
  __shared__ double s[kVecThreads / 64];
  const int t = threadIdx.x;
  double acc = 0.0;
  const double* p = partial + (int64_t)col * nb;
  for (int b = t; b < nb; b += kVecThreads) acc += p[b];
  acc = wave_sum(acc);
  if ((t & 63) == 0) s[t >> 6] = acc;
  __syncthreads();
  const double r = ((s[0] + s[1]) + s[2]) + s[3];
  __syncthreads();
  return r;
}

// one block per column
__global__ __launch_bounds__(kVecThreads) void k_reduce_h1(const double* __restrict__ partial, int nb,
                                                           GmState* __restrict__ st) {
  if (st->done) return;
  const double v = block_fold(partial, nb, blockIdx.x);
  if (threadIdx.x == 0) st->h1[blockIdx.x] = v;
}
__global__ __launch_bounds__(kVecThreads) void k_reduce_h2(const double* __restrict__ partial, int nb,
                                                           GmState* __restrict__ st) {
  if (st->done) return;
  const double v = block_fold(partial, nb, blockIdx.x);
  if (threadIdx.x == 0) st->h2[blockIdx.x] = v;
}

// Column j of the Hessenberg matrix, its Givens rotations and the residual
// estimate |g_{j+1}| from beta = |w|: the column and the rotations are staged
// in LDS by the whole block, the rotation chain runs on one thread from there.
__device__ void finish_step(double beta, int j, GmState* __restrict__ st) {
  __shared__ double hc[kMaxRestart + 2], cs[kMaxRestart], sn[kMaxRestart];
  const int t = threadIdx.x;
  for (int i = t; i <= j; i += kVecThreads) hc[i] = st->h1[i] + st->h2[i];
  for (int i = t; i < j; i += kVecThreads) {
    cs[i] = st->cs[i];
    sn[i] = st->sn[i];
  }
  __syncthreads();
  double* Hr = st->Hraw + (int64_t)j * (kMaxRestart + 1);
  for (int i = t; i <= j; i += kVecThreads) Hr[i] = hc[i];
  if (t == 0) {
    Hr[j + 1] = beta;
    hc[j + 1] = beta;
    for (int i = 0; i < j; ++i) {
      const double a = hc[i], b = hc[i + 1];
      hc[i] = cs[i] * a + sn[i] * b;
      hc[i + 1] = -sn[i] * a + cs[i] * b;
    }
    const double a = hc[j], b = hc[j + 1];
    const double rho = hypot(a, b);
    double c = 1.0, s = 0.0;
    if (rho != 0.0) {
      c = a / rho;
      s = b / rho;
    }
    st->cs[j] = c;
    st->sn[j] = s;
    hc[j] = rho;
    hc[j + 1] = 0.0;
    const double gj = st->g[j];
    st->g[j + 1] = -s * gj;
    st->g[j] = c * gj;
    st->k = j + 1;
    st->inv_beta = beta > 0.0 ? 1.0 / beta : 0.0;
    const bool finite = isfinite(beta) && isfinite(rho) && isfinite(st->g[j + 1]);
    if (!finite) {
      st->breakdown = 1;
      st->done = 1;
      st->k = j;  // drop the column that went bad
    } else if (fabs(st->g[j + 1]) <= st->tol_abs || beta == 0.0 || rho == 0.0) {
      st->done = 1;
    }
  }
  __syncthreads();
  double* Hc = st->H + (int64_t)j * (kMaxRestart + 1);
  for (int i = t; i <= j + 1; i += kVecThreads) Hc[i] = hc[i];
}

// pass 3 and the end of step j: beta = |w - V h2| from |w|^2 - |h2|^2 (the
// folded column ncols of pass 2 and h2), v_{j+1} = (w - V h2) / beta formed
// in float64 and rounded to T once; block 0 also runs finish_step.  Every
// block forms beta from the same folded values in the same order (the same
// bits).  A block that already sees the stop flag block 0 may set skips the
// sweep: the column past the last step of a cycle is never read.
template <class T>
__global__ __launch_bounds__(kVecThreads) void k_update_scale(const T* __restrict__ V, int64_t ldv, int ncols,
                                                              const T* __restrict__ w, int64_t n, int j,
                                                              GmState* __restrict__ st, T* __restrict__ out) {
  if (st->done) return;
  __shared__ double h[kMaxRestart + 1];
  for (int i = threadIdx.x; i < ncols; i += kVecThreads) h[i] = st->h2[i];
  __syncthreads();
  double hh = 0.0;
  for (int i = 0; i < ncols; ++i) hh = fma(h[i], h[i], hh);
  const double beta = sqrt(fmax(st->h2[ncols] - hh, 0.0));
  if (blockIdx.x == 0) finish_step(beta, j, st);
  const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
  const int64_t base = (int64_t)blockIdx.x * kRowsPerBlock + threadIdx.x;
  for (int q = 0; q < kRowsPerThread; ++q) {
    const int64_t r = base + (int64_t)q * kVecThreads;
    if (r < n) {
      double v = (double)w[r];
      for (int i = 0; i < ncols; ++i) v = fma(-h[i], (double)V[(int64_t)i * ldv + r], v);
      out[r] = (T)(v * inv);
    }
  }
}

constexpr int kScaleRows = 4;   // elements per thread of the start's scaling

// r = b - y and |r|^2 partials (y may be null: r = b)
__global__ __launch_bounds__(kVecThreads) void k_residual(const double* __restrict__ b, const double* __restrict__ y,
                                                          double* __restrict__ r, int64_t n,
                                                          double* __restrict__ partial) {
  const int64_t base = (int64_t)blockIdx.x * kRowsPerBlock + threadIdx.x;
  double a = 0.0;
  for (int q = 0; q < kRowsPerThread; ++q) {
    const int64_t i = base + (int64_t)q * kVecThreads;
    if (i < n) {
      const double v = y ? b[i] - y[i] : b[i];
      r[i] = v;
      a = fma(v, v, a);
    }
  }
  __shared__ double s[kVecThreads / 64][kMaxRestart + 1];
  wave_partial(a, 0, s);
  block_store(s, 1, partial);
}

// Start of a cycle from the residual partials: beta = |r|, the state, and
// v_0 = r / beta.  Every block folds the partials itself (the same fixed
// order: the same beta in all of them); block 0 writes the state.  Nothing
// is scaled when beta is 0 or not finite (the cycle is done at once).
template <class T>
__global__ __launch_bounds__(kVecThreads) void k_start_scale(const double* __restrict__ partial, int nb, int m,
                                                             double tol_abs, GmState* __restrict__ st,
                                                             const double* __restrict__ r, int64_t n,
                                                             T* __restrict__ out) {
  const double beta = sqrt(block_fold(partial, nb, 0));
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->m = m;
    st->k = 0;
    st->tol_abs = tol_abs;
    st->beta0 = beta;
    st->g[0] = beta;
    for (int i = 1; i <= kMaxRestart; ++i) st->g[i] = 0.0;
    st->breakdown = isfinite(beta) ? 0 : 1;
    st->done = (beta == 0.0 || !isfinite(beta)) ? 1 : 0;
    st->inv_beta = beta > 0.0 ? 1.0 / beta : 0.0;
  }
  if (beta == 0.0 || !isfinite(beta)) return;
  const double inv = 1.0 / beta;
  const int64_t base = (int64_t)blockIdx.x * (kVecThreads * kScaleRows) + threadIdx.x;
#pragma unroll
  for (int q = 0; q < kScaleRows; ++q) {
    const int64_t i = base + (int64_t)q * kVecThreads;
    if (i < n) out[i] = (T)(r[i] * inv);
  }
}

// Least squares: back substitution with the rotated Hessenberg matrix, by
// one wave: the triangle and g are staged in LDS by all lanes, then row i's
// sum over l > i is spread over the lanes and added in a fixed order.
__global__ __launch_bounds__(64) void k_solve_y(GmState* __restrict__ st) {
  __shared__ double Hs[kMaxRestart * kMaxRestart];   // Hs[l * k + i] = H(i, l), i <= l
  __shared__ double ys[kMaxRestart + 1];
  const int lane = threadIdx.x;
  const int ld = kMaxRestart + 1;
  const int k = st->k;
  for (int e = lane; e < k * k; e += 64) {
    const int l = e / k, i = e % k;
    Hs[e] = i <= l ? st->H[(int64_t)l * ld + i] : 0.0;
  }
  for (int i = lane; i < k; i += 64) ys[i] = st->g[i];
  __syncthreads();
  for (int i = k - 1; i >= 0; --i) {
    double part = 0.0;
    for (int l = i + 1 + lane; l < k; l += 64) part = fma(Hs[l * k + i], ys[l], part);
    part = wave_sum(part);
    if (lane == 0) ys[i] = (ys[i] - part) / Hs[i * k + i];
    __syncthreads();
  }
  for (int i = lane; i < k; i += 64) st->y[i] = ys[i];
}

__global__ void k_set_tol(GmState* __restrict__ st, double tol_abs) {
  if (threadIdx.x == 0) st->tol_abs = tol_abs;
}

// x <- x + V y  (k columns, k read from the state)
template <class T>
__global__ __launch_bounds__(kVecThreads) void k_update_x(const T* __restrict__ V, int64_t ldv,
                                                          const GmState* __restrict__ st, double* __restrict__ x,
                                                          int64_t n) {
  const int k = st->k;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n || k == 0) return;
  double v = x[i];
  for (int l = 0; l < k; ++l) v = fma(st->y[l], (double)V[(int64_t)l * ldv + i], v);
  x[i] = v;
}

__global__ void k_to_f64(const float* __restrict__ x, double* __restrict__ y, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[i] = (double)x[i];
}

// x += y
__global__ void k_vec_add(double* __restrict__ x, const double* __restrict__ y, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) x[i] += y[i];
}

__global__ void k_gather(const double* __restrict__ src, const uint32_t* __restrict__ perm, int64_t m,
                         double* __restrict__ dst) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < m) dst[k] = src[perm[k]];
}
// The right-hand side of the interpolation system in sorted order: centre
// perm[k] of the paper order is an on-surface point (value 0) for index < n,
// an outer off-surface point (+eps) below 2n, an inner one (-eps) above.
__global__ void k_rhs_sorted(const uint32_t* __restrict__ perm, int64_t m, int64_t n, double eps,
                             double* __restrict__ dst) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < m) {
    const int64_t i = perm[k];
    dst[k] = i < n ? 0.0 : (i < 2 * n ? eps : -eps);
  }
}
__global__ void k_scatter(const double* __restrict__ src, const uint32_t* __restrict__ perm, int64_t m,
                          double* __restrict__ dst) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < m) dst[perm[k]] = src[k];
}

}  // namespace

// ===========================================================================
// Host side
// ===========================================================================
static unsigned vec_blocks(int64_t n) { return (unsigned)std::max<int64_t>(1, ceil_div(n, kRowsPerBlock)); }
static unsigned elt_blocks(int64_t n) { return (unsigned)std::max<int64_t>(1, ceil_div(n, kVecThreads)); }

void vec_add(double* x, const double* y, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_vec_add, dim3(elt_blocks(n)), dim3(kVecThreads), 0, s, x, y, n);
  RBF_HIP(hipGetLastError());
}

void gather_to_sorted(const double* src, const uint32_t* perm, int64_t m, double* dst_sorted, hipStream_t s) {
  hipLaunchKernelGGL(k_gather, dim3(elt_blocks(m)), dim3(kVecThreads), 0, s, src, perm, m, dst_sorted);
  RBF_HIP(hipGetLastError());
}
void rhs_sorted(const uint32_t* perm, int64_t m, int64_t n, double eps, double* dst_sorted, hipStream_t s) {
  hipLaunchKernelGGL(k_rhs_sorted, dim3(elt_blocks(m)), dim3(kVecThreads), 0, s, perm, m, n, eps, dst_sorted);
  RBF_HIP(hipGetLastError());
}
void scatter_from_sorted(const double* src_sorted, const uint32_t* perm, int64_t m, double* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_scatter, dim3(elt_blocks(m)), dim3(kVecThreads), 0, s, src_sorted, perm, m, dst);
  RBF_HIP(hipGetLastError());
}

int gm_max_restart() { return kMaxRestart; }
size_t gm_state_bytes() { return sizeof(GmState); }
int64_t gm_partial_count(int64_t n) { return (int64_t)vec_blocks(n) * (kMaxRestart + 1); }

// r = b - y (y may be null); starts a cycle: beta0 = |r|, v_0 = r / beta0.
template <class T>
static void gm_start_t(const double* b, const double* y, double* r, int64_t n, T* V, double* partial, int m,
                       double tol_abs, GmState* st, hipStream_t s) {
  const unsigned nb = vec_blocks(n);
  hipLaunchKernelGGL(k_residual, dim3(nb), dim3(kVecThreads), 0, s, b, y, r, n, partial);
  const unsigned sb = (unsigned)std::max<int64_t>(1, ceil_div(n, (int64_t)kVecThreads * kScaleRows));
  hipLaunchKernelGGL(k_start_scale<T>, dim3(sb), dim3(kVecThreads), 0, s, partial, (int)nb, m, tol_abs, st, r, n, V);
  RBF_HIP(hipGetLastError());
}
void gm_start(const double* b, const double* y, double* r, int64_t n, void* V, bool f32, double* partial, int m,
              double tol_abs, void* state, hipStream_t s) {
  GmState* st = static_cast<GmState*>(state);
  if (f32)
    gm_start_t(b, y, r, n, static_cast<float*>(V), partial, m, tol_abs, st, s);
  else
    gm_start_t(b, y, r, n, static_cast<double*>(V), partial, m, tol_abs, st, s);
}

// Orthogonalisation and bookkeeping of step j after w = A v_j.
template <class T>
static void gm_step_t(T* V, int64_t ldv, T* w, int64_t n, int j, double* partial, GmState* st, hipStream_t s) {
  const unsigned nb = vec_blocks(n);
  const int ncols = j + 1;
  hipLaunchKernelGGL(k_dots<T>, dim3(nb), dim3(kVecThreads), 0, s, V, ldv, ncols, w, n, st, partial);
  hipLaunchKernelGGL(k_reduce_h1, dim3(ncols), dim3(kVecThreads), 0, s, partial, (int)nb, st);
  if constexpr (std::is_same<T, float>::value) {
    switch ((ncols + kColPad - 1) / kColPad) {
      case 1: hipLaunchKernelGGL(k_update_dots_reg<1>, dim3(nb), dim3(kVecThreads), 0, s, V, ldv, ncols, w, n, st, partial); break;
      case 2: hipLaunchKernelGGL(k_update_dots_reg<2>, dim3(nb), dim3(kVecThreads), 0, s, V, ldv, ncols, w, n, st, partial); break;
      case 3: hipLaunchKernelGGL(k_update_dots_reg<3>, dim3(nb), dim3(kVecThreads), 0, s, V, ldv, ncols, w, n, st, partial); break;
      case 4: hipLaunchKernelGGL(k_update_dots_reg<4>, dim3(nb), dim3(kVecThreads), 0, s, V, ldv, ncols, w, n, st, partial); break;
      default: hipLaunchKernelGGL(k_update_dots<T>, dim3(nb), dim3(kVecThreads), 0, s, V, ldv, ncols, w, n, st, partial);
    }
  } else {
    hipLaunchKernelGGL(k_update_dots<T>, dim3(nb), dim3(kVecThreads), 0, s, V, ldv, ncols, w, n, st, partial);
  }
  // (ncols + 1 columns: h2 and |w|^2)
  hipLaunchKernelGGL(k_reduce_h2, dim3(ncols + 1), dim3(kVecThreads), 0, s, partial, (int)nb, st);
  hipLaunchKernelGGL(k_update_scale<T>, dim3(nb), dim3(kVecThreads), 0, s, V, ldv, ncols, w, n, j, st,
                     V + (int64_t)(j + 1) * ldv);
  RBF_HIP(hipGetLastError());
}
void gm_step(void* V, int64_t ldv, void* w, bool f32, int64_t n, int j, double* partial, void* state,
             hipStream_t s) {
  GmState* st = static_cast<GmState*>(state);
  if (f32)
    gm_step_t(static_cast<float*>(V), ldv, static_cast<float*>(w), n, j, partial, st, s);
  else
    gm_step_t(static_cast<double*>(V), ldv, static_cast<double*>(w), n, j, partial, st, s);
}

// x += V y after the cycle.
void gm_finish(const void* V, int64_t ldv, bool f32, double* x, int64_t n, void* state, hipStream_t s) {
  GmState* st = static_cast<GmState*>(state);
  hipLaunchKernelGGL(k_solve_y, dim3(1), dim3(64), 0, s, st);  // one wave
  if (f32)
    hipLaunchKernelGGL(k_update_x<float>, dim3(elt_blocks(n)), dim3(kVecThreads), 0, s, static_cast<const float*>(V),
                       ldv, st, x, n);
  else
    hipLaunchKernelGGL(k_update_x<double>, dim3(elt_blocks(n)), dim3(kVecThreads), 0, s,
                       static_cast<const double*>(V), ldv, st, x, n);
  RBF_HIP(hipGetLastError());
}

// float32 -> float64 copy (a basis vector handed to the preconditioner)
void to_f64(const float* x, double* y, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_to_f64, dim3(elt_blocks(n)), dim3(kVecThreads), 0, s, x, y, n);
  RBF_HIP(hipGetLastError());
}

// Sets the stopping tolerance of the cycle gm_start began (stream-ordered).
void gm_set_tol(void* state, double tol_abs, hipStream_t s) {
  hipLaunchKernelGGL(k_set_tol, dim3(1), dim3(64), 0, s, static_cast<GmState*>(state), tol_abs);
  RBF_HIP(hipGetLastError());
}

// Host copy of the fields the driver loop needs.
void gm_read(const void* state, int* k, int* done, int* breakdown, double* beta0, double* gk, hipStream_t s) {
  GmState h;
  RBF_HIP(hipMemcpyAsync(&h, state, offsetof(GmState, h1), hipMemcpyDeviceToHost, s));
  RBF_HIP(hipStreamSynchronize(s));
  *k = h.k;
  *done = h.done;
  *breakdown = h.breakdown;
  *beta0 = h.beta0;
  *gk = h.g[h.k];
}

const int* gm_done_flag(const void* state) { return &static_cast<const GmState*>(state)->done; }

// The unrotated Hessenberg matrix of the last cycle into H (host, (m+1) x m,
// row-major, zero outside the computed columns' upper Hessenberg part);
// returns the columns computed and whether a non-finite value stopped it.
int gm_read_hessenberg(const void* state, int m, double* H, int* breakdown, hipStream_t s) {
  GmState h;
  RBF_HIP(hipMemcpyAsync(&h, state, sizeof(GmState), hipMemcpyDeviceToHost, s));
  RBF_HIP(hipStreamSynchronize(s));
  const int ld = kMaxRestart + 1;
  for (int i = 0; i <= m; ++i)
    for (int j = 0; j < m; ++j) H[(int64_t)i * m + j] = (j < h.k && i <= j + 1) ? h.Hraw[(int64_t)j * ld + i] : 0.0;
  *breakdown = h.breakdown;
  return h.k;
}

}  // namespace rbf
