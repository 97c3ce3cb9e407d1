// Density measures of the point cloud (Sec. IV, eqs. sepDist, fillDist and
// hmax): nearest-neighbour distances by an exact float64 all-pairs scan with
// LDS tiles.  The squared distance is formed as (dx*dx + dy*dy) + dz*dz and
// minimised before any square root, so the results are the exact minima of
// the float64 distances.
#include "common.h"

namespace rbf {

namespace {

constexpr int kDThreads = 256;

// best[i] = min_{j != i} |p_i - p_j|^2 (self excluded by index), or, when
// `queries` is given, min_j |q_i - p_j|^2.
__global__ __launch_bounds__(kDThreads) void k_nearest(const double* __restrict__ P, int64_t n,
                                                       const double* __restrict__ queries, int64_t nq,
                                                       double* __restrict__ best) {
  __shared__ double tile[kDThreads][3];
  const int64_t i = blockIdx.x * (int64_t)kDThreads + threadIdx.x;
  const bool self = queries == nullptr;
  double qx = 0, qy = 0, qz = 0;
  if (i < nq) {
    const double* src = self ? P : queries;
    qx = src[3 * i];
    qy = src[3 * i + 1];
    qz = src[3 * i + 2];
  }
  double m = INFINITY;
  for (int64_t j0 = 0; j0 < n; j0 += kDThreads) {
    const int64_t j = j0 + threadIdx.x;
    if (j < n) {
      tile[threadIdx.x][0] = P[3 * j];
      tile[threadIdx.x][1] = P[3 * j + 1];
      tile[threadIdx.x][2] = P[3 * j + 2];
    }
    __syncthreads();
    const int cnt = (int)min<int64_t>(kDThreads, n - j0);
    for (int k = 0; k < cnt; ++k) {
      const double dx = qx - tile[k][0], dy = qy - tile[k][1], dz = qz - tile[k][2];
      const double r2 = (dx * dx + dy * dy) + dz * dz;
      if (!(self && j0 + k == i)) m = fmin(m, r2);
    }
    __syncthreads();
  }
  if (i < nq) best[i] = m;
}

// out[0] = min, out[1] = max of v[0..n) (one block; min/max are exact in any order)
__global__ __launch_bounds__(kDThreads) void k_minmax(const double* __restrict__ v, int64_t n,
                                                      double* __restrict__ out) {
  __shared__ double lo[kDThreads], hi[kDThreads];
  double a = INFINITY, b = -INFINITY;
  for (int64_t i = threadIdx.x; i < n; i += kDThreads) {
    a = fmin(a, v[i]);
    b = fmax(b, v[i]);
  }
  lo[threadIdx.x] = a;
  hi[threadIdx.x] = b;
  __syncthreads();
  for (int w = kDThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      lo[threadIdx.x] = fmin(lo[threadIdx.x], lo[threadIdx.x + w]);
      hi[threadIdx.x] = fmax(hi[threadIdx.x], hi[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = lo[0];
    out[1] = hi[0];
  }
}

}  // namespace

void density_measures(const double* P, int64_t n, const double* samples, int64_t ns, double* q, double* hmax,
                      double* hfill, hipStream_t s) {
  double* best = talloc<double>(std::max<int64_t>(n, ns));
  double* mm = talloc<double>(4);
  double host[4] = {INFINITY, -INFINITY, INFINITY, -INFINITY};
  if (n >= 2) {
    hipLaunchKernelGGL(k_nearest, dim3((unsigned)ceil_div(n, kDThreads)), dim3(kDThreads), 0, s, P, n,
                       (const double*)nullptr, n, best);
    hipLaunchKernelGGL(k_minmax, dim3(1), dim3(kDThreads), 0, s, best, n, mm);
    RBF_HIP(hipGetLastError());
    RBF_HIP(hipMemcpyAsync(host, mm, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  }
  if (samples && ns > 0) {
    hipLaunchKernelGGL(k_nearest, dim3((unsigned)ceil_div(ns, kDThreads)), dim3(kDThreads), 0, s, P, n, samples, ns,
                       best);
    hipLaunchKernelGGL(k_minmax, dim3(1), dim3(kDThreads), 0, s, best, ns, mm + 2);
    RBF_HIP(hipGetLastError());
    RBF_HIP(hipMemcpyAsync(host + 2, mm + 2, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  }
  RBF_HIP(hipStreamSynchronize(s));
  temp_free(best);
  temp_free(mm);
  if (q) *q = n >= 2 ? 0.5 * std::sqrt(host[0]) : NAN;
  if (hmax) *hmax = n >= 2 ? std::sqrt(host[1]) : NAN;
  if (hfill) *hfill = (samples && ns > 0) ? std::sqrt(host[3]) : NAN;
}

}  // namespace rbf
