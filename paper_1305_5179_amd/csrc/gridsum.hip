// Grid evaluation without source lists: the sum of eq. matxvet at the nodes
// of a regular grid, truncated as in Sec. III.A, float32 terms.
//
// A grid's lists are used once, so building them (classify every candidate,
// write the list and the masks, read them back in the pair kernel) costs
// more than the sums themselves.  Here one wave owns a brick of 4 x 2 x 2
// nodes and walks the brick's candidate sources directly, with the list
// builder's classification: sources within r_in of the brick's anchor are
// inside the cutoff of every node, sources beyond r_out of none, and the
// shell in between gets the exact float64 test of every node.  Kept sources
// are queued in LDS and summed 64 at a time, one source per lane.
//
// Terms (lane = source s, 16 nodes n = c + h (i, j, k) of the brick, c its
// corner node, coordinates scaled by sqrt(k) so that phi = exp2(-d)):
//   d = |u|^2 - 2 u.Hn + |Hn|^2,   u = s - c,
//   phi_n = 2^{-|u|^2} X^i Y^j Z^k 2^{-|Hn|^2},   X = 2^{2 h_x u_x} (and y, z),
// so a source costs four exponentials and a few products for its 16 terms;
// the node factor 2^{-|Hn|^2} multiplies the node's sum once.  The exact
// truncation test takes the node coordinates as the grid defines them and
// r^2 = (dx dx + dy dy) + dz dz in float64, and shares the squared axis
// differences between the nodes of a row (four x values, two y, two z).
// The per-lane sums of each node are added across the wave through LDS in a
// fixed order, so the result does not depend on timing.
#include <type_traits>

#include "cells.h"

namespace rbf {

namespace {

constexpr int kBrickWaves = 4;
constexpr int kRedPitch = kGroup + 1;   // LDS row pitch of the cross-lane sums (odd: no bank conflicts)

struct BrickArgs {
  GridDesc gd;
  const int64_t* ids;    // brick ids (null: brick g is id g)
  int64_t nb;            // bricks
  const double4* xs;     // unscaled sorted sources
  const double* w;       // sorted weights
  const int32_t* cstart;
  const int32_t* ccount;
  const int32_t* cmap;
  Lattice lat;
  double rc, rc2, sqrt_k;
  double hk[3];          // scaled grid spacing h sqrt(k) per axis
  float* out;
  int64_t* useful;       // per brick: pairs inside the cutoff (with `examined`, optional)
  int64_t* examined;     // per brick: queued sources x 16
};

struct BrickNodes {
  double x[4], y[2], z[2];   // node coordinates as the grid defines them: o + i h
  uint32_t vmask;            // nodes inside the grid
  int nvalid;
  int64_t i0, j0, k0;        // first node of the brick
};

__device__ __forceinline__ BrickNodes brick_nodes(const GridDesc& gd, int64_t b) {
  BrickNodes bn;
  const int64_t bx = b % gd.nb[0], by = (b / gd.nb[0]) % gd.nb[1], bz = b / (gd.nb[0] * gd.nb[1]);
  bn.i0 = 4 * bx;
  bn.j0 = 2 * by;
  bn.k0 = 2 * bz;
  for (int i = 0; i < 4; ++i) bn.x[i] = gd.o[0] + (double)(bn.i0 + i) * gd.h[0];
  for (int j = 0; j < 2; ++j) {
    bn.y[j] = gd.o[1] + (double)(bn.j0 + j) * gd.h[1];
    bn.z[j] = gd.o[2] + (double)(bn.k0 + j) * gd.h[2];
  }
  bn.vmask = 0u;
  bn.nvalid = 0;
  for (int l = 0; l < kGroup; ++l) {
    if (bn.i0 + (l & 3) < gd.n[0] && bn.j0 + ((l >> 2) & 1) < gd.n[1] && bn.k0 + (l >> 3) < gd.n[2]) {
      bn.vmask |= 1u << l;
      ++bn.nvalid;
    }
  }
  return bn;
}

// Terms of `cnt` (<= 64) queued sources, one per lane, added to the lane's 16
// node sums.  SHELL: each term only where the exact test puts the pair
// inside the cutoff.  COUNT: add the pairs inside the cutoff to `use`.
template <bool SHELL, bool COUNT>
__device__ __forceinline__ void brick_batch(const BrickArgs& a, const BrickNodes& bn, const uint32_t* q, int cnt,
                                            float acc[kGroup], int64_t& use) {
  const int lane = threadIdx.x & 63;
  const bool valid = lane < cnt;
  // lanes without a source take the corner node with weight 0: every term 0
  double4 s = make_double4(bn.x[0], bn.y[0], bn.z[0], 0.0);
  double wk = 0.0;
  if (valid) {
    const uint32_t k = q[lane];
    s = a.xs[k];
    wk = a.w[k];
  }
  const double dx = (s.x - bn.x[0]) * a.sqrt_k, dy = (s.y - bn.y[0]) * a.sqrt_k, dz = (s.z - bn.z[0]) * a.sqrt_k;
  const double uq = fma(dx, dx, fma(dy, dy, dz * dz));
  // every exponent is formed in float64 and rounded once
  const float W = (float)wk * __builtin_amdgcn_exp2f(-(float)uq);
  const float X = __builtin_amdgcn_exp2f((float)(2.0 * a.hk[0] * dx));
  const float Y = __builtin_amdgcn_exp2f((float)(2.0 * a.hk[1] * dy));
  const float Z = __builtin_amdgcn_exp2f((float)(2.0 * a.hk[2] * dz));
  float A[4];
  A[0] = W;
  A[1] = A[0] * X;
  A[2] = A[1] * X;
  A[3] = A[2] * X;
  if constexpr (!SHELL) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float B = A[i] * Y;
      acc[i] += A[i];
      acc[i + 4] += B;
      acc[i + 8] = __builtin_fmaf(A[i], Z, acc[i + 8]);
      acc[i + 12] = __builtin_fmaf(B, Z, acc[i + 12]);
    }
    if (COUNT) use += (int64_t)cnt * bn.nvalid;
  } else {
    // the exact test, r^2 = (dx dx + dy dy) + dz dz with d = node - source
    double ex2[4], ey2[2], ez2[2];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double e = bn.x[i] - s.x;
      ex2[i] = e * e;
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const double ey = bn.y[j] - s.y, ez = bn.z[j] - s.z;
      ey2[j] = ey * ey;
      ez2[j] = ez * ez;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float B = A[i] * Y;
      const float T[4] = {A[i], B, A[i] * Z, B * Z};
#pragma unroll
      for (int jk = 0; jk < 4; ++jk) {
        const int l = i + 4 * jk;
        const double r2 = (ex2[i] + ey2[jk & 1]) + ez2[jk >> 1];
        const bool in = valid && r2 <= a.rc2;
        acc[l] += in ? T[jk] : 0.0f;
        if (COUNT) use += __popcll(ballot(in) & (((bn.vmask >> l) & 1u) ? ~0ull : 0ull));
      }
    }
  }
}

template <bool COUNT>
__global__ __launch_bounds__(kBrickWaves * kWave, 5) void k_brick_sum_f32(BrickArgs a) {
  // per wave: the two source queues and the cell prefix of the walk, later
  // the cross-lane sums
  __shared__ uint32_t lds_s[kBrickWaves][kWave * kRedPitch];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint32_t* const lds = lds_s[wave];
  const int lane = threadIdx.x & 63;
  const int64_t g = xcd_remap(blockIdx.x, gridDim.x) * kBrickWaves + wave;
  if (g >= a.nb) return;
  const int64_t b = a.ids ? a.ids[g] : g;
  const BrickNodes bn = brick_nodes(a.gd, b);
  int64_t use = 0, queued = 0;
  float acc[kGroup];
#pragma unroll
  for (int l = 0; l < kGroup; ++l) acc[l] = 0.0f;
  if (bn.nvalid > 0) {
    // anchor (centre of the valid nodes' box) and radius, as the list builder
    // takes them
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int l = 0; l < kGroup; ++l) {
      if ((bn.vmask >> l) & 1u) {
        const double t[3] = {bn.x[l & 3], bn.y[(l >> 2) & 1], bn.z[l >> 3]};
        for (int d = 0; d < 3; ++d) {
          lo[d] = fmin(lo[d], t[d]);
          hi[d] = fmax(hi[d], t[d]);
        }
      }
    }
    const double ac[3] = {0.5 * (lo[0] + hi[0]), 0.5 * (lo[1] + hi[1]), 0.5 * (lo[2] + hi[2])};
    double rad = 0.0;
    for (int l = 0; l < kGroup; ++l) {
      if ((bn.vmask >> l) & 1u) {
        const double ex = bn.x[l & 3] - ac[0], ey = bn.y[(l >> 2) & 1] - ac[1], ez = bn.z[l >> 3] - ac[2];
        rad = fmax(rad, sqrt((ex * ex + ey * ey) + ez * ez));
      }
    }
    const double r_in = a.rc * (1.0 - 1e-12) - rad;   // |s - a| <= r_in: inside for every node
    const double r_out = a.rc * (1.0 + 1e-12) + rad;  // |s - a| >  r_out: inside for none
    const double r_in2 = r_in > 0.0 ? r_in * r_in : -1.0;
    const double r_out2 = r_out * r_out;
    int cl[3], cn[3];
    cell_cube(ac, r_out, a.lat, cl, cn);
    uint32_t* qin = lds;
    uint32_t* qsh = lds + 2 * kWave;
    int32_t* cpre = reinterpret_cast<int32_t*>(lds + 4 * kWave);
    int32_t* cst = reinterpret_cast<int32_t*>(lds + 5 * kWave);
    uint8_t* cwhole = reinterpret_cast<uint8_t*>(lds + 6 * kWave);
    int nin = 0, nsh = 0;
    // take 64 queued sources from the front of a queue and move the rest down
    auto drain = [&](uint32_t* qq, int& nq, auto shell) {
      wave_sync_lds();
      brick_batch<decltype(shell)::value, COUNT>(a, bn, qq, kWave, acc, use);
      const uint32_t rest = lane + kWave < nq ? qq[kWave + lane] : 0u;
      wave_sync_lds();
      if (lane + kWave < nq) qq[lane] = rest;
      nq -= kWave;
      queued += kWave;
      wave_sync_lds();
    };
    walk_candidates<false>(ac, r_in2, r_out2, cl, cn, a.xs, a.cstart, a.ccount, a.cmap, a.lat, cpre, cst, cwhole,
                           [&](bool, uint32_t k, bool is_in, bool is_shell) {
                             const uint64_t mi = ballot(is_in), ms = ballot(is_shell);
                             if (is_in) qin[nin + lanes_below(mi)] = k;
                             if (is_shell) qsh[nsh + lanes_below(ms)] = k;
                             nin += __popcll(mi);
                             nsh += __popcll(ms);
                             if (nin >= kWave) drain(qin, nin, std::false_type{});
                             if (nsh >= kWave) drain(qsh, nsh, std::true_type{});
                           });
    wave_sync_lds();
    if (nin > 0) brick_batch<false, COUNT>(a, bn, qin, nin, acc, use);
    if (nsh > 0) brick_batch<true, COUNT>(a, bn, qsh, nsh, acc, use);
    queued += nin + nsh;
  }
  // node sums across the wave: lane L adds node L % 16 over the 16 lanes of
  // part L / 16, then the four parts are added
  float* red = reinterpret_cast<float*>(lds);
  wave_sync_lds();
#pragma unroll
  for (int l = 0; l < kGroup; ++l) red[lane * kRedPitch + l] = acc[l];
  wave_sync_lds();
  const int node = lane & 15, part = lane >> 4;
  float v = 0.0f;
#pragma unroll
  for (int t = 0; t < 16; ++t) v += red[(part * 16 + t) * kRedPitch + node];
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  if (lane < kGroup && ((bn.vmask >> lane) & 1u)) {
    const int i = lane & 3, j = (lane >> 2) & 1, k = lane >> 3;
    const double hx = a.hk[0] * i, hy = a.hk[1] * j, hz = a.hk[2] * k;
    const double nf = exp2(-((hx * hx + hy * hy) + hz * hz));
    a.out[(bn.i0 + i) + a.gd.n[0] * ((bn.j0 + j) + a.gd.n[1] * (bn.k0 + k))] = (float)((double)v * nf);
  }
  if (COUNT && lane == 0) {
    a.useful[g] = use;
    a.examined[g] = queued * kGroup;
  }
}

}  // namespace

// The product form's exponents stay in range, and its rounding at a few
// float32 units of the term, when every queued source lies within
// umax = sqrt(k) (r_c + brick diagonal) of the corner node (scaled units) and
// umax^2 + 2 umax (3 hk_x + hk_y + hk_z) <= 64.
bool brick_sum_applies(const Ctx& c, const rbf_grid& g) {
  if (!std::isfinite(c.rc2) || !c.cell_map) return false;
  const double diag = std::sqrt((3.0 * g.h[0]) * (3.0 * g.h[0]) + g.h[1] * g.h[1] + g.h[2] * g.h[2]);
  const double umax = c.sqrt_k * (c.cutoff + diag) * (1.0 + 1e-6);
  const double hsum = c.sqrt_k * (3.0 * g.h[0] + g.h[1] + g.h[2]);
  return umax * umax + 2.0 * umax * hsum <= 64.0;
}

void brick_sum_f32(const Ctx& c, const rbf_grid& g, const int64_t* ids, int64_t nact, const double* w_sorted,
                   float* out, int64_t* useful, int64_t* examined, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
  if (nact <= 0) return;
  BrickArgs a;
  a.gd = grid_desc(g);
  a.ids = ids;
  a.nb = nact;
  a.xs = c.xs;
  a.w = w_sorted;
  a.cstart = c.cell_start;
  a.ccount = c.cell_count;
  a.cmap = c.cell_map;
  a.lat = c.lat;
  a.rc = c.cutoff;
  a.rc2 = c.rc2;
  a.sqrt_k = c.sqrt_k;
  for (int d = 0; d < 3; ++d) a.hk[d] = g.h[d] * c.sqrt_k;
  a.out = out;
  a.useful = useful;
  a.examined = examined;
  const int64_t nb = ceil_div(nact, kBrickWaves);
  if (useful && examined)
    hipExtLaunchKernelGGL(k_brick_sum_f32<true>, dim3((unsigned)nb), dim3(kBrickWaves * kWave), 0, s, t0, t1, 0, a);
  else
    hipExtLaunchKernelGGL(k_brick_sum_f32<false>, dim3((unsigned)nb), dim3(kBrickWaves * kWave), 0, s, t0, t1, 0, a);
  RBF_HIP(hipGetLastError());
}

}  // namespace rbf
