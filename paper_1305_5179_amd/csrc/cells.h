// Device helpers shared by the list builder (setup.hip) and the kernels that
// walk the coarse cells or the target groups directly (pairsum.hip,
// gridsum.hip).
#pragma once

#include "common.h"

namespace rbf {

// Lanes below this one whose bit is set in `mask`.
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Inclusive prefix sum over the wave's 64 lanes by DPP moves: shifts by 1,
// 2, 4 and 8 lanes within each 16-lane row (a lane shifted in from outside
// the row adds 0) give the row scans; then the last lane of rows 0 and 2 is
// added to rows 1 and 3 (row_bcast:15), and lane 31 to rows 2 and 3
// (row_bcast:31).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int32_t dpp_or_zero(int32_t v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROW_MASK, 0xf, false);
}
__device__ __forceinline__ int32_t wave_incl_scan(int32_t v) {
  v += dpp_or_zero<0x111, 0xf>(v);   // row_shr:1
  v += dpp_or_zero<0x112, 0xf>(v);   // row_shr:2
  v += dpp_or_zero<0x114, 0xf>(v);   // row_shr:4
  v += dpp_or_zero<0x118, 0xf>(v);   // row_shr:8
  v += dpp_or_zero<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp_or_zero<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
  return v;
}

// Bitwise OR over the wave's 64 lanes, the same in every lane: quads,
// half-rows and rows by DPP (quad_perm, row_half_mirror, row_mirror), then
// rows 0+1 and 2+3 (row_bcast:15) and all four (row_bcast:31) into lane 63,
// read back as a uniform value.
__device__ __forceinline__ uint32_t wave_or(uint32_t v) {
  const int32_t x = (int32_t)v;
  int32_t y = x | dpp_or_zero<0xB1, 0xf>(x);    // quad_perm [1,0,3,2]
  y |= dpp_or_zero<0x4E, 0xf>(y);               // quad_perm [2,3,0,1]
  y |= dpp_or_zero<0x141, 0xf>(y);              // row_half_mirror
  y |= dpp_or_zero<0x140, 0xf>(y);              // row_mirror
  y |= dpp_or_zero<0x142, 0xa>(y);              // row_bcast:15 into rows 1 and 3
  y |= dpp_or_zero<0x143, 0xc>(y);              // row_bcast:31 into rows 2 and 3
  return (uint32_t)__builtin_amdgcn_readlane(y, 63);
}

// Orders the LDS accesses of one wave around this point (the wave's lanes
// exchange data through LDS; no other wave takes part).
__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Block b of a launch runs on XCD b % 8; give every XCD a contiguous range of
// blocks so that neighbouring groups (which share sources) share an L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb) {
  const int64_t q = nb / 8, r = nb % 8, x = b % 8;
  const int64_t first = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
  return first + b / 8;
}

// The cube of coarse cells holding every coordinate within r_out of the
// anchor along each axis.  The relative pad keeps the float64 rounding of
// the cell index (here and in the sources' own cell keys, both
// floor((x - origin) / fine) up to a power of two) from dropping the cell of
// a source at the boundary.
__device__ __forceinline__ void cell_cube(const double ac[3], double r_out, const Lattice& lat, int cl[3], int cn[3]) {
  for (int d = 0; d < 3; ++d) {
    const double pad = r_out * (1.0 + 1e-9) + 1e-12 * (fabs(ac[d]) + fabs(lat.origin[d]) + r_out);
    const double a = floor((ac[d] - pad - lat.origin[d]) / lat.coarse);
    const double b = floor((ac[d] + pad - lat.origin[d]) / lat.coarse);
    const int ia = (int)fmax(0.0, fmin(a, (double)(lat.cdims[d] - 1)));
    const int ib = (int)fmax(0.0, fmin(b, (double)(lat.cdims[d] - 1)));
    cl[d] = ia;
    cn[d] = ib - ia + 1;
  }
}

// n / d for 0 <= n < 2^20 and 1 <= d, with inv_d = 1 / d in float32: the
// float quotient is within one of n / d (relative error below 2^-22), and
// one integer product corrects it.
__device__ __forceinline__ int div_small(int n, int d, float inv_d) {
  int q = (int)((float)n * inv_d);
  if (q * d > n)
    --q;
  else if ((q + 1) * d <= n)
    ++q;
  return q;
}

// The candidate sources of a group with anchor `ac`: every source of the
// occupied coarse cells of the cube [cl, cl + cn) whose box comes within
// r_out of the anchor.  The cells are examined one per lane, 64 at a time;
// the sources of the cells that remain are then taken 64 at a time across
// cell boundaries (cpre, cst and cwhole in LDS hold the start, first source
// and whole-cell flag of the occupied cells, 64 entries of the calling wave;
// a lane finds its cell from a count of the cells that start before the
// round and a mask of those that start within it).
// visit(valid, k, is_in, is_shell, whole, s) runs once per round of 64
// candidates, in the same order on every call: k is this lane's sorted source
// (when valid), is_in marks a source within r_in of the anchor (a whole cell
// within r_in counts without loading its sources: then `whole` is set and s
// is not loaded), is_shell one within r_out but not r_in, s the source's
// (unscaled) coordinates when loaded.  r_in2 < 0 marks no inner sources.
// Returns the number of candidates; CELLS_ONLY stops after the cell phase
// (the count alone).
template <bool CELLS_ONLY, class Visit>
__device__ __forceinline__ int64_t walk_candidates(const double ac[3], double r_in2, double r_out2, const int cl[3],
                                                   const int cn[3], const double4* __restrict__ xs,
                                                   const int32_t* __restrict__ cstart,
                                                   const int32_t* __restrict__ ccount,
                                                   const int32_t* __restrict__ cmap, const Lattice& lat,
                                                   int32_t* cpre, int32_t* cst, uint8_t* cwhole, Visit&& visit) {
  const int lane = threadIdx.x & 63;
  const int ncube = cn[0] * cn[1] * cn[2];
  const bool small = ncube < (1 << 20);
  const float inv0 = 1.0f / (float)cn[0], inv1 = 1.0f / (float)cn[1];
  int64_t cand = 0;
  for (int c0 = 0; c0 < ncube; c0 += kWave) {
    // one cell of the cube per lane: occupied? how far from the anchor?
    const int ci = c0 + lane;
    int32_t cid = -1;
    bool whole = false;
    if (ci < ncube) {
      int cx, cy, cz;
      if (small) {
        const int t = div_small(ci, cn[0], inv0);
        cz = div_small(t, cn[1], inv1);
        cx = cl[0] + (ci - t * cn[0]);
        cy = cl[1] + (t - cz * cn[1]);
        cz += cl[2];
      } else {
        cx = cl[0] + ci % cn[0];
        cy = cl[1] + (ci / cn[0]) % cn[1];
        cz = cl[2] + ci / (cn[0] * cn[1]);
      }
      cid = cmap[(int64_t)cx + (int64_t)lat.cdims[0] * ((int64_t)cy + (int64_t)lat.cdims[1] * cz)];
      if (cid >= 0) {
        const int cc[3] = {cx, cy, cz};
        double dmin2 = 0.0, dmax2 = 0.0;
        for (int d = 0; d < 3; ++d) {
          const double b0 = lat.origin[d] + cc[d] * lat.coarse, b1 = b0 + lat.coarse;
          const double gap = fmax(0.0, fmax(b0 - ac[d], ac[d] - b1));
          const double far = fmax(fabs(ac[d] - b0), fabs(ac[d] - b1));
          dmin2 += gap * gap;
          dmax2 += far * far;
        }
        if (dmin2 > r_out2 * (1.0 + 1e-9)) cid = -1;
        whole = dmax2 * (1.0 + 1e-9) <= r_in2;
      }
    }
    // the occupied cells of this block, compacted in lane order, with the
    // exclusive prefix of their source counts
    const int32_t ct = cid >= 0 ? ccount[cid] : 0;
    const int32_t st = cid >= 0 ? cstart[cid] : 0;
    const bool occ = ct > 0;   // (empty cells would break the search below)
    const uint64_t sel = ballot(occ);
    const int nocc = __popcll(sel);
    const int32_t incl = wave_incl_scan(ct);
    // (read-lane: a uniform value, so the trip count below is uniform too)
    const int32_t total = __builtin_amdgcn_readlane(incl, kWave - 1);
    cand += total;
    if (CELLS_ONLY) continue;
    wave_sync_lds();
    if (occ) {
      const int pos = lanes_below(sel);
      cpre[pos] = incl - ct;
      cst[pos] = st;
      cwhole[pos] = whole ? 1 : 0;
    }
    wave_sync_lds();
    const int32_t start = incl - ct;   // of this lane's cell, when occupied
    const uint64_t below_lane = lane == kWave - 1 ? ~0ull : (2ull << lane) - 1;
    for (int32_t b0 = 0; b0 < total; b0 += kWave) {
      const int32_t f = b0 + lane;
      const bool valid = f < total;
      // the cell of flattened source f is the last occupied cell that starts
      // at or before f (the starts rise with the compacted index): its index
      // is the number of cells starting before b0, plus those starting in
      // [b0, f], minus one
      const int32_t r = start - b0;
      const int before = __popcll(ballot(occ && r < 0));
      const uint32_t lo = wave_or(occ && r >= 0 && r < 32 ? 1u << r : 0u);
      const uint32_t hi = wave_or(occ && r >= 32 && r < 64 ? 1u << (r - 32) : 0u);
      const uint64_t starts = ((uint64_t)hi << 32) | lo;
      const int j = min(max(before + __popcll(starts & below_lane) - 1, 0), nocc - 1);
      const uint32_t k = (uint32_t)(cst[j] + (f - cpre[j]));
      bool is_in = false, is_shell = false;
      const bool whole = valid && cwhole[j];
      double4 s = make_double4(0.0, 0.0, 0.0, 0.0);
      if (valid) {
        if (whole) {
          is_in = true;
        } else {
          s = xs[k];
          const double dx = s.x - ac[0], dy = s.y - ac[1], dz = s.z - ac[2];
          const double d2 = (dx * dx + dy * dy) + dz * dz;
          is_in = d2 <= r_in2;
          is_shell = !is_in && d2 <= r_out2;
        }
      }
      visit(valid, k, is_in, is_shell, whole, s);
    }
  }
  return cand;
}

}  // namespace rbf
