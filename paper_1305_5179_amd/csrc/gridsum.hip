// Grid evaluation without source lists: the sum of eq. matxvet at the nodes
// of a regular grid, truncated as in Sec. III.A, float32 terms.
//
// A grid's lists are used once, so building them (classify every candidate,
// write the list and the masks, read them back in the pair kernel) costs
// more than the sums themselves.  Here one wave owns a tile of 4 x 4 x 2
// nodes, two bricks of 4 x 2 x 2 (one along x and z, two along y), walks
// the tile's candidate sources once and classifies each for every brick with
// the list builder's rule: sources within r_in of the brick's anchor are
// inside the cutoff of every node, sources beyond r_out of none, and the
// shell in between gets the exact float64 test of every node.  Kept sources
// go to the brick's two LDS queues and are summed 64 at a time, one source
// per lane.  Sharing the walk (cell cube, candidate loads) between bricks is
// the point of the tile: the walk cost more than the sums.
//
// Terms (lane = source s, 16 nodes n = c + h (i, j, k) of a brick, c its
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

// setup.hip
int64_t scan_ws_elems(int64_t n);
void scan_exclusive_i64_ws(const int64_t* in, int64_t* out, int64_t n, int64_t* ws, hipStream_t s);

namespace {

constexpr int kTileWaves = 4;          // tiles (waves) per workgroup
constexpr int kTileY = 2, kTileZ = 1;  // bricks of a tile along y and z (one along x)
constexpr int kTileBricks = kTileY * kTileZ;
constexpr int kRedPitch = kGroup + 1;  // LDS row pitch of the cross-lane sums (odd: no bank conflicts)
constexpr int kQueue = 2 * kWave;      // entries of a source queue (drained at 64)
constexpr int kThreadsT = 256;

struct TileArgs {
  GridDesc gd;
  const int64_t* tiles;  // tile ids t = tx + nt0 (ty + nt1 tz)
  const int64_t* masks;  // per tile: bit b (b = dy + kTileY dz) for each brick to evaluate
  int64_t nt;            // tiles in the list
  int64_t nt0, nt1;      // tiles along x and y
  const double4* xs;     // unscaled sorted sources
  const double* w;       // sorted weights
  const int32_t* cstart;
  const int32_t* ccount;
  const int32_t* cmap;
  Lattice lat;
  double rc, rc2, sqrt_k;
  double hk[3];          // scaled grid spacing h sqrt(k) per axis
  float* out;
  int64_t* useful;       // per tile: pairs inside the cutoff (with `examined`, optional)
  int64_t* examined;     // per tile: queued sources x 16
};

// One brick of a tile (uniform).  Its anchor is the centre of its whole
// 4 x 2 x 2 box of nodes (also where the grid ends: nodes beyond it are never
// stored, and classifying against the whole box is conservative for the
// nodes that exist), so every brick has the same radius.
struct Brick {
  double y0, z0;         // its first node along y and z
  double ay, az;         // anchor along y and z (x: the tile's)
  uint32_t vmask;        // nodes inside the grid (bit i + 4 j + 8 k); 0: not evaluated
  int nvalid;
  int64_t j0, k0;        // first node along y and z
};

// Radius of a box of nodes with sides (e0, e1, e2) around its centre: the
// half diagonal, padded for the rounding of the centre and of the nodes.
__device__ __forceinline__ double box_radius(double e0, double e1, double e2) {
  return sqrt((e0 * e0 + e1 * e1) + e2 * e2) * (0.5 + 1e-14);
}

// Terms of `cnt` (<= 64) queued sources, one per lane, added to the lane's 16
// node sums of one brick.  SHELL: each term only where the exact test puts
// the pair inside the cutoff.  COUNT: add the pairs inside the cutoff to `use`.
template <bool SHELL, bool COUNT>
__device__ __forceinline__ void brick_batch(const TileArgs& a, const double (&x)[4], const Brick& bk,
                                            const uint32_t* q, int cnt, float acc[kGroup], int64_t& use) {
  const int lane = threadIdx.x & 63;
  const bool valid = lane < cnt;
  // lanes without a source take the corner node with weight 0: every term 0
  double4 s = make_double4(x[0], bk.y0, bk.z0, 0.0);
  double wk = 0.0;
  if (valid) {
    const uint32_t k = q[lane];
    s = a.xs[k];
    wk = a.w[k];
  }
  const double dx = (s.x - x[0]) * a.sqrt_k, dy = (s.y - bk.y0) * a.sqrt_k, dz = (s.z - bk.z0) * a.sqrt_k;
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
    if (COUNT) use += (int64_t)cnt * bk.nvalid;
  } else {
    // the exact test, r^2 = (dx dx + dy dy) + dz dz with d = node - source
    double ex2[4], ey2[2], ez2[2];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double e = x[i] - s.x;
      ex2[i] = e * e;
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      // the node coordinates as the grid defines them: o + index h
      const double ey = (a.gd.o[1] + (double)(bk.j0 + j) * a.gd.h[1]) - s.y;
      const double ez = (a.gd.o[2] + (double)(bk.k0 + j) * a.gd.h[2]) - s.z;
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
        if (COUNT) use += __popcll(ballot(in) & (((bk.vmask >> l) & 1u) ? ~0ull : 0ull));
      }
    }
  }
}

// The 16 node sums of a brick added across the wave (lane L adds node L % 16
// over the 16 lanes of part L / 16, then the four parts are added) and
// stored with the node factor.
__device__ __forceinline__ void brick_store(const TileArgs& a, const Brick& bk, int64_t i0, const float acc[kGroup],
                                            float* red) {
  const int lane = threadIdx.x & 63;
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
  if (lane < kGroup && ((bk.vmask >> lane) & 1u)) {
    const int i = lane & 3, j = (lane >> 2) & 1, k = lane >> 3;
    const double hx = a.hk[0] * i, hy = a.hk[1] * j, hz = a.hk[2] * k;
    const double nf = exp2(-((hx * hx + hy * hy) + hz * hz));
    a.out[(i0 + i) + a.gd.n[0] * ((bk.j0 + j) + a.gd.n[1] * (bk.k0 + k))] = (float)((double)v * nf);
  }
}

template <bool COUNT>
__global__ __launch_bounds__(kTileWaves * kWave, 4) void k_brick_sum_f32(TileArgs a) {
  // per wave: two source queues per brick and the cell prefix of the walk,
  // later (the same words) the cross-lane sums
  constexpr int kQWords = 2 * kTileBricks * kQueue;
  constexpr int kWaveWords = kQWords + 3 * kWave > kWave * kRedPitch ? kQWords + 3 * kWave : kWave * kRedPitch;
  static_assert(kWaveWords >= kWave * kRedPitch && kWaveWords >= kQWords + 3 * kWave,
                "a wave's LDS words hold its queues and walk prefix, and later its cross-lane sums");
  __shared__ uint32_t lds_s[kTileWaves][kWaveWords];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint32_t* const lds = lds_s[wave];
  const int lane = threadIdx.x & 63;
  const int64_t g = xcd_remap(blockIdx.x, gridDim.x) * kTileWaves + wave;
  if (g >= a.nt) return;
  const GridDesc& gd = a.gd;
  const int64_t t = a.tiles[g];
  const uint32_t tmask = (uint32_t)a.masks[g];
  const int64_t tx = t % a.nt0, ty = (t / a.nt0) % a.nt1, tz = t / (a.nt0 * a.nt1);
  // the tile's nodes: 4 along x (shared by its bricks), 2 per brick along y and z
  const int64_t i0 = 4 * tx, j0 = 2 * kTileY * ty, k0 = 2 * kTileZ * tz;
  const int nx = (int)min<int64_t>(4, gd.n[0] - i0);
  const int ny = (int)min<int64_t>(2 * kTileY, gd.n[1] - j0);
  const int nz = (int)min<int64_t>(2 * kTileZ, gd.n[2] - k0);
  double x[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) x[i] = gd.o[0] + (double)(i0 + i) * gd.h[0];
  const double ax = gd.o[0] + ((double)i0 + 1.5) * gd.h[0];
  Brick bk[kTileBricks];
#pragma unroll
  for (int b = 0; b < kTileBricks; ++b) {
    const int dyb = b % kTileY, dzb = b / kTileY;
    Brick& r = bk[b];
    r.j0 = j0 + 2 * dyb;
    r.k0 = k0 + 2 * dzb;
    r.y0 = gd.o[1] + (double)r.j0 * gd.h[1];
    r.z0 = gd.o[2] + (double)r.k0 * gd.h[2];
    r.ay = gd.o[1] + ((double)r.j0 + 0.5) * gd.h[1];
    r.az = gd.o[2] + ((double)r.k0 + 0.5) * gd.h[2];
    const int by = max(0, min(2, ny - 2 * dyb)), bz = max(0, min(2, nz - 2 * dzb));
    r.nvalid = ((tmask >> b) & 1u) ? nx * by * bz : 0;
    r.vmask = 0u;
    if (r.nvalid > 0)
      for (int k = 0; k < bz; ++k)
        for (int j = 0; j < by; ++j) r.vmask |= ((1u << nx) - 1u) << (4 * j + 8 * k);
  }
  // every brick's radius (whole 4 x 2 x 2 box) and the tile's (its whole box)
  const double rad = box_radius(3.0 * gd.h[0], gd.h[1], gd.h[2]);
  const double r_in = a.rc * (1.0 - 1e-12) - rad, r_out = a.rc * (1.0 + 1e-12) + rad;
  const double r_in2 = r_in > 0.0 ? r_in * r_in : -1.0, r_out2 = r_out * r_out;
  const double ac[3] = {ax, gd.o[1] + ((double)j0 + (kTileY - 0.5)) * gd.h[1],
                        gd.o[2] + ((double)k0 + (kTileZ - 0.5)) * gd.h[2]};
  const double rad_t = box_radius(3.0 * gd.h[0], (2 * kTileY - 1) * gd.h[1], (2 * kTileZ - 1) * gd.h[2]);
  const double rt_in = a.rc * (1.0 - 1e-12) - rad_t, rt_out = a.rc * (1.0 + 1e-12) + rad_t;
  const double rt_in2 = rt_in > 0.0 ? rt_in * rt_in : -1.0, rt_out2 = rt_out * rt_out;

  int64_t use = 0, queued = 0;
  float acc[kTileBricks][kGroup];
#pragma unroll
  for (int b = 0; b < kTileBricks; ++b)
#pragma unroll
    for (int l = 0; l < kGroup; ++l) acc[b][l] = 0.0f;
  int nin[kTileBricks] = {}, nsh[kTileBricks] = {};
  uint32_t* const qbase = lds;
  int32_t* cpre = reinterpret_cast<int32_t*>(lds + kQWords);
  int32_t* cst = reinterpret_cast<int32_t*>(lds + kQWords + kWave);
  uint8_t* cwhole = reinterpret_cast<uint8_t*>(lds + kQWords + 2 * kWave);
  // take 64 queued sources from the front of a queue and move the rest down
  auto drain = [&](uint32_t* qq, int& nq, const Brick& r, float (&ab)[kGroup], auto shell) {
    wave_sync_lds();
    brick_batch<decltype(shell)::value, COUNT>(a, x, r, qq, kWave, ab, use);
    const uint32_t rest = lane + kWave < nq ? qq[kWave + lane] : 0u;
    wave_sync_lds();
    if (lane + kWave < nq) qq[lane] = rest;
    nq -= kWave;
    queued += kWave;
    wave_sync_lds();
  };
  int cl[3], cn[3];
  cell_cube(ac, rt_out, a.lat, cl, cn);
  walk_candidates<false>(
      ac, rt_in2, rt_out2, cl, cn, a.xs, a.cstart, a.ccount, a.cmap, a.lat, cpre, cst, cwhole,
      [&](bool valid, uint32_t k, bool, bool, bool whole, const double4& s) {
        const double ex = s.x - ax;
        const double ex2 = ex * ex;
#pragma unroll
        for (int b = 0; b < kTileBricks; ++b) {
          if (bk[b].nvalid == 0) continue;
          const double ey = s.y - bk[b].ay, ez = s.z - bk[b].az;
          const double d2 = (ex2 + ey * ey) + ez * ez;
          const bool is_in = valid && (whole || d2 <= r_in2);
          const bool is_sh = valid && !is_in && d2 <= r_out2;
          const uint64_t mi = ballot(is_in), ms = ballot(is_sh);
          uint32_t* qin = qbase + (2 * b) * kQueue;
          uint32_t* qsh = qbase + (2 * b + 1) * kQueue;
          if (is_in) qin[nin[b] + lanes_below(mi)] = k;
          if (is_sh) qsh[nsh[b] + lanes_below(ms)] = k;
          nin[b] += __popcll(mi);
          nsh[b] += __popcll(ms);
          if (nin[b] >= kWave) drain(qin, nin[b], bk[b], acc[b], std::false_type{});
          if (nsh[b] >= kWave) drain(qsh, nsh[b], bk[b], acc[b], std::true_type{});
        }
      });
  wave_sync_lds();
#pragma unroll
  for (int b = 0; b < kTileBricks; ++b) {
    if (bk[b].nvalid == 0) continue;
    if (nin[b] > 0) brick_batch<false, COUNT>(a, x, bk[b], qbase + (2 * b) * kQueue, nin[b], acc[b], use);
    if (nsh[b] > 0) brick_batch<true, COUNT>(a, x, bk[b], qbase + (2 * b + 1) * kQueue, nsh[b], acc[b], use);
    queued += nin[b] + nsh[b];
  }
  // the sums of every evaluated brick (the queues' LDS is free now)
  float* red = reinterpret_cast<float*>(lds);
#pragma unroll
  for (int b = 0; b < kTileBricks; ++b)
    if (bk[b].nvalid > 0) brick_store(a, bk[b], i0, acc[b], red);
  if (COUNT && lane == 0) {
    a.useful[g] = use;
    a.examined[g] = queued * kGroup;
  }
}

// Launch order of the tiles.  The tiles are listed block by block, blocks of
// 16 x 16 x 16 tiles in raster order and the tiles of a block in raster
// order, so that the waves resident on one XCD at a time (about 512, about
// the support tiles of one block near a surface) cover a compact part of the
// grid and share the sources they gather in that XCD's L2 (in plain raster
// order they cover a thin slab).  A slot is a position in that order over
// the grid's tiles padded to whole blocks.
constexpr int kSlotBlock = 16;
struct SlotSpace {
  int64_t nt0, nt1, nt2;   // tiles per axis
  int64_t b0, b1;          // blocks along x and y
  int64_t n;               // slots (whole blocks)
};
SlotSpace slot_space(int64_t nt0, int64_t nt1, int64_t nt2) {
  SlotSpace S;
  S.nt0 = nt0;
  S.nt1 = nt1;
  S.nt2 = nt2;
  S.b0 = ceil_div(nt0, (int64_t)kSlotBlock);
  S.b1 = ceil_div(nt1, (int64_t)kSlotBlock);
  S.n = S.b0 * S.b1 * ceil_div(nt2, (int64_t)kSlotBlock) * (kSlotBlock * kSlotBlock * kSlotBlock);
  return S;
}
__device__ __forceinline__ int64_t tile_slot(const SlotSpace& S, int64_t tx, int64_t ty, int64_t tz) {
  constexpr int B = kSlotBlock;
  const int64_t blk = tx / B + S.b0 * (ty / B + S.b1 * (tz / B));
  return blk * (B * B * B) + tx % B + B * (ty % B + B * (tz % B));
}
// The tile of slot p; false for the padding slots.
__device__ __forceinline__ bool slot_tile(const SlotSpace& S, int64_t p, int64_t& tx, int64_t& ty, int64_t& tz) {
  constexpr int B = kSlotBlock;
  const int64_t blk = p / (B * B * B), w = p % (B * B * B);
  tx = B * (blk % S.b0) + w % B;
  ty = B * ((blk / S.b0) % S.b1) + (w / B) % B;
  tz = B * (blk / (S.b0 * S.b1)) + w / (B * B);
  return tx < S.nt0 && ty < S.nt1 && tz < S.nt2;
}

// Tiles of the listed bricks: tmask[slot of the tile] |= bit of the brick.
__global__ void k_tile_mark(const int64_t* __restrict__ ids, int64_t nact, GridDesc gd, SlotSpace S,
                            unsigned long long* __restrict__ tmask) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= nact) return;
  const int64_t b = ids[e];
  const int64_t bx = b % gd.nb[0], by = (b / gd.nb[0]) % gd.nb[1], bz = b / (gd.nb[0] * gd.nb[1]);
  atomicOr(tmask + tile_slot(S, bx, by / kTileY, bz / kTileZ), 1ull << (by % kTileY + kTileY * (bz % kTileZ)));
}

// The tile masks of a brick marking (mark[b] != 0: brick b belongs), by
// slot, and flag[p] = 1 for the slots of tiles with a marked brick.
__global__ void k_tiles_from_marks(const int64_t* __restrict__ mark, GridDesc gd, SlotSpace S,
                                   int64_t* __restrict__ tmask, int64_t* __restrict__ flag) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= S.n) return;
  int64_t tx, ty, tz, m = 0;
  if (slot_tile(S, p, tx, ty, tz)) {
    for (int b = 0; b < kTileBricks; ++b) {
      const int64_t by = kTileY * ty + b % kTileY, bz = kTileZ * tz + b / kTileY;
      if (by < gd.nb[1] && bz < gd.nb[2] && mark[tx + gd.nb[0] * (by + gd.nb[1] * bz)]) m |= int64_t(1) << b;
    }
  }
  tmask[p] = m;
  flag[p] = m != 0 ? 1 : 0;
}

__global__ void k_fill_zero(int64_t* __restrict__ p, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

__global__ void k_nonzero(const int64_t* __restrict__ v, int64_t n, int64_t* __restrict__ flag) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) flag[i] = v[i] != 0 ? 1 : 0;
}

// The marked slots in slot order: tiles[] their tiles' raster indices
// (tx + nt0 (ty + nt1 tz)), masks[] their brick masks.
__global__ void k_tile_compact(const int64_t* __restrict__ tmask, const int64_t* __restrict__ pos, SlotSpace S,
                               int64_t* __restrict__ tiles, int64_t* __restrict__ masks) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= S.n || tmask[p] == 0) return;
  int64_t tx, ty, tz;
  slot_tile(S, p, tx, ty, tz);
  tiles[pos[p]] = tx + S.nt0 * (ty + S.nt1 * tz);
  masks[pos[p]] = tmask[p];
}

inline unsigned blocks_of(int64_t n) { return (unsigned)std::max<int64_t>(1, ceil_div(n, kThreadsT)); }

void tile_dims(const GridDesc& gd, int64_t* nt0, int64_t* nt1, int64_t* nt2) {
  *nt0 = gd.nb[0];
  *nt1 = ceil_div(gd.nb[1], kTileY);
  *nt2 = ceil_div(gd.nb[2], kTileZ);
}

SlotSpace grid_slots(const GridDesc& gd) {
  int64_t nt0, nt1, nt2;
  tile_dims(gd, &nt0, &nt1, &nt2);
  return slot_space(nt0, nt1, nt2);
}

// Workspace of the tile compaction: tmask, flag and pos by slot (S.n each),
// tiles and masks (one per tile), and the scan's workspace.
int64_t compact_ws_elems(const SlotSpace& S) {
  return 3 * S.n + 2 * S.nt0 * S.nt1 * S.nt2 + scan_ws_elems(S.n);
}
int64_t* compact_tiles_out(int64_t* ws, const SlotSpace& S) { return ws + 3 * S.n; }
int64_t* compact_masks_out(int64_t* ws, const SlotSpace& S) { return ws + 3 * S.n + S.nt0 * S.nt1 * S.nt2; }

// Scan of the slot flags and compaction of the marked tiles in slot order;
// returns the count (waits for it).  pinned: the count's two parts are read
// through pinned slots (one wait); else into pageable memory (a wait per
// copy, and no allocation on any call, also the first of a thread).
int64_t compact_tiles(int64_t* ws, const SlotSpace& S, hipStream_t s, bool pinned = true) {
  int64_t* tmask = ws;
  int64_t* flag = ws + S.n;
  int64_t* pos = ws + 2 * S.n;
  scan_exclusive_i64_ws(flag, pos, S.n, ws + 3 * S.n + 2 * S.nt0 * S.nt1 * S.nt2, s);
  hipLaunchKernelGGL(k_tile_compact, dim3(blocks_of(S.n)), dim3(kThreadsT), 0, s, tmask, pos, S,
                     compact_tiles_out(ws, S), compact_masks_out(ws, S));
  RBF_HIP(hipGetLastError());
  if (!pinned) {
    int64_t h[2] = {0, 0};
    RBF_HIP(hipMemcpyAsync(h, pos + (S.n - 1), sizeof(int64_t), hipMemcpyDeviceToHost, s));
    RBF_HIP(hipMemcpyAsync(h + 1, flag + (S.n - 1), sizeof(int64_t), hipMemcpyDeviceToHost, s));
    RBF_HIP(hipStreamSynchronize(s));
    return h[0] + h[1];
  }
  PinnedSlots last(2);
  RBF_HIP(hipMemcpyAsync(last.p, pos + (S.n - 1), sizeof(int64_t), hipMemcpyDeviceToHost, s));
  RBF_HIP(hipMemcpyAsync(last.p + 1, flag + (S.n - 1), sizeof(int64_t), hipMemcpyDeviceToHost, s));
  RBF_HIP(hipStreamSynchronize(s));
  return last.p[0] + last.p[1];
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

int64_t support_tiles_ws_elems(const rbf_grid& g) {
  const GridDesc gd = grid_desc(g);
  return gd.nb[0] * gd.nb[1] * gd.nb[2] + compact_ws_elems(grid_slots(gd));
}

int64_t support_tiles(const Ctx& c, const rbf_grid& g, int64_t* ws, const int64_t** tiles, const int64_t** masks,
                      hipStream_t s, bool pinned) {
  const GridDesc gd = grid_desc(g);
  const SlotSpace S = grid_slots(gd);
  const int64_t nbricks = gd.nb[0] * gd.nb[1] * gd.nb[2];
  int64_t* mark = ws;
  int64_t* tw = ws + nbricks;
  mark_support(c, gd, mark, nbricks, s);
  hipLaunchKernelGGL(k_tiles_from_marks, dim3(blocks_of(S.n)), dim3(kThreadsT), 0, s, mark, gd, S, tw, tw + S.n);
  RBF_HIP(hipGetLastError());
  const int64_t nt = compact_tiles(tw, S, s, pinned);
  *tiles = compact_tiles_out(tw, S);
  *masks = compact_masks_out(tw, S);
  return nt;
}

void brick_sum_tiles(const Ctx& c, const rbf_grid& g, const int64_t* tiles, const int64_t* masks, int64_t nt,
                     const double* w_sorted, float* out, int64_t* useful, int64_t* examined, hipStream_t s,
                     hipEvent_t t0, hipEvent_t t1) {
  if (useful) *useful = 0;
  if (examined) *examined = 0;
  if (nt <= 0) return;
  const GridDesc gd = grid_desc(g);
  int64_t nt0, nt1, nt2;
  tile_dims(gd, &nt0, &nt1, &nt2);
  TileArgs a;
  a.gd = gd;
  a.tiles = tiles;
  a.masks = masks;
  a.nt = nt;
  a.nt0 = nt0;
  a.nt1 = nt1;
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
  a.useful = nullptr;
  a.examined = nullptr;
  const int64_t nb = ceil_div(nt, kTileWaves);
  if (useful && examined) {
    int64_t* cnt = talloc<int64_t>(2 * nt + 2);
    a.useful = cnt;
    a.examined = cnt + nt;
    hipExtLaunchKernelGGL(k_brick_sum_f32<true>, dim3((unsigned)nb), dim3(kTileWaves * kWave), 0, s, t0, t1, 0, a);
    RBF_HIP(hipGetLastError());
    sum_i64(cnt, nt, cnt + 2 * nt, s);
    sum_i64(cnt + nt, nt, cnt + 2 * nt + 1, s);
    int64_t h[2] = {0, 0};
    RBF_HIP(hipMemcpyAsync(h, cnt + 2 * nt, sizeof(h), hipMemcpyDeviceToHost, s));
    RBF_HIP(hipStreamSynchronize(s));
    temp_free(cnt);
    *useful = h[0];
    *examined = h[1];
  } else {
    hipExtLaunchKernelGGL(k_brick_sum_f32<false>, dim3((unsigned)nb), dim3(kTileWaves * kWave), 0, s, t0, t1, 0, a);
    RBF_HIP(hipGetLastError());
  }
}

void brick_sum_f32(const Ctx& c, const rbf_grid& g, const int64_t* ids, int64_t nact, const double* w_sorted,
                   float* out, int64_t* useful, int64_t* examined, hipStream_t s) {
  if (useful) *useful = 0;
  if (examined) *examined = 0;
  if (nact <= 0) return;
  const GridDesc gd = grid_desc(g);
  const SlotSpace S = grid_slots(gd);
  int64_t* ws = talloc<int64_t>(compact_ws_elems(S));
  hipLaunchKernelGGL(k_fill_zero, dim3(blocks_of(S.n)), dim3(kThreadsT), 0, s, ws, S.n);
  hipLaunchKernelGGL(k_tile_mark, dim3(blocks_of(nact)), dim3(kThreadsT), 0, s, ids, nact, gd, S,
                     reinterpret_cast<unsigned long long*>(ws));
  hipLaunchKernelGGL(k_nonzero, dim3(blocks_of(S.n)), dim3(kThreadsT), 0, s, ws, S.n, ws + S.n);
  RBF_HIP(hipGetLastError());
  const int64_t nt = compact_tiles(ws, S, s);
  brick_sum_tiles(c, g, compact_tiles_out(ws, S), compact_masks_out(ws, S), nt, w_sorted, out, useful, examined, s);
  temp_free(ws);
}

}  // namespace rbf
