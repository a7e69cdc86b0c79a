// rhd_tile.hpp -- tiled radiation Van Leer stages for 3D grids (gfx950).
//
// A block of 64 x BY threads owns an x-y tile of 64 x BY cells, one wavefront per x-row,
// and walks a chunk of z planes. Each thread owns the faces on the low side of its cell:
// in x and y the neighbour's data comes through LDS, in z from the registers of the
// previous plane, so every face flux inside a tile is evaluated once. The faces on the
// high x and y edges of a tile (and, in the predictor, the closure data of the cells just
// outside it) are extra work items gathered into one or two wavefronts of the block, so
// no thread of a tile exists only to supply a halo. Every global load and store of a row
// is one coalesced 64-wide access.
//
// Both kernels produce what the per-cell kernels of rhd_device.hpp produce: the
// predictor writes U^{m+1/2} on the interior plus two ghost layers, the corrector
// overwrites U^m with U^{m+1} on the interior.
#pragma once

#include "rhd_device.hpp"

namespace rhdk {

constexpr int TILE_BX = 64;
// Minimum wavefronts per SIMD the FP32 stages are compiled for (HIP's second launch
// bound). The predictor keeps the z data of its previous plane in LDS instead of ten
// registers and fits 96 VGPRs, so five 4-row blocks share a CU (five waves per SIMD;
// their LDS, 31 KB each, fills 155 of its 160 KB); the FP32 predictor therefore always
// runs 4-row tiles, whatever the corrector's. The corrector gets 128 VGPRs: unbounded,
// its four-plane unrolled loop takes up to 140 and would drop to three waves.
constexpr int PREDICT_WAVES_FP32 = 5;
constexpr int PREDICT_ROWS_FP32 = 4;
constexpr int CORRECT_WAVES_FP32 = 4;

__host__ __device__ __forceinline__ int clamp_i(int q, int lo, int hi) {
  return q < lo ? lo : (q > hi ? hi : q);
}

// Planes per z chunk: the requested chunk length rebalanced so that the chunks of a
// range of L planes are as even as possible.
__host__ __device__ __forceinline__ int balanced_chunk(int L, int zc) {
  const int chunks = (L + zc - 1) / zc;
  return (L + chunks - 1) / chunks;
}

// XCD-aware tile order. The dispatcher hands workgroup L (x fastest over the grid) to
// XCD L mod 8, and each XCD has its own L2. Tile L of a launch of N is therefore
// renumbered so that every XCD gets one contiguous range of tiles in x-fastest order:
// the x and y neighbours of a tile, whose rows hold its halo cells, then run on the same
// XCD at about the same time and the shared cache lines come from its L2 instead of
// memory. The map is a permutation of [0, N).
__host__ __device__ __forceinline__ int xcd_tile(int L, int N) {
  const int j = L & 7, k = L >> 3, q = N >> 3, r = N & 7;
  return j * q + (j < r ? j : r) + k;
}

// Tile coordinates of this block of a 3D tile grid in the XCD-aware order.
__device__ __forceinline__ void xcd_block(int& bx, int& by, int& bz) {
  const int gx = int(gridDim.x), gy = int(gridDim.y);
  const int L = int(blockIdx.x) + gx * (int(blockIdx.y) + gy * int(blockIdx.z));
  const int T = xcd_tile(L, gx * gy * int(gridDim.z));
  bx = T % gx;
  by = (T / gx) % gy;
  bz = T / (gx * gy);
}

template <typename T>
struct alignas(4 * sizeof(T)) V4 {
  T v[4];
};
template <typename T>
struct alignas(2 * sizeof(T)) V2 {
  T v[2];
};

template <typename T>
__device__ __forceinline__ void put4(V4<T>& d, const T s[4]) {
  V4<T> t;
#pragma unroll
  for (int q = 0; q < 4; ++q) t.v[q] = s[q];
  d = t;
}

template <typename T>
__device__ __forceinline__ void get4(const V4<T>& d, T s[4]) {
  const V4<T> t = d;
#pragma unroll
  for (int q = 0; q < 4; ++q) s[q] = t.v[q];
}

// Closure data (state, physical flux, wave speeds) of R x C cells for the faces of one
// direction, stored so that each part is one vector LDS access per lane.
template <typename T, int R, int C>
struct SideTile {
  V4<T> U[R][C];
  V4<T> P[R][C];
  V2<T> L[R][C];
  __device__ __forceinline__ void put(int r, int c, const FaceSide<T>& s) {
    put4(U[r][c], s.U);
    put4(P[r][c], s.Phi);
    V2<T> l;
    l.v[0] = s.lmin;
    l.v[1] = s.lmax;
    L[r][c] = l;
  }
  __device__ __forceinline__ FaceSide<T> get(int r, int c) const {
    FaceSide<T> s;
    get4(U[r][c], s.U);
    get4(P[r][c], s.Phi);
    const V2<T> l = L[r][c];
    s.lmin = l.v[0];
    s.lmax = l.v[1];
    return s;
  }
};

template <typename T>
__device__ __forceinline__ FaceSide<T> side_dir(const M1State<T>& m, const T U[4], int d, T c,
                                                T inv_c, T chat) {
  FaceSide<T> q;
#pragma unroll
  for (int k = 0; k < 4; ++k) q.U[k] = U[k];
  m1_dir(m, d, c, inv_c, chat, q.Phi, q.lmin, q.lmax);
  return q;
}

// ---------------------------------------------------------------------------
// predictor: first-order HLL fluxes of U^m, half step, on the interior plus two ghost
// layers of a 3D grid
// ---------------------------------------------------------------------------
//
// Grid: (ntx + 1, ceil((n1 + 4)/BY), ceil((n2 + 4)/zc)) with ntx = ceil(n0/64). Block
// (bx < ntx, by, bz) covers x in [64 bx, 64 bx + 64) within [0, n0), y in
// [-2 + BY by, -2 + BY (by + 1)) within [-2, n1 + 2) and z in [-2 + zc bz, -2 + zc (bz + 1))
// within [-2, n2 + 2). Block bx = ntx evaluates the four ghost columns x = -2, -1, n0,
// n0 + 1 of the same y-z range cell by cell.

// Inside a row the x faces need no LDS: a row is one wavefront, and lane i takes the
// closure data of lane i - 1 and the flux of lane i + 1 by a cross-lane shift. Only the
// two faces on the row's ends go through LDS. Keeping the x data out of LDS halves the
// block's LDS, so that four blocks fit on a CU instead of two.
template <typename T, int BY>
struct PredictShared {
  SideTile<T, BY + 2, TILE_BX> sy;  // [r][c]: y data of cell (x0 + c, y0 - 1 + r)
  SideTile<T, BY, 4> sxe;           // [r][k]: x data of cells x0 - 1, x0, x0 + 63, x0 + 64
  V4<T> fxe[BY][2];                 // [r][k]: flux through the x face x0 (k = 0), x0 + 64 (1)
  V4<T> fy[BY + 1][TILE_BX];        // [j][c]: flux through the low y face of (x0 + c, y0 + j)
  SideTile<T, BY, TILE_BX> zp;      // [r][c]: z data of cell (x0 + c, y0 + r) in plane t-1
};

// Cross-lane shifts within a wavefront (DPP wave_shr:1 / wave_shl:1): lane i receives
// the value of lane i - 1 (from_left) or lane i + 1 (from_right); the lane at the end,
// which has no such neighbour, keeps `edge`. Every lane of the wavefront must be active.
__device__ __forceinline__ float lane_from_left(float v, float edge) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(v), 0x138, 0xF, 0xF, false));
}
__device__ __forceinline__ float lane_from_right(float v, float edge) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(v), 0x130, 0xF, 0xF, false));
}
__device__ __forceinline__ double lane_shift64(double v, double edge, bool left) {
  const long long a = __double_as_longlong(v), e = __double_as_longlong(edge);
  const int lo = int(a & 0xffffffffLL), hi = int(a >> 32);
  const int elo = int(e & 0xffffffffLL), ehi = int(e >> 32);
  const int rlo = left ? __builtin_amdgcn_update_dpp(elo, lo, 0x138, 0xF, 0xF, false)
                       : __builtin_amdgcn_update_dpp(elo, lo, 0x130, 0xF, 0xF, false);
  const int rhi = left ? __builtin_amdgcn_update_dpp(ehi, hi, 0x138, 0xF, 0xF, false)
                       : __builtin_amdgcn_update_dpp(ehi, hi, 0x130, 0xF, 0xF, false);
  return __longlong_as_double((static_cast<long long>(rhi) << 32) |
                              static_cast<long long>(static_cast<unsigned>(rlo)));
}
__device__ __forceinline__ double lane_from_left(double v, double edge) {
  return lane_shift64(v, edge, true);
}
__device__ __forceinline__ double lane_from_right(double v, double edge) {
  return lane_shift64(v, edge, false);
}

template <typename T>
__device__ __forceinline__ FaceSide<T> side_from_left(const FaceSide<T>& s) {
  FaceSide<T> q;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    q.U[k] = lane_from_left(s.U[k], s.U[k]);
    q.Phi[k] = lane_from_left(s.Phi[k], s.Phi[k]);
  }
  q.lmin = lane_from_left(s.lmin, s.lmin);
  q.lmax = lane_from_left(s.lmax, s.lmax);
  return q;
}

template <typename T, int BY>
__device__ __forceinline__ void rad_predict_tile_body(const RadPtrs<T>& Um, const RadPtrs<T>& Uh,
                                                      const GasView<T>& gas, const Geom& G,
                                                      const RadConst<T>& K, T h, int zc, int bx,
                                                      int by, int bz, PredictShared<T, BY>& sh) {
  static_assert(BY >= 4, "the extra work items need four wavefronts");
  const int tx = int(threadIdx.x), ty = int(threadIdx.y);
  const int n0 = G.n[0], n1 = G.n[1], n2 = G.n[2];
  const int ntx = (n0 + TILE_BX - 1) / TILE_BX;
  const int y0 = -2 + by * BY;
  const int z0 = -2 + bz * zc;
  const int z1 = min(z0 + zc, n2 + 2);
  if (bx >= ntx) {
    // the ghost columns, one cell per work item
    const int ylim = min(y0 + BY, n1 + 2);
    const int items = 4 * BY * (z1 - z0);
    for (int e = tx + TILE_BX * ty; e < items; e += TILE_BX * BY) {
      const int g = e & 3;
      const int r = (e >> 2) % BY;
      const int p = (e >> 2) / BY;
      const int x = g < 2 ? g - 2 : n0 + g - 2;
      if (y0 + r < ylim) rad_predict_cell(Um, Uh, gas, G, K, FixedFaces<T>{}, h, x, y0 + r, z0 + p);
    }
    return;
  }
  const int x0 = bx * TILE_BX;
  const int x = x0 + tx, y = y0 + ty;
  // every read stays within [-3, n + 2], where the boundary mapping is defined
  const int xl = min(x, n0 + 2), yl = min(y, n1 + 2);
  const bool out_xy = x < n0 && y < n1 + 2;
  // extra items, one per wavefront on different SIMDs (wave w runs on SIMD w mod 4):
  // before the first barrier wave 0 brings the y data of row y0 - 1, wave 1 that of row
  // y0 + BY and lanes < 2 BY of wave 2 the x data of cells x0 - 1 and x0 + 64 of row
  // lane mod BY; between the barriers wave 3 takes the high y faces and lanes < 2 BY of
  // wave 0 the x faces on the two ends of row lane mod BY
  const int hrole = ty == 0 ? 1 : (ty == 1 ? 2 : ((ty == 2 && tx < 2 * BY) ? 3 : 0));
  const int hrow = tx % BY;
  const int hx = hrole == 3 ? (tx < BY ? x0 - 1 : min(x0 + TILE_BX, n0 + 2)) : xl;
  const int hy = hrole == 1 ? y0 - 1 : (hrole == 2 ? min(y0 + BY, n1 + 2) : min(y0 + hrow, n1 + 2));
  const bool need_v = K.beta != 0;
  const T c = K.c, ic = K.inv_c, fc = K.fclo, chat = K.chat;

  // loads run one plane ahead of their use: U^m of the own cell, the extra item's cell
  // and the gas data of the cell being updated
  T Un[4], Hn[4] = {T(0), T(0), T(0), T(0)};
  int nU, nH = 0;
  load_rad_raw<T, true>(Um, G, xl, yl, z0 - 1, Un, nU);
  if (hrole) load_rad_raw<T, true>(Um, G, hx, hy, z0, Hn, nH);
  FrozenRaw<T> gn = {};

  T fzprev[4] = {T(0), T(0), T(0), T(0)};
  T divprev[4] = {T(0), T(0), T(0), T(0)};
  for (int t = z0 - 1; t <= z1; ++t) {
    // z data of plane t-1, kept in the thread's own LDS slot between planes
    const FaceSide<T> zprev = sh.zp.get(ty, tx);
    T U[4] = {Un[0], Un[1], Un[2], Un[3]};
    unflip_rad(U, nU);
    if (t < z1) load_rad_raw<T, true>(Um, G, xl, yl, t + 1, Un, nU);
    const M1State<T> m = m1_state(U, fc, chat);
    // z face t-1/2, then plane t-1 is complete: its z faces are t-3/2 and t-1/2
    const FaceSide<T> fzs = side_dir(m, U, 2, c, ic, chat);
    T fz[4] = {T(0), T(0), T(0), T(0)};
    if (t > z0 - 1) hll(zprev, fzs, fz);
    if (t > z0 && out_xy) {
      T d[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) d[q] = divprev[q] + (fz[q] - fzprev[q]) * K.inv_w[2];
      const Frozen<T> gz = frozen_make(gn, need_v);
      T out[4];
      bool ef, fc;
      rad_update(K, h, zprev.U, zprev.U, d, gz, out, ef, fc);
      const int p = padded_cell(G, x, y, t - 1);
      elem<true>(Uh.E, p) = out[0];
      elem<true>(Uh.F[0], p) = out[1];
      elem<true>(Uh.F[1], p) = out[2];
      elem<true>(Uh.F[2], p) = out[3];
    }
    if (t >= z0 && t < z1) {
      int s[3];
      gn = frozen_load<T, true>(gas, mapped_cell(G, xl, yl, t, s), s, need_v);
    }
    sh.zp.put(ty, tx, fzs);
#pragma unroll
    for (int q = 0; q < 4; ++q) fzprev[q] = fz[q];
    if (t >= z0 && t < z1) {
      // x faces of plane t inside the row (lane 0's is redone below), y data to LDS
      T fl[4];
      {
        const FaceSide<T> sxo = side_dir(m, U, 0, c, ic, chat);
        hll(side_from_left(sxo), sxo, fl);
        if (tx == 0 || tx == TILE_BX - 1) sh.sxe.put(ty, tx == 0 ? 1 : 2, sxo);
      }
      sh.sy.put(ty + 1, tx, side_dir(m, U, 1, c, ic, chat));
      if (hrole) {
        T H[4] = {Hn[0], Hn[1], Hn[2], Hn[3]};
        unflip_rad(H, nH);
        const FaceSide<T> hs = face_side(H, hrole == 3 ? 0 : 1, c, ic, fc, chat);
        if (hrole == 1)
          sh.sy.put(0, tx, hs);
        else if (hrole == 2)
          sh.sy.put(BY + 1, tx, hs);
        else
          sh.sxe.put(hrow, tx < BY ? 0 : 3, hs);
        if (t + 1 < z1) load_rad_raw<T, true>(Um, G, hx, hy, t + 1, Hn, nH);
      }
      __syncthreads();
      T fb[4];
      hll(sh.sy.get(ty, tx), sh.sy.get(ty + 1, tx), fb);
      put4(sh.fy[ty][tx], fb);
      if (ty == 0 && tx < 2 * BY) {
        // x face x0 (lanes < BY) or x0 + 64 (lanes BY .. 2 BY - 1) of row lane mod BY
        const int k = tx < BY ? 0 : 1;
        T f[4];
        hll(sh.sxe.get(hrow, 2 * k), sh.sxe.get(hrow, 2 * k + 1), f);
        put4(sh.fxe[hrow][k], f);
      }
      if (ty == 3) {
        T f[4];
        hll(sh.sy.get(BY, tx), sh.sy.get(BY + 1, tx), f);
        put4(sh.fy[BY][tx], f);
      }
      __syncthreads();
      T fr[4], ft[4], fe[4], f0[4];
      get4(sh.fxe[ty][1], fe);
      get4(sh.fxe[ty][0], f0);
#pragma unroll
      for (int q = 0; q < 4; ++q) fr[q] = lane_from_right(fl[q], fe[q]);
      if (tx == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) fl[q] = f0[q];
      }
      get4(sh.fy[ty + 1][tx], ft);
#pragma unroll
      for (int q = 0; q < 4; ++q)
        divprev[q] = (fr[q] - fl[q]) * K.inv_w[0] + (ft[q] - fb[q]) * K.inv_w[1];
    }
  }
}

template <typename T, int BY>
__global__ void __launch_bounds__(TILE_BX * BY, sizeof(T) == 4 ? PREDICT_WAVES_FP32 : 2) k_rad_predict_tile(RadPtrs<T> Um, RadPtrs<T> Uh,
                                                                   GasView<T> gas, Geom G,
                                                                   RadConst<T> K, T h, int zc) {
  __shared__ PredictShared<T, BY> sh;
  int bx, by, bz;
  xcd_block(bx, by, bz);
  rad_predict_tile_body<T, BY>(Um, Uh, gas, G, K, h, zc, bx, by, bz, sh);
}

// ---------------------------------------------------------------------------
// corrector: MC-limited reconstruction of U^{m+1/2}, HLL fluxes, full step from U^m
// with sources at U^{m+1/2}; U^{m+1} overwrites U^m on the interior of a 3D grid
// ---------------------------------------------------------------------------
//
// Grid: (ceil(n0/64), ceil(n1/BY), ceil(n2/zc)); block (bx, by, bz) covers
// x in [64 bx, 64 bx + 64), y in [BY by, BY (by + 1)), z in [zc bz, zc (bz + 1)), each
// within [0, n). The current plane of U^{m+1/2} sits in LDS with a two-cell ring; the
// ring's cells of the next plane are loaded while the current one is processed.

// As in the predictor, the x faces inside a row use cross-lane shifts: lane i limits its
// own cell only and takes the high-side state of lane i - 1 and the flux of lane i + 1,
// so every x slope is evaluated once; the two faces on the row's ends go through LDS.
//
// One barrier per plane: the LDS arrays come in two copies, one per plane parity. The
// barrier of plane t both publishes plane t's states and closes the flux writes of plane
// t - 1, whose divergence and update are finished right after it; a copy is written
// again only two planes later, after the next barrier has ordered every read of it.
template <typename T, int BY>
struct CorrectShared {
  V4<T> U[2][BY + 4][TILE_BX + 4];  // [b][r][c]: U^{m+1/2} of cell (x0 - 2 + c, y0 - 2 + r)
  V4<T> fxe[2][BY][2];              // [b][r][k]: flux through the x face x0 (k = 0), x0 + 64 (1)
  V4<T> fy[2][BY + 1][TILE_BX];     // [b][j][c]: flux through the low y face of (x0 + c, y0 + j)
};

template <int BY>
struct CorrectRing {
  static constexpr int W = TILE_BX + 4;
  static constexpr int cells = 4 * W + 4 * BY;  // two rows below and above, two columns each side
  static constexpr int threads = TILE_BX * BY;
  static constexpr int per_thread = (cells + threads - 1) / threads;
  // LDS position (row r, column c) of ring cell e
  __host__ __device__ static void rc(int e, int& r, int& c) {
    if (e < 4 * W) {
      const int q = e / W;
      c = e - q * W;
      r = q < 2 ? q : BY + q;
    } else {
      const int k = e - 4 * W;
      const int s = k & 3;
      c = s < 2 ? s : TILE_BX + s;
      r = 2 + (k >> 2);
    }
  }
};

// MC-limited face states of a cell with neighbours um (below) and up (above) along one
// direction: lo on its low face, hi on its high face. E_r of a face state is raised to
// ef: a face state may reach a neighbour's value, and next to a cell at the floor
// rounding can take it to zero, where the closure has no direction.
template <typename T>
__device__ __forceinline__ void mc_states(const T um[4], const T u[4], const T up[4], T lo[4],
                                          T hi[4], T ef) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const T hs = mc_half_slope(u[q] - um[q], up[q] - u[q]);
    lo[q] = u[q] - hs;
    hi[q] = u[q] + hs;
  }
  lo[0] = vmax(lo[0], ef);
  hi[0] = vmax(hi[0], ef);
}

// HLL flux through the face between cells b and c of the row a, b, c, d along direction
// dir, from the MC-limited states of b (high side) and c (low side).
template <typename T>
__device__ __forceinline__ void face_flux4(const T a[4], const T b[4], const T cc[4], const T d[4],
                                           int dir, T c, T ic, T fc, T chat, T ef, T f[4]) {
  T lo[4], hi[4], bh[4], cl[4];
  mc_states(a, b, cc, lo, bh, ef);
  mc_states(b, cc, d, cl, hi, ef);
  hll(face_side(bh, dir, c, ic, fc, chat), face_side(cl, dir, c, ic, fc, chat), f);
}

template <typename T, int BY>
__device__ __forceinline__ void rad_correct_tile_body(const RadPtrs<T>& Um, const RadPtrs<T>& Uh,
                                                      const GasView<T>& gas, const Geom& G,
                                                      const RadConst<T>& K, T h, int zc, int bx,
                                                      int by, int bz, unsigned long long* ctr,
                                                      CorrectShared<T, BY>& sh) {
  using Ring = CorrectRing<BY>;
  constexpr int RP = Ring::per_thread;
  const int tx = int(threadIdx.x), ty = int(threadIdx.y);
  const int tid = tx + TILE_BX * ty;
  const int n0 = G.n[0], n1 = G.n[1], n2 = G.n[2];
  const int x0 = bx * TILE_BX, y0 = by * BY;
  const int z0 = bz * zc;
  const int z1 = min(z0 + zc, n2);
  const int zs = G.ps[0] * G.ps[1];
  const T c = K.c, ic = K.inv_c, fc = K.fclo, chat = K.chat, ef = K.er_floor;
  // the ring of the LDS plane, loaded one plane ahead; the half-step arrays hold valid
  // values on [-2, n + 2) in every dimension
  int rpos[RP], rcol[RP];
#pragma unroll
  for (int s = 0; s < RP; ++s) {
    const int e = tid + s * Ring::threads;
    rpos[s] = -1;
    rcol[s] = 0;
    if (e < Ring::cells) {
      int r, cc;
      Ring::rc(e, r, cc);
      rpos[s] = r * (TILE_BX + 4) + cc;
      rcol[s] = padded_cell(G, clamp_i(x0 - 2 + cc, -2, n0 + 1), clamp_i(y0 - 2 + r, -2, n1 + 1), 0);
    }
  }
  T ring[RP][4];
#pragma unroll
  for (int s = 0; s < RP; ++s)
    if (rpos[s] >= 0) load_padded4<T, true>(Uh, rcol[s] + z0 * zs, ring[s]);

  const int x = x0 + tx, y = y0 + ty;
  const bool out_xy = x < n0 && y < n1;
  const int pcol = padded_cell(G, clamp_i(x, -2, n0 + 1), clamp_i(y, -2, n1 + 1), 0);
  // the own column of U^{m+1/2}: planes t-1, t, t+1 and t+2 of plane step t, held in
  // four arrays whose roles rotate by one each step (the plane loop is unrolled by four,
  // so the rotation is a renaming and costs no moves)
  T Ua[4], Ub[4], Uc[4], Ud[4];
  load_padded4<T, true>(Uh, pcol + (z0 - 2) * zs, Ua);
  load_padded4<T, true>(Uh, pcol + (z0 - 1) * zs, Ub);
  load_padded4<T, true>(Uh, pcol + z0 * zs, Uc);
  // U^m and the gas data of the cell updated at the next plane, loaded one plane ahead
  const bool need_v = K.beta != 0;
  const int s1[3] = {1, 1, 1};
  FrozenRaw<T> gn = {};
  T Uon[4] = {T(0), T(0), T(0), T(0)};
  FaceSide<T> zplus;  // high-z face data of plane t-1
  T fzprev[4] = {T(0), T(0), T(0), T(0)};
  // fluxes through the low x and y faces of the own cell in plane t-1 (lane 0's x face
  // is replaced by the row-end item)
  T flp[4] = {T(0), T(0), T(0), T(0)}, fbp[4] = {T(0), T(0), T(0), T(0)};
  unsigned long long nef = 0, nfc = 0;
  auto plane_step = [&](const int t, T (&Uzm)[4], T (&Uz0)[4], T (&Uzp)[4],
                        T (&Upp)[4]) __attribute__((always_inline)) {
    const bool plane = t >= z0 && t < z1;  // planes whose x and y faces are needed
    const int b = t & 1;
    if (plane) {
      V4<T>* const sUf = &sh.U[b][0][0];
      put4(sh.U[b][ty + 2][tx + 2], Uz0);
#pragma unroll
      for (int s = 0; s < RP; ++s)
        if (rpos[s] >= 0) put4(sUf[rpos[s]], ring[s]);
      if (t + 1 < z1) {
#pragma unroll
        for (int s = 0; s < RP; ++s)
          if (rpos[s] >= 0) load_padded4<T, true>(Uh, rcol[s] + (t + 1) * zs, ring[s]);
      }
    }
    if (t < z1) load_padded4<T, true>(Uh, pcol + (t + 2) * zs, Upp);
    // z: limited states of the own cell; the low z face pairs them with plane t-1
    T mz[4], pz[4];
    mc_states(Uzm, Uz0, Uzp, mz, pz, ef);
    T fz[4] = {T(0), T(0), T(0), T(0)};
    if (t > z0 - 1) hll(zplus, face_side(mz, 2, c, ic, fc, chat), fz);
    if (t >= z0) __syncthreads();
    if (t > z0) {
      // plane t-1 is complete: its x and y fluxes are in LDS copy (t-1) & 1, its z faces
      // are t-3/2 (fzprev) and t-1/2 (fz)
      const int pb = b ^ 1;
      T fr[4], ft[4], fe[4], f0[4];
      get4(sh.fxe[pb][ty][1], fe);
      get4(sh.fxe[pb][ty][0], f0);
#pragma unroll
      for (int q = 0; q < 4; ++q) fr[q] = lane_from_right(flp[q], fe[q]);
      if (tx == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) flp[q] = f0[q];
      }
      get4(sh.fy[pb][ty + 1][tx], ft);
      if (out_xy) {
        T d[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const T dxy = (fr[q] - flp[q]) * K.inv_w[0] + (ft[q] - fbp[q]) * K.inv_w[1];
          d[q] = dxy + (fz[q] - fzprev[q]) * K.inv_w[2];
        }
        const int a = x + n0 * (y + n1 * (t - 1));
        const Frozen<T> gz = frozen_make(gn, need_v);
        T out[4];
        bool ef, fc;
        rad_update(K, h, Uon, Uzm, d, gz, out, ef, fc);
        nef += ef ? 1ull : 0ull;
        nfc += fc ? 1ull : 0ull;
        elem<true>(Um.E, a) = out[0];
        elem<true>(Um.F[0], a) = out[1];
        elem<true>(Um.F[1], a) = out[2];
        elem<true>(Um.F[2], a) = out[3];
      }
    }
    if (plane && out_xy) {
      const int a = x + n0 * (y + n1 * t);
      gn = frozen_load<T, true>(gas, a, s1, need_v);
      Uon[0] = elem<true>(Um.E, a);
      Uon[1] = elem<true>(Um.F[0], a);
      Uon[2] = elem<true>(Um.F[1], a);
      Uon[3] = elem<true>(Um.F[2], a);
    }
    if (t < z1) zplus = face_side(pz, 2, c, ic, fc, chat);
#pragma unroll
    for (int q = 0; q < 4; ++q) fzprev[q] = fz[q];
    if (plane) {
      {
        // lane 0's low x face is replaced by the row-end item below
        T bb[4], d[4], lo[4], hi[4], bh[4];
        get4(sh.U[b][ty + 2][tx + 1], bb);
        get4(sh.U[b][ty + 2][tx + 3], d);
        mc_states(bb, Uz0, d, lo, hi, ef);
#pragma unroll
        for (int q = 0; q < 4; ++q) bh[q] = lane_from_left(hi[q], hi[q]);
        hll(face_side(bh, 0, c, ic, fc, chat), face_side(lo, 0, c, ic, fc, chat), flp);
      }
      {
        T a[4], bb[4], d[4];
        get4(sh.U[b][ty][tx + 2], a);
        get4(sh.U[b][ty + 1][tx + 2], bb);
        get4(sh.U[b][ty + 3][tx + 2], d);
        face_flux4(a, bb, Uz0, d, 1, c, ic, fc, chat, ef, fbp);
      }
      put4(sh.fy[b][ty][tx], fbp);
      // extra items on waves of different SIMDs (wave w runs on SIMD w mod 4)
      if (ty == 0 && tx < 2 * BY) {
        // x face x0 (lanes < BY: cells x0 - 2 ... x0 + 1) or x0 + 64 (lanes BY .. 2 BY - 1:
        // cells x0 + 62 ... x0 + 65) of row lane mod BY
        const int r = tx % BY, k = tx < BY ? 0 : 1, c0 = k ? TILE_BX : 0;
        T a[4], bb[4], cc[4], d[4], f[4];
        get4(sh.U[b][r + 2][c0], a);
        get4(sh.U[b][r + 2][c0 + 1], bb);
        get4(sh.U[b][r + 2][c0 + 2], cc);
        get4(sh.U[b][r + 2][c0 + 3], d);
        face_flux4(a, bb, cc, d, 0, c, ic, fc, chat, ef, f);
        put4(sh.fxe[b][r][k], f);
      }
      if (ty == BY - 1) {
        // high y face of column tx: rows y0 + BY - 2 ... y0 + BY + 1
        T a[4], cc[4], d[4], f[4];
        get4(sh.U[b][BY][tx + 2], a);
        get4(sh.U[b][BY + 2][tx + 2], cc);
        get4(sh.U[b][BY + 3][tx + 2], d);
        face_flux4(a, Uz0, cc, d, 1, c, ic, fc, chat, ef, f);
        put4(sh.fy[b][BY][tx], f);
      }
    }
  };
  for (int t = z0 - 1; t <= z1; t += 4) {
    plane_step(t, Ua, Ub, Uc, Ud);
    if (t + 1 > z1) break;
    plane_step(t + 1, Ub, Uc, Ud, Ua);
    if (t + 2 > z1) break;
    plane_step(t + 2, Uc, Ud, Ua, Ub);
    if (t + 3 > z1) break;
    plane_step(t + 3, Ud, Ua, Ub, Uc);
  }
  wave_add(ctr + CTR_RAD_EFLOOR, nef);
  wave_add(ctr + CTR_RAD_FCLAMP, nfc);
}

template <typename T, int BY>
__global__ void __launch_bounds__(TILE_BX * BY, sizeof(T) == 4 ? CORRECT_WAVES_FP32 : 1) k_rad_correct_tile(RadPtrs<T> Um, RadPtrs<T> Uh,
                                                                   GasView<T> gas, Geom G,
                                                                   RadConst<T> K, T h, int zc,
                                                                   unsigned long long* ctr) {
  __shared__ CorrectShared<T, BY> sh;
  int bx, by, bz;
  xcd_block(bx, by, bz);
  rad_correct_tile_body<T, BY>(Um, Uh, gas, G, K, h, zc, bx, by, bz, ctr, sh);
}

// Tile counts of the two launches for a grid n and requested chunk length zc, with the
// rebalanced chunk lengths they use.
struct TileGrid {
  int pred[3], corr[3];
  int zc_pred, zc_corr;
};

template <int BY>
__host__ __device__ inline TileGrid tile_grid(const int n[3], int zc) {
  TileGrid g;
  const int ntx = (n[0] + TILE_BX - 1) / TILE_BX;
  g.zc_pred = balanced_chunk(n[2] + 4, zc);
  g.zc_corr = balanced_chunk(n[2], zc);
  g.pred[0] = ntx + 1;
  g.pred[1] = (n[1] + 4 + BY - 1) / BY;
  g.pred[2] = (n[2] + 4 + g.zc_pred - 1) / g.zc_pred;
  g.corr[0] = ntx;
  g.corr[1] = (n[1] + BY - 1) / BY;
  g.corr[2] = (n[2] + g.zc_corr - 1) / g.zc_corr;
  return g;
}

// ---------------------------------------------------------------------------
// many independent solves in one launch: a packed list of tiles
// ---------------------------------------------------------------------------

// Everything one solve's radiation stages need; one entry per member of a batch.
template <typename T>
struct SolveDesc {
  RadPtrs<T> Um, Uh;
  GasView<T> gas;
  Geom G;
  RadConst<T> K;
  T h_pred, h_corr;
  int zc_pred, zc_corr;
  int tiles_pred, tiles_corr;  // tiles of one predictor and one corrector launch
  unsigned long long* ctr;
};

// Tile i of a launch is (solve, bx, by, bz) = tiles[i], taken in the XCD-aware order over
// the ntiles active blocks; blocks past ntiles exit at once, so one grid size serves
// every round.
template <typename T, int BY>
__global__ void __launch_bounds__(TILE_BX * BY, sizeof(T) == 4 ? PREDICT_WAVES_FP32 : 2) k_rad_predict_batch(const SolveDesc<T>* __restrict__ sd,
                                                                    const int4* __restrict__ tiles,
                                                                    const int* __restrict__ ntiles) {
  const int nt = *ntiles;
  if (int(blockIdx.x) >= nt) return;
  const int4 tr = tiles[xcd_tile(int(blockIdx.x), nt)];
  const SolveDesc<T> d = sd[tr.x];
  __shared__ PredictShared<T, BY> sh;
  rad_predict_tile_body<T, BY>(d.Um, d.Uh, d.gas, d.G, d.K, d.h_pred, d.zc_pred, tr.y, tr.z, tr.w,
                               sh);
}

template <typename T, int BY>
__global__ void __launch_bounds__(TILE_BX * BY, sizeof(T) == 4 ? CORRECT_WAVES_FP32 : 1) k_rad_correct_batch(const SolveDesc<T>* __restrict__ sd,
                                                                    const int4* __restrict__ tiles,
                                                                    const int* __restrict__ ntiles) {
  const int nt = *ntiles;
  if (int(blockIdx.x) >= nt) return;
  const int4 tr = tiles[xcd_tile(int(blockIdx.x), nt)];
  const SolveDesc<T> d = sd[tr.x];
  __shared__ CorrectShared<T, BY> sh;
  rad_correct_tile_body<T, BY>(d.Um, d.Uh, d.gas, d.G, d.K, d.h_corr, d.zc_corr, tr.y, tr.z, tr.w,
                               d.ctr, sh);
}

// ---------------------------------------------------------------------------
// many independent solves in one persistent launch
// ---------------------------------------------------------------------------
//
// The work of all subcycles of all members is one list of items, numbered level by
// level: level l is the predictor (l even) or the corrector (l odd) of subcycle l/2 and
// covers the first level_start[l+1] - level_start[l] tiles of that stage's packed list
// (members sorted by decreasing nsub, so the members still subcycling at level l are a
// prefix of the list). Blocks take items in order from one ticket counter. Member k's
// counter done[k] counts its finished items; an item of level l of member k may start
// once done[k] holds all of that member's items of the levels below l:
//   (l / 2) (tiles_pred + tiles_corr) + (l odd ? tiles_pred : 0).
// A block only ever waits for items with smaller tickets, which blocks already running
// hold, so the smallest unfinished item can always proceed: no deadlock, whatever the
// number of blocks that fit on the chip. Members do not wait for each other, so a member
// with few subcycles finishes without lock-step rounds, and the stages of different
// members overlap.
// Counters of a persistent launch sit one per 128-byte line (member k's at done[32 k]),
// so the polls of one member's waiters, another member's increments and the ticket
// claims do not queue on one line.
constexpr int COUNTER_STRIDE = 32;

struct PersistentPlan {
  const int4* tiles[2];     // packed tile lists of the predictor and the corrector
  const int* level_start;   // levels + 1 entries
  int levels;
  unsigned* done;           // per member, COUNTER_STRIDE apart
  unsigned* ticket;
  unsigned* error;          // set when a wait ran out of time; every block then exits
  unsigned long long wait_ticks;  // longest wait for a stage, in real-time counter ticks
};

// Level of item t: the last l with level_start[l] <= t.
__device__ __forceinline__ int plan_level(const int* __restrict__ start, int levels, int t) {
  int lo = 0, hi = levels - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= t)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

template <typename T, int BY>
union BatchShared {
  PredictShared<T, BY> p;
  CorrectShared<T, BY> c;
};

template <typename T, int BY>
__global__ void __launch_bounds__(TILE_BX * BY, sizeof(T) == 4 ? CORRECT_WAVES_FP32 : 2)
    k_rad_batch_persistent(const SolveDesc<T>* __restrict__ sd, PersistentPlan plan) {
  __shared__ BatchShared<T, BY> sh;
  __shared__ int s_item, s_level;
  const bool lead = threadIdx.x == 0 && threadIdx.y == 0;
  const int total = plan.level_start[plan.levels];
  for (;;) {
    if (lead) {
      int t = int(atomicAdd(plan.ticket, 1u));
      if (__hip_atomic_load(plan.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) t = total;
      if (t < total) {
        const int l = plan_level(plan.level_start, plan.levels, t);
        s_level = l;
        if (l > 0) {
          const int4 tr = plan.tiles[l & 1][t - plan.level_start[l]];
          const SolveDesc<T>& d = sd[tr.x];
          const unsigned need = unsigned(l >> 1) * unsigned(d.tiles_pred + d.tiles_corr) +
                                ((l & 1) ? unsigned(d.tiles_pred) : 0u);
          // bounded wait, by the real-time clock: a wait that runs out of time marks the
          // launch failed and every block leaves, so the launch always ends
          // (the clock is read every poll; the shared error flag every 64th poll, so the
          // waiters' polls stay on their own member's line)
          const unsigned* cnt = plan.done + COUNTER_STRIDE * tr.x;
          const unsigned long long start = __builtin_amdgcn_s_memrealtime();
          unsigned polls = 0;
          while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
            ++polls;
            if (__builtin_amdgcn_s_memrealtime() - start > plan.wait_ticks ||
                ((polls & 63u) == 0u &&
                 __hip_atomic_load(plan.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
              __hip_atomic_store(plan.error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              t = total;
              break;
            }
            __builtin_amdgcn_s_sleep(20);
          }
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
      }
      s_item = t;
    }
    __syncthreads();
    const int t = s_item;
    if (t >= total) return;
    const int l = s_level;
    // acquire: every wave sees the stores of the items it waited for
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const int4 tr = plan.tiles[l & 1][t - plan.level_start[l]];
    const SolveDesc<T> d = sd[tr.x];
    if ((l & 1) == 0)
      rad_predict_tile_body<T, BY>(d.Um, d.Uh, d.gas, d.G, d.K, d.h_pred, d.zc_pred, tr.y, tr.z,
                                   tr.w, sh.p);
    else
      rad_correct_tile_body<T, BY>(d.Um, d.Uh, d.gas, d.G, d.K, d.h_corr, d.zc_corr, tr.y, tr.z,
                                   tr.w, d.ctr, sh.c);
    // release: every wave's stores are complete and written back before the count
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (lead)
      __hip_atomic_fetch_add(plan.done + COUNTER_STRIDE * tr.x, 1u, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
  }
}

}  // namespace rhdk
