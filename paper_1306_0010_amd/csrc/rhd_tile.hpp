// rhd_tile.hpp -- tiled radiation Van Leer stages for 3D grids (gfx950).
//
// A block of 64 x BY threads owns an x-y tile of (64 - 2) x (BY - 2) output cells and
// walks a chunk of zc planes along z. Every thread evaluates the M1 closure of its own
// cell (predictor) or of its own reconstructed face states (corrector) exactly once:
// x- and y-neighbours exchange closure data and face fluxes through LDS, and the z
// neighbour's data is carried in registers from the previous plane, so each face flux
// of the HLL solver is computed once. The outer ring of threads of a tile only supplies
// the data for the faces on the tile's edge. One wavefront is one x-row of 64 cells,
// so every global load and store of a row is one coalesced access.
//
// Both kernels produce exactly what the per-cell kernels of rhd_device.hpp produce:
// the predictor writes U^{m+1/2} on the interior plus two ghost layers, the corrector
// overwrites U^m with U^{m+1} on the interior.
#pragma once

#include "rhd_device.hpp"

namespace rhdk {

constexpr int TILE_BX = 64;

__device__ __forceinline__ int clamp_i(int q, int lo, int hi) { return q < lo ? lo : (q > hi ? hi : q); }

template <typename T>
__device__ __forceinline__ FaceSide<T> side_dir(const M1State<T>& m, const T U[4], int d, T c,
                                                T inv_c, T chat) {
  FaceSide<T> q;
#pragma unroll
  for (int k = 0; k < 4; ++k) q.U[k] = U[k];
  m1_dir(m, d, c, inv_c, chat, q.Phi, q.lmin, q.lmax);
  return q;
}

// Predictor: first-order HLL fluxes of U^m, half step, on the interior plus two ghost
// layers of a 3D grid. Grid: (ceil((nx+4)/62), ceil((ny+4)/(BY-2)), ceil((nz+4)/zc)).
template <typename T, int BY>
struct PredictShared {
  FaceSide<T> sx[BY][TILE_BX];
  FaceSide<T> sy[BY][TILE_BX];
  T sfx[BY][TILE_BX][4];
  T sfy[BY][TILE_BX][4];
};

// One tile (bx, by, bz) of the predictor; called by every thread of the block.
template <typename T, int BY>
__device__ __forceinline__ void rad_predict_tile_body(const RadPtrs<T>& Um, const RadPtrs<T>& Uh,
                                                      const GasView<T>& gas, const Geom& G,
                                                      const RadConst<T>& K, T h, int zc, int bx,
                                                      int by, int bz, PredictShared<T, BY>& sh) {
  constexpr int BX = TILE_BX, TX = BX - 2, TY = BY - 2;
  auto& sx = sh.sx;
  auto& sy = sh.sy;
  auto& sfx = sh.sfx;
  auto& sfy = sh.sfy;
  const int tx = int(threadIdx.x), ty = int(threadIdx.y);
  const int x = -2 + bx * TX + tx - 1;
  const int y = -2 + by * TY + ty - 1;
  const int xhi = G.n[0] + 2, yhi = G.n[1] + 2;
  // stencil reads stay within [-3, n + 2] in every dimension
  const int xl = x < xhi ? x : xhi;
  const int yl = y < yhi ? y : yhi;
  const bool out_xy = tx >= 1 && tx <= TX && ty >= 1 && ty <= TY && x < xhi && y < yhi;
  const int z0 = -2 + bz * zc;
  const int z1 = min(z0 + zc, G.n[2] + 2);
  const T c = K.c, ic = K.inv_c, chat = K.chat;

  FaceSide<T> zprev;
  T fzprev[4] = {T(0), T(0), T(0), T(0)};
  T divprev[4] = {T(0), T(0), T(0), T(0)};
  for (int t = z0 - 1; t <= z1; ++t) {
    T U[4];
    load_rad_mapped(Um, G, xl, yl, t, U);
    const M1State<T> m = m1_state(U, ic, chat);
    const bool xy = t >= z0 && t < z1;  // planes whose own update is produced
    FaceSide<T> fxs, fys;
    if (xy) {
      fxs = side_dir(m, U, 0, c, ic, chat);
      fys = side_dir(m, U, 1, c, ic, chat);
      sx[ty][tx] = fxs;
      sy[ty][tx] = fys;
    }
    const FaceSide<T> fzs = side_dir(m, U, 2, c, ic, chat);
    __syncthreads();
    T fl[4] = {T(0), T(0), T(0), T(0)}, fb[4] = {T(0), T(0), T(0), T(0)};
    if (xy) {
      if (tx >= 1) hll(sx[ty][tx - 1], fxs, fl);
      if (ty >= 1) hll(sy[ty - 1][tx], fys, fb);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        sfx[ty][tx][q] = fl[q];
        sfy[ty][tx][q] = fb[q];
      }
    }
    T fz[4] = {T(0), T(0), T(0), T(0)};
    if (t > z0 - 1) hll(zprev, fzs, fz);
    __syncthreads();
    T div[4] = {T(0), T(0), T(0), T(0)};
    if (xy && tx < BX - 1 && ty < BY - 1) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        div[q] = (sfx[ty][tx + 1][q] - fl[q]) * K.inv_w[0] + (sfy[ty + 1][tx][q] - fb[q]) * K.inv_w[1];
    }
    if (t > z0 && out_xy) {
      // plane t-1 is complete: its z faces are t-3/2 (fzprev) and t-1/2 (fz)
      T d[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) d[q] = divprev[q] + (fz[q] - fzprev[q]) * K.inv_w[2];
      int s[3];
      const int a = mapped_cell(G, xl, yl, t - 1, s);
      const Frozen<T> gz = frozen_at(gas, a, s, K.beta != 0);
      T out[4];
      bool ef, fc;
      rad_update(K, h, zprev.U, zprev.U, d, gz, out, ef, fc);
      const int p = padded_cell(G, x, y, t - 1);
      Uh.E[p] = out[0];
      Uh.F[0][p] = out[1];
      Uh.F[1][p] = out[2];
      Uh.F[2][p] = out[3];
    }
    zprev = fzs;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      fzprev[q] = fz[q];
      divprev[q] = div[q];
    }
  }
}

template <typename T, int BY>
__global__ void __launch_bounds__(TILE_BX * BY) k_rad_predict_tile(RadPtrs<T> Um, RadPtrs<T> Uh,
                                                                   GasView<T> gas, Geom G,
                                                                   RadConst<T> K, T h, int zc) {
  __shared__ PredictShared<T, BY> sh;
  rad_predict_tile_body<T, BY>(Um, Uh, gas, G, K, h, zc, int(blockIdx.x), int(blockIdx.y),
                               int(blockIdx.z), sh);
}

// Corrector: MC-limited reconstruction of U^{m+1/2}, HLL fluxes, full step from U^m
// with sources at U^{m+1/2}; U^{m+1} overwrites U^m on the interior of a 3D grid.
// Grid: (ceil(nx/62), ceil(ny/(BY-2)), ceil(nz/zc)).
template <typename T, int BY>
struct CorrectShared {
  T sU[BY + 2][TILE_BX + 2][4];   // U^{m+1/2} of plane t with a one-cell ring
  FaceSide<T> sq[BY][TILE_BX];    // plus-side face data (x faces, then y faces)
  T sf[BY][TILE_BX][4];           // left (x) then bottom (y) face fluxes
};

// One tile (bx, by, bz) of the corrector; called by every thread of the block.
template <typename T, int BY>
__device__ __forceinline__ void rad_correct_tile_body(const RadPtrs<T>& Um, const RadPtrs<T>& Uh,
                                                      const GasView<T>& gas, const Geom& G,
                                                      const RadConst<T>& K, T h, int zc, int bx,
                                                      int by, int bz, unsigned long long* ctr,
                                                      CorrectShared<T, BY>& sh) {
  constexpr int BX = TILE_BX, TX = BX - 2, TY = BY - 2;
  constexpr int RX = BX + 2, RY = BY + 2;
  auto& sU = sh.sU;
  auto& sq = sh.sq;
  auto& sf = sh.sf;
  const int tx = int(threadIdx.x), ty = int(threadIdx.y);
  const int tid = tx + BX * ty;
  const int n0 = G.n[0], n1 = G.n[1], n2 = G.n[2];
  const int x0 = bx * TX, y0 = by * TY;
  const int x = x0 + tx - 1, y = y0 + ty - 1;
  const bool out_xy = tx >= 1 && tx <= TX && ty >= 1 && ty <= TY && x < n0 && y < n1;
  const int z0 = bz * zc;
  const int z1 = min(z0 + zc, n2);
  // the half-step arrays hold valid values on [-2, n + 2)
  const int xl = clamp_i(x, -2, n0 + 1), yl = clamp_i(y, -2, n1 + 1);
  const int zstride = G.ps[0] * G.ps[1];
  const int pcol = padded_cell(G, xl, yl, 0);
  const T c = K.c, ic = K.inv_c, chat = K.chat;

  T Uzm[4], Uz0[4], Uzp[4];
  load_padded4(Uh, pcol + (z0 - 2) * zstride, Uzm);
  load_padded4(Uh, pcol + (z0 - 1) * zstride, Uz0);
  FaceSide<T> zplus;  // plus-z face data of plane t-1
  T fzprev[4] = {T(0), T(0), T(0), T(0)};
  T divprev[4] = {T(0), T(0), T(0), T(0)};
  T Uhprev[4] = {T(0), T(0), T(0), T(0)};
  unsigned long long nef = 0, nfc = 0;
  for (int t = z0 - 1; t <= z1; ++t) {
    load_padded4(Uh, pcol + (t + 1) * zstride, Uzp);
    for (int idx = tid; idx < RX * RY; idx += BX * BY) {
      const int ix = idx % RX, iy = idx / RX;
      const int gx = clamp_i(x0 - 2 + ix, -2, n0 + 1);
      const int gy = clamp_i(y0 - 2 + iy, -2, n1 + 1);
      const int p = padded_cell(G, gx, gy, t);
      sU[iy][ix][0] = Uh.E[p];
      sU[iy][ix][1] = Uh.F[0][p];
      sU[iy][ix][2] = Uh.F[1][p];
      sU[iy][ix][3] = Uh.F[2][p];
    }
    __syncthreads();
    const bool xy = t >= z0 && t < z1;
    // limited slopes and the face states of this cell
    T mx[4], px[4], my[4], py[4], mz[4], pz[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const T u = Uz0[q];
      const T sxq = mc_slope(u - sU[ty + 1][tx][q], sU[ty + 1][tx + 2][q] - u);
      const T syq = mc_slope(u - sU[ty][tx + 1][q], sU[ty + 2][tx + 1][q] - u);
      const T szq = mc_slope(u - Uzm[q], Uzp[q] - u);
      mx[q] = u - T(0.5) * sxq;
      px[q] = u + T(0.5) * sxq;
      my[q] = u - T(0.5) * syq;
      py[q] = u + T(0.5) * syq;
      mz[q] = u - T(0.5) * szq;
      pz[q] = u + T(0.5) * szq;
    }
    T fl[4] = {T(0), T(0), T(0), T(0)}, fb[4] = {T(0), T(0), T(0), T(0)}, fr[4] = {T(0), T(0), T(0), T(0)};
    if (xy) sq[ty][tx] = face_side(px, 0, c, ic, chat);
    __syncthreads();
    if (xy && tx >= 1) hll(sq[ty][tx - 1], face_side(mx, 0, c, ic, chat), fl);
    __syncthreads();
    if (xy) {
      sq[ty][tx] = face_side(py, 1, c, ic, chat);
#pragma unroll
      for (int q = 0; q < 4; ++q) sf[ty][tx][q] = fl[q];
    }
    __syncthreads();
    if (xy) {
      if (tx < BX - 1) {
#pragma unroll
        for (int q = 0; q < 4; ++q) fr[q] = sf[ty][tx + 1][q];
      }
      if (ty >= 1) hll(sq[ty - 1][tx], face_side(my, 1, c, ic, chat), fb);
    }
    __syncthreads();
    if (xy) {
#pragma unroll
      for (int q = 0; q < 4; ++q) sf[ty][tx][q] = fb[q];
    }
    __syncthreads();
    T div[4] = {T(0), T(0), T(0), T(0)};
    if (xy && tx < BX - 1 && ty < BY - 1) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        div[q] = (fr[q] - fl[q]) * K.inv_w[0] + (sf[ty + 1][tx][q] - fb[q]) * K.inv_w[1];
    }
    T fz[4] = {T(0), T(0), T(0), T(0)};
    if (t > z0 - 1) hll(zplus, face_side(mz, 2, c, ic, chat), fz);
    if (t > z0 && out_xy) {
      T d[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) d[q] = divprev[q] + (fz[q] - fzprev[q]) * K.inv_w[2];
      const int a = x + n0 * (y + n1 * (t - 1));
      const int s[3] = {1, 1, 1};
      const Frozen<T> gz = frozen_at(gas, a, s, K.beta != 0);
      T Uo[4] = {Um.E[a], Um.F[0][a], Um.F[1][a], Um.F[2][a]};
      T out[4];
      bool ef, fc;
      rad_update(K, h, Uo, Uhprev, d, gz, out, ef, fc);
      nef += ef ? 1ull : 0ull;
      nfc += fc ? 1ull : 0ull;
      Um.E[a] = out[0];
      Um.F[0][a] = out[1];
      Um.F[1][a] = out[2];
      Um.F[2][a] = out[3];
    }
    if (t < z1) zplus = face_side(pz, 2, c, ic, chat);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      fzprev[q] = fz[q];
      divprev[q] = div[q];
      Uhprev[q] = Uz0[q];
      Uzm[q] = Uz0[q];
      Uz0[q] = Uzp[q];
    }
  }
  wave_add(ctr + CTR_RAD_EFLOOR, nef);
  wave_add(ctr + CTR_RAD_FCLAMP, nfc);
}

template <typename T, int BY>
__global__ void __launch_bounds__(TILE_BX * BY) k_rad_correct_tile(RadPtrs<T> Um, RadPtrs<T> Uh,
                                                                   GasView<T> gas, Geom G,
                                                                   RadConst<T> K, T h, int zc,
                                                                   unsigned long long* ctr) {
  __shared__ CorrectShared<T, BY> sh;
  rad_correct_tile_body<T, BY>(Um, Uh, gas, G, K, h, zc, int(blockIdx.x), int(blockIdx.y),
                               int(blockIdx.z), ctr, sh);
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
  unsigned long long* ctr;
};

// Tile i of a launch is (solve, bx, by, bz) = tiles[i]; blocks past ntiles exit at once,
// so one grid size serves every round.
template <typename T, int BY>
__global__ void __launch_bounds__(TILE_BX * BY) k_rad_predict_batch(const SolveDesc<T>* __restrict__ sd,
                                                                    const int4* __restrict__ tiles,
                                                                    const int* __restrict__ ntiles,
                                                                    int zc) {
  if (int(blockIdx.x) >= *ntiles) return;
  const int4 tr = tiles[blockIdx.x];
  const SolveDesc<T> d = sd[tr.x];
  __shared__ PredictShared<T, BY> sh;
  rad_predict_tile_body<T, BY>(d.Um, d.Uh, d.gas, d.G, d.K, d.h_pred, zc, tr.y, tr.z, tr.w, sh);
}

template <typename T, int BY>
__global__ void __launch_bounds__(TILE_BX * BY) k_rad_correct_batch(const SolveDesc<T>* __restrict__ sd,
                                                                    const int4* __restrict__ tiles,
                                                                    const int* __restrict__ ntiles,
                                                                    int zc) {
  if (int(blockIdx.x) >= *ntiles) return;
  const int4 tr = tiles[blockIdx.x];
  const SolveDesc<T> d = sd[tr.x];
  __shared__ CorrectShared<T, BY> sh;
  rad_correct_tile_body<T, BY>(d.Um, d.Uh, d.gas, d.G, d.K, d.h_corr, zc, tr.y, tr.z, tr.w, d.ctr, sh);
}

}  // namespace rhdk
