// rhd_gas_tile.hpp -- tiled gas Van Leer stages for 3D grids (gfx950).
//
// The tiling of the radiation stages (rhd_tile.hpp) applied to the gas: a block of
// 64 x BY threads owns 64 x BY cells of an x-y tile, one wavefront per x-row, and walks a
// chunk of z planes. Each thread evaluates the primitives of its own cell once and solves
// the Riemann problems of the faces on the low side of its cell, with its x and y
// neighbours' primitives in LDS and its z neighbour's in registers of the previous plane,
// so every face is solved once. Extra work items on wavefronts of different SIMDs bring
// the primitives just outside the tile and solve the faces on its high x and y edges. The
// predictor writes U^{n+1/2} on the interior plus two ghost layers (its ghost columns in
// x come from one extra block per y-z tile, cell by cell); the corrector overwrites U^n
// with U^{n+1,*} on the interior and keeps s_n and (rho, v)^{n+1/2} for the correction.
// Both produce what the per-cell kernels of rhd_device.hpp produce, to rounding.
#pragma once

#include "rhd_tile.hpp"

namespace rhdk {

// Primitives (rho, v, P) of R x C cells: (rho, v) as one vector, P beside it.
template <typename T, int R, int C>
struct PrimTile {
  V4<T> a[R][C];
  T p[R][C];
  __device__ __forceinline__ void put(int r, int c, const T W[5]) {
    put4(a[r][c], W);
    p[r][c] = W[4];
  }
  __device__ __forceinline__ void get(int r, int c, T W[5]) const {
    get4(a[r][c], W);
    W[4] = p[r][c];
  }
};

// Five-component fluxes of R x C faces.
template <typename T, int R, int C>
struct FluxTile {
  V4<T> a[R][C];
  T e[R][C];
  __device__ __forceinline__ void put(int r, int c, const T f[5]) {
    put4(a[r][c], f);
    e[r][c] = f[4];
  }
  __device__ __forceinline__ void get(int r, int c, T f[5]) const {
    get4(a[r][c], f);
    f[4] = e[r][c];
  }
};

// U_g of the boundary-mapped cell (i, j, k) as loaded; neg marks the momentum components
// a reflecting boundary flips (apply with unflip_gas before use).
template <typename T>
__device__ __forceinline__ void load_gas_raw(const GasPtrs<T>& Gp, const Geom& G, int i, int j,
                                             int k, T U[5], int& neg) {
  int s[3];
  const int a = mapped_cell(G, i, j, k, s);
  U[0] = Gp.rho[a];
  U[1] = Gp.m[0][a];
  U[2] = Gp.m[1][a];
  U[3] = Gp.m[2][a];
  U[4] = Gp.E[a];
  neg = neg_mask(s);
}

template <typename T>
__device__ __forceinline__ void unflip_gas(T U[5], int neg) {
  U[1] = flip(U[1], neg, 1);
  U[2] = flip(U[2], neg, 2);
  U[3] = flip(U[3], neg, 4);
}

template <typename T>
__device__ __forceinline__ void load_gas_padded(const GasPtrs<T>& Gp, int p, T U[5]) {
  U[0] = Gp.rho[p];
  U[1] = Gp.m[0][p];
  U[2] = Gp.m[1][p];
  U[3] = Gp.m[2][p];
  U[4] = Gp.E[p];
}

// The radiation data and flux opacity one cell's gas source needs, as loaded.
template <typename T>
struct GasRadRaw {
  T Er, F[3], kF;
  int neg;
};

template <typename T>
__device__ __forceinline__ GasRadRaw<T> gas_rad_load(const RadPtrs<T>& Ur, const T* kF, T kF_s,
                                                     int a, const int s[3]) {
  GasRadRaw<T> r;
  r.Er = Ur.E[a];
  r.F[0] = Ur.F[0][a];
  r.F[1] = Ur.F[1][a];
  r.F[2] = Ur.F[2][a];
  r.kF = kF ? kF[a] : kF_s;
  r.neg = neg_mask(s);
  return r;
}

// S_e,gas of a cell with primitives W and the loaded radiation data r.
template <typename T>
__device__ __forceinline__ void gas_source_at(const GasConst<T>& K, const T W[5],
                                              const GasRadRaw<T>& r, T S[5]) {
  const T F[3] = {flip(r.F[0], r.neg, 1), flip(r.F[1], r.neg, 2), flip(r.F[2], r.neg, 4)};
  const T v[3] = {W[1], W[2], W[3]};
  gas_source(K, W[0] * r.kF, v, r.Er, F, S);
}

// ---------------------------------------------------------------------------
// predictor: first-order Riemann fluxes of U^n and S_e,gas(U^n, U_r^n), half step, on
// the interior plus two ghost layers (grid and tiles as the radiation predictor's)
// ---------------------------------------------------------------------------

template <typename T, int BY>
struct GasPredictShared {
  PrimTile<T, BY + 2, TILE_BX + 2> w;  // [r][c]: primitives of cell (x0 - 1 + c, y0 - 1 + r)
  FluxTile<T, BY, TILE_BX + 1> fx;     // [r][i]: flux through the low x face of (x0 + i, y0 + r)
  FluxTile<T, BY + 1, TILE_BX> fy;     // [j][c]: flux through the low y face of (x0 + c, y0 + j)
};

template <typename T, int BY>
__device__ __forceinline__ void gas_predict_tile_body(const GasPtrs<T>& Un, const GasPtrs<T>& Uh,
                                                      const RadPtrs<T>& Ur, const T* kF, T kF_s,
                                                      const Geom& G, const GasConst<T>& K, T h,
                                                      int zc, int bx, int by, int bz,
                                                      GasPredictShared<T, BY>& sh) {
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
      if (y0 + r < ylim) gas_predict_cell(Un, Uh, Ur, kF, kF_s, G, K, h, x, y0 + r, z0 + p);
    }
    return;
  }
  const int x0 = bx * TILE_BX;
  const int x = x0 + tx, y = y0 + ty;
  // every read stays within [-3, n + 2], where the boundary mapping is defined
  const int xl = min(x, n0 + 2), yl = min(y, n1 + 2);
  const bool out_xy = x < n0 && y < n1 + 2;
  // extra items as in the radiation predictor: before the first barrier wave 0 brings the
  // primitives of row y0 - 1, wave 1 those of row y0 + BY and lanes < 2 BY of wave 2 those
  // of cells x0 - 1 and x0 + 64 of row lane mod BY; between the barriers wave 3 solves the
  // high y faces and lanes < BY of wave 0 the high x faces
  const int hrole = ty == 0 ? 1 : (ty == 1 ? 2 : ((ty == 2 && tx < 2 * BY) ? 3 : 0));
  const int hrow = tx % BY;
  const int hx = hrole == 3 ? (tx < BY ? x0 - 1 : min(x0 + TILE_BX, n0 + 2)) : xl;
  const int hy = hrole == 1 ? y0 - 1 : (hrole == 2 ? min(y0 + BY, n1 + 2) : min(y0 + hrow, n1 + 2));
  const int hr = hrole == 1 ? 0 : (hrole == 2 ? BY + 1 : hrow + 1);
  const int hc = hrole == 3 ? (tx < BY ? 0 : TILE_BX + 1) : tx + 1;

  // loads run one plane ahead of their use
  T Un_[5], Hn[5] = {T(0), T(0), T(0), T(0), T(0)};
  int nU, nH = 0;
  load_gas_raw(Un, G, xl, yl, z0 - 1, Un_, nU);
  if (hrole) load_gas_raw(Un, G, hx, hy, z0, Hn, nH);
  GasRadRaw<T> rn = {};

  T Wprev[5], Uprev[5];  // plane t-1
  T fzprev[5] = {T(0), T(0), T(0), T(0), T(0)};
  T divprev[5] = {T(0), T(0), T(0), T(0), T(0)};
  for (int t = z0 - 1; t <= z1; ++t) {
    T U[5] = {Un_[0], Un_[1], Un_[2], Un_[3], Un_[4]};
    unflip_gas(U, nU);
    if (t < z1) load_gas_raw(Un, G, xl, yl, t + 1, Un_, nU);
    T W[5];
    gas_prim(K, U, W);
    // z face t-1/2, then plane t-1 is complete: its z faces are t-3/2 and t-1/2
    T fz[5] = {T(0), T(0), T(0), T(0), T(0)};
    if (t > z0 - 1) gas_riemann(K, Wprev, W, 2, fz);
    if (t > z0 && out_xy) {
      T S[5], out[5];
      gas_source_at(K, Wprev, rn, S);
#pragma unroll
      for (int q = 0; q < 5; ++q)
        out[q] = Uprev[q] - h * (divprev[q] + (fz[q] - fzprev[q]) * K.inv_w[2]) + h * S[q];
      if (K.iso) out[4] = Uprev[4];
      bool rf, pf;
      gas_floors(K, out, rf, pf);
      const int p = padded_cell(G, x, y, t - 1);
      Uh.rho[p] = out[0];
      Uh.m[0][p] = out[1];
      Uh.m[1][p] = out[2];
      Uh.m[2][p] = out[3];
      Uh.E[p] = out[4];
    }
    if (t >= z0 && t < z1) {
      int s[3];
      const int a = mapped_cell(G, xl, yl, t, s);
      rn = gas_rad_load(Ur, kF, kF_s, a, s);
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      Wprev[q] = W[q];
      Uprev[q] = U[q];
      fzprev[q] = fz[q];
    }
    if (t >= z0 && t < z1) {
      // x and y faces of plane t
      sh.w.put(ty + 1, tx + 1, W);
      if (hrole) {
        T H[5] = {Hn[0], Hn[1], Hn[2], Hn[3], Hn[4]}, HW[5];
        unflip_gas(H, nH);
        gas_prim(K, H, HW);
        sh.w.put(hr, hc, HW);
        if (t + 1 < z1) load_gas_raw(Un, G, hx, hy, t + 1, Hn, nH);
      }
      __syncthreads();
      T fl[5], fb[5];
      {
        T Wn[5];
        sh.w.get(ty + 1, tx, Wn);
        gas_riemann(K, Wn, W, 0, fl);
        sh.w.get(ty, tx + 1, Wn);
        gas_riemann(K, Wn, W, 1, fb);
      }
      sh.fx.put(ty, tx, fl);
      sh.fy.put(ty, tx, fb);
      if (ty == 0 && tx < BY) {
        T A[5], B[5], f[5];
        sh.w.get(tx + 1, TILE_BX, A);
        sh.w.get(tx + 1, TILE_BX + 1, B);
        gas_riemann(K, A, B, 0, f);
        sh.fx.put(tx, TILE_BX, f);
      }
      if (ty == 3) {
        T A[5], B[5], f[5];
        sh.w.get(BY, tx + 1, A);
        sh.w.get(BY + 1, tx + 1, B);
        gas_riemann(K, A, B, 1, f);
        sh.fy.put(BY, tx, f);
      }
      __syncthreads();
      T fr[5], ft[5];
      sh.fx.get(ty, tx + 1, fr);
      sh.fy.get(ty + 1, tx, ft);
#pragma unroll
      for (int q = 0; q < 5; ++q)
        divprev[q] = (fr[q] - fl[q]) * K.inv_w[0] + (ft[q] - fb[q]) * K.inv_w[1];
    }
  }
}

template <typename T, int BY>
__global__ void __launch_bounds__(TILE_BX * BY, sizeof(T) == 4 ? 4 : 2) k_gas_predict_tile(GasPtrs<T> Un, GasPtrs<T> Uh,
                                                                   RadPtrs<T> Ur, const T* kF,
                                                                   T kF_s, Geom G, GasConst<T> K,
                                                                   T h, int zc) {
  __shared__ GasPredictShared<T, BY> sh;
  int bx, by, bz;
  xcd_block(bx, by, bz);
  gas_predict_tile_body<T, BY>(Un, Uh, Ur, kF, kF_s, G, K, h, zc, bx, by, bz, sh);
}

// ---------------------------------------------------------------------------
// corrector: MC-limited reconstruction of the primitives of U^{n+1/2}, Riemann fluxes,
// full step from U^n with S_e,gas(U^{n+1/2}, U_r^n) (grid and tiles as the radiation
// corrector's)
// ---------------------------------------------------------------------------

template <typename T, int BY>
struct GasCorrectShared {
  PrimTile<T, BY + 4, TILE_BX + 4> w;  // [r][c]: primitives of U^{n+1/2} at (x0 - 2 + c, y0 - 2 + r)
  FluxTile<T, BY, TILE_BX + 1> fx;
  FluxTile<T, BY + 1, TILE_BX> fy;
};

// Riemann flux through the face between cells b and c of the row a, b, c, d along dir,
// from the MC-limited primitive states of b (high side) and c (low side).
template <typename T>
__device__ __forceinline__ void gas_face_flux(const GasConst<T>& K, const T a[5], const T b[5],
                                              const T c[5], const T d[5], int dir, T f[5]) {
  T L[5], R[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    L[q] = b[q] + mc_half_slope(b[q] - a[q], c[q] - b[q]);
    R[q] = c[q] - mc_half_slope(c[q] - b[q], d[q] - c[q]);
  }
  gas_riemann(K, L, R, dir, f);
}

template <typename T, int BY>
__device__ __forceinline__ void gas_correct_tile_body(
    const GasPtrs<T>& Un, const GasPtrs<T>& Uh, const RadPtrs<T>& Ur, const T* kF, T kF_s,
    const Geom& G, const GasConst<T>& K, T h, int zc, int bx, int by, int bz, T* sn0, T* sn1,
    T* sn2, T* sn3, T* wh0, T* wh1, T* wh2, T* wh3, unsigned long long* ctr,
    GasCorrectShared<T, BY>& sh) {
  using Ring = CorrectRing<BY>;
  constexpr int RP = Ring::per_thread;
  const int tx = int(threadIdx.x), ty = int(threadIdx.y);
  const int tid = tx + TILE_BX * ty;
  const int n0 = G.n[0], n1 = G.n[1], n2 = G.n[2];
  const int x0 = bx * TILE_BX, y0 = by * BY;
  const int x = x0 + tx, y = y0 + ty;
  const bool out_xy = x < n0 && y < n1;
  const int z0 = bz * zc;
  const int z1 = min(z0 + zc, n2);
  const int zs = G.ps[0] * G.ps[1];
  // the half-step arrays hold valid values on [-2, n + 2) in every dimension
  const int pcol = padded_cell(G, clamp_i(x, -2, n0 + 1), clamp_i(y, -2, n1 + 1), 0);
  int rr[RP], rcc[RP], rcol[RP];
#pragma unroll
  for (int s = 0; s < RP; ++s) {
    const int e = tid + s * Ring::threads;
    rr[s] = -1;
    rcc[s] = 0;
    rcol[s] = 0;
    if (e < Ring::cells) {
      Ring::rc(e, rr[s], rcc[s]);
      rcol[s] = padded_cell(G, clamp_i(x0 - 2 + rcc[s], -2, n0 + 1),
                            clamp_i(y0 - 2 + rr[s], -2, n1 + 1), 0);
    }
  }

  T Wzm[5], Wz0[5], Wzp[5], Upp[5];
  {
    T U[5];
    load_gas_padded(Uh, pcol + (z0 - 2) * zs, U);
    gas_prim(K, U, Wzm);
    load_gas_padded(Uh, pcol + (z0 - 1) * zs, U);
    gas_prim(K, U, Wz0);
    load_gas_padded(Uh, pcol + z0 * zs, U);
    gas_prim(K, U, Wzp);
  }
  T ring[RP][5];
#pragma unroll
  for (int s = 0; s < RP; ++s)
    if (rr[s] >= 0) load_gas_padded(Uh, rcol[s] + z0 * zs, ring[s]);
  // U^n and the radiation data of the cell updated at the next plane, loaded one plane
  // ahead
  const int s1[3] = {1, 1, 1};
  GasRadRaw<T> rn = {};
  T Uon[5] = {T(0), T(0), T(0), T(0), T(0)};
  T zplus[5] = {T(0), T(0), T(0), T(0), T(0)};  // high-z state of plane t-1
  T fzprev[5] = {T(0), T(0), T(0), T(0), T(0)};
  T divprev[5] = {T(0), T(0), T(0), T(0), T(0)};
  unsigned long long nrf = 0, npf = 0;
  for (int t = z0 - 1; t <= z1; ++t) {
    const bool plane = t >= z0 && t < z1;  // planes whose x and y faces are needed
    if (plane) {
      sh.w.put(ty + 2, tx + 2, Wz0);
#pragma unroll
      for (int s = 0; s < RP; ++s) {
        if (rr[s] < 0) continue;
        T W[5];
        gas_prim(K, ring[s], W);
        sh.w.put(rr[s], rcc[s], W);
        if (t + 1 < z1) load_gas_padded(Uh, rcol[s] + (t + 1) * zs, ring[s]);
      }
    }
    if (t < z1) load_gas_padded(Uh, pcol + (t + 2) * zs, Upp);
    {
      // z: limited states of the own cell; the low z face pairs them with plane t-1
      T mz[5], pz[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        const T sz = mc_half_slope(Wz0[q] - Wzm[q], Wzp[q] - Wz0[q]);
        mz[q] = Wz0[q] - sz;
        pz[q] = Wz0[q] + sz;
      }
      T fz[5] = {T(0), T(0), T(0), T(0), T(0)};
      if (t > z0 - 1) gas_riemann(K, zplus, mz, 2, fz);
      if (t > z0 && out_xy) {
        // plane t-1 is complete: its z faces are t-3/2 (fzprev) and t-1/2 (fz)
        const int a = x + n0 * (y + n1 * (t - 1));
        T S[5], out[5];
        gas_source_at(K, Wzm, rn, S);
#pragma unroll
        for (int q = 0; q < 5; ++q)
          out[q] = Uon[q] - h * (divprev[q] + (fz[q] - fzprev[q]) * K.inv_w[2]) + h * S[q];
        if (K.iso) out[4] = Uon[4];
        bool rf, pf;
        gas_floors(K, out, rf, pf);
        nrf += rf ? 1ull : 0ull;
        npf += pf ? 1ull : 0ull;
        Un.rho[a] = out[0];
        Un.m[0][a] = out[1];
        Un.m[1][a] = out[2];
        Un.m[2][a] = out[3];
        Un.E[a] = out[4];
        sn0[a] = S[1];
        sn1[a] = S[2];
        sn2[a] = S[3];
        sn3[a] = S[4];
        wh0[a] = Wzm[0];
        wh1[a] = Wzm[1];
        wh2[a] = Wzm[2];
        wh3[a] = Wzm[3];
      }
      if (t >= z0 && t < z1 && out_xy) {
        const int a = x + n0 * (y + n1 * t);
        rn = gas_rad_load(Ur, kF, kF_s, a, s1);
        load_gas_padded(Un, a, Uon);
      }
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        if (t < z1) zplus[q] = pz[q];
        fzprev[q] = fz[q];
      }
    }
    if (plane) {
      __syncthreads();
      T fl[5], fb[5];
      {
        T a[5], b[5], d[5];
        sh.w.get(ty + 2, tx, a);
        sh.w.get(ty + 2, tx + 1, b);
        sh.w.get(ty + 2, tx + 3, d);
        gas_face_flux(K, a, b, Wz0, d, 0, fl);
        sh.w.get(ty, tx + 2, a);
        sh.w.get(ty + 1, tx + 2, b);
        sh.w.get(ty + 3, tx + 2, d);
        gas_face_flux(K, a, b, Wz0, d, 1, fb);
      }
      sh.fx.put(ty, tx, fl);
      sh.fy.put(ty, tx, fb);
      // extra items on waves of different SIMDs (wave w runs on SIMD w mod 4)
      if (ty == 0 && tx < BY) {
        // high x face of row tx: cells x0 + 62 ... x0 + 65
        T a[5], b[5], c[5], d[5], f[5];
        sh.w.get(tx + 2, TILE_BX, a);
        sh.w.get(tx + 2, TILE_BX + 1, b);
        sh.w.get(tx + 2, TILE_BX + 2, c);
        sh.w.get(tx + 2, TILE_BX + 3, d);
        gas_face_flux(K, a, b, c, d, 0, f);
        sh.fx.put(tx, TILE_BX, f);
      }
      if (ty == BY - 1) {
        // high y face of column tx: rows y0 + BY - 2 ... y0 + BY + 1
        T a[5], c[5], d[5], f[5];
        sh.w.get(BY, tx + 2, a);
        sh.w.get(BY + 2, tx + 2, c);
        sh.w.get(BY + 3, tx + 2, d);
        gas_face_flux(K, a, Wz0, c, d, 1, f);
        sh.fy.put(BY, tx, f);
      }
      __syncthreads();
      T fr[5], ft[5];
      sh.fx.get(ty, tx + 1, fr);
      sh.fy.get(ty + 1, tx, ft);
#pragma unroll
      for (int q = 0; q < 5; ++q)
        divprev[q] = (fr[q] - fl[q]) * K.inv_w[0] + (ft[q] - fb[q]) * K.inv_w[1];
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      Wzm[q] = Wz0[q];
      Wz0[q] = Wzp[q];
    }
    if (t < z1) gas_prim(K, Upp, Wzp);
  }
  wave_add(ctr + CTR_GAS_RHOFLOOR, nrf);
  wave_add(ctr + CTR_GAS_PFLOOR, npf);
}

template <typename T, int BY>
__global__ void __launch_bounds__(TILE_BX * BY, sizeof(T) == 4 ? 4 : 2) k_gas_correct_tile(
    GasPtrs<T> Un, GasPtrs<T> Uh, RadPtrs<T> Ur, const T* kF, T kF_s, Geom G, GasConst<T> K,
    T h, int zc, T* sn0, T* sn1, T* sn2, T* sn3, T* wh0, T* wh1, T* wh2, T* wh3,
    unsigned long long* ctr) {
  __shared__ GasCorrectShared<T, BY> sh;
  int bx, by, bz;
  xcd_block(bx, by, bz);
  gas_correct_tile_body<T, BY>(Un, Uh, Ur, kF, kF_s, G, K, h, zc, bx, by, bz, sn0, sn1, sn2,
                               sn3, wh0, wh1, wh2, wh3, ctr, sh);
}

}  // namespace rhdk
