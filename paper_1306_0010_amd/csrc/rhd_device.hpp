// rhd_device.hpp -- device code of the gfx950 library for the gray M1
// radiation-hydrodynamics step of Skinner & Ostriker (2013).
//
// Layout: one array per field (structure of arrays), cell (i, j, k) at
// i + nx*(j + ny*k), x fastest, so a wavefront reads 64 consecutive x-cells of a field
// in one coalesced access. Boundary conditions are applied by index mapping when a
// stencil reads outside the grid (periodic wrap, zero-gradient clamp, mirror with the
// normal vector components negated), so no ghost-fill pass touches HBM.
//
// The half-step states of the Van Leer predictor live in padded scratch arrays with
// two ghost layers per active dimension: the predictor is evaluated there from the
// boundary-mapped old state, and the corrector reads those predicted ghost values
// directly (no boundary refill between the two stages).
//
// T is the type of the stencil arithmetic and of the stored state (double in FP64
// mode, float in mixed mode). The energy exchange, the ledger and all counters are
// FP64 / 64-bit whatever T is.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace rhdk {

enum { BC_PERIODIC = 0, BC_OUTFLOW = 1, BC_REFLECT = 2, BC_FIXED = 3 };

enum {
  CTR_EXCH_THETA1 = 0,
  CTR_EXCH_BISECT,
  CTR_NEWTON_ITERS,
  CTR_NEWTON_MAX,
  CTR_RAD_FCLAMP,
  CTR_RAD_EFLOOR,
  CTR_GAS_RHOFLOOR,
  CTR_GAS_PFLOOR,
  CTR_NONFINITE,
  CTR_FIRST_BAD,
  CTR_COUNT
};

struct Geom {
  int n[3];    // interior cells per dimension
  int act[3];  // 1 when the dimension is active (n > 1)
  int bc[6];   // boundary kind per face
  int g[3];    // ghost width of the padded half-step arrays (2 if active, else 0)
  int ps[3];   // padded extents n + 2 g
};

template <typename T>
struct RadPtrs {
  T* E;
  T* F[3];
};

template <typename T>
struct GasPtrs {
  T* rho;
  T* m[3];
  T* E;
};

// Frozen gas seen by the radiation subcycles.
template <typename T>
struct GasView {
  const T* rho;
  const T* m[3];
  const T* kP;  // per-cell specific opacity, or null for the scalar below
  const T* kF;
  const T* j;   // emissivity or null
  T kP_s, kF_s;
};

template <typename T>
struct RadConst {
  T c, inv_c, chat;
  T fclo;      // 1/c, or 0 for the P1 closure (f is taken as 0 in the closure: T = I/3)
  T inv_w[3];
  T theta;
  T er_floor;
  int beta;    // O(beta tau) terms on
  int absorb;  // absorption-only mode: E_r damped with kappa_P on each stage
};

// Element i of a device array. With O32 the address is the array's base plus a 32-bit
// byte offset: an SGPR pair and one VGPR, with no 64-bit address arithmetic per access.
// The tiled radiation kernels use it; the host runs them only on grids whose arrays hold
// at most 4 GiB each.
template <bool O32, typename T>
__device__ __forceinline__ T& elem(T* p, int i) {
  if constexpr (O32) {
    using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
    return *reinterpret_cast<T*>(reinterpret_cast<B*>(p) + unsigned(i) * unsigned(sizeof(T)));
  } else {
    return p[i];
  }
}

// Radiation state (E_r, F_x, F_y, F_z) of each fixed (Dirichlet) face; bit f of mask
// marks face f = x-, x+, y-, y+, z-, z+ as fixed.
template <typename T>
struct FixedFaces {
  T v[6][4];
  int mask;
};

template <typename T>
struct GasConst {
  T c, inv_c;
  T inv_w[3];
  T gamma, gm1, cs2;
  T rho_floor, p_floor;
  int beta;
  int iso;
};

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

// Source index of coordinate q (in [-2n, 3n)) after the boundary mapping of one
// dimension, and the sign the vector component along that dimension takes there.
// Written with selects only: a branchy form of this mapping, with the sign updated
// through a reference inside the branches, was compiled for wave-uniform coordinates
// (y and z rows) so that the reflecting high face lost its sign change.
__device__ __forceinline__ int map_index(int q, int n, int lo, int hi, int& sign) {
  const bool low = q < 0;
  const bool high = q >= n;
  const int kind = low ? lo : (high ? hi : -1);
  int per = q + (q < 0 ? n : 0);
  per += per < 0 ? n : 0;
  per -= per >= n ? n : 0;
  per -= per >= n ? n : 0;
  const int clamp = low ? 0 : n - 1;
  const int mirror = low ? -1 - q : 2 * n - 1 - q;
  // a fixed face maps like an outflow face; its radiation state replaces the radiation
  // fields where the radiation stages read them (fixed_face below)
  const int r = kind == BC_PERIODIC
                    ? per
                    : ((kind == BC_OUTFLOW || kind == BC_FIXED) ? clamp : (kind == BC_REFLECT ? mirror : q));
  sign = kind == BC_REFLECT ? -sign : sign;
  return r;
}

// Flat interior index of a possibly out-of-range cell after boundary mapping, and
// the sign each vector component takes there.
__device__ __forceinline__ int mapped_cell(const Geom& G, int i, int j, int k, int s[3]) {
  s[0] = s[1] = s[2] = 1;
  int si = G.act[0] ? map_index(i, G.n[0], G.bc[0], G.bc[1], s[0]) : 0;
  int sj = G.act[1] ? map_index(j, G.n[1], G.bc[2], G.bc[3], s[1]) : 0;
  int sk = G.act[2] ? map_index(k, G.n[2], G.bc[4], G.bc[5], s[2]) : 0;
  return si + G.n[0] * (sj + G.n[1] * sk);
}

__device__ __forceinline__ int padded_cell(const Geom& G, int i, int j, int k) {
  return (i + G.g[0]) + G.ps[0] * ((j + G.g[1]) + G.ps[1] * (k + G.g[2]));
}

__device__ __forceinline__ bool is_interior(const Geom& G, int i, int j, int k) {
  return i >= 0 && i < G.n[0] && j >= 0 && j < G.n[1] && k >= 0 && k < G.n[2];
}

template <typename T>
__device__ __forceinline__ T tmin(T a, T b) { return a < b ? a : b; }
template <typename T>
__device__ __forceinline__ T tmax(T a, T b) { return a > b ? a : b; }
// IEEE minNum / maxNum: one v_min / v_max (or a v_min3 / v_max3 for a nest), for values
// that are finite by construction.
__device__ __forceinline__ float vmin(float a, float b) { return __builtin_fminf(a, b); }
__device__ __forceinline__ double vmin(double a, double b) { return __builtin_fmin(a, b); }
__device__ __forceinline__ float vmax(float a, float b) { return __builtin_fmaxf(a, b); }
__device__ __forceinline__ double vmax(double a, double b) { return __builtin_fmax(a, b); }

// Monotonised-central limited slope: minmod(2 dm, 2 dp, (dm + dp)/2), zero unless the
// one-sided differences dm and dp share a sign.
__device__ __forceinline__ double mc_slope(double dm, double dp) {
  if (dm * dp <= 0.0) return 0.0;
  const double a = fabs(0.5 * (dm + dp));
  const double b = 2.0 * fabs(dm);
  const double e = 2.0 * fabs(dp);
  const double m = tmin(a, tmin(b, e));
  return dm > 0.0 ? m : -m;
}

// Half the limited slope, the offset from the cell value to its face states. FP32:
// minmod(a, b) is the median of (a, b, 0), the three-argument minmod is
// minmod(a, minmod(b, c)), and halving every argument of a median halves it exactly,
// so the half slope is minmod(dm, dp, (dm + dp)/4): two v_med3_f32, no branch.
__device__ __forceinline__ double mc_half_slope(double dm, double dp) {
  return 0.5 * mc_slope(dm, dp);
}
__device__ __forceinline__ float mc_half_slope(float dm, float dp) {
  const float inner = __builtin_amdgcn_fmed3f(dp, 0.25f * (dm + dp), 0.0f);
  return __builtin_amdgcn_fmed3f(dm, inner, 0.0f);
}

// Sum of v over the wavefront; lane 0 adds it to *ctr. Every lane must call it.
__device__ __forceinline__ void wave_add(unsigned long long* ctr, unsigned long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if (__lane_id() == 0 && v != 0ull) atomicAdd(ctr, v);
}

__device__ __forceinline__ void wave_max(unsigned long long* ctr, unsigned long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    unsigned long long o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  if (__lane_id() == 0 && v != 0ull) atomicMax(ctr, v);
}

// ---------------------------------------------------------------------------
// M1 closure, eigenvalues and HLL flux (Sec. 2.3, Sec. 3.3)
// ---------------------------------------------------------------------------

// Reciprocal and square roots: the hardware approximations (about 1 ulp) in FP32,
// correctly rounded operations in FP64.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }
__device__ __forceinline__ float rsqrt_(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_(double x) { return 1.0 / sqrt(x); }
// a / b: the hardware reciprocal times a in FP32 (about 1.5 ulp), a correctly rounded
// division in FP64.
__device__ __forceinline__ float vdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double vdiv(double a, double b) { return a / b; }

// Smallest normal number of each precision.
template <typename T>
__device__ __forceinline__ constexpr T min_normal() {
  if constexpr (sizeof(T) == 4)
    return T(1.17549435e-38f);
  else
    return T(2.2250738585072014e-308);
}

// Direction-independent part of the M1 closure of one state (E_r, F).
//
// With the reduced flux f = F/(c E) (norm clamped to 1) and s = sqrt(4 - 3 f^2), the
// Eddington factor of Eq. m1:chi equals (5 - 2 s)/3, so the tensor of Eq. m1:m1tns is
//   T = (s - 1)/3 I + 3 f f / (2 + s),
// with no division by |F| and no special case at F = 0. One reciprocal of s (2 + s)
// gives both 1/s (for the wave speeds) and 3/(2 + s).
template <typename T>
struct M1State {
  T E, F[3];     // the state
  T f[3];        // reduced flux after the clamp
  T s;           // sqrt(4 - 3 f^2)
  T iso;         // (s - 1)/3, the isotropic part of T
  T dir;         // 3/(2 + s), the f f part of T
  T chat_s;      // chat / s
};

template <typename T>
__device__ __forceinline__ M1State<T> m1_state(const T U[4], T fclo, T chat) {
  M1State<T> m;
  m.E = U[0];
  m.F[0] = U[1];
  m.F[1] = U[2];
  m.F[2] = U[3];
  const T icE = fclo * rcp(U[0]);
  m.f[0] = U[1] * icE;
  m.f[1] = U[2] * icE;
  m.f[2] = U[3] * icE;
  T ff = m.f[0] * m.f[0] + m.f[1] * m.f[1] + m.f[2] * m.f[2];
  if (!(ff <= T(1))) {
    // f = F/|F|, taken from F itself: near E_r = 0 the product F/(c E_r) overflows,
    // and a zero component of F times an infinite 1/(c E_r) is NaN (so is ff then).
    // ff is then exactly 1, as the branch point of the closure at f = 1 needs. In FP32
    // |F|^2 is kept normal for the hardware reciprocal square root; below that f falls
    // short of unit length, and ff is taken from f.
    const T n2 = U[1] * U[1] + U[2] * U[2] + U[3] * U[3];
    T r;
    if constexpr (sizeof(T) == 4)
      r = rsqrt_(vmax(n2, min_normal<T>()));
    else
      r = rsqrt_(n2);
    m.f[0] = U[1] * r;
    m.f[1] = U[2] * r;
    m.f[2] = U[3] * r;
    ff = T(1);
    if constexpr (sizeof(T) == 4)
      if (n2 < min_normal<T>()) ff = m.f[0] * m.f[0] + m.f[1] * m.f[1] + m.f[2] * m.f[2];
  }
  const T q = T(4) - T(3) * ff;  // s^2, in [1, 4]
  if constexpr (sizeof(T) == 4) {
    // one reciprocal square root gives s and 1/s, one reciprocal 3/(2 + s)
    const T rs = rsqrt_(q);
    m.s = q * rs;
    m.dir = T(3) * rcp(T(2) + m.s);
    m.chat_s = chat * rs;
  } else {
    m.s = sqrt_(q);
    const T two_s = T(2) + m.s;
    const T r2 = rcp(m.s * two_s);
    m.dir = T(3) * m.s * r2;
    m.chat_s = chat * two_s * r2;
  }
  m.iso = (m.s - T(1)) * T(1.0 / 3.0);
  return m;
}

// Physical flux normal to d (chat F_d / c, chat c P_d.) and the extreme wave speeds of
// Eq. hyperbolic:evals13. With mu f = f_d, the radicand
//   (2/3)(4 - 3 f^2 - s) + 2 mu^2 (2 - f^2 - s)
// equals (2/3)(s - 1)(s - 3 f_d^2 / (2 + s)), which is free of 1/|F| and carries the
// factor (s - 1) that vanishes at f = 1 explicitly.
template <typename T>
__device__ __forceinline__ void m1_dir(const M1State<T>& m, int d, T c, T inv_c, T chat,
                                       T Phi[4], T& lmin, T& lmax) {
  const T fd = d == 0 ? m.f[0] : (d == 1 ? m.f[1] : m.f[2]);
  const T scale = (chat * c) * m.E;
  const T a = m.dir * fd;
  Phi[0] = (chat * inv_c) * m.F[d];
  Phi[1] = scale * (a * m.f[0] + (d == 0 ? m.iso : T(0)));
  Phi[2] = scale * (a * m.f[1] + (d == 1 ? m.iso : T(0)));
  Phi[3] = scale * (a * m.f[2] + (d == 2 ? m.iso : T(0)));
  T rad = T(2.0 / 3.0) * (m.s - T(1)) * (m.s - a * fd);
  rad = vmax(rad, T(0));
  const T r = sqrt_(rad);
  lmin = (fd - r) * m.chat_s;
  lmax = (fd + r) * m.chat_s;
}

// Closure data of one state for the faces normal to d: the state, its physical flux and
// its extreme wave speeds.
template <typename T>
struct FaceSide {
  T U[4];
  T Phi[4];
  T lmin, lmax;
};

template <typename T>
__device__ __forceinline__ FaceSide<T> face_side(const T U[4], int d, T c, T inv_c, T fclo,
                                                 T chat) {
  FaceSide<T> q;
  const M1State<T> m = m1_state(U, fclo, chat);
#pragma unroll
  for (int k = 0; k < 4; ++k) q.U[k] = U[k];
  m1_dir(m, d, c, inv_c, chat, q.Phi, q.lmin, q.lmax);
  return q;
}

// HLL flux of Eq. hyperbolic:hllflux2 with S_L = min(lambda_1(U_L), lambda_1(U_R)) and
// S_R = max(lambda_3(U_L), lambda_3(U_R)); the central flux when both bounds vanish.
// A bound difference below the smallest normal number counts as vanishing: its
// reciprocal overflows to infinity while the products it multiplies underflow to zero
// (0 * inf). Such bounds come only from beams with f = 1 parallel to the face (s = 1, a
// zero radicand, a subnormal f_d), whose fluxes through the face are as small, so the
// two fluxes differ by a negligible amount.
template <typename T>
__device__ __forceinline__ void hll(const FaceSide<T>& L, const FaceSide<T>& R, T flux[4]) {
  const T SLm = vmin(vmin(L.lmin, R.lmin), T(0));
  const T SRp = vmax(vmax(L.lmax, R.lmax), T(0));
  const T den = SRp - SLm;
  if (den >= min_normal<T>()) {
    const T id = rcp(den);
    const T pr = SRp * SLm;
#pragma unroll
    for (int q = 0; q < 4; ++q) flux[q] = (SRp * L.Phi[q] - SLm * R.Phi[q] + pr * (R.U[q] - L.U[q])) * id;
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) flux[q] = T(0.5) * (L.Phi[q] + R.Phi[q]);
  }
}

template <typename T>
__device__ __forceinline__ void rad_hll(const T UL[4], const T UR[4], int d, T c, T inv_c,
                                        T fclo, T chat, T flux[4]) {
  hll(face_side(UL, d, c, inv_c, fclo, chat), face_side(UR, d, c, inv_c, fclo, chat), flux);
}

// ---------------------------------------------------------------------------
// radiation stage update (Sec. 3.4)
// ---------------------------------------------------------------------------

template <typename T>
struct Frozen {
  T rkF, rkP;
  T v[3];
  T j;
};

// The gas data of one cell as loaded, before any arithmetic, so that a load can be
// issued well ahead of its use; neg has bit d set where a reflecting boundary flips v_d.
template <typename T>
struct FrozenRaw {
  T rho, kF, kP, m[3], j;
  int neg;
};

__device__ __forceinline__ int neg_mask(const int s[3]) {
  return (s[0] < 0 ? 1 : 0) | (s[1] < 0 ? 2 : 0) | (s[2] < 0 ? 4 : 0);
}

template <typename T>
__device__ __forceinline__ T flip(T v, int neg, int bit) {
  return (neg & bit) ? -v : v;
}

template <typename T, bool O32 = false>
__device__ __forceinline__ FrozenRaw<T> frozen_load(const GasView<T>& g, int a, const int s[3],
                                                    bool need_v) {
  FrozenRaw<T> r;
  r.rho = elem<O32>(g.rho, a);
  r.kF = g.kF ? elem<O32>(g.kF, a) : g.kF_s;
  r.kP = g.kP ? elem<O32>(g.kP, a) : g.kP_s;
  if (need_v) {
    r.m[0] = elem<O32>(g.m[0], a);
    r.m[1] = elem<O32>(g.m[1], a);
    r.m[2] = elem<O32>(g.m[2], a);
  } else {
    r.m[0] = r.m[1] = r.m[2] = T(0);
  }
  r.j = g.j ? g.j[a] : T(0);
  r.neg = neg_mask(s);
  return r;
}

template <typename T>
__device__ __forceinline__ Frozen<T> frozen_make(const FrozenRaw<T>& r, bool need_v) {
  Frozen<T> fz;
  fz.rkF = r.rho * r.kF;
  fz.rkP = r.rho * r.kP;
  if (need_v) {
    const T ir = rcp(r.rho);
    fz.v[0] = flip(r.m[0], r.neg, 1) * ir;
    fz.v[1] = flip(r.m[1], r.neg, 2) * ir;
    fz.v[2] = flip(r.m[2], r.neg, 4) * ir;
  } else {
    fz.v[0] = fz.v[1] = fz.v[2] = T(0);
  }
  fz.j = r.j;
  return fz;
}

template <typename T>
__device__ __forceinline__ Frozen<T> frozen_at(const GasView<T>& g, int a, const int s[3],
                                               bool need_v) {
  return frozen_make(frozen_load(g, a, s, need_v), need_v);
}

// New (E_r, F) of a stage of length h from the old state Uo, the flux divergence and
// the explicit sources at Us. F gets the theta-scheme absorption of
// Eq. source:stiff:radmomentum:soln with the divergence and the explicit terms on the
// same implicit footing; E_r gets the same form with kappa_P in absorption-only mode
// (Eq. source:stiff:radenergy:soln). Then E_r >= er_floor and |F| <= c E_r.
template <typename T>
__device__ __forceinline__ void rad_update(const RadConst<T>& K, T h, const T Uo[4],
                                           const T Us[4], const T div[4], const Frozen<T>& fz,
                                           T out[4], bool& efloor, bool& fclamp) {
  const T chat = K.chat;
  const T b = K.beta ? T(1) : T(0);
  const T th = K.theta;
  const T vF = fz.v[0] * Us[1] + fz.v[1] * Us[2] + fz.v[2] * Us[3];
  const T srcE = b * chat * fz.rkF * vF * K.inv_c * K.inv_c + chat * K.inv_c * fz.j;
  T En;
  if (K.absorb) {
    const T aP = chat * fz.rkP * h;
    En = (Uo[0] * (T(1) - (T(1) - th) * aP) + h * (-div[0] + srcE)) * rcp(T(1) + th * aP);
  } else {
    En = Uo[0] + h * (-div[0] + srcE);
  }
  const T a = chat * fz.rkF * h;
  const T keep = T(1) - (T(1) - th) * a;
  const T inv = rcp(T(1) + th * a);
  const T adv = b * T(4.0 / 3.0) * chat * fz.rkF * Us[0];
  T Fn[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) Fn[q] = (Uo[1 + q] * keep + h * (-div[1 + q] + adv * fz.v[q])) * inv;
  efloor = false;
  fclamp = false;
  if (En < K.er_floor) {
    En = K.er_floor;
    efloor = true;
  }
  const T cE = K.c * En;
  const T Fm2 = Fn[0] * Fn[0] + Fn[1] * Fn[1] + Fn[2] * Fn[2];
  if (Fm2 > cE * cE) {
    // FP32: near the E_r floor both squares can be subnormal, which the hardware
    // reciprocal square root reads as zero (an infinite scale); from the smallest normal
    // up the scale is finite and still brings |F| to at most c E_r
    T m2 = Fm2;
    if constexpr (sizeof(T) == 4) m2 = vmax(Fm2, min_normal<T>());
    const T scale = cE * rsqrt_(m2);
    Fn[0] *= scale;
    Fn[1] *= scale;
    Fn[2] *= scale;
    fclamp = true;
  }
  out[0] = En;
  out[1] = Fn[0];
  out[2] = Fn[1];
  out[3] = Fn[2];
}

// U^m of the boundary-mapped cell (i, j, k) as loaded; neg marks the flux components a
// reflecting boundary flips (apply with unflip_rad before use).
template <typename T, bool O32 = false>
__device__ __forceinline__ void load_rad_raw(const RadPtrs<T>& R, const Geom& G, int i, int j,
                                             int k, T U[4], int& neg) {
  int s[3];
  const int a = mapped_cell(G, i, j, k, s);
  U[0] = elem<O32>(R.E, a);
  U[1] = elem<O32>(R.F[0], a);
  U[2] = elem<O32>(R.F[1], a);
  U[3] = elem<O32>(R.F[2], a);
  neg = neg_mask(s);
}

template <typename T>
__device__ __forceinline__ void unflip_rad(T U[4], int neg) {
  U[1] = flip(U[1], neg, 1);
  U[2] = flip(U[2], neg, 2);
  U[3] = flip(U[3], neg, 4);
}

template <typename T>
__device__ __forceinline__ void load_rad_mapped(const RadPtrs<T>& R, const Geom& G, int i, int j,
                                                int k, T U[4]) {
  int neg;
  load_rad_raw(R, G, i, j, k, U, neg);
  unflip_rad(U, neg);
}

// The fixed face whose radiation state the cell (i, j, k) holds, or -1: of the
// dimensions in which the cell lies beyond a fixed face, the last in the order x, y, z.
__device__ __forceinline__ int fixed_face(const Geom& G, int mask, int i, int j, int k) {
  int f = -1;
  if ((mask & 1) && i < 0) f = 0;
  if ((mask & 2) && i >= G.n[0]) f = 1;
  if ((mask & 4) && j < 0) f = 2;
  if ((mask & 8) && j >= G.n[1]) f = 3;
  if ((mask & 16) && k < 0) f = 4;
  if ((mask & 32) && k >= G.n[2]) f = 5;
  return f;
}

template <typename T>
__device__ __forceinline__ void fixed_state(const FixedFaces<T>& B, int f, T U[4]) {
#pragma unroll
  for (int g = 0; g < 6; ++g)
    if (g == f) {
#pragma unroll
      for (int q = 0; q < 4; ++q) U[q] = B.v[g][q];
    }
}

// U^m of cell (i, j, k): the fixed state beyond a fixed face, else the mapped cell.
template <typename T>
__device__ __forceinline__ void load_rad_bc(const RadPtrs<T>& R, const Geom& G,
                                            const FixedFaces<T>& B, int i, int j, int k, T U[4]) {
  const int f = B.mask ? fixed_face(G, B.mask, i, j, k) : -1;
  if (f >= 0)
    fixed_state(B, f, U);
  else
    load_rad_mapped(R, G, i, j, k, U);
}

// Radiation predictor at one cell (i, j, k) of the padded region: first-order HLL fluxes
// of U^m, half step, result written to the padded half-step arrays.
// A ghost cell beyond a fixed face keeps the face's state in U^{m+1/2} too.
template <typename T>
__device__ __forceinline__ void rad_predict_cell(const RadPtrs<T>& Um, const RadPtrs<T>& Uh,
                                                 const GasView<T>& gas, const Geom& G,
                                                 const RadConst<T>& K, const FixedFaces<T>& B,
                                                 T h, int i, int j, int k) {
  const int p = padded_cell(G, i, j, k);
  const int fb = B.mask ? fixed_face(G, B.mask, i, j, k) : -1;
  if (fb >= 0) {
    T Ub[4];
    fixed_state(B, fb, Ub);
    Uh.E[p] = Ub[0];
    Uh.F[0][p] = Ub[1];
    Uh.F[1][p] = Ub[2];
    Uh.F[2][p] = Ub[3];
    return;
  }
  T U0[4];
  load_rad_bc(Um, G, B, i, j, k, U0);
  const M1State<T> m0 = m1_state(U0, K.fclo, K.chat);
  T div[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (!G.act[d]) continue;
    const int di = d == 0, dj = d == 1, dk = d == 2;
    FaceSide<T> own;
#pragma unroll
    for (int q = 0; q < 4; ++q) own.U[q] = U0[q];
    m1_dir(m0, d, K.c, K.inv_c, K.chat, own.Phi, own.lmin, own.lmax);
    T Ul[4], Ur[4], fl[4], fr[4];
    load_rad_bc(Um, G, B, i - di, j - dj, k - dk, Ul);
    load_rad_bc(Um, G, B, i + di, j + dj, k + dk, Ur);
    hll(face_side(Ul, d, K.c, K.inv_c, K.fclo, K.chat), own, fl);
    hll(own, face_side(Ur, d, K.c, K.inv_c, K.fclo, K.chat), fr);
#pragma unroll
    for (int q = 0; q < 4; ++q) div[q] += (fr[q] - fl[q]) * K.inv_w[d];
  }
  int s[3];
  const int a = mapped_cell(G, i, j, k, s);
  const Frozen<T> fz = frozen_at(gas, a, s, K.beta != 0);
  T out[4];
  bool ef, fc;
  rad_update(K, h, U0, U0, div, fz, out, ef, fc);
  Uh.E[p] = out[0];
  Uh.F[0][p] = out[1];
  Uh.F[1][p] = out[2];
  Uh.F[2][p] = out[3];
}

// Radiation predictor: first-order HLL fluxes of U^m, half step, on the interior plus
// two ghost layers, written to the padded half-step arrays.
template <typename T>
__global__ void __launch_bounds__(256) k_rad_predict(RadPtrs<T> Um, RadPtrs<T> Uh, GasView<T> gas,
                                                     Geom G, RadConst<T> K, FixedFaces<T> B, T h) {
  const int i = int(blockIdx.x * blockDim.x + threadIdx.x) - G.g[0];
  const int j = int(blockIdx.y * blockDim.y + threadIdx.y) - G.g[1];
  const int k = int(blockIdx.z) - G.g[2];
  if (i >= G.n[0] + G.g[0] || j >= G.n[1] + G.g[1]) return;
  rad_predict_cell(Um, Uh, gas, G, K, B, h, i, j, k);
}

template <typename T, bool O32 = false>
__device__ __forceinline__ void load_padded4(const RadPtrs<T>& R, int p, T U[4]) {
  U[0] = elem<O32>(R.E, p);
  U[1] = elem<O32>(R.F[0], p);
  U[2] = elem<O32>(R.F[1], p);
  U[3] = elem<O32>(R.F[2], p);
}

// Radiation corrector at interior cell (i, j, k): MC-limited linear reconstruction of
// U^{m+1/2}, HLL fluxes, full step from U^m with sources at U^{m+1/2}; writes U^{m+1}
// over U^m (U^m is read only in the cell itself). ef / fc report the E_r floor and the
// flux clamp.
template <typename T>
__device__ __forceinline__ void rad_correct_cell(const RadPtrs<T>& Um, const RadPtrs<T>& Uh,
                                                 const GasView<T>& gas, const Geom& G,
                                                 const RadConst<T>& K, T h, int i, int j, int k,
                                                 bool& ef, bool& fc) {
  const int pc = padded_cell(G, i, j, k);
  T Uc[4];
  load_padded4(Uh, pc, Uc);
  T div[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (!G.act[d]) continue;
    const int stride = d == 0 ? 1 : (d == 1 ? G.ps[0] : G.ps[0] * G.ps[1]);
    T Um2[4], Um1[4], Up1[4], Up2[4];
    load_padded4(Uh, pc - 2 * stride, Um2);
    load_padded4(Uh, pc - stride, Um1);
    load_padded4(Uh, pc + stride, Up1);
    load_padded4(Uh, pc + 2 * stride, Up2);
    T Lm[4], Rm[4], Lp[4], Rp[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const T sm = mc_half_slope(Um1[q] - Um2[q], Uc[q] - Um1[q]);
      const T s0 = mc_half_slope(Uc[q] - Um1[q], Up1[q] - Uc[q]);
      const T sp = mc_half_slope(Up1[q] - Uc[q], Up2[q] - Up1[q]);
      Lm[q] = Um1[q] + sm;
      Rm[q] = Uc[q] - s0;
      Lp[q] = Uc[q] + s0;
      Rp[q] = Up1[q] - sp;
    }
    // E_r of a face state is raised to the floor (rounding next to a cell at the floor
    // can take it to zero)
    Lm[0] = vmax(Lm[0], K.er_floor);
    Rm[0] = vmax(Rm[0], K.er_floor);
    Lp[0] = vmax(Lp[0], K.er_floor);
    Rp[0] = vmax(Rp[0], K.er_floor);
    T fl[4], fr[4];
    rad_hll(Lm, Rm, d, K.c, K.inv_c, K.fclo, K.chat, fl);
    rad_hll(Lp, Rp, d, K.c, K.inv_c, K.fclo, K.chat, fr);
#pragma unroll
    for (int q = 0; q < 4; ++q) div[q] += (fr[q] - fl[q]) * K.inv_w[d];
  }
  const int a = i + G.n[0] * (j + G.n[1] * k);
  const int s[3] = {1, 1, 1};
  const Frozen<T> fz = frozen_at(gas, a, s, K.beta != 0);
  T Uo[4] = {Um.E[a], Um.F[0][a], Um.F[1][a], Um.F[2][a]};
  T out[4];
  rad_update(K, h, Uo, Uc, div, fz, out, ef, fc);
  Um.E[a] = out[0];
  Um.F[0][a] = out[1];
  Um.F[1][a] = out[2];
  Um.F[2][a] = out[3];
}

// Radiation corrector on the interior, one thread per cell.
template <typename T>
__global__ void __launch_bounds__(256) k_rad_correct(RadPtrs<T> Um, RadPtrs<T> Uh, GasView<T> gas,
                                                     Geom G, RadConst<T> K, T h,
                                                     unsigned long long* ctr) {
  const int i = int(blockIdx.x * blockDim.x + threadIdx.x);
  const int j = int(blockIdx.y * blockDim.y + threadIdx.y);
  const int k = int(blockIdx.z);
  bool ef = false, fc = false;
  if (i < G.n[0] && j < G.n[1]) rad_correct_cell(Um, Uh, gas, G, K, h, i, j, k, ef, fc);
  wave_add(ctr + CTR_RAD_EFLOOR, ef ? 1ull : 0ull);
  wave_add(ctr + CTR_RAD_FCLAMP, fc ? 1ull : 0ull);
}

// ---------------------------------------------------------------------------
// face-split radiation stages (small grids)
// ---------------------------------------------------------------------------
//
// On grids of a few thousand cells the per-cell kernels above wait on one thread's
// chain of work: every face of its cell in turn. Here a block takes 64 consecutive cells
// and one wavefront per face of a cell: role 2 s is the low face and role 2 s + 1 the
// high face of the s-th active dimension (in the order x, y, z). Each wavefront evaluates
// its face flux for the 64 cells with the device code of the per-cell kernels, the
// fluxes meet in LDS, and the first wavefront forms the divergence in the per-cell
// kernels' order and updates the cells. The arithmetic is the per-cell kernels'; the
// compiler may contract its multiply-adds differently in the two, so results agree to
// rounding.

constexpr int FS_LANES = 64;
constexpr int FS_MAX_ROLES = 6;

template <typename T>
struct FaceFluxes {
  T f[4][FS_MAX_ROLES][FS_LANES];  // [component][role][lane]
};

// The s-th active dimension.
__device__ __forceinline__ int active_dim(const Geom& G, int s) {
  int d = 0;
  for (; d < 2; ++d) {
    if (G.act[d]) {
      if (s == 0) break;
      --s;
    }
  }
  return d;
}

// The flux through the low (high = false) or high face normal to D of cell (i, j, k),
// whose state is U0, from the first-order states of U^m.
template <int D, typename T>
__device__ __forceinline__ void predict_face(const RadPtrs<T>& Um, const Geom& G,
                                             const RadConst<T>& K, const FixedFaces<T>& B,
                                             const T U0[4], int i, int j, int k, bool high,
                                             T f[4]) {
  constexpr int di = D == 0, dj = D == 1, dk = D == 2;
  const M1State<T> m0 = m1_state(U0, K.fclo, K.chat);
  FaceSide<T> own;
#pragma unroll
  for (int q = 0; q < 4; ++q) own.U[q] = U0[q];
  m1_dir(m0, D, K.c, K.inv_c, K.chat, own.Phi, own.lmin, own.lmax);
  T Un[4];
  if (high) {
    load_rad_bc(Um, G, B, i + di, j + dj, k + dk, Un);
    hll(own, face_side(Un, D, K.c, K.inv_c, K.fclo, K.chat), f);
  } else {
    load_rad_bc(Um, G, B, i - di, j - dj, k - dk, Un);
    hll(face_side(Un, D, K.c, K.inv_c, K.fclo, K.chat), own, f);
  }
}

// The flux through the low or high face normal to D of the cell at padded index pc, whose
// half-step state is Uc, from the MC-limited reconstruction of U^{m+1/2}.
template <int D, typename T>
__device__ __forceinline__ void correct_face(const RadPtrs<T>& Uh, const Geom& G,
                                             const RadConst<T>& K, const T Uc[4], int pc,
                                             bool high, T f[4]) {
  const int stride = D == 0 ? 1 : (D == 1 ? G.ps[0] : G.ps[0] * G.ps[1]);
  T L[4], R[4];
  if (high) {
    T Um1[4], Up1[4], Up2[4];
    load_padded4(Uh, pc - stride, Um1);
    load_padded4(Uh, pc + stride, Up1);
    load_padded4(Uh, pc + 2 * stride, Up2);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const T s0 = mc_half_slope(Uc[q] - Um1[q], Up1[q] - Uc[q]);
      const T sp = mc_half_slope(Up1[q] - Uc[q], Up2[q] - Up1[q]);
      L[q] = Uc[q] + s0;
      R[q] = Up1[q] - sp;
    }
  } else {
    T Um2[4], Um1[4], Up1[4];
    load_padded4(Uh, pc - 2 * stride, Um2);
    load_padded4(Uh, pc - stride, Um1);
    load_padded4(Uh, pc + stride, Up1);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const T sm = mc_half_slope(Um1[q] - Um2[q], Uc[q] - Um1[q]);
      const T s0 = mc_half_slope(Uc[q] - Um1[q], Up1[q] - Uc[q]);
      L[q] = Um1[q] + sm;
      R[q] = Uc[q] - s0;
    }
  }
  L[0] = vmax(L[0], K.er_floor);
  R[0] = vmax(R[0], K.er_floor);
  rad_hll(L, R, D, K.c, K.inv_c, K.fclo, K.chat, f);
}

// The divergence of the fluxes in LDS for lane l, summed over the active dimensions in
// the order x, y, z as the per-cell kernels sum it.
template <typename T>
__device__ __forceinline__ void face_divergence(const FaceFluxes<T>& sh, const Geom& G,
                                                const RadConst<T>& K, int l, T div[4]) {
  int r = 0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (!G.act[d]) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) div[q] += (sh.f[q][r + 1][l] - sh.f[q][r][l]) * K.inv_w[d];
    r += 2;
  }
}

// Predictor over the padded region; block b covers padded cells [64 b, 64 b + 64), with
// blockDim = (64, 2 x the active dimensions).
template <typename T>
__global__ void __launch_bounds__(FS_LANES * FS_MAX_ROLES)
    k_rad_predict_fs(RadPtrs<T> Um, RadPtrs<T> Uh, GasView<T> gas, Geom G, RadConst<T> K,
                     FixedFaces<T> B, T h, int NP) {
  __shared__ FaceFluxes<T> sh;
  const int lane = int(threadIdx.x), role = int(threadIdx.y);
  const unsigned pu = blockIdx.x * unsigned(FS_LANES) + unsigned(lane);
  const bool live = pu < unsigned(NP);
  const int p = int(pu);
  int i = 0, j = 0, k = 0;
  if (live) {
    const int q = p / G.ps[0];
    i = p - q * G.ps[0] - G.g[0];
    j = q % G.ps[1] - G.g[1];
    k = q / G.ps[1] - G.g[2];
  }
  const int fb = (live && B.mask) ? fixed_face(G, B.mask, i, j, k) : -1;
  T U0[4] = {T(0), T(0), T(0), T(0)};
  // the first wavefront issues the cell's gas loads before its face, off the critical path
  FrozenRaw<T> raw{};
  if (live && fb < 0) {
    if (role == 0) {
      int s[3];
      const int a = mapped_cell(G, i, j, k, s);
      raw = frozen_load(gas, a, s, K.beta != 0);
    }
    load_rad_bc(Um, G, B, i, j, k, U0);
    const int d = active_dim(G, role >> 1);
    const bool high = (role & 1) != 0;
    T f[4];
    if (d == 0)
      predict_face<0>(Um, G, K, B, U0, i, j, k, high, f);
    else if (d == 1)
      predict_face<1>(Um, G, K, B, U0, i, j, k, high, f);
    else
      predict_face<2>(Um, G, K, B, U0, i, j, k, high, f);
#pragma unroll
    for (int q = 0; q < 4; ++q) sh.f[q][role][lane] = f[q];
  }
  __syncthreads();
  if (role != 0 || !live) return;
  T out[4];
  if (fb >= 0) {
    fixed_state(B, fb, out);
  } else {
    T div[4] = {T(0), T(0), T(0), T(0)};
    face_divergence(sh, G, K, lane, div);
    const Frozen<T> fz = frozen_make(raw, K.beta != 0);
    bool ef, fc;
    rad_update(K, h, U0, U0, div, fz, out, ef, fc);
  }
  Uh.E[p] = out[0];
  Uh.F[0][p] = out[1];
  Uh.F[1][p] = out[2];
  Uh.F[2][p] = out[3];
}

// Corrector over the interior; block b covers cells [64 b, 64 b + 64), with blockDim as
// for the predictor.
template <typename T>
__global__ void __launch_bounds__(FS_LANES * FS_MAX_ROLES)
    k_rad_correct_fs(RadPtrs<T> Um, RadPtrs<T> Uh, GasView<T> gas, Geom G, RadConst<T> K, T h,
                     int N, unsigned long long* ctr) {
  __shared__ FaceFluxes<T> sh;
  const int lane = int(threadIdx.x), role = int(threadIdx.y);
  const unsigned au = blockIdx.x * unsigned(FS_LANES) + unsigned(lane);
  const bool live = au < unsigned(N);
  const int a = int(au);
  int pc = 0;
  T Uc[4] = {T(0), T(0), T(0), T(0)};
  // the first wavefront issues the cell's gas and U^m loads before its face
  FrozenRaw<T> raw{};
  T Uo[4] = {T(0), T(0), T(0), T(0)};
  if (live) {
    if (role == 0) {
      const int s[3] = {1, 1, 1};
      raw = frozen_load(gas, a, s, K.beta != 0);
      Uo[0] = Um.E[a];
      Uo[1] = Um.F[0][a];
      Uo[2] = Um.F[1][a];
      Uo[3] = Um.F[2][a];
    }
    const int q = a / G.n[0];
    const int i = a - q * G.n[0];
    const int j = q % G.n[1];
    const int k = q / G.n[1];
    pc = padded_cell(G, i, j, k);
    load_padded4(Uh, pc, Uc);
    const int d = active_dim(G, role >> 1);
    const bool high = (role & 1) != 0;
    T f[4];
    if (d == 0)
      correct_face<0>(Uh, G, K, Uc, pc, high, f);
    else if (d == 1)
      correct_face<1>(Uh, G, K, Uc, pc, high, f);
    else
      correct_face<2>(Uh, G, K, Uc, pc, high, f);
#pragma unroll
    for (int q = 0; q < 4; ++q) sh.f[q][role][lane] = f[q];
  }
  __syncthreads();
  if (role != 0) return;
  // the first wavefront, all 64 lanes, down to the counters
  bool ef = false, fc = false;
  if (live) {
    T div[4] = {T(0), T(0), T(0), T(0)};
    face_divergence(sh, G, K, lane, div);
    const Frozen<T> fz = frozen_make(raw, K.beta != 0);
    T out[4];
    rad_update(K, h, Uo, Uc, div, fz, out, ef, fc);
    Um.E[a] = out[0];
    Um.F[0][a] = out[1];
    Um.F[1][a] = out[2];
    Um.F[2][a] = out[3];
  }
  wave_add(ctr + CTR_RAD_EFLOOR, ef ? 1ull : 0ull);
  wave_add(ctr + CTR_RAD_FCLAMP, fc ? 1ull : 0ull);
}

// ---------------------------------------------------------------------------
// gas subsystem
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ void gas_prim(const GasConst<T>& K, const T U[5], T W[5]) {
  const T ir = rcp(U[0]);
  W[0] = U[0];
  W[1] = U[1] * ir;
  W[2] = U[2] * ir;
  W[3] = U[3] * ir;
  if (K.iso) {
    W[4] = U[0] * K.cs2;
  } else {
    W[4] = K.gm1 * (U[4] - T(0.5) * (U[1] * W[1] + U[2] * W[2] + U[3] * W[3]));
  }
}

// Euler flux normal to d of a primitive state plus its conserved state.
template <typename T>
__device__ __forceinline__ void gas_flux(const GasConst<T>& K, const T W[5], int d, T U[5],
                                         T F[5]) {
  const T P = K.iso ? W[0] * K.cs2 : W[4];
  U[0] = W[0];
  U[1] = W[0] * W[1];
  U[2] = W[0] * W[2];
  U[3] = W[0] * W[3];
  U[4] = K.iso ? T(0)
               : vdiv(P, K.gm1) + T(0.5) * W[0] * (W[1] * W[1] + W[2] * W[2] + W[3] * W[3]);
  const T un = W[1 + d];
  F[0] = U[0] * un;
  F[1] = U[1] * un;
  F[2] = U[2] * un;
  F[3] = U[3] * un;
  F[1 + d] += P;
  F[4] = K.iso ? T(0) : (U[4] + P) * un;
}

// HLLC with Davis wave-speed bounds (HLLE for an isothermal gas).
template <typename T>
__device__ __forceinline__ void gas_riemann(const GasConst<T>& K, const T WL[5], const T WR[5],
                                            int d, T flux[5]) {
  const T aL = K.iso ? sqrt_(K.cs2) : sqrt_(vdiv(K.gamma * WL[4], WL[0]));
  const T aR = K.iso ? sqrt_(K.cs2) : sqrt_(vdiv(K.gamma * WR[4], WR[0]));
  const T uL = WL[1 + d], uR = WR[1 + d];
  const T SL = tmin(uL - aL, uR - aR);
  const T SR = tmax(uL + aL, uR + aR);
  T UL[5], UR[5], FL[5], FR[5];
  gas_flux(K, WL, d, UL, FL);
  gas_flux(K, WR, d, UR, FR);
  if (K.iso) {
    const T SLm = tmin(SL, T(0)), SRp = tmax(SR, T(0));
    const T id = rcp(SRp - SLm);
#pragma unroll
    for (int q = 0; q < 4; ++q) flux[q] = (SRp * FL[q] - SLm * FR[q] + SRp * SLm * (UR[q] - UL[q])) * id;
    flux[4] = T(0);
    return;
  }
  if (SL >= T(0)) {
#pragma unroll
    for (int q = 0; q < 5; ++q) flux[q] = FL[q];
    return;
  }
  if (SR <= T(0)) {
#pragma unroll
    for (int q = 0; q < 5; ++q) flux[q] = FR[q];
    return;
  }
  const T rL = WL[0], rR = WR[0];
  const T SM = vdiv(WR[4] - WL[4] + rL * uL * (SL - uL) - rR * uR * (SR - uR),
                    rL * (SL - uL) - rR * (SR - uR));
  const bool left = SM >= T(0);
  const T* Wk = left ? WL : WR;
  const T* Uk = left ? UL : UR;
  const T* Fk = left ? FL : FR;
  const T Sk = left ? SL : SR;
  const T uk = Wk[1 + d];
  const T fac = vdiv(Wk[0] * (Sk - uk), Sk - SM);
  T Us[5];
  Us[0] = fac;
  Us[1] = fac * Wk[1];
  Us[2] = fac * Wk[2];
  Us[3] = fac * Wk[3];
  Us[1 + d] = fac * SM;
  Us[4] = fac * (vdiv(Uk[4], Wk[0]) + (SM - uk) * (SM + vdiv(Wk[4], Wk[0] * (Sk - uk))));
#pragma unroll
  for (int q = 0; q < 5; ++q) flux[q] = Fk[q] + Sk * (Us[q] - Uk[q]);
}

// Explicit gas source (Eq. algorithm:source:explicit:gas, no gravity): momentum
// rho kF F/c - b (4/3) rho kF E_r v/c; energy -b rho kF v.F/c. S[0] = 0.
template <typename T>
__device__ __forceinline__ void gas_source(const GasConst<T>& K, T rk, const T v[3], T Er,
                                           const T F[3], T S[5]) {
  const T b = K.beta ? T(1) : T(0);
  S[0] = T(0);
#pragma unroll
  for (int q = 0; q < 3; ++q) S[1 + q] = rk * F[q] * K.inv_c - b * T(4.0 / 3.0) * rk * Er * v[q] * K.inv_c;
  S[4] = K.iso ? T(0) : -b * rk * (v[0] * F[0] + v[1] * F[1] + v[2] * F[2]) * K.inv_c;
}

template <typename T>
__device__ __forceinline__ void gas_floors(const GasConst<T>& K, T U[5], bool& rf, bool& pf) {
  rf = pf = false;
  if (U[0] < K.rho_floor) {
    U[0] = K.rho_floor;
    rf = true;
  }
  if (!K.iso) {
    const T ke = vdiv(T(0.5) * (U[1] * U[1] + U[2] * U[2] + U[3] * U[3]), U[0]);
    const T P = K.gm1 * (U[4] - ke);
    if (P < K.p_floor) {
      U[4] = vdiv(K.p_floor, K.gm1) + ke;
      pf = true;
    }
  }
}

template <typename T>
__device__ __forceinline__ void load_gas_mapped(const GasPtrs<T>& Gp, const Geom& G, int i, int j,
                                                int k, T U[5]) {
  int s[3];
  const int a = mapped_cell(G, i, j, k, s);
  U[0] = Gp.rho[a];
  U[1] = T(s[0]) * Gp.m[0][a];
  U[2] = T(s[1]) * Gp.m[1][a];
  U[3] = T(s[2]) * Gp.m[2][a];
  U[4] = Gp.E[a];
}

// Gas predictor at one cell (i, j, k) of the padded region: first-order fluxes of U^n and
// S_e,gas(U^n, U_r^n), half step, result written to the padded half-step arrays.
template <typename T>
__device__ __forceinline__ void gas_predict_cell(const GasPtrs<T>& Un, const GasPtrs<T>& Uh,
                                                 const RadPtrs<T>& Ur, const T* kF, T kF_s,
                                                 const Geom& G, const GasConst<T>& K, T h, int i,
                                                 int j, int k) {
  T U0[5], W0[5];
  load_gas_mapped(Un, G, i, j, k, U0);
  gas_prim(K, U0, W0);
  T div[5] = {T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (!G.act[d]) continue;
    const int di = d == 0, dj = d == 1, dk = d == 2;
    T Ul[5], Ur2[5], Wl[5], Wr[5], fl[5], fr[5];
    load_gas_mapped(Un, G, i - di, j - dj, k - dk, Ul);
    load_gas_mapped(Un, G, i + di, j + dj, k + dk, Ur2);
    gas_prim(K, Ul, Wl);
    gas_prim(K, Ur2, Wr);
    gas_riemann(K, Wl, W0, d, fl);
    gas_riemann(K, W0, Wr, d, fr);
#pragma unroll
    for (int q = 0; q < 5; ++q) div[q] += (fr[q] - fl[q]) * K.inv_w[d];
  }
  int s[3];
  const int a = mapped_cell(G, i, j, k, s);
  const T rk = W0[0] * (kF ? kF[a] : kF_s);
  const T Er = Ur.E[a];
  const T F[3] = {T(s[0]) * Ur.F[0][a], T(s[1]) * Ur.F[1][a], T(s[2]) * Ur.F[2][a]};
  const T v[3] = {W0[1], W0[2], W0[3]};
  T S[5];
  gas_source(K, rk, v, Er, F, S);
  T out[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) out[q] = U0[q] - h * div[q] + h * S[q];
  if (K.iso) out[4] = U0[4];
  bool rf, pf;
  gas_floors(K, out, rf, pf);
  const int p = padded_cell(G, i, j, k);
  Uh.rho[p] = out[0];
  Uh.m[0][p] = out[1];
  Uh.m[1][p] = out[2];
  Uh.m[2][p] = out[3];
  Uh.E[p] = out[4];
}

// Gas predictor: first-order fluxes of U^n and S_e,gas(U^n, U_r^n), half step, on the
// interior plus two ghost layers.
template <typename T>
__global__ void __launch_bounds__(256) k_gas_predict(GasPtrs<T> Un, GasPtrs<T> Uh, RadPtrs<T> Ur,
                                                     const T* kF, T kF_s, Geom G, GasConst<T> K,
                                                     T h) {
  const int i = int(blockIdx.x * blockDim.x + threadIdx.x) - G.g[0];
  const int j = int(blockIdx.y * blockDim.y + threadIdx.y) - G.g[1];
  const int k = int(blockIdx.z) - G.g[2];
  if (i >= G.n[0] + G.g[0] || j >= G.n[1] + G.g[1]) return;
  gas_predict_cell(Un, Uh, Ur, kF, kF_s, G, K, h, i, j, k);
}

// Gas corrector: MC-limited reconstruction of the primitives of U^{n+1/2}, Riemann
// fluxes, full step from U^n with S_e,gas(U^{n+1/2}, U_r^n). Writes U^{n+1,*} over U^n
// and keeps s_n = S_e,gas(U^{n+1/2}, U_r^n) and (rho, v)^{n+1/2} for the correction.
template <typename T>
__global__ void __launch_bounds__(256) k_gas_correct(GasPtrs<T> Un, GasPtrs<T> Uh, RadPtrs<T> Ur,
                                                     const T* kF, T kF_s, Geom G, GasConst<T> K,
                                                     T h, T* sn0, T* sn1, T* sn2, T* sn3,
                                                     T* wh0, T* wh1, T* wh2, T* wh3,
                                                     unsigned long long* ctr) {
  const int i = int(blockIdx.x * blockDim.x + threadIdx.x);
  const int j = int(blockIdx.y * blockDim.y + threadIdx.y);
  const int k = int(blockIdx.z);
  const bool valid = i < G.n[0] && j < G.n[1];
  bool rf = false, pf = false;
  if (valid) {
    const int pc = padded_cell(G, i, j, k);
    T Wc[5];
    {
      T Uc[5] = {Uh.rho[pc], Uh.m[0][pc], Uh.m[1][pc], Uh.m[2][pc], Uh.E[pc]};
      gas_prim(K, Uc, Wc);
    }
    T div[5] = {T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (!G.act[d]) continue;
      const int stride = d == 0 ? 1 : (d == 1 ? G.ps[0] : G.ps[0] * G.ps[1]);
      T W[5][5];
#pragma unroll
      for (int t = -2; t <= 2; ++t) {
        if (t == 0) {
#pragma unroll
          for (int q = 0; q < 5; ++q) W[2][q] = Wc[q];
          continue;
        }
        const int p = pc + t * stride;
        T U[5] = {Uh.rho[p], Uh.m[0][p], Uh.m[1][p], Uh.m[2][p], Uh.E[p]};
        gas_prim(K, U, W[t + 2]);
      }
      T Lm[5], Rm[5], Lp[5], Rp[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        const T sm = mc_half_slope(W[1][q] - W[0][q], W[2][q] - W[1][q]);
        const T s0 = mc_half_slope(W[2][q] - W[1][q], W[3][q] - W[2][q]);
        const T sp = mc_half_slope(W[3][q] - W[2][q], W[4][q] - W[3][q]);
        Lm[q] = W[1][q] + sm;
        Rm[q] = W[2][q] - s0;
        Lp[q] = W[2][q] + s0;
        Rp[q] = W[3][q] - sp;
      }
      T fl[5], fr[5];
      gas_riemann(K, Lm, Rm, d, fl);
      gas_riemann(K, Lp, Rp, d, fr);
#pragma unroll
      for (int q = 0; q < 5; ++q) div[q] += (fr[q] - fl[q]) * K.inv_w[d];
    }
    const int a = i + G.n[0] * (j + G.n[1] * k);
    const T rk = Wc[0] * (kF ? kF[a] : kF_s);
    const T F[3] = {Ur.F[0][a], Ur.F[1][a], Ur.F[2][a]};
    const T v[3] = {Wc[1], Wc[2], Wc[3]};
    T S[5];
    gas_source(K, rk, v, Ur.E[a], F, S);
    T U0[5] = {Un.rho[a], Un.m[0][a], Un.m[1][a], Un.m[2][a], Un.E[a]};
    T out[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) out[q] = U0[q] - h * div[q] + h * S[q];
    if (K.iso) out[4] = U0[4];
    gas_floors(K, out, rf, pf);
    Un.rho[a] = out[0];
    Un.m[0][a] = out[1];
    Un.m[1][a] = out[2];
    Un.m[2][a] = out[3];
    Un.E[a] = out[4];
    sn0[a] = S[1];
    sn1[a] = S[2];
    sn2[a] = S[3];
    sn3[a] = S[4];
    wh0[a] = Wc[0];
    wh1[a] = Wc[1];
    wh2[a] = Wc[2];
    wh3[a] = Wc[3];
  }
  wave_add(ctr + CTR_GAS_RHOFLOOR, rf ? 1ull : 0ull);
  wave_add(ctr + CTR_GAS_PFLOOR, pf ? 1ull : 0ull);
}

// Second-order gas source correction: U += (dt/2)[S_e,gas(W_1/2, U_r^{n+1}) - s_n].
template <typename T>
__global__ void __launch_bounds__(256) k_gas_source_correct(GasPtrs<T> Ug, RadPtrs<T> Ur,
                                                            const T* kF, T kF_s, GasConst<T> K,
                                                            T half_dt, const T* sn0, const T* sn1,
                                                            const T* sn2, const T* sn3,
                                                            const T* wh0, const T* wh1,
                                                            const T* wh2, const T* wh3, int N,
                                                            unsigned long long* ctr) {
  const int a = int(blockIdx.x * blockDim.x + threadIdx.x);
  bool rf = false, pf = false;
  if (a < N) {
    const T rho_h = wh0[a];
    const T v[3] = {wh1[a], wh2[a], wh3[a]};
    const T F[3] = {Ur.F[0][a], Ur.F[1][a], Ur.F[2][a]};
    T S[5];
    gas_source(K, rho_h * (kF ? kF[a] : kF_s), v, Ur.E[a], F, S);
    T U[5] = {Ug.rho[a], Ug.m[0][a], Ug.m[1][a], Ug.m[2][a], Ug.E[a]};
    U[1] += half_dt * (S[1] - sn0[a]);
    U[2] += half_dt * (S[2] - sn1[a]);
    U[3] += half_dt * (S[3] - sn2[a]);
    if (!K.iso) U[4] += half_dt * (S[4] - sn3[a]);
    gas_floors(K, U, rf, pf);
    Ug.rho[a] = U[0];
    Ug.m[0][a] = U[1];
    Ug.m[1][a] = U[2];
    Ug.m[2][a] = U[3];
    Ug.E[a] = U[4];
  }
  wave_add(ctr + CTR_GAS_RHOFLOOR, rf ? 1ull : 0ull);
  wave_add(ctr + CTR_GAS_PFLOOR, pf ? 1ull : 0ull);
}

// ---------------------------------------------------------------------------
// implicit energy exchange (Sec. 3.4), FP64 whatever T is
// ---------------------------------------------------------------------------

struct ExchConst {
  double c, chat, dt;
  double gm1, a_rad, r_gas;
  double theta, rtol;
  double eps_cv;  // 4 a_R / alpha when c_v = alpha T^3 (a_R T^4 = eps_cv e), else 0
  double er_floor;
  int maxit;
};

__device__ __forceinline__ double quart(double c4, double c1, double c0, double x) {
  const double x2 = x * x;
  return c4 * x2 * x2 + c1 * x + c0;
}

__device__ __forceinline__ double newton(double c4, double c1, double c0, double x) {
  const double x2 = x * x;
  return x - (c4 * x2 * x2 + c1 * x + c0) / (4.0 * c4 * x2 * x + c1);
}

// theta-scheme update of (e, E_r) over dt with Ebar = e + (c/chat) E_r held fixed:
// the new internal energy x solves c4 x^4 + c1 x + c0 = 0 (Eq. source:polynomial) with
// its root in (0, min(-c0/c1, (-c0/c4)^{1/4})]. Newton starts at that upper bound
// (f is increasing and convex, so the iterates fall monotonically onto the root),
// stops at |dx| <= eps x and takes one more step; bisection with a final Newton step
// takes over if it leaves the bracket or runs out of iterations. c0 > 0 (possible for
// theta < 1) redoes the cell with theta = 1.
__device__ __forceinline__ double exchange_root(const ExchConst& X, double rho, double e,
                                                double Er, double kP, double& Er_new, int& iters,
                                                bool& th1, bool& bis) {
  // emission a_R T^4 as a function of e: alpha e^4 (ideal gas), or eps_cv e when
  // c_v = alpha T^3 (Sec. 4.1.3), which leaves a linear equation (c4 = 0)
  const double g = X.gm1 / (rho * X.r_gas);
  const double g2 = g * g;
  const double lin = X.eps_cv;
  const double alpha = lin > 0.0 ? 0.0 : X.a_rad * g2 * g2;
  const double eta = X.c * rho * kP * X.dt;
  const double rc = X.chat / X.c;
  const double Ebar = e + Er / rc;
  double theta = X.theta;
  th1 = false;
  bis = false;
  iters = 0;
  const double e2 = e * e;
  double c4 = alpha * eta * theta;
  double c1 = 1.0 + (rc + lin) * eta * theta;
  double c0 = (1.0 - theta) * eta * (alpha * e2 * e2 + lin * e - Er) - (e + rc * eta * theta * Ebar);
  if (c0 > 0.0 && theta < 1.0) {
    theta = 1.0;
    th1 = true;
    c4 = alpha * eta;
    c1 = 1.0 + (rc + lin) * eta;
    c0 = -(e + rc * eta * Ebar);
  }
  double x;
  if (c0 >= 0.0) {
    x = 0.0;
  } else if (c4 == 0.0) {
    x = -c0 / c1;
  } else {
    const double u = fmin(-c0 / c1, sqrt(sqrt(-c0 / c4)));
    x = u;
    bool conv = false;
    for (int it = 0; it < X.maxit; ++it) {
      const double xn = newton(c4, c1, c0, x);
      ++iters;
      const double dx = x - xn;
      x = xn;
      if (!(x >= 0.0 && x <= u)) break;
      if (fabs(dx) <= X.rtol * x) {
        conv = true;
        break;
      }
    }
    if (conv) {
      x = newton(c4, c1, c0, x);
    } else {
      bis = true;
      double lo = 0.0, hi = u;
      for (int b = 0; b < 200 && hi - lo > X.rtol * hi; ++b) {
        const double mid = 0.5 * (lo + hi);
        if (quart(c4, c1, c0, mid) < 0.0)
          lo = mid;
        else
          hi = mid;
      }
      x = newton(c4, c1, c0, 0.5 * (lo + hi));
    }
  }
  Er_new = rc * (Ebar - x);
  return x;
}

// Exchange of cell a over X.dt (FP64 whatever T is): new gas energy and E_r, and the
// solver statistics of the cell added to the running counts.
// The opacity law kappa = k0 (T_gas / T0)^a (rho / rho0)^b (shadow test, Sec. 4.1.1).
struct OpacityLaw {
  double k0, T0, rho0, a, b;
  double gm1_over_r;  // (gamma - 1) / r_gas: T = gm1_over_r e / rho for the ideal gas
  double T_iso;       // c_s^2 / r_gas for the isothermal gas
  double cv_4;        // 4 / cv_alpha when c_v = cv_alpha T^3: T^4 = cv_4 e
  int mode;           // 0 ideal gas, 1 isothermal, 2 c_v = alpha T^3
};

// The law's opacity of cell a from its gas temperature and density, in FP64.
template <typename T>
__device__ __forceinline__ double law_kappa(const GasPtrs<T>& g, const OpacityLaw& L, int a) {
  const double rho = double(g.rho[a]);
  double Tg = L.T_iso;
  if (L.mode != 1) {
    const double m0 = double(g.m[0][a]), m1 = double(g.m[1][a]), m2 = double(g.m[2][a]);
    const double e = double(g.E[a]) - 0.5 * (m0 * m0 + m1 * m1 + m2 * m2) / rho;
    Tg = L.mode == 2 ? sqrt(sqrt(L.cv_4 * e)) : L.gm1_over_r * e / rho;
  }
  return L.k0 * pow(Tg / L.T0, L.a) * pow(rho / L.rho0, L.b);
}

template <typename T>
__device__ __forceinline__ void exchange_cell(const GasPtrs<T>& Ug, const RadPtrs<T>& Ur,
                                              const T* kP, double kP_s, const ExchConst& X, int a,
                                              unsigned& n_th1, unsigned& n_bis, unsigned& n_it,
                                              unsigned& it_max) {
  const double rho = double(Ug.rho[a]);
  const double m0 = double(Ug.m[0][a]), m1 = double(Ug.m[1][a]), m2 = double(Ug.m[2][a]);
  const double Et = double(Ug.E[a]);
  const double ke = 0.5 * (m0 * m0 + m1 * m1 + m2 * m2) / rho;
  const double e = Et - ke;
  double Er_new;
  int it = 0;
  bool th1 = false, bis = false;
  const double x = exchange_root(X, rho, e, double(Ur.E[a]), kP ? double(kP[a]) : kP_s, Er_new,
                                 it, th1, bis);
  Ug.E[a] = T(Et + (x - e));
  // E_r = (chat/c)(Ebar - x) loses K eps of its precision (Eq. source:kappacond) and can
  // round to zero or below in a cell whose radiation is negligible beside its gas
  // energy; it is raised to the floor as after a radiation stage
  Ur.E[a] = T(Er_new < X.er_floor ? X.er_floor : Er_new);
  n_th1 += th1 ? 1u : 0u;
  n_bis += bis ? 1u : 0u;
  n_it += unsigned(it);
  it_max = unsigned(it) > it_max ? unsigned(it) : it_max;
}

// The exchange kernel keeps its solver statistics (theta = 1 fallbacks, bisections,
// Newton iterations and their maximum) in registers, reduces them over the block and
// writes one record of EXCH_STATS values per block; k_exchange_final folds the records
// into the counters. No atomics: a same-address atomic per wave costs more than the
// exchange itself.
constexpr int EXCH_THREADS = 256;
constexpr int EXCH_STATS = 4;

template <typename T>
__global__ void __launch_bounds__(EXCH_THREADS) k_exchange(GasPtrs<T> Ug, RadPtrs<T> Ur,
                                                           const T* kP, double kP_s, ExchConst X,
                                                           int N, unsigned long long* part,
                                                           OpacityLaw L, T* lawP, T* lawF) {
  __shared__ unsigned long long sh[EXCH_STATS][EXCH_THREADS / 64];
  unsigned n_th1 = 0, n_bis = 0, n_it = 0, it_max = 0;
  const int stride = int(gridDim.x * blockDim.x);
  for (int a = int(blockIdx.x * blockDim.x + threadIdx.x); a < N; a += stride) {
    if (lawP) {
      // the opacity law from the state before the exchange, as k_opacity_law would leave
      // it; the exchange then reads kappa_P back from the same array (kP == lawP)
      const T k = T(law_kappa(Ug, L, a));
      lawP[a] = k;
      lawF[a] = k;
    }
    exchange_cell(Ug, Ur, kP, kP_s, X, a, n_th1, n_bis, n_it, it_max);
  }
  unsigned long long v[EXCH_STATS] = {n_th1, n_bis, n_it, it_max};
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] += __shfl_xor(v[k], off, 64);
    const unsigned long long o = __shfl_xor(v[3], off, 64);
    v[3] = o > v[3] ? o : v[3];
  }
  const int w = int(threadIdx.x) >> 6;
  if (__lane_id() == 0) {
#pragma unroll
    for (int k = 0; k < EXCH_STATS; ++k) sh[k][w] = v[k];
  }
  __syncthreads();
  if (threadIdx.x < EXCH_STATS) {
    const int k = int(threadIdx.x);
    unsigned long long r = sh[k][0];
    for (int q = 1; q < EXCH_THREADS / 64; ++q) r = k == 3 ? (sh[k][q] > r ? sh[k][q] : r) : r + sh[k][q];
    part[size_t(blockIdx.x) * EXCH_STATS + k] = r;
  }
}

// One block: folds the nblocks records of k_exchange into the counters.
__global__ void __launch_bounds__(EXCH_THREADS) k_exchange_final(const unsigned long long* part,
                                                                 int nblocks,
                                                                 unsigned long long* ctr) {
  __shared__ unsigned long long sh[EXCH_STATS][EXCH_THREADS];
  unsigned long long v[EXCH_STATS] = {0ull, 0ull, 0ull, 0ull};
  for (int b = int(threadIdx.x); b < nblocks; b += EXCH_THREADS) {
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] += part[size_t(b) * EXCH_STATS + k];
    const unsigned long long m = part[size_t(b) * EXCH_STATS + 3];
    v[3] = m > v[3] ? m : v[3];
  }
#pragma unroll
  for (int k = 0; k < EXCH_STATS; ++k) sh[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int s = EXCH_THREADS / 2; s > 0; s >>= 1) {
    if (int(threadIdx.x) < s) {
#pragma unroll
      for (int k = 0; k < 3; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
      const unsigned long long o = sh[3][threadIdx.x + s];
      sh[3][threadIdx.x] = o > sh[3][threadIdx.x] ? o : sh[3][threadIdx.x];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    ctr[CTR_EXCH_THETA1] += sh[0][0];
    ctr[CTR_EXCH_BISECT] += sh[1][0];
    ctr[CTR_NEWTON_ITERS] += sh[2][0];
    ctr[CTR_NEWTON_MAX] = sh[3][0] > ctr[CTR_NEWTON_MAX] ? sh[3][0] : ctr[CTR_NEWTON_MAX];
  }
}

// ---------------------------------------------------------------------------
// reductions: FP64 ledger with non-finite check, and v_max for the CFL step
// ---------------------------------------------------------------------------

constexpr int RED_THREADS = 256;

// Block b sums cells b, b + B, b + 2B, ... in a fixed order per thread and a fixed
// tree over the block, so the result does not depend on scheduling.
template <typename T>
__global__ void __launch_bounds__(RED_THREADS) k_ledger(GasPtrs<T> Ug, RadPtrs<T> Ur,
                                                        double c_over_chat, double inv_cchat,
                                                        int N, double* partials,
                                                        unsigned long long* ctr) {
  __shared__ double sh[5][RED_THREADS];
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  unsigned long long bad = 0;
  unsigned long long first = ~0ull;
  const int stride = int(gridDim.x * blockDim.x);
  for (int a = int(blockIdx.x * blockDim.x + threadIdx.x); a < N; a += stride) {
    const double rho = double(Ug.rho[a]);
    const double m[3] = {double(Ug.m[0][a]), double(Ug.m[1][a]), double(Ug.m[2][a])};
    const double E = double(Ug.E[a]);
    const double Er = double(Ur.E[a]);
    const double F[3] = {double(Ur.F[0][a]), double(Ur.F[1][a]), double(Ur.F[2][a])};
    acc[0] += E + c_over_chat * Er;
    acc[1] += m[0] + F[0] * inv_cchat;
    acc[2] += m[1] + F[1] * inv_cchat;
    acc[3] += m[2] + F[2] * inv_cchat;
    acc[4] += rho;
    const bool fin = isfinite(rho) && isfinite(m[0]) && isfinite(m[1]) && isfinite(m[2]) &&
                     isfinite(E) && isfinite(Er) && isfinite(F[0]) && isfinite(F[1]) &&
                     isfinite(F[2]);
    if (!fin) {
      ++bad;
      if ((unsigned long long)a < first) first = (unsigned long long)a;
    }
  }
#pragma unroll
  for (int q = 0; q < 5; ++q) sh[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) {
#pragma unroll
      for (int q = 0; q < 5; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < 5; ++q) partials[5 * blockIdx.x + q] = sh[q][0];
  }
  wave_add(ctr + CTR_NONFINITE, bad);
  if (bad) atomicMin(ctr + CTR_FIRST_BAD, first);
}

__global__ void __launch_bounds__(RED_THREADS) k_ledger_final(const double* partials, int nblocks,
                                                              double dV, double* out) {
  __shared__ double sh[5][RED_THREADS];
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int b = int(threadIdx.x); b < nblocks; b += RED_THREADS) {
#pragma unroll
    for (int q = 0; q < 5; ++q) acc[q] += partials[5 * b + q];
  }
#pragma unroll
  for (int q = 0; q < 5; ++q) sh[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) {
#pragma unroll
      for (int q = 0; q < 5; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < 5; ++q) out[q] = sh[q][0] * dV;
  }
}

struct CflConst {
  double gamma, gm1, cs2;
  double dxmin;
  int iso;
};

// max over cells of |v| + c_eff, c_eff^2 = (gamma P + (4/9) E_r (1 - exp(-rho kF dx)))/rho
// (Eq. algorithm:ceff). Computed in T; the maximum itself is exact.
template <typename T>
__global__ void __launch_bounds__(RED_THREADS) k_vmax(GasPtrs<T> Ug, RadPtrs<T> Ur, const T* kF,
                                                      T kF_s, CflConst C, int N, T* partials) {
  __shared__ T sh[RED_THREADS];
  T best = T(0);
  const int stride = int(gridDim.x * blockDim.x);
  const T gamma = T(C.gamma), gm1 = T(C.gm1), cs2 = T(C.cs2), dxm = T(C.dxmin);
  for (int a = int(blockIdx.x * blockDim.x + threadIdx.x); a < N; a += stride) {
    const T rho = Ug.rho[a];
    const T ir = T(1) / rho;
    const T v0 = Ug.m[0][a] * ir, v1 = Ug.m[1][a] * ir, v2 = Ug.m[2][a] * ir;
    const T v2s = v0 * v0 + v1 * v1 + v2 * v2;
    const T gP = C.iso ? rho * cs2 : gamma * gm1 * (Ug.E[a] - T(0.5) * rho * v2s);
    const T k = kF ? kF[a] : kF_s;
    const T ceff = sqrt((gP + T(4.0 / 9.0) * Ur.E[a] * (T(1) - exp(-rho * k * dxm))) * ir);
    const T s = sqrt(v2s) + ceff;
    best = s > best ? s : best;
  }
  sh[threadIdx.x] = best;
  __syncthreads();
  for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) sh[threadIdx.x] = tmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = sh[0];
}

template <typename T>
__global__ void __launch_bounds__(RED_THREADS) k_vmax_final(const T* partials, int nblocks,
                                                            double* out) {
  __shared__ T sh[RED_THREADS];
  T best = T(0);
  for (int b = int(threadIdx.x); b < nblocks; b += RED_THREADS) best = tmax(best, partials[b]);
  sh[threadIdx.x] = best;
  __syncthreads();
  for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) sh[threadIdx.x] = tmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = double(sh[0]);
}

// ---------------------------------------------------------------------------
// opacity law kappa = k0 (T_gas / T0)^a (rho / rho0)^b (shadow test, Sec. 4.1.1)
// ---------------------------------------------------------------------------

// The one absorption opacity of every cell (kappa_P = kappa_F) from its gas temperature
// and density, in FP64, stored as T.
template <typename T>
__global__ void __launch_bounds__(256) k_opacity_law(GasPtrs<T> g, T* kP, T* kF, OpacityLaw L,
                                                     int N) {
  const int a = int(blockIdx.x * blockDim.x + threadIdx.x);
  if (a >= N) return;
  const T k = T(law_kappa(g, L, a));
  kP[a] = k;
  kF[a] = k;
}

// ---------------------------------------------------------------------------
// many gas steps of a small 1D radiation-only grid in one launch
// ---------------------------------------------------------------------------

// One gas step of a sequence: its length, subcycle count and fixed-face states.
template <typename T>
struct RunStep {
  double dt;
  int nsub;
  int pad;
  T bv[6][4];
};

constexpr int RUN1D_THREADS = 1024;
// Largest grid the fused path takes: one workgroup does all the arithmetic, so beyond one
// cell per thread in FP64 (two in FP32) separate launches over the whole GPU are faster.
template <typename T>
constexpr int run1d_max_cells() {
  return sizeof(T) == 4 ? 2 * RUN1D_THREADS : RUN1D_THREADS;
}

// One workgroup advances a 1D grid of at most run1d_max_cells<T>() cells with the gas frozen
// by nsteps gas steps: per step the exchange over dt (if do_exch), then nsub radiation
// Van Leer subcycles, each stage a loop of the workgroup over the cells with a barrier
// after it. The per-cell work is the same device code as the separate launches, so the
// result is the same bit for bit; what goes is the launch latency between the stages,
// which dominates at these sizes. Every loop runs a bounded count, so the workgroup
// always finishes. Exchange statistics go to part[0 .. EXCH_STATS) as one block record.
// ns radiation Van Leer subcycles of length hr on a 1D grid along x by one workgroup of
// RUN1D_THREADS threads (thread tid): each stage a loop over the cells with a barrier
// after it, the per-cell device code of k_rad_predict and k_rad_correct. nef and nfc
// count the E_r floors and flux clamps of the thread's cells.
template <typename T>
__device__ __forceinline__ void subcycles_1d(const RadPtrs<T>& Um, const RadPtrs<T>& Uh,
                                             const GasView<T>& view, const Geom& G,
                                             const RadConst<T>& K, const FixedFaces<T>& B,
                                             double hr, int ns, int tid, unsigned long long& nef,
                                             unsigned long long& nfc) {
  const int n0 = G.n[0], g0 = G.g[0];
  const T hp = T(0.5 * hr), hc = T(hr);
  for (int m = 0; m < ns; ++m) {
    for (int p = tid; p < n0 + 2 * g0; p += RUN1D_THREADS)
      rad_predict_cell(Um, Uh, view, G, K, B, hp, p - g0, 0, 0);
    __syncthreads();
    for (int a = tid; a < n0; a += RUN1D_THREADS) {
      bool ef = false, fc = false;
      rad_correct_cell(Um, Uh, view, G, K, hc, a, 0, 0, ef, fc);
      nef += ef ? 1ull : 0ull;
      nfc += fc ? 1ull : 0ull;
    }
    __syncthreads();
  }
}

// The ns subcycles of one gas step of a small 1D grid along x in one launch of one
// workgroup (in place of 2 ns launches of the per-cell kernels, whose results it gives
// bit for bit).
template <typename T>
__global__ void __launch_bounds__(RUN1D_THREADS) k_subcycles_1d(RadPtrs<T> Um, RadPtrs<T> Uh,
                                                                GasView<T> view, Geom G,
                                                                RadConst<T> K, FixedFaces<T> B,
                                                                double hr, int ns,
                                                                unsigned long long* ctr) {
  unsigned long long nef = 0, nfc = 0;
  subcycles_1d(Um, Uh, view, G, K, B, hr, ns, int(threadIdx.x), nef, nfc);
  wave_add(ctr + CTR_RAD_EFLOOR, nef);
  wave_add(ctr + CTR_RAD_FCLAMP, nfc);
}

template <typename T>
__global__ void __launch_bounds__(RUN1D_THREADS) k_run_1d(GasPtrs<T> Ug, RadPtrs<T> Um,
                                                          RadPtrs<T> Uh, GasView<T> view, Geom G,
                                                          RadConst<T> K, ExchConst X, const T* kP,
                                                          double kP_s, int do_exch, int fixed_mask,
                                                          const RunStep<T>* __restrict__ steps,
                                                          int nsteps, unsigned long long* part,
                                                          unsigned long long* ctr) {
  __shared__ unsigned long long sh[EXCH_STATS][RUN1D_THREADS / 64];
  const int tid = int(threadIdx.x);
  const int n0 = G.n[0];
  unsigned n_th1 = 0, n_bis = 0, n_it = 0, it_max = 0;
  unsigned long long nef = 0, nfc = 0;
  for (int k = 0; k < nsteps; ++k) {
    const double dt = steps[k].dt;
    const int ns = steps[k].nsub;
    if (do_exch) {
      ExchConst Xk = X;
      Xk.dt = dt;
      for (int a = tid; a < n0; a += RUN1D_THREADS)
        exchange_cell(Ug, Um, kP, kP_s, Xk, a, n_th1, n_bis, n_it, it_max);
      __syncthreads();
    }
    if (ns <= 0) continue;
    FixedFaces<T> B;
    B.mask = fixed_mask;
#pragma unroll
    for (int f = 0; f < 6; ++f)
#pragma unroll
      for (int q = 0; q < 4; ++q) B.v[f][q] = steps[k].bv[f][q];
    subcycles_1d(Um, Uh, view, G, K, B, dt / ns, ns, tid, nef, nfc);
  }
  wave_add(ctr + CTR_RAD_EFLOOR, nef);
  wave_add(ctr + CTR_RAD_FCLAMP, nfc);
  unsigned long long v[EXCH_STATS] = {n_th1, n_bis, n_it, it_max};
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
    for (int q = 0; q < 3; ++q) v[q] += __shfl_xor(v[q], off, 64);
    const unsigned long long o = __shfl_xor(v[3], off, 64);
    v[3] = o > v[3] ? o : v[3];
  }
  if (__lane_id() == 0) {
#pragma unroll
    for (int q = 0; q < EXCH_STATS; ++q) sh[q][tid >> 6] = v[q];
  }
  __syncthreads();
  if (tid < EXCH_STATS) {
    unsigned long long r = sh[tid][0];
    for (int w = 1; w < RUN1D_THREADS / 64; ++w)
      r = tid == 3 ? (sh[tid][w] > r ? sh[tid][w] : r) : r + sh[tid][w];
    part[tid] = r;
  }
}

// ---------------------------------------------------------------------------
// conversions between the caller's FP64 arrays and the stored type
// ---------------------------------------------------------------------------

template <typename T>
__global__ void __launch_bounds__(256) k_from_f64(const double* __restrict__ src, T* __restrict__ dst,
                                                  int n) {
  const int a = int(blockIdx.x * blockDim.x + threadIdx.x);
  if (a < n) dst[a] = T(src[a]);
}

template <typename T>
__global__ void __launch_bounds__(256) k_to_f64(const T* __restrict__ src, double* __restrict__ dst,
                                                int n) {
  const int a = int(blockIdx.x * blockDim.x + threadIdx.x);
  if (a < n) dst[a] = double(src[a]);
}

template <typename T>
__global__ void __launch_bounds__(256) k_fill(T* dst, T value, int n) {
  const int a = int(blockIdx.x * blockDim.x + threadIdx.x);
  if (a < n) dst[a] = value;
}

__global__ void k_reset_counters(unsigned long long* ctr) {
  const int q = int(threadIdx.x);
  if (q < CTR_COUNT) ctr[q] = q == CTR_FIRST_BAD ? ~0ull : 0ull;
}

}  // namespace rhdk
