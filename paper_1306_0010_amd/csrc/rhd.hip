// rhd.hip -- host runtime and C interface (include/rhd.h) of the gfx950 library for
// the gray M1 radiation-hydrodynamics step of Skinner & Ostriker (2013), Sec. 3.1.
//
// A handle owns every device buffer it needs, allocated once in rhd_create; rhd_step
// only enqueues kernels on the handle's stream:
//   exchange (FP64) -> gas predictor -> gas corrector
//   -> nsub x [radiation predictor -> radiation corrector]
//   -> gas source correction -> FP64 ledger with non-finite check.
#include "rhd_device.hpp"
#include "rhd_tile.hpp"
#include "rhd_gas_tile.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/rhd.h"

namespace {

thread_local char g_create_error[512] = "no error";

constexpr int LEDGER_BLOCKS = 1024;
constexpr int VMAX_BLOCKS = 1024;
constexpr int EXCH_BLOCKS = 2048;  // grid-stride exchange: 8 waves per SIMD

struct Buffers {
  // one device allocation holds every buffer below up to ctr (created with the handle);
  // kP, kF, j and the run tables are allocated on their own when first needed
  void* slab = nullptr;
  void* gas[5] = {};   // rho, mx, my, mz, E
  void* rad[4] = {};   // Er, Fx, Fy, Fz
  void* kP = nullptr;  // per-cell opacities (null when scalar)
  void* kF = nullptr;
  void* j = nullptr;   // emissivity or null
  void* gh[5] = {};    // padded gas half-step
  void* rh[4] = {};    // padded radiation half-step
  void* sn[4] = {};    // saved gas sources s_n
  void* wh[4] = {};    // saved (rho, v) at the gas half step
  double* ledger_partials = nullptr; // 5 x LEDGER_BLOCKS
  double* ledger = nullptr;          // 5
  void* vmax_partials = nullptr;     // VMAX_BLOCKS of T
  double* vmax = nullptr;            // 1
  unsigned long long* exch_partials = nullptr;  // EXCH_STATS x EXCH_BLOCKS
  unsigned long long* ctr = nullptr; // rhdk::CTR_COUNT
  // step tables of rhd_run (two chunks each), made on its first fused call
  void* run_dev = nullptr;
  void* run_host = nullptr;          // pinned
  hipEvent_t run_ev[2] = {nullptr, nullptr};
  bool run_ev_used[2] = {false, false};
};

enum KernelClass {
  KC_EXCHANGE = 0,
  KC_GAS_PREDICT,
  KC_GAS_CORRECT,
  KC_RAD_PREDICT,
  KC_RAD_CORRECT,
  KC_GAS_SOURCE,
  KC_LEDGER,
  KC_VMAX,
  KC_RUN_1D,
  KC_COUNT
};
const char* const kKernelNames[KC_COUNT] = {"exchange",    "gas_predict",        "gas_correct",
                                            "rad_predict", "rad_correct",        "gas_source_correct",
                                            "ledger",      "vmax",               "run_1d"};

// Event pairs around kernel launches, drained into per-kernel totals.
struct Timer {
  static constexpr int POOL = 2048;
  bool on = false;
  int used = 0;
  hipEvent_t* start = nullptr;
  hipEvent_t* stop = nullptr;
  int cls[POOL] = {};
  long long calls[KC_COUNT] = {};
  double ms[KC_COUNT] = {};
  long long cells[KC_COUNT] = {};
};

}  // namespace

struct rhd {
  rhd_params p;
  bool mixed = false;
  size_t esize = 8;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  rhdk::Geom G;
  int N = 0;
  int NP = 0;
  double dxmin = 0.0;
  Buffers b;
  bool kappa_scalar = true;
  double kP_s = 0.0, kF_s = 0.0;
  bool have_state = false;
  long long steps = 0, subcycles = 0;
  double vmax_last = 0.0;
  long long bytes = 0;
  bool in_batch = false;
  rhd_batch* batch = nullptr;  // the batch this handle is a member of, if in_batch
  int variant = RHD_KERNELS_TILED;
  bool tile_ok = true;         // every array the tiled radiation kernels touch holds <= 4 GiB
  bool law_fresh = false;      // the opacity law's kappa arrays match the current gas state
  int tile_rows = 8;
  int zchunk = 8;
  int fixed_mask = 0;          // bit f: face f is RHD_BC_FIXED (of an active dimension)
  double bval[6][4] = {};      // radiation state of each fixed face (rhd_set_boundary)
  // HIP graph of the subcycle loop (rhd_set_graph), replayed while its key holds
  bool graph_on = false;
  bool capturing = false;
  hipGraphExec_t graph_exec = nullptr;
  int g_nsub = -1, g_variant = -1, g_rows = 0, g_zchunk = 0;
  double g_hr = 0.0, g_chat = 0.0;
  long long graph_captures = 0, graph_replays = 0;
  Timer timer;
  char err[512] = "no error";
};

namespace {

// Kernel choices found by rhd_autotune, shared by later handles of the same grid shape,
// precision and flags in this process.
struct TuneKey {
  int n[3];
  bool mixed;
  unsigned flags;
};

struct TuneEntry {
  TuneKey key;
  int variant, rows, zchunk;
};

std::mutex g_tune_mutex;
TuneEntry g_tuned[64];
int g_ntuned = 0;

bool same_key(const TuneKey& a, const TuneKey& b) {
  return a.n[0] == b.n[0] && a.n[1] == b.n[1] && a.n[2] == b.n[2] && a.mixed == b.mixed &&
         a.flags == b.flags;
}

TuneKey tune_key(const rhd_t* h) {
  TuneKey k;
  for (int d = 0; d < 3; ++d) k.n[d] = h->G.n[d];
  k.mixed = h->mixed;
  k.flags = h->p.flags;
  return k;
}

int fail(rhd_t* h, int code, const char* fmt, ...) {
  char* dst = h ? h->err : g_create_error;
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(dst, 512, fmt, ap);
  va_end(ap);
  return code;
}

#define HIP_TRY(h, call)                                                                    \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return fail((h), RHD_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));         \
  } while (0)

double min_width(const rhd_params* p) {
  double w = p->dx;
  if (p->ny > 1) w = std::min(w, p->dy);
  if (p->nz > 1) w = std::min(w, p->dz);
  return w;
}

int validate(const rhd_params* p) {
  if (!p) return fail(nullptr, RHD_EINVAL, "params is NULL");
  if (p->nx < 1 || p->ny < 1 || p->nz < 1)
    return fail(nullptr, RHD_EINVAL, "grid sizes must be >= 1 (got %d %d %d)", p->nx, p->ny, p->nz);
  const int ns[3] = {p->nx, p->ny, p->nz};
  long long padded = 1, cells = 1;
  for (int d = 0; d < 3; ++d) {
    cells *= ns[d];
    padded *= ns[d] > 1 ? ns[d] + 4 : 1;
  }
  if (padded >= (1ll << 31))
    return fail(nullptr, RHD_EINVAL, "grid too large: %lld padded cells (limit 2^31)", padded);
  const double ws[3] = {p->dx, p->dy, p->dz};
  for (int d = 0; d < 3; ++d) {
    if (ns[d] > 1 && !(ws[d] > 0.0)) return fail(nullptr, RHD_EINVAL, "cell width %d must be > 0", d);
    if (ns[d] > 1) {
      for (int s = 0; s < 2; ++s) {
        const int kind = p->bc[2 * d + s];
        if (kind < RHD_BC_PERIODIC || kind > RHD_BC_FIXED)
          return fail(nullptr, RHD_EINVAL, "unknown boundary kind %d on face %d", kind, 2 * d + s);
        if (kind == RHD_BC_FIXED && !(p->flags & RHD_RAD_ONLY))
          return fail(nullptr, RHD_EINVAL, "fixed faces need RHD_RAD_ONLY (face %d)", 2 * d + s);
        if (kind == RHD_BC_REFLECT && ns[d] < 3)
          return fail(nullptr, RHD_EINVAL, "reflecting faces need at least 3 cells");
      }
      if ((p->bc[2 * d] == RHD_BC_PERIODIC) != (p->bc[2 * d + 1] == RHD_BC_PERIODIC))
        return fail(nullptr, RHD_EINVAL, "periodic faces must come in pairs (dimension %d)", d);
    }
  }
  if (!(p->c_light > 0.0) || !(p->a_rad >= 0.0) || !(p->r_gas > 0.0))
    return fail(nullptr, RHD_EINVAL, "c_light and r_gas must be > 0, a_rad >= 0");
  if (!(p->flags & RHD_ISOTHERMAL) && !(p->gamma > 1.0))
    return fail(nullptr, RHD_EINVAL, "gamma must be > 1 for an ideal gas");
  if ((p->flags & RHD_ISOTHERMAL) && !(p->iso_cs > 0.0))
    return fail(nullptr, RHD_EINVAL, "iso_cs must be > 0 for an isothermal gas");
  if (!(p->cfl > 0.0 && p->cfl <= 1.0)) return fail(nullptr, RHD_EINVAL, "cfl must be in (0, 1]");
  if (!(p->theta_E >= 0.5 && p->theta_E <= 1.0) || !(p->theta_F >= 0.5 && p->theta_F <= 1.0))
    return fail(nullptr, RHD_EINVAL, "theta_E and theta_F must be in [0.5, 1]");
  if (!(p->newton_rtol > 0.0 && p->newton_rtol < 1.0) || p->newton_maxit < 0)
    return fail(nullptr, RHD_EINVAL, "newton_rtol must be in (0, 1) and newton_maxit >= 0");
  if (!(p->rho_floor >= 0.0) || !(p->p_floor >= 0.0) || !(p->er_floor >= 0.0))
    return fail(nullptr, RHD_EINVAL, "floors must be >= 0");
  if ((p->flags & RHD_EXCHANGE_MASK) == (3u << 1))
    return fail(nullptr, RHD_EINVAL, "unknown exchange mode");
  if (p->flags & ~((1u << 9) - 1)) return fail(nullptr, RHD_EINVAL, "unknown flag bits");
  if (p->flags & RHD_OPACITY_LAW) {
    const double* L = p->kappa_law;
    if (!(L[0] >= 0.0) || !(L[1] > 0.0) || !(L[2] > 0.0) || !std::isfinite(L[0]) ||
        !std::isfinite(L[1]) || !std::isfinite(L[2]) || !std::isfinite(L[3]) || !std::isfinite(L[4]))
      return fail(nullptr, RHD_EINVAL, "kappa_law needs k0 >= 0, T0 > 0, rho0 > 0, finite exponents");
  }
  if (p->flags & RHD_GAS_CV_T3) {
    if (!(p->flags & RHD_RAD_ONLY) || (p->flags & RHD_ISOTHERMAL))
      return fail(nullptr, RHD_EINVAL, "RHD_GAS_CV_T3 needs RHD_RAD_ONLY and an ideal gas");
    if (!(p->cv_alpha > 0.0)) return fail(nullptr, RHD_EINVAL, "cv_alpha must be > 0");
  }
  (void)cells;
  return RHD_OK;
}

rhdk::Geom make_geom(const rhd_params* p) {
  rhdk::Geom G;
  const int ns[3] = {p->nx, p->ny, p->nz};
  for (int d = 0; d < 3; ++d) {
    G.n[d] = ns[d];
    G.act[d] = ns[d] > 1;
    G.g[d] = ns[d] > 1 ? 2 : 0;
    G.ps[d] = ns[d] + 2 * G.g[d];
  }
  for (int f = 0; f < 6; ++f) G.bc[f] = p->bc[f];
  return G;
}

// A handle's buffers share one allocation, each starting on a page boundary.
constexpr long long SLAB_ALIGN = 4096;
constexpr long long slab_round(long long bytes) { return (bytes + SLAB_ALIGN - 1) / SLAB_ALIGN * SLAB_ALIGN; }

long long footprint(const rhd_params* p, long long* N_out, long long* NP_out) {
  const bool mixed = (p->flags & RHD_PRECISION_MIXED) != 0;
  const long long es = mixed ? 4 : 8;
  const int ns[3] = {p->nx, p->ny, p->nz};
  long long N = 1, NP = 1;
  for (int d = 0; d < 3; ++d) {
    N *= ns[d];
    NP *= ns[d] > 1 ? ns[d] + 4 : 1;
  }
  if (N_out) *N_out = N;
  if (NP_out) *NP_out = NP;
  const bool gas = !(p->flags & RHD_RAD_ONLY);
  const long long cell = slab_round(N * es), pad = slab_round(NP * es);
  long long bytes = 0;
  bytes += 9 * cell;                    // state
  bytes += 4 * pad;                     // radiation half step
  if (gas) bytes += 5 * pad + 8 * cell; // gas half step, s_n, W_1/2
  bytes += slab_round(5 * LEDGER_BLOCKS * 8) + slab_round(5 * 8) + slab_round(VMAX_BLOCKS * 8) +
           slab_round(8) + slab_round(rhdk::EXCH_STATS * EXCH_BLOCKS * 8) +
           slab_round(rhdk::CTR_COUNT * 8);
  return bytes;
}

template <typename T>
T* as(void* p) {
  return static_cast<T*>(p);
}

template <typename T>
rhdk::RadPtrs<T> rad_ptrs(void* const* a) {
  rhdk::RadPtrs<T> r;
  r.E = as<T>(a[0]);
  r.F[0] = as<T>(a[1]);
  r.F[1] = as<T>(a[2]);
  r.F[2] = as<T>(a[3]);
  return r;
}

template <typename T>
rhdk::GasPtrs<T> gas_ptrs(void* const* a) {
  rhdk::GasPtrs<T> g;
  g.rho = as<T>(a[0]);
  g.m[0] = as<T>(a[1]);
  g.m[1] = as<T>(a[2]);
  g.m[2] = as<T>(a[3]);
  g.E = as<T>(a[4]);
  return g;
}

int blocks_for(long long n, int threads) { return int((n + threads - 1) / threads); }

int timer_drain(rhd_t* h) {
  Timer& t = h->timer;
  if (t.used == 0) return RHD_OK;
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  for (int i = 0; i < t.used; ++i) {
    float ms = 0.0f;
    HIP_TRY(h, hipEventElapsedTime(&ms, t.start[i], t.stop[i]));
    t.ms[t.cls[i]] += double(ms);
  }
  t.used = 0;
  return RHD_OK;
}

// Record a start event for one launch of kernel class kc over `cells` cells; returns the
// pool slot, or -1 when timing is off.
int tbegin(rhd_t* h, int kc, long long cells) {
  Timer& t = h->timer;
  if (!t.on) return -1;
  if (t.used == Timer::POOL && timer_drain(h) != RHD_OK) return -1;
  const int i = t.used++;
  t.cls[i] = kc;
  t.calls[kc] += 1;
  t.cells[kc] = cells;
  if (hipEventRecord(t.start[i], h->stream) != hipSuccess) return -1;
  return i;
}

void tend(rhd_t* h, int i) {
  if (i >= 0) (void)hipEventRecord(h->timer.stop[i], h->stream);
}

// Launch shape for a (possibly padded) region of extents e[3]: x fastest.
void region_launch(const int e[3], dim3& grid, dim3& block) {
  if (e[1] == 1) {
    block = dim3(256, 1, 1);
  } else {
    block = dim3(64, 4, 1);
  }
  grid = dim3((e[0] + block.x - 1) / block.x, (e[1] + block.y - 1) / block.y, e[2]);
}

template <typename T>
rhdk::GasView<T> gas_view(rhd_t* h) {
  rhdk::GasView<T> g;
  g.rho = as<T>(h->b.gas[0]);
  g.m[0] = as<T>(h->b.gas[1]);
  g.m[1] = as<T>(h->b.gas[2]);
  g.m[2] = as<T>(h->b.gas[3]);
  g.kP = h->kappa_scalar ? nullptr : as<T>(h->b.kP);
  g.kF = h->kappa_scalar ? nullptr : as<T>(h->b.kF);
  g.j = h->b.j ? as<T>(h->b.j) : nullptr;
  g.kP_s = T(h->kP_s);
  g.kF_s = T(h->kF_s);
  return g;
}

template <typename T>
int enqueue_ledger(rhd_t* h, double chat) {
  const double c = h->p.c_light;
  const double dV = h->p.dx * h->p.dy * h->p.dz;
  const int ti = tbegin(h, KC_LEDGER, h->N);
  hipLaunchKernelGGL(rhdk::k_ledger<T>, dim3(LEDGER_BLOCKS), dim3(rhdk::RED_THREADS), 0, h->stream,
                     gas_ptrs<T>(h->b.gas), rad_ptrs<T>(h->b.rad), c / chat, 1.0 / (c * chat), h->N,
                     h->b.ledger_partials, h->b.ctr);
  hipLaunchKernelGGL(rhdk::k_ledger_final, dim3(1), dim3(rhdk::RED_THREADS), 0, h->stream,
                     h->b.ledger_partials, LEDGER_BLOCKS, dV, h->b.ledger);
  tend(h, ti);
  HIP_TRY(h, hipGetLastError());
  return RHD_OK;
}

// Tile rows of the predictor for corrector tiles of BY rows: the FP32 predictor always
// runs 4-row tiles (five blocks per CU), the FP64 one the corrector's.
template <typename T, int BY>
constexpr int predict_rows() {
  return sizeof(T) == 4 ? rhdk::PREDICT_ROWS_FP32 : BY;
}

int predict_rows(bool mixed, int rows) { return mixed ? rhdk::PREDICT_ROWS_FP32 : rows; }

// Planes per z chunk of the predictor for a corrector chunk of zchunk planes: the FP32
// predictor takes at most 11 (at 256^3 its launches took 224-229 us at chunks of 8 to 14
// against 235 us at 16 and 245 at 32, while the corrector is fastest at 64; at 128^3 it
// is fastest at the corrector's 8, 42.5 against 43.8 us at 11, where fewer blocks than
// the chip holds at once would run), the FP64 one the corrector's.
constexpr int PREDICT_ZCHUNK_FP32 = 11;
template <typename T>
constexpr int predict_chunk(int zchunk) {
  return sizeof(T) == 4 ? std::min(zchunk, PREDICT_ZCHUNK_FP32) : zchunk;
}

int predict_chunk(bool mixed, int zchunk) {
  return mixed ? std::min(zchunk, PREDICT_ZCHUNK_FP32) : zchunk;
}

// One radiation subcycle with the tiled kernels (3D grids).
template <typename T, int BY>
void launch_tiled_rows(rhd_t* h, rhdk::RadPtrs<T> rad, rhdk::RadPtrs<T> rh, rhdk::GasView<T> view,
                       const rhdk::RadConst<T>& RK, T h_pred, T h_corr) {
  constexpr int PBY = predict_rows<T, BY>();
  const rhdk::Geom& G = h->G;
  const rhdk::TileGrid tp = rhdk::tile_grid<PBY>(G.n, predict_chunk<T>(h->zchunk));
  const rhdk::TileGrid tg = rhdk::tile_grid<BY>(G.n, h->zchunk);
  const dim3 gp(tp.pred[0], tp.pred[1], tp.pred[2]);
  const dim3 gc(tg.corr[0], tg.corr[1], tg.corr[2]);
  int ti = tbegin(h, KC_RAD_PREDICT, h->NP);
  hipLaunchKernelGGL((rhdk::k_rad_predict_tile<T, PBY>), gp, dim3(rhdk::TILE_BX, PBY, 1), 0,
                     h->stream, rad, rh, view, G, RK, h_pred, tp.zc_pred);
  tend(h, ti);
  ti = tbegin(h, KC_RAD_CORRECT, h->N);
  hipLaunchKernelGGL((rhdk::k_rad_correct_tile<T, BY>), gc, dim3(rhdk::TILE_BX, BY, 1), 0,
                     h->stream, rad, rh, view, G, RK, h_corr, tg.zc_corr, h->b.ctr);
  tend(h, ti);
}

template <typename T>
int launch_tiled(rhd_t* h, rhdk::RadPtrs<T> rad, rhdk::RadPtrs<T> rh, rhdk::GasView<T> view,
                 const rhdk::RadConst<T>& RK, T h_pred, T h_corr) {
  switch (h->tile_rows) {
    case 4:
      launch_tiled_rows<T, 4>(h, rad, rh, view, RK, h_pred, h_corr);
      break;
    case 8:
      launch_tiled_rows<T, 8>(h, rad, rh, view, RK, h_pred, h_corr);
      break;
    default:
      if constexpr (sizeof(T) == 4) {
        launch_tiled_rows<T, 16>(h, rad, rh, view, RK, h_pred, h_corr);
      } else {
        return fail(h, RHD_EINVAL, "tile rows %d not available in FP64", h->tile_rows);
      }
  }
  HIP_TRY(h, hipGetLastError());
  return RHD_OK;
}

template <typename T>
rhdk::RadConst<T> rad_const(const rhd_t* h, double chat) {
  const rhd_params& p = h->p;
  const rhdk::Geom& G = h->G;
  rhdk::RadConst<T> RK;
  RK.c = T(p.c_light);
  RK.inv_c = T(1.0 / p.c_light);
  RK.fclo = (p.flags & RHD_CLOSURE_P1) ? T(0) : T(1.0 / p.c_light);
  RK.chat = T(chat);
  RK.inv_w[0] = G.act[0] ? T(1.0 / p.dx) : T(0);
  RK.inv_w[1] = G.act[1] ? T(1.0 / p.dy) : T(0);
  RK.inv_w[2] = G.act[2] ? T(1.0 / p.dz) : T(0);
  RK.theta = T(p.theta_F);
  RK.er_floor = T(p.er_floor);
  RK.beta = (p.flags & RHD_BETA_TAU) != 0;
  RK.absorb = (p.flags & RHD_EXCHANGE_MASK) == RHD_EXCHANGE_ABSORB_ONLY;
  return RK;
}

// Grids that do not take the tiled kernels run the face-split ones up to this many cells
// and the per-cell ones beyond (where the per-cell kernels fill the chip and the
// face-split ones' extra closure evaluations and LDS round trip cost more than they save).
constexpr int FACE_SPLIT_MAX_CELLS = 1 << 17;

template <typename T>
int enqueue_subcycles(rhd_t* h, double dt, double chat, int nsub);

// The subcycle loop as a HIP graph: captured from the stream the first time a key
// (nsub, dt/nsub, chat, kernel choice) is seen, replayed while it holds. A new key is
// captured again and written into the existing executable graph (hipGraphExecUpdate),
// or a new one is instantiated when the update is refused. The loop holds kernel
// launches only (no memset or copy nodes).
template <typename T>
int enqueue_subcycles_graph(rhd_t* h, double dt, double chat, int nsub) {
  const double hr = dt / nsub;
  if (h->graph_exec && h->g_nsub == nsub && h->g_hr == hr && h->g_chat == chat &&
      h->g_variant == h->variant && h->g_rows == h->tile_rows && h->g_zchunk == h->zchunk) {
    HIP_TRY(h, hipGraphLaunch(h->graph_exec, h->stream));
    h->graph_replays += 1;
    return RHD_OK;
  }
  HIP_TRY(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
  h->capturing = true;
  const int rc = enqueue_subcycles<T>(h, dt, chat, nsub);
  h->capturing = false;
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(h->stream, &graph);
  if (rc) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (ec != hipSuccess || !graph)
    return fail(h, RHD_EDEVICE, "hipStreamEndCapture failed: %s", hipGetErrorString(ec));
  if (h->graph_exec) {
    hipGraphNode_t bad = nullptr;
    hipGraphExecUpdateResult res;
    if (hipGraphExecUpdate(h->graph_exec, graph, &bad, &res) != hipSuccess ||
        res != hipGraphExecUpdateSuccess) {
      (void)hipGetLastError();
      (void)hipGraphExecDestroy(h->graph_exec);
      h->graph_exec = nullptr;
    }
  }
  if (!h->graph_exec) {
    const hipError_t ei = hipGraphInstantiate(&h->graph_exec, graph, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
      (void)hipGraphDestroy(graph);
      h->graph_exec = nullptr;
      return fail(h, RHD_EDEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(ei));
    }
  }
  (void)hipGraphDestroy(graph);
  h->g_nsub = nsub;
  h->g_hr = hr;
  h->g_chat = chat;
  h->g_variant = h->variant;
  h->g_rows = h->tile_rows;
  h->g_zchunk = h->zchunk;
  h->graph_captures += 1;
  HIP_TRY(h, hipGraphLaunch(h->graph_exec, h->stream));
  return RHD_OK;
}

// nsub radiation Van Leer subcycles of dt/nsub with the gas frozen (Sec. 3.3, 3.4).
template <typename T>
int enqueue_subcycles(rhd_t* h, double dt, double chat, int nsub) {
  if (h->graph_on && !h->capturing && !h->timer.on && h->stream && nsub > 0)
    return enqueue_subcycles_graph<T>(h, dt, chat, nsub);
  const rhdk::Geom& G = h->G;
  const rhdk::RadConst<T> RK = rad_const<T>(h, chat);
  auto rad = rad_ptrs<T>(h->b.rad);
  auto rh = rad_ptrs<T>(h->b.rh);
  auto view = gas_view<T>(h);
  const double hr = dt / nsub;
  const bool three_d = G.act[0] && G.act[1] && G.act[2];
  // fixed faces run the per-cell kernels, which read their states
  if (three_d && h->variant == RHD_KERNELS_TILED && !h->fixed_mask && h->tile_ok) {
    for (int m = 0; m < nsub; ++m) {
      int rc = launch_tiled<T>(h, rad, rh, view, RK, T(0.5 * hr), T(hr));
      if (rc) return rc;
    }
    return RHD_OK;
  }
  rhdk::FixedFaces<T> B{};
  B.mask = h->fixed_mask;
  for (int f = 0; f < 6; ++f)
    for (int q = 0; q < 4; ++q) B.v[f][q] = T(h->bval[f][q]);
  // a small 1D grid along x runs all nsub subcycles in one workgroup, one launch. Measured:
  // that wins where the subcycles are several or the grid tiny; one subcycle of a few
  // hundred cells or more, or a grid of more than half a cell per thread (FP64) or one
  // (FP32), runs faster as the two launches spread over the chip
  if (h->variant == RHD_KERNELS_TILED && G.act[0] && !G.act[1] && !G.act[2] &&
      h->N <= rhdk::run1d_max_cells<T>() / 2 && (nsub >= 2 || h->N <= 256)) {
    const int ti = tbegin(h, KC_RUN_1D, (long long)h->N * nsub);
    hipLaunchKernelGGL(rhdk::k_subcycles_1d<T>, dim3(1), dim3(rhdk::RUN1D_THREADS), 0, h->stream,
                       rad, rh, view, G, RK, B, hr, nsub, h->b.ctr);
    tend(h, ti);
    HIP_TRY(h, hipGetLastError());
    return RHD_OK;
  }
  // below ~1e5 cells the per-cell kernels leave most of the chip idle and wait on one
  // thread's chain of faces; the face-split kernels spread a cell's faces over wavefronts.
  // 1D grids keep the per-cell kernels by default: they share their device code with the
  // one-workgroup kernel of rhd_run, so stepping and rhd_run agree bit for bit there.
  const int roles = 2 * (G.act[0] + G.act[1] + G.act[2]);
  const bool face_split = h->variant == RHD_KERNELS_FACE_SPLIT ||
                          (h->variant == RHD_KERNELS_TILED && roles >= 4 &&
                           h->N <= FACE_SPLIT_MAX_CELLS);
  if (face_split && roles > 0) {
    const dim3 block(rhdk::FS_LANES, roles);
    const dim3 gp((h->NP + rhdk::FS_LANES - 1) / rhdk::FS_LANES);
    const dim3 gc((h->N + rhdk::FS_LANES - 1) / rhdk::FS_LANES);
    for (int m = 0; m < nsub; ++m) {
      int ti = tbegin(h, KC_RAD_PREDICT, h->NP);
      hipLaunchKernelGGL(rhdk::k_rad_predict_fs<T>, gp, block, 0, h->stream, rad, rh, view, G, RK,
                         B, T(0.5 * hr), h->NP);
      tend(h, ti);
      ti = tbegin(h, KC_RAD_CORRECT, h->N);
      hipLaunchKernelGGL(rhdk::k_rad_correct_fs<T>, gc, block, 0, h->stream, rad, rh, view, G, RK,
                         T(hr), h->N, h->b.ctr);
      tend(h, ti);
    }
    HIP_TRY(h, hipGetLastError());
    return RHD_OK;
  }
  dim3 gp, bp, gc, bc;
  region_launch(G.ps, gp, bp);
  region_launch(G.n, gc, bc);
  for (int m = 0; m < nsub; ++m) {
    int ti = tbegin(h, KC_RAD_PREDICT, h->NP);
    hipLaunchKernelGGL(rhdk::k_rad_predict<T>, gp, bp, 0, h->stream, rad, rh, view, G, RK, B,
                       T(0.5 * hr));
    tend(h, ti);
    ti = tbegin(h, KC_RAD_CORRECT, h->N);
    hipLaunchKernelGGL(rhdk::k_rad_correct<T>, gc, bc, 0, h->stream, rad, rh, view, G, RK, T(hr),
                       h->b.ctr);
    tend(h, ti);
  }
  HIP_TRY(h, hipGetLastError());
  return RHD_OK;
}

template <typename T>
rhdk::GasConst<T> gas_const(const rhd_t* h) {
  const rhd_params& p = h->p;
  const rhdk::Geom& G = h->G;
  rhdk::GasConst<T> GK;
  GK.c = T(p.c_light);
  GK.inv_c = T(1.0 / p.c_light);
  GK.inv_w[0] = G.act[0] ? T(1.0 / p.dx) : T(0);
  GK.inv_w[1] = G.act[1] ? T(1.0 / p.dy) : T(0);
  GK.inv_w[2] = G.act[2] ? T(1.0 / p.dz) : T(0);
  GK.gamma = T(p.gamma);
  GK.gm1 = T(p.gamma - 1.0);
  GK.cs2 = T(p.iso_cs * p.iso_cs);
  GK.rho_floor = T(p.rho_floor);
  GK.p_floor = T(p.p_floor);
  GK.beta = (p.flags & RHD_BETA_TAU) != 0;
  GK.iso = (p.flags & RHD_ISOTHERMAL) != 0;
  return GK;
}

// Steps 2-3 of a gas step (Sec. 3.1): the implicit exchange and the gas Van Leer step.
// The gas Van Leer stages with the tiled kernels (3D grids), on the radiation stages'
// tile shape.
template <typename T, int BY>
int launch_gas_tiled(rhd_t* h, double dt) {
  const rhdk::Geom& G = h->G;
  const rhdk::TileGrid tg = rhdk::tile_grid<BY>(G.n, h->zchunk);
  const dim3 block(rhdk::TILE_BX, BY, 1);
  const rhdk::GasConst<T> GK = gas_const<T>(h);
  auto gas = gas_ptrs<T>(h->b.gas);
  auto gh = gas_ptrs<T>(h->b.gh);
  auto rad = rad_ptrs<T>(h->b.rad);
  const T* kFp = h->kappa_scalar ? nullptr : as<T>(h->b.kF);
  int ti = tbegin(h, KC_GAS_PREDICT, h->NP);
  hipLaunchKernelGGL((rhdk::k_gas_predict_tile<T, BY>), dim3(tg.pred[0], tg.pred[1], tg.pred[2]),
                     block, 0, h->stream, gas, gh, rad, kFp, T(h->kF_s), G, GK, T(0.5 * dt),
                     tg.zc_pred);
  tend(h, ti);
  ti = tbegin(h, KC_GAS_CORRECT, h->N);
  hipLaunchKernelGGL((rhdk::k_gas_correct_tile<T, BY>), dim3(tg.corr[0], tg.corr[1], tg.corr[2]),
                     block, 0, h->stream, gas, gh, rad, kFp, T(h->kF_s), G, GK, T(dt),
                     tg.zc_corr, as<T>(h->b.sn[0]), as<T>(h->b.sn[1]), as<T>(h->b.sn[2]),
                     as<T>(h->b.sn[3]), as<T>(h->b.wh[0]), as<T>(h->b.wh[1]), as<T>(h->b.wh[2]),
                     as<T>(h->b.wh[3]), h->b.ctr);
  tend(h, ti);
  HIP_TRY(h, hipGetLastError());
  return RHD_OK;
}

rhdk::ExchConst exch_const(const rhd_t* h, double chat, double dt) {
  const rhd_params& p = h->p;
  rhdk::ExchConst X;
  X.c = p.c_light;
  X.chat = chat;
  X.dt = dt;
  X.gm1 = p.gamma - 1.0;
  X.a_rad = p.a_rad;
  X.r_gas = p.r_gas;
  X.theta = p.theta_E;
  X.rtol = p.newton_rtol;
  X.eps_cv = (p.flags & RHD_GAS_CV_T3) ? 4.0 * p.a_rad / p.cv_alpha : 0.0;
  X.er_floor = p.er_floor;
  X.maxit = p.newton_maxit;
  return X;
}

rhdk::OpacityLaw law_params(const rhd_t* h) {
  const rhd_params& p = h->p;
  rhdk::OpacityLaw L;
  L.k0 = p.kappa_law[0];
  L.T0 = p.kappa_law[1];
  L.rho0 = p.kappa_law[2];
  L.a = p.kappa_law[3];
  L.b = p.kappa_law[4];
  L.gm1_over_r = (p.gamma - 1.0) / p.r_gas;
  L.T_iso = p.iso_cs * p.iso_cs / p.r_gas;
  L.cv_4 = (p.flags & RHD_GAS_CV_T3) ? 4.0 / p.cv_alpha : 0.0;
  L.mode = (p.flags & RHD_ISOTHERMAL) ? 1 : ((p.flags & RHD_GAS_CV_T3) ? 2 : 0);
  return L;
}

// Refill the per-cell opacities from the law (RHD_OPACITY_LAW) for the current state.
template <typename T>
int enqueue_opacity_law(rhd_t* h) {
  if (!(h->p.flags & RHD_OPACITY_LAW)) return RHD_OK;
  // a frozen gas that no exchange heats keeps its temperature: the law's values of the
  // last evaluation still hold
  if (h->law_fresh) return RHD_OK;
  const rhd_params& p = h->p;
  hipLaunchKernelGGL(rhdk::k_opacity_law<T>, dim3(blocks_for(h->N, 256)), dim3(256), 0, h->stream,
                     gas_ptrs<T>(h->b.gas), as<T>(h->b.kP), as<T>(h->b.kF), law_params(h), h->N);
  HIP_TRY(h, hipGetLastError());
  h->law_fresh = (p.flags & RHD_RAD_ONLY) && (p.flags & RHD_EXCHANGE_MASK) != RHD_EXCHANGE_FULL;
  return RHD_OK;
}

template <typename T>
int enqueue_pre(rhd_t* h, double dt, double chat) {
  const rhd_params& p = h->p;
  const unsigned mode = p.flags & RHD_EXCHANGE_MASK;
  const bool iso = (p.flags & RHD_ISOTHERMAL) != 0;
  const bool rad_only = (p.flags & RHD_RAD_ONLY) != 0;
  const rhdk::Geom& G = h->G;
  auto gas = gas_ptrs<T>(h->b.gas);
  auto rad = rad_ptrs<T>(h->b.rad);
  const T* kFp = h->kappa_scalar ? nullptr : as<T>(h->b.kF);
  const T* kPp = h->kappa_scalar ? nullptr : as<T>(h->b.kP);
  // an opacity law is evaluated once per gas step, from the state at its start; when the
  // exchange runs, inside it (each cell before its own exchange), one launch fewer
  const bool exchange = mode == RHD_EXCHANGE_FULL && !iso;
  const bool law_in_exchange = exchange && (p.flags & RHD_OPACITY_LAW) && !h->law_fresh;
  if (!law_in_exchange)
    if (int rc = enqueue_opacity_law<T>(h)) return rc;

  // implicit energy exchange over dt_gas (FP64)
  if (exchange) {
    const rhdk::ExchConst X = exch_const(h, chat, dt);
    const int ti = tbegin(h, KC_EXCHANGE, h->N);
    const int eb = std::min(EXCH_BLOCKS, blocks_for(h->N, rhdk::EXCH_THREADS));
    T* lawP = law_in_exchange ? as<T>(h->b.kP) : nullptr;
    T* lawF = law_in_exchange ? as<T>(h->b.kF) : nullptr;
    hipLaunchKernelGGL(rhdk::k_exchange<T>, dim3(eb), dim3(rhdk::EXCH_THREADS), 0, h->stream, gas,
                       rad, kPp, h->kP_s, X, h->N, h->b.exch_partials, law_params(h), lawP, lawF);
    tend(h, ti);
    hipLaunchKernelGGL(rhdk::k_exchange_final, dim3(1), dim3(rhdk::EXCH_THREADS), 0, h->stream,
                       h->b.exch_partials, eb, h->b.ctr);
  }

  // gas Van Leer step with S_e,gas at first order
  if (!rad_only && G.act[0] && G.act[1] && G.act[2] && h->variant == RHD_KERNELS_TILED) {
    int rc = RHD_OK;
    switch (h->tile_rows) {
      case 4:
        rc = launch_gas_tiled<T, 4>(h, dt);
        break;
      case 8:
        rc = launch_gas_tiled<T, 8>(h, dt);
        break;
      default:
        if constexpr (sizeof(T) == 4) {
          rc = launch_gas_tiled<T, 16>(h, dt);
        } else {
          return fail(h, RHD_EINVAL, "tile rows %d not available in FP64", h->tile_rows);
        }
    }
    if (rc) return rc;
  } else if (!rad_only) {
    const rhdk::GasConst<T> GK = gas_const<T>(h);
    dim3 grid, block;
    region_launch(G.ps, grid, block);
    auto gh = gas_ptrs<T>(h->b.gh);
    int ti = tbegin(h, KC_GAS_PREDICT, h->NP);
    hipLaunchKernelGGL(rhdk::k_gas_predict<T>, grid, block, 0, h->stream, gas, gh, rad, kFp,
                       T(h->kF_s), G, GK, T(0.5 * dt));
    tend(h, ti);
    region_launch(G.n, grid, block);
    ti = tbegin(h, KC_GAS_CORRECT, h->N);
    hipLaunchKernelGGL(rhdk::k_gas_correct<T>, grid, block, 0, h->stream, gas, gh, rad, kFp,
                       T(h->kF_s), G, GK, T(dt), as<T>(h->b.sn[0]), as<T>(h->b.sn[1]),
                       as<T>(h->b.sn[2]), as<T>(h->b.sn[3]), as<T>(h->b.wh[0]), as<T>(h->b.wh[1]),
                       as<T>(h->b.wh[2]), as<T>(h->b.wh[3]), h->b.ctr);
    tend(h, ti);
  }
  HIP_TRY(h, hipGetLastError());
  return RHD_OK;
}

// Steps 6 and the ledger: second-order gas source correction, then the FP64 ledger.
template <typename T>
int enqueue_post(rhd_t* h, double dt, double chat, bool ledger = true) {
  const bool rad_only = (h->p.flags & RHD_RAD_ONLY) != 0;
  if (!rad_only) {
    const rhdk::GasConst<T> GK = gas_const<T>(h);
    const T* kFp = h->kappa_scalar ? nullptr : as<T>(h->b.kF);
    const int threads = 256;
    const int ti = tbegin(h, KC_GAS_SOURCE, h->N);
    hipLaunchKernelGGL(rhdk::k_gas_source_correct<T>, dim3(blocks_for(h->N, threads)), dim3(threads),
                       0, h->stream, gas_ptrs<T>(h->b.gas), rad_ptrs<T>(h->b.rad), kFp,
                       T(h->kF_s), GK, T(0.5 * dt), as<T>(h->b.sn[0]), as<T>(h->b.sn[1]),
                       as<T>(h->b.sn[2]), as<T>(h->b.sn[3]), as<T>(h->b.wh[0]), as<T>(h->b.wh[1]),
                       as<T>(h->b.wh[2]), as<T>(h->b.wh[3]), h->N, h->b.ctr);
    tend(h, ti);
    HIP_TRY(h, hipGetLastError());
  }
  return ledger ? enqueue_ledger<T>(h, chat) : RHD_OK;
}

template <typename T>
int enqueue_step(rhd_t* h, double dt, double chat, int nsub, bool ledger = true) {
  int rc = enqueue_pre<T>(h, dt, chat);
  if (rc) return rc;
  if (nsub > 0 && (rc = enqueue_subcycles<T>(h, dt, chat, nsub))) return rc;
  return enqueue_post<T>(h, dt, chat, ledger);
}

constexpr int RUN_CHUNK = 1024;  // steps per launch of the fused 1D path

template <typename T>
bool run_fused(const rhd_t* h) {
  // an opacity law is refreshed per step by its own kernel, which the fused path does not run
  return h->G.act[0] && !h->G.act[1] && !h->G.act[2] && h->N <= rhdk::run1d_max_cells<T>() &&
         (h->p.flags & RHD_RAD_ONLY) && !(h->p.flags & RHD_OPACITY_LAW);
}

// Fixed-face states of step k of rhd_run: from the table when given, else the handle's.
void run_faces(const rhd_t* h, const double* bvals, int k, double out[6][4]) {
  for (int f = 0; f < 6; ++f)
    for (int q = 0; q < 4; ++q)
      out[f][q] = (bvals && (h->fixed_mask & (1 << f))) ? bvals[size_t(k) * 24 + 4 * f + q]
                                                        : h->bval[f][q];
}

template <typename T>
int run_impl(rhd_t* h, int nsteps, const double* dt, const int* nsub, double chat,
             const double* bvals) {
  if (!run_fused<T>(h)) {
    // the ledger is taken once, after the last step
    for (int k = 0; k < nsteps; ++k) {
      run_faces(h, bvals, k, h->bval);
      if (int rc = enqueue_step<T>(h, dt[k], chat, nsub[k], false)) return rc;
      h->steps += 1;
      h->subcycles += nsub[k];
    }
    return nsteps > 0 ? enqueue_ledger<T>(h, chat) : RHD_OK;
  }
  using Step = rhdk::RunStep<T>;
  if (!h->b.run_dev) {
    const size_t bytes = 2 * size_t(RUN_CHUNK) * sizeof(Step);
    HIP_TRY(h, hipMalloc(&h->b.run_dev, bytes));
    HIP_TRY(h, hipHostMalloc(&h->b.run_host, bytes, hipHostMallocDefault));
    for (auto& e : h->b.run_ev) HIP_TRY(h, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    h->bytes += (long long)bytes;
  }
  const rhd_params& p = h->p;
  const unsigned mode = p.flags & RHD_EXCHANGE_MASK;
  const int do_exch = mode == RHD_EXCHANGE_FULL && !(p.flags & RHD_ISOTHERMAL);
  const rhdk::RadConst<T> RK = rad_const<T>(h, chat);
  const rhdk::ExchConst X = exch_const(h, chat, 0.0);
  const T* kPp = h->kappa_scalar ? nullptr : as<T>(h->b.kP);
  for (int c0 = 0; c0 < nsteps; c0 += RUN_CHUNK) {
    const int cnt = std::min(RUN_CHUNK, nsteps - c0);
    const int half = (c0 / RUN_CHUNK) & 1;
    Step* hs = static_cast<Step*>(h->b.run_host) + size_t(half) * RUN_CHUNK;
    Step* ds = static_cast<Step*>(h->b.run_dev) + size_t(half) * RUN_CHUNK;
    // the copy that last read this half of the host table must have finished
    if (h->b.run_ev_used[half]) HIP_TRY(h, hipEventSynchronize(h->b.run_ev[half]));
    for (int k = 0; k < cnt; ++k) {
      double bv[6][4];
      run_faces(h, bvals, c0 + k, bv);
      hs[k].dt = dt[c0 + k];
      hs[k].nsub = nsub[c0 + k];
      hs[k].pad = 0;
      for (int f = 0; f < 6; ++f)
        for (int q = 0; q < 4; ++q) hs[k].bv[f][q] = T(bv[f][q]);
    }
    HIP_TRY(h, hipMemcpyAsync(ds, hs, size_t(cnt) * sizeof(Step), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, hipEventRecord(h->b.run_ev[half], h->stream));
    h->b.run_ev_used[half] = true;
    long long sub = 0;
    for (int k = 0; k < cnt; ++k) sub += nsub[c0 + k];
    const int ti = tbegin(h, KC_RUN_1D, h->N * sub);
    hipLaunchKernelGGL(rhdk::k_run_1d<T>, dim3(1), dim3(rhdk::RUN1D_THREADS), 0, h->stream,
                       gas_ptrs<T>(h->b.gas), rad_ptrs<T>(h->b.rad), rad_ptrs<T>(h->b.rh),
                       gas_view<T>(h), h->G, RK, X, kPp, h->kP_s, do_exch, h->fixed_mask, ds, cnt,
                       h->b.exch_partials, h->b.ctr);
    tend(h, ti);
    hipLaunchKernelGGL(rhdk::k_exchange_final, dim3(1), dim3(rhdk::EXCH_THREADS), 0, h->stream,
                       h->b.exch_partials, 1, h->b.ctr);
    HIP_TRY(h, hipGetLastError());
    h->steps += cnt;
    h->subcycles += sub;
  }
  if (nsteps > 0) run_faces(h, bvals, nsteps - 1, h->bval);
  return enqueue_ledger<T>(h, chat);
}

// Host transfers go through pairs of pinned chunks: the host converts (FP32 state) or
// copies one chunk while the copy engine moves the other, so a transfer needs no device
// staging array, no conversion kernel and no pageable copy (which the runtime stages with
// copy kernels that compete with other work for the compute units). The pairs are shared
// by every handle and kept until the process ends; a transfer holds one for its duration.
struct Stager {
  int device = 0;
  void* buf[2] = {nullptr, nullptr};
  hipEvent_t ev[2] = {nullptr, nullptr};
  bool pending[2] = {false, false};
};
constexpr size_t STAGE_BYTES = size_t(4) << 20;
std::mutex g_stage_mutex;
std::vector<Stager*> g_stage_free;

// A stager of the handle's device for the current transfer; null when pinned memory or
// events cannot be had. Its chunks' copies have finished when it is returned.
class StagerLease {
 public:
  explicit StagerLease(int device) {
    {
      std::lock_guard<std::mutex> lock(g_stage_mutex);
      for (size_t i = 0; i < g_stage_free.size(); ++i)
        if (g_stage_free[i]->device == device) {
          st_ = g_stage_free[i];
          g_stage_free.erase(g_stage_free.begin() + long(i));
          return;
        }
    }
    Stager* st = new (std::nothrow) Stager();
    if (!st) return;
    st->device = device;
    bool ok = true;
    for (int k = 0; k < 2 && ok; ++k) {
      ok = hipHostMalloc(&st->buf[k], STAGE_BYTES, hipHostMallocDefault) == hipSuccess;
      ok = ok && hipEventCreateWithFlags(&st->ev[k], hipEventDisableTiming) == hipSuccess;
    }
    if (!ok) {
      for (int k = 0; k < 2; ++k) {
        if (st->buf[k]) (void)hipHostFree(st->buf[k]);
        if (st->ev[k]) (void)hipEventDestroy(st->ev[k]);
      }
      delete st;
      return;
    }
    st_ = st;
  }
  ~StagerLease() {
    if (!st_) return;
    for (int k = 0; k < 2; ++k)
      if (st_->pending[k]) {
        (void)hipEventSynchronize(st_->ev[k]);
        st_->pending[k] = false;
      }
    std::lock_guard<std::mutex> lock(g_stage_mutex);
    g_stage_free.push_back(st_);
  }
  StagerLease(const StagerLease&) = delete;
  StagerLease& operator=(const StagerLease&) = delete;
  Stager* operator->() const { return st_; }
  explicit operator bool() const { return st_ != nullptr; }

 private:
  Stager* st_ = nullptr;
};

// Host FP64 values into a device array of T (rounded to nearest in FP32); from device
// FP64 values when from_host is false. The host array has been read when this returns.
template <typename T>
int upload_field(rhd_t* h, const double* src, void* dst, int n, bool from_host) {
  if (!from_host) {
    hipLaunchKernelGGL(rhdk::k_from_f64<T>, dim3(blocks_for(n, 256)), dim3(256), 0, h->stream,
                       src, as<T>(dst), n);
    HIP_TRY(h, hipGetLastError());
    return RHD_OK;
  }
  StagerLease st(h->device);
  if (!st) return fail(h, RHD_ENOMEM, "pinned host staging could not be allocated");
  constexpr size_t per = STAGE_BYTES / sizeof(T);
  T* d = as<T>(dst);
  int k = 0;
  for (size_t o = 0; o < size_t(n); o += per, k ^= 1) {
    const size_t c = std::min(per, size_t(n) - o);
    if (st->pending[k]) {
      HIP_TRY(h, hipEventSynchronize(st->ev[k]));
      st->pending[k] = false;
    }
    T* q = static_cast<T*>(st->buf[k]);
    for (size_t i = 0; i < c; ++i) q[i] = T(src[o + i]);
    HIP_TRY(h, hipMemcpyAsync(d + o, q, c * sizeof(T), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, hipEventRecord(st->ev[k], h->stream));
    st->pending[k] = true;
  }
  return RHD_OK;
}

// A device array of T into host FP64 values (or into device FP64 values when to_host is
// false); the host array holds them when this returns.
template <typename T>
int download_field(rhd_t* h, const void* src, double* dst, int n, bool to_host) {
  const T* s = as<T>(const_cast<void*>(src));
  if (!to_host) {
    hipLaunchKernelGGL(rhdk::k_to_f64<T>, dim3(blocks_for(n, 256)), dim3(256), 0, h->stream, s,
                       dst, n);
    HIP_TRY(h, hipGetLastError());
    return RHD_OK;
  }
  StagerLease st(h->device);
  if (!st) return fail(h, RHD_ENOMEM, "pinned host staging could not be allocated");
  constexpr size_t per = STAGE_BYTES / sizeof(T);
  const size_t chunks = (size_t(n) + per - 1) / per;
  // chunk j travels through buffer j mod 2; chunk j + 1 is on its way while j is converted
  auto issue = [&](size_t j) -> int {
    const size_t o = j * per, c = std::min(per, size_t(n) - o);
    HIP_TRY(h, hipMemcpyAsync(st->buf[j & 1], s + o, c * sizeof(T), hipMemcpyDeviceToHost,
                              h->stream));
    HIP_TRY(h, hipEventRecord(st->ev[j & 1], h->stream));
    st->pending[j & 1] = true;
    return RHD_OK;
  };
  if (chunks > 0)
    if (int rc = issue(0)) return rc;
  for (size_t j = 0; j < chunks; ++j) {
    if (j + 1 < chunks)
      if (int rc = issue(j + 1)) return rc;
    HIP_TRY(h, hipEventSynchronize(st->ev[j & 1]));
    st->pending[j & 1] = false;
    const size_t o = j * per, c = std::min(per, size_t(n) - o);
    const T* q = static_cast<const T*>(st->buf[j & 1]);
    for (size_t i = 0; i < c; ++i) dst[o + i] = double(q[i]);
  }
  return RHD_OK;
}

template <typename T>
int set_state_impl(rhd_t* h, const double* rho, const double* mom, const double* E,
                   const double* Er, const double* Fr, const double* kappaP, const double* kappaF,
                   int kappa_scalar, bool host) {
  const bool law = (h->p.flags & RHD_OPACITY_LAW) != 0;
  if (!rho || !mom || !Er || !Fr || ((!kappaP || !kappaF) && !law))
    return fail(h, RHD_EINVAL, "rho, mom, Er, Fr, kappaP and kappaF must be non-NULL");
  const bool iso = (h->p.flags & RHD_ISOTHERMAL) != 0;
  if (!E && !iso) return fail(h, RHD_EINVAL, "E must be non-NULL for an ideal gas");
  const int N = h->N;
  int rc;
  h->law_fresh = false;  // a new gas state: the law's values must be evaluated again
  if ((rc = upload_field<T>(h, rho, h->b.gas[0], N, host))) return rc;
  for (int q = 0; q < 3; ++q)
    if ((rc = upload_field<T>(h, mom + size_t(q) * N, h->b.gas[1 + q], N, host))) return rc;
  if (E) {
    if ((rc = upload_field<T>(h, E, h->b.gas[4], N, host))) return rc;
  } else {
    hipLaunchKernelGGL(rhdk::k_fill<T>, dim3(blocks_for(N, 256)), dim3(256), 0, h->stream,
                       as<T>(h->b.gas[4]), T(0), N);
  }
  if ((rc = upload_field<T>(h, Er, h->b.rad[0], N, host))) return rc;
  for (int q = 0; q < 3; ++q)
    if ((rc = upload_field<T>(h, Fr + size_t(q) * N, h->b.rad[1 + q], N, host))) return rc;
  if (law) {
    // the opacities come from the law; the arrays given (if any) are not read
    if (!h->b.kP) {
      HIP_TRY(h, hipMalloc(&h->b.kP, size_t(N) * h->esize));
      HIP_TRY(h, hipMalloc(&h->b.kF, size_t(N) * h->esize));
      h->bytes += 2ll * N * (long long)h->esize;
    }
    h->kappa_scalar = false;
    if ((rc = enqueue_opacity_law<T>(h))) return rc;
    if (host) HIP_TRY(h, hipStreamSynchronize(h->stream));
  } else if (kappa_scalar) {
    double kp = 0.0, kf = 0.0;
    if (host) {
      kp = kappaP[0];
      kf = kappaF[0];
    } else {
      HIP_TRY(h, hipMemcpyAsync(&kp, kappaP, sizeof(double), hipMemcpyDeviceToHost, h->stream));
      HIP_TRY(h, hipMemcpyAsync(&kf, kappaF, sizeof(double), hipMemcpyDeviceToHost, h->stream));
      HIP_TRY(h, hipStreamSynchronize(h->stream));
    }
    h->kappa_scalar = true;
    h->kP_s = double(T(kp));
    h->kF_s = double(T(kf));
  } else {
    if (!h->b.kP) {
      HIP_TRY(h, hipMalloc(&h->b.kP, size_t(N) * h->esize));
      HIP_TRY(h, hipMalloc(&h->b.kF, size_t(N) * h->esize));
      h->bytes += 2ll * N * (long long)h->esize;
    }
    if ((rc = upload_field<T>(h, kappaP, h->b.kP, N, host))) return rc;
    if ((rc = upload_field<T>(h, kappaF, h->b.kF, N, host))) return rc;
    h->kappa_scalar = false;
  }
  h->have_state = true;
  return RHD_OK;
}

template <typename T>
int get_state_impl(rhd_t* h, double* rho, double* mom, double* E, double* Er, double* Fr,
                   bool host) {
  const int N = h->N;
  int rc;
  if (rho && (rc = download_field<T>(h, h->b.gas[0], rho, N, host))) return rc;
  if (mom)
    for (int q = 0; q < 3; ++q)
      if ((rc = download_field<T>(h, h->b.gas[1 + q], mom + size_t(q) * N, N, host))) return rc;
  if (E && (rc = download_field<T>(h, h->b.gas[4], E, N, host))) return rc;
  if (Er && (rc = download_field<T>(h, h->b.rad[0], Er, N, host))) return rc;
  if (Fr)
    for (int q = 0; q < 3; ++q)
      if ((rc = download_field<T>(h, h->b.rad[1 + q], Fr + size_t(q) * N, N, host))) return rc;
  return RHD_OK;
}

template <typename T>
int suggest_impl(rhd_t* h, double chat, double* dt_gas, int* nsub) {
  if (int rc = enqueue_opacity_law<T>(h)) return rc;
  rhdk::CflConst C;
  C.gamma = h->p.gamma;
  C.gm1 = h->p.gamma - 1.0;
  C.cs2 = h->p.iso_cs * h->p.iso_cs;
  C.dxmin = h->dxmin;
  C.iso = (h->p.flags & RHD_ISOTHERMAL) != 0;
  const T* kFp = h->kappa_scalar ? nullptr : as<T>(h->b.kF);
  const int ti = tbegin(h, KC_VMAX, h->N);
  hipLaunchKernelGGL(rhdk::k_vmax<T>, dim3(VMAX_BLOCKS), dim3(rhdk::RED_THREADS), 0, h->stream,
                     gas_ptrs<T>(h->b.gas), rad_ptrs<T>(h->b.rad), kFp, T(h->kF_s), C, h->N,
                     as<T>(h->b.vmax_partials));
  hipLaunchKernelGGL(rhdk::k_vmax_final<T>, dim3(1), dim3(rhdk::RED_THREADS), 0, h->stream,
                     as<T>(h->b.vmax_partials), VMAX_BLOCKS, h->b.vmax);
  tend(h, ti);
  HIP_TRY(h, hipGetLastError());
  double vmax = 0.0;
  HIP_TRY(h, hipMemcpyAsync(&vmax, h->b.vmax, sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  h->vmax_last = vmax;
  if (!(vmax > 0.0) || !std::isfinite(vmax))
    return fail(h, RHD_ENONFINITE, "v_max of the state is %g", vmax);
  *dt_gas = h->p.cfl * h->dxmin / vmax;
  const double r = std::ceil(chat / vmax);
  *nsub = r < 1.0 ? 1 : (r > 1e9 ? 1000000000 : int(r));
  return RHD_OK;
}

void free_buffers(rhd_t* h) {
  auto fr = [](void* p) {
    if (p) (void)hipFree(p);
  };
  fr(h->b.slab);
  fr(h->b.kP);
  fr(h->b.kF);
  fr(h->b.j);
  fr(h->b.run_dev);
  if (h->b.run_host) (void)hipHostFree(h->b.run_host);
  for (auto& e : h->b.run_ev)
    if (e) (void)hipEventDestroy(e);
  h->b = Buffers();
}

}  // namespace

namespace {

template <typename T>
int time_subcycles(rhd_t* h, double chat, double dt_rad, int reps, double* ms_per) {
  hipEvent_t a, b;
  HIP_TRY(h, hipEventCreate(&a));
  HIP_TRY(h, hipEventCreate(&b));
  int rc = enqueue_subcycles<T>(h, dt_rad, chat, 1);  // warm-up
  if (!rc) {
    (void)hipEventRecord(a, h->stream);
    rc = enqueue_subcycles<T>(h, dt_rad * reps, chat, reps);
    (void)hipEventRecord(b, h->stream);
  }
  if (!rc) {
    float ms = 0.0f;
    if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess)
      rc = fail(h, RHD_EDEVICE, "autotune event timing failed");
    *ms_per = double(ms) / reps;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return rc;
}

template <typename T>
int autotune_impl(rhd_t* h, double chat, double dt_rad, int reps) {
  const size_t bytes = size_t(h->N) * h->esize;
  void* save[4] = {};
  for (int q = 0; q < 4; ++q) {
    if (hipMalloc(&save[q], bytes) != hipSuccess) {
      for (int r = 0; r < q; ++r) (void)hipFree(save[r]);
      return fail(h, RHD_ENOMEM, "autotune snapshot allocation failed");
    }
    HIP_TRY(h, hipMemcpyAsync(save[q], h->b.rad[q], bytes, hipMemcpyDeviceToDevice, h->stream));
  }
  unsigned long long ctr_save[rhdk::CTR_COUNT];
  HIP_TRY(h, hipMemcpyAsync(ctr_save, h->b.ctr, sizeof(ctr_save), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  const bool was_timing = h->timer.on;
  h->timer.on = false;
  const bool three_d = h->G.act[0] && h->G.act[1] && h->G.act[2];
  struct Cand {
    int variant, rows, zchunk;
  };
  Cand cands[32];
  int nc = 0;
  cands[nc++] = {RHD_KERNELS_PER_CELL, 8, 16};
  cands[nc++] = {RHD_KERNELS_FACE_SPLIT, 8, 16};
  // on grids the tiled kernels do not take, the default choice (the one-workgroup kernel
  // on a small 1D grid, face-split or per-cell by size otherwise)
  if (!(three_d && !h->fixed_mask && h->tile_ok)) cands[nc++] = {RHD_KERNELS_TILED, 8, 8};
  if (three_d && !h->fixed_mask && h->tile_ok) {
    const int rows_list[3] = {4, 8, 16};
    const int zc_list[4] = {6, 8, 12, 16};
    for (int r : rows_list) {
      if (r == 16 && !h->mixed) continue;
      for (int z : zc_list) cands[nc++] = {RHD_KERNELS_TILED, r, z};
    }
  }
  double best = 1e300;
  Cand choice = cands[0];
  int rc = RHD_OK;
  for (int c = 0; c < nc && !rc; ++c) {
    h->variant = cands[c].variant;
    h->tile_rows = cands[c].rows;
    h->zchunk = cands[c].zchunk;
    double ms = 0.0;
    rc = time_subcycles<T>(h, chat, dt_rad, reps, &ms);
    for (int q = 0; q < 4 && !rc; ++q)
      if (hipMemcpyAsync(h->b.rad[q], save[q], bytes, hipMemcpyDeviceToDevice, h->stream) != hipSuccess)
        rc = fail(h, RHD_EDEVICE, "autotune restore failed");
    if (!rc && ms < best) {
      best = ms;
      choice = cands[c];
    }
  }
  if (hipMemcpyAsync(h->b.ctr, ctr_save, sizeof(ctr_save), hipMemcpyHostToDevice, h->stream) != hipSuccess && !rc)
    rc = fail(h, RHD_EDEVICE, "autotune counter restore failed");
  (void)hipStreamSynchronize(h->stream);
  for (int q = 0; q < 4; ++q) (void)hipFree(save[q]);
  h->timer.on = was_timing;
  h->variant = choice.variant;
  h->tile_rows = choice.rows;
  h->zchunk = choice.zchunk;
  if (!rc) {
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    int slot = -1;
    for (int t = 0; t < g_ntuned; ++t)
      if (same_key(g_tuned[t].key, tune_key(h))) slot = t;
    if (slot < 0 && g_ntuned < 64) slot = g_ntuned++;
    if (slot >= 0) g_tuned[slot] = {tune_key(h), choice.variant, choice.rows, choice.zchunk};
  }
  return rc;
}

}  // namespace

extern "C" {

void rhd_default_params(rhd_params* p, int nx, int ny, int nz) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->nx = nx;
  p->ny = ny;
  p->nz = nz;
  p->dx = nx > 0 ? 1.0 / nx : 1.0;
  p->dy = ny > 0 ? 1.0 / ny : 1.0;
  p->dz = nz > 0 ? 1.0 / nz : 1.0;
  p->gamma = 5.0 / 3.0;
  p->c_light = 1.0;
  p->a_rad = 1.0;
  p->r_gas = 1.0;
  p->iso_cs = 1.0;
  p->cfl = 0.4;
  p->theta_E = 1.0;
  p->theta_F = 0.51;
  p->newton_rtol = 1e-10;
  p->newton_maxit = 50;
  p->rho_floor = 1e-10;
  p->p_floor = 1e-14;
  p->er_floor = 1e-30;
  for (int f = 0; f < 6; ++f) p->bc[f] = RHD_BC_PERIODIC;
  p->flags = RHD_EXCHANGE_FULL;
  p->cv_alpha = 0.0;
  for (int q = 0; q < 5; ++q) p->kappa_law[q] = 0.0;
}

long long rhd_footprint_bytes(const rhd_params* p) {
  if (validate(p) != RHD_OK) return -1;
  return footprint(p, nullptr, nullptr);
}

int rhd_create(const rhd_params* p, void* hip_stream, rhd_t** out) {
  if (!out) return fail(nullptr, RHD_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(p);
  if (rc) return rc;
  rhd_t* h = new (std::nothrow) rhd();
  if (!h) return fail(nullptr, RHD_ENOMEM, "host allocation failed");
  h->p = *p;
  h->mixed = (p->flags & RHD_PRECISION_MIXED) != 0;
  h->esize = h->mixed ? 4 : 8;
  h->G = make_geom(p);
  for (int f = 0; f < 6; ++f)
    if (h->G.act[f / 2] && p->bc[f] == RHD_BC_FIXED) h->fixed_mask |= 1 << f;
  long long N, NP;
  footprint(p, &N, &NP);
  h->N = int(N);
  h->NP = int(NP);
  // the tiled radiation kernels address with 32-bit byte offsets; the padded half-step
  // arrays are the largest they touch
  h->tile_ok = (unsigned long long)NP * (unsigned long long)h->esize <= (1ull << 32);
  if (!h->tile_ok) h->variant = RHD_KERNELS_PER_CELL;
  h->dxmin = min_width(p);
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return fail(nullptr, RHD_EDEVICE, "no HIP device");
  }
  if (hip_stream) {
    h->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) {
      delete h;
      return fail(nullptr, RHD_EDEVICE, "hipStreamCreate failed");
    }
    h->own_stream = true;
  }
  const size_t es = h->esize;
  // the handle's buffers are carved out of one allocation, each on a page boundary: a
  // handle is then freed with one hipFree (each of which waits for the device) instead
  // of one per buffer, which matters where solves come and go while others run
  std::vector<std::pair<void**, size_t>> parts;
  auto alloc = [&](void** ptr, size_t bytes) { parts.emplace_back(ptr, bytes); };
  for (auto& q : h->b.gas) alloc(&q, N * es);
  for (auto& q : h->b.rad) alloc(&q, N * es);
  for (auto& q : h->b.rh) alloc(&q, NP * es);
  if (!(p->flags & RHD_RAD_ONLY)) {
    for (auto& q : h->b.gh) alloc(&q, NP * es);
    for (auto& q : h->b.sn) alloc(&q, N * es);
    for (auto& q : h->b.wh) alloc(&q, N * es);
  }
  alloc(reinterpret_cast<void**>(&h->b.ledger_partials), 5 * LEDGER_BLOCKS * sizeof(double));
  alloc(reinterpret_cast<void**>(&h->b.ledger), 5 * sizeof(double));
  alloc(&h->b.vmax_partials, VMAX_BLOCKS * sizeof(double));
  alloc(reinterpret_cast<void**>(&h->b.vmax), sizeof(double));
  alloc(reinterpret_cast<void**>(&h->b.exch_partials),
        rhdk::EXCH_STATS * EXCH_BLOCKS * sizeof(unsigned long long));
  alloc(reinterpret_cast<void**>(&h->b.ctr), rhdk::CTR_COUNT * sizeof(unsigned long long));
  size_t slab_bytes = 0;
  for (const auto& pr : parts) slab_bytes += size_t(slab_round((long long)pr.second));
  bool ok = hipMalloc(&h->b.slab, slab_bytes) == hipSuccess;
  if (ok) {
    char* base = static_cast<char*>(h->b.slab);
    size_t off = 0;
    for (const auto& pr : parts) {
      *pr.first = base + off;
      off += size_t(slab_round((long long)pr.second));
    }
    h->bytes += (long long)slab_bytes;
  } else {
    h->b.slab = nullptr;
  }
  if (!ok) {
    free_buffers(h);
    if (h->own_stream) (void)hipStreamDestroy(h->stream);
    delete h;
    return fail(nullptr, RHD_ENOMEM, "device allocation of %lld bytes failed", footprint(p, 0, 0));
  }
  std::unique_lock<std::mutex> lock(g_tune_mutex);
  for (int t = 0; t < g_ntuned; ++t) {
    if (same_key(g_tuned[t].key, tune_key(h))) {
      h->variant = g_tuned[t].variant;
      h->tile_rows = g_tuned[t].rows;
      h->zchunk = g_tuned[t].zchunk;
    }
  }
  if (!h->tile_ok) h->variant = RHD_KERNELS_PER_CELL;
  lock.unlock();
  hipLaunchKernelGGL(rhdk::k_reset_counters, dim3(1), dim3(64), 0, h->stream, h->b.ctr);
  if (hipMemsetAsync(h->b.ledger, 0, 5 * sizeof(double), h->stream) != hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess) {
    free_buffers(h);
    if (h->own_stream) (void)hipStreamDestroy(h->stream);
    delete h;
    return fail(nullptr, RHD_EDEVICE, "initialisation failed");
  }
  *out = h;
  return RHD_OK;
}

int rhd_set_state(rhd_t* h, const double* rho, const double* mom, const double* E,
                  const double* Er, const double* Fr, const double* kappaP, const double* kappaF,
                  int kappa_scalar) {
  if (!h) return fail(nullptr, RHD_EINVAL, "handle is NULL");
  return h->mixed ? set_state_impl<float>(h, rho, mom, E, Er, Fr, kappaP, kappaF, kappa_scalar, true)
                  : set_state_impl<double>(h, rho, mom, E, Er, Fr, kappaP, kappaF, kappa_scalar, true);
}

int rhd_set_state_device(rhd_t* h, const double* rho, const double* mom, const double* E,
                         const double* Er, const double* Fr, const double* kappaP,
                         const double* kappaF, int kappa_scalar) {
  if (!h) return fail(nullptr, RHD_EINVAL, "handle is NULL");
  return h->mixed ? set_state_impl<float>(h, rho, mom, E, Er, Fr, kappaP, kappaF, kappa_scalar, false)
                  : set_state_impl<double>(h, rho, mom, E, Er, Fr, kappaP, kappaF, kappa_scalar, false);
}

int rhd_set_emission(rhd_t* h, const double* j) {
  if (!h) return fail(nullptr, RHD_EINVAL, "handle is NULL");
  if (!j) {
    if (h->b.j) {
      HIP_TRY(h, hipStreamSynchronize(h->stream));
      HIP_TRY(h, hipFree(h->b.j));
      h->b.j = nullptr;
      h->bytes -= (long long)h->N * (long long)h->esize;
    }
    return RHD_OK;
  }
  if (!h->b.j) {
    HIP_TRY(h, hipMalloc(&h->b.j, size_t(h->N) * h->esize));
    h->bytes += (long long)h->N * (long long)h->esize;
  }
  return h->mixed ? upload_field<float>(h, j, h->b.j, h->N, true)
                  : upload_field<double>(h, j, h->b.j, h->N, true);
}

int rhd_set_boundary(rhd_t* h, int face, const double U[4]) {
  if (!h) return fail(nullptr, RHD_EINVAL, "handle is NULL");
  if (face < 0 || face > 5 || !U) return fail(h, RHD_EINVAL, "face must be 0..5 and U non-NULL");
  if (!(h->fixed_mask & (1 << face)))
    return fail(h, RHD_EINVAL, "face %d is not a fixed face of an active dimension", face);
  for (int q = 0; q < 4; ++q)
    if (!std::isfinite(U[q])) return fail(h, RHD_EINVAL, "boundary state must be finite");
  if (!(U[0] > 0.0)) return fail(h, RHD_EINVAL, "boundary E_r must be > 0");
  for (int q = 0; q < 4; ++q) h->bval[face][q] = U[q];
  return RHD_OK;
}

int rhd_step(rhd_t* h, double dt_gas, double chat, int nsub) {
  if (!h) return fail(nullptr, RHD_EINVAL, "handle is NULL");
  if (!h->have_state) return fail(h, RHD_ESTATE, "rhd_step before rhd_set_state");
  if (!(dt_gas > 0.0) || !std::isfinite(dt_gas))
    return fail(h, RHD_EINVAL, "dt_gas must be finite and > 0 (got %g)", dt_gas);
  if (!(chat > 0.0) || !std::isfinite(chat))
    return fail(h, RHD_EINVAL, "chat must be finite and > 0 (got %g)", chat);
  if (nsub < 0 || nsub > (1 << 20))
    return fail(h, RHD_EINVAL, "nsub must be in [0, 2^20] (got %d)", nsub);
  if (nsub > 0 && chat * dt_gas / nsub > h->p.cfl * h->dxmin * (1.0 + 1e-12))
    return fail(h, RHD_ECFL, "chat dt_gas / nsub = %g exceeds K0 dx = %g",
                chat * dt_gas / nsub, h->p.cfl * h->dxmin);
  int rc = h->mixed ? enqueue_step<float>(h, dt_gas, chat, nsub)
                    : enqueue_step<double>(h, dt_gas, chat, nsub);
  if (rc == RHD_OK) {
    h->steps += 1;
    h->subcycles += nsub;
  }
  return rc;
}

int rhd_run(rhd_t* h, int nsteps, const double* dt_gas, const int* nsub, double chat,
            const double* bvals) {
  if (!h) return fail(nullptr, RHD_EINVAL, "handle is NULL");
  if (!h->have_state) return fail(h, RHD_ESTATE, "rhd_run before rhd_set_state");
  if (nsteps < 0) return fail(h, RHD_EINVAL, "nsteps must be >= 0");
  if (nsteps > 0 && (!dt_gas || !nsub)) return fail(h, RHD_EINVAL, "dt_gas and nsub must be non-NULL");
  if (!(chat > 0.0) || !std::isfinite(chat))
    return fail(h, RHD_EINVAL, "chat must be finite and > 0 (got %g)", chat);
  // every step is checked before anything is enqueued
  for (int k = 0; k < nsteps; ++k) {
    if (!(dt_gas[k] > 0.0) || !std::isfinite(dt_gas[k]))
      return fail(h, RHD_EINVAL, "step %d: dt_gas must be finite and > 0", k);
    if (nsub[k] < 0 || nsub[k] > (1 << 20)) return fail(h, RHD_EINVAL, "step %d: nsub out of range", k);
    if (nsub[k] > 0 && chat * dt_gas[k] / nsub[k] > h->p.cfl * h->dxmin * (1.0 + 1e-12))
      return fail(h, RHD_ECFL, "step %d: chat dt_gas / nsub exceeds K0 dx", k);
    if (!bvals) continue;
    for (int f = 0; f < 6; ++f) {
      if (!(h->fixed_mask & (1 << f))) continue;
      const double* U = bvals + size_t(k) * 24 + 4 * f;
      if (!(U[0] > 0.0) || !std::isfinite(U[0]) || !std::isfinite(U[1]) || !std::isfinite(U[2]) ||
          !std::isfinite(U[3]))
        return fail(h, RHD_EINVAL, "step %d: state of fixed face %d must be finite with E_r > 0", k, f);
    }
  }
  return h->mixed ? run_impl<float>(h, nsteps, dt_gas, nsub, chat, bvals)
                  : run_impl<double>(h, nsteps, dt_gas, nsub, chat, bvals);
}

int rhd_suggest_dt(rhd_t* h, double chat, double* dt_gas, int* nsub) {
  if (!h) return fail(nullptr, RHD_EINVAL, "handle is NULL");
  if (!dt_gas || !nsub) return fail(h, RHD_EINVAL, "dt_gas and nsub must be non-NULL");
  if (!h->have_state) return fail(h, RHD_ESTATE, "rhd_suggest_dt before rhd_set_state");
  if (!(chat > 0.0)) return fail(h, RHD_EINVAL, "chat must be > 0");
  return h->mixed ? suggest_impl<float>(h, chat, dt_gas, nsub)
                  : suggest_impl<double>(h, chat, dt_gas, nsub);
}

int rhd_ledger(rhd_t* h, double chat) {
  if (!h) return fail(nullptr, RHD_EINVAL, "handle is NULL");
  if (!h->have_state) return fail(h, RHD_ESTATE, "rhd_ledger before rhd_set_state");
  if (!(chat > 0.0)) return fail(h, RHD_EINVAL, "chat must be > 0");
  return h->mixed ? enqueue_ledger<float>(h, chat) : enqueue_ledger<double>(h, chat);
}

int rhd_get_state(rhd_t* h, double* rho, double* mom, double* E, double* Er, double* Fr) {
  if (!h) return fail(nullptr, RHD_EINVAL, "handle is NULL");
  if (!h->have_state) return fail(h, RHD_ESTATE, "rhd_get_state before rhd_set_state");
  return h->mixed ? get_state_impl<float>(h, rho, mom, E, Er, Fr, true)
                  : get_state_impl<double>(h, rho, mom, E, Er, Fr, true);
}

int rhd_get_state_device(rhd_t* h, double* rho, double* mom, double* E, double* Er, double* Fr) {
  if (!h) return fail(nullptr, RHD_EINVAL, "handle is NULL");
  if (!h->have_state) return fail(h, RHD_ESTATE, "rhd_get_state_device before rhd_set_state");
  return h->mixed ? get_state_impl<float>(h, rho, mom, E, Er, Fr, false)
                  : get_state_impl<double>(h, rho, mom, E, Er, Fr, false);
}

int rhd_get_diagnostics(rhd_t* h, rhd_diag* out) {
  if (!h) return fail(nullptr, RHD_EINVAL, "handle is NULL");
  if (!out) return fail(h, RHD_EINVAL, "out is NULL");
  unsigned long long c[rhdk::CTR_COUNT];
  double led[5];
  HIP_TRY(h, hipMemcpyAsync(c, h->b.ctr, sizeof(c), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipMemcpyAsync(led, h->b.ledger, sizeof(led), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  std::memset(out, 0, sizeof(*out));
  for (int q = 0; q < 5; ++q) out->ledger[q] = led[q];
  out->vmax = h->vmax_last;
  out->exch_theta1 = (long long)c[rhdk::CTR_EXCH_THETA1];
  out->exch_bisect = (long long)c[rhdk::CTR_EXCH_BISECT];
  out->newton_iters = (long long)c[rhdk::CTR_NEWTON_ITERS];
  out->newton_max = (long long)c[rhdk::CTR_NEWTON_MAX];
  out->rad_fclamp = (long long)c[rhdk::CTR_RAD_FCLAMP];
  out->rad_efloor = (long long)c[rhdk::CTR_RAD_EFLOOR];
  out->gas_rhofloor = (long long)c[rhdk::CTR_GAS_RHOFLOOR];
  out->gas_pfloor = (long long)c[rhdk::CTR_GAS_PFLOOR];
  out->nonfinite = (long long)c[rhdk::CTR_NONFINITE];
  out->first_nonfinite_cell = c[rhdk::CTR_FIRST_BAD] == ~0ull ? -1 : (long long)c[rhdk::CTR_FIRST_BAD];
  out->steps = h->steps;
  out->subcycles = h->subcycles;
  return RHD_OK;
}

int rhd_reset_diagnostics(rhd_t* h) {
  if (!h) return fail(nullptr, RHD_EINVAL, "handle is NULL");
  hipLaunchKernelGGL(rhdk::k_reset_counters, dim3(1), dim3(64), 0, h->stream, h->b.ctr);
  HIP_TRY(h, hipGetLastError());
  h->steps = 0;
  h->subcycles = 0;
  return RHD_OK;
}

int rhd_sync(rhd_t* h) {
  if (!h) return fail(nullptr, RHD_EINVAL, "handle is NULL");
  unsigned long long bad = 0;
  HIP_TRY(h, hipMemcpyAsync(&bad, h->b.ctr + rhdk::CTR_NONFINITE, sizeof(bad),
                            hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  if (bad) return fail(h, RHD_ENONFINITE, "%llu non-finite values in the state", bad);
  return RHD_OK;
}

int rhd_set_timing(rhd_t* h, int enable) {
  if (!h) return fail(nullptr, RHD_EINVAL, "handle is NULL");
  Timer& t = h->timer;
  if (enable && !t.start) {
    t.start = new (std::nothrow) hipEvent_t[Timer::POOL];
    t.stop = new (std::nothrow) hipEvent_t[Timer::POOL];
    if (!t.start || !t.stop) return fail(h, RHD_ENOMEM, "event pool allocation failed");
    for (int i = 0; i < Timer::POOL; ++i) {
      HIP_TRY(h, hipEventCreate(&t.start[i]));
      HIP_TRY(h, hipEventCreate(&t.stop[i]));
    }
  }
  if (!enable) {
    int rc = timer_drain(h);
    t.on = false;
    return rc;
  }
  int rc = timer_drain(h);
  if (rc) return rc;
  for (int k = 0; k < KC_COUNT; ++k) {
    t.calls[k] = 0;
    t.ms[k] = 0.0;
    t.cells[k] = 0;
  }
  t.on = true;
  return RHD_OK;
}

int rhd_get_timing(rhd_t* h, rhd_timing* out) {
  if (!h) return fail(nullptr, RHD_EINVAL, "handle is NULL");
  if (!out) return fail(h, RHD_EINVAL, "out is NULL");
  int rc = timer_drain(h);
  if (rc) return rc;
  std::memset(out, 0, sizeof(*out));
  out->nkernels = KC_COUNT;
  for (int k = 0; k < KC_COUNT; ++k) {
    std::snprintf(out->name[k], sizeof(out->name[k]), "%s", kKernelNames[k]);
    out->calls[k] = h->timer.calls[k];
    out->total_ms[k] = h->timer.ms[k];
    out->cells[k] = h->timer.cells[k];
  }
  return RHD_OK;
}

int rhd_set_kernel_variant(rhd_t* h, int variant, int tile_rows, int zchunk) {
  if (!h) return fail(nullptr, RHD_EINVAL, "handle is NULL");
  if (variant != RHD_KERNELS_PER_CELL && variant != RHD_KERNELS_TILED &&
      variant != RHD_KERNELS_FACE_SPLIT)
    return fail(h, RHD_EINVAL, "unknown kernel variant %d", variant);
  const bool rows_ok = tile_rows == 4 || tile_rows == 8 || (tile_rows == 16 && h->mixed);
  if (!rows_ok) return fail(h, RHD_EINVAL, "tile rows must be 4, 8 (or 16 in mixed precision)");
  if (zchunk < 1) return fail(h, RHD_EINVAL, "zchunk must be >= 1");
  if (variant == RHD_KERNELS_TILED && !h->tile_ok)
    return fail(h, RHD_EINVAL, "the tiled kernels need arrays of at most 4 GiB; this grid's "
                               "half-step arrays hold %lld bytes", (long long)h->NP * h->esize);
  h->variant = variant;
  h->tile_rows = tile_rows;
  h->zchunk = zchunk;
  return RHD_OK;
}

int rhd_autotune(rhd_t* h, double chat, double dt_rad, int reps, int* variant, int* tile_rows,
                 int* zchunk) {
  if (!h) return fail(nullptr, RHD_EINVAL, "handle is NULL");
  if (!h->have_state) return fail(h, RHD_ESTATE, "rhd_autotune before rhd_set_state");
  if (!(chat > 0.0) || !(dt_rad > 0.0) || reps < 1)
    return fail(h, RHD_EINVAL, "chat and dt_rad must be > 0 and reps >= 1");
  if (chat * dt_rad > h->p.cfl * h->dxmin * (1.0 + 1e-12))
    return fail(h, RHD_ECFL, "chat dt_rad exceeds K0 dx");
  // fixed faces, and grids too large for the tiled kernels, choose between the per-cell
  // and the face-split kernels
  const int rc = h->mixed ? autotune_impl<float>(h, chat, dt_rad, reps)
                          : autotune_impl<double>(h, chat, dt_rad, reps);
  if (variant) *variant = h->variant;
  if (tile_rows) *tile_rows = h->tile_rows;
  if (zchunk) *zchunk = h->zchunk;
  return rc;
}

int rhd_set_graph(rhd_t* h, int enable) {
  if (!h) return fail(nullptr, RHD_EINVAL, "handle is NULL");
  if (enable && !h->stream)
    return fail(h, RHD_EINVAL, "graph capture needs a stream other than the null stream");
  h->graph_on = enable != 0;
  return RHD_OK;
}

int rhd_get_graph_stats(const rhd_t* h, long long* captures, long long* replays) {
  if (!h) return fail(nullptr, RHD_EINVAL, "handle is NULL");
  if (captures) *captures = h->graph_captures;
  if (replays) *replays = h->graph_replays;
  return RHD_OK;
}

long long rhd_device_bytes(const rhd_t* h) { return h ? h->bytes : 0; }

}  // extern "C"

// ---------------------------------------------------------------------------
// batch of independent solves
// ---------------------------------------------------------------------------

struct rhd_batch {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int max_solves = 0;
  int rows = 8;
  int zchunk = 8;
  int precision = -1;  // -1 unset, 0 FP64, 1 mixed
  std::vector<rhd_t*> members;
  std::vector<double> chat;
  std::vector<hipStream_t> saved_streams;
  void* d_desc = nullptr;
  int4* d_tiles_pred = nullptr;
  int4* d_tiles_corr = nullptr;
  int* d_counts = nullptr;
  void* h_desc = nullptr;
  int4* h_tiles_pred = nullptr;
  int4* h_tiles_corr = nullptr;
  int* h_counts = nullptr;
  double* h_vmax = nullptr;
  int cap_pred = 0, cap_corr = 0;
  // orders a joining member's stream before the batch stream, and the batch stream before
  // a leaving member's own stream, on the device (the host does not wait)
  hipEvent_t order_ev = nullptr;
  // persistent launch: level table and per-member counters + ticket. Switched off: the
  // launch did not finish on the GPU (rhd_batch_set_persistent refuses to enable it)
  bool persistent = false;
  int* d_level = nullptr;
  int* h_level = nullptr;      // pinned
  unsigned* d_done = nullptr;  // max_solves counters, then the ticket and the error flag,
                               // rhdk::COUNTER_STRIDE apart
  unsigned* h_err = nullptr;   // pinned copy of the error flag of the last persistent launch
  bool err_pending = false;    // a persistent launch was enqueued since its flag was read
  // longest wait of a tile for its member's previous stage: 2 s of the 100 MHz real-time
  // counter, far above any stage's time
  unsigned long long wait_ticks = 200000000ull;
  int resident[3] = {0, 0, 0}; // blocks of the persistent kernel that fit the chip, per tile rows 4/8/16
  char err[512] = "no error";
};

namespace {

constexpr int BATCH_MAX_ROUNDS = 4096;

thread_local char g_batch_error[512] = "no error";

int bfail(rhd_batch_t* b, int code, const char* fmt, ...) {
  char* dst = b ? b->err : g_batch_error;
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(dst, 512, fmt, ap);
  va_end(ap);
  return code;
}

#define BHIP_TRY(b, call)                                                                   \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return bfail((b), RHD_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));        \
  } while (0)

rhdk::TileGrid tile_counts(const rhd_t* h, int rows, int zc) {
  switch (rows) {
    case 4:
      return rhdk::tile_grid<4>(h->G.n, zc);
    case 8:
      return rhdk::tile_grid<8>(h->G.n, zc);
    default:
      return rhdk::tile_grid<16>(h->G.n, zc);
  }
}

int batch_reserve(rhd_batch_t* b, int need_pred, int need_corr) {
  // the tile lists are read by the copies and kernels of a step still in flight
  if (need_pred > b->cap_pred || need_corr > b->cap_corr)
    BHIP_TRY(b, hipStreamSynchronize(b->stream));
  if (need_pred > b->cap_pred) {
    int cap = std::max(need_pred, 2 * b->cap_pred);
    if (b->d_tiles_pred) BHIP_TRY(b, hipFree(b->d_tiles_pred));
    if (b->h_tiles_pred) BHIP_TRY(b, hipHostFree(b->h_tiles_pred));
    b->d_tiles_pred = nullptr;
    b->h_tiles_pred = nullptr;
    BHIP_TRY(b, hipMalloc(&b->d_tiles_pred, size_t(cap) * sizeof(int4)));
    BHIP_TRY(b, hipHostMalloc(&b->h_tiles_pred, size_t(cap) * sizeof(int4), hipHostMallocDefault));
    b->cap_pred = cap;
  }
  if (need_corr > b->cap_corr) {
    int cap = std::max(need_corr, 2 * b->cap_corr);
    if (b->d_tiles_corr) BHIP_TRY(b, hipFree(b->d_tiles_corr));
    if (b->h_tiles_corr) BHIP_TRY(b, hipHostFree(b->h_tiles_corr));
    b->d_tiles_corr = nullptr;
    b->h_tiles_corr = nullptr;
    BHIP_TRY(b, hipMalloc(&b->d_tiles_corr, size_t(cap) * sizeof(int4)));
    BHIP_TRY(b, hipHostMalloc(&b->h_tiles_corr, size_t(cap) * sizeof(int4), hipHostMallocDefault));
    b->cap_corr = cap;
  }
  return RHD_OK;
}

template <typename T, int BY>
void launch_batch_round(rhd_batch_t* b, int total_pred, int total_corr, int r) {
  constexpr int PBY = predict_rows<T, BY>();
  const auto* sd = static_cast<const rhdk::SolveDesc<T>*>(b->d_desc);
  hipLaunchKernelGGL((rhdk::k_rad_predict_batch<T, PBY>), dim3(total_pred),
                     dim3(rhdk::TILE_BX, PBY, 1), 0, b->stream, sd, b->d_tiles_pred,
                     b->d_counts + 2 * r);
  hipLaunchKernelGGL((rhdk::k_rad_correct_batch<T, BY>), dim3(total_corr),
                     dim3(rhdk::TILE_BX, BY, 1), 0, b->stream, sd, b->d_tiles_corr,
                     b->d_counts + 2 * r + 1);
}

// After a synchronisation: the error flag of the last persistent launch, if one ran.
int batch_check_persistent(rhd_batch_t* b) {
  if (!b->err_pending) return RHD_OK;
  b->err_pending = false;
  if (*b->h_err)
    return bfail(b, RHD_EDEVICE, "a persistent batch launch gave up waiting for a stage: "
                                 "its members' states are not valid");
  return RHD_OK;
}

// The persistent launch: counters and ticket cleared by a kernel, then as many blocks as
// fit on the chip at once (at most one per item).
template <typename T, int BY>
int launch_persistent(rhd_batch_t* b, int S, int levels, int items, int widest) {
  const int ri = BY == 4 ? 0 : (BY == 8 ? 1 : 2);
  auto kern = rhdk::k_rad_batch_persistent<T, BY>;
  if (b->resident[ri] <= 0) {
    int per_cu = 0, dev = 0, cus = 0;
    BHIP_TRY(b, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, rhdk::TILE_BX * BY, 0));
    BHIP_TRY(b, hipGetDevice(&dev));
    BHIP_TRY(b, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    b->resident[ri] = std::max(1, per_cu * cus);
  }
  const int words = (S + 2) * rhdk::COUNTER_STRIDE;
  hipLaunchKernelGGL(rhdk::k_fill<unsigned>, dim3(blocks_for(words, 256)), dim3(256), 0, b->stream,
                     b->d_done, 0u, words);
  rhdk::PersistentPlan plan;
  plan.tiles[0] = b->d_tiles_pred;
  plan.tiles[1] = b->d_tiles_corr;
  plan.level_start = b->d_level;
  plan.levels = levels;
  plan.done = b->d_done;
  plan.ticket = b->d_done + size_t(S) * rhdk::COUNTER_STRIDE;
  plan.error = b->d_done + size_t(S + 1) * rhdk::COUNTER_STRIDE;
  plan.wait_ticks = b->wait_ticks;
  const dim3 block(rhdk::TILE_BX, BY, 1);
  // at most two levels' worth of blocks: more could only wait, polling the counters
  const int grid = std::max(1, std::min({items, b->resident[ri], 2 * widest}));
  hipLaunchKernelGGL(kern, dim3(grid), block, 0, b->stream,
                     static_cast<const rhdk::SolveDesc<T>*>(b->d_desc), plan);
  BHIP_TRY(b, hipMemcpyAsync(b->h_err, plan.error, sizeof(unsigned), hipMemcpyDeviceToHost,
                             b->stream));
  b->err_pending = true;
  return RHD_OK;
}

template <typename T>
int batch_step_impl(rhd_batch_t* b, int* nsub_out, double* dt_out) {
  const int S = int(b->members.size());
  // 1. v_max of every member, one synchronisation
  for (int i = 0; i < S; ++i) {
    rhd_t* h = b->members[i];
    if (int rc = enqueue_opacity_law<T>(h)) return bfail(b, rc, "member %d: %s", i, h->err);
    rhdk::CflConst C;
    C.gamma = h->p.gamma;
    C.gm1 = h->p.gamma - 1.0;
    C.cs2 = h->p.iso_cs * h->p.iso_cs;
    C.dxmin = h->dxmin;
    C.iso = (h->p.flags & RHD_ISOTHERMAL) != 0;
    const T* kFp = h->kappa_scalar ? nullptr : as<T>(h->b.kF);
    hipLaunchKernelGGL(rhdk::k_vmax<T>, dim3(VMAX_BLOCKS), dim3(rhdk::RED_THREADS), 0, b->stream,
                       gas_ptrs<T>(h->b.gas), rad_ptrs<T>(h->b.rad), kFp, T(h->kF_s), C, h->N,
                       as<T>(h->b.vmax_partials));
    hipLaunchKernelGGL(rhdk::k_vmax_final<T>, dim3(1), dim3(rhdk::RED_THREADS), 0, b->stream,
                       as<T>(h->b.vmax_partials), VMAX_BLOCKS, h->b.vmax);
    BHIP_TRY(b, hipMemcpyAsync(b->h_vmax + i, h->b.vmax, sizeof(double), hipMemcpyDeviceToHost,
                               b->stream));
  }
  BHIP_TRY(b, hipStreamSynchronize(b->stream));
  if (int rc = batch_check_persistent(b)) return rc;
  std::vector<int> nsub(S);
  std::vector<double> dt(S);
  for (int i = 0; i < S; ++i) {
    rhd_t* h = b->members[i];
    const double vmax = b->h_vmax[i];
    h->vmax_last = vmax;
    // a member that cannot step is named in nsub_out (-1) before anything is enqueued
    auto reject = [&](int code) {
      if (nsub_out)
        for (int k = 0; k < S; ++k) nsub_out[k] = k == i ? -1 : 0;
      return code;
    };
    if (!(vmax > 0.0) || !std::isfinite(vmax))
      return reject(bfail(b, RHD_ENONFINITE, "member %d: v_max is %g", i, vmax));
    dt[i] = h->p.cfl * h->dxmin / vmax;
    const double r = std::ceil(b->chat[i] / vmax);
    nsub[i] = r < 1.0 ? 1 : (r > BATCH_MAX_ROUNDS ? BATCH_MAX_ROUNDS + 1 : int(r));
    if (nsub[i] > BATCH_MAX_ROUNDS)
      return reject(bfail(b, RHD_EINVAL, "member %d needs %d subcycles (limit %d)", i, nsub[i],
                          BATCH_MAX_ROUNDS));
  }
  // 2. exchange and gas step of every member
  for (int i = 0; i < S; ++i) {
    rhd_t* h = b->members[i];
    if (int rc = enqueue_pre<T>(h, dt[i], b->chat[i])) return bfail(b, rc, "member %d: %s", i, h->err);
  }
  // 3. radiation subcycles: members by decreasing nsub, so round r covers a prefix
  std::vector<int> order(S);
  for (int i = 0; i < S; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return nsub[a] > nsub[c]; });
  auto* desc = static_cast<rhdk::SolveDesc<T>*>(b->h_desc);
  std::vector<int> pred_end(S), corr_end(S);
  int np = 0, nc = 0;
  for (int k = 0; k < S; ++k) {
    const int i = order[k];
    rhd_t* h = b->members[i];
    rhdk::SolveDesc<T> d;
    d.Um = rad_ptrs<T>(h->b.rad);
    d.Uh = rad_ptrs<T>(h->b.rh);
    d.gas = gas_view<T>(h);
    d.G = h->G;
    d.K = rad_const<T>(h, b->chat[i]);
    const double hr = dt[i] / nsub[i];
    d.h_pred = T(0.5 * hr);
    d.h_corr = T(hr);
    d.ctr = h->b.ctr;
    // the persistent launch runs both stages at the batch's rows
    const rhdk::TileGrid tp =
        b->persistent ? tile_counts(h, b->rows, b->zchunk)
                      : tile_counts(h, predict_rows(h->mixed, b->rows), predict_chunk(h->mixed, b->zchunk));
    const rhdk::TileGrid tg = tile_counts(h, b->rows, b->zchunk);
    d.zc_pred = tp.zc_pred;
    d.zc_corr = tg.zc_corr;
    d.tiles_pred = tp.pred[0] * tp.pred[1] * tp.pred[2];
    d.tiles_corr = tg.corr[0] * tg.corr[1] * tg.corr[2];
    desc[k] = d;
    for (int z = 0; z < tp.pred[2]; ++z)
      for (int y = 0; y < tp.pred[1]; ++y)
        for (int x = 0; x < tp.pred[0]; ++x) b->h_tiles_pred[np++] = make_int4(k, x, y, z);
    for (int z = 0; z < tg.corr[2]; ++z)
      for (int y = 0; y < tg.corr[1]; ++y)
        for (int x = 0; x < tg.corr[0]; ++x) b->h_tiles_corr[nc++] = make_int4(k, x, y, z);
    pred_end[k] = np;
    corr_end[k] = nc;
  }
  const int rounds = S > 0 ? nsub[order[0]] : 0;
  for (int r = 0; r < rounds; ++r) {
    int k = 0;
    while (k < S && nsub[order[k]] > r) ++k;
    b->h_counts[2 * r] = k > 0 ? pred_end[k - 1] : 0;
    b->h_counts[2 * r + 1] = k > 0 ? corr_end[k - 1] : 0;
  }
  BHIP_TRY(b, hipMemcpyAsync(b->d_desc, desc, size_t(S) * sizeof(rhdk::SolveDesc<T>),
                             hipMemcpyHostToDevice, b->stream));
  BHIP_TRY(b, hipMemcpyAsync(b->d_tiles_pred, b->h_tiles_pred, size_t(np) * sizeof(int4),
                             hipMemcpyHostToDevice, b->stream));
  BHIP_TRY(b, hipMemcpyAsync(b->d_tiles_corr, b->h_tiles_corr, size_t(nc) * sizeof(int4),
                             hipMemcpyHostToDevice, b->stream));
  BHIP_TRY(b, hipMemcpyAsync(b->d_counts, b->h_counts, size_t(2 * rounds) * sizeof(int),
                             hipMemcpyHostToDevice, b->stream));
  if (b->persistent && rounds > 0) {
    // one launch for every subcycle of every member: level l is stage l of the rounds
    int acc = 0, widest = 0;
    for (int l = 0; l < 2 * rounds; ++l) {
      b->h_level[l] = acc;
      acc += b->h_counts[l];
      widest = std::max(widest, b->h_counts[l]);
    }
    b->h_level[2 * rounds] = acc;
    BHIP_TRY(b, hipMemcpyAsync(b->d_level, b->h_level, size_t(2 * rounds + 1) * sizeof(int),
                               hipMemcpyHostToDevice, b->stream));
    switch (b->rows) {
      case 4:
        if (int rc = launch_persistent<T, 4>(b, S, 2 * rounds, acc, widest)) return rc;
        break;
      case 8:
        if (int rc = launch_persistent<T, 8>(b, S, 2 * rounds, acc, widest)) return rc;
        break;
      default:
        if constexpr (sizeof(T) == 4) {
          if (int rc = launch_persistent<T, 16>(b, S, 2 * rounds, acc, widest)) return rc;
        }
        break;
    }
  } else {
    for (int r = 0; r < rounds; ++r) {
      switch (b->rows) {
        case 4:
          launch_batch_round<T, 4>(b, np, nc, r);
          break;
        case 8:
          launch_batch_round<T, 8>(b, np, nc, r);
          break;
        default:
          if constexpr (sizeof(T) == 4) launch_batch_round<T, 16>(b, np, nc, r);
          break;
      }
    }
  }
  BHIP_TRY(b, hipGetLastError());
  // 4. correction and ledger of every member
  for (int i = 0; i < S; ++i) {
    rhd_t* h = b->members[i];
    if (int rc = enqueue_post<T>(h, dt[i], b->chat[i])) return bfail(b, rc, "member %d: %s", i, h->err);
    h->steps += 1;
    h->subcycles += nsub[i];
    if (nsub_out) nsub_out[i] = nsub[i];
    if (dt_out) dt_out[i] = dt[i];
  }
  return RHD_OK;
}

}  // namespace

extern "C" {

int rhd_batch_create(void* hip_stream, int max_solves, int tile_rows, int zchunk,
                     rhd_batch_t** out) {
  if (!out) return bfail(nullptr, RHD_EINVAL, "out is NULL");
  *out = nullptr;
  if (max_solves < 1) return bfail(nullptr, RHD_EINVAL, "max_solves must be >= 1");
  if (tile_rows != 4 && tile_rows != 8 && tile_rows != 16)
    return bfail(nullptr, RHD_EINVAL, "tile_rows must be 4, 8 or 16");
  if (zchunk < 1) return bfail(nullptr, RHD_EINVAL, "zchunk must be >= 1");
  rhd_batch_t* b = new (std::nothrow) rhd_batch();
  if (!b) return bfail(nullptr, RHD_ENOMEM, "host allocation failed");
  b->max_solves = max_solves;
  b->rows = tile_rows;
  b->zchunk = zchunk;
  bool ok = true;
  if (hip_stream) {
    b->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    ok = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) == hipSuccess;
    b->own_stream = ok;
  }
  const size_t desc_bytes = size_t(max_solves) * sizeof(rhdk::SolveDesc<double>);
  ok = ok && hipMalloc(&b->d_desc, desc_bytes) == hipSuccess;
  ok = ok && hipHostMalloc(&b->h_desc, desc_bytes, hipHostMallocDefault) == hipSuccess;
  ok = ok && hipMalloc(&b->d_counts, 2 * BATCH_MAX_ROUNDS * sizeof(int)) == hipSuccess;
  ok = ok && hipHostMalloc(&b->h_counts, 2 * BATCH_MAX_ROUNDS * sizeof(int), hipHostMallocDefault) == hipSuccess;
  ok = ok && hipHostMalloc(&b->h_vmax, size_t(max_solves) * sizeof(double), hipHostMallocDefault) == hipSuccess;
  ok = ok && hipMalloc(&b->d_level, (2 * BATCH_MAX_ROUNDS + 1) * sizeof(int)) == hipSuccess;
  ok = ok && hipHostMalloc(&b->h_level, (2 * BATCH_MAX_ROUNDS + 1) * sizeof(int), hipHostMallocDefault) == hipSuccess;
  ok = ok && hipMalloc(&b->d_done, size_t(max_solves + 2) * rhdk::COUNTER_STRIDE * sizeof(unsigned)) ==
                   hipSuccess;
  ok = ok && hipHostMalloc(&b->h_err, sizeof(unsigned), hipHostMallocDefault) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&b->order_ev, hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    rhd_batch_destroy(b);
    return bfail(nullptr, RHD_ENOMEM, "batch allocation failed");
  }
  *out = b;
  return RHD_OK;
}

int rhd_batch_add(rhd_batch_t* b, rhd_t* h, double chat) {
  if (!b || !h) return bfail(b, RHD_EINVAL, "batch or handle is NULL");
  if (int(b->members.size()) >= b->max_solves) return bfail(b, RHD_EINVAL, "batch is full");
  if (!h->have_state) return bfail(b, RHD_ESTATE, "member has no state");
  if (!(h->G.act[0] && h->G.act[1] && h->G.act[2])) return bfail(b, RHD_EINVAL, "members must be 3D");
  if (h->fixed_mask) return bfail(b, RHD_EINVAL, "members cannot have fixed faces");
  if (!h->tile_ok) return bfail(b, RHD_EINVAL, "members' arrays must hold at most 4 GiB each");
  if (!(chat > 0.0)) return bfail(b, RHD_EINVAL, "chat must be > 0");
  for (rhd_t* m : b->members)
    if (m == h) return bfail(b, RHD_EINVAL, "handle is already a member");
  if (h->in_batch) return bfail(b, RHD_EINVAL, "handle belongs to another batch");
  const int prec = h->mixed ? 1 : 0;
  if (b->precision >= 0 && prec != b->precision)
    return bfail(b, RHD_EINVAL, "member precision differs from the batch's");
  if (!h->mixed && b->rows == 16) return bfail(b, RHD_EINVAL, "16-row tiles need mixed precision");
  // room for the predictor's tiles at either row count (the persistent launch uses the
  // batch's rows, the round launches the predictor's own)
  auto pred_tiles = [&](const rhd_t* m) {
    const rhdk::TileGrid a = tile_counts(m, b->rows, b->zchunk);
    const rhdk::TileGrid c =
        tile_counts(m, predict_rows(m->mixed, b->rows), predict_chunk(m->mixed, b->zchunk));
    return std::max(a.pred[0] * a.pred[1] * a.pred[2], c.pred[0] * c.pred[1] * c.pred[2]);
  };
  const rhdk::TileGrid tg = tile_counts(h, b->rows, b->zchunk);
  int need_p = pred_tiles(h), need_c = tg.corr[0] * tg.corr[1] * tg.corr[2];
  for (rhd_t* m : b->members) {
    const rhdk::TileGrid t2 = tile_counts(m, b->rows, b->zchunk);
    need_p += pred_tiles(m);
    need_c += t2.corr[0] * t2.corr[1] * t2.corr[2];
  }
  if (int rc = batch_reserve(b, need_p, need_c)) return rc;
  // the batch stream takes over the member: its work waits for what the member's own
  // stream holds (the state upload, for instance)
  BHIP_TRY(b, hipEventRecord(b->order_ev, h->stream));
  BHIP_TRY(b, hipStreamWaitEvent(b->stream, b->order_ev, 0));
  b->precision = prec;
  b->members.push_back(h);
  b->chat.push_back(chat);
  b->saved_streams.push_back(h->stream);
  h->stream = b->stream;
  h->in_batch = true;
  h->batch = b;
  return RHD_OK;
}

int rhd_batch_remove(rhd_batch_t* b, rhd_t* h) {
  if (!b || !h) return bfail(b, RHD_EINVAL, "batch or handle is NULL");
  for (size_t i = 0; i < b->members.size(); ++i) {
    if (b->members[i] != h) continue;
    // the member's own stream takes over after the batch's work enqueued so far
    BHIP_TRY(b, hipEventRecord(b->order_ev, b->stream));
    BHIP_TRY(b, hipStreamWaitEvent(b->saved_streams[i], b->order_ev, 0));
    h->stream = b->saved_streams[i];
    h->in_batch = false;
    h->batch = nullptr;
    b->members.erase(b->members.begin() + long(i));
    b->chat.erase(b->chat.begin() + long(i));
    b->saved_streams.erase(b->saved_streams.begin() + long(i));
    return RHD_OK;
  }
  return bfail(b, RHD_EINVAL, "handle is not a member");
}

int rhd_batch_step(rhd_batch_t* b, int* nsub_out, double* dt_out) {
  if (!b) return bfail(nullptr, RHD_EINVAL, "batch is NULL");
  if (b->members.empty()) return RHD_OK;
  return b->precision == 1 ? batch_step_impl<float>(b, nsub_out, dt_out)
                           : batch_step_impl<double>(b, nsub_out, dt_out);
}

int rhd_batch_size(const rhd_batch_t* b) { return b ? int(b->members.size()) : 0; }

int rhd_batch_set_persistent(rhd_batch_t* b, int on) {
  if (!b) return bfail(nullptr, RHD_EINVAL, "batch is NULL");
  if (on)
    return bfail(b, RHD_EINVAL, "the persistent launch is switched off: it did not finish on "
                                "the GPU; batches run their subcycles as rounds of launches");
  b->persistent = false;
  return RHD_OK;
}

int rhd_batch_sync(rhd_batch_t* b) {
  if (!b) return bfail(nullptr, RHD_EINVAL, "batch is NULL");
  BHIP_TRY(b, hipStreamSynchronize(b->stream));
  return batch_check_persistent(b);
}

void rhd_batch_destroy(rhd_batch_t* b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  for (size_t i = 0; i < b->members.size(); ++i) {
    b->members[i]->stream = b->saved_streams[i];
    b->members[i]->in_batch = false;
    b->members[i]->batch = nullptr;
  }
  if (b->d_desc) (void)hipFree(b->d_desc);
  if (b->h_desc) (void)hipHostFree(b->h_desc);
  if (b->d_tiles_pred) (void)hipFree(b->d_tiles_pred);
  if (b->h_tiles_pred) (void)hipHostFree(b->h_tiles_pred);
  if (b->d_tiles_corr) (void)hipFree(b->d_tiles_corr);
  if (b->h_tiles_corr) (void)hipHostFree(b->h_tiles_corr);
  if (b->d_counts) (void)hipFree(b->d_counts);
  if (b->h_counts) (void)hipHostFree(b->h_counts);
  if (b->h_vmax) (void)hipHostFree(b->h_vmax);
  if (b->d_level) (void)hipFree(b->d_level);
  if (b->h_level) (void)hipHostFree(b->h_level);
  if (b->d_done) (void)hipFree(b->d_done);
  if (b->h_err) (void)hipHostFree(b->h_err);
  if (b->order_ev) (void)hipEventDestroy(b->order_ev);
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

const char* rhd_batch_last_error(const rhd_batch_t* b) { return b ? b->err : g_batch_error; }

void rhd_destroy(rhd_t* h) {
  if (!h) return;
  // a member leaves its batch first, so the batch holds no pointer to freed buffers
  if (h->in_batch && h->batch) (void)rhd_batch_remove(h->batch, h);
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  if (h->timer.start) {
    for (int i = 0; i < Timer::POOL; ++i) {
      (void)hipEventDestroy(h->timer.start[i]);
      (void)hipEventDestroy(h->timer.stop[i]);
    }
    delete[] h->timer.start;
    delete[] h->timer.stop;
  }
  if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
  free_buffers(h);
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
}

const char* rhd_last_error(const rhd_t* h) { return h ? h->err : g_create_error; }

}  // extern "C"

// ---------------------------------------------------------------------------
// radiation subcycles without allocation (rhd_subcycles_noalloc)
// ---------------------------------------------------------------------------
//
// The half-step arrays and the counters live in one file-scope device array. In host
// code its name is only a host-side stand-in: its device address comes from
// hipGetSymbolAddress, once per device, and only that address is handed to kernels.

static __device__ __align__(256) unsigned char scratch[RHD_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Device address of the scratch array on device dev, looked up on the first call there.
int scratch_on_device(int dev, unsigned char** out) {
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
    return fail(nullptr, RHD_EDEVICE, "device %d out of range for the scratch table", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(nullptr, RHD_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s",
                  hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
  return RHD_OK;
}

}  // namespace

extern "C" {

long long rhd_subcycles_noalloc_bytes(const rhd_params* p) {
  if (!p || p->nx < 1 || p->ny < 1 || p->nz < 1) return -1;
  long long N, NP;
  footprint(p, &N, &NP);
  const size_t es = (p->flags & RHD_PRECISION_MIXED) ? 4 : 8;
  return (long long)(align256(rhdk::CTR_COUNT * sizeof(unsigned long long)) +
                     4 * align256(size_t(NP) * es));
}

int rhd_subcycles_noalloc(const rhd_params* p, void* hip_stream, void* Er, void* Fr,
                          const void* rho, const void* mom, const void* kappaP,
                          const void* kappaF, double kappaP_s, double kappaF_s, const void* j,
                          double dt_gas, double chat, int nsub) {
  int rc = validate(p);
  if (rc) return rc;
  if (p->flags & RHD_OPACITY_LAW)
    return fail(nullptr, RHD_EINVAL, "RHD_OPACITY_LAW is not available without allocation");
  for (int f = 0; f < 6; ++f)
    if (p->bc[f] == RHD_BC_FIXED && (f < 2 ? p->nx : (f < 4 ? p->ny : p->nz)) > 1)
      return fail(nullptr, RHD_EINVAL, "fixed faces are not available without allocation");
  const long long need = rhd_subcycles_noalloc_bytes(p);
  if (need > (long long)RHD_NOALLOC_SCRATCH_BYTES)
    return fail(nullptr, RHD_EINVAL,
                "grid %dx%dx%d needs %lld bytes of scratch, above the limit of %lld bytes",
                p->nx, p->ny, p->nz, need, (long long)RHD_NOALLOC_SCRATCH_BYTES);
  if (!Er || !Fr || !rho) return fail(nullptr, RHD_EINVAL, "Er, Fr and rho must be non-NULL");
  if ((p->flags & RHD_BETA_TAU) && !mom)
    return fail(nullptr, RHD_EINVAL, "RHD_BETA_TAU needs the momentum (mom)");
  if ((kappaP == nullptr) != (kappaF == nullptr))
    return fail(nullptr, RHD_EINVAL, "give both per-cell opacity arrays or neither");
  if (!kappaP && (!(kappaP_s >= 0.0) || !(kappaF_s >= 0.0)))
    return fail(nullptr, RHD_EINVAL, "scalar opacities must be >= 0");
  if (!(dt_gas > 0.0) || !std::isfinite(dt_gas))
    return fail(nullptr, RHD_EINVAL, "dt_gas must be finite and > 0 (got %g)", dt_gas);
  if (!(chat > 0.0) || !std::isfinite(chat))
    return fail(nullptr, RHD_EINVAL, "chat must be finite and > 0 (got %g)", chat);
  if (nsub < 1) return fail(nullptr, RHD_EINVAL, "nsub must be >= 1 (got %d)", nsub);
  if (chat * dt_gas / nsub > p->cfl * min_width(p) * (1.0 + 1e-12))
    return fail(nullptr, RHD_ECFL, "chat dt_gas / nsub = %g exceeds K0 dx = %g",
                chat * dt_gas / nsub, p->cfl * min_width(p));
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(nullptr, RHD_EDEVICE, "no HIP device");
  unsigned char* base = nullptr;
  if ((rc = scratch_on_device(dev, &base))) return rc;

  // a handle on the stack: it owns nothing, and points at the caller's arrays and at
  // the scratch array
  rhd h;
  h.p = *p;
  h.mixed = (p->flags & RHD_PRECISION_MIXED) != 0;
  h.esize = h.mixed ? 4 : 8;
  h.stream = static_cast<hipStream_t>(hip_stream);
  h.device = dev;
  h.G = make_geom(p);
  long long N, NP;
  footprint(p, &N, &NP);
  h.N = int(N);
  h.NP = int(NP);
  h.dxmin = min_width(p);
  h.tile_ok = true;  // NP * esize is below the scratch limit, far below 4 GiB
  const size_t es = h.esize;
  unsigned char* fr = static_cast<unsigned char*>(Fr);
  h.b.rad[0] = Er;
  for (int q = 0; q < 3; ++q) h.b.rad[1 + q] = fr + size_t(q) * size_t(N) * es;
  h.b.gas[0] = const_cast<void*>(rho);
  for (int q = 0; q < 3; ++q)
    h.b.gas[1 + q] = mom ? static_cast<unsigned char*>(const_cast<void*>(mom)) + size_t(q) * size_t(N) * es
                         : nullptr;
  h.kappa_scalar = kappaP == nullptr;
  h.b.kP = const_cast<void*>(kappaP);
  h.b.kF = const_cast<void*>(kappaF);
  h.kP_s = kappaP_s;
  h.kF_s = kappaF_s;
  h.b.j = const_cast<void*>(j);
  h.b.ctr = reinterpret_cast<unsigned long long*>(base);
  size_t off = align256(rhdk::CTR_COUNT * sizeof(unsigned long long));
  for (int q = 0; q < 4; ++q) {
    h.b.rh[q] = base + off;
    off += align256(size_t(NP) * es);
  }
  // the counters start from zero on every call, with a kernel (a captured memset node
  // is what this entry point's callers avoid)
  hipLaunchKernelGGL(rhdk::k_reset_counters, dim3(1), dim3(64), 0, h.stream, h.b.ctr);
  rc = h.mixed ? enqueue_subcycles<float>(&h, dt_gas, chat, nsub)
               : enqueue_subcycles<double>(&h, dt_gas, chat, nsub);
  if (rc == RHD_OK) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
      rc = fail(&h, RHD_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
  }
  if (rc != RHD_OK) snprintf(g_create_error, sizeof(g_create_error), "%s", h.err);
  return rc;
}

}  // extern "C"
