/*
 * rhd_oracle.c -- plain FP64 CPU oracle for one operator-split step of the gray
 * two-moment (M1) radiation-hydrodynamics method of Skinner & Ostriker (2013),
 * "A two-moment radiation hydrodynamics module in Athena using a time-explicit
 * Godunov method".
 *
 * TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg of
 * the benchmark are the only users. Nothing here is shared with the GPU library.
 *
 * Every quantity is double precision. The code is written for checking by eye
 * against the paper, not for speed: each field set is copied into arrays with
 * explicit ghost layers, ghosts are filled from the boundary conditions, each stage
 * loops over cells and recomputes both face fluxes of every cell, and each step of
 * the algorithm of Sec. 3.1 is a function of its own.
 *
 * Readings taken where the paper is silent or garbled (each is also listed in the
 * design notes of the repository):
 *  - the implicit exchange runs once per gas step on dt_gas (Sec. 3.4 text and
 *    step 2 of the algorithm in Sec. 3.1), not on dt_rad as Eq. source:energyupdate
 *    is printed;
 *  - the radiation subcycles see the gas state after the gas transport step and
 *    before the second-order source correction (Sec. 3.4, last paragraphs);
 *  - the theta-scheme of Eq. source:stiff:radmomentum:soln is applied to F in each
 *    Van Leer stage over that stage's step, from the old state U^m, with the flux
 *    divergence and the explicit sources added on the same implicit footing;
 *  - piecewise-linear reconstruction uses the monotonised-central (MC) limiter,
 *    componentwise, on (E_r, F) and on the gas primitives (rho, v, P);
 *  - the reduced flux is clamped to f <= 1 and the eigenvalue radicand to >= 0;
 *    mu = 0 when F = 0; HLL falls back to the central flux when S_R+ - S_L- = 0;
 *  - the HLL flux is Eq. hyperbolic:hllflux2 (Eq. hyperbolic:hllflux1 is garbled);
 *  - the gas Riemann solver is HLLC with Davis wave speeds (HLLE when isothermal);
 *  - the O(beta tau) switch turns all four velocity terms of S_e on or off
 *    together; the radiation force rho kappa_F F/c on the gas is always on;
 *  - kappa_P multiplies the (a_R T^4 - E_r) terms and kappa_F the F and v terms;
 *  - the predictor is evaluated on the interior plus two ghost layers from U^m
 *    with three ghost layers filled; the corrector uses those predicted ghosts
 *    directly (no boundary refill between the stages);
 *  - after every radiation stage E_r is raised to er_floor and then F is scaled
 *    back to |F| = c E_r if it exceeds it, and E_r of every reconstructed face state
 *    is raised to er_floor before its closure; E_r after the exchange is raised to
 *    er_floor too (Eq. source:eradupdate can round to zero or below when K of
 *    Eq. source:kappacond is large); after every gas stage rho and P are
 *    raised to their floors;
 *  - emission j adds (chat/c) j to dE_r/dt, so that div F = j in a steady state;
 *  - in ABSORB_ONLY mode E_r is damped with kappa_P by the same theta-form as F,
 *    with theta_F, on each radiation stage;
 *  - a fixed (Dirichlet) radiation face, as the Marshak problem of Sec. 4.1.3 needs,
 *    holds its state in every ghost cell beyond it, for U^m and for the predicted
 *    U^{m+1/2} (the predictor does not evolve those ghosts), while the gas fields
 *    continue zero-gradient there;
 *  - with c_v = alpha T^3 (Sec. 4.1.3) the exchange keeps the theta-scheme form of
 *    Eq. source:energyupdate with a_R T^4 = (4 a_R/alpha) e, which makes the update
 *    linear in e; with chat = c it is the update printed with that problem;
 *  - an opacity law kappa(T_gas, rho) (the shadow test of Sec. 4.1.1) gives the one
 *    absorption opacity for kappa_P and kappa_F, evaluated from the gas state at the
 *    start of each gas step and held through the step (exchange, gas step and
 *    subcycles), and from the current state for the CFL step.
 */
#include "rhd_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* padded grid                                                               */
/* ------------------------------------------------------------------------- */

typedef struct {
  int n[3]; /* interior cells per dimension            */
  int g[3]; /* ghost width (0 in an inactive dimension) */
  int s[3]; /* padded extent n + 2 g                    */
} pgrid;

static pgrid make_grid(const orc_params *p, int ng) {
  pgrid G;
  G.n[0] = p->nx;
  G.n[1] = p->ny;
  G.n[2] = p->nz;
  for (int d = 0; d < 3; ++d) {
    G.g[d] = G.n[d] > 1 ? ng : 0;
    G.s[d] = G.n[d] + 2 * G.g[d];
  }
  return G;
}

static long at(const pgrid *G, int i, int j, int k) {
  return (long)(i + G->g[0]) +
         (long)G->s[0] * ((long)(j + G->g[1]) + (long)G->s[1] * (long)(k + G->g[2]));
}

static long padded_size(const pgrid *G) {
  return (long)G->s[0] * G->s[1] * G->s[2];
}

static long interior_index(const orc_params *p, int i, int j, int k) {
  return (long)i + (long)p->nx * ((long)j + (long)p->ny * k);
}

static double *alloc_field(const pgrid *G) {
  return (double *)calloc((size_t)padded_size(G), sizeof(double));
}

static double cell_width(const orc_params *p, int d) {
  return d == 0 ? p->dx : (d == 1 ? p->dy : p->dz);
}

static double min_width(const orc_params *p) {
  double w = p->dx;
  if (p->ny > 1 && p->dy < w) w = p->dy;
  if (p->nz > 1 && p->dz < w) w = p->dz;
  return w;
}

/* Copy an interior array into a padded array (ghosts left for fill_ghosts). */
static void load_padded(const orc_params *p, const pgrid *G, const double *src, double *dst) {
  for (int k = 0; k < p->nz; ++k)
    for (int j = 0; j < p->ny; ++j)
      for (int i = 0; i < p->nx; ++i)
        dst[at(G, i, j, k)] = src[interior_index(p, i, j, k)];
}

static void store_interior(const orc_params *p, const pgrid *G, const double *src, double *dst) {
  for (int k = 0; k < p->nz; ++k)
    for (int j = 0; j < p->ny; ++j)
      for (int i = 0; i < p->nx; ++i)
        dst[interior_index(p, i, j, k)] = src[at(G, i, j, k)];
}

/*
 * Fill the ghost layers of nf padded fields. comp[f] is the Cartesian component a
 * vector field carries (0, 1, 2) or -1 for a scalar: a reflecting face flips the
 * component normal to it. Dimensions are filled in order x, y, z over the full
 * padded range of the other dimensions, so edges and corners are filled too.
 */
static void fill_ghosts(const orc_params *p, const pgrid *G, double **f, const int *comp, int nf) {
  for (int d = 0; d < 3; ++d) {
    if (G->g[d] == 0) continue;
    const int n = G->n[d];
    int lo[3], hi[3];
    for (int e = 0; e < 3; ++e) {
      lo[e] = -G->g[e];
      hi[e] = G->n[e] + G->g[e];
    }
    for (int k = lo[2]; k < hi[2]; ++k)
      for (int j = lo[1]; j < hi[1]; ++j)
        for (int i = lo[0]; i < hi[0]; ++i) {
          int c[3] = {i, j, k};
          int q = c[d];
          if (q >= 0 && q < n) continue;
          int kind = q < 0 ? p->bc[2 * d] : p->bc[2 * d + 1];
          int src = 0;
          double flip = 1.0;
          if (kind == ORC_BC_PERIODIC) {
            src = ((q % n) + n) % n;
          } else if (kind == ORC_BC_OUTFLOW || kind == ORC_BC_FIXED) {
            src = q < 0 ? 0 : n - 1;
          } else { /* reflect */
            src = q < 0 ? -1 - q : 2 * n - 1 - q;
            flip = -1.0;
          }
          int cs[3] = {i, j, k};
          cs[d] = src;
          long dst_at = at(G, c[0], c[1], c[2]);
          long src_at = at(G, cs[0], cs[1], cs[2]);
          for (int m = 0; m < nf; ++m)
            f[m][dst_at] = (comp[m] == d ? flip : 1.0) * f[m][src_at];
        }
  }
}

/*
 * The fixed face whose radiation state the padded cell (i, j, k) holds, or -1: of the
 * dimensions in which the cell lies beyond a fixed face, the last in the order x, y, z
 * (the order fill_ghosts fills them in).
 */
static int fixed_face(const orc_params *p, const pgrid *G, int i, int j, int k) {
  const int c[3] = {i, j, k};
  int face = -1;
  for (int d = 0; d < 3; ++d) {
    if (G->g[d] == 0) continue;
    if (c[d] < 0 && p->bc[2 * d] == ORC_BC_FIXED) face = 2 * d;
    if (c[d] >= G->n[d] && p->bc[2 * d + 1] == ORC_BC_FIXED) face = 2 * d + 1;
  }
  return face;
}

/* Put the fixed faces' radiation states into the ghost cells of (E_r, F_x, F_y, F_z). */
static void apply_fixed(const orc_params *p, const pgrid *G, double *const U[4]) {
  int any = 0;
  for (int f = 0; f < 6; ++f) any |= p->bc[f] == ORC_BC_FIXED;
  if (!any) return;
  for (int k = -G->g[2]; k < G->n[2] + G->g[2]; ++k)
    for (int j = -G->g[1]; j < G->n[1] + G->g[1]; ++j)
      for (int i = -G->g[0]; i < G->n[0] + G->g[0]; ++i) {
        const int f = fixed_face(p, G, i, j, k);
        if (f < 0) continue;
        const long a = at(G, i, j, k);
        for (int q = 0; q < 4; ++q) U[q][a] = p->bval[f][q];
      }
}

/* ------------------------------------------------------------------------- */
/* M1 closure (Sec. 2.3)                                                      */
/* ------------------------------------------------------------------------- */

/* Levermore's Eddington factor chi(f), Eq. m1:chi. */
void orc_m1_eddington_factor(double f, double *chi) {
  *chi = (3.0 + 4.0 * f * f) / (5.0 + 2.0 * sqrt(4.0 - 3.0 * f * f));
}

static double reduced_flux(double E, const double F[3], double c, double *Fnorm) {
  double Fn = sqrt(F[0] * F[0] + F[1] * F[1] + F[2] * F[2]);
  *Fnorm = Fn;
  double f = Fn / (c * E);
  if (f > 1.0) f = 1.0; /* realizability clamp */
  return f;
}

/*
 * Radiation pressure tensor P = E T with the M1 Eddington tensor
 * T = (1-chi)/2 I + (3 chi - 1)/2 n n, n = F/|F| (Eqs. m1:m1tns, m1:nhat, m1:chi).
 * P is returned row-major, P[3*a + b].
 */
void orc_m1_pressure(double E, const double F[3], double c, double P[9]) {
  double Fn;
  double f = reduced_flux(E, F, c, &Fn);
  double chi;
  orc_m1_eddington_factor(f, &chi);
  double iso = 0.5 * (1.0 - chi);
  double dir = 0.5 * (3.0 * chi - 1.0);
  double n[3] = {0.0, 0.0, 0.0};
  if (Fn > 0.0) {
    n[0] = F[0] / Fn;
    n[1] = F[1] / Fn;
    n[2] = F[2] / Fn;
  }
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      P[3 * a + b] = E * ((a == b ? iso : 0.0) + dir * n[a] * n[b]);
}

/*
 * Fastest left- and right-going wave speeds lambda_1, lambda_3 of the radiation
 * subsystem in direction d, Eq. hyperbolic:evals13, with mu = cos of the angle
 * between F and the face normal.
 */
void orc_m1_eigen(double E, const double F[3], double c, double chat, int d,
                  double *l1, double *l3) {
  double Fn;
  double f = reduced_flux(E, F, c, &Fn);
  double mu = Fn > 0.0 ? F[d] / Fn : 0.0;
  double s = sqrt(4.0 - 3.0 * f * f);
  double rad = (2.0 / 3.0) * (4.0 - 3.0 * f * f - s) + 2.0 * mu * mu * (2.0 - f * f - s);
  if (rad < 0.0) rad = 0.0;
  double r = sqrt(rad);
  *l1 = chat * (mu * f - r) / s;
  *l3 = chat * (mu * f + r) / s;
}

/* Physical flux of (E_r, F) in direction d: (chat F_d / c, chat c P_d.). */
static void rad_physical_flux(const double U[4], int d, double c, double chat, double Phi[4]) {
  double P[9];
  orc_m1_pressure(U[0], U + 1, c, P);
  Phi[0] = chat * U[1 + d] / c;
  Phi[1] = chat * c * P[3 * d + 0];
  Phi[2] = chat * c * P[3 * d + 1];
  Phi[3] = chat * c * P[3 * d + 2];
}

/*
 * HLL flux, Eq. hyperbolic:hllflux2, with S_L = min(lambda_1(U_L), lambda_1(U_R))
 * and S_R = max(lambda_3(U_L), lambda_3(U_R)). Central flux when both bounds
 * vanish (f = 1 streaming parallel to the face).
 */
void orc_rad_hll_flux(const double UL[4], const double UR[4], int d, double c,
                      double chat, double flux[4]) {
  double l1L, l3L, l1R, l3R;
  orc_m1_eigen(UL[0], UL + 1, c, chat, d, &l1L, &l3L);
  orc_m1_eigen(UR[0], UR + 1, c, chat, d, &l1R, &l3R);
  double SL = l1L < l1R ? l1L : l1R;
  double SR = l3L > l3R ? l3L : l3R;
  double SLm = SL < 0.0 ? SL : 0.0;
  double SRp = SR > 0.0 ? SR : 0.0;
  double PhiL[4], PhiR[4];
  rad_physical_flux(UL, d, c, chat, PhiL);
  rad_physical_flux(UR, d, c, chat, PhiR);
  double den = SRp - SLm;
  for (int q = 0; q < 4; ++q) {
    if (den > 0.0)
      flux[q] = (SRp * PhiL[q] - SLm * PhiR[q] + SRp * SLm * (UR[q] - UL[q])) / den;
    else
      flux[q] = 0.5 * (PhiL[q] + PhiR[q]);
  }
}

/*
 * HLL flux of the Eddington (P1) closure (Sec. 2.3: T proportional to I, so T = I/3
 * and P = E_r/3 I whatever F is). The wave speeds of that system are the f -> 0 limits
 * lambda_{1,3} = -+chat/sqrt(3) of Sec. 2.4 for every state; they enter
 * Eq. hyperbolic:hllflux2 as S_L and S_R.
 */
void orc_p1_hll_flux(const double UL[4], const double UR[4], int d, double c, double chat,
                     double flux[4]) {
  const double SL = -chat / sqrt(3.0), SR = chat / sqrt(3.0);
  double PhiL[4], PhiR[4];
  PhiL[0] = chat * UL[1 + d] / c;
  PhiR[0] = chat * UR[1 + d] / c;
  for (int e = 0; e < 3; ++e) {
    PhiL[1 + e] = e == d ? chat * c * UL[0] / 3.0 : 0.0;
    PhiR[1 + e] = e == d ? chat * c * UR[0] / 3.0 : 0.0;
  }
  for (int q = 0; q < 4; ++q)
    flux[q] = (SR * PhiL[q] - SL * PhiR[q] + SR * SL * (UR[q] - UL[q])) / (SR - SL);
}

/* The face flux of the closure the flags choose. */
static void face_flux(const orc_params *p, const double UL[4], const double UR[4], int d,
                      double chat, double flux[4]) {
  if (p->flags & ORC_CLOSURE_P1)
    orc_p1_hll_flux(UL, UR, d, p->c_light, chat, flux);
  else
    orc_rad_hll_flux(UL, UR, d, p->c_light, chat, flux);
}

/* ------------------------------------------------------------------------- */
/* piecewise-linear reconstruction                                            */
/* ------------------------------------------------------------------------- */

/* Monotonised-central limited slope from the backward and forward differences. */
double orc_mc_slope(double dm, double dp) {
  if (dm * dp <= 0.0) return 0.0;
  double a = fabs(0.5 * (dm + dp));
  double b = 2.0 * fabs(dm);
  double e = 2.0 * fabs(dp);
  double m = a < b ? a : b;
  m = m < e ? m : e;
  return dm > 0.0 ? m : -m;
}

/* ------------------------------------------------------------------------- */
/* radiation subsystem: one Van Leer stage (Sec. 3.3, Sec. 3.4)               */
/* ------------------------------------------------------------------------- */

typedef struct {
  double *rkF, *rkP; /* rho kappa_F, rho kappa_P of the frozen gas (padded) */
  double *v[3];      /* frozen gas velocity (padded)                         */
  double *j;         /* emissivity (padded) or NULL                          */
} frozen_gas;

static void gather4(double *const U[4], long a, double out[4]) {
  for (int q = 0; q < 4; ++q) out[q] = U[q][a];
}

/*
 * One stage of the radiation update on cells [lo, hi) per active dimension.
 *  Uin  : state whose face fluxes are taken (U^m in the predictor, U^{m+1/2} in
 *         the corrector), padded with valid values wide enough for the stencil;
 *  Uold : U^m, the state the stage advances from and that the theta-terms use;
 *  Usrc : state at which the explicit sources are evaluated (U^m, then U^{m+1/2}).
 * First-order fluxes take the cell states on each side of a face; second-order
 * fluxes take MC-limited linear reconstructions (Sec. 3.3).
 */
static void rad_stage(const orc_params *p, const pgrid *G, double chat, double h,
                      int second_order, int ext, double *const Uin[4],
                      double *const Uold[4], double *const Usrc[4], const frozen_gas *fg,
                      double *Uout[4], orc_counts *cnt) {
  const double c = p->c_light;
  const double b = (p->flags & ORC_BETA_TAU) ? 1.0 : 0.0;
  const int absorb_only = (p->flags & ORC_EXCH_MASK) == ORC_EXCH_ABSORB_ONLY;
  const double th = p->theta_F;
  int lo[3], hi[3];
  for (int d = 0; d < 3; ++d) {
    int e = G->g[d] > 0 ? ext : 0;
    lo[d] = -e;
    hi[d] = G->n[d] + e;
  }
  for (int k = lo[2]; k < hi[2]; ++k)
    for (int j = lo[1]; j < hi[1]; ++j)
      for (int i = lo[0]; i < hi[0]; ++i) {
        long a0 = at(G, i, j, k);
        double div[4] = {0.0, 0.0, 0.0, 0.0};
        for (int d = 0; d < 3; ++d) {
          if (G->g[d] == 0) continue;
          int off[3] = {0, 0, 0};
          off[d] = 1;
          long am1 = at(G, i - off[0], j - off[1], k - off[2]);
          long ap1 = at(G, i + off[0], j + off[1], k + off[2]);
          double fl[4], fr[4];
          if (!second_order) {
            double Um[4], U0[4], Up[4];
            gather4(Uin, am1, Um);
            gather4(Uin, a0, U0);
            gather4(Uin, ap1, Up);
            face_flux(p, Um, U0, d, chat, fl);
            face_flux(p, U0, Up, d, chat, fr);
          } else {
            long am2 = at(G, i - 2 * off[0], j - 2 * off[1], k - 2 * off[2]);
            long ap2 = at(G, i + 2 * off[0], j + 2 * off[1], k + 2 * off[2]);
            double Um2[4], Um[4], U0[4], Up[4], Up2[4];
            gather4(Uin, am2, Um2);
            gather4(Uin, am1, Um);
            gather4(Uin, a0, U0);
            gather4(Uin, ap1, Up);
            gather4(Uin, ap2, Up2);
            double sm[4], s0[4], sp[4];
            for (int q = 0; q < 4; ++q) {
              sm[q] = orc_mc_slope(Um[q] - Um2[q], U0[q] - Um[q]);
              s0[q] = orc_mc_slope(U0[q] - Um[q], Up[q] - U0[q]);
              sp[q] = orc_mc_slope(Up[q] - U0[q], Up2[q] - Up[q]);
            }
            double Lm[4], Rm[4], Lp[4], Rp[4];
            for (int q = 0; q < 4; ++q) {
              Lm[q] = Um[q] + 0.5 * sm[q]; /* left state of face i-1/2  */
              Rm[q] = U0[q] - 0.5 * s0[q]; /* right state of face i-1/2 */
              Lp[q] = U0[q] + 0.5 * s0[q]; /* left state of face i+1/2  */
              Rp[q] = Up[q] - 0.5 * sp[q]; /* right state of face i+1/2 */
            }
            /* E_r of a face state is raised to the floor: a face state may reach a
               neighbour's value, and next to a cell at the floor rounding can take it to
               zero, where the closure has no direction */
            Lm[0] = Lm[0] > p->er_floor ? Lm[0] : p->er_floor;
            Rm[0] = Rm[0] > p->er_floor ? Rm[0] : p->er_floor;
            Lp[0] = Lp[0] > p->er_floor ? Lp[0] : p->er_floor;
            Rp[0] = Rp[0] > p->er_floor ? Rp[0] : p->er_floor;
            face_flux(p, Lm, Rm, d, chat, fl);
            face_flux(p, Lp, Rp, d, chat, fr);
          }
          double w = cell_width(p, d);
          for (int q = 0; q < 4; ++q) div[q] += (fr[q] - fl[q]) / w;
        }

        double rkF = fg->rkF[a0], rkP = fg->rkP[a0];
        double v[3] = {fg->v[0][a0], fg->v[1][a0], fg->v[2][a0]};
        double Es = Usrc[0][a0];
        double Fs[3] = {Usrc[1][a0], Usrc[2][a0], Usrc[3][a0]};
        double vF = v[0] * Fs[0] + v[1] * Fs[1] + v[2] * Fs[2];

        /* radiation energy: transport + O(beta tau) work term + emission */
        double srcE = b * chat * rkF * vF / (c * c);
        if (fg->j) srcE += (chat / c) * fg->j[a0];
        double Eo = Uold[0][a0];
        double En;
        if (absorb_only) {
          double aP = chat * rkP * h;
          En = (Eo * (1.0 - (1.0 - th) * aP) + h * (-div[0] + srcE)) / (1.0 + th * aP);
        } else {
          En = Eo + h * (-div[0] + srcE);
        }

        /* radiation flux: theta-scheme absorption, Eq. source:stiff:radmomentum:soln */
        double a = chat * rkF * h;
        double Fn[3];
        for (int q = 0; q < 3; ++q) {
          double rhs = -div[1 + q] + b * (4.0 / 3.0) * chat * rkF * Es * v[q];
          Fn[q] = (Uold[1 + q][a0] * (1.0 - (1.0 - th) * a) + h * rhs) / (1.0 + th * a);
        }

        int interior = i >= 0 && i < G->n[0] && j >= 0 && j < G->n[1] && k >= 0 && k < G->n[2];
        if (En < p->er_floor) {
          En = p->er_floor;
          if (interior && cnt) cnt->rad_efloor++;
        }
        double Fmag = sqrt(Fn[0] * Fn[0] + Fn[1] * Fn[1] + Fn[2] * Fn[2]);
        if (Fmag > c * En) {
          double scale = c * En / Fmag;
          for (int q = 0; q < 3; ++q) Fn[q] *= scale;
          if (interior && cnt) cnt->rad_fclamp++;
        }
        Uout[0][a0] = En;
        Uout[1][a0] = Fn[0];
        Uout[2][a0] = Fn[1];
        Uout[3][a0] = Fn[2];
      }
}

/* ------------------------------------------------------------------------- */
/* gas subsystem                                                              */
/* ------------------------------------------------------------------------- */

static int isothermal(const orc_params *p) { return (p->flags & ORC_ISOTHERMAL) != 0; }

/* primitive state W = (rho, vx, vy, vz, P) from conserved U = (rho, m, E) */
static void cons_to_prim(const orc_params *p, const double U[5], double W[5]) {
  W[0] = U[0];
  W[1] = U[1] / U[0];
  W[2] = U[2] / U[0];
  W[3] = U[3] / U[0];
  if (isothermal(p)) {
    W[4] = U[0] * p->iso_cs * p->iso_cs;
  } else {
    double ke = 0.5 * (U[1] * U[1] + U[2] * U[2] + U[3] * U[3]) / U[0];
    W[4] = (p->gamma - 1.0) * (U[4] - ke);
  }
}

static void prim_to_cons(const orc_params *p, const double W[5], double U[5]) {
  U[0] = W[0];
  U[1] = W[0] * W[1];
  U[2] = W[0] * W[2];
  U[3] = W[0] * W[3];
  if (isothermal(p))
    U[4] = 0.0;
  else
    U[4] = W[4] / (p->gamma - 1.0) + 0.5 * W[0] * (W[1] * W[1] + W[2] * W[2] + W[3] * W[3]);
}

static double sound_speed(const orc_params *p, const double W[5]) {
  if (isothermal(p)) return p->iso_cs;
  return sqrt(p->gamma * W[4] / W[0]);
}

/* Euler flux in direction d from a primitive state (Eq. algorithm:variables); an
 * isothermal gas takes P = rho c_s^2 whatever W[4] holds. */
void orc_gas_flux(const double W[5], int d, const orc_params *p, double flux[5]) {
  double U[5];
  prim_to_cons(p, W, U);
  double un = W[1 + d];
  double P = isothermal(p) ? W[0] * p->iso_cs * p->iso_cs : W[4];
  flux[0] = U[0] * un;
  flux[1] = U[1] * un;
  flux[2] = U[2] * un;
  flux[3] = U[3] * un;
  flux[1 + d] += P;
  flux[4] = isothermal(p) ? 0.0 : (U[4] + P) * un;
}

/*
 * Gas Riemann solver across a face normal to d: HLLC with Davis wave-speed bounds
 * for an ideal gas, HLLE for an isothermal gas.
 */
void orc_gas_riemann(const double WL[5], const double WR[5], int d, const orc_params *p,
                     double flux[5]) {
  double aL = sound_speed(p, WL), aR = sound_speed(p, WR);
  double uL = WL[1 + d], uR = WR[1 + d];
  double SL = uL - aL < uR - aR ? uL - aL : uR - aR;
  double SR = uL + aL > uR + aR ? uL + aL : uR + aR;
  double UL[5], UR[5], FL[5], FR[5];
  prim_to_cons(p, WL, UL);
  prim_to_cons(p, WR, UR);
  orc_gas_flux(WL, d, p, FL);
  orc_gas_flux(WR, d, p, FR);

  if (isothermal(p)) {
    double SLm = SL < 0.0 ? SL : 0.0;
    double SRp = SR > 0.0 ? SR : 0.0;
    double den = SRp - SLm;
    for (int q = 0; q < 4; ++q)
      flux[q] = (SRp * FL[q] - SLm * FR[q] + SRp * SLm * (UR[q] - UL[q])) / den;
    flux[4] = 0.0;
    return;
  }

  if (SL >= 0.0) {
    for (int q = 0; q < 5; ++q) flux[q] = FL[q];
    return;
  }
  if (SR <= 0.0) {
    for (int q = 0; q < 5; ++q) flux[q] = FR[q];
    return;
  }
  /* contact speed and star states (Toro, HLLC) */
  double rL = WL[0], rR = WR[0], PL = WL[4], PR = WR[4];
  double SM = (PR - PL + rL * uL * (SL - uL) - rR * uR * (SR - uR)) /
              (rL * (SL - uL) - rR * (SR - uR));
  const double *Wk, *Uk, *Fk;
  double Sk;
  if (SM >= 0.0) {
    Wk = WL; Uk = UL; Fk = FL; Sk = SL;
  } else {
    Wk = WR; Uk = UR; Fk = FR; Sk = SR;
  }
  double uk = Wk[1 + d];
  double fac = Wk[0] * (Sk - uk) / (Sk - SM);
  double Us[5];
  Us[0] = fac;
  Us[1] = fac * Wk[1];
  Us[2] = fac * Wk[2];
  Us[3] = fac * Wk[3];
  Us[1 + d] = fac * SM;
  Us[4] = fac * (Uk[4] / Wk[0] + (SM - uk) * (SM + Wk[4] / (Wk[0] * (Sk - uk))));
  for (int q = 0; q < 5; ++q) flux[q] = Fk[q] + Sk * (Us[q] - Uk[q]);
}

/*
 * Explicit gas source S_e,gas (Eq. algorithm:source:explicit:gas without gravity):
 * momentum rho kF F/c - b (4/3) rho kF E_r v/c, energy -b rho kF v.F/c.
 * S[0] (density) is zero.
 */
static void gas_explicit_source(const orc_params *p, double rho, const double v[3],
                                double kF, double Er, const double F[3], double S[5]) {
  const double c = p->c_light;
  const double b = (p->flags & ORC_BETA_TAU) ? 1.0 : 0.0;
  double rk = rho * kF;
  S[0] = 0.0;
  for (int q = 0; q < 3; ++q) S[1 + q] = rk * F[q] / c - b * (4.0 / 3.0) * rk * Er * v[q] / c;
  S[4] = isothermal(p) ? 0.0 : -b * rk * (v[0] * F[0] + v[1] * F[1] + v[2] * F[2]) / c;
}

static void apply_gas_floors(const orc_params *p, double U[5], int interior, orc_counts *cnt) {
  if (U[0] < p->rho_floor) {
    U[0] = p->rho_floor;
    if (interior && cnt) cnt->gas_rhofloor++;
  }
  if (!isothermal(p)) {
    double ke = 0.5 * (U[1] * U[1] + U[2] * U[2] + U[3] * U[3]) / U[0];
    double P = (p->gamma - 1.0) * (U[4] - ke);
    if (P < p->p_floor) {
      U[4] = p->p_floor / (p->gamma - 1.0) + ke;
      if (interior && cnt) cnt->gas_pfloor++;
    }
  }
}

/*
 * One Van Leer stage of the gas subsystem (Eq. algorithm:gastransport) on cells
 * [lo, hi): U_out = U_old - h div F(U_in) + h S_e,gas(U_in, U_r). When s_save is
 * given, the source values and (rho, v) of U_in are stored per interior cell for
 * the second-order correction after the radiation subcycles.
 */
static void gas_stage(const orc_params *p, const pgrid *G, double h, int second_order,
                      int ext, double *const Uin[5], double *const Uold[5],
                      double *const Ur[4], const double *kF, double *Uout[5],
                      double *s_save[4], double *w_save[4], orc_counts *cnt) {
  int lo[3], hi[3];
  for (int d = 0; d < 3; ++d) {
    int e = G->g[d] > 0 ? ext : 0;
    lo[d] = -e;
    hi[d] = G->n[d] + e;
  }
  for (int k = lo[2]; k < hi[2]; ++k)
    for (int j = lo[1]; j < hi[1]; ++j)
      for (int i = lo[0]; i < hi[0]; ++i) {
        long a0 = at(G, i, j, k);
        double div[5] = {0, 0, 0, 0, 0};
        for (int d = 0; d < 3; ++d) {
          if (G->g[d] == 0) continue;
          int off[3] = {0, 0, 0};
          off[d] = 1;
          double W[5][5]; /* primitives at i-2 .. i+2 along d */
          int reach = second_order ? 2 : 1;
          for (int t = -reach; t <= reach; ++t) {
            long a = at(G, i + t * off[0], j + t * off[1], k + t * off[2]);
            double U[5] = {Uin[0][a], Uin[1][a], Uin[2][a], Uin[3][a], Uin[4][a]};
            cons_to_prim(p, U, W[t + 2]);
          }
          double fl[5], fr[5];
          if (!second_order) {
            orc_gas_riemann(W[1], W[2], d, p, fl);
            orc_gas_riemann(W[2], W[3], d, p, fr);
          } else {
            double sm[5], s0[5], sp[5];
            for (int q = 0; q < 5; ++q) {
              sm[q] = orc_mc_slope(W[1][q] - W[0][q], W[2][q] - W[1][q]);
              s0[q] = orc_mc_slope(W[2][q] - W[1][q], W[3][q] - W[2][q]);
              sp[q] = orc_mc_slope(W[3][q] - W[2][q], W[4][q] - W[3][q]);
            }
            double Lm[5], Rm[5], Lp[5], Rp[5];
            for (int q = 0; q < 5; ++q) {
              Lm[q] = W[1][q] + 0.5 * sm[q];
              Rm[q] = W[2][q] - 0.5 * s0[q];
              Lp[q] = W[2][q] + 0.5 * s0[q];
              Rp[q] = W[3][q] - 0.5 * sp[q];
            }
            orc_gas_riemann(Lm, Rm, d, p, fl);
            orc_gas_riemann(Lp, Rp, d, p, fr);
          }
          double w = cell_width(p, d);
          for (int q = 0; q < 5; ++q) div[q] += (fr[q] - fl[q]) / w;
        }
        double rho = Uin[0][a0];
        double v[3] = {Uin[1][a0] / rho, Uin[2][a0] / rho, Uin[3][a0] / rho};
        double F[3] = {Ur[1][a0], Ur[2][a0], Ur[3][a0]};
        double S[5];
        gas_explicit_source(p, rho, v, kF[a0], Ur[0][a0], F, S);
        double Un[5];
        for (int q = 0; q < 5; ++q) Un[q] = Uold[q][a0] - h * div[q] + h * S[q];
        if (isothermal(p)) Un[4] = Uold[4][a0];
        int interior = i >= 0 && i < G->n[0] && j >= 0 && j < G->n[1] && k >= 0 && k < G->n[2];
        apply_gas_floors(p, Un, interior, cnt);
        for (int q = 0; q < 5; ++q) Uout[q][a0] = Un[q];
        if (s_save && interior) {
          long ii = interior_index(p, i, j, k);
          s_save[0][ii] = S[1];
          s_save[1][ii] = S[2];
          s_save[2][ii] = S[3];
          s_save[3][ii] = S[4];
          w_save[0][ii] = rho;
          w_save[1][ii] = v[0];
          w_save[2][ii] = v[1];
          w_save[3][ii] = v[2];
        }
      }
}

/* ------------------------------------------------------------------------- */
/* implicit gas-radiation energy exchange (Sec. 3.4)                          */
/* ------------------------------------------------------------------------- */

static double quartic(double c4, double c1, double c0, double x) {
  return c4 * x * x * x * x + c1 * x + c0;
}

static double newton_step(double c4, double c1, double c0, double x) {
  double fx = quartic(c4, c1, c0, x);
  double dfx = 4.0 * c4 * x * x * x + c1;
  return x - fx / dfx;
}

/*
 * theta-scheme energy update of one cell over dt (Eqs. source:energyexchange to
 * source:polynomial). The unknown is the new internal energy x = e^{n+1}; the
 * combined energy Ebar = e + (c/chat) E_r is held fixed, so E_r^{n+1} =
 * (chat/c)(Ebar - x) (Eq. source:eradupdate). Returns x and writes E_r^{n+1}.
 *
 * Root finding: the quartic f(x) = c4 x^4 + c1 x + c0 is increasing and convex on
 * x > 0 and has its root in (0, u], u = min(-c0/c1, (-c0/c4)^{1/4}), when c0 <= 0.
 * Newton starts at u, so its iterates decrease monotonically onto the root; it stops
 * when |dx| <= eps x and takes one more step. If it leaves [0, u] or does not stop
 * within newton_maxit iterations, bisection on [0, u] to relative width eps (at
 * most 200 halvings) takes over, followed by one Newton step. If c0 > 0 (possible for theta < 1), the cell is
 * redone with theta = 1, which always gives c0 <= 0.
 */
double orc_exchange_cell(double rho, double e, double Er, double kP, double dt,
                         double chat, const orc_params *p, double *Er_new, int *iters,
                         int *used_theta1, int *used_bisect) {
  const double c = p->c_light;
  const int cv_t3 = (p->flags & ORC_GAS_CV_T3) != 0;
  double gm1_over = (p->gamma - 1.0) / (rho * p->r_gas);
  /* emission a_R T^4 as a function of e: alpha e^4 for the ideal gas, eps e when
     c_v = cv_alpha T^3 (e = cv_alpha T^4 / 4, eps = 4 a_R / cv_alpha) */
  double alpha = cv_t3 ? 0.0 : p->a_rad * gm1_over * gm1_over * gm1_over * gm1_over;
  double eps = cv_t3 ? 4.0 * p->a_rad / p->cv_alpha : 0.0;
  double eta = c * rho * kP * dt;
  double Ebar = e + (c / chat) * Er;
  double theta = p->theta_E;
  double c4, c1, c0;
  *iters = 0;
  *used_theta1 = 0;
  *used_bisect = 0;
  for (;;) {
    c4 = alpha * eta * theta;
    c1 = 1.0 + (chat / c) * eta * theta + eps * eta * theta;
    c0 = (1.0 - theta) * eta * (alpha * e * e * e * e + eps * e - Er) -
         (e + (chat / c) * eta * theta * Ebar);
    if (c0 > 0.0 && theta < 1.0) {
      theta = 1.0;
      *used_theta1 = 1;
      continue;
    }
    break;
  }
  double x;
  if (c0 >= 0.0) {
    x = 0.0;
  } else if (c4 == 0.0) {
    x = -c0 / c1;
  } else {
    double u1 = -c0 / c1;
    double u2 = pow(-c0 / c4, 0.25);
    double u = u1 < u2 ? u1 : u2;
    const double eps = p->newton_rtol;
    x = u;
    int converged = 0;
    for (int it = 0; it < p->newton_maxit; ++it) {
      double xn = newton_step(c4, c1, c0, x);
      (*iters)++;
      double dx = x - xn;
      x = xn;
      if (!(x >= 0.0 && x <= u)) break;
      if (fabs(dx) <= eps * x) {
        converged = 1;
        break;
      }
    }
    if (converged) {
      x = newton_step(c4, c1, c0, x);
    } else {
      *used_bisect = 1;
      double lo = 0.0, hi = u;
      for (int b = 0; b < 200 && hi - lo > eps * hi; ++b) {
        double mid = 0.5 * (lo + hi);
        if (quartic(c4, c1, c0, mid) < 0.0)
          lo = mid;
        else
          hi = mid;
      }
      x = newton_step(c4, c1, c0, 0.5 * (lo + hi));
    }
  }
  *Er_new = (chat / c) * (Ebar - x);
  return x;
}

/* ------------------------------------------------------------------------- */
/* opacity law (Sec. 4.1.1): kappa = k0 (T_gas/T0)^a (rho/rho0)^b             */
/* ------------------------------------------------------------------------- */

/* Gas temperature of cell a: P/(rho r_gas) for the ideal gas, c_s^2/r_gas when
   isothermal, and from a_R T^4 = (4 a_R/alpha) e when c_v = alpha T^3. */
static double gas_temperature(const orc_params *p, const orc_fields *s, long a) {
  double rho = s->rho[a];
  if (isothermal(p)) return p->iso_cs * p->iso_cs / p->r_gas;
  double e = s->E[a] - 0.5 * (s->mx[a] * s->mx[a] + s->my[a] * s->my[a] + s->mz[a] * s->mz[a]) / rho;
  if (p->flags & ORC_GAS_CV_T3) return pow(4.0 * e / p->cv_alpha, 0.25);
  return (p->gamma - 1.0) * e / (rho * p->r_gas);
}

/* The law's opacity of every cell into kap (N values). */
static void opacity_law(const orc_params *p, const orc_fields *s, double *kap) {
  const long N = (long)p->nx * p->ny * p->nz;
  const double *L = p->kappa_law;
  for (long a = 0; a < N; ++a) {
    double T = gas_temperature(p, s, a);
    kap[a] = L[0] * pow(T / L[1], L[3]) * pow(s->rho[a] / L[2], L[4]);
  }
}

/* ------------------------------------------------------------------------- */
/* time step (Sec. 3.1, Eqs. algorithm:ceff to algorithm:radtimestep)         */
/* ------------------------------------------------------------------------- */

int orc_suggest_dt(const orc_params *p, const orc_fields *s, double chat, double *dt_gas,
                   int *nsub, double *vmax_out) {
  const double dxm = min_width(p);
  double vmax = 0.0;
  long N = (long)p->nx * p->ny * p->nz;
  orc_fields local;
  double *law = NULL;
  if (p->flags & ORC_OPACITY_LAW) {
    law = (double *)malloc((size_t)N * sizeof(double));
    opacity_law(p, s, law);
    local = *s;
    local.kP = local.kF = law;
    s = &local;
  }
  for (long a = 0; a < N; ++a) {
    double rho = s->rho[a];
    double v[3] = {s->mx[a] / rho, s->my[a] / rho, s->mz[a] / rho};
    double vn = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    double gP;
    if (isothermal(p)) {
      gP = rho * p->iso_cs * p->iso_cs;
    } else {
      double ke = 0.5 * rho * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
      gP = p->gamma * (p->gamma - 1.0) * (s->E[a] - ke);
    }
    double ceff = sqrt((gP + (4.0 / 9.0) * s->Er[a] * (1.0 - exp(-rho * s->kF[a] * dxm))) / rho);
    if (vn + ceff > vmax) vmax = vn + ceff;
  }
  free(law);
  *vmax_out = vmax;
  if (!(vmax > 0.0)) return -1;
  *dt_gas = p->cfl * dxm / vmax;
  *nsub = (int)ceil(chat / vmax);
  if (*nsub < 1) *nsub = 1;
  return 0;
}

/* ------------------------------------------------------------------------- */
/* conservation ledger (Sec. 2.1)                                             */
/* ------------------------------------------------------------------------- */

/* Sums of E + (c/chat) E_r, m + F/(c chat) (three components) and rho, times dV. */
void orc_ledger(const orc_params *p, const orc_fields *s, double chat, double out[5]) {
  const double c = p->c_light;
  const double dV = p->dx * p->dy * p->dz;
  long N = (long)p->nx * p->ny * p->nz;
  double acc[5] = {0, 0, 0, 0, 0};
  for (long a = 0; a < N; ++a) {
    acc[0] += s->E[a] + (c / chat) * s->Er[a];
    acc[1] += s->mx[a] + s->Fx[a] / (c * chat);
    acc[2] += s->my[a] + s->Fy[a] / (c * chat);
    acc[3] += s->mz[a] + s->Fz[a] / (c * chat);
    acc[4] += s->rho[a];
  }
  for (int q = 0; q < 5; ++q) out[q] = acc[q] * dV;
}

/* ------------------------------------------------------------------------- */
/* one operator-split step (Sec. 3.1, algorithm steps 2-6)                    */
/* ------------------------------------------------------------------------- */

static void free_fields(double **f, int n) {
  for (int q = 0; q < n; ++q) free(f[q]);
}

/*
 * Advance the state by one gas step dt_gas with nsub radiation subcycles of
 * dt_gas/nsub each. nsub = 0 advances only the exchange and the gas.
 * Returns 0, -1 for invalid arguments, -2 when chat dt_gas/nsub exceeds K0 dx.
 */
int orc_step(const orc_params *p, orc_fields *s, double dt_gas, double chat, int nsub,
             orc_counts *cnt) {
  if (!(dt_gas > 0.0) || !(chat > 0.0) || nsub < 0) return -1;
  if (nsub > 0 && chat * dt_gas / nsub > p->cfl * min_width(p) * (1.0 + 1e-12)) return -2;
  const long N = (long)p->nx * p->ny * p->nz;
  const unsigned mode = p->flags & ORC_EXCH_MASK;
  const int rad_only = (p->flags & ORC_RAD_ONLY) != 0;

  /* opacity law: evaluated once from the state at the start of the step */
  orc_fields local = *s;
  double *law = NULL;
  if (p->flags & ORC_OPACITY_LAW) {
    law = (double *)malloc((size_t)N * sizeof(double));
    opacity_law(p, s, law);
    local.kP = local.kF = law;
  }
  s = &local;

  /* step 2: implicit energy exchange S_i over dt_gas */
  if (mode == ORC_EXCH_FULL && !isothermal(p)) {
    for (long a = 0; a < N; ++a) {
      double rho = s->rho[a];
      double ke = 0.5 * (s->mx[a] * s->mx[a] + s->my[a] * s->my[a] + s->mz[a] * s->mz[a]) / rho;
      double e = s->E[a] - ke;
      double Er_new;
      int it, th1, bis;
      double x = orc_exchange_cell(rho, e, s->Er[a], s->kP[a], dt_gas, chat, p, &Er_new, &it,
                                   &th1, &bis);
      s->E[a] += x - e;
      /* E_r from Eq. source:eradupdate is a difference of nearly equal energies when
         the condition number K of Eq. source:kappacond is large, and can round to
         zero or below; it is raised to the floor as after a radiation stage */
      s->Er[a] = Er_new < p->er_floor ? p->er_floor : Er_new;
      if (cnt) {
        cnt->newton_iters += it;
        if (it > cnt->newton_max) cnt->newton_max = it;
        cnt->exch_theta1 += th1;
        cnt->exch_bisect += bis;
      }
    }
  }

  pgrid G = make_grid(p, 3);
  double *s_n[4] = {0}, *w_h[4] = {0};
  int comp_gas[5] = {-1, 0, 1, 2, -1};
  int comp_rad[4] = {-1, 0, 1, 2};
  int comp_scalar[1] = {-1};

  /* step 3: gas transport with S_e,gas at first order, radiation held at t^n */
  if (!rad_only) {
    double *Ug[5], *Uh[5], *Un[5], *Ur[4], *kFp;
    for (int q = 0; q < 5; ++q) {
      Ug[q] = alloc_field(&G);
      Uh[q] = alloc_field(&G);
      Un[q] = alloc_field(&G);
    }
    for (int q = 0; q < 4; ++q) Ur[q] = alloc_field(&G);
    kFp = alloc_field(&G);
    double *gsrc[5] = {s->rho, s->mx, s->my, s->mz, s->E};
    double *rsrc[4] = {s->Er, s->Fx, s->Fy, s->Fz};
    for (int q = 0; q < 5; ++q) load_padded(p, &G, gsrc[q], Ug[q]);
    for (int q = 0; q < 4; ++q) load_padded(p, &G, rsrc[q], Ur[q]);
    load_padded(p, &G, s->kF, kFp);
    fill_ghosts(p, &G, Ug, comp_gas, 5);
    fill_ghosts(p, &G, Ur, comp_rad, 4);
    apply_fixed(p, &G, Ur);
    fill_ghosts(p, &G, &kFp, comp_scalar, 1);
    for (int q = 0; q < 4; ++q) {
      s_n[q] = (double *)calloc((size_t)N, sizeof(double));
      w_h[q] = (double *)calloc((size_t)N, sizeof(double));
    }
    gas_stage(p, &G, 0.5 * dt_gas, 0, 2, Ug, Ug, Ur, kFp, Uh, NULL, NULL, cnt);
    gas_stage(p, &G, dt_gas, 1, 0, Uh, Ug, Ur, kFp, Un, s_n, w_h, cnt);
    for (int q = 0; q < 5; ++q) store_interior(p, &G, Un[q], gsrc[q]);
    free_fields(Ug, 5);
    free_fields(Uh, 5);
    free_fields(Un, 5);
    free_fields(Ur, 4);
    free(kFp);
  }

  /* steps 4-5: nsub radiation subcycles with the gas frozen */
  if (nsub > 0) {
    frozen_gas fg;
    fg.rkF = alloc_field(&G);
    fg.rkP = alloc_field(&G);
    for (int q = 0; q < 3; ++q) fg.v[q] = alloc_field(&G);
    fg.j = s->j ? alloc_field(&G) : NULL;
    for (int k = 0; k < p->nz; ++k)
      for (int j = 0; j < p->ny; ++j)
        for (int i = 0; i < p->nx; ++i) {
          long ii = interior_index(p, i, j, k), a = at(&G, i, j, k);
          double rho = s->rho[ii];
          fg.rkF[a] = rho * s->kF[ii];
          fg.rkP[a] = rho * s->kP[ii];
          fg.v[0][a] = s->mx[ii] / rho;
          fg.v[1][a] = s->my[ii] / rho;
          fg.v[2][a] = s->mz[ii] / rho;
          if (fg.j) fg.j[a] = s->j[ii];
        }
    double *gf[6] = {fg.rkF, fg.rkP, fg.v[0], fg.v[1], fg.v[2], fg.j};
    int gcomp[6] = {-1, -1, 0, 1, 2, -1};
    fill_ghosts(p, &G, gf, gcomp, fg.j ? 6 : 5);

    double *Um[4], *Uh[4], *Un[4];
    for (int q = 0; q < 4; ++q) {
      Um[q] = alloc_field(&G);
      Uh[q] = alloc_field(&G);
      Un[q] = alloc_field(&G);
    }
    double *rsrc[4] = {s->Er, s->Fx, s->Fy, s->Fz};
    const double hr = dt_gas / nsub;
    for (int m = 0; m < nsub; ++m) {
      for (int q = 0; q < 4; ++q) load_padded(p, &G, rsrc[q], Um[q]);
      fill_ghosts(p, &G, Um, comp_rad, 4);
      apply_fixed(p, &G, Um);
      rad_stage(p, &G, chat, 0.5 * hr, 0, 2, Um, Um, Um, &fg, Uh, NULL);
      apply_fixed(p, &G, Uh);
      rad_stage(p, &G, chat, hr, 1, 0, Uh, Um, Uh, &fg, Un, cnt);
      for (int q = 0; q < 4; ++q) store_interior(p, &G, Un[q], rsrc[q]);
    }
    free_fields(Um, 4);
    free_fields(Uh, 4);
    free_fields(Un, 4);
    free(fg.rkF);
    free(fg.rkP);
    free_fields(fg.v, 3);
    free(fg.j);
  }

  /* step 6: second-order correction of S_e,gas with the radiation at t^{n+1} */
  if (!rad_only) {
    for (long a = 0; a < N; ++a) {
      double rho = w_h[0][a];
      double v[3] = {w_h[1][a], w_h[2][a], w_h[3][a]};
      double F[3] = {s->Fx[a], s->Fy[a], s->Fz[a]};
      double S[5];
      gas_explicit_source(p, rho, v, s->kF[a], s->Er[a], F, S);
      double U[5] = {s->rho[a], s->mx[a], s->my[a], s->mz[a], s->E[a]};
      U[1] += 0.5 * dt_gas * (S[1] - s_n[0][a]);
      U[2] += 0.5 * dt_gas * (S[2] - s_n[1][a]);
      U[3] += 0.5 * dt_gas * (S[3] - s_n[2][a]);
      if (!isothermal(p)) U[4] += 0.5 * dt_gas * (S[4] - s_n[3][a]);
      apply_gas_floors(p, U, 1, cnt);
      s->rho[a] = U[0];
      s->mx[a] = U[1];
      s->my[a] = U[2];
      s->mz[a] = U[3];
      s->E[a] = U[4];
    }
    free_fields(s_n, 4);
    free_fields(w_h, 4);
  }
  free(law);
  return 0;
}
