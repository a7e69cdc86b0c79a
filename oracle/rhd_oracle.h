/*
 * rhd_oracle.h -- interface of the plain FP64 CPU oracle for the gray two-moment
 * (M1) radiation-hydrodynamics step of Skinner & Ostriker, "A two-moment radiation
 * hydrodynamics module in Athena using a time-explicit Godunov method" (2013).
 *
 * TEST INFRASTRUCTURE ONLY. The test suite, the smoke check and the CPU-baseline
 * leg of the benchmark are the only code that may load this library. The GPU
 * library neither includes this header nor links this code, and this code does
 * not include or link anything of the GPU library.
 *
 * The parameter block and flag values describe the same physical problem as the
 * GPU library's C interface, field by field, so that a test can describe one
 * problem once and hand it to both; the two definitions are written separately.
 */
#ifndef RHD_ORACLE_H
#define RHD_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* boundary kinds, per face x-, x+, y-, y+, z-, z+ */
enum { ORC_BC_PERIODIC = 0, ORC_BC_OUTFLOW = 1, ORC_BC_REFLECT = 2, ORC_BC_FIXED = 3 };
/* ORC_BC_FIXED: every ghost cell beyond the face holds the radiation state
   bval[face] = (E_r, F_x, F_y, F_z), in U^m and in the predicted U^{m+1/2} alike (a
   cell beyond several fixed faces takes the last of them in the order x, y, z); gas
   and frozen-gas fields continue zero-gradient there. */

/* flag bits */
#define ORC_ISOTHERMAL        (1u << 0)
#define ORC_EXCH_MASK         (3u << 1)
#define ORC_EXCH_FULL         (0u << 1)   /* implicit exchange on the gas step        */
#define ORC_EXCH_ABSORB_ONLY  (1u << 1)   /* absorption only, on each radiation stage */
#define ORC_EXCH_NONE         (2u << 1)   /* radiative equilibrium: no exchange       */
#define ORC_BETA_TAU          (1u << 3)   /* keep the O(beta tau) velocity terms      */
#define ORC_RAD_ONLY          (1u << 4)   /* gas frozen: no gas transport             */
#define ORC_PRECISION_MIXED   (1u << 5)   /* ignored by the oracle (always FP64)      */
#define ORC_GAS_CV_T3         (1u << 6)   /* heat capacity c_v = cv_alpha T^3, so that
                                             a_R T^4 = (4 a_R / cv_alpha) e            */
#define ORC_CLOSURE_P1        (1u << 8)   /* Eddington closure T = I/3, speeds -+chat/sqrt 3 */
#define ORC_OPACITY_LAW       (1u << 7)   /* kappa_P = kappa_F = k0 (T/T0)^a (rho/rho0)^b
                                             from the gas state at the start of each
                                             step; kappa_law = {k0, T0, rho0, a, b}     */

typedef struct {
  int nx, ny, nz;                 /* interior cells; ny = nz = 1 for 1D           */
  double dx, dy, dz;              /* cell widths                                  */
  double gamma;                   /* ratio of specific heats                      */
  double c_light, a_rad, r_gas;   /* c, a_R and k_B/mu (P = rho r_gas T)          */
  double iso_cs;                  /* isothermal sound speed                       */
  double cfl;                     /* Courant number K0                            */
  double theta_E, theta_F;        /* theta for the exchange and for the flux      */
  double newton_rtol;             /* relative tolerance epsilon of the root solve */
  int newton_maxit;               /* Newton iterations before bisection (def. 50) */
  double rho_floor, p_floor, er_floor;
  int bc[6];
  unsigned flags;
  double cv_alpha;                /* alpha of c_v = alpha T^3 (ORC_GAS_CV_T3)     */
  double bval[6][4];              /* radiation state of each ORC_BC_FIXED face    */
  double kappa_law[5];            /* k0, T0, rho0, a, b of ORC_OPACITY_LAW        */
} orc_params;

typedef struct {
  double *rho, *mx, *my, *mz, *E; /* gas density, momentum, total energy          */
  double *Er, *Fx, *Fy, *Fz;      /* radiation energy density and flux            */
  const double *kP, *kF;          /* Planck-mean and flux-mean specific opacity   */
  const double *j;                /* emissivity per cell, or NULL                 */
} orc_fields;

typedef struct {
  long exch_theta1;     /* cells whose exchange was redone with theta = 1   */
  long exch_bisect;     /* cells whose root needed bisection                */
  long newton_iters;    /* total Newton iterations                          */
  long newton_max;      /* largest iteration count in one cell              */
  long rad_fclamp;      /* |F| > c E rescaled                               */
  long rad_efloor;      /* E_r raised to the floor                          */
  long gas_rhofloor;    /* rho raised to the floor                          */
  long gas_pfloor;      /* P raised to the floor                            */
} orc_counts;

/* single-state pieces, exported so the tests can pin them one by one */
void   orc_m1_eddington_factor(double f, double *chi);
void   orc_m1_pressure(double E, const double F[3], double c, double P[9]);
void   orc_m1_eigen(double E, const double F[3], double c, double chat, int d,
                    double *l1, double *l3);
void   orc_rad_hll_flux(const double UL[4], const double UR[4], int d, double c,
                        double chat, double flux[4]);
void   orc_p1_hll_flux(const double UL[4], const double UR[4], int d, double c,
                       double chat, double flux[4]);
void   orc_gas_flux(const double W[5], int d, const orc_params *p, double flux[5]);
void   orc_gas_riemann(const double WL[5], const double WR[5], int d,
                       const orc_params *p, double flux[5]);
double orc_exchange_cell(double rho, double e, double Er, double kP, double dt,
                         double chat, const orc_params *p, double *Er_new,
                         int *iters, int *used_theta1, int *used_bisect);
double orc_mc_slope(double dm, double dp);

/* whole-grid operations */
int  orc_step(const orc_params *p, orc_fields *s, double dt_gas, double chat,
              int nsub, orc_counts *cnt);
int  orc_suggest_dt(const orc_params *p, const orc_fields *s, double chat,
                    double *dt_gas, int *nsub, double *vmax);
void orc_ledger(const orc_params *p, const orc_fields *s, double chat,
                double out[5]);

#ifdef __cplusplus
}
#endif
#endif
