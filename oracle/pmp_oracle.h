/*
 * Serial CPU oracle for the particle-mesh-particle (PMP) interaction step.
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the HIP library; it is
 * called from the test suite, from the smoke check and from the benchmark's
 * CPU-baseline leg, and from nowhere else.  It shares no code, header, table
 * or constant with the HIP library.
 *
 * It computes, in plain double precision (or in exact int64 fixed point with
 * 40 fractional bits, or with the error bound and mantissa truncation of the
 * paper's App. A.1), one pass of the method of He et al. (2025), Sec. 2.2:
 *   Step 1  particle -> ghost-zoned buffer (CIC mass, uniform-sphere
 *           supernova injection, Gaussian-kernel sink removal),
 *   Step 2  ghost -> owner summation (here: periodic images / neighbouring
 *           boxes of one address space),
 *   Step 3  cell-wise limiter (sink removal limiter of Sec. 3.1.1 and the
 *           momentum/energy limiter of Sec. 3.2.1, eq. "lambda"),
 *   Step 4  sink update with the limited changes,
 *   Step 5  mesh update,
 * and, after the step, sink creation (Sec. 3.1.2).
 * Every loop runs in the order of the definitions; no blocking, fusion or
 * reordering.  Floating-point expressions are written in one fixed order and
 * the file is compiled without contraction (-ffp-contract=off).
 *
 * Units: positions are in cell units of the global index space (a particle
 * at x lies in cell floor(x)); dx is the cell edge, V = dx*dx*dx.
 *
 * Layout (the library interface, mirrored here independently):
 *   state  = concatenation over boxes of double [5][nz][ny][nx]
 *            (rho, px, py, pz, E), x fastest;
 *   buffer = concatenation over boxes of [F][nz+2g][ny+2g][nx+2g] with
 *            F = 5 (+1 removal channel K when sinks are present);
 *            double (ORC_F64) or int64 with scale 2^40 (ORC_FIX64).
 *
 * Parity pins: see the tests.  Every function below is pinned by at least
 * one check against closed forms, the paper's worked example (Fig. 1),
 * lattice counts, invariants or brute force.
 */
#ifndef PMP_ORACLE_H
#define PMP_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ORC_F64R: double sums with the error bound and truncation of App. A.1
 * (orc_deposit_r); fold, sink update and apply treat its buffer as ORC_F64. */
enum { ORC_F64 = 0, ORC_FIX64 = 1, ORC_F64R = 2 };

enum {
  ORC_OK = 0,
  ORC_EINVAL = -1,     /* bad argument */
  ORC_EOUTSIDE = -2,   /* particle host cell not in its box */
  ORC_EREACH = -3,     /* stencil member outside the ghost-zoned buffer */
  ORC_EOVERFLOW = -4,  /* fixed-point value out of range */
  ORC_ENOMEM = -5,
  ORC_EOVERLAP = -6    /* boxes overlap */
};

typedef struct {
  int32_t nbox;
  const int32_t *lo;   /* [nbox][3] x,y,z: first owned global cell */
  const int32_t *n;    /* [nbox][3] owned cells per axis */
  int32_t ghost;       /* ghost width g */
  int32_t domain[3];   /* periodic domain, cells per axis */
  double dx;           /* cell edge */
  int32_t nfield;      /* 5, or 6 with the sink removal channel */
} orc_mesh;

typedef struct { const double *x, *y, *z, *m; const int64_t *box_off; } orc_cic;
typedef struct { const double *x, *y, *z, *m, *e, *r; const int64_t *box_off; } orc_sn;
/* Sink request rate: a fixed fraction a of the kernel gas mass with a fixed
 * Gaussian width, or the Bondi-Hoyle-Lyttleton rate of Sec. 3.1.1 (eqs.
 * "rbh", "mdot") with the width r_acc clamped to [dx/4, r_K/2]. */
enum { ORC_RATE_FRACTION = 0, ORC_RATE_BONDI = 1 };

typedef struct {
  const double *x, *y, *z, *a;   /* a: requested fraction of the kernel mass */
  const int64_t *box_off;
  double r_k;                    /* kernel radius (cells) */
  double r_gauss;                /* Gaussian width r_acc (cells), fraction rate */
  /* Bondi-Hoyle rate only */
  const double *m, *vx, *vy, *vz;   /* sink mass and velocity */
  int32_t rate;                     /* ORC_RATE_* */
  double G, dt, gamma, lambda;      /* gravity constant, time step, adiabatic
                                       index of the gas, the BHL lambda */
} orc_sinks;
/* Supernova remnants, the variant of the TIGRESS prescription of Sec. 3.2.1
 * (orc_deposit_snr).  Code units throughout: nh_per_rho converts a mass
 * density to the number density of H nuclei n_H in cm^-3 (1/(mu_H m_H)),
 * msf_coef and psnr_coef are the shell-formation mass and the terminal
 * momentum at n_H = 1 cm^-3 (1679 Msun and 2.8e5 Msun km/s in the paper). */
typedef struct {
  const double *x, *y, *z;       /* position (cells) */
  const double *m, *e;           /* ejecta mass M_ej, supernova energy E_sn */
  const double *vx, *vy, *vz;    /* velocity of the exploding particle */
  const int64_t *box_off;
  double r_k;                    /* kernel radius (cells) */
  int32_t sub;                   /* sample points per axis of the covered
                                    fraction: 1, 2, 4, 8 or 16 */
  double nh_per_rho, msf_coef, psnr_coef;
  double eps_k;                  /* kinetic fraction in the Sedov-Taylor phase */
} orc_snr;

/* Limiter parameters.  rho_tr is the Truelove density as a constant; with
 * truelove_J > 0 each cell has its own, J^2 pi c_s^2 / (G dx^2) (Sec. 3.1.1,
 * eq. "truelove"), c_s from the cell's state as in the Bondi-Hoyle rate. */
typedef struct {
  double rho_floor, rho_tr, cap;
  int32_t eint_mode;
  double truelove_J, G, gamma;
} orc_limits;
typedef struct {
  int64_t touched;   /* cells with K > 0 */
  int64_t bind;      /* cells where the removal limiter binds (Kl < K) */
  int64_t lam;       /* cells with lambda < 1 */
  int64_t fall;      /* cells where lambda = 0 is still infeasible */
} orc_counters;

int64_t orc_buffer_elems(const orc_mesh *M);
int64_t orc_state_elems(const orc_mesh *M);
double  orc_exp(double x);
double  orc_log(double x);
double  orc_pow(double x, double a);   /* orc_exp(a orc_log(x)), x > 0 */

/* sink_w, sink_mreq, sink_racc [n sinks]: the kernel weight sum, the
 * requested mass and the Gaussian width r_acc (cells) of each sink. */
int orc_deposit(const orc_mesh *M, int mode, const orc_cic *cic, const orc_sn *sn,
                const orc_sinks *sk, const orc_limits *L, const double *state, void *buf,
                double *sink_w, double *sink_mreq, double *sink_racc);
int orc_deposit_r(const orc_mesh *M, const orc_cic *cic, const orc_sn *sn,
                  const orc_sinks *sk, const orc_limits *L, const double *state, double *buf,
                  double *err, int margin, double *sink_w, double *sink_mreq,
                  double *sink_racc);
double orc_truncate_err(double v, double err, int margin);
/* Supernova remnants (TIGRESS variant), added to a deposited buffer;
 * info [4][n] (may be NULL): V_snr, M_snr, n_H, |p_rad| per supernova. */
int orc_deposit_snr(const orc_mesh *M, int mode, const orc_snr *S, const double *state,
                    void *buf, double *info);
int orc_fold(const orc_mesh *M, int mode, void *buf);
int orc_sink_update(const orc_mesh *M, int mode, const double *state, const void *buf,
                    const orc_sinks *sk, const orc_limits *L, const double *sink_w,
                    const double *sink_mreq, const double *sink_racc, double *dm, double *dpx,
                    double *dpy, double *dpz);
int orc_apply(const orc_mesh *M, int mode, double *state, const void *buf,
              const orc_limits *L, double *eta, orc_counters *cnt);
/* Sink creation of Sec. 3.1.2 on any box layout (state updated in place;
 * out [7][max_new]: x, y, z, m, px, py, pz in global cell index order).
 * existing: the sinks already present (positions and box_off only; may be
 * NULL); L: the Truelove density (constant or per cell). */
int orc_sink_create(const orc_mesh *M, int mode, double *state, const void *buf,
                    const orc_sinks *existing, double r_k, const orc_limits *L,
                    int64_t max_new, double *out, int64_t *count);

#ifdef __cplusplus
}
#endif
#endif
