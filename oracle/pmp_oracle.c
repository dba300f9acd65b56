/*
 * Serial CPU oracle for the particle-mesh-particle step.  TEST INFRASTRUCTURE
 * ONLY: see pmp_oracle.h for scope, layout and units.
 *
 * Compiled with: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -shared -fPIC
 */
#include "pmp_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define FIX_SCALE 1099511627776.0        /* 2^40: fixed-point scale */
#define FIX_INV (1.0 / 1099511627776.0)  /* 2^-40 */
#define FIX_LIMIT 4611686018427387904.0  /* 2^62: largest magnitude accepted */

/* ------------------------------------------------------------------ helpers */

/* Quantise v to the 2^-40 grid, round half to even (llrint in the default
 * rounding mode).  Fails when the scaled value leaves (-2^62, 2^62). */
static int q40(double v, int64_t *out) {
  double s = v * FIX_SCALE;
  if (!(fabs(s) < FIX_LIMIT)) return ORC_EOVERFLOW;
  *out = llrint(s);
  return ORC_OK;
}

/* int64 add without signed-overflow undefined behaviour. */
static int64_t iadd(int64_t a, int64_t b) { return (int64_t)((uint64_t)a + (uint64_t)b); }

static int64_t imod(int64_t a, int64_t n) {
  int64_t r = a % n;
  return r < 0 ? r + n : r;
}

/* exp(x) for the sink kernel weights of Sec. 3.1.1, eq. "kernel".
 * Method: Cody & Waite (1980) argument reduction x = k ln2 + r with ln2 split
 * into a high part on the 2^-32 grid (29 significant bits, so k*hi is exact
 * for |k| < 2^24)
 * and a low part, then the Taylor series of exp(r) through degree 13 in Horner
 * form on |r| <= ln2/2, then scaling by 2^k.  Written from the method, not
 * from any library.  Accurate to a few ulp (checked against libm). */
double orc_exp(double x) {
  if (x != x) return x;
  if (x > 709.0) return HUGE_VAL;
  if (x < -745.0) return 0.0;
  /* ln2_hi = ln 2 rounded to a multiple of 2^-32; ln2_lo = ln 2 - ln2_hi
   * rounded to double; inv_ln2 = 1/ln 2 rounded to double */
  const double ln2_hi = 0x1.62e42ffp-1;
  const double ln2_lo = -0x1.718432a1b0e26p-35;
  const double inv_ln2 = 0x1.71547652b82fep+0;
  double k = nearbyint(x * inv_ln2);
  double r = (x - k * ln2_hi) - k * ln2_lo;
  /* coefficients 1/n!, n = 13 .. 0, each one correctly rounded division */
  double p = 1.0 / 6227020800.0;
  p = p * r + 1.0 / 479001600.0;
  p = p * r + 1.0 / 39916800.0;
  p = p * r + 1.0 / 3628800.0;
  p = p * r + 1.0 / 362880.0;
  p = p * r + 1.0 / 40320.0;
  p = p * r + 1.0 / 5040.0;
  p = p * r + 1.0 / 720.0;
  p = p * r + 1.0 / 120.0;
  p = p * r + 1.0 / 24.0;
  p = p * r + 1.0 / 6.0;
  p = p * r + 0.5;
  p = p * r + 1.0;
  p = p * r + 1.0;
  return ldexp(p, (int)k);
}

typedef struct {
  int64_t *soff;   /* state offset of box b (elements) */
  int64_t *boff;   /* buffer offset of box b (elements) */
  int32_t *owner;  /* owner box of each domain cell, or -1; NULL until built */
} geom;

static int64_t box_cells(const orc_mesh *M, int b) {
  return (int64_t)M->n[3 * b] * M->n[3 * b + 1] * M->n[3 * b + 2];
}
static int64_t box_pad_cells(const orc_mesh *M, int b) {
  int64_t g2 = 2 * (int64_t)M->ghost;
  return (M->n[3 * b] + g2) * (M->n[3 * b + 1] + g2) * (M->n[3 * b + 2] + g2);
}

int64_t orc_buffer_elems(const orc_mesh *M) {
  int64_t s = 0;
  for (int b = 0; b < M->nbox; ++b) s += (int64_t)M->nfield * box_pad_cells(M, b);
  return s;
}
int64_t orc_state_elems(const orc_mesh *M) {
  int64_t s = 0;
  for (int b = 0; b < M->nbox; ++b) s += 5 * box_cells(M, b);
  return s;
}

static int check_mesh(const orc_mesh *M) {
  if (!M || M->nbox < 1 || !M->lo || !M->n || M->ghost < 0) return ORC_EINVAL;
  if (M->nfield != 5 && M->nfield != 6) return ORC_EINVAL;
  if (!(M->dx > 0)) return ORC_EINVAL;
  for (int a = 0; a < 3; ++a)
    if (M->domain[a] < 1) return ORC_EINVAL;
  for (int b = 0; b < M->nbox; ++b)
    for (int a = 0; a < 3; ++a) {
      if (M->n[3 * b + a] < 1 || M->lo[3 * b + a] < 0) return ORC_EINVAL;
      if (M->lo[3 * b + a] + M->n[3 * b + a] > M->domain[a]) return ORC_EINVAL;
    }
  return ORC_OK;
}

static void geom_free(geom *G) {
  free(G->soff);
  free(G->boff);
  free(G->owner);
}

/* Offsets of every box, and (if want_owner) the map from a domain cell to the
 * box that owns it, painted box by box so that overlaps are detected. */
static int geom_build(const orc_mesh *M, geom *G, int want_owner) {
  memset(G, 0, sizeof *G);
  G->soff = (int64_t *)malloc(sizeof(int64_t) * (size_t)M->nbox);
  G->boff = (int64_t *)malloc(sizeof(int64_t) * (size_t)M->nbox);
  if (!G->soff || !G->boff) { geom_free(G); return ORC_ENOMEM; }
  int64_t s = 0, q = 0;
  for (int b = 0; b < M->nbox; ++b) {
    G->soff[b] = s;
    G->boff[b] = q;
    s += 5 * box_cells(M, b);
    q += (int64_t)M->nfield * box_pad_cells(M, b);
  }
  if (!want_owner) return ORC_OK;
  int64_t nd = (int64_t)M->domain[0] * M->domain[1] * M->domain[2];
  G->owner = (int32_t *)malloc(sizeof(int32_t) * (size_t)nd);
  if (!G->owner) { geom_free(G); return ORC_ENOMEM; }
  for (int64_t c = 0; c < nd; ++c) G->owner[c] = -1;
  for (int b = 0; b < M->nbox; ++b) {
    const int32_t *lo = M->lo + 3 * b, *n = M->n + 3 * b;
    for (int64_t k = lo[2]; k < lo[2] + n[2]; ++k)
      for (int64_t j = lo[1]; j < lo[1] + n[1]; ++j)
        for (int64_t i = lo[0]; i < lo[0] + n[0]; ++i) {
          int64_t c = (k * M->domain[1] + j) * M->domain[0] + i;
          if (G->owner[c] != -1) { geom_free(G); return ORC_EOVERLAP; }
          G->owner[c] = b;
        }
  }
  return ORC_OK;
}

/* Buffer element of box b, field f, at global cell (i,j,k) taken without
 * wrapping (it may lie in the ghost zone).  -1 if outside the padded box. */
static int64_t buf_index(const orc_mesh *M, const geom *G, int b, int f, int64_t i,
                         int64_t j, int64_t k) {
  const int32_t *lo = M->lo + 3 * b, *n = M->n + 3 * b;
  int64_t g = M->ghost;
  int64_t px = n[0] + 2 * g, py = n[1] + 2 * g, pz = n[2] + 2 * g;
  int64_t li = i - lo[0] + g, lj = j - lo[1] + g, lk = k - lo[2] + g;
  if (li < 0 || lj < 0 || lk < 0 || li >= px || lj >= py || lk >= pz) return -1;
  return G->boff[b] + (int64_t)f * px * py * pz + (lk * py + lj) * px + li;
}

/* Owned buffer element (field f) and state cell of the periodic image of a
 * global cell; returns the owning box or -1. */
static int owner_of(const orc_mesh *M, const geom *G, int64_t i, int64_t j, int64_t k,
                    int64_t *iw, int64_t *jw, int64_t *kw) {
  *iw = imod(i, M->domain[0]);
  *jw = imod(j, M->domain[1]);
  *kw = imod(k, M->domain[2]);
  return G->owner[(*kw * M->domain[1] + *jw) * M->domain[0] + *iw];
}

static int64_t state_index(const orc_mesh *M, const geom *G, int b, int f, int64_t iw,
                           int64_t jw, int64_t kw) {
  const int32_t *lo = M->lo + 3 * b, *n = M->n + 3 * b;
  int64_t li = iw - lo[0], lj = jw - lo[1], lk = kw - lo[2];
  return G->soff[b] + (int64_t)f * box_cells(M, b) + (lk * n[1] + lj) * n[0] + li;
}

/* Host cell floor(x) must lie in box b (particles follow the mesh
 * decomposition, Sec. 2.1). */
static int host_in_box(const orc_mesh *M, int b, const int64_t h[3]) {
  for (int a = 0; a < 3; ++a)
    if (h[a] < M->lo[3 * b + a] || h[a] >= (int64_t)M->lo[3 * b + a] + M->n[3 * b + a])
      return 0;
  return 1;
}

/* Distance test of Sec. 2.1: a cell takes part when its centre lies within
 * the kernel radius (inclusive).  Fixed evaluation order. */
static double dist2(double x, double y, double z, int64_t i, int64_t j, int64_t k) {
  double ddx = ((double)i + 0.5) - x;
  double ddy = ((double)j + 0.5) - y;
  double ddz = ((double)k + 0.5) - z;
  return (ddx * ddx + ddy * ddy) + ddz * ddz;
}

/* Candidate index range along one axis for a sphere of radius r around p:
 * every cell whose centre can satisfy |i + 1/2 - p| <= r. */
static void sphere_range(double p, double r, int64_t *lo, int64_t *hi) {
  *lo = (int64_t)floor(p - r - 0.5) - 1;
  *hi = (int64_t)floor(p + r - 0.5) + 1;
}

/* Double-precision accumulation.  With err (mode ORC_F64R, App. A.1 item 2)
 * the cell's error bound also grows by eps |sum after the addition|. */
#define ORC_EPS 0x1p-52 /* double machine epsilon */
static void add_f64(void *buf, double *err, int64_t idx, double v) {
  double *B = (double *)buf;
  B[idx] += v;
  if (err) err[idx] += ORC_EPS * fabs(B[idx]);
}
static void add_fix(void *buf, int64_t idx, int64_t q) {
  int64_t *B = (int64_t *)buf;
  B[idx] = iadd(B[idx], q);
}

/* ---------------------------------------------------------- Step 1: deposit */

/* CIC mass assignment (cloud-in-cell, cell-centred): per axis t = x - 1/2,
 * i0 = floor(t), f = t - i0, weights (1-f, f) on cells (i0, i0+1).  The
 * paper's PM deposit (Sec. 3.1, item 1; Sec. 2.2 "steps 1, 2 and 5") does not
 * name its assignment scheme; CIC is the textbook one. */
static int deposit_cic(const orc_mesh *M, const geom *G, int mode, const orc_cic *P,
                       void *buf, double *err, double V) {
  for (int b = 0; b < M->nbox; ++b) {
    for (int64_t p = P->box_off[b]; p < P->box_off[b + 1]; ++p) {
      double pos[3] = {P->x[p], P->y[p], P->z[p]};
      double m = P->m[p];
      int64_t h[3], i0[3];
      double w[3][2];
      for (int a = 0; a < 3; ++a) {
        h[a] = (int64_t)floor(pos[a]);
        double t = pos[a] - 0.5;
        double fl = floor(t);
        double f = t - fl;
        i0[a] = (int64_t)fl;
        w[a][0] = 1.0 - f;
        w[a][1] = f;
      }
      if (!host_in_box(M, b, h)) return ORC_EOUTSIDE;
      int64_t qsum = 0;
      for (int dk = 0; dk < 2; ++dk)
        for (int dj = 0; dj < 2; ++dj)
          for (int di = 0; di < 2; ++di) {
            double wx = w[0][di], wy = w[1][dj], wz = w[2][dk];
            if (wx == 0.0 || wy == 0.0 || wz == 0.0) continue;
            double c = ((m * wx) * wy) * wz / V;
            int64_t idx = buf_index(M, G, b, 0, i0[0] + di, i0[1] + dj, i0[2] + dk);
            if (idx < 0) return ORC_EREACH;
            if (mode != ORC_FIX64) {
              add_f64(buf, err, idx, c);
            } else {
              int64_t q;
              if (q40(c, &q)) return ORC_EOVERFLOW;
              add_fix(buf, idx, q);
              qsum += q;
            }
          }
      if (mode == ORC_FIX64) {
        /* remainder rule: the particle's total lands exactly, the rounding
         * residue goes to the host cell (always a nonzero-weight member) */
        int64_t Q;
        if (q40(m / V, &Q)) return ORC_EOVERFLOW;
        add_fix(buf, buf_index(M, G, b, 0, h[0], h[1], h[2]), Q - qsum);
      }
    }
  }
  return ORC_OK;
}

/* Uniform-sphere supernova injection: mass m and energy e shared equally over
 * the N cells whose centres lie within r (Sec. 3.2.1, eq. "du" with full
 * coverage and no momentum term).  Fields 0 (rho) and 4 (E). */
static int deposit_sn(const orc_mesh *M, const geom *G, int mode, const orc_sn *P, void *buf,
                      double *err, double V) {
  for (int b = 0; b < M->nbox; ++b) {
    for (int64_t p = P->box_off[b]; p < P->box_off[b + 1]; ++p) {
      double x = P->x[p], y = P->y[p], z = P->z[p], m = P->m[p], e = P->e[p], r = P->r[p];
      double r2 = r * r;
      int64_t h[3] = {(int64_t)floor(x), (int64_t)floor(y), (int64_t)floor(z)};
      if (!host_in_box(M, b, h)) return ORC_EOUTSIDE;
      int64_t lo[3], hi[3];
      sphere_range(x, r, &lo[0], &hi[0]);
      sphere_range(y, r, &lo[1], &hi[1]);
      sphere_range(z, r, &lo[2], &hi[2]);
      int64_t N = 0, first[3] = {0, 0, 0};
      int host_member = 0;
      for (int64_t k = lo[2]; k <= hi[2]; ++k)
        for (int64_t j = lo[1]; j <= hi[1]; ++j)
          for (int64_t i = lo[0]; i <= hi[0]; ++i)
            if (dist2(x, y, z, i, j, k) <= r2) {
              if (N == 0) { first[0] = i; first[1] = j; first[2] = k; }
              if (i == h[0] && j == h[1] && k == h[2]) host_member = 1;
              ++N;
            }
      int only_host = (N == 0);
      if (only_host) { N = 1; host_member = 1; }
      double cr = m / ((double)N * V);
      double ce = e / ((double)N * V);
      int64_t qr = 0, qe = 0;
      if (mode == ORC_FIX64) {
        if (q40(cr, &qr) || q40(ce, &qe)) return ORC_EOVERFLOW;
      }
      for (int64_t k = lo[2]; k <= hi[2]; ++k)
        for (int64_t j = lo[1]; j <= hi[1]; ++j)
          for (int64_t i = lo[0]; i <= hi[0]; ++i) {
            int in = only_host ? (i == h[0] && j == h[1] && k == h[2])
                               : (dist2(x, y, z, i, j, k) <= r2);
            if (!in) continue;
            int64_t i0 = buf_index(M, G, b, 0, i, j, k);
            int64_t i4 = buf_index(M, G, b, 4, i, j, k);
            if (i0 < 0 || i4 < 0) return ORC_EREACH;
            if (mode != ORC_FIX64) {
              add_f64(buf, err, i0, cr);
              add_f64(buf, err, i4, ce);
            } else {
              add_fix(buf, i0, qr);
              add_fix(buf, i4, qe);
            }
          }
      if (mode == ORC_FIX64) {
        int64_t Qr, Qe;
        if (q40(m / V, &Qr) || q40(e / V, &Qe)) return ORC_EOVERFLOW;
        const int64_t *t = host_member ? h : first;
        add_fix(buf, buf_index(M, G, b, 0, t[0], t[1], t[2]), Qr - N * qr);
        add_fix(buf, buf_index(M, G, b, 4, t[0], t[1], t[2]), Qe - N * qe);
      }
    }
  }
  return ORC_OK;
}

#define ORC_FOUR_PI (4.0 * 3.141592653589793)

/* Bondi-Hoyle request of one sink (Sec. 3.1.1, eqs. "rbh" and "mdot", and
 * the clamp of r_acc).  Over the kernel cells (centres within r_K of the
 * sink), each sum on the 2^-40 grid:
 *   M     = sum rho V                      (kernel gas mass),
 *   u     = sum p V / M - v_sink           (mass-weighted mean gas velocity
 *                                           relative to the sink), v_inf = |u|,
 *   c_inf = sum rho V c_s / M              (mass-weighted mean sound speed),
 *           c_s^2 = gamma (gamma - 1) e_int / rho for an ideal gas, with
 *           e_int = E - |p|^2 / (2 rho) taken as 0 where it is negative and
 *           c_s = 0 where rho <= 0,
 *   rho_inf = M / (N V)                    (mean density of the N cells).
 * Then r_BH = G m / (v_inf^2 + c_inf^2) and the second form of eq. "mdot",
 * mdot = 4 pi rho_inf r_BH^2 (lambda^2 c_inf^2 + v_inf^2)^(1/2).  The request
 * mdot dt is capped at M (also when v_inf = c_inf = 0, where the rate has no
 * finite value), and the Gaussian width is r_BH / dx clamped to
 * [1/4, r_K / 2] cells (r_K / 2 when the rate has no finite value).  M <= 0
 * requests nothing. */
static int bondi_request(const orc_mesh *M, const geom *G, const orc_sinks *S, int64_t s,
                         const int64_t lo[3], const int64_t hi[3], const double *state,
                         double V, double *req_out, double *racc_out) {
  const double x = S->x[s], y = S->y[s], z = S->z[s];
  const double r2 = S->r_k * S->r_k;
  int64_t ncell = 0, qm = 0, qx = 0, qy = 0, qz = 0, qc = 0;
  for (int64_t k = lo[2]; k <= hi[2]; ++k)
    for (int64_t j = lo[1]; j <= hi[1]; ++j)
      for (int64_t i = lo[0]; i <= hi[0]; ++i) {
        double d2 = dist2(x, y, z, i, j, k);
        if (!(d2 <= r2)) continue;
        int64_t iw, jw, kw;
        int ob = owner_of(M, G, i, j, k, &iw, &jw, &kw);
        if (ob < 0) return ORC_EINVAL;
        double rho = state[state_index(M, G, ob, 0, iw, jw, kw)];
        double px = state[state_index(M, G, ob, 1, iw, jw, kw)];
        double py = state[state_index(M, G, ob, 2, iw, jw, kw)];
        double pz = state[state_index(M, G, ob, 3, iw, jw, kw)];
        double E = state[state_index(M, G, ob, 4, iw, jw, kw)];
        double cs = 0.0;
        if (rho > 0.0) {
          double eint = E - ((px * px + py * py) + pz * pz) / (2.0 * rho);
          if (!(eint > 0.0)) eint = 0.0;
          cs = sqrt(((S->gamma * (S->gamma - 1.0)) * eint) / rho);
        }
        double m = rho * V;
        int64_t a0, a1, a2, a3, a4;
        if (q40(m, &a0) || q40(px * V, &a1) || q40(py * V, &a2) || q40(pz * V, &a3) ||
            q40(m * cs, &a4))
          return ORC_EOVERFLOW;
        qm += a0; qx += a1; qy += a2; qz += a3; qc += a4;
        ++ncell;
      }
  const double half = 0.5 * S->r_k;
  const double Mk = (double)qm * FIX_INV;
  *req_out = 0.0;
  *racc_out = half;
  if (!(Mk > 0.0)) return ORC_OK;
  const double ux = ((double)qx * FIX_INV) / Mk - S->vx[s];
  const double uy = ((double)qy * FIX_INV) / Mk - S->vy[s];
  const double uz = ((double)qz * FIX_INV) / Mk - S->vz[s];
  const double v2 = (ux * ux + uy * uy) + uz * uz;
  const double cinf = ((double)qc * FIX_INV) / Mk;
  const double c2 = cinf * cinf;
  const double den = v2 + c2;
  if (!(den > 0.0)) {
    *req_out = Mk;
    return ORC_OK;
  }
  const double rho_inf = Mk / ((double)ncell * V);
  const double rbh = (S->G * S->m[s]) / den;
  const double mdot =
      ((ORC_FOUR_PI * rho_inf) * (rbh * rbh)) * sqrt((S->lambda * S->lambda) * c2 + v2);
  const double req = mdot * S->dt;
  *req_out = (req <= Mk) ? req : Mk;
  const double rc = rbh / M->dx;
  *racc_out = (rc < 0.25) ? 0.25 : ((rc > half) ? half : rc);
  return ORC_OK;
}

#define ORC_PI 3.141592653589793

/* Truelove density of one cell (Sec. 3.1.1, eq. "truelove"): the caller's
 * constant rho_tr, or with truelove_J > 0 the cell's own
 * rho_Tr = J^2 pi c_s^2 / (G dx^2), the sound speed from the cell's state as
 * in the Bondi-Hoyle rate, c_s^2 = gamma (gamma - 1) e_int / rho with
 * e_int = E - |p|^2 / (2 rho) taken as 0 where negative, and c_s = 0 where
 * rho <= 0. */
static double truelove_rho(const orc_limits *L, double dx, double rho, double px, double py,
                           double pz, double E) {
  if (!(L->truelove_J > 0.0)) return L->rho_tr;
  double c2 = 0.0;
  if (rho > 0.0) {
    double eint = E - ((px * px + py * py) + pz * pz) / (2.0 * rho);
    if (!(eint > 0.0)) eint = 0.0;
    c2 = ((L->gamma * (L->gamma - 1.0)) * eint) / rho;
  }
  return (((L->truelove_J * L->truelove_J) * ORC_PI) * c2) / ((L->G * dx) * dx);
}

/* The Truelove density of the cell whose field-0 state element is i0 in a
 * box of `step` cells per field. */
static double truelove_at(const orc_limits *L, double dx, const double *state, int64_t i0,
                          int64_t step) {
  return truelove_rho(L, dx, state[i0], state[i0 + step], state[i0 + 2 * step],
                      state[i0 + 3 * step], state[i0 + 4 * step]);
}

/* Limiter parameters: a per-cell Truelove density needs G > 0 and a finite
 * gamma >= 1. */
static int check_limits(const orc_limits *L) {
  if (L->rho_tr != L->rho_tr) return ORC_EINVAL;
  if (L->truelove_J > 0.0 &&
      (!(L->G > 0.0) || !isfinite(L->G) || !(L->gamma >= 1.0) || !isfinite(L->gamma) ||
       !isfinite(L->truelove_J)))
    return ORC_EINVAL;
  return ORC_OK;
}

/* Sink removal request (Sec. 3.1.1).  Per sink: Gaussian weights
 * w = exp(-d^2/r_acc^2) over the kernel (eq. "kernel"), normalised by their
 * sum (eq. "kernel_wgt"); the requested mass is either a fixed fraction a of
 * the gas mass in the kernel with a fixed width r_acc, or the Bondi-Hoyle
 * request of bondi_request with its own width; each cell's removal is
 * max(request * phi / V, rho - rho_Tr) (eq. "accretion_function" with the
 * Truelove term).  The kernel sums are taken in 2^-40 fixed point so that
 * they do not depend on summation order.  Field 5 holds the removed density
 * K >= 0. */
static int deposit_sinks(const orc_mesh *M, const geom *G, int mode, const orc_sinks *S,
                         const orc_limits *L, const double *state, void *buf, double *err,
                         double V, double *sink_w, double *sink_mreq, double *sink_racc) {
  double r2 = S->r_k * S->r_k;
  for (int b = 0; b < M->nbox; ++b) {
    for (int64_t s = S->box_off[b]; s < S->box_off[b + 1]; ++s) {
      double x = S->x[s], y = S->y[s], z = S->z[s];
      int64_t h[3] = {(int64_t)floor(x), (int64_t)floor(y), (int64_t)floor(z)};
      if (!host_in_box(M, b, h)) return ORC_EOUTSIDE;
      int64_t lo[3], hi[3];
      sphere_range(x, S->r_k, &lo[0], &hi[0]);
      sphere_range(y, S->r_k, &lo[1], &hi[1]);
      sphere_range(z, S->r_k, &lo[2], &hi[2]);
      double racc = S->r_gauss, Mbondi = 0.0;
      if (S->rate == ORC_RATE_BONDI) {
        int rc = bondi_request(M, G, S, s, lo, hi, state, V, &Mbondi, &racc);
        if (rc) return rc;
      }
      const double g2 = racc * racc;
      sink_racc[s] = racc;
      int64_t Wq = 0, Mq = 0;
      for (int64_t k = lo[2]; k <= hi[2]; ++k)
        for (int64_t j = lo[1]; j <= hi[1]; ++j)
          for (int64_t i = lo[0]; i <= hi[0]; ++i) {
            double d2 = dist2(x, y, z, i, j, k);
            if (!(d2 <= r2)) continue;
            int64_t iw, jw, kw;
            int ob = owner_of(M, G, i, j, k, &iw, &jw, &kw);
            if (ob < 0) return ORC_EINVAL;
            double rho = state[state_index(M, G, ob, 0, iw, jw, kw)];
            double w = orc_exp(-(d2 / g2));
            int64_t qw, qm;
            if (q40(w, &qw) || q40(rho * V, &qm)) return ORC_EOVERFLOW;
            Wq += qw;
            Mq += qm;
          }
      sink_w[s] = 0.0;
      sink_mreq[s] = 0.0;
      if (Wq <= 0) continue;
      double W = (double)Wq * FIX_INV;
      double Mreq = (S->rate == ORC_RATE_BONDI) ? Mbondi : S->a[s] * ((double)Mq * FIX_INV);
      sink_w[s] = W;
      sink_mreq[s] = Mreq;
      int64_t qreq_sum = 0, first[3] = {0, 0, 0};
      int host_member = 0, nmem = 0;
      for (int64_t k = lo[2]; k <= hi[2]; ++k)
        for (int64_t j = lo[1]; j <= hi[1]; ++j)
          for (int64_t i = lo[0]; i <= hi[0]; ++i) {
            double d2 = dist2(x, y, z, i, j, k);
            if (!(d2 <= r2)) continue;
            if (nmem++ == 0) { first[0] = i; first[1] = j; first[2] = k; }
            if (i == h[0] && j == h[1] && k == h[2]) host_member = 1;
            int64_t iw, jw, kw;
            int ob = owner_of(M, G, i, j, k, &iw, &jw, &kw);
            int64_t i0 = state_index(M, G, ob, 0, iw, jw, kw);
            double rho = state[i0];
            double w = orc_exp(-(d2 / g2));
            double kreq = (Mreq * w) / (W * V);
            double tr = rho - truelove_at(L, M->dx, state, i0, box_cells(M, ob));
            double kc = (tr > kreq) ? tr : kreq;
            int64_t idx = buf_index(M, G, b, 5, i, j, k);
            if (idx < 0) return ORC_EREACH;
            if (mode != ORC_FIX64) {
              add_f64(buf, err, idx, kc);
            } else {
              int64_t qk, qr;
              if (q40(kc, &qk) || q40(kreq, &qr)) return ORC_EOVERFLOW;
              add_fix(buf, idx, qk);
              qreq_sum += qr;
            }
          }
      if (mode == ORC_FIX64) {
        int64_t Q;
        if (q40(Mreq / V, &Q)) return ORC_EOVERFLOW;
        const int64_t *t = host_member ? h : first;
        add_fix(buf, buf_index(M, G, b, 5, t[0], t[1], t[2]), Q - qreq_sum);
      }
    }
  }
  return ORC_OK;
}

static int check_fix_range(const void *buf, int64_t n) {
  const int64_t *B = (const int64_t *)buf;
  const int64_t lim = (int64_t)1 << 62;
  for (int64_t i = 0; i < n; ++i)
    if (B[i] >= lim || B[i] <= -lim) return ORC_EOVERFLOW;
  return ORC_OK;
}

/* App. A.1 items 3-4: the relative error bound r = err / |v| of a summed
 * cell, then v with its lowest nb = 52 + M + ceil(log2 r) mantissa bits
 * cleared (nb clamped to [0, 52]).  ceil(log2 r) is read off frexp exactly:
 * r = m 2^k with m in [1/2, 1), so it is k - 1 when m = 1/2 and k otherwise.
 * Zero and non-finite sums, and cells nothing was added to, stay as they are. */
static double truncate_err(double v, double err, int margin) {
  if (v == 0.0 || !isfinite(v) || !(err > 0.0)) return v;
  int k;
  const double m = frexp(err / fabs(v), &k);
  int nb = 52 + margin + ((m == 0.5) ? k - 1 : k);
  if (nb <= 0) return v;
  if (nb > 52) nb = 52;
  uint64_t bits;
  memcpy(&bits, &v, sizeof bits);
  bits &= ~((((uint64_t)1) << nb) - 1);
  memcpy(&v, &bits, sizeof v);
  return v;
}

/* Sink parameters: a kernel radius, and for the Bondi-Hoyle rate the sink
 * masses and velocities and finite G, dt >= 0, gamma >= 1, lambda >= 0, with
 * r_K >= 1/2 so that the clamp interval [1/4, r_K/2] is not empty. */
static int check_sinks(const orc_sinks *S) {
  if (!(S->r_k > 0.0)) return ORC_EINVAL;
  if (S->rate == ORC_RATE_FRACTION) return (S->r_gauss > 0.0) ? ORC_OK : ORC_EINVAL;
  if (S->rate != ORC_RATE_BONDI) return ORC_EINVAL;
  if (!S->m || !S->vx || !S->vy || !S->vz) return ORC_EINVAL;
  if (!(S->r_k >= 0.5) || !(S->G >= 0.0) || !isfinite(S->G) || !(S->dt >= 0.0) ||
      !isfinite(S->dt) || !(S->gamma >= 1.0) || !isfinite(S->gamma) ||
      !(S->lambda >= 0.0) || !isfinite(S->lambda))
    return ORC_EINVAL;
  return ORC_OK;
}

static int deposit_all(const orc_mesh *M, int mode, const orc_cic *cic, const orc_sn *sn,
                       const orc_sinks *sk, const orc_limits *L, const double *state,
                       void *buf, double *err, double *sink_w, double *sink_mreq,
                       double *sink_racc) {
  int rc = check_mesh(M);
  if (rc) return rc;
  if (sk && (M->nfield != 6 || !state || !L || !sink_w || !sink_mreq || !sink_racc))
    return ORC_EINVAL;
  if (sk && (rc = check_sinks(sk))) return rc;
  if (sk && (rc = check_limits(L))) return rc;
  geom G;
  rc = geom_build(M, &G, sk != NULL);
  if (rc) return rc;
  int64_t nb = orc_buffer_elems(M);
  memset(buf, 0, (size_t)nb * 8);
  if (err) memset(err, 0, (size_t)nb * 8);
  double V = (M->dx * M->dx) * M->dx;
  if (cic) rc = deposit_cic(M, &G, mode, cic, buf, err, V);
  if (!rc && sn) rc = deposit_sn(M, &G, mode, sn, buf, err, V);
  if (!rc && sk)
    rc = deposit_sinks(M, &G, mode, sk, L, state, buf, err, V, sink_w, sink_mreq, sink_racc);
  if (!rc && mode == ORC_FIX64) rc = check_fix_range(buf, nb);
  geom_free(&G);
  return rc;
}

/* Step 1 (Sec. 2.2, eq. "delta_u_buf"): zero the buffer, then add every
 * particle's deposition function; CIC first, then supernovae, then sinks,
 * each in array order. */
int orc_deposit(const orc_mesh *M, int mode, const orc_cic *cic, const orc_sn *sn,
                const orc_sinks *sk, const orc_limits *L, const double *state, void *buf,
                double *sink_w, double *sink_mreq, double *sink_racc) {
  if (mode != ORC_F64 && mode != ORC_FIX64) return ORC_EINVAL;
  return deposit_all(M, mode, cic, sn, sk, L, state, buf, NULL, sink_w, sink_mreq, sink_racc);
}

/* Step 1 in the reproducibility mode of App. A.1: the double-precision sums
 * of orc_deposit (same order) with an error bound per buffer element, then
 * every element truncated by truncate_err.  err (same size as buf) receives
 * the bounds. */
int orc_deposit_r(const orc_mesh *M, const orc_cic *cic, const orc_sn *sn,
                  const orc_sinks *sk, const orc_limits *L, const double *state, double *buf,
                  double *err, int margin, double *sink_w, double *sink_mreq,
                  double *sink_racc) {
  if (!err || margin < 0 || margin > 52) return ORC_EINVAL;
  int rc = deposit_all(M, ORC_F64R, cic, sn, sk, L, state, buf, err, sink_w, sink_mreq,
                       sink_racc);
  if (rc) return rc;
  const int64_t nb = orc_buffer_elems(M);
  for (int64_t i = 0; i < nb; ++i) buf[i] = truncate_err(buf[i], err[i], margin);
  return ORC_OK;
}

/* The truncation alone, for checks. */
double orc_truncate_err(double v, double err, int margin) { return truncate_err(v, err, margin); }

/* ------------------------------------------------------------- Step 2: fold */

/* Sec. 2.2 Step 2: every ghost cell of every box is added into the owned cell
 * of whichever box owns its periodic image.  Ghost cells are only read and
 * owned cells only written, so the result is the plain sum. */
int orc_fold(const orc_mesh *M, int mode, void *buf) {
  int rc = check_mesh(M);
  if (rc) return rc;
  geom G;
  rc = geom_build(M, &G, 1);
  if (rc) return rc;
  int64_t g = M->ghost;
  for (int b = 0; b < M->nbox; ++b) {
    const int32_t *lo = M->lo + 3 * b, *n = M->n + 3 * b;
    for (int64_t lk = 0; lk < n[2] + 2 * g; ++lk)
      for (int64_t lj = 0; lj < n[1] + 2 * g; ++lj)
        for (int64_t li = 0; li < n[0] + 2 * g; ++li) {
          int interior = (li >= g && li < n[0] + g) && (lj >= g && lj < n[1] + g) &&
                         (lk >= g && lk < n[2] + g);
          if (interior) continue;
          int64_t i = lo[0] + li - g, j = lo[1] + lj - g, k = lo[2] + lk - g;
          int64_t iw, jw, kw;
          int ob = owner_of(M, &G, i, j, k, &iw, &jw, &kw);
          if (ob < 0) continue; /* no owner: contribution leaves this level */
          for (int f = 0; f < M->nfield; ++f) {
            int64_t src = buf_index(M, &G, b, f, i, j, k);
            int64_t dst = buf_index(M, &G, ob, f, iw, jw, kw);
            if (mode != ORC_FIX64)
              ((double *)buf)[dst] += ((double *)buf)[src];
            else
              add_fix(buf, dst, ((int64_t *)buf)[src]);
          }
        }
  }
  if (mode == ORC_FIX64) rc = check_fix_range(buf, orc_buffer_elems(M));
  geom_free(&G);
  return rc;
}

/* ------------------------------------------------------- Step 3: limiters */

/* Removal limiter of Sec. 3.1.1: a cell loses at most cap*rho unless the
 * Truelove condition (the cell's Truelove density rho_tr) asks for more, and
 * never falls below rho_floor.
 * Returns the limited removal Kl for a requested removal K >= 0. */
static double limited_removal(double K, double rho, double rho_tr, const orc_limits *L) {
  if (!(K > 0.0)) return 0.0;
  double capped = (K < L->cap * rho) ? K : L->cap * rho;
  double tr = rho - rho_tr;
  double lim = (capped > tr) ? capped : tr;
  double room = rho - L->rho_floor;
  if (room < 0.0) room = 0.0;
  return (lim < room) ? lim : room;
}

static double buf_value(int mode, const void *buf, int64_t idx) {
  if (mode != ORC_FIX64) return ((const double *)buf)[idx];
  return (double)((const int64_t *)buf)[idx] * FIX_INV;
}

/* ---------------------------------------------------- Step 4: sink update */

/* Sec. 2.2 Step 4: each sink re-evaluates its deposition function and gains
 * the limited amount, sum_c eta_c k_c V (mass) and the same times the cell
 * velocity p/rho (momentum).  eta_c = Kl_c / K_c from the folded buffer and
 * the state before Step 5; W, the request and r_acc are Step 1's. */
int orc_sink_update(const orc_mesh *M, int mode, const double *state, const void *buf,
                    const orc_sinks *S, const orc_limits *L, const double *sink_w,
                    const double *sink_mreq, const double *sink_racc, double *dm, double *dpx,
                    double *dpy, double *dpz) {
  int rc = check_mesh(M);
  if (rc) return rc;
  if (M->nfield != 6 || !L || check_limits(L)) return ORC_EINVAL;
  geom G;
  rc = geom_build(M, &G, 1);
  if (rc) return rc;
  double V = (M->dx * M->dx) * M->dx;
  double r2 = S->r_k * S->r_k;
  if (!sink_w || !sink_mreq || !sink_racc) rc = ORC_EINVAL;
  for (int b = 0; b < M->nbox && !rc; ++b) {
    for (int64_t s = S->box_off[b]; s < S->box_off[b + 1]; ++s) {
      double x = S->x[s], y = S->y[s], z = S->z[s];
      double W = sink_w[s], Mreq = sink_mreq[s];
      double g2 = sink_racc[s] * sink_racc[s];
      double sm = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
      int64_t qm = 0, qx = 0, qy = 0, qz = 0;
      if (W > 0.0) {
        int64_t lo[3], hi[3];
        sphere_range(x, S->r_k, &lo[0], &hi[0]);
        sphere_range(y, S->r_k, &lo[1], &hi[1]);
        sphere_range(z, S->r_k, &lo[2], &hi[2]);
        for (int64_t k = lo[2]; k <= hi[2]; ++k)
          for (int64_t j = lo[1]; j <= hi[1]; ++j)
            for (int64_t i = lo[0]; i <= hi[0]; ++i) {
              double d2 = dist2(x, y, z, i, j, k);
              if (!(d2 <= r2)) continue;
              int64_t iw, jw, kw;
              int ob = owner_of(M, &G, i, j, k, &iw, &jw, &kw);
              int64_t i0 = state_index(M, &G, ob, 0, iw, jw, kw);
              double rho = state[i0];
              double w = orc_exp(-(d2 / g2));
              double kreq = (Mreq * w) / (W * V);
              double rtr = truelove_at(L, M->dx, state, i0, box_cells(M, ob));
              double tr = rho - rtr;
              double kc = (tr > kreq) ? tr : kreq;
              double K = buf_value(mode, buf, buf_index(M, &G, ob, 5, iw, jw, kw));
              double Kl = limited_removal(K, rho, rtr, L);
              double eta = (K > 0.0) ? Kl / K : 1.0;
              double term = (eta * kc) * V;
              double vx = state[state_index(M, &G, ob, 1, iw, jw, kw)] / rho;
              double vy = state[state_index(M, &G, ob, 2, iw, jw, kw)] / rho;
              double vz = state[state_index(M, &G, ob, 3, iw, jw, kw)] / rho;
              if (mode != ORC_FIX64) {
                sm += term;
                sx += term * vx;
                sy += term * vy;
                sz += term * vz;
              } else {
                int64_t a, bq, c, d;
                if (q40(term, &a) || q40(term * vx, &bq) || q40(term * vy, &c) ||
                    q40(term * vz, &d)) {
                  rc = ORC_EOVERFLOW;
                  break;
                }
                qm += a; qx += bq; qy += c; qz += d;
              }
            }
      }
      if (mode == ORC_FIX64) {
        sm = (double)qm * FIX_INV;
        sx = (double)qx * FIX_INV;
        sy = (double)qy * FIX_INV;
        sz = (double)qz * FIX_INV;
      }
      dm[s] = sm;
      dpx[s] = sx;
      dpy[s] = sy;
      dpz[s] = sz;
    }
  }
  geom_free(&G);
  return rc;
}

/* ------------------------------------------- Steps 3 + 5: limit and apply */

/* Per owned cell, in double precision:
 *  - sink removal K is limited to Kl (Sec. 3.1.1) and removes the fraction
 *    Kl/rho of the cell's mass, momentum and total energy (the accretion
 *    function removes gas at the cell's own velocity and specific energy);
 *  - sources (CIC mass, supernova mass/energy, momentum) are added in full,
 *    except that the momentum change is scaled by the largest lambda in [0,1]
 *    that keeps the internal energy at or above its floor (Sec. 3.2.1,
 *    eq. "lambda");  floor mode 0: e_int >= 0; mode 1: the specific internal
 *    energy of the cell before the update (the paper's C_V T);
 *  - if even lambda = 0 violates the floor, E is raised to the floor and the
 *    cell is counted (the paper does not treat this case).
 * Step 5 then writes U + Delta U^lim.  A cell whose buffer is zero in every
 * channel receives no update: it keeps its state as it is (eta = 1), whether
 * or not that state meets the floors. */
int orc_apply(const orc_mesh *M, int mode, double *state, const void *buf,
              const orc_limits *L, double *eta, orc_counters *cnt) {
  int rc = check_mesh(M);
  if (rc) return rc;
  if (!L || check_limits(L)) return ORC_EINVAL;
  geom G;
  rc = geom_build(M, &G, 0);
  if (rc) return rc;
  orc_counters C = {0, 0, 0, 0};
  int64_t ecell = 0;
  for (int b = 0; b < M->nbox; ++b) {
    const int32_t *lo = M->lo + 3 * b, *n = M->n + 3 * b;
    int64_t nc = box_cells(M, b);
    double *S = state + G.soff[b];
    for (int64_t k = 0; k < n[2]; ++k)
      for (int64_t j = 0; j < n[1]; ++j)
        for (int64_t i = 0; i < n[0]; ++i) {
          int64_t c = (k * n[1] + j) * n[0] + i;
          int64_t gi = lo[0] + i, gj = lo[1] + j, gk = lo[2] + k;
          double rho = S[c], px = S[nc + c], py = S[2 * nc + c], pz = S[3 * nc + c],
                 E = S[4 * nc + c];
          double Dr = buf_value(mode, buf, buf_index(M, &G, b, 0, gi, gj, gk));
          double qx = buf_value(mode, buf, buf_index(M, &G, b, 1, gi, gj, gk));
          double qy = buf_value(mode, buf, buf_index(M, &G, b, 2, gi, gj, gk));
          double qz = buf_value(mode, buf, buf_index(M, &G, b, 3, gi, gj, gk));
          double DE = buf_value(mode, buf, buf_index(M, &G, b, 4, gi, gj, gk));
          double K = 0.0;
          if (M->nfield == 6) K = buf_value(mode, buf, buf_index(M, &G, b, 5, gi, gj, gk));
          if (Dr == 0.0 && qx == 0.0 && qy == 0.0 && qz == 0.0 && DE == 0.0 && K == 0.0) {
            /* no particle reaches the cell: Step 5 adds a zero update and the
             * limiters, which act on updates, leave it alone (eta = 1) */
            if (eta) eta[ecell + c] = 1.0;
            continue;
          }
          double Kl = 0.0;
          if (K > 0.0)
            Kl = limited_removal(K, rho, truelove_rho(L, M->dx, rho, px, py, pz, E), L);
          double et = (K > 0.0) ? Kl / K : 1.0;
          if (K > 0.0) {
            C.touched++;
            if (Kl < K) C.bind++;
          }
          double f = 1.0 - Kl / rho;
          double rho1 = f * rho + Dr;
          double E1 = f * E + DE;
          double p0x = f * px, p0y = f * py, p0z = f * pz;
          double emin = 0.0;
          if (L->eint_mode == 1) {
            double eint0 = E - ((px * px + py * py) + pz * pz) / (2.0 * rho);
            emin = rho1 * (eint0 / rho);
          }
          double Kc = (2.0 * rho1) * (E1 - emin);
          double sx = p0x + qx, sy = p0y + qy, sz = p0z + qz;
          double g1 = ((sx * sx + sy * sy) + sz * sz) - Kc;
          double pp = (p0x * p0x + p0y * p0y) + p0z * p0z;
          double g0 = pp - Kc;
          double lam;
          if (g1 <= 0.0) {
            lam = 1.0;
          } else if (g0 <= 0.0) {
            /* largest root of |q|^2 l^2 + 2 (p0.q) l + (|p0|^2 - Kc) = 0,
             * in the cancellation-free form */
            double qq = (qx * qx + qy * qy) + qz * qz;
            double pq = (p0x * qx + p0y * qy) + p0z * qz;
            double disc = pq * pq - qq * g0;
            double sq = sqrt(disc);
            lam = (pq > 0.0) ? (-g0) / (pq + sq) : (sq - pq) / qq;
            if (lam > 1.0) lam = 1.0;
            if (lam < 0.0) lam = 0.0;
          } else {
            lam = 0.0;
            E1 = emin + pp / (2.0 * rho1);
            C.fall++;
          }
          if (lam < 1.0) C.lam++;
          S[c] = rho1;
          S[nc + c] = p0x + lam * qx;
          S[2 * nc + c] = p0y + lam * qy;
          S[3 * nc + c] = p0z + lam * qz;
          S[4 * nc + c] = E1;
          if (eta) eta[ecell + c] = et;
        }
    ecell += nc;
  }
  if (cnt) *cnt = C;
  geom_free(&G);
  return rc;
}

/* ------------------------------------------- supernova remnants (TIGRESS) */

/* Natural logarithm for the power laws of Sec. 3.2.1 (M_sf, P_snr).
 * Method: x = m 2^e with m in [sqrt(1/2), sqrt(2)), then
 * ln m = 2 atanh(s) = 2 (s + s^3/3 + ... + s^23/23) with s = (m-1)/(m+1)
 * (|s| <= 0.172, so the omitted terms are below 2^-60 relative) in Horner
 * form, plus e ln 2 with ln 2 split as in orc_exp.  Written from the series,
 * not from any library; checked against libm. */
double orc_log(double x) {
  if (x != x || x < 0.0) return NAN;
  if (x == 0.0) return -HUGE_VAL;
  if (isinf(x)) return x;
  int e;
  double m = frexp(x, &e);
  if (m < 0x1.6a09e667f3bcdp-1) {  /* sqrt(1/2) rounded to double */
    m = m * 2.0;
    e = e - 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double s2 = s * s;
  double t = 1.0 / 23.0;
  t = t * s2 + 1.0 / 21.0;
  t = t * s2 + 1.0 / 19.0;
  t = t * s2 + 1.0 / 17.0;
  t = t * s2 + 1.0 / 15.0;
  t = t * s2 + 1.0 / 13.0;
  t = t * s2 + 1.0 / 11.0;
  t = t * s2 + 1.0 / 9.0;
  t = t * s2 + 1.0 / 7.0;
  t = t * s2 + 1.0 / 5.0;
  t = t * s2 + 1.0 / 3.0;
  t = t * s2 + 1.0;
  const double lnm = (2.0 * s) * t;
  const double ln2_hi = 0x1.62e42ffp-1;
  const double ln2_lo = -0x1.718432a1b0e26p-35;
  const double k = (double)e;
  return k * ln2_hi + (k * ln2_lo + lnm);
}

/* x^a = exp(a ln x) for x > 0, from orc_log and orc_exp. */
double orc_pow(double x, double a) { return orc_exp(a * orc_log(x)); }

/* Covered fraction of cell (i, j, k) by the sphere of squared radius r2
 * around (x, y, z): the number of its ns^3 sample points, the centres of
 * the sub-cells of edge 1/ns (ns a power of two, so every coordinate is
 * exact), whose squared distance to the centre, summed in x, y, z order,
 * is at most r2. */
static int64_t covered_samples(double x, double y, double z, double r2, int64_t i, int64_t j,
                               int64_t k, int ns) {
  int64_t c = 0;
  for (int c3 = 0; c3 < ns; ++c3) {
    const double dz = ((double)k + ((double)c3 + 0.5) / (double)ns) - z;
    for (int c2 = 0; c2 < ns; ++c2) {
      const double dy = ((double)j + ((double)c2 + 0.5) / (double)ns) - y;
      for (int c1 = 0; c1 < ns; ++c1) {
        const double ddx = ((double)i + ((double)c1 + 0.5) / (double)ns) - x;
        if ((ddx * ddx + dy * dy) + dz * dz <= r2) ++c;
      }
    }
  }
  return c;
}

/* Covered fraction w of cell (i, j, k) (the host cell h alone, with w = 1,
 * when no sample point of any cell lies within r). */
static double snr_weight(double x, double y, double z, double r2, int64_t i, int64_t j,
                         int64_t k, int ns, double nsamp, int alone, const int64_t h[3]) {
  if (alone) return (i == h[0] && j == h[1] && k == h[2]) ? 1.0 : 0.0;
  const int64_t c = covered_samples(x, y, z, r2, i, j, k, ns);
  return c ? (double)c / nsamp : 0.0;
}

static int snr_params_ok(const orc_snr *S) {
  if (!S || !S->x || !S->y || !S->z || !S->m || !S->e || !S->vx || !S->vy || !S->vz ||
      !S->box_off)
    return 0;
  if (!(S->r_k >= 0.0) || !(S->r_k <= 16.0)) return 0;
  if (S->sub < 1 || S->sub > 16 || (S->sub & (S->sub - 1)) != 0) return 0;
  if (!(S->nh_per_rho > 0.0) || !(S->msf_coef > 0.0) || !(S->psnr_coef >= 0.0) ||
      !(S->eps_k >= 0.0))
    return 0;
  if (!isfinite(S->nh_per_rho) || !isfinite(S->msf_coef) || !isfinite(S->psnr_coef) ||
      !isfinite(S->eps_k))
    return 0;
  return 1;
}

/* Supernova remnants with the variant of the TIGRESS prescription of
 * Sec. 3.2.1 (eqs. "du", "dp", "psnr"), added to the buffer (after
 * orc_deposit).  Per supernova s at x_s with ejecta mass M_ej, energy E_sn
 * and velocity v_s:
 *   kernel    every cell with a covered fraction w > 0 (covered_samples /
 *             sub^3; r_K = S->r_k); if no sample point lies within r_K, the
 *             host cell alone with w = 1;
 *   sums      on the 2^-40 grid: V_snr = sum w V, M_gas = sum w rho V,
 *             P_gas = sum w p V (the state read in place, periodic);
 *   scalars   M_snr = M_gas + M_ej, n_H = nh_per_rho M_snr / V_snr,
 *             M_sf = msf_coef n_H^-0.26, R_M = M_snr / M_sf,
 *             |p_rad| = psnr_coef n_H^-0.17 (R_M > 1, MC),
 *                       sqrt(2 M_ej eps_k E_sn) (0.027 < R_M <= 1, ST),
 *                       0 (EJ),
 *             v_COM = (P_gas + M_ej v_s) / M_snr, E_kin = M_ej |v_s|^2 / 2;
 *   per cell  a = w / V_snr, rhat the unit vector from x_s to the cell
 *             centre (0 at x_s), p_rad = a |p_rad| rhat,
 *             d rho = a M_ej,
 *             d p   = w ((rho + M_ej / V_snr) v_COM - p) + p_rad,
 *             d E   = a (E_sn + E_kin) + v_COM . p_rad.
 * Fixed point: every term rounded on the 2^-40 grid; the mass and the
 * injected energy a (E_sn + E_kin) keep the remainder rule (residue of
 * rint(M_ej / V 2^40), rint((E_sn + E_kin) / V 2^40) to the host cell if it
 * is a kernel cell, else the first in (k, j, i) order); momentum and v_COM .
 * p_rad are rounded per cell.  info (may be NULL) receives per supernova
 * [4][n]: V_snr, M_snr, n_H, |p_rad|.  Fields 0 (rho), 1-3 (p), 4 (E). */
int orc_deposit_snr(const orc_mesh *M, int mode, const orc_snr *S, const double *state,
                    void *buf, double *info) {
  int rc = check_mesh(M);
  if (rc) return rc;
  if (!snr_params_ok(S) || !state || !buf) return ORC_EINVAL;
  if (mode != ORC_F64 && mode != ORC_FIX64) return ORC_EINVAL;
  geom G;
  rc = geom_build(M, &G, 1);
  if (rc) return rc;
  const double V = (M->dx * M->dx) * M->dx;
  const double r2 = S->r_k * S->r_k;
  const int ns = S->sub;
  const double nsamp = (double)ns * (double)ns * (double)ns;
  const int64_t ntot = S->box_off[M->nbox];
  for (int b = 0; b < M->nbox && !rc; ++b) {
    for (int64_t p = S->box_off[b]; p < S->box_off[b + 1] && !rc; ++p) {
      const double x = S->x[p], y = S->y[p], z = S->z[p];
      const double Mej = S->m[p], Esn = S->e[p];
      const double vs[3] = {S->vx[p], S->vy[p], S->vz[p]};
      const int64_t h[3] = {(int64_t)floor(x), (int64_t)floor(y), (int64_t)floor(z)};
      if (!host_in_box(M, b, h)) { rc = ORC_EOUTSIDE; break; }
      int64_t lo[3], hi[3];
      const double pos[3] = {x, y, z};
      for (int a = 0; a < 3; ++a) {
        lo[a] = (int64_t)floor(pos[a] - S->r_k) - 1;
        hi[a] = (int64_t)floor(pos[a] + S->r_k) + 1;
      }
      /* the kernel: cells with a covered sample point, or the host cell alone */
      int any = 0;
      for (int64_t k = lo[2]; k <= hi[2] && !any; ++k)
        for (int64_t j = lo[1]; j <= hi[1] && !any; ++j)
          for (int64_t i = lo[0]; i <= hi[0] && !any; ++i)
            any = covered_samples(x, y, z, r2, i, j, k, ns) > 0;
      const int alone = !any;
      /* kernel sums on the 2^-40 grid */
      int64_t qV = 0, qM = 0, qP[3] = {0, 0, 0}, first[3] = {0, 0, 0};
      int nmem = 0, host_member = 0;
      for (int64_t k = lo[2]; k <= hi[2] && !rc; ++k)
        for (int64_t j = lo[1]; j <= hi[1] && !rc; ++j)
          for (int64_t i = lo[0]; i <= hi[0] && !rc; ++i) {
            const double w = snr_weight(x, y, z, r2, i, j, k, ns, nsamp, alone, h);
            if (w == 0.0) continue;
            if (nmem++ == 0) { first[0] = i; first[1] = j; first[2] = k; }
            if (i == h[0] && j == h[1] && k == h[2]) host_member = 1;
            int64_t iw, jw, kw;
            const int ob = owner_of(M, &G, i, j, k, &iw, &jw, &kw);
            if (ob < 0) { rc = ORC_EINVAL; break; }
            const int64_t i0 = state_index(M, &G, ob, 0, iw, jw, kw);
            const int64_t st = box_cells(M, ob);
            int64_t a0, a1, a2, a3, a4;
            if (q40(w * V, &a0) || q40((w * state[i0]) * V, &a1) ||
                q40((w * state[i0 + st]) * V, &a2) || q40((w * state[i0 + 2 * st]) * V, &a3) ||
                q40((w * state[i0 + 3 * st]) * V, &a4)) {
              rc = ORC_EOVERFLOW;
              break;
            }
            qV += a0; qM += a1; qP[0] += a2; qP[1] += a3; qP[2] += a4;
          }
      if (rc) break;
      /* the remnant's scalars (eqs. "dp", "psnr") */
      const double Vsnr = (double)qV * FIX_INV;
      if (!(Vsnr > 0.0)) { rc = ORC_EINVAL; break; }
      const double Msnr = (double)qM * FIX_INV + Mej;
      const double nH = (Msnr / Vsnr) * S->nh_per_rho;
      const double Msf = S->msf_coef * orc_pow(nH, -0.26);
      const double RM = Msnr / Msf;
      double P = 0.0;
      if (RM > 1.0) P = S->psnr_coef * orc_pow(nH, -0.17);
      else if (RM > 0.027) P = sqrt(((2.0 * Mej) * S->eps_k) * Esn);
      double vc[3];
      for (int a = 0; a < 3; ++a) vc[a] = ((double)qP[a] * FIX_INV + Mej * vs[a]) / Msnr;
      const double Ekin = (0.5 * Mej) * ((vs[0] * vs[0] + vs[1] * vs[1]) + vs[2] * vs[2]);
      const double Eall = Esn + Ekin;
      const double dens_ej = Mej / Vsnr;
      if (info) {
        info[p] = Vsnr;
        info[ntot + p] = Msnr;
        info[2 * ntot + p] = nH;
        info[3 * ntot + p] = P;
      }
      /* the deposition function (eq. "du") */
      int64_t qr_sum = 0, qe_sum = 0;
      for (int64_t k = lo[2]; k <= hi[2] && !rc; ++k)
        for (int64_t j = lo[1]; j <= hi[1] && !rc; ++j)
          for (int64_t i = lo[0]; i <= hi[0] && !rc; ++i) {
            const double w = snr_weight(x, y, z, r2, i, j, k, ns, nsamp, alone, h);
            if (w == 0.0) continue;
            int64_t iw, jw, kw;
            const int ob = owner_of(M, &G, i, j, k, &iw, &jw, &kw);
            const int64_t i0 = state_index(M, &G, ob, 0, iw, jw, kw);
            const int64_t st = box_cells(M, ob);
            const double rho = state[i0];
            const double pc[3] = {state[i0 + st], state[i0 + 2 * st], state[i0 + 3 * st]};
            const double aw = w / Vsnr;
            const double dr = aw * Mej;
            const double d[3] = {((double)i + 0.5) - x, ((double)j + 0.5) - y,
                                 ((double)k + 0.5) - z};
            const double len = sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
            const double pr = aw * P;
            double prad[3], dp[3];
            for (int a = 0; a < 3; ++a) {
              prad[a] = (len > 0.0) ? pr * (d[a] / len) : 0.0;
              dp[a] = w * ((rho + dens_ej) * vc[a] - pc[a]) + prad[a];
            }
            const double einj = aw * Eall;
            const double ecross = (vc[0] * prad[0] + vc[1] * prad[1]) + vc[2] * prad[2];
            int64_t idx[5];
            for (int f = 0; f < 5; ++f) {
              idx[f] = buf_index(M, &G, b, f, i, j, k);
              if (idx[f] < 0) rc = ORC_EREACH;
            }
            if (rc) break;
            if (mode == ORC_F64) {
              add_f64(buf, NULL, idx[0], dr);
              for (int a = 0; a < 3; ++a) add_f64(buf, NULL, idx[1 + a], dp[a]);
              add_f64(buf, NULL, idx[4], einj + ecross);
            } else {
              int64_t q[6];
              if (q40(dr, &q[0]) || q40(dp[0], &q[1]) || q40(dp[1], &q[2]) ||
                  q40(dp[2], &q[3]) || q40(einj, &q[4]) || q40(ecross, &q[5])) {
                rc = ORC_EOVERFLOW;
                break;
              }
              for (int f = 0; f < 4; ++f) add_fix(buf, idx[f], q[f]);
              add_fix(buf, idx[4], iadd(q[4], q[5]));
              qr_sum = iadd(qr_sum, q[0]);
              qe_sum = iadd(qe_sum, q[4]);
            }
          }
      if (rc) break;
      if (mode == ORC_FIX64) {
        /* remainder rule: mass and injected energy land exactly */
        int64_t Qr, Qe;
        if (q40(Mej / V, &Qr) || q40(Eall / V, &Qe)) { rc = ORC_EOVERFLOW; break; }
        const int64_t *t = host_member ? h : first;
        add_fix(buf, buf_index(M, &G, b, 0, t[0], t[1], t[2]), iadd(Qr, -qr_sum));
        add_fix(buf, buf_index(M, &G, b, 4, t[0], t[1], t[2]), iadd(Qe, -qe_sum));
      }
    }
  }
  geom_free(&G);
  return rc;
}

/* ------------------------------------------------------ sink creation */

/* Whether cell (i, j, k) lies within r of the sink at (x, y, z): the kernel
 * membership test (squared distance between the cell centre and the sink,
 * summed in x, y, z order, <= r^2) on the cell's periodic images one domain
 * length away along each axis, so that it matches the stencil a kernel
 * near a domain face enumerates. */
static int within_kernel(const orc_mesh *M, double x, double y, double z, int64_t i, int64_t j,
                         int64_t k, double r2) {
  for (int c = -1; c <= 1; ++c)
    for (int b = -1; b <= 1; ++b)
      for (int a = -1; a <= 1; ++a)
        if (dist2(x, y, z, i + a * (int64_t)M->domain[0], j + b * (int64_t)M->domain[1],
                  k + c * (int64_t)M->domain[2]) <= r2)
          return 1;
  return 0;
}

/* Sink creation (Sec. 3.1.2).  A cell c of the periodic domain, owned by
 * some box, becomes a sink when
 *   (1) rho_c > rho_Tr,c (its Truelove density, eq. "truelove": the
 *       limiter's constant, or the cell's own with truelove_J > 0),
 *   (2) c is the densest cell among those whose centres lie within r_K of
 *       its centre (the cell itself included; cells no box owns are left
 *       out; equal densities are ranked by the global linear cell index, the
 *       lower index counting as denser), and
 *   (3) no existing sink lies within r_K of c's centre (the kernel
 *       membership test, periodic), and, where a buffer with the removal
 *       channel K is given, K is zero at c (the paper's form of the same
 *       test: a cell in no sink's kernel receives no removal).
 * Every test reads the state as it was before any creation, so the result
 * does not depend on the order of the cells.  A new sink sits at the cell
 * centre with mass (rho_c - rho_Tr,c) V and momentum (mass) p_c / rho_c; the
 * cell keeps its velocity and specific energy: rho -> rho_Tr,c,
 * p -> (p / rho) rho_Tr,c, E -> (E / rho) rho_Tr,c (specific energies, and so
 * the per-cell rho_Tr, do not change).  The sinks are listed in increasing
 * global linear cell index (x fastest) in out [7][max_new] (x, y, z, m, px,
 * py, pz); *count receives the number of qualifying cells, and when it
 * exceeds max_new nothing is created.  buf may be NULL, or a buffer without
 * the K channel (nfield 5); existing may be NULL (no sinks). */
int orc_sink_create(const orc_mesh *M, int mode, double *state, const void *buf,
                    const orc_sinks *existing, double r_k, const orc_limits *L,
                    int64_t max_new, double *out, int64_t *count) {
  int rc = check_mesh(M);
  if (rc) return rc;
  if (!state || !count || !L || max_new < 0 || (max_new > 0 && !out)) return ORC_EINVAL;
  if (!(r_k >= 0.0) || !(r_k <= 16.0) || check_limits(L)) return ORC_EINVAL;
  if (mode != ORC_F64 && mode != ORC_FIX64) return ORC_EINVAL;
  const int64_t nsink = existing ? existing->box_off[M->nbox] : 0;
  geom G;
  rc = geom_build(M, &G, 1);
  if (rc) return rc;
  const int64_t nx = M->domain[0], ny = M->domain[1], nz = M->domain[2];
  const int64_t ncell = nx * ny * nz;
  const double V = (M->dx * M->dx) * M->dx;
  const int64_t R = (int64_t)floor(r_k);
  const double r2 = r_k * r_k;
  int64_t *made = (int64_t *)malloc((size_t)(ncell > 0 ? ncell : 1) * sizeof(int64_t));
  if (!made) {
    geom_free(&G);
    return ORC_ENOMEM;
  }
  int64_t n_new = 0;
  for (int64_t k = 0; k < nz; ++k)
    for (int64_t j = 0; j < ny; ++j)
      for (int64_t i = 0; i < nx; ++i) {
        const int64_t c = (k * ny + j) * nx + i;
        int64_t iw, jw, kw;
        const int ob = owner_of(M, &G, i, j, k, &iw, &jw, &kw);
        if (ob < 0) continue;
        const int64_t i0 = state_index(M, &G, ob, 0, iw, jw, kw);
        const double rho = state[i0];
        if (!(rho > truelove_at(L, M->dx, state, i0, box_cells(M, ob)))) continue;
        if (buf && M->nfield == 6 &&
            buf_value(mode, buf, buf_index(M, &G, ob, 5, iw, jw, kw)) != 0.0)
          continue;
        int near = 0;
        for (int64_t s = 0; s < nsink && !near; ++s)
          near = within_kernel(M, existing->x[s], existing->y[s], existing->z[s], i, j, k, r2);
        if (near) continue;
        int densest = 1;
        for (int64_t dk = -R; dk <= R && densest; ++dk)
          for (int64_t dj = -R; dj <= R && densest; ++dj)
            for (int64_t di = -R; di <= R && densest; ++di) {
              if (!((double)(di * di + dj * dj + dk * dk) <= r2)) continue;
              int64_t ii, jj, kk;
              const int on = owner_of(M, &G, i + di, j + dj, k + dk, &ii, &jj, &kk);
              if (on < 0) continue;
              const int64_t o = (kk * ny + jj) * nx + ii;
              if (o == c) continue;
              const double ro = state[state_index(M, &G, on, 0, ii, jj, kk)];
              if (ro > rho || (ro == rho && o < c)) densest = 0;
            }
        if (densest) made[n_new++] = c;
      }
  *count = n_new;
  if (n_new <= max_new) {
    for (int64_t s = 0; s < n_new; ++s) {
      const int64_t c = made[s];
      const int64_t i = c % nx, j = (c / nx) % ny, k = c / (nx * ny);
      int64_t iw, jw, kw;
      const int ob = owner_of(M, &G, i, j, k, &iw, &jw, &kw);
      const int64_t i0 = state_index(M, &G, ob, 0, iw, jw, kw);
      const int64_t step = box_cells(M, ob);
      const double rho = state[i0];
      const double rtr = truelove_at(L, M->dx, state, i0, step);
      const double m = (rho - rtr) * V;
      out[0 * max_new + s] = (double)i + 0.5;
      out[1 * max_new + s] = (double)j + 0.5;
      out[2 * max_new + s] = (double)k + 0.5;
      out[3 * max_new + s] = m;
      for (int a = 0; a < 3; ++a) {
        const double v = state[i0 + (1 + a) * step] / rho;
        out[(4 + a) * max_new + s] = m * v;
        state[i0 + (1 + a) * step] = v * rtr;
      }
      state[i0 + 4 * step] = (state[i0 + 4 * step] / rho) * rtr;
      state[i0] = rtr;
    }
  }
  free(made);
  geom_free(&G);
  return ORC_OK;
}
