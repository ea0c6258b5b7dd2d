/* mro.c -- CPU oracle for one MRLT/NERK3 macro step (arXiv:1905.08717).
 *
 * TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The HIP path shares
 * no code with it.
 *
 * Plain FP64, dense per-level arrays, row-major cell index.  Every formula
 * is written with explicit parentheses so that its rounding order is fixed;
 * build with -ffp-contract=off.  Where the paper is silent or ambiguous the
 * reading taken is stated at the place it is used.
 *
 * Paper passages followed (section / equation labels of the paper):
 *   Sec. 2        finite-volume form, eq. (pde), (int); source at the average
 *   Sec. 2 "Projection and prediction operators": projection = mean of the
 *                 children; 1D prediction q_i -/+ (q_{i+1}-q_{i-1})/8;
 *                 details d = q - q~ (eq. waveletcoeff); locality and
 *                 consistency of the prediction
 *   Sec. 3        compact RK2/RK3, NERK partials at theta = 1/4, 1/2, 3/4
 *   Sec. 4        dt_l = 2^{L-l} dt (eq. dt), l_min(n), Sec. 4.1.1 (eqs.
 *                 projleaf, projnode), Sec. 4.1.2 (eq. rk3proj), Sec. 4.2
 *                 (eq. refreshRk2, ProjRK3equations1/2), Sec. 4.3, and the
 *                 remark that remeshing only touches evolved scales
 *   Appendix      Alg. AdaptiveMesh, waveletThres, alg-LTS, projRK2, Steprk2,
 *                 projRK3, Steprk3, refRK2, refRK22
 *   Sec. 5        AUSM+ flux for Burgers and Euler; Neumann / periodic BC
 */
#include "mro.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ABSENT 0
#define LEAF 1
#define INTERNAL 2

/* time slots per cell */
enum { S_Q0, S_Q1, S_H1, S_N14, S_N34, S_QH, S_QE, S_X2, S_Q1REF, S_Q1SW,
       S_CBM, S_CBE, NSLOT };

typedef struct {
  int n;            /* cells per dimension */
  int64_t ncell;    /* n^d */
  uint8_t* st;      /* ABSENT / LEAF / INTERNAL */
  double* slot[NSLOT];
  double* regc;     /* [2d][m][ncell]      coarse-side flux accumulator   */
  double* regf;     /* [2d][nsub][m][ncell] fine-side accumulator per subface */
  uint8_t* W;       /* remesh: candidate internal set */
  uint8_t* sig;     /* remesh: significant */
  uint8_t* fresh;   /* remesh: node created by this remesh */
} level_t;

struct mro_ctx {
  int d, L, l0, m, nsub;
  double eps;
  mro_scheme s;
  level_t lv[MRO_MAXLEV + 1];
  double dx[MRO_MAXLEV + 1][3], invdx[MRO_MAXLEV + 1][3], vol[MRO_MAXLEV + 1];
  double t, dt;
  double vel[3];    /* advection velocity of the flame PDEs this macro step */
  int lmin;
  int64_t leaf_updates, near_thr, iters;
  int nonfinite, bad;
  char err[256];
  /* near-threshold decisions |D - eps_l| <= 1e-12 eps_l: fine iterations
   * completed before the remesh, level and Morton key of the node */
  int64_t* near_iter;
  int32_t* near_lev;
  uint64_t* near_key;
  int64_t near_n, near_cap;
};

/* RK coefficients of the compact forms (Sec. 3) and the NERK partials.  */
static const double C_HALF = 0.5, C_3_4 = 0.75, C_1_4 = 0.25;
static const double C_7_32 = 7.0 / 32.0, C_15_32 = 15.0 / 32.0;
static const double C_1_32 = 1.0 / 32.0, C_9_32 = 9.0 / 32.0;
#define C_1_3 (1.0 / 3.0)
#define C_2_3 (2.0 / 3.0)
#define C_1_6 (1.0 / 6.0)

static void fail(mro_ctx* c, const char* fmt, ...) {
#pragma omp critical(mro_fail)
  {
    if (!c->bad) {
      va_list ap;
      va_start(ap, fmt);
      vsnprintf(c->err, sizeof c->err, fmt, ap);
      va_end(ap);
      c->bad = 1;
    }
  }
}

#define SL(c, lev, s, k, i) ((c)->lv[lev].slot[s][(int64_t)(k) * (c)->lv[lev].ncell + (i)])

/* ----------------------------------------------------------------------- */
/* geometry and boundary conditions                                          */

static int64_t cidx(const mro_ctx* c, int lev, const int* x) {
  int64_t n = c->lv[lev].n;
  int64_t i = x[0];
  if (c->d > 1) i += n * x[1];
  if (c->d > 2) i += n * n * x[2];
  return i;
}

static void ccoord(const mro_ctx* c, int lev, int64_t i, int* x) {
  int64_t n = c->lv[lev].n;
  x[0] = (int)(i % n);
  x[1] = c->d > 1 ? (int)((i / n) % n) : 0;
  x[2] = c->d > 2 ? (int)(i / (n * n)) : 0;
}

/* Stencil coordinate: periodic wraps, homogeneous Neumann reflects evenly
 * (q_{-1} = q_0, q_{-2} = q_1), the reading of the paper's Neumann BC.
 * Homogeneous Dirichlet (Q = 0 on the boundary, Sec. 5 2D Burgers) uses the
 * same mirror cell with the sign flipped (q_{-1} = -q_0, q_{-2} = -q_1):
 * see stencil_flip.                                                        */
static int map_stencil(const mro_ctx* c, int a, int i, int n) {
  if (i < 0) return c->s.bc[a][0] == MRO_BC_PERIODIC ? i + n : -1 - i;
  if (i >= n) return c->s.bc[a][1] == MRO_BC_PERIODIC ? i - n : 2 * n - 1 - i;
  return i;
}

/* 1 when stencil coordinate i along axis a lies outside the domain on a
 * Dirichlet side: the mirrored value enters with its sign flipped.        */
static int stencil_flip(const mro_ctx* c, int a, int i, int n) {
  if (i < 0) return c->s.bc[a][0] == MRO_BC_DIRICHLET;
  if (i >= n) return c->s.bc[a][1] == MRO_BC_DIRICHLET;
  return 0;
}

/* Neighbourhood coordinate in the remesh rules: wraps when periodic and is
 * -1 outside the domain otherwise.                                         */
static int map_nbr(const mro_ctx* c, int a, int i, int n) {
  if (i < 0) return c->s.bc[a][0] == MRO_BC_PERIODIC ? i + n : -1;
  if (i >= n) return c->s.bc[a][1] == MRO_BC_PERIODIC ? i - n : -1;
  return i;
}

static uint64_t morton(int d, const int* x) {
  uint64_t k = 0;
  for (int b = 0; b < 21; b++)
    for (int a = 0; a < d; a++)
      k |= (uint64_t)((x[a] >> b) & 1) << (d * b + a);
  return k;
}

static void demorton(int d, uint64_t k, int* x) {
  x[0] = x[1] = x[2] = 0;
  for (int b = 0; b < 21; b++)
    for (int a = 0; a < d; a++)
      x[a] |= (int)((k >> (d * b + a)) & 1) << b;
}

/* ----------------------------------------------------------------------- */
/* projection and prediction (Sec. 2, "Projection and prediction operators") */

/* Projection: the parent is the mean of its 2^d children, summed in child
 * order a | b<<1 | c<<2 and multiplied by 2^{-d}.                          */
static double proj_scale(int d) { return d == 1 ? 0.5 : (d == 2 ? 0.25 : 0.125); }

/* Prediction of child cb (bit a = x, bit 1 = y, bit 2 = z) of the middle
 * cell of a 3^d stencil.  1D: q -/+ (q_{i+1} - q_{i-1})/8 as printed in the
 * paper.  Multi-D: the tensor product of the 1D operator (the paper refers
 * to another work for these; the tensor product is local, exact on
 * per-dimension quadratics and keeps projection o prediction = identity).
 * Stencil index (ox+1) + 3(oy+1) + 9(oz+1).                                */
static double predict1(int d, const double* S, int cb) {
#define P(ox, oy, oz) S[((ox) + 1) + 3 * ((oy) + 1) + 9 * ((oz) + 1)]
  int a = cb & 1, b = (cb >> 1) & 1, e = (cb >> 2) & 1;
  double q = P(0, 0, 0);
  if (d == 1) {
    double qx = (P(1, 0, 0) - P(-1, 0, 0)) * 0.125;
    return a ? q + qx : q - qx;
  }
  if (d == 2) {
    double qx = (P(1, 0, 0) - P(-1, 0, 0)) * 0.125;
    double qy = (P(0, 1, 0) - P(0, -1, 0)) * 0.125;
    double qxy = ((P(1, 1, 0) - P(1, -1, 0)) - (P(-1, 1, 0) - P(-1, -1, 0))) * 0.015625;
    double v = q;
    v = a ? v + qx : v - qx;
    v = b ? v + qy : v - qy;
    v = (a == b) ? v + qxy : v - qxy;
    return v;
  }
  {
    double qx = (P(1, 0, 0) - P(-1, 0, 0)) * 0.125;
    double qy = (P(0, 1, 0) - P(0, -1, 0)) * 0.125;
    double qz = (P(0, 0, 1) - P(0, 0, -1)) * 0.125;
    double qxy = ((P(1, 1, 0) - P(1, -1, 0)) - (P(-1, 1, 0) - P(-1, -1, 0))) * 0.015625;
    double qxz = ((P(1, 0, 1) - P(1, 0, -1)) - (P(-1, 0, 1) - P(-1, 0, -1))) * 0.015625;
    double qyz = ((P(0, 1, 1) - P(0, 1, -1)) - (P(0, -1, 1) - P(0, -1, -1))) * 0.015625;
    double qxyz = (((P(1, 1, 1) - P(1, 1, -1)) - (P(1, -1, 1) - P(1, -1, -1))) -
                   ((P(-1, 1, 1) - P(-1, 1, -1)) - (P(-1, -1, 1) - P(-1, -1, -1)))) *
                  0.001953125;
    double v = q;
    v = a ? v + qx : v - qx;
    v = b ? v + qy : v - qy;
    v = e ? v + qz : v - qz;
    v = (a == b) ? v + qxy : v - qxy;
    v = (a == e) ? v + qxz : v - qxz;
    v = (b == e) ? v + qyz : v - qyz;
    v = ((a ^ b ^ e) == 1) ? v + qxyz : v - qxyz;
    return v;
  }
#undef P
}

/* ----------------------------------------------------------------------- */
/* which time slot holds which value (Sec. 4; readings in the design notes)  */

/* Level l's own stencil state at stage s: S1 q^n, S2 q* (internal nodes:
 * the projection of Alg. projRK2), S3 q** (internal: Alg. projRK3).       */
static int slot_own(int st, int stage) {
  if (stage == 1) return S_Q0;
  if (stage == 2) return st == LEAF ? S_Q1 : S_Q1SW;
  return S_QH;
}

/* Slot of a level-p cell used to predict virtual children for level p+1 at
 * stage s.  Case A (p >= l_min, both levels start at t^n): S1 q^n, S2 the
 * first-order theta=1/2 value (Sec. 4.1.1), S3 theta=1/4 (Alg. refRK22).
 * Case B (p = l_min - 1, mid-step): S1 q** (RK3) or the NERK theta=1/2
 * value (RK2) of leaves (Sec. 4.3; both kept in QH) or the fresh
 * projection of internal nodes (Alg. alg-LTS); S2 the end value of leaves or
 * the end value of Sec. 4.3 of internal nodes; S3 theta=3/4 (Alg. refRK22). */
static int slot_parent(const mro_ctx* c, int p, int st, int stage) {
  if (!c->s.lt) {
    /* global time step (the MR/RK comparison scheme): every level is at
     * the same stage time, internal nodes hold the children's projection */
    return slot_own(st, stage);
  }
  if (p >= c->lmin) {
    if (stage == 1) return S_Q0;
    if (stage == 2) return S_H1;
    return S_N14;
  }
  if (p == c->lmin - 1) {
    if (stage == 1) return st == LEAF ? S_QH : S_CBM;
    if (stage == 2) return st == LEAF ? S_QE : S_CBE;
    return S_N34;
  }
  return -1;
}

/* Gather the 3^d stencil around x at level lev, component k, through `pick`
 * (slot chooser).  Returns 0 if a stencil cell does not exist.              */
typedef int (*slot_fn)(const mro_ctx*, int lev, int st, int stage);

static int own_pick(const mro_ctx* c, int lev, int st, int stage) {
  (void)c; (void)lev;
  return slot_own(st, stage);
}
static int parent_pick(const mro_ctx* c, int lev, int st, int stage) {
  return slot_parent(c, lev, st, stage);
}
static int q0_pick(const mro_ctx* c, int lev, int st, int stage) {
  (void)c; (void)lev; (void)st; (void)stage;
  return S_Q0;
}

static int gather3(mro_ctx* c, int lev, const int* x, int stage, slot_fn pick, double* S /*[m][27]*/) {
  int n = c->lv[lev].n, d = c->d;
  for (int s = 0; s < 27; s++)
    for (int k = 0; k < c->m; k++) S[k * 27 + s] = 0.0;
  for (int oz = (d > 2 ? -1 : 0); oz <= (d > 2 ? 1 : 0); oz++)
    for (int oy = (d > 1 ? -1 : 0); oy <= (d > 1 ? 1 : 0); oy++)
      for (int ox = -1; ox <= 1; ox++) {
        int y[3] = {0, 0, 0};
        int off[3] = {ox, oy, oz};
        int flip = 0;
        for (int a = 0; a < d; a++) {
          y[a] = map_stencil(c, a, x[a] + off[a], n);
          flip ^= stencil_flip(c, a, x[a] + off[a], n);
        }
        int64_t i = cidx(c, lev, y);
        int st = c->lv[lev].st[i];
        if (st == ABSENT) return 0;
        int sl = pick(c, lev, st, stage);
        if (sl < 0) return 0;
        int s = (ox + 1) + 3 * (oy + 1) + 9 * (oz + 1);
        for (int k = 0; k < c->m; k++) {
          double v = SL(c, lev, sl, k, i);
          S[k * 27 + s] = flip ? -v : v;
        }
      }
  return 1;
}

/* Value of the cell y (already inside the domain) at level lev in the
 * stencil of level lev's stage s: real cells give their slot, virtual
 * cells (children of a leaf) are predicted from the parent level.         */
static void stage_value(mro_ctx* c, int lev, const int* y, int stage, double* out) {
  int64_t i = cidx(c, lev, y);
  int st = c->lv[lev].st[i];
  if (st != ABSENT) {
    int sl = slot_own(st, stage);
    for (int k = 0; k < c->m; k++) out[k] = SL(c, lev, sl, k, i);
    return;
  }
  int p[3] = {y[0] >> 1, y[1] >> 1, y[2] >> 1};
  int64_t pi = cidx(c, lev - 1, p);
  if (lev - 1 < c->l0 || c->lv[lev - 1].st[pi] != LEAF) {
    fail(c, "stencil cell at level %d has no leaf parent (grading violated)", lev);
    for (int k = 0; k < c->m; k++) out[k] = 0.0;
    return;
  }
  double S[5 * 27];
  if (!gather3(c, lev - 1, p, stage, parent_pick, S)) {
    fail(c, "prediction stencil incomplete at level %d", lev - 1);
    for (int k = 0; k < c->m; k++) out[k] = 0.0;
    return;
  }
  int cb = (y[0] & 1) | ((y[1] & 1) << 1) | ((y[2] & 1) << 2);
  for (int k = 0; k < c->m; k++) out[k] = predict1(c->d, S + 27 * k, cb);
}

/* Finer-side cell (level flev) seen by level flev-1's stage s at its own
 * time: S1 q^n; S2 the extrapolation to t^n + 2 dt_{l+1}: eq. projleaf for
 * leaves, eq. projnode (2 q* - q^n) for internal nodes; S3 the stage-3
 * result (leaves) or the eq. rk3proj value (internal nodes).               */
static void finer_value(mro_ctx* c, int flev, const int* y, int stage, double* out) {
  int64_t i = cidx(c, flev, y);
  int st = c->lv[flev].st[i];
  if (st == ABSENT) {
    fail(c, "finer-side cell missing at level %d", flev);
    for (int k = 0; k < c->m; k++) out[k] = 0.0;
    return;
  }
  if (!c->s.lt) {
    int sl = slot_own(st, stage);
    for (int k = 0; k < c->m; k++) out[k] = SL(c, flev, sl, k, i);
    return;
  }
  for (int k = 0; k < c->m; k++) {
    if (stage == 1)
      out[k] = SL(c, flev, S_Q0, k, i);
    else if (stage == 2)
      out[k] = st == LEAF ? SL(c, flev, S_X2, k, i)
                          : (2.0 * SL(c, flev, S_Q1SW, k, i)) - SL(c, flev, S_Q0, k, i);
    else
      out[k] = SL(c, flev, S_QE, k, i);
  }
}

/* ----------------------------------------------------------------------- */
/* numerical fluxes (Sec. 5)                                                 */

static double minmod(double a, double b) {
  if (a > 0.0 && b > 0.0) return a < b ? a : b;
  if (a < 0.0 && b < 0.0) return a > b ? a : b;
  return 0.0;
}

/* Face states from the four cells a-1, a, a+1, a+2 along the normal.
 * MUSCL with the minmod limiter (the paper does not state its spatial
 * reconstruction; second order MUSCL-minmod is the reading taken).        */
static void recon4(int mode, double c0, double c1, double c2, double c3, double* qL, double* qR) {
  if (mode == 1) {
    double sl = minmod(c1 - c0, c2 - c1);
    double sr = minmod(c2 - c1, c3 - c2);
    *qL = c1 + 0.5 * sl;
    *qR = c2 - 0.5 * sr;
  } else {
    *qL = c1;
    *qR = c2;
  }
}

static void euler_prim(int d, double gm1, const double* q, double* w) {
  double rho = q[0];
  double kin = 0.0;
  w[0] = rho;
  for (int i = 0; i < d; i++) {
    double u = q[1 + i] / rho;
    w[1 + i] = u;
    kin = (i == 0) ? (u * u) : (kin + (u * u));
  }
  w[d + 1] = gm1 * (q[d + 1] - ((0.5 * rho) * kin));
}

/* AUSM+ split Mach numbers and pressures (Liou 1996), beta = 1/8,
 * alpha = 3/16.                                                             */
static double mach_plus(double M) {
  if (fabs(M) < 1.0) {
    double t = M + 1.0, q = (M * M) - 1.0;
    return (0.25 * (t * t)) + (0.125 * (q * q));
  }
  return 0.5 * (M + fabs(M));
}
static double mach_minus(double M) {
  if (fabs(M) < 1.0) {
    double t = M - 1.0, q = (M * M) - 1.0;
    return (-(0.25 * (t * t))) - (0.125 * (q * q));
  }
  return 0.5 * (M - fabs(M));
}
static double pres_plus(double M) {
  if (fabs(M) < 1.0) {
    double t = M + 1.0, q = (M * M) - 1.0;
    return ((0.25 * (t * t)) * (2.0 - M)) + ((0.1875 * M) * (q * q));
  }
  return M > 0.0 ? 1.0 : 0.0;
}
static double pres_minus(double M) {
  if (fabs(M) < 1.0) {
    double t = M - 1.0, q = (M * M) - 1.0;
    return ((0.25 * (t * t)) * (2.0 + M)) - ((0.1875 * M) * (q * q));
  }
  return M < 0.0 ? 1.0 : 0.0;
}

/* AUSM+ flux from primitive face states (rho, u_1..u_d, p).  Interface
 * sound speed: the mean of the two sides (not fixed by the paper).        */
static void ausm_plus(int d, int dir, double gamma, const double* wl, const double* wr, double* F) {
  double gm1 = gamma - 1.0;
  double rl = wl[0], pl = wl[d + 1], rr = wr[0], pr = wr[d + 1];
  double al = sqrt((gamma * pl) / rl), ar = sqrt((gamma * pr) / rr);
  double ah = 0.5 * (al + ar);
  double ml = wl[1 + dir] / ah, mr = wr[1 + dir] / ah;
  double mh = mach_plus(ml) + mach_minus(mr);
  double ph = (pres_plus(ml) * pl) + (pres_minus(mr) * pr);
  double mp = 0.5 * (mh + fabs(mh)), mm = 0.5 * (mh - fabs(mh));
  double kl = 0.0, kr = 0.0;
  for (int i = 0; i < d; i++) {
    kl = (i == 0) ? (wl[1] * wl[1]) : (kl + (wl[1 + i] * wl[1 + i]));
    kr = (i == 0) ? (wr[1] * wr[1]) : (kr + (wr[1 + i] * wr[1 + i]));
  }
  double hl = ((pl / gm1) + ((0.5 * rl) * kl)) + pl; /* rho H = E + p */
  double hr = ((pr / gm1) + ((0.5 * rr) * kr)) + pr;
  F[0] = ah * ((mp * rl) + (mm * rr));
  for (int i = 0; i < d; i++) F[1 + i] = ah * ((mp * (rl * wl[1 + i])) + (mm * (rr * wr[1 + i])));
  F[1 + dir] = F[1 + dir] + ph;
  F[d + 1] = ah * ((mp * hl) + (mm * hr));
}

/* Numerical flux across the face between cells a and a+1 along dir at
 * level lev; `cells` holds a-1, a, a+1, a+2 as [4][m].                   */
static void face_flux(const mro_ctx* c, int lev, int dir, const double* cells, double* F) {
  int m = c->m;
  double ix = c->invdx[lev][dir];
#define CV(j, k) cells[(j) * m + (k)]
  switch (c->s.pde) {
    case MRO_PDE_ADVECTION: {
      double vel = c->s.adv_vel[dir];
      if (c->s.recon == 2) {
        F[0] = vel * (0.5 * (CV(1, 0) + CV(2, 0)));
      } else {
        double qL, qR;
        recon4(c->s.recon, CV(0, 0), CV(1, 0), CV(2, 0), CV(3, 0), &qL, &qR);
        F[0] = vel >= 0.0 ? vel * qL : vel * qR;
      }
      break;
    }
    case MRO_PDE_BURGERS: {
      /* Exact Godunov flux for f = u^2/2 (the paper names AUSM+, which is not
       * defined for a scalar law) plus the centred viscous flux.            */
      double uL, uR;
      recon4(c->s.recon, CV(0, 0), CV(1, 0), CV(2, 0), CV(3, 0), &uL, &uR);
      double a = uL > 0.0 ? uL : 0.0;
      double b = uR < 0.0 ? uR : 0.0;
      double fa = 0.5 * (a * a), fb = 0.5 * (b * b);
      double fadv = fa > fb ? fa : fb;
      double nudx = c->s.nu * ix;
      F[0] = fadv - (nudx * (CV(2, 0) - CV(1, 0)));
      break;
    }
    case MRO_PDE_NAGUMO:
    case MRO_PDE_LINEAR: {
      double nudx = c->s.nu * ix;
      F[0] = -(nudx * (CV(2, 0) - CV(1, 0)));
      break;
    }
    case MRO_PDE_FLAME:
    case MRO_PDE_FLAMEBALL: {
      /* advective part: upwind value of the reconstructed face states (the
       * MUSCL construction of van Leer); then the two-point diffusive flux,
       * coefficient 1 for T and 1/Le for Y                                 */
      double vel = c->vel[dir];
      for (int k = 0; k < m; k++) {
        double fadv;
        if (c->s.recon == 2) {
          fadv = vel * (0.5 * (CV(1, k) + CV(2, k)));
        } else {
          double qL, qR;
          recon4(c->s.recon, CV(0, k), CV(1, k), CV(2, k), CV(3, k), &qL, &qR);
          fadv = vel >= 0.0 ? vel * qL : vel * qR;
        }
        double dif = k == 0 ? 1.0 : 1.0 / c->s.lewis;
        F[k] = fadv - ((dif * ix) * (CV(2, k) - CV(1, k)));
      }
      break;
    }
    case MRO_PDE_EULER: {
      int d = c->d;
      double gm1 = c->s.gamma - 1.0;
      double w[4][5], wl[5], wr[5];
      for (int j = 0; j < 4; j++) euler_prim(d, gm1, cells + j * m, w[j]);
      for (int k = 0; k < m; k++) recon4(c->s.recon, w[0][k], w[1][k], w[2][k], w[3][k], &wl[k], &wr[k]);
      ausm_plus(d, dir, c->s.gamma, wl, wr, F);
      break;
    }
  }
#undef CV
}

static int has_source(const mro_ctx* c) {
  return c->s.pde == MRO_PDE_NAGUMO || c->s.pde == MRO_PDE_LINEAR || c->s.pde == MRO_PDE_FLAME ||
         c->s.pde == MRO_PDE_FLAMEBALL;
}

/* Reaction rate of the one-dimensional flame (Sec. 5): equal heat and mass
 * diffusion, Y = 1 - T, written as the paper gives it in terms of 1 - T.   */
static double omega_flame(const mro_ctx* c, double T) {
  double ze = c->s.ze, u = 1.0 - T;
  return ((0.5 * (ze * ze)) * u) * exp((ze * u) / ((c->s.tau * u) - 1.0));
}

/* Reaction rate of the flame ball (Sec. 5, three-dimensional case).       */
static double omega_ball(const mro_ctx* c, double T, double Y) {
  double ze = c->s.ze, le = c->s.lewis;
  return (((ze * ze) / (2.0 * le)) * Y) * exp((ze * (T - 1.0)) / (1.0 + (c->s.tau * (T - 1.0))));
}

/* Radiative heat loss (Stefan-Boltzmann, Sec. 5).                          */
static double radiation(const mro_ctx* c, double T) {
  double a = (T + (1.0 / c->s.tau)) - 1.0, b = (1.0 / c->s.tau) - 1.0;
  return c->s.kappa * (((a * a) * (a * a)) - ((b * b) * (b * b)));
}

static double reaction_rate(const mro_ctx* c, const double* q) {
  return c->s.pde == MRO_PDE_FLAME ? omega_flame(c, q[0]) : omega_ball(c, q[0], q[1]);
}

/* Pointwise source at the cell average (Sec. 2), added to R per component. */
static void add_source(const mro_ctx* c, const double* q, double* R) {
  switch (c->s.pde) {
    case MRO_PDE_NAGUMO:
      R[0] = R[0] + (((c->s.k_react * q[0]) * (1.0 - q[0])) * (q[0] - c->s.a_react));
      break;
    case MRO_PDE_LINEAR:
      R[0] = R[0] + (c->s.k_react * q[0]);
      break;
    case MRO_PDE_FLAME:
      R[0] = R[0] + omega_flame(c, q[0]);
      break;
    case MRO_PDE_FLAMEBALL: {
      double w = omega_ball(c, q[0], q[1]);
      R[0] = R[0] + (w - radiation(c, q[0]));
      R[1] = R[1] - w;
      break;
    }
  }
}

/* Flame velocity v_f: the reaction rate integrated over the leaves (cell
 * average times cell volume), divided by the cross-section normal to axis
 * 0.  Summed level by level in cell order.                                */
static double flame_speed(const mro_ctx* c) {
  double s = 0.0, area = 1.0;
  for (int a = 1; a < c->d; a++) area = area * (c->s.hi[a] - c->s.lo[a]);
  for (int lev = c->l0; lev <= c->L; lev++) {
    const level_t* LV = &c->lv[lev];
    for (int64_t i = 0; i < LV->ncell; i++) {
      if (LV->st[i] != LEAF) continue;
      double q[2];
      for (int k = 0; k < c->m; k++) q[k] = LV->slot[S_Q0][(int64_t)k * LV->ncell + i];
      s = s + (reaction_rate(c, q) * c->vol[lev]);
    }
  }
  return s / area;
}

/* Advection velocity of the flame PDEs for the coming macro step.          */
static void set_velocity(mro_ctx* c) {
  for (int a = 0; a < 3; a++) c->vel[a] = c->s.adv_vel[a];
  if ((c->s.pde == MRO_PDE_FLAME || c->s.pde == MRO_PDE_FLAMEBALL) && c->s.flame_speed != 0) {
    c->vel[0] = (double)c->s.flame_speed * flame_speed(c);
    c->vel[1] = c->vel[2] = 0.0;
  }
}

/* ----------------------------------------------------------------------- */
/* fluxes of one leaf                                                        */

static void transverse_dims(int d, int dir, int* t0, int* t1) {
  int j = 0, t[2] = {-1, -1};
  for (int a = 0; a < d; a++)
    if (a != dir) t[j++] = a;
  *t0 = t[0];
  *t1 = t[1];
}

/* Flux through face (dir, side) of the leaf x at level lev for stage s.
 * Returns 1 when the neighbour across the face is an internal node: then
 * the flux is the mean of the 2^{d-1} subface fluxes computed at level
 * lev+1 from the leaf's virtual children (predicted from level lev's own
 * stage state) and the neighbour's children (finer-side values) -- the
 * leaf / internal node scenario of Sec. 2.                                  */
static int leaf_face_flux(mro_ctx* c, int lev, const int* x, int dir, int side, int stage, double* F) {
  int d = c->d, m = c->m, n = c->lv[lev].n;
  double cells[4 * 5];
  int nbx = map_nbr(c, dir, x[dir] + (side ? 1 : -1), n);
  int refined = 0;
  if (nbx >= 0) {
    int y[3] = {x[0], x[1], x[2]};
    y[dir] = nbx;
    refined = c->lv[lev].st[cidx(c, lev, y)] == INTERNAL;
  }
  if (!refined) {
    int a = side ? x[dir] : x[dir] - 1;
    for (int j = 0; j < 4; j++) {
      int y[3] = {x[0], x[1], x[2]};
      y[dir] = map_stencil(c, dir, a - 1 + j, n);
      stage_value(c, lev, y, stage, cells + j * m);
      if (stencil_flip(c, dir, a - 1 + j, n))
        for (int k = 0; k < m; k++) cells[j * m + k] = -cells[j * m + k];
    }
    face_flux(c, lev, dir, cells, F);
    return 0;
  }
  /* leaf / internal node: subfaces at level lev+1 */
  double S[5 * 27];
  if (!gather3(c, lev, x, stage, own_pick, S)) {
    fail(c, "stencil of a coarse leaf incomplete at level %d", lev);
    return 1;
  }
  int t0, t1;
  transverse_dims(d, dir, &t0, &t1);
  double Fs[5], Fb[5];
  for (int b = 0; b < c->nsub; b++) {
    int fy[3] = {2 * x[0], 2 * x[1], 2 * x[2]};
    int cbt = 0; /* child bits of the transverse coordinates */
    if (t0 >= 0) { fy[t0] += b & 1; cbt |= (b & 1) << t0; }
    if (t1 >= 0) { fy[t1] += (b >> 1) & 1; cbt |= ((b >> 1) & 1) << t1; }
    double own[2][5], fin[2][5];
    for (int e = 0; e < 2; e++) {
      int cb = cbt | (e << dir);
      for (int k = 0; k < m; k++) own[e][k] = predict1(d, S + 27 * k, cb);
      int y[3] = {fy[0], fy[1], fy[2]};
      y[dir] = 2 * nbx + e;
      finer_value(c, lev + 1, y, stage, fin[e]);
    }
    for (int k = 0; k < m; k++) {
      if (side) { /* X | N : X children low, N children high */
        cells[0 * m + k] = own[0][k]; cells[1 * m + k] = own[1][k];
        cells[2 * m + k] = fin[0][k]; cells[3 * m + k] = fin[1][k];
      } else {
        cells[0 * m + k] = fin[0][k]; cells[1 * m + k] = fin[1][k];
        cells[2 * m + k] = own[0][k]; cells[3 * m + k] = own[1][k];
      }
    }
    face_flux(c, lev + 1, dir, cells, Fb);
    for (int k = 0; k < m; k++) Fs[k] = (b == 0) ? Fb[k] : (Fs[k] + Fb[k]);
  }
  double sc = c->nsub == 1 ? 1.0 : (c->nsub == 2 ? 0.5 : 0.25);
  for (int k = 0; k < m; k++) F[k] = Fs[k] * sc;
  return 1;
}

/* ----------------------------------------------------------------------- */
/* one compact RK stage on the leaves of one level (Sec. 3 and Algs.
 * alg-LTS (stage 1), Steprk2, Steprk3)                                     */

#define REGC(c, lev, f, k, i) \
  ((c)->lv[lev].regc[((int64_t)(f) * (c)->m + (k)) * (c)->lv[lev].ncell + (i)])
#define REGF(c, lev, f, b, k, i) \
  ((c)->lv[lev].regf[(((int64_t)(f) * (c)->nsub + (b)) * (c)->m + (k)) * (c)->lv[lev].ncell + (i)])

static void stage_level(mro_ctx* c, int lev, int stage) {
  int d = c->d, m = c->m;
  level_t* LV = &c->lv[lev];
  double h = c->s.lt ? ldexp(c->dt, c->L - lev) : c->dt; /* eq. dt; global step without LT */
  /* weights b_i of the RK method (Sec. 3): RK3 (1/6, 1/6, 2/3), RK2 (1/2, 1/2) */
  double w = c->s.rk == 2 ? C_HALF : (stage == 3 ? C_2_3 : C_1_6);
  double wh = w * h;
  int64_t nc = LV->ncell;
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t i = 0; i < nc; i++) {
    if (LV->st[i] != LEAF) continue;
    int x[3];
    ccoord(c, lev, i, x);
    double Fm[3][5], Fp[3][5], R[5];
    int refm[3], refp[3];
    for (int dir = 0; dir < d; dir++) {
      refm[dir] = leaf_face_flux(c, lev, x, dir, 0, stage, Fm[dir]);
      refp[dir] = leaf_face_flux(c, lev, x, dir, 1, stage, Fp[dir]);
    }
    for (int k = 0; k < m; k++) {
      for (int dir = 0; dir < d; dir++) {
        double r = (Fm[dir][k] - Fp[dir][k]) * c->invdx[lev][dir];
        R[k] = dir == 0 ? r : (R[k] + r);
      }
    }
    if (has_source(c)) {
      int sl = slot_own(LEAF, stage);
      double q[5];
      for (int k = 0; k < m; k++) q[k] = SL(c, lev, sl, k, i);
      add_source(c, q, R);
    }
    for (int k = 0; k < m; k++) {
      double q0 = SL(c, lev, S_Q0, k, i);
      double r = R[k];
      if (c->s.rk == 2) {
        /* compact RK2 with the NERK theta=1/2 value in two parts, 3/8 after
         * the first stage and 1/8 after the second (Sec. 3); the first-order
         * theta=1/2 value H1 serves the finer level's stage 2 (Sec. 4.1.1) */
        if (stage == 1) {
          SL(c, lev, S_Q1, k, i) = q0 + (h * r);
          SL(c, lev, S_H1, k, i) = q0 + ((C_HALF * h) * r);
          SL(c, lev, S_QH, k, i) = q0 + ((0.375 * h) * r);
        } else {
          double q1 = SL(c, lev, S_Q1, k, i);
          double qe = ((C_HALF * q0) + (C_HALF * q1)) + ((C_HALF * h) * r);
          SL(c, lev, S_QE, k, i) = qe;
          SL(c, lev, S_X2, k, i) = q1 + (h * r);
          SL(c, lev, S_QH, k, i) = SL(c, lev, S_QH, k, i) + ((0.125 * h) * r);
          if (!isfinite(qe)) c->nonfinite = 1;
        }
        continue;
      }
      if (stage == 1) {
        SL(c, lev, S_Q1, k, i) = q0 + (h * r);
        SL(c, lev, S_H1, k, i) = q0 + ((C_HALF * h) * r);
        SL(c, lev, S_N14, k, i) = q0 + ((C_7_32 * h) * r);
        SL(c, lev, S_N34, k, i) = q0 + ((C_15_32 * h) * r);
      } else if (stage == 2) {
        double q1 = SL(c, lev, S_Q1, k, i);
        SL(c, lev, S_QH, k, i) = ((C_3_4 * q0) + (C_1_4 * q1)) + ((C_1_4 * h) * r);
        SL(c, lev, S_X2, k, i) = q1 + (h * r);
        SL(c, lev, S_N14, k, i) = SL(c, lev, S_N14, k, i) + ((C_1_32 * h) * r);
        SL(c, lev, S_N34, k, i) = SL(c, lev, S_N34, k, i) + ((C_9_32 * h) * r);
      } else {
        double qh = SL(c, lev, S_QH, k, i);
        double qe = ((C_1_3 * q0) + (C_2_3 * qh)) + ((C_2_3 * h) * r);
        SL(c, lev, S_QE, k, i) = qe;
        if (!isfinite(qe)) c->nonfinite = 1;
      }
    }
    if (!c->s.reflux) continue;
    /* Conservative flux accumulation (not in the paper, see the design
     * notes): the coarse side keeps sum_s w_s h Fbar_s per refined face.   */
    for (int dir = 0; dir < d; dir++) {
      for (int side = 0; side < 2; side++) {
        int ref = side ? refp[dir] : refm[dir];
        double* F = side ? Fp[dir] : Fm[dir];
        int f = 2 * dir + side;
        if (ref) {
          for (int k = 0; k < m; k++) REGC(c, lev, f, k, i) = REGC(c, lev, f, k, i) + (wh * F[k]);
          continue;
        }
        /* fine side: the neighbour position is virtual (child of a leaf) */
        int n = LV->n;
        int nbx = map_nbr(c, dir, x[dir] + (side ? 1 : -1), n);
        if (nbx < 0) continue;
        int y[3] = {x[0], x[1], x[2]};
        y[dir] = nbx;
        if (LV->st[cidx(c, lev, y)] != ABSENT) continue;
        int px[3] = {y[0] >> 1, y[1] >> 1, y[2] >> 1};
        int64_t pi = cidx(c, lev - 1, px);
        if (c->lv[lev - 1].st[pi] != LEAF) {
          fail(c, "fine-side register without a coarse leaf at level %d", lev - 1);
          continue;
        }
        int t0, t1;
        transverse_dims(d, dir, &t0, &t1);
        int b = 0;
        if (t0 >= 0) b |= x[t0] & 1;
        if (t1 >= 0) b |= (x[t1] & 1) << 1;
        int fX = 2 * dir + (side ? 0 : 1);
        for (int k = 0; k < m; k++)
          REGF(c, lev - 1, fX, b, k, pi) = REGF(c, lev - 1, fX, b, k, pi) + (wh * F[k]);
      }
    }
  }
}

/* ----------------------------------------------------------------------- */
/* projections and the synchronisation values of internal nodes              */

typedef void (*child_val_fn)(mro_ctx* c, int flev, int64_t i, int k, double* v);

static double project_children(mro_ctx* c, int lev, int64_t i, int k, child_val_fn fn) {
  int x[3];
  ccoord(c, lev, i, x);
  int nch = 1 << c->d;
  double s = 0.0;
  for (int cb = 0; cb < nch; cb++) {
    int y[3] = {2 * x[0] + (cb & 1), 2 * x[1] + ((cb >> 1) & 1), 2 * x[2] + ((cb >> 2) & 1)};
    int64_t j = cidx(c, lev + 1, y);
    if (c->lv[lev + 1].st[j] == ABSENT) fail(c, "internal node with a missing child at level %d", lev);
    double v;
    fn(c, lev + 1, j, k, &v);
    s = (cb == 0) ? v : (s + v);
  }
  return s * proj_scale(c->d);
}

static void cv_q0(mro_ctx* c, int f, int64_t j, int k, double* v) { *v = SL(c, f, S_Q0, k, j); }
static void cv_qstar(mro_ctx* c, int f, int64_t j, int k, double* v) {
  *v = c->lv[f].st[j] == LEAF ? SL(c, f, S_Q1, k, j) : SL(c, f, S_Q1REF, k, j);
}
static void cv_x2(mro_ctx* c, int f, int64_t j, int k, double* v) {
  *v = c->lv[f].st[j] == LEAF ? SL(c, f, S_X2, k, j)
                              : (2.0 * SL(c, f, S_Q1SW, k, j)) - SL(c, f, S_Q0, k, j);
}
static void cv_qh(mro_ctx* c, int f, int64_t j, int k, double* v) { *v = SL(c, f, S_QH, k, j); }
static void cv_qe(mro_ctx* c, int f, int64_t j, int k, double* v) { *v = SL(c, f, S_QE, k, j); }

static void cv_q1(mro_ctx* c, int f, int64_t j, int k, double* v) {
  *v = c->lv[f].st[j] == LEAF ? SL(c, f, S_Q1, k, j) : SL(c, f, S_Q1SW, k, j);
}

/* Global time step: internal stage states are the projections of the
 * children's stage states (the MR scheme of Sec. 2 at one time). */
static void project_stage(mro_ctx* c, int stage) {
  for (int lev = c->L - 1; lev >= c->l0; lev--) {
    level_t* LV = &c->lv[lev];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < LV->ncell; i++) {
      if (LV->st[i] != INTERNAL) continue;
      for (int k = 0; k < c->m; k++) {
        if (stage == 2) SL(c, lev, S_Q1SW, k, i) = project_children(c, lev, i, k, cv_q1);
        else SL(c, lev, S_QH, k, i) = project_children(c, lev, i, k, cv_qh);
      }
    }
  }
}

/* Alg. alg-LTS first loop: internal q^n = mean of children. */
static void project_q0(mro_ctx* c, int lev_hi, int lev_lo) {
  for (int lev = lev_hi; lev >= lev_lo; lev--) {
    level_t* LV = &c->lv[lev];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < LV->ncell; i++) {
      if (LV->st[i] != INTERNAL) continue;
      for (int k = 0; k < c->m; k++) SL(c, lev, S_Q0, k, i) = project_children(c, lev, i, k, cv_q0);
    }
  }
}

/* Internal nodes of level l_min - 1 (mid-step): the theta = 1/2 value by
 * projecting q^n of level l_min (Alg. alg-LTS) and the end value
 * -2 q^n - q* + 4 q_{1/2} of Sec. 4.3, with q* the refresh value.         */
static void case_b(mro_ctx* c, int lev) {
  level_t* LV = &c->lv[lev];
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < LV->ncell; i++) {
    if (LV->st[i] != INTERNAL) continue;
    for (int k = 0; k < c->m; k++) {
      double mid = project_children(c, lev, i, k, cv_q0);
      SL(c, lev, S_CBM, k, i) = mid;
      SL(c, lev, S_CBE, k, i) =
          ((-2.0 * SL(c, lev, S_Q0, k, i)) - SL(c, lev, S_Q1REF, k, i)) + (4.0 * mid);
    }
  }
}

/* Alg. refRK2: internal value at t + dt_l/2 as the mean of the children's
 * q*, then q* = 2 q(t + dt_l/2) - q^n (eq. refreshRk2).                     */
static void refresh2(mro_ctx* c) {
  for (int lev = c->L - 1; lev >= c->lmin; lev--) {
    level_t* LV = &c->lv[lev];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < LV->ncell; i++) {
      if (LV->st[i] != INTERNAL) continue;
      for (int k = 0; k < c->m; k++) {
        double h1 = project_children(c, lev, i, k, cv_qstar);
        SL(c, lev, S_H1, k, i) = h1;
        SL(c, lev, S_Q1REF, k, i) = (2.0 * h1) - SL(c, lev, S_Q0, k, i);
      }
    }
  }
}

/* Alg. projRK2: q*_l = mean over children of the extrapolations to
 * t^n + 2 dt_{l+1} (eq. projleaf for leaves, eq. projnode for nodes).      */
static void proj_rk2(mro_ctx* c, int lev) {
  level_t* LV = &c->lv[lev];
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < LV->ncell; i++) {
    if (LV->st[i] != INTERNAL) continue;
    for (int k = 0; k < c->m; k++) SL(c, lev, S_Q1SW, k, i) = project_children(c, lev, i, k, cv_x2);
  }
}

/* Alg. refRK22: q_{1/4} = mean of the children's q**, then
 * q_{3/4} = -13/2 q^n - 3/2 q* + 9 q_{1/4} (eq. ProjRK3equations1) and
 * q** = -11/2 q^n - 3/2 q* + 8 q_{1/4} (eq. ProjRK3equations2).            */
static void refresh3(mro_ctx* c) {
  for (int lev = c->L - 1; lev >= c->lmin; lev--) {
    level_t* LV = &c->lv[lev];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < LV->ncell; i++) {
      if (LV->st[i] != INTERNAL) continue;
      for (int k = 0; k < c->m; k++) {
        double q14 = project_children(c, lev, i, k, cv_qh);
        double q0 = SL(c, lev, S_Q0, k, i), qs = SL(c, lev, S_Q1REF, k, i);
        SL(c, lev, S_N14, k, i) = q14;
        SL(c, lev, S_N34, k, i) = ((-6.5 * q0) - (1.5 * qs)) + (9.0 * q14);
        SL(c, lev, S_QH, k, i) = ((-5.5 * q0) - (1.5 * qs)) + (8.0 * q14);
      }
    }
  }
}

/* Alg. projRK3: q** = mean of the children's stage-3 results, then the
 * end value q^n + 2 (q_{3/4} - q_{1/4}) (eq. rk3proj).                     */
static void proj_rk3(mro_ctx* c, int lev) {
  level_t* LV = &c->lv[lev];
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < LV->ncell; i++) {
    if (LV->st[i] != INTERNAL) continue;
    for (int k = 0; k < c->m; k++) {
      SL(c, lev, S_QH, k, i) = project_children(c, lev, i, k, cv_qe);
      SL(c, lev, S_QE, k, i) =
          SL(c, lev, S_Q0, k, i) + (2.0 * (SL(c, lev, S_N34, k, i) - SL(c, lev, S_N14, k, i)));
    }
  }
}

/* End of the steps of levels >= lnext: q^n <- stage-3 result, then the
 * conservative correction sigma (A_c - A_f)/dx on every refined face, faces
 * in the order x-, x+, y-, y+, z-, z+.                                      */
static void finalize(mro_ctx* c, int lnext) {
  int d = c->d, m = c->m;
  double sc = c->nsub == 1 ? 1.0 : (c->nsub == 2 ? 0.5 : 0.25);
  for (int lev = lnext; lev <= c->L; lev++) {
    level_t* LV = &c->lv[lev];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < LV->ncell; i++) {
      if (LV->st[i] != LEAF) continue;
      for (int k = 0; k < m; k++) SL(c, lev, S_Q0, k, i) = SL(c, lev, S_QE, k, i);
      if (!c->s.reflux || lev == c->L) continue;
      int x[3];
      ccoord(c, lev, i, x);
      for (int dir = 0; dir < d; dir++)
        for (int side = 0; side < 2; side++) {
          int nbx = map_nbr(c, dir, x[dir] + (side ? 1 : -1), LV->n);
          if (nbx < 0) continue;
          int y[3] = {x[0], x[1], x[2]};
          y[dir] = nbx;
          if (LV->st[cidx(c, lev, y)] != INTERNAL) continue;
          int f = 2 * dir + side;
          for (int k = 0; k < m; k++) {
            double af = 0.0;
            for (int b = 0; b < c->nsub; b++)
              af = (b == 0) ? REGF(c, lev, f, b, k, i) : (af + REGF(c, lev, f, b, k, i));
            af = af * sc;
            double D = (REGC(c, lev, f, k, i) - af) * c->invdx[lev][dir];
            SL(c, lev, S_Q0, k, i) = side ? SL(c, lev, S_Q0, k, i) + D : SL(c, lev, S_Q0, k, i) - D;
          }
        }
    }
    if (lev < c->L) {
      memset(LV->regc, 0, sizeof(double) * (size_t)(2 * d * m) * (size_t)LV->ncell);
      memset(LV->regf, 0, sizeof(double) * (size_t)(2 * d * c->nsub * m) * (size_t)LV->ncell);
    }
  }
}

/* ----------------------------------------------------------------------- */
/* remesh (Alg. AdaptiveMesh, Alg. waveletThres, and the remark that only
 * scales evolved in the current iteration may split or merge)               */

static double level_eps(const mro_ctx* c, int lam) {
  if (c->s.thresh) return ldexp(c->eps, c->d * (lam - c->L));
  return c->eps;
}

static uint64_t morton(int d, const int* x);

/* append one near-threshold decision (node i of level lev) */
static void near_record(mro_ctx* c, int lev, int64_t i) {
  int x[3];
  ccoord(c, lev, i, x);
  if (c->near_n == c->near_cap) {
    int64_t cap = c->near_cap ? 2 * c->near_cap : 64;
    int64_t* it = (int64_t*)realloc(c->near_iter, sizeof(int64_t) * (size_t)cap);
    if (it) c->near_iter = it;
    int32_t* lv = (int32_t*)realloc(c->near_lev, sizeof(int32_t) * (size_t)cap);
    if (lv) c->near_lev = lv;
    uint64_t* ky = (uint64_t*)realloc(c->near_key, sizeof(uint64_t) * (size_t)cap);
    if (ky) c->near_key = ky;
    if (!it || !lv || !ky) return;
    c->near_cap = cap;
  }
  c->near_iter[c->near_n] = c->iters;
  c->near_lev[c->near_n] = lev;
  c->near_key[c->near_n] = morton(c->d, x);
  c->near_n++;
}

/* max over children and components of |q_c - q~_c| / scale_k */
static double detail_norm(mro_ctx* c, int lev, int64_t i) {
  int x[3];
  ccoord(c, lev, i, x);
  double S[5 * 27];
  if (!gather3(c, lev, x, 1, q0_pick, S)) {
    fail(c, "detail stencil incomplete at level %d", lev);
    return 0.0;
  }
  double D = 0.0;
  for (int cb = 0; cb < (1 << c->d); cb++) {
    int y[3] = {2 * x[0] + (cb & 1), 2 * x[1] + ((cb >> 1) & 1), 2 * x[2] + ((cb >> 2) & 1)};
    int64_t j = cidx(c, lev + 1, y);
    for (int k = 0; k < c->m; k++) {
      double pred = predict1(c->d, S + 27 * k, cb);
      double det = fabs(SL(c, lev + 1, S_Q0, k, j) - pred) / c->s.detail_scale[k];
      if (det > D) D = det;
    }
  }
  return D;
}

/* all cells within infinity-distance r of x at level lev (wrapped when
 * periodic, clipped otherwise); calls fn for each, stops when it returns 0 */
typedef int (*nbr_fn)(mro_ctx* c, int lev, int64_t j, void* ud);
static int for_nbrs(mro_ctx* c, int lev, const int* x, int r, nbr_fn fn, void* ud) {
  int d = c->d, n = c->lv[lev].n;
  for (int oz = (d > 2 ? -r : 0); oz <= (d > 2 ? r : 0); oz++)
    for (int oy = (d > 1 ? -r : 0); oy <= (d > 1 ? r : 0); oy++)
      for (int ox = -r; ox <= r; ox++) {
        int off[3] = {ox, oy, oz}, y[3] = {0, 0, 0}, ok = 1;
        for (int a = 0; a < d; a++) {
          y[a] = map_nbr(c, a, x[a] + off[a], n);
          if (y[a] < 0) ok = 0;
        }
        if (!ok) continue;
        if (!fn(c, lev, cidx(c, lev, y), ud)) return 0;
      }
  return 1;
}

static int nb_exists_mark(mro_ctx* c, int lev, int64_t j, void* ud) {
  (void)ud;
  if (c->lv[lev].st[j] != ABSENT) c->lv[lev].W[j] = 1;
  return 1;
}

typedef struct { int la; int changed; } close_ud;

/* (G): every cell N within distance 2 of Y must exist: parent(N) in W */
static int nb_close(mro_ctx* c, int lev, int64_t j, void* ud) {
  close_ud* u = (close_ud*)ud;
  int y[3];
  ccoord(c, lev, j, y);
  int p[3] = {y[0] >> 1, y[1] >> 1, y[2] >> 1};
  int64_t pi = cidx(c, lev - 1, p);
  if (!c->lv[lev - 1].W[pi]) {
    c->lv[lev - 1].W[pi] = 1;
    u->changed = 1;
  }
  return 1;
}

/* does cell N (level lev) exist in the new tree? */
static int nb_valid(mro_ctx* c, int lev, int64_t j, void* ud) {
  close_ud* u = (close_ud*)ud;
  if (lev == c->l0) return 1;
  int y[3];
  ccoord(c, lev, j, y);
  int p[3] = {y[0] >> 1, y[1] >> 1, y[2] >> 1};
  int64_t pi = cidx(c, lev - 1, p);
  if (lev == u->la) return c->lv[lev - 1].st[pi] == INTERNAL; /* frozen */
  return c->lv[lev - 1].W[pi] != 0;
}

/* One remesh in which levels below la are frozen: the set of nodes at
 * levels <= la does not change, internal status may change at levels >= la.
 *   1. significant internal nodes P (detail > eps_{l(P)+1}) at [la, L-1];
 *      the flags of the frozen level la-1 are those of its last remesh
 *      (Sec. 4, adapting the grid during local time stepping: apart from
 *      splitting and merging only between scales at the same instant, the
 *      remesh is the multiresolution one, so a significant node of the
 *      frozen level still keeps its children refined);
 *   2. safety: existing nodes within distance 1 of P (space) and the
 *      children of P if they are below L (scale);
 *   3. closure: the least set W containing those seeds with the tree rule
 *      (parent of a member is a member, above la) and the grading rule
 *      (every cell within distance 2 of a member exists);
 *   4. pruning: the greatest subset of W in which every member still has
 *      both rules satisfied, with frozen existence at level la;
 *   5. W becomes the internal set; new nodes are predicted coarse to fine.
 * With eps = 0 every internal node counts as significant (no coarsening). */
static void remesh(mro_ctx* c, int la) {
  int L = c->L;
  if (la > L - 1) return;
  for (int lev = c->l0; lev <= L; lev++) {
    memset(c->lv[lev].W, 0, (size_t)c->lv[lev].ncell);
    if (lev >= la) memset(c->lv[lev].sig, 0, (size_t)c->lv[lev].ncell);
    memset(c->lv[lev].fresh, 0, (size_t)c->lv[lev].ncell);
  }
  /* 1. significance */
  for (int lev = la; lev <= L - 1; lev++) {
    level_t* LV = &c->lv[lev];
    double e = level_eps(c, lev + 1);
    int64_t near = 0;
#pragma omp parallel for schedule(static) reduction(+ : near)
    for (int64_t i = 0; i < LV->ncell; i++) {
      if (LV->st[i] != INTERNAL) continue;
      if (c->eps == 0.0) {
        LV->sig[i] = 1;
        continue;
      }
      double D = detail_norm(c, lev, i);
      LV->sig[i] = D > e;
      if (fabs(D - e) <= 1e-12 * e) {
        near++;
#pragma omp critical(near_list)
        near_record(c, lev, i);
      }
    }
    c->near_thr += near;
  }
  /* 2. seeds: significance, space safety and scale safety; of the frozen
   * level la-1 only its scale safety reaches the levels that may change */
  for (int lev = (la > c->l0 ? la - 1 : la); lev <= L - 1; lev++) {
    level_t* LV = &c->lv[lev];
    for (int64_t i = 0; i < LV->ncell; i++) {
      if (!LV->sig[i] || (lev < la && LV->st[i] != INTERNAL)) continue;
      int x[3];
      ccoord(c, lev, i, x);
      if (lev >= la) {
        LV->W[i] = 1;
        for_nbrs(c, lev, x, 1, nb_exists_mark, NULL);
      }
      if (lev + 1 <= L - 1) {
        for (int cb = 0; cb < (1 << c->d); cb++) {
          int y[3] = {2 * x[0] + (cb & 1), 2 * x[1] + ((cb >> 1) & 1), 2 * x[2] + ((cb >> 2) & 1)};
          c->lv[lev + 1].W[cidx(c, lev + 1, y)] = 1;
        }
      }
    }
  }
  /* 3. closure (least fixed point): repeat until nothing is added */
  close_ud u = {la, 1};
  while (u.changed) {
    u.changed = 0;
    for (int lev = L - 1; lev > la; lev--) {
      level_t* LV = &c->lv[lev];
      for (int64_t i = 0; i < LV->ncell; i++) {
        if (!LV->W[i]) continue;
        int x[3];
        ccoord(c, lev, i, x);
        for_nbrs(c, lev, x, 2, nb_close, &u); /* includes x itself: tree rule */
      }
    }
  }
  /* 4. pruning (greatest fixed point): repeat until nothing is removed */
  int changed = 1;
  while (changed) {
    changed = 0;
    for (int lev = la; lev <= L - 1; lev++) {
      level_t* LV = &c->lv[lev];
      for (int64_t i = 0; i < LV->ncell; i++) {
        if (!LV->W[i]) continue;
        int x[3];
        ccoord(c, lev, i, x);
        int ok = 1;
        if (lev > c->l0) {
          int p[3] = {x[0] >> 1, x[1] >> 1, x[2] >> 1};
          int64_t pi = cidx(c, lev - 1, p);
          ok = (lev == la) ? c->lv[lev - 1].st[pi] == INTERNAL : c->lv[lev - 1].W[pi] != 0;
        }
        if (ok) ok = for_nbrs(c, lev, x, 2, nb_valid, &u);
        if (!ok) {
          LV->W[i] = 0;
          changed = 1;
        }
      }
    }
  }
  /* 5. apply, coarse to fine; new nodes predicted from the new parent level */
  for (int lev = la; lev <= L; lev++) {
    level_t* LV = &c->lv[lev];
    for (int64_t i = 0; i < LV->ncell; i++) {
      int old = LV->st[i], nw;
      if (lev == la) {
        nw = old == ABSENT ? ABSENT : (LV->W[i] ? INTERNAL : LEAF);
      } else {
        int x[3];
        ccoord(c, lev, i, x);
        int p[3] = {x[0] >> 1, x[1] >> 1, x[2] >> 1};
        int pst = c->lv[lev - 1].st[cidx(c, lev - 1, p)];
        nw = pst == INTERNAL ? ((lev <= L - 1 && LV->W[i]) ? INTERNAL : LEAF) : ABSENT;
      }
      LV->st[i] = (uint8_t)nw;
      LV->fresh[i] = (old == ABSENT && nw != ABSENT);
    }
  }
  for (int lev = la + 1; lev <= L; lev++) {
    level_t* LV = &c->lv[lev];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < LV->ncell; i++) {
      if (!LV->fresh[i]) continue;
      int x[3];
      ccoord(c, lev, i, x);
      int p[3] = {x[0] >> 1, x[1] >> 1, x[2] >> 1};
      double S[5 * 27];
      if (!gather3(c, lev - 1, p, 1, q0_pick, S)) {
        fail(c, "prediction stencil of a new node incomplete at level %d", lev - 1);
        continue;
      }
      int cb = (x[0] & 1) | ((x[1] & 1) << 1) | ((x[2] & 1) << 2);
      for (int k = 0; k < c->m; k++) SL(c, lev, S_Q0, k, i) = predict1(c->d, S + 27 * k, cb);
    }
  }
}

/* ----------------------------------------------------------------------- */
/* the LT iteration (Alg. alg-LTS) and the macro step                        */

static int lmin_of(const mro_ctx* c, int64_t n) {
  for (int lev = c->l0; lev <= c->L; lev++)
    if (n % ((int64_t)1 << (c->L - lev)) == 0) return lev;
  return c->L;
}

/* One iteration of the MR scheme with a global time step (the comparison
 * method of the paper): all leaves advance by dt, remesh every step. */
static void mr_iteration(mro_ctx* c) {
  int L = c->L;
  c->lmin = c->l0;
  project_q0(c, L - 1, c->l0);
  if (c->s.remesh) {
    remesh(c, c->l0);
    project_q0(c, L - 1, c->l0);
  }
  for (int lev = c->l0; lev <= L; lev++) {
    int64_t nl = 0;
    for (int64_t i = 0; i < c->lv[lev].ncell; i++) nl += c->lv[lev].st[i] == LEAF;
    c->leaf_updates += nl;
  }
  for (int lev = c->l0; lev <= L; lev++) stage_level(c, lev, 1);
  project_stage(c, 2);
  for (int lev = c->l0; lev <= L; lev++) stage_level(c, lev, 2);
  if (c->s.rk == 3) {
    project_stage(c, 3);
    for (int lev = c->l0; lev <= L; lev++) stage_level(c, lev, 3);
  }
  finalize(c, c->l0);
  c->iters++;
}

static void lt_iteration(mro_ctx* c, int64_t n, int64_t N) {
  int L = c->L;
  if (!c->s.lt) {
    (void)n;
    (void)N;
    mr_iteration(c);
    return;
  }
  int lmin = lmin_of(c, n);
  c->lmin = lmin;
  project_q0(c, L - 1, lmin);
  if (c->s.remesh && lmin <= L - 1) {
    remesh(c, lmin);
    project_q0(c, L - 1, lmin);
  }
  if (lmin > c->l0) case_b(c, lmin - 1);
  for (int lev = lmin; lev <= L; lev++) {
    int64_t nl = 0;
    for (int64_t i = 0; i < c->lv[lev].ncell; i++) nl += c->lv[lev].st[i] == LEAF;
    c->leaf_updates += nl;
  }
  for (int lev = lmin; lev <= L; lev++) stage_level(c, lev, 1);
  refresh2(c);
  for (int lev = L; lev >= lmin; lev--) {
    if (lev < L) proj_rk2(c, lev);
    stage_level(c, lev, 2);
  }
  if (c->s.rk == 2) {
    /* RK2: the step ends with stage 2 */
    int lnext2 = (n + 1 == N) ? c->l0 : lmin_of(c, n + 1);
    finalize(c, lnext2);
    c->iters++;
    return;
  }
  refresh3(c);
  for (int lev = L; lev >= lmin; lev--) {
    if (lev < L) proj_rk3(c, lev);
    stage_level(c, lev, 3);
  }
  int lnext = (n + 1 == N) ? c->l0 : lmin_of(c, n + 1);
  finalize(c, lnext);
  c->iters++;
}

/* ----------------------------------------------------------------------- */
/* public interface                                                          */

static void free_levels(mro_ctx* c) {
  for (int lev = 0; lev <= MRO_MAXLEV; lev++) {
    level_t* LV = &c->lv[lev];
    free(LV->st);
    for (int s = 0; s < NSLOT; s++) free(LV->slot[s]);
    free(LV->regc);
    free(LV->regf);
    free(LV->W);
    free(LV->sig);
    free(LV->fresh);
    memset(LV, 0, sizeof *LV);
  }
}

int mro_init(int dim, int L, double eps, const mro_scheme* s, mro_ctx** out) {
  if (!out || !s) return MRO_EINVAL;
  *out = NULL;
  if (dim < 1 || dim > 3 || !(eps >= 0.0)) return MRO_EINVAL;
  if (s->l0 < 2 || L < s->l0 || L > MRO_MAXLEV || (int64_t)dim * L > 40) return MRO_EINVAL;
  if ((s->rk != 2 && s->rk != 3) || (s->lt != 0 && s->lt != 1) || s->pde < 0 || s->pde > MRO_PDE_FLAMEBALL)
    return MRO_EINVAL;
  int flame = s->pde == MRO_PDE_FLAME || s->pde == MRO_PDE_FLAMEBALL;
  if (flame && !(s->ze > 0.0 && s->tau > 0.0 && s->tau < 1.0 && s->lewis > 0.0 && s->kappa >= 0.0))
    return MRO_EINVAL;
  if (s->flame_speed < -1 || s->flame_speed > 1 || (s->flame_speed != 0 && !flame)) return MRO_EINVAL;
  if (L - s->l0 > 20) return MRO_EINVAL;
  for (int a = 0; a < dim; a++) {
    if ((s->bc[a][0] == MRO_BC_PERIODIC) != (s->bc[a][1] == MRO_BC_PERIODIC)) return MRO_EINVAL;
    for (int side = 0; side < 2; side++) {
      if (s->bc[a][side] < MRO_BC_PERIODIC || s->bc[a][side] > MRO_BC_DIRICHLET) return MRO_EINVAL;
      /* a homogeneous Dirichlet value is meaningful for a scalar field only */
      if (s->bc[a][side] == MRO_BC_DIRICHLET && s->pde == MRO_PDE_EULER) return MRO_EINVAL;
    }
    if (!(s->hi[a] > s->lo[a])) return MRO_EINVAL;
  }
  mro_ctx* c = (mro_ctx*)calloc(1, sizeof *c);
  if (!c) return MRO_ENOMEM;
  c->d = dim;
  c->L = L;
  c->l0 = s->l0;
  c->s = *s;
  c->eps = eps;
  c->m = s->pde == MRO_PDE_EULER ? dim + 2 : (s->pde == MRO_PDE_FLAMEBALL ? 2 : 1);
  for (int a = 0; a < 3; a++) c->vel[a] = s->adv_vel[a];
  c->nsub = 1 << (dim - 1);
  for (int k = 0; k < c->m; k++)
    if (!(c->s.detail_scale[k] > 0.0)) c->s.detail_scale[k] = 1.0;
  for (int lev = c->l0; lev <= L; lev++) {
    level_t* LV = &c->lv[lev];
    LV->n = 1 << lev;
    LV->ncell = (int64_t)1 << (dim * lev);
    size_t nc = (size_t)LV->ncell;
    LV->st = (uint8_t*)calloc(nc, 1);
    LV->W = (uint8_t*)calloc(nc, 1);
    LV->sig = (uint8_t*)calloc(nc, 1);
    LV->fresh = (uint8_t*)calloc(nc, 1);
    int ok = LV->st && LV->W && LV->sig && LV->fresh;
    for (int sl = 0; sl < NSLOT; sl++) {
      LV->slot[sl] = (double*)calloc(nc * (size_t)c->m, sizeof(double));
      ok = ok && LV->slot[sl];
    }
    if (lev < L) {
      LV->regc = (double*)calloc(nc * (size_t)(2 * dim * c->m), sizeof(double));
      LV->regf = (double*)calloc(nc * (size_t)(2 * dim * c->nsub * c->m), sizeof(double));
      ok = ok && LV->regc && LV->regf;
    }
    if (!ok) {
      free_levels(c);
      free(c);
      return MRO_ENOMEM;
    }
    double v = 1.0;
    for (int a = 0; a < 3; a++) {
      if (a < dim) {
        c->dx[lev][a] = (s->hi[a] - s->lo[a]) / (double)LV->n;
        c->invdx[lev][a] = 1.0 / c->dx[lev][a];
        v = v * c->dx[lev][a];
      } else {
        c->dx[lev][a] = 1.0;
        c->invdx[lev][a] = 1.0;
      }
    }
    c->vol[lev] = v;
  }
  *out = c;
  return MRO_OK;
}

void mro_destroy(mro_ctx* c) {
  if (!c) return;
  free_levels(c);
  free(c->near_iter);
  free(c->near_lev);
  free(c->near_key);
  free(c);
}

typedef struct { int64_t it; int32_t lev; uint64_t key; } near_t;
static int near_cmp(const void* a, const void* b) {
  const near_t* x = (const near_t*)a;
  const near_t* y = (const near_t*)b;
  if (x->it != y->it) return x->it < y->it ? -1 : 1;
  if (x->lev != y->lev) return x->lev < y->lev ? -1 : 1;
  return x->key < y->key ? -1 : (x->key > y->key ? 1 : 0);
}

int mro_near_threshold(mro_ctx* c, int64_t* iter, int32_t* level, uint64_t* key, int64_t cap, int64_t* n) {
  if (!c || !n) return MRO_EINVAL;
  *n = c->near_n;
  if (!iter || !level || !key) return MRO_OK;
  if (cap < c->near_n) return MRO_EINVAL;
  near_t* v = (near_t*)malloc(sizeof(near_t) * (size_t)(c->near_n + 1));
  if (!v) return MRO_ENOMEM;
  for (int64_t j = 0; j < c->near_n; j++) {
    v[j].it = c->near_iter[j];
    v[j].lev = c->near_lev[j];
    v[j].key = c->near_key[j];
  }
  qsort(v, (size_t)c->near_n, sizeof(near_t), near_cmp);
  for (int64_t j = 0; j < c->near_n; j++) {
    iter[j] = v[j].it;
    level[j] = v[j].lev;
    key[j] = v[j].key;
  }
  free(v);
  return MRO_OK;
}

int mro_ncomp(const mro_ctx* c) { return c ? c->m : 0; }

int mro_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

const char* mro_last_error(const mro_ctx* c) { return c ? c->err : "null context"; }

static int finish(mro_ctx* c) {
  if (c->bad) return MRO_ESTATE;
  if (c->nonfinite) return MRO_ENONFINITE;
  return MRO_OK;
}

int mro_adapt(mro_ctx* c) {
  if (!c) return MRO_EINVAL;
  project_q0(c, c->L - 1, c->l0);
  c->lmin = c->l0;
  remesh(c, c->l0);
  project_q0(c, c->L - 1, c->l0);
  return finish(c);
}

int mro_load_finest(mro_ctx* c, const double* q0) {
  if (!c || !q0) return MRO_EINVAL;
  int L = c->L;
  for (int lev = c->l0; lev <= L; lev++) {
    memset(c->lv[lev].st, lev == L ? LEAF : INTERNAL, (size_t)c->lv[lev].ncell);
    if (lev < L) {
      memset(c->lv[lev].regc, 0, sizeof(double) * (size_t)(2 * c->d * c->m) * (size_t)c->lv[lev].ncell);
      memset(c->lv[lev].regf, 0, sizeof(double) * (size_t)(2 * c->d * c->nsub * c->m) * (size_t)c->lv[lev].ncell);
    }
  }
  memcpy(c->lv[L].slot[S_Q0], q0, sizeof(double) * (size_t)c->m * (size_t)c->lv[L].ncell);
  c->t = 0.0;
  /* counters and the near-threshold list start again with the new state */
  c->near_n = 0;
  c->iters = 0;
  c->leaf_updates = 0;
  c->near_thr = 0;
  c->nonfinite = 0;
  c->bad = 0;
  c->err[0] = 0;
  return mro_adapt(c);
}

int mro_lt_step(mro_ctx* c, double dt) {
  if (!c || !(dt > 0.0) || !isfinite(dt)) return MRO_EINVAL;
  if (c->bad || c->nonfinite) return MRO_ESTATE;
  int64_t N = (int64_t)1 << (c->L - c->l0);
  c->dt = dt;
  set_velocity(c);
  for (int64_t n = 0; n < N; n++) {
    lt_iteration(c, n, N);
    if (c->bad) break;
  }
  c->t = c->t + (double)N * dt;
  return finish(c);
}

int mro_reconstruct(mro_ctx* c, double* q_out) {
  if (!c || !q_out) return MRO_EINVAL;
  project_q0(c, c->L - 1, c->l0);
  int m = c->m, d = c->d, L = c->L;
  /* dense values per level, coarse to fine: predicted where absent */
  double* prev = NULL;
  for (int lev = c->l0; lev <= L; lev++) {
    level_t* LV = &c->lv[lev];
    double* cur = (double*)malloc(sizeof(double) * (size_t)m * (size_t)LV->ncell);
    if (!cur) {
      free(prev);
      return MRO_ENOMEM;
    }
    for (int64_t i = 0; i < LV->ncell; i++) {
      if (LV->st[i] != ABSENT || lev == c->l0) {
        for (int k = 0; k < m; k++) cur[(int64_t)k * LV->ncell + i] = SL(c, lev, S_Q0, k, i);
        continue;
      }
      int x[3];
      ccoord(c, lev, i, x);
      int p[3] = {x[0] >> 1, x[1] >> 1, x[2] >> 1};
      int np = c->lv[lev - 1].n;
      double S[27];
      for (int k = 0; k < m; k++) {
        for (int s = 0; s < 27; s++) S[s] = 0.0;
        for (int oz = (d > 2 ? -1 : 0); oz <= (d > 2 ? 1 : 0); oz++)
          for (int oy = (d > 1 ? -1 : 0); oy <= (d > 1 ? 1 : 0); oy++)
            for (int ox = -1; ox <= 1; ox++) {
              int off[3] = {ox, oy, oz}, y[3] = {0, 0, 0}, flip = 0;
              for (int a = 0; a < d; a++) {
                y[a] = map_stencil(c, a, p[a] + off[a], np);
                flip ^= stencil_flip(c, a, p[a] + off[a], np);
              }
              const double v = prev[(int64_t)k * c->lv[lev - 1].ncell + cidx(c, lev - 1, y)];
              S[(ox + 1) + 3 * (oy + 1) + 9 * (oz + 1)] = flip ? -v : v;
            }
        int cb = (x[0] & 1) | ((x[1] & 1) << 1) | ((x[2] & 1) << 2);
        cur[(int64_t)k * LV->ncell + i] = predict1(d, S, cb);
      }
    }
    free(prev);
    prev = cur;
  }
  memcpy(q_out, prev, sizeof(double) * (size_t)m * (size_t)c->lv[L].ncell);
  free(prev);
  return finish(c);
}

int mro_flame_speed(mro_ctx* c, double* vf) {
  if (!c || !vf) return MRO_EINVAL;
  if (c->s.pde != MRO_PDE_FLAME && c->s.pde != MRO_PDE_FLAMEBALL) return MRO_EINVAL;
  *vf = flame_speed(c);
  return MRO_OK;
}

int mro_max_wavespeed(mro_ctx* c, double* out) {
  if (!c || !out) return MRO_EINVAL;
  set_velocity(c);
  double mx = 0.0;
  int d = c->d, m = c->m;
  for (int lev = c->l0; lev <= c->L; lev++) {
    level_t* LV = &c->lv[lev];
    for (int64_t i = 0; i < LV->ncell; i++) {
      if (LV->st[i] != LEAF) continue;
      double q[5], v = 0.0;
      for (int k = 0; k < m; k++) q[k] = SL(c, lev, S_Q0, k, i);
      if (c->s.pde == MRO_PDE_BURGERS) {
        /* f_i(u) = u^2/2 in every direction: sum_i |f_i'(u)| */
        for (int j = 0; j < d; j++) v = (j == 0) ? fabs(q[0]) : (v + fabs(q[0]));
      } else if (c->s.pde == MRO_PDE_EULER) {
        double w[5];
        euler_prim(d, c->s.gamma - 1.0, q, w);
        double a = sqrt((c->s.gamma * w[d + 1]) / w[0]);
        for (int j = 0; j < d; j++) v = (j == 0) ? (fabs(w[1]) + a) : (v + (fabs(w[1 + j]) + a));
      } else if (c->s.pde == MRO_PDE_ADVECTION) {
        for (int j = 0; j < d; j++) v = v + fabs(c->s.adv_vel[j]);
      } else if (c->s.pde == MRO_PDE_FLAME || c->s.pde == MRO_PDE_FLAMEBALL) {
        for (int j = 0; j < d; j++) v = v + fabs(c->vel[j]);
      }
      if (v > mx) mx = v;
    }
  }
  *out = mx;
  return MRO_OK;
}

typedef struct { uint64_t key; int64_t idx; } kv_t;
static int kv_cmp(const void* a, const void* b) {
  uint64_t x = ((const kv_t*)a)->key, y = ((const kv_t*)b)->key;
  return x < y ? -1 : (x > y ? 1 : 0);
}

int mro_get_leaves(mro_ctx* c, uint64_t* keys, double* q, int64_t cap, int64_t* n) {
  if (!c || !n) return MRO_EINVAL;
  int64_t tot = 0;
  for (int lev = c->l0; lev <= c->L; lev++)
    for (int64_t i = 0; i < c->lv[lev].ncell; i++) tot += c->lv[lev].st[i] == LEAF;
  *n = tot;
  if (!keys || !q) return MRO_OK;
  if (cap < tot) return MRO_EINVAL;
  kv_t* kv = (kv_t*)malloc(sizeof(kv_t) * (size_t)(tot > 0 ? tot : 1));
  if (!kv) return MRO_ENOMEM;
  int64_t j = 0;
  for (int lev = c->l0; lev <= c->L; lev++) {
    int64_t j0 = j;
    for (int64_t i = 0; i < c->lv[lev].ncell; i++) {
      if (c->lv[lev].st[i] != LEAF) continue;
      int x[3];
      ccoord(c, lev, i, x);
      kv[j].key = ((uint64_t)lev << 56) | morton(c->d, x);
      kv[j].idx = i;
      j++;
    }
    qsort(kv + j0, (size_t)(j - j0), sizeof(kv_t), kv_cmp);
  }
  for (int64_t r = 0; r < tot; r++) {
    int lev = (int)(kv[r].key >> 56);
    keys[r] = kv[r].key;
    for (int k = 0; k < c->m; k++) q[(int64_t)k * tot + r] = SL(c, lev, S_Q0, k, kv[r].idx);
  }
  free(kv);
  return MRO_OK;
}

static int g_check(mro_ctx* c, int lev, int64_t j, void* ud) {
  (void)ud;
  return c->lv[lev].st[j] != ABSENT;
}

int mro_set_leaves(mro_ctx* c, const uint64_t* keys, const double* q, int64_t n, double t) {
  if (!c || (n > 0 && (!keys || !q))) return MRO_EINVAL;
  int L = c->L, d = c->d;
  for (int lev = c->l0; lev <= L; lev++) {
    memset(c->lv[lev].st, ABSENT, (size_t)c->lv[lev].ncell);
    if (lev < L) {
      memset(c->lv[lev].regc, 0, sizeof(double) * (size_t)(2 * d * c->m) * (size_t)c->lv[lev].ncell);
      memset(c->lv[lev].regf, 0, sizeof(double) * (size_t)(2 * d * c->nsub * c->m) * (size_t)c->lv[lev].ncell);
    }
  }
  for (int64_t r = 0; r < n; r++) {
    int lev = (int)(keys[r] >> 56);
    uint64_t mk = keys[r] & (((uint64_t)1 << 56) - 1);
    if (lev < c->l0 || lev > L || (mk >> (d * lev)) != 0) return MRO_EINVAL;
    int x[3];
    demorton(d, mk, x);
    int64_t i = cidx(c, lev, x);
    if (c->lv[lev].st[i] != ABSENT) return MRO_EINVAL;
    c->lv[lev].st[i] = LEAF;
    for (int k = 0; k < c->m; k++) SL(c, lev, S_Q0, k, i) = q[(int64_t)k * n + r];
  }
  for (int lev = L; lev > c->l0; lev--)
    for (int64_t i = 0; i < c->lv[lev].ncell; i++) {
      if (c->lv[lev].st[i] == ABSENT) continue;
      int x[3];
      ccoord(c, lev, i, x);
      int p[3] = {x[0] >> 1, x[1] >> 1, x[2] >> 1};
      int64_t pi = cidx(c, lev - 1, p);
      if (c->lv[lev - 1].st[pi] == LEAF) return MRO_EINVAL;
      c->lv[lev - 1].st[pi] = INTERNAL;
    }
  /* completeness: level l0 covered, internal nodes have every child,
   * grading radius 2 around every internal node                           */
  for (int64_t i = 0; i < c->lv[c->l0].ncell; i++)
    if (c->lv[c->l0].st[i] == ABSENT) return MRO_EINVAL;
  for (int lev = c->l0; lev < L; lev++)
    for (int64_t i = 0; i < c->lv[lev].ncell; i++) {
      if (c->lv[lev].st[i] != INTERNAL) continue;
      int x[3];
      ccoord(c, lev, i, x);
      for (int cb = 0; cb < (1 << d); cb++) {
        int y[3] = {2 * x[0] + (cb & 1), 2 * x[1] + ((cb >> 1) & 1), 2 * x[2] + ((cb >> 2) & 1)};
        if (c->lv[lev + 1].st[cidx(c, lev + 1, y)] == ABSENT) return MRO_EINVAL;
      }
      if (!for_nbrs(c, lev, x, 2, g_check, NULL)) return MRO_EINVAL;
    }
  project_q0(c, L - 1, c->l0);
  c->t = t;
  c->near_n = 0;
  c->iters = 0;
  c->leaf_updates = 0;
  c->near_thr = 0;
  c->nonfinite = 0;
  c->bad = 0;
  c->err[0] = 0;
  return MRO_OK;
}

int mro_stats(mro_ctx* c, mro_stats_t* out) {
  if (!c || !out) return MRO_EINVAL;
  memset(out, 0, sizeof *out);
  out->t = c->t;
  out->leaf_updates = c->leaf_updates;
  out->near_threshold = c->near_thr;
  out->iterations = c->iters;
  for (int lev = c->l0; lev <= c->L; lev++) {
    level_t* LV = &c->lv[lev];
    for (int64_t i = 0; i < LV->ncell; i++) {
      if (LV->st[i] != LEAF) continue;
      out->leaves[lev]++;
      for (int k = 0; k < c->m; k++) out->mass[k] = out->mass[k] + (c->vol[lev] * SL(c, lev, S_Q0, k, i));
    }
  }
  return MRO_OK;
}

int mro_get_level(mro_ctx* c, int level, uint8_t* status, double* q0) {
  if (!c || level < c->l0 || level > c->L) return MRO_EINVAL;
  level_t* LV = &c->lv[level];
  if (status) memcpy(status, LV->st, (size_t)LV->ncell);
  if (q0) memcpy(q0, LV->slot[S_Q0], sizeof(double) * (size_t)c->m * (size_t)LV->ncell);
  return MRO_OK;
}

int mro_remesh(mro_ctx* c, int la) {
  if (!c || la < c->l0 || la > c->L) return MRO_EINVAL;
  project_q0(c, c->L - 1, la);
  remesh(c, la);
  project_q0(c, c->L - 1, la);
  return finish(c);
}

int mro_predict(int dim, int m, const double* stencil, double* children) {
  if (dim < 1 || dim > 3 || m < 1 || !stencil || !children) return MRO_EINVAL;
  for (int k = 0; k < m; k++)
    for (int cb = 0; cb < (1 << dim); cb++) children[cb * m + k] = predict1(dim, stencil + 27 * k, cb);
  return MRO_OK;
}

int mro_project(int dim, int m, const double* children, double* parent) {
  if (dim < 1 || dim > 3 || m < 1 || !children || !parent) return MRO_EINVAL;
  for (int k = 0; k < m; k++) {
    double s = 0.0;
    for (int cb = 0; cb < (1 << dim); cb++) s = (cb == 0) ? children[cb * m + k] : (s + children[cb * m + k]);
    parent[k] = s * proj_scale(dim);
  }
  return MRO_OK;
}

int mro_face_flux(mro_ctx* c, int level, int dir, const double* cells, double* F) {
  if (!c || level < c->l0 || level > c->L || dir < 0 || dir >= c->d || !cells || !F) return MRO_EINVAL;
  face_flux(c, level, dir, cells, F);
  return MRO_OK;
}

int mro_details(mro_ctx* c, int level, double* D) {
  if (!c || level < c->l0 || level >= c->L || !D) return MRO_EINVAL;
  level_t* LV = &c->lv[level];
  for (int64_t i = 0; i < LV->ncell; i++) D[i] = LV->st[i] == INTERNAL ? detail_norm(c, level, i) : -1.0;
  return finish(c);
}
