/* mro.h -- C interface of the CPU oracle for one MRLT/NERK macro step.
 *
 * TEST INFRASTRUCTURE ONLY.  The oracle is a plain, slow, FP64 CPU
 * implementation of the space-time adaptive multiresolution finite-volume
 * method with local time stepping and NERK synchronisation (Lopes, Domingues,
 * Mendes, Schneider, arXiv:1905.08717).  It exists to check the HIP path; only
 * the tests, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header or table with the HIP library.
 *
 * Data model: dense per-level arrays, row-major cell index x + n*(y + n*z)
 * with n = 2^level, status ABSENT / LEAF / INTERNAL per cell, one array per
 * time slot (Q0, Q1, H1, N14, N34, QH, QE, X2, Q1ref, Q1sw, CBm, CBe), each
 * field-major [m][ncell].
 */
#ifndef MRO_H
#define MRO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { MRO_OK = 0, MRO_EINVAL = -1, MRO_ENOMEM = -2, MRO_ESTATE = -4,
       MRO_ENONFINITE = -5 };

enum { MRO_PDE_ADVECTION = 0, MRO_PDE_BURGERS = 1, MRO_PDE_NAGUMO = 2,
       MRO_PDE_EULER = 3, MRO_PDE_LINEAR = 4,
       MRO_PDE_FLAME = 5,      /* Sec. 5 one-dimensional flame: T, Y = 1 - T */
       MRO_PDE_FLAMEBALL = 6   /* Sec. 5 three-dimensional flame ball: T, Y */ };

enum { MRO_BC_PERIODIC = 0, MRO_BC_NEUMANN = 1, MRO_BC_DIRICHLET = 2 /* homogeneous, scalar PDEs */ };

#define MRO_MAXLEV 30

typedef struct {
  int32_t pde;        /* MRO_PDE_* */
  int32_t rk;         /* 3 (MRLT/NERK3) or 2 (MRLT/NERK2) */
  int32_t lt;         /* 1 local time stepping (MRLT), 0 global step (MR) */
  int32_t l0;         /* coarsest level */
  int32_t recon;      /* 0 first order, 1 MUSCL-minmod, 2 centred (advection) */
  int32_t thresh;     /* 1 level-dependent eps_l = 2^{d(l-L)} eps, 0 fixed */
  int32_t reflux;     /* 1 conservative flux accumulation, 0 off */
  int32_t remesh;     /* 1 remesh every iteration, 0 frozen tree */
  int32_t bc[3][2];   /* per dimension, low and high side */
  double lo[3], hi[3];
  double nu, k_react, a_react, gamma, adv_vel[3];
  double detail_scale[5];
  /* reaction-diffusion flames (Sec. 5): Zeldovich number, temperature
   * ratio tau, Lewis number, radiation coefficient kappa.  flame_speed 0:
   * the advection velocity is adv_vel; +1 / -1: it is +v_f / -v_f along
   * axis 0 with v_f the integral of the reaction rate over the domain (per
   * unit cross-section), taken at the start of every macro step.          */
  double ze, tau, lewis, kappa;
  int32_t flame_speed;
} mro_scheme;

typedef struct {
  double t;
  int64_t leaves[MRO_MAXLEV + 1];
  int64_t leaf_updates;   /* cumulative: one per leaf per full RK step */
  int64_t near_threshold; /* cumulative count of near-threshold decisions */
  int64_t iterations;     /* cumulative fine iterations */
  double mass[5];         /* sum over leaves of |cell| * q, per component */
} mro_stats_t;

typedef struct mro_ctx mro_ctx;

int  mro_init(int dim, int L, double eps, const mro_scheme* s, mro_ctx** out);
void mro_destroy(mro_ctx* c);
int  mro_ncomp(const mro_ctx* c);
int  mro_num_threads(void);                               /* OpenMP threads used */
int  mro_load_finest(mro_ctx* c, const double* q0);   /* [m][2^{dL}] x fastest */
int  mro_adapt(mro_ctx* c);
int  mro_lt_step(mro_ctx* c, double dt_L);
int  mro_reconstruct(mro_ctx* c, double* q_out);      /* [m][2^{dL}] x fastest */
int  mro_max_wavespeed(mro_ctx* c, double* out);
int  mro_flame_speed(mro_ctx* c, double* vf);         /* integral of omega */
int  mro_get_leaves(mro_ctx* c, uint64_t* keys, double* q, int64_t cap, int64_t* n);
int  mro_set_leaves(mro_ctx* c, const uint64_t* keys, const double* q, int64_t n, double t);
int  mro_stats(mro_ctx* c, mro_stats_t* out);
const char* mro_last_error(const mro_ctx* c);

/* Test hooks. */
int  mro_get_level(mro_ctx* c, int level, uint8_t* status, double* q0); /* row-major */
int  mro_remesh(mro_ctx* c, int la);                 /* one remesh with frozen levels < la */
int  mro_predict(int dim, int m, const double* stencil, double* children);
int  mro_project(int dim, int m, const double* children, double* parent);
int  mro_face_flux(mro_ctx* c, int level, int dir, const double* cells, double* F);
int  mro_details(mro_ctx* c, int level, double* D);  /* detail norm per internal node, -1 else */
/* near-threshold decisions since the last load / set_leaves, sorted by
 * (iteration, level, key): iteration = fine iterations completed before the
 * remesh that took the decision; with iter == NULL only *n is set */
int  mro_near_threshold(mro_ctx* c, int64_t* iter, int32_t* level, uint64_t* key, int64_t cap, int64_t* n);

#ifdef __cplusplus
}
#endif
#endif
