/* mrlt.h -- C ABI of the MI355X (gfx950) library for one local-time-stepping
 * macro step of the space-time adaptive multiresolution finite-volume method
 * with NERK synchronisation (MRLT/NERK3), arXiv:1905.08717.
 *
 * Problem (Sec. 2, eq. pde): dQ/dt = -div F(Q, grad Q) + S(Q) on a box in
 * d = 1, 2, 3 dimensions, discretised by cell averages on a dynamic graded
 * dyadic tree of levels l0..L (Sec. 2), advanced by compact RK3 (Sec. 3)
 * with level-dependent steps dt_l = 2^{L-l} dt_L (Sec. 4, eq. dt) and NERK
 * synchronisation between levels (Sec. 4.1-4.3, appendix algorithms).
 *
 * Conventions for every call:
 *  - Return value: mr_status, 0 = MR_OK, negative = error.  No exception or
 *    abort crosses the interface; mr_last_error() describes the last error.
 *  - All floating point data are FP64.
 *  - "device" pointers are HIP device memory (e.g. a torch tensor's
 *    data_ptr()); "host" pointers are ordinary host memory.
 *  - The context owns all of its device memory; input buffers are borrowed
 *    (copied in), output buffers are allocated by the caller.
 *  - Work is queued on the stream given to mr_set_stream / mr_load_finest
 *    (default: a non-blocking stream the context creates; mr_init returns
 *    with its zero fills and uploads complete).  mr_lt_step, mr_reconstruct,
 *    mr_max_wavespeed, mr_get_leaves, mr_stats synchronise that stream
 *    before returning.
 *  - One host thread per context at a time.
 *  - A batch context holds n_inst independent solves with the same dim, L,
 *    scheme and per-instance eps; every kernel launch advances all of them.
 *    The single-solve calls act on a batch of one.
 *  - Errors are sticky: after MR_ENONFINITE or MR_ESTATE the context refuses
 *    mr_lt_step until mr_load_finest or mr_set_leaves resets it.
 *  - Environment, read by mr_init / mr_init_batch: MRLT_CHECK (set: the
 *    kernels also verify the tree invariants the grading guarantees --
 *    stencil cells exist, the coarse side of a refined face is a leaf --
 *    and report a violation as MR_ESTATE; results are the same);
 *    MRLT_NO_GRAPH (set: launch every kernel of a macro step eagerly
 *    instead of replaying the captured graph).
 */
#ifndef MRLT_H
#define MRLT_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mr_ctx mr_ctx;

typedef enum {
  MR_OK = 0,
  MR_EINVAL = -1,      /* bad argument */
  MR_ENOMEM = -2,      /* device allocation failed */
  MR_EDEVICE = -3,     /* HIP runtime error */
  MR_ESTATE = -4,      /* tree invariant violated or context in error state */
  MR_ENONFINITE = -5,  /* a cell average became NaN / Inf */
  MR_ECAPACITY = -6    /* output buffer too small */
} mr_status;

enum { MR_PDE_ADVECTION = 0, MR_PDE_BURGERS = 1, MR_PDE_NAGUMO = 2, MR_PDE_EULER = 3, MR_PDE_LINEAR = 4,
       MR_PDE_FLAME = 5, MR_PDE_FLAMEBALL = 6 };
/* Boundary conditions per side of an axis: periodic wrap (both sides or
 * neither); homogeneous Neumann, stencil cells outside mirror evenly
 * (q_{-1} = q_0, q_{-2} = q_1); homogeneous Dirichlet (Q = 0 on the
 * boundary: the paper's 2D Burgers problem and the 1D flame's T(15) = 0,
 * Sec. 5), mirror cells enter with the opposite sign (q_{-1} = -q_0,
 * q_{-2} = -q_1); every field, not for the Euler system.                  */
enum { MR_BC_PERIODIC = 0, MR_BC_NEUMANN = 1, MR_BC_DIRICHLET = 2 };

#define MR_MAXLEV 24

/* Scheme description (Sec. 2 and Sec. 5 of the paper for the PDEs):
 *  pde     advection (m=1, flux a.q), Burgers (m=1, u^2/2 - nu u_x, exact
 *          Godunov advective flux), Nagumo (m=1, -nu grad u, source
 *          k u (1-u)(u-a)), Euler (m=d+2: rho, rho u_i, E; AUSM+), linear
 *          (m=1, -nu grad u, source k u); the flames of Sec. 5: flame (m=1:
 *          T; T_t + v.grad T = Lap T + omega(T), omega = Ze^2/2 (1-T)
 *          exp(Ze (1-T) / (tau (1-T) - 1))), flameball (m=2: T, Y;
 *          T_t + v.grad T = Lap T + omega - s(T), Y_t + v.grad Y = Lap Y / Le
 *          - omega, omega = Ze^2/(2 Le) Y exp(Ze (T-1) / (1 + tau (T-1))),
 *          s = kappa ((T + 1/tau - 1)^4 - (1/tau - 1)^4)); advective flux:
 *          upwind value of the reconstructed face states
 *  rk      3 (MRLT/NERK3: compact RK3 with NERK partials at theta 1/4, 3/4)
 *          or 2 (MRLT/NERK2: compact RK2 with the NERK theta = 1/2 value), Sec. 3
 *  lt      1: local time stepping (MRLT, Sec. 4); 0: one global step dt_L
 *          for every level (the MR comparison scheme)
 *  l0      coarsest level, >= 2
 *  recon   0 first order, 1 MUSCL-minmod, 2 centred (advection only)
 *  thresh  1: eps_l = 2^{d(l-L)} eps for details of level l, 0: fixed eps
 *  reflux  1: conservative correction of coarse leaves at level interfaces
 *  remesh  1: remesh the evolved levels every iteration, 0: frozen tree
 *  bc      per dimension, low/high side: MR_BC_PERIODIC, MR_BC_NEUMANN or
 *          MR_BC_DIRICHLET (see above)
 *  lo, hi  box, per dimension
 *  detail_scale  per component divisor in the detail norm (0 -> 1.0)
 *  ze, tau, lewis, kappa  flames: Zeldovich number, temperature ratio
 *          (0 < tau < 1), Lewis number, radiation coefficient (>= 0)
 *  flame_speed  flames: 0 the velocity is adv_vel; +1 / -1 it is +v_f / -v_f
 *          along axis 0, v_f the integral of omega over the leaves per unit
 *          cross-section, taken at the start of every macro step (Sec. 5;
 *          -1 is the frame that moves with a front burning towards +x)    */
typedef struct {
  int32_t pde, rk, lt, l0, recon, thresh, reflux, remesh;
  int32_t bc[3][2];
  double lo[3], hi[3];
  double nu, k_react, a_react, gamma, adv_vel[3];
  double detail_scale[5];
  double ze, tau, lewis, kappa;
  int32_t flame_speed;
} mr_scheme;

typedef struct {
  double t;                        /* time of the instance */
  int64_t leaves[MR_MAXLEV + 1];   /* leaves per level */
  int64_t leaf_updates;            /* cumulative, one per leaf per full RK step */
  int64_t near_threshold;          /* cumulative |detail - eps_l| <= 1e-12 eps_l decisions */
  int64_t iterations;              /* cumulative fine iterations */
  double mass[5];                  /* sum over leaves of |cell| q, per component */
} mr_stats_t;

/* Device memory of a context from the caller's allocator (for example
 * PyTorch's caching allocator): alloc(bytes, user) returns device memory of
 * at least `bytes` bytes aligned to 256 bytes, or NULL when it has none;
 * free(ptr, user) takes back a pointer alloc returned.  The context calls
 * alloc from mr_init / mr_init_batch and from the calls that stage host
 * data (mr_get_leaves, mr_set_leaves), on the calling thread, and frees
 * everything in mr_destroy after its stream is idle.  A NULL mr_alloc (or
 * alloc == free == NULL) means hipMalloc / hipFree.                        */
typedef struct {
  void* (*alloc)(size_t bytes, void* user);
  void (*free)(void* ptr, void* user);
  void* user;
} mr_alloc;

/* Create a single solve (Sec. 2: the IVP on a box; Alg. waveletThres takes
 * the finest level L, the level-L solution and the threshold eps).
 * dim in 1..3, l0 >= 2, l0 <= L, L - l0 <= 20, dim*L <= 3*MR_MAXLEV,
 * eps >= 0 (eps = 0 keeps the full tree); a: allocator or NULL.
 * *out receives the context.                                               */
mr_status mr_init(int dim, int L, double eps, const mr_scheme* s, const mr_alloc* a, mr_ctx** out);

/* Create a batch of n_inst independent solves sharing dim, L and scheme;
 * eps is a host array of n_inst thresholds; a: allocator or NULL.         */
mr_status mr_init_batch(int dim, int L, int n_inst, const double* eps, const mr_scheme* s, const mr_alloc* a,
                        mr_ctx** out);

/* Device bytes the context holds (its tables are dense over the full tree
 * of every instance: the footprint depends on dim, L, m and n_inst, not on
 * how many leaves the trees keep).                                         */
mr_status mr_footprint(mr_ctx* c, size_t* bytes);

/* Stream (hipStream_t, may be NULL) on which later work is queued. */
mr_status mr_set_stream(mr_ctx* c, void* hip_stream);

/* Number of conserved fields m of the scheme. */
int mr_ncomp(const mr_ctx* c);

/* Load finest-level cell averages and build the adapted tree: all levels
 * below L internal, projection bottom-up (Sec. 2), then mr_adapt.
 * q0: device, [n_inst][m][2^{dL}], x fastest (index x + n(y + n z)).      */
mr_status mr_load_finest(mr_ctx* c, const double* q0, void* hip_stream);

/* Load one instance of a batch (a free or finished slot) and build its
 * adapted tree; the other instances are not changed.
 * q0: device, [m][2^{dL}], x fastest.                                      */
mr_status mr_load_finest_inst(mr_ctx* c, int inst, const double* q0);

/* Load one instance with its own finest level L_inst (l0 <= L_inst <= L)
 * and threshold eps: q0 holds its finest-level averages (device,
 * [m][2^{d L_inst}], x fastest).  The instance never refines past L_inst,
 * its level-dependent thresholds are eps_l = 2^{d(l - L_inst)} eps, and its
 * level l steps by 2^{L-l} dt_L: with dt_L = 2^{L_inst - L} times its own
 * finest step, a context macro step is one macro step of the solve with
 * finest level L_inst, and its leaves and values are those of that solve
 * bit for bit.  So solves of uneven finest levels share every launch.
 * mr_reconstruct gives its averages on the level-L grid.                   */
mr_status mr_load_inst(mr_ctx* c, int inst, int L_inst, double eps, const double* q0);

/* Free one instance of a batch: all of its cells become absent, it drops out
 * of every kernel's work until it is loaded again.                         */
mr_status mr_clear_instance(mr_ctx* c, int inst);

/* Error flags of one instance: bit 0 non-finite value, bit 1 tree
 * invariant violated.  Clearing the failed instances (mr_clear_instance)
 * lets the others continue.                                                 */
mr_status mr_instance_flags(mr_ctx* c, int inst, int* flags);

/* Threshold eps >= 0 of one instance, used from its next load / remesh. */
mr_status mr_set_eps(mr_ctx* c, int inst, double eps);

/* Full remesh at the current synchronised time (Alg. AdaptiveMesh with
 * Alg. waveletThres; no level frozen).                                     */
mr_status mr_adapt(mr_ctx* c);

/* One macro step of 2^{L-l0} fine iterations of Alg. alg-LTS with finest
 * step dt_L > 0: all instances use dt_L.  Synchronises the stream and
 * returns MR_ENONFINITE if a value became NaN/Inf.                         */
mr_status mr_lt_step(mr_ctx* c, double dt_L);

/* Same, with a per-instance finest step (host array of n_inst values).    */
mr_status mr_lt_step_batch(mr_ctx* c, const double* dt_L);

/* Dense finest-level averages from the tree: projection, then prediction
 * coarse to fine where cells are absent (the inverse MR transform, Sec. 2).
 * q_out: device, [n_inst][m][2^{dL}], x fastest.                          */
mr_status mr_reconstruct(mr_ctx* c, double* q_out);

/* CFL helper: per instance the maximum over leaves of sum_i |f_i'(q)|:
 * d |u| (Burgers), sum_i (|u_i| + c) (Euler), sum_i |a_i| (advection and
 * flames, with the frame velocity of the current leaves when flame_speed is
 * set), 0 otherwise (diffusion and reaction limits are the caller's).
 * out: host array of n_inst values.                                        */
mr_status mr_max_wavespeed(mr_ctx* c, double* out);

/* Launch configuration of a context: the most workgroups given to the
 * list-driven kernels (stage, ghost values, projections, end of step;
 * default 1536), to the interface-leaf stage launches (512) and to the
 * list compaction (8192); the kernels loop over the rest.  bulk_levels is
 * the block-to-level schedule of the bulk stage kernel: 1 (default) one
 * launch per stage whose workgroups take the leaves of all levels of the
 * stage as one list, 2 one launch per level.  Tuning knobs only: results
 * are identical for every setting.  A value of 0 keeps the current one;
 * grids outside 0..65535 and bulk_levels outside 0..2 give MR_EINVAL.
 * Setting it drops the captured macro-step graph (recaptured by the next
 * mr_lt_step).                                                            */
typedef struct {
  int32_t list_grid, iface_grid, comp_grid, bulk_levels;
} mr_launch;
mr_status mr_set_launch(mr_ctx* c, const mr_launch* l);
mr_status mr_get_launch(mr_ctx* c, mr_launch* l);   /* l: host struct, filled */

/* Flame velocity of Sec. 5, v_f = integral of the reaction rate omega over
 * the domain, per unit cross-section normal to axis 0: per instance the sum
 * over its current leaves of omega(cell average) times the cell volume, in a
 * fixed order.  Flame problems only (else MR_EINVAL).
 * vf: host array of n_inst values.                                         */
mr_status mr_flame_speed(mr_ctx* c, double* vf);

/* Leaves of instance 0 (or `inst`) sorted by (level, Morton key):
 * key = level << 56 | morton, values q[k * n + i] (host buffers).  With
 * keys == NULL only *n is set.  MR_ECAPACITY if cap < number of leaves.    */
mr_status mr_get_leaves(mr_ctx* c, uint64_t* keys, double* q, int64_t cap, int64_t* n);
mr_status mr_get_leaves_inst(mr_ctx* c, int inst, uint64_t* keys, double* q, int64_t cap, int64_t* n);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops and harnesses that forbid allocation): the leaves
 * of instance `inst` as mr_get_leaves_inst returns them, staged through a
 * fixed device array of the library instead of buffers allocated per call.
 * The array holds MR_NOALLOC_MAX_LEAVES leaves of up to 5 components
 * (48 MiB per GPU, resolved when the first context on a GPU is created and
 * held until the process ends); MR_ECAPACITY if the instance has more
 * leaves, or if cap is smaller than their number.  Allocates nothing.
 * Every call on one GPU uses the same array: calls that overlap on one GPU
 * (from several threads or contexts at once) race.                        */
#define MR_NOALLOC_MAX_LEAVES (1 << 20)
mr_status mr_get_leaves_noalloc(mr_ctx* c, int inst, uint64_t* keys, double* q, int64_t cap, int64_t* n);

/* Replace the tree of instance 0 (or `inst`) by the given leaves (same key
 * and value layout, host buffers) at time t.  The leaves must form a
 * complete tree over level l0 that is graded (every cell within distance 2
 * of an internal node exists); MR_EINVAL otherwise.                        */
mr_status mr_set_leaves(mr_ctx* c, const uint64_t* keys, const double* q, int64_t n, double t);
mr_status mr_set_leaves_inst(mr_ctx* c, int inst, const uint64_t* keys, const double* q, int64_t n, double t);

/* Statistics of instance 0 (or `inst`). */
mr_status mr_stats(mr_ctx* c, mr_stats_t* out);
mr_status mr_stats_inst(mr_ctx* c, int inst, mr_stats_t* out);

/* Near-threshold decisions of instance `inst` (Alg. waveletThres: a node
 * is kept when its detail exceeds the level's threshold; a decision with
 * |detail - eps_l| <= 1e-12 eps_l is near the threshold, where rounding
 * could decide it): one entry per decision since the instance's last load
 * or set_leaves, sorted by (iteration, level, key).  iter[j] = fine
 * iterations completed before the remesh that took it (0 for the remesh of
 * the load), level[j] = the node's level, key[j] = its Morton key (host
 * arrays of cap entries).  With iter == NULL only *n is set.  MR_ECAPACITY
 * if cap is too small, or if the context recorded more than 65536
 * decisions since mr_load_finest (the list is then incomplete).           */
mr_status mr_near_threshold(mr_ctx* c, int inst, int64_t* iter, int32_t* level, uint64_t* key, int64_t cap,
                            int64_t* n);

/* Measurement support.  Cumulative leaf-updates of instance `inst` per
 * level (host array of MR_MAXLEV + 1 entries; one update = one leaf
 * advanced by one full RK step at that level).                           */
mr_status mr_level_updates(mr_ctx* c, int inst, int64_t* per_level);

/* Kernel classes for mr_timing_start. */
enum {
  MR_KC_STAGE_FINEST = 1,  /* RK stage kernels on the finest level */
  MR_KC_STAGE = 2,         /* RK stage kernels on all levels */
  MR_KC_PROJECT = 3,       /* projections and synchronisation values of internal nodes */
  MR_KC_GHOST = 4,         /* virtual-cell prediction */
  MR_KC_REMESH = 5,        /* details, safety, closure, pruning, apply, ghost flags */
  MR_KC_FINALIZE = 6,      /* end of step and conservative correction */
  MR_KC_STAGE_BULK = 7     /* the bulk RK stage kernel alone: leaves whose stencil
                              reaches no internal cell, all levels of a stage */
};

/* Measurement support.  Cumulative leaf-stage updates done by the bulk RK
 * stage kernel (class MR_KC_STAGE_BULK), summed over instances, for stages
 * 1, 2, 3 (host array of 3 entries).  With the algorithmic bytes of a stage
 * (Sec. 3: stage 1 reads q^n and writes q*, stage 2 reads q^n and q* and
 * writes q**, stage 3 reads q^n and q** and writes q^{n+1}: 16m, 24m, 24m
 * bytes per leaf) this gives the kernel's algorithmic traffic.  Synchronises
 * the context's stream.                                                   */
mr_status mr_stage_items(mr_ctx* c, int64_t* per_stage);

/* Bracket every later launch of one kernel class with a pair of HIP events
 * on the context's stream, until mr_timing_stop.                          */
mr_status mr_timing_start(mr_ctx* c, int kernel_class);

/* Synchronise; *total_ms = summed event time of the timed launches,
 * *launches = their number.  Ends the timing.                             */
mr_status mr_timing_stop(mr_ctx* c, double* total_ms, int64_t* launches);

/* ---- systems forms: many solves of uneven size under one scheduler ------
 *
 * A batch serves solves grouped in classes.  A class is one context: the
 * scheme, dim, its largest finest level L_max and a number of slots; each
 * slot holds one solve with its own finest level L <= L_max (mr_load_inst),
 * threshold, final time and CFL step, so every kernel launch of a macro
 * step serves all the class's solves, uneven trees included.  A class's
 * context is created when a solve is first admitted to it, if its device
 * footprint fits the batch's HBM budget (contexts of idle classes are
 * destroyed to make room), and classes step on their own streams, so their
 * work overlaps on the device.  Slots are numbered over the classes in
 * order (class 0 has slots 0 .. slots_0 - 1, and so on).                   */
typedef struct mr_batch mr_batch;

typedef struct {
  int32_t dim, L_max, slots;
  mr_scheme scheme;
} mr_class_desc;

/* One solve: its class is the first whose scheme, dim and l0 match and whose
 * L_max >= L.  Each macro step takes the finest step
 * dt = min(cfl / (w / dx + 2 d D / dx^2 + R), dt_max, (t_final - t) / N)
 * with dx the finest cell width along axis 0, w the largest wave speed of
 * its leaves (mr_max_wavespeed), D the largest diffusion coefficient (nu;
 * max(1, 1/Le) for the flames), R = 0.8 k for the Nagumo source (0
 * otherwise), dt_max > 0 an optional cap and N = 2^{L - l0} fine iterations
 * per macro step, so that the last macro step ends at t_final.            */
typedef struct {
  int32_t dim, L;
  double eps, t_final, cfl, dt_max;
  mr_scheme scheme;
} mr_instance_desc;

enum { MR_SLOT_FREE = 0, MR_SLOT_RUNNING = 1, MR_SLOT_DONE = 2, MR_SLOT_FAILED = 3 };

/* An empty batch of n_classes classes (host array) whose contexts may hold
 * at most hbm_budget device bytes together; a: allocator or NULL.         */
mr_status mr_batch_create(int n_classes, const mr_class_desc* classes, size_t hbm_budget, const mr_alloc* a,
                          mr_batch** out);

/* Admit a solve into a free slot of its class: q0 device, [m][2^{d L}],
 * x fastest (copied in; the tree is adapted at once).  *slot receives the
 * slot.  MR_ECAPACITY if its class has no free slot, or if creating the
 * class's context would exceed the budget; MR_EINVAL if no class fits it. */
mr_status mr_batch_admit(mr_batch* b, const mr_instance_desc* d, const double* q0, int* slot);

/* One macro step of every running solve (each with its own dt, above);
 * classes are queued on their own streams before any wait.  A solve whose
 * values become non-finite fails alone (state MR_SLOT_FAILED).            */
mr_status mr_batch_step(mr_batch* b);

/* Slots that reached their final time (MR_SLOT_DONE) or failed since the
 * last poll (host array of cap entries; *n receives their number).        */
mr_status mr_batch_poll(mr_batch* b, int* done_slots, int cap, int* n);

/* State (MR_SLOT_*), time and macro steps taken of one slot. */
mr_status mr_batch_slot_info(mr_batch* b, int slot, int* state, double* t, int64_t* macro_steps);

/* Leaves of a slot (layout of mr_get_leaves; host buffers). */
mr_status mr_batch_get_leaves(mr_batch* b, int slot, uint64_t* keys, double* q, int64_t cap, int64_t* n);

/* Free a slot (its cells become absent; it drops out of every launch). */
mr_status mr_batch_release(mr_batch* b, int slot);

/* Device bytes the batch's class contexts hold. */
mr_status mr_batch_footprint(mr_batch* b, size_t* bytes);

/* Description of the batch's last error (never NULL). */
const char* mr_batch_last_error(const mr_batch* b);

/* Destroy the batch and every class context (NULL is ignored). */
void mr_batch_destroy(mr_batch* b);

/* Wait for all queued work of the context. */
mr_status mr_synchronize(mr_ctx* c);

/* Description of the last error of the context (never NULL). */
const char* mr_last_error(const mr_ctx* c);

/* Release the context and all of its device memory (NULL is ignored). */
void mr_destroy(mr_ctx* c);

#ifdef __cplusplus
}
#endif
#endif
