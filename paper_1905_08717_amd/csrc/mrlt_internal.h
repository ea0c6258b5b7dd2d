// mrlt_internal.h -- device-side data model of the MRLT/NERK3 HIP library.
//
// Storage: for every level l in [l0, L] and every instance of a batch, a
// dense array of 2^{d l} cells indexed by the Morton key of the cell (the key
// is the slot: a collision-free, direct-mapped table).  Global cell index
//   G = off[l] + inst * n[l] + morton.
// Children of cell (l, t) with t = inst * n[l] + key are (l+1, (t << d) + c),
// c = a | b<<1 | e<<2: a child group is contiguous.
// Level tables start at multiples of 256 cells (off[l] is padded), so byte
// tables can be read 16 cells at a time.
// Values are FP64, field-major per time slot: slot[s][k * Ntot + G].
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define MRD_MAXLEV 24
#define BS_SHIFT 12  // block summaries cover 4096 cells

enum { ST_ABSENT = 0, ST_LEAF = 1, ST_INTERNAL = 2 };

// Time slots.  Internal nodes reuse slots: Q1 holds the stage-2 projection
// (Alg. projRK2) of internal nodes, QH / QE of the mid-step level hold the
// theta=1/2 projection and the end value of Sec. 4.3 during Case B.
enum { SL_Q0 = 0, SL_Q1, SL_H1, SL_N14, SL_N34, SL_QH, SL_QE, SL_X2, SL_Q1REF, SL_COUNT };

enum { PDE_ADVECTION = 0, PDE_BURGERS = 1, PDE_NAGUMO = 2, PDE_EULER = 3, PDE_LINEAR = 4,
       PDE_FLAME = 5, PDE_FLAMEBALL = 6 };

// projection kinds (one kernel, selected by mode)
enum { PJ_Q0 = 0, PJ_CASEB, PJ_REF2, PJ_RK2, PJ_REF3, PJ_RK3, PJ_ST2, PJ_ST3 };

// counters per instance
enum { CNT_UPDATES = 0, CNT_NEAR, CNT_NONFINITE, CNT_BAD, CNT_LEVEL0 };
// per instance: the four counters above, then leaf-updates per level
#define CNT_PER_INST (CNT_LEVEL0 + MRD_MAXLEV + 1)

struct Geo {
  int d, L, l0, m, nsub, B;
  int pde, recon, thresh, reflux;
  int rk;  // 3: compact RK3 (NERK3), 2: compact RK2 (NERK2)
  int lt;  // 1: local time stepping, 0: one global step for every level
  int periodic[3];
  int dirichlet[3];  // homogeneous Dirichlet sides of the axis: bit 0 low, bit 1 high
  int two_point;     // the fluxes read only the two cells next to a face
  int64_t n[MRD_MAXLEV + 1];     // cells per instance at level l (2^{d l})
  int64_t off[MRD_MAXLEV + 1];   // first global index of level l
  int64_t Ntot;                  // total cells over levels and instances
  int64_t rc_off[MRD_MAXLEV + 1];  // coarse-side register block of level l
  int64_t rf_off[MRD_MAXLEV + 1];  // fine-side register block of level l
  double invdx[MRD_MAXLEV + 1][3];
  double vol[MRD_MAXLEV + 1];
  double nu, k_react, a_react, gamma, adv[3];
  double scale[5];
  // flames: Zeldovich number, temperature ratio, Lewis number, radiation
  // coefficient; flame_speed 0: velocity adv, +-1: +-v_f along axis 0
  double ze, tau, lewis, kappa;
  double flame_area;  // cross-section normal to axis 0 (v_f per unit area)
  int flame_speed;
  // list compaction: level l is cut into blocks of comp_chunk[l] cells (a
  // power of two <= 4096 that never straddles two instances); its blocks are
  // comp_first[l] .. comp_first[l+1]-1 of a global block numbering
  int64_t comp_first[MRD_MAXLEV + 2];
  int comp_chunk[MRD_MAXLEV + 1];
  // superblocks of 2^sb_shift[l] compaction blocks (at most 64, never
  // straddling an instance): level l's are sb_first[l] .. sb_first[l+1]-1
  int64_t sb_first[MRD_MAXLEV + 2];
  int sb_shift[MRD_MAXLEV + 1];
  // 4096-cell blocks of level l (one summary byte each) start at bs_off[l]
  int64_t bs_off[MRD_MAXLEV + 2];
  // instances [i0, i1) that the remesh sweeps may change (all of them inside a
  // macro step; one instance when it is loaded or adapted on its own)
  int i0, i1;
  // launch knobs (no effect on results): grid caps of the list-driven
  // kernels, of the interface-leaf stage launches and of the compaction
  int list_grid, iface_grid, comp_grid;
  int bulk_split;  // 1: the bulk stage kernel is launched once per level (mr_launch.bulk_levels = 2)
  // verify tree invariants the grading guarantees (stencil cells exist, the
  // coarse side of a refined face is a leaf) as the kernels read them; a
  // violation is reported as MR_ESTATE (environment MRLT_CHECK at init)
  int check;
};

// per-level lists of cell indices (within-level index t = inst * n[l] + key):
// leaves, internal nodes, virtual (ghost) cells read by leaf stencils, and
// LS_IFACE: the leaves of LS_LEAF below L whose stencil (offsets 1, and 2
// with the MUSCL reconstruction, along an axis) reaches an internal cell
enum { LS_LEAF = 0, LS_INTERNAL = 1, LS_GHOST = 2, LS_IFACE = 3, LS_COUNT = 4 };

struct Dev {
  uint8_t* st;     // status per cell
  uint8_t* rf;     // remesh scratch: bit1 member of W (nodes that will be internal)
  uint8_t* sigt;   // per internal node: significant at the last remesh that evaluated its level
  uint8_t* ccode;  // list codes per cell, from the compaction's count pass to its write pass
  uint8_t* bsum;   // per 4096-cell block: 1 a cell exists, 2 one is internal, 4 one is a leaf
  uint8_t* wsum;   // per 4096-cell block: 1 when the block may hold W marks
  uint8_t* nsum;   // per 4096-cell block: 1 when an internal node is in it or a neighbour block
  double* q[SL_COUNT];
  double* regc;    // [level block][2d][m][B n_l]
  double* regf;    // [level block][2d][nsub][m][B n_l]
  double* rflux;   // [level block][2d][m][B n_l] refined-face fluxes of the interface leaves in the
                   // current stage (PDEs of four or more fields only; else null)
  const double* dt;   // [B] dt of the finest level
  const double* eps;  // [B]
  unsigned long long* cnt;  // [B][CNT_PER_INST]
  int* lst[LS_COUNT];       // level l's list starts at off[l], capacity B n[l]
  int* lcnt;                // [LS_COUNT][MRD_MAXLEV + 1] list lengths
  int* bcnt;                // [LS_COUNT][blocks] compaction block counts
  int* sbcnt;               // [LS_COUNT][superblocks] their sums (zero between compactions)
  int* sboff;               // [LS_COUNT][superblocks] list offset of each superblock
  int* leafcnt;             // [B][MRD_MAXLEV + 1] leaves per instance and level
  unsigned long long* items;  // [3] leaf-stage updates of the bulk stage launches, per stage
  unsigned* lflag;          // [MRD_MAXLEV + 1] level flags (kernels.hip, LF_*)
  double* vel;              // [2B] flames: velocity along axis 0 this macro step, then v_f
  double* vfpart;           // [compaction blocks] flames: partial integrals of omega
  // near-threshold decisions |D - eps_l| <= 1e-12 eps_l: entry j is
  // near[2j] = fine iterations completed before the remesh,
  // near[2j+1] = inst << 45 | level << 40 | Morton key; near_n counts them
  // (entries beyond NEAR_CAP are counted, not stored)
  unsigned long long* near;
  unsigned long long* near_n;
  const long long* iterb;   // fine iterations completed before the current macro step
  // [B] finest level of each instance (<= L): an instance whose finest level
  // is below L never refines past it, and its level-dependent thresholds
  // are those of a solve with that finest level
  const uint8_t* lcap;
};

#define NEAR_CAP 65536

// ---- launchers (kernels.hip) -------------------------------------------
void launch_fill_status(const Geo& g, const Dev& p, int lev, uint8_t v, hipStream_t s);
// finest-level averages of every instance (inst < 0, level L) or of one
// instance at its own finest level Li
void launch_load_finest(const Geo& g, const Dev& p, const double* src, int inst, int Li, hipStream_t s);
// statuses of one instance for a load at finest level Li (inst >= 0), or
// all absent (inst = -1 - slot)
void launch_fill_instance(const Geo& g, const Dev& p, int inst, int Li, hipStream_t s);
void launch_project(const Geo& g, const Dev& p, int lev, int mode, hipStream_t s);
// virtual cells of levels lo..hi at `stage`; level cb_lev (if in range) is
// the child of the mid-step level (case B)
void launch_ghost(const Geo& g, const Dev& p, int lo, int hi, int cb_lev, int stage, hipStream_t s);
// stage kernel over the leaves of levels lo..hi: part 0 the leaves whose
// stencil reaches no internal cell (stage 1 also adds the leaf-updates of
// these levels to the counters), part 1 the interface leaves
// part 0: bulk leaves of levels lo..hi (levels >= lq0 also store q^n at
// the last stage); part 1: interface leaves
void launch_stage(const Geo& g, const Dev& p, int lo, int hi, int stage, int part, hipStream_t s,
                  int lq0 = MRD_MAXLEV + 1);
// end of step of the leaves of levels lo..min(hi, L-1) (all leaves, or the
// interface leaves only)
void launch_finalize(const Geo& g, const Dev& p, int lo, int hi, bool iface_only, hipStream_t s);
// remesh byte table cleared on levels lo..hi
void launch_remesh_clear(const Geo& g, const Dev& p, int lo, int hi, hipStream_t s);
// level flags before the apply passes of a remesh at la
void launch_level_w(const Geo& g, const Dev& p, int la, hipStream_t s);
// details of the internal nodes of levels la..hi and the seed of W, with the
// scale safety of the frozen level la - 1
// n_it: fine iteration of the macro step (0 outside a macro step), recorded
// with near-threshold decisions
void launch_detail_seed(const Geo& g, const Dev& p, int la, int hi, int n_it, hipStream_t s);
// flames: v_f of every instance from its leaves; vel = flame_speed * v_f
void launch_flame_speed(const Geo& g, const Dev& p, hipStream_t s);
// lists of levels lo..L; full: rebuild without trusting the block summaries
void launch_compact(const Geo& g, const Dev& p, int lo, bool full, hipStream_t s);
void launch_close(const Geo& g, const Dev& p, int lev, hipStream_t s);
void launch_prune(const Geo& g, const Dev& p, int lev, int la, hipStream_t s);
void launch_apply(const Geo& g, const Dev& p, int lev, int la, hipStream_t s);
void launch_recon_level(const Geo& g, const Dev& p, int lev, double* dense, hipStream_t s);
void launch_to_rowmajor(const Geo& g, const double* dense, double* out, hipStream_t s);
void launch_count(const Geo& g, const Dev& p, int lev, int inst, uint8_t want, int* blockcnt,
                  int nblk, hipStream_t s);
void launch_scan_blocks(int* blockcnt, int nblk, long long* total, hipStream_t s);
void launch_gather_leaves(const Geo& g, const Dev& p, int lev, int inst, const int* blockoff,
                          int nblk, long long base, unsigned long long* keys, double* vals,
                          long long vstride, hipStream_t s);
void launch_scatter_leaves(const Geo& g, const Dev& p, int inst, const unsigned long long* keys,
                           const double* vals, long long n, int* err, hipStream_t s);
void launch_mark_parents(const Geo& g, const Dev& p, int lev, int* err, hipStream_t s);
void launch_validate(const Geo& g, const Dev& p, int lev, int* err, hipStream_t s);
void launch_wavespeed(const Geo& g, const Dev& p, int lev, unsigned long long* out, hipStream_t s);
void launch_mass_partial(const Geo& g, const Dev& p, int lev, int inst, double* part, int nblk,
                         hipStream_t s);
void launch_clear_regs(const Geo& g, const Dev& p, hipStream_t s);
int blocks_for(int64_t n);
