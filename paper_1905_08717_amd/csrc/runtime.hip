// runtime.hip -- host runtime behind the C ABI of include/mrlt.h.
//
// Owns the device memory of a context, sequences the kernels of one
// local-time-stepping macro step (Alg. alg-LTS of arXiv:1905.08717, one call
// per fine iteration n = 0 .. 2^{L-l0}-1) and marshals the boundary calls.
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "mrlt.h"
#include "mrlt_internal.h"

struct mr_ctx {
  Geo g;
  Dev p;
  mr_scheme s;
  hipStream_t stream = nullptr;
  std::vector<double> eps, t, dt_host;
  std::vector<unsigned long long> cnt_host;
  int64_t iters = 0;
  bool broken = false;
  std::string err;
  std::vector<void*> allocs;
  mr_alloc alloc{};                   // caller's device allocator (alloc == NULL: hipMalloc)
  size_t bytes = 0;                   // device bytes the context holds
  double* ws_host = nullptr;          // pinned [B]: wave speeds read back without blocking
  double* dt_d = nullptr;
  double* eps_d = nullptr;
  int* blockcnt_d = nullptr;
  long long* total_d = nullptr;
  int* err_d = nullptr;
  unsigned long long* ws_d = nullptr;
  double* part_d = nullptr;
  void* scratch_d = nullptr;          // staging array of this context's device
  int max_blocks = 0;
  hipStream_t own_stream = nullptr;   // default stream of the context
  bool use_graph = true;              // replay the captured macro step
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  long long* iterb_d = nullptr;       // fine iterations before the current macro step
  uint8_t* lcap_d = nullptr;          // finest level of each instance
  std::vector<uint8_t> lcap_host;
  long long iter_upload = 0;          // host copy of it, written only before an upload
  std::vector<int64_t> it_start;      // per instance: iterations at its last load / set
  int timed_class = 0;          // kernel class under HIP-event timing (0: none)
  std::vector<hipEvent_t> ev;   // event pairs around timed launches
  size_t ev_used = 0;
};

// Staging array of mr_get_leaves_noalloc: keys of up to MR_NOALLOC_MAX_LEAVES
// leaves, then their values (up to 5 components), in device memory the
// library holds on every GPU it runs on until the process ends.  Host code
// uses the address hipGetSymbolAddress gives for the current device, never
// the array's name.
#define NOALLOC_BYTES ((size_t)MR_NOALLOC_MAX_LEAVES * 8u * 6u)
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// address of the staging array on the current device (resolved once per
// device, at the first context created there)
hipError_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

mr_status set_err(mr_ctx* c, mr_status st, const std::string& msg) {
  if (c) c->err = msg;
  return st;
}

mr_status hip_check(mr_ctx* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return MR_OK;
  return set_err(c, e == hipErrorOutOfMemory ? MR_ENOMEM : MR_EDEVICE,
                 std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(c, call)                                  \
  do {                                                   \
    mr_status st__ = hip_check((c), (call), #call);      \
    if (st__ != MR_OK) return st__;                      \
  } while (0)

// device memory through the caller's allocator when one was given, else
// hipMalloc; tmp_free returns it
void* raw_alloc(mr_ctx* c, size_t bytes) {
  if (c->alloc.alloc) return c->alloc.alloc(bytes, c->alloc.user);
  void* ptr = nullptr;
  if (hipMalloc(&ptr, bytes) != hipSuccess) return nullptr;
  return ptr;
}

void raw_free(mr_ctx* c, void* ptr) {
  if (!ptr) return;
  if (c->alloc.alloc) c->alloc.free(ptr, c->alloc.user);
  else (void)hipFree(ptr);
}

mr_status dalloc(mr_ctx* c, void** ptr, size_t bytes) {
  *ptr = nullptr;
  if (bytes == 0) bytes = 8;
  bytes = (bytes + 255) & ~(size_t)255;
  *ptr = raw_alloc(c, bytes);
  if (!*ptr) return set_err(c, MR_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  c->allocs.push_back(*ptr);
  c->bytes += bytes;
  return hip_check(c, hipMemsetAsync(*ptr, 0, bytes, c->stream), "hipMemsetAsync");
}

int lmin_of(const Geo& g, int64_t n) {
  for (int lev = g.l0; lev <= g.L; lev++)
    if (n % ((int64_t)1 << (g.L - lev)) == 0) return lev;
  return g.L;
}

mr_status check_launch(mr_ctx* c, const char* what) {
  return hip_check(c, hipGetLastError(), what);
}

// run `launch` and, when its kernel class is being timed, bracket it with a
// pair of HIP events on the context's stream
template <class F>
void timed(mr_ctx* c, int kc, F&& launch) {
  const bool on = c->timed_class == kc || (c->timed_class == MR_KC_STAGE && kc == MR_KC_STAGE_FINEST);
  if (!on) {
    launch();
    return;
  }
  if (c->ev_used + 2 > c->ev.size()) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
      launch();
      return;
    }
    c->ev.push_back(a);
    c->ev.push_back(b);
  }
  (void)hipEventRecord(c->ev[c->ev_used], c->stream);
  launch();
  (void)hipEventRecord(c->ev[c->ev_used + 1], c->stream);
  c->ev_used += 2;
}

void project_range(mr_ctx* c, int hi, int lo, int mode) {
  for (int lev = hi; lev >= lo; lev--)
    timed(c, MR_KC_PROJECT, [&] { launch_project(c->g, c->p, lev, mode, c->stream); });
}

// leaf / internal / interface / ghost lists of levels la..L; full after
// status changes made outside the remesh
void refresh_lists(mr_ctx* c, int la, bool full) {
  timed(c, MR_KC_REMESH, [&] { launch_compact(c->g, c->p, la, full, c->stream); });
}

// the iteration count the detail kernel records with near-threshold
// decisions: iterations completed before the macro step (or remesh) that
// follows on the stream
mr_status upload_iter_base(mr_ctx* c) {
  c->iter_upload = (long long)c->iters;
  return hip_check(c, hipMemcpyAsync(c->iterb_d, &c->iter_upload, sizeof(long long), hipMemcpyHostToDevice, c->stream),
                   "iteration upload");
}

// remesh with levels below la frozen; statuses, new values and lists;
// n_it: fine iteration of the macro step (0 outside one)
void remesh(mr_ctx* c, int la, int n_it = 0) {
  const Geo& g = c->g;
  if (la > g.L - 1) return;
  hipStream_t s = c->stream;
  timed(c, MR_KC_REMESH, [&] { launch_remesh_clear(g, c->p, la, g.L - 1, s); });
  timed(c, MR_KC_REMESH, [&] { launch_detail_seed(g, c->p, la, g.L - 1, n_it, s); });
  for (int lev = g.L - 2; lev >= la; lev--) timed(c, MR_KC_REMESH, [&] { launch_close(g, c->p, lev, s); });
  for (int lev = la; lev <= g.L - 1; lev++) timed(c, MR_KC_REMESH, [&] { launch_prune(g, c->p, lev, la, s); });
  timed(c, MR_KC_REMESH, [&] { launch_level_w(g, c->p, la, s); });
  for (int lev = la; lev <= g.L; lev++) timed(c, MR_KC_REMESH, [&] { launch_apply(g, c->p, lev, la, s); });
  refresh_lists(c, la, false);
}

void ghost_fill(mr_ctx* c, int lmin, int stage) {
  const Geo& g = c->g;
  const int lo = lmin > g.l0 ? lmin : g.l0 + 1;
  const int cb = lmin > g.l0 ? lmin : -1;
  timed(c, MR_KC_GHOST, [&] { launch_ghost(g, c->p, lo, g.L, cb, stage, c->stream); });
}

// one step of the MR scheme with a global time step (the paper's
// comparison method): every level advances by dt at the same stage times
// RK stage st on the leaves of levels lo..hi: the bulk launch (timed under
// MR_KC_STAGE_BULK too; at the last stage its leaves of levels >= lq0 also
// store q^n of their next step) and the interface launch
void stage_launch(mr_ctx* c, int lo, int hi, int st, bool bulk, bool iface, int lq0 = MRD_MAXLEV + 1) {
  const Geo& g = c->g;
  hipStream_t s = c->stream;
  const int cls = lo == g.L ? MR_KC_STAGE_FINEST : MR_KC_STAGE;
  if (bulk) {
    // block-to-level schedule: all levels of the stage in one launch, or
    // one launch per level (the bulk leaves read only their own level)
    if (g.bulk_split) {
      for (int lev = lo; lev <= hi; lev++)
        timed(c, cls, [&] { timed(c, MR_KC_STAGE_BULK, [&] { launch_stage(g, c->p, lev, lev, st, 0, s, lq0); }); });
    } else {
      timed(c, cls, [&] { timed(c, MR_KC_STAGE_BULK, [&] { launch_stage(g, c->p, lo, hi, st, 0, s, lq0); }); });
    }
  }
  if (iface && lo <= g.L - 1)
    timed(c, cls, [&] { launch_stage(g, c->p, lo, hi < g.L ? hi : g.L - 1, st, 1, s); });
}

void mr_iteration(mr_ctx* c, int n_it) {
  const Geo& g = c->g;
  const int L = g.L;
  hipStream_t s = c->stream;
  auto stage = [&](int st) { stage_launch(c, g.l0, L, st, true, true, st == g.rk ? g.l0 : MRD_MAXLEV + 1); };
  project_range(c, L - 1, g.l0, PJ_Q0);
  if (c->s.remesh && g.l0 <= L - 1) {
    remesh(c, g.l0, n_it);
    project_range(c, L - 1, g.l0, PJ_Q0);
  }
  ghost_fill(c, g.l0, 1);
  stage(1);
  project_range(c, L - 1, g.l0, PJ_ST2);
  ghost_fill(c, g.l0, 2);
  stage(2);
  if (g.rk == 3) {
    project_range(c, L - 1, g.l0, PJ_ST3);
    ghost_fill(c, g.l0, 3);
    stage(3);
  }
  timed(c, MR_KC_FINALIZE, [&] { launch_finalize(g, c->p, g.l0, L, true, s); });
}

// one iteration of Alg. alg-LTS
void lt_iteration(mr_ctx* c, int64_t n, int64_t N) {
  const Geo& g = c->g;
  const int L = g.L;
  if (!g.lt) {
    mr_iteration(c, (int)n);
    return;
  }
  const int lmin = lmin_of(g, n);
  // the steps of levels >= lnext end with this iteration (the next one
  // starts there); of those, only the finest level's step also ran in it
  const int lnext = (n + 1 == N) ? g.l0 : lmin_of(g, n + 1);
  project_range(c, L - 1, lmin, PJ_Q0);
  if (c->s.remesh && lmin <= L - 1) {
    remesh(c, lmin, (int)n);
    project_range(c, L - 1, lmin, PJ_Q0);
  }
  hipStream_t s = c->stream;
  if (lmin > g.l0) project_range(c, lmin - 1, lmin - 1, PJ_CASEB);
  ghost_fill(c, lmin, 1);
  stage_launch(c, lmin, L, 1, true, true);
  project_range(c, L - 1, lmin, PJ_REF2);
  ghost_fill(c, lmin, 2);
  // stage-2 sweep L -> lmin: the bulk leaves of every level read only their
  // own level, so they go first in one launch; the interface leaves of a
  // level need the finer level's stage-2 values and its projection
  stage_launch(c, lmin, L, 2, true, false, g.rk == 2 ? L : MRD_MAXLEV + 1);
  for (int lev = L - 1; lev >= lmin; lev--) {
    project_range(c, lev, lev, PJ_RK2);
    stage_launch(c, lev, lev, 2, false, true);
  }
  if (g.rk == 2) {
    // RK2: the step ends after the second stage
    timed(c, MR_KC_FINALIZE, [&] { launch_finalize(g, c->p, lnext, L, false, s); });
    return;
  }
  project_range(c, L - 1, lmin, PJ_REF3);
  ghost_fill(c, lmin, 3);
  stage_launch(c, lmin, L, 3, true, false, L);
  for (int lev = L - 1; lev >= lmin; lev--) {
    project_range(c, lev, lev, PJ_RK3);
    stage_launch(c, lev, lev, 3, false, true);
  }
  timed(c, MR_KC_FINALIZE, [&] { launch_finalize(g, c->p, lnext, L, false, s); });
}

mr_status read_counters(mr_ctx* c) {
  const size_t nb = sizeof(unsigned long long) * c->g.B * CNT_PER_INST;
  HIPCHK(c, hipMemcpyAsync(c->cnt_host.data(), c->p.cnt, nb, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return MR_OK;
}

mr_status check_flags(mr_ctx* c) {
  mr_status st = read_counters(c);
  if (st != MR_OK) return st;
  for (int i = 0; i < c->g.B; i++) {
    const unsigned long long bad = c->cnt_host[i * CNT_PER_INST + CNT_BAD];
    if (bad) {
      c->broken = true;
      char buf[160];
      snprintf(buf, sizeof buf, "tree invariant violated in instance %d (code 0x%llx)", i, bad);
      return set_err(c, MR_ESTATE, buf);
    }
  }
  for (int i = 0; i < c->g.B; i++)
    if (c->cnt_host[i * CNT_PER_INST + CNT_NONFINITE]) {
      c->broken = true;
      char buf[96];
      snprintf(buf, sizeof buf, "non-finite cell average in instance %d", i);
      return set_err(c, MR_ENONFINITE, buf);
    }
  return MR_OK;
}

mr_status adapt_impl(mr_ctx* c) {
  const Geo& g = c->g;
  mr_status st0 = upload_iter_base(c);
  if (st0 != MR_OK) return st0;
  project_range(c, g.L - 1, g.l0, PJ_Q0);
  if (g.l0 <= g.L - 1) remesh(c, g.l0);
  else refresh_lists(c, g.l0, true);
  project_range(c, g.L - 1, g.l0, PJ_Q0);
  mr_status st = check_launch(c, "adapt");
  if (st != MR_OK) return st;
  return check_flags(c);
}

mr_status upload_lcap(mr_ctx* c) {
  return hip_check(c, hipMemcpyAsync(c->lcap_d, c->lcap_host.data(), c->g.B, hipMemcpyHostToDevice, c->stream),
                   "finest level upload");
}

mr_status level_count(mr_ctx* c, int lev, int inst, uint8_t want, long long* total) {
  const int nblk = (int)((c->g.n[lev] + 255) / 256);
  launch_count(c->g, c->p, lev, inst, want, c->blockcnt_d, nblk, c->stream);
  launch_scan_blocks(c->blockcnt_d, nblk, c->total_d, c->stream);
  HIPCHK(c, hipMemcpyAsync(total, c->total_d, sizeof(long long), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return check_launch(c, "count");
}

}  // namespace

extern "C" {

int mr_ncomp(const mr_ctx* c) { return c ? c->g.m : 0; }

const char* mr_last_error(const mr_ctx* c) { return c ? c->err.c_str() : "null context"; }

void mr_destroy(mr_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  for (void* a : c->allocs) raw_free(c, a);
  if (c->ws_host) (void)hipHostFree(c->ws_host);
  if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
  delete c;
}

mr_status mr_init_batch(int dim, int L, int n_inst, const double* eps, const mr_scheme* s, const mr_alloc* a,
                        mr_ctx** out) {
  if (!out) return MR_EINVAL;
  *out = nullptr;
  if (!s || !eps || dim < 1 || dim > 3 || n_inst < 1) return MR_EINVAL;
  if (a && ((a->alloc == nullptr) != (a->free == nullptr))) return MR_EINVAL;
  if (s->l0 < 2 || L < s->l0 || L > MR_MAXLEV || L - s->l0 > 20 || dim * L > 40) return MR_EINVAL;
  if ((s->rk != 2 && s->rk != 3) || (s->lt != 0 && s->lt != 1) || s->pde < MR_PDE_ADVECTION ||
      s->pde > MR_PDE_FLAMEBALL)
    return MR_EINVAL;
  if (s->recon < 0 || s->recon > 2) return MR_EINVAL;
  const bool flame = s->pde == MR_PDE_FLAME || s->pde == MR_PDE_FLAMEBALL;
  if (flame && !(s->ze > 0.0 && s->tau > 0.0 && s->tau < 1.0 && s->lewis > 0.0 && s->kappa >= 0.0))
    return MR_EINVAL;
  if (s->flame_speed < -1 || s->flame_speed > 1 || (s->flame_speed != 0 && !flame)) return MR_EINVAL;
  for (int a = 0; a < dim; a++) {
    // periodic on both sides or on neither; Dirichlet not for the Euler system
    if ((s->bc[a][0] == MR_BC_PERIODIC) != (s->bc[a][1] == MR_BC_PERIODIC)) return MR_EINVAL;
    for (int side = 0; side < 2; side++) {
      if (s->bc[a][side] < MR_BC_PERIODIC || s->bc[a][side] > MR_BC_DIRICHLET) return MR_EINVAL;
      if (s->bc[a][side] == MR_BC_DIRICHLET && s->pde == MR_PDE_EULER) return MR_EINVAL;
    }
    if (!(s->hi[a] > s->lo[a])) return MR_EINVAL;
  }
  for (int i = 0; i < n_inst; i++)
    if (!(eps[i] >= 0.0) || !std::isfinite(eps[i])) return MR_EINVAL;

  mr_ctx* c = new mr_ctx();
  c->s = *s;
  if (a) c->alloc = *a;
  if (hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    return MR_EDEVICE;
  }
  if (scratch_address(&c->scratch_d) != hipSuccess) {
    (void)hipStreamDestroy(c->own_stream);
    delete c;
    return MR_EDEVICE;
  }
  c->stream = c->own_stream;
  c->use_graph = getenv("MRLT_NO_GRAPH") == nullptr;
  Geo& g = c->g;
  memset(&g, 0, sizeof g);
  g.d = dim;
  g.L = L;
  g.l0 = s->l0;
  g.m = s->pde == MR_PDE_EULER ? dim + 2 : (s->pde == MR_PDE_FLAMEBALL ? 2 : 1);
  g.nsub = 1 << (dim - 1);
  g.B = n_inst;
  g.i0 = 0;
  g.i1 = n_inst;
  g.pde = s->pde;
  g.recon = s->recon;
  g.thresh = s->thresh;
  g.reflux = s->reflux;
  g.rk = s->rk;
  g.lt = s->lt;
  for (int a = 0; a < 3; a++) {
    g.periodic[a] = a < dim && s->bc[a][0] == MR_BC_PERIODIC;
    g.dirichlet[a] = a < dim ? (s->bc[a][0] == MR_BC_DIRICHLET ? 1 : 0) | (s->bc[a][1] == MR_BC_DIRICHLET ? 2 : 0)
                             : 0;
  }
  int64_t off = 0, rc = 0, rf = 0;
  for (int lev = g.l0; lev <= L; lev++) {
    g.n[lev] = (int64_t)1 << (dim * lev);
    g.off[lev] = off;
    off += (g.B * g.n[lev] + 255) & ~(int64_t)255;
    g.rc_off[lev] = rc;
    g.rf_off[lev] = rf;
    if (lev < L) {
      rc += (int64_t)2 * dim * g.m * g.B * g.n[lev];
      rf += (int64_t)2 * dim * g.nsub * g.m * g.B * g.n[lev];
    }
    double v = 1.0;
    for (int a = 0; a < 3; a++) {
      if (a < dim) {
        const double dx = (s->hi[a] - s->lo[a]) / (double)((int64_t)1 << lev);
        g.invdx[lev][a] = 1.0 / dx;
        v = v * dx;
      } else {
        g.invdx[lev][a] = 1.0;
      }
    }
    g.vol[lev] = v;
  }
  g.Ntot = off;
  {
    int64_t nbs = 0;
    for (int lev = g.l0; lev <= L; lev++) {
      g.bs_off[lev] = nbs;
      nbs += (g.B * g.n[lev] + (1 << BS_SHIFT) - 1) >> BS_SHIFT;
    }
    g.bs_off[L + 1] = nbs;
  }
  {
    int64_t nb = 0;
    for (int lev = g.l0; lev <= L; lev++) {
      // 4096-cell blocks of 16-cell lane groups, else one cell per lane
      const int64_t ch = g.n[lev] >= 4096 ? 4096 : (g.n[lev] < 256 ? g.n[lev] : 256);
      g.comp_chunk[lev] = (int)ch;
      g.comp_first[lev] = nb;
      nb += g.B * g.n[lev] / ch;
    }
    g.comp_first[L + 1] = nb;
    int64_t ns = 0;
    for (int lev = g.l0; lev <= L; lev++) {
      const int64_t bpi = g.n[lev] / g.comp_chunk[lev];  // blocks per instance
      int sh = 0;
      while (sh < 6 && ((int64_t)2 << sh) <= bpi) sh++;
      g.sb_shift[lev] = sh;
      g.sb_first[lev] = ns;
      ns += (g.B * bpi) >> sh;
    }
    g.sb_first[L + 1] = ns;
    for (int lev = g.l0; lev <= L; lev++)
      if (g.B * g.n[lev] >= ((int64_t)1 << 31)) {
        (void)hipStreamDestroy(c->own_stream);
        delete c;
        return MR_EINVAL;
      }
  }
  g.list_grid = 1536;  // six resident 4-wave workgroups per CU
  g.bulk_split = 0;
  g.iface_grid = 512;
  g.comp_grid = 8192;
  g.check = getenv("MRLT_CHECK") != nullptr ? 1 : 0;
  g.nu = s->nu;
  g.k_react = s->k_react;
  g.a_react = s->a_react;
  g.gamma = s->gamma;
  for (int a = 0; a < 3; a++) g.adv[a] = s->adv_vel[a];
  for (int k = 0; k < 5; k++) g.scale[k] = s->detail_scale[k] > 0.0 ? s->detail_scale[k] : 1.0;
  g.ze = s->ze;
  g.tau = s->tau;
  g.lewis = s->lewis;
  g.kappa = s->kappa;
  g.flame_speed = s->flame_speed;
  g.flame_area = 1.0;
  for (int a = 1; a < dim; a++) g.flame_area = g.flame_area * (s->hi[a] - s->lo[a]);
  {
    bool still = s->flame_speed == 0;
    for (int a = 0; a < dim; a++) still = still && s->adv_vel[a] == 0.0;
    g.two_point = s->pde == MR_PDE_NAGUMO || s->pde == MR_PDE_LINEAR || (flame && still);
  }

  c->eps.assign(eps, eps + n_inst);
  c->t.assign(n_inst, 0.0);
  c->dt_host.assign(n_inst, 0.0);
  c->cnt_host.assign((size_t)n_inst * CNT_PER_INST, 0);
  c->it_start.assign(n_inst, 0);
  c->lcap_host.assign(n_inst, (uint8_t)L);
  c->max_blocks = (int)((g.n[L] + 255) / 256);

  mr_status st = MR_OK;
  void* ptr;
#define ALLOC(field, type, count)                                          \
  do {                                                                     \
    st = dalloc(c, &ptr, sizeof(type) * (size_t)(count));                  \
    if (st != MR_OK) goto fail;                                            \
    field = (type*)ptr;                                                    \
  } while (0)
  ALLOC(c->p.st, uint8_t, g.Ntot);
  ALLOC(c->p.rf, uint8_t, g.Ntot);
  ALLOC(c->p.sigt, uint8_t, g.Ntot);
  ALLOC(c->p.ccode, uint8_t, g.Ntot);
  ALLOC(c->p.bsum, uint8_t, g.bs_off[L + 1]);
  ALLOC(c->p.wsum, uint8_t, g.bs_off[L + 1]);
  ALLOC(c->p.nsum, uint8_t, g.bs_off[L + 1]);
  for (int sl = 0; sl < SL_COUNT; sl++) ALLOC(c->p.q[sl], double, (int64_t)g.m * g.Ntot);
  ALLOC(c->p.regc, double, g.rc_off[L]);
  ALLOC(c->p.regf, double, g.rf_off[L]);
  c->p.rflux = nullptr;
  if (g.m >= 4) ALLOC(c->p.rflux, double, g.rc_off[L]);
  ALLOC(c->dt_d, double, n_inst);
  ALLOC(c->eps_d, double, n_inst);
  ALLOC(c->p.cnt, unsigned long long, (int64_t)n_inst * CNT_PER_INST);
  ALLOC(c->blockcnt_d, int, c->max_blocks + 1);
  ALLOC(c->total_d, long long, 1);
  ALLOC(c->err_d, int, 1);
  ALLOC(c->ws_d, unsigned long long, n_inst);
  ALLOC(c->part_d, double, (int64_t)(c->max_blocks + 1) * g.m);
  for (int k = 0; k < LS_COUNT; k++) ALLOC(c->p.lst[k], int, g.Ntot);
  ALLOC(c->p.lcnt, int, LS_COUNT * (MRD_MAXLEV + 1));
  ALLOC(c->p.bcnt, int, LS_COUNT * (g.comp_first[L + 1] + 1));
  ALLOC(c->p.sbcnt, int, LS_COUNT * (g.sb_first[L + 1] + 1));
  ALLOC(c->p.sboff, int, LS_COUNT * (g.sb_first[L + 1] + 1));
  ALLOC(c->p.leafcnt, int, (int64_t)n_inst * (MRD_MAXLEV + 1));
  ALLOC(c->p.items, unsigned long long, 3);
  ALLOC(c->p.lflag, unsigned, MRD_MAXLEV + 1);
  ALLOC(c->p.vel, double, 2 * n_inst);
  if (flame) ALLOC(c->p.vfpart, double, g.comp_first[L + 1]);
  if (hipHostMalloc((void**)&c->ws_host, sizeof(double) * (size_t)n_inst, hipHostMallocDefault) != hipSuccess) {
    c->ws_host = nullptr;
    st = set_err(c, MR_ENOMEM, "pinned host buffer");
    goto fail;
  }
  ALLOC(c->p.near, unsigned long long, 2 * NEAR_CAP);
  ALLOC(c->p.near_n, unsigned long long, 1);
  ALLOC(c->iterb_d, long long, 1);
  ALLOC(c->lcap_d, uint8_t, n_inst);
#undef ALLOC
  c->p.dt = c->dt_d;
  c->p.eps = c->eps_d;
  c->p.iterb = c->iterb_d;
  c->p.lcap = c->lcap_d;
  // the zero fills of the allocations are queued on the context's own
  // non-blocking stream, which does not order with the null stream: the
  // upload goes behind them on the same stream (a blocking hipMemcpy could
  // land first and then be zeroed, leaving every threshold at 0)
  st = hip_check(c, hipMemcpyAsync(c->eps_d, c->eps.data(), sizeof(double) * n_inst, hipMemcpyHostToDevice,
                                   c->stream),
                 "eps upload");
  if (st != MR_OK) goto fail;
  st = hip_check(c, hipMemcpyAsync(c->lcap_d, c->lcap_host.data(), n_inst, hipMemcpyHostToDevice, c->stream),
                 "finest level upload");
  if (st != MR_OK) goto fail;
  st = hip_check(c, hipStreamSynchronize(c->stream), "init");
  if (st != MR_OK) goto fail;
  *out = c;
  return MR_OK;
fail:
  mr_destroy(c);
  return st;
}

mr_status mr_init(int dim, int L, double eps, const mr_scheme* s, const mr_alloc* a, mr_ctx** out) {
  return mr_init_batch(dim, L, 1, &eps, s, a, out);
}

mr_status mr_set_stream(mr_ctx* c, void* hip_stream) {
  if (!c) return MR_EINVAL;
  c->stream = hip_stream ? (hipStream_t)hip_stream : c->own_stream;
  return MR_OK;
}

mr_status mr_synchronize(mr_ctx* c) {
  if (!c) return MR_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return MR_OK;
}

mr_status mr_load_finest(mr_ctx* c, const double* q0, void* hip_stream) {
  if (!c || !q0) return MR_EINVAL;
  if (hip_stream) c->stream = (hipStream_t)hip_stream;
  const Geo& g = c->g;
  std::fill(c->lcap_host.begin(), c->lcap_host.end(), (uint8_t)g.L);
  {
    mr_status su = upload_lcap(c);
    if (su != MR_OK) return su;
  }
  for (int lev = g.l0; lev < g.L; lev++) launch_fill_status(g, c->p, lev, ST_INTERNAL, c->stream);
  launch_load_finest(g, c->p, q0, -1, g.L, c->stream);
  launch_clear_regs(g, c->p, c->stream);
  refresh_lists(c, g.l0, true);
  HIPCHK(c, hipMemsetAsync(c->p.cnt, 0, sizeof(unsigned long long) * g.B * CNT_PER_INST, c->stream));
  HIPCHK(c, hipMemsetAsync(c->p.near_n, 0, sizeof(unsigned long long), c->stream));
  mr_status st = check_launch(c, "load_finest");
  if (st != MR_OK) return st;
  std::fill(c->t.begin(), c->t.end(), 0.0);
  std::fill(c->it_start.begin(), c->it_start.end(), 0);
  c->iters = 0;
  c->broken = false;
  c->err.clear();
  return adapt_impl(c);
}

__global__ void k_reset_counters(unsigned long long* cnt, int inst);

static mr_status load_inst_impl(mr_ctx* c, int inst, int Li, const double* q0) {
  if (c->broken) return set_err(c, MR_ESTATE, "context in error state");
  Geo& g = c->g;
  c->lcap_host[inst] = (uint8_t)Li;
  {
    mr_status su = upload_lcap(c);
    if (su != MR_OK) return su;
  }
  launch_fill_instance(g, c->p, inst, Li, c->stream);
  launch_load_finest(g, c->p, q0, inst, Li, c->stream);
  launch_clear_regs(g, c->p, c->stream);
  k_reset_counters<<<1, 64, 0, c->stream>>>(c->p.cnt, inst);
  refresh_lists(c, g.l0, true);
  project_range(c, g.L - 1, g.l0, PJ_Q0);
  c->it_start[inst] = c->iters;
  {
    mr_status su = upload_iter_base(c);
    if (su != MR_OK) return su;
  }
  if (g.l0 <= g.L - 1) {
    // only this instance is remeshed; the others keep their trees
    g.i0 = inst;
    g.i1 = inst + 1;
    remesh(c, g.l0);
    g.i0 = 0;
    g.i1 = g.B;
    project_range(c, g.L - 1, g.l0, PJ_Q0);
  }
  c->t[inst] = 0.0;
  mr_status st = check_launch(c, "load_finest_inst");
  if (st != MR_OK) return st;
  return check_flags(c);
}

mr_status mr_load_finest_inst(mr_ctx* c, int inst, const double* q0) {
  if (!c || !q0 || inst < 0 || inst >= c->g.B) return MR_EINVAL;
  return load_inst_impl(c, inst, c->g.L, q0);
}

mr_status mr_load_inst(mr_ctx* c, int inst, int L_inst, double eps, const double* q0) {
  if (!c || !q0 || inst < 0 || inst >= c->g.B) return MR_EINVAL;
  if (L_inst < c->g.l0 || L_inst > c->g.L) return set_err(c, MR_EINVAL, "instance finest level outside l0..L");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return set_err(c, MR_EINVAL, "eps must be finite and >= 0");
  c->eps[inst] = eps;
  HIPCHK(c, hipMemcpyAsync(c->eps_d, c->eps.data(), sizeof(double) * c->g.B, hipMemcpyHostToDevice, c->stream));
  return load_inst_impl(c, inst, L_inst, q0);
}

mr_status mr_clear_instance(mr_ctx* c, int inst) {
  if (!c || inst < 0 || inst >= c->g.B) return MR_EINVAL;
  launch_fill_instance(c->g, c->p, -1 - inst, c->g.L, c->stream);
  k_reset_counters<<<1, 64, 0, c->stream>>>(c->p.cnt, inst);
  refresh_lists(c, c->g.l0, true);
  c->t[inst] = 0.0;
  mr_status st = check_launch(c, "clear_instance");
  if (st != MR_OK) return st;
  // a failure of this instance no longer blocks the others
  st = read_counters(c);
  if (st != MR_OK) return st;
  bool any = false;
  for (int i = 0; i < c->g.B; i++)
    any = any || c->cnt_host[i * CNT_PER_INST + CNT_BAD] || c->cnt_host[i * CNT_PER_INST + CNT_NONFINITE];
  if (!any) {
    c->broken = false;
    c->err.clear();
  }
  return MR_OK;
}

mr_status mr_instance_flags(mr_ctx* c, int inst, int* flags) {
  if (!c || !flags || inst < 0 || inst >= c->g.B) return MR_EINVAL;
  mr_status st = read_counters(c);
  if (st != MR_OK) return st;
  *flags = (c->cnt_host[inst * CNT_PER_INST + CNT_NONFINITE] ? 1 : 0) |
           (c->cnt_host[inst * CNT_PER_INST + CNT_BAD] ? 2 : 0);
  return MR_OK;
}

mr_status mr_set_eps(mr_ctx* c, int inst, double eps) {
  if (!c || inst < 0 || inst >= c->g.B || !(eps >= 0.0) || !std::isfinite(eps)) return MR_EINVAL;
  c->eps[inst] = eps;
  HIPCHK(c, hipMemcpyAsync(c->eps_d, c->eps.data(), sizeof(double) * c->g.B, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return MR_OK;
}

mr_status mr_adapt(mr_ctx* c) {
  if (!c) return MR_EINVAL;
  if (c->broken) return set_err(c, MR_ESTATE, "context in error state");
  return adapt_impl(c);
}

// start of a macro step: the flames' frame velocity from the synchronised
// leaves (Sec. 5: v_f is the integral of the reaction rate)
static void macro_begin(mr_ctx* c) {
  if (c->g.flame_speed) launch_flame_speed(c->g, c->p, c->stream);
}

}  // extern "C"

// queue one macro step (no wait); ctx_step_finish waits and checks the flags
mr_status ctx_step_enqueue(mr_ctx* c, const double* dt) {
  if (!c || !dt) return MR_EINVAL;
  if (c->broken) return set_err(c, MR_ESTATE, "context in error state: reload or set leaves");
  for (int i = 0; i < c->g.B; i++)
    if (!(dt[i] > 0.0) || !std::isfinite(dt[i])) return set_err(c, MR_EINVAL, "dt_L must be positive");
  c->dt_host.assign(dt, dt + c->g.B);
  HIPCHK(c, hipMemcpyAsync(c->dt_d, c->dt_host.data(), sizeof(double) * c->g.B, hipMemcpyHostToDevice, c->stream));
  const int64_t N = (int64_t)1 << (c->g.L - c->g.l0);
  {
    mr_status su = upload_iter_base(c);
    if (su != MR_OK) return su;
  }
  // The launch sequence of a macro step depends only on the iteration index
  // and the kernels read counts, lists and dt from device memory, so the whole
  // macro step is captured once into a HIP graph and replayed.
  if (c->use_graph && c->timed_class == 0 && c->stream != nullptr) {
    if (!c->graph_exec) {
      HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
      macro_begin(c);
      for (int64_t n = 0; n < N; n++) lt_iteration(c, n, N);
      hipGraph_t gr = nullptr;
      HIPCHK(c, hipStreamEndCapture(c->stream, &gr));
      c->graph = gr;
      HIPCHK(c, hipGraphInstantiate(&c->graph_exec, gr, nullptr, nullptr, 0));
    }
    HIPCHK(c, hipGraphLaunch(c->graph_exec, c->stream));
  } else {
    macro_begin(c);
    for (int64_t n = 0; n < N; n++) lt_iteration(c, n, N);
  }
  mr_status st = check_launch(c, "lt_step");
  if (st != MR_OK) return st;
  for (int i = 0; i < c->g.B; i++) c->t[i] = c->t[i] + (double)N * dt[i];
  c->iters += N;
  return MR_OK;
}

mr_status ctx_step_finish(mr_ctx* c) { return check_flags(c); }

// queue the wave-speed reduction into the pinned buffer; ctx_wavespeed_finish
// waits and returns it
mr_status ctx_wavespeed_enqueue(mr_ctx* c) {
  const Geo& g = c->g;
  if (g.flame_speed) launch_flame_speed(g, c->p, c->stream);
  HIPCHK(c, hipMemsetAsync(c->ws_d, 0, sizeof(unsigned long long) * g.B, c->stream));
  for (int lev = g.l0; lev <= g.L; lev++) launch_wavespeed(g, c->p, lev, c->ws_d, c->stream);
  HIPCHK(c, hipMemcpyAsync(c->ws_host, c->ws_d, sizeof(double) * g.B, hipMemcpyDeviceToHost, c->stream));
  return check_launch(c, "max_wavespeed");
}

mr_status ctx_wavespeed_finish(mr_ctx* c, double* out) {
  HIPCHK(c, hipStreamSynchronize(c->stream));
  memcpy(out, c->ws_host, sizeof(double) * c->g.B);  // the bits of non-negative doubles
  return MR_OK;
}

size_t ctx_footprint(const mr_ctx* c) { return c ? c->bytes : 0; }

int ctx_instances(const mr_ctx* c) { return c ? c->g.B : 0; }

extern "C" {

mr_status mr_lt_step_batch(mr_ctx* c, const double* dt) {
  mr_status st = ctx_step_enqueue(c, dt);
  if (st != MR_OK) return st;
  return ctx_step_finish(c);
}

mr_status mr_footprint(mr_ctx* c, size_t* bytes) {
  if (!c || !bytes) return MR_EINVAL;
  *bytes = c->bytes;
  return MR_OK;
}

mr_status mr_lt_step(mr_ctx* c, double dt_L) {
  if (!c) return MR_EINVAL;
  std::vector<double> dt((size_t)c->g.B, dt_L);
  return mr_lt_step_batch(c, dt.data());
}

mr_status mr_reconstruct(mr_ctx* c, double* q_out) {
  if (!c || !q_out) return MR_EINVAL;
  const Geo& g = c->g;
  project_range(c, g.L - 1, g.l0, PJ_Q0);
  double* dense = c->p.q[SL_H1];
  for (int lev = g.l0; lev <= g.L; lev++) launch_recon_level(g, c->p, lev, dense, c->stream);
  launch_to_rowmajor(g, dense, q_out, c->stream);
  mr_status st = check_launch(c, "reconstruct");
  if (st != MR_OK) return st;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return MR_OK;
}

mr_status mr_set_launch(mr_ctx* c, const mr_launch* l) {
  if (!c || !l) return MR_EINVAL;
  const int32_t v[3] = {l->list_grid, l->iface_grid, l->comp_grid};
  for (int j = 0; j < 3; j++)
    if (v[j] < 0 || v[j] > 65535) return set_err(c, MR_EINVAL, "launch grid outside 0..65535");
  if (l->bulk_levels < 0 || l->bulk_levels > 2) return set_err(c, MR_EINVAL, "bulk_levels outside 0..2");
  if (l->list_grid) c->g.list_grid = l->list_grid;
  if (l->iface_grid) c->g.iface_grid = l->iface_grid;
  if (l->comp_grid) c->g.comp_grid = l->comp_grid;
  if (l->bulk_levels) c->g.bulk_split = l->bulk_levels == 2 ? 1 : 0;
  // the captured macro step holds the old grids (destroyed once no replay
  // of it is in flight)
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->graph_exec = nullptr;
  c->graph = nullptr;
  return MR_OK;
}

mr_status mr_get_launch(mr_ctx* c, mr_launch* l) {
  if (!c || !l) return MR_EINVAL;
  l->list_grid = c->g.list_grid;
  l->iface_grid = c->g.iface_grid;
  l->comp_grid = c->g.comp_grid;
  l->bulk_levels = c->g.bulk_split ? 2 : 1;
  return MR_OK;
}

mr_status mr_flame_speed(mr_ctx* c, double* vf) {
  if (!c || !vf) return MR_EINVAL;
  const Geo& g = c->g;
  if (g.pde != PDE_FLAME && g.pde != PDE_FLAMEBALL) return set_err(c, MR_EINVAL, "not a flame problem");
  launch_flame_speed(g, c->p, c->stream);
  HIPCHK(c, hipMemcpyAsync(vf, c->p.vel + g.B, sizeof(double) * g.B, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return check_launch(c, "flame_speed");
}

mr_status mr_max_wavespeed(mr_ctx* c, double* out) {
  if (!c || !out) return MR_EINVAL;
  mr_status st = ctx_wavespeed_enqueue(c);
  if (st != MR_OK) return st;
  return ctx_wavespeed_finish(c, out);
}

mr_status mr_get_leaves_inst(mr_ctx* c, int inst, uint64_t* keys, double* q, int64_t cap, int64_t* n) {
  if (!c || !n || inst < 0 || inst >= c->g.B) return MR_EINVAL;
  const Geo& g = c->g;
  std::vector<long long> per(MR_MAXLEV + 1, 0);
  long long tot = 0;
  for (int lev = g.l0; lev <= g.L; lev++) {
    mr_status st = level_count(c, lev, inst, ST_LEAF, &per[lev]);
    if (st != MR_OK) return st;
    tot += per[lev];
  }
  *n = tot;
  if (!keys || !q) return MR_OK;
  if (cap < tot) return set_err(c, MR_ECAPACITY, "leaf buffer too small");
  void* kd = raw_alloc(c, sizeof(unsigned long long) * (size_t)(tot + 1));
  void* vd = kd ? raw_alloc(c, sizeof(double) * (size_t)(tot + 1) * g.m) : nullptr;
  if (!vd) {
    raw_free(c, kd);
    return set_err(c, MR_ENOMEM, "leaf staging buffer");
  }
  long long base = 0;
  for (int lev = g.l0; lev <= g.L; lev++) {
    const int nblk = (int)((g.n[lev] + 255) / 256);
    launch_count(g, c->p, lev, inst, ST_LEAF, c->blockcnt_d, nblk, c->stream);
    launch_scan_blocks(c->blockcnt_d, nblk, c->total_d, c->stream);
    launch_gather_leaves(g, c->p, lev, inst, c->blockcnt_d, nblk, base, (unsigned long long*)kd, (double*)vd,
                         tot, c->stream);
    base += per[lev];
  }
  hipError_t e1 = hipMemcpyAsync(keys, kd, sizeof(uint64_t) * (size_t)tot, hipMemcpyDeviceToHost, c->stream);
  hipError_t e2 = hipMemcpyAsync(q, vd, sizeof(double) * (size_t)tot * g.m, hipMemcpyDeviceToHost, c->stream);
  hipError_t e3 = hipStreamSynchronize(c->stream);
  raw_free(c, kd);
  raw_free(c, vd);
  HIPCHK(c, e1);
  HIPCHK(c, e2);
  HIPCHK(c, e3);
  return check_launch(c, "get_leaves");
}

mr_status mr_get_leaves(mr_ctx* c, uint64_t* keys, double* q, int64_t cap, int64_t* n) {
  return mr_get_leaves_inst(c, 0, keys, q, cap, n);
}

mr_status mr_get_leaves_noalloc(mr_ctx* c, int inst, uint64_t* keys, double* q, int64_t cap, int64_t* n) {
  if (!c || !n || inst < 0 || inst >= c->g.B) return MR_EINVAL;
  const Geo& g = c->g;
  std::vector<long long> per(MR_MAXLEV + 1, 0);
  long long tot = 0;
  for (int lev = g.l0; lev <= g.L; lev++) {
    mr_status st = level_count(c, lev, inst, ST_LEAF, &per[lev]);
    if (st != MR_OK) return st;
    tot += per[lev];
  }
  *n = tot;
  if (!keys || !q) return MR_OK;
  if (cap < tot) return set_err(c, MR_ECAPACITY, "leaf buffer too small");
  if (tot > MR_NOALLOC_MAX_LEAVES)
    return set_err(c, MR_ECAPACITY, "more leaves than the staging array of mr_get_leaves_noalloc holds");
  unsigned long long* kd = (unsigned long long*)c->scratch_d;
  double* vd = (double*)((unsigned char*)c->scratch_d + (size_t)MR_NOALLOC_MAX_LEAVES * 8u);
  long long base = 0;
  for (int lev = g.l0; lev <= g.L; lev++) {
    const int nblk = (int)((g.n[lev] + 255) / 256);
    launch_count(g, c->p, lev, inst, ST_LEAF, c->blockcnt_d, nblk, c->stream);
    launch_scan_blocks(c->blockcnt_d, nblk, c->total_d, c->stream);
    launch_gather_leaves(g, c->p, lev, inst, c->blockcnt_d, nblk, base, kd, vd, tot, c->stream);
    base += per[lev];
  }
  if (tot > 0) {
    HIPCHK(c, hipMemcpyAsync(keys, kd, sizeof(uint64_t) * (size_t)tot, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(q, vd, sizeof(double) * (size_t)tot * g.m, hipMemcpyDeviceToHost, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return check_launch(c, "get_leaves_noalloc");
}

__global__ void k_fill_range(uint8_t* st, int64_t base, int64_t n, uint8_t v) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    st[base + t] = v;
}

__global__ void k_reset_counters(unsigned long long* cnt, int inst) {
  if (threadIdx.x < CNT_PER_INST) cnt[inst * CNT_PER_INST + threadIdx.x] = 0;
}

mr_status mr_set_leaves_inst(mr_ctx* c, int inst, const uint64_t* keys, const double* q, int64_t n, double t) {
  if (!c || inst < 0 || inst >= c->g.B || n < 0 || (n > 0 && (!keys || !q))) return MR_EINVAL;
  const Geo& g = c->g;
  for (int lev = g.l0; lev <= g.L; lev++) {
    const int64_t base = g.off[lev] + (int64_t)inst * g.n[lev];
    k_fill_range<<<blocks_for(g.n[lev]), 256, 0, c->stream>>>(c->p.st, base, g.n[lev], ST_ABSENT);
  }
  void* kd = raw_alloc(c, sizeof(uint64_t) * (size_t)(n + 1));
  void* vd = kd ? raw_alloc(c, sizeof(double) * (size_t)(n + 1) * g.m) : nullptr;
  if (!vd) {
    raw_free(c, kd);
    return set_err(c, MR_ENOMEM, "leaf staging buffer");
  }
  int herr = 0;
  hipError_t e = hipMemsetAsync(c->err_d, 0, sizeof(int), c->stream);
  if (e == hipSuccess && n > 0)
    e = hipMemcpyAsync(kd, keys, sizeof(uint64_t) * (size_t)n, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess && n > 0)
    e = hipMemcpyAsync(vd, q, sizeof(double) * (size_t)n * g.m, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) {
    launch_scatter_leaves(g, c->p, inst, (const unsigned long long*)kd, (const double*)vd, n, c->err_d, c->stream);
    for (int lev = g.L; lev > g.l0; lev--) launch_mark_parents(g, c->p, lev, c->err_d, c->stream);
    for (int lev = g.l0; lev <= g.L; lev++) launch_validate(g, c->p, lev, c->err_d, c->stream);
    e = hipMemcpyAsync(&herr, c->err_d, sizeof(int), hipMemcpyDeviceToHost, c->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  raw_free(c, kd);
  raw_free(c, vd);
  HIPCHK(c, e);
  if (herr) {
    char buf[96];
    snprintf(buf, sizeof buf, "leaves do not form a complete graded tree (code %d)", herr);
    c->broken = true;
    return set_err(c, MR_EINVAL, buf);
  }
  launch_compact(g, c->p, g.l0, true, c->stream);  // internal lists for the projection
  project_range(c, g.L - 1, g.l0, PJ_Q0);
  launch_clear_regs(g, c->p, c->stream);
  refresh_lists(c, g.l0, true);
  k_reset_counters<<<1, 64, 0, c->stream>>>(c->p.cnt, inst);
  mr_status st = check_launch(c, "set_leaves");
  if (st != MR_OK) return st;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->t[inst] = t;
  c->it_start[inst] = c->iters;
  c->lcap_host[inst] = (uint8_t)g.L;
  {
    mr_status su = upload_lcap(c);
    if (su != MR_OK) return su;
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  c->broken = false;
  c->err.clear();
  return MR_OK;
}

mr_status mr_set_leaves(mr_ctx* c, const uint64_t* keys, const double* q, int64_t n, double t) {
  return mr_set_leaves_inst(c, 0, keys, q, n, t);
}

mr_status mr_stats_inst(mr_ctx* c, int inst, mr_stats_t* out) {
  if (!c || !out || inst < 0 || inst >= c->g.B) return MR_EINVAL;
  const Geo& g = c->g;
  memset(out, 0, sizeof *out);
  out->t = c->t[inst];
  out->iterations = c->iters;
  std::vector<double> part;
  for (int lev = g.l0; lev <= g.L; lev++) {
    long long nl = 0;
    mr_status st = level_count(c, lev, inst, ST_LEAF, &nl);
    if (st != MR_OK) return st;
    out->leaves[lev] = nl;
    const int nblk = (int)((g.n[lev] + 255) / 256);
    launch_mass_partial(g, c->p, lev, inst, c->part_d, nblk, c->stream);
    part.resize((size_t)nblk * g.m);
    HIPCHK(c, hipMemcpyAsync(part.data(), c->part_d, sizeof(double) * part.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int b = 0; b < nblk; b++)
      for (int k = 0; k < g.m; k++) out->mass[k] = out->mass[k] + part[(size_t)b * g.m + k];
  }
  mr_status st = read_counters(c);
  if (st != MR_OK) return st;
  for (int lev = g.l0; lev <= g.L; lev++)
    out->leaf_updates += (int64_t)c->cnt_host[inst * CNT_PER_INST + CNT_LEVEL0 + lev];
  out->near_threshold = (int64_t)c->cnt_host[inst * CNT_PER_INST + CNT_NEAR];
  return check_launch(c, "stats");
}

mr_status mr_stats(mr_ctx* c, mr_stats_t* out) { return mr_stats_inst(c, 0, out); }

mr_status mr_near_threshold(mr_ctx* c, int inst, int64_t* iter, int32_t* level, uint64_t* key, int64_t cap,
                            int64_t* n) {
  if (!c || !n || inst < 0 || inst >= c->g.B) return MR_EINVAL;
  unsigned long long cnt = 0;
  HIPCHK(c, hipMemcpyAsync(&cnt, c->p.near_n, sizeof cnt, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (cnt > NEAR_CAP) return set_err(c, MR_ECAPACITY, "near-threshold list overflowed (more than 65536 decisions)");
  std::vector<unsigned long long> raw(2 * (size_t)cnt + 2);
  if (cnt) {
    HIPCHK(c, hipMemcpyAsync(raw.data(), c->p.near, sizeof(unsigned long long) * 2 * cnt, hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  struct E { int64_t it; int32_t lev; uint64_t key; };
  std::vector<E> v;
  for (unsigned long long j = 0; j < cnt; j++) {
    const unsigned long long w = raw[2 * j + 1];
    const int64_t it = (int64_t)raw[2 * j];
    if ((int)(w >> 45) != inst || it < c->it_start[inst]) continue;
    // in the instance's own iterations: its finest level takes one
    // iteration per 2^{L - Li} of the context's
    const int sh = c->g.L - c->lcap_host[inst];
    v.push_back(E{(it - c->it_start[inst]) >> sh, (int32_t)((w >> 40) & 31u), w & ((1ull << 40) - 1)});
  }
  std::sort(v.begin(), v.end(), [](const E& a, const E& b) {
    if (a.it != b.it) return a.it < b.it;
    if (a.lev != b.lev) return a.lev < b.lev;
    return a.key < b.key;
  });
  *n = (int64_t)v.size();
  if (!iter || !level || !key) return MR_OK;
  if (cap < (int64_t)v.size()) return set_err(c, MR_ECAPACITY, "near-threshold buffer too small");
  for (size_t j = 0; j < v.size(); j++) {
    iter[j] = v[j].it;
    level[j] = v[j].lev;
    key[j] = v[j].key;
  }
  return MR_OK;
}

mr_status mr_level_updates(mr_ctx* c, int inst, int64_t* per_level) {
  if (!c || !per_level || inst < 0 || inst >= c->g.B) return MR_EINVAL;
  mr_status st = read_counters(c);
  if (st != MR_OK) return st;
  for (int lev = 0; lev <= MR_MAXLEV; lev++)
    per_level[lev] = (lev >= c->g.l0 && lev <= c->g.L) ? (int64_t)c->cnt_host[inst * CNT_PER_INST + CNT_LEVEL0 + lev] : 0;
  return MR_OK;
}

mr_status mr_stage_items(mr_ctx* c, int64_t* per_stage) {
  if (!c || !per_stage) return MR_EINVAL;
  unsigned long long h[3] = {0ull, 0ull, 0ull};
  HIPCHK(c, hipMemcpyAsync(h, c->p.items, sizeof h, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int i = 0; i < 3; i++) per_stage[i] = (int64_t)h[i];
  return MR_OK;
}

mr_status mr_timing_start(mr_ctx* c, int kernel_class) {
  if (!c || kernel_class < MR_KC_STAGE_FINEST || kernel_class > MR_KC_STAGE_BULK) return MR_EINVAL;
  c->timed_class = kernel_class;
  c->ev_used = 0;
  return MR_OK;
}

mr_status mr_timing_stop(mr_ctx* c, double* total_ms, int64_t* launches) {
  if (!c || !total_ms || !launches) return MR_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double tot = 0.0;
  for (size_t i = 0; i + 1 < c->ev_used; i += 2) {
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]));
    tot += ms;
  }
  *total_ms = tot;
  *launches = (int64_t)(c->ev_used / 2);
  c->timed_class = 0;
  c->ev_used = 0;
  return MR_OK;
}

}  // extern "C"
