// batch.hip -- the systems forms behind the C ABI: solves of uneven size
// grouped in classes, one context per class, admitted by device footprint,
// stepped together with per-solve CFL steps, retired at their final time.
//
// A class's context has the class's largest finest level; a solve with a
// smaller finest level L runs in it with dt_L scaled by 2^{L - L_max}
// (mr_load_inst), so one macro step of the context is one macro step of
// every solve in it.  Classes step on their own streams: the wave speeds of
// all classes are queued before the first wait, then the macro steps of all
// classes, then the waits.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "mrlt.h"

// context internals (runtime.hip)
mr_status ctx_step_enqueue(mr_ctx* c, const double* dt);
mr_status ctx_step_finish(mr_ctx* c);
mr_status ctx_wavespeed_enqueue(mr_ctx* c);
mr_status ctx_wavespeed_finish(mr_ctx* c, double* out);
size_t ctx_footprint(const mr_ctx* c);

namespace {

struct Slot {
  int state = MR_SLOT_FREE;
  mr_instance_desc d{};
  double t = 0.0;
  int64_t steps = 0;
  std::vector<uint64_t> keys;  // result of a finished solve
  std::vector<double> q;
};

struct Class {
  mr_class_desc desc{};
  mr_ctx* ctx = nullptr;
  int first = 0;  // global number of its slot 0
  std::vector<Slot> slots;
  uint64_t last_use = 0;

  bool busy() const {
    for (const Slot& s : slots)
      if (s.state == MR_SLOT_RUNNING) return true;
    return false;
  }
};

bool same_scheme(const mr_scheme& a, const mr_scheme& b, int dim) {
  if (a.pde != b.pde || a.rk != b.rk || a.lt != b.lt || a.l0 != b.l0 || a.recon != b.recon ||
      a.thresh != b.thresh || a.reflux != b.reflux || a.remesh != b.remesh || a.flame_speed != b.flame_speed)
    return false;
  for (int ax = 0; ax < dim; ax++) {
    if (a.bc[ax][0] != b.bc[ax][0] || a.bc[ax][1] != b.bc[ax][1]) return false;
    if (a.lo[ax] != b.lo[ax] || a.hi[ax] != b.hi[ax] || a.adv_vel[ax] != b.adv_vel[ax]) return false;
  }
  if (a.nu != b.nu || a.k_react != b.k_react || a.a_react != b.a_react || a.gamma != b.gamma) return false;
  for (int k = 0; k < 5; k++)
    if (a.detail_scale[k] != b.detail_scale[k]) return false;
  return a.ze == b.ze && a.tau == b.tau && a.lewis == b.lewis && a.kappa == b.kappa;
}

int ncomp_of(const mr_scheme& s, int dim) {
  return s.pde == MR_PDE_EULER ? dim + 2 : (s.pde == MR_PDE_FLAMEBALL ? 2 : 1);
}

}  // namespace

struct mr_batch {
  std::vector<Class> cls;
  size_t budget = 0;
  mr_alloc alloc{};
  bool has_alloc = false;
  std::string err;
  std::vector<int> done;  // finished or failed slots not yet polled
  uint64_t tick = 0;
};

namespace {

mr_status berr(mr_batch* b, mr_status st, const std::string& msg) {
  b->err = msg;
  return st;
}

bool locate(mr_batch* b, int slot, Class** c, Slot** s, int* local) {
  for (Class& k : b->cls)
    if (slot >= k.first && slot < k.first + (int)k.slots.size()) {
      *c = &k;
      *local = slot - k.first;
      *s = &k.slots[*local];
      return true;
    }
  return false;
}

size_t used_bytes(const mr_batch* b) {
  size_t u = 0;
  for (const Class& k : b->cls) u += ctx_footprint(k.ctx);
  return u;
}

// the class's context, created now if needed; contexts of classes without a
// running solve are destroyed (least recently used first) to keep the sum
// of footprints within the budget
mr_status ensure_context(mr_batch* b, Class& k) {
  if (k.ctx) return MR_OK;
  std::vector<double> eps(k.slots.size(), 0.0);
  mr_ctx* ctx = nullptr;
  mr_status st = mr_init_batch(k.desc.dim, k.desc.L_max, (int)k.slots.size(), eps.data(), &k.desc.scheme,
                               b->has_alloc ? &b->alloc : nullptr, &ctx);
  if (st != MR_OK) return berr(b, st == MR_ENOMEM ? MR_ECAPACITY : st, "class context could not be created");
  const size_t need = ctx_footprint(ctx);
  for (;;) {
    if (used_bytes(b) + need <= b->budget) break;
    Class* victim = nullptr;
    for (Class& o : b->cls) {
      if (!o.ctx || &o == &k || o.busy()) continue;
      bool held = false;  // a finished result is kept on the host, so DONE slots do not hold the context
      for (const Slot& s : o.slots) held = held || s.state == MR_SLOT_RUNNING;
      if (held) continue;
      if (!victim || o.last_use < victim->last_use) victim = &o;
    }
    if (!victim) {
      mr_destroy(ctx);
      return berr(b, MR_ECAPACITY, "class context does not fit the HBM budget");
    }
    mr_destroy(victim->ctx);
    victim->ctx = nullptr;
  }
  k.ctx = ctx;
  return MR_OK;
}

// finest step of one solve for its next macro step
double solve_dt(const mr_instance_desc& d, double ws, double t) {
  const mr_scheme& s = d.scheme;
  const double dx = (s.hi[0] - s.lo[0]) / std::ldexp(1.0, d.L);
  double diff = 0.0;
  if (s.pde == MR_PDE_BURGERS || s.pde == MR_PDE_NAGUMO || s.pde == MR_PDE_LINEAR) diff = s.nu;
  if (s.pde == MR_PDE_FLAME || s.pde == MR_PDE_FLAMEBALL) diff = s.lewis < 1.0 ? 1.0 / s.lewis : 1.0;
  double rate = ws / dx + 2.0 * d.dim * diff / (dx * dx);
  if (s.pde == MR_PDE_NAGUMO) rate += 0.8 * s.k_react;
  const double n_it = std::ldexp(1.0, d.L - s.l0);
  double dt = rate > 0.0 ? d.cfl / rate : (d.t_final - t) / n_it;
  if (d.dt_max > 0.0 && d.dt_max < dt) dt = d.dt_max;
  const double rest = (d.t_final - t) / n_it;
  return rest < dt ? rest : dt;
}

// keep a finished solve's leaves on the host and free its cells
mr_status retire(mr_batch* b, Class& k, int local, int state) {
  Slot& s = k.slots[local];
  if (state == MR_SLOT_DONE) {
    int64_t n = 0;
    mr_status st = mr_get_leaves_inst(k.ctx, local, nullptr, nullptr, 0, &n);
    if (st != MR_OK) return berr(b, st, mr_last_error(k.ctx));
    s.keys.resize((size_t)n);
    s.q.resize((size_t)n * ncomp_of(k.desc.scheme, k.desc.dim));
    st = mr_get_leaves_inst(k.ctx, local, s.keys.data(), s.q.data(), n, &n);
    if (st != MR_OK) return berr(b, st, mr_last_error(k.ctx));
  }
  mr_status st = mr_clear_instance(k.ctx, local);
  if (st != MR_OK) return berr(b, st, mr_last_error(k.ctx));
  s.state = state;
  b->done.push_back(k.first + local);
  return MR_OK;
}

}  // namespace

extern "C" {

mr_status mr_batch_create(int n_classes, const mr_class_desc* classes, size_t hbm_budget, const mr_alloc* a,
                          mr_batch** out) {
  if (!out) return MR_EINVAL;
  *out = nullptr;
  if (n_classes < 1 || !classes) return MR_EINVAL;
  if (a && ((a->alloc == nullptr) != (a->free == nullptr))) return MR_EINVAL;
  mr_batch* b = new mr_batch();
  b->budget = hbm_budget;
  if (a && a->alloc) {
    b->alloc = *a;
    b->has_alloc = true;
  }
  int first = 0;
  for (int i = 0; i < n_classes; i++) {
    const mr_class_desc& d = classes[i];
    if (d.dim < 1 || d.dim > 3 || d.slots < 1 || d.L_max < d.scheme.l0 || d.L_max > MR_MAXLEV) {
      delete b;
      return MR_EINVAL;
    }
    Class k;
    k.desc = d;
    k.first = first;
    k.slots.resize((size_t)d.slots);
    first += d.slots;
    b->cls.push_back(std::move(k));
  }
  *out = b;
  return MR_OK;
}

mr_status mr_batch_admit(mr_batch* b, const mr_instance_desc* d, const double* q0, int* slot) {
  if (!b || !d || !q0 || !slot) return MR_EINVAL;
  if (!(d->t_final > 0.0) || !(d->cfl > 0.0) || !(d->eps >= 0.0) || !std::isfinite(d->eps))
    return berr(b, MR_EINVAL, "bad solve description");
  bool matched = false;
  mr_status last = MR_ECAPACITY;
  std::string why = "no free slot in a matching class";
  for (Class& k : b->cls) {
    if (k.desc.dim != d->dim || d->L > k.desc.L_max || d->L < k.desc.scheme.l0 ||
        !same_scheme(k.desc.scheme, d->scheme, d->dim))
      continue;
    matched = true;
    int local = -1;
    for (size_t i = 0; i < k.slots.size(); i++)
      if (k.slots[i].state == MR_SLOT_FREE) {
        local = (int)i;
        break;
      }
    if (local < 0) continue;
    last = ensure_context(b, k);
    if (last != MR_OK) {
      why = b->err;
      continue;
    }
    mr_status st = mr_load_inst(k.ctx, local, d->L, d->eps, q0);
    if (st != MR_OK) return berr(b, st, mr_last_error(k.ctx));
    Slot& s = k.slots[(size_t)local];
    s = Slot();
    s.state = MR_SLOT_RUNNING;
    s.d = *d;
    k.last_use = ++b->tick;
    *slot = k.first + local;
    return MR_OK;
  }
  if (!matched) return berr(b, MR_EINVAL, "no class matches the solve");
  return berr(b, last == MR_OK ? MR_ECAPACITY : last, why);
}

mr_status mr_batch_step(mr_batch* b) {
  if (!b) return MR_EINVAL;
  std::vector<Class*> act;
  for (Class& k : b->cls)
    if (k.ctx && k.busy()) act.push_back(&k);
  for (Class* k : act) {
    mr_status st = ctx_wavespeed_enqueue(k->ctx);
    if (st != MR_OK) return berr(b, st, mr_last_error(k->ctx));
  }
  std::vector<std::vector<double>> dts(act.size());
  for (size_t j = 0; j < act.size(); j++) {
    Class& k = *act[j];
    std::vector<double> ws(k.slots.size());
    mr_status st = ctx_wavespeed_finish(k.ctx, ws.data());
    if (st != MR_OK) return berr(b, st, mr_last_error(k.ctx));
    dts[j].assign(k.slots.size(), 1.0);  // free slots hold no cell: any step
    for (size_t i = 0; i < k.slots.size(); i++) {
      const Slot& s = k.slots[i];
      if (s.state != MR_SLOT_RUNNING) continue;
      dts[j][i] = std::ldexp(solve_dt(s.d, ws[i], s.t), s.d.L - k.desc.L_max);
    }
    st = ctx_step_enqueue(k.ctx, dts[j].data());
    if (st != MR_OK) return berr(b, st, mr_last_error(k.ctx));
  }
  for (size_t j = 0; j < act.size(); j++) {
    Class& k = *act[j];
    mr_status st = ctx_step_finish(k.ctx);
    if (st == MR_ENONFINITE || st == MR_ESTATE) {
      // failed solves fail alone
      for (size_t i = 0; i < k.slots.size(); i++) {
        if (k.slots[i].state != MR_SLOT_RUNNING) continue;
        int flags = 0;
        if (mr_instance_flags(k.ctx, (int)i, &flags) == MR_OK && flags) {
          mr_status sr = retire(b, k, (int)i, MR_SLOT_FAILED);
          if (sr != MR_OK) return sr;
        }
      }
    } else if (st != MR_OK) {
      return berr(b, st, mr_last_error(k.ctx));
    }
    k.last_use = ++b->tick;
    for (size_t i = 0; i < k.slots.size(); i++) {
      Slot& s = k.slots[i];
      if (s.state != MR_SLOT_RUNNING) continue;
      s.t = s.t + std::ldexp(1.0, k.desc.L_max - k.desc.scheme.l0) * dts[j][i];
      s.steps++;
      if (s.t >= s.d.t_final * (1.0 - 1e-12)) {
        mr_status sr = retire(b, k, (int)i, MR_SLOT_DONE);
        if (sr != MR_OK) return sr;
      }
    }
  }
  return MR_OK;
}

mr_status mr_batch_poll(mr_batch* b, int* done_slots, int cap, int* n) {
  if (!b || !n || (cap > 0 && !done_slots)) return MR_EINVAL;
  const int k = (int)b->done.size() < cap ? (int)b->done.size() : cap;
  for (int i = 0; i < k; i++) done_slots[i] = b->done[(size_t)i];
  b->done.erase(b->done.begin(), b->done.begin() + k);
  *n = k;
  return MR_OK;
}

mr_status mr_batch_slot_info(mr_batch* b, int slot, int* state, double* t, int64_t* macro_steps) {
  Class* k;
  Slot* s;
  int local;
  if (!b || !locate(b, slot, &k, &s, &local)) return MR_EINVAL;
  if (state) *state = s->state;
  if (t) *t = s->t;
  if (macro_steps) *macro_steps = s->steps;
  return MR_OK;
}

mr_status mr_batch_get_leaves(mr_batch* b, int slot, uint64_t* keys, double* q, int64_t cap, int64_t* n) {
  Class* k;
  Slot* s;
  int local;
  if (!b || !n || !locate(b, slot, &k, &s, &local)) return MR_EINVAL;
  if (s->state == MR_SLOT_RUNNING) return mr_get_leaves_inst(k->ctx, local, keys, q, cap, n);
  if (s->state != MR_SLOT_DONE) return berr(b, MR_ESTATE, "slot holds no solve");
  *n = (int64_t)s->keys.size();
  if (!keys || !q) return MR_OK;
  if (cap < *n) return berr(b, MR_ECAPACITY, "leaf buffer too small");
  memcpy(keys, s->keys.data(), sizeof(uint64_t) * s->keys.size());
  memcpy(q, s->q.data(), sizeof(double) * s->q.size());
  return MR_OK;
}

mr_status mr_batch_release(mr_batch* b, int slot) {
  Class* k;
  Slot* s;
  int local;
  if (!b || !locate(b, slot, &k, &s, &local)) return MR_EINVAL;
  if (s->state == MR_SLOT_RUNNING && k->ctx) {
    mr_status st = mr_clear_instance(k->ctx, local);
    if (st != MR_OK) return berr(b, st, mr_last_error(k->ctx));
  }
  *s = Slot();
  return MR_OK;
}

mr_status mr_batch_footprint(mr_batch* b, size_t* bytes) {
  if (!b || !bytes) return MR_EINVAL;
  *bytes = used_bytes(b);
  return MR_OK;
}

const char* mr_batch_last_error(const mr_batch* b) { return b ? b->err.c_str() : "null batch"; }

void mr_batch_destroy(mr_batch* b) {
  if (!b) return;
  for (Class& k : b->cls) mr_destroy(k.ctx);
  delete b;
}

}  // extern "C"
