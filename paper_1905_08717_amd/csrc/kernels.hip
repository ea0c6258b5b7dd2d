// kernels.hip -- HIP kernels of the MRLT/NERK3 macro step for gfx950.
//
// Every kernel walks one level of every instance of a batch with a
// grid-stride loop over the level's Morton-indexed cells (instance in the
// high bits of the loop index).  FP64 throughout; the library is built with
// -ffp-contract=off so each expression rounds exactly as written.
//
// Method: arXiv:1905.08717 (Lopes, Domingues, Mendes, Schneider), Secs. 2-4
// and the appendix algorithms; readings where the paper is silent are noted
// where they are used.
#include "mrlt_internal.h"
#include "group_codes.h"

#define GSL(t, N) \
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < (N); \
       t += (int64_t)gridDim.x * blockDim.x)

static constexpr int TPB = 256;

// s_waitcnt vmcnt(0) alone (expcnt and lgkmcnt at their no-wait maxima)
__device__ __forceinline__ void vm_wait_all() { __builtin_amdgcn_s_waitcnt(0x0F70); }

int blocks_for(int64_t n) {
  int64_t b = (n + TPB - 1) / TPB;
  if (b < 1) b = 1;
  if (b > 2048) b = 2048;  // 8 waves per CU on 256 CUs; loops stride over the rest
  return (int)b;
}
// grid of the list-driven kernels (stage, ghost, projection, finalize): at
// most g.list_grid workgroups, the loops stride over the rest (a launch knob
// of the context, tuned by measurement; results do not depend on it)
int list_blocks(const Geo& g, int64_t n) {
  int64_t b = (n + TPB - 1) / TPB;
  if (b < 1) b = 1;
  if (b > g.list_grid) b = g.list_grid;
  return (int)b;
}

// ---------------------------------------------------------------------------
// Morton keys and boundary maps

// Within-instance Morton keys have at most 30 bits (a level holds fewer
// than 2^30 cells per instance), so the bit interleaving works on 32-bit
// words: spread / compact by binary magic numbers (the shift-or-mask
// construction for interleaved codes), one instruction per step.
__device__ __forceinline__ uint32_t part1by1(uint32_t x) {  // x < 2^15
  x &= 0x0000ffffu;
  x = (x | (x << 8)) & 0x00ff00ffu;
  x = (x | (x << 4)) & 0x0f0f0f0fu;
  x = (x | (x << 2)) & 0x33333333u;
  x = (x | (x << 1)) & 0x55555555u;
  return x;
}
__device__ __forceinline__ uint32_t compact1by1(uint32_t x) {
  x &= 0x55555555u;
  x = (x | (x >> 1)) & 0x33333333u;
  x = (x | (x >> 2)) & 0x0f0f0f0fu;
  x = (x | (x >> 4)) & 0x00ff00ffu;
  x = (x | (x >> 8)) & 0x0000ffffu;
  return x;
}
__device__ __forceinline__ uint32_t part1by2(uint32_t x) {  // x < 2^10
  x &= 0x3ffu;
  x = (x | (x << 16)) & 0x030000ffu;
  x = (x | (x << 8)) & 0x0300f00fu;
  x = (x | (x << 4)) & 0x030c30c3u;
  x = (x | (x << 2)) & 0x09249249u;
  return x;
}
__device__ __forceinline__ uint32_t compact1by2(uint32_t x) {
  x &= 0x09249249u;
  x = (x | (x >> 2)) & 0x030c30c3u;
  x = (x | (x >> 4)) & 0x0300f00fu;
  x = (x | (x >> 8)) & 0x030000ffu;
  x = (x | (x >> 16)) & 0x000003ffu;
  return x;
}

template <int D>
__device__ __forceinline__ uint64_t menc(const int* x) {
  if (D == 1) return (uint64_t)x[0];
  if (D == 2) return (uint64_t)(part1by1((uint32_t)x[0]) | (part1by1((uint32_t)x[1]) << 1));
  return (uint64_t)(part1by2((uint32_t)x[0]) | (part1by2((uint32_t)x[1]) << 1) | (part1by2((uint32_t)x[2]) << 2));
}

template <int D>
__device__ __forceinline__ void mdec(uint64_t k, int* x) {
  x[1] = x[2] = 0;
  if (D == 1) {
    x[0] = (int)k;
  } else if (D == 2) {
    const uint32_t k32 = (uint32_t)k;
    x[0] = (int)compact1by1(k32);
    x[1] = (int)compact1by1(k32 >> 1);
  } else {
    const uint32_t k32 = (uint32_t)k;
    x[0] = (int)compact1by2(k32);
    x[1] = (int)compact1by2(k32 >> 1);
    x[2] = (int)compact1by2(k32 >> 2);
  }
}

// Morton bits of axis a (a, a + D, a + 2D, ...) of a 32-bit key
template <int D>
__device__ __forceinline__ constexpr uint32_t axis_mask(int a) {
  return D == 1 ? ~0u
         : D == 2 ? (a == 0 ? 0x55555555u : 0xaaaaaaaau)
                  : (a == 0 ? 0x49249249u : (a == 1 ? 0x92492492u : 0x24924924u));
}
// key of the cell o cells (|o| <= 2) along axis a from key k, the coordinate
// staying on the level: an add on the dilated coordinate (the other axes'
// bits are set to 1 so that carries pass them, or cleared so that borrows
// do), a few operations instead of a decode and an encode
template <int D>
__device__ __forceinline__ uint64_t morton_step(uint64_t k, int a, int o) {
  if (D == 1) return o > 0 ? k + (uint64_t)o : k - (uint64_t)(-o);
  const uint32_t k32 = (uint32_t)k;
  const uint32_t m = axis_mask<D>(a);
  const uint32_t d = (o == 1 || o == -1) ? (1u << a) : (1u << (D + a));
  if (o > 0) return (uint64_t)((((k32 | ~m) + d) & m) | (k32 & ~m));
  return (uint64_t)((((k32 & m) - d) & m) | (k32 & ~m));
}

// stencil coordinate: periodic wraps, homogeneous Neumann reflects evenly
__device__ __forceinline__ int map_st(int i, int n, int per) {
  if (i < 0) return per ? i + n : -1 - i;
  if (i >= n) return per ? i - n : 2 * n - 1 - i;
  return i;
}
// 1 when stencil coordinate i lies outside on a side with homogeneous
// Dirichlet conditions (mask bit 0: low side, bit 1: high side): the mirror
// cell of map_st enters with its sign flipped (q_{-1} = -q_0, q_{-2} = -q_1)
__device__ __forceinline__ bool st_flip(int i, int n, int dirichlet) {
  return (i < 0 && (dirichlet & 1)) || (i >= n && (dirichlet & 2));
}
// neighbourhood coordinate: wraps when periodic, -1 outside otherwise
__device__ __forceinline__ int map_nb(int i, int n, int per) {
  if (i < 0) return per ? i + n : -1;
  if (i >= n) return per ? i - n : -1;
  return i;
}

// within-instance key of the stencil cell at offset o along axis a of the
// cell (coordinates x, key k) on a level of n cells per axis; *fl: the
// Dirichlet sign flip of a mirrored cell
template <int D>
__device__ __forceinline__ uint64_t stencil_key(const Geo& g, const int* x, uint64_t k, int n, int a, int o,
                                                bool* fl) {
  const int c = x[a] + o;
  if (c >= 0 && c < n) {
    *fl = false;
    return morton_step<D>(k, a, o);
  }
  int y[3] = {x[0], x[1], x[2]};
  y[a] = map_st(c, n, g.periodic[a]);
  *fl = st_flip(c, n, g.dirichlet[a]);
  return menc<D>(y);
}
// the same with the neighbourhood mapping: false when outside the domain
template <int D>
__device__ __forceinline__ bool nbhd_key(const Geo& g, const int* x, uint64_t k, int n, int a, int o,
                                         uint64_t* out) {
  const int c = x[a] + o;
  if (c >= 0 && c < n) {
    *out = morton_step<D>(k, a, o);
    return true;
  }
  const int u = map_nb(c, n, g.periodic[a]);
  if (u < 0) return false;
  int y[3] = {x[0], x[1], x[2]};
  y[a] = u;
  *out = menc<D>(y);
  return true;
}

__device__ __forceinline__ void flag_bad(const Dev& p, int64_t inst, unsigned long long code) {
  atomicOr(&p.cnt[inst * CNT_PER_INST + CNT_BAD], code);
}

// ---------------------------------------------------------------------------
// prediction (Sec. 2): 1D q -/+ (q_{i+1}-q_{i-1})/8, tensor product in
// multi-D.  Terms T: q, qx, qy, qz, qxy, qxz, qyz, qxyz; child c = a|b<<1|e<<2.

template <int D>
__device__ __forceinline__ void pred_terms(const double* S, double* T) {
#define P(ox, oy, oz) S[((ox) + 1) + 3 * ((oy) + 1) + 9 * ((oz) + 1)]
  T[0] = P(0, 0, 0);
  T[1] = (P(1, 0, 0) - P(-1, 0, 0)) * 0.125;
  if (D >= 2) {
    T[2] = (P(0, 1, 0) - P(0, -1, 0)) * 0.125;
    T[4] = ((P(1, 1, 0) - P(1, -1, 0)) - (P(-1, 1, 0) - P(-1, -1, 0))) * 0.015625;
  }
  if (D == 3) {
    T[3] = (P(0, 0, 1) - P(0, 0, -1)) * 0.125;
    T[5] = ((P(1, 0, 1) - P(1, 0, -1)) - (P(-1, 0, 1) - P(-1, 0, -1))) * 0.015625;
    T[6] = ((P(0, 1, 1) - P(0, 1, -1)) - (P(0, -1, 1) - P(0, -1, -1))) * 0.015625;
    T[7] = (((P(1, 1, 1) - P(1, 1, -1)) - (P(1, -1, 1) - P(1, -1, -1))) -
            ((P(-1, 1, 1) - P(-1, 1, -1)) - (P(-1, -1, 1) - P(-1, -1, -1)))) *
           0.001953125;
  }
#undef P
}

template <int D>
__device__ __forceinline__ double pred_child(const double* T, int cb) {
  const int a = cb & 1, b = (cb >> 1) & 1, e = (cb >> 2) & 1;
  double v = T[0];
  v = a ? v + T[1] : v - T[1];
  if (D == 1) return v;
  v = b ? v + T[2] : v - T[2];
  if (D == 2) return (a == b) ? v + T[4] : v - T[4];
  v = e ? v + T[3] : v - T[3];
  v = (a == b) ? v + T[4] : v - T[4];
  v = (a == e) ? v + T[5] : v - T[5];
  v = (b == e) ? v + T[6] : v - T[6];
  v = ((a ^ b ^ e) == 1) ? v + T[7] : v - T[7];
  return v;
}

// 3^D stencil of component k of `src` around x at level lev (mapped by the
// boundary conditions); returns false when a stencil cell does not exist.
template <int D>
__device__ __forceinline__ bool gather27(const Geo& g, const Dev& p, const double* src, int lev,
                                         int64_t ibase, const int* x, int k, double* S) {
  const int n = 1 << lev;
  bool ok = true;
#pragma unroll
  for (int oz = (D > 2 ? -1 : 0); oz <= (D > 2 ? 1 : 0); oz++)
#pragma unroll
    for (int oy = (D > 1 ? -1 : 0); oy <= (D > 1 ? 1 : 0); oy++)
#pragma unroll
      for (int ox = -1; ox <= 1; ox++) {
        int y[3] = {map_st(x[0] + ox, n, g.periodic[0]), 0, 0};
        if (D > 1) y[1] = map_st(x[1] + oy, n, g.periodic[1]);
        if (D > 2) y[2] = map_st(x[2] + oz, n, g.periodic[2]);
        bool fl = st_flip(x[0] + ox, n, g.dirichlet[0]);
        if (D > 1) fl = fl != st_flip(x[1] + oy, n, g.dirichlet[1]);
        if (D > 2) fl = fl != st_flip(x[2] + oz, n, g.dirichlet[2]);
        const int64_t G = ibase + (int64_t)menc<D>(y);
        if (g.check) ok = ok && (p.st[G] != ST_ABSENT);  // grading: the stencil exists
        const double v = src[(int64_t)k * g.Ntot + G];
        S[(ox + 1) + 3 * (oy + 1) + 9 * (oz + 1)] = fl ? -v : v;
      }
  return ok;
}

// ---------------------------------------------------------------------------
// numerical fluxes (Sec. 5 of the paper names AUSM+; readings: MUSCL-minmod
// reconstruction, exact Godunov flux for the scalar Burgers law, centred
// two-point diffusion, interface sound speed = mean of the two sides)

__device__ __forceinline__ double minmod(double a, double b) {
  if (a > 0.0 && b > 0.0) return a < b ? a : b;
  if (a < 0.0 && b < 0.0) return a > b ? a : b;
  return 0.0;
}

__device__ __forceinline__ void recon4(int mode, double c0, double c1, double c2, double c3,
                                       double& qL, double& qR) {
  if (mode == 1) {
    const double sl = minmod(c1 - c0, c2 - c1);
    const double sr = minmod(c2 - c1, c3 - c2);
    qL = c1 + 0.5 * sl;
    qR = c2 - 0.5 * sr;
  } else {
    qL = c1;
    qR = c2;
  }
}

__device__ __forceinline__ double mach_plus(double M) {
  if (fabs(M) < 1.0) {
    const double t = M + 1.0, q = (M * M) - 1.0;
    return (0.25 * (t * t)) + (0.125 * (q * q));
  }
  return 0.5 * (M + fabs(M));
}
__device__ __forceinline__ double mach_minus(double M) {
  if (fabs(M) < 1.0) {
    const double t = M - 1.0, q = (M * M) - 1.0;
    return (-(0.25 * (t * t))) - (0.125 * (q * q));
  }
  return 0.5 * (M - fabs(M));
}
__device__ __forceinline__ double pres_plus(double M) {
  if (fabs(M) < 1.0) {
    const double t = M + 1.0, q = (M * M) - 1.0;
    return ((0.25 * (t * t)) * (2.0 - M)) + ((0.1875 * M) * (q * q));
  }
  return M > 0.0 ? 1.0 : 0.0;
}
__device__ __forceinline__ double pres_minus(double M) {
  if (fabs(M) < 1.0) {
    const double t = M - 1.0, q = (M * M) - 1.0;
    return ((0.25 * (t * t)) * (2.0 + M)) - ((0.1875 * M) * (q * q));
  }
  return M < 0.0 ? 1.0 : 0.0;
}

template <int D>
__device__ __forceinline__ void euler_prim(double gm1, const double* q, double* w) {
  const double rho = q[0];
  double kin = 0.0;
  w[0] = rho;
#pragma unroll
  for (int i = 0; i < D; i++) {
    const double u = q[1 + i] / rho;
    w[1 + i] = u;
    kin = (i == 0) ? (u * u) : (kin + (u * u));
  }
  w[D + 1] = gm1 * (q[D + 1] - ((0.5 * rho) * kin));
}

template <int D>
__device__ __forceinline__ void ausm_plus(int dir, double gamma, const double* wl, const double* wr,
                                          double* F) {
  const double gm1 = gamma - 1.0;
  const double rl = wl[0], pl = wl[D + 1], rr = wr[0], pr = wr[D + 1];
  const double al = sqrt((gamma * pl) / rl), ar = sqrt((gamma * pr) / rr);
  const double ah = 0.5 * (al + ar);
  const double ml = wl[1 + dir] / ah, mr = wr[1 + dir] / ah;
  const double mh = mach_plus(ml) + mach_minus(mr);
  const double ph = (pres_plus(ml) * pl) + (pres_minus(mr) * pr);
  const double mp = 0.5 * (mh + fabs(mh)), mm = 0.5 * (mh - fabs(mh));
  double kl = 0.0, kr = 0.0;
#pragma unroll
  for (int i = 0; i < D; i++) {
    kl = (i == 0) ? (wl[1] * wl[1]) : (kl + (wl[1 + i] * wl[1 + i]));
    kr = (i == 0) ? (wr[1] * wr[1]) : (kr + (wr[1 + i] * wr[1 + i]));
  }
  const double hl = ((pl / gm1) + ((0.5 * rl) * kl)) + pl;
  const double hr = ((pr / gm1) + ((0.5 * rr) * kr)) + pr;
  F[0] = ah * ((mp * rl) + (mm * rr));
#pragma unroll
  for (int i = 0; i < D; i++) F[1 + i] = ah * ((mp * (rl * wl[1 + i])) + (mm * (rr * wr[1 + i])));
  F[1 + dir] = F[1 + dir] + ph;
  F[D + 1] = ah * ((mp * hl) + (mm * hr));
}

template <int D, int PDE>
struct NC {
  static constexpr int M = (PDE == PDE_EULER) ? D + 2 : (PDE == PDE_FLAMEBALL ? 2 : 1);
};

// how far along an axis a leaf's stencil reads: 2 with the MUSCL
// reconstruction, 1 for two-point diffusion (no advection), first order or
// centred fluxes
__host__ __device__ __forceinline__ int stencil_reach(const Geo& g) {
  return (g.two_point || g.recon != 1) ? 1 : 2;
}

template <int PDE>
__host__ __device__ __forceinline__ constexpr bool is_flame() {
  return PDE == PDE_FLAME || PDE == PDE_FLAMEBALL;
}

// fluxes that read only the two cells next to the face
template <int PDE>
__device__ __forceinline__ bool two_point(const Geo& g) {
  return PDE == PDE_NAGUMO || PDE == PDE_LINEAR || (is_flame<PDE>() && g.two_point);
}

// advection velocity along dir of instance inst: the flames' frame velocity
// (+-v_f along axis 0, set at the start of each macro step) or the fixed one
template <int PDE>
__device__ __forceinline__ double adv_velocity(const Geo& g, const Dev& p, int64_t inst, int dir) {
  if (is_flame<PDE>() && g.flame_speed) return dir == 0 ? p.vel[inst] : 0.0;
  return g.adv[dir];
}

// flux across the face between cells a and a+1 along dir; c holds a-1..a+2;
// vel is the advection velocity along dir (advection and flames); ix is the
// inverse cell width along dir
template <int D, int PDE>
__device__ __forceinline__ void face_flux_ix(const Geo& g, double ix, int dir, double vel,
                                             const double (*c)[NC<D, PDE>::M], double* F) {
  if (PDE == PDE_ADVECTION) {
    if (g.recon == 2) {
      F[0] = vel * (0.5 * (c[1][0] + c[2][0]));
    } else {
      double qL, qR;
      recon4(g.recon, c[0][0], c[1][0], c[2][0], c[3][0], qL, qR);
      F[0] = vel >= 0.0 ? vel * qL : vel * qR;
    }
  } else if (PDE == PDE_BURGERS) {
    double uL, uR;
    recon4(g.recon, c[0][0], c[1][0], c[2][0], c[3][0], uL, uR);
    const double a = uL > 0.0 ? uL : 0.0;
    const double b = uR < 0.0 ? uR : 0.0;
    const double fa = 0.5 * (a * a), fb = 0.5 * (b * b);
    const double fadv = fa > fb ? fa : fb;
    const double nudx = g.nu * ix;
    F[0] = fadv - (nudx * (c[2][0] - c[1][0]));
  } else if (PDE == PDE_NAGUMO || PDE == PDE_LINEAR) {
    const double nudx = g.nu * ix;
    F[0] = -(nudx * (c[2][0] - c[1][0]));
  } else if (is_flame<PDE>()) {
    // upwind value of the reconstructed face states, then the two-point
    // diffusive flux (coefficient 1 for T, 1/Le for Y)
    constexpr int M = NC<D, PDE>::M;
#pragma unroll
    for (int k = 0; k < M; k++) {
      double fadv;
      if (g.recon == 2) {
        fadv = vel * (0.5 * (c[1][k] + c[2][k]));
      } else {
        double qL, qR;
        recon4(g.recon, c[0][k], c[1][k], c[2][k], c[3][k], qL, qR);
        fadv = vel >= 0.0 ? vel * qL : vel * qR;
      }
      const double dif = k == 0 ? 1.0 : 1.0 / g.lewis;
      F[k] = fadv - ((dif * ix) * (c[2][k] - c[1][k]));
    }
  } else {
    constexpr int M = D + 2;
    const double gm1 = g.gamma - 1.0;
    double w[4][M], wl[M], wr[M];
#pragma unroll
    for (int j = 0; j < 4; j++) euler_prim<D>(gm1, c[j], w[j]);
#pragma unroll
    for (int k = 0; k < M; k++) recon4(g.recon, w[0][k], w[1][k], w[2][k], w[3][k], wl[k], wr[k]);
    ausm_plus<D>(dir, g.gamma, wl, wr, F);
  }
}
template <int D, int PDE>
__device__ __forceinline__ void face_flux(const Geo& g, int lev, int dir, double vel,
                                          const double (*c)[NC<D, PDE>::M], double* F) {
  face_flux_ix<D, PDE>(g, g.invdx[lev][dir], dir, vel, c, F);
}

template <int PDE>
__host__ __device__ __forceinline__ constexpr bool has_source() {
  return PDE == PDE_NAGUMO || PDE == PDE_LINEAR || is_flame<PDE>();
}

// reaction rate of the flames (Sec. 5): the 1D flame's form in u = 1 - T
// (Y = 1 - T, unit Lewis number); the flame ball's in (T, Y)
__device__ __forceinline__ double omega_front(const Geo& g, double T) {
  const double u = 1.0 - T;
  return ((0.5 * (g.ze * g.ze)) * u) * exp((g.ze * u) / ((g.tau * u) - 1.0));
}
__device__ __forceinline__ double omega_ball(const Geo& g, double T, double Y) {
  const double tm1 = T - 1.0;
  return (((g.ze * g.ze) / (2.0 * g.lewis)) * Y) * exp((g.ze * tm1) / (1.0 + (g.tau * tm1)));
}
// radiative loss kappa ((T + 1/tau - 1)^4 - (1/tau - 1)^4)
__device__ __forceinline__ double radiation(const Geo& g, double T) {
  const double a = (T + (1.0 / g.tau)) - 1.0, b = (1.0 / g.tau) - 1.0;
  return g.kappa * (((a * a) * (a * a)) - ((b * b) * (b * b)));
}
template <int PDE>
__device__ __forceinline__ double reaction_rate(const Geo& g, const double* q) {
  if (PDE == PDE_FLAME) return omega_front(g, q[0]);
  return omega_ball(g, q[0], q[1]);
}

// pointwise source at the cell average, added to R
template <int PDE>
__device__ __forceinline__ void add_source(const Geo& g, const double* q, double* R) {
  if (PDE == PDE_NAGUMO) {
    R[0] = R[0] + (((g.k_react * q[0]) * (1.0 - q[0])) * (q[0] - g.a_react));
  } else if (PDE == PDE_LINEAR) {
    R[0] = R[0] + (g.k_react * q[0]);
  } else if (PDE == PDE_FLAME) {
    R[0] = R[0] + omega_front(g, q[0]);
  } else if (PDE == PDE_FLAMEBALL) {
    const double w = omega_ball(g, q[0], q[1]);
    R[0] = R[0] + (w - radiation(g, q[0]));
    R[1] = R[1] - w;
  }
}

// ---------------------------------------------------------------------------
// status fill, initial load, dense reconstruction

__global__ void k_fill_status(uint8_t* st, int64_t base, int64_t n, uint8_t v) {
  GSL(t, n) st[base + t] = v;
}

void launch_fill_status(const Geo& g, const Dev& p, int lev, uint8_t v, hipStream_t s) {
  const int64_t n = g.B * g.n[lev];
  k_fill_status<<<blocks_for(n), TPB, 0, s>>>(p.st, g.off[lev], n, v);
}

// finest-level averages into level L (the instance's own finest level when
// one instance is loaded)
template <int D>
__global__ void k_load_finest(Geo g, Dev p, const double* src, int only, int L) {
  const int64_t nl = g.n[L], N = (only >= 0 ? 1 : g.B) * nl;
  const int n = 1 << L;
  GSL(u, N) {
    const int64_t t = only >= 0 ? (int64_t)only * nl + u : u;
    const int64_t inst = t >> (D * L);
    const int64_t isrc = only >= 0 ? 0 : inst;
    int x[3];
    mdec<D>((uint64_t)(t & (nl - 1)), x);
    const int64_t r = x[0] + (int64_t)n * (x[1] + (int64_t)n * x[2]);
    const int64_t G = g.off[L] + t;
    for (int k = 0; k < g.m; k++) p.q[SL_Q0][(int64_t)k * g.Ntot + G] = src[(isrc * g.m + k) * nl + r];
    p.st[G] = ST_LEAF;
  }
}

// statuses of one instance: levels below its finest level Li internal, the
// others absent (level Li is then written by k_load_finest); or all absent
// (free slot)
__global__ void k_fill_instance(Geo g, Dev p, int inst, int free_slot, int Li) {
  for (int lev = g.l0; lev <= g.L; lev++) {
    const int64_t nl = g.n[lev];
    const uint8_t v = free_slot ? ST_ABSENT : (lev < Li ? ST_INTERNAL : ST_ABSENT);
    GSL(u, nl) p.st[g.off[lev] + (int64_t)inst * nl + u] = v;
  }
}

void launch_fill_instance(const Geo& g, const Dev& p, int inst, int Li, hipStream_t s) {
  k_fill_instance<<<blocks_for(g.n[g.L]), TPB, 0, s>>>(g, p, inst >= 0 ? inst : -1 - inst, inst < 0, Li);
}

template <int D>
__global__ void k_recon_level(Geo g, Dev p, int lev, double* dense) {
  const int64_t nl = g.n[lev], N = g.B * nl;
  GSL(t, N) {
    const int64_t G = g.off[lev] + t;
    if (lev == g.l0 || p.st[G] != ST_ABSENT) {
      for (int k = 0; k < g.m; k++) dense[(int64_t)k * g.Ntot + G] = p.q[SL_Q0][(int64_t)k * g.Ntot + G];
      continue;
    }
    const int64_t inst = t >> (D * lev);
    int x[3];
    mdec<D>((uint64_t)(t & (nl - 1)), x);
    const int px[3] = {x[0] >> 1, x[1] >> 1, x[2] >> 1};
    const int n = 1 << (lev - 1);
    const int64_t ibp = g.off[lev - 1] + inst * g.n[lev - 1];
    const int cb = (x[0] & 1) | ((x[1] & 1) << 1) | ((x[2] & 1) << 2);
    for (int k = 0; k < g.m; k++) {
      double S[27], T[8];
#pragma unroll
      for (int oz = (D > 2 ? -1 : 0); oz <= (D > 2 ? 1 : 0); oz++)
#pragma unroll
        for (int oy = (D > 1 ? -1 : 0); oy <= (D > 1 ? 1 : 0); oy++)
#pragma unroll
          for (int ox = -1; ox <= 1; ox++) {
            int y[3] = {map_st(px[0] + ox, n, g.periodic[0]), 0, 0};
            if (D > 1) y[1] = map_st(px[1] + oy, n, g.periodic[1]);
            if (D > 2) y[2] = map_st(px[2] + oz, n, g.periodic[2]);
            bool fl = st_flip(px[0] + ox, n, g.dirichlet[0]);
            if (D > 1) fl = fl != st_flip(px[1] + oy, n, g.dirichlet[1]);
            if (D > 2) fl = fl != st_flip(px[2] + oz, n, g.dirichlet[2]);
            const double v = dense[(int64_t)k * g.Ntot + ibp + (int64_t)menc<D>(y)];
            S[(ox + 1) + 3 * (oy + 1) + 9 * (oz + 1)] = fl ? -v : v;
          }
      pred_terms<D>(S, T);
      dense[(int64_t)k * g.Ntot + G] = pred_child<D>(T, cb);
    }
  }
}

template <int D>
__global__ void k_to_rowmajor(Geo g, const double* dense, double* out) {
  const int L = g.L;
  const int64_t nl = g.n[L], N = g.B * nl;
  const int n = 1 << L;
  GSL(t, N) {
    const int64_t inst = t >> (D * L);
    int x[3];
    mdec<D>((uint64_t)(t & (nl - 1)), x);
    const int64_t r = x[0] + (int64_t)n * (x[1] + (int64_t)n * x[2]);
    for (int k = 0; k < g.m; k++) out[(inst * g.m + k) * nl + r] = dense[(int64_t)k * g.Ntot + g.off[L] + t];
  }
}

// ---------------------------------------------------------------------------
// projections: the parent value is the mean of its 2^d children, summed in
// child order and scaled by 2^{-d} (Sec. 2).  The modes are the internal-
// node synchronisation values of Sec. 4:
//   PJ_Q0    Alg. alg-LTS: q^n of internal nodes
//   PJ_CASEB Alg. alg-LTS / Sec. 4.3, level l_min - 1 at mid-step: the
//            theta=1/2 value (into QH) and -2 q^n - q* + 4 q_{1/2} (into QE)
//   PJ_REF2  Alg. refRK2: q(t + dt/2) from the children's q* (eq.
//            refreshRk2 for internal children), then q* = 2 q(t+dt/2) - q^n
//   PJ_RK2   Alg. projRK2: mean of the children's extrapolations to
//            t + 2 dt_{l+1} (eqs. projleaf and projnode)
//   PJ_REF3  Alg. refRK22: q_{1/4} from the children's q**, then
//            eqs. ProjRK3equations1 / ProjRK3equations2
//   PJ_RK3   Alg. projRK3: q** from the children's stage-3 values, then
//            eq. rk3proj

// Levels with >= 4096 cells per instance and >= 2^20 cells in all are
// "wide": their dense passes take 16 cells per lane, their 4096-cell blocks
// are the compaction blocks, and they keep block summaries.
__host__ __device__ __forceinline__ bool wide_level(const Geo& g, int lev) {
  return g.comp_chunk[lev] == (1 << BS_SHIFT) && g.B * g.n[lev] >= ((int64_t)1 << 20);
}

// Wave-uniform values: the first active lane's value, and loads through the
// scalar data cache of memory that no kernel writes while it runs (the
// address must be wave-uniform).  The load waits for its reply in the same
// asm block; being opaque, it also keeps the compiler from turning it back
// into a per-lane load where it can prove the lane's own index equal.  A
// byte is read as the aligned 32-bit word that holds it (same page).
__device__ __forceinline__ int64_t rfl64(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
// Workgroups are placed on the eight XCDs in turn.  For a grid of a
// multiple of 128 workgroups this numbering gives the workgroups of one XCD
// runs of 16 consecutive chunks of a pass, the runs handed to the XCDs in
// turn: list entries that share cache lines (neighbouring chunks of a
// Morton-ordered list) then meet in one L2, and a short list still spreads
// over all XCDs.  Other grids keep the hardware's order.
__device__ __forceinline__ int xcd_run_block() {
  int bx = (int)blockIdx.x;
  if (gridDim.x % 128u == 0u) {
    const int x = bx & 7, j = bx >> 3;
    bx = (((j >> 4) << 3) + x) * 16 + (j & 15);
  }
  return bx;
}

// b[j] and d[k] in one round trip
__device__ __forceinline__ void uload_u8_f64(const uint8_t* b, int64_t j, const double* d, int64_t k, uint8_t* bv,
                                             double* dv) {
  const uintptr_t ab = (uintptr_t)(b + j);
  const uint32_t* w = (const uint32_t*)(ab & ~(uintptr_t)3);
  const double* ad = d + k;
  uint32_t wv;
  double v;
  asm volatile("s_load_dword %0, %2, 0x0\n\ts_load_dwordx2 %1, %3, 0x0\n\ts_waitcnt lgkmcnt(0)"
               : "=&s"(wv), "=&s"(v)
               : "s"(w), "s"(ad)
               : "memory");
  *bv = (uint8_t)(wv >> (8 * (int)(ab & 3)));
  *dv = v;
}

// list codes per cell (group_codes.h), written by the compaction's count
// pass; in 1D and 2D, bit CODE_FACE0 << (2 a + s): the face neighbour of a
// leaf along axis a (side s) is absent and inside the domain
static constexpr uint32_t CODE_LEAF = 1u, CODE_INT = 2u, CODE_IFACE = 4u, CODE_GHOST = 8u, CODE_FACE0 = 16u;

// Per-level constants of a launch, staged in LDS: kernels whose lanes work on
// different levels would otherwise index the kernel arguments by a per-lane
// level, a vector load of its own in front of every cell's loads.
struct LevTab {
  int64_t off[MRD_MAXLEV + 1];    // first cell of the level table
  int64_t bsoff[MRD_MAXLEV + 1];  // first 4096-cell block summary
  int64_t rc[MRD_MAXLEV + 1];     // coarse-side register block
  int64_t rf[MRD_MAXLEV + 1];     // fine-side register block
  double ix[MRD_MAXLEV + 1][3];   // inverse cell widths
  int wide[MRD_MAXLEV + 1];       // wide_level
};
// filled by the first MRD_MAXLEV + 1 threads; the caller synchronises
__device__ __forceinline__ void levtab_fill(const Geo& g, LevTab& lt) {
  const int l = (int)threadIdx.x;
  if (l > MRD_MAXLEV) return;
  lt.off[l] = g.off[l];
  lt.bsoff[l] = g.bs_off[l];
  lt.rc[l] = g.rc_off[l];
  lt.rf[l] = g.rf_off[l];
  for (int a = 0; a < 3; a++) lt.ix[l][a] = g.invdx[l][a];
  lt.wide[l] = (l >= g.l0 && l <= g.L) ? (wide_level(g, l) ? 1 : 0) : 0;
}

__device__ __forceinline__ int list_len(const Dev& p, int type, int lev) {
  return p.lcnt[type * (MRD_MAXLEV + 1) + lev];
}

// The lists of levels lo..hi as one index space, so that a lane takes one
// item whatever its level (no per-lane walk over the levels): the lengths
// go to shared memory, a lane finds its level by a scan of them.
__device__ __forceinline__ int64_t flat_setup(const Dev& p, int type, int lo, int hi, int* s_cnt) {
  const int nlv = hi - lo + 1;
  if ((int)threadIdx.x < nlv) s_cnt[threadIdx.x] = list_len(p, type, lo + (int)threadIdx.x);
  __syncthreads();
  int64_t tot = 0;
  for (int j = 0; j < nlv; j++) tot += s_cnt[j];
  return tot;
}
__device__ __forceinline__ int flat_level(const int* s_cnt, int lo, int64_t& k) {
  int j = 0;
  while (k >= s_cnt[j]) {
    k -= s_cnt[j];
    j++;
  }
  return lo + j;
}

// the mode is a template argument, so each mode loads only what it uses;
// the next list entry is fetched while a node is processed, and a node's
// loads (children of every field, its own values the mode combines) are all
// issued before the first is used: one memory round trip per node, two where
// the mode selects a child's slot by the child's status
template <int D, int mode>
__global__ __launch_bounds__(TPB) void k_project(Geo g, Dev p, int lev) {
  constexpr int NCH = 1 << D;
  constexpr int MF = D + 2;  // most fields of any PDE in D dimensions
  constexpr double sc = D == 1 ? 0.5 : (D == 2 ? 0.25 : 0.125);
  constexpr bool NEED_ST = mode == PJ_REF2;
  const int64_t NT = g.Ntot;
  const int m = g.m;
  const int n = list_len(p, LS_INTERNAL, lev);
  const int* lst = p.lst[LS_INTERNAL] + g.off[lev];
  const int step = (int)(gridDim.x * blockDim.x);
  int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  int t_next = i < n ? lst[i] : 0;
  // wait for the first entry here: the loop then needs no wait at its top,
  // where one would also cover the previous pass's stores (the vector memory
  // counter counts loads and stores in issue order) and put a store round
  // trip before every pass's loads
  vm_wait_all();
  for (; i < n; i += step) {
    const int64_t t = t_next;
    if (i + step < n) t_next = lst[i + step];
    const int64_t G = g.off[lev] + t;
    const int64_t C0 = g.off[lev + 1] + (t << D);
    bool leaf[NCH];
#pragma unroll
    for (int cb = 0; cb < NCH; cb++) leaf[cb] = NEED_ST ? p.st[C0 + cb] == ST_LEAF : true;
    double v[MF][NCH], o0[MF], o1[MF], o2[MF];
#pragma unroll
    for (int k = 0; k < MF; k++) {
      if (k >= m) break;
      const int64_t kk = (int64_t)k * NT;
#pragma unroll
      for (int cb = 0; cb < NCH; cb++) {
        const int64_t C = kk + C0 + cb;
        double x;
        if (mode == PJ_Q0 || mode == PJ_CASEB) {
          x = p.q[SL_Q0][C];
        } else if (mode == PJ_REF2) {
          x = (leaf[cb] ? p.q[SL_Q1] : p.q[SL_Q1REF])[C];
        } else if (mode == PJ_RK2) {
          // a leaf child's X2 is its stage-2 Euler value; an internal
          // child's X2 was set to 2 Q1 - Q0 by its own level's pass
          x = p.q[SL_X2][C];
        } else if (mode == PJ_REF3 || mode == PJ_ST3) {
          x = p.q[SL_QH][C];
        } else if (mode == PJ_ST2) {
          x = p.q[SL_Q1][C];
        } else {
          x = p.q[SL_QE][C];
        }
        v[k][cb] = x;
      }
      const int64_t I = kk + G;
      o0[k] = o1[k] = o2[k] = 0.0;
      if (mode == PJ_CASEB || mode == PJ_REF3) {
        o0[k] = p.q[SL_Q0][I];
        o1[k] = p.q[SL_Q1REF][I];
      } else if (mode == PJ_REF2 || mode == PJ_RK2) {
        o0[k] = p.q[SL_Q0][I];
      } else if (mode == PJ_RK3) {
        o0[k] = p.q[SL_Q0][I];
        o1[k] = p.q[SL_N34][I];
        o2[k] = p.q[SL_N14][I];
      }
    }
#pragma unroll
    for (int k = 0; k < MF; k++) {
      if (k >= m) break;
      double s = v[k][0];
#pragma unroll
      for (int cb = 1; cb < NCH; cb++) s = s + v[k][cb];
      s = s * sc;
      const int64_t I = (int64_t)k * NT + G;
      if (mode == PJ_ST2) {
        p.q[SL_Q1][I] = s;          // global step: stage-2 state of the node
      } else if (mode == PJ_ST3) {
        p.q[SL_QH][I] = s;          // global step: stage-3 state of the node
      } else if (mode == PJ_Q0) {
        p.q[SL_Q0][I] = s;
      } else if (mode == PJ_CASEB) {
        p.q[SL_QH][I] = s;
        p.q[SL_QE][I] = ((-2.0 * o0[k]) - o1[k]) + (4.0 * s);
      } else if (mode == PJ_REF2) {
        p.q[SL_H1][I] = s;
        p.q[SL_Q1REF][I] = (2.0 * s) - o0[k];
      } else if (mode == PJ_RK2) {
        // the node's stage-2 value: its Q1, and 2 Q1 - Q0 in its X2 for the
        // coarser level's pass and the refined faces of coarser leaves
        p.q[SL_Q1][I] = s;
        p.q[SL_X2][I] = (2.0 * s) - o0[k];
      } else if (mode == PJ_REF3) {
        const double q0 = o0[k], qs = o1[k];
        p.q[SL_N14][I] = s;
        p.q[SL_N34][I] = ((-6.5 * q0) - (1.5 * qs)) + (9.0 * s);
        p.q[SL_QH][I] = ((-5.5 * q0) - (1.5 * qs)) + (8.0 * s);
      } else {
        p.q[SL_QH][I] = s;
        p.q[SL_QE][I] = o0[k] + (2.0 * (o1[k] - o2[k]));
      }
    }
  }
}

template <int D>
static void project_d(const Geo& g, const Dev& p, int lev, int mode, int nb, hipStream_t s) {
  switch (mode) {
    case PJ_Q0: k_project<D, PJ_Q0><<<nb, TPB, 0, s>>>(g, p, lev); break;
    case PJ_CASEB: k_project<D, PJ_CASEB><<<nb, TPB, 0, s>>>(g, p, lev); break;
    case PJ_REF2: k_project<D, PJ_REF2><<<nb, TPB, 0, s>>>(g, p, lev); break;
    case PJ_RK2: k_project<D, PJ_RK2><<<nb, TPB, 0, s>>>(g, p, lev); break;
    case PJ_REF3: k_project<D, PJ_REF3><<<nb, TPB, 0, s>>>(g, p, lev); break;
    case PJ_RK3: k_project<D, PJ_RK3><<<nb, TPB, 0, s>>>(g, p, lev); break;
    case PJ_ST2: k_project<D, PJ_ST2><<<nb, TPB, 0, s>>>(g, p, lev); break;
    default: k_project<D, PJ_ST3><<<nb, TPB, 0, s>>>(g, p, lev); break;
  }
}

void launch_project(const Geo& g, const Dev& p, int lev, int mode, hipStream_t s) {
  const int64_t n = g.B * g.n[lev];
  const int nb = list_blocks(g, n);
  if (g.d == 1) project_d<1>(g, p, lev, mode, nb, s);
  else if (g.d == 2) project_d<2>(g, p, lev, mode, nb, s);
  else project_d<3>(g, p, lev, mode, nb, s);
}

// ---------------------------------------------------------------------------
// virtual cells: absent cells read by a leaf stencil get the value predicted
// from the parent level at the time the stage needs (Sec. 4):
//   case A (parent level also starts at t^n): S1 q^n, S2 first-order
//     theta=1/2 value, S3 theta=1/4 value (Alg. refRK22)
//   case B (parent level l_min - 1 at mid-step): S1 q** / theta=1/2
//     projection, S2 end value, S3 theta=3/4 value (Alg. refRK22, Sec. 4.3)

template <class T>
__device__ __forceinline__ T block_exscan(T v, T* sh, T* tot);  // block-wide exclusive scan (below)

template <int D>
__global__ __launch_bounds__(TPB) void k_ghost(Geo g, Dev p, int lo, int hi, int cb_lev, int srcA, int srcB,
                                              int dst) {
  // siblings are adjacent in a level's list (Morton order), and all of them
  // are predicted from the same parent stencil: a block takes 1024 list
  // entries (four per lane), gathers the first listed sibling of each
  // parent into shared memory, and each lane then predicts one parent's
  // listed children from one gather of its stencil
  constexpr int PER = 4, CH = TPB * PER, NS = 1 << D;
  __shared__ int s_cnt[MRD_MAXLEV + 1];
  __shared__ int s_lead[CH];
  __shared__ int s_t[CH + NS - 1];  // the block's list entries and the next NS - 1, read again by the leaders
  __shared__ int sh[TPB / 64];
  __shared__ LevTab lt;
  levtab_fill(g, lt);  // flat_setup synchronises
  const int64_t ntot = flat_setup(p, LS_GHOST, lo, hi, s_cnt);
  // the two source slots, selected per lane by level below (the slot array
  // indexed by a per-lane value would be a vector load of its own)
  const double* qA = p.q[srcA];
  const double* qB = p.q[srcB];
  // runs of chunks per XCD: neighbouring virtual cells share parent stencils
  for (int64_t base = (int64_t)xcd_run_block() * CH; base < ntot; base += (int64_t)gridDim.x * CH) {
    // the lane's entries (and, for the block's first, the entry before it)
    int tv[PER], kv[PER], prev0 = 0;
#pragma unroll
    for (int e = 0; e < PER; e++) {
      tv[e] = 0;
      kv[e] = -1;
    }
#pragma unroll
    for (int e = 0; e < PER; e++) {
      const int64_t i = base + PER * (int64_t)threadIdx.x + e;
      if (i >= ntot) break;
      int64_t kk = i;
      const int lev = flat_level(s_cnt, lo, kk);
      const int* lst = p.lst[LS_GHOST] + lt.off[lev];
      tv[e] = lst[kk];
      kv[e] = (int)kk;
      if (e == 0 && threadIdx.x == 0 && kk > 0) prev0 = lst[kk - 1];
    }
#pragma unroll
    for (int e = 0; e < PER; e++) s_t[PER * threadIdx.x + e] = tv[e];
    // the entries just past the block, for the groups that straddle its end
    if (threadIdx.x < NS - 1) {
      int64_t kk = base + CH + threadIdx.x;
      int u = 0;
      if (kk < ntot) {
        const int lev = flat_level(s_cnt, lo, kk);
        u = p.lst[LS_GHOST][lt.off[lev] + kk];
      }
      s_t[CH + threadIdx.x] = u;
    }
    __syncthreads();
    uint32_t lead = 0u;  // bit e: entry base + PER * threadIdx.x + e leads its sibling group
#pragma unroll
    for (int e = 0; e < PER; e++) {
      if (kv[e] < 0) break;
      const int q = PER * (int)threadIdx.x + e;
      const int pt = q > 0 ? s_t[q - 1] : prev0;
      if (kv[e] == 0 || (pt >> D) != (tv[e] >> D)) lead |= 1u << e;
    }
    int tot;
    int pos = block_exscan<int>(__popc(lead), sh, &tot);
    while (lead) {
      const int e = __builtin_ctz(lead);
      lead &= lead - 1u;
      s_lead[pos++] = PER * (int)threadIdx.x + e;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < tot; q += TPB) {
      const int ql = s_lead[q];
      int64_t kk = base + ql;
      const int lev = flat_level(s_cnt, lo, kk);
      const int64_t nl = (int64_t)1 << (D * lev);
      const double* src = lev == cb_lev ? qB : qA;
      const int len = s_cnt[lev - lo];
      const int t = s_t[ql];
      // the group's listed siblings follow it in the list (the block's
      // entries and the NS - 1 after them, all in LDS)
      uint32_t cbits = 1u << (t & (NS - 1));
      for (int e = 1; e < NS && kk + e < len; e++) {
        const int u = s_t[ql + e];
        if ((u >> D) != (t >> D)) break;
        cbits |= 1u << (u & (NS - 1));
      }
      const int64_t G0 = lt.off[lev] + (int64_t)(t & ~(NS - 1));  // child 0 of the parent
      const int64_t inst = (int64_t)t >> (D * lev);
      int x[3];
      mdec<D>((uint64_t)((int64_t)t & (nl - 1)), x);
      const int px[3] = {x[0] >> 1, x[1] >> 1, x[2] >> 1};
      const int64_t ibp = lt.off[lev - 1] + inst * (nl >> D);
      for (int k = 0; k < g.m; k++) {
        double S[27], T[8];
        if (!gather27<D>(g, p, src, lev - 1, ibp, px, k, S)) flag_bad(p, inst, 1);
        pred_terms<D>(S, T);
#pragma unroll
        for (int cb = 0; cb < NS; cb++)
          if ((cbits >> cb) & 1u) p.q[dst][(int64_t)k * g.Ntot + G0 + cb] = pred_child<D>(T, cb);
      }
    }
    __syncthreads();  // s_lead is reused
  }
}

void launch_ghost(const Geo& g, const Dev& p, int lo, int hi, int cb_lev, int stage, hipStream_t s) {
  if (lo > hi) return;
  const int dst = stage == 1 ? SL_Q0 : (stage == 2 ? SL_Q1 : SL_QH);
  const int srcB = stage == 1 ? SL_QH : (stage == 2 ? SL_QE : SL_N34);
  // global step: the parent level's own stage state; LT case A: q^n,
  // first-order theta=1/2, theta=1/4
  const int srcA = !g.lt ? dst : (stage == 1 ? SL_Q0 : (stage == 2 ? SL_H1 : SL_N14));
  const int64_t n = g.B * g.n[hi];
  const int nb = list_blocks(g, n);
  if (g.d == 1) k_ghost<1><<<nb, TPB, 0, s>>>(g, p, lo, hi, cb_lev, srcA, srcB, dst);
  else if (g.d == 2) k_ghost<2><<<nb, TPB, 0, s>>>(g, p, lo, hi, cb_lev, srcA, srcB, dst);
  else k_ghost<3><<<nb, TPB, 0, s>>>(g, p, lo, hi, cb_lev, srcA, srcB, dst);
}

// ---------------------------------------------------------------------------
// one compact RK3 stage on the leaves of one level (Sec. 3, Algs. alg-LTS,
// Steprk2, Steprk3) with the NERK partials and the flux registers

__device__ __forceinline__ double* regc_at(const Geo& g, const Dev& p, int lev, int f, int k, int64_t t) {
  const int64_t Nl = g.B * g.n[lev];
  return p.regc + g.rc_off[lev] + (int64_t)(f * g.m + k) * Nl + t;
}
__device__ __forceinline__ double* regf_at(const Geo& g, const Dev& p, int lev, int f, int b, int k, int64_t t) {
  const int64_t Nl = g.B * g.n[lev];
  return p.regf + g.rf_off[lev] + (int64_t)((f * g.nsub + b) * g.m + k) * Nl + t;
}

template <int D>
__device__ __forceinline__ void transverse(int dir, int& t0, int& t1) {
  t0 = -1;
  t1 = -1;
  int j = 0;
#pragma unroll
  for (int a = 0; a < D; a++)
    if (a != dir) {
      if (j == 0) t0 = a; else t1 = a;
      j++;
    }
}

// Leaf / internal node face (Sec. 2): mean of the 2^{d-1} subface fluxes at
// level lev+1, from the leaf's virtual children (predicted from level lev's
// own stage state) and the neighbour's children (finer-side values: S1 q^n,
// S2 eq. projleaf / projnode, S3 stage-3 or eq. rk3proj values).
template <int D, int PDE>
__device__ __forceinline__ void refined_flux(const Geo& g, const LevTab& lt, const Dev& p, int lev, int stage,
                                             int64_t inst, const int* x, int dir, int side, int nbx, double* F) {
  constexpr int M = NC<D, PDE>::M;
  const double* cur = p.q[stage == 1 ? SL_Q0 : (stage == 2 ? SL_Q1 : SL_QH)];
  // level constants from the launch's LDS table (lev differs per lane)
  const int64_t ib = lt.off[lev] + inst * ((int64_t)1 << (D * lev));
  const int64_t ibf = lt.off[lev + 1] + inst * ((int64_t)1 << (D * (lev + 1)));
  double T[M][8];
#pragma unroll
  for (int k = 0; k < M; k++) {
    double S[27];
    if (!gather27<D>(g, p, cur, lev, ib, x, k, S)) flag_bad(p, inst, 2);
    pred_terms<D>(S, T[k]);
  }
  int t0, t1;
  transverse<D>(dir, t0, t1);
  double Fs[M], Fb[M];
#pragma unroll
  for (int b = 0; b < (1 << (D - 1)); b++) {
    int fy[3] = {2 * x[0], 2 * x[1], 2 * x[2]};
    int cbt = 0;
    if (t0 >= 0) { fy[t0] += b & 1; cbt |= (b & 1) << t0; }
    if (t1 >= 0) { fy[t1] += (b >> 1) & 1; cbt |= ((b >> 1) & 1) << t1; }
    double own[2][M], fin[2][M];
#pragma unroll
    for (int e = 0; e < 2; e++) {
      const int cb = cbt | (e << dir);
#pragma unroll
      for (int k = 0; k < M; k++) own[e][k] = pred_child<D>(T[k], cb);
      int y[3] = {fy[0], fy[1], fy[2]};
      y[dir] = 2 * nbx + e;
      const int64_t Gf = ibf + (int64_t)menc<D>(y);
      // the finer cell's status is read only to verify that the cell exists
      // (its stage-2 value is in its X2 slot whether it is a leaf or not)
      const uint8_t sf = g.check ? p.st[Gf] : (uint8_t)ST_LEAF;
      if (g.check && sf == ST_ABSENT) flag_bad(p, inst, 4);
#pragma unroll
      for (int k = 0; k < M; k++) {
        const int64_t I = (int64_t)k * g.Ntot + Gf;
        if (!g.lt) fin[e][k] = cur[I];
        else if (stage == 1) fin[e][k] = p.q[SL_Q0][I];
        else if (stage == 2) fin[e][k] = p.q[SL_X2][I];
        else fin[e][k] = p.q[SL_QE][I];
      }
    }
    double c[4][M];
#pragma unroll
    for (int k = 0; k < M; k++) {
      if (side) {
        c[0][k] = own[0][k]; c[1][k] = own[1][k]; c[2][k] = fin[0][k]; c[3][k] = fin[1][k];
      } else {
        c[0][k] = fin[0][k]; c[1][k] = fin[1][k]; c[2][k] = own[0][k]; c[3][k] = own[1][k];
      }
    }
    face_flux_ix<D, PDE>(g, lt.ix[lev + 1][dir], dir, adv_velocity<PDE>(g, p, inst, dir), c, Fb);
#pragma unroll
    for (int k = 0; k < M; k++) Fs[k] = (b == 0) ? Fb[k] : (Fs[k] + Fb[k]);
  }
  const double sc = D == 1 ? 1.0 : (D == 2 ? 0.5 : 0.25);
#pragma unroll
  for (int k = 0; k < M; k++) F[k] = Fs[k] * sc;
}

// IFACE = false: every leaf whose stencil reaches no internal cell (the bulk
// of the work, lean in registers); it reads only leaves and virtual cells of
// its own level, so one launch serves all levels of a stage.  IFACE = true:
// the leaves of levels below L whose stencil reaches an internal cell (a
// refined face neighbour, evaluated on the finer level, or an internal cell
// at distance 2 read through its projected value); they run level by level
// inside the stage sweeps.  The two sets are disjoint and every leaf writes
// only its own values and flux-register entries.  At the last stage, bulk
// leaves of levels >= lq0 (levels whose step both runs and ends in this
// fine iteration: the finest level under local time stepping, every level
// with one global step) also store their end value as q^n of the next
// step: no kernel reads a leaf's q^n after its last stage, and a bulk leaf
// has no refined face to correct.
template <int D, int PDE, bool IFACE, int stage>
__global__ __launch_bounds__(TPB) void k_stage(Geo g, Dev p, int lo, int hi, int lq0) {
  constexpr int M = NC<D, PDE>::M;
  constexpr double C_1_6 = 1.0 / 6.0, C_2_3 = 2.0 / 3.0, C_1_3 = 1.0 / 3.0;
  constexpr int LS = IFACE ? LS_IFACE : LS_LEAF;
  // leaf-stage updates of this bulk launch (measurement)
  if (!IFACE && blockIdx.x == 0 && threadIdx.x == 0) {
    unsigned long long it = 0ull;
    for (int lev = lo; lev <= hi; lev++)
      it += (unsigned long long)(list_len(p, LS_LEAF, lev) - (lev < g.L ? list_len(p, LS_IFACE, lev) : 0));
    atomicAdd(&p.items[stage - 1], it);
  }
  // one leaf-update per leaf and full RK step: counted once, at stage 1
  if (!IFACE && stage == 1 && blockIdx.x == 0) {
    const int nlv = hi - lo + 1;
    for (int j = threadIdx.x; j < g.B * nlv; j += blockDim.x) {
      const int inst = j / nlv, lev = lo + j % nlv;
      p.cnt[(int64_t)inst * CNT_PER_INST + CNT_LEVEL0 + lev] +=
          (unsigned long long)p.leafcnt[inst * (MRD_MAXLEV + 1) + lev];
    }
  }
  const int64_t NT = g.Ntot;
  const double* cur = p.q[stage == 1 ? SL_Q0 : (stage == 2 ? SL_Q1 : SL_QH)];
  // bulk leaves: the stencil values of every axis, the neighbour statuses
  // and the leaf's own slots are all requested before any of them is used
  // (one memory round trip per leaf), and the next list entry is fetched
  // while a leaf is processed; a leaf found to be an interface leaf is
  // computed but not stored.  Wide stencils of many fields load per axis.
  constexpr bool PRE = !IFACE && D * M <= 6;
  // many fields: the refined faces of the interface leaves were evaluated
  // by k_rface, one lane per face (inline, their registers would add to the
  // leaf's and leave one wave per SIMD)
  constexpr bool RSPLIT = IFACE && M >= 4;
  __shared__ int s_cnt[MRD_MAXLEV + 1];
  __shared__ LevTab lt;
  levtab_fill(g, lt);  // flat_setup synchronises
  const int64_t ntot = flat_setup(p, LS, lo, hi, s_cnt);
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  // bulk launches: runs of chunks per XCD (the stencil lines that
  // neighbouring chunks share then meet in one L2)
  const int bx = IFACE ? (int)blockIdx.x : xcd_run_block();
  int64_t i = (int64_t)bx * blockDim.x + threadIdx.x;
  // a lane's list positions only grow: its level and the offset of that
  // level in the flat index space are advanced, not searched again
  int lev_c = lo;
  int64_t base_c = 0;
  auto locate = [&](int64_t idx, int64_t& kk) {
    while (idx - base_c >= s_cnt[lev_c - lo]) {
      base_c += s_cnt[lev_c - lo];
      lev_c++;
    }
    kk = idx - base_c;
    return lev_c;
  };
  int lev_n = lo, e_n = 0;
  if (i < ntot) {
    int64_t kk;
    lev_n = locate(i, kk);
    e_n = p.lst[LS][lt.off[lev_n] + kk];
  }
  // Nagumo and linear diffusion read only the face neighbours: their bulk
  // leaves find them from the key bits (edge tests and dilated steps)
  // without decoding the coordinates, and use one key per neighbour for its
  // status and its value
  constexpr bool FAST = !IFACE && (PDE == PDE_NAGUMO || PDE == PDE_LINEAR);
  for (; i < ntot; i += step) {
    {
      const int lev = lev_n;
      const int64_t t = e_n;
      if (i + step < ntot) {
        int64_t kk;
        lev_n = locate(i + step, kk);
        e_n = p.lst[LS][lt.off[lev_n] + kk];
      }
      const int64_t nl = (int64_t)1 << (D * lev);
      const int n = 1 << lev;
      const bool finest = lev == g.L;
      const int64_t G = lt.off[lev] + t;
      const int64_t inst = t >> (D * lev);
      const uint64_t key = (uint64_t)(t & (nl - 1));
      int x[3] = {0, 0, 0};
      if (!FAST) mdec<D>(key, x);
      const int64_t ib = lt.off[lev] + inst * nl;
      // the tile flag that says whether the leaf keeps NERK values and the
      // instance's finest step, through the scalar data cache: each pass
      // serves the lanes that share the first pending lane's 4096-cell tile
      // and instance (one pass for most waves), so these values take no
      // vector memory instruction
      const bool tiled = !IFACE && !finest && g.lt && lt.wide[lev];
      const int64_t tix = tiled ? lt.bsoff[lev] + (t >> BS_SHIFT) : (int64_t)0;
      uint8_t nsv = 0;
      double dti = 0.0;
      for (bool pend = true; pend;) {
        const int64_t tix0 = rfl64(tix), inst0 = rfl64(inst);
        uint8_t ns;
        double dv;
        uload_u8_f64(p.nsum, tix0, p.dt, inst0, &ns, &dv);
        const bool mine = tix == tix0 && inst == inst0;
        nsv = mine ? ns : nsv;
        dti = mine ? dv : dti;
        pend = !mine;
      }
      const uint8_t nflag = tiled ? nsv : (uint8_t)1;
      // status of the 2d face neighbours (3: outside the domain); a cell
      // outside loads its own status instead, so that every load is issued
      // at once without a branch.  Bulk leaves in 1D and 2D read their list
      // code instead (one byte of their own, written by the compaction): it
      // says whether the stencil reaches an internal cell (the interface
      // launch owns the leaf) and which face neighbours are absent (the
      // fine side of a refined face); the other face neighbours of a bulk
      // leaf are leaves or virtual cells, which it reads alike.
      constexpr bool CODED = !IFACE && D <= 2;
      // (3D leaves take from it whether their stencil reaches an internal
      // cell, the reach-2 test included, and load the face statuses)
      const uint8_t code = IFACE ? (uint8_t)0 : p.ccode[G];
      int nbs[D][2];
      uint8_t sts[D][2];
      uint64_t fkey[D][2];  // key of the face neighbour (the cell itself outside the domain)
      bool fflip[D][2];     // FAST: Dirichlet sign of that value
      bool refined = false;
      if (FAST) {
        const uint32_t k32 = (uint32_t)key;
        const uint32_t lvm = (D * lev >= 32) ? ~0u : ((1u << (D * lev)) - 1u);
#pragma unroll
        for (int dir = 0; dir < D; dir++) {
          const uint32_t ma = axis_mask<D>(dir) & lvm;
          const uint32_t bits = k32 & ma;
#pragma unroll
          for (int side = 0; side < 2; side++) {
            const bool edge = side ? bits == ma : bits == 0u;
            const bool per = g.periodic[dir] != 0;
            uint64_t ky;
            if (!edge) ky = morton_step<D>(key, dir, side ? 1 : -1);
            else if (per) ky = (uint64_t)(side ? (k32 & ~ma) : ((k32 & ~ma) | ma));
            else ky = key;  // even or odd mirror: the cell itself
            const bool in = !edge || per;
            fkey[dir][side] = ky;
            fflip[dir][side] = edge && !per && ((g.dirichlet[dir] >> side) & 1);
            const uint8_t sv = CODED ? (((code >> (4 + 2 * dir + side)) & 1u) ? (uint8_t)ST_ABSENT : (uint8_t)ST_LEAF)
                                     : p.st[ib + (int64_t)ky];
            sts[dir][side] = in ? sv : (uint8_t)3;
            nbs[dir][side] = in ? 0 : -1;  // coordinates only where needed (below)
            refined = refined || (in && sv == ST_INTERNAL);
          }
        }
      } else {
#pragma unroll
        for (int dir = 0; dir < D; dir++)
#pragma unroll
          for (int side = 0; side < 2; side++) {
            const int nb = map_nb(x[dir] + (side ? 1 : -1), n, g.periodic[dir]);
            nbs[dir][side] = nb;
            uint64_t ky;
            const bool in = nbhd_key<D>(g, x, key, n, dir, side ? 1 : -1, &ky);
            const uint8_t sv = CODED ? (((code >> (4 + 2 * dir + side)) & 1u) ? (uint8_t)ST_ABSENT : (uint8_t)ST_LEAF)
                                     : p.st[ib + (int64_t)(in ? ky : key)];
            sts[dir][side] = in ? sv : (uint8_t)3;
            fkey[dir][side] = in ? ky : key;
            fflip[dir][side] = false;
            refined = refined || (in && sv == ST_INTERNAL);
          }
      }
      if (!IFACE) refined = (code & CODE_IFACE) != 0;
      // stencils of all axes (PRE) and the leaf's own slots
      double c5a[PRE ? D : 1][5][M];
      if (PRE) {
#pragma unroll
        for (int dir = 0; dir < (PRE ? D : 1); dir++)
#pragma unroll
          for (int o = -2; o <= 2; o++) {
            if (two_point<PDE>(g) && (o == -2 || o == 2)) continue;
            bool fl = false;
            int64_t Gy;
            if (o == 0) {
              Gy = G;
            } else if (FAST) {
              Gy = ib + (int64_t)fkey[dir][o > 0];
              fl = fflip[dir][o > 0];
            } else {
              Gy = ib + (int64_t)stencil_key<D>(g, x, key, n, dir, o, &fl);
            }
#pragma unroll
            for (int k = 0; k < M; k++) {
              const double v = cur[(int64_t)k * NT + Gy];
              c5a[dir][o + 2][k] = fl ? -v : v;
            }
          }
      }
      // the leaf's own slots; at stage 2 also the NERK partial values it adds
      // to where it keeps them (the loads that do not wait for the tile flag
      // go first)
      double q0v[M], qsv[M], n14v[M], n34v[M];
#pragma unroll
      for (int k = 0; k < M; k++) {
        const int64_t I = (int64_t)k * NT + G;
        q0v[k] = p.q[SL_Q0][I];
        qsv[k] = stage == 2 ? p.q[SL_Q1][I] : (stage == 3 ? p.q[SL_QH][I] : 0.0);
      }
#pragma unroll
      for (int k = 0; k < M; k++) n14v[k] = n34v[k] = 0.0;
      if (PRE && stage == 2 && g.lt && !finest && nflag != 0) {
        // only the leaves that keep NERK values read their partials: the
        // flag is per 4096-cell tile, so the branch is uniform over most
        // waves, and a load that is not issued costs no cache access
#pragma unroll
        for (int k = 0; k < M; k++) {
          const int64_t I = (int64_t)k * NT + G;
          n14v[k] = p.q[g.rk == 2 ? SL_QH : SL_N14][I];
          n34v[k] = g.rk == 2 ? 0.0 : p.q[SL_N34][I];
        }
      }
      if (!PRE && !IFACE && refined && !finest) continue;  // the interface launch owns it
      const bool active = IFACE || finest || !refined;
      const double h = g.lt ? ldexp(dti, g.L - lev) : dti;
      // weights b_i of the RK method: RK3 (1/6, 1/6, 2/3), RK2 (1/2, 1/2)
      const double wh = (g.rk == 2 ? 0.5 : (stage == 3 ? C_2_3 : C_1_6)) * h;
      double R[M];
#pragma unroll
      for (int dir = 0; dir < D; dir++) {
        double c5[5][M];
        if (PRE) {
#pragma unroll
          for (int o = 0; o < 5; o++)
#pragma unroll
            for (int k = 0; k < M; k++) c5[o][k] = c5a[PRE ? dir : 0][o][k];
        } else {
#pragma unroll
          for (int o = -2; o <= 2; o++) {
            // two-point diffusion needs only the face neighbours
            if (two_point<PDE>(g) && (o == -2 || o == 2)) continue;
            bool fl = false;
            const int64_t Gy = o == 0 ? G : ib + (int64_t)stencil_key<D>(g, x, key, n, dir, o, &fl);
#pragma unroll
            for (int k = 0; k < M; k++) {
              const double v = cur[(int64_t)k * NT + Gy];
              c5[o + 2][k] = fl ? -v : v;
            }
          }
        }
        if (two_point<PDE>(g)) {
#pragma unroll
          for (int k = 0; k < M; k++) c5[0][k] = c5[4][k] = 0.0;
        }
        const double vel = adv_velocity<PDE>(g, p, inst, dir);
        double Fm[M], Fp[M];
#pragma unroll
        for (int side = 0; side < 2; side++) {
          double* F = side ? Fp : Fm;
          if (IFACE && sts[dir][side] == ST_INTERNAL) {
            if (RSPLIT) {
#pragma unroll
              for (int k = 0; k < M; k++)
                F[k] = p.rflux[lt.rc[lev] + (int64_t)((2 * dir + side) * M + k) * (g.B * nl) + t];
            } else {
              refined_flux<D, PDE>(g, lt, p, lev, stage, inst, x, dir, side, nbs[dir][side], F);
            }
          }
          else
            face_flux_ix<D, PDE>(g, lt.ix[lev][dir], dir, vel, c5 + side, F);
        }
#pragma unroll
        for (int k = 0; k < M; k++) {
          const double r = (Fm[k] - Fp[k]) * lt.ix[lev][dir];
          R[k] = dir == 0 ? r : (R[k] + r);
        }
        if (g.reflux && active) {
#pragma unroll
          for (int side = 0; side < 2; side++) {
            const double* F = side ? Fp : Fm;
            if (IFACE && sts[dir][side] == ST_INTERNAL) {
#pragma unroll
              for (int k = 0; k < M; k++) {
                double* r = p.regc + lt.rc[lev] + (int64_t)((2 * dir + side) * g.m + k) * (g.B * nl) + t;
                *r = *r + (wh * F[k]);
              }
            } else if (sts[dir][side] == ST_ABSENT) {
              // fine side of a coarse leaf's refined face: the coarse leaf is
              // the parent of the absent neighbour (its key shifted by d
              // bits), and the subface is the leaf's position within its own
              // parent along the transverse axes (bit a of the key: x_a & 1)
              const int64_t tX = inst * (nl >> D) + (int64_t)(fkey[dir][side] >> D);
              if (g.check && p.st[lt.off[lev - 1] + tX] != ST_LEAF) flag_bad(p, inst, 8);
              int t0, t1;
              transverse<D>(dir, t0, t1);
              int b = 0;
              if (t0 >= 0) b |= (int)((key >> t0) & 1u);
              if (t1 >= 0) b |= (int)((key >> t1) & 1u) << 1;
              const int fX = 2 * dir + (side ? 0 : 1);
              for (int k = 0; k < M; k++) {
                double* r = p.regf + lt.rf[lev - 1] + (int64_t)((fX * g.nsub + b) * g.m + k) * (g.B * (nl >> D)) + tX;
                *r = *r + (wh * F[k]);
              }
            }
          }
        }
      }
      if (has_source<PDE>()) {
        // the stage value of the leaf itself: q^n, q* or q**
        double qs[M];
#pragma unroll
        for (int k = 0; k < M; k++) qs[k] = stage == 1 ? q0v[k] : qsv[k];
        add_source<PDE>(g, qs, R);
      }
      if (!active) continue;
      // the NERK values of a leaf (H1, N14, N34; the theta=1/2 value of RK2)
      // feed only the virtual cells of the next finer level, whose parent
      // stencils lie within Chebyshev distance 2 of an internal node of the
      // leaf's level; with one global step they are not used at all
      const bool nerk = !finest && g.lt && nflag != 0;
#pragma unroll
      for (int k = 0; k < M; k++) {
        const int64_t I = (int64_t)k * NT + G;
        const double q0 = q0v[k];
        const double r = R[k];
        if (g.rk == 2) {
          // compact RK2; the NERK theta=1/2 value in parts 3/8 and 1/8 (Sec. 3)
          if (stage == 1) {
            p.q[SL_Q1][I] = q0 + (h * r);
            if (nerk) {
              p.q[SL_H1][I] = q0 + ((0.5 * h) * r);
              p.q[SL_QH][I] = q0 + ((0.375 * h) * r);
            }
          } else {
            const double q1 = qsv[k];
            const double qe = ((0.5 * q0) + (0.5 * q1)) + ((0.5 * h) * r);
            p.q[SL_QE][I] = qe;
            if (!IFACE && lev >= lq0) p.q[SL_Q0][I] = qe;
            p.q[SL_X2][I] = q1 + (h * r);
            if (nerk) p.q[SL_QH][I] = (PRE ? n14v[k] : p.q[SL_QH][I]) + ((0.125 * h) * r);
            if (!isfinite(qe)) atomicOr(&p.cnt[inst * CNT_PER_INST + CNT_NONFINITE], 1ull);
          }
          continue;
        }
        if (stage == 1) {
          p.q[SL_Q1][I] = q0 + (h * r);
          if (nerk) {
            p.q[SL_H1][I] = q0 + ((0.5 * h) * r);
            p.q[SL_N14][I] = q0 + (((7.0 / 32.0) * h) * r);
            p.q[SL_N34][I] = q0 + (((15.0 / 32.0) * h) * r);
          }
        } else if (stage == 2) {
          const double q1 = qsv[k];
          p.q[SL_QH][I] = ((0.75 * q0) + (0.25 * q1)) + ((0.25 * h) * r);
          p.q[SL_X2][I] = q1 + (h * r);
          if (nerk) {
            // with few fields the partials were loaded with the stencil;
            // with many they are read here (registers)
            const double a14 = PRE ? n14v[k] : p.q[SL_N14][I];
            const double a34 = PRE ? n34v[k] : p.q[SL_N34][I];
            p.q[SL_N14][I] = a14 + (((1.0 / 32.0) * h) * r);
            p.q[SL_N34][I] = a34 + (((9.0 / 32.0) * h) * r);
          }
        } else {
          const double qh = qsv[k];
          const double qe = ((C_1_3 * q0) + (C_2_3 * qh)) + ((C_2_3 * h) * r);
          p.q[SL_QE][I] = qe;
          if (!IFACE && lev >= lq0) p.q[SL_Q0][I] = qe;
          if (!isfinite(qe)) atomicOr(&p.cnt[inst * CNT_PER_INST + CNT_NONFINITE], 1ull);
        }
      }
    }
  }
}

// Refined faces of the interface leaves of levels lo..hi (PDEs of four or
// more fields): one work item per (listed leaf, face); where the face
// neighbour is internal, the face flux (the mean of the 2^{d-1} subface
// fluxes, Sec. 2) is stored for the stage kernel, which reads it in place of
// evaluating it.  Same function, same arguments: the values are identical.
template <int D, int PDE, int stage>
__global__ __launch_bounds__(TPB) void k_rface(Geo g, Dev p, int lo, int hi) {
  constexpr int M = NC<D, PDE>::M;
  constexpr int NF = 2 * D;
  __shared__ int s_cnt[MRD_MAXLEV + 1];
  __shared__ LevTab lt;
  __shared__ int s_t[TPB], s_lev[TPB];  // the chunk's entries and their levels
  __shared__ int s_q[TPB * NF];         // its refined faces: lane << 3 | face
  __shared__ int s_n;
  levtab_fill(g, lt);  // flat_setup synchronises
  const int64_t ntot = flat_setup(p, LS_IFACE, lo, hi, s_cnt);
  // a chunk of TPB listed leaves per pass: each lane tests its leaf's faces
  // and queues the refined ones in LDS, then the lanes evaluate the queue
  // densely (few faces of an interface leaf are refined)
  for (int64_t base = (int64_t)blockIdx.x * TPB; base < ntot; base += (int64_t)gridDim.x * TPB) {
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    const int64_t i = base + threadIdx.x;
    if (i < ntot) {
      int64_t kk = i;
      const int lev = flat_level(s_cnt, lo, kk);
      const int t = p.lst[LS_IFACE][lt.off[lev] + kk];
      s_t[threadIdx.x] = t;
      s_lev[threadIdx.x] = lev;
      const int64_t nl = (int64_t)1 << (D * lev);
      const int n = 1 << lev;
      const uint64_t key = (uint64_t)((int64_t)t & (nl - 1));
      int x[3] = {0, 0, 0};
      mdec<D>(key, x);
      const int64_t ib = lt.off[lev] + ((int64_t)t >> (D * lev)) * nl;
      uint8_t sv[NF];
      bool in[NF];
#pragma unroll
      for (int f = 0; f < NF; f++) {
        uint64_t ky;
        in[f] = nbhd_key<D>(g, x, key, n, f >> 1, (f & 1) ? 1 : -1, &ky);
        sv[f] = p.st[ib + (int64_t)(in[f] ? ky : key)];
      }
#pragma unroll
      for (int f = 0; f < NF; f++)
        if (in[f] && sv[f] == ST_INTERNAL) s_q[atomicAdd(&s_n, 1)] = ((int)threadIdx.x << 3) | f;
    }
    __syncthreads();
    const int nq = s_n;
    for (int q = threadIdx.x; q < nq; q += TPB) {
      const int e = s_q[q];
      const int f = e & 7, ln = e >> 3;
      const int64_t t = s_t[ln];
      const int lev = s_lev[ln];
      const int64_t nl = (int64_t)1 << (D * lev);
      const int n = 1 << lev;
      const int64_t inst = t >> (D * lev);
      int x[3] = {0, 0, 0};
      mdec<D>((uint64_t)(t & (nl - 1)), x);
      const int dir = f >> 1, side = f & 1;
      const int nb = map_nb(x[dir] + (side ? 1 : -1), n, g.periodic[dir]);
      double F[M];
      refined_flux<D, PDE>(g, lt, p, lev, stage, inst, x, dir, side, nb, F);
#pragma unroll
      for (int k = 0; k < M; k++) p.rflux[lt.rc[lev] + (int64_t)(f * M + k) * (g.B * nl) + t] = F[k];
    }
    __syncthreads();  // s_t, s_q and s_n are rewritten by the next chunk
  }
}

// the stage is a template argument: the stage arrays a leaf reads and
// writes are known at compile time (its own value is loaded once)
template <int D, int PDE, bool IFACE>
static void stage_launch_st(int stage, int nb, const Geo& g, const Dev& p, int lo, int hi, int lq0, hipStream_t s) {
  if (stage == 1) k_stage<D, PDE, IFACE, 1><<<nb, TPB, 0, s>>>(g, p, lo, hi, lq0);
  else if (stage == 2) k_stage<D, PDE, IFACE, 2><<<nb, TPB, 0, s>>>(g, p, lo, hi, lq0);
  else k_stage<D, PDE, IFACE, 3><<<nb, TPB, 0, s>>>(g, p, lo, hi, lq0);
}

template <int D, int PDE>
static void stage_dp(const Geo& g, const Dev& p, int lo, int hi, int stage, int part, int lq0, hipStream_t s) {
  if (part == 0) {
    stage_launch_st<D, PDE, false>(stage, list_blocks(g, g.B * g.n[hi]), g, p, lo, hi, lq0, s);
    return;
  }
  const int hif = hi < g.L ? hi : g.L - 1;
  if (lo > hif) return;
  // interface leaves lie along refinement boundaries: a small fraction
  int nb = blocks_for(g.B * g.n[hif]);
  if (nb > g.iface_grid) nb = g.iface_grid;
  if constexpr (NC<D, PDE>::M >= 4) {
    const int nbf = nb;
    if (stage == 1) k_rface<D, PDE, 1><<<nbf, TPB, 0, s>>>(g, p, lo, hif);
    else if (stage == 2) k_rface<D, PDE, 2><<<nbf, TPB, 0, s>>>(g, p, lo, hif);
    else k_rface<D, PDE, 3><<<nbf, TPB, 0, s>>>(g, p, lo, hif);
  }
  stage_launch_st<D, PDE, true>(stage, nb, g, p, lo, hif, MRD_MAXLEV + 1, s);
}

template <int D>
static void stage_d(const Geo& g, const Dev& p, int lo, int hi, int stage, int part, int lq0, hipStream_t s) {
  switch (g.pde) {
    case PDE_ADVECTION: stage_dp<D, PDE_ADVECTION>(g, p, lo, hi, stage, part, lq0, s); break;
    case PDE_BURGERS: stage_dp<D, PDE_BURGERS>(g, p, lo, hi, stage, part, lq0, s); break;
    case PDE_NAGUMO: stage_dp<D, PDE_NAGUMO>(g, p, lo, hi, stage, part, lq0, s); break;
    case PDE_EULER: stage_dp<D, PDE_EULER>(g, p, lo, hi, stage, part, lq0, s); break;
    case PDE_FLAME: stage_dp<D, PDE_FLAME>(g, p, lo, hi, stage, part, lq0, s); break;
    case PDE_FLAMEBALL: stage_dp<D, PDE_FLAMEBALL>(g, p, lo, hi, stage, part, lq0, s); break;
    default: stage_dp<D, PDE_LINEAR>(g, p, lo, hi, stage, part, lq0, s); break;
  }
}

void launch_stage(const Geo& g, const Dev& p, int lo, int hi, int stage, int part, hipStream_t s, int lq0) {
  if (lo > hi) return;
  if (g.d == 1) stage_d<1>(g, p, lo, hi, stage, part, lq0, s);
  else if (g.d == 2) stage_d<2>(g, p, lo, hi, stage, part, lq0, s);
  else stage_d<3>(g, p, lo, hi, stage, part, lq0, s);
}

// ---------------------------------------------------------------------------
// end of the steps of a level: q^n <- stage-3 value, then on every refined
// face the conservative correction sigma (A_c - A_f) / dx (faces x-, x+,
// y-, y+, z-, z+), registers cleared after use.  Levels lo..min(hi, L-1):
// the finest level's leaves stored q^n in their last stage (they have no
// refined face).  Only interface leaves have refined faces: a plain copy
// over all leaves (list LS_LEAF, reflux 0), then the corrected values of
// the interface leaves (LS_IFACE, reflux 1) over it; with one global step
// every bulk leaf stored q^n itself and only the second pass runs.

template <int D>
__global__ __launch_bounds__(TPB) void k_finalize(Geo g, Dev p, int lo, int hi, int list, int reflux) {
  const double sc = D == 1 ? 1.0 : (D == 2 ? 0.5 : 0.25);
  constexpr int MF = D + 2;
  __shared__ int s_cnt[MRD_MAXLEV + 1];
  __shared__ LevTab lt;
  levtab_fill(g, lt);  // flat_setup synchronises
  const int64_t ntot = flat_setup(p, list, lo, hi, s_cnt);
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool regs_on = reflux && g.reflux;
  // the next list entry is fetched while a leaf is processed (a lane's list
  // positions only grow, so its level is advanced, not searched again)
  int lev_c = lo;
  int64_t base_c = 0;
  auto locate = [&](int64_t idx) {
    while (idx - base_c >= s_cnt[lev_c - lo]) {
      base_c += s_cnt[lev_c - lo];
      lev_c++;
    }
    return idx - base_c;
  };
  int lev_n = lo, t_n = 0;
  if (i < ntot) {
    const int64_t kk = locate(i);
    lev_n = lev_c;
    t_n = p.lst[list][lt.off[lev_n] + kk];
  }
  vm_wait_all();  // the first entry: no wait at the loop's top (see k_project)
  for (; i < ntot; i += step) {
    const int lev = lev_n;
    const int64_t t = t_n;
    if (i + step < ntot) {
      const int64_t kk = locate(i + step);
      lev_n = lev_c;
      t_n = p.lst[list][lt.off[lev_n] + kk];
    }
    const int64_t G = lt.off[lev] + t;
    double q[MF];
#pragma unroll
    for (int k = 0; k < MF; k++)
      if (k < g.m) q[k] = p.q[SL_QE][(int64_t)k * g.Ntot + G];
    if (regs_on && lev < g.L) {
      // the statuses of the 2d face neighbours, requested with the end
      // values (a neighbour outside the domain reads the leaf's own status)
      const int64_t nl = (int64_t)1 << (D * lev), Nl = g.B * nl;
      const int n = 1 << lev;
      int x[3] = {0, 0, 0};
      mdec<D>((uint64_t)(t & (nl - 1)), x);
      const int64_t ib = lt.off[lev] + (t >> (D * lev)) * nl;
      uint8_t sn[D][2];
#pragma unroll
      for (int dir = 0; dir < D; dir++)
#pragma unroll
        for (int side = 0; side < 2; side++) {
          const int nb = map_nb(x[dir] + (side ? 1 : -1), n, g.periodic[dir]);
          int y[3] = {x[0], x[1], x[2]};
          if (nb >= 0) y[dir] = nb;
          sn[dir][side] = p.st[ib + (int64_t)menc<D>(y)];
        }
#pragma unroll
      for (int dir = 0; dir < D; dir++)
#pragma unroll
        for (int side = 0; side < 2; side++) {
          if (sn[dir][side] != ST_INTERNAL) continue;  // the leaf itself, or no refined face
          const int f = 2 * dir + side;
#pragma unroll
          for (int k = 0; k < MF; k++) {
            if (k >= g.m) break;
            double af = 0.0;
            for (int b = 0; b < (1 << (D - 1)); b++) {
              double* r = p.regf + lt.rf[lev] + (int64_t)((f * g.nsub + b) * g.m + k) * Nl + t;
              af = (b == 0) ? *r : (af + *r);
              *r = 0.0;
            }
            af = af * sc;
            double* rc = p.regc + lt.rc[lev] + (int64_t)(f * g.m + k) * Nl + t;
            const double Dd = (*rc - af) * lt.ix[lev][dir];
            *rc = 0.0;
            q[k] = side ? q[k] + Dd : q[k] - Dd;
          }
        }
    }
#pragma unroll
    for (int k = 0; k < MF; k++)
      if (k < g.m) p.q[SL_Q0][(int64_t)k * g.Ntot + G] = q[k];
  }
}

void launch_finalize(const Geo& g, const Dev& p, int lo, int hi, bool iface_only, hipStream_t s) {
  if (hi > g.L - 1) hi = g.L - 1;  // the finest level is done
  if (lo > hi) return;
  const int64_t n = g.B * g.n[hi];
  const int nb = list_blocks(g, n);
  for (int pass = iface_only ? 1 : 0; pass < 2; pass++) {
    const int list = pass ? LS_IFACE : LS_LEAF;
    const int nbp = pass ? (nb < g.iface_grid ? nb : g.iface_grid) : nb;
    if (g.d == 1) k_finalize<1><<<nbp, TPB, 0, s>>>(g, p, lo, hi, list, pass);
    else if (g.d == 2) k_finalize<2><<<nbp, TPB, 0, s>>>(g, p, lo, hi, list, pass);
    else k_finalize<3><<<nbp, TPB, 0, s>>>(g, p, lo, hi, list, pass);
  }
}

__global__ void k_zero(double* a, int64_t n) { GSL(t, n) a[t] = 0.0; }

void launch_clear_regs(const Geo& g, const Dev& p, hipStream_t s) {
  const int64_t nc = g.rc_off[g.L], nf = g.rf_off[g.L];
  if (nc > 0) k_zero<<<blocks_for(nc), TPB, 0, s>>>(p.regc, nc);
  if (nf > 0) k_zero<<<blocks_for(nf), TPB, 0, s>>>(p.regf, nf);
}

// ---------------------------------------------------------------------------
// remesh (Alg. AdaptiveMesh, Alg. waveletThres; only scales evolved in the
// current iteration may split or merge).  Levels below la are frozen.  The
// set W of nodes that will be internal is built in the remesh byte table:
//   detail + seed (one pass over the internal nodes): a node is significant
//            when max_{c,k} |q_c - q~_c| / scale_k > eps_{l+1} (level-
//            dependent 2^{d(l+1-L)} eps; eps = 0 keeps every node); it puts
//            itself, its existing neighbours at distance 1 (space safety)
//            and, below L-1, its children (scale safety) into W
//   close:   least superset closed under the tree rule and the radius-2
//            grading rule; every implication points one level down, so one
//            fine-to-coarse sweep: each W node at l+1 adds the 3^d cells of
//            level l whose children's radius-2 neighbourhood holds it
//   prune:   greatest subset still satisfying both rules with existence
//            frozen at la; one coarse-to-fine sweep
//   apply:   new status, new nodes predicted from the parent level
// Marks only ever grow inside a pass, so the passes that add them use
// atomic ORs on the 32-bit word holding the byte and give the same set in
// any order.  The dense passes read 16 cells per lane with one 16-byte load;
// a block gathers the cells that need work into shared memory and then
// spreads them over its lanes.

static constexpr uint8_t RF_W = 2;
// block summaries (4096-cell blocks of a level): any cell exists / is
// internal / is a leaf
static constexpr unsigned BS_EXIST = 1u, BS_INT = 2u, BS_LEAF = 4u;
// level flags (Dev::lflag): a cell / leaf / internal node exists (set by
// every list compaction from its totals), some W mark exists (set before
// the apply passes), a cell exists after this remesh's apply pass
static constexpr unsigned LF_EXIST = 1u, LF_LEAF = 2u, LF_INT = 4u, LF_W = 8u, LF_NEW = 16u;
static constexpr int GRP = 16;            // cells per lane in the dense passes of large levels

// true when the cell's instance is outside the remesh window
__device__ __forceinline__ bool inst_of_window_skip(const Geo& g, int64_t t, int shift) {
  const int64_t inst = t >> shift;
  return inst < g.i0 || inst >= g.i1;
}

// bytes of cells [t0, t0+16) of a level table (zero past the level end);
// level tables start at multiples of 256 cells, so the load is aligned
__device__ __forceinline__ uint4 ld16(const uint8_t* base, int64_t t0, int64_t N) {
  // 16-cell groups are used on levels of at least 4096 cells per instance
  // (wide levels), so N and t0 are multiples of 16: a group is whole or
  // past the end.  No partial-group path: its branch would make the
  // compiler wait for the group's load where the two paths join.
  return t0 < N ? *reinterpret_cast<const uint4*>(base + t0) : make_uint4(0u, 0u, 0u, 0u);
}
// G = 16: ld16; G = 1: the one byte of cell t0 (zero past the level end)
template <int G>
__device__ __forceinline__ uint4 ldg(const uint8_t* base, int64_t t0, int64_t N) {
  if (G == 16) return ld16(base, t0, N);
  return make_uint4(t0 < N ? (uint32_t)base[t0] : 0u, 0u, 0u, 0u);
}
__device__ __forceinline__ uint8_t byte_of(const uint4& v, int j) {
  const uint32_t w = j < 4 ? v.x : (j < 8 ? v.y : (j < 12 ? v.z : v.w));
  return (uint8_t)(w >> (8 * (j & 3)));
}
__device__ __forceinline__ bool any16(const uint4& v, uint32_t mask) {
  return ((v.x | v.y | v.z | v.w) & mask) != 0u;
}
// the 16 >> D parent statuses of a group (parent k of cell j: k = j >> D);
// with G = 1 the parent of cell t0
template <int D, int G = 16>
__device__ __forceinline__ uint64_t ld_parents(const uint8_t* stp, int64_t t0, int64_t N) {
  const int64_t p0 = t0 >> D;
  if (G == 1) return t0 < N ? (uint64_t)stp[p0] : 0ull;
  // whole groups only (see ld16)
  if (t0 >= N) return 0ull;
  if (D == 1) return *reinterpret_cast<const uint64_t*>(stp + p0);
  if (D == 2) return *reinterpret_cast<const uint32_t*>(stp + p0);
  return *reinterpret_cast<const uint16_t*>(stp + p0);
}

// block summary of a wide level; unknown (all bits) elsewhere
__device__ __forceinline__ unsigned bsum_of(const Geo& g, const Dev& p, int lev, int64_t sb) {
  return wide_level(g, lev) ? p.bsum[g.bs_off[lev] + sb] : 0xffu;
}

// cell t of level lev into W; its 4096-cell block is flagged in wsum (every
// writer of the flag stores the same value)
__device__ __forceinline__ void mark_w(const Geo& g, const Dev& p, int lev, int64_t t) {
  const int64_t G = g.off[lev] + t;
  atomicOr(reinterpret_cast<unsigned*>(p.rf + (G & ~(int64_t)3)), (unsigned)RF_W << (8 * (int)(G & 3)));
  p.wsum[g.bs_off[lev] + (t >> BS_SHIFT)] = 1;
}
// the same with the level constants from the launch's table in LDS
__device__ __forceinline__ void mark_w(const LevTab& lt, const Dev& p, int lev, int64_t t) {
  const int64_t G = lt.off[lev] + t;
  atomicOr(reinterpret_cast<unsigned*>(p.rf + (G & ~(int64_t)3)), (unsigned)RF_W << (8 * (int)(G & 3)));
  p.wsum[lt.bsoff[lev] + (t >> BS_SHIFT)] = 1;
}
// A marking pass first reads the current bytes of all its targets (loads
// only, so they are in flight together), then sets the missing marks (atomics
// only): one memory round trip per item, and no atomic for a mark that is
// already there.

// exclusive scan over the 256 threads of a block: a shuffle scan inside
// each 64-lane wave, the wave totals through shared memory (sh: TPB / 64
// entries); *tot receives the block total.  Two barriers.
template <class T>
__device__ __forceinline__ T block_exscan(T v, T* sh, T* tot) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  T x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const T u = __shfl_up(x, (unsigned)o, 64);
    if (lane >= o) x += u;
  }
  if (lane == 63) sh[wv] = x;
  __syncthreads();
  T pre = (T)0, all = (T)0;
#pragma unroll
  for (int w = 0; w < TPB / 64; w++) {
    const T s = sh[w];
    if (w < wv) pre += s;
    all += s;
  }
  *tot = all;
  __syncthreads();  // sh is free again on return
  return pre + x - v;
}

// block-wide gather of work cells: lane i offers the cells of its group
// flagged in `mask`; returns their number, block-local indices in `items`
template <int G>
__device__ __forceinline__ int block_items(uint32_t mask, int* items, int* sh) {
  if (!__syncthreads_or(mask != 0u)) return 0;  // nothing anywhere: one barrier
  int tot;
  int k = block_exscan<int>(__popc(mask), sh, &tot);
  while (mask) {
    const int j = __builtin_ctz(mask);
    mask &= mask - 1u;
    items[k++] = (int)threadIdx.x * G + j;
  }
  __syncthreads();
  return tot;
}

// block-wide gather of sibling groups: with 16-cell lane groups, one work
// item per sibling group (2^d cells with one parent) that has a cell in
// `mask`, the group's first cell in bits 0-15 and the child mask in bits
// 16-23; with one cell per lane (G = 1), one item per cell as block_items.
// Returns their number.
template <int D, int G>
__device__ __forceinline__ int block_sib_items(uint32_t mask, int* items, int* sh) {
  if (G == 1) {
    const int cnt = block_items<G>(mask, items, sh);
    return cnt;
  }
  constexpr uint32_t CM = (1u << (1 << D)) - 1u;
  uint32_t gmask = 0u;
#pragma unroll
  for (int gi = 0; gi < (16 >> D); gi++)
    if ((mask >> (gi << D)) & CM) gmask |= 1u << gi;
  if (!__syncthreads_or(gmask != 0u)) return 0;
  int tot;
  int k = block_exscan<int>(__popc(gmask), sh, &tot);
  while (gmask) {
    const int gi = __builtin_ctz(gmask);
    gmask &= gmask - 1u;
    items[k++] = ((int)threadIdx.x * 16 + (gi << D)) | (int)(((mask >> (gi << D)) & CM) << 16);
  }
  __syncthreads();
  return tot;
}
// an item of block_sib_items: first cell (within-level index) and child mask
template <int D, int G>
__device__ __forceinline__ int64_t sib_item(int it, int64_t tb, uint32_t* cbits) {
  if (G == 1) {
    const int64_t t = tb + it;
    *cbits = 1u << (int)(t & ((1 << D) - 1));
    return t & ~(int64_t)((1 << D) - 1);
  }
  *cbits = (uint32_t)it >> 16;
  return tb + (it & 0xffff);
}

// remesh table and W flags cleared on levels lo..hi: one workgroup per
// 4096-cell block, only blocks flagged in wsum hold marks
__global__ __launch_bounds__(TPB) void k_clear_w(Geo g, Dev p, int lo, int hi) {
  for (int64_t sb = g.bs_off[lo] + blockIdx.x; sb < g.bs_off[hi + 1]; sb += gridDim.x) {
    if (p.wsum[sb] == 0) continue;
    int lev = lo;
    while (sb >= g.bs_off[lev + 1]) lev++;
    const int64_t n256 = (g.B * g.n[lev] + 255) & ~(int64_t)255;  // padded level table
    const int64_t t = ((sb - g.bs_off[lev]) << BS_SHIFT) + (int64_t)threadIdx.x * 16;
    if (t < n256) *reinterpret_cast<uint4*>(p.rf + g.off[lev] + t) = make_uint4(0u, 0u, 0u, 0u);
    __syncthreads();
    if (threadIdx.x == 0) p.wsum[sb] = 0;
  }
}

// before the apply passes of a remesh at la: LF_W on levels la..L-1 from
// the block W flags, LF_NEW cleared on levels la..L (one workgroup)
__global__ __launch_bounds__(TPB) void k_level_w(Geo g, Dev p, int la) {
  for (int lev = la; lev <= g.L; lev++) {
    int any = 0;
    if (lev <= g.L - 1)
      for (int64_t j = g.bs_off[lev] + threadIdx.x; j < g.bs_off[lev + 1]; j += TPB) any |= p.wsum[j];
    any = __syncthreads_or(any);
    if (threadIdx.x == 0) p.lflag[lev] = (p.lflag[lev] & ~(LF_W | LF_NEW)) | (any ? LF_W : 0u);
  }
}

// Internal nodes of levels lo..hi: lo = la evaluates details from la on;
// lo = la - 1 also visits the frozen level la - 1, whose nodes keep the
// significance of their last evaluation (sigt) and pass on only their scale
// safety (Sec. 4: apart from which scales may split or merge, the LT remesh
// is the multiresolution remesh).
template <int D>
__global__ __launch_bounds__(TPB) void k_detail_seed(Geo g, Dev p, int lo, int hi, int la, int n_it) {
  __shared__ int s_cnt[MRD_MAXLEV + 1];
  __shared__ LevTab lt;
  levtab_fill(g, lt);  // flat_setup synchronises
  const int64_t ntot = flat_setup(p, LS_INTERNAL, lo, hi, s_cnt);
  GSL(i, ntot) {
    {
      int64_t kk = i;
      const int lev = flat_level(s_cnt, lo, kk);
      const int64_t nl = (int64_t)1 << (D * lev);
      const int n = 1 << lev;
      const int64_t t = p.lst[LS_INTERNAL][lt.off[lev] + kk];
      if (inst_of_window_skip(g, t, D * lev)) continue;
      const int64_t inst = t >> (D * lev);
      const int Lc = p.lcap[inst];  // the instance's finest level
      if (lev < la) {
        // frozen level: scale safety of a node significant at its last remesh
        if (!p.sigt[lt.off[lev] + t] || lev + 1 > Lc - 1) continue;
        uint32_t need = 0u;
#pragma unroll
        for (int cb = 0; cb < (1 << D); cb++)
          if (!(p.rf[lt.off[lev + 1] + (t << D) + cb] & RF_W)) need |= 1u << cb;
#pragma unroll
        for (int cb = 0; cb < (1 << D); cb++)
          if ((need >> cb) & 1u) mark_w(lt, p, lev + 1, (t << D) + cb);
        continue;
      }
      const int64_t ib = lt.off[lev] + inst * nl;
      int x[3];
      mdec<D>((uint64_t)(t & (nl - 1)), x);
      const double e0 = p.eps[inst];
      bool sig = true;
      if (e0 != 0.0) {
        const double e = g.thresh ? ldexp(e0, D * (lev + 1 - Lc)) : e0;
        const int64_t C0 = lt.off[lev + 1] + (t << D);
        double Dm = 0.0;
        for (int k = 0; k < g.m; k++) {
          double S[27], T[8];
          if (!gather27<D>(g, p, p.q[SL_Q0], lev, ib, x, k, S)) flag_bad(p, inst, 16);
          pred_terms<D>(S, T);
#pragma unroll
          for (int cb = 0; cb < (1 << D); cb++) {
            const double det = fabs(p.q[SL_Q0][(int64_t)k * g.Ntot + C0 + cb] - pred_child<D>(T, cb)) / g.scale[k];
            if (det > Dm) Dm = det;
          }
        }
        sig = Dm > e;
        if (fabs(Dm - e) <= 1e-12 * e) {
          atomicAdd(&p.cnt[inst * CNT_PER_INST + CNT_NEAR], 1ull);
          const unsigned long long j = atomicAdd(p.near_n, 1ull);
          if (j < NEAR_CAP) {
            p.near[2 * j] = (unsigned long long)(*p.iterb + n_it);
            p.near[2 * j + 1] = ((unsigned long long)inst << 45) | ((unsigned long long)lev << 40) |
                                (unsigned long long)(t & (nl - 1));
          }
        }
      }
      p.sigt[lt.off[lev] + t] = sig ? 1 : 0;
      if (!sig) continue;
      // targets: the 3^d neighbourhood (existing cells; the node itself is
      // internal) and, below L-1, the 2^d children
      constexpr int NN = D == 1 ? 3 : (D == 2 ? 9 : 27);
      const bool kids = lev + 1 <= Lc - 1;
      // the targets' statuses and marks are requested together (a target
      // outside the domain reads the node's own bytes, masked; the children's
      // marks are read whether or not they are targets)
      uint8_t sv[NN], rv[NN], rk[1 << D];
      bool inb[NN];
#pragma unroll
      for (int o = 0; o < NN; o++) {
        const int ox = o % 3 - 1, oy = D > 1 ? (o / 3) % 3 - 1 : 0, oz = D > 2 ? o / 9 - 1 : 0;
        int y[3] = {map_nb(x[0] + ox, n, g.periodic[0]), 0, 0};
        if (D > 1) y[1] = map_nb(x[1] + oy, n, g.periodic[1]);
        if (D > 2) y[2] = map_nb(x[2] + oz, n, g.periodic[2]);
        inb[o] = y[0] >= 0 && y[1] >= 0 && y[2] >= 0;
        const int yc[3] = {y[0] < 0 ? 0 : y[0], y[1] < 0 ? 0 : y[1], y[2] < 0 ? 0 : y[2]};
        const int64_t Gy = inb[o] ? ib + (int64_t)menc<D>(yc) : lt.off[lev] + t;
        sv[o] = p.st[Gy];
        rv[o] = p.rf[Gy];
      }
#pragma unroll
      for (int cb = 0; cb < (1 << D); cb++) rk[cb] = p.rf[lt.off[lev + 1] + (t << D) + cb];
      uint64_t need = 0ull;
#pragma unroll
      for (int o = 0; o < NN; o++)
        if (inb[o] && sv[o] != ST_ABSENT && !(rv[o] & RF_W)) need |= 1ull << o;
      if (kids) {
#pragma unroll
        for (int cb = 0; cb < (1 << D); cb++)
          if (!(rk[cb] & RF_W)) need |= 1ull << (NN + cb);
      }
#pragma unroll
      for (int o = 0; o < NN; o++) {
        if (!((need >> o) & 1ull)) continue;
        const int ox = o % 3 - 1, oy = D > 1 ? (o / 3) % 3 - 1 : 0, oz = D > 2 ? o / 9 - 1 : 0;
        int y[3] = {map_nb(x[0] + ox, n, g.periodic[0]), 0, 0};
        if (D > 1) y[1] = map_nb(x[1] + oy, n, g.periodic[1]);
        if (D > 2) y[2] = map_nb(x[2] + oz, n, g.periodic[2]);
        mark_w(lt, p, lev, inst * nl + (int64_t)menc<D>(y));
      }
#pragma unroll
      for (int cb = 0; cb < (1 << D); cb++)
        if ((need >> (NN + cb)) & 1ull) mark_w(lt, p, lev + 1, (t << D) + cb);
    }
  }
}

// mask of the W cells of a group inside the remesh window
template <int G>
__device__ __forceinline__ uint32_t w_mask(const Geo& g, const uint4& v, int64_t t0, int shift) {
  uint32_t mask = 0u;
  if (!any16(v, 0x02020202u)) return 0u;
  if (G == 1) return inst_of_window_skip(g, t0, shift) ? 0u : 1u;
#pragma unroll
  for (int j = 0; j < 16; j++)
    if (byte_of(v, j) & RF_W) mask |= 1u << j;
  // a group never straddles two instances unless the level has < 16 cells
  if (mask && (inst_of_window_skip(g, t0, shift) || inst_of_window_skip(g, t0 + 15, shift)))
    for (int j = 0; j < 16; j++)
      if (inst_of_window_skip(g, t0 + j, shift)) mask &= ~(1u << j);
  return mask;
}

// W nodes of level lev+1 put the cells of level lev into W whose children's
// radius-2 neighbourhood (fine offsets -2..3 per axis) holds them: per axis
// the coarse cells (y >> 1) + {-1, 0, 1}, mapped by the boundary conditions
template <int D, int G>
__global__ __launch_bounds__(TPB) void k_close(Geo g, Dev p, int lev) {
  __shared__ int sh[TPB];
  __shared__ int items[TPB * G];
  const int lf = lev + 1;
  const int64_t nf = g.n[lf], N = g.B * nf;
  const int nc = 1 << lev;
  const uint8_t* rff = p.rf + g.off[lf];
  for (int64_t tb = (int64_t)blockIdx.x * (TPB * G); tb < N; tb += (int64_t)gridDim.x * (TPB * G)) {
    if (p.wsum[g.bs_off[lf] + (tb >> BS_SHIFT)] == 0) continue;  // no W in the block
    const int64_t t0 = tb + (int64_t)threadIdx.x * G;
    const uint32_t mask = t0 < N ? w_mask<G>(g, ldg<G>(rff, t0, N), t0, D * lf) : 0u;
    // the marks depend only on the parent: one item per sibling group
    const int cnt = block_sib_items<D, G>(mask, items, sh);
    for (int i = threadIdx.x; i < cnt; i += TPB) {
      uint32_t cbits;
      const int64_t t = sib_item<D, G>(items[i], tb, &cbits);
      const int64_t inst = t >> (D * lf);
      const int64_t ibc = inst * g.n[lev];
      int y[3];
      mdec<D>((uint64_t)(t & (nf - 1)), y);
      constexpr int NN = D == 1 ? 3 : (D == 2 ? 9 : 27);
      // the targets' marks are requested together (a target outside the
      // domain reads the parent's own byte, masked)
      const int yp[3] = {y[0] >> 1, y[1] >> 1, y[2] >> 1};
      uint8_t rv[NN];
      bool inb[NN];
#pragma unroll
      for (int o = 0; o < NN; o++) {
        const int ox = o % 3 - 1, oy = D > 1 ? (o / 3) % 3 - 1 : 0, oz = D > 2 ? o / 9 - 1 : 0;
        int X[3] = {map_nb(yp[0] + ox, nc, g.periodic[0]), 0, 0};
        if (D > 1) X[1] = map_nb(yp[1] + oy, nc, g.periodic[1]);
        if (D > 2) X[2] = map_nb(yp[2] + oz, nc, g.periodic[2]);
        inb[o] = X[0] >= 0 && X[1] >= 0 && X[2] >= 0;
        rv[o] = p.rf[g.off[lev] + ibc + (int64_t)menc<D>(inb[o] ? X : yp)];
      }
      uint32_t need = 0u;
#pragma unroll
      for (int o = 0; o < NN; o++)
        if (inb[o] && !(rv[o] & RF_W)) need |= 1u << o;
#pragma unroll
      for (int o = 0; o < NN; o++) {
        if (!((need >> o) & 1u)) continue;
        const int ox = o % 3 - 1, oy = D > 1 ? (o / 3) % 3 - 1 : 0, oz = D > 2 ? o / 9 - 1 : 0;
        int X[3] = {map_nb((y[0] >> 1) + ox, nc, g.periodic[0]), 0, 0};
        if (D > 1) X[1] = map_nb((y[1] >> 1) + oy, nc, g.periodic[1]);
        if (D > 2) X[2] = map_nb((y[2] >> 1) + oz, nc, g.periodic[2]);
        mark_w(g, p, lev, ibc + (int64_t)menc<D>(X));
      }
    }
    __syncthreads();
  }
}

// a W node of level lev > l0 stays in W only if the 3^d neighbourhood of its
// parent is in W (levels >= la) or internal (frozen levels)
template <int D, int G>
__global__ __launch_bounds__(TPB) void k_prune(Geo g, Dev p, int lev, int la) {
  __shared__ int sh[TPB];
  __shared__ int items[TPB * G];
  const int64_t nl = g.n[lev], N = g.B * nl;
  const int np = 1 << (lev - 1);
  uint8_t* rfl = p.rf + g.off[lev];
  for (int64_t tb = (int64_t)blockIdx.x * (TPB * G); tb < N; tb += (int64_t)gridDim.x * (TPB * G)) {
    if (p.wsum[g.bs_off[lev] + (tb >> BS_SHIFT)] == 0) continue;  // no W in the block
    const int64_t t0 = tb + (int64_t)threadIdx.x * G;
    const uint32_t mask = t0 < N ? w_mask<G>(g, ldg<G>(rfl, t0, N), t0, D * lev) : 0u;
    // the test depends only on the parent: one item per sibling group
    const int cnt = block_sib_items<D, G>(mask, items, sh);
    for (int i = threadIdx.x; i < cnt; i += TPB) {
      uint32_t cbits;
      const int64_t t = sib_item<D, G>(items[i], tb, &cbits);
      const int64_t inst = t >> (D * lev);
      int x[3];
      mdec<D>((uint64_t)(t & (nl - 1)), x);
      const int px[3] = {x[0] >> 1, x[1] >> 1, x[2] >> 1};
      const int64_t ibp = g.off[lev - 1] + inst * g.n[lev - 1];
      // the parent neighbourhood's bytes are requested together (outside
      // the domain: the parent's own byte, masked); above la the W marks,
      // on the frozen level the statuses
      const bool wl = lev - 1 >= la;
      const uint8_t* tab = wl ? p.rf : p.st;
      constexpr int NN = D == 1 ? 3 : (D == 2 ? 9 : 27);
      uint8_t v[NN];
      bool inb[NN];
#pragma unroll
      for (int o = 0; o < NN; o++) {
        const int ox = o % 3 - 1, oy = D > 1 ? (o / 3) % 3 - 1 : 0, oz = D > 2 ? o / 9 - 1 : 0;
        int y[3] = {map_nb(px[0] + ox, np, g.periodic[0]), 0, 0};
        if (D > 1) y[1] = map_nb(px[1] + oy, np, g.periodic[1]);
        if (D > 2) y[2] = map_nb(px[2] + oz, np, g.periodic[2]);
        inb[o] = y[0] >= 0 && y[1] >= 0 && y[2] >= 0;
        v[o] = tab[ibp + (int64_t)menc<D>(inb[o] ? y : px)];
      }
      bool ok = true;
#pragma unroll
      for (int o = 0; o < NN; o++)
        if (inb[o]) ok = ok & (wl ? ((v[o] & RF_W) != 0) : (v[o] == ST_INTERNAL));
      if (!ok) {
#pragma unroll
        for (int cb = 0; cb < (1 << D); cb++)
          if ((cbits >> cb) & 1u) rfl[t + cb] = 0;  // the byte holds only the W bit
      }
    }
    __syncthreads();
  }
}

// summary bits of eight packed statuses
__device__ __forceinline__ unsigned group_summary(uint64_t s) {
  const uint64_t lo = s & 0x0101010101010101ull, hi = (s >> 1) & 0x0101010101010101ull;
  return (s ? BS_EXIST : 0u) | (lo ? BS_LEAF : 0u) | (hi ? BS_INT : 0u);
}

// new status of the cells of level lev (parents already updated); cells
// that come into existence get the value predicted from the parent level
template <int D, int G>
__global__ __launch_bounds__(TPB) void k_apply(Geo g, Dev p, int lev, int la) {
  __shared__ int sh[TPB];
  __shared__ int items[TPB * G];
  __shared__ unsigned bor;
  const int64_t nl = g.n[lev], N = g.B * nl;
  uint8_t* stl = p.st + g.off[lev];
  const uint8_t* stp = p.st + g.off[lev - 1];
  // the whole level stays absent: nothing exists on it and no parent will
  // be internal (W marks above la, internal nodes on the frozen level)
  {
    const unsigned fl = p.lflag[lev], fp = lev > g.l0 ? p.lflag[lev - 1] : 0u;
    if (!(fl & LF_EXIST) && (lev == la || !(fp & (lev - 1 >= la ? LF_W : LF_INT)))) return;
  }
  if (threadIdx.x == 0) bor = 0u;
  __syncthreads();
  // block summaries of the level and, where it keeps them, of the parent
  // level (else the level's own are read again and ignored, and every
  // block is visited); on the frozen level la no parent can turn a cell
  // into existence
  const bool pw = lev > la && wide_level(g, lev - 1);
  const uint8_t* bs_lev = p.bsum + (G == 16 ? g.bs_off[lev] : 0);
  const uint8_t* bs_up = pw ? p.bsum + g.bs_off[lev - 1] : bs_lev;
  const int bs_up_shift = pw ? D : 0;
  const unsigned bs_up_mask = pw ? (unsigned)BS_INT : 0u;
  const unsigned bs_visit = (lev > la && !pw) ? 1u : 0u;  // parent level unknown: always visit
  for (int64_t tb = (int64_t)blockIdx.x * (TPB * G); tb < N; tb += (int64_t)gridDim.x * (TPB * G)) {
    // nothing exists in the block and no parent is internal: it stays absent
    const int64_t sb = tb >> BS_SHIFT;
    bool skip;
    if (G == 16) {
      // a wide level: both summaries in one round trip (where the parent
      // level keeps none, the own one is read again and "unknown" taken)
      const unsigned b_own = bs_lev[sb];
      const unsigned b_par = bs_up[sb >> bs_up_shift];
      skip = ((b_own & BS_EXIST) | (b_par & bs_up_mask) | bs_visit) == 0u;
    } else {
      skip = !(bsum_of(g, p, lev, sb) & BS_EXIST) && (lev == la || !(bsum_of(g, p, lev - 1, sb >> D) & BS_INT));
    }
    if (skip) continue;
    const int64_t t0 = tb + (int64_t)threadIdx.x * G;
    uint32_t mask = 0u;
    if (t0 < N) {
      const uint4 so = ldg<G>(stl, t0, N);
      const uint64_t par = lev > la ? ld_parents<D, G>(stp, t0, N) : 0ull;
      // the W marks, requested with the statuses (a group that turns out to
      // stay absent has read 16 bytes for nothing; one round trip saved)
      const uint4 wv = lev <= g.L - 1 ? ldg<G>(p.rf + g.off[lev], t0, N) : make_uint4(0u, 0u, 0u, 0u);
      // a parent that is internal after the update has all its children
      bool par_int = false;
#pragma unroll
      for (int k = 0; k < (G == 1 ? 1 : (16 >> D)); k++) par_int = par_int || ((par >> (8 * k)) & 0xff) == ST_INTERNAL;
      // nothing exists and nothing will: the group stays absent
      if (any16(so, 0xffffffffu) || par_int) {
        uint64_t nlo = 0ull, nhi = 0ull;  // new statuses of cells 0-7, 8-15
        if (G == 16 && t0 + 16 <= N) {
          // four cells per 32-bit word (statuses 0, 1, 2 and the W bit add
          // without carries): existing / created cells are 1, plus 1 where W
          const bool keep = inst_of_window_skip(g, t0, D * lev);  // the group is one instance
          const uint32_t ow[4] = {so.x, so.y, so.z, so.w}, ww[4] = {wv.x, wv.y, wv.z, wv.w};
          uint32_t nv[4], clr = 0u;
#pragma unroll
          for (int q = 0; q < 4; q++) {
            const uint32_t o = ow[q], onz = (o | (o >> 1)) & 0x01010101u;
            uint32_t base;
            if (lev == la) {
              base = onz;
            } else {
              // children 4q..4q+3 of parents (4q) >> D .. (4q + 3) >> D
              const uint32_t pa = (uint32_t)(par >> (8 * ((4 * q) >> D))) & 0xffu;
              if (D == 1) {
                const uint32_t pb = (uint32_t)(par >> (8 * (2 * q + 1))) & 0xffu;
                base = (pa == ST_INTERNAL ? 0x00000101u : 0u) | (pb == ST_INTERNAL ? 0x01010000u : 0u);
              } else {
                base = pa == ST_INTERNAL ? 0x01010101u : 0u;
              }
            }
            const uint32_t nw = keep ? o : base + (base & (ww[q] >> 1) & 0x01010101u);
            nv[q] = nw;
            const uint32_t nnz = (nw | (nw >> 1)) & 0x01010101u;
            if (lev > la) mask |= gcodes::word_bits<1>(nnz & ~onz) << (4 * q);
            clr |= gcodes::word_bits<1>((nw >> 1) & ~(o >> 1) & 0x01010101u) << (4 * q);
          }
          // a node that turns internal has no significance of its own yet
          while (clr) {
            const int j = __builtin_ctz(clr);
            clr &= clr - 1u;
            p.sigt[g.off[lev] + t0 + j] = 0;
          }
          nlo = (uint64_t)nv[0] | ((uint64_t)nv[1] << 32);
          nhi = (uint64_t)nv[2] | ((uint64_t)nv[3] << 32);
        } else {
#pragma unroll
        for (int j = 0; j < G; j++) {
          const int64_t t = t0 + j;
          const uint8_t old = byte_of(so, j);
          uint8_t nw = old;
          if (t < N && !inst_of_window_skip(g, t, D * lev)) {
            const bool w = (byte_of(wv, j) & RF_W) != 0;
            if (lev == la) {
              nw = old == ST_ABSENT ? ST_ABSENT : (w ? ST_INTERNAL : ST_LEAF);
            } else {
              const uint8_t ps = (uint8_t)(par >> (8 * (G == 1 ? 0 : (j >> D))));
              nw = ps == ST_INTERNAL ? ((lev <= g.L - 1 && w) ? ST_INTERNAL : ST_LEAF) : ST_ABSENT;
            }
            if (lev > la && old == ST_ABSENT && nw != ST_ABSENT) mask |= 1u << j;
            // a node that turns internal has no significance of its own yet
            if (nw == ST_INTERNAL && old != ST_INTERNAL) p.sigt[g.off[lev] + t] = 0;
          }
          if (j < 8) nlo |= (uint64_t)nw << (8 * j);
          else nhi |= (uint64_t)nw << (8 * (j - 8));
        }
        }
        if (G == 1) {
          stl[t0] = (uint8_t)nlo;
        } else if (t0 + 16 <= N) {
          *reinterpret_cast<uint4*>(stl + t0) =
              make_uint4((uint32_t)nlo, (uint32_t)(nlo >> 32), (uint32_t)nhi, (uint32_t)(nhi >> 32));
        } else {
          for (int j = 0; t0 + j < N; j++) stl[t0 + j] = (uint8_t)(j < 8 ? nlo >> (8 * j) : nhi >> (8 * (j - 8)));
        }
        const unsigned bits = group_summary(nlo) | group_summary(nhi);
        if (bits) atomicOr(&bor, bits);
      }
    }
    // work items: G = 16, one per sibling group with new cells (one parent
    // stencil feeds all its new children; the child mask rides in bits
    // 16-23); G = 1, one per new cell
    int cnt;
    if (G == 16) {
      constexpr uint32_t CM = (1u << (1 << D)) - 1u;
      uint32_t gmask = 0u;
#pragma unroll
      for (int gi = 0; gi < (16 >> D); gi++)
        if ((mask >> (gi << D)) & CM) gmask |= 1u << gi;
      cnt = 0;
      if (__syncthreads_or(gmask != 0u)) {
        int k = block_exscan<int>(__popc(gmask), sh, &cnt);
        while (gmask) {
          const int gi = __builtin_ctz(gmask);
          gmask &= gmask - 1u;
          items[k++] = ((int)threadIdx.x * 16 + (gi << D)) | (int)(((mask >> (gi << D)) & CM) << 16);
        }
        __syncthreads();
      }
    } else {
      cnt = block_items<G>(mask, items, sh);
    }
    // G = 16 blocks are the summary blocks; G = 1 levels keep no summary
    if (threadIdx.x == 0) {
      if (G == 16) p.bsum[g.bs_off[lev] + sb] = (uint8_t)bor;
      if (bor & BS_EXIST) atomicOr(&p.lflag[lev], LF_NEW);
      bor = 0u;
    }
    for (int i = threadIdx.x; i < cnt; i += TPB) {
      const int it = items[i];
      const int64_t t = tb + (it & 0xffff);  // G = 16: first child of the group
      const uint32_t cbits = G == 16 ? (uint32_t)(it >> 16) : 1u << (int)(t & ((1 << D) - 1));
      const int64_t inst = t >> (D * lev);
      int x[3];
      mdec<D>((uint64_t)(t & (nl - 1)), x);
      const int px[3] = {x[0] >> 1, x[1] >> 1, x[2] >> 1};
      const int64_t ibp = g.off[lev - 1] + inst * g.n[lev - 1];
      const int64_t c0 = g.off[lev] + (t & ~(int64_t)((1 << D) - 1));  // child 0 of the group
      for (int k = 0; k < g.m; k++) {
        double S[27], T[8];
        if (!gather27<D>(g, p, p.q[SL_Q0], lev - 1, ibp, px, k, S)) flag_bad(p, inst, 32);
        pred_terms<D>(S, T);
#pragma unroll
        for (int cb = 0; cb < (1 << D); cb++)
          if ((cbits >> cb) & 1u) p.q[SL_Q0][(int64_t)k * g.Ntot + c0 + cb] = pred_child<D>(T, cb);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// ordered compaction of the per-level lists of levels lo..L: leaves,
// internal nodes, interface leaves (below L, with an internal face
// neighbour) and virtual cells (absent cells that a leaf stencil reads at
// offsets 1 and 2 along an axis; their parent is then a leaf by grading:
// the virtual leaves of Fig. 1).  Per-block counts, an exclusive scan per
// level, then each block writes its cells at their rank (list order =
// Morton order within an instance).  On levels with >= 4096 cells a lane
// classifies a 16-cell Morton group (extent 16, 4x4 or 4x2x2) from the
// group and its 2d face-adjacent groups, one 16-byte load each; on smaller
// levels a lane takes one cell.

__device__ __forceinline__ int comp_level(const Geo& g, int lo, int64_t b) {
  int lev = lo;
  while (lev < g.L && b >= g.comp_first[lev + 1]) lev++;
  return lev;
}

// list k of the packed counts (16 bits each) and codes (4 bits per cell)
static constexpr int NCL = 4;
__device__ __forceinline__ constexpr int clist(int k) {
  return k == 0 ? LS_LEAF : (k == 1 ? LS_INTERNAL : (k == 2 ? LS_IFACE : LS_GHOST));
}
__device__ __forceinline__ uint64_t code_count(uint32_t c) {
  return (uint64_t)(c & 1u) | ((uint64_t)((c >> 1) & 1u) << 16) | ((uint64_t)((c >> 2) & 1u) << 32) |
         ((uint64_t)((c >> 3) & 1u) << 48);
}

// one cell, direct loads
template <int D>
__device__ __forceinline__ uint32_t cell_code(const Geo& g, const Dev& p, int lev, int64_t t) {
  const int64_t nl = g.n[lev];
  const uint8_t st = p.st[g.off[lev] + t];
  if (st == ST_INTERNAL) return CODE_INT;
  const bool leaf = st == ST_LEAF;
  if (!leaf && (lev == g.l0 || p.st[g.off[lev - 1] + (t >> D)] != ST_LEAF)) return 0u;
  const int n = 1 << lev;
  const int64_t ib = g.off[lev] + (t >> (D * lev)) * nl;
  int x[3];
  mdec<D>((uint64_t)(t & (nl - 1)), x);
  bool hit = false;
  uint32_t faces = 0u;
#pragma unroll
  for (int dir = 0; dir < D; dir++)
#pragma unroll
    for (int o = -2; o <= 2; o++) {
      if (o == 0 || (leaf && stencil_reach(g) == 1 && (o == -2 || o == 2))) continue;
      const int u = map_nb(x[dir] + o, n, g.periodic[dir]);
      if (u < 0) continue;
      int y[3] = {x[0], x[1], x[2]};
      y[dir] = u;
      const uint8_t sy = p.st[ib + (int64_t)menc<D>(y)];
      hit = hit || sy == (leaf ? ST_INTERNAL : ST_LEAF);
      if (D <= 2 && leaf && (o == -1 || o == 1) && sy == ST_ABSENT) faces |= CODE_FACE0 << (2 * dir + (o > 0));
    }
  if (leaf) return CODE_LEAF | (hit ? CODE_IFACE : 0u) | faces;
  return hit ? CODE_GHOST : 0u;
}

// codes of the 16 cells of the Morton group at t0 (one byte per cell in
// out[4]) and their packed list counts: the group, its parents and its 2d
// face-adjacent groups are loaded together (one memory round trip), then
// classified bit-parallel (group_codes.h)
template <int D>
__device__ __forceinline__ uint64_t group_codes(const Geo& g, const Dev& p, int lev, int64_t t0, uint32_t* out) {
  constexpr int W[3] = {gcodes::width<D>(0), gcodes::width<D>(1), gcodes::width<D>(2)};
  const int64_t nl = g.n[lev];
  const uint8_t* stl = p.st + g.off[lev];
  const uint4 c = *reinterpret_cast<const uint4*>(stl + t0);
  const uint64_t par = lev > g.l0 ? ld_parents<D>(p.st + g.off[lev - 1], t0, g.B * nl) : 0ull;
  const int n = 1 << lev;
  const int64_t ib = g.off[lev] + (t0 >> (D * lev)) * nl;
  int x0[3];
  mdec<D>((uint64_t)(t0 & (nl - 1)), x0);
  uint32_t m[3][4], q[3][4];
  uint32_t outside = 0u;
#pragma unroll
  for (int a = 0; a < 3; a++) {
#pragma unroll
    for (int s = 0; s < 2; s++) {
      uint4 v = make_uint4(0u, 0u, 0u, 0u);  // outside the domain: no status
      if (a < D) {
        const int u = map_nb(x0[a] + (s ? W[a] : -W[a]), n, g.periodic[a]);
        if (u >= 0) {
          int y[3] = {x0[0], x0[1], x0[2]};
          y[a] = u;
          v = *reinterpret_cast<const uint4*>(p.st + ib + (int64_t)menc<D>(y));
        } else {
          outside |= 1u << (2 * a + s);
        }
      }
      uint32_t* w = s ? q[a] : m[a];
      w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
    }
  }
  const uint32_t cw[4] = {c.x, c.y, c.z, c.w};
  return gcodes::codes16<D>(cw, m, q, outside, par, stencil_reach(g), out);
}

// per-lane cell range of block b: [t0, t0 + cpt)
struct CompRange {
  int lev, cpt;
  int64_t t0, tb;  // first cell of the lane, of the block
  bool act;
};
__device__ __forceinline__ CompRange comp_range(const Geo& g, int lo, int64_t b) {
  CompRange r;
  r.lev = comp_level(g, lo, b);
  const int chunk = g.comp_chunk[r.lev];
  r.cpt = chunk > TPB ? chunk / TPB : 1;
  r.tb = (b - g.comp_first[r.lev]) * (int64_t)chunk;
  r.t0 = r.tb + (int64_t)threadIdx.x * r.cpt;
  r.act = (int)threadIdx.x * r.cpt < chunk;
  return r;
}

// a block with no existing cell whose parents hold no leaf has nothing to
// list (virtual cells are children of leaves); decided from the summaries
// a block lists nothing when no cell of it exists and no leaf of its level
// lies in it or in an adjacent 4096-cell tile (a virtual cell is within two
// cells of a leaf of its level); 4096-cell blocks of a level are tiles of
// 4096, 64x64 or 16x16x16 cells in Morton order
template <int D>
__device__ __forceinline__ bool comp_skip(const Geo& g, const Dev& p, const CompRange& r) {
  if (!wide_level(g, r.lev)) return false;
  const int64_t sb = r.tb >> BS_SHIFT;
  const uint8_t* bs = p.bsum + g.bs_off[r.lev];
  if (bs[sb] & BS_EXIST) return false;
  const int64_t tpi = g.n[r.lev] >> BS_SHIFT;  // tiles per instance
  const int64_t i0 = sb - (sb & (tpi - 1));
  const int nt = D == 1 ? (int)tpi : (D == 2 ? (1 << (r.lev - 6)) : (1 << (r.lev - 4)));
  int x[3];
  mdec<D>((uint64_t)(sb & (tpi - 1)), x);
  bool leaf = false;
#pragma unroll
  for (int o = 0; o < (D == 1 ? 3 : (D == 2 ? 9 : 27)); o++) {
    const int ox = o % 3 - 1, oy = D > 1 ? (o / 3) % 3 - 1 : 0, oz = D > 2 ? o / 9 - 1 : 0;
    int y[3] = {map_nb(x[0] + ox, nt, g.periodic[0]), 0, 0};
    if (D > 1) y[1] = map_nb(x[1] + oy, nt, g.periodic[1]);
    if (D > 2) y[2] = map_nb(x[2] + oz, nt, g.periodic[2]);
    if (y[0] < 0 || y[1] < 0 || y[2] < 0) continue;
    leaf = leaf || (bs[i0 + (int64_t)menc<D>(y)] & BS_LEAF);
  }
  return !leaf;
}

// packed counts of the lane's cells; out[] gets their code bytes (16 for a
// group, else the one cell's in out[0])
template <int D>
__device__ __forceinline__ uint64_t lane_counts(const Geo& g, const Dev& p, const CompRange& r, uint32_t* out) {
  out[0] = out[1] = out[2] = out[3] = 0u;
  if (!r.act) return 0ull;
  if (r.cpt == GRP) return group_codes<D>(g, p, r.lev, r.t0, out);
  const uint32_t cd = cell_code<D>(g, p, r.lev, r.t0);
  out[0] = cd;
  return code_count(cd);
}

// a level with no cell after this remesh's apply pass lists nothing (not in
// full mode, where the flags are not trusted)
__device__ __forceinline__ bool level_empty(const Dev& p, int lev, int full) {
  return !full && !(p.lflag[lev] & LF_NEW);
}

// full: statuses changed outside the remesh, the summaries are not trusted.
// Compaction blocks are taken grid-stride, so an empty level costs a loop
// step per block, not a workgroup.
template <int D>
__global__ __launch_bounds__(TPB) void k_comp_count(Geo g, Dev p, int lo, int full) {
  __shared__ uint64_t sh[TPB / 64];
  __shared__ unsigned long long s_work;
  const int64_t nbt = g.comp_first[g.L + 1];
  // the workgroup's next 64 blocks are tested for work by the 64 lanes of
  // its first wave at once (empty level, or nothing to list), then only the
  // blocks with work are visited
  for (int64_t b0 = g.comp_first[lo] + blockIdx.x; b0 < nbt; b0 += 64 * (int64_t)gridDim.x) {
    if (threadIdx.x < 64) {
      const int64_t bj = b0 + (int64_t)threadIdx.x * gridDim.x;
      bool work = false;
      if (bj < nbt) {
        const CompRange rj = comp_range(g, lo, bj);
        if (!level_empty(p, rj.lev, full)) {
          if (!full && comp_skip<D>(g, p, rj)) {
#pragma unroll
            for (int k = 0; k < NCL; k++) p.bcnt[clist(k) * nbt + bj] = 0;
          } else {
            work = true;
          }
        }
      }
      const unsigned long long wm = __ballot(work);
      if (threadIdx.x == 0) s_work = wm;
    }
    __syncthreads();
    unsigned long long wm = s_work;
    __syncthreads();  // s_work is rewritten by the next group of blocks
    while (wm) {
      const int jb = __builtin_ctzll(wm);
      wm &= wm - 1ull;
      const int64_t b = b0 + (int64_t)jb * gridDim.x;
      const CompRange r = comp_range(g, lo, b);
      uint32_t cb[4];
      uint64_t tot;
      block_exscan<uint64_t>(lane_counts<D>(g, p, r, cb), sh, &tot);
      // the codes, one byte per cell, for the write pass
      if (r.act) {
        uint8_t* cc = p.ccode + g.off[r.lev] + r.t0;
        if (r.cpt == GRP) *reinterpret_cast<uint4*>(cc) = make_uint4(cb[0], cb[1], cb[2], cb[3]);
        else cc[0] = (uint8_t)cb[0];
      }
      if (threadIdx.x == 0) {
        const int64_t nsbt = g.sb_first[g.L + 1];
        const int64_t sbi = g.sb_first[r.lev] + ((b - g.comp_first[r.lev]) >> g.sb_shift[r.lev]);
  #pragma unroll
        for (int k = 0; k < NCL; k++) {
          const int cnt = (int)((tot >> (16 * k)) & 0xffffull);
          p.bcnt[clist(k) * nbt + b] = cnt;
          if (cnt) atomicAdd(&p.sbcnt[clist(k) * nsbt + sbi], cnt);
        }
      }
    }
  }
}

// one workgroup per level: exclusive scans of the superblock sums of the
// four lists (which it clears for the next compaction), the list lengths,
// the level flags and the leaves per instance
__global__ __launch_bounds__(TPB) void k_comp_scan(Geo g, Dev p, int lo, int full) {
  __shared__ int4 sh[TPB / 64];
  const int lev = lo + blockIdx.x;
  if (level_empty(p, lev, full)) {
    for (int inst = threadIdx.x; inst < g.B; inst += TPB) p.leafcnt[inst * (MRD_MAXLEV + 1) + lev] = 0;
    if (threadIdx.x == 0) {
#pragma unroll
      for (int k = 0; k < NCL; k++) p.lcnt[clist(k) * (MRD_MAXLEV + 1) + lev] = 0;
      p.lflag[lev] &= ~(LF_EXIST | LF_LEAF | LF_INT);
    }
    return;
  }
  const int64_t nsbt = g.sb_first[g.L + 1];
  const int64_t s0 = g.sb_first[lev];
  const int ns = (int)(g.sb_first[lev + 1] - s0);
  const int spi = (int)((g.n[lev] / g.comp_chunk[lev]) >> g.sb_shift[lev]);  // superblocks per instance
  int* sc[NCL];
  int* so[NCL];
#pragma unroll
  for (int k = 0; k < NCL; k++) {
    sc[k] = p.sbcnt + clist(k) * nsbt + s0;
    so[k] = p.sboff + clist(k) * nsbt + s0;
  }
  const int tid = threadIdx.x;
  const int per = (ns + TPB - 1) / TPB;
  const int j0 = tid * per;
  const int j1 = j0 + per < ns ? j0 + per : ns;
  // pass 1: the thread's sums; pass 2: its offsets (and the sums cleared)
  int4 loc = make_int4(0, 0, 0, 0);
  for (int j = j0; j < j1; j++) {
    loc.x += sc[0][j]; loc.y += sc[1][j]; loc.z += sc[2][j]; loc.w += sc[3][j];
  }
  int4 tot;
  const int lane = tid & 63, wv = tid >> 6;
  int4 x = loc;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int ux = __shfl_up(x.x, (unsigned)o, 64), uy = __shfl_up(x.y, (unsigned)o, 64);
    const int uz = __shfl_up(x.z, (unsigned)o, 64), uw = __shfl_up(x.w, (unsigned)o, 64);
    if (lane >= o) { x.x += ux; x.y += uy; x.z += uz; x.w += uw; }
  }
  if (lane == 63) sh[wv] = x;
  __syncthreads();
  int4 run = make_int4(x.x - loc.x, x.y - loc.y, x.z - loc.z, x.w - loc.w);
  tot = make_int4(0, 0, 0, 0);
#pragma unroll
  for (int w = 0; w < TPB / 64; w++) {
    const int4 s = sh[w];
    if (w < wv) { run.x += s.x; run.y += s.y; run.z += s.z; run.w += s.w; }
    tot.x += s.x; tot.y += s.y; tot.z += s.z; tot.w += s.w;
  }
  for (int j = j0; j < j1; j++) {
    const int4 v = make_int4(sc[0][j], sc[1][j], sc[2][j], sc[3][j]);
    so[0][j] = run.x; so[1][j] = run.y; so[2][j] = run.z; so[3][j] = run.w;
    sc[0][j] = 0; sc[1][j] = 0; sc[2][j] = 0; sc[3][j] = 0;
    run.x += v.x; run.y += v.y; run.z += v.z; run.w += v.w;
  }
  if (tid == 0) {
    p.lcnt[clist(0) * (MRD_MAXLEV + 1) + lev] = tot.x;
    p.lcnt[clist(1) * (MRD_MAXLEV + 1) + lev] = tot.y;
    p.lcnt[clist(2) * (MRD_MAXLEV + 1) + lev] = tot.z;
    p.lcnt[clist(3) * (MRD_MAXLEV + 1) + lev] = tot.w;
    unsigned f = p.lflag[lev] & ~(LF_EXIST | LF_LEAF | LF_INT);
    if (tot.x) f |= LF_EXIST | LF_LEAF;
    if (tot.y) f |= LF_EXIST | LF_INT;
    p.lflag[lev] = f;
  }
  __syncthreads();  // the offsets of every thread are written
  for (int inst = tid; inst < g.B; inst += TPB) {
    const int s = so[0][(int64_t)inst * spi];
    const int e = inst + 1 < g.B ? so[0][(int64_t)(inst + 1) * spi] : tot.x;
    p.leafcnt[inst * (MRD_MAXLEV + 1) + lev] = e - s;
  }
}

template <int D>
__global__ __launch_bounds__(TPB) void k_comp_write(Geo g, Dev p, int lo, int full) {
  __shared__ uint64_t sh[TPB / 64];
  __shared__ int4 s_pre;
  __shared__ int s_ent[TPB * GRP];  // one list's entries of the block, in order
  __shared__ unsigned long long s_work;
  const int64_t nbt = g.comp_first[g.L + 1];
  // as in the count pass: the next 64 blocks are tested at once (empty
  // level, or nothing listed: the count pass left the block's counts)
  for (int64_t b0 = g.comp_first[lo] + blockIdx.x; b0 < nbt; b0 += 64 * (int64_t)gridDim.x) {
    if (threadIdx.x < 64) {
      const int64_t bj = b0 + (int64_t)threadIdx.x * gridDim.x;
      bool work = false;
      if (bj < nbt) {
        const CompRange rj = comp_range(g, lo, bj);
        if (!level_empty(p, rj.lev, full)) {
          const int n0 = p.bcnt[clist(0) * nbt + bj], n1 = p.bcnt[clist(1) * nbt + bj];
          const int n2 = p.bcnt[clist(2) * nbt + bj], n3 = p.bcnt[clist(3) * nbt + bj];
          if ((n0 | n1 | n2 | n3) == 0) {
            if (wide_level(g, rj.lev)) p.bsum[g.bs_off[rj.lev] + (rj.tb >> BS_SHIFT)] = 0;
          } else {
            work = true;
          }
        }
      }
      const unsigned long long wm = __ballot(work);
      if (threadIdx.x == 0) s_work = wm;
    }
    __syncthreads();
    unsigned long long wm = s_work;
    __syncthreads();  // s_work is rewritten by the next group of blocks
    while (wm) {
      const int jb = __builtin_ctzll(wm);
      wm &= wm - 1ull;
      const int64_t b = b0 + (int64_t)jb * gridDim.x;
      const CompRange r = comp_range(g, lo, b);
      // the lane's cells of each list as a mask (bit j: cell t0 + j)
      uint32_t mk[NCL] = {0u, 0u, 0u, 0u};
      if (r.act) {
        const uint8_t* cc = p.ccode + g.off[r.lev] + r.t0;
        if (r.cpt == GRP) {
          const uint4 v = *reinterpret_cast<const uint4*>(cc);
          const uint32_t w[4] = {v.x, v.y, v.z, v.w};
  #pragma unroll
          for (int k = 0; k < NCL; k++)
  #pragma unroll
            for (int q = 0; q < 4; q++) mk[k] |= gcodes::word_bits<1>((w[q] >> k) & 0x01010101u) << (4 * q);
        } else {
  #pragma unroll
          for (int k = 0; k < NCL; k++) mk[k] = ((uint32_t)cc[0] >> k) & 1u;
        }
      }
      uint64_t c = 0ull, tot;
  #pragma unroll
      for (int k = 0; k < NCL; k++) c |= (uint64_t)__popc(mk[k]) << (16 * k);
      const uint64_t ex = block_exscan<uint64_t>(c, sh, &tot);
      // list offsets of the block: its superblock's plus the counts of the
      // preceding blocks of the superblock (fewer than 64: wave 0 sums them)
      int4 pre = make_int4(0, 0, 0, 0);
      if (tot != 0ull) {
        const int64_t bl = b - g.comp_first[r.lev];
        const int sh2 = g.sb_shift[r.lev];
        const int64_t bs = g.comp_first[r.lev] + ((bl >> sh2) << sh2);
        const int nprev = (int)(b - bs);
        if (threadIdx.x < 64) {
          int4 v = make_int4(0, 0, 0, 0);
          if ((int)threadIdx.x < nprev) {
            const int64_t j = bs + threadIdx.x;
            v = make_int4(p.bcnt[clist(0) * nbt + j], p.bcnt[clist(1) * nbt + j], p.bcnt[clist(2) * nbt + j],
                          p.bcnt[clist(3) * nbt + j]);
          }
  #pragma unroll
          for (int o = 32; o > 0; o >>= 1) {
            v.x += __shfl_xor(v.x, o, 64); v.y += __shfl_xor(v.y, o, 64);
            v.z += __shfl_xor(v.z, o, 64); v.w += __shfl_xor(v.w, o, 64);
          }
          if (threadIdx.x == 0) s_pre = v;
        }
        __syncthreads();
        pre = s_pre;
        const int64_t sbi = g.sb_first[r.lev] + (bl >> sh2);
        const int64_t nsbt = g.sb_first[g.L + 1];
        pre.x += p.sboff[clist(0) * nsbt + sbi]; pre.y += p.sboff[clist(1) * nsbt + sbi];
        pre.z += p.sboff[clist(2) * nsbt + sbi]; pre.w += p.sboff[clist(3) * nsbt + sbi];
        __syncthreads();  // s_pre is free again
      }
      // block summary of a 4096-cell block (levels with >= 4096 cells)
      if (threadIdx.x == 0 && wide_level(g, r.lev)) {
        unsigned bits = 0u;
        if (tot & 0xffffull) bits |= BS_EXIST | BS_LEAF;
        if ((tot >> 16) & 0xffffull) bits |= BS_EXIST | BS_INT;
        p.bsum[g.bs_off[r.lev] + (r.tb >> BS_SHIFT)] = (uint8_t)bits;
      }
      // each list's entries of the block are one contiguous range of the
      // list: staged in order in shared memory, then stored with consecutive
      // lanes on consecutive entries
      const int base[NCL] = {pre.x, pre.y, pre.z, pre.w};
      const int64_t o = g.off[r.lev];
  #pragma unroll
      for (int k = 0; k < NCL; k++) {
        const int tk = (int)((tot >> (16 * k)) & 0xffffull);
        if (tk == 0) continue;  // the same in every lane
        int pos = (int)((ex >> (16 * k)) & 0xffffull);
        uint32_t m = mk[k];
        while (m) {
          const int j = __builtin_ctz(m);
          m &= m - 1u;
          s_ent[pos++] = (int)(r.t0 + j);
        }
        __syncthreads();
        int* dst = p.lst[clist(k)] + o + base[k];
        for (int i = threadIdx.x; i < tk; i += TPB) dst[i] = s_ent[i];
        __syncthreads();
      }
    }
  }
}

// per 4096-cell tile of the wide levels lo..L: 1 when an internal node lies
// in the tile or in one of its 3^d neighbours (periodic wrap at tile level),
// i.e. when leaves of the tile may feed the virtual cells of the next level
template <int D>
__global__ __launch_bounds__(TPB) void k_nerk_tiles(Geo g, Dev p, int lo) {
  GSL(j, g.bs_off[g.L + 1] - g.bs_off[lo]) {
    const int64_t jj = g.bs_off[lo] + j;
    int lev = lo;
    while (jj >= g.bs_off[lev + 1]) lev++;
    if (!wide_level(g, lev)) continue;
    const int64_t sb = jj - g.bs_off[lev];
    const uint8_t* bs = p.bsum + g.bs_off[lev];
    const int64_t tpi = g.n[lev] >> BS_SHIFT;  // tiles per instance
    const int64_t i0 = sb - (sb & (tpi - 1));
    const int nt = D == 1 ? (int)tpi : (D == 2 ? (1 << (lev - 6)) : (1 << (lev - 4)));
    int x[3];
    mdec<D>((uint64_t)(sb & (tpi - 1)), x);
    bool in = false;
#pragma unroll
    for (int o = 0; o < (D == 1 ? 3 : (D == 2 ? 9 : 27)); o++) {
      const int ox = o % 3 - 1, oy = D > 1 ? (o / 3) % 3 - 1 : 0, oz = D > 2 ? o / 9 - 1 : 0;
      int y[3] = {map_nb(x[0] + ox, nt, g.periodic[0]), 0, 0};
      if (D > 1) y[1] = map_nb(x[1] + oy, nt, g.periodic[1]);
      if (D > 2) y[2] = map_nb(x[2] + oz, nt, g.periodic[2]);
      if (y[0] < 0 || y[1] < 0 || y[2] < 0) continue;
      in = in || (bs[i0 + (int64_t)menc<D>(y)] & BS_INT);
    }
    p.nsum[jj] = in ? 1 : 0;
  }
}

void launch_compact(const Geo& g, const Dev& p, int lo, bool full, hipStream_t s) {
  int64_t nb = g.comp_first[g.L + 1] - g.comp_first[lo];
  if (nb > g.comp_grid) nb = g.comp_grid;
  const int f = full ? 1 : 0;
  if (g.d == 1) k_comp_count<1><<<(unsigned)nb, TPB, 0, s>>>(g, p, lo, f);
  else if (g.d == 2) k_comp_count<2><<<(unsigned)nb, TPB, 0, s>>>(g, p, lo, f);
  else k_comp_count<3><<<(unsigned)nb, TPB, 0, s>>>(g, p, lo, f);
  k_comp_scan<<<(unsigned)(g.L - lo + 1), TPB, 0, s>>>(g, p, lo, f);
  if (g.d == 1) k_comp_write<1><<<(unsigned)nb, TPB, 0, s>>>(g, p, lo, f);
  else if (g.d == 2) k_comp_write<2><<<(unsigned)nb, TPB, 0, s>>>(g, p, lo, f);
  else k_comp_write<3><<<(unsigned)nb, TPB, 0, s>>>(g, p, lo, f);
  const int ntb = blocks_for(g.bs_off[g.L + 1] - g.bs_off[lo]);
  if (g.d == 1) k_nerk_tiles<1><<<ntb, TPB, 0, s>>>(g, p, lo);
  else if (g.d == 2) k_nerk_tiles<2><<<ntb, TPB, 0, s>>>(g, p, lo);
  else k_nerk_tiles<3><<<ntb, TPB, 0, s>>>(g, p, lo);
}

#define DISPATCH_D(kern, n, ...)                                                  \
  do {                                                                            \
    const int nb_ = blocks_for(n);                                                \
    if (g.d == 1) kern<1><<<nb_, TPB, 0, s>>>(__VA_ARGS__);                       \
    else if (g.d == 2) kern<2><<<nb_, TPB, 0, s>>>(__VA_ARGS__);                  \
    else kern<3><<<nb_, TPB, 0, s>>>(__VA_ARGS__);                                \
  } while (0)

void launch_load_finest(const Geo& g, const Dev& p, const double* src, int inst, int Li, hipStream_t s) {
  DISPATCH_D(k_load_finest, (inst >= 0 ? 1 : g.B) * g.n[Li], g, p, src, inst, Li);
}
void launch_recon_level(const Geo& g, const Dev& p, int lev, double* dense, hipStream_t s) {
  DISPATCH_D(k_recon_level, g.B * g.n[lev], g, p, lev, dense);
}
void launch_to_rowmajor(const Geo& g, const double* dense, double* out, hipStream_t s) {
  DISPATCH_D(k_to_rowmajor, g.B * g.n[g.L], g, dense, out);
}
void launch_level_w(const Geo& g, const Dev& p, int la, hipStream_t s) {
  k_level_w<<<1, TPB, 0, s>>>(g, p, la);
}

// remesh table and W flags cleared on levels lo..hi
void launch_remesh_clear(const Geo& g, const Dev& p, int lo, int hi, hipStream_t s) {
  if (lo > hi) return;
  int64_t nb = g.bs_off[hi + 1] - g.bs_off[lo];
  if (nb > 2048) nb = 2048;
  k_clear_w<<<(unsigned)nb, TPB, 0, s>>>(g, p, lo, hi);
}
void launch_detail_seed(const Geo& g, const Dev& p, int la, int hi, int n_it, hipStream_t s) {
  if (la > hi) return;
  const int lo = la > g.l0 ? la - 1 : la;
  DISPATCH_D(k_detail_seed, g.B * g.n[hi], g, p, lo, hi, la, n_it);
}
// dense passes: 16 cells per lane on levels with >= 2^20 cells (where the
// block summaries let whole blocks be skipped), one cell per lane below (so
// a block never hands a lane more than one work item there)
#define DISPATCH_DG(kern, lev_, ...)                                                     \
  do {                                                                                   \
    const int64_t cells_ = g.B * g.n[lev_];                                              \
    if (wide_level(g, lev_)) {                                                           \
      const int nb_ = blocks_for((cells_ + 15) >> 4);                                    \
      if (g.d == 1) kern<1, 16><<<nb_, TPB, 0, s>>>(__VA_ARGS__);                        \
      else if (g.d == 2) kern<2, 16><<<nb_, TPB, 0, s>>>(__VA_ARGS__);                   \
      else kern<3, 16><<<nb_, TPB, 0, s>>>(__VA_ARGS__);                                 \
    } else {                                                                             \
      int64_t b_ = (cells_ + TPB - 1) / TPB;                                             \
      const int nb_ = (int)(b_ > 4096 ? 4096 : b_);                                      \
      if (g.d == 1) kern<1, 1><<<nb_, TPB, 0, s>>>(__VA_ARGS__);                         \
      else if (g.d == 2) kern<2, 1><<<nb_, TPB, 0, s>>>(__VA_ARGS__);                    \
      else kern<3, 1><<<nb_, TPB, 0, s>>>(__VA_ARGS__);                                  \
    }                                                                                    \
  } while (0)
void launch_close(const Geo& g, const Dev& p, int lev, hipStream_t s) {
  DISPATCH_DG(k_close, lev + 1, g, p, lev);
}
void launch_prune(const Geo& g, const Dev& p, int lev, int la, hipStream_t s) {
  if (lev == g.l0) return;
  DISPATCH_DG(k_prune, lev, g, p, lev, la);
}
void launch_apply(const Geo& g, const Dev& p, int lev, int la, hipStream_t s) {
  DISPATCH_DG(k_apply, lev, g, p, lev, la);
}
// ---------------------------------------------------------------------------
// leaf lists of one instance and level in Morton order: wavefront ballot +
// popcount, per-block counts, an exclusive scan of the block counts, then a
// second pass that writes every leaf at its rank (order = Morton order)

__global__ __launch_bounds__(TPB) void k_count(const uint8_t* st, int64_t base, int64_t n, uint8_t want,
                                               int* blockcnt) {
  __shared__ int wsum[TPB / 64];
  const int64_t t = (int64_t)blockIdx.x * TPB + threadIdx.x;
  const bool hit = t < n && st[base + t] == want;
  const unsigned long long bal = __ballot(hit);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = __popcll(bal);
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int w = 0; w < TPB / 64; w++) s += wsum[w];
    blockcnt[blockIdx.x] = s;
  }
}

void launch_count(const Geo& g, const Dev& p, int lev, int inst, uint8_t want, int* blockcnt, int nblk,
                  hipStream_t s) {
  const int64_t base = g.off[lev] + (int64_t)inst * g.n[lev];
  k_count<<<nblk, TPB, 0, s>>>(p.st, base, g.n[lev], want, blockcnt);
}

__global__ void k_scan_blocks(int* cnt, int n, long long* total) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  long long s = 0;
  for (int i = 0; i < n; i++) {
    const int c = cnt[i];
    cnt[i] = (int)s;
    s += c;
  }
  *total = s;
}

void launch_scan_blocks(int* blockcnt, int nblk, long long* total, hipStream_t s) {
  k_scan_blocks<<<1, 64, 0, s>>>(blockcnt, nblk, total);
}

__global__ __launch_bounds__(TPB) void k_gather_leaves(Geo g, Dev p, int lev, int64_t base, int64_t n,
                                                       const int* blockoff, long long out0,
                                                       unsigned long long* keys, double* vals,
                                                       long long vstride) {
  __shared__ int wsum[TPB / 64];
  const int64_t t = (int64_t)blockIdx.x * TPB + threadIdx.x;
  const bool hit = t < n && p.st[base + t] == ST_LEAF;
  const unsigned long long bal = __ballot(hit);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) wsum[wv] = __popcll(bal);
  __syncthreads();
  if (!hit) return;
  int off = blockoff[blockIdx.x];
  for (int w = 0; w < wv; w++) off += wsum[w];
  off += __popcll(bal & ((1ull << lane) - 1ull));
  const long long o = out0 + off;
  keys[o] = ((unsigned long long)lev << 56) | (unsigned long long)t;
  for (int k = 0; k < g.m; k++) vals[(long long)k * vstride + o] = p.q[SL_Q0][(int64_t)k * g.Ntot + base + t];
}

void launch_gather_leaves(const Geo& g, const Dev& p, int lev, int inst, const int* blockoff, int nblk,
                          long long base_out, unsigned long long* keys, double* vals, long long vstride,
                          hipStream_t s) {
  const int64_t base = g.off[lev] + (int64_t)inst * g.n[lev];
  k_gather_leaves<<<nblk, TPB, 0, s>>>(g, p, lev, base, g.n[lev], blockoff, base_out, keys, vals, vstride);
}

__global__ void k_scatter_leaves(Geo g, Dev p, int64_t inst, const unsigned long long* keys,
                                 const double* vals, long long n, int* err) {
  GSL(r, n) {
    const unsigned long long key = keys[r];
    const int lev = (int)(key >> 56);
    const unsigned long long mk = key & ((1ull << 56) - 1ull);
    if (lev < g.l0 || lev > g.L || (mk >> (g.d * lev)) != 0) {
      atomicOr(err, 1);
      continue;
    }
    const int64_t G = g.off[lev] + inst * g.n[lev] + (int64_t)mk;
    p.st[G] = ST_LEAF;
    for (int k = 0; k < g.m; k++) p.q[SL_Q0][(int64_t)k * g.Ntot + G] = vals[(long long)k * n + r];
  }
}

void launch_scatter_leaves(const Geo& g, const Dev& p, int inst, const unsigned long long* keys,
                           const double* vals, long long n, int* err, hipStream_t s) {
  if (n <= 0) return;
  k_scatter_leaves<<<blocks_for(n), TPB, 0, s>>>(g, p, inst, keys, vals, n, err);
}

__global__ void k_mark_parents(Geo g, Dev p, int lev, int* err) {
  const int64_t N = g.B * g.n[lev];
  GSL(t, N) {
    if (p.st[g.off[lev] + t] == ST_ABSENT) continue;
    const int64_t P = g.off[lev - 1] + (t >> g.d);
    if (p.st[P] == ST_LEAF) atomicOr(err, 2);
    p.st[P] = ST_INTERNAL;
  }
}

void launch_mark_parents(const Geo& g, const Dev& p, int lev, int* err, hipStream_t s) {
  k_mark_parents<<<blocks_for(g.B * g.n[lev]), TPB, 0, s>>>(g, p, lev, err);
}

template <int D>
__global__ void k_validate(Geo g, Dev p, int lev, int* err) {
  const int64_t nl = g.n[lev], N = g.B * nl;
  const int n = 1 << lev;
  GSL(t, N) {
    const int64_t G = g.off[lev] + t;
    const uint8_t s = p.st[G];
    if (lev == g.l0 && s == ST_ABSENT) atomicOr(err, 4);
    if (s != ST_INTERNAL) continue;
    if (lev == g.L) {
      atomicOr(err, 32);
      continue;
    }
    const int64_t C0 = g.off[lev + 1] + (t << D);
    for (int cb = 0; cb < (1 << D); cb++)
      if (p.st[C0 + cb] == ST_ABSENT) atomicOr(err, 8);
    const int64_t inst = t >> (D * lev);
    const int64_t ib = g.off[lev] + inst * nl;
    int x[3];
    mdec<D>((uint64_t)(t & (nl - 1)), x);
    for (int oz = (D > 2 ? -2 : 0); oz <= (D > 2 ? 2 : 0); oz++)
      for (int oy = (D > 1 ? -2 : 0); oy <= (D > 1 ? 2 : 0); oy++)
        for (int ox = -2; ox <= 2; ox++) {
          int y[3] = {map_nb(x[0] + ox, n, g.periodic[0]), 0, 0};
          if (D > 1) y[1] = map_nb(x[1] + oy, n, g.periodic[1]);
          if (D > 2) y[2] = map_nb(x[2] + oz, n, g.periodic[2]);
          if (y[0] < 0 || y[1] < 0 || y[2] < 0) continue;
          if (p.st[ib + (int64_t)menc<D>(y)] == ST_ABSENT) atomicOr(err, 16);
        }
  }
}

void launch_validate(const Geo& g, const Dev& p, int lev, int* err, hipStream_t s) {
  DISPATCH_D(k_validate, g.B * g.n[lev], g, p, lev, err);
}

// ---------------------------------------------------------------------------
// reductions: maximum wave speed per instance (monotone bit pattern of a
// non-negative double, integer atomicMax), leaf mass partial sums per block

template <int D>
__global__ void k_wavespeed(Geo g, Dev p, int lev, unsigned long long* out) {
  // the maximum is taken over each wave first (it is exact and
  // order-independent), so that one atomic per wave and instance reaches
  // memory instead of one per leaf
  const int64_t nl = g.n[lev], N = g.B * nl;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t start = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // every lane of a wave runs the same number of rounds (the wave votes)
  const int64_t rounds = (N + stride - 1) / stride;
  for (int64_t r = 0; r < rounds; r++) {
    const int64_t t = start + r * stride;
    const bool in = t < N;
    const int64_t G = g.off[lev] + (in ? t : 0);
    const bool leaf = in && p.st[G] == ST_LEAF;
    const int64_t inst = in ? t >> (D * lev) : -1;
    double q[5], v = 0.0;
    if (leaf) {
    for (int k = 0; k < g.m; k++) q[k] = p.q[SL_Q0][(int64_t)k * g.Ntot + G];
    if (g.pde == PDE_BURGERS) {
      // f_i(u) = u^2/2 in every direction: sum_i |f_i'(u)|
      for (int j = 0; j < D; j++) v = (j == 0) ? fabs(q[0]) : (v + fabs(q[0]));
    } else if (g.pde == PDE_EULER) {
      double w[5];
      euler_prim<D>(g.gamma - 1.0, q, w);
      const double a = sqrt((g.gamma * w[D + 1]) / w[0]);
      for (int j = 0; j < D; j++) v = (j == 0) ? (fabs(w[1]) + a) : (v + (fabs(w[1 + j]) + a));
    } else if (g.pde == PDE_ADVECTION) {
      for (int j = 0; j < D; j++) v = v + fabs(g.adv[j]);
    } else if (g.pde == PDE_FLAME || g.pde == PDE_FLAMEBALL) {
      if (g.flame_speed) v = fabs(p.vel[inst]);
      else
        for (int j = 0; j < D; j++) v = v + fabs(g.adv[j]);
    }
    }
    // non-negative doubles order like their bit patterns
    unsigned long long bits = leaf ? (unsigned long long)__double_as_longlong(v) : 0ull;
    const int64_t i0 = __shfl(inst, 0);
    const bool one_inst = __all(!leaf || inst == i0);
    const bool any_leaf = __any(leaf);
    if (one_inst) {
      for (int o = 32; o >= 1; o >>= 1) {
        const unsigned long long u = __shfl_xor(bits, o);
        bits = u > bits ? u : bits;
      }
      if ((threadIdx.x & 63) == 0 && any_leaf) atomicMax(&out[i0], bits);
    } else if (leaf) {
      atomicMax(&out[inst], bits);
    }
  }
}

void launch_wavespeed(const Geo& g, const Dev& p, int lev, unsigned long long* out, hipStream_t s) {
  DISPATCH_D(k_wavespeed, g.B * g.n[lev], g, p, lev, out);
}

// flame velocity v_f (Sec. 5): the reaction rate at every leaf times the leaf
// volume, summed per compaction block (blocks never straddle instances) and
// then per instance over its blocks in level and block order, divided by the
// cross-section normal to axis 0.  Fixed summation order: reproducible.
template <int PDE>
__global__ __launch_bounds__(TPB) void k_flame_part(Geo g, Dev p) {
  __shared__ double sh[TPB];
  const int64_t b = blockIdx.x;
  int lev = g.l0;
  while (lev < g.L && b >= g.comp_first[lev + 1]) lev++;
  const int64_t ch = g.comp_chunk[lev];
  const int64_t G0 = g.off[lev] + (b - g.comp_first[lev]) * ch;
  double s = 0.0;
  for (int64_t j = threadIdx.x; j < ch; j += TPB) {
    const int64_t G = G0 + j;
    if (p.st[G] != ST_LEAF) continue;
    double q[2];
    q[0] = p.q[SL_Q0][G];
    q[1] = PDE == PDE_FLAMEBALL ? p.q[SL_Q0][g.Ntot + G] : 0.0;
    s = s + (reaction_rate<PDE>(g, q) * g.vol[lev]);
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = TPB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = sh[threadIdx.x] + sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) p.vfpart[b] = sh[0];
}

__global__ __launch_bounds__(TPB) void k_flame_sum(Geo g, Dev p) {
  __shared__ double sh[TPB];
  const int64_t inst = blockIdx.x;
  int64_t tot = 0;
  for (int lev = g.l0; lev <= g.L; lev++) tot += g.n[lev] / g.comp_chunk[lev];
  double s = 0.0;
  for (int64_t j = threadIdx.x; j < tot; j += TPB) {
    int lev = g.l0;
    int64_t jj = j;
    while (jj >= g.n[lev] / g.comp_chunk[lev]) {
      jj -= g.n[lev] / g.comp_chunk[lev];
      lev++;
    }
    s = s + p.vfpart[g.comp_first[lev] + inst * (g.n[lev] / g.comp_chunk[lev]) + jj];
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = TPB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = sh[threadIdx.x] + sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double vf = sh[0] / g.flame_area;
    p.vel[g.B + inst] = vf;
    p.vel[inst] = (double)g.flame_speed * vf;
  }
}

void launch_flame_speed(const Geo& g, const Dev& p, hipStream_t s) {
  const int64_t nb = g.comp_first[g.L + 1];
  if (g.pde == PDE_FLAME) k_flame_part<PDE_FLAME><<<nb, TPB, 0, s>>>(g, p);
  else k_flame_part<PDE_FLAMEBALL><<<nb, TPB, 0, s>>>(g, p);
  k_flame_sum<<<g.B, TPB, 0, s>>>(g, p);
}

__global__ __launch_bounds__(TPB) void k_mass_partial(Geo g, Dev p, int64_t base, int64_t n, double vol,
                                                      double* part) {
  __shared__ double sh[5][TPB];
  const int64_t t = (int64_t)blockIdx.x * TPB + threadIdx.x;
  const bool leaf = t < n && p.st[base + t] == ST_LEAF;
  for (int k = 0; k < g.m; k++) sh[k][threadIdx.x] = leaf ? vol * p.q[SL_Q0][(int64_t)k * g.Ntot + base + t] : 0.0;
  __syncthreads();
  for (int w = TPB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int k = 0; k < g.m; k++) sh[k][threadIdx.x] = sh[k][threadIdx.x] + sh[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < g.m; k++) part[(int64_t)blockIdx.x * g.m + k] = sh[k][0];
}

void launch_mass_partial(const Geo& g, const Dev& p, int lev, int inst, double* part, int nblk, hipStream_t s) {
  const int64_t base = g.off[lev] + (int64_t)inst * g.n[lev];
  k_mass_partial<<<nblk, TPB, 0, s>>>(g, p, base, g.n[lev], g.vol[lev], part);
}
