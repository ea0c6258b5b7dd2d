// group_codes.h -- list codes of a 16-cell Morton group, bit-parallel.
//
// The ordered compaction classifies every cell of a level into the lists
// the kernels walk: leaves, internal nodes, interface leaves (leaves with
// an internal neighbour within the stencil reach along an axis) and
// virtual cells (absent cells whose parent is a leaf and that have a leaf
// of their own level within two cells along an axis: the virtual leaves
// that leaf stencils read, Fig. 1 and Sec. 2 of arXiv:1905.08717).
//
// A lane classifies the 16 cells of one Morton group (extent 16, 4x4 or
// 4x2x2) from the status bytes of the group, of its 2d face-adjacent groups
// and of its parents.  Here the statuses become 16-bit masks in row-major
// order of the group, neighbours are masks shifted along an axis (bits that
// leave the group come in from the adjacent group), and the codes are
// Boolean combinations of masks: a few dozen integer operations per group
// instead of a branch per cell and neighbour.
//
// Status bytes: 0 absent, 1 leaf, 2 internal; a neighbour group outside the
// domain is passed as all zeros, with its bit set in `outside`.  Codes (one
// byte per cell, Morton order): 1 leaf, 2 internal, 4 interface leaf, 8
// virtual cell; in 1D and 2D also bit 4 + 2a + s: a leaf whose face
// neighbour along axis a (s = 0 below, 1 above) is absent and inside the
// domain, i.e. the fine side of a refined face (the neighbour is a virtual
// cell whose parent is a coarser leaf).  The face bits mark no list; the
// stage kernels read them instead of the neighbours' statuses (3D has six
// faces, more than the byte holds, and its kernels read the statuses).
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define GC_HD __host__ __device__ __forceinline__
#else
#define GC_HD inline
#endif

namespace gcodes {

// extent and row-major stride of a group along axis a
template <int D>
GC_HD constexpr int width(int a) {
  return D == 1 ? (a == 0 ? 16 : 1) : (D == 2 ? (a < 2 ? 4 : 1) : (a == 0 ? 4 : 2));
}
template <int D>
GC_HD constexpr int stride(int a) {
  return a == 0 ? 1 : (a == 1 ? width<D>(0) : width<D>(0) * width<D>(1));
}
// row-major cells of the group whose coordinate along axis a is < k
template <int D>
GC_HD constexpr uint32_t below(int a, int k) {
  uint32_t m = 0u;
  for (int r = 0; r < 16; r++)
    if ((r / stride<D>(a)) % width<D>(a) < k) m |= 1u << r;
  return m;
}
// The four bytes of status word q are Morton cells 4q..4q+3; their
// row-major positions are off(q) + {0, 1, 2, 3} in 1D and
// off(q) + {0, 1, 4, 5} in 2D and 3D.  A multiply gathers bit 0 of the
// four bytes into those positions (no two partial products meet, so there
// are no carries into the result bits).
template <int D>
GC_HD constexpr int off(int q) {
  return D == 1 ? 4 * q : (D == 2 ? (q == 0 ? 0 : q == 1 ? 2 : q == 2 ? 8 : 10) : (q == 0 ? 0 : q == 1 ? 8 : q == 2 ? 2 : 10));
}
template <int D>
GC_HD uint32_t word_bits(uint32_t x) {  // x: one bit at 0, 8, 16, 24
  return D == 1 ? ((x * 0x01020408u) >> 24) & 0xFu : ((x * 0x01021020u) >> 24) & 0x33u;
}
// the inverse: Morton nibble of word q from a row-major mask
template <int D>
GC_HD uint32_t nibble(uint32_t m, int q) {
  if (D == 1) return (m >> (4 * q)) & 0xFu;
  const uint32_t t = m >> off<D>(q);
  return (t & 3u) | ((t >> 2) & 0xCu);
}
// four bits to bit 0 of four bytes
GC_HD uint32_t spread(uint32_t n) { return (n * 0x00204081u) & 0x01010101u; }

// row-major mask of the cells whose status byte has bit b (0 leaf, 1 internal)
template <int D>
GC_HD uint32_t status_mask(const uint32_t* w, int b) {
  uint32_t m = 0u;
#pragma unroll
  for (int q = 0; q < 4; q++) m |= word_bits<D>((w[q] >> b) & 0x01010101u) << off<D>(q);
  return m;
}

// cells whose neighbour at offset o (|o| <= 2) along axis a is set in the
// masks of the group (own), of the adjacent group below (lo) and above (hi)
template <int D>
GC_HD uint32_t shifted(uint32_t own, uint32_t lo, uint32_t hi, int a, int o) {
  const int w = width<D>(a), s = stride<D>(a);
  if (o > 0) {
    const uint32_t in = o < w ? ((own >> (o * s)) & below<D>(a, w - o)) : 0u;
    return in | ((hi << ((w - o) * s)) & ~below<D>(a, w - o) & 0xFFFFu);
  }
  const int k = -o;
  const uint32_t in = k < w ? ((own << (k * s)) & ~below<D>(a, k) & 0xFFFFu) : 0u;
  return in | ((lo >> ((w - k) * s)) & below<D>(a, k));
}

// row-major cells of the group under parent k (Morton order of the parents)
template <int D>
GC_HD constexpr uint32_t parent_cells(int k) {
  return D == 1 ? (3u << (2 * k)) : (D == 2 ? (0x33u << off<2>(k)) : (0x3333u << (2 * k)));
}

// c: the group's four status words; m[a], p[a]: the adjacent groups below /
// above along axis a; outside: bit 2a (2a + 1) set when m[a] (p[a]) lies
// outside the domain; par: the 16 >> D parent status bytes (0 on the
// coarsest level); reach: stencil reach of a leaf (1 or 2).  Writes the 16
// code bytes to out[4]; returns the counts of the four lists (leaf,
// internal, interface, virtual), 16 bits each.
template <int D>
GC_HD uint64_t codes16(const uint32_t* c, const uint32_t (*m)[4], const uint32_t (*p)[4], uint32_t outside,
                       uint64_t par, int reach, uint32_t* out) {
  const uint32_t Lc = status_mask<D>(c, 0), Ic = status_mask<D>(c, 1);
  uint32_t near_int = 0u, near_leaf = 0u;
  uint32_t Af[4] = {0u, 0u, 0u, 0u};  // leaves whose face neighbour (axis a, side s) is absent: Af[2a + s]
#pragma unroll
  for (int a = 0; a < D; a++) {
    const uint32_t Lm = status_mask<D>(m[a], 0), Lp = status_mask<D>(p[a], 0);
    const uint32_t Im = status_mask<D>(m[a], 1), Ip = status_mask<D>(p[a], 1);
#pragma unroll
    for (int o = -2; o <= 2; o++) {
      if (o == 0) continue;
      const uint32_t sL = shifted<D>(Lc, Lm, Lp, a, o);
      near_leaf |= sL;
      if (o == -1 || o == 1 || reach == 2) {
        const uint32_t sI = shifted<D>(Ic, Im, Ip, a, o);
        near_int |= sI;
        if (D <= 2 && (o == -1 || o == 1)) {
          // the face neighbour is a leaf, internal, or outside the domain
          // (the edge row of the group next to an outside group): else absent
          const uint32_t edge = o < 0 ? (((outside >> (2 * a)) & 1u) ? below<D>(a, 1) : 0u)
                                      : (((outside >> (2 * a + 1)) & 1u) ? (~below<D>(a, width<D>(a) - 1) & 0xFFFFu) : 0u);
          Af[(2 * a + (o > 0)) & 3] = Lc & ~(sL | sI | edge) & 0xFFFFu;
        }
      }
    }
  }
  uint32_t pleaf = 0u;
#pragma unroll
  for (int k = 0; k < (16 >> D); k++)
    if ((par >> (8 * k)) & 1ull) pleaf |= parent_cells<D>(k);
  const uint32_t F = Lc & near_int;
  const uint32_t V = ~(Lc | Ic) & 0xFFFFu & pleaf & near_leaf;
#pragma unroll
  for (int q = 0; q < 4; q++) {
    out[q] = spread(nibble<D>(Lc, q)) | (spread(nibble<D>(Ic, q)) << 1) | (spread(nibble<D>(F, q)) << 2) |
             (spread(nibble<D>(V, q)) << 3);
#pragma unroll
    for (int f = 0; f < 2 * D && D <= 2; f++) out[q] |= spread(nibble<D>(Af[f & 3], q)) << (4 + f);
  }
  return (uint64_t)__builtin_popcount(Lc) | ((uint64_t)__builtin_popcount(Ic) << 16) |
         ((uint64_t)__builtin_popcount(F) << 32) | ((uint64_t)__builtin_popcount(V) << 48);
}

}  // namespace gcodes
