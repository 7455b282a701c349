// lbm_impl.hpp -- templated kernels of the fused central-moment
// stream-and-collide step (gfx950, one node per thread, structure-of-arrays
// populations).  Included by one translation unit per lattice.
//
// Work split per step:
//   bulk nodes      every node of class CLS_BULK (no cut link, not EQ/OUTLET):
//                   pull of Q populations per lattice, velocity from f (or
//                   prescribed), central-moment collision in registers, store.
//   boundary nodes  one thread per node: pull, wall links (BB/IBB on f,
//                   ABB/IABB on h), outlet copy, EQ reset, then the same
//                   collision.
//
// Streaming layouts (LAY):
//   LAY_AB    two arrays: read the post-collision state of step t-1 from the
//             source array (g*_i at node x in slot i), pull g_i(x) =
//             g*_i(x - e_i), write g*_i(x) to slot i of node x in the other
//             array.
//   LAY_AA_S  one array, "swapped" layout: slot opp(i) of node x holds
//             g*_i(x).  The step pulls slot opp(i) of x - e_i and pushes the
//             new g*_i(x) to slot i of x + e_i, which leaves the array in ...
//   LAY_AA_N  ... the "streamed" layout: slot i of node y holds
//             g*_i(y - e_i), the pulled value of y.  The step reads its own
//             slots and writes g*_i(x) to slot opp(i) of x (back to S).
// In both AA steps every slot a thread reads is written in that step by the
// same thread only, so the in-place update has no race.  Two inputs of the
// boundary rules are the exception: the post-collision value g*_opp(i)(x_b)
// of a boundary node and its velocity at t-1 sit in slots another thread
// overwrites, so each boundary node keeps them in side buffers (per link and
// per node) that it reads and rewrites itself.  An outlet node's thread also
// updates its upstream node, reading both before writing either.
#pragma once

#include <type_traits>

#include "lbm_device.hpp"
#include "lbm_kernels.hpp"

namespace lbm {

// ---------------------------------------------------------------------------
// Storage traits
// ---------------------------------------------------------------------------
template <int ST>
struct StT;
template <>
struct StT<ST_FP64> {
  using S = double;
  using R = double;
  static constexpr bool DEV = false;
};
template <>
struct StT<ST_FP32> {
  using S = float;
  using R = float;
  static constexpr bool DEV = false;
};
template <>
struct StT<ST_FP32_DEV> {
  using S = float;
  using R = float;
  static constexpr bool DEV = true;
};
template <>
struct StT<ST_FP16_DEV> {
  using S = __half;
  using R = float;
  static constexpr bool DEV = true;
};
template <>
struct StT<ST_FP32_SR> {
  using S = float;
  using R = double;
  static constexpr bool DEV = false;
};
template <>
struct StT<ST_FP16_SR> {
  using S = __half;
  using R = float;
  static constexpr bool DEV = true;
};
// FP16 deviation storage (either rounding), and the storages that round
// stochastically.
__host__ __device__ constexpr bool half_st(int st) { return st == ST_FP16_DEV || st == ST_FP16_SR; }
__host__ __device__ constexpr bool sr_st(int st) { return st == ST_FP32_SR || st == ST_FP16_SR; }

// Stochastic rounding of the FP32_SR storage.  A node draws one 32-bit
// value per step, the hash "lowbias32" (C. Wellons' integer hash prospector,
// public domain) of the node and the step's seed; the k-th value it stores
// in that step (f then h, direction order) takes the draw plus k times the
// golden-ratio increment 2^32 / phi (a Weyl sequence), so each draw stays
// uniform and each rounding unbiased.  Adding 29 bits of a draw to the 29
// mantissa bits of a double that FP32 does not hold, then clearing them,
// rounds the magnitude up with probability equal to the dropped fraction of
// an FP32 ulp and down otherwise (both signs alike); the result is then an
// exact FP32 value.
constexpr uint32_t SR_WEYL = 0x9E3779B9u;
__device__ __forceinline__ uint32_t sr_hash(uint32_t node, uint32_t seed) {
  uint32_t x = node * SR_WEYL ^ seed;
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}
__device__ __forceinline__ float sr_round(double v, uint32_t r) {
  unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
  b += static_cast<unsigned long long>(r >> 3);
  b &= ~((1ull << 29) - 1ull);
  return static_cast<float>(__longlong_as_double(static_cast<long long>(b)));
}
// FP16_SR: an FP32 deviation d rounded stochastically to FP16.  The FP16
// spacing at |d| is q = 2^(e - 10) for |d| >= 2^-14 (e: the exponent of d)
// and q = 2^-24 below, among the FP16 subnormals.  A uniform draw in [0, q)
// in steps of q / 2^13 (bits 10-22 of r as the top mantissa bits of a number
// in [q, 2q), minus q) is added to |d| and the sum is truncated toward zero onto
// the FP16 numbers, which rounds |d| up with probability equal to its
// distance above the lower neighbour in units of q.  The steps are FP32's
// spacing at |d| in the normal FP16 range, so the sum is exact there, and an
// FP16 value d never moves.  sr16_noised returns d with the draw added; the
// truncation is the round-toward-zero conversion (two values per
// instruction).
typedef __fp16 fp16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float sr16_noised(float d, uint32_t r) {
  const uint32_t b = __float_as_uint(d);
  const uint32_t qb = max(b & 0x7f800000u, 0x38800000u) - (10u << 23);
  const float noise = __uint_as_float(qb | (r & 0x007ffc00u)) - __uint_as_float(qb);
  return d + copysignf(noise, d);
}
// The FP16 value of one rounding, as FP32 (so a conversion that follows is
// exact).
__device__ __forceinline__ float sr16_round(float d, uint32_t r) {
  const fp16x2 p = __builtin_amdgcn_cvt_pkrtz(sr16_noised(d, r), 0.0f);
  return static_cast<float>(p.x);
}

// Population storage.  FP64 and FP32 elements: tiles of
// T = pop_tile_bytes(Q) / sizeof(S) consecutive nodes; a tile holds the Q
// slots of every lattice of its nodes one after the other (f then h when both
// are stored), [m / T][lattice][tile_pos(slot)][m % T], so the buffer of h
// starts Q T elements after that of f and ps = Q x (number of lattices) slots
// per tile.  A block then reads and writes runs of consecutive bytes per slot
// and tile, and all slots of a tile share DRAM pages.  Inside a tile the slots
// of equal (e_z, e_y), which are pulled from one neighbouring row, are
// adjacent.  FP16 elements with both lattices ("pairs"): the f and h values
// of one slot and node sit side by side in a 4-byte element, and those
// elements take the tile layout above with one lattice per tile, [m / T]
// [tile_pos(slot)][m % T][f, h] with T = pop_tile_bytes(Q) / 4, so the buffer
// of h starts one 2-byte element after that of f.  A step then moves both
// lattices of a slot with one 4-byte access per node.  On MI355X the same
// pulls over 54 2-byte planes reached 5.5 TB/s in a plain probe at 256^3, as
// 4-byte pairs in planes 5.6 TB/s and as pairs in tiles 6.0 TB/s.  FP16
// elements of one lattice: one plane of ps elements per slot, [slot][m].
template <class S, int NL>
__host__ __device__ constexpr bool fp16_pairs() {
  return sizeof(S) == 2 && NL == 2;
}
template <int Q>
__device__ __forceinline__ constexpr int tile_pos(int s) {
  return ((Lat<Q>::ez(s) + 1) * 3 + (Lat<Q>::ey(s) + 1)) * 3 + (Lat<Q>::ex(s) + 1) - (Lat<Q>::D == 2 ? 9 : 0);
}

// Direction whose slot sits at tile position k, so that k = 0 .. Q-1 visits
// the slots of a tile in address order.
template <int Q>
__device__ __forceinline__ constexpr int dir_at_pos(int k) {
  for (int i = 0; i < Q; i++)
    if (tile_pos<Q>(i) == k) return i;
  return 0;
}

// NL: lattices per tile (1 or 2) when the caller knows it at compile time,
// else 0 and ps holds the slots per tile (FP16 callers always know it).  A
// population's element index is
// slot_offset(slot) + node_offset(m): the first is uniform over a wavefront
// (it folds into the scalar base address), the second is shared by the slots
// pulled from one node.  Node indices are below 2^31 (the host rejects larger
// lattices), so (m / T) x (slots per tile) < 2^31 / 128 x 54 < 2^32 for every
// tile (T >= 128 nodes, at most 54 slots).
template <int Q, class S, int NL>
__device__ __forceinline__ int64_t slot_offset(int slot, int64_t ps) {
  if constexpr (fp16_pairs<S, NL>())
    return (int64_t)2 * tile_pos<Q>(slot) * (pop_tile_bytes(Q) / 4);
  else if constexpr (sizeof(S) == 2)
    return (int64_t)slot * ps;
  else
    return (int64_t)tile_pos<Q>(slot) * (pop_tile_bytes(Q) / (int)sizeof(S));
}

template <int Q, class S, int NL>
__device__ __forceinline__ uint64_t node_offset(int64_t ps, int64_t m) {
  const uint32_t u = (uint32_t)m;
  if constexpr (fp16_pairs<S, NL>()) {
    constexpr uint32_t T = pop_tile_bytes(Q) / 4;
    return 2 * ((uint64_t)u + (uint64_t)(u / T) * ((Q - 1) * T));
  } else if constexpr (sizeof(S) == 2) {
    return u;
  } else {
    constexpr uint32_t T = pop_tile_bytes(Q) / sizeof(S);
    const uint32_t spt = NL ? (uint32_t)(Q * NL) : (uint32_t)ps;
    uint64_t o = (uint64_t)((u / T) * spt) * T + (u % T);
    // one 64-bit value per pulled node, added once per access (the compiler
    // would otherwise split the sum and redo the 64-bit adds per slot)
    asm("" : "+v"(o));
    return o;
  }
}

// Base address of one slot, as a global-memory pointer.  Every caller passes
// a kernel-argument base and a slot fixed by an unrolled direction loop, so
// the address is uniform over the wavefront; the empty asm keeps it as one
// scalar value instead of letting the compiler fold the slot's constant
// offset into per-lane adds.
template <class E>
using global_ptr = __attribute__((address_space(1))) E *;

template <class E>
__device__ __forceinline__ global_ptr<E> uniform_base(E *p) {
  uint64_t v = reinterpret_cast<uint64_t>(p);
  asm("" : "+s"(v));
  return (global_ptr<E>)v;
}

// Load / store population i (stored in slot `slot`) of node m; ps is the
// slots per tile (FP64/FP32) or the plane stride (FP16) of the layout.  The
// deviation storages keep g_i - w_i g_ref; w_i = w_opp(i), so a swapped slot
// needs no other weight.
// 2-byte planes: the element's byte offset 2m (m < 2^31) fits in 32 bits, so
// the access is a scalar plane base plus one zero-extended 32-bit lane offset,
// which the pulls of both lattices from one node share (the scalar-base form
// of the global loads and stores); wider elements use 64-bit offsets.
template <class S, int NL, class P>
__device__ __forceinline__ P elem_at(P p, uint64_t off) {
  if constexpr (sizeof(S) == 2 && !fp16_pairs<S, NL>()) {
    using C = typename std::conditional<std::is_const<typename std::remove_pointer<P>::type>::value,
                                        __attribute__((address_space(1))) const char,
                                        __attribute__((address_space(1))) char>::type;
    const uint32_t b = (uint32_t)off * 2u;
    return (P)((C *)p + (uint64_t)b);
  } else {
    return p + off;
  }
}

template <int Q, int ST, int NL = 0>
__device__ __forceinline__ typename StT<ST>::R ldp(const void *base, int slot, int64_t ps, int64_t m,
                                                   typename StT<ST>::R ref) {
  using T = StT<ST>;
  using R = typename T::R;
  const global_ptr<const typename T::S> p =
      uniform_base(static_cast<const typename T::S *>(base) + slot_offset<Q, typename T::S, NL>(slot, ps));
  R v = StoreT<typename T::S>::ld(elem_at<typename T::S, NL>(p, node_offset<Q, typename T::S, NL>(ps, m)));
  if constexpr (T::DEV) v += weight<Q, R>(slot) * ref;
  return v;
}

// sr: the value's rounding draw (FP32_SR storage only).
template <int Q, int ST, int NL = 0>
__device__ __forceinline__ void stp(void *base, int slot, int64_t ps, int64_t m, typename StT<ST>::R v,
                                    typename StT<ST>::R ref, uint32_t sr = 0) {
  using T = StT<ST>;
  if constexpr (T::DEV) v -= weight<Q, typename T::R>(slot) * ref;
  const global_ptr<typename T::S> p =
      uniform_base(static_cast<typename T::S *>(base) + slot_offset<Q, typename T::S, NL>(slot, ps));
  if constexpr (ST == ST_FP32_SR)
    StoreT<float>::st(elem_at<float, NL>(p, node_offset<Q, float, NL>(ps, m)), sr_round(v, sr));
  else if constexpr (ST == ST_FP16_SR)
    StoreT<__half>::st(elem_at<__half, NL>(p, node_offset<Q, __half, NL>(ps, m)), sr16_round(v, sr));
  else
    StoreT<typename T::S>::st(elem_at<typename T::S, NL>(p, node_offset<Q, typename T::S, NL>(ps, m)), v);
}

// FP16 pairs: both lattices of slot `slot` of node m with one 4-byte access
// at the f element (the h element is the next one).  With T = 2^k nodes per
// tile the pair of node u sits 4 (u + (u / T)(Q - 1) T) bytes after the
// slot's first element; W64 = false computes that in 32 bits (the host picks
// it when 4 Q n < 2^32), so the access is a scalar slot base plus a 32-bit
// lane offset.
typedef _Float16 hpair __attribute__((ext_vector_type(2)));

template <int Q>
__host__ __device__ constexpr int pair_tile_log2() {
  int k = 0;
  while ((1 << (k + 1)) <= pop_tile_bytes(Q) / 4) k++;
  return k;
}
static_assert((1 << pair_tile_log2<9>()) == pop_tile_bytes(9) / 4, "pair tiles must be powers of two");
static_assert((1 << pair_tile_log2<27>()) == pop_tile_bytes(27) / 4, "pair tiles must be powers of two");

template <int Q, bool W64>
__device__ __forceinline__ uint64_t pair_byte_off(uint32_t u) {
  constexpr int LT = pair_tile_log2<Q>();
  constexpr uint32_t C = 4u * (Q - 1) * (1u << LT);
  if constexpr (W64)
    return ((uint64_t)u << 2) + (uint64_t)(u >> LT) * C;
  else
    return (uint64_t)((u << 2) + (u >> LT) * C);
}

template <int Q>
__device__ __forceinline__ const char *pair_slot_base(const void *fbase, int slot) {
  return static_cast<const char *>(fbase) + (size_t)4 * tile_pos<Q>(slot) * (pop_tile_bytes(Q) / 4);
}

template <int Q, bool W64>
__device__ __forceinline__ void ldp_pair(const void *fbase, int slot, int64_t m, float fref, float href, float &f,
                                         float &h) {
  const global_ptr<const char> p = uniform_base(pair_slot_base<Q>(fbase, slot));
  const hpair w = *reinterpret_cast<const __attribute__((address_space(1))) hpair *>(p + pair_byte_off<Q, W64>((uint32_t)m));
  f = (float)w.x + weight<Q, float>(slot) * fref;
  h = (float)w.y + weight<Q, float>(slot) * href;
}

// SR: FP16_SR storage, with the rounding draws rf and rh of the two values.
template <int Q, bool W64, bool SR = false>
__device__ __forceinline__ void stp_pair(void *fbase, int slot, int64_t m, float f, float h, float fref, float href,
                                         uint32_t rf = 0, uint32_t rh = 0) {
  const global_ptr<char> p = uniform_base(const_cast<char *>(pair_slot_base<Q>(fbase, slot)));
  hpair w;
  if constexpr (SR) {
    const fp16x2 v = __builtin_amdgcn_cvt_pkrtz(sr16_noised(f - weight<Q, float>(slot) * fref, rf),
                                                sr16_noised(h - weight<Q, float>(slot) * href, rh));
    w = __builtin_bit_cast(hpair, v);
  } else {
    w.x = (_Float16)(f - weight<Q, float>(slot) * fref);
    w.y = (_Float16)(h - weight<Q, float>(slot) * href);
  }
  __builtin_nontemporal_store(w, reinterpret_cast<__attribute__((address_space(1))) hpair *>(p + pair_byte_off<Q, W64>((uint32_t)m)));
}

// Value a store followed by a load of population i would return.
template <int Q, int ST>
__device__ __forceinline__ typename StT<ST>::R roundtrip(int i, typename StT<ST>::R v, typename StT<ST>::R ref,
                                                         uint32_t sr = 0) {
  using T = StT<ST>;
  using R = typename T::R;
  if constexpr (ST == ST_FP32_SR) {
    return R(sr_round(v, sr));
  } else if constexpr (ST == ST_FP16_SR) {
    return sr16_round(v - weight<Q, R>(i) * ref, sr) + weight<Q, R>(i) * ref;
  } else if constexpr (!T::DEV) {
    return v;
  } else {
    const R d = v - weight<Q, R>(i) * ref;
    R back;
    if constexpr (sizeof(typename T::S) == 2)
      back = __half2float(__float2half_rn(d));
    else
      back = d;
    return back + weight<Q, R>(i) * ref;
  }
}

template <class R>
__device__ __forceinline__ const R *rates(const KArgs &a, bool f);
template <>
__device__ __forceinline__ const double *rates<double>(const KArgs &a, bool f) {
  return f ? a.sf : a.sh;
}
template <>
__device__ __forceinline__ const float *rates<float>(const KArgs &a, bool f) {
  return f ? a.sf32 : a.sh32;
}
// Difference between the trace rate of f's second-order block and its
// diagonal rate (0: the trace relaxes with the deviator).
template <class R>
__device__ __forceinline__ R bulk_delta(const KArgs &a);
template <>
__device__ __forceinline__ double bulk_delta<double>(const KArgs &a) {
  return a.dbulk_f;
}
template <>
__device__ __forceinline__ float bulk_delta<float>(const KArgs &a) {
  return a.dbulk_f32;
}

__device__ __forceinline__ int wrapm(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Coordinates of a node and the index parts of its neighbours: node
// (x + dx, y + dy, z + dz), wrapped periodically, has index
// X[dx + 1] + Y[dy + 1] + Z[dz + 1].
struct Node {
  int x, y, z;
  uint32_t X[3], Y[3], Z[3];
};

// floor(m / d) for m < 2^31 from the divisor's multiplier M and shift s (set
// on the host): M = ceil(2^s / d), s = 31 + ceil(log2 d).
__device__ __forceinline__ uint32_t div_magic(uint32_t m, uint32_t M, int s) {
  return (uint32_t)(((uint64_t)m * M) >> s);
}

__device__ __forceinline__ uint32_t wrap_lo(uint32_t v, uint32_t n) { return v == 0 ? n - 1 : v - 1; }
__device__ __forceinline__ uint32_t wrap_hi(uint32_t v, uint32_t n) { return v + 1 == n ? 0 : v + 1; }

template <int Q>
__device__ __forceinline__ Node coords(const KArgs &a, int64_t m64) {
  const uint32_t m = (uint32_t)m64;
  const uint32_t nx = (uint32_t)a.nx, ny = (uint32_t)a.ny;
  const uint32_t r = div_magic(m, a.div_nx, a.sh_nx);
  uint32_t y = r, z = 0;
  if constexpr (Lat<Q>::D == 3) {
    z = div_magic(r, a.div_ny, a.sh_ny);
    y = r - z * ny;
  }
  const uint32_t x = m - r * nx;
  Node c;
  c.x = (int)x;
  c.y = (int)y;
  c.z = (int)z;
  c.X[0] = wrap_lo(x, nx);
  c.X[1] = x;
  c.X[2] = wrap_hi(x, nx);
  c.Y[0] = wrap_lo(y, ny) * nx;
  c.Y[1] = y * nx;
  c.Y[2] = wrap_hi(y, ny) * nx;
  if constexpr (Lat<Q>::D == 3) {
    const uint32_t nxy = nx * ny, nz = (uint32_t)a.nz;
    c.Z[0] = wrap_lo(z, nz) * nxy;
    c.Z[1] = z * nxy;
    c.Z[2] = wrap_hi(z, nz) * nxy;
  } else {
    c.Z[0] = c.Z[1] = c.Z[2] = 0;
  }
  return c;
}

// node x + sign * e_i with periodic wrap
template <int Q>
__device__ __forceinline__ int64_t shifted(const KArgs &a, const Node &c, int i, int sign) {
  (void)a;
  uint32_t m = c.X[1 + sign * Lat<Q>::ex(i)] + c.Y[1 + sign * Lat<Q>::ey(i)];
  if constexpr (Lat<Q>::D == 3) m += c.Z[1 + sign * Lat<Q>::ez(i)];
  return (int64_t)m;
}

// Prescribed velocity at node m (field or uniform).
template <int Q, class R>
__device__ __forceinline__ void prescribed_u(const KArgs &a, int64_t m, R &ux, R &uy, R &uz) {
  if (a.with_uvel) {
    const R *u = static_cast<const R *>(a.uvel);
    ux = u[m];
    uy = u[a.n + m];
    uz = Lat<Q>::D == 3 ? u[2 * a.n + m] : R(0);
  } else {
    ux = R(a.u0[0]);
    uy = R(a.u0[1]);
    uz = Lat<Q>::D == 3 ? R(a.u0[2]) : R(0);
  }
}

// rho and velocity of a population set in direction order.
template <int Q, class R>
__device__ __forceinline__ void velocity_dir(const R *f, R &rho, R &ux, R &uy, R &uz) {
  R r = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
  for (int i = 0; i < Q; i++) {
    r += f[i];
    if (Lat<Q>::ex(i) > 0) jx += f[i];
    if (Lat<Q>::ex(i) < 0) jx -= f[i];
    if (Lat<Q>::ey(i) > 0) jy += f[i];
    if (Lat<Q>::ey(i) < 0) jy -= f[i];
    if (Lat<Q>::ez(i) > 0) jz += f[i];
    if (Lat<Q>::ez(i) < 0) jz -= f[i];
  }
  const R inv = R(1) / r;
  rho = r;
  ux = jx * inv;
  uy = jy * inv;
  uz = Lat<Q>::D == 3 ? jz * inv : R(0);
}

// ---------------------------------------------------------------------------
// Layout-dependent addressing
// ---------------------------------------------------------------------------
// (slot, node) holding the pulled pre-collision value g_i(x) = g*_i(x - e_i)
template <int Q, int LAY>
__device__ __forceinline__ void pull_addr(const KArgs &a, Node c, int64_t m, int i, int &slot, int64_t &node) {
  if constexpr (LAY == LAY_AA_N) {
    slot = i;
    node = m;
  } else {
    slot = LAY == LAY_AA_S ? Lat<Q>::opp(i) : i;
    node = shifted<Q>(a, c, i, -1);
  }
}

// (slot, node) receiving the new post-collision value g*_i(x)
template <int Q, int LAY>
__device__ __forceinline__ void store_addr(const KArgs &a, Node c, int64_t m, int i, int &slot, int64_t &node) {
  if constexpr (LAY == LAY_AB) {
    slot = i;
    node = m;
  } else if constexpr (LAY == LAY_AA_S) {
    slot = i;
    node = shifted<Q>(a, c, i, +1);
  } else {
    slot = Lat<Q>::opp(i);
    node = m;
  }
}

// (slot, node) holding the stored post-collision value g*_i(x) of step t-1
// (read-only use: output passes, side rebuild, AB boundary rules)
template <int Q, int LAY>
__device__ __forceinline__ void post_addr(const KArgs &a, Node c, int64_t m, int i, int &slot, int64_t &node) {
  if constexpr (LAY == LAY_AB) {
    slot = i;
    node = m;
  } else if constexpr (LAY == LAY_AA_S) {
    slot = Lat<Q>::opp(i);
    node = m;
  } else {
    slot = i;
    node = shifted<Q>(a, c, i, +1);
  }
}

// Access order of a bulk node.  The D3Q27 steps and the D2Q9 in-place steps
// with central moments or order-limited cumulants pull all of f and then all
// of h, and store, each in address order within a tile: f's collision then
// waits only for f's loads while h's are still in flight.  On MI355X this
// measured faster at 256^3 (central moments 1.7%, FP32 and FP16-dev;
// cumulants 2.3% with the residency cap) and for the 2048^2 D2Q9 AA step
// (central moments 0.5%, cumulants 1.8%).  The D2Q9 two-array and the full
// cumulant steps keep direction order with f and h interleaved, which
// measured faster for them.
template <int Q, int LAY, int CU>
__device__ __forceinline__ constexpr bool split_order() {
  return (Lat<Q>::D == 3 || LAY != LAY_AB) && ((CU & 7) == 0 || (CU & 4));
}

// ---------------------------------------------------------------------------
// Realigned x-pushes of the swapped in-place phase (XR).  That phase stores
// g*_i(x) at x + e_i, so for e_x != 0 every wavefront's store lands one node
// off the line grid and neighbouring wavefronts share the edge lines of every
// slot.  When a block holds 256 consecutive nodes of one x-row (nx a multiple
// of 256, no geometry), the pushes with e_x != 0 are exchanged through LDS:
// thread t stores the push of thread s = (t - e_x) mod 256, whose destination
// (x_s + e_x, y + e_y, z + e_z) is t's own x for every t but one per direction
// (t = 0 for e_x = +1, t = 255 for e_x = -1, which stores the push that
// leaves the block; with nx = 256 the periodic wrap brings it back to t's own
// x).  Every store is the same push as before, made by another thread of the
// same block after one barrier, so the results are bit-identical; each
// wavefront then writes whole aligned lines except at the block's two edges.
// Measured on MI355X, in place, per step: 256^3 D3Q27 coupled FP32 1260 ->
// 1250 us (central moments), 1274 -> 1250 us (cumulant pair), FP16 741 -> 714
// us; 2048^2 D2Q9 coupled periodic FP32 96.5 -> 92.6 us, FP16 unchanged
// (48 us).  Plain (cached) stores for the misaligned pushes instead gained
// 1.5% on D2Q9 and nothing on D3Q27.  Lattices with geometry keep the plain
// push: in the fused bulk-and-boundary kernel (142 VGPRs, 3 blocks per CU)
// the realignment, with a flag per node for solid and listed nodes and its
// barrier reached from converged control flow, was bit-identical but slowed
// the 2048^2 heated-cylinder step from 92.5 to 95.2 us (cumulant pair 92.9 to
// 99.9).
// ---------------------------------------------------------------------------
template <int Q>
__device__ __forceinline__ constexpr int xr_index(int i) {
  int j = 0;
  for (int k = 0; k < i; k++)
    if (Lat<Q>::ex(k) != 0) j++;
  return j;
}
template <int Q>
constexpr int xr_dirs() {
  return 2 * Q / 3;
}
// LDS bytes of an XR step kernel: both lattices' x-pushes of 256 nodes.
template <int Q, class R>
constexpr size_t xr_lds_bytes() {
  return (size_t)2 * xr_dirs<Q>() * 256 * sizeof(R);
}

template <class R>
__device__ __forceinline__ R *xr_lds() {
  extern __shared__ __align__(16) unsigned char lbm_dyn_lds[];
  return reinterpret_cast<R *>(lbm_dyn_lds);
}

// Lattice lat (0 f, 1 h): hand the push of direction i (e_x != 0) to LDS.
template <int Q, class R>
__device__ __forceinline__ void xr_put(int lat, int i, R v) {
  xr_lds<R>()[(lat * xr_dirs<Q>() + xr_index<Q>(i)) * 256 + threadIdx.x] = v;
}

template <int Q, int ST, bool W64>
__device__ __forceinline__ void xr_pair_stores(const KArgs &a, const Node &c, const float *lds, int sp, int sm,
                                               uint32_t xp, uint32_t xm, uint32_t src) {
  constexpr bool SR = sr_st(ST);
#pragma unroll
  for (int k = 0; k < Q; k++) {
    const int i = dir_at_pos<Q>(k);
    if (Lat<Q>::ex(i) == 0) continue;
    const int s = Lat<Q>::ex(i) > 0 ? sp : sm;
    uint32_t node = (Lat<Q>::ex(i) > 0 ? xp : xm) + c.Y[1 + Lat<Q>::ey(i)];
    if constexpr (Lat<Q>::D == 3) node += c.Z[1 + Lat<Q>::ez(i)];
    // FP16_SR: the draws of the value's node and direction
    const uint32_t r = SR ? sr_hash(src + (uint32_t)s, a.sr_seed) : 0u;
    stp_pair<Q, W64, SR>(a.fdst, i, (int64_t)node, lds[xr_index<Q>(i) * 256 + s],
                         lds[(xr_dirs<Q>() + xr_index<Q>(i)) * 256 + s], float(a.fref), float(a.href),
                         r + (uint32_t)i * SR_WEYL, r + (uint32_t)(Q + i) * SR_WEYL);
  }
}

// After both lattices are handed over: one barrier, then each thread stores
// the pushes of its source threads (slot i, node x_s + e_i), in the tile's
// address order.
template <int Q, int ST, bool NS, int CU>
__device__ __forceinline__ void xr_store(const KArgs &a, const Node &c) {
  using R = typename StT<ST>::R;
  const R *lds = xr_lds<R>();
  __syncthreads();
  const int t = threadIdx.x;
  const uint32_t nx = (uint32_t)a.nx;
  const uint32_t x0 = (uint32_t)c.x - (uint32_t)t;  // first x of the block's row segment
  const int sp = (t - 1) & 255, sm = (t + 1) & 255;   // source threads for e_x = +1, -1
  uint32_t xp = x0 + (uint32_t)sp + 1u;
  if (xp >= nx) xp -= nx;
  const uint32_t xm = (x0 + (uint32_t)sm == 0u) ? nx - 1u : x0 + (uint32_t)sm - 1u;
  // node of source thread s: src + s (FP16_SR draws follow the value's node,
  // as in the other layouts)
  uint32_t src = x0 + c.Y[1];
  if constexpr (Lat<Q>::D == 3) src += c.Z[1];
  if constexpr (NS && half_st(ST)) {
    // FP16 pairs: f and h of a slot in one store
    if (a.pair64)
      xr_pair_stores<Q, ST, true>(a, c, lds, sp, sm, xp, xm, src);
    else
      xr_pair_stores<Q, ST, false>(a, c, lds, sp, sm, xp, xm, src);
    return;
  }
#pragma unroll
  for (int lat = NS ? 0 : 1; lat < 2; lat++) {
#pragma unroll
    for (int k = 0; k < Q; k++) {
      const int i = split_order<Q, LAY_AA_S, CU>() ? dir_at_pos<Q>(k) : k;
      if (Lat<Q>::ex(i) == 0) continue;
      const bool plus = Lat<Q>::ex(i) > 0;
      const R v = lds[(lat * xr_dirs<Q>() + xr_index<Q>(i)) * 256 + (plus ? sp : sm)];
      uint32_t node = (plus ? xp : xm) + c.Y[1 + Lat<Q>::ey(i)];
      if constexpr (Lat<Q>::D == 3) node += c.Z[1 + Lat<Q>::ez(i)];
      stp<Q, ST, NS ? 2 : 1>(lat ? a.hdst : a.fdst, i, a.ps, (int64_t)node, v, R(lat ? a.href : a.fref),
                             sr_st(ST) ? sr_hash(src + (uint32_t)(plus ? sp : sm), a.sr_seed) +
                                             (uint32_t)(lat ? Q + i : i) * SR_WEYL
                                       : 0u);
    }
  }
}

// Pulls and stores of FP16 pairs (both lattices), in the tile's address
// order; XR leaves the x-pushes to xr_store.
template <int Q, int LAY, bool W64>
__device__ __forceinline__ void pair_loads(const KArgs &a, const Node &c, int64_t m, float *f, float *h) {
#pragma unroll
  for (int k = 0; k < Q; k++) {
    const int i = dir_at_pos<Q>(k);
    int sl;
    int64_t nd;
    pull_addr<Q, LAY>(a, c, m, i, sl, nd);
    ldp_pair<Q, W64>(a.fsrc, sl, nd, float(a.fref), float(a.href), f[i], h[i]);
  }
}
template <int Q, int ST, int LAY, bool XR, bool W64>
__device__ __forceinline__ void pair_stores(const KArgs &a, const Node &c, int64_t m, const float *f, const float *h) {
  constexpr bool SR = sr_st(ST);
  const uint32_t r = SR ? sr_hash((uint32_t)m, a.sr_seed) : 0u;
#pragma unroll
  for (int k = 0; k < Q; k++) {
    const int i = dir_at_pos<Q>(k);
    if (XR && Lat<Q>::ex(i) != 0) continue;
    int sl;
    int64_t nd;
    store_addr<Q, LAY>(a, c, m, i, sl, nd);
    stp_pair<Q, W64, SR>(a.fdst, sl, nd, f[i], h[i], float(a.fref), float(a.href), r + (uint32_t)i * SR_WEYL,
                         r + (uint32_t)(Q + i) * SR_WEYL);
  }
}

// ---------------------------------------------------------------------------
// Epilogue: pre-collision populations f, h (direction order) of node m ->
// collide and store (f, h then hold the stored post-collision values), or
// write them / their moments out.
// ---------------------------------------------------------------------------
// CU selects the collision of each lattice: bit 0 h, bit 1 f use the cumulant
// collision (Eqs. hydro_cu_collision, H_cu_collision), else central moments;
// bit 2: the cumulants above second order (f) and first order (h) have rate 1,
// so their transform is skipped (the Cumulants-1st and hydrodynamic presets).
// XR: the swapped in-place phase's x-pushes go through LDS (xr_store; the
// whole block must reach it).
// FP16 pairs store f and h of a slot together once both are collided.
template <int Q, int ST, bool NS, int MODE, int LAY, int CU = 0, bool XR = false>
__device__ __forceinline__ void finish_node(const KArgs &a, Node c, int64_t m, typename StT<ST>::R *f,
                                            typename StT<ST>::R *h) {
  using R = typename StT<ST>::R;
  constexpr int D = Lat<Q>::D;
  constexpr bool PR = NS && half_st(ST);
  // a central-moment f step takes rho and u from its own transform
  constexpr bool OWN_U = NS && MODE == MODE_STEP && !(CU & 2);
  R rho = 0, ux = 0, uy = 0, uz = 0;
  if constexpr (NS && !OWN_U)
    velocity_dir<Q, R>(f, rho, ux, uy, uz);
  else if constexpr (!NS)
    prescribed_u<Q, R>(a, m, ux, uy, uz);
  const R src = a.src ? static_cast<const R *>(a.src)[m] : R(0);
  const uint32_t sr = sr_st(ST) ? sr_hash((uint32_t)m, a.sr_seed) : 0u;
  if constexpr (MODE == MODE_STEP) {
    R g[Q];
    if constexpr (NS) {
#pragma unroll
      for (int i = 0; i < Q; i++) g[Lat<Q>::slot(i)] = f[i];
      if constexpr ((CU & 2) && (CU & 4))
        collide_cu<D, R, 2, true>(g, rates<R>(a, true), ux, uy, uz, R(0), bulk_delta<R>(a));
      else if constexpr (CU & 2)
        collide_cu<D, R, 0, true>(g, rates<R>(a, true), ux, uy, uz, R(0), bulk_delta<R>(a));
      else
        collide_own_u<D, R, true, (CU & 8) ? RATE1_ORD3 : RATE1_NONE>(g, rates<R>(a, true), rho, ux, uy, uz,
                                                                       bulk_delta<R>(a));
#pragma unroll
      for (int k = 0; k < Q; k++) {
        const int i = split_order<Q, LAY, CU>() ? dir_at_pos<Q>(k) : k;
        int sl;
        int64_t nd;
        f[i] = g[Lat<Q>::slot(i)];
        if constexpr (XR) {
          if (Lat<Q>::ex(i) != 0) {
            xr_put<Q, R>(0, i, f[i]);
            continue;
          }
        }
        if constexpr (PR) continue;
        store_addr<Q, LAY>(a, c, m, i, sl, nd);
        stp<Q, ST, NS ? 2 : 1>(a.fdst, sl, a.ps, nd, f[i], R(a.fref), sr + (uint32_t)i * SR_WEYL);
      }
    }
#pragma unroll
    for (int i = 0; i < Q; i++) g[Lat<Q>::slot(i)] = h[i];
    if constexpr ((CU & 1) && (CU & 4))
      collide_cu<D, R, 1>(g, rates<R>(a, false), ux, uy, uz, src);
    else if constexpr (CU & 1)
      collide_cu<D, R>(g, rates<R>(a, false), ux, uy, uz, src);
    else
      collide<D, R, false, (CU & 32) ? RATE1_ORD2 : (CU & 16) ? RATE1_EVEN : RATE1_NONE>(g, rates<R>(a, false), ux,
                                                                                          uy, uz, src);
#pragma unroll
    for (int k = 0; k < Q; k++) {
      const int i = split_order<Q, LAY, CU>() ? dir_at_pos<Q>(k) : k;
      int sl;
      int64_t nd;
      h[i] = g[Lat<Q>::slot(i)];
      if constexpr (XR) {
        if (Lat<Q>::ex(i) != 0) {
          xr_put<Q, R>(1, i, h[i]);
          continue;
        }
      }
      if constexpr (PR) continue;
      store_addr<Q, LAY>(a, c, m, i, sl, nd);
      stp<Q, ST, NS ? 2 : 1>(a.hdst, sl, a.ps, nd, h[i], R(a.href), sr + (uint32_t)(Q + i) * SR_WEYL);
    }
    if constexpr (PR) {
      if (a.pair64)
        pair_stores<Q, ST, LAY, XR, true>(a, c, m, f, h);
      else
        pair_stores<Q, ST, LAY, XR, false>(a, c, m, f, h);
    }
    if constexpr (XR) {
      static_assert(LAY == LAY_AA_S, "realigned pushes belong to the swapped in-place phase");
      xr_store<Q, ST, NS, CU>(a, c);
    }
  } else if constexpr (MODE == MODE_PRE) {
#pragma unroll
    for (int i = 0; i < Q; i++) {
      if constexpr (NS)
        if (a.out0) a.out0[i * a.n + m] = double(f[i]);
      if (a.out1) a.out1[i * a.n + m] = double(h[i]);
    }
  } else {
    double H = 0.0, qx = 0.0;
#pragma unroll
    for (int i = 0; i < Q; i++) {
      H += double(h[i]);
      qx += double(Lat<Q>::ex(i)) * double(h[i]);
    }
    H += 0.5 * double(src);
    if (a.out0) a.out0[m] = double(rho);
    if (a.out1) {
      a.out1[m] = double(ux);
      a.out1[a.n + m] = double(uy);
      a.out1[2 * a.n + m] = double(uz);
    }
    if (a.out2) a.out2[m] = H;
    if (a.out3) a.out3[m] = qx;
  }
}

// Solid nodes carry no state: the output modes report zeros for them.
template <int Q, bool NS, int MODE>
__device__ __forceinline__ void solid_node(const KArgs &a, int64_t m) {
  if constexpr (MODE == MODE_PRE) {
#pragma unroll
    for (int i = 0; i < Q; i++) {
      if constexpr (NS)
        if (a.out0) a.out0[i * a.n + m] = 0.0;
      if (a.out1) a.out1[i * a.n + m] = 0.0;
    }
  } else if constexpr (MODE == MODE_MACRO) {
    if (a.out0) a.out0[m] = 0.0;
    if (a.out1) {
      a.out1[m] = 0.0;
      a.out1[a.n + m] = 0.0;
      a.out1[2 * a.n + m] = 0.0;
    }
    if (a.out2) a.out2[m] = 0.0;
    if (a.out3) a.out3[m] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// Block -> tile order.  Workgroups of one dispatch go round-robin to the 8
// XCDs (block b runs on XCD b % 8), and each XCD has its own L2.
//  - one slab per XCD: block b takes tile (b % 8) * per + b / 8, so each XCD
//    streams through one contiguous eighth of the lattice, and the cache lines
//    that neighbouring tiles of a row share through the +-1 pull shifts stay in
//    one L2 (wide 2-D rows span several blocks);
//  - chunks per XCD: runs of G consecutive blocks (G = row_blocks, a whole
//    number of x-rows) stay on one XCD and consecutive chunks go to
//    consecutive XCDs, so all XCDs work on nearby memory while the cache
//    lines shared along a row stay in one L2.
// Tail blocks that do not fill a whole round keep their own index.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t nb) {
  const int64_t per = nb / 8;
  return b < per * 8 ? (b % 8) * per + b / 8 : b;
}

__device__ __forceinline__ int64_t row_tile(int64_t b, int64_t nb, int64_t G) {
  const int64_t full = nb - nb % (8 * G);
  if (b >= full) return b;
  const int64_t x = b % 8, k = b / 8;
  return ((k / G) * 8 + x) * G + (k % G);
}

__device__ __forceinline__ int64_t tile_of(const KArgs &a, int64_t b, int64_t nb) {
  if (a.tilemap == 0) return xcd_tile(b, nb);
  if (a.tilemap == 1) return row_tile(b, nb, a.row_blocks);
  return b;
}

// ---------------------------------------------------------------------------
// Bulk nodes
// ---------------------------------------------------------------------------
// Populations of an EQ node of group g after streaming (Sec. 3): the
// equilibrium of the group's values, with the per-node velocity field when one
// is set, else the group's velocity (with f) or the prescribed one.
template <int Q, int ST, bool NS>
__device__ __forceinline__ void eq_node(const KArgs &a, int64_t m, int g, typename StT<ST>::R *f,
                                        typename StT<ST>::R *h) {
  using R = typename StT<ST>::R;
  const DevGroup &G = a.groups[g];
  R ux, uy, uz;
  if (NS && !a.with_uvel) {
    ux = R(G.u_w[0]);
    uy = R(G.u_w[1]);
    uz = Lat<Q>::D == 3 ? R(G.u_w[2]) : R(0);
  } else {
    prescribed_u<Q, R>(a, m, ux, uy, uz);
  }
#pragma unroll
  for (int i = 0; i < Q; i++) {
    if constexpr (NS) f[i] = geq_dir<Q, R>(i, R(G.rho_w), ux, uy, uz);
    h[i] = geq_dir<Q, R>(i, R(G.H_w), ux, uy, uz);
  }
}

// One node per thread, m = tile * 256 + threadIdx.x, so lane = m % 64.  With
// geometry the class byte is loaded alongside the populations so that its
// latency overlaps theirs (the pulls of a solid or listed node are in bounds
// and unused).  Bulk-class EQ nodes take their equilibrium; a bulk-class
// outlet node (zero gradient along x) takes the e_x < 0 populations of its
// upstream node x - 1, which the previous lane of the same wavefront has just
// pulled (that node has no cut links, so these are its final values).
template <int Q, int ST, bool NS, bool GEOM, int MODE, int LAY, int CU = 0, bool XR = false>
__device__ __forceinline__ void bulk_node(const KArgs &a, int64_t m) {
  using R = typename StT<ST>::R;
  if (m >= a.n) return;
  uint8_t cl = CLS_BULK;
  if constexpr (GEOM) cl = a.cls[m];
  const Node c = coords<Q>(a, m);
  R f[Q], h[Q];
  if constexpr (NS && half_st(ST)) {
    if (a.pair64)
      pair_loads<Q, LAY, true>(a, c, m, f, h);
    else
      pair_loads<Q, LAY, false>(a, c, m, f, h);
  } else if constexpr (split_order<Q, LAY, CU>()) {
    if constexpr (NS) {
#pragma unroll
      for (int k = 0; k < Q; k++) {
        const int i = dir_at_pos<Q>(k);
        int sl;
        int64_t nd;
        pull_addr<Q, LAY>(a, c, m, i, sl, nd);
        f[i] = ldp<Q, ST, NS ? 2 : 1>(a.fsrc, sl, a.ps, nd, R(a.fref));
      }
    }
#pragma unroll
    for (int k = 0; k < Q; k++) {
      const int i = dir_at_pos<Q>(k);
      int sl;
      int64_t nd;
      pull_addr<Q, LAY>(a, c, m, i, sl, nd);
      h[i] = ldp<Q, ST, NS ? 2 : 1>(a.hsrc, sl, a.ps, nd, R(a.href));
    }
  } else {
#pragma unroll
    for (int i = 0; i < Q; i++) {
      int sl;
      int64_t nd;
      pull_addr<Q, LAY>(a, c, m, i, sl, nd);
      if constexpr (NS) f[i] = ldp<Q, ST, NS ? 2 : 1>(a.fsrc, sl, a.ps, nd, R(a.fref));
      h[i] = ldp<Q, ST, NS ? 2 : 1>(a.hsrc, sl, a.ps, nd, R(a.href));
    }
  }
  if constexpr (GEOM) {
    if (__ballot(cl == CLS_OUTLET)) {
#pragma unroll
      for (int i = 0; i < Q; i++) {
        if (Lat<Q>::ex(i) >= 0) continue;
        if constexpr (NS) {
          const R fu = __shfl_up(f[i], 1);
          if (cl == CLS_OUTLET) f[i] = fu;
        }
        const R hu = __shfl_up(h[i], 1);
        if (cl == CLS_OUTLET) h[i] = hu;
      }
    }
    if (cl == CLS_SOLID) {
      solid_node<Q, NS, MODE>(a, m);
      return;
    }
    if (cl == CLS_SPECIAL) return;
    if (cl >= CLS_EQ) eq_node<Q, ST, NS>(a, m, cl - CLS_EQ, f, h);
  }
  finish_node<Q, ST, NS, MODE, LAY, CU, XR>(a, c, m, f, h);
}

// XR (realigned x-pushes) needs a block of 256 nodes of one x-row, all in the
// lattice (the host checks nx % 256 == 0), and no geometry.
template <int Q, int ST, bool NS, bool GEOM, int MODE, int LAY, int CU = 0, bool XR = false>
__global__ void __launch_bounds__(256) k_bulk(const KArgs a) {
  static_assert(!XR || (!GEOM && MODE == MODE_STEP), "realigned pushes need a plain step");
  const int64_t tile = tile_of(a, blockIdx.x, gridDim.x);
  bulk_node<Q, ST, NS, GEOM, MODE, LAY, CU, XR>(a, tile * 256 + threadIdx.x);
}

// ---------------------------------------------------------------------------
// Boundary nodes
// ---------------------------------------------------------------------------
// Pulled populations of node m plus the wall links in mask (links stored from
// lb, one per set bit in increasing direction), direction order.  side_node
// indexes the node's velocity entry of the AA side buffer.  flux (optional)
// receives h_opp(x_b, t) - h*_i(x_b, t-1) per link.
//
// Every value read here depends only on (m, lb, mask), so all loads are issued
// before the first use: while the bulk of the step saturates HBM a memory
// round trip takes microseconds, and a chain of them per link (record, group,
// then populations) would outlast the bulk nodes of the same launch.
template <int Q, int ST, bool NS, int LAY>
__device__ __forceinline__ void pull_links(const KArgs &a, int64_t m, int32_t lb, uint32_t mask, int64_t side_node,
                                           typename StT<ST>::R *f, typename StT<ST>::R *h, double *flux) {
  using R = typename StT<ST>::R;
  const Node c = coords<Q>(a, m);
  const R fref = R(a.fref), href = R(a.href);
#pragma unroll
  for (int i = 0; i < Q; i++) {
    int sl;
    int64_t nd;
    pull_addr<Q, LAY>(a, c, m, i, sl, nd);
    if constexpr (NS) f[i] = ldp<Q, ST, NS ? 2 : 1>(a.fsrc, sl, a.ps, nd, fref);
    h[i] = ldp<Q, ST, NS ? 2 : 1>(a.hsrc, sl, a.ps, nd, href);
  }
  if (mask == 0) return;
  if constexpr (LAY != LAY_AB) {
    // AA: the boundary node's velocity at t-1 from the side buffer, then one
    // link at a time (few registers: this path sets the register budget of
    // the fused step kernel)
    R ux, uy, uz;
    if constexpr (NS) {
      const R *su = static_cast<const R *>(a.side_u) + 3 * side_node;
      ux = su[0];
      uy = su[1];
      uz = su[2];
    } else {
      prescribed_u<Q, R>(a, m, ux, uy, uz);
    }
    const DevWall<R> *walls = static_cast<const DevWall<R> *>(a.walls);
#pragma unroll
    for (int i = 1; i < Q; i++) {
      if (!((mask >> i) & 1u)) continue;
      const int32_t l = lb + __popc(mask & ((1u << i) - 1u));
      const DevWall<R> w = walls[l];
      const int o = Lat<Q>::opp(i);
      int sl;
      int64_t nd;
      post_addr<Q, LAY>(a, c, m, i, sl, nd);
      // g*_i(x_b) at its post-collision address, g*_opp(i)(x_b) from the side
      // buffer (its slot is rewritten by another node in this step)
      if constexpr (NS) {
        const R gbi = ldp<Q, ST, NS ? 2 : 1>(a.fsrc, sl, a.ps, nd, fref);
        const R gbo = static_cast<const R *>(a.side_f)[l];
        f[o] = (w.interp & 1) ? wall_ibb<R>(w.q, gbi, gbo, f[i]) : gbi;
      }
      const R gbi = ldp<Q, ST, NS ? 2 : 1>(a.hsrc, sl, a.ps, nd, href);
      const R gbo = static_cast<const R *>(a.side_h)[l];
      const R geq = geq_dir<Q, R>(i, w.H_w, ux, uy, uz);
      h[o] = (w.interp & 2) ? wall_iabb<R>(w.q, gbi, gbo, h[i], geq) : -gbi + R(2) * geq;
      if (flux) flux[l] = double(h[o]) - double(gbi);
    }
    return;
  }
  // AB: g*_i(x_b) and g*_opp(i)(x_b) of step t-1 are the node's own stored
  // values; the wall velocity is the momentum over density of all of its f.
  // One link at a time, as in AA.
  R ux, uy, uz;
  if constexpr (NS) {
    R fb[Q], rho;
#pragma unroll
    for (int i = 0; i < Q; i++) fb[i] = ldp<Q, ST, NS ? 2 : 1>(a.fsrc, i, a.ps, m, fref);
    velocity_dir<Q, R>(fb, rho, ux, uy, uz);
    // the links reload their two values (from cache) instead of keeping all
    // of f live in registers
    asm volatile("" ::: "memory");
  } else {
    prescribed_u<Q, R>(a, m, ux, uy, uz);
  }
  const DevWall<R> *walls = static_cast<const DevWall<R> *>(a.walls);
#pragma unroll
  for (int i = 1; i < Q; i++) {
    if (!((mask >> i) & 1u)) continue;
    const int32_t l = lb + __popc(mask & ((1u << i) - 1u));
    const DevWall<R> w = walls[l];
    const int o = Lat<Q>::opp(i);
    // g*_i(x_f) is the pulled value f[i] / h[i] (never rewritten by another
    // link when it is used: that link would need x_f solid)
    if constexpr (NS) {
      const R gbi = ldp<Q, ST, NS ? 2 : 1>(a.fsrc, i, a.ps, m, fref);
      const R gbo = ldp<Q, ST, NS ? 2 : 1>(a.fsrc, o, a.ps, m, fref);
      f[o] = (w.interp & 1) ? wall_ibb<R>(w.q, gbi, gbo, f[i]) : gbi;  // else bounce-back (Eq. IBB at q = 1/2)
    }
    const R gbi = ldp<Q, ST, NS ? 2 : 1>(a.hsrc, i, a.ps, m, href);
    const R gbo = ldp<Q, ST, NS ? 2 : 1>(a.hsrc, o, a.ps, m, href);
    const R geq = geq_dir<Q, R>(i, w.H_w, ux, uy, uz);
    // else anti-bounce-back (Eq. IABB at q = 1/2)
    h[o] = (w.interp & 2) ? wall_iabb<R>(w.q, gbi, gbo, h[i], geq) : -gbi + R(2) * geq;
    if (flux) flux[l] = double(h[o]) - double(gbi);
  }
}

// AA side values of one boundary node after its update: g*_opp(i)(x_b) per
// link and the velocity of the stored f, both as they read back from storage
// (sr: the node's rounding draw of the step, FP32_SR storage).
template <int Q, int ST, bool NS>
__device__ __forceinline__ void save_side(const KArgs &a, int32_t lb, uint32_t mask, int64_t side_node,
                                          const typename StT<ST>::R *fpost, const typename StT<ST>::R *hpost,
                                          uint32_t sr = 0) {
  using R = typename StT<ST>::R;
  if constexpr (NS) {
    R fr[Q], rho, ux, uy, uz;
#pragma unroll
    for (int i = 0; i < Q; i++) fr[i] = roundtrip<Q, ST>(i, fpost[i], R(a.fref), sr + (uint32_t)i * SR_WEYL);
    if (mask) {
      R *su = static_cast<R *>(a.side_u) + 3 * side_node;
      velocity_dir<Q, R>(fr, rho, ux, uy, uz);
      su[0] = ux;
      su[1] = uy;
      su[2] = uz;
    }
#pragma unroll
    for (int i = 1; i < Q; i++) {
      if (!((mask >> i) & 1u)) continue;
      const int32_t l = lb + __popc(mask & ((1u << i) - 1u));
      static_cast<R *>(a.side_f)[l] = fr[Lat<Q>::opp(i)];
    }
  }
#pragma unroll
  for (int i = 1; i < Q; i++) {
    if (!((mask >> i) & 1u)) continue;
    const int32_t l = lb + __popc(mask & ((1u << i) - 1u));
    const int o = Lat<Q>::opp(i);
    static_cast<R *>(a.side_h)[l] = roundtrip<Q, ST>(o, hpost[o], R(a.href), sr + (uint32_t)(Q + o) * SR_WEYL);
  }
}

template <int Q, int ST, bool NS, int MODE, int LAY, int CU = 0>
__device__ __forceinline__ void special_node(const KArgs &a, int64_t t) {
  using R = typename StT<ST>::R;
  constexpr bool AA = LAY != LAY_AB;
  if (t >= a.nspecial) return;
  const DevSpecial sp = a.special[t];
  const int64_t m = sp.node;
  const Node c = coords<Q>(a, m);
  double *flux = MODE == MODE_MACRO ? a.link_flux : nullptr;
  R f[Q], h[Q];
  if (sp.type == NODE_EQ) {
    if (flux) pull_links<Q, ST, NS, LAY>(a, m, sp.lb, sp.mask, 2 * t, f, h, flux);
    eq_node<Q, ST, NS>(a, m, sp.group, f, h);
  } else {
    pull_links<Q, ST, NS, LAY>(a, m, sp.lb, sp.mask, 2 * t, f, h, flux);
    if (sp.type == NODE_OUTLET) {
      const int64_t up = c.x == 0 ? m + a.nx - 1 : m - 1;
      R fu[Q], hu[Q];
      // AA: this thread also owns the upstream node (its flux included)
      pull_links<Q, ST, NS, LAY>(a, up, sp.ub, sp.umask, 2 * t + 1, fu, hu, AA ? flux : nullptr);
#pragma unroll
      for (int i = 0; i < Q; i++) {
        if (Lat<Q>::ex(i) < 0) {
          if constexpr (NS) f[i] = fu[i];
          h[i] = hu[i];
        }
      }
      if constexpr (AA) {
        finish_node<Q, ST, NS, MODE, LAY, CU>(a, coords<Q>(a, up), up, fu, hu);
        if constexpr (MODE == MODE_STEP)
          save_side<Q, ST, NS>(a, sp.ub, sp.umask, 2 * t + 1, fu, hu,
                               sr_st(ST) ? sr_hash((uint32_t)up, a.sr_seed) : 0u);
      }
    }
  }
  finish_node<Q, ST, NS, MODE, LAY, CU>(a, c, m, f, h);
  if constexpr (AA && MODE == MODE_STEP)
    save_side<Q, ST, NS>(a, sp.lb, sp.mask, 2 * t, f, h, sr_st(ST) ? sr_hash((uint32_t)m, a.sr_seed) : 0u);
}

template <int Q, int ST, bool NS, int MODE, int LAY, int CU = 0>
__global__ void __launch_bounds__(64) k_special(const KArgs a) {
  special_node<Q, ST, NS, MODE, LAY, CU>(a, (int64_t)blockIdx.x * 64 + threadIdx.x);
}

// One launch per step with geometry (D2Q9): the first `sblocks` blocks (a
// multiple of 8, so the XCD of a bulk block is unchanged) take the boundary
// nodes, whose long chains of dependent loads then overlap the bulk stream
// instead of running after it.
template <int Q, int ST, bool NS, int LAY, int CU>
__device__ __forceinline__ void fused_body(const KArgs &a, int sblocks) {
  if ((int)blockIdx.x < sblocks) {
    special_node<Q, ST, NS, MODE_STEP, LAY, CU>(a, (int64_t)blockIdx.x * 256 + threadIdx.x);
    return;
  }
  const int64_t tile = tile_of(a, blockIdx.x - sblocks, gridDim.x - sblocks);
  bulk_node<Q, ST, NS, true, MODE_STEP, LAY, CU>(a, tile * 256 + threadIdx.x);
}

// (The scalar state of the boundary path limits this launch to 7 waves per
// SIMD where the bulk kernel runs 8; forcing 8 measured slower on MI355X.)
template <int Q, int ST, bool NS, int LAY, int CU>
__global__ void __launch_bounds__(256) k_fused(const KArgs a, int sblocks) {
  fused_body<Q, ST, NS, LAY, CU>(a, sblocks);
}

// AA side buffers from the stored state (after init, set or load).
template <int Q, int ST, bool NS, int LAY>
__global__ void __launch_bounds__(64) k_side(const KArgs a) {
  using R = typename StT<ST>::R;
  const int64_t t = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (t >= a.nspecial) return;
  const DevSpecial sp = a.special[t];
  for (int k = 0; k < 2; k++) {
    if (k == 1 && sp.type != NODE_OUTLET) break;
    const int64_t m = k == 0 ? sp.node : (sp.node % a.nx == 0 ? sp.node + a.nx - 1 : sp.node - 1);
    const Node c = coords<Q>(a, m);
    R f[Q], h[Q];
#pragma unroll
    for (int i = 0; i < Q; i++) {
      int sl;
      int64_t nd;
      post_addr<Q, LAY>(a, c, m, i, sl, nd);
      if constexpr (NS) f[i] = ldp<Q, ST, NS ? 2 : 1>(a.fsrc, sl, a.ps, nd, R(a.fref));
      else f[i] = R(0);
      h[i] = ldp<Q, ST, NS ? 2 : 1>(a.hsrc, sl, a.ps, nd, R(a.href));
    }
    save_side<Q, ST, NS>(a, k == 0 ? sp.lb : sp.ub, k == 0 ? sp.mask : sp.umask, 2 * t + k, f, h);
  }
}

// ---------------------------------------------------------------------------
// Initial state: g*_i(x) = g^eq_i(fields at x + e_i) in FP64, stored at the
// post-collision address of the layout (AB, or the swapped AA layout).
// ---------------------------------------------------------------------------
template <int Q, int ST, bool NS, int LAY>
__global__ void __launch_bounds__(256) k_init(const InitArgs a) {
  using R = typename StT<ST>::R;
  const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (m >= a.n) return;
  const int x = (int)(m % a.nx);
  const int64_t r = m / a.nx;
  const int y = (int)(r % a.ny);
  const int z = (int)(r / a.ny);
#pragma unroll
  for (int i = 0; i < Q; i++) {
    const int xs = wrapm(x + Lat<Q>::ex(i), a.nx);
    const int ys = wrapm(y + Lat<Q>::ey(i), a.ny);
    const int zs = wrapm(z + Lat<Q>::ez(i), a.nz);
    const int64_t s = xs + (int64_t)a.nx * (ys + (int64_t)a.ny * zs);
    double ux, uy, uz;
    if (a.u) {
      ux = a.u[s];
      uy = a.u[a.n + s];
      uz = a.u[2 * a.n + s];
    } else if (a.uvel) {
      const R *u = static_cast<const R *>(a.uvel);
      ux = double(u[s]);
      uy = double(u[a.n + s]);
      uz = Lat<Q>::D == 3 ? double(u[2 * a.n + s]) : 0.0;
    } else {
      ux = a.u0[0];
      uy = a.u0[1];
      uz = a.u0[2];
    }
    if (Lat<Q>::D == 2) uz = 0.0;
    const int slot = LAY == LAY_AB ? i : Lat<Q>::opp(i);
    const uint32_t sr = sr_st(ST) ? sr_hash((uint32_t)m, 0u) : 0u;
    if constexpr (NS) {
      const double rho = a.rho ? a.rho[s] : 1.0;
      stp<Q, ST, NS ? 2 : 1>(a.fdst, slot, a.ps, m, R(geq_dir<Q, double>(i, rho, ux, uy, uz)), R(a.fref),
                             sr + (uint32_t)i * SR_WEYL);
    }
    stp<Q, ST, NS ? 2 : 1>(a.hdst, slot, a.ps, m, R(geq_dir<Q, double>(i, a.H[s], ux, uy, uz)), R(a.href),
                           sr + (uint32_t)(Q + i) * SR_WEYL);
  }
}

// Stored post-collision state <-> FP64 [Q][n] (direction order).  Reading
// out, solid nodes (cls) report zeros; writing in fills the layout's
// post-collision addresses.
template <int Q, int ST, int LAY, bool TO_STORAGE, int NL>
__global__ void __launch_bounds__(256) k_convert(const KArgs a, const void *from, void *to, double ref) {
  using R = typename StT<ST>::R;
  const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (m >= a.n) return;
  const Node c = coords<Q>(a, m);
  const bool solid = a.cls && a.cls[m] == CLS_SOLID;
  const uint32_t sr = sr_st(ST) ? sr_hash((uint32_t)m, a.sr_seed) : 0u;
#pragma unroll
  for (int i = 0; i < Q; i++) {
    int sl;
    int64_t nd;
    post_addr<Q, LAY>(a, c, m, i, sl, nd);
    if constexpr (TO_STORAGE)
      stp<Q, ST, NL>(to, sl, a.ps, nd, R(static_cast<const double *>(from)[i * a.n + m]), R(ref),
                     sr + (uint32_t)i * SR_WEYL);
    else
      static_cast<double *>(to)[i * a.n + m] = solid ? 0.0 : double(ldp<Q, ST, NL>(from, sl, a.ps, nd, R(ref)));
  }
}

// ---------------------------------------------------------------------------
// Discrete adjoint of the periodic advection-diffusion step: node y
// gathers lam_next_i(y + e_i) (transpose of the pull), applies the transposed
// collision of node y and writes lam_prev(y); dJdQ(y) += b^T lam.
// ---------------------------------------------------------------------------
template <int Q, class R>
__global__ void __launch_bounds__(256) k_adjoint(const KArgs a, const R *lam_next, R *lam_prev, double *dJdQ) {
  constexpr int D = Lat<Q>::D;
  const int64_t m = tile_of(a, blockIdx.x, gridDim.x) * 256 + threadIdx.x;
  if (m >= a.n) return;
  const Node c = coords<Q>(a, m);
  R g[Q];
#pragma unroll
  for (int i = 0; i < Q; i++) {
    const int64_t d = shifted<Q>(a, c, i, +1);
    g[Lat<Q>::slot(i)] = __builtin_nontemporal_load(lam_next + (int64_t)i * a.n + d);
  }
  R ux, uy, uz;
  prescribed_u<Q, R>(a, m, ux, uy, uz);
  const R dq = collide_adjoint<D, R>(g, rates<R>(a, false), ux, uy, uz);
#pragma unroll
  for (int i = 0; i < Q; i++) __builtin_nontemporal_store(g[Lat<Q>::slot(i)], lam_prev + (int64_t)i * a.n + m);
  if (dJdQ) dJdQ[m] += double(dq);
}

// Discrete adjoint of the advection-diffusion step with geometry (walls
// ABB/IABB of Eq. IABB, EQ nodes, outlets).  With mu = S^T lam_next (the
// transpose of streaming with the wall rules), lam_prev = C^T mu node by
// node, and C^T is linear, so:
//  1. k_adj_bulk gathers mu_i(y) = lam_next_i(y + e_i) where node y + e_i
//     pulls h*_i(y) (not solid, not an EQ node, not the e_x < 0 populations
//     of a bulk outlet, plus the copy of a bulk outlet whose upstream node
//     y + e_i is) and applies C^T in registers, as the periodic kernel;
//  2. k_adj_fix walks the boundary-node list.  Each record lists the terms
//     of mu that pass 1 got wrong (its wall rules; for a listed EQ node or
//     outlet the gathered terms that are not pulls, and for an outlet the
//     transpose of its copy), and adds C^T of each term to lam_prev of the
//     node it belongs to, with atomics: two records can share a node.
template <int Q, class R>
__global__ void __launch_bounds__(256) k_adj_bulk(const KArgs a, const R *lam_next, R *lam_prev, double *dJdQ) {
  constexpr int D = Lat<Q>::D;
  const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (m >= a.n) return;
  if (a.cls[m] == CLS_SOLID) {
#pragma unroll
    for (int i = 0; i < Q; i++) lam_prev[(int64_t)i * a.n + m] = R(0);
    return;
  }
  const Node c = coords<Q>(a, m);
  R g[Q];
#pragma unroll
  for (int i = 0; i < Q; i++) {
    const int64_t d = shifted<Q>(a, c, i, +1);
    const uint8_t cd = a.cls[d];
    // a bulk outlet copies its e_x < 0 populations from node x - 1 instead
    const bool copied = Lat<Q>::ex(i) < 0 && cd == CLS_OUTLET;
    const bool pulled = cd != CLS_SOLID && cd < CLS_EQ && !copied;
    R v = pulled ? lam_next[(int64_t)i * a.n + d] : R(0);
    if (Lat<Q>::ex(i) < 0 && pulled && cd == CLS_BULK) {
      // node d + e_x may be a bulk outlet that copies h_i(d) = h*_i(m)
      int64_t d2 = c.X[1] + c.Y[1 + Lat<Q>::ey(i)];
      if constexpr (Lat<Q>::D == 3) d2 += c.Z[1 + Lat<Q>::ez(i)];
      if (a.cls[d2] == CLS_OUTLET) v += lam_next[(int64_t)i * a.n + d2];
    }
    g[Lat<Q>::slot(i)] = v;
  }
  R ux, uy, uz;
  prescribed_u<Q, R>(a, m, ux, uy, uz);
  const R dq = collide_adjoint<D, R>(g, rates<R>(a, false), ux, uy, uz);
#pragma unroll
  for (int i = 0; i < Q; i++) lam_prev[(int64_t)i * a.n + m] = g[Lat<Q>::slot(i)];
  if (dJdQ) dJdQ[m] += double(dq);
}

// One term v of mu_k(node) missed or mis-taken by k_adj_bulk.
template <class R>
struct AdjTerm {
  int64_t node;
  int32_t k;
  R v;
};

// Terms of the wall rule that writes h_o(x) from h*_i(x), h*_o(x) and the
// pulled h*_i(x - e_i) (o = opp(i)), for the adjoint lo of h_o(x).
template <int Q, class R>
__device__ __forceinline__ void adj_wall_terms(const KArgs &a, const Node &c, int64_t m, int i, const DevWall<R> &w,
                                               R lo, AdjTerm<R> *t, int &nt) {
  const int o = Lat<Q>::opp(i);
  if (!(w.interp & 2)) {
    t[nt++] = {m, i, -lo};
  } else if (w.q <= R(0.5)) {
    t[nt++] = {m, i, -R(2) * w.q * lo};
    t[nt++] = {shifted<Q>(a, c, i, -1), i, -(R(1) - R(2) * w.q) * lo};
  } else {
    t[nt++] = {m, i, -lo / (R(2) * w.q)};
    t[nt++] = {m, o, (R(2) * w.q - R(1)) * lo / (R(2) * w.q)};
  }
}

// One thread per (boundary-node record, direction dir): the terms of that
// direction (as the cut link dir, and for an outlet as the copied direction
// dir), so that the few terms of a record spread over Q threads.
template <int Q, class R>
__global__ void __launch_bounds__(256) k_adj_fix(const KArgs a, const R *lam_next, R *lam_prev, double *dJdQ) {
  constexpr int D = Lat<Q>::D;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= a.nspecial * Q) return;
  const int64_t r = idx / Q;
  const int dir = (int)(idx - r * Q);
  const DevSpecial sp = a.special[r];
  const int64_t m = sp.node;
  const Node c = coords<Q>(a, m);
  AdjTerm<R> t[5];
  int nt = 0;
  if (sp.type == NODE_EQ) {
    // pass 1 gathered lam_dir(x_eq) into a neighbour, but EQ nodes pull nothing
    const int64_t y = shifted<Q>(a, c, dir, -1);
    if (a.cls[y] != CLS_SOLID) t[nt++] = {y, dir, -lam_next[(int64_t)dir * a.n + m]};
  } else {
    const bool outlet = sp.type == NODE_OUTLET;
    const DevWall<R> *walls = static_cast<const DevWall<R> *>(a.walls);
    const int o = Lat<Q>::opp(dir);
    // an outlet's e_x < 0 populations are copied, not taken from its walls
    if (((sp.mask >> dir) & 1u) && !(outlet && Lat<Q>::ex(o) < 0)) {
      const DevWall<R> w = walls[sp.lb + __popc(sp.mask & ((1u << dir) - 1u))];
      adj_wall_terms<Q, R>(a, c, m, dir, w, lam_next[(int64_t)o * a.n + m], t, nt);
    }
    if (outlet && Lat<Q>::ex(dir) < 0) {
      // h_dir(x_o) = h_dir(u), u = x_o - 1: pass 1 took lam_dir(x_o) as a
      // pull, which it is not; it goes to what h_dir(u) came from instead
      const int j = dir;
      const int64_t u = c.x == 0 ? m + a.nx - 1 : m - 1;
      const Node cu = coords<Q>(a, u);
      const R lx = lam_next[(int64_t)j * a.n + m];
      const int64_t y = shifted<Q>(a, c, j, -1);
      if (a.cls[y] != CLS_SOLID) t[nt++] = {y, j, -lx};
      const int i = Lat<Q>::opp(j);
      if ((sp.umask >> i) & 1u) {
        // h_j(u) is the wall rule of u's cut link i
        const DevWall<R> w = walls[sp.ub + __popc(sp.umask & ((1u << i) - 1u))];
        adj_wall_terms<Q, R>(a, cu, u, i, w, lx, t, nt);
      } else {
        t[nt++] = {shifted<Q>(a, cu, j, -1), j, lx};
      }
    }
  }
  for (int e = 0; e < nt; e++) {
    const AdjTerm<R> te = t[e];
    R g[Q];
#pragma unroll
    for (int i = 0; i < Q; i++) g[Lat<Q>::slot(i)] = i == te.k ? te.v : R(0);
    R ux, uy, uz;
    prescribed_u<Q, R>(a, te.node, ux, uy, uz);
    const R dq = collide_adjoint<D, R>(g, rates<R>(a, false), ux, uy, uz);
#pragma unroll
    for (int i = 0; i < Q; i++) atomicAdd(lam_prev + (int64_t)i * a.n + te.node, g[Lat<Q>::slot(i)]);
    if (dJdQ) atomicAdd(dJdQ + te.node, double(dq));
  }
}

// Objective J = 1/2 sum (H - H*)^2 over the non-solid nodes (solid nodes
// carry no state): seeds lam = dJ/dpre (every direction
// H - H*), sets dJdQ = (H - H*)/2 (Q enters H as Q/2), leaves (H - H*)^2 in sq.
template <int Q, class R>
__global__ void __launch_bounds__(256) k_seed(const double *H, const double *Ht, const uint8_t *cls, int64_t n, R *lam,
                                              double *dJdQ, double *sq) {
  const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (m >= n) return;
  const double d = (cls && cls[m] == CLS_SOLID) ? 0.0 : H[m] - Ht[m];
#pragma unroll
  for (int i = 0; i < Q; i++) lam[(int64_t)i * n + m] = R(d);
  dJdQ[m] = 0.5 * d;
  sq[m] = d * d;
}

// ---------------------------------------------------------------------------
// Launchers for one lattice
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

#define LBM_DISPATCH_LAY(LAY_VAL, CALL) \
  switch (LAY_VAL) {                    \
    case LAY_AB: {                      \
      constexpr int LAY = LAY_AB;       \
      return CALL;                      \
    }                                   \
    case LAY_AA_S: {                    \
      constexpr int LAY = LAY_AA_S;     \
      return CALL;                      \
    }                                   \
    case LAY_AA_N: {                    \
      constexpr int LAY = LAY_AA_N;     \
      return CALL;                      \
    }                                   \
    default:                            \
      return hipErrorInvalidValue;      \
  }

// cu (bit 0 h, bit 1 f: cumulant collision; bit 2: order-limited cumulant
// transform; bit 3: central-moment f with every rate of order >= 3 equal to
// 1; bits 4 / 5: central-moment h with every even-order rate / every rate but
// the first order equal to 1) as a compile-time CU for CALL; f bits need the
// hydrodynamic lattice, bit 2 a cumulant bit.  The host picks the rate bits
// only for the combinations listed here.
#define LBM_CU_CASE(NS_VAL, V, CALL)       \
  case V:                                   \
    if constexpr (!((V) & 10) || NS_VAL) {  \
      constexpr int CU = V;                 \
      CALL;                                 \
      break;                                \
    } else {                                \
      return hipErrorInvalidValue;          \
    }
#define LBM_DISPATCH_CU(NS_VAL, CU_VAL, CALL) \
  switch (CU_VAL) {                           \
    LBM_CU_CASE(NS_VAL, 0, CALL)              \
    LBM_CU_CASE(NS_VAL, 1, CALL)              \
    LBM_CU_CASE(NS_VAL, 2, CALL)              \
    LBM_CU_CASE(NS_VAL, 3, CALL)              \
    LBM_CU_CASE(NS_VAL, 5, CALL)              \
    LBM_CU_CASE(NS_VAL, 6, CALL)              \
    LBM_CU_CASE(NS_VAL, 7, CALL)              \
    LBM_CU_CASE(NS_VAL, 8, CALL)              \
    LBM_CU_CASE(NS_VAL, 16, CALL)             \
    LBM_CU_CASE(NS_VAL, 22, CALL)             \
    LBM_CU_CASE(NS_VAL, 24, CALL)             \
    LBM_CU_CASE(NS_VAL, 32, CALL)             \
    LBM_CU_CASE(NS_VAL, 40, CALL)             \
    default:                                  \
      return hipErrorInvalidValue;            \
  }

// Residency cap of a step kernel.  The step kernels use no LDS; an unused
// dynamic LDS request caps the blocks of 256 threads resident on one CU (160
// KB of LDS) at `blocks`.  On MI355X the FP32 steps of D3Q27 and the D2Q9
// two-array step stream faster under a cap than at the residency their
// register count allows.  At 256^3 the D3Q27 central-moment step takes 1178
// us at 2 blocks per CU against 1235 uncapped (AA: 1266 against 1369), the
// order-limited cumulant step 1192 at 2 against 1218 at 3 and 1244 at 4 (AA:
// 1273 against 1326 at 3); at 2048^2 the D2Q9 two-array step takes 97.2 us
// at 3 against 100.9, and with FP64 storage 196.1 at 2 against 203.5 (the
// D2Q9 in-place fused step: fused_lds).  The FP16 two-array steps, the FP64
// D3Q27 steps and the full cumulant transform measured no gain or a loss.  The in-place D3Q27 FP16
// central-moment step takes 630 us at 3 blocks per CU in its streamed phase
// against 646 uncapped (641 at 2, 632 at 4; the swapped phase holds 4 blocks
// per CU through its LDS exchange).  FP32 storage with FP64 arithmetic
// (stochastic rounding): the in-place D3Q27 step takes 1288 us at 2 blocks
// per CU against 1330 uncapped; its two-array D3Q27 and its D2Q9 steps run
// fastest uncapped.  0 = no cap.
constexpr size_t lds_for_blocks(int blocks) { return (size_t)(160 * 1024) / (blocks + 1) + 1024; }

template <int Q, int ST, int LAY, int CU>
constexpr size_t step_lds() {
  constexpr bool fp32 = (ST == ST_FP32 || ST == ST_FP32_DEV) && ((CU & 7) == 0 || (CU & 4));
  if constexpr (Q == 27 && fp32) return lds_for_blocks(2);
  if constexpr (Q == 27 && ST == ST_FP16_DEV && LAY == LAY_AA_N && (CU & 7) == 0) return lds_for_blocks(3);
  if constexpr (Q == 27 && ST == ST_FP32_SR && LAY != LAY_AB && ((CU & 7) == 0 || (CU & 4)))
    return lds_for_blocks(2);
  if constexpr (Q == 9 && fp32 && LAY == LAY_AB) return lds_for_blocks(3);
  if constexpr (Q == 9 && ST == ST_FP64 && LAY == LAY_AB && ((CU & 7) == 0 || (CU & 4))) return lds_for_blocks(2);
  return 0;
}

template <int Q, int ST, bool NS, bool GEOM, int LAY>
static hipError_t pass_t(int mode, int cu, const KArgs &a, hipStream_t s) {
  const unsigned g = blocks_for(a.n, 256);
  if constexpr (!GEOM && LAY == LAY_AA_S && sizeof(typename StT<ST>::R) == 4) {
    if (mode == MODE_STEP && a.xr) {
      if (a.nx % 256 != 0) return hipErrorInvalidValue;
      constexpr size_t lx = xr_lds_bytes<Q, float>();
      LBM_DISPATCH_CU(NS, cu, (k_bulk<Q, ST, NS, false, MODE_STEP, LAY, CU, true>
                               <<<g, 256, step_lds<Q, ST, LAY, CU>() > lx ? step_lds<Q, ST, LAY, CU>() : lx, s>>>(a)))
      return hipGetLastError();
    }
  }
  if (mode == MODE_STEP)
    LBM_DISPATCH_CU(NS, cu, (k_bulk<Q, ST, NS, GEOM, MODE_STEP, LAY, CU><<<g, 256, step_lds<Q, ST, LAY, CU>(), s>>>(a)))
  else if (mode == MODE_PRE)
    k_bulk<Q, ST, NS, GEOM, MODE_PRE, LAY><<<g, 256, 0, s>>>(a);
  else
    k_bulk<Q, ST, NS, GEOM, MODE_MACRO, LAY><<<g, 256, 0, s>>>(a);
  return hipGetLastError();
}

template <int Q, int ST, bool NS, int LAY>
static hipError_t special_t(int mode, int cu, const KArgs &a, hipStream_t s) {
  if (a.nspecial == 0) return hipSuccess;
  const unsigned g = blocks_for(a.nspecial, 64);
  if (mode == MODE_STEP)
    LBM_DISPATCH_CU(NS, cu, (k_special<Q, ST, NS, MODE_STEP, LAY, CU><<<g, 64, 0, s>>>(a)))
  else if (mode == MODE_PRE)
    k_special<Q, ST, NS, MODE_PRE, LAY><<<g, 64, 0, s>>>(a);
  else
    k_special<Q, ST, NS, MODE_MACRO, LAY><<<g, 64, 0, s>>>(a);
  return hipGetLastError();
}

// The fused D2Q9 step in place: FP32 at 3 blocks per CU in the swapped phase
// and 4 in the streamed one.  With the one-link-at-a-time wall path (96 and
// 70 VGPRs, where the swapped phase took 142 before) the uncapped 2048^2
// heated-cylinder step ran 97.5 us, capped 92.5 (the cumulant pair 97.6 and
// 93.3); FP16 runs fastest uncapped (48.0 us).  FP64 in place: 2 blocks per CU
// in both phases, 218.5 us against 223.8 uncapped.
template <int Q, int ST, int LAY, int CU>
constexpr size_t fused_lds() {
  constexpr bool limited = (CU & 7) == 0 || (CU & 4);
  constexpr bool fp32 = (ST == ST_FP32 || ST == ST_FP32_DEV) && limited;
  if constexpr (Q == 9 && fp32 && LAY == LAY_AA_S) return lds_for_blocks(3);
  if constexpr (Q == 9 && fp32 && LAY == LAY_AA_N) return lds_for_blocks(4);
  if constexpr (Q == 9 && ST == ST_FP64 && limited && LAY != LAY_AB) return lds_for_blocks(2);
  return step_lds<Q, ST, LAY, CU>();
}

template <int Q, int ST, bool NS, int LAY>
static hipError_t fused_t(int cu, const KArgs &a, hipStream_t s) {
  const int sblocks = (int)((blocks_for(a.nspecial, 256) + 7) / 8 * 8);
  LBM_DISPATCH_CU(NS, cu, (k_fused<Q, ST, NS, LAY, CU><<<blocks_for(a.n, 256) + sblocks, 256, fused_lds<Q, ST, LAY, CU>(), s>>>(a, sblocks)))
  return hipGetLastError();
}

template <int Q, int ST, bool NS, int LAY>
static hipError_t side_t(const KArgs &a, hipStream_t s) {
  if (a.nspecial == 0) return hipSuccess;
  k_side<Q, ST, NS, LAY><<<blocks_for(a.nspecial, 64), 64, 0, s>>>(a);
  return hipGetLastError();
}

template <int Q, int ST, bool NS, int LAY>
static hipError_t init_t(const InitArgs &a, hipStream_t s) {
  k_init<Q, ST, NS, LAY><<<blocks_for(a.n, 256), 256, 0, s>>>(a);
  return hipGetLastError();
}

// The lattice count of the layout comes from the arguments: f is set only
// when both lattices are stored.
template <int Q, int ST, int LAY>
static hipError_t convert_t(bool to_storage, const KArgs &a, const void *from, void *to, double ref, hipStream_t s) {
  const unsigned g = blocks_for(a.n, 256);
  if (a.fsrc) {
    if (to_storage)
      k_convert<Q, ST, LAY, true, 2><<<g, 256, 0, s>>>(a, from, to, ref);
    else
      k_convert<Q, ST, LAY, false, 2><<<g, 256, 0, s>>>(a, from, to, ref);
  } else {
    if (to_storage)
      k_convert<Q, ST, LAY, true, 1><<<g, 256, 0, s>>>(a, from, to, ref);
    else
      k_convert<Q, ST, LAY, false, 1><<<g, 256, 0, s>>>(a, from, to, ref);
  }
  return hipGetLastError();
}

template <int Q, class R>
static hipError_t adjoint_t(const KArgs &a, const void *ln, void *lp, void *dq, hipStream_t s) {
  const R *lam_next = static_cast<const R *>(ln);
  R *lam_prev = static_cast<R *>(lp);
  double *dJdQ = static_cast<double *>(dq);
  if (!a.cls) {
    k_adjoint<Q, R><<<blocks_for(a.n, 256), 256, 0, s>>>(a, lam_next, lam_prev, dJdQ);
    return hipGetLastError();
  }
  k_adj_bulk<Q, R><<<blocks_for(a.n, 256), 256, 0, s>>>(a, lam_next, lam_prev, dJdQ);
  if (hipError_t e = hipGetLastError()) return e;
  if (a.nspecial > 0) k_adj_fix<Q, R><<<blocks_for(a.nspecial * Q, 256), 256, 0, s>>>(a, lam_next, lam_prev, dJdQ);
  return hipGetLastError();
}

// Launchers of one (lattice, storage) pair; LBM_INSTANTIATE below gives them
// plain names in one translation unit per pair (compiled in parallel).
template <int Q, int ST>
struct Launch {
  static hipError_t pass(bool ns, bool geom, int lay, int mode, int cu, const KArgs &a, hipStream_t s) {
    if (ns) {
      if (geom) return pass_lay<true, true>(lay, mode, cu, a, s);
      return pass_lay<true, false>(lay, mode, cu, a, s);
    }
    if (geom) return pass_lay<false, true>(lay, mode, cu, a, s);
    return pass_lay<false, false>(lay, mode, cu, a, s);
  }
  template <bool NS, bool GEOM>
  static hipError_t pass_lay(int lay, int mode, int cu, const KArgs &a, hipStream_t s) {
    LBM_DISPATCH_LAY(lay, (pass_t<Q, ST, NS, GEOM, LAY>(mode, cu, a, s)))
  }
  static hipError_t special(bool ns, int lay, int mode, int cu, const KArgs &a, hipStream_t s) {
    return ns ? special_lay<true>(lay, mode, cu, a, s) : special_lay<false>(lay, mode, cu, a, s);
  }
  template <bool NS>
  static hipError_t special_lay(int lay, int mode, int cu, const KArgs &a, hipStream_t s) {
    LBM_DISPATCH_LAY(lay, (special_t<Q, ST, NS, LAY>(mode, cu, a, s)))
  }
  static hipError_t fused(bool ns, int lay, int cu, const KArgs &a, hipStream_t s) {
    return ns ? fused_lay<true>(lay, cu, a, s) : fused_lay<false>(lay, cu, a, s);
  }
  template <bool NS>
  static hipError_t fused_lay(int lay, int cu, const KArgs &a, hipStream_t s) {
    LBM_DISPATCH_LAY(lay, (fused_t<Q, ST, NS, LAY>(cu, a, s)))
  }
  static hipError_t side(bool ns, int lay, const KArgs &a, hipStream_t s) {
    return ns ? side_lay<true>(lay, a, s) : side_lay<false>(lay, a, s);
  }
  template <bool NS>
  static hipError_t side_lay(int lay, const KArgs &a, hipStream_t s) {
    LBM_DISPATCH_LAY(lay, (side_t<Q, ST, NS, LAY>(a, s)))
  }
  static hipError_t init(bool ns, int lay, const InitArgs &a, hipStream_t s) {
    if (lay == LAY_AB) return ns ? init_t<Q, ST, true, LAY_AB>(a, s) : init_t<Q, ST, false, LAY_AB>(a, s);
    return ns ? init_t<Q, ST, true, LAY_AA_S>(a, s) : init_t<Q, ST, false, LAY_AA_S>(a, s);
  }
  static hipError_t convert(int lay, bool to_storage, const KArgs &a, const void *from, void *to, double ref,
                            hipStream_t s) {
    LBM_DISPATCH_LAY(lay, (convert_t<Q, ST, LAY>(to_storage, a, from, to, ref, s)))
  }
  // adjoint and seed depend on the arithmetic type only
  static hipError_t adjoint(const KArgs &a, const void *ln, void *lp, void *dq, hipStream_t s) {
    return adjoint_t<Q, typename StT<ST>::R>(a, ln, lp, dq, s);
  }
  static hipError_t seed(const double *H, const double *Ht, const uint8_t *cls, int64_t n, void *lam, void *dq,
                         double *sq, hipStream_t s) {
    using R = typename StT<ST>::R;
    k_seed<Q, R><<<blocks_for(n, 256), 256, 0, s>>>(H, Ht, cls, n, static_cast<R *>(lam), static_cast<double *>(dq),
                                                      sq);
    return hipGetLastError();
  }
};

#define LBM_INSTANTIATE(Q, ST, NAME)                                                                          \
  hipError_t NAME##_pass(bool ns, bool geom, int lay, int mode, int cu, const KArgs &a, hipStream_t s) {      \
    return Launch<Q, ST>::pass(ns, geom, lay, mode, cu, a, s);                                                \
  }                                                                                                           \
  hipError_t NAME##_special(bool ns, int lay, int mode, int cu, const KArgs &a, hipStream_t s) {              \
    return Launch<Q, ST>::special(ns, lay, mode, cu, a, s);                                                   \
  }                                                                                                           \
  hipError_t NAME##_fused(bool ns, int lay, int cu, const KArgs &a, hipStream_t s) {                          \
    return Launch<Q, ST>::fused(ns, lay, cu, a, s);                                                           \
  }                                                                                                           \
  hipError_t NAME##_side(bool ns, int lay, const KArgs &a, hipStream_t s) {                                   \
    return Launch<Q, ST>::side(ns, lay, a, s);                                                                \
  }                                                                                                           \
  hipError_t NAME##_init(bool ns, int lay, const InitArgs &a, hipStream_t s) {                                \
    return Launch<Q, ST>::init(ns, lay, a, s);                                                                \
  }                                                                                                           \
  hipError_t NAME##_convert(int lay, bool to_storage, const KArgs &a, const void *from, void *to, double ref,  \
                            hipStream_t s) {                                                                  \
    return Launch<Q, ST>::convert(lay, to_storage, a, from, to, ref, s);                                      \
  }                                                                                                           \
  hipError_t NAME##_adjoint(const KArgs &a, const void *ln, void *lp, void *dq, hipStream_t s) {              \
    return Launch<Q, ST>::adjoint(a, ln, lp, dq, s);                                                          \
  }                                                                                                           \
  hipError_t NAME##_seed(const double *H, const double *Ht, const uint8_t *cls, int64_t n, void *lam, void *dq, \
                         double *sq, hipStream_t s) {                                                         \
    return Launch<Q, ST>::seed(H, Ht, cls, n, lam, dq, sq, s);                                                \
  }

}  // namespace lbm
