// lbm_device.hpp -- device-side building blocks of the fused central-moment
// lattice Boltzmann step for gfx950: lattice tables, storage conversion, the
// factorised raw/central-moment transforms, relaxation and the wall rules.
//
// Populations live in registers in "chimera" slots: the population of
// velocity (ex, ey, ez) sits in slot (ex+1)*9 + (ey+1)*3 + (ez+1) (D3Q27) or
// (ex+1)*3 + (ey+1) (D2Q9).  Because every velocity component is in
// {-1, 0, 1} and every moment index in {0, 1, 2}, the central-moment transform
// T(u) = N(u) M of Sec. 2.1 / App. C is a tensor product of one 3x3 transform
// per axis; applying it axis by axis (z, then y, then x) turns the slot of
// velocity (ex, ey, ez) into the slot of central moment (m, n, o).  Relaxation
// then acts per slot, and the inverse per-axis transform (x, y, z) gives the
// post-collision populations.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// ---------------------------------------------------------------------------
// Lattices.  Direction order: D3Q27 as in Sec. 2.1; D2Q9 is its e_z = 0
// subset in the same order.
// ---------------------------------------------------------------------------
template <int Q>
struct Lat;

template <>
struct Lat<9> {
  static constexpr int D = 2;
  __host__ __device__ static constexpr int ex(int i) {
    constexpr int t[9] = {0, 1, 0, 1, -1, 0, 1, -1, -1};
    return t[i];
  }
  __host__ __device__ static constexpr int ey(int i) {
    constexpr int t[9] = {0, 0, 1, 1, 0, -1, -1, 1, -1};
    return t[i];
  }
  __host__ __device__ static constexpr int ez(int) { return 0; }
  __host__ __device__ static constexpr int opp(int i) {
    constexpr int t[9] = {0, 4, 5, 8, 1, 2, 7, 6, 3};
    return t[i];
  }
  // chimera slot of direction i
  __host__ __device__ static constexpr int slot(int i) { return (ex(i) + 1) * 3 + (ey(i) + 1); }
};

template <>
struct Lat<27> {
  static constexpr int D = 3;
  __host__ __device__ static constexpr int ex(int i) {
    constexpr int t[27] = {0, 1, 0, 0, 1, 1, 0, -1, 0, 0, 1, 1, -1, -1,
                           0, 0, 1, -1, -1, 0, -1, 1, 1, 1, -1, -1, -1};
    return t[i];
  }
  __host__ __device__ static constexpr int ey(int i) {
    constexpr int t[27] = {0, 0, 1, 0, 1, 0, 1, 0, -1, 0, -1, 0, 1, 0,
                           1, -1, 1, -1, 0, -1, 1, -1, 1, -1, 1, -1, -1};
    return t[i];
  }
  __host__ __device__ static constexpr int ez(int i) {
    constexpr int t[27] = {0, 0, 0, 1, 0, 1, 1, 0, 0, -1, 0, -1, 0, 1,
                           -1, 1, 1, 0, -1, -1, 1, 1, -1, -1, -1, 1, -1};
    return t[i];
  }
  __host__ __device__ static constexpr int opp(int i) {
    constexpr int t[27] = {0, 7, 8, 9, 17, 18, 19, 1, 2, 3, 12, 13, 10, 11,
                           15, 14, 26, 4, 5, 6, 23, 24, 25, 20, 21, 22, 16};
    return t[i];
  }
  __host__ __device__ static constexpr int slot(int i) {
    return (ex(i) + 1) * 9 + (ey(i) + 1) * 3 + (ez(i) + 1);
  }
};

// ---------------------------------------------------------------------------
// Storage <-> arithmetic conversion.  DEV storages keep g_i - w_i g_ref.
// ---------------------------------------------------------------------------
template <class S>
struct StoreT;
// Loads and stores of the population arrays.  Each stored element is written
// once per step and read back only in the next one, so stores bypass the
// caches (non-temporal); loads are ordinary (measured faster on MI355X).
// P: a pointer to the element type, generic or global address space.
template <>
struct StoreT<double> {
  template <class P>
  __device__ static double ld(P p) { return *p; }
  template <class P>
  __device__ static void st(P p, double v) { __builtin_nontemporal_store(v, p); }
};
template <>
struct StoreT<float> {
  template <class P>
  __device__ static float ld(P p) { return *p; }
  template <class P>
  __device__ static void st(P p, float v) { __builtin_nontemporal_store(v, p); }
};
template <>
struct StoreT<__half> {
  __device__ static float ld(const __half *p) { return ld_bits(*reinterpret_cast<const unsigned short *>(p)); }
  __device__ static float ld(const __attribute__((address_space(1))) __half *p) {
    return ld_bits(*reinterpret_cast<const __attribute__((address_space(1))) unsigned short *>(p));
  }
  __device__ static void st(__half *p, float v) {
    __builtin_nontemporal_store(st_bits(v), reinterpret_cast<unsigned short *>(p));
  }
  __device__ static void st(__attribute__((address_space(1))) __half *p, float v) {
    __builtin_nontemporal_store(st_bits(v), reinterpret_cast<__attribute__((address_space(1))) unsigned short *>(p));
  }
  __device__ static float ld_bits(unsigned short b) { return __half2float(__ushort_as_half(b)); }
  __device__ static unsigned short st_bits(float v) { return __half_as_ushort(__float2half_rn(v)); }
};

// Rest-equilibrium weight of direction i (product of 1-D weights 2/3, 1/6).
template <int Q, class R>
__host__ __device__ constexpr R weight(int i) {
  R w = R(1);
  int c[3] = {Lat<Q>::ex(i), Lat<Q>::ey(i), Lat<Q>::ez(i)};
  for (int d = 0; d < Lat<Q>::D; d++) w *= (c[d] == 0) ? R(2) / R(3) : R(1) / R(6);
  return w;
}

// ---------------------------------------------------------------------------
// One-axis central-moment transform of three populations at velocities
// -1, 0, +1 (a, b, c) about velocity u:
//   k0 = a + b + c,  k1 = sum (e - u) g,  k2 = sum (e - u)^2 g.
// ---------------------------------------------------------------------------
template <class R>
__device__ __forceinline__ void fwd3(R &a, R &b, R &c, R u) {
  const R k0 = a + b + c;
  const R d = c - a;
  const R k1 = d - u * k0;
  const R k2 = (c + a) - R(2) * u * d + u * u * k0;
  a = k0;
  b = k1;
  c = k2;
}

// Inverse of fwd3: (K0, K1, K2) -> populations at -1, 0, +1.
template <class R>
__device__ __forceinline__ void inv3(R &a, R &b, R &c, R u) {
  const R K0 = a, K1 = b, K2 = c;
  const R D = K1 + u * K0;                    // c - a
  const R S = K2 + R(2) * u * K1 + u * u * K0; // c + a
  a = R(0.5) * (S - D);
  b = K0 - S;
  c = R(0.5) * (S + D);
}

// In-place transform of the chimera slots to central moments (slot m,n[,o]).
template <int D, class R>
__device__ __forceinline__ void to_central(R *g, R ux, R uy, R uz) {
  if constexpr (D == 2) {
#pragma unroll
    for (int cx = 0; cx < 3; cx++) fwd3(g[cx * 3 + 0], g[cx * 3 + 1], g[cx * 3 + 2], uy);
#pragma unroll
    for (int my = 0; my < 3; my++) fwd3(g[0 + my], g[3 + my], g[6 + my], ux);
  } else {
#pragma unroll
    for (int cxy = 0; cxy < 9; cxy++) fwd3(g[cxy * 3 + 0], g[cxy * 3 + 1], g[cxy * 3 + 2], uz);
#pragma unroll
    for (int cx = 0; cx < 3; cx++)
#pragma unroll
      for (int mz = 0; mz < 3; mz++)
        fwd3(g[cx * 9 + 0 + mz], g[cx * 9 + 3 + mz], g[cx * 9 + 6 + mz], uy);
#pragma unroll
    for (int myz = 0; myz < 9; myz++) fwd3(g[myz], g[9 + myz], g[18 + myz], ux);
  }
}

// The same transform in two stages: raw moments first (k0 = a + b + c,
// k1 = c - a, k2 = c + a per axis), whose zeroth and first orders give rho and
// the momentum, then the shift of each axis to central moments about u
// (k1 - u k0, k2 - 2 u k1 + u^2 k0).  Both stages together cost what the
// direct transform costs, and the velocity needs no separate sums.
template <class R>
__device__ __forceinline__ void raw3(R &a, R &b, R &c) {
  const R k0 = a + b + c;
  const R k1 = c - a;
  const R k2 = c + a;
  a = k0;
  b = k1;
  c = k2;
}

template <class R>
__device__ __forceinline__ void shift3(R &a, R &b, R &c, R u) {
  const R k1 = b - u * a;
  const R k2 = c - R(2) * u * b + u * u * a;
  b = k1;
  c = k2;
}

template <int D, class R>
__device__ __forceinline__ void to_raw(R *g) {
  if constexpr (D == 2) {
#pragma unroll
    for (int cx = 0; cx < 3; cx++) raw3(g[cx * 3 + 0], g[cx * 3 + 1], g[cx * 3 + 2]);
#pragma unroll
    for (int my = 0; my < 3; my++) raw3(g[0 + my], g[3 + my], g[6 + my]);
  } else {
#pragma unroll
    for (int cxy = 0; cxy < 9; cxy++) raw3(g[cxy * 3 + 0], g[cxy * 3 + 1], g[cxy * 3 + 2]);
#pragma unroll
    for (int cx = 0; cx < 3; cx++)
#pragma unroll
      for (int mz = 0; mz < 3; mz++) raw3(g[cx * 9 + 0 + mz], g[cx * 9 + 3 + mz], g[cx * 9 + 6 + mz]);
#pragma unroll
    for (int myz = 0; myz < 9; myz++) raw3(g[myz], g[9 + myz], g[18 + myz]);
  }
}

template <int D, class R>
__device__ __forceinline__ void raw_to_central(R *g, R ux, R uy, R uz) {
  if constexpr (D == 2) {
#pragma unroll
    for (int mx = 0; mx < 3; mx++) shift3(g[mx * 3 + 0], g[mx * 3 + 1], g[mx * 3 + 2], uy);
#pragma unroll
    for (int my = 0; my < 3; my++) shift3(g[0 + my], g[3 + my], g[6 + my], ux);
  } else {
#pragma unroll
    for (int mxy = 0; mxy < 9; mxy++) shift3(g[mxy * 3 + 0], g[mxy * 3 + 1], g[mxy * 3 + 2], uz);
#pragma unroll
    for (int mx = 0; mx < 3; mx++)
#pragma unroll
      for (int mz = 0; mz < 3; mz++) shift3(g[mx * 9 + 0 + mz], g[mx * 9 + 3 + mz], g[mx * 9 + 6 + mz], uy);
#pragma unroll
    for (int myz = 0; myz < 9; myz++) shift3(g[myz], g[9 + myz], g[18 + myz], ux);
  }
}

// Chimera slots of the first-order moments 100, 010 (and 001).
template <int D>
__host__ __device__ constexpr int first_order_slot(int d) {
  return D == 2 ? (d == 0 ? 3 : 1) : (d == 0 ? 9 : (d == 1 ? 3 : 1));
}

template <int D, class R>
__device__ __forceinline__ void from_central(R *g, R ux, R uy, R uz) {
  if constexpr (D == 2) {
#pragma unroll
    for (int my = 0; my < 3; my++) inv3(g[0 + my], g[3 + my], g[6 + my], ux);
#pragma unroll
    for (int cx = 0; cx < 3; cx++) inv3(g[cx * 3 + 0], g[cx * 3 + 1], g[cx * 3 + 2], uy);
  } else {
#pragma unroll
    for (int myz = 0; myz < 9; myz++) inv3(g[myz], g[9 + myz], g[18 + myz], ux);
#pragma unroll
    for (int cx = 0; cx < 3; cx++)
#pragma unroll
      for (int mz = 0; mz < 3; mz++)
        inv3(g[cx * 9 + 0 + mz], g[cx * 9 + 3 + mz], g[cx * 9 + 6 + mz], uy);
#pragma unroll
    for (int cxy = 0; cxy < 9; cxy++) inv3(g[cxy * 3 + 0], g[cxy * 3 + 1], g[cxy * 3 + 2], uz);
  }
}

// Transposes of the one-axis transforms (reverse-mode of the collision).
// fwd3_T: (K0, K1, K2) -> the transpose of fwd3 applied to them.
template <class R>
__device__ __forceinline__ void fwd3_T(R &a, R &b, R &c, R u) {
  const R K0 = a, K1 = b, K2 = c;
  const R up = R(1) + u, um = R(1) - u;
  a = K0 - up * K1 + up * up * K2;
  b = K0 - u * K1 + u * u * K2;
  c = K0 + um * K1 + um * um * K2;
}

// inv3_T: transpose of inv3, populations (a, b, c) -> moment space.
template <class R>
__device__ __forceinline__ void inv3_T(R &a, R &b, R &c, R u) {
  const R A = a, B = b, C = c;
  a = R(0.5) * (u * u - u) * A + (R(1) - u * u) * B + R(0.5) * (u * u + u) * C;
  b = (u - R(0.5)) * A - R(2) * u * B + (u + R(0.5)) * C;
  c = R(0.5) * A - B + R(0.5) * C;
}

// T(u)^T: central-moment slots -> velocity slots (passes x, y, z).
template <int D, class R>
__device__ __forceinline__ void to_central_T(R *g, R ux, R uy, R uz) {
  if constexpr (D == 2) {
#pragma unroll
    for (int my = 0; my < 3; my++) fwd3_T(g[0 + my], g[3 + my], g[6 + my], ux);
#pragma unroll
    for (int cx = 0; cx < 3; cx++) fwd3_T(g[cx * 3 + 0], g[cx * 3 + 1], g[cx * 3 + 2], uy);
  } else {
#pragma unroll
    for (int myz = 0; myz < 9; myz++) fwd3_T(g[myz], g[9 + myz], g[18 + myz], ux);
#pragma unroll
    for (int cx = 0; cx < 3; cx++)
#pragma unroll
      for (int mz = 0; mz < 3; mz++)
        fwd3_T(g[cx * 9 + 0 + mz], g[cx * 9 + 3 + mz], g[cx * 9 + 6 + mz], uy);
#pragma unroll
    for (int cxy = 0; cxy < 9; cxy++) fwd3_T(g[cxy * 3 + 0], g[cxy * 3 + 1], g[cxy * 3 + 2], uz);
  }
}

// T(u)^-T: velocity slots -> central-moment slots (passes z, y, x).
template <int D, class R>
__device__ __forceinline__ void from_central_T(R *g, R ux, R uy, R uz) {
  if constexpr (D == 2) {
#pragma unroll
    for (int cx = 0; cx < 3; cx++) inv3_T(g[cx * 3 + 0], g[cx * 3 + 1], g[cx * 3 + 2], uy);
#pragma unroll
    for (int my = 0; my < 3; my++) inv3_T(g[0 + my], g[3 + my], g[6 + my], ux);
  } else {
#pragma unroll
    for (int cxy = 0; cxy < 9; cxy++) inv3_T(g[cxy * 3 + 0], g[cxy * 3 + 1], g[cxy * 3 + 2], uz);
#pragma unroll
    for (int cx = 0; cx < 3; cx++)
#pragma unroll
      for (int mz = 0; mz < 3; mz++)
        inv3_T(g[cx * 9 + 0 + mz], g[cx * 9 + 3 + mz], g[cx * 9 + 6 + mz], uy);
#pragma unroll
    for (int myz = 0; myz < 9; myz++) inv3_T(g[myz], g[9 + myz], g[18 + myz], ux);
  }
}

// Central-moment equilibrium factor of one moment index (0 -> 1, 1 -> 0,
// 2 -> cs^2 = 1/3): the equilibrium of moment (m,n,o) is psi * c(m) c(n) c(o),
// i.e. psi at 000, psi cs^2 at 200/020/002, psi cs^4 at 220/202/022,
// psi cs^6 at 222, zero elsewhere.
template <class R>
__host__ __device__ constexpr R ceq1(int m) {
  return m == 0 ? R(1) : (m == 1 ? R(0) : R(1) / R(3));
}

// Chimera slots of the diagonal second-order moments 200, 020 (and 002).
template <int D>
__host__ __device__ constexpr int diag2(int d) {
  return D == 2 ? (d == 0 ? 6 : 2) : (d == 0 ? 18 : (d == 1 ? 6 : 2));
}

// Trace of the diagonal second-order block (central moments or cumulants).
template <int D, class R>
__device__ __forceinline__ R trace2(const R *K) {
  R t = K[diag2<D>(0)] + K[diag2<D>(1)];
  if constexpr (D == 3) t += K[diag2<D>(2)];
  return t;
}

// Separate rate of that trace (bulk viscosity).  After the diagonal
// relaxation at s of 200 (= 020 = 002), adding db (teq / D - t / D) to each
// diagonal moment, with t the pre-collision trace, teq its equilibrium and
// db = s_bulk - s_200, moves the trace at s_bulk and leaves the differences
// of the diagonal moments (the deviator) as the diagonal rate left them.
template <int D, class R>
__device__ __forceinline__ void bulk_shift(R *K, R t_pre, R teq, R db) {
  const R d = db * (teq - t_pre) * (R(1) / R(D));
  K[diag2<D>(0)] += d;
  K[diag2<D>(1)] += d;
  if constexpr (D == 3) K[diag2<D>(2)] += d;
}

// Moments whose rate the caller guarantees to be exactly 1 (compile time),
// by total order m + n + o: RATE1_NONE none; RATE1_ORD3 every order >= 3 (the
// hydrodynamic preset); RATE1_EVEN every even order, 0 included (CM-TRT);
// RATE1_ORD2 order 0 and every order >= 2 (CM-1st).  Such a moment takes its
// equilibrium directly, so its pre-collision value is never used and the
// forward transform drops the arithmetic that only feeds it.
enum : int { RATE1_NONE = 0, RATE1_ORD3 = 1, RATE1_EVEN = 2, RATE1_ORD2 = 3 };
__host__ __device__ constexpr bool rate_is_one(int pattern, int order) {
  return pattern == RATE1_ORD3 ? order >= 3
         : pattern == RATE1_EVEN ? order % 2 == 0
         : pattern == RATE1_ORD2 ? order != 1
                                 : false;
}

// Relaxation toward the central-moment equilibrium, in place on the central
// moments K (chimera order), rates s (chimera order).  psi is the conserved
// zeroth moment used by the equilibrium; src the source of App. D (0 if none).
// TR: the trace of the second-order block relaxes at s_200 + db.  ONE: a
// RATE1_* pattern of rates known to be 1.
template <int D, class R, bool TR = false, int ONE = RATE1_NONE>
__device__ __forceinline__ void relax(R *K, const R *s, R psi, R src, R db = R(0)) {
  constexpr int NQ = D == 2 ? 9 : 27;
  R t_pre = R(0);
  if constexpr (TR) t_pre = trace2<D, R>(K);
#pragma unroll
  for (int k = 0; k < NQ; k++) {
    const int m = D == 2 ? k / 3 : k / 9;
    const int n = D == 2 ? k % 3 : (k / 3) % 3;
    const int o = D == 2 ? 0 : k % 3;
    const R c = ceq1<R>(m) * ceq1<R>(n) * ceq1<R>(o);
    if (rate_is_one(ONE, m + n + o))
      K[k] = psi * c;
    else if (c == R(0))
      K[k] = K[k] - s[k] * K[k];
    else
      K[k] = K[k] + s[k] * (psi * c - K[k]);
  }
  if constexpr (TR) bulk_shift<D, R>(K, t_pre, psi * (R(D) / R(3)), db);
  K[0] += (R(1) - R(0.5) * s[0]) * src;
}

// Full central-moment collision of one lattice (chimera slots in, chimera
// slots out): g* = T(u)^-1 [Y~ + S (Y~eq - Y~)].
template <int D, class R, bool TR = false, int ONE = RATE1_NONE>
__device__ __forceinline__ void collide(R *g, const R *s, R ux, R uy, R uz, R src, R db = R(0)) {
  to_central<D, R>(g, ux, uy, uz);
  const R psi = g[0] + R(0.5) * src;
  relax<D, R, TR, ONE>(g, s, psi, src, db);
  from_central<D, R>(g, ux, uy, uz);
}

// The same collision for the hydrodynamic lattice, whose velocity comes from
// its own moments: rho and u are read off the raw moments, which are then
// shifted to central moments (source-free).
template <int D, class R, bool TR = false, int ONE = RATE1_NONE>
__device__ __forceinline__ void collide_own_u(R *g, const R *s, R &rho, R &ux, R &uy, R &uz, R db = R(0)) {
  to_raw<D, R>(g);
  rho = g[0];
  const R inv = R(1) / rho;
  ux = g[first_order_slot<D>(0)] * inv;
  uy = g[first_order_slot<D>(1)] * inv;
  uz = D == 3 ? g[first_order_slot<D>(2)] * inv : R(0);
  raw_to_central<D, R>(g, ux, uy, uz);
  relax<D, R, TR, ONE>(g, s, g[0], R(0), db);
  from_central<D, R>(g, ux, uy, uz);
}

// ---------------------------------------------------------------------------
// Cumulant collision (Sec. 2.1.1, Eqs. hydro_cu_collision and
// H_cu_collision, with the source of App. D).  The zeroth cumulant is the sum
// of the populations; the others are the cumulants of the normalised
// distribution, computed here from its central moments about u (first-order
// cumulants are then mean - u, higher ones do not depend on the shift).  With
// mu = normalised central moments and the multi-index identity
// d_j M = M d_j log M, for n = n' + e_j:
//   mu_n = sum_{k <= n'} B(n', k) mu_{n'-k} c_{k+e_j},  B = prod_d binom(n'_d, k_d),
// solved for c_n in increasing total order (forward) or read as it stands
// (inverse).  The equilibrium about u: 0 at first order, cs^2 at 200/020/002,
// 0 elsewhere.
// ---------------------------------------------------------------------------
template <int D>
__host__ __device__ constexpr int cm_x(int k) { return D == 2 ? k / 3 : k / 9; }
template <int D>
__host__ __device__ constexpr int cm_y(int k) { return D == 2 ? k % 3 : (k / 3) % 3; }
template <int D>
__host__ __device__ constexpr int cm_z(int k) { return D == 2 ? 0 : k % 3; }
template <int D>
__host__ __device__ constexpr int cm_slot(int m, int n, int o) { return D == 2 ? m * 3 + n : m * 9 + n * 3 + o; }
__host__ __device__ constexpr int binom2(int n, int k) { return (n == 2 && k == 1) ? 2 : 1; }

template <int D>
__host__ __device__ constexpr int cm_order(int k) { return cm_x<D>(k) + cm_y<D>(k) + cm_z<D>(k); }
// Equilibrium cumulant about u of index k > 0: cs^2 at 200/020/002, else 0.
template <int D>
__host__ __device__ constexpr bool cu_pure2(int k) {
  return cm_order<D>(k) == 2 && (cm_x<D>(k) == 2 || cm_y<D>(k) == 2 || cm_z<D>(k) == 2);
}
// With every cumulant above order K relaxed at rate 1 (K > 0), the post-
// collision cumulant of index k is its equilibrium; true where that is zero.
template <int D, int K>
__host__ __device__ constexpr bool cu_post_zero(int k) {
  return K > 0 && cm_order<D>(k) > K && !cu_pure2<D>(k);
}

// FWD: c[k] (k > 0) from mu; else mu[k] (k > 0) from c.  mu[0] = 1.
// K > 0: every cumulant above order K relaxes at rate 1, so the forward pass
// stops at order K and the inverse pass drops the terms whose cumulant is
// then zero (each such term would add a signed zero).
template <int D, bool FWD, class R, int K = 0>
__device__ __forceinline__ void cumulant_recursion(R *mu, R *c) {
  constexpr int NQ = D == 2 ? 9 : 27;
#pragma unroll
  for (int t = 1; t <= 2 * D; t++) {
    if (FWD && K > 0 && t > K) break;
#pragma unroll
    for (int k = 1; k < NQ; k++) {
      const int m = cm_x<D>(k), n = cm_y<D>(k), o = cm_z<D>(k);
      if (m + n + o != t) continue;
      const int jx = m > 0 ? 1 : 0, jy = (!jx && n > 0) ? 1 : 0, jz = (!jx && !jy) ? 1 : 0;
      const int pm = m - jx, pn = n - jy, po = o - jz;
      R acc = FWD ? mu[k] : R(0);
#pragma unroll
      for (int a = 0; a < 3; a++)
#pragma unroll
        for (int b = 0; b < 3; b++)
#pragma unroll
          for (int e = 0; e < (D == 3 ? 3 : 1); e++) {
            if (a > pm || b > pn || e > po) continue;
            if (FWD && a == pm && b == pn && e == po) continue;
            const int ci = cm_slot<D>(a + jx, b + jy, e + jz);
            if (!FWD && cu_post_zero<D, K>(ci)) continue;
            const R B = R(binom2(pm, a) * binom2(pn, b) * binom2(po, e));
            const R term = B * mu[cm_slot<D>(pm - a, pn - b, po - e)] * c[ci];
            acc = FWD ? acc - term : acc + term;
          }
      if (FWD)
        c[k] = acc;
      else
        mu[k] = acc;
    }
  }
}

// K > 0: the rates of every cumulant above order K are 1 (the caller checks),
// which those cumulants then reach exactly; K = 0: no assumption.  TR: the
// trace of the second-order cumulants relaxes at s_200 + db (bulk_shift).
template <int D, class R, int K = 0, bool TR = false>
__device__ __forceinline__ void collide_cu(R *g, const R *s, R ux, R uy, R uz, R src, R db = R(0)) {
  constexpr int NQ = D == 2 ? 9 : 27;
  to_central<D, R>(g, ux, uy, uz);
  const R k0 = g[0];
  const R inv = R(1) / k0;
  g[0] = R(1);
#pragma unroll
  for (int k = 1; k < NQ; k++) g[k] *= inv;
  R c[NQ];
  c[0] = k0;
  cumulant_recursion<D, true, R, K>(g, c);
  R t_pre = R(0);
  if constexpr (TR) t_pre = trace2<D, R>(c);
#pragma unroll
  for (int k = 1; k < NQ; k++) {
    const R eq = cu_pure2<D>(k) ? R(1) / R(3) : R(0);
    if (K > 0 && cm_order<D>(k) > K)
      c[k] = eq;
    else
      c[k] = c[k] + s[k] * (eq - c[k]);
  }
  if constexpr (TR) bulk_shift<D, R>(c, t_pre, R(D) / R(3), db);
  const R psi = k0 + R(0.5) * src;
  const R c0 = k0 + s[0] * (psi - k0) + (R(1) - R(0.5) * s[0]) * src;
  cumulant_recursion<D, false, R, K>(g, c);
  g[0] = c0;
#pragma unroll
  for (int k = 1; k < NQ; k++) g[k] *= c0;
  from_central<D, R>(g, ux, uy, uz);
}

// Reverse-mode of collide() for the advection-diffusion lattice, whose
// collision is affine in (g, src) for a prescribed u:
//   g* = A g + b src,  A = T^-1 [(1 - S) T + S ceq 1^T],
//   b = T^-1 [S ceq / 2 + (1 - s_000/2) e_000].
// In place: lam (velocity slots, adjoint of g*) -> A^T lam; returns b^T lam.
// With mu = T^-T lam:  A^T lam = T^T [(1 - S) mu + e_000 (ceq . S mu)].
template <int D, class R>
__device__ __forceinline__ R collide_adjoint(R *g, const R *s, R ux, R uy, R uz) {
  constexpr int NQ = D == 2 ? 9 : 27;
  from_central_T<D, R>(g, ux, uy, uz);
  R csm = 0;
#pragma unroll
  for (int k = 0; k < NQ; k++) {
    const int m = D == 2 ? k / 3 : k / 9;
    const int n = D == 2 ? k % 3 : (k / 3) % 3;
    const int o = D == 2 ? 0 : k % 3;
    const R c = ceq1<R>(m) * ceq1<R>(n) * ceq1<R>(o);
    if (c != R(0)) csm += c * s[k] * g[k];
  }
  const R dq = R(0.5) * csm + (R(1) - R(0.5) * s[0]) * g[0];
#pragma unroll
  for (int k = 0; k < NQ; k++) g[k] = (R(1) - s[k]) * g[k];
  g[0] += csm;
  to_central_T<D, R>(g, ux, uy, uz);
  return dq;
}

// Discrete equilibrium of direction i in product form:
// psi * prod_d phi(e_d, u_d), phi(0, u) = 2/3 - u^2, phi(+-1, u) = (1/3 + u^2 +- u)/2.
template <class R>
__device__ __forceinline__ R phi1(int c, R u) {
  return c == 0 ? (R(2) / R(3) - u * u) : R(0.5) * (R(1) / R(3) + u * u + R(c) * u);
}

template <int Q, class R>
__device__ __forceinline__ R geq_dir(int i, R psi, R ux, R uy, R uz) {
  R v = psi * phi1<R>(Lat<Q>::ex(i), ux) * phi1<R>(Lat<Q>::ey(i), uy);
  if constexpr (Lat<Q>::D == 3) v *= phi1<R>(Lat<Q>::ez(i), uz);
  return v;
}

// Wall rules of Sec. 3.  q in (0, 1]; gb_i, gb_o: post-collision values of
// the boundary node in the wall direction i and the opposite one; gf_i: the
// post-collision value of x_f = x_b - e_i in direction i.
template <class R>
__device__ __forceinline__ R wall_ibb(R q, R gb_i, R gb_o, R gf_i) {
  if (q <= R(0.5)) return R(2) * q * gb_i + (R(1) - R(2) * q) * gf_i;
  return (gb_i + (R(2) * q - R(1)) * gb_o) / (R(2) * q);
}

template <class R>
__device__ __forceinline__ R wall_iabb(R q, R gb_i, R gb_o, R gf_i, R geq_i) {
  if (q <= R(0.5)) return -(R(2) * q * gb_i + (R(1) - R(2) * q) * gf_i) + R(2) * geq_i;
  return (-gb_i + (R(2) * q - R(1)) * gb_o + R(2) * geq_i) / (R(2) * q);
}

}  // namespace lbm
