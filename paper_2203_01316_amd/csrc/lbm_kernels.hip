// lbm_kernels.hip -- fused central-moment stream-and-collide kernels for
// gfx950 (one node per thread, structure-of-arrays populations, pull
// streaming between two arrays).
//
// Work split per step:
//   k_bulk     every node of class CLS_BULK (no cut link, not EQ/OUTLET):
//              periodic pull of Q populations per lattice, velocity from f (or
//              prescribed), central-moment collision in registers, store.
//   k_special  one thread per boundary node: pull, wall links (BB/IBB on f,
//              ABB/IABB on h), outlet copy, EQ reset, then the same collision.
// Both read the stored post-collision state of step t-1 and write step t into
// the other array; they touch disjoint nodes, so they can run back to back.
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

template <int Q, int ST>
__device__ __forceinline__ typename StT<ST>::R ldp(const void *base, int i, int64_t n, int64_t m,
                                                   typename StT<ST>::R ref) {
  using T = StT<ST>;
  using R = typename T::R;
  const typename T::S *p = static_cast<const typename T::S *>(base) + (int64_t)i * n + m;
  R v = StoreT<typename T::S>::ld(p);
  if constexpr (T::DEV) v += weight<Q, R>(i) * ref;
  return v;
}

template <int Q, int ST>
__device__ __forceinline__ void stp(void *base, int i, int64_t n, int64_t m, typename StT<ST>::R v,
                                    typename StT<ST>::R ref) {
  using T = StT<ST>;
  if constexpr (T::DEV) v -= weight<Q, typename T::R>(i) * ref;
  typename T::S *p = static_cast<typename T::S *>(base) + (int64_t)i * n + m;
  StoreT<typename T::S>::st(p, v);
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

__device__ __forceinline__ int wrapm(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

template <int Q>
__device__ __forceinline__ int64_t shifted(const KArgs &a, int x, int y, int z, int i, int sign) {
  const int xs = wrapm(x + sign * Lat<Q>::ex(i), a.nx);
  const int ys = wrapm(y + sign * Lat<Q>::ey(i), a.ny);
  const int zs = wrapm(z + sign * Lat<Q>::ez(i), a.nz);
  return xs + (int64_t)a.nx * (ys + (int64_t)a.ny * zs);
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

// Epilogue shared by the bulk and the boundary kernels: pre-collision
// populations f, h (direction order) of node m -> collide and store, or
// write them / their moments out.
template <int Q, int ST, bool NS, int MODE>
__device__ __forceinline__ void finish_node(const KArgs &a, int64_t m, typename StT<ST>::R *f,
                                            typename StT<ST>::R *h) {
  using R = typename StT<ST>::R;
  constexpr int D = Lat<Q>::D;
  R rho = 0, ux, uy, uz;
  if constexpr (NS)
    velocity_dir<Q, R>(f, rho, ux, uy, uz);
  else
    prescribed_u<Q, R>(a, m, ux, uy, uz);
  const R src = a.src ? static_cast<const R *>(a.src)[m] : R(0);
  if constexpr (MODE == MODE_STEP) {
    R g[Q];
    if constexpr (NS) {
#pragma unroll
      for (int i = 0; i < Q; i++) g[Lat<Q>::slot(i)] = f[i];
      collide<D, R>(g, rates<R>(a, true), ux, uy, uz, R(0));
#pragma unroll
      for (int i = 0; i < Q; i++) stp<Q, ST>(a.fdst, i, a.n, m, g[Lat<Q>::slot(i)], R(a.fref));
    }
#pragma unroll
    for (int i = 0; i < Q; i++) g[Lat<Q>::slot(i)] = h[i];
    collide<D, R>(g, rates<R>(a, false), ux, uy, uz, src);
#pragma unroll
    for (int i = 0; i < Q; i++) stp<Q, ST>(a.hdst, i, a.n, m, g[Lat<Q>::slot(i)], R(a.href));
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
template <int Q, int ST, bool NS, int MODE>
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
// Bulk nodes: one thread per node, 256 nodes (4 wavefronts) per block.
// ---------------------------------------------------------------------------
// Workgroups of one dispatch go round-robin to the 8 XCDs (block b runs on
// XCD b % 8), and each XCD has its own L2.  Mapping block b to tile
// (b % 8) * per + b / 8 hands every XCD one contiguous slab of the lattice, so
// the cache lines that neighbouring tiles share through the +-1 shifts of the
// pull stay in one L2 instead of being fetched once per XCD.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t nb) {
  const int64_t per = nb / 8;
  return b < per * 8 ? (b % 8) * per + b / 8 : b;
}

template <int Q, int ST, bool NS, bool GEOM, int MODE, bool BITS = false>
__device__ __forceinline__ void bulk_node(const KArgs &a, int64_t m) {
  using R = typename StT<ST>::R;
  if (m >= a.n) return;
  if constexpr (BITS) {
    // step kernel: solid and boundary nodes are skipped (1 bit per node)
    if ((a.skip[m >> 5] >> (m & 31)) & 1u) return;
  } else if constexpr (GEOM) {
    const uint8_t c = a.cls[m];
    if (c == CLS_SPECIAL) return;
    if (c == CLS_SOLID) {
      solid_node<Q, ST, NS, MODE>(a, m);
      return;
    }
  }
  const int x = (int)(m % a.nx);
  const int64_t r = m / a.nx;
  const int y = (int)(r % a.ny);
  const int z = (int)(r / a.ny);
  // source coordinate of a population moving with velocity component c
  // (index c + 1): x - c with periodic wrap
  const int xs[3] = {x + 1 == a.nx ? 0 : x + 1, x, x == 0 ? a.nx - 1 : x - 1};
  const int ys[3] = {y + 1 == a.ny ? 0 : y + 1, y, y == 0 ? a.ny - 1 : y - 1};
  const int zs[3] = {z + 1 == a.nz ? 0 : z + 1, z, z == 0 ? a.nz - 1 : z - 1};
  R f[Q], h[Q];
#pragma unroll
  for (int i = 0; i < Q; i++) {
    const int64_t src = xs[Lat<Q>::ex(i) + 1] +
                        (int64_t)a.nx * (ys[Lat<Q>::ey(i) + 1] + (int64_t)a.ny * zs[Lat<Q>::ez(i) + 1]);
    if constexpr (NS) f[i] = ldp<Q, ST>(a.fsrc, i, a.n, src, R(a.fref));
    h[i] = ldp<Q, ST>(a.hsrc, i, a.n, src, R(a.href));
  }
  finish_node<Q, ST, NS, MODE>(a, m, f, h);
}

template <int Q, int ST, bool NS, bool GEOM, int MODE>
__global__ void __launch_bounds__(256) k_bulk(const KArgs a) {
  const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
  bulk_node<Q, ST, NS, GEOM, MODE>(a, tile * 256 + threadIdx.x);
}

// ---------------------------------------------------------------------------
// Boundary nodes
// ---------------------------------------------------------------------------
// Pulled populations of node m plus the wall links in mask (links stored from
// lb), direction order.  flux (optional) receives h_opp(x_b, t) - h*_i(x_b, t-1)
// per link.
template <int Q, int ST, bool NS>
__device__ __forceinline__ void pull_links(const KArgs &a, int64_t m, int32_t lb, uint32_t mask,
                                           typename StT<ST>::R *f, typename StT<ST>::R *h,
                                           double *flux) {
  using R = typename StT<ST>::R;
  const int x = (int)(m % a.nx);
  const int64_t r = m / a.nx;
  const int y = (int)(r % a.ny);
  const int z = (int)(r / a.ny);
  const R fref = R(a.fref), href = R(a.href);
#pragma unroll
  for (int i = 0; i < Q; i++) {
    const int64_t s = shifted<Q>(a, x, y, z, i, -1);
    if constexpr (NS) f[i] = ldp<Q, ST>(a.fsrc, i, a.n, s, fref);
    h[i] = ldp<Q, ST>(a.hsrc, i, a.n, s, href);
  }
  if (mask == 0) return;
  // velocity of the boundary node for the wall equilibrium: post-collision f
  // of step t-1 (momentum over density), or the prescribed velocity
  R ux, uy, uz;
  if constexpr (NS) {
    R fb[Q], rho;
#pragma unroll
    for (int i = 0; i < Q; i++) fb[i] = ldp<Q, ST>(a.fsrc, i, a.n, m, fref);
    velocity_dir<Q, R>(fb, rho, ux, uy, uz);
  } else {
    prescribed_u<Q, R>(a, m, ux, uy, uz);
  }
#pragma unroll
  for (int i = 1; i < Q; i++) {
    if (!((mask >> i) & 1u)) continue;
    const int o = Lat<Q>::opp(i);
    const int32_t l = lb + __popc(mask & ((1u << i) - 1u));
    const DevLink lk = a.links[l];
    const DevGroup &G = a.groups[lk.group];
    const int64_t xf = shifted<Q>(a, x, y, z, i, -1);
    if constexpr (NS) {
      const R qf = (G.f_scheme == 0 || lk.xf_solid) ? R(0.5) : R(lk.q);
      f[o] = wall_ibb<R>(qf, ldp<Q, ST>(a.fsrc, i, a.n, m, fref), ldp<Q, ST>(a.fsrc, o, a.n, m, fref),
                         ldp<Q, ST>(a.fsrc, i, a.n, xf, fref));
    }
    const R qh = (G.h_scheme == 0 || lk.xf_solid) ? R(0.5) : R(lk.q);
    const R hbi = ldp<Q, ST>(a.hsrc, i, a.n, m, href);
    const R geq = geq_dir<Q, R>(i, R(G.H_w), ux, uy, uz);
    h[o] = wall_iabb<R>(qh, hbi, ldp<Q, ST>(a.hsrc, o, a.n, m, href),
                        ldp<Q, ST>(a.hsrc, i, a.n, xf, href), geq);
    if (flux) flux[l] = double(h[o]) - double(hbi);
  }
}

template <int Q, int ST, bool NS, int MODE>
__device__ __forceinline__ void special_node(const KArgs &a, int64_t t) {
  using R = typename StT<ST>::R;
  if (t >= a.nspecial) return;
  const DevSpecial sp = a.special[t];
  const int64_t m = sp.node;
  double *flux = MODE == MODE_MACRO ? a.link_flux : nullptr;
  R f[Q], h[Q];
  if (sp.type == NODE_EQ) {
    if (flux) pull_links<Q, ST, NS>(a, m, sp.lb, sp.mask, f, h, flux);
    const DevGroup &G = a.groups[sp.group];
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
  } else {
    pull_links<Q, ST, NS>(a, m, sp.lb, sp.mask, f, h, flux);
    if (sp.type == NODE_OUTLET) {
      const int x = (int)(m % a.nx);
      const int64_t up = x == 0 ? m + a.nx - 1 : m - 1;
      R fu[Q], hu[Q];
      pull_links<Q, ST, NS>(a, up, sp.ub, sp.umask, fu, hu, nullptr);
#pragma unroll
      for (int i = 0; i < Q; i++) {
        if (Lat<Q>::ex(i) < 0) {
          if constexpr (NS) f[i] = fu[i];
          h[i] = hu[i];
        }
      }
    }
  }
  finish_node<Q, ST, NS, MODE>(a, m, f, h);
}

template <int Q, int ST, bool NS, int MODE>
__global__ void __launch_bounds__(64) k_special(const KArgs a) {
  special_node<Q, ST, NS, MODE>(a, (int64_t)blockIdx.x * 64 + threadIdx.x);
}

// One launch per step with geometry (D2Q9): the first `sblocks` blocks (a
// multiple of 8, so the XCD of a bulk block is unchanged) take the boundary
// nodes, whose long chains of dependent loads then overlap the bulk stream
// instead of running after it.
template <int Q, int ST, bool NS>
__global__ void __launch_bounds__(256) k_fused(const KArgs a, int sblocks) {
  if ((int)blockIdx.x < sblocks) {
    special_node<Q, ST, NS, MODE_STEP>(a, (int64_t)blockIdx.x * 256 + threadIdx.x);
    return;
  }
  const int64_t tile = xcd_tile(blockIdx.x - sblocks, gridDim.x - sblocks);
  bulk_node<Q, ST, NS, true, MODE_STEP, true>(a, tile * 256 + threadIdx.x);
}

// ---------------------------------------------------------------------------
// Discrete adjoint of the advection-diffusion step (no geometry): node y
// gathers lam_next_i(y + e_i) (transpose of the pull), applies the transposed
// collision of node y and writes lam_prev(y); dJdQ(y) += b^T lam.
// ---------------------------------------------------------------------------
template <int Q, class R>
__global__ void __launch_bounds__(256) k_adjoint(const KArgs a, const R *lam_next, R *lam_prev, double *dJdQ) {
  constexpr int D = Lat<Q>::D;
  const int64_t m = xcd_tile(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
  if (m >= a.n) return;
  const int x = (int)(m % a.nx);
  const int64_t r = m / a.nx;
  const int y = (int)(r % a.ny);
  const int z = (int)(r / a.ny);
  // destination coordinate of a population moving with component c: x + c
  const int xd[3] = {x == 0 ? a.nx - 1 : x - 1, x, x + 1 == a.nx ? 0 : x + 1};
  const int yd[3] = {y == 0 ? a.ny - 1 : y - 1, y, y + 1 == a.ny ? 0 : y + 1};
  const int zd[3] = {z == 0 ? a.nz - 1 : z - 1, z, z + 1 == a.nz ? 0 : z + 1};
  R g[Q];
#pragma unroll
  for (int i = 0; i < Q; i++) {
    const int64_t d = xd[Lat<Q>::ex(i) + 1] +
                      (int64_t)a.nx * (yd[Lat<Q>::ey(i) + 1] + (int64_t)a.ny * zd[Lat<Q>::ez(i) + 1]);
    g[Lat<Q>::slot(i)] = __builtin_nontemporal_load(lam_next + (int64_t)i * a.n + d);
  }
  R ux, uy, uz;
  prescribed_u<Q, R>(a, m, ux, uy, uz);
  const R dq = collide_adjoint<D, R>(g, rates<R>(a, false), ux, uy, uz);
#pragma unroll
  for (int i = 0; i < Q; i++) __builtin_nontemporal_store(g[Lat<Q>::slot(i)], lam_prev + (int64_t)i * a.n + m);
  if (dJdQ) dJdQ[m] += double(dq);
}

// Objective J = 1/2 sum (H - H*)^2 on the canonical state: H from a macro
// pass (FP64 scratch).  Seeds lam = dJ/dpre (every direction H - H*), sets
// dJdQ = (H - H*)/2 (Q enters H as Q/2) and leaves (H - H*)^2 in sq.
template <int Q, class R>
__global__ void __launch_bounds__(256) k_seed(const double *H, const double *Ht, int64_t n, R *lam, double *dJdQ,
                                              double *sq) {
  const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (m >= n) return;
  const double d = H[m] - Ht[m];
#pragma unroll
  for (int i = 0; i < Q; i++) lam[(int64_t)i * n + m] = R(d);
  dJdQ[m] = 0.5 * d;
  sq[m] = d * d;
}

// ---------------------------------------------------------------------------
// Initial state: g*_i(x) = g^eq_i(fields at x + e_i) in FP64, then stored.
// ---------------------------------------------------------------------------
template <int Q, int ST, bool NS>
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
    if constexpr (NS) {
      const double rho = a.rho ? a.rho[s] : 1.0;
      stp<Q, ST>(a.fdst, i, a.n, m, R(geq_dir<Q, double>(i, rho, ux, uy, uz)), R(a.fref));
    }
    stp<Q, ST>(a.hdst, i, a.n, m, R(geq_dir<Q, double>(i, a.H[s], ux, uy, uz)), R(a.href));
  }
}

// FP64 [Q][n] <-> storage.
// FP64 [Q][n] <-> storage.  Reading out, solid nodes (cls) report zeros.
template <int Q, int ST, bool TO_STORAGE>
__global__ void __launch_bounds__(256) k_convert(const void *from, void *to, int64_t n, double ref,
                                                 const uint8_t *cls) {
  using R = typename StT<ST>::R;
  const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (m >= n) return;
  const bool solid = cls && cls[m] == CLS_SOLID;
#pragma unroll
  for (int i = 0; i < Q; i++) {
    if constexpr (TO_STORAGE)
      stp<Q, ST>(to, i, n, m, R(static_cast<const double *>(from)[i * n + m]), R(ref));
    else
      static_cast<double *>(to)[i * n + m] = solid ? 0.0 : double(ldp<Q, ST>(from, i, n, m, R(ref)));
  }
}

// ---------------------------------------------------------------------------
// Deterministic FP64 reductions (fixed grid, fixed tree order).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double v, double *sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (t < w) sh[t] += sh[t + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// partials[b] = (sum rho, sum H) over a fixed strided subset of nodes
__global__ void __launch_bounds__(256) k_sum_partials(const double *rho, const double *H, int64_t n,
                                                      double *partials) {
  __shared__ double sh[256];
  double sr = 0.0, sH = 0.0;
  for (int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x; m < n; m += (int64_t)gridDim.x * 256) {
    sr += rho ? rho[m] : 0.0;
    sH += H[m];
  }
  sr = block_sum(sr, sh);
  sH = block_sum(sH, sh);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = sr;
    partials[2 * blockIdx.x + 1] = sH;
  }
}

__global__ void __launch_bounds__(256) k_sum_final(const double *partials, int np, double *out) {
  __shared__ double sh[256];
  double sr = 0.0, sH = 0.0;
  for (int b = threadIdx.x; b < np; b += 256) {
    sr += partials[2 * b];
    sH += partials[2 * b + 1];
  }
  sr = block_sum(sr, sh);
  sH = block_sum(sH, sh);
  if (threadIdx.x == 0) {
    out[0] = sr;
    out[1] = sH;
  }
}

// out[2] = sum of link_flux over the links of one group
__global__ void __launch_bounds__(256) k_group_flux(const double *flux, const DevLink *links,
                                                    int64_t nl, int group, double *out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t l = threadIdx.x; l < nl; l += 256)
    if (links[l].group == group) s += flux[l];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[2] = s;
}

// out[3 + j] = sum over y, z of qx at x = cols[j]; one block per column
__global__ void __launch_bounds__(256) k_column_sum(const double *qx, int nx, int ny, int nz,
                                                    const int32_t *cols, double *out) {
  __shared__ double sh[256];
  const int X = cols[blockIdx.x];
  double s = 0.0;
  const int64_t nyz = (int64_t)ny * nz;
  for (int64_t k = threadIdx.x; k < nyz; k += 256) s += qx[X + (int64_t)nx * k];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[3 + blockIdx.x] = s;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

#define LBM_DISPATCH_ST(ST_VAL, CALL) \
  switch (ST_VAL) {                   \
    case ST_FP64: {                   \
      constexpr int ST = ST_FP64;     \
      return CALL;                    \
    }                                 \
    case ST_FP32: {                   \
      constexpr int ST = ST_FP32;     \
      return CALL;                    \
    }                                 \
    case ST_FP32_DEV: {               \
      constexpr int ST = ST_FP32_DEV; \
      return CALL;                    \
    }                                 \
    case ST_FP16_DEV: {               \
      constexpr int ST = ST_FP16_DEV; \
      return CALL;                    \
    }                                 \
    default:                          \
      return hipErrorInvalidValue;    \
  }

template <int Q, int ST, bool NS, bool GEOM>
static hipError_t pass_t(int mode, const KArgs &a, hipStream_t s) {
  const unsigned g = blocks_for(a.n, 256);
  if (mode == MODE_STEP)
    k_bulk<Q, ST, NS, GEOM, MODE_STEP><<<g, 256, 0, s>>>(a);
  else if (mode == MODE_PRE)
    k_bulk<Q, ST, NS, GEOM, MODE_PRE><<<g, 256, 0, s>>>(a);
  else
    k_bulk<Q, ST, NS, GEOM, MODE_MACRO><<<g, 256, 0, s>>>(a);
  return hipGetLastError();
}

template <int Q, int ST, bool NS>
static hipError_t fused_t(const KArgs &a, hipStream_t s) {
  const int sblocks = (int)((blocks_for(a.nspecial, 256) + 7) / 8 * 8);
  k_fused<Q, ST, NS><<<blocks_for(a.n, 256) + sblocks, 256, 0, s>>>(a, sblocks);
  return hipGetLastError();
}

hipError_t launch_fused(int storage, bool ns, const KArgs &a, hipStream_t s) {
  if (ns) LBM_DISPATCH_ST(storage, (fused_t<9, ST, true>(a, s)))
  LBM_DISPATCH_ST(storage, (fused_t<9, ST, false>(a, s)))
}

template <int Q, int ST, bool NS>
static hipError_t special_t(int mode, const KArgs &a, hipStream_t s) {
  if (a.nspecial == 0) return hipSuccess;
  const unsigned g = blocks_for(a.nspecial, 64);
  if (mode == MODE_STEP)
    k_special<Q, ST, NS, MODE_STEP><<<g, 64, 0, s>>>(a);
  else if (mode == MODE_PRE)
    k_special<Q, ST, NS, MODE_PRE><<<g, 64, 0, s>>>(a);
  else
    k_special<Q, ST, NS, MODE_MACRO><<<g, 64, 0, s>>>(a);
  return hipGetLastError();
}

template <int Q>
static hipError_t pass_q(int storage, bool ns, bool geom, int mode, const KArgs &a, hipStream_t s) {
  if (ns) {
    if (geom) LBM_DISPATCH_ST(storage, (pass_t<Q, ST, true, true>(mode, a, s)))
    LBM_DISPATCH_ST(storage, (pass_t<Q, ST, true, false>(mode, a, s)))
  }
  if (geom) LBM_DISPATCH_ST(storage, (pass_t<Q, ST, false, true>(mode, a, s)))
  LBM_DISPATCH_ST(storage, (pass_t<Q, ST, false, false>(mode, a, s)))
}

hipError_t launch_pass(int Q, int storage, bool ns, bool geom, int mode, const KArgs &a,
                       hipStream_t s) {
  if (Q == 9) return pass_q<9>(storage, ns, geom, mode, a, s);
  if (Q == 27) return pass_q<27>(storage, ns, geom, mode, a, s);
  return hipErrorInvalidValue;
}

template <int Q>
static hipError_t special_q(int storage, bool ns, int mode, const KArgs &a, hipStream_t s) {
  if (ns) LBM_DISPATCH_ST(storage, (special_t<Q, ST, true>(mode, a, s)))
  LBM_DISPATCH_ST(storage, (special_t<Q, ST, false>(mode, a, s)))
}

hipError_t launch_special(int Q, int storage, bool ns, int mode, const KArgs &a, hipStream_t s) {
  if (Q == 9) return special_q<9>(storage, ns, mode, a, s);
  if (Q == 27) return special_q<27>(storage, ns, mode, a, s);
  return hipErrorInvalidValue;
}

template <int Q, int ST, bool NS>
static hipError_t init_t(const InitArgs &a, hipStream_t s) {
  k_init<Q, ST, NS><<<blocks_for(a.n, 256), 256, 0, s>>>(a);
  return hipGetLastError();
}

template <int Q>
static hipError_t init_q(int storage, bool ns, const InitArgs &a, hipStream_t s) {
  if (ns) LBM_DISPATCH_ST(storage, (init_t<Q, ST, true>(a, s)))
  LBM_DISPATCH_ST(storage, (init_t<Q, ST, false>(a, s)))
}

hipError_t launch_init(int Q, int storage, bool ns, const InitArgs &a, hipStream_t s) {
  if (Q == 9) return init_q<9>(storage, ns, a, s);
  if (Q == 27) return init_q<27>(storage, ns, a, s);
  return hipErrorInvalidValue;
}

template <int Q, int ST>
static hipError_t convert_t(bool to_storage, const void *from, void *to, int64_t n, double ref,
                            const uint8_t *cls, hipStream_t s) {
  if (to_storage)
    k_convert<Q, ST, true><<<blocks_for(n, 256), 256, 0, s>>>(from, to, n, ref, cls);
  else
    k_convert<Q, ST, false><<<blocks_for(n, 256), 256, 0, s>>>(from, to, n, ref, cls);
  return hipGetLastError();
}

hipError_t launch_convert(int Q, int storage, bool to_storage, const void *from, void *to, int64_t n,
                          double ref, const uint8_t *cls, hipStream_t s) {
  if (Q == 9) LBM_DISPATCH_ST(storage, (convert_t<9, ST>(to_storage, from, to, n, ref, cls, s)))
  if (Q == 27) LBM_DISPATCH_ST(storage, (convert_t<27, ST>(to_storage, from, to, n, ref, cls, s)))
  return hipErrorInvalidValue;
}

template <int Q, class R>
static hipError_t adjoint_t(const KArgs &a, const void *ln, void *lp, void *dq, hipStream_t s) {
  k_adjoint<Q, R><<<blocks_for(a.n, 256), 256, 0, s>>>(a, static_cast<const R *>(ln), static_cast<R *>(lp),
                                                         static_cast<double *>(dq));
  return hipGetLastError();
}

hipError_t launch_adjoint(int Q, bool fp64, const KArgs &a, const void *lam_next, void *lam_prev, void *dJdQ,
                          hipStream_t s) {
  if (Q == 9) return fp64 ? adjoint_t<9, double>(a, lam_next, lam_prev, dJdQ, s)
                          : adjoint_t<9, float>(a, lam_next, lam_prev, dJdQ, s);
  if (Q == 27) return fp64 ? adjoint_t<27, double>(a, lam_next, lam_prev, dJdQ, s)
                           : adjoint_t<27, float>(a, lam_next, lam_prev, dJdQ, s);
  return hipErrorInvalidValue;
}

hipError_t launch_seed(int Q, bool fp64, const double *H, const double *Ht, int64_t n, void *lam, void *dJdQ,
                       double *sq, hipStream_t s) {
  const unsigned g = blocks_for(n, 256);
  if (Q == 9) {
    if (fp64) k_seed<9, double><<<g, 256, 0, s>>>(H, Ht, n, static_cast<double *>(lam), static_cast<double *>(dJdQ), sq);
    else k_seed<9, float><<<g, 256, 0, s>>>(H, Ht, n, static_cast<float *>(lam), static_cast<double *>(dJdQ), sq);
  } else {
    if (fp64) k_seed<27, double><<<g, 256, 0, s>>>(H, Ht, n, static_cast<double *>(lam), static_cast<double *>(dJdQ), sq);
    else k_seed<27, float><<<g, 256, 0, s>>>(H, Ht, n, static_cast<float *>(lam), static_cast<double *>(dJdQ), sq);
  }
  return hipGetLastError();
}

hipError_t launch_reduce(const double *rho, const double *H, const double *qx, int64_t n, int nx,
                         int ny, int nz, const int32_t *cols, int ncols, const double *link_flux,
                         const DevLink *links, int64_t nlinks, int group, double *partials,
                         int npartials, double *out, hipStream_t s) {
  k_sum_partials<<<npartials, 256, 0, s>>>(rho, H, n, partials);
  k_sum_final<<<1, 256, 0, s>>>(partials, npartials, out);
  k_group_flux<<<1, 256, 0, s>>>(link_flux, links, nlinks, group, out);
  if (ncols > 0) k_column_sum<<<ncols, 256, 0, s>>>(qx, nx, ny, nz, cols, out);
  return hipGetLastError();
}

}  // namespace lbm
