// lbm_kernels.hip -- lattice dispatch of the launchers (kernels instantiated
// per lattice in lbm_q9.hip / lbm_q27.hip) and the deterministic FP64
// reductions.
#include "lbm_kernels.hpp"

namespace lbm {

#define LBM_DECLARE(NAME)                                                                             \
  hipError_t NAME##_pass(bool, bool, int, int, int, const KArgs &, hipStream_t);                      \
  hipError_t NAME##_special(bool, int, int, int, const KArgs &, hipStream_t);                         \
  hipError_t NAME##_fused(bool, int, int, const KArgs &, hipStream_t);                                \
  hipError_t NAME##_side(bool, int, const KArgs &, hipStream_t);                                      \
  hipError_t NAME##_init(bool, int, const InitArgs &, hipStream_t);                                   \
  hipError_t NAME##_convert(int, bool, const KArgs &, const void *, void *, double, hipStream_t);      \
  hipError_t NAME##_adjoint(const KArgs &, const void *, void *, void *, hipStream_t);                \
  hipError_t NAME##_seed(const double *, const double *, const uint8_t *, int64_t, void *, void *, double *,  \
                         hipStream_t);
LBM_DECLARE(q9_fp64)
LBM_DECLARE(q9_fp32)
LBM_DECLARE(q9_fp32dev)
LBM_DECLARE(q9_fp16dev)
LBM_DECLARE(q27_fp64)
LBM_DECLARE(q27_fp32)
LBM_DECLARE(q27_fp32dev)
LBM_DECLARE(q27_fp16dev)
LBM_DECLARE(q9_fp32sr)
LBM_DECLARE(q27_fp32sr)
LBM_DECLARE(q9_fp16sr)
LBM_DECLARE(q27_fp16sr)

// (lattice, storage) -> the launcher of that translation unit
#define LBM_SELECT(Q, ST, F, ...)                                              \
  do {                                                                         \
    if (Q == 9) {                                                              \
      switch (ST) {                                                            \
        case ST_FP64: return q9_fp64_##F(__VA_ARGS__);                         \
        case ST_FP32: return q9_fp32_##F(__VA_ARGS__);                         \
        case ST_FP32_DEV: return q9_fp32dev_##F(__VA_ARGS__);                  \
        case ST_FP16_DEV: return q9_fp16dev_##F(__VA_ARGS__);                  \
        case ST_FP32_SR: return q9_fp32sr_##F(__VA_ARGS__);                    \
        case ST_FP16_SR: return q9_fp16sr_##F(__VA_ARGS__);                    \
      }                                                                        \
    } else if (Q == 27) {                                                      \
      switch (ST) {                                                            \
        case ST_FP64: return q27_fp64_##F(__VA_ARGS__);                        \
        case ST_FP32: return q27_fp32_##F(__VA_ARGS__);                        \
        case ST_FP32_DEV: return q27_fp32dev_##F(__VA_ARGS__);                 \
        case ST_FP16_DEV: return q27_fp16dev_##F(__VA_ARGS__);                 \
        case ST_FP32_SR: return q27_fp32sr_##F(__VA_ARGS__);                   \
        case ST_FP16_SR: return q27_fp16sr_##F(__VA_ARGS__);                   \
      }                                                                        \
    }                                                                          \
    return hipErrorInvalidValue;                                               \
  } while (0)

hipError_t launch_pass(int Q, int storage, bool ns, bool geom, int lay, int mode, int cu, const KArgs &a,
                       hipStream_t s) {
  LBM_SELECT(Q, storage, pass, ns, geom, lay, mode, cu, a, s);
}
hipError_t launch_special(int Q, int storage, bool ns, int lay, int mode, int cu, const KArgs &a, hipStream_t s) {
  LBM_SELECT(Q, storage, special, ns, lay, mode, cu, a, s);
}
hipError_t launch_fused(int Q, int storage, bool ns, int lay, int cu, const KArgs &a, hipStream_t s) {
  LBM_SELECT(Q, storage, fused, ns, lay, cu, a, s);
}
hipError_t launch_side(int Q, int storage, bool ns, int lay, const KArgs &a, hipStream_t s) {
  LBM_SELECT(Q, storage, side, ns, lay, a, s);
}
hipError_t launch_init(int Q, int storage, bool ns, int lay, const InitArgs &a, hipStream_t s) {
  LBM_SELECT(Q, storage, init, ns, lay, a, s);
}
hipError_t launch_convert(int Q, int storage, int lay, bool to_storage, const KArgs &a, const void *from, void *to,
                          double ref, hipStream_t s) {
  LBM_SELECT(Q, storage, convert, lay, to_storage, a, from, to, ref, s);
}
hipError_t launch_adjoint(int Q, bool fp64, const KArgs &a, const void *lam_next, void *lam_prev, void *dJdQ,
                          hipStream_t s) {
  LBM_SELECT(Q, fp64 ? ST_FP64 : ST_FP32, adjoint, a, lam_next, lam_prev, dJdQ, s);
}
hipError_t launch_seed(int Q, bool fp64, const double *H, const double *Ht, const uint8_t *cls, int64_t n, void *lam,
                       void *dJdQ, double *sq, hipStream_t s) {
  LBM_SELECT(Q, fp64 ? ST_FP64 : ST_FP32, seed, H, Ht, cls, n, lam, dJdQ, sq, s);
}

// ---------------------------------------------------------------------------
// Tracking objectives: residual and adjoint seed (one thread per node).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_resid(const double *H, const double *Ht, const uint8_t *cls, int64_t n,
                                               double *d, double *sq) {
  const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (m >= n) return;
  const double r = (cls && cls[m] == CLS_SOLID) ? 0.0 : H[m] - Ht[m];
  d[m] = r;
  sq[m] = r * r;
}

template <class R, bool ACC>
__global__ void __launch_bounds__(256) k_seed_add(const double *d, int Q, int64_t n, R *lam, double *dJdQ) {
  const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (m >= n) return;
  const double r = d[m];
  for (int i = 0; i < Q; i++) {
    R *p = lam + (int64_t)i * n + m;
    *p = ACC ? *p + R(r) : R(r);
  }
  dJdQ[m] = ACC ? dJdQ[m] + 0.5 * r : 0.5 * r;
}

hipError_t launch_resid(const double *H, const double *Ht, const uint8_t *cls, int64_t n, double *d, double *sq,
                        hipStream_t s) {
  k_resid<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(H, Ht, cls, n, d, sq);
  return hipGetLastError();
}

hipError_t launch_seed_add(int Q, bool fp64, bool accumulate, const double *d, int64_t n, void *lam, double *dJdQ,
                           hipStream_t s) {
  const unsigned g = (unsigned)((n + 255) / 256);
  if (fp64) {
    if (accumulate)
      k_seed_add<double, true><<<g, 256, 0, s>>>(d, Q, n, static_cast<double *>(lam), dJdQ);
    else
      k_seed_add<double, false><<<g, 256, 0, s>>>(d, Q, n, static_cast<double *>(lam), dJdQ);
  } else {
    if (accumulate)
      k_seed_add<float, true><<<g, 256, 0, s>>>(d, Q, n, static_cast<float *>(lam), dJdQ);
    else
      k_seed_add<float, false><<<g, 256, 0, s>>>(d, Q, n, static_cast<float *>(lam), dJdQ);
  }
  return hipGetLastError();
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
__global__ void __launch_bounds__(256) k_group_flux(const double *flux, const DevLink *links, int64_t nl, int group,
                                                    double *out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t l = threadIdx.x; l < nl; l += 256)
    if (links[l].group == group) s += flux[l];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[2] = s;
}

// out[3 + j] = sum over y, z of qx at x = cols[j]; one block per column
__global__ void __launch_bounds__(256) k_column_sum(const double *qx, int nx, int ny, int nz, const int32_t *cols,
                                                    double *out) {
  __shared__ double sh[256];
  const int X = cols[blockIdx.x];
  double s = 0.0;
  const int64_t nyz = (int64_t)ny * nz;
  for (int64_t k = threadIdx.x; k < nyz; k += 256) s += qx[X + (int64_t)nx * k];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[3 + blockIdx.x] = s;
}

// Streaming copy that measures the practical HBM ceiling: 16-byte
// non-temporal loads and stores (measured fastest of plain / non-temporal
// loads and stores and 1-8 vectors per thread); blocks = 0: one vector per
// thread, else a grid-stride loop over that many blocks.
typedef float v4f __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_copy16(const v4f *__restrict__ src, v4f *__restrict__ dst, int64_t n16) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += stride) {
    const v4f v = __builtin_nontemporal_load(&src[i]);
    __builtin_nontemporal_store(v, &dst[i]);
  }
}

hipError_t launch_copy16(const void *src, void *dst, int64_t n16, int blocks, hipStream_t s) {
  if (n16 <= 0) return hipSuccess;
  const int64_t one_each = (n16 + 255) / 256;
  const int64_t g = blocks > 0 && blocks < one_each ? blocks : one_each;
  k_copy16<<<(unsigned)g, 256, 0, s>>>(static_cast<const v4f *>(src), static_cast<v4f *>(dst), n16);
  return hipGetLastError();
}

hipError_t launch_reduce(const double *rho, const double *H, const double *qx, int64_t n, int nx, int ny, int nz,
                         const int32_t *cols, int ncols, const double *link_flux, const DevLink *links, int64_t nlinks,
                         int group, double *partials, int npartials, double *out, hipStream_t s) {
  k_sum_partials<<<npartials, 256, 0, s>>>(rho, H, n, partials);
  k_sum_final<<<1, 256, 0, s>>>(partials, npartials, out);
  k_group_flux<<<1, 256, 0, s>>>(link_flux, links, nlinks, group, out);
  if (ncols > 0) k_column_sum<<<ncols, 256, 0, s>>>(qx, nx, ny, nz, cols, out);
  return hipGetLastError();
}

}  // namespace lbm
