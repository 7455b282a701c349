// lbm_kernels.hpp -- HIP kernels of the fused central-moment stream-and-collide
// step and their launchers (instantiated in lbm_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// Bytes per slot of a population tile (FP64 and FP32 storage, see
// lbm_impl.hpp; measured best on MI355X): a tile holds pop_tile_bytes(Q) /
// sizeof(element) consecutive nodes.  The node count of a lattice is padded
// to a multiple of pop_pad(Q) nodes, a multiple of its tiles.
constexpr int pop_tile_bytes(int Q) { return Q == 27 ? 32768 : 4096; }
constexpr int pop_pad(int Q) { return pop_tile_bytes(Q) / 4 > 1024 ? pop_tile_bytes(Q) / 4 : 1024; }

// Device copy of one cut link; same layout as lbm_link.
struct DevLink {
  int32_t node;
  int32_t dir;
  int32_t group;
  int32_t xf_solid;
  double q;
};

// What the wall rules of one cut link read, in the arithmetic type R; derived
// from the link and the group of its solid node when the geometry is set, so
// a boundary node needs no dependent load of its group.
template <class R>
struct DevWall {
  R q;             // link fraction (Eqs. IBB and IABB)
  R H_w;           // wall value of h of the group
  int32_t interp;  // bit 0: interpolated rule for f (else bounce-back),
                   // bit 1: interpolated rule for h (else anti-bounce-back)
};

// Boundary node handled by the boundary kernel: EQ and OUTLET nodes and
// non-solid nodes with at least one cut link.  Links of a node are stored
// contiguously from lb in increasing direction, one per set bit of mask.
// ub/umask give the links of the upstream (x - 1) node of an OUTLET node.
struct DevSpecial {
  int32_t node;
  int32_t type;
  int32_t group;
  int32_t lb;
  uint32_t mask;
  int32_t ub;
  uint32_t umask;
  int32_t pad;
};

// Same layout as lbm_group.
struct DevGroup {
  int32_t f_scheme;
  int32_t h_scheme;
  double rho_w;
  double u_w[3];
  double H_w;
};

enum : int { NODE_FLUID = 0, NODE_SOLID = 1, NODE_EQ = 2, NODE_OUTLET = 3 };
// Node classes (one byte per node).  EQ nodes without cut links and outlet
// nodes whose upstream node is a plain fluid node of the same wavefront are
// handled by the bulk threads, where their loads and stores coalesce with the
// neighbours'; every other boundary node has a record in the boundary list.
enum : uint8_t {
  CLS_BULK = 0,
  CLS_SOLID = 1,
  CLS_SPECIAL = 2,  // processed from the boundary-node list
  CLS_OUTLET = 3,   // outlet, upstream node = previous lane
  CLS_EQ = 4        // CLS_EQ + g: EQ node of group g <= CLS_EQ_MAX_GROUP
};
constexpr int CLS_EQ_MAX_GROUP = 255 - CLS_EQ;

// Streaming layouts (see lbm_impl.hpp): two arrays, or one array in the
// swapped (S) or streamed (N) AA layout.
enum : int { LAY_AB = 0, LAY_AA_S = 1, LAY_AA_N = 2 };

// What a pass over the lattice produces.
enum : int {
  MODE_STEP = 0,  // collide and store the post-collision state (next buffer)
  MODE_PRE = 1,   // write the canonical pre-collision state as FP64 [Q][n]
  MODE_MACRO = 2  // write rho, u, H (and the x-flux of h) as FP64 fields
};

struct KArgs {
  const void *fsrc;
  void *fdst;
  const void *hsrc;
  void *hdst;
  const uint8_t *cls;      // node classes, or null when there is no geometry
  const void *uvel;        // [3][n] arithmetic type, or null
  const void *src;         // [n] arithmetic type, or null
  const DevLink *links;
  const void *walls;       // DevWall<arithmetic type> per link
  const DevSpecial *special;
  const DevGroup *groups;
  int64_t nspecial;
  int64_t n;
  int64_t ps;              // population layout: slots per tile, or the FP16 plane stride
  int32_t nx, ny, nz;
  uint32_t div_nx, div_ny; // division by nx and ny (multiplier and shift, see
  int32_t sh_nx, sh_ny;    // div_magic in lbm_impl.hpp)
  int32_t with_uvel;       // advection velocity from the field (else u0)
  int32_t tilemap;         // block -> tile order: 0 one slab per XCD, 1 chunks per XCD,
                           // 2 dispatch order
  int32_t row_blocks;      // consecutive blocks per XCD chunk (tilemap 1)
  int32_t xr;              // swapped in-place phase without geometry: the x-pushes
                           // go through LDS (needs nx % 256 == 0)
  int32_t pair64;          // FP16 pairs: 64-bit lane offsets (4 Q n >= 2^32)
  uint32_t sr_seed;        // FP32_SR: step counter hashed into the rounding draws
  double sf[27];           // rates of f, chimera order
  double sh[27];           // rates of h, chimera order
  float sf32[27];          // the same rates rounded for FP32 arithmetic
  float sh32[27];
  double dbulk_f;          // trace rate of f's second-order block minus its
  float dbulk_f32;         // diagonal rate (0: no separate trace rate)
  double u0[3];
  double fref, href;       // deviation references (0 unless *_DEV storage)
  double *out0, *out1, *out2, *out3;  // MODE_PRE / MODE_MACRO outputs
  double *link_flux;       // MODE_MACRO: per-link injected energy
  void *side_f;            // AA: g*_opp(i)(x_b) of f per link (arithmetic type)
  void *side_h;            // AA: the same for h
  void *side_u;            // AA: velocity at t-1 per boundary node, 2 entries
                           //     per boundary-node record (node, upstream node)
};

struct InitArgs {
  void *fdst;
  void *hdst;
  const double *rho;  // [n] or null (= 1)
  const double *u;    // [3][n] or null
  const void *uvel;   // fallback field, arithmetic type, or null
  const double *H;    // [n]
  int64_t n;
  int64_t ps;         // population layout: slots per tile, or the FP16 plane stride
  int32_t nx, ny, nz;
  double u0[3];
  double fref, href;
};

// storage codes (lbm_storage)
enum : int { ST_FP64 = 0, ST_FP32 = 1, ST_FP32_DEV = 2, ST_FP16_DEV = 3, ST_FP32_SR = 4, ST_FP16_SR = 5 };

// Launchers; return hipSuccess or the launch error.  lay: LAY_*.  cu: the
// collision of each lattice in MODE_STEP (bit 0 h, bit 1 f: cumulants, else
// central moments; bit 2 with a cumulant bit: every cumulant above order 2 of
// f and above order 1 of h has rate 1).
hipError_t launch_pass(int Q, int storage, bool ns, bool geom, int lay, int mode, int cu, const KArgs &a,
                       hipStream_t s);
hipError_t launch_special(int Q, int storage, bool ns, int lay, int mode, int cu, const KArgs &a, hipStream_t s);
// D2Q9 step with geometry: boundary and bulk nodes in one launch.
hipError_t launch_fused(int Q, int storage, bool ns, int lay, int cu, const KArgs &a, hipStream_t s);
// AA side buffers from the stored state.
hipError_t launch_side(int Q, int storage, bool ns, int lay, const KArgs &a, hipStream_t s);
hipError_t launch_init(int Q, int storage, bool ns, int lay, const InitArgs &a, hipStream_t s);
hipError_t launch_convert(int Q, int storage, int lay, bool to_storage, const KArgs &a, const void *from, void *to,
                          double ref, hipStream_t s);
hipError_t launch_reduce(const double *rho, const double *H, const double *qx, int64_t n, int nx,
                         int ny, int nz, const int32_t *cols, int ncols, const double *link_flux,
                         const DevLink *links, int64_t nlinks, int group, double *partials,
                         int npartials, double *out, hipStream_t s);
hipError_t launch_copy16(const void *src, void *dst, int64_t n16, int blocks, hipStream_t s);
hipError_t launch_adjoint(int Q, bool fp64, const KArgs &a, const void *lam_next, void *lam_prev, void *dJdQ,
                          hipStream_t s);
// cls: node classes or null; solid nodes are left out of the objective.
hipError_t launch_seed(int Q, bool fp64, const double *H, const double *Ht, const uint8_t *cls, int64_t n, void *lam,
                       void *dJdQ, double *sq, hipStream_t s);
// Residual d = H - Ht (zero at solid nodes) and d^2 per node.
hipError_t launch_resid(const double *H, const double *Ht, const uint8_t *cls, int64_t n, double *d, double *sq,
                        hipStream_t s);
// Adjoint seed from a residual: lam[i][m] (+)= d[m] for i < Q, dJdQ[m] (+)= d[m] / 2.
hipError_t launch_seed_add(int Q, bool fp64, bool accumulate, const double *d, int64_t n, void *lam, double *dJdQ,
                           hipStream_t s);

}  // namespace lbm
