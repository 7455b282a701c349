// lbm_host.hip -- C ABI of liblbm.so: parameter validation, relaxation
// presets, workspace layout, geometry (cut-link table and boundary-node list)
// and the calls that launch the kernels of lbm_kernels.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_device.hpp"
#include "lbm_kernels.hpp"

using namespace lbm;

// Static device scratch of lbm_reduce_noalloc(): the partial sums of the
// first reduction pass, the result vector and the column list.  One copy per
// GPU, held until the process ends.  In host code `scratch` is only a
// stand-in: its device address comes from hipGetSymbolAddress (per device).
namespace {
constexpr int kScratchPartials = 1024;
constexpr int kScratchColumns = 64;
constexpr size_t kScratchBytes =
    sizeof(double) * (2 * kScratchPartials + 3 + kScratchColumns) + sizeof(int32_t) * kScratchColumns;
constexpr int kMaxDevices = 64;
}  // namespace
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static void *g_scratch_ptr[kMaxDevices];
static bool g_scratch_set[kMaxDevices];

static_assert(sizeof(DevLink) == sizeof(lbm_link), "link layout");
static_assert(sizeof(DevGroup) == sizeof(lbm_group), "group layout");

namespace {

thread_local std::string g_err;

constexpr size_t kAlign = 256;
constexpr int kPartials = 1024;  // blocks of the first reduction pass
constexpr int kMaxColumns = 64;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Moment orders (per-moment rates are given in these orders): Sec. 2.1 for
// D3Q27, App. A for D2Q9.
const char *kMom27[27] = {"000", "100", "010", "001", "110", "101", "011", "200", "020",
                          "002", "120", "102", "210", "201", "012", "021", "111", "220",
                          "202", "022", "211", "121", "112", "122", "212", "221", "222"};
const char *kMom9[9] = {"00", "10", "01", "20", "02", "11", "21", "12", "22"};

void moment_index(int Q, int k, int m[3]) {
  if (Q == 27) {
    for (int d = 0; d < 3; d++) m[d] = kMom27[k][d] - '0';
  } else {
    m[0] = kMom9[k][0] - '0';
    m[1] = kMom9[k][1] - '0';
    m[2] = 0;
  }
}

// Position of moment (m, n, o) in the kernels' chimera layout.
int chimera_index(int Q, const int m[3]) { return Q == 27 ? m[0] * 9 + m[1] * 3 + m[2] : m[0] * 3 + m[1]; }

struct Layout {
  size_t pop_bytes;     // one copy of one lattice
  size_t region_bytes;  // one copy of every stored lattice
  size_t off_region[2];
  size_t off_pop[2][2];  // base of lattice 0 (f) and 1 (h) inside the regions
  int64_t ps;            // slots per tile, or the FP16 plane stride
  size_t off_cls, off_links, off_walls, off_special, off_groups, off_rho, off_H, off_qx, off_flux, off_part,
      off_res, off_cols, off_side_f, off_side_h, off_side_u;
  size_t total;
};

size_t storage_size(int st) {
  switch (st) {
    case LBM_FP64: return 8;
    case LBM_FP32:
    case LBM_FP32_DEV:
    case LBM_FP32_SR: return 4;
    case LBM_FP16_DEV:
    case LBM_FP16_SR: return 2;
    default: return 0;
  }
}

// Arithmetic in FP64 (the storage types whose kernels compute in double).
bool arith64(int st) { return st == LBM_FP64 || st == LBM_FP32_SR; }

// Seed of the FP32_SR rounding draws of the writes made at time t: a new
// draw per step (Fibonacci hashing of t).
static uint32_t sr_seed(int64_t t) { return (uint32_t)((uint64_t)t * 0x9E3779B97F4A7C15ull >> 32); }

// FP16 deviation storage (either rounding); storage of deviations from the
// reference values (FP32 or FP16).
static bool half16(int st) { return st == LBM_FP16_DEV || st == LBM_FP16_SR; }
static bool deviations(int st) { return st == LBM_FP32_DEV || half16(st); }

bool set_err(std::string *dst, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (dst) *dst = buf;
  g_err = buf;
  return false;
}

int64_t node_count(const lbm_params *p) { return (int64_t)p->nx * p->ny * p->nz; }

bool validate(const lbm_params *p, std::string *err) {
  if (!p) return set_err(err, "params is NULL");
  if (p->lattice != LBM_D2Q9 && p->lattice != LBM_D3Q27)
    return set_err(err, "lattice must be 9 (D2Q9) or 27 (D3Q27), got %d", p->lattice);
  if (p->nx < 1 || p->ny < 1 || p->nz < 1)
    return set_err(err, "nx, ny, nz must be >= 1 (got %d, %d, %d)", p->nx, p->ny, p->nz);
  if (p->lattice == LBM_D2Q9 && p->nz != 1) return set_err(err, "D2Q9 needs nz == 1 (got %d)", p->nz);
  if ((int64_t)p->nx * p->ny * p->nz > (int64_t)1 << 31)
    return set_err(err, "too many nodes (%lld), limit 2^31", (long long)node_count(p));
  if (storage_size(p->storage) == 0) return set_err(err, "unknown storage %d", p->storage);
  if (p->stream != LBM_STREAM_AB && p->stream != LBM_STREAM_AA)
    return set_err(err, "unknown stream mode %d", p->stream);
  if (p->with_ns != 0 && p->with_ns != 1) return set_err(err, "with_ns must be 0 or 1");
  if (p->relax_h < LBM_CM_SRT || p->relax_h > LBM_CM_CUSTOM) return set_err(err, "unknown relax_h %d", p->relax_h);
  if (p->with_ns && (p->relax_f < LBM_CM_SRT || p->relax_f > LBM_CM_CUSTOM))
    return set_err(err, "unknown relax_f %d", p->relax_f);
  if (p->relax_h != LBM_CM_CUSTOM && !(p->k > 0.0 && std::isfinite(p->k)))
    return set_err(err, "conductivity k must be finite and > 0 (got %g)", p->k);
  if (p->with_ns && p->relax_f != LBM_CM_CUSTOM && !(p->nu > 0.0 && std::isfinite(p->nu)))
    return set_err(err, "viscosity nu must be finite and > 0 (got %g)", p->nu);
  if (p->u_mode != 0 && p->u_mode != 1) return set_err(err, "u_mode must be 0 or 1");
  if (p->with_source && p->with_ns) return set_err(err, "a source needs with_ns == 0");
  if (p->cumulant < 0 || p->cumulant > 3) return set_err(err, "cumulant must be a bit set of 1 (h) and 2 (f)");
  if ((p->cumulant & 2) && !p->with_ns) return set_err(err, "a cumulant f collision needs with_ns == 1");
  if (p->max_links < 0 || p->max_special < 0) return set_err(err, "max_links/max_special must be >= 0");
  for (int d = 0; d < 3; d++)
    if (!std::isfinite(p->u0[d])) return set_err(err, "u0[%d] is not finite", d);
  if (!std::isfinite(p->rho_ref) || !std::isfinite(p->H_ref)) return set_err(err, "rho_ref/H_ref not finite");
  if (!(p->s_bulk_f >= 0.0 && p->s_bulk_f < 2.0))
    return set_err(err, "s_bulk_f must be 0 (default) or a rate in (0, 2), got %g", p->s_bulk_f);
  if (p->with_ns && p->s_bulk_f > 0.0 && p->relax_f == LBM_CM_CUSTOM) {
    // the deviatoric rate is the common rate of the diagonal second-order moments
    const int Q = p->lattice;
    double r[3];
    int nd = 0;
    for (int k = 0; k < Q; k++) {
      int m[3];
      moment_index(Q, k, m);
      if (m[0] + m[1] + m[2] == 2 && (m[0] == 2 || m[1] == 2 || m[2] == 2)) r[nd++] = p->s_custom_f[k];
    }
    for (int d = 1; d < nd; d++)
      if (r[d] != r[0])
        return set_err(err, "s_bulk_f > 0 needs equal custom rates of f at the diagonal second-order moments");
  }
  return true;
}

// Trace rate of f's second-order block: s_bulk_f, or 1 for the LBM_CM_NS
// preset when s_bulk_f is 0; 0 (no separate rate) otherwise.
double bulk_rate(const lbm_params *p) {
  if (!p->with_ns) return 0.0;
  if (p->s_bulk_f > 0.0) return p->s_bulk_f;
  return p->relax_f == LBM_CM_NS ? 1.0 : 0.0;
}

void preset_rates(const lbm_params *p, int relax, double rate, const double *custom, double *s) {
  const int Q = p->lattice;
  for (int k = 0; k < 27; k++) s[k] = 1.0;
  for (int k = 0; k < Q; k++) {
    int m[3];
    moment_index(Q, k, m);
    const int order = m[0] + m[1] + m[2];
    switch (relax) {
      case LBM_CM_SRT: s[k] = rate; break;
      case LBM_CM_1ST: s[k] = order == 1 ? rate : 1.0; break;
      case LBM_CM_TRT: s[k] = (order % 2 == 1) ? rate : 1.0; break;
      case LBM_CM_NS: s[k] = order == 2 ? rate : 1.0; break;
      default: s[k] = custom[k]; break;
    }
  }
}

void compute_rates(const lbm_params *p, double *sf, double *sh) {
  const double s_nu = p->with_ns ? 1.0 / (3.0 * p->nu + 0.5) : 1.0;
  const double s_H = p->relax_h == LBM_CM_CUSTOM ? 1.0 : 1.0 / (3.0 * p->k + 0.5);
  preset_rates(p, p->with_ns ? p->relax_f : LBM_CM_NS, s_nu, p->s_custom_f, sf);
  preset_rates(p, p->relax_h, s_H, p->s_custom_h, sh);
}

// Node count of a population buffer: padded to whole tiles; also the plane
// stride of the FP16 layout.
int64_t plane_nodes(int64_t n, int Q) { return (n + pop_pad(Q) - 1) / pop_pad(Q) * pop_pad(Q); }

Layout layout(const lbm_params *p) {
  Layout L;
  const int64_t n = node_count(p);
  const int Q = p->lattice;
  size_t off = 0;
  // One region per copy holds every stored lattice (lbm_impl.hpp): tiles of
  // consecutive nodes with the Q slots of f then of h (FP64/FP32), tiles of
  // (f, h) pairs (FP16 with both lattices: h starts one element after f), or
  // Q planes of plane_nodes() elements (FP16, h only).
  const size_t es = storage_size(p->storage);
  const bool fp16 = half16(p->storage);
  const bool planes = fp16 && !p->with_ns;
  const int nlat = p->with_ns ? 2 : 1;
  L.pop_bytes = align_up((size_t)Q * plane_nodes(n, Q) * es);
  L.region_bytes = (size_t)nlat * L.pop_bytes;
  L.ps = planes ? plane_nodes(n, Q) : (int64_t)Q * nlat;
  const int copies = p->stream == LBM_STREAM_AA ? 1 : 2;
  for (int c = 0; c < 2; c++) {
    L.off_region[c] = c < copies ? off : L.off_region[0];
    if (c < copies) off += L.region_bytes;
    const size_t h_at = !p->with_ns ? 0 : fp16 ? es : (size_t)Q * (pop_tile_bytes(Q) / es) * es;
    L.off_pop[0][c] = L.off_region[c];
    L.off_pop[1][c] = L.off_region[c] + h_at;
  }
  L.off_cls = off;
  off += align_up((size_t)n);
  L.off_links = off;
  off += align_up(sizeof(DevLink) * (size_t)p->max_links);
  L.off_walls = off;
  off += align_up((arith64(p->storage) ? sizeof(DevWall<double>) : sizeof(DevWall<float>)) *
                  (size_t)p->max_links);
  L.off_special = off;
  off += align_up(sizeof(DevSpecial) * (size_t)p->max_special);
  L.off_groups = off;
  off += align_up(sizeof(DevGroup) * LBM_MAX_GROUPS);
  L.off_rho = off;
  off += align_up(sizeof(double) * (size_t)n);
  L.off_H = off;
  off += align_up(sizeof(double) * (size_t)n);
  L.off_qx = off;
  off += align_up(sizeof(double) * (size_t)n);
  L.off_flux = off;
  off += align_up(sizeof(double) * (size_t)p->max_links);
  L.off_part = off;
  off += align_up(sizeof(double) * 2 * kPartials);
  L.off_res = off;
  off += align_up(sizeof(double) * (3 + kMaxColumns));
  L.off_cols = off;
  off += align_up(sizeof(int32_t) * kMaxColumns);
  // AA side buffers (arithmetic type): per link f and h, 2 x 3 per boundary node
  const size_t rsz = arith64(p->storage) ? 8 : 4;
  const bool aa = p->stream == LBM_STREAM_AA;
  L.off_side_f = off;
  off += aa ? align_up(rsz * (size_t)p->max_links) : 0;
  L.off_side_h = off;
  off += aa ? align_up(rsz * (size_t)p->max_links) : 0;
  L.off_side_u = off;
  off += aa ? align_up(rsz * 6 * (size_t)p->max_special) : 0;
  L.total = off;
  return L;
}

// Geometry built on the host.
struct Geometry {
  std::vector<DevLink> links;
  std::vector<DevSpecial> special;
  std::vector<uint8_t> cls;
  bool any = false;
};

int ntype(const uint16_t *flags, int64_t n) { return flags ? (flags[n] & 15) : 0; }
int ngroup(const uint16_t *flags, int64_t n) { return flags ? ((flags[n] >> 4) & 255) : 0; }

template <int Q>
int64_t shift(const lbm_params *p, int64_t n, int i, int sign) {
  const int64_t nx = p->nx, ny = p->ny, nz = p->nz;
  int64_t x = n % nx, y = (n / nx) % ny, z = n / (nx * ny);
  x = ((x + sign * Lat<Q>::ex(i)) % nx + nx) % nx;
  y = ((y + sign * Lat<Q>::ey(i)) % ny + ny) % ny;
  z = ((z + sign * Lat<Q>::ez(i)) % nz + nz) % nz;
  return x + nx * (y + ny * z);
}

template <int Q>
bool build_geometry_q(const lbm_params *p, const uint16_t *flags, const double *q, int n_groups,
                      bool want_links, Geometry *G, int64_t *nlinks, int64_t *nspecial, std::string *err) {
  const int64_t N = node_count(p);
  const bool aa = p->stream == LBM_STREAM_AA;
  int64_t cl = 0, cs = 0;
  if (flags) {
    for (int64_t n = 0; n < N; n++) {
      const int t = flags[n] & 15;
      if (t > 3) return set_err(err, "node %lld: unknown node type %d", (long long)n, t);
      if (t != LBM_NODE_FLUID && t != LBM_NODE_OUTLET && ngroup(flags, n) >= n_groups)
        return set_err(err, "node %lld: group %d >= n_groups %d", (long long)n, ngroup(flags, n), n_groups);
    }
  }
  if (want_links) G->cls.assign(N, CLS_BULK);
  auto links_of = [&](int64_t n, uint32_t *mask, bool emit) -> bool {
    *mask = 0;
    for (int i = 1; i < Q; i++) {
      const int64_t w = shift<Q>(p, n, i, +1);
      if (ntype(flags, w) != LBM_NODE_SOLID) continue;
      const double qv = q ? q[(int64_t)i * N + n] : 0.5;
      if (!(qv > 0.0 && qv <= 1.0))
        return set_err(err, "cut link (node %lld, dir %d): q = %.17g outside (0, 1]", (long long)n, i, qv);
      *mask |= 1u << i;
      if (emit) {
        DevLink L;
        L.node = (int32_t)n;
        L.dir = i;
        L.group = ngroup(flags, w);
        L.xf_solid = ntype(flags, shift<Q>(p, n, i, -1)) == LBM_NODE_SOLID;
        L.q = qv;
        G->links.push_back(L);
      }
    }
    return true;
  };
  // upstream node of an outlet (x - 1, periodic in x)
  auto upstream = [&](int64_t n) -> int64_t { return n % p->nx == 0 ? n + p->nx - 1 : n - 1; };
  // An outlet node is handled by the bulk threads when neither it nor its
  // upstream node has cut links, the upstream node is a plain fluid node, and
  // both lie in one wavefront of 64 consecutive nodes (n % 64 != 0, x != 0):
  // the outlet's lane then reads the upstream populations from the previous
  // lane.  EQ nodes without cut links are handled there too.
  auto bulk_outlet = [&](int64_t n, uint32_t mask, bool *ok) -> bool {
    *ok = true;
    if (mask || n % p->nx == 0 || n % 64 == 0) return false;
    const int64_t up = n - 1;
    if (ntype(flags, up) != LBM_NODE_FLUID) return false;
    uint32_t umask;
    if (!links_of(up, &umask, false)) {
      *ok = false;
      return false;
    }
    return umask == 0;
  };
  std::vector<char> listed_outlet;
  if (aa && flags) listed_outlet.assign((size_t)N, 0);
  for (int64_t n = 0; flags && n < N; n++) {
    const int t = ntype(flags, n);
    if (t == LBM_NODE_SOLID) {
      if (want_links) G->cls[n] = CLS_SOLID;
      G->any = true;
      continue;
    }
    uint32_t mask;
    const int64_t lb = cl;
    if (!links_of(n, &mask, want_links)) return false;
    cl += __builtin_popcount(mask);
    if (t == LBM_NODE_EQ || t == LBM_NODE_OUTLET || mask) {
      G->any = true;
      if (t == LBM_NODE_OUTLET && ntype(flags, upstream(n)) == LBM_NODE_SOLID)
        return set_err(err, "outlet node %lld: upstream node %lld is solid", (long long)n, (long long)upstream(n));
      if (t == LBM_NODE_EQ && mask == 0 && ngroup(flags, n) <= CLS_EQ_MAX_GROUP) {
        if (want_links) G->cls[n] = (uint8_t)(CLS_EQ + ngroup(flags, n));
        continue;
      }
      if (t == LBM_NODE_OUTLET) {
        bool ok;
        const bool in_bulk = bulk_outlet(n, mask, &ok);
        if (!ok) return false;
        if (in_bulk) {
          if (want_links) G->cls[n] = CLS_OUTLET;
          continue;
        }
        if (aa) listed_outlet[n] = 1;
      }
      if (want_links) {
        DevSpecial s;
        memset(&s, 0, sizeof(s));
        s.node = (int32_t)n;
        s.type = t;
        s.group = ngroup(flags, n);
        s.lb = (int32_t)lb;
        s.mask = mask;
        G->special.push_back(s);
        G->cls[n] = CLS_SPECIAL;
      }
      cs++;
    }
  }
  if (aa && flags) {
    // AA: the thread of a listed outlet node also updates its upstream node,
    // which then needs no record of its own (see lbm_impl.hpp)
    std::vector<char> absorbed((size_t)N, 0);
    for (int64_t n = 0; n < N; n++) {
      if (ntype(flags, n) != LBM_NODE_OUTLET) continue;
      const int64_t up = upstream(n);
      if (ntype(flags, up) != LBM_NODE_FLUID)
        return set_err(err, "AA layout: outlet node %lld needs a FLUID upstream node (node %lld)", (long long)n,
                       (long long)up);
      if (!listed_outlet[n]) continue;
      absorbed[up] = 1;
      if (want_links) G->cls[up] = CLS_SPECIAL;
    }
    // an absorbed node that had a record of its own (a fluid node with cut
    // links) loses it
    for (int64_t n = 0; n < N; n++) {
      if (!absorbed[n]) continue;
      uint32_t m;
      if (!links_of(n, &m, false)) return false;
      if (m) cs--;
    }
    if (want_links) {
      std::vector<DevSpecial> kept;
      for (const auto &sp : G->special)
        if (!absorbed[sp.node]) kept.push_back(sp);
      G->special.swap(kept);
    }
  }
  if (want_links) {
    // upstream link ranges of outlet nodes (links are sorted by node)
    for (auto &s : G->special) {
      if (s.type != LBM_NODE_OUTLET) continue;
      const int64_t up = upstream(s.node);
      size_t lo = 0, hi = G->links.size();
      while (lo < hi) {
        const size_t mid = (lo + hi) / 2;
        if (G->links[mid].node < up) lo = mid + 1; else hi = mid;
      }
      uint32_t umask = 0;
      for (size_t l = lo; l < G->links.size() && G->links[l].node == up; l++) umask |= 1u << G->links[l].dir;
      s.ub = (int32_t)lo;
      s.umask = umask;
    }
  }
  if (nlinks) *nlinks = cl;
  if (nspecial) *nspecial = cs;
  return true;
}

// Per-link wall records in the arithmetic type R.  A link takes the plain
// (anti-)bounce-back rule when its group asks for it, when q = 1/2, where both
// branches of the interpolated rules reduce to it, and when the q <= 1/2
// branch (the only one that reads x_f = x_b - e_i) meets a solid x_f (a
// one-node gap).  The q > 1/2 branch reads x_b only and stays interpolated
// in a gap (Sec. 3, Eqs. IBB and IABB).  The branch test is made on q as the
// kernels see it, in R.
template <class R>
void wall_records(const std::vector<DevLink> &links, const std::vector<DevGroup> &groups, std::vector<char> *out) {
  out->assign(sizeof(DevWall<R>) * links.size(), 0);
  DevWall<R> *w = reinterpret_cast<DevWall<R> *>(out->data());
  for (size_t l = 0; l < links.size(); l++) {
    const DevLink &k = links[l];
    const DevGroup &g = groups[k.group];
    const bool plain = k.q == 0.5 || (k.xf_solid && R(k.q) <= R(0.5));
    w[l].q = R(k.q);
    w[l].H_w = R(g.H_w);
    w[l].interp = (g.f_scheme == LBM_WALL_IBB && !plain ? 1 : 0) | (g.h_scheme == LBM_WALL_IABB && !plain ? 2 : 0);
  }
}

bool build_geometry(const lbm_params *p, const uint16_t *flags, const double *q, int n_groups,
                    bool want_links, Geometry *G, int64_t *nlinks, int64_t *nspecial, std::string *err) {
  if (p->lattice == 9) return build_geometry_q<9>(p, flags, q, n_groups, want_links, G, nlinks, nspecial, err);
  return build_geometry_q<27>(p, flags, q, n_groups, want_links, G, nlinks, nspecial, err);
}

}  // namespace

struct lbm_ctx {
  lbm_params p;
  int Q;
  int64_t n;
  hipStream_t stream;
  int device;
  char *ws;
  Layout L;
  int cur;    // AB: copy holding the stored state
  int phase;  // AA: 0 swapped layout (next step pulls and pushes), 1 streamed layout
  bool initialized;
  bool geom;
  int64_t nlinks, nspecial;
  const void *uvel;
  const void *src;
  double sf[27], sh[27];  // moment order of the header
  double sfc[27], shc[27];  // chimera order
  int cu_kernel;            // collision selector of the step kernels (cumulant bits,
                            // plus 4 when the order-limited cumulant transform applies)
  int64_t t;
  std::string err;
  std::vector<DevLink> host_links;
  std::vector<int32_t> host_cols;
  // opt-in per-kernel timing: events around each bulk and boundary launch
  std::vector<hipEvent_t> ev;
  int64_t ev_used = 0;
  bool profiling = false;
  struct {
    int64_t magic, t, Q, n, storage, with_ns, bytes, phase;
  } hdr;
  void *pop(int lat, int c) { return ws + L.off_pop[lat][c]; }
  bool aa() const { return p.stream == LBM_STREAM_AA; }
  int lay() const { return !aa() ? LAY_AB : (phase == 0 ? LAY_AA_S : LAY_AA_N); }
};

#define CTX_CHECK(ctx)                                                        \
  do {                                                                        \
    if (!(ctx)) {                                                             \
      g_err = "context is NULL";                                              \
      return LBM_EINVAL;                                                      \
    }                                                                         \
  } while (0)

static lbm_status hip_fail(lbm_ctx *ctx, hipError_t e, const char *what) {
  set_err(ctx ? &ctx->err : nullptr, "%s: %s", what, hipGetErrorString(e));
  return LBM_EDEVICE;
}

#define HIP_TRY(ctx, expr, what)                 \
  do {                                           \
    hipError_t e_ = (expr);                      \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, what); \
  } while (0)

static lbm_status activate(lbm_ctx *ctx) {
  int d = -1;
  if (hipGetDevice(&d) != hipSuccess || d != ctx->device)
    HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  return LBM_OK;
}

// Multiplier and shift for exact division of node indices (below 2^31) by d:
// with s = 31 + ceil(log2 d) and M = ceil(2^s / d) < 2^32, floor(m M / 2^s) =
// floor(m / d), since M d - 2^s < d <= 2^(s - 31) bounds the error of m M / 2^s
// against m / d below 1 / d (Granlund and Montgomery, division by invariant
// integers using multiplication, 1994).
static void divisor_magic(uint32_t d, uint32_t *M, int32_t *s) {
  int l = 0;
  while (((uint64_t)1 << l) < d) l++;
  *s = 31 + l;
  *M = (uint32_t)((((uint64_t)1 << *s) + d - 1) / d);
}

// Highest total order m + n + o among the moments k > 0 whose rate (chimera
// order) is not 1.
static int top_rate_order(int Q, const double *sc) {
  int top = 0;
  for (int k = 1; k < Q; k++) {
    const int m = Q == 9 ? k / 3 : k / 9, n = Q == 9 ? k % 3 : (k / 3) % 3, o = Q == 9 ? 0 : k % 3;
    if (sc[k] != 1.0 && m + n + o > top) top = m + n + o;
  }
  return top;
}

// Whether every rate (chimera order) of a class of moments is exactly 1:
// cls 3 every order >= 3; cls 1 every even order (0 included); cls 2 order 0
// and every order >= 2.
static bool rates_one_where(int Q, const double *sc, int cls) {
  for (int k = 0; k < Q; k++) {
    const int m = Q == 9 ? k / 3 : k / 9, n = Q == 9 ? k % 3 : (k / 3) % 3, o = Q == 9 ? 0 : k % 3;
    const int order = m + n + o;
    const bool in = cls == 3 ? order >= 3 : cls == 1 ? order % 2 == 0 : order != 1;
    if (in && sc[k] != 1.0) return false;
  }
  return true;
}

static KArgs make_args(lbm_ctx *ctx, int src_copy) {
  KArgs a;
  memset(&a, 0, sizeof(a));
  const bool ns = ctx->p.with_ns;
  const int dst_copy = ctx->aa() ? src_copy : src_copy ^ 1;  // AA updates in place
  a.fsrc = ns ? ctx->pop(0, src_copy) : nullptr;
  a.fdst = ns ? ctx->pop(0, dst_copy) : nullptr;
  a.hsrc = ctx->pop(1, src_copy);
  a.hdst = ctx->pop(1, dst_copy);
  a.side_f = ctx->ws + ctx->L.off_side_f;
  a.side_h = ctx->ws + ctx->L.off_side_h;
  a.side_u = ctx->ws + ctx->L.off_side_u;
  a.cls = ctx->geom ? reinterpret_cast<const uint8_t *>(ctx->ws + ctx->L.off_cls) : nullptr;
  a.uvel = ctx->uvel;
  a.with_uvel = ctx->uvel != nullptr;
  a.src = ctx->p.with_source ? ctx->src : nullptr;
  a.links = reinterpret_cast<const DevLink *>(ctx->ws + ctx->L.off_links);
  a.walls = ctx->ws + ctx->L.off_walls;
  a.special = reinterpret_cast<const DevSpecial *>(ctx->ws + ctx->L.off_special);
  a.groups = reinterpret_cast<const DevGroup *>(ctx->ws + ctx->L.off_groups);
  a.nspecial = ctx->geom ? ctx->nspecial : 0;
  a.n = ctx->n;
  a.ps = ctx->L.ps;
  a.nx = ctx->p.nx;
  a.ny = ctx->p.ny;
  a.nz = ctx->p.nz;
  divisor_magic((uint32_t)a.nx, &a.div_nx, &a.sh_nx);
  divisor_magic((uint32_t)a.ny, &a.div_ny, &a.sh_ny);
  // block orders measured best on MI355X: D2Q9 tiles one slab per XCD in
  // place (AA), chunks of two x-rows per XCD with two arrays (AB); D2Q9 FP16
  // planes one slab per XCD (dispatch order in the streamed AA phase); D3Q27
  // tiles dispatch order (the orders measured within 1% of each other);
  // D3Q27 FP16 planes chunks of two x-rows per XCD.  FP16 pairs are tiles.
  const bool planes = half16(ctx->p.storage) && !ctx->p.with_ns;
  if (ctx->Q == 27)
    a.tilemap = planes ? 1 : 2;
  else if (!planes)
    a.tilemap = ctx->aa() ? 0 : 1;
  else
    a.tilemap = ctx->lay() == LAY_AA_N ? 2 : 0;
  a.row_blocks = 2 * ((ctx->p.nx + 255) / 256);
  // the swapped in-place phase of a lattice without geometry whose x-rows
  // are whole blocks realigns its x-pushes through LDS (k_bulk XR)
  a.xr = !ctx->geom && !arith64(ctx->p.storage) && ctx->p.nx % 256 == 0;
  a.sr_seed = sr_seed(ctx->t);
  // FP16 pairs address a byte offset of up to 4 Q (padded nodes) per slot base
  a.pair64 = (double)4 * ctx->Q * (double)plane_nodes(ctx->n, ctx->Q) >= 4294967296.0;
  for (int k = 0; k < 27; k++) {
    a.sf[k] = ctx->sfc[k];
    a.sh[k] = ctx->shc[k];
    a.sf32[k] = (float)ctx->sfc[k];
    a.sh32[k] = (float)ctx->shc[k];
  }
  // chimera slot 2 is the moment 020 (D2Q9: 02), one of the diagonal ones
  const double sb = bulk_rate(&ctx->p);
  a.dbulk_f = sb > 0.0 ? sb - ctx->sfc[2] : 0.0;
  a.dbulk_f32 = sb > 0.0 ? (float)sb - (float)ctx->sfc[2] : 0.0f;
  for (int d = 0; d < 3; d++) a.u0[d] = ctx->p.u0[d];
  const bool dev = deviations(ctx->p.storage);
  a.fref = dev ? ctx->p.rho_ref : 0.0;
  a.href = dev ? ctx->p.H_ref : 0.0;
  return a;
}

static lbm_status run_pass(lbm_ctx *ctx, int mode, const KArgs &a) {
  const bool timed = ctx->profiling && mode == MODE_STEP && ctx->ev_used + 3 <= (int64_t)ctx->ev.size();
  if (timed) HIP_TRY(ctx, hipEventRecord(ctx->ev[ctx->ev_used], ctx->stream), "event record");
  if (mode == MODE_STEP && ctx->geom && ctx->Q == 9) {
    // bulk and boundary nodes in one launch; the boundary time is inside it
    HIP_TRY(ctx, launch_fused(ctx->Q, ctx->p.storage, ctx->p.with_ns, ctx->lay(), ctx->cu_kernel, a, ctx->stream),
            "step kernel launch");
    if (timed) {
      HIP_TRY(ctx, hipEventRecord(ctx->ev[ctx->ev_used + 1], ctx->stream), "event record");
      HIP_TRY(ctx, hipEventRecord(ctx->ev[ctx->ev_used + 2], ctx->stream), "event record");
      ctx->ev_used += 3;
    }
    return LBM_OK;
  }
  HIP_TRY(ctx, launch_pass(ctx->Q, ctx->p.storage, ctx->p.with_ns, ctx->geom, ctx->lay(), mode, ctx->cu_kernel, a,
                           ctx->stream),
          "bulk kernel launch");
  if (timed) HIP_TRY(ctx, hipEventRecord(ctx->ev[ctx->ev_used + 1], ctx->stream), "event record");
  if (ctx->geom)
    HIP_TRY(ctx, launch_special(ctx->Q, ctx->p.storage, ctx->p.with_ns, ctx->lay(), mode, ctx->cu_kernel, a, ctx->stream),
            "boundary kernel launch");
  if (timed) {
    HIP_TRY(ctx, hipEventRecord(ctx->ev[ctx->ev_used + 2], ctx->stream), "event record");
    ctx->ev_used += 3;
  }
  return LBM_OK;
}

// AA: side buffers of the boundary nodes from the stored state.
static lbm_status rebuild_side(lbm_ctx *ctx) {
  if (!ctx->aa() || !ctx->geom || ctx->nspecial == 0) return LBM_OK;
  KArgs a = make_args(ctx, 0);
  HIP_TRY(ctx, launch_side(ctx->Q, ctx->p.storage, ctx->p.with_ns, ctx->lay(), a, ctx->stream), "side kernel launch");
  return LBM_OK;
}

static lbm_status need_ready(lbm_ctx *ctx) {
  if (!ctx->initialized) {
    set_err(&ctx->err, "state not initialised: call lbm_init_equilibrium or lbm_set_populations first");
    return LBM_ESTATE;
  }
  if (!ctx->p.with_ns && ctx->p.u_mode == 1 && !ctx->uvel) {
    set_err(&ctx->err, "u_mode = 1 but no velocity field set (lbm_set_velocity)");
    return LBM_ESTATE;
  }
  if (ctx->p.with_source && !ctx->src) {
    set_err(&ctx->err, "with_source = 1 but no source set (lbm_set_source)");
    return LBM_ESTATE;
  }
  return LBM_OK;
}

extern "C" {

const char *lbm_version(void) { return "liblbm 0.1 (gfx950, central-moment LBM)"; }

size_t lbm_workspace_bytes(const lbm_params *p) {
  if (!validate(p, nullptr)) return 0;
  return layout(p).total;
}

lbm_status lbm_relaxation_rates(const lbm_params *p, double *s_f, double *s_h, double *s_bulk_f) {
  if (!validate(p, nullptr)) return LBM_EINVAL;
  double a[27], b[27];
  compute_rates(p, a, b);
  if (s_f) memcpy(s_f, a, sizeof(a));
  if (s_h) memcpy(s_h, b, sizeof(b));
  if (s_bulk_f) *s_bulk_f = bulk_rate(p);
  return LBM_OK;
}

lbm_status lbm_count_geometry(const lbm_params *p, const uint16_t *flags, int64_t *n_links,
                              int64_t *n_special) {
  if (!validate(p, nullptr)) return LBM_EINVAL;
  Geometry G;
  int64_t nl = 0, ns = 0;
  if (!build_geometry(p, flags, nullptr, LBM_MAX_GROUPS, false, &G, &nl, &ns, nullptr)) return LBM_EINVAL;
  if (n_links) *n_links = nl;
  if (n_special) *n_special = ns;
  return LBM_OK;
}

lbm_status lbm_build_links(const lbm_params *p, const uint16_t *flags, const double *q, int32_t n_groups,
                           lbm_link *out, int64_t cap, int64_t *count) {
  if (!validate(p, nullptr)) return LBM_EINVAL;
  if (n_groups < 0 || n_groups > LBM_MAX_GROUPS) {
    set_err(nullptr, "n_groups %d outside [0, %d]", n_groups, LBM_MAX_GROUPS);
    return LBM_EINVAL;
  }
  Geometry G;
  int64_t nl = 0, ns = 0;
  if (!build_geometry(p, flags, q, n_groups, true, &G, &nl, &ns, nullptr)) return LBM_EINVAL;
  if (count) *count = nl;
  if (out)
    for (int64_t i = 0; i < nl && i < cap; i++) memcpy(&out[i], &G.links[i], sizeof(lbm_link));
  return LBM_OK;
}

const char *lbm_last_error(const lbm_ctx *ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

lbm_status lbm_create(const lbm_params *p, void *workspace_dev, void *hip_stream, lbm_ctx **out) {
  if (!out) {
    g_err = "out is NULL";
    return LBM_EINVAL;
  }
  *out = nullptr;
  if (!validate(p, nullptr)) return LBM_EINVAL;
  if (!workspace_dev || (reinterpret_cast<uintptr_t>(workspace_dev) % kAlign) != 0) {
    set_err(nullptr, "workspace must be a non-NULL, %zu-byte aligned device pointer", kAlign);
    return LBM_EINVAL;
  }
  lbm_ctx *ctx = new (std::nothrow) lbm_ctx();
  if (!ctx) {
    g_err = "out of host memory";
    return LBM_ENOMEM;
  }
  ctx->p = *p;
  ctx->Q = p->lattice;
  ctx->n = node_count(p);
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  if (hipGetDevice(&ctx->device) != hipSuccess) {
    delete ctx;
    g_err = "hipGetDevice failed";
    return LBM_EDEVICE;
  }
  // device address of the static scratch, looked up once per device with
  // that device current (each GPU holds its own copy of the array)
  if (ctx->device < 0 || ctx->device >= kMaxDevices) {
    delete ctx;
    set_err(nullptr, "device index outside [0, %d)", kMaxDevices);
    return LBM_EDEVICE;
  }
  if (!g_scratch_set[ctx->device]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      delete ctx;
      set_err(nullptr, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
      return LBM_EDEVICE;
    }
    g_scratch_ptr[ctx->device] = ptr;
    g_scratch_set[ctx->device] = true;
  }
  ctx->ws = static_cast<char *>(workspace_dev);
  ctx->L = layout(p);
  ctx->cur = 0;
  ctx->phase = 0;
  ctx->initialized = false;
  ctx->geom = false;
  ctx->nlinks = ctx->nspecial = 0;
  ctx->uvel = ctx->src = nullptr;
  ctx->t = 0;
  compute_rates(p, ctx->sf, ctx->sh);
  for (int k = 0; k < 27; k++) ctx->sfc[k] = ctx->shc[k] = 1.0;
  for (int k = 0; k < ctx->Q; k++) {
    int m[3];
    moment_index(ctx->Q, k, m);
    ctx->sfc[chimera_index(ctx->Q, m)] = ctx->sf[k];
    ctx->shc[chimera_index(ctx->Q, m)] = ctx->sh[k];
  }
  // the cumulant transform stops at second order (f) and first order (h)
  // when every rate above is 1 (the hydrodynamic and Cumulants-1st presets)
  ctx->cu_kernel = p->cumulant;
  if (p->cumulant && (!(p->cumulant & 2) || top_rate_order(ctx->Q, ctx->sfc) <= 2) &&
      (!(p->cumulant & 1) || top_rate_order(ctx->Q, ctx->shc) <= 1))
    ctx->cu_kernel |= 4;
  // central-moment lattices whose rates are 1 on a whole class of orders take
  // those moments' equilibria directly (the hydrodynamic preset for f,
  // CM-TRT or CM-1st for h): bits 3, 4 and 5 of the collision selector, for
  // the combinations the kernels are built for
  {
    int pat = 0;
    if (p->with_ns && !(p->cumulant & 2) && rates_one_where(ctx->Q, ctx->sfc, 3)) pat |= 8;
    if (!(p->cumulant & 1)) {
      if (rates_one_where(ctx->Q, ctx->shc, 2))
        pat |= 32;
      else if (rates_one_where(ctx->Q, ctx->shc, 1))
        pat |= 16;
    }
    const int sel = ctx->cu_kernel | pat;
    if (sel == 8 || sel == 16 || sel == 22 || sel == 24 || sel == 32 || sel == 40) ctx->cu_kernel = sel;
  }
  *out = ctx;
  return LBM_OK;
}

void lbm_destroy(lbm_ctx *ctx) {
  if (!ctx) return;
  for (hipEvent_t e : ctx->ev) (void)hipEventDestroy(e);
  delete ctx;
}

lbm_status lbm_set_geometry(lbm_ctx *ctx, const uint16_t *flags, const double *q, const lbm_group *groups,
                            int32_t n_groups) {
  CTX_CHECK(ctx);
  if (n_groups < 0 || n_groups > LBM_MAX_GROUPS || (n_groups > 0 && !groups)) {
    set_err(&ctx->err, "groups must hold n_groups in [0, %d] entries", LBM_MAX_GROUPS);
    return LBM_EINVAL;
  }
  for (int g = 0; g < n_groups; g++) {
    if (groups[g].f_scheme != LBM_WALL_BB && groups[g].f_scheme != LBM_WALL_IBB) {
      set_err(&ctx->err, "group %d: unknown f_scheme %d", g, groups[g].f_scheme);
      return LBM_EINVAL;
    }
    if (groups[g].h_scheme != LBM_WALL_ABB && groups[g].h_scheme != LBM_WALL_IABB) {
      set_err(&ctx->err, "group %d: unknown h_scheme %d", g, groups[g].h_scheme);
      return LBM_EINVAL;
    }
  }
  Geometry G;
  std::vector<char> walls;
  int64_t nl = 0, ns = 0;
  if (!build_geometry(&ctx->p, flags, q, n_groups, true, &G, &nl, &ns, &ctx->err)) return LBM_EINVAL;
  if (nl > ctx->p.max_links || ns > ctx->p.max_special) {
    set_err(&ctx->err, "geometry has %lld cut links and %lld boundary nodes; capacity is max_links=%d, "
            "max_special=%d", (long long)nl, (long long)ns, ctx->p.max_links, ctx->p.max_special);
    return LBM_ENOMEM;
  }
  if (lbm_status st = activate(ctx)) return st;
  std::vector<DevGroup> dg(LBM_MAX_GROUPS);
  memset(dg.data(), 0, sizeof(DevGroup) * dg.size());
  for (int g = 0; g < n_groups; g++) memcpy(&dg[g], &groups[g], sizeof(DevGroup));
  HIP_TRY(ctx, hipMemcpyAsync(ctx->ws + ctx->L.off_groups, dg.data(), sizeof(DevGroup) * dg.size(),
                              hipMemcpyHostToDevice, ctx->stream), "copy groups");
  if (G.any) {
    HIP_TRY(ctx, hipMemcpyAsync(ctx->ws + ctx->L.off_cls, G.cls.data(), G.cls.size(), hipMemcpyHostToDevice,
                                ctx->stream), "copy node classes");
    if (nl) {
      HIP_TRY(ctx, hipMemcpyAsync(ctx->ws + ctx->L.off_links, G.links.data(), sizeof(DevLink) * nl,
                                  hipMemcpyHostToDevice, ctx->stream), "copy links");
      if (arith64(ctx->p.storage))
        wall_records<double>(G.links, dg, &walls);
      else
        wall_records<float>(G.links, dg, &walls);
      HIP_TRY(ctx, hipMemcpyAsync(ctx->ws + ctx->L.off_walls, walls.data(), walls.size(), hipMemcpyHostToDevice,
                                  ctx->stream), "copy wall records");
    }
    if (ns)
      HIP_TRY(ctx, hipMemcpyAsync(ctx->ws + ctx->L.off_special, G.special.data(), sizeof(DevSpecial) * ns,
                                  hipMemcpyHostToDevice, ctx->stream), "copy boundary nodes");
  }
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "geometry upload");
  ctx->geom = G.any;
  ctx->nlinks = nl;
  ctx->nspecial = ns;
  ctx->host_links = std::move(G.links);
  if (ctx->initialized) return rebuild_side(ctx);
  return LBM_OK;
}

lbm_status lbm_get_links(lbm_ctx *ctx, lbm_link *out, int64_t cap, int64_t *count) {
  CTX_CHECK(ctx);
  if (lbm_status st = activate(ctx)) return st;
  if (count) *count = ctx->nlinks;
  if (!out || cap <= 0 || ctx->nlinks == 0) return LBM_OK;
  const int64_t m = cap < ctx->nlinks ? cap : ctx->nlinks;
  HIP_TRY(ctx, hipMemcpyAsync(out, ctx->ws + ctx->L.off_links, sizeof(lbm_link) * m, hipMemcpyDeviceToHost,
                              ctx->stream), "copy links to host");
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "copy links to host");
  return LBM_OK;
}

lbm_status lbm_set_velocity(lbm_ctx *ctx, const void *u_dev) {
  CTX_CHECK(ctx);
  ctx->uvel = u_dev;
  return LBM_OK;
}

lbm_status lbm_set_source(lbm_ctx *ctx, const void *Q_dev) {
  CTX_CHECK(ctx);
  if (!ctx->p.with_source) {
    set_err(&ctx->err, "context was created with with_source = 0");
    return LBM_EINVAL;
  }
  ctx->src = Q_dev;
  return LBM_OK;
}

lbm_status lbm_init_equilibrium(lbm_ctx *ctx, const double *rho_dev, const double *u_dev, const double *H_dev) {
  CTX_CHECK(ctx);
  if (!H_dev) {
    set_err(&ctx->err, "H must not be NULL");
    return LBM_EINVAL;
  }
  if (lbm_status st = activate(ctx)) return st;
  InitArgs a;
  memset(&a, 0, sizeof(a));
  ctx->cur = 0;
  ctx->phase = 0;
  a.fdst = ctx->p.with_ns ? ctx->pop(0, 0) : nullptr;
  a.hdst = ctx->pop(1, 0);
  a.rho = rho_dev;
  a.u = u_dev;
  a.uvel = (!ctx->p.with_ns && ctx->p.u_mode == 1) ? ctx->uvel : nullptr;
  if (!u_dev && !ctx->p.with_ns && ctx->p.u_mode == 1 && !ctx->uvel) {
    set_err(&ctx->err, "u_mode = 1: set the velocity field before lbm_init_equilibrium or pass u");
    return LBM_ESTATE;
  }
  a.H = H_dev;
  a.n = ctx->n;
  a.ps = ctx->L.ps;
  a.nx = ctx->p.nx;
  a.ny = ctx->p.ny;
  a.nz = ctx->p.nz;
  for (int d = 0; d < 3; d++) a.u0[d] = ctx->p.u0[d];
  const bool dev = deviations(ctx->p.storage);
  a.fref = dev ? ctx->p.rho_ref : 0.0;
  a.href = dev ? ctx->p.H_ref : 0.0;
  HIP_TRY(ctx, launch_init(ctx->Q, ctx->p.storage, ctx->p.with_ns, ctx->lay(), a, ctx->stream),
          "init kernel launch");
  ctx->t = 0;
  ctx->initialized = true;
  return rebuild_side(ctx);
}

lbm_status lbm_step(lbm_ctx *ctx, int32_t nsteps) {
  CTX_CHECK(ctx);
  if (nsteps < 0) {
    set_err(&ctx->err, "nsteps must be >= 0 (got %d)", nsteps);
    return LBM_EINVAL;
  }
  if (lbm_status st = need_ready(ctx)) return st;
  if (lbm_status st = activate(ctx)) return st;
  for (int s = 0; s < nsteps; s++) {
    KArgs a = make_args(ctx, ctx->cur);
    if (lbm_status st = run_pass(ctx, MODE_STEP, a)) return st;
    if (ctx->aa())
      ctx->phase ^= 1;
    else
      ctx->cur ^= 1;
    ctx->t++;
  }
  return LBM_OK;
}

lbm_status lbm_macroscopic(lbm_ctx *ctx, double *rho_dev, double *u_dev, double *H_dev) {
  CTX_CHECK(ctx);
  if (lbm_status st = need_ready(ctx)) return st;
  if (lbm_status st = activate(ctx)) return st;
  KArgs a = make_args(ctx, ctx->cur);
  a.out0 = rho_dev;
  a.out1 = u_dev;
  a.out2 = H_dev;
  a.out3 = nullptr;
  a.link_flux = reinterpret_cast<double *>(ctx->ws + ctx->L.off_flux);
  return run_pass(ctx, MODE_MACRO, a);
}

lbm_status lbm_get_populations(lbm_ctx *ctx, int32_t lattice, int32_t which, double *dst_dev) {
  CTX_CHECK(ctx);
  if (lattice != 0 && lattice != 1) {
    set_err(&ctx->err, "lattice must be 0 (f) or 1 (h), got %d", lattice);
    return LBM_EINVAL;
  }
  if (lattice == 0 && !ctx->p.with_ns) {
    set_err(&ctx->err, "no f lattice (with_ns = 0)");
    return LBM_EINVAL;
  }
  if ((which != 0 && which != 1) || !dst_dev) {
    set_err(&ctx->err, "which must be 0 (pre-collision) or 1 (stored post-collision), dst non-NULL");
    return LBM_EINVAL;
  }
  if (lbm_status st = need_ready(ctx)) return st;
  if (lbm_status st = activate(ctx)) return st;
  const bool dev = deviations(ctx->p.storage);
  if (which == 1) {
    const double ref = dev ? (lattice == 0 ? ctx->p.rho_ref : ctx->p.H_ref) : 0.0;
    KArgs a = make_args(ctx, ctx->cur);
    HIP_TRY(ctx, launch_convert(ctx->Q, ctx->p.storage, ctx->lay(), false, a, ctx->pop(lattice, ctx->cur), dst_dev,
                                ref, ctx->stream), "convert kernel launch");
    return LBM_OK;
  }
  KArgs a = make_args(ctx, ctx->cur);
  a.out0 = lattice == 0 ? dst_dev : nullptr;
  a.out1 = lattice == 1 ? dst_dev : nullptr;
  return run_pass(ctx, MODE_PRE, a);
}

lbm_status lbm_set_populations(lbm_ctx *ctx, int32_t lattice, const double *src_dev, int64_t t) {
  CTX_CHECK(ctx);
  if ((lattice != 0 && lattice != 1) || (lattice == 0 && !ctx->p.with_ns) || !src_dev) {
    set_err(&ctx->err, "invalid lattice %d or NULL source", lattice);
    return LBM_EINVAL;
  }
  if (lbm_status st = activate(ctx)) return st;
  const bool dev = deviations(ctx->p.storage);
  const double ref = dev ? (lattice == 0 ? ctx->p.rho_ref : ctx->p.H_ref) : 0.0;
  KArgs a = make_args(ctx, ctx->cur);
  a.cls = nullptr;
  a.sr_seed = sr_seed(t);
  HIP_TRY(ctx, launch_convert(ctx->Q, ctx->p.storage, ctx->lay(), true, a, src_dev, ctx->pop(lattice, ctx->cur), ref,
                              ctx->stream), "convert kernel launch");
  ctx->t = t;
  ctx->initialized = true;
  return rebuild_side(ctx);
}

// Reductions of lbm_reduce with their scratch (partials of the first pass,
// the device result vector, the device column list) at the given addresses.
static lbm_status reduce_impl(lbm_ctx *ctx, int32_t group, const int32_t *columns, int32_t n_columns, double *out,
                              int32_t nout, double *part, int npart, double *res, int32_t *cols) {
  CTX_CHECK(ctx);
  if (n_columns < 0 || n_columns > kMaxColumns || (n_columns > 0 && !columns)) {
    set_err(&ctx->err, "n_columns must be in [0, %d]", kMaxColumns);
    return LBM_EINVAL;
  }
  if (!out || nout < 3 + n_columns) {
    set_err(&ctx->err, "out needs at least 3 + n_columns = %d entries", 3 + n_columns);
    return LBM_EINVAL;
  }
  for (int j = 0; j < n_columns; j++)
    if (columns[j] < 0 || columns[j] >= ctx->p.nx) {
      set_err(&ctx->err, "columns[%d] = %d outside [0, nx)", j, columns[j]);
      return LBM_EINVAL;
    }
  if (lbm_status st = need_ready(ctx)) return st;
  if (lbm_status st = activate(ctx)) return st;
  double *rho = reinterpret_cast<double *>(ctx->ws + ctx->L.off_rho);
  double *H = reinterpret_cast<double *>(ctx->ws + ctx->L.off_H);
  double *qx = reinterpret_cast<double *>(ctx->ws + ctx->L.off_qx);
  double *flux = reinterpret_cast<double *>(ctx->ws + ctx->L.off_flux);
  KArgs a = make_args(ctx, ctx->cur);
  a.out0 = ctx->p.with_ns ? rho : nullptr;
  a.out2 = H;
  a.out3 = qx;
  a.link_flux = flux;
  if (lbm_status st = run_pass(ctx, MODE_MACRO, a)) return st;
  ctx->host_cols.assign(columns, columns + n_columns);
  if (n_columns)
    HIP_TRY(ctx, hipMemcpyAsync(cols, ctx->host_cols.data(), sizeof(int32_t) * n_columns, hipMemcpyHostToDevice,
                                ctx->stream), "copy columns");
  HIP_TRY(ctx, launch_reduce(ctx->p.with_ns ? rho : nullptr, H, qx, ctx->n, ctx->p.nx, ctx->p.ny, ctx->p.nz, cols,
                             n_columns, flux, reinterpret_cast<const DevLink *>(ctx->ws + ctx->L.off_links),
                             ctx->geom ? ctx->nlinks : 0, group, part, npart, res, ctx->stream),
          "reduction launch");
  double host[3 + kMaxColumns];
  HIP_TRY(ctx, hipMemcpyAsync(host, res, sizeof(double) * (3 + n_columns), hipMemcpyDeviceToHost, ctx->stream),
          "copy reductions");
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "reduction");
  memcpy(out, host, sizeof(double) * (3 + n_columns));
  if (!std::isfinite(out[0]) || !std::isfinite(out[1])) {
    set_err(&ctx->err, "non-finite mass or energy sum (mass %g, energy %g) at t = %lld", out[0], out[1],
            (long long)ctx->t);
    return LBM_EDIVERGED;
  }
  return LBM_OK;
}

lbm_status lbm_reduce(lbm_ctx *ctx, int32_t group, const int32_t *columns, int32_t n_columns, double *out,
                      int32_t nout) {
  CTX_CHECK(ctx);
  return reduce_impl(ctx, group, columns, n_columns, out, nout,
                     reinterpret_cast<double *>(ctx->ws + ctx->L.off_part), kPartials,
                     reinterpret_cast<double *>(ctx->ws + ctx->L.off_res),
                     reinterpret_cast<int32_t *>(ctx->ws + ctx->L.off_cols));
}

lbm_status lbm_device_copy(void *dst_dev, const void *src_dev, size_t bytes, int32_t blocks, void *hip_stream) {
  if (!dst_dev || !src_dev || bytes % 16 != 0 || reinterpret_cast<uintptr_t>(dst_dev) % 16 != 0 ||
      reinterpret_cast<uintptr_t>(src_dev) % 16 != 0 || blocks < 0) {
    set_err(nullptr, "lbm_device_copy: needs non-NULL 16-byte aligned pointers, a multiple of 16 bytes and "
            "blocks >= 0");
    return LBM_EINVAL;
  }
  const hipError_t e = launch_copy16(src_dev, dst_dev, (int64_t)(bytes / 16), blocks,
                                     static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) {
    set_err(nullptr, "lbm_device_copy launch: %s", hipGetErrorString(e));
    return LBM_EDEVICE;
  }
  return LBM_OK;
}

lbm_status lbm_reduce_noalloc(lbm_ctx *ctx, int32_t group, const int32_t *columns, int32_t n_columns, double *out,
                              int32_t nout) {
  CTX_CHECK(ctx);
  static_assert(kScratchPartials == kPartials && kScratchColumns == kMaxColumns, "scratch sizes");
  if (n_columns > kScratchColumns) {
    set_err(&ctx->err, "n_columns = %d exceeds the static scratch (at most %d columns)", n_columns,
            kScratchColumns);
    return LBM_EINVAL;
  }
  if (!g_scratch_set[ctx->device]) {
    set_err(&ctx->err, "static scratch not set up on device %d", ctx->device);
    return LBM_ESTATE;
  }
  char *base = static_cast<char *>(g_scratch_ptr[ctx->device]);
  double *part = reinterpret_cast<double *>(base);
  double *res = part + 2 * kScratchPartials;
  int32_t *cols = reinterpret_cast<int32_t *>(res + 3 + kScratchColumns);
  return reduce_impl(ctx, group, columns, n_columns, out, nout, part, kScratchPartials, res, cols);
}

lbm_status lbm_nusselt(lbm_ctx *ctx, int32_t group, int32_t x_in, int32_t x_out, double T_wall, double T_in,
                       double *out, int32_t nout) {
  CTX_CHECK(ctx);
  if (!out || nout < 5) {
    set_err(&ctx->err, "out needs at least 5 entries");
    return LBM_EINVAL;
  }
  if (!(ctx->p.k > 0.0) || !std::isfinite(ctx->p.k)) {
    set_err(&ctx->err, "the context's conductivity k = %g must be finite and > 0", ctx->p.k);
    return LBM_EINVAL;
  }
  if (!std::isfinite(T_wall) || !std::isfinite(T_in) || T_wall == T_in) {
    set_err(&ctx->err, "T_wall (%g) and T_in (%g) must be finite and differ", T_wall, T_in);
    return LBM_EINVAL;
  }
  const int32_t cols[2] = {x_in, x_out};
  double red[5];
  if (lbm_status st = lbm_reduce(ctx, group, cols, 2, red, 5)) return st;
  // Sec. 4.4: Nu = varsigma D / k with varsigma = qdot / (pi D (T_wall - T_in))
  // per unit depth (nz layers), qdot the mean of the heater flux and the
  // energy the flow gains between the two sections
  const double q_s = red[2], q_in = red[3], q_out = red[4];
  const double scale = M_PI * ctx->p.k * (T_wall - T_in) * (double)ctx->p.nz;
  out[0] = 0.5 * (q_s + q_out - q_in) / scale;
  out[1] = q_s / scale;
  out[2] = q_s;
  out[3] = q_in;
  out[4] = q_out;
  return LBM_OK;
}

static lbm_status need_adjoint(lbm_ctx *ctx) {
  if (ctx->p.with_ns || (ctx->p.cumulant & 1) || ctx->p.storage == LBM_FP32_SR || ctx->p.storage == LBM_FP16_SR) {
    set_err(&ctx->err, "the adjoint is built for advection-only contexts with the central-moment collision "
                       "(storage other than LBM_FP32_SR and LBM_FP16_SR)");
    return LBM_EUNSUPPORTED;
  }
  if (ctx->p.u_mode == 1 && !ctx->uvel) {
    set_err(&ctx->err, "u_mode = 1 but no velocity field set (lbm_set_velocity)");
    return LBM_ESTATE;
  }
  return LBM_OK;
}

lbm_status lbm_objective(lbm_ctx *ctx, const double *H_target_dev, void *lambda_dev, void *dJdQ_dev, double *J) {
  CTX_CHECK(ctx);
  if (!H_target_dev || !lambda_dev || !dJdQ_dev) {
    set_err(&ctx->err, "H_target, lambda and dJdQ must not be NULL");
    return LBM_EINVAL;
  }
  if (lbm_status st = need_adjoint(ctx)) return st;
  if (lbm_status st = need_ready(ctx)) return st;
  if (lbm_status st = activate(ctx)) return st;
  double *H = reinterpret_cast<double *>(ctx->ws + ctx->L.off_H);
  double *sq = reinterpret_cast<double *>(ctx->ws + ctx->L.off_qx);
  double *res = reinterpret_cast<double *>(ctx->ws + ctx->L.off_res);
  KArgs a = make_args(ctx, ctx->cur);
  a.out2 = H;
  if (lbm_status st = run_pass(ctx, MODE_MACRO, a)) return st;
  HIP_TRY(ctx, launch_seed(ctx->Q, ctx->p.storage == LBM_FP64, H, H_target_dev, a.cls, ctx->n, lambda_dev, dJdQ_dev, sq,
                           ctx->stream), "seed kernel launch");
  HIP_TRY(ctx, launch_reduce(nullptr, sq, nullptr, ctx->n, ctx->p.nx, ctx->p.ny, ctx->p.nz, nullptr, 0, nullptr,
                             nullptr, 0, 0, reinterpret_cast<double *>(ctx->ws + ctx->L.off_part), kPartials, res,
                             ctx->stream), "reduction launch");
  double host[3];
  HIP_TRY(ctx, hipMemcpyAsync(host, res, sizeof(host), hipMemcpyDeviceToHost, ctx->stream), "copy objective");
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "objective");
  if (J) *J = 0.5 * host[1];
  return LBM_OK;
}

lbm_status lbm_objective_residual(lbm_ctx *ctx, const double *H_target_dev, double *resid_dev, double *J) {
  CTX_CHECK(ctx);
  if (!H_target_dev || !resid_dev) {
    set_err(&ctx->err, "H_target and resid must not be NULL");
    return LBM_EINVAL;
  }
  if (lbm_status st = need_adjoint(ctx)) return st;
  if (lbm_status st = need_ready(ctx)) return st;
  if (lbm_status st = activate(ctx)) return st;
  double *H = reinterpret_cast<double *>(ctx->ws + ctx->L.off_H);
  double *sq = reinterpret_cast<double *>(ctx->ws + ctx->L.off_qx);
  double *res = reinterpret_cast<double *>(ctx->ws + ctx->L.off_res);
  KArgs a = make_args(ctx, ctx->cur);
  a.out2 = H;
  if (lbm_status st = run_pass(ctx, MODE_MACRO, a)) return st;
  HIP_TRY(ctx, launch_resid(H, H_target_dev, a.cls, ctx->n, resid_dev, sq, ctx->stream), "residual kernel launch");
  HIP_TRY(ctx, launch_reduce(nullptr, sq, nullptr, ctx->n, ctx->p.nx, ctx->p.ny, ctx->p.nz, nullptr, 0, nullptr,
                             nullptr, 0, 0, reinterpret_cast<double *>(ctx->ws + ctx->L.off_part), kPartials, res,
                             ctx->stream), "reduction launch");
  double host[3];
  HIP_TRY(ctx, hipMemcpyAsync(host, res, sizeof(host), hipMemcpyDeviceToHost, ctx->stream), "copy objective");
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "objective");
  if (J) *J = 0.5 * host[1];
  return LBM_OK;
}

lbm_status lbm_adjoint_seed(lbm_ctx *ctx, const double *resid_dev, void *lambda_dev, void *dJdQ_dev,
                            int32_t accumulate) {
  CTX_CHECK(ctx);
  if (!resid_dev || !lambda_dev || !dJdQ_dev) {
    set_err(&ctx->err, "resid, lambda and dJdQ must not be NULL");
    return LBM_EINVAL;
  }
  if (lbm_status st = need_adjoint(ctx)) return st;
  if (lbm_status st = activate(ctx)) return st;
  HIP_TRY(ctx, launch_seed_add(ctx->Q, ctx->p.storage == LBM_FP64, accumulate != 0, resid_dev, ctx->n, lambda_dev,
                               static_cast<double *>(dJdQ_dev), ctx->stream),
          "seed kernel launch");
  return LBM_OK;
}

lbm_status lbm_adjoint_step(lbm_ctx *ctx, const void *lambda_next_dev, void *lambda_prev_dev, void *dJdQ_dev) {
  CTX_CHECK(ctx);
  if (!lambda_next_dev || !lambda_prev_dev || lambda_next_dev == lambda_prev_dev) {
    set_err(&ctx->err, "lambda_next and lambda_prev must be distinct non-NULL buffers");
    return LBM_EINVAL;
  }
  if (lbm_status st = need_adjoint(ctx)) return st;
  if (lbm_status st = activate(ctx)) return st;
  KArgs a = make_args(ctx, ctx->cur);
  HIP_TRY(ctx, launch_adjoint(ctx->Q, ctx->p.storage == LBM_FP64, a, lambda_next_dev, lambda_prev_dev, dJdQ_dev,
                              ctx->stream), "adjoint kernel launch");
  return LBM_OK;
}

size_t lbm_state_bytes(const lbm_ctx *ctx) {
  if (!ctx) return 0;
  return kAlign + ctx->L.region_bytes;
}

lbm_status lbm_save_state(lbm_ctx *ctx, void *dst_dev) {
  CTX_CHECK(ctx);
  if (!dst_dev) {
    set_err(&ctx->err, "dst is NULL");
    return LBM_EINVAL;
  }
  if (lbm_status st = need_ready(ctx)) return st;
  if (lbm_status st = activate(ctx)) return st;
  ctx->hdr.magic = 0x4c424d5354415445LL;
  ctx->hdr.t = ctx->t;
  ctx->hdr.Q = ctx->Q;
  ctx->hdr.n = ctx->n;
  ctx->hdr.storage = ctx->p.storage | (ctx->p.stream << 8);
  ctx->hdr.with_ns = ctx->p.with_ns;
  ctx->hdr.bytes = (int64_t)lbm_state_bytes(ctx);
  ctx->hdr.phase = ctx->aa() ? ctx->phase : 0;
  char *d = static_cast<char *>(dst_dev);
  HIP_TRY(ctx, hipMemcpyAsync(d, &ctx->hdr, sizeof(ctx->hdr), hipMemcpyHostToDevice, ctx->stream), "save header");
  HIP_TRY(ctx, hipMemcpyAsync(d + kAlign, ctx->ws + ctx->L.off_region[ctx->cur], ctx->L.region_bytes,
                              hipMemcpyDeviceToDevice, ctx->stream), "save populations");
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "save state");
  return LBM_OK;
}

lbm_status lbm_load_state(lbm_ctx *ctx, const void *src_dev) {
  CTX_CHECK(ctx);
  if (!src_dev) {
    set_err(&ctx->err, "src is NULL");
    return LBM_EINVAL;
  }
  if (lbm_status st = activate(ctx)) return st;
  decltype(ctx->hdr) h;
  HIP_TRY(ctx, hipMemcpyAsync(&h, src_dev, sizeof(h), hipMemcpyDeviceToHost, ctx->stream), "load header");
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "load header");
  if (h.magic != 0x4c424d5354415445LL || h.Q != ctx->Q || h.n != ctx->n ||
      h.storage != (ctx->p.storage | (ctx->p.stream << 8)) ||
      h.with_ns != ctx->p.with_ns || h.bytes != (int64_t)lbm_state_bytes(ctx)) {
    set_err(&ctx->err, "snapshot does not match this context (lattice, size, storage, layout or lattices differ)");
    return LBM_EINVAL;
  }
  const char *s = static_cast<const char *>(src_dev);
  HIP_TRY(ctx, hipMemcpyAsync(ctx->ws + ctx->L.off_region[ctx->cur], s + kAlign, ctx->L.region_bytes,
                              hipMemcpyDeviceToDevice, ctx->stream), "load populations");
  ctx->t = h.t;
  ctx->phase = ctx->aa() ? (int)(h.phase & 1) : 0;
  ctx->initialized = true;
  return rebuild_side(ctx);
}

int64_t lbm_time(const lbm_ctx *ctx) { return ctx ? ctx->t : -1; }

lbm_status lbm_profile_begin(lbm_ctx *ctx, int32_t max_steps) {
  CTX_CHECK(ctx);
  if (max_steps < 0 || max_steps > (1 << 20)) {
    set_err(&ctx->err, "max_steps must be in [0, 2^20]");
    return LBM_EINVAL;
  }
  if (lbm_status st = activate(ctx)) return st;
  const size_t need = 3 * (size_t)max_steps;
  while (ctx->ev.size() < need) {
    hipEvent_t e;
    HIP_TRY(ctx, hipEventCreate(&e), "hipEventCreate");
    ctx->ev.push_back(e);
  }
  ctx->ev_used = 0;
  ctx->profiling = max_steps > 0;
  return LBM_OK;
}

lbm_status lbm_profile_end(lbm_ctx *ctx, double *bulk_ms, double *boundary_ms, int64_t *steps) {
  CTX_CHECK(ctx);
  if (lbm_status st = activate(ctx)) return st;
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "stream synchronise");
  double b = 0.0, s = 0.0;
  for (int64_t i = 0; i + 3 <= ctx->ev_used; i += 3) {
    float t0 = 0.f, t1 = 0.f;
    HIP_TRY(ctx, hipEventElapsedTime(&t0, ctx->ev[i], ctx->ev[i + 1]), "hipEventElapsedTime");
    HIP_TRY(ctx, hipEventElapsedTime(&t1, ctx->ev[i + 1], ctx->ev[i + 2]), "hipEventElapsedTime");
    b += t0;
    s += t1;
  }
  if (bulk_ms) *bulk_ms = b;
  if (boundary_ms) *boundary_ms = s;
  if (steps) *steps = ctx->ev_used / 3;
  ctx->profiling = false;
  ctx->ev_used = 0;
  return LBM_OK;
}

lbm_status lbm_sync(lbm_ctx *ctx) {
  CTX_CHECK(ctx);
  if (lbm_status st = activate(ctx)) return st;
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "stream synchronise");
  return LBM_OK;
}

}  // extern "C"
