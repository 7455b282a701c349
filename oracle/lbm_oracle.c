/*
 * lbm_oracle.c -- plain FP64 CPU oracle of the central-moment lattice
 * Boltzmann stream-and-collide step (D2Q9 and D3Q27, advection-diffusion
 * lattice h and optional hydrodynamic lattice f, wall/EQ/outlet nodes).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this file's library.  It shares
 * no code, table or header with the GPU library: every table below is typed
 * from the paper, every matrix is built from its defining formula.
 *
 * Written for clarity, not speed: the collision builds the dense transform
 * T(u) of the central moments for every node and multiplies it out; the
 * back-transform uses the inverse of the raw-moment matrix M (computed once by
 * Gauss-Jordan elimination) and the binomial shift N(-u) = N(u)^-1.
 *
 * Paper: Gruszczynski & Laniewski-Wollk, "A comparative study of 3D Cumulant
 * and Central Moments lattice Boltzmann schemes with interpolated boundary
 * conditions for the simulation of thermal flows in high Prandtl number
 * regime" (arXiv 2203.01316).
 *
 * Readings where the paper is silent (all also listed in the design notes):
 *   - hydrodynamic lattice f uses the same central-moment collision with psi =
 *     rho (App. A), second-order moments relaxed at s_nu, all others at 1;
 *   - canonical state is the pre-collision, post-stream population set;
 *   - initial post-collision state is the equilibrium field "pre-streamed"
 *     backwards, so that streaming it reproduces the equilibrium in the bulk;
 *   - u in the wall term of IABB/ABB is the velocity of the boundary node at
 *     the time of the post-collision values (prescribed field, or momentum
 *     over density of the post-collision f);
 *   - EQ is node-wise, the outlet is a zero-gradient copy of the unknown
 *     (e_x < 0) populations from the upstream neighbour;
 *   - source term in central-moment space adds (1 - s_000/2) Q to the zeroth
 *     moment, with the equilibrium evaluated at H = sum(h) + Q/2 (App. D).
 */
#include <math.h>
#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_MAXQ 27

/* Threads the node loops may use (1 without OpenMP). */
int ora_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Sets the threads the node loops use (timing only; results do not depend on
 * it).  Returns the previous count. */
int ora_set_threads(int n) {
  const int prev = ora_threads();
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
  return prev;
}

/* ---------------------------------------------------------------------------
 * Velocity sets and moment orders.
 * D3Q27 velocities in the paper's order (Sec. 2.1, vectors e_x, e_y, e_z).
 * ------------------------------------------------------------------------- */
static const int EX27[27] = {0, 1, 0, 0, 1, 1, 0, -1, 0, 0, 1, 1, -1, -1,
                             0, 0, 1, -1, -1, 0, -1, 1, 1, 1, -1, -1, -1};
static const int EY27[27] = {0, 0, 1, 0, 1, 0, 1, 0, -1, 0, -1, 0, 1, 0,
                             1, -1, 1, -1, 0, -1, 1, -1, 1, -1, 1, -1, -1};
static const int EZ27[27] = {0, 0, 0, 1, 0, 1, 1, 0, 0, -1, 0, -1, 0, 1,
                             -1, 1, 1, 0, -1, -1, 1, 1, -1, -1, -1, 1, -1};

/* Moment order of Sec. 2.1 (three-indices m n o, each below 3). */
static const char *MOM27[27] = {"000", "100", "010", "001", "110", "101", "011",
                                "200", "020", "002", "120", "102", "210", "201",
                                "012", "021", "111", "220", "202", "022", "211",
                                "121", "112", "122", "212", "221", "222"};
/* D2Q9 moment order of App. A. */
static const char *MOM9[9] = {"00", "10", "01", "20", "02", "11", "21", "12", "22"};

typedef struct {
  int Q;
  int e[ORA_MAXQ][3];
  int opp[ORA_MAXQ];
  int mo[ORA_MAXQ][3];
} ora_lat;

/* D2Q9 is the restriction of the D3Q27 set to e_z = 0, in the D3Q27 order
 * (Sec. 2.1: restrictions to two dimensions follow from the same formulas). */
static int build_lattice(int Q, ora_lat *L) {
  int k = 0;
  if (Q != 9 && Q != 27) return -1;
  L->Q = Q;
  for (int a = 0; a < 27; a++) {
    if (Q == 9 && EZ27[a] != 0) continue;
    L->e[k][0] = EX27[a];
    L->e[k][1] = EY27[a];
    L->e[k][2] = EZ27[a];
    k++;
  }
  if (k != Q) return -1;
  for (int a = 0; a < Q; a++) {
    L->opp[a] = -1;
    for (int b = 0; b < Q; b++)
      if (L->e[b][0] == -L->e[a][0] && L->e[b][1] == -L->e[a][1] &&
          L->e[b][2] == -L->e[a][2])
        L->opp[a] = b;
    if (Q == 27) {
      for (int d = 0; d < 3; d++) L->mo[a][d] = MOM27[a][d] - '0';
    } else {
      L->mo[a][0] = MOM9[a][0] - '0';
      L->mo[a][1] = MOM9[a][1] - '0';
      L->mo[a][2] = 0;
    }
  }
  return 0;
}

int ora_lattice(int Q, int *e, int *opp, int *mo) {
  ora_lat L;
  if (build_lattice(Q, &L)) return -1;
  for (int a = 0; a < Q; a++) {
    for (int d = 0; d < 3; d++) {
      e[3 * a + d] = L.e[a][d];
      mo[3 * a + d] = L.mo[a][d];
    }
    opp[a] = L.opp[a];
  }
  return 0;
}

static double ipow(double x, int m) {
  double r = 1.0;
  for (int i = 0; i < m; i++) r *= x;
  return r;
}

/* ---------------------------------------------------------------------------
 * Transform matrices (App. C): M_{mno,a} = ex^m ey^n ez^o and
 * T_{mno,a} = (ex-ux)^m (ey-uy)^n (ez-uz)^o.  Row-major Q x Q.
 * ------------------------------------------------------------------------- */
static void matrix_T(const ora_lat *L, const double u[3], double *T) {
  int Q = L->Q;
  for (int k = 0; k < Q; k++)
    for (int a = 0; a < Q; a++) {
      double v = 1.0;
      for (int d = 0; d < 3; d++) v *= ipow((double)L->e[a][d] - u[d], L->mo[k][d]);
      T[k * Q + a] = v;
    }
}

/* Binomial shift between raw and central moments (Eq. to_cmom):
 * (e-u)^m = sum_j C(m,j) e^j (-u)^(m-j), so N(u)_{mno,jkl} =
 * prod_d C(m_d, j_d) (-u_d)^(m_d - j_d) for j_d <= m_d.  Since the moment set
 * is closed under lowering an index, N(u) N(-u) = 1. */
static double binom(int m, int j) {
  if (j < 0 || j > m) return 0.0;
  if (m == 2 && j == 1) return 2.0;
  return 1.0;
}

static void matrix_N(const ora_lat *L, const double u[3], double *N) {
  int Q = L->Q;
  for (int k = 0; k < Q; k++)
    for (int c = 0; c < Q; c++) {
      double v = 1.0;
      for (int d = 0; d < 3; d++) {
        int m = L->mo[k][d], j = L->mo[c][d];
        if (j > m) {
          v = 0.0;
          break;
        }
        v *= binom(m, j) * ipow(-u[d], m - j);
      }
      N[k * Q + c] = v;
    }
}

/* Gauss-Jordan inverse with partial pivoting. Returns 0 on success. */
static int invert(int n, const double *A, double *Ainv) {
  double W[ORA_MAXQ][2 * ORA_MAXQ];
  for (int i = 0; i < n; i++)
    for (int j = 0; j < 2 * n; j++)
      W[i][j] = j < n ? A[i * n + j] : (j - n == i ? 1.0 : 0.0);
  for (int c = 0; c < n; c++) {
    int p = c;
    for (int r = c + 1; r < n; r++)
      if (fabs(W[r][c]) > fabs(W[p][c])) p = r;
    if (W[p][c] == 0.0) return -1;
    if (p != c)
      for (int j = 0; j < 2 * n; j++) {
        double t = W[p][j];
        W[p][j] = W[c][j];
        W[c][j] = t;
      }
    double piv = W[c][c];
    for (int j = 0; j < 2 * n; j++) W[c][j] /= piv;
    for (int r = 0; r < n; r++) {
      if (r == c || W[r][c] == 0.0) continue;
      double f = W[r][c];
      for (int j = 0; j < 2 * n; j++) W[r][j] -= f * W[c][j];
    }
  }
  for (int i = 0; i < n; i++)
    for (int j = 0; j < n; j++) Ainv[i * n + j] = W[i][n + j];
  return 0;
}

int ora_matrix_M(int Q, double *M) {
  ora_lat L;
  double z[3] = {0, 0, 0};
  if (build_lattice(Q, &L)) return -1;
  matrix_T(&L, z, M); /* T(0) is M by definition */
  return 0;
}

int ora_matrix_T(int Q, const double *u, double *T) {
  ora_lat L;
  if (build_lattice(Q, &L)) return -1;
  matrix_T(&L, u, T);
  return 0;
}

int ora_matrix_N(int Q, const double *u, double *N) {
  ora_lat L;
  if (build_lattice(Q, &L)) return -1;
  matrix_N(&L, u, N);
  return 0;
}

int ora_matrix_Minv(int Q, double *Minv) {
  double M[ORA_MAXQ * ORA_MAXQ];
  if (ora_matrix_M(Q, M)) return -1;
  return invert(Q, M, Minv);
}

/* ---------------------------------------------------------------------------
 * Central-moment equilibrium (Sec. 2.1.1 vector for h, App. A with psi =
 * density or internal energy): nonzero only at 000 (psi), 200/020/002
 * (psi cs^2), 220/202/022 (psi cs^4) and 222 (psi cs^6), cs^2 = 1/3.
 * ------------------------------------------------------------------------- */
static const double CS2 = 1.0 / 3.0;

static void cm_equilibrium(const ora_lat *L, double psi, double *eq) {
  for (int k = 0; k < L->Q; k++) {
    const int *m = L->mo[k];
    int n2 = 0, odd_or_one = 0;
    for (int d = 0; d < 3; d++) {
      if (m[d] == 1) odd_or_one = 1;
      if (m[d] == 2) n2++;
    }
    eq[k] = odd_or_one ? 0.0 : psi * ipow(CS2, n2);
  }
}

typedef struct {
  ora_lat L;
  double Minv[ORA_MAXQ * ORA_MAXQ];
} ora_ctx;

/* Position of the moment with multi-index n in the lattice's moment order. */
static int mom_slot(const ora_lat *L, const int n[3]) {
  for (int k = 0; k < L->Q; k++)
    if (L->mo[k][0] == n[0] && L->mo[k][1] == n[1] && L->mo[k][2] == n[2]) return k;
  return -1;
}

static int ctx_init(int Q, ora_ctx *C) {
  if (build_lattice(Q, &C->L)) return -1;
  return ora_matrix_Minv(Q, C->Minv);
}

/* g = M^-1 N(u)^-1 Y~ with N(u)^-1 = N(-u). */
static void from_central(const ora_ctx *C, const double u[3], const double *cm, double *g) {
  int Q = C->L.Q;
  double N[ORA_MAXQ * ORA_MAXQ], raw[ORA_MAXQ];
  double mu[3] = {-u[0], -u[1], -u[2]};
  matrix_N(&C->L, mu, N);
  for (int k = 0; k < Q; k++) {
    double s = 0.0;
    for (int c = 0; c < Q; c++) s += N[k * Q + c] * cm[c];
    raw[k] = s;
  }
  for (int a = 0; a < Q; a++) {
    double s = 0.0;
    for (int k = 0; k < Q; k++) s += C->Minv[a * Q + k] * raw[k];
    g[a] = s;
  }
}

/* Discrete equilibrium (Eq. dedf_full_u): g^eq = M^-1 N^-1 Y~^eq. */
static void equilibrium(const ora_ctx *C, double psi, const double u[3], double *geq) {
  double eq[ORA_MAXQ];
  cm_equilibrium(&C->L, psi, eq);
  from_central(C, u, eq, geq);
}

int ora_equilibrium(int Q, double psi, const double *u, double *geq) {
  ora_ctx C;
  if (ctx_init(Q, &C)) return -1;
  equilibrium(&C, psi, u, geq);
  return 0;
}

int ora_cm_equilibrium(int Q, double psi, double *eq) {
  ora_lat L;
  if (build_lattice(Q, &L)) return -1;
  cm_equilibrium(&L, psi, eq);
  return 0;
}

/* Relaxation of a moment (or cumulant) vector v toward its equilibrium veq
 * with the diagonal rates s.  With s_bulk > 0 the second-order diagonal block
 * (200, 020, 002; 20, 02 in two dimensions) is relaxed in the basis of its
 * trace and its deviatoric parts instead: the trace t = sum_d v_dd at
 * s_bulk, the differences v_xx - v_dd (d != x) at s of 200, which must equal
 * those of 020 and 002.  The trace carries the bulk viscosity, the deviator
 * the shear viscosity (Geier et al. 2015, whose hydrodynamic kernel the paper
 * adopts, relaxes the two with separate rates). */
static void relax_moments(const ora_lat *L, double *v, const double *veq, const double *s, double s_bulk) {
  int Q = L->Q, D = Q == 27 ? 3 : 2;
  int dia[3] = {-1, -1, -1};
  double pre[ORA_MAXQ];
  for (int k = 0; k < Q; k++) {
    pre[k] = v[k];
    v[k] = v[k] + s[k] * (veq[k] - v[k]);
  }
  if (!(s_bulk > 0.0)) return;
  for (int d = 0; d < D; d++) {
    int n[3] = {0, 0, 0};
    n[d] = 2;
    dia[d] = mom_slot(L, n);
  }
  {
    double t = 0.0, teq = 0.0, dev[3], deveq[3], tpost, devpost[3];
    for (int d = 0; d < D; d++) {
      t += pre[dia[d]];
      teq += veq[dia[d]];
    }
    for (int d = 1; d < D; d++) {
      dev[d] = pre[dia[0]] - pre[dia[d]];
      deveq[d] = veq[dia[0]] - veq[dia[d]];
    }
    tpost = t + s_bulk * (teq - t);
    for (int d = 1; d < D; d++) devpost[d] = dev[d] + s[dia[0]] * (deveq[d] - dev[d]);
    /* invert t = v_x + sum_d v_d, dev_d = v_x - v_d:  D v_x = t + sum_d dev_d */
    {
      double vx = tpost;
      for (int d = 1; d < D; d++) vx += devpost[d];
      vx /= (double)D;
      v[dia[0]] = vx;
      for (int d = 1; d < D; d++) v[dia[d]] = vx - devpost[d];
    }
  }
}

/* One central-moment collision (Eq. H_cm_collision, relaxation of Sec. 2.1.1,
 * source of App. D carried over to central moments):
 *   Y~  = T(u) g
 *   psi = Y~_000 + src/2
 *   Y~* = Y~ + S (Y~eq(psi) - Y~) + (1 - s_000/2) src e_000
 *   g*  = M^-1 N(-u) Y~*
 * (S with the trace split of relax_moments when s_bulk > 0).               */
static void collide_node(const ora_ctx *C, const double *g, const double u[3],
                         const double *s, double s_bulk, double src, double *gs) {
  int Q = C->L.Q;
  double T[ORA_MAXQ * ORA_MAXQ], cm[ORA_MAXQ], eq[ORA_MAXQ];
  matrix_T(&C->L, u, T);
  for (int k = 0; k < Q; k++) {
    double v = 0.0;
    for (int a = 0; a < Q; a++) v += T[k * Q + a] * g[a];
    cm[k] = v;
  }
  cm_equilibrium(&C->L, cm[0] + 0.5 * src, eq);
  relax_moments(&C->L, cm, eq, s, s_bulk);
  cm[0] += (1.0 - 0.5 * s[0]) * src;
  from_central(C, u, cm, gs);
}

int ora_collide_node(int Q, const double *g, const double *u, const double *s,
                     double src, double s_bulk, double *gs) {
  ora_ctx C;
  if (ctx_init(Q, &C)) return -1;
  collide_node(&C, g, u, s, s_bulk, src, gs);
  return 0;
}

/* ---------------------------------------------------------------------------
 * Cumulants (Sec. 2.1.1, Eqs. hydro_cu_collision and H_cu_collision; the
 * transform of Geier et al. 2015 that the paper adopts).  For a population set
 * g with raw moments m_n = sum_a g_a e_a^n (multi-index n, every exponent
 * below 3) the zeroth cumulant is c_0 = m_0 and, for n != 0, c_n is the
 * cumulant of the normalised distribution g / m_0: the coefficient of the
 * logarithm of its moment generating function.  With mu = m / m_0 the
 * identity d_j M = M d_j log M gives, for n = n' + e_j,
 *   mu_n = sum_{k <= n'} B(n', k) mu_{n'-k} c_{k+e_j},
 *   B(n', k) = prod_d binomial(n'_d, k_d),
 * which is solved for c_n (the k = n' term is c_n itself) in increasing total
 * order, and read forwards for the inverse.  Every index it touches stays
 * inside the moment set, so the 27 (9) cumulants are exactly those of the
 * lattice's moments.
 * ------------------------------------------------------------------------- */

static int mom_order(const ora_lat *L, int k) { return L->mo[k][0] + L->mo[k][1] + L->mo[k][2]; }

/* first axis j with n_j > 0 */
static int first_axis(const int n[3]) { return n[0] ? 0 : (n[1] ? 1 : 2); }

/* sum_{k <= np, k != skip_top ? np : -} B(np, k) mu[np - k] c[k + e_j] */
static double recursion_sum(const ora_lat *L, const int np[3], int j, const double *mu, const double *c,
                            int include_top) {
  double acc = 0.0;
  for (int kx = 0; kx <= np[0]; kx++)
    for (int ky = 0; ky <= np[1]; ky++)
      for (int kz = 0; kz <= np[2]; kz++) {
        const int k[3] = {kx, ky, kz};
        if (!include_top && kx == np[0] && ky == np[1] && kz == np[2]) continue;
        const int rest[3] = {np[0] - kx, np[1] - ky, np[2] - kz};
        int kj[3] = {kx, ky, kz};
        kj[j] += 1;
        const double B = binom(np[0], kx) * binom(np[1], ky) * binom(np[2], kz);
        acc += B * mu[mom_slot(L, rest)] * c[mom_slot(L, kj)];
      }
  return acc;
}

/* raw moments of g -> cumulants c (c[0] = m_0) */
static void cumulants(const ora_lat *L, const double *g, double *c) {
  int Q = L->Q;
  double m[ORA_MAXQ], mu[ORA_MAXQ];
  for (int k = 0; k < Q; k++) {
    double v = 0.0;
    for (int a = 0; a < Q; a++)
      v += g[a] * ipow(L->e[a][0], L->mo[k][0]) * ipow(L->e[a][1], L->mo[k][1]) * ipow(L->e[a][2], L->mo[k][2]);
    m[k] = v;
  }
  for (int k = 0; k < Q; k++) mu[k] = m[k] / m[0];
  c[0] = m[0];
  for (int t = 1; t <= 6; t++)
    for (int k = 1; k < Q; k++) {
      if (mom_order(L, k) != t) continue;
      const int j = first_axis(L->mo[k]);
      int np[3] = {L->mo[k][0], L->mo[k][1], L->mo[k][2]};
      np[j] -= 1;
      c[k] = mu[k] - recursion_sum(L, np, j, mu, c, 0);
    }
}

/* cumulants c -> populations g (raw moments m = c_0 mu, then M^-1) */
static void from_cumulants(const ora_ctx *C, const double *c, double *g) {
  const ora_lat *L = &C->L;
  int Q = L->Q;
  double mu[ORA_MAXQ], m[ORA_MAXQ];
  mu[0] = 1.0;
  for (int t = 1; t <= 6; t++)
    for (int k = 1; k < Q; k++) {
      if (mom_order(L, k) != t) continue;
      const int j = first_axis(L->mo[k]);
      int np[3] = {L->mo[k][0], L->mo[k][1], L->mo[k][2]};
      np[j] -= 1;
      mu[k] = recursion_sum(L, np, j, mu, c, 1);
    }
  for (int k = 0; k < Q; k++) m[k] = c[0] * mu[k];
  for (int a = 0; a < Q; a++) {
    double v = 0.0;
    for (int k = 0; k < Q; k++) v += C->Minv[a * Q + k] * m[k];
    g[a] = v;
  }
}

/* Equilibrium cumulants (Sec. 2.1.1, the vector C^H,eq; the same shape with
 * psi = rho for f): psi at 000, u at the first order, cs^2 at 200/020/002,
 * zero elsewhere. */
static void cu_equilibrium(const ora_lat *L, double psi, const double u[3], double *eq) {
  for (int k = 0; k < L->Q; k++) {
    const int *n = L->mo[k];
    const int ord = n[0] + n[1] + n[2];
    const int pure = (n[0] == ord) || (n[1] == ord) || (n[2] == ord);
    if (ord == 0)
      eq[k] = psi;
    else if (ord == 1)
      eq[k] = n[0] ? u[0] : (n[1] ? u[1] : u[2]);
    else if (ord == 2 && pure)
      eq[k] = CS2;
    else
      eq[k] = 0.0;
  }
}

/* One cumulant collision with the source of App. D (Eq. H_cu_collision_with_Q):
 *   C   = cumulants(g),  psi = C_000 + src/2,
 *   C*  = C + S (C^eq(psi, u) - C) + (1 - s_000/2) src e_000,
 *   g*  = cumulants^-1(C*).                                                 */
static void collide_node_cu(const ora_ctx *C, const double *g, const double u[3], const double *s, double s_bulk,
                            double src, double *gs) {
  double c[ORA_MAXQ], eq[ORA_MAXQ];
  cumulants(&C->L, g, c);
  cu_equilibrium(&C->L, c[0] + 0.5 * src, u, eq);
  relax_moments(&C->L, c, eq, s, s_bulk);
  c[0] += (1.0 - 0.5 * s[0]) * src;
  from_cumulants(C, c, gs);
}

int ora_cumulants(int Q, const double *g, double *c) {
  ora_lat L;
  if (build_lattice(Q, &L)) return -1;
  cumulants(&L, g, c);
  return 0;
}

int ora_from_cumulants(int Q, const double *c, double *g) {
  ora_ctx C;
  if (ctx_init(Q, &C)) return -1;
  from_cumulants(&C, c, g);
  return 0;
}

int ora_collide_node_cu(int Q, const double *g, const double *u, const double *s, double src, double s_bulk,
                        double *gs) {
  ora_ctx C;
  if (ctx_init(Q, &C)) return -1;
  collide_node_cu(&C, g, u, s, s_bulk, src, gs);
  return 0;
}

/* ---------------------------------------------------------------------------
 * Whole-lattice configuration.
 * ------------------------------------------------------------------------- */
enum { ORA_FLUID = 0, ORA_SOLID = 1, ORA_EQ = 2, ORA_OUTLET = 3 };
enum { ORA_BB = 0, ORA_IBB = 1 };   /* f wall schemes */
enum { ORA_ABB = 0, ORA_IABB = 1 }; /* h wall schemes */

typedef struct {
  int32_t f_scheme;
  int32_t h_scheme;
  double rho_w;
  double u_w[3];
  double H_w;
} ora_group;

typedef struct {
  int32_t Q;
  int32_t nx, ny, nz;
  int32_t with_ns;
  int32_t u_field;      /* 0: uniform u0, 1: per-node field uvel[d*n + node] */
  double s_f[27];
  double s_h[27];
  double u0[3];
  const double *uvel;   /* [3][n] or NULL */
  const double *src;    /* [n] source Q or NULL */
  const uint16_t *flags;/* [n]: type in bits 0-3, group in bits 4-11; NULL = fluid */
  const double *qlink;  /* [Q][n] wall distances; NULL = 0.5 everywhere */
  int32_t n_groups;
  int32_t collide_off;  /* 1: collision is the identity (streaming checks) */
  const ora_group *groups;
  int32_t cu_f;         /* 1: f uses the cumulant collision, 0: central moments */
  int32_t cu_h;         /* the same for h */
  double s_bulk_f;      /* > 0: trace of the second-order block of f relaxed at
                         * this rate, its deviator at s_f of 200 (relax_moments);
                         * 0: the diagonal rates s_f alone */
} ora_cfg;

typedef struct {
  int32_t node;
  int32_t dir;   /* direction from the boundary node towards the wall */
  int32_t group;
  int32_t xf_solid; /* 1 when x_b - e_dir is solid: below q = 1/2 the rule is plain (A)BB */
  double q;
} ora_link;

static long nnodes(const ora_cfg *c) { return (long)c->nx * c->ny * c->nz; }

static int ntype(const ora_cfg *c, long n) { return c->flags ? (c->flags[n] & 15) : ORA_FLUID; }
static int ngroup(const ora_cfg *c, long n) { return c->flags ? ((c->flags[n] >> 4) & 255) : 0; }

static long wrapi(long v, long n) { return ((v % n) + n) % n; }

static long neighbour(const ora_cfg *c, long n, const int e[3], int sign) {
  long x = n % c->nx, y = (n / c->nx) % c->ny, z = n / ((long)c->nx * c->ny);
  x = wrapi(x + sign * e[0], c->nx);
  y = wrapi(y + sign * e[1], c->ny);
  z = wrapi(z + sign * e[2], c->nz);
  return x + c->nx * (y + (long)c->ny * z);
}

static void node_velocity_prescribed(const ora_cfg *c, long n, double u[3]) {
  long N = nnodes(c);
  for (int d = 0; d < 3; d++) u[d] = c->u_field ? c->uvel[d * N + n] : c->u0[d];
  if (c->Q == 9) u[2] = 0.0;
}

static void moments_f(const ora_lat *L, const double *f, long N, long n, double *rho, double u[3]) {
  double r = 0.0, j[3] = {0, 0, 0};
  for (int a = 0; a < L->Q; a++) {
    double v = f[a * N + n];
    r += v;
    for (int d = 0; d < 3; d++) j[d] += L->e[a][d] * v;
  }
  *rho = r;
  for (int d = 0; d < 3; d++) u[d] = j[d] / r;
}

static int check_cfg(const ora_cfg *c) {
  if (c->Q != 9 && c->Q != 27) return -1;
  if (c->nx < 1 || c->ny < 1 || c->nz < 1) return -1;
  if (c->Q == 9 && c->nz != 1) return -1;
  if (c->u_field && !c->uvel) return -1;
  return 0;
}

/* Velocity used by the equilibrium of an EQ node: the per-node field when
 * one is given, else the group's wall velocity. */
static void eq_node_velocity(const ora_cfg *c, long n, double u[3]) {
  if (!c->with_ns || c->u_field) {
    node_velocity_prescribed(c, n, u);
  } else {
    const ora_group *G = &c->groups[ngroup(c, n)];
    for (int d = 0; d < 3; d++) u[d] = G->u_w[d];
    if (c->Q == 9) u[2] = 0.0;
  }
}

/* Collision of every non-solid node: f (when with_ns) then h with the
 * velocity of f, or with the prescribed velocity. */
int ora_collide(const ora_cfg *c, const double *f, const double *h, double *fs, double *hs) {
  ora_ctx C;
  long N;
  if (check_cfg(c) || ctx_init(c->Q, &C)) return -1;
  N = nnodes(c);
#pragma omp parallel for schedule(static)
  for (long n = 0; n < N; n++) {
    int Q = c->Q;
    double g[ORA_MAXQ], gs[ORA_MAXQ], u[3], rho;
    if (ntype(c, n) == ORA_SOLID) {
      for (int a = 0; a < Q; a++) {
        if (c->with_ns) fs[a * N + n] = f[a * N + n];
        hs[a * N + n] = h[a * N + n];
      }
      continue;
    }
    if (c->with_ns) {
      moments_f(&C.L, f, N, n, &rho, u);
      for (int a = 0; a < Q; a++) g[a] = f[a * N + n];
      if (c->collide_off)
        memcpy(gs, g, sizeof(double) * Q);
      else if (c->cu_f)
        collide_node_cu(&C, g, u, c->s_f, c->s_bulk_f, 0.0, gs);
      else
        collide_node(&C, g, u, c->s_f, c->s_bulk_f, 0.0, gs);
      for (int a = 0; a < Q; a++) fs[a * N + n] = gs[a];
    } else {
      node_velocity_prescribed(c, n, u);
    }
    for (int a = 0; a < Q; a++) g[a] = h[a * N + n];
    if (c->collide_off)
      memcpy(gs, g, sizeof(double) * Q);
    else if (c->cu_h)
      collide_node_cu(&C, g, u, c->s_h, 0.0, c->src ? c->src[n] : 0.0, gs);
    else
      collide_node(&C, g, u, c->s_h, 0.0, c->src ? c->src[n] : 0.0, gs);
    for (int a = 0; a < Q; a++) hs[a * N + n] = gs[a];
  }
  return 0;
}

/* Cut links: every (non-solid x_b, direction i != 0) with x_b + e_i solid,
 * in increasing (node, direction) order.  q is the fraction of the link
 * vector between x_b and the wall (Sec. 3). */
/* Cut links of node n (writes at most Q entries to out when non-NULL). */
static int node_links(const ora_cfg *c, const ora_lat *L, long n, ora_link *out) {
  long N = nnodes(c);
  int cnt = 0;
  if (ntype(c, n) == ORA_SOLID) return 0;
  for (int a = 1; a < c->Q; a++) {
    long w = neighbour(c, n, L->e[a], +1);
    if (ntype(c, w) != ORA_SOLID) continue;
    if (out) {
      long xf = neighbour(c, n, L->e[a], -1);
      out[cnt].node = (int32_t)n;
      out[cnt].dir = a;
      out[cnt].group = ngroup(c, w);
      out[cnt].xf_solid = ntype(c, xf) == ORA_SOLID;
      out[cnt].q = c->qlink ? c->qlink[(long)a * N + n] : 0.5;
    }
    cnt++;
  }
  return cnt;
}

long ora_links(const ora_cfg *c, ora_link *out, long cap) {
  ora_lat L;
  long N, total = 0;
  long *first;
  if (check_cfg(c) || build_lattice(c->Q, &L)) return -1;
  if (!c->flags) return 0;
  N = nnodes(c);
  /* count per node, then fill each node's run at its offset (node-major
   * order, as a serial scan would produce it) */
  first = (long *)malloc(sizeof(long) * (N + 1));
  if (!first) return -1;
#pragma omp parallel for schedule(static)
  for (long n = 0; n < N; n++) first[n] = node_links(c, &L, n, NULL);
  for (long n = 0; n < N; n++) {
    long k = first[n];
    first[n] = total;
    total += k;
  }
  first[N] = total;
  if (out) {
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; n++) {
      ora_link tmp[ORA_MAXQ];
      int k = node_links(c, &L, n, tmp);
      for (int j = 0; j < k; j++)
        if (first[n] + j < cap) out[first[n] + j] = tmp[j];
    }
  }
  free(first);
  return total;
}

/* Interpolated bounce-back (Eq. IBB) for f; q = 1/2 without interpolation
 * (plain BB), or when the q <= 1/2 branch would need x_f and x_f is solid. */
static double ibb(double q, double gb_i, double gb_opp, double gf_i) {
  if (q <= 0.5) return 2.0 * q * gb_i + (1.0 - 2.0 * q) * gf_i;
  return (gb_i + (2.0 * q - 1.0) * gb_opp) / (2.0 * q);
}

/* Interpolated anti-bounce-back (Eq. IABB) for h; ABB is the q = 1/2 case. */
static double iabb(double q, double gb_i, double gb_opp, double gf_i, double geq_i) {
  if (q <= 0.5) return -(2.0 * q * gb_i + (1.0 - 2.0 * q) * gf_i) + 2.0 * geq_i;
  return (-gb_i + (2.0 * q - 1.0) * gb_opp + 2.0 * geq_i) / (2.0 * q);
}

/* Streaming and boundary handling: post-collision state (fs, hs) at t to
 * pre-collision state (f, h) at t+1.  Steps, in order of precedence from
 * lowest to highest:
 *   1. push streaming g_i(x + e_i) = g*_i(x) into non-solid nodes, periodic;
 *   2. wall links (BB/IBB on f, ABB/IABB on h);
 *   3. outlet: unknown populations (e_x < 0) copied from the upstream
 *      neighbour's values after steps 1-2;
 *   4. EQ nodes: whole population set replaced by the equilibrium.
 * link_flux (optional, one entry per cut link in ora_links order) receives
 * h_opp(x_b, t+1) - h*_i(x_b, t), the energy a wall link injects. */
int ora_stream(const ora_cfg *c, const double *fs, const double *hs, double *f, double *h,
               double *link_flux) {
  ora_ctx C;
  long N, nl, li;
  int Q = c->Q;
  ora_link *links = NULL;
  double *f3 = NULL, *h3 = NULL;
  if (check_cfg(c) || ctx_init(Q, &C)) return -1;
  N = nnodes(c);

  /* 1. push streaming (each target population has exactly one source) */
#pragma omp parallel for schedule(static)
  for (long n = 0; n < N; n++) {
    if (ntype(c, n) == ORA_SOLID) continue;
    for (int a = 0; a < Q; a++) {
      long m = neighbour(c, n, C.L.e[a], +1);
      if (ntype(c, m) == ORA_SOLID) continue;
      if (c->with_ns) f[a * N + m] = fs[a * N + n];
      h[a * N + m] = hs[a * N + n];
    }
  }
  /* solid nodes keep their (unused) values */
#pragma omp parallel for schedule(static)
  for (long n = 0; n < N; n++) {
    if (ntype(c, n) != ORA_SOLID) continue;
    for (int a = 0; a < Q; a++) {
      if (c->with_ns) f[a * N + n] = fs[a * N + n];
      h[a * N + n] = hs[a * N + n];
    }
  }

  /* 2. wall links */
  nl = ora_links(c, NULL, 0);
  if (nl < 0) return -1;
  if (nl > 0) {
    links = (ora_link *)malloc(sizeof(ora_link) * nl);
    if (!links) return -1;
    ora_links(c, links, nl);
  }
  /* each link writes its own (node, opposite direction) population */
#pragma omp parallel for schedule(static)
  for (li = 0; li < nl; li++) {
    const ora_link *k = &links[li];
    const ora_group *G = &c->groups[k->group];
    long b = k->node;
    int a = k->dir, o = C.L.opp[a];
    long xf = neighbour(c, b, C.L.e[a], -1);
    double q = k->q;
    if (c->with_ns) {
      /* the q > 1/2 branch reads only x_b, so a solid x_f (one-node gap)
       * forces plain bounce-back only below q = 1/2 */
      double qf = (G->f_scheme == ORA_BB || (k->xf_solid && q < 0.5)) ? 0.5 : q;
      f[o * N + b] = ibb(qf, fs[a * N + b], fs[o * N + b], fs[a * N + xf]);
    }
    {
      double u[3], rho, geq[ORA_MAXQ];
      double qh = (G->h_scheme == ORA_ABB || (k->xf_solid && q < 0.5)) ? 0.5 : q;
      if (c->with_ns)
        moments_f(&C.L, fs, N, b, &rho, u);
      else
        node_velocity_prescribed(c, b, u);
      equilibrium(&C, G->H_w, u, geq);
      h[o * N + b] = iabb(qh, hs[a * N + b], hs[o * N + b], hs[a * N + xf], geq[a]);
      if (link_flux) link_flux[li] = h[o * N + b] - hs[a * N + b];
    }
  }
  free(links);

  /* 3. outlet (zero-gradient copy from x - 1 using values after step 2: the
   * upstream values are read into a buffer before any outlet is written) */
  {
    long no = 0, j = 0;
    long *outl;
    for (long n = 0; n < N; n++) no += ntype(c, n) == ORA_OUTLET;
    if (no > 0) {
      int ex[3] = {1, 0, 0};
      outl = (long *)malloc(sizeof(long) * no);
      f3 = (double *)malloc(sizeof(double) * Q * no);
      h3 = (double *)malloc(sizeof(double) * Q * no);
      if (!outl || !f3 || !h3) {
        free(outl);
        free(f3);
        free(h3);
        return -1;
      }
      for (long n = 0; n < N; n++)
        if (ntype(c, n) == ORA_OUTLET) outl[j++] = n;
      for (j = 0; j < no; j++) {
        long up = neighbour(c, outl[j], ex, -1);
        for (int a = 0; a < Q; a++) {
          if (c->with_ns) f3[j * Q + a] = f[a * N + up];
          h3[j * Q + a] = h[a * N + up];
        }
      }
      for (j = 0; j < no; j++)
        for (int a = 0; a < Q; a++) {
          if (C.L.e[a][0] >= 0) continue;
          if (c->with_ns) f[a * N + outl[j]] = f3[j * Q + a];
          h[a * N + outl[j]] = h3[j * Q + a];
        }
      free(outl);
      free(f3);
      free(h3);
    }
  }

  /* 4. EQ nodes */
#pragma omp parallel for schedule(static)
  for (long n = 0; n < N; n++) {
    double u[3], geq[ORA_MAXQ];
    const ora_group *G;
    if (ntype(c, n) != ORA_EQ) continue;
    G = &c->groups[ngroup(c, n)];
    eq_node_velocity(c, n, u);
    if (c->with_ns) {
      equilibrium(&C, G->rho_w, u, geq);
      for (int a = 0; a < Q; a++) f[a * N + n] = geq[a];
    }
    equilibrium(&C, G->H_w, u, geq);
    for (int a = 0; a < Q; a++) h[a * N + n] = geq[a];
  }
  return 0;
}

/* Initial post-collision state: the equilibrium field pre-streamed backwards,
 * g*_i(x) = g^eq_i(x + e_i), so that streaming reproduces g^eq in the bulk.
 * rho (with_ns), u ([3][n]) and H ([n]) are the initial fields. */
int ora_init_post(const ora_cfg *c, const double *rho, const double *u, const double *H,
                  double *fs, double *hs) {
  ora_ctx C;
  long N;
  double *feq, *heq;
  if (check_cfg(c) || ctx_init(c->Q, &C)) return -1;
  N = nnodes(c);
  feq = (double *)malloc(sizeof(double) * c->Q * N);
  heq = (double *)malloc(sizeof(double) * c->Q * N);
  if (!feq || !heq) {
    free(feq);
    free(heq);
    return -1;
  }
  /* equilibrium of every node from its own fields */
#pragma omp parallel for schedule(static)
  for (long m = 0; m < N; m++) {
    double um[3], geq[ORA_MAXQ];
    for (int d = 0; d < 3; d++) um[d] = u[d * N + m];
    if (c->Q == 9) um[2] = 0.0;
    if (c->with_ns) {
      equilibrium(&C, rho[m], um, geq);
      for (int a = 0; a < c->Q; a++) feq[a * N + m] = geq[a];
    }
    equilibrium(&C, H[m], um, geq);
    for (int a = 0; a < c->Q; a++) heq[a * N + m] = geq[a];
  }
  /* g*_a(x) = g^eq_a(x + e_a) */
  for (long n = 0; n < N; n++)
    for (int a = 0; a < c->Q; a++) {
      long m = neighbour(c, n, C.L.e[a], +1);
      if (c->with_ns) fs[a * N + n] = feq[a * N + m];
      hs[a * N + n] = heq[a * N + m];
    }
  free(feq);
  free(heq);
  return 0;
}

/* Macroscopic fields of a pre-collision state (Eqs. f_0th_mom, f_1st_mom,
 * h_0th_mom): rho = sum f, rho u = sum e f, H = sum h (+ Q/2 with a source).
 * Solid nodes report zeros.  Any output pointer may be NULL. */
int ora_macroscopic(const ora_cfg *c, const double *f, const double *h, double *rho,
                    double *u, double *H) {
  ora_lat L;
  long N;
  if (check_cfg(c) || build_lattice(c->Q, &L)) return -1;
  N = nnodes(c);
  for (long n = 0; n < N; n++) {
    double r = 0.0, uu[3] = {0, 0, 0}, e = 0.0;
    if (ntype(c, n) != ORA_SOLID) {
      if (c->with_ns)
        moments_f(&L, f, N, n, &r, uu);
      else
        node_velocity_prescribed(c, n, uu);
      for (int a = 0; a < c->Q; a++) e += h[a * N + n];
      if (c->src) e += 0.5 * c->src[n];
    }
    if (rho) rho[n] = r;
    if (u)
      for (int d = 0; d < 3; d++) u[d * N + n] = uu[d];
    if (H) H[n] = e;
  }
  return 0;
}

/* Heat flux through the cross-section x = X of a pre-collision state
 * (Eq. heat_flux_section): sum over non-solid nodes of the column of
 * sum_a e_ax h_a. */
double ora_section_flux(const ora_cfg *c, const double *h, int X) {
  ora_lat L;
  long N;
  double s = 0.0;
  if (check_cfg(c) || build_lattice(c->Q, &L)) return NAN;
  N = nnodes(c);
  for (long z = 0; z < c->nz; z++)
    for (long y = 0; y < c->ny; y++) {
      long n = X + c->nx * (y + (long)c->ny * z);
      if (ntype(c, n) == ORA_SOLID) continue;
      for (int a = 0; a < c->Q; a++) s += L.e[a][0] * h[a * N + n];
    }
  return s;
}

/* Nusselt number of a heated body (Sec. 4.4, Eqs. heat_flux_thorough_heater,
 * heat_flux_section and the Nu definition that follows them) from the post-
 * collision state (fs, hs) of step t-1: the canonical state at t is streamed
 * from it, with the energy each wall link injects.
 *   q_s   = sum over the cut links into group `group` of h_opp(x_b, t) - h*_i(x_b, t-1)
 *   q_in  = section flux of column x_in, q_out = that of column x_out
 *   qdot  = (q_s + q_out - q_in) / 2  (heater and the flow's gain, averaged)
 *   Nu    = qdot / (pi k (T_w - T_in) nz)   (Nu = varsigma D / k with
 *           varsigma = qdot / (pi D (T_w - T_in)) per unit depth; nz layers)
 * out: Nu, Nu from q_s alone, q_s, q_in, q_out.  Returns 0, or -1 on bad input. */
int ora_nusselt(const ora_cfg *c, const double *fs, const double *hs, int group, int x_in, int x_out,
                double k, double T_w, double T_in, double *out) {
  long N, nl;
  int Q = c->Q;
  double *f = NULL, *h = NULL, *flux = NULL;
  ora_link *links = NULL;
  double qs = 0.0, qin, qout, depth;
  if (check_cfg(c) || x_in < 0 || x_in >= c->nx || x_out < 0 || x_out >= c->nx) return -1;
  if (!(k > 0.0) || T_w == T_in) return -1;
  N = nnodes(c);
  nl = ora_links(c, NULL, 0);
  if (nl < 0) return -1;
  f = (double *)malloc(sizeof(double) * Q * N);
  h = (double *)malloc(sizeof(double) * Q * N);
  flux = (double *)malloc(sizeof(double) * (nl > 0 ? nl : 1));
  links = (ora_link *)malloc(sizeof(ora_link) * (nl > 0 ? nl : 1));
  if (!f || !h || !flux || !links) {
    free(f);
    free(h);
    free(flux);
    free(links);
    return -1;
  }
  memcpy(h, hs, sizeof(double) * Q * N);
  if (c->with_ns) memcpy(f, fs, sizeof(double) * Q * N);
  if (ora_stream(c, fs, hs, f, h, flux) != 0) {
    free(f);
    free(h);
    free(flux);
    free(links);
    return -1;
  }
  ora_links(c, links, nl);
  for (long l = 0; l < nl; l++)
    if (links[l].group == group) qs += flux[l];
  qin = ora_section_flux(c, h, x_in);
  qout = ora_section_flux(c, h, x_out);
  depth = (double)c->nz;
  out[0] = 0.5 * (qs + qout - qin) / (M_PI * k * (T_w - T_in) * depth);
  out[1] = qs / (M_PI * k * (T_w - T_in) * depth);
  out[2] = qs;
  out[3] = qin;
  out[4] = qout;
  free(f);
  free(h);
  free(flux);
  free(links);
  return 0;
}

/* ---------------------------------------------------------------------------
 * Discrete adjoint of the advection-diffusion step (prescribed velocity,
 * fully periodic lattice, optional source Q).  Not in the paper: defined as
 * the exact transpose of the forward step above.
 *
 * Per node the collision is affine: g* = A g + b Q with
 *   A = T^-1 [(1 - S) T + S ceq 1^T],   b = T^-1 [S ceq / 2 + (1 - s_000/2) e_000],
 * where ceq is the central-moment equilibrium per unit psi and 1^T g = Y~_000.
 * Streaming is the permutation pre_a(x) = post_a(x - e_a).
 * With lam_pre(t+1) = dJ/dpre(t+1):
 *   lam_post(t)_a(x) = lam_pre(t+1)_a(x + e_a)          (transpose of streaming)
 *   lam_pre(t)       = A^T lam_post(t)                  (per node)
 *   dJdQ(x)         += b^T lam_post(t)(x)
 * A and b are assembled here as explicit matrices from T(u), M^-1, N(-u).
 * ------------------------------------------------------------------------- */
static void collision_matrix(const ora_ctx *C, const double u[3], const double *s, double *A,
                             double *b) {
  int Q = C->L.Q;
  double T[ORA_MAXQ * ORA_MAXQ], Tinv[ORA_MAXQ * ORA_MAXQ], ceq[ORA_MAXQ];
  double Nm[ORA_MAXQ * ORA_MAXQ], mu[3] = {-u[0], -u[1], -u[2]};
  double K[ORA_MAXQ * ORA_MAXQ], v[ORA_MAXQ];
  matrix_T(&C->L, u, T);
  matrix_N(&C->L, mu, Nm);
  /* T^-1 = M^-1 N(-u) */
  for (int a = 0; a < Q; a++)
    for (int k = 0; k < Q; k++) {
      double acc = 0.0;
      for (int j = 0; j < Q; j++) acc += C->Minv[a * Q + j] * Nm[j * Q + k];
      Tinv[a * Q + k] = acc;
    }
  cm_equilibrium(&C->L, 1.0, ceq);
  /* K = (1 - S) T + S ceq 1^T   (row k) */
  for (int k = 0; k < Q; k++)
    for (int a = 0; a < Q; a++) K[k * Q + a] = (1.0 - s[k]) * T[k * Q + a] + s[k] * ceq[k];
  for (int a = 0; a < Q; a++)
    for (int c = 0; c < Q; c++) {
      double acc = 0.0;
      for (int k = 0; k < Q; k++) acc += Tinv[a * Q + k] * K[k * Q + c];
      A[a * Q + c] = acc;
    }
  for (int k = 0; k < Q; k++) v[k] = 0.5 * s[k] * ceq[k] + (k == 0 ? 1.0 - 0.5 * s[0] : 0.0);
  for (int a = 0; a < Q; a++) {
    double acc = 0.0;
    for (int k = 0; k < Q; k++) acc += Tinv[a * Q + k] * v[k];
    b[a] = acc;
  }
}

int ora_collision_matrix(int Q, const double *u, const double *s, double *A, double *b) {
  ora_ctx C;
  if (ctx_init(Q, &C)) return -1;
  collision_matrix(&C, u, s, A, b);
  return 0;
}

/* One reverse step: lam_next = dJ/dpre(t+1) -> lam_prev = dJ/dpre(t), and
 * dJdQ += dJ/dQ through the collision of step t.  Advection-only, no
 * geometry. */
int ora_adjoint_step(const ora_cfg *c, const double *lam_next, double *lam_prev, double *dJdQ) {
  ora_ctx C;
  long N;
  if (check_cfg(c) || ctx_init(c->Q, &C) || c->with_ns || c->flags) return -1;
  N = nnodes(c);
#pragma omp parallel for schedule(static)
  for (long n = 0; n < N; n++) {
    int Q = c->Q;
    double u[3], A[ORA_MAXQ * ORA_MAXQ], b[ORA_MAXQ], lp[ORA_MAXQ];
    node_velocity_prescribed(c, n, u);
    collision_matrix(&C, u, c->s_h, A, b);
    for (int a = 0; a < Q; a++) lp[a] = lam_next[a * N + neighbour(c, n, C.L.e[a], +1)];
    for (int a = 0; a < Q; a++) {
      double acc = 0.0;
      for (int k = 0; k < Q; k++) acc += A[k * Q + a] * lp[k];
      lam_prev[a * N + n] = acc;
    }
    if (dJdQ) {
      double acc = 0.0;
      for (int a = 0; a < Q; a++) acc += b[a] * lp[a];
      dJdQ[n] += acc;
    }
  }
  return 0;
}
