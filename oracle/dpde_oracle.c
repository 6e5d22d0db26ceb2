/*
 * dpde_oracle.c -- plain CPU FP64 reference for one DPDE timestep:
 * velocity-Verlet on the conservative part, then the fluctuation/dissipation
 * part by SER (Splitting with Energy Reinjection) or, for comparison, SEM.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  The HIP product
 * library never links, loads or calls it, and the two share no source,
 * header, table or constant generator.  Inputs (positions, momenta, internal
 * energies, seeds) come from the seeded generators in workloads/, which hold
 * none of the method's arithmetic.
 *
 * Paper: Homman, Maillet, Roussel, Stoltz, "New parallelizable schemes for
 * integrating the Dissipative Particle Dynamics with Energy Conservation",
 * arXiv:1507.06643.  Every routine cites the section/equation it follows.
 *
 * Readings where the paper is silent or inconsistent (all listed in the
 * design notes of the repository):
 *  - total energy uses sum p^2/(2m) (Sec. 2.1 prints p^2/m; only 1/(2m)
 *    balances the internal-energy equation of eq. (DPDE));
 *  - the SER internal-energy update carries the factor -1/2 of
 *    eq. (SER_eint_discretization); the summary eq. (SER_fd) drops it;
 *  - the conservative force is by default the soft DPD force a(1-r/rc) r_hat
 *    with potential (a rc/2)(1-r/rc)^2; the paper's splined LJ (eq. Ep) is the
 *    other choice, with its cut-off rc supplied by the caller (the paper
 *    does not state it);
 *  - the Gaussian increments G_ij^n come from Philox-4x32-10 (Salmon et al.,
 *    SC'11) keyed by (seed, replica) with counter (lo id, hi id, n), followed
 *    by Box-Muller; the paper only requires that G_ij^n be a function of
 *    (i, j, n) (Sec. 3.2.1) with G_ji = -G_ij (Sec. 3.1.1);
 *  - the pair set is {r_ij^2 < rc^2}; chi(rc) = 0 so the dynamics is the same
 *    as with r <= rc (eq. pot_mou).
 *
 * Compiled with -O2 -ffp-contract=off: no fused multiply-adds, so every
 * expression is evaluated exactly as written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_EBOX (-2)
#define OR_ENOMEM (-3)
#define OR_ENEG_EINT (-5)
#define OR_EEOS (-6)

typedef struct {
  double box[3];
  double mass, rc, a, gamma, kT_ref, dt;
  double cv, eos_n, eos_omega, eos_c0;
  int64_t n;
  int64_t step;      /* n of G_ij^n for the next step */
  uint64_t seed;
  int32_t periodic[3];
  int32_t eos;       /* 0: eps = cv*theta ; 1: eps = n w/(exp(w/theta)-1) + c0 theta */
  int32_t replica;
  int32_t scheme;    /* 0: SER (Sec. 3.2.1) ; 1: SEM (Sec. 3.1.1) ;
                        2: Hybrid (Sec. 3.2.2): SSA inside domains, SER across */
  int32_t project;   /* 1: eps_i -= (E - E0)/N after every step (Sec. 4.2) */
  int32_t model;     /* 0: friction/noise along v_ij (eq. DPDE, the paper's variant);
                        1: projected on e_ij (the original DPDE model, Sec. 2.1) */
  int32_t potential; /* 0: soft v = (a rc/2)(1-r/rc)^2 ; 1: splined LJ (eq. Ep) */
  int32_t pad_;
  double E0;         /* target energy of the projection */
  double eps_lj, r_lj;
  int32_t ndom[3];   /* Hybrid (scheme 2): domains per dimension (Sec. 3.2.2) */
  int32_t pad2_;
} or_params;

/* ------------------------------------------------------------------------
 * Counter-based generator.  Philox-4x32-10 as defined by Salmon, Moraes,
 * Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11):
 * ten rounds of two 32x32->64 multiplications, the key bumped by the two
 * Weyl increments between rounds.
 * ---------------------------------------------------------------------- */
static const uint32_t PH_M0 = 0xD2511F53u, PH_M1 = 0xCD9E8D57u;
static const uint32_t PH_W0 = 0x9E3779B9u, PH_W1 = 0xBB67AE85u;

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += PH_W0; k1 += PH_W1; }
    uint64_t prod0 = (uint64_t)PH_M0 * (uint64_t)x0;
    uint64_t prod1 = (uint64_t)PH_M1 * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
    uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* The four 32-bit words of G_ij^n: key (seed low word, seed high word xor
 * replica), counter (lo id, hi id, n low word, n high word). */
void or_pair_words(uint64_t seed, uint32_t replica, int64_t step, uint32_t lo, uint32_t hi,
                   uint32_t out[4]) {
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32) ^ replica};
  uint64_t n = (uint64_t)step;
  uint32_t ctr[4] = {lo, hi, (uint32_t)n, (uint32_t)(n >> 32)};
  or_philox4x32_10(ctr, key, out);
}

/* G_ij^n for the ordered pair lo < hi (the increment seen by particle lo):
 * uniforms u_k = (x_k + 1/2) 2^-32 in (0,1), then Box-Muller on (u0,u1) and
 * (u2,u3), keeping three of the four normals. */
void or_gauss3(uint64_t seed, uint32_t replica, int64_t step, uint32_t lo, uint32_t hi,
               double g[3]) {
  uint32_t w[4];
  or_pair_words(seed, replica, step, lo, hi, w);
  const double two_m32 = 2.3283064365386963e-10; /* 2^-32 */
  double u0 = ((double)w[0] + 0.5) * two_m32;
  double u1 = ((double)w[1] + 0.5) * two_m32;
  double u2 = ((double)w[2] + 0.5) * two_m32;
  double u3 = ((double)w[3] + 0.5) * two_m32;
  const double twopi = 6.283185307179586;
  double rho1 = sqrt(-2.0 * log(u0));
  double rho2 = sqrt(-2.0 * log(u2));
  g[0] = rho1 * cos(twopi * u1);
  g[1] = rho1 * sin(twopi * u1);
  g[2] = rho2 * cos(twopi * u3);
}

/* ------------------------------------------------------------------------
 * Geometry: periodic wrap, minimum image, cells of side >= r_cut
 * (Sec. 3.1.2 mentions cells of size r_cut as the linear-scaling device).
 * ---------------------------------------------------------------------- */
static int n_cells_dim(const or_params* P, int d) { return (int)floor(P->box[d] / P->rc); }

double or_wrap(double x, double L) {
  if (x < 0.0 || x >= L) {
    x = x - L * floor(x / L);
    if (x >= L) x = 0.0; /* -tiny + L rounds to L */
  }
  return x;
}

static double min_image(double d, double L) { return d - L * rint(d / L); }

/* cell coordinate along dimension d: floor(x * nc/L), clamped to [0, nc-1] */
static int cell_coord(const or_params* P, int d, double x) {
  int nc = n_cells_dim(P, d);
  double s = (double)nc / P->box[d];
  double c = floor(x * s);
  if (c < 0.0) c = 0.0;
  if (c > (double)(nc - 1)) c = (double)(nc - 1);
  return (int)c;
}

int64_t or_cell_index(const or_params* P, const double q[3]) {
  int nx = n_cells_dim(P, 0), ny = n_cells_dim(P, 1);
  int cx = cell_coord(P, 0, q[0]), cy = cell_coord(P, 1, q[1]), cz = cell_coord(P, 2, q[2]);
  return (int64_t)cx + (int64_t)nx * ((int64_t)cy + (int64_t)ny * (int64_t)cz);
}

/* Separation d = q_i - q_j (minimum image along periodic dimensions) and
 * r^2 = (dx*dx + dy*dy) + dz*dz, evaluated exactly in that order. */
static double separation(const or_params* P, const double* qi, const double* qj, double d[3]) {
  for (int k = 0; k < 3; ++k) {
    d[k] = qi[k] - qj[k];
    if (P->periodic[k]) d[k] = min_image(d[k], P->box[k]);
  }
  return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
}

int or_check_box(const or_params* P) {
  if (P->n < 2 || !(P->rc > 0.0) || !(P->dt > 0.0) || !(P->mass > 0.0)) return OR_EINVAL;
  for (int d = 0; d < 3; ++d) {
    if (!(P->box[d] > 0.0)) return OR_EINVAL;
    if (n_cells_dim(P, d) < 3) return OR_EBOX;
  }
  return OR_OK;
}

static int cmp_pair(const void* a, const void* b) {
  const int32_t* x = (const int32_t*)a;
  const int32_t* y = (const int32_t*)b;
  if (x[0] != y[0]) return x[0] < y[0] ? -1 : 1;
  if (x[1] != y[1]) return x[1] < y[1] ? -1 : 1;
  return 0;
}

/* All pairs lo < hi with r^2 < rc^2 by checking every couple: O(N^2). */
int or_pairs_brute(const or_params* P, const double* q, int64_t* npairs, int32_t* lohi,
                   int64_t cap) {
  const double rc2 = P->rc * P->rc;
  int64_t m = 0;
  for (int64_t i = 0; i < P->n; ++i)
    for (int64_t j = i + 1; j < P->n; ++j) {
      double d[3];
      if (separation(P, &q[3 * i], &q[3 * j], d) < rc2) {
        if (m < cap) { lohi[2 * m] = (int32_t)i; lohi[2 * m + 1] = (int32_t)j; }
        ++m;
      }
    }
  *npairs = m;
  return m <= cap ? OR_OK : OR_ENOMEM;
}

/* The same set through a linked cell list: each particle meets the 27 cells
 * around its own (3 per dimension; periodic dimensions wrap, the others are
 * clipped).  Output sorted lexicographically by (lo, hi). */
int or_pairs_cells(const or_params* P, const double* q, int64_t* npairs, int32_t* lohi,
                   int64_t cap) {
  int rc_ = or_check_box(P);
  if (rc_ != OR_OK) return rc_;
  int nc[3] = {n_cells_dim(P, 0), n_cells_dim(P, 1), n_cells_dim(P, 2)};
  int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
  int64_t* head = (int64_t*)malloc(sizeof(int64_t) * ncell);
  int64_t* next = (int64_t*)malloc(sizeof(int64_t) * P->n);
  int* cc = (int*)malloc(sizeof(int) * 3 * P->n);
  if (!head || !next || !cc) { free(head); free(next); free(cc); return OR_ENOMEM; }
  for (int64_t c = 0; c < ncell; ++c) head[c] = -1;
  /* insert in decreasing index order so each cell lists increasing indices */
  for (int64_t i = P->n - 1; i >= 0; --i) {
    for (int d = 0; d < 3; ++d) cc[3 * i + d] = cell_coord(P, d, q[3 * i + d]);
    int64_t c = cc[3 * i] + (int64_t)nc[0] * (cc[3 * i + 1] + (int64_t)nc[1] * cc[3 * i + 2]);
    next[i] = head[c];
    head[c] = i;
  }
  const double rc2 = P->rc * P->rc;
  int64_t m = 0;
  for (int64_t i = 0; i < P->n; ++i) {
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          int c3[3] = {cc[3 * i] + dx, cc[3 * i + 1] + dy, cc[3 * i + 2] + dz};
          int skip = 0;
          for (int d = 0; d < 3; ++d) {
            if (c3[d] < 0 || c3[d] >= nc[d]) {
              if (P->periodic[d]) c3[d] = (c3[d] + nc[d]) % nc[d];
              else skip = 1;
            }
          }
          if (skip) continue;
          int64_t c = c3[0] + (int64_t)nc[0] * (c3[1] + (int64_t)nc[1] * c3[2]);
          for (int64_t j = head[c]; j >= 0; j = next[j]) {
            if (j <= i) continue;
            double d[3];
            if (separation(P, &q[3 * i], &q[3 * j], d) < rc2) {
              if (m < cap) { lohi[2 * m] = (int32_t)i; lohi[2 * m + 1] = (int32_t)j; }
              ++m;
            }
          }
        }
  }
  free(head); free(next); free(cc);
  *npairs = m;
  if (m > cap) return OR_ENOMEM;
  qsort(lohi, (size_t)m, 2 * sizeof(int32_t), cmp_pair);
  return OR_OK;
}

/* Builds the pair list into freshly allocated memory (cell list). */
static int build_pairs(const or_params* P, const double* q, int32_t** out, int64_t* npairs) {
  int64_t cap = 16 * P->n + 64;
  for (;;) {
    int32_t* buf = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)cap);
    if (!buf) return OR_ENOMEM;
    int64_t m = 0;
    int rc_ = or_pairs_cells(P, q, &m, buf, cap);
    if (rc_ == OR_OK) { *out = buf; *npairs = m; return OR_OK; }
    free(buf);
    if (rc_ != OR_ENOMEM || m <= cap) return rc_;
    cap = m + 64;
  }
}

/* ------------------------------------------------------------------------
 * Conservative part.  Soft pair potential v(r) = (a rc/2)(1 - r/rc)^2 for
 * r < rc, force on i from j: a (1 - r/rc) (q_i - q_j)/r; U = sum_{i<j} v(r_ij)
 * (eq. def_potential_energy with this v).  A coincident pair (r = 0) has no
 * direction and contributes v(0) to U and nothing to the forces.
 * ---------------------------------------------------------------------- */
/* Pair potential v(r) and its first two derivatives, r < rc.
 *   potential 0: v = (a rc/2)(1 - r/rc)^2, v' = -a (1 - r/rc), v'' = a/rc;
 *   potential 1 (eq. Ep): v = v_LJ(r) - v_LJ(rc) - v_LJ'(rc)(r - rc) with
 *     v_LJ = 4 eps_lj ((r_lj/r)^12 - (r_lj/r)^6), so that v(rc) = v'(rc) = 0.
 */
static void lj_terms(const or_params* P, double r, double* v, double* dv, double* d2v) {
  double s6 = pow(P->r_lj / r, 6.0);
  double s12 = s6 * s6;
  *v = 4.0 * P->eps_lj * (s12 - s6);
  *dv = -24.0 * P->eps_lj * (2.0 * s12 - s6) / r;
  *d2v = 4.0 * P->eps_lj * (156.0 * s12 - 42.0 * s6) / (r * r);
}

void or_pair_potential(const or_params* P, double r, double* v, double* dv, double* d2v) {
  if (P->potential == 1) {
    double vc, dvc, d2vc;
    lj_terms(P, P->rc, &vc, &dvc, &d2vc);
    lj_terms(P, r, v, dv, d2v);
    *v = *v - vc - dvc * (r - P->rc);
    *dv = *dv - dvc;
  } else {
    double w = 1.0 - r / P->rc;
    *v = 0.5 * P->a * P->rc * w * w;
    *dv = -P->a * w;
    *d2v = P->a / P->rc;
  }
}

/* Conservative forces F_i = -grad_i U with U = sum_{i<j} v(r_ij)
 * (eq. def_potential_energy).  A coincident pair (r = 0) contributes its
 * energy but no force. */
void or_forces_pairs(const or_params* P, const double* q, const int32_t* lohi, int64_t npairs,
                     double* F, double* U) {
  memset(F, 0, sizeof(double) * 3 * (size_t)P->n);
  double u = 0.0;
  for (int64_t k = 0; k < npairs; ++k) {
    int64_t i = lohi[2 * k], j = lohi[2 * k + 1];
    double d[3];
    double r2 = separation(P, &q[3 * i], &q[3 * j], d);
    double r = sqrt(r2);
    if (P->potential == 0) {
      double w = 1.0 - r / P->rc;
      u += 0.5 * P->a * P->rc * w * w;
      if (r > 0.0) {
        for (int c = 0; c < 3; ++c) {
          double f = P->a * w * d[c] / r;
          F[3 * i + c] += f;
          F[3 * j + c] -= f;
        }
      }
    } else {
      double v, dv, d2v;
      or_pair_potential(P, r, &v, &dv, &d2v);
      u += v;
      if (r > 0.0) {
        for (int c = 0; c < 3; ++c) {
          double f = -dv * d[c] / r;
          F[3 * i + c] += f;
          F[3 * j + c] -= f;
        }
      }
    }
  }
  *U = u;
}

/* Ingredients of the configurational temperature (eq. Tcon):
 * |grad U|^2 = sum_i |F_i|^2 and Delta U = sum_i Laplacian_{q_i} U
 *            = 2 sum_{i<j} (v''(r) + (d-1) v'(r)/r), d = 3. */
int or_config_temperature(const or_params* P, const double* q, double* grad2, double* lap);

int or_forces(const or_params* P, const double* q, double* F, double* U) {
  int32_t* pairs = NULL;
  int64_t np = 0;
  int rc_ = build_pairs(P, q, &pairs, &np);
  if (rc_ != OR_OK) return rc_;
  or_forces_pairs(P, q, pairs, np, F, U);
  free(pairs);
  return OR_OK;
}

/* ------------------------------------------------------------------------
 * Internal equation of state (eq. DPDE_internalEOS).
 *   eos 0: constant heat capacity, eps = cv * theta (Sec. 4.1);
 *   eos 1: eps(theta) = n w / (exp(w/theta) - 1) + c0 theta, an Einstein
 *          solid of n oscillators of energy w plus a constant-c0 part;
 *          C_v(theta) = n (w/theta)^2 e^{w/theta}/(e^{w/theta}-1)^2 + c0.
 * The Einstein part is evaluated through t = exp(-w/theta):
 *   n w t/(1-t) and n x^2 t/(1-t)^2, with 1-t = -expm1(-x).
 * ---------------------------------------------------------------------- */
double or_eos_energy(const or_params* P, double theta) {
  if (P->eos == 0) return P->cv * theta;
  double x = P->eos_omega / theta;
  double t = exp(-x);
  double one_m_t = -expm1(-x);
  return P->eos_n * P->eos_omega * t / one_m_t + P->eos_c0 * theta;
}

double or_eos_cv(const or_params* P, double theta) {
  if (P->eos == 0) return P->cv;
  double x = P->eos_omega / theta;
  double t = exp(-x);
  double one_m_t = -expm1(-x);
  return P->eos_n * x * x * t / (one_m_t * one_m_t) + P->eos_c0;
}

/* theta(eps) by Newton's method from the high-temperature asymptote
 * theta0 = (eps + n w/2)/(n + c0), which lies to the right of the root of the
 * increasing convex map theta -> eps(theta); stop when the Newton correction
 * is at most 4 ulp of theta, or after 60 iterations. */
double or_theta_newton(const or_params* P, double eps, int* iters) {
  if (P->eos == 0) { if (iters) *iters = 0; return eps / P->cv; }
  double theta = (eps + 0.5 * P->eos_n * P->eos_omega) / (P->eos_n + P->eos_c0);
  int it = 0;
  for (; it < 60; ++it) {
    double f = or_eos_energy(P, theta) - eps;
    double dth = f / or_eos_cv(P, theta);
    double next = theta - dth;
    if (!(next > 0.0)) next = 0.5 * theta;
    theta = next;
    if (fabs(dth) <= 4.0 * DBL_EPSILON * theta) { ++it; break; }
  }
  if (iters) *iters = it;
  return theta;
}

/* 1/T_i for every particle; fails on eps_i <= 0 or T_i <= 0. */
int or_inv_temperature(const or_params* P, const double* eps, double* invT) {
  for (int64_t i = 0; i < P->n; ++i) {
    if (!(eps[i] > 0.0)) return OR_ENEG_EINT;
    double th = or_theta_newton(P, eps[i], NULL);
    if (!(th > 0.0) || !isfinite(th)) return OR_EEOS;
    invT[i] = 1.0 / th;
  }
  return OR_OK;
}

/* ------------------------------------------------------------------------
 * Fluctuation/dissipation by SER (Sec. 3.2.1), at fixed positions.
 * For each pair (i,j), i<j, with w = 1 - r/rc, chi = w^2 (eq. pot_mou) and
 * gamma_ij = (gamma kT_ref/2)(1/T_i + 1/T_j) (eqs. DPDE_fd, alternative_FDR
 * with k_B = 1, sigma^2 = 2 gamma kT_ref):
 *   dp_ij = -gamma_ij chi v_ij dt + sigma w G_ij sqrt(dt)          (eq. SER_p)
 *   dp_i  = sum_j dp_ij ,   dp_ji = -dp_ij
 * then (eq. SER_eint_discretization)
 *   d eps_i = -1/2 sum_j dp_ij . (v_ij + (dp_i - dp_j)/(2m)),  p_i += dp_i.
 * The increments dp_ij of the first sweep are kept, so this reference does
 * not need to regenerate the noise in the second sweep.
 * SEM (Sec. 3.1.1, eq. SEM_fd) uses the same momenta and the Euler-Maruyama
 * internal-energy update
 *   d eps_i = 1/2 sum_j (gamma_ij v_ij^2 - d sigma^2/m) chi dt
 *           - 1/2 sum_j sigma w v_ij . G_ij sqrt(dt).
 * Model 1 (the original DPDE model with friction and noise along
 * e_ij = (q_i - q_j)/r_ij, Sec. 2.1) replaces v_ij by (e_ij . v_ij) e_ij and
 * G_ij by xi_ij e_ij with one scalar normal xi_ij (the first of the three):
 *   dp_ij = (-gamma_ij chi (e_ij . v_ij) dt + sigma w xi_ij sqrt(dt)) e_ij,
 * the same reinjection for SER, and for SEM
 *   d eps_i = 1/2 sum_j (gamma_ij (e_ij . v_ij)^2 - sigma^2/m) chi dt
 *           - 1/2 sum_j sigma w (e_ij . v_ij) xi_ij sqrt(dt).
 * A coincident pair (r = 0) has no direction and no interaction in model 1.
 * ---------------------------------------------------------------------- */
int or_fd_pairs(const or_params* P, const double* q, double* p, double* eps,
                const int32_t* lohi, int64_t npairs, double* dp_out) {
  const int64_t n = P->n;
  double* invT = (double*)malloc(sizeof(double) * n);
  double* dpij = (double*)malloc(sizeof(double) * 3 * (size_t)(npairs > 0 ? npairs : 1));
  double* dp = (double*)calloc(3 * (size_t)n, sizeof(double));
  double* deps = (double*)calloc((size_t)n, sizeof(double));
  if (!invT || !dpij || !dp || !deps) { free(invT); free(dpij); free(dp); free(deps); return OR_ENOMEM; }
  int rc_ = or_inv_temperature(P, eps, invT);
  if (rc_ != OR_OK) { free(invT); free(dpij); free(dp); free(deps); return rc_; }

  const double sigma = sqrt(2.0 * P->gamma * P->kT_ref);
  const double sqdt = sqrt(P->dt);
  /* first sweep: dp_ij and dp_i */
  for (int64_t k = 0; k < npairs; ++k) {
    int64_t i = lohi[2 * k], j = lohi[2 * k + 1];
    double d[3];
    double r = sqrt(separation(P, &q[3 * i], &q[3 * j], d));
    double w = 1.0 - r / P->rc;
    double chi = w * w;
    double gij = 0.5 * P->gamma * P->kT_ref * (invT[i] + invT[j]);
    double G[3];
    or_gauss3(P->seed, (uint32_t)P->replica, P->step, (uint32_t)i, (uint32_t)j, G);
    double vij[3];
    for (int c = 0; c < 3; ++c) vij[c] = p[3 * i + c] / P->mass - p[3 * j + c] / P->mass;
    if (P->model == 1) {
      double e[3] = {0.0, 0.0, 0.0};
      if (r > 0.0)
        for (int c = 0; c < 3; ++c) e[c] = d[c] / r;
      double ev = e[0] * vij[0] + e[1] * vij[1] + e[2] * vij[2];
      double xi = G[0];
      double mag = -gij * chi * ev * P->dt + sigma * w * xi * sqdt;
      for (int c = 0; c < 3; ++c) {
        double v = mag * e[c];
        dpij[3 * k + c] = v;
        dp[3 * i + c] += v;
        dp[3 * j + c] -= v;
      }
      if (P->scheme == 1 && r > 0.0) {
        double de = 0.5 * (gij * ev * ev - sigma * sigma / P->mass) * chi * P->dt
                  - 0.5 * sigma * w * ev * xi * sqdt;
        deps[i] += de;
        deps[j] += de;
      }
      continue;
    }
    for (int c = 0; c < 3; ++c) {
      double v = -gij * chi * vij[c] * P->dt + sigma * w * G[c] * sqdt;
      dpij[3 * k + c] = v;
      dp[3 * i + c] += v;
      dp[3 * j + c] -= v;
    }
    if (P->scheme == 1) {
      double vsq = 0.0, vG = 0.0;
      for (int c = 0; c < 3; ++c) {
        vsq += vij[c] * vij[c];
        vG += vij[c] * G[c];
      }
      double e = 0.5 * (gij * vsq - 3.0 * sigma * sigma / P->mass) * chi * P->dt
               - 0.5 * sigma * w * vG * sqdt;
      deps[i] += e;
      deps[j] += e;
    }
  }
  /* second sweep (SER): symmetric reinjection of the kinetic-energy change */
  if (P->scheme == 0) {
    for (int64_t k = 0; k < npairs; ++k) {
      int64_t i = lohi[2 * k], j = lohi[2 * k + 1];
      double s = 0.0;
      for (int c = 0; c < 3; ++c) {
        double vij = p[3 * i + c] / P->mass - p[3 * j + c] / P->mass;
        s += dpij[3 * k + c] * (vij + (dp[3 * i + c] - dp[3 * j + c]) / (2.0 * P->mass));
      }
      double e = -0.5 * s;
      deps[i] += e;
      deps[j] += e;
    }
  }
  for (int64_t i = 0; i < n; ++i) {
    for (int c = 0; c < 3; ++c) p[3 * i + c] += dp[3 * i + c];
    eps[i] += deps[i];
  }
  if (dp_out) memcpy(dp_out, dp, sizeof(double) * 3 * (size_t)n);
  free(invT); free(dpij); free(dp); free(deps);
  for (int64_t i = 0; i < n; ++i)
    if (!(eps[i] > 0.0)) return OR_ENEG_EINT;
  return OR_OK;
}

/* ------------------------------------------------------------------------
 * Hybrid (Sec. 3.2.2).  The box is split into ndom[0] x ndom[1] x ndom[2]
 * equal domains (the paper's processors); a particle belongs to the domain
 * of its position at the start of the fluctuation/dissipation step.  The
 * pairs A with both particles in one domain are integrated one after the
 * other by SSA (Sec. 3.1.2, eq. SSA_ij), in increasing (lo id, hi id) order;
 * then the remaining pairs A^c by SER on the updated state:
 * Phi^Hybrid = Phi^{SER,A^c} o Phi^{SSA,A}.
 * SSA pair update at fixed gamma_ij (exact Ornstein-Uhlenbeck step of
 * p_ij = p_i - p_j), with a = +(2 gamma_ij/m) chi dt (eq. SSA_ij prints a
 * minus sign; only the positive sign gives the decaying solution):
 *   D = (e^{-a} - 1) p_ij + sigma sqrt(m (1 - e^{-2a}) / gamma_ij) G_ij,
 *   p_i += D/2, p_j -= D/2, eps_i and eps_j -= dK_ij/2,
 * with gamma_ij from the current internal energies and
 * dK_ij = ((p_i')^2 + (p_j')^2 - p_i^2 - p_j^2)/(2m).
 * ---------------------------------------------------------------------- */
static int64_t domain_of(const or_params* P, const double* qi) {
  int64_t c[3];
  for (int d = 0; d < 3; ++d) {
    double s = (double)P->ndom[d] / P->box[d];
    double x = floor(qi[d] * s);
    if (x < 0.0) x = 0.0;
    if (x > (double)(P->ndom[d] - 1)) x = (double)(P->ndom[d] - 1);
    c[d] = (int64_t)x;
  }
  return c[0] + (int64_t)P->ndom[0] * (c[1] + (int64_t)P->ndom[1] * c[2]);
}

static int ssa_pair(const or_params* P, int64_t i, int64_t j, double r, double* p, double* eps) {
  double thi = or_theta_newton(P, eps[i], NULL), thj = or_theta_newton(P, eps[j], NULL);
  if (!(eps[i] > 0.0) || !(eps[j] > 0.0) || !(thi > 0.0) || !(thj > 0.0)) return OR_ENEG_EINT;
  double w = 1.0 - r / P->rc;
  double chi = w * w;
  double gij = 0.5 * P->gamma * P->kT_ref * (1.0 / thi + 1.0 / thj);
  double sigma = sqrt(2.0 * P->gamma * P->kT_ref);
  double a = 2.0 * gij / P->mass * chi * P->dt;
  double decay = expm1(-a);                              /* e^{-a} - 1 */
  double var = gij > 0.0 ? -expm1(-2.0 * a) / gij : 4.0 * chi * P->dt / P->mass;
  double amp = sigma * sqrt(P->mass * var);
  double G[3];
  or_gauss3(P->seed, (uint32_t)P->replica, P->step, (uint32_t)i, (uint32_t)j, G);
  double k0 = 0.0, k1 = 0.0;
  for (int c = 0; c < 3; ++c) {
    double pij = p[3 * i + c] - p[3 * j + c];
    double D = decay * pij + amp * G[c];
    double pi = p[3 * i + c] + 0.5 * D, pj = p[3 * j + c] - 0.5 * D;
    k0 += p[3 * i + c] * p[3 * i + c] + p[3 * j + c] * p[3 * j + c];
    k1 += pi * pi + pj * pj;
    p[3 * i + c] = pi;
    p[3 * j + c] = pj;
  }
  double dK = (k1 - k0) / (2.0 * P->mass);
  eps[i] -= 0.5 * dK;
  eps[j] -= 0.5 * dK;
  return OR_OK;
}

int or_fd_hybrid(const or_params* P, const double* q, double* p, double* eps,
                 const int32_t* lohi, int64_t npairs) {
  int32_t* cross = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)(npairs > 0 ? npairs : 1));
  if (!cross) return OR_ENOMEM;
  int64_t nc = 0;
  for (int64_t k = 0; k < npairs; ++k) {  /* lohi is sorted by (lo, hi) */
    int64_t i = lohi[2 * k], j = lohi[2 * k + 1];
    if (domain_of(P, &q[3 * i]) == domain_of(P, &q[3 * j])) {
      double d[3];
      double r = sqrt(separation(P, &q[3 * i], &q[3 * j], d));
      int rc_ = ssa_pair(P, i, j, r, p, eps);
      if (rc_ != OR_OK) { free(cross); return rc_; }
    } else {
      cross[2 * nc] = (int32_t)i;
      cross[2 * nc + 1] = (int32_t)j;
      ++nc;
    }
  }
  or_params Q = *P;
  Q.scheme = 0;
  int rc_ = or_fd_pairs(&Q, q, p, eps, cross, nc, NULL);
  free(cross);
  return rc_;
}

/* FD sub-step alone at the current positions (pairs from the cell list). */
int or_fd(const or_params* P, const double* q, double* p, double* eps, double* dp_out) {
  int32_t* pairs = NULL;
  int64_t np = 0;
  int rc_ = build_pairs(P, q, &pairs, &np);
  if (rc_ != OR_OK) return rc_;
  if (P->scheme == 2) {
    double* p0 = dp_out ? (double*)malloc(sizeof(double) * 3 * (size_t)P->n) : NULL;
    if (p0) memcpy(p0, p, sizeof(double) * 3 * (size_t)P->n);
    rc_ = or_fd_hybrid(P, q, p, eps, pairs, np);
    if (p0) {
      for (int64_t k = 0; k < 3 * P->n; ++k) dp_out[k] = p[k] - p0[k];
      free(p0);
    }
  } else {
    rc_ = or_fd_pairs(P, q, p, eps, pairs, np, dp_out);
  }
  free(pairs);
  return rc_;
}

/* ------------------------------------------------------------------------
 * One step n -> n+1 (Sec. 3.1: velocity-Verlet on the Hamiltonian part,
 * then the fluctuation/dissipation part on the new positions):
 *   p <- p + dt/2 F(q);  q <- q + dt p/m (wrapped);  F <- F(q);
 *   p <- p + dt/2 F;     (p, eps) <- FD(q, p, eps; G^n).
 * F holds F(q^n) on entry and F(q^{n+1}) on exit; U receives U(q^{n+1}).
 * ---------------------------------------------------------------------- */
int or_step(or_params* P, double* q, double* p, double* eps, double* F, double* U) {
  int rc_ = or_check_box(P);
  if (rc_ != OR_OK) return rc_;
  const int64_t n = P->n;
  for (int64_t i = 0; i < n; ++i)
    for (int c = 0; c < 3; ++c) {
      p[3 * i + c] = p[3 * i + c] + 0.5 * P->dt * F[3 * i + c];
      q[3 * i + c] = q[3 * i + c] + P->dt * p[3 * i + c] / P->mass;
      if (P->periodic[c]) q[3 * i + c] = or_wrap(q[3 * i + c], P->box[c]);
    }
  int32_t* pairs = NULL;
  int64_t np = 0;
  rc_ = build_pairs(P, q, &pairs, &np);
  if (rc_ != OR_OK) return rc_;
  or_forces_pairs(P, q, pairs, np, F, U);
  for (int64_t i = 0; i < n; ++i)
    for (int c = 0; c < 3; ++c) p[3 * i + c] = p[3 * i + c] + 0.5 * P->dt * F[3 * i + c];
  rc_ = P->scheme == 2 ? or_fd_hybrid(P, q, p, eps, pairs, np)
                      : or_fd_pairs(P, q, p, eps, pairs, np, NULL);
  free(pairs);
  P->step += 1;
  if (rc_ == OR_OK && P->project) {
    /* Sec. 4.2: eps_i <- eps_i - (E(x~) - E0)/N, x~ the unconstrained update */
    double K = 0.0, S = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      K += (p[3 * i] * p[3 * i] + p[3 * i + 1] * p[3 * i + 1] + p[3 * i + 2] * p[3 * i + 2]) /
           (2.0 * P->mass);
      S += eps[i];
    }
    double shift = (*U + K + S - P->E0) / (double)n;
    for (int64_t i = 0; i < n; ++i) {
      eps[i] -= shift;
      if (!(eps[i] > 0.0)) rc_ = OR_ENEG_EINT;
    }
  }
  return rc_;
}

int or_run(or_params* P, double* q, double* p, double* eps, double* F, double* U, int64_t nsteps,
           double* energies_out /* nsteps x 10 or NULL */);

/* ------------------------------------------------------------------------
 * Observables (Sec. 2.1 energy with p^2/(2m); Sec. 2.2 eqs. Tkin, Tint):
 * out = {U, K, sum eps, E, Px, Py, Pz, T_kin, T_int, step}
 * with T_kin = sum p^2/m / (3(N-1)) and T_int = N / sum_i 1/T_i.
 * ---------------------------------------------------------------------- */
int or_energies(const or_params* P, const double* p, const double* eps, double U, double out[10]) {
  double K = 0.0, E = 0.0, Px = 0.0, Py = 0.0, Pz = 0.0, sinv = 0.0;
  for (int64_t i = 0; i < P->n; ++i) {
    double p2 = p[3 * i] * p[3 * i] + p[3 * i + 1] * p[3 * i + 1] + p[3 * i + 2] * p[3 * i + 2];
    K += p2 / (2.0 * P->mass);
    E += eps[i];
    Px += p[3 * i]; Py += p[3 * i + 1]; Pz += p[3 * i + 2];
    if (!(eps[i] > 0.0)) return OR_ENEG_EINT;
    sinv += 1.0 / or_theta_newton(P, eps[i], NULL);
  }
  out[0] = U;
  out[1] = K;
  out[2] = E;
  out[3] = U + K + E;
  out[4] = Px; out[5] = Py; out[6] = Pz;
  out[7] = 2.0 * K / (3.0 * (double)(P->n - 1));
  out[8] = (double)P->n / sinv;
  out[9] = (double)P->step;
  return OR_OK;
}

int or_run(or_params* P, double* q, double* p, double* eps, double* F, double* U, int64_t nsteps,
           double* energies_out) {
  for (int64_t s = 0; s < nsteps; ++s) {
    int rc_ = or_step(P, q, p, eps, F, U);
    if (rc_ != OR_OK) return rc_;
    if (energies_out) {
      rc_ = or_energies(P, p, eps, *U, &energies_out[10 * s]);
      if (rc_ != OR_OK) return rc_;
    }
  }
  return OR_OK;
}

int or_config_temperature(const or_params* P, const double* q, double* grad2, double* lap) {
  int32_t* pairs = NULL;
  int64_t np = 0;
  int rc_ = build_pairs(P, q, &pairs, &np);
  if (rc_ != OR_OK) return rc_;
  double* F = (double*)malloc(sizeof(double) * 3 * (size_t)P->n);
  if (!F) { free(pairs); return OR_ENOMEM; }
  double U;
  or_forces_pairs(P, q, pairs, np, F, &U);
  double g = 0.0, l = 0.0;
  for (int64_t i = 0; i < 3 * P->n; ++i) g += F[i] * F[i];
  for (int64_t k = 0; k < np; ++k) {
    double d[3];
    double r = sqrt(separation(P, &q[3 * pairs[2 * k]], &q[3 * pairs[2 * k + 1]], d));
    if (!(r > 0.0)) continue;
    double v, dv, d2v;
    or_pair_potential(P, r, &v, &dv, &d2v);
    l += 2.0 * (d2v + 2.0 * dv / r);
  }
  free(F);
  free(pairs);
  *grad2 = g;
  *lap = l;
  return OR_OK;
}

/* Projection on the internal energies (Sec. 4.2): eps_i -= (E - E0)/N. */
void or_project(const or_params* P, double* eps, double E, double E0) {
  double shift = (E - E0) / (double)P->n;
  for (int64_t i = 0; i < P->n; ++i) eps[i] -= shift;
}

/* ------------------------------------------------------------------------
 * Surrogate for theta(eps): a 1 -> 32 -> 32 -> 1 perceptron with tanh hidden
 * units, in FP64, used to check the GPU training gradients and inference.
 *   x  = (ln eps - in_c) / in_s
 *   h1 = tanh(W1 x + b1),  h2 = tanh(W2 h1 + b2),  y = W3 . h2 + b3
 *   theta = exp(out_c + out_s y)
 * Weights are packed as W1[32], b1[32], W2[32][32] (row = output unit),
 * b2[32], W3[32], b3[1]: 1153 values.  The loss over a batch is
 * mean_k (y_k - t_k)^2 with t_k = (ln theta_k - out_c)/out_s.
 * ---------------------------------------------------------------------- */
#define MLP_H 32
#define MLP_NPARAM (MLP_H + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1)

int or_mlp_nparam(void) { return MLP_NPARAM; }

static void mlp_forward1(const double* w, double x, double h1[MLP_H], double h2[MLP_H], double* y) {
  const double* W1 = w;
  const double* b1 = W1 + MLP_H;
  const double* W2 = b1 + MLP_H;
  const double* b2 = W2 + MLP_H * MLP_H;
  const double* W3 = b2 + MLP_H;
  const double* b3 = W3 + MLP_H;
  for (int a = 0; a < MLP_H; ++a) h1[a] = tanh(W1[a] * x + b1[a]);
  for (int a = 0; a < MLP_H; ++a) {
    double s = b2[a];
    for (int b = 0; b < MLP_H; ++b) s += W2[a * MLP_H + b] * h1[b];
    h2[a] = tanh(s);
  }
  double s = b3[0];
  for (int a = 0; a < MLP_H; ++a) s += W3[a] * h2[a];
  *y = s;
}

void or_mlp_forward(const double* w, const double* x, double* y, int64_t n) {
  double h1[MLP_H], h2[MLP_H];
  for (int64_t k = 0; k < n; ++k) mlp_forward1(w, x[k], h1, h2, &y[k]);
}

/* loss and its gradient with respect to the packed weights (backprop) */
double or_mlp_loss_grad(const double* w, const double* x, const double* t, int64_t n,
                        double* grad) {
  const double* W2 = w + 2 * MLP_H;
  const double* W3 = W2 + MLP_H * MLP_H + MLP_H;
  double* gW1 = grad;
  double* gb1 = gW1 + MLP_H;
  double* gW2 = gb1 + MLP_H;
  double* gb2 = gW2 + MLP_H * MLP_H;
  double* gW3 = gb2 + MLP_H;
  double* gb3 = gW3 + MLP_H;
  memset(grad, 0, sizeof(double) * MLP_NPARAM);
  double loss = 0.0;
  double h1[MLP_H], h2[MLP_H], d2[MLP_H], d1[MLP_H];
  for (int64_t k = 0; k < n; ++k) {
    double y;
    mlp_forward1(w, x[k], h1, h2, &y);
    double e = y - t[k];
    loss += e * e;
    double dy = 2.0 * e / (double)n;
    gb3[0] += dy;
    for (int a = 0; a < MLP_H; ++a) {
      gW3[a] += dy * h2[a];
      d2[a] = dy * W3[a] * (1.0 - h2[a] * h2[a]);
    }
    for (int a = 0; a < MLP_H; ++a) {
      gb2[a] += d2[a];
      for (int b = 0; b < MLP_H; ++b) gW2[a * MLP_H + b] += d2[a] * h1[b];
    }
    for (int b = 0; b < MLP_H; ++b) {
      double s = 0.0;
      for (int a = 0; a < MLP_H; ++a) s += W2[a * MLP_H + b] * d2[a];
      d1[b] = s * (1.0 - h1[b] * h1[b]);
      gb1[b] += d1[b];
      gW1[b] += d1[b] * x[k];
    }
  }
  return loss / (double)n;
}
