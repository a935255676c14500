/*
 * asqtad_oracle.c -- plain FP64 CPU oracle for the even-odd asqtad CG.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library includes, links or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark load it.  It shares no code with the HIP path.
 *
 * What it computes (the paper's CG workload on MILC asqtad lattices,
 * "GTX Titan Black" section, CG performance figure and table; the paper
 * states no formulas, so the standard staggered definitions are used):
 *
 *   (D psi)(x) = sum_mu eta_mu(x) [ F_mu(x) psi(x+mu) - F_mu(x-mu)^dag psi(x-mu)
 *                                 + L_mu(x) psi(x+3mu) - L_mu(x-3mu)^dag psi(x-3mu) ]
 *
 *   eta_x = 1, eta_y = (-1)^x, eta_z = (-1)^(x+y), eta_t = (-1)^(x+y+z)
 *   psi is periodic in x, y, z and antiperiodic in t: a neighbour whose
 *   unwrapped time coordinate leaves [0, T) contributes with a minus sign.
 *   Links are periodic in every direction.
 *
 *   M = 2m + D,   A = (M^dag M)_ee = 4 m^2 - D_eo D_oe   (even sites)
 *
 * CG is Hestenes-Stiefel from x0 = 0 with the recursive-residual stop
 * |r| <= tol |b|; the true residual |b - A x| / |b| is reported.
 *
 * Layouts (host, double precision, complex numbers as (re, im) pairs):
 *   links  [V][4][3][3][2], lex = x + X*(y + Y*(z + Z*t)), mu = x,y,z,t,
 *          (U psi)_a = sum_b U[a][b] psi_b, U_mu(x) multiplies psi(x+mu)
 *   vectors of one parity [V/2][3][2], index lex/2 (checkerboard order)
 *
 * The site loop of the operator is shared out over OpenMP threads; every
 * reduction runs serially in site order.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

static long vol(const int d[4]) { return (long)d[0] * d[1] * d[2] * d[3]; }

static void coords_of(const int d[4], long lex, int c[4]) {
  c[0] = (int)(lex % d[0]); lex /= d[0];
  c[1] = (int)(lex % d[1]); lex /= d[1];
  c[2] = (int)(lex % d[2]); lex /= d[2];
  c[3] = (int)lex;
}

static long lex_of(const int d[4], const int c[4]) {
  return c[0] + (long)d[0] * (c[1] + (long)d[1] * (c[2] + (long)d[2] * c[3]));
}

static int parity_of(const int c[4]) { return (c[0] + c[1] + c[2] + c[3]) & 1; }

/* MILC staggered phase eta_mu(x) = (-1)^(sum of the coordinates before mu). */
static double eta(int mu, const int c[4]) {
  int s = 0;
  for (int nu = 0; nu < mu; ++nu) s += c[nu];
  return (s & 1) ? -1.0 : 1.0;
}

/* Site x + h*mu with periodic wrap; *sign is -1 when the hop crosses the
   time boundary (antiperiodic fermions), else +1. */
static long hop(const int d[4], const int c[4], int mu, int h, double* sign) {
  int n[4] = {c[0], c[1], c[2], c[3]};
  int u = c[mu] + h;
  *sign = 1.0;
  if (mu == 3 && (u < 0 || u >= d[3])) *sign = -1.0;
  u %= d[mu];
  if (u < 0) u += d[mu];
  n[mu] = u;
  return lex_of(d, n);
}

static const cplx* link_at(const double* links, long lex, int mu) {
  return (const cplx*)(links + ((lex * 4 + mu) * 9) * 2);
}

/* acc += s * U psi */
static void mul_add(cplx acc[3], double s, const cplx* U, const cplx* psi) {
  for (int a = 0; a < 3; ++a) {
    cplx v = 0;
    for (int b = 0; b < 3; ++b) v += U[a * 3 + b] * psi[b];
    acc[a] += s * v;
  }
}

/* acc += s * U^dag psi */
static void mul_adj_add(cplx acc[3], double s, const cplx* U, const cplx* psi) {
  for (int a = 0; a < 3; ++a) {
    cplx v = 0;
    for (int b = 0; b < 3; ++b) v += conj(U[b * 3 + a]) * psi[b];
    acc[a] += s * v;
  }
}

static int check_dims(const int d[4]) {
  for (int mu = 0; mu < 4; ++mu)
    if (d[mu] < 4 || (d[mu] & 1)) return -1;
  return 0;
}

/* out (parity p sites) = D restricted to parity p <- parity 1-p. */
int oracle_dslash(const int dims[4], const double* fat, const double* lng, int out_parity,
                  const double* in, double* out) {
  if (check_dims(dims) || (out_parity != 0 && out_parity != 1)) return -1;
  const long V = vol(dims);
  const cplx* psi = (const cplx*)in;
  cplx* res = (cplx*)out;
#pragma omp parallel for schedule(static)
  for (long lex = 0; lex < V; ++lex) {
    int c[4];
    coords_of(dims, lex, c);
    if (parity_of(c) != out_parity) continue;
    cplx acc[3] = {0, 0, 0};
    for (int mu = 0; mu < 4; ++mu) {
      const double e = eta(mu, c);
      double s;
      long y;
      /* one-hop forward and backward */
      y = hop(dims, c, mu, +1, &s);
      mul_add(acc, e * s, link_at(fat, lex, mu), psi + (y / 2) * 3);
      y = hop(dims, c, mu, -1, &s);
      mul_adj_add(acc, -e * s, link_at(fat, y, mu), psi + (y / 2) * 3);
      /* three-hop forward and backward */
      y = hop(dims, c, mu, +3, &s);
      mul_add(acc, e * s, link_at(lng, lex, mu), psi + (y / 2) * 3);
      y = hop(dims, c, mu, -3, &s);
      mul_adj_add(acc, -e * s, link_at(lng, y, mu), psi + (y / 2) * 3);
    }
    for (int a = 0; a < 3; ++a) res[(lex / 2) * 3 + a] = acc[a];
  }
  return 0;
}

/* out = (4 m^2 - D_eo D_oe) in, on even sites. */
int oracle_apply_A(const int dims[4], const double* fat, const double* lng, double mass,
                   const double* in, double* out) {
  if (check_dims(dims)) return -1;
  const long n = vol(dims) / 2 * 3;
  cplx* t = (cplx*)malloc(sizeof(cplx) * n);
  cplx* u = (cplx*)malloc(sizeof(cplx) * n);
  if (!t || !u) { free(t); free(u); return -2; }
  oracle_dslash(dims, fat, lng, 1, in, (double*)t);
  oracle_dslash(dims, fat, lng, 0, (const double*)t, (double*)u);
  const cplx* v = (const cplx*)in;
  cplx* w = (cplx*)out;
  for (long k = 0; k < n; ++k) w[k] = 4.0 * mass * mass * v[k] - u[k];
  free(t);
  free(u);
  return 0;
}

static double norm2(const cplx* a, long n) {
  double s = 0;
  for (long k = 0; k < n; ++k) s += creal(a[k]) * creal(a[k]) + cimag(a[k]) * cimag(a[k]);
  return s;
}

static double redot(const cplx* a, const cplx* b, long n) {
  double s = 0;
  for (long k = 0; k < n; ++k) s += creal(conj(a[k]) * b[k]);
  return s;
}

/* |b - A x| / |b| (0 when b = 0 and x = 0). */
double oracle_true_residual(const int dims[4], const double* fat, const double* lng, double mass,
                            const double* b, const double* x) {
  if (check_dims(dims)) return -1.0;
  const long n = vol(dims) / 2 * 3;
  cplx* Ax = (cplx*)malloc(sizeof(cplx) * n);
  if (!Ax) return -2.0;
  oracle_apply_A(dims, fat, lng, mass, x, (double*)Ax);
  const cplx* bb = (const cplx*)b;
  double rr = 0, b2 = norm2(bb, n);
  for (long k = 0; k < n; ++k) {
    cplx r = bb[k] - Ax[k];
    rr += creal(r) * creal(r) + cimag(r) * cimag(r);
  }
  free(Ax);
  if (b2 == 0) return sqrt(rr);
  return sqrt(rr / b2);
}

/*
 * Plain CG on A x = b from x = 0.  Returns 0 on convergence, 1 when maxiter
 * iterations ran without meeting the stop rule, <0 on bad arguments.
 * When resid_hist is not NULL it receives |r_k|/|b| for k = 0..iters.
 */
int oracle_cg(const int dims[4], const double* fat, const double* lng, double mass,
              const double* b, double* x, double tol, int maxiter, int* iters_out,
              double* true_resid_out, double* resid_hist) {
  if (check_dims(dims) || tol <= 0 || maxiter < 0) return -1;
  const long n = vol(dims) / 2 * 3;
  const cplx* bb = (const cplx*)b;
  cplx* xx = (cplx*)x;
  cplx* r = (cplx*)malloc(sizeof(cplx) * n);
  cplx* p = (cplx*)malloc(sizeof(cplx) * n);
  cplx* Ap = (cplx*)malloc(sizeof(cplx) * n);
  if (!r || !p || !Ap) { free(r); free(p); free(Ap); return -2; }
  for (long k = 0; k < n; ++k) { xx[k] = 0; r[k] = bb[k]; p[k] = bb[k]; }
  const double b2 = norm2(bb, n);
  double rr = b2;
  int it = 0, status = 1;
  if (resid_hist) resid_hist[0] = (b2 > 0) ? 1.0 : 0.0;
  if (b2 == 0) status = 0;
  while (status == 1 && it < maxiter) {
    oracle_apply_A(dims, fat, lng, mass, (const double*)p, (double*)Ap);
    const double alpha = rr / redot(p, Ap, n);
    for (long k = 0; k < n; ++k) { xx[k] += alpha * p[k]; r[k] -= alpha * Ap[k]; }
    const double rr_new = norm2(r, n);
    ++it;
    if (resid_hist) resid_hist[it] = sqrt(rr_new / b2);
    if (sqrt(rr_new) <= tol * sqrt(b2)) { status = 0; break; }
    const double beta = rr_new / rr;
    for (long k = 0; k < n; ++k) p[k] = r[k] + beta * p[k];
    rr = rr_new;
  }
  if (iters_out) *iters_out = it;
  if (true_resid_out) *true_resid_out = oracle_true_residual(dims, fat, lng, mass, b, x);
  free(r); free(p); free(Ap);
  return status;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/*
 * Asqtad link construction from thin links.  The paper's lattices are MILC
 * asqtad ensembles (CG benchmark, "GTX Titan Black" section) but it prints no
 * smearing formula, so the standard asqtad action is written out here as a
 * plain sum over paths:
 *
 *   F_mu(x) = sum over the paths P listed below of c(P) * (ordered product of
 *             thin links along P), every P running from x to x + mu
 *   L_mu(x) = c_N U_mu(x) U_mu(x+mu) U_mu(x+2mu)
 *
 * nu, rho, sigma are signed directions on pairwise different axes, none on
 * mu's axis:
 *
 *   one link             [mu]                                  c1 = 5/8
 *   3-staple   (6 paths) [nu, mu, -nu]                         c3 = 1/16  / u0^2
 *   5-staple  (24 paths) [nu, rho, mu, -rho, -nu]              c5 = 1/64  / u0^4
 *   7-staple  (48 paths) [nu, rho, sigma, mu, -sigma, -rho, -nu]  c7 = 1/384 / u0^6
 *   Lepage     (6 paths) [nu, nu, mu, -nu, -nu]                cL = -1/16 / u0^4
 *   Naik                 [mu, mu, mu]                          cN = -1/24 / u0^2
 *
 * A step +nu from site y multiplies U_nu(y); a step -nu multiplies
 * U_nu(y - nu)^dag.  Thin links are periodic in every direction (the time
 * boundary sign belongs to the operator).  u0 is the tadpole factor.
 */
static void mat_mul_into(cplx C[9], const cplx A[9], const cplx B[9]) {
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      cplx v = 0;
      for (int k = 0; k < 3; ++k) v += A[a * 3 + k] * B[k * 3 + b];
      C[a * 3 + b] = v;
    }
}

static void mat_mul_adj_into(cplx C[9], const cplx A[9], const cplx B[9]) {
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      cplx v = 0;
      for (int k = 0; k < 3; ++k) v += A[a * 3 + k] * conj(B[b * 3 + k]);
      C[a * 3 + b] = v;
    }
}

/* acc += coeff * (product of the thin links along the signed steps, from site c);
   a step is +(axis + 1) or -(axis + 1). */
static void add_path(const int d[4], const double* thin, const int c[4], const int* steps, int n,
                     double coeff, cplx acc[9]) {
  int y[4] = {c[0], c[1], c[2], c[3]};
  cplx P[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, Q[9];
  for (int k = 0; k < n; ++k) {
    const int mu = abs(steps[k]) - 1;
    if (steps[k] > 0) {
      mat_mul_into(Q, P, link_at(thin, lex_of(d, y), mu));
      y[mu] = (y[mu] + 1) % d[mu];
    } else {
      y[mu] = (y[mu] - 1 + d[mu]) % d[mu];
      mat_mul_adj_into(Q, P, link_at(thin, lex_of(d, y), mu));
    }
    memcpy(P, Q, sizeof(P));
  }
  for (int k = 0; k < 9; ++k) acc[k] += coeff * P[k];
}

static void asqtad_site(const int d[4], const double* thin, double u0, long lex, cplx* fat, cplx* lng) {
  const double u2 = u0 * u0, u4 = u2 * u2, u6 = u4 * u2;
  const double c1 = 5.0 / 8.0, c3 = 1.0 / 16.0 / u2, c5 = 1.0 / 64.0 / u4, c7 = 1.0 / 384.0 / u6;
  const double cL = -1.0 / 16.0 / u4, cN = -1.0 / 24.0 / u2;
  int c[4];
  coords_of(d, lex, c);
  for (int mu = 0; mu < 4; ++mu) {
    const int m = mu + 1;
    cplx* F = fat + mu * 9;
    cplx* L = lng + mu * 9;
    for (int k = 0; k < 9; ++k) F[k] = L[k] = 0;
    const int one[1] = {m};
    add_path(d, thin, c, one, 1, c1, F);
    for (int nu = -4; nu <= 4; ++nu) {
      if (nu == 0 || abs(nu) == m) continue;
      const int staple[3] = {nu, m, -nu};
      add_path(d, thin, c, staple, 3, c3, F);
      const int lepage[5] = {nu, nu, m, -nu, -nu};
      add_path(d, thin, c, lepage, 5, cL, F);
      for (int rho = -4; rho <= 4; ++rho) {
        if (rho == 0 || abs(rho) == m || abs(rho) == abs(nu)) continue;
        const int five[5] = {nu, rho, m, -rho, -nu};
        add_path(d, thin, c, five, 5, c5, F);
        for (int sg = -4; sg <= 4; ++sg) {
          if (sg == 0 || abs(sg) == m || abs(sg) == abs(nu) || abs(sg) == abs(rho)) continue;
          const int seven[7] = {nu, rho, sg, m, -sg, -rho, -nu};
          add_path(d, thin, c, seven, 7, c7, F);
        }
      }
    }
    const int naik[3] = {m, m, m};
    add_path(d, thin, c, naik, 3, cN, L);
  }
}

/*
 * Fat and long links from thin links [V][4][3][3][2].  With sites == NULL the
 * outputs cover every site in lexicographic order, [V][4][3][3][2]; otherwise
 * they hold the nsites listed sites in the given order, [nsites][4][3][3][2].
 */
int oracle_asqtad_links(const int dims[4], const double* thin, double u0, const long* sites, long nsites,
                        double* fat, double* lng) {
  if (check_dims(dims) || !(u0 > 0)) return -1;
  const long V = vol(dims);
  const long n = sites ? nsites : V;
  for (long k = 0; sites && k < n; ++k)
    if (sites[k] < 0 || sites[k] >= V) return -1;
#pragma omp parallel for schedule(dynamic, 64)
  for (long k = 0; k < n; ++k) {
    const long lex = sites ? sites[k] : k;
    asqtad_site(dims, thin, u0, lex, (cplx*)fat + k * 36, (cplx*)lng + k * 36);
  }
  return 0;
}

/*
 * Mean plaquette of thin links (the tadpole factor of the asqtad coefficients
 * is u0 = P^(1/4)):
 *   P = 1 / (6 V) sum_x sum_{mu < nu} (1/3) Re tr[ U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag ]
 * Thin links are periodic in every direction.  Summed serially in site order.
 */
double oracle_plaquette(const int dims[4], const double* thin) {
  if (check_dims(dims)) return -1.0;
  const long V = vol(dims);
  double total = 0;
  for (long lex = 0; lex < V; ++lex) {
    int c[4];
    coords_of(dims, lex, c);
    for (int mu = 0; mu < 4; ++mu)
      for (int nu = mu + 1; nu < 4; ++nu) {
        cplx acc[9] = {0};
        const int loop[4] = {mu + 1, nu + 1, -(mu + 1), -(nu + 1)};
        add_path(dims, thin, c, loop, 4, 1.0, acc);
        total += creal(acc[0] + acc[4] + acc[8]) / 3.0;
      }
  }
  return total / (6.0 * (double)V);
}
