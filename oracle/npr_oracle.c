/*
 * FP64 CPU oracle of the one-colour four-fermion operator of the paper's NPR
 * code (section "GTX Titan Black", Eq. (1)): TEST INFRASTRUCTURE ONLY, loaded by
 * the tests, the smoke check and the benchmark's CPU baseline.  It shares no
 * code with the GPU library.
 *
 * Eq. (1) pairs two staggered bilinears over the sixteen corners A, B, C, D of
 * the hypercube z (site 2z + A etc.), with spin-taste matrices
 * (gamma_S (x) xi_F)bar_{AB} and colour joined across the bilinears by the gauge
 * link averaged over all shortest paths between two corners:
 *   O(z) = chibar_{c1}(z_A) M1_{AB} chi_{c2}(z_B) chibar_{c3}(z_C) M2_{CD} chi_{c4}(z_D)
 *          [U_AD]_{c1 c4}(z) [U_CB]_{c3 c2}(z)
 * Its matrix element between quark states (the part the NPR code spends its
 * time on) replaces each chi(x) by a propagator G(x) from a common source and
 * each chibar(x) by its staggered conjugate eps(x) G(x)^dagger, with
 * eps(x) = (-1)^(x+y+z+t); the source colours a1..a4 stay free:
 *   V[a1][a2][a3][a4](z) = sum_{A,B,C,D} M1_{AB} M2_{CD} eps(z_A) eps(z_C)
 *       (G1(z_A)^dag U_AD G4(z_D))_{a1 a4} (G3(z_C)^dag U_CB G2(z_B))_{a3 a2}
 * The paper gives no further formula; the readings (this replacement, the
 * definition of the spin-taste matrix, the path average) are stated here:
 *   (gamma_S (x) xi_F)bar_{AB} = (1/4) Tr[gamma_A^dag gamma_S gamma_B gamma_F^dag],
 *   gamma_A = gamma_1^A1 gamma_2^A2 gamma_3^A3 gamma_4^A4 (Euclidean, Hermitian),
 *   U_AD = the mean over every shortest path from z_A to z_D inside the
 *   hypercube of the ordered product of links (U_mu(x) stepping +mu from x,
 *   U_mu(x - mu)^dag stepping -mu), the identity for A = D.
 * Corner and spin-taste labels are 4-bit masks: bit mu (x, y, z, t) = component mu.
 */
#include <complex.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* Euclidean gamma matrices in a chiral representation: Hermitian, squaring to
   one, pairwise anticommuting (checked by the tests). */
static void gamma_mu(int mu, cplx g[4][4]) {
  memset(g, 0, sizeof(cplx) * 16);
  const cplx ii = 1.0 * _Complex_I;
  switch (mu) {
    case 0: g[0][3] = ii; g[1][2] = ii; g[2][1] = -ii; g[3][0] = -ii; break;
    case 1: g[0][3] = -1; g[1][2] = 1; g[2][1] = 1; g[3][0] = -1; break;
    case 2: g[0][2] = ii; g[1][3] = -ii; g[2][0] = -ii; g[3][1] = ii; break;
    default: g[0][2] = 1; g[1][3] = 1; g[2][0] = 1; g[3][1] = 1; break;
  }
}

static void mat4_mul(const cplx a[4][4], const cplx b[4][4], cplx c[4][4]) {
  cplx t[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      cplx s = 0;
      for (int k = 0; k < 4; ++k) s += a[i][k] * b[k][j];
      t[i][j] = s;
    }
  memcpy(c, t, sizeof(t));
}

/* gamma_X = gamma_1^X1 gamma_2^X2 gamma_3^X3 gamma_4^X4 */
static void gamma_mask(int X, cplx g[4][4]) {
  memset(g, 0, sizeof(cplx) * 16);
  for (int i = 0; i < 4; ++i) g[i][i] = 1;
  for (int mu = 0; mu < 4; ++mu)
    if (X >> mu & 1) {
      cplx m[4][4];
      gamma_mu(mu, m);
      mat4_mul(g, m, g);
    }
}

static void dagger4(const cplx a[4][4], cplx b[4][4]) {
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) b[i][j] = conj(a[j][i]);
}

/* The 16 x 16 spin-taste matrix (1/4) Tr[gamma_A^dag gamma_S gamma_B gamma_F^dag],
   row A, column B, as complex numbers (re, im interleaved). */
int oracle_spin_taste(int S, int F, double* out) {
  if (S < 0 || S > 15 || F < 0 || F > 15 || !out) return -1;
  cplx gS[4][4], gF[4][4], gFd[4][4];
  gamma_mask(S, gS);
  gamma_mask(F, gF);
  dagger4(gF, gFd);
  for (int A = 0; A < 16; ++A) {
    cplx gA[4][4], gAd[4][4], t[4][4];
    gamma_mask(A, gA);
    dagger4(gA, gAd);
    mat4_mul(gAd, gS, t);
    for (int B = 0; B < 16; ++B) {
      cplx gB[4][4], u[4][4];
      gamma_mask(B, gB);
      mat4_mul(t, gB, u);
      mat4_mul(u, gFd, u);
      const cplx tr = 0.25 * (u[0][0] + u[1][1] + u[2][2] + u[3][3]);
      out[2 * (A * 16 + B)] = creal(tr);
      out[2 * (A * 16 + B) + 1] = cimag(tr);
    }
  }
  return 0;
}

/* ---- lattice helpers ------------------------------------------------------ */

static long site_lex(const int d[4], const int c[4]) {
  return c[0] + (long)d[0] * (c[1] + (long)d[1] * (c[2] + (long)d[2] * c[3]));
}

/* corner A of hypercube z: site coordinates 2z + A */
static void corner(const int zc[4], int A, int c[4]) {
  for (int mu = 0; mu < 4; ++mu) c[mu] = 2 * zc[mu] + (A >> mu & 1);
}

static void mat3_mul(const cplx* a, const cplx* b, cplx* c) {
  cplx t[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      cplx s = 0;
      for (int k = 0; k < 3; ++k) s += a[3 * i + k] * b[3 * k + j];
      t[3 * i + j] = s;
    }
  memcpy(c, t, sizeof(t));
}

static void mat3_dag(const cplx* a, cplx* b) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) b[3 * i + j] = conj(a[3 * j + i]);
}

/* The link of one step from corner `from` along mu inside hypercube z: +mu when
   bit mu of `from` is 0 (U_mu at that site), -mu when it is 1 (the adjoint of
   U_mu at the site one step back). */
static void step_link(const int d[4], const cplx* thin, const int zc[4], int from, int mu, cplx* out) {
  int c[4];
  if (!(from >> mu & 1)) {
    corner(zc, from, c);
    memcpy(out, thin + (site_lex(d, c) * 4 + mu) * 9, sizeof(cplx) * 9);
  } else {
    corner(zc, from ^ (1 << mu), c);
    mat3_dag(thin + (site_lex(d, c) * 4 + mu) * 9, out);
  }
}

/* U_AD(z): every ordering of the directions in which A and D differ is one
   shortest path; the mean of the ordered link products over all of them. */
int oracle_link_average(const int d[4], const double* thin_d, const int zc[4], int A, int D, double* out) {
  if (!d || !thin_d || !zc || !out || A < 0 || A > 15 || D < 0 || D > 15) return -1;
  const cplx* thin = (const cplx*)thin_d;
  int dirs[4], n = 0;
  for (int mu = 0; mu < 4; ++mu)
    if ((A ^ D) >> mu & 1) dirs[n++] = mu;
  cplx acc[9] = {0};
  long npath = 0;
  /* all n! orders of dirs, by Heap's algorithm */
  int perm[4], cnt[4] = {0, 0, 0, 0};
  for (int k = 0; k < n; ++k) perm[k] = dirs[k];
  for (;;) {
    cplx p[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    int at = A;
    for (int k = 0; k < n; ++k) {
      cplx L[9];
      step_link(d, thin, zc, at, perm[k], L);
      mat3_mul(p, L, p);
      at ^= 1 << perm[k];
    }
    for (int k = 0; k < 9; ++k) acc[k] += p[k];
    ++npath;
    /* next permutation (Heap, iterative) */
    int i = 1;
    while (i < n && cnt[i] >= i) cnt[i++] = 0;
    if (i >= n) break;
    const int j = (i & 1) ? cnt[i] : 0;
    const int t = perm[i];
    perm[i] = perm[j];
    perm[j] = t;
    ++cnt[i];
  }
  for (int k = 0; k < 9; ++k) {
    const cplx v = acc[k] / (double)npath;
    out[2 * k] = creal(v);
    out[2 * k + 1] = cimag(v);
  }
  return 0;
}

/*
 * V_I(z) for nop operators I = (S1, F1, S2, F2) (ops[4 * k ...]) at the hypercubes
 * listed in zs (nz entries; NULL: every hypercube in lexicographic order of
 * z = (zx, zy, zz, zt) with zx fastest).  thin: [V][4][3][3] complex links.
 * G1..G4: [V][3][3] complex propagators, row = colour at the site, column =
 * source colour.  out: [nop][nz][3][3][3][3] complex, index [a1][a2][a3][a4].
 */
int oracle_npr_fourfermion(const int d[4], const double* thin_d, const double* g1, const double* g2,
                           const double* g3, const double* g4, int nop, const int* ops, const long* zs, long nz,
                           double* out_d) {
  if (!d || !thin_d || !g1 || !g2 || !g3 || !g4 || !ops || !out_d || nop <= 0) return -1;
  for (int mu = 0; mu < 4; ++mu)
    if (d[mu] < 2 || (d[mu] & 1)) return -1;
  const cplx* thin = (const cplx*)thin_d;
  const cplx* G[4] = {(const cplx*)g1, (const cplx*)g2, (const cplx*)g3, (const cplx*)g4};
  const long hz[4] = {d[0] / 2, d[1] / 2, d[2] / 2, d[3] / 2};
  const long nz_all = hz[0] * hz[1] * hz[2] * hz[3];
  const long n = zs ? nz : nz_all;
  cplx* out = (cplx*)out_d;
  double* M = (double*)malloc(sizeof(double) * 2 * 256 * 2 * nop);
  if (!M) return -2;
  for (int k = 0; k < nop; ++k) {
    if (oracle_spin_taste(ops[4 * k], ops[4 * k + 1], M + 2 * 256 * (2 * k)) ||
        oracle_spin_taste(ops[4 * k + 2], ops[4 * k + 3], M + 2 * 256 * (2 * k + 1))) {
      free(M);
      return -1;
    }
  }
  int bad = 0;
#pragma omp parallel for schedule(dynamic)
  for (long iz = 0; iz < n; ++iz) {
    long zl = zs ? zs[iz] : iz;
    if (zl < 0 || zl >= nz_all) {
      bad = 1;
      continue;
    }
    int zc[4];
    for (int mu = 0; mu < 4; ++mu) {
      zc[mu] = (int)(zl % hz[mu]);
      zl /= hz[mu];
    }
    /* every pair's link average, then the two bilinear colour matrices */
    cplx U[16][16][9];
    for (int A = 0; A < 16; ++A)
      for (int D = 0; D < 16; ++D) oracle_link_average(d, thin_d, zc, A, D, (double*)U[A][D]);
    const cplx* Gs[4][16];
    double eps[16];
    for (int A = 0; A < 16; ++A) {
      int c[4];
      corner(zc, A, c);
      const long s = site_lex(d, c);
      for (int f = 0; f < 4; ++f) Gs[f][A] = G[f] + s * 9;
      eps[A] = ((c[0] + c[1] + c[2] + c[3]) & 1) ? -1.0 : 1.0;
    }
    for (int k = 0; k < nop; ++k) {
      const double* M1 = M + 2 * 256 * (2 * k);
      const double* M2 = M + 2 * 256 * (2 * k + 1);
      cplx V[81] = {0};
      for (int A = 0; A < 16; ++A)
        for (int B = 0; B < 16; ++B) {
          const cplx m1 = M1[2 * (16 * A + B)] + M1[2 * (16 * A + B) + 1] * _Complex_I;
          if (m1 == 0) continue;
          for (int C = 0; C < 16; ++C)
            for (int D = 0; D < 16; ++D) {
              const cplx m2 = M2[2 * (16 * C + D)] + M2[2 * (16 * C + D) + 1] * _Complex_I;
              if (m2 == 0) continue;
              const cplx w = m1 * m2 * eps[A] * eps[C];
              /* X = G1(z_A)^dag U_AD G4(z_D),  Y = G3(z_C)^dag U_CB G2(z_B) */
              cplx X[9], Y[9], h[9];
              mat3_dag(Gs[0][A], h);
              mat3_mul(h, U[A][D], X);
              mat3_mul(X, Gs[3][D], X);
              mat3_dag(Gs[2][C], h);
              mat3_mul(h, U[C][B], Y);
              mat3_mul(Y, Gs[1][B], Y);
              for (int a1 = 0; a1 < 3; ++a1)
                for (int a2 = 0; a2 < 3; ++a2)
                  for (int a3 = 0; a3 < 3; ++a3)
                    for (int a4 = 0; a4 < 3; ++a4)
                      V[27 * a1 + 9 * a2 + 3 * a3 + a4] += w * X[3 * a1 + a4] * Y[3 * a3 + a2];
            }
        }
      memcpy(out + ((long)k * n + iz) * 81, V, sizeof(V));
    }
  }
  free(M);
  return bad ? -1 : 0;
}
