/*
 * oracle.c -- plain, slow, obviously correct CPU reference for the short-range
 * molecular-dynamics hot path (Lennard-Jones pair forces over a Verlet list,
 * skin-triggered rebuilds, leapfrog NVE / Nose-Hoover NVT).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path may include,
 * link or call this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no code, header or table with the
 * GPU implementation.
 *
 * What it computes (all O(N^2), double precision unless stated):
 *
 *  - pair sets: the set of ordered pairs (i, j), i != j, whose float32
 *    squared minimum-image distance is strictly below (r_c,ab + s)^2 rounded once
 *    to float32.  This is the content of a full (both-direction) Verlet list with
 *    skin s (paper section 3: neighbours within r_c + s are listed; sections 6 and
 *    7: strict "<" test against the per-type-pair cut-plus-skin squared; no
 *    Newton's third law).  The float32 squared distance follows one fixed
 *    operation sequence (below) built only from correctly rounded IEEE
 *    operations, so any correct implementation obtains the same bits.
 *
 *  - forces / energies / virial: the direct sum over all pairs inside the
 *    cutoff (a Verlet list with skin is an exact acceleration of this sum, paper
 *    section 3).  12-6 Lennard-Jones with the three cutoff methods of paper
 *    section 2 (truncated, shifted potential, shifted force = linear term added).
 *    Each pair's in/out decision is taken in float32 against r_c,ab^2 rounded to
 *    float32 (the decision a float32 implementation takes), its value in FP64.
 *    The potential energy of a particle is half its pair energies (paper, force
 *    kernel figure: compensation for double counting).
 *
 *  - optionally, in place of 12-6 Lennard-Jones, the pair potential
 *    U(r) = A (sigma/r)^m - B (sigma/r)^n with even integer exponents (paper section 2
 *    lists generalised Lennard-Jones and inverse-power-law potentials among the
 *    pair potentials: both are of this form), with the same three cutoff methods.
 *
 *  - optionally, the further pair potentials paper section 2 names (Yukawa,
 *    Buckingham, Gaussian core, Dzugutov, Girifalco) in their textbook forms (see
 *    gen_uf and girifalco_uf), with the same three cutoff methods.
 *
 *  - optionally, Coulomb interactions with a shifted-force cutoff (paper section
 *    9): between charges q_a, q_b (per type, reduced units in which the Coulomb
 *    constant is one) U(r) = q_a q_b (1/r - 1/r_cc + (r - r_cc)/r_cc^2) and
 *    F(r) = q_a q_b (1/r^2 - 1/r_cc^2) for r < r_cc, one cutoff r_cc for every
 *    type pair, added to the Lennard-Jones term of the pair.  The in/out decision
 *    for this term is r2_f32 < (float)(r_cc^2).
 *
 *  - the leapfrog / Nose-Hoover integrator and the displacement criterion that
 *    triggers a rebuild (paper section 6: rebuild once any particle has moved
 *    more than half the skin since the last build).
 *
 * Float32 squared distance (the specified sequence, per axis k):
 *      dx   = x_j - x_i                       (float32 subtraction)
 *      m    = rintf(dx * invL_k)              (float32 product, ties-to-even)
 *      dx   = fmaf(-m, L_k, dx)
 *      r2   = fmaf(dz, dz, fmaf(dy, dy, dx * dx))
 * with L_k the float32 box side and invL_k = (float)(1.0 / (double)L_k).
 * This file must be compiled with -ffp-contract=off and without fast-math.
 *
 * Parity status of every function: pinned (see the test-suite for the pins).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_TRUNC 0
#define ORACLE_SP 1
#define ORACLE_SF 2

/* threads the OpenMP loops of this file use */
int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* set the thread count of later OpenMP loops (k >= 1); results do not depend on it */
void oracle_set_num_threads(int k) {
#ifdef _OPENMP
  if (k >= 1) omp_set_num_threads(k);
#else
  (void)k;
#endif
}

/* ---- compensated (Neumaier) summation ------------------------------------ */
typedef struct {
  double s, c;
} nsum_t;

static void nsum_add(nsum_t *a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x))
    a->c += (a->s - t) + x;
  else
    a->c += (x - t) + a->s;
  a->s = t;
}

static double nsum_value(const nsum_t *a) { return a->s + a->c; }

/* ---- float32 squared distance, the specified sequence -------------------- */
static float r2_f32(const float *pi, const float *pj, const float *L, const float *invL) {
  float d[3];
  for (int k = 0; k < 3; ++k) {
    float dx = pj[k] - pi[k];
    float m = rintf(dx * invL[k]);
    d[k] = fmaf(-m, L[k], dx);
  }
  return fmaf(d[2], d[2], fmaf(d[1], d[1], d[0] * d[0]));
}

static void box_f32(const double *box, float *L, float *invL) {
  for (int k = 0; k < 3; ++k) {
    L[k] = (float)box[k];
    invL[k] = (float)(1.0 / (double)L[k]);
  }
}

/* cut-plus-skin squared per type pair, rounded once to float32 */
void oracle_cut_tables(int ntypes, const double *rc, double skin, float *cs2, float *rc2) {
  for (int a = 0; a < ntypes * ntypes; ++a) {
    double rs = rc[a] + skin;
    cs2[a] = (float)(rs * rs);
    rc2[a] = (float)(rc[a] * rc[a]);
  }
}

/* Neighbours of particle i (ascending j): every j != i with r2_f32 < cs2[t_i][t_j].
 * Returns the count; writes at most cap indices to out. */
long long oracle_neighbors_of(int n, const float *pos, const int *type, const double *box, int ntypes,
                              const float *cs2, int i, int *out, long long cap) {
  float L[3], invL[3];
  box_f32(box, L, invL);
  long long cnt = 0;
  for (int j = 0; j < n; ++j) {
    if (j == i) continue;
    float r2 = r2_f32(pos + 3 * i, pos + 3 * j, L, invL);
    if (r2 < cs2[type[i] * ntypes + type[j]]) {
      if (cnt < cap) out[cnt] = j;
      ++cnt;
    }
  }
  return cnt;
}

/* Full pair set, lexicographically sorted (i ascending, then j ascending).
 * pairs has room for 2*cap ints; returns the total count (may exceed cap). */
long long oracle_pair_set(int n, const float *pos, const int *type, const double *box, int ntypes,
                          const float *cs2, int *pairs, long long cap) {
  long long *counts = (long long *)malloc(sizeof(long long) * (size_t)(n + 1));
  if (!counts) return -1;
#pragma omp parallel for schedule(dynamic, 16)
  for (int i = 0; i < n; ++i) counts[i] = oracle_neighbors_of(n, pos, type, box, ntypes, cs2, i, NULL, 0);
  long long total = 0;
  for (int i = 0; i < n; ++i) {
    long long c = counts[i];
    counts[i] = total;
    total += c;
  }
  counts[n] = total;
  if (total <= cap) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int i = 0; i < n; ++i) {
      long long c = counts[i + 1] - counts[i];
      int *tmp = (int *)malloc(sizeof(int) * (size_t)(c > 0 ? c : 1));
      oracle_neighbors_of(n, pos, type, box, ntypes, cs2, i, tmp, c);
      for (long long k = 0; k < c; ++k) {
        pairs[2 * (counts[i] + k)] = i;
        pairs[2 * (counts[i] + k) + 1] = tmp[k];
      }
      free(tmp);
    }
  }
  free(counts);
  return total;
}

/* ---- Lennard-Jones pair function ------------------------------------------ */
/* U(r) = 4 eps [(sig/r)^12 - (sig/r)^6];  F(r) = -dU/dr = 24 eps [2 (sig/r)^12 - (sig/r)^6] / r */
static void lj_uf(double r, double sig, double eps, double *u, double *f) {
  double sr = sig / r;
  double sr6 = sr * sr * sr * sr * sr * sr;
  double sr12 = sr6 * sr6;
  *u = 4.0 * eps * (sr12 - sr6);
  *f = 24.0 * eps * (2.0 * sr12 - sr6) / r;
}

/* pair energy and radial force magnitude (positive = repulsive) for a cutoff method */
void oracle_pair(double r, double sig, double eps, double rc, int method, double *u, double *f) {
  double ur, fr;
  lj_uf(r, sig, eps, &ur, &fr);
  if (method == ORACLE_TRUNC) {
    *u = ur;
    *f = fr;
    return;
  }
  double uc, fc;
  lj_uf(rc, sig, eps, &uc, &fc);
  if (method == ORACLE_SP) {
    *u = ur - uc;
    *f = fr;
  } else { /* shifted force: U(r) - U(rc) + (r - rc) F(rc);  force F(r) - F(rc) */
    *u = ur - uc + (r - rc) * fc;
    *f = fr - fc;
  }
}

/* ---- two-power pair potential ---------------------------------------------- */
/* U(r) = A (sig/r)^m - B (sig/r)^n;  F(r) = -dU/dr = (m A (sig/r)^m - n B (sig/r)^n) / r */
static void mie_uf(double r, double A, double B, int m, int n, double sig, double *u, double *f) {
  double s = sig / r;
  double sm = pow(s, (double)m), sn = pow(s, (double)n);
  *u = A * sm - B * sn;
  *f = ((double)m * A * sm - (double)n * B * sn) / r;
}

/* pair energy and radial force of the two-power potential under a cutoff method */
void oracle_pair_mie(double r, double A, double B, int m, int n, double sig, double rc, int method, double *u,
                     double *f) {
  double ur, fr;
  mie_uf(r, A, B, m, n, sig, &ur, &fr);
  if (method == ORACLE_TRUNC) {
    *u = ur;
    *f = fr;
    return;
  }
  double uc, fc;
  mie_uf(rc, A, B, m, n, sig, &uc, &fc);
  if (method == ORACLE_SP) {
    *u = ur - uc;
    *f = fr;
  } else {
    *u = ur - uc + (r - rc) * fc;
    *f = fr - fc;
  }
}

/* ---- further pair potentials of paper section 2 ------------------------------ */
/* The paper names these potentials only; the forms are the textbook ones:
 *   kind 2, Yukawa (screened Coulomb):  U = eps (sig/r) exp(-kappa (r - sig)),       p = {eps, kappa}
 *   kind 3, Buckingham (exp-6):         U = A exp(-r/rho) - C / r^6,                  p = {A, rho, C}
 *   kind 4, Gaussian core:              U = eps exp(-(r/sig)^2),                      p = {eps}
 *   kind 5, Dzugutov (reduced x = r/sig, scaled by eps):
 *     U = eps [ a1 (x^-16 - b1) exp(c1 / (x - x1)) for x < x1
 *              + b1 exp(d1 / (x - x2))             for x < x2 ],
 *     a1 = 5.82, b1 = 1.28, c1 = 1.1, x1 = 1.87, d1 = 0.27, x2 = 1.94         p = {eps}
 * F(r) = -dU/dr in closed form; kind 1 is the two-power potential above. */
static const double DZ_A = 5.82, DZ_B = 1.28, DZ_C = 1.1, DZ_X1 = 1.87, DZ_D = 0.27, DZ_X2 = 1.94;
static const int DZ_M = 16;

static void gen_uf(int kind, const double *p, double sig, double r, double *u, double *f) {
  if (kind == 2) {
    double e = exp(-p[1] * (r - sig));
    *u = p[0] * sig / r * e;
    *f = p[0] * sig * e * (1.0 + p[1] * r) / (r * r);
  } else if (kind == 3) {
    double e = exp(-r / p[1]);
    double r6 = r * r * r * r * r * r;
    *u = p[0] * e - p[2] / r6;
    *f = p[0] / p[1] * e - 6.0 * p[2] / (r6 * r);
  } else if (kind == 4) {
    double e = exp(-(r / sig) * (r / sig));
    *u = p[0] * e;
    *f = 2.0 * p[0] * r / (sig * sig) * e;
  } else { /* Dzugutov */
    double x = r / sig, du = 0.0, uu = 0.0;
    if (x < DZ_X1) {
      double e = exp(DZ_C / (x - DZ_X1)), xm = pow(x, -(double)DZ_M);
      uu += DZ_A * (xm - DZ_B) * e;
      du += DZ_A * e * (-(double)DZ_M * xm / x - (xm - DZ_B) * DZ_C / ((x - DZ_X1) * (x - DZ_X1)));
    }
    if (x < DZ_X2) {
      double e = exp(DZ_D / (x - DZ_X2));
      uu += DZ_B * e;
      du += -DZ_B * e * DZ_D / ((x - DZ_X2) * (x - DZ_X2));
    }
    *u = p[0] * uu;
    *f = -p[0] * du / sig;
  }
}

/* Girifalco (kind 6; the sphere-sphere form, s = r/sig with sig the sphere
 * diameter d, p = {alpha, beta}):
 *   U = -alpha [1/(s(s-1)^3) + 1/(s(s+1)^3) - 2/s^4] + beta [1/(s(s-1)^9) + 1/(s(s+1)^9) - 2/s^10]. */
static void girifalco_uf(const double *p, double sig, double r, double *u, double *f) {
  double s = r / sig, a = s - 1.0, b = s + 1.0;
  double a3 = a * a * a, b3 = b * b * b, a9 = a3 * a3 * a3, b9 = b3 * b3 * b3;
  double s4 = s * s * s * s, s10 = s4 * s4 * s * s;
  double att = 1.0 / (s * a3) + 1.0 / (s * b3) - 2.0 / s4;
  double rep = 1.0 / (s * a9) + 1.0 / (s * b9) - 2.0 / s10;
  /* d/ds of each bracket */
  double datt = -(1.0 / (s * s * a3) + 3.0 / (s * a3 * a)) - (1.0 / (s * s * b3) + 3.0 / (s * b3 * b)) + 8.0 / (s4 * s);
  double drep = -(1.0 / (s * s * a9) + 9.0 / (s * a9 * a)) - (1.0 / (s * s * b9) + 9.0 / (s * b9 * b)) + 20.0 / (s10 * s);
  *u = -p[0] * att + p[1] * rep;
  *f = -(-p[0] * datt + p[1] * drep) / sig;
}

/* pair energy and radial force of the further potentials (kind 2..6) under a cutoff method */
static void further_uf(int kind, const double *p, double sig, double r, double *u, double *f) {
  if (kind == 6)
    girifalco_uf(p, sig, r, u, f);
  else
    gen_uf(kind, p, sig, r, u, f);
}

void oracle_pair_further(double r, int kind, const double *p, double sig, double rc, int method, double *u, double *f) {
  double ur, fr;
  further_uf(kind, p, sig, r, &ur, &fr);
  if (method == ORACLE_TRUNC) {
    *u = ur;
    *f = fr;
    return;
  }
  double uc, fc;
  further_uf(kind, p, sig, rc, &uc, &fc);
  if (method == ORACLE_SP) {
    *u = ur - uc;
    *f = fr;
  } else {
    *u = ur - uc + (r - rc) * fc;
    *f = fr - fc;
  }
}

/* One pair's short-range term: Lennard-Jones, or, when pot is given, the potential
 * of kind pot[0] (1 the two-power potential, 2..6 the further potentials above) with
 * the parameters of type pair ab at pot[1 + 4 ab .. 4 + 4 ab] (two-power: A, B, m, n). */
static void short_pair(const double *pot, int ab, double r, const double *sigma, const double *eps, const double *rc,
                       int method, double *u, double *f) {
  if (!pot) {
    oracle_pair(r, sigma[ab], eps[ab], rc[ab], method, u, f);
    return;
  }
  const int kind = (int)pot[0];
  const double *q = pot + 1 + 4 * ab;
  if (kind == 1)
    oracle_pair_mie(r, q[0], q[1], (int)q[2], (int)q[3], sigma[ab], rc[ab], method, u, f);
  else
    oracle_pair_further(r, kind, q, sigma[ab], rc[ab], method, u, f);
}

/* ---- Coulomb with a shifted-force cutoff (paper section 9) ---------------- */
/* The plain Coulomb pair force qq / r^2 with its value at r_cc subtracted, and
 * the potential that integrates it back from r_cc (zero at r_cc):
 *   F(r) = qq (1/r^2 - 1/r_cc^2),  U(r) = qq (1/r - 1/r_cc + (r - r_cc)/r_cc^2). */
void oracle_coulomb_sf(double r, double qq, double rcc, double *u, double *f) {
  *u = qq * (1.0 / r - 1.0 / rcc + (r - rcc) / (rcc * rcc));
  *f = qq * (1.0 / (r * r) - 1.0 / (rcc * rcc));
}

/* Forces, per-particle energy and per-particle virial on float32 positions.
 *  sel == NULL: every particle; else the nsel particles listed in sel.
 *  Outputs (length nsel or n): F[3*k..], pe[k] = 1/2 sum_j u_ij,
 *  w[k] = 1/2 * 1/3 sum_j (r_i - r_j) . F_ij.   Totals (over the selection):
 *  totals[0] = sum pe, totals[1] = sum w.  In/out decision: r2_f32 < rc2_f32.
 *  pot: NULL for Lennard-Jones, else the potential block of short_pair. */
void oracle_forces_f32_g(int n, const float *pos, const int *type, const double *box, int ntypes,
                         const double *sigma, const double *eps, const double *rc, int method, const double *pot,
                         const double *charge, double rcc, int nsel, const int *sel, double *F, double *pe,
                         double *w, double *totals) {
  float L32[3], invL[3];
  box_f32(box, L32, invL);
  double L[3] = {(double)L32[0], (double)L32[1], (double)L32[2]};
  float *rc2 = (float *)malloc(sizeof(float) * (size_t)(ntypes * ntypes));
  for (int a = 0; a < ntypes * ntypes; ++a) rc2[a] = (float)(rc[a] * rc[a]);
  const float rcc2 = charge ? (float)(rcc * rcc) : 0.0f;
  int cnt = sel ? nsel : n;
#pragma omp parallel for schedule(dynamic, 8)
  for (int k = 0; k < cnt; ++k) {
    int i = sel ? sel[k] : k;
    nsum_t fx = {0, 0}, fy = {0, 0}, fz = {0, 0}, su = {0, 0}, sw = {0, 0};
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      int ab = type[i] * ntypes + type[j];
      const float r2s = r2_f32(pos + 3 * i, pos + 3 * j, L32, invL);
      const int in_lj = r2s < rc2[ab], in_c = charge && r2s < rcc2;
      if (!in_lj && !in_c) continue;
      double d[3];
      for (int c = 0; c < 3; ++c) {
        d[c] = (double)pos[3 * i + c] - (double)pos[3 * j + c]; /* r_i - r_j */
        d[c] -= L[c] * rint(d[c] / L[c]);
      }
      double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      double u = 0.0, f = 0.0;
      if (in_lj) short_pair(pot, ab, r, sigma, eps, rc, method, &u, &f);
      if (in_c) {
        double uc, fc;
        oracle_coulomb_sf(r, charge[type[i]] * charge[type[j]], rcc, &uc, &fc);
        u += uc;
        f += fc;
      }
      nsum_add(&fx, f * d[0] / r);
      nsum_add(&fy, f * d[1] / r);
      nsum_add(&fz, f * d[2] / r);
      nsum_add(&su, 0.5 * u);
      nsum_add(&sw, 0.5 * r * f / 3.0);
    }
    F[3 * k] = nsum_value(&fx);
    F[3 * k + 1] = nsum_value(&fy);
    F[3 * k + 2] = nsum_value(&fz);
    pe[k] = nsum_value(&su);
    w[k] = nsum_value(&sw);
  }
  nsum_t tu = {0, 0}, tw = {0, 0};
  for (int k = 0; k < cnt; ++k) {
    nsum_add(&tu, pe[k]);
    nsum_add(&tw, w[k]);
  }
  totals[0] = nsum_value(&tu);
  totals[1] = nsum_value(&tw);
  free(rc2);
}

/* Lennard-Jones with the optional Coulomb term. */
void oracle_forces_f32_q(int n, const float *pos, const int *type, const double *box, int ntypes,
                         const double *sigma, const double *eps, const double *rc, int method,
                         const double *charge, double rcc, int nsel, const int *sel, double *F, double *pe,
                         double *w, double *totals) {
  oracle_forces_f32_g(n, pos, type, box, ntypes, sigma, eps, rc, method, NULL, charge, rcc, nsel, sel, F, pe, w,
                      totals);
}

/* The Lennard-Jones-only form (no charges). */
void oracle_forces_f32(int n, const float *pos, const int *type, const double *box, int ntypes,
                       const double *sigma, const double *eps, const double *rc, int method, int nsel,
                       const int *sel, double *F, double *pe, double *w, double *totals) {
  oracle_forces_f32_g(n, pos, type, box, ntypes, sigma, eps, rc, method, NULL, NULL, 0.0, nsel, sel, F, pe, w,
                      totals);
}

/* Forces on double-precision positions, in/out decision r^2 < rc^2 in FP64
 * (and r^2 < r_cc^2 for the Coulomb term when charge != NULL).
 * Used by the reference integrator. */
void oracle_forces_f64_g(int n, const double *pos, const int *type, const double *box, int ntypes,
                         const double *sigma, const double *eps, const double *rc, int method, const double *pot,
                         const double *charge, double rcc, double *F, double *pe, double *w, double *totals) {
#pragma omp parallel for schedule(dynamic, 8)
  for (int i = 0; i < n; ++i) {
    nsum_t fx = {0, 0}, fy = {0, 0}, fz = {0, 0}, su = {0, 0}, sw = {0, 0};
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      int ab = type[i] * ntypes + type[j];
      double d[3];
      for (int c = 0; c < 3; ++c) {
        d[c] = pos[3 * i + c] - pos[3 * j + c];
        d[c] -= box[c] * rint(d[c] / box[c]);
      }
      double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      const int in_lj = r2 < rc[ab] * rc[ab], in_c = charge && r2 < rcc * rcc;
      if (!in_lj && !in_c) continue;
      double r = sqrt(r2);
      double u = 0.0, f = 0.0;
      if (in_lj) short_pair(pot, ab, r, sigma, eps, rc, method, &u, &f);
      if (in_c) {
        double uc, fc;
        oracle_coulomb_sf(r, charge[type[i]] * charge[type[j]], rcc, &uc, &fc);
        u += uc;
        f += fc;
      }
      nsum_add(&fx, f * d[0] / r);
      nsum_add(&fy, f * d[1] / r);
      nsum_add(&fz, f * d[2] / r);
      nsum_add(&su, 0.5 * u);
      nsum_add(&sw, 0.5 * r * f / 3.0);
    }
    F[3 * i] = nsum_value(&fx);
    F[3 * i + 1] = nsum_value(&fy);
    F[3 * i + 2] = nsum_value(&fz);
    pe[i] = nsum_value(&su);
    w[i] = nsum_value(&sw);
  }
  nsum_t tu = {0, 0}, tw = {0, 0};
  for (int i = 0; i < n; ++i) {
    nsum_add(&tu, pe[i]);
    nsum_add(&tw, w[i]);
  }
  totals[0] = nsum_value(&tu);
  totals[1] = nsum_value(&tw);
}

void oracle_forces_f64_q(int n, const double *pos, const int *type, const double *box, int ntypes,
                         const double *sigma, const double *eps, const double *rc, int method,
                         const double *charge, double rcc, double *F, double *pe, double *w, double *totals) {
  oracle_forces_f64_g(n, pos, type, box, ntypes, sigma, eps, rc, method, NULL, charge, rcc, F, pe, w, totals);
}

void oracle_forces_f64(int n, const double *pos, const int *type, const double *box, int ntypes,
                       const double *sigma, const double *eps, const double *rc, int method, double *F,
                       double *pe, double *w, double *totals) {
  oracle_forces_f64_g(n, pos, type, box, ntypes, sigma, eps, rc, method, NULL, NULL, 0.0, F, pe, w, totals);
}

/* Kinetic energy 1/2 sum m v^2 (compensated). */
double oracle_kinetic(int n, const double *vel, const int *type, const double *mass) {
  nsum_t s = {0, 0};
  for (int i = 0; i < n; ++i) {
    double m = mass[type[i]];
    nsum_add(&s, 0.5 * m * (vel[3 * i] * vel[3 * i] + vel[3 * i + 1] * vel[3 * i + 1] + vel[3 * i + 2] * vel[3 * i + 2]));
  }
  return nsum_value(&s);
}

/* Largest squared minimum-image displacement since the last build, in FP64 from
 * float32 positions: d = (double)x - (double)x0, d -= L rint(d / L),
 * d2 = (dx*dx + dy*dy) + dz*dz.  The rebuild fires when this exceeds (s/2)^2. */
double oracle_max_disp2(int n, const float *pos, const float *pos0, const double *box) {
  float L32[3], invL[3];
  box_f32(box, L32, invL);
  double best = 0.0;
  for (int i = 0; i < n; ++i) {
    double d[3];
    for (int c = 0; c < 3; ++c) {
      double L = (double)L32[c];
      d[c] = (double)pos[3 * i + c] - (double)pos0[3 * i + c];
      d[c] -= L * rint(d[c] / L);
    }
    double d2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
    if (d2 > best) best = d2;
  }
  return best;
}

int oracle_rebuild_needed(int n, const float *pos, const float *pos0, const double *box, double skin) {
  double h = 0.5 * skin;
  return oracle_max_disp2(n, pos, pos0, box) > h * h;
}

/*
 * Leapfrog with a Nose-Hoover thermostat, FP64 state.  With thermostat == 0 the
 * friction xi stays zero and the scheme is plain leapfrog (NVE).
 *   v^{n+1/2} = [ v^{n-1/2} (1 - xi^n dt/2) + (F^n / m) dt ] / (1 + xi^n dt/2)
 *   r^{n+1}   = r^n + v^{n+1/2} dt            (then wrapped into [-L/2, L/2))
 *   T^{n+1/2} = 2 KE(v^{n+1/2}) / g,          g = 3N - 3
 *   xi^{n+1}  = xi^n + dt (T^{n+1/2} / T0 - 1) / tau^2
 *   I^{n+1}   = I^n + dt (xi^n + xi^{n+1}) / 2   (integral of xi)
 * Thermo of step n (row n of thermo, 9 doubles):
 *   PE(r^n), KE(v^n) with v^n = (v^{n-1/2} + v^{n+1/2}) / 2, W(r^n), T^n = 2 KE / g,
 *   P^n = (2 KE / 3 + W) / V, xi^n, I^n, H^n = KE + PE + g T0 (tau^2 xi^2 / 2 + I), KE(v^{n+1/2}).
 * inv_tau2 = 1/tau^2 (0 means no coupling).  image counts crossings of the box.
 */
int oracle_integrate_g(int n, double *pos, double *vel, int *image, const int *type, const double *mass,
                       const double *box, int ntypes, const double *sigma, const double *eps, const double *rc,
                       int method, const double *pot, const double *charge, double rcc, double dt, int thermostat,
                       double T0, double inv_tau2, double *xi, double *xi_int, int nsteps, double *thermo) {
  double *F = (double *)malloc(sizeof(double) * 3 * (size_t)n);
  double *pe = (double *)malloc(sizeof(double) * (size_t)n);
  double *w = (double *)malloc(sizeof(double) * (size_t)n);
  double *vnew = (double *)malloc(sizeof(double) * 3 * (size_t)n);
  double *vmid = (double *)malloc(sizeof(double) * 3 * (size_t)n);
  if (!F || !pe || !w || !vnew || !vmid) return -1;
  double g = 3.0 * n - 3.0;
  double V = box[0] * box[1] * box[2];
  for (int step = 0; step < nsteps; ++step) {
    double tot[2];
    oracle_forces_f64_g(n, pos, type, box, ntypes, sigma, eps, rc, method, pot, charge, rcc, F, pe, w, tot);
    double x = thermostat ? *xi : 0.0;
    double a = 1.0 - x * dt / 2.0, b = 1.0 + x * dt / 2.0;
    for (int i = 0; i < n; ++i) {
      double m = mass[type[i]];
      for (int c = 0; c < 3; ++c) {
        vnew[3 * i + c] = (vel[3 * i + c] * a + F[3 * i + c] / m * dt) / b;
        vmid[3 * i + c] = 0.5 * (vel[3 * i + c] + vnew[3 * i + c]);
      }
    }
    double ke_half = oracle_kinetic(n, vnew, type, mass);
    double ke_int = oracle_kinetic(n, vmid, type, mass);
    if (thermo) {
      double *row = thermo + 9 * (size_t)step;
      double T = 2.0 * ke_int / g;
      row[0] = tot[0];
      row[1] = ke_int;
      row[2] = tot[1];
      row[3] = T;
      row[4] = (2.0 * ke_int / 3.0 + tot[1]) / V;
      row[5] = x;
      row[6] = *xi_int;
      row[7] = ke_int + tot[0];
      if (thermostat && inv_tau2 > 0.0) row[7] += g * T0 * (x * x / (2.0 * inv_tau2) + *xi_int);
      row[8] = ke_half;
    }
    for (int i = 0; i < n; ++i) {
      for (int c = 0; c < 3; ++c) {
        vel[3 * i + c] = vnew[3 * i + c];
        double p = pos[3 * i + c] + vnew[3 * i + c] * dt;
        double h = box[c] / 2.0;
        if (p >= h) {
          p -= box[c];
          image[3 * i + c] += 1;
        } else if (p < -h) {
          p += box[c];
          image[3 * i + c] -= 1;
        }
        pos[3 * i + c] = p;
      }
    }
    if (thermostat) {
      double Th = 2.0 * ke_half / g;
      double xn = x + dt * (Th / T0 - 1.0) * inv_tau2;
      *xi_int += dt * (x + xn) / 2.0;
      *xi = xn;
    }
  }
  free(F);
  free(pe);
  free(w);
  free(vnew);
  free(vmid);
  return 0;
}

int oracle_integrate_q(int n, double *pos, double *vel, int *image, const int *type, const double *mass,
                       const double *box, int ntypes, const double *sigma, const double *eps, const double *rc,
                       int method, const double *charge, double rcc, double dt, int thermostat, double T0,
                       double inv_tau2, double *xi, double *xi_int, int nsteps, double *thermo) {
  return oracle_integrate_g(n, pos, vel, image, type, mass, box, ntypes, sigma, eps, rc, method, NULL, charge, rcc,
                            dt, thermostat, T0, inv_tau2, xi, xi_int, nsteps, thermo);
}

/* The Lennard-Jones-only form (no charges). */
int oracle_integrate(int n, double *pos, double *vel, int *image, const int *type, const double *mass,
                     const double *box, int ntypes, const double *sigma, const double *eps, const double *rc,
                     int method, double dt, int thermostat, double T0, double inv_tau2, double *xi,
                     double *xi_int, int nsteps, double *thermo) {
  return oracle_integrate_g(n, pos, vel, image, type, mass, box, ntypes, sigma, eps, rc, method, NULL, NULL, 0.0,
                            dt, thermostat, T0, inv_tau2, xi, xi_int, nsteps, thermo);
}
