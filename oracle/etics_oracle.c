/*
 * etics_oracle.c -- plain FP64 CPU oracle for the expansion force calculation
 * of Meiron, Li, Holley-Bockelmann & Spurzem, "Expansion Techniques for
 * Collisionless Stellar Dynamical Simulations" (arXiv:1406.4254).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into oracle/liboracle.so,
 * which only the test suite, the smoke check and the benchmark's CPU-baseline
 * leg load.  The GPU library never links, includes or calls it, and it shares
 * no code with the GPU library: every table, recurrence and normalisation here
 * is written out separately, in FP64, in the order the method defines it.
 *
 * Conventions (G = M_total-free, a = 1, expansion centre at the origin):
 *   xi = (r-1)/(r+1);  alpha_l = 2l + 3/2
 *   PhiT_nl(r) = -sqrt(4 pi) r^l / (1+r)^(2l+1) C_n^(alpha_l)(xi)
 *   rhoT_nl(r) = K_nl/(2 pi) sqrt(4 pi) r^(l-1) / (1+r)^(2l+3) C_n^(alpha_l)(xi)
 *   K_nl = n(n+4l+3)/2 + (l+1)(2l+1)
 *   Atilde_nl = 1 / I_nl,  I_nl = int rhoT_nl PhiT_nl r^2 dr
 *   Ybar_lm  = orthonormal real-form spherical harmonic amplitude (Condon-Shortley)
 *   A_nlm = (2 - delta_m0) Atilde_nl sum_k m_k PhiT_nl(r_k) Ybar_lm(theta_k) cos(m phi_k)
 *   B_nlm = same with sin(m phi_k)
 *   Phi(x) = sum_{n,l,m>=0} PhiT_nl(r) Ybar_lm(theta) [A_nlm cos m phi + B_nlm sin m phi]
 * Coefficient arrays use idx(n,l,m) = n (lmax+1)(lmax+2)/2 + l(l+1)/2 + m.
 *
 * The SCF expansion is the paper's Section 2.4 (eq. scf-phi) with the
 * Hernquist-Ostriker basis the paper adopts (Section 2.5); the serial loop order
 * (particle loop outermost, special functions then the n-l-m accumulation) is the
 * one the paper describes for the serial code in Section 3.3.  MEX is eqs.
 * mex-phi, mex-qlm, mex-plm of Section 2.4 with the exclusive sorted sweeps of
 * Section 3.2.
 *
 * A second radial basis, the Clutton-Brock one that Section 2.5 describes as the
 * alternative for cored (Plummer-like) systems, is selected by basis = 1:
 *   xi = (r^2-1)/(r^2+1);  alpha_l = l + 1
 *   PhiT_nl(r) = -sqrt(4 pi) r^l / (1+r^2)^(l+1/2) C_n^(alpha_l)(xi)
 *   rhoT_nl(r) = K_nl/(4 pi) sqrt(4 pi) r^l / (1+r^2)^(l+5/2) C_n^(alpha_l)(xi)
 *   K_nl = 4n(n+2l+2) + (2l+1)(2l+3)
 *   I_nl = int rhoT_nl PhiT_nl r^2 dr = -K_nl pi 2^(-4l-4) Gamma(n+2l+2) / (n! (n+l+1) (l!)^2)
 * with the same normalisation conventions as above (basis 0 = Hernquist-Ostriker).
 *
 * Self-interaction: SCF coefficients include every particle (a field method);
 * MEX excludes the particle itself (strict inequalities of eqs. mex-qlm/plm).
 * At r = 0 the l = 0 SCF radial force has no direction; it is taken as 0.
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif
#define FOUR_PI (4.0 * M_PI)
/* Type of every running sum over particles or over expansion terms.  The oracle is
   built with plain double; a second build with long double measures how much of the
   oracle's own result is rounding of its sequential sums (each term is still formed
   in double, so only the additions differ). */
#ifndef ORACLE_ACC
#define ORACLE_ACC double
#endif
typedef ORACLE_ACC acc_t;
/* fixed particle chunking for the coefficient sums: the result does not depend on
   the number of threads that happen to run the chunks */
#define ORACLE_NCHUNK 64

static inline int lm_index(int l, int m) { return l * (l + 1) / 2 + m; }

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ---------------------------------------------------------------- Gegenbauer */
/* C_0..C_nmax of C_n^(alpha)(x) by the three-term recurrence
   n C_n = 2 (n + alpha - 1) x C_{n-1} - (n + 2 alpha - 2) C_{n-2}.               */
void oracle_gegenbauer(int nmax, double alpha, double x, double *c) {
  if (nmax < 0) return;
  c[0] = 1.0;
  if (nmax >= 1) c[1] = 2.0 * alpha * x;
  for (int n = 2; n <= nmax; ++n)
    c[n] = (2.0 * (n + alpha - 1.0) * x * c[n - 1] - (n + 2.0 * alpha - 2.0) * c[n - 2]) / n;
}

/* ----------------------------------------------------------------- Legendre */
/* Unnormalised associated Legendre P_l^m(x), Condon-Shortley phase, 0<=m<=l<=lmax:
   P_m^m = (-1)^m (2m-1)!! s^m,  P_{m+1}^m = (2m+1) x P_m^m,
   (l-m) P_l^m = (2l-1) x P_{l-1}^m - (l+m-1) P_{l-2}^m.   s = sin(theta) >= 0.  */
static void plm_unnorm(int lmax, double x, double s, double *P) {
  double pmm = 1.0;
  for (int m = 0; m <= lmax; ++m) {
    if (m > 0) pmm *= -(2.0 * m - 1.0) * s;
    P[lm_index(m, m)] = pmm;
    if (m + 1 <= lmax) P[lm_index(m + 1, m)] = (2.0 * m + 1.0) * x * pmm;
    for (int l = m + 2; l <= lmax; ++l)
      P[lm_index(l, m)] = ((2.0 * l - 1.0) * x * P[lm_index(l - 1, m)] -
                           (l + m - 1.0) * P[lm_index(l - 2, m)]) / (double)(l - m);
  }
}

/* normalisation N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) */
static double ylm_norm(int l, int m) {
  return sqrt((2.0 * l + 1.0) / FOUR_PI * exp(lgamma(l - m + 1.0) - lgamma(l + m + 1.0)));
}

/* Ybar_lm(theta) = N_lm P_l^m(cos theta) for 0<=m<=l<=lmax, index l(l+1)/2+m */
void oracle_ylm(int lmax, double costh, double sinth, double *Y) {
  plm_unnorm(lmax, costh, sinth, Y);
  for (int l = 0; l <= lmax; ++l)
    for (int m = 0; m <= l; ++m) Y[lm_index(l, m)] *= ylm_norm(l, m);
}

/* Ybar, dYbar/dtheta and m Ybar / sin(theta), from division-free ladder identities
   of the unnormalised functions:
     dP_l^m/dtheta = (P_l^{m+1} - (l+m)(l-m+1) P_l^{m-1}) / 2   (m >= 1),
     dP_l^0/dtheta = P_l^1,
     m P_l^m / sin(theta) = -(P_{l+1}^{m+1} + (l-m+1)(l-m+2) P_{l+1}^{m-1}) / 2.      */
void oracle_ylm_deriv(int lmax, double costh, double sinth, double *Y, double *dY,
                      double *mYs) {
  int L1 = lmax + 1;
  double *P = (double *)malloc(sizeof(double) * (size_t)((L1 + 1) * (L1 + 2) / 2));
  plm_unnorm(L1, costh, sinth, P);
  for (int l = 0; l <= lmax; ++l) {
    for (int m = 0; m <= l; ++m) {
      double N = ylm_norm(l, m);
      double plm = P[lm_index(l, m)];
      double pup = (m + 1 <= l) ? P[lm_index(l, m + 1)] : 0.0;
      double d;
      if (m == 0) d = pup;
      else d = 0.5 * (pup - (double)(l + m) * (l - m + 1) * P[lm_index(l, m - 1)]);
      double ms = 0.0;
      if (m >= 1)
        ms = -0.5 * (P[lm_index(l + 1, m + 1)] +
                     (double)(l - m + 1) * (l - m + 2) * P[lm_index(l + 1, m - 1)]);
      Y[lm_index(l, m)] = N * plm;
      if (dY) dY[lm_index(l, m)] = N * d;
      if (mYs) mYs[lm_index(l, m)] = N * ms;
    }
  }
  free(P);
}

/* ------------------------------------------------------------- radial basis */
double oracle_knl(int n, int l) { return 0.5 * n * (n + 4.0 * l + 3.0) + (l + 1.0) * (2.0 * l + 1.0); }

/* I_nl = -(4 pi K_nl / 2^(8l+6)) Gamma(n+4l+3) / (n! (n+2l+3/2) Gamma(2l+3/2)^2);  Atilde = 1/I */
double oracle_anl_tilde(int n, int l) {
  double logI = log(FOUR_PI * oracle_knl(n, l)) - (8.0 * l + 6.0) * log(2.0) +
                lgamma(n + 4.0 * l + 3.0) - lgamma(n + 1.0) - log(n + 2.0 * l + 1.5) -
                2.0 * lgamma(2.0 * l + 1.5);
  return -exp(-logI);
}

/* Clutton-Brock basis: K_nl = 4n(n+2l+2) + (2l+1)(2l+3) */
double oracle_knl_cb(int n, int l) { return 4.0 * n * (n + 2.0 * l + 2.0) + (2.0 * l + 1.0) * (2.0 * l + 3.0); }

/* I_nl = -K_nl pi 2^(-4l-4) Gamma(n+2l+2) / (n! (n+l+1) (l!)^2);  Atilde = 1/I */
double oracle_anl_tilde_cb(int n, int l) {
  double logI = log(M_PI * oracle_knl_cb(n, l)) - (4.0 * l + 4.0) * log(2.0) + lgamma(n + 2.0 * l + 2.0) -
                lgamma(n + 1.0) - log(n + l + 1.0) - 2.0 * lgamma(l + 1.0);
  return -exp(-logI);
}

double oracle_anl_tilde_basis(int basis, int n, int l) {
  return basis == 1 ? oracle_anl_tilde_cb(n, l) : oracle_anl_tilde(n, l);
}

/* PhiT_nl(r), dPhiT_nl/dr and (l >= 1) PhiT_nl(r)/r of either basis, arrays
   [(nmax+1)*(lmax+1)] indexed n*(lmax+1)+l (any of the three may be NULL).  With
   f(r) the r-dependent prefactor and xi(r) the Gegenbauer argument:
     HO: f = r^l (1+r)^-(2l+1),   xi = (r-1)/(r+1),      dxi/dr = 2/(1+r)^2,
         f' = l r^(l-1) (1+r)^-(2l+1) - (2l+1) r^l (1+r)^-(2l+2);
     CB: f = r^l (1+r^2)^-(l+1/2), xi = (r^2-1)/(r^2+1), dxi/dr = 4r/(1+r^2)^2,
         f' = l r^(l-1) (1+r^2)^-(l+1/2) - (2l+1) r^(l+1) (1+r^2)^-(l+3/2);
   dPhiT = -sqrt(4 pi) (f' C_n + f dC_n/dxi dxi/dr),  dC_n^a/dxi = 2a C_{n-1}^(a+1).
   PhiT/r uses r^(l-1) directly, so it is finite at r = 0 for l >= 1 (0 for l = 0). */
static void radial_basis(int basis, int nmax, int lmax, double r, double *phi, double *dphi,
                         double *phir) {
  double xi = basis == 1 ? (r * r - 1.0) / (r * r + 1.0) : (r - 1.0) / (r + 1.0);
  double *c = (double *)malloc(sizeof(double) * (size_t)(nmax + 1));
  double *c1 = (double *)malloc(sizeof(double) * (size_t)(nmax + 1));
  double s4pi = sqrt(FOUR_PI);
  for (int l = 0; l <= lmax; ++l) {
    double alpha = basis == 1 ? l + 1.0 : 2.0 * l + 1.5;
    oracle_gegenbauer(nmax, alpha, xi, c);
    oracle_gegenbauer(nmax, alpha + 1.0, xi, c1);
    double f, fp, dxi, fr;
    if (basis == 1) {
      double q = 1.0 + r * r;
      f = pow(r, l) / pow(q, l + 0.5);
      fp = (l > 0 ? l * pow(r, l - 1) / pow(q, l + 0.5) : 0.0) - (2.0 * l + 1.0) * pow(r, l + 1) / pow(q, l + 1.5);
      dxi = 4.0 * r / (q * q);
      fr = (l >= 1) ? -s4pi * pow(r, l - 1.0) / pow(q, l + 0.5) : 0.0;
    } else {
      f = pow(r, l) / pow(1.0 + r, 2.0 * l + 1.0);
      fp = (l > 0 ? l * pow(r, l - 1) / pow(1.0 + r, 2.0 * l + 1.0) : 0.0) -
           (2.0 * l + 1.0) * pow(r, l) / pow(1.0 + r, 2.0 * l + 2.0);
      dxi = 2.0 / ((1.0 + r) * (1.0 + r));
      fr = (l >= 1) ? -s4pi * pow(r, l - 1.0) / pow(1.0 + r, 2.0 * l + 1.0) : 0.0;
    }
    for (int n = 0; n <= nmax; ++n) {
      double dc = (n >= 1) ? 2.0 * alpha * c1[n - 1] : 0.0;
      if (phi) phi[n * (lmax + 1) + l] = -s4pi * f * c[n];
      if (dphi) dphi[n * (lmax + 1) + l] = -s4pi * (fp * c[n] + f * dc * dxi);
      if (phir) phir[n * (lmax + 1) + l] = fr * c[n];
    }
  }
  free(c);
  free(c1);
}

/* PhiT_nl(r) and dPhiT_nl/dr of the Hernquist-Ostriker basis (basis 0) */
void oracle_phi_nl(int nmax, int lmax, double r, double *phi, double *dphi) {
  radial_basis(0, nmax, lmax, r, phi, dphi, NULL);
}

void oracle_phi_nl_basis(int basis, int nmax, int lmax, double r, double *phi, double *dphi) {
  radial_basis(basis, nmax, lmax, r, phi, dphi, NULL);
}

/* rhoT_nl(r), same layout (used only by the Poisson and biorthogonality checks) */
void oracle_rho_nl_basis(int basis, int nmax, int lmax, double r, double *rho) {
  double xi = basis == 1 ? (r * r - 1.0) / (r * r + 1.0) : (r - 1.0) / (r + 1.0);
  double *c = (double *)malloc(sizeof(double) * (size_t)(nmax + 1));
  for (int l = 0; l <= lmax; ++l) {
    oracle_gegenbauer(nmax, basis == 1 ? l + 1.0 : 2.0 * l + 1.5, xi, c);
    for (int n = 0; n <= nmax; ++n) {
      double v;
      if (basis == 1)
        v = oracle_knl_cb(n, l) / FOUR_PI * sqrt(FOUR_PI) * pow(r, (double)l) / pow(1.0 + r * r, l + 2.5);
      else
        v = oracle_knl(n, l) / (2.0 * M_PI) * sqrt(FOUR_PI) * pow(r, l - 1.0) / pow(1.0 + r, 2.0 * l + 3.0);
      rho[n * (lmax + 1) + l] = v * c[n];
    }
  }
  free(c);
}

void oracle_rho_nl(int nmax, int lmax, double r, double *rho) { oracle_rho_nl_basis(0, nmax, lmax, r, rho); }

/* ---------------------------------------------------- spherical coordinates */
typedef struct {
  double r, costh, sinth, cosph, sinph;
} sph_t;

/* r=0 -> theta=0; R=0 -> phi=0 */
static sph_t to_sph(double x, double y, double z) {
  sph_t s;
  double R = sqrt(x * x + y * y);
  s.r = sqrt(x * x + y * y + z * z);
  if (s.r > 0.0) {
    s.costh = z / s.r;
    s.sinth = R / s.r;
  } else {
    s.costh = 1.0;
    s.sinth = 0.0;
  }
  double ph = atan2(y, x);
  s.cosph = cos(ph);
  s.sinph = sin(ph);
  return s;
}

static void to_cart(const sph_t *s, double ar, double at, double ap, double *ax, double *ay,
                    double *az) {
  *ax = s->sinth * s->cosph * ar + s->costh * s->cosph * at - s->sinph * ap;
  *ay = s->sinth * s->sinph * ar + s->costh * s->sinph * at + s->cosph * ap;
  *az = s->costh * ar - s->sinth * at;
}

/* ------------------------------------------------------------ SCF oracle */
int oracle_coeff_count(int nmax, int lmax) { return (nmax + 1) * (lmax + 1) * (lmax + 2) / 2; }

/* Coefficients A, B [K] from particles (x,y,z,m)[n] in radial basis `basis`. */
void oracle_scf_coeffs_basis(int basis, const double *x, const double *y, const double *z,
                             const double *mass, int64_t np, int nmax, int lmax, double *A,
                             double *B) {
  int K = oracle_coeff_count(nmax, lmax);
  int L2 = (lmax + 1) * (lmax + 2) / 2;
  acc_t *SA = (acc_t *)calloc((size_t)ORACLE_NCHUNK * K, sizeof(acc_t));
  acc_t *SB = (acc_t *)calloc((size_t)ORACLE_NCHUNK * K, sizeof(acc_t));
#pragma omp parallel for schedule(dynamic, 1)
  for (int ch = 0; ch < ORACLE_NCHUNK; ++ch) {
    int64_t j0 = np * ch / ORACLE_NCHUNK, j1 = np * (ch + 1) / ORACLE_NCHUNK;
    double *phi = (double *)malloc(sizeof(double) * (size_t)((nmax + 1) * (lmax + 1)));
    double *Y = (double *)malloc(sizeof(double) * (size_t)L2);
    double *cm = (double *)malloc(sizeof(double) * (size_t)(lmax + 1));
    double *sm = (double *)malloc(sizeof(double) * (size_t)(lmax + 1));
    acc_t *sa = SA + (size_t)ch * K, *sb = SB + (size_t)ch * K;
    for (int64_t j = j0; j < j1; ++j) {
      /* (1a) special functions of this particle */
      sph_t s = to_sph(x[j], y[j], z[j]);
      radial_basis(basis, nmax, lmax, s.r, phi, NULL, NULL);
      oracle_ylm(lmax, s.costh, s.sinth, Y);
      double ph = atan2(s.sinph, s.cosph);
      for (int m = 0; m <= lmax; ++m) {
        cm[m] = cos(m * ph);
        sm[m] = sin(m * ph);
      }
      /* (1b) contribution to every coefficient, n-l-m order */
      for (int n = 0; n <= nmax; ++n)
        for (int l = 0; l <= lmax; ++l) {
          double w = mass[j] * phi[n * (lmax + 1) + l];
          for (int m = 0; m <= l; ++m) {
            int k = n * L2 + lm_index(l, m);
            sa[k] += (acc_t)(w * Y[lm_index(l, m)] * cm[m]);
            sb[k] += (acc_t)(w * Y[lm_index(l, m)] * sm[m]);
          }
        }
    }
    free(phi);
    free(Y);
    free(cm);
    free(sm);
  }
  for (int n = 0; n <= nmax; ++n)
    for (int l = 0; l <= lmax; ++l) {
      double at = oracle_anl_tilde_basis(basis, n, l);
      for (int m = 0; m <= l; ++m) {
        int k = n * L2 + lm_index(l, m);
        acc_t sa = 0.0, sb = 0.0;
        for (int ch = 0; ch < ORACLE_NCHUNK; ++ch) {
          sa += SA[(size_t)ch * K + k];
          sb += SB[(size_t)ch * K + k];
        }
        double f = (m == 0 ? 1.0 : 2.0) * at;
        A[k] = (double)(f * sa);
        B[k] = (m == 0) ? 0.0 : (double)(f * sb);
      }
    }
  free(SA);
  free(SB);
}

void oracle_scf_coeffs(const double *x, const double *y, const double *z, const double *mass,
                       int64_t np, int nmax, int lmax, double *A, double *B) {
  oracle_scf_coeffs_basis(0, x, y, z, mass, np, nmax, lmax, A, B);
}

/* Potential and acceleration a = -grad Phi at the points (x,y,z)[n] from
   coefficients A, B of radial basis `basis`.  pot/ax/ay/az may individually be NULL. */
void oracle_scf_force_basis(int basis, const double *x, const double *y, const double *z,
                            int64_t np, int nmax, int lmax, const double *A, const double *B,
                            double *pot, double *ax, double *ay, double *az) {
  int L2 = (lmax + 1) * (lmax + 2) / 2;
#pragma omp parallel
  {
    double *phi = (double *)malloc(sizeof(double) * (size_t)((nmax + 1) * (lmax + 1)));
    double *dphi = (double *)malloc(sizeof(double) * (size_t)((nmax + 1) * (lmax + 1)));
    double *phir = (double *)malloc(sizeof(double) * (size_t)((nmax + 1) * (lmax + 1)));
    double *Y = (double *)malloc(sizeof(double) * (size_t)L2);
    double *dY = (double *)malloc(sizeof(double) * (size_t)L2);
    double *mYs = (double *)malloc(sizeof(double) * (size_t)L2);
#pragma omp for schedule(static)
    for (int64_t i = 0; i < np; ++i) {
      /* (2a) special functions and their derivatives */
      sph_t s = to_sph(x[i], y[i], z[i]);
      double r = s.r;
      radial_basis(basis, nmax, lmax, r, phi, dphi, phir); /* PhiT/r without dividing by r */
      oracle_ylm_deriv(lmax, s.costh, s.sinth, Y, dY, mYs);
      double ph = atan2(s.sinph, s.cosph);
      /* (2b) sums over the coefficients */
      acc_t P = 0.0, ar = 0.0, at = 0.0, ap = 0.0;
      for (int l = 0; l <= lmax; ++l) {
        for (int m = 0; m <= l; ++m) {
          double cm = cos(m * ph), sm = sin(m * ph);
          for (int n = 0; n <= nmax; ++n) {
            int k = n * L2 + lm_index(l, m);
            double e = A[k] * cm + B[k] * sm;    /* d/dphi -> m(-A sin + B cos) */
            double f = -A[k] * sm + B[k] * cm;
            double ph_nl = phi[n * (lmax + 1) + l];
            double dph_nl = dphi[n * (lmax + 1) + l];
            P += (acc_t)(ph_nl * Y[lm_index(l, m)] * e);
            if (!(l == 0 && r == 0.0)) ar -= (acc_t)(dph_nl * Y[lm_index(l, m)] * e);
            if (l >= 1) {
              double por = phir[n * (lmax + 1) + l];
              at -= (acc_t)(por * dY[lm_index(l, m)] * e);
              ap -= (acc_t)(por * mYs[lm_index(l, m)] * f);
            }
          }
        }
      }
      double gx, gy, gz;
      to_cart(&s, (double)ar, (double)at, (double)ap, &gx, &gy, &gz);
      if (pot) pot[i] = (double)P;
      if (ax) ax[i] = gx;
      if (ay) ay[i] = gy;
      if (az) az[i] = gz;
    }
    free(phi);
    free(dphi);
    free(phir);
    free(Y);
    free(dY);
    free(mYs);
  }
}

void oracle_scf_force(const double *x, const double *y, const double *z, int64_t np, int nmax,
                      int lmax, const double *A, const double *B, double *pot, double *ax,
                      double *ay, double *az) {
  oracle_scf_force_basis(0, x, y, z, np, nmax, lmax, A, B, pot, ax, ay, az);
}

/* ------------------------------------------------------------ MEX oracle */
typedef struct {
  double key;
  int64_t idx;
} keyidx_t;

static int cmp_keyidx(const void *a, const void *b) {
  const keyidx_t *p = (const keyidx_t *)a, *q = (const keyidx_t *)b;
  if (p->key < q->key) return -1;
  if (p->key > q->key) return 1;
  return (p->idx < q->idx) ? -1 : (p->idx > q->idx);
}

/* the radius key: ((x*x + y*y) + z*z) in FP64, each product and sum rounded
   separately (this file is compiled with FMA contraction off) */
double oracle_r2_key(double x, double y, double z) {
  volatile double xx = x * x, yy = y * y, zz = z * z;
  volatile double s = xx + yy;
  return s + zz;
}

/* order[n]: particle indices sorted by (key, index) */
void oracle_mex_order(const double *x, const double *y, const double *z, int64_t np,
                      int64_t *order) {
  keyidx_t *ki = (keyidx_t *)malloc(sizeof(keyidx_t) * (size_t)(np > 0 ? np : 1));
  for (int64_t i = 0; i < np; ++i) {
    ki[i].key = oracle_r2_key(x[i], y[i], z[i]);
    ki[i].idx = i;
  }
  qsort(ki, (size_t)np, sizeof(keyidx_t), cmp_keyidx);
  for (int64_t i = 0; i < np; ++i) order[i] = ki[i].idx;
  free(ki);
}

/* Multipole expansion (eqs. mex-phi, mex-qlm, mex-plm), real form:
     q^{c,s}_lm(i) = sum_{j before i} m_j r_j^l Ybar_lm(j) (cos, sin)(m phi_j)
     p^{c,s}_lm(i) = sum_{j after i}  m_j r_j^-(l+1) Ybar_lm(j) (cos, sin)(m phi_j)
     Phi_i = -sum_l 4pi/(2l+1) sum_m (2-delta_m0) Ybar_lm(i)
               [ (q^c r^-(l+1) + p^c r^l) cos m phi_i + (q^s r^-(l+1) + p^s r^l) sin m phi_i ]
   "before/after" is the (key, index) order.  The force is -grad Phi with q and p
   held fixed.  The inward (q) part is done in a forward sweep, the outward (p) part
   in a reverse sweep; each sweep reads the running sums before adding particle i
   (exclusive).  A particle exactly at r = 0 has no inward part, and contributes
   nothing to the outward sums of others. */
void oracle_mex_force(const double *x, const double *y, const double *z, const double *mass,
                      int64_t np, int lmax, double *pot, double *ax, double *ay, double *az) {
  int L2 = (lmax + 1) * (lmax + 2) / 2;
  int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(np > 0 ? np : 1));
  oracle_mex_order(x, y, z, np, order);
  acc_t *P = (acc_t *)calloc((size_t)(np > 0 ? np : 1), sizeof(acc_t));
  acc_t *AR = (acc_t *)calloc((size_t)(np > 0 ? np : 1), sizeof(acc_t));
  acc_t *AT = (acc_t *)calloc((size_t)(np > 0 ? np : 1), sizeof(acc_t));
  acc_t *AP = (acc_t *)calloc((size_t)(np > 0 ? np : 1), sizeof(acc_t));
  double *Y = (double *)malloc(sizeof(double) * (size_t)L2);
  double *dY = (double *)malloc(sizeof(double) * (size_t)L2);
  double *mYs = (double *)malloc(sizeof(double) * (size_t)L2);
  acc_t *sc = (acc_t *)calloc((size_t)L2, sizeof(acc_t));
  acc_t *ss = (acc_t *)calloc((size_t)L2, sizeof(acc_t));
  for (int pass = 0; pass < 2; ++pass) { /* 0: inward sums q (forward); 1: outward p (reverse) */
    memset(sc, 0, sizeof(acc_t) * (size_t)L2);
    memset(ss, 0, sizeof(acc_t) * (size_t)L2);
    for (int64_t k = 0; k < np; ++k) {
      int64_t i = pass == 0 ? order[k] : order[np - 1 - k];
      sph_t s = to_sph(x[i], y[i], z[i]);
      double r = s.r;
      double ph = atan2(s.sinph, s.cosph);
      oracle_ylm_deriv(lmax, s.costh, s.sinth, Y, dY, mYs);
      /* field of the running sums at particle i */
      acc_t Pi = 0.0, ar = 0.0, at = 0.0, ap = 0.0;
      for (int l = 0; l <= lmax; ++l) {
        double g = FOUR_PI / (2.0 * l + 1.0);
        double rad, drad, rado; /* radial factor, its r-derivative, factor / r */
        if (pass == 0) {
          if (r == 0.0) continue;
          rad = pow(r, -(l + 1.0));
          drad = -(l + 1.0) * pow(r, -(l + 2.0));
          rado = pow(r, -(l + 2.0));
        } else {
          rad = pow(r, (double)l);
          drad = (l >= 1) ? l * pow(r, l - 1.0) : 0.0;
          rado = (l >= 1) ? pow(r, l - 1.0) : 0.0;
        }
        for (int m = 0; m <= l; ++m) {
          double w = (m == 0 ? 1.0 : 2.0) * g;
          double cm = cos(m * ph), sm = sin(m * ph);
          acc_t e = sc[lm_index(l, m)] * cm + ss[lm_index(l, m)] * sm;
          acc_t f = -sc[lm_index(l, m)] * sm + ss[lm_index(l, m)] * cm;
          Pi -= w * Y[lm_index(l, m)] * e * rad;
          ar += w * Y[lm_index(l, m)] * e * drad;
          at += w * dY[lm_index(l, m)] * e * rado;
          ap += w * mYs[lm_index(l, m)] * f * rado;
        }
      }
      P[i] += Pi;
      AR[i] += ar;
      AT[i] += at;
      AP[i] += ap;
      /* then add particle i to the running sums */
      if (pass == 1 && r == 0.0) continue;
      for (int l = 0; l <= lmax; ++l) {
        double rp = (pass == 0) ? pow(r, (double)l) : pow(r, -(l + 1.0));
        for (int m = 0; m <= l; ++m) {
          sc[lm_index(l, m)] += (acc_t)(mass[i] * rp * Y[lm_index(l, m)] * cos(m * ph));
          ss[lm_index(l, m)] += (acc_t)(mass[i] * rp * Y[lm_index(l, m)] * sin(m * ph));
        }
      }
    }
  }
  for (int64_t i = 0; i < np; ++i) {
    sph_t s = to_sph(x[i], y[i], z[i]);
    double gx, gy, gz;
    to_cart(&s, (double)AR[i], (double)AT[i], (double)AP[i], &gx, &gy, &gz);
    if (pot) pot[i] = (double)P[i];
    if (ax) ax[i] = gx;
    if (ay) ay[i] = gy;
    if (az) az[i] = gz;
  }
  free(order);
  free(P);
  free(AR);
  free(AT);
  free(AP);
  free(Y);
  free(dY);
  free(mYs);
  free(sc);
  free(ss);
}

/* ------------------------------------------------- brute-force references */
/* Legendre polynomial P_l(x), l = 0..L, by Bonnet's recurrence */
static void legendre_pl(int L, double x, double *p) {
  p[0] = 1.0;
  if (L >= 1) p[1] = x;
  for (int l = 2; l <= L; ++l) p[l] = ((2.0 * l - 1.0) * x * p[l - 1] - (l - 1.0) * p[l - 2]) / l;
}

/* Truncated Laplace expansion of the Green's function summed over sources j,
   evaluated at field points (fx,fy,fz)[nf]:
     Phi(f) = -sum_{j != skip(f)} m_j sum_{l<=lmax} r_<^l / r_>^(l+1) P_l(cos gamma).
   If skip_self, field point f is source f and is skipped.  This is the addition-
   theorem form of the multipole expansion and does not use spherical harmonics.  */
void oracle_mex_brute(const double *x, const double *y, const double *z, const double *mass,
                      int64_t np, int lmax, const double *fx, const double *fy, const double *fz,
                      int64_t nf, int skip_self, double *pot) {
#pragma omp parallel
  {
    double *p = (double *)malloc(sizeof(double) * (size_t)(lmax + 1));
#pragma omp for schedule(static)
    for (int64_t i = 0; i < nf; ++i) {
      double ri = sqrt(fx[i] * fx[i] + fy[i] * fy[i] + fz[i] * fz[i]);
      double acc = 0.0;
      for (int64_t j = 0; j < np; ++j) {
        if (skip_self && j == i) continue;
        double rj = sqrt(x[j] * x[j] + y[j] * y[j] + z[j] * z[j]);
        double cg = (ri > 0.0 && rj > 0.0) ? (fx[i] * x[j] + fy[i] * y[j] + fz[i] * z[j]) / (ri * rj) : 1.0;
        if (cg > 1.0) cg = 1.0;
        if (cg < -1.0) cg = -1.0;
        legendre_pl(lmax, cg, p);
        double rl = ri < rj ? ri : rj, rg = ri < rj ? rj : ri;
        double term = 0.0;
        for (int l = 0; l <= lmax; ++l) term += pow(rl, (double)l) / pow(rg, l + 1.0) * p[l];
        acc -= mass[j] * term;
      }
      pot[i] = acc;
    }
    free(p);
  }
}

/* Direct (unsoftened) summation: Phi_i = -sum_{j != i} m_j / |x_i - x_j|, a = -grad Phi */
void oracle_direct(const double *x, const double *y, const double *z, const double *mass,
                   int64_t np, double *pot, double *ax, double *ay, double *az) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < np; ++i) {
    double P = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    for (int64_t j = 0; j < np; ++j) {
      if (j == i) continue;
      double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
      double d = sqrt(dx * dx + dy * dy + dz * dz);
      P -= mass[j] / d;
      double d3 = d * d * d;
      gx += mass[j] * dx / d3;
      gy += mass[j] * dy / d3;
      gz += mass[j] * dz / d3;
    }
    pot[i] = P;
    ax[i] = gx;
    ay[i] = gy;
    az[i] = gz;
  }
}

/* ------------------------------------------------------- leapfrog (KDK) */
/* nsys independent systems, particles offsets[s]..offsets[s+1]; each step:
   v += dt/2 a(x); x += dt v; v += dt/2 a(x), with a from that system's own SCF
   coefficients recomputed at the current positions. */
void oracle_leapfrog_scf(double *x, double *y, double *z, double *vx, double *vy, double *vz,
                         const double *mass, const int64_t *offsets, int nsys, int nmax, int lmax,
                         double dt, int nsteps) {
  int K = oracle_coeff_count(nmax, lmax);
  double *A = (double *)malloc(sizeof(double) * (size_t)K);
  double *B = (double *)malloc(sizeof(double) * (size_t)K);
  for (int s = 0; s < nsys; ++s) {
    int64_t o = offsets[s], n = offsets[s + 1] - offsets[s];
    if (n <= 0) continue;
    double *gx = (double *)malloc(sizeof(double) * (size_t)n);
    double *gy = (double *)malloc(sizeof(double) * (size_t)n);
    double *gz = (double *)malloc(sizeof(double) * (size_t)n);
    oracle_scf_coeffs(x + o, y + o, z + o, mass + o, n, nmax, lmax, A, B);
    oracle_scf_force(x + o, y + o, z + o, n, nmax, lmax, A, B, NULL, gx, gy, gz);
    for (int step = 0; step < nsteps; ++step) {
      for (int64_t i = 0; i < n; ++i) {
        vx[o + i] += 0.5 * dt * gx[i];
        vy[o + i] += 0.5 * dt * gy[i];
        vz[o + i] += 0.5 * dt * gz[i];
        x[o + i] += dt * vx[o + i];
        y[o + i] += dt * vy[o + i];
        z[o + i] += dt * vz[o + i];
      }
      oracle_scf_coeffs(x + o, y + o, z + o, mass + o, n, nmax, lmax, A, B);
      oracle_scf_force(x + o, y + o, z + o, n, nmax, lmax, A, B, NULL, gx, gy, gz);
      for (int64_t i = 0; i < n; ++i) {
        vx[o + i] += 0.5 * dt * gx[i];
        vy[o + i] += 0.5 * dt * gy[i];
        vz[o + i] += 0.5 * dt * gz[i];
      }
    }
    free(gx);
    free(gy);
    free(gz);
  }
  free(A);
  free(B);
}
