/*
 * oracle.c -- FP64 CPU oracle for the line-by-line opacity hot path of
 * HELIOS-K 2.0 (Grimm et al. 2021, arXiv:2101.02005).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do. It shares no code, header, table or constant with the HIP path.
 *
 * What it computes (plain definitions, slow and direct, all in IEEE double,
 * compiled with -ffp-contract=off):
 *
 *   line strength   S_i(T)  : Sec. 2.2.2 "Line intensity", eq. (S) rewritten as
 *                             eq. (S1) with the temperature-independent S'
 *                             (Sec. 2.4.3, step 1). S' is recovered from the
 *                             input strength at the reference temperature.
 *   Doppler width   alpha_i : eq. (gammaD) without the sqrt(ln 2) factor, i.e.
 *                             the inverse of eq. (alphaD):
 *                             alpha = (nu0 / c) sqrt(2 k_B T / m).
 *   Lorentz width   gamma_i : ExoMol form, Sec. 2.2 (equation after eq. gammaL)
 *                             without the natural-broadening A/(4 pi c) term:
 *                             gamma = gamma_ref (T_ref/T)^n (P/P_ref).
 *   Voigt profile   V       : Re w(x + i y) / (sqrt(pi) alpha) with
 *                             x = (nu - nu0)/alpha, y = gamma/alpha
 *                             (Sec. 2.4.2, eqs. for x, y and alphaD);
 *                             unit area in nu.
 *   opacity         k_j     : sum over lines with |nu_j - nu_i| <= cut of
 *                             S_i V(nu_j - nu_i) (Sec. 2.4.3 step 4, fixed
 *                             cutting length), grid nu_j = nu_start + j dnu.
 *   options (or_opacity_ex) : the four line profiles of Sec. 2.1 (Voigt, Lorentz,
 *                             Doppler, binned Gaussian integrated cross section),
 *                             plinth removal (Sec. 2.1.1: the line's own value at its
 *                             cutting length subtracted inside the cut), and the cut
 *                             as a fixed length or a multiple of the Doppler or the
 *                             Lorentz half-width (Sec. 2.4.3 step 4, Sec. 2.4.5).
 *   gradient                : analytic adjoint of k (no counterpart in the paper):
 *                             profile derivatives from w'(z) = -2 z w(z) + 2i/sqrt(pi)
 *                             for |z| < 10, and by Gauss-Hermite quadrature of the
 *                             Gaussian-Lorentzian convolution, differentiated under
 *                             the integral, for |z| >= 10 (see or_voigt_derivs).
 *
 * The Faddeeva function w(z) = exp(-z^2) erfc(-iz) is this file's own FP64
 * implementation of a published method: W. Gautschi, "Efficient computation of
 * the complex error function", SIAM J. Numer. Anal. 7 (1970) 187-198, with the
 * region boundaries and term counts of G.P.M. Poppe & C.M.J. Wijers, "More
 * efficient computation of the complex error function", ACM TOMS 16 (1990)
 * 38-46 (power series near the origin, Laplace continued fraction far out,
 * Gautschi's truncated-Taylor + continued-fraction combination in between).
 *
 * Pins (tests/, run without a GPU): scipy.special.wofz and mpmath on a
 * log-polar sweep, w(0)=1, w(iy)=erfcx(y), Re w(x)=exp(-x^2),
 * Im w(x)=(2/sqrt(pi)) Dawson(x), Gaussian and Lorentz limits of V, unit
 * normalization, S(T_ref)=S_ref, the eq. (S) form with synthetic A, g', m,
 * brute-force sums, finite differences of the gradient and its exact invariants.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- constants */
/* Boltzmann constant, as printed with eq. (gammaD) [erg/K] */
static const double OR_KB = 1.3806489e-16;
/* speed of light, as printed with eq. (S) [cm/s] */
static const double OR_CLIGHT = 2.99792458e10;
/* Planck constant [erg s]: not printed in the paper; CODATA 2010, the vintage of k_B */
static const double OR_H = 6.62606957e-27;
/* atomic mass unit [g] (molar mass / Avogadro; CODATA 2010) */
static const double OR_AMU = 1.660538921e-24;
static const double OR_SQRT_PI = 1.7724538509055160273;
static const double OR_TWO_OVER_SQRT_PI = 1.1283791670955125739;
static const double OR_PI = 3.14159265358979323846;

typedef struct or_species {
  double mass_amu;   /* molecular mass [amu] */
  double T_ref;      /* reference temperature of S_ref and gamma_ref [K] */
  double P_ref_atm;  /* reference pressure of gamma_ref [atm] */
  double q_a, q_b;   /* partition function Q(T) = q_a T^q_b */
} or_species;

static double or_c2(void) { return OR_H * OR_CLIGHT / OR_KB; } /* second radiation constant [cm K] */

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------ compensated summation */
/* Neumaier's improved Kahan summation (A. Neumaier, ZAMM 54 (1974) 39-51). */
typedef struct { double s, c; } or_sum;
static inline void or_sum_add(or_sum* a, double v) {
  double t = a->s + v;
  if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
  else a->c += (v - t) + a->s;
  a->s = t;
}
static inline double or_sum_get(const or_sum* a) { return a->s + a->c; }

/* ------------------------------------------------------- Faddeeva function */
/* w(z) for z = xa + i ya in the closed first quadrant (xa >= 0, ya >= 0). */
static void or_w_q1(double xa, double ya, double* u, double* v) {
  const double xs = xa / 6.3, ys = ya / 4.4;
  const double rho2 = xs * xs + ys * ys;
  if (rho2 < 0.085264) {
    /* Near the origin: w = exp(-z^2) [1 + (2i/sqrt(pi)) z sum_k (z^2)^k / (k! (2k+1))]
     * (the Maclaurin series of erf(iz)); the sum is evaluated by Horner's rule. */
    const double xq = (xa - ya) * (xa + ya), yq = 2.0 * xa * ya; /* z^2 */
    const double r = (1.0 - 0.85 * ys) * sqrt(rho2);
    const int nterm = (int)lround(6.0 + 72.0 * r);
    double sr = 1.0 / (2.0 * nterm + 1.0), si = 0.0;
    for (int k = nterm; k >= 1; --k) {
      const double tr = (sr * xq - si * yq) / k;
      si = (sr * yq + si * xq) / k;
      sr = tr + 1.0 / (2.0 * k - 1.0);
    }
    const double u1 = 1.0 - OR_TWO_OVER_SQRT_PI * (sr * ya + si * xa);
    const double v1 = OR_TWO_OVER_SQRT_PI * (sr * xa - si * ya);
    const double e = exp(-xq);
    const double u2 = e * cos(yq), v2 = -e * sin(yq);
    *u = u1 * u2 - v1 * v2;
    *v = u1 * v2 + v1 * u2;
    return;
  }
  /* Elsewhere: Laplace continued fraction r_n = (1/2) / (h - i z + (n+1) r_{n+1}),
   * run from depth nu down to 0. For h = 0 (far from the origin) w = (2/sqrt(pi)) r_0.
   * For 0 < h (intermediate region) Gautschi's combination with the truncated Taylor
   * series about z + i h is used: s_n = r_n (lambda_n + s_{n+1}), lambda_n = (2h)^n,
   * w = (2/sqrt(pi)) s_0. */
  double h = 0.0, h2 = 0.0, lam = 0.0;
  int kapn = 0, depth;
  if (rho2 > 1.0) {
    depth = (int)(3.0 + 1442.0 / (26.0 * sqrt(rho2) + 77.0));
  } else {
    const double r = (1.0 - ys) * sqrt(1.0 - rho2);
    h = 1.88 * r;
    h2 = 2.0 * h;
    kapn = (int)lround(7.0 + 34.0 * r);
    depth = (int)lround(16.0 + 26.0 * r);
    lam = pow(h2, (double)kapn);
  }
  double rx = 0.0, ry = 0.0, sx = 0.0, sy = 0.0;
  for (int n = depth; n >= 0; --n) {
    const double np1 = (double)(n + 1);
    double tx = ya + h + np1 * rx;
    double ty = xa - np1 * ry;
    const double c = 0.5 / (tx * tx + ty * ty);
    rx = c * tx;
    ry = c * ty;
    if (h > 0.0 && n <= kapn) {
      tx = lam + sx;
      const double nsx = rx * tx - ry * sy;
      sy = ry * tx + rx * sy;
      sx = nsx;
      lam /= h2;
    }
  }
  if (h == 0.0) { *u = OR_TWO_OVER_SQRT_PI * rx; *v = OR_TWO_OVER_SQRT_PI * ry; }
  else { *u = OR_TWO_OVER_SQRT_PI * sx; *v = OR_TWO_OVER_SQRT_PI * sy; }
  if (ya == 0.0) *u = exp(-xa * xa); /* on the real axis Re w(x) = exp(-x^2) exactly */
}

/* w(x + i y) for y >= 0, using w(-x + iy) = conj(w(x + iy)). */
void or_faddeeva(double x, double y, double* re, double* im) {
  double u, v;
  or_w_q1(fabs(x), y, &u, &v);
  *re = u;
  *im = x < 0.0 ? -v : v;
}

void or_faddeeva_arr(int64_t n, const double* x, const double* y, double* re, double* im) {
  #pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) or_faddeeva(x[i], y[i], re + i, im + i);
}

/* --------------------------------------------------------- line parameters */
static double or_Q(const or_species* sp, double T) { return sp->q_a * pow(T, sp->q_b); }

/* S(T) following eq. (S1): first the temperature-independent S' (the inverse of
 * eq. (S1) at T_ref, since the input is the strength at T_ref), then
 * S = S'/Q(T) exp(-c2 E''/T) (1 - exp(-c2 nu0/T)); 1 - exp(-a) is taken as -expm1(-a). */
static double or_strength(const or_species* sp, double T, double nu0, double Sref, double E) {
  const double c2 = or_c2();
  const double stim_ref = -expm1(-c2 * nu0 / sp->T_ref);
  const double stim = -expm1(-c2 * nu0 / T);
  const double bexp_ref = c2 * E / sp->T_ref;
  if (bexp_ref < 700.0) {
    const double Sprime = Sref * or_Q(sp, sp->T_ref) * exp(bexp_ref) / stim_ref;
    return Sprime / or_Q(sp, T) * exp(-c2 * E / T) * stim;
  }
  /* exp(c2 E''/T_ref) would overflow: the same product with the exponents combined, and with
   * S_ref inside the exponential, since exp(c2 E'' (1/T_ref - 1/T)) alone can still overflow
   * while S(T) itself is representable */
  if (!(Sref > 0.0)) return 0.0;
  return exp(log(Sref) + c2 * E * (1.0 / sp->T_ref - 1.0 / T)) * (or_Q(sp, sp->T_ref) / or_Q(sp, T)) *
         (stim / stim_ref);
}

static double or_alpha(const or_species* sp, double T, double nu0) {
  const double m = sp->mass_amu * OR_AMU;
  return nu0 / OR_CLIGHT * sqrt(2.0 * OR_KB * T / m);
}

static double or_gamma(const or_species* sp, double T, double P, double gref, double n) {
  return gref * pow(sp->T_ref / T, n) * (P / sp->P_ref_atm);
}

void or_line_params(int64_t N, const double* nu, const double* Sref, const double* E,
                    const double* gref, const double* nexp, const or_species* sp, double T, double P,
                    double* S_T, double* alpha, double* gamma) {
  #pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    if (S_T) S_T[i] = or_strength(sp, T, nu[i], Sref[i], E[i]);
    if (alpha) alpha[i] = or_alpha(sp, T, nu[i]);
    if (gamma) gamma[i] = or_gamma(sp, T, P, gref[i], nexp[i]);
  }
}

/* Voigt profile with unit area */
static double or_voigt(double delta, double alpha, double gamma) {
  double re, im;
  or_faddeeva(delta / alpha, gamma / alpha, &re, &im);
  return re / (OR_SQRT_PI * alpha);
}

void or_voigt_arr(int64_t n, const double* delta, const double* alpha, const double* gamma, double* V) {
  #pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) V[i] = or_voigt(delta[i], alpha[i], gamma[i]);
}

/* Gauss-Hermite rule for the weight exp(-t^2): nodes and weights are handed in by the Python
 * side (a library routine), OR_GH_MAX at most. */
#define OR_GH_MAX 64
static int or_gh_n = 0;
static double or_gh_t[OR_GH_MAX], or_gh_w[OR_GH_MAX];

int or_set_gauss_hermite(int n, const double* t, const double* w) {
  if (n < 1 || n > OR_GH_MAX) return -1;
  for (int k = 0; k < n; ++k) { or_gh_t[k] = t[k]; or_gh_w[k] = w[k]; }
  or_gh_n = n;
  return 0;
}

/* |z| from which the profile derivatives are integrated instead of taken from w'(z). */
#define OR_DERIV_ZQUAD 10.0

/* dV/dgamma and dV/dalpha of the unit-area Voigt profile at offset delta.
 * Near the centre (|z| < 10, z = (delta + i gamma)/alpha) from w'(z) = -2 z w(z) + 2i/sqrt(pi):
 *   dK/dx = -2 (xK - yL),  dK/dy = 2 (xL + yK) - 2/sqrt(pi),
 *   dV/dgamma = (dK/dy) / (sqrt(pi) alpha^2),  dV/dalpha = -(K + x dK/dx + y dK/dy) / (sqrt(pi) alpha^2).
 * These lose about |z|^2 in relative precision to cancellation (dK/dy falls as 1/|z|^2 while each of
 * its terms stays O(1)), so for |z| >= 10 the profile is written as the convolution of the Gaussian
 * and the Lorentzian, V = pi^-1/2 int exp(-t^2) L(delta - alpha t) dt with L(x) = gamma/(pi (x^2 + gamma^2)),
 * the derivatives are taken under the integral and the integral is done by Gauss-Hermite
 * quadrature (the integrand is analytic in |t| < |z|, so the rule converges geometrically):
 *   dV/dgamma = pi^-1/2 sum_k w_k (x_k^2 - gamma^2) / (pi (x_k^2 + gamma^2)^2),
 *   dV/dalpha = pi^-1/2 sum_k w_k t_k 2 gamma x_k / (pi (x_k^2 + gamma^2)^2),  x_k = delta - alpha t_k. */
static void or_voigt_derivs3(double delta, double alpha, double gamma, double* dVdg, double* dVda,
                             double* dVdd) {
  const double x = delta / alpha, y = gamma / alpha;
  if (x * x + y * y < OR_DERIV_ZQUAD * OR_DERIV_ZQUAD || or_gh_n == 0) {
    double K, L;
    or_faddeeva(x, y, &K, &L);
    const double Kx = -2.0 * (x * K - y * L);
    const double Ky = 2.0 * (x * L + y * K) - OR_TWO_OVER_SQRT_PI;
    const double den = OR_SQRT_PI * alpha * alpha;
    *dVdg = Ky / den;
    *dVda = -(K + x * Kx + y * Ky) / den;
    *dVdd = Kx / den;
    return;
  }
  /* d/d(delta) of the Lorentzian under the integral: -2 gamma x_k / (pi (x_k^2 + gamma^2)^2) */
  double sg = 0.0, sa = 0.0, sd = 0.0;
  for (int k = 0; k < or_gh_n; ++k) {
    const double xk = delta - alpha * or_gh_t[k];
    const double d = xk * xk + gamma * gamma;
    const double inv = 1.0 / (OR_PI * d * d);
    sg += or_gh_w[k] * (xk * xk - gamma * gamma) * inv;
    sa += or_gh_w[k] * or_gh_t[k] * 2.0 * gamma * xk * inv;
    sd -= or_gh_w[k] * 2.0 * gamma * xk * inv;
  }
  *dVdg = sg / OR_SQRT_PI;
  *dVda = sa / OR_SQRT_PI;
  *dVdd = sd / OR_SQRT_PI;
}

static void or_voigt_derivs(double delta, double alpha, double gamma, double* dVdg, double* dVda) {
  double dd;
  or_voigt_derivs3(delta, alpha, gamma, dVdg, dVda, &dd);
}

void or_voigt_derivs_arr(int64_t n, const double* delta, const double* alpha, const double* gamma,
                         double* dVdg, double* dVda, double* dVdd) {
  #pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double dd;
    or_voigt_derivs3(delta[i], alpha[i], gamma[i], &dVdg[i], &dVda[i], &dd);
    if (dVdd) dVdd[i] = dd;
  }
}

/* grid point: nu_j = nu_start + j*dnu, a product then a sum */
static inline double or_grid(double nu_start, double dnu, int64_t j) {
  const double p = (double)j * dnu;
  return nu_start + p;
}

/* Grid-index range [*j0, *j1] of the points with |nu_j - nu0| <= cut (empty: *j1 < *j0).
 * nu_j - nu0 is non-decreasing in j, so the points form one contiguous run; candidates
 * from ceil/floor are refined with the exact predicate. */
static void or_jrange(double nu0, double nu_start, double dnu, int64_t n_grid, double cut,
                      int64_t* j0, int64_t* j1) {
  if (isinf(cut)) { *j0 = 0; *j1 = n_grid - 1; return; }
  double lo = ceil((nu0 - cut - nu_start) / dnu) - 2.0;
  double hi = floor((nu0 + cut - nu_start) / dnu) + 2.0;
  if (lo < 0.0) lo = 0.0;
  if (hi > (double)(n_grid - 1)) hi = (double)(n_grid - 1);
  if (!(lo <= hi)) { *j0 = 0; *j1 = -1; return; }
  int64_t a = (int64_t)lo, b = (int64_t)hi;
  while (a <= b && !(fabs(or_grid(nu_start, dnu, a) - nu0) <= cut)) ++a;
  while (b >= a && !(fabs(or_grid(nu_start, dnu, b) - nu0) <= cut)) --b;
  *j0 = a;
  *j1 = b;
}

/* ------------------------------------------------------------ sorted lines */
typedef struct { double nu; int64_t i; } or_key;
static int or_key_cmp(const void* a, const void* b) {
  const or_key* x = (const or_key*)a;
  const or_key* y = (const or_key*)b;
  if (x->nu < y->nu) return -1;
  if (x->nu > y->nu) return 1;
  return (x->i > y->i) - (x->i < y->i);
}

/* first position in the sorted keys with nu >= v */
static int64_t or_lower(const or_key* k, int64_t N, double v) {
  int64_t lo = 0, hi = N;
  while (lo < hi) { int64_t m = lo + (hi - lo) / 2; if (k[m].nu < v) lo = m + 1; else hi = m; }
  return lo;
}

/* ------------------------------------------------------------------ opacity */
/* k at the requested grid indices pts[0..n_pts): direct compensated sum over every
 * line with |nu_j - nu_i| <= cut (cut = +inf: all lines). Returns 0, or -1 on bad input. */
int or_opacity(int64_t N, const double* nu, const double* Sref, const double* E, const double* gref,
               const double* nexp, const or_species* sp, double T, double P, double nu_start,
               double dnu, double cut, int64_t n_pts, const int64_t* pts, double* k_out) {
  if (N < 0 || n_pts < 0 || !(T > 0.0) || !(P >= 0.0) || !(dnu > 0.0) || !(cut > 0.0)) return -1;
  double* S = (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
  double* al = (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
  double* ga = (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
  or_key* key = (or_key*)malloc(sizeof(or_key) * (size_t)(N > 0 ? N : 1));
  if (!S || !al || !ga || !key) { free(S); free(al); free(ga); free(key); return -2; }
  or_line_params(N, nu, Sref, E, gref, nexp, sp, T, P, S, al, ga);
  for (int64_t i = 0; i < N; ++i) { key[i].nu = nu[i]; key[i].i = i; }
  qsort(key, (size_t)N, sizeof(or_key), or_key_cmp);
  const int nocut = isinf(cut);
  #pragma omp parallel for schedule(dynamic, 16)
  for (int64_t q = 0; q < n_pts; ++q) {
    const double nuj = or_grid(nu_start, dnu, pts[q]);
    int64_t a = 0, b = N;
    if (!nocut) {
      /* candidate range, widened; the exact predicate below decides */
      const double pad = cut * 1e-9 + fabs(nuj) * 1e-12;
      a = or_lower(key, N, nuj - cut - pad);
      b = or_lower(key, N, nuj + cut + pad);
      while (b < N && key[b].nu <= nuj + cut + pad) ++b;
    }
    or_sum acc = {0.0, 0.0};
    for (int64_t p = a; p < b; ++p) {
      const int64_t i = key[p].i;
      const double d = nuj - nu[i];
      if (!nocut && !(fabs(d) <= cut)) continue;
      or_sum_add(&acc, S[i] * or_voigt(d, al[i], ga[i]));
    }
    k_out[q] = or_sum_get(&acc);
  }
  free(S); free(al); free(ga); free(key);
  return 0;
}

/* --------------------------------------------------------------- gradient */
/* Adjoint of L = sum_j g_j k_j for the lines sel[0..n_sel), with g = dL/dk on the whole
 * grid [0, n_grid). Per selected line (outputs indexed like sel):
 *   GS  = sum_j g_j V_ij,   Gg = S_i sum_j g_j dV_ij/dgamma,   Ga = S_i sum_j g_j dV_ij/dalpha
 *   dSref = (S_i/Sref_i) GS,  dgref = (gamma_i/gref_i) Gg,  dn = gamma_i ln(T_ref/T) Gg,
 *   dT_part = GS dS_i/dT + Ga alpha_i/(2T) - Gg n_i gamma_i/T,   dlnP_part = gamma_i Gg.
 * With x = d/alpha, y = gamma/alpha, w = K + iL:
 *   dK/dx = -2(xK - yL),  dK/dy = 2(xL + yK) - 2/sqrt(pi)    (from w' = -2zw + 2i/sqrt(pi))
 *   dV/dgamma = K_y/(sqrt(pi) alpha^2),  dV/dalpha = -(K + x K_x + y K_y)/(sqrt(pi) alpha^2). */
int or_gradient(int64_t N, const double* nu, const double* Sref, const double* E, const double* gref,
                const double* nexp, const or_species* sp, double T, double P, double nu_start,
                double dnu, int64_t n_grid, double cut, const double* g, int64_t n_sel,
                const int64_t* sel, double* GS, double* Gg, double* Ga, double* dSref, double* dgref,
                double* dn, double* dT_part, double* dlnP_part) {
  if (N < 0 || n_sel < 0 || n_grid < 0 || !(T > 0.0) || !(P >= 0.0) || !(dnu > 0.0) || !(cut > 0.0))
    return -1;
  const double c2 = or_c2();
  #pragma omp parallel for schedule(dynamic, 4)
  for (int64_t q = 0; q < n_sel; ++q) {
    const int64_t i = sel[q];
    const double S = or_strength(sp, T, nu[i], Sref[i], E[i]);
    const double al = or_alpha(sp, T, nu[i]);
    const double ga = or_gamma(sp, T, P, gref[i], nexp[i]);
    int64_t j0, j1;
    or_jrange(nu[i], nu_start, dnu, n_grid, cut, &j0, &j1);
    or_sum sV = {0, 0}, sY = {0, 0}, sA = {0, 0};
    for (int64_t j = j0; j <= j1; ++j) {
      const double d = or_grid(nu_start, dnu, j) - nu[i];
      double dVdg, dVda;
      or_voigt_derivs(d, al, ga, &dVdg, &dVda);
      or_sum_add(&sV, g[j] * or_voigt(d, al, ga));
      or_sum_add(&sY, g[j] * dVdg);
      or_sum_add(&sA, g[j] * dVda);
    }
    const double gs = or_sum_get(&sV), gg = S * or_sum_get(&sY), gal = S * or_sum_get(&sA);
    if (GS) GS[q] = gs;
    if (Gg) Gg[q] = gg;
    if (Ga) Ga[q] = gal;
    /* d ln S / dT = -q_b/T + c2 E''/T^2 - (c2 nu/T^2) / expm1(c2 nu/T) */
    const double dlnS_dT = -sp->q_b / T + c2 * E[i] / (T * T) - (c2 * nu[i] / (T * T)) / expm1(c2 * nu[i] / T);
    if (dSref) dSref[q] = (Sref[i] != 0.0 ? S / Sref[i] : 0.0) * gs;
    if (dgref) dgref[q] = (gref[i] != 0.0 ? ga / gref[i] : 0.0) * gg;
    if (dn) dn[q] = ga * log(sp->T_ref / T) * gg;
    if (dT_part) dT_part[q] = gs * S * dlnS_dT + gal * al / (2.0 * T) - gg * nexp[i] * ga / T;
    if (dlnP_part) dlnP_part[q] = ga * gg;
  }
  return 0;
}

/* Single-line functional L_i = sum_j g_j S_i V_ij (the part of L carried by line i),
 * for finite-difference checks of the per-line gradient. */
int or_line_functional(int64_t n_sel, const double* nu, const double* Sref, const double* E,
                       const double* gref, const double* nexp, const or_species* sp, double T, double P,
                       double nu_start, double dnu, int64_t n_grid, double cut, const double* g,
                       double* Li) {
  #pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < n_sel; ++i) {
    const double S = or_strength(sp, T, nu[i], Sref[i], E[i]);
    const double al = or_alpha(sp, T, nu[i]);
    const double ga = or_gamma(sp, T, P, gref[i], nexp[i]);
    int64_t j0, j1;
    or_jrange(nu[i], nu_start, dnu, n_grid, cut, &j0, &j1);
    or_sum acc = {0, 0};
    for (int64_t j = j0; j <= j1; ++j) {
      const double d = or_grid(nu_start, dnu, j) - nu[i];
      or_sum_add(&acc, g[j] * S * or_voigt(d, al, ga));
    }
    Li[i] = or_sum_get(&acc);
  }
  return 0;
}

/* number of (line, grid point) pairs with |nu_j - nu_i| <= cut, 0 <= j < n_grid, per line
 * (the Voigt-evaluation count that defines the throughput unit) */
int64_t or_count_evals(int64_t N, const double* nu, double nu_start, double dnu, int64_t n_grid,
                       double cut) {
  int64_t total = 0;
  #pragma omp parallel for schedule(static) reduction(+ : total)
  for (int64_t i = 0; i < N; ++i) {
    int64_t j0, j1;
    or_jrange(nu[i], nu_start, dnu, n_grid, cut, &j0, &j1);
    if (j1 >= j0) total += j1 - j0 + 1;
  }
  return total;
}

/* per-line point ranges (for tests of the cut predicate) */
void or_jranges(int64_t N, const double* nu, double nu_start, double dnu, int64_t n_grid, double cut,
                int64_t* j0, int64_t* j1) {
  #pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) or_jrange(nu[i], nu_start, dnu, n_grid, cut, j0 + i, j1 + i);
}

/* ===================================================================== options */
/* The four line profiles HELIOS-K offers (Sec. 2.1), per unit strength, at offset d from the
 * line centre:
 *   0 Voigt            Re w((d + i gamma)/alpha) / (sqrt(pi) alpha)
 *   1 Lorentz          gamma / (pi (d^2 + gamma^2))            (gamma = 0: zero)
 *   2 Doppler          exp(-(d/alpha)^2) / (sqrt(pi) alpha)
 *   3 binned Gaussian  the Doppler profile averaged over the grid bin [d - dnu/2, d + dnu/2]
 *                      (the integrated cross section per bin, divided by the bin width):
 *                      (erf((d + dnu/2)/alpha) - erf((d - dnu/2)/alpha)) / (2 dnu), the
 *                      difference of erfc taken where both arguments have the same sign */
enum { OR_VOIGT = 0, OR_LORENTZ = 1, OR_DOPPLER = 2, OR_BINNED_GAUSS = 3 };
/* The cutting length of a line (Sec. 2.4.3 step 4): a fixed length, or the given multiple of its
 * Doppler half-width Gamma_D = sqrt(ln 2) alpha (eq. gammaD) or of its Lorentz half-width gamma. */
enum { OR_CUT_FIXED = 0, OR_CUT_DOPPLER = 1, OR_CUT_LORENTZ = 2 };

static double or_profile(int prof, double d, double alpha, double gamma, double dnu) {
  if (prof == OR_LORENTZ) return gamma > 0.0 ? gamma / (OR_PI * (d * d + gamma * gamma)) : 0.0;
  if (prof == OR_DOPPLER) {
    const double x = d / alpha;
    return exp(-x * x) / (OR_SQRT_PI * alpha);
  }
  if (prof == OR_BINNED_GAUSS) {
    const double a = (d - 0.5 * dnu) / alpha, b = (d + 0.5 * dnu) / alpha;
    double diff;
    if (a >= 0.0) diff = erfc(a) - erfc(b);
    else if (b <= 0.0) diff = erfc(-b) - erfc(-a);
    else diff = erf(b) - erf(a);
    return diff / (2.0 * dnu);
  }
  return or_voigt(d, alpha, gamma);
}

static double or_cut_length(int mode, double cut, double alpha, double gamma) {
  if (isinf(cut)) return cut;
  if (mode == OR_CUT_DOPPLER) return cut * sqrt(log(2.0)) * alpha;
  if (mode == OR_CUT_LORENTZ) return cut * gamma;
  return cut;
}

/* per-line cut lengths at (T, P) */
void or_cut_lengths(int64_t N, const double* nu, const double* gref, const double* nexp,
                    const or_species* sp, double T, double P, int cut_mode, double cut, double* out) {
  #pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i)
    out[i] = or_cut_length(cut_mode, cut, or_alpha(sp, T, nu[i]), or_gamma(sp, T, P, gref[i], nexp[i]));
}

/* k at the grid indices pts with a profile, a cut mode and optional plinth removal: per point, the
 * compensated sum over the lines with |nu_j - nu_i| <= cut_i of S_i (f(nu_j - nu_i) - [plinth]
 * f(cut_i)), f the profile (the plinth is zero without a cut). Returns 0, or -1 on bad input. */
int or_opacity_ex(int64_t N, const double* nu, const double* Sref, const double* E, const double* gref,
                  const double* nexp, const or_species* sp, double T, double P, double nu_start,
                  double dnu, double cut, int cut_mode, int profile, int plinth, int64_t n_pts,
                  const int64_t* pts, double* k_out) {
  if (N < 0 || n_pts < 0 || !(T > 0.0) || !(P >= 0.0) || !(dnu > 0.0) || !(cut > 0.0)) return -1;
  if (cut_mode < 0 || cut_mode > 2 || profile < 0 || profile > 3) return -1;
  const size_t NN = (size_t)(N > 0 ? N : 1);
  double* S = (double*)malloc(sizeof(double) * NN);
  double* al = (double*)malloc(sizeof(double) * NN);
  double* ga = (double*)malloc(sizeof(double) * NN);
  double* cl = (double*)malloc(sizeof(double) * NN);
  double* pl = (double*)malloc(sizeof(double) * NN);
  or_key* key = (or_key*)malloc(sizeof(or_key) * NN);
  if (!S || !al || !ga || !cl || !pl || !key) {
    free(S); free(al); free(ga); free(cl); free(pl); free(key);
    return -2;
  }
  or_line_params(N, nu, Sref, E, gref, nexp, sp, T, P, S, al, ga);
  double cmax = 0.0;
  for (int64_t i = 0; i < N; ++i) {
    cl[i] = or_cut_length(cut_mode, cut, al[i], ga[i]);
    pl[i] = (plinth && !isinf(cl[i])) ? or_profile(profile, cl[i], al[i], ga[i], dnu) : 0.0;
    if (cl[i] > cmax) cmax = cl[i];
    key[i].nu = nu[i];
    key[i].i = i;
  }
  qsort(key, (size_t)N, sizeof(or_key), or_key_cmp);
  #pragma omp parallel for schedule(dynamic, 16)
  for (int64_t q = 0; q < n_pts; ++q) {
    const double nuj = or_grid(nu_start, dnu, pts[q]);
    int64_t a = 0, b = N;
    if (!isinf(cmax)) {
      const double pad = cmax * 1e-9 + fabs(nuj) * 1e-12;
      a = or_lower(key, N, nuj - cmax - pad);
      b = or_lower(key, N, nuj + cmax + pad);
      while (b < N && key[b].nu <= nuj + cmax + pad) ++b;
    }
    or_sum acc = {0.0, 0.0};
    for (int64_t p = a; p < b; ++p) {
      const int64_t i = key[p].i;
      const double d = nuj - nu[i];
      if (!(fabs(d) <= cl[i])) continue;
      or_sum_add(&acc, S[i] * (or_profile(profile, d, al[i], ga[i], dnu) - pl[i]));
    }
    k_out[q] = or_sum_get(&acc);
  }
  free(S); free(al); free(ga); free(cl); free(pl); free(key);
  return 0;
}

/* The adjoint of L = sum_j g_j k_j for the Voigt profile with a cut mode and optional plinth
 * removal, per selected line (outputs as or_gradient). The cut indicator is not differentiated;
 * the plinth S_i V(c_i) is, including the cut length c_i's own dependence on alpha (Doppler mode,
 * c = m sqrt(ln 2) alpha) or gamma (Lorentz mode, c = m gamma):
 *   GS -= G_box V(c),  Gg -= S G_box (dV/dgamma + [Lorentz] m dV/dd),
 *   Ga -= S G_box (dV/dalpha + [Doppler] m sqrt(ln 2) dV/dd),  G_box = sum of g over the cut range. */
int or_gradient_ex(int64_t N, const double* nu, const double* Sref, const double* E, const double* gref,
                   const double* nexp, const or_species* sp, double T, double P, double nu_start,
                   double dnu, int64_t n_grid, double cut, int cut_mode, int plinth, const double* g,
                   int64_t n_sel, const int64_t* sel, double* GS, double* Gg, double* Ga, double* dSref,
                   double* dgref, double* dn, double* dT_part, double* dlnP_part) {
  if (N < 0 || n_sel < 0 || n_grid < 0 || !(T > 0.0) || !(P >= 0.0) || !(dnu > 0.0) || !(cut > 0.0))
    return -1;
  if (cut_mode < 0 || cut_mode > 2) return -1;
  const double c2 = or_c2();
  #pragma omp parallel for schedule(dynamic, 4)
  for (int64_t q = 0; q < n_sel; ++q) {
    const int64_t i = sel[q];
    const double S = or_strength(sp, T, nu[i], Sref[i], E[i]);
    const double al = or_alpha(sp, T, nu[i]);
    const double ga = or_gamma(sp, T, P, gref[i], nexp[i]);
    const double ci = or_cut_length(cut_mode, cut, al, ga);
    int64_t j0, j1;
    or_jrange(nu[i], nu_start, dnu, n_grid, ci, &j0, &j1);
    or_sum sV = {0, 0}, sY = {0, 0}, sA = {0, 0}, sB = {0, 0};
    for (int64_t j = j0; j <= j1; ++j) {
      const double d = or_grid(nu_start, dnu, j) - nu[i];
      double dVdg, dVda;
      or_voigt_derivs(d, al, ga, &dVdg, &dVda);
      or_sum_add(&sV, g[j] * or_voigt(d, al, ga));
      or_sum_add(&sY, g[j] * dVdg);
      or_sum_add(&sA, g[j] * dVda);
      or_sum_add(&sB, g[j]);
    }
    double gs = or_sum_get(&sV), yy = or_sum_get(&sY), aa = or_sum_get(&sA);
    if (plinth && !isinf(ci) && j1 >= j0) {
      const double Gbox = or_sum_get(&sB);
      double pg, pa, pd;
      or_voigt_derivs3(ci, al, ga, &pg, &pa, &pd);
      if (cut_mode == OR_CUT_LORENTZ) pg += cut * pd;                   /* dc/dgamma = m */
      if (cut_mode == OR_CUT_DOPPLER) pa += cut * sqrt(log(2.0)) * pd;  /* dc/dalpha = m sqrt(ln 2) */
      gs -= Gbox * or_voigt(ci, al, ga);
      yy -= Gbox * pg;
      aa -= Gbox * pa;
    }
    const double gg = S * yy, gal = S * aa;
    if (GS) GS[q] = gs;
    if (Gg) Gg[q] = gg;
    if (Ga) Ga[q] = gal;
    const double dlnS_dT = -sp->q_b / T + c2 * E[i] / (T * T) - (c2 * nu[i] / (T * T)) / expm1(c2 * nu[i] / T);
    if (dSref) dSref[q] = (Sref[i] != 0.0 ? S / Sref[i] : 0.0) * gs;
    if (dgref) dgref[q] = (gref[i] != 0.0 ? ga / gref[i] : 0.0) * gg;
    if (dn) dn[q] = ga * log(sp->T_ref / T) * gg;
    if (dT_part) dT_part[q] = gs * S * dlnS_dT + gal * al / (2.0 * T) - gg * nexp[i] * ga / T;
    if (dlnP_part) dlnP_part[q] = ga * gg;
  }
  return 0;
}

/* ======================================================= HITRAN widths and shift */
/* The HITRAN form of the Lorentz half-width, eq. (gammaL) without the natural A/(4 pi c) term,
 *   gamma = (T/T_ref)^(-n) [gamma_air (P - P_self) + gamma_self P_self] / P_ref,
 * and the pressure-shifted line centre nu* = nu + delta_air P / P_ref, delta_air being the
 * pressure-dependent line shift of Table binary2 (cm^-1 atm^-1). The shift moves only the centre
 * of the profile: the strength and the Doppler width are those of the transition wavenumber nu.
 * k at the grid indices pts: per point, the compensated sum over the lines with
 * |nu_j - nu*_i| <= cut_i of S_i (f(nu_j - nu*_i) - [plinth] f(cut_i)), with the profile, cut mode
 * and plinth options of or_opacity_ex. Returns 0, or -1 on bad input. */
int or_opacity_hitran(int64_t N, const double* nu, const double* Sref, const double* E, const double* gair,
                      const double* gself, const double* nexp, const double* delta, const or_species* sp,
                      double T, double P, double Pself, double nu_start, double dnu, double cut, int cut_mode,
                      int profile, int plinth, int64_t n_pts, const int64_t* pts, double* k_out) {
  if (N < 0 || n_pts < 0 || !(T > 0.0) || !(P >= 0.0) || !(Pself >= 0.0) || Pself > P || !(dnu > 0.0) ||
      !(cut > 0.0))
    return -1;
  if (cut_mode < 0 || cut_mode > 2 || profile < 0 || profile > 3) return -1;
  const size_t NN = (size_t)(N > 0 ? N : 1);
  double* S = (double*)malloc(sizeof(double) * NN);
  double* al = (double*)malloc(sizeof(double) * NN);
  double* ga = (double*)malloc(sizeof(double) * NN);
  double* cl = (double*)malloc(sizeof(double) * NN);
  double* pl = (double*)malloc(sizeof(double) * NN);
  double* cen = (double*)malloc(sizeof(double) * NN);
  or_key* key = (or_key*)malloc(sizeof(or_key) * NN);
  if (!S || !al || !ga || !cl || !pl || !cen || !key) {
    free(S); free(al); free(ga); free(cl); free(pl); free(cen); free(key);
    return -2;
  }
  double cmax = 0.0;
  for (int64_t i = 0; i < N; ++i) {
    S[i] = or_strength(sp, T, nu[i], Sref[i], E[i]);
    al[i] = or_alpha(sp, T, nu[i]);
    ga[i] = pow(T / sp->T_ref, -nexp[i]) * (gair[i] * (P - Pself) + gself[i] * Pself) / sp->P_ref_atm;
    cen[i] = nu[i] + delta[i] * P / sp->P_ref_atm;
    cl[i] = or_cut_length(cut_mode, cut, al[i], ga[i]);
    pl[i] = (plinth && !isinf(cl[i])) ? or_profile(profile, cl[i], al[i], ga[i], dnu) : 0.0;
    if (cl[i] > cmax) cmax = cl[i];
    key[i].nu = cen[i];
    key[i].i = i;
  }
  qsort(key, (size_t)N, sizeof(or_key), or_key_cmp);
  #pragma omp parallel for schedule(dynamic, 16)
  for (int64_t q = 0; q < n_pts; ++q) {
    const double nuj = or_grid(nu_start, dnu, pts[q]);
    int64_t a = 0, b = N;
    if (!isinf(cmax)) {
      const double pad = cmax * 1e-9 + fabs(nuj) * 1e-12;
      a = or_lower(key, N, nuj - cmax - pad);
      b = or_lower(key, N, nuj + cmax + pad);
      while (b < N && key[b].nu <= nuj + cmax + pad) ++b;
    }
    or_sum acc = {0.0, 0.0};
    for (int64_t p = a; p < b; ++p) {
      const int64_t i = key[p].i;
      const double d = nuj - cen[i];
      if (!(fabs(d) <= cl[i])) continue;
      or_sum_add(&acc, S[i] * (or_profile(profile, d, al[i], ga[i], dnu) - pl[i]));
    }
    k_out[q] = or_sum_get(&acc);
  }
  free(S); free(al); free(ga); free(cl); free(pl); free(cen); free(key);
  return 0;
}
