/*
 * linegen_core.h -- seeded synthetic spectral-line lists (input recipe only).
 *
 * This header is the single definition of the synthetic inputs used by the
 * tests and the benchmark. It is compiled twice: by gcc for the host twin
 * (linegen_cpu.c) and by hipcc for the device twin (linegen_gpu.hip). Every
 * operation is plain IEEE double arithmetic with contraction disabled, and the
 * transcendental helpers below are written out here (not taken from libm or
 * the device math library), so both twins produce bit-identical lines.
 *
 * It holds none of the opacity method's arithmetic: it only draws the five
 * per-line fields (nu, S_ref, E'', gamma_ref, n) from distributions shaped like
 * the paper's workloads.
 *
 * Counter-based uniform (splitmix64 finaliser of Steele, Lea & Flood 2014):
 *   u(seed,i,f) = (splitmix64(seed ^ i*G ^ f*H) >> 11) * 2^-53 + 2^-54   in (0,1)
 * with G = 0x9E3779B97F4A7C15, H = 0xD1B54A32D192ED03; field f = 0..4 is
 * nu, log10-intensity scale s, E'', gamma_ref, n.
 */
#ifndef LINEGEN_CORE_H
#define LINEGEN_CORE_H
#include <stdint.h>

#ifdef __HIPCC__
#define LG_FN __host__ __device__ static inline
#else
#define LG_FN static inline
#endif

typedef struct lg_recipe {
  int32_t nu_law;     /* 0: uniform on [nu_lo, nu_hi);  1: nu_hi * u^2 (density rising to low nu) */
  int32_t e_law;      /* 0: exponential with mean e_par;  1: uniform on [0, e_par) */
  int32_t s_reading;  /* 0: literal, S_ref = 10^s;
                         1: scale reading, S_ref = 10^s e^{-c2 E/T_ref} (1 - e^{-c2 nu/T_ref}) */
  int32_t pad_;
  double nu_lo, nu_hi;
  double s_lo, s_hi;  /* s = log10 intensity scale, uniform */
  double e_par;
  double g_lo, g_hi;  /* gamma_ref [cm^-1 atm^-1], uniform */
  double n_lo, n_hi;  /* temperature exponent, uniform */
  double T_ref;       /* [K] */
} lg_recipe;

/* second radiation constant h c / k_B [cm K] from h = 6.62606957e-27 erg s,
 * c = 2.99792458e10 cm/s, k_B = 1.3806489e-16 erg/K (used only to form S_ref) */
#define LG_C2 1.438776855773617
#define LG_LN2_HI 6.93147180369123816490e-01
#define LG_LN2_LO 1.90821492927058770002e-10
#define LG_LN10 2.302585092994045684

LG_FN uint64_t lg_splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

LG_FN double lg_uniform(uint64_t seed, uint64_t i, uint64_t f) {
  uint64_t h = lg_splitmix64(seed ^ (i * 0x9E3779B97F4A7C15ull) ^ (f * 0xD1B54A32D192ED03ull));
  return (double)(h >> 11) * 0x1.0p-53 + 0x1.0p-54;
}

LG_FN double lg_from_bits(uint64_t b) { union { uint64_t u; double d; } c; c.u = b; return c.d; }
LG_FN uint64_t lg_to_bits(double d) { union { uint64_t u; double d; } c; c.d = d; return c.u; }

/* 2^k as a double, -1022 <= k <= 1023 */
LG_FN double lg_pow2i(int k) { return lg_from_bits((uint64_t)(k + 1023) << 52); }

/* e^x: x = k ln2 + r with |r| <= ln2/2; degree-13 Taylor polynomial of e^r; times 2^k */
LG_FN double lg_exp(double x) {
  if (x != x) return x;
  if (x > 709.7) return lg_from_bits(0x7FF0000000000000ull);
  if (x < -745.2) return 0.0;
  double kd = x * 1.4426950408889634074;
  kd = kd < 0.0 ? (double)(int64_t)(kd - 0.5) : (double)(int64_t)(kd + 0.5);
  int k = (int)kd;
  double r = (x - kd * LG_LN2_HI) - kd * LG_LN2_LO;
  double p = 1.0 / 6227020800.0;
  p = p * r + 1.0 / 479001600.0;
  p = p * r + 1.0 / 39916800.0;
  p = p * r + 1.0 / 3628800.0;
  p = p * r + 1.0 / 362880.0;
  p = p * r + 1.0 / 40320.0;
  p = p * r + 1.0 / 5040.0;
  p = p * r + 1.0 / 720.0;
  p = p * r + 1.0 / 120.0;
  p = p * r + 1.0 / 24.0;
  p = p * r + 1.0 / 6.0;
  p = p * r + 0.5;
  p = p * r + 1.0;
  p = p * r + 1.0;
  if (k > 1023) return (p * lg_pow2i(1023)) * lg_pow2i(k - 1023);
  if (k < -1022) return (p * lg_pow2i(k + 200)) * lg_pow2i(-200);
  return p * lg_pow2i(k);
}

/* e^x - 1, Taylor series (to x^17/17!) for |x| <= 0.3 to avoid cancellation */
LG_FN double lg_expm1(double x) {
  if (x > 0.3 || x < -0.3) return lg_exp(x) - 1.0;
  double p = 1.0 / 355687428096000.0;            /* 1/17! */
  p = p * x + 1.0 / 20922789888000.0;            /* 1/16! */
  p = p * x + 1.0 / 1307674368000.0;
  p = p * x + 1.0 / 87178291200.0;
  p = p * x + 1.0 / 6227020800.0;
  p = p * x + 1.0 / 479001600.0;
  p = p * x + 1.0 / 39916800.0;
  p = p * x + 1.0 / 3628800.0;
  p = p * x + 1.0 / 362880.0;
  p = p * x + 1.0 / 40320.0;
  p = p * x + 1.0 / 5040.0;
  p = p * x + 1.0 / 720.0;
  p = p * x + 1.0 / 120.0;
  p = p * x + 1.0 / 24.0;
  p = p * x + 1.0 / 6.0;
  p = p * x + 0.5;
  p = p * x + 1.0;                               /* 1/1! */
  return x * p;
}

/* natural log for finite x > 0 (normal numbers): x = m 2^e, m in [sqrt(1/2), sqrt(2)),
 * log m = 2 atanh(s), s = (m-1)/(m+1), odd series to s^27 */
LG_FN double lg_log(double x) {
  uint64_t b = lg_to_bits(x);
  int e = (int)((b >> 52) & 0x7FF) - 1023;
  double m = lg_from_bits((b & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull);
  if (m > 1.4142135623730951) { m = m * 0.5; e += 1; }
  double s = (m - 1.0) / (m + 1.0);
  double s2 = s * s;
  double p = 1.0 / 27.0;
  p = p * s2 + 1.0 / 25.0;
  p = p * s2 + 1.0 / 23.0;
  p = p * s2 + 1.0 / 21.0;
  p = p * s2 + 1.0 / 19.0;
  p = p * s2 + 1.0 / 17.0;
  p = p * s2 + 1.0 / 15.0;
  p = p * s2 + 1.0 / 13.0;
  p = p * s2 + 1.0 / 11.0;
  p = p * s2 + 1.0 / 9.0;
  p = p * s2 + 1.0 / 7.0;
  p = p * s2 + 1.0 / 5.0;
  p = p * s2 + 1.0 / 3.0;
  p = p * s2 + 1.0;
  double lm = 2.0 * s * p;
  double ed = (double)e;
  return ed * LG_LN2_HI + (ed * LG_LN2_LO + lm);
}

/* all five fields of line i */
LG_FN void lg_line(const lg_recipe* r, uint64_t seed, uint64_t i,
                   double* nu, double* S, double* E, double* g, double* n) {
  double u0 = lg_uniform(seed, i, 0);
  double u1 = lg_uniform(seed, i, 1);
  double u2 = lg_uniform(seed, i, 2);
  double u3 = lg_uniform(seed, i, 3);
  double u4 = lg_uniform(seed, i, 4);
  double v = r->nu_law == 1 ? r->nu_hi * (u0 * u0) : r->nu_lo + (r->nu_hi - r->nu_lo) * u0;
  double s = r->s_lo + (r->s_hi - r->s_lo) * u1;
  double e = r->e_law == 1 ? r->e_par * u2 : -r->e_par * lg_log(u2);
  double sref;
  if (r->s_reading == 1)
    sref = lg_exp(s * LG_LN10 - LG_C2 * e / r->T_ref) * (-lg_expm1(-LG_C2 * v / r->T_ref));
  else
    sref = lg_exp(s * LG_LN10);
  *nu = v;
  *S = sref;
  *E = e;
  *g = r->g_lo + (r->g_hi - r->g_lo) * u3;
  *n = r->n_lo + (r->n_hi - r->n_lo) * u4;
}

/* nu of line i only (cheap pre-selection of windows) */
LG_FN double lg_line_nu(const lg_recipe* r, uint64_t seed, uint64_t i) {
  double u0 = lg_uniform(seed, i, 0);
  return r->nu_law == 1 ? r->nu_hi * (u0 * u0) : r->nu_lo + (r->nu_hi - r->nu_lo) * u0;
}
#endif
