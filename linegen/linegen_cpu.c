/* Host twin of the synthetic line generator (see linegen_core.h). OpenMP-parallel. */
#include "linegen_core.h"
#include <stddef.h>

void lg_generate(const lg_recipe* r, uint64_t seed, int64_t i0, int64_t count,
                 double* nu, double* S, double* E, double* g, double* n) {
  #pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < count; ++k)
    lg_line(r, seed, (uint64_t)(i0 + k), nu + k, S + k, E + k, g + k, n + k);
}

/* Lines among [0, N) whose nu lies in [nu_lo, nu_hi); writes up to cap of them in index
 * order and returns the total count (may exceed cap: then only the first cap are written). */
int64_t lg_select(const lg_recipe* r, uint64_t seed, int64_t N, double nu_lo, double nu_hi,
                  int64_t cap, int64_t* idx, double* nu, double* S, double* E, double* g, double* n) {
  int64_t total = 0;
  const int64_t block = 1 << 20;
  for (int64_t b0 = 0; b0 < N; b0 += block) {
    int64_t b1 = b0 + block < N ? b0 + block : N;
    for (int64_t i = b0; i < b1; ++i) {
      double v = lg_line_nu(r, seed, (uint64_t)i);
      if (v >= nu_lo && v < nu_hi) {
        if (total < cap) {
          idx[total] = i;
          lg_line(r, seed, (uint64_t)i, nu + total, S + total, E + total, g + total, n + total);
        }
        ++total;
      }
    }
  }
  return total;
}

/* parallel variant of lg_select: per-thread counting then ordered fill */
int64_t lg_select_par(const lg_recipe* r, uint64_t seed, int64_t N, double nu_lo, double nu_hi,
                      int64_t cap, int64_t* idx, double* nu, double* S, double* E, double* g, double* n,
                      int64_t* scratch_counts, int nblocks) {
  /* scratch_counts: nblocks entries */
  int64_t bs = (N + nblocks - 1) / nblocks;
  #pragma omp parallel for schedule(dynamic, 1)
  for (int b = 0; b < nblocks; ++b) {
    int64_t lo = (int64_t)b * bs, hi = lo + bs < N ? lo + bs : N, c = 0;
    for (int64_t i = lo; i < hi; ++i) {
      double v = lg_line_nu(r, seed, (uint64_t)i);
      c += (v >= nu_lo && v < nu_hi);
    }
    scratch_counts[b] = c;
  }
  int64_t total = 0;
  for (int b = 0; b < nblocks; ++b) { int64_t c = scratch_counts[b]; scratch_counts[b] = total; total += c; }
  #pragma omp parallel for schedule(dynamic, 1)
  for (int b = 0; b < nblocks; ++b) {
    int64_t lo = (int64_t)b * bs, hi = lo + bs < N ? lo + bs : N, o = scratch_counts[b];
    for (int64_t i = lo; i < hi; ++i) {
      double v = lg_line_nu(r, seed, (uint64_t)i);
      if (v >= nu_lo && v < nu_hi) {
        if (o < cap) {
          idx[o] = i;
          lg_line(r, seed, (uint64_t)i, nu + o, S + o, E + o, g + o, n + o);
        }
        ++o;
      }
    }
  }
  return total;
}

/* raw uniform draws, for tests of the counter-based generator itself */
void lg_uniforms(uint64_t seed, int64_t i0, int64_t count, int64_t f, double* out) {
  for (int64_t k = 0; k < count; ++k) out[k] = lg_uniform(seed, (uint64_t)(i0 + k), (uint64_t)f);
}

/* helpers exposed for tests of the generator's own exp/log/expm1 */
void lg_math(int which, int64_t count, const double* x, double* y) {
  for (int64_t k = 0; k < count; ++k)
    y[k] = which == 0 ? lg_exp(x[k]) : which == 1 ? lg_expm1(x[k]) : lg_log(x[k]);
}
