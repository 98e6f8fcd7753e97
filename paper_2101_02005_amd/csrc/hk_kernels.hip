// HIP kernels of the line-by-line opacity hot path for gfx950 (MI355X).
//
//   validate / keys / radix passes / gather : binning of the line list along nu
//                                            (the paper sorts line quantities along nu,
//                                            Sec. 2.4.3 step 3)
//   prep      : per temperature, S(T) and gamma_ref (T_ref/T)^n per line (Sec. 2.4.3
//               step 2; eqs. S1, alphaD; ExoMol Lorentz width of Sec. 2.2)
//   worklist  : per grid tile, the range of binned lines within the cutting length
//               (Sec. 2.4.4, wavenumber limits of line blocks) and its split into work items
//   voigt     : persistent tile-owner kernel; each workgroup owns a tile of grid points,
//               stages batches of lines in LDS and accumulates S V per point with
//               compensated FP32 sums (Sec. 2.4.4 tiling of the nu-line plane, redesigned)
//   combine   : fixed-order merge of the partial tiles of heavy tiles
//
// No floating-point atomics are used; every sum runs in a fixed order, so results are
// bitwise reproducible for a fixed tuning.
#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdint>

#include "hk_internal.h"

namespace hk {

__constant__ double c_weid[kWeidN];  // Weideman (1994) coefficients a_1..a_N (host-computed)
__constant__ double c_weidL;         // its scale L = sqrt(N / sqrt 2)

// grid point nu_j = nu_start + j dnu: a rounded product, then a rounded sum (no FMA)
__device__ __forceinline__ double grid_nu(double nu_start, double dnu, int64_t j) {
  return __dadd_rn(nu_start, __dmul_rn((double)j, dnu));
}

// Inclusive grid range of |nu_j - nu0| <= cut, evaluated exactly as defined in FP64.
// nu_j - nu0 is non-decreasing in j, so the range is contiguous; the ceil/floor candidates
// lie within two points of the true bounds and are refined by the predicate itself.
__device__ __forceinline__ void cut_range(double nu0, double nu_start, double dnu, int64_t n,
                                          double cut, int64_t& lo, int64_t& hi) {
  if (isinf(cut)) { lo = 0; hi = n - 1; return; }
  double a = ceil((nu0 - cut - nu_start) / dnu) - 2.0;
  double b = floor((nu0 + cut - nu_start) / dnu) + 2.0;
  if (a < 0.0) a = 0.0;
  if (b > (double)(n - 1)) b = (double)(n - 1);
  if (!(a <= b)) { lo = 0; hi = -1; return; }
  int64_t ia = (int64_t)a, ib = (int64_t)b;
  for (int it = 0; it < 8 && ia <= ib && !(fabs(__dsub_rn(grid_nu(nu_start, dnu, ia), nu0)) <= cut); ++it) ++ia;
  for (int it = 0; it < 8 && ib >= ia && !(fabs(__dsub_rn(grid_nu(nu_start, dnu, ib), nu0)) <= cut); ++it) --ib;
  lo = ia;
  hi = ib;
}

__device__ __forceinline__ uint32_t bin_key(double v, const KeyMap& km) {
  double f = floor((v - km.numin) * km.scale);
  if (!(f > 0.0)) return 0u;
  if (f >= (double)km.kmax) return km.kmax;
  return (uint32_t)f;
}

// ------------------------------------------------------------------------- binning
__global__ void k_validate_init(unsigned long long* mm, int* flags) {
  mm[0] = ~0ull;
  mm[1] = 0ull;
  flags[0] = 0;
}

__global__ __launch_bounds__(kThreads) void k_validate(const double* __restrict__ nu,
    const double* __restrict__ S, const double* __restrict__ E, const double* __restrict__ g,
    const double* __restrict__ n, int64_t N, unsigned long long* mm, int* flags) {
  __shared__ unsigned long long smin[kThreads], smax[kThreads];
  __shared__ int sbad;
  if (threadIdx.x == 0) sbad = 0;
  unsigned long long lmin = ~0ull, lmax = 0ull;
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double v = nu[i];
    const bool ok = (v > 0.0) && isfinite(v) && (S[i] >= 0.0) && isfinite(S[i]) && isfinite(E[i]) &&
                    (g[i] >= 0.0) && isfinite(g[i]) && isfinite(n[i]);
    if (!ok) { bad = 1; continue; }
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);  // v > 0: order-preserving
    lmin = b < lmin ? b : lmin;
    lmax = b > lmax ? b : lmax;
  }
  smin[threadIdx.x] = lmin;
  smax[threadIdx.x] = lmax;
  __syncthreads();
  if (bad) atomicOr(&sbad, 1);
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      smin[threadIdx.x] = smin[threadIdx.x + s] < smin[threadIdx.x] ? smin[threadIdx.x + s] : smin[threadIdx.x];
      smax[threadIdx.x] = smax[threadIdx.x + s] > smax[threadIdx.x] ? smax[threadIdx.x + s] : smax[threadIdx.x];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicMin(&mm[0], smin[0]);
    atomicMax(&mm[1], smax[0]);
    if (sbad) atomicOr(flags, 1);
  }
}

__global__ void k_keys(const double* __restrict__ nu, int64_t N, KeyMap km, uint32_t* __restrict__ keys,
                       int32_t* __restrict__ vals) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  keys[i] = bin_key(nu[i], km);
  vals[i] = (int32_t)i;
}

// Per-block digit histogram: hist[d * G + b].
__global__ __launch_bounds__(kThreads) void k_radix_hist(const uint32_t* __restrict__ kin, int64_t N,
                                                         int shift, uint32_t* __restrict__ hist) {
  __shared__ uint32_t cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortBlock;
  for (int r = 0; r < kSortItems; ++r) {
    int64_t i = base + (int64_t)r * kThreads + threadIdx.x;
    if (i < N) atomicAdd(&cnt[(kin[i] >> shift) & 255u], 1u);  // integer: order-independent
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = cnt[threadIdx.x];
}

// Exclusive scan of one digit's per-block counts (one workgroup per digit); total -> dig_tot[d].
__global__ __launch_bounds__(1024) void k_radix_scan(uint32_t* __restrict__ hist, int G,
                                                     uint32_t* __restrict__ dig_tot) {
  __shared__ uint32_t s[1024];
  __shared__ uint32_t carry;
  uint32_t* h = hist + (int64_t)blockIdx.x * G;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int c0 = 0; c0 < G; c0 += 1024) {
    int i = c0 + threadIdx.x;
    uint32_t v = i < G ? h[i] : 0u;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      uint32_t t = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0u;
      __syncthreads();
      s[threadIdx.x] += t;
      __syncthreads();
    }
    uint32_t incl = s[threadIdx.x];
    if (i < G) h[i] = carry + incl - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry += incl;
    __syncthreads();
  }
  if (threadIdx.x == 0) dig_tot[blockIdx.x] = carry;
}

// Stable scatter: keys of block b keep their order within each digit.
__global__ __launch_bounds__(kThreads) void k_radix_scatter(const uint32_t* __restrict__ kin,
    const int32_t* __restrict__ vin, uint32_t* __restrict__ kout, int32_t* __restrict__ vout, int64_t N,
    int shift, const uint32_t* __restrict__ hist, const uint32_t* __restrict__ dig_tot) {
  __shared__ uint32_t base[256];
  __shared__ uint32_t wcnt[kWavesPerWG][256];
  __shared__ uint32_t scan[256];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // digit start = (sum of smaller digits' totals) + (this block's offset inside the digit)
  scan[tid] = dig_tot[tid];
  for (int i = 0; i < kWavesPerWG; ++i) wcnt[i][tid] = 0;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    uint32_t t = tid >= off ? scan[tid - off] : 0u;
    __syncthreads();
    scan[tid] += t;
    __syncthreads();
  }
  base[tid] = scan[tid] - dig_tot[tid] + hist[(int64_t)tid * gridDim.x + blockIdx.x];
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t b0 = (int64_t)blockIdx.x * kSortBlock;
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t i = b0 + (int64_t)r * kThreads + tid;
    const bool valid = i < N;
    const uint32_t key = valid ? kin[i] : 0u;
    const uint32_t d = (key >> shift) & 255u;
    uint64_t peers = __ballot(valid);
    for (int bit = 0; bit < 8; ++bit) {
      const bool on = (d >> bit) & 1u;
      const uint64_t m = __ballot(on);
      peers &= on ? m : ~m;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    if (valid && rank == 0) wcnt[wv][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t o = base[d] + rank;
      for (int w = 0; w < wv; ++w) o += wcnt[w][d];
      kout[o] = key;
      vout[o] = vin[i];
    }
    uint32_t add = 0;
    for (int w = 0; w < kWavesPerWG; ++w) add += wcnt[w][tid];
    __syncthreads();
    base[tid] += add;
    for (int w = 0; w < kWavesPerWG; ++w) wcnt[w][tid] = 0;
    __syncthreads();
  }
}

__global__ void k_gather(const int32_t* __restrict__ perm, int64_t N, const double* __restrict__ nu,
                         const double* __restrict__ S, const double* __restrict__ E,
                         const double* __restrict__ g, const double* __restrict__ n,
                         double* __restrict__ onu, double* __restrict__ oS, double* __restrict__ oE,
                         double* __restrict__ og, double* __restrict__ on) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int32_t s = perm[i];
  onu[i] = nu[s];
  oS[i] = S[s];
  oE[i] = E[s];
  og[i] = g[s];
  on[i] = n[s];
}

// ---------------------------------------------------------------------------- prep
// S(T) = S_ref Q(T_ref)/Q(T) exp(c2 E''(1/T_ref - 1/T)) (1-e^{-c2 nu/T})/(1-e^{-c2 nu/T_ref})
// (eq. S1 with S' eliminated through S(T_ref) = S_ref), and gamma_ref (T_ref/T)^n; FP64.
__global__ __launch_bounds__(kThreads) void k_prep(PrepArgs a, float* __restrict__ S_T,
                                                   float* __restrict__ gT, double* __restrict__ S64,
                                                   double* __restrict__ a64, double* __restrict__ g64) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.N) return;
  double Sref, gref, nexp;
  if (a.ovr_S || a.ovr_g || a.ovr_n) {
    const int32_t c = a.perm[i];
    Sref = a.ovr_S ? a.ovr_S[c] : a.Sref[i];
    gref = a.ovr_g ? a.ovr_g[c] : a.gref[i];
    nexp = a.ovr_n ? a.ovr_n[c] : a.nexp[i];
  } else {
    Sref = a.Sref[i];
    gref = a.gref[i];
    nexp = a.nexp[i];
  }
  const double v = a.nu[i];
  const double stim = expm1(-a.c2_over_T * v) / expm1(-a.c2_over_Tref * v);
  const double S = Sref * a.q_ratio * exp(a.c2E_coef * a.E[i]) * stim;
  const double g = gref * exp(nexp * a.log_tr);
  if (S_T) S_T[i] = (float)S;
  if (gT) gT[i] = (float)g;
  if (S64) S64[a.perm[i]] = S;
  if (a64) a64[a.perm[i]] = v * a.beta;
  if (g64) g64[a.perm[i]] = g * a.pfac;
}

struct PairPack {
  PairDesc p[kFillPairs];
  int count;
};

__global__ void k_fill_pairs(PairPack pk, PairDesc* dst) {
  if ((int)threadIdx.x < pk.count) dst[threadIdx.x] = pk.p[threadIdx.x];
}

// ------------------------------------------------------------------------ worklist
__device__ __forceinline__ int find_pair(const PairDesc* pairs, int n_pairs, int g) {
  int lo = 0, hi = n_pairs - 1;
  while (lo < hi) {
    int m = (lo + hi + 1) >> 1;
    if (pairs[m].tile_base <= g) lo = m; else hi = m - 1;
  }
  return lo;
}

__global__ void k_worklist(const uint32_t* __restrict__ keys, int64_t N, KeyMap km, double numin, double numax,
                           const PairDesc* __restrict__ pairs, int n_pairs, int n_tiles_total,
                           int tile_w, double cut, int chunk, int32_t* __restrict__ lo_out,
                           int32_t* __restrict__ hi_out, int32_t* __restrict__ nc_out) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_tiles_total) return;
  const PairDesc pd = pairs[find_pair(pairs, n_pairs, g)];
  const int64_t t = g - pd.tile_base;
  const int64_t j0 = t * tile_w;
  const int64_t j1 = (j0 + tile_w < pd.n ? j0 + tile_w : pd.n) - 1;
  int64_t lo = 0, hi = N;
  if (!isinf(cut)) {
    const double va = __dsub_rn(grid_nu(pd.nu_start, pd.dnu, j0), cut);
    const double vb = __dadd_rn(grid_nu(pd.nu_start, pd.dnu, j1), cut);
    if (vb < numin || va > numax) { lo_out[g] = 0; hi_out[g] = 0; nc_out[g] = 1; return; }
    uint32_t ka = bin_key(va, km), kb = bin_key(vb, km);
    ka = ka > 0 ? ka - 1 : 0;
    kb = kb < km.kmax ? kb + 1 : km.kmax;
    int64_t a = 0, b = N;  // first key >= ka
    while (a < b) { int64_t m = (a + b) >> 1; if (keys[m] < ka) a = m + 1; else b = m; }
    lo = a;
    b = N;                 // first key > kb
    while (a < b) { int64_t m = (a + b) >> 1; if (keys[m] <= kb) a = m + 1; else b = m; }
    hi = a;
  }
  const int64_t cnt = hi - lo;
  int64_t nc = (cnt + chunk - 1) / chunk;
  lo_out[g] = (int32_t)lo;
  hi_out[g] = (int32_t)hi;
  nc_out[g] = (int32_t)(nc > 0 ? nc : 1);
}

// item_base = exclusive scan of nc; item_base[n] = total; also resets the item dispenser.
__global__ __launch_bounds__(1024) void k_item_scan(const int32_t* __restrict__ nc, int n,
                                                    int32_t* __restrict__ item_base, int* counter) {
  __shared__ int32_t s[1024];
  __shared__ int32_t carry;
  if (threadIdx.x == 0) { carry = 0; counter[0] = 0; }
  __syncthreads();
  for (int c0 = 0; c0 < n; c0 += 1024) {
    const int i = c0 + threadIdx.x;
    const int32_t v = i < n ? nc[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      int32_t t = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0;
      __syncthreads();
      s[threadIdx.x] += t;
      __syncthreads();
    }
    const int32_t incl = s[threadIdx.x];
    if (i < n) item_base[i] = carry + incl - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry += incl;
    __syncthreads();
  }
  if (threadIdx.x == 0) item_base[n] = carry;
}

// ----------------------------------------------------------------- Voigt profile
// Re w(x + iy), y >= 0, by J.A.C. Weideman's rational approximation ("Computation of the
// complex error function", SIAM J. Numer. Anal. 31 (1994) 1497-1518) with N = kWeidN terms:
// w = 2 p(Z)/(L - iz)^2 + (1/sqrt(pi))/(L - iz), Z = (L + iz)/(L - iz), in FP64.
__device__ __forceinline__ double weideman_re(double x, double y) {
  const double L = c_weidL;
  const double dr = L + y, di = -x;  // L - iz
  const double nr = L - y, ni = x;   // L + iz
  const double inv = 1.0 / (dr * dr + di * di);
  const double Zr = (nr * dr + ni * di) * inv;
  const double Zi = (ni * dr - nr * di) * inv;
  double pr = c_weid[kWeidN - 1], pi = 0.0;
#pragma unroll
  for (int m = kWeidN - 2; m >= 0; --m) {
    const double t = fma(pr, Zr, fma(-pi, Zi, c_weid[m]));
    pi = fma(pr, Zi, pi * Zr);
    pr = t;
  }
  const double ur = dr * inv, ui = -di * inv;        // 1/(L - iz)
  const double vr = ur * ur - ui * ui, vi = 2.0 * ur * ui;  // 1/(L - iz)^2
  return 2.0 * (pr * vr - pi * vi) + 0.56418958354775628695 * ur;
}

// Line record layout in LDS (structure of arrays, one entry per staged line):
//   F0 = (dh, jt, dnh, gh): offset delta/sqrt(s), reference index - tile start, dnu/sqrt(s),
//        gamma^2/s, with s = max(alpha^2, gamma^2)
//   F1 = (Ah, lo_rel, hi_rel, ampc): S gamma/(pi s), cut bounds relative to the reference
//        index, S/(sqrt(pi) alpha)
//   K2, K3, K4a/K4b: Ah * series coefficients for orders 2, 3, 4
//   D64, IA, Y: FP64 offset, 1/alpha, gamma/alpha for the core
//   code[w]: per wave, 4 bits per slot (bits 0-2 path: 0 skip, 1-4 series order, 5 core;
//            bit 3: the slot straddles a cut bound)
struct LineLDS {
  float4 F0[kLB];
  float4 F1[kLB];
  float2 K2[kLB];
  float4 K3[kLB];
  float4 K4a[kLB];
  float2 K4b[kLB];
  double D64[kLB];
  double IA[kLB];
  double Y[kLB];
  uint32_t code[kWavesPerWG][kLB];
};

// Far-wing series of the Voigt profile in q = 1/(D^2 + gamma^2), from the asymptotic
// expansion w(z) ~ (i/sqrt(pi)) sum_k (2k-1)!!/(2^k z^(2k+1)): with t = alpha^2 q and
// u = gamma^2 q,  V = (S gamma/pi) q sum_{k<K} a_k t^k P_k(u), a_k = (2k-1)!!/2^k,
// P_k(u) = U_2k(sqrt(1-u)) (Chebyshev polynomials of the second kind) expanded in u.
// Truncated at order K its relative error is below 2e-6 for |z| above zK[K-1].
// Written as a polynomial in qh = s q (s = max(alpha^2, gamma^2), so qh <= 1) with
// coefficients C_M = sum_{k+l=M, k<K} a_k f_{k,l} (alpha^2/s)^k (-gamma^2/s)^l.
__device__ __forceinline__ void series_coeffs(int K, double a2, double g2, double* C) {
  // f_{k,l}: coefficients of P_k(u) = sum_l f_{k,l} (-u)^l
  const double f[4][4] = {{1, 0, 0, 0}, {3, 4, 0, 0}, {5, 20, 16, 0}, {7, 56, 112, 64}};
  const double ak[4] = {1.0, 0.5, 0.75, 1.875};
  for (int M = 1; M <= 2 * K - 2; ++M) {
    double c = 0.0;
    for (int k = (M + 1) / 2; k <= M && k < K; ++k) {
      const int l = M - k;
      if (l > k) continue;
      double term = ak[k] * f[k][l];
      for (int r = 0; r < k; ++r) term *= a2;
      for (int r = 0; r < l; ++r) term *= -g2;
      c += term;
    }
    C[M - 1] = c;
  }
}

template <int P>
__device__ __forceinline__ void kahan_flush(float (&part)[P], float (&s)[P], float (&c)[P]) {
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const float y = part[p] - c[p];
    const float t = s[p] + y;
    c[p] = (t - s[p]) - y;
    s[p] = t;
    part[p] = 0.0f;
  }
}

// Stage one line for a tile: every tile-dependent quantity the waves need, and for each
// wave a 4-bit path code per 64-point slot. Lines that do not reach the tile get code 0.
template <int P>
__device__ __forceinline__ void stage_line(LineLDS& L, int tid, double nu0, double S, double gTv,
                                           const PairDesc& pd, double cut, const double* zK,
                                           int64_t tile0, uint32_t (&codes)[kWavesPerWG]) {
  constexpr int W = kWavesPerWG * kWave * P;
  const double gam = gTv * pd.pfac;
  const double alpha = nu0 * pd.beta;
  int64_t jlo, jhi;
  cut_range(nu0, pd.nu_start, pd.dnu, pd.n, cut, jlo, jhi);
  const int64_t tile1 = tile0 + W - 1;
  if (!(S > 0.0) || jlo > jhi || jhi < tile0 || jlo > tile1) return;
  const double a2 = alpha * alpha, g2 = gam * gam;
  const double sc = a2 > g2 ? a2 : g2;
  const double rs = 1.0 / sqrt(sc);
  if (!(sc > 0.0) || !isfinite(rs)) return;
  const double cpos = (nu0 - pd.nu_start) / pd.dnu;  // line centre in grid units
  double jr = rint(cpos);
  jr = jr < 0.0 ? 0.0 : (jr > (double)(pd.n - 1) ? (double)(pd.n - 1) : jr);
  const int64_t jref = (int64_t)jr;  // grid point nearest the centre, clamped to the grid
  const double delta = __dsub_rn(grid_nu(pd.nu_start, pd.dnu, jref), nu0);
  const double Ah = S * gam / (M_PI * sc);
  L.F0[tid] = make_float4((float)(delta * rs), (float)(jref - tile0), (float)(pd.dnu * rs), (float)(g2 / sc));
  L.F1[tid] = make_float4((float)Ah, (float)(jlo - jref), (float)(jhi - jref),
                          (float)(S / (1.7724538509055160273 * alpha)));
  double C[6];
  series_coeffs(2, a2 / sc, g2 / sc, C);
  L.K2[tid] = make_float2((float)(Ah * C[0]), (float)(Ah * C[1]));
  series_coeffs(3, a2 / sc, g2 / sc, C);
  L.K3[tid] = make_float4((float)(Ah * C[0]), (float)(Ah * C[1]), (float)(Ah * C[2]), (float)(Ah * C[3]));
  series_coeffs(4, a2 / sc, g2 / sc, C);
  L.K4a[tid] = make_float4((float)(Ah * C[0]), (float)(Ah * C[1]), (float)(Ah * C[2]), (float)(Ah * C[3]));
  L.K4b[tid] = make_float2((float)(Ah * C[4]), (float)(Ah * C[5]));
  L.D64[tid] = delta;
  L.IA[tid] = 1.0 / alpha;
  L.Y[tid] = gam / alpha;
  // zone K: points with |z| < zK[K], i.e. |nu_j - nu0| < sqrt(zK^2 alpha^2 - gamma^2); as a
  // range of slots (slot sigma covers points tile0 + 64 sigma .. + 63), widened slightly
  int zlo[kKmax], zhi[kKmax];
  const double crel = cpos - (double)tile0;
  for (int K = 0; K < kKmax; ++K) {
    const double zz = zK[K] * alpha;
    const double h2 = zz * zz - g2;
    if (h2 <= 0.0) { zlo[K] = 1; zhi[K] = 0; continue; }
    const double h = sqrt(h2) / pd.dnu * (1.0 + 1e-6) + 1e-3;
    double lo_s = ceil((crel - h - 63.0) / 64.0), hi_s = floor((crel + h) / 64.0);
    lo_s = lo_s < -1.0 ? -1.0 : (lo_s > 1e6 ? 1e6 : lo_s);
    hi_s = hi_s < -1.0 ? -1.0 : (hi_s > 1e6 ? 1e6 : hi_s);
    zlo[K] = (int)lo_s;
    zhi[K] = (int)hi_s;
  }
  for (int w = 0; w < kWavesPerWG; ++w) {
    uint32_t cw = 0u;
    for (int p = 0; p < P; ++p) {
      const int sg = w * P + p;
      const int64_t s0 = tile0 + (int64_t)sg * kWave, s1 = s0 + kWave - 1;
      if (s1 < jlo || s0 > jhi) continue;
      uint32_t path = 1u;
      for (int K = 0; K < kKmax; ++K) path += (sg >= zlo[K] && sg <= zhi[K]) ? 1u : 0u;
      const uint32_t msk = (s0 >= jlo && s1 <= jhi) ? 0u : 8u;
      cw |= (path | msk) << (4 * p);
    }
    codes[w] = cw;
  }
}

template <int P>
__global__ __launch_bounds__(kThreads) void k_voigt(VoigtArgs a) {
  constexpr int W = kWavesPerWG * kWave * P;  // tile width in grid points
  __shared__ LineLDS L;
  __shared__ int sItem, sTile, sPair;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int total = a.item_base[a.n_tiles_total];

  for (;;) {
    if (tid == 0) {
      const int it = atomicAdd(a.counter, 1);
      sItem = it;
      if (it < total) {
        int lo = 0, hi = a.n_tiles_total - 1;  // last tile with item_base <= it
        while (lo < hi) {
          const int m = (lo + hi + 1) >> 1;
          if (a.item_base[m] <= it) lo = m; else hi = m - 1;
        }
        sTile = lo;
        sPair = find_pair(a.pairs, a.n_pairs, lo);
      }
    }
    __syncthreads();
    const int it = sItem;
    if (it >= total) break;
    const int g = sTile;
    const PairDesc pd = a.pairs[sPair];
    const int chunk_idx = it - a.item_base[g];
    const int nc = a.tile_nc[g];
    const int64_t tile0 = (int64_t)(g - pd.tile_base) * W;
    const int64_t line_lo = (int64_t)a.tile_lo[g] + (int64_t)chunk_idx * a.chunk;
    int64_t line_hi = line_lo + a.chunk;
    if (line_hi > a.tile_hi[g]) line_hi = a.tile_hi[g];
    const float* __restrict__ S_T = a.S_T + (int64_t)pd.tidx * a.N;
    const float* __restrict__ gT = a.gT + (int64_t)pd.tidx * a.N;

    float jl[P], s[P], cc[P], part[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
      jl[p] = (float)(wv * kWave * P + p * kWave + lane);
      s[p] = 0.0f;
      cc[p] = 0.0f;
      part[p] = 0.0f;
    }

    for (int64_t b = line_lo; b < line_hi; b += kLB) {
      // ---- stage one batch of lines: one thread per line, FP64 where it matters
      {
        const int64_t li = b + tid;
        uint32_t codes[kWavesPerWG] = {0u, 0u, 0u, 0u};
        if (li < line_hi)
          stage_line<P>(L, tid, a.nu[li], (double)S_T[li], (double)gT[li], pd, a.cut, a.zK, tile0, codes);
        for (int w = 0; w < kWavesPerWG; ++w) L.code[w][tid] = codes[w];
      }
      __syncthreads();

      // ---- accumulate: this wave's slots over the staged lines, in staging order
      const int nb = (int)((line_hi - b) < kLB ? (line_hi - b) : kLB);
      for (int l = 0; l < nb; ++l) {
        const uint32_t code = __builtin_amdgcn_readfirstlane(L.code[wv][l]);
        if (code != 0u) {
          const float4 f0 = L.F0[l];
          const float4 f1 = L.F1[l];
          uint32_t core_slots = 0u;
#pragma unroll
          for (int p = 0; p < P; ++p) {
            const uint32_t cs = (code >> (4 * p)) & 15u;
            if (cs == 0u) continue;
            const uint32_t path = cs & 7u;
            if (path == 5u) { core_slots |= 1u << p; continue; }
            const float kf = jl[p] - f0.y;
            const float D = __builtin_fmaf(kf, f0.z, f0.x);
            const float R = __builtin_fmaf(D, D, f0.w);
            const float q = __builtin_amdgcn_rcpf(R);
            float t;
            if (path == 1u) {
              t = f1.x;
            } else if (path == 2u) {
              const float2 c = L.K2[l];
              t = __builtin_fmaf(c.y, q, c.x);
              t = __builtin_fmaf(t, q, f1.x);
            } else if (path == 3u) {
              const float4 c = L.K3[l];
              t = __builtin_fmaf(c.w, q, c.z);
              t = __builtin_fmaf(t, q, c.y);
              t = __builtin_fmaf(t, q, c.x);
              t = __builtin_fmaf(t, q, f1.x);
            } else {
              const float4 c = L.K4a[l];
              const float2 e = L.K4b[l];
              t = __builtin_fmaf(e.y, q, e.x);
              t = __builtin_fmaf(t, q, c.w);
              t = __builtin_fmaf(t, q, c.z);
              t = __builtin_fmaf(t, q, c.y);
              t = __builtin_fmaf(t, q, c.x);
              t = __builtin_fmaf(t, q, f1.x);
            }
            if (cs & 8u) {
              const bool in = (kf >= f1.y) && (kf <= f1.z);
              part[p] = in ? __builtin_fmaf(t, q, part[p]) : part[p];
            } else {
              part[p] = __builtin_fmaf(t, q, part[p]);
            }
          }
          // core slots: FP64 rational approximation for every lane of the slot
          while (core_slots) {
            const int p = __builtin_ctz(core_slots);
            core_slots &= core_slots - 1u;
            const float kf = (float)(wv * kWave * P + p * kWave + lane) - f0.y;
            const double D = fma((double)kf, pd.dnu, L.D64[l]);
            const float v = f1.w * (float)weideman_re(D * L.IA[l], L.Y[l]);
            const bool msk = ((code >> (4 * p)) & 8u) != 0u;
            const bool in = !msk || ((kf >= f1.y) && (kf <= f1.z));
            const float add = in ? v : 0.0f;
#pragma unroll
            for (int q2 = 0; q2 < P; ++q2)
              if (q2 == p) part[q2] += add;
          }
        }
        if ((l & 15) == 15) kahan_flush<P>(part, s, cc);
      }
      kahan_flush<P>(part, s, cc);
      __syncthreads();
    }

    // ---- output: the tile directly, or this chunk's partial tile
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int local = wv * kWave * P + p * kWave + lane;
      const float v = s[p] - cc[p];
      if (nc == 1) {
        if (tile0 + local < pd.n) a.k[pd.out_off + tile0 + local] = v;
      } else {
        a.partial[((int64_t)(a.item_base[g] + chunk_idx)) * W + local] = v;
      }
    }
    __syncthreads();
  }
}

// Fixed-order (chunk 0, 1, ...) FP64 sum of the partial tiles of multi-chunk tiles;
// one workgroup per tile.
template <int P>
__global__ __launch_bounds__(kThreads) void k_combine(VoigtArgs a) {
  constexpr int W = kWavesPerWG * kWave * P;
  const int g = blockIdx.x;
  const int nc = a.tile_nc[g];
  if (nc <= 1) return;
  const PairDesc pd = a.pairs[find_pair(a.pairs, a.n_pairs, g)];
  const int64_t tile0 = (int64_t)(g - pd.tile_base) * W;
  const int base = a.item_base[g];
  for (int local = threadIdx.x; local < W; local += kThreads) {
    if (tile0 + local >= pd.n) continue;
    double acc = 0.0;
    for (int c = 0; c < nc; ++c) acc += (double)a.partial[(int64_t)(base + c) * W + local];
    a.k[pd.out_off + tile0 + local] = (float)acc;
  }
}

__global__ void k_cut_bounds(const double* __restrict__ nu, const int32_t* __restrict__ perm, int64_t N,
                             double nu_start, double dnu, int64_t n, double cut, int32_t* jlo,
                             int32_t* jhi) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  int64_t lo, hi;
  cut_range(nu[i], nu_start, dnu, n, cut, lo, hi);
  jlo[perm[i]] = (int32_t)lo;
  jhi[perm[i]] = (int32_t)hi;
}

// ----------------------------------------------------------------- launch wrappers
static inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

hipError_t launch_validate(const double* nu, const double* S, const double* E, const double* g,
                           const double* n, int64_t N, unsigned long long* mm, int* flags, hipStream_t st) {
  hipLaunchKernelGGL(k_validate_init, dim3(1), dim3(1), 0, st, mm, flags);
  int64_t blocks = blocks_for(N, kThreads);
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_validate, dim3((unsigned)blocks), dim3(kThreads), 0, st, nu, S, E, g, n, N, mm, flags);
  return hipGetLastError();
}

hipError_t launch_keys(const double* nu, int64_t N, KeyMap km, uint32_t* keys, int32_t* vals, hipStream_t st) {
  hipLaunchKernelGGL(k_keys, dim3(blocks_for(N, kThreads)), dim3(kThreads), 0, st, nu, N, km, keys, vals);
  return hipGetLastError();
}

hipError_t launch_radix_pass(const uint32_t* kin, const int32_t* vin, uint32_t* kout, int32_t* vout,
                             int64_t N, int shift, uint32_t* hist, uint32_t* dig_tot, hipStream_t st) {
  const unsigned G = blocks_for(N, kSortBlock);
  hipLaunchKernelGGL(k_radix_hist, dim3(G), dim3(kThreads), 0, st, kin, N, shift, hist);
  hipLaunchKernelGGL(k_radix_scan, dim3(256), dim3(1024), 0, st, hist, (int)G, dig_tot);
  hipLaunchKernelGGL(k_radix_scatter, dim3(G), dim3(kThreads), 0, st, kin, vin, kout, vout, N, shift,
                     (const uint32_t*)hist, (const uint32_t*)dig_tot);
  return hipGetLastError();
}

hipError_t launch_gather(const int32_t* perm, int64_t N, const double* nu, const double* S, const double* E,
                         const double* g, const double* n, double* onu, double* oS, double* oE, double* og,
                         double* on, hipStream_t st) {
  hipLaunchKernelGGL(k_gather, dim3(blocks_for(N, kThreads)), dim3(kThreads), 0, st, perm, N, nu, S, E, g, n,
                     onu, oS, oE, og, on);
  return hipGetLastError();
}

hipError_t launch_prep(const PrepArgs& a, float* S_T, float* gT, double* S64, double* a64, double* g64,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_prep, dim3(blocks_for(a.N, kThreads)), dim3(kThreads), 0, st, a, S_T, gT, S64, a64, g64);
  return hipGetLastError();
}

hipError_t launch_fill_pairs(const PairDesc* host_pairs, int count, PairDesc* dst, hipStream_t st) {
  for (int c0 = 0; c0 < count; c0 += kFillPairs) {
    PairPack pk;
    pk.count = count - c0 < kFillPairs ? count - c0 : kFillPairs;
    for (int i = 0; i < pk.count; ++i) pk.p[i] = host_pairs[c0 + i];
    hipLaunchKernelGGL(k_fill_pairs, dim3(1), dim3(64), 0, st, pk, dst + c0);
  }
  return hipGetLastError();
}

hipError_t launch_worklist(const uint32_t* keys, int64_t N, KeyMap km, double numin, double numax,
                           const PairDesc* pairs, int n_pairs,
                           int n_tiles_total, int tile_w, double cut, int chunk, int32_t* lo, int32_t* hi,
                           int32_t* nc, hipStream_t st) {
  hipLaunchKernelGGL(k_worklist, dim3(blocks_for(n_tiles_total, kThreads)), dim3(kThreads), 0, st, keys, N, km,
                     numin, numax, pairs, n_pairs, n_tiles_total, tile_w, cut, chunk, lo, hi, nc);
  return hipGetLastError();
}

hipError_t launch_item_scan(const int32_t* nc, int n_tiles_total, int32_t* item_base, int* counter,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_item_scan, dim3(1), dim3(1024), 0, st, nc, n_tiles_total, item_base, counter);
  return hipGetLastError();
}

hipError_t launch_voigt(const VoigtArgs& a, int slots, int grid, hipStream_t st) {
  if (slots == 8) hipLaunchKernelGGL(k_voigt<8>, dim3(grid), dim3(kThreads), 0, st, a);
  else if (slots == 4) hipLaunchKernelGGL(k_voigt<4>, dim3(grid), dim3(kThreads), 0, st, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_combine(const VoigtArgs& a, int slots, hipStream_t st) {
  dim3 grid((unsigned)a.n_tiles_total);
  if (slots == 8) hipLaunchKernelGGL(k_combine<8>, grid, dim3(kThreads), 0, st, a);
  else if (slots == 4) hipLaunchKernelGGL(k_combine<4>, grid, dim3(kThreads), 0, st, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_cut_bounds(const double* nu, const int32_t* perm, int64_t N, double nu_start, double dnu,
                             int64_t n, double cut, int32_t* jlo, int32_t* jhi, hipStream_t st) {
  hipLaunchKernelGGL(k_cut_bounds, dim3(blocks_for(N, kThreads)), dim3(kThreads), 0, st, nu, perm, N, nu_start,
                     dnu, n, cut, jlo, jhi);
  return hipGetLastError();
}

int voigt_max_blocks_per_cu(int slots) {
  int nb = 0;
  if (slots == 8) (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_voigt<8>, kThreads, 0);
  else (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_voigt<4>, kThreads, 0);
  return nb > 0 ? nb : 1;
}

hipError_t upload_weideman(const double* coef, double L) {
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_weid), coef, sizeof(double) * kWeidN);
  if (e != hipSuccess) return e;
  return hipMemcpyToSymbol(HIP_SYMBOL(c_weidL), &L, sizeof(double));
}

}  // namespace hk
