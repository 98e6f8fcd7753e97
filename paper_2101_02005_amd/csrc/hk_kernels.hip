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

__constant__ float c_weid32[kWeidN];  // Weideman (1994) coefficients a_1..a_N (host-computed in
__constant__ float c_weidL32;         // FP64, rounded) and the scale L (an FP32 number)
__constant__ double c_weid40[kWeidN40];  // the coefficients of the 40-term form in FP64 (the plinth
__constant__ double c_weid40L;           // values and the line-core pass's FP64 rounds) and its L

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
  flags[1] = 0;
}

// nu > 0 and finite, and its range (the other fields are checked by k_keys, which reads them).
__global__ __launch_bounds__(kThreads) void k_validate(const double* __restrict__ nu, int64_t N,
                                                       unsigned long long* mm, int* flags) {
  __shared__ unsigned long long smin[kThreads], smax[kThreads];
  __shared__ int sbad;
  if (threadIdx.x == 0) sbad = 0;
  unsigned long long lmin = ~0ull, lmax = 0ull;
  int bad = 0;
  auto take = [&](double v) {
    if (!((v > 0.0) && isfinite(v))) { bad = 1; return; }
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);  // v > 0: order-preserving
    lmin = b < lmin ? b : lmin;
    lmax = b > lmax ? b : lmax;
  };
  // grid-stride, four independent loads in flight per thread
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < N; i += 4 * stride) {
    const double v0 = nu[i], v1 = nu[i + stride], v2 = nu[i + 2 * stride], v3 = nu[i + 3 * stride];
    take(v0);
    take(v1);
    take(v2);
    take(v3);
  }
  for (; i < N; i += stride) take(nu[i]);
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

// Bin keys, identity values, and a record-per-line copy of the five fields (so that the
// gather after the sort reads one record, not five scattered words, per line); also checks
// S_ref >= 0, gamma_ref >= 0 and finite E, S_ref, gamma_ref, n (flags[1] = 1 if not).
__global__ __launch_bounds__(kThreads) void k_keys(const double* __restrict__ nu, const double* __restrict__ S,
                                                   const double* __restrict__ E, const double* __restrict__ g,
                                                   const double* __restrict__ n, int64_t N, KeyMap km,
                                                   uint32_t* __restrict__ keys, int32_t* __restrict__ vals,
                                                   double* __restrict__ rec, int* flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool bad = false;
  if (i < N) {
    const double v = nu[i];
    const double Si = S[i], Ei = E[i], gi = g[i], ni = n[i];
    bad = !((Si >= 0.0) && isfinite(Si) && isfinite(Ei) && (gi >= 0.0) && isfinite(gi) && isfinite(ni));
    keys[i] = bin_key(v, km);
    vals[i] = (int32_t)i;
    double* r = rec + 5 * i;
    r[0] = v;
    r[1] = Si;
    r[2] = Ei;
    r[3] = gi;
    r[4] = ni;
  }
  if (__ballot(bad) != 0ull && (threadIdx.x & (kWave - 1)) == 0) atomicOr(flags + 1, 1);
}

// Per-block digit histogram: hist[d * G + b].
__global__ __launch_bounds__(kThreads) void k_radix_hist(const uint32_t* __restrict__ kin, int64_t N,
                                                         int shift, uint32_t* __restrict__ hist) {
  __shared__ uint32_t cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortBlock;
  uint32_t rkey[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t i = base + (int64_t)r * kThreads + threadIdx.x;
    rkey[r] = i < N ? kin[i] : 0u;
  }
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t i = base + (int64_t)r * kThreads + threadIdx.x;
    if (i < N) atomicAdd(&cnt[(rkey[r] >> shift) & 255u], 1u);  // integer: order-independent
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
// Stable scatter of one 8-bit digit: each block orders its keys by digit in LDS (ranks from
// wave ballots, waves and rounds in index order), then writes every digit's run to its global
// place with consecutive threads on consecutive addresses.
__global__ __launch_bounds__(kThreads) void k_radix_scatter(const uint32_t* __restrict__ kin,
    const int32_t* __restrict__ vin, uint32_t* __restrict__ kout, int32_t* __restrict__ vout, int64_t N,
    int shift, const uint32_t* __restrict__ hist, const uint32_t* __restrict__ dig_tot) {
  __shared__ uint32_t sk[kSortBlock];
  __shared__ int32_t sv[kSortBlock];
  __shared__ uint32_t gbase[256];   // global start of this block's run of digit d
  __shared__ uint32_t lstart[256];  // start of digit d in the block's ordered keys
  __shared__ uint32_t run[256];     // keys of digit d placed so far
  __shared__ uint32_t wcnt[kWavesPerWG][256];
  __shared__ uint32_t scan[256];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // hist holds, per digit, the exclusive scan of the blocks' counts (this block's offset inside
  // the digit); this block's own count is the difference to the next block's offset
  const int64_t hb = (int64_t)tid * gridDim.x + blockIdx.x;
  const uint32_t boff = hist[hb];
  const uint32_t mine = (blockIdx.x + 1 < gridDim.x ? hist[hb + 1] : dig_tot[tid]) - boff;
  // global digit starts: scan over digit totals, plus this block's offset inside the digit
  scan[tid] = dig_tot[tid];
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const uint32_t t = tid >= off ? scan[tid - off] : 0u;
    __syncthreads();
    scan[tid] += t;
    __syncthreads();
  }
  gbase[tid] = scan[tid] - dig_tot[tid] + boff;
  __syncthreads();
  // local digit starts: scan of this block's counts
  scan[tid] = mine;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const uint32_t t = tid >= off ? scan[tid - off] : 0u;
    __syncthreads();
    scan[tid] += t;
    __syncthreads();
  }
  lstart[tid] = scan[tid] - mine;
  run[tid] = 0;
  for (int i = 0; i < kWavesPerWG; ++i) wcnt[i][tid] = 0;
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t b0 = (int64_t)blockIdx.x * kSortBlock;
  // every round's key and value are loaded up front (one memory latency, not one per round)
  uint32_t rkey[kSortItems];
  int32_t rval[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t i = b0 + (int64_t)r * kThreads + tid;
    rkey[r] = i < N ? kin[i] : 0u;
    rval[r] = i < N ? vin[i] : 0;
  }
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t i = b0 + (int64_t)r * kThreads + tid;
    const bool valid = i < N;
    const uint32_t key = rkey[r];
    const int32_t val = rval[r];
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
      uint32_t o = lstart[d] + run[d] + rank;
      for (int w = 0; w < wv; ++w) o += wcnt[w][d];
      sk[o] = key;
      sv[o] = val;
    }
    uint32_t add = 0;
    for (int w = 0; w < kWavesPerWG; ++w) add += wcnt[w][tid];
    __syncthreads();
    run[tid] += add;
    for (int w = 0; w < kWavesPerWG; ++w) wcnt[w][tid] = 0;
    __syncthreads();
  }
  const int nvalid = (int)((N - b0) < kSortBlock ? (N - b0) : kSortBlock);
  for (int j = tid; j < nvalid; j += kThreads) {
    const uint32_t key = sk[j];
    const uint32_t d = (key >> shift) & 255u;
    const uint32_t o = gbase[d] + ((uint32_t)j - lstart[d]);
    kout[o] = key;
    vout[o] = sv[j];
  }
}

__global__ void k_gather(const int32_t* __restrict__ perm, int64_t N, const double* __restrict__ rec,
                         double* __restrict__ onu, double* __restrict__ oS, double* __restrict__ oE,
                         double* __restrict__ og, double* __restrict__ on) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double* r = rec + 5 * (int64_t)perm[i];
  onu[i] = r[0];
  oS[i] = r[1];
  oE[i] = r[2];
  og[i] = r[3];
  on[i] = r[4];
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
  // a Boltzmann factor ratio beyond the FP64 range is taken with S_ref inside the exponential
  const double arg = a.c2E_coef * a.E[i];
  const double S = arg < 700.0 ? Sref * a.q_ratio * exp(arg) * stim
                               : (Sref > 0.0 ? exp(log(Sref) + arg) * a.q_ratio * stim : 0.0);
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

// Copies the pair descriptors; also clears the call's status word when given (a kernel, not a
// memset, so that the call can be recorded into a graph).
__global__ void k_fill_pairs(PairPack pk, PairDesc* dst, int* status) {
  if ((int)threadIdx.x < pk.count) dst[threadIdx.x] = pk.p[threadIdx.x];
  if (status && threadIdx.x == 0) *status = 0;
}

// Force a value that is uniform across the wave into scalar registers (its load may have
// been a vector load, e.g. through a pointer the compiler cannot prove unclobbered).
template <typename T>
__device__ __forceinline__ T wave_uniform(const T& v) {
  static_assert(sizeof(T) % 4 == 0, "4-byte granular");
  T out;
  const int* src = reinterpret_cast<const int*>(&v);
  int* dst = reinterpret_cast<int*>(&out);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) dst[i] = __builtin_amdgcn_readfirstlane(src[i]);
  return out;
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

// Index range [a, b) within [lo, hi) of the lines whose key lies strictly between the keys of
// v0 and v1 (v0 = -inf / v1 = +inf: unbounded). Keys are monotone in nu, so every such line has
// v0 < nu < v1 whatever the rounding of the key map; the range may miss a few lines near the
// bounds, never include one outside.
__device__ __forceinline__ void key_range(const uint32_t* __restrict__ keys, int64_t lo, int64_t hi, double v0,
                                          double v1, const KeyMap& km, int64_t& ra, int64_t& rb) {
  ra = rb = lo;
  if (!(v0 < v1)) return;
  const uint32_t kl = isinf(v0) ? 0u : bin_key(v0, km) + 1u;
  const uint32_t k1 = isinf(v1) ? km.kmax + 1u : bin_key(v1, km);
  if (k1 == 0u || kl > k1 - 1u) return;
  const uint32_t kr = k1 - 1u;
  int64_t a = lo, b = hi;  // first key >= kl
  while (a < b) { int64_t m = (a + b) >> 1; if (keys[m] < kl) a = m + 1; else b = m; }
  ra = a;
  b = hi;                  // first key > kr
  while (a < b) { int64_t m = (a + b) >> 1; if (keys[m] <= kr) a = m + 1; else b = m; }
  rb = a;
}

// core_z > 0: the list for the line-core pass. A line reaches a tile point with |z| < core_z
// only if its centre lies within core_z alpha of it, and alpha = beta nu <= beta (nu_j1 + cut),
// so the window shrinks to that half-width (with slack for the FP32 zone test of the core pass).
// far != null (wing pass): also the tile-far ranges of full tiles, the lines that (1) keep the
// whole tile inside their cut (with half a grid step to spare), (2) lie at least kTileFar tile
// widths from the tile centre, and (3) lie farther from the tile than far_z alpha_max, the
// largest reach of the core |z| < far_z (zone half-widths are at most far_z alpha), so that
// they have no core point on the tile. These three facts
// follow from the bounds alone, so the tile-far pass needs no per-line test and the wing
// pass skips the ranges; every other line of [lo, hi) stays in the wing pass.
__global__ void k_worklist(const uint32_t* __restrict__ keys, int64_t N, KeyMap km, double numin, double numax,
                           const PairDesc* __restrict__ pairs, int n_pairs, int n_tiles_total,
                           int tile_w, double cut, double core_z, int chunk, int32_t* __restrict__ lo_out,
                           int32_t* __restrict__ hi_out, int32_t* __restrict__ nc_out, int4* __restrict__ far_out,
                           int32_t* __restrict__ nf_out, int far_chunk, double far_z, int direct_only,
                           double core_pad) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_tiles_total) return;
  const PairDesc pd = pairs[find_pair(pairs, n_pairs, g)];
  const int64_t t = g - pd.tile_base;
  const int64_t j0 = t * tile_w;
  const int64_t j1 = (j0 + tile_w < pd.n ? j0 + tile_w : pd.n) - 1;
  int64_t lo = 0, hi = N;
  double hw = cut;
  if (core_z > 0.0) {
    const double vmax = fabs(grid_nu(pd.nu_start, pd.dnu, j1)) + (isinf(cut) ? numax : cut);
    // core_pad: the largest alpha increase of a list whose centres are shifted from the
    // wavenumbers their widths are taken at, times core_z
    const double hc = core_z * pd.beta * (vmax > numax ? numax : vmax) * 1.0001 + 0.01 * pd.dnu + core_pad + 1e-300;
    hw = hc < cut ? hc : cut;
  }
  if (!isinf(hw)) {
    const double va = __dsub_rn(grid_nu(pd.nu_start, pd.dnu, j0), hw);
    const double vb = __dadd_rn(grid_nu(pd.nu_start, pd.dnu, j1), hw);
    if (vb < numin || va > numax) {
      lo_out[g] = 0; hi_out[g] = 0; nc_out[g] = 1;
      if (far_out) {
        far_out[2 * g] = far_out[2 * g + 1] = make_int4(0, 0, 0, 0);
        nf_out[g] = nf_out[n_tiles_total + g] = 0;
      }
      return;
    }
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
  int64_t a1 = lo, b1 = lo, a2 = hi, b2 = hi, x1 = lo, x2 = hi;
  if (far_out && !direct_only && j0 + tile_w <= pd.n && hi > lo) {
    const double nA = grid_nu(pd.nu_start, pd.dnu, j0), nB = grid_nu(pd.nu_start, pd.dnu, j0 + tile_w - 1);
    const double nc = 0.5 * (nA + nB), half = 0.5 * (nB - nA);
    const double wlo = isinf(cut) ? numin : fmax(numin, nA - cut);
    const double whi = isinf(cut) ? numax : fmin(numax, nB + cut);
    const double amax = pd.beta * fmax(fabs(wlo), fabs(whi));
    const double reach = half + far_z * amax * 1.001 + 2.0 * pd.dnu;
    const double dfar = fmax(kTileFar * tile_w * pd.dnu, reach);
    const double d8 = fmax(kFar8Spans * tile_w * pd.dnu, reach);
    const double m = 0.5 * pd.dnu;
    const double v0 = isinf(cut) ? -INFINITY : nB - cut + m, v1 = isinf(cut) ? INFINITY : nA + cut - m;
    key_range(keys, lo, hi, v0, nc - dfar, km, a1, b1);
    key_range(keys, lo, hi, nc + dfar, v1, km, a2, b2);
    if (a1 == b1) a1 = b1 = lo;
    if (a2 == b2) a2 = b2 = hi;
    if (b1 > a2) { a1 = b1 = lo; a2 = b2 = hi; }  // cannot happen (disjoint key ranges); kept safe
    // the class-1 parts: the same outer bounds, so the same first (last) line when not empty
    int64_t e1 = lo, f1 = lo, e2 = hi, f2 = hi;
    key_range(keys, lo, hi, v0, nc - d8, km, e1, f1);
    key_range(keys, lo, hi, nc + d8, v1, km, e2, f2);
    x1 = (e1 < f1 && e1 == a1 && f1 <= b1) ? f1 : a1;
    x2 = (e2 < f2 && f2 == b2 && e2 >= a2) ? e2 : b2;
  } else {
    x1 = a1;
    x2 = b2;
  }
  const int64_t cnt = (a1 - lo) + (a2 - b1) + (hi - b2);
  int64_t nc = (cnt + chunk - 1) / chunk;
  lo_out[g] = (int32_t)lo;
  hi_out[g] = (int32_t)hi;
  nc_out[g] = (int32_t)(nc > 0 ? nc : 1);
  if (far_out) {
    // class 0: [x1, b1) and [a2, x2); class 1: [a1, x1) and [x2, b2)
    far_out[2 * g] = make_int4((int)x1, (int)b1, (int)a2, (int)x2);
    far_out[2 * g + 1] = make_int4((int)a1, (int)x1, (int)x2, (int)b2);
    const int64_t n0 = (b1 - x1) + (x2 - a2), n1 = (x1 - a1) + (b2 - x2);
    nf_out[g] = (int32_t)((n0 + far_chunk - 1) / far_chunk);
    nf_out[n_tiles_total + g] = (int32_t)((n1 + far_chunk - 1) / far_chunk);
  }
}

// Line segments of each span of the wing pass: the span's window of lines (as in k_worklist),
// minus the tile-far ranges of its tile (evaluated by the tile-far pass), split into far
// segments -- lines that keep the whole span inside their cut (half a grid step to spare), lie
// at least kFarSpans spans from the span centre and farther from the span than the reach of the
// core (far_z alpha_max), so that they have no core point there, all from the bounds alone --
// middle segments (the same with kMidSpans in place of kFarSpans, closer than the far ones),
// masked segments (lines whose cut bound falls on the span, at least kMaskSpans spans from its
// centre and beyond the core's reach: on the left, lines that reach a prefix of the span's
// points; on the right, a suffix), and direct segments (every other line), in list order.
__global__ void k_span_segments(const uint32_t* __restrict__ keys, int64_t N, KeyMap km, double numin,
                                double numax, const PairDesc* __restrict__ spairs,
                                const PairDesc* __restrict__ tpairs, int n_pairs, int n_spans, int span_w,
                                double cut, double far_z, const int4* __restrict__ tile_far, int chunk,
                                SpanSeg* __restrict__ segs, int32_t* __restrict__ nc_out, int direct_only) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_spans) return;
  const int p = find_pair(spairs, n_pairs, g);
  const PairDesc pd = spairs[p];
  const int64_t t = g - pd.tile_base;
  const int64_t j0 = t * span_w;
  const int64_t j1 = (j0 + span_w < pd.n ? j0 + span_w : pd.n) - 1;
  const double nA = grid_nu(pd.nu_start, pd.dnu, j0), nB = grid_nu(pd.nu_start, pd.dnu, j1);
  SpanSeg sg;
  sg.n = 0;
  int64_t lo = 0, hi = N;
  if (!isinf(cut)) {
    const double va = __dsub_rn(nA, cut), vb = __dadd_rn(nB, cut);
    if (vb < numin || va > numax) { segs[g] = sg; nc_out[g] = 1; return; }
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
  // tile-far ranges of the span's tile
  int64_t ta1 = lo, tb1 = lo, ta2 = hi, tb2 = hi;
  if (tile_far) {
    const int tg = tpairs[p].tile_base + (int)(t / kWavesPerWG);
    const int4 c0 = tile_far[2 * tg], c1 = tile_far[2 * tg + 1];
    ta1 = c1.x; tb1 = c0.y; ta2 = c0.z; tb2 = c1.w;  // the union of the two classes' ranges
  }
  // far, middle and masked ranges of the span (full spans only); the middle ones contain the
  // far ones; the masked ones lie beyond the far ones' cut-side bounds
  int64_t fa1 = lo, fb1 = lo, fa2 = hi, fb2 = hi, ma1 = lo, mb1 = lo, ma2 = hi, mb2 = hi;
  int64_t la = lo, lb = lo, ra = hi, rb = hi, ea1 = lo, eb1 = lo, ea2 = hi, eb2 = hi;
  if (!direct_only && j0 + span_w <= pd.n && hi > lo) {
    const double c = 0.5 * (nA + nB), half = 0.5 * (nB - nA);
    const double wlo = isinf(cut) ? numin : fmax(numin, nA - cut);
    const double whi = isinf(cut) ? numax : fmin(numax, nB + cut);
    const double amax = pd.beta * fmax(fabs(wlo), fabs(whi));
    const double reach = half + far_z * amax * 1.001 + 2.0 * pd.dnu;
    const double d = fmax(kFarSpans * span_w * pd.dnu, reach);
    const double dm = fmax(kMidSpans * span_w * pd.dnu, reach);
    const double d8 = fmax(kFar8Spans * span_w * pd.dnu, reach);
    const double dk = fmax(kMaskSpans * span_w * pd.dnu, reach);
    const double m = 0.5 * pd.dnu;
    const double v0 = isinf(cut) ? -INFINITY : nB - cut + m, v1 = isinf(cut) ? INFINITY : nA + cut - m;
    key_range(keys, lo, hi, v0, c - d, km, fa1, fb1);
    key_range(keys, lo, hi, c + d, v1, km, fa2, fb2);
    key_range(keys, lo, hi, v0, c - dm, km, ma1, mb1);
    key_range(keys, lo, hi, c + dm, v1, km, ma2, mb2);
    key_range(keys, lo, hi, v0, c - d8, km, ea1, eb1);
    key_range(keys, lo, hi, c + d8, v1, km, ea2, eb2);
    if (!isinf(cut) && cut > 2.0 * (nB - nA) + 2.0 * pd.dnu && span_w <= kMaskMaxSpan) {
      // below v0 a line's cut range ends on the span (or before it) and starts far left of it;
      // above v1 it starts on the span (or after it) and ends far right of it
      key_range(keys, lo, hi, -INFINITY, fmin(v0 - 2.0 * m, c - dk), km, la, lb);
      key_range(keys, lo, hi, fmax(v1 + 2.0 * m, c + dk), INFINITY, km, ra, rb);
    }
  }
  // elementary intervals between all range ends, in order; tile-far ones are left out
  constexpr int NB = 22;
  int64_t bp[NB] = {lo, hi, fa1, fb1, fa2, fb2, ma1, mb1, ma2, mb2, ta1, tb1, ta2, tb2, la, lb, ra, rb,
                    ea1, eb1, ea2, eb2};
  for (int i = 0; i < NB; ++i) bp[i] = bp[i] < lo ? lo : (bp[i] > hi ? hi : bp[i]);
  for (int i = 1; i < NB; ++i)
    for (int j = i; j > 0 && bp[j - 1] > bp[j]; --j) { const int64_t x = bp[j]; bp[j] = bp[j - 1]; bp[j - 1] = x; }
  int64_t total = 0;
  for (int i = 0; i + 1 < NB; ++i) {
    const int64_t x = bp[i], y = bp[i + 1];
    if (x >= y) continue;
    if ((x >= ta1 && y <= tb1) || (x >= ta2 && y <= tb2)) continue;
    const uint8_t kind = ((x >= ea1 && y <= eb1) || (x >= ea2 && y <= eb2))   ? kSegFar8
                         : ((x >= fa1 && y <= fb1) || (x >= fa2 && y <= fb2)) ? kSegFar
                         : ((x >= ma1 && y <= mb1) || (x >= ma2 && y <= mb2)) ? kSegMid
                         : (x >= la && y <= lb)                               ? kSegMaskLeft
                         : (x >= ra && y <= rb)                               ? kSegMaskRight
                                                                              : kSegDirect;
    const int q = (int)sg.n - 1;
    if (q >= 0 && (int64_t)sg.lo[q] + sg.len[q] == x && sg.kind[q] == kind) {
      sg.len[q] += (int32_t)(y - x);
    } else if (sg.n < kMaxSeg) {
      sg.lo[sg.n] = (int32_t)x;
      sg.len[sg.n] = (int32_t)(y - x);
      sg.kind[sg.n] = kind;
      ++sg.n;
    }
    total += y - x;
  }
  segs[g] = sg;
  const int64_t nc = (total + chunk - 1) / chunk;
  nc_out[g] = (int32_t)(nc > 0 ? nc : 1);
}

// item_base = exclusive scan of nc; item_base[n] = total; also resets the item dispenser.
__global__ __launch_bounds__(1024) void k_item_scan(const int32_t* __restrict__ nc, int n,
                                                    int32_t* __restrict__ item_base, int* counter) {
  __shared__ int32_t s[1024];
  __shared__ int32_t carry;
  if (threadIdx.x == 0) { carry = 0; counter[0] = 0; counter[1] = 0; }
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
// w(x + iy), y >= 0, by J.A.C. Weideman's rational approximation ("Computation of the complex
// error function", SIAM J. Numer. Anal. 31 (1994) 1497-1518) with N = kWeidN terms:
// w = 2 p(Z) u^2 + u/sqrt(pi), u = 1/(L - iz), Z = (L + iz)/(L - iz), p(Z) = sum_m a_m Z^m. The
// coefficients live in constant memory and are read with scalar loads into SGPRs (the loops are
// fully unrolled). p has real coefficients, so it is evaluated by the second-order recurrence
// of division by the real quadratic Z^2 - r Z + s (r = 2 Re Z, s = |Z|^2) of which Z is a root
// (Knuth, TAOCP vol. 2, Sec. 4.6.4): b_m = a_m + r b_(m+1) - s b_(m+2), p = a_0 - s b_2 + Z b_1;
// two real FMAs per coefficient instead of four for complex Horner.
static_assert(kWeidN >= 3, "the recurrence needs three coefficients");

// Re w(x + iy), y >= 0, in FP32 (the line-core pass): Re(2 p u^2 + u/sqrt(pi)) = Re(u t) with
// t = 2 p u + 1/sqrt(pi). Two choices keep it within about 4.5e-7 of the profile's peak Re w(iy)
// for |z| < 6.75 (against scipy's wofz; the approximation's own error is 7.4e-9): the reciprocal of |L - iz|^2 takes one
// Newton step, and Z is formed as 1 + (Z - 1) with Z - 1 = 2iz u computed from z and
// u = 1/(L - iz), not as 2Lu - 1, whose rounding the polynomial amplifies most near z = 0
// (7e-7 of the peak with 2Lu - 1).
__device__ __forceinline__ float weideman_re32(float x, float y) {
  const float L = c_weidL32;
  const float dr = L + y;  // L - iz = dr - ix
  const float d = __builtin_fmaf(dr, dr, x * x);
  float inv = __builtin_amdgcn_rcpf(d);
  inv = __builtin_fmaf(inv, __builtin_fmaf(-d, inv, 1.0f), inv);
  const float ur = dr * inv, ui = x * inv;  // u = (dr + ix)/(dr^2 + x^2)
  // Z - 1 = 2iz u = -2(y ur + x ui) + 2i(x ur - y ui)
  const float Zr = __builtin_fmaf(-2.0f * x, ui, __builtin_fmaf(-2.0f * y, ur, 1.0f));
  const float Zi = 2.0f * __builtin_fmaf(x, ur, -y * ui);
  // p(Z) by the real-quadratic recurrence, as in the FP64 form
  const float r = 2.0f * Zr, s = __builtin_fmaf(Zr, Zr, Zi * Zi);
  float b2 = c_weid32[kWeidN - 1];
  float b1 = __builtin_fmaf(r, b2, c_weid32[kWeidN - 2]);
#pragma unroll
  for (int m = kWeidN - 3; m >= 1; --m) {
    const float t = __builtin_fmaf(r, b1, __builtin_fmaf(-s, b2, c_weid32[m]));
    b2 = b1;
    b1 = t;
  }
  const float pr = __builtin_fmaf(Zr, b1, __builtin_fmaf(-s, b2, c_weid32[0]));
  const float pi = Zi * b1;
  const float tr = 2.0f * __builtin_fmaf(pr, ur, -pi * ui) + 0.564189583547756287f;
  const float ti = 2.0f * __builtin_fmaf(pr, ui, pi * ur);
  return __builtin_fmaf(ur, tr, -ui * ti);
}

// The same in FP64 with kWeidN40 = 40 terms, for the line-core rounds that hold a pair of a line
// whose peak falls between grid points: the grid samples such a line only on its flanks, where
// the FP32 form's error, a fraction of the line's peak, can be a large part of the values, and
// 18 terms in FP64 still leave 7e-9 of the peak (a relative 1e-3 of a Gaussian at |x| = 3.5); 40
// terms keep 3.4e-9 of the value itself out to |x| = 4.3.
__device__ __forceinline__ double rcp64(double d) {  // 1/d for normal d > 0: estimate, two Newton steps
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  return fma(r, fma(-d, r, 1.0), r);
}

// The coefficients c (FP64) come from LDS: as constants they would take 80 scalar registers
// from the FP32 form, whose coefficients then spill.
__device__ __forceinline__ double weideman_re64(double x, double y, const double* c) {
  const double L = c_weid40L;
  const double dr = L + y;
  const double inv = rcp64(fma(dr, dr, x * x));
  const double ur = dr * inv, ui = x * inv;
  const double Zr = fma(-2.0 * x, ui, fma(-2.0 * y, ur, 1.0));
  const double Zi = 2.0 * fma(x, ur, -y * ui);
  const double r = 2.0 * Zr, s = fma(Zr, Zr, Zi * Zi);
  double b2 = c[kWeidN40 - 1];
  double b1 = fma(r, b2, c[kWeidN40 - 2]);
#pragma unroll 4
  for (int m = kWeidN40 - 3; m >= 1; --m) {
    const double t = fma(r, b1, fma(-s, b2, c[m]));
    b2 = b1;
    b1 = t;
  }
  const double pr = fma(Zr, b1, fma(-s, b2, c[0]));
  const double pi = Zi * b1;
  const double tr = 2.0 * fma(pr, ur, -pi * ui) + 0.56418958354775628695;
  const double ti = 2.0 * fma(pr, ui, pi * ur);
  return fma(ur, tr, -ui * ti);
}

// Per-line, per-grid record: the parts of a line's evaluation that depend on the grid but
// not on T or P, all decided in FP64: x = bits of the FP32 offset delta = nu_{jref} - nu_i,
// y = jref (grid point nearest the centre, clamped to the grid), z, w = inclusive cut bounds
// (z > w: the line reaches no point).
__global__ __launch_bounds__(kThreads) void k_gridrec(const double* __restrict__ nu, int64_t N, double nu_start,
                                                      double dnu, int64_t n, double cut, int4* __restrict__ grec) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double nu0 = nu[i];
  int64_t jlo, jhi;
  cut_range(nu0, nu_start, dnu, n, cut, jlo, jhi);
  double jr = rint((nu0 - nu_start) / dnu);
  jr = jr < 0.0 ? 0.0 : (jr > (double)(n - 1) ? (double)(n - 1) : jr);
  const int64_t jref = (int64_t)jr;
  const double delta = __dsub_rn(grid_nu(nu_start, dnu, jref), nu0);
  if (jlo > jhi) { jlo = 1; jhi = 0; }
  grec[i] = make_int4(__float_as_int((float)delta), (int)jref, (int)jlo, (int)jhi);
}

// Per-wave record of the lines of a direct segment staged in LDS (structure of arrays, one
// entry per lane):
//   F0 = (dh, jt, dnh, gh): offset delta/sqrt(s), reference index - span start, dnu/sqrt(s),
//        gamma^2/s, with s = max(alpha^2, gamma^2)
//   F1 = (Ah, lo_rel, hi_rel, a): S gamma/(pi s), cut bounds relative to the reference
//        index, alpha^2/s
//   KA, KB, KC: Ah times the far-wing series coefficients of orders 2-4 (see wing_coeffs)
//   K5, K5C: c4-c7 and c8 of order 5 (c1-c3 as order 4), for lines that need order 5
//   CZ: the line's core points (|z| below the core threshold zcore) within its cut range,
//       as an inclusive span-local range (empty: x > y)
//   A line that needs an order above 5 on the span (points next to its core) holds instead
//   Ah times c1-c16 of order kKw: KA = c1-c4, KB = c5-c8, K5 = c9-c12, KC = c13, K5C = c14,
//   F1.w = c15, CZ.y = c16 (bits), and its core range in CZ.x (low and high 16 bits).
//   list: the staged lines that reach the span, grouped by how they are evaluated (see
//         direct_group), in staging order within a group
//   node, node_mid: the span's node sums of the item's far and middle-distance lines
struct WaveLDS {
  float4 F0[kWave];
  float4 F1[kWave];
  float4 KA[kWave];  // c1, c2(K=2), c2(K>=3), c3(K=3)
  float4 KB[kWave];  // c4(K=3), c3(K=4), c4(K=4), c5(K=4)
  float KC[kWave];   // c6(K=4)
  float4 K5[kWave];  // c4-c7(K=5)
  float K5C[kWave];  // c8(K=5)
  int2 CZ[kWave];
  uint8_t list[kWave];
  double node[kNodes];
  double node8[kFar8Nodes];
  double node_mid[kMidNodes];
};

// Evaluation group of a staged line: 0 does not reach the span; 1-4 all points inside the cut,
// no core points, series order 1-4; 5-8 the same with some points outside the cut; 9 order 5
// (no core points); 10 order kKw (points next to the core, core points excluded).
constexpr int kDirectGroups = 10;
__device__ __forceinline__ int direct_group(uint32_t code) {
  if (code == 0u) return 0;
  const int K = (int)(code & 15u);
  if ((code & 32u) || K > kKmax) return 10;
  if (K == kKmax) return 9;
  return (code & 16u) ? 4 + K : K;
}
// Far-wing series of the Voigt profile in q = 1/(D^2 + gamma^2), from the asymptotic
// expansion w(z) ~ (i/sqrt(pi)) sum_k (2k-1)!!/(2^k z^(2k+1)): with t = alpha^2 q and
// u = gamma^2 q,  V = (S gamma/pi) q sum_{k<K} a_k t^k P_k(u), a_k = (2k-1)!!/2^k,
// P_k(u) = U_2k(sqrt(1-u)) (Chebyshev polynomials of the second kind) expanded in u:
// P_0 = 1, P_1 = 3 - 4u, P_2 = 5 - 20u + 16u^2, P_3 = 7 - 56u + 112u^2 - 64u^3.
// Truncated at order K its relative error is below 2e-6 for |z| above zK[K-1].
// Written as a polynomial sum_M c_M qh^(M+1) in qh = s q (s = max(alpha^2, gamma^2) keeps
// qh <= 1 and the coefficients O(1)), with a = alpha^2/s, g = gamma^2/s in [0, 1]:
//   K=2: c1 = 3a/2, c2 = -2ag
//   K=3: c1, c2 = -2ag + 15a^2/4, c3 = -15a^2 g, c4 = 12 a^2 g^2
//   K=4: c1, c2 (as K=3), c3 = -15a^2 g + 105a^3/8, c4 = 12a^2g^2 - 105a^3 g, c5 = 210 a^3 g^2,
//        c6 = -120 a^3 g^3
//   K=5: c1..c3 (as K=4), c4 = 12a^2g^2 - 105a^3g + 945a^4/16, c5 = 210a^3g^2 - 1575a^4g/2,
//        c6 = -120a^3g^3 + 2835a^4g^2, c7 = -3780a^4g^3, c8 = 1680a^4g^4
//   (a_4 = 105/16; P_4(u) = 9 - 120u + 432u^2 - 576u^3 + 256u^4)
// Order 9 (terms k <= 8; P_(k+1) = (2 - 4u) P_k - P_(k-1), P_(-1) = -1), c1-c3 as order 4:
//   c4  = 12a^2g^2 - 105a^3g + 945a^4/16
//   c5  = 210a^3g^2 - 1575a^4g/2 + 10395a^5/32
//   c6  = -120a^3g^3 + 2835a^4g^2 - 51975a^5g/8 + 135135a^6/64
//   c7  = -3780a^4g^3 + 72765a^5g^2/2 - 945945a^6g/16 + 2027025a^7/128
//   c8  = 1680a^4g^4 - 83160a^5g^3 + 945945a^6g^2/2 - 4729725a^7g/8 + 34459425a^8/256
//   c9  = 83160a^5g^4 - 1621620a^6g^3 + 25540515a^7g^2/4 - 103378275a^8g/16
//   c10 = -30240a^5g^5 + 2702700a^6g^4 - 30405375a^7g^3 + 723647925a^8g^2/8
//   c11 = -2162160a^6g^5 + 74324250a^7g^4 - 1137161025a^8g^3/2
//   c12 = 665280a^6g^6 - 97297200a^7g^5 + 1895268375a^8g^4
//   c13 = 64864800a^7g^6 - 3583780200a^8g^5
//   c14 = -17297280a^7g^7 + 3859455600a^8g^6
//   c15 = -2205403200a^8g^7
//   c16 = 518918400a^8g^8
// For |z| >= 4.4 the order-9 series is within 1.3e-7 of the line's peak value (FP32 Horner).
__device__ __forceinline__ void order9_coeffs(float a, float g, float Ah, float4& c1_4, float4& c5_8, float4& c9_12,
                                              float& c13, float& c14, float& c15, float& c16) {
  const float a2 = a * a, a3 = a2 * a, a4 = a2 * a2, a5 = a4 * a, a6 = a3 * a3, a7 = a6 * a, a8 = a4 * a4;
  const float g2 = g * g, g3 = g2 * g, g4 = g2 * g2, g5 = g4 * g, g6 = g3 * g3, g7 = g6 * g, g8 = g4 * g4;
  c1_4 = make_float4(Ah * (1.5f * a), Ah * (-2.0f * a * g + 3.75f * a2), Ah * (-15.0f * a2 * g + 13.125f * a3),
                     Ah * (12.0f * a2 * g2 - 105.0f * a3 * g + 59.0625f * a4));
  c5_8 = make_float4(Ah * (210.0f * a3 * g2 - 787.5f * a4 * g + 324.84375f * a5),
                     Ah * (-120.0f * a3 * g3 + 2835.0f * a4 * g2 - 6496.875f * a5 * g + 2111.484375f * a6),
                     Ah * (-3780.0f * a4 * g3 + 36382.5f * a5 * g2 - 59121.5625f * a6 * g + 15836.1328125f * a7),
                     Ah * (1680.0f * a4 * g4 - 83160.0f * a5 * g3 + 472972.5f * a6 * g2 - 591215.625f * a7 * g +
                           134607.12890625f * a8));
  c9_12 = make_float4(
      Ah * (83160.0f * a5 * g4 - 1621620.0f * a6 * g3 + 6385128.75f * a7 * g2 - 6461142.1875f * a8 * g),
      Ah * (-30240.0f * a5 * g5 + 2702700.0f * a6 * g4 - 30405375.0f * a7 * g3 + 90455990.625f * a8 * g2),
      Ah * (-2162160.0f * a6 * g5 + 74324250.0f * a7 * g4 - 568580512.5f * a8 * g3),
      Ah * (665280.0f * a6 * g6 - 97297200.0f * a7 * g5 + 1895268375.0f * a8 * g4));
  c13 = Ah * (64864800.0f * a7 * g6 - 3583780200.0f * a8 * g5);
  c14 = Ah * (-17297280.0f * a7 * g7 + 3859455600.0f * a8 * g6);
  c15 = Ah * (-2205403200.0f * a8 * g7);
  c16 = Ah * (518918400.0f * a8 * g8);
}

__device__ __forceinline__ void wing_coeffs(float a, float g, float Ah, float4& KA, float4& KB, float& KC) {
  const float a2 = a * a, a3 = a2 * a, g2 = g * g;
  const float c2_2 = -2.0f * a * g;
  const float c3_3 = -15.0f * a2 * g;
  const float c4_3 = 12.0f * a2 * g2;
  KA = make_float4(Ah * (1.5f * a), Ah * c2_2, Ah * (c2_2 + 3.75f * a2), Ah * c3_3);
  KB = make_float4(Ah * c4_3, Ah * (c3_3 + 13.125f * a3), Ah * (c4_3 - 105.0f * a3 * g), Ah * (210.0f * a3 * g2));
  KC = Ah * (-120.0f * a3 * g2 * g);
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

// Core points of a line relative to its reference point j_ref: the integers r with
// |r - c| < h, where c = -delta/dnu is the centre in grid units and h = sqrt(zc^2 alpha^2 -
// gamma^2)/dnu (with a little slack). Evaluated in FP32 from the same inputs in the wing and
// the core pass, so both classify every (line, point) pair identically whatever their tiling.
__device__ __forceinline__ bool core_rel(float alpha, float gam, float delta, float inv_dnu, float zc, int& rlo,
                                         int& rhi) {
  const float af = alpha * inv_dnu, gf = gam * inv_dnu;
  const float zz = zc * af;
  const float h2 = zz * zz - gf * gf;
  if (!(h2 > 0.0f)) return false;
  const float h = sqrtf(h2) * 1.00001f + 1e-3f;
  const float c = -delta * inv_dnu;
  const float fl = floorf(c - h) + 1.0f, fh = ceilf(c + h) - 1.0f;
  rlo = fl < -2.0e9f ? -2000000000 : (int)fl;
  rhi = fh > 2.0e9f ? 2000000000 : (int)fh;
  return rlo <= rhi;
}

// Stage one line for a span (64 P points from global point span0) from its grid record and its
// strength/width at T: the FP32 quantities of the evaluation, and the code word: bits 0-3 the
// highest series order its span points need (0: the line does not reach the span), bit 4 some
// points fall outside its cut range, bit 5 some of its points are core points (|z| < zcore).
// Every decision that needs FP64 (cut bounds, reference point, offset) is already in the grid
// record; the rest needs ~1e-7 and is done in FP32 (products ordered so that no intermediate
// underflows for relevant lines).
template <int P>
__device__ __forceinline__ uint32_t stage_span_line(WaveLDS& L, int lane, const int4 gr, double nu0, float S,
                                                    float gTv, const PairDesc& pd, const float* zw, float zcore,
                                                    int64_t span0) {
  constexpr int W = kWave * P;
  const int jref = gr.y, jlo = gr.z, jhi = gr.w;
  if (!(S > 0.0f) || jlo > jhi || (int64_t)jhi < span0 || (int64_t)jlo > span0 + (W - 1)) return 0u;
  const float alpha = (float)(nu0 * pd.beta);
  const float gam = gTv * (float)pd.pfac;
  const float a2 = alpha * alpha, g2 = gam * gam;
  const float sc = a2 > g2 ? a2 : g2;
  if (!(sc > 0.0f)) return 0u;
  const float rs = __frsqrt_rn(sc);
  const float isc = rs * rs;
  const float delta = __int_as_float(gr.x);
  const int jt = (int)((int64_t)jref - span0);
  const float Ah = S * (gam * isc) * 0.318309886183790672f;  // S gamma / (pi s)
  const float av = a2 * isc, gv = g2 * isc;
  L.F0[lane] = make_float4(delta * rs, (float)jt, (float)pd.dnu * rs, gv);
  L.F1[lane] = make_float4(Ah, (float)(jlo - jref), (float)(jhi - jref), av);
  // zone K: points with |z| < zw[K], i.e. |j - c| < sqrt(zw^2 alpha^2 - gamma^2)/dnu around the
  // centre c (span-local points); a slot [s0, s1] meets it when s0 < c + h and s1 > c - h
  const float inv_dnu = (float)(1.0 / pd.dnu);
  const float af = alpha * inv_dnu, gf = gam * inv_dnu;
  const float c = (float)jt - delta * inv_dnu;
  const int clo = (int)((int64_t)jlo - span0 < -1 ? -1 : (int64_t)jlo - span0);
  const int chi = (int)((int64_t)jhi - span0 > W ? W : (int64_t)jhi - span0);
  // zone half-widths, once per line (the hardware square root: the bounds carry a relative slack
  // of 1e-5 and only choose how many series terms the span's points get)
  float hz[kKw - 1];
#pragma unroll
  for (int z = 0; z < kKw - 1; ++z) {
    const float zz = zw[z] * af;
    const float h2 = zz * zz - gf * gf;
    hz[z] = h2 > 0.0f ? __builtin_amdgcn_sqrtf(h2) * 1.00001f + 1e-3f : -1.0f;
  }
  uint32_t K = 1u;
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int s0 = p * kWave, s1 = s0 + kWave - 1;
    if (s1 < clo || s0 > chi) continue;  // no point of the slot in the cut
    uint32_t path = 1u;
#pragma unroll
    for (int z = 0; z < kKw - 1; ++z) path += ((float)s0 < c + hz[z] && (float)s1 > c - hz[z]) ? 1u : 0u;
    K = path > K ? path : K;
  }
  // core points: strictly inside the core zone, and within the cut range
  int czl = 1, czh = 0, rlo, rhi;
  if (core_rel(alpha, gam, delta, inv_dnu, zcore, rlo, rhi)) {
    const int64_t gl = (int64_t)jref + rlo - span0, gh = (int64_t)jref + rhi - span0;
    czl = (int)(gl < clo ? clo : (gl > W + 1 ? W + 1 : gl));
    czh = (int)(gh > chi ? chi : (gh < -2 ? -2 : gh));
  }
  const bool core = (czl > 0 ? czl : 0) <= (czh < W - 1 ? czh : W - 1);
  if (core || K > (uint32_t)kKmax) {
    // order kKw for all its span points (the coefficient layout of the order-kKw group)
    float4 c1_4, c5_8, c9_12;
    float c13, c14, c15, c16;
    order9_coeffs(av, gv, Ah, c1_4, c5_8, c9_12, c13, c14, c15, c16);
    L.KA[lane] = c1_4;
    L.KB[lane] = c5_8;
    L.K5[lane] = c9_12;
    L.KC[lane] = c13;
    L.K5C[lane] = c14;
    L.F1[lane].w = c15;
    L.CZ[lane] = make_int2((int)(((uint32_t)czl & 0xffffu) | ((uint32_t)czh << 16)), __float_as_int(c16));
    if (core) K = kKw;
  } else {
    wing_coeffs(av, gv, Ah, L.KA[lane], L.KB[lane], L.KC[lane]);
    if (K == (uint32_t)kKmax) {
      const float a3 = av * av * av, a4 = a3 * av, g2v = gv * gv, g3v = g2v * gv;
      L.K5[lane] = make_float4(Ah * (12.0f * av * av * g2v - 105.0f * a3 * gv + 59.0625f * a4),
                               Ah * (210.0f * a3 * g2v - 787.5f * a4 * gv), Ah * (-120.0f * a3 * g3v + 2835.0f * a4 * g2v),
                               Ah * (-3780.0f * a4 * g3v));
      L.K5C[lane] = Ah * (1680.0f * a4 * g2v * g2v);
    }
  }
  const bool masked = !(clo <= 0 && chi >= W - 1);
  return K | (masked ? 16u : 0u) | (core ? 32u : 0u);
}

// One line, all slots of this wave, series order K. MASK: lanes outside the cut range add
// nothing. EXCL: lanes in [xl, xh] (the line's core points, relative index) add nothing.
template <int P, int K, bool MASK, bool EXCL>
__device__ __forceinline__ void wing_slots(float (&part)[P], float kf0, const float4& f0, const float4& f1,
                                           const float4& ka, const float4& kb, float kc, float xl = 0.f,
                                           float xh = -1.f) {
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const float kf = kf0 + (float)(kWave * p);
    const float D = __builtin_fmaf(kf, f0.z, f0.x);
    const float R = __builtin_fmaf(D, D, f0.w);
    const float q = __builtin_amdgcn_rcpf(R);
    float t;
    if (K == 1) {
      t = f1.x;
    } else if (K == 2) {
      t = __builtin_fmaf(ka.y, q, ka.x);
      t = __builtin_fmaf(t, q, f1.x);
    } else if (K == 3) {
      t = __builtin_fmaf(kb.x, q, ka.w);
      t = __builtin_fmaf(t, q, ka.z);
      t = __builtin_fmaf(t, q, ka.x);
      t = __builtin_fmaf(t, q, f1.x);
    } else if (K == 4) {
      t = __builtin_fmaf(kc, q, kb.w);
      t = __builtin_fmaf(t, q, kb.z);
      t = __builtin_fmaf(t, q, kb.y);
      t = __builtin_fmaf(t, q, ka.z);
      t = __builtin_fmaf(t, q, ka.x);
      t = __builtin_fmaf(t, q, f1.x);
    } else {  // K == 5: ka = (c1, c2, c3, c4), kb = (c5, c6, c7, c8)
      t = __builtin_fmaf(kb.w, q, kb.z);
      t = __builtin_fmaf(t, q, kb.y);
      t = __builtin_fmaf(t, q, kb.x);
      t = __builtin_fmaf(t, q, ka.w);
      t = __builtin_fmaf(t, q, ka.z);
      t = __builtin_fmaf(t, q, ka.y);
      t = __builtin_fmaf(t, q, ka.x);
      t = __builtin_fmaf(t, q, f1.x);
    }
    if (EXCL) {
      // excluded core points may have R = 0 (q infinite): select the sum, not the term
      bool in = (kf < xl) || (kf > xh);
      if (MASK) in = in && (kf >= f1.y) && (kf <= f1.z);
      part[p] = in ? __builtin_fmaf(t, q, part[p]) : part[p];
    } else if (MASK) {
      // points outside the cut are far from the centre (q finite): zero the term
      const float tm = (kf >= f1.y && kf <= f1.z) ? t : 0.0f;
      part[p] = __builtin_fmaf(tm, q, part[p]);
    } else {
      part[p] = __builtin_fmaf(t, q, part[p]);
    }
  }
}

// One staged line (uniform index l), all slots of this wave, series order K 1-4, no core points.
template <int P, int K, bool MASK>
__device__ __forceinline__ void wing_line(const WaveLDS& L, int l, float jl0, float (&part)[P]) {
  const float4 f0 = L.F0[l];
  const float4 f1 = L.F1[l];
  float4 ka = make_float4(0.f, 0.f, 0.f, 0.f), kb = ka;
  float kc = 0.f;
  if (K >= 2) ka = L.KA[l];
  if (K >= 3) kb = L.KB[l];
  if (K >= 4) kc = L.KC[l];
  wing_slots<P, K, MASK, false>(part, jl0 - f0.y, f0, f1, ka, kb, kc);
}

// One staged line of order 5 (no core points on the span), all slots, points outside the cut
// masked.
template <int P>
__device__ __forceinline__ void wing_line_order5(const WaveLDS& L, int l, float jl0, float (&part)[P]) {
  const float4 f0 = L.F0[l];
  const float4 f1 = L.F1[l];
  const float4 ka = L.KA[l], kb = L.KB[l], k5 = L.K5[l];
  // order 5 as wing_slots takes it: ka = (c1, c2, c3, c4), kb = (c5, c6, c7, c8)
  const float4 k5a = make_float4(ka.x, ka.z, kb.y, k5.x);
  const float4 k5b = make_float4(k5.y, k5.z, k5.w, L.K5C[l]);
  wing_slots<P, 5, true, false>(part, jl0 - f0.y, f0, f1, k5a, k5b, 0.f);
}

// One staged line of order kKw (points next to its core on the span), all slots: Horner in q
// over c16..c1 and the amplitude; points outside the cut, and with EXCL its core points
// [xl, xh] (relative index; they may have R = 0, q infinite: the sum is selected, not the
// term), add nothing.
template <int P, bool EXCL>
__device__ __forceinline__ void wing_slots9(float (&part)[P], float kf0, const float4& f0, const float4& f1,
                                            const float4& c1_4, const float4& c5_8, const float4& c9_12, float c13,
                                            float c14, float c15, float c16, float xl, float xh) {
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const float kf = kf0 + (float)(kWave * p);
    const float D = __builtin_fmaf(kf, f0.z, f0.x);
    const float R = __builtin_fmaf(D, D, f0.w);
    const float q = __builtin_amdgcn_rcpf(R);
    float t = __builtin_fmaf(c16, q, c15);
    t = __builtin_fmaf(t, q, c14);
    t = __builtin_fmaf(t, q, c13);
    t = __builtin_fmaf(t, q, c9_12.w);
    t = __builtin_fmaf(t, q, c9_12.z);
    t = __builtin_fmaf(t, q, c9_12.y);
    t = __builtin_fmaf(t, q, c9_12.x);
    t = __builtin_fmaf(t, q, c5_8.w);
    t = __builtin_fmaf(t, q, c5_8.z);
    t = __builtin_fmaf(t, q, c5_8.y);
    t = __builtin_fmaf(t, q, c5_8.x);
    t = __builtin_fmaf(t, q, c1_4.w);
    t = __builtin_fmaf(t, q, c1_4.z);
    t = __builtin_fmaf(t, q, c1_4.y);
    t = __builtin_fmaf(t, q, c1_4.x);
    t = __builtin_fmaf(t, q, f1.x);
    bool in = (kf >= f1.y) && (kf <= f1.z);
    if (EXCL) in = in && ((kf < xl) || (kf > xh));
    part[p] = in ? __builtin_fmaf(t, q, part[p]) : part[p];
  }
}

template <int P>
__device__ __forceinline__ void wing_line_order9(const WaveLDS& L, int l, uint32_t code, float jl0,
                                                 float (&part)[P]) {
  const float4 f0 = L.F0[l];
  const float4 f1 = L.F1[l];
  const float4 c1_4 = L.KA[l], c5_8 = L.KB[l], c9_12 = L.K5[l];
  const float c13 = L.KC[l], c14 = L.K5C[l];
  const int2 cz = L.CZ[l];
  const float kf0 = jl0 - f0.y;
  if (code & 32u) {
    const uint32_t zz = (uint32_t)__builtin_amdgcn_readfirstlane(cz.x);
    const float jt = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(f0.y)));
    const float xl = (float)(int)(int16_t)(zz & 0xffffu) - jt, xh = (float)(int)(int16_t)(zz >> 16) - jt;
    wing_slots9<P, true>(part, kf0, f0, f1, c1_4, c5_8, c9_12, c13, c14, f1.w, __int_as_float(cz.y), xl, xh);
  } else {
    wing_slots9<P, false>(part, kf0, f0, f1, c1_4, c5_8, c9_12, c13, c14, f1.w, __int_as_float(cz.y), 0.f, -1.f);
  }
}

// The lines of one group (list entries [i0, i1)): blocks of four lines (the list read four
// entries at a time into a scalar register), a compensated flush after every 16 lines.
template <int P, int K, bool MASK>
__device__ __forceinline__ void direct_loop(const WaveLDS& L, int i0, int i1, float jl0, float (&part)[P],
                                            float (&s)[P], float (&cc)[P]) {
  if (i0 >= i1) return;
  int i = i0;
  for (; i < i1 && (i & 3); ++i)  // unaligned head
    wing_line<P, K, MASK>(L, __builtin_amdgcn_readfirstlane((int)L.list[i]), jl0, part);
  int since = 0;
  for (; i + 4 <= i1; i += 4) {
    const uint32_t w4 = (uint32_t)__builtin_amdgcn_readfirstlane((int)*reinterpret_cast<const uint32_t*>(&L.list[i]));
    wing_line<P, K, MASK>(L, (int)(w4 & 255u), jl0, part);
    wing_line<P, K, MASK>(L, (int)((w4 >> 8) & 255u), jl0, part);
    wing_line<P, K, MASK>(L, (int)((w4 >> 16) & 255u), jl0, part);
    wing_line<P, K, MASK>(L, (int)(w4 >> 24), jl0, part);
    since += 4;
    if (since == 16) {
      kahan_flush<P>(part, s, cc);
      since = 0;
    }
  }
  for (; i < i1; ++i) wing_line<P, K, MASK>(L, __builtin_amdgcn_readfirstlane((int)L.list[i]), jl0, part);
  kahan_flush<P>(part, s, cc);
}

__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// ------------------------------------------------------- lines far from a span or a tile
// A line whose centre lies far outside an interval of grid points (a span or a tile; see
// k_span_segments and k_worklist for the bounds that make it so) is smooth on it: it is
// evaluated at the interval's Chebyshev nodes only, one line per lane, with the far-wing
// series of the order its nearest point of the interval needs (the largest over the wave's
// lines; the bounds keep every point of the interval outside the line's core, where order 5
// holds). The node sums are later interpolated to the interval's points with the nodes'
// Lagrange weights.
struct FarLine {
  float h, e;   // node offset D = x h + e (x: node position in grid steps), in units of sqrt(s)
  float gq, a;  // gamma^2/s, alpha^2/s
  float A;      // S gamma / (pi s)
  int K;        // series order the line needs on the interval
};

// The far-wing series coefficients c_1 .. c_(2K-2) of order K (see wing_coeffs), times A, formed
// for the wave's order only.
template <int K>
__device__ __forceinline__ void far_coeffs(const FarLine& f, float (&c)[2 * kKmax - 2]) {
  const float a = f.a, g = f.gq, A = f.A;
  const float a2 = a * a, a3 = a2 * a, a4 = a2 * a2, g2 = g * g, g3 = g2 * g;
  if (K >= 2) c[0] = A * (1.5f * a);
  if (K == 2) c[1] = A * (-2.0f * a * g);
  if (K >= 3) c[1] = A * (-2.0f * a * g + 3.75f * a2);
  if (K == 3) {
    c[2] = A * (-15.0f * a2 * g);
    c[3] = A * (12.0f * a2 * g2);
  }
  if (K >= 4) c[2] = A * (-15.0f * a2 * g + 13.125f * a3);
  if (K == 4) {
    c[3] = A * (12.0f * a2 * g2 - 105.0f * a3 * g);
    c[4] = A * (210.0f * a3 * g2);
    c[5] = A * (-120.0f * a3 * g3);
  }
  if (K == 5) {
    c[3] = A * (12.0f * a2 * g2 - 105.0f * a3 * g + 59.0625f * a4);
    c[4] = A * (210.0f * a3 * g2 - 787.5f * a4 * g);
    c[5] = A * (-120.0f * a3 * g3 + 2835.0f * a4 * g2);
    c[6] = A * (-3780.0f * a4 * g3);
    c[7] = A * (1680.0f * a4 * g2 * g2);
  }
}

// The constants of one line for the interval of grid points [nu_a, nu_b] (an idle lane, or a
// line with S = 0, evaluates A = 0 at D = 1 and adds zero).
__device__ __forceinline__ FarLine far_line(bool valid, double nu, float S, float gTv, const PairDesc& pd,
                                            double nu_a, double nu_b, float inv_dnu, const float* zK) {
  FarLine f;
  f.h = 0.0f; f.e = 1.0f; f.gq = 1.0f; f.a = 0.0f; f.A = 0.0f;
  f.K = 1;
  if (!valid) return f;
  const float alpha = (float)(nu * pd.beta);
  const float gam = gTv * (float)pd.pfac;
  const float a2 = alpha * alpha, g2 = gam * gam;
  const float sc = a2 > g2 ? a2 : g2;
  if (!(S > 0.0f && sc > 0.0f)) return f;
  const float rs = __frsqrt_rn(sc);
  const float isc = rs * rs;
  f.A = S * (gam * isc) * 0.318309886183790672f;  // S gamma / (pi s)
  f.gq = g2 * isc;
  f.a = a2 * isc;
  f.h = (float)pd.dnu * rs;                       // one grid step in units of sqrt(s)
  f.e = -((float)(nu - nu_a) * inv_dnu) * f.h;    // minus the line's position, same units
  const float dmin = (float)(nu < nu_a ? nu_a - nu : nu - nu_b);  // to the nearest point
  const float r2 = dmin * dmin + g2;
#pragma unroll
  for (int z = 0; z < kKmax - 1; ++z) f.K += (zK[z] * zK[z] * a2 > r2) ? 1 : 0;
  return f;
}

// Node positions: compile-time ones of a span (literal operands), or kernel arguments.
template <int S, int M>
struct SpanNodes {
  __device__ constexpr float operator()(int k) const { return node_pos(S, M, k); }
};
struct ArgNodes {
  const float* x;
  __device__ float operator()(int k) const { return x[k]; }
};

// Adds f at nodes G0..G0+CNT-1 of xs to acc[G0..], with the series of order K
template <int K, int G0, int NN, class NS, int CNT = kNodes>
__device__ __forceinline__ void far_nodes(const NS& xs, const FarLine& f, float (&acc)[NN]) {
  float c[2 * kKmax - 2];
  far_coeffs<K>(f, c);
#pragma unroll
  for (int k = G0; k < G0 + CNT; ++k) {
    const float D = __builtin_fmaf(xs(k), f.h, f.e);
    const float R = __builtin_fmaf(D, D, f.gq);
    const float q = __builtin_amdgcn_rcpf(R);
    float t = K == 1 ? f.A : c[2 * K - 3];
#pragma unroll
    for (int m = 2 * K - 4; m >= 0; --m) t = __builtin_fmaf(t, q, c[m]);
    if (K > 1) t = __builtin_fmaf(t, q, f.A);
    acc[k] = __builtin_fmaf(t, q, acc[k]);
  }
}

// The wave's order: the largest its lines need.
__device__ __forceinline__ int wave_order(const FarLine& f) {
  return 1 + (__ballot(f.K >= 2) != 0ull ? 1 : 0) + (__ballot(f.K >= 3) != 0ull ? 1 : 0) +
         (__ballot(f.K >= 4) != 0ull ? 1 : 0) + (__ballot(f.K >= 5) != 0ull ? 1 : 0);
}

// Adds each lane's line at the NN nodes to its node sums (acc), with the wave's order.
template <int NN, class NS>
__device__ __forceinline__ void far_accumulate(const NS& xs, const FarLine& f, float (&acc)[NN]) {
  const int Kw = wave_order(f);
  if (Kw == 1) far_nodes<1, 0, NN, NS, NN>(xs, f, acc);
  else if (Kw == 2) far_nodes<2, 0, NN, NS, NN>(xs, f, acc);
  else if (Kw == 3) far_nodes<3, 0, NN, NS, NN>(xs, f, acc);
  else if (Kw == 4) far_nodes<4, 0, NN, NS, NN>(xs, f, acc);
  else far_nodes<5, 0, NN, NS, NN>(xs, f, acc);
}

// Adds the wave's node sums to node[k] (in a fixed order) and clears the lanes' FP32 sums; every
// 16 lines per lane at most, so that the FP32 sums stay short. A reduce-scatter by recursive
// halving over the lane bits 5, 4, ...: in the step on bit b a lane keeps the half of its node
// values selected by its bit b and adds its partner's (lane ^ 2^b) copy of that half; after
// log2(NN) steps lane L holds the sum, over the lanes that differ from it in those bits, of node
// L >> (6 - log2(NN)); butterflies over the remaining bits complete it over the wave.
// The steps on bits 5, 4, 3 (sums of 8 lanes' values) are FP32, in place, without LDS: for the
// pair (x = acc[i], y = acc[h + i]), gfx950's permlane32_swap exchanges the upper 32 lanes of x
// with the lower 32 lanes of y, after which x + y is node i's pair sum in the lower half of the
// wave and node h + i's in the upper half; permlane16_swap does the same for odd and even 16-lane
// rows; bit 3 uses a rotation by 8 within the 16-lane rows (lane ^ 8). The rest is FP64: three
// exchanges of doubles for 8 or 16 nodes (6 NN with one butterfly per node).
template <int NN>
__device__ __forceinline__ void far_flush(float (&acc)[NN], int lane, double* node) {
  static_assert(NN >= 8 && NN <= kWave && (NN & (NN - 1)) == 0, "node count: a power of two, 8 to 64");
#pragma unroll
  for (int i = 0; i < NN / 2; ++i) {  // lane bit 5
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(acc[i]), __float_as_uint(acc[NN / 2 + i]), false,
                                                    false);
    acc[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
#pragma unroll
  for (int i = 0; i < NN / 4; ++i) {  // lane bit 4
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(acc[i]), __float_as_uint(acc[NN / 4 + i]), false,
                                                    false);
    acc[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  {
    const bool up = (lane >> 3) & 1;  // lane bit 3: row rotation by 8 (DPP row_ror:8)
#pragma unroll
    for (int i = 0; i < NN / 8; ++i) {
      const float send = up ? acc[i] : acc[NN / 8 + i];
      const float keep = up ? acc[NN / 8 + i] : acc[i];
      acc[i] = keep + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(send), 0x128, 0xf, 0xf, false));
    }
  }
  constexpr int F = NN / 8;  // values per lane from here on, FP64
  double v[F];
#pragma unroll
  for (int k = 0; k < F; ++k) v[k] = (double)acc[k];
#pragma unroll
  for (int k = 0; k < NN; ++k) acc[k] = 0.0f;
  int bit = 2;
#pragma unroll
  for (int h = F / 2; h >= 1; h >>= 1, --bit) {
    const bool up = (lane >> bit) & 1;
#pragma unroll
    for (int i = 0; i < h; ++i) {
      const double send = up ? v[i] : v[h + i];
      const double keep = up ? v[h + i] : v[i];
      v[i] = keep + __shfl_xor(send, 1 << bit, kWave);
    }
  }
#pragma unroll
  for (; bit >= 0; --bit) v[0] += __shfl_xor(v[0], 1 << bit, kWave);
  constexpr int lo = 6 - __builtin_ctz(NN);  // lane bits below the node index
  if ((lane & ((1 << lo) - 1)) == 0) node[lane >> lo] += v[0];
}

__device__ __forceinline__ float wave_sum64f(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// The same for the middle-distance segments: lane half h holds node j (h = 0) or 31 - j (h = 1)
// in acc[j]; the sums are over the 32 lanes of each half.
// By the reduce-scatter of far_flush within each 32-lane half (bits 4, 3 in FP32, then FP64):
// lane 2 j of the lower half ends with node j, of the upper half with node 31 - j.
__device__ __forceinline__ void mid_flush(float (&acc)[kNodes], int lane, double* node) {
  static_assert(kNodes == 16 && kMidNodes == 32, "two 16-value halves");
#pragma unroll
  for (int i = 0; i < 8; ++i) {  // lane bit 4: odd and even 16-lane rows of each half
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(acc[i]), __float_as_uint(acc[8 + i]), false, false);
    acc[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  {
    const bool up = (lane >> 3) & 1;  // lane bit 3: row rotation by 8
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float send = up ? acc[i] : acc[4 + i];
      const float keep = up ? acc[4 + i] : acc[i];
      acc[i] = keep + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(send), 0x128, 0xf, 0xf, false));
    }
  }
  double v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = (double)acc[k];
#pragma unroll
  for (int k = 0; k < kNodes; ++k) acc[k] = 0.0f;
  {
    const bool up = (lane >> 2) & 1;  // lane bit 2
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const double send = up ? v[i] : v[2 + i];
      const double keep = up ? v[2 + i] : v[i];
      v[i] = keep + __shfl_xor(send, 4, kWave);
    }
  }
  {
    const bool up = (lane >> 1) & 1;  // lane bit 1
    const double send = up ? v[0] : v[1];
    const double keep = up ? v[1] : v[0];
    v[0] = keep + __shfl_xor(send, 2, kWave);
  }
  v[0] += __shfl_xor(v[0], 1, kWave);  // lane bit 0
  const int j = (lane >> 1) & 15;
  if ((lane & 1) == 0) node[lane < 32 ? j : kMidNodes - 1 - j] += v[0];
}

// One far segment of a span of S points: lines [i0, i1), one per lane, at its NN nodes; the
// node sums go to node[] (see far_flush).
template <int S, int NN>
__device__ __forceinline__ void far_segment(const VoigtArgs& a, const PairDesc& pd, const float* __restrict__ S_T,
                                            const float* __restrict__ gT, int i0, int i1, int lane, double nu_a,
                                            double nu_b, double* node) {
  const float inv_dnu = (float)(1.0 / pd.dnu);
  float acc[NN];
#pragma unroll
  for (int k = 0; k < NN; ++k) acc[k] = 0.0f;
  int n = 0;
  for (int b = i0; b < i1; b += kWave) {
    const int li = b + lane;
    const bool valid = li < i1;
    const FarLine f = far_line(valid, valid ? a.nu[li] : 0.0, valid ? S_T[li] : 0.0f, valid ? gT[li] : 0.0f, pd,
                               nu_a, nu_b, inv_dnu, a.zK);
    far_accumulate<NN>(SpanNodes<S, NN>(), f, acc);
    if (++n == 16 || b + kWave >= i1) {
      far_flush<NN>(acc, lane, node);
      n = 0;
    }
  }
}

// One middle-distance segment: lines [i0, i1), each on two lanes (lane and lane + 32), at the
// span's kMidNodes nodes. The nodes are symmetric (x_(31-j) = S - 1 - x_j), so the upper half
// evaluates node 31 - j as node j with the step negated and the offset moved by S - 1 steps,
// and each lane keeps kNodes sums (see mid_flush).
template <int S>
__device__ __forceinline__ void mid_segment(const VoigtArgs& a, const PairDesc& pd, const float* __restrict__ S_T,
                                            const float* __restrict__ gT, int i0, int i1, int lane, double nu_a,
                                            double nu_b, double* node) {
  const float inv_dnu = (float)(1.0 / pd.dnu);
  const bool upper = lane >= 32;
  float acc[kNodes];
#pragma unroll
  for (int k = 0; k < kNodes; ++k) acc[k] = 0.0f;
  int n = 0;
  for (int b = i0; b < i1; b += 32) {
    const int li = b + (lane & 31);
    const bool valid = li < i1;
    FarLine f = far_line(valid, valid ? a.nu[li] : 0.0, valid ? S_T[li] : 0.0f, valid ? gT[li] : 0.0f, pd, nu_a,
                         nu_b, inv_dnu, a.zK);
    if (upper) {
      f.e = __builtin_fmaf((float)(S - 1), f.h, f.e);
      f.h = -f.h;
    }
    far_accumulate<kNodes>(SpanNodes<S, kMidNodes>(), f, acc);
    if (++n == 16 || b + 32 >= i1) {
      mid_flush(acc, lane, node);
      n = 0;
    }
  }
}

// One masked segment of a span of W = 64 P points: far lines whose cut bound falls on the span,
// one per lane, at the span's kMaskNodes nodes. A line adds its interpolant to the points
// 0..b (LEFT: b = its last point inside the cut) or b..W-1 (b = its first), so the node values
// are summed per bound b (over the lanes of each bound present in the batch, by a butterfly;
// bound b's sums are held by lane b mod 64 in slot b / 64), and at the end each point j takes
// the sums of the bounds b >= j (LEFT) or b <= j (a scan over the points) and interpolates them.
template <int P, bool LEFT>
__device__ __forceinline__ void masked_segment(const VoigtArgs& a, const PairDesc& pd, const float* __restrict__ S_T,
                                               const float* __restrict__ gT, const int4* __restrict__ grec, int i0,
                                               int i1, int lane, int64_t span0, double nu_a, double nu_b,
                                               float (&part)[P]) {
  constexpr int W = kWave * P;
  const float inv_dnu = (float)(1.0 / pd.dnu);
  float B[kMaskNodes][P];
#pragma unroll
  for (int k = 0; k < kMaskNodes; ++k)
#pragma unroll
    for (int p = 0; p < P; ++p) B[k][p] = 0.0f;
  for (int b0 = i0; b0 < i1; b0 += kWave) {
    const int li = b0 + lane;
    const bool valid = li < i1;
    const FarLine f = far_line(valid, valid ? a.nu[li] : 0.0, valid ? S_T[li] : 0.0f, valid ? gT[li] : 0.0f, pd,
                               nu_a, nu_b, inv_dnu, a.zK);
    // LEFT: the line reaches points 0..bnd; otherwise bnd..W-1 (live: at least one point)
    int bnd = 0;
    bool live = false;
    if (valid) {
      const int4 gr = grec[li];
      if (gr.z <= gr.w) {
        const int64_t e = LEFT ? (int64_t)gr.w - span0 : (int64_t)gr.z - span0;
        live = LEFT ? e >= 0 : e <= W - 1;
        bnd = (int)(LEFT ? (e > W - 1 ? W - 1 : e) : (e < 0 ? 0 : e));
      }
    }
    float v[kMaskNodes];
#pragma unroll
    for (int k = 0; k < kMaskNodes; ++k) v[k] = 0.0f;
    const int Kw = wave_order(f);
    const SpanNodes<W, kMaskNodes> xs;
    if (Kw == 1) far_nodes<1, 0, kMaskNodes, SpanNodes<W, kMaskNodes>, kMaskNodes>(xs, f, v);
    else if (Kw == 2) far_nodes<2, 0, kMaskNodes, SpanNodes<W, kMaskNodes>, kMaskNodes>(xs, f, v);
    else if (Kw == 3) far_nodes<3, 0, kMaskNodes, SpanNodes<W, kMaskNodes>, kMaskNodes>(xs, f, v);
    else if (Kw == 4) far_nodes<4, 0, kMaskNodes, SpanNodes<W, kMaskNodes>, kMaskNodes>(xs, f, v);
    else far_nodes<5, 0, kMaskNodes, SpanNodes<W, kMaskNodes>, kMaskNodes>(xs, f, v);
    // the bounds present, in lane order of their first line
    uint64_t rem = __ballot(live);
    while (rem) {
      const int bs = __builtin_amdgcn_readlane(bnd, (int)__builtin_ctzll(rem));
      const bool in = live && bnd == bs;
      rem &= ~__ballot(in);
#pragma unroll
      for (int k = 0; k < kMaskNodes; ++k) {
        const float t = wave_sum64f(in ? v[k] : 0.0f);
#pragma unroll
        for (int p = 0; p < P; ++p)
          if (p * kWave + lane == bs) B[k][p] += t;
      }
    }
  }
  // scan over the points (LEFT: sums of the bounds >= j; otherwise <= j), then interpolation
  float out[P];
#pragma unroll
  for (int p = 0; p < P; ++p) out[p] = 0.0f;
#pragma unroll
  for (int k = 0; k < kMaskNodes; ++k) {
    float carry = 0.0f;
#pragma unroll
    for (int pp = 0; pp < P; ++pp) {
      const int p = LEFT ? P - 1 - pp : pp;
      float x = B[k][p];
#pragma unroll
      for (int off = 1; off < kWave; off <<= 1) {
        const float t = LEFT ? __shfl_down(x, off, 64) : __shfl_up(x, off, 64);
        if (LEFT ? lane + off < kWave : lane >= off) x += t;
      }
      const float tot = __shfl(x, LEFT ? 0 : kWave - 1, 64);
      x += carry;
      carry += tot;
      out[p] = __builtin_fmaf(x, a.mask_w[k * W + p * kWave + lane], out[p]);
    }
  }
#pragma unroll
  for (int p = 0; p < P; ++p) part[p] += out[p];
}

// ------------------------------------------------------------------- wing pass
// One wave per span of 64 P grid points (lane + 64 p, p < P). A work item is a span and a
// chunk of its line segments (k_span_segments), taken in list order:
//  * a direct segment is staged 64 lines at a time in the wave's LDS (one line per lane),
//    and every staged line that reaches the span is evaluated at all its points with the
//    series order it needs there (lanes outside its cut range and its core points add
//    nothing; the core points are the line-core pass's), in staging order, into per-lane
//    FP32 sums with a compensated flush every 16 lines;
//  * a far, very far or middle segment is evaluated at the span's kNodes, kFar8Nodes or
//    kMidNodes Chebyshev nodes, one line per lane (two for middle lines; per lane in FP32 over
//    16 lines, then FP64; over the wave by a butterfly, the same on every lane), and the node
//    sums are interpolated to the span's points in FP64 at the end of the item;
//  * a masked segment is evaluated at kMaskNodes nodes and added to the prefix or suffix of
//    the span's points inside each line's cut (masked_segment).
// A span with one item writes k; otherwise each item writes its partial span and k_combine
// sums them in item order. No workgroup barrier: waves run independently.
template <int P>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(P <= 4 ? 6 : 4))) void k_wing(VoigtArgs a) {
  constexpr int W = kWave * P;  // span width in grid points
  __shared__ WaveLDS L;
  const int lane = threadIdx.x;
  const int total = a.item_base[a.n_tiles_total];
  const float jl0 = (float)lane;  // this lane's first span point
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  long long n_direct = 0, n_node = 0, n_mid = 0, n_mask = 0, n_far8 = 0;

  for (;;) {
    int mine = 0;
    if (lane == 0) mine = atomicAdd(a.counter, 1);
    const int it = __builtin_amdgcn_readfirstlane(mine);
    if (it >= total) break;
    int g = 0;
    {
      int lo = 0, hi = a.n_tiles_total - 1;  // last span with item_base <= it
      while (lo < hi) {
        const int m = (lo + hi + 1) >> 1;
        if (a.item_base[m] <= it) lo = m; else hi = m - 1;
      }
      g = lo;
    }
    const PairDesc pd = wave_uniform(a.pairs[find_pair(a.pairs, a.n_pairs, g)]);
    const int nc = a.tile_nc[g];
    const int v_lo = (it - a.item_base[g]) * a.chunk;
    const int64_t span0 = (int64_t)(g - pd.tile_base) * W;
    const float* __restrict__ S_T = a.S_T + (int64_t)pd.tidx * a.N;
    const float* __restrict__ gT = a.gT + (int64_t)pd.tidx * a.N;
    const int4* __restrict__ grec = a.grec + (int64_t)pd.gidx * a.N;
    const SpanSeg* __restrict__ sg = a.segs + g;
    const int nseg = sg->n;

    float s[P], cc[P], part[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
      s[p] = 0.0f;
      cc[p] = 0.0f;
      part[p] = 0.0f;
    }
    if (lane < kNodes) L.node[lane] = 0.0;
    if (lane < kFar8Nodes) L.node8[lane] = 0.0;
    if (lane < kMidNodes) L.node_mid[lane] = 0.0;
    bool any_far = false, any_far8 = false, any_mid = false;
    int cum = 0, v_hi = v_lo;
    for (int q = 0; q < nseg; ++q) {
      const int len = sg->len[q];
      const int x0 = v_lo > cum ? v_lo : cum;
      const int x1 = (v_lo + a.chunk < cum + len) ? v_lo + a.chunk : cum + len;
      if (x0 < x1) {
        const int i0 = sg->lo[q] + (x0 - cum), i1 = i0 + (x1 - x0);
        v_hi = x1;
        const int kind = sg->kind[q];
        if (W <= kMaskMaxSpan && (kind == kSegMaskLeft || kind == kSegMaskRight)) {
          // ---- masked segment: bound-bucketed node sums, one line per lane
          n_mask += i1 - i0;
          const double nu_a = grid_nu(pd.nu_start, pd.dnu, span0);
          const double nu_b = grid_nu(pd.nu_start, pd.dnu, span0 + W - 1);
          if (kind == kSegMaskLeft) masked_segment<P, true>(a, pd, S_T, gT, grec, i0, i1, lane, span0, nu_a, nu_b, part);
          else masked_segment<P, false>(a, pd, S_T, gT, grec, i0, i1, lane, span0, nu_a, nu_b, part);
          kahan_flush<P>(part, s, cc);
        } else if (kind == kSegFar || kind == kSegFar8 || kind == kSegMid) {
          // ---- far or middle segment: node sums, one line per lane
          n_node += i1 - i0;
          const double nu_a = grid_nu(pd.nu_start, pd.dnu, span0);
          const double nu_b = grid_nu(pd.nu_start, pd.dnu, span0 + W - 1);
          if (kind == kSegFar) {
            any_far = true;
            far_segment<W, kNodes>(a, pd, S_T, gT, i0, i1, lane, nu_a, nu_b, L.node);
          } else if (kind == kSegFar8) {
            any_far8 = true;
            n_far8 += i1 - i0;
            far_segment<W, kFar8Nodes>(a, pd, S_T, gT, i0, i1, lane, nu_a, nu_b, L.node8);
          } else {
            any_mid = true;
            n_mid += i1 - i0;
            mid_segment<W>(a, pd, S_T, gT, i0, i1, lane, nu_a, nu_b, L.node_mid);
          }
        } else {
          // ---- direct segment: 64 lines per stage
          for (int b = i0; b < i1; b += kWave) {
            const int li = b + lane;
            uint32_t code = 0u;
            if (li < i1)
              code = stage_span_line<P>(L, lane, grec[li], a.nu[li], S_T[li], gT[li], pd, a.zw, a.zcore, span0);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // group the staged lines (wave ballots; staging order within a group)
            int o[kDirectGroups + 2];
            {
              const int grp = direct_group(code);
              o[1] = 0;
#pragma unroll
              for (int gg = 1; gg <= kDirectGroups; ++gg) {
                const uint64_t m = __ballot(grp == gg);
                if (grp == gg) L.list[o[gg] + (int)__popcll(m & lt)] = (uint8_t)lane;
                o[gg + 1] = o[gg] + (int)__popcll(m);
              }
            }
            n_direct += o[kDirectGroups + 1] - o[1];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            direct_loop<P, 1, false>(L, o[1], o[2], jl0, part, s, cc);
            direct_loop<P, 2, false>(L, o[2], o[3], jl0, part, s, cc);
            direct_loop<P, 3, false>(L, o[3], o[4], jl0, part, s, cc);
            direct_loop<P, 4, false>(L, o[4], o[5], jl0, part, s, cc);
            direct_loop<P, 1, true>(L, o[5], o[6], jl0, part, s, cc);
            direct_loop<P, 2, true>(L, o[6], o[7], jl0, part, s, cc);
            direct_loop<P, 3, true>(L, o[7], o[8], jl0, part, s, cc);
            direct_loop<P, 4, true>(L, o[8], o[9], jl0, part, s, cc);
            for (int i = o[9]; i < o[10]; ++i) {
              wing_line_order5<P>(L, __builtin_amdgcn_readfirstlane((int)L.list[i]), jl0, part);
              if (((i - o[9]) & 15) == 15) kahan_flush<P>(part, s, cc);
            }
            kahan_flush<P>(part, s, cc);
            for (int i = o[10]; i < o[11]; ++i) {
              const int l = __builtin_amdgcn_readfirstlane((int)L.list[i]);
              wing_line_order9<P>(L, l, (uint32_t)__builtin_amdgcn_readlane((int)code, l), jl0, part);
              if (((i - o[10]) & 15) == 15) kahan_flush<P>(part, s, cc);
            }
            kahan_flush<P>(part, s, cc);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          }
          kahan_flush<P>(part, s, cc);
        }
      }
      cum += len;
    }
    (void)v_hi;
    // ---- far and middle lines: interpolation of the node sums to the span's points, in FP64
    if (any_far || any_far8 || any_mid) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      double v[P];
#pragma unroll
      for (int p = 0; p < P; ++p) v[p] = 0.0;
      if (any_far) {
#pragma unroll 1
        for (int k = 0; k < kNodes; ++k) {
          const double ns = L.node[k];
          const double* __restrict__ wk = a.cheb_w + k * W + lane;
#pragma unroll
          for (int p = 0; p < P; ++p) v[p] = fma(ns, wk[p * kWave], v[p]);
        }
      }
      if (any_far8) {
#pragma unroll 1
        for (int k = 0; k < kFar8Nodes; ++k) {
          const double ns = L.node8[k];
          const double* __restrict__ wk = a.far8_w + k * W + lane;
#pragma unroll
          for (int p = 0; p < P; ++p) v[p] = fma(ns, wk[p * kWave], v[p]);
        }
      }
      if (any_mid) {
#pragma unroll 1
        for (int k = 0; k < kMidNodes; ++k) {
          const double ns = L.node_mid[k];
          const double* __restrict__ wk = a.mid_w + k * W + lane;
#pragma unroll
          for (int p = 0; p < P; ++p) v[p] = fma(ns, wk[p * kWave], v[p]);
        }
      }
#pragma unroll
      for (int p = 0; p < P; ++p) part[p] += (float)v[p];
      kahan_flush<P>(part, s, cc);
    }
    // ---- output: the span directly, or this item's partial span
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int local = p * kWave + lane;
      const float v = s[p] - cc[p];
      if (nc == 1) {
        if (span0 + local < pd.n) a.k[pd.out_off + span0 + local] = v;
      } else if (it < a.items_cap) {
        a.partial[((int64_t)it) * W + local] = v;
      }
    }
    // an item beyond the partial rows (the host bound is a proof, so never expected): flagged,
    // and the combine writes NaN over its span
    if (nc != 1 && it >= a.items_cap && a.status && lane == 0) atomicOr(a.status, 1);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  // evaluations made, per class: [0] direct (every point of the span), [1] far (kNodes nodes),
  // [2] very far (kFar8Nodes), [3] middle (kMidNodes), [4] masked (kMaskNodes)
  if (a.stats && lane == 0) {
    const int nb = gridDim.x;
    a.stats[blockIdx.x] = n_direct * W;
    a.stats[nb + blockIdx.x] = (n_node - n_mid - n_far8) * kNodes;
    a.stats[2 * nb + blockIdx.x] = n_far8 * kFar8Nodes;
    a.stats[3 * nb + blockIdx.x] = n_mid * kMidNodes;
    a.stats[4 * nb + blockIdx.x] = n_mask * kMaskNodes;
  }
}


// --------------------------------------------------------------- tile-far pass
// The lines of a tile's tile-far ranges (see k_worklist), far from the whole tile (4 spans),
// are evaluated at the tile's Chebyshev nodes (far_line, far_accumulate). A work item is a tile
// and a chunk of its tile-far lines; it writes its kNodes node sums (per lane in FP32 over 16
// lines, then FP64; over the workgroup in a fixed order), and k_combine_far adds their
// interpolation to the tile.
template <int C>
__global__ __launch_bounds__(kThreads) void k_far(FarArgs a) {
  constexpr int NN = C == 0 ? kNodes : kFar8Nodes;
  __shared__ double sRed[kWavesPerWG][NN];
  __shared__ int sItem, sTile, sPair;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int32_t* __restrict__ item_base = a.item_base[C];
  const int total = item_base[a.n_tiles_total];
  long long n_lines = 0;
  for (;;) {
    if (tid == 0) {
      const int it = atomicAdd(a.counter[C], 1);
      sItem = it;
      if (it < total) {
        int lo = 0, hi = a.n_tiles_total - 1;  // last tile with item_base <= it
        while (lo < hi) {
          const int m = (lo + hi + 1) >> 1;
          if (item_base[m] <= it) lo = m; else hi = m - 1;
        }
        sTile = lo;
        sPair = find_pair(a.pairs, a.n_pairs, lo);
      }
    }
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(sItem);
    if (it >= total) break;
    const int g = __builtin_amdgcn_readfirstlane(sTile);
    const PairDesc pd = wave_uniform(a.pairs[__builtin_amdgcn_readfirstlane(sPair)]);
    const int ibase = __builtin_amdgcn_readfirstlane(item_base[g]);
    const int4 tf = wave_uniform(a.tile_far[2 * g + C]);
    const int nl = tf.y - tf.x, nv = nl + (tf.w - tf.z);
    const int v_lo = (it - ibase) * a.chunk;
    const int v_hi = v_lo + a.chunk < nv ? v_lo + a.chunk : nv;
    n_lines += v_hi > v_lo ? v_hi - v_lo : 0;
    const int64_t tile0 = (int64_t)(g - pd.tile_base) * a.W;
    const double nu0 = grid_nu(pd.nu_start, pd.dnu, tile0);
    const double nu1 = grid_nu(pd.nu_start, pd.dnu, tile0 + a.W - 1);
    const float inv_dnu = (float)(1.0 / pd.dnu);
    const float* __restrict__ S_T = a.S_T + (int64_t)pd.tidx * a.N;
    const float* __restrict__ gT = a.gT + (int64_t)pd.tidx * a.N;

    float acc[NN];
#pragma unroll
    for (int k = 0; k < NN; ++k) acc[k] = 0.0f;
    if (lane < NN) sRed[wv][lane] = 0.0;
    int n = 0;
    for (int b = v_lo; b < v_hi; b += kThreads) {
      const int v = b + tid;
      const bool valid = v < v_hi;
      const int64_t li = v < nl ? (int64_t)tf.x + v : (int64_t)tf.z + (v - nl);
      const FarLine f = far_line(valid, valid ? a.nu[li] : 0.0, valid ? S_T[li] : 0.0f, valid ? gT[li] : 0.0f,
                                 pd, nu0, nu1, inv_dnu, a.zK);
      far_accumulate<NN>(ArgNodes{C == 0 ? a.tile_x : a.tile_x8}, f, acc);
      if (++n == 16 || b + kThreads >= v_hi) {
        far_flush<NN>(acc, lane, sRed[wv]);
        n = 0;
      }
    }
    __syncthreads();
    if (tid < NN) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < kWavesPerWG; ++w) t += sRed[w][tid];
      if (it < a.items_cap[C]) a.node_part[C][(int64_t)it * NN + tid] = t;
      else if (a.status && tid == 0) atomicOr(a.status, 1);
    }
    __syncthreads();
  }
  if (a.stats && tid == 0) a.stats[C * gridDim.x + blockIdx.x] = n_lines * NN;
}

// k += interpolation onto the tile of the fixed-order (class 0 then 1; item 0, 1, ...) sums of
// its node sums.
__global__ __launch_bounds__(kThreads) void k_combine_far(FarArgs a) {
  __shared__ double ns[kNodes + kFar8Nodes];
  const int g = blockIdx.x;
  const int b0 = a.item_base[0][g], n0 = a.item_base[0][g + 1] - b0;
  const int b1 = a.item_base[1][g], n1 = a.item_base[1][g + 1] - b1;
  if (n0 <= 0 && n1 <= 0) return;
  const PairDesc pd = a.pairs[find_pair(a.pairs, a.n_pairs, g)];
  // items beyond the node-sum rows were not stored (flagged by k_far): the tile gets NaN
  const bool lost = b0 + n0 > a.items_cap[0] || b1 + n1 > a.items_cap[1];
  if (threadIdx.x < kNodes) {
    double t = 0.0;
    for (int c = 0; c < n0 && b0 + c < a.items_cap[0]; ++c) t += a.node_part[0][(int64_t)(b0 + c) * kNodes + threadIdx.x];
    ns[threadIdx.x] = lost ? NAN : t;
  } else if (threadIdx.x < kNodes + kFar8Nodes) {
    const int k = threadIdx.x - kNodes;
    double t = 0.0;
    for (int c = 0; c < n1 && b1 + c < a.items_cap[1]; ++c) t += a.node_part[1][(int64_t)(b1 + c) * kFar8Nodes + k];
    ns[threadIdx.x] = lost ? NAN : t;
  }
  __syncthreads();
  const int64_t tile0 = (int64_t)(g - pd.tile_base) * a.W;
  for (int local = threadIdx.x; local < a.W; local += kThreads) {
    if (tile0 + local >= pd.n) continue;
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < kNodes; ++k) v = fma(ns[k], a.tile_w[0][k * a.W + local], v);
#pragma unroll
    for (int k = 0; k < kFar8Nodes; ++k) v = fma(ns[kNodes + k], a.tile_w[1][k * a.W + local], v);
    float* dst = a.k + pd.out_off + tile0 + local;
    *dst = (float)((double)*dst + v);
  }
}

// ------------------------------------------------------------------- core pass
// The core points of every line (|z| below the last series threshold, within the cut) are
// evaluated here, after the wing pass and its combine. A workgroup is one wave and owns a
// core tile of 64 P grid points; its work list holds the lines whose centre lies within the
// largest core half-width of the tile. The wave stages 64 lines at a time (one per lane; the
// next batch is loaded while the current one is queued), appends the (line, point) pairs of
// lines with core points on the tile to a queue held in registers (one pair per lane, with
// the line's constants; a position finds its line by a bit count of the line starts below it),
// evaluates 64 pairs at a time with the FP32 rational approximation,
// and adds them to its LDS accumulator one line segment at a time (a line's
// pairs are contiguous in the queue and have distinct points, so each segment is one
// conflict-free update, applied in line order). Every 8 rounds the accumulator goes into
// compensated per-lane sums. No workgroup barrier couples waves with unequal work.
template <int P>
struct CoreLDS {
  float acc[kWave * P];
  // the staged batch, one entry per line with pairs on the tile (its slot: such lines in lane
  // order), in units of alpha: offset of the reference point (from the grid record's offset,
  // subtracted in FP64) and grid step; y = gamma/alpha; the tile-local point of the line's pair g
  // minus g, tile-local reference point, amplitude
  float x0[kWave], h[kWave], y[kWave];
  // for a line whose peak falls between grid points (its reference point more than a quarter of
  // max(alpha, gamma) from the centre; its amplitude is stored negated): its FP64 offset and
  // 1/alpha
  double d64[kWave], ia64[kWave];
  int off[kWave], jr[kWave];  // (256-byte aligned: one address reads both)
  float amp[kWave];
  int ex[kWave];    // the first pair of each line (slot) in the batch's staging order
  int mark[kWave];  // queue positions where a line starts inside a fill: the fill's tag
  double w64[kWeidN40];  // the FP64 Weideman coefficients (40 terms)
};

template <int P>
__device__ __forceinline__ void core_round(CoreLDS<P>& L, int lane, int qn, uint64_t segs, float qx, float qxlo,
                                           float qy, float qa, int qj) {
  // a round with a pair of a line whose peak falls between grid points (marked by a negative
  // amplitude; its x is qx + qxlo to FP64 precision) is evaluated in FP64, every lane (the
  // round's branch stays uniform). Lanes at and above qn evaluate what they hold from an earlier
  // round (finite values, or the zeros they start with) and add nothing.
  const uint64_t qmask = (qn >= 64) ? ~0ull : ((1ull << qn) - 1ull);
  const bool any64 = (__builtin_amdgcn_ballot_w64(qa < 0.0f) & qmask) != 0ull;
  float v;
  if (any64) {
    asm volatile("" ::: "memory");  // the FP64 coefficients are read from LDS here, not held
    const double xlo = qa < 0.0f ? (double)qxlo : 0.0;  // qxlo is set for marked pairs only
    v = fabsf(qa) * (float)weideman_re64((double)qx + xlo, (double)qy, L.w64);
  } else {
    v = qa * weideman_re32(qx, qy);
  }
  // one conflict-free LDS update per line segment, in queue (line) order. Position 0 always
  // starts a segment, so a lane's segment is the number of starts at positions 1 .. lane (lanes
  // at and above qn count as further starts: their segments lie beyond the last); a line's pairs
  // have distinct points, and the LDS operations of a wave (its workgroup) complete in order.
  // (LDS atomic adds in place of the read and write were much slower here.)
  const int nseg = __popcll(segs & qmask);
  const uint64_t above = (segs | ~qmask) >> 1;
  const int sid = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(above >> 32),
                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)above, 0u));
  for (int k = 0; k < nseg; ++k)
    if (sid == k) L.acc[qj] += v;
}

template <int P>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(P == 2 ? 8 : (P == 1 ? 7 : (P == 4 ? 6 : 5))))) void k_core(VoigtArgs a) {
  constexpr int W = kWave * P;  // core tile width in grid points
  __shared__ CoreLDS<P> L;
  const int lane = threadIdx.x;
#pragma unroll
  for (int p = 0; p < P; ++p) L.acc[p * kWave + lane] = 0.0f;
  if (lane < kWeidN40) L.w64[lane] = c_weid40[lane];
  L.mark[lane] = -1;
  int tag = 0;  // the fills' tags, one per fill over the wave's lifetime
  const int total = a.item_base[a.n_tiles_total];
  const float zc = a.zcore;
  long long ncore = 0;  // core evaluations of this wave (statistics only)

  for (;;) {
    int itv = 0;
    if (lane == 0) itv = atomicAdd(a.counter + 1, 1);
    const int it = __builtin_amdgcn_readfirstlane(__shfl(itv, 0));
    if (it >= total) break;
    int lo = 0, hi = a.n_tiles_total - 1;  // last tile with item_base <= it
    while (lo < hi) {
      const int m = (lo + hi + 1) >> 1;
      if (__builtin_amdgcn_readfirstlane(a.item_base[m]) <= it) lo = m; else hi = m - 1;
    }
    const int g = lo;
    const PairDesc pd = wave_uniform(a.pairs[find_pair(a.pairs, a.n_pairs, g)]);
    const int ibase = __builtin_amdgcn_readfirstlane(a.item_base[g]);
    const int nc = __builtin_amdgcn_readfirstlane(a.tile_nc[g]);
    const int64_t tile0 = (int64_t)(g - pd.tile_base) * W;
    const int64_t line_lo = (int64_t)__builtin_amdgcn_readfirstlane(a.tile_lo[g]) + (int64_t)(it - ibase) * a.chunk;
    int64_t line_hi = line_lo + a.chunk;
    const int64_t thi = __builtin_amdgcn_readfirstlane(a.tile_hi[g]);
    if (line_hi > thi) line_hi = thi;
    const float* __restrict__ S_T = a.S_T + (int64_t)pd.tidx * a.N;
    const float* __restrict__ gT = a.gT + (int64_t)pd.tidx * a.N;
    const int4* __restrict__ grec = a.grec + (int64_t)pd.gidx * a.N;
    const float inv_dnu = (float)(1.0 / pd.dnu);

    float s[P], cc[P], part[P];
#pragma unroll
    for (int p = 0; p < P; ++p) { s[p] = 0.0f; cc[p] = 0.0f; part[p] = 0.0f; }
    bool any = false;
    int rounds = 0;
    // the queue: lane k < qn holds one pair (x, y, amplitude, tile-local point)
    int qn = 0;
    uint64_t segs = 0ull;  // lanes where a line's segment starts
    float qx = 0.0f, qxlo = 0.0f, qy = 0.0f;
    float qa = 0.0f;
    int qj = 0;

    auto flush_acc = [&]() {
#pragma unroll
      for (int p = 0; p < P; ++p) {
        part[p] += L.acc[p * kWave + lane];
        L.acc[p * kWave + lane] = 0.0f;
      }
      kahan_flush<P>(part, s, cc);
    };
    auto run_round = [&]() {
      core_round<P>(L, lane, qn, segs, qx, qxlo, qy, qa, qj);
      ncore += qn;
      qn = 0;
      segs = 0ull;
      any = true;
      if (++rounds == 8) {
        flush_acc();
        rounds = 0;
      }
    };

    // software pipeline: the next batch's line data is loaded before the current one is queued
    int4 nx_gr = make_int4(0, 0, 1, 0);
    float nx_S = 0.0f, nx_g = 0.0f;
    double nx_nu = 1.0;
    if (line_lo + lane < line_hi) {
      const int64_t li = line_lo + lane;
      nx_gr = grec[li]; nx_S = S_T[li]; nx_g = gT[li]; nx_nu = a.nu[li];
    }
    for (int64_t b = line_lo; b < line_hi; b += kWave) {
      const int4 gr = nx_gr;
      const float S = nx_S, gTv = nx_g;
      const double nu0 = nx_nu;
      const bool valid = b + lane < line_hi;
      if (b + kWave + lane < line_hi) {
        const int64_t li = b + kWave + lane;
        nx_gr = grec[li]; nx_S = S_T[li]; nx_g = gT[li]; nx_nu = a.nu[li];
      }
      // this lane's line: its core points on the tile (tile-local, inclusive)
      int czl = 1, czh = 0;
      float lx0 = 0.0f, lh = 0.0f, ly = 0.0f;
      float lamp = 0.0f;
      double ld64 = 0.0, lia64 = 0.0;
      const int jref = gr.y, jlo = gr.z, jhi = gr.w;
      if (valid && S > 0.0f && jlo <= jhi) {
        const float alpha = (float)(nu0 * pd.beta);
        const float gam = gTv * (float)pd.pfac;
        int rlo, rhi;
        if (core_rel(alpha, gam, __int_as_float(gr.x), inv_dnu, zc, rlo, rhi)) {
          int64_t gl = (int64_t)jref + rlo, gh = (int64_t)jref + rhi;
          if (gl < jlo) gl = jlo;
          if (gh > jhi) gh = jhi;
          if (gl < tile0) gl = tile0;
          if (gh > tile0 + W - 1) gh = tile0 + W - 1;
          if (gh > pd.n - 1) gh = pd.n - 1;
          if (gl <= gh) {
            czl = (int)(gl - tile0);
            czh = (int)(gh - tile0);
            const float ia = 1.0f / alpha;
            lamp = S * ia * 0.564189583547756287f;  // S/(sqrt(pi) alpha)
            lx0 = __int_as_float(gr.x) * ia;
            lh = (float)pd.dnu * ia;
            ly = gam * ia;
            if (fabsf(__int_as_float(gr.x)) > 0.25f * (alpha > gam ? alpha : gam)) {
              lia64 = 1.0 / (nu0 * pd.beta);
              ld64 = __dsub_rn(grid_nu(pd.nu_start, pd.dnu, (int64_t)jref), a.nu_pos ? a.nu_pos[b + lane] : nu0);
              lamp = -lamp;  // marks the line's pairs for the FP64 rounds
            }
          }
        }
      }
      const int jrl = (int)((int64_t)jref - tile0);
      // the batch's pairs in staging order: line l (lane l) holds pairs excl .. incl - 1
      const int nl = czl <= czh ? czh - czl + 1 : 0;
      int incl = nl;
      // the lane index is made opaque here, so that the shuffles' lane addresses are formed per
      // batch rather than held in registers across the loop (where they were spilled)
      int ls = lane;
      asm volatile("" : "+v"(ls));
#pragma unroll
      for (int d = 1; d < kWave; d <<= 1) {
        const int t = __builtin_amdgcn_ds_bpermute((ls - d) << 2, incl);  // lanes below d: masked
        if (ls >= d) incl += t;
      }
      const int T = __builtin_amdgcn_readlane(incl, kWave - 1);
      if (T == 0) continue;
      const int excl = incl - nl;
      // the lines with pairs, compacted into slots in lane order (their first pairs increase)
      const uint64_t hasp = __builtin_amdgcn_ballot_w64(nl > 0);
      const int nslots = __popcll(hasp);
      if (nl > 0) {
        const int sl = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(hasp >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)hasp, 0u));
        L.off[sl] = czl - excl;
        L.jr[sl] = jrl;
        L.amp[sl] = lamp;
        L.x0[sl] = lx0;
        L.h[sl] = lh;
        L.y[sl] = ly;
        L.d64[sl] = ld64;
        L.ia64[sl] = lia64;
        L.ex[sl] = excl;
      }
      // lane s: the first pair of slot s (none beyond the last slot)
      const int exs = lane < nslots ? ((volatile __attribute__((address_space(3))) int*)L.ex)[lane] : 0x7fffffff;
      const int exs1 = exs - 1;
      // fills: pairs g0 .. g0 + take - 1 go to queue positions qn .. qn + take - 1
      for (int g0 = 0; g0 < T;) {
        const int take = (T - g0) < (kWave - qn) ? (T - g0) : (kWave - qn);
        // a line that starts inside the fill (after its first pair) marks its queue position with
        // this fill's tag. LDS operations of a wave stay in order; the accesses are volatile so
        // that the compiler keeps every one of them (a lane reads marks that other lanes wrote,
        // which it cannot see)
        volatile __attribute__((address_space(3))) int* mark = (volatile __attribute__((address_space(3))) int*)L.mark;
        ++tag;
        const int t1 = exs1 - g0;  // the line's start after pair g0, less one
        if ((unsigned)t1 < (unsigned)(take - 1)) mark[t1 + qn + 1] = tag;
        const uint64_t inner = __builtin_amdgcn_ballot_w64(mark[lane] == tag);  // positions qn+1 ..
        // the slot of the line of pair g0 (slot 0 starts at pair 0)
        const int cur = __popcll(__builtin_amdgcn_ballot_w64(exs <= g0)) - 1;
        segs |= inner | (1ull << qn);  // position qn starts a segment
        const int r = lane - qn;
        if ((unsigned)r < (unsigned)take) {
          // this position's line: cur plus the starts at positions qn+1 .. lane
          const uint64_t sh = inner >> 1;
          const int li = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(sh >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)sh, (uint32_t)cur));
          const int j = g0 + r + L.off[li];
          qj = j;
          qx = __builtin_fmaf((float)(j - L.jr[li]), L.h[li], L.x0[li]);
          qy = L.y[li];
          qa = L.amp[li];  // negative: a line whose peak falls between grid points
          if (qa < 0.0f) {  // its x to FP64 precision, as qx + qxlo
            const double x64 = ((double)(j - L.jr[li]) * pd.dnu + L.d64[li]) * L.ia64[li];
            qx = (float)x64;
            qxlo = (float)(x64 - (double)qx);
          }
        }
        qn += take;
        g0 += take;
        if (qn == kWave) run_round();
      }
    }
    if (qn > 0) run_round();
    flush_acc();

    // single-item tiles add their core sums to k (the wing pass and its combine are done);
    // items of split tiles store theirs for the fixed-order core combine
    if (nc == 1) {
      if (any) {
#pragma unroll
        for (int p = 0; p < P; ++p) {
          const int local = p * kWave + lane;
          if (tile0 + local < pd.n) {
            float* dst = a.k + pd.out_off + tile0 + local;
            *dst = *dst + (s[p] - cc[p]);
          }
        }
      }
    } else if (it < a.items_cap) {
      // the address is formed here (an opaque lane), not held in registers across the item loop
      int ls = lane;
      asm volatile("" : "+v"(ls));
#pragma unroll
      for (int p = 0; p < P; ++p) a.partial[(int64_t)it * W + p * kWave + ls] = s[p] - cc[p];
    } else if (a.status && lane == 0) {
      atomicOr(a.status, 1);
    }
  }
  if (a.stats && lane == 0) a.stats[blockIdx.x] = ncore;
}

// --------------------------------------------------- line profiles, plinth and cut options
// The four line profiles of Sec. 2.1, per unit strength at offset d from the line centre:
//   Voigt           Re w((d + i gamma)/alpha) / (sqrt(pi) alpha)
//   Lorentz         gamma / (pi (d^2 + gamma^2))                 (gamma = 0: no contribution)
//   Doppler         exp(-(d/alpha)^2) / (sqrt(pi) alpha)
//   binned Gaussian the Doppler profile averaged over the grid bin [d - dnu/2, d + dnu/2] (the
//                   integrated cross section of the bin over its width):
//                   (erf((d + dnu/2)/alpha) - erf((d - dnu/2)/alpha)) / (2 dnu)
// Plinth removal (Sec. 2.1.1) subtracts a line's own profile value at its cutting length from
// every point inside its cut. The cutting length (Sec. 2.4.3 step 4) is a fixed length, or a
// multiple of the line's Doppler half-width sqrt(ln 2) alpha or of its Lorentz half-width gamma.


// Re w(x + iy), y >= 0, for the plinth values (one evaluation per line, in FP64): Weideman's
// approximation with 40 terms for |z| < 8 (about 1e-15 of w(0)), the Laplace continued fraction
// w = (i/sqrt(pi)) / (z - (1/2)/(z - (2/2)/(z - (3/2)/(z - ...)))) with 20 levels beyond (about
// 1e-14 relative there).
__device__ double re_w_accurate(double x, double y) {
  if (x * x + y * y < 64.0) {
    const double L = c_weid40L;
    const double dr = L + y, di = -x;  // L - iz
    const double inv = 1.0 / (dr * dr + di * di);
    const double ur = dr * inv, ui = -di * inv;  // 1/(L - iz)
    const double Zr = 2.0 * L * ur - 1.0, Zi = 2.0 * L * ui;
    double pr = c_weid40[kWeidN40 - 1], pi = 0.0;  // complex Horner in Z
    for (int m = kWeidN40 - 2; m >= 0; --m) {
      const double t = pr * Zr - pi * Zi + c_weid40[m];
      pi = pr * Zi + pi * Zr;
      pr = t;
    }
    const double tr = 2.0 * (pr * ur - pi * ui) + 0.56418958354775628695;
    const double ti = 2.0 * (pr * ui + pi * ur);
    return ur * tr - ui * ti;
  }
  double tr = 0.0, ti = 0.0;  // innermost level first: t = (k/2)/(z - t)
  for (int k = 20; k >= 1; --k) {
    const double dr = x - tr, di = y - ti;
    const double f = (0.5 * k) / (dr * dr + di * di);
    tr = dr * f;
    ti = -di * f;
  }
  const double dr = x - tr, di = y - ti;
  return di * (0.56418958354775628695 / (dr * dr + di * di));  // Re i/(sqrt(pi)(z - t))
}

// A profile's value per unit strength at offset d >= 0, in FP64 (the plinth of a line).
__device__ double profile_value64(int prof, double d, double alpha, double gamma, double dnu) {
  if (prof == kProfLorentz) return gamma > 0.0 ? gamma / (3.14159265358979323846 * (d * d + gamma * gamma)) : 0.0;
  if (prof == kProfDoppler) {
    const double x = d / alpha;
    return exp(-x * x) / (1.7724538509055160273 * alpha);
  }
  if (prof == kProfBinned) {
    const double lo = (d - 0.5 * dnu) / alpha, hi = (d + 0.5 * dnu) / alpha;
    const double diff = lo >= 0.0 ? erfc(lo) - erfc(hi) : (hi <= 0.0 ? erfc(-hi) - erfc(-lo) : erf(hi) - erf(lo));
    return diff / (2.0 * dnu);
  }
  return re_w_accurate(d / alpha, gamma / alpha) / (1.7724538509055160273 * alpha);
}

// Grid record of each line (as k_gridrec) with the line's own cutting length, and its plinth
// S(T) f(cut) (0 without plinth removal or without a cut). The length is decided in FP64 from
// alpha = (nu/c) sqrt(2 k_B T/m) and gamma = gamma_ref (T_ref/T)^n P/P_ref.
__global__ __launch_bounds__(kThreads) void k_gridrec_ex(GridRecArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.pa.N) return;
  double gref, nexp;
  if (a.pa.ovr_g || a.pa.ovr_n) {
    const int32_t c = a.pa.perm[i];
    gref = a.pa.ovr_g ? a.pa.ovr_g[c] : a.pa.gref[i];
    nexp = a.pa.ovr_n ? a.pa.ovr_n[c] : a.pa.nexp[i];
  } else {
    gref = a.pa.gref[i];
    nexp = a.pa.nexp[i];
  }
  const double nuw = a.pa.nu[i];                       // the transition wavenumber (widths)
  const double nu0 = a.nu_pos ? a.nu_pos[i] : nuw;      // the line centre (position)
  const double alpha = nuw / a.c_light * a.alpha_fac;
  const double gam = gref * pow(a.t_ratio, nexp) * a.pa.pfac;
  double cut = a.cut;
  if (!isinf(cut)) {
    if (a.cut_mode == kCutDoppler) cut = a.cut_dop * alpha;
    else if (a.cut_mode == kCutLorentz) cut = a.cut * gam;
  }
  int64_t jlo, jhi;
  cut_range(nu0, a.nu_start, a.dnu, a.n, cut, jlo, jhi);
  double jr = rint((nu0 - a.nu_start) / a.dnu);
  jr = jr < 0.0 ? 0.0 : (jr > (double)(a.n - 1) ? (double)(a.n - 1) : jr);
  const int64_t jref = (int64_t)jr;
  const double delta = __dsub_rn(grid_nu(a.nu_start, a.dnu, jref), nu0);
  if (jlo > jhi) { jlo = 1; jhi = 0; }
  a.grec[i] = make_int4(__float_as_int((float)delta), (int)jref, (int)jlo, (int)jhi);
  if (a.plin) {
    float p = 0.0f;
    if (a.plinth && !isinf(cut) && jlo <= jhi)
      p = (float)((double)a.S_T[i] * profile_value64(a.profile, cut, alpha, gam, a.dnu));
    a.plin[i] = p;
  }
}

// Direct evaluation of every (line, point) pair inside the lines' cuts, for every profile, with
// optional plinth removal and per-line cutting lengths (the grid records of k_gridrec_ex). One
// wave per work item: a span of 64 P grid points and a chunk of the lines whose centre lies
// within the largest cutting length of it. The wave stages 64 lines at a time in LDS (one per
// lane) and evaluates each staged line that reaches the span at all its points, into per-lane
// FP32 sums with a compensated flush every 16 lines. The Voigt profile takes the far-wing series
// of the order the line's points on the span need (the wing pass's zones) at every point outside
// the line's core (|z| >= the last series threshold); its core points are added by k_core, whose
// classification (core_rel) is the same. The plinth is subtracted at every point inside the cut,
// core points included.
// Staged lines are grouped: 1-5 (Voigt: series order; Lorentz: 1) for lines whose cut covers
// the whole span with no core point on it, evaluated without masks; kDirGeneral for the rest.
constexpr int kDirGeneral = kKmax + 1;
struct DirectLDS {
  float4 F0[kWave];  // offset / scale, reference index - span start, dnu / scale, r (see stage_direct)
  float4 F1[kWave];  // amplitude (Voigt: the series' leading coefficient), plinth
  float4 KA[kWave];  // Voigt: series coefficients c1..c4 times the amplitude
  float4 KB[kWave];  // Voigt: c5..c8
  int4 B[kWave];     // span-local inclusive cut range, core range (empty: x > y)
  uint8_t list[kWave];
};

// Stage one line for the span starting at span0; its group, 0: it adds nothing there. The scale is
// sqrt(max(alpha^2, gamma^2)) (Voigt), gamma (Lorentz) or alpha (Doppler, binned Gaussian);
// r is gamma^2 / scale^2 (Voigt) or dnu / (2 alpha) (binned Gaussian). For the Voigt profile the
// series order K is the one the line's points on the span need (as in the wing pass: one more
// term per zone |z| < zK of the thresholds the points reach), and KA, KB hold that order's
// coefficients c1..c(2K-2) (zero beyond); its points with |z| < zc are k_core's.
template <int P, int PROF>
__device__ __forceinline__ int stage_direct(DirectLDS& L, int lane, const int4 gr, double nu0, float S, float gTv,
                                            float pl, const PairDesc& pd, const float* zK, float zc,
                                            int64_t span0) {
  constexpr int W = kWave * P;
  const int jref = gr.y, jlo = gr.z, jhi = gr.w;
  if (!(S > 0.0f) || jlo > jhi || (int64_t)jhi < span0 || (int64_t)jlo > span0 + (W - 1)) return 0;
  const float alpha = (float)(nu0 * pd.beta);
  const float gam = gTv * (float)pd.pfac;
  const float delta = __int_as_float(gr.x);
  const float dnf = (float)pd.dnu;
  const int64_t rl = (int64_t)jlo - span0, rh = (int64_t)jhi - span0;
  int clo = (int)(rl < -1 ? -1 : rl), chi = (int)(rh > W ? W : rh);
  int czl = 1, czh = 0;
  float rs, amp, r = 0.0f, order = 1.0f;
  if (PROF == kProfVoigt) {
    const float a2 = alpha * alpha, g2 = gam * gam;
    const float sc = a2 > g2 ? a2 : g2;
    if (!(sc > 0.0f)) return 0;
    rs = __frsqrt_rn(sc);
    const float isc = rs * rs;
    amp = S * (gam * isc) * 0.318309886183790672f;  // S gamma / (pi s)
    const float av = a2 * isc, gv = g2 * isc;
    r = gv;
    // the order the line's points on the span need: zones |z| < zK[z] around the centre c
    const float inv_dnu = (float)(1.0 / pd.dnu);
    const float af = alpha * inv_dnu, gf = gam * inv_dnu;
    const float c = (float)((int64_t)jref - span0) - delta * inv_dnu;
    const float x0 = (float)(clo > 0 ? clo : 0), x1 = (float)(chi < W - 1 ? chi : W - 1);
    int K = 1;
#pragma unroll
    for (int z = 0; z < kKmax - 1; ++z) {
      const float zz = zK[z] * af;
      const float h2 = zz * zz - gf * gf;
      const float h = h2 > 0.0f ? __builtin_amdgcn_sqrtf(h2) * 1.00001f + 1e-3f : -1.0f;
      K += (h > 0.0f && x0 < c + h && x1 > c - h) ? 1 : 0;
    }
    order = (float)K;
    const float a3 = av * av * av, a4 = a3 * av, gv2 = gv * gv, gv3 = gv2 * gv;
    float4 ka = make_float4(0.f, 0.f, 0.f, 0.f), kb = ka;
    if (K == 2) {
      ka = make_float4(amp * (1.5f * av), amp * (-2.0f * av * gv), 0.f, 0.f);
    } else if (K == 3) {
      ka = make_float4(amp * (1.5f * av), amp * (-2.0f * av * gv + 3.75f * av * av), amp * (-15.0f * av * av * gv),
                       amp * (12.0f * av * av * gv2));
    } else if (K == 4) {
      ka = make_float4(amp * (1.5f * av), amp * (-2.0f * av * gv + 3.75f * av * av),
                       amp * (-15.0f * av * av * gv + 13.125f * a3), amp * (12.0f * av * av * gv2 - 105.0f * a3 * gv));
      kb = make_float4(amp * (210.0f * a3 * gv2), amp * (-120.0f * a3 * gv3), 0.f, 0.f);
    } else if (K == 5) {
      ka = make_float4(amp * (1.5f * av), amp * (-2.0f * av * gv + 3.75f * av * av),
                       amp * (-15.0f * av * av * gv + 13.125f * a3),
                       amp * (12.0f * av * av * gv2 - 105.0f * a3 * gv + 59.0625f * a4));
      kb = make_float4(amp * (210.0f * a3 * gv2 - 787.5f * a4 * gv), amp * (-120.0f * a3 * gv3 + 2835.0f * a4 * gv2),
                       amp * (-3780.0f * a4 * gv3), amp * (1680.0f * a4 * gv2 * gv2));
    }
    L.KA[lane] = ka;
    L.KB[lane] = kb;
    int rlo, rhi;
    if (core_rel(alpha, gam, delta, (float)(1.0 / pd.dnu), zc, rlo, rhi)) {
      const int64_t gl = (int64_t)jref + rlo - span0, gh = (int64_t)jref + rhi - span0;
      czl = (int)(gl < -1 ? -1 : (gl > W ? W : gl));
      czh = (int)(gh < -1 ? -1 : (gh > W ? W : gh));
    }
  } else if (PROF == kProfLorentz) {
    if (!(gam > 0.0f)) return 0;
    rs = 1.0f / gam;
    amp = S * rs * 0.318309886183790672f;  // S / (pi gamma)
  } else {
    if (!(alpha > 0.0f)) return 0;
    rs = 1.0f / alpha;
    // a Gaussian (or its bin average) is below e^-81 of its peak beyond 9 alpha (+ a bin):
    // only those points are evaluated (the window of the work list is cut the same way)
    const float inv = 1.0f / dnf;
    const float cen = (float)((int64_t)jref - span0) - delta * inv;
    const float R = (9.0f * alpha + dnf) * inv + 1.0f;
    const float fl = fmaxf(fminf(floorf(cen - R), (float)(W + 1)), -2.0f);
    const float fh = fmaxf(fminf(ceilf(cen + R), (float)(W + 1)), -2.0f);
    const int gl = (int)fl, gh = (int)fh;
    if (gl > clo) clo = gl;
    if (gh < chi) chi = gh;
    if (clo > chi || chi < 0 || clo > W - 1) return 0;
    if (PROF == kProfDoppler) {
      amp = S * rs * 0.564189583547756287f;  // S / (sqrt(pi) alpha)
    } else {
      amp = S / (2.0f * dnf);
      r = 0.5f * dnf * rs;
    }
  }
  L.F0[lane] = make_float4(delta * rs, (float)((int64_t)jref - span0), dnf * rs, r);
  L.F1[lane] = make_float4(amp, pl, order, 0.0f);
  L.B[lane] = make_int4(clo, chi, czl, czh);
  // a Voigt or Lorentz line whose cut covers the whole span and that has no core point on it
  // takes the unmasked loop of its order (its plinth is added once per span, not per point)
  const bool full = clo <= 0 && chi >= W - 1;
  const bool core = czl <= czh && czh >= 0 && czl <= W - 1;
  if (PROF == kProfVoigt && full && !core) return (int)order;
  if (PROF == kProfLorentz && full) return 1;
  return kDirGeneral;
}

// erf(b) - erf(a) for a <= b in FP32, from erfc where both have one sign (no cancellation of
// values near 1).
__device__ __forceinline__ float erf_diff(float a, float b) {
  if (a >= 0.0f) return erfcf(a) - erfcf(b);
  if (b <= 0.0f) return erfcf(-b) - erfcf(-a);
  return erff(b) - erff(a);
}

// The Voigt far-wing series of order K in q (coefficients c1..c(2K-2) in ka, kb; c0 = amp).
template <int K>
__device__ __forceinline__ float voigt_series(float q, const float4& ka, const float4& kb, float amp) {
  float t;
  if (K == 1) {
    t = amp;
  } else if (K == 2) {
    t = __builtin_fmaf(ka.y, q, ka.x);
    t = __builtin_fmaf(t, q, amp);
  } else if (K == 3) {
    t = __builtin_fmaf(ka.w, q, ka.z);
    t = __builtin_fmaf(t, q, ka.y);
    t = __builtin_fmaf(t, q, ka.x);
    t = __builtin_fmaf(t, q, amp);
  } else if (K == 4) {
    t = __builtin_fmaf(kb.y, q, kb.x);
    t = __builtin_fmaf(t, q, ka.w);
    t = __builtin_fmaf(t, q, ka.z);
    t = __builtin_fmaf(t, q, ka.y);
    t = __builtin_fmaf(t, q, ka.x);
    t = __builtin_fmaf(t, q, amp);
  } else {
    t = __builtin_fmaf(kb.w, q, kb.z);
    t = __builtin_fmaf(t, q, kb.y);
    t = __builtin_fmaf(t, q, kb.x);
    t = __builtin_fmaf(t, q, ka.w);
    t = __builtin_fmaf(t, q, ka.z);
    t = __builtin_fmaf(t, q, ka.y);
    t = __builtin_fmaf(t, q, ka.x);
    t = __builtin_fmaf(t, q, amp);
  }
  return t * q;
}

// One staged Voigt line of series order K at all P points of this lane.
template <int P, int K>
__device__ __forceinline__ void direct_voigt(const DirectLDS& L, int l, int lane, float (&part)[P]) {
  const float4 f0 = L.F0[l];
  const float4 f1 = L.F1[l];
  const int4 bb = L.B[l];
  float4 ka = make_float4(0.f, 0.f, 0.f, 0.f), kb = ka;
  if (K >= 2) ka = L.KA[l];
  if (K >= 4) kb = L.KB[l];
  const float kf0 = (float)lane - f0.y;
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int j = lane + kWave * p;
    const float D = __builtin_fmaf(kf0 + (float)(kWave * p), f0.z, f0.x);
    const float q = __builtin_amdgcn_rcpf(__builtin_fmaf(D, D, f0.w));
    const float v = voigt_series<K>(q, ka, kb, f1.x);
    // core points (k_core's) take only the plinth; excluded points may have q infinite
    const float t = (j >= bb.z && j <= bb.w) ? 0.0f : v;
    const bool in = j >= bb.x && j <= bb.y;
    part[p] += in ? t - f1.y : 0.0f;
  }
}

// One staged line of a full-span group at all P points of this lane: Voigt of series order K
// (PROF = kProfVoigt), or Lorentz (K = 1). No point is masked: the plinth is not taken here.
template <int P, int PROF, int K>
__device__ __forceinline__ void direct_full(const DirectLDS& L, int l, int lane, float (&part)[P]) {
  const float4 f0 = L.F0[l];
  const float amp = L.F1[l].x;
  float4 ka = make_float4(0.f, 0.f, 0.f, 0.f), kb = ka;
  if (K >= 2) ka = L.KA[l];
  if (K >= 4) kb = L.KB[l];
  const float kf0 = (float)lane - f0.y;
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const float D = __builtin_fmaf(kf0 + (float)(kWave * p), f0.z, f0.x);
    if (PROF == kProfVoigt) {
      const float q = __builtin_amdgcn_rcpf(__builtin_fmaf(D, D, f0.w));
      float t;
      if (K == 1) {
        t = amp;
      } else if (K == 2) {
        t = __builtin_fmaf(ka.y, q, ka.x);
        t = __builtin_fmaf(t, q, amp);
      } else if (K == 3) {
        t = __builtin_fmaf(ka.w, q, ka.z);
        t = __builtin_fmaf(t, q, ka.y);
        t = __builtin_fmaf(t, q, ka.x);
        t = __builtin_fmaf(t, q, amp);
      } else if (K == 4) {
        t = __builtin_fmaf(kb.y, q, kb.x);
        t = __builtin_fmaf(t, q, ka.w);
        t = __builtin_fmaf(t, q, ka.z);
        t = __builtin_fmaf(t, q, ka.y);
        t = __builtin_fmaf(t, q, ka.x);
        t = __builtin_fmaf(t, q, amp);
      } else {
        t = __builtin_fmaf(kb.w, q, kb.z);
        t = __builtin_fmaf(t, q, kb.y);
        t = __builtin_fmaf(t, q, kb.x);
        t = __builtin_fmaf(t, q, ka.w);
        t = __builtin_fmaf(t, q, ka.z);
        t = __builtin_fmaf(t, q, ka.y);
        t = __builtin_fmaf(t, q, ka.x);
        t = __builtin_fmaf(t, q, amp);
      }
      part[p] = __builtin_fmaf(t, q, part[p]);
    } else {
      part[p] = __builtin_fmaf(amp, __builtin_amdgcn_rcpf(__builtin_fmaf(D, D, 1.0f)), part[p]);
    }
  }
}

// One staged line (uniform index l) at all P points of this lane.
template <int P, int PROF>
__device__ __forceinline__ void direct_eval(const DirectLDS& L, int l, int lane, float (&part)[P]) {
  if (PROF == kProfVoigt) {
    const int K = __builtin_amdgcn_readfirstlane(__float_as_int(L.F1[l].z));  // the line's order (uniform)
    if (K == __float_as_int(1.0f)) direct_voigt<P, 1>(L, l, lane, part);
    else if (K == __float_as_int(2.0f)) direct_voigt<P, 2>(L, l, lane, part);
    else if (K == __float_as_int(3.0f)) direct_voigt<P, 3>(L, l, lane, part);
    else if (K == __float_as_int(4.0f)) direct_voigt<P, 4>(L, l, lane, part);
    else direct_voigt<P, 5>(L, l, lane, part);
    return;
  }
  const float4 f0 = L.F0[l];
  const float4 f1 = L.F1[l];
  const int4 bb = L.B[l];
  const float kf0 = (float)lane - f0.y;
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int j = lane + kWave * p;
    const float D = __builtin_fmaf(kf0 + (float)(kWave * p), f0.z, f0.x);
    float v;
    if (PROF == kProfLorentz) {
      v = f1.x * __builtin_amdgcn_rcpf(__builtin_fmaf(D, D, 1.0f));
    } else if (PROF == kProfDoppler) {
      v = f1.x * __builtin_amdgcn_exp2f(-(D * D) * 1.44269504088896341f);
    } else {
      v = f1.x * erf_diff(D - f0.w, D + f0.w);
    }
    const bool in = j >= bb.x && j <= bb.y;
    part[p] += in ? v - f1.y : 0.0f;
  }
}

// The staged lines of one group (list entries [i0, i1)), a compensated flush after every 16
// lines counted over the groups of the batch (since).
template <int P, int PROF, int G>
__device__ __forceinline__ void direct_one(const DirectLDS& L, int l, int lane, float (&part)[P], float (&s)[P],
                                           float (&cc)[P], int& since) {
  if (G == kDirGeneral) direct_eval<P, PROF>(L, l, lane, part);
  else direct_full<P, PROF, G>(L, l, lane, part);
  if (++since == 16) {
    kahan_flush<P>(part, s, cc);
    since = 0;
  }
}

template <int P, int PROF, int G>
__device__ __forceinline__ void direct_group_loop(const DirectLDS& L, int i0, int i1, int lane, float (&part)[P],
                                                  float (&s)[P], float (&cc)[P], int& since) {
  int i = i0;
  for (; i < i1 && (i & 3); ++i)  // unaligned head
    direct_one<P, PROF, G>(L, __builtin_amdgcn_readfirstlane((int)L.list[i]), lane, part, s, cc, since);
  for (; i + 4 <= i1; i += 4) {  // four list entries per scalar read
    const uint32_t w4 = (uint32_t)__builtin_amdgcn_readfirstlane((int)*reinterpret_cast<const uint32_t*>(&L.list[i]));
    direct_one<P, PROF, G>(L, (int)(w4 & 255u), lane, part, s, cc, since);
    direct_one<P, PROF, G>(L, (int)((w4 >> 8) & 255u), lane, part, s, cc, since);
    direct_one<P, PROF, G>(L, (int)((w4 >> 16) & 255u), lane, part, s, cc, since);
    direct_one<P, PROF, G>(L, (int)(w4 >> 24), lane, part, s, cc, since);
  }
  for (; i < i1; ++i)
    direct_one<P, PROF, G>(L, __builtin_amdgcn_readfirstlane((int)L.list[i]), lane, part, s, cc, since);
}

template <int P, int PROF>
__global__ __launch_bounds__(kWave) void k_direct(VoigtArgs a, const float* __restrict__ plin_all) {
  constexpr int W = kWave * P;
  __shared__ DirectLDS L;
  const int lane = threadIdx.x;
  const int total = a.item_base[a.n_tiles_total];
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  long long n_lines = 0;
  for (;;) {
    int mine = 0;
    if (lane == 0) mine = atomicAdd(a.counter, 1);
    const int it = __builtin_amdgcn_readfirstlane(mine);
    if (it >= total) break;
    int lo = 0, hi = a.n_tiles_total - 1;  // last span with item_base <= it
    while (lo < hi) {
      const int m = (lo + hi + 1) >> 1;
      if (a.item_base[m] <= it) lo = m; else hi = m - 1;
    }
    const int g = lo;
    const PairDesc pd = wave_uniform(a.pairs[find_pair(a.pairs, a.n_pairs, g)]);
    const int ibase = __builtin_amdgcn_readfirstlane(a.item_base[g]);
    const int nc = __builtin_amdgcn_readfirstlane(a.tile_nc[g]);
    const int64_t span0 = (int64_t)(g - pd.tile_base) * W;
    const int64_t line_lo = (int64_t)__builtin_amdgcn_readfirstlane(a.tile_lo[g]) + (int64_t)(it - ibase) * a.chunk;
    int64_t line_hi = line_lo + a.chunk;
    const int64_t thi = __builtin_amdgcn_readfirstlane(a.tile_hi[g]);
    if (line_hi > thi) line_hi = thi;
    const float* __restrict__ S_T = a.S_T + (int64_t)pd.tidx * a.N;
    const float* __restrict__ gT = a.gT + (int64_t)pd.tidx * a.N;
    const int4* __restrict__ grec = a.grec + (int64_t)pd.gidx * a.N;
    const float* __restrict__ plin = plin_all ? plin_all + (int64_t)pd.gidx * a.N : nullptr;

    float s[P], cc[P], part[P];
#pragma unroll
    for (int p = 0; p < P; ++p) { s[p] = 0.0f; cc[p] = 0.0f; part[p] = 0.0f; }
    double pl_full = 0.0;  // this lane's share of the plinths of the full-span lines
    for (int64_t b = line_lo; b < line_hi; b += kWave) {
      const int64_t li = b + lane;
      int code = 0;
      float pl = 0.0f;
      if (li < line_hi) {
        pl = plin ? plin[li] : 0.0f;
        code = stage_direct<P, PROF>(L, lane, grec[li], a.nu[li], S_T[li], gT[li], pl, pd, a.zK, a.zcore, span0);
      }
      if (code > 0 && code < kDirGeneral) pl_full += (double)pl;
      // the list, grouped: full-span groups 1..kKmax in order, then the general one
      int start[kDirGeneral + 2];
      int base = 0, pos = -1;
#pragma unroll
      for (int g = 1; g <= kDirGeneral; ++g) {
        const uint64_t m = __ballot(code == g);
        start[g] = base;
        if (code == g) pos = base + (int)__popcll(m & lt);
        base += (int)__popcll(m);
      }
      start[kDirGeneral + 1] = base;
      if (pos >= 0) L.list[pos] = (uint8_t)lane;
      const int cnt = base;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      int since = 0;
      if (PROF == kProfVoigt) {
        direct_group_loop<P, PROF, 1>(L, start[1], start[2], lane, part, s, cc, since);
        direct_group_loop<P, PROF, 2>(L, start[2], start[3], lane, part, s, cc, since);
        direct_group_loop<P, PROF, 3>(L, start[3], start[4], lane, part, s, cc, since);
        direct_group_loop<P, PROF, 4>(L, start[4], start[5], lane, part, s, cc, since);
        direct_group_loop<P, PROF, 5>(L, start[5], start[6], lane, part, s, cc, since);
      } else if (PROF == kProfLorentz) {
        direct_group_loop<P, PROF, 1>(L, start[1], start[2], lane, part, s, cc, since);
      }
      direct_group_loop<P, PROF, kDirGeneral>(L, start[kDirGeneral], start[kDirGeneral + 1], lane, part, s, cc,
                                               since);
      kahan_flush<P>(part, s, cc);
      n_lines += cnt;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (plin) {
      // the full-span lines' plinths: one subtraction at every point of the span
      const float tot = (float)wave_sum64(pl_full);
#pragma unroll
      for (int p = 0; p < P; ++p) part[p] = -tot;
      kahan_flush<P>(part, s, cc);
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int local = p * kWave + lane;
      const float v = s[p] - cc[p];
      if (nc == 1) {
        if (span0 + local < pd.n) a.k[pd.out_off + span0 + local] = v;
      } else if (it < a.items_cap) {
        a.partial[((int64_t)it) * W + local] = v;
      }
    }
    if (nc != 1 && it >= a.items_cap && a.status && lane == 0) atomicOr(a.status, 1);
  }
  if (a.stats && lane == 0) a.stats[blockIdx.x] = n_lines * W;
}

// Order-preserving map of doubles to unsigned 64-bit integers (integer max/min = FP64 max/min).
__device__ __forceinline__ unsigned long long double_to_ordered(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__global__ void k_line_stats_init(unsigned long long* out) {
  out[0] = 0ull;     // max gamma_ref
  out[1] = ~0ull;    // min n
  out[2] = 0ull;     // max n
}

// The list's largest gamma_ref and smallest and largest n (integer atomics on ordered words:
// the result does not depend on the order).
__global__ __launch_bounds__(kThreads) void k_line_stats(const double* __restrict__ gref,
                                                        const double* __restrict__ nexp, int64_t N,
                                                        unsigned long long* out) {
  unsigned long long gmax = 0ull, nmin = ~0ull, nmax = 0ull;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long g = double_to_ordered(gref[i]), n = double_to_ordered(nexp[i]);
    gmax = g > gmax ? g : gmax;
    nmin = n < nmin ? n : nmin;
    nmax = n > nmax ? n : nmax;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long a = __shfl_xor(gmax, off, 64), b = __shfl_xor(nmin, off, 64),
                             c = __shfl_xor(nmax, off, 64);
    gmax = a > gmax ? a : gmax;
    nmin = b < nmin ? b : nmin;
    nmax = c > nmax ? c : nmax;
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(out, gmax);
    atomicMin(out + 1, nmin);
    atomicMax(out + 2, nmax);
  }
}

// Per-line cut bounds and plinth values of sorted-order grid records, in the caller's order.
__global__ __launch_bounds__(kThreads) void k_scatter_grec(const int4* __restrict__ grec,
                                                          const float* __restrict__ plin,
                                                          const int32_t* __restrict__ perm, int64_t N,
                                                          int32_t* __restrict__ jlo, int32_t* __restrict__ jhi,
                                                          float* __restrict__ plin_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int4 g = grec[i];
  const int32_t c = perm[i];
  if (jlo) jlo[c] = g.z;
  if (jhi) jhi[c] = g.w;
  if (plin_out) plin_out[c] = plin ? plin[i] : 0.0f;
}

// ------------------------------------------------------- HITRAN widths and line shift
// A HITRAN-style list adds per line the self-broadening coefficient gamma_self and the pressure
// shift delta_air (Table binary2). At pressure P with self partial pressure P_self the Lorentz
// half-width is eq. (gammaL) without the natural term, (T_ref/T)^n (gamma_air (P - P_self) +
// gamma_self P_self)/P_ref, and the centre moves to nu* = nu + delta_air P/P_ref, which can change
// the order along nu (Sec. 2.4.3 step 3): such a call bins the list again by nu*.

// gamma_self >= 0 and finite, delta finite (flags[0] = 1 if not); out[0] = ordered max |delta|,
// out[1] = ordered max gamma_self.
__global__ __launch_bounds__(kThreads) void k_hitran_check(const double* __restrict__ gself,
                                                          const double* __restrict__ delta, int64_t N, int* flags,
                                                          unsigned long long* out) {
  unsigned long long dmax = double_to_ordered(0.0), gmax = double_to_ordered(0.0);
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    const double g = gself[i], d = delta[i];
    bad |= !(g >= 0.0) || isinf(g) || !isfinite(d);
    const unsigned long long dw = double_to_ordered(fabs(d)), gw = double_to_ordered(g);
    if (isfinite(d)) dmax = dw > dmax ? dw : dmax;
    if (g >= 0.0 && !isinf(g)) gmax = gw > gmax ? gw : gmax;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long a = __shfl_xor(dmax, off, 64), b = __shfl_xor(gmax, off, 64);
    dmax = a > dmax ? a : dmax;
    gmax = b > gmax ? b : gmax;
  }
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flags, 1);
  if ((threadIdx.x & 63) == 0) {
    atomicMax(out, dmax);
    atomicMax(out + 1, gmax);
  }
}

__global__ void k_hitran_check_init(int* flags, unsigned long long* out) {
  flags[0] = 0;
  out[0] = double_to_ordered(0.0);
  out[1] = double_to_ordered(0.0);
}

// The two extra fields in the handle's (sorted) order: out[s] = in[perm[s]].
__global__ __launch_bounds__(kThreads) void k_gather2(const int32_t* __restrict__ perm, int64_t N,
                                                     const double* __restrict__ a, const double* __restrict__ b,
                                                     double* __restrict__ oa, double* __restrict__ ob) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= N) return;
  const int32_t c = perm[s];
  oa[s] = a[c];
  ob[s] = b[c];
}

// Keys of the shifted centres (handle order), with identity values for the radix sort.
__global__ __launch_bounds__(kThreads) void k_shift_keys(const double* __restrict__ nu,
                                                        const double* __restrict__ delta, int64_t N, double pshift,
                                                        KeyMap km, uint32_t* __restrict__ keys,
                                                        int32_t* __restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  keys[i] = bin_key(nu[i] + delta[i] * pshift, km);
  vals[i] = (int32_t)i;
}

// The view of the list at one pressure, sorted by shifted centre: for view position s, handle
// line i = src[s]: the transition wavenumber (strength and widths), the centre, S_ref, E'', the
// reference width that gives the HITRAN half-width through gamma_ref (T_ref/T)^n P/P_ref, n, and
// the caller index.
__global__ __launch_bounds__(kThreads) void k_shift_gather(ShiftArgs a) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= a.N) return;
  const int32_t i = a.src[s];
  const double v = a.nu[i];
  a.o_nu[s] = v;
  a.o_pos[s] = v + a.delta[i] * a.pshift;
  a.o_S[s] = a.Sref[i];
  a.o_E[s] = a.E[i];
  a.o_g[s] = a.P > 0.0 ? (a.gair[i] * (a.P - a.Pself) + a.gself[i] * a.Pself) / a.P : 0.0;
  a.o_n[s] = a.nexp[i];
  a.o_perm[s] = a.perm[i];
}

// ------------------------------------------------------------ streamed line lists
// k[i] = 0 (a kernel, so that it may be recorded into a graph) and k[i] += t[i] (a chunk's
// contribution, added in chunk order).
__global__ __launch_bounds__(kThreads) void k_fill0(float* __restrict__ k, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) k[i] = 0.0f;
}
__global__ __launch_bounds__(kThreads) void k_accumulate(float* __restrict__ k, const float* __restrict__ t,
                                                        int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) k[i] += t[i];
}

// Scratch of the allocation-free entry point: a fixed device array that stands in for the
// caller's workspace. Host code never names it as an address: it takes the array's device
// address once per device (scratch_address) and passes that.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_address(void** p) {
  *p = nullptr;
  return hipGetSymbolAddress(p, HIP_SYMBOL(scratch));
}

// ------------------------------------------------------------------------ adjoint
// w(x + iy) = K + iL in FP32 by the same rational approximation as the line-core pass (both
// parts): w = u t, t = 2 p u + 1/sqrt(pi).
__device__ __forceinline__ void weideman_w32(float x, float y, float& K, float& L) {
  const float Lw = c_weidL32;
  const float dr = Lw + y;
  const float d = __builtin_fmaf(dr, dr, x * x);
  float inv = __builtin_amdgcn_rcpf(d);
  inv = __builtin_fmaf(inv, __builtin_fmaf(-d, inv, 1.0f), inv);
  const float ur = dr * inv, ui = x * inv;
  const float Zr = __builtin_fmaf(-2.0f * x, ui, __builtin_fmaf(-2.0f * y, ur, 1.0f));
  const float Zi = 2.0f * __builtin_fmaf(x, ur, -y * ui);
  const float r = 2.0f * Zr, s = __builtin_fmaf(Zr, Zr, Zi * Zi);
  float b2 = c_weid32[kWeidN - 1];
  float b1 = __builtin_fmaf(r, b2, c_weid32[kWeidN - 2]);
#pragma unroll
  for (int m = kWeidN - 3; m >= 1; --m) {
    const float t = __builtin_fmaf(r, b1, __builtin_fmaf(-s, b2, c_weid32[m]));
    b2 = b1;
    b1 = t;
  }
  const float pr = __builtin_fmaf(Zr, b1, __builtin_fmaf(-s, b2, c_weid32[0]));
  const float pi = Zi * b1;
  const float tr = 2.0f * __builtin_fmaf(pr, ur, -pi * ui) + 0.564189583547756287f;
  const float ti = 2.0f * __builtin_fmaf(pr, ui, pi * ur);
  K = __builtin_fmaf(ur, tr, -ui * ti);
  L = __builtin_fmaf(ur, ti, ui * tr);
}

// Far-wing profile and its gamma and alpha derivatives as real polynomials in q = s/(D^2 +
// gamma^2) (s = max(alpha^2, gamma^2)), from the asymptotic series of w truncated after KD terms:
// with a = alpha^2/s, g = gamma^2/s, u = g q, c = sqrt(1 - u), a_k = (2k-1)!!/2^k,
//   V         = gamma/(pi s)       sum_k a_k a^k q^(k+1) U_2k(c)
//   dV/dalpha = gamma/(pi s alpha) sum_k 2k a_k a^k q^(k+1) U_2k(c)
//   dV/dgamma = 1/(pi s)           sum_k (2k+1) a_k a^k q^(k+1) T_(2k+2)(c)
// (V per unit strength; term by term derivatives of -Im (D + i gamma)^-(2k+1) alpha^2k/pi).
// U and T are Chebyshev polynomials written in powers of u (c^2 = 1 - u).
constexpr int kAdjDeg = 2 * (kKmax + 1) + 1;  // highest power of q + 1
struct AdjPoly {
  float v[kAdjDeg], da[kAdjDeg], dg[kAdjDeg];  // coefficient of q^M at [M]
};

// Chebyshev polynomials in powers of u (c^2 = 1 - u): U_2k (k = 0..5) and T_(2k+2).
__constant__ float c_adjU[6][8] = {{1, 0, 0, 0, 0, 0, 0, 0},          {3, -4, 0, 0, 0, 0, 0, 0},
                                   {5, -20, 16, 0, 0, 0, 0, 0},       {7, -56, 112, -64, 0, 0, 0, 0},
                                   {9, -120, 432, -576, 256, 0, 0, 0}, {11, -220, 1232, -2816, 2816, -1024, 0, 0}};
__constant__ float c_adjT[6][8] = {{1, -2, 0, 0, 0, 0, 0, 0},           {1, -8, 8, 0, 0, 0, 0, 0},
                                   {1, -18, 48, -32, 0, 0, 0, 0},       {1, -32, 160, -256, 128, 0, 0, 0},
                                   {1, -50, 400, -1120, 1280, -512, 0, 0}, {1, -72, 840, -3584, 6912, -6144, 2048, 0}};

// Coefficients of q^M (one M per lane) of the three polynomials, series truncated after KD terms
// (1..kKmax + 1; three sets are formed in one pass, one per 16-lane group). U and T are the
// workgroup's LDS copies of c_adjU and c_adjT (the lanes index them by their own M).
__device__ __forceinline__ void adj_coef_rt(int KD, int M, float a, float g, const float (*U)[8],
                                            const float (*T)[8], float& v, float& da, float& dg) {
  constexpr float ak[6] = {1.0f, 0.5f, 0.75f, 1.875f, 6.5625f, 29.53125f};
  v = da = dg = 0.0f;
  // powers of g up to kKmax + 1, picked by selects (no per-lane loop)
  float gpw[kKmax + 2];
  gpw[0] = 1.0f;
#pragma unroll
  for (int t = 1; t < kKmax + 2; ++t) gpw[t] = gpw[t - 1] * g;
  float ap = 1.0f;
#pragma unroll
  for (int k = 0; k < kKmax + 1; ++k) {
    const int j = M - k - 1;  // power of u
    if (k < KD && j >= 0 && j <= k + 1) {
      float gp = gpw[0];
#pragma unroll
      for (int t = 1; t <= k + 1; ++t) gp = j == t ? gpw[t] : gp;
      const float w = ak[k] * ap * gp;
      if (j <= k) {
        v += w * U[k][j];
        da += 2.0f * k * w * U[k][j];
      }
      dg += (2.0f * k + 1.0f) * w * T[k][j];
    }
    ap *= a;
  }
}

// sum_M c[M] q^M for M = 1 .. DEG (Horner)
template <int DEG>
__device__ __forceinline__ float adj_horner(const float* c, float q) {
  float t = c[DEG];
#pragma unroll
  for (int M = DEG - 1; M >= 1; --M) t = __builtin_fmaf(t, q, c[M]);
  return t * q;
}

// sum_M c[M] q^(M-1) for M = 1 .. DEG
template <int DEG>
__device__ __forceinline__ float adj_horner1(const float* c, float q) {
  float t = c[DEG];
#pragma unroll
  for (int M = DEG - 1; M >= 1; --M) t = __builtin_fmaf(t, q, c[M]);
  return t;
}

// One step of NP x 64 far-wing points: accumulate g V, g dV/dalpha, g dV/dgamma (per unit
// strength, up to the line's constant factors) with polynomials of the given degrees.
template <int NP, int DV, int DA, int DG>
__device__ __forceinline__ void adj_step(const AdjPoly& P, int jc, int lane, int jref, int jhi, float dnh, float dh,
                                         float gh, const float (&gcur)[NP], float& bV, float& bA, float& bG) {
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const int j = jc + p * kWave + lane;
    const float D = __builtin_fmaf((float)(j - jref), dnh, dh);
    const float q = __builtin_amdgcn_rcpf(__builtin_fmaf(D, D, gh * gh));  // q = s/(D^2 + gamma^2) <= 1
    const float gq = (j <= jhi ? gcur[p] : 0.0f) * q;  // points beyond jhi hold a clamped load
    bV = __builtin_fmaf(gq, adj_horner1<DV>(P.v, q), bV);
    bA = __builtin_fmaf(gq, adj_horner1<DA>(P.da, q), bA);
    bG = __builtin_fmaf(gq, adj_horner1<DG>(P.dg, q), bG);
  }
}


// Node weights of dL/dk for the adjoint's far units, one level (units of W points): for unit u
// (points u W + jj) and node k, the prefix sums over jj of g_j L_k(jj) (L_k: the Lagrange weight
// of node k of the unit at its point jj), in FP64 in a fixed order (each thread sums its
// W / kAdjSpan consecutive points, then a scan over the threads' totals). A line that covers
// points a..b of a unit far from its centre then takes sum_j g_j f(j) = sum_k f(x_k) (P_k(b) -
// P_k(a - 1)) up to the interpolation error of f on the unit.
template <int W>
__global__ __launch_bounds__(kAdjSpan) void k_adj_nodes(const float* __restrict__ g, int64_t n,
                                                        const double* __restrict__ w, double* __restrict__ gpref) {
  constexpr int R = W / kAdjSpan;  // points per thread
  __shared__ double sc[kAdjSpan];
  const int u = blockIdx.x, t = threadIdx.x;
  const int64_t j0 = (int64_t)u * W + (int64_t)t * R;
  double gv[R];
#pragma unroll
  for (int r = 0; r < R; ++r) gv[r] = j0 + r < n ? (double)g[j0 + r] : 0.0;
  for (int k = 0; k < kNodes; ++k) {
    double loc[R];
    double run = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      run += gv[r] * w[k * W + t * R + r];
      loc[r] = run;
    }
    double v = run;
    sc[t] = v;
    __syncthreads();
    for (int off = 1; off < kAdjSpan; off <<= 1) {
      const double x = t >= off ? sc[t - off] : 0.0;
      __syncthreads();
      v += x;
      sc[t] = v;
      __syncthreads();
    }
    const double excl = v - run;
    double* out = gpref + ((int64_t)u * kNodes + k) * W + (int64_t)t * R;
#pragma unroll
    for (int r = 0; r < R; ++r) out[r] = R == 1 ? v : loc[r] + excl;
    __syncthreads();
  }
}

// Far units of the adjoint: a unit (a span of kAdjSpan points, or 4 or 16 of them) at least this
// many unit widths from the line centre (unit centre to line centre) and clear of its core zone
// takes the node weights of dL/dk over its points.
constexpr double kAdjFarSpans = 1.5;

// Per-line bounds of the adjoint's walk over a line's points (grid indices): the series zones
// zlo[K] .. zhi[K] (|z| < zK[K]; the last is the core zone; half-widths from an FP32 square root:
// they carry a relative slack of 1e-5 and only choose how many series terms a step takes) and,
// per far-unit level L (units of kAdjSpan 4^L points), the last far unit on the left uL[L] and the
// first on the right uR[L]. out = zlo[kKmax], zhi[kKmax], uL[kAdjLevels], uR[kAdjLevels].
static_assert(2 * kKmax + 2 * kAdjLevels == 16, "16 bounds per line");
__device__ __forceinline__ void adj_line_bounds(const AdjArgs& a, double alpha, double g2d, const int4 gr,
                                                int4* __restrict__ out) {
  const double inv_dnu = 1.0 / a.dnu;
  const double cpos = (double)gr.y - (double)__int_as_float(gr.x) * inv_dnu;
  int b[16];
#pragma unroll
  for (int K = 0; K < kKmax; ++K) {
    const double zz = (double)a.zK[K] * alpha;
    const double h2 = zz * zz - g2d;
    int lo_i = 2000000000, hi_i = -2000000000;  // empty zone: no chunk intersects it
    if (h2 > 0.0) {
      const double h = (double)__builtin_amdgcn_sqrtf((float)h2) * inv_dnu * 1.00001 + 1e-3;
      const double lo = ceil(cpos - h), hi = floor(cpos + h);
      lo_i = lo < -1.0 ? -1 : (lo > 2.0e9 ? 2000000000 : (int)lo);
      hi_i = hi < -1.0 ? -1 : (hi > 2.0e9 ? 2000000000 : (int)hi);
    }
    b[K] = lo_i;
    b[kKmax + K] = hi_i;
  }
#pragma unroll
  for (int L = 0; L < kAdjLevels; ++L) {
    const double Wd = (double)(kAdjSpan << (2 * L)), iW = 1.0 / Wd;  // a power of two: exact
    const double reach = kAdjFarSpans * Wd, half = 0.5 * (Wd - 1.0);
    const double l = fmin(floor((cpos - reach - half) * iW), floor(((double)b[kKmax - 1] - Wd) * iW));
    const double r = fmax(ceil((cpos + reach - half) * iW), floor((double)b[2 * kKmax - 1] * iW) + 1.0);
    b[2 * kKmax + L] = l < -2.0 ? -2 : (l > 1.0e8 ? 100000000 : (int)l);
    b[2 * kKmax + kAdjLevels + L] = r > 1.0e8 ? 100000000 : (r < -2.0 ? -2 : (int)r);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) out[q] = make_int4(b[4 * q], b[4 * q + 1], b[4 * q + 2], b[4 * q + 3]);
}

// One wave per line (static assignment), lanes over its grid points inside the cut.
// Per-line FP64 quantities of the adjoint, one thread per line (sorted order), kept apart from
// the point loop so that the transcendental functions do not hold registers there:
// rec[8 i ..] = (S, gamma, S/S_ref, gamma/gamma_ref, S dlnS/dT, n gamma / T, 1/sqrt(s), 1/alpha)
// with s = max(alpha^2, gamma^2), and the line's walk bounds (adj_line_bounds): values uniform
// over the line's wave in k_adjoint, computed here once rather than on each of its lanes.
__global__ __launch_bounds__(kThreads) void k_adj_lines(AdjArgs a) {
  const PrepArgs& pa = a.pa;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= pa.N) return;
  const int32_t c = pa.perm[i];
  const double Sref = pa.ovr_S ? pa.ovr_S[c] : pa.Sref[i];
  const double gref = pa.ovr_g ? pa.ovr_g[c] : pa.gref[i];
  const double nexp = pa.ovr_n ? pa.ovr_n[c] : pa.nexp[i];
  const double nu0 = pa.nu[i];
  const double E = pa.E[i];
  const double Rs = pa.q_ratio * exp(pa.c2E_coef * E) * (expm1(-pa.c2_over_T * nu0) / expm1(-pa.c2_over_Tref * nu0));
  const double S = Rs * Sref;
  const double gfac = exp(nexp * pa.log_tr) * pa.pfac;  // gamma / gamma_ref
  const double gam = gref * gfac;
  const double T = a.T;
  const double c2nu = pa.c2_over_T * nu0;
  const double dlnS_dT = -a.q_b / T + pa.c2_over_T * E / T - (c2nu / T) / expm1(c2nu);
  double* r = a.lrec + 8 * i;
  r[0] = S;
  r[1] = gam;
  r[2] = Rs;
  r[3] = gfac;
  r[4] = S * dlnS_dT;
  r[5] = nexp * gam / T;
  const double alpha = nu0 * pa.beta;
  const double a2d = alpha * alpha, g2d = gam * gam;
  const double scd = a2d > g2d ? a2d : g2d;
  r[6] = 1.0 / sqrt(scd);
  r[7] = 1.0 / alpha;
  adj_line_bounds(a, alpha, g2d, a.grec[i], reinterpret_cast<int4*>(a.lzone) + 4 * i);
}

constexpr int kAdjSpansPerPass = kWave / kNodes;  // far units per wave pass (one lane per node)

__device__ __forceinline__ int floor_div4(int x) { return x >= 0 ? x / 4 : -((-x + 3) / 4); }

// One far-span pass: lanes 16 q + k evaluate the profile polynomials of the set P at node k of
// span s (lane-dependent), weighted by that span's node weight G of dL/dk over the line's points.
template <int DV, int DA, int DG>
__device__ __forceinline__ void adj_far(const AdjPoly& P, float G, float xoff, float xk, float dnh, float dh, float gh,
                                        float& bV, float& bA, float& bG) {
  const float D = __builtin_fmaf(xoff, dnh, __builtin_fmaf(xk, dnh, dh));
  const float q = __builtin_amdgcn_rcpf(__builtin_fmaf(D, D, gh * gh));
  const float gq = G * q;
  bV = __builtin_fmaf(gq, adj_horner1<DV>(P.v, q), bV);
  bA = __builtin_fmaf(gq, adj_horner1<DA>(P.da, q), bA);
  bG = __builtin_fmaf(gq, adj_horner1<DG>(P.dg, q), bG);
}

__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(5))) void k_adjoint(AdjArgs a) {
  __shared__ AdjPoly sP[kWavesPerWG][3];
  __shared__ float sU[6][8], sT[6][8];
  const int tid = threadIdx.x, lane = tid & 63;
  if (tid < 48) {
    sU[tid >> 3][tid & 7] = c_adjU[tid >> 3][tid & 7];
    sT[tid >> 3][tid & 7] = c_adjT[tid >> 3][tid & 7];
  }
  __syncthreads();
  // the far units' node weights per level (uniform pointers: a lane selects one without a
  // memory access)
  static_assert(kAdjLevels == 3, "one pointer per far-unit level");
  const double* const gp0 = a.gpref[0];
  const double* const gp1 = a.gpref[1];
  const double* const gp2 = a.gpref[2];
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t nw = (int64_t)gridDim.x * kWavesPerWG;
  const PrepArgs& pa = a.pa;
  // node position of this lane in a far unit of each level (node k = lane mod kNodes)
  const int kn = lane & (kNodes - 1);
  float xk0 = 0.0f, xk1 = 0.0f, xk2 = 0.0f;
#pragma unroll
  for (int k = 0; k < kNodes; ++k) {
    xk0 = kn == k ? node_pos(kAdjSpan, kNodes, k) : xk0;
    xk1 = kn == k ? node_pos(4 * kAdjSpan, kNodes, k) : xk1;
    xk2 = kn == k ? node_pos(16 * kAdjSpan, kNodes, k) : xk2;
  }
  long long n_eval = 0;  // evaluations this wave made (statistics only)
  const double inv_dnu = 1.0 / a.dnu, inv_2T = 0.5 / a.T;
  for (int64_t i = (int64_t)blockIdx.x * kWavesPerWG + wv; i < pa.N; i += nw) {
    // every per-line value is loaded here, before any store of the line (one memory latency)
    const double* lr = a.lrec + 8 * i;
    const double lS = lr[0], gam = lr[1], lRs = lr[2], lgf = lr[3], lST = lr[4], lgT = lr[5];
    const double lrsd = lr[6], lia = lr[7];
    const int4* lb = reinterpret_cast<const int4*>(a.lzone) + 4 * i;
    const int4 b0 = lb[0], b1 = lb[1], b2 = lb[2], b3 = lb[3];
    const double nu0 = pa.nu[i];
    const int32_t lc = pa.perm[i];
    const double alpha = nu0 * pa.beta;
    const int4 gr = a.grec[i];
    const int jref = gr.y, jlo0 = gr.z, jhi0 = gr.w;
    double SVw = 0.0, SGw = 0.0, SAw = 0.0, SVc = 0.0, SGc = 0.0, SAc = 0.0;
    const double a2d = alpha * alpha, g2d = gam * gam;
    const double scd = a2d > g2d ? a2d : g2d;
    if (jlo0 <= jhi0 && scd > 0.0) {
      const double rsd = lrsd, isc = rsd * rsd;  // 1/sqrt(s), 1/s
      const float rs = (float)rsd;
      const float dh = __int_as_float(gr.x) * rs, dnh = (float)a.dnu * rs, gh = (float)gam * rs;
      // coefficient sets of this line, 2, 3 and 6 terms (chunks of series order <= 1, 2 and the
      // rest), one set per 16-lane group, one power of q per lane
      {
        const float ah = (float)(a2d * isc), gh2 = (float)(g2d * isc);
        const int M = lane & 15, set = lane >> 4;
        if (M < kAdjDeg && set < 3) {
          float v, da, dg;
          adj_coef_rt(set == 0 ? 2 : (set == 1 ? 3 : kKmax + 1), M, ah, gh2, sU, sT, v, da, dg);
          sP[wv][set].v[M] = v; sP[wv][set].da[M] = da; sP[wv][set].dg[M] = dg;
        }
      }
      // the line's zones and far-unit limits (adj_line_bounds), in scalar registers
      const int bnd[16] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w, b2.x, b2.y, b2.z, b2.w, b3.x, b3.y, b3.z, b3.w};
      int zlo[kKmax], zhi[kKmax];
#pragma unroll
      for (int K = 0; K < kKmax; ++K) {
        zlo[K] = __builtin_amdgcn_readfirstlane(bnd[K]);
        zhi[K] = __builtin_amdgcn_readfirstlane(bnd[kKmax + K]);
      }
      const double ia = lia;
      // core points in units of alpha, FP32: x = (j - jref) h + x0 (x0 from the grid record's
      // offset, subtracted in FP64)
      const float yf = (float)(gam * ia), x0f = __int_as_float(gr.x) * (float)ia, hf = (float)(a.dnu * ia);
      const float zc2 = a.zK[kKmax - 1] * a.zK[kKmax - 1];
      float bV = 0.f, bG = 0.f, bA = 0.f;
      // spans sa..sb of the line's points: far on the left up to sL, far on the right from sR,
      // direct in between (the direct spans are the ones near the centre and its core zone)
      const int sa = jlo0 / kAdjSpan, sb = jhi0 / kAdjSpan;
      // the last far unit of each level on the left and the first on the right (level L: units of
      // kAdjSpan 4^L points)
      int uL[kAdjLevels], uR[kAdjLevels];
#pragma unroll
      for (int L = 0; L < kAdjLevels; ++L) {
        uL[L] = __builtin_amdgcn_readfirstlane(bnd[2 * kKmax + L]);
        uR[L] = __builtin_amdgcn_readfirstlane(bnd[2 * kKmax + kAdjLevels + L]);
      }
      const int sL = uL[0] < sb ? (uL[0] < sa - 1 ? sa - 1 : uL[0]) : sb;
      const int sR = uR[0] > sa ? (uR[0] > sb + 1 ? sb + 1 : uR[0]) : sa;
      // direct points: the line's points in spans sL + 1 .. sR - 1, in steps of kAdjP x 64 points
      // (kAdjP per lane); the first step's dL/dk is loaded now (its latency overlaps the far
      // passes), each later step's one step ahead
      const int jlo = jlo0 > (sL + 1) * kAdjSpan ? jlo0 : (sL + 1) * kAdjSpan;
      const int jhi = jhi0 < sR * kAdjSpan - 1 ? jhi0 : sR * kAdjSpan - 1;
      if (jhi >= jlo) n_eval += jhi - jlo + 1;
      constexpr int kAdjP = 4, kStep = kAdjP * kWave;
      // dL/dk of a step's points, loaded without a condition from indices clamped to the cut range
      // (no select waits on the load); points beyond jhi are masked where they are used
      float gcur[kAdjP];
      auto load_first_step = [&]() {
#pragma unroll
        for (int p = 0; p < kAdjP; ++p) {
          const int j = jlo + p * kWave + lane;
          gcur[p] = a.g[j < jhi0 ? j : jhi0];
        }
      };
      // walking outward from the direct spans, a side switches to the next level at the first
      // unit boundary whose unit of that level is far: left, spans sL down to s1 + 1, level-1
      // units t1 down to u2 + 1, level-2 units t2 = u2 / 4 down; right, spans sR up to r1 - 1,
      // level-1 units f1 = r1 / 4 up to v2 - 1, level-2 units f2 = v2 / 4 up (each level clipped
      // to the cut range)
      int n0L, n1L = 0, n2L = 0, t1 = 0, t2 = 0, n0R, n1R = 0, n2R = 0, f1 = 0, f2 = 0;
      {
        const int s1 = min(4 * floor_div4(sL + 1) - 1, 4 * uL[1] + 3);
        if (s1 < sa) {
          n0L = sL - sa + 1;
        } else {
          n0L = sL - s1;
          t1 = s1 / 4;
          const int b1 = sa / 4;
          const int u2 = min(4 * floor_div4(t1 + 1) - 1, 4 * uL[2] + 3);
          if (u2 < b1) {
            n1L = t1 - b1 + 1;
          } else {
            n1L = t1 - u2;
            t2 = u2 / 4;
            n2L = t2 - sa / 16 + 1;
          }
        }
        const int r1 = max(4 * ((sR + 3) / 4), 4 * uR[1]);
        if (r1 > sb) {
          n0R = sb - sR + 1;
        } else {
          n0R = r1 - sR;
          f1 = r1 / 4;
          const int e1 = sb / 4;
          const int v2 = max(4 * ((f1 + 3) / 4), 4 * uR[2]);
          if (v2 > e1) {
            n1R = e1 - f1 + 1;
          } else {
            n1R = v2 - f1;
            f2 = v2 / 4;
            n2R = sb / 16 - f2 + 1;
          }
        }
        n0L = n0L < 0 ? 0 : n0L;
        n0R = n0R < 0 ? 0 : n0R;
      }
      const int nF = n0L + n1L + n2L + n0R + n1R + n2R;
      n_eval += (long long)kNodes * nF;
      // this lane's far unit of pass entry f (level and index); f is clamped to the last unit
      auto unit_of = [&](int f, int& lv, int& u) {
        int r = f < nF ? f : nF - 1;
        if (r < n0L) { lv = 0; u = sL - r; }
        else if ((r -= n0L) < n1L) { lv = 1; u = t1 - r; }
        else if ((r -= n1L) < n2L) { lv = 2; u = t2 - r; }
        else if ((r -= n2L) < n0R) { lv = 0; u = sR + r; }
        else if ((r -= n0R) < n1R) { lv = 1; u = f1 + r; }
        else { lv = 2; u = f2 + (r - n1R); }
      };
      // the far passes in chunks: the node weights of a chunk's passes are loaded together
      // (independent loads in flight at once), then the passes are evaluated
      constexpr int kFarChunk = 6;
      for (int fc = 0; fc < nF; fc += kFarChunk * kAdjSpansPerPass) {
        float Gc[kFarChunk];
#pragma unroll
        for (int c = 0; c < kFarChunk; ++c) {
          const int f = fc + c * kAdjSpansPerPass + (lane >> 4);
          int lv, u;
          unit_of(f, lv, u);
          const int Wl = kAdjSpan << (2 * lv);
          const int s0 = u * Wl;
          const int pa0 = (jlo0 > s0 ? jlo0 : s0) - s0, pb = (jhi0 < s0 + Wl - 1 ? jhi0 : s0 + Wl - 1) - s0;
          const double* pr = (lv == 0 ? gp0 : (lv == 1 ? gp1 : gp2)) + ((int64_t)u * kNodes + kn) * Wl;
          const double hi = pr[pb];
          const double lo = pa0 > 0 ? pr[pa0 - 1] : 0.0;
          Gc[c] = f < nF ? (float)(hi - lo) : 0.0f;
        }
        load_first_step();  // in flight with the chunk's loads (the same values in every chunk)
#pragma unroll
        for (int c = 0; c < kFarChunk; ++c) {
          const int fb = fc + c * kAdjSpansPerPass;
          if (fb >= nF) break;
          asm volatile("" ::: "memory");
          int lv, u;
          unit_of(fb + (lane >> 4), lv, u);
          const int Wl = kAdjSpan << (2 * lv);
          const int s0 = u * Wl;
          const int pa0 = (jlo0 > s0 ? jlo0 : s0) - s0, pb = (jhi0 < s0 + Wl - 1 ? jhi0 : s0 + Wl - 1) - s0;
          const float G = Gc[c];
          // series terms for this pass: one more than the profile needs at the pass's points
          int KL = 2;
#pragma unroll
          for (int z = 0; z < kKmax - 1; ++z) KL += (s0 + pb >= zlo[z] && s0 + pa0 <= zhi[z]) ? 1 : 0;
          const int KD = 2 + (__ballot(KL >= 3) != 0ull ? 1 : 0) + (__ballot(KL >= 4) != 0ull ? 1 : 0);
          const float xoff = (float)(s0 - jref);
          const float xk = lv == 0 ? xk0 : (lv == 1 ? xk1 : xk2);
          if (KD == 2) {
            adj_far<3, 3, 4>(sP[wv][0], G, xoff, xk, dnh, dh, gh, bV, bA, bG);
          } else if (KD == 3) {
            adj_far<5, 5, 6>(sP[wv][1], G, xoff, xk, dnh, dh, gh, bV, bA, bG);
          } else {
            adj_far<kAdjDeg - 2, kAdjDeg - 2, kAdjDeg - 1>(sP[wv][2], G, xoff, xk, dnh, dh, gh, bV, bA, bG);
          }
          SVw += (double)bV; SGw += (double)bG; SAw += (double)bA;
          bV = bG = bA = 0.f;
        }
      }
      if (nF == 0) load_first_step();
      int nstep = 0;
      for (int jc = jlo; jc <= jhi; jc += kStep) {
        // the coefficient sets are read from LDS in every step rather than held in registers
        asm volatile("" ::: "memory");
        float gnx[kAdjP] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (jc + kStep <= jhi) {  // no loads past the last step (the line's last writes would wait for them)
#pragma unroll
          for (int p = 0; p < kAdjP; ++p) {
            const int j = jc + kStep + p * kWave + lane;
            gnx[p] = a.g[j < jhi0 ? j : jhi0];
          }
        }
        const int je = jc + kStep - 1;
        // terms of the series for this step: one more than the profile needs, for dV/dalpha
        int KD = 2;
#pragma unroll
        for (int z = 0; z < kKmax - 1; ++z) KD += (je >= zlo[z] && jc <= zhi[z]) ? 1 : 0;
        const bool core_step = je >= zlo[kKmax - 1] && jc <= zhi[kKmax - 1];
        if (core_step) {
          // lanes with |z| below the last threshold take the rational approximation, the
          // others the longest series
          const AdjPoly& PP = sP[wv][2];
#pragma unroll 1
          for (int p = 0; p < kAdjP; ++p) {
            asm volatile("" ::: "memory");
            const int j = jc + p * kWave + lane;
            const float gv = j <= jhi ? gcur[p] : 0.0f;
            const float x = __builtin_fmaf((float)(j - jref), hf, x0f);
            if (__builtin_fmaf(x, x, yf * yf) < zc2) {
              float K, L;
              weideman_w32(x, yf, K, L);
              const float Kx = -2.0f * __builtin_fmaf(x, K, -yf * L);
              const float Ky = 2.0f * __builtin_fmaf(x, L, yf * K) - 1.12837916709551257f;
              const double gd = (double)gv;
              SVc += gd * (double)K;
              SGc += gd * (double)Ky;
              SAc += gd * (double)(-(K + __builtin_fmaf(x, Kx, yf * Ky)));
            } else {
              const float D = __builtin_fmaf((float)(j - jref), dnh, dh);
              const float q = __builtin_amdgcn_rcpf(__builtin_fmaf(D, D, gh * gh));
              const float gq = gv * q;
              bV = __builtin_fmaf(gq, adj_horner1<kAdjDeg - 2>(PP.v, q), bV);
              bA = __builtin_fmaf(gq, adj_horner1<kAdjDeg - 2>(PP.da, q), bA);
              bG = __builtin_fmaf(gq, adj_horner1<kAdjDeg - 1>(PP.dg, q), bG);
            }
          }
        } else if (KD == 2) {
          adj_step<kAdjP, 3, 3, 4>(sP[wv][0], jc, lane, jref, jhi, dnh, dh, gh, gcur, bV, bA, bG);
        } else if (KD == 3) {
          adj_step<kAdjP, 5, 5, 6>(sP[wv][1], jc, lane, jref, jhi, dnh, dh, gh, gcur, bV, bA, bG);
        } else {
          // rare steps near the core: one point at a time, coefficients re-read from LDS
#pragma unroll 1
          for (int p = 0; p < kAdjP; ++p) {
            asm volatile("" ::: "memory");
            float g1[1] = {gcur[0]};
            if (p == 1) g1[0] = gcur[1];
            if (p == 2) g1[0] = gcur[2];
            if (p == 3) g1[0] = gcur[3];
            adj_step<1, kAdjDeg - 2, kAdjDeg - 2, kAdjDeg - 1>(sP[wv][2], jc + p * kWave, lane, jref, jhi, dnh, dh, gh,
                                                             g1, bV, bA, bG);
          }
        }
        if (++nstep == 2) {
          SVw += (double)bV; SGw += (double)bG; SAw += (double)bA;
          bV = bG = bA = 0.f;
          nstep = 0;
        }
#pragma unroll
        for (int p = 0; p < kAdjP; ++p) gcur[p] = gnx[p];
      }
      SVw += (double)bV; SGw += (double)bG; SAw += (double)bA;
      // the wing and core sums of each lane with the line's factors, then per-wave sums (fixed
      // butterfly order)
      const double isp = 0.56418958354775628695;  // 1/sqrt(pi)
      const double ipis = isc * 0.31830988618379067154;  // 1/(pi s), s = max(alpha^2, gamma^2)
      const double GV = wave_sum64(gam * ipis * SVw + SVc * isp * ia);                 // sum g V
      const double GGs = wave_sum64(ipis * SGw + SGc * isp * ia * ia);                 // sum g dV/dgamma
      const double GAs = wave_sum64(gam * ipis * ia * SAw + SAc * isp * ia * ia);      // sum g dV/dalpha
      SVw = GV; SGw = lS * GGs; SAw = lS * GAs;
    }
    if (lane == 0) {
      // SVw, SGw, SAw now hold sum_j g_j V_ij, dL/dgamma_i, dL/dalpha_i (zero without points)
      const double GS = SVw, Gg = SGw, Ga = SAw;
      const int32_t c = lc;
      if (a.dSref) a.dSref[c] = lRs * GS;
      if (a.dgref) a.dgref[c] = (float)(lgf * Gg);
      if (a.dn) a.dn[c] = (float)(gam * pa.log_tr * Gg);
      a.contrib[2 * i] = GS * lST + Ga * alpha * inv_2T - Gg * lgT;
      a.contrib[2 * i + 1] = gam * Gg;
    }
  }
  if (a.stats && lane == 0) a.stats[(int64_t)blockIdx.x * kWavesPerWG + wv] = n_eval;
}

// Fixed-order sums of the per-line (dL/dT, dL/dlnP) terms: per-block tree sums, then one block.
__global__ __launch_bounds__(1024) void k_reduce2(const double* __restrict__ in, int64_t N, double* __restrict__ out) {
  __shared__ double s0[1024], s1[1024];
  const int64_t per = (N + gridDim.x - 1) / gridDim.x;
  const int64_t b0 = (int64_t)blockIdx.x * per, b1 = b0 + per < N ? b0 + per : N;
  double a0 = 0.0, a1 = 0.0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += 1024) { a0 += in[2 * i]; a1 += in[2 * i + 1]; }
  s0[threadIdx.x] = a0;
  s1[threadIdx.x] = a1;
  __syncthreads();
  for (int st = 512; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) { s0[threadIdx.x] += s0[threadIdx.x + st]; s1[threadIdx.x] += s1[threadIdx.x + st]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) { out[2 * blockIdx.x] = s0[0]; out[2 * blockIdx.x + 1] = s1[0]; }
}

// k = (ADD ? k : 0) + fixed-order (item 0, 1, ...) sum of the partial spans of multi-item
// spans (wing pass: k =; line-core pass: k +=).
template <int P, bool ADD>
__global__ __launch_bounds__(kThreads) void k_combine(VoigtArgs a) {
  constexpr int W = kWave * P;
  const int g = blockIdx.x;
  const int nc = a.tile_nc[g];
  if (nc <= 1) return;
  const PairDesc pd = a.pairs[find_pair(a.pairs, a.n_pairs, g)];
  const int64_t span0 = (int64_t)(g - pd.tile_base) * W;
  const int base = a.item_base[g];
  // items beyond the partial rows were not stored (flagged by their pass): the span gets NaN
  const bool lost = base + nc > a.items_cap;
  for (int local = threadIdx.x; local < W; local += kThreads) {
    if (span0 + local >= pd.n) continue;
    double acc = lost ? (double)NAN : 0.0;
    for (int c = 0; c < nc && base + c < a.items_cap; ++c) acc += (double)a.partial[(int64_t)(base + c) * W + local];
    float* dst = a.k + pd.out_off + span0 + local;
    *dst = ADD ? *dst + (float)acc : (float)acc;
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

hipError_t launch_validate(const double* nu, int64_t N, unsigned long long* mm, int* flags, hipStream_t st) {
  hipLaunchKernelGGL(k_validate_init, dim3(1), dim3(1), 0, st, mm, flags);
  int64_t blocks = blocks_for(N, kThreads);
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_validate, dim3((unsigned)blocks), dim3(kThreads), 0, st, nu, N, mm, flags);
  return hipGetLastError();
}

hipError_t launch_keys(const double* nu, const double* S, const double* E, const double* g, const double* n,
                       int64_t N, KeyMap km, uint32_t* keys, int32_t* vals, double* rec, int* flags,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_keys, dim3(blocks_for(N, kThreads)), dim3(kThreads), 0, st, nu, S, E, g, n, N, km, keys,
                     vals, rec, flags);
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

hipError_t launch_gather(const int32_t* perm, int64_t N, const double* rec, double* onu, double* oS, double* oE,
                         double* og, double* on, hipStream_t st) {
  hipLaunchKernelGGL(k_gather, dim3(blocks_for(N, kThreads)), dim3(kThreads), 0, st, perm, N, rec, onu, oS, oE, og,
                     on);
  return hipGetLastError();
}

hipError_t launch_prep(const PrepArgs& a, float* S_T, float* gT, double* S64, double* a64, double* g64,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_prep, dim3(blocks_for(a.N, kThreads)), dim3(kThreads), 0, st, a, S_T, gT, S64, a64, g64);
  return hipGetLastError();
}

hipError_t launch_fill_pairs(const PairDesc* host_pairs, int count, PairDesc* dst, int* status, hipStream_t st) {
  for (int c0 = 0; c0 < count; c0 += kFillPairs) {
    PairPack pk;
    pk.count = count - c0 < kFillPairs ? count - c0 : kFillPairs;
    for (int i = 0; i < pk.count; ++i) pk.p[i] = host_pairs[c0 + i];
    hipLaunchKernelGGL(k_fill_pairs, dim3(1), dim3(64), 0, st, pk, dst + c0, c0 == 0 ? status : nullptr);
  }
  return hipGetLastError();
}

hipError_t launch_worklist(const uint32_t* keys, int64_t N, KeyMap km, double numin, double numax,
                           const PairDesc* pairs, int n_pairs,
                           int n_tiles_total, int tile_w, double cut, double core_z, int chunk, int32_t* lo,
                           int32_t* hi, int32_t* nc, int4* far, int32_t* nf, int far_chunk, double far_z,
                           int direct_only, double core_pad, hipStream_t st) {
  hipLaunchKernelGGL(k_worklist, dim3(blocks_for(n_tiles_total, kThreads)), dim3(kThreads), 0, st, keys, N, km,
                     numin, numax, pairs, n_pairs, n_tiles_total, tile_w, cut, core_z, chunk, lo, hi, nc, far, nf,
                     far_chunk, far_z, direct_only, core_pad);
  return hipGetLastError();
}

hipError_t launch_item_scan(const int32_t* nc, int n_tiles_total, int32_t* item_base, int* counter,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_item_scan, dim3(1), dim3(1024), 0, st, nc, n_tiles_total, item_base, counter);
  return hipGetLastError();
}

hipError_t launch_gridrec(const double* nu, int64_t N, double nu_start, double dnu, int64_t n, double cut,
                          int4* grec, hipStream_t st) {
  hipLaunchKernelGGL(k_gridrec, dim3(blocks_for(N, kThreads)), dim3(kThreads), 0, st, nu, N, nu_start, dnu, n, cut,
                     grec);
  return hipGetLastError();
}

// Tunings: P (64-point slots per wave; tile width 256 P) in {1, 2, 4, 8}; a wave stages 64 lines
// (one per lane) per LDS batch.
template <template <int> class F, typename... A>
static hipError_t by_slots(int slots, A... args) {
  switch (slots) {
    case 1: return F<1>::run(args...);
    case 2: return F<2>::run(args...);
    case 4: return F<4>::run(args...);
    case 8: return F<8>::run(args...);
    default: return hipErrorInvalidValue;
  }
}

template <int P>
struct WingL {
  static hipError_t run(const VoigtArgs& a, int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_wing<P>, dim3(grid), dim3(kWave), 0, st, a);
    return hipGetLastError();
  }
};
template <int P>
struct CoreL {
  static hipError_t run(const VoigtArgs& a, int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_core<P>, dim3(grid), dim3(kWave), 0, st, a);
    return hipGetLastError();
  }
};
template <int P>
struct CombineL {
  static hipError_t run(const VoigtArgs& a, bool add, hipStream_t st) {
    if (add) hipLaunchKernelGGL((k_combine<P, true>), dim3((unsigned)a.n_tiles_total), dim3(kThreads), 0, st, a);
    else hipLaunchKernelGGL((k_combine<P, false>), dim3((unsigned)a.n_tiles_total), dim3(kThreads), 0, st, a);
    return hipGetLastError();
  }
};
template <int P>
struct WingOcc {
  static hipError_t run(int* nb) { return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, k_wing<P>, kWave, 0); }
};
template <int P>
struct CoreOcc {
  static hipError_t run(int* nb) { return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, k_core<P>, kWave, 0); }
};

hipError_t launch_span_segments(const uint32_t* keys, int64_t N, KeyMap km, double numin, double numax,
                                const PairDesc* spairs, const PairDesc* tpairs, int n_pairs, int n_spans,
                                int span_w, double cut, double far_z, const int4* tile_far, int chunk,
                                SpanSeg* segs, int32_t* nc, int direct_only, hipStream_t st) {
  hipLaunchKernelGGL(k_span_segments, dim3(blocks_for(n_spans, kThreads)), dim3(kThreads), 0, st, keys, N, km,
                     numin, numax, spairs, tpairs, n_pairs, n_spans, span_w, cut, far_z, tile_far, chunk, segs, nc,
                     direct_only);
  return hipGetLastError();
}

hipError_t launch_wing(const VoigtArgs& a, int slots, int grid, hipStream_t st) {
  return by_slots<WingL>(slots, a, grid, st);
}

hipError_t launch_core(const VoigtArgs& a, int slots, int grid, hipStream_t st) {
  return by_slots<CoreL>(slots, a, grid, st);
}

hipError_t launch_combine(const VoigtArgs& a, int slots, bool add, hipStream_t st) {
  return by_slots<CombineL>(slots, a, add, st);
}

hipError_t launch_cut_bounds(const double* nu, const int32_t* perm, int64_t N, double nu_start, double dnu,
                             int64_t n, double cut, int32_t* jlo, int32_t* jhi, hipStream_t st) {
  hipLaunchKernelGGL(k_cut_bounds, dim3(blocks_for(N, kThreads)), dim3(kThreads), 0, st, nu, perm, N, nu_start,
                     dnu, n, cut, jlo, jhi);
  return hipGetLastError();
}

hipError_t launch_far(const FarArgs& a, int cls, int grid, hipStream_t st) {
  if (cls == 0) hipLaunchKernelGGL(k_far<0>, dim3(grid), dim3(kThreads), 0, st, a);
  else hipLaunchKernelGGL(k_far<1>, dim3(grid), dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_combine_far(const FarArgs& a, hipStream_t st) {
  if (a.n_tiles_total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_combine_far, dim3(a.n_tiles_total), dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

int adj_max_blocks_per_cu() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_adjoint, kThreads, 0) != hipSuccess) return 1;
  return n > 0 ? n : 1;
}

int far_max_blocks_per_cu() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_far<0>, kThreads, 0) != hipSuccess) return 1;
  return n > 0 ? n : 1;
}

hipError_t launch_adj_nodes(const float* g, int64_t n, int level, const double* w, double* gpref, hipStream_t st) {
  if (level == 0)
    hipLaunchKernelGGL(k_adj_nodes<kAdjSpan>, dim3(blocks_for(n, kAdjSpan)), dim3(kAdjSpan), 0, st, g, n, w, gpref);
  else if (level == 1)
    hipLaunchKernelGGL(k_adj_nodes<4 * kAdjSpan>, dim3(blocks_for(n, 4 * kAdjSpan)), dim3(kAdjSpan), 0, st, g, n, w,
                       gpref);
  else
    hipLaunchKernelGGL(k_adj_nodes<16 * kAdjSpan>, dim3(blocks_for(n, 16 * kAdjSpan)), dim3(kAdjSpan), 0, st, g, n,
                       w, gpref);
  return hipGetLastError();
}

hipError_t launch_adjoint(const AdjArgs& a, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_lines, dim3(blocks_for(a.pa.N, kThreads)), dim3(kThreads), 0, st, a);
  hipLaunchKernelGGL(k_adjoint, dim3(grid), dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_reduce2(const double* contrib, int64_t N, double* partial, int n_partial, double* out,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_reduce2, dim3(n_partial), dim3(1024), 0, st, contrib, N, partial);
  hipLaunchKernelGGL(k_reduce2, dim3(1), dim3(1024), 0, st, (const double*)partial, (int64_t)n_partial, out);
  return hipGetLastError();
}

int core_max_blocks_per_cu(int slots) {
  int nb = 0;
  (void)by_slots<CoreOcc>(slots, &nb);
  return nb > 0 ? nb : 1;
}

int wing_max_blocks_per_cu(int slots) {
  int nb = 0;
  (void)by_slots<WingOcc>(slots, &nb);
  return nb > 0 ? nb : 1;
}

template <int P>
struct DirectL {
  static hipError_t run(const VoigtArgs& a, const float* plin, int prof, int grid, hipStream_t st) {
    switch (prof) {
      case kProfVoigt: hipLaunchKernelGGL((k_direct<P, kProfVoigt>), dim3(grid), dim3(kWave), 0, st, a, plin); break;
      case kProfLorentz: hipLaunchKernelGGL((k_direct<P, kProfLorentz>), dim3(grid), dim3(kWave), 0, st, a, plin); break;
      case kProfDoppler: hipLaunchKernelGGL((k_direct<P, kProfDoppler>), dim3(grid), dim3(kWave), 0, st, a, plin); break;
      case kProfBinned: hipLaunchKernelGGL((k_direct<P, kProfBinned>), dim3(grid), dim3(kWave), 0, st, a, plin); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
};

hipError_t launch_direct(const VoigtArgs& a, const float* plin, int prof, int slots, int grid, hipStream_t st) {
  return by_slots<DirectL>(slots, a, plin, prof, grid, st);
}

template <int P>
struct DirectOcc {
  static hipError_t run(int* nb) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, k_direct<P, kProfBinned>, kWave, 0);
  }
};
int direct_max_blocks_per_cu(int slots) {
  int nb = 0;
  (void)by_slots<DirectOcc>(slots, &nb);
  return nb > 0 ? nb : 1;
}

hipError_t launch_gridrec_ex(const GridRecArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_gridrec_ex, dim3(blocks_for(a.pa.N, kThreads)), dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_line_stats(const double* gref, const double* nexp, int64_t N, unsigned long long* out,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_line_stats_init, dim3(1), dim3(1), 0, st, out);
  int64_t blocks = blocks_for(N, kThreads);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_line_stats, dim3((unsigned)blocks), dim3(kThreads), 0, st, gref, nexp, N, out);
  return hipGetLastError();
}

hipError_t launch_scatter_grec(const int4* grec, const float* plin, const int32_t* perm, int64_t N, int32_t* jlo,
                               int32_t* jhi, float* plin_out, hipStream_t st) {
  hipLaunchKernelGGL(k_scatter_grec, dim3(blocks_for(N, kThreads)), dim3(kThreads), 0, st, grec, plin, perm, N, jlo,
                     jhi, plin_out);
  return hipGetLastError();
}

hipError_t launch_hitran_check(const double* gself, const double* delta, int64_t N, int* flags,
                               unsigned long long* out, hipStream_t st) {
  hipLaunchKernelGGL(k_hitran_check_init, dim3(1), dim3(1), 0, st, flags, out);
  int64_t blocks = blocks_for(N, kThreads);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_hitran_check, dim3((unsigned)blocks), dim3(kThreads), 0, st, gself, delta, N, flags, out);
  return hipGetLastError();
}

hipError_t launch_gather2(const int32_t* perm, int64_t N, const double* a, const double* b, double* oa, double* ob,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_gather2, dim3(blocks_for(N, kThreads)), dim3(kThreads), 0, st, perm, N, a, b, oa, ob);
  return hipGetLastError();
}

hipError_t launch_shift_keys(const double* nu, const double* delta, int64_t N, double pshift, KeyMap km,
                             uint32_t* keys, int32_t* vals, hipStream_t st) {
  hipLaunchKernelGGL(k_shift_keys, dim3(blocks_for(N, kThreads)), dim3(kThreads), 0, st, nu, delta, N, pshift, km,
                     keys, vals);
  return hipGetLastError();
}

hipError_t launch_shift_gather(const ShiftArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_shift_gather, dim3(blocks_for(a.N, kThreads)), dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_fill0(float* k, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill0, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, st, k, n);
  return hipGetLastError();
}

hipError_t launch_accumulate(float* k, const float* t, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_accumulate, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, st, k, t, n);
  return hipGetLastError();
}

hipError_t upload_weideman40(const double* coef, double L) {
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_weid40), coef, sizeof(double) * kWeidN40);
  if (e != hipSuccess) return e;
  return hipMemcpyToSymbol(HIP_SYMBOL(c_weid40L), &L, sizeof(double));
}

hipError_t upload_weideman(const double* coef, double L) {
  float c32[kWeidN];
  for (int i = 0; i < kWeidN; ++i) c32[i] = (float)coef[i];
  const float L32 = (float)L;
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_weid32), c32, sizeof(c32));
  if (e != hipSuccess) return e;
  return hipMemcpyToSymbol(HIP_SYMBOL(c_weidL32), &L32, sizeof(float));
}

}  // namespace hk
