// Host side of the opacity library: argument validation, memory layout, planning of the
// tile work list, launches, graph cache and timing. The C ABI is declared in include/hk.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "hk.h"
#include "hk_internal.h"

struct hk_lines {
  int device;
  int64_t N;
  hk_species sp;
  hk::KeyMap km;
  double numin, numax;
  double *nu, *Sref, *E, *gref, *nexp;  // sorted by bin key (stable)
  uint32_t* keys;                       // sorted bin keys
  int32_t* perm;                        // sorted position -> caller index
  void* mem;
  size_t mem_bytes;                     // size of the block mem (from the block cache)
  // largest gamma_ref and range of n over the list (the bound of Lorentz-multiple cutting
  // lengths), computed on first need
  std::mutex stats_mu;
  bool have_stats = false;
  double gref_max = 0.0, n_min = 0.0, n_max = 0.0;
  // a HITRAN-style list (hk_prepare_lines_hitran): gamma_self and delta_air in the handle's order,
  // the largest |delta_air| and gamma_self; a view of such a list at one pressure, sorted by the
  // shifted centres, sets nu_pos (nu then holds the transition wavenumbers)
  double* gself = nullptr;
  double* delta = nullptr;
  void* mem2 = nullptr;
  size_t mem2_bytes = 0;
  double dmax = 0.0, gself_max = 0.0;
  const double* nu_pos = nullptr;
  double shift_max = 0.0;  // a view: the largest |centre - transition wavenumber|
  // the streams work was issued on through the handle, each with an event recorded after its
  // last call there (hk_release_lines waits for these); untracked: a use that could not be
  // recorded (a capturing stream, more than kUseSlots streams, or an allocation-free call on a
  // new stream), after which release waits for the whole device
  static constexpr int kUseSlots = 8;
  std::mutex use_mu;
  hipStream_t use_stream[kUseSlots] = {};
  hipEvent_t use_event[kUseSlots] = {};
  int n_use = 0;
  bool untracked = false;
};

namespace {

// Physical constants of the product (the paper prints k_B with eq. gammaD and c with eq. S;
// h and the atomic mass unit are CODATA 2010 values of the same vintage).
constexpr double kB = 1.3806489e-16;      // erg / K
constexpr double kC = 2.99792458e10;      // cm / s
constexpr double kH = 6.62606957e-27;     // erg s
constexpr double kAMU = 1.660538921e-24;  // g
constexpr double kC2 = kH * kC / kB;      // cm K

// |z| thresholds of the far-wing series orders 1..5: at and above zK[K-1] the series of order K
// is within 1.4e-7 of the line's peak value Re w(iy) (and within 2e-6 relative); below the last
// one the core approximation is used
constexpr double kZK[hk::kKmax] = {870.0, 37.5, 13.8, 8.7, 6.75};
// the same for orders 1..9 (orders 6-9 within 1.3e-7 of the peak); the default path's wing pass
// takes lines next to their cores down to |z| = 4.4 with them, and its core pass the rest
constexpr double kZW[hk::kKw] = {870.0, 37.5, 13.8, 8.7, 6.75, 5.65, 5.0, 4.65, 4.4};

// |z| below which a pair is a core point: the default path's (the wing pass has orders up to
// kKw), or that of the options path (k_direct has orders up to kKmax)
double core_threshold(bool default_path) { return default_path ? kZW[hk::kKw - 1] : kZK[hk::kKmax - 1]; }

thread_local std::string g_err;
thread_local hk_timings g_tim = {-1, -1, -1, -1, -1, -1, 0, 0, 0, 0, -1, -1, -1, -1, {-1, -1, -1, -1, -1, -1, -1, -1}, 0, -1};

hk_status fail(hk_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HK_HIP(call)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess) return fail(HK_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

bool env_flag(const char* name, bool dflt) {
  const char* v = getenv(name);
  if (!v || !*v) return dflt;
  return !(v[0] == '0' || v[0] == 'n' || v[0] == 'N' || v[0] == 'f' || v[0] == 'F');
}

int env_int(const char* name, int dflt) {
  const char* v = getenv(name);
  return (v && *v) ? atoi(v) : dflt;
}

struct DevInfo {
  int cus = 0;
  int wing_per_cu[4] = {};    // wing kernel (one-wave workgroups) occupancy per slots 1/2/4/8
  int core_per_cu[4] = {};    // core kernel (one-wave workgroups) occupancy per slots
  double* cheb_w[4] = {};     // device: Lagrange weights of the span nodes, per slots 1/2/4/8
  float cheb_x[4][hk::kNodes] = {};  // node positions relative to the span's first point
  double* tile_w[4] = {};     // device: the same for the tile-far tile (4 spans), per slots
  float tile_x[4][hk::kNodes] = {};
  double* tile_w8[4] = {};    // device: the tile's very-far nodes (kFar8Nodes), per slots
  float tile_x8[4][hk::kFar8Nodes] = {};
  double* far8_w[4] = {};     // device: the span's very-far nodes (kFar8Nodes), per slots
  float far8_x[4][hk::kFar8Nodes] = {};
  double* mid_w[4] = {};      // device: the span's middle-distance nodes (kMidNodes), per slots
  float mid_x[4][hk::kMidNodes] = {};
  float* mask_w[4] = {};      // device: the span's nodes for lines with a cut bound on it (FP32)
  float mask_x[4][hk::kMaskNodes] = {};
  double* adj_w[hk::kAdjLevels] = {};  // device: node weights of the adjoint's far units, per level
  int far_per_cu = 1;         // tile-far kernel occupancy
  int adj_per_cu = 1;         // adjoint kernel occupancy
  int direct_per_cu[4] = {};  // direct-evaluation kernel occupancy per slots
  void* scratch = nullptr;    // device address of the allocation-free entry point's scratch array
  unsigned long long* stats_buf = nullptr;  // device: line statistics (3 words)
};
std::mutex g_stats_mu;

std::mutex g_mu;
std::map<int, DevInfo> g_dev;

// Cached graphs of batched calls, keyed by every argument value and pointer of the call.
struct GraphEntry {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};
std::mutex g_graph_mu;
std::map<std::string, GraphEntry> g_graphs;
std::map<int, hipStream_t> g_capture_stream;  // per device

// Weideman (1994) coefficients: a = Re DFT(fftshift(f)) / (2M), f(t) = e^{-t^2}(L^2 + t^2) at
// t = L tan(theta/2), theta = k pi / M, k = -M+1..M-1 (f = 0 at k = -M), M = 2N, L = sqrt(N/sqrt2)
// rounded to FP32 (any L > 0 is valid with its own coefficients; an L that FP32 holds exactly
// keeps the line-core pass's FP32 evaluation consistent with its coefficients).
void weideman_coeffs(int N, double* a_out, double* L_out) {
  const int M = 2 * N, n2 = 2 * M;
  const double L = (double)(float)sqrt(N / sqrt(2.0));
  std::vector<double> f(n2), g(n2);
  f[0] = 0.0;
  for (int k = -M + 1; k <= M - 1; ++k) {
    const double th = k * M_PI / M;
    const double t = L * tan(th / 2);
    f[k + M] = exp(-t * t) * (L * L + t * t);
  }
  for (int m = 0; m < n2; ++m) g[m] = f[(m + M) % n2];
  for (int n = 1; n <= N; ++n) {
    double re = 0.0;
    for (int r = 0; r < n2; ++r) re += g[r] * cos(2.0 * M_PI * (double)n * r / n2);
    a_out[n - 1] = re / n2;
  }
  *L_out = L;
}

// m Chebyshev points of the first kind on a span of S grid points [0, S-1], at the FP32
// positions the kernels evaluate (node_pos), and for every grid point of the span the Lagrange
// weights of those nodes (barycentric form with the weights of the actual positions):
// weights[k * S + j].
void span_nodes(int S, int m, float* x_out, std::vector<double>& weights) {
  std::vector<double> x(m), bw(m);
  for (int k = 0; k < m; ++k) {
    x_out[k] = hk::node_pos(S, m, k);
    x[k] = (double)x_out[k];
  }
  for (int k = 0; k < m; ++k) {
    double p = 1.0;
    for (int i = 0; i < m; ++i)
      if (i != k) p *= (x[k] - x[i]) / (0.25 * S);  // scaled differences keep the product in range
    bw[k] = 1.0 / p;
  }
  weights.assign((size_t)m * S, 0.0);
  for (int j = 0; j < S; ++j) {
    int hit = -1;
    double den = 0.0;
    for (int k = 0; k < m; ++k) {
      const double d = j - x[k];
      if (d == 0.0) { hit = k; break; }
      den += bw[k] / d;
    }
    for (int k = 0; k < m; ++k)
      weights[(size_t)k * S + j] = hit >= 0 ? (k == hit ? 1.0 : 0.0) : (bw[k] / (j - x[k])) / den;
  }
}

// The compiled Chebyshev tables against cos.
bool cheb_tables_ok() {
  for (int m : {6, 8, 16, 32})
    for (int k = 0; k < m; ++k)
      if (std::fabs(hk::cheb_cos(m, k) - std::cos((2 * k + 1) * M_PI / (2.0 * m))) > 1e-15) return false;
  return true;
}

hk_status device_init(int* dev_out, DevInfo* info) {
  int dev = -1;
  HK_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_dev.find(dev);
  if (it == g_dev.end()) {
    hipDeviceProp_t prop;
    HK_HIP(hipGetDeviceProperties(&prop, dev));
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
      return fail(HK_EUNSUPPORTED, "device %d is %s; this library is built for gfx950", dev, prop.gcnArchName);
    if (!cheb_tables_ok()) return fail(HK_EDEVICE, "Chebyshev node table does not match cos");
    double a[hk::kWeidN], L;
    weideman_coeffs(hk::kWeidN, a, &L);
    HK_HIP(hk::upload_weideman(a, L));
    double a40[hk::kWeidN40], L40;
    weideman_coeffs(hk::kWeidN40, a40, &L40);
    HK_HIP(hk::upload_weideman40(a40, L40));
    DevInfo di;
    di.cus = prop.multiProcessorCount;
    // the scratch array's address on this device (the device is current here)
    HK_HIP(hk::scratch_address(&di.scratch));
    if (!di.scratch) return fail(HK_EDEVICE, "scratch array has no device address");
    for (int si = 0; si < 4; ++si) {
      di.wing_per_cu[si] = hk::wing_max_blocks_per_cu(1 << si);
      di.core_per_cu[si] = hk::core_max_blocks_per_cu(1 << si);
      di.direct_per_cu[si] = hk::direct_max_blocks_per_cu(1 << si);
      const int S = hk::kWave << si;
      std::vector<double> wts;
      span_nodes(S, hk::kNodes, di.cheb_x[si], wts);
      HK_HIP(hipMalloc(&di.cheb_w[si], sizeof(double) * wts.size()));  // held for the process lifetime
      HK_HIP(hipMemcpy(di.cheb_w[si], wts.data(), sizeof(double) * wts.size(), hipMemcpyHostToDevice));
      span_nodes(hk::kWavesPerWG * S, hk::kNodes, di.tile_x[si], wts);
      HK_HIP(hipMalloc(&di.tile_w[si], sizeof(double) * wts.size()));  // held for the process lifetime
      HK_HIP(hipMemcpy(di.tile_w[si], wts.data(), sizeof(double) * wts.size(), hipMemcpyHostToDevice));
      span_nodes(hk::kWavesPerWG * S, hk::kFar8Nodes, di.tile_x8[si], wts);
      HK_HIP(hipMalloc(&di.tile_w8[si], sizeof(double) * wts.size()));  // held for the process lifetime
      HK_HIP(hipMemcpy(di.tile_w8[si], wts.data(), sizeof(double) * wts.size(), hipMemcpyHostToDevice));
      span_nodes(S, hk::kFar8Nodes, di.far8_x[si], wts);
      HK_HIP(hipMalloc(&di.far8_w[si], sizeof(double) * wts.size()));  // held for the process lifetime
      HK_HIP(hipMemcpy(di.far8_w[si], wts.data(), sizeof(double) * wts.size(), hipMemcpyHostToDevice));
      span_nodes(S, hk::kMidNodes, di.mid_x[si], wts);
      HK_HIP(hipMalloc(&di.mid_w[si], sizeof(double) * wts.size()));  // held for the process lifetime
      HK_HIP(hipMemcpy(di.mid_w[si], wts.data(), sizeof(double) * wts.size(), hipMemcpyHostToDevice));
      span_nodes(S, hk::kMaskNodes, di.mask_x[si], wts);
      std::vector<float> wf(wts.begin(), wts.end());
      HK_HIP(hipMalloc(&di.mask_w[si], sizeof(float) * wf.size()));  // held for the process lifetime
      HK_HIP(hipMemcpy(di.mask_w[si], wf.data(), sizeof(float) * wf.size(), hipMemcpyHostToDevice));
    }
    for (int lv = 0; lv < hk::kAdjLevels; ++lv) {
      float xs[hk::kNodes];
      std::vector<double> wts;
      span_nodes(hk::kAdjSpan << (2 * lv), hk::kNodes, xs, wts);
      HK_HIP(hipMalloc(&di.adj_w[lv], sizeof(double) * wts.size()));  // held for the process lifetime
      HK_HIP(hipMemcpy(di.adj_w[lv], wts.data(), sizeof(double) * wts.size(), hipMemcpyHostToDevice));
    }
    di.far_per_cu = hk::far_max_blocks_per_cu();
    di.adj_per_cu = hk::adj_max_blocks_per_cu();
    HK_HIP(hipMalloc(&di.stats_buf, 4 * sizeof(unsigned long long)));  // held for the process lifetime
    it = g_dev.emplace(dev, di).first;
  }
  *dev_out = dev;
  *info = it->second;
  return HK_OK;
}

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Block cache for the library's own large device allocations (a line handle's arrays and the
// binning temporaries). A released block is kept, per device, for a later request of about its
// size instead of going back to the driver: memory another process freed can be cleared by the
// driver when it is handed out again, which cost about 0.5 s per 48 GB handle. At most
// kPoolMaxBlocks blocks and kPoolMaxBytes are kept (oldest returned first); a failed hipMalloc
// empties the device's cache and tries again; HK_NO_CACHE=1 turns the cache off and
// hk_empty_cache() returns every cached block. Blocks are cached only after the work that used
// them has completed.
struct PoolBlock {
  int dev;
  void* p;
  size_t bytes;
};
std::mutex g_pool_mu;
std::vector<PoolBlock> g_pool;  // oldest first
constexpr size_t kPoolMaxBlocks = 8;
constexpr size_t kPoolMaxBytes = size_t(128) << 30;

void pool_return(const std::vector<PoolBlock>& blocks) {
  if (blocks.empty()) return;
  int cur = -1;
  (void)hipGetDevice(&cur);
  for (const PoolBlock& b : blocks) {
    if (b.dev != cur) (void)hipSetDevice(b.dev);
    (void)hipFree(b.p);
    if (b.dev != cur && cur >= 0) (void)hipSetDevice(cur);
  }
}

// Every cached block of device dev (all devices for dev < 0) back to the driver.
void pool_drain(int dev) {
  std::vector<PoolBlock> drop;
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    for (size_t i = 0; i < g_pool.size();) {
      if (dev < 0 || g_pool[i].dev == dev) {
        drop.push_back(g_pool[i]);
        g_pool.erase(g_pool.begin() + (std::ptrdiff_t)i);
      } else {
        ++i;
      }
    }
  }
  pool_return(drop);
}

// A block of at least `bytes` on the current device dev: the smallest cached one that is no
// more than a quarter (plus 64 MiB) larger, else a new one. *got receives its size.
hipError_t pool_alloc(int dev, size_t bytes, void** p, size_t* got) {
  *p = nullptr;
  *got = 0;
  if (!env_flag("HK_NO_CACHE", false)) {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    int best = -1;
    for (size_t i = 0; i < g_pool.size(); ++i) {
      const PoolBlock& b = g_pool[i];
      if (b.dev == dev && b.bytes >= bytes && b.bytes - bytes <= bytes / 4 + (size_t(64) << 20) &&
          (best < 0 || b.bytes < g_pool[(size_t)best].bytes))
        best = (int)i;
    }
    if (best >= 0) {
      *p = g_pool[(size_t)best].p;
      *got = g_pool[(size_t)best].bytes;
      g_pool.erase(g_pool.begin() + best);
      return hipSuccess;
    }
  }
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    pool_drain(dev);
    e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      *p = nullptr;
      return e;
    }
  }
  *got = bytes;
  return hipSuccess;
}

// Returns a block whose work has completed to the cache (or to the driver without the cache).
void pool_free(int dev, void* p, size_t bytes) {
  if (!p) return;
  if (env_flag("HK_NO_CACHE", false)) {
    pool_return({PoolBlock{dev, p, bytes}});
    return;
  }
  std::vector<PoolBlock> drop;
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    g_pool.push_back(PoolBlock{dev, p, bytes});
    size_t total = 0;
    for (const PoolBlock& b : g_pool) total += b.bytes;
    while (g_pool.size() > kPoolMaxBlocks || total > kPoolMaxBytes) {
      drop.push_back(g_pool.front());
      total -= g_pool.front().bytes;
      g_pool.erase(g_pool.begin());
    }
  }
  pool_return(drop);
}

bool species_ok(const hk_species* sp) {
  return sp && std::isfinite(sp->mass_amu) && sp->mass_amu > 0 && std::isfinite(sp->T_ref) && sp->T_ref > 0 &&
         std::isfinite(sp->P_ref_atm) && sp->P_ref_atm > 0 && std::isfinite(sp->q_a) && sp->q_a > 0 &&
         std::isfinite(sp->q_b);
}

bool grid_ok(const hk_grid& g) {
  return std::isfinite(g.nu_start) && std::isfinite(g.dnu) && g.dnu > 0 && g.n >= 1 && g.n < (int64_t(1) << 31) &&
         std::isfinite(g.nu_start + (double)(g.n - 1) * g.dnu);
}

bool cut_ok(double c) { return c > 0 && (std::isfinite(c) || std::isinf(c)); }

// Profile, cutting-length mode, plinth removal and evaluation mode of a call (hk_options).
struct Opts {
  int profile = hk::kProfVoigt;
  int cut_mode = hk::kCutFixed;
  int plinth = 0;
  int direct = 0;  // default path only: every (line, point) pair evaluated in the wing pass
  int shifted = 0; // a HITRAN-style list's view at one pressure (centres moved by the shift)
  // the default path: Voigt, fixed cut, no plinth (wing, tile-far and core passes); any other
  // option runs the direct-evaluation pass (k_direct) with per-pair grid records
  bool default_path() const {
    return profile == hk::kProfVoigt && cut_mode == hk::kCutFixed && !plinth && !shifted;
  }
};

hk_status opts_from(const hk_options* o, Opts* out) {
  *out = Opts{};
  if (!o) return HK_OK;
  if (o->profile < 0 || o->profile > 3) return fail(HK_EINVAL, "profile %d", o->profile);
  if (o->cut_mode < 0 || o->cut_mode > 2) return fail(HK_EINVAL, "cut_mode %d", o->cut_mode);
  if (o->plinth != 0 && o->plinth != 1) return fail(HK_EINVAL, "plinth must be 0 or 1");
  if (o->direct != 0 && o->direct != 1) return fail(HK_EINVAL, "direct must be 0 or 1");
  out->profile = o->profile;
  out->cut_mode = o->cut_mode;
  out->plinth = o->plinth;
  out->direct = o->direct;
  return HK_OK;
}

// ------------------------------------------------------------------ forward plan
struct Plan {
  int slots = 4;
  int W = 1024;    // tile width of the tile-far pass (4 spans)
  int W_c = 256;   // span width of the wing and line-core passes (one wave, 64 slots)
  int chunk = 0;   // lines per work item of the wing pass
  int chunk_c = 0; // lines per work item of the line-core pass
  int n_pairs = 0, n_temps = 0;
  int n_tiles_total = 0;  // tiles
  int n_tiles_c = 0;      // spans
  size_t off_S = 0, off_g = 0, off_gr = 0, off_pairs = 0, off_pairs_c = 0, off_cnt = 0, off_stats = 0, total = 0;
  // the tile-far pass: per-tile window and tile-far ranges, its work items and their node sums
  size_t off_lo = 0, off_hi = 0, off_nc = 0, off_far = 0, off_nf = 0, off_ibf = 0, off_partf = 0;
  int64_t items_bound_f = 0;
  int chunk_f = 0, grid_f = 0;
  // the wing pass: per-span line segments, work items and partial spans
  size_t off_segs = 0, off_nc_w = 0, off_ib_w = 0, off_part_w = 0;
  int64_t items_bound_w = 0;
  int grid_w = 0;
  // the line-core pass: per-span line window, work items and partial spans
  size_t off_lo_c = 0, off_hi_c = 0, off_nc_c = 0, off_ib_c = 0, off_part_c = 0;
  int64_t items_bound_c = 0;
  int grid_c = 0;
  // the options path: per-pair grid records and plinth values, the direct pass's span work list
  Opts opts;
  double cut_w = 0.0;     // window half-width: the largest cutting length of any line of any pair
  double core_pad = 0.0;  // a shifted list's view: core_z beta times the largest centre shift
  size_t off_plin = 0, off_lo_d = 0, off_hi_d = 0, off_nc_d = 0, off_ib_d = 0, off_part_d = 0, off_status = 0;
  int64_t items_bound_d = 0;
  int chunk_d = 0, grid_d = 0;
  std::vector<hk::PairDesc> pairs;    // the pairs with the tile-far pass's tiling
  std::vector<hk::PairDesc> pairs_c;  // the pairs with the span tiling (wing and line-core passes)
  int n_grids = 0;
  std::vector<double> temps;
  std::vector<hk_grid> grids;  // distinct grids
};

// A tuning of the Voigt passes: slots P (span width 64 P points, tile width 256 P).
struct Tuning {
  int slots = 4;
};
inline int slot_index(int slots) { return slots == 1 ? 0 : slots == 2 ? 1 : slots == 4 ? 2 : 3; }
const Tuning kCandidates[] = {{1}, {2}, {4}, {8}};

// The tuning forced by HK_SLOTS, if any.
bool env_tuning(Tuning* t) {
  const int sl = env_int("HK_SLOTS", 0);
  if (sl == 0) return false;
  t->slots = (sl == 1 || sl == 2 || sl == 4 || sl == 8) ? sl : 4;
  return true;
}

// Tiles a line can be counted in: windows [nu_j0 - cut, nu_j1 + cut] widened by two bins.
int64_t visits_per_line(const hk_lines* L, const hk_grid& g, double cut, int W, int64_t n_tiles) {
  if (std::isinf(cut)) return n_tiles;
  const double binw = L->km.scale > 0 ? 1.0 / L->km.scale : 0.0;
  const double ell = 2.0 * cut + 4.0 * binw;
  const double v = std::floor(ell / (W * g.dnu)) + 2.0;
  return v > (double)n_tiles ? n_tiles : (int64_t)v;
}

// The largest cutting length of any line at (T, P) (+inf without a cut): the fixed length, or the
// multiple of the largest Doppler or Lorentz half-width, from the list's range of nu (and of
// gamma_ref and n, line_stats) with a relative slack for rounding.
double max_cut_length(const hk_lines* L, const Opts& o, double cut, double T, double P) {
  if (std::isinf(cut) || o.cut_mode == hk::kCutFixed) return cut;
  if (o.cut_mode == hk::kCutDoppler) {
    const double af = std::sqrt(2.0 * kB * T / (L->sp.mass_amu * kAMU));
    return cut * std::sqrt(std::log(2.0)) * (L->numax / kC * af) * (1.0 + 1e-9);
  }
  const double tr = L->sp.T_ref / T;
  const double f = std::max(std::pow(tr, L->n_min), std::pow(tr, L->n_max));
  return cut * L->gref_max * f * (P / L->sp.P_ref_atm) * (1.0 + 1e-9);
}

hk_status make_plan(const hk_lines* L, int n_pairs, int n_temps_bound, const double* T, const double* P,
                    const hk_grid* grids, const int64_t* out_off, double cut_arg, const DevInfo& di, Tuning tu,
                    const Opts& opts, Plan* pl) {
  pl->slots = tu.slots;
  pl->opts = opts;
  const bool dflt = opts.default_path();
  // window half-width: the cutting length, or the largest per-line one over the pairs
  double cut = cut_arg;
  if (!dflt && opts.cut_mode != hk::kCutFixed && !std::isinf(cut_arg)) {
    if (!T || !P) return fail(HK_EINVAL, "a width-multiple cutting length needs T and P");
    cut = 0.0;
    for (int p = 0; p < n_pairs; ++p) cut = std::max(cut, max_cut_length(L, opts, cut_arg, T[p], P[p]));
    if (!(cut > 0.0)) cut = 1e-300;  // every line's cut is empty but its centre point (gamma = 0)
  }
  if (!dflt && (opts.profile == hk::kProfDoppler || opts.profile == hk::kProfBinned) && T) {
    // a Gaussian line reaches no further than 9 alpha (+ a bin) above e^-81 of its peak: the
    // window need not (k_direct evaluates only those points)
    double reach = 0.0;
    for (int p = 0; p < n_pairs; ++p) {
      const double a = std::sqrt(2.0 * kB * T[p] / (L->sp.mass_amu * kAMU)) / kC * std::fabs(L->numax);
      reach = std::max(reach, (9.0 * a + 2.0 * grids[p].dnu) * (1.0 + 1e-6));
    }
    cut = std::min(cut, reach);
  }
  pl->cut_w = cut;
  if (L->shift_max > 0.0 && T) {
    double bmax = 0.0;
    for (int p = 0; p < n_pairs; ++p) bmax = std::max(bmax, std::sqrt(2.0 * kB * T[p] / (L->sp.mass_amu * kAMU)) / kC);
    pl->core_pad = core_threshold(dflt) * bmax * L->shift_max * 1.001;
  }
  pl->W = hk::kWavesPerWG * hk::kWave * pl->slots;
  pl->n_pairs = n_pairs;
  const int64_t N = L->N;
  // distinct temperatures
  pl->temps.clear();
  std::vector<int> tidx(n_pairs, 0);
  if (T) {
    for (int p = 0; p < n_pairs; ++p) {
      int found = -1;
      for (size_t t = 0; t < pl->temps.size(); ++t)
        if (pl->temps[t] == T[p]) { found = (int)t; break; }
      if (found < 0) { found = (int)pl->temps.size(); pl->temps.push_back(T[p]); }
      tidx[p] = found;
    }
    pl->n_temps = (int)pl->temps.size();
  } else {
    pl->n_temps = n_temps_bound;
  }
  // distinct grids (pairs with equal grids share one grid-record array)
  pl->grids.clear();
  std::vector<int> gidx(n_pairs, 0);
  for (int p = 0; p < n_pairs; ++p) {
    int found = -1;
    for (size_t q = 0; q < pl->grids.size() && dflt; ++q)  // options: one record array per pair
      if (pl->grids[q].nu_start == grids[p].nu_start && pl->grids[q].dnu == grids[p].dnu &&
          pl->grids[q].n == grids[p].n) { found = (int)q; break; }
    if (found < 0) { found = (int)pl->grids.size(); pl->grids.push_back(grids[p]); }
    gidx[p] = found;
  }
  pl->n_grids = (int)pl->grids.size();
  // tiles, spans and the bounds on line visits (tile windows, span windows, and the narrower
  // windows of the core pass)
  int64_t tiles = 0, tiles_c = 0;
  double visits = 0.0, visits_w = 0.0, visits_c = 0.0;
  // the wing pass visits a line on the spans within the tile-far bound (1.5 tile widths of the
  // tile centre) and on the two spans of its cut bounds only: at most this many spans per line
  const int64_t wing_span_visits = 2 * (int64_t)(hk::kTileFar * hk::kWavesPerWG + hk::kWavesPerWG) + 4;
  double visits_wing = 0.0;
  pl->W_c = hk::kWave * pl->slots;
  pl->pairs.assign(n_pairs, hk::PairDesc{});
  pl->pairs_c.assign(n_pairs, hk::PairDesc{});
  for (int p = 0; p < n_pairs; ++p) {
    const int64_t nt = (grids[p].n + pl->W - 1) / pl->W;
    if (tiles + nt >= (int64_t(1) << 30)) return fail(HK_ENOMEM, "too many grid tiles");
    hk::PairDesc& d = pl->pairs[p];
    d.nu_start = grids[p].nu_start;
    d.dnu = grids[p].dnu;
    d.n = grids[p].n;
    d.out_off = out_off ? out_off[p] : 0;
    d.pfac = P ? P[p] / L->sp.P_ref_atm : 1.0;
    d.beta = T ? std::sqrt(2.0 * kB * T[p] / (L->sp.mass_amu * kAMU)) / kC : 0.0;
    d.tidx = tidx[p];
    d.gidx = gidx[p];
    d.tile_base = (int32_t)tiles;
    d.n_tiles = (int32_t)nt;
    tiles += nt;
    visits += (double)N * (double)visits_per_line(L, grids[p], cut, pl->W, nt);
    const double gend = std::max(std::fabs(grids[p].nu_start),
                                 std::fabs(grids[p].nu_start + (double)grids[p].n * grids[p].dnu));
    const double vmax = std::min(L->numax, gend + (std::isinf(cut) ? L->numax : cut));
    const double hc = std::min(cut, core_threshold(dflt) * d.beta * vmax * 1.0001 + 0.01 * grids[p].dnu);
    const int64_t nt_c = (grids[p].n + pl->W_c - 1) / pl->W_c;
    if (tiles_c + nt_c >= (int64_t(1) << 30)) return fail(HK_ENOMEM, "too many grid tiles");
    hk::PairDesc& dc = pl->pairs_c[p];
    dc = d;
    dc.tile_base = (int32_t)tiles_c;
    dc.n_tiles = (int32_t)nt_c;
    tiles_c += nt_c;
    const int64_t vw = visits_per_line(L, grids[p], cut, pl->W_c, nt_c);
    visits_w += (double)N * (double)vw;
    visits_wing += (double)N * (double)std::min<int64_t>(vw, wing_span_visits);
    visits_c += (double)N * (double)visits_per_line(L, grids[p], T ? hc : cut, pl->W_c, nt_c);
  }
  pl->n_tiles_total = (int)tiles;
  pl->n_tiles_c = (int)tiles_c;
  // work-item sizes: enough items to balance the persistent grids (measured on the large list:
  // the wing pass gains down to about 64 items per wave slot, the core pass loses below about 1)
  const int wgs_w = di.cus * di.wing_per_cu[slot_index(pl->slots)];
  const int wgs_c = di.cus * di.core_per_cu[slot_index(pl->slots)];
  double c = std::ceil(visits_wing / (64.0 * (wgs_w > 0 ? wgs_w : 4096)));
  const int env_chunk = env_int("HK_CHUNK", 0);
  if (env_chunk > 0) c = env_chunk;
  if (c < 256) c = 256;
  if (c > (1 << 22)) c = 1 << 22;
  pl->chunk = (int)(std::ceil(c / hk::kWave) * hk::kWave);
  const double items_w = (double)tiles_c + std::ceil(visits_w / pl->chunk);
  if (items_w >= 2.0e9) return fail(HK_ENOMEM, "work list too large (%.3g items)", items_w);
  pl->items_bound_w = (int64_t)items_w;
  double cc = std::ceil(visits_c / (double)(wgs_c > 0 ? wgs_c : 4096));
  if (cc < 4096) cc = 4096;
  if (cc > (1 << 22)) cc = 1 << 22;
  pl->chunk_c = (int)(std::ceil(cc / hk::kWave) * hk::kWave);
  const double items_c = (double)tiles_c + std::ceil(visits_c / pl->chunk_c);
  if (items_c >= 2.0e9) return fail(HK_ENOMEM, "core work list too large (%.3g items)", items_c);
  pl->items_bound_c = (int64_t)items_c;
  // tile-far items: large chunks (a line costs kNodes evaluations), still enough to balance
  const int wgs_f = di.cus * di.far_per_cu;
  double cf = std::ceil(visits / (16.0 * (wgs_f > 0 ? wgs_f : 1024)));
  if (cf < 4096) cf = 4096;
  if (cf > (1 << 22)) cf = 1 << 22;
  pl->chunk_f = (int)(std::ceil(cf / hk::kThreads) * hk::kThreads);
  const double items_f = (double)tiles + std::ceil(visits / pl->chunk_f);
  if (items_f >= 2.0e9) return fail(HK_ENOMEM, "tile-far work list too large (%.3g items)", items_f);
  pl->items_bound_f = (int64_t)items_f;
  pl->grid_w = (int)std::max<int64_t>(1, std::min<int64_t>(pl->items_bound_w, (int64_t)(wgs_w > 0 ? wgs_w : 4096)));
  pl->grid_f = (int)std::max<int64_t>(1, std::min<int64_t>(pl->items_bound_f, (int64_t)(wgs_f > 0 ? wgs_f : 1024)));
  pl->grid_c = (int)std::max<int64_t>(1, std::min<int64_t>(pl->items_bound_c, (int64_t)(wgs_c > 0 ? wgs_c : 4096)));
  // the options path's direct pass: every line of a span's window, one evaluation per point
  if (!dflt) {
    const int wgs_d = di.cus * di.direct_per_cu[slot_index(pl->slots)];
    double cd = std::ceil(visits_w / (16.0 * (wgs_d > 0 ? wgs_d : 4096)));
    if (env_chunk > 0) cd = env_chunk;
    if (cd < 256) cd = 256;
    if (cd > (1 << 22)) cd = 1 << 22;
    pl->chunk_d = (int)(std::ceil(cd / hk::kWave) * hk::kWave);
    const double items_d = (double)tiles_c + std::ceil(visits_w / pl->chunk_d);
    if (items_d >= 2.0e9) return fail(HK_ENOMEM, "direct work list too large (%.3g items)", items_d);
    pl->items_bound_d = (int64_t)items_d;
    pl->grid_d = (int)std::max<int64_t>(1, std::min<int64_t>(pl->items_bound_d, (int64_t)(wgs_d > 0 ? wgs_d : 4096)));
  } else {
    pl->chunk_d = 0;
    pl->items_bound_d = 0;
    pl->grid_d = 0;
  }
  // workspace layout (256-byte aligned sections); the options path leaves out the wing and
  // tile-far sections, the default path the direct pass's
  const size_t tw = dflt ? (size_t)tiles : 0, tcw = dflt ? (size_t)tiles_c : 0, tcd = dflt ? 0 : (size_t)tiles_c;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes, 256); return o; };
  pl->off_S = take(sizeof(float) * (size_t)N * pl->n_temps);
  pl->off_g = take(sizeof(float) * (size_t)N * pl->n_temps);
  pl->off_gr = take(sizeof(int4) * (size_t)N * pl->n_grids);
  pl->off_plin = take(dflt ? 0 : sizeof(float) * (size_t)N * pl->n_grids);
  pl->off_pairs = take(sizeof(hk::PairDesc) * n_pairs);
  pl->off_pairs_c = take(sizeof(hk::PairDesc) * n_pairs);
  pl->off_cnt = take(sizeof(int) * 64);
  pl->off_stats = take(sizeof(long long) * (5 * (size_t)pl->grid_w + pl->grid_c + 2 * (size_t)pl->grid_f +
                                            (size_t)pl->grid_d));
  pl->off_lo = take(sizeof(int32_t) * tw);
  pl->off_hi = take(sizeof(int32_t) * tw);
  pl->off_nc = take(sizeof(int32_t) * tw);
  pl->off_far = take(sizeof(int4) * 2 * tw);
  pl->off_nf = take(sizeof(int32_t) * 2 * tw);
  pl->off_ibf = take(sizeof(int32_t) * 2 * (tw + 1));
  pl->off_partf = take(dflt ? sizeof(double) * (hk::kNodes + hk::kFar8Nodes) * (size_t)pl->items_bound_f : 0);
  pl->off_segs = take(sizeof(hk::SpanSeg) * tcw);
  pl->off_nc_w = take(sizeof(int32_t) * tcw);
  pl->off_ib_w = take(sizeof(int32_t) * (tcw + 1));
  pl->off_part_w = take(dflt ? sizeof(float) * (size_t)pl->items_bound_w * pl->W_c : 0);
  pl->off_lo_d = take(sizeof(int32_t) * tcd);
  pl->off_hi_d = take(sizeof(int32_t) * tcd);
  pl->off_nc_d = take(sizeof(int32_t) * tcd);
  pl->off_ib_d = take(sizeof(int32_t) * (tcd + 1));
  pl->off_part_d = take(sizeof(float) * (size_t)pl->items_bound_d * pl->W_c);
  pl->off_lo_c = take(sizeof(int32_t) * tiles_c);
  pl->off_hi_c = take(sizeof(int32_t) * tiles_c);
  pl->off_nc_c = take(sizeof(int32_t) * tiles_c);
  pl->off_ib_c = take(sizeof(int32_t) * (tiles_c + 1));
  pl->off_part_c = take(sizeof(float) * (size_t)pl->items_bound_c * pl->W_c);
  pl->total = off;
  return HK_OK;
}

// Backward workspace: grid records, per-line (dL/dT, dL/dlnP) terms, reduction partials,
// per-line FP64 records and the node weights of dL/dk per span of the grid.
constexpr int kBwdPartials = 256;
struct BwdLayout {
  size_t off_gr = 0, off_contrib = 0, off_part = 0, off_lrec = 0, off_lzone = 0, off_pref[hk::kAdjLevels] = {},
         off_stats = 0, total = 0;
};
constexpr int64_t kAdjMaxWaves = 1 << 16;  // bound of the adjoint's waves (its grid is capped below)
BwdLayout backward_layout(int64_t N, int64_t n_grid) {
  BwdLayout b;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes, 256); return o; };
  b.off_gr = take(sizeof(int4) * (size_t)N);
  b.off_stats = take(sizeof(long long) * kAdjMaxWaves);
  b.off_contrib = take(2 * sizeof(double) * (size_t)N);
  b.off_part = take(2 * sizeof(double) * kBwdPartials);
  b.off_lrec = take(8 * sizeof(double) * (size_t)N);
  b.off_lzone = take(16 * sizeof(int) * (size_t)N);
  for (int lv = 0; lv < hk::kAdjLevels; ++lv) {
    const size_t W = (size_t)hk::kAdjSpan << (2 * lv);
    const size_t units = ((size_t)n_grid + W - 1) / W;
    b.off_pref[lv] = take(sizeof(double) * hk::kNodes * W * units);
  }
  b.total = off;
  return b;
}

hk::PrepArgs prep_args(const hk_lines* L, const hk_line_override* ovr, double T) {
  hk::PrepArgs a;
  a.nu = L->nu;
  a.Sref = L->Sref;
  a.E = L->E;
  a.gref = L->gref;
  a.nexp = L->nexp;
  a.perm = L->perm;
  a.ovr_S = ovr ? ovr->S_ref : nullptr;
  a.ovr_g = ovr ? ovr->gamma_ref : nullptr;
  a.ovr_n = ovr ? ovr->n_exp : nullptr;
  a.N = L->N;
  a.c2_over_T = kC2 / T;
  a.c2_over_Tref = kC2 / L->sp.T_ref;
  a.c2E_coef = kC2 * (1.0 / L->sp.T_ref - 1.0 / T);
  a.q_ratio = std::pow(L->sp.T_ref / T, L->sp.q_b);
  a.log_tr = std::log(L->sp.T_ref / T);
  a.beta = std::sqrt(2.0 * kB * T / (L->sp.mass_amu * kAMU)) / kC;
  a.pfac = 1.0;
  return a;
}

struct Timer {
  bool on;
  hipStream_t st;
  std::vector<hipEvent_t> ev;
  explicit Timer(hipStream_t s) : on(env_flag("HK_TIMING", false)), st(s) {}
  void mark() {
    if (!on) return;
    hipEvent_t e;
    if (hipEventCreate(&e) == hipSuccess) { hipEventRecord(e, st); ev.push_back(e); }
  }
  double ms(size_t i) {
    if (!on || i + 1 >= ev.size()) return -1.0;
    float t = 0;
    hipEventElapsedTime(&t, ev[i], ev[i + 1]);
    return t;
  }
  void finish() {
    if (on && !ev.empty()) hipEventSynchronize(ev.back());
  }
  ~Timer() {
    for (auto e : ev) hipEventDestroy(e);
  }
};

// GridRecArgs of pair p of a plan (per-line cutting lengths and plinth values).
hk::GridRecArgs gridrec_args(const hk_lines* L, const hk_line_override* ovr, const Plan& pl, int p, double T,
                             double P_atm, const hk_grid& g, double cut, const float* S_T, int4* grec, float* plin) {
  hk::GridRecArgs ga;
  memset(&ga, 0, sizeof ga);
  ga.pa = prep_args(L, ovr, T);
  ga.pa.pfac = P_atm / L->sp.P_ref_atm;
  ga.S_T = S_T;
  ga.nu_start = g.nu_start;
  ga.dnu = g.dnu;
  ga.n = g.n;
  ga.cut = cut;
  ga.cut_dop = cut * std::sqrt(std::log(2.0));
  ga.c_light = kC;
  ga.alpha_fac = std::sqrt(2.0 * kB * T / (L->sp.mass_amu * kAMU));
  ga.t_ratio = L->sp.T_ref / T;
  ga.cut_mode = pl.opts.cut_mode;
  ga.profile = pl.opts.profile;
  ga.plinth = pl.opts.plinth;
  ga.grec = grec;
  ga.plin = plin;
  ga.nu_pos = L->nu_pos;
  (void)p;
  return ga;
}

hk_status run_forward(const hk_lines* L, const hk_line_override* ovr, const Plan& pl, const double* T,
                      const double* P, double cut, float* k, char* ws, hipStream_t st, bool timed = true) {
  Timer tm(st);
  tm.on = tm.on && timed;
  const bool dflt = pl.opts.default_path();
  tm.mark();
  float* S_T = reinterpret_cast<float*>(ws + pl.off_S);
  float* gT = reinterpret_cast<float*>(ws + pl.off_g);
  for (int t = 0; t < pl.n_temps; ++t) {
    hk::PrepArgs a = prep_args(L, ovr, pl.temps[t]);
    HK_HIP(hk::launch_prep(a, S_T + (size_t)t * L->N, gT + (size_t)t * L->N, nullptr, nullptr, nullptr, st));
  }
  int4* grec = reinterpret_cast<int4*>(ws + pl.off_gr);
  float* plin = dflt ? nullptr : reinterpret_cast<float*>(ws + pl.off_plin);
  if (dflt) {
    for (int q = 0; q < pl.n_grids; ++q)
      HK_HIP(hk::launch_gridrec(L->nu, L->N, pl.grids[q].nu_start, pl.grids[q].dnu, pl.grids[q].n, cut,
                                grec + (size_t)q * L->N, st));
  } else {
    for (int p = 0; p < pl.n_pairs; ++p) {
      const hk::GridRecArgs ga = gridrec_args(L, ovr, pl, p, T[p], P[p], pl.grids[p], cut,
                                              S_T + (size_t)pl.pairs_c[p].tidx * L->N, grec + (size_t)p * L->N,
                                              plin + (size_t)p * L->N);
      HK_HIP(hk::launch_gridrec_ex(ga, st));
    }
  }
  tm.mark();
  // work lists: tile windows and tile-far ranges, span segments, span core windows
  // lines evaluated at nodes must keep the interval outside their core (|z| >= the last threshold)
  const double far_z = kZK[hk::kKmax - 1], core_z = core_threshold(dflt);
  const double cut_w = pl.cut_w;
  hk::PairDesc* dpairs = reinterpret_cast<hk::PairDesc*>(ws + pl.off_pairs);
  hk::PairDesc* dpairs_c = reinterpret_cast<hk::PairDesc*>(ws + pl.off_pairs_c);
  // dispensers: wing [0], core [8], tile-far [16] and [24], direct [32]; status word [48]
  int* cnt = reinterpret_cast<int*>(ws + pl.off_cnt);
  int* status = cnt + 48;
  int32_t* lo = reinterpret_cast<int32_t*>(ws + pl.off_lo);
  int32_t* hi = reinterpret_cast<int32_t*>(ws + pl.off_hi);
  int32_t* nc = reinterpret_cast<int32_t*>(ws + pl.off_nc);
  int4* tfar = reinterpret_cast<int4*>(ws + pl.off_far);
  int32_t* nf = reinterpret_cast<int32_t*>(ws + pl.off_nf);
  int32_t* ibf = reinterpret_cast<int32_t*>(ws + pl.off_ibf);
  hk::SpanSeg* segs = reinterpret_cast<hk::SpanSeg*>(ws + pl.off_segs);
  int32_t* nc_w = reinterpret_cast<int32_t*>(ws + pl.off_nc_w);
  int32_t* ib_w = reinterpret_cast<int32_t*>(ws + pl.off_ib_w);
  int32_t* lo_c = reinterpret_cast<int32_t*>(ws + pl.off_lo_c);
  int32_t* hi_c = reinterpret_cast<int32_t*>(ws + pl.off_hi_c);
  int32_t* nc_c = reinterpret_cast<int32_t*>(ws + pl.off_nc_c);
  int32_t* ib_c = reinterpret_cast<int32_t*>(ws + pl.off_ib_c);
  int32_t* lo_d = reinterpret_cast<int32_t*>(ws + pl.off_lo_d);
  int32_t* hi_d = reinterpret_cast<int32_t*>(ws + pl.off_hi_d);
  int32_t* nc_d = reinterpret_cast<int32_t*>(ws + pl.off_nc_d);
  int32_t* ib_d = reinterpret_cast<int32_t*>(ws + pl.off_ib_d);
  HK_HIP(hk::launch_fill_pairs(pl.pairs.data(), pl.n_pairs, dpairs, status, st));
  HK_HIP(hk::launch_fill_pairs(pl.pairs_c.data(), pl.n_pairs, dpairs_c, nullptr, st));
  const int direct_only = pl.opts.direct ? 1 : 0;
  if (dflt) {
    HK_HIP(hk::launch_worklist(L->keys, L->N, L->km, L->numin, L->numax, dpairs, pl.n_pairs, pl.n_tiles_total,
                               pl.W, cut, 0.0, pl.chunk, lo, hi, nc, tfar, nf, pl.chunk_f, far_z, direct_only, 0.0,
                               st));
    HK_HIP(hk::launch_item_scan(nf, pl.n_tiles_total, ibf, cnt + 16, st));
    HK_HIP(hk::launch_item_scan(nf + pl.n_tiles_total, pl.n_tiles_total, ibf + pl.n_tiles_total + 1, cnt + 24, st));
    HK_HIP(hk::launch_span_segments(L->keys, L->N, L->km, L->numin, L->numax, dpairs_c, dpairs, pl.n_pairs,
                                    pl.n_tiles_c, pl.W_c, cut, far_z, tfar, pl.chunk, segs, nc_w, direct_only, st));
    HK_HIP(hk::launch_item_scan(nc_w, pl.n_tiles_c, ib_w, cnt, st));
  } else {
    HK_HIP(hk::launch_worklist(L->keys, L->N, L->km, L->numin, L->numax, dpairs_c, pl.n_pairs, pl.n_tiles_c,
                               pl.W_c, cut_w, 0.0, pl.chunk_d, lo_d, hi_d, nc_d, nullptr, nullptr, 1, 0.0, 0, 0.0,
                               st));
    HK_HIP(hk::launch_item_scan(nc_d, pl.n_tiles_c, ib_d, cnt + 32, st));
  }
  const bool core_pass = pl.opts.profile == hk::kProfVoigt;
  if (core_pass) {
    HK_HIP(hk::launch_worklist(L->keys, L->N, L->km, L->numin, L->numax, dpairs_c, pl.n_pairs, pl.n_tiles_c,
                               pl.W_c, cut_w, core_z, pl.chunk_c, lo_c, hi_c, nc_c, nullptr, nullptr, 1, 0.0, 0,
                               pl.core_pad, st));
    HK_HIP(hk::launch_item_scan(nc_c, pl.n_tiles_c, ib_c, cnt + 8, st));
  }
  tm.mark();
  int dev = 0;
  DevInfo di;
  hk_status ds = device_init(&dev, &di);
  if (ds != HK_OK) return ds;
  const int si = slot_index(pl.slots);
  // evaluation counts (timed calls only): per workgroup of the wing (5 classes), core, tile-far
  // (2 classes) and direct kernels
  long long* stats = reinterpret_cast<long long*>(ws + pl.off_stats);
  long long* stats_c = stats + 5 * (size_t)pl.grid_w;
  long long* stats_f = stats_c + pl.grid_c;
  long long* stats_d = stats_f + 2 * (size_t)pl.grid_f;
  hk::VoigtArgs va;
  memset(&va, 0, sizeof va);
  va.nu = L->nu;
  va.S_T = S_T;
  va.gT = gT;
  va.grec = grec;
  va.pairs = dpairs_c;
  va.k = k;
  va.N = L->N;
  va.cut = cut_w;
  for (int i = 0; i < hk::kKmax; ++i) va.zK[i] = (float)kZK[i];
  for (int i = 0; i < hk::kKw; ++i) va.zw[i] = (float)kZW[i];
  va.zcore = (float)core_z;
  va.n_pairs = pl.n_pairs;
  va.n_tiles_total = pl.n_tiles_c;
  va.status = status;
  va.nu_pos = L->nu_pos;
  const int64_t icap = env_int("HK_DEBUG_ITEMS_CAP", 0);  // tests of the overflow flag only
  auto cap = [&](int64_t bound) { return (int32_t)std::min<int64_t>(icap > 0 ? icap : bound, INT32_MAX); };
  if (dflt) {
    // wing pass over spans
    va.segs = segs;
    va.tile_nc = nc_w;
    va.item_base = ib_w;
    va.partial = reinterpret_cast<float*>(ws + pl.off_part_w);
    va.counter = cnt;
    va.stats = tm.on ? stats : nullptr;
    va.chunk = pl.chunk;
    va.items_cap = cap(pl.items_bound_w);
    va.cheb_w = di.cheb_w[si];
    va.mid_w = di.mid_w[si];
    va.far8_w = di.far8_w[si];
    va.mask_w = di.mask_w[si];
    HK_HIP(hk::launch_wing(va, pl.slots, pl.grid_w, st));
    tm.mark();
    HK_HIP(hk::launch_combine(va, pl.slots, false, st));
    tm.mark();
    // tile-far pass
    hk::FarArgs fa;
    memset(&fa, 0, sizeof fa);
    fa.nu = L->nu;
    fa.S_T = S_T;
    fa.gT = gT;
    fa.pairs = dpairs;
    fa.tile_far = tfar;
    fa.item_base[0] = ibf;
    fa.item_base[1] = ibf + pl.n_tiles_total + 1;
    fa.node_part[0] = reinterpret_cast<double*>(ws + pl.off_partf);
    fa.node_part[1] = fa.node_part[0] + (size_t)hk::kNodes * pl.items_bound_f;
    fa.counter[0] = cnt + 16;
    fa.counter[1] = cnt + 24;
    fa.stats = tm.on ? stats_f : nullptr;
    fa.tile_w[0] = di.tile_w[si];
    fa.tile_w[1] = di.tile_w8[si];
    fa.k = k;
    fa.N = L->N;
    for (int i = 0; i < hk::kKmax; ++i) fa.zK[i] = (float)kZK[i];
    fa.n_pairs = pl.n_pairs;
    fa.n_tiles_total = pl.n_tiles_total;
    fa.chunk = pl.chunk_f;
    fa.items_cap[0] = fa.items_cap[1] = cap(pl.items_bound_f);
    fa.W = pl.W;
    for (int q = 0; q < hk::kNodes; ++q) fa.tile_x[q] = di.tile_x[si][q];
    for (int q = 0; q < hk::kFar8Nodes; ++q) fa.tile_x8[q] = di.tile_x8[si][q];
    fa.status = status;
    HK_HIP(hk::launch_far(fa, 0, pl.grid_f, st));
    HK_HIP(hk::launch_far(fa, 1, pl.grid_f, st));
    HK_HIP(hk::launch_combine_far(fa, st));
    tm.mark();
  } else {
    // direct pass over spans (every profile; Voigt core points excepted)
    va.tile_lo = lo_d;
    va.tile_hi = hi_d;
    va.tile_nc = nc_d;
    va.item_base = ib_d;
    va.partial = reinterpret_cast<float*>(ws + pl.off_part_d);
    va.counter = cnt + 32;
    va.stats = tm.on ? stats_d : nullptr;
    va.chunk = pl.chunk_d;
    va.items_cap = cap(pl.items_bound_d);
    HK_HIP(hk::launch_direct(va, plin, pl.opts.profile, pl.slots, pl.grid_d, st));
    tm.mark();
    HK_HIP(hk::launch_combine(va, pl.slots, false, st));
    tm.mark();
    tm.mark();
  }
  // line-core pass over its own (narrower) work list, after the other sums are final
  hk::VoigtArgs vc = va;
  if (core_pass) {
    vc.chunk = pl.chunk_c;
    vc.segs = nullptr;
    vc.tile_lo = lo_c;
    vc.tile_hi = hi_c;
    vc.tile_nc = nc_c;
    vc.item_base = ib_c;
    vc.counter = cnt + 8;
    vc.partial = reinterpret_cast<float*>(ws + pl.off_part_c);
    vc.items_cap = cap(pl.items_bound_c);
    vc.stats = tm.on ? stats_c : nullptr;
    HK_HIP(hk::launch_core(vc, pl.slots, pl.grid_c, st));
    HK_HIP(hk::launch_combine(vc, pl.slots, true, st));
  }
  tm.mark();
  tm.finish();
  g_tim.prep_ms = tm.ms(0);
  g_tim.worklist_ms = tm.ms(1);
  g_tim.voigt_ms = tm.ms(2);
  g_tim.combine_ms = tm.ms(3);
  g_tim.far_ms = tm.ms(4);
  g_tim.core_ms = tm.ms(5);
  g_tim.backward_ms = -1;
  g_tim.core_evals = -1;
  g_tim.wing_evals = -1;
  for (int c = 0; c < 8; ++c) g_tim.class_evals[c] = -1;
  g_tim.status = 0;
  if (tm.on) {
    const size_t nw = 5 * (size_t)pl.grid_w, ncr = pl.grid_c, nfar = 2 * (size_t)pl.grid_f, nd = pl.grid_d;
    std::vector<long long> h(nw + ncr + nfar + nd);
    HK_HIP(hipMemcpy(h.data(), stats, sizeof(long long) * h.size(), hipMemcpyDeviceToHost));
    int hstatus = 0;
    HK_HIP(hipMemcpy(&hstatus, status, sizeof(int), hipMemcpyDeviceToHost));
    long long cls[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (dflt) {
      for (size_t i = 0; i < nw; ++i) cls[i / pl.grid_w] += h[i];
      for (size_t i = 0; i < nfar; ++i) cls[5 + i / pl.grid_f] += h[nw + ncr + i];
    } else {
      for (size_t i = 0; i < nd; ++i) cls[0] += h[nw + ncr + nfar + i];
    }
    if (core_pass)
      for (size_t i = 0; i < ncr; ++i) cls[7] += h[nw + i];
    long long tw = 0;
    for (int c = 0; c < 7; ++c) tw += cls[c];
    for (int c = 0; c < 8; ++c) g_tim.class_evals[c] = cls[c];
    g_tim.core_evals = cls[7];
    g_tim.wing_evals = tw;
    g_tim.status = hstatus;
    if (hstatus != 0)
      return fail(HK_EDEVICE, "a work item fell beyond the workspace's partial rows (status %d); k holds NaN there",
                  hstatus);
  }
  g_tim.tile_width = pl.W_c;
  g_tim.lines_per_batch = hk::kWave;
  g_tim.chunk_lines = dflt ? pl.chunk : pl.chunk_d;
  g_tim.n_items = (int32_t)(dflt ? pl.items_bound_w : pl.items_bound_d);
  return HK_OK;
}

// Records the completion of the work just issued through L on stream st (see hk_lines::use_*).
// may_create: an event may be created for a stream not seen before.
void note_use(hk_lines* L, hipStream_t st, bool may_create) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  std::lock_guard<std::mutex> lk(L->use_mu);
  if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
    (void)hipGetLastError();
    L->untracked = true;
    return;
  }
  int slot = -1;
  for (int i = 0; i < L->n_use; ++i)
    if (L->use_stream[i] == st) { slot = i; break; }
  if (slot < 0) {
    hipEvent_t e = nullptr;
    if (!may_create || L->n_use >= hk_lines::kUseSlots || hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      L->untracked = true;
      return;
    }
    slot = L->n_use++;
    L->use_stream[slot] = st;
    L->use_event[slot] = e;
  }
  if (hipEventRecord(L->use_event[slot], st) != hipSuccess) {
    (void)hipGetLastError();
    L->untracked = true;
  }
}

hk_status check_lines(const hk_lines* L) {
  if (!L) return fail(HK_EINVAL, "lines handle is NULL");
  int dev = -1;
  HK_HIP(hipGetDevice(&dev));
  if (dev != L->device) return fail(HK_EINVAL, "current device %d differs from the handle's device %d", dev, L->device);
  return HK_OK;
}

// Tuning for a call: forced by the environment, else the cached autotuner choice for this
// key, else (HK_AUTOTUNE=1) timed now over the candidates on the caller's data, else default.
// Autotuning runs the forward path once per candidate on `stream` and synchronizes.
std::mutex g_tune_mu;
std::map<std::string, Tuning> g_tune;

std::string tune_key(const hk_lines* L, int n_pairs, const double* T, const hk_grid* grids, double cut,
                     const Opts& o) {
  std::string key;
  auto put = [&](const void* p, size_t n) { key.append(static_cast<const char*>(p), n); };
  put(&L->N, sizeof L->N);
  put(&L->device, sizeof L->device);
  put(&n_pairs, sizeof n_pairs);
  put(&cut, sizeof cut);
  int64_t pts = 0;
  for (int p = 0; p < n_pairs; ++p) pts += grids[p].n;
  put(&pts, sizeof pts);
  put(&grids[0].dnu, sizeof(double));
  const int ov[4] = {o.profile, o.cut_mode, o.plinth, o.direct};
  put(ov, sizeof ov);
  (void)T;  // the choice depends on the list, the grids, the cut and the options, not on the exact (T, P)
  return key;
}

hk_status choose_tuning(const hk_lines* L, const hk_line_override* ovr, int n_pairs, const double* T,
                        const double* P, const hk_grid* grids, const int64_t* out_off, double cut, const Opts& o,
                        float* k, char* ws, size_t ws_bytes, hipStream_t st, const DevInfo& di, Tuning* out) {
  if (env_tuning(out)) return HK_OK;
  const std::string key = tune_key(L, n_pairs, T, grids, cut, o);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) { *out = it->second; return HK_OK; }
  }
  *out = Tuning{};
  if (!env_flag("HK_AUTOTUNE", false)) return HK_OK;
  float best_ms = 0.0f, default_ms = -1.0f;
  bool have = false;
  hipEvent_t e0, e1;
  HK_HIP(hipEventCreate(&e0));
  HK_HIP(hipEventCreate(&e1));
  for (const Tuning& tu : kCandidates) {
    Plan pl;
    hk_status s = make_plan(L, n_pairs, n_pairs, T, P, grids, out_off, cut, di, tu, o, &pl);
    if (s != HK_OK || pl.total > ws_bytes) continue;
    HK_HIP(hipEventRecord(e0, st));
    s = run_forward(L, ovr, pl, T, P, cut, k, ws, st, false);
    if (s != HK_OK) return s;
    HK_HIP(hipEventRecord(e1, st));
    HK_HIP(hipEventSynchronize(e1));
    float ms = 0.0f;
    HK_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (tu.slots == Tuning{}.slots) default_ms = ms;
    if (!have || ms < best_ms) { best_ms = ms; *out = tu; have = true; }
  }
  // keep the default unless another tuning is clearly faster (timing noise must not flip it)
  if (default_ms > 0.0f && default_ms <= 1.03f * best_ms) *out = Tuning{};
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[key] = *out;
  return HK_OK;
}

// The list's largest gamma_ref and range of n (bounds of Lorentz-multiple cutting lengths), read
// back once per handle on `st` (the call synchronizes that once).
hk_status ensure_line_stats(hk_lines* L, hipStream_t st) {
  std::lock_guard<std::mutex> lk(L->stats_mu);
  if (L->have_stats) return HK_OK;
  int dev;
  DevInfo di;
  hk_status s = device_init(&dev, &di);
  if (s != HK_OK) return s;
  std::lock_guard<std::mutex> lk2(g_stats_mu);  // one device buffer per device
  unsigned long long h[3] = {0, 0, 0};
  hipError_t e = hk::launch_line_stats(L->gref, L->nexp, L->N, di.stats_buf, st);
  if (e == hipSuccess) e = hipMemcpyAsync(h, di.stats_buf, sizeof h, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(HK_EDEVICE, "line statistics: %s", hipGetErrorString(e));
  double v[3];
  for (int i = 0; i < 3; ++i) v[i] = hk::ordered_to_double(h[i]);
  L->gref_max = v[0];
  L->n_min = v[1];
  L->n_max = v[2];
  L->have_stats = true;
  return HK_OK;
}

// Validation shared by the opacity entry points' options.
hk_status check_opts(hk_lines* L, const hk_line_override* ovr, const Opts& o, hipStream_t st) {
  if (o.direct && !o.default_path()) return fail(HK_EINVAL, "direct applies to the default path only");
  if (o.cut_mode == hk::kCutLorentz) {
    if (ovr && (ovr->gamma_ref || ovr->n_exp))
      return fail(HK_EUNSUPPORTED, "Lorentz-multiple cutting lengths with overridden widths are not supported");
    return ensure_line_stats(L, st);
  }
  return HK_OK;
}

hk_status opacity_impl(const hk_lines* lines, const hk_line_override* ovr, double T, double P_atm, hk_grid grid,
                       double cutoff, const hk_options* options, float* k, void* ws, size_t ws_bytes,
                       hipStream_t stream, bool scratch) {
  if (!(std::isfinite(T) && T > 0)) return fail(HK_EINVAL, "T must be finite and > 0");
  if (!(std::isfinite(P_atm) && P_atm >= 0)) return fail(HK_EINVAL, "P must be finite and >= 0");
  if (!grid_ok(grid)) return fail(HK_EINVAL, "invalid grid");
  if (!cut_ok(cutoff)) return fail(HK_EINVAL, "cutoff must be > 0 (or +inf)");
  if (!k) return fail(HK_EINVAL, "k is NULL");
  if (!scratch && !ws) return fail(HK_EINVAL, "workspace is NULL");
  if (!scratch && (reinterpret_cast<uintptr_t>(ws) & 255u) != 0)
    return fail(HK_EINVAL, "workspace must be 256-byte aligned");
  Opts o;
  hk_status s = opts_from(options, &o);
  if (s != HK_OK) return s;
  s = check_lines(lines);
  if (s != HK_OK) return s;
  int dev;
  DevInfo di;
  s = device_init(&dev, &di);
  if (s != HK_OK) return s;
  if (scratch) {
    ws = di.scratch;
    ws_bytes = hk::kScratchBytes;
  }
  s = check_opts(const_cast<hk_lines*>(lines), ovr, o, stream);
  if (s != HK_OK) return s;
  const int64_t zero = 0;
  Tuning tu;
  s = choose_tuning(lines, ovr, 1, &T, &P_atm, &grid, &zero, cutoff, o, k, static_cast<char*>(ws), ws_bytes, stream,
                    di, &tu);
  if (s != HK_OK) return s;
  Plan pl;
  s = make_plan(lines, 1, 1, &T, &P_atm, &grid, &zero, cutoff, di, tu, o, &pl);
  if (s != HK_OK) return s;
  if (ws_bytes < pl.total)
    return fail(scratch ? HK_ENOMEM : HK_EINVAL, "%s too small: %zu < %zu bytes",
                scratch ? "scratch array" : "workspace", ws_bytes, pl.total);
  return run_forward(lines, ovr, pl, &T, &P_atm, cutoff, k, static_cast<char*>(ws), stream);
}

hk_status batched_impl(const hk_lines* lines, int32_t n_pairs, const double* T, const double* P_atm,
                       const hk_grid* grids, const int64_t* out_offset, double cutoff, const hk_options* options,
                       float* k, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (n_pairs < 1) return fail(HK_EINVAL, "n_pairs must be >= 1");
  if (!T || !P_atm || !grids || !out_offset) return fail(HK_EINVAL, "NULL host array");
  if (!k || !ws) return fail(HK_EINVAL, "k or workspace is NULL");
  if ((reinterpret_cast<uintptr_t>(ws) & 255u) != 0) return fail(HK_EINVAL, "workspace must be 256-byte aligned");
  if (!cut_ok(cutoff)) return fail(HK_EINVAL, "cutoff must be > 0 (or +inf)");
  for (int p = 0; p < n_pairs; ++p) {
    if (!(std::isfinite(T[p]) && T[p] > 0)) return fail(HK_EINVAL, "T[%d] must be finite and > 0", p);
    if (!(std::isfinite(P_atm[p]) && P_atm[p] >= 0)) return fail(HK_EINVAL, "P[%d] must be finite and >= 0", p);
    if (!grid_ok(grids[p])) return fail(HK_EINVAL, "grid %d invalid", p);
    if (out_offset[p] < 0) return fail(HK_EINVAL, "out_offset[%d] < 0", p);
  }
  // output ranges must not overlap
  {
    std::vector<std::pair<int64_t, int64_t>> r(n_pairs);
    for (int p = 0; p < n_pairs; ++p) r[p] = {out_offset[p], out_offset[p] + grids[p].n};
    std::sort(r.begin(), r.end());
    for (int p = 1; p < n_pairs; ++p)
      if (r[p].first < r[p - 1].second) return fail(HK_EINVAL, "output ranges overlap");
  }
  Opts o;
  hk_status s = opts_from(options, &o);
  if (s != HK_OK) return s;
  s = check_lines(lines);
  if (s != HK_OK) return s;
  int dev;
  DevInfo di;
  s = device_init(&dev, &di);
  if (s != HK_OK) return s;
  s = check_opts(const_cast<hk_lines*>(lines), nullptr, o, stream);
  if (s != HK_OK) return s;
  Tuning tu;
  s = choose_tuning(lines, nullptr, n_pairs, T, P_atm, grids, out_offset, cutoff, o, k, static_cast<char*>(ws),
                    ws_bytes, stream, di, &tu);
  if (s != HK_OK) return s;
  Plan pl;
  s = make_plan(lines, n_pairs, n_pairs, T, P_atm, grids, out_offset, cutoff, di, tu, o, &pl);
  if (s != HK_OK) return s;
  if (ws_bytes < pl.total) return fail(HK_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, pl.total);
  if (!env_flag("HK_GRAPH", true))
    return run_forward(lines, nullptr, pl, T, P_atm, cutoff, k, static_cast<char*>(ws), stream);
  // graph key: every argument value and pointer, the options and the tuning
  std::string key;
  auto put = [&](const void* p, size_t n) { key.append(static_cast<const char*>(p), n); };
  const void* ptrs[3] = {lines, k, ws};
  put(ptrs, sizeof ptrs);
  put(&ws_bytes, sizeof ws_bytes);
  put(&cutoff, sizeof cutoff);
  put(&n_pairs, sizeof n_pairs);
  put(&pl.slots, sizeof pl.slots);
  put(&pl.chunk, sizeof pl.chunk);
  put(&pl.chunk_c, sizeof pl.chunk_c);
  const int ov[4] = {o.profile, o.cut_mode, o.plinth, o.direct};
  put(ov, sizeof ov);
  put(T, sizeof(double) * n_pairs);
  put(P_atm, sizeof(double) * n_pairs);
  put(grids, sizeof(hk_grid) * n_pairs);
  put(out_offset, sizeof(int64_t) * n_pairs);
  std::lock_guard<std::mutex> lk(g_graph_mu);
  auto it = g_graphs.find(key);
  if (it == g_graphs.end()) {
    hipStream_t cap;
    auto cs = g_capture_stream.find(dev);
    if (cs == g_capture_stream.end()) {
      HK_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
      g_capture_stream[dev] = cap;
    } else {
      cap = cs->second;
    }
    GraphEntry ge;
    HK_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    hk_status rs = run_forward(lines, nullptr, pl, T, P_atm, cutoff, k, static_cast<char*>(ws), cap, false);
    hipGraph_t graph = nullptr;
    hipError_t ec = hipStreamEndCapture(cap, &graph);
    if (rs != HK_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return rs;
    }
    if (ec != hipSuccess) return fail(HK_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(ec));
    ge.graph = graph;
    hipError_t ei = hipGraphInstantiate(&ge.exec, graph, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return fail(HK_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(ei));
    }
    it = g_graphs.emplace(key, ge).first;
  }
  Timer tm(stream);
  tm.mark();
  HK_HIP(hipGraphLaunch(it->second.exec, stream));
  tm.mark();
  tm.finish();
  g_tim.prep_ms = g_tim.worklist_ms = g_tim.combine_ms = -1;
  g_tim.voigt_ms = tm.ms(0);  // whole graph
  g_tim.core_ms = g_tim.far_ms = -1;
  g_tim.core_evals = g_tim.wing_evals = -1;
  for (int c = 0; c < 8; ++c) g_tim.class_evals[c] = -1;
  g_tim.status = 0;
  g_tim.tile_width = pl.W_c;
  g_tim.lines_per_batch = hk::kWave;
  g_tim.chunk_lines = o.default_path() ? pl.chunk : pl.chunk_d;
  g_tim.n_items = (int32_t)(o.default_path() ? pl.items_bound_w : pl.items_bound_d);
  if (tm.on) {
    int hstatus = 0;
    HK_HIP(hipMemcpy(&hstatus, static_cast<char*>(ws) + pl.off_cnt + 48 * sizeof(int), sizeof(int),
                     hipMemcpyDeviceToHost));
    g_tim.status = hstatus;
    if (hstatus != 0) return fail(HK_EDEVICE, "a work item fell beyond the workspace's partial rows (status %d)", hstatus);
  }
  return HK_OK;
}

hk_status workspace_impl(const hk_lines* lines, int mode, int32_t n_pairs, int32_t n_temps, const double* T,
                         const double* P, const hk_grid* grids, double cutoff, const hk_options* options,
                         hipStream_t st, size_t* bytes) {
  if (!bytes || !grids) return fail(HK_EINVAL, "NULL argument");
  if (mode < 0 || mode > 2) return fail(HK_EINVAL, "mode %d", mode);
  if (n_pairs < 1 || ((mode == 0 || mode == 2) && n_pairs != 1)) return fail(HK_EINVAL, "n_pairs %d", n_pairs);
  if (n_temps < 1 || n_temps > n_pairs) n_temps = n_pairs;
  if (!cut_ok(cutoff)) return fail(HK_EINVAL, "cutoff must be > 0 (or +inf)");
  for (int p = 0; p < n_pairs; ++p)
    if (!grid_ok(grids[p])) return fail(HK_EINVAL, "grid %d invalid", p);
  Opts o;
  hk_status s = opts_from(options, &o);
  if (s != HK_OK) return s;
  if (mode == 2 && (options && !(o.default_path() && !o.direct)))
    return fail(HK_EUNSUPPORTED, "the adjoint supports the default options only");
  s = check_lines(lines);
  if (s != HK_OK) return s;
  int dev;
  DevInfo di;
  s = device_init(&dev, &di);
  if (s != HK_OK) return s;
  if (mode == 2) {
    *bytes = backward_layout(lines->N, grids[0].n).total;
    return HK_OK;
  }
  if (!o.default_path() && o.cut_mode != hk::kCutFixed && !std::isinf(cutoff)) {
    if (!T || !P) return fail(HK_EINVAL, "a width-multiple cutting length needs T and P");
    for (int p = 0; p < n_pairs; ++p)
      if (!(std::isfinite(T[p]) && T[p] > 0) || !(std::isfinite(P[p]) && P[p] >= 0))
        return fail(HK_EINVAL, "T[%d] or P[%d] invalid", p, p);
    s = check_opts(const_cast<hk_lines*>(lines), nullptr, o, st);
    if (s != HK_OK) return s;
  }
  // enough for every tuning the autotuner may pick (T and P, when given, fix the distinct
  // temperatures and the width-multiple cutting lengths)
  const double* Tp = (T && P) ? T : nullptr;
  size_t best = 0;
  for (const Tuning& tu : kCandidates) {
    Plan pl;
    s = make_plan(lines, n_pairs, n_temps, Tp, Tp ? P : nullptr, grids, nullptr, cutoff, di, tu, o, &pl);
    if (s != HK_OK) return s;
    best = std::max(best, pl.total);
  }
  *bytes = best;
  return HK_OK;
}

// The view of a HITRAN-style list at one pressure: the list re-binned by its shifted centres, in
// the first `total` bytes of the caller's workspace.
struct ViewLayout {
  size_t o_nu = 0, o_pos = 0, o_S = 0, o_E = 0, o_g = 0, o_n = 0, o_perm = 0, o_kA = 0, o_vA = 0, o_kB = 0, o_vB = 0,
         o_hist = 0, o_dtot = 0, total = 0;
};
ViewLayout view_layout(int64_t N) {
  ViewLayout v;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes, 256); return o; };
  const size_t n = (size_t)N;
  const size_t G = (size_t)((N + hk::kSortBlock - 1) / hk::kSortBlock);
  v.o_nu = take(8 * n);
  v.o_pos = take(8 * n);
  v.o_S = take(8 * n);
  v.o_E = take(8 * n);
  v.o_g = take(8 * n);
  v.o_n = take(8 * n);
  v.o_perm = take(4 * n);
  v.o_kA = take(4 * n);
  v.o_vA = take(4 * n);
  v.o_kB = take(4 * n);
  v.o_vB = take(4 * n);
  v.o_hist = take(4 * 256 * G);
  v.o_dtot = take(4 * 256);
  v.total = off;
  return v;
}

// Host fields of the view V of L at pressure P (device arrays at ws; ws may be null for sizing).
void view_fields(const hk_lines* L, double P, char* ws, const ViewLayout& vl, hk_lines* V) {
  const double dP = L->dmax * (P / L->sp.P_ref_atm) * (1.0 + 1e-12);
  V->device = L->device;
  V->N = L->N;
  V->sp = L->sp;
  V->numin = L->numin - dP;
  V->numax = L->numax + dP;
  V->km.numin = V->numin;
  V->km.kmax = (1u << hk::kKeyBits) - 1u;
  V->km.scale = V->numax > V->numin ? (double)V->km.kmax / (V->numax - V->numin) : 0.0;
  V->km.pad = 0;
  V->shift_max = dP;
  // bounds of the view's reference widths (convex combinations of gamma_air and gamma_self)
  V->have_stats = L->have_stats;
  V->gref_max = std::max(L->gref_max, L->gself_max);
  V->n_min = L->n_min;
  V->n_max = L->n_max;
  if (ws) {
    V->nu = reinterpret_cast<double*>(ws + vl.o_nu);
    V->nu_pos = reinterpret_cast<double*>(ws + vl.o_pos);
    V->Sref = reinterpret_cast<double*>(ws + vl.o_S);
    V->E = reinterpret_cast<double*>(ws + vl.o_E);
    V->gref = reinterpret_cast<double*>(ws + vl.o_g);
    V->nexp = reinterpret_cast<double*>(ws + vl.o_n);
    V->perm = reinterpret_cast<int32_t*>(ws + vl.o_perm);
    V->keys = reinterpret_cast<uint32_t*>(ws + vl.o_kB);
  }
}

// Bins L by its centres shifted to pressure P into the view V (view_fields done).
hk_status build_view(const hk_lines* L, double P, double Pself, char* ws, const ViewLayout& vl, hk_lines* V,
                     hipStream_t st) {
  const int64_t N = L->N;
  uint32_t* kA = reinterpret_cast<uint32_t*>(ws + vl.o_kA);
  int32_t* vA = reinterpret_cast<int32_t*>(ws + vl.o_vA);
  uint32_t* kB = reinterpret_cast<uint32_t*>(ws + vl.o_kB);
  int32_t* vB = reinterpret_cast<int32_t*>(ws + vl.o_vB);
  uint32_t* hist = reinterpret_cast<uint32_t*>(ws + vl.o_hist);
  uint32_t* dtot = reinterpret_cast<uint32_t*>(ws + vl.o_dtot);
  const double pshift = P / L->sp.P_ref_atm;
  HK_HIP(hk::launch_shift_keys(L->nu, L->delta, N, pshift, V->km, kA, vA, st));
  HK_HIP(hk::launch_radix_pass(kA, vA, kB, vB, N, 0, hist, dtot, st));
  HK_HIP(hk::launch_radix_pass(kB, vB, kA, vA, N, 8, hist, dtot, st));
  HK_HIP(hk::launch_radix_pass(kA, vA, kB, vB, N, 16, hist, dtot, st));
  hk::ShiftArgs a;
  memset(&a, 0, sizeof a);
  a.src = vB;
  a.nu = L->nu;
  a.Sref = L->Sref;
  a.E = L->E;
  a.gair = L->gref;
  a.gself = L->gself;
  a.nexp = L->nexp;
  a.delta = L->delta;
  a.perm = L->perm;
  a.N = N;
  a.pshift = pshift;
  a.P = P;
  a.Pself = Pself;
  a.o_nu = const_cast<double*>(V->nu);
  a.o_pos = const_cast<double*>(V->nu_pos);
  a.o_S = V->Sref;
  a.o_E = V->E;
  a.o_g = V->gref;
  a.o_n = V->nexp;
  a.o_perm = V->perm;
  HK_HIP(hk::launch_shift_gather(a, st));
  return HK_OK;
}

hk_status hitran_checks(const hk_lines* lines, double T, double P_atm, double P_self, const hk_grid& grid,
                        double cutoff) {
  hk_status s = check_lines(lines);
  if (s != HK_OK) return s;
  if (!lines->gself || !lines->delta) return fail(HK_EINVAL, "not a HITRAN-style handle (hk_prepare_lines_hitran)");
  if (!(std::isfinite(T) && T > 0)) return fail(HK_EINVAL, "T must be finite and > 0");
  if (!(std::isfinite(P_atm) && P_atm >= 0)) return fail(HK_EINVAL, "P must be finite and >= 0");
  if (!(std::isfinite(P_self) && P_self >= 0 && P_self <= P_atm)) return fail(HK_EINVAL, "need 0 <= P_self <= P");
  if (!grid_ok(grid)) return fail(HK_EINVAL, "invalid grid");
  if (!cut_ok(cutoff)) return fail(HK_EINVAL, "cutoff must be > 0 (or +inf)");
  return HK_OK;
}

}  // namespace

extern "C" {

const char* hk_last_error(void) { return g_err.c_str(); }
const char* hk_version(void) { return "hk 0.1 (gfx950)"; }

hk_status hk_get_timings(hk_timings* out) {
  if (!out) return fail(HK_EINVAL, "out is NULL");
  *out = g_tim;
  return HK_OK;
}

int64_t hk_lines_count(const hk_lines* lines) { return lines ? lines->N : -1; }

hk_status hk_prepare_lines(const double* nu, const double* S_ref, const double* E_low, const double* gamma_ref,
                           const double* n_exp, int64_t n_lines, const hk_species* sp, hipStream_t stream,
                           hk_lines** out) {
  if (!out) return fail(HK_EINVAL, "out is NULL");
  if (!nu || !S_ref || !E_low || !gamma_ref || !n_exp) return fail(HK_EINVAL, "a line array is NULL");
  if (n_lines < 1 || n_lines >= (int64_t(1) << 31) - 1) return fail(HK_EINVAL, "n_lines %lld out of range", (long long)n_lines);
  if (!species_ok(sp)) return fail(HK_EINVAL, "invalid species constants");
  int dev;
  DevInfo di;
  hk_status s = device_init(&dev, &di);
  if (s != HK_OK) return s;
  const int64_t N = n_lines;
  Timer tm(stream);
  tm.mark();
  // handle memory
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes, 256); return o; };
  const size_t o_nu = take(8 * N), o_S = take(8 * N), o_E = take(8 * N), o_g = take(8 * N), o_n = take(8 * N),
               o_k = take(4 * N), o_p = take(4 * N);
  const size_t hbytes = off;
  // temporaries
  const int64_t G = (N + hk::kSortBlock - 1) / hk::kSortBlock;
  off = 0;
  const size_t t_k = take(4 * N), t_v = take(4 * N), t_h = take(4 * 256 * (size_t)G), t_d = take(4 * 256),
               t_mm = take(16), t_f = take(16), t_r = take(40 * N);
  const size_t tbytes = off;
  std::unique_ptr<hk_lines> L(new hk_lines());
  L->device = dev;
  L->N = N;
  L->sp = *sp;
  char* hm = nullptr;
  char* tmp = nullptr;
  size_t hgot = 0, tgot = 0;
  if (pool_alloc(dev, hbytes, reinterpret_cast<void**>(&hm), &hgot) != hipSuccess)
    return fail(HK_ENOMEM, "hipMalloc of %zu bytes failed", hbytes);
  if (pool_alloc(dev, tbytes, reinterpret_cast<void**>(&tmp), &tgot) != hipSuccess) {
    pool_free(dev, hm, hgot);
    return fail(HK_ENOMEM, "hipMalloc of %zu bytes failed", tbytes);
  }
  L->mem = hm;
  L->mem_bytes = hgot;
  L->nu = reinterpret_cast<double*>(hm + o_nu);
  L->Sref = reinterpret_cast<double*>(hm + o_S);
  L->E = reinterpret_cast<double*>(hm + o_E);
  L->gref = reinterpret_cast<double*>(hm + o_g);
  L->nexp = reinterpret_cast<double*>(hm + o_n);
  L->keys = reinterpret_cast<uint32_t*>(hm + o_k);
  L->perm = reinterpret_cast<int32_t*>(hm + o_p);
  uint32_t* kA = reinterpret_cast<uint32_t*>(tmp + t_k);
  int32_t* vA = reinterpret_cast<int32_t*>(tmp + t_v);
  uint32_t* hist = reinterpret_cast<uint32_t*>(tmp + t_h);
  uint32_t* dtot = reinterpret_cast<uint32_t*>(tmp + t_d);
  unsigned long long* mm = reinterpret_cast<unsigned long long*>(tmp + t_mm);
  int* flags = reinterpret_cast<int*>(tmp + t_f);
  double* rec = reinterpret_cast<double*>(tmp + t_r);
  auto cleanup_fail = [&](hk_status st, const char* what, hipError_t e) {
    if (hipStreamSynchronize(stream) == hipSuccess) {
      pool_free(dev, tmp, tgot);
      pool_free(dev, hm, hgot);
    } else {
      (void)hipGetLastError();  // the blocks' work did not complete: leak them rather than reuse them
    }
    return fail(st, "%s: %s", what, e == hipSuccess ? "" : hipGetErrorString(e));
  };
  hipError_t e = hk::launch_validate(nu, N, mm, flags, stream);
  if (e != hipSuccess) return cleanup_fail(HK_EDEVICE, "validate", e);
  unsigned long long hmm[2] = {0, 0};
  int hflag = 0;
  e = hipMemcpyAsync(hmm, mm, 16, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&hflag, flags, 4, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return cleanup_fail(HK_EDEVICE, "validate readback", e);
  if (hflag) {
    pool_free(dev, tmp, tgot);
    pool_free(dev, hm, hgot);
    return fail(HK_EINVAL, "line data invalid: need nu > 0 and finite");
  }
  double vmin, vmax;
  memcpy(&vmin, &hmm[0], 8);
  memcpy(&vmax, &hmm[1], 8);
  L->numin = vmin;
  L->numax = vmax;
  L->km.numin = vmin;
  L->km.kmax = (1u << hk::kKeyBits) - 1u;
  L->km.scale = vmax > vmin ? (double)L->km.kmax / (vmax - vmin) : 0.0;
  L->km.pad = 0;
  // keys -> stable LSD radix sort (3 passes of 8 bits; ping-pong ends in the handle arrays)
  e = hk::launch_keys(nu, S_ref, E_low, gamma_ref, n_exp, N, L->km, kA, vA, rec, flags, stream);
  if (e == hipSuccess) e = hk::launch_radix_pass(kA, vA, L->keys, L->perm, N, 0, hist, dtot, stream);
  if (e == hipSuccess) e = hk::launch_radix_pass(L->keys, L->perm, kA, vA, N, 8, hist, dtot, stream);
  if (e == hipSuccess) e = hk::launch_radix_pass(kA, vA, L->keys, L->perm, N, 16, hist, dtot, stream);
  if (e == hipSuccess)
    e = hk::launch_gather(L->perm, N, rec, L->nu, L->Sref, L->E, L->gref, L->nexp, stream);
  tm.mark();
  if (e == hipSuccess) e = hipMemcpyAsync(&hflag, flags + 1, 4, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return cleanup_fail(HK_EDEVICE, "binning", e);
  pool_free(dev, tmp, tgot);
  if (hflag) {
    pool_free(dev, hm, hgot);
    return fail(HK_EINVAL, "line data invalid: need S_ref >= 0, gamma_ref >= 0, E, n finite");
  }
  g_tim.bin_ms = tm.ms(0);
  *out = L.release();
  return HK_OK;
}

hk_status hk_release_lines(hk_lines* lines) {
  if (!lines) return HK_OK;
  {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    for (auto it = g_graphs.begin(); it != g_graphs.end();) {
      const void* h = nullptr;
      memcpy(&h, it->first.data(), sizeof h);
      if (h == lines) {
        (void)hipGraphExecDestroy(it->second.exec);
        (void)hipGraphDestroy(it->second.graph);
        it = g_graphs.erase(it);
      } else {
        ++it;
      }
    }
  }
  int cur = -1;
  (void)hipGetDevice(&cur);
  if (cur != lines->device) (void)hipSetDevice(lines->device);
  // wait for the work issued through the handle: the last call on each stream it was used on
  // (a device-wide wait only when a use could not be tracked)
  hipError_t e = hipSuccess;
  {
    std::lock_guard<std::mutex> lk(lines->use_mu);
    if (lines->untracked) e = hipDeviceSynchronize();
    for (int i = 0; i < lines->n_use; ++i) {
      hipError_t w = hipEventSynchronize(lines->use_event[i]);
      if (e == hipSuccess) e = w;
      (void)hipEventDestroy(lines->use_event[i]);
    }
    lines->n_use = 0;
  }
  hipError_t f = hipSuccess;
  if (e == hipSuccess) {
    pool_free(lines->device, lines->mem, lines->mem_bytes);  // its work has completed: reusable
    if (lines->mem2) pool_free(lines->device, lines->mem2, lines->mem2_bytes);
  } else {
    f = hipFree(lines->mem);
    if (lines->mem2) (void)hipFree(lines->mem2);
  }
  if (cur >= 0 && cur != lines->device) (void)hipSetDevice(cur);
  delete lines;
  if (e != hipSuccess) return fail(HK_EDEVICE, "waiting for the handle's work: %s", hipGetErrorString(e));
  if (f != hipSuccess) return fail(HK_EDEVICE, "hipFree: %s", hipGetErrorString(f));
  return HK_OK;
}

hk_status hk_empty_cache(void) {
  pool_drain(-1);
  return HK_OK;
}

hk_status hk_workspace_size(const hk_lines* lines, int mode, int32_t n_pairs, int32_t n_temps,
                            const hk_grid* grids, double cutoff, size_t* bytes) {
  return workspace_impl(lines, mode, n_pairs, n_temps, nullptr, nullptr, grids, cutoff, nullptr, nullptr, bytes);
}

hk_status hk_workspace_size_ex(const hk_lines* lines, int mode, int32_t n_pairs, const double* T,
                               const double* P_atm, const hk_grid* grids, double cutoff, const hk_options* options,
                               hipStream_t stream, size_t* bytes) {
  return workspace_impl(lines, mode, n_pairs, n_pairs, T, P_atm, grids, cutoff, options, stream, bytes);
}

hk_status hk_opacity(const hk_lines* lines, const hk_line_override* ovr, double T, double P_atm, hk_grid grid,
                     double cutoff, float* k, void* ws, size_t ws_bytes, hipStream_t stream) {
  hk_status s = opacity_impl(lines, ovr, T, P_atm, grid, cutoff, nullptr, k, ws, ws_bytes, stream, false);
  if (s == HK_OK) note_use(const_cast<hk_lines*>(lines), stream, true);
  return s;
}

hk_status hk_opacity_ex(const hk_lines* lines, const hk_line_override* ovr, double T, double P_atm, hk_grid grid,
                        double cutoff, const hk_options* options, float* k, void* ws, size_t ws_bytes,
                        hipStream_t stream) {
  hk_status s = opacity_impl(lines, ovr, T, P_atm, grid, cutoff, options, k, ws, ws_bytes, stream, false);
  if (s == HK_OK) note_use(const_cast<hk_lines*>(lines), stream, true);
  return s;
}

hk_status hk_opacity_noalloc(const hk_lines* lines, const hk_line_override* ovr, double T, double P_atm,
                             hk_grid grid, double cutoff, float* k, hipStream_t stream) {
  hk_status s = opacity_impl(lines, ovr, T, P_atm, grid, cutoff, nullptr, k, nullptr, 0, stream, true);
  if (s == HK_OK) note_use(const_cast<hk_lines*>(lines), stream, false);
  return s;
}

size_t hk_noalloc_max_bytes(void) { return hk::kScratchBytes; }

hk_status hk_opacity_batched(const hk_lines* lines, int32_t n_pairs, const double* T, const double* P_atm,
                             const hk_grid* grids, const int64_t* out_offset, double cutoff, float* k, void* ws,
                             size_t ws_bytes, hipStream_t stream) {
  hk_status s = batched_impl(lines, n_pairs, T, P_atm, grids, out_offset, cutoff, nullptr, k, ws, ws_bytes, stream);
  if (s == HK_OK) note_use(const_cast<hk_lines*>(lines), stream, true);
  return s;
}

hk_status hk_opacity_batched_ex(const hk_lines* lines, int32_t n_pairs, const double* T, const double* P_atm,
                                const hk_grid* grids, const int64_t* out_offset, double cutoff,
                                const hk_options* options, float* k, void* ws, size_t ws_bytes,
                                hipStream_t stream) {
  hk_status s = batched_impl(lines, n_pairs, T, P_atm, grids, out_offset, cutoff, options, k, ws, ws_bytes, stream);
  if (s == HK_OK) note_use(const_cast<hk_lines*>(lines), stream, true);
  return s;
}

hk_status hk_prepare_lines_hitran(const double* nu, const double* S_ref, const double* E_low, const double* gamma_air,
                                  const double* gamma_self, const double* n_exp, const double* delta_air,
                                  int64_t n_lines, const hk_species* sp, hipStream_t stream, hk_lines** out) {
  if (!out) return fail(HK_EINVAL, "out is NULL");
  if (!gamma_self || !delta_air) return fail(HK_EINVAL, "gamma_self or delta_air is NULL");
  hk_lines* L = nullptr;
  hk_status s = hk_prepare_lines(nu, S_ref, E_low, gamma_air, n_exp, n_lines, sp, stream, &L);
  if (s != HK_OK) return s;
  int dev;
  DevInfo di;
  s = device_init(&dev, &di);
  if (s != HK_OK) {
    hk_release_lines(L);
    return s;
  }
  const int64_t N = L->N;
  const size_t o_d = align_up(8 * (size_t)N, 256), bytes = o_d + 8 * (size_t)N;
  void* m2 = nullptr;
  size_t got = 0;
  if (pool_alloc(dev, bytes, &m2, &got) != hipSuccess) {
    hk_release_lines(L);
    return fail(HK_ENOMEM, "hipMalloc of %zu bytes failed", bytes);
  }
  L->mem2 = m2;
  L->mem2_bytes = got;
  L->gself = static_cast<double*>(m2);
  L->delta = reinterpret_cast<double*>(static_cast<char*>(m2) + o_d);
  unsigned long long h[4] = {0, 0, 0, 0};
  hipError_t e;
  {
    std::lock_guard<std::mutex> lk(g_stats_mu);
    e = hk::launch_hitran_check(gamma_self, delta_air, N, reinterpret_cast<int*>(di.stats_buf + 3), di.stats_buf,
                                stream);
    if (e == hipSuccess) e = hk::launch_gather2(L->perm, N, gamma_self, delta_air, L->gself, L->delta, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(h, di.stats_buf, sizeof h, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
  }
  if (e != hipSuccess) {
    hk_release_lines(L);
    return fail(HK_EDEVICE, "HITRAN fields: %s", hipGetErrorString(e));
  }
  int bad = 0;
  memcpy(&bad, &h[3], sizeof bad);
  if (bad) {
    hk_release_lines(L);
    return fail(HK_EINVAL, "line data invalid: need gamma_self >= 0 and finite, delta_air finite");
  }
  L->dmax = hk::ordered_to_double(h[0]);
  L->gself_max = hk::ordered_to_double(h[1]);
  *out = L;
  return HK_OK;
}

hk_status hk_workspace_size_hitran(const hk_lines* lines, double T, double P_atm, double P_self, hk_grid grid,
                                   double cutoff, const hk_options* options, hipStream_t stream, size_t* bytes) {
  if (!bytes) return fail(HK_EINVAL, "bytes is NULL");
  hk_status s = hitran_checks(lines, T, P_atm, P_self, grid, cutoff);
  if (s != HK_OK) return s;
  Opts o;
  s = opts_from(options, &o);
  if (s != HK_OK) return s;
  o.shifted = 1;
  int dev;
  DevInfo di;
  s = device_init(&dev, &di);
  if (s != HK_OK) return s;
  s = check_opts(const_cast<hk_lines*>(lines), nullptr, o, stream);
  if (s != HK_OK) return s;
  const ViewLayout vl = view_layout(lines->N);
  hk_lines V;
  view_fields(lines, P_atm, nullptr, vl, &V);
  size_t best = 0;
  for (const Tuning& tu : kCandidates) {
    Plan pl;
    s = make_plan(&V, 1, 1, &T, &P_atm, &grid, nullptr, cutoff, di, tu, o, &pl);
    if (s != HK_OK) return s;
    best = std::max(best, pl.total);
  }
  *bytes = vl.total + best;
  return HK_OK;
}

hk_status hk_opacity_hitran(const hk_lines* lines, double T, double P_atm, double P_self, hk_grid grid,
                            double cutoff, const hk_options* options, float* k, void* ws, size_t ws_bytes,
                            hipStream_t stream) {
  hk_status s = hitran_checks(lines, T, P_atm, P_self, grid, cutoff);
  if (s != HK_OK) return s;
  if (!k || !ws) return fail(HK_EINVAL, "k or workspace is NULL");
  if ((reinterpret_cast<uintptr_t>(ws) & 255u) != 0) return fail(HK_EINVAL, "workspace must be 256-byte aligned");
  Opts o;
  s = opts_from(options, &o);
  if (s != HK_OK) return s;
  o.shifted = 1;
  int dev;
  DevInfo di;
  s = device_init(&dev, &di);
  if (s != HK_OK) return s;
  s = check_opts(const_cast<hk_lines*>(lines), nullptr, o, stream);
  if (s != HK_OK) return s;
  const ViewLayout vl = view_layout(lines->N);
  if (ws_bytes < vl.total) return fail(HK_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, vl.total);
  char* w = static_cast<char*>(ws);
  hk_lines V;
  view_fields(lines, P_atm, w, vl, &V);
  // plan first (no device work before every argument is known to fit)
  const int64_t zero = 0;
  Tuning tu;
  if (!env_tuning(&tu)) tu = Tuning{};
  Plan pl;
  s = make_plan(&V, 1, 1, &T, &P_atm, &grid, &zero, cutoff, di, tu, o, &pl);
  if (s != HK_OK) return s;
  if (ws_bytes < vl.total + pl.total)
    return fail(HK_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, vl.total + pl.total);
  s = build_view(lines, P_atm, P_self, w, vl, &V, stream);
  if (s != HK_OK) return s;
  s = run_forward(&V, nullptr, pl, &T, &P_atm, cutoff, k, w + vl.total, stream);
  if (s == HK_OK) note_use(const_cast<hk_lines*>(lines), stream, true);
  return s;
}

hk_status hk_opacity_stream(const double* nu, const double* S_ref, const double* E_low, const double* gamma_ref,
                            const double* n_exp, int64_t n_lines, const hk_species* sp, double T, double P_atm,
                            hk_grid grid, double cutoff, const hk_options* options, int64_t chunk_lines, float* k,
                            hipStream_t stream) {
  if (!nu || !S_ref || !E_low || !gamma_ref || !n_exp) return fail(HK_EINVAL, "a host line array is NULL");
  if (n_lines < 1) return fail(HK_EINVAL, "n_lines must be >= 1");
  if (chunk_lines < 1 || chunk_lines >= (int64_t(1) << 31) - 1) return fail(HK_EINVAL, "chunk_lines out of range");
  if (!species_ok(sp)) return fail(HK_EINVAL, "invalid species constants");
  if (!(std::isfinite(T) && T > 0)) return fail(HK_EINVAL, "T must be finite and > 0");
  if (!(std::isfinite(P_atm) && P_atm >= 0)) return fail(HK_EINVAL, "P must be finite and >= 0");
  if (!grid_ok(grid)) return fail(HK_EINVAL, "invalid grid");
  if (!cut_ok(cutoff)) return fail(HK_EINVAL, "cutoff must be > 0 (or +inf)");
  if (!k) return fail(HK_EINVAL, "k is NULL");
  Opts o;
  hk_status s = opts_from(options, &o);
  if (s != HK_OK) return s;
  if (o.direct && !o.default_path()) return fail(HK_EINVAL, "direct applies to the default path only");
  int dev;
  DevInfo di;
  s = device_init(&dev, &di);
  if (s != HK_OK) return s;
  const int64_t C = std::min(chunk_lines, n_lines);
  // device blocks: two raw chunk buffers (5 fields each) and one chunk result on the grid; the
  // opacity workspace grows to the largest chunk's need
  const size_t raw = align_up(40 * (size_t)C, 256), tmpb = align_up(4 * (size_t)grid.n, 256);
  void* blk = nullptr;
  size_t blk_got = 0;
  if (pool_alloc(dev, 2 * raw + tmpb, &blk, &blk_got) != hipSuccess)
    return fail(HK_ENOMEM, "hipMalloc of %zu bytes failed", 2 * raw + tmpb);
  char* bc = static_cast<char*>(blk);
  float* ktmp = reinterpret_cast<float*>(bc + 2 * raw);
  void* wsb = nullptr;
  size_t ws_got = 0;
  hipStream_t cs = nullptr;
  hipEvent_t copied[2] = {nullptr, nullptr};
  hk_status rs = HK_OK;
  auto put = [&](int64_t c, hipStream_t st) -> hipError_t {  // H2D copy of chunk c into buffer c % 2
    const int64_t i0 = c * C, m = std::min(C, n_lines - i0);
    double* b = reinterpret_cast<double*>(bc + (size_t)(c % 2) * raw);
    const double* src[5] = {nu, S_ref, E_low, gamma_ref, n_exp};
    for (int f = 0; f < 5; ++f) {
      hipError_t e = hipMemcpyAsync(b + (size_t)f * C, src[f] + i0, 8 * (size_t)m, hipMemcpyHostToDevice, st);
      if (e != hipSuccess) return e;
    }
    return hipEventRecord(copied[c % 2], st);
  };
  do {
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&copied[0], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&copied[1], hipEventDisableTiming);
    if (e == hipSuccess) e = hk::launch_fill0(k, grid.n, stream);
    if (e == hipSuccess) e = put(0, cs);
    if (e != hipSuccess) { rs = fail(HK_EDEVICE, "stream set-up: %s", hipGetErrorString(e)); break; }
    const int64_t nc = (n_lines + C - 1) / C;
    for (int64_t c = 0; c < nc && rs == HK_OK; ++c) {
      const int64_t m = std::min(C, n_lines - c * C);
      // the next chunk's copy runs on the copy engine while this one is binned and evaluated
      // (its buffer's previous chunk was consumed by a binning that has completed)
      if (c + 1 < nc && (e = put(c + 1, cs)) != hipSuccess) { rs = fail(HK_EDEVICE, "copy: %s", hipGetErrorString(e)); break; }
      if ((e = hipStreamWaitEvent(stream, copied[c % 2], 0)) != hipSuccess) {
        rs = fail(HK_EDEVICE, "wait: %s", hipGetErrorString(e));
        break;
      }
      double* b = reinterpret_cast<double*>(bc + (size_t)(c % 2) * raw);
      hk_lines* L = nullptr;
      rs = hk_prepare_lines(b, b + C, b + 2 * (size_t)C, b + 3 * (size_t)C, b + 4 * (size_t)C, m, sp, stream, &L);
      if (rs != HK_OK) break;
      // the chunk's band of the grid: points within its largest cutting length of its lines
      if (o.cut_mode == hk::kCutLorentz) rs = ensure_line_stats(L, stream);
      int64_t j0 = 0, j1 = grid.n - 1;
      if (rs == HK_OK && !std::isinf(cutoff)) {
        const double cm = max_cut_length(L, o, cutoff, T, P_atm);
        const double a = std::floor((L->numin - cm - grid.nu_start) / grid.dnu) - 2.0;
        const double bb = std::ceil((L->numax + cm - grid.nu_start) / grid.dnu) + 2.0;
        j0 = a < 0.0 ? 0 : (a > (double)(grid.n - 1) ? grid.n : (int64_t)a);
        j1 = bb > (double)(grid.n - 1) ? grid.n - 1 : (bb < 0.0 ? -1 : (int64_t)bb);
      }
      if (rs == HK_OK && j0 <= j1) {
        // evaluated on the grid's own points 0..j1 (the same nu_start: grid points are a rounded
        // product and a rounded sum, so a re-based grid would move them by rounding); spans
        // below j0 hold no line of the chunk and cost only their empty work items, and only
        // j0..j1 are added to k
        const hk_grid g = {grid.nu_start, grid.dnu, j1 + 1};
        size_t need = 0;
        rs = workspace_impl(L, 0, 1, 1, &T, &P_atm, &g, cutoff, options, stream, &need);
        if (rs == HK_OK && need > ws_got) {
          if (wsb) {
            (void)hipStreamSynchronize(stream);
            pool_free(dev, wsb, ws_got);
            wsb = nullptr;
            ws_got = 0;
          }
          if (pool_alloc(dev, need, &wsb, &ws_got) != hipSuccess) rs = fail(HK_ENOMEM, "hipMalloc of %zu bytes failed", need);
        }
        if (rs == HK_OK) rs = opacity_impl(L, nullptr, T, P_atm, g, cutoff, options, ktmp, wsb, ws_got, stream, false);
        if (rs == HK_OK && (e = hk::launch_accumulate(k + j0, ktmp + j0, j1 - j0 + 1, stream)) != hipSuccess)
          rs = fail(HK_EDEVICE, "accumulate: %s", hipGetErrorString(e));
        if (rs == HK_OK) note_use(L, stream, true);
      }
      hk_status r2 = hk_release_lines(L);  // waits for the chunk's work
      if (rs == HK_OK) rs = r2;
    }
  } while (false);
  hipError_t ew = hipStreamSynchronize(stream);
  if (cs) { (void)hipStreamSynchronize(cs); (void)hipStreamDestroy(cs); }
  for (auto& ev : copied) if (ev) (void)hipEventDestroy(ev);
  if (ew == hipSuccess) {
    pool_free(dev, blk, blk_got);
    if (wsb) pool_free(dev, wsb, ws_got);
  }
  if (rs == HK_OK && ew != hipSuccess) rs = fail(HK_EDEVICE, "stream: %s", hipGetErrorString(ew));
  return rs;
}

hk_status hk_opacity_backward(const hk_lines* lines, const hk_line_override* ovr, double T, double P_atm,
                              hk_grid grid, double cutoff, const float* dL_dk, double* dL_dT_lnP, double* dL_dSref,
                              float* dL_dgref, float* dL_dn, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!(std::isfinite(T) && T > 0)) return fail(HK_EINVAL, "T must be finite and > 0");
  if (!(std::isfinite(P_atm) && P_atm >= 0)) return fail(HK_EINVAL, "P must be finite and >= 0");
  if (!grid_ok(grid)) return fail(HK_EINVAL, "invalid grid");
  if (!cut_ok(cutoff)) return fail(HK_EINVAL, "cutoff must be > 0 (or +inf)");
  if (!dL_dk || !dL_dT_lnP || !ws) return fail(HK_EINVAL, "dL_dk, dL_dT_lnP or workspace is NULL");
  if ((reinterpret_cast<uintptr_t>(ws) & 255u) != 0) return fail(HK_EINVAL, "workspace must be 256-byte aligned");
  hk_status s = check_lines(lines);
  if (s != HK_OK) return s;
  int dev;
  DevInfo di;
  s = device_init(&dev, &di);
  if (s != HK_OK) return s;
  const BwdLayout bl = backward_layout(lines->N, grid.n);
  if (ws_bytes < bl.total) return fail(HK_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, bl.total);
  Timer tm(stream);
  tm.mark();
  char* w = static_cast<char*>(ws);
  int4* grec = reinterpret_cast<int4*>(w + bl.off_gr);
  double* contrib = reinterpret_cast<double*>(w + bl.off_contrib);
  double* part = reinterpret_cast<double*>(w + bl.off_part);
  HK_HIP(hk::launch_gridrec(lines->nu, lines->N, grid.nu_start, grid.dnu, grid.n, cutoff, grec, stream));
  hk::AdjArgs a;
  memset(&a, 0, sizeof a);
  a.pa = prep_args(lines, ovr, T);
  a.pa.pfac = P_atm / lines->sp.P_ref_atm;
  a.grec = grec;
  a.g = dL_dk;
  a.nu_start = grid.nu_start;
  a.dnu = grid.dnu;
  a.n = grid.n;
  a.T = T;
  a.q_b = lines->sp.q_b;
  for (int i = 0; i < hk::kKmax; ++i) a.zK[i] = (float)kZK[i];
  a.dSref = dL_dSref;
  a.dgref = dL_dgref;
  a.dn = dL_dn;
  a.contrib = contrib;
  a.lrec = reinterpret_cast<double*>(w + bl.off_lrec);
  a.lzone = reinterpret_cast<int*>(w + bl.off_lzone);
  double* gpref[hk::kAdjLevels];
  for (int lv = 0; lv < hk::kAdjLevels; ++lv) {
    gpref[lv] = reinterpret_cast<double*>(w + bl.off_pref[lv]);
    a.gpref[lv] = gpref[lv];
  }
  const int64_t want = (lines->N + hk::kWavesPerWG - 1) / hk::kWavesPerWG;
  // two rounds of resident workgroups (lines are assigned statically, round-robin over the waves)
  const int64_t cap = std::min<int64_t>((int64_t)di.cus * 2 * di.adj_per_cu, kAdjMaxWaves / hk::kWavesPerWG);
  const int blocks = (int)std::max<int64_t>(1, std::min(want, cap));
  long long* stats = reinterpret_cast<long long*>(w + bl.off_stats);
  a.stats = tm.on ? stats : nullptr;
  if (lines->N > 0) {
    // node weights of the adjoint's far units: Lagrange weights of 16 nodes over 256, 1024 and
    // 4096 points
    for (int lv = 0; lv < hk::kAdjLevels; ++lv)
      HK_HIP(hk::launch_adj_nodes(dL_dk, grid.n, lv, di.adj_w[lv], gpref[lv], stream));
    HK_HIP(hk::launch_adjoint(a, blocks, stream));
  }
  HK_HIP(hk::launch_reduce2(contrib, lines->N, part, kBwdPartials, dL_dT_lnP, stream));
  tm.mark();
  tm.finish();
  g_tim.prep_ms = g_tim.worklist_ms = g_tim.voigt_ms = g_tim.combine_ms = g_tim.core_ms = g_tim.far_ms = -1;
  g_tim.core_evals = g_tim.wing_evals = -1;
  for (int c = 0; c < 8; ++c) g_tim.class_evals[c] = -1;
  g_tim.backward_ms = tm.ms(0);
  g_tim.backward_evals = -1;
  if (tm.on && lines->N > 0) {
    std::vector<long long> h((size_t)blocks * hk::kWavesPerWG);
    HK_HIP(hipMemcpy(h.data(), stats, sizeof(long long) * h.size(), hipMemcpyDeviceToHost));
    long long t = 0;
    for (long long v : h) t += v;
    g_tim.backward_evals = t;
  }
  note_use(const_cast<hk_lines*>(lines), stream, true);
  return HK_OK;
}

hk_status hk_debug_cut_bounds(const hk_lines* lines, hk_grid grid, double cutoff, int32_t* j_lo, int32_t* j_hi,
                              hipStream_t stream) {
  hk_status s = check_lines(lines);
  if (s != HK_OK) return s;
  if (!grid_ok(grid) || !cut_ok(cutoff) || !j_lo || !j_hi) return fail(HK_EINVAL, "invalid argument");
  HK_HIP(hk::launch_cut_bounds(lines->nu, lines->perm, lines->N, grid.nu_start, grid.dnu, grid.n, cutoff, j_lo,
                               j_hi, stream));
  note_use(const_cast<hk_lines*>(lines), stream, true);
  return HK_OK;
}

hk_status hk_debug_grid_records(const hk_lines* lines, double T, double P_atm, hk_grid grid, double cutoff,
                                const hk_options* options, void* ws, size_t ws_bytes, int32_t* j_lo, int32_t* j_hi,
                                float* plinth, hipStream_t stream) {
  hk_status s = check_lines(lines);
  if (s != HK_OK) return s;
  if (!grid_ok(grid) || !cut_ok(cutoff) || !(std::isfinite(T) && T > 0) || !(std::isfinite(P_atm) && P_atm >= 0))
    return fail(HK_EINVAL, "invalid argument");
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255u) != 0) return fail(HK_EINVAL, "workspace NULL or unaligned");
  const size_t N = (size_t)lines->N;
  const size_t need = align_up(8 * N, 256) + align_up(16 * N, 256) + align_up(4 * N, 256);
  if (ws_bytes < need) return fail(HK_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, need);
  Opts o;
  s = opts_from(options, &o);
  if (s != HK_OK) return s;
  int dev;
  DevInfo di;
  s = device_init(&dev, &di);
  if (s != HK_OK) return s;
  s = check_opts(const_cast<hk_lines*>(lines), nullptr, o, stream);
  if (s != HK_OK) return s;
  char* w = static_cast<char*>(ws);
  float* S_T = reinterpret_cast<float*>(w);
  float* gT = S_T + N;
  int4* grec = reinterpret_cast<int4*>(w + align_up(8 * N, 256));
  float* plin = reinterpret_cast<float*>(w + align_up(8 * N, 256) + align_up(16 * N, 256));
  hk::PrepArgs pa = prep_args(lines, nullptr, T);
  HK_HIP(hk::launch_prep(pa, S_T, gT, nullptr, nullptr, nullptr, stream));
  Plan pl;
  pl.opts = o;
  const hk::GridRecArgs ga = gridrec_args(lines, nullptr, pl, 0, T, P_atm, grid, cutoff, S_T, grec, plin);
  HK_HIP(hk::launch_gridrec_ex(ga, stream));
  HK_HIP(hk::launch_scatter_grec(grec, plin, lines->perm, lines->N, j_lo, j_hi, plinth, stream));
  note_use(const_cast<hk_lines*>(lines), stream, true);
  return HK_OK;
}

hk_status hk_debug_sorted(const hk_lines* lines, uint32_t* keys, int32_t* perm, hipStream_t stream) {
  hk_status s = check_lines(lines);
  if (s != HK_OK) return s;
  if (!keys || !perm) return fail(HK_EINVAL, "NULL argument");
  HK_HIP(hipMemcpyAsync(keys, lines->keys, 4 * lines->N, hipMemcpyDeviceToDevice, stream));
  HK_HIP(hipMemcpyAsync(perm, lines->perm, 4 * lines->N, hipMemcpyDeviceToDevice, stream));
  note_use(const_cast<hk_lines*>(lines), stream, true);
  return HK_OK;
}

hk_status hk_debug_line_params(const hk_lines* lines, double T, double P_atm, double* S_T, double* alpha,
                               double* gamma, hipStream_t stream) {
  hk_status s = check_lines(lines);
  if (s != HK_OK) return s;
  if (!(std::isfinite(T) && T > 0) || !(std::isfinite(P_atm) && P_atm >= 0)) return fail(HK_EINVAL, "bad T or P");
  hk::PrepArgs a = prep_args(lines, nullptr, T);
  a.pfac = P_atm / lines->sp.P_ref_atm;
  HK_HIP(hk::launch_prep(a, nullptr, nullptr, S_T, alpha, gamma, stream));
  note_use(const_cast<hk_lines*>(lines), stream, true);
  return HK_OK;
}

}  // extern "C"
