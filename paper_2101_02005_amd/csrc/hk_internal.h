// Internal declarations shared by the kernels (hk_kernels.hip) and the host library
// (hk_api.cpp). Not part of the public interface.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace hk {

constexpr int kWave = 64;        // CDNA wavefront width
constexpr int kThreads = 256;    // threads per workgroup of the tile-far and sort kernels
constexpr int kWavesPerWG = kThreads / kWave;  // spans per tile of the tile-far pass
constexpr int kKmax = 5;         // highest order of the far-wing series
constexpr int kKw = 9;           // ... in the wing pass next to the line cores (the default path)
constexpr int kWeidN = 18;       // terms of the FP64 core rational approximation
constexpr int kWeidN40 = 40;     // terms of the FP64 approximation (plinth values, line-core FP64 rounds)
constexpr int kKeyBits = 24;     // linear wavenumber-bin key width
constexpr int kRadixBits = 8;
constexpr int kSortItems = 32;   // keys per thread per sort block
constexpr int kSortBlock = kThreads * kSortItems;
constexpr int kFillPairs = 48;   // pair descriptors per fill launch (kernel-argument space)
constexpr int kNodes = 16;       // Chebyshev nodes of a span or tile for lines far from it
constexpr double kFarSpans = 1.5;  // far: centre at least 1.5 spans (3 half-spans) from the span centre
constexpr int kFar8Nodes = 8;    // Chebyshev nodes of a span for lines very far from it
constexpr double kFar8Spans = 3.0; // very far: centre at least 3 spans (6 half-spans) from the span centre
constexpr int kMidNodes = 32;    // Chebyshev nodes of a span for lines at middle distance
constexpr double kMidSpans = 0.75; // middle: centre 0.75-1.5 spans (1.5-3 half-spans) from the span centre
constexpr int kMaskNodes = 6;    // Chebyshev nodes of a span for lines whose cut bound falls on it
constexpr double kMaskSpans = 6.0; // such lines are evaluated at nodes when at least 6 spans away
constexpr int kMaskMaxSpan = 128;  // ... and only on spans of at most 128 points (P <= 2)
constexpr double kTileFar = 1.5;   // tile-far: centre at least 1.5 tile widths from the tile centre

// cos((2k + 1) pi / (2m)), k < m: Chebyshev points of the first kind on [-1, 1] for m = 6, 8, 16
// and 32 (the host checks the tables against cos at initialisation).
__host__ __device__ constexpr double cheb_cos8(int k) {
  switch (k) {
    case 0: return 0.98078528040323043;
    case 1: return 0.83146961230254524;
    case 2: return 0.55557023301960229;
    case 3: return 0.19509032201612833;
    case 4: return -0.19509032201612819;
    case 5: return -0.55557023301960196;
    case 6: return -0.83146961230254535;
    case 7: return -0.98078528040323043;
    default: return 0.0;
  }
}
__host__ __device__ constexpr double cheb_cos6(int k) {
  switch (k) {
    case 0: return 0.96592582628906831;
    case 1: return 0.70710678118654757;
    case 2: return 0.25881904510252074;
    case 3: return -0.25881904510252063;
    case 4: return -0.70710678118654746;
    case 5: return -0.9659258262890682;
    default: return 0.0;
  }
}
__host__ __device__ constexpr double cheb_cos16(int k) {
  switch (k) {
    case 0: return 0.99518472667219693;
    case 1: return 0.95694033573220882;
    case 2: return 0.88192126434835505;
    case 3: return 0.77301045336273699;
    case 4: return 0.63439328416364549;
    case 5: return 0.47139673682599781;
    case 6: return 0.29028467725446233;
    case 7: return 0.09801714032956077;
    case 8: return -0.098017140329560645;
    case 9: return -0.29028467725446216;
    case 10: return -0.4713967368259977;
    case 11: return -0.63439328416364538;
    case 12: return -0.77301045336273699;
    case 13: return -0.88192126434835494;
    case 14: return -0.95694033573220882;
    case 15: return -0.99518472667219682;
    default: return 0.0;
  }
}
__host__ __device__ constexpr double cheb_cos32(int k) {
  switch (k) {
    case 0: return 0.99879545620517241;
    case 1: return 0.98917650996478101;
    case 2: return 0.97003125319454397;
    case 3: return 0.94154406518302081;
    case 4: return 0.90398929312344334;
    case 5: return 0.85772861000027212;
    case 6: return 0.80320753148064494;
    case 7: return 0.74095112535495911;
    case 8: return 0.67155895484701833;
    case 9: return 0.59569930449243347;
    case 10: return 0.51410274419322166;
    case 11: return 0.4275550934302822;
    case 12: return 0.33688985339222005;
    case 13: return 0.24298017990326398;
    case 14: return 0.14673047445536175;
    case 15: return 0.049067674327418126;
    case 16: return -0.049067674327418008;
    case 17: return -0.14673047445536164;
    case 18: return -0.24298017990326387;
    case 19: return -0.33688985339221994;
    case 20: return -0.42755509343028186;
    case 21: return -0.51410274419322166;
    case 22: return -0.59569930449243336;
    case 23: return -0.67155895484701844;
    case 24: return -0.74095112535495888;
    case 25: return -0.80320753148064483;
    case 26: return -0.85772861000027201;
    case 27: return -0.90398929312344334;
    case 28: return -0.9415440651830207;
    case 29: return -0.97003125319454397;
    case 30: return -0.98917650996478101;
    case 31: return -0.99879545620517241;
    default: return 0.0;
  }
}
// Node k of m (6, 8, 16 or 32) on a span of S grid points [0, S - 1], in FP32: the device
// evaluates the lines there, and the host's interpolation weights are exact for these positions.
__host__ __device__ constexpr double cheb_cos(int m, int k) {
  return m == 6 ? cheb_cos6(k) : m == 8 ? cheb_cos8(k) : m == 16 ? cheb_cos16(k) : cheb_cos32(k);
}
__host__ __device__ constexpr float node_pos(int S, int m, int k) {
  return (float)(0.5 * (S - 1) * (1.0 + cheb_cos(m, k)));
}

// Wavenumber -> bin key: clamp(floor((v - numin) * scale), 0, kmax), evaluated in FP64.
struct KeyMap {
  double numin, scale;
  uint32_t kmax;
  uint32_t pad;
};

// One (T, P, grid) evaluation of a call.
struct PairDesc {
  double nu_start, dnu;
  int64_t n;
  int64_t out_off;
  double pfac;        // P / P_ref
  double beta;        // alpha = nu * beta at this T
  int32_t tidx;       // which per-temperature prep arrays
  int32_t tile_base;  // first global tile of this pair
  int32_t n_tiles;
  int32_t gidx;       // which grid-record array (pairs with equal grids share one)
};

// The lines of one span (64 P grid points, one wave of the wing pass) as segments of the
// sorted list, in list order; the tile-far ranges of its tile are left out.
constexpr int kMaxSeg = 21;  // elementary intervals between 22 range ends
enum SegKind : uint8_t {
  kSegDirect = 0,     // evaluated at every point of the span
  kSegFar = 1,        // far: at the span's kNodes nodes
  kSegMid = 2,        // middle distance: at the span's kMidNodes nodes
  kSegMaskLeft = 3,   // far, cut bound on the span, reaching it from the left: kMaskNodes nodes
  kSegMaskRight = 4,  // the same from the right
  kSegFar8 = 5,       // very far: at the span's kFar8Nodes nodes
};
struct SpanSeg {
  int32_t lo[kMaxSeg];   // first line of segment q
  int32_t len[kMaxSeg];  // its line count
  uint8_t kind[kMaxSeg]; // its SegKind
  uint8_t n;             // segment count
};

// Arguments of the persistent Voigt kernels (wing pass over spans, line-core pass).
struct VoigtArgs {
  const double* nu;        // sorted, N
  const float* S_T;        // [n_temps][N] strength at T
  const float* gT;         // [n_temps][N] gamma_ref (T_ref/T)^n
  const int4* grec;        // [n_grids][N] (offset bits, reference index, cut lo, cut hi)
  const PairDesc* pairs;
  const int32_t* tile_lo;  // core pass, per span: first line
  const int32_t* tile_hi;  // core pass, per span: one past the last line
  const SpanSeg* segs;     // wing pass, per span: its line segments
  const int32_t* tile_nc;  // per span: chunks (work items)
  const int32_t* item_base;// per span: first item; [n_tiles_total] = total items
  float* k;
  float* partial;          // [item][64 P]: chunk sums of multi-chunk spans (each pass its own)
  int* counter;            // work-item dispenser (scheduling only)
  long long* stats;        // nullable: per-wave count of the evaluations made: core evaluations
                           // (k_core), or 64 P per line evaluated directly plus kNodes per line
                           // evaluated at the span's nodes (k_wing)
  int64_t N;
  double cut;              // > 0; +inf: no cut
  float zK[kKmax];         // |z| above which the series of order K (1..kKmax) is used
  float zw[kKw];           // the same for orders 1..kKw (the wing pass's lines next to their cores)
  float zcore;             // core points: |z| below it (k_core's; the wing pass and k_direct skip them)
  int32_t n_pairs;
  int32_t n_tiles_total;   // spans
  int32_t chunk;           // lines per work item
  int32_t items_cap;       // rows of `partial` (work items beyond it are never written)
  const double* cheb_w;    // [kNodes][64 P] Lagrange weights of the span's Chebyshev nodes
  const double* far8_w;    // [kFar8Nodes][64 P] the same for the very-far nodes
  const double* mid_w;     // [kMidNodes][64 P] the same for the middle-distance nodes
  const float* mask_w;     // [kMaskNodes][64 P] the same for the nodes of lines with a cut bound on it
  int* status;             // nullable: bit 0 set when a work item fell beyond the partial rows
  const double* nu_pos;    // nullable: line centres when they differ from nu (a shifted list's
                           // view; nu then holds the transition wavenumbers the widths are taken at)
};

// Arguments of the tile-far pass (lines evaluated at the tile's Chebyshev nodes) and its combine.
// Tile-far lines come in two classes: c = 0 (1.5-3 tile widths from the tile centre) at the
// tile's kNodes nodes, c = 1 (at least 3) at its kFar8Nodes nodes.
struct FarArgs {
  const double* nu;        // sorted, N
  const float* S_T;        // [n_temps][N]
  const float* gT;         // [n_temps][N]
  const PairDesc* pairs;
  const int4* tile_far;    // [tile][c]: the class-c line ranges [x, y) and [z, w)
  const int32_t* item_base[2];  // per class, per global tile: first item; [n_tiles_total] = total
  double* node_part[2];    // per class: [item][node count] node sums of one work item
  int* counter[2];         // per class: work-item dispenser (scheduling only)
  long long* stats;        // nullable: [class][block] count of node evaluations
  const double* tile_w[2]; // per class: [node count][tile width] Lagrange weights of the tile's nodes
  float* k;
  int64_t N;
  float zK[kKmax];
  int32_t n_pairs;
  int32_t n_tiles_total;
  int32_t chunk;           // tile-far lines per work item
  int32_t items_cap[2];    // rows of node_part
  int32_t W;               // tile width in grid points
  float tile_x[kNodes];    // class-0 node positions relative to the tile's first point
  float tile_x8[kFar8Nodes];  // class-1 node positions
  int* status;             // nullable: bit 0 set when a work item fell beyond the node-sum rows
};

struct PrepArgs {
  const double* nu;        // sorted
  const double* Sref;      // sorted
  const double* E;         // sorted
  const double* gref;      // sorted
  const double* nexp;      // sorted
  const int32_t* perm;     // sorted position -> caller index
  const double* ovr_S;     // caller order or null
  const double* ovr_g;
  const double* ovr_n;
  int64_t N;
  double c2_over_T;        // c2 / T
  double c2_over_Tref;     // c2 / T_ref
  double c2E_coef;         // c2 (1/T_ref - 1/T)
  double q_ratio;          // Q(T_ref)/Q(T)
  double log_tr;           // ln(T_ref/T)
  double beta;             // alpha = nu * beta (debug output only)
  double pfac;             // P / P_ref (debug output only)
};

// Arguments of the adjoint kernel (one (T, P) and one grid).
struct AdjArgs {
  PrepArgs pa;             // line data, temperature constants, beta and pfac
  const int4* grec;        // grid records of the grid
  const float* g;          // dL/dk on the grid
  double nu_start, dnu;
  int64_t n;
  double T, q_b;
  float zK[kKmax];
  double* dSref;           // caller order, nullable
  float* dgref;            // caller order, nullable
  float* dn;               // caller order, nullable
  double* contrib;         // [N][2], sorted order: per-line dL/dT and dL/dlnP terms
  double* lrec;            // [N][8], sorted order: per-line FP64 quantities (k_adj_lines)
  int* lzone;              // [N][16], sorted order: per-line walk bounds (k_adj_lines), 16-byte aligned
  long long* stats;        // nullable: per wave of k_adjoint, the evaluations it made
  const double* gpref[3];  // per level L: [unit][kNodes][kAdjSpan 4^L]: per far unit of kAdjSpan 4^L
                           // points, the prefix sums over its points j of dL/dk_j times node k's
                           // Lagrange weight at j
};
constexpr int kAdjSpan = 256;   // points per span of the adjoint (one step of a wave)
constexpr int kAdjLevels = 3;   // far units of kAdjSpan, 4 kAdjSpan and 16 kAdjSpan points

// Line profiles and cutting-length modes of the options path.
enum { kProfVoigt = 0, kProfLorentz = 1, kProfDoppler = 2, kProfBinned = 3 };
enum { kCutFixed = 0, kCutDoppler = 1, kCutLorentz = 2 };

// Arguments of the per-line grid records with per-line cutting lengths and plinth values.
struct GridRecArgs {
  PrepArgs pa;             // sorted line data, overrides, pfac
  const float* S_T;        // strength at T (plinth values)
  double nu_start, dnu;
  int64_t n;
  double cut;              // fixed length, or the multiple of the line's width (+inf: no cut)
  double cut_dop;          // cut sqrt(ln 2): multiple of alpha for the Doppler half-width mode
  double c_light;          // alpha = (nu / c_light) alpha_fac
  double alpha_fac;        // sqrt(2 k_B T / m)
  double t_ratio;          // T_ref / T
  int32_t cut_mode, profile, plinth;
  int4* grec;              // out: per line (offset bits, reference index, cut lo, cut hi)
  float* plin;             // out, nullable: per line S(T) f(cut)
  const double* nu_pos;    // nullable: line centres when they differ from pa.nu (shifted list)
};

// Arguments of the shifted view of a HITRAN-style list at one pressure (k_shift_gather).
struct ShiftArgs {
  const int32_t* src;      // view position -> handle position (sorted by shifted centre)
  const double *nu, *Sref, *E, *gair, *gself, *nexp, *delta;  // handle (sorted by nu) arrays
  const int32_t* perm;     // handle position -> caller index
  int64_t N;
  double pshift;           // P / P_ref: centre = nu + delta pshift
  double P, Pself;         // atm
  double *o_nu, *o_pos, *o_S, *o_E, *o_g, *o_n;
  int32_t* o_perm;
};

// Bytes of the fixed scratch array of the allocation-free entry point.
constexpr size_t kScratchBytes = size_t(64) << 20;

// Launch wrappers (hk_kernels.hip); each returns the launch status.
// flags[0]: a nu <= 0 or non-finite (k_validate); flags[1]: another field invalid (k_keys)
hipError_t launch_validate(const double* nu, int64_t N, unsigned long long* mm, int* flags, hipStream_t st);
hipError_t launch_keys(const double* nu, const double* S, const double* E, const double* g, const double* n,
                       int64_t N, KeyMap km, uint32_t* keys, int32_t* vals, double* rec, int* flags,
                       hipStream_t st);
hipError_t launch_radix_pass(const uint32_t* kin, const int32_t* vin, uint32_t* kout, int32_t* vout,
                             int64_t N, int shift, uint32_t* hist, uint32_t* dig_tot, hipStream_t st);
hipError_t launch_gather(const int32_t* perm, int64_t N, const double* rec, double* onu, double* oS, double* oE,
                         double* og, double* on, hipStream_t st);
hipError_t launch_prep(const PrepArgs& a, float* S_T, float* gT, double* S64, double* a64, double* g64,
                       hipStream_t st);
hipError_t launch_fill_pairs(const PairDesc* host_pairs, int count, PairDesc* dst, int* status, hipStream_t st);
hipError_t launch_worklist(const uint32_t* keys, int64_t N, KeyMap km, double numin, double numax,
                           const PairDesc* pairs,
                           int n_pairs, int n_tiles_total, int tile_w, double cut, double core_z, int chunk,
                           int32_t* lo, int32_t* hi, int32_t* nc, int4* far, int32_t* nf, int far_chunk,
                           double far_z, int direct_only, double core_pad,
                           hipStream_t st);  // far: [tile][2]; nf: [2][tiles]
hipError_t launch_item_scan(const int32_t* nc, int n_tiles_total, int32_t* item_base, int* counter,
                            hipStream_t st);
hipError_t launch_gridrec(const double* nu, int64_t N, double nu_start, double dnu, int64_t n, double cut,
                          int4* grec, hipStream_t st);
hipError_t launch_span_segments(const uint32_t* keys, int64_t N, KeyMap km, double numin, double numax,
                                const PairDesc* spairs, const PairDesc* tpairs, int n_pairs, int n_spans,
                                int span_w, double cut, double far_z, const int4* tile_far, int chunk,
                                SpanSeg* segs, int32_t* nc, int direct_only, hipStream_t st);
hipError_t launch_wing(const VoigtArgs& a, int slots, int grid, hipStream_t st);
hipError_t launch_core(const VoigtArgs& a, int slots, int grid, hipStream_t st);
// k = (add ? k : 0) + fixed-order sum of the partial spans of multi-item spans
hipError_t launch_combine(const VoigtArgs& a, int slots, bool add, hipStream_t st);
hipError_t launch_cut_bounds(const double* nu, const int32_t* perm, int64_t N, double nu_start,
                             double dnu, int64_t n, double cut, int32_t* jlo, int32_t* jhi,
                             hipStream_t st);
hipError_t launch_far(const FarArgs& a, int cls, int grid, hipStream_t st);
hipError_t launch_combine_far(const FarArgs& a, hipStream_t st);
int far_max_blocks_per_cu();
int adj_max_blocks_per_cu();
// gpref of AdjArgs from dL/dk (g, n points) and the node weights w [kNodes][kAdjSpan]
// the prefix sums of one level of far units (kAdjSpan << 2 level points each) with its node weights
hipError_t launch_adj_nodes(const float* g, int64_t n, int level, const double* w, double* gpref, hipStream_t st);
hipError_t launch_adjoint(const AdjArgs& a, int grid, hipStream_t st);
hipError_t launch_reduce2(const double* contrib, int64_t N, double* partial, int n_partial, double* out,
                          hipStream_t st);
int wing_max_blocks_per_cu(int slots);
int core_max_blocks_per_cu(int slots);
hipError_t upload_weideman(const double* coef, double L);
hipError_t upload_weideman40(const double* coef, double L);
hipError_t launch_gridrec_ex(const GridRecArgs& a, hipStream_t st);
// HITRAN-style lists: field check and max |delta|, max gamma_self (ordered words); gather of the two
// extra fields into the handle's order; keys of the shifted centres; the shifted view
hipError_t launch_hitran_check(const double* gself, const double* delta, int64_t N, int* flags,
                               unsigned long long* out, hipStream_t st);
hipError_t launch_gather2(const int32_t* perm, int64_t N, const double* a, const double* b, double* oa, double* ob,
                          hipStream_t st);
hipError_t launch_shift_keys(const double* nu, const double* delta, int64_t N, double pshift, KeyMap km,
                             uint32_t* keys, int32_t* vals, hipStream_t st);
hipError_t launch_shift_gather(const ShiftArgs& a, hipStream_t st);
// k[0..n) = 0; k[0..n) += t[0..n)
hipError_t launch_fill0(float* k, int64_t n, hipStream_t st);
hipError_t launch_accumulate(float* k, const float* t, int64_t n, hipStream_t st);
// k_direct over the span work list of a (tile_lo/tile_hi/tile_nc/item_base), profile prof
hipError_t launch_direct(const VoigtArgs& a, const float* plin, int prof, int slots, int grid, hipStream_t st);
int direct_max_blocks_per_cu(int slots);
// device address of the allocation-free entry point's scratch array on the current device
hipError_t scratch_address(void** p);
// out[0..2] = ordered words of max gamma_ref, min n, max n (see ordered_to_double)
hipError_t launch_line_stats(const double* gref, const double* nexp, int64_t N, unsigned long long* out,
                             hipStream_t st);
hipError_t launch_scatter_grec(const int4* grec, const float* plin, const int32_t* perm, int64_t N, int32_t* jlo,
                               int32_t* jhi, float* plin_out, hipStream_t st);
// inverse of the kernels' order-preserving map of doubles to unsigned words
inline double ordered_to_double(unsigned long long w) {
  const unsigned long long b = (w >> 63) ? (w & 0x7FFFFFFFFFFFFFFFull) : ~w;
  double v;
  __builtin_memcpy(&v, &b, sizeof v);
  return v;
}

}  // namespace hk
