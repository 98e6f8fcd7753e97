/*
 * hk.h -- C ABI of the MI355X (gfx950) line-by-line opacity library.
 *
 * The library computes the hot path of the line-by-line opacity method of
 * HELIOS-K 2.0 (Grimm et al. 2021, arXiv:2101.02005):
 *
 *   k(nu_j) = sum over lines i with |nu_j - nu_i| <= cut of S_i(T) V(nu_j - nu_i; alpha_i, gamma_i)
 *
 *   S_i(T)  line strength at T: eq. (S) in the form of eq. (S1) (Sec. 2.2.2, Sec. 2.4.3
 *           step 1); from the strength S_ref at T_ref it is
 *           S_ref Q(T_ref)/Q(T) exp(c2 E''(1/T_ref - 1/T)) (1 - e^{-c2 nu/T})/(1 - e^{-c2 nu/T_ref}),
 *           with Q(T) = q_a T^q_b and c2 = h c / k_B.
 *   alpha_i Doppler width without the sqrt(ln 2) factor, the inverse of eq. (alphaD):
 *           alpha = (nu/c) sqrt(2 k_B T / m).
 *   gamma_i Lorentz half-width, ExoMol form of Sec. 2.2 without the natural term:
 *           gamma = gamma_ref (T_ref/T)^n (P/P_ref).
 *   V       unit-area Voigt profile Re w((d + i gamma)/alpha) / (sqrt(pi) alpha), w the
 *           Faddeeva function (Sec. 2.2.3, Sec. 2.4.2 parameters x and y).
 *   grid    nu_j = nu_start + j dnu, 0 <= j < n (uniform resolution, Sec. 2.4.2 eq. x).
 *   cut     fixed cutting length in cm^-1, inclusive (Sec. 2.4.3 step 4); +INFINITY: none.
 *
 * Units: nu, dnu, cut, E'' in cm^-1; S_ref in cm/molecule at T_ref; gamma_ref in
 * cm^-1 atm^-1; T in K; P in atm; k in cm^2/molecule (the paper's cm^2/g is k/m).
 *
 * Conventions shared by every entry point:
 *  - Array arguments are DEVICE pointers unless the comment says "host". Inputs and
 *    outputs belong to the caller; the library never frees them.
 *  - All arguments are validated on the host before any device work. A rejected call
 *    returns HK_EINVAL and leaves every output untouched. Device failures return
 *    HK_EDEVICE. hk_last_error() gives a thread-local message for the last failure.
 *  - Work is enqueued on the caller's stream. hk_opacity, hk_opacity_batched and
 *    hk_opacity_backward do not synchronize the host, except for the first call with a
 *    new tuning key when autotuning is enabled (HK_AUTOTUNE=1), and for building the
 *    graph of a new batched configuration (documented below).
 *  - Results are bitwise deterministic for a fixed tuning (no floating-point atomics;
 *    all sums run in a fixed order). hk_get_timings() reports the tuning used.
 *  - Calls on different streams with distinct workspaces may overlap.
 *  - No C++ exception crosses this interface.
 */
#ifndef HK_H
#define HK_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum hk_status {
  HK_OK = 0,
  HK_EINVAL = 1,        /* invalid argument (nothing was launched, outputs untouched) */
  HK_ENOMEM = 2,        /* device or host allocation failed, or a size overflowed */
  HK_EDEVICE = 3,       /* a HIP call failed (message in hk_last_error) */
  HK_EUNSUPPORTED = 4   /* the current device is not gfx950 */
} hk_status;

/* Species constants. Q(T) = q_a T^q_b. */
typedef struct hk_species {
  double mass_amu;   /* molecular mass [amu], > 0 */
  double T_ref;      /* reference temperature of S_ref and gamma_ref [K], > 0 */
  double P_ref_atm;  /* reference pressure of gamma_ref [atm], > 0 */
  double q_a, q_b;   /* partition function coefficients, q_a > 0 */
} hk_species;

/* Uniform grid nu_j = nu_start + j*dnu, 0 <= j < n (dnu > 0, 0 <= n < 2^31). */
typedef struct hk_grid {
  double nu_start, dnu;
  int64_t n;
} hk_grid;

/* Optional per-line replacements (device, caller's line order, length n_lines; any may be
 * NULL). Used by automatic differentiation to evaluate with the current parameters without
 * re-binning. */
typedef struct hk_line_override {
  const double* S_ref;
  const double* gamma_ref;
  const double* n_exp;
} hk_line_override;

/* Opaque handle: the line list binned by wavenumber (device copies sorted by nu-bin,
 * stable within a bin), the permutation to the caller's order, and the species. */
typedef struct hk_lines hk_lines;

/* Timings and tuning of the last completed call on this thread (milliseconds, filled only
 * when HK_TIMING=1 is set in the environment; otherwise the times are negative).
 * hk_opacity: voigt_ms is the wing kernel (spans), far_ms the tile-far pass (lines far from a whole
 * tile, evaluated at its Chebyshev nodes and interpolated), core_ms the line-core kernel,
 * core_evals the number of (line, point) evaluations the core kernel made. hk_opacity_batched: voigt_ms is
 * the whole graph. hk_opacity_backward: backward_ms. */
typedef struct hk_timings {
  double prep_ms, worklist_ms, voigt_ms, combine_ms, backward_ms, bin_ms;
  int32_t tile_width;      /* grid points per span (one wave of the wing pass; 64 slots) */
  int32_t lines_per_batch; /* lines a wave stages in LDS per batch */
  int32_t chunk_lines;     /* lines per work item of a heavy tile */
  int32_t n_items;         /* upper bound of work items of the last call */
  double core_ms;
  int64_t core_evals;
  double far_ms;           /* tile-far pass (node evaluation and interpolation) */
  int64_t wing_evals;      /* profile evaluations the wing and tile-far passes made: every
                              point of a wave for a line evaluated directly, 16 per line
                              evaluated at the Chebyshev nodes of a wave span or a tile */
  int64_t class_evals[8];  /* the same per evaluation class: [0] lines evaluated at every point
                              of a span (wing pass, or the direct pass of the options path),
                              [1] far lines at a span's 16 nodes, [2] very far lines at its 8
                              nodes, [3] middle-distance lines at its 32 nodes, [4] lines with a
                              cut bound on the span at its 6 nodes, [5] and [6] tile-far lines at
                              a tile's 16 and 8 nodes, [7] core evaluations */
  int32_t status;          /* status word of the last timed call (0: every work item stored) */
  int64_t backward_evals;  /* profile evaluations the last timed hk_opacity_backward made: every
                              point of a line's direct spans, 16 per far unit of 256, 1024 or
                              4096 points (each with the profile and its two width derivatives) */
} hk_timings;

/* Options of hk_opacity_ex / hk_opacity_batched_ex (NULL: all zero).
 *   profile  : the line profile (Sec. 2.1): HK_PROFILE_VOIGT (default); HK_PROFILE_LORENTZ,
 *              gamma/(pi (d^2 + gamma^2)); HK_PROFILE_DOPPLER, exp(-(d/alpha)^2)/(sqrt(pi) alpha);
 *              HK_PROFILE_BINNED_GAUSS, the Doppler profile averaged over each grid bin (the
 *              integrated cross section of the bin over its width; Sec. 2.1 and the comparison
 *              with ExoCross in Sec. 3.2): (erf((d + dnu/2)/alpha) - erf((d - dnu/2)/alpha))/(2 dnu).
 *   cut_mode : HK_CUT_FIXED, cutoff is the cutting length in cm^-1 (default); HK_CUT_DOPPLER,
 *              each line's cutting length is cutoff x its Doppler half-width sqrt(ln 2) alpha;
 *              HK_CUT_LORENTZ, cutoff x its Lorentz half-width gamma (Sec. 2.4.3 step 4).
 *              Per-line lengths are decided in FP64 as alpha = (nu/c) sqrt(2 k_B T/m),
 *              gamma = gamma_ref (T_ref/T)^n P/P_ref. The first HK_CUT_LORENTZ call on a handle
 *              reads back the list's largest gamma_ref and range of n (one host synchronization),
 *              and such calls reject an override of gamma_ref or n (HK_EUNSUPPORTED).
 *   plinth   : 1 subtracts each line's own profile value at its cutting length from every point
 *              inside its cut (plinth removal, Sec. 2.1.1); needs a finite cut.
 *   direct   : 1 makes the default path (Voigt, fixed cut, no plinth) evaluate every (line,
 *              point) pair inside the cut: lines far from a span or a tile are then not evaluated
 *              at its Chebyshev nodes and interpolated. For measurement of the per-pair rate.
 * Any option other than the default Voigt with a fixed cut and no plinth runs a direct pass that
 * evaluates every (line, point) pair inside each line's own cut in FP32 with compensated sums
 * (the Voigt core points, |z| < 6.75, go to the core pass). */
enum { HK_PROFILE_VOIGT = 0, HK_PROFILE_LORENTZ = 1, HK_PROFILE_DOPPLER = 2, HK_PROFILE_BINNED_GAUSS = 3 };
enum { HK_CUT_FIXED = 0, HK_CUT_DOPPLER = 1, HK_CUT_LORENTZ = 2 };
typedef struct hk_options {
  int32_t profile;
  int32_t cut_mode;
  int32_t plinth;
  int32_t direct;
} hk_options;

/*
 * hk_prepare_lines -- bin a line list by wavenumber (the paper sorts the line quantities
 * along nu, Sec. 2.4.3 step 3). Stable counting (radix) sort on a 24-bit linear bin key,
 * then a gather of the five fields into sorted device arrays owned by the handle.
 *
 *   nu, S_ref, E_low, gamma_ref, n_exp : device, float64[n_lines], caller order.
 *       nu > 0 and finite; S_ref >= 0 finite; E_low finite; gamma_ref >= 0 finite;
 *       n_exp finite. Checked on the device; a violation returns HK_EINVAL.
 *   n_lines : 1 <= n_lines < 2^31.
 *   sp      : host pointer, validated (all fields finite, mass, T_ref, P_ref, q_a > 0).
 *   stream  : work is ordered on this stream; the call blocks the host twice: after the
 *             first pass (nu checked, its range read back for the bin key) and at the end
 *             (the other fields' check, made while the records are copied for the sort).
 *   out     : host pointer receiving the handle (set only on HK_OK).
 * Memory: about 56 bytes per line are held by the handle (+ 24 temporary).
 */
hk_status hk_prepare_lines(const double* nu, const double* S_ref, const double* E_low,
                           const double* gamma_ref, const double* n_exp, int64_t n_lines,
                           const hk_species* sp, hipStream_t stream, hk_lines** out);

/* Release a handle; blocks until the work issued through it has completed (the last call on each
 * stream it was used on; the whole device only when a use could not be tracked: a call on a
 * capturing stream, on more than 8 streams, or an allocation-free call on a new stream). Other
 * work on the device is not waited for. NULL is accepted. The handle's device block goes to the library's block cache (see
 * hk_empty_cache), not back to the driver. */
hk_status hk_release_lines(hk_lines* lines);

/* The library keeps the device blocks of released handles and of hk_prepare_lines' temporaries
 * for reuse by later hk_prepare_lines calls of about the same size on the same device (at most
 * 8 blocks and 128 GiB; the oldest go back first). Memory that another process freed can be
 * cleared by the driver when it is allocated again, which would otherwise be paid on every
 * prepare. A hipMalloc that fails empties the device's cache and is tried again. This call
 * returns every cached block to the driver (all devices); HK_NO_CACHE=1 in the environment
 * turns the cache off. The cache is shared by all threads and holds only blocks whose work has
 * completed, so this call is safe at any time. Returns HK_OK. */
hk_status hk_empty_cache(void);

/* Number of lines held by a handle (host). */
int64_t hk_lines_count(const hk_lines* lines);

/*
 * hk_workspace_size -- bytes of device workspace needed by a call.
 *   mode 0: hk_opacity (n_pairs must be 1, grids = &grid)
 *   mode 1: hk_opacity_batched (n_pairs pairs, grids[n_pairs] host array; n_temps distinct
 *           temperatures, pass n_pairs if unknown: it is an upper bound)
 *   mode 2: hk_opacity_backward (n_pairs = 1; grows with the line count and with the grid:
 *           per line 80 B, per grid point 384 B of node sums of dL/dk, three unit widths)
 * The workspace must be 256-byte aligned. Returns HK_EINVAL for bad arguments.
 */
hk_status hk_workspace_size(const hk_lines* lines, int mode, int32_t n_pairs, int32_t n_temps,
                            const hk_grid* grids, double cutoff, size_t* bytes);

/*
 * hk_opacity -- k on one grid at one (T, P).
 *   T > 0, P_atm >= 0 finite; grid valid; cutoff > 0 (finite or +INFINITY).
 *   ovr : host pointer or NULL (per-line replacements, see hk_line_override).
 *   k   : device float32[grid.n], written entirely (points no line reaches get 0).
 *   ws  : device workspace of at least hk_workspace_size(mode 0) bytes.
 * Precision: S(T), widths, line-centre offsets and cut bounds in FP64; the profile and the
 * per-point sums in FP32 with compensated (Kahan) accumulation; k stored as FP32.
 */
hk_status hk_opacity(const hk_lines* lines, const hk_line_override* ovr, double T, double P_atm,
                     hk_grid grid, double cutoff, float* k, void* ws, size_t ws_bytes,
                     hipStream_t stream);

/*
 * hk_opacity_batched -- k for many (T, P) pairs in one persistent launch (the paper's
 * several pressures per run, Sec. 3.5 and Table timing2, extended to temperatures).
 *   n_pairs >= 1; T, P_atm : host float64[n_pairs]; grids : host hk_grid[n_pairs] (may
 *   differ per pair); out_offset : host int64[n_pairs], pair p writes
 *   k[out_offset[p] .. out_offset[p] + grids[p].n). Output ranges must not overlap.
 *   Pairs with equal T share one strength/width pass.
 * The call records its kernels in a hipGraph on first use of a configuration (argument
 * values and pointers) and replays the cached graph afterwards; building the graph blocks
 * the host once. Set HK_GRAPH=0 to launch without a graph.
 */
hk_status hk_opacity_batched(const hk_lines* lines, int32_t n_pairs, const double* T,
                             const double* P_atm, const hk_grid* grids, const int64_t* out_offset,
                             double cutoff, float* k, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * hk_opacity_ex, hk_opacity_batched_ex -- hk_opacity and hk_opacity_batched with options (see
 * hk_options; NULL: the defaults). With a width-multiple cut mode, cutoff is the multiple.
 * The workspace must hold hk_workspace_size_ex bytes for the same arguments.
 */
hk_status hk_opacity_ex(const hk_lines* lines, const hk_line_override* ovr, double T, double P_atm,
                        hk_grid grid, double cutoff, const hk_options* options, float* k, void* ws,
                        size_t ws_bytes, hipStream_t stream);
hk_status hk_opacity_batched_ex(const hk_lines* lines, int32_t n_pairs, const double* T,
                                const double* P_atm, const hk_grid* grids, const int64_t* out_offset,
                                double cutoff, const hk_options* options, float* k, void* ws,
                                size_t ws_bytes, hipStream_t stream);
/* Workspace bytes of hk_opacity_ex (mode 0, n_pairs 1) or hk_opacity_batched_ex (mode 1): T and
 * P_atm are host arrays of n_pairs (needed for width-multiple cut modes, which size the work
 * lists by the largest cutting length; may be NULL otherwise); stream orders the one-time read
 * of the list's width statistics (HK_CUT_LORENTZ). */
hk_status hk_workspace_size_ex(const hk_lines* lines, int mode, int32_t n_pairs, const double* T,
                               const double* P_atm, const hk_grid* grids, double cutoff,
                               const hk_options* options, hipStream_t stream, size_t* bytes);

/*
 * HITRAN-style lists: air and self broadening and the pressure shift of line centres.
 *
 * hk_prepare_lines_hitran -- as hk_prepare_lines, with the Lorentz half-width of eq. (gammaL)
 * (Sec. 2.2, without the natural term A/(4 pi c)) in place of the ExoMol form,
 *   gamma = (T_ref/T)^n [gamma_air (P - P_self) + gamma_self P_self] / P_ref,
 * and line centres moved by the pressure shift of Table binary2, nu* = nu + delta_air P/P_ref.
 * The strength and the Doppler width keep the transition wavenumber nu.
 *   gamma_air, gamma_self : device float64[n_lines], >= 0 and finite (cm^-1 atm^-1)
 *   delta_air             : device float64[n_lines], finite (cm^-1 atm^-1)
 * Other arguments, checks and memory as hk_prepare_lines (plus 16 bytes per line); the call
 * blocks the host once more (the check of the two extra fields).
 *
 * hk_opacity_hitran -- k on one grid at (T, P) with self partial pressure 0 <= P_self <= P. The
 * shift can change the order of the centres along nu (the paper sorts after applying it, Sec.
 * 2.4.3 step 3), so each call bins the list again by nu* in its workspace, then evaluates every
 * (line, point) pair inside each line's cut (the direct pass of the options path; the Voigt core
 * points by the core pass). options as hk_opacity_ex (direct must be 0); the workspace must
 * hold hk_workspace_size_hitran bytes (about 68 bytes per line more than hk_opacity_ex).
 */
hk_status hk_prepare_lines_hitran(const double* nu, const double* S_ref, const double* E_low,
                                  const double* gamma_air, const double* gamma_self, const double* n_exp,
                                  const double* delta_air, int64_t n_lines, const hk_species* sp,
                                  hipStream_t stream, hk_lines** out);
hk_status hk_workspace_size_hitran(const hk_lines* lines, double T, double P_atm, double P_self,
                                   hk_grid grid, double cutoff, const hk_options* options, hipStream_t stream,
                                   size_t* bytes);
hk_status hk_opacity_hitran(const hk_lines* lines, double T, double P_atm, double P_self, hk_grid grid,
                            double cutoff, const hk_options* options, float* k, void* ws, size_t ws_bytes,
                            hipStream_t stream);

/*
 * hk_opacity_stream -- k of a line list held in HOST memory, larger than the device can hold
 * at once, processed in chunks of chunk_lines lines (the paper streams blocks of the list from
 * host memory to the GPU, overlapping the transfers with the computation, Sec. 2.4.1 and
 * Sec. 2.4.6 with Fig. stream). While one chunk is binned and evaluated on `stream`, the next
 * is copied on a copy stream of the library. Each chunk is evaluated on the band of the grid
 * within its largest cutting length of its lines (for a list sorted along nu, as the paper's
 * preprocessed files are, a band is a small part of the grid), and the chunk results are added
 * to k in chunk order, so the result is deterministic for a given chunk_lines and equals the
 * one-call result up to FP32 rounding of those additions.
 *   nu, S_ref, E_low, gamma_ref, n_exp : HOST float64[n_lines] (pinned memory lets the copies
 *       overlap the computation); checked per chunk as in hk_prepare_lines.
 *   chunk_lines : >= 1; device memory used is about (56 + 80) bytes per chunk line plus the
 *       workspace of one chunk's hk_opacity_ex and 4 bytes per grid point, from the library's
 *       block cache (this entry point allocates; it is not for graph capture).
 *   options : as hk_opacity_ex. k : device float32[grid.n], written entirely.
 * The call returns when k is complete (it synchronizes `stream`).
 */
hk_status hk_opacity_stream(const double* nu, const double* S_ref, const double* E_low,
                            const double* gamma_ref, const double* n_exp, int64_t n_lines,
                            const hk_species* sp, double T, double P_atm, hk_grid grid, double cutoff,
                            const hk_options* options, int64_t chunk_lines, float* k, hipStream_t stream);

/*
 * hk_opacity_noalloc -- hk_opacity without a workspace argument, for callers that cannot
 * allocate device memory (code under graph capture, tight serving loops). The workspace is a
 * fixed device array of the library (hk_noalloc_max_bytes() bytes, held on each device the
 * library runs on until the process ends); the call performs no device or host allocation.
 * A problem whose workspace (hk_workspace_size mode 0 for the tuning in use) exceeds it returns
 * HK_ENOMEM before any launch. Every call on a device shares that device's array: calls that
 * overlap in time on one device (different streams, or different threads) race and must be
 * serialized by the caller. Arguments, results and determinism as hk_opacity. Its work is
 * tracked by hk_release_lines only on streams the handle has already been used on with another
 * entry point; otherwise release waits for the whole device.
 */
hk_status hk_opacity_noalloc(const hk_lines* lines, const hk_line_override* ovr, double T, double P_atm,
                             hk_grid grid, double cutoff, float* k, hipStream_t stream);
size_t hk_noalloc_max_bytes(void);

/*
 * hk_opacity_backward -- adjoint of L = sum_j dL_dk[j] k_j at one (T, P) (not in the paper;
 * derived from eqs. S1, alphaD and the ExoMol width). Strengths and widths are recomputed.
 *   dL_dk     : device float32[grid.n] upstream gradient.
 *   dL_dT_lnP : device float64[2] receives dL/dT and dL/d(ln P).
 *   dL_dSref  : device float64[n_lines], caller order (FP64: S(T)/S_ref spans beyond FP32).
 *   dL_dgref, dL_dn : device float32[n_lines], caller order. Any of the three may be NULL.
 *   The cut indicator is not differentiated (the cut is fixed in cm^-1).
 */
hk_status hk_opacity_backward(const hk_lines* lines, const hk_line_override* ovr, double T,
                              double P_atm, hk_grid grid, double cutoff, const float* dL_dk,
                              double* dL_dT_lnP, double* dL_dSref, float* dL_dgref, float* dL_dn,
                              void* ws, size_t ws_bytes, hipStream_t stream);

/* Per-line cut bounds of the last prepared grid, for tests: writes for every line (caller
 * order) the inclusive grid range [j_lo, j_hi] of |nu_j - nu_i| <= cut (j_hi < j_lo: empty).
 * j_lo, j_hi: device int32[n_lines]. */
hk_status hk_debug_cut_bounds(const hk_lines* lines, hk_grid grid, double cutoff, int32_t* j_lo,
                              int32_t* j_hi, hipStream_t stream);

/* Per-line grid records of a call with options, for tests: the inclusive grid range [j_lo, j_hi]
 * of each line's own cutting length and its plinth S(T) f(cut) (0 without plinth removal), in
 * caller order (device int32/float32 arrays of n_lines, any may be NULL). ws: device scratch of
 * at least 28 n_lines + 768 bytes, 256-byte aligned. */
hk_status hk_debug_grid_records(const hk_lines* lines, double T, double P_atm, hk_grid grid, double cutoff,
                                const hk_options* options, void* ws, size_t ws_bytes, int32_t* j_lo,
                                int32_t* j_hi, float* plinth, hipStream_t stream);

/* Sorted view for tests: copies the handle's bin keys (uint32) and permutation (int32:
 * sorted position -> caller index) to device buffers of n_lines elements. */
hk_status hk_debug_sorted(const hk_lines* lines, uint32_t* keys, int32_t* perm, hipStream_t stream);

/* Per-line strength and widths at (T, P) in caller order (device float64 arrays of
 * n_lines; any may be NULL): S(T), alpha, gamma, as the kernels use them. */
hk_status hk_debug_line_params(const hk_lines* lines, double T, double P_atm, double* S_T,
                               double* alpha, double* gamma, hipStream_t stream);

hk_status hk_get_timings(hk_timings* out);
const char* hk_last_error(void);
const char* hk_version(void);

#ifdef __cplusplus
}
#endif
#endif /* HK_H */
