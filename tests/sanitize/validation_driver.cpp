// Calls every entry point of the C ABI with invalid arguments (and with no device present) and
// checks the returned status; run under AddressSanitizer and UndefinedBehaviorSanitizer.
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "hk.h"

static int failures = 0;
#define EXPECT(call, want)                                                                      \
  do {                                                                                          \
    hk_status s_ = (call);                                                                      \
    if (s_ != (want)) {                                                                         \
      std::printf("FAIL %s -> %d (want %d): %s\n", #call, (int)s_, (int)(want), hk_last_error()); \
      ++failures;                                                                               \
    }                                                                                           \
  } while (0)
#define EXPECT_NOT_OK(call)                                                     \
  do {                                                                          \
    hk_status s_ = (call);                                                      \
    if (s_ == HK_OK) {                                                          \
      std::printf("FAIL %s returned HK_OK\n", #call);                           \
      ++failures;                                                               \
    }                                                                           \
  } while (0)

int main() {
  double buf[8] = {1, 2, 3, 4, 5, 6, 7, 8};
  float k[8];
  hk_species sp = {18.0, 296.0, 1.0, 0.05, 1.5};
  hk_species bad_sp = {-1.0, 296.0, 1.0, 0.05, 1.5};
  hk_grid g = {0.0, 0.1, 100};
  hk_grid bad_g = {0.0, -0.1, 100};
  hk_lines* L = nullptr;
  // preparation: argument checks before any device work
  EXPECT(hk_prepare_lines(buf, buf, buf, buf, buf, 8, &sp, nullptr, nullptr), HK_EINVAL);
  EXPECT(hk_prepare_lines(nullptr, buf, buf, buf, buf, 8, &sp, nullptr, &L), HK_EINVAL);
  EXPECT(hk_prepare_lines(buf, buf, buf, buf, buf, 0, &sp, nullptr, &L), HK_EINVAL);
  EXPECT(hk_prepare_lines(buf, buf, buf, buf, buf, 8, &bad_sp, nullptr, &L), HK_EINVAL);
  EXPECT(hk_prepare_lines(buf, buf, buf, buf, buf, 8, nullptr, nullptr, &L), HK_EINVAL);
  EXPECT(hk_prepare_lines_hitran(buf, buf, buf, buf, nullptr, buf, buf, 8, &sp, nullptr, &L), HK_EINVAL);
  EXPECT_NOT_OK(hk_prepare_lines(buf, buf, buf, buf, buf, 8, &sp, nullptr, &L));  // no device
  if (L != nullptr) { std::printf("FAIL handle set on failure\n"); ++failures; }
  // forward calls
  char ws[512];
  void* wsa = (void*)(((unsigned long)ws + 255) & ~255ul);
  EXPECT(hk_opacity(nullptr, nullptr, -1.0, 1.0, g, 25.0, k, wsa, 256, nullptr), HK_EINVAL);
  EXPECT(hk_opacity(nullptr, nullptr, NAN, 1.0, g, 25.0, k, wsa, 256, nullptr), HK_EINVAL);
  EXPECT(hk_opacity(nullptr, nullptr, 300.0, -1.0, g, 25.0, k, wsa, 256, nullptr), HK_EINVAL);
  EXPECT(hk_opacity(nullptr, nullptr, 300.0, 1.0, bad_g, 25.0, k, wsa, 256, nullptr), HK_EINVAL);
  EXPECT(hk_opacity(nullptr, nullptr, 300.0, 1.0, g, 0.0, k, wsa, 256, nullptr), HK_EINVAL);
  EXPECT(hk_opacity(nullptr, nullptr, 300.0, 1.0, g, NAN, k, wsa, 256, nullptr), HK_EINVAL);
  EXPECT(hk_opacity(nullptr, nullptr, 300.0, 1.0, g, 25.0, nullptr, wsa, 256, nullptr), HK_EINVAL);
  EXPECT(hk_opacity(nullptr, nullptr, 300.0, 1.0, g, 25.0, k, (char*)wsa + 8, 256, nullptr), HK_EINVAL);
  EXPECT(hk_opacity(nullptr, nullptr, 300.0, 1.0, g, 25.0, k, wsa, 256, nullptr), HK_EINVAL);  // NULL handle
  hk_options bad_o = {7, 0, 0, 0};
  EXPECT(hk_opacity_ex(nullptr, nullptr, 300.0, 1.0, g, 25.0, &bad_o, k, wsa, 256, nullptr), HK_EINVAL);
  hk_options bad_c = {0, 5, 0, 0};
  EXPECT(hk_opacity_ex(nullptr, nullptr, 300.0, 1.0, g, 25.0, &bad_c, k, wsa, 256, nullptr), HK_EINVAL);
  EXPECT(hk_opacity_noalloc(nullptr, nullptr, 300.0, 1.0, g, 25.0, nullptr, nullptr), HK_EINVAL);
  // batched: host-array checks, overlapping outputs
  double T[2] = {300.0, 400.0}, P[2] = {1.0, 2.0};
  hk_grid G[2] = {g, g};
  int64_t off[2] = {0, 50};
  EXPECT(hk_opacity_batched(nullptr, 0, T, P, G, off, 25.0, k, wsa, 256, nullptr), HK_EINVAL);
  EXPECT(hk_opacity_batched(nullptr, 2, nullptr, P, G, off, 25.0, k, wsa, 256, nullptr), HK_EINVAL);
  EXPECT(hk_opacity_batched(nullptr, 2, T, P, G, off, 25.0, k, wsa, 256, nullptr), HK_EINVAL);  // overlap
  double Tb[2] = {300.0, -4.0};
  int64_t off2[2] = {0, 100};
  EXPECT(hk_opacity_batched(nullptr, 2, Tb, P, G, off2, 25.0, k, wsa, 256, nullptr), HK_EINVAL);
  // workspace sizes, backward, HITRAN, streamed
  size_t bytes = 0;
  EXPECT(hk_workspace_size(nullptr, 3, 1, 1, &g, 25.0, &bytes), HK_EINVAL);
  EXPECT(hk_workspace_size(nullptr, 0, 2, 1, G, 25.0, &bytes), HK_EINVAL);
  EXPECT(hk_workspace_size(nullptr, 0, 1, 1, &g, 25.0, nullptr), HK_EINVAL);
  EXPECT(hk_workspace_size(nullptr, 0, 1, 1, &g, 25.0, &bytes), HK_EINVAL);  // NULL handle
  double out2[2];
  EXPECT(hk_opacity_backward(nullptr, nullptr, 300.0, 1.0, g, 25.0, nullptr, out2, nullptr, nullptr, nullptr, wsa, 256,
                             nullptr), HK_EINVAL);
  EXPECT(hk_opacity_hitran(nullptr, 300.0, 1.0, 2.0, g, 25.0, nullptr, k, wsa, 256, nullptr), HK_EINVAL);
  EXPECT(hk_workspace_size_hitran(nullptr, 300.0, 1.0, 0.5, g, 25.0, nullptr, nullptr, &bytes), HK_EINVAL);
  EXPECT(hk_opacity_stream(buf, buf, buf, buf, buf, 8, &sp, 300.0, 1.0, g, 25.0, nullptr, 0, k, nullptr), HK_EINVAL);
  EXPECT(hk_opacity_stream(nullptr, buf, buf, buf, buf, 8, &sp, 300.0, 1.0, g, 25.0, nullptr, 4, k, nullptr), HK_EINVAL);
  EXPECT(hk_release_lines(nullptr), HK_OK);
  EXPECT(hk_get_timings(nullptr), HK_EINVAL);
  hk_timings tm;
  EXPECT(hk_get_timings(&tm), HK_OK);
  EXPECT(hk_empty_cache(), HK_OK);
  std::printf("%s: %d failures\n", failures ? "FAILED" : "ok", failures);
  return failures ? 1 : 0;
}
