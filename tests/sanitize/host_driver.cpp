// Host-only driver for a sanitizer build (AddressSanitizer + UndefinedBehavior-
// Sanitizer, built with g++) of the library's host code: parameter resolution
// and NTT-table generation, the packing planner, stride maps and the argument
// checks of the C ABI.  No GPU: every kernel launcher is a stub that reports
// no device, so a context creation that passes validation ends at the device
// allocations or the key generation launch.  Test infrastructure only.
#include <cstdio>
#include <cstring>

#include "../../include/pencil.h"
#include "../../paper_2403_11166_amd/csrc/pencil_internal.h"

namespace pencil {
#define NODEV return hipErrorNoDevice
hipError_t launch_ntt_plain(uint64_t*, int64_t, bool, const Consts&, const Tables&, hipStream_t) { NODEV; }
hipError_t launch_ntt_ct(const uint64_t*, uint64_t*, int64_t, const int64_t*, const Geo&, const View&, const Consts&,
                         const Tables&, hipStream_t) { NODEV; }
hipError_t launch_ntt_pt(const int64_t*, uint64_t*, int64_t, int, const Geo&, const View&, const Consts&,
                         const Tables&, hipStream_t) { NODEV; }
hipError_t launch_ntt_ternary(uint64_t*, int64_t, uint64_t, uint64_t, uint32_t, int, const Consts&, const Tables&,
                              hipStream_t) { NODEV; }
hipError_t launch_mac(const MacArgs&, int64_t, const Geo&, const Consts&, hipStream_t) { NODEV; }
hipError_t launch_flood_mask(uint64_t*, int64_t, int64_t*, const int64_t*, const Geo&, const View&, uint64_t,
                             uint64_t, const Consts&, hipStream_t) { NODEV; }
hipError_t launch_encrypt(const uint64_t*, const int64_t*, uint64_t*, int64_t, int, const Geo&, const View&,
                          const uint64_t*, const uint64_t*, uint64_t, uint64_t, const Consts&, const Tables&,
                          hipStream_t) { NODEV; }
hipError_t launch_phase(const uint64_t*, uint64_t*, int64_t, const uint64_t*, const uint64_t*, const Consts&,
                        const Tables&, hipStream_t) { NODEV; }
hipError_t launch_decode(const uint64_t*, int64_t*, int64_t, const Geo&, const View&, const Consts&, uint32_t*,
                         hipStream_t) { NODEV; }
hipError_t launch_zt_combine(const ZtTerms&, const int64_t*, int64_t*, int64_t, const Consts&, hipStream_t) { NODEV; }
hipError_t launch_bias_grad(const int64_t*, int64_t*, int, int, int, const Consts&, hipStream_t) { NODEV; }
hipError_t launch_dp_noise(int64_t*, int64_t, double, uint64_t, uint64_t, const Consts&, hipStream_t) { NODEV; }
hipError_t launch_stride_relayout(const Relayout&, const int64_t*, int64_t*, hipStream_t) { NODEV; }
hipError_t launch_zt_corr(const int64_t*, const int64_t*, int64_t*, const Geo&, const View&, const View&, const View&,
                          const Consts&, hipStream_t) { NODEV; }
hipError_t launch_step_ntt(int, int, bool, const StepPhase&, int64_t, hipStream_t) { NODEV; }
hipError_t launch_step_mac(const StepPhase&, int64_t, int, hipStream_t) { NODEV; }
hipError_t launch_step_flood(int, const StepPhase&, int64_t, hipStream_t) { NODEV; }
hipError_t launch_set_u64(uint64_t*, uint64_t, int, hipStream_t) { NODEV; }
hipError_t launch_keygen(uint64_t*, int64_t*, uint64_t*, uint64_t*, const Consts&, const Tables&, hipStream_t) {
  NODEV;
}
hipError_t configure_lds_limits() { return hipSuccess; }
hipError_t scratch_address(int, void**) { NODEV; }
hipError_t launch_probe_mul(int, uint64_t*, int64_t, int, hipStream_t) { NODEV; }
hipError_t launch_zt_encode(const double*, int64_t*, int64_t, const Consts&, hipStream_t) { NODEV; }
hipError_t launch_zt_decode(const int64_t*, double*, int64_t, const Consts&, hipStream_t) { NODEV; }
hipError_t launch_zt_share(const int64_t*, int64_t*, int64_t*, int64_t, uint64_t, uint64_t, const Consts&, hipStream_t) {
  NODEV;
}
#undef NODEV
}  // namespace pencil

static int failures = 0;
#define EXPECT(cond)                                                   \
  do {                                                                 \
    if (!(cond)) {                                                     \
      std::fprintf(stderr, "FAILED %s:%d: %s\n", __FILE__, __LINE__, #cond); \
      ++failures;                                                      \
    }                                                                  \
  } while (0)

static bool tile_fits(const pencil_tile& t, int n) {
  return (long long)t.m * t.r * t.k * (t.oh + t.kh - 1) * (t.ow + t.kw - 1) <= n && t.m > 0 && t.r > 0 && t.k > 0;
}

int main() {
  // 1) the planner over a sweep of FC, Conv2d and Conv1d shapes and ring degrees
  int planned = 0, refused = 0;
  const int batches[] = {1, 3, 64, 128};
  const int chans[] = {1, 3, 10, 64, 256};
  const int sizes[] = {1, 5, 8, 16, 28, 32};
  for (int log2n = 10; log2n <= 14; log2n += 2)
    for (int kind = 0; kind < 3; ++kind)
      for (int b : batches)
        for (int ci : chans)
          for (int co : chans)
            for (int hw : sizes)
              for (int k = 1; k <= 5; k += 2) {
                if (kind == 0 && (hw != 1 || k != 1)) continue;
                if (kind != 0 && k > hw + 2) continue;
                pencil_layer L{kind, b, ci, co, kind == 2 ? 1 : hw, hw, k, kind == 0 ? 0 : k / 2, 1};
                pencil_plan P;
                std::memset(&P, 0, sizeof P);
                const pencil_status st = pencil_plan_auto_n((uint32_t)log2n, &L, &P);
                if (st == PENCIL_OK) {
                  ++planned;
                  EXPECT(tile_fits(P.fwd, 1 << log2n));
                  EXPECT(tile_fits(P.dx, 1 << log2n));
                  EXPECT(tile_fits(P.dw, 1 << log2n));
                  for (int op = 0; op < 3; ++op) EXPECT(P.sched[op] >= 0 && P.sched[op] < 9);
                } else {
                  ++refused;
                  EXPECT(st == PENCIL_EINVAL || st == PENCIL_EUNSUPPORTED);
                  EXPECT(pencil_last_error(nullptr) != nullptr);
                }
              }
  EXPECT(planned > 1000);
  // 2) stride maps of strided Conv2d and Conv1d layers
  for (int s = 2; s <= 3; ++s)
    for (int k = 1; k <= 5; ++k)
      for (int kind = 1; kind <= 2; ++kind) {
        pencil_layer L{kind, 4, 3, 5, kind == 2 ? 1 : 28, 28, k, k / 2, s}, E;
        const pencil_status st = pencil_stride_map(&L, &E);
        EXPECT(st == PENCIL_OK);
        if (st == PENCIL_OK) EXPECT(E.stride <= 1 && E.c_in == 3 * (kind == 2 ? s : s * s));
      }
  EXPECT(pencil_stride_map(nullptr, nullptr) == PENCIL_EINVAL);
  // 3) parameter validation, then table generation (host), then the first
  //    device call, which fails without a GPU (or succeeds on a GPU host)
  pencil_ctx* ctx = nullptr;
  EXPECT(pencil_ctx_create(nullptr, &ctx) == PENCIL_EINVAL);
  pencil_params bad[6];
  std::memset(bad, 0, sizeof bad);
  bad[0].log2_n = 9, bad[0].num_limbs = 2, bad[0].prime_bits = 50;   // N too small
  bad[1].log2_n = 13, bad[1].num_limbs = 5, bad[1].prime_bits = 60;  // too many limbs
  bad[2].log2_n = 13, bad[2].num_limbs = 3, bad[2].prime_bits = 61;  // primes too large
  bad[3].log2_n = 13, bad[3].num_limbs = 1, bad[3].primes[0] = 97;   // not 1 mod 2N
  bad[4].log2_n = 13, bad[4].num_limbs = 2, bad[4].prime_bits = 60, bad[4].t = 12;  // t not prime
  bad[5].log2_n = 12, bad[5].num_limbs = 1, bad[5].prime_bits = 40;  // q / t leaves no noise budget
  for (auto& p : bad) {
    EXPECT(pencil_ctx_create(&p, &ctx) == PENCIL_EINVAL);
    EXPECT(ctx == nullptr);
    EXPECT(std::strlen(pencil_last_error(nullptr)) > 0);
  }
  const uint32_t shapes[][3] = {{12, 2, 50}, {13, 3, 60}, {14, 4, 60}};
  for (auto& sh : shapes) {
    pencil_params p;
    std::memset(&p, 0, sizeof p);
    p.log2_n = sh[0], p.num_limbs = sh[1], p.prime_bits = sh[2], p.seed = 7;
    const pencil_status st = pencil_ctx_create(&p, &ctx);
    EXPECT(st == PENCIL_EHIP || st == PENCIL_ENOMEM || st == PENCIL_OK);
    if (st == PENCIL_OK) pencil_ctx_destroy(ctx);
  }
  // 4) calls on NULL handles are rejected before any device work
  EXPECT(pencil_layout(nullptr, nullptr, nullptr, nullptr) == PENCIL_EINVAL);
  EXPECT(pencil_decrypt_checked(nullptr, nullptr, nullptr, 0, nullptr, nullptr, nullptr, nullptr, nullptr) ==
         PENCIL_EINVAL);
  EXPECT(pencil_step_create(nullptr, nullptr, nullptr, 0, 7, nullptr) == PENCIL_EINVAL);
  EXPECT(pencil_ctx_destroy(nullptr) == PENCIL_OK);
  std::printf("planned %d layers (%d refused); %d failures\n", planned, refused, failures);
  return failures ? 1 : 0;
}
