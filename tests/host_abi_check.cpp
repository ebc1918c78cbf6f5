// Host-side checks of the C ABI's argument validation, built with
// AddressSanitizer and UndefinedBehaviorSanitizer on the host code (see
// paper_2603_19600_amd/sanitize.py).  Every call here is rejected before any
// device work, so the program runs without a GPU; it exits non-zero on the
// first unexpected status and the sanitizers abort on any memory or UB error.
#include <cstdio>
#include <cstring>

#include "furax.h"

static int failures = 0;

static void expect(const char *what, furax_status got, furax_status want,
                   const char *msg_part = nullptr) {
  const char *msg = furax_last_error();
  const bool ok = got == want && msg && (!msg_part || std::strstr(msg, msg_part));
  if (!ok) {
    std::printf("FAIL %s: status %d (want %d), message '%s'\n", what, (int)got, (int)want,
                msg ? msg : "(null)");
    ++failures;
  }
}

int main() {
  const void *one = reinterpret_cast<const void *>(static_cast<uintptr_t>(1));
  if (furax_version() < 100) {
    std::printf("FAIL version %d\n", furax_version());
    ++failures;
  }
  furax_pointing P{};
  P.nside = 0;
  P.n_det = 1;
  P.n_samp = 10;
  P.dtype = FURAX_F64;
  P.theta = P.phi = P.psi = one;
  P.hwp_den = 1;
  expect("nside 0", furax_pointing_apply(&P, FURAX_F64, one, FURAX_F64, const_cast<void *>(one),
                                         nullptr), FURAX_EINVAL, "nside");
  P.nside = 16;
  P.theta = nullptr;
  expect("NULL theta", furax_pointing_apply(&P, FURAX_F64, one, FURAX_F64,
                                            const_cast<void *>(one), nullptr), FURAX_EINVAL);
  P.theta = one;
  expect("FP32 tod with FP64 pointing",
         furax_pointing_apply(&P, FURAX_F32, one, FURAX_F64, const_cast<void *>(one), nullptr),
         FURAX_EINVAL);
  P.hwp = 1;
  P.hwp_den = 0;
  double *dmap = static_cast<double *>(const_cast<void *>(one));
  expect("HWP with den 0", furax_pointing_transpose(&P, FURAX_F64, one, dmap, 0, nullptr),
         FURAX_EINVAL);
  P.hwp = 0;
  P.hwp_den = 1;
  expect("bad nside 9000", furax_ang2pix(9000, FURAX_F64, one, one, 4,
                                         reinterpret_cast<int64_t *>(const_cast<void *>(one)),
                                         nullptr), FURAX_EINVAL);

  furax_noise N{};
  N.kind = 1;
  N.n_det = 1;
  N.n_samp = 10;
  N.bandwidth = 11;                       // b > n_samp
  N.toeplitz = static_cast<const double *>(one);
  expect("band wider than the stream", furax_noise_apply(&N, FURAX_F64, one,
                                                         const_cast<void *>(one), nullptr),
         FURAX_EINVAL);
  N.n_samp = 100000;
  N.bandwidth = 8193;                     // above the supported band
  expect("band above 8192 (FP64)", furax_noise_apply(&N, FURAX_F64, one,
                                                     const_cast<void *>(one), nullptr),
         FURAX_EUNSUPPORTED);
  expect("band above 8192 (FP32)", furax_noise_apply(&N, FURAX_F32, one,
                                                     const_cast<void *>(one), nullptr),
         FURAX_EUNSUPPORTED);
  N.n_samp = 100;
  N.bandwidth = 4;
  double buf[2];
  expect("aliasing in/out", furax_noise_apply(&N, FURAX_F64, buf, buf, nullptr), FURAX_EINVAL);

  furax_noise Nd{};
  Nd.kind = 0;
  Nd.n_det = 1;
  Nd.n_samp = 10;
  Nd.inv_var = static_cast<const double *>(one);
  furax_pcg_opts opt{};
  opt.max_iter = -1;
  opt.precision = FURAX_F64;
  furax_pcg_info info{};
  expect("max_iter < 0", furax_pcg_mapmake(&P, &Nd, FURAX_F64, one, nullptr, nullptr, &opt, &info,
                                           nullptr), FURAX_EINVAL);
  expect("NULL session", furax_pcg_iterate(nullptr, 1), FURAX_EINVAL);
  expect("chi2 grad with a NULL map",
         furax_chi2_grad(&P, &Nd, FURAX_F64, nullptr, one, nullptr, dmap, nullptr, nullptr,
                         nullptr), FURAX_EINVAL);

  furax_gapfill_opts go{};
  go.max_iter = 10;
  go.rtol = -1.0;
  furax_noise Cb = N;
  Cb.n_det = 1;
  Cb.n_samp = 100;
  expect("gap fill with rtol < 0", furax_gap_fill(&Cb, FURAX_F64,
                                                  static_cast<const uint8_t *>(one), one, one,
                                                  const_cast<void *>(one), &go, nullptr, nullptr),
         FURAX_EINVAL);
  expect("gap fill with NULL covariance", furax_gap_fill(nullptr, FURAX_F64, nullptr, nullptr,
                                                         nullptr, nullptr, &go, nullptr, nullptr),
         FURAX_EINVAL);
  std::printf("%d failures\n", failures);
  return failures == 0 ? 0 : 1;
}
