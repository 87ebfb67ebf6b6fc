// Host-code checks of libbfvec's C entry points that need no device (built by
// tests/test_sanitizers.py with g++ under AddressSanitizer and
// UndefinedBehaviorSanitizer): whitening in every mode, the term draws, the
// order rule, the spatial taps, and their error paths.  Prints one PASS line
// per group; any mismatch prints FAIL and exits nonzero.

#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "bfvec.h"
#include "host.h"

static int failures = 0;

static void check(bool ok, const char* what) {
  if (!ok) {
    std::printf("FAIL %s\n", what);
    ++failures;
  }
}

// random SPD matrix A A^T + d I (row-major)
static std::vector<double> spd(int d, std::mt19937& g) {
  std::normal_distribution<double> n(0.0, 1.0);
  std::vector<double> A(d * d), C(d * d, 0.0);
  for (double& a : A) a = n(g);
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      double s = i == j ? d : 0.0;
      for (int k = 0; k < d; ++k) s += A[i * d + k] * A[j * d + k];
      C[i * d + j] = s;
    }
  return C;
}

int main() {
  std::mt19937 g(7);
  // whitening: W^T W C = I in every mode
  for (int d = 1; d <= 8; ++d)
    for (int mode = 0; mode < 3; ++mode) {
      const std::vector<double> C = spd(d, g);
      std::vector<double> W(d * d);
      check(bf_whiten_mode(d, C.data(), mode, W.data()) == BF_OK, "whiten status");
      double err = 0.0;
      for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
          double s = 0.0;   // (W^T W C)_ij
          for (int k = 0; k < d; ++k) {
            double wtw = 0.0;
            for (int m = 0; m < d; ++m) wtw += W[m * d + i] * W[m * d + k];
            s += wtw * C[k * d + j];
          }
          err = std::fmax(err, std::fabs(s - (i == j ? 1.0 : 0.0)));
        }
      check(err < 1e-10, "W^T W C = I");
    }
  {
    const double bad[4] = {1.0, 2.0, 2.0, 1.0};
    double W[4];
    for (int mode = 0; mode < 3; ++mode)
      check(bf_whiten_mode(2, bad, mode, W) == BF_ENOTSPD, "indefinite C rejected");
    check(bf_whiten_mode(2, bad, 7, W) == BF_EINVAL, "unknown mode rejected");
    check(bf_whiten(9, bad, W) == BF_EINVAL, "d = 9 rejected");
    check(bf_whiten(2, nullptr, W) == BF_EINVAL, "null C rejected");
  }
  std::printf("PASS whitening\n");

  // draws: Y = N - 2X with X in [0, N], same parity as N; w = W^T Y / sqrt(N)
  for (int d = 1; d <= 8; ++d) {
    const std::vector<double> C = spd(d, g);
    for (int N : {1, 10, 37, 1000}) {
      const int K = 33;
      std::vector<int32_t> Y(K * d);
      std::vector<double> w(K * d), W(d * d);
      check(bf_sample_terms(d, C.data(), N, K, 12345u + d, BF_WHITEN_EIG, Y.data(), w.data()) ==
                BF_OK,
            "sample status");
      check(bf_whiten(d, C.data(), W.data()) == BF_OK, "whiten");
      for (int t = 0; t < K; ++t)
        for (int j = 0; j < d; ++j) {
          const int y = Y[t * d + j];
          check(y >= -N && y <= N && ((N - y) % 2) == 0, "Y range and parity");
          double s = 0.0;
          for (int k = 0; k < d; ++k) s += Y[t * d + k] * W[k * d + j];
          check(std::fabs(s / std::sqrt((double)N) - w[t * d + j]) <= 1e-12 * (1.0 + std::fabs(s)),
                "w = W^T Y / sqrt(N)");
        }
    }
  }
  check(bf_sample_terms(3, nullptr, 10, 4, 1, BF_WHITEN_EIG, nullptr, nullptr) == BF_EINVAL ||
            bf_sample_terms(3, nullptr, 10, 4, 1, BF_WHITEN_EIG, nullptr, nullptr) == BF_ENOTSPD,
        "null C rejected by the sampler");
  {
    const double C[4] = {1.0, 0.3, 0.3, 2.0};
    check(bf_sample_terms(2, C, 10, 4, 1, 3, nullptr, nullptr) == BF_EINVAL,
          "unknown whitening mode rejected by the sampler");
  }
  std::printf("PASS draws\n");

  // order rule: pi sqrt(N) >= T + 4 with N minimal and at least 10
  {
    // C = 0.01 I: W = 10 I in every whitening mode
    const double C[9] = {0.01, 0, 0, 0, 0.01, 0, 0, 0, 0.01};
    const float lo[3] = {0, 0, 0}, hi[3] = {1, 0.5f, 0.25f};
    int N = 0;
    check(bf_choose_N(3, C, lo, hi, BF_WHITEN_EIG, &N) == BF_OK, "choose_N status");
    const double T = 10.0;   // max_k sum_m |W_km| (hi - lo)_m
    check(M_PI * std::sqrt((double)N) >= T + 4 && (N == 10 || M_PI * std::sqrt(N - 1.0) < T + 4),
          "order rule");
  }
  std::printf("PASS order\n");

  // spatial taps: sums (2r+1)^n for boxes; the Gaussian's centre tap is 1
  for (int n = 1; n <= 3; ++n)
    for (double s : {0.0, 0.7, 2.0, 5.5, 10.0}) {
      const std::vector<double> t = bfvec::spatial_taps(s, n);
      const int r = bfvec::box_radius(s, n);
      check((int)t.size() == 2 * n * r + 1, "box taps length");
      double sum = 0.0;
      for (double v : t) sum += v;
      check(sum == std::pow(2.0 * r + 1.0, n), "box taps sum");
    }
  for (double s : {0.0, 1.0, 10.0}) {
    const std::vector<double> t = bfvec::spatial_taps(s);
    check(t[t.size() / 2] == 1.0 && (int)t.size() == 2 * bfvec::window_radius(s) + 1,
          "gaussian taps");
  }
  std::printf("PASS taps\n");

  // FP16 storage range: max(1, max_m |f_m - c_m|) * sum(omega_1) <= 32768
  {
    double sw = 0.0;   // sigma_s = 10: sum of the 61 Gaussian taps, about 25.07
    for (double v : bfvec::spatial_taps(10.0)) sw += v;
    const float lo[3] = {0.0f, -5.0f, 0.0f}, hi[3] = {1.0f, 5.0f, 0.0f};
    const float mid[3] = {0.5f, 0.0f, 0.0f}, zero[3] = {0.0f, 0.0f, 0.0f};
    check(bfvec::check_fp16_range(3, 10.0, 0, lo, hi, mid) == BF_OK, "fp16 range: unit data");
    const float big_lo[1] = {0.0f}, big_hi[1] = {2000.0f};
    const float c1000[1] = {1000.0f};
    check(1000.0 * sw < bfvec::kFP16Limit && 2000.0 * sw > bfvec::kFP16Limit, "fp16 range: setup");
    check(bfvec::check_fp16_range(1, 10.0, 0, big_lo, big_hi, c1000) == BF_OK,
          "fp16 range: centred 2000-wide channel fits");
    check(bfvec::check_fp16_range(1, 10.0, 0, big_lo, big_hi, zero) == BF_EUNSUPPORTED,
          "fp16 range: the same channel uncentred is refused");
    const float wide_hi[1] = {3000.0f}, c1500[1] = {1500.0f};
    check(bfvec::check_fp16_range(1, 10.0, 0, big_lo, wide_hi, c1500) == BF_EUNSUPPORTED,
          "fp16 range: a 3000-wide channel is refused at sigma_s = 10");
    // sigma_s = 0: one tap of weight 1, so |f - c| up to 32768 fits
    const float h2[1] = {60000.0f}, c2[1] = {30000.0f};
    check(bfvec::check_fp16_range(1, 0.0, 0, big_lo, h2, c2) == BF_OK, "fp16 range: identity");
  }
  std::printf("PASS fp16 range\n");
  return failures ? 1 : 0;
}
