// Host-side FP64 logic of libbfvec: validation, whitening (eq. (COB)),
// Philox draws (Proposition 2), the order rule and the spatial taps.
// No HIP calls: these functions run on any machine.

#include "host.h"

#include <algorithm>
#include <cmath>
#include <cstring>

#include "bfvec.h"

namespace bfvec {

namespace {
thread_local std::string g_error;
}

void set_error(const std::string& msg) { g_error = msg; }
void clear_error() { g_error.clear(); }

int fail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}

int box_radius(double sigma_s, int n) {
  const double x = (std::sqrt(12.0 * sigma_s * sigma_s / n + 1.0) - 1.0) / 2.0;
  return (int)std::floor(x + 0.5);
}

int window_radius(double sigma_s, int spatial) {
  if (spatial > 0) return spatial * box_radius(sigma_s, spatial);
  if (sigma_s == 0.0) return 0;
  return (int)std::ceil(3.0 * sigma_s);
}

std::vector<double> spatial_taps(double sigma_s, int spatial) {
  if (spatial > 0) {
    // repeated convolution with a box of 2r+1 ones, in integers (exact)
    const int r = box_radius(sigma_s, spatial);
    std::vector<long long> c(1, 1);
    for (int k = 0; k < spatial; ++k) {
      std::vector<long long> nc(c.size() + 2 * r, 0);
      for (size_t i = 0; i < c.size(); ++i)
        for (int j = 0; j <= 2 * r; ++j) nc[i + j] += c[i];
      c.swap(nc);
    }
    return std::vector<double>(c.begin(), c.end());
  }
  const int R = window_radius(sigma_s);
  std::vector<double> t(2 * R + 1, 1.0);
  if (R == 0) return t;
  for (int u = -R; u <= R; ++u)
    t[u + R] = std::exp(-((double)u * (double)u) / (2.0 * sigma_s * sigma_s));
  return t;
}

// ---------------------------------------------------------------------------
// Whitening.  C = V diag(lambda) V^T by the cyclic Jacobi method; row k of W
// is q_k^T / sqrt(lambda_k) so that W^T W = C^{-1} and (W x)_k = alpha_k y_k
// with y = Q^T x (eq. (COB)).
// ---------------------------------------------------------------------------

namespace {

// Symmetric eigen-decomposition of the n x n matrix A (row-major, destroyed).
// On return the diagonal of A holds the eigenvalues and column k of V the
// corresponding unit eigenvector.
void jacobi_eigen(int n, double* A, double* V) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) V[i * n + j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < n; ++i) {
      diag += A[i * n + i] * A[i * n + i];
      for (int j = i + 1; j < n; ++j) off += A[i * n + j] * A[i * n + j];
    }
    if (off == 0.0 || off < 1e-36 * diag) break;
    for (int p = 0; p < n; ++p) {
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p * n + q];
        if (apq == 0.0) continue;
        const double app = A[p * n + p], aqq = A[q * n + q];
        // rotation angle that annihilates A[p][q]
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) /
                         (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        A[p * n + q] = A[q * n + p] = 0.0;
        for (int k = 0; k < n; ++k) {
          const double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
      }
    }
  }
}

}  // namespace

int whiten(int d, const double* C, double* W, int mode) {
  if (d < 1 || d > 8) return fail(BF_EINVAL, "d must be in [1, 8]");
  if (mode != BF_WHITEN_EIG && mode != BF_WHITEN_CHOL && mode != BF_WHITEN_SYM)
    return fail(BF_EINVAL, "whitening mode must be BF_WHITEN_EIG, _CHOL or _SYM");
  if (!C || !W) return fail(BF_EINVAL, "C and W must be non-null");
  double scale = 0.0;
  for (int i = 0; i < d * d; ++i) {
    if (!std::isfinite(C[i])) return fail(BF_ENOTSPD, "C has a non-finite entry");
    scale = std::max(scale, std::fabs(C[i]));
  }
  if (scale == 0.0) return fail(BF_ENOTSPD, "C is zero");
  bool diagonal = true;
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      if (i != j && C[i * d + j] != 0.0) diagonal = false;
      if (std::fabs(C[i * d + j] - C[j * d + i]) > 1e-12 * scale)
        return fail(BF_ENOTSPD, "C is not symmetric");
    }
  if (diagonal) {
    for (int i = 0; i < d; ++i)
      if (!(C[i * d + i] > 0.0)) return fail(BF_ENOTSPD, "C is not positive definite");
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j)
        W[i * d + j] = (i == j) ? 1.0 / std::sqrt(C[i * d + i]) : 0.0;
    return BF_OK;
  }
  double A[64], V[64];
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) A[i * d + j] = 0.5 * (C[i * d + j] + C[j * d + i]);
  if (mode == BF_WHITEN_CHOL) {
    // C = L L^T (Cholesky-Banachiewicz), then W = L^{-1} by forward substitution
    double L[64] = {0};
    for (int i = 0; i < d; ++i)
      for (int j = 0; j <= i; ++j) {
        double s = A[i * d + j];
        for (int k = 0; k < j; ++k) s -= L[i * d + k] * L[j * d + k];
        if (i == j) {
          if (!(s > 0.0)) return fail(BF_ENOTSPD, "C is not positive definite");
          L[i * d + i] = std::sqrt(s);
        } else {
          L[i * d + j] = s / L[j * d + j];
        }
      }
    for (int i = 0; i < d * d; ++i) W[i] = 0.0;
    for (int j = 0; j < d; ++j)
      for (int i = j; i < d; ++i) {
        double s = i == j ? 1.0 : 0.0;
        for (int k = j; k < i; ++k) s -= L[i * d + k] * W[k * d + j];
        W[i * d + j] = s / L[i * d + i];
      }
    return BF_OK;
  }
  jacobi_eigen(d, A, V);
  if (mode == BF_WHITEN_SYM) {
    // W = V diag(lambda^{-1/2}) V^T
    for (int k = 0; k < d; ++k)
      if (!(A[k * d + k] > 0.0)) return fail(BF_ENOTSPD, "C is not positive definite");
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j) {
        double s = 0.0;
        for (int k = 0; k < d; ++k) s += V[i * d + k] * V[j * d + k] / std::sqrt(A[k * d + k]);
        W[i * d + j] = s;
      }
    return BF_OK;
  }
  int order[8];
  for (int k = 0; k < d; ++k) order[k] = k;
  std::stable_sort(order, order + d,
                   [&](int a, int b) { return A[a * d + a] < A[b * d + b]; });
  for (int r = 0; r < d; ++r) {
    const int k = order[r];
    const double lam = A[k * d + k];
    if (!(lam > 0.0)) return fail(BF_ENOTSPD, "C is not positive definite");
    double vmax = 0.0;
    for (int i = 0; i < d; ++i) vmax = std::max(vmax, std::fabs(V[i * d + k]));
    double sign = 1.0;
    for (int i = 0; i < d; ++i)
      if (std::fabs(V[i * d + k]) > 1e-6 * vmax) {
        sign = V[i * d + k] < 0 ? -1.0 : 1.0;
        break;
      }
    const double inv = sign / std::sqrt(lam);
    for (int i = 0; i < d; ++i) W[r * d + i] = V[i * d + k] * inv;
  }
  return BF_OK;
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of
//   (c0,c1,c2,c3) <- (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))
// with the key bumped by two Weyl constants between rounds.
// ---------------------------------------------------------------------------

void philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)M0 * c0, p1 = (uint64_t)M1 * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n1 = (uint32_t)p1;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    const uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += W0; k1 += W1;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

int binomial_draw(uint64_t seed, int t, int m, int N) {
  const uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
  int X = 0, left = N;
  for (uint32_t q = 0; left > 0; ++q) {
    const uint32_t ctr[4] = {(uint32_t)t, (uint32_t)m, q, 0u};
    uint32_t words[4];
    philox4x32_10(ctr, key, words);
    for (int l = 0; l < 4 && left > 0; ++l) {
      uint32_t wd = words[l];
      if (left < 32) wd &= (1u << left) - 1u;
      X += __builtin_popcount(wd);
      left -= 32;
    }
  }
  return X;
}

int choose_order(int d, const double* W, const float* lo, const float* hi, int* N) {
  double T = 0.0;
  for (int k = 0; k < d; ++k) {
    double s = 0.0;
    for (int m = 0; m < d; ++m) s += std::fabs(W[k * d + m]) * ((double)hi[m] - (double)lo[m]);
    T = std::max(T, s);
  }
  const double pi = 3.141592653589793238462643383279502884;
  const double n = std::ceil(((T + 4.0) / pi) * ((T + 4.0) / pi));
  if (!(n <= 65536.0))
    return fail(BF_EUNSUPPORTED,
                "automatic order exceeds 65536 (range too wide for C); pass N explicitly");
  *N = std::max(10, (int)n);
  return BF_OK;
}

int check_fp16_range(int d, double sigma_s, int spatial, const float* lo, const float* hi,
                     const float* cen) {
  // FP16 storage holds c (f - c_m), s (f - c_m), cos, sin and their
  // horizontal-pass sums: |value| <= max(1, max_m |f_m - c_m|) * sum_u omega_1(u)
  const std::vector<double> taps = spatial_taps(sigma_s, spatial);
  double sw = 0.0;
  for (double t : taps) sw += t;
  double dev = 1.0;
  for (int m = 0; m < d; ++m)
    dev = std::max(dev, std::max((double)hi[m] - (double)cen[m], (double)cen[m] - (double)lo[m]));
  if (dev * sw > kFP16Limit)
    return fail(BF_EUNSUPPORTED,
                "image range too wide for FP16 storage: max |f - c| x sum(omega_1) = " +
                    std::to_string(dev * sw) + " exceeds 32768; use BF_BF16 or BF_FP32");
  return BF_OK;
}

int check_common(const void* f, int H, int W, int d, double sigma_s, const void* out) {
  if (!f || !out) return fail(BF_EINVAL, "f and out must be non-null device pointers");
  if (H < 1 || W < 1 || H > 65536 || W > 65536)
    return fail(BF_EINVAL, "H and W must be in [1, 65536]");
  if (d < 1 || d > 8) return fail(BF_EINVAL, "d must be in [1, 8]");
  if (!std::isfinite(sigma_s) || sigma_s < 0.0 || sigma_s > 32.0)
    return fail(BF_EINVAL, "sigma_s must be finite and in [0, 32]");
  const size_t bytes = (size_t)H * W * d * sizeof(float);
  const char* a = (const char*)f;
  const char* b = (const char*)out;
  if (a < b + bytes && b < a + bytes) return fail(BF_EINVAL, "out must not overlap f");
  return BF_OK;
}

}  // namespace bfvec

// ---------------------------------------------------------------------------
// Host-only C entry points
// ---------------------------------------------------------------------------

extern "C" {

void bf_opts_init(bf_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->N = 0;
  o->precision = BF_FP32;
  o->center = 1;
  o->time_kernel = 0;
  o->kernel_ms = 0.0f;
}

const char* bf_last_error(void) { return bfvec::g_error.c_str(); }

int bf_version(void) { return 10000; }

int bf_whiten(int d, const double* C, double* W) {
  bfvec::clear_error();
  return bfvec::whiten(d, C, W);
}

int bf_whiten_mode(int d, const double* C, int mode, double* W) {
  bfvec::clear_error();
  return bfvec::whiten(d, C, W, mode);
}

int bf_sample_terms(int d, const double* C, int N, int K, uint64_t seed, int whiten, int32_t* Y,
                    double* w) {
  bfvec::clear_error();
  if (N < 1 || N > 65536) return bfvec::fail(BF_EINVAL, "N must be in [1, 65536]");
  if (K < 1 || K > 65536) return bfvec::fail(BF_EINVAL, "K must be in [1, 65536]");
  if (whiten < BF_WHITEN_EIG || whiten > BF_WHITEN_SYM)
    return bfvec::fail(BF_EINVAL, "whiten must be BF_WHITEN_EIG, _CHOL or _SYM");
  double Wm[64];
  int st = bfvec::whiten(d, C, Wm, whiten);
  if (st) return st;
  const double sqn = std::sqrt((double)N);
  for (int t = 0; t < K; ++t) {
    int Yt[8];
    for (int m = 0; m < d; ++m) Yt[m] = N - 2 * bfvec::binomial_draw(seed, t, m, N);
    if (Y)
      for (int m = 0; m < d; ++m) Y[(size_t)t * d + m] = Yt[m];
    if (w)
      for (int j = 0; j < d; ++j) {
        double s = 0.0;
        for (int k = 0; k < d; ++k) s += (double)Yt[k] * Wm[k * d + j];
        w[(size_t)t * d + j] = s / sqn;
      }
  }
  return BF_OK;
}

int bf_choose_N(int d, const double* C, const float* lo, const float* hi, int whiten, int* N) {
  bfvec::clear_error();
  if (d < 1 || d > 8) return bfvec::fail(BF_EINVAL, "d must be in [1, 8]");
  if (!C || !lo || !hi || !N) return bfvec::fail(BF_EINVAL, "null argument");
  if (whiten < BF_WHITEN_EIG || whiten > BF_WHITEN_SYM)
    return bfvec::fail(BF_EINVAL, "whiten must be BF_WHITEN_EIG, _CHOL or _SYM");
  for (int m = 0; m < d; ++m)
    if (!std::isfinite(lo[m]) || !std::isfinite(hi[m]) || hi[m] < lo[m])
      return bfvec::fail(BF_EINVAL, "lo/hi must be finite with lo <= hi");
  double Wm[64];
  int st = bfvec::whiten(d, C, Wm, whiten);
  if (st) return st;
  return bfvec::choose_order(d, Wm, lo, hi, N);
}

}  // extern "C"
