// Internal host-side helpers of libbfvec (not part of the C ABI).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace bfvec {

// Thread-local error message, reported through bf_last_error().
void set_error(const std::string& msg);
void clear_error();

// Returns a status code after recording msg.
int fail(int code, const std::string& msg);

// Window radius: R = ceil(3 sigma_s) for the Gaussian (spatial = 0; square
// window of the paper's Section 1), R = n r for the n-fold box (spatial = n).
int window_radius(double sigma_s, int spatial = 0);

// Half-width r of one box of the n-fold box filter standing in for a Gaussian
// of deviation sigma_s: the integer nearest the root of
// n((2r+1)^2 - 1)/12 = sigma_s^2 (the n-fold box's variance), halves up.
int box_radius(double sigma_s, int n);

// One-dimensional factor omega_1(u), u = -R..R, of the separable spatial
// filter: exp(-u^2 / 2 sigma_s^2) (eq. (kernel)) for spatial = 0, the n-fold
// convolution of a box of 2r+1 ones for spatial = n (1 box, 2 hat, 3 three
// boxes; Section 3 allows any spatial filter in place of the Gaussian).
std::vector<double> spatial_taps(double sigma_s, int spatial = 0);

// Whitening per eq. (COB); see bf_whiten in bfvec.h.  Returns a status.
// mode: BF_WHITEN_EIG (eq. (COB)), BF_WHITEN_CHOL, BF_WHITEN_SYM.
int whiten(int d, const double* C, double* W, int mode = 0);

// Philox4x32-10 block function (Salmon et al., SC'11).
void philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

// X[t][m] ~ B(N, 1/2) from the Philox stream of (seed, t, m).
int binomial_draw(uint64_t seed, int t, int m, int N);

// Order rule; see bf_choose_N.
int choose_order(int d, const double* W, const float* lo, const float* hi, int* N);

// FP16 storage range: the stored channels c (f_m - c_m), s (f_m - c_m), cos,
// sin and their horizontal-pass sums are bounded by
// max(1, max_m |f_m - c_m|) * sum_u omega_1(u) (|cos|, |sin| <= 1; the taps
// are positive).  Above kFP16Limit (half the FP16 maximum, 65504) a launch
// is refused: BF_EUNSUPPORTED with the message set.  lo/hi: the image's
// per-channel extrema; cen: the centre subtracted before the phase.
constexpr double kFP16Limit = 32768.0;
int check_fp16_range(int d, double sigma_s, int spatial, const float* lo, const float* hi,
                     const float* cen);

// Argument validation shared by the entry points.
int check_common(const void* f, int H, int W, int d, double sigma_s, const void* out);

}  // namespace bfvec
