// Shared declarations of the device kernels and their host launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace bfvec {

// Tile geometry of the fused kernels.
constexpr int kTW = 16;   // output columns per workgroup strip
constexpr int kB = 16;    // input rows per pipeline step
constexpr int kP1 = 8;    // horizontal-pass outputs per item (register block)
constexpr int kP2 = 4;    // vertical-pass outputs per item (register block)
constexpr int kRMax = 40; // largest window radius handled by the fused kernels
// taps padded to a multiple of 8 (zero taps), staging row width, and its bound
inline constexpr int ntaps_padded(int R) { return ((2 * R + 1 + 7) / 8) * 8; }
inline constexpr int stage_width(int R) { return kTW + ntaps_padded(R) + 4; }
constexpr int kSWMax = stage_width(kRMax);

struct FusedArgs {
  const float* f;        // H*W*d input (device)
  float* out;            // H*W*d output (device)
  float* num_out;        // optional H*W*d numerator (device) or null
  float* z_out;          // optional H*W normaliser (device) or null
  const float* terms;    // K*(d+1): w_t / (2 pi) (revolutions per unit), pad
  const float* weights;  // K term weights or null
  const float* taps;     // ntp spatial taps, zero padded
  float cen[8];          // per-channel centre subtracted before the phase
  int H, W, K, R, ntp, taps_al;
  int TH;                // strip height (multiple of kB)
  int nsx, nsy;          // strips across and down
  int SW;                // staging row width (floats)
  int RSB, CRB;          // ring sizes in blocks of kB rows
  int steps, lag;        // steps per term, and 2R look-ahead in steps
};

size_t fused_lds_bytes(int d, int R, int TH);
hipError_t launch_fused_fp32(int d, const FusedArgs& a, hipStream_t st);

}  // namespace bfvec
