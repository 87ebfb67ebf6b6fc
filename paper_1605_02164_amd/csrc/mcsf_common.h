// Shared declarations of the device kernels and their host launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace bfvec {

// Tile geometry of the fused kernels.
constexpr int kTW = 16;   // output columns per workgroup strip
constexpr int kB = 8;     // input rows per pipeline step
constexpr int kP1 = 4;    // horizontal-pass outputs per item (register block)
constexpr int kP2 = 4;    // vertical-pass outputs per item (register block)
constexpr int kRMax = 40; // largest window radius handled by the fused kernels

// Staging row width for radius R: at least TW + 2R + 4 floats (the
// horizontal window of a 4-output block plus one spare block), and equal to
// 16 modulo 32: measured on gfx950, that residue makes the 128-bit window
// loads of the horizontal pass free of LDS bank conflicts for the lane order
// used (widths of other residues cost one to two extra passes per load).
inline constexpr int stage_width(int R) {
  return 32 * ((kTW + 2 * R + 4 - 16 + 31) / 32) + 16;
}
// Same for 16-bit storage (elements, always even): at least TW + 2R + 4, with
// the row width in dwords not a multiple of 16 -- measured on gfx950, 64-bit
// window loads then conflict 2-way, against 4- to 8-way for multiples of 16.
inline constexpr int stage_width16(int R) {
  const int dw = (kTW + 2 * R + 4 + 3) / 4 * 2;   // dwords, even (64-bit aligned rows)
  return 2 * (dw % 16 == 0 ? dw + 2 : dw);
}
constexpr int kSWMax = stage_width(kRMax);
// 2R rows of look-ahead, in steps of kB rows
inline constexpr int lag_steps(int R) { return (2 * R + kB - 1) / kB; }

struct FusedArgs {
  const float* f;        // H*W*d input (device)
  float* acc;            // (d+1)*Hp*Wp accumulators, planar [m][y][x] (device),
                         // padded to whole strips: Hp = nsy*TH, Wp = nsx*kTW
  const float* taps;     // 2R+1 spatial taps (device), zero padded to a multiple of 4
  float cen[8];          // per-channel centre subtracted before the phase
  int H, W, K, R;
  int TH;                // strip height (multiple of kB)
  int Hp;                // padded accumulator rows (nsy*TH)
  int nsx, nsy;          // strips across and down
  int SW;                // staging row width (floats)
  int RSB, CRB;          // ring sizes in blocks of kB rows
  int steps, lag;        // steps per term, and 2R look-ahead in steps
};

struct FinalizeArgs {
  const float* acc;      // (d+1)*Hp*Wp planar accumulators
  float* out;            // H*W*d
  float* num_out;        // optional H*W*d numerator (uncentred) or null
  float* z_out;          // optional H*W normaliser or null
  float cen[8];
  int H, W, Hp, Wp;
};

// prec: 0 = FP32 channels, 1 = FP16 storage, 2 = BF16 storage (FP32 accumulation)
size_t fused_lds_bytes(int d, int R, int prec);
// resident workgroups per compute unit for this kernel instance (device query)
int fused_blocks_per_cu(int d, int R, int prec);
hipError_t launch_fused(int d, int prec, const FusedArgs& a, const float* terms,
                        const float* weights, hipStream_t st);
hipError_t launch_finalize(int d, const FinalizeArgs& a, hipStream_t st);

}  // namespace bfvec
