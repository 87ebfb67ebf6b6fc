// Shared declarations of the device kernels and their host launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

namespace bfvec {

// Tile geometry of the fused kernels.
constexpr int kTW = 16;   // output columns per workgroup strip (the default width)
constexpr int kTWMax = 32; // the wide strips of some instances (64 (d+1) * 2 threads)
constexpr int kB = 8;     // input rows per pipeline step
constexpr int kP1 = 4;    // horizontal-pass outputs per item (register block)
constexpr int kP2 = 4;    // vertical-pass outputs per item (register block)
constexpr int kRMax = 40; // largest window radius handled by the fused kernels
// Phases (in turns) above this are reduced in FP64: an FP32 phase of 2^8
// turns keeps 2^-16 turns of resolution, ~1e-4 rad.  Launches whose phase
// bound sum_m max_t |w_tm/2pi| max|f_m - c_m| stays at or below kPhaseBound
// (a margin below kPhaseExact for the bound's own rounding) run the kernel
// instance without the FP64 path; in the other instance lanes below
// kPhaseExact compute the same operations, so both give the same bits there.
constexpr float kPhaseExact = 256.0f;
constexpr float kPhaseBound = 255.0f;

// Staging row width for radius R: at least TW + 2R + 4 floats (the
// horizontal window of a 4-output block plus one spare block), and equal to
// 16 modulo 32: measured on gfx950, that residue makes the 128-bit window
// loads of the horizontal pass free of LDS bank conflicts for the lane order
// used (widths of other residues cost one to two extra passes per load).
inline constexpr int stage_width(int R, int TW = kTW) {
  return 32 * ((TW + 2 * R + 4 - 16 + 31) / 32) + 16;
}
// Same for 16-bit storage (elements, always even): at least TW + 2R + 4, with
// the row width in dwords not a multiple of 16 -- measured on gfx950, 64-bit
// window loads then conflict 2-way, against 4- to 8-way for multiples of 16.
inline constexpr int stage_width16(int R, int TW = kTW) {
  const int dw = (TW + 2 * R + 4 + 3) / 4 * 2;   // dwords, even (64-bit aligned rows)
  return 2 * (dw % 16 == 0 ? dw + 2 : dw);
}
// Staging row width of the matrix-core passes (16-bit storage, either
// strip width): the banded product reads 16 + 32*ceil((16 + 2R)/32) samples
// per row (16-column output blocks, k-blocks of 32 samples; at least the
// TW + 2R modulated ones), plus 8 elements so that the row stride is 4 mod 8
// dwords: the 16 rows one 128-bit operand read touches then spread over the
// LDS banks.
inline constexpr int stage_width_mf(int R) { return 16 + 32 * ((16 + 2 * R + 31) / 32) + 8; }
// Pair-row padding of the 16-bit ring for the matrix-core vertical pass, in
// dwords: the four 16-lane groups of an operand read sit 2 pair-rows apart,
// which a stride of 8 mod 32 dwords spreads over all banks.
constexpr int kRingPadMF = 4;
// Matrix-core passes for a launch with strip width TW, on the instances that
// have them (compile-time radius): always with 16-bit storage; for FP32 (the
// horizontal pass, 32-column strips) from R = 12 up -- measured at 4096^2,
// K = 32: 3-17% faster at R = 12..30, 3-5% slower at R = 6 and 9.
inline constexpr bool use_mf(int TW, int prec, int R) {
  return prec == 1 || prec == 2 || (TW == kTWMax && prec == 0 && R >= 12);
}
// FP32 matrix-core instances from R = 21 run both passes on the matrix cores
// in a one-barrier pipeline (two staging buffers, two more ring steps): there
// one workgroup fills a CU's LDS with or without it, and the pipeline
// overlaps the products with the modulation on the VALU.  Below R = 21 the
// extra LDS would halve the resident workgroups.
inline constexpr bool use_pipe(int prec, int R, bool mf) {
  return mf && ((prec == 0 && R >= 21) || (prec == 5 && R >= 18));
}
// Variant 5 (FP32 channels, split vertical pass): the pipelined instances with
// the horizontal-pass rows kept as FP16 pairs hi + lo and the vertical pass as
// 16x16x32 FP16 products (hi.hi + lo.hi + hi.lo, FP32 accumulation).  They
// exist for d = 3, 32-column strips and the compile-time radii from 18 up
// (at 18 the FP32 instance already runs one workgroup per CU, so the
// pipeline's extra LDS costs no residency there).
inline constexpr bool split_radius(int R) { return R == 18 || R == 21 || R == 24 || R == 30; }
// Ring row padding of those instances, in floats (16 mod 32: conflict-free
// reads of 4 rows x 16 columns).
constexpr int kRingPadPipe = 16;
// FP32 staging row width of the matrix-core horizontal pass: 16 + 4*ceil((16
// + 2R)/4) samples read per row (k-blocks of 4), rounded to 4 mod 8 floats so
// that the 16 rows x 4 columns one operand read touches fall on distinct banks.
inline constexpr int stage_width_mf32(int R) {
  const int need = 16 + 4 * ((16 + 2 * R + 3) / 4);
  return need % 8 == 0 ? need + 4 : need;
}
constexpr int kSWMax = stage_width(kRMax);
// 2R rows of look-ahead, in steps of kB rows
inline constexpr int lag_steps(int R) { return (2 * R + kB - 1) / kB; }
// Cos/sin ring of the pipelined FP32 instances, in steps of kB rows: a pair
// window starting lag + 2 steps behind the newest modulated step reads the
// cos/sin of its rows R .. R + 15, so (lag + 4) kB - R rows are live.
inline constexpr int pipe_cs_steps(int R) { return ((lag_steps(R) + 4) * kB - R + kB - 1) / kB; }
// Row padding of the cos/sin ring where the matrix-core vertical pass reads
// it in 16-lane groups 4 rows apart (pipelined FP32, 16-bit storage in
// 32-column strips): 4 rows of 2 TW + 4 floats are 16 mod 64 floats apart,
// so the groups fall on different LDS banks.
inline constexpr int cs_row_pad(bool padded) { return padded ? 4 : 0; }
// Ring of horizontal-pass rows, in steps of kB rows: the FIR vertical pass
// reads the 2R rows behind the newest step (vbox = 0); the running-sum pass
// of the n-fold box also reads the n rows before those (vbox = n).
inline constexpr int ring_steps(int R, int vbox) { return (2 * R + vbox + 2 * kB - 1) / kB; }

// Spatial option: the number n of boxes (0 = Gaussian) in the low bits, and
// the flag (16) asking for the running-sum vertical pass.
inline int spatial_boxes(int spatial) { return spatial & 3; }
inline bool spatial_runsum(int spatial) { return (spatial & 16) != 0; }
// Kernel variants: 0 FP32, 1 FP16 storage, 2 BF16 storage (FIR passes with
// any spatial taps), 3 FP32 with the running-sum vertical pass of the n-fold
// box filters (requested by the flag), 4 FP32 three-box filter with sliding
// box sums in the vertical pass and the horizontal pass on the matrix cores
// (the flag with three boxes and 32-column strips asked for, where such an
// instance exists).
inline int kernel_variant(int precision, int spatial) {
  return precision == 0 && spatial_runsum(spatial) && spatial_boxes(spatial) > 0 ? 3 : precision;
}
// kernel_variant, with variant 4 in place of 3 for three boxes at d = 3, a
// compile-time radius (multiple of 3), W >= 32, tile_w = 32 and matrix-core
// passes allowed (the automatic width keeps variant 3, measured faster).
int select_variant(int d, int R, int precision, int spatial, int W, int tile_w, int valu);
// BF_OK, or BF_EINVAL / BF_EUNSUPPORTED with the message set.
int check_spatial(int spatial, int precision);

struct FusedArgs {
  const float* f;        // input (device), row y at f + y*fpitch*d
  float* acc;            // (d+1)*Hp*Wp accumulators, planar [m][y][x] (device),
                         // padded to whole strips: Hp = nsy*TH, Wp = nsx*TWc
  const float* taps;     // 2R+1 spatial taps (device), zero padded to a multiple of 4
  const float* terms;    // term table (device): row t holds w_t / 2pi in its first d of d+1 floats
  const float* terms_lo; // same layout: w_t / 2pi minus its FP32 value (for large phases)
  const float* weights;  // K term weights (device), or null for equal weights
  float cen[8];          // per-channel centre subtracted before the phase
  const float* cen_dev;  // or null; else the centre is read here (device, d floats)
  int H, W, R;
  int fpitch;            // pixels between vertically adjacent pixels of f (>= W)
  int t0, t1;            // term range of this launch; the accumulators start at zero at term 0
  int TH;                // strip height (multiple of kB)
  int Hp;                // padded accumulator rows (nsy*TH)
  int nsx, nsy;          // strips across and down
  int SW;                // staging row width (floats)
  int RSB, CRB;          // ring sizes in blocks of kB rows
  int steps, lag;        // steps per term, and 2R look-ahead in steps
  int vbox;              // variant 3: n of the n-fold box (R = n r); else 0
  int TWc;               // strip width: kTW, or kTWMax for the wide-strip instances
  int p64;               // 1: instance with the FP64 phase path (phase bound unknown or
                         // above kPhaseBound), 0: without it
  float wmax[8];         // max_t |w_tm / 2pi| over the table's FP32 values
  int valu;              // 1: no matrix-core passes (the VALU instance of this width)
};

// Host side of the FP64-phase decision: 1 unless the per-channel ranges
// [lo, hi] (or none known: lo = hi = null) bound every phase by kPhaseBound.
int phase64_flag(int d, const float* wmax, const float* cen, const float* lo, const float* hi);
// max_t |row t, channel m| of a term table's FP32 frequency rows.
void table_wmax(int d, int K, const float* tab, float* wmax);

// Several requests of one kernel instance (same d, R, precision) in one
// launch: workgroups first[i] .. first[i+1]-1 take the strips of req[i].
constexpr int kMaxBatch = 16;
struct BatchArgs {
  int n;
  int first[kMaxBatch + 1];
  FusedArgs req[kMaxBatch];
};

struct FinalizeArgs {
  const float* acc;      // (d+1)*Hp*Wp planar accumulators
  float* out;            // H*W*d
  float* num_out;        // optional H*W*d numerator (uncentred) or null
  float* z_out;          // optional H*W normaliser or null
  const float* cen_dev;  // or null; else the centre is read here (device)
  float cen[8];
  int H, W, Hp, Wp;
};

// prec: the kernel variant (kernel_variant): 0 = FP32 channels, 1 = FP16
// storage, 2 = BF16 storage (FP32 accumulation), 3 = FP32 with the
// running-sum vertical pass; TW: strip width
size_t fused_lds_bytes(int d, int R, int prec, int TW = kTW, int mf = 0);
// resident workgroups per compute unit for this kernel instance (device query);
// valu = 1: the instance without matrix-core passes
int fused_blocks_per_cu(int d, int R, int prec, int TW = kTW, int valu = 0);
// 1 if a launch of this (d, R, variant, width) runs a pass on the matrix cores
int fused_uses_mf(int d, int R, int prec, int TW, int valu);
// Strip heights of this instance are multiples of this many rows: 16 for the
// pipelined FP32 matrix-core instances (their vertical pass takes pairs of
// 8-row steps), else kB.
int strip_row_multiple(int d, int R, int prec, int TW, int valu);
// Strip width for a launch into *TW.  requested: kTW or kTWMax forces it
// (kTWMax needs a wide-strip instance: d = 3, a specialised radius, variants
// 0-2, W >= kTWMax; else BF_EUNSUPPORTED); 0 picks kTWMax where such an
// instance exists, fits the LDS, keeps at least three quarters of the waves
// per CU resident that kTW strips keep, and the image is large enough that
// kTW strips of kB rows would give at least two workgroups per CU; else kTW.
int choose_strip_width(int d, int R, int prec, int H, int W, int requested, int* TW);
// The occupancy rule alone, for an instance that has both widths.
int model_strip_width(int d, int R, int prec);
hipError_t launch_fused(int d, int prec, const FusedArgs& a, hipStream_t st);
// All requests of b share d, R and prec (and hence LDS size and staging width).
hipError_t launch_fused_batch(int d, int R, int prec, const BatchArgs& b, hipStream_t st);
hipError_t launch_finalize(int d, const FinalizeArgs& a, hipStream_t st);

// Per-channel extrema of an image with row pitch `pitch` pixels, in two
// kernels: nparts partial blocks into part (nparts*17 floats), then the
// final reduction into res (kMMResult floats: d minima at 0.., d maxima at
// 8.., a non-finite flag at 16, and the midpoints (float)((lo + hi) / 2),
// formed in FP64 as the host does, at 17.. (zero past d)).
constexpr int kMMResult = 25;
int minmax_parts(size_t npx);
hipError_t launch_minmax(const float* f, int H, int W, int pitch, int d, float* part, int nparts,
                         float* res, hipStream_t st);

// ---- host planning shared by the entry points and the serving scheduler ----
// BF_EUNSUPPORTED (with the message set) if the fused kernels cannot take
// this image: radius above kRMax, or sizes past 32-bit element offsets.
int check_fused_size(int H, int W, int pitch, int d, int R);
// Strip height: requested > 0 forces it; otherwise a height measured by
// bf_autotune for this device and shape, else the occupancy model.
// The height is at most the image height rounded up to kB rows (one strip).
int choose_strip_height(int d, int R, int prec, int H, int W, int requested, int* TH,
                        int TW = kTW, int valu = 0);
// The occupancy model alone: minimises (waves of workgroups) x (rows + halo).
int model_strip_height(int d, int R, int prec, int H, int W, int TW = kTW, int valu = 0);
// BF_EUNSUPPORTED (message set) if the planned accumulators of a (after
// fused_geometry) need 32-bit element offsets of 2^30 or more.
int check_acc_size(const FusedArgs& a, int d);

// Process-wide table of measured strip heights, keyed by the current device,
// d, R, precision, the image shape and the strip width.
// A measurement also stands for its size class (H and W in half octaves,
// round(2 log2 n)): shapes of the class without their own entry take its
// number of strips down the image.
void record_tuned_height(int d, int R, int prec, int H, int W, int TH, int TW = kTW);
int tuned_height(int d, int R, int prec, int H, int W, int TW = kTW);
// 1 if a strip height was measured for this size class
int tuned_class_known(int d, int R, int prec, int H, int W, int TW = kTW);
// Measure and record the fastest strip height for an image (bf_autotune's
// probes; row pitch `pitch` pixels) on stream st.  th / ms may be null.
int autotune_strip_height(const float* f, int H, int W, int pitch, int d, double sigma_s,
                          int prec, hipStream_t st, int* th, float* ms_per_term);
// Strip geometry, staging width and ring sizes of a FusedArgs (TH is raised
// to 16 when R = 0 so that every term has at least two pipeline steps);
// vbox = n for variant 3, else 0.
void fused_geometry(FusedArgs& a, int H, int W, int R, int prec, int TH, int vbox = 0,
                    int TW = kTW);
// Accumulator floats of a planned FusedArgs: (d+1) planes of Hp x Wp.
size_t fused_acc_floats(const FusedArgs& a, int d);
// Host term table: K rows of w_t/2pi (stride d+1, FP32) | K rows of the
// remainders w_t/2pi - FP32(w_t/2pi) | K weights (if any) | 2R+1 taps of the
// spatial filter.  The remainders start at K*(d+1); the offsets of the
// weights and taps are returned in floats.
std::vector<float> term_table(int d, int K, const double* w, const double* weights,
                              double sigma_s, size_t* off_weights, size_t* off_taps,
                              int spatial = 0);
// Frequencies w_t = W^T Y_t / sqrt(N) of K terms drawn from seed (K x d, radians).
void frequency_table(int d, const double* Wm, int N, int K, uint64_t seed, double* w);
// The same K draws merged by +-Y (first nonzero entry of Y made positive), in
// order of first occurrence: distinct frequencies (n x d) and multiplicities.
void distinct_terms(int d, const double* Wm, int N, int K, uint64_t seed, std::vector<double>* w,
                    std::vector<double>* weight);

}  // namespace bfvec
