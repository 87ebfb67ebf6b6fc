// Single-request launches of the fused MCSF kernel, the finalize kernel,
// and the occupancy and LDS sizing used to plan strips.

#include "mcsf_fused_dev.h"

#include <array>
#include <cmath>
#include <map>
#include <mutex>

#include "bfvec.h"
#include "host.h"

namespace bfvec {

// out = num / Z + c ; optional uncentred numerator and normaliser
template <int D>
__global__ __launch_bounds__(256) void mcsf_finalize(FinalizeArgs a) {
  const size_t npx = (size_t)a.H * a.W;
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= npx) return;
  const size_t y = i / a.W, x = i - y * a.W;
  const size_t plane = (size_t)a.Hp * a.Wp, j = y * a.Wp + x;
  const float Z = a.acc[(size_t)D * plane + j];
#pragma unroll
  for (int m = 0; m < D; ++m) {
    const float num = a.acc[(size_t)m * plane + j];
    const float c = a.cen_dev ? a.cen_dev[m] : a.cen[m];
    a.out[i * D + m] = num / Z + c;
    if (a.num_out) a.num_out[i * D + m] = fmaf(c, Z, num);
  }
  if (a.z_out) a.z_out[i] = Z;
}

// ---------------------------------------------------------------------------
// Host-side launch helpers
// ---------------------------------------------------------------------------

size_t fused_lds_bytes(int d, int R, int prec, int TW, int mf) {
  const int NP = d + 1, NC = 2 * NP;
  if (prec == 4) {   // taps | two staging buffers | ring | first-stage sums | cos/sin
    const int w = 2 * (R / 3) + 1;
    const int taps_al = ((2 * R + 1 + 3) / 4 * 4 + 7) / 8 * 8;
    const size_t fl = (size_t)taps_al + 2 * (size_t)kB * NC * stage_width_mf32(R) +
                      (size_t)((w + 16 + 7) / 8 * 8) * NC * kTWMax +
                      (size_t)((2 * w + 8 + 7) / 8 * 8) * NC * kTWMax +
                      (size_t)((R + 24 + 7) / 8 * 8) * 2 * kTWMax;
    return fl * sizeof(float);
  }
  const bool lp = prec == 1 || prec == 2, vb = prec == 3;
  const int ntap4 = (2 * R + 1 + 3) / 4 * 4;
  const int taps_al = (ntap4 + 7) / 8 * 8;
  const int tapp_al = (R + 1 + 3) / 4 * 4;
  const int lag = lag_steps(R);
  // FP32 matrix-core instances from R = 21 run the one-barrier pipeline:
  // two staging buffers and two more ring steps
  const bool pipe = use_pipe(prec, R, mf != 0);
  // variant 3 sizes the ring for the largest n (three boxes)
  const int RS = (ring_steps(R, vb ? 3 : 0) + (pipe ? 2 : 0)) * kB;
  const int CRS = (pipe ? pipe_cs_steps(R) : lag + 2) * kB;
  const int CST = 2 * TW + cs_row_pad(pipe || (mf && lp && TW == kTWMax));
  const size_t fl = (size_t)taps_al + (lp ? 2 * (size_t)tapp_al : 0) +
                    (size_t)kB * NC * (pipe ? 2 : 1) *
                        (lp ? (mf ? stage_width_mf(R) : stage_width16(R, TW)) / 2
                            : (mf ? stage_width_mf32(R) : stage_width(R, TW))) +
                    (size_t)(lp ? RS / 2 : RS) *
                        (NC * TW + (mf && lp ? kRingPadMF : 0) +
                         (pipe && prec != 5 ? kRingPadPipe : 0)) +
                    (size_t)CRS * CST +
                    (vb ? (size_t)16 * NC * TW : 0);
  return fl * sizeof(float);
}

// Resident workgroups per CU from the instance's register count and LDS:
// a CU has 160 KB of LDS and 4 SIMDs of 512 VGPRs per lane (at most 8 waves
// each); a workgroup of (D+1)*TW/16 waves puts a quarter of them, rounded
// up, on a SIMD.
template <int D, int RC, int PREC>
static int blocks_per_cu_drp(int R, int TW, int valu) {
  // the instance launch_drp picks for this width
  int mf = 0;
  const void* kern = reinterpret_cast<const void*>(mcsf_fused<D, RC, PREC, false>);
  if constexpr (kHasMF<D, RC, PREC, kTW>)
    if (TW == kTW && use_mf(TW, PREC, R) && !valu) {
      kern = reinterpret_cast<const void*>(mcsf_fused<D, RC, PREC, false, kTW, true>);
      mf = 1;
    }
  if constexpr (kHasWide<D, RC, PREC>)
    if (TW == kTWMax) kern = reinterpret_cast<const void*>(mcsf_fused<D, RC, PREC, false, kTWMax>);
  if constexpr (kHasMF<D, RC, PREC, kTWMax>)
    if (TW == kTWMax && use_mf(TW, PREC, R) && !valu) {
      kern = reinterpret_cast<const void*>(mcsf_fused<D, RC, PREC, false, kTWMax, true>);
      mf = 1;
    }
  const size_t lds = fused_lds_bytes(D, R, PREC, TW, mf);
  hipFuncAttributes at{};
  int vgpr = 256;
  if (hipFuncGetAttributes(&at, kern) == hipSuccess && at.numRegs > 0) vgpr = at.numRegs;
  const int waves_per_simd = std::min(8, 512 / ((vgpr + 7) / 8 * 8));
  const int per_block = ((D + 1) * (TW / kTW) + 3) / 4;
  const int by_vgpr = waves_per_simd / per_block;
  const int by_lds = (int)((160 * 1024) / lds);
  return std::max(1, std::min(by_vgpr, by_lds));
}

template <int D, int PREC>
static int bpc_dp(int R, int TW, int valu) {
  switch (R) {
    case 6: return blocks_per_cu_drp<D, 6, PREC>(R, TW, valu);
    case 9: return blocks_per_cu_drp<D, 9, PREC>(R, TW, valu);
    case 12: return blocks_per_cu_drp<D, 12, PREC>(R, TW, valu);
    case 15: return blocks_per_cu_drp<D, 15, PREC>(R, TW, valu);
    case 18: return blocks_per_cu_drp<D, 18, PREC>(R, TW, valu);
    case 21: return blocks_per_cu_drp<D, 21, PREC>(R, TW, valu);
    case 24: return blocks_per_cu_drp<D, 24, PREC>(R, TW, valu);
    case 30: return blocks_per_cu_drp<D, 30, PREC>(R, TW, valu);
    default: return blocks_per_cu_drp<D, -1, PREC>(R, TW, valu);
  }
}

template <int PREC>
static int bpc_p(int d, int R, int TW, int valu) {
  switch (d) {
    case 1: return blocks_per_cu_drp<1, -1, PREC>(R, TW, valu);
    case 2: return blocks_per_cu_drp<2, -1, PREC>(R, TW, valu);
    case 3: return bpc_dp<3, PREC>(R, TW, valu);
    case 4: return blocks_per_cu_drp<4, -1, PREC>(R, TW, valu);
    case 5: return blocks_per_cu_drp<5, -1, PREC>(R, TW, valu);
    case 6: return bpc_dp<6, PREC>(R, TW, valu);
    case 7: return blocks_per_cu_drp<7, -1, PREC>(R, TW, valu);
    default: return blocks_per_cu_drp<8, -1, PREC>(R, TW, valu);
  }
}

// the radii with compile-time instances (launch_dp in the device header)
static bool specialised_radius(int R) {
  switch (R) {
    case 6: case 9: case 12: case 15: case 18: case 21: case 24: case 30: return true;
    default: return false;
  }
}

// variant 4: one 8-wave workgroup per CU by its LDS (checked against the
// instance's registers)
template <int RC>
static int blocks_per_cu_sl() {
  hipFuncAttributes at{};
  int vgpr = 256;
  if (hipFuncGetAttributes(&at, reinterpret_cast<const void*>(
                                    mcsf_fused<3, RC, 4, false, kTWMax, true>)) == hipSuccess &&
      at.numRegs > 0)
    vgpr = at.numRegs;
  const int by_vgpr = std::min(8, 512 / ((vgpr + 7) / 8 * 8)) / 2;
  const int by_lds = (int)((160 * 1024) / fused_lds_bytes(3, RC, 4, kTWMax, 1));
  return std::max(1, std::min(by_vgpr, by_lds));
}

// variant 5: one 8-wave workgroup per CU by its LDS (checked against the
// instance's registers)
template <int RC>
static int blocks_per_cu_sp() {
  hipFuncAttributes at{};
  int vgpr = 256;
  if (hipFuncGetAttributes(&at, reinterpret_cast<const void*>(
                                    mcsf_fused<3, RC, 5, false, kTWMax, true>)) == hipSuccess &&
      at.numRegs > 0)
    vgpr = at.numRegs;
  const int by_vgpr = std::min(8, 512 / ((vgpr + 7) / 8 * 8)) / 2;
  const int by_lds = (int)((160 * 1024) / fused_lds_bytes(3, RC, 5, kTWMax, 1));
  return std::max(1, std::min(by_vgpr, by_lds));
}

int fused_blocks_per_cu(int d, int R, int prec, int TW, int valu) {
  switch (prec) {
    case 5:
      switch (R) {
        case 18: return blocks_per_cu_sp<18>();
        case 21: return blocks_per_cu_sp<21>();
        case 24: return blocks_per_cu_sp<24>();
        default: return blocks_per_cu_sp<30>();
      }
    case 0: return bpc_p<0>(d, R, TW, valu);
    case 1: return bpc_p<1>(d, R, TW, valu);
    case 2: return bpc_p<2>(d, R, TW, valu);
    case 4:
      switch (R) {
        case 6: return blocks_per_cu_sl<6>();
        case 9: return blocks_per_cu_sl<9>();
        case 12: return blocks_per_cu_sl<12>();
        case 15: return blocks_per_cu_sl<15>();
        case 18: return blocks_per_cu_sl<18>();
        case 21: return blocks_per_cu_sl<21>();
        case 24: return blocks_per_cu_sl<24>();
        default: return blocks_per_cu_sl<30>();
      }
    default: return bpc_p<3>(d, R, TW, valu);
  }
}

int select_variant(int d, int R, int precision, int spatial, int W, int tile_w, int valu) {
  const int v = kernel_variant(precision, spatial);
  // variant 4 only where 32-column strips are asked for: at 4096^2, R = 30,
  // K = 256 it took 216 ms against 174 ms for the 16-column running sums
  // (variant 3), so the automatic choice keeps variant 3
  if (v == 3 && spatial_boxes(spatial) == 3 && d == 3 && specialised_radius(R) && R % 3 == 0 &&
      W >= kTWMax && tile_w == kTWMax && !valu)
    return 4;
  return v;
}

int fused_uses_mf(int d, int R, int prec, int TW, int valu) {
  if (prec == 4 || prec == 5) return 1;   // variant 4: its horizontal pass; 5: both
  if (valu || !specialised_radius(R) || (d != 3 && d != 6) || prec > 2) return 0;
  const bool inst = TW == kTWMax ? d == 3 : (prec == 1 || prec == 2);
  return inst && use_mf(TW, prec, R) ? 1 : 0;
}

int strip_row_multiple(int d, int R, int prec, int TW, int valu) {
  return fused_uses_mf(d, R, prec, TW, valu) && use_pipe(prec, R, true) ? 2 * kB : kB;
}

int choose_strip_width(int d, int R, int prec, int H, int W, int requested, int* TW) {
  if (prec == 4) {   // select_variant guarantees the instance
    *TW = kTWMax;
    return BF_OK;
  }
  if (prec == 5) {
    if (d != 3 || !split_radius(R) || W < kTWMax || requested == kTW)
      return fail(BF_EUNSUPPORTED,
                  "BF_FP32_SPLIT needs d = 3, a window radius of 18, 21, 24 or 30 (sigma_s 6, "
                  "7, 8 or 10 for the Gaussian), W >= 32 and 32-column strips");
    *TW = kTWMax;
    return BF_OK;
  }
  const bool wide_ok = d == 3 && prec <= 2 && W >= kTWMax && specialised_radius(R) &&
                       fused_lds_bytes(d, R, prec, kTWMax) <= 160 * 1024;
  if (requested == kTWMax && !wide_ok)
    return fail(BF_EUNSUPPORTED,
                "32-column strips need d = 3, a window radius with a compile-time kernel "
                "(6, 9, ..., 24 or 30), FP32/FP16/BF16 without the running-sum pass, and W >= 32");
  if (requested == kTW || requested == kTWMax) {
    *TW = requested;
    return BF_OK;
  }
  *TW = wide_ok ? model_strip_width(d, R, prec) : kTW;
  // A small image is latency-bound: its few workgroups each run the whole
  // step chain, and narrow strips spread them over twice as many CUs
  // (measured at 128^2, sigma_s = 2: 32-column strips 7% slower per call).
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if ((long)((W + kTW - 1) / kTW) * ((H + kB - 1) / kB) < 2L * std::max(ncu, 1)) *TW = kTW;
  return BF_OK;
}

int model_strip_width(int d, int R, int prec) {
  // Wide strips halve the halo columns each workgroup modulates and filters
  // but hold more registers and LDS per wave.  Measured at 4096^2, K = 32,
  // every radius: they ran 3-13% faster wherever they kept at least three
  // quarters of the narrow strips' resident waves (also at 16 of 20 waves
  // with 16-bit storage), and 4.8% slower at FP32, R = 18 (8 of 12 waves).
  const int narrow_waves = fused_blocks_per_cu(d, R, prec, kTW) * (d + 1);
  const int wide_waves = fused_blocks_per_cu(d, R, prec, kTWMax) * 2 * (d + 1);
  return 4 * wide_waves >= 3 * narrow_waves ? kTWMax : kTW;
}

// ---------------------------------------------------------------------------
// Strip height.  Each workgroup streams one strip per term and recomputes 2R
// halo rows per strip, so tall strips waste less; but all compute units
// should be busy (two workgroups fit on a CU).  Choose the number of strips
// down the image that minimises (waves of workgroups) x (rows per strip incl.
// halo).
// ---------------------------------------------------------------------------

namespace {
std::mutex g_tuned_mu;
// (device, d, R, precision, H, W, strip width) -> strip height
std::map<std::array<int, 7>, int> g_tuned;
// (device, d, R, precision, size class of H, size class of W, strip width)
// -> strips down the image, from the latest measurement in that class
std::map<std::array<int, 7>, int> g_tuned_class;
}  // namespace

int size_class(int n) { return (int)std::floor(2.0 * std::log2((double)std::max(n, 1)) + 0.5); }

void record_tuned_height(int d, int R, int prec, int H, int W, int TH, int TW) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_tuned_mu);
  g_tuned[{dev, d, R, prec, H, W, TW}] = TH;
  g_tuned_class[{dev, d, R, prec, size_class(H), size_class(W), TW}] = (H + TH - 1) / TH;
}

int tuned_height(int d, int R, int prec, int H, int W, int TW) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  int nsy = 0;
  {
    std::lock_guard<std::mutex> lk(g_tuned_mu);
    auto it = g_tuned.find({dev, d, R, prec, H, W, TW});
    if (it != g_tuned.end()) return it->second;
    auto ic = g_tuned_class.find({dev, d, R, prec, size_class(H), size_class(W), TW});
    if (ic == g_tuned_class.end()) return 0;
    nsy = ic->second;
  }
  // the class's strip count, on this image's height
  const int mult = strip_row_multiple(d, R, prec, TW, 0);
  return ((H + nsy - 1) / nsy + mult - 1) / mult * mult;
}

int tuned_class_known(int d, int R, int prec, int H, int W, int TW) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_tuned_mu);
  return g_tuned_class.count({dev, d, R, prec, size_class(H), size_class(W), TW}) ? 1 : 0;
}

int choose_strip_height(int d, int R, int prec, int H, int W, int requested, int* TH, int TW,
                        int valu) {
  if (fused_lds_bytes(d, R, prec, TW) > 160 * 1024)
    return fail(BF_EUNSUPPORTED, "window too large for the fused kernel's LDS budget");
  // one strip covers the image: taller strips only add padded rows (and
  // would push accumulator offsets past 32 bits for huge requests)
  const int mult = strip_row_multiple(d, R, prec, TW, valu);
  const int one = (H + mult - 1) / mult * mult;
  if (requested > 0) {
    *TH = (int)std::min<long>(((long)requested + mult - 1) / mult * mult, one);
    return BF_OK;
  }
  if (!valu && (*TH = tuned_height(d, R, prec, H, W, TW)) > 0) return BF_OK;
  *TH = std::min(model_strip_height(d, R, prec, H, W, TW, valu), one);
  return BF_OK;
}

int model_strip_height(int d, int R, int prec, int H, int W, int TW, int valu) {
  const int nsx = (W + TW - 1) / TW;
  // resident workgroups on the GPU
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  const int slots = fused_blocks_per_cu(d, R, prec, TW, valu) * std::max(ncu, 1);
  const int halo = lag_steps(R) * kB;
  // The accumulators of the resident workgroups are read and written once
  // per term.  On the 4096^2 workload, strips half as tall (two waves of
  // workgroups, accumulators within ~60% of the 256 MB last-level cache) ran
  // 0.6% (FP32) and 4.6% (FP16) faster than one wave of taller strips, though
  // they re-read more halo: a footprint above that share costs 10% here.
  constexpr double kCacheShare = 0.6 * 256.0 * 1024 * 1024;
  double best = -1.0;
  int best_th = kB;
  const int mult = strip_row_multiple(d, R, prec, TW, valu);
  for (int nsy = 1; nsy <= (H + mult - 1) / mult; ++nsy) {
    const int th = ((H + nsy - 1) / nsy + mult - 1) / mult * mult;
    const long nwg = (long)nsx * ((H + th - 1) / th);
    const long waves = (nwg + slots - 1) / slots;
    const double resident = (double)std::min<long>(nwg, slots) * th * TW * (d + 1) * 4.0;
    const double cost = (double)waves * (th + halo) * (resident > kCacheShare ? 1.1 : 1.0);
    if (best < 0 || cost < best) {
      best = cost;
      best_th = th;
    }
    if (nwg > 16L * slots) break;
  }
  return best_th;
}

hipError_t launch_fused(int d, int prec, const FusedArgs& a, hipStream_t st) {
  switch (prec) {
    case 0: return launch_p<0>(d, a, a.R, st);
    case 1: return launch_p<1>(d, a, a.R, st);
    case 2: return launch_p<2>(d, a, a.R, st);
    case 3: return launch_p<3>(d, a, a.R, st);
    case 4: return d == 3 ? launch_sl_r(a, a.R, st) : hipErrorInvalidValue;
    case 5: return d == 3 ? launch_sp_r(a, a.R, st) : hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_finalize(int d, const FinalizeArgs& a, hipStream_t st) {
  const size_t plane = (size_t)a.H * a.W;
  const dim3 grid((unsigned)((plane + 255) / 256));
  switch (d) {
    case 1: hipLaunchKernelGGL(mcsf_finalize<1>, grid, dim3(256), 0, st, a); break;
    case 2: hipLaunchKernelGGL(mcsf_finalize<2>, grid, dim3(256), 0, st, a); break;
    case 3: hipLaunchKernelGGL(mcsf_finalize<3>, grid, dim3(256), 0, st, a); break;
    case 4: hipLaunchKernelGGL(mcsf_finalize<4>, grid, dim3(256), 0, st, a); break;
    case 5: hipLaunchKernelGGL(mcsf_finalize<5>, grid, dim3(256), 0, st, a); break;
    case 6: hipLaunchKernelGGL(mcsf_finalize<6>, grid, dim3(256), 0, st, a); break;
    case 7: hipLaunchKernelGGL(mcsf_finalize<7>, grid, dim3(256), 0, st, a); break;
    case 8: hipLaunchKernelGGL(mcsf_finalize<8>, grid, dim3(256), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace bfvec
