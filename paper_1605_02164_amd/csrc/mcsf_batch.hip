// Batched launches of the fused MCSF kernel: several requests that share d,
// the window radius and the storage precision in one grid (continuous
// batching of the serving scheduler).  Each request brings its own image,
// accumulators, term table and term range.

#include "mcsf_fused_dev.h"

namespace bfvec {

hipError_t launch_fused_batch(int d, int R, int prec, const BatchArgs& b, hipStream_t st) {
  if (b.n < 1 || b.n > kMaxBatch) return hipErrorInvalidValue;
  switch (prec) {
    case 0: return launch_p<0>(d, b, R, st);
    case 1: return launch_p<1>(d, b, R, st);
    case 2: return launch_p<2>(d, b, R, st);
    case 3: return launch_p<3>(d, b, R, st);
    case 4: return d == 3 ? launch_sl_r(b, R, st) : hipErrorInvalidValue;
    case 5: return d == 3 ? launch_sp_r(b, R, st) : hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

}  // namespace bfvec
