// Fused MCSF kernel for gfx950 (CDNA4), FP32 channels.
//
// One workgroup owns a strip of TW output columns and TH output rows and keeps
// the numerator and normaliser of every strip pixel in LDS for the whole run
// (Algorithm 1, accumulators P and Z).  For each of the K terms it streams
// down the strip in steps of B input rows; a step
//   1. modulates B haloed rows: theta = <w_t, f - c>, H = cos + i sin
//      (eq. (Ht)), writing the 2(d+1) real channels
//      {cos f_m, sin f_m (m < d), cos, sin} to a staging buffer (zero outside
//      the image: out-of-domain pixels contribute nothing);
//   2. runs the horizontal pass of the separable truncated Gaussian omega on
//      those rows, writing into a ring of the last RS rows;
//   3. once 2R rows of look-ahead are in the ring, runs the vertical pass for B
//      output rows and demodulates into the accumulators:
//      P_m += cos * (omega*cos f_m) + sin * (omega*sin f_m),
//      Z   += cos * (omega*cos)     + sin * (omega*sin)   (eqs. (numerator), (denom)).
// After the last term out = P / Z is written (Algorithm 1, last step).
//
// Work per output pixel and term: 2(d+1)(2R+1) FMAs per pass.  Both passes are
// register-blocked sliding windows reading LDS with 128-bit loads; taps are
// read from LDS as wave-uniform broadcasts.  No MFMA: the passes are stencils.

#include <hip/hip_runtime.h>

#include "mcsf_common.h"

namespace bfvec {

namespace {

template <int D>
struct Geo {
  static constexpr int NP = D + 1;        // channel pairs (d numerators + Z)
  static constexpr int NC = 2 * NP;       // real channels
  static constexpr int NT = 64 * NP;      // threads per workgroup
  // modulation slots per thread (B x SW pixels, SW <= SW_MAX)
  static constexpr int MI = (kB * kSWMax + NT - 1) / NT;
};

__device__ __forceinline__ int wrap(int r, int n) { return r >= n ? r - n : r; }

__device__ __forceinline__ void ld8(float (&v)[8], const float* p) {
  const float4 a = *reinterpret_cast<const float4*>(p);
  const float4 b = *reinterpret_cast<const float4*>(p + 4);
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}

__device__ __forceinline__ void ld4(float (&v)[8], const float* p) {
  const float4 a = *reinterpret_cast<const float4*>(p);
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
}

// Sliding-window FMAs of a P-output register block.  The window is two
// P-blocks (lo | hi); output p takes taps t[i] against window[p + i].
// fma_lo applies the terms that fall in the lo block, fma_hi the rest.
template <int P, int N>
__device__ __forceinline__ void fma_lo(float (&acc)[P], const float* t, const float (&lo)[N]) {
#pragma unroll
  for (int i = 0; i < P; ++i)
#pragma unroll
    for (int p = 0; p + i < P; ++p) acc[p] = fmaf(t[i], lo[p + i], acc[p]);
}

template <int P, int N>
__device__ __forceinline__ void fma_hi(float (&acc)[P], const float* t, const float (&hi)[N]) {
#pragma unroll
  for (int i = 1; i < P; ++i)
#pragma unroll
    for (int p = P - i; p < P; ++p) acc[p] = fmaf(t[i], hi[p + i - P], acc[p]);
}

}  // namespace

template <int D>
__global__ __launch_bounds__(64 * (D + 1)) void mcsf_fused_fp32(FusedArgs a,
                                                                const float* __restrict__ terms,
                                                                const float* __restrict__ weights) {
  using G = Geo<D>;
  constexpr int NP = G::NP, NC = G::NC, NT = G::NT, MI = G::MI;
  constexpr int TW = kTW, B = kB, P1 = kP1, P2 = kP2;
  constexpr int RST = 2 * NP * TW;         // ring row stride [k][m][x]
  constexpr int CST = 2 * TW;              // cos/sin ring row stride [k][x]
  constexpr int AST = NP * TW;             // accumulator row stride [m][x]

  extern __shared__ float4 lds4[];
  float* lds = reinterpret_cast<float*>(lds4);
  const int SW = a.SW, R = a.R, ntp = a.ntp, TH = a.TH;
  const int RS = a.RSB * B, CRS = a.CRB * B;
  float* s_taps = lds;
  float* s_stage = s_taps + a.taps_al;
  float* s_ring = s_stage + B * NC * SW;
  float* s_cs = s_ring + RS * RST;
  float* s_acc = s_cs + CRS * CST;

  const int tid = threadIdx.x;
  // XCD-aware tile order: consecutive dispatch ids go round-robin over the 8
  // XCDs; give each XCD a contiguous run of strips so that neighbouring strips
  // (which share their halo of f) meet in the same L2.
  const int nt = a.nsx * a.nsy;
  int bid = blockIdx.x;
  {
    const int per = (nt + 7) / 8;
    const int xcd = bid % 8, loc = bid / 8;
    const int remapped = xcd * per + loc;
    bid = (nt % 8 == 0) ? remapped : bid;
  }
  const int sx = bid % a.nsx, sy = bid / a.nsx;
  const int x0 = sx * TW, y0 = sy * TH;

  for (int i = tid; i < a.taps_al; i += NT) s_taps[i] = i < ntp ? a.taps[i] : 0.0f;
  for (int i = tid; i < RS * RST; i += NT) s_ring[i] = 0.0f;
  for (int i = tid; i < TH * AST; i += NT) s_acc[i] = 0.0f;

  // ---- per-thread fixed roles --------------------------------------------
  // modulation: pixel slots tid + i*NT of the B x SW step tile
  // pass 1 item: channel ch, row rr, column block xb (P1 outputs)
  const int p1_ch = tid % NC;
  const int p1_rr = ((tid / NC) % 2) + 2 * (tid / (4 * NC));
  const int p1_xb = (tid / (2 * NC)) % 2;
  const int p1_k = p1_ch % 2, p1_m = p1_ch / 2;
  // pass 2 item: column x, pair m, row group g (P2 outputs)
  const int p2_x = tid % TW;
  const int p2_m = (tid / TW) % NP;
  int p2_g = tid / (TW * NP);
  if constexpr (TW * NP == 64) p2_g = __builtin_amdgcn_readfirstlane(p2_g);

  const int nmod = B * SW;
  const int Wd = a.W, Hd = a.H;

  // Modulation slots: pixel tid + i*NT of the B x SW step tile.  Their row,
  // column and column validity do not change between steps: precompute them.
  int m_rr[MI], m_off[MI], m_x[MI];
  bool m_xin[MI];
#pragma unroll
  for (int i = 0; i < MI; ++i) {
    const int pi = min(tid + i * NT, nmod - 1);
    m_rr[i] = pi / SW;
    const int j = pi - m_rr[i] * SW;
    m_off[i] = m_rr[i] * NC * SW + j;
    m_x[i] = x0 - R + j;
    m_xin[i] = tid + i * NT < nmod && j < TW + 2 * R && m_x[i] >= 0 && m_x[i] < Wd;
  }
  const int ybase = y0 - R;
  const float* fcol = a.f;

  // Prefetch registers: raw f of each slot for the next step.  Loads are
  // unconditional from a clamped (in-image) address so they stay in flight
  // across the passes; masking happens at use.
  float fcur[MI][D];
  auto load_step = [&](int s, float (&dst)[MI][D]) {
#pragma unroll
    for (int i = 0; i < MI; ++i) {
      if (i * NT < nmod) {  // wave-uniform: skip slots beyond the step tile
        const int y = min(max(ybase + s * B + m_rr[i], 0), Hd - 1);
        const int x = min(max(m_x[i], 0), Wd - 1);
        const float* src = fcol + ((size_t)y * Wd + x) * D;
#pragma unroll
        for (int m = 0; m < D; ++m) dst[i][m] = src[m];
      }
    }
  };
  load_step(0, fcur);
  __syncthreads();

  const int steps = a.steps, lag = a.lag;
  const float* termp = terms;
  for (int t = 0; t < a.K; ++t, termp += NP) {
    float wr[D];
#pragma unroll
    for (int m = 0; m < D; ++m) wr[m] = termp[m];
    const float tw = weights ? weights[t] : 1.0f;

    for (int s = 0; s < steps; ++s) {
      const int gs = t * steps + s;
      const int rslot = (gs % a.RSB) * B;
      const int cslot = (gs % a.CRB) * B;

      // ---- 1. modulation ---------------------------------------------------
#pragma unroll
      for (int i = 0; i < MI; ++i) {
        if (i * NT < nmod && tid + i * NT < nmod) {
          const int y = ybase + s * B + m_rr[i];
          const bool in = m_xin[i] && y >= 0 && y < Hd;
          float fv[D];
#pragma unroll
          for (int m = 0; m < D; ++m) fv[m] = in ? fcur[i][m] - a.cen[m] : 0.0f;
          float rho = 0.0f;
#pragma unroll
          for (int m = 0; m < D; ++m) rho = fmaf(wr[m], fv[m], rho);
          const float fr = __builtin_amdgcn_fractf(rho);
          float c = __builtin_amdgcn_cosf(fr), sn = __builtin_amdgcn_sinf(fr);
          c = in ? c : 0.0f;
          sn = in ? sn : 0.0f;
          float* st = s_stage + m_off[i];
#pragma unroll
          for (int m = 0; m < D; ++m) {
            st[(2 * m) * SW] = c * fv[m];
            st[(2 * m + 1) * SW] = sn * fv[m];
          }
          st[(2 * D) * SW] = c;
          st[(2 * D + 1) * SW] = sn;
          const int xc = m_x[i] - x0;
          if (xc >= 0 && xc < TW) {
            s_cs[(cslot + m_rr[i]) * CST + xc] = c;
            s_cs[(cslot + m_rr[i]) * CST + TW + xc] = sn;
          }
        }
      }
      // prefetch f for the next step (wrapping into the next term)
      {
        const int ns = (s + 1 == steps) ? 0 : s + 1;
        load_step(ns, fcur);
      }
      __syncthreads();

      // ---- 2. horizontal pass ------------------------------------------------
      // Sliding window of two 8-float blocks (ra | rb); each block is reloaded
      // right after its last use so the LDS latency hides behind 32+ FMAs.
      {
        const float* src = s_stage + (p1_rr * NC + p1_ch) * SW + p1_xb * P1;
        const int nblk = ntp / P1;                 // tap blocks; window needs nblk+1
        float acc[P1];
#pragma unroll
        for (int p = 0; p < P1; ++p) acc[p] = 0.0f;
        float ra[8], rb[8], ta[8], tb[8];
        ld8(ra, src);
        ld8(rb, src + 8);
        int b = 0;
        for (; b + 2 <= nblk; b += 2) {
          ld8(ta, s_taps + b * 8);
          ld8(tb, s_taps + b * 8 + 8);
          fma_lo<P1>(acc, ta, ra);
          ld8(ra, src + b * 8 + 16);                         // b + 2 <= nblk here
          fma_hi<P1>(acc, ta, rb);
          fma_lo<P1>(acc, tb, rb);
          ld8(rb, src + min(b + 3, nblk) * 8);               // clamped: no branch
          fma_hi<P1>(acc, tb, ra);
        }
        if (b < nblk) {
          ld8(ta, s_taps + b * 8);
          fma_lo<P1>(acc, ta, ra);
          fma_hi<P1>(acc, ta, rb);
        }
        float* dst = s_ring + (rslot + p1_rr) * RST + (p1_k * NP + p1_m) * TW + p1_xb * P1;
        *reinterpret_cast<float4*>(dst) = make_float4(acc[0], acc[1], acc[2], acc[3]);
        *reinterpret_cast<float4*>(dst + 4) = make_float4(acc[4], acc[5], acc[6], acc[7]);
      }
      __syncthreads();

      // ---- 3. vertical pass + demodulation -----------------------------------
      if (s >= lag) {
        const int ob = s - lag;                      // output block in the strip
        const int base = ((gs - lag) % a.RSB) * B + p2_g * P2;
        float a0[P2], a1[P2];
#pragma unroll
        for (int p = 0; p < P2; ++p) a0[p] = a1[p] = 0.0f;
        // column of this item in plane k = 0; plane k = 1 sits NP*TW further
        const float* col = s_ring + p2_m * TW + p2_x;
        const int nblk = ntp / P2;
        // ping-pong 4-row blocks (xa | xb), both planes
        float xa0[4], xa1[4], xb0[4], xb1[4], tq[8];
        auto ldblk = [&](float (&v0)[4], float (&v1)[4], int blk) {
          const float* r = col + wrap(base + blk * P2, RS) * RST;  // aligned block: no wrap inside
#pragma unroll
          for (int p = 0; p < 4; ++p) {
            v0[p] = r[p * RST];
            v1[p] = r[p * RST + NP * TW];
          }
        };
        ldblk(xa0, xa1, 0);
        ldblk(xb0, xb1, 1);
        int b = 0;
        for (; b + 2 <= nblk; b += 2) {
          ld8(tq, s_taps + b * 4);
          fma_lo<P2>(a0, tq, xa0);
          fma_lo<P2>(a1, tq, xa1);
          ldblk(xa0, xa1, b + 2);                            // b + 2 <= nblk here
          fma_hi<P2>(a0, tq, xb0);
          fma_hi<P2>(a1, tq, xb1);
          fma_lo<P2>(a0, tq + 4, xb0);
          fma_lo<P2>(a1, tq + 4, xb1);
          ldblk(xb0, xb1, min(b + 3, nblk));                 // clamped: no branch
          fma_hi<P2>(a0, tq + 4, xa0);
          fma_hi<P2>(a1, tq + 4, xa1);
        }
        if (b < nblk) {
          ld4(tq, s_taps + b * 4);
          fma_lo<P2>(a0, tq, xa0);
          fma_lo<P2>(a1, tq, xa1);
          fma_hi<P2>(a0, tq, xb0);
          fma_hi<P2>(a1, tq, xb1);
        }
        // demodulate with cos/sin at the output pixels (input row yo + R)
        const int cbase = ((gs - lag) % a.CRB) * B;
#pragma unroll
        for (int p = 0; p < P2; ++p) {
          const int yo = ob * B + p2_g * P2 + p;       // output row within strip
          const int crow = wrap(cbase + p2_g * P2 + p + R, CRS);
          const float c = s_cs[crow * CST + p2_x];
          const float sn = s_cs[crow * CST + TW + p2_x];
          float* ac = s_acc + yo * AST + p2_m * TW + p2_x;
          *ac = fmaf(tw * sn, a1[p], fmaf(tw * c, a0[p], *ac));
        }
      }
    }
  }
  __syncthreads();

  // ---- final division and store ---------------------------------------------
  for (int i = tid; i < TH * TW; i += NT) {
    const int yl = i / TW, xl = i - yl * TW;
    const int y = y0 + yl, x = x0 + xl;
    if (y < Hd && x < Wd) {
      const float* ac = s_acc + yl * AST + xl;
      const float Z = ac[D * TW];
      float* o = a.out + ((size_t)y * Wd + x) * D;
#pragma unroll
      for (int m = 0; m < D; ++m) o[m] = ac[m * TW] / Z + a.cen[m];
      if (a.num_out) {
        float* nn = a.num_out + ((size_t)y * Wd + x) * D;
#pragma unroll
        for (int m = 0; m < D; ++m) nn[m] = fmaf(a.cen[m], Z, ac[m * TW]);
      }
      if (a.z_out) a.z_out[(size_t)y * Wd + x] = Z;
    }
  }
}

// ---------------------------------------------------------------------------
// Host-side launch helpers for the fused kernel
// ---------------------------------------------------------------------------

size_t fused_lds_bytes(int d, int R, int TH) {
  const int NP = d + 1, NC = 2 * NP;
  const int ntp = ntaps_padded(R);
  const int SW = kTW + ntp + 4;
  const int lag = (2 * R + kB - 1) / kB;
  const int RS = (lag + 1) * kB, CRS = (lag + 2) * kB;
  const size_t fl = (size_t)((ntp + 3) / 4 * 4) + (size_t)kB * NC * SW +
                    (size_t)RS * 2 * NP * kTW + (size_t)CRS * 2 * kTW +
                    (size_t)TH * NP * kTW;
  return fl * sizeof(float);
}

template <int D>
static hipError_t launch_d(const FusedArgs& a, int nblocks, size_t lds, hipStream_t st) {
  auto kern = mcsf_fused_fp32<D>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(nblocks), dim3(64 * (D + 1)), lds, st, a, a.terms, a.weights);
  return hipGetLastError();
}

hipError_t launch_fused_fp32(int d, const FusedArgs& a, hipStream_t st) {
  const size_t lds = fused_lds_bytes(d, a.R, a.TH);
  const int nblocks = a.nsx * a.nsy;
  switch (d) {
    case 1: return launch_d<1>(a, nblocks, lds, st);
    case 2: return launch_d<2>(a, nblocks, lds, st);
    case 3: return launch_d<3>(a, nblocks, lds, st);
    case 4: return launch_d<4>(a, nblocks, lds, st);
    case 5: return launch_d<5>(a, nblocks, lds, st);
    case 6: return launch_d<6>(a, nblocks, lds, st);
    case 7: return launch_d<7>(a, nblocks, lds, st);
    case 8: return launch_d<8>(a, nblocks, lds, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace bfvec
