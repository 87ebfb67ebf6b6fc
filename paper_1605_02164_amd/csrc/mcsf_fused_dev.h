#pragma once

// Device code of the fused MCSF kernels and their instance dispatch,
// shared by the single-request (mcsf_fused.hip) and batched
// (mcsf_batch.hip) translation units.
//
// Fused MCSF kernel for gfx950 (CDNA4), FP32 channels.
//
// One workgroup owns a strip of TW output columns and TH output rows (TH is
// normally a large fraction of the image height).  For each of the K terms
// it streams down the strip in steps of B input rows; a step
//   1. modulates B haloed rows: theta = <w_t, f - c>, H = cos + i sin
//      (eq. (Ht)), writing the 2(d+1) real channels
//      {cos f_m, sin f_m (m < d), cos, sin} to a staging buffer (zero outside
//      the image: out-of-domain pixels contribute nothing);
//   2. runs the horizontal pass of the truncated separable Gaussian omega
//      over those rows into a ring holding the last RS rows;
//   3. once 2R rows of look-ahead are in the ring, runs the vertical pass for
//      B output rows and demodulates:
//      P_m += cos (omega * cos f_m) + sin (omega * sin f_m),
//      Z   += cos (omega * cos)     + sin (omega * sin)    (eqs. (numerator), (denom)),
//      adding into planar accumulators in device memory (Algorithm 1, P and Z).
// A separate finalize kernel divides (Algorithm 1, last step).
//
// Work per output pixel and term: 2(d+1)(2R+1) FMAs per pass.  On the VALU
// both passes are register-blocked sliding windows over LDS (4 outputs per
// item).  With R fixed at compile time the window loops unroll completely
// and the taps live in registers; a runtime-R variant serves every other
// radius.  At the compile-time radii the passes can also run as banded
// (Toeplitz) matrix products on the matrix cores (MF instances, below): both
// passes with 16-bit storage; in 32-column FP32 strips the horizontal pass
// from R = 12 and, from R = 21, both passes in a software pipeline with one
// barrier per step (PIPE, below).  A VALU instance of every width stays
// available (bf_opts.valu_only).
//
// Low-precision variants (PREC 1 = FP16, 2 = BF16) store the modulated
// channels and the horizontal-pass rows as 16-bit pairs; their VALU passes
// use v_dot2_f32_{f16,bf16}: two taps times two adjacent samples added into
// an FP32 accumulator.  With the taps split by parity, output 2q takes
// (w[2i], w[2i+1]) against samples (2q+2i, 2q+2i+1) and output 2q+1 takes
// (w[2i-1], w[2i]) against the same aligned pair, so every window read is an
// aligned 32-bit pair and each output costs R+1 dot2 instead of 2R+1 FMAs.
// Demodulation, accumulation and the division stay FP32.
//
// Variant 3 (FP32) runs the n-fold box filters (box, hat, three boxes; the
// paper allows any spatial filter in place of the Gaussian) with a vertical
// pass whose cost does not depend on the radius: the n-fold box sum over
// rows i-2R..i equals the sparse difference
//   v(i) = sum_{k=0..n} (-1)^k C(n,k) u(i - k(2r+1))
// of the horizontal-pass rows u, integrated n times (running sums).  The
// running sums are FP64 registers of a lane per (column, channel), reset at
// the top of each term's strip; n+1 ring reads and about 14 FP64 operations
// per output replace 2R+1 FMAs.  The horizontal pass stays a FIR over the box
// taps: inside a 16-column strip a running sum would still have to start 2R
// columns to the left.  (Measured on gfx950 this pass is slower than the FIR
// vertical pass at every radius up to 40, so the library runs box filters as
// FIR taps unless the running-sum pass is requested.)
//
// Variant 4 (FP32, three boxes, d = 3, 32-column strips asked for) runs the
// vertical pass as three cascaded sliding box sums and the horizontal pass
// on the matrix cores (described at its loop below).  It too measures slower
// than the FIR passes at R = 30, so the automatic strip width keeps variant 3.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "mcsf_common.h"

namespace bfvec {

namespace {

template <int D, int TW = kTW>
struct Geo {
  static constexpr int NP = D + 1;   // channel pairs (d numerators + Z)
  static constexpr int NC = 2 * NP;  // real channels
  static constexpr int NT = 64 * NP * (TW / 16);  // threads per workgroup
  static constexpr int MI = (kB * stage_width(kRMax, TW) + NT - 1) / NT;  // modulation slots
};

__device__ __forceinline__ int wrap(int r, int n) { return r >= n ? r - n : r; }

__device__ __forceinline__ void ld4(float* v, const float* p) {
  const float4 a = *reinterpret_cast<const float4*>(p);
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
}

// Sliding-window FMAs of a 4-output register block against taps t[0..3]:
// output p takes t[i] * window[p + i]; the window is two 4-blocks (lo | hi).
__device__ __forceinline__ void fma_lo(float (&acc)[4], const float* t, const float* lo) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int p = 0; p + i < 4; ++p) acc[p] = fmaf(t[i], lo[p + i], acc[p]);
}
__device__ __forceinline__ void fma_hi(float (&acc)[4], const float* t, const float* hi) {
#pragma unroll
  for (int i = 1; i < 4; ++i)
#pragma unroll
    for (int p = 4 - i; p < 4; ++p) acc[p] = fmaf(t[i], hi[p + i - 4], acc[p]);
}

// ---- 16-bit storage helpers --------------------------------------------------
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
typedef short short2_t __attribute__((ext_vector_type(2)));

template <int PREC>
__device__ __forceinline__ unsigned short to16(float x) {
  if constexpr (PREC == 1) return __builtin_bit_cast(unsigned short, (_Float16)x);
  else return __builtin_bit_cast(unsigned short, (__bf16)x);
}

// a.lo*b.lo + a.hi*b.hi + c, products and sum in FP32
template <int PREC>
__device__ __forceinline__ float dot2(unsigned a, unsigned b, float c) {
  if constexpr (PREC == 1)
    return __builtin_amdgcn_fdot2(__builtin_bit_cast(half2_t, a), __builtin_bit_cast(half2_t, b), c,
                                  false);
  else
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(short2_t, a),
                                           __builtin_bit_cast(short2_t, b), c, false);
}

__device__ __forceinline__ unsigned pack16(unsigned short lo, unsigned short hi) {
  return (unsigned)lo | ((unsigned)hi << 16);
}

// Swap lanes 32..63 of a with lanes 0..31 of b (v_permlane32_swap_b32).
// Written as a register-only instruction with both operands read and written:
// the compiler builtin's second result was dropped in generated code.  The
// s_nop pairs cover the VALU-write/permlane-read hazard windows.
__device__ __forceinline__ void swap_halves(unsigned& a, unsigned& b) {
  asm volatile("s_nop 4\n\tv_permlane32_swap_b32 %0, %1\n\ts_nop 4" : "+v"(a), "+v"(b));
}

// Exchange rows 1, 3 of a with rows 0, 2 of b (rows of 16 lanes;
// v_permlane16_swap_b32), written like swap_halves.
__device__ __forceinline__ void swap_rows16(unsigned& a, unsigned& b) {
  asm volatile("s_nop 4\n\tv_permlane16_swap_b32 %0, %1\n\ts_nop 4" : "+v"(a), "+v"(b));
}

// two FP32 values to one packed 16-bit pair (single v_cvt_pk_* instruction)
typedef float float2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
template <int PREC>
__device__ __forceinline__ unsigned pack2(float lo, float hi) {
  const float2_t v = {lo, hi};
  if constexpr (PREC == 1) return __builtin_bit_cast(unsigned, __builtin_convertvector(v, half2_t));
  else return __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2_t));
}

typedef float f32x4_t __attribute__((ext_vector_type(4)));
// x as an FP16 pair hi + lo: hi = x rounded to FP16, lo = the remainder
// x - hi rounded to FP16 (exact in FP32), so hi + lo carries about 22
// significant bits (fewer where lo is subnormal, |x| < 2^-3: an absolute
// error below 2^-25 there).
__device__ __forceinline__ void split16(float x, unsigned short& h, unsigned short& l) {
  const _Float16 hh = (_Float16)x;
  const _Float16 ll = (_Float16)(x - (float)hh);
  h = __builtin_bit_cast(unsigned short, hh);
  l = __builtin_bit_cast(unsigned short, ll);
}
// 16x16x4 FP32 product: lane l holds a[l%16][l/16], b[l/16][l%16] and d as
// above.
__device__ __forceinline__ f32x4_t mfma4(float a, float b, f32x4_t d) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, d, 0, 0, 0);
}
// 16x16x32 form (gfx950): eight 16-bit values per lane, a[l%16][8(l/16)+v],
// b[8(l/16)+v][l%16]; d as above.
typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
template <int PREC>
__device__ __forceinline__ f32x4_t mfma32(uint4 a, uint4 b, f32x4_t d) {
  if constexpr (PREC == 1)
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(half8_t, a),
                                                  __builtin_bit_cast(half8_t, b), d, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                   __builtin_bit_cast(bf16x8_t, b), d, 0, 0, 0);
}
// Four outputs (p = 0..3, starting at an even sample) of a 2R+1-tap window
// over aligned sample pairs x2[j] = (x[2j], x[2j+1]):
//   out[2q]   = sum_i te[i] . x2[q+i],   te[i] = (w[2i],   w[2i+1])
//   out[2q+1] = sum_i to[i] . x2[q+i],   to[i] = (w[2i-1], w[2i])
template <int PREC, int R>
__device__ __forceinline__ void window4_lp(const unsigned* x2, const unsigned* te, const unsigned* to,
                                           float (&acc)[4]) {
#pragma unroll
  for (int i = 0; i <= R; ++i) {
    acc[0] = dot2<PREC>(te[i], x2[i], acc[0]);
    acc[1] = dot2<PREC>(to[i], x2[i], acc[1]);
    acc[2] = dot2<PREC>(te[i], x2[i + 1], acc[2]);
    acc[3] = dot2<PREC>(to[i], x2[i + 1], acc[3]);
  }
}

// Horizontal pass, 16-bit storage: src points at the dword holding samples
// (first output, first output + 1) of the window start.
template <int PREC, int RC>
__device__ __forceinline__ void hpass_lp(const unsigned* src, const unsigned* te, const unsigned* to,
                                         const unsigned* s_te, const unsigned* s_to, int R,
                                         float (&acc)[4]) {
  if constexpr (RC >= 0) {
    constexpr int NWD = RC + 2, NL = (NWD + 1) / 2;
    unsigned x2[2 * NL];
#pragma unroll
    for (int j = 0; j < NL; ++j) {
      const uint2 v = *reinterpret_cast<const uint2*>(src + 2 * j);
      x2[2 * j] = v.x;
      x2[2 * j + 1] = v.y;
    }
    window4_lp<PREC, RC>(x2, te, to, acc);
  } else {
    unsigned cur = src[0];
    for (int i = 0; i <= R; ++i) {
      const unsigned nxt = src[i + 1];
      const unsigned ei = s_te[i], oi = s_to[i];
      acc[0] = dot2<PREC>(ei, cur, acc[0]);
      acc[1] = dot2<PREC>(oi, cur, acc[1]);
      acc[2] = dot2<PREC>(ei, nxt, acc[2]);
      acc[3] = dot2<PREC>(oi, nxt, acc[3]);
      cur = nxt;
    }
  }
}

// Vertical pass, 16-bit storage: the ring holds row pairs (even row in the
// low half); col points at this item's channel column in pair-row 0, pb is
// the pair-row of the first window row; pair-rows wrap at RSP (blocks of two
// pair-rows are aligned and never straddle the wrap).
template <int PREC, int RC, int RSTD>
__device__ __forceinline__ void vpass_lp(const unsigned* col, int pb, int RSP, const unsigned* te,
                                         const unsigned* to, const unsigned* s_te,
                                         const unsigned* s_to, int R, float (&acc)[4]) {
  if constexpr (RC >= 0) {
    constexpr int NWD = RC + 2, NB = (NWD + 1) / 2;
    unsigned y2[2 * NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const unsigned* r = col + wrap(pb + 2 * b, RSP) * RSTD;
      y2[2 * b] = r[0];
      y2[2 * b + 1] = r[RSTD];
    }
    window4_lp<PREC, RC>(y2, te, to, acc);
  } else {
    unsigned cur = col[wrap(pb, RSP) * RSTD];
    for (int i = 0; i <= R; ++i) {
      const unsigned nxt = col[wrap(pb + i + 1, RSP) * RSTD];
      const unsigned ei = s_te[i], oi = s_to[i];
      acc[0] = dot2<PREC>(ei, cur, acc[0]);
      acc[1] = dot2<PREC>(oi, cur, acc[1]);
      acc[2] = dot2<PREC>(ei, nxt, acc[2]);
      acc[3] = dot2<PREC>(oi, nxt, acc[3]);
      cur = nxt;
    }
  }
}

// Horizontal pass of one item: 4 consecutive outputs of one channel of one
// row; src points at the staging column of the first output's window start.
template <int RC>
__device__ __forceinline__ void hpass(const float* src, const float* tapr, const float* s_taps,
                                      int ntap4, float (&acc)[4]) {
  if constexpr (RC >= 0) {
    constexpr int NW = 2 * RC + 4, NB = (NW + 3) / 4;
    float x[NB * 4];
#pragma unroll
    for (int b = 0; b < NB; ++b) ld4(x + 4 * b, src + 4 * b);
#pragma unroll
    for (int u = 0; u <= 2 * RC; ++u)
#pragma unroll
      for (int p = 0; p < 4; ++p) acc[p] = fmaf(tapr[u <= RC ? u : 2 * RC - u], x[p + u], acc[p]);
  } else {
    const int nblk = ntap4 / 4;
    float ra[4], rb[4], t[8];
    ld4(ra, src);
    ld4(rb, src + 4);
    int b = 0;
    for (; b + 2 <= nblk; b += 2) {
      ld4(t, s_taps + 4 * b);
      ld4(t + 4, s_taps + 4 * b + 4);
      fma_lo(acc, t, ra);
      ld4(ra, src + 4 * b + 8);                       // b + 2 <= nblk here
      fma_hi(acc, t, rb);
      fma_lo(acc, t + 4, rb);
      ld4(rb, src + 4 * min(b + 3, nblk));            // clamped: no branch
      fma_hi(acc, t + 4, ra);
    }
    if (b < nblk) {
      ld4(t, s_taps + 4 * b);
      fma_lo(acc, t, ra);
      fma_hi(acc, t, rb);
    }
  }
}

// Vertical pass of one item: 4 consecutive output rows of one channel of one
// column.  col points at the channel column in ring row 0; rb is the ring row
// of the first window row; ring rows wrap at RS (window blocks of 4 rows are
// aligned, so a block never straddles the wrap).
template <int RC, int RST>
__device__ __forceinline__ void vpass(const float* col, int rb, int RS, const float* tapr,
                                      const float* s_taps, int ntap4, float (&acc)[4]) {
  if constexpr (RC >= 0) {
    constexpr int NW = 2 * RC + 4, NB = (NW + 3) / 4;
    float x[NB * 4];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const float* r = col + wrap(rb + 4 * b, RS) * RST;
#pragma unroll
      for (int i = 0; i < 4; ++i) x[4 * b + i] = r[i * RST];
    }
#pragma unroll
    for (int u = 0; u <= 2 * RC; ++u)
#pragma unroll
      for (int p = 0; p < 4; ++p) acc[p] = fmaf(tapr[u <= RC ? u : 2 * RC - u], x[p + u], acc[p]);
  } else {
    const int nblk = ntap4 / 4;
    auto ldb = [&](float* v, int blk) {
      const float* r = col + wrap(rb + 4 * blk, RS) * RST;
#pragma unroll
      for (int i = 0; i < 4; ++i) v[i] = r[i * RST];
    };
    float ra[4], rbv[4], t[8];
    ldb(ra, 0);
    ldb(rbv, 1);
    int b = 0;
    for (; b + 2 <= nblk; b += 2) {
      ld4(t, s_taps + 4 * b);
      ld4(t + 4, s_taps + 4 * b + 4);
      fma_lo(acc, t, ra);
      ldb(ra, b + 2);
      fma_hi(acc, t, rbv);
      fma_lo(acc, t + 4, rbv);
      ldb(rbv, min(b + 3, nblk));
      fma_hi(acc, t + 4, ra);
    }
    if (b < nblk) {
      ld4(t, s_taps + 4 * b);
      fma_lo(acc, t, ra);
      fma_hi(acc, t, rbv);
    }
  }
}

}  // namespace

// Buffer-resource access with 32-bit byte offsets (raw buffer, no stride):
// the address arithmetic stays 32-bit.  Offsets must stay below 4 GiB (the
// planner limits images accordingly).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, -1, 0x00020000);
}
// One pixel's D channels: D dword loads from one address register with
// immediate offsets.  (The 96-bit buffer-load builtin compiled to a single
// dword load in this toolchain, so wide loads are not used.)
template <int D>
__device__ __forceinline__ void buf_load_px(__amdgpu_buffer_rsrc_t r, unsigned byte_off, float (&v)[D]) {
#pragma unroll
  for (int m = 0; m < D; ++m)
    v[m] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)(byte_off + 4 * m), 0, 0));
}
__device__ __forceinline__ float buf_load1(__amdgpu_buffer_rsrc_t r, unsigned byte_off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)byte_off, 0, 0));
}
__device__ __forceinline__ void buf_store1(__amdgpu_buffer_rsrc_t r, unsigned byte_off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)byte_off, 0, 0);
}
// The same with the address split into a per-lane part (voff, a VGPR kept
// across the loop) and a wave-uniform part (soff, an SGPR): the uniform row
// offsets of a step then cost no vector instructions.
__device__ __forceinline__ float buf_load1s(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ void buf_store1s(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff,
                                            float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)voff, (int)soff, 0);
}

// Read-only table entry through the constant address space: a uniform index
// then becomes a scalar load.
__device__ __forceinline__ float ld_const(const float* p, int i) {
  typedef const __attribute__((address_space(4))) float cfloat;
  return ((cfloat*)p)[i];
}

// One workgroup: strip `bid` of the request described by `a`, terms
// a.t0 .. a.t1-1 (Algorithm 1's term loop over one strip).
// RC: window radius fixed at compile time, or -1 for a runtime radius.
// PREC: 0 FP32 channels; 1 FP16 / 2 BF16 storage of channels and ring rows.
// MF: the passes on the matrix cores, at a compile-time radius: both with
// 16-bit storage (either strip width), the horizontal one for FP32 (32-column
// strips).
template <int D, int RC, int PREC, bool P64, int TW = kTW, bool MF = false>
__device__ __forceinline__ void fused_strip(const FusedArgs& a, int bid) {
  static_assert(PREC >= 0 && PREC <= 5, "kernel variant");
  static_assert(PREC != 5 || (TW == 32 && MF && D == 3 && RC >= 18),
                "split vertical pass: pipelined 32-column FP32 instances");
  static_assert(TW == 16 || (TW == 32 && (2 * (D + 1)) % 4 == 0 && PREC != 3), "strip width");
  static_assert(PREC != 4 || (TW == 32 && MF && D == 3 && RC >= 0 && RC % 3 == 0),
                "sliding three-box vertical pass: 32-column matrix-core instances");
  static_assert(!MF || (RC >= 0 && (TW == 32 ? D == 3 && (PREC <= 2 || PREC == 4 || PREC == 5)
                                             : PREC == 1 || PREC == 2)),
                "matrix-core passes");
  using G = Geo<D, TW>;
  constexpr int NP = G::NP, NC = G::NC, NT = G::NT, MI = G::MI;
  constexpr int B = kB;
  constexpr bool MFV = MF && (PREC == 1 || PREC == 2);   // vertical pass on the matrix cores too
  // PIPE (FP32 matrix-core instances, R >= 21; variant 5 from R = 18): both passes on the matrix
  // cores, the vertical one over pairs of steps (16 output rows), and one
  // barrier per step (the loop below).  That needs two staging buffers and
  // two more ring steps: step g is written while the pair's window, steps
  // g - 2 - lag .. g - 1, is read.  Its ring rows are padded by 16 floats:
  // an operand read of the vertical pass touches 4 consecutive rows x 16
  // columns, which a stride of 16 mod 32 floats spreads over the LDS banks.
  constexpr bool PIPE = use_pipe(PREC, RC, MF);
  // Variant 5: the ring holds the horizontal-pass rows as FP16 pairs hi + lo
  // in two planes, and the vertical pass runs on FP16 products.  A plane
  // holds one slot per 8-row step, [ch][x][q] with q the step's pair-row
  // (rows 2q, 2q+1 as the low and high halves of a dword): the 4 dwords a
  // lane's product operand needs (8 consecutive rows of one column) are
  // then one 128-bit read.  RST: dwords per row pair over all slots' width
  // (NC x TW), so that a plane is RS/2 x RST dwords.
  constexpr bool SPV = PREC == 5;
  constexpr int RST = NC * TW + (MFV ? kRingPadMF : 0) +
                      (PIPE && !SPV ? kRingPadPipe : 0);   // ring row stride: [ch][x]
  constexpr int CST = 2 * TW + cs_row_pad(PIPE || (MFV && TW == 32));   // cos/sin ring row: [k][x]
  constexpr bool LP = PREC == 1 || PREC == 2;   // 16-bit storage
  constexpr bool VB = PREC == 3;                 // running-sum vertical pass
  // Variant 4 (FP32, three boxes, 32-column strips): horizontal pass on the
  // matrix cores over the box taps; vertical pass as three cascaded sliding
  // box sums, O(1) operations per output whatever the radius (below).
  constexpr bool SLV = PREC == 4;
  constexpr int SLW = SLV ? 2 * (RC / 3) + 1 : 1;   // box width 2r + 1 (R = 3r)
  constexpr int SL_RS = (SLW + 16 + 7) / 8 * 8;      // ring: rows i - w .. newest step
  constexpr int SL_CRS = (RC + 24 + 7) / 8 * 8;      // cos/sin: rows i - R .. newest step
  constexpr int SL_S1R = (2 * SLW + 8 + 7) / 8 * 8;  // first-stage sums: rows i - 2w .. i
  constexpr int NTAPR = (RC >= 0 && !LP) ? RC + 1 : 1;    // taps 0..R (symmetric)
  constexpr int NTAPP = (RC >= 0 && LP) ? RC + 1 : 1;   // packed tap pairs

  extern __shared__ float4 lds4[];
  float* lds = reinterpret_cast<float*>(lds4);
  const int R = RC >= 0 ? RC : a.R;
  const int SW = RC >= 0 ? (MF ? (LP ? stage_width_mf(RC) : stage_width_mf32(RC))
                               : LP ? stage_width16(RC, TW) : stage_width(RC, TW))
                          : a.SW;
  const int MW = RC >= 0 ? TW + 2 * RC : SW;   // modulated columns per staging row
  const int ntap4 = (2 * R + 1 + 3) / 4 * 4;
  const int taps_al = (ntap4 + 7) / 8 * 8;
  const int tapp_al = (R + 1 + 3) / 4 * 4;
  const int CRB = PIPE ? pipe_cs_steps(RC) : a.CRB;
  const int RS = SLV ? SL_RS : (a.RSB + (PIPE ? 2 : 0)) * B, CRS = SLV ? SL_CRS : CRB * B;
  // LDS carve-up: FP32 taps | packed tap pairs (16-bit modes) | staging (two
  // buffers with PIPE) | ring | cos/sin ring.  16-bit modes store the ring as
  // row pairs.
  const int stage_floats = LP ? B * NC * SW / 2 : B * NC * SW;
  float* s_taps = lds;
  unsigned* s_te = reinterpret_cast<unsigned*>(s_taps + taps_al);
  unsigned* s_to = s_te + (LP ? tapp_al : 0);
  float* s_stage = reinterpret_cast<float*>(s_to + (LP ? tapp_al : 0));
  unsigned short* s_stage16 = reinterpret_cast<unsigned short*>(s_stage);
  float* s_ring = s_stage + stage_floats * (PIPE || SLV ? 2 : 1);
  unsigned* s_ring32 = reinterpret_cast<unsigned*>(s_ring);
  unsigned short* s_ring16 = reinterpret_cast<unsigned short*>(s_ring);
  float* s_s1 = s_ring + (LP ? RS / 2 : RS) * RST;   // variant 4: first-stage sums [row][ch][x]
  float* s_cs = s_s1 + (SLV ? SL_S1R * NC * TW : 0);
  float* s_vr = s_cs + CRS * CST;   // variant 3: 16-row ring of vertical-pass outputs

  const int tid = threadIdx.x;
  const int sx = bid % a.nsx, sy = bid / a.nsx;
  const int x0 = sx * TW, y0 = sy * a.TH;
  const int Wd = a.W, Hd = a.H;

  for (int i = tid; i < taps_al; i += NT) s_taps[i] = i < 2 * R + 1 ? a.taps[i] : 0.0f;
  for (int i = tid; i < (LP ? RS / 2 : RS) * RST + (SLV ? SL_S1R * NC * TW : 0); i += NT)
    s_ring[i] = 0.0f;   // ring, and the first-stage sums of variant 4 (read before written)
  for (int i = tid; i < (PIPE || SLV ? 2 : 1) * B * NC * (SW - MW); i += NT) {   // staging padding columns
    const int row = i / (SW - MW), col = MW + i % (SW - MW);   // rows of both buffers (PIPE)
    if constexpr (LP) s_stage16[row * SW + col] = 0;
    else s_stage[row * SW + col] = 0.0f;
  }
  __syncthreads();
  if constexpr (LP) {
    // tap pairs by parity: te[i] = (w[2i], w[2i+1]), to[i] = (w[2i-1], w[2i]),
    // with w[-1] = w[2R+1] = 0
    for (int i = tid; i < tapp_al; i += NT) {
      const float w0 = 2 * i <= 2 * R ? s_taps[2 * i] : 0.0f;
      const float w1 = 2 * i + 1 <= 2 * R ? s_taps[2 * i + 1] : 0.0f;
      const float wm = i > 0 && 2 * i - 1 <= 2 * R ? s_taps[2 * i - 1] : 0.0f;
      s_te[i] = pack16(to16<PREC>(w0), to16<PREC>(w1));
      s_to[i] = pack16(to16<PREC>(wm), to16<PREC>(w0));
    }
    __syncthreads();
  }
  float tapr[NTAPR];
#pragma unroll
  for (int u = 0; u < NTAPR; ++u) tapr[u] = s_taps[u];
  // 16-bit tap pairs: the even-parity pairs as scalar operands (SGPRs), the
  // odd-parity ones in VGPRs (an opaque move keeps the compiler from also
  // making them scalar: with both sets in SGPRs it ran out and spilled other
  // scalars to VGPR lanes).  v_dot2 takes no operand-select modifiers on
  // gfx950, so the odd pairs cannot be derived from the even ones for free.
  unsigned tpe[NTAPP], tpo[NTAPP];
#pragma unroll
  for (int i = 0; i < NTAPP; ++i) {
    tpe[i] = LP ? __builtin_amdgcn_readfirstlane(s_te[i]) : 0u;
    unsigned v = LP ? s_to[i] : 0u;
    asm("v_mov_b32 %0, %1" : "=v"(v) : "v"(v));
    tpo[i] = v;
  }
  // Matrix-core passes: constant tap operands of the banded products.
  // Horizontal: out[m][x] = sum_j stage[m][j] w[j - x] over k-blocks of 32
  // samples (KSH of them cover 16 + 2R); this lane holds the B rows
  // k = 8(l/16)+v (v = 0..7) of column x = l%16.  Vertical: out[r][n] =
  // sum_i w[i - r] ring[i][n] over KSV k-blocks of 32 covering B + 2R ring
  // rows; this lane holds the A row r = l%16 (rows 8-15 zero: a step has 8
  // output rows).  FP32 horizontal pass: k-blocks of 4 samples.
  constexpr int KSH = MFV ? (16 + 2 * RC + 31) / 32 : 1;
  constexpr int KSV = MFV ? (kB + 2 * RC + 31) / 32 : 1;
  // FP32 horizontal pass: k-blocks of 4 samples, one tap per lane and block
  constexpr int KS4 = (MF && !LP) ? (16 + 2 * RC + 3) / 4 : 1;
  uint4 hb[KSH], va[KSV];
  float hb4[KS4];
  if constexpr (MF && !LP) {
    const int ln = tid & 63;
#pragma unroll
    for (int s = 0; s < KS4; ++s) {
      const int u = 4 * s + (ln >> 4) - (ln & 15);
      hb4[s] = u >= 0 && u <= 2 * RC ? s_taps[u] : 0.0f;
    }
  }
  if constexpr (MFV) {
    const int ln = tid & 63;
    auto tap16 = [&](int u, bool on) -> unsigned {
      return (unsigned)to16<PREC>(on && u >= 0 && u <= 2 * RC ? s_taps[u] : 0.0f);
    };
#pragma unroll
    for (int s = 0; s < KSH; ++s) {
      const int u = 32 * s + 8 * (ln >> 4) - (ln & 15);
      hb[s] = make_uint4(tap16(u, true) | tap16(u + 1, true) << 16,
                         tap16(u + 2, true) | tap16(u + 3, true) << 16,
                         tap16(u + 4, true) | tap16(u + 5, true) << 16,
                         tap16(u + 6, true) | tap16(u + 7, true) << 16);
    }
#pragma unroll
    for (int s = 0; s < KSV; ++s) {
      const int u = 32 * s + 8 * (ln >> 4) - (ln & 15);
      const bool on = (ln & 15) < kB;
      va[s] = make_uint4(tap16(u, on) | tap16(u + 1, on) << 16,
                         tap16(u + 2, on) | tap16(u + 3, on) << 16,
                         tap16(u + 4, on) | tap16(u + 5, on) << 16,
                         tap16(u + 6, on) | tap16(u + 7, on) << 16);
    }
  }

  // Variant 5: tap operands of the vertical FP16 products, as hi and lo
  // halves: A[r][k] = w[32s + k - r] for the pair's 16 output rows r and the
  // 32 window rows k of k-block s (KBS blocks cover the 16 + 2R rows); this
  // lane holds row r = l%16, k = 8(l/16) .. +7.
  constexpr int KBS = SPV ? (16 + 2 * RC + 31) / 32 : 1;
  uint4 vah[KBS], val[KBS];
  if constexpr (SPV) {
    const int ln = tid & 63;
    auto tap = [&](int u, bool lo) -> unsigned {
      unsigned short h, l;
      split16(u >= 0 && u <= 2 * RC ? s_taps[u] : 0.0f, h, l);
      return lo ? l : h;
    };
#pragma unroll
    for (int s = 0; s < KBS; ++s) {
      const int u = 32 * s + 8 * (ln >> 4) - (ln & 15);
      vah[s] = make_uint4(tap(u, false) | tap(u + 1, false) << 16,
                          tap(u + 2, false) | tap(u + 3, false) << 16,
                          tap(u + 4, false) | tap(u + 5, false) << 16,
                          tap(u + 6, false) | tap(u + 7, false) << 16);
      val[s] = make_uint4(tap(u, true) | tap(u + 1, true) << 16, tap(u + 2, true) | tap(u + 3, true) << 16,
                          tap(u + 4, true) | tap(u + 5, true) << 16, tap(u + 6, true) | tap(u + 7, true) << 16);
    }
  }
  // Variant 5: this lane's ring store offset in halves within a step slot:
  // dword ((g/2) TW + x) 4 + mb of the slot, half g & 1 (see hmf_store)
  const int spv_st = [&] {
    const int ln = tid & 63, mb = (tid >> 6) % NP, nb = (tid >> 6) / NP, g = ln >> 4;
    return 2 * (((g >> 1) * TW + 16 * nb + (ln & 15)) * 4 + mb) + (g & 1);
  }();
  // ---- per-thread fixed roles -------------------------------------------------
  // pass 1 item: 4-column block xq, channel ch, row rr of the step.  xq varies
  // fastest across lanes: the items' 128-bit ring writes then cover contiguous
  // LDS (a channel-fastest order measured a 7-way bank conflict on them).
  // Wide strips: 8 blocks x 4 channels x a row pair per wave, the pair's rows
  // in lanes l and l + 32 (as for d = 3 in 16-column strips).
  int p1_xq, p1_ch, p1_rr;
  if constexpr (TW == 16) {
    p1_xq = tid % 4;
    p1_ch = (tid / 4) % NC;
    p1_rr = tid / (4 * NC);
  } else {
    const int wv = tid >> 6;
    p1_xq = tid % 8;
    p1_ch = (wv % (NC / 4)) * 4 + (tid / 8) % 4;
    p1_rr = 2 * (wv / (NC / 4)) + ((tid >> 5) & 1);
  }
  // pass 2 item: column x, cos/sin half k, pair m, 4-row group g (the cos and
  // sin halves of a column in lanes TW apart)
  constexpr int LTW = TW == 16 ? 4 : 5;
  const int p2_x = tid & (TW - 1);
  const int p2_k = (tid >> LTW) & 1;
  const int p2_m = (tid >> (LTW + 1)) % NP;
  int p2_g = (tid >> (LTW + 1)) / NP;
  if constexpr (NP % 2 == 0 || TW == 32) p2_g = __builtin_amdgcn_readfirstlane(p2_g);
  const int p2_ch = 2 * p2_m + p2_k;
  // accumulators: planar [m][Hp][Wp] padded to whole strips, so every lane
  // owns valid storage; 32-bit element offsets from the (uniform) base
  const int Wp = a.nsx * TW;
  // matrix-core vertical pass: wave w filters pair w/(TW/16) over columns
  // 16(w%(TW/16)) .. +15; lanes 0-31 hold output rows 4(l/16) .. +3 of the step
  const int mf_m = (tid >> 6) / (TW / 16), mf_x = 16 * ((tid >> 6) % (TW / 16)) + (tid & 15);
  const int mf_r0 = 4 * ((tid >> 4) & 1);
  const bool mf_on = (tid & 63) < 32;
  const unsigned acc_lane =
      MFV ? (unsigned)(mf_m * a.Hp + y0 + mf_r0) * Wp + x0 + mf_x
         : (unsigned)(p2_m * a.Hp + y0 + 2 * p2_k) * Wp + x0 + p2_x;
  // matrix-core vertical pass: this lane's operand column in the ring, and
  // its pair-row group 4g (g = (lane / 16) % 4) within a k-block
  const int mf_g4 = 4 * ((tid >> 4) & 3);
  const int mfv_lane = (2 * mf_m) * TW + mf_x + mf_g4 * RST;
  // matrix-core horizontal pass with 16-bit storage (d = 3): this lane's
  // ring offset in halves, without the step's rows (the store below)
  const int hs_lane = [&] {
    const int ln = tid & 63, mb = (tid >> 6) % NP, nb = (tid >> 6) / NP, g = ln >> 4;
    return 2 * (mb * RST + 4 * (g & 1) * TW + 16 * nb + (ln & 15)) + (g >> 1);
  }();
  // variant 3: running sums of one (column, channel) per lane of the first
  // 16*NC lanes; sparse-difference weights (-1)^k C(n,k), offsets k(2r+1)
  const int vb_x = tid & 15, vb_ch = tid >> 4;
  const bool vb_on = VB && vb_ch < NC;
  const int vn = VB ? a.vbox : 1;
  const int vw = VB ? 2 * (R / vn) + 1 : 1;
  // weights of the lags (zero past n) and 0/1 weights picking running sum n
  const double vc1 = -vn, vc2 = vn == 2 ? 1.0 : vn == 3 ? 3.0 : 0.0, vc3 = vn == 3 ? -1.0 : 0.0;
  const double ve1 = vn == 1 ? 1.0 : 0.0, ve2 = vn == 2 ? 1.0 : 0.0, ve3 = vn == 3 ? 1.0 : 0.0;
  double vI1 = 0.0, vI2 = 0.0, vI3 = 0.0;

  // Modulation slots: pixel tid + i*NT of the B x MW step tile.  With R fixed
  // the passes read only the TW + 2R window columns; the runtime-R loops also
  // read zero-tap padding, so they modulate the whole row.  Columns beyond MW
  // are zeroed once below and never written again.
  const int nmod = B * MW;
  int m_rr[MI], m_off[MI], m_x[MI];
  bool m_xin[MI];
#pragma unroll
  for (int i = 0; i < MI; ++i) {
    const int pi = min(tid + i * NT, nmod - 1);
    m_rr[i] = pi / MW;
    const int j = pi - m_rr[i] * MW;
    m_off[i] = m_rr[i] * NC * SW + j;
    m_x[i] = x0 - R + j;
    m_xin[i] = tid + i * NT < nmod && j < TW + 2 * R && m_x[i] >= 0 && m_x[i] < Wd;
  }
  const int ybase = y0 - R;
  // cos/sin ring slot of each modulation slot whose column is an output
  // column (row within the step, column): a per-lane offset from the ring
  // row of the step
  int m_cs[MI];
  bool m_csin[MI];
#pragma unroll
  for (int i = 0; i < MI; ++i) {
    const int xc = m_x[i] - x0;
    m_csin[i] = xc >= 0 && xc < TW;
    m_cs[i] = m_rr[i] * CST + xc;
  }

  // Prefetch buffers, two steps deep (ping-pong A/B by step parity): raw f of
  // each modulation slot, loaded from a clamped in-image address so the loads
  // stay in flight across the passes, and this lane's accumulators for the
  // output rows of the step.
  const int steps = a.steps, lag = a.lag, t0 = a.t0, t1 = a.t1;
  float cen[D];   // per-channel centre: kernel argument, or device memory (graph plans)
#pragma unroll
  for (int m = 0; m < D; ++m) cen[m] = a.cen_dev ? ld_const(a.cen_dev, m) : a.cen[m];
  const unsigned frow = (unsigned)a.fpitch * D;  // floats per row of f
  float fA[MI][D], fB[MI][D];
  // accumulators of this lane's output rows: 2 rows, or 4 (lanes 0-31) with
  // the matrix-core vertical pass
  constexpr int NACC = MFV ? 4 : 2;
  float aA[NACC], aB[NACC];
#pragma unroll
  for (int v = 0; v < NACC; ++v) aA[v] = aB[v] = 0.0f;
  int m_fx[MI];  // clamped column offset of each slot, in floats
#pragma unroll
  for (int i = 0; i < MI; ++i) m_fx[i] = min(max(m_x[i], 0), Wd - 1) * D;
  const __amdgpu_buffer_rsrc_t f_rsrc = buf_rsrc(a.f), acc_rsrc = buf_rsrc(a.acc);
  auto load_f = [&](float (&dst)[MI][D], int s) {
#pragma unroll
    for (int i = 0; i < MI; ++i) {
      if (i * NT < nmod) {
        const int y = min(max(ybase + s * B + m_rr[i], 0), Hd - 1);
        const unsigned o = (unsigned)y * frow + (unsigned)m_fx[i];
        buf_load_px<D>(f_rsrc, 4u * o, dst[i]);
      }
    }
  };
  // The accumulator loads are issued by every lane in every step, whether
  // or not the value is used (t = 0, t past the range, s < lag, the upper
  // half of a matrix-core wave): the addresses are always rows of this strip
  // (s < lag reads its first output step; upper lanes repeat the lower
  // lanes' rows).  Without a branch around them the compiler knows how many
  // memory operations follow each prefetch, and the modulation's wait for
  // its f values no longer also waits for the accumulators just requested.
  auto load_acc = [&](float (&dst)[NACC], int t, int s) {
    (void)t;
    const int so = max(s - lag, 0);
    if constexpr (MFV) {
#pragma unroll
      for (int v = 0; v < 4; ++v)
        dst[v] = buf_load1s(acc_rsrc, 4u * acc_lane, 4u * (unsigned)(so * B + v) * Wp);
    } else {
      const unsigned o = acc_lane + (unsigned)(so * B + p2_g * 4) * Wp;
      dst[0] = buf_load1(acc_rsrc, 4u * o);
      dst[1] = buf_load1(acc_rsrc, 4u * (o + Wp));
    }
  };

  // ring positions of the current step (rows written) and of the step lag
  // behind it (rows the vertical pass starts from), advanced by B per step
  const int RSBk = RS / B;
  int rslot = 0, cslot = 0;
  int rslot_lag = (RSBk - lag % RSBk) % RSBk * B, cslot_lag = (CRB - lag % CRB) % CRB * B;
  float wr[D];       // frequencies of the term being modulated
  float tw = 1.0f;   // weight of the term being demodulated
  auto load_wr = [&](int t) {
#pragma unroll
    for (int m = 0; m < D; ++m) wr[m] = ld_const(a.terms, t * NP + m);
  };
  auto load_tw = [&](int t) { tw = a.weights ? ld_const(a.weights, t) : 1.0f; };
  auto load_term = [&](int t) {
    load_wr(t);
    load_tw(t);
  };

  // ---- 1. modulation of step s of term t from the prefetched f values
  // fcur into the staging buffer stg (16-bit modes: its 16-bit view) and
  // the cos/sin ring rows at cs0 ------------------------------------------------
  auto modulate = [&](int t, int s, const float (&fcur)[MI][D], float* stg, int cs0) {
    unsigned short* stg16 = reinterpret_cast<unsigned short*>(stg);
#pragma unroll
    for (int i = 0; i < MI; ++i) {
      if (i * NT < nmod && tid + i * NT < nmod) {
        const int y = ybase + s * B + m_rr[i];
        const bool in = m_xin[i] && y >= 0 && y < Hd;
        float fv[D];
#pragma unroll
        for (int m = 0; m < D; ++m) fv[m] = fcur[i][m] - cen[m];
        float rho = 0.0f;
#pragma unroll
        for (int m = 0; m < D; ++m) rho = fmaf(wr[m], fv[m], rho);
        float fr = __builtin_amdgcn_fractf(rho);
        if (P64 && fabsf(rho) > kPhaseExact) {
          // beyond 2^8 turns the FP32 phase keeps too few fraction bits:
          // reduce it in FP64 from w/2pi to ~48 bits (FP32 value + remainder)
          // and the exact difference f - c
          double rd = 0.0;
#pragma unroll
          for (int m = 0; m < D; ++m)
            rd = fma((double)wr[m] + (double)ld_const(a.terms_lo, t * NP + m),
                     (double)fcur[i][m] - (double)cen[m], rd);
          fr = (float)(rd - floor(rd));
        }
        float c = __builtin_amdgcn_cosf(fr), sn = __builtin_amdgcn_sinf(fr);
        c = in ? c : 0.0f;
        sn = in ? sn : 0.0f;
        if constexpr (LP) {
          unsigned short* st = stg16 + m_off[i];
#pragma unroll
          for (int m = 0; m < D; ++m) {
            st[(2 * m) * SW] = to16<PREC>(c * fv[m]);
            st[(2 * m + 1) * SW] = to16<PREC>(sn * fv[m]);
          }
          st[(2 * D) * SW] = to16<PREC>(c);
          st[(2 * D + 1) * SW] = to16<PREC>(sn);
        } else {
          float* st = stg + m_off[i];
#pragma unroll
          for (int m = 0; m < D; ++m) {
            st[(2 * m) * SW] = c * fv[m];
            st[(2 * m + 1) * SW] = sn * fv[m];
          }
          st[(2 * D) * SW] = c;
          st[(2 * D + 1) * SW] = sn;
        }
        if (m_csin[i]) {
          s_cs[cs0 * CST + m_cs[i]] = c;
          s_cs[cs0 * CST + m_cs[i] + TW] = sn;
        }
      }
    }
  };

  // FP32 matrix-core horizontal pass in two parts, so that the pipelined
  // schedule can place the vertical pass's ring loads between the products
  // and the ring stores: the banded product of the staging buffer stg, then
  // the store of its results into ring rows r0.
  // Product row m of block mb is staging row 2mb + ((m >> 2) & 1) (of the
  // step), channel 2 (m & 3) + (m >> 3): lane l then holds row 2mb + (l/16
  // & 1) of channels 2v + l/32, v < 4, so that the four 16-lane groups of a
  // ring store sit at 0, RST, TW and RST + TW floats: 0, 16, 32 and 48 mod 64
  // with the pipelined ring's padding, each group on 16 banks of its own.
  auto hmf = [&](const float* stg) {
    static_assert(!(MF && !LP) || NC == 8, "FP32 matrix-core pass: 2 rows x 8 channels per block");
    const int ln = tid & 63, mb = (tid >> 6) % NP, nb = (tid >> 6) / NP;
    const int m = ln & 15, srow = (2 * mb + ((m >> 2) & 1)) * NC + 2 * (m & 3) + (m >> 3);
    const float* arow = stg + srow * SW + 16 * nb + (ln >> 4);
    f32x4_t d = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int k = 0; k < KS4; ++k) d = mfma4(arow[4 * k], hb4[k], d);
    return d;
  };
  auto hmf_store = [&](const f32x4_t& d, int r0) {
    const int ln = tid & 63, mb = (tid >> 6) % NP, nb = (tid >> 6) / NP;
    const int g = ln >> 4, row = 2 * mb + (g & 1);
    if constexpr (SPV) {
      // row r0 + row is half (g & 1) of pair-row q = mb of step slot r0/8
      // (r0 is a multiple of 8): dword (r0/8) 4 RST + ((2v + g/2) TW + x) 4
      // + mb; the lo plane follows the hi plane's RS/2 x RST dwords
      unsigned short* const hp16 = s_ring16 + 2 * (r0 / 8) * 4 * RST;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        unsigned short h, l;
        split16(d[v], h, l);
        hp16[spv_st + 16 * v * TW] = h;
        hp16[spv_st + 16 * v * TW + RS * RST] = l;
      }
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v)
        s_ring[(r0 + row) * RST + (2 * v + (g >> 1)) * TW + 16 * nb + (ln & 15)] = d[v];
    }
  };

  // ---- FP32 matrix-core vertical pass of a pair of steps (PIPE instances) --
  // out[r][n] = sum_k w[k - r] ring[k][n] over the pair's 16 output rows r
  // and 16 + 2R window rows k (k-blocks of 4: KS4 of them, the horizontal
  // pass's count): the tap operand is the horizontal pass's register hb4
  // (lane l holds w[4kb + l/16 - l%16], here as A[r = l%16][k = l/16]); the
  // ring operand is one value per lane, B[k = l/16][n = l%16].  Wave w takes
  // pair m = w % NP (its cos and sin channels, two product chains) and
  // columns 16(w/NP) .. +15; lane l then holds output rows 4(l/16) .. +3 of
  // column l%16, demodulates them with the cos/sin of the output pixels and
  // updates four accumulator rows.  pr: strip row of the pair's first output
  // row; rl / cl: ring / cos-sin rows of its first window row; ap: this
  // lane's accumulators of the pair (prefetched; unused for t = 0).
  // this lane's accumulator column and first row of a pair, without the
  // pair's first output row (a uniform offset)
  const unsigned accp_lane = [&] {
    const int ln = tid & 63, m = (tid >> 6) % NP, nb = (tid >> 6) / NP;
    return (unsigned)(m * a.Hp + y0 + 4 * (ln >> 4)) * Wp + x0 + 16 * nb + (ln & 15);
  }();
  auto load_accp = [&](float (&dst)[4], int t, int pr) {
    (void)t;   // loaded whatever t is, like load_acc
#pragma unroll
    for (int v = 0; v < 4; ++v)
      dst[v] = buf_load1s(acc_rsrc, 4u * accp_lane, 4u * (unsigned)(pr + v) * Wp);
  };
  auto vpair = [&](int t, int pr, const float (&ap)[4], int rl, int cl) {
    const int ln = tid & 63, m = (tid >> 6) % NP, nb = (tid >> 6) / NP;
    const int col = 16 * nb + (ln & 15);
    // ring rows rl + 4k + l/16: k-blocks of 4 rows start at multiples of 4
    // (rl is a multiple of 8, the ring of 8), so only the uniform part wraps
    const float* cc = s_ring + ((ln >> 4) * RST + (2 * m) * TW + col);
    f32x4_t dc = {0.0f, 0.0f, 0.0f, 0.0f}, ds = {0.0f, 0.0f, 0.0f, 0.0f};
    if constexpr (SPV) {
      // KBS k-blocks of 32 window rows; in block kb lane group l/16 reads
      // its 8 rows of one column, step slot rl/8 + 4kb + l/16 (wrapped over
      // the RS/8 slots: a uniform slot and a per-lane choice of two
      // offsets), as one 128-bit read per plane and channel.  Window rows
      // past 16 + 2R meet zero taps: at R = 30 the last block reaches the
      // slot of the step being stored and, past the ring's end, the
      // window's first slot again (finite values either way).
      (void)cc;
      const uint4* hp = reinterpret_cast<const uint4*>(s_ring32) + (2 * m) * TW + col;
      const uint4* lp = hp + (RS / 2) * RST / 4;
      const int ns = RS / B, g = ln >> 4;
#pragma unroll
      for (int kb = 0; kb < KBS; ++kb) {
        const int u = __builtin_amdgcn_readfirstlane(wrap(rl / B + 4 * kb, ns));
        const int pb = (u + g - (g >= ns - u ? ns : 0)) * RST;   // in uint4 units: slot x RST
        const uint4 hc = hp[pb], lc = lp[pb], hs = hp[pb + TW], ls = lp[pb + TW];
        dc = mfma32<1>(vah[kb], hc, dc);
        ds = mfma32<1>(vah[kb], hs, ds);
        dc = mfma32<1>(vah[kb], lc, dc);
        ds = mfma32<1>(vah[kb], ls, ds);
        dc = mfma32<1>(val[kb], hc, dc);
        ds = mfma32<1>(val[kb], hs, ds);
      }
    } else {
#pragma unroll
      for (int k = 0; k < KS4; ++k) {
        const int row = wrap(rl + 4 * k, RS);
        dc = mfma4(hb4[k], cc[row * RST], dc);
        ds = mfma4(hb4[k], cc[row * RST + TW], ds);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float* cs = s_cs + wrap(cl + R + 4 * (ln >> 4) + v, CRS) * CST + col;
      const float q = fmaf(cs[TW], ds[v], cs[0] * dc[v]);
      buf_store1s(acc_rsrc, 4u * accp_lane, 4u * (unsigned)(pr + v) * Wp,
                  fmaf(tw, q, t > 0 ? ap[v] : 0.0f));
    }
  };

  // ---- 2. horizontal pass of the staging buffer stg into ring rows r0 -------
  auto hpass_step = [&](const float* stg, int r0) {
    const unsigned short* stg16 = reinterpret_cast<const unsigned short*>(stg);
    const int rslot = r0;
    // Matrix-core horizontal pass: the step's staging rows m = NC row +
    // channel (16 NP of them) form NP blocks of 16; wave w takes block w % NP
    // and output columns 16(w/NP) .. +15.  Lane l's results are items
    // m = 16(w%NP) + 4(l/16) + v, column 16(w/NP) + l%16 (FP32: items in
    // the order given at hmf).
    if constexpr (MF && !LP) {
      // FP32: k-blocks of 4 samples (one per lane group of 16)
      hmf_store(hmf(stg), rslot);
    } else if constexpr (MF) {
      const int ln = tid & 63, mb = (tid >> 6) % NP, nb = (tid >> 6) / NP;
      const unsigned short* arow = stg16 + (16 * mb + (ln & 15)) * SW + 16 * nb + 8 * (ln >> 4);
      f32x4_t d = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int k = 0; k < KSH; ++k)
        d = mfma32<PREC>(*reinterpret_cast<const uint4*>(arow + 32 * k), hb[k], d);
      // row r of the step is the low (even r) or high (odd r) half of pair-row
      // (rslot + r)/2.  Each lane stores its own halves: no lane exchange, so
      // no hand-written instruction reads the product's registers (the
      // compiler places the wait states a matrix-core result needs only before
      // the instructions it generates).
      if constexpr (NC == 8) {
        // item m = 16mb + 4g + v (g = lane / 16) is row 2mb + g/2 of the
        // step, channel 4(g & 1) + v: with rslot even, pair-row rslot/2 + mb,
        // half g/2 -- a per-lane offset plus rslot * RST and v * 2 TW
#pragma unroll
        for (int v = 0; v < 4; ++v)
          s_ring16[rslot * RST + hs_lane + v * 2 * TW] = to16<PREC>(d[v]);
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int m = 16 * mb + 4 * (ln >> 4) + v, row = m / NC;
          s_ring16[2 * (((rslot + row) >> 1) * RST + (m - row * NC) * TW + 16 * nb + (ln & 15)) +
                   (row & 1)] = to16<PREC>(d[v]);
        }
      }
    } else {
      float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
      if constexpr (LP) {
        const unsigned* src =
            reinterpret_cast<const unsigned*>(stg16 + (p1_rr * NC + p1_ch) * SW) + p1_xq * 2;
        hpass_lp<PREC, RC>(src, tpe, tpo, s_te, s_to, R, acc);
        // row r goes to the low (even r) or high (odd r) half of pair-row r/2
        const int r = rslot + p1_rr;
        if constexpr ((TW == 16 && 4 * NC == 32) || TW == 32) {
          // rows 2w and 2w+1 of this item sit in lanes l and l+32: swap halves so
          // the lower lanes hold both rows of columns 2,3 and the upper lanes
          // both rows of columns 0,1, then write one packed 64-bit chunk each
          unsigned a2 = __builtin_bit_cast(unsigned, acc[2]), a0 = __builtin_bit_cast(unsigned, acc[0]);
          unsigned a3 = __builtin_bit_cast(unsigned, acc[3]), a1 = __builtin_bit_cast(unsigned, acc[1]);
          swap_halves(a2, a0);   // lower lanes: (e2, o2); upper lanes: (e0, o0)
          swap_halves(a3, a1);   // lower lanes: (e3, o3); upper lanes: (e1, o1)
          const unsigned da = pack2<PREC>(__builtin_bit_cast(float, a2), __builtin_bit_cast(float, a0));
          const unsigned db = pack2<PREC>(__builtin_bit_cast(float, a3), __builtin_bit_cast(float, a1));
          const int upper = (tid >> 5) & 1;   // odd row of the pair
          *reinterpret_cast<uint2*>(s_ring32 + (r >> 1) * RST + p1_ch * TW + p1_xq * 4 +
                                    (upper ? 0 : 2)) = make_uint2(da, db);
        } else {
          unsigned short* dst = s_ring16 + 2 * ((r >> 1) * RST + p1_ch * TW + p1_xq * 4) + (r & 1);
#pragma unroll
          for (int p = 0; p < 4; ++p) dst[2 * p] = to16<PREC>(acc[p]);
        }
      } else {
        hpass<RC>(stg + (p1_rr * NC + p1_ch) * SW + p1_xq * 4, tapr, s_taps, ntap4, acc);
        *reinterpret_cast<float4*>(s_ring + (rslot + p1_rr) * RST + p1_ch * TW + p1_xq * 4) =
            make_float4(acc[0], acc[1], acc[2], acc[3]);
      }
    }
  };

  // ---- 3. vertical pass of step s of term t (weight tw), demodulation and
  // accumulation: ring rows from rl, cos/sin rows from cl; acur holds this
  // step's prefetched accumulators -------------------------------------------
  auto vpass_step = [&](int t, int s, const float (&acur)[NACC], int rl, int cl) {
    const int rslot_lag = rl, cslot_lag = cl;
    if (MFV && s >= lag) {
      if constexpr (MFV) {
        // out[r][n] for the pair's cos and sin channels over this wave's 16
        // columns; the window's ring rows 8(l/16)+v of each k-block are four
        // aligned pair-rows (rslot_lag is a multiple of 8, the ring a
        // multiple of 4 pair-rows).  Rows past the window (taps zero) wrap
        // around the ring and read finite values.
        constexpr int RSP = ring_steps(RC, 0) * kB / 2;
        static_assert(RSP % 4 == 0 && (RSP - 4) + 16 * (KSV - 1) + 12 < 3 * RSP, "pair-row wrap");
        // Lane group g reads pair-rows p = rslot_lag/2 + 16k + 4g (mod RSP):
        // the uniform part is reduced on the scalar unit, and a lane whose 4g
        // carries it past RSP takes the other of two uniform offsets.
        const unsigned* colc = s_ring32 + mfv_lane;
        f32x4_t dc = {0.0f, 0.0f, 0.0f, 0.0f}, ds = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int k = 0; k < KSV; ++k) {
          int u = rslot_lag / 2 + 16 * k;
          u = u >= RSP ? u - RSP : u;
          u = u >= RSP ? u - RSP : u;
          const unsigned* r0 = colc + u * RST - (mf_g4 >= RSP - u ? RSP * RST : 0);
          dc = mfma32<PREC>(va[k], make_uint4(r0[0], r0[RST], r0[2 * RST], r0[3 * RST]), dc);
          ds = mfma32<PREC>(va[k], make_uint4(r0[TW], r0[RST + TW], r0[2 * RST + TW], r0[3 * RST + TW]), ds);
        }
        if (mf_on) {
          const int cb = cslot_lag + R;   // cos/sin row of output row 0 of the step
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            // rows cb + v (lanes 0-15) and cb + 4 + v (lanes 16-31)
            // (offsets multiplied before the select: readfirstlane keeps the
            // compiler from moving the multiply after it, onto the lanes)
            const int oa = __builtin_amdgcn_readfirstlane(wrap(cb + v, CRS) * CST);
            const int ob = __builtin_amdgcn_readfirstlane(wrap(cb + 4 + v, CRS) * CST);
            const float* cs = s_cs + mf_x + (mf_r0 ? ob : oa);
            const float q = fmaf(cs[TW], ds[v], cs[0] * dc[v]);
            buf_store1s(acc_rsrc, 4u * acc_lane, 4u * (unsigned)((s - lag) * B + v) * Wp,
                        fmaf(tw, q, t > 0 ? acur[v] : 0.0f));
          }
        }
      }
    } else if (!MFV && s >= lag) {
      float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
      if constexpr (VB) {
        // output rows (s - lag)*B .. +7 of the strip: the first lag*B - 2R of
        // them were completed in the previous step, the others in this one
        const int ob = (s - lag) * B + p2_g * 4;
#pragma unroll
        for (int p = 0; p < 4; ++p) acc[p] = s_vr[((ob + p) & 15) * RST + p2_ch * TW + p2_x];
      } else if constexpr (LP) {
        vpass_lp<PREC, RC, RST>(s_ring32 + p2_ch * TW + p2_x, (rslot_lag + p2_g * 4) >> 1, RS / 2,
                                tpe, tpo, s_te, s_to, R, acc);
      } else {
        vpass<RC, RST>(s_ring + p2_ch * TW + p2_x, rslot_lag + p2_g * 4, RS, tapr, s_taps, ntap4,
                       acc);
      }
      const int cb = cslot_lag + p2_g * 4 + R;
      float q[4];
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const float cs = s_cs[wrap(cb + p, CRS) * CST + p2_k * TW + p2_x];
        q[p] = cs * acc[p];
      }
      {  // lane k adds rows 2k and 2k+1 of the pair's 4-row block
        // The cos half (k = 0, even rows of 16 lanes) and the sin half (k = 1,
        // odd rows) of a column sit 16 lanes apart.  Exchanging odd rows of
        // q[0] with even rows of q[2] leaves, in every lane, its own and its
        // partner's value of row p = 2k (p = 0 on the cos side, 2 on the sin
        // side); likewise q[1], q[3] for rows 2k + 1.
        unsigned e0 = __builtin_bit_cast(unsigned, q[0]), e2 = __builtin_bit_cast(unsigned, q[2]);
        unsigned e1 = __builtin_bit_cast(unsigned, q[1]), e3 = __builtin_bit_cast(unsigned, q[3]);
        if constexpr (TW == 16) {
          swap_rows16(e0, e2);
          swap_rows16(e1, e3);
        } else {   // halves 32 lanes apart: the same exchange across wave halves
          swap_halves(e0, e2);
          swap_halves(e1, e3);
        }
        const float v0 = __builtin_bit_cast(float, e0) + __builtin_bit_cast(float, e2);
        const float v1 = __builtin_bit_cast(float, e1) + __builtin_bit_cast(float, e3);
        const unsigned o = acc_lane + (unsigned)((s - lag) * B + p2_g * 4) * Wp;
        buf_store1(acc_rsrc, 4u * o, fmaf(tw, v0, t > 0 ? acur[0] : 0.0f));
        buf_store1(acc_rsrc, 4u * (o + Wp), fmaf(tw, v1, t > 0 ? acur[1] : 0.0f));
      }
    }
  };

  // One pipeline step s of term t (two barriers; every instance but PIPE);
  // fcur/acur hold this step's prefetched data and are refilled for the step
  // two ahead.
  auto step = [&](int t, int s, float (&fcur)[MI][D], float (&acur)[NACC]) {
    modulate(t, s, fcur, s_stage, cslot);
    // the step two ahead, possibly in the next term(s)
    int s2 = s + 2, t2 = t;
    if (s2 >= steps) { s2 -= steps; ++t2; }
    if (s2 >= steps) { s2 -= steps; ++t2; }
    load_f(fcur, s2);
    __syncthreads();
    hpass_step(s_stage, rslot);
    __syncthreads();
    // variant 3: running sums of the rows just written
    if constexpr (VB) {
      // input row i = s*B + j of the term (strip row i - R) completes the box
      // sum of output row i - 2R; rows before the term's first (i < k w) are
      // the previous term's and read as zero
      if (vb_on) {
        if (s == 0) vI1 = vI2 = vI3 = 0.0;
        const float* col = s_ring + vb_ch * TW + vb_x;
        // all ring reads of the step first (no branch between them): row i
        // and rows i - k w, k <= n; a lag that is not part of the sum (k > n,
        // or a row before the term's first) reads an in-ring slot and gets
        // weight zero (ring values are finite)
        const int o1 = vw, o2 = vn >= 2 ? 2 * vw : 0, o3 = vn >= 3 ? 3 * vw : 0;
        float u[B][4];
#pragma unroll
        for (int j = 0; j < B; ++j) {
          const int sl = wrap(rslot + j, RS);
          const int s1 = sl - o1, s2 = sl - o2, s3 = sl - o3;
          u[j][0] = col[sl * RST];
          u[j][1] = col[(s1 < 0 ? s1 + RS : s1) * RST];
          u[j][2] = col[(s2 < 0 ? s2 + RS : s2) * RST];
          u[j][3] = col[(s3 < 0 ? s3 + RS : s3) * RST];
        }
        // rows before the term's first only occur in its first steps: one
        // uniform test per step, then a loop without per-row conditions
        auto rows = [&](auto head) {
          constexpr bool HEAD = decltype(head)::value;
#pragma unroll
          for (int j = 0; j < B; ++j) {
            const int i = s * B + j;
            const double c1 = !HEAD || i >= o1 ? vc1 : 0.0;
            const double c2 = !HEAD || i >= o2 ? vc2 : 0.0;
            const double c3 = !HEAD || i >= o3 ? vc3 : 0.0;
            double v = (double)u[j][0];
            v = fma(c1, (double)u[j][1], v);
            v = fma(c2, (double)u[j][2], v);
            v = fma(c3, (double)u[j][3], v);
            vI1 += v;
            vI2 += vI1;
            vI3 += vI2;
            // output row i - 2R; rows outside 0..TH-1 land in ring slots that
            // are rewritten before the demodulation reads them
            s_vr[((i - 2 * R) & 15) * RST + vb_ch * TW + vb_x] =
                (float)fma(ve3, vI3, fma(ve2, vI2, ve1 * vI1));
          }
        };
        if (s * B >= vn * vw) rows(std::false_type{});
        else rows(std::true_type{});
      }
      __syncthreads();
    }
    vpass_step(t, s, acur, rslot_lag, cslot_lag);
    load_acc(acur, t2, s2);
    rslot = wrap(rslot + B, RS);
    cslot = wrap(cslot + B, CRS);
    rslot_lag = wrap(rslot_lag + B, RS);
    cslot_lag = wrap(cslot_lag + B, CRS);
  };

  // Flattened loop over (term, step) pairs of global steps, two per trip so
  // the A/B prefetch buffers keep fixed roles.
  load_f(fA, 0);
  load_f(fB, steps > 1 ? 1 : 0);
  // Accumulators of global steps 0 and 1.  Later steps are prefetched two
  // ahead inside the loop, which is exact because a term has at least two
  // steps (the host guarantees it): the rows of step g + 2 were last written
  // in step g + 2 - steps <= g.  These two only matter when the launch
  // resumes a term range (t0 > 0) and the vertical pass already writes in
  // step 0 or 1 (2R <= 8 rows of look-ahead).
  load_acc(aA, t0, 0);
  if (steps > 1) load_acc(aB, t0, 1);
  else load_acc(aB, t0 + 1, 0);
  load_term(t0);
  const int total = (t1 - t0) * steps;
  if constexpr (PIPE) {
    // Software pipeline, one barrier per step: iteration g runs the
    // horizontal pass of global step g, the modulation of step g + 1 and,
    // when step g - 1 completes a pair of output steps (s - lag odd), the
    // pair's vertical pass: matrix-core products of both passes overlap the
    // modulation on the VALU.  Staging and f are double-buffered by step
    // parity (f: fA even steps, fB odd); a strip has an even number of
    // output steps (TH a multiple of 16, checked at launch).
    float* const stg0 = s_stage;
    float* const stg1 = s_stage + stage_floats;
    float ap[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    load_accp(ap, t0, 0);
    modulate(t0, 0, fA, stg0, 0);
    load_f(fA, 2 % steps);             // step 2 (the next term's first when steps = 2)
    __syncthreads();
    int tv = t0, sv = 0;               // step g - 1 (advanced from g = 1 on)
    int tm = t0, sm = 1;               // step modulated in iteration g (g + 1)
    if (sm == steps) { sm = 0; ++tm; }
    if (tm < t1) load_wr(tm);
    // ring rows of step g (horizontal pass) and of step g - 2 - lag (the
    // window of the pair ending at step g - 1); cos/sin rows of step g + 1
    // (modulation) and of step g - 2 - lag
    int rh = 0;
    int rl = (RSBk - (lag + 2) % RSBk) % RSBk * B;
    int cm = B % CRS;
    int cl = (CRB - (lag + 2) % CRB) % CRB * B;
    auto iter = [&](int g, const float* stg_h, float* stg_m, float (&fm)[MI][D]) {
      if (g >= 1 && sv > lag && ((sv - lag) & 1)) {
        // the pair (sv - 1, sv) of term tv and the horizontal pass of step
        // g in one block; the ring stores after the pair's ring loads
        const f32x4_t hd = hmf(stg_h);
        vpair(tv, (sv - 1 - lag) * B, ap, rl, cl);
        hmf_store(hd, rh);
      } else {
        hpass_step(stg_h, rh);
      }
      {
        // the accumulators of the next pair, (re)loaded in every iteration
        // (a load on one side of the branch only made the compiler wait for
        // it at the merge): after a pair, the one starting at step sv + 1
        // (the next term's first, at output row 0, past the term's end);
        // otherwise the one starting at step max(sv, lag)
        int pn;
        if (g >= 1 && sv > lag && ((sv - lag) & 1)) pn = sv + 1 >= steps ? 0 : (sv + 1 - lag) * B;
        else pn = g >= 1 && sv > lag ? (sv - lag) * B : 0;
        load_accp(ap, 0, pn);
      }
      if (g >= 1 && ++sv == steps) {
        sv = 0;
        if (++tv < t1) load_tw(tv);
      }
      rl = wrap(rl + B, RS);
      cl = wrap(cl + B, CRS);
      if (g + 1 < total) {
        modulate(tm, sm, fm, stg_m, cm);
        int s3 = sm + 2;               // f rows of step g + 3
        if (s3 >= steps) s3 -= steps;
        if (s3 >= steps) s3 -= steps;
        load_f(fm, s3);
        if (++sm == steps) {
          sm = 0;
          if (++tm < t1) load_wr(tm);
        }
        cm = wrap(cm + B, CRS);
      }
      __syncthreads();
      rh = wrap(rh + B, RS);
    };
    for (int g = 0; g < total; g += 2) {
      iter(g, stg0, stg1, fB);
      if (g + 1 < total) iter(g + 1, stg1, stg0, fA);
    }
    // the last pair (its second step is the launch's last)
    vpair(tv, (sv - 1 - lag) * B, ap, rl, cl);
    return;
  }
  if constexpr (SLV) {
    // Three-box vertical pass as cascaded sliding sums, with the same one-
    // barrier pipeline as PIPE: iteration g runs the horizontal pass of global
    // step g (matrix cores), the vertical pass of step g - 1 and the
    // modulation of step g + 1.  With u the horizontal-pass rows of a term
    // (input row i of the strip's haloed rows) and w = 2r + 1:
    //   S1(i) = S1(i-1) + u(i) - u(i-w)         (box over u)
    //   S2(i) = S2(i-1) + S1(i) - S1(i-w)       (box over S1)
    //   L2(i) = L2(i-1) + S1(i-w) - S1(i-2w)    (= S2(i-w))
    //   S3(i) = S3(i-1) + S2(i) - L2(i)         (box over S2)
    // so S3(i) is the three-box filter of u over rows i - 2R .. i, the
    // vertical pass of output row o = i - 2R (rows before the term's first
    // count as zero).  The sums are FP64 registers of one lane per (column,
    // channel) (waves 0..NP-1), reset at each term's first row; S1 is stored
    // rounded to FP32 and S2, L2 add and subtract those same stored values,
    // so the telescoping sums stay exact and nothing drifts down the strip.
    // The cos and sin channels of a pair sit in lanes l and l + 32 and
    // exchange halves for the demodulation; each lane then updates 4 rows.
    float* const stg0 = s_stage;
    float* const stg1 = s_stage + stage_floats;
    const bool sl_on = tid < 64 * NP;
    const int sl_x = tid & 31, sl_k = (tid >> 5) & 1, sl_m = tid >> 6;
    const int sl_col = (2 * sl_m + sl_k) * TW + sl_x;     // [ch][x] within a ring row
    double S1 = 0.0, S2 = 0.0, L2 = 0.0, S3 = 0.0;
    float sa[4] = {0.0f, 0.0f, 0.0f, 0.0f}, sb[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    // accumulator rows of this lane in v-step s: o = 8s + (k ? 4 : 0) + v - 2R
    // (issued by every lane whatever t is, from rows clamped into the strip,
    // for the reason given at load_acc)
    auto load_accs = [&](float (&dst)[4], int t, int sv2) {
      (void)t;
      const int mc = min(sl_m, NP - 1);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int o = min(max(B * sv2 + 4 * sl_k + v - 2 * R, 0), a.TH - 1);
        dst[v] = buf_load1(acc_rsrc, 4u * ((unsigned)(mc * a.Hp + y0 + o) * Wp + x0 + sl_x));
      }
    };
    auto slide = [&](int t, int sv, const float (&av)[4], int rv, int sr, int cv) {
      if (!sl_on) return;
      if (sv == 0) S1 = S2 = L2 = S3 = 0.0;
      // every LDS read of the step first (rows of earlier steps, or of this
      // step's first-stage sums when w < 8), then the four recurrences
      float un[B], uo[B], fb[B], cs[B];
#pragma unroll
      for (int j = 0; j < B; ++j) {
        const int i = B * sv + j;
        un[j] = s_ring[(rv + j) * RST + sl_col];
        int ro = rv + j - SLW;
        ro = ro < 0 ? ro + RS : ro;
        uo[j] = i >= SLW ? s_ring[ro * RST + sl_col] : 0.0f;
        int rb = sr + j - 2 * SLW;
        rb = rb < 0 ? rb + SL_S1R : rb;
        rb = rb < 0 ? rb + SL_S1R : rb;
        fb[j] = i >= 2 * SLW ? s_s1[rb * (NC * TW) + sl_col] : 0.0f;
        int rc = cv + j - R;   // cos/sin row of output pixel o = i - 2R: input row i - R
        rc = rc < 0 ? rc + CRS : rc;
        cs[j] = s_cs[rc * CST + sl_k * TW + sl_x];
      }
      float fa[B];
#pragma unroll
      for (int j = 0; j < B; ++j) {
        if (j < SLW) {   // row i - w lies in an earlier step
          int ra = sr + j - SLW;
          ra = ra < 0 ? ra + SL_S1R : ra;
          fa[j] = B * sv + j >= SLW ? s_s1[ra * (NC * TW) + sl_col] : 0.0f;
        }
      }
      float s1f[B], q[B];
#pragma unroll
      for (int j = 0; j < B; ++j) {
        S1 += (double)un[j] - (double)uo[j];
        s1f[j] = (float)S1;
        if (j >= SLW) fa[j] = s1f[j - SLW];   // w < 8: this step's own sums
        S2 += (double)s1f[j] - (double)fa[j];
        L2 += (double)fa[j] - (double)fb[j];
        S3 += S2 - L2;
        q[j] = cs[j] * (float)S3;
      }
#pragma unroll
      for (int j = 0; j < B; ++j) s_s1[(sr + j) * (NC * TW) + sl_col] = s1f[j];
      // lanes 0-31 take rows 0-3, lanes 32-63 rows 4-7 (cos + sin of a pair)
      float r4[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        unsigned lo = __builtin_bit_cast(unsigned, q[v]), hi = __builtin_bit_cast(unsigned, q[v + 4]);
        swap_halves(lo, hi);
        r4[v] = __builtin_bit_cast(float, lo) + __builtin_bit_cast(float, hi);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int o = B * sv + 4 * sl_k + v - 2 * R;
        if (o >= 0 && o < a.TH)
          buf_store1(acc_rsrc, 4u * ((unsigned)(sl_m * a.Hp + y0 + o) * Wp + x0 + sl_x),
                     fmaf(tw, r4[v], t > 0 ? av[v] : 0.0f));
      }
    };
    load_accs(sa, t0, 0);
    load_accs(sb, steps > 1 ? t0 : t0 + 1, steps > 1 ? 1 : 0);
    modulate(t0, 0, fA, stg0, 0);
    load_f(fA, 2 % steps);
    __syncthreads();
    int tv = t0, sv = 0, tm = t0, sm = 1;
    if (sm == steps) { sm = 0; ++tm; }
    if (tm < t1) load_wr(tm);
    // rows of step g (horizontal pass), of step g - 1 (vertical pass: ring,
    // first-stage sums, cos/sin) and of step g + 1 (modulation: cos/sin)
    int rh = 0, rv = RS - B, sr = SL_S1R - B, cv = CRS - B, cm = B;
    auto iter = [&](int g, const float* stg_h, float* stg_m, float (&fm)[MI][D],
                    float (&av)[4]) {
      // the sliding sums first: while waves 0..NP-1 run them on the VALU,
      // the other waves' horizontal-pass products have the matrix cores
      if (g >= 1) {
        slide(tv, sv, av, rv, sr, cv);
        int s2 = sv + 2, t2 = tv;       // accumulators of step g + 1
        if (s2 >= steps) { s2 -= steps; ++t2; }
        if (s2 >= steps) { s2 -= steps; ++t2; }
        load_accs(av, t2, s2);
        if (++sv == steps) {
          sv = 0;
          if (++tv < t1) load_tw(tv);
        }
      }
      hpass_step(stg_h, rh);
      if (g + 1 < total) {
        modulate(tm, sm, fm, stg_m, cm);
        int s3 = sm + 2;
        if (s3 >= steps) s3 -= steps;
        if (s3 >= steps) s3 -= steps;
        load_f(fm, s3);
        if (++sm == steps) {
          sm = 0;
          if (++tm < t1) load_wr(tm);
        }
      }
      __syncthreads();
      rh = wrap(rh + B, RS);
      rv = wrap(rv + B, RS);
      sr = wrap(sr + B, SL_S1R);
      cv = wrap(cv + B, CRS);
      cm = wrap(cm + B, CRS);
    };
    // v-step g - 1 uses the accumulators of its parity: sa even, sb odd
    for (int g = 0; g < total; g += 2) {
      iter(g, stg0, stg1, fB, sb);
      if (g + 1 < total) iter(g + 1, stg1, stg0, fA, sa);
    }
    if ((total - 1) & 1) slide(tv, sv, sb, rv, sr, cv);
    else slide(tv, sv, sa, rv, sr, cv);
    return;
  }
  int t = t0, s = 0;
  for (int gs = 0; gs < total; gs += 2) {
    step(t, s, fA, aA);
    if (++s == steps) {
      s = 0;
      if (++t < t1) load_term(t);
    }
    if (gs + 1 < total) {
      step(t, s, fB, aB);
      if (++s == steps) {
        s = 0;
        if (++t < t1) load_term(t);
      }
    }
  }
}

// XCD-aware order: dispatch ids go round-robin over the 8 XCDs; give each XCD
// a contiguous run of strips so neighbours (which share their halo of f) meet
// in the same L2.
__device__ __forceinline__ int xcd_order(int bid, int n) {
  return n % 8 == 0 ? (bid % 8) * (n / 8) + bid / 8 : bid;
}

// One request: one workgroup per strip.  P64: instance with the FP64 phase
// path (its branches cost the common path a few percent, so launches whose
// phases are bounded below 2^8 turns use the instance without it).  TW: strip
// width, 16 columns (D+1 waves) or 32 (2(D+1) waves).
template <int D, int RC, int PREC, bool P64, int TW = kTW, bool MF = false>
__global__ __launch_bounds__(64 * (D + 1) * (TW / 16)) void mcsf_fused(FusedArgs a) {
  fused_strip<D, RC, PREC, P64, TW, MF>(a, xcd_order(blockIdx.x, a.nsx * a.nsy));
}

// Several requests of the same instance in one launch (continuous batching):
// the workgroup finds its request in the prefix table.
template <int D, int RC, int PREC, bool P64, int TW = kTW, bool MF = false>
__global__ __launch_bounds__(64 * (D + 1) * (TW / 16)) void mcsf_fused_batch(BatchArgs g) {
  const int bid = xcd_order(blockIdx.x, g.first[g.n]);
  int i = 0;
  while (i + 1 < g.n && bid >= g.first[i + 1]) ++i;
  fused_strip<D, RC, PREC, P64, TW, MF>(g.req[i], bid - g.first[i]);
}


// One instance's launch: A is FusedArgs (one request) or BatchArgs.
// Instances with wide strips: d = 3 with a compile-time radius, variants 0-2
// (choose_strip_width selects them).
template <int D, int RC, int PREC>
inline constexpr bool kHasWide = D == 3 && RC >= 0 && PREC <= 2;
// Instances with matrix-core passes (chosen at launch by use_mf): the wide
// ones, and the 16-column 16-bit ones at a compile-time radius.
template <int D, int RC, int PREC, int TW>
inline constexpr bool kHasMF =
    TW == kTWMax ? kHasWide<D, RC, PREC> : RC >= 0 && (PREC == 1 || PREC == 2);

inline int a_tw(const FusedArgs& a) { return a.TWc; }
inline int a_tw(const BatchArgs& b) { return b.req[0].TWc; }

template <int D, int RC, int PREC, class A>
static hipError_t launch_drp(const A& a, int R, hipStream_t st) {
  int nwg, TW = kTW;
  void (*kern)(A);
  int mf = 0;
  bool want_mf = use_mf(a_tw(a), PREC, R);
  if constexpr (std::is_same_v<A, BatchArgs>) {   // the batch shares p64, valu and the width
    const bool p64 = a.req[0].p64;
    for (int k = 1; k < a.n; ++k)
      if (a.req[k].p64 != a.req[0].p64 || a.req[k].TWc != a.req[0].TWc ||
          a.req[k].valu != a.req[0].valu)
        return hipErrorInvalidValue;
    want_mf = want_mf && !a.req[0].valu;
    kern = p64 ? mcsf_fused_batch<D, RC, PREC, true> : mcsf_fused_batch<D, RC, PREC, false>;
    if constexpr (kHasMF<D, RC, PREC, kTW>) {
      if (want_mf) {
        kern = p64 ? mcsf_fused_batch<D, RC, PREC, true, kTW, true>
                   : mcsf_fused_batch<D, RC, PREC, false, kTW, true>;
        mf = 1;
      }
    }
    if constexpr (kHasWide<D, RC, PREC>) {
      if (a.req[0].TWc == kTWMax) {
        kern = p64 ? mcsf_fused_batch<D, RC, PREC, true, kTWMax>
                   : mcsf_fused_batch<D, RC, PREC, false, kTWMax>;
        TW = kTWMax;
        mf = 0;
        if constexpr (kHasMF<D, RC, PREC, kTWMax>) {
          if (want_mf) {
            kern = p64 ? mcsf_fused_batch<D, RC, PREC, true, kTWMax, true>
                       : mcsf_fused_batch<D, RC, PREC, false, kTWMax, true>;
            mf = 1;
          }
        }
      }
    }
    if (a.req[0].TWc != TW) return hipErrorInvalidValue;   // no instance for this width
    nwg = a.first[a.n];
  } else {
    want_mf = want_mf && !a.valu;
    kern = a.p64 ? mcsf_fused<D, RC, PREC, true> : mcsf_fused<D, RC, PREC, false>;
    if constexpr (kHasMF<D, RC, PREC, kTW>) {
      if (want_mf) {
        kern = a.p64 ? mcsf_fused<D, RC, PREC, true, kTW, true> : mcsf_fused<D, RC, PREC, false, kTW, true>;
        mf = 1;
      }
    }
    if constexpr (kHasWide<D, RC, PREC>) {
      if (a.TWc == kTWMax) {
        kern = a.p64 ? mcsf_fused<D, RC, PREC, true, kTWMax> : mcsf_fused<D, RC, PREC, false, kTWMax>;
        TW = kTWMax;
        mf = 0;
        if constexpr (kHasMF<D, RC, PREC, kTWMax>) {
          if (want_mf) {
            kern = a.p64 ? mcsf_fused<D, RC, PREC, true, kTWMax, true>
                         : mcsf_fused<D, RC, PREC, false, kTWMax, true>;
            mf = 1;
          }
        }
      }
    }
    if (a.TWc != TW) return hipErrorInvalidValue;   // no instance for this width
    nwg = a.nsx * a.nsy;
  }
  // the pipelined instances take pairs of output steps: whole pairs per strip
  if (mf && use_pipe(PREC, R, true)) {
    if constexpr (std::is_same_v<A, BatchArgs>) {
      for (int k = 0; k < a.n; ++k)
        if (a.req[k].TH % (2 * kB)) return hipErrorInvalidValue;
    } else if (a.TH % (2 * kB)) {
      return hipErrorInvalidValue;
    }
  }
  const size_t lds = fused_lds_bytes(D, R, PREC, TW, mf);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (nwg <= 0) return hipSuccess;
  hipLaunchKernelGGL(kern, dim3(nwg), dim3(64 * (D + 1) * (TW / 16)), lds, st, a);
  return hipGetLastError();
}

// Variant 4 (three boxes, sliding sums): only the 32-column matrix-core
// instances at the compile-time radii exist.
template <int RC, class A>
static hipError_t launch_sl(const A& a, hipStream_t st) {
  int nwg;
  void (*kern)(A);
  if constexpr (std::is_same_v<A, BatchArgs>) {
    for (int k = 0; k < a.n; ++k)
      if (a.req[k].p64 != a.req[0].p64 || a.req[k].TWc != kTWMax) return hipErrorInvalidValue;
    kern = a.req[0].p64 ? mcsf_fused_batch<3, RC, 4, true, kTWMax, true>
                        : mcsf_fused_batch<3, RC, 4, false, kTWMax, true>;
    nwg = a.first[a.n];
  } else {
    if (a.TWc != kTWMax) return hipErrorInvalidValue;
    kern = a.p64 ? mcsf_fused<3, RC, 4, true, kTWMax, true> : mcsf_fused<3, RC, 4, false, kTWMax, true>;
    nwg = a.nsx * a.nsy;
  }
  const size_t lds = fused_lds_bytes(3, RC, 4, kTWMax, 1);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (nwg <= 0) return hipSuccess;
  hipLaunchKernelGGL(kern, dim3(nwg), dim3(64 * 4 * 2), lds, st, a);
  return hipGetLastError();
}

template <class A>
static hipError_t launch_sl_r(const A& a, int R, hipStream_t st) {
  switch (R) {
    case 6: return launch_sl<6>(a, st);
    case 9: return launch_sl<9>(a, st);
    case 12: return launch_sl<12>(a, st);
    case 15: return launch_sl<15>(a, st);
    case 18: return launch_sl<18>(a, st);
    case 21: return launch_sl<21>(a, st);
    case 24: return launch_sl<24>(a, st);
    case 30: return launch_sl<30>(a, st);
    default: return hipErrorInvalidValue;
  }
}

// Variant 5 (split vertical pass): the pipelined 32-column instances at
// R = 18, 21, 24 and 30 (whole pairs of 8-row steps per strip).
template <int RC, class A>
static hipError_t launch_sp(const A& a, hipStream_t st) {
  int nwg;
  void (*kern)(A);
  if constexpr (std::is_same_v<A, BatchArgs>) {
    for (int k = 0; k < a.n; ++k)
      if (a.req[k].p64 != a.req[0].p64 || a.req[k].TWc != kTWMax || a.req[k].valu ||
          a.req[k].TH % (2 * kB))
        return hipErrorInvalidValue;
    kern = a.req[0].p64 ? mcsf_fused_batch<3, RC, 5, true, kTWMax, true>
                        : mcsf_fused_batch<3, RC, 5, false, kTWMax, true>;
    nwg = a.first[a.n];
  } else {
    if (a.TWc != kTWMax || a.valu || a.TH % (2 * kB)) return hipErrorInvalidValue;
    kern = a.p64 ? mcsf_fused<3, RC, 5, true, kTWMax, true> : mcsf_fused<3, RC, 5, false, kTWMax, true>;
    nwg = a.nsx * a.nsy;
  }
  const size_t lds = fused_lds_bytes(3, RC, 5, kTWMax, 1);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (nwg <= 0) return hipSuccess;
  hipLaunchKernelGGL(kern, dim3(nwg), dim3(64 * 4 * 2), lds, st, a);
  return hipGetLastError();
}

template <class A>
static hipError_t launch_sp_r(const A& a, int R, hipStream_t st) {
  switch (R) {
    case 18: return launch_sp<18>(a, st);
    case 21: return launch_sp<21>(a, st);
    case 24: return launch_sp<24>(a, st);
    case 30: return launch_sp<30>(a, st);
    default: return hipErrorInvalidValue;
  }
}

// Radii with a fully unrolled specialisation (the workload radii and the
// serving range); every other radius takes the runtime-R variant.
template <int D, int PREC, class A>
static hipError_t launch_dp(const A& a, int R, hipStream_t st) {
  switch (R) {
    case 6: return launch_drp<D, 6, PREC>(a, R, st);
    case 9: return launch_drp<D, 9, PREC>(a, R, st);
    case 12: return launch_drp<D, 12, PREC>(a, R, st);
    case 15: return launch_drp<D, 15, PREC>(a, R, st);
    case 18: return launch_drp<D, 18, PREC>(a, R, st);
    case 21: return launch_drp<D, 21, PREC>(a, R, st);
    case 24: return launch_drp<D, 24, PREC>(a, R, st);
    case 30: return launch_drp<D, 30, PREC>(a, R, st);
    default: return launch_drp<D, -1, PREC>(a, R, st);
  }
}

template <int PREC, class A>
static hipError_t launch_p(int d, const A& a, int R, hipStream_t st) {
  switch (d) {
    case 1: return launch_drp<1, -1, PREC>(a, R, st);
    case 2: return launch_drp<2, -1, PREC>(a, R, st);
    case 3: return launch_dp<3, PREC>(a, R, st);
    case 4: return launch_drp<4, -1, PREC>(a, R, st);
    case 5: return launch_drp<5, -1, PREC>(a, R, st);
    case 6: return launch_dp<6, PREC>(a, R, st);
    case 7: return launch_drp<7, -1, PREC>(a, R, st);
    case 8: return launch_drp<8, -1, PREC>(a, R, st);
    default: return hipErrorInvalidValue;
  }
}


}  // namespace bfvec
