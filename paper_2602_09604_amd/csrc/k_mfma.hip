// Matrix-core passes for fused gates with k >= 4.
//
// The group matvecs of one pass (Eq. 4) are batched into a real GEMM in the
// 4M form: with rows ordered (amplitude, re/im), the 2^(k+1) x 2^(k+1) real
// matrix A' has blocks [[Ur, -Ui], [Ui, Ur]] and Y' = A' X', where column m of
// X' is one group's 2^k amplitudes.  The state is the B operand: each lane
// owns one column (or, in the PAIR layout, two columns that differ only in
// bit 0, fetched with one 16-byte load per amplitude), so the gathers stay
// coalesced 16-byte loads and the results leave as 16-byte stores.
//
// A' is encoded on the host in MFMA fragment order and copied once per
// workgroup into LDS; every wave then streams 32-group tiles through it.
//
//   FP32_MFMA: v_mfma_f32_32x32x2f32, one product.
//   BF16X3:    operands split into bf16 hi + lo (lo = bf16(x - hi)); three
//              v_mfma_f32_32x32x16_bf16 products hi*hi + hi*lo + lo*hi,
//              FP32 accumulation.
//   FP16X3:    as BF16X3 in fp16 with the lo halves scaled by 2^11, amplitudes
//              scaled by 2^14 before the split (every amplitude of a
//              normalised state, |c| <= 1, stays below the fp16 maximum and
//              amplitudes down to ~4e-9 stay normal); two FP32 accumulators
//              (hi*hi and the 2^11-scaled cross terms) combined at the end.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <type_traits>

#include "k_common.h"

namespace sv {

namespace {
using kern::gld;
using kern::gst;
using kern::compress_bits;
using kern::LowBits;
using kern::xtranspose;

typedef __attribute__((__vector_size__(8 * sizeof(short)))) short bf16x8;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int kLayoutPair = 0;  // bit 0 not a target: float4 = (group 2j, group 2j+1) at one amplitude
constexpr int kLayoutQ0 = 1;    // bit 0 is target 0: float4 = amplitudes (2t, 2t+1) of one group
constexpr float kF16Scale = 16384.f;       // 2^14
constexpr float kF16LoScale = 2048.f;      // 2^11

// ---- host-side conversions (round to nearest even) ------------------------
uint16_t host_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
float host_bf16_to_f(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}
// IEEE binary16 from binary32, round to nearest even, by integer arithmetic
// (the compiler's own conversion is a library call on the host, ten times
// slower than the rest of the encoding).
uint16_t host_f16(float f) {
  uint32_t x;
  std::memcpy(&x, &f, 4);
  const uint32_t sign = (x >> 16) & 0x8000u;
  x &= 0x7FFFFFFFu;
  if (x >= 0x47800000u) return (uint16_t)(sign | (x > 0x7F800000u ? 0x7E00u : 0x7C00u));  // >= 2^16, inf, NaN
  if (x < 0x38800000u) {  // below 2^-14: a subnormal half (or zero); the float add rounds to even
    float t;
    std::memcpy(&t, &x, 4);
    t += 0.5f;  // 0.5 has the exponent that leaves the subnormal half's bits at the bottom
    uint32_t u;
    std::memcpy(&u, &t, 4);
    return (uint16_t)(sign | (u - 0x3F000000u));
  }
  x += 0xC8000FFFu + ((x >> 13) & 1u);  // rebias the exponent by 15 - 127, round to nearest even
  return (uint16_t)(sign | (x >> 13));
}
float host_f16_to_f(uint16_t h) {
  const uint32_t e = (h >> 10) & 0x1Fu, m = h & 0x3FFu;
  float f;
  if (e == 0) {
    f = std::ldexp((float)m, -24);
  } else if (e == 31) {
    f = m ? std::numeric_limits<float>::quiet_NaN() : std::numeric_limits<float>::infinity();
  } else {
    const uint32_t u = ((e + 112u) << 23) | (m << 13);
    std::memcpy(&f, &u, 4);
  }
  return (h & 0x8000u) ? -f : f;
}

// ---- device-side conversions (gfx950 converts to bf16 natively, RNE) -------
__device__ __forceinline__ short dev_bf16(float f) { return __builtin_bit_cast(short, (__bf16)f); }
__device__ __forceinline__ float dev_bf16_f(short h) { return __uint_as_float((uint32_t)(uint16_t)h << 16); }

// Controls of a controlled pass: the pass covers only the groups whose
// control bits equal cval; at most kMfmaCtrl of them.
constexpr int kMfmaCtrl = 3;

struct MfmaArgs {
  uint64_t tiles;                          // 32-column tiles per control value
  uint64_t ins[SV_MAX_K + kMfmaCtrl];      // element-space zero-insertion masks of the targets
                                           // and controls, ascending; ~0 (a no-op) in unused slots
  uint64_t cbits[1 << kMfmaCtrl];          // element-space control bits of control value v,
                                           // ORed into every base of that value's groups
  uint64_t stride[SV_MAX_K];               // element stride of local bit j (element = float4)
  int kq;                                  // number of element-space targets
  int vbits;                               // log2 of the control values this launch covers; the
                                           // matrix of value v follows that of v - 1
};

template <int KQ>
__device__ __forceinline__ uint64_t mf_base(uint64_t g, uint64_t cb, const MfmaArgs& a) {
#pragma unroll
  for (int j = 0; j < KQ + kMfmaCtrl; ++j) g = ((g & ~a.ins[j]) << 1) | (g & a.ins[j]);
  return g | cb;
}

template <int KQ>
__device__ __forceinline__ uint64_t mf_off(int l, const MfmaArgs& a) {
  uint64_t o = 0;
#pragma unroll
  for (int j = 0; j < KQ; ++j)
    if ((l >> j) & 1) o += a.stride[j];
  return o;
}

// PREC: SV_PREC_FP32_MFMA, SV_PREC_BF16X3 or SV_PREC_FP16X3.  The output
// tiles are computed one at a time (loop not unrolled) with two waves per
// SIMD: unrolled, the compiler kept every tile's accumulators live and the
// streaming k = 6 forms needed all 256 VGPRs (one wave per SIMD, measured
// 1.5-2x slower for FP32 and BF16).
template <int K, int PREC, int LAYOUT, bool NT>
__device__ __forceinline__ void mfma_body(float4* __restrict__ psi, const float4* __restrict__ Ag, const MfmaArgs& a,
                                          float4* lds4) {
  constexpr int DK = 1 << K;                 // amplitudes per group
  constexpr int MT = (2 * DK) / 32;          // 32-row output tiles
  constexpr bool SPLIT = PREC != SV_PREC_FP32_MFMA;
  constexpr int KS = SPLIT ? (2 * DK) / 16 : DK;   // k-steps
  constexpr int FRAG_BYTES = SPLIT ? MT * KS * 2 * 64 * 16 : MT * KS * 64 * 4;
  constexpr int KQ = LAYOUT == kLayoutPair ? K : K - 1;  // element-space targets
  constexpr int COLS = LAYOUT == kLayoutPair ? 2 : 1;    // column tiles per lane
  const int tid = threadIdx.x;
  // workgroups are dealt round-robin to the control values; each loads the
  // matrix of its value and walks that value's tiles
  const unsigned v = blockIdx.x & ((1u << a.vbits) - 1);
  const uint64_t wg = blockIdx.x >> a.vbits;
  const uint64_t cb = a.cbits[v];
  Ag += (size_t)v * (FRAG_BYTES / 16);
  for (int i = tid; i < FRAG_BYTES / 16; i += 256) lds4[i] = Ag[i];
  __syncthreads();
  const int lane = tid & 63, h = lane >> 5, j = lane & 31;
  const uint64_t wstride = (uint64_t)(gridDim.x >> a.vbits) * 4;
  for (uint64_t wt = wg * 4 + (tid >> 6); wt < a.tiles; wt += wstride) {
    const uint64_t base = mf_base<KQ>(wt * 32 + j, cb, a);
    if constexpr (!SPLIT) {
      // ---- FP32: k-step s is amplitude s; this lane supplies part h ----
      float b[COLS][KS];
      if constexpr (LAYOUT == kLayoutPair) {
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          const float4 f = gld<NT>(psi + base + mf_off<KQ>(s, a));
          b[0][s] = h ? f.y : f.x;
          b[1][s] = h ? f.w : f.z;
        }
      } else {
#pragma unroll
        for (int t = 0; t < KS / 2; ++t) {
          const float4 f = gld<NT>(psi + base + mf_off<KQ>(t, a));
          b[0][2 * t] = h ? f.y : f.x;
          b[0][2 * t + 1] = h ? f.w : f.z;
        }
      }
      const float* A = reinterpret_cast<const float*>(lds4);
#pragma unroll 1
      for (int mt = 0; mt < MT; ++mt) {
        f32x16 acc[COLS];
#pragma unroll
        for (int c = 0; c < COLS; ++c)
#pragma unroll
          for (int v = 0; v < 16; ++v) acc[c][v] = 0.f;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          const float av = A[(mt * KS + s) * 64 + lane];
#pragma unroll
          for (int c = 0; c < COLS; ++c) acc[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, b[c][s], acc[c], 0, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = 16 * mt + 4 * q + 2 * h;  // rows 2r, 2r+1, 2r+2, 2r+3
          if constexpr (LAYOUT == kLayoutPair) {
            gst<NT>(psi + base + mf_off<KQ>(r, a), make_float4(acc[0][4 * q], acc[0][4 * q + 1], acc[1][4 * q], acc[1][4 * q + 1]));
            gst<NT>(psi + base + mf_off<KQ>(r + 1, a), make_float4(acc[0][4 * q + 2], acc[0][4 * q + 3], acc[1][4 * q + 2], acc[1][4 * q + 3]));
          } else {
            gst<NT>(psi + base + mf_off<KQ>(r >> 1, a), make_float4(acc[0][4 * q], acc[0][4 * q + 1], acc[0][4 * q + 2], acc[0][4 * q + 3]));
          }
        }
      }
    } else {
      // ---- split precision: k-step s covers amplitudes 8s .. 8s+7; this
      //      lane supplies amplitudes 8s + 4h .. 8s + 4h + 3 (re, im each) ----
      using frag_t = typename std::conditional<PREC == SV_PREC_BF16X3, bf16x8, f16x8>::type;
      frag_t bhi[COLS][KS], blo[COLS][KS];
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        float x[COLS][8];
        if constexpr (LAYOUT == kLayoutPair) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float4 f = gld<NT>(psi + base + mf_off<KQ>(8 * s + 4 * h + q, a));
            x[0][2 * q] = f.x;
            x[0][2 * q + 1] = f.y;
            x[1][2 * q] = f.z;
            x[1][2 * q + 1] = f.w;
          }
        } else {
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const float4 f = gld<NT>(psi + base + mf_off<KQ>(4 * s + 2 * h + q, a));
            x[0][4 * q] = f.x;
            x[0][4 * q + 1] = f.y;
            x[0][4 * q + 2] = f.z;
            x[0][4 * q + 3] = f.w;
          }
        }
#pragma unroll
        for (int c = 0; c < COLS; ++c)
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            if constexpr (PREC == SV_PREC_BF16X3) {
              const short hi = dev_bf16(x[c][e]);
              bhi[c][s][e] = hi;
              blo[c][s][e] = dev_bf16(x[c][e] - dev_bf16_f(hi));
            } else {
              const float xs = x[c][e] * kF16Scale;
              const _Float16 hi = (_Float16)xs;
              bhi[c][s][e] = hi;
              blo[c][s][e] = (_Float16)((xs - (float)hi) * kF16LoScale);
            }
          }
      }
      const frag_t* A = reinterpret_cast<const frag_t*>(lds4);
#pragma unroll 1
      for (int mt = 0; mt < MT; ++mt) {
        f32x16 acc[COLS], cor[COLS];
#pragma unroll
        for (int c = 0; c < COLS; ++c)
#pragma unroll
          for (int v = 0; v < 16; ++v) acc[c][v] = cor[c][v] = 0.f;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          const frag_t ahi = A[((mt * KS + s) * 2 + 0) * 64 + lane];
          const frag_t alo = A[((mt * KS + s) * 2 + 1) * 64 + lane];
#pragma unroll
          for (int c = 0; c < COLS; ++c) {
            if constexpr (PREC == SV_PREC_BF16X3) {
              acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, bhi[c][s], acc[c], 0, 0, 0);
              acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, blo[c][s], acc[c], 0, 0, 0);
              acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo, bhi[c][s], acc[c], 0, 0, 0);
            } else {
              acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ahi, bhi[c][s], acc[c], 0, 0, 0);
              cor[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ahi, blo[c][s], cor[c], 0, 0, 0);
              cor[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(alo, bhi[c][s], cor[c], 0, 0, 0);
            }
          }
        }
        if constexpr (PREC == SV_PREC_FP16X3) {
#pragma unroll
          for (int c = 0; c < COLS; ++c)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[c][v] = (acc[c][v] + cor[c][v] * (1.f / kF16LoScale)) * (1.f / kF16Scale);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = 16 * mt + 4 * q + 2 * h;
          if constexpr (LAYOUT == kLayoutPair) {
            gst<NT>(psi + base + mf_off<KQ>(r, a), make_float4(acc[0][4 * q], acc[0][4 * q + 1], acc[1][4 * q], acc[1][4 * q + 1]));
            gst<NT>(psi + base + mf_off<KQ>(r + 1, a), make_float4(acc[0][4 * q + 2], acc[0][4 * q + 3], acc[1][4 * q + 2], acc[1][4 * q + 3]));
          } else {
            gst<NT>(psi + base + mf_off<KQ>(r >> 1, a), make_float4(acc[0][4 * q], acc[0][4 * q + 1], acc[0][4 * q + 2], acc[0][4 * q + 3]));
          }
        }
      }
    }
  }
}

template <int K, int PREC, int LAYOUT, bool NT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8))) void k_apply_mfma_rolled(
    float4* __restrict__ psi, const float4* __restrict__ Ag, const MfmaArgs a) {
  extern __shared__ float4 lds4[];
  mfma_body<K, PREC, LAYOUT, NT>(psi, Ag, a, lds4);
}

// ---- passes with targets on amplitude bits 1..3 -----------------------------
//
// A target on element bit t in {0, 1, 2} (amplitude bit t + 1) splits every
// 128-byte line (8 elements) between the loads of different local indices:
// a load instruction of the plain layout touches only half (or a quarter, or
// an eighth) of each line, so such passes cannot stream non-temporally.  Here
// the m low targets (set TM, m = popcount) are handled by a lane exchange:
//
//   * lane j (of 32) owns the group G(j) = u(j) | c(j) << (5 - m) of the
//     tile, where c(j) are j's bits at the positions in TM and u(j) its
//     other bits (both packed ascending);
//   * load "slot" X of a unit reads, in lane j, the element of group
//     u(j) | X << (5 - m) whose low-target local bits are c(j): the 8 lanes
//     of an aligned octet then read the 8 elements of one whole line;
//   * after the 2^m slots of a unit are loaded, a butterfly over the m
//     targets (swaps with lane j ^ 2^t, t in TM) is the transpose that gives
//     every lane the 2^m elements of its own group; stores undo it the same
//     way (the transpose is its own inverse).
//
// A unit is 8 elements per lane covering element-local bits 0..2 (4 for the
// k = 4 bit-0-target layout); the real matrix A' is encoded with its rows
// and columns permuted so that each lane's k-rows (loads) and output rows
// (stores) of one unit are exactly those 8 elements.

// Unit geometry, shared by the kernel and the host encoding.
//   PAIR split loads:  k-steps 2p, 2p+1; element e = 16p + 8h + 4 (s & 1) + q
//   Q0 split loads:    k >= 5: k-steps 4p..4p+3, element t = 16p + 8h + 2 (s & 3) + q;
//                      k = 4: t = 4h + 2s + q
//   stores (every precision; output row i = 8q + 4h + 2w + ri of tile mt):
//     PAIR: amplitude 16 mt + 8h + 2q + w;
//     Q0:   amplitude 2t + w, t = 16 (mt >> 1) + 8h + 4 (mt & 1) + q (k >= 5), t = 4h + q (k = 4)
//   FP32 loads keep the natural order (every lane loads every element).
inline int x_pair_load_amp(int s, int h, int q) { return 16 * (s >> 1) + 8 * h + 4 * (s & 1) + q; }
inline int x_q0_load_elem(int k, int s, int h, int q) {
  return k >= 5 ? 16 * (s >> 2) + 8 * h + 2 * (s & 3) + q : 4 * h + 2 * s + q;
}
inline int x_store_amp(int layout, int k, int mt, int i) {
  const int q = i >> 3, h = (i >> 2) & 1, w = (i >> 1) & 1;
  if (layout == kLayoutPair) return 16 * mt + 8 * h + 2 * q + w;
  const int t = k >= 5 ? 16 * (mt >> 1) + 8 * h + 4 * (mt & 1) + q : 4 * h + q;
  return 2 * t + w;
}

template <int K, int PREC, int LAYOUT, int TM>
__device__ __forceinline__ void mfma_body_x(float4* __restrict__ psi, const float4* __restrict__ Ag,
                                            const MfmaArgs& a, float4* lds4) {
  constexpr int DK = 1 << K;
  constexpr int MT = (2 * DK) / 32;
  constexpr bool SPLIT = PREC != SV_PREC_FP32_MFMA;
  constexpr int KS = SPLIT ? (2 * DK) / 16 : DK;
  constexpr int FRAG_BYTES = SPLIT ? MT * KS * 2 * 64 * 16 : MT * KS * 64 * 4;
  constexpr int KQ = LAYOUT == kLayoutPair ? K : K - 1;
  constexpr int COLS = LAYOUT == kLayoutPair ? 2 : 1;
  constexpr int M = LowBits<TM>::m;
  constexpr int XM = (1 << M) - 1;
  constexpr bool Q0K4 = LAYOUT == kLayoutQ0 && K == 4;  // 4-element units
  static_assert(!(Q0K4 && M > 2), "k = 4 with bit 0 as a target covers two low local bits per unit");
  const int tid = threadIdx.x;
  const unsigned v = blockIdx.x & ((1u << a.vbits) - 1);
  const uint64_t wg = blockIdx.x >> a.vbits;
  const uint64_t cb = a.cbits[v];
  Ag += (size_t)v * (FRAG_BYTES / 16);
  for (int i = tid; i < FRAG_BYTES / 16; i += 256) lds4[i] = Ag[i];
  __syncthreads();
  const int lane = tid & 63, h = lane >> 5, j = lane & 31;
  const int uj = compress_bits<5>(j, ~TM & 31), cj = compress_bits<5>(j, TM);
  // element offsets of the slots' group bits and of this lane's low-target bits
  uint64_t xoff[XM + 1];
#pragma unroll
  for (int X = 0; X <= XM; ++X) {
    uint64_t g = (uint64_t)X << (5 - M);
#pragma unroll
    for (int q = 0; q < KQ + kMfmaCtrl; ++q) g = ((g & ~a.ins[q]) << 1) | (g & a.ins[q]);
    xoff[X] = g;
  }
  uint64_t offc = 0;
#pragma unroll
  for (int i = 0; i < M; ++i)
    if ((cj >> i) & 1) offc += a.stride[i];
  uint64_t stride[KQ];  // local copy: the helpers below never take the kernel argument's address
#pragma unroll
  for (int i = 0; i < KQ; ++i) stride[i] = a.stride[i];
  auto off = [&](int l) __attribute__((always_inline)) {
    uint64_t o = 0;
#pragma unroll
    for (int i = 0; i < KQ; ++i)
      if ((l >> i) & 1) o += stride[i];
    return o;
  };
  // one unit: N registers; register r reads slot r & XM at local index
  // ebase + (r & ~XM) (its low-target bits come from this lane's c)
  auto load_unit = [&](auto& R, uint64_t b0, int ebase) __attribute__((always_inline)) {
    constexpr int N = sizeof(R) / sizeof(R[0]);
#pragma unroll
    for (int r = 0; r < N; ++r) R[r] = gld<true>(psi + b0 + xoff[r & XM] + off(ebase + (r & ~XM)));
    xtranspose<TM>(R, j);
  };
  auto store_unit = [&](auto& R, uint64_t b0, int ebase) __attribute__((always_inline)) {
    constexpr int N = sizeof(R) / sizeof(R[0]);
    xtranspose<TM>(R, j);
#pragma unroll
    for (int r = 0; r < N; ++r) gst<true>(psi + b0 + xoff[r & XM] + off(ebase + (r & ~XM)), R[r]);
  };
  const uint64_t wstride = (uint64_t)(gridDim.x >> a.vbits) * 4;
  for (uint64_t wt = wg * 4 + (tid >> 6); wt < a.tiles; wt += wstride) {
    const uint64_t b0 = mf_base<KQ>(wt * 32 + uj, cb, a) + offc;
    // ---------------- B operand ----------------
    using frag_t = typename std::conditional<PREC == SV_PREC_BF16X3, bf16x8, f16x8>::type;
    float bf[COLS][SPLIT ? 1 : KS];
    frag_t bhi[COLS][SPLIT ? KS : 1], blo[COLS][SPLIT ? KS : 1];
    auto split = [&](int c, int s, const float (&x)[8]) __attribute__((always_inline)) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        if constexpr (PREC == SV_PREC_BF16X3) {
          const short hi = dev_bf16(x[e]);
          bhi[c][s][e] = hi;
          blo[c][s][e] = dev_bf16(x[e] - dev_bf16_f(hi));
        } else {
          const float xs = x[e] * kF16Scale;
          const _Float16 hi = (_Float16)xs;
          bhi[c][s][e] = hi;
          blo[c][s][e] = (_Float16)((xs - (float)hi) * kF16LoScale);
        }
      }
    };
    if constexpr (!SPLIT) {
      if constexpr (LAYOUT == kLayoutPair) {
#pragma unroll
        for (int p = 0; p < KS / 8; ++p) {
          float4 R[8];
          load_unit(R, b0, 8 * p);
#pragma unroll
          for (int r = 0; r < 8; ++r) {
            bf[0][8 * p + r] = h ? R[r].y : R[r].x;
            bf[1][8 * p + r] = h ? R[r].w : R[r].z;
          }
        }
      } else {
#pragma unroll
        for (int p = 0; p < KS / 16; ++p) {
          float4 R[8];
          load_unit(R, b0, 8 * p);
#pragma unroll
          for (int r = 0; r < 8; ++r) {
            bf[0][2 * (8 * p + r)] = h ? R[r].y : R[r].x;
            bf[0][2 * (8 * p + r) + 1] = h ? R[r].w : R[r].z;
          }
        }
      }
    } else if constexpr (LAYOUT == kLayoutPair) {
#pragma unroll
      for (int p = 0; p < KS / 2; ++p) {
        float4 R[8];
        load_unit(R, b0, 16 * p + 8 * h);
#pragma unroll
        for (int s1 = 0; s1 < 2; ++s1) {
          float x0[8], x1[8];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float4 f = R[4 * s1 + q];
            x0[2 * q] = f.x;
            x0[2 * q + 1] = f.y;
            x1[2 * q] = f.z;
            x1[2 * q + 1] = f.w;
          }
          split(0, 2 * p + s1, x0);
          split(1, 2 * p + s1, x1);
        }
      }
    } else if constexpr (!Q0K4) {
#pragma unroll
      for (int p = 0; p < KS / 4; ++p) {
        float4 R[8];
        load_unit(R, b0, 16 * p + 8 * h);
#pragma unroll
        for (int s3 = 0; s3 < 4; ++s3) {
          float x[8];
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const float4 f = R[2 * s3 + q];
            x[4 * q] = f.x;
            x[4 * q + 1] = f.y;
            x[4 * q + 2] = f.z;
            x[4 * q + 3] = f.w;
          }
          split(0, 4 * p + s3, x);
        }
      }
    } else {
      float4 R[4];
      load_unit(R, b0, 4 * h);
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        float x[8];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const float4 f = R[2 * s + q];
          x[4 * q] = f.x;
          x[4 * q + 1] = f.y;
          x[4 * q + 2] = f.z;
          x[4 * q + 3] = f.w;
        }
        split(0, s, x);
      }
    }
    // ---------------- products of one 32-row output tile ----------------
    auto tile = [&](int mt, f32x16 (&acc)[COLS]) __attribute__((always_inline)) {
      if constexpr (!SPLIT) {
        const float* A = reinterpret_cast<const float*>(lds4);
#pragma unroll
        for (int c = 0; c < COLS; ++c)
#pragma unroll
          for (int e = 0; e < 16; ++e) acc[c][e] = 0.f;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          const float av = A[(mt * KS + s) * 64 + lane];
#pragma unroll
          for (int c = 0; c < COLS; ++c) acc[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bf[c][s], acc[c], 0, 0, 0);
        }
      } else {
        const frag_t* A = reinterpret_cast<const frag_t*>(lds4);
        f32x16 cor[COLS];
#pragma unroll
        for (int c = 0; c < COLS; ++c)
#pragma unroll
          for (int e = 0; e < 16; ++e) acc[c][e] = cor[c][e] = 0.f;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          const frag_t ahi = A[((mt * KS + s) * 2 + 0) * 64 + lane];
          const frag_t alo = A[((mt * KS + s) * 2 + 1) * 64 + lane];
#pragma unroll
          for (int c = 0; c < COLS; ++c) {
            if constexpr (PREC == SV_PREC_BF16X3) {
              acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, bhi[c][s], acc[c], 0, 0, 0);
              acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, blo[c][s], acc[c], 0, 0, 0);
              acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo, bhi[c][s], acc[c], 0, 0, 0);
            } else {
              acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ahi, bhi[c][s], acc[c], 0, 0, 0);
              cor[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ahi, blo[c][s], cor[c], 0, 0, 0);
              cor[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(alo, bhi[c][s], cor[c], 0, 0, 0);
            }
          }
        }
        if constexpr (PREC == SV_PREC_FP16X3) {
#pragma unroll
          for (int c = 0; c < COLS; ++c)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[c][e] = (acc[c][e] + cor[c][e] * (1.f / kF16LoScale)) * (1.f / kF16Scale);
        }
      }
    };
    // ---------------- outputs ----------------
    if constexpr (LAYOUT == kLayoutPair) {
#pragma unroll 1
      for (int mt = 0; mt < MT; ++mt) {
        f32x16 acc[COLS];
        tile(mt, acc);
        float4 O[8];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int w = 0; w < 2; ++w)
            O[2 * q + w] = make_float4(acc[0][4 * q + 2 * w], acc[0][4 * q + 2 * w + 1], acc[1][4 * q + 2 * w],
                                       acc[1][4 * q + 2 * w + 1]);
        store_unit(O, b0, 16 * mt + 8 * h);
      }
    } else if constexpr (!Q0K4) {
#pragma unroll 1
      for (int mp = 0; mp < MT / 2; ++mp) {
        float4 O[8];
#pragma unroll
        for (int w = 0; w < 2; ++w) {
          f32x16 acc[COLS];
          tile(2 * mp + w, acc);
#pragma unroll
          for (int q = 0; q < 4; ++q)
            O[4 * w + q] = make_float4(acc[0][4 * q], acc[0][4 * q + 1], acc[0][4 * q + 2], acc[0][4 * q + 3]);
        }
        store_unit(O, b0, 16 * mp + 8 * h);
      }
    } else {
      f32x16 acc[COLS];
      tile(0, acc);
      float4 O[4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        O[q] = make_float4(acc[0][4 * q], acc[0][4 * q + 1], acc[0][4 * q + 2], acc[0][4 * q + 3]);
      store_unit(O, b0, 4 * h);
    }
  }
}

template <int K, int PREC, int LAYOUT, int TM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8))) void k_apply_mfma_x(
    float4* __restrict__ psi, const float4* __restrict__ Ag, const MfmaArgs a) {
  extern __shared__ float4 lds4[];
  mfma_body_x<K, PREC, LAYOUT, TM>(psi, Ag, a, lds4);
}

constexpr uint64_t kMfmaGroups = 65536;  // workgroup cap of a matrix-core launch

size_t frag_bytes(int k, int prec) {
  const int dk = 1 << k, mt = 2 * dk / 32;
  if (prec == SV_PREC_FP32_MFMA) return (size_t)mt * dk * 64 * 4;
  return (size_t)mt * (2 * dk / 16) * 2 * 64 * 16;
}

// Entry (row, col) of the real 4M-form matrix with (amplitude, re/im) order.
inline double a4m(const double* mat, int dk, int row, int col) {
  const int r = row >> 1, pr = row & 1, c = col >> 1, pc = col & 1;
  const double ur = mat[2 * (r * dk + c)], ui = mat[2 * (r * dk + c) + 1];
  if (pr == 0) return pc == 0 ? ur : -ui;
  return pc == 0 ? ui : ur;
}

template <int K, int PREC, int LAYOUT, bool NT>
void launch_t(const MfmaArgs& a, void* psi, const unsigned char* data, hipStream_t st) {
  const size_t lds = frag_bytes(K, PREC);
  // Up to 65536 workgroups (256 per CU; 512 are resident at a time), shared
  // out evenly over the control values.  Swept at 30, 32 and 34 qubits over
  // 2048..262144: 65536 is the best or within noise of it for every target
  // set, 2-5 % ahead of 8192 (which gave each wave 8x more tiles at 34 qubits).
  uint64_t per_value = (a.tiles + 3) / 4;
  if (per_value > (kMfmaGroups >> a.vbits)) per_value = kMfmaGroups >> a.vbits;
  const uint64_t blocks = per_value << a.vbits;
  hipLaunchKernelGGL((k_apply_mfma_rolled<K, PREC, LAYOUT, NT>), dim3((unsigned)blocks), dim3(256), lds, st,
                     (float4*)psi, (const float4*)data, a);
}

template <int PREC, int LAYOUT>
void launch_k(int k, bool nt, const MfmaArgs& a, void* psi, const unsigned char* data, hipStream_t st) {
  switch (k * 2 + (nt ? 1 : 0)) {
    case 8: return launch_t<4, PREC, LAYOUT, false>(a, psi, data, st);
    case 9: return launch_t<4, PREC, LAYOUT, true>(a, psi, data, st);
    case 10: return launch_t<5, PREC, LAYOUT, false>(a, psi, data, st);
    case 11: return launch_t<5, PREC, LAYOUT, true>(a, psi, data, st);
    case 12: return launch_t<6, PREC, LAYOUT, false>(a, psi, data, st);
    case 13: return launch_t<6, PREC, LAYOUT, true>(a, psi, data, st);
    default: throw DeviceError{hipErrorInvalidValue, "k_apply_mfma: k must be 4..6"};
  }
}

template <int K, int PREC, int LAYOUT, int TM>
void launch_x_t(const MfmaArgs& a, void* psi, const unsigned char* data, hipStream_t st) {
  const size_t lds = frag_bytes(K, PREC);
  uint64_t per_value = (a.tiles + 3) / 4;
  if (per_value > (kMfmaGroups >> a.vbits)) per_value = kMfmaGroups >> a.vbits;
  const uint64_t blocks = per_value << a.vbits;
  hipLaunchKernelGGL((k_apply_mfma_x<K, PREC, LAYOUT, TM>), dim3((unsigned)blocks), dim3(256), lds, st,
                     (float4*)psi, (const float4*)data, a);
}

template <int PREC, int LAYOUT, int TM>
void launch_x_k(int k, const MfmaArgs& a, void* psi, const unsigned char* data, hipStream_t st) {
  switch (k) {
    case 4:
      if constexpr (!(LAYOUT == kLayoutQ0 && LowBits<TM>::m > 2)) return launch_x_t<4, PREC, LAYOUT, TM>(a, psi, data, st);
      break;
    case 5: return launch_x_t<5, PREC, LAYOUT, TM>(a, psi, data, st);
    case 6: return launch_x_t<6, PREC, LAYOUT, TM>(a, psi, data, st);
    default: break;
  }
  throw DeviceError{hipErrorInvalidValue, "k_apply_mfma_x: unsupported k / low targets"};
}

template <int PREC, int LAYOUT>
void launch_x(int tm, int k, const MfmaArgs& a, void* psi, const unsigned char* data, hipStream_t st) {
  switch (tm) {
    case 1: return launch_x_k<PREC, LAYOUT, 1>(k, a, psi, data, st);
    case 2: return launch_x_k<PREC, LAYOUT, 2>(k, a, psi, data, st);
    case 3: return launch_x_k<PREC, LAYOUT, 3>(k, a, psi, data, st);
    case 4: return launch_x_k<PREC, LAYOUT, 4>(k, a, psi, data, st);
    case 5: return launch_x_k<PREC, LAYOUT, 5>(k, a, psi, data, st);
    case 6: return launch_x_k<PREC, LAYOUT, 6>(k, a, psi, data, st);
    case 7: return launch_x_k<PREC, LAYOUT, 7>(k, a, psi, data, st);
    default: throw DeviceError{hipErrorInvalidValue, "k_apply_mfma_x: low-target mask"};
  }
}

}  // namespace

// Low-target mask of the lane-exchange form (0: the plain kernel).  Used for
// streamed states when a target (other than bit 0) sits on amplitude bits
// 1..3 and no control does; a bit-0-target pass with k = 4 covers only two
// low local bits per unit.
int mfma_exchange_mask(int n, const Pass& p) {
  if (n < kern::kNtMinQubits || (p.cmask & 0xEull)) return 0;
  const bool q0 = p.s[0] == 0;
  int tm = 0;
  for (int j = q0 ? 1 : 0; j < p.k; ++j)
    if (p.s[j] >= 1 && p.s[j] <= 3) tm |= 1 << (p.s[j] - 1);
  if (q0 && p.k == 4 && __builtin_popcount(tm) > 2) return 0;
  return tm;
}

bool mfma_supported(int k, int precision) {
  return k >= 4 && k <= 6 &&
         (precision == SV_PREC_FP32_MFMA || precision == SV_PREC_BF16X3 || precision == SV_PREC_FP16X3);
}

size_t mfma_data_bytes(const Pass& p) { return frag_bytes(p.k, p.precision) * (p.nmux > 1 ? p.nmux : 1); }

// A' in fragment order.  FP32: [mt][s][lane] with lane (h, i) holding
// A'[32 mt + i][2 s + h].  Split: [mt][s][part][lane][e] with lane (h, i)
// holding A'[32 mt + i][16 s + 8 h + e]; part 0 = hi, part 1 = lo.
void mfma_encode(const Pass& p, const double* mat, unsigned char* dst) {
  const int dk = 1 << p.k, mt_n = 2 * dk / 32;
  // With the lane exchange (p.mfma_x) the rows and the split modes' columns
  // of A' are permuted to the unit geometry of the exchange kernel.
  const int layout = p.s[0] == 0 ? kLayoutQ0 : kLayoutPair;
  auto row_of = [&](int mt, int i) {
    return p.mfma_x ? 2 * x_store_amp(layout, p.k, mt, i) + (i & 1) : 32 * mt + i;
  };
  auto split_col_of = [&](int s, int h, int e) {
    if (!p.mfma_x) return 16 * s + 8 * h + e;
    if (layout == kLayoutPair) return 2 * x_pair_load_amp(s, h, e >> 1) + (e & 1);
    return 2 * (2 * x_q0_load_elem(p.k, s, h, e >> 2) + ((e >> 1) & 1)) + (e & 1);
  };
  if (p.precision == SV_PREC_FP32_MFMA) {
    float* f = reinterpret_cast<float*>(dst);
    for (int mt = 0; mt < mt_n; ++mt)
      for (int s = 0; s < dk; ++s)
        for (int lane = 0; lane < 64; ++lane) {
          const int h = lane >> 5, i = lane & 31;
          f[(mt * dk + s) * 64 + lane] = (float)a4m(mat, dk, row_of(mt, i), 2 * s + h);
        }
    return;
  }
  const int ks_n = 2 * dk / 16;
  uint16_t* o = reinterpret_cast<uint16_t*>(dst);
  for (int mt = 0; mt < mt_n; ++mt)
    for (int s = 0; s < ks_n; ++s)
      for (int lane = 0; lane < 64; ++lane)
        for (int e = 0; e < 8; ++e) {
          const int h = lane >> 5, i = lane & 31;
          const double v = a4m(mat, dk, row_of(mt, i), split_col_of(s, h, e));
          uint16_t hi, lo;
          if (p.precision == SV_PREC_BF16X3) {
            hi = host_bf16((float)v);
            lo = host_bf16((float)(v - (double)host_bf16_to_f(hi)));
          } else {
            hi = host_f16((float)v);
            lo = host_f16((float)((v - (double)host_f16_to_f(hi)) * (double)kF16LoScale));
          }
          const size_t base = (((size_t)(mt * ks_n + s) * 2) * 64 + lane) * 8 + e;
          o[base] = hi;
          o[base + (size_t)64 * 8] = lo;
        }
}

bool mfma_ctrl_supported(int n, int k, uint64_t cmask) {
  const int c = __builtin_popcountll(cmask);
  return c <= kMfmaCtrl && (cmask & 1) == 0 && n - 1 - k - c >= 5;
}

void launch_mfma(const Pass& p, int n, void* psi, const unsigned char* data, hipStream_t st) {
  if (p.cmask && !mfma_ctrl_supported(n, p.k, p.cmask))
    throw DeviceError{hipErrorInvalidValue, "k_apply_mfma: unsupported controls"};
  MfmaArgs a{};
  int pos[SV_MAX_K];
  int layout;
  const int c = __builtin_popcountll(p.cmask);
  if (p.s[0] == 0) {
    layout = kLayoutQ0;
    a.kq = p.k - 1;
    for (int j = 0; j < a.kq; ++j) pos[j] = p.s[j + 1] - 1;
    a.tiles = ((uint64_t)1 << (n - p.k - c)) / 32;
  } else {
    layout = kLayoutPair;
    a.kq = p.k;
    for (int j = 0; j < a.kq; ++j) pos[j] = p.s[j] - 1;
    a.tiles = ((uint64_t)1 << (n - 1 - p.k - c)) / 32;
  }
  for (int j = 0; j < a.kq; ++j) a.stride[j] = (uint64_t)1 << pos[j];
  // zero insertion at targets and controls together, in ascending position;
  // amplitude bit b >= 1 is element bit b - 1 (an element holds bits 0 free)
  // With nmux > 1 one launch covers every control value: value v sets the
  // t-th control (ascending) to bit t of v; else the one value p.cval.
  int ins[SV_MAX_K + kMfmaCtrl], m = 0, cpos[kMfmaCtrl], nc = 0;
  for (int j = 0; j < a.kq; ++j) ins[m++] = pos[j];
  for (int b = 1; b < 64; ++b)
    if ((p.cmask >> b) & 1) {
      ins[m++] = b - 1;
      cpos[nc++] = b - 1;
    }
  std::sort(ins, ins + m);
  if (p.nmux > 1) {
    if (p.nmux != (1 << nc)) throw DeviceError{hipErrorInvalidValue, "k_apply_mfma: control values"};
    a.vbits = nc;
    for (int v = 0; v < p.nmux; ++v)
      for (int t = 0; t < nc; ++t)
        if ((v >> t) & 1) a.cbits[v] |= (uint64_t)1 << cpos[t];
  } else {
    for (int t = 0; t < nc; ++t)
      if ((p.cval >> (cpos[t] + 1)) & 1) a.cbits[0] |= (uint64_t)1 << cpos[t];
  }
  for (int j = 0; j < SV_MAX_K + kMfmaCtrl; ++j) a.ins[j] = j < m ? ((uint64_t)1 << ins[j]) - 1 : ~(uint64_t)0;
  if (a.tiles == 0) throw DeviceError{hipErrorInvalidValue, "k_apply_mfma: state too small for a 32-group tile"};
  const bool pair = layout == kLayoutPair;
  if (p.mfma_x) {
    if (p.mfma_x != mfma_exchange_mask(n, p)) throw DeviceError{hipErrorInvalidValue, "k_apply_mfma: stale exchange mask"};
    switch (p.precision) {
      case SV_PREC_FP32_MFMA:
        return pair ? launch_x<SV_PREC_FP32_MFMA, kLayoutPair>(p.mfma_x, p.k, a, psi, data, st)
                    : launch_x<SV_PREC_FP32_MFMA, kLayoutQ0>(p.mfma_x, p.k, a, psi, data, st);
      case SV_PREC_BF16X3:
        return pair ? launch_x<SV_PREC_BF16X3, kLayoutPair>(p.mfma_x, p.k, a, psi, data, st)
                    : launch_x<SV_PREC_BF16X3, kLayoutQ0>(p.mfma_x, p.k, a, psi, data, st);
      case SV_PREC_FP16X3:
        return pair ? launch_x<SV_PREC_FP16X3, kLayoutPair>(p.mfma_x, p.k, a, psi, data, st)
                    : launch_x<SV_PREC_FP16X3, kLayoutQ0>(p.mfma_x, p.k, a, psi, data, st);
      default:
        throw DeviceError{hipErrorInvalidValue, "k_apply_mfma: precision"};
    }
  }
  // streaming stores only when no target or control leaves partial lines
  bool nt = kern::gather_nt(n, p.k, p.s);
  if (p.cmask & 0xEull) nt = false;
  switch (p.precision) {
    case SV_PREC_FP32_MFMA:
      pair ? launch_k<SV_PREC_FP32_MFMA, kLayoutPair>(p.k, nt, a, psi, data, st)
           : launch_k<SV_PREC_FP32_MFMA, kLayoutQ0>(p.k, nt, a, psi, data, st);
      break;
    case SV_PREC_BF16X3:
      pair ? launch_k<SV_PREC_BF16X3, kLayoutPair>(p.k, nt, a, psi, data, st)
           : launch_k<SV_PREC_BF16X3, kLayoutQ0>(p.k, nt, a, psi, data, st);
      break;
    case SV_PREC_FP16X3:
      pair ? launch_k<SV_PREC_FP16X3, kLayoutPair>(p.k, nt, a, psi, data, st)
           : launch_k<SV_PREC_FP16X3, kLayoutQ0>(p.k, nt, a, psi, data, st);
      break;
    default:
      throw DeviceError{hipErrorInvalidValue, "k_apply_mfma: precision"};
  }
}

}  // namespace sv
