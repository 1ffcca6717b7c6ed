// Reads of the state that write nothing back (the expectation-value kernel
// of Sec. IV, and the Born probabilities of Eq. 1 behind measurement):
// Pauli-string expectations, marginal probabilities and inverse-CDF
// sampling.  Every sum is in FP64 in a fixed order, so results do not vary
// between runs; squares and products of complex64 amplitudes are formed in
// FP64, where they are exact.
#include "k_common.h"

namespace sv {

namespace {
using kern::gld;

constexpr int kThreads = 256;
constexpr int kMaxBlocks = 2048;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double sq(const float2 a) {
  return (double)a.x * (double)a.x + (double)a.y * (double)a.y;
}

// ------------------------------------------------------------ Pauli strings
// Up to kTerms strings that share the flip mask f = X|Y part.  For P = i^ny
// X^f Z^z: <psi|P|psi> = i^ny sum_i (-1)^{|(i^f) & z|} conj(c_i) c_{i^f}.
// With f != 0 the sum runs over pairs (i, j = i^f) with bit h (the highest
// bit of f) clear in i; the pair contributes s_i w + s_j conj(w), w =
// conj(c_i) c_j, s_j = (-1)^{|i & z|} and s_i = s_j (-1)^{|f & z|}.  So a
// term with |f & z| even collects 2 s_j Re w (a real sum) and one with
// |f & z| odd collects -2i s_j Im w.  Each amplitude is read once.
constexpr int kTerms = 8;
struct PauliArgs {
  uint64_t f;
  uint64_t items;          // float4 elements (f == 0 or f == 1) or element quads; a power of two
  uint64_t lowmask;        // ones below bit h
  uint64_t z[kTerms];
  uint32_t chi[kTerms][4]; // high words of the FP64 coefficients (+-1 or 0) of each item value
  uint32_t odd;            // bit t: |f & z_t| is odd
};

// First amplitude index of item x: 2x for elements; for quads, 2x with a
// zero inserted at bit h (the bit-h-clear member of the pair).
template <int MODE>
__device__ __forceinline__ uint64_t first_amp(const PauliArgs& a, uint64_t x) {
  const uint64_t g = 2 * x;
  return MODE == 2 ? ((g & ~a.lowmask) << 1) | (g & a.lowmask) : g;
}

__device__ __forceinline__ uint32_t sign_bits(const PauliArgs& a, uint64_t i, int terms) {
  uint32_t s = 0;
#pragma unroll
  for (int t = 0; t < kTerms; ++t)
    if (t < terms) s |= (uint32_t)(__popcll(i & a.z[t]) & 1) << t;
  return s;
}

__device__ __forceinline__ double coef(uint32_t hi, uint32_t sign) {
  return __longlong_as_double((long long)((uint64_t)(hi ^ (sign << 31)) << 32));
}

// The values an item contributes, before signs: MODE 0, the two Born
// probabilities |c_i|^2, |c_{i+1}|^2; MODE 1, Re and Im of w = conj(c_i)
// c_{i+1}; MODE 2, Re and Im of w for the pairs at i and i + 1.
template <int MODE>
__device__ __forceinline__ void item_values(const float4 A, const float4 B, bool fodd, double* v) {
  if (MODE == 0) {
    v[0] = sq(make_float2(A.x, A.y));
    v[1] = sq(make_float2(A.z, A.w));
  } else if (MODE == 1) {
    v[0] = (double)A.x * A.z + (double)A.y * A.w;
    v[1] = (double)A.x * A.w - (double)A.y * A.z;
  } else {
    const float2 c0 = make_float2(A.x, A.y), c1 = make_float2(A.z, A.w);
    const float2 p0 = fodd ? make_float2(B.z, B.w) : make_float2(B.x, B.y);
    const float2 p1 = fodd ? make_float2(B.x, B.y) : make_float2(B.z, B.w);
    v[0] = (double)c0.x * p0.x + (double)c0.y * p0.y;
    v[1] = (double)c0.x * p0.y - (double)c0.y * p0.x;
    v[2] = (double)c1.x * p1.x + (double)c1.y * p1.y;
    v[3] = (double)c1.x * p1.y - (double)c1.y * p1.x;
  }
}

__device__ __forceinline__ double flip_if(double x, uint32_t bit) {
  return __longlong_as_double(__double_as_longlong(x) ^ (long long)((uint64_t)bit << 63));
}

// Two ways to apply the per-m signs (bit t of bits for term t):
// - SIGNS: bits are this item's signs; the coefficients take them (a sign
//   flip of each coefficient's high word, scalar work per value and term);
// - FLIPS: the accumulator holds B_t = (sign of the last item) * (sum so
//   far) and bits are where the sign changed since the last item: B_t is
//   turned over (one vector XOR per term), then the values are added with
//   fixed coefficients.
// Quads (mode 2: four values per item) measured faster with FLIPS (5.7
// against 6.1 ms for 8 terms at 32 qubits), elements (two values) with
// SIGNS (5.6-5.7 against 6.3 ms).
template <int MODE>
constexpr bool kFlips = MODE == 2;

template <int MODE, int TERMS>
__device__ __forceinline__ void accumulate(double* acc, const PauliArgs& a, uint32_t bits, const double* v) {
  constexpr int NV = MODE == 2 ? 4 : 2;
#pragma unroll
  for (int t = 0; t < TERMS; ++t) {
    const uint32_t b = (bits >> t) & 1u;
    if constexpr (kFlips<MODE>) {
      acc[t] = flip_if(acc[t], b);
#pragma unroll
      for (int c = 0; c < NV; ++c) acc[t] = fma(coef(a.chi[t][c], 0u), v[c], acc[t]);
    } else {
#pragma unroll
      for (int c = 0; c < NV; ++c) acc[t] = fma(coef(a.chi[t][c], b), v[c], acc[t]);
    }
  }
}

// Apply each thread's own signs (bit t of own), then sum the block's
// threads in a fixed order into partials[block][t].
__device__ __forceinline__ void block_partials(const double* acc, uint32_t own, double* __restrict__ partials) {
  __shared__ double part[kThreads / 64][kTerms];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int t = 0; t < kTerms; ++t) {
    const double r = wave_sum(((own >> t) & 1) ? -acc[t] : acc[t]);
    if (lane == 0) part[w][t] = r;
  }
  __syncthreads();
  if (threadIdx.x < kTerms) {
    double v = 0.0;
    for (int x = 0; x < kThreads / 64; ++x) v += part[x][threadIdx.x];
    partials[(size_t)blockIdx.x * kTerms + threadIdx.x] = v;
  }
}

// Thread T of the grid (nth = gridDim.x * kThreads threads, a power of two)
// owns items x = T + m nth, m = 0, 1, ...  The bits of first_amp(T) and
// first_amp(m nth) are disjoint, so the sign (-1)^{|i & z_t|} of every pair
// splits into a per-thread sign and a per-m sign that is the same for every
// lane; it reaches the sums through wave-uniform coefficients (+-1 or 0:
// the real-or-imaginary choice and the sign of bit 0 of z_t folded in), in
// one of the two ways described at accumulate, and the thread's own sign is
// applied once at the end.  Mode 0 and 1 items are float4 elements
// (amplitudes 2x, 2x + 1); mode 2 items are quads: the element at i (bit h
// clear, i even) and the element holding its partners i ^ f and
// (i + 1) ^ f.  Every thread keeps two items in flight.
template <bool NT, int MODE, int TERMS>
__global__ __launch_bounds__(kThreads) void k_pauli_partial(const float4* __restrict__ psi, const PauliArgs a,
                                                           double* __restrict__ partials) {
  constexpr int NV = MODE == 2 ? 4 : 2;
  double acc[kTerms];
#pragma unroll
  for (int t = 0; t < kTerms; ++t) acc[t] = 0.0;
  const uint64_t nth = (uint64_t)gridDim.x * kThreads;
  const uint64_t T = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
  const uint64_t iT = first_amp<MODE>(a, T);
  const uint64_t i_step = first_amp<MODE>(a, nth);
  const uint32_t step = sign_bits(a, i_step, TERMS);  // m even: m + 1 flips these
  const bool fodd = a.f & 1;  // the partner of i is the odd amplitude of its element
  uint32_t last = 0;  // per-m sign bits of the last item added (FLIPS)
  if (T < a.items) {  // false only past the end of a state of fewer than nth items
    // the trip count and has1 are the same for every lane, so the four
    // loads of an iteration issue back to back (a lone last item loads
    // its own element twice)
    const uint64_t M = a.items >= nth ? a.items / nth : 1;
    for (uint64_t m = 0; m < M; m += 2) {
      const bool has1 = m + 1 < M;
      const uint64_t im = first_amp<MODE>(a, m * nth);
      const uint64_t i0 = iT | im, i1 = has1 ? i0 | i_step : i0;
      const float4 A0 = gld<NT>(psi + (i0 >> 1));
      const float4 A1 = gld<NT>(psi + (i1 >> 1));
      float4 B0 = A0, B1 = A1;
      if (MODE == 2) {
        B0 = gld<NT>(psi + (((i0 ^ a.f) & ~(uint64_t)1) >> 1));
        B1 = gld<NT>(psi + (((i1 ^ a.f) & ~(uint64_t)1) >> 1));
      }
      const uint32_t sig = sign_bits(a, im, TERMS);
      double v[NV];
      item_values<MODE>(A0, B0, fodd, v);
      accumulate<MODE, TERMS>(acc, a, kFlips<MODE> ? sig ^ last : sig, v);
      last = sig;
      if (has1) {
        item_values<MODE>(A1, B1, fodd, v);
        accumulate<MODE, TERMS>(acc, a, kFlips<MODE> ? step : sig ^ step, v);
        last = sig ^ step;
      }
    }
  }
  const uint32_t own = sign_bits(a, iT, TERMS) ^ (kFlips<MODE> ? last : 0u);
  block_partials(acc, own, partials);
}

// The same sums on a streamed state, walked the way the sampling chunk sums
// walk it: wave W of NW takes chunks of R = 2048 consecutive items, W,
// W + NW, W + 2 NW, ..., each in 32 steps of 64 lanes, two steps in flight
// (so the waves in flight read a moving window of the state, each its own
// 32 KiB run; the grid-stride walk above spreads every wave over the whole
// state).  Item x = c NW R + W R + k 64 + lane splits into disjoint bit
// fields, so the per-thread part of every sign comes from W R + lane and
// the wave-uniform part from c NW R + k 64.  Needs items to be a multiple
// of NW R.
constexpr uint64_t kChunkItems = 2048;
template <int MODE, int TERMS>
__global__ __launch_bounds__(kThreads) void k_pauli_chunks(const float4* __restrict__ psi, const PauliArgs a,
                                                          double* __restrict__ partials) {
  constexpr int NV = MODE == 2 ? 4 : 2;
  double acc[kTerms];
#pragma unroll
  for (int t = 0; t < kTerms; ++t) acc[t] = 0.0;
  const uint64_t NW = (uint64_t)gridDim.x * (kThreads / 64);
  const uint64_t W = (uint64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const uint64_t iT = first_amp<MODE>(a, W * kChunkItems + lane);
  const uint64_t rounds = a.items / (NW * kChunkItems);
  const bool fodd = a.f & 1;
  uint32_t last = 0;
  for (uint64_t c = 0; c < rounds; ++c) {
    for (uint64_t k = 0; k < kChunkItems / 64; k += 2) {
      const uint64_t im0 = first_amp<MODE>(a, c * NW * kChunkItems + k * 64);
      const uint64_t im1 = first_amp<MODE>(a, c * NW * kChunkItems + (k + 1) * 64);
      const uint64_t i0 = iT | im0, i1 = iT | im1;
      const float4 A0 = gld<true>(psi + (i0 >> 1));
      const float4 A1 = gld<true>(psi + (i1 >> 1));
      float4 B0 = A0, B1 = A1;
      if (MODE == 2) {
        B0 = gld<true>(psi + (((i0 ^ a.f) & ~(uint64_t)1) >> 1));
        B1 = gld<true>(psi + (((i1 ^ a.f) & ~(uint64_t)1) >> 1));
      }
      const uint32_t sig0 = sign_bits(a, im0, TERMS), sig1 = sign_bits(a, im1, TERMS);
      double v[NV];
      item_values<MODE>(A0, B0, fodd, v);
      accumulate<MODE, TERMS>(acc, a, kFlips<MODE> ? sig0 ^ last : sig0, v);
      item_values<MODE>(A1, B1, fodd, v);
      accumulate<MODE, TERMS>(acc, a, kFlips<MODE> ? sig1 ^ sig0 : sig1, v);
      last = sig1;
    }
  }
  const uint32_t own = sign_bits(a, iT, TERMS) ^ (kFlips<MODE> ? last : 0u);
  block_partials(acc, own, partials);
}

// Column sums of the blocks x width matrix of per-block partials, in a fixed
// order: workgroup g owns columns 64 g .. 64 g + 63 (one per lane); each of
// its 16 waves sums a contiguous run of rows, and wave 0 then adds the 16
// wave sums in wave order.  With PAULI the column sums S_t become
// out[2t], out[2t + 1] = Re, Im of sum_i (-1)^{|(i^f) & z_t|} conj(c_i)
// c_{i^f} (the i^ny factor is applied on the host); otherwise out[col] is
// the sum itself.
constexpr int kFinalWaves = 16;
template <bool PAULI>
__global__ __launch_bounds__(64 * kFinalWaves) void k_column_sums(const double* __restrict__ partials, int blocks,
                                                                  int width, int mode, uint32_t odd,
                                                                  double* __restrict__ out) {
  __shared__ double part[kFinalWaves][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int col = blockIdx.x * 64 + lane;
  const int per = (blocks + kFinalWaves - 1) / kFinalWaves;
  const int b0 = w * per, b1 = b0 + per < blocks ? b0 + per : blocks;
  double s = 0.0;
  if (col < width) {
#pragma unroll 8
    for (int b = b0; b < b1; ++b) s += partials[(size_t)b * width + col];
  }
  part[w][lane] = s;
  __syncthreads();
  if (w != 0 || col >= width) return;
  double t = 0.0;
  for (int x = 0; x < kFinalWaves; ++x) t += part[x][lane];
  if (PAULI) {
    const double scale = mode == 0 ? 1.0 : 2.0;
    const bool is_odd = (odd >> col) & 1;
    out[2 * col] = is_odd ? 0.0 : scale * t;
    out[2 * col + 1] = is_odd ? -scale * t : 0.0;
  } else {
    out[col] = t;
  }
}

// ------------------------------------------------------- marginal probabilities
// Chunks of 64 consecutive amplitudes are visited in the order c' = (oh,
// free): chunk c = deposit(free, fc) | deposit(oh, hc), where hc holds the
// measured qubits at or above bit 6 (in chunk units) and fc the others.
// Each wave walks a contiguous range of c', so within a run of equal oh its
// lanes accumulate privately (lane = index bits 0..5).  When oh changes, a
// butterfly over the lane bits that are not measured leaves, in the lanes
// whose unmeasured lane bits are zero, the sum over lanes sharing their
// measured low bits; those lanes (distinct outcomes) add it to the wave's
// own LDS histogram, so no two lanes update one bin at once and the order of
// every sum is fixed.
constexpr int kMaxMeasured = 10;
struct MargArgs {
  uint64_t len;          // 2^n
  uint64_t nchunks;      // 2^(n-6), or 1 for n < 6
  uint64_t fc;           // chunk-index bits that are not measured
  uint64_t hc;           // chunk-index bits that are measured (qubit q >= 6 -> bit q - 6)
  int free_bits;         // popcount(fc)
  int m;
  int q[kMaxMeasured];
  uint32_t low_meas;     // measured qubits among bits 0..5
};

__device__ __forceinline__ uint64_t deposit(uint64_t x, uint64_t mask) {
  uint64_t r = 0;
  for (uint64_t m = mask; m; m &= m - 1, x >>= 1)
    if (x & 1) r |= m & (~m + 1);
  return r;
}

__device__ __forceinline__ int outcome(uint64_t i, const MargArgs& a) {
  int o = 0;
#pragma unroll
  for (int j = 0; j < kMaxMeasured; ++j)
    if (j < a.m) o |= (int)((i >> a.q[j]) & 1) << j;
  return o;
}

template <bool NT>
__global__ __launch_bounds__(kThreads) void k_marginal_partial(const float2* __restrict__ psi, const MargArgs a,
                                                              double* __restrict__ partials) {
  extern __shared__ double hist[];  // [4 waves][2^m]
  const int M = 1 << a.m;
  for (int x = threadIdx.x; x < 4 * M; x += kThreads) hist[x] = 0.0;
  __syncthreads();
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double* __restrict__ h = hist + w * M;
  const bool owner = ((uint32_t)lane & ~a.low_meas & 63u) == 0;
  const uint64_t waves = (uint64_t)gridDim.x * 4;
  const uint64_t per = (a.nchunks + waves - 1) / waves;
  const uint64_t c0 = ((uint64_t)blockIdx.x * 4 + w) * per;
  const uint64_t c1 = c0 + per < a.nchunks ? c0 + per : a.nchunks;
  if (c0 < c1) {
    uint64_t oh = c0 >> a.free_bits;
    uint64_t cf = deposit(c0 & (((uint64_t)1 << a.free_bits) - 1), a.fc);
    uint64_t ch = deposit(oh, a.hc);
    for (uint64_t cp = c0; cp < c1;) {
      const uint64_t run_end = ((oh + 1) << a.free_bits) < c1 ? ((oh + 1) << a.free_bits) : c1;
      double acc = 0.0;
      for (; cp + 4 <= run_end; cp += 4) {
        uint64_t c[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          c[u] = cf | ch;
          cf = ((cf | ~a.fc) + 1) & a.fc;
        }
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = sq(gld<NT>(psi + (c[u] << 6) + lane));
#pragma unroll
        for (int u = 0; u < 4; ++u) acc += v[u];
      }
      for (; cp < run_end; ++cp) {
        const uint64_t i = ((cf | ch) << 6) + lane;
        acc += i < a.len ? sq(psi[i]) : 0.0;
        cf = ((cf | ~a.fc) + 1) & a.fc;
      }
#pragma unroll
      for (int b = 0; b < 6; ++b)
        if (!((a.low_meas >> b) & 1)) acc += __shfl_xor(acc, 1 << b, 64);
      if (owner) h[outcome((ch << 6) + lane, a)] += acc;
      ++oh;
      ch = deposit(oh, a.hc);
    }
  }
  __syncthreads();
  for (int o = threadIdx.x; o < M; o += kThreads) {
    double v = 0.0;
    for (int x = 0; x < 4; ++x) v += hist[x * M + o];
    partials[(size_t)blockIdx.x * M + o] = v;
  }
}

// ------------------------------------------------------------------ sampling
// 1. chunk sums of |c_i|^2 (one wave per chunk of 2^c amplitudes);
// 2. inclusive prefix sums of the chunk sums (blocks of 2048, then the block
//    totals, then the offsets added back);
// 3. per shot (one wave): binary search for the first chunk whose inclusive
//    prefix exceeds u * total, then a wave-wide inclusive scan through that
//    chunk for the first amplitude that crosses the remainder.
template <bool NT>
__global__ __launch_bounds__(kThreads) void k_chunk_sums(const float2* __restrict__ psi, int cbits,
                                                        uint64_t nchunks, double* __restrict__ sums) {
  const uint64_t ch = ((uint64_t)blockIdx.x * kThreads + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (ch >= nchunks) return;  // whole waves leave together
  // 16-byte loads (two amplitudes per lane), several in flight: the sum
  // order per lane stays fixed (cbits >= 1, so a chunk is whole elements)
  const uint64_t len4 = (uint64_t)1 << (cbits - 1);
  const float4* __restrict__ p = reinterpret_cast<const float4*>(psi + (ch << cbits));
  double v = 0.0;
#pragma unroll 8
  for (uint64_t i = lane; i < len4; i += 64) {
    const float4 a = gld<NT>(p + i);
    v += sq(make_float2(a.x, a.y));
    v += sq(make_float2(a.z, a.w));
  }
  v = wave_sum(v);
  if (lane == 0) sums[ch] = v;
}

constexpr int kScanPer = 8;                       // elements per thread
constexpr int kScanBlock = kThreads * kScanPer;   // 2048 elements per block

__device__ double block_exclusive_scan(double v, double* total) {
  __shared__ double wsum[kThreads / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const double y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  double off = 0.0, all = 0.0;
  for (int i = 0; i < kThreads / 64; ++i) {
    if (i < w) off += wsum[i];
    all += wsum[i];
  }
  __syncthreads();
  *total = all;
  return off + x - v;
}

// In place: inclusive prefix within each block of kScanBlock; block totals out.
__global__ __launch_bounds__(kThreads) void k_scan_blocks(double* __restrict__ x, uint64_t count,
                                                         double* __restrict__ totals) {
  const uint64_t base = (uint64_t)blockIdx.x * kScanBlock + (uint64_t)threadIdx.x * kScanPer;
  double loc[kScanPer];
  double run = 0.0;
#pragma unroll
  for (int e = 0; e < kScanPer; ++e) {
    loc[e] = base + e < count ? x[base + e] : 0.0;
    run += loc[e];
    loc[e] = run;
  }
  double total;
  const double off = block_exclusive_scan(run, &total);
#pragma unroll
  for (int e = 0; e < kScanPer; ++e)
    if (base + e < count) x[base + e] = off + loc[e];
  if (threadIdx.x == 0 && totals) totals[blockIdx.x] = total;
}

__global__ __launch_bounds__(kThreads) void k_scan_add(double* __restrict__ x, uint64_t count,
                                                      const double* __restrict__ incl_totals) {
  if (blockIdx.x == 0) return;
  const double off = incl_totals[blockIdx.x - 1];
  const uint64_t base = (uint64_t)blockIdx.x * kScanBlock;
  for (int e = threadIdx.x; e < kScanBlock; e += kThreads)
    if (base + e < count) x[base + e] += off;
}

constexpr uint64_t kNoSample = ~(uint64_t)0;

__global__ __launch_bounds__(kThreads) void k_sample(const float2* __restrict__ psi, int cbits,
                                                    const double* __restrict__ incl, uint64_t nchunks,
                                                    const double* __restrict__ u, uint64_t shots,
                                                    uint64_t* __restrict__ out) {
  const uint64_t shot = ((uint64_t)blockIdx.x * kThreads + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (shot >= shots) return;  // whole waves leave together
  const double total = incl[nchunks - 1];
  if (!(total > 0.0)) {
    if (lane == 0) out[shot] = kNoSample;
    return;
  }
  double target = u[shot] * total;
  const bool past_end = !(target < total);
  // first chunk with incl > target (or, past the end, the first reaching total)
  uint64_t lo = 0, hi = nchunks - 1;
  while (lo < hi) {
    const uint64_t mid = lo + (hi - lo) / 2;
    const bool go_left = past_end ? !(incl[mid] < total) : incl[mid] > target;
    if (go_left) hi = mid;
    else lo = mid + 1;
  }
  const uint64_t ch = lo;
  const double r = (past_end ? total : target) - (ch > 0 ? incl[ch - 1] : 0.0);
  const uint64_t len = (uint64_t)1 << cbits;
  const uint64_t base = ch << cbits;
  double acc = 0.0;
  uint64_t last_nz = kNoSample, found = kNoSample;
  for (uint64_t s = 0; s < len && found == kNoSample; s += 64) {
    const uint64_t i = s + lane;
    const double v = i < len ? sq(psi[base + i]) : 0.0;
    double x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const double y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    const uint64_t nz = __ballot(v > 0.0);
    if (nz) last_nz = base + s + 63 - __clzll(nz);
    if (!past_end) {
      const uint64_t cross = __ballot(acc + x > r && v > 0.0);
      if (cross) found = base + s + __ffsll((long long)cross) - 1;
    }
    acc += __shfl(x, 63, 64);
  }
  if (lane == 0) out[shot] = found != kNoSample ? found : last_nz;
}

unsigned blocks_for(uint64_t items, uint64_t per_thread) {
  uint64_t b = (items + kThreads * per_thread - 1) / (kThreads * per_thread);
  if (b > (uint64_t)kMaxBlocks) b = kMaxBlocks;
  return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

size_t pauli_scratch_bytes() { return sizeof(double) * ((size_t)kMaxBlocks + 1) * 2 * kTerms; }

// out: 2 * kTerms doubles (device).  scratch: pauli_scratch_bytes().
void launch_pauli(const void* psi, int n, uint64_t f, int nt, const uint64_t* z, double* scratch, double* out,
                  hipStream_t st) {
  if (nt < 1 || nt > kTerms) throw DeviceError{hipErrorInvalidValue, "k_pauli: 1..8 terms per sweep"};
  PauliArgs a{};
  a.f = f;
  for (int t = 0; t < nt; ++t) {
    a.z[t] = z[t];
    if (__builtin_popcountll(f & z[t]) & 1) a.odd |= 1u << t;
  }
  if (n < 1 || (n < 64 && (f >> n) != 0)) throw DeviceError{hipErrorInvalidValue, "k_pauli: flip mask past n"};
  int mode;
  if (f == 0 || f == 1) {
    mode = (int)f;
    a.items = (uint64_t)1 << (n - 1);  // n = 1: one element
  } else {
    const int h = 63 - __builtin_clzll(f);  // h >= 1, so n >= 2
    mode = 2;
    a.lowmask = ((uint64_t)1 << h) - 1;
    a.items = (uint64_t)1 << (n - 2);
  }
  // coefficients of the item values: mode 0 (|c_i|^2, |c_{i+1}|^2) with the
  // sign of z_t bit 0 on the second; modes 1, 2: Re w for an even |f & z_t|,
  // Im w for an odd one, and in mode 2 the pair at i + 1 again signed by bit 0
  constexpr uint32_t kOne = 0x3FF00000u, kNeg = 0x80000000u;
  for (int t = 0; t < nt; ++t) {
    const uint32_t zeta = (z[t] & 1) ? kNeg : 0u;
    const bool im = (a.odd >> t) & 1;
    if (mode == 0) {
      a.chi[t][0] = kOne;
      a.chi[t][1] = kOne | zeta;
    } else {
      a.chi[t][0] = im ? 0u : kOne;
      a.chi[t][1] = im ? kOne : 0u;
      a.chi[t][2] = a.chi[t][0] ? a.chi[t][0] | zeta : 0u;
      a.chi[t][3] = a.chi[t][1] ? a.chi[t][1] | zeta : 0u;
    }
  }
  const unsigned blocks = blocks_for(a.items, 2);  // a power of two, as the kernel's split of signs needs
  const int terms = nt <= 1 ? 1 : nt <= 2 ? 2 : nt <= 4 ? 4 : 8;
  const bool nt_loads = n >= kern::kNtMinQubits;
  using Kern = void (*)(const float4*, PauliArgs, double*);
  static constexpr Kern table[2][3][4] = {
      {{k_pauli_partial<false, 0, 1>, k_pauli_partial<false, 0, 2>, k_pauli_partial<false, 0, 4>,
        k_pauli_partial<false, 0, 8>},
       {k_pauli_partial<false, 1, 1>, k_pauli_partial<false, 1, 2>, k_pauli_partial<false, 1, 4>,
        k_pauli_partial<false, 1, 8>},
       {k_pauli_partial<false, 2, 1>, k_pauli_partial<false, 2, 2>, k_pauli_partial<false, 2, 4>,
        k_pauli_partial<false, 2, 8>}},
      {{k_pauli_partial<true, 0, 1>, k_pauli_partial<true, 0, 2>, k_pauli_partial<true, 0, 4>,
        k_pauli_partial<true, 0, 8>},
       {k_pauli_partial<true, 1, 1>, k_pauli_partial<true, 1, 2>, k_pauli_partial<true, 1, 4>,
        k_pauli_partial<true, 1, 8>},
       {k_pauli_partial<true, 2, 1>, k_pauli_partial<true, 2, 2>, k_pauli_partial<true, 2, 4>,
        k_pauli_partial<true, 2, 8>}}};
  const int ti = terms == 1 ? 0 : terms == 2 ? 1 : terms == 4 ? 2 : 3;
  unsigned used = blocks;
  const uint64_t chunk_waves = (uint64_t)kMaxBlocks * (kThreads / 64);
  if (nt_loads && a.items % (chunk_waves * kChunkItems) == 0) {
    static constexpr Kern chunks[3][4] = {
        {k_pauli_chunks<0, 1>, k_pauli_chunks<0, 2>, k_pauli_chunks<0, 4>, k_pauli_chunks<0, 8>},
        {k_pauli_chunks<1, 1>, k_pauli_chunks<1, 2>, k_pauli_chunks<1, 4>, k_pauli_chunks<1, 8>},
        {k_pauli_chunks<2, 1>, k_pauli_chunks<2, 2>, k_pauli_chunks<2, 4>, k_pauli_chunks<2, 8>}};
    used = kMaxBlocks;
    hipLaunchKernelGGL(chunks[mode][ti], dim3(used), dim3(kThreads), 0, st, (const float4*)psi, a, scratch);
  } else {
    hipLaunchKernelGGL(table[nt_loads][mode][ti], dim3(blocks), dim3(kThreads), 0, st, (const float4*)psi, a,
                       scratch);
  }
  hipLaunchKernelGGL(k_column_sums<true>, dim3(1), dim3(64 * kFinalWaves), 0, st, (const double*)scratch,
                     (int)used, kTerms, mode, a.odd, out);
  SV_HIP(hipGetLastError());
}

int marginal_max_qubits() { return kMaxMeasured; }
size_t marginal_scratch_bytes(int m) { return sizeof(double) * (size_t)kMaxBlocks << m; }

void launch_marginal(const void* psi, int n, int m, const int* qubits, double* scratch, double* out,
                     hipStream_t st) {
  if (m < 1 || m > kMaxMeasured || m > n) throw DeviceError{hipErrorInvalidValue, "k_marginal: bad m"};
  MargArgs a{};
  a.len = (uint64_t)1 << n;
  const int cbits = n > 6 ? n - 6 : 0;
  a.nchunks = (uint64_t)1 << cbits;
  a.m = m;
  for (int j = 0; j < m; ++j) {
    if (qubits[j] < 0 || qubits[j] >= n) throw DeviceError{hipErrorInvalidValue, "k_marginal: qubit past n"};
    a.q[j] = qubits[j];
    if (qubits[j] < 6) a.low_meas |= 1u << qubits[j];
    else a.hc |= (uint64_t)1 << (qubits[j] - 6);
  }
  a.fc = (a.nchunks - 1) & ~a.hc;
  a.free_bits = __builtin_popcountll(a.fc);
  const unsigned blocks = blocks_for(a.nchunks * 64, 16);
  const int M = 1 << m;
  if (n >= kern::kNtMinQubits)
    hipLaunchKernelGGL(k_marginal_partial<true>, dim3(blocks), dim3(kThreads), sizeof(double) * 4 * M, st,
                       (const float2*)psi, a, scratch);
  else
    hipLaunchKernelGGL(k_marginal_partial<false>, dim3(blocks), dim3(kThreads), sizeof(double) * 4 * M, st,
                       (const float2*)psi, a, scratch);
  hipLaunchKernelGGL(k_column_sums<false>, dim3((M + 63) / 64), dim3(64 * kFinalWaves), 0, st,
                     (const double*)scratch, (int)blocks, M, 0, 0u, out);
  SV_HIP(hipGetLastError());
}

// Chunk size 2^c: 4096 amplitudes, or larger so that at most 2^22 chunks
// (2048 scan blocks) exist.
int sample_chunk_bits(int n) {
  int c = n < 12 ? n : 12;
  if (n - c > 22) c = n - 22;
  return c;
}
size_t sample_scratch_bytes(int n) {
  const uint64_t nchunks = (uint64_t)1 << (n - sample_chunk_bits(n));
  return sizeof(double) * (nchunks + kMaxBlocks);
}

// prepare: build the chunk prefix sums in scratch (needed once per state);
// then draw `shots` samples.  uniforms / out: device arrays of `shots`; out
// gets all ones for a zero state.
void launch_sample(const void* psi, int n, bool prepare, const double* uniforms, uint64_t shots, uint64_t* out,
                   double* scratch, hipStream_t st) {
  const int c = sample_chunk_bits(n);
  if (c < 1) throw DeviceError{hipErrorInvalidValue, "k_sample: a chunk must hold whole 16-byte elements"};
  const uint64_t nchunks = (uint64_t)1 << (n - c);
  double* incl = scratch;
  double* totals = scratch + nchunks;
  if (prepare) {
    const uint64_t waves_blocks = (nchunks * 64 + kThreads - 1) / kThreads;
    if (n >= kern::kNtMinQubits)
      hipLaunchKernelGGL(k_chunk_sums<true>, dim3((unsigned)waves_blocks), dim3(kThreads), 0, st,
                         (const float2*)psi, c, nchunks, incl);
    else
      hipLaunchKernelGGL(k_chunk_sums<false>, dim3((unsigned)waves_blocks), dim3(kThreads), 0, st,
                         (const float2*)psi, c, nchunks, incl);
    const uint64_t sblocks = (nchunks + kScanBlock - 1) / kScanBlock;
    if (sblocks > (uint64_t)kScanBlock) throw DeviceError{hipErrorInvalidValue, "k_sample: too many chunks"};
    hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)sblocks), dim3(kThreads), 0, st, incl, nchunks, totals);
    if (sblocks > 1) {
      hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kThreads), 0, st, totals, sblocks, (double*)nullptr);
      hipLaunchKernelGGL(k_scan_add, dim3((unsigned)sblocks), dim3(kThreads), 0, st, incl, nchunks,
                         (const double*)totals);
    }
  }
  if (shots) {
    const uint64_t blocks = (shots * 64 + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(k_sample, dim3((unsigned)blocks), dim3(kThreads), 0, st, (const float2*)psi, c,
                       (const double*)incl, nchunks, uniforms, shots, out);
  }
  SV_HIP(hipGetLastError());
}

}  // namespace sv
