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

__device__ __forceinline__ double parity_sign(uint64_t x) { return (__popcll(x) & 1) ? -1.0 : 1.0; }

// ------------------------------------------------------------ Pauli strings
// Up to kTerms strings that share the flip mask f = X|Y part.  For P = i^ny
// X^f Z^z: <psi|P|psi> = i^ny sum_i (-1)^{|(i^f) & z|} conj(c_i) c_{i^f}.
// With f != 0 the sum runs over pairs (i, j = i^f) with bit h (the highest
// bit of f) clear in i; the pair contributes s_i w + s_j conj(w), w =
// conj(c_i) c_j, s_j = (-1)^{|i & z|} and s_i = s_j (-1)^{|f & z|}.  So a
// term with |f & z| even collects 2 s_j Re w (a real sum) and one with
// |f & z| odd collects -2i s_j Im w; each term needs one parity per pair.
// Each amplitude is read once.
constexpr int kTerms = 8;
struct PauliArgs {
  uint64_t f;
  uint64_t items;          // float4 elements (f == 0 or f == 1) or element quads
  uint64_t lowmask;        // ones below bit h
  uint64_t z[kTerms];
  uint32_t odd;            // bit t: |f & z_t| is odd
  int nt;
  int mode;                // 0: diagonal (f == 0); 1: f == 1; 2: h >= 1
};

__device__ __forceinline__ double signed_by(uint64_t x, double v) { return (__popcll(x) & 1) ? -v : v; }

// Amplitudes i (even) and i + 1 of one element: their signs differ exactly
// when z has bit 0 set.
__device__ __forceinline__ void diag_add(double* acc, const PauliArgs& a, uint64_t i, const float4 v) {
  const double p0 = sq(make_float2(v.x, v.y)), p1 = sq(make_float2(v.z, v.w));
  const double same = p0 + p1, diff = p0 - p1;
#pragma unroll
  for (int t = 0; t < kTerms; ++t)
    if (t < a.nt) acc[t] += signed_by(i & a.z[t], (a.z[t] & 1) ? diff : same);
}

// Pair (i, i ^ f), i with bit h clear.
__device__ __forceinline__ void pair_add(double* acc, const PauliArgs& a, uint64_t i, const float2 ci,
                                         const float2 cj) {
  const double wr = (double)ci.x * cj.x + (double)ci.y * cj.y;
  const double wi = (double)ci.x * cj.y - (double)ci.y * cj.x;
#pragma unroll
  for (int t = 0; t < kTerms; ++t)
    if (t < a.nt) acc[t] += signed_by(i & a.z[t], ((a.odd >> t) & 1) ? wi : wr);
}

// Block b owns a contiguous slice of items; every thread keeps two items in
// flight.  Mode 0 and 1 items are float4 elements (amplitudes 2e, 2e + 1);
// mode 2 items are quads: the element at i (bit h clear, i even) and the
// element holding its partners i ^ f and (i + 1) ^ f.
template <bool NT>
__global__ __launch_bounds__(kThreads) void k_pauli_partial(const float4* __restrict__ psi, const PauliArgs a,
                                                           double* __restrict__ partials) {
  double acc[kTerms];
#pragma unroll
  for (int t = 0; t < kTerms; ++t) acc[t] = 0.0;
  const uint64_t per = (a.items + gridDim.x - 1) / gridDim.x;
  const uint64_t lo = (uint64_t)blockIdx.x * per;
  const uint64_t hi = lo + per < a.items ? lo + per : a.items;
  for (uint64_t x0 = lo + threadIdx.x; x0 < hi; x0 += 2 * kThreads) {
    const uint64_t x1 = x0 + kThreads;
    const bool has1 = x1 < hi;
    if (a.mode == 0) {
      const float4 v0 = gld<NT>(psi + x0);
      const float4 v1 = has1 ? gld<NT>(psi + x1) : make_float4(0.f, 0.f, 0.f, 0.f);
      diag_add(acc, a, 2 * x0, v0);
      if (has1) diag_add(acc, a, 2 * x1, v1);
    } else if (a.mode == 1) {
      const float4 v0 = gld<NT>(psi + x0);
      const float4 v1 = has1 ? gld<NT>(psi + x1) : make_float4(0.f, 0.f, 0.f, 0.f);
      pair_add(acc, a, 2 * x0, make_float2(v0.x, v0.y), make_float2(v0.z, v0.w));
      if (has1) pair_add(acc, a, 2 * x1, make_float2(v1.x, v1.y), make_float2(v1.z, v1.w));
    } else {
      const uint64_t g0 = 2 * x0, g1 = 2 * x1;
      const uint64_t i0 = ((g0 & ~a.lowmask) << 1) | (g0 & a.lowmask);
      const uint64_t i1 = ((g1 & ~a.lowmask) << 1) | (g1 & a.lowmask);
      const uint64_t j0 = (i0 ^ a.f) & ~(uint64_t)1, j1 = (i1 ^ a.f) & ~(uint64_t)1;
      const float4 A0 = gld<NT>(psi + (i0 >> 1)), B0 = gld<NT>(psi + (j0 >> 1));
      float4 A1 = make_float4(0.f, 0.f, 0.f, 0.f), B1 = A1;
      if (has1) {
        A1 = gld<NT>(psi + (i1 >> 1));
        B1 = gld<NT>(psi + (j1 >> 1));
      }
      const bool odd = a.f & 1;  // the partner of i is the odd amplitude of its element
      pair_add(acc, a, i0, make_float2(A0.x, A0.y), odd ? make_float2(B0.z, B0.w) : make_float2(B0.x, B0.y));
      pair_add(acc, a, i0 + 1, make_float2(A0.z, A0.w), odd ? make_float2(B0.x, B0.y) : make_float2(B0.z, B0.w));
      if (has1) {
        pair_add(acc, a, i1, make_float2(A1.x, A1.y), odd ? make_float2(B1.z, B1.w) : make_float2(B1.x, B1.y));
        pair_add(acc, a, i1 + 1, make_float2(A1.z, A1.w),
                 odd ? make_float2(B1.x, B1.y) : make_float2(B1.z, B1.w));
      }
    }
  }
  __shared__ double part[kThreads / 64][kTerms];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int t = 0; t < kTerms; ++t) {
    const double r = wave_sum(acc[t]);
    if (lane == 0) part[w][t] = r;
  }
  __syncthreads();
  if (threadIdx.x < kTerms) {
    double v = 0.0;
    for (int x = 0; x < kThreads / 64; ++x) v += part[x][threadIdx.x];
    partials[(size_t)blockIdx.x * kTerms + threadIdx.x] = v;
  }
}

// Sum the per-block partials in block order and form S_t = sum_i
// (-1)^{|(i^f) & z_t|} conj(c_i) c_{i^f}: out[2t], out[2t+1] = Re, Im (the
// i^ny factor is applied on the host).
__global__ __launch_bounds__(64) void k_pauli_final(const double* __restrict__ partials, int blocks, int mode,
                                                   uint32_t odd, double* __restrict__ out) {
  const int t = threadIdx.x;
  if (t >= kTerms) return;
  double s = 0.0;
  for (int b = 0; b < blocks; ++b) s += partials[(size_t)b * kTerms + t];
  const double scale = mode == 0 ? 1.0 : 2.0;
  const bool is_odd = (odd >> t) & 1;
  out[2 * t] = is_odd ? 0.0 : scale * s;
  out[2 * t + 1] = is_odd ? -scale * s : 0.0;
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

__global__ __launch_bounds__(kThreads) void k_marginal_final(const double* __restrict__ partials, int blocks, int M,
                                                            double* __restrict__ out) {
  const int o = blockIdx.x * kThreads + threadIdx.x;
  if (o >= M) return;
  double s = 0.0;
  for (int b = 0; b < blocks; ++b) s += partials[(size_t)b * M + o];
  out[o] = s;
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
  const uint64_t len = (uint64_t)1 << cbits;
  const float2* __restrict__ p = psi + (ch << cbits);
  double v = 0.0;
  for (uint64_t i = lane; i < len; i += 64) v += sq(gld<NT>(p + i));
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
  a.nt = nt;
  for (int t = 0; t < nt; ++t) {
    a.z[t] = z[t];
    if (__builtin_popcountll(f & z[t]) & 1) a.odd |= 1u << t;
  }
  if (n < 1 || (n < 64 && (f >> n) != 0)) throw DeviceError{hipErrorInvalidValue, "k_pauli: flip mask past n"};
  if (f == 0 || f == 1) {
    a.mode = (int)f;
    a.items = (uint64_t)1 << (n - 1);  // n = 1: one element
  } else {
    const int h = 63 - __builtin_clzll(f);  // h >= 1, so n >= 2
    a.mode = 2;
    a.lowmask = ((uint64_t)1 << h) - 1;
    a.items = (uint64_t)1 << (n - 2);
  }
  const unsigned blocks = blocks_for(a.items, 2);
  if (n >= kern::kNtMinQubits)
    hipLaunchKernelGGL(k_pauli_partial<true>, dim3(blocks), dim3(kThreads), 0, st, (const float4*)psi, a, scratch);
  else
    hipLaunchKernelGGL(k_pauli_partial<false>, dim3(blocks), dim3(kThreads), 0, st, (const float4*)psi, a, scratch);
  hipLaunchKernelGGL(k_pauli_final, dim3(1), dim3(64), 0, st, (const double*)scratch, (int)blocks, a.mode, a.odd,
                     out);
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
  hipLaunchKernelGGL(k_marginal_final, dim3((M + kThreads - 1) / kThreads), dim3(kThreads), 0, st,
                     (const double*)scratch, (int)blocks, M, out);
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
