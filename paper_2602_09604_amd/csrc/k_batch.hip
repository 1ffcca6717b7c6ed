// Batched simulation of many independent small circuits.
//
// Two kernels, both launched inside one captured hipGraph:
//   k_batch_lds    one workgroup per circuit whose state fits in LDS: load the
//                  state once, apply every fused pass of the circuit from LDS,
//                  store once.  HBM traffic is one read and one write per
//                  circuit instead of one per pass.
//   k_batch_level  every larger circuit advances one fused pass per launch;
//                  a launch covers pass L of all circuits that have one, each
//                  workgroup owning 256 lane work items of one circuit, so the
//                  grid is filled by the whole batch instead of by one state.
//                  The kernel boundary is the barrier between dependent passes
//                  of a circuit (it also makes every XCD's writes visible to
//                  the next pass without spinning on device flags).  A level
//                  is one launch per pass shape; k_batch_level_x is the
//                  lane-exchange form for targets on amplitude bits 1..3.
// The LDS branch runs on a forked capture stream, so it overlaps the level
// launches of the large circuits.  The LDS-resident size limit is chosen by
// the autotuner (up to 14 qubits, 128 KiB, where the device allows it).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <exception>
#include <thread>
#include <cstring>
#include <mutex>

#include <stdexcept>

#include "k_common.h"

namespace sv {

void* state_psi(sv_state* s);
int state_n(sv_state* s);
hipStream_t state_stream(sv_state* s);
bool state_poisoned(sv_state* s);
void state_poison(sv_state* s);
void state_note_gates(sv_state* s, const sv_gate* g, size_t n);

namespace {
using namespace kern;

// One fused pass of one circuit, in element space (see k_apply_reg modes).
struct BPass {
  uint64_t items;             // lane work items
  uint64_t lowmask[SV_MAX_K];
  uint64_t stride[SV_MAX_K];
  uint32_t mat;               // float2 index of the complex64 matrix
  int mode, K;
  int tm;                     // element bits 0..2 among the targets (lane exchange), 0: none
};

struct BCirc {
  float2* psi;
  int n;
  int pass0, npass;
};

// Element access of apply_item: plain for LDS and for cached global
// memory, non-temporal (streaming) for the level sweeps, which touch every
// active circuit's state once per level (gigabytes, far over the last-level
// cache): measured 49.6 against 52.7 ms for the 512-circuit batch.
template <bool NT, typename PTR>
__device__ __forceinline__ auto load_at(PTR p, uint64_t i) {
  if constexpr (NT) return gld<true>(p + i);
  else return p[i];
}
template <bool NT, typename PTR, typename T>
__device__ __forceinline__ void store_at(PTR p, uint64_t i, const T& v) {
  if constexpr (NT) gst<true>(p + i, v);
  else p[i] = v;
}

template <int K, int MODE, bool NT = false, typename PTR2, typename PTR4>
__device__ __forceinline__ void apply_item(PTR2 psi2, PTR4 psi4, const float2* __restrict__ U, const BPass& p,
                                           uint64_t g) {
  constexpr int D = 1 << K;
  uint64_t base = g;
#pragma unroll
  for (int j = 0; j < K; ++j) base = ((base & ~p.lowmask[j]) << 1) | (base & p.lowmask[j]);
  if constexpr (MODE == 2) {
    float2 v[D];
#pragma unroll
    for (int l = 0; l < D; ++l) v[l] = load_at<NT>(psi2, base + local_offset<K, uint64_t>(l, p.stride));
#pragma unroll
    for (int r = 0; r < D; ++r) {
      float2 acc = make_float2(0.f, 0.f);
#pragma unroll
      for (int c = 0; c < D; ++c) cmac(acc, U[r * D + c], v[c]);
      store_at<NT>(psi2, base + local_offset<K, uint64_t>(r, p.stride), acc);
    }
  } else {
    float4 v[D];
#pragma unroll
    for (int l = 0; l < D; ++l) v[l] = load_at<NT>(psi4, base + local_offset<K, uint64_t>(l, p.stride));
#pragma unroll
    for (int r = 0; r < D; ++r)
      store_at<NT>(psi4, base + local_offset<K, uint64_t>(r, p.stride), pair_row<K, MODE>(v, U, r));
  }
}

// Dispatch on the pass shape (uniform across the workgroup).
template <typename PTR2, typename PTR4>
__device__ void apply_dispatch(PTR2 psi2, PTR4 psi4, const float2* __restrict__ U, const BPass& p, uint64_t g) {
  switch (p.mode * 8 + p.K) {
    case 0 * 8 + 1: apply_item<1, 0>(psi2, psi4, U, p, g); break;
    case 0 * 8 + 2: apply_item<2, 0>(psi2, psi4, U, p, g); break;
    case 0 * 8 + 3: apply_item<3, 0>(psi2, psi4, U, p, g); break;
    case 0 * 8 + 4: apply_item<4, 0>(psi2, psi4, U, p, g); break;
    case 0 * 8 + 5: apply_item<5, 0>(psi2, psi4, U, p, g); break;
    case 1 * 8 + 0: apply_item<0, 1>(psi2, psi4, U, p, g); break;
    case 1 * 8 + 1: apply_item<1, 1>(psi2, psi4, U, p, g); break;
    case 1 * 8 + 2: apply_item<2, 1>(psi2, psi4, U, p, g); break;
    case 1 * 8 + 3: apply_item<3, 1>(psi2, psi4, U, p, g); break;
    case 1 * 8 + 4: apply_item<4, 1>(psi2, psi4, U, p, g); break;
    case 1 * 8 + 5: apply_item<5, 1>(psi2, psi4, U, p, g); break;
    case 2 * 8 + 6: apply_item<6, 2>(psi2, psi4, U, p, g); break;
    default: break;  // shapes are checked on the host
  }
}

// One workgroup per LDS-resident circuit (state of 2^n <= 2^14 amplitudes).
__global__ __launch_bounds__(256) void k_batch_lds(const BCirc* __restrict__ circs, const int* __restrict__ which,
                                                   const BPass* __restrict__ passes, const float2* __restrict__ mats) {
  extern __shared__ float4 st4[];
  float2* st2 = reinterpret_cast<float2*>(st4);
  const BCirc c = circs[which[blockIdx.x]];
  const int pairs = 1 << (c.n - 1);
  float4* g4 = reinterpret_cast<float4*>(c.psi);
  for (int i = threadIdx.x; i < pairs; i += 256) st4[i] = g4[i];
  __syncthreads();
  for (int pi = 0; pi < c.npass; ++pi) {
    const BPass p = passes[c.pass0 + pi];
    for (uint64_t g = threadIdx.x; g < p.items; g += 256) apply_dispatch(st2, st4, mats + p.mat, p, g);
    __syncthreads();
  }
  for (int i = threadIdx.x; i < pairs; i += 256) g4[i] = st4[i];
}

// Pass `level` of every circuit in `active` (count entries), all of one
// shape <K, MODE>; first_block is the prefix sum of workgroups per active
// circuit (count + 1 entries).  One instantiation per shape keeps each
// launch free of the shape dispatch (a call with a stack frame, and the
// register budget of the largest shape).
template <int K, int MODE>
__global__ __launch_bounds__(256) void k_batch_level(const BCirc* __restrict__ circs, const int* __restrict__ active,
                                                     const uint64_t* __restrict__ first_block, int count, int level,
                                                     const BPass* __restrict__ passes,
                                                     const float2* __restrict__ mats) {
  const uint64_t b = blockIdx.x;
  int lo = 0, hi = count - 1;  // last entry with first_block <= b
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first_block[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  const BCirc c = circs[active[lo]];
  const BPass p = passes[c.pass0 + level];
  const uint64_t g = (b - first_block[lo]) * 256 + threadIdx.x;
  if (g >= p.items) return;
  apply_item<K, MODE, true>(c.psi, reinterpret_cast<float4*>(c.psi), mats + p.mat, p, g);
}

// The same with targets on element bits 0..2 (set TM): the lane exchange of
// k_common.h, so that every load and store instruction covers whole lines.
// A wave's 64 work items belong to one circuit (items are a multiple of 64).
template <int K, int MODE, int TM>
__global__ __launch_bounds__(256) void k_batch_level_x(const BCirc* __restrict__ circs, const int* __restrict__ active,
                                                       const uint64_t* __restrict__ first_block, int count, int level,
                                                       const BPass* __restrict__ passes,
                                                       const float2* __restrict__ mats) {
  constexpr int D = 1 << K;
  constexpr int M = LowBits<TM>::m;
  constexpr int XM = (1 << M) - 1;
  static_assert(M <= K, "every low target is an element-space target");
  const uint64_t b = blockIdx.x;
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first_block[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  const BCirc c = circs[active[lo]];
  const BPass p = passes[c.pass0 + level];
  const uint64_t wave0 = (b - first_block[lo]) * 256 + (threadIdx.x & ~63u);
  if (wave0 >= p.items) return;
  float4* __restrict__ psi = reinterpret_cast<float4*>(c.psi);
  const float2* __restrict__ U = mats + p.mat;
  const int j = threadIdx.x & 63;
  const int uj = compress_bits<6>(j, ~TM & 63), cj = compress_bits<6>(j, TM);
  uint64_t offc = 0;
#pragma unroll
  for (int i = 0; i < M; ++i)
    if ((cj >> i) & 1) offc += p.stride[i];
  uint64_t xoff[XM + 1];
#pragma unroll
  for (int X = 0; X <= XM; ++X) xoff[X] = insert_zeros<K, uint64_t>((uint64_t)X << (6 - M), p.lowmask);
  const uint64_t b0 = insert_zeros<K, uint64_t>(wave0 + uj, p.lowmask) + offc;
  float4 v[D];
#pragma unroll
  for (int r = 0; r < D; ++r) v[r] = gld<true>(psi + b0 + xoff[r & XM] + local_offset<K, uint64_t>(r & ~XM, p.stride));
  xtranspose<TM>(v, j);
#pragma unroll
  for (int h0 = 0; h0 < D; h0 += XM + 1) {
    float4 o[XM + 1];
#pragma unroll
    for (int x = 0; x <= XM; ++x) o[x] = pair_row<K, MODE>(v, U, h0 | x);
    xtranspose<TM>(o, j);
#pragma unroll
    for (int x = 0; x <= XM; ++x) gst<true>(psi + b0 + xoff[x] + local_offset<K, uint64_t>(h0, p.stride), o[x]);
  }
}

// the pass shapes the batch supports: index mode * 8 + K
constexpr int kShapes = 8 * 24;
bool shape_supported(int mode, int K) {
  return (mode == 0 && K >= 1 && K <= 5) || (mode == 1 && K >= 0 && K <= 5) || (mode == 2 && K == 6);
}

template <int K, int MODE, int TM>
void launch_x(unsigned blocks, hipStream_t st, const BCirc* circs, const int* active, const uint64_t* first,
              int count, int level, const BPass* passes, const float2* mats) {
  if constexpr (LowBits<TM>::m <= K)
    hipLaunchKernelGGL((k_batch_level_x<K, MODE, TM>), dim3(blocks), dim3(256), 0, st, circs, active, first, count,
                       level, passes, mats);
  else
    throw DeviceError{hipErrorInvalidValue, "batch: low targets"};
}

template <int K, int MODE>
void launch_xk(int tm, unsigned blocks, hipStream_t st, const BCirc* circs, const int* active, const uint64_t* first,
               int count, int level, const BPass* passes, const float2* mats) {
  switch (tm) {
    case 1: return launch_x<K, MODE, 1>(blocks, st, circs, active, first, count, level, passes, mats);
    case 2: return launch_x<K, MODE, 2>(blocks, st, circs, active, first, count, level, passes, mats);
    case 3: return launch_x<K, MODE, 3>(blocks, st, circs, active, first, count, level, passes, mats);
    case 4: return launch_x<K, MODE, 4>(blocks, st, circs, active, first, count, level, passes, mats);
    case 5: return launch_x<K, MODE, 5>(blocks, st, circs, active, first, count, level, passes, mats);
    case 6: return launch_x<K, MODE, 6>(blocks, st, circs, active, first, count, level, passes, mats);
    case 7: return launch_x<K, MODE, 7>(blocks, st, circs, active, first, count, level, passes, mats);
    default: throw DeviceError{hipErrorInvalidValue, "batch: low targets"};
  }
}

void launch_level(int shape, unsigned blocks, hipStream_t st, const BCirc* circs, const int* active,
                  const uint64_t* first, int count, int level, const BPass* passes, const float2* mats) {
  const int tm = shape / 24, sh = shape % 24;
  if (tm) {
    switch (sh) {
      case 0 * 8 + 1: launch_xk<1, 0>(tm, blocks, st, circs, active, first, count, level, passes, mats); break;
      case 0 * 8 + 2: launch_xk<2, 0>(tm, blocks, st, circs, active, first, count, level, passes, mats); break;
      case 0 * 8 + 3: launch_xk<3, 0>(tm, blocks, st, circs, active, first, count, level, passes, mats); break;
      case 0 * 8 + 4: launch_xk<4, 0>(tm, blocks, st, circs, active, first, count, level, passes, mats); break;
      case 1 * 8 + 1: launch_xk<1, 1>(tm, blocks, st, circs, active, first, count, level, passes, mats); break;
      case 1 * 8 + 2: launch_xk<2, 1>(tm, blocks, st, circs, active, first, count, level, passes, mats); break;
      case 1 * 8 + 3: launch_xk<3, 1>(tm, blocks, st, circs, active, first, count, level, passes, mats); break;
      default: throw DeviceError{hipErrorInvalidValue, "batch: unsupported exchange shape"};
    }
    SV_HIP(hipGetLastError());
    return;
  }
  shape = sh;
#define SV_LEVEL(K_, M_)                                                                                     \
  case M_ * 8 + K_:                                                                                          \
    hipLaunchKernelGGL((k_batch_level<K_, M_>), dim3(blocks), dim3(256), 0, st, circs, active, first, count, \
                       level, passes, mats);                                                                  \
    break;
  switch (shape) {
    SV_LEVEL(1, 0) SV_LEVEL(2, 0) SV_LEVEL(3, 0) SV_LEVEL(4, 0) SV_LEVEL(5, 0)
    SV_LEVEL(0, 1) SV_LEVEL(1, 1) SV_LEVEL(2, 1) SV_LEVEL(3, 1) SV_LEVEL(4, 1) SV_LEVEL(5, 1)
    SV_LEVEL(6, 2)
    default: throw DeviceError{hipErrorInvalidValue, "batch: unsupported pass shape"};
  }
#undef SV_LEVEL
  SV_HIP(hipGetLastError());
}

std::mutex g_batch_mu;
int g_lds_max_n = 12;  // largest LDS-resident state (qubits); set by the autotuner
constexpr int kBatchLdsMaxQubits = 14;
constexpr int kBatchExchangeMinQubits = 18;

void fill_pass(BPass& bp, int n, const FusedGate& f, uint32_t mat) {
  int pos[SV_MAX_K];
  if (f.q[0] == 0) {
    bp.mode = 1;
    bp.K = f.k - 1;
    for (int j = 0; j < bp.K; ++j) pos[j] = f.q[j + 1] - 1;
    bp.items = (uint64_t)1 << (n - 1 - bp.K);
  } else if (f.k <= 5) {
    bp.mode = 0;
    bp.K = f.k;
    for (int j = 0; j < bp.K; ++j) pos[j] = f.q[j] - 1;
    bp.items = (uint64_t)1 << (n - 1 - bp.K);
  } else {
    bp.mode = 2;
    bp.K = f.k;
    for (int j = 0; j < bp.K; ++j) pos[j] = f.q[j];
    bp.items = (uint64_t)1 << (n - bp.K);
  }
  for (int j = 0; j < SV_MAX_K; ++j) {
    bp.lowmask[j] = j < bp.K ? ((uint64_t)1 << pos[j]) - 1 : 0;
    bp.stride[j] = j < bp.K ? (uint64_t)1 << pos[j] : 0;
  }
  bp.mat = mat;
  // Passes with targets on element bits 0..2 of circuits of at least
  // kBatchExchangeMinQubits qubits take the lane-exchange level kernel; on
  // smaller states the extra launch per level costs more than the partial
  // lines (the L2 completes them).
  bp.tm = 0;
  if (n >= kBatchExchangeMinQubits && ((bp.mode == 0 && bp.K <= 4) || (bp.mode == 1 && bp.K >= 1 && bp.K <= 3)) &&
      bp.items % 64 == 0)
    for (int j = 0; j < bp.K; ++j)
      if (pos[j] <= 2) bp.tm |= 1 << pos[j];
}

}  // namespace

int batch_lds_max_n() {
  std::lock_guard<std::mutex> lk(g_batch_mu);
  return g_lds_max_n;
}
void set_batch_lds_max_n(int n) {
  std::lock_guard<std::mutex> lk(g_batch_mu);
  g_lds_max_n = std::max(1, std::min(kBatchLdsMaxQubits, n));
}

// Largest LDS-resident state the current device allows: 8 * 2^n bytes of
// dynamic LDS per workgroup (gfx950 has 160 KiB per CU), at most 14 qubits.
int batch_lds_cap() {
  int dev = 0, bytes = 0;
  SV_HIP(hipGetDevice(&dev));
  SV_HIP(hipDeviceGetAttribute(&bytes, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  int n = 1;
  while (n < kBatchLdsMaxQubits && ((size_t)8 << (n + 1)) <= (size_t)bytes) ++n;
  return n;
}

int plan_fusion(const sv_gate* g, size_t n, int n_qubits, const sv_run_opts& o, std::vector<FusedGate>& fused,
                std::vector<int32_t>& block_of, int max_ctrl);

// Batched run on explicit buffers; lds_max_n < 0 uses the tuned limit.
void batch_run_impl(void* const* psis, const int* ns, const sv_gate* const* circuits, const size_t* n_gates,
                    size_t n_circ, const sv_run_opts& o, hipStream_t st, int lds_max_n, double* gpu_s,
                    uint64_t* passes_out, double* fuse_s, uint64_t* bytes_out, uint64_t* launches_out) {
  const int lds_n = std::min(lds_max_n < 0 ? batch_lds_max_n() : lds_max_n, batch_lds_cap());
  const auto t0 = std::chrono::steady_clock::now();
  std::vector<BCirc> circs(n_circ);
  std::vector<BPass> passes;
  std::vector<float> mats;  // complex64, interleaved
  int max_levels = 0;
  // Fusion of independent circuits on host threads (each circuit's plan is
  // computed by one thread; the assembly below stays in circuit order).
  std::vector<std::vector<FusedGate>> plans(n_circ);
  {
    const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    const unsigned nt = (unsigned)std::min<size_t>(hw, std::max<size_t>(1, n_circ / 8));
    std::atomic<size_t> next{0};
    std::vector<std::exception_ptr> errs(nt);
    auto worker = [&](unsigned w) {
      set_host_pool_worker(true);
      struct Reset {
        ~Reset() { set_host_pool_worker(false); }
      } reset;
      try {
        for (size_t c = next++; c < n_circ; c = next++) {
          std::vector<int32_t> block_of;
          plan_fusion(circuits[c], n_gates[c], ns[c], o, plans[c], block_of, 0);  // batched passes take no controls
        }
      } catch (...) {
        errs[w] = std::current_exception();
        next = n_circ;
      }
    };
    std::vector<std::thread> pool;
    for (unsigned w = 1; w < nt; ++w) pool.emplace_back(worker, w);
    worker(0);
    for (auto& t : pool) t.join();
    for (auto& e : errs)
      if (e) std::rethrow_exception(e);
  }
  for (size_t c = 0; c < n_circ; ++c) {
    const std::vector<FusedGate>& fused = plans[c];
    circs[c].psi = (float2*)psis[c];
    circs[c].n = ns[c];
    circs[c].pass0 = (int)passes.size();
    circs[c].npass = (int)fused.size();
    for (auto& f : fused) {
      if (f.cmask)
        throw std::invalid_argument("sv_batch_run: a controlled gate wider than max_k qubits (targets plus "
                                    "controls) cannot run in the batched kernel");
      BPass bp{};
      fill_pass(bp, ns[c], f, (uint32_t)(mats.size() / 2));
      passes.push_back(bp);
      for (double v : f.mat) mats.push_back((float)v);
    }
    if (ns[c] > lds_n) max_levels = std::max(max_levels, (int)fused.size());
  }
  if (fuse_s) *fuse_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  // LDS-resident circuits and, per level, the active large circuits
  std::vector<int> small;
  for (size_t c = 0; c < n_circ; ++c)
    if (ns[c] <= lds_n && circs[c].npass > 0) small.push_back((int)c);
  int small_n = 1;
  for (int c : small) small_n = std::max(small_n, ns[c]);
  // per level, one launch per pass shape present: the active large circuits
  // whose pass at that level has the shape, with their workgroup prefix sums
  struct Launch {
    int level, shape;
    std::vector<int> active;
    std::vector<uint64_t> first;
  };
  std::vector<Launch> launch_list;
  size_t level_ints = 0, level_u64 = 0;
  for (int L = 0; L < max_levels; ++L) {
    std::vector<int> slot(kShapes, -1);
    for (size_t c = 0; c < n_circ; ++c) {
      if (ns[c] <= lds_n || circs[c].npass <= L) continue;
      const BPass& bp = passes[circs[c].pass0 + L];
      if (!shape_supported(bp.mode, bp.K)) throw std::invalid_argument("sv_batch_run: unsupported pass shape");
      const int sh = bp.tm * 24 + bp.mode * 8 + bp.K;
      if (slot[sh] < 0) {
        slot[sh] = (int)launch_list.size();
        launch_list.push_back(Launch{L, sh, {}, {}});
      }
      Launch& l = launch_list[slot[sh]];
      const uint64_t acc = l.first.empty() ? 0 : l.first.back();
      if (l.first.empty()) l.first.push_back(0);
      l.active.push_back((int)c);
      l.first.push_back(acc + (bp.items + 255) / 256);
    }
  }
  for (auto& l : launch_list) {
    level_ints += l.active.size();
    level_u64 += l.first.size();
  }
  // one device buffer: circuits | passes | first-block prefixes | ints | matrices
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t off_circ = 0;
  const size_t off_pass = al(off_circ + sizeof(BCirc) * n_circ);
  const size_t off_first = al(off_pass + sizeof(BPass) * passes.size());
  const size_t off_int = al(off_first + sizeof(uint64_t) * level_u64);
  const size_t off_mat = al(off_int + sizeof(int) * (level_ints + small.size()));
  const size_t total = al(off_mat + sizeof(float) * mats.size());
  std::vector<unsigned char> host(total, 0);
  std::memcpy(host.data() + off_circ, circs.data(), sizeof(BCirc) * n_circ);
  std::memcpy(host.data() + off_pass, passes.data(), sizeof(BPass) * passes.size());
  std::vector<size_t> lvl_first_off(launch_list.size()), lvl_int_off(launch_list.size());
  size_t fu = 0, iu = 0;
  for (size_t i = 0; i < launch_list.size(); ++i) {
    const Launch& l = launch_list[i];
    lvl_first_off[i] = off_first + sizeof(uint64_t) * fu;
    std::memcpy(host.data() + lvl_first_off[i], l.first.data(), sizeof(uint64_t) * l.first.size());
    fu += l.first.size();
    lvl_int_off[i] = off_int + sizeof(int) * iu;
    std::memcpy(host.data() + lvl_int_off[i], l.active.data(), sizeof(int) * l.active.size());
    iu += l.active.size();
  }
  const size_t small_off = off_int + sizeof(int) * iu;
  std::memcpy(host.data() + small_off, small.data(), sizeof(int) * small.size());
  std::memcpy(host.data() + off_mat, mats.data(), sizeof(float) * mats.size());

  unsigned char* dev = nullptr;
  unsigned char* pinned = nullptr;
  hipStream_t side = nullptr, own = nullptr;
  hipEvent_t fork = nullptr, join = nullptr, e0 = nullptr, e1 = nullptr;
  hipGraphExec_t exec = nullptr;
  auto cleanup = [&]() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (side) (void)hipStreamDestroy(side);
    if (own) (void)hipStreamDestroy(own);
    if (fork) (void)hipEventDestroy(fork);
    if (join) (void)hipEventDestroy(join);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (dev) (void)hipFree(dev);
    if (pinned) (void)hipHostFree(pinned);
  };
  try {
    if (st == nullptr) {
      // graphs cannot be captured on the legacy default stream: drain it and
      // run this (synchronous) call on a private blocking stream instead
      SV_HIP(hipStreamSynchronize(nullptr));
      SV_HIP(hipStreamCreate(&own));
      st = own;
    }
    SV_HIP(hipMalloc(&dev, total));
    SV_HIP(hipHostMalloc(&pinned, total, hipHostMallocDefault));
    std::memcpy(pinned, host.data(), total);
    SV_HIP(hipMemcpyAsync(dev, pinned, total, hipMemcpyHostToDevice, st));
    SV_HIP(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
    SV_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    SV_HIP(hipEventCreateWithFlags(&join, hipEventDisableTiming));
    SV_HIP(hipEventCreate(&e0));
    SV_HIP(hipEventCreate(&e1));
    const BCirc* d_circ = (const BCirc*)(dev + off_circ);
    const BPass* d_pass = (const BPass*)(dev + off_pass);
    const float2* d_mat = (const float2*)(dev + off_mat);
    const bool graph = true;
    // states above 64 KiB of LDS (14 qubits) need the larger dynamic-LDS
    // limit set on the kernel before it is captured
    if (!small.empty() && ((size_t)8 << small_n) > 65536)
      SV_HIP(hipFuncSetAttribute((const void*)k_batch_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)((size_t)8 << small_n)));
    uint64_t launches = 0;
    if (graph) SV_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    try {
      hipStream_t sst = st;
      if (graph && !small.empty()) {  // fork: LDS branch on the side stream
        SV_HIP(hipEventRecord(fork, st));
        SV_HIP(hipStreamWaitEvent(side, fork, 0));
        sst = side;
      }
      if (!small.empty()) {
        ++launches;
        hipLaunchKernelGGL(k_batch_lds, dim3((unsigned)small.size()), dim3(256), (size_t)8 << small_n, sst, d_circ,
                           (const int*)(dev + small_off), d_pass, d_mat);
        SV_HIP(hipGetLastError());
      }
      for (size_t i = 0; i < launch_list.size(); ++i) {
        const Launch& l = launch_list[i];
        const uint64_t blocks = l.first.back();
        if (blocks == 0) continue;
        if (blocks >= ((uint64_t)1 << 31)) throw DeviceError{hipErrorInvalidValue, "batch level too large"};
        ++launches;
        launch_level(l.shape, (unsigned)blocks, st, d_circ, (const int*)(dev + lvl_int_off[i]),
                     (const uint64_t*)(dev + lvl_first_off[i]), (int)l.active.size(), l.level, d_pass, d_mat);
      }
      if (graph && !small.empty()) {  // join
        SV_HIP(hipEventRecord(join, side));
        SV_HIP(hipStreamWaitEvent(st, join, 0));
      }
    } catch (...) {
      if (graph) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(st, &g);
        if (g) (void)hipGraphDestroy(g);
      }
      throw;
    }
    if (graph) {
      hipGraph_t g = nullptr;
      SV_HIP(hipStreamEndCapture(st, &g));
      hipError_t e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) throw DeviceError{e, "hipGraphInstantiate"};
      SV_HIP(hipEventRecord(e0, st));
      SV_HIP(hipGraphLaunch(exec, st));
      SV_HIP(hipEventRecord(e1, st));
    }
    SV_HIP(hipStreamSynchronize(st));
    if (gpu_s) {
      float ms = 0.f;
      if (graph) SV_HIP(hipEventElapsedTime(&ms, e0, e1));
      *gpu_s = ms * 1e-3;
    }
    if (passes_out) *passes_out = passes.size();
    if (launches_out) *launches_out = launches;
    if (bytes_out) {
      uint64_t b = 0;
      for (size_t c = 0; c < n_circ; ++c)
        b += ((uint64_t)16 << ns[c]) * (ns[c] <= lds_n ? (circs[c].npass > 0 ? 1 : 0) : (uint64_t)circs[c].npass);
      *bytes_out = b;
    }
    cleanup();
  } catch (...) {
    cleanup();
    throw;
  }
}

int validate_gates(const sv_gate* g, size_t n, int n_qubits);

}  // namespace sv

using namespace sv;

extern "C" int sv_batch_run(sv_state* const* states, const sv_gate* const* circuits, const size_t* n_gates,
                            size_t n_circuits, const sv_run_opts* opts, sv_run_stats* stats) {
  if (n_circuits == 0) return SV_OK;
  if (!states || !circuits || !n_gates) return fail(SV_EINVAL, "NULL argument");
  sv_run_opts o{};
  if (opts) {
    o = *opts;
  } else {
    o.max_k = 4;
    o.fusion = SV_FUSE_GREEDY;
  }
  if (o.fusion < SV_FUSE_NONE || o.fusion > SV_FUSE_BLOCK || (o.fusion != SV_FUSE_NONE && (o.max_k < 1 || o.max_k > SV_MAX_K)))
    return fail(SV_EINVAL, "opts invalid");
  std::vector<void*> psis(n_circuits);
  std::vector<int> ns(n_circuits);
  for (size_t c = 0; c < n_circuits; ++c) {
    if (!states[c]) return fail(SV_EINVAL, "states[" + std::to_string(c) + "] is NULL");
    if (state_poisoned(states[c])) return fail(SV_ESTATE, "a handle is poisoned");
    ns[c] = state_n(states[c]);
    if (ns[c] > 30) return fail(SV_EINVAL, "batched circuits are limited to 30 qubits");
    psis[c] = state_psi(states[c]);
    if (int rc = validate_gates(circuits[c], n_gates[c], ns[c])) return rc;
  }
  // batched passes run on the VALU kernels; the precision field only selects FP32
  o.precision = SV_PREC_FP32_VALU;
  std::vector<hipEvent_t> waits;
  try {
    // work already queued on the other handles' streams (initialisation,
    // earlier passes) must finish before the batch touches their states
    const hipStream_t st0 = state_stream(states[0]);
    std::vector<hipStream_t> seen{st0};
    for (size_t c = 1; c < n_circuits; ++c) {
      const hipStream_t sc = state_stream(states[c]);
      if (std::find(seen.begin(), seen.end(), sc) != seen.end()) continue;
      seen.push_back(sc);
      hipEvent_t ev = nullptr;
      SV_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      waits.push_back(ev);
      SV_HIP(hipEventRecord(ev, sc));
      SV_HIP(hipStreamWaitEvent(st0, ev, 0));
    }
    double gpu_s = 0, fuse_s = 0;
    uint64_t np = 0, bytes = 0, launches = 0;
    batch_run_impl(psis.data(), ns.data(), circuits, n_gates, n_circuits, o, st0, -1, &gpu_s, &np, &fuse_s, &bytes,
                   &launches);
    for (hipEvent_t ev : waits) (void)hipEventDestroy(ev);
    waits.clear();
    for (size_t c = 0; c < n_circuits; ++c) state_note_gates(states[c], circuits[c], n_gates[c]);
    if (stats) {
      *stats = sv_run_stats{};
      uint64_t gi = 0;
      for (size_t c = 0; c < n_circuits; ++c) gi += n_gates[c];
      stats->gates_in = gi;
      stats->passes = np;
      stats->gpu_s = gpu_s;
      stats->fuse_s = fuse_s;
      stats->bytes = bytes;
      stats->launches = launches;
    }
    return SV_OK;
  } catch (const DeviceError& e) {
    for (hipEvent_t ev : waits) (void)hipEventDestroy(ev);
    for (size_t c = 0; c < n_circuits; ++c) state_poison(states[c]);
    return fail(SV_EDEVICE, std::string(e.what) + ": " + hipGetErrorString(e.err));
  } catch (const std::bad_alloc&) {
    for (hipEvent_t ev : waits) (void)hipEventDestroy(ev);
    return fail(SV_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    for (hipEvent_t ev : waits) (void)hipEventDestroy(ev);
    return fail(SV_EINVAL, e.what());
  } catch (...) {
    for (hipEvent_t ev : waits) (void)hipEventDestroy(ev);
    return fail(SV_EINVAL, "unknown failure");
  }
}
