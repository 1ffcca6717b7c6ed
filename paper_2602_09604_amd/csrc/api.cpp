// C ABI of libsv.so: state handles, gate application, fusion entry points,
// norm and read-back.  All device work goes to the handle's stream.
#include <atomic>
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <unordered_map>

#include "sv_internal.h"

struct sv_state {
  int n = 0;
  void* psi = nullptr;          // borrowed complex64 buffer
  hipStream_t stream = nullptr;
  int device = 0;
  bool poisoned = false;
  // matrix arena: pinned host staging + device copy, used as a ring
  unsigned char* arena_dev = nullptr;
  unsigned char* arena_host = nullptr;
  size_t arena_cap = 0;
  size_t ring_pos = 0;
  // reductions
  double* partials = nullptr;
  double* norm_dev = nullptr;
  double* norm_host = nullptr;  // pinned
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipEvent_t queued = nullptr;  // recorded after each launched chunk of passes
  // graph of the last use_graph call, with its own device copy of the pass
  // data; a later call whose passes encode to the same bytes relaunches it
  hipGraphExec_t graph_exec = nullptr;
  unsigned char* graph_dev = nullptr;
  size_t graph_cap = 0;
  std::vector<unsigned char> graph_key;
  // the call that produced the kept graph (gates, options, planning epoch)
  // and its pass figures: an identical call relaunches without fusing again
  std::vector<unsigned char> graph_input;
  uint64_t graph_passes = 0, graph_bytes = 0;
  double graph_flops = 0.0;
  bool graph_launched = false;  // the last run_passes launched the kept graph
  hipStream_t capture_stream = nullptr;  // graphs are captured here, launched on `stream`
  std::vector<hipEvent_t> pass_events;  // per-pass timing events (grown on demand)
  // state-read scratch (expectations, marginals, sampling), grown on demand
  unsigned char* meas_dev = nullptr;
  size_t meas_cap = 0;
  unsigned char* meas_host = nullptr;  // pinned
  size_t meas_host_cap = 0;
  // sum |c_i|^2 of the state as far as the host knows it once the queued
  // work has run (basis states and unitary passes keep 1; sv_norm measures
  // it); negative when unknown (after sv_write_amplitudes or a gate that is
  // not unitary).  FP16X3 passes need it bounded (see fp16x3_range_ok).
  double norm_known = 1.0;
};

namespace sv {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }
int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

static constexpr size_t kArenaInit = (size_t)4 << 20;

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static void arena_reserve(sv_state* s, size_t bytes) {
  if (bytes <= s->arena_cap) return;
  SV_HIP(hipStreamSynchronize(s->stream));
  if (s->arena_dev) SV_HIP(hipFree(s->arena_dev));
  if (s->arena_host) SV_HIP(hipHostFree(s->arena_host));
  s->arena_dev = nullptr;
  s->arena_host = nullptr;
  s->arena_cap = 0;
  size_t cap = kArenaInit;
  while (cap < bytes) cap *= 2;
  SV_HIP(hipMalloc(&s->arena_dev, cap));
  SV_HIP(hipHostMalloc(&s->arena_host, cap, hipHostMallocDefault));
  s->arena_cap = cap;
  s->ring_pos = 0;
}

// Reserve `bytes` of the ring; waits for the stream when the ring wraps so
// that pinned staging bytes still being copied are never overwritten.
static size_t arena_take(sv_state* s, size_t bytes) {
  bytes = align256(bytes);
  if (bytes > s->arena_cap) arena_reserve(s, bytes);
  if (s->ring_pos + bytes > s->arena_cap) {
    SV_HIP(hipStreamSynchronize(s->stream));
    s->ring_pos = 0;
  }
  const size_t off = s->ring_pos;
  s->ring_pos += bytes;
  return off;
}

// Device and pinned host scratch for state reads; waits for the stream
// before replacing a buffer that queued work may still use.
static void meas_reserve(sv_state* s, size_t dev_bytes, size_t host_bytes) {
  if (dev_bytes > s->meas_cap) {
    SV_HIP(hipStreamSynchronize(s->stream));
    if (s->meas_dev) SV_HIP(hipFree(s->meas_dev));
    s->meas_dev = nullptr;
    s->meas_cap = 0;
    SV_HIP(hipMalloc(&s->meas_dev, dev_bytes));
    s->meas_cap = dev_bytes;
  }
  if (host_bytes > s->meas_host_cap) {
    SV_HIP(hipStreamSynchronize(s->stream));
    if (s->meas_host) SV_HIP(hipHostFree(s->meas_host));
    s->meas_host = nullptr;
    s->meas_host_cap = 0;
    SV_HIP(hipHostMalloc(&s->meas_host, host_bytes, hipHostMallocDefault));
    s->meas_host_cap = host_bytes;
  }
}

static std::atomic<uint64_t> g_plan_epoch{0};
uint64_t plan_epoch() { return g_plan_epoch.load(); }
void bump_plan_epoch() { ++g_plan_epoch; }

// Everything a call's plan depends on besides the library's tables: state
// size, options, planning epoch and every gate with its matrix values.
static std::vector<unsigned char> call_key(int n, const sv_run_opts& o, const sv_gate* g, size_t ng) {
  std::vector<unsigned char> key;
  auto put = [&](const void* p, size_t b) {
    const unsigned char* c = static_cast<const unsigned char*>(p);
    key.insert(key.end(), c, c + b);
  };
  const int32_t hdr[5] = {n, o.max_k, o.fusion, o.precision, o.variant};
  const uint64_t epoch = plan_epoch();
  put(hdr, sizeof(hdr));
  put(&epoch, sizeof(epoch));
  for (size_t i = 0; i < ng; ++i) {
    put(&g[i].k, sizeof(int32_t));
    put(g[i].qubits, sizeof(int32_t) * g[i].k);
    put(&g[i].cmask, sizeof(uint64_t));
    put(&g[i].cval, sizeof(uint64_t));
    put(g[i].matrix, sizeof(double) * ((size_t)2 << (2 * g[i].k)));
  }
  return key;
}

static void drop_graph(sv_state* s) {
  s->graph_key.clear();
  s->graph_input.clear();
  if (s->graph_exec) {
    SV_HIP(hipStreamSynchronize(s->stream));
    SV_HIP(hipGraphExecDestroy(s->graph_exec));
    s->graph_exec = nullptr;
  }
}

// Everything a captured graph depends on besides the state buffer: each
// pass's launch parameters and the encoded pass data (offsets relative to the
// start of the data).
static std::vector<unsigned char> graph_key(const std::vector<Pass>& passes, const unsigned char* data,
                                            size_t total) {
  std::vector<int64_t> f;
  f.reserve(passes.size() * 28);
  for (const Pass& p : passes) {
    f.insert(f.end(), {p.k, p.variant, p.precision, (int64_t)p.mat_off, (int64_t)p.mat_bytes, p.tile_bits,
                       p.reg_iters, p.mfma_cols, (int64_t)p.cmask, (int64_t)p.cval, p.nmux, p.mfma_x});
    f.insert(f.end(), p.s, p.s + SV_MAX_K);
  }
  std::vector<unsigned char> key(f.size() * sizeof(int64_t) + total);
  std::memcpy(key.data(), f.data(), f.size() * sizeof(int64_t));
  std::memcpy(key.data() + f.size() * sizeof(int64_t), data, total);
  return key;
}

// Flops and algorithmic bytes of one pass; a controlled pass with c controls
// works on 2^(n-k-c) groups and moves 16 * 2^(n-c) bytes.
static int covered_ctrl_bits(const Pass& p) { return p.nmux > 1 ? 0 : __builtin_popcountll(p.cmask); }
static double useful_flops(int n, const Pass& p) {
  const int c = covered_ctrl_bits(p);
  return std::ldexp(1.0, n - p.k - c) * (double)(1 << p.k) * (8.0 * (1 << p.k) - 2.0);
}
static uint64_t pass_bytes(int n, const Pass& p) { return (uint64_t)16 << (n - covered_ctrl_bits(p)); }

// Resolve variants, encode all pass data into one staging region, copy it
// with one host-to-device transfer, and launch the passes (optionally as one
// captured graph).
static void run_passes(sv_state* s, const std::vector<FusedGate>& fused, const sv_run_opts& o,
                       sv_run_stats* stats) {
  // With PHASE fusion every maximal run of pure-phase gates (k <= 2) becomes
  // one phase pass; everything else is a matrix pass.
  std::vector<Pass> passes;
  std::vector<const double*> mats;               // matrix passes: the fused matrix
  std::vector<std::vector<const double*>> mux;   // multiplexed passes: the matrix of each control value
  std::vector<std::vector<unsigned char>> phase_bytes;  // phase passes: their coefficients and table
  size_t total = 0;
  auto add = [&](Pass& p) {
    if (p.variant == V_MFMA) {
      p.mfma_x = mfma_exchange_mask(s->n, p);
      p.mat_bytes = pass_data_bytes(p);
    }
    p.mat_off = total;
    total += align256(p.mat_bytes);
    passes.push_back(p);
  };
  for (size_t i = 0; i < fused.size();) {
    auto phase_gate = [&](const FusedGate& f) { return !f.cmask && is_phase_matrix(f.k, f.mat.data()); };
    if ((o.fusion == SV_FUSE_PHASE || o.fusion == SV_FUSE_LEARNED) && phase_gate(fused[i])) {
      PhasePoly poly(s->n);
      size_t j = i;
      for (; j < fused.size() && phase_gate(fused[j]); ++j)
        poly.add_gate(fused[j].k, fused[j].q, fused[j].mat.data());
      Pass p;
      p.k = 0;
      p.variant = V_PHASE;
      p.mat_bytes = phase_data_bytes(s->n);
      std::vector<unsigned char> bytes(p.mat_bytes);
      phase_data(poly, s->n, bytes.data());
      add(p);
      mats.push_back(nullptr);
      mux.emplace_back();
      phase_bytes.push_back(std::move(bytes));
      i = j;
      continue;
    }
    Pass p;
    p.k = fused[i].k;
    std::copy(fused[i].q, fused[i].q + p.k, p.s);
    p.precision = o.precision;
    p.cmask = fused[i].cmask;
    p.cval = fused[i].cval;
    if (p.cmask) {  // controlled passes: matrix cores when they take the controls, else registers in FP32
      const bool mfma = mfma_supported(p.k, o.precision) && mfma_ctrl_supported(s->n, p.k, p.cmask) &&
                        o.variant != SV_VARIANT_REG && o.variant != SV_VARIANT_LDS && o.variant != SV_VARIANT_SHFL;
      // A block with controls comes as one gate per control value on the
      // same targets: on the matrix cores all of them are one launch.
      const int c = __builtin_popcountll(p.cmask);
      size_t j = i;
      std::vector<const double*> by_value;
      if (mfma) {
        int cbit[kBlockCtrl + 1], nc = 0;
        for (int b = 0; b < 64 && nc <= kBlockCtrl; ++b)
          if ((p.cmask >> b) & 1) cbit[nc++] = b;
        by_value.assign((size_t)1 << c, nullptr);
        while (j < fused.size() && j - i < by_value.size() && fused[j].cmask == p.cmask && fused[j].k == p.k &&
               std::equal(fused[j].q, fused[j].q + p.k, fused[i].q)) {
          int v = 0;
          for (int t = 0; t < nc; ++t)
            if ((fused[j].cval >> cbit[t]) & 1) v |= 1 << t;
          if (by_value[v]) break;  // a repeated value starts another block
          by_value[v] = fused[j].mat.data();
          ++j;
        }
      }
      if (mfma && c >= 1 && j - i == ((size_t)1 << c)) {
        p.variant = V_MFMA;
        p.nmux = 1 << c;
        p.mat_bytes = pass_data_bytes(p);
        add(p);
        mats.push_back(nullptr);
        mux.push_back(std::move(by_value));
        phase_bytes.emplace_back();
        i = j;
        continue;
      }
      if (mfma) {
        p.variant = V_MFMA;
      } else {
        p.precision = SV_PREC_FP32_VALU;
        p.variant = V_REG;
      }
      p.mat_bytes = pass_data_bytes(p);
      add(p);
      mats.push_back(fused[i].mat.data());
      mux.emplace_back();
      phase_bytes.emplace_back();
      ++i;
      continue;
    }
    p.variant = choose_variant(s->n, p.k, p.s, o.precision, o.variant == SV_VARIANT_SHFL ? V_SHFL : o.variant);
    const Shape sh = tuned_shape(p.variant, s->n, p.k, p.s, o.precision);
    p.tile_bits = sh.tile_bits;
    p.reg_iters = sh.reg_iters;
    p.mfma_cols = sh.mfma_cols;
    p.mat_bytes = pass_data_bytes(p);
    add(p);
    mats.push_back(fused[i].mat.data());
    mux.emplace_back();
    phase_bytes.emplace_back();
    ++i;
  }
  if (total == 0) return;
  const size_t base = arena_take(s, total);
  std::vector<size_t> rel(passes.size());  // offsets of each pass's data from base
  for (size_t i = 0; i < passes.size(); ++i) rel[i] = passes[i].mat_off;
  auto encode = [&](size_t i) {
    unsigned char* dst = s->arena_host + base + rel[i];
    if (passes[i].variant == V_PHASE) {
      std::memcpy(dst, phase_bytes[i].data(), passes[i].mat_bytes);
    } else if (passes[i].nmux > 1) {
      const size_t each = passes[i].mat_bytes / passes[i].nmux;
      for (int v = 0; v < passes[i].nmux; ++v) encode_pass_data(passes[i], mux[i][v], dst + v * each);
    } else {
      encode_pass_data(passes[i], mats[i], dst);
    }
  };
  const bool timing = o.timing && stats;
  const bool graph = o.use_graph && !timing;
  if (timing)
    while (s->pass_events.size() < 2 * passes.size()) {  // a start and an end per pass
      hipEvent_t e;
      SV_HIP(hipEventCreate(&e));
      s->pass_events.push_back(e);
    }
  auto launch = [&](size_t i) {
    if (timing) SV_HIP(hipEventRecord(s->pass_events[2 * i], s->stream));
    launch_pass(passes[i], s->n, s->psi, s->arena_dev, s->stream);
    if (timing) SV_HIP(hipEventRecord(s->pass_events[2 * i + 1], s->stream));
  };
  if (graph) {
    for (size_t i = 0; i < passes.size(); ++i) encode(i);
    // The graph reads its pass data from its own buffer, so ring uploads of
    // later calls never disturb it; relaunch when nothing it encodes changed.
    std::vector<unsigned char> key = graph_key(passes, s->arena_host + base, total);
    const bool relaunch = s->graph_exec && key == s->graph_key;
    if (stats) stats->graph_relaunched = relaunch ? 1 : 0;
    if (!relaunch) {
      drop_graph(s);
      if (total > s->graph_cap) {
        SV_HIP(hipStreamSynchronize(s->stream));
        if (s->graph_dev) SV_HIP(hipFree(s->graph_dev));
        s->graph_dev = nullptr;
        s->graph_cap = 0;
        SV_HIP(hipMalloc(&s->graph_dev, total));
        s->graph_cap = total;
      }
      SV_HIP(hipMemcpyAsync(s->graph_dev, s->arena_host + base, total, hipMemcpyHostToDevice, s->stream));
      // Capture records without executing, so a private stream serves any
      // caller stream, the legacy null stream included.
      if (!s->capture_stream) SV_HIP(hipStreamCreateWithFlags(&s->capture_stream, hipStreamNonBlocking));
      hipStream_t cs = s->capture_stream;
      SV_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      try {
        for (const Pass& p : passes) launch_pass(p, s->n, s->psi, s->graph_dev, cs);
      } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(cs, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      hipGraph_t g = nullptr;
      SV_HIP(hipStreamEndCapture(cs, &g));
      hipError_t e = hipGraphInstantiate(&s->graph_exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) {
        s->graph_exec = nullptr;
        throw DeviceError{e, "hipGraphInstantiate"};
      }
      s->graph_key = std::move(key);
    }
    s->graph_launched = true;
    s->graph_passes = passes.size();
    s->graph_bytes = 0;
    s->graph_flops = 0.0;
    for (const Pass& p : passes) {
      s->graph_bytes += pass_bytes(s->n, p);
      if (p.variant != V_PHASE) s->graph_flops += useful_flops(s->n, p);
    }
    if (stats) SV_HIP(hipEventRecord(s->ev0, s->stream));
    SV_HIP(hipGraphLaunch(s->graph_exec, s->stream));
  } else {
    // Passes go out in chunks: the first pass alone, then each time as many
    // as the host encodes while the GPU still has queued work (an event after
    // every chunk tells), so encoding hides behind the passes instead of
    // preceding them.
    for (Pass& p : passes) p.mat_off += base;
    size_t next = 0;
    while (next < passes.size()) {
      const size_t lo = next;
      encode(next++);
      while (lo > 0 && next < passes.size()) {
        const hipError_t q = hipEventQuery(s->queued);
        if (q == hipSuccess) break;  // the GPU ran dry: send what is ready
        if (q != hipErrorNotReady) throw DeviceError{q, "hipEventQuery"};
        encode(next++);
      }
      const size_t from = rel[lo], to = next < passes.size() ? rel[next] : total;
      SV_HIP(hipMemcpyAsync(s->arena_dev + base + from, s->arena_host + base + from, to - from,
                            hipMemcpyHostToDevice, s->stream));
      if (lo == 0 && stats) SV_HIP(hipEventRecord(s->ev0, s->stream));
      for (size_t i = lo; i < next; ++i) launch(i);
      SV_HIP(hipEventRecord(s->queued, s->stream));
    }
  }
  if (stats) {
    SV_HIP(hipEventRecord(s->ev1, s->stream));
    SV_HIP(hipEventSynchronize(s->ev1));
    float ms = 0.f;
    SV_HIP(hipEventElapsedTime(&ms, s->ev0, s->ev1));
    stats->gpu_s = ms * 1e-3;
    stats->passes = passes.size();
    stats->launches = passes.size();
    stats->bytes = 0;
    double fl = 0.0;
    for (const Pass& p : passes) {
      stats->bytes += pass_bytes(s->n, p);
      if (p.variant != V_PHASE) fl += useful_flops(s->n, p);
    }
    stats->useful_flops = fl;
    if (timing) {
      for (size_t i = 0; i < passes.size(); ++i) {
        float pm = 0.f;
        SV_HIP(hipEventElapsedTime(&pm, s->pass_events[2 * i], s->pass_events[2 * i + 1]));
        const int v = variant_family(passes[i].variant);
        stats->variant_s[v] += pm * 1e-3;
        stats->variant_passes[v] += 1;
        stats->variant_bytes[v] += pass_bytes(s->n, passes[i]);
      }
    }
  }
}

static sv_run_opts default_opts() {
  sv_run_opts o{};
  o.max_k = 4;
  o.fusion = SV_FUSE_GREEDY;
  o.precision = SV_PREC_FP32_VALU;
  o.use_graph = 0;
  o.variant = SV_VARIANT_AUTO;
  return o;
}

static int check_opts(const sv_run_opts& o) {
  if (o.fusion < SV_FUSE_NONE || o.fusion > SV_FUSE_BLOCK) return fail(SV_EINVAL, "opts.fusion invalid");
  if (o.fusion != SV_FUSE_NONE && (o.max_k < 1 || o.max_k > SV_MAX_K))
    return fail(SV_EINVAL, "opts.max_k must be 1..6");
  if (o.precision < SV_PREC_FP32_VALU || o.precision > SV_PREC_FP16X3)
    return fail(SV_EINVAL, "opts.precision invalid");
  if (o.variant < SV_VARIANT_AUTO || o.variant > SV_VARIANT_SHFL) return fail(SV_EINVAL, "opts.variant invalid");
  if (o.timing != 0 && o.timing != 1) return fail(SV_EINVAL, "opts.timing must be 0 or 1");
  return SV_OK;
}

// Fuse per opts into `fused`.
// Controls a fused block may take: only where its per-value matrices run as
// one matrix-core launch (a precision the matrix cores take) on a state of at
// least kBlockCtrlMinQubits; elsewhere the per-value passes would be
// separate FP32 register launches, slower than the sweeps they save.
static int block_ctrl(int n_qubits, int precision) {
  return n_qubits >= kBlockCtrlMinQubits && mfma_supported(4, precision) ? kBlockCtrl : 0;
}

int plan_fusion(const sv_gate* g_in, size_t n, int n_qubits, const sv_run_opts& o, std::vector<FusedGate>& fused,
                std::vector<int32_t>& block_of, int max_ctrl) {
  // controlled gates narrow enough to fuse are lifted to dense gates first
  std::vector<sv_gate> lowered;
  std::vector<std::vector<double>> store;
  const sv_gate* g = g_in;
  if (o.fusion != SV_FUSE_NONE) {
    bool any = false;
    for (size_t i = 0; i < n && !any; ++i) any = g_in[i].cmask != 0;
    if (any) {
      lower_controlled(g_in, n, o.max_k, lowered, store);
      g = lowered.data();
    }
  }
  if (o.fusion == SV_FUSE_NONE) {
    fuse_none(g, n, fused, block_of);
  } else if (o.fusion == SV_FUSE_PHASE) {
    fuse_phase(g, n, o.max_k, fused, block_of);
  } else if (o.fusion == SV_FUSE_LEARNED) {
    fuse_learned(g, n, n_qubits, o.max_k, o.precision, fused, block_of, max_ctrl);
  } else if (o.fusion == SV_FUSE_BLOCK) {
    fuse_maxblock(g, n, o.max_k, fused, block_of);
  } else {
    fuse_greedy(g, n, o.max_k, fused, block_of);
  }
  return SV_OK;
}

}  // namespace sv

using namespace sv;

#define SV_GUARD_BEGIN try {
#define SV_GUARD_END(handle)                                                                  \
  }                                                                                           \
  catch (const DeviceError& e) {                                                              \
    if (handle) (handle)->poisoned = true;                                                    \
    return fail(SV_EDEVICE, std::string(e.what) + ": " + hipGetErrorString(e.err));           \
  }                                                                                           \
  catch (const std::bad_alloc&) {                                                             \
    return fail(SV_ENOMEM, "host allocation failed");                                         \
  }                                                                                           \
  catch (const std::exception& e) {                                                           \
    return fail(SV_EINVAL, e.what());                                                         \
  }                                                                                           \
  catch (...) {                                                                               \
    return fail(SV_EINVAL, "unknown failure");                                                \
  }

// FP16X3 scales amplitudes by 2^14 before rounding to fp16 (largest finite
// 65504): |c| must stay below ~3.99.  Every |c| <= sqrt(sum |c|^2), so a
// state with sum |c|^2 <= 15 is safe, and unitary passes keep that sum.
static constexpr double kFp16x3MaxNormSq = 15.0;

// Every gate unitary to 1e-6 per entry of U^dagger U - I (FP64, host).
static bool gates_unitary(const sv_gate* g, size_t n) {
  for (size_t i = 0; i < n; ++i) {
    const int d = 1 << g[i].k;
    const double* m = g[i].matrix;
    for (int a = 0; a < d; ++a)
      for (int b = a; b < d; ++b) {
        double re = 0.0, im = 0.0;  // (U^dagger U)[a][b] = sum_r conj(U[r][a]) U[r][b]
        for (int r = 0; r < d; ++r) {
          const double ar = m[2 * (r * d + a)], ai = m[2 * (r * d + a) + 1];
          const double br = m[2 * (r * d + b)], bi = m[2 * (r * d + b) + 1];
          re += ar * br + ai * bi;
          im += ar * bi - ai * br;
        }
        if (std::fabs(re - (a == b ? 1.0 : 0.0)) > 1e-6 || std::fabs(im) > 1e-6) return false;
      }
  }
  return true;
}

static int check_handle(sv_state* s) {
  if (!s) return fail(SV_EINVAL, "state handle is NULL");
  if (s->poisoned) return fail(SV_ESTATE, "handle poisoned by an earlier device failure");
  return SV_OK;
}

extern "C" {

const char* sv_last_error(void) { return g_last_error.c_str(); }
const char* sv_version(void) { return "libsv 0.1.0 (gfx950)"; }
size_t sv_struct_size(int which) {
  switch (which) {
    case 0: return sizeof(sv_gate);
    case 1: return sizeof(sv_run_opts);
    case 2: return sizeof(sv_run_stats);
    default: return 0;
  }
}

int sv_alloc(int n_qubits, int dtype, void* dev_buf, size_t buf_bytes, void* hip_stream, sv_state** out) {
  if (!out) return fail(SV_EINVAL, "out is NULL");
  *out = nullptr;
  if (dtype != SV_C64) return fail(SV_EINVAL, "only SV_C64 states are supported");
  if (n_qubits < 1 || n_qubits > SV_MAX_QUBITS) return fail(SV_EINVAL, "n_qubits must be 1..40");
  if (!dev_buf) return fail(SV_EINVAL, "dev_buf is NULL");
  const size_t need = (size_t)8 << n_qubits;
  if (buf_bytes < need) return fail(SV_ENOMEM, "buffer holds " + std::to_string(buf_bytes) + " bytes, need " +
                                                   std::to_string(need));
  if (((uintptr_t)dev_buf & 15) != 0) return fail(SV_EINVAL, "dev_buf must be 16-byte aligned");
  sv_state* s = nullptr;
  SV_GUARD_BEGIN
  s = new sv_state();
  s->n = n_qubits;
  s->psi = dev_buf;
  s->stream = (hipStream_t)hip_stream;
  SV_HIP(hipGetDevice(&s->device));
  SV_HIP(hipMalloc(&s->partials, sizeof(double) * (norm_partials_needed() + 1)));
  s->norm_dev = s->partials + norm_partials_needed();
  SV_HIP(hipHostMalloc(&s->norm_host, sizeof(double), hipHostMallocDefault));
  SV_HIP(hipEventCreate(&s->ev0));
  SV_HIP(hipEventCreate(&s->ev1));
  SV_HIP(hipEventCreateWithFlags(&s->queued, hipEventDisableTiming));
  // the matrix arena is allocated on the first gate upload
  launch_init_basis(s->psi, s->n, 0, s->stream);
  *out = s;
  return SV_OK;
  }
  catch (const DeviceError& e) {
    sv_free(s);
    return fail(e.err == hipErrorOutOfMemory ? SV_ENOMEM : SV_EDEVICE,
                std::string(e.what) + ": " + hipGetErrorString(e.err));
  }
  catch (const std::bad_alloc&) {
    sv_free(s);
    return fail(SV_ENOMEM, "host allocation failed");
  }
  catch (...) {
    sv_free(s);
    return fail(SV_EINVAL, "unknown failure");
  }
}

int sv_free(sv_state* s) {
  if (!s) return SV_OK;
  (void)hipSetDevice(s->device);
  (void)hipStreamSynchronize(s->stream);
  if (s->graph_exec) (void)hipGraphExecDestroy(s->graph_exec);
  if (s->graph_dev) (void)hipFree(s->graph_dev);
  if (s->capture_stream) (void)hipStreamDestroy(s->capture_stream);
  if (s->arena_dev) (void)hipFree(s->arena_dev);
  if (s->arena_host) (void)hipHostFree(s->arena_host);
  if (s->partials) (void)hipFree(s->partials);
  if (s->norm_host) (void)hipHostFree(s->norm_host);
  if (s->ev0) (void)hipEventDestroy(s->ev0);
  if (s->ev1) (void)hipEventDestroy(s->ev1);
  if (s->queued) (void)hipEventDestroy(s->queued);
  for (hipEvent_t e : s->pass_events) (void)hipEventDestroy(e);
  if (s->meas_dev) (void)hipFree(s->meas_dev);
  if (s->meas_host) (void)hipHostFree(s->meas_host);
  delete s;
  return SV_OK;
}

int sv_num_qubits(const sv_state* s) { return s ? s->n : fail(SV_EINVAL, "state handle is NULL"); }

int sv_set_basis(sv_state* s, uint64_t index) {
  if (int rc = check_handle(s)) return rc;
  if (index >> s->n) return fail(SV_EINVAL, "basis index out of range");
  SV_GUARD_BEGIN
  SV_HIP(hipSetDevice(s->device));
  launch_init_basis(s->psi, s->n, index, s->stream);
  s->norm_known = 1.0;
  return SV_OK;
  SV_GUARD_END(s)
}

int sv_apply_gate(sv_state* s, const int32_t* qubits, int k, const double* matrix) {
  if (int rc = check_handle(s)) return rc;
  if (!qubits) return fail(SV_EINVAL, "qubits is NULL");
  if (k < 1 || k > SV_MAX_K) return fail(SV_EINVAL, "k must be 1..6");
  sv_gate g{};
  g.k = k;
  std::copy(qubits, qubits + k, g.qubits);
  g.matrix = matrix;
  if (int rc = validate_gates(&g, 1, s->n)) return rc;
  SV_GUARD_BEGIN
  SV_HIP(hipSetDevice(s->device));
  std::vector<FusedGate> fused;
  std::vector<int32_t> block_of;
  fuse_none(&g, 1, fused, block_of);
  sv_run_opts o = default_opts();
  o.fusion = SV_FUSE_NONE;
  run_passes(s, fused, o, nullptr);
  if (!gates_unitary(&g, 1)) s->norm_known = -1.0;
  return SV_OK;
  SV_GUARD_END(s)
}

int sv_apply_controlled_gate(sv_state* s, const int32_t* qubits, int k, const double* matrix, int nc,
                             const int32_t* controls, const int32_t* control_values) {
  if (int rc = check_handle(s)) return rc;
  if (!qubits) return fail(SV_EINVAL, "qubits is NULL");
  if (k < 1 || k > SV_MAX_K) return fail(SV_EINVAL, "k must be 1..6");
  if (nc < 0 || nc > s->n || (nc > 0 && !controls)) return fail(SV_EINVAL, "bad control list");
  sv_gate g{};
  g.k = k;
  std::copy(qubits, qubits + k, g.qubits);
  g.matrix = matrix;
  for (int j = 0; j < nc; ++j) {
    const int q = controls[j];
    if (q < 0 || q >= s->n) return fail(SV_EINVAL, "control " + std::to_string(q) + " out of range");
    if ((g.cmask >> q) & 1) return fail(SV_EINVAL, "control " + std::to_string(q) + " repeated");
    const int v = control_values ? control_values[j] : 1;
    if (v != 0 && v != 1) return fail(SV_EINVAL, "control values must be 0 or 1");
    g.cmask |= (uint64_t)1 << q;
    if (v) g.cval |= (uint64_t)1 << q;
  }
  if (int rc = validate_gates(&g, 1, s->n)) return rc;
  SV_GUARD_BEGIN
  SV_HIP(hipSetDevice(s->device));
  std::vector<FusedGate> fused;
  std::vector<int32_t> block_of;
  fuse_none(&g, 1, fused, block_of);
  sv_run_opts o = default_opts();
  o.fusion = SV_FUSE_NONE;
  run_passes(s, fused, o, nullptr);
  if (!gates_unitary(&g, 1)) s->norm_known = -1.0;
  return SV_OK;
  SV_GUARD_END(s)
}

int sv_apply_circuit(sv_state* s, const sv_gate* gates, size_t n_gates, const sv_run_opts* opts,
                     sv_run_stats* stats) {
  if (int rc = check_handle(s)) return rc;
  const sv_run_opts o = opts ? *opts : default_opts();
  if (int rc = check_opts(o)) return rc;
  if (int rc = validate_gates(gates, n_gates, s->n)) return rc;
  const bool unitary = gates_unitary(gates, n_gates);
  if (o.precision == SV_PREC_FP16X3 && !unitary)
    return fail(SV_EINVAL, "FP16X3 needs unitary gates (a gate's U^dagger U differs from I by more than 1e-6): "
                           "use FP32_MFMA or BF16X3");
  SV_GUARD_BEGIN
  SV_HIP(hipSetDevice(s->device));
  if (o.precision == SV_PREC_FP16X3) {
    if (s->norm_known < 0.0) {  // measure it once (one read sweep)
      launch_norm(s->psi, s->n, s->partials, norm_partials_needed(), s->norm_dev, s->stream);
      SV_HIP(hipMemcpyAsync(s->norm_host, s->norm_dev, sizeof(double), hipMemcpyDeviceToHost, s->stream));
      SV_HIP(hipStreamSynchronize(s->stream));
      s->norm_known = *s->norm_host;
    }
    if (!(s->norm_known <= kFp16x3MaxNormSq))
      return fail(SV_EINVAL, "FP16X3 needs sum |c|^2 <= 15 (amplitudes above ~4 overflow fp16 after the 2^14 "
                             "scale); the state has " + std::to_string(s->norm_known) + ": use FP32_MFMA or BF16X3");
  }
  if (!unitary) s->norm_known = -1.0;
  if (stats) *stats = sv_run_stats{};
  const bool graph = o.use_graph && !(o.timing && stats);
  std::vector<unsigned char> key;
  if (graph) {
    // the same gates and options as the kept graph's call: relaunch it
    // without fusing or uploading anything
    key = call_key(s->n, o, gates, n_gates);
    if (s->graph_exec && key == s->graph_input) {
      if (stats) SV_HIP(hipEventRecord(s->ev0, s->stream));
      SV_HIP(hipGraphLaunch(s->graph_exec, s->stream));
      if (stats) {
        SV_HIP(hipEventRecord(s->ev1, s->stream));
        SV_HIP(hipEventSynchronize(s->ev1));
        float ms = 0.f;
        SV_HIP(hipEventElapsedTime(&ms, s->ev0, s->ev1));
        stats->gpu_s = ms * 1e-3;
        stats->passes = s->graph_passes;
        stats->launches = s->graph_passes;
        stats->bytes = s->graph_bytes;
        stats->useful_flops = s->graph_flops;
        stats->gates_in = n_gates;
        stats->graph_relaunched = 1;
      }
      return SV_OK;
    }
  }
  const auto t0 = std::chrono::steady_clock::now();
  std::vector<FusedGate> fused;
  std::vector<int32_t> block_of;
  plan_fusion(gates, n_gates, s->n, o, fused, block_of, block_ctrl(s->n, o.precision));
  const double fuse_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  s->graph_launched = false;
  run_passes(s, fused, o, stats);
  if (graph && s->graph_launched) s->graph_input = std::move(key);
  if (stats) {
    stats->gates_in = n_gates;
    stats->fuse_s = fuse_s;
  }
  return SV_OK;
  SV_GUARD_END(s)
}

int sv_fuse(const sv_gate* in, size_t n_in, int n_qubits, const sv_run_opts* opts, sv_gate** out, size_t* n_out,
            int32_t** block_of_gate) {
  if (!out || !n_out) return fail(SV_EINVAL, "out / n_out is NULL");
  *out = nullptr;
  *n_out = 0;
  if (block_of_gate) *block_of_gate = nullptr;
  if (n_qubits < 1 || n_qubits > SV_MAX_QUBITS) return fail(SV_EINVAL, "n_qubits must be 1..40");
  const sv_run_opts o = opts ? *opts : default_opts();
  if (int rc = check_opts(o)) return rc;
  if (int rc = validate_gates(in, n_in, n_qubits)) return rc;
  try {
    std::vector<FusedGate> fused;
    std::vector<int32_t> block_of;
    plan_fusion(in, n_in, n_qubits, o, fused, block_of, block_ctrl(n_qubits, o.precision));
    // one allocation for the gate array, a second for all matrices
    size_t doubles = 0;
    for (auto& f : fused) doubles += f.mat.size();
    sv_gate* g = (sv_gate*)std::malloc(sizeof(sv_gate) * (fused.size() ? fused.size() : 1));
    double* m = (double*)std::malloc(sizeof(double) * (doubles ? doubles : 1));
    if (!g || !m) {
      std::free(g);
      std::free(m);
      return fail(SV_ENOMEM, "host allocation failed");
    }
    size_t pos = 0;
    for (size_t i = 0; i < fused.size(); ++i) {
      g[i] = sv_gate{};
      g[i].k = fused[i].k;
      std::copy(fused[i].q, fused[i].q + fused[i].k, g[i].qubits);
      g[i].cmask = fused[i].cmask;
      g[i].cval = fused[i].cval;
      std::memcpy(m + pos, fused[i].mat.data(), sizeof(double) * fused[i].mat.size());
      g[i].matrix = m + pos;
      pos += fused[i].mat.size();
    }
    if (fused.empty()) std::free(m);
    if (block_of_gate) {
      int32_t* b = (int32_t*)std::malloc(sizeof(int32_t) * (n_in ? n_in : 1));
      if (!b) {
        std::free(g);
        if (!fused.empty()) std::free(m);
        return fail(SV_ENOMEM, "host allocation failed");
      }
      std::copy(block_of.begin(), block_of.end(), b);
      *block_of_gate = b;
    }
    *out = g;
    *n_out = fused.size();
    return SV_OK;
  } catch (const std::bad_alloc&) {
    return fail(SV_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(SV_EINVAL, e.what());
  } catch (...) {
    return fail(SV_EINVAL, "unknown failure");
  }
}

int sv_fused_free(sv_gate* fused, size_t n, int32_t* block_of_gate) {
  if (fused && n > 0) std::free((void*)fused[0].matrix);
  std::free(fused);
  std::free(block_of_gate);
  return SV_OK;
}

int sv_norm(sv_state* s, double* norm_sq) {
  if (int rc = check_handle(s)) return rc;
  if (!norm_sq) return fail(SV_EINVAL, "norm_sq is NULL");
  SV_GUARD_BEGIN
  SV_HIP(hipSetDevice(s->device));
  launch_norm(s->psi, s->n, s->partials, norm_partials_needed(), s->norm_dev, s->stream);
  SV_HIP(hipMemcpyAsync(s->norm_host, s->norm_dev, sizeof(double), hipMemcpyDeviceToHost, s->stream));
  SV_HIP(hipStreamSynchronize(s->stream));
  *norm_sq = *s->norm_host;
  s->norm_known = *norm_sq;
  return SV_OK;
  SV_GUARD_END(s)
}

int sv_norm_noalloc(const void* dev_state, int n_qubits, size_t buf_bytes, void* hip_stream, double* dev_out) {
  if (!dev_state || !dev_out) return fail(SV_EINVAL, "dev_state / dev_out is NULL");
  if (n_qubits < 1 || n_qubits > SV_MAX_QUBITS) return fail(SV_EINVAL, "n_qubits must be 1..40");
  const size_t need = (size_t)8 << n_qubits;
  if (buf_bytes < need)
    return fail(SV_EINVAL, "buffer holds " + std::to_string(buf_bytes) + " bytes, need " + std::to_string(need));
  if (((uintptr_t)dev_state & 15) != 0) return fail(SV_EINVAL, "dev_state must be 16-byte aligned");
  if (((uintptr_t)dev_out & 7) != 0) return fail(SV_EINVAL, "dev_out must be 8-byte aligned");
  try {
    int dev = 0;
    SV_HIP(hipGetDevice(&dev));
    for (const void* p : {dev_state, static_cast<const void*>(dev_out)}) {
      hipPointerAttribute_t attr{};
      if (hipPointerGetAttributes(&attr, p) != hipSuccess || attr.type != hipMemoryTypeDevice) {
        (void)hipGetLastError();
        return fail(SV_EINVAL, "dev_state and dev_out must be device memory");
      }
      if (attr.device != dev) return fail(SV_EINVAL, "dev_state and dev_out must be on the current device");
    }
    launch_norm_noalloc(dev_state, n_qubits, dev_out, (hipStream_t)hip_stream);
    return SV_OK;
  } catch (const DeviceError& e) {
    return fail(SV_EDEVICE, std::string(e.what) + ": " + hipGetErrorString(e.err));
  } catch (...) {
    return fail(SV_EDEVICE, "unknown failure");
  }
}

int sv_expect_pauli(sv_state* s, size_t n_terms, const uint64_t* xmask, const uint64_t* zmask, double* out) {
  if (int rc = check_handle(s)) return rc;
  if (n_terms == 0) return SV_OK;
  if (!xmask || !zmask || !out) return fail(SV_EINVAL, "xmask / zmask / out is NULL");
  for (size_t t = 0; t < n_terms; ++t)
    if (s->n < 64 && ((xmask[t] | zmask[t]) >> s->n) != 0)
      return fail(SV_EINVAL, "term " + std::to_string(t) + ": Pauli mask past qubit n-1");
  SV_GUARD_BEGIN
  SV_HIP(hipSetDevice(s->device));
  // sweeps: terms grouped by their flip mask, at most 8 per sweep, in first-seen order
  std::vector<uint64_t> sweep_f;
  std::vector<std::vector<size_t>> sweep_terms;
  {
    std::unordered_map<uint64_t, size_t> open;  // flip mask -> the sweep being filled
    for (size_t t = 0; t < n_terms; ++t) {
      auto it = open.find(xmask[t]);
      if (it == open.end() || sweep_terms[it->second].size() == 8) {
        const size_t w = sweep_f.size();
        sweep_f.push_back(xmask[t]);
        sweep_terms.emplace_back();
        open[xmask[t]] = w;
        sweep_terms[w].push_back(t);
      } else {
        sweep_terms[it->second].push_back(t);
      }
    }
  }
  const size_t outs = sizeof(double) * 16 * sweep_f.size();
  meas_reserve(s, pauli_scratch_bytes() + outs, outs);
  double* scratch = reinterpret_cast<double*>(s->meas_dev);
  double* res = reinterpret_cast<double*>(s->meas_dev + pauli_scratch_bytes());
  for (size_t w = 0; w < sweep_f.size(); ++w) {
    uint64_t z[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (size_t j = 0; j < sweep_terms[w].size(); ++j) z[j] = zmask[sweep_terms[w][j]];
    launch_pauli(s->psi, s->n, sweep_f[w], (int)sweep_terms[w].size(), z, scratch, res + 16 * w, s->stream);
  }
  SV_HIP(hipMemcpyAsync(s->meas_host, res, outs, hipMemcpyDeviceToHost, s->stream));
  SV_HIP(hipStreamSynchronize(s->stream));
  const double* h = reinterpret_cast<const double*>(s->meas_host);
  for (size_t w = 0; w < sweep_f.size(); ++w)
    for (size_t j = 0; j < sweep_terms[w].size(); ++j) {
      const size_t t = sweep_terms[w][j];
      const double re = h[16 * w + 2 * j], im = h[16 * w + 2 * j + 1];
      // P = i^ny X^f Z^z with ny = |f & z| (the Y letters): Re(i^ny (re + i im))
      switch (__builtin_popcountll(xmask[t] & zmask[t]) & 3) {
        case 0: out[t] = re; break;
        case 1: out[t] = -im; break;
        case 2: out[t] = -re; break;
        default: out[t] = im; break;
      }
    }
  return SV_OK;
  SV_GUARD_END(s)
}

int sv_marginal_probs(sv_state* s, int n_meas, const int32_t* qubits, double* out) {
  if (int rc = check_handle(s)) return rc;
  if (!qubits || !out) return fail(SV_EINVAL, "qubits / out is NULL");
  if (n_meas < 1 || n_meas > marginal_max_qubits() || n_meas > s->n)
    return fail(SV_EINVAL, "n_meas must be 1..min(10, n)");
  int q[16];
  for (int j = 0; j < n_meas; ++j) {
    q[j] = qubits[j];
    if (q[j] < 0 || q[j] >= s->n) return fail(SV_EINVAL, "qubit " + std::to_string(q[j]) + " out of range");
    for (int a = 0; a < j; ++a)
      if (q[a] == q[j]) return fail(SV_EINVAL, "qubit " + std::to_string(q[j]) + " repeated");
  }
  SV_GUARD_BEGIN
  SV_HIP(hipSetDevice(s->device));
  const size_t outs = sizeof(double) << n_meas;
  meas_reserve(s, marginal_scratch_bytes(n_meas) + outs, outs);
  double* res = reinterpret_cast<double*>(s->meas_dev + marginal_scratch_bytes(n_meas));
  launch_marginal(s->psi, s->n, n_meas, q, reinterpret_cast<double*>(s->meas_dev), res, s->stream);
  SV_HIP(hipMemcpyAsync(s->meas_host, res, outs, hipMemcpyDeviceToHost, s->stream));
  SV_HIP(hipStreamSynchronize(s->stream));
  std::memcpy(out, s->meas_host, outs);
  return SV_OK;
  SV_GUARD_END(s)
}

int sv_sample(sv_state* s, size_t n_shots, const double* uniforms, uint64_t* out) {
  if (int rc = check_handle(s)) return rc;
  if (n_shots == 0) return SV_OK;
  if (!uniforms || !out) return fail(SV_EINVAL, "uniforms / out is NULL");
  for (size_t j = 0; j < n_shots; ++j)
    if (!(uniforms[j] >= 0.0 && uniforms[j] < 1.0))
      return fail(SV_EINVAL, "uniform " + std::to_string(j) + " outside [0, 1)");
  SV_GUARD_BEGIN
  SV_HIP(hipSetDevice(s->device));
  constexpr size_t kBatch = (size_t)1 << 20;  // shots per upload
  const size_t batch = std::min(n_shots, kBatch);
  const size_t sbytes = (sample_scratch_bytes(s->n) + 255) & ~(size_t)255;
  meas_reserve(s, sbytes + 16 * batch, 16 * batch);
  double* scratch = reinterpret_cast<double*>(s->meas_dev);
  double* u_dev = reinterpret_cast<double*>(s->meas_dev + sbytes);
  uint64_t* o_dev = reinterpret_cast<uint64_t*>(s->meas_dev + sbytes + 8 * batch);
  double* u_host = reinterpret_cast<double*>(s->meas_host);
  uint64_t* o_host = reinterpret_cast<uint64_t*>(s->meas_host + 8 * batch);
  for (size_t done = 0; done < n_shots; done += batch) {
    const size_t m = std::min(batch, n_shots - done);
    SV_HIP(hipStreamSynchronize(s->stream));  // the pinned staging is free again
    std::memcpy(u_host, uniforms + done, 8 * m);
    SV_HIP(hipMemcpyAsync(u_dev, u_host, 8 * m, hipMemcpyHostToDevice, s->stream));
    launch_sample(s->psi, s->n, done == 0, u_dev, m, o_dev, scratch, s->stream);
    SV_HIP(hipMemcpyAsync(o_host, o_dev, 8 * m, hipMemcpyDeviceToHost, s->stream));
    SV_HIP(hipStreamSynchronize(s->stream));
    for (size_t j = 0; j < m; ++j) {
      if (o_host[j] == ~(uint64_t)0) return fail(SV_EINVAL, "cannot sample a zero state");
      out[done + j] = o_host[j];
    }
  }
  return SV_OK;
  SV_GUARD_END(s)
}

int sv_read_amplitudes(sv_state* s, uint64_t start, uint64_t count, float* host_out) {
  if (int rc = check_handle(s)) return rc;
  if (!host_out && count) return fail(SV_EINVAL, "host_out is NULL");
  const uint64_t len = (uint64_t)1 << s->n;
  if (start > len || count > len - start) return fail(SV_EINVAL, "amplitude range out of bounds");
  SV_GUARD_BEGIN
  SV_HIP(hipSetDevice(s->device));
  const uint64_t chunk = (uint64_t)1 << 26;
  for (uint64_t done = 0; done < count; done += chunk) {
    const uint64_t c = std::min(chunk, count - done);
    SV_HIP(hipMemcpyAsync(host_out + 2 * done, (const float*)s->psi + 2 * (start + done), c * 8,
                          hipMemcpyDeviceToHost, s->stream));
  }
  SV_HIP(hipStreamSynchronize(s->stream));
  return SV_OK;
  SV_GUARD_END(s)
}

int sv_write_amplitudes(sv_state* s, uint64_t start, uint64_t count, const float* host_in) {
  if (int rc = check_handle(s)) return rc;
  if (!host_in && count) return fail(SV_EINVAL, "host_in is NULL");
  const uint64_t len = (uint64_t)1 << s->n;
  if (start > len || count > len - start) return fail(SV_EINVAL, "amplitude range out of bounds");
  SV_GUARD_BEGIN
  SV_HIP(hipSetDevice(s->device));
  const uint64_t chunk = (uint64_t)1 << 26;
  for (uint64_t done = 0; done < count; done += chunk) {
    const uint64_t c = std::min(chunk, count - done);
    SV_HIP(hipMemcpyAsync((float*)s->psi + 2 * (start + done), host_in + 2 * done, c * 8, hipMemcpyHostToDevice,
                          s->stream));
  }
  SV_HIP(hipStreamSynchronize(s->stream));
  if (count) s->norm_known = -1.0;
  return SV_OK;
  SV_GUARD_END(s)
}

}  // extern "C"

// Accessors for the other translation units (batch, tuner).
namespace sv {
void* state_psi(sv_state* s) { return s->psi; }
int state_n(sv_state* s) { return s->n; }
hipStream_t state_stream(sv_state* s) { return s->stream; }
bool state_poisoned(sv_state* s) { return s->poisoned; }
void state_poison(sv_state* s) { s->poisoned = true; }
// After a batched run: a circuit with a gate that is not unitary leaves the
// state's norm unknown to the host.
void state_note_gates(sv_state* s, const sv_gate* g, size_t n) {
  if (!gates_unitary(g, n)) s->norm_known = -1.0;
}
}  // namespace sv
