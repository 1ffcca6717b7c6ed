// Learned fusion: the installed MLP predicts the time of one pass from
// (k, target mask, n, precision); the partition search scores candidate
// partitions with it and keeps the cheapest.  Without a model every pass is
// priced the same, so the candidate with the fewest passes wins.
//
// Prediction target: ln(pass seconds * 1e9 / 2^n), i.e. the log of the pass
// time per amplitude in nanoseconds, which stays comparable across state
// sizes.  A pass costs exp(pred) * 2^n ns plus a fixed launch overhead.
//
// Candidates (Sec. IV-D: the best fusion size depends on circuit and
// platform, Sec. VII-B picks it by measurement):
//   - greedy max-k partitions for k = 1 .. max_k;
//   - largest-block partitions for k = max_k and max_k - 1;
//   - cost-aware greedy: a gate that would grow a block joins only when the
//     predicted cost of the larger block does not exceed the smaller block's
//     cost plus alpha times the cost of running the gate as a pass of its own,
//     for several alpha.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <exception>
#include <fstream>
#include <functional>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "sv_internal.h"

namespace sv {

void greedy_partition(const sv_gate* g, size_t n, int max_k, std::vector<std::vector<int>>& blocks);
void greedy_partition_cost(const sv_gate* g, size_t n, int max_k,
                           const std::function<bool(uint64_t, uint64_t, uint64_t)>& accept,
                           std::vector<std::vector<int>>& blocks);

namespace {

constexpr int F = SV_COST_FEATURES;
constexpr double kLaunchOverheadNs = 4000.0;
// beam searches over largest-block passes: partial partitions kept per pass
// (two widths; the search is not monotone in it), candidate sets tried per
// partial partition, and the largest circuit searched
constexpr int kBeamWidths[2] = {32, 64};
constexpr int kBeamMoves = 8;
constexpr size_t kBeamMaxGates = (size_t)1 << 14;
// predicted saving a partition with more passes needs over the fewest-pass one
constexpr double kFewerPassMargin = 0.05;

std::mutex g_mu;
std::vector<float> g_params;
int g_width = 0;

int num_params(int w) { return w * F + w + w * w + w + w + 1; }

double forward(const std::vector<float>& P, int W, const float* x) {
  const float* W1 = P.data();
  const float* b1 = W1 + W * F;
  const float* W2 = b1 + W;
  const float* b2 = W2 + W * W;
  const float* W3 = b2 + W;
  const float* b3 = W3 + W;
  std::vector<double> h1(W), h2(W);
  for (int j = 0; j < W; ++j) {
    double a = b1[j];
    for (int f = 0; f < F; ++f) a += (double)W1[j * F + f] * x[f];
    h1[j] = a > 0 ? a : 0;
  }
  for (int j = 0; j < W; ++j) {
    double a = b2[j];
    for (int q = 0; q < W; ++q) a += (double)W2[j * W + q] * h1[q];
    h2[j] = a > 0 ? a : 0;
  }
  double y = b3[0];
  for (int q = 0; q < W; ++q) y += (double)W3[q] * h2[q];
  return y;
}

}  // namespace

void cost_features(int k, const int* qubits, int n, int precision, float* out) {
  for (int i = 0; i < F; ++i) out[i] = 0.f;
  out[0] = k / 6.0f;
  out[1] = n / 34.0f;
  for (int j = 0; j < k; ++j)
    if (qubits[j] >= 0 && qubits[j] < 34) out[2 + qubits[j]] = 1.f;
  if (precision >= 0 && precision < 4) out[36 + precision] = 1.f;
}

void cost_model_set(const std::vector<float>& params, int width) {
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_params = params;
    g_width = width;
  }
  bump_plan_epoch();
}

bool cost_model_ready() {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_width > 0 && (int)g_params.size() == num_params(g_width);
}

double cost_model_predict_log(int k, const int* qubits, int n, int precision) {
  float x[F];
  cost_features(k, qubits, n, precision, x);
  std::lock_guard<std::mutex> lk(g_mu);
  return forward(g_params, g_width, x);
}

bool fuse_learned(const sv_gate* g, size_t n, int n_qubits, int max_k, int precision, std::vector<FusedGate>& out,
                  std::vector<int32_t>& block_of, int max_ctrl) {
  // Without a model every pass costs the same (it moves the same bytes): the
  // search then keeps the candidate with the fewest passes.
  const bool model = cost_model_ready();
  std::unordered_map<uint64_t, double> cache;
  const double amps = std::ldexp(1.0, n_qubits);
  auto pass_ns = [&](uint64_t mask) {
    if (!model) return 1.0;
    auto it = cache.find(mask);
    if (it != cache.end()) return it->second;
    int q[64], k = 0;
    for (int b = 0; b < 64 && k < SV_MAX_K; ++b)
      if ((mask >> b) & 1) q[k++] = b;
    const double t = std::exp(cost_model_predict_log(k, q, n_qubits, precision)) * amps + kLaunchOverheadNs;
    cache[mask] = t;
    return t;
  };
  auto mask_of = [&](int i) {
    uint64_t m = 0;
    for (int j = 0; j < g[i].k; ++j) m |= (uint64_t)1 << g[i].qubits[j];
    return m;
  };
  // a controlled pass of its own touches 2^-c of the state (c controls)
  auto ctrl_ns = [&](uint64_t targets, uint64_t cmask) {
    return pass_ns(targets) * std::ldexp(1.0, -__builtin_popcountll(cmask));
  };
  // A block with c controls sweeps the state once, in 2^c launches on its
  // targets, each over 2^-c of the state.
  auto total = [&](const std::vector<std::vector<int>>& blocks, int ctrl) {
    double t = 0;
    for (auto& b : blocks) {
      if (b.size() == 1 && g[b[0]].cmask) {
        t += ctrl_ns(mask_of(b[0]), g[b[0]].cmask);
        continue;
      }
      uint64_t S = 0, Cm = 0;
      if (ctrl > 0) {
        block_split(g, b, ctrl, S, Cm);
      } else {
        for (int i : b) S |= mask_of(i);
      }
      t += pass_ns(S) + (model ? ((1 << __builtin_popcountll(Cm)) - 1) * kLaunchOverheadNs : 0.0);
    }
    return t;
  };
  // The largest-block partitions and the phase partition take longest to
  // build; they are built on threads while the greedy candidates are scored.
  // (Inline, not on threads, when this search already runs on a pool worker.)
  const bool inline_only = host_pool_worker();
  struct Cand {
    std::vector<std::vector<int>> blocks;
    int ctrl = 0;  // controls a block may take
  };
  std::vector<Cand> blk;
  std::vector<std::thread> pool;
  std::vector<std::exception_ptr> errs;
  std::mutex err_mu;
  auto spawn = [&](std::function<void()> f) {
    if (inline_only) {
      f();
      return;
    }
    pool.emplace_back([f, &errs, &err_mu] {
      try {
        f();
      } catch (...) {  // carried back to the caller; an exception must not end a thread
        std::lock_guard<std::mutex> lk(err_mu);
        errs.push_back(std::current_exception());
      }
    });
  };
  // broad and narrow rule at max_k and max_k - 1, then (when controls are
  // allowed) both rules at max_k with controls, then the beam searches, with
  // controls when allowed (the beams without them found no fewer sweeps on
  // any workload tried and cost half the search time); sized before any
  // thread starts so that the slots never move
  const bool beam = n <= kBeamMaxGates;
  const int ctrl_rounds = max_ctrl > 0 ? 2 : 1;
  for (int r = 0; r < ctrl_rounds; ++r) {
    const int ctrl = r ? max_ctrl : 0;
    for (int K = max_k; K >= 1 && K >= max_k - (r ? 0 : 1); --K)
      for (int narrow = 0; narrow < 2; ++narrow) {
        blk.emplace_back();
        blk.back().ctrl = ctrl;
      }
    for (int w = 0; beam && r == ctrl_rounds - 1 && w < 2; ++w) {
      blk.emplace_back();
      blk.back().ctrl = ctrl;
    }
  }
  {
    size_t i = 0;
    for (int r = 0; r < ctrl_rounds; ++r) {
      const int ctrl = r ? max_ctrl : 0;
      for (int K = max_k; K >= 1 && K >= max_k - (r ? 0 : 1); --K)
        for (int narrow = 0; narrow < 2; ++narrow) {
          std::vector<std::vector<int>>* dst = &blk[i++].blocks;
          spawn([=] { maxblock_partition(g, n, K, narrow != 0, *dst, ctrl); });
        }
      for (int w = 0; beam && r == ctrl_rounds - 1 && w < 2; ++w) {  // beam searches at max_k
        std::vector<std::vector<int>>* dst = &blk[i++].blocks;
        const int width = kBeamWidths[w];
        spawn([=] { beam_partition(g, n, max_k, width, kBeamMoves, *dst, ctrl); });
      }
    }
  }
  std::vector<FusedGate> ph;
  std::vector<int32_t> ph_of;
  spawn([&] { fuse_phase(g, n, max_k, ph, ph_of); });
  struct Joiner {
    std::vector<std::thread>& p;
    ~Joiner() {
      for (auto& t : p)
        if (t.joinable()) t.join();
    }
  } joiner{pool};
  // The predicted-cheapest candidate and the candidate with the fewest passes
  // (the cheaper of those on ties) are both tracked; see the choice below.
  std::vector<std::vector<int>> best, fewest, cand;
  int best_ctrl = 0, fewest_ctrl = 0;
  double best_t = 1e300, fewest_t = 1e300;
  size_t fewest_n = SIZE_MAX;
  auto consider = [&](const std::vector<std::vector<int>>& c, int ctrl) {
    const double t = total(c, ctrl);
    if (t < best_t) {
      best_t = t;
      best = c;
      best_ctrl = ctrl;
    }
    if (c.size() < fewest_n || (c.size() == fewest_n && t < fewest_t)) {
      fewest_n = c.size();
      fewest_t = t;
      fewest = c;
      fewest_ctrl = ctrl;
    }
  };
  for (int K = 1; K <= max_k; ++K) {
    greedy_partition(g, n, K, cand);
    consider(cand, 0);
  }
  for (double alpha : {0.25, 0.5, 1.0}) {
    if (!model) break;  // the cost-aware variants need predicted times
    greedy_partition_cost(
        g, n, max_k,
        [&](uint64_t S, uint64_t S2, uint64_t qh) {
          if (S2 == S) return true;  // vertical fusion never costs a pass
          return pass_ns(S2) - pass_ns(S) <= alpha * pass_ns(qh);
        },
        cand);
    consider(cand, 0);
  }
  for (auto& t : pool) t.join();
  if (!errs.empty()) std::rethrow_exception(errs.front());
  for (auto& b : blk) consider(b.blocks, b.ctrl);  // largest-block partitions, in the order they were started
  // The phase-block partition: each run of phase gates is one elementwise
  // sweep, priced as a one-qubit pass on the top qubit (same traffic, no gather).
  double t_ph = 0;
  size_t n_ph = 0;
  bool in_run = false;
  for (const FusedGate& f : ph) {
    if (!f.cmask && is_phase_matrix(f.k, f.mat.data())) {
      if (!in_run) {
        t_ph += pass_ns((uint64_t)1 << (n_qubits - 1));
        ++n_ph;
      }
      in_run = true;
    } else {
      in_run = false;
      uint64_t m = 0;
      for (int j = 0; j < f.k; ++j) m |= (uint64_t)1 << f.q[j];
      t_ph += f.cmask ? ctrl_ns(m, f.cmask) : pass_ns(m);
      ++n_ph;
    }
  }
  // Every pass moves the whole state, so a partition with more passes is only
  // taken when the model predicts it clearly cheaper than the fewest-pass one:
  // the argmin over many candidates otherwise tends to pick the one whose
  // passes the model happens to under-predict.
  const bool phase_best = t_ph < best_t;
  const double chosen_t = phase_best ? t_ph : best_t;
  const size_t chosen_n = phase_best ? n_ph : best.size();
  const bool phase_fewest = n_ph < fewest_n || (n_ph == fewest_n && t_ph < fewest_t);
  if (phase_fewest) {
    fewest_n = n_ph;
    fewest_t = t_ph;
  }
  const bool keep_fewest = model && chosen_n > fewest_n && chosen_t > (1.0 - kFewerPassMargin) * fewest_t;
  const bool use_phase = keep_fewest ? phase_fewest : phase_best;
  if (use_phase) {
    out = std::move(ph);
    block_of = std::move(ph_of);
    return true;
  }
  if (keep_fewest) {
    best.swap(fewest);
    best_ctrl = fewest_ctrl;
  }
  fuse_blocks(g, n, best, out, block_of, best_ctrl);
  return true;
}

}  // namespace sv

using namespace sv;

// File: "SVCM" magic, u32 version 1, u32 width, u32 features, u32 count,
// then count little-endian float32 parameters.
extern "C" {

int sv_cost_model_save(const char* path) {
  return host_guard([&]() -> int {
    if (!path) return fail(SV_EINVAL, "path is NULL");
    std::vector<float> p;
    int w;
    {
      std::lock_guard<std::mutex> lk(g_mu);
      p = g_params;
      w = g_width;
    }
    if (w == 0) return fail(SV_EINVAL, "no cost model installed");
    std::ofstream f(path, std::ios::binary);
    if (!f) return fail(SV_EINVAL, std::string("cannot write ") + path);
    const uint32_t hdr[5] = {0x4D435653u, 1u, (uint32_t)w, (uint32_t)F, (uint32_t)p.size()};
    f.write((const char*)hdr, sizeof(hdr));
    f.write((const char*)p.data(), sizeof(float) * p.size());
    return f ? SV_OK : fail(SV_EINVAL, "write failed");
  });
}

int sv_cost_model_load(const char* path) {
  return host_guard([&]() -> int {
    if (!path) return fail(SV_EINVAL, "path is NULL");
    std::ifstream f(path, std::ios::binary);
    if (!f) return fail(SV_EINVAL, std::string("cannot read ") + path);
    uint32_t hdr[5];
    if (!f.read((char*)hdr, sizeof(hdr))) return fail(SV_EINVAL, "truncated cost model file");
    if (hdr[0] != 0x4D435653u || hdr[1] != 1u) return fail(SV_EINVAL, "not a cost model file");
    if (hdr[2] != 64 || hdr[3] != (uint32_t)F || hdr[4] != (uint32_t)num_params((int)hdr[2]))
      return fail(SV_EINVAL, "cost model shape mismatch");
    std::vector<float> p(hdr[4]);
    if (!f.read((char*)p.data(), sizeof(float) * p.size())) return fail(SV_EINVAL, "truncated cost model file");
    for (float v : p)
      if (!std::isfinite(v)) return fail(SV_EINVAL, "non-finite parameter");
    cost_model_set(p, (int)hdr[2]);
    return SV_OK;
  });
}

int sv_cost_model_clear(void) {
  return host_guard([&]() -> int {
    cost_model_set(std::vector<float>(), 0);
    return SV_OK;
  });
}

int sv_cost_model_predict(int k, const int32_t* qubits, int n_qubits, int precision, double* out) {
  return host_guard([&]() -> int {
    if (!qubits || !out || k < 1 || k > SV_MAX_K || n_qubits < 1 || n_qubits > SV_MAX_QUBITS)
      return fail(SV_EINVAL, "bad arguments");
    if (!cost_model_ready()) return fail(SV_EINVAL, "no cost model installed");
    int q[SV_MAX_K];
    for (int j = 0; j < k; ++j) q[j] = qubits[j];
    *out = cost_model_predict_log(k, q, n_qubits, precision);
    return SV_OK;
  });
}

int sv_cost_features(int k, const int32_t* qubits, int n_qubits, int precision, float* out) {
  return host_guard([&]() -> int {
    if (!qubits || !out || k < 1 || k > SV_MAX_K) return fail(SV_EINVAL, "bad arguments");
    int q[SV_MAX_K];
    for (int j = 0; j < k; ++j) q[j] = qubits[j];
    cost_features(k, q, n_qubits, precision, out);
    return SV_OK;
  });
}

}  // extern "C"
