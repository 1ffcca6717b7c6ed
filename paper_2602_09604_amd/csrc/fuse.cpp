// Gate fusion on the host in FP64 (Sec. II-C, Sec. IV-D).
//
// Vertical fusion multiplies gates on the same qubits; horizontal fusion
// takes the tensor product of gates on disjoint qubits (Eq. 3).  Both come
// out of one rule: a block is an ordered list of gates whose qubit union has
// at most max_k qubits, and its matrix is the ordered product of its gates,
// each lifted to the block's qubits.
//
// Greedy partition: seed a block with the earliest unconsumed gate and scan
// forward.  A later gate joins when the union stays within max_k qubits and
// none of its qubits is "blocked"; a gate that cannot join blocks all of its
// qubits, because every later gate that touches them must stay behind it.
// A joined gate therefore commutes with every skipped gate before it (they
// share no qubit), so emitting the block at the seed's position and the
// skipped gates after it preserves the circuit's action.
//
// Controlled gates (Eq. 4's indicator 1_c): one whose targets and controls
// fit in max_k qubits is lifted to a dense gate on their union and fused like
// any other; a wider one stays a block of its own (a controlled pass) and
// blocks all of its qubits, controls included, for every other block.
#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstring>
#include <exception>
#include <functional>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <thread>
#include <unordered_map>

#include "sv_internal.h"

namespace sv {

int validate_gates(const sv_gate* g, size_t n, int n_qubits) {
  if (n > 0 && !g) return fail(SV_EINVAL, "gates is NULL");
  for (size_t i = 0; i < n; ++i) {
    const int k = g[i].k;
    if (k < 1 || k > SV_MAX_K || k > n_qubits)
      return fail(SV_EINVAL, "gate " + std::to_string(i) + ": k=" + std::to_string(k) +
                                 " outside 1..min(6, n)");
    if (!g[i].matrix) return fail(SV_EINVAL, "gate " + std::to_string(i) + ": matrix is NULL");
    for (int j = 0; j < k; ++j) {
      const int q = g[i].qubits[j];
      if (q < 0 || q >= n_qubits)
        return fail(SV_EINVAL, "gate " + std::to_string(i) + ": qubit " + std::to_string(q) +
                                   " out of range");
      for (int a = 0; a < j; ++a)
        if (g[i].qubits[a] == q)
          return fail(SV_EINVAL, "gate " + std::to_string(i) + ": qubit " + std::to_string(q) +
                                     " repeated");
      if ((g[i].cmask >> q) & 1)
        return fail(SV_EINVAL, "gate " + std::to_string(i) + ": qubit " + std::to_string(q) +
                                   " is both a target and a control");
    }
    const uint64_t cm = g[i].cmask;
    if (n_qubits < 64 && (cm >> n_qubits) != 0)
      return fail(SV_EINVAL, "gate " + std::to_string(i) + ": control out of range");
    if ((g[i].cval & ~cm) != 0)
      return fail(SV_EINVAL, "gate " + std::to_string(i) + ": control value outside the control mask");
    if (k + __builtin_popcountll(cm) > n_qubits)
      return fail(SV_EINVAL, "gate " + std::to_string(i) + ": more targets and controls than qubits");
  }
  return SV_OK;
}

static uint64_t qmask(const sv_gate& g) { return gate_span(g); }

namespace {
thread_local bool t_pool_worker = false;
}
bool host_pool_worker() { return t_pool_worker; }
void set_host_pool_worker(bool on) { t_pool_worker = on; }

void lower_controlled(const sv_gate* g, size_t n, int max_k, std::vector<sv_gate>& out,
                      std::vector<std::vector<double>>& store) {
  out.assign(g, g + n);
  store.clear();
  size_t lifted = 0;
  for (size_t i = 0; i < n; ++i)
    if (g[i].cmask && g[i].k + __builtin_popcountll(g[i].cmask) <= std::min(max_k, SV_MAX_K)) ++lifted;
  store.reserve(lifted);
  for (size_t i = 0; i < n; ++i) {
    const sv_gate& src = g[i];
    const int nc = __builtin_popcountll(src.cmask);
    if (!src.cmask || src.k + nc > std::min(max_k, SV_MAX_K)) continue;
    // local bits 0..k-1: the targets as given; k..k+nc-1: the controls, ascending
    sv_gate d{};
    d.k = src.k + nc;
    std::copy(src.qubits, src.qubits + src.k, d.qubits);
    int cv = 0, j = src.k;
    for (int q = 0; q < 64; ++q)
      if ((src.cmask >> q) & 1) {
        if ((src.cval >> q) & 1) cv |= 1 << (j - src.k);
        d.qubits[j++] = q;
      }
    const int dt = 1 << src.k, D = 1 << d.k;
    std::vector<double> m((size_t)2 * D * D, 0.0);
    for (int hi = 0; hi < (1 << nc); ++hi)
      for (int r = 0; r < dt; ++r)
        for (int c = 0; c < dt; ++c) {
          const size_t e = (size_t)(hi * dt + r) * D + (hi * dt + c);
          if (hi == cv) {
            m[2 * e] = src.matrix[2 * (r * dt + c)];
            m[2 * e + 1] = src.matrix[2 * (r * dt + c) + 1];
          } else if (r == c) {
            m[2 * e] = 1.0;
          }
        }
    store.push_back(std::move(m));
    d.matrix = store.back().data();
    out[i] = d;
  }
}

// M <- G M, where M is the 2^K x 2^K block matrix (row-major, real and
// imaginary parts held apart) and G acts on block-local bits pos[0..k-1]
// (local bit j of G = block bit pos[j]).  The rows of M that differ only in
// G's bits are combined whole, so the inner loop runs over contiguous columns.
static void left_multiply(std::vector<double>& Mr, std::vector<double>& Mi, int K, const sv_gate& g,
                          const int* pos) {
  const int d = 1 << K, k = g.k, dk = 1 << k;
  int sorted[SV_MAX_K];
  std::copy(pos, pos + k, sorted);
  std::sort(sorted, sorted + k);
  int off[1 << SV_MAX_K];
  for (int l = 0; l < dk; ++l) {
    int o = 0;
    for (int j = 0; j < k; ++j)
      if ((l >> j) & 1) o |= 1 << pos[j];
    off[l] = o;
  }
  std::vector<double> tr((size_t)dk * d), ti((size_t)dk * d);
  for (int grp = 0; grp < (d >> k); ++grp) {
    int base = grp;
    for (int j = 0; j < k; ++j) {
      const int lm = (1 << sorted[j]) - 1;
      base = ((base & ~lm) << 1) | (base & lm);
    }
    std::fill(tr.begin(), tr.end(), 0.0);
    std::fill(ti.begin(), ti.end(), 0.0);
    for (int r = 0; r < dk; ++r) {
      double* __restrict__ orr = tr.data() + (size_t)r * d;
      double* __restrict__ ori = ti.data() + (size_t)r * d;
      for (int c = 0; c < dk; ++c) {
        const double a = g.matrix[2 * (r * dk + c)], bb = g.matrix[2 * (r * dk + c) + 1];
        const double* __restrict__ xr = Mr.data() + (size_t)(base + off[c]) * d;
        const double* __restrict__ xi = Mi.data() + (size_t)(base + off[c]) * d;
        for (int col = 0; col < d; ++col) {
          orr[col] += a * xr[col] - bb * xi[col];
          ori[col] += a * xi[col] + bb * xr[col];
        }
      }
    }
    for (int r = 0; r < dk; ++r) {
      std::copy(tr.begin() + (size_t)r * d, tr.begin() + (size_t)(r + 1) * d, Mr.begin() + (size_t)(base + off[r]) * d);
      std::copy(ti.begin() + (size_t)r * d, ti.begin() + (size_t)(r + 1) * d, Mi.begin() + (size_t)(base + off[r]) * d);
    }
  }
}

// Build the fused gate of an ordered member list.
static void build_block(const sv_gate* g, const std::vector<int>& members, FusedGate& out) {
  if (members.size() == 1 && g[members[0]].cmask) {  // a controlled pass of its own
    const sv_gate& c = g[members[0]];
    out.k = c.k;
    normalise_gate(c.k, c.qubits, c.matrix, out.q, out.mat);
    out.cmask = c.cmask;
    out.cval = c.cval;
    return;
  }
  uint64_t S = 0;
  for (int i : members) S |= qmask(g[i]);
  int K = 0;
  int bitpos[64];
  for (int q = 0; q < 64; ++q)
    if ((S >> q) & 1) {
      bitpos[q] = K;
      out.q[K++] = q;
    }
  out.k = K;
  const int d = 1 << K;
  std::vector<double> Mr((size_t)d * d, 0.0), Mi((size_t)d * d, 0.0);
  for (int i = 0; i < d; ++i) Mr[(size_t)i * d + i] = 1.0;
  for (int i : members) {
    int pos[SV_MAX_K];
    for (int j = 0; j < g[i].k; ++j) pos[j] = bitpos[g[i].qubits[j]];
    left_multiply(Mr, Mi, K, g[i], pos);
  }
  out.mat.resize((size_t)2 * d * d);
  for (size_t i = 0; i < (size_t)d * d; ++i) {
    out.mat[2 * i] = Mr[i];
    out.mat[2 * i + 1] = Mi[i];
  }
}

bool is_diagonal_gate(const sv_gate& g) {
  if (g.cmask) return false;
  const int d = 1 << g.k;
  for (int r = 0; r < d; ++r)
    for (int c = 0; c < d; ++c)
      if (r != c && (g.matrix[2 * (r * d + c)] != 0.0 || g.matrix[2 * (r * d + c) + 1] != 0.0)) return false;
  return true;
}

void block_split(const sv_gate* g, const std::vector<int>& members, int max_ctrl, uint64_t& targets,
                 uint64_t& controls) {
  uint64_t all = 0, dense = 0;
  for (int i : members) {
    all |= qmask(g[i]);
    if (max_ctrl > 0 && !is_diagonal_gate(g[i])) dense |= qmask(g[i]);
  }
  controls = 0;
  if (max_ctrl > 0 && !(members.size() == 1 && g[members[0]].cmask)) {
    uint64_t cand = all & ~dense & ~kCtrlLowBits;
    for (int b = 63; b >= 0 && __builtin_popcountll(controls) < max_ctrl; --b)
      if ((cand >> b) & 1) controls |= (uint64_t)1 << b;
    if (controls == all) controls &= controls - 1;  // keep the lowest as the target
  }
  targets = all & ~controls;
}

// The fused gates of one block: one dense gate, or with controls one gate per
// control value v, each the ordered product of the members with every
// diagonal member that reaches a control restricted to the control bits of v
// (a diagonal gate on its target part, or a phase when it has none there).
static void build_block_mux(const sv_gate* g, const std::vector<int>& members, int max_ctrl,
                            std::vector<FusedGate>& outs) {
  uint64_t S = 0, Cm = 0;
  block_split(g, members, max_ctrl, S, Cm);
  outs.clear();
  if (Cm == 0) {
    outs.emplace_back();
    build_block(g, members, outs.back());
    return;
  }
  if (__builtin_popcountll(S) > SV_MAX_K) throw std::logic_error("block with controls wider than SV_MAX_K targets");
  int K = 0, bitpos[64], cbits[64], nc = 0;
  int q[SV_MAX_K];
  for (int b = 0; b < 64; ++b) {
    if ((S >> b) & 1) {
      bitpos[b] = K;
      q[K++] = b;
    }
    if ((Cm >> b) & 1) cbits[nc++] = b;
  }
  const int d = 1 << K;
  std::vector<double> Mr, Mi, dmat;
  for (int v = 0; v < (1 << nc); ++v) {
    uint64_t cval = 0;
    for (int t = 0; t < nc; ++t)
      if ((v >> t) & 1) cval |= (uint64_t)1 << cbits[t];
    Mr.assign((size_t)d * d, 0.0);
    Mi.assign((size_t)d * d, 0.0);
    for (int i = 0; i < d; ++i) Mr[(size_t)i * d + i] = 1.0;
    for (int i : members) {
      const sv_gate& h = g[i];
      int pos[SV_MAX_K];
      if ((qmask(h) & Cm) == 0) {
        for (int j = 0; j < h.k; ++j) pos[j] = bitpos[h.qubits[j]];
        left_multiply(Mr, Mi, K, h, pos);
        continue;
      }
      // diagonal member reaching controls: its entries with the control bits fixed
      const int dk = 1 << h.k;
      int tj[SV_MAX_K], nt = 0, fixed = 0;
      for (int j = 0; j < h.k; ++j) {
        const int b = h.qubits[j];
        if ((Cm >> b) & 1) {
          if ((cval >> b) & 1) fixed |= 1 << j;
        } else {
          tj[nt] = j;
          pos[nt++] = bitpos[b];
        }
      }
      const int dr = 1 << nt;
      dmat.assign((size_t)2 * dr * dr, 0.0);
      for (int r = 0; r < dr; ++r) {
        int l = fixed;
        for (int t = 0; t < nt; ++t)
          if ((r >> t) & 1) l |= 1 << tj[t];
        dmat[2 * ((size_t)r * dr + r)] = h.matrix[2 * ((size_t)l * dk + l)];
        dmat[2 * ((size_t)r * dr + r) + 1] = h.matrix[2 * ((size_t)l * dk + l) + 1];
      }
      if (nt == 0) {  // a phase for this control value
        const double pr = dmat[0], pi = dmat[1];
        for (size_t e = 0; e < (size_t)d * d; ++e) {
          const double xr = Mr[e], xi = Mi[e];
          Mr[e] = pr * xr - pi * xi;
          Mi[e] = pr * xi + pi * xr;
        }
        continue;
      }
      sv_gate rg{};
      rg.k = nt;
      for (int t = 0; t < nt; ++t) rg.qubits[t] = h.qubits[tj[t]];
      rg.matrix = dmat.data();
      left_multiply(Mr, Mi, K, rg, pos);
    }
    FusedGate f;
    f.k = K;
    std::copy(q, q + K, f.q);
    f.mat.resize((size_t)2 * d * d);
    for (size_t e = 0; e < (size_t)d * d; ++e) {
      f.mat[2 * e] = Mr[e];
      f.mat[2 * e + 1] = Mi[e];
    }
    f.cmask = Cm;
    f.cval = cval;
    outs.push_back(std::move(f));
  }
}

void fuse_none(const sv_gate* g, size_t n, std::vector<FusedGate>& out, std::vector<int32_t>& block_of) {
  out.clear();
  out.reserve(n);
  block_of.assign(n, 0);
  for (size_t i = 0; i < n; ++i) {
    FusedGate f;
    f.k = g[i].k;
    normalise_gate(g[i].k, g[i].qubits, g[i].matrix, f.q, f.mat);
    f.cmask = g[i].cmask;
    f.cval = g[i].cval;
    out.push_back(std::move(f));
    block_of[i] = (int32_t)i;
  }
}

// Greedy partition into member lists (indices into g), blocks in emission
// order.  accept(S, S_new, q) may veto a join that passes the size and
// blocking rules (S = block qubits now, S_new = after the join, q = the
// gate's qubits); a vetoed gate blocks its qubits like any other skipped gate.
void greedy_partition_cost(const sv_gate* g, size_t n, int max_k,
                           const std::function<bool(uint64_t, uint64_t, uint64_t)>& accept,
                           std::vector<std::vector<int>>& blocks) {
  blocks.clear();
  std::vector<uint64_t> masks(n);
  uint64_t all = 0;
  for (size_t i = 0; i < n; ++i) all |= masks[i] = qmask(g[i]);
  std::vector<char> consumed(n, 0);
  for (size_t seed = 0; seed < n; ++seed) {
    if (consumed[seed]) continue;
    std::vector<int> members{(int)seed};
    consumed[seed] = 1;
    if (g[seed].cmask) {  // a remaining controlled gate is a block of its own
      blocks.push_back(std::move(members));
      continue;
    }
    uint64_t S = masks[seed], blocked = 0;
    for (size_t h = seed + 1; h < n; ++h) {
      if (consumed[h]) continue;
      const uint64_t qh = masks[h];
      const uint64_t S2 = S | qh;
      if (!g[h].cmask && (qh & blocked) == 0 && __builtin_popcountll(S2) <= max_k &&
          (!accept || accept(S, S2, qh))) {
        S = S2;
        members.push_back((int)h);
        consumed[h] = 1;
      } else {
        blocked |= qh;
      }
      // no later gate can join once the block is full and all its qubits are
      // blocked, or once every qubit of the circuit is blocked
      if ((__builtin_popcountll(S) >= max_k && (S & ~blocked) == 0) || (all & ~blocked) == 0) break;
    }
    blocks.push_back(std::move(members));
  }
}

void greedy_partition(const sv_gate* g, size_t n, int max_k, std::vector<std::vector<int>>& blocks) {
  greedy_partition_cost(g, n, max_k, nullptr, blocks);
}

// Largest-block partition.  Greedy in passes rather than in gates: each pass
// takes the qubit set S (at most max_k qubits) that absorbs the most gates.
// A gate is absorbed when its qubits lie in S and no earlier gate left for a
// later pass shares a qubit with it (the same blocking rule as above, so
// absorbed gates commute with everything they skip).  Candidate sets grow
// from each gate of the current front: at every step the qubits of one gate
// that touches S are added, choosing the addition that absorbs the most gates
// (fewer qubits on ties), until no addition fits; the best set seen along the
// way is kept.  Additions come from the outside qubits of gates that touch S
// (all of them, or with `narrow` only those whose qubits in S are not yet
// blocked) and from every other gate of the front (horizontal fusion).  A
// remaining controlled gate is a pass of its own as soon as it reaches the
// front.
// Absorbed-gate counts of one search step, keyed by the qubit set (never
// 0): open addressing with linear probing, emptied by advancing a stamp, so
// the thousands of lookups per step neither allocate nor rehash often.
class CountMemo {
 public:
  template <class Eval>
  int get(uint64_t S, Eval&& eval) {
    if (2 * (used_ + 1) > key_.size()) grow();
    size_t i = slot(S);
    while (stamp_[i] == gen_) {
      if (key_[i] == S) return val_[i];
      i = (i + 1) & (key_.size() - 1);
    }
    const int c = eval(S);
    stamp_[i] = gen_;
    key_[i] = S;
    val_[i] = c;
    ++used_;
    return c;
  }
  void clear() {
    used_ = 0;
    if (++gen_ == 0) {  // the stamp wrapped: forget every slot explicitly
      std::fill(stamp_.begin(), stamp_.end(), 0u);
      gen_ = 1;
    }
  }
  size_t size() const { return used_; }
  template <class F>
  void for_each(F&& f) const {
    for (size_t i = 0; i < key_.size(); ++i)
      if (stamp_[i] == gen_) f(key_[i], val_[i]);
  }

 private:
  size_t slot(uint64_t x) const {
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    return (size_t)x & (key_.size() - 1);
  }
  void grow() {
    std::vector<uint64_t> k;
    std::vector<int> v;
    for_each([&](uint64_t a, int b) {
      k.push_back(a);
      v.push_back(b);
    });
    const size_t cap = std::max<size_t>(1024, 2 * key_.size());
    key_.assign(cap, 0);
    val_.assign(cap, 0);
    stamp_.assign(cap, 0u);
    gen_ = 1;
    used_ = 0;
    for (size_t j = 0; j < k.size(); ++j) {
      size_t i = slot(k[j]);
      while (stamp_[i] == gen_) i = (i + 1) & (cap - 1);
      stamp_[i] = gen_;
      key_[i] = k[j];
      val_[i] = v[j];
      ++used_;
    }
  }
  std::vector<uint64_t> key_;
  std::vector<int> val_;
  std::vector<uint32_t> stamp_;
  size_t used_ = 0;
  uint32_t gen_ = 1;
};

namespace {
struct BlockSearch {
  const sv_gate* g;
  std::vector<uint64_t> masks;
  std::vector<char> diag;  // diagonal gates (candidates for control absorption)
  std::vector<int> live;   // indices of gates not yet emitted, in order
  // the qubit masks and kinds of the live gates, in live order: the scans
  // below read these two arrays front to back instead of the gate structs
  std::vector<uint64_t> live_mask;
  std::vector<unsigned char> live_kind;
  static constexpr unsigned char kControlled = 1, kDiagonal = 2;

  // Gates absorbed by S (indices into g, in order); optionally the candidate
  // qubit additions seen before S is fully blocked.
  bool narrow = false;  // additions only from gates whose qubits in S are not yet blocked
  // With max_ctrl > 0 a diagonal gate that touches S may also reach up to
  // max_ctrl qubits outside S (at or above kCtrlMinBit): those become control
  // bits of the pass, which then applies one matrix per control value.
  int max_ctrl = 0;
  CountMemo memo;  // scratch for the beam steps run on this search

  // refresh live_mask / live_kind after live changed
  void sync_live() {
    live_mask.resize(live.size());
    live_kind.resize(live.size());
    for (size_t i = 0; i < live.size(); ++i) {
      const int h = live[i];
      live_mask[i] = masks[h];
      live_kind[i] = (g[h].cmask ? kControlled : 0) | (diag[h] ? kDiagonal : 0);
    }
  }

  int absorb(uint64_t S, std::vector<int>* got, std::vector<uint64_t>* adds) const {
    uint64_t blocked = 0, ctrl = 0;
    int count = 0;
    const size_t L = live.size();
    const uint64_t* lm = live_mask.data();
    const unsigned char* lk = live_kind.data();
    for (size_t i = 0; i < L; ++i) {
      if ((S & ~blocked) == 0) break;  // every qubit of S is blocked: nothing more can join
      const uint64_t qh = lm[i];
      const unsigned kind = lk[i];
      if ((qh & blocked) == 0 && !(kind & kControlled)) {
        const uint64_t out = qh & ~S;
        if (out == 0 || (max_ctrl > 0 && (kind & kDiagonal) && (qh & S) && (out & kCtrlLowBits) == 0 &&
                         __builtin_popcountll(ctrl | out) <= max_ctrl)) {
          ctrl |= out;
          ++count;
          if (got) got->push_back(live[i]);
          continue;
        }
      }
      if (adds && !(kind & kControlled) && (qh & S & (narrow ? ~blocked : ~(uint64_t)0)) && (qh & ~S))
        adds->push_back(qh & ~S);
      blocked |= qh;
    }
    return count;
  }
};
}  // namespace

namespace {
// The first remaining gate on each of its qubits.
std::vector<int> front_of(const BlockSearch& b) {
  std::vector<int> front;
  uint64_t blocked = 0;
  for (size_t i = 0; i < b.live.size(); ++i) {
    if ((b.live_mask[i] & blocked) == 0) front.push_back(b.live[i]);
    blocked |= b.live_mask[i];
  }
  return front;
}

// Grow a candidate set from front gate f (the growth described above);
// returns the best (count, set) seen along the way.  count_of evaluates and
// memoises absorbed-gate counts.
template <class CountOf>
std::pair<int, uint64_t> grow_from(const BlockSearch& b, const std::vector<int>& front, int f, int max_k,
                                   CountOf&& count_of, std::vector<uint64_t>& adds) {
  uint64_t S = b.masks[f];
  int seen = count_of(S);
  uint64_t seen_S = S;
  while (true) {
    // additions: the outside qubits of a gate that touches S, or a whole
    // front gate elsewhere (horizontal fusion)
    adds.clear();
    b.absorb(S, nullptr, &adds);
    for (int f2 : front)
      if (!b.g[f2].cmask && (b.masks[f2] & ~S)) adds.push_back(b.masks[f2] & ~S);
    std::sort(adds.begin(), adds.end());
    adds.erase(std::unique(adds.begin(), adds.end()), adds.end());
    int step_count = -1, step_bits = 0;
    uint64_t step_S = 0;
    for (uint64_t add : adds) {
      const uint64_t S2 = S | add;
      const int bits = __builtin_popcountll(S2);
      if (bits > max_k) continue;
      const int c = count_of(S2);
      if (c > step_count || (c == step_count && bits < step_bits)) {
        step_count = c;
        step_bits = bits;
        step_S = S2;
      }
    }
    if (step_count < 0) break;
    S = step_S;
    if (step_count > seen) {
      seen = step_count;
      seen_S = S;
    }
  }
  return {seen, seen_S};
}

void init_search(BlockSearch& b, const sv_gate* g, size_t n, int max_ctrl) {
  b.g = g;
  b.max_ctrl = max_ctrl;
  b.masks.resize(n);
  b.diag.assign(n, 0);
  b.live.clear();
  for (size_t i = 0; i < n; ++i) {
    b.masks[i] = qmask(g[i]);
    if (max_ctrl > 0) b.diag[i] = is_diagonal_gate(g[i]);
    b.live.push_back((int)i);
  }
  b.sync_live();
}
}  // namespace

void maxblock_partition(const sv_gate* g, size_t n, int max_k, bool narrow, std::vector<std::vector<int>>& blocks,
                        int max_ctrl) {
  blocks.clear();
  BlockSearch b;
  init_search(b, g, n, max_ctrl);
  b.narrow = narrow;
  std::vector<char> done(n, 0);
  std::vector<uint64_t> adds;
  CountMemo memo;
  while (!b.live.empty()) {
    const std::vector<int> front = front_of(b);
    std::vector<int> chosen;
    for (int f : front)
      if (g[f].cmask) {  // a wide controlled gate: its own pass
        chosen.push_back(f);
        break;
      }
    if (chosen.empty()) {
      int best_count = -1;
      uint64_t best_S = 0;
      memo.clear();  // absorbed-gate counts of this pass
      auto count_of = [&](uint64_t S) {
        return memo.get(S, [&](uint64_t T) { return b.absorb(T, nullptr, nullptr); });
      };
      for (int f : front) {
        if (g[f].cmask) continue;
        const auto r = grow_from(b, front, f, max_k, count_of, adds);
        if (r.first > best_count) {
          best_count = r.first;
          best_S = r.second;
        }
      }
      b.absorb(best_S, &chosen, nullptr);
    }
    for (int h : chosen) done[h] = 1;
    std::vector<int> rest;
    rest.reserve(b.live.size() - chosen.size());
    for (int h : b.live)
      if (!done[h]) rest.push_back(h);
    b.live.swap(rest);
    b.sync_live();
    blocks.push_back(std::move(chosen));
  }
}

// Beam search over largest-block passes.  A partial partition is ranked by
// the gates it leaves; each one is extended by the `topm` sets that absorb the
// most gates among all the sets the growth search evaluates (more absorbed
// first, then fewer qubits, then the smaller mask), and after every pass the
// `width` best distinct partial partitions are kept.  The first to absorb the
// whole circuit is returned, so it has the fewest passes the beam found.  The
// partial partitions of a pass are extended on host threads; the result does
// not depend on how many.
namespace {
struct BeamChain {  // the passes of a partial partition, last first
  std::vector<int> block;
  std::shared_ptr<const BeamChain> prev;
};
struct BeamNode {
  std::vector<int> live;
  std::shared_ptr<const BeamChain> passes;
};

void beam_expand(BlockSearch& b, const BeamNode& nd, int max_k, int topm, std::vector<uint64_t>& adds,
                 std::vector<char>& taken, std::vector<BeamNode>& kids) {
  b.live = nd.live;
  b.sync_live();
  const std::vector<int> front = front_of(b);
  std::vector<uint64_t> moves;  // candidate sets; 0 stands for a controlled front gate
  int ctrl = -1;
  for (int f : front)
    if (b.g[f].cmask) {
      ctrl = f;
      break;
    }
  if (ctrl < 0) {
    CountMemo& memo = b.memo;
    memo.clear();
    auto count_of = [&](uint64_t S) {
      return memo.get(S, [&](uint64_t T) { return b.absorb(T, nullptr, nullptr); });
    };
    for (int f : front) (void)grow_from(b, front, f, max_k, count_of, adds);
    std::vector<std::pair<int, uint64_t>> ranked;
    ranked.reserve(memo.size());
    memo.for_each([&](uint64_t S, int c) { ranked.push_back({c, S}); });
    // the topm best in the total order below (count, then size, then mask)
    const size_t top = std::min(ranked.size(), (size_t)topm);
    std::partial_sort(ranked.begin(), ranked.begin() + top, ranked.end(), [](const std::pair<int, uint64_t>& x, const std::pair<int, uint64_t>& y) {
      if (x.first != y.first) return x.first > y.first;
      const int bx = __builtin_popcountll(x.second), by = __builtin_popcountll(y.second);
      if (bx != by) return bx < by;
      return x.second < y.second;
    });
    for (size_t i = 0; i < top; ++i)
      if (ranked[i].first > 0) moves.push_back(ranked[i].second);
  } else {
    moves.push_back(0);
  }
  for (uint64_t S : moves) {
    BeamNode child;
    std::vector<int> chosen;
    if (S == 0) chosen.push_back(ctrl);
    else b.absorb(S, &chosen, nullptr);
    for (int h : chosen) taken[h] = 1;
    child.live.reserve(b.live.size() - chosen.size());
    for (int h : b.live)
      if (!taken[h]) child.live.push_back(h);
    for (int h : chosen) taken[h] = 0;
    child.passes = std::make_shared<const BeamChain>(BeamChain{std::move(chosen), nd.passes});
    kids.push_back(std::move(child));
  }
}

// Host threads kept for a whole search: run() wakes every worker for one
// round of body(w) (the caller runs body(0)) and returns when all are done.
// body must not throw.
class RoundPool {
 public:
  RoundPool(unsigned threads, std::function<void(unsigned)> body) : body_(std::move(body)) {
    try {
      for (unsigned w = 1; w < threads; ++w) threads_.emplace_back([this, w] { loop(w); });
    } catch (...) {
      shutdown();
      throw;
    }
  }
  ~RoundPool() { shutdown(); }
  void run() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      ++round_;
      busy_ = (unsigned)threads_.size();
    }
    wake_.notify_all();
    body_(0);
    std::unique_lock<std::mutex> lk(mu_);
    idle_.wait(lk, [&] { return busy_ == 0; });
  }

 private:
  void loop(unsigned w) {
    uint64_t seen = 0;
    while (true) {
      {
        std::unique_lock<std::mutex> lk(mu_);
        wake_.wait(lk, [&] { return stop_ || round_ != seen; });
        if (stop_) return;
        seen = round_;
      }
      body_(w);
      std::lock_guard<std::mutex> lk(mu_);
      if (--busy_ == 0) idle_.notify_one();
    }
  }
  void shutdown() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    wake_.notify_all();
    for (auto& t : threads_) t.join();
    threads_.clear();
  }
  std::function<void(unsigned)> body_;
  std::vector<std::thread> threads_;
  std::mutex mu_;
  std::condition_variable wake_, idle_;
  uint64_t round_ = 0;
  unsigned busy_ = 0;
  bool stop_ = false;
};
}  // namespace

void beam_partition(const sv_gate* g, size_t n, int max_k, int width, int topm,
                    std::vector<std::vector<int>>& blocks, int max_ctrl) {
  blocks.clear();
  if (n == 0) return;
  width = std::max(width, 1);
  topm = std::max(topm, 1);
  BlockSearch proto;
  init_search(proto, g, n, max_ctrl);
  std::vector<BeamNode> beam(1);
  beam[0].live = proto.live;
  const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  const unsigned nt = host_pool_worker() ? 1u : (unsigned)std::min<size_t>(hw, width);
  std::vector<std::vector<BeamNode>> kids;
  std::atomic<size_t> next{0};
  std::vector<std::exception_ptr> errs(nt);
  std::vector<BlockSearch> search(nt, proto);
  RoundPool pool(nt, [&](unsigned w) {
    try {
      std::vector<uint64_t> adds;
      std::vector<char> taken(n, 0);
      for (size_t i = next++; i < beam.size(); i = next++)
        beam_expand(search[w], beam[i], max_k, topm, adds, taken, kids[i]);
    } catch (...) {  // carried back to the caller; an exception must not end a thread
      errs[w] = std::current_exception();
      next = beam.size();
    }
  });
  while (true) {
    kids.assign(beam.size(), {});
    next = 0;
    pool.run();
    for (auto& e : errs)
      if (e) std::rethrow_exception(e);
    std::vector<BeamNode> cand;
    for (auto& ks : kids)
      for (auto& c : ks) {
        if (c.live.empty()) {  // the first complete partition, in beam order
          for (const BeamChain* p = c.passes.get(); p; p = p->prev.get()) blocks.push_back(p->block);
          std::reverse(blocks.begin(), blocks.end());
          return;
        }
        cand.push_back(std::move(c));
      }
    std::stable_sort(cand.begin(), cand.end(),
                     [](const BeamNode& x, const BeamNode& y) { return x.live.size() < y.live.size(); });
    beam.clear();
    std::unordered_map<uint64_t, std::vector<size_t>> seen;  // hash of the remaining gates -> kept nodes
    for (BeamNode& c : cand) {
      if ((int)beam.size() >= width) break;
      uint64_t h = 1469598103934665603ull;
      for (int v : c.live) h = (h ^ (uint64_t)v) * 1099511628211ull;
      auto& bucket = seen[h];
      bool dup = false;
      for (size_t j : bucket)
        if (beam[j].live == c.live) {
          dup = true;
          break;
        }
      if (dup) continue;
      bucket.push_back(beam.size());
      beam.push_back(std::move(c));
    }
  }
}

// BLOCK fusion: the two candidate rules of the largest-block search, keeping
// the partition with fewer passes (the first on ties).
void fuse_maxblock(const sv_gate* g, size_t n, int max_k, std::vector<FusedGate>& out,
                   std::vector<int32_t>& block_of) {
  std::vector<std::vector<int>> blocks, other;
  maxblock_partition(g, n, max_k, false, blocks);
  maxblock_partition(g, n, max_k, true, other);
  if (other.size() < blocks.size()) blocks.swap(other);
  fuse_blocks(g, n, blocks, out, block_of);
}

void fuse_blocks(const sv_gate* g, size_t n, const std::vector<std::vector<int>>& blocks,
                 std::vector<FusedGate>& out, std::vector<int32_t>& block_of, int max_ctrl) {
  out.clear();
  block_of.assign(n, -1);
  // The block matrices are independent: build them on host threads when
  // there is enough work to pay for the threads (many large blocks), and
  // never from inside another pool's worker.
  const size_t nb = blocks.size();
  std::vector<std::vector<FusedGate>> built(nb);
  size_t work = 0;  // gate products times block dimension squared
  for (size_t b = 0; b < nb; ++b) {
    uint64_t S = 0;
    for (int i : blocks[b]) S |= qmask(g[i]);
    work += blocks[b].size() << (2 * std::min(__builtin_popcountll(S), SV_MAX_K));
  }
  const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  // (one thread per block up to the core count: the per-block work is uneven,
  // 2^c matrices for c control bits; measured 2-3 ms faster on the 34-qubit
  // grid's 29 blocks than one thread per four blocks)
  const unsigned nt = host_pool_worker() || work < ((size_t)1 << 20) ? 1u : (unsigned)std::min<size_t>(hw, nb);
  if (nt <= 1) {
    for (size_t b = 0; b < nb; ++b) build_block_mux(g, blocks[b], max_ctrl, built[b]);
  } else {
    std::atomic<size_t> next{0};
    std::vector<std::exception_ptr> errs(nt);
    auto worker = [&](unsigned w) {
      try {
        for (size_t b = next++; b < nb; b = next++) build_block_mux(g, blocks[b], max_ctrl, built[b]);
      } catch (...) {  // carried back to the caller; an exception must not end a thread
        errs[w] = std::current_exception();
        next = nb;
      }
    };
    std::vector<std::thread> pool;
    for (unsigned w = 1; w < nt; ++w) pool.emplace_back(worker, w);
    worker(0);
    for (auto& t : pool) t.join();
    for (auto& e : errs)
      if (e) std::rethrow_exception(e);
  }
  size_t total = 0;
  for (auto& v : built) total += v.size();
  out.reserve(total);
  for (size_t b = 0; b < nb; ++b) {
    for (int i : blocks[b]) block_of[i] = (int32_t)out.size();
    for (auto& f : built[b]) out.push_back(std::move(f));
  }
}

void fuse_greedy(const sv_gate* g, size_t n, int max_k, std::vector<FusedGate>& out,
                 std::vector<int32_t>& block_of) {
  std::vector<std::vector<int>> blocks;
  greedy_partition(g, n, max_k, blocks);
  fuse_blocks(g, n, blocks, out, block_of);
}

}  // namespace sv
