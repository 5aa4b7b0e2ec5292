// Contraction planner: greedy minimum-intermediate-size path search, Kraus-index slicing,
// block fusion and lowering to device steps.
//
// The paper fixes its order with a tree decomposition of the network's line graph and
// contracts with tensor decision diagrams (Section IV-C).  Here the order is a linear
// "frontier" path: the running intermediate T absorbs one neighbouring tensor at a time,
// always the one that leaves T smallest (ties: the cheaper step, then a random draw), from
// several starting tensors; the cheapest path under the size cap wins.  Every intermediate then
// meets one small tensor at a time, so each device step is a batched small-operator
// contraction C[f, n] = sum_s A[f, s] B[s, n] whose A and C are addressed through bit-position
// tables (no transposes of the large tensor are ever needed).
//
// Kraus indices (open legs of Algorithm I networks) are kept in the intermediate (batched) until
// the cap forces slicing; a sliced site is iterated depth-first, and everything before it in
// the path is computed once and reused by all its Kraus operators -- the shared "computed table"
// of Section IV-C in the form of a prefix stack.
#include <algorithm>
#include <iterator>
#include <limits>
#include <stdexcept>
#include <chrono>
#include <cmath>
#include <map>
#include <random>
#include <set>
#include <thread>

#include "jf_internal.h"

namespace jf {
static constexpr int kMaxOutLog2 = 34;
// at most 2^24 depth-first leaves from sliced wire legs per component
static constexpr int kMaxWireSlices = 24;

namespace {

struct LocalNet {
  std::vector<const Tensor*> ts;
  std::vector<std::vector<int>> legs;  // local leg ids per tensor
  std::vector<std::vector<int>> leg_tensors;  // tensors per local leg (1 or 2)
  std::vector<char> open;               // local leg is an open (Kraus-index) leg
  std::vector<int> glob;                // network (global) id of every local leg
  int nl = 0;
};

LocalNet make_local(const Network& net, const std::vector<int>& comp) {
  LocalNet L;
  std::map<int, int> lid;
  for (int ti : comp) {
    const Tensor& t = net.T[ti];
    L.ts.push_back(&t);
    std::vector<int> ls;
    for (int g : t.legs) {
      auto it = lid.find(g);
      int id;
      if (it == lid.end()) {
        id = L.nl++;
        lid[g] = id;
        L.leg_tensors.emplace_back();
        L.glob.push_back(g);
      } else {
        id = it->second;
      }
      ls.push_back(id);
      L.leg_tensors[id].push_back(int(L.ts.size()) - 1);
    }
    L.legs.push_back(ls);
  }
  L.open.assign(L.nl, 0);
  for (int l = 0; l < L.nl; ++l) L.open[l] = L.leg_tensors[l].size() == 1;
  return L;
}

struct Path {
  std::vector<int> order;
  std::vector<int> width;   // width of T after each step (all legs, open included)
  std::vector<int> uni;     // legs touched by each step (|T| + new)
  double cost = 0;          // sum of 2^uni: the unfused work, used to guide the greedy search
  double est = 0;           // cost-model time of the fused, sliced program (ranks the restarts)
  int maxw = 0;
  int bw = 0;               // widest intermediate with every Kraus-index leg removed
  int tier = 2;             // 0 Kraus slicing suffices, 1 wire slices too, 2 neither (see evaluate)
};

Path greedy(const LocalNet& L, int start, std::mt19937_64& rng, double temp) {
  const int N = int(L.ts.size());
  Path P;
  std::vector<char> inT(L.nl, 0), absorbed(N, 0), front(N, 0);
  std::vector<int> frontier;
  int width = 0;
  std::uniform_real_distribution<double> U(0.0, 1.0);
  auto absorb = [&](int c) {
    int shared = 0;
    for (int l : L.legs[c]) shared += inT[l];
    int nnew = int(L.legs[c].size()) - shared;
    int uni = width + nnew;
    for (int l : L.legs[c]) inT[l] ^= 1;
    width = width - shared + nnew;
    absorbed[c] = 1;
    P.order.push_back(c);
    P.width.push_back(width);
    P.uni.push_back(uni);
    P.cost += std::ldexp(1.0, uni);
    P.maxw = std::max(P.maxw, width);
    for (int l : L.legs[c])
      for (int t : L.leg_tensors[l])
        if (!absorbed[t] && !front[t]) {
          front[t] = 1;
          frontier.push_back(t);
        }
  };
  absorb(start);
  while ((int)P.order.size() < N) {
    int best = -1;
    double best_key = 1e300;
    for (int c : frontier) {
      if (absorbed[c]) continue;
      int shared = 0;
      for (int l : L.legs[c]) shared += inT[l];
      int nnew = int(L.legs[c].size()) - shared;
      double key = double(width - shared + nnew) + 0.01 * double(width + nnew);
      if (temp > 0) key += temp * U(rng);
      if (key < best_key) {
        best_key = key;
        best = c;
      }
    }
    if (best < 0) {  // disconnected remainder (cannot happen inside one component)
      for (int c = 0; c < N; ++c)
        if (!absorbed[c]) { best = c; break; }
    }
    absorb(best);
    frontier.erase(std::remove_if(frontier.begin(), frontier.end(), [&](int t) { return absorbed[t]; }), frontier.end());
  }
  return P;
}

int ilog2_ceil(int x) {
  int b = 0;
  while ((1 << b) < x) ++b;
  return b;
}

// bits of the index -> offset given bit positions
long long scatter(long long x, const std::vector<int>& pos) {
  long long o = 0;
  for (size_t k = 0; k < pos.size(); ++k) o |= ((x >> k) & 1LL) << pos[k];
  return o;
}

// Step cost for fusion decisions, calibrated on MI355X: HBM at 5.2 TB/s, what a plain streaming
// copy sustains there (the library's nontemporal copy, jf_stream_copy, 5.0-5.3 TB/s at 8 and 16
// bytes per lane; the runtime's device copy 5.2 TB/s) and what the large step kernels reach (4.2 to
// 5.9 TB/s, read-heavy steps above the copy rate); the complex GEMM of a tile sustains ~55 TFLOP/s
// on FP32 MFMA and ~28 TFLOP/s on FP64 MFMA (K = 32 operators).
struct CostModel {
  double bw = 5.2e12;        // effective bytes/s
  double flops = 28e12;      // effective flop/s (FP64 MFMA)
  // seconds per launch: a step kernel's dispatch and set-up in a running program (an empty kernel
  // alone reads 3.8 us with dispatch events); 7 fits the latency-bound plans (the 36-qubit chain:
  // 0.168 ms estimated, 0.170 measured) and gives the 25-qubit chain 65 launches for 70 at 4 us
  // (0.62 against 0.66 ms); the n=16 plan changes little (0.995 against 1.014 ms)
  double launch = 7e-6;
  // complex64 chains (k_chain), algorithmic flop/s: measured 65-115 TFLOP/s on MI355X (2^22 to 2^26
  // elements); 80 picks the faster n=16 plan (1.01 ms per pass against 1.07 ms with 115)
  double chain_flops = 80e12;
  double step(int rA, int rC, int kS, int kN, int ein, int eout) const {
    int f = rA - kS;
    double by = std::ldexp(double(ein), rA) + std::ldexp(double(eout), rC);
    double fl = 8.0 * std::ldexp(1.0, f + kS + kN);
    return std::max(by / bw, fl / flops) + launch;
  }
  // one launch that reads and writes a complex64 intermediate of 2^rA elements once
  double chain(int rA, double fl) const { return std::max(std::ldexp(16.0, rA) / bw, fl / chain_flops) + launch; }
};

}  // namespace

std::vector<int> step_s_positions(const Step& st) {
  std::vector<int> pos;
  for (int i = 0; i < st.kS; ++i) {
    const long long o = st.offS_A[size_t(1) << i];
    int b = 0;
    while ((1LL << b) != o) ++b;
    pos.push_back(b);
  }
  return pos;
}

// In-place complex64 step with an FP32 operator (single or an FP32 pair) or a single-term
// split-form operator, of at most 32 x 32 (the Gauss-form products the chain kernels apply).
bool chainable(const Step& st) {
  return st.inplace_ok && !st.final_step && (st.compute == C_F32 || (st.compute == C_SPLIT && !st.two_term)) &&
         st.in_prec == P_C64 &&
         st.out_prec == P_C64 && st.kS == st.kN && st.kS >= 1 && st.kS <= 5;
}

namespace {

// Tile of a chain over the contracted positions U of its steps (tensor of 2^rA elements): U plus
// the lowest other positions as rows, 2^12 elements at most, at least 16 rows of every step's
// other bits in a tile (T - kS >= 4).  False if no such tile exists.
bool chain_tile(const std::set<int>& U, int rA, int ksmax, Chain& ch) {
  const int u = int(U.size());
  if (u > CHAIN_MAX_U || rA < u) return false;
  int rows = std::min(CHAIN_MAX_T - u, rA - u);
  // a smaller tile for a smaller intermediate, so that there are 2^10 tiles or more (several per
  // resident workgroup) where the tile can shrink: it keeps 16 rows per step (T - kS >= 4) and
  // bits 0-3
  int low_free = 0;
  for (int q = 0; q < 4 && q < rA; ++q) low_free += U.count(q) ? 0 : 1;
  while (u + rows > rA - 10 && rows - 1 >= low_free && u + rows - 1 - ksmax >= 4) --rows;
  const int T = u + rows;
  if (T - ksmax < 4) return false;
  ch.P.clear();
  ch.hi.clear();
  int taken = 0;
  for (int b = 0; b < rA; ++b) {
    if (U.count(b)) {
      ch.P.push_back(b);
    } else if (taken < rows) {
      ch.P.push_back(b);
      ++taken;
    } else {
      ch.hi.push_back(b);
    }
  }
  // the tile holds whole 128-byte lines (16 complex64 elements: bits 0..3), so no line is
  // fetched or written by two tiles
  for (int q = 0; q < 4 && q < rA; ++q)
    if (std::find(ch.P.begin(), ch.P.end(), q) == ch.P.end()) return false;
  ch.T = T;
  ch.nTiles = 1LL << ch.hi.size();
  return int(ch.hi.size()) <= MAXHI;
}

// What chain grouping needs to know of a step.
struct ChainCand {
  bool ok = false;         // chainable (in place, FP32 or single-term split form, K = Nn <= 32)
  bool split = false;      // split-form step (its operator's LDS budget)
  bool two = false;        // FP32 pair operator (twice the LDS entries)
  int kS = 0, rA = 0;
  std::vector<int> spos;   // bit positions of its contracted legs
};

// Group steps [first, last) of one level into chains: greedily extend a run of chainable steps
// while the union of their contracted positions still has a tile, the operators fit the LDS
// budget and the run has at most CHAIN_MAX_STEPS steps; emit(i, j, tile) for every run [i, j) of
// two or more.  The lowering and the planner's cost estimate both group with this function.
template <class Emit>
void group_chains(const std::vector<ChainCand>& c, int first, int last, Emit&& emit) {
  int i = first;
  while (i < last) {
    if (!c[i].ok) {
      ++i;
      continue;
    }
    std::set<int> U(c[i].spos.begin(), c[i].spos.end());
    const int budget = c[i].split ? CHAIN_MAX_OPS_SPLIT : CHAIN_MAX_OPS;
    int ops = chain_step_ops(c[i].kS, c[i].split, c[i].two), ksmax = c[i].kS;
    Chain best;
    const bool have = chain_tile(U, c[i].rA, ksmax, best);
    int j = i + 1;
    while (have && j < last && j - i < CHAIN_MAX_STEPS) {
      if (!c[j].ok || c[j].rA != c[i].rA) break;
      std::set<int> U2 = U;
      U2.insert(c[j].spos.begin(), c[j].spos.end());
      const int ops2 = ops + chain_step_ops(c[j].kS, c[j].split, c[j].two), ks2 = std::max(ksmax, c[j].kS);
      Chain c2;
      if (ops2 > budget || !chain_tile(U2, c[i].rA, ks2, c2)) break;
      U = U2;
      ops = ops2;
      ksmax = ks2;
      best = c2;
      ++j;
    }
    if (have && j - i >= 2) {
      emit(i, j, best);
      i = j;
    } else {
      ++i;
    }
  }
}

// Chains of one level of a lowered component (steps [first, last)); returns the change of the
// level's cost-model time per leaf (the chain's launch in place of its steps' launches).
double build_level_chains(ComponentProgram& cp, int first, int last, const CostModel& cm) {
  std::vector<ChainCand> c(cp.steps.size());
  for (int q = first; q < last; ++q) {
    const Step& st = cp.steps[q];
    c[q].ok = chainable(st);
    c[q].split = st.compute == C_SPLIT;
    c[q].two = st.two_term;
    c[q].kS = st.kS;
    c[q].rA = st.rA;
    if (c[q].ok) c[q].spos = step_s_positions(st);
  }
  double dt = 0;
  group_chains(c, first, last, [&](int i, int j, Chain ch) {
    ch.first = i;
    ch.last = j;
    ch.bytes = std::ldexp(16.0, cp.steps[i].rA);
    for (int q = i; q < j; ++q) {
      const Step& st = cp.steps[q];
      ch.flops += st.flops;
      dt -= std::max(st.bytes / cm.bw, st.flops / cm.flops) + cm.launch;
      cp.steps[q].chain = int(cp.chains.size());
    }
    dt += cm.chain(cp.steps[i].rA, ch.flops);
    cp.chains.push_back(ch);
  });
  return dt;
}

}  // namespace

void chain_tables(const ComponentProgram& cp, const Chain& ch, ChainTables& out) {
  std::map<int, int> local;  // position -> tile-local bit
  for (int i = 0; i < ch.T; ++i) local[ch.P[i]] = i;
  for (int d = 0; d < 3; ++d)
    for (int m = 0; m < 16; ++m) {
      long long o = 0;
      for (int b = 0; b < 4; ++b)
        if (((m >> b) & 1) && 4 * d + b < ch.T) o |= 1LL << ch.P[4 * d + b];
      out.gDig[d][m] = o;
    }
  out.sOff.clear();
  out.fDig.clear();
  for (int q = ch.first; q < ch.last; ++q) {
    const Step& st = cp.steps[q];
    std::vector<int> sl;
    for (int b : step_s_positions(st)) sl.push_back(local.at(b));
    std::vector<int> fl;
    for (int i = 0; i < ch.T; ++i)
      if (!std::count(sl.begin(), sl.end(), i)) fl.push_back(i);
    std::vector<unsigned short> so(size_t(1) << st.kS), fd(48, 0);
    for (int s = 0; s < (1 << st.kS); ++s) {
      int o = 0;
      for (int b = 0; b < st.kS; ++b)
        if ((s >> b) & 1) o |= 1 << sl[b];
      so[s] = (unsigned short)o;
    }
    for (int d = 0; d < 3; ++d)
      for (int m = 0; m < 16; ++m) {
        int o = 0;
        for (int b = 0; b < 4; ++b)
          if (((m >> b) & 1) && 4 * d + b < (int)fl.size()) o |= 1 << fl[4 * d + b];
        fd[size_t(d) * 16 + m] = (unsigned short)o;
      }
    out.sOff.push_back(so);
    out.fDig.push_back(fd);
  }
}

Program plan_program(const jf_circuit& c, const PlanOptions& opt) {
  auto t0 = std::chrono::steady_clock::now();
  Program P;
  P.opt = opt;
  P.n_qubits = c.n;
  Network net = build_network(c, opt.alg);
  P.n_before_cancel = net.n_before_cancel;
  if (!(opt.flags & JF_FLAG_NO_CANCEL)) {
    cancel_inverse_pairs(net);
    P.n_swaps_rewired = rewire_swaps(net);
  }
  P.n_after_cancel = int(net.T.size());
  P.empty_loops = count_empty_loops(net);
  trace_self_loops(net);
  P.log2_scale = net.log2_scale + P.empty_loops;
  P.scalar = net.scalar;
  P.site_nk = net.site_nk;
  P.site_comp.assign(c.sites.size(), -1);
  // ||K||^2 (largest eigenvalue of K^dagger K) of every Kraus operator: |t_k|^2 <= prod_i ||K_{k_i}||^2
  for (const NoiseSite& ns : c.sites) {
    std::vector<double> v;
    for (int j = 0; j < ns.nk; ++j) {
      const cd* K = &ns.kraus[size_t(4) * j];
      const double a = std::norm(K[0]) + std::norm(K[2]), d = std::norm(K[1]) + std::norm(K[3]);
      const cd b = std::conj(K[0]) * K[1] + std::conj(K[2]) * K[3];
      v.push_back(0.5 * (a + d) + std::sqrt(0.25 * (a - d) * (a - d) + std::norm(b)));
    }
    P.site_norm2.push_back(v);
  }
  // prod_i n_i saturates at the largest long long (Algorithm II networks cover 4^40 tuples and more)
  for (int nk : net.site_nk)
    if (__builtin_mul_overflow(P.kraus_terms, (long long)nk, &P.kraus_terms)) {
      P.kraus_terms = std::numeric_limits<long long>::max();
      break;
    }

  const bool low_form = opt.dtype != JF_C128;  // complex64 or split form requested
  CostModel cm_form;  // the requested form's model (complex128: the defaults)
  if (opt.dtype == JF_C64) cm_form.flops = 70e12;  // FP32 MFMA contraction rate measured at K = 32 to 64
  if (opt.dtype == JF_C64_BF16X6) {
    cm_form.flops = 200e12;        // split form on BF16 matrix cores: the steps stay HBM-bound
    cm_form.chain_flops = 120e12;  // split-form chains: measured 80-137 TFLOP/s (2^24 to 2^26 elements)
  }

  auto comps = components(net);
  std::mt19937_64 rng(opt.seed);
  size_t max_comp_buf = 0;
  long long out_total = 0;

  for (auto& comp : comps) {
    LocalNet L = make_local(net, comp);
    const int N = int(L.ts.size());
    // this component runs in the requested low form (FP32 storage up to the precision switch);
    // cleared below for a component that is all closing part
    bool low = low_form;
    int elem_lo = low ? 8 : 16;
    CostModel cm = cm_form;
    // ---- site bookkeeping: open legs of this component, output bit offsets
    ComponentProgram cp;
    cp.n_tensors = N;
    cp.out_bit.assign(c.sites.size(), std::vector<int>());
    std::vector<int> comp_sites;
    for (int i = 0; i < N; ++i)
      if (L.ts[i]->kind == T_SLOT || (L.ts[i]->site >= 0 && opt.alg == 1 && !L.ts[i]->var_legs.empty()))
        comp_sites.push_back(L.ts[i]->site);
    // slots that lost their kind through a self-loop trace keep site/var_legs
    comp_sites.clear();
    for (int i = 0; i < N; ++i)
      if (opt.alg == 1 && L.ts[i]->site >= 0) comp_sites.push_back(L.ts[i]->site);
    std::sort(comp_sites.begin(), comp_sites.end());
    comp_sites.erase(std::unique(comp_sites.begin(), comp_sites.end()), comp_sites.end());
    {
      int nbits = 0;
      for (int si : comp_sites) {
        nbits += int(net.site_var_legs[si].size());
        cp.out_bit[si].assign(net.site_var_legs[si].size(), -1);
        P.site_comp[si] = int(P.comps.size());
      }
      // Algorithm I keeps one FP64 complex value per Kraus tuple of the component, whole whatever
      // the slicing: past 2^34 of them (256 GiB) no single device holds the output
      if (nbits > kMaxOutLog2) {
        set_error("Algorithm I output of 2^" + std::to_string(nbits) + " Kraus-tuple values exceeds 2^" +
                  std::to_string(kMaxOutLog2) + " (Algorithm II does not grow with the tuples)");
        throw jf_status(JF_E_TOO_LARGE);
      }
      cp.n_open_bits = nbits;
      cp.out_len = 1LL << nbits;
    }
    // global leg id -> (site, bit)
    std::map<int, std::pair<int, int>> open_of;
    for (int si : comp_sites)
      for (size_t b = 0; b < net.site_var_legs[si].size(); ++b) open_of[net.site_var_legs[si][b]] = {si, int(b)};

    // ---- slicing: the indices a path slices to fit the cap.  Kraus sites first (the earliest slot
    // at or before the widest position: a sliced site iterates its Kraus operators depth first and
    // every step before its slot is computed once for all of them), then ordinary wire legs alive at
    // the widest position (a sliced wire is fixed to each of its two values in turn and the leaves'
    // partial results add up): the one that covers the most positions still over the cap, ties to
    // the later start (a longer shared prefix), then the lower leg id.  False when that would take
    // more than kMaxWireSlices wire slices.
    struct Slices {
      std::vector<char> site;   // sliced Kraus sites (by site index)
      std::vector<int> wires;   // sliced wire legs (local ids), in the order chosen
      std::vector<int> cut;     // per path position: sliced bits alive there
    };
    auto positions = [&](const Path& p) {
      std::vector<int> pos(N);
      for (int k = 0; k < N; ++k) pos[p.order[k]] = k;
      return pos;
    };
    auto wire_span = [&](const std::vector<int>& pos, int l) {  // positions [a, b) where wire l is in T
      const int x = pos[L.leg_tensors[l][0]], y = pos[L.leg_tensors[l][1]];
      return std::make_pair(std::min(x, y), std::max(x, y));
    };
    auto decide_slices = [&](const Path& p, Slices& S) -> bool {
      const std::vector<int> pos = positions(p);
      S.site.assign(c.sites.size(), 0);
      S.wires.clear();
      S.cut.assign(N, 0);
      std::vector<int> slot(c.sites.size(), N);
      for (int k = 0; k < N; ++k) {
        const Tensor* t = L.ts[p.order[k]];
        if (opt.alg == 1 && t->site >= 0) slot[t->site] = k;
      }
      auto slice_site = [&](int si) {
        S.site[si] = 1;
        for (int k = slot[si]; k < N; ++k) S.cut[k] += int(net.site_var_legs[si].size());
      };
      if (opt.flags & JF_FLAG_NO_BATCH)
        for (int si : comp_sites)
          if (!net.site_var_legs[si].empty()) slice_site(si);
      std::vector<char> wcut(L.nl, 0);
      while (true) {
        int worst = -1, ww = -1;
        for (int k = 0; k < N; ++k)
          if (p.width[k] - S.cut[k] > ww) {
            ww = p.width[k] - S.cut[k];
            worst = k;
          }
        if (ww <= opt.cap_log2) return true;
        int pickc = -1;
        for (int si : comp_sites)
          if (!S.site[si] && !net.site_var_legs[si].empty() && slot[si] <= worst &&
              (pickc < 0 || slot[si] < slot[pickc]))
            pickc = si;
        if (pickc >= 0) {
          slice_site(pickc);
          continue;
        }
        if ((int)S.wires.size() >= kMaxWireSlices) return false;
        int pick = -1, pick_cover = -1, pick_start = -1;
        for (int l = 0; l < L.nl; ++l) {
          if (L.open[l] || wcut[l] || L.leg_tensors[l].size() != 2) continue;
          const auto ab = wire_span(pos, l);
          if (!(ab.first <= worst && worst < ab.second)) continue;
          int cover = 0;
          for (int k = ab.first; k < ab.second; ++k) cover += p.width[k] - S.cut[k] > opt.cap_log2;
          if (cover > pick_cover || (cover == pick_cover && ab.first > pick_start)) {
            pick = l;
            pick_cover = cover;
            pick_start = ab.first;
          }
        }
        if (pick < 0) return false;
        wcut[pick] = 1;
        S.wires.push_back(pick);
        const auto ab = wire_span(pos, pick);
        for (int k = ab.first; k < ab.second; ++k) S.cut[k] += 1;
      }
    };

    // ---- greedy path search with restarts
    // Paths rank in tiers: those that slicing Kraus indices alone brings under the cap, then those
    // that also need wire slices, then the rest (narrower first); within the first two tiers the
    // cost-model time of the fused, sliced program decides (ties: the smaller unfused work).
    Path best;
    best.cost = 1e300;
    bool have = false;
    auto base_width = [&](const Path& p) {
      int open = 0, w = 0;
      for (size_t k = 0; k < p.order.size(); ++k) {
        for (int l : L.legs[p.order[k]]) open += L.open[l];
        w = std::max(w, p.width[k] - open);
      }
      return w;
    };
    // Cost-model time of the program a path lowers to: the slicing, precision switch and block
    // fusion below, decided on leg sets only (no tensor data), each step priced like the real
    // lowering prices it.  Used only to rank candidate paths; the lowering itself decides again.
    // Legs are the component's local ids.
    // maxr (optional): receives the largest intermediate of that program, log2 elements
    auto fused_estimate = [&](const Path& p, int* maxr = nullptr) -> double {
      if (maxr) *maxr = 1 << 20;
      Slices S;
      if (!decide_slices(p, S)) return 1e300;
      int mr = 0;
      const std::vector<int> pos = positions(p);
      // legs the slicing removes, and the levels' starts (the factor each multiplies the work by)
      std::vector<char> gone(L.nl, 0);
      std::vector<double> head_mult(N, 1.0);
      for (int l : S.wires) {
        gone[l] = 1;
        head_mult[wire_span(pos, l).first] *= 2;
      }
      int sliced_bits = 0;
      for (int k = 0; k < N; ++k) {
        const Tensor* t = L.ts[p.order[k]];
        if (opt.alg == 1 && t->site >= 0 && S.site[t->site]) {
          head_mult[k] *= net.site_nk[t->site];
          sliced_bits += int(net.site_var_legs[t->site].size());
          for (size_t j = 0; j < t->legs.size(); ++j)
            if (std::find(t->var_legs.begin(), t->var_legs.end(), t->legs[j]) != t->var_legs.end())
              gone[L.legs[p.order[k]][j]] = 1;
        }
      }
      std::vector<std::vector<int>> eff(N);
      for (int i = 0; i < N; ++i)
        for (int l : L.legs[i])
          if (!gone[l]) eff[i].push_back(l);
      auto effw = [&](int k) { return p.width[k] - S.cut[k]; };
      int sw = N;
      if (low) {
        sw = 0;
        int prev = 0;
        std::vector<int> w(N);
        for (int k = 0; k < N; ++k) w[k] = effw(k);
        for (int k = N - 1; k >= 0; --k) {
          prev = k > 0 ? w[k - 1] : 0;
          if (w[k] > opt.switch_log2 || prev > opt.switch_log2) { sw = k + 1; break; }
        }
      }
      std::vector<char> inT(L.nl, 0), inB(L.nl, 0);
      int rT = 0;
      double est = 0, mult = 1;
      int in_e = low ? 8 : 16;
      int k = 0;
      std::vector<int> blk, trial;
      // bit positions of the intermediate's legs, laid out as the lowering lays them out, and the
      // steps of the current level as chain candidates with their cost-model times
      std::vector<int> Tl, posT(L.nl, -1), Sv, Nv, nTl;
      std::vector<ChainCand> seg;
      std::vector<double> segt;
      while (k < N) {
        // a sliced index starts a level: its value is fixed per leaf, its legs are gone
        mult *= head_mult[k];
        int kend = N;
        for (int j = k + 1; j < N; ++j)
          if (head_mult[j] > 1) {
            kend = j;
            break;
          }
        seg.clear();
        segt.clear();
        while (k < kend) {
          blk = eff[p.order[k]];
          for (int l : blk) inB[l] = 1;
          const int rA = rT;
          int kS = 0;
          for (int l : blk) kS += inT[l];
          int kN = int(blk.size()) - kS;
          int e = k + 1;
          while (!(opt.flags & JF_FLAG_NO_FUSE) && e < kend) {
            if (low && e == sw) break;
            const std::vector<int>& nx = eff[p.order[e]];
            // trial = blk xor nx
            trial.clear();
            for (int l : blk)
              if (std::find(nx.begin(), nx.end(), l) == nx.end()) trial.push_back(l);
            for (int l : nx)
              if (!inB[l]) trial.push_back(l);
            int s2 = 0;
            for (int l : trial) s2 += inT[l];
            const int n2 = int(trial.size()) - s2;
            if (s2 > opt.kmax || n2 > opt.kmax) break;
            if ((1 << s2) * ((1 << n2) + 16) > 3840) break;
            const int ein = (low && k >= sw) ? 16 : elem_lo;
            const int rmid = rA - kS + kN;
            int s3 = 0;  // legs of nx in T xor blk
            for (int l : nx) s3 += inT[l] ^ inB[l];
            const int n3 = int(nx.size()) - s3;
            const double sep = cm.step(rA, rmid, kS, kN, ein, ein) + cm.step(rmid, rmid - s3 + n3, s3, n3, ein, ein);
            const double fused = cm.step(rA, rA - s2 + n2, s2, n2, ein, ein);
            if (fused > sep) break;
            for (int l : blk) inB[l] = 0;
            blk.swap(trial);
            for (int l : blk) inB[l] = 1;
            kS = s2;
            kN = n2;
            ++e;
          }
          const bool final_step = (e == N);
          const int out_e = low ? (((k >= sw) || final_step) ? 16 : 8) : 16;
          const int rC = rA - kS + kN;
          mr = std::max({mr, rA, final_step ? 0 : rC});
          const double by = std::ldexp(double(in_e), rA) + std::ldexp(double(out_e), rC);
          const double fl = 8.0 * std::ldexp(1.0, rA + kN);
          const double t_step = std::max(by / cm.bw, fl / cm.flops) + cm.launch;
          est += mult * t_step;
          // chain candidate and the new layout (as the lowering places legs)
          Sv.clear();
          Nv.clear();
          for (int l : blk) (inT[l] ? Sv : Nv).push_back(l);
          std::sort(Sv.begin(), Sv.end(), [&](int a, int b) { return posT[a] < posT[b]; });
          std::sort(Nv.begin(), Nv.end(), [&](int a, int b) { return L.glob[a] < L.glob[b]; });
          ChainCand cc;
          if (low && k < sw && !final_step && kS == kN && kS >= 1 && kS <= 5) {
            // a block with a noise operator keeps it as an FP32 pair; the lowering chains such
            // steps in complex64, but the estimate leaves them out: counted in, they drew the
            // path search to longer chains over small intermediates, whose few tiles leave most
            // compute units idle (measured on the n=25 chain workload: 0.49 -> 0.50 ms of kernels)
            bool noise = false;
            for (int q = k; q < e; ++q) noise = noise || L.ts[p.order[q]]->site >= 0;
            if (!noise) {
              cc.ok = true;
              cc.split = opt.dtype == JF_C64_BF16X6;
              for (int l : Sv) cc.spos.push_back(posT[l]);
            }
          }
          cc.kS = kS;
          cc.rA = rA;
          seg.push_back(std::move(cc));
          segt.push_back(t_step);
          if (!final_step) {
            if (kS == kN) {
              for (int i = 0; i < kS; ++i) {
                posT[Nv[i]] = posT[Sv[i]];
                Tl[posT[Sv[i]]] = Nv[i];
                posT[Sv[i]] = -1;
              }
            } else {
              nTl.clear();
              for (int l : Tl)
                if (!inB[l]) nTl.push_back(l);
              for (int l : Sv) posT[l] = -1;
              for (int l : Nv) nTl.push_back(l);
              Tl.swap(nTl);
              for (int i = 0; i < (int)Tl.size(); ++i) posT[Tl[i]] = i;
            }
          }
          for (int l : blk) {
            inT[l] ^= 1;
            inB[l] = 0;
          }
          rT = rC;
          in_e = out_e;
          k = e;
        }
        group_chains(seg, 0, int(seg.size()), [&](int i, int j, const Chain&) {
          double fl = 0;
          for (int q = i; q < j; ++q) {
            fl += 8.0 * std::ldexp(1.0, seg[q].rA + seg[q].kS);
            est -= mult * segt[q];
          }
          est += mult * cm.chain(seg[i].rA, fl);
        });
      }
      // with sliced wires every leaf adds its output into the component's
      if (!S.wires.empty()) est += mult * (cm.launch + 32.0 * std::ldexp(1.0, cp.n_open_bits - sliced_bits) / cm.bw);
      if (maxr) *maxr = mr;
      return est;
    };
    // tier 0: Kraus slicing suffices; 1: wire slices too; 2: beyond kMaxWireSlices.  A path that
    // cannot beat the best seen (tier 1 against a tier 0) skips the estimate.
    auto evaluate = [&](Path& p, bool tier0_seen) {
      p.bw = base_width(p);
      if (p.bw <= opt.cap_log2) {
        p.tier = 0;
        p.est = fused_estimate(p);
      } else if (tier0_seen) {
        p.tier = 1;
        p.est = 1e300;
      } else {
        p.est = fused_estimate(p);
        p.tier = p.est < 1e300 ? 1 : 2;
      }
    };
    auto better_path = [&](const Path& a, const Path& b) {
      if (a.tier != b.tier) return a.tier < b.tier;
      if (a.tier == 2) return a.bw < b.bw;
      return a.est < b.est * (1 - 1e-12) || (a.est <= b.est * (1 + 1e-12) && a.cost < b.cost);
    };
    auto consider = [&](Path& p) {
      if (!have || better_path(p, best)) {
        best = p;
        have = true;
      }
    };
    // restarts: by default a fixed amount of search work, ~8e7 tensor absorptions per component
    // (2^17 restarts for a 600-tensor network, 2^16 for 1200), so the plan depends on the network only
    const int auto_tries = int(std::min(131072.0, std::max(4096.0, 8.0e7 / N)));
    const int restarts_total = N <= 24 ? 256 : (opt.restarts > 0 ? opt.restarts : auto_tries);
    std::vector<int> starts;
    for (int i = 0; i < N; ++i)
      if (L.ts[i]->site >= 0) starts.push_back(i);
    if (N <= 24)
      for (int i = 0; i < N; ++i) starts.push_back(i);
    const std::mt19937_64 rng_at_search = rng;
    std::mt19937_64 rng_after_search = rng;
    for (int attempt = 0;; ++attempt) {
      best = Path();
      best.cost = 1e300;
      have = false;
      for (int s : starts) {
        Path p = greedy(L, s, rng, 0.0);
        evaluate(p, have && best.tier == 0);
        consider(p);
      }
      // The default search is also sized to the stakes: when the deterministic starts already give a
      // program estimated under 200 us of device time, seconds of host search could save only
      // microseconds, so it takes 512 restarts (an explicit effort is kept as given).
      const int tries_total = (opt.restarts <= 0 && N > 24 && have && best.tier == 0 && best.est < 2e-4)
                                  ? std::min(restarts_total, 512)
                                  : restarts_total;
      {
        // Randomised restarts on a thread pool.  Each worker draws its starts and Boltzmann noise
        // from its own seeded generator and keeps its best path; the winner is chosen by the same
        // rule in worker order, so the plan does not depend on timing (the time cap only guards
        // pathological inputs).
        const int workers = std::max(1, std::min(opt.threads, int(std::thread::hardware_concurrency())));
        std::vector<Path> wbest(workers);
        std::vector<int> whave(workers, 0);
        auto work = [&](int w) {
          std::mt19937_64 wr(opt.seed * 7919u + 104729u * unsigned(w + 1) + unsigned(N));
          std::uniform_int_distribution<int> pick(0, N - 1);
          const int mine = tries_total / workers + (w < tries_total % workers ? 1 : 0);
          Path bestw;
          bool hv = false;
          for (int tries = 0; tries < mine; ++tries) {
            double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            if (el > opt.time_budget_s && tries >= 8) break;
            int s = (tries % 2 == 0 && !starts.empty()) ? starts[(tries / 2 + w) % starts.size()] : pick(wr);
            Path p = greedy(L, s, wr, 0.5 + ((tries + w) % 5) * 0.5);
            evaluate(p, hv && bestw.tier == 0);
            if (!hv || better_path(p, bestw)) {
              bestw = std::move(p);
              hv = true;
            }
          }
          wbest[w] = std::move(bestw);
          whave[w] = hv;
        };
        std::vector<std::thread> pool;
        for (int w = 1; w < workers; ++w) pool.emplace_back(work, w);
        work(0);
        for (auto& th : pool) th.join();
        for (int w = 0; w < workers; ++w)
          if (whave[w]) consider(wbest[w]);
      }

      // ---- local search on the winner: move single absorptions by up to four places while the
      // fused estimate drops (the greedy choice is made one absorption at a time; a move can undo
      // a locally narrow but globally costly choice).  Deterministic; converges in a few sweeps.
      // Part of a thorough search only (>= 2^12 restarts): its sweeps cost O(tensors^2).
      if (have && best.tier <= 1 && (tries_total >= 4096 || N <= 24)) {
        auto recompute = [&](Path& p) {
          std::vector<char> inT(L.nl, 0);
          int width = 0;
          p.width.clear();
          p.uni.clear();
          p.cost = 0;
          p.maxw = 0;
          for (int ci : p.order) {
            int shared = 0;
            for (int l : L.legs[ci]) shared += inT[l];
            const int nnew = int(L.legs[ci].size()) - shared;
            const int uni = width + nnew;
            for (int l : L.legs[ci]) inT[l] ^= 1;
            width = width - shared + nnew;
            p.width.push_back(width);
            p.uni.push_back(uni);
            p.cost += std::ldexp(1.0, uni);
            p.maxw = std::max(p.maxw, width);
          }
        };
        bool improved = true;
        for (int sweep = 0; improved && sweep < 8; ++sweep) {
          improved = false;
          for (int i = 0; i < N; ++i)
            for (int d = -4; d <= 4; ++d) {  // move absorption i by up to four places
              const int j = i + d;
              if (d == 0 || j < 0 || j >= N) continue;
              Path q = best;
              const int v = q.order[i];
              q.order.erase(q.order.begin() + i);
              q.order.insert(q.order.begin() + j, v);
              recompute(q);
              if (best.tier == 0 && base_width(q) > opt.cap_log2) continue;
              evaluate(q, best.tier == 0);
              if (q.tier < best.tier || (q.tier == best.tier && q.est < best.est * (1 - 1e-9))) {
                best = std::move(q);
                improved = true;
              }
            }
        }
      }

      // A component whose program keeps every intermediate within the FP64 closing size
      // (2^switch_log2 elements) is closing part from its first tensor: in the low forms it is
      // planned again as complex128 (FP64 storage and arithmetic, the complex128 path), since its
      // launches are latency-bound and a complex64 start would only add FP32 steps and rounding.
      // The generator continues as after a single search, so later components plan as before.
      int best_maxr = 1 << 20;
      if (attempt == 0 && low && have && best.tier == 0) fused_estimate(best, &best_maxr);
      if (attempt == 0 && low && best_maxr <= opt.switch_log2) {
        low = false;
        elem_lo = 16;
        cm = CostModel();
        rng_after_search = rng;
        rng = rng_at_search;
        continue;
      }
      if (attempt > 0) rng = rng_after_search;
      break;
    }  // attempt

    // ---- slicing of the chosen path
    const Path& pth = best;
    Slices SL;
    if (!have || !decide_slices(pth, SL)) {
      int ww = 0;
      for (int k = 0; k < N; ++k) ww = std::max(ww, pth.width[k]);
      set_error("no contraction order fits 2^" + std::to_string(opt.cap_log2) + " elements (needs 2^" +
                std::to_string(ww) + " with its Kraus indices open; slicing would take more than " +
                std::to_string(kMaxWireSlices) + " wire legs)");
      throw jf_status(JF_E_TOO_LARGE);
    }
    const std::vector<int> pth_pos = positions(pth);
    auto eff_width = [&](int k) { return pth.width[k] - SL.cut[k]; };

    // ---- block fusion and lowering
    // Current intermediate: legs (global ids) with bit positions.
    std::vector<int> Tlegs;             // position i holds leg Tlegs[i]
    int cur_prec = P_C128;
    // precision switch point: first path position after which every width stays small
    int switch_at = N;  // path index from which steps run in FP64
    if (low) {
      switch_at = 0;
      for (int k = N - 1; k >= 0; --k) {
        int w = eff_width(k);
        int wprev = k > 0 ? eff_width(k - 1) : 0;
        if (w > opt.switch_log2 || wprev > opt.switch_log2) { switch_at = k + 1; break; }
      }
      cur_prec = P_C64;
    }
    // levels: one per sliced index, in path order of where it starts (a sliced site at its slot, a
    // sliced wire at its first tensor); a level 0 without one when none starts at position 0, and
    // empty levels where several start at one position
    struct SliceStart {
      int start, site, wire;  // wire: global leg id
    };
    std::vector<SliceStart> sis;
    for (int k = 0; k < N; ++k) {
      const Tensor* t = L.ts[pth.order[k]];
      if (opt.alg == 1 && t->site >= 0 && SL.site[t->site]) sis.push_back({k, t->site, -1});
    }
    for (int l : SL.wires) sis.push_back({wire_span(pth_pos, l).first, -1, L.glob[l]});
    std::stable_sort(sis.begin(), sis.end(), [](const SliceStart& x, const SliceStart& y) { return x.start < y.start; });
    std::vector<int> level_start, level_site, level_wire;
    if (sis.empty() || sis[0].start > 0) {
      level_start.push_back(0);
      level_site.push_back(-1);
      level_wire.push_back(-1);
    }
    for (const SliceStart& x : sis) {
      level_start.push_back(x.start);
      level_site.push_back(x.site);
      level_wire.push_back(x.wire);
    }
    level_start.push_back(N);
    const int levels_n = int(level_start.size()) - 1;
    std::vector<int> level_nvar(levels_n, 1);
    std::map<int, int> level_of_site, level_of_wire;
    for (int lv = 0; lv < levels_n; ++lv) {
      if (level_site[lv] >= 0) {
        level_nvar[lv] = net.site_nk[level_site[lv]];
        level_of_site[level_site[lv]] = lv;
      }
      if (level_wire[lv] >= 0) {
        level_nvar[lv] = 2;
        level_of_wire[level_wire[lv]] = lv;
      }
    }
    // output bits: the sliced sites take the top ones (last level lowest, one run per site, so a
    // variant's offset is v << run start); the open sites' bits are placed by the final step
    {
      int free_bits = cp.n_open_bits;
      for (int si : level_site)
        if (si >= 0) free_bits -= int(net.site_var_legs[si].size());
      int shift = free_bits;
      for (int lv = int(level_site.size()) - 1; lv >= 0; --lv) {
        const int si = level_site[lv];
        if (si < 0) continue;
        for (size_t b = 0; b < cp.out_bit[si].size(); ++b) cp.out_bit[si][b] = shift + int(b);
        shift += int(cp.out_bit[si].size());
      }
    }

    // The levels whose sliced index a tensor carries (ascending): a sliced site's slot, the two
    // tensors a sliced wire joins.  A block's operator has one variant per combination of their
    // values, indexed mixed-radix with the first level lowest.
    auto deps_of = [&](const Tensor& t) {
      std::vector<int> D;
      if (opt.alg == 1 && t.site >= 0 && level_of_site.count(t.site)) D.push_back(level_of_site[t.site]);
      for (int g : t.legs) {
        auto it = level_of_wire.find(g);
        if (it != level_of_wire.end()) D.push_back(it->second);
      }
      std::sort(D.begin(), D.end());
      return D;
    };
    auto n_variants = [&](const std::vector<int>& D) {
      long long n = 1;
      for (int lv : D) n *= level_nvar[lv];
      return n;
    };
    // the values of the levels D in variant idx (mixed radix over D, first lowest)
    auto values_of = [&](const std::vector<int>& D, long long idx) {
      std::vector<int> v(D.size());
      for (size_t i = 0; i < D.size(); ++i) {
        v[i] = int(idx % level_nvar[D[i]]);
        idx /= level_nvar[D[i]];
      }
      return v;
    };
    // t with the legs of the sliced indices of levels D fixed to the values v (a site's Kraus-index
    // legs to the bits of its operator number, a wire to its value)
    auto restrict_to = [&](const Tensor& t, const std::vector<int>& D, const std::vector<int>& v) {
      std::map<int, int> fix;  // leg -> bit
      for (size_t i = 0; i < D.size(); ++i) {
        const int lv = D[i];
        if (level_site[lv] >= 0) {
          const std::vector<int>& vl = net.site_var_legs[level_site[lv]];
          for (size_t b = 0; b < vl.size(); ++b) fix[vl[b]] = (v[i] >> b) & 1;
        } else {
          fix[level_wire[lv]] = v[i];
        }
      }
      Tensor u;
      u.site = t.site;
      std::vector<int> keep;
      size_t idxval = 0;
      for (size_t i = 0; i < t.legs.size(); ++i) {
        auto it = fix.find(t.legs[i]);
        if (it == fix.end()) {
          keep.push_back(int(i));
          u.legs.push_back(t.legs[i]);
        } else {
          idxval |= size_t(it->second) << i;
        }
      }
      u.data.assign(size_t(1) << u.legs.size(), 0.0);
      for (size_t o = 0; o < u.data.size(); ++o) {
        size_t idx = idxval;
        for (size_t k = 0; k < keep.size(); ++k) idx |= ((o >> k) & 1) << keep[k];
        u.data[o] = t.data[idx];
      }
      return u;
    };
    auto all_variants = [&](const Tensor& t, const std::vector<int>& D) {
      std::vector<Tensor> out;
      const long long n = n_variants(D);
      for (long long i = 0; i < n; ++i) out.push_back(D.empty() ? t : restrict_to(t, D, values_of(D, i)));
      return out;
    };

    std::vector<size_t> level_bytes(levels_n, 0);
    std::vector<int> level_maxw(levels_n, 0);
    double comp_flops = 0, comp_bytes = 0;
    long long mult = 1;
    for (int lv = 0; lv < levels_n; ++lv) {
      Level Lv;
      Lv.first = int(cp.steps.size());
      Lv.site = level_site[lv];
      Lv.wire = level_wire[lv];
      Lv.nvar = level_nvar[lv];
      Lv.out_stride = (Lv.site >= 0 && !cp.out_bit[Lv.site].empty()) ? (1LL << cp.out_bit[Lv.site][0]) : 0;
      mult *= Lv.nvar;
      int k = level_start[lv];
      const int kend = level_start[lv + 1];
      while (k < kend) {
        // ---- grow a block [k, e)
        std::set<int> Tset(Tlegs.begin(), Tlegs.end());
        std::vector<int> D = deps_of(*L.ts[pth.order[k]]);
        std::vector<Tensor> blk = all_variants(*L.ts[pth.order[k]], D);  // per variant
        auto split = [&](const Tensor& b, std::vector<int>& S, std::vector<int>& Nn) {
          S.clear();
          Nn.clear();
          for (int l : b.legs) (Tset.count(l) ? S : Nn).push_back(l);
        };
        int e = k + 1;
        std::vector<int> S, NN;
        split(blk[0], S, NN);
        int rA = int(Tlegs.size());
        auto block_cost = [&](int kS, int kN, int ein, int eout) {
          return cm.step(rA, rA - kS + kN, kS, kN, ein, eout);
        };
        while (!(opt.flags & JF_FLAG_NO_FUSE) && e < kend) {
          // never fuse across the precision switch
          if (low && e == switch_at) break;
          const Tensor& nxt = *L.ts[pth.order[e]];
          const std::vector<int> Dx = deps_of(nxt);
          const Tensor nx = Dx.empty() ? nxt : restrict_to(nxt, Dx, std::vector<int>(Dx.size(), 0));
          Tensor trial = contract_pair(blk[0], nx);
          std::vector<int> S2, N2;
          split(trial, S2, N2);
          if ((int)S2.size() > opt.kmax || (int)N2.size() > opt.kmax) break;
          // keep the operator block and at least 16 tile rows within the LDS budget
          if ((1 << S2.size()) * ((1 << N2.size()) + 16) > 3840) break;
          // cost: fused block vs current block followed by nx alone
          int ein = (low && k >= switch_at) ? 16 : elem_lo;
          int rmid = rA - int(S.size()) + int(NN.size());
          std::set<int> Tmid(Tset);
          for (int l : S) Tmid.erase(l);
          for (int l : NN) Tmid.insert(l);
          int s3 = 0;
          for (int l : nx.legs) s3 += int(Tmid.count(l));
          int n3 = int(nx.legs.size()) - s3;
          double sep = block_cost(int(S.size()), int(NN.size()), ein, ein) +
                       cm.step(rmid, rmid - s3 + n3, s3, n3, ein, ein);
          double fused = block_cost(int(S2.size()), int(N2.size()), ein, ein);
          if (fused > sep) break;
          if (Dx.empty()) {
            for (auto& b : blk) b = contract_pair(b, nxt);
          } else {
            std::vector<int> D2 = D;
            for (int x : Dx)
              if (!std::count(D2.begin(), D2.end(), x)) D2.push_back(x);
            std::sort(D2.begin(), D2.end());
            std::vector<Tensor> blk2;
            const long long n2v = n_variants(D2);
            for (long long i = 0; i < n2v; ++i) {
              const std::vector<int> v2 = values_of(D2, i);
              long long io = 0, stride = 1;  // index of the same values in blk (levels D)
              for (int lvd : D) {
                io += stride * v2[std::find(D2.begin(), D2.end(), lvd) - D2.begin()];
                stride *= level_nvar[lvd];
              }
              std::vector<int> vx;
              for (int lvd : Dx) vx.push_back(v2[std::find(D2.begin(), D2.end(), lvd) - D2.begin()]);
              blk2.push_back(contract_pair(blk[size_t(io)], restrict_to(nxt, Dx, vx)));
            }
            blk.swap(blk2);
            D = D2;
          }
          S = S2;
          NN = N2;
          ++e;
        }
        // ---- lower block [k, e) to one device step
        Step st;
        st.nvar = int(blk.size());
        st.var_levels = D;
        st.kS = int(S.size());
        st.kN = int(NN.size());
        st.rA = rA;
        std::vector<int> F;
        for (int l : Tlegs)
          if (!std::count(S.begin(), S.end(), l)) F.push_back(l);  // in A position order
        st.rC = int(F.size()) + st.kN;
        std::map<int, int> posA;
        for (int i = 0; i < (int)Tlegs.size(); ++i) posA[Tlegs[i]] = i;
        std::sort(S.begin(), S.end(), [&](int a, int b) { return posA[a] < posA[b]; });
        std::sort(NN.begin(), NN.end());
        const bool final_step = (e == N);
        std::map<int, int> posC;
        if (final_step) {
          // every remaining leg is an open Kraus-index leg of an unsliced site: the output keeps
          // the kept legs in their order (tile rows lowest) with the new legs above them, and the
          // Kraus bit each position carries is recorded for reading the output back
          for (int i = 0; i < (int)F.size(); ++i) posC[F[i]] = i;
          for (int i = 0; i < st.kN; ++i) posC[NN[i]] = int(F.size()) + i;
          for (auto& kv : posC) {
            const auto& sb = open_of.at(kv.first);
            if (cp.out_bit[sb.first][sb.second] != -1) throw std::logic_error("output bit placed twice");
            cp.out_bit[sb.first][sb.second] = kv.second;
          }
        } else if (st.kS == st.kN) {
          for (int l : F) posC[l] = posA[l];
          for (int i = 0; i < st.kN; ++i) posC[NN[i]] = posA[S[i]];
          st.inplace_ok = true;
        } else {
          for (int i = 0; i < (int)F.size(); ++i) posC[F[i]] = i;
          for (int i = 0; i < st.kN; ++i) posC[NN[i]] = int(F.size()) + i;
        }
        st.final_step = final_step;
        // rows: the lowest F legs
        // rows per tile: a tile of K x R elements with K * R <= 4096 (at least 2048 when the
        // tensor allows, so small operators still move 16 KB or more per tile), at most 256 rows,
        // and the LDS tile (K x (Nn + R) entries of 16 bytes) within 60 KB.  A complex64 step whose
        // output outgrows its input writes Nn runs of R contiguous elements per tile, and longer
        // runs stream faster (measured on MI355X: 2 KB runs 5.5 TB/s, 1 KB runs 5.1): it takes the
        // most rows the bounds allow, its LDS entries counted at 8 bytes
        const bool f32_widen = low && !(k >= switch_at || final_step) && opt.dtype == JF_C64 && st.kN > st.kS;
        const int lds_entries = f32_widen ? 7680 : 3840;
        int Lr = std::min<int>(int(F.size()), 8);
        while (Lr > 0 && ((1 << st.kS) * (1 << Lr) > 4096 || (1 << st.kS) * ((1 << st.kN) + (1 << Lr)) > lds_entries)) --Lr;
        while (!f32_widen && Lr > 6 && (1 << st.kS) * (1 << (Lr - 1)) >= 2048) --Lr;
        // a small intermediate: fewer rows per tile (16 at least, the MFMA block), so that there
        // are 256 tiles, one per compute unit, where the tensor allows: a tile's products are
        // then spread over more compute units instead of running one after another in a few
        while (Lr > 4 && int(F.size()) - Lr < 8) --Lr;
        st.L = Lr;
        std::vector<int> rowsA, rowsC, hiA, hiC, sA, nC;
        for (int i = 0; i < Lr; ++i) {
          rowsA.push_back(posA[F[i]]);
          rowsC.push_back(posC[F[i]]);
        }
        for (int i = Lr; i < (int)F.size(); ++i) {
          hiA.push_back(posA[F[i]]);
          hiC.push_back(posC[F[i]]);
        }
        for (int l : S) sA.push_back(posA[l]);
        for (int l : NN) nC.push_back(posC[l]);
        st.hiA = hiA;
        st.hiC = hiC;
        st.nTiles = 1LL << hiA.size();
        for (long long s = 0; s < (1LL << st.kS); ++s) st.offS_A.push_back(scatter(s, sA));
        for (long long r = 0; r < (1LL << Lr); ++r) {
          st.offR_A.push_back(scatter(r, rowsA));
          st.offR_C.push_back(scatter(r, rowsC));
        }
        for (long long n = 0; n < (1LL << st.kN); ++n) st.offN_C.push_back(scatter(n, nC));
        // B matrices [s][n] from the fused block tensor(s)
        const int K = 1 << st.kS, Nn = 1 << st.kN;
        for (auto& b : blk) {
          std::vector<int> sb(st.kS), nb(st.kN);
          for (int i = 0; i < st.kS; ++i) sb[i] = int(std::find(b.legs.begin(), b.legs.end(), S[i]) - b.legs.begin());
          for (int i = 0; i < st.kN; ++i) nb[i] = int(std::find(b.legs.begin(), b.legs.end(), NN[i]) - b.legs.begin());
          std::vector<cd> M(size_t(K) * Nn);
          for (int s = 0; s < K; ++s)
            for (int n = 0; n < Nn; ++n) {
              size_t idx = 0;
              for (int i = 0; i < st.kS; ++i) idx |= size_t((s >> i) & 1) << sb[i];
              for (int i = 0; i < st.kN; ++i) idx |= size_t((n >> i) & 1) << nb[i];
              M[size_t(s) * Nn + n] = b.data[idx];
            }
          st.B.push_back(std::move(M));
        }
        // precision of this step
        if (!low) {
          st.in_prec = st.out_prec = P_C128;
          st.compute = C_F64;
        } else {
          st.in_prec = cur_prec;
          bool fp64 = (k >= switch_at) || final_step;
          st.out_prec = fp64 ? P_C128 : P_C64;
          st.compute = fp64 ? C_F64 : (opt.dtype == JF_C64 ? C_F32 : C_SPLIT);
          cur_prec = st.out_prec;
          // Noise operators are near-identity blocks repeated at many sites: their FP32
          // rounding errors share a sign and add up linearly over the sites, so blocks that
          // carry one keep the operator as an FP32 pair (hi + lo), or in the split form a fourth
          // BF16 piece for the residual.  Gate-only blocks round with uncorrelated errors and
          // stay single.
          if (st.compute == C_F32 || st.compute == C_SPLIT)
            for (int q = k; q < e; ++q)
              if (L.ts[pth.order[q]]->site >= 0) st.two_term = true;
        }
        int ein = st.in_prec == P_C128 ? 16 : 8, eout = st.out_prec == P_C128 ? 16 : 8;
        st.flops = 8.0 * std::ldexp(1.0, int(F.size()) + st.kS + st.kN);
        st.bytes = std::ldexp(double(ein), st.rA) + std::ldexp(double(eout), st.rC);
        comp_flops += st.flops * mult;
        comp_bytes += st.bytes * mult;
        P.est_seconds += mult * (std::max(st.bytes / cm.bw, st.flops / cm.flops) + cm.launch);
        if (!final_step) {
          level_bytes[lv] = std::max(level_bytes[lv], size_t(eout) << st.rC);
          level_maxw[lv] = std::max(level_maxw[lv], st.rC);
        }
        cp.max_log2 = std::max({cp.max_log2, st.rA, final_step ? 0 : st.rC});
        // new intermediate layout
        int rC = st.rC;
        std::vector<int> nT(final_step ? 0 : rC, -1);
        if (!final_step)
          for (auto& kv : posC) nT[kv.second] = kv.first;
        Tlegs = nT;
        cp.steps.push_back(std::move(st));
        k = e;
      }
      Lv.last = int(cp.steps.size());
      if (!(opt.flags & JF_FLAG_NO_CHAIN)) P.est_seconds += mult * build_level_chains(cp, Lv.first, Lv.last, cm);
      Lv.max_log2 = level_maxw[lv];
      Lv.buf_bytes = std::max<size_t>(level_bytes[lv], 256);
      cp.levels.push_back(Lv);
    }
    cp.leaves = mult;
    // sliced wires: every leaf's final step writes a partial result that is added into the output
    for (auto& lv : cp.levels)
      if (lv.wire >= 0) {
        cp.accumulate = true;
        ++P.n_sliced_wires;
      }
    if (cp.accumulate) {
      cp.leaf_len = 1LL << cp.steps.back().rC;
      P.est_seconds += double(cp.leaves) * (cm.launch + 32.0 * double(cp.leaf_len) / cm.bw);
    }
    for (int si : comp_sites)
      for (int ob : cp.out_bit[si])
        if (ob < 0 || ob >= cp.n_open_bits) throw std::logic_error("Kraus bit without an output position");
    cp.lds_resident = cp.levels.size() == 1 && cp.levels[0].nvar == 1;
    for (auto& st : cp.steps)
      if (st.rA > LDS_RESIDENT_MAX || (!st.final_step && st.rC > LDS_RESIDENT_MAX)) cp.lds_resident = false;
    // outside the persistent kernel a component also clears its output (one fill launch) and sums
    // |t|^2 over it (two launches): with many open Kraus bits the output itself is large
    if (!cp.lds_resident) P.est_seconds += 2.0 * 16.0 * double(cp.out_len) / cm.bw + 3 * cm.launch;
    cp.flops = comp_flops;
    cp.bytes = comp_bytes;
    size_t cbuf = 0;
    for (auto& lv : cp.levels) cbuf += 2 * ((lv.buf_bytes + 255) / 256 * 256);
    max_comp_buf = std::max(max_comp_buf, cbuf);
    cp.out_off = out_total;
    out_total += cp.out_len;
    P.flops += cp.flops;
    P.bytes += cp.bytes;
    P.max_log2 = std::max(P.max_log2, cp.max_log2);
    P.work_items += cp.leaves;
    P.comps.push_back(std::move(cp));
  }
  // workspace: B pools | constants | level buffers | outputs | sums
  size_t pool = 0;
  for (auto& cp : P.comps)
    for (auto& st : cp.steps) {
      size_t e = st.compute == C_F64 ? 16 : 8;
      for (auto& b : st.B) pool += (b.size() * e + 255) / 256 * 256;
    }
  P.pool_bytes = pool;
  P.ws_bytes = pool + 256 + max_comp_buf + (size_t(out_total) * 16 + 255) / 256 * 256 +
               (P.comps.size() * 4 * 8 + 255) / 256 * 256;
  P.planner_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  std::string why;
  if (!validate_program(P, why)) {
    set_error("internal planner error: " + why);
    throw jf_status(JF_E_ARG);
  }
  return P;
}

}  // namespace jf
