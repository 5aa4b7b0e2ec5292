// Tensor networks of the two algorithms and their exact simplification.
//
// Algorithm I (Section IV-A, Fig. 4): the miter of the noisy circuit E and U^dagger (the ideal
// gates Hermitian-conjugated in reverse order), every output wire connected back to its input
// (Fig. 3: the trace as a closed network).  Every noise site becomes a "slot" tensor whose
// extra legs index its Kraus operators; leaving those legs open makes one network carry all
// prod_k n_k traces of Algorithm I at once.
//
// Algorithm II (Section IV-B, steps 1-4): wires q and q'; every gate V becomes V on q and V* on
// q'; every noise site N = {N_k} becomes M_N = sum_k N_k (x) N_k* on (q, q'); U^dagger (x) U^T
// closes the ring.
//
// Local optimisation (Section IV-C): adjacent gates whose product is the identity are removed,
// including across the closing wires at both ends of the miter.  Repeating it to a fixed point
// removes every gate outside the region between the first and the last noise site that those
// sites can reach, which is where the cost of the method lies.
#include <algorithm>
#include <cstring>
#include <functional>
#include <numeric>

#include "jf_internal.h"

namespace jf {

static cd op_entry(const GateOp& g, int dag, int conj, int r, int c) {
  int D = 1 << g.nq;
  cd v = dag ? std::conj(g.m[c * D + r]) : g.m[r * D + c];
  return conj ? std::conj(v) : v;
}

// Gate tensor: legs [in_0..in_{nq-1}, out_0..out_{nq-1}] (qubit j = g.q[j]); entry
// T[in bits | out bits << nq] = op(M)[row(out), col(in)], qubit 0 of the gate most significant.
static Tensor gate_tensor(const GateOp& g, int dag, int conj, const std::vector<int>& ins, const std::vector<int>& outs) {
  Tensor t;
  t.kind = T_GATE;
  t.src = &g;
  t.dag = dag;
  t.conj = conj;
  t.ins = ins;
  t.outs = outs;
  int nq = g.nq;
  t.legs = ins;
  t.legs.insert(t.legs.end(), outs.begin(), outs.end());
  t.data.assign(size_t(1) << (2 * nq), 0.0);
  for (int idx = 0; idx < (1 << (2 * nq)); ++idx) {
    int row = 0, col = 0;
    for (int j = 0; j < nq; ++j) {
      col = 2 * col + ((idx >> j) & 1);
      row = 2 * row + ((idx >> (nq + j)) & 1);
    }
    t.data[idx] = op_entry(g, dag, conj, row, col);
  }
  return t;
}

static int ceil_log2(int x) {
  int b = 0;
  while ((1 << b) < x) ++b;
  return b;
}

Network build_network(const jf_circuit& c, int alg) {
  Network net;
  net.n_qubits = c.n;
  net.alg = alg;
  const int n = c.n;
  const int W = alg == 1 ? n : 2 * n;
  int next_leg = 0;
  std::vector<int> start(W), cur(W);
  for (int w = 0; w < W; ++w) start[w] = cur[w] = next_leg++;
  auto advance = [&](const std::vector<int>& wires, std::vector<int>& ins, std::vector<int>& outs) {
    ins.clear();
    outs.clear();
    for (int w : wires) {
      ins.push_back(cur[w]);
      cur[w] = next_leg++;
      outs.push_back(cur[w]);
    }
  };
  net.site_var_legs.resize(c.sites.size());
  net.site_nk.resize(c.sites.size());

  auto add_gate = [&](const GateOp& g, int dag) {
    std::vector<int> ins, outs;
    std::vector<int> wq(g.q, g.q + g.nq);
    advance(wq, ins, outs);
    net.T.push_back(gate_tensor(g, dag, 0, ins, outs));
    if (alg == 2) {
      std::vector<int> wq2;
      for (int j = 0; j < g.nq; ++j) wq2.push_back(g.q[j] + n);
      advance(wq2, ins, outs);
      net.T.push_back(gate_tensor(g, dag, 1, ins, outs));
    }
  };
  auto add_site = [&](int si) {
    const NoiseSite& s = c.sites[si];
    net.site_nk[si] = s.nk;
    std::vector<int> ins, outs;
    if (alg == 1) {
      advance({s.qubit}, ins, outs);
      Tensor t;
      t.kind = T_SLOT;
      t.site = si;
      t.nk = s.nk;
      t.ins = ins;
      t.outs = outs;
      int v = ceil_log2(s.nk);
      t.legs = {ins[0], outs[0]};
      for (int b = 0; b < v; ++b) {
        t.var_legs.push_back(next_leg);
        t.legs.push_back(next_leg++);
      }
      net.site_var_legs[si] = t.var_legs;
      t.data.assign(size_t(4) << v, 0.0);
      for (int k = 0; k < s.nk; ++k)
        for (int in = 0; in < 2; ++in)
          for (int out = 0; out < 2; ++out) t.data[in | (out << 1) | (k << 2)] = s.kraus[4 * k + 2 * out + in];
      net.T.push_back(std::move(t));
    } else {
      advance({s.qubit, s.qubit + n}, ins, outs);
      // M_N[(a a'), (b b')] = sum_k K_k[a][b] conj(K_k[a'][b'])
      Tensor t;
      t.kind = T_NOISE;
      t.site = si;
      t.ins = ins;
      t.outs = outs;
      t.legs = {ins[0], ins[1], outs[0], outs[1]};
      t.data.assign(16, 0.0);
      for (int idx = 0; idx < 16; ++idx) {
        int b = idx & 1, bp = (idx >> 1) & 1, a = (idx >> 2) & 1, ap = (idx >> 3) & 1;
        cd acc = 0;
        for (int k = 0; k < s.nk; ++k) acc += s.kraus[4 * k + 2 * a + b] * std::conj(s.kraus[4 * k + 2 * ap + bp]);
        t.data[idx] = acc;
      }
      net.T.push_back(std::move(t));
    }
  };

  // noisy implementation E in time order (sites sorted by the gate they follow)
  size_t si = 0;
  while (si < c.sites.size() && c.sites[si].after == -1) add_site(int(si++));
  for (size_t g = 0; g < c.noisy.size(); ++g) {
    add_gate(c.noisy[g], 0);
    while (si < c.sites.size() && c.sites[si].after == int(g)) add_site(int(si++));
  }
  // U^dagger: ideal gates Hermitian-conjugated, in reverse order
  for (size_t g = c.ideal.size(); g-- > 0;) add_gate(c.ideal[g], 1);
  // close every wire: its last leg is its first leg
  std::vector<int> ren(next_leg);
  std::iota(ren.begin(), ren.end(), 0);
  for (int w = 0; w < W; ++w) ren[cur[w]] = start[w];
  net.leg_alive.assign(next_leg, 1);
  for (int w = 0; w < W; ++w)
    if (cur[w] != start[w]) net.leg_alive[cur[w]] = 0;
  for (auto& t : net.T) {
    for (auto& l : t.legs) l = ren[l];
    for (auto& l : t.ins) l = ren[l];
    for (auto& l : t.outs) l = ren[l];
  }
  net.n_before_cancel = int(net.T.size());
  // normalisation: Alg I returns t_k/d, Alg II returns T/d^2 (exact powers of two)
  net.log2_scale = alg == 1 ? -double(n) : -2.0 * n;
  return net;
}

// --------------------------------------------------------------------------- cancellation --

static bool is_inverse_pair(const Tensor& a, const Tensor& b) {
  if (a.kind != T_GATE || b.kind != T_GATE || !a.src || !b.src) return false;
  if (a.dag == b.dag || a.conj != b.conj) return false;
  const GateOp& ga = *a.src;
  const GateOp& gb = *b.src;
  if (ga.nq != gb.nq) return false;
  for (int j = 0; j < ga.nq; ++j)
    if (ga.q[j] != gb.q[j]) return false;
  int D = 1 << ga.nq;
  for (int i = 0; i < D * D; ++i)
    if (ga.m[i] != gb.m[i]) return false;
  return a.outs == b.ins;
}

void cancel_inverse_pairs(Network& net) {
  int max_leg = 0;
  for (auto& t : net.T)
    for (int l : t.legs) max_leg = std::max(max_leg, l);
  std::vector<std::vector<int>> refs(max_leg + 1);
  for (int i = 0; i < (int)net.T.size(); ++i)
    for (int l : net.T[i].legs) refs[l].push_back(i);
  std::vector<char> alive(net.T.size(), 1);
  std::vector<int> work(net.T.size());
  std::iota(work.begin(), work.end(), 0);
  auto other = [&](int leg, int self) {
    for (int t : refs[leg])
      if (t != self) return t;
    return -1;
  };
  auto replace_leg = [&](Tensor& t, int from, int to) {
    for (auto& l : t.legs) if (l == from) l = to;
    for (auto& l : t.ins) if (l == from) l = to;
    for (auto& l : t.outs) if (l == from) l = to;
  };
  while (!work.empty()) {
    int a = work.back();
    work.pop_back();
    if (!alive[a] || net.T[a].kind != T_GATE || net.T[a].outs.empty()) continue;
    Tensor& A = net.T[a];
    int b = other(A.outs[0], a);
    if (b < 0 || !alive[b]) continue;
    Tensor& B = net.T[b];
    if (!is_inverse_pair(A, B)) continue;
    alive[a] = alive[b] = 0;
    for (int l : A.outs) net.leg_alive[l] = 0;
    // drop the references of A and B
    for (int l : A.legs) refs[l].erase(std::remove(refs[l].begin(), refs[l].end(), a), refs[l].end());
    for (int l : B.legs) refs[l].erase(std::remove(refs[l].begin(), refs[l].end(), b), refs[l].end());
    // B.outs[j] becomes A.ins[j]
    for (size_t j = 0; j < B.outs.size(); ++j) {
      int from = B.outs[j], to = A.ins[j];
      if (from == to) continue;
      net.leg_alive[from] = 0;
      std::vector<int> rs = refs[from];
      for (int t : rs) {
        replace_leg(net.T[t], from, to);
        refs[to].push_back(t);
      }
      refs[from].clear();
    }
    // neighbours of the removed pair may now form new adjacent pairs
    for (int l : A.ins)
      for (int t : refs[l]) work.push_back(t);
  }
  std::vector<Tensor> kept;
  for (size_t i = 0; i < net.T.size(); ++i)
    if (alive[i]) kept.push_back(std::move(net.T[i]));
  net.T = std::move(kept);
}

// SWAP gates carry no arithmetic (Section IV-C lists the exact simplifications): each one left
// after the cancellation is removed and its wires are joined crosswise, the out leg of qubit j
// becoming the in leg of the other qubit (its entry is 1 exactly where out_0 = in_1 and
// out_1 = in_0, for U, U^dagger and their conjugates alike).  Joins are taken with union-find,
// so runs of SWAPs collapse; a wire closed on itself by SWAPs alone ends as an empty loop.
int rewire_swaps(Network& net) {
  auto is_swap = [](const Tensor& t) {
    if (t.kind != T_GATE || !t.src || t.src->nq != 2 || t.ins.size() != 2 || t.outs.size() != 2) return false;
    for (int r = 0; r < 4; ++r)
      for (int c = 0; c < 4; ++c) {
        const bool one = c == ((r & 1) << 1 | (r >> 1));
        if (t.src->m[r * 4 + c] != cd(one ? 1.0 : 0.0, 0.0)) return false;
      }
    return true;
  };
  std::vector<int> parent(net.leg_alive.size());
  std::iota(parent.begin(), parent.end(), 0);
  std::function<int(int)> find = [&](int x) { return parent[x] == x ? x : parent[x] = find(parent[x]); };
  auto join = [&](int a, int b) {
    a = find(a);
    b = find(b);
    if (a == b) return;
    if (a < b) std::swap(a, b);
    parent[a] = b;  // the smaller id stays
    net.leg_alive[a] = 0;
  };
  std::vector<Tensor> kept;
  int removed = 0;
  for (auto& t : net.T) {
    if (is_swap(t)) {
      join(t.outs[0], t.ins[1]);
      join(t.outs[1], t.ins[0]);
      ++removed;
    } else {
      kept.push_back(std::move(t));
    }
  }
  for (auto& t : kept) {
    for (auto& l : t.legs) l = find(l);
    for (auto& l : t.ins) l = find(l);
    for (auto& l : t.outs) l = find(l);
    for (auto& l : t.var_legs) l = find(l);
  }
  net.T = std::move(kept);
  return removed;
}

// Empty loops: a wire whose every tensor was cancelled leaves one live leg that no tensor
// references; it is a closed loop worth tr(I_2) = 2.
int count_empty_loops(const Network& net) {
  std::vector<char> used(net.leg_alive.size(), 0);
  for (auto& t : net.T)
    for (int l : t.legs) used[l] = 1;
  int e = 0;
  for (size_t l = 0; l < net.leg_alive.size(); ++l) e += net.leg_alive[l] && !used[l];
  return e;
}

void trace_self_loops(Network& net) {
  std::vector<Tensor> kept;
  for (auto& t : net.T) {
    bool dup = true;
    while (dup) {
      dup = false;
      int r = int(t.legs.size());
      for (int i = 0; i < r && !dup; ++i)
        for (int j = i + 1; j < r && !dup; ++j)
          if (t.legs[i] == t.legs[j]) {
            dup = true;
            Tensor u = t;
            u.legs.clear();
            for (int k = 0; k < r; ++k)
              if (k != i && k != j) u.legs.push_back(t.legs[k]);
            u.data.assign(size_t(1) << u.legs.size(), 0.0);
            for (size_t idx = 0; idx < t.data.size(); ++idx) {
              if (((idx >> i) & 1) != ((idx >> j) & 1)) continue;
              size_t o = 0;
              int ob = 0;
              for (int k = 0; k < r; ++k) {
                if (k == i || k == j) continue;
                o |= ((idx >> k) & 1) << ob;
                ++ob;
              }
              u.data[o] += t.data[idx];
            }
            u.ins.clear();
            u.outs.clear();
            u.kind = T_OTHER;
            t = std::move(u);
          }
    }
    if (t.legs.empty()) {
      net.scalar *= t.data[0];
      continue;
    }
    kept.push_back(std::move(t));
  }
  net.T = std::move(kept);
}

std::vector<std::vector<int>> components(const Network& net) {
  int N = int(net.T.size());
  std::vector<int> par(N);
  std::iota(par.begin(), par.end(), 0);
  std::function<int(int)> find = [&](int x) { return par[x] == x ? x : par[x] = find(par[x]); };
  int max_leg = 0;
  for (auto& t : net.T)
    for (int l : t.legs) max_leg = std::max(max_leg, l);
  std::vector<int> owner(max_leg + 1, -1);
  for (int i = 0; i < N; ++i)
    for (int l : net.T[i].legs) {
      if (owner[l] < 0) owner[l] = i;
      else par[find(i)] = find(owner[l]);
    }
  std::vector<std::vector<int>> comps;
  std::vector<int> id(N, -1);
  for (int i = 0; i < N; ++i) {
    int r = find(i);
    if (id[r] < 0) {
      id[r] = int(comps.size());
      comps.emplace_back();
    }
    comps[id[r]].push_back(i);
  }
  return comps;
}

// --------------------------------------------------------------------- small host algebra --

Tensor contract_pair(const Tensor& a, const Tensor& b) {
  std::vector<int> shared, fa, fb;  // positions
  std::vector<int> sa, sb;
  for (int i = 0; i < (int)a.legs.size(); ++i) {
    auto it = std::find(b.legs.begin(), b.legs.end(), a.legs[i]);
    if (it != b.legs.end()) {
      sa.push_back(i);
      sb.push_back(int(it - b.legs.begin()));
    } else {
      fa.push_back(i);
    }
  }
  for (int j = 0; j < (int)b.legs.size(); ++j)
    if (std::find(a.legs.begin(), a.legs.end(), b.legs[j]) == a.legs.end()) fb.push_back(j);
  Tensor c;
  for (int i : fa) c.legs.push_back(a.legs[i]);
  for (int j : fb) c.legs.push_back(b.legs[j]);
  int rc = int(c.legs.size()), ks = int(sa.size());
  c.data.assign(size_t(1) << rc, 0.0);
  for (size_t ci = 0; ci < c.data.size(); ++ci) {
    size_t ia = 0, ib = 0;
    for (int k = 0; k < (int)fa.size(); ++k) ia |= ((ci >> k) & 1) << fa[k];
    for (int k = 0; k < (int)fb.size(); ++k) ib |= ((ci >> (fa.size() + k)) & 1) << fb[k];
    cd acc = 0;
    for (size_t s = 0; s < (size_t(1) << ks); ++s) {
      size_t ja = ia, jb = ib;
      for (int k = 0; k < ks; ++k) {
        ja |= ((s >> k) & 1) << sa[k];
        jb |= ((s >> k) & 1) << sb[k];
      }
      acc += a.data[ja] * b.data[jb];
    }
    c.data[ci] = acc;
  }
  c.kind = T_OTHER;
  return c;
}

}  // namespace jf
