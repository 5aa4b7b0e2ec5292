// Result assembly shared by the GPU executor and the host emulation, and the host emulation
// itself.  The emulation runs a plan's step program in FP64 with the very offset tables the
// GPU kernels read; it exists so that the CPU test suite can validate the planner, slicing,
// block fusion and output placement.  No fidelity entry point calls it.
#include <algorithm>
#include <cmath>
#include <string>

#include "jf_internal.h"

namespace jf {

// Largest element index a step touches in A and in C must lie inside the tensors (and inside
// the level buffer / output array that hold them).  Checked on the host before any launch.
bool validate_program(const Program& P, std::string& why) {
  for (size_t c = 0; c < P.comps.size(); ++c) {
    const ComponentProgram& cp = P.comps[c];
    for (size_t s = 0; s < cp.steps.size(); ++s) {
      const Step& st = cp.steps[s];
      const int K = 1 << st.kS, Nn = 1 << st.kN, R = 1 << st.L;
      const size_t entry = st.compute == C_F64 ? 16 : 8;  // LDS bytes per operator / tile entry
      if (K > MAXK || Nn > MAXK || R > MAXR || (int)st.hiA.size() > MAXHI || (int)st.offS_A.size() != K ||
          (int)st.offN_C.size() != Nn || (int)st.offR_A.size() != R || st.nTiles != (1LL << st.hiA.size()) ||
          size_t(K) * (Nn + R) * entry > 61440) {
        why = "step table sizes out of range";
        return false;
      }
      long long maxA = 0, maxC = 0;
      long long mS = 0, mRA = 0, mN = 0, mRC = 0, hA = 0, hC = 0;
      for (auto v : st.offS_A) mS = std::max(mS, v);
      for (auto v : st.offR_A) mRA = std::max(mRA, v);
      for (auto v : st.offN_C) mN = std::max(mN, v);
      for (auto v : st.offR_C) mRC = std::max(mRC, v);
      for (size_t b = 0; b < st.hiA.size(); ++b) {
        hA += 1LL << st.hiA[b];
        hC += 1LL << st.hiC[b];
      }
      maxA = hA + mS + mRA;
      maxC = hC + mN + mRC;
      const long long sizeA = 1LL << st.rA;
      const long long sizeC = st.final_step ? (cp.accumulate ? cp.leaf_len : cp.out_len) : (1LL << st.rC);
      if (maxA >= sizeA || maxC >= sizeC) {
        why = "step " + std::to_string(s) + " addresses outside its tensors";
        return false;
      }
      for (auto& b : st.B)
        if ((long long)b.size() != (long long)K * Nn) {
          why = "operator block size mismatch";
          return false;
        }
      // operator variants: one per combination of the values of levels at or above the step's own
      int own = -1;
      for (size_t l = 0; l < cp.levels.size(); ++l)
        if ((int)s >= cp.levels[l].first && (int)s < cp.levels[l].last) own = int(l);
      long long nv = 1;
      int prev = -1;
      for (int lv : st.var_levels) {
        if (lv <= prev || lv > own) {
          why = "step " + std::to_string(s) + " depends on a level it does not lie in";
          return false;
        }
        prev = lv;
        nv *= cp.levels[lv].nvar;
      }
      if ((long long)st.B.size() != nv) {
        why = "step " + std::to_string(s) + " has the wrong number of operator variants";
        return false;
      }
    }
    for (size_t q = 0; q < cp.chains.size(); ++q) {
      const Chain& ch = cp.chains[q];
      const int rA = (ch.first >= 0 && ch.first < (int)cp.steps.size()) ? cp.steps[ch.first].rA : -1;
      bool ok = ch.first >= 0 && ch.last <= (int)cp.steps.size() && ch.last - ch.first >= 2 &&
                ch.last - ch.first <= CHAIN_MAX_STEPS && ch.T >= 4 && ch.T <= CHAIN_MAX_T &&
                (int)ch.P.size() == ch.T && (int)ch.hi.size() <= MAXHI && ch.nTiles == (1LL << ch.hi.size()) &&
                ch.T + (int)ch.hi.size() == rA;
      std::vector<char> seen(rA > 0 ? rA : 0, 0);
      for (int b : ch.P) ok = ok && b >= 0 && b < rA && !seen[b] && (seen[b] = 1);
      for (int b : ch.hi) ok = ok && b >= 0 && b < rA && !seen[b] && (seen[b] = 1);
      for (int b = 0; b < 4 && b < rA; ++b) ok = ok && std::count(ch.P.begin(), ch.P.end(), b) == 1;  // whole lines
      int ops = 0, lvl = -1;
      for (int s = ch.first; ok && s < ch.last; ++s) {
        const Step& st = cp.steps[s];
        ok = chainable(st) && st.chain == int(q) && st.rA == rA && ch.T - st.kS >= 4;
        for (int b : step_s_positions(st)) ok = ok && std::count(ch.P.begin(), ch.P.end(), b) == 1;
        ops += chain_step_ops(st.kS, st.compute == C_SPLIT, st.two_term);
        for (size_t l = 0; l < cp.levels.size(); ++l)
          if (s >= cp.levels[l].first && s < cp.levels[l].last) {
            if (lvl < 0) lvl = int(l);
            ok = ok && lvl == int(l);
          }
      }
      const bool split = ch.first < (int)cp.steps.size() && cp.steps[ch.first].compute == C_SPLIT;
      for (int s = ch.first; ok && s < ch.last; ++s) ok = (cp.steps[s].compute == C_SPLIT) == split;
      if (!ok || ops > (split ? CHAIN_MAX_OPS_SPLIT : CHAIN_MAX_OPS)) {
        why = "chain " + std::to_string(q) + " of component " + std::to_string(c) + " is malformed";
        return false;
      }
    }
    for (size_t s = 0; s < cp.steps.size(); ++s) {
      const int q = cp.steps[s].chain;
      if (q >= 0 && (q >= (int)cp.chains.size() || (int)s < cp.chains[q].first || (int)s >= cp.chains[q].last)) {
        why = "step " + std::to_string(s) + " names a chain that does not hold it";
        return false;
      }
    }
    {  // the offsets of the Kraus-site levels and a leaf's output stay inside the output array
      long long top = 0;
      for (auto& lv : cp.levels) top += (lv.nvar - 1) * lv.out_stride;
      const long long span = cp.accumulate ? cp.leaf_len : 1;
      if (top + span > cp.out_len || (cp.accumulate && cp.leaf_len < 1)) {
        why = "component " + std::to_string(c) + " output offsets exceed its array";
        return false;
      }
    }
    for (auto& lv : cp.levels)
      for (int s = lv.first; s < lv.last; ++s) {
        const Step& st = cp.steps[s];
        size_t e = st.out_prec == P_C128 ? 16 : 8;
        if (!st.final_step && (size_t(e) << st.rC) > lv.buf_bytes) {
          why = "level buffer smaller than a step output";
          return false;
        }
      }
  }
  return true;
}

void static_result(const Program& p, jf_result* out) {
  jf_result r = {};
  r.kraus_terms = p.kraus_terms;
  r.work_items = p.work_items;
  r.max_log2_intermediate = p.max_log2;
  r.path_flops = p.flops;
  r.path_bytes = p.bytes;
  *out = r;
}

void gather_terms(const Program& p, const std::vector<std::vector<cd>>& comp_out, double* tt) {
  const int m = int(p.site_nk.size());
  const double s = std::exp2(p.log2_scale);
  std::vector<int> j(m, 0);
  long long idx = 0;
  while (true) {
    cd t = s * p.scalar;
    for (size_t c = 0; c < p.comps.size(); ++c) {
      long long o = 0;
      for (int i = 0; i < m; ++i)
        if (p.site_comp[i] == int(c)) {
          const std::vector<int>& ob = p.comps[c].out_bit[i];
          for (size_t b = 0; b < ob.size(); ++b) o |= (long long)((j[i] >> b) & 1) << ob[b];
        }
      t *= comp_out[c][o];
    }
    tt[2 * idx] = t.real();
    tt[2 * idx + 1] = t.imag();
    ++idx;
    int i = m - 1;
    while (i >= 0 && ++j[i] == p.site_nk[i]) j[i--] = 0;
    if (i < 0) break;
  }
}

namespace {

// C[baseC + offN[n] + offRC[r]] = sum_s A[baseA + offS[s] + offRA[r]] * B[s][n]
void emulate_step(const Step& st, const std::vector<cd>& B, const cd* A, cd* C) {
  const int K = 1 << st.kS, Nn = 1 << st.kN, R = 1 << st.L;
  std::vector<cd> tile(size_t(K) * R);
  for (long long t = 0; t < st.nTiles; ++t) {
    long long bA = 0, bC = 0;
    for (size_t b = 0; b < st.hiA.size(); ++b)
      if ((t >> b) & 1) {
        bA |= 1LL << st.hiA[b];
        bC |= 1LL << st.hiC[b];
      }
    for (int s = 0; s < K; ++s)
      for (int r = 0; r < R; ++r) tile[size_t(s) * R + r] = A[bA + st.offS_A[s] + st.offR_A[r]];
    for (int n = 0; n < Nn; ++n)
      for (int r = 0; r < R; ++r) {
        cd acc = 0;
        for (int s = 0; s < K; ++s) acc += tile[size_t(s) * R + r] * B[size_t(s) * Nn + n];
        C[bC + st.offN_C[n] + st.offR_C[r]] = acc;
      }
  }
}

// A chain on the host with the tile-local tables of the chain kernel: per tile, gather 2^T
// elements, apply every step of the chain in place on the tile, scatter the tile back.
void emulate_chain(const ComponentProgram& cp, const Chain& ch, const std::vector<const std::vector<cd>*>& Bs,
                   std::vector<cd>& X) {
  ChainTables tb;
  chain_tables(cp, ch, tb);
  const int E = 1 << ch.T;
  std::vector<cd> tile(E);
  for (long long t = 0; t < ch.nTiles; ++t) {
    long long base = 0;
    for (size_t b = 0; b < ch.hi.size(); ++b)
      if ((t >> b) & 1) base |= 1LL << ch.hi[b];
    auto goff = [&](int l) { return tb.gDig[0][l & 15] + tb.gDig[1][(l >> 4) & 15] + tb.gDig[2][(l >> 8) & 15]; };
    for (int l = 0; l < E; ++l) tile[l] = X[base + goff(l)];
    for (int j = 0; j < ch.last - ch.first; ++j) {
      const Step& st = cp.steps[ch.first + j];
      const int K = 1 << st.kS, nf = 1 << (ch.T - st.kS);
      const std::vector<unsigned short>& so = tb.sOff[j];
      const std::vector<unsigned short>& fd = tb.fDig[j];
      const std::vector<cd>& B = *Bs[j];
      std::vector<cd> a(K);
      for (int f = 0; f < nf; ++f) {
        const int fl = fd[f & 15] + fd[16 + ((f >> 4) & 15)] + fd[32 + ((f >> 8) & 15)];
        for (int s = 0; s < K; ++s) a[s] = tile[fl + so[s]];
        for (int n = 0; n < K; ++n) {
          cd acc = 0;
          for (int s = 0; s < K; ++s) acc += a[s] * B[size_t(s) * K + n];
          tile[fl + so[n]] = acc;
        }
      }
    }
    for (int l = 0; l < E; ++l) X[base + goff(l)] = tile[l];
  }
}

void emulate_level(const ComponentProgram& cp, int lv, const std::vector<cd>& parent, long long out_base,
                   std::vector<int>& vv, std::vector<cd>& out) {
  const Level& L = cp.levels[lv];
  for (int v = 0; v < L.nvar; ++v) {
    vv[lv] = v;
    std::vector<cd> cur = parent, nxt;
    for (int si = L.first; si < L.last; ++si) {
      const Step& st = cp.steps[si];
      const std::vector<cd>& B = st.B[variant_index(cp, st, vv)];
      if (st.chain >= 0 && cp.chains[st.chain].first == si) {
        const Chain& ch = cp.chains[st.chain];
        std::vector<const std::vector<cd>*> Bs;
        for (int q = ch.first; q < ch.last; ++q) Bs.push_back(&cp.steps[q].B[variant_index(cp, cp.steps[q], vv)]);
        emulate_chain(cp, ch, Bs, cur);
        si = ch.last - 1;
        continue;
      }
      if (st.final_step) {
        cd* dst = out.data() + out_base + v * L.out_stride;
        if (cp.accumulate) {  // a partial result of the sliced wires: added in
          std::vector<cd> leaf(size_t(cp.leaf_len), 0.0);
          emulate_step(st, B, cur.data(), leaf.data());
          for (long long i = 0; i < cp.leaf_len; ++i) dst[i] += leaf[size_t(i)];
        } else {
          emulate_step(st, B, cur.data(), dst);
        }
      } else {
        nxt.assign(size_t(1) << st.rC, 0.0);
        emulate_step(st, B, cur.data(), nxt.data());
        cur.swap(nxt);
      }
    }
    if (lv + 1 < (int)cp.levels.size()) emulate_level(cp, lv + 1, cur, out_base + v * L.out_stride, vv, out);
  }
}

}  // namespace

void emulate_program(const Program& p, std::vector<std::vector<cd>>& comp_out) {
  comp_out.clear();
  for (auto& cp : p.comps) {
    std::vector<cd> out(size_t(cp.out_len), 0.0);
    std::vector<cd> one(1, 1.0);
    std::vector<int> vv(cp.levels.size(), 0);
    emulate_level(cp, 0, one, 0, vv, out);
    comp_out.push_back(std::move(out));
  }
}

}  // namespace jf
