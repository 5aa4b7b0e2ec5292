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
      if (K > MAXK || Nn > MAXK || R > MAXR || (int)st.hiA.size() > MAXHI || (int)st.offS_A.size() != K ||
          (int)st.offN_C.size() != Nn || (int)st.offR_A.size() != R || st.nTiles != (1LL << st.hiA.size()) ||
          size_t(K) * (Nn + R) * 16 > 61440) {
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
      const long long sizeC = st.final_step ? cp.out_len : (1LL << st.rC);
      if (maxA >= sizeA || maxC >= sizeC) {
        why = "step " + std::to_string(s) + " addresses outside its tensors";
        return false;
      }
      for (auto& b : st.B)
        if ((long long)b.size() != (long long)K * Nn) {
          why = "operator block size mismatch";
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

void assemble_result(const Program& p, const std::vector<CompSum>& sums, jf_result* out) {
  jf_result r = {};
  const double s = std::exp2(p.log2_scale);  // exact: an integer power of two
  if (p.opt.alg == 1) {
    // F_J = (s |scalar|)^2 * prod_c sum_k |t_ck|^2, each sum a double-double (hi, lo)
    double a = s * s * std::norm(p.scalar);
    double hi = a, lo = 0;
    for (auto& cs : sums) {
      double h = hi * cs.hi;
      double l = std::fma(hi, cs.hi, -h) + hi * cs.lo + lo * cs.hi;
      hi = h + l;
      lo = l - (hi - h);
    }
    r.fj = hi + lo;
    // 1 - F_J: 1 - hi is exact when hi is in [0.5, 2] (Sterbenz); then subtract lo
    r.one_minus_fj = (1.0 - hi) - lo;
    r.imag_residual = 0;
  } else {
    cd v = s * p.scalar;
    for (auto& cs : sums) v *= cs.value;
    r.fj = v.real();
    r.one_minus_fj = 1.0 - v.real();
    r.imag_residual = std::abs(v.imag());
  }
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
        if (p.site_comp[i] == int(c)) o |= (long long)j[i] << p.comps[c].out_site_shift[i];
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

void emulate_level(const ComponentProgram& cp, int lv, const std::vector<cd>& parent, long long out_base,
                   std::vector<cd>& out) {
  const Level& L = cp.levels[lv];
  for (int v = 0; v < L.nvar; ++v) {
    std::vector<cd> cur = parent, nxt;
    for (int si = L.first; si < L.last; ++si) {
      const Step& st = cp.steps[si];
      const std::vector<cd>& B = st.B[si == L.first && L.site >= 0 ? v : 0];
      if (st.final_step) {
        emulate_step(st, B, cur.data(), out.data() + out_base + v * L.out_stride);
      } else {
        nxt.assign(size_t(1) << st.rC, 0.0);
        emulate_step(st, B, cur.data(), nxt.data());
        cur.swap(nxt);
      }
    }
    if (lv + 1 < (int)cp.levels.size()) emulate_level(cp, lv + 1, cur, out_base + v * L.out_stride, out);
  }
}

}  // namespace

void emulate_program(const Program& p, std::vector<std::vector<cd>>& comp_out) {
  comp_out.clear();
  for (auto& cp : p.comps) {
    std::vector<cd> out(size_t(cp.out_len), 0.0);
    std::vector<cd> one(1, 1.0);
    emulate_level(cp, 0, one, 0, out);
    comp_out.push_back(std::move(out));
  }
}

}  // namespace jf
