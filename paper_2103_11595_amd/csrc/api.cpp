// C ABI: argument checking, planning entry points and handle management.  The GPU entry points
// (jf_fidelity_alg1/alg2/batch, jf_batch_workspace) live in executor.hip.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <exception>
#include <string>

#include "jf_internal.h"

namespace jf {
static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
}  // namespace jf

using namespace jf;

extern "C" const char* jf_last_error(void) { return g_err.c_str(); }

extern "C" jf_status jf_plan_contraction(const jf_circuit* c, int alg, jf_dtype dtype, int max_log2, unsigned flags,
                                         jf_plan** out) {
  if (c && out && alg == 0) {
    // Algorithm I grows with the number of Kraus tuples, Algorithm II with the doubled wires
    // (Section IV): plan both and keep the one with the smaller estimated device time.
    jf_plan *p1 = nullptr, *p2 = nullptr;
    const jf_status s1 = jf_plan_contraction(c, 1, dtype, max_log2, flags, &p1);
    const std::string e1 = s1 == JF_OK ? std::string() : std::string(jf_last_error());
    const jf_status s2 = jf_plan_contraction(c, 2, dtype, max_log2, flags, &p2);
    if (s1 != JF_OK && s2 != JF_OK) {
      set_error("jf_plan_contraction: neither algorithm plans: " + e1 + "; " + jf_last_error());
      return s2;
    }
    const bool take1 = s2 != JF_OK || (s1 == JF_OK && p1->prog.est_seconds <= p2->prog.est_seconds);
    *out = take1 ? p1 : p2;
    jf_free_plan(take1 ? p2 : p1);
    return JF_OK;
  }
  if (!c || !out || (alg != 1 && alg != 2) || dtype < JF_C128 || dtype > JF_C64_BF16X6) {
    set_error("jf_plan_contraction: bad argument");
    return JF_E_ARG;
  }
  PlanOptions opt;
  opt.alg = alg;
  opt.dtype = dtype;
  opt.cap_log2 = max_log2 > 0 ? max_log2 : 30;  // 8 GiB (c64) / 16 GiB (c128) per buffer: MI355X holds 288 GB
  if (opt.cap_log2 > 36) {
    set_error("jf_plan_contraction: max_log2_intermediate above 36");
    return JF_E_ARG;
  }
  opt.flags = flags;
  const unsigned effort = (flags >> 8) & 15u;
  if (effort) opt.restarts = 1 << (effort + 5);
  opt.kmax = 6;  // blocks of up to 64 x 64: the Gauss-form MFMA kernels keep them HBM-bound
  try {
    auto p = new jf_plan;
    p->prog = plan_program(*c, opt);
    *out = p;
    return JF_OK;
  } catch (jf_status st) {
    return st;
  } catch (std::exception& e) {
    set_error(std::string("planner: ") + e.what());
    return JF_E_ARG;
  }
}

namespace jf {
size_t plan_workspace_bytes(jf_plan* p);  // executor.hip: exact device layout of the plan
}

extern "C" jf_status jf_plan_info(const jf_plan* p, size_t* ws, jf_result* costs) {
  if (!p) {
    set_error("jf_plan_info: NULL plan");
    return JF_E_ARG;
  }
  if (ws) *ws = plan_workspace_bytes(const_cast<jf_plan*>(p));
  if (costs) {
    jf_result r = {};
    r.kraus_terms = p->prog.kraus_terms;
    r.work_items = p->prog.work_items;
    r.max_log2_intermediate = p->prog.max_log2;
    r.path_flops = p->prog.flops;
    r.path_bytes = p->prog.bytes;
    *costs = r;
  }
  return JF_OK;
}

extern "C" jf_status jf_plan_stats_get(const jf_plan* p, jf_plan_stats* s) {
  if (!p || !s) {
    set_error("jf_plan_stats_get: bad argument");
    return JF_E_ARG;
  }
  jf_plan_stats r = {};
  for (auto& cp : p->prog.comps) r.n_steps += int(cp.steps.size());
  r.n_components = int(p->prog.comps.size());
  for (auto& cp : p->prog.comps)
    for (auto& lv : cp.levels) r.n_sliced_sites += lv.site >= 0;
  for (auto& cp : p->prog.comps) r.n_open_bits += cp.n_open_bits;
  r.n_tensors_before_cancel = p->prog.n_before_cancel;
  r.n_tensors_after_cancel = p->prog.n_after_cancel;
  r.planner_seconds = p->prog.planner_seconds;
  r.empty_loops = p->prog.empty_loops;
  r.alg = p->prog.opt.alg;
  r.est_seconds = p->prog.est_seconds;
  r.n_swaps_rewired = p->prog.n_swaps_rewired;
  r.n_sliced_wires = p->prog.n_sliced_wires;
  *s = r;
  return JF_OK;
}

extern "C" jf_status jf_emulate_plan(const jf_plan* p, double* out, long long out_len) {
  if (!p || !out) {
    set_error("jf_emulate_plan: bad argument");
    return JF_E_ARG;
  }
  const Program& P = p->prog;
  long long need = P.opt.alg == 1 ? 2 * P.kraus_terms : 2;
  if (out_len < need) {
    set_error("jf_emulate_plan: output too short");
    return JF_E_ARG;
  }
  std::vector<std::vector<cd>> co;
  emulate_program(P, co);
  if (P.opt.alg == 1) {
    gather_terms(P, co, out);
  } else {
    cd v = std::exp2(P.log2_scale) * P.scalar;
    for (auto& c : co) v *= c[0];
    out[0] = v.real();
    out[1] = v.imag();
  }
  return JF_OK;
}

extern "C" int jf_is_equivalent(const jf_result* r, double eps) {
  if (!r) return -1;
  return r->fj > 1.0 - eps ? 1 : 0;
}

extern "C" void jf_free_plan(jf_plan* p);  // executor.hip (releases device state too)

extern "C" long long jf_plan_describe(const jf_plan* p, char* buf, long long len) {
  if (!p) return -1;
  std::string out;
  const char* pn[] = {"c128", "c64"};
  const char* cn[] = {"f64", "f32", "split"};
  for (size_t c = 0; c < p->prog.comps.size(); ++c) {
    const ComponentProgram& cp = p->prog.comps[c];
    for (size_t lv = 0; lv < cp.levels.size(); ++lv)
      for (int s = cp.levels[lv].first; s < cp.levels[lv].last; ++s) {
        const Step& st = cp.steps[s];
        char line[256];
        snprintf(line, sizeof(line), "%zu %d %zu %d %d %d %d %d %lld %s %s %s %d %.6g %.6g", c, s, lv, st.kS, st.kN, st.L,
                 st.rA, st.rC, st.nTiles, pn[st.in_prec], pn[st.out_prec],
                 (st.compute == C_F32 && st.two_term) ? "f32x2" : (st.compute == C_SPLIT && st.two_term) ? "split4"
                                                                                            : cn[st.compute],
                 st.nvar, st.flops, st.bytes);
        out += line;
        // bit positions (in A, resp. C) of the tile rows, the summed legs and the new legs
        auto bits = [](const std::vector<long long>& off, int n) {
          std::string b;
          for (int i = 0; i < n; ++i) {
            const long long v = off[size_t(1) << i];
            int pos = 0;
            while ((1LL << pos) < v) ++pos;
            b += (i ? "," : "") + std::to_string(pos);
          }
          return b.empty() ? std::string("-") : b;
        };
        out += " " + bits(st.offR_A, st.L) + " " + bits(st.offR_C, st.L) + " " + bits(st.offS_A, st.kS) + " " +
               bits(st.offN_C, st.kN) + " " + std::to_string(st.chain) + "\n";
      }
  }
  if (buf && len > 0) {
    long long n = std::min<long long>(len - 1, (long long)out.size());
    memcpy(buf, out.data(), size_t(n));
    buf[n] = 0;
  }
  return (long long)out.size() + 1;
}
