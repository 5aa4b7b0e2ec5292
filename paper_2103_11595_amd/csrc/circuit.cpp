// Ingest of the ideal circuit, its noisy implementation and the noise sites (Problem 1), with
// the validity checks of Section II: gates are unitary, noise sites are Kraus sets with
// sum_i E_i^dagger E_i = I (Section II-B).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "jf_internal.h"

namespace jf {

static const double kR2 = 0.70710678118654752440;

// Gate matrices (Section II-A, Example 1).  Two-qubit matrices act on (q0, q1) with q0 the
// more significant bit; CX/CZ/CS are controlled on q0.
static bool gate_matrix(const jf_gate& g, GateOp& op) {
  cd* m = op.m;
  for (int i = 0; i < 16; ++i) m[i] = 0.0;
  const cd I(0.0, 1.0);
  auto set2 = [&](cd a, cd b, cd c, cd d) { m[0] = a; m[1] = b; m[2] = c; m[3] = d; op.nq = 1; };
  auto rz = [&](double t, cd* o) { o[0] = std::exp(-0.5 * t * I); o[1] = 0; o[2] = 0; o[3] = std::exp(0.5 * t * I); };
  auto ry = [&](double t, cd* o) {
    double c = std::cos(0.5 * t), s = std::sin(0.5 * t);
    o[0] = c; o[1] = -s; o[2] = s; o[3] = c;
  };
  auto mul2 = [](const cd* a, const cd* b, cd* o) {
    cd r[4] = {a[0] * b[0] + a[1] * b[2], a[0] * b[1] + a[1] * b[3], a[2] * b[0] + a[3] * b[2], a[2] * b[1] + a[3] * b[3]};
    for (int i = 0; i < 4; ++i) o[i] = r[i];
  };
  switch (g.kind) {
    case JF_GATE_H: set2(kR2, kR2, kR2, -kR2); break;
    case JF_GATE_S: set2(1.0, 0.0, 0.0, I); break;
    case JF_GATE_SDG: set2(1.0, 0.0, 0.0, -I); break;
    case JF_GATE_T: set2(1.0, 0.0, 0.0, cd(kR2, kR2)); break;
    case JF_GATE_TDG: set2(1.0, 0.0, 0.0, cd(kR2, -kR2)); break;
    case JF_GATE_X: set2(0.0, 1.0, 1.0, 0.0); break;
    case JF_GATE_Y: set2(0.0, -I, I, 0.0); break;
    case JF_GATE_Z: set2(1.0, 0.0, 0.0, -1.0); break;
    case JF_GATE_SX: set2(cd(0.5, 0.5), cd(0.5, -0.5), cd(0.5, -0.5), cd(0.5, 0.5)); break;
    case JF_GATE_RZ: op.nq = 1; rz(g.theta[0], m); break;
    case JF_GATE_RY: op.nq = 1; ry(g.theta[0], m); break;
    case JF_GATE_RX: {
      double c = std::cos(0.5 * g.theta[0]), s = std::sin(0.5 * g.theta[0]);
      set2(c, -I * s, -I * s, c);
      break;
    }
    case JF_GATE_SU2: {
      cd a[4], b[4], c[4], t[4];
      rz(g.theta[0], a); ry(g.theta[1], b); rz(g.theta[2], c);
      mul2(a, b, t); mul2(t, c, m); op.nq = 1;
      break;
    }
    case JF_GATE_CX: op.nq = 2; m[0] = 1; m[5] = 1; m[11] = 1; m[14] = 1; break;
    case JF_GATE_CZ: op.nq = 2; m[0] = 1; m[5] = 1; m[10] = 1; m[15] = -1.0; break;
    case JF_GATE_CS: op.nq = 2; m[0] = 1; m[5] = 1; m[10] = 1; m[15] = I; break;
    case JF_GATE_SWAP: op.nq = 2; m[0] = 1; m[6] = 1; m[9] = 1; m[15] = 1; break;
    case JF_GATE_MAT1:
      if (!g.mat) return false;
      op.nq = 1;
      for (int i = 0; i < 4; ++i) m[i] = cd(g.mat[2 * i], g.mat[2 * i + 1]);
      break;
    case JF_GATE_MAT2:
      if (!g.mat) return false;
      op.nq = 2;
      for (int i = 0; i < 16; ++i) m[i] = cd(g.mat[2 * i], g.mat[2 * i + 1]);
      break;
    default: return false;
  }
  op.q[0] = g.q0;
  op.q[1] = op.nq == 2 ? g.q1 : 0;
  return true;
}

// max_ij |(A^dagger A - I)_ij| for a dim x dim row-major matrix
static double unitarity_defect(const cd* a, int dim) {
  double worst = 0;
  for (int i = 0; i < dim; ++i)
    for (int j = 0; j < dim; ++j) {
      cd s = 0;
      for (int k = 0; k < dim; ++k) s += std::conj(a[k * dim + i]) * a[k * dim + j];
      if (i == j) s -= 1.0;
      worst = std::max(worst, std::abs(s));
    }
  return worst;
}

static bool kraus_set(const jf_noise& s, NoiseSite& out) {
  const cd I(0.0, 1.0);
  auto push = [&](cd a, cd b, cd c, cd d) {
    out.kraus.push_back(a); out.kraus.push_back(b); out.kraus.push_back(c); out.kraus.push_back(d);
    out.nk++;
  };
  double p = s.p;
  switch (s.channel) {
    case JF_NOISE_KRAUS:
      if (!s.kraus || s.n_kraus < 1 || s.n_kraus > 16) return false;
      for (int k = 0; k < s.n_kraus; ++k) {
        const double* m = s.kraus + 8 * k;
        push(cd(m[0], m[1]), cd(m[2], m[3]), cd(m[4], m[5]), cd(m[6], m[7]));
      }
      return true;
    case JF_NOISE_DEPOLARIZING: {
      if (!(p >= 0 && p <= 1)) return false;
      double a = std::sqrt(1 - p), b = std::sqrt(p / 3);
      push(a, 0, 0, a); push(0, b, b, 0); push(0, -I * b, I * b, 0); push(b, 0, 0, -b);
      return true;
    }
    case JF_NOISE_BIT_FLIP:
    case JF_NOISE_PHASE_FLIP:
    case JF_NOISE_BIT_PHASE_FLIP: {
      if (!(p >= 0 && p <= 1)) return false;
      double a = std::sqrt(1 - p), b = std::sqrt(p);
      push(a, 0, 0, a);
      if (s.channel == JF_NOISE_BIT_FLIP) push(0, b, b, 0);
      else if (s.channel == JF_NOISE_PHASE_FLIP) push(b, 0, 0, -b);
      else push(0, -I * b, I * b, 0);
      return true;
    }
    case JF_NOISE_AMPLITUDE_DAMPING: {
      if (!(p >= 0 && p <= 1)) return false;
      push(1.0, 0, 0, std::sqrt(1 - p));
      push(0, std::sqrt(p), 0, 0);
      return true;
    }
    default: return false;
  }
}

static double tp_defect(const NoiseSite& s) {
  cd acc[4] = {0, 0, 0, 0};
  for (int k = 0; k < s.nk; ++k) {
    const cd* K = &s.kraus[4 * k];
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j)
        for (int r = 0; r < 2; ++r) acc[2 * i + j] += std::conj(K[2 * r + i]) * K[2 * r + j];
  }
  acc[0] -= 1.0; acc[3] -= 1.0;
  double w = 0;
  for (auto& a : acc) w = std::max(w, std::abs(a));
  return w;
}

static jf_status load_gates(int n, const jf_gate* gs, int cnt, double tol, std::vector<GateOp>& out, const char* which) {
  out.clear();
  out.reserve(cnt);
  for (int i = 0; i < cnt; ++i) {
    GateOp op;
    if (!gate_matrix(gs[i], op)) {
      set_error(std::string(which) + " gate " + std::to_string(i) + ": unknown kind or missing matrix");
      return JF_E_ARG;
    }
    for (int j = 0; j < op.nq; ++j)
      if (op.q[j] < 0 || op.q[j] >= n) {
        set_error(std::string(which) + " gate " + std::to_string(i) + ": qubit out of range");
        return JF_E_QUBIT;
      }
    if (op.nq == 2 && op.q[0] == op.q[1]) {
      set_error(std::string(which) + " gate " + std::to_string(i) + ": two-qubit gate on one qubit");
      return JF_E_QUBIT;
    }
    double d = unitarity_defect(op.m, 1 << op.nq);
    if (!(d <= tol)) {
      set_error(std::string(which) + " gate " + std::to_string(i) + ": not unitary (defect " + std::to_string(d) + ")");
      return JF_E_NOT_UNITARY;
    }
    out.push_back(op);
  }
  return JF_OK;
}

}  // namespace jf

using namespace jf;

extern "C" jf_status jf_load_circuit(int n_qubits, const jf_gate* ideal, int n_ideal, const jf_gate* noisy_gates,
                                     int n_noisy, const jf_noise* noise, int n_noise, double tol, jf_circuit** out) {
  if (!out || n_qubits < 1 || n_qubits > 62 || n_ideal < 0 || n_noise < 0 || (n_ideal > 0 && !ideal) ||
      (n_noise > 0 && !noise) || (noisy_gates && n_noisy < 0)) {
    set_error("jf_load_circuit: bad argument");
    return JF_E_ARG;
  }
  if (!(tol > 0)) tol = 1e-10;
  auto c = std::make_unique<jf_circuit>();
  c->n = n_qubits;
  jf_status st = load_gates(n_qubits, ideal, n_ideal, tol, c->ideal, "ideal");
  if (st != JF_OK) return st;
  if (noisy_gates) {
    st = load_gates(n_qubits, noisy_gates, n_noisy, tol, c->noisy, "noisy");
    if (st != JF_OK) return st;
  } else {
    c->noisy = c->ideal;
  }
  for (int i = 0; i < n_noise; ++i) {
    NoiseSite s;
    s.after = noise[i].after_op;
    s.qubit = noise[i].qubit;
    if (s.after < -1 || s.after >= (int)c->noisy.size()) {
      set_error("noise site " + std::to_string(i) + ": after_op out of range");
      return JF_E_ARG;
    }
    if (s.qubit < 0 || s.qubit >= n_qubits) {
      set_error("noise site " + std::to_string(i) + ": qubit out of range");
      return JF_E_QUBIT;
    }
    if (!kraus_set(noise[i], s)) {
      set_error("noise site " + std::to_string(i) + ": bad channel, strength or Kraus array");
      return JF_E_ARG;
    }
    double d = tp_defect(s);
    if (!(d <= tol)) {
      set_error("noise site " + std::to_string(i) + ": Kraus set not trace preserving (defect " + std::to_string(d) + ")");
      return JF_E_NOT_TP;
    }
    c->sites.push_back(std::move(s));
  }
  // time order of the sites: by the gate they follow, ties in array order
  std::stable_sort(c->sites.begin(), c->sites.end(), [](const NoiseSite& a, const NoiseSite& b) { return a.after < b.after; });
  *out = c.release();
  return JF_OK;
}

extern "C" void jf_free_circuit(jf_circuit* c) { delete c; }
