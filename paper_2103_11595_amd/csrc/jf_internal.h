// Internal host-side structures of the Jamiolkowski-fidelity library.
//
// Pipeline: circuit (ingest, validation) -> tensor network (Algorithm I miter or Algorithm II
// doubled network) -> exact cancellation of adjacent U^dagger U pairs -> connected components ->
// greedy frontier contraction path per component -> slicing of Kraus indices -> block fusion
// and lowering to device "absorb" steps -> execution (GPU) or emulation (host, validation only).
#pragma once

#include <atomic>
#include <complex>
#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "../../include/jf.h"

namespace jf {

using cd = std::complex<double>;

// ---------------------------------------------------------------- circuit ---
struct GateOp {
  int nq = 1;           // 1 or 2
  int q[2] = {0, 0};
  cd m[16];             // row-major 2^nq x 2^nq, q[0] the more significant bit
};

struct NoiseSite {
  int after = -1;       // acts right after noisy gate `after` (-1: before gate 0)
  int qubit = 0;
  int nk = 0;           // number of Kraus operators
  std::vector<cd> kraus;  // nk x 4 (row-major 2x2)
};

}  // namespace jf

struct jf_circuit {
  int n = 0;
  std::vector<jf::GateOp> ideal, noisy;
  std::vector<jf::NoiseSite> sites;
};

namespace jf {

void set_error(const std::string& msg);

// ---------------------------------------------------------------- network ---
enum TensorKind { T_GATE = 0, T_SLOT = 1, T_NOISE = 2, T_OTHER = 3 };

struct Tensor {
  std::vector<int> legs;  // element index bit i <-> legs[i]
  std::vector<cd> data;   // 2^legs.size() entries
  int kind = T_OTHER;
  // gates: operator is op(M) with M = src->m, op = dagger if dag, conjugate if conj
  const GateOp* src = nullptr;
  int dag = 0, conj = 0;
  std::vector<int> ins, outs;  // gate/noise ports per qubit (leg ids), for adjacency checks
  // Algorithm I slots: site index, Kraus count and variant (open) legs
  int site = -1, nk = 0;
  std::vector<int> var_legs;   // LSB first; also present in legs
};

struct Network {
  int n_qubits = 0;
  int alg = 1;
  std::vector<Tensor> T;
  // open legs: for every site (time order) its variant legs, LSB first (Alg I only)
  std::vector<std::vector<int>> site_var_legs;
  std::vector<int> site_nk;
  double log2_scale = 0.0;   // exact power-of-two factor: empty loops and 1/d normalisation
  cd scalar = cd(1.0, 0.0);  // product of fully traced scalar tensors
  int n_before_cancel = 0, n_after_cancel = 0, empty_loops = 0;
  std::vector<char> leg_alive;  // legs still present (renamed or contracted legs are dead)
};

Network build_network(const jf_circuit& c, int alg);
void cancel_inverse_pairs(Network& net);
int rewire_swaps(Network& net);  // returns the number of SWAP tensors removed
void trace_self_loops(Network& net);
std::vector<std::vector<int>> components(const Network& net);
int count_empty_loops(const Network& net);

// small host tensor algebra (FP64)
Tensor contract_pair(const Tensor& a, const Tensor& b);

// ---------------------------------------------------------------- program ---
enum Prec { P_C128 = 0, P_C64 = 1 };            // storage
// C_SPLIT: every real product from three-way BF16 splits of both operands (six piece products on
// the BF16 matrix cores, FP32 accumulation)
enum Compute { C_F64 = 0, C_F32 = 1, C_SPLIT = 2 };

constexpr int MAXK = 64;     // max K (=2^kS) and Nn (=2^kN) of one device step
constexpr int MAXR = 256;    // max rows per tile
constexpr int MAXHI = 48;    // max high (tile-index) bits
// components whose intermediates all fit 2^11 elements run whole in one workgroup of the persistent
// kernel (two FP64 ping-pong buffers of 32 KB in LDS).  2^12 would fit the 160 KB of a gfx950
// compute unit, but one workgroup per component is slower there than the step kernels: the
// 36-qubit chain took 0.297 ms against 0.160 ms in complex64 (measured on MI355X).
constexpr int LDS_RESIDENT_MAX = 11;

// One device step: C[f, n] = sum_s A[f, s] * B[s, n]  (complex), see kernels.hip.
struct Step {
  int kS = 0, kN = 0, L = 0;
  int rA = 0, rC = 0;            // log2 sizes of input / output tensors
  long long nTiles = 1;
  std::vector<long long> offS_A, offR_A, offN_C, offR_C;
  std::vector<int> hiA, hiC;     // bit positions in A / C of the tile-index bits (LSB first)
  bool inplace_ok = false;       // C layout == A layout (can run in place)
  int in_prec = P_C128, out_prec = P_C128, compute = C_F64;
  // Variants of the operator: one per combination of the values of the levels in var_levels
  // (ascending; mixed radix, the first level lowest) -- the levels whose sliced index (a Kraus
  // site's operator, a wire's value) this block carries.  nvar = B.size().
  int nvar = 1;
  std::vector<int> var_levels;
  std::vector<std::vector<cd>> B; // per variant: K x Nn row-major ([s][n])
  bool final_step = false;       // writes the component output (strided into the out array)
  bool two_term = false;         // FP32 steps: operator stored as an FP32 pair (hi + lo)
  double flops = 0, bytes = 0;
  // device-side B offsets (filled at upload), per variant, in the pool of the compute type
  std::vector<long long> b_off;
  int chain = -1;                // index into ComponentProgram::chains, -1: runs on its own
};

// A chain: consecutive in-place FP32 steps of one level [first, last) whose contracted bits
// together span few positions.  It runs as one launch: a workgroup loads a tile of 2^T elements
// (positions P: the union of the steps' contracted positions plus the lowest other positions as
// rows) into LDS, applies every step of the chain there and writes the tile back, so the
// intermediate crosses HBM once for the whole chain.
constexpr int CHAIN_MAX_STEPS = 8;   // steps per chain
constexpr int CHAIN_MAX_T = 12;      // log2 elements of a tile (32 KB of complex64)
constexpr int CHAIN_MAX_U = 10;      // contracted positions of a chain
constexpr int CHAIN_MAX_OPS = 4096;        // FP32 chains: K^2 per step (2 K^2 for an FP32 pair), summed
constexpr int CHAIN_MAX_OPS_SPLIT = 2304;  // split chains: 16-byte operator fragments in LDS (36 KB)
// LDS entries the operator of a chain step takes, against the budget of its kind above
inline int chain_step_ops(int kS, bool split, bool two_term = false) {
  return split ? 576 * (kS > 4 ? 1 << (kS - 4) : 1) : (two_term ? 2 : 1) << (2 * kS);
}
struct Chain {
  int first = 0, last = 0;       // steps of the component
  int T = 0;                     // tile bits
  std::vector<int> P;            // tile positions, ascending (tile-local index = compressed over P)
  std::vector<int> hi;           // the other positions, ascending (tile index bits)
  long long nTiles = 1;
  double flops = 0, bytes = 0;   // algorithmic cost of one launch (the tensor read and written once)
};
// Tile-local addressing of a chain, as the chain kernel reads it:
//   global offset of tile-local index l = gDig[0][l & 15] + gDig[1][(l >> 4) & 15] + gDig[2][l >> 8]
//   step j, contracted index s and the others f:  local index = sOff[j][s] + fDig[j][0][f & 15] +
//   fDig[j][1][(f >> 4) & 15] + fDig[j][2][f >> 8]  (the output index n uses sOff like s)
struct ChainTables {
  long long gDig[3][16] = {};
  std::vector<std::vector<unsigned short>> sOff;   // per step: 2^kS entries
  std::vector<std::vector<unsigned short>> fDig;   // per step: 3 x 16 entries
};

struct Level {
  int first = 0, last = 0;       // steps [first, last)
  int site = -1;                 // sliced Kraus site iterated at this level (-1: none)
  int wire = -1;                 // sliced wire leg iterated at this level (network leg id; -1: none)
  int nvar = 1;                  // values iterated at this level (Kraus operators, or 2 for a wire)
  long long out_stride = 0;      // output offset per variant of this level's site
  int max_log2 = 0;              // largest tensor of the segment
  size_t buf_bytes = 0;          // bytes of each of the level's two buffers
};

struct ComponentProgram {
  std::vector<Step> steps;
  std::vector<Level> levels;
  int n_open_bits = 0;           // bits of this component's output (padded variant index)
  // per network site: output bit of each Kraus-index bit (empty: not in this component).  Sliced
  // sites hold the top bits, one contiguous run each; the open sites' bits follow the final
  // step's own layout, so its writes are as contiguous as its reads.
  std::vector<std::vector<int>> out_bit;
  long long out_len = 1;         // complex entries of the component output
  // sliced wires: a leaf's final step writes leaf_len partial values, added into the output at the
  // leaf's Kraus-site offset (the sum over the wires' values is the trace)
  bool accumulate = false;
  long long leaf_len = 0;
  long long leaves = 1;          // DFS leaves
  double flops = 0, bytes = 0;
  double est_seconds = 0;          // cost-model estimate of the device time of one run
  int max_log2 = 0;
  int n_tensors = 0;
  // device: offset of the component output (double2 elements) in the output region
  long long out_off = 0;
  // one level and every intermediate <= 2^LDS_RESIDENT_MAX elements: runs whole in one workgroup (LDS)
  bool lds_resident = false;
  std::vector<Chain> chains;
};

void chain_tables(const ComponentProgram& cp, const Chain& ch, ChainTables& out);
// index into st.B of the variant selected by the values vv[lv] of the enclosing levels
inline size_t variant_index(const ComponentProgram& cp, const Step& st, const std::vector<int>& vv) {
  size_t idx = 0, stride = 1;
  for (int lv : st.var_levels) {
    idx += stride * size_t(vv[lv]);
    stride *= size_t(cp.levels[lv].nvar);
  }
  return idx;
}
// positions of a step's contracted bits in A (offS_A is their scatter), in its s-bit order
std::vector<int> step_s_positions(const Step& st);
// in-place complex64 step with a single-term FP32 operator of at most 32 x 32
bool chainable(const Step& st);

struct PlanOptions {
  int alg = 1;
  int dtype = JF_C128;
  int cap_log2 = 30;
  unsigned flags = 0;
  int kmax = 5;                  // fused block limit on |S| and |N|
  int switch_log2 = 12;          // steps whose tensors stay <= 2^switch run in FP64 (closing part)
  double time_budget_s = 60.0;   // safety cap on the restart search (plans are reproducible below it)
  int restarts = 0;              // randomised greedy restarts per component (0: sized to the network)
  int threads = 8;               // planner worker threads
  unsigned seed = 12345;
};

struct Program {
  PlanOptions opt;
  int n_qubits = 0;
  double log2_scale = 0;
  cd scalar = 1.0;
  std::vector<ComponentProgram> comps;
  std::vector<int> site_nk;        // actual Kraus counts per site (time order)
  std::vector<int> site_comp;      // component holding each site (-1: none)
  std::vector<std::vector<double>> site_norm2;  // squared operator norm of every Kraus operator
  long long kraus_terms = 1;
  int n_before_cancel = 0, n_after_cancel = 0, empty_loops = 0, n_swaps_rewired = 0;
  int n_sliced_wires = 0;
  double planner_seconds = 0;
  double flops = 0, bytes = 0;
  double est_seconds = 0;          // cost-model estimate of the device time of one run
  int max_log2 = 0;
  long long work_items = 0;
  size_t ws_bytes = 0;             // workspace bytes
  // host copies of B pools per compute type (uploaded once into the workspace)
  std::vector<cd> pool64;          // FP64 / FP32 entries (converted at upload for FP32)
  size_t pool_bytes = 0;
};

Program plan_program(const jf_circuit& c, const PlanOptions& opt);

// bounds check of every step's addresses, table sizes and LDS budget (host; before any launch)
bool validate_program(const Program& P, std::string& why);

// host emulation of the lowered program (validation only; no fidelity entry point calls it)
void emulate_program(const Program& p, std::vector<std::vector<cd>>& comp_out);

// the fields of a result that the plan fixes (terms covered, leaves, sizes, flops, bytes); F_J,
// 1 - F_J and the residual come from the device
void static_result(const Program& p, jf_result* out);
void gather_terms(const Program& p, const std::vector<std::vector<cd>>& comp_out, double* term_traces);

}  // namespace jf

struct jf_plan {
  jf::Program prog;
  // device state (lazily created by the executor)
  void* dev = nullptr;
  // process-unique identity: a plan allocated where a freed one lived must not match caches
  // keyed by the freed plan (the batch graph)
  const unsigned long long uid = next_uid();
  static unsigned long long next_uid() {
    static std::atomic<unsigned long long> n{0};
    return ++n;
  }
};
