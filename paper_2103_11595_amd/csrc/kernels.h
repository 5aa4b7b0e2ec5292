// Device-side step descriptor and kernel launchers (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace jf {

constexpr int DMAXK = 64;   // entries of the s / n offset tables
constexpr int DMAXR = 256;  // rows per tile
constexpr int DMAXHI = 48;  // tile-index bits

// One contraction step C[f, n] = sum_s A[f, s] B[s, n] on bit-addressed tensors:
//   A element of (tile t, s, row r) at  baseA(t) + offS_A[s] + offR_A[r]
//   C element of (tile t, n, row r) at  baseC(t) + offN_C[n] + offR_C[r]
//   baseA(t) = sum_b bit_b(t) << hiA[b],  baseC(t) = sum_b bit_b(t) << hiC[b]
// K = 2^kS, Nn = 2^kN, R = 2^L rows per tile, nTiles = 2^nHi tiles.
struct StepDesc {
  long long offS_A[DMAXK];
  long long offR_A[DMAXR];
  long long offN_C[DMAXK];
  long long offR_C[DMAXR];
  int hiA[DMAXHI];
  int hiC[DMAXHI];
  int nHi, kS, kN, L;
  long long nTiles;
  int mode;       // arithmetic of the step (see KernelMode)
  int variant;    // kernel used for it (see KernelVariant); read on the host only
  // split-form steps: offsets (16-byte units, from the start of the operator block) of its BF16
  // fragments in the two matrix-core layouts (Gauss form, real embedding); -1 where absent
  int frag_gauss, frag_embed;
  // tile bases by 4-bit digits of the tile index: digit c with value m sets the address bits
  // digA[16 c + m] (digC for C); the host fills them, the MFMA kernels copy them into LDS
  long long digA[DMAXHI / 4 * 16], digC[DMAXHI / 4 * 16];
};

// Kernels that can run a step.  KV_AUTO applies the fixed rule of launch_step; the others are
// used where the step's shape allows them (launch_step falls back to KV_AUTO elsewhere).
enum KernelVariant {
  KV_AUTO = 0,
  KV_STAGED_256 = 1,  // MFMA, A tile staged through LDS, 256 threads
  KV_STAGED_512 = 2,  // the same, 512 threads
  KV_DIRECT_256 = 3,  // MFMA, A operands loaded straight into registers, 256 threads
  KV_DIRECT_512 = 4,  // the same, 512 threads
  KV_FMA = 5,         // plain FMA on LDS tiles
  KV_GAUSS_256 = 6,   // register-direct, three real products per complex one (two-term: residual first)
  KV_GAUSS_512 = 7,   // the same, 512 threads
  KV_COUNT = 8,
  KV_CHAIN = 8,       // (profiles only) a chain of steps in one launch, k_chain
};

// Whether a variant can run the step described by h (mode, kS, kN, L).
bool variant_applies(const StepDesc& h, int variant);
// The variant launch_step actually uses for h (KV_AUTO and inapplicable choices resolved).
int resolve_variant(const StepDesc& h);

enum KernelMode {
  KM_F64 = 0,       // double2 -> double2, FP64
  KM_F32 = 1,       // float2 -> float2, FP32
  KM_F32_TO_F64 = 2,// float2 -> double2, FP64 (closing part of the low-precision modes)
  KM_SPLIT = 3,     // float2 -> float2, split form: every real product from three-way BF16 splits
                    // (six piece products, FP32 accumulation); operator in 3 pieces
  KM_F32X2 = 4,     // float2 -> float2, FP32, operator as an FP32 pair (hi + lo) -- noise-carrying blocks
  KM_SPLIT4 = 5,    // the split form with a fourth operator piece (the FP64 residual) -- noise-carrying blocks
};
// Operator block of a split-form step: P pieces (3, or 4 for KM_SPLIT4) of K x Nn entries,
// row-major [s][n], each entry float4 (Re, Im, Re + Im, 0) whose values are exact BF16 numbers;
// after them the same pieces as BF16 matrix-core fragments in LDS order (StepDesc::frag_gauss,
// frag_embed; see split_gauss_frags / split_embed_frags).
//   Gauss form (P = 3): MB = max(1, Nn / 16), KC = max(1, K / 32); entry e of 3 MB KC 64 3:
//     piece q = e % 3, lane = (e / 3) % 64, kc, mb, x (Re, Im, Re + Im) the next mixed-radix digits;
//     dword d holds the BF16 pair of component x at s = 32 kc + 8 (lane / 16) + 2 d (+ 1), n = 16 mb +
//     lane % 16 (zero outside K x Nn)
//   real embedding: MB = max(1, Nn / 8), KC = max(1, K / 16); entry e of MB KC 64 P: piece q = e % P,
//     lane, kc, mb as above; dword d holds k = 2 s (low half) and 2 s + 1 (high) of B_real column
//     2 n + b for s = 16 kc + 4 (lane / 16) + d, n = 8 mb + (lane % 16) / 2, b = lane % 2
//     (B_real[2s + a][2n + b] = [[Re, Im], [-Im, Re]][a][b] of B[s][n])
__host__ __device__ inline int split_gauss_mb(int kN) { return kN <= 4 ? 1 : 1 << (kN - 4); }
__host__ __device__ inline int split_gauss_kc(int kS) { return kS <= 5 ? 1 : 1 << (kS - 5); }
__host__ __device__ inline int split_embed_mb(int kN) { return kN <= 3 ? 1 : 1 << (kN - 3); }
__host__ __device__ inline int split_embed_kc(int kS) { return kS <= 4 ? 1 : 1 << (kS - 4); }

// Launch one step.  A / C may alias (in-place steps): every tile reads exactly the elements it
// writes and stages them in LDS before writing.  B: K x Nn row-major, in the compute type
// (double2 for FP64 modes, float2 for FP32 modes, the pieces above for the split modes).
hipError_t launch_step(const StepDesc* d_desc, const StepDesc& h_desc, const void* A, void* C, const void* B,
                       hipStream_t stream);

// Chains: up to CHAIN_STEPS consecutive in-place FP32 or split-form steps of one level (each
// K = Nn <= 32, every step keeping the intermediate's layout) applied to one LDS tile of
// 2^T <= 2^CHAIN_T elements per HBM pass.  Tile-local index l (compressed over the tile's positions) sits in the tensor at
//   tile base + gDig[l & 15] + gDig[16 + ((l >> 4) & 15)] + gDig[32 + (l >> 8)],
// the tile base being the scatter of the tile index over hi[0 .. nHi).  Step j contracts its K
// indices s at tile-local sOff[s] against the remaining tile bits f at
//   fDig[f & 15] + fDig[16 + ((f >> 4) & 15)] + fDig[32 + (f >> 8)],
// and writes n at the same places (sOff[n]).  Its operator (K x K, row-major [s][n]: float2, or
// the split-form pieces) is ops.B[j]; in LDS it sits at entry boff (float2 entries for FP32 steps:
// K^2, or 2 K^2 for an FP32 pair, the residual block after the leading one; 16-byte BF16
// fragments for split steps: 576 max(1, K / 16) of them per step).
constexpr int CHAIN_STEPS = 8;
constexpr int CHAIN_T = 12;
constexpr int CHAIN_OPS = 4096;        // float2 entries of all operators of an FP32 chain
constexpr int CHAIN_OPS_SPLIT = 2304;  // 16-byte fragments of all operators of a split chain (36 KB)
struct ChainStepDesc {
  int kS, boff;
  int frag;  // split chains: offset (16-byte units) of the Gauss-form fragments in the operator block
  int two;   // FP32 chains: 1 when the operator is an FP32 pair (K x K leading part, then the residual)
  unsigned short sOff[32];
  unsigned short fDig[48];
};
struct ChainDesc {
  long long gDig[48];
  int hi[DMAXHI];
  long long nTiles;
  int nsteps, T, nHi, ops;
  int split;  // 1: split-form steps
  int pad;
  ChainStepDesc st[CHAIN_STEPS];
};
struct ChainOps {
  const void* B[CHAIN_STEPS];
};
// A and C may alias (in place): a tile is read whole before any of it is written.
hipError_t launch_chain(const ChainDesc* d_desc, const ChainDesc& h_desc, const void* A, void* C, const ChainOps& ops,
                        hipStream_t stream);

// Persistent executor of small component programs (every intermediate <= 2^11 elements, one
// level): one workgroup per item, both ping-pong buffers in LDS, FP64 throughout.  A step entry
// points at its descriptor and operator block (compute type given by mode; FP32 two-term blocks
// are summed hi + lo); the final step writes the item's output and its double-double sum of
// |t|^2 (sums[0..1]) and t_0 (sums[2..3]).
constexpr int LDS_RESIDENT_LOG2 = 11;  // two FP64 buffers of 32 KB
struct LdsStep {
  const StepDesc* desc;
  const void* B;
  int mode;
  int final_step;
};
struct LdsItem {
  int first, count;   // steps [first, first + count) of the step table
  double2* out;       // component output (double2 x out_len)
  double* sums;       // 4 doubles
  long long out_len;
};
// The assembly of F_J from a plan's component sums (see launch_assemble), passed by value.
struct AssembleArgs {
  const double* sums;
  int ncomp, alg;
  double a, v0re, v0im;
  double* res;
  double* host;        // pinned host landing area or null
  unsigned* counter;   // zero before the launch, zero again after it (the last workgroup resets it)
};
hipError_t launch_persistent(const LdsItem* items, int n_items, const LdsStep* steps, hipStream_t stream);
// Workgroup sizes launch_step and launch_chain use for a step / a chain.
int step_threads(const StepDesc& h);
int chain_threads(const ChainDesc& h);
// The same launch, ending with the assembly: the last workgroup to finish (counted on *counter)
// assembles F_J from every item's sums -- for plans whose components are all LDS-resident, one
// launch per run.
hipError_t launch_persistent_assemble(const LdsItem* items, int n_items, const LdsStep* steps,
                                      const AssembleArgs& as, hipStream_t stream);

// Attach a start / stop event pair to the step-kernel launches of this thread (nullptr, nullptr
// to stop): the events then bracket the kernel execution itself.
void set_launch_events(hipEvent_t start, hipEvent_t stop);

// out[i] = 0 for i < n (double2 entries)
hipError_t launch_zero(void* out, long long n_double2, hipStream_t stream);
// Streaming copy of bytes (a multiple of bpl = 8 or 16 bytes per lane, nontemporal, resident grid)
// between the two events: the HBM ceiling of the step kernels' access pattern.
hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, int bpl, hipStream_t stream, hipEvent_t ev0,
                              hipEvent_t ev1);
// res[0..3] = F_J, 1 - F_J, |Im| (Algorithm II), 0 from the components' sums (4 doubles each:
// double-double sum of |t|^2, first entry): the product over components on the device; host, if not
// null, is pinned host memory that receives the same four values
hipError_t launch_assemble(const double* sums, int ncomp, int alg, double a, double v0re, double v0im, double* res,
                           double* host, hipStream_t stream);
// out[i] += part[i] for i < n (double2 entries): a leaf's partial result of sliced wires
hipError_t launch_accumulate(void* out, const void* part, long long n_double2, hipStream_t stream);

// sums[0..1] = double-double sum_i |x_i|^2 (TwoSum, fixed partition and reduction trees);
// sums[2..3] = x_0 (re, im).  scratch: 2 SUMSQ_BLOCKS doubles of device memory for the partial
// sums of the first pass (used and released within the stream order of the call).
constexpr int SUMSQ_BLOCKS = 1024;
hipError_t launch_sumsq(const void* x, long long n, double* sums, double* scratch, hipStream_t stream);

}  // namespace jf
