// HIP kernels (gfx950) of the contraction executor.
//
// Every step kernel computes one contraction step of the running intermediate A with a small
// operator B,
//   C[f, n] = sum_s A[f, s] * B[s, n],
// where f, s, n are bit-fields of the tensors' element indices scattered over arbitrary bit
// positions (see StepDesc).  The work is cut into tiles of 2^L rows (the lowest free bits, so
// 16 consecutive rows are one contiguous run) times all K contracted combinations; tiles are
// disjoint, so a step whose output layout equals its input layout runs in place.  Kernels:
//   k_absorb, k_absorb_f32x2, k_absorb_split    vector FMA on a tile staged in LDS
//   k_absorb_mfma        matrix cores on the real embedding, tile staged in LDS
//   k_absorb_mfma_rd     matrix cores on the real embedding, operands straight into registers
//   k_absorb_mfma_gauss  matrix cores, three real products per complex one, register-direct
//   k_absorb_split_gauss, k_absorb_split_embed  the split form (three-way BF16 splits, six
//                        piece products) on BF16 matrix cores, register-direct
//   k_chain, k_chain_pairs, k_chain_split  several in-place FP32 (single or FP32-pair operators)
//                        / split-form steps applied to one LDS tile per HBM pass
//   k_persistent         whole small components in one workgroup's LDS (and, for a plan made
//                        of them only, the assembly of F_J by the last workgroup)
//   k_sumsq_part/_final  the FP64 double-double sum of |t|^2 (two fixed-tree passes); k_sumsq_one
//                        the same for a small output in one launch
//   k_assemble           F_J and 1 - F_J from the components' sums (device and pinned host)
//   k_accumulate, k_zero a wire-sliced leaf's partial traces into the output; a graph-safe fill
//   k_stream_copy        the streaming copy that measures the HBM ceiling
// launch_step picks the kernel of a step (its variant, or the fixed rule).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

#include "kernels.h"

namespace jf {

// Streaming accesses of the big intermediates: a step reads every element of A once and writes
// every element of C once, so the MFMA kernels load and store them with the nontemporal hint
// (no reuse to keep in the caches).  Measured on MI355X: with resident grids, 1.32 -> 1.24 ms
// per complex64 pass of the n=16 workload.
typedef float f32v2 __attribute__((ext_vector_type(2)));
typedef double f64v2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 ld_stream(const float2* p) {
  const f32v2 w = __builtin_nontemporal_load(reinterpret_cast<const f32v2*>(p));
  return make_float2(w.x, w.y);
}
__device__ __forceinline__ double2 ld_stream(const double2* p) {
  const f64v2 w = __builtin_nontemporal_load(reinterpret_cast<const f64v2*>(p));
  return make_double2(w.x, w.y);
}
__device__ __forceinline__ void st_stream(float2* p, float2 v) {
  f32v2 w;
  w.x = v.x;
  w.y = v.y;
  __builtin_nontemporal_store(w, reinterpret_cast<f32v2*>(p));
}
__device__ __forceinline__ void st_stream(double2* p, double2 v) {
  f64v2 w;
  w.x = v.x;
  w.y = v.y;
  __builtin_nontemporal_store(w, reinterpret_cast<f64v2*>(p));
}

// ------------------------------------------------------------------ complex helpers ---
__device__ __forceinline__ double2 cfma(double2 acc, double2 a, double2 b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
  return acc;
}
__device__ __forceinline__ float2 cfma(float2 acc, float2 a, float2 b) {
  acc.x = fmaf(a.x, b.x, acc.x);
  acc.x = fmaf(-a.y, b.y, acc.x);
  acc.y = fmaf(a.x, b.y, acc.y);
  acc.y = fmaf(a.y, b.x, acc.y);
  return acc;
}
template <typename T> __device__ __forceinline__ T czero();
template <> __device__ __forceinline__ double2 czero<double2>() { return make_double2(0.0, 0.0); }
template <> __device__ __forceinline__ float2 czero<float2>() { return make_float2(0.f, 0.f); }
template <typename TO, typename TI> __device__ __forceinline__ TO cconv(TI v);
template <> __device__ __forceinline__ double2 cconv<double2, double2>(double2 v) { return v; }
template <> __device__ __forceinline__ float2 cconv<float2, float2>(float2 v) { return v; }
template <> __device__ __forceinline__ double2 cconv<double2, float2>(float2 v) { return make_double2(v.x, v.y); }
template <> __device__ __forceinline__ float2 cconv<float2, double2>(double2 v) { return make_float2(float(v.x), float(v.y)); }

// ------------------------------------------------------------------- three-way BF16 split ---
// The split form computes every real product a * b of an FP32 step from BF16 pieces: each FP32
// operand is written as three BF16 values, x = x0 + x1 + x2 exactly (x0 = bf16(x), x1 = bf16(x - x0),
// x2 = x - x0 - x1, which has at most 8 significant bits left; both roundings to nearest even, so
// the pieces carry no sign bias), and the product keeps the six piece products of order 2^-16 of
// it or more,
//   a0 b0 + (a0 b1 + a1 b0) + (a0 b2 + a1 b1 + a2 b0),
// each exact in FP32 (8 x 8 bits) and accumulated in FP32, the five small ones (smallest first)
// before a0 b0; the three dropped products are below 2^-24 of the product, the accumulation rounds
// as FP32 accumulation does.  Operator pieces come from the host as FP32 values that
// are exact BF16 numbers: P = 3 pieces of the FP32 block, or P = 4 for noise-carrying blocks, whose
// fourth piece is the residual of the FP64 block (it pairs with a0 only).  Layout of an operator
// block: P pieces of K x Nn entries (row-major [s][n]), each entry float4 (Re, Im, Re + Im, 0).
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x2v __attribute__((ext_vector_type(2)));

// Pieces of two FP32 values, each piece a packed BF16 pair (the first value in the low half).
__device__ __forceinline__ void split3_pair(float x, float y, uint32_t& p0, uint32_t& p1, uint32_t& p2) {
  const f32x2v v = {x, y};
  const bf16x2v b0 = __builtin_convertvector(v, bf16x2v);
  const f32x2v r1 = v - __builtin_convertvector(b0, f32x2v);
  const bf16x2v b1 = __builtin_convertvector(r1, bf16x2v);
  const f32x2v r2 = r1 - __builtin_convertvector(b1, f32x2v);
  const bf16x2v b2 = __builtin_convertvector(r2, bf16x2v);  // exact: r2 has at most 8 significant bits
  p0 = __builtin_bit_cast(uint32_t, b0);
  p1 = __builtin_bit_cast(uint32_t, b1);
  p2 = __builtin_bit_cast(uint32_t, b2);
}
// Pieces of eight FP32 values (k = 0..7 of one matrix-core operand): three BF16 octets.
__device__ __forceinline__ void split3_oct(const float (&v)[8], bf16x8& p0, bf16x8& p1, bf16x8& p2) {
  uint4 w0, w1, w2;
  split3_pair(v[0], v[1], w0.x, w1.x, w2.x);
  split3_pair(v[2], v[3], w0.y, w1.y, w2.y);
  split3_pair(v[4], v[5], w0.z, w1.z, w2.z);
  split3_pair(v[6], v[7], w0.w, w1.w, w2.w);
  p0 = __builtin_bit_cast(bf16x8, w0);
  p1 = __builtin_bit_cast(bf16x8, w1);
  p2 = __builtin_bit_cast(bf16x8, w2);
}
// BF16 bit pattern of an FP32 value that is exactly a BF16 number (an operator piece).
__device__ __forceinline__ uint32_t bf16_of(float x) { return __float_as_uint(x) >> 16; }
__device__ __forceinline__ uint32_t bf16_pack(float lo, float hi) { return bf16_of(lo) | (bf16_of(hi) << 16); }
__device__ __forceinline__ bf16x8 as_bf16x8(uint4 w) { return __builtin_bit_cast(bf16x8, w); }

// ----------------------------------------------------------------------- absorb step ---
struct Tables {
  long long offS[DMAXK], offRA[DMAXR], offN[DMAXK], offRC[DMAXR];
  int hiA[DMAXHI], hiC[DMAXHI];
};

__device__ __forceinline__ void load_tables(const StepDesc* __restrict__ d, Tables& tb, int K, int Nn, int R, int nHi) {
  for (int i = threadIdx.x; i < K; i += blockDim.x) tb.offS[i] = d->offS_A[i];
  for (int i = threadIdx.x; i < Nn; i += blockDim.x) tb.offN[i] = d->offN_C[i];
  for (int i = threadIdx.x; i < R; i += blockDim.x) {
    tb.offRA[i] = d->offR_A[i];
    tb.offRC[i] = d->offR_C[i];
  }
  for (int i = threadIdx.x; i < nHi; i += blockDim.x) {
    tb.hiA[i] = d->hiA[i];
    tb.hiC[i] = d->hiC[i];
  }
}

// Tile base addresses of the MFMA kernels by table look-up: the tile index t is cut into 4-bit
// digits and ch[c][m] holds the address bits that digit c with value m sets (bit b of the digit
// sets bit hi[4 c + b]).  base(t) is then the OR of DMAXHI / 4 independent LDS reads (rows past
// the tile bits are zero), where a loop over the bits of t would chain nHi dependent ones.  The
// host computes the tables (StepDesc::digA, digC); a workgroup copies them into LDS.
constexpr int NDIG = DMAXHI / 4;
struct TileBases {
  long long chA[NDIG][16], chC[NDIG][16];
};
__device__ __forceinline__ void load_tile_bases(const StepDesc* __restrict__ d, TileBases& tbb, int) {
  for (int i = threadIdx.x; i < NDIG * 16; i += blockDim.x) {
    tbb.chA[i >> 4][i & 15] = d->digA[i];
    tbb.chC[i >> 4][i & 15] = d->digC[i];
  }
}
__device__ __forceinline__ long long tile_base(const long long (*ch)[16], long long t) {
  long long b = 0;
#pragma unroll
  for (int c = 0; c < NDIG; ++c) b |= ch[c][(t >> (4 * c)) & 15];
  return b;
}

// Generic FMA path (FP64, FP32 and the FP32->FP64 closing switch).
template <typename TI, typename TO, typename TC>
__global__ __launch_bounds__(256) void k_absorb(const StepDesc* __restrict__ d, const TI* A, TO* C,
                                                const TC* __restrict__ B) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ Tables tb;
  const int kS = d->kS, kN = d->kN, L = d->L, nHi = d->nHi;
  const int K = 1 << kS, Nn = 1 << kN, R = 1 << L;
  const long long nTiles = d->nTiles;
  load_tables(d, tb, K, Nn, R, nHi);
  TC* sB = reinterpret_cast<TC*>(smem);
  TC* sA = sB + K * Nn;
  for (int i = threadIdx.x; i < K * Nn; i += blockDim.x) sB[i] = B[i];
  __syncthreads();
  for (long long t = blockIdx.x; t < nTiles; t += gridDim.x) {
    long long bA = 0, bC = 0;
    for (int b = 0; b < nHi; ++b)
      if ((t >> b) & 1) {
        bA |= 1LL << tb.hiA[b];
        bC |= 1LL << tb.hiC[b];
      }
    for (int i = threadIdx.x; i < K * R; i += blockDim.x) {
      const int s = i >> L, r = i & (R - 1);
      sA[i] = cconv<TC, TI>(A[bA + tb.offS[s] + tb.offRA[r]]);
    }
    __syncthreads();
    for (int o = threadIdx.x; o < Nn * R; o += blockDim.x) {
      const int n = o >> L, r = o & (R - 1);
      TC acc = czero<TC>();
      for (int s = 0; s < K; ++s) acc = cfma(acc, sA[s * R + r], sB[s * Nn + n]);
      C[bC + tb.offN[n] + tb.offRC[r]] = cconv<TO, TC>(acc);
    }
    __syncthreads();
  }
}

// FP32 path with a two-term operator: B = Bhi + Blo (both FP32, Blo the rounding residual of
// the FP64 block), so the operator itself carries no rounding error; A and the accumulation
// stay FP32.
__global__ __launch_bounds__(256) void k_absorb_f32x2(const StepDesc* __restrict__ d, const float2* A, float2* C,
                                                      const float2* __restrict__ B) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ Tables tb;
  const int kS = d->kS, kN = d->kN, L = d->L, nHi = d->nHi;
  const int K = 1 << kS, Nn = 1 << kN, R = 1 << L;
  const long long nTiles = d->nTiles;
  load_tables(d, tb, K, Nn, R, nHi);
  float2* sB = reinterpret_cast<float2*>(smem);   // hi then lo
  float2* sA = sB + 2 * K * Nn;
  for (int i = threadIdx.x; i < 2 * K * Nn; i += blockDim.x) sB[i] = B[i];
  __syncthreads();
  for (long long t = blockIdx.x; t < nTiles; t += gridDim.x) {
    long long bA = 0, bC = 0;
    for (int b = 0; b < nHi; ++b)
      if ((t >> b) & 1) {
        bA |= 1LL << tb.hiA[b];
        bC |= 1LL << tb.hiC[b];
      }
    for (int i = threadIdx.x; i < K * R; i += blockDim.x) {
      const int s = i >> L, r = i & (R - 1);
      sA[i] = A[bA + tb.offS[s] + tb.offRA[r]];
    }
    __syncthreads();
    for (int o = threadIdx.x; o < Nn * R; o += blockDim.x) {
      const int n = o >> L, r = o & (R - 1);
      float2 acc = make_float2(0.f, 0.f);
      for (int s = 0; s < K; ++s) acc = cfma(acc, sA[s * R + r], sB[K * Nn + s * Nn + n]);  // residual first
      for (int s = 0; s < K; ++s) acc = cfma(acc, sA[s * R + r], sB[s * Nn + n]);
      C[bC + tb.offN[n] + tb.offRC[r]] = acc;
    }
    __syncthreads();
  }
}

// Split form on the vector units (any shape): per real product the six (P = 4: seven) piece
// products of the split form.
// acc += the piece products of a * b, the small ones first (smallest first), a0 b0 last
template <int P>
__device__ __forceinline__ float mul6(const float (&a)[3], const float (&b)[4], float acc) {
  if (P == 4) acc = fmaf(a[0], b[3], acc);
  acc = fmaf(a[2], b[0], acc);
  acc = fmaf(a[1], b[1], acc);
  acc = fmaf(a[0], b[2], acc);
  acc = fmaf(a[1], b[0], acc);
  acc = fmaf(a[0], b[1], acc);
  return fmaf(a[0], b[0], acc);
}

// LDS: the A tile in FP32 (K x R), split when it is used; the operator's P pieces as packed BF16
// (Re in the low half, Im in the high half), [s][n][piece].
template <int P>
__global__ __launch_bounds__(256) void k_absorb_split(const StepDesc* __restrict__ d, const float2* A, float2* C,
                                                      const float4* __restrict__ B) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ Tables tb;
  const int kS = d->kS, kN = d->kN, L = d->L, nHi = d->nHi;
  const int K = 1 << kS, Nn = 1 << kN, R = 1 << L;
  const long long nTiles = d->nTiles;
  load_tables(d, tb, K, Nn, R, nHi);
  uint32_t* sB = reinterpret_cast<uint32_t*>(smem);
  float2* sA = reinterpret_cast<float2*>(sB + P * K * Nn);
  for (int i = threadIdx.x; i < K * Nn; i += blockDim.x)
    for (int q = 0; q < P; ++q) {
      const float4 b = B[q * K * Nn + i];
      sB[i * P + q] = bf16_pack(b.x, b.y);
    }
  __syncthreads();
  for (long long t = blockIdx.x; t < nTiles; t += gridDim.x) {
    long long bA = 0, bC = 0;
    for (int b = 0; b < nHi; ++b)
      if ((t >> b) & 1) {
        bA |= 1LL << tb.hiA[b];
        bC |= 1LL << tb.hiC[b];
      }
    for (int i = threadIdx.x; i < K * R; i += blockDim.x) {
      const int s = i >> L, r = i & (R - 1);
      sA[i] = A[bA + tb.offS[s] + tb.offRA[r]];
    }
    __syncthreads();
    for (int o = threadIdx.x; o < Nn * R; o += blockDim.x) {
      const int n = o >> L, r = o & (R - 1);
      float re = 0.f, im = 0.f;
      for (int s = 0; s < K; ++s) {
        const float2 av = sA[s * R + r];
        uint32_t p0, p1, p2;
        split3_pair(av.x, av.y, p0, p1, p2);
        const float ar[3] = {__uint_as_float(p0 << 16), __uint_as_float(p1 << 16), __uint_as_float(p2 << 16)};
        const float ai[3] = {__uint_as_float(p0 & 0xFFFF0000u), __uint_as_float(p1 & 0xFFFF0000u),
                             __uint_as_float(p2 & 0xFFFF0000u)};
        const float nai[3] = {-ai[0], -ai[1], -ai[2]};
        float br[4] = {0.f, 0.f, 0.f, 0.f}, bi[4] = {0.f, 0.f, 0.f, 0.f};
        for (int q = 0; q < P; ++q) {
          const uint32_t w = sB[(s * Nn + n) * P + q];
          br[q] = __uint_as_float(w << 16);
          bi[q] = __uint_as_float(w & 0xFFFF0000u);
        }
        re = mul6<P>(ar, br, re);   // Re C += Re A Re B - Im A Im B
        re = mul6<P>(nai, bi, re);
        im = mul6<P>(ar, bi, im);   // Im C += Re A Im B + Im A Re B
        im = mul6<P>(ai, br, im);
      }
      C[bC + tb.offN[n] + tb.offRC[r]] = make_float2(re, im);
    }
    __syncthreads();
  }
}


// ------------------------------------------------------------------ MFMA path (gfx950) ---
// The tile product is computed transposed on the matrix cores: with the complex embedding
//   A_real[r][2s + a] = (Re, Im)[a] of A[s][r]          (R x 2K)
//   B_real[2s + a][2n + b] = [[Re, Im], [-Im, Re]][a][b] of B[s][n]   (2K x 2Nn)
// one real GEMM gives C_real = A_real B_real, whose columns 2n, 2n + 1 are Re, Im of C[., n].
// The MFMA computes D = B_real^T A_real^T (M = 2Nn, N = R, K = 2K) so that the 16 lanes of a
// lane group hold 16 consecutive tile rows: their stores are contiguous runs.
// v_mfma_*_16x16x4: lane l supplies A-operand (row l%16, k l/16) and B-operand (k l/16, col l%16).
// Accumulator register v of lane group g = l/16 holds D row 4g + v (FP32) or 4v + g (FP64);
// the mapping of MFMA rows to (complex column, component) below makes registers (0, 1) and
// (2, 3) of every lane the (Re, Im) pairs of two complex outputs.
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
template <> struct Mfma<float> {
  using acc_t = floatx4;
  using c2 = float2;
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row_of(int g, int v) { return 4 * g + v; }
  static __device__ __forceinline__ int n_of(int i) { return i >> 1; }
  static __device__ __forceinline__ int c_of(int i) { return i & 1; }
};
template <> struct Mfma<double> {
  using acc_t = doublex4;
  using c2 = double2;
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row_of(int g, int v) { return 4 * v + g; }
  static __device__ __forceinline__ int n_of(int i) { return (i & 3) + 4 * (i >> 3); }
  static __device__ __forceinline__ int c_of(int i) { return (i >> 2) & 1; }
};

// Requires R >= 16, K >= 2 and K * R <= 4096 (the executor checks); Nn < 8 pads the operator
// to one 16-row block and stores only the Nn real columns.  LDS: the real
// B^T operand, k-major (2K x 2Nn; a second copy holds the residual operator for two-term steps),
// and the A tile as Re / Im planes (K x R each).  The next tile is fetched into registers while
// the current one is multiplied (NT threads, K * R / NT elements each).  With TWO_TERM the
// operator is Bhi + Blo (an FP32 pair); the small Blo products are accumulated first so that the
// correction survives the FP32 roundings of the running sum.
template <typename T, bool TWO_TERM, int NT, int MB>
__global__ __launch_bounds__(NT) void k_absorb_mfma(const StepDesc* __restrict__ d,
                                                    const typename Mfma<T>::c2* A,
                                                    typename Mfma<T>::c2* C,
                                                    const typename Mfma<T>::c2* __restrict__ B) {
  using M = Mfma<T>;
  using C2 = typename M::c2;
  constexpr int MAXE = 4096 / NT;  // staged elements per thread
  constexpr int NW = NT / 64;      // waves
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ Tables tb;
  __shared__ TileBases tbb;
  const int kS = d->kS, kN = d->kN, L = d->L, nHi = d->nHi;
  const int K = 1 << kS, Nn = 1 << kN, R = 1 << L;
  // M2: MFMA rows of the operator, at least one 16-row block (rows past 2Nn are zero)
  const int K2 = 2 * K, M2 = 2 * Nn < 16 ? 16 : 2 * Nn, KR = K * R;
  const long long nTiles = d->nTiles;
  load_tables(d, tb, K, Nn, R, nHi);
  load_tile_bases(d, tbb, nHi);
  T* sBt = reinterpret_cast<T*>(smem);            // [k][i] (hi), then [k][i] (lo)
  T* sAr = sBt + (TWO_TERM ? 2 : 1) * K2 * M2;    // [s][r]
  T* sAi = sAr + KR;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, l16 = lane & 15;
  const int Nb = R >> 4;  // MB = M2 / 16 output blocks per row block (the launcher checks)
  C2 stage[MAXE];
  auto fetch = [&](long long t) {
    const long long bA = tile_base(tbb.chA, t);
#pragma unroll
    for (int e = 0; e < MAXE; ++e) {
      const int i = threadIdx.x + NT * e;
      if (i < KR) stage[e] = ld_stream(&A[bA + tb.offS[i >> L] + tb.offRA[i & (R - 1)]]);
    }
  };
  __syncthreads();  // offset tables visible
  // a workgroup with a single tile issues its loads before the operator's, so that the two
  // latencies overlap (measured: shorter small steps; longer large ones if every workgroup does it)
  long long t = blockIdx.x;
  const bool early = nTiles <= (long long)gridDim.x;
  if (early && t < nTiles) fetch(t);
  // B^T operand: row i of M-block mb maps to complex column mb * 8 + n_of(i % 16), component c_of
  for (int idx = threadIdx.x; idx < K2 * M2; idx += NT) {
    const int k = idx / M2, i = idx - k * M2;
    const int n = (i >> 4) * 8 + M::n_of(i & 15), cb = M::c_of(i & 15);
    const int s = k >> 1, ca = k & 1;
    const C2 bv = n < Nn ? B[s * Nn + n] : C2{0, 0};
    const T v = (ca ^ cb) ? bv.y : bv.x;
    sBt[idx] = (ca && !cb) ? -v : v;
    if (TWO_TERM) {
      const C2 bl = n < Nn ? B[K * Nn + s * Nn + n] : C2{0, 0};
      const T w = (ca ^ cb) ? bl.y : bl.x;
      sBt[K2 * M2 + idx] = (ca && !cb) ? -w : w;
    }
  }
  if (!early && t < nTiles) fetch(t);
  __syncthreads();  // B^T visible to every wave before the first tile
  // Work of a tile: Nb row blocks x MB output blocks.  Where there are fewer row blocks than
  // waves, the output blocks of a row block are shared out in groups of MU, so that every wave
  // (and so every SIMD) has products to issue; a group's waves read the same A values.
  const int want = (NW + Nb - 1) / Nb;  // groups per row block that would occupy every wave
  auto products = [&](auto mu_tag, long long bC) {
    constexpr int MU = decltype(mu_tag)::value, SG = MB / MU;
    for (int u = wave; u < Nb * SG; u += NW) {
      const int nb = u / SG, m0 = (u - nb * SG) * MU;
      const int j = nb * 16 + l16;  // tile row supplied / produced by this lane
      // k outermost: each A value is read from LDS once and used by all MU output blocks
      typename M::acc_t acc[MU];
#pragma unroll
      for (int mb = 0; mb < MU; ++mb) acc[mb] = typename M::acc_t{0, 0, 0, 0};
      const T* bt = sBt + l16 + 16 * m0;
      if (TWO_TERM) {
        for (int kk = 0; kk < K2; kk += 4) {
          const int k = kk + g;
          const T a = ((k & 1) ? sAi : sAr)[(k >> 1) * R + j];
#pragma unroll
          for (int mb = 0; mb < MU; ++mb) acc[mb] = M::op(bt[K2 * M2 + k * M2 + 16 * mb], a, acc[mb]);
        }
      }
      for (int kk = 0; kk < K2; kk += 4) {
        const int k = kk + g;
        const T a = ((k & 1) ? sAi : sAr)[(k >> 1) * R + j];
#pragma unroll
        for (int mb = 0; mb < MU; ++mb) acc[mb] = M::op(bt[k * M2 + 16 * mb], a, acc[mb]);
      }
#pragma unroll
      for (int mb = 0; mb < MU; ++mb) {
        for (int p = 0; p < 2; ++p) {
          const int n = (m0 + mb) * 8 + M::n_of(M::row_of(g, 2 * p));
          C2 o;
          o.x = acc[mb][2 * p];
          o.y = acc[mb][2 * p + 1];
          if (MB > 1 || n < Nn) st_stream(&C[bC + tb.offN[n] + tb.offRC[j]], o);
        }
      }
    }
  };
  for (; t < nTiles; t += gridDim.x) {
    const long long bC = tile_base(tbb.chC, t);
    __syncthreads();  // every wave is done with the previous tile's planes
#pragma unroll
    for (int e = 0; e < MAXE; ++e) {
      const int i = threadIdx.x + NT * e;
      if (i < KR) {
        sAr[i] = stage[e].x;
        sAi[i] = stage[e].y;
      }
    }
    __syncthreads();
    // the next tile belongs to this workgroup only: its loads overlap this tile's products
    if (t + gridDim.x < nTiles) fetch(t + gridDim.x);
    if (MB >= 8 && want >= 8)
      products(std::integral_constant<int, (MB >= 8 ? MB / 8 : 1)>{}, bC);
    else if (MB >= 4 && want >= 4)
      products(std::integral_constant<int, (MB >= 4 ? MB / 4 : 1)>{}, bC);
    else if (MB >= 2 && want >= 2)
      products(std::integral_constant<int, (MB >= 2 ? MB / 2 : 1)>{}, bC);
    else
      products(std::integral_constant<int, MB>{}, bC);
  }
}


// Register-direct variant: no A tile in LDS.  The sum over the 2K real k indices may be taken in
// any order, so MFMA k-step t, lane group g is given real index (s = 4 (t / 2) + g, component
// t % 2): a lane then needs Re and Im of the same A[s][row], one complex load, used on two
// consecutive k-steps.  A work unit is (tile, block of 16 tile rows); each wave takes units
// independently (no barrier after set-up) and loads its next unit while multiplying the current
// one.  KQ = ceil(K / 4) complex values per lane and unit; lanes with s >= K supply zero.  The
// operator (two copies for TWO_TERM) stays in LDS, k-major in the same order.  In-place steps
// are safe: a unit writes exactly the elements it has read, after reading all of them.
template <typename T, bool TWO_TERM, int NT, int MB, int KQ>
__global__ __launch_bounds__(NT) void k_absorb_mfma_rd(const StepDesc* __restrict__ d,
                                                       const typename Mfma<T>::c2* A,
                                                       typename Mfma<T>::c2* C,
                                                       const typename Mfma<T>::c2* __restrict__ B) {
  using M = Mfma<T>;
  using C2 = typename M::c2;
  constexpr int NW = NT / 64, KT = 2 * KQ, M2 = 16 * MB;  // MFMA k-steps, operator rows (padded)
  constexpr int BT = KT * 4 * M2;                         // operator entries per copy
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ Tables tb;
  __shared__ TileBases tbb;
  const int kS = d->kS, kN = d->kN, L = d->L, nHi = d->nHi;
  const int K = 1 << kS, Nn = 1 << kN, R = 1 << L;
  const int rbits = L - 4;
  const long long nUnits = d->nTiles << rbits;
  load_tables(d, tb, K, Nn, R, nHi);
  load_tile_bases(d, tbb, nHi);
  T* sBt = reinterpret_cast<T*>(smem);  // [4 t + g][i] (hi), then the same for lo
  for (int idx = threadIdx.x; idx < BT; idx += NT) {
    const int kr = idx / M2, i = idx - kr * M2;
    const int t = kr >> 2, g = kr & 3;
    const int s = 4 * (t >> 1) + g, ca = t & 1;
    const int n = (i >> 4) * 8 + M::n_of(i & 15), cb = M::c_of(i & 15);
    T v = 0, w = 0;
    if (s < K && n < Nn) {
      const C2 bv = B[s * Nn + n];
      v = (ca ^ cb) ? bv.y : bv.x;
      if (ca && !cb) v = -v;
      if (TWO_TERM) {
        const C2 bl = B[K * Nn + s * Nn + n];
        w = (ca ^ cb) ? bl.y : bl.x;
        if (ca && !cb) w = -w;
      }
    }
    sBt[idx] = v;
    if (TWO_TERM) sBt[BT + idx] = w;
  }
  __syncthreads();  // offset tables and operator visible to every wave
  const int lane = threadIdx.x & 63, g = lane >> 4, l16 = lane & 15;
  const long long wstride = (long long)gridDim.x * NW;
  auto row_of_unit = [&](long long v) { return ((int)(v & ((1 << rbits) - 1)) << 4) + l16; };
  C2 nxt[KQ];
  auto fetch = [&](long long v) {
    const long long bA = tile_base(tbb.chA, v >> rbits) + tb.offRA[row_of_unit(v)];
#pragma unroll
    for (int u = 0; u < KQ; ++u) {
      const int s = 4 * u + g;
      const C2 x = ld_stream(&A[bA + tb.offS[s < K ? s : K - 1]]);  // in-bounds address for every lane
      nxt[u] = s < K ? x : C2{0, 0};
    }
  };
  long long v = (long long)blockIdx.x * NW + (threadIdx.x >> 6);
  if (v < nUnits) fetch(v);
  for (; v < nUnits; v += wstride) {
    C2 cur[KQ];
#pragma unroll
    for (int u = 0; u < KQ; ++u) cur[u] = nxt[u];
    if (v + wstride < nUnits) fetch(v + wstride);
    typename M::acc_t acc[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) acc[mb] = typename M::acc_t{0, 0, 0, 0};
    if (TWO_TERM) {  // residual products first: the correction survives the FP32 running sum
#pragma unroll
      for (int t = 0; t < KT; ++t) {
        const T a = (t & 1) ? cur[t >> 1].y : cur[t >> 1].x;
        const T* bt = sBt + BT + (4 * t + g) * M2 + l16;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) acc[mb] = M::op(bt[16 * mb], a, acc[mb]);
      }
    }
#pragma unroll
    for (int t = 0; t < KT; ++t) {
      const T a = (t & 1) ? cur[t >> 1].y : cur[t >> 1].x;
      const T* bt = sBt + (4 * t + g) * M2 + l16;
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) acc[mb] = M::op(bt[16 * mb], a, acc[mb]);
    }
    const long long bC = tile_base(tbb.chC, v >> rbits) + tb.offRC[row_of_unit(v)];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        const int n = mb * 8 + M::n_of(M::row_of(g, 2 * p));
        C2 o;
        o.x = acc[mb][2 * p];
        o.y = acc[mb][2 * p + 1];
        if (MB > 1 || n < Nn) st_stream(&C[bC + tb.offN[n]], o);
      }
    }
  }
}


// Gauss (3M) form of the register-direct kernel: three real products per complex one,
//   T1 = sum Re B Re A,  T2 = sum Im B Im A,  T3 = sum (Re B + Im B)(Re A + Im A),
//   Re C = T1 - T2,  Im C = T3 - T1 - T2,
// a quarter fewer matrix-core products than the real embedding, at the price of a rounding
// error relative to the larger of |T1|, |T2|, |T3| for Im C.  MFMA k runs over s directly: lane
// group g of k-step t supplies s = 4 t + g, and the 16 MFMA rows of block mb are n = 16 mb + 0..15.
// The operator sits in LDS as [t][lane][x][mb] (x = Re, Im, Re + Im), so that every lane reads
// its 3 MB values of a k-step from consecutive addresses.  Units, prefetch and in-place safety as
// in k_absorb_mfma_rd.
template <typename T, int NT, int MB, int KQ, bool TWO_TERM = false>
__global__ __launch_bounds__(NT) void k_absorb_mfma_gauss(const StepDesc* __restrict__ d,
                                                          const typename Mfma<T>::c2* A,
                                                          typename Mfma<T>::c2* C,
                                                          const typename Mfma<T>::c2* __restrict__ B) {
  using M = Mfma<T>;
  using C2 = typename M::c2;
  constexpr int NW = NT / 64, W = 3 * MB;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ Tables tb;
  __shared__ TileBases tbb;
  const int kS = d->kS, kN = d->kN, L = d->L, nHi = d->nHi;
  const int K = 1 << kS, Nn = 1 << kN, R = 1 << L;
  const int rbits = L - 4;
  const long long nUnits = d->nTiles << rbits;
  load_tables(d, tb, K, Nn, R, nHi);
  load_tile_bases(d, tbb, nHi);
  T* sB = reinterpret_cast<T*>(smem);  // [t][lane][x][mb] (hi), then the same for lo (TWO_TERM)
  constexpr int BT = KQ * 64 * W;
  for (int idx = threadIdx.x; idx < (TWO_TERM ? 2 : 1) * BT; idx += NT) {
    const int part = idx >= BT, i2 = idx - part * BT;
    const int t = i2 / (64 * W), rem = i2 - t * 64 * W;
    const int ln = rem / W, e = rem - ln * W;
    const int x = e / MB, mb = e - x * MB;
    const int s = 4 * t + (ln >> 4), n = mb * 16 + (ln & 15);
    T v = 0;
    if (s < K && n < Nn) {
      const C2 bv = B[part * K * Nn + s * Nn + n];
      v = x == 0 ? bv.x : x == 1 ? bv.y : bv.x + bv.y;
    }
    sB[idx] = v;
  }
  __syncthreads();  // offset tables and operator visible to every wave
  const int lane = threadIdx.x & 63, g = lane >> 4, l16 = lane & 15;
  const long long wstride = (long long)gridDim.x * NW;
  auto row_of_unit = [&](long long v) { return ((int)(v & ((1 << rbits) - 1)) << 4) + l16; };
  C2 nxt[KQ];
  auto fetch = [&](long long v) {
    const long long bA = tile_base(tbb.chA, v >> rbits) + tb.offRA[row_of_unit(v)];
#pragma unroll
    for (int u = 0; u < KQ; ++u) {
      const int s = 4 * u + g;
      const C2 x = ld_stream(&A[bA + tb.offS[s < K ? s : K - 1]]);  // in-bounds address for every lane
      nxt[u] = s < K ? x : C2{0, 0};
    }
  };
  long long v = (long long)blockIdx.x * NW + (threadIdx.x >> 6);
  if (v < nUnits) fetch(v);
  for (; v < nUnits; v += wstride) {
    C2 cur[KQ];
#pragma unroll
    for (int u = 0; u < KQ; ++u) cur[u] = nxt[u];
    if (v + wstride < nUnits) fetch(v + wstride);
    typename M::acc_t acc[3][MB];
#pragma unroll
    for (int x = 0; x < 3; ++x)
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) acc[x][mb] = typename M::acc_t{0, 0, 0, 0};
    // two-term operators: the residual's products first, so that the correction survives the
    // FP32 roundings of the running sums (as in the other two-term kernels)
#pragma unroll 1
    for (int part = TWO_TERM ? 1 : 0; part >= 0; --part) {
#pragma unroll
      for (int t = 0; t < KQ; ++t) {
        const T ar = cur[t].x, ai = cur[t].y, as = ar + ai;
        const T* bp = sB + part * BT + (t * 64 + lane) * W;
        T bv[W];
#pragma unroll
        for (int e = 0; e < W; ++e) bv[e] = bp[e];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          acc[0][mb] = M::op(bv[mb], ar, acc[0][mb]);
          acc[1][mb] = M::op(bv[MB + mb], ai, acc[1][mb]);
          acc[2][mb] = M::op(bv[2 * MB + mb], as, acc[2][mb]);
        }
      }
    }
    const long long bC = tile_base(tbb.chC, v >> rbits) + tb.offRC[row_of_unit(v)];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int n = mb * 16 + M::row_of(g, r);  // MFMA row held in accumulator register r
        C2 o;
        o.x = acc[0][mb][r] - acc[1][mb][r];
        o.y = acc[2][mb][r] - acc[0][mb][r] - acc[1][mb][r];
        if (n < Nn) st_stream(&C[bC + tb.offN[n]], o);
      }
    }
  }
}

// One step of a chain on the LDS tile: the Gauss-form products of k_absorb_mfma_gauss (lane
// group g of k-step t supplies s = 4 t + g; the 16 MFMA rows of block mb are n = 16 mb + 0..15;
// the same k order and the same FP32 operations, so the same results).  A unit is 16 values of
// the step's untouched tile bits f; its outputs overwrite exactly the elements it read, after the
// wave has read all of them (the products consume every read before any write), and the units of
// different waves are disjoint.
// KS > 0 fixes the step's kS at compile time (then the padding tests fold away); KS = 0 reads it.
// TWO: the operator is an FP32 pair, the leading K x K block followed by the residual one; the
// residual's products go into the accumulators first, as in k_absorb_mfma_gauss.
template <int NT, int KQ, int MB, int KS, bool TWO>
__device__ __forceinline__ void chain_step(float2* tile, const float2* __restrict__ B, const ChainStepDesc& sd,
                                           int T) {
  using M = Mfma<float>;
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, g = lane >> 4, l16 = lane & 15, wave = threadIdx.x >> 6;
  const int K = KS > 0 ? 1 << KS : 1 << sd.kS;
  const int units = 1 << (T - sd.kS - 4);
  for (int u = wave; u < units; u += NW) {
    const int f = (u << 4) + l16;
    const int fl = sd.fDig[f & 15] + sd.fDig[16 + ((f >> 4) & 15)] + sd.fDig[32 + ((f >> 8) & 15)];
    float2 a[KQ];
#pragma unroll
    for (int t = 0; t < KQ; ++t) {
      const int s = 4 * t + g;
      const float2 x = tile[fl + sd.sOff[s < K ? s : K - 1]];
      a[t] = s < K ? x : float2{0.f, 0.f};
    }
    M::acc_t acc[3][MB];
#pragma unroll
    for (int x = 0; x < 3; ++x)
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) acc[x][mb] = M::acc_t{0, 0, 0, 0};
#pragma unroll 1
    for (int part = TWO ? 1 : 0; part >= 0; --part) {
      const float2* Bp = B + part * K * K;
#pragma unroll
      for (int t = 0; t < KQ; ++t) {
        const float ar = a[t].x, ai = a[t].y, as = ar + ai;
        const int s = 4 * t + g;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          const int n = mb * 16 + l16;
          const float2 bv = (s < K && n < K) ? Bp[s * K + n] : float2{0.f, 0.f};
          acc[0][mb] = M::op(bv.x, ar, acc[0][mb]);
          acc[1][mb] = M::op(bv.y, ai, acc[1][mb]);
          acc[2][mb] = M::op(bv.x + bv.y, as, acc[2][mb]);
        }
      }
    }
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int n = mb * 16 + M::row_of(g, r);
        if (n < K) {
          float2 o;
          o.x = acc[0][mb][r] - acc[1][mb][r];
          o.y = acc[2][mb][r] - acc[0][mb][r] - acc[1][mb][r];
          tile[fl + sd.sOff[n]] = o;
        }
      }
    }
  }
}

// Split form on the matrix cores (v_mfma_f32_16x16x32_bf16, gfx950).  Operand layout of the
// instruction: lane l supplies A-operand row l % 16, k = 8 (l / 16) .. + 7 and B-operand column
// l % 16, same k (8 BF16 values, 16 bytes); accumulator register v holds row 4 (l / 16) + v.  The
// operator is the A-operand (rows = outputs), the data the B-operand (columns = 16 tile rows of a
// unit).  Operator pieces sit in LDS in fragment order: the P (or 3) 16-byte pieces a lane feeds
// to one instruction are consecutive, so a lane's reads are contiguous and conflict free.
__device__ __forceinline__ floatx4 mfma_bf16(bf16x8 op, bf16x8 x, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(op, x, c, 0, 0, 0);
}

// Gauss form: T1 = sum Re B . Re A, T2 = sum Im B . Im A, T3 = sum (Re B + Im B)(Re A + Im A),
// Re C = T1 - T2, Im C = T3 - T1 - T2; MFMA k runs over s (32 per chunk kc), the 16 rows of block mb
// are n = 16 mb + 0..15.  Fragments (three pieces per lane and instruction) as kernels.h lays out.
__device__ __forceinline__ void copy_frags(const uint4* __restrict__ src, uint4* dst, int n, int tid, int nt) {
  for (int i = tid; i < n; i += nt) dst[i] = src[i];
}

// The Gauss-form split products of one unit (16 columns): a[kc][e] is A at s = 32 kc + 8 g + e for
// this lane's column (zero past K).  T[x][mb] = T1, T2, T3 of output rows n = 16 mb + 4 g + v.  The
// step kernel and the chain kernel both call this, so a chain reproduces its steps bit for bit.
template <int MB, int KC>
__device__ __forceinline__ void gauss6_products(const float2 (&a)[KC][8], const uint4* __restrict__ fr, int lane,
                                                floatx4 (&T)[3][MB]) {
#pragma unroll
  for (int x = 0; x < 3; ++x)
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) T[x][mb] = floatx4{0, 0, 0, 0};
#pragma unroll
  for (int kc = 0; kc < KC; ++kc) {
    float vr[8], vi[8], vs[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      vr[e] = a[kc][e].x;
      vi[e] = a[kc][e].y;
      vs[e] = vr[e] + vi[e];
    }
    bf16x8 A[3][3];
    split3_oct(vr, A[0][0], A[0][1], A[0][2]);
    split3_oct(vi, A[1][0], A[1][1], A[1][2]);
    split3_oct(vs, A[2][0], A[2][1], A[2][2]);
#pragma unroll
    for (int x = 0; x < 3; ++x)
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        const uint4* f = fr + ((((x * MB + mb) * KC + kc) * 64 + lane) * 3);
        const bf16x8 b0 = as_bf16x8(f[0]), b1 = as_bf16x8(f[1]), b2 = as_bf16x8(f[2]);
        floatx4 t = T[x][mb];
        t = mfma_bf16(b0, A[x][2], t);
        t = mfma_bf16(b1, A[x][1], t);
        t = mfma_bf16(b2, A[x][0], t);
        t = mfma_bf16(b0, A[x][1], t);
        t = mfma_bf16(b1, A[x][0], t);
        T[x][mb] = mfma_bf16(b0, A[x][0], t);
      }
  }
}

// Register-direct Gauss-form split kernel (single-term operators, P = 3).  Units, prefetch and
// in-place safety as in k_absorb_mfma_rd: a unit is (tile, block of 16 tile rows), each wave takes
// units independently and loads its next unit while multiplying the current one.
template <int NT, int MB, int KC>
__global__ __launch_bounds__(NT) void k_absorb_split_gauss(const StepDesc* __restrict__ d, const float2* A, float2* C,
                                                           const float4* __restrict__ B) {
  constexpr int NW = NT / 64;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ Tables tb;
  __shared__ TileBases tbb;
  const int kS = d->kS, kN = d->kN, L = d->L, nHi = d->nHi;
  const int K = 1 << kS, Nn = 1 << kN, R = 1 << L;
  const int rbits = L - 4;
  const long long nUnits = d->nTiles << rbits;
  load_tables(d, tb, K, Nn, R, nHi);
  load_tile_bases(d, tbb, nHi);
  uint4* fr = reinterpret_cast<uint4*>(smem);
  copy_frags(reinterpret_cast<const uint4*>(B) + d->frag_gauss, fr, 3 * MB * KC * 64 * 3, threadIdx.x, NT);
  __syncthreads();  // offset tables and operator visible to every wave
  const int lane = threadIdx.x & 63, g = lane >> 4, l16 = lane & 15;
  const long long wstride = (long long)gridDim.x * NW;
  auto row_of_unit = [&](long long v) { return ((int)(v & ((1 << rbits) - 1)) << 4) + l16; };
  float2 nxt[KC][8];
  auto fetch = [&](long long v) {
    const long long bA = tile_base(tbb.chA, v >> rbits) + tb.offRA[row_of_unit(v)];
#pragma unroll
    for (int kc = 0; kc < KC; ++kc)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int sv = 32 * kc + 8 * g + e;
        const float2 x = ld_stream(&A[bA + tb.offS[sv < K ? sv : K - 1]]);  // in-bounds address for every lane
        nxt[kc][e] = sv < K ? x : float2{0.f, 0.f};
      }
  };
  long long v = (long long)blockIdx.x * NW + (threadIdx.x >> 6);
  if (v < nUnits) fetch(v);
  for (; v < nUnits; v += wstride) {
    float2 cur[KC][8];
#pragma unroll
    for (int kc = 0; kc < KC; ++kc)
#pragma unroll
      for (int e = 0; e < 8; ++e) cur[kc][e] = nxt[kc][e];
    if (v + wstride < nUnits) fetch(v + wstride);
    floatx4 T[3][MB];
    gauss6_products<MB, KC>(cur, fr, lane, T);
    const long long bC = tile_base(tbb.chC, v >> rbits) + tb.offRC[row_of_unit(v)];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int n = mb * 16 + 4 * g + r;
        float2 o;
        o.x = T[0][mb][r] - T[1][mb][r];
        o.y = T[2][mb][r] - T[0][mb][r] - T[1][mb][r];
        if (n < Nn) st_stream(&C[bC + tb.offN[n]], o);
      }
  }
}

// Register-direct split kernel on the real embedding (any operator, P = 3 or 4): A_real[r][2s + a],
// B_real[2s + a][2n + b] = [[Re, Im], [-Im, Re]][a][b] of B[s][n].  Block mb holds outputs
// n = 8 mb + 0..7, MFMA row 2 (n - 8 mb) + b (so accumulator registers (0, 1) and (2, 3) of a lane
// are the (Re, Im) pairs of n = 8 mb + 2 g and + 1); chunk kc holds k = 2s + a for s = 16 kc + 4 g
// + 0..3 in lane group g.  Fragments (P pieces per lane and instruction) as kernels.h lays out.
template <int NT, int MB, int KC, int P>
__global__ __launch_bounds__(NT) void k_absorb_split_embed(const StepDesc* __restrict__ d, const float2* A, float2* C,
                                                           const float4* __restrict__ B) {
  constexpr int NW = NT / 64;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ Tables tb;
  __shared__ TileBases tbb;
  const int kS = d->kS, kN = d->kN, L = d->L, nHi = d->nHi;
  const int K = 1 << kS, Nn = 1 << kN, R = 1 << L;
  const int rbits = L - 4;
  const long long nUnits = d->nTiles << rbits;
  load_tables(d, tb, K, Nn, R, nHi);
  load_tile_bases(d, tbb, nHi);
  uint4* fr = reinterpret_cast<uint4*>(smem);
  copy_frags(reinterpret_cast<const uint4*>(B) + d->frag_embed, fr, MB * KC * 64 * P, threadIdx.x, NT);
  __syncthreads();  // offset tables and operator visible to every wave
  const int lane = threadIdx.x & 63, g = lane >> 4, l16 = lane & 15;
  const long long wstride = (long long)gridDim.x * NW;
  auto row_of_unit = [&](long long v) { return ((int)(v & ((1 << rbits) - 1)) << 4) + l16; };
  float2 nxt[KC][4];
  auto fetch = [&](long long v) {
    const long long bA = tile_base(tbb.chA, v >> rbits) + tb.offRA[row_of_unit(v)];
#pragma unroll
    for (int kc = 0; kc < KC; ++kc)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int sv = 16 * kc + 4 * g + e;
        const float2 x = ld_stream(&A[bA + tb.offS[sv < K ? sv : K - 1]]);  // in-bounds address for every lane
        nxt[kc][e] = sv < K ? x : float2{0.f, 0.f};
      }
  };
  long long v = (long long)blockIdx.x * NW + (threadIdx.x >> 6);
  if (v < nUnits) fetch(v);
  for (; v < nUnits; v += wstride) {
    float2 cur[KC][4];
#pragma unroll
    for (int kc = 0; kc < KC; ++kc)
#pragma unroll
      for (int e = 0; e < 4; ++e) cur[kc][e] = nxt[kc][e];
    if (v + wstride < nUnits) fetch(v + wstride);
    floatx4 acc[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) acc[mb] = floatx4{0, 0, 0, 0};
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
      const float vv[8] = {cur[kc][0].x, cur[kc][0].y, cur[kc][1].x, cur[kc][1].y,
                           cur[kc][2].x, cur[kc][2].y, cur[kc][3].x, cur[kc][3].y};
      bf16x8 a0, a1, a2;
      split3_oct(vv, a0, a1, a2);
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        const uint4* f = fr + (((mb * KC + kc) * 64 + lane) * P);
        const bf16x8 b0 = as_bf16x8(f[0]), b1 = as_bf16x8(f[1]), b2 = as_bf16x8(f[2]);
        floatx4 t = acc[mb];
        if (P == 4) t = mfma_bf16(as_bf16x8(f[3]), a0, t);
        t = mfma_bf16(b0, a2, t);
        t = mfma_bf16(b1, a1, t);
        t = mfma_bf16(b2, a0, t);
        t = mfma_bf16(b0, a1, t);
        t = mfma_bf16(b1, a0, t);
        acc[mb] = mfma_bf16(b0, a0, t);
      }
    }
    const long long bC = tile_base(tbb.chC, v >> rbits) + tb.offRC[row_of_unit(v)];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      const floatx4 t = acc[mb];
#pragma unroll
      for (int p2 = 0; p2 < 2; ++p2) {
        const int n = 8 * mb + 2 * g + p2;
        if (n < Nn) st_stream(&C[bC + tb.offN[n]], make_float2(t[2 * p2], t[2 * p2 + 1]));
      }
    }
  }
}

// One step of a split-form chain on the LDS tile: the Gauss-form split products of
// k_absorb_split_gauss (gauss6_products, the same operations in the same order), a unit being 16
// values of the step's untouched tile bits whose outputs overwrite exactly the elements it read.
template <int NT, int MB>
__device__ __forceinline__ void chain_step_split(float2* tile, const uint4* __restrict__ fr, const ChainStepDesc& sd,
                                                 int T) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, g = lane >> 4, l16 = lane & 15, wave = threadIdx.x >> 6;
  const int K = 1 << sd.kS;
  const int units = 1 << (T - sd.kS - 4);
  for (int u = wave; u < units; u += NW) {
    const int f = (u << 4) + l16;
    const int fl = sd.fDig[f & 15] + sd.fDig[16 + ((f >> 4) & 15)] + sd.fDig[32 + ((f >> 8) & 15)];
    float2 a[1][8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int sv = 8 * g + e;
      const float2 x = tile[fl + sd.sOff[sv < K ? sv : K - 1]];
      a[0][e] = sv < K ? x : float2{0.f, 0.f};
    }
    floatx4 Tm[3][MB];
    gauss6_products<MB, 1>(a, fr, lane, Tm);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int n = mb * 16 + 4 * g + r;
        if (n < K) {
          float2 o;
          o.x = Tm[0][mb][r] - Tm[1][mb][r];
          o.y = Tm[2][mb][r] - Tm[0][mb][r] - Tm[1][mb][r];
          tile[fl + sd.sOff[n]] = o;
        }
      }
  }
}

// A chain of in-place steps, one HBM pass (see ChainDesc).  Each workgroup loops over tiles with
// the grid stride: the tile's 2^T elements go from registers into LDS, the next tile's loads are
// issued, every step of the chain runs on the LDS tile (a barrier after each), and the tile goes
// back to HBM.  Element l of the tile belongs to thread l % NT throughout the loads, the LDS fill
// and the stores, so the store phase and the next fill need no barrier between them.  SPLIT: the
// steps compute the split form (operators as BF16 fragments in LDS), else FP32 (complex operators
// in LDS).
template <int NT, bool SPLIT, bool PAIRS = false>
__device__ __forceinline__ void chain_body(const ChainDesc* __restrict__ d, const float2* A, float2* C,
                                           const ChainOps& ops) {
  static_assert(NT % 256 == 0 && NT <= 1024, "digits 0 and 1 of a thread's elements are its own");
  constexpr int EPT = (1 << CHAIN_T) / NT;
  __shared__ float2 tile[1 << CHAIN_T];
  __shared__ ChainStepDesc sd[CHAIN_STEPS];
  __shared__ long long gd[48];
  __shared__ long long hb[NDIG][16];
  extern __shared__ __align__(16) unsigned char smem[];
  const int nsteps = d->nsteps, T = d->T, nHi = d->nHi;
  const long long nTiles = d->nTiles;
  for (int i = threadIdx.x; i < 48; i += NT) gd[i] = d->gDig[i];
  for (int i = threadIdx.x; i < NDIG * 16; i += NT) {
    const int c = i >> 4, m = i & 15;
    long long o = 0;
    for (int b = 0; b < 4; ++b)
      if (((m >> b) & 1) && 4 * c + b < nHi) o |= 1LL << d->hi[4 * c + b];
    hb[c][m] = o;
  }
  {
    const int* src = reinterpret_cast<const int*>(d->st);
    int* dst = reinterpret_cast<int*>(sd);
    const int words = int(sizeof(ChainStepDesc) / sizeof(int)) * nsteps;
    for (int i = threadIdx.x; i < words; i += NT) dst[i] = src[i];
  }
  __syncthreads();  // digit tables visible
  const int E = 1 << T;
  const int tid = threadIdx.x;
  const long long own = gd[tid & 15] + gd[16 + ((tid >> 4) & 15)];
  auto base = [&](long long t) {
    long long b = 0;
#pragma unroll
    for (int c = 0; c < NDIG; ++c) b |= hb[c][(t >> (4 * c)) & 15];
    return b;
  };
  float2 pre[EPT];
  auto fetch = [&](long long t) {
    const long long b = base(t) + own;
#pragma unroll
    for (int k = 0; k < EPT; ++k)
      if (tid + NT * k < E) pre[k] = ld_stream(&A[b + gd[32 + ((tid + NT * k) >> 8)]]);
  };
  // a workgroup with a single tile issues its loads before the operators' (see k_absorb_mfma)
  long long t = blockIdx.x;
  const bool early = nTiles <= (long long)gridDim.x;
  if (early && t < nTiles) fetch(t);
  for (int j = 0; j < nsteps; ++j) {
    const int kS = d->st[j].kS, bo = d->st[j].boff;
    if (SPLIT) {
      copy_frags(static_cast<const uint4*>(ops.B[j]) + d->st[j].frag, reinterpret_cast<uint4*>(smem) + bo,
                 576 * split_gauss_mb(kS), threadIdx.x, NT);
    } else {
      const float2* Bj = static_cast<const float2*>(ops.B[j]);
      float2* sOp = reinterpret_cast<float2*>(smem);
      const int n = (d->st[j].two ? 2 : 1) << (2 * kS);
      for (int i = threadIdx.x; i < n; i += NT) sOp[bo + i] = Bj[i];
    }
  }
  if (!early && t < nTiles) fetch(t);
  __syncthreads();  // operators visible to every wave
  for (; t < nTiles; t += gridDim.x) {
#pragma unroll
    for (int k = 0; k < EPT; ++k)
      if (tid + NT * k < E) tile[tid + NT * k] = pre[k];
    __syncthreads();  // the whole tile is in LDS
    if (t + gridDim.x < nTiles) fetch(t + gridDim.x);
    for (int j = 0; j < nsteps; ++j) {
      if (SPLIT) {
        const uint4* fr = reinterpret_cast<const uint4*>(smem) + sd[j].boff;
        if (sd[j].kS == 5) chain_step_split<NT, 2>(tile, fr, sd[j], T);
        else chain_step_split<NT, 1>(tile, fr, sd[j], T);  // kS = 1 .. 4
      } else {
        const float2* Bj = reinterpret_cast<const float2*>(smem) + sd[j].boff;
        if (PAIRS && sd[j].two) {
          switch (sd[j].kS) {
            case 5: chain_step<NT, 8, 2, 5, true>(tile, Bj, sd[j], T); break;
            case 4: chain_step<NT, 4, 1, 4, true>(tile, Bj, sd[j], T); break;
            case 3: chain_step<NT, 2, 1, 3, true>(tile, Bj, sd[j], T); break;
            default: chain_step<NT, 1, 1, 0, true>(tile, Bj, sd[j], T); break;  // kS = 1, 2
          }
        } else {
          switch (sd[j].kS) {
            case 5: chain_step<NT, 8, 2, 5, false>(tile, Bj, sd[j], T); break;
            case 4: chain_step<NT, 4, 1, 4, false>(tile, Bj, sd[j], T); break;
            case 3: chain_step<NT, 2, 1, 3, false>(tile, Bj, sd[j], T); break;
            default: chain_step<NT, 1, 1, 0, false>(tile, Bj, sd[j], T); break;  // kS = 1, 2
          }
        }
      }
      __syncthreads();  // step j complete on the whole tile
    }
    const long long b = base(t) + own;
#pragma unroll
    for (int k = 0; k < EPT; ++k)
      if (tid + NT * k < E) st_stream(&C[b + gd[32 + ((tid + NT * k) >> 8)]], tile[tid + NT * k]);
  }
}

// FP32 chains at occupancy 3 (three 256-thread workgroups per CU when the operators leave room in
// LDS): with the register budget that gives, the n=16 workload's 2^26-element chain takes 300 us
// against 337 us at the compiler's default of 2 and 406 us with 512-thread workgroups (measured on
// MI355X).  Split-form chains hold up to 36 KB of operator fragments beside the 32 KB tile, so
// two workgroups share a CU.
template <int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3))) void k_chain(const ChainDesc* __restrict__ d,
                                                                                    const float2* A, float2* C,
                                                                                    ChainOps ops) {
  chain_body<NT, false>(d, A, C, ops);
}
// Chains with FP32-pair steps: their own kernel, so that the pair path's registers do not weigh
// on the single-term chains (in one kernel they made the compiler spill the prefetched tile).
template <int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3))) void k_chain_pairs(
    const ChainDesc* __restrict__ d, const float2* A, float2* C, ChainOps ops) {
  chain_body<NT, false, true>(d, A, C, ops);
}
template <int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void k_chain_split(
    const ChainDesc* __restrict__ d, const float2* A, float2* C, ChainOps ops) {
  chain_body<NT, true>(d, A, C, ops);
}

// ---------------------------------------------------------------------- small kernels ---
__global__ void k_zero(double2* out, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    out[i] = make_double2(0.0, 0.0);
}

__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// Double-double sum of |x_i|^2 with a fixed partition and fixed trees (deterministic): block b of
// k_sumsq_part sums the chunk [b c, (b + 1) c) (thread t takes elements t, t + 256, ... of it, then a
// tree over the block) into part[2b], part[2b + 1]; k_sumsq_final adds the G partials the same way
// and writes out[0..1] = the sum, out[2..3] = x_0.  With one block the result is that of a single
// block over all of x.
__device__ __forceinline__ void dd_tree256(double* sh, double* sl, double hi, double lo) {
  sh[threadIdx.x] = hi;
  sl[threadIdx.x] = lo;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      double s, e;
      two_sum(sh[threadIdx.x], sh[threadIdx.x + w], s, e);
      e += sl[threadIdx.x] + sl[threadIdx.x + w];
      double h = s + e;
      sl[threadIdx.x] = e - (h - s);
      sh[threadIdx.x] = h;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_sumsq_part(const double2* x, long long n, long long chunk, double* part) {
  __shared__ double sh[256], sl[256];
  const long long b0 = (long long)blockIdx.x * chunk;
  const long long b1 = b0 + chunk < n ? b0 + chunk : n;
  double hi = 0.0, lo = 0.0;
  for (long long i = b0 + threadIdx.x; i < b1; i += 256) {
    const double2 v = ld_stream(&x[i]);
    const double p = fma(v.x, v.x, v.y * v.y);
    double s, e;
    two_sum(hi, p, s, e);
    hi = s;
    lo += e;
  }
  dd_tree256(sh, sl, hi, lo);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sh[0];
    part[2 * blockIdx.x + 1] = sl[0];
  }
}

// The same sum over a small output in one block: the chunk loop of k_sumsq_part over everything,
// the fixed tree, and the first entry beside it.
__global__ __launch_bounds__(256) void k_sumsq_one(const double2* x, long long n, double* out) {
  __shared__ double sh[256], sl[256];
  double hi = 0.0, lo = 0.0;
  for (long long i = threadIdx.x; i < n; i += 256) {
    const double2 v = ld_stream(&x[i]);
    const double p = fma(v.x, v.x, v.y * v.y);
    double s, e;
    two_sum(hi, p, s, e);
    hi = s;
    lo += e;
  }
  dd_tree256(sh, sl, hi, lo);
  if (threadIdx.x == 0) {
    out[0] = sh[0];
    out[1] = sl[0];
    out[2] = n > 0 ? x[0].x : 0.0;
    out[3] = n > 0 ? x[0].y : 0.0;
  }
}

__global__ __launch_bounds__(256) void k_sumsq_final(const double* part, int G, const double2* x, long long n,
                                                     double* out) {
  __shared__ double sh[256], sl[256];
  double hi = 0.0, lo = 0.0;
  for (int g = threadIdx.x; g < G; g += 256) {
    double s, e;
    two_sum(hi, part[2 * g], s, e);
    e += lo + part[2 * g + 1];
    hi = s + e;
    lo = e - (hi - s);
  }
  dd_tree256(sh, sl, hi, lo);
  if (threadIdx.x == 0) {
    out[0] = sh[0];
    out[1] = sl[0];
    out[2] = n > 0 ? x[0].x : 0.0;
    out[3] = n > 0 ? x[0].y : 0.0;
  }
}


// ------------------------------------------------------------ persistent LDS executor ---
// Items are whole component programs whose tensors fit in LDS.  Each workgroup takes items
// blockIdx.x, blockIdx.x + gridDim.x, ... (static assignment: deterministic results).  A step
// computes every output element with one thread (no in-place: the two buffers alternate).
__device__ __forceinline__ double2 load_op(const void* B, int mode, int idx, int KN) {
  if (mode == KM_F64 || mode == KM_F32_TO_F64) return reinterpret_cast<const double2*>(B)[idx];
  if (mode == KM_SPLIT || mode == KM_SPLIT4) {  // the sum of the pieces
    double2 v = make_double2(0.0, 0.0);
    for (int q = 0; q < (mode == KM_SPLIT4 ? 4 : 3); ++q) {
      const float4 b = reinterpret_cast<const float4*>(B)[q * KN + idx];
      v.x += b.x;
      v.y += b.y;
    }
    return v;
  }
  const float2 h = reinterpret_cast<const float2*>(B)[idx];
  double2 v = make_double2(h.x, h.y);
  if (mode == KM_F32X2) {
    const float2 l = reinterpret_cast<const float2*>(B)[KN + idx];
    v.x += l.x;
    v.y += l.y;
  }
  return v;
}

constexpr int PERSIST_NT = 1024;  // 16 waves: the FP64 products of one component hide each other's latency

__device__ void assemble_result(const double* sums, int ncomp, int alg, double a, double v0re, double v0im,
                                double* res, double* host);

__global__ __launch_bounds__(PERSIST_NT) void k_persistent(const LdsItem* __restrict__ items, int n_items,
                                                           const LdsStep* __restrict__ steps, AssembleArgs as) {
  __shared__ double2 buf[2][1 << LDS_RESIDENT_LOG2];
  __shared__ double2 sB[DMAXK * DMAXK];  // the step's operator, in FP64 (read K times per output)
  // the step's offset tables; LDS-resident tensors have at most 2^LDS_RESIDENT_LOG2 elements
  __shared__ int offS[DMAXK], offN[DMAXK], offRA[DMAXR], offRC[DMAXR], hiA[DMAXHI], hiC[DMAXHI];
  __shared__ double rh[PERSIST_NT], rl[PERSIST_NT];
  __shared__ double2 first;
  const int tid = threadIdx.x;
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const LdsItem item = items[it];
    int cur = -1;  // -1: the scalar 1
    double hi = 0.0, lo = 0.0;
    if (tid == 0) first = make_double2(0.0, 0.0);
    for (int q = 0; q < item.count; ++q) {
      const LdsStep st = steps[item.first + q];
      const StepDesc* d = st.desc;
      const int kS = d->kS, kN = d->kN, L = d->L, nHi = d->nHi;
      const int K = 1 << kS, Nn = 1 << kN, R = 1 << L;
      __syncthreads();  // previous step complete before its tables and operator are replaced
      for (int i = tid; i < K; i += PERSIST_NT) offS[i] = int(d->offS_A[i]);
      for (int i = tid; i < Nn; i += PERSIST_NT) offN[i] = int(d->offN_C[i]);
      for (int i = tid; i < R; i += PERSIST_NT) {
        offRA[i] = int(d->offR_A[i]);
        offRC[i] = int(d->offR_C[i]);
      }
      for (int i = tid; i < nHi; i += PERSIST_NT) {
        hiA[i] = d->hiA[i];
        hiC[i] = d->hiC[i];
      }
      for (int i = tid; i < K * Nn; i += PERSIST_NT) sB[i] = load_op(st.B, st.mode, i, K * Nn);
      __syncthreads();
      const int dst = cur == 0 ? 1 : 0;
      const int total = int(d->nTiles << (kN + L));
      const double2* A = cur < 0 ? nullptr : buf[cur];
      for (int o = tid; o < total; o += PERSIST_NT) {
        const int r = o & (R - 1);
        const int n = (o >> L) & (Nn - 1);
        const int t = o >> (L + kN);
        int bA = 0, bC = 0;
        for (int b = 0; b < nHi; ++b)
          if ((t >> b) & 1) {
            bA |= 1 << hiA[b];
            bC |= 1 << hiC[b];
          }
        double2 acc;
        if (!A) {  // the input is the scalar 1 (a first step: K = 1)
          acc = make_double2(0.0, 0.0);
          for (int s2 = 0; s2 < K; ++s2) acc = make_double2(acc.x + sB[s2 * Nn + n].x, acc.y + sB[s2 * Nn + n].y);
        } else {
          // two independent running sums (even / odd s) keep two FMA chains in flight
          const int a0 = bA + offRA[r];
          double2 e = make_double2(0.0, 0.0), f = make_double2(0.0, 0.0);
          int s2 = 0;
          for (; s2 + 1 < K; s2 += 2) {
            e = cfma(e, A[a0 + offS[s2]], sB[s2 * Nn + n]);
            f = cfma(f, A[a0 + offS[s2 + 1]], sB[(s2 + 1) * Nn + n]);
          }
          if (s2 < K) e = cfma(e, A[a0 + offS[s2]], sB[s2 * Nn + n]);
          acc = make_double2(e.x + f.x, e.y + f.y);
        }
        const int oc = bC + offN[n] + offRC[r];
        if (st.final_step) {
          item.out[oc] = acc;
          const double p = fma(acc.x, acc.x, acc.y * acc.y);
          double sum, err;
          two_sum(hi, p, sum, err);
          hi = sum;
          lo += err;
          if (oc == 0) first = acc;
        } else {
          buf[dst][oc] = acc;
        }
      }
      cur = dst;
    }
    // double-double reduction of the |t|^2 partial sums (fixed tree)
    rh[tid] = hi;
    rl[tid] = lo;
    __syncthreads();
    for (int w = PERSIST_NT / 2; w > 0; w >>= 1) {
      if (tid < w) {
        double sum, err;
        two_sum(rh[tid], rh[tid + w], sum, err);
        err += rl[tid] + rl[tid + w];
        const double h2 = sum + err;
        rl[tid] = err - (h2 - sum);
        rh[tid] = h2;
      }
      __syncthreads();
    }
    if (tid == 0) {
      item.sums[0] = rh[0];
      item.sums[1] = rl[0];
      item.sums[2] = first.x;
      item.sums[3] = first.y;
    }
    __syncthreads();
  }
  if (as.counter && tid == 0) {
    // release this workgroup's sums, count it; the last one acquires every sum and assembles
    const unsigned done = __hip_atomic_fetch_add(as.counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (done == gridDim.x - 1) {
      assemble_result(as.sums, as.ncomp, as.alg, as.a, as.v0re, as.v0im, as.res, as.host);
      __hip_atomic_store(as.counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);  // ready for the next run
    }
  }
}

// ------------------------------------------------------------------------- launchers ---
// When a profiler has set a pair of events, step kernels are launched with them attached to the
// dispatch itself (hipExtLaunchKernelGGL): the events then time the kernel alone, without the
// queue gaps around it.
namespace {
thread_local hipEvent_t t_ev_start = nullptr, t_ev_stop = nullptr;
}
void set_launch_events(hipEvent_t start, hipEvent_t stop) {
  t_ev_start = start;
  t_ev_stop = stop;
}
#define JF_LAUNCH(kernel, grid, block, sm, stream, ...)                                              \
  do {                                                                                             \
    if (t_ev_start)                                                                                \
      hipExtLaunchKernelGGL(kernel, grid, block, uint32_t(sm), stream, t_ev_start, t_ev_stop, 0, __VA_ARGS__); \
    else                                                                                           \
      hipLaunchKernelGGL(kernel, grid, block, sm, stream, __VA_ARGS__);                            \
  } while (0)
static unsigned grid_for(long long nTiles) {
  const long long cap = 256 * 16;
  return unsigned(nTiles < cap ? nTiles : cap);
}

// Grid of the MFMA kernels: as many workgroups as the device holds at once (the kernel's
// occupancy at its LDS size times the compute units), at most one per work item.  Every
// workgroup loops over the items with the grid stride, so the set-up (offset tables, operator
// in LDS, first fetch) is paid once per resident workgroup, the next item's loads overlap the
// current one's products throughout, and no second round of workgroups starts behind a partly
// drained first one.  Occupancies are cached per (device, kernel, block, LDS bytes).  A failed
// query leaves its error for the launch status.
static unsigned resident_grid(const void* kernel, int nt, size_t sm, long long items) {
  struct Key {
    int dev;
    const void* k;
    int nt;
    size_t sm;
    bool operator<(const Key& o) const {
      return std::tie(dev, k, nt, sm) < std::tie(o.dev, o.k, o.nt, o.sm);
    }
  };
  static std::mutex mu;
  static std::map<Key, long long> cache;
  int dev = 0;
  long long cap = 2048;
  if (hipGetDevice(&dev) != hipSuccess) return unsigned(items < cap ? (items < 1 ? 1 : items) : cap);
  {
    std::lock_guard<std::mutex> lk(mu);
    const Key key{dev, kernel, nt, sm};
    auto it = cache.find(key);
    if (it != cache.end()) {
      cap = it->second;
    } else {
      int per_cu = 0, cus = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, nt, sm) == hipSuccess &&
          hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && per_cu > 0 &&
          cus > 0) {
        cap = (long long)per_cu * cus;
        cache[key] = cap;
      }
    }
  }
  return unsigned(items < cap ? (items < 1 ? 1 : items) : cap);
}
#define JF_RESIDENT(kernel, nt, sm, items) resident_grid(reinterpret_cast<const void*>(kernel), nt, sm, items)
// launch of an MFMA step kernel with the resident grid (names NT, sm, stream, d_desc, a, c, b in scope)
#define JF_LAUNCH_RESIDENT(kernel, items) \
  JF_LAUNCH(kernel, dim3(JF_RESIDENT(kernel, NT, sm, items)), dim3(NT), sm, stream, d_desc, a, c, b)

// LDS-staged MFMA launch with the output block count (Nn / 8 blocks of 16 MFMA rows, at least
// one) fixed at compile time.
template <typename T, bool TWO_TERM, int NT>
void launch_staged(const StepDesc& h, hipStream_t stream, const StepDesc* d_desc, const void* A, void* C,
                   const void* B) {
  using C2 = typename Mfma<T>::c2;
  const C2* a = (const C2*)A;
  const C2* b = (const C2*)B;
  C2* c = (C2*)C;
  const int K = 1 << h.kS, Nn = 1 << h.kN, R = 1 << h.L;
  const size_t sm = size_t((TWO_TERM ? 8 : 4) * K * (Nn < 8 ? 8 : Nn) + 2 * K * R) * sizeof(T);
  switch (Nn) {
    case 1: case 2: case 4: case 8: JF_LAUNCH_RESIDENT((k_absorb_mfma<T, TWO_TERM, NT, 1>), h.nTiles); break;
    case 16: JF_LAUNCH_RESIDENT((k_absorb_mfma<T, TWO_TERM, NT, 2>), h.nTiles); break;
    case 32: JF_LAUNCH_RESIDENT((k_absorb_mfma<T, TWO_TERM, NT, 4>), h.nTiles); break;
    default: /* 64, the largest Nn a step may have */ JF_LAUNCH_RESIDENT((k_absorb_mfma<T, TWO_TERM, NT, 8>), h.nTiles); break;
  }
}

// Register-direct launch with (MB, KQ) fixed at compile time.
template <typename T, bool TWO_TERM, int NT, int MB>
void launch_direct_mb(const StepDesc& h, hipStream_t stream, const StepDesc* d_desc, const void* A, void* C,
                      const void* B) {
  using C2 = typename Mfma<T>::c2;
  const C2* a = (const C2*)A;
  const C2* b = (const C2*)B;
  C2* c = (C2*)C;
  const int KQ = ((1 << h.kS) + 3) / 4;
  const long long units = h.nTiles << (h.L - 4);
  const long long wgs = (units + NT / 64 - 1) / (NT / 64);
  const size_t sm = size_t((TWO_TERM ? 2 : 1) * 2 * KQ * 4 * 16 * MB) * sizeof(T);
  switch (KQ) {
    case 1: JF_LAUNCH_RESIDENT((k_absorb_mfma_rd<T, TWO_TERM, NT, MB, 1>), wgs); break;
    case 2: JF_LAUNCH_RESIDENT((k_absorb_mfma_rd<T, TWO_TERM, NT, MB, 2>), wgs); break;
    case 4: JF_LAUNCH_RESIDENT((k_absorb_mfma_rd<T, TWO_TERM, NT, MB, 4>), wgs); break;
    default: JF_LAUNCH_RESIDENT((k_absorb_mfma_rd<T, TWO_TERM, NT, MB, 8>), wgs); break;
  }
}

template <typename T, bool TWO_TERM, int NT>
void launch_direct(const StepDesc& h, hipStream_t stream, const StepDesc* d_desc, const void* A, void* C,
                   const void* B) {
  const int Nn = 1 << h.kN;
  if (Nn <= 8) launch_direct_mb<T, TWO_TERM, NT, 1>(h, stream, d_desc, A, C, B);
  else if (Nn == 16) launch_direct_mb<T, TWO_TERM, NT, 2>(h, stream, d_desc, A, C, B);
  else launch_direct_mb<T, TWO_TERM, NT, 4>(h, stream, d_desc, A, C, B);
}

template <typename T, int NT, int MB, bool TWO_TERM>
void launch_gauss_mb(const StepDesc& h, hipStream_t stream, const StepDesc* d_desc, const void* A, void* C,
                     const void* B) {
  using C2 = typename Mfma<T>::c2;
  const C2* a = (const C2*)A;
  const C2* b = (const C2*)B;
  C2* c = (C2*)C;
  const int KQ = ((1 << h.kS) + 3) / 4;
  const long long units = h.nTiles << (h.L - 4);
  const long long wgs = (units + NT / 64 - 1) / (NT / 64);
  const size_t sm = size_t((TWO_TERM ? 2 : 1) * KQ * 64 * 3 * MB) * sizeof(T);
  switch (KQ) {
    case 1: JF_LAUNCH_RESIDENT((k_absorb_mfma_gauss<T, NT, MB, 1, TWO_TERM>), wgs); break;
    case 2: JF_LAUNCH_RESIDENT((k_absorb_mfma_gauss<T, NT, MB, 2, TWO_TERM>), wgs); break;
    case 4: JF_LAUNCH_RESIDENT((k_absorb_mfma_gauss<T, NT, MB, 4, TWO_TERM>), wgs); break;
    case 8: JF_LAUNCH_RESIDENT((k_absorb_mfma_gauss<T, NT, MB, 8, TWO_TERM>), wgs); break;
    default: JF_LAUNCH_RESIDENT((k_absorb_mfma_gauss<T, NT, MB, 16, TWO_TERM>), wgs); break;
  }
}

template <typename T, int NT, bool TWO_TERM = false>
void launch_gauss(const StepDesc& h, hipStream_t stream, const StepDesc* d_desc, const void* A, void* C,
                  const void* B) {
  if (h.kN <= 4) launch_gauss_mb<T, NT, 1, TWO_TERM>(h, stream, d_desc, A, C, B);
  else if (h.kN == 5) launch_gauss_mb<T, NT, 2, TWO_TERM>(h, stream, d_desc, A, C, B);
  else launch_gauss_mb<T, NT, 4, TWO_TERM>(h, stream, d_desc, A, C, B);
}

// Split-form launches with the operator block counts fixed at compile time.
template <int NT, int MB, int KC>
void launch_split_gauss_mk(const StepDesc& h, hipStream_t stream, const StepDesc* d_desc, const void* A, void* C,
                           const void* B) {
  const float2* a = (const float2*)A;
  const float4* b = (const float4*)B;
  float2* c = (float2*)C;
  const long long units = h.nTiles << (h.L - 4);
  const long long wgs = (units + NT / 64 - 1) / (NT / 64);
  const size_t sm = size_t(3 * MB * KC * 64 * 3) * sizeof(uint4);
  JF_LAUNCH_RESIDENT((k_absorb_split_gauss<NT, MB, KC>), wgs);
}
template <int NT>
void launch_split_gauss(const StepDesc& h, hipStream_t stream, const StepDesc* d_desc, const void* A, void* C,
                        const void* B) {
  if (h.kS == 6) return launch_split_gauss_mk<NT, 1, 2>(h, stream, d_desc, A, C, B);  // kN <= 4
  if (h.kN <= 4) return launch_split_gauss_mk<NT, 1, 1>(h, stream, d_desc, A, C, B);
  if (h.kN == 5) return launch_split_gauss_mk<NT, 2, 1>(h, stream, d_desc, A, C, B);
  launch_split_gauss_mk<NT, 4, 1>(h, stream, d_desc, A, C, B);
}
template <int MB, int KC, int P>
void launch_split_embed_mkp(const StepDesc& h, hipStream_t stream, const StepDesc* d_desc, const void* A, void* C,
                            const void* B) {
  constexpr int NT = 256;
  const float2* a = (const float2*)A;
  const float4* b = (const float4*)B;
  float2* c = (float2*)C;
  const long long units = h.nTiles << (h.L - 4);
  const long long wgs = (units + NT / 64 - 1) / (NT / 64);
  const size_t sm = size_t(MB * KC * 64 * P) * sizeof(uint4);
  JF_LAUNCH_RESIDENT((k_absorb_split_embed<NT, MB, KC, P>), wgs);
}
template <int P>
void launch_split_embed(const StepDesc& h, hipStream_t stream, const StepDesc* d_desc, const void* A, void* C,
                        const void* B) {
  const int MB = h.kN <= 3 ? 1 : 1 << (h.kN - 3), KC = h.kS <= 4 ? 1 : 1 << (h.kS - 4);
  switch (MB * 16 + KC) {
    case 16 + 1: return launch_split_embed_mkp<1, 1, P>(h, stream, d_desc, A, C, B);
    case 16 + 2: return launch_split_embed_mkp<1, 2, P>(h, stream, d_desc, A, C, B);
    case 16 + 4: return launch_split_embed_mkp<1, 4, P>(h, stream, d_desc, A, C, B);
    case 32 + 1: return launch_split_embed_mkp<2, 1, P>(h, stream, d_desc, A, C, B);
    case 32 + 2: return launch_split_embed_mkp<2, 2, P>(h, stream, d_desc, A, C, B);
    case 32 + 4: return launch_split_embed_mkp<2, 4, P>(h, stream, d_desc, A, C, B);
    case 64 + 1: return launch_split_embed_mkp<4, 1, P>(h, stream, d_desc, A, C, B);
    case 64 + 2: return launch_split_embed_mkp<4, 2, P>(h, stream, d_desc, A, C, B);
    default: /* MB 8, KC 1 (split_direct_ok admits no other shape) */ return launch_split_embed_mkp<8, 1, P>(h, stream, d_desc, A, C, B);
  }
}

static bool staged_ok(const StepDesc& h) {
  const int K = 1 << h.kS, R = 1 << h.L;
  return R >= 16 && K >= 2 && K * R <= 4096;
}
static bool direct_ok(const StepDesc& h) { return h.L >= 4 && h.kS <= 5 && h.kN <= 5; }
// (kS + kN <= 10: the larger blocks would spill registers)
static bool gauss_ok(const StepDesc& h) {
  return h.L >= 4 && h.kS <= 6 && h.kN <= 6 && h.kS + h.kN <= 10;
}
// split form: Gauss products for single-term operators; the real embedding for any operator with
// at most 8 blocks x chunks of fragments (<= 32 KB of LDS, registers within budget)
static bool split_gauss_ok(const StepDesc& h) {
  return h.mode == KM_SPLIT && h.L >= 4 && h.kS <= 6 && h.kN <= 6 && h.kS + h.kN <= 10;
}
static bool split_direct_ok(const StepDesc& h) {
  const int MB = h.kN <= 3 ? 1 : 1 << (h.kN - 3), KC = h.kS <= 4 ? 1 : 1 << (h.kS - 4);
  return h.L >= 4 && MB * KC <= 8;
}

bool variant_applies(const StepDesc& h, int v) {
  switch (h.mode) {
    case KM_F64:
    case KM_F32:
    case KM_F32X2:
      if (v == KV_AUTO || v == KV_FMA) return true;
      if (v == KV_STAGED_256 || v == KV_STAGED_512) return staged_ok(h);
      if (v == KV_DIRECT_256 || v == KV_DIRECT_512) return direct_ok(h);
      if (v == KV_GAUSS_256 || v == KV_GAUSS_512) return gauss_ok(h);
      return false;
    case KM_SPLIT:
    case KM_SPLIT4:
      if (v == KV_AUTO || v == KV_FMA) return true;
      if (v == KV_DIRECT_256) return split_direct_ok(h);
      if (v == KV_GAUSS_256 || v == KV_GAUSS_512) return split_gauss_ok(h);
      return false;
    case KM_F32_TO_F64:
      return v == KV_AUTO || v == KV_FMA;
    default:
      return false;
  }
}

// The fixed rule (KV_AUTO), from measurements on MI355X: register-direct for FP64 up to Nn = 32
// and for FP32 with Nn <= 8; for FP32 blocks with K * Nn >= 512 (matrix-core bound at
// 4 products per complex one) the Gauss form; staged MFMA otherwise; FMA for shapes no MFMA
// kernel takes.  Split form: Gauss products where the operator is single-term, the real
// embedding otherwise, FMA where neither applies.
static int auto_variant(const StepDesc& h) {
  const int Nn = 1 << h.kN;
  switch (h.mode) {
    case KM_F64:
      if (direct_ok(h) && Nn <= 32) return KV_DIRECT_256;
      return staged_ok(h) ? KV_STAGED_512 : KV_FMA;
    case KM_F32:
    case KM_F32X2:
      if (direct_ok(h) && Nn <= 8) return KV_DIRECT_512;
      if (h.kS + h.kN >= 9 && gauss_ok(h)) return KV_GAUSS_512;
      return staged_ok(h) ? KV_STAGED_256 : KV_FMA;
    case KM_SPLIT:
    case KM_SPLIT4:
      if (split_gauss_ok(h)) return KV_GAUSS_512;
      return split_direct_ok(h) ? KV_DIRECT_256 : KV_FMA;
    default:
      return KV_FMA;
  }
}

int resolve_variant(const StepDesc& h) {
  return (h.variant != KV_AUTO && variant_applies(h, h.variant)) ? h.variant : auto_variant(h);
}

template <typename T, bool TWO_TERM>
static void launch_mfma_variant(int v, const StepDesc& h, hipStream_t stream, const StepDesc* d_desc, const void* A,
                                void* C, const void* B) {
  if constexpr (!TWO_TERM || std::is_same<T, float>::value) {  // two-term operators exist in FP32 only
    if (v == KV_GAUSS_256) return launch_gauss<T, 256, TWO_TERM>(h, stream, d_desc, A, C, B);
    if (v == KV_GAUSS_512) return launch_gauss<T, 512, TWO_TERM>(h, stream, d_desc, A, C, B);
  }
  switch (v) {
    case KV_STAGED_256: launch_staged<T, TWO_TERM, 256>(h, stream, d_desc, A, C, B); break;
    case KV_STAGED_512: launch_staged<T, TWO_TERM, 512>(h, stream, d_desc, A, C, B); break;
    case KV_DIRECT_256: launch_direct<T, TWO_TERM, 256>(h, stream, d_desc, A, C, B); break;
    default: launch_direct<T, TWO_TERM, 512>(h, stream, d_desc, A, C, B); break;
  }
}

hipError_t launch_step(const StepDesc* d_desc, const StepDesc& h, const void* A, void* C, const void* B,
                       hipStream_t stream) {
  const int K = 1 << h.kS, Nn = 1 << h.kN, R = 1 << h.L;
  const unsigned grid = grid_for(h.nTiles);
  const int v = resolve_variant(h);
  switch (h.mode) {
    case KM_F64:
      if (v != KV_FMA) {
        launch_mfma_variant<double, false>(v, h, stream, d_desc, A, C, B);
      } else {
        size_t sm = size_t(K * Nn + K * R) * sizeof(double2);
        JF_LAUNCH((k_absorb<double2, double2, double2>), dim3(grid), dim3(256), sm, stream, d_desc,
                           (const double2*)A, (double2*)C, (const double2*)B);
      }
      break;
    case KM_F32:
      if (v != KV_FMA) {
        launch_mfma_variant<float, false>(v, h, stream, d_desc, A, C, B);
      } else {
        size_t sm = size_t(K * Nn + K * R) * sizeof(float2);
        JF_LAUNCH((k_absorb<float2, float2, float2>), dim3(grid), dim3(256), sm, stream, d_desc,
                           (const float2*)A, (float2*)C, (const float2*)B);
      }
      break;
    case KM_F32X2:
      if (v != KV_FMA) {
        launch_mfma_variant<float, true>(v, h, stream, d_desc, A, C, B);
      } else {
        size_t sm = size_t(2 * K * Nn + K * R) * sizeof(float2);
        JF_LAUNCH(k_absorb_f32x2, dim3(grid), dim3(256), sm, stream, d_desc, (const float2*)A, (float2*)C,
                           (const float2*)B);
      }
      break;
    case KM_F32_TO_F64: {
      size_t sm = size_t(K * Nn + K * R) * sizeof(double2);
      JF_LAUNCH((k_absorb<float2, double2, double2>), dim3(grid), dim3(256), sm, stream, d_desc,
                         (const float2*)A, (double2*)C, (const double2*)B);
      break;
    }
    case KM_SPLIT:
    case KM_SPLIT4: {
      const bool four = h.mode == KM_SPLIT4;
      if (v == KV_GAUSS_256) launch_split_gauss<256>(h, stream, d_desc, A, C, B);
      else if (v == KV_GAUSS_512) launch_split_gauss<512>(h, stream, d_desc, A, C, B);
      else if (v == KV_DIRECT_256) {
        if (four) launch_split_embed<4>(h, stream, d_desc, A, C, B);
        else launch_split_embed<3>(h, stream, d_desc, A, C, B);
      } else {
        const int P = four ? 4 : 3;
        const size_t sm = size_t(P * K * Nn) * sizeof(uint32_t) + size_t(K * R) * sizeof(float2);
        if (four)
          JF_LAUNCH(k_absorb_split<4>, dim3(grid), dim3(256), sm, stream, d_desc, (const float2*)A, (float2*)C,
                    (const float4*)B);
        else
          JF_LAUNCH(k_absorb_split<3>, dim3(grid), dim3(256), sm, stream, d_desc, (const float2*)A, (float2*)C,
                    (const float4*)B);
      }
      break;
    }
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int step_threads(const StepDesc& h) {
  const int v = resolve_variant(h);
  return (v == KV_STAGED_512 || v == KV_DIRECT_512 || v == KV_GAUSS_512) ? 512 : 256;
}

int chain_threads(const ChainDesc& h) { return !h.split && h.nTiles <= 256 ? 512 : 256; }

hipError_t launch_chain(const ChainDesc* d_desc, const ChainDesc& h, const void* A, void* C, const ChainOps& ops,
                        hipStream_t stream) {
  if (h.nsteps < 1 || h.nsteps > CHAIN_STEPS || h.T < 4 || h.T > CHAIN_T || h.nHi > DMAXHI ||
      h.ops > (h.split ? CHAIN_OPS_SPLIT : CHAIN_OPS))
    return hipErrorInvalidValue;
  for (int j = 0; j < h.nsteps; ++j) {
    const int kS = h.st[j].kS, two = h.st[j].two;
    const int need = h.split ? 576 * (kS > 4 ? 1 << (kS - 4) : 1) : (two ? 2 : 1) << (2 * kS);
    if (kS < 1 || kS > 5 || h.T - kS < 4 || (two != 0 && (two != 1 || h.split)) || h.st[j].boff < 0 ||
        h.st[j].boff + need > h.ops)
      return hipErrorInvalidValue;
  }
  constexpr int NT = 256;
  bool pairs = false;
  for (int j = 0; j < h.nsteps; ++j) pairs = pairs || h.st[j].two;
  // A chain with at most one tile per compute unit keeps most of the device idle while each
  // workgroup runs the steps one after another: there 512-thread workgroups (one unit of a K = 32
  // step per wave on a 2^12 tile) shorten each step (measured on MI355X: the n=25 chain pass
  // 505 -> 495 us; with 512 tiles of 2^9 elements, one unit per step, 9.3 -> 12.4 us a launch).
  const bool wide = chain_threads(h) == 512;
  const size_t smf = size_t(h.ops) * sizeof(float2);
  if (pairs && wide) {
    JF_LAUNCH(k_chain_pairs<512>, dim3(JF_RESIDENT(k_chain_pairs<512>, 512, smf, h.nTiles)), dim3(512), smf, stream,
              d_desc, (const float2*)A, (float2*)C, ops);
  } else if (pairs) {
    JF_LAUNCH(k_chain_pairs<NT>, dim3(JF_RESIDENT(k_chain_pairs<NT>, NT, smf, h.nTiles)), dim3(NT), smf, stream,
              d_desc, (const float2*)A, (float2*)C, ops);
  } else if (wide) {
    JF_LAUNCH(k_chain<512>, dim3(JF_RESIDENT(k_chain<512>, 512, smf, h.nTiles)), dim3(512), smf, stream, d_desc,
              (const float2*)A, (float2*)C, ops);
  } else if (h.split) {
    const size_t sm = size_t(h.ops) * sizeof(uint4);
    JF_LAUNCH(k_chain_split<NT>, dim3(JF_RESIDENT(k_chain_split<NT>, NT, sm, h.nTiles)), dim3(NT), sm, stream, d_desc,
              (const float2*)A, (float2*)C, ops);
  } else {
    const size_t sm = size_t(h.ops) * sizeof(float2);
    JF_LAUNCH(k_chain<NT>, dim3(JF_RESIDENT(k_chain<NT>, NT, sm, h.nTiles)), dim3(NT), sm, stream, d_desc,
              (const float2*)A, (float2*)C, ops);
  }
  return hipGetLastError();
}

hipError_t launch_persistent(const LdsItem* items, int n_items, const LdsStep* steps, hipStream_t stream) {
  if (n_items <= 0) return hipSuccess;
  const int grid = n_items < 2048 ? n_items : 2048;
  hipLaunchKernelGGL(k_persistent, dim3(grid), dim3(PERSIST_NT), 0, stream, items, n_items, steps, AssembleArgs{});
  return hipGetLastError();
}

hipError_t launch_persistent_assemble(const LdsItem* items, int n_items, const LdsStep* steps,
                                      const AssembleArgs& as, hipStream_t stream) {
  if (n_items <= 0 || !as.counter) return hipErrorInvalidValue;
  const int grid = n_items < 2048 ? n_items : 2048;
  hipLaunchKernelGGL(k_persistent, dim3(grid), dim3(PERSIST_NT), 0, stream, items, n_items, steps, as);
  return hipGetLastError();
}

// ---------------------------------------------------------------- streaming-copy ceiling ---
// A plain streaming copy, the reference for what HBM sustains with the access pattern of the
// step kernels: nontemporal loads and stores of BPL bytes per lane, a resident grid looping with
// the grid stride, the next element's load issued before the current one is stored.  (Four loads
// in flight per lane measured slower on MI355X: 4.7 / 4.4 TB/s against 5.3 / 5.0.)
template <int BPL>
__global__ __launch_bounds__(256) void k_stream_copy(const unsigned char* __restrict__ src, unsigned char* __restrict__ dst,
                                                     long long n) {
  typedef float f32v4 __attribute__((ext_vector_type(4)));
  using W = typename std::conditional<BPL == 16, f32v4, f32v2>::type;
  const W* s = reinterpret_cast<const W*>(src);
  W* d = reinterpret_cast<W*>(dst);
  const long long stride = (long long)gridDim.x * blockDim.x;
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  W v = __builtin_nontemporal_load(&s[i]);
  for (; i + stride < n; i += stride) {
    const W w = __builtin_nontemporal_load(&s[i + stride]);
    __builtin_nontemporal_store(v, &d[i]);
    v = w;
  }
  __builtin_nontemporal_store(v, &d[i]);
}

hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, int bpl, hipStream_t stream,
                              hipEvent_t ev0, hipEvent_t ev1) {
  if ((bpl != 8 && bpl != 16) || bytes % size_t(bpl)) return hipErrorInvalidValue;
  const long long n = (long long)(bytes / size_t(bpl));
  if (n == 0) return hipSuccess;
  const void* k = bpl == 16 ? reinterpret_cast<const void*>(k_stream_copy<16>) : reinterpret_cast<const void*>(k_stream_copy<8>);
  const unsigned grid = resident_grid(k, 256, 0, (n + 255) / 256);
  if (bpl == 16)
    hipExtLaunchKernelGGL(k_stream_copy<16>, dim3(grid), dim3(256), 0, stream, ev0, ev1, 0, (const unsigned char*)src,
                          (unsigned char*)dst, n);
  else
    hipExtLaunchKernelGGL(k_stream_copy<8>, dim3(grid), dim3(256), 0, stream, ev0, ev1, 0, (const unsigned char*)src,
                          (unsigned char*)dst, n);
  return hipGetLastError();
}

// F_J of a plan from its components' sums, on the device (one thread).  Algorithm I: the
// double-double product a prod_c (hi_c + lo_c), a = (2^scale |scalar|)^2 (a power of two times the
// squared modulus of the traced-out scalar), F_J = hi + lo and 1 - F_J = (1 - hi) - lo, where 1 - hi
// is exact for hi in [0.5, 2] (Sterbenz).  Algorithm II: T / d^2 = v0 prod_c value_c (complex),
// F_J = Re, 1 - F_J = 1 - Re (exact for Re in [0.5, 2]), |Im| the residual.  res[0..2].
__device__ void assemble_result(const double* sums, int ncomp, int alg, double a, double v0re, double v0im,
                                double* res, double* host) {
  if (alg == 1) {
    double hi = a, lo = 0.0;
    for (int c = 0; c < ncomp; ++c) {
      const double sh = sums[4 * c], sl = sums[4 * c + 1];
      const double h = hi * sh;
      const double l = fma(hi, sh, -h) + hi * sl + lo * sh;
      hi = h + l;
      lo = l - (hi - h);
    }
    res[0] = hi + lo;
    res[1] = (1.0 - hi) - lo;
    res[2] = 0.0;
  } else {
    double vr = v0re, vi = v0im;
    for (int c = 0; c < ncomp; ++c) {
      const double cr = sums[4 * c + 2], ci = sums[4 * c + 3];
      const double nr = vr * cr - vi * ci;
      vi = vr * ci + vi * cr;
      vr = nr;
    }
    res[0] = vr;
    res[1] = 1.0 - vr;
    res[2] = fabs(vi);
  }
  res[3] = 0.0;
  if (host)  // the caller's pinned host landing area: the result needs no copy back
    for (int i = 0; i < 4; ++i) host[i] = res[i];
}

__global__ void k_assemble(const double* sums, int ncomp, int alg, double a, double v0re, double v0im, double* res,
                           double* host) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  assemble_result(sums, ncomp, alg, a, v0re, v0im, res, host);
}

hipError_t launch_assemble(const double* sums, int ncomp, int alg, double a, double v0re, double v0im, double* res,
                           double* host, hipStream_t stream) {
  hipLaunchKernelGGL(k_assemble, dim3(1), dim3(64), 0, stream, sums, ncomp, alg, a, v0re, v0im, res, host);
  return hipGetLastError();
}

__global__ void k_accumulate(double2* out, const double2* part, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double2 a = out[i], b = part[i];
    out[i] = make_double2(a.x + b.x, a.y + b.y);
  }
}

hipError_t launch_accumulate(void* out, const void* part, long long n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  long long blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_accumulate, dim3(unsigned(blocks)), dim3(256), 0, stream, (double2*)out, (const double2*)part, n);
  return hipGetLastError();
}

hipError_t launch_zero(void* out, long long n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  long long blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_zero, dim3(unsigned(blocks)), dim3(256), 0, stream, (double2*)out, n);
  return hipGetLastError();
}

hipError_t launch_sumsq(const void* x, long long n, double* sums, double* scratch, hipStream_t stream) {
  // at least 16K elements per block, at most SUMSQ_BLOCKS blocks; one block takes a small output
  // whole, in one launch
  long long G = (n + 16383) / 16384;
  if (G <= 1) {
    hipLaunchKernelGGL(k_sumsq_one, dim3(1), dim3(256), 0, stream, (const double2*)x, n, sums);
    return hipGetLastError();
  }
  if (G > SUMSQ_BLOCKS) G = SUMSQ_BLOCKS;
  const long long chunk = n > 0 ? (n + G - 1) / G : 0;
  hipLaunchKernelGGL(k_sumsq_part, dim3(unsigned(G)), dim3(256), 0, stream, (const double2*)x, n, chunk, scratch);
  hipLaunchKernelGGL(k_sumsq_final, dim3(1), dim3(256), 0, stream, (const double*)scratch, int(G),
                     (const double2*)x, n, sums);
  return hipGetLastError();
}

}  // namespace jf
