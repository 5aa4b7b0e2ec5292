// GPU executor: uploads a plan's step descriptors and operator blocks into the caller's
// workspace, walks the depth-first tree of sliced Kraus sites (every prefix computed once and
// kept in its level buffer), launches one step kernel per step, reduces each component's output
// in FP64 and assembles F_J on the host from the few FP64 numbers copied back.  Also here: the
// batched submission (one persistent launch for the small components, hipGraph capture), the
// kernel autotuner, per-launch profiling, the early Definition 1 decision, and the FP32 rounding
// of operator blocks.
//
// Workspace layout (every region 256-byte aligned):
//   [step descriptors][operator pools][constants][level buffers][component outputs][sums]
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cfloat>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "jf_internal.h"
#include "kernels.h"

namespace jf {

static_assert(LDS_RESIDENT_MAX == LDS_RESIDENT_LOG2, "the planner's LDS-resident components fit the persistent kernel");

namespace {

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

struct DevLayout {
  size_t desc_off = 0, pool_off = 0, const_off = 0, buf_off = 0, out_off = 0, sums_off = 0, total = 0;
  size_t image_end = 0;  // end of the host image (descriptors, operators, constants, LDS tables)
  size_t sumsq_off = 0;  // scratch of the two-pass sum of |t|^2 (2 SUMSQ_BLOCKS doubles)
  size_t res_off = 0;    // F_J, 1 - F_J, |Im|, written by the device
  size_t lds_items_off = 0, lds_steps_off = 0;
  size_t ctr_off = 0;    // counter of the persistent launch's fused assembly (zero in the image)
  std::vector<size_t> leaf_off;                           // per component with sliced wires: its leaf buffer
  std::vector<int> lds_comps;                             // components run by the persistent kernel
  int lds_steps = 0;
  std::vector<std::vector<size_t>> step_desc;             // per component, per step: descriptor offset
  std::vector<std::vector<size_t>> chain_desc;            // per component, per chain: descriptor offset
  std::vector<std::vector<std::vector<size_t>>> step_b;   // per component, step, variant: B offset
  std::vector<std::vector<size_t>> level_buf;             // per component: 2 buffers per level, offsets in
                                                          // the buffer region [buf_off, total)
};

struct DevState {
  DevLayout lay;
  std::vector<unsigned char> host_image;  // descriptors + pools + constants, uploaded as one copy
  const void* uploaded_to = nullptr;
  size_t uploaded_bytes = 0;
  hipGraphExec_t graph = nullptr;
  const void* graph_ws = nullptr;
  hipStream_t graph_stream = nullptr;
  std::vector<unsigned long long> graph_plans;  // uids of the batch the cached graph was captured for
  std::vector<unsigned> graph_gens;         // and the kernel-choice generation of each plan
  unsigned variant_gen = 0;                 // bumped whenever a step's kernel choice changes
  // single-plan runs: the step program captured once per (workspace, stream, kernel choice)
  hipGraphExec_t run_graph = nullptr;
  const void* run_graph_ws = nullptr;
  hipStream_t run_graph_stream = nullptr;
  unsigned run_graph_gen = 0;
  hipStream_t own_stream = nullptr;         // used when the caller passes the null stream
  // the persistent launch of the small components runs on this stream beside the other
  // components' steps (fork and join by events, also inside a captured graph)
  hipStream_t side_stream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // per component, per chain: 1 = run its steps one launch each (the autotuner found the chain
  // slower, or a kernel variant was forced on every step)
  std::vector<std::vector<char>> chain_off;
  bool validated = false;                   // the program passed validate_program (plans are immutable)
  hipEvent_t ev_order = nullptr, ev0 = nullptr, ev1 = nullptr;
  // pinned host landing area of the component sums (4 doubles each): a pageable destination
  // costs the runtime a staging copy on every call, which small programs feel
  double* pinned_sums = nullptr;
  // pinned host landing area of F_J, 1 - F_J, |Im| (4 doubles), written by the assembly kernel
  // itself: allocated before the first enqueue of the allocating entry points, so every program
  // enqueued or captured after that writes it
  double* pinned_res = nullptr;
  double* pinned_res_dev = nullptr;  // its device address (hipHostGetDevicePointer)
};

std::atomic<unsigned> g_variant_gen{1};

std::mutex g_upload_mu;
// Plans whose tables a workspace holds: start address -> (plan, bytes of the plan's whole region:
// tables, buffers, outputs and sums).  A run writes its whole region, so an upload forgets every
// entry whose region overlaps the new one (a batch member inside a larger plan's buffers, or a
// larger plan over the members of an earlier batch); live entries never overlap.
struct Upload {
  const void* plan;
  size_t bytes;
};
std::map<const void*, Upload> g_last_upload;

// Forget every upload whose region meets [lo, hi) (caller holds g_upload_mu).
void forget_uploads(uintptr_t lo, uintptr_t hi) {
  for (auto it = g_last_upload.begin(); it != g_last_upload.end();) {
    const auto a = reinterpret_cast<uintptr_t>(it->first);
    if (a < hi && lo < a + std::max<size_t>(it->second.bytes, 1)) it = g_last_upload.erase(it);
    else ++it;
  }
}

int mode_of(const Step& st) {
  if (st.compute == C_F64) return st.in_prec == P_C64 ? KM_F32_TO_F64 : KM_F64;
  if (st.compute == C_F32) return st.two_term ? KM_F32X2 : KM_F32;
  return st.two_term ? KM_SPLIT4 : KM_SPLIT;
}

// Nearest BF16 number (ties to even) of an FP32 value, as an FP32 value.
float bf16_rne(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  u &= 0xFFFF0000u;
  float r;
  std::memcpy(&r, &u, 4);
  return r;
}
// Exact three-way split of an FP32 value into BF16 numbers: x = p[0] + p[1] + p[2] (each remainder
// is exact in FP32, and the last has at most 8 significant bits left).
void split3(float x, float p[3]) {
  p[0] = bf16_rne(x);
  const float r1 = x - p[0];
  p[1] = bf16_rne(r1);
  p[2] = bf16_rne(r1 - p[1]);
}

void balanced_round(const std::vector<cd>& M, std::vector<float>& out);

// Split-form operator block (kernels.h): P pieces of float4 entries, then the BF16 fragments of the
// Gauss form (single-term blocks) and of the real embedding.  Offsets in 16-byte units.
struct SplitLayout {
  int P = 3;
  long long gauss = -1, embed = -1, total = 0;
};
SplitLayout split_layout(const Step& st) {
  SplitLayout l;
  l.P = st.two_term ? 4 : 3;
  const long long pieces = (long long)l.P << (st.kS + st.kN);
  long long off = pieces;
  if (!st.two_term) {
    l.gauss = off;
    off += 576LL * split_gauss_mb(st.kN) * split_gauss_kc(st.kS);
  }
  l.embed = off;
  off += 64LL * l.P * split_embed_mb(st.kN) * split_embed_kc(st.kS);
  l.total = off;
  return l;
}
uint32_t bf16_bits(float x) {  // x is a BF16 number
  uint32_t u;
  std::memcpy(&u, &x, 4);
  return u >> 16;
}
uint32_t bf16_pair(float lo, float hi) { return bf16_bits(lo) | (bf16_bits(hi) << 16); }

// Fill one split-form block at dst from the FP64 block M (K x Nn, row-major [s][n]).
void fill_split_block(const Step& st, const std::vector<cd>& M, unsigned char* dst) {
  const SplitLayout l = split_layout(st);
  const int K = 1 << st.kS, Nn = 1 << st.kN;
  const size_t nb = M.size();
  // pieces of the FP32 block (balanced rounding for single-term blocks, as the FP32 steps round),
  // and for two-term blocks a fourth piece: the BF16 residual of the FP64 block
  std::vector<float> bal;
  if (!st.two_term) balanced_round(M, bal);
  std::vector<float> pc(size_t(l.P) * nb * 4, 0.f);  // [q][i][Re, Im, Re + Im, 0]
  for (size_t i = 0; i < nb; ++i) {
    const double re64 = M[i].real(), im64 = M[i].imag();
    const float re = st.two_term ? float(re64) : bal[2 * i], im = st.two_term ? float(im64) : bal[2 * i + 1];
    float pr[3], pi[3], ps[3];
    split3(re, pr);
    split3(im, pi);
    split3(re + im, ps);
    for (int q = 0; q < 3; ++q) {
      pc[(q * nb + i) * 4 + 0] = pr[q];
      pc[(q * nb + i) * 4 + 1] = pi[q];
      pc[(q * nb + i) * 4 + 2] = ps[q];
    }
    if (l.P == 4) {
      pc[(3 * nb + i) * 4 + 0] = bf16_rne(float(re64 - double(re)));
      pc[(3 * nb + i) * 4 + 1] = bf16_rne(float(im64 - double(im)));
    }
  }
  std::memcpy(dst, pc.data(), pc.size() * 4);
  auto piece = [&](int q, int s, int n, int x) {
    return (s < K && n < Nn) ? pc[((size_t(q) * nb) + size_t(s) * Nn + n) * 4 + x] : 0.f;
  };
  uint32_t* w = reinterpret_cast<uint32_t*>(dst);
  if (l.gauss >= 0) {
    const int MB = split_gauss_mb(st.kN), KC = split_gauss_kc(st.kS);
    for (int e = 0; e < 3 * MB * KC * 64 * 3; ++e) {
      const int q = e % 3, rest = e / 3, lane = rest & 63, r2 = rest >> 6;
      const int kc = r2 % KC, r3 = r2 / KC, mb = r3 % MB, x = r3 / MB;
      const int n = 16 * mb + (lane & 15), s0 = 32 * kc + 8 * (lane >> 4);
      for (int dd = 0; dd < 4; ++dd)
        w[4 * (l.gauss + e) + dd] = bf16_pair(piece(q, s0 + 2 * dd, n, x), piece(q, s0 + 2 * dd + 1, n, x));
    }
  }
  const int MB = split_embed_mb(st.kN), KC = split_embed_kc(st.kS);
  for (int e = 0; e < MB * KC * 64 * l.P; ++e) {
    const int q = e % l.P, rest = e / l.P, lane = rest & 63, r2 = rest >> 6;
    const int kc = r2 % KC, mb = r2 / KC;
    const int n = 8 * mb + ((lane & 15) >> 1), b = lane & 1, s0 = 16 * kc + 4 * (lane >> 4);
    for (int dd = 0; dd < 4; ++dd) {
      const float re = piece(q, s0 + dd, n, 0), im = piece(q, s0 + dd, n, 1);
      w[4 * (l.embed + e) + dd] = b == 0 ? bf16_pair(re, -im) : bf16_pair(im, re);
    }
  }
}

// FP32 image of a complex FP64 operator block for single-term FP32 steps.  Every entry is one of
// its two FP32 neighbours; among those choices the rounding keeps Re<B, fl(B) - B> (summed over
// real and imaginary parts) near zero.  In a miter network the rest of the network around a block
// is close to the block's inverse, so that inner product is the first-order change the rounding
// makes to the traces.  Round-to-nearest alone biases it whenever many entries share a value
// (the 1/sqrt(2) of H and T rounds down by 1.7e-8 in FP32, so such blocks shrink every trace by
// the same factor, step after step).  Start from round-to-nearest, then move single entries to
// their other neighbour, largest effect first, while that brings the sum closer to zero.
void balanced_round(const std::vector<cd>& M, std::vector<float>& out) {
  const size_t n = 2 * M.size();
  out.resize(n);
  struct Flip {
    double dT;
    size_t k;
    float alt;
  };
  std::vector<Flip> flips;
  double T = 0;
  for (size_t i = 0; i < n; ++i) {
    const double x = (i & 1) ? M[i / 2].imag() : M[i / 2].real();
    const float f = float(x);
    out[i] = f;
    const double d = double(f) - x;
    T += x * d;
    if (d != 0) {
      const float alt = std::nextafter(f, d > 0 ? -INFINITY : INFINITY);
      flips.push_back({x * (double(alt) - x - d), i, alt});
    }
  }
  std::sort(flips.begin(), flips.end(), [](const Flip& a, const Flip& b) {
    return std::fabs(a.dT) != std::fabs(b.dT) ? std::fabs(a.dT) > std::fabs(b.dT) : a.k < b.k;
  });
  for (const Flip& f : flips)
    if (std::fabs(T + f.dT) < std::fabs(T)) {
      T += f.dT;
      out[f.k] = f.alt;
    }
}

void build_layout(const Program& P, DevState& S) {
  DevLayout& L = S.lay;
  size_t off = 0;
  L.desc_off = 0;
  L.step_desc.resize(P.comps.size());
  for (size_t c = 0; c < P.comps.size(); ++c)
    for (size_t s = 0; s < P.comps[c].steps.size(); ++s) {
      L.step_desc[c].push_back(off);
      off += align256(sizeof(StepDesc));
    }
  L.chain_desc.resize(P.comps.size());
  S.chain_off.resize(P.comps.size());
  for (size_t c = 0; c < P.comps.size(); ++c) {
    S.chain_off[c].assign(P.comps[c].chains.size(), 0);
    for (size_t q = 0; q < P.comps[c].chains.size(); ++q) {
      L.chain_desc[c].push_back(off);
      off += align256(sizeof(ChainDesc));
    }
  }
  L.pool_off = off;
  L.step_b.resize(P.comps.size());
  for (size_t c = 0; c < P.comps.size(); ++c) {
    L.step_b[c].resize(P.comps[c].steps.size());
    for (size_t s = 0; s < P.comps[c].steps.size(); ++s) {
      const Step& st = P.comps[c].steps[s];
      // FP64 steps: double2 blocks; FP32 steps: hi and lo float2 blocks (b = hi + lo to ~48 bits);
      // split steps: pieces and fragments (split_layout)
      const size_t e = st.compute == C_F64 ? 16 : st.two_term ? 16 : 8;
      for (auto& b : st.B) {
        L.step_b[c][s].push_back(off);
        off += align256(st.compute == C_SPLIT ? size_t(split_layout(st).total) * 16 : b.size() * e);
      }
    }
  }
  L.const_off = off;
  off += 256;  // double2 one at +0, float2 one at +16
  for (size_t c = 0; c < P.comps.size(); ++c)
    if (P.comps[c].lds_resident) {
      L.lds_comps.push_back(int(c));
      L.lds_steps += int(P.comps[c].steps.size());
    }
  L.lds_items_off = off;
  off += align256(L.lds_comps.size() * sizeof(LdsItem));
  L.lds_steps_off = off;
  off += align256(size_t(L.lds_steps) * sizeof(LdsStep));
  L.ctr_off = off;
  off += 256;
  L.image_end = off;
  L.out_off = off;
  long long outn = 0;
  for (auto& cp : P.comps) outn += cp.out_len;
  off += align256(size_t(outn) * 16);
  L.leaf_off.assign(P.comps.size(), 0);
  for (size_t c = 0; c < P.comps.size(); ++c)
    if (P.comps[c].accumulate) {
      L.leaf_off[c] = off;
      off += align256(size_t(P.comps[c].leaf_len) * 16);
    }
  L.sums_off = off;
  off += align256(P.comps.size() * 4 * sizeof(double));
  L.res_off = off;
  off += 256;
  L.sumsq_off = off;
  off += align256(2 * SUMSQ_BLOCKS * sizeof(double));
  // the level buffers last: the members of a batch, which run one after another on one stream,
  // share one buffer region (jf_fidelity_batch)
  L.buf_off = off;
  size_t maxbuf = 0;
  L.level_buf.resize(P.comps.size());
  for (size_t c = 0; c < P.comps.size(); ++c) {
    size_t o = 0;
    if (P.comps[c].lds_resident) {
      L.level_buf[c].assign(2 * P.comps[c].levels.size(), 0);
      continue;
    }
    for (auto& lv : P.comps[c].levels) {
      L.level_buf[c].push_back(o);
      o += align256(lv.buf_bytes);
      L.level_buf[c].push_back(o);
      o += align256(lv.buf_bytes);
    }
    maxbuf = std::max(maxbuf, o);
  }
  L.total = off + maxbuf;

  // host image of descriptors, pools and constants
  S.host_image.assign(L.image_end, 0);
  for (size_t c = 0; c < P.comps.size(); ++c)
    for (size_t s = 0; s < P.comps[c].steps.size(); ++s) {
      const Step& st = P.comps[c].steps[s];
      StepDesc d;
      std::memset(&d, 0, sizeof(d));
      for (size_t i = 0; i < st.offS_A.size(); ++i) d.offS_A[i] = st.offS_A[i];
      for (size_t i = 0; i < st.offR_A.size(); ++i) d.offR_A[i] = st.offR_A[i];
      for (size_t i = 0; i < st.offN_C.size(); ++i) d.offN_C[i] = st.offN_C[i];
      for (size_t i = 0; i < st.offR_C.size(); ++i) d.offR_C[i] = st.offR_C[i];
      for (size_t i = 0; i < st.hiA.size(); ++i) {
        d.hiA[i] = st.hiA[i];
        d.hiC[i] = st.hiC[i];
      }
      d.nHi = int(st.hiA.size());
      for (int q = 0; q < DMAXHI / 4 * 16; ++q) {
        const int c = q >> 4, m = q & 15;
        long long a = 0, o = 0;
        for (int b = 0; b < 4; ++b)
          if (((m >> b) & 1) && 4 * c + b < d.nHi) {
            a |= 1LL << st.hiA[4 * c + b];
            o |= 1LL << st.hiC[4 * c + b];
          }
        d.digA[q] = a;
        d.digC[q] = o;
      }
      d.kS = st.kS;
      d.kN = st.kN;
      d.L = st.L;
      d.nTiles = st.nTiles;
      d.mode = mode_of(st);
      d.frag_gauss = d.frag_embed = -1;
      if (st.compute == C_SPLIT) {
        const SplitLayout sl = split_layout(st);
        d.frag_gauss = int(sl.gauss);
        d.frag_embed = int(sl.embed);
      }
      std::memcpy(&S.host_image[L.step_desc[c][s]], &d, sizeof(d));
      for (size_t v = 0; v < st.B.size(); ++v) {
        unsigned char* dst = &S.host_image[L.step_b[c][s][v]];
        if (st.compute == C_F64) {
          for (size_t i = 0; i < st.B[v].size(); ++i) {
            double re = st.B[v][i].real(), im = st.B[v][i].imag();
            std::memcpy(dst + 16 * i, &re, 8);
            std::memcpy(dst + 16 * i + 8, &im, 8);
          }
        } else if (st.compute == C_SPLIT) {
          fill_split_block(st, st.B[v], dst);
        } else {
          const size_t nb = st.B[v].size();
          std::vector<float> bal;
          const bool single = !st.two_term;
          if (single) balanced_round(st.B[v], bal);
          for (size_t i = 0; i < nb; ++i) {
            float re = float(st.B[v][i].real()), im = float(st.B[v][i].imag());
            if (single) {
              re = bal[2 * i];
              im = bal[2 * i + 1];
            }
            std::memcpy(dst + 8 * i, &re, 4);
            std::memcpy(dst + 8 * i + 4, &im, 4);
            if (!single) {
              float rl = float(st.B[v][i].real() - double(re)), il = float(st.B[v][i].imag() - double(im));
              std::memcpy(dst + 8 * (nb + i), &rl, 4);
              std::memcpy(dst + 8 * (nb + i) + 4, &il, 4);
            }
          }
        }
      }
    }
  for (size_t c = 0; c < P.comps.size(); ++c)
    for (size_t q = 0; q < P.comps[c].chains.size(); ++q) {
      const Chain& ch = P.comps[c].chains[q];
      ChainTables tb;
      chain_tables(P.comps[c], ch, tb);
      ChainDesc d;
      std::memset(&d, 0, sizeof(d));
      for (int i = 0; i < 48; ++i) d.gDig[i] = tb.gDig[i / 16][i % 16];
      for (size_t i = 0; i < ch.hi.size(); ++i) d.hi[i] = ch.hi[i];
      d.nTiles = ch.nTiles;
      d.nsteps = ch.last - ch.first;
      d.T = ch.T;
      d.nHi = int(ch.hi.size());
      d.split = P.comps[c].steps[ch.first].compute == C_SPLIT ? 1 : 0;
      int boff = 0;
      for (int j = 0; j < d.nsteps; ++j) {
        const Step& st = P.comps[c].steps[ch.first + j];
        d.st[j].kS = st.kS;
        d.st[j].boff = boff;
        d.st[j].frag = d.split ? int(split_layout(st).gauss) : 0;
        d.st[j].two = st.two_term ? 1 : 0;
        boff += chain_step_ops(st.kS, d.split != 0, st.two_term);
        for (size_t i = 0; i < tb.sOff[j].size(); ++i) d.st[j].sOff[i] = tb.sOff[j][i];
        for (int i = 0; i < 48; ++i) d.st[j].fDig[i] = tb.fDig[j][i];
      }
      d.ops = boff;
      std::memcpy(&S.host_image[L.chain_desc[c][q]], &d, sizeof(d));
    }
  double one = 1.0, zero = 0.0;
  float onef = 1.0f, zerof = 0.0f;
  std::memcpy(&S.host_image[L.const_off], &one, 8);
  std::memcpy(&S.host_image[L.const_off + 8], &zero, 8);
  std::memcpy(&S.host_image[L.const_off + 16], &onef, 4);
  std::memcpy(&S.host_image[L.const_off + 20], &zerof, 4);
}

// Persistent-kernel tables of a plan whose workspace starts at ws (absolute device pointers).
void fill_lds_tables(const Program& P, const DevLayout& L, unsigned char* ws, LdsItem* items, LdsStep* steps,
                     int step_base) {
  int si = 0;
  for (size_t q = 0; q < L.lds_comps.size(); ++q) {
    const int c = L.lds_comps[q];
    const ComponentProgram& cp = P.comps[c];
    LdsItem it;
    it.first = step_base + si;
    it.count = int(cp.steps.size());
    it.out = reinterpret_cast<double2*>(ws + L.out_off + size_t(cp.out_off) * 16);
    it.sums = reinterpret_cast<double*>(ws + L.sums_off) + 4 * c;
    it.out_len = cp.out_len;
    items[q] = it;
    for (size_t k = 0; k < cp.steps.size(); ++k) {
      LdsStep e;
      e.desc = reinterpret_cast<const StepDesc*>(ws + L.step_desc[c][k]);
      e.B = ws + L.step_b[c][k][0];
      e.mode = mode_of(cp.steps[k]);
      e.final_step = cp.steps[k].final_step ? 1 : 0;
      steps[si++] = e;
    }
  }
}

DevState& state_of(jf_plan* p) {
  if (!p->dev) {
    auto* s = new DevState;
    build_layout(p->prog, *s);
    p->dev = s;
  }
  return *static_cast<DevState*>(p->dev);
}

#define JF_HIP(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) {                                                            \
      set_error(std::string(#call) + ": " + hipGetErrorString(e_));                    \
      return JF_E_HIP;                                                                 \
    }                                                                                  \
  } while (0)

struct Prof {
  std::vector<hipEvent_t> ev;  // pairs around every contraction-step launch (owned)
  std::vector<jf_step_profile> rec;  // one per launch, ms filled in after the run
  double bytes = 0, flops = 0;
  Prof() = default;
  Prof(const Prof&) = delete;
  Prof& operator=(const Prof&) = delete;
  ~Prof() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
};

// Two timing events, destroyed on every way out of the scope that made them.
struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  ~EventPair() {
    if (a) hipEventDestroy(a);
    if (b) hipEventDestroy(b);
  }
};

// Autotuning state of one run: which steps have been timed already.
struct Tune {
  int reps = 3;
  std::vector<std::vector<char>> done;
};

// Process-wide cache of tuned choices, keyed by step shape.
std::mutex g_tune_mu;
std::map<std::vector<long long>, int> g_tune_cache;

// Time every variant that can run this step (on its real input and output buffers) and keep the
// fastest in the host descriptor.  In-place steps are re-applied to their own output: the data
// is garbage afterwards, which is why tuning runs are never used for results.
jf_status tune_step(StepDesc* hd, const StepDesc* dd, const void* A, void* C, const void* B, hipStream_t stream,
                    int reps, bool inplace) {
  const std::vector<long long> key = {hd->mode, hd->kS, hd->kN, hd->L, hd->nTiles, inplace ? 1 : 0};
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      hd->variant = it->second;
      return JF_OK;
    }
  }
  EventPair ev;
  JF_HIP(hipEventCreate(&ev.a));
  JF_HIP(hipEventCreate(&ev.b));
  hipEvent_t e0 = ev.a, e1 = ev.b;
  int best = KV_AUTO;
  float best_ms = FLT_MAX;
  for (int v = KV_AUTO + 1; v < KV_COUNT; ++v) {
    if (!variant_applies(*hd, v)) continue;
    hd->variant = v;
    JF_HIP(launch_step(dd, *hd, A, C, B, stream));  // warm-up
    JF_HIP(hipEventRecord(e0, stream));
    for (int r = 0; r < reps; ++r) JF_HIP(launch_step(dd, *hd, A, C, B, stream));
    JF_HIP(hipEventRecord(e1, stream));
    JF_HIP(hipEventSynchronize(e1));
    float ms = 0;
    JF_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best_ms) {
      best_ms = ms;
      best = v;
    }
  }
  hd->variant = best;
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune_cache[key] = best;
  return JF_OK;
}

// Process-wide cache of chain decisions (1 = run the steps one launch each), keyed by the chain's
// tile shape and its steps' shapes and kernels.
std::map<std::vector<long long>, int> g_chain_cache;

// Time a chain against its steps run one launch each (every step with its tuned kernel, in place
// on the chain's output after the first) and keep the faster.  Like tune_step, this clobbers the
// data.
jf_status tune_chain(DevState& S, size_t c, int q, const ChainDesc* dd, const ChainDesc& hd,
                     const void* A, void* C, const ChainOps& ops, const std::vector<const StepDesc*>& sdd,
                     const std::vector<const StepDesc*>& shd, hipStream_t stream, int reps) {
  std::vector<long long> key = {hd.T, hd.nTiles, A == C ? 1 : 0, hd.split};
  for (const StepDesc* h : shd) {
    key.push_back(h->kS);
    key.push_back(resolve_variant(*h));
  }
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_chain_cache.find(key);
    if (it != g_chain_cache.end()) {
      S.chain_off[c][q] = char(it->second);
      return JF_OK;
    }
  }
  auto run_steps = [&]() -> hipError_t {
    for (size_t j = 0; j < shd.size(); ++j) {
      const hipError_t e = launch_step(sdd[j], *shd[j], j == 0 ? A : C, C, ops.B[j], stream);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  EventPair ev;
  JF_HIP(hipEventCreate(&ev.a));
  JF_HIP(hipEventCreate(&ev.b));
  hipEvent_t e0 = ev.a, e1 = ev.b;
  float ms[2] = {0, 0};
  for (int mode = 0; mode < 2; ++mode) {
    JF_HIP(mode == 0 ? launch_chain(dd, hd, A, C, ops, stream) : run_steps());  // warm-up
    JF_HIP(hipEventRecord(e0, stream));
    for (int r = 0; r < reps; ++r) JF_HIP(mode == 0 ? launch_chain(dd, hd, A, C, ops, stream) : run_steps());
    JF_HIP(hipEventRecord(e1, stream));
    JF_HIP(hipEventSynchronize(e1));
    JF_HIP(hipEventElapsedTime(&ms[mode], e0, e1));
  }
  S.chain_off[c][q] = ms[0] <= ms[1] ? 0 : 1;
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_chain_cache[key] = S.chain_off[c][q];
  return JF_OK;
}

// Enqueue the steps of level lv of component c for Kraus variant v of the level's sliced site,
// starting from `parent` (nullptr: the constant 1 of the first step's precision), the component's
// output at element offset `base`; *end receives the level's last output (no synchronisation).
jf_status enqueue_level(jf_plan* p, unsigned char* ws, unsigned char* bufs, hipStream_t stream, size_t c, int lv,
                        const std::vector<int>& vv, const void* parent, long long base, const void** end, Prof* prof,
                        Tune* tune) {
  const ComponentProgram& cp = p->prog.comps[c];
  DevState& S = state_of(p);
  const DevLayout& L = S.lay;
  const Level& lev = cp.levels[lv];
  unsigned char* out = ws + L.out_off + size_t(cp.out_off) * 16;
  const void* cur = parent;
  if (!cur) {
    const Step& s0 = cp.steps[lev.first < lev.last ? lev.first : 0];
    cur = ws + L.const_off + (s0.in_prec == P_C64 ? 16 : 0);
  }
  unsigned char* b0 = bufs + L.level_buf[c][2 * lv];
  unsigned char* b1 = bufs + L.level_buf[c][2 * lv + 1];
  for (int si = lev.first; si < lev.last; ++si) {
    const Step& st = cp.steps[si];
    if (st.chain >= 0 && cp.chains[st.chain].first == si && (tune || !S.chain_off[c][st.chain])) {
      // a chain: steps [first, last) in one launch, in place when the input is this level's
      const Chain& ch = cp.chains[st.chain];
      void* dst = (cur == b0 || cur == b1) ? const_cast<void*>(cur) : b0;
      ChainOps ops = {};
      std::vector<const StepDesc*> sdd, shd;
      for (int q = ch.first; q < ch.last; ++q) {
        ops.B[q - ch.first] = ws + L.step_b[c][q][variant_index(cp, cp.steps[q], vv)];
        sdd.push_back(reinterpret_cast<const StepDesc*>(ws + L.step_desc[c][q]));
        shd.push_back(reinterpret_cast<const StepDesc*>(&S.host_image[L.step_desc[c][q]]));
      }
      const ChainDesc* dd = reinterpret_cast<const ChainDesc*>(ws + L.chain_desc[c][st.chain]);
      const ChainDesc& hd = *reinterpret_cast<const ChainDesc*>(&S.host_image[L.chain_desc[c][st.chain]]);
      if (tune && !tune->done[c][si]) {
        for (int q = ch.first; q < ch.last; ++q) {  // the steps' own kernels first
          jf_status ts = tune_step(const_cast<StepDesc*>(shd[q - ch.first]), sdd[q - ch.first], q == ch.first ? cur : dst,
                                   dst, ops.B[q - ch.first], stream, tune->reps, q == ch.first ? dst == cur : true);
          if (ts != JF_OK) return ts;
          tune->done[c][q] = 1;
        }
        jf_status ts = tune_chain(S, c, st.chain, dd, hd, cur, dst, ops, sdd, shd, stream, tune->reps);
        if (ts != JF_OK) return ts;
      }
      if (!S.chain_off[c][st.chain]) {
        if (prof) {
          hipEvent_t a = nullptr, b = nullptr;
          JF_HIP(hipEventCreate(&a));
          prof->ev.push_back(a);
          JF_HIP(hipEventCreate(&b));
          prof->ev.push_back(b);
          set_launch_events(a, b);
          const hipError_t le = launch_chain(dd, hd, cur, dst, ops, stream);
          set_launch_events(nullptr, nullptr);
          JF_HIP(le);
          prof->bytes += ch.bytes;
          prof->flops += ch.flops;
          jf_step_profile r = {};
          r.flops = ch.flops;
          r.bytes = ch.bytes;
          for (const StepDesc* h : shd) r.kS = std::max(r.kS, h->kS);
          r.kN = r.kS;
          r.L = ch.T;
          bool pairs = false;
          for (int j = 0; j < hd.nsteps; ++j) pairs = pairs || hd.st[j].two;
          r.mode = hd.split ? KM_SPLIT : pairs ? KM_F32X2 : KM_F32;
          r.variant = KV_CHAIN;
          r.component = int(c);
          r.steps = ch.last - ch.first;
          r.threads = chain_threads(hd);
          prof->rec.push_back(r);
        } else {
          JF_HIP(launch_chain(dd, hd, cur, dst, ops, stream));
        }
        cur = dst;
        si = ch.last - 1;
        continue;
      }
    }
    void* dst;
    if (st.final_step) {
      // with sliced wires the leaf's partial result goes to the leaf buffer and is added in below
      dst = cp.accumulate ? static_cast<void*>(ws + L.leaf_off[c]) : static_cast<void*>(out + size_t(base) * 16);
    } else if (st.inplace_ok && st.in_prec == st.out_prec && (cur == b0 || cur == b1)) {
      dst = const_cast<void*>(cur);
    } else {
      dst = (cur == b0) ? b1 : b0;
    }
    const size_t var = variant_index(cp, st, vv);
    const StepDesc* dd = reinterpret_cast<const StepDesc*>(ws + L.step_desc[c][si]);
    const StepDesc* hd = reinterpret_cast<const StepDesc*>(&S.host_image[L.step_desc[c][si]]);
    const void* B = ws + L.step_b[c][si][var];
    if (tune && !tune->done[c][si]) {
      jf_status ts = tune_step(const_cast<StepDesc*>(hd), dd, cur, dst, B, stream, tune->reps, dst == cur);
      if (ts != JF_OK) return ts;
      tune->done[c][si] = 1;
    }
    if (prof) {
      hipEvent_t a = nullptr, b = nullptr;
      JF_HIP(hipEventCreate(&a));
      prof->ev.push_back(a);
      JF_HIP(hipEventCreate(&b));
      prof->ev.push_back(b);
      set_launch_events(a, b);
      const hipError_t le = launch_step(dd, *hd, cur, dst, B, stream);
      set_launch_events(nullptr, nullptr);
      JF_HIP(le);
      prof->bytes += st.bytes;
      prof->flops += st.flops;
      jf_step_profile r = {};
      r.flops = st.flops;
      r.bytes = st.bytes;
      r.kS = st.kS;
      r.kN = st.kN;
      r.L = st.L;
      r.mode = hd->mode;
      r.variant = resolve_variant(*hd);
      r.component = int(c);
      r.steps = 1;
      r.threads = step_threads(*hd);
      prof->rec.push_back(r);
    } else {
      JF_HIP(launch_step(dd, *hd, cur, dst, B, stream));
    }
    if (st.final_step && cp.accumulate)
      JF_HIP(launch_accumulate(out + size_t(base) * 16, dst, cp.leaf_len, stream));
    cur = dst;
  }
  *end = cur;
  return JF_OK;
}

// Clear component c's output and walk its levels depth first: every prefix is computed once and
// kept in its level buffer while the Kraus operators of the next sliced site are iterated.
jf_status enqueue_component(jf_plan* p, unsigned char* ws, unsigned char* bufs, hipStream_t stream, size_t c, Prof* prof,
                            Tune* tune) {
  const ComponentProgram& cp = p->prog.comps[c];
  const DevLayout& L = state_of(p).lay;
  // Every output entry is written by the final steps of the leaves, except where leaves add
  // partial traces into it (sliced wires) or a site's Kraus count is no power of two (padded
  // variants): only then is the output cleared first.
  bool clear = cp.accumulate;
  for (size_t site = 0; site < cp.out_bit.size() && site < p->prog.site_nk.size() && !clear; ++site) {
    const int nk = p->prog.site_nk[site];
    if (!cp.out_bit[site].empty() && (nk & (nk - 1))) clear = true;
  }
  if (clear) JF_HIP(launch_zero(ws + L.out_off + size_t(cp.out_off) * 16, cp.out_len, stream));
  struct Frame {
    int lv;
    int v;
    const void* parent;
    long long base;
  };
  std::vector<int> vv(cp.levels.size(), 0);  // the values of the levels on the current path
  std::vector<Frame> stack;
  stack.push_back({0, 0, nullptr, 0});
  while (!stack.empty()) {
    Frame f = stack.back();
    stack.pop_back();
    const Level& lev = cp.levels[f.lv];
    if (f.v + 1 < lev.nvar) stack.push_back({f.lv, f.v + 1, f.parent, f.base});
    vv[f.lv] = f.v;
    const long long base = f.base + f.v * lev.out_stride;
    const void* cur = nullptr;
    jf_status st = enqueue_level(p, ws, bufs, stream, c, f.lv, vv, f.parent, base, &cur, prof, tune);
    if (st != JF_OK) return st;
    if (f.lv + 1 < (int)cp.levels.size()) stack.push_back({f.lv + 1, 0, cur, base});
  }
  return JF_OK;
}

// Enqueue the whole program (no synchronisation, no host copies): used eagerly and for capture.
// bufs: the level-buffer region (nullptr: the plan's own, at the end of its workspace).
// The plan's side stream and its fork / join events (created on first use, default priority).
jf_status side_of(jf_plan* p, hipStream_t* side) {
  DevState& S = state_of(p);
  // each object once (a failure part-way leaves the ones made for the next call to keep)
  if (!S.ev_fork) JF_HIP(hipEventCreateWithFlags(&S.ev_fork, hipEventDisableTiming));
  if (!S.ev_join) JF_HIP(hipEventCreateWithFlags(&S.ev_join, hipEventDisableTiming));
  if (!S.side_stream) JF_HIP(hipStreamCreateWithFlags(&S.side_stream, hipStreamNonBlocking));
  *side = S.side_stream;
  return JF_OK;
}

// Launch the persistent kernel over items on `side` (forked from and joined back to `stream` by
// fork / join; the caller waits on join) or, with no side stream, on `stream` itself.
jf_status launch_persistent_beside(const LdsItem* items, int n, const LdsStep* steps, hipStream_t stream,
                                   hipStream_t side, hipEvent_t fork, hipEvent_t join) {
  if (!side) {
    JF_HIP(launch_persistent(items, n, steps, stream));
    return JF_OK;
  }
  JF_HIP(hipEventRecord(fork, stream));
  JF_HIP(hipStreamWaitEvent(side, fork, 0));
  JF_HIP(launch_persistent(items, n, steps, side));
  JF_HIP(hipEventRecord(join, side));
  return JF_OK;
}

// Enqueue one whole pass of a plan.  side: a stream for the persistent launch of the small
// components, which then overlaps the other components' steps (one workgroup per component, so
// it leaves the rest of the device to them); null runs everything on `stream` in order.
// Arguments of the assembly of a plan's F_J from its component sums (device addresses in ws).
AssembleArgs assemble_args(jf_plan* p, unsigned char* ws) {
  const Program& P = p->prog;
  const DevState& S = state_of(p);
  const double s = std::exp2(P.log2_scale);  // exact: an integer power of two
  const cd v0 = s * P.scalar;
  AssembleArgs a;
  a.sums = reinterpret_cast<const double*>(ws + S.lay.sums_off);
  a.ncomp = int(P.comps.size());
  a.alg = P.opt.alg;
  a.a = s * s * std::norm(P.scalar);
  a.v0re = v0.real();
  a.v0im = v0.imag();
  a.res = reinterpret_cast<double*>(ws + S.lay.res_off);
  a.host = S.pinned_res_dev;
  a.counter = reinterpret_cast<unsigned*>(ws + S.lay.ctr_off);
  return a;
}

// The product over components and 1 - F_J of a plan, on the device (after all its components).
jf_status enqueue_assemble(jf_plan* p, unsigned char* ws, hipStream_t stream) {
  const AssembleArgs a = assemble_args(p, ws);
  JF_HIP(launch_assemble(a.sums, a.ncomp, a.alg, a.a, a.v0re, a.v0im, a.res, a.host, stream));
  return JF_OK;
}

jf_status enqueue_program(jf_plan* p, unsigned char* ws, hipStream_t stream, Prof* prof = nullptr,
                          bool skip_lds = false, Tune* tune = nullptr, unsigned char* bufs = nullptr,
                          hipStream_t side = nullptr, bool assemble = true) {
  const Program& P = p->prog;
  DevState& S = state_of(p);
  const DevLayout& L = S.lay;
  if (!bufs) bufs = ws + L.buf_off;
  const bool lds = !skip_lds && !L.lds_comps.empty();
  if (lds && assemble && L.lds_comps.size() == P.comps.size()) {
    // every component in the persistent launch, which also assembles: one launch per run
    JF_HIP(launch_persistent_assemble(reinterpret_cast<const LdsItem*>(ws + L.lds_items_off),
                                      int(L.lds_comps.size()),
                                      reinterpret_cast<const LdsStep*>(ws + L.lds_steps_off), assemble_args(p, ws),
                                      stream));
    return JF_OK;
  }
  if (!lds) side = nullptr;
  if (lds) {
    const jf_status st = launch_persistent_beside(reinterpret_cast<const LdsItem*>(ws + L.lds_items_off),
                                                  int(L.lds_comps.size()),
                                                  reinterpret_cast<const LdsStep*>(ws + L.lds_steps_off), stream,
                                                  side, S.ev_fork, S.ev_join);
    if (st != JF_OK) return st;
  }
  for (size_t c = 0; c < P.comps.size(); ++c) {
    const ComponentProgram& cp = P.comps[c];
    if (cp.lds_resident) continue;
    jf_status st = enqueue_component(p, ws, bufs, stream, c, prof, tune);
    if (st != JF_OK) return st;
    JF_HIP(launch_sumsq(ws + L.out_off + size_t(cp.out_off) * 16, cp.out_len,
                        reinterpret_cast<double*>(ws + L.sums_off) + 4 * c,
                        reinterpret_cast<double*>(ws + L.sumsq_off), stream));
  }
  if (side) JF_HIP(hipStreamWaitEvent(stream, S.ev_join, 0));
  return assemble ? enqueue_assemble(p, ws, stream) : JF_OK;
}

// Copy the plan's tables into ws (unless they are there already).  region: the bytes from ws on
// that the plan's runs write (0: its whole workspace); every other upload in it is forgotten.
jf_status upload(jf_plan* p, void* ws, hipStream_t stream, size_t region = 0) {
  DevState& S = state_of(p);
  if (!region) region = S.lay.total;
  std::lock_guard<std::mutex> g(g_upload_mu);
  if (S.uploaded_to == ws) {
    auto it = g_last_upload.find(ws);
    if (it != g_last_upload.end() && it->second.plan == p) return JF_OK;
  }
  fill_lds_tables(p->prog, S.lay, static_cast<unsigned char*>(ws),
                  reinterpret_cast<LdsItem*>(&S.host_image[S.lay.lds_items_off]),
                  reinterpret_cast<LdsStep*>(&S.host_image[S.lay.lds_steps_off]), 0);
  JF_HIP(hipMemcpyAsync(ws, S.host_image.data(), S.host_image.size(), hipMemcpyHostToDevice, stream));
  JF_HIP(hipStreamSynchronize(stream));
  S.uploaded_to = ws;
  const auto a = reinterpret_cast<uintptr_t>(ws);
  forget_uploads(a, a + region);
  g_last_upload[ws] = Upload{p, region};
  return JF_OK;
}

jf_status check_ws(jf_plan* p, void* ws, size_t ws_bytes) {
  DevState& S = state_of(p);
  if (!S.validated) {
    std::string why;
    if (!validate_program(p->prog, why)) {
      set_error("plan failed validation: " + why);
      return JF_E_ARG;
    }
    S.validated = true;
  }
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255)) {
    set_error("workspace must be a 256-byte aligned device pointer");
    return JF_E_ARG;
  }
  if (ws_bytes < S.lay.total) {
    set_error("workspace of " + std::to_string(ws_bytes) + " bytes, plan needs " + std::to_string(S.lay.total));
    return JF_E_OOM;
  }
  return JF_OK;
}

// The plan's pinned landing area: 4 doubles per component (every read-back of sums fits in it).
jf_status pinned_sums(jf_plan* p, double** out) {
  DevState& S = state_of(p);
  if (!S.pinned_sums)
    JF_HIP(hipHostMalloc(reinterpret_cast<void**>(&S.pinned_sums),
                         std::max<size_t>(p->prog.comps.size(), 1) * 4 * sizeof(double), hipHostMallocDefault));
  *out = S.pinned_sums;
  return JF_OK;
}

// Coherent (fine-grained) pinned memory: the assembly kernel's four stores reach the host without
// any cache flush, and the host reads them after the stream synchronisation.
jf_status pinned_res_of(jf_plan* p) {
  DevState& S = state_of(p);
  if (!S.pinned_res) {
    double* h = nullptr;
    JF_HIP(hipHostMalloc(reinterpret_cast<void**>(&h), 4 * sizeof(double), hipHostMallocCoherent));
    void* d = nullptr;
    const hipError_t e = hipHostGetDevicePointer(&d, h, 0);
    if (e != hipSuccess || !d) {
      (void)hipHostFree(h);
      set_error(std::string("hipHostGetDevicePointer: ") + hipGetErrorString(e));
      return JF_E_HIP;
    }
    S.pinned_res = h;
    S.pinned_res_dev = static_cast<double*>(d);
  }
  return JF_OK;
}

// Wait for the run and read F_J back (with terms, also the per-tuple outputs).  With pinned, the
// assembly kernel has written the result into the plan's pinned landing area (pinned_res_of before
// the enqueue), so only the terms need a copy; without (the no-allocation entry point: no host
// allocation by the library), the result is copied into pageable host memory.
jf_status read_results(jf_plan* p, unsigned char* ws, hipStream_t stream, jf_result* out, double* terms,
                       bool pinned = true) {
  const Program& P = p->prog;
  DevState& S = state_of(p);
  double res[4];
  const bool on_host = pinned && S.pinned_res;
  if (!on_host) JF_HIP(hipMemcpyAsync(res, ws + S.lay.res_off, sizeof(res), hipMemcpyDeviceToHost, stream));
  std::vector<std::vector<cd>> co;
  if (terms) {
    for (auto& cp : P.comps) {
      std::vector<cd> v(size_t(cp.out_len));
      JF_HIP(hipMemcpyAsync(v.data(), ws + S.lay.out_off + size_t(cp.out_off) * 16, size_t(cp.out_len) * 16,
                            hipMemcpyDeviceToHost, stream));
      co.push_back(std::move(v));
    }
  }
  JF_HIP(hipStreamSynchronize(stream));
  if (on_host) std::memcpy(res, S.pinned_res, sizeof(res));
  jf_result r;
  static_result(P, &r);
  r.fj = res[0];
  r.one_minus_fj = res[1];
  r.imag_residual = res[2];
  *out = r;
  if (terms) gather_terms(P, co, terms);
  return JF_OK;
}

// One run of a plan.  With JF_FLAG_GRAPH the step program is captured into a hipGraph on the first
// run for a (workspace, stream, kernel choice) and replayed after that (the per-step cost here is
// on the GPU side, so replay saves little; see the flag).  The null stream cannot be captured: then
// the plan's own stream runs the graph, ordered after the work already on the null stream.
jf_status run_one(jf_plan* p, void* ws, size_t ws_bytes, hipStream_t stream, jf_result* out, double* terms) {
  jf_status st = check_ws(p, ws, ws_bytes);
  if (st != JF_OK) return st;
  st = upload(p, ws, stream);
  if (st != JF_OK) return st;
  st = pinned_res_of(p);  // before any enqueue or capture: the assembly writes the result there
  if (st != JF_OK) return st;
  DevState& S = state_of(p);
  if (!S.ev0) {
    JF_HIP(hipEventCreate(&S.ev0));
    JF_HIP(hipEventCreate(&S.ev1));
    JF_HIP(hipEventCreateWithFlags(&S.ev_order, hipEventDisableTiming));
  }
  unsigned char* w = static_cast<unsigned char*>(ws);
  const bool graph = (p->prog.opt.flags & JF_FLAG_GRAPH) != 0;
  hipStream_t s = stream;
  if (graph && stream == nullptr) {
    if (!S.own_stream) JF_HIP(hipStreamCreateWithFlags(&S.own_stream, hipStreamNonBlocking));
    JF_HIP(hipEventRecord(S.ev_order, nullptr));
    JF_HIP(hipStreamWaitEvent(S.own_stream, S.ev_order, 0));
    s = S.own_stream;
  }
  hipStream_t side = nullptr;
  if (!S.lay.lds_comps.empty() && S.lay.lds_comps.size() < p->prog.comps.size()) {
    st = side_of(p, &side);
    if (st != JF_OK) return st;
  }
  if (graph && (!S.run_graph || S.run_graph_ws != ws || S.run_graph_stream != s || S.run_graph_gen != S.variant_gen)) {
    if (S.run_graph) {
      hipGraphExecDestroy(S.run_graph);
      S.run_graph = nullptr;
    }
    hipGraph_t g = nullptr;
    JF_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    st = enqueue_program(p, w, s, nullptr, false, nullptr, nullptr, side);
    const hipError_t ce = hipStreamEndCapture(s, &g);
    if (st != JF_OK) {
      if (ce == hipSuccess && g) hipGraphDestroy(g);
      return st;
    }
    if (ce != hipSuccess) {
      set_error(std::string("hipStreamEndCapture: ") + hipGetErrorString(ce));
      return JF_E_HIP;
    }
    const hipError_t ie = hipGraphInstantiate(&S.run_graph, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (ie != hipSuccess) {
      S.run_graph = nullptr;
      set_error(std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
      return JF_E_HIP;
    }
    S.run_graph_ws = ws;
    S.run_graph_stream = s;
    S.run_graph_gen = S.variant_gen;
  }
  JF_HIP(hipEventRecord(S.ev0, s));
  if (graph) {
    JF_HIP(hipGraphLaunch(S.run_graph, s));
  } else {
    st = enqueue_program(p, w, s, nullptr, false, nullptr, nullptr, side);
    if (st != JF_OK) return st;
  }
  JF_HIP(hipEventRecord(S.ev1, s));
  jf_result r;
  st = read_results(p, w, s, &r, terms);
  if (st != JF_OK) return st;
  float ms = 0;
  JF_HIP(hipEventElapsedTime(&ms, S.ev0, S.ev1));
  r.seconds = ms * 1e-3;
  *out = r;
  return JF_OK;
}

}  // namespace

size_t plan_workspace_bytes(jf_plan* p) { return state_of(p).lay.total; }

}  // namespace jf

using namespace jf;

extern "C" jf_status jf_fidelity_alg1(jf_plan* p, void* ws, size_t ws_bytes, void* stream, jf_result* out,
                                      double* terms) {
  if (!p || !out || p->prog.opt.alg != 1) {
    set_error("jf_fidelity_alg1: NULL argument or not an Algorithm I plan");
    return JF_E_ARG;
  }
  return run_one(p, ws, ws_bytes, static_cast<hipStream_t>(stream), out, terms);
}

// ------------------------------------------------------------- no-allocation entry point ---
// Device scratch of jf_fidelity_noalloc: one copy per GPU, held until the process ends.  In host
// code the name `scratch` is a host-side stand-in, never a device address: the device address
// comes from hipGetSymbolAddress, taken once per device with that device current.
static __device__ __align__(256) unsigned char scratch[JF_NOALLOC_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch (looked up on its first use on that device).
jf_status scratch_of_current_device(void** out) {
  int dev = 0;
  JF_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("jf_fidelity_noalloc: device index " + std::to_string(dev) + " beyond the supported " +
              std::to_string(kMaxDevices));
    return JF_E_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    JF_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) {
      set_error("jf_fidelity_noalloc: hipGetSymbolAddress returned no address for the scratch");
      return JF_E_HIP;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return JF_OK;
}
}  // namespace

extern "C" jf_status jf_fidelity_noalloc(jf_plan* p, void* stream_v, jf_result* out, double* terms) {
  if (!p || !out || (p->prog.opt.alg != 1 && p->prog.opt.alg != 2)) {
    set_error("jf_fidelity_noalloc: NULL argument or no algorithm in the plan");
    return JF_E_ARG;
  }
  if (terms && p->prog.opt.alg != 1) {
    set_error("jf_fidelity_noalloc: per-term traces exist for Algorithm I plans only");
    return JF_E_ARG;
  }
  const size_t need = state_of(p).lay.total;
  if (need > JF_NOALLOC_BYTES) {
    set_error("jf_fidelity_noalloc: the plan needs a workspace of " + std::to_string(need) +
              " bytes; the no-allocation scratch holds " + std::to_string((size_t)JF_NOALLOC_BYTES));
    return JF_E_OOM;
  }
  void* ws = nullptr;
  jf_status st = scratch_of_current_device(&ws);
  if (st != JF_OK) return st;
  hipStream_t stream = static_cast<hipStream_t>(stream_v);
  st = check_ws(p, ws, JF_NOALLOC_BYTES);
  if (st != JF_OK) return st;
  const auto t0 = std::chrono::steady_clock::now();
  st = upload(p, ws, stream);  // a copy of the plan's tables (every plan shares the scratch)
  if (st != JF_OK) return st;
  st = enqueue_program(p, static_cast<unsigned char*>(ws), stream);  // eager: no graph, no events
  if (st != JF_OK) return st;
  jf_result r;
  st = read_results(p, static_cast<unsigned char*>(ws), stream, &r, terms, false);
  if (st != JF_OK) return st;
  r.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  *out = r;
  return JF_OK;
}

extern "C" jf_status jf_stream_copy(const void* src, void* dst, size_t bytes, int bytes_per_lane, void* stream_v,
                                    double* ms) {
  if (ms && bytes == 0 && (bytes_per_lane == 8 || bytes_per_lane == 16)) {  // nothing to copy, no launch
    *ms = 0.0;
    return JF_OK;
  }
  if (!src || !dst || !ms || (bytes_per_lane != 8 && bytes_per_lane != 16) || bytes % size_t(bytes_per_lane) ||
      (reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16) {
    set_error("jf_stream_copy: bad argument (16-byte aligned buffers, bytes a multiple of 8 or 16 bytes per lane)");
    return JF_E_ARG;
  }
  hipStream_t stream = static_cast<hipStream_t>(stream_v);
  EventPair ev;
  JF_HIP(hipEventCreate(&ev.a));
  JF_HIP(hipEventCreate(&ev.b));
  JF_HIP(launch_stream_copy(src, dst, bytes, bytes_per_lane, stream, ev.a, ev.b));
  JF_HIP(hipEventSynchronize(ev.b));
  float t = 0;
  JF_HIP(hipEventElapsedTime(&t, ev.a, ev.b));
  *ms = t;
  return JF_OK;
}

extern "C" jf_status jf_profile_run(jf_plan* p, void* ws, size_t ws_bytes, void* stream_v, jf_profile* out) {
  if (!p || !out) {
    set_error("jf_profile_run: bad argument");
    return JF_E_ARG;
  }
  hipStream_t stream = static_cast<hipStream_t>(stream_v);
  jf_status st = check_ws(p, ws, ws_bytes);
  if (st != JF_OK) return st;
  st = upload(p, ws, stream);
  if (st != JF_OK) return st;
  Prof prof;
  EventPair ev;
  JF_HIP(hipEventCreate(&ev.a));
  JF_HIP(hipEventCreate(&ev.b));
  hipEvent_t e0 = ev.a, e1 = ev.b;
  JF_HIP(hipEventRecord(e0, stream));
  st = enqueue_program(p, static_cast<unsigned char*>(ws), stream, &prof);
  if (st != JF_OK) return st;
  JF_HIP(hipEventRecord(e1, stream));
  JF_HIP(hipStreamSynchronize(stream));
  jf_profile r = {};
  r.launches = (long long)prof.ev.size() / 2;
  for (size_t i = 0; i + 1 < prof.ev.size(); i += 2) {
    float ms = 0;
    JF_HIP(hipEventElapsedTime(&ms, prof.ev[i], prof.ev[i + 1]));
    r.kernel_ms += ms;
    r.max_launch_ms = std::max(r.max_launch_ms, double(ms));
  }
  float tot = 0;
  JF_HIP(hipEventElapsedTime(&tot, e0, e1));
  r.total_ms = tot;
  r.bytes = prof.bytes;
  r.flops = prof.flops;
  *out = r;
  return JF_OK;
}

extern "C" jf_status jf_profile_steps(jf_plan* p, void* ws, size_t ws_bytes, void* stream_v, jf_step_profile* out,
                                      int cap, int* n_launches) {
  if (!p || !n_launches || cap < 0 || (cap > 0 && !out)) {
    set_error("jf_profile_steps: bad argument");
    return JF_E_ARG;
  }
  hipStream_t stream = static_cast<hipStream_t>(stream_v);
  jf_status st = check_ws(p, ws, ws_bytes);
  if (st != JF_OK) return st;
  st = upload(p, ws, stream);
  if (st != JF_OK) return st;
  Prof prof;
  st = enqueue_program(p, static_cast<unsigned char*>(ws), stream, &prof);
  if (st != JF_OK) return st;
  JF_HIP(hipStreamSynchronize(stream));
  const int n = int(prof.rec.size());
  for (int i = 0; i < n; ++i) {
    float ms = 0;
    JF_HIP(hipEventElapsedTime(&ms, prof.ev[2 * i], prof.ev[2 * i + 1]));
    prof.rec[i].ms = ms;
    if (i < cap) out[i] = prof.rec[i];
  }
  *n_launches = n;
  return JF_OK;
}

extern "C" jf_status jf_autotune(jf_plan* p, void* ws, size_t ws_bytes, void* stream_v, int reps) {
  if (!p) {
    set_error("jf_autotune: bad argument");
    return JF_E_ARG;
  }
  hipStream_t stream = static_cast<hipStream_t>(stream_v);
  jf_status st = check_ws(p, ws, ws_bytes);
  if (st != JF_OK) return st;
  st = upload(p, ws, stream);
  if (st != JF_OK) return st;
  Tune tune;
  tune.reps = reps > 0 ? reps : 3;
  tune.done.resize(p->prog.comps.size());
  for (size_t c = 0; c < p->prog.comps.size(); ++c) tune.done[c].assign(p->prog.comps[c].steps.size(), 0);
  st = enqueue_program(p, static_cast<unsigned char*>(ws), stream, nullptr, false, &tune);
  if (st != JF_OK) return st;
  JF_HIP(hipStreamSynchronize(stream));
  state_of(p).variant_gen = g_variant_gen.fetch_add(1);
  return JF_OK;
}

extern "C" jf_status jf_set_kernel_variant(jf_plan* p, int variant) {
  if (!p || variant < KV_AUTO || variant >= KV_COUNT) {
    set_error("jf_set_kernel_variant: bad argument");
    return JF_E_ARG;
  }
  DevState& S = state_of(p);
  for (size_t c = 0; c < p->prog.comps.size(); ++c)
    for (size_t s = 0; s < p->prog.comps[c].steps.size(); ++s) {
      StepDesc* hd = reinterpret_cast<StepDesc*>(&S.host_image[S.lay.step_desc[c][s]]);
      hd->variant = variant_applies(*hd, variant) ? variant : KV_AUTO;
    }
  // a forced kernel runs every step on its own, except the Gauss-form kernels, whose products the
  // chains repeat; AUTO brings the chains back
  const bool keep = variant == KV_AUTO || variant == KV_GAUSS_256 || variant == KV_GAUSS_512;
  for (auto& v : S.chain_off) std::fill(v.begin(), v.end(), char(!keep));
  S.variant_gen = g_variant_gen.fetch_add(1);
  return JF_OK;
}

// Definition 1 decided with early stopping (Algorithm I, Section IV-A: the terms are
// nonnegative, so a running sum above 1 - eps proves equivalence).  Every component but the one
// with the most depth-first leaves runs in full; that one runs leaf by leaf.  After each leaf:
//   lower = a * prod_{other c} S_c * S_last(partial)           (the terms done so far)
//   upper = lower + (mass of the leaves not run) * prod_{sites outside} sum_j ||K_j||^2
// because |t_k|^2 = |tr(U^dagger E_k)|^2 / d^2 <= prod_i ||K_{k_i}||^2 for every Kraus tuple.
extern "C" jf_status jf_decide_equivalence(jf_plan* p, double eps, void* ws, size_t ws_bytes, void* stream_v,
                                           jf_decision* out) {
  if (!p || !out || !(eps > 0.0) || !(eps <= 1.0)) {
    set_error("jf_decide_equivalence: NULL argument or eps outside (0, 1]");
    return JF_E_ARG;
  }
  hipStream_t stream = static_cast<hipStream_t>(stream_v);
  jf_status st = check_ws(p, ws, ws_bytes);
  if (st != JF_OK) return st;
  st = upload(p, ws, stream);
  if (st != JF_OK) return st;
  const Program& P = p->prog;
  const DevLayout& L = state_of(p).lay;
  unsigned char* w = static_cast<unsigned char*>(ws);
  // arithmetic margin of the form (the parity bar of its results)
  const double margin = P.opt.dtype == JF_C128 ? 1e-12 : 1e-6;
  const double thr = 1.0 - eps;
  jf_decision d = {};
  d.margin = margin;
  d.leaves_total = P.work_items;
  EventPair ev;
  JF_HIP(hipEventCreate(&ev.a));
  JF_HIP(hipEventCreate(&ev.b));
  hipEvent_t e0 = ev.a, e1 = ev.b;
  JF_HIP(hipEventRecord(e0, stream));
  auto decide = [&](double lo, double hi) {
    if (lo - margin > thr) return 1;
    if (hi + margin <= thr) return 0;
    return -1;
  };
  int last = -1;
  long long most = 1;
  bool wires = false;  // a leaf of a component with sliced wires holds partial sums, not terms
  for (const ComponentProgram& cp : P.comps) wires = wires || cp.accumulate;
  if (P.opt.alg == 1 && !wires)
    for (size_t c = 0; c < P.comps.size(); ++c)
      if (!P.comps[c].lds_resident && P.comps[c].leaves > most) {
        most = P.comps[c].leaves;
        last = int(c);
      }
  if (last < 0) {  // one pass computes every term
    st = pinned_res_of(p);
    if (st != JF_OK) return st;
    st = enqueue_program(p, w, stream);
    if (st != JF_OK) return st;
    jf_result r;
    st = read_results(p, w, stream, &r, nullptr);
    if (st != JF_OK) return st;
    d.fj_lower = d.fj_upper = r.fj;
    d.leaves_run = d.leaves_total;
    d.decision = decide(r.fj, r.fj);
  } else {
    // everything except the last component, in full
    if (!L.lds_comps.empty())
      JF_HIP(launch_persistent(reinterpret_cast<const LdsItem*>(w + L.lds_items_off), int(L.lds_comps.size()),
                               reinterpret_cast<const LdsStep*>(w + L.lds_steps_off), stream));
    for (size_t c = 0; c < P.comps.size(); ++c) {
      const ComponentProgram& cp = P.comps[c];
      if (cp.lds_resident || int(c) == last) continue;
      st = enqueue_component(p, w, w + L.buf_off, stream, c, nullptr, nullptr);
      if (st != JF_OK) return st;
      JF_HIP(launch_sumsq(w + L.out_off + size_t(cp.out_off) * 16, cp.out_len,
                          reinterpret_cast<double*>(w + L.sums_off) + 4 * c,
                          reinterpret_cast<double*>(w + L.sumsq_off), stream));
    }
    double* pin = nullptr;
    st = pinned_sums(p, &pin);
    if (st != JF_OK) return st;
    std::vector<double> sums(4 * P.comps.size());
    JF_HIP(hipMemcpyAsync(pin, w + L.sums_off, sums.size() * sizeof(double), hipMemcpyDeviceToHost, stream));
    JF_HIP(hipStreamSynchronize(stream));
    std::memcpy(sums.data(), pin, sums.size() * sizeof(double));
    const double sc = std::exp2(P.log2_scale);
    double prod_other = sc * sc * std::norm(P.scalar);
    for (size_t c = 0; c < P.comps.size(); ++c)
      if (int(c) != last) prod_other *= sums[4 * c] + sums[4 * c + 1];
    // masses: sites of the last component, and the rest
    const ComponentProgram& cp = P.comps[last];
    double mass_outside = 1.0, mass_unsliced = 1.0;
    std::vector<char> sliced(P.site_norm2.size(), 0);
    for (const Level& lev : cp.levels)
      if (lev.site >= 0) sliced[lev.site] = 1;
    for (size_t i = 0; i < P.site_norm2.size(); ++i) {
      double t = 0;
      for (double x : P.site_norm2[i]) t += x;
      if (P.site_comp[i] != last) mass_outside *= t;
      else if (!sliced[i]) mass_unsliced *= t;
    }
    double mass_total = mass_unsliced;
    for (const Level& lev : cp.levels)
      if (lev.site >= 0) {
        double t = 0;
        for (double x : P.site_norm2[lev.site]) t += x;
        mass_total *= t;
      }
    // the last component, leaf by leaf (depth first, prefixes kept in the level buffers)
    unsigned char* out_last = w + L.out_off + size_t(cp.out_off) * 16;
    double* sums_last = reinterpret_cast<double*>(w + L.sums_off) + 4 * last;
    JF_HIP(launch_zero(out_last, cp.out_len, stream));
    const int nl = int(cp.levels.size());
    std::vector<int> v(nl, 0);
    std::vector<const void*> end(nl, nullptr);
    std::vector<long long> base(nl, 0);
    int from = 0;
    double mass_done = 0;
    d.decision = -1;
    while (true) {
      for (int lv = from; lv < nl; ++lv) {
        base[lv] = (lv ? base[lv - 1] : 0) + v[lv] * cp.levels[lv].out_stride;
        st = enqueue_level(p, w, w + L.buf_off, stream, size_t(last), lv, v, lv ? end[lv - 1] : nullptr, base[lv], &end[lv],
                           nullptr, nullptr);
        if (st != JF_OK) return st;
      }
      JF_HIP(launch_sumsq(out_last, cp.out_len, sums_last, reinterpret_cast<double*>(w + L.sumsq_off), stream));
      double part[2];
      JF_HIP(hipMemcpyAsync(pin, sums_last, sizeof(part), hipMemcpyDeviceToHost, stream));
      JF_HIP(hipStreamSynchronize(stream));
      std::memcpy(part, pin, sizeof(part));
      double m = mass_unsliced;
      for (int lv = 0; lv < nl; ++lv)
        if (cp.levels[lv].site >= 0) {
          const auto& nrm = P.site_norm2[cp.levels[lv].site];
          m *= v[lv] < int(nrm.size()) ? nrm[v[lv]] : 0.0;  // padding variants are zero operators
        }
      mass_done += m;
      ++d.leaves_run;
      d.fj_lower = prod_other * (part[0] + part[1]);
      d.fj_upper = d.fj_lower + std::max(0.0, mass_total - mass_done) * mass_outside;
      d.decision = decide(d.fj_lower, d.fj_upper);
      if (d.decision >= 0) break;
      // next leaf in depth-first order
      int lv = nl - 1;
      while (lv >= 0 && v[lv] + 1 >= cp.levels[lv].nvar) --lv;
      if (lv < 0) break;
      ++v[lv];
      for (int k = lv + 1; k < nl; ++k) v[k] = 0;
      from = lv;
    }
    d.leaves_run += P.work_items - cp.leaves;  // the other components ran in full
    if (d.leaves_run == P.work_items) d.fj_upper = d.fj_lower;  // every term is in
  }
  JF_HIP(hipEventRecord(e1, stream));
  JF_HIP(hipEventSynchronize(e1));
  float ms = 0;
  JF_HIP(hipEventElapsedTime(&ms, e0, e1));
  d.seconds = ms * 1e-3;
  *out = d;
  return JF_OK;
}

extern "C" jf_status jf_fidelity_alg2(jf_plan* p, void* ws, size_t ws_bytes, void* stream, jf_result* out) {
  if (!p || !out || p->prog.opt.alg != 2) {
    set_error("jf_fidelity_alg2: NULL argument or not an Algorithm II plan");
    return JF_E_ARG;
  }
  return run_one(p, ws, ws_bytes, static_cast<hipStream_t>(stream), out, nullptr);
}

// A batch shares one workspace: each plan keeps its tables, outputs and sums in a region of its
// own, and since the plans run one after another on one stream, their level buffers share one
// region sized for the largest; the persistent kernel's item and step tables follow.
namespace jf {
namespace {
struct BatchLayout {
  std::vector<size_t> base;  // each plan's region
  size_t bufs = 0, items = 0, steps = 0, total = 0;
};
BatchLayout batch_layout(jf_plan* const* plans, int n) {
  BatchLayout b;
  size_t off = 0, maxbuf = 0, items = 0, steps = 0;
  for (int i = 0; i < n; ++i) {
    const DevLayout& L = state_of(plans[i]).lay;
    b.base.push_back(off);
    off += align256(L.buf_off);
    maxbuf = std::max(maxbuf, L.total - L.buf_off);
    items += L.lds_comps.size();
    steps += L.lds_steps;
  }
  b.bufs = off;
  off += align256(maxbuf);
  b.items = off;
  off += align256(items * sizeof(LdsItem));
  b.steps = off;
  off += align256(steps * sizeof(LdsStep));
  b.total = off;
  return b;
}
}  // namespace
}  // namespace jf

extern "C" jf_status jf_batch_workspace(jf_plan* const* plans, int n, size_t* bytes) {
  if (!plans || n < 0 || !bytes) {
    set_error("jf_batch_workspace: bad argument");
    return JF_E_ARG;
  }
  for (int i = 0; i < n; ++i)
    if (!plans[i]) {
      set_error("jf_batch_workspace: NULL plan");
      return JF_E_ARG;
    }
  *bytes = batch_layout(plans, n).total;
  return JF_OK;
}

extern "C" jf_status jf_workspace_release(const void* dev_ws, size_t ws_bytes) {
  if (!dev_ws) {
    set_error("jf_workspace_release: NULL workspace");
    return JF_E_ARG;
  }
  // forget every upload whose region meets [dev_ws, dev_ws + ws_bytes): the plans whose tables
  // were there upload them again on their next call (batch members sit at offsets inside the range)
  const auto lo = reinterpret_cast<uintptr_t>(dev_ws);
  const auto hi = lo + (ws_bytes ? ws_bytes : 1);
  std::lock_guard<std::mutex> g(g_upload_mu);
  forget_uploads(lo, hi);
  return JF_OK;
}

extern "C" jf_status jf_fidelity_batch(jf_plan* const* plans, int n, void* ws, size_t ws_bytes, void* stream_v,
                                       jf_result* out) {
  size_t need = 0;
  jf_status st = jf_batch_workspace(plans, n, &need);
  if (st != JF_OK) return st;
  if (n == 0) return JF_OK;
  if (!out || !ws || (reinterpret_cast<uintptr_t>(ws) & 255)) {
    set_error("jf_fidelity_batch: bad output or workspace");
    return JF_E_ARG;
  }
  if (ws_bytes < need) {
    set_error("jf_fidelity_batch: workspace too small");
    return JF_E_OOM;
  }
  hipStream_t stream = static_cast<hipStream_t>(stream_v);
  const BatchLayout bl = batch_layout(plans, n);
  unsigned char* w = static_cast<unsigned char*>(ws);
  unsigned char* bufs = w + bl.bufs;
  {
    // the shared buffers and the persistent tables are written by this call: no plan's tables
    // uploaded there before survive it
    std::lock_guard<std::mutex> g(g_upload_mu);
    const auto a = reinterpret_cast<uintptr_t>(bufs);
    forget_uploads(a, a + (bl.total - bl.bufs));
  }
  std::vector<unsigned char*> base(n);
  for (int i = 0; i < n; ++i) {
    base[i] = w + bl.base[i];
    st = check_ws(plans[i], base[i], state_of(plans[i]).lay.total);
    if (st != JF_OK) return st;
    st = upload(plans[i], base[i], stream, state_of(plans[i]).lay.buf_off);
    if (st != JF_OK) return st;
    st = pinned_res_of(plans[i]);  // before the capture: each member's assembly writes its result there
    if (st != JF_OK) return st;
  }
  // every small component of every plan in one persistent launch
  std::vector<LdsItem> items;
  std::vector<LdsStep> lsteps;
  for (int i = 0; i < n; ++i) {
    const DevLayout& L = state_of(plans[i]).lay;
    std::vector<LdsItem> it(L.lds_comps.size());
    std::vector<LdsStep> ss(L.lds_steps);
    fill_lds_tables(plans[i]->prog, L, base[i], it.data(), ss.data(), int(lsteps.size()));
    items.insert(items.end(), it.begin(), it.end());
    lsteps.insert(lsteps.end(), ss.begin(), ss.end());
  }
  unsigned char* items_dev = w + bl.items;
  unsigned char* steps_dev = w + bl.steps;
  if (!items.empty()) {
    JF_HIP(hipMemcpyAsync(items_dev, items.data(), items.size() * sizeof(LdsItem), hipMemcpyHostToDevice, stream));
    JF_HIP(hipMemcpyAsync(steps_dev, lsteps.data(), lsteps.size() * sizeof(LdsStep), hipMemcpyHostToDevice, stream));
    JF_HIP(hipStreamSynchronize(stream));
  }
  EventPair ev;
  JF_HIP(hipEventCreate(&ev.a));
  JF_HIP(hipEventCreate(&ev.b));
  hipEvent_t e0 = ev.a, e1 = ev.b;
  DevState& S0 = state_of(plans[0]);
  const bool use_graph = n > 0 && stream != nullptr;
  // the small members' persistent launch beside the larger members' programs
  bool large = false;
  for (int i = 0; i < n; ++i) large = large || state_of(plans[i]).lay.lds_comps.size() < plans[i]->prog.comps.size();
  hipStream_t side = nullptr;
  if (!items.empty() && large) {
    st = side_of(plans[0], &side);
    if (st != JF_OK) return st;
  }
  std::vector<unsigned long long> key(n);
  for (int i = 0; i < n; ++i) key[i] = plans[i]->uid;
  std::vector<unsigned> gens(n);
  for (int i = 0; i < n; ++i) gens[i] = state_of(plans[i]).variant_gen;
  if (use_graph && (S0.graph == nullptr || S0.graph_ws != ws || S0.graph_stream != stream || S0.graph_plans != key ||
                    S0.graph_gens != gens)) {
    if (S0.graph) {
      hipGraphExecDestroy(S0.graph);
      S0.graph = nullptr;
    }
    hipGraph_t g = nullptr;
    JF_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
    if (!items.empty())
      st = launch_persistent_beside(reinterpret_cast<const LdsItem*>(items_dev), int(items.size()),
                                    reinterpret_cast<const LdsStep*>(steps_dev), stream, side, S0.ev_fork, S0.ev_join);
    // with the persistent launch beside them, every member's assembly (which reads its small
    // components' sums) waits for it
    for (int i = 0; i < n && st == JF_OK; ++i)
      st = enqueue_program(plans[i], base[i], stream, nullptr, true, nullptr, bufs, nullptr, side == nullptr);
    if (st == JF_OK && side) {
      if (hipStreamWaitEvent(stream, S0.ev_join, 0) != hipSuccess) st = JF_E_HIP;
      for (int i = 0; i < n && st == JF_OK; ++i) st = enqueue_assemble(plans[i], base[i], stream);
    }
    hipError_t ce = hipStreamEndCapture(stream, &g);
    if (st != JF_OK) {
      if (ce == hipSuccess && g) hipGraphDestroy(g);
      return st;
    }
    if (ce != hipSuccess) {
      set_error(std::string("hipStreamEndCapture: ") + hipGetErrorString(ce));
      return JF_E_HIP;
    }
    JF_HIP(hipGraphInstantiate(&S0.graph, g, nullptr, nullptr, 0));
    JF_HIP(hipGraphDestroy(g));
    S0.graph_ws = ws;
    S0.graph_stream = stream;
    S0.graph_plans = key;
    S0.graph_gens = gens;
  }
  JF_HIP(hipEventRecord(e0, stream));
  if (use_graph) {
    JF_HIP(hipGraphLaunch(S0.graph, stream));
  } else {
    if (!items.empty()) {
      st = launch_persistent_beside(reinterpret_cast<const LdsItem*>(items_dev), int(items.size()),
                                    reinterpret_cast<const LdsStep*>(steps_dev), stream, side, S0.ev_fork, S0.ev_join);
      if (st != JF_OK) return st;
    }
    for (int i = 0; i < n; ++i) {
      st = enqueue_program(plans[i], base[i], stream, nullptr, true, nullptr, bufs, nullptr, side == nullptr);
      if (st != JF_OK) return st;
    }
    if (side) {
      JF_HIP(hipStreamWaitEvent(stream, S0.ev_join, 0));
      for (int i = 0; i < n; ++i) {
        st = enqueue_assemble(plans[i], base[i], stream);
        if (st != JF_OK) return st;
      }
    }
  }
  JF_HIP(hipEventRecord(e1, stream));
  for (int i = 0; i < n; ++i) {
    st = read_results(plans[i], base[i], stream, &out[i], nullptr);
    if (st != JF_OK) return st;
  }
  float ms = 0;
  JF_HIP(hipEventElapsedTime(&ms, e0, e1));
  for (int i = 0; i < n; ++i) out[i].seconds = ms * 1e-3;
  return JF_OK;
}

extern "C" void jf_free_plan(jf_plan* p) {
  if (!p) return;
  if (p->dev) {
    auto* s = static_cast<DevState*>(p->dev);
    if (s->graph) hipGraphExecDestroy(s->graph);
    if (s->run_graph) hipGraphExecDestroy(s->run_graph);
    if (s->own_stream) {
      hipStreamSynchronize(s->own_stream);
      hipStreamDestroy(s->own_stream);
    }
    if (s->side_stream) {
      hipStreamSynchronize(s->side_stream);
      hipStreamDestroy(s->side_stream);
    }
    for (hipEvent_t e : {s->ev0, s->ev1, s->ev_order, s->ev_fork, s->ev_join})
      if (e) hipEventDestroy(e);
    if (s->pinned_sums) hipHostFree(s->pinned_sums);
    if (s->pinned_res) hipHostFree(s->pinned_res);
    {
      std::lock_guard<std::mutex> g(g_upload_mu);
      for (auto it = g_last_upload.begin(); it != g_last_upload.end();)
        if (it->second.plan == p) it = g_last_upload.erase(it);
        else ++it;
    }
    delete s;
  }
  delete p;
}
