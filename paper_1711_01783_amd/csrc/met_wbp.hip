// Weighted BP on the GPU: forward with message checkpoints and the reverse
// sweep with hand-written adjoint kernels.
//
// Weighted BP is the decoder of met_decode.hip (Methods, Steps 2-5, eq.
// (1)-(5)) run for a fixed number L of iterations with one change: the
// check-to-variable message of an edge of type t produced in iteration l is
// scaled by w[t][l] after the syndrome sign, before the variable update.
//
// Forward state after iteration l ("posterior form"): c2v^l per message edge
// and P^l per variable node of degree >= 2.  Iteration l computes
//   x_e   = clamp(P^{l-1}_v(e) - c2v^{l-1}_e, +-30)          (x = L on iteration 1)
//   R_e   = s_j prod_{e' != e} sgn(x_e') phi( sum_{e' != e} phi(|x_e'|) )
//   c2v^l = w[t(e)][l] R_e,    P^l_v = L_v + sum_{e in E(v)} c2v^l_e.
// Leaf (degree-1) VNs always send their LLR; their posterior L + c2v^L counts
// only after the last iteration.  States at every k-th iteration are kept.
//
// Reverse sweep, with g_e = dLoss/dc2v^l_e = Pbar^l_v(e) + Cbar^l_e, where Cbar^l
// is the adjoint that reaches c2v^l through x^{l+1} = P^l - c2v^l:
//   dLoss/dw[t][l] += sum_{e of type t} g_e R_e
//   Rbar_e = g_e w[t(e)][l]
//   xbar_e' = sgn(x_e') sum_{e != e'} Rbar_e sgn(R_e) sinh(A_e') / sinh(A_e' + r_ee')
//       (A = phi(|x|), r_ee' = sum of A over the check's other inputs: the
//        derivative of the leave-one-out boxplus, since phi'(y) = -1/sinh(y) and
//        sinh(phi(y)) = 1/sinh(y)); evaluated without overflow or cancellation
//        as e^{-r} expm1(-2 A_e') / expm1(-2 (A_e' + r_ee')), where
//        A_e' + r_ee' is the leave-one-out sum of e.
//   vbar_e' = xbar_e' where the clamp is inactive, else 0
//   Cbar^{l-1}_e' = -vbar_e',   Pbar^{l-1}_v = sum_{e in E(v)} vbar_e.
// Each segment between checkpoints but the last (whose states the forward pass
// leaves in the segment slots) is recomputed forward before its reverse pass.
// All reductions run in a fixed order (deterministic gradients).
#include "met_gpu.h"

namespace met {
namespace {

constexpr int kMaxT = MET_MAX_EDGE_TYPES;

struct AdjParams {
  const int32_t *edge_msgvn;
  const int8_t *edge_type, *leaf_type;
  const int32_t *chk_msg_ptr, *chk_leaf_ptr;
  int64_t M, N2, E12, EL;
  const float *Pin;      // [G][N2][W] P^{l-1} (the LLRs when l == 1)
  const float *c2v_in;   // [G][E12][W] c2v^{l-1} (unused when l == 1)
  const float *Lphi;     // [G][EL][W]
  const uint64_t *synw;  // [G][M]
  const float *Pbar;     // [G][N2][W] adjoint of P^l
  float *Cbar;           // [G][E12][W] in: Cbar^l, out: Cbar^{l-1}
  const float *gleaf;    // [G][EL][W] adjoint of leaf posteriors (l == L), or NULL
  const float *weights;  // [T][wstride]
  float *partial;        // [blocks][kMaxT] per-block sums of dLoss/dw[.][l]
  int64_t partial_base;  // first partial row of this launch
  int32_t wstride, it, first;
};

// e^y - 1 for y <= 0, the sinh-ratio factors of the check adjoint.  Near zero
// the Taylor series through y^7 (the first dropped term is below 2e-8 of the
// result for |y| < 0.35); further out the hardware exponential minus one, whose
// rounding the subtraction magnifies at most 3.4-fold there.  Both are formed
// and one is selected, so the wave does not diverge.
__device__ __forceinline__ float expm1_nonpos(float y) {
  float t = fmaf(y, 1.0f / 5040.0f, 1.0f / 720.0f);
  t = fmaf(y, t, 1.0f / 120.0f);
  t = fmaf(y, t, 1.0f / 24.0f);
  t = fmaf(y, t, 1.0f / 6.0f);
  t = fmaf(y, t, 0.5f);
  t = fmaf(y, t, 1.0f);
  const float series = y * t;
  const float direct = __expf(y) - 1.0f;
  return y > -0.35f ? series : direct;
}

// Adjoint of one check's update: compile-time shape (NM message + NL leaf
// inputs) when NM > 0, run-time degrees (up to MET_MAX_CHECK_DEGREE) otherwise.
constexpr int kMaxAdjDegree = 16;  // run-time-degree checks in weighted BP

template <int W, int NM, int NL>
__global__ __launch_bounds__(kBlock) void k_check_adj(const AdjParams p, const ClassArgs c) {
  constexpr bool GEN = NM == 0;
  constexpr int D = GEN ? kMaxAdjDegree : NM + NL;
  constexpr int UNR = GEN ? 1 : D;  // compiled shapes unroll fully
  const int g = blockIdx.y;
  const int lane = threadIdx.x & 63, wv = wave_id();
  const int w = lane % W, q = lane / W;
  const int64_t i = ((int64_t)blockIdx.x * kWavesPerBlock + wv) * (64 / W) + q;
  const bool valid = i < c.n_checks;
  const int64_t item = valid ? i : 0;
  const int64_t j = c.first_check + item;
  int64_t m0, l0;
  int nm, nl;
  if (GEN) {
    m0 = p.chk_msg_ptr[j];
    l0 = p.chk_leaf_ptr[j];
    nm = p.chk_msg_ptr[j + 1] - (int32_t)m0;
    nl = p.chk_leaf_ptr[j + 1] - (int32_t)l0;
  } else {
    m0 = c.first_msg + item * NM;
    l0 = c.first_leaf + item * NL;
    nm = NM;
    nl = NL;
  }
  const uint32_t s = (uint32_t)(p.synw[(int64_t)g * p.M + j] >> w) & 1u;
  float A[D], gsum[D];
  int8_t ty[D];
  uint32_t neg = 0, inrange = 0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    A[k] = 0.0f;  // absent input: no contribution to any sum
    gsum[k] = 0.0f;
    ty[k] = 0;
    if (k < nm) {
      const int64_t e = m0 + k;
      const int32_t vi = p.edge_msgvn[e];
      const float pv = p.Pin[((int64_t)g * p.N2 + vi) * W + w];
      const float cv = p.first ? 0.0f : ld_stream<W>(&p.c2v_in[((int64_t)g * p.E12 + e) * W + w]);
      const float v = pv - cv;
      inrange |= (uint32_t)(fabsf(v) < kLlrMax) << k;
      const float x = clamp_llr(v);
      A[k] = phi(fabsf(x));
      neg |= sign_bit(x) << k;
      gsum[k] = p.Pbar[((int64_t)g * p.N2 + vi) * W + w] +
                ld_stream<W>(&p.Cbar[((int64_t)g * p.E12 + e) * W + w]);
      ty[k] = (int8_t)edge_type_of<W>(p.edge_type, e);
    } else if (k < nm + nl) {
      const int64_t le = l0 + (k - nm);
      const float f = p.Lphi[((int64_t)g * p.EL + le) * W + w];
      A[k] = fabsf(f);
      neg |= sign_bit(f) << k;
      gsum[k] = p.gleaf ? p.gleaf[((int64_t)g * p.EL + le) * W + w] : 0.0f;
      ty[k] = (int8_t)edge_type_of<W>(p.leaf_type, le);
    }
    if (!valid) gsum[k] = 0.0f;
  }
  const uint32_t tot = (__popc(neg) & 1u) ^ s;
  float pre[D], suf[D];
  pre[0] = 0.0f;
#pragma unroll
  for (int k = 1; k < D; ++k) pre[k] = pre[k - 1] + A[k - 1];
  suf[D - 1] = 0.0f;
#pragma unroll
  for (int k = D - 2; k >= 0; --k) suf[k] = suf[k + 1] + A[k + 1];
  float acc[kMaxT];
#pragma unroll
  for (int t = 0; t < kMaxT; ++t) acc[t] = 0.0f;
  float Q[D];  // Rbar_e * sgn(R_e)
#pragma unroll
  for (int k = 0; k < D; ++k) {
    Q[k] = 0.0f;
    if (k < nm + nl) {
      const float R = phi(pre[k] + suf[k]);
      const bool rneg = (tot ^ (neg >> k)) & 1u;
      const float contrib = gsum[k] * (rneg ? -R : R);
#pragma unroll
      for (int t = 0; t < kMaxT; ++t) acc[t] += (ty[k] == t) ? contrib : 0.0f;
      const float wt = p.weights[(int64_t)ty[k] * p.wstride + (p.it - 1)];
      const float rbar = gsum[k] * wt;
      Q[k] = rneg ? -rbar : rbar;
    }
  }
  if (!p.first) {
    // sinh(A_k) / sinh(S_e) = e^{-r_ek} expm1(-2 A_k) / expm1(-2 S_e), with
    // S_e = A_k + r_ek the leave-one-out sum of e: the factor of e is shared
    // by all targets k and the factor of k by all sources e.
    float Qd[D];
#pragma unroll UNR
    for (int e = 0; e < D; ++e)
      Qd[e] = e < nm + nl ? Q[e] * __builtin_amdgcn_rcpf(expm1_nonpos(-2.0f * (pre[e] + suf[e]))) : 0.0f;
    // e^{-r_ek} for the leave-two-out sums r_ek (A over the inputs other than
    // e and k) as products of the inputs' e^{-A}: one exponential per input
    // instead of one per (source, target) pair
    float E[D];
#pragma unroll UNR
    for (int o = 0; o < D; ++o) E[o] = __expf(-A[o]);  // absent inputs: A = 0, E = 1
#pragma unroll UNR
    for (int k = 0; k < D; ++k) {
      if (k >= nm) continue;
      float pb[D], sb[D];
      pb[0] = 1.0f;
#pragma unroll UNR
      for (int o = 1; o < D; ++o) pb[o] = pb[o - 1] * (o - 1 == k ? 1.0f : E[o - 1]);
      sb[D - 1] = 1.0f;
#pragma unroll UNR
      for (int o = D - 2; o >= 0; --o) sb[o] = sb[o + 1] * (o + 1 == k ? 1.0f : E[o + 1]);
      float xs = 0.0f;
#pragma unroll UNR
      for (int e = 0; e < D; ++e)
        if (e != k && e < nm + nl) xs += Qd[e] * (pb[e] * sb[e]);
      float xb = expm1_nonpos(-2.0f * A[k]) * xs;
      if ((neg >> k) & 1u) xb = -xb;
      const float vbar = ((inrange >> k) & 1u) ? xb : 0.0f;
      if (valid) st_stream<W>(-vbar, &p.Cbar[((int64_t)g * p.E12 + m0 + k) * W + w]);
    }
  }
  // block sums of dLoss/dw, in a fixed order.  Wave sums of all types at
  // once: each of the first three exchange steps hands half of the types
  // still held to the partner lane and keeps the other half, so after them
  // lane l holds a partial of type (l >> 3) alone; three more steps finish
  // its sum (10 exchanges instead of 6 per type).
  static_assert(kMaxT == 8, "exchange pattern assumes 8 types over 64 lanes");
  __shared__ float red[kWavesPerBlock][kMaxT];
  {
    float v4[4], v2[2];
    const bool h32 = lane & 32, h16 = lane & 16, h8 = lane & 8;
#pragma unroll
    for (int j = 0; j < 4; ++j)
      v4[j] = (h32 ? acc[4 + j] : acc[j]) + __shfl_xor(h32 ? acc[j] : acc[4 + j], 32);
#pragma unroll
    for (int j = 0; j < 2; ++j)
      v2[j] = (h16 ? v4[2 + j] : v4[j]) + __shfl_xor(h16 ? v4[j] : v4[2 + j], 16);
    float v = (h8 ? v2[1] : v2[0]) + __shfl_xor(h8 ? v2[0] : v2[1], 8);
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 1);
    if ((lane & 7) == 0) red[threadIdx.x >> 6][lane >> 3] = v;
  }
  __syncthreads();
  if (threadIdx.x < kMaxT) {
    float v = 0.0f;
    for (int k = 0; k < kWavesPerBlock; ++k) v += red[k][threadIdx.x];
    p.partial[(p.partial_base + (int64_t)blockIdx.y * gridDim.x + blockIdx.x) * kMaxT + threadIdx.x] = v;
  }
}

// Pbar^{l-1}_v = sum over v's message edges of vbar = -Cbar^{l-1}.
struct VarAdjParams {
  const int32_t *vn_ptr, *vn_edges;
  int64_t N2, E12;
  const float *Cbar;
  float *Pbar;
};

template <int W>
__global__ __launch_bounds__(kBlock) void k_variable_adj(const VarAdjParams p) {
  const int g = blockIdx.y;
  const int lane = threadIdx.x & 63, w = lane % W, q = lane / W;
  const int64_t i = ((int64_t)blockIdx.x * kWavesPerBlock + wave_id()) * (64 / W) + q;
  if (i >= p.N2) return;
  const float *cb = p.Cbar + (int64_t)g * p.E12 * W + w;
  const int32_t e1 = ldro(p.vn_ptr, i + 1);
  int32_t e = ldro(p.vn_ptr, i);
  float s = 0.0f;
  // gathers issued in batches, summed in edge order; the adjoint rows are
  // streamed (non-temporal hint), as the decoder's message rows
  for (; e + 8 <= e1; e += 8) {
    float a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = ld_stream<W>(cb + (int64_t)ldro(p.vn_edges, e + u) * W);
#pragma unroll
    for (int u = 0; u < 8; ++u) s += a[u];
  }
  if (e + 4 <= e1) {
    float a[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) a[u] = ld_stream<W>(cb + (int64_t)ldro(p.vn_edges, e + u) * W);
#pragma unroll
    for (int u = 0; u < 4; ++u) s += a[u];
    e += 4;
  }
  if (e + 2 <= e1) {
    const float a0 = ld_stream<W>(cb + (int64_t)ldro(p.vn_edges, e) * W),
                a1 = ld_stream<W>(cb + (int64_t)ldro(p.vn_edges, e + 1) * W);
    s += a0;
    s += a1;
    e += 2;
  }
  if (e < e1) s += ld_stream<W>(cb + (int64_t)ldro(p.vn_edges, e) * W);
  p.Pbar[((int64_t)g * p.N2 + i) * W + w] = -s;
}

// First level of the reduction of the per-block partial sums: block c sums
// rows [c * chunk, (c + 1) * chunk) in a fixed order (the chunking depends only
// on the row count, so the result is the same on every run).
__global__ __launch_bounds__(kBlock) void k_reduce_wgrad_chunks(const float *partial, int64_t rows, int64_t chunk,
                                                                float *out) {
  const int t = threadIdx.x >> 5, lane = threadIdx.x & 31;
  const int64_t r0 = (int64_t)blockIdx.x * chunk, r1 = min(rows, r0 + chunk);
  float v = 0.0f;
  for (int64_t r = r0 + lane; r < r1; r += 32) v += partial[r * kMaxT + t];
  for (int off = 16; off >= 1; off >>= 1) v += __shfl_xor(v, off, 32);
  if (lane == 0) out[(int64_t)blockIdx.x * kMaxT + t] = v;
}

constexpr int kReduceChunks = 1024;

// dLoss/dw[t][l] from the per-block partial sums (fixed summation order).
__global__ __launch_bounds__(kBlock) void k_reduce_wgrad(const float *partial, int64_t rows, float *grad,
                                                         int32_t ntypes, int32_t wstride, int32_t it) {
  const int t = threadIdx.x >> 5, lane = threadIdx.x & 31;
  float v = 0.0f;
  for (int64_t r = lane; r < rows; r += 32) v += partial[r * kMaxT + t];
  for (int off = 16; off >= 1; off >>= 1) v += __shfl_xor(v, off, 32);
  if (lane == 0 && t < ntypes) grad[(int64_t)t * wstride + (it - 1)] = v;
}

// Seeds of the reverse sweep from dLoss/dposterior [B][N] (user order).
struct SeedParams {
  const float *gpost;
  const int32_t *msg_vn_user, *leaf_vn;
  int64_t N, N2, EL;
  int32_t B;
  float *Pbar, *gleaf;
};

template <int W>
__global__ __launch_bounds__(kBlock) void k_wbp_seed(const SeedParams p) {
  const int g = blockIdx.y;
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t item = idx / W;
  const int w = (int)(idx % W);
  const int f = g * W + w;
  if (item < p.N2) {
    p.Pbar[((int64_t)g * p.N2 + item) * W + w] = f < p.B ? p.gpost[(int64_t)f * p.N + p.msg_vn_user[item]] : 0.0f;
  } else if (item < p.N2 + p.EL) {
    const int64_t le = item - p.N2;
    p.gleaf[((int64_t)g * p.EL + le) * W + w] = f < p.B ? p.gpost[(int64_t)f * p.N + p.leaf_vn[le]] : 0.0f;
  }
}

__global__ __launch_bounds__(kBlock) void k_fill_zero(float *x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) x[i] = 0.0f;
}

// ----------------------------------------------------------------------------
// Workspace: the decoder's arrays plus forward states (c2v, P) in slots.

struct WbpPlan {
  Plan base;             // decoder layout (its c2v and P are state slot "work 0")
  int L = 0, k = 1, nck = 0, nseg = 0;
  size_t slot_c2v = 0, slot_P = 0, slot_bytes = 0;
  size_t off_slots = 0;  // work 1, checkpoints, segment states
  size_t off_cbar = 0, off_pbar = 0, off_gleaf = 0, off_partial = 0, off_chunks = 0, off_bits = 0, off_iters = 0,
         off_conv = 0;
  int64_t partial_rows = 0;
  size_t total = 0;
};

int64_t adj_blocks(const met_code *c, int W) {
  int64_t rows = 0;
  const int64_t per = (int64_t)kWavesPerBlock * (64 / W);
  for (const CheckClass &cc : c->classes) rows += (cc.n_checks + per - 1) / per;
  return rows;
}

WbpPlan make_wbp_plan(const met_code *c, int B, int L, int k) {
  WbpPlan p;
  const int W = choose_interleave(B);
  p.base = make_plan(c, B, true, true, W);
  p.L = L;
  p.k = k;
  p.nck = (L + k - 1) / k - 1;
  p.nseg = k - 1;
  const size_t GW = (size_t)p.base.G * W;
  p.slot_c2v = align256(GW * c->E12 * sizeof(float));
  p.slot_P = align256(GW * c->N2 * sizeof(float));
  p.slot_bytes = p.slot_c2v + p.slot_P;
  size_t o = p.base.total;
  p.off_slots = o;
  o += (size_t)(1 + p.nck + p.nseg) * p.slot_bytes;
  p.off_cbar = o;
  o += align256(GW * c->E12 * sizeof(float));
  p.off_pbar = o;
  o += align256(GW * c->N2 * sizeof(float));
  p.off_gleaf = o;
  o += align256(GW * c->EL * sizeof(float));
  p.partial_rows = adj_blocks(c, W) * p.base.G;
  p.off_partial = o;
  o += align256((size_t)p.partial_rows * kMaxT * sizeof(float));
  p.off_chunks = o;
  o += align256((size_t)kReduceChunks * kMaxT * sizeof(float));
  p.off_bits = o;
  o += align256((size_t)B * c->N);
  p.off_iters = o;
  o += align256((size_t)B * sizeof(int32_t));
  p.off_conv = o;
  o += align256((size_t)B);
  p.total = o;
  return p;
}

struct State {
  float *c2v;
  float *P;
};

struct Wbp {
  const met_code *c;
  const DeviceCode *d;
  WbpPlan pl;
  char *ws;
  hipStream_t st;
  int B;
  const float *weights;

  template <typename T>
  T *at(size_t off) const { return reinterpret_cast<T *>(ws + off); }

  // slot 0: the decoder's own c2v / P arrays; slots 1..: work 1, checkpoints, segment.
  State slot(int s) const {
    if (s == 0) return {at<float>(pl.base.off_c2v), at<float>(pl.base.off_P)};
    char *b = ws + pl.off_slots + (size_t)(s - 1) * pl.slot_bytes;
    return {reinterpret_cast<float *>(b), reinterpret_cast<float *>(b + pl.slot_c2v)};
  }
  State work(int l) const { return slot(l & 1); }
  State ckpt(int a) const { return slot(2 + (a / pl.k - 1)); }
  State seg(int off) const { return slot(2 + pl.nck + (off - 1)); }

  template <int W>
  void init(const float *llr, const uint8_t *syn, int32_t *iters, uint8_t *conv) {
    const Plan &b = pl.base;
    InitParams ip{};
    ip.llr = llr;
    ip.syn = syn;
    ip.msg_vn_user = d->msg_vn_user;
    ip.leaf_vn = d->leaf_vn;
    ip.chk_pos = d->chk_pos;
    ip.N = c->N;
    ip.M = c->M;
    ip.N2 = c->N2;
    ip.EL = c->EL;
    ip.B = B;
    ip.G = b.G;
    ip.Lt = at<float>(b.off_c2v);
    ip.L2 = at<float>(b.off_L2);
    ip.Lphi = at<float>(b.off_Lphi);
    ip.Lraw = at<float>(b.off_Lraw);
    ip.synw = at<uint64_t>(b.off_synw);
    ip.active = at<uint64_t>(b.off_active);
    ip.unsat = at<uint64_t>(b.off_unsat);
    ip.iters = iters;
    ip.converged = conv;
    hipLaunchKernelGGL(k_transpose<W>, dim3((unsigned)((c->N + 63) / 64), b.G), dim3(kBlock), 0, st, ip);
    const int64_t n = (c->N2 + c->EL) * W;
    if (n > 0)
      hipLaunchKernelGGL(k_init_items<W>, dim3((unsigned)((n + kBlock - 1) / kBlock), b.G), dim3(kBlock), 0, st,
                         ip);
    hipLaunchKernelGGL(k_pack_syndrome<W>, dim3((unsigned)std::max<int64_t>(1, (c->M + kBlock - 1) / kBlock), b.G),
                       dim3(kBlock), 0, st, ip);
  }

  // Forward iteration l from state `in` (l == 1: the LLRs) to state `out`.
  template <int W>
  void iterate(int l, State in, State out, bool post) {
    const Plan &b = pl.base;
    const size_t leaf_words = (size_t)b.G * c->EL, leaf_floats = leaf_words * W;
    CheckParams cp{};
    cp.edge_msgvn = d->edge_msgvn;
    cp.edge_type = d->edge_type;
    cp.leaf_type = d->leaf_type;
    cp.chk_msg_ptr = d->chk_msg_ptr;
    cp.chk_leaf_ptr = d->chk_leaf_ptr;
    cp.M = c->M;
    cp.N2 = c->N2;
    cp.E12 = c->E12;
    cp.EL = c->EL;
    cp.Pin = l == 1 ? at<float>(b.off_L2) : in.P;
    cp.c2v_in = in.c2v;
    cp.c2v = out.c2v;
    cp.Lphi = at<float>(b.off_Lphi);
    cp.Lraw = at<float>(b.off_Lraw);
    cp.P1 = at<float>(b.off_P1) + (size_t)(l & 1) * leaf_floats;
    cp.synw = at<uint64_t>(b.off_synw);
    cp.B1in = at<uint64_t>(b.off_B1) + (size_t)((l - 1) & 1) * leaf_words;
    cp.B1out = at<uint64_t>(b.off_B1) + (size_t)(l & 1) * leaf_words;
    cp.unsat = at<uint64_t>(b.off_unsat);
    cp.active = at<uint64_t>(b.off_active);
    cp.weights = weights;
    cp.wstride = pl.L;
    cp.it = l;
    cp.flags = F_WEIGHTED | (l == 1 ? F_FIRST : 0) | (post ? F_POST : 0);
    cp.G = b.G;
    const std::vector<ClassArgs> classes = class_args(c);
    for (const ClassArgs &a : classes) {
      ScopedTimer t(st, "k_check_weighted");
      launch_check<W>(cp, a, M_SPECIAL, 4, b.G, st);
    }
    VarParams vp{};
    vp.vn_ptr = d->vn_ptr;
    vp.vn_edges = d->vn_edges;
    vp.N2 = c->N2;
    vp.E12 = c->E12;
    vp.L2 = at<float>(b.off_L2);
    vp.c2v = out.c2v;
    vp.P = out.P;
    vp.active = at<uint64_t>(b.off_active);
    vp.it = l;
    vp.retire = 0;
    vp.G = b.G;
    const int64_t per = (int64_t)kWavesPerBlock * (64 / W);
    if (c->N2 > 0) {
      ScopedTimer t(st, "k_variable");
      hipLaunchKernelGGL((k_variable<W, 16>), dim3((unsigned)((c->N2 + per - 1) / per), b.G), dim3(kBlock), 0, st,
                         vp);
    }
  }

  template <int W>
  int forward(const float *llr, const uint8_t *syn, float *posterior, uint8_t *bits, uint8_t *conv) {
    const Plan &b = pl.base;
    int32_t *iters = at<int32_t>(pl.off_iters);
    if (!bits) bits = at<uint8_t>(pl.off_bits);
    if (!conv) conv = at<uint8_t>(pl.off_conv);
    init<W>(llr, syn, iters, conv);
    // the last segment's states go straight to the segment slots, where the
    // reverse sweep needs them (it recomputes the other segments only)
    const int a_last = (pl.L - 1) / pl.k * pl.k;
    State prev{nullptr, nullptr};
    for (int l = 1; l <= pl.L; ++l) {
      const State out = (l % pl.k == 0 && l < pl.L) ? ckpt(l) : (l > a_last && l < pl.L) ? seg(l - a_last) : work(l);
      iterate<W>(l, prev, out, l == pl.L);
      prev = out;
    }
    // syndrome test of the final decisions, then outputs in user order
    const size_t leaf_words = (size_t)b.G * c->EL, leaf_floats = leaf_words * W;
    TestParams tp{};
    tp.edge_msgvn = d->edge_msgvn;
    tp.chk_msg_ptr = d->chk_msg_ptr;
    tp.chk_leaf_ptr = d->chk_leaf_ptr;
    tp.M = c->M;
    tp.N2 = c->N2;
    tp.E12 = c->E12;
    tp.EL = c->EL;
    tp.P = prev.P;
    tp.synw = at<uint64_t>(b.off_synw);
    tp.B1 = at<uint64_t>(b.off_B1) + (size_t)(pl.L & 1) * leaf_words;
    tp.active = at<uint64_t>(b.off_active);
    tp.unsat = at<uint64_t>(b.off_unsat) + (size_t)(pl.L & 1) * b.G;
    const int64_t per = (int64_t)kWavesPerBlock * (64 / W);
    hipLaunchKernelGGL(k_test<W>, dim3((unsigned)((c->M + per - 1) / per), b.G), dim3(kBlock), 0, st, tp);
    FinalParams fp{};
    fp.vn_slot = d->vn_slot;
    fp.N = c->N;
    fp.N2 = c->N2;
    fp.EL = c->EL;
    fp.B = B;
    fp.max_iter = pl.L;
    fp.P = prev.P;
    fp.P1a = at<float>(b.off_P1);
    fp.P1b = at<float>(b.off_P1) + leaf_floats;
    fp.B1a = at<uint64_t>(b.off_B1);
    fp.B1b = at<uint64_t>(b.off_B1) + leaf_words;
    fp.active = at<uint64_t>(b.off_active);
    fp.unsat_last = tp.unsat;
    fp.iters = iters;
    fp.converged = conv;
    fp.bits = bits;
    fp.posterior = posterior;
    fp.G = b.G;
    hipLaunchKernelGGL(k_final_status<W>, dim3((B + kBlock - 1) / kBlock), dim3(kBlock), 0, st, fp);
    hipLaunchKernelGGL(k_finalize<W>, dim3((unsigned)((c->N + 63) / 64), b.G), dim3(kBlock), 0, st, fp);
    HIP_TRY(hipGetLastError());
    return MET_OK;
  }

  template <int W>
  void launch_adj(const AdjParams &p, const ClassArgs &a, unsigned blocks) {
    const dim3 grid(blocks, pl.base.G), block(kBlock);
    switch (a.shape) {
      case 0: hipLaunchKernelGGL((k_check_adj<W, 3, 1>), grid, block, 0, st, p, a); break;
      case 1: hipLaunchKernelGGL((k_check_adj<W, 2, 1>), grid, block, 0, st, p, a); break;
      case 2: hipLaunchKernelGGL((k_check_adj<W, 12, 0>), grid, block, 0, st, p, a); break;
      case 3: hipLaunchKernelGGL((k_check_adj<W, 11, 0>), grid, block, 0, st, p, a); break;
      case 4: hipLaunchKernelGGL((k_check_adj<W, 6, 0>), grid, block, 0, st, p, a); break;
      case 5: hipLaunchKernelGGL((k_check_adj<W, 5, 0>), grid, block, 0, st, p, a); break;
      case 6: hipLaunchKernelGGL((k_check_adj<W, 4, 0>), grid, block, 0, st, p, a); break;
      default: hipLaunchKernelGGL((k_check_adj<W, 0, 0>), grid, block, 0, st, p, a); break;
    }
  }

  template <int W>
  int backward(const float *gpost, float *grad_w) {
    const Plan &b = pl.base;
    const int G = b.G;
    float *cbar = at<float>(pl.off_cbar), *pbar = at<float>(pl.off_pbar), *gleaf = at<float>(pl.off_gleaf);
    float *partial = at<float>(pl.off_partial);
    const int64_t ncb = (int64_t)G * c->E12 * W;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)std::min<int64_t>(65535, (ncb + kBlock - 1) / kBlock + 1)),
                       dim3(kBlock), 0, st, cbar, ncb);
    SeedParams sp{};
    sp.gpost = gpost;
    sp.msg_vn_user = d->msg_vn_user;
    sp.leaf_vn = d->leaf_vn;
    sp.N = c->N;
    sp.N2 = c->N2;
    sp.EL = c->EL;
    sp.B = B;
    sp.Pbar = pbar;
    sp.gleaf = gleaf;
    {
      const int64_t n = (c->N2 + c->EL) * W;
      if (n > 0)
        hipLaunchKernelGGL(k_wbp_seed<W>, dim3((unsigned)((n + kBlock - 1) / kBlock), G), dim3(kBlock), 0, st, sp);
    }
    AdjParams ap{};
    ap.edge_msgvn = d->edge_msgvn;
    ap.edge_type = d->edge_type;
    ap.leaf_type = d->leaf_type;
    ap.chk_msg_ptr = d->chk_msg_ptr;
    ap.chk_leaf_ptr = d->chk_leaf_ptr;
    ap.M = c->M;
    ap.N2 = c->N2;
    ap.E12 = c->E12;
    ap.EL = c->EL;
    ap.Lphi = at<float>(b.off_Lphi);
    ap.synw = at<uint64_t>(b.off_synw);
    ap.Pbar = pbar;
    ap.Cbar = cbar;
    ap.weights = weights;
    ap.partial = partial;
    ap.wstride = pl.L;
    VarAdjParams vp{};
    vp.vn_ptr = d->vn_ptr;
    vp.vn_edges = d->vn_edges;
    vp.N2 = c->N2;
    vp.E12 = c->E12;
    vp.Cbar = cbar;
    vp.Pbar = pbar;
    const std::vector<ClassArgs> classes = class_args(c);
    const int64_t per = (int64_t)kWavesPerBlock * (64 / W);
    const int nsegs = (pl.L + pl.k - 1) / pl.k;
    for (int sg = nsegs - 1; sg >= 0; --sg) {
      const int a = sg * pl.k, bnd = std::min(a + pl.k, pl.L);
      // recompute states a+1 .. bnd-1 from the checkpoint at a (the last
      // segment's are still in the segment slots from the forward pass)
      State prev = a == 0 ? State{nullptr, nullptr} : ckpt(a);
      for (int l = a + 1; l < bnd && sg < nsegs - 1; ++l) {
        const State out = seg(l - a);
        iterate<W>(l, prev, out, false);
        prev = out;
      }
      for (int l = bnd; l > a; --l) {
        const State in = (l - 1 == a) ? (a == 0 ? State{nullptr, nullptr} : ckpt(a)) : seg(l - 1 - a);
        ap.Pin = l == 1 ? at<float>(b.off_L2) : in.P;
        ap.c2v_in = in.c2v;
        ap.gleaf = l == pl.L ? gleaf : nullptr;
        ap.it = l;
        ap.first = l == 1;
        int64_t row = 0;
        {
          ScopedTimer t(st, "k_check_adj");
          for (const ClassArgs &cl : classes) {
            const unsigned blocks = (unsigned)((cl.n_checks + per - 1) / per);
            ap.partial_base = row;
            launch_adj<W>(ap, cl, blocks);
            row += (int64_t)blocks * G;
          }
        }
        {
          // two levels: up to kReduceChunks blocks of fixed row ranges, then one block
          ScopedTimer t(st, "k_reduce_wgrad");
          const int64_t chunk = std::max<int64_t>(32, (row + kReduceChunks - 1) / kReduceChunks);
          const int64_t nch = (row + chunk - 1) / chunk;
          float *chunks = at<float>(pl.off_chunks);
          if (nch > 0)
            hipLaunchKernelGGL(k_reduce_wgrad_chunks, dim3((unsigned)nch), dim3(kBlock), 0, st, partial, row, chunk,
                               chunks);
          hipLaunchKernelGGL(k_reduce_wgrad, dim3(1), dim3(kBlock), 0, st, chunks, nch, grad_w, c->ntypes, pl.L, l);
        }
        if (l > 1 && c->N2 > 0) {
          ScopedTimer t(st, "k_variable_adj");
          hipLaunchKernelGGL(k_variable_adj<W>, dim3((unsigned)((c->N2 + per - 1) / per), G), dim3(kBlock), 0, st,
                             vp);
        }
      }
    }
    HIP_TRY(hipGetLastError());
    return MET_OK;
  }
};

int validate_wbp(const met_code *c, int32_t B, int32_t L, int32_t k) {
  if (!c) return fail(MET_EINVAL, "NULL code");
  for (const CheckClass &cc : c->classes)
    if (cc.shape == kShapeGeneric)
      for (int64_t j = cc.first_check; j < cc.first_check + cc.n_checks; ++j)
        if (c->chk_ptr[j + 1] - c->chk_ptr[j] > kMaxAdjDegree)
          return fail(MET_EINVAL, "weighted BP supports irregular checks of degree <= %d", kMaxAdjDegree);
  if (B < 1 || B > 65535) return fail(MET_EINVAL, "B = %d outside 1..65535", B);
  if (L < 1 || L > 100000) return fail(MET_EINVAL, "iterations = %d outside 1..100000", L);
  if (k < 1 || k > L) return fail(MET_EINVAL, "ckpt_every = %d outside 1..iterations", k);
  return MET_OK;
}

}  // namespace
}  // namespace met

using met::fail;

extern "C" int met_wbp_workspace_bytes(const met_code *c, int32_t B, int32_t iterations, int32_t ckpt_every,
                                       size_t *bytes) { return met::guarded("met_wbp_workspace_bytes", [&]() -> int {
  met::clear_error();
  int rc = met::validate_wbp(c, B, iterations, ckpt_every);
  if (rc) return rc;
  if (!bytes) return fail(MET_EINVAL, "NULL bytes");
  *bytes = met::make_wbp_plan(c, B, iterations, ckpt_every).total;
  return MET_OK;
  });
}

static int wbp_common(const met_code *c, int32_t B, int32_t L, int32_t k, const float *weights, void *ws,
                      size_t ws_bytes, met::WbpPlan *pl, const met::DeviceCode **d) {
  int rc = met::validate_wbp(c, B, L, k);
  if (rc) return rc;
  if (!weights || !ws) return fail(MET_EINVAL, "NULL buffer");
  if (((uintptr_t)weights & 3)) return fail(MET_EINVAL, "misaligned weights");
  if ((uintptr_t)ws & 255) return fail(MET_EINVAL, "workspace must be 256-byte aligned");
  *pl = met::make_wbp_plan(c, B, L, k);
  if (ws_bytes < pl->total) return fail(MET_EINVAL, "workspace of %zu bytes, %zu needed", ws_bytes, pl->total);
  return met::device_code(c, d);
}

extern "C" int met_wbp_forward(const met_code *c, const float *llr, const uint8_t *syn, int32_t B,
                               int32_t iterations, const float *weights, int32_t ckpt_every, float *posterior,
                               uint8_t *bits, uint8_t *converged, void *workspace, size_t ws_bytes, void *stream) { return met::guarded("met_wbp_forward", [&]() -> int {
  met::clear_error();
  if (!llr || !syn || !posterior) return fail(MET_EINVAL, "NULL buffer");
  if (((uintptr_t)llr & 3) || ((uintptr_t)posterior & 3)) return fail(MET_EINVAL, "misaligned float buffer");
  met::WbpPlan pl;
  const met::DeviceCode *d = nullptr;
  int rc = wbp_common(c, B, iterations, ckpt_every, weights, workspace, ws_bytes, &pl, &d);
  if (rc) return rc;
  met::Wbp w{c, d, pl, static_cast<char *>(workspace), (hipStream_t)stream, B, weights};
  switch (pl.base.W) {
    case 1: return w.forward<1>(llr, syn, posterior, bits, converged);
    case 4: return w.forward<4>(llr, syn, posterior, bits, converged);
    case 16: return w.forward<16>(llr, syn, posterior, bits, converged);
    case 32: return w.forward<32>(llr, syn, posterior, bits, converged);
    default: return w.forward<64>(llr, syn, posterior, bits, converged);
  }
  });
}

extern "C" int met_wbp_backward(const met_code *c, const float *grad_posterior, int32_t B, int32_t iterations,
                                const float *weights, int32_t ckpt_every, float *grad_weights, void *workspace,
                                size_t ws_bytes, void *stream) { return met::guarded("met_wbp_backward", [&]() -> int {
  met::clear_error();
  if (!grad_posterior || !grad_weights) return fail(MET_EINVAL, "NULL buffer");
  if (((uintptr_t)grad_posterior & 3) || ((uintptr_t)grad_weights & 3)) return fail(MET_EINVAL, "misaligned buffer");
  met::WbpPlan pl;
  const met::DeviceCode *d = nullptr;
  int rc = wbp_common(c, B, iterations, ckpt_every, weights, workspace, ws_bytes, &pl, &d);
  if (rc) return rc;
  met::Wbp w{c, d, pl, static_cast<char *>(workspace), (hipStream_t)stream, B, weights};
  switch (pl.base.W) {
    case 1: return w.backward<1>(grad_posterior, grad_weights);
    case 4: return w.backward<4>(grad_posterior, grad_weights);
    case 16: return w.backward<16>(grad_posterior, grad_weights);
    case 32: return w.backward<32>(grad_posterior, grad_weights);
    default: return w.backward<64>(grad_posterior, grad_weights);
  }
  });
}
