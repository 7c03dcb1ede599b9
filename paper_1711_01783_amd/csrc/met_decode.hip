// MI355X (gfx950) kernels and launch orchestration of the syndrome BP decoder.
//
// Algorithm: flooding sum-product belief propagation of the paper's Methods
// section (Steps 2-5, eq. (1)-(5)) in log-likelihood ratios, decoding B frames
// at once (Results, "High speed error correction with MET-LDPC codes").
//
// Formulation used on the GPU ("posterior form"): per message edge e = (v, j)
// the kernels keep only the check-to-variable message c2v_e, and per
// variable node of degree >= 2 its posterior P_v.  The variable-to-check
// message of eq. (4) is re-formed where it is consumed, v2c_e = P_v - c2v_e,
// which is eq. (4) in logarithms (L_v plus all incoming messages but e's own).
// Initialisation (Step 2, eq. (1)): P_v = L_v and c2v = 0.
//
// Check update (Step 3, eq. (2)-(3)) in the phi domain, phi(x) = ln coth(x/2):
//   |c2v_e| = phi( sum_{e' != e} phi(|x_e'|) ),  x = clamp(v2c, +-30)
//   sign(c2v_e) = (-1)^{s_j} * prod_{e' != e} sign(x_e')
// (the syndrome bit flips the sign: the decoder's target is Bob's syndrome,
// Step 1 and Step 5).  Leave-one-out sums use prefix/suffix sums, never a
// subtraction.  Degree-1 variable nodes ("leaves") never enter the iterations
// (Results; Table 1 note 1): their message into the check is the channel LLR,
// precomputed once as phi(|L|) with L's sign.
//
// Variable update (Step 4, eq. (4)-(5)): P_v = L_v + sum_e c2v_e over v's
// message edges, summed in a fixed order (deterministic).
//
// Syndrome test (Step 5) in early-exit mode: the check kernel of iteration l
// also evaluates H c = s for iteration l-1 from the signs of P^{l-1} and the
// stored leaf decisions of l-1, so the test costs no extra pass; the variable
// kernel of iteration l then retires frames whose test passed (their state
// stays at iteration l-1).  One final test pass covers the last iteration.
//
// Data layout (frame interleaved): B frames form G = ceil(B / W) groups of W
// frames; every per-item float array is [G][items][W], so one item's W
// frames are contiguous (W = 64: one 256-byte row per item, one lane per
// frame).  Per-item bit words (syndrome, leaf decisions, flags) hold the W
// frames of a group in one uint64.
//
// Compaction (early exit, groups of 64 frames): every few iterations, frames
// that stopped have their outputs written and their lanes freed; when the
// frames still running would fill markedly fewer groups than they occupy, they
// are moved into the fullest groups (all per-frame state: c2v, P, L, leaf
// inputs, syndrome and the last leaf decisions), so later launches skip the
// emptied groups.  A frame's arithmetic does not depend on its lane, so the
// results are identical with and without compaction.
#include "met_gpu.h"

namespace met {

TimingState g_timing;

namespace {

constexpr int kCompactEvery = 4;    // iterations between compaction points
constexpr int kCompactMinLeft = 4;  // no compaction this close to the budget
constexpr int kMaxGroups = 1024;    // 65535 frames in groups of 64

// flag = 1 if any frame of any group still runs (one block).
__global__ __launch_bounds__(kBlock) void k_any_active(const uint64_t *active, int G, uint32_t *flag) {
  uint64_t any = 0;
  for (int g = threadIdx.x; g < G; g += kBlock) any |= active[g];
  const int r = __syncthreads_or(any != 0ull);
  if (threadIdx.x == 0) *flag = (uint32_t)r;
}

struct CompactView {
  int32_t *n_dest, *dest, *src;  // header, receiving groups, [n_dest][64] source slots
};

__device__ __forceinline__ CompactView compact_view(int32_t *table, int G) {
  CompactView v;
  v.n_dest = table;
  v.dest = table + 64;
  v.src = table + 64 + ((G * 4 + 255) & ~255) / 4;  // as compact_table_bytes
  return v;
}

// Plans a compaction (one block).  Lanes whose frame stopped running had their
// outputs written by the flush that precedes this kernel: they are freed.  If
// the running frames would fit in at least a quarter fewer groups than hold
// them, the fullest groups become targets and every running frame of the
// other groups is assigned a free lane of a target; the frame map and the
// masks are updated here, the state is moved by k_compact_move*.
__global__ __launch_bounds__(kBlock) void k_compact_plan(uint64_t *active, int32_t *slot_frame, int32_t *table,
                                                        int G) {
  __shared__ int32_t cnt[kMaxGroups], order[kMaxGroups];
  __shared__ int32_t s_targets;
  const CompactView tv = compact_view(table, G);
  for (int s = threadIdx.x; s < G * 64; s += kBlock)
    if (slot_frame[s] >= 0 && !((active[s / 64] >> (s % 64)) & 1ull)) slot_frame[s] = -1;
  for (int g = threadIdx.x; g < G; g += kBlock) cnt[g] = __popcll(active[g]);
  __syncthreads();
  if (threadIdx.x == 0) {
    int A = 0, Gn = 0;
    for (int g = 0; g < G; ++g) {
      A += cnt[g];
      Gn += cnt[g] > 0;
    }
    const int Gt = (A + 63) / 64;
    int targets = 0;
    if (Gn - Gt >= max(1, Gn / 4)) {
      // groups by decreasing count (counting sort; ties by index)
      int start[66];
      for (int k = 0; k <= 65; ++k) start[k] = 0;
      for (int g = 0; g < G; ++g) ++start[64 - cnt[g] + 1];
      for (int k = 1; k <= 65; ++k) start[k] += start[k - 1];
      for (int g = 0; g < G; ++g) order[start[64 - cnt[g]]++] = g;
      targets = Gt;
    }
    s_targets = targets;
    *tv.n_dest = targets;
  }
  __syncthreads();
  const int T = s_targets;
  if (T == 0) return;
  for (int i = threadIdx.x; i < T * 64; i += kBlock) tv.src[i] = -1;
  for (int t = threadIdx.x; t < T; t += kBlock) tv.dest[t] = order[t];
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    uint64_t tact = active[order[0]];
    for (int k = T; k < G; ++k) {
      const int gs = order[k];
      uint64_t a = active[gs];
      while (a) {
        const int ws = __ffsll((unsigned long long)a) - 1;
        a &= a - 1;
        while (tact == ~0ull) {
          active[order[t]] = tact;
          tact = active[order[++t]];
        }
        const int wt = __ffsll((unsigned long long)~tact) - 1;
        tact |= 1ull << wt;
        const int gt = order[t];
        tv.src[t * 64 + wt] = gs * 64 + ws;
        slot_frame[gt * 64 + wt] = slot_frame[gs * 64 + ws];
        slot_frame[gs * 64 + ws] = -1;
      }
      active[gs] = 0ull;
    }
    active[order[t]] = tact;
  }
}

// Moves the W = 64 lanes of float rows [G][items][64] into the receiving groups.
__global__ __launch_bounds__(kBlock) void k_compact_move(int32_t *table, int G, float *arr, int64_t items) {
  const CompactView tv = compact_view(table, G);
  const int t = blockIdx.y;
  if (t >= *tv.n_dest) return;
  const int lane = threadIdx.x & 63;
  const int src = tv.src[t * 64 + lane];
  if (!__syncthreads_or(src >= 0)) return;
  const int64_t gt = tv.dest[t], gs = src >> 6, ws = src & 63;
  for (int64_t i = (int64_t)blockIdx.x * kWavesPerBlock + wave_id(); i < items;
       i += (int64_t)gridDim.x * kWavesPerBlock)
    if (src >= 0) arr[(gt * items + i) * 64 + lane] = arr[(gs * items + i) * 64 + ws];
}

// Moves bits of per-item words [G][items] (bit w = frame w of the group).
__global__ __launch_bounds__(kBlock) void k_compact_move_bits(int32_t *table, int G, uint64_t *arr, int64_t items) {
  __shared__ int32_t in_lane[64], in_src[64];
  __shared__ int32_t n_in;
  const CompactView tv = compact_view(table, G);
  const int t = blockIdx.y;
  if (t >= *tv.n_dest) return;
  if (threadIdx.x == 0) {
    int n = 0;
    for (int w = 0; w < 64; ++w) {
      const int src = tv.src[t * 64 + w];
      if (src >= 0) {
        in_lane[n] = w;
        in_src[n] = src;
        ++n;
      }
    }
    n_in = n;
  }
  __syncthreads();
  const int n = n_in;
  if (n == 0) return;
  const int64_t gt = tv.dest[t];
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < items; i += (int64_t)gridDim.x * kBlock) {
    uint64_t word = arr[gt * items + i];
    for (int k = 0; k < n; ++k) {
      const int src = in_src[k];
      const uint64_t bit = (arr[(int64_t)(src >> 6) * items + i] >> (src & 63)) & 1ull;
      word = (word & ~(1ull << in_lane[k])) | (bit << in_lane[k]);
    }
    arr[gt * items + i] = word;
  }
}

__global__ __launch_bounds__(kBlock) void k_init_slots(int32_t *slot_frame, int B, int GW) {
  for (int s = blockIdx.x * kBlock + threadIdx.x; s < GW; s += gridDim.x * kBlock) slot_frame[s] = s < B ? s : -1;
}

struct Decoder {
  const met_code *c;
  const DeviceCode *d;
  Plan pl;
  char *ws;
  hipStream_t st;
  int B;
  int cn_ipw = 4;    // check steps per wave (W = 64 only): 1, 2 or 4
  int vn_chunk = 16; // gathers in flight per variable node: 8, 16 or 32

  template <typename T>
  T *at(size_t off) const { return reinterpret_cast<T *>(ws + off); }

  // CT: storage type of the check-to-variable messages (float, or half_t for
  // MET_C2V_FP16; the arithmetic is float either way).
  template <int W, typename CT = float>
  int run(const float *llr, const uint8_t *syn, int max_iter, uint32_t flags, uint8_t *bits, int32_t *iters,
          uint8_t *conv, float *post, const float *weights, int32_t wstride) {
    const int G = pl.G;
    float *c2v = at<float>(pl.off_c2v), *P = at<float>(pl.off_P), *L2 = at<float>(pl.off_L2);
    float *Lphi = at<float>(pl.off_Lphi);
    float *Lraw = pl.lraw ? at<float>(pl.off_Lraw) : nullptr;
    float *P1 = pl.p1 ? at<float>(pl.off_P1) : nullptr;
    uint64_t *synw = at<uint64_t>(pl.off_synw), *B1 = at<uint64_t>(pl.off_B1);
    uint64_t *unsat = at<uint64_t>(pl.off_unsat), *active = at<uint64_t>(pl.off_active);
    const size_t leaf_words = (size_t)G * c->EL;
    const size_t leaf_floats = (size_t)G * c->EL * W;

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
    ip.G = G;
    ip.Lt = c2v;
    ip.L2 = L2;
    ip.Lphi = Lphi;
    ip.Lraw = Lraw;
    ip.synw = synw;
    ip.active = active;
    ip.unsat = unsat;
    ip.iters = iters;
    ip.converged = conv;
    {
      ScopedTimer t(st, "k_transpose");
      hipLaunchKernelGGL(k_transpose<W>, dim3((unsigned)((c->N + 63) / 64), G), dim3(kBlock), 0, st, ip);
    }
    {
      const int64_t n = (c->N2 + c->EL) * W;
      ScopedTimer t(st, "k_init_items");
      if (n > 0)
        hipLaunchKernelGGL(k_init_items<W>, dim3((unsigned)((n + kBlock - 1) / kBlock), G), dim3(kBlock), 0, st, ip);
    }
    {
      ScopedTimer t(st, "k_pack_syndrome");
      hipLaunchKernelGGL(k_pack_syndrome<W>, dim3((unsigned)std::max<int64_t>(1, (c->M + kBlock - 1) / kBlock), G),
                         dim3(kBlock), 0, st, ip);
    }

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
    cp.c2v = c2v;
    cp.c2v_in = c2v;
    cp.Lphi = Lphi;
    cp.Lraw = Lraw;
    cp.synw = synw;
    cp.active = active;
    cp.weights = weights;
    cp.wstride = wstride;
    cp.G = G;
    const std::vector<ClassArgs> classes = class_args(c);
    VarParams vp{};
    vp.vn_ptr = d->vn_ptr;
    vp.vn_edges = d->vn_edges;
    vp.N2 = c->N2;
    vp.E12 = c->E12;
    vp.L2 = L2;
    vp.c2v = c2v;
    vp.P = P;
    vp.active = active;
    vp.iters = iters;
    vp.converged = conv;
    vp.G = G;
    const int64_t vn_per_block = (int64_t)kWavesPerBlock * (64 / W);
    const unsigned vn_blocks = (unsigned)((c->N2 + vn_per_block - 1) / vn_per_block);
    const bool early = !(flags & MET_FIXED_ITERS);
    const bool special = post || weights;
    // (compaction moves float message rows: not with half-precision storage)
    const bool compact = W == 64 && G > 1 && early && !special && !(flags & MET_NO_COMPACT) &&
                         std::is_same<CT, float>::value;
    int32_t *slot_frame = compact ? at<int32_t>(pl.off_slot) : nullptr;
    int32_t *ctab = at<int32_t>(pl.off_ctab);
    vp.slot_frame = slot_frame;
    if (compact)
      hipLaunchKernelGGL(k_init_slots, dim3((unsigned)((G * W + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                         slot_frame, B, G * W);
    FinalParams fp{};
    fp.vn_slot = d->vn_slot;
    fp.N = c->N;
    fp.N2 = c->N2;
    fp.EL = c->EL;
    fp.B = B;
    fp.max_iter = max_iter;
    fp.P = P;
    fp.P1a = P1;
    fp.P1b = P1 ? P1 + leaf_floats : nullptr;
    fp.B1a = B1;
    fp.B1b = B1 + leaf_words;
    fp.active = active;
    fp.iters = iters;
    fp.converged = conv;
    fp.bits = bits;
    fp.posterior = post;
    fp.slot_frame = slot_frame;
    fp.G = G;
    const int base_flags = (post ? F_POST : 0) | (weights ? F_WEIGHTED : 0);
    // Early stop of the launch sequence: in early-exit mode the host reads
    // whether any frame still runs after iterations 4, 8, 16, ... (a stream
    // synchronisation each, so a doubling schedule); once none does, the
    // remaining iterations would launch kernels with nothing to do, and the
    // final test and outputs follow at once.  Not while the stream is being
    // captured into a graph (no synchronisation is possible there).
    bool can_stop = early;
    if (can_stop) {
      hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
      HIP_TRY(hipStreamIsCapturing(st, &cs));
      can_stop = cs == hipStreamCaptureStatusNone;
    }
    int next_check = 4;
    uint32_t *flag = at<uint32_t>(pl.off_flag);

    for (int it = 1; it <= max_iter; ++it) {
      cp.it = it;
      cp.flags = base_flags | (it == 1 ? F_FIRST : 0) | (early && it >= 2 ? F_TEST : 0);
      cp.Pin = it == 1 ? L2 : P;
      cp.B1in = B1 + (size_t)((it - 1) & 1) * leaf_words;
      cp.B1out = B1 + (size_t)(it & 1) * leaf_words;
      cp.P1 = P1 ? P1 + (size_t)(it & 1) * leaf_floats : nullptr;
      cp.unsat = unsat + (size_t)((it - 1) & 1) * G;
      const int mode = special ? M_SPECIAL : (it == 1 ? M_FIRST : M_MAIN);
      for (size_t k = 0; k < classes.size(); ++k) {
        cp.unsat_clear = k == 0 ? unsat + (size_t)(it & 1) * G : nullptr;
        ScopedTimer t(st, kCheckKernelName[classes[k].shape]);
        launch_check<W, CT>(cp, classes[k], mode, cn_ipw, G, st);
      }
      vp.it = it;
      vp.retire = early && it >= 2;
      vp.unsat = unsat + (size_t)((it - 1) & 1) * G;
      if (vn_blocks > 0) {
        ScopedTimer t(st, "k_variable");
        const dim3 grid(vn_blocks, G);
        if (vn_chunk == 32)
          hipLaunchKernelGGL((k_variable<W, 32, CT>), grid, dim3(kBlock), 0, st, vp);
        else if (vn_chunk == 16)
          hipLaunchKernelGGL((k_variable<W, 16, CT>), grid, dim3(kBlock), 0, st, vp);
        else
          hipLaunchKernelGGL((k_variable<W, 8, CT>), grid, dim3(kBlock), 0, st, vp);
      }
      if (compact && it % kCompactEvery == 0 && max_iter - it >= kCompactMinLeft) {
        ScopedTimer t(st, "k_compact");
        // outputs of frames that stopped, then the plan, then the state the
        // next check update reads: P, c2v, L, leaf inputs, syndrome, and the
        // leaf decisions of this iteration (tested by the next check update)
        FinalParams ff = fp;
        ff.flush = 1;
        hipLaunchKernelGGL(k_finalize<W>, dim3((unsigned)((c->N + 63) / 64), G), dim3(kBlock), 0, st, ff);
        hipLaunchKernelGGL(k_compact_plan, dim3(1), dim3(kBlock), 0, st, active, slot_frame, ctab, G);
        auto move = [&](float *a, int64_t items) {
          if (items > 0)
            hipLaunchKernelGGL(k_compact_move, dim3((unsigned)std::min<int64_t>(2048, (items + 3) / 4), G),
                               dim3(kBlock), 0, st, ctab, G, a, items);
        };
        auto move_bits = [&](uint64_t *a, int64_t items) {
          if (items > 0)
            hipLaunchKernelGGL(k_compact_move_bits, dim3((unsigned)std::min<int64_t>(1024, (items + 255) / 256), G),
                               dim3(kBlock), 0, st, ctab, G, a, items);
        };
        move(c2v, c->E12);
        move(P, c->N2);
        move(L2, c->N2);
        move(Lphi, c->EL);
        move_bits(synw, c->M);
        move_bits(B1 + (size_t)(it & 1) * leaf_words, c->EL);
      }
      if (can_stop && it == next_check && it < max_iter) {
        next_check *= 2;
        hipLaunchKernelGGL(k_any_active, dim3(1), dim3(kBlock), 0, st, active, G, flag);
        uint32_t any = 1;
        HIP_TRY(hipMemcpyAsync(&any, flag, sizeof any, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (!any) break;  // every frame has stopped
      }
    }
    TestParams tp{};
    tp.edge_msgvn = d->edge_msgvn;
    tp.chk_msg_ptr = d->chk_msg_ptr;
    tp.chk_leaf_ptr = d->chk_leaf_ptr;
    tp.M = c->M;
    tp.N2 = c->N2;
    tp.E12 = c->E12;
    tp.EL = c->EL;
    tp.P = P;
    tp.synw = synw;
    tp.B1 = B1 + (size_t)(max_iter & 1) * leaf_words;
    tp.active = active;
    tp.unsat = unsat + (size_t)(max_iter & 1) * G;
    {
      const int64_t per = (int64_t)kWavesPerBlock * (64 / W);
      ScopedTimer t(st, "k_test");
      hipLaunchKernelGGL(k_test<W>, dim3((unsigned)((c->M + per - 1) / per), G), dim3(kBlock), 0, st, tp);
    }
    fp.unsat_last = unsat + (size_t)(max_iter & 1) * G;
    {
      ScopedTimer t(st, "k_finalize");
      hipLaunchKernelGGL(k_final_status<W>, dim3((B + kBlock - 1) / kBlock), dim3(kBlock), 0, st, fp);
      hipLaunchKernelGGL(k_finalize<W>, dim3((unsigned)((c->N + 63) / 64), G), dim3(kBlock), 0, st, fp);
    }
    HIP_TRY(hipGetLastError());
    return MET_OK;
  }
};

}  // namespace

int device_code(const met_code *cc, const DeviceCode **out) {
  met_code *c = const_cast<met_code *>(cc);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(MET_EINVAL, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(c->mu);
  DeviceCode &d = c->dev[dev];
  if (d.ready) {
    *out = &d;
    return MET_OK;
  }
  struct Part {
    const void *src;
    size_t bytes;
    size_t off;
  };
  std::vector<Part> parts = {
      {c->edge_msgvn.data(), c->edge_msgvn.size() * 4, 0},   {c->edge_type_msg.data(), c->edge_type_msg.size(), 0},
      {c->vn_ptr.data(), c->vn_ptr.size() * 4, 0},           {c->vn_edges.data(), c->vn_edges.size() * 4, 0},
      {c->leaf_vn_user.data(), c->leaf_vn_user.size() * 4, 0}, {c->leaf_type.data(), c->leaf_type.size(), 0},
      {c->msg_vn_user.data(), c->msg_vn_user.size() * 4, 0}, {c->vn_slot.data(), c->vn_slot.size() * 4, 0},
      {c->chk_msg_ptr.data(), c->chk_msg_ptr.size() * 4, 0}, {c->chk_leaf_ptr.data(), c->chk_leaf_ptr.size() * 4, 0},
      {c->vn.data(), c->vn.size() * 4, 0},                   {c->chk_ptr.data(), c->chk_ptr.size() * 4, 0},
      {c->chk_pos.data(), c->chk_pos.size() * 4, 0},
  };
  size_t total = 0;
  for (Part &p : parts) {
    p.off = total;
    total += align256(std::max<size_t>(p.bytes, 4));
  }
  void *base = nullptr;
  hipError_t e = hipMalloc(&base, total);
  if (e != hipSuccess) return fail(MET_ENOMEM, "hipMalloc(%zu) for the adjacency: %s", total, hipGetErrorString(e));
  for (const Part &p : parts) {
    if (p.bytes == 0) continue;
    e = hipMemcpy(static_cast<char *>(base) + p.off, p.src, p.bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(base);
      return fail(MET_EHIP, "hipMemcpy of the adjacency: %s", hipGetErrorString(e));
    }
  }
  char *b = static_cast<char *>(base);
  d.base = base;
  d.bytes = total;
  d.edge_msgvn = reinterpret_cast<const int32_t *>(b + parts[0].off);
  d.edge_type = reinterpret_cast<const int8_t *>(b + parts[1].off);
  d.vn_ptr = reinterpret_cast<const int32_t *>(b + parts[2].off);
  d.vn_edges = reinterpret_cast<const int32_t *>(b + parts[3].off);
  d.leaf_vn = reinterpret_cast<const int32_t *>(b + parts[4].off);
  d.leaf_type = reinterpret_cast<const int8_t *>(b + parts[5].off);
  d.msg_vn_user = reinterpret_cast<const int32_t *>(b + parts[6].off);
  d.vn_slot = reinterpret_cast<const int32_t *>(b + parts[7].off);
  d.chk_msg_ptr = reinterpret_cast<const int32_t *>(b + parts[8].off);
  d.chk_leaf_ptr = reinterpret_cast<const int32_t *>(b + parts[9].off);
  d.all_vn = reinterpret_cast<const int32_t *>(b + parts[10].off);
  d.all_ptr = reinterpret_cast<const int32_t *>(b + parts[11].off);
  d.chk_pos = reinterpret_cast<const int32_t *>(b + parts[12].off);
  d.ready = true;
  *out = &d;
  return MET_OK;
}

}  // namespace met

using met::fail;

extern "C" void met_code_free(met_code *c) {
  if (!c) return;
  met_code_free(c->all_vns);
  int cur = -1;
  const bool have = hipGetDevice(&cur) == hipSuccess;
  for (int k = 0; k < met::kMaxDevices; ++k) {
    if (c->dev[k].ready) {
      if (hipSetDevice(k) == hipSuccess) (void)hipFree(c->dev[k].base);
    }
  }
  if (have && cur >= 0) (void)hipSetDevice(cur);
  delete c;
}

extern "C" int met_syndrome(const met_code *c, const uint8_t *bits, int32_t B, uint8_t *syn, void *stream) { return met::guarded("met_syndrome", [&]() -> int {
  met::clear_error();
  if (!c || !bits || !syn) return fail(MET_EINVAL, "met_syndrome: NULL argument");
  if (B < 1 || B > 65535) return fail(MET_EINVAL, "met_syndrome: B = %d outside 1..65535", B);
  const met::DeviceCode *d = nullptr;
  int rc = met::device_code(c, &d);
  if (rc) return rc;
  hipLaunchKernelGGL(met::k_syndrome, dim3((unsigned)((c->M + met::kBlock - 1) / met::kBlock), B),
                     dim3(met::kBlock), 0, (hipStream_t)stream, d->all_vn, d->all_ptr, c->N, c->M, bits, syn);
  HIP_TRY(hipGetLastError());
  return MET_OK;
  });
}

static int validate_decode(const met_code *c, int32_t B, uint32_t flags) {
  if (!c) return fail(MET_EINVAL, "NULL code");
  if (B < 1 || B > 65535) return fail(MET_EINVAL, "B = %d outside 1..65535", B);
  if (flags & ~(uint32_t)(MET_FIXED_ITERS | MET_NO_COMPACT | MET_NO_DEG1_SKIP | MET_C2V_FP16 | MET_C2V_Q8 |
                          MET_CHECK_LUT))
    return fail(MET_EINVAL, "unknown flags 0x%x", flags);
  if ((flags & MET_C2V_FP16) && (flags & MET_C2V_Q8))
    return fail(MET_EINVAL, "MET_C2V_FP16 and MET_C2V_Q8 exclude each other");
  if ((flags & MET_CHECK_LUT) && !(flags & MET_C2V_Q8))
    return fail(MET_EINVAL, "MET_CHECK_LUT needs MET_C2V_Q8 (its tables live on the 8-bit grid)");
  if ((flags & (MET_C2V_FP16 | MET_C2V_Q8)) && met::choose_interleave(B) != 64)
    return fail(MET_EINVAL, "reduced message storage needs groups of 64 frames (B > 32), B = %d", B);
  return MET_OK;
}

static size_t c2v_bytes(uint32_t flags) {
  if (flags & MET_C2V_Q8) return sizeof(met::q8_t);
  return (flags & MET_C2V_FP16) ? sizeof(met::half_t) : sizeof(float);
}

// The layout a decode with these flags runs on: the code's own, or its view
// with degree-1 variable nodes iterated.
static int decode_layout(const met_code *c, uint32_t flags, const met_code **out) {
  if (flags & MET_NO_DEG1_SKIP) return met::all_vns_view(c, out);
  *out = c;
  return MET_OK;
}

extern "C" int met_decode_workspace_bytes(const met_code *c, int32_t B, uint32_t flags, int32_t want_posterior,
                                          size_t *bytes) { return met::guarded("met_decode_workspace_bytes", [&]() -> int {
  met::clear_error();
  int rc = validate_decode(c, B, flags);
  if (rc) return rc;
  if (!bytes) return fail(MET_EINVAL, "NULL bytes");
  rc = decode_layout(c, flags, &c);
  if (rc) return rc;
  *bytes = met::make_plan(c, B, want_posterior != 0, false, met::choose_interleave(B), c2v_bytes(flags)).total;
  return MET_OK;
  });
}

extern "C" int met_decode_ex(const met_code *c, const float *llr, const uint8_t *syn, int32_t B, int32_t max_iter,
                             uint32_t flags, uint8_t *bits, int32_t *iters, uint8_t *converged, float *posterior,
                             void *workspace, size_t ws_bytes, const met_tuning *tuning, void *stream) { return met::guarded("met_decode_ex", [&]() -> int {
  met::clear_error();
  int rc = validate_decode(c, B, flags);
  if (rc) return rc;
  if (!llr || !syn || !bits || !iters || !converged || !workspace) return fail(MET_EINVAL, "NULL buffer");
  if (max_iter < 1 || max_iter > 1000000) return fail(MET_EINVAL, "max_iter = %d outside 1..10^6", max_iter);
  if (((uintptr_t)llr & 3) || ((uintptr_t)posterior & 3) || ((uintptr_t)iters & 3))
    return fail(MET_EINVAL, "misaligned float/int buffer");
  if ((uintptr_t)workspace & 255) return fail(MET_EINVAL, "workspace must be 256-byte aligned");
  int ipw = 4, chunk = 16;
  if (tuning) {
    const int s = tuning->check_steps_per_wave;
    if (s != 0 && s != 1 && s != 2 && s != 4) return fail(MET_EINVAL, "check_steps_per_wave must be 0, 1, 2 or 4");
    if (s) ipw = s;
    const int u = tuning->variable_chunk;
    if (u != 0 && u != 8 && u != 16 && u != 32) return fail(MET_EINVAL, "variable_chunk must be 0, 8, 16 or 32");
    if (u) chunk = u;
    if (tuning->interleave) return fail(MET_EINVAL, "interleave applies to batched decoding only");
    for (int r = 0; r < 3; ++r)
      if (tuning->reserved[r]) return fail(MET_EINVAL, "reserved tuning fields must be 0");
  }
  rc = decode_layout(c, flags, &c);
  if (rc) return rc;
  const int W = met::choose_interleave(B);
  const met::Plan pl = met::make_plan(c, B, posterior != nullptr, false, W, c2v_bytes(flags));
  if (ws_bytes < pl.total) return fail(MET_EINVAL, "workspace of %zu bytes, %zu needed", ws_bytes, pl.total);
  const met::DeviceCode *d = nullptr;
  rc = met::device_code(c, &d);
  if (rc) return rc;
  met::Decoder dec{c, d, pl, static_cast<char *>(workspace), (hipStream_t)stream, B, ipw, chunk};
  if (flags & MET_C2V_FP16)
    return dec.run<64, met::half_t>(llr, syn, max_iter, flags, bits, iters, converged, posterior, nullptr, 0);
  if (flags & MET_CHECK_LUT)
    return dec.run<64, met::q8lut_t>(llr, syn, max_iter, flags, bits, iters, converged, posterior, nullptr, 0);
  if (flags & MET_C2V_Q8)
    return dec.run<64, met::q8_t>(llr, syn, max_iter, flags, bits, iters, converged, posterior, nullptr, 0);
  switch (W) {
    case 1: return dec.run<1>(llr, syn, max_iter, flags, bits, iters, converged, posterior, nullptr, 0);
    case 4: return dec.run<4>(llr, syn, max_iter, flags, bits, iters, converged, posterior, nullptr, 0);
    case 16: return dec.run<16>(llr, syn, max_iter, flags, bits, iters, converged, posterior, nullptr, 0);
    case 32: return dec.run<32>(llr, syn, max_iter, flags, bits, iters, converged, posterior, nullptr, 0);
    default: return dec.run<64>(llr, syn, max_iter, flags, bits, iters, converged, posterior, nullptr, 0);
  }
  });
}

extern "C" int met_decode(const met_code *c, const float *llr, const uint8_t *syn, int32_t B, int32_t max_iter,
                          uint32_t flags, uint8_t *bits, int32_t *iters, uint8_t *converged, float *posterior,
                          void *workspace, size_t ws_bytes, void *stream) { return met::guarded("met_decode", [&]() -> int {
  return met_decode_ex(c, llr, syn, B, max_iter, flags, bits, iters, converged, posterior, workspace, ws_bytes,
                       nullptr, stream);
  });
}

// ---- Decoding without allocation ------------------------------------------
// The workspace of met_decode_noalloc lives in a fixed device array of this
// translation unit.  Host code never uses the array's name as an address (on
// the host it is only a stand-in): the device address is looked up once per
// device with hipGetSymbolAddress and kept.
namespace {
constexpr size_t kScratchBytes = (size_t)MET_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[met::kMaxDevices] = {};

int scratch_address(void **out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= met::kMaxDevices) return fail(MET_EINVAL, "device %d beyond %d", dev, met::kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return fail(MET_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    if (!ptr || ((uintptr_t)ptr & 255)) return fail(MET_EHIP, "scratch array at %p is not 256-byte aligned", ptr);
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return MET_OK;
}
}  // namespace

extern "C" int met_decode_noalloc(const met_code *c, const float *llr, const uint8_t *syn, int32_t B,
                                  int32_t max_iter, uint32_t flags, uint8_t *bits, int32_t *iters,
                                  uint8_t *converged, float *posterior, void *stream) { return met::guarded("met_decode_noalloc", [&]() -> int {
  met::clear_error();
  int rc = validate_decode(c, B, flags);
  if (rc) return rc;
  if (flags & MET_NO_DEG1_SKIP)
    return fail(MET_EINVAL, "MET_NO_DEG1_SKIP builds a second layout of the code (allocates): not here");
  const met::Plan pl = met::make_plan(c, B, posterior != nullptr, false, met::choose_interleave(B), c2v_bytes(flags));
  if (pl.total > kScratchBytes)
    return fail(MET_EINVAL, "decode needs %zu bytes of workspace, the fixed scratch array holds %zu", pl.total,
                kScratchBytes);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= met::kMaxDevices) return fail(MET_EINVAL, "device %d beyond %d", dev, met::kMaxDevices);
  {
    // the adjacency must already be on this device: uploading it allocates
    std::lock_guard<std::mutex> lock(const_cast<met_code *>(c)->mu);
    if (!c->dev[dev].ready)
      return fail(MET_ESTATE, "the code's adjacency is not on device %d yet (a met_decode or met_syndrome call "
                  "on that device uploads it)", dev);
  }
  {
    std::lock_guard<std::mutex> lock(met::g_timing.mu);
    if (met::g_timing.on) return fail(MET_ESTATE, "per-launch timing is on (it creates HIP events)");
  }
  void *ws = nullptr;
  rc = scratch_address(&ws);
  if (rc) return rc;
  return met_decode_ex(c, llr, syn, B, max_iter, flags, bits, iters, converged, posterior, ws, kScratchBytes,
                       nullptr, stream);
  });
}

extern "C" int met_timing_enable(int32_t on) { return met::guarded("met_timing_enable", [&]() -> int {
  met::clear_error();
  std::lock_guard<std::mutex> lock(met::g_timing.mu);
  met::g_timing.on = on != 0;
  return MET_OK;
  });
}

extern "C" int met_timing_collect(met_kernel_time *out, int32_t max_entries, int32_t *n_entries) { return met::guarded("met_timing_collect", [&]() -> int {
  met::clear_error();
  if (!out || !n_entries || max_entries < 0) return fail(MET_EINVAL, "met_timing_collect: bad output");
  std::vector<met::TimingState::Rec> recs;
  {
    std::lock_guard<std::mutex> lock(met::g_timing.mu);
    recs.swap(met::g_timing.recs);
  }
  int32_t n = 0;
  int rc = MET_OK;
  for (const auto &r : recs) {
    float ms = 0.0f;
    hipError_t e = hipEventSynchronize(r.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess && rc == MET_OK) rc = fail(MET_EHIP, "timing events: %s", hipGetErrorString(e));
    int32_t k = 0;
    while (k < n && std::strncmp(out[k].name, r.name, sizeof out[k].name) != 0) ++k;
    if (k == n) {
      if (n == max_entries) continue;
      std::memset(&out[k], 0, sizeof out[k]);
      std::strncpy(out[k].name, r.name, sizeof out[k].name - 1);
      ++n;
    }
    out[k].launches++;
    out[k].total_ms += ms;
  }
  {
    std::lock_guard<std::mutex> lock(met::g_timing.mu);
    for (const auto &r : recs) {
      met::g_timing.pool.push_back(r.a);
      met::g_timing.pool.push_back(r.b);
    }
  }
  *n_entries = n;
  return rc;
  });
}
