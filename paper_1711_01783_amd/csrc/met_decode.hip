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
#include "met_gpu.h"

namespace met {

TimingState g_timing;

namespace {

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

  template <int W>
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
    const int base_flags = (post ? F_POST : 0) | (weights ? F_WEIGHTED : 0);

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
        launch_check<W>(cp, classes[k], mode, cn_ipw, G, st);
      }
      vp.it = it;
      vp.retire = early && it >= 2;
      vp.unsat = unsat + (size_t)((it - 1) & 1) * G;
      if (vn_blocks > 0) {
        ScopedTimer t(st, "k_variable");
        const dim3 grid(vn_blocks, G);
        if (vn_chunk == 32)
          hipLaunchKernelGGL((k_variable<W, 32>), grid, dim3(kBlock), 0, st, vp);
        else if (vn_chunk == 16)
          hipLaunchKernelGGL((k_variable<W, 16>), grid, dim3(kBlock), 0, st, vp);
        else
          hipLaunchKernelGGL((k_variable<W, 8>), grid, dim3(kBlock), 0, st, vp);
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
    fp.unsat_last = unsat + (size_t)(max_iter & 1) * G;
    fp.iters = iters;
    fp.converged = conv;
    fp.bits = bits;
    fp.posterior = post;
    fp.G = G;
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
  d.ready = true;
  *out = &d;
  return MET_OK;
}

}  // namespace met

using met::fail;

extern "C" void met_code_free(met_code *c) {
  if (!c) return;
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

extern "C" int met_syndrome(const met_code *c, const uint8_t *bits, int32_t B, uint8_t *syn, void *stream) {
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
}

static int validate_decode(const met_code *c, int32_t B, uint32_t flags) {
  if (!c) return fail(MET_EINVAL, "NULL code");
  if (B < 1 || B > 65535) return fail(MET_EINVAL, "B = %d outside 1..65535", B);
  if (flags & ~(uint32_t)MET_FIXED_ITERS) return fail(MET_EINVAL, "unknown flags 0x%x", flags);
  return MET_OK;
}

extern "C" int met_decode_workspace_bytes(const met_code *c, int32_t B, uint32_t flags, int32_t want_posterior,
                                          size_t *bytes) {
  met::clear_error();
  int rc = validate_decode(c, B, flags);
  if (rc) return rc;
  if (!bytes) return fail(MET_EINVAL, "NULL bytes");
  *bytes = met::make_plan(c, B, want_posterior != 0, false, met::choose_interleave(B)).total;
  return MET_OK;
}

extern "C" int met_decode_ex(const met_code *c, const float *llr, const uint8_t *syn, int32_t B, int32_t max_iter,
                             uint32_t flags, uint8_t *bits, int32_t *iters, uint8_t *converged, float *posterior,
                             void *workspace, size_t ws_bytes, const met_tuning *tuning, void *stream) {
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
    for (int r = 0; r < 4; ++r)
      if (tuning->reserved[r]) return fail(MET_EINVAL, "reserved tuning fields must be 0");
  }
  const int W = met::choose_interleave(B);
  const met::Plan pl = met::make_plan(c, B, posterior != nullptr, false, W);
  if (ws_bytes < pl.total) return fail(MET_EINVAL, "workspace of %zu bytes, %zu needed", ws_bytes, pl.total);
  const met::DeviceCode *d = nullptr;
  rc = met::device_code(c, &d);
  if (rc) return rc;
  met::Decoder dec{c, d, pl, static_cast<char *>(workspace), (hipStream_t)stream, B, ipw, chunk};
  switch (W) {
    case 1: return dec.run<1>(llr, syn, max_iter, flags, bits, iters, converged, posterior, nullptr, 0);
    case 4: return dec.run<4>(llr, syn, max_iter, flags, bits, iters, converged, posterior, nullptr, 0);
    case 16: return dec.run<16>(llr, syn, max_iter, flags, bits, iters, converged, posterior, nullptr, 0);
    default: return dec.run<64>(llr, syn, max_iter, flags, bits, iters, converged, posterior, nullptr, 0);
  }
}

extern "C" int met_decode(const met_code *c, const float *llr, const uint8_t *syn, int32_t B, int32_t max_iter,
                          uint32_t flags, uint8_t *bits, int32_t *iters, uint8_t *converged, float *posterior,
                          void *workspace, size_t ws_bytes, void *stream) {
  return met_decode_ex(c, llr, syn, B, max_iter, flags, bits, iters, converged, posterior, workspace, ws_bytes,
                       nullptr, stream);
}

extern "C" int met_timing_enable(int32_t on) {
  met::clear_error();
  std::lock_guard<std::mutex> lock(met::g_timing.mu);
  met::g_timing.on = on != 0;
  return MET_OK;
}

extern "C" int met_timing_collect(met_kernel_time *out, int32_t max_entries, int32_t *n_entries) {
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
}
