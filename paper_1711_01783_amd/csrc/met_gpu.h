// Device kernels and host launch helpers shared by the decoder and the
// weighted-BP translation units (each includes this header once).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <vector>

#include "met_internal.h"

namespace met {

// Optional per-launch timing with HIP events on the launch stream.
struct TimingState {
  std::mutex mu;
  bool on = false;
  struct Rec {
    const char *name;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};

extern TimingState g_timing;

struct ScopedTimer {
  hipStream_t st;
  const char *name;
  hipEvent_t a = nullptr, b = nullptr;
  ScopedTimer(hipStream_t s, const char *n) : st(s), name(n) {
    if (!g_timing.on) return;
    std::lock_guard<std::mutex> lock(g_timing.mu);
    a = g_timing.get();
    b = g_timing.get();
    if (a && b) (void)hipEventRecord(a, st);
  }
  ~ScopedTimer() {
    if (!a || !b) return;
    (void)hipEventRecord(b, st);
    std::lock_guard<std::mutex> lock(g_timing.mu);
    g_timing.recs.push_back({name, a, b});
  }
};

namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / 64;
constexpr float kLlrMax = 30.0f;
constexpr int kXcds = 8;  // accelerator dies; the hardware deals block b to die b mod 8

// Storage of check-to-variable messages: float, or IEEE half (MET_C2V_FP16),
// converted to float on load and rounded to nearest on store; the arithmetic
// is float either way.
using half_t = _Float16;

// 8-bit storage (MET_C2V_Q8): sign in bit 7 and the magnitude as an index k
// into a log-uniform grid, k = 0 for 0 and m_k = 2^(kQ8Lo + (k - 1) / kQ8PerOctave)
// for k = 1..127 (2^-14 to 2^5: magnitudes are at most about 30 after the
// clamp, and below 2^-14 a message moves no posterior that matters).  Codes
// are formed by rounding log2|v| on that grid (the geometric midpoints are the
// thresholds: relative error at most 2^(1/(2 kQ8PerOctave)) - 1 = 5.4 %) and
// read back through a 128-entry table of the grid values.
constexpr float kQ8Lo = -14.0f, kQ8Hi = 5.0f;
constexpr float kQ8PerOctave = 126.0f / (kQ8Hi - kQ8Lo);
// Grid index of a magnitude m >= 0 (0 for 0 and NaN, 127 for infinity).
__device__ __forceinline__ uint32_t q8_mag_code(float m) {
  float t = fmaf(__builtin_amdgcn_logf(m) - kQ8Lo, kQ8PerOctave, 1.0f);  // log2 on the grid
  return (uint32_t)fminf(fmaxf(__builtin_rintf(t), 0.0f), 127.0f);
}
__device__ __forceinline__ uint32_t q8_encode(float v) {
  return q8_mag_code(fabsf(v)) | ((__float_as_uint(v) >> 24) & 128u);
}
struct q8_t {
  uint8_t c;
  q8_t() = default;
  __device__ explicit q8_t(float v) : c((uint8_t)q8_encode(v)) {}
  __device__ operator float() const;
};
// The decoding table, built at compile time: 2^x as 2^n e^(f ln 2), the
// exponential by its Taylor series in double (f ln 2 < 0.7: 24 terms leave no
// error in double), rounded once to float.
struct Q8Table {
  float v[128];
};
constexpr double q8_exp2(double x) {
  int n = 0;
  while (x < 0.0) {
    x += 1.0;
    --n;
  }
  while (x >= 1.0) {
    x -= 1.0;
    ++n;
  }
  const double y = x * 0.69314718055994530942;
  double term = 1.0, sum = 1.0;
  for (int i = 1; i < 24; ++i) {
    term *= y / i;
    sum += term;
  }
  for (; n > 0; --n) sum *= 2.0;
  for (; n < 0; ++n) sum *= 0.5;
  return sum;
}
constexpr Q8Table make_q8_table() {
  Q8Table t{};
  t.v[0] = 0.0f;
  for (int k = 1; k < 128; ++k) t.v[k] = (float)q8_exp2((double)kQ8Lo + (double)(k - 1) / (double)kQ8PerOctave);
  return t;
}
[[maybe_unused]] static __constant__ Q8Table kQ8Table = make_q8_table();
__device__ __forceinline__ q8_t::operator float() const {
  const float m = kQ8Table.v[c & 127u];
  return (c & 128u) ? -m : m;
}

// Table-driven check update (MET_CHECK_LUT, with 8-bit storage; the
// lookup-table form of the update in the last Methods paragraph): a message
// input's phi is read from a table at the index of its magnitude on a grid
// kLutSub times finer than the storage grid, and an output's 8-bit code from a
// second table at the fine index of its phi-domain sum, so neither phi nor the
// logarithm of the store is evaluated per edge beyond the index.  Fine index
// i >= 1 stands for m_i = 2^(kQ8Lo + (i - kLutSub) / (kLutSub kQ8PerOctave))
// (i = kLutSub k is the storage grid's m_k), i = 0 for 0: 1.3 % rounding at
// most on either side.  The storage type q8lut_t is q8_t's codes; it selects
// the table form in the check kernels.
struct q8lut_t : q8_t {
  q8lut_t() = default;
  __device__ explicit q8lut_t(float v) : q8_t(v) {}
};
constexpr int kLutSub = 4, kLutSize = 128 * kLutSub;
__device__ __forceinline__ uint32_t lut_index(float m) {
  float t = fmaf(__builtin_amdgcn_logf(m) - kQ8Lo, kQ8PerOctave * kLutSub, (float)kLutSub);
  return (uint32_t)fminf(fmaxf(__builtin_rintf(t), 0.0f), (float)(kLutSize - 1));
}
struct PhiTables {
  float a[kLutSize];      // phi(m_i); phi(0) = infinity
  uint8_t out[kLutSize];  // storage code of phi(m_i)
};
// ln y for y > 0 in double: y = 2^n f with f in [1, 2), ln f = 2 artanh((f-1)/(f+1))
// by its series ((f-1)/(f+1) <= 1/3: 40 terms leave no error in double).
constexpr double ct_ln(double y) {
  if (y < 1.0) return -ct_ln(1.0 / y);
  int n = 0;
  while (y >= 2.0) {
    y *= 0.5;
    ++n;
  }
  const double z = (y - 1.0) / (y + 1.0), z2 = z * z;
  double term = z, sum = 0.0;
  for (int i = 0; i < 40; ++i) {
    sum += term / (2 * i + 1);
    term *= z2;
  }
  return n * 0.69314718055994530942 + 2.0 * sum;
}
// phi(m) = ln((1 + a) / (1 - a)) = 2 artanh(a), a = e^-m: the artanh series
// where a <= 1/2, else the logarithm with 1 - a from the series of -expm1(-m)
// (no cancellation for small m).
constexpr double ct_phi(double m) {
  const double a = q8_exp2(-m * 1.4426950408889634074);
  if (a <= 0.5) {
    const double a2 = a * a;
    double term = a, sum = 0.0;
    for (int i = 0; i < 60; ++i) {
      sum += term / (2 * i + 1);
      term *= a2;
    }
    return 2.0 * sum;
  }
  double t = 1.0, one_minus_a = 0.0;  // 1 - e^-m = m - m^2/2 + m^3/6 - ...
  for (int i = 1; i < 30; ++i) {
    t *= -m / i;
    one_minus_a -= t;
  }
  return ct_ln((2.0 - one_minus_a) / one_minus_a);
}
constexpr PhiTables make_phi_tables() {
  PhiTables t{};
  t.a[0] = __builtin_huge_valf();
  t.out[0] = 127;
  for (int k = 1; k < kLutSize; ++k) {
    const double m = q8_exp2((double)kQ8Lo + (double)(k - kLutSub) / ((double)kQ8PerOctave * kLutSub));
    const double ph = ct_phi(m);
    t.a[k] = (float)ph;
    double c = (ct_ln(ph) * 1.4426950408889634074 - (double)kQ8Lo) * (double)kQ8PerOctave + 1.0;
    c = c < 0.0 ? 0.0 : c > 127.0 ? 127.0 : c;
    t.out[k] = (uint8_t)(int)(c + 0.5);
  }
  return t;
}
[[maybe_unused]] static __constant__ PhiTables kPhiTables = make_phi_tables();

// Message rows are streamed: each kernel reads (and the check update writes)
// every row once, so rows of 256 bytes (64 frames per item, float messages)
// are loaded and stored with the non-temporal hint, which keeps them from
// displacing the rows that are reused (the gathered posteriors) in the
// caches.  Shorter rows (16 or 32 frames per item, 16-bit or 8-bit messages)
// share a 128-byte line with their neighbours, and the decodes that use 16 or
// 32 frames per item mostly fit in the Infinity Cache: there the hint made
// the decoders slower, and such rows are loaded and stored plainly.
template <int W, typename T>
constexpr bool kStreamRows = W * sizeof(T) >= 256;
template <int W, typename T>
__device__ __forceinline__ T ld_stream(const T *p) {
  if constexpr (kStreamRows<W, T>)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}
template <int W, typename T>
__device__ __forceinline__ void st_stream(T v, T *p) {
  if constexpr (kStreamRows<W, T>)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}
template <int W, typename CT>
__device__ __forceinline__ float ld_msg(const CT *p) {
  if constexpr (std::is_class<CT>::value) {  // 8-bit codes: their byte
    CT r;
    r.c = ld_stream<W>(reinterpret_cast<const uint8_t *>(p));
    return (float)r;
  } else {
    return (float)ld_stream<W>(p);
  }
}
template <int W, typename CT>
__device__ __forceinline__ float ld_c2v(const float *base, int64_t i) {
  return ld_msg<W, CT>(reinterpret_cast<const CT *>(base) + i);
}
template <int W, typename CT>
__device__ __forceinline__ void st_c2v(float *base, int64_t i, float v) {
  if constexpr (std::is_class<CT>::value) {
    const CT q(v);
    st_stream<W>(q.c, reinterpret_cast<uint8_t *>(base) + i);
  } else {
    st_stream<W>((CT)v, reinterpret_cast<CT *>(base) + i);
  }
}

enum : int32_t {
  F_FIRST = 1,     // iteration 1: P = L, c2v = 0
  F_TEST = 2,      // evaluate the syndrome test of the previous iteration
  F_POST = 4,      // store leaf posteriors
  F_WEIGHTED = 8,  // scale c2v by a per-(edge type, iteration) weight
};

// Compile-time modes of the fixed-shape check kernel.
enum : int { M_FIRST = 0, M_MAIN = 1, M_SPECIAL = 2 };

// phi(x) = ln coth(x/2) = -ln tanh(x/2) for x >= 0; phi(0) = inf, phi(inf) = 0.
// Two pieces, both evaluated (a select, no divergence):
//  x < 1:  ln(2/x) + z p(z), z = x^2 -- p approximates (ln coth(x/2) - ln(2/x))/x^2
//  x >= 1: 2u (1 + v q(v)), u = e^-x, v = u^2 -- q approximates (artanh(u)/u - 1)/u^2
// The four coefficients of p and of q are least-squares fits to those smooth
// functions on [0, 1] and [0, e^-2] (relative error of phi below 5e-8).
constexpr float kP0 = 0.08333319759866183f, kP1 = -0.004859869600170282f;
constexpr float kP2 = 0.00033799735484266977f, kP3 = -2.1679784689824217e-05f;
constexpr float kQ0 = 0.3333317118955837f, kQ1 = 0.2001411345623163f;
constexpr float kQ2 = 0.1393155479518919f, kQ3 = 0.1439900625146655f;
constexpr float kLn2 = 0.69314718055994531f;
constexpr float kLog2e = 1.4426950408889634f;

__device__ __forceinline__ float phi(float x) {
  const float z = x * x;
  const float ps = z * fmaf(z, fmaf(z, fmaf(z, kP3, kP2), kP1), kP0);
  const float lo = fmaf(-kLn2, __builtin_amdgcn_logf(x), kLn2) + ps;
  const float u = __builtin_amdgcn_exp2f(-x * kLog2e);
  const float v = u * u;
  const float hi = 2.0f * u * fmaf(v, fmaf(v, fmaf(v, fmaf(v, kQ3, kQ2), kQ1), kQ0), 1.0f);
  return x < 1.0f ? lo : hi;
}

// Index of the calling wave within its block, as a wave-uniform value (so that
// per-wave addresses stay in scalar registers and index loads are scalar).
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

// Tile of block (bx, g) of a (tiles, frame groups) grid: within each frame
// group, each XCD takes one contiguous range of tiles in order (rather than
// every 8th tile), so neighbouring checks, which share variable nodes in the
// decoder check order, and neighbouring variable nodes meet in the same L2.
// The hardware deals blocks by their linear index, so block (bx, g) runs on
// XCD (g nx + bx) mod 8; the XCDs' ranges are laid out in XCD order, and the
// groups keep the dispatch order (one after the other on all XCDs).  Measured
// against the hardware order: variable update 4 % and main check update 1 %
// faster; the weighted check update and the adjoint kernels were 2-3 % slower
// and keep the hardware order.
struct GridTile {
  int64_t bx;
  int g;
};
__device__ __forceinline__ GridTile xcd_grid_tile() {
  const int64_t nx = gridDim.x, bx = blockIdx.x;
  const int s = (int)(((int64_t)blockIdx.y * nx) % kXcds);  // XCD of the group's first block
  const int x = (int)((s + bx) % kXcds);
  int64_t first = 0;  // tiles of the XCDs before x
  for (int y = 0; y < x; ++y) {
    const int64_t r = (y - s + kXcds) % kXcds;  // first block of the group on XCD y
    if (r < nx) first += (nx - r + kXcds - 1) / kXcds;
  }
  return {first + bx / kXcds, (int)blockIdx.y};
}

// Load from memory that no kernel writes while the current one runs (the
// adjacency, packed syndromes, decisions of the previous iteration).  Going
// through the constant address space lets wave-uniform loads use the scalar
// unit (one fetch per wave, batched into wide scalar loads).
template <typename T>
__device__ __forceinline__ T ldro(const T *p, int64_t i) {
  return ((const __attribute__((address_space(4))) T *)p)[i];
}

// Edge type (scale table row) of edge e.  With 64 frames per item the index is
// the same in every lane; the byte is then cut from the aligned 32-bit word
// that holds it, which the scalar unit can fetch (it has no byte loads), so
// the scale lookup that depends on it stays scalar too.  Every device array
// of the adjacency is padded to 256 bytes, so the word is inside it.
template <int W>
__device__ __forceinline__ int32_t edge_type_of(const int8_t *t, int64_t e) {
  if constexpr (W == 64) {
    const uint32_t word = ldro(reinterpret_cast<const uint32_t *>(t), e >> 2);
    return (int32_t)(int8_t)(uint8_t)(word >> ((uint32_t)(e & 3) * 8u));
  } else {
    return ldro(t, e);
  }
}

// Scale w[type of the edge, it - 1] of the edge at offset `off` of this lane's
// item, items being `per` edges apart from `first`.  A wave holds 64 / W
// consecutive items (lane group q = lane / W has item0 + q); with at most four
// of them each item's scale is looked up on the scalar unit and the lane picks
// its own, otherwise every lane loads its type.  Items past n_items (lanes
// that store nothing) read item 0's.
template <int W>
__device__ __forceinline__ float edge_scale(const float *weights, int64_t wstride, int col, const int8_t *types,
                                            int64_t first, int per, int off, int64_t item0, int64_t n_items, int q,
                                            int64_t e_lane) {
  constexpr int IPWAVE = 64 / W;
  if constexpr (IPWAVE == 1) {
    return ldro(weights, (int64_t)edge_type_of<64>(types, e_lane) * wstride + col);
  } else if constexpr (IPWAVE <= 4) {
    float r = 0.0f;
#pragma unroll
    for (int u = 0; u < IPWAVE; ++u) {
      const int64_t iu = item0 + u < n_items ? item0 + u : 0;
      const float wu = ldro(weights, (int64_t)edge_type_of<64>(types, first + iu * per + off) * wstride + col);
      r = (q == u) ? wu : r;
    }
    return r;
  } else {
    return ldro(weights, (int64_t)ldro(types, e_lane) * wstride + col);
  }
}

__device__ __forceinline__ float clamp_llr(float x) { return fminf(fmaxf(x, -kLlrMax), kLlrMax); }

__device__ __forceinline__ uint32_t sign_bit(float x) { return __float_as_uint(x) >> 31; }

template <int W>
__device__ __forceinline__ uint64_t wmask() {
  return W == 64 ? ~0ull : ((1ull << W) - 1ull);
}

// OR of the W-bit chunks of a wave ballot (lane = item * W + frame).
template <int W>
__device__ __forceinline__ uint64_t fold(uint64_t b) {
  uint64_t r = 0;
#pragma unroll
  for (int q = 0; q < 64 / W; ++q) r |= (b >> (q * W)) & wmask<W>();
  return r;
}

// Records frames with an unsatisfied check; one atomic per wave at most, and
// none once the group's flags already hold these bits.
__device__ __forceinline__ void flag_unsat(uint64_t *dst, uint64_t f) {
  if (!f) return;
  const uint64_t seen = __hip_atomic_load(dst, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (f & ~seen) __hip_atomic_fetch_or(dst, f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct ClassArgs {
  int32_t shape, n_msg, n_leaf, pad;
  int64_t first_check, n_checks, first_msg, first_leaf;
};

struct CheckParams {
  const int32_t *edge_msgvn;
  const int8_t *edge_type;
  const int8_t *leaf_type;
  const int32_t *chk_msg_ptr;
  const int32_t *chk_leaf_ptr;
  int64_t M, N2, E12, EL;
  const float *Pin;      // [G][N2][W]  P^{l-1} (L when F_FIRST)
  const float *c2v_in;   // [G][E12][W] c2v^{l-1} (not read when F_FIRST); may equal c2v
  float *c2v;            // [G][E12][W] c2v^l
  const float *Lphi;     // [G][EL][W]  sign(L) * phi(|L|) of leaf VNs
  const float *Lraw;     // [G][EL][W]  leaf LLRs (F_POST / F_WEIGHTED)
  float *P1;             // [G][EL][W]  leaf posteriors of this iteration (F_POST)
  const uint64_t *synw;  // [G][M]
  const uint64_t *B1in;  // [G][EL] leaf decisions of iteration l-1 (F_TEST)
  uint64_t *B1out;       // [G][EL] leaf decisions of iteration l
  uint64_t *unsat;       // [G] frames with an unsatisfied check (F_TEST)
  uint64_t *unsat_clear; // [G] buffer to zero for iteration l+1's test, or NULL
  const uint64_t *active;
  const float *weights;  // [T][wstride]
  int32_t wstride, it, flags, G;
};

// Decision of a leaf VN after the check update: c = 1 iff L + c2v < 0, with
// c2v = sgn * phi(S) and |L| = phi(A).  Since phi decreases, |c2v| > |L| iff
// S < A; a tie (P = 0) decides 0.
__device__ __forceinline__ uint32_t leaf_bit(uint32_t neg_l, uint32_t neg_c, float S, float A) {
  if (neg_l == neg_c) return neg_l & (uint32_t)!(isinf(A) && isinf(S));
  if (S < A) return neg_c;
  if (S > A) return neg_l;
  return 0u;
}

// Writes the W leaf decisions of one item, keeping the stored bits of frames
// that are no longer active.
template <int W>
__device__ __forceinline__ void store_leaf_word(uint64_t *dst, uint64_t ball, int q, uint64_t act) {
  const uint64_t chunk = (ball >> (q * W)) & wmask<W>();
  *dst = (act == wmask<W>()) ? chunk : ((*dst & ~act) | (chunk & act));
}

__device__ __forceinline__ void clear_next_unsat(const CheckParams &p, int64_t bx, int g) {
  if (p.unsat_clear && bx == 0 && g == 0)
    for (int gg = threadIdx.x; gg < p.G; gg += kBlock) p.unsat_clear[gg] = 0ull;
}

// Loads of words that an earlier phase of the same persistent launch may have
// written.  The phase barrier orders those writes before this load, so a plain
// vector load sees them; the scalar cache, which no barrier invalidates, must
// not be used (the launch stores to these buffers, so the compiler keeps such
// loads in the vector path).  Outside persistent launches the words are
// constant for the kernel and go through the scalar cache.
template <bool PERSIST>
__device__ __forceinline__ uint64_t ld_word(const uint64_t *p, int64_t i) {
  if (PERSIST) return p[i];
  return ldro(p, i);
}

// Load of a word that another block may write in the same phase (the frame
// mask during retirement): a device-scope atomic load.
template <bool PERSIST>
__device__ __forceinline__ uint64_t ld_racy(const uint64_t *p, int64_t i) {
  if (PERSIST) return __hip_atomic_load(p + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return p[i];
}

// Check update of one class of checks with a compile-time shape (NM message
// edges, NL leaf edges per check).  Each wave takes IPW consecutive steps of
// 64/W checks; all loads of its checks are issued before any arithmetic.
template <int W, int NM, int NL, int MODE, int IPW, bool PERSIST, typename CT = float>
__device__ __forceinline__ void check_fixed_body(const CheckParams &p, const ClassArgs &c, int64_t bx, int g) {
  constexpr int D = NM + NL;
  constexpr int IPWAVE = 64 / W;
  constexpr bool lut = std::is_same<CT, q8lut_t>::value;
  clear_next_unsat(p, bx, g);
  [[maybe_unused]] const float *tab_a = nullptr;
  [[maybe_unused]] const uint8_t *tab_out = nullptr;
  if constexpr (lut) {  // the tables in LDS, before any thread of the block can leave
    __shared__ float s_a[kLutSize];
    __shared__ uint8_t s_out[kLutSize];
    for (int i = threadIdx.x; i < kLutSize; i += kBlock) {
      s_a[i] = kPhiTables.a[i];
      s_out[i] = kPhiTables.out[i];
    }
    __syncthreads();
    tab_a = s_a;
    tab_out = s_out;
  }
  const uint64_t act = p.active[g];  // not written during check updates
  if (act == 0ull) return;
  const int lane = threadIdx.x & 63, wv = wave_id();
  const int w = lane % W, q = lane / W;
  const bool lane_act = (act >> w) & 1ull;
  const bool first = MODE == M_FIRST || (MODE == M_SPECIAL && (p.flags & F_FIRST));
  const bool test = MODE != M_FIRST && (p.flags & F_TEST);
  const bool post = MODE == M_SPECIAL && (p.flags & F_POST);
  const bool weighted = MODE == M_SPECIAL && (p.flags & F_WEIGHTED);
  const int64_t base = (bx * kWavesPerBlock + wv) * IPW * IPWAVE;
  if (W == 64 && base >= c.n_checks) return;

  int64_t item[IPW];
  bool valid[IPW];
  float pv[IPW][NM > 0 ? NM : 1], cv[IPW][NM > 0 ? NM : 1], lf[IPW][NL > 0 ? NL : 1];
  uint64_t sw[IPW], b1[IPW][NL > 0 ? NL : 1];
#pragma unroll
  for (int k = 0; k < IPW; ++k) {
    const int64_t i = base + k * IPWAVE + q;
    valid[k] = i < c.n_checks;
    item[k] = valid[k] ? i : 0;
  }
  // loads: P gathers, c2v rows, leaf inputs, syndrome and previous decisions
#pragma unroll
  for (int k = 0; k < IPW; ++k) {
    const int64_t m0 = c.first_msg + item[k] * NM, l0 = c.first_leaf + item[k] * NL;
    sw[k] = ldro(p.synw, (int64_t)g * p.M + c.first_check + item[k]);
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      const int32_t vi = ldro(p.edge_msgvn, m0 + m);
      pv[k][m] = p.Pin[((int64_t)g * p.N2 + vi) * W + w];
      cv[k][m] = first ? 0.0f : ld_c2v<W, CT>(p.c2v_in, ((int64_t)g * p.E12 + m0 + m) * W + w);
    }
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      lf[k][l] = ld_stream<W>(&p.Lphi[((int64_t)g * p.EL + l0 + l) * W + w]);
      b1[k][l] = test ? ld_word<PERSIST>(p.B1in, (int64_t)g * p.EL + l0 + l) : 0ull;
    }
  }
  uint32_t bad = 0;
#pragma unroll
  for (int k = 0; k < IPW; ++k) {
    const int64_t m0 = c.first_msg + item[k] * NM, l0 = c.first_leaf + item[k] * NL;
    const uint32_t s = (uint32_t)(sw[k] >> w) & 1u;
    float A[D];
    uint32_t neg = 0, parity = s;
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      parity ^= (uint32_t)(pv[k][m] < 0.0f);
      const float x = clamp_llr(pv[k][m] - cv[k][m]);
      if constexpr (lut)
        A[m] = tab_a[lut_index(fabsf(x))];
      else
        A[m] = phi(fabsf(x));
      neg |= sign_bit(x) << m;
    }
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      A[NM + l] = fabsf(lf[k][l]);
      neg |= sign_bit(lf[k][l]) << (NM + l);
      parity ^= (uint32_t)(b1[k][l] >> w) & 1u;
    }
    if (test) bad |= parity & (uint32_t)(valid[k] && lane_act);
    const uint32_t tot = (__popc(neg) & 1u) ^ s;
    // leave-one-out sums S[m] = sum of A over the other inputs, from prefix
    // and suffix sums (no subtraction; no additions of zero)
    float pre[D], suf[D], S[D];
    pre[1] = A[0];
#pragma unroll
    for (int m = 2; m < D; ++m) pre[m] = pre[m - 1] + A[m - 1];
    suf[D - 2] = A[D - 1];
#pragma unroll
    for (int m = D - 3; m >= 0; --m) suf[m] = suf[m + 1] + A[m + 1];
    S[0] = suf[0];
    S[D - 1] = pre[D - 1];
#pragma unroll
    for (int m = 1; m < D - 1; ++m) S[m] = pre[m] + suf[m];
    const bool store = valid[k] && lane_act;
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      if constexpr (lut) {
        const uint32_t code = tab_out[lut_index(S[m])] | (((tot ^ (neg >> m)) & 1u) << 7);
        if (store)
          st_stream<W>((uint8_t)code, reinterpret_cast<uint8_t *>(p.c2v) + ((int64_t)g * p.E12 + m0 + m) * W + w);
      } else {
        const float mag = phi(S[m]);
        float out = ((tot ^ (neg >> m)) & 1u) ? -mag : mag;
        if (weighted)
          out *= edge_scale<W>(p.weights, p.wstride, p.it - 1, p.edge_type, c.first_msg, NM, m, base + k * IPWAVE,
                               c.n_checks, q, m0 + m);
        if (store) st_c2v<W, CT>(p.c2v, ((int64_t)g * p.E12 + m0 + m) * W + w, out);
      }
    }
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      const int64_t le = l0 + l;
      const uint32_t neg_l = (neg >> (NM + l)) & 1u;
      const uint32_t neg_c = (tot ^ neg_l) & 1u;
      float wt = 1.0f;
      if (weighted)
        wt = edge_scale<W>(p.weights, p.wstride, p.it - 1, p.leaf_type, c.first_leaf, NL, l, base + k * IPWAVE,
                           c.n_checks, q, le);
      uint32_t bit;
      if (wt == 1.0f) {
        bit = leaf_bit(neg_l, neg_c, S[NM + l], A[NM + l]);
      } else {
        const float lr = p.Lraw[((int64_t)g * p.EL + le) * W + w];
        const float mag = phi(S[NM + l]);
        bit = (uint32_t)(lr + wt * (neg_c ? -mag : mag) < 0.0f);
      }
      if (post && store) {
        const float lr = p.Lraw[((int64_t)g * p.EL + le) * W + w];
        const float mag = phi(S[NM + l]);
        p.P1[((int64_t)g * p.EL + le) * W + w] = lr + wt * (neg_c ? -mag : mag);
      }
      const uint64_t ball = __ballot((int)(bit & (uint32_t)valid[k]));
      if (w == 0 && valid[k]) store_leaf_word<W>(p.B1out + (int64_t)g * p.EL + le, ball, q, act);
    }
  }
  if (test) {
    const uint64_t f = fold<W>(__ballot((int)bad));
    if (lane == 0) flag_unsat(p.unsat + g, f);
  }
}

template <int W, int NM, int NL, int MODE, int IPW, typename CT = float>
__global__ __launch_bounds__(kBlock) void k_check_fixed(const CheckParams p, const ClassArgs c) {
  const GridTile t = MODE == M_SPECIAL ? GridTile{blockIdx.x, (int)blockIdx.y} : xcd_grid_tile();
  check_fixed_body<W, NM, NL, MODE, IPW, false, CT>(p, c, t.bx, t.g);
}

// Check update with run-time degrees (total degree <= MET_MAX_CHECK_DEGREE),
// for classes without a compiled shape.  One check per lane group.
template <int W, bool PERSIST, typename CT = float>
__device__ __forceinline__ void check_generic_body(const CheckParams &p, const ClassArgs &c, int64_t bx, int g) {
  constexpr int D = MET_MAX_CHECK_DEGREE;
  clear_next_unsat(p, bx, g);
  const uint64_t act = p.active[g];  // not written during check updates
  if (act == 0ull) return;
  const int lane = threadIdx.x & 63, wv = wave_id();
  const int w = lane % W, q = lane / W;
  const bool lane_act = (act >> w) & 1ull;
  const int64_t i = (bx * kWavesPerBlock + wv) * (64 / W) + q;
  if (W == 64 && i >= c.n_checks) return;
  const bool valid = i < c.n_checks;
  const int64_t j = c.first_check + (valid ? i : 0);
  const bool first = p.flags & F_FIRST, test = p.flags & F_TEST;
  const bool weighted = p.flags & F_WEIGHTED;
  const int64_t m0 = p.chk_msg_ptr[j], l0 = p.chk_leaf_ptr[j];
  const int nm = p.chk_msg_ptr[j + 1] - (int32_t)m0;
  const int nl = p.chk_leaf_ptr[j + 1] - (int32_t)l0;
  const uint32_t s = (uint32_t)(p.synw[(int64_t)g * p.M + j] >> w) & 1u;
  float A[D];
  uint32_t neg = 0, parity = s;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    A[k] = 0.0f;  // phi-domain identity: an absent input adds nothing
    if (k < nm) {
      const int64_t e = m0 + k;
      const float pv = p.Pin[((int64_t)g * p.N2 + p.edge_msgvn[e]) * W + w];
      const float cv = first ? 0.0f : ld_c2v<W, CT>(p.c2v_in, ((int64_t)g * p.E12 + e) * W + w);
      parity ^= (uint32_t)(pv < 0.0f);
      const float x = clamp_llr(pv - cv);
      A[k] = phi(fabsf(x));
      neg |= sign_bit(x) << k;
    } else if (k < nm + nl) {
      const int64_t le = l0 + (k - nm);
      const float f = p.Lphi[((int64_t)g * p.EL + le) * W + w];
      A[k] = fabsf(f);
      neg |= sign_bit(f) << k;
      if (test) parity ^= (uint32_t)(ld_word<PERSIST>(p.B1in, (int64_t)g * p.EL + le) >> w) & 1u;
    }
  }
  const uint32_t bad = test ? (parity & (uint32_t)(valid && lane_act)) : 0u;
  const uint32_t tot = (__popc(neg) & 1u) ^ s;
  float pre[D], suf[D];
  pre[0] = 0.0f;
#pragma unroll
  for (int k = 1; k < D; ++k) pre[k] = pre[k - 1] + A[k - 1];
  suf[D - 1] = 0.0f;
#pragma unroll
  for (int k = D - 2; k >= 0; --k) suf[k] = suf[k + 1] + A[k + 1];
  const bool store = valid && lane_act;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    if (k < nm) {
      const float mag = phi(pre[k] + suf[k]);
      float out = ((tot ^ (neg >> k)) & 1u) ? -mag : mag;
      if (weighted) out *= p.weights[(int64_t)p.edge_type[m0 + k] * p.wstride + (p.it - 1)];
      if (store) st_c2v<W, CT>(p.c2v, ((int64_t)g * p.E12 + m0 + k) * W + w, out);
    }
  }
  // Leaf decisions: ballots must be executed by every lane of the wave, so the
  // loop runs to the wave-wide maximum leaf count.
  int nl_max = valid ? nl : 0;
  for (int off = 32; off >= 1; off >>= 1) nl_max = max(nl_max, __shfl_xor(nl_max, off));
  for (int k = 0; k < nl_max; ++k) {
    const bool has = valid && k < nl;
    const int kk = nm + k;
    const int64_t le = l0 + (has ? k : 0);
    float S = 0.0f, Aleaf = 0.0f;
#pragma unroll
    for (int r = 0; r < D; ++r)
      if (r == kk) {
        S = pre[r] + suf[r];
        Aleaf = A[r];
      }
    const uint32_t neg_l = (neg >> (kk & 31)) & 1u;
    const uint32_t neg_c = (tot ^ neg_l) & 1u;
    uint32_t bit = 0;
    if (has) {
      float wt = 1.0f;
      if (weighted) wt = ldro(p.weights, (int64_t)ldro(p.leaf_type, le) * p.wstride + (p.it - 1));
      if (wt == 1.0f) {
        bit = leaf_bit(neg_l, neg_c, S, Aleaf);
      } else {
        const float lr = p.Lraw[((int64_t)g * p.EL + le) * W + w];
        const float mag = phi(S);
        bit = (uint32_t)(lr + wt * (neg_c ? -mag : mag) < 0.0f);
      }
      if ((p.flags & F_POST) && store) {
        const float lr = p.Lraw[((int64_t)g * p.EL + le) * W + w];
        const float mag = phi(S);
        p.P1[((int64_t)g * p.EL + le) * W + w] = lr + wt * (neg_c ? -mag : mag);
      }
    }
    const uint64_t ball = __ballot((int)bit);
    if (w == 0 && has) store_leaf_word<W>(p.B1out + (int64_t)g * p.EL + le, ball, q, act);
  }
  if (test) {
    const uint64_t f = fold<W>(__ballot((int)bad));
    if (lane == 0) flag_unsat(p.unsat + g, f);
  }
}

template <int W, typename CT = float>
__global__ __launch_bounds__(kBlock) void k_check_generic(const CheckParams p, const ClassArgs c) {
  const GridTile t = xcd_grid_tile();
  check_generic_body<W, false, CT>(p, c, t.bx, t.g);
}

// Syndrome test only (after the last iteration): parity of the hard decisions
// of P^l (message VNs) and of the stored leaf decisions against s.
struct TestParams {
  const int32_t *edge_msgvn, *chk_msg_ptr, *chk_leaf_ptr;
  int64_t M, N2, E12, EL;
  const float *P;
  const uint64_t *synw, *B1, *active;
  uint64_t *unsat;
};

template <int W>
__global__ __launch_bounds__(kBlock) void k_test(const TestParams p) {
  const int g = blockIdx.y;
  const uint64_t act = p.active[g];
  if (act == 0ull) return;
  const int lane = threadIdx.x & 63, w = lane % W, q = lane / W;
  const int64_t j = ((int64_t)blockIdx.x * kWavesPerBlock + wave_id()) * (64 / W) + q;
  uint32_t bad = 0;
  if (j < p.M) {
    uint32_t parity = (uint32_t)(p.synw[(int64_t)g * p.M + j] >> w) & 1u;
    for (int32_t e = p.chk_msg_ptr[j]; e < p.chk_msg_ptr[j + 1]; ++e)
      parity ^= (uint32_t)(p.P[((int64_t)g * p.N2 + p.edge_msgvn[e]) * W + w] < 0.0f);
    for (int32_t e = p.chk_leaf_ptr[j]; e < p.chk_leaf_ptr[j + 1]; ++e)
      parity ^= (uint32_t)(p.B1[(int64_t)g * p.EL + e] >> w) & 1u;
    bad = parity & (uint32_t)((act >> w) & 1ull);
  }
  const uint64_t f = fold<W>(__ballot((int)bad));
  if (lane == 0) flag_unsat(p.unsat + g, f);
}

struct VarParams {
  const int32_t *vn_ptr, *vn_edges;
  int64_t N2, E12;
  const float *L2;       // [G][N2][W]
  const float *c2v;      // [G][E12][W]
  float *P;              // [G][N2][W]
  uint64_t *active;      // [G]
  const uint64_t *unsat; // [G] test result of iteration it-1 (retire mode)
  int32_t *iters;
  uint8_t *converged;
  const int32_t *slot_frame;  // [G*W] frame held by each lane, -1 none (NULL: lane s holds frame s)
  int32_t it, retire, G;
};

// Frame held by lane w of group g.
template <int W>
__device__ __forceinline__ int lane_frame(const int32_t *slot_frame, int g, int w) {
  return slot_frame ? slot_frame[g * W + w] : g * W + w;
}

// Variable update: P_v = L_v + sum of c2v over v's message edges (gathered U
// at a time, summed in list order).
template <int W, int U, bool PERSIST, typename CT = float>
__device__ __forceinline__ void variable_body(const VarParams &p, int64_t bx, int g) {
  uint64_t act = ld_racy<PERSIST>(p.active, g);
  if (p.retire) {
    // Frames whose test of iteration it-1 passed stop here; their P stays at
    // iteration it-1.  Block (0,0) records the outcome for every group.
    if (bx == 0 && g == 0) {
      for (int gg = threadIdx.x; gg < p.G; gg += kBlock) {
        const uint64_t a = p.active[gg];  // only this block writes the mask
        const uint64_t u = p.unsat[gg];
        const uint64_t done = a & ~u;
        if (done) {
          for (int w = 0; w < W; ++w)
            if ((done >> w) & 1ull) {
              const int f = lane_frame<W>(p.slot_frame, gg, w);
              p.iters[f] = p.it - 1;
              p.converged[f] = 1;
            }
          p.active[gg] = a & u;
        }
      }
    }
    act &= p.unsat[g];
  }
  if (act == 0ull) return;
  const int lane = threadIdx.x & 63, wv = wave_id(), w = lane % W, q = lane / W;
  const bool lane_act = (act >> w) & 1ull;
  const int64_t i = (bx * kWavesPerBlock + wv) * (64 / W) + q;
  if (i >= p.N2) return;
  const int32_t e0 = ldro(p.vn_ptr, i), e1 = ldro(p.vn_ptr, i + 1);
  float P = p.L2[((int64_t)g * p.N2 + i) * W + w];
  const CT *c2v = reinterpret_cast<const CT *>(p.c2v) + (int64_t)g * p.E12 * W + w;
  int32_t e = e0;
  for (; e + U <= e1; e += U) {
    float a[U];
#pragma unroll
    for (int u = 0; u < U; ++u) a[u] = ld_msg<W, CT>(c2v + (int64_t)ldro(p.vn_edges, e + u) * W);
#pragma unroll
    for (int u = 0; u < U; ++u) P += a[u];
  }
  if (U > 8)
    for (; e + 8 <= e1; e += 8) {
      float a[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] = ld_msg<W, CT>(c2v + (int64_t)ldro(p.vn_edges, e + u) * W);
#pragma unroll
      for (int u = 0; u < 8; ++u) P += a[u];
    }
  for (; e < e1; ++e) P += ld_msg<W, CT>(c2v + (int64_t)ldro(p.vn_edges, e) * W);
  if (lane_act) p.P[((int64_t)g * p.N2 + i) * W + w] = P;
}

template <int W, int U, typename CT = float>
__global__ __launch_bounds__(kBlock) void k_variable(const VarParams p) {
  const GridTile t = xcd_grid_tile();
  variable_body<W, U, false, CT>(p, t.bx, t.g);
}

// ----------------------------------------------------------------------------
// Set-up and output kernels

struct InitParams {
  const float *llr;       // [B][N]
  const uint8_t *syn;     // [B][M]
  const int32_t *msg_vn_user, *leaf_vn;
  const int32_t *chk_pos;   // [M] check of the code (syndrome index) -> decoder check order
  int64_t N, M, N2, EL;
  int32_t B, G;
  float *Lt;              // [G][N][W] staging
  float *L2, *Lphi, *Lraw;
  uint64_t *synw, *active, *unsat;
  int32_t *iters;
  uint8_t *converged;
};

// llr [B][N] -> Lt [G][N][W] through an LDS tile of 64 VNs x W frames: reads
// are rows of 64 consecutive VNs, writes are W*64 consecutive floats.
template <int W>
__global__ __launch_bounds__(kBlock) void k_transpose(const InitParams p) {
  __shared__ float tile[W][65];
  const int g = blockIdx.y;
  const int64_t v0 = (int64_t)blockIdx.x * 64;
  for (int idx = threadIdx.x; idx < W * 64; idx += kBlock) {
    const int f = idx / 64, v = idx % 64;
    const int frame = g * W + f;
    tile[f][v] = (frame < p.B && v0 + v < p.N) ? p.llr[(int64_t)frame * p.N + v0 + v] : 0.0f;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < W * 64; idx += kBlock) {
    const int v = idx / W, f = idx % W;
    if (v0 + v < p.N) p.Lt[((int64_t)g * p.N + v0 + v) * W + f] = tile[f][v];
  }
}

template <int W>
__global__ __launch_bounds__(kBlock) void k_init_items(const InitParams p) {
  const int g = blockIdx.y;
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;  // item * W + w
  const int64_t item = idx / W;
  const int w = (int)(idx % W);
  if (item < p.N2) {
    p.L2[((int64_t)g * p.N2 + item) * W + w] = p.Lt[((int64_t)g * p.N + p.msg_vn_user[item]) * W + w];
  } else if (item < p.N2 + p.EL) {
    const int64_t le = item - p.N2;
    const float l = p.Lt[((int64_t)g * p.N + p.leaf_vn[le]) * W + w];
    // a leaf's variable-to-check message is its LLR, clamped like every input
    p.Lphi[((int64_t)g * p.EL + le) * W + w] = copysignf(phi(fabsf(clamp_llr(l))), l);
    if (p.Lraw) p.Lraw[((int64_t)g * p.EL + le) * W + w] = l;
  }
}

template <int W>
__global__ __launch_bounds__(kBlock) void k_pack_syndrome(const InitParams p) {
  const int g = blockIdx.y;
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j < p.M) {
    // j counts in the code's check order (the syndrome's, so that the frame
    // rows are read contiguously); the word goes to the decoder's position
    uint64_t word = 0;
    for (int w = 0; w < W; ++w) {
      const int f = g * W + w;
      if (f < p.B) word |= (uint64_t)(p.syn[(int64_t)f * p.M + j] & 1u) << w;
    }
    p.synw[(int64_t)g * p.M + p.chk_pos[j]] = word;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const int valid = min(W, p.B - g * W);
    p.active[g] = valid >= 64 ? ~0ull : ((1ull << valid) - 1ull);
    p.unsat[g] = 0ull;
    p.unsat[p.G + g] = 0ull;
    for (int w = 0; w < valid; ++w) {
      p.iters[g * W + w] = 0;
      p.converged[g * W + w] = 0;
    }
  }
}

struct FinalParams {
  const int32_t *vn_slot;
  int64_t N, N2, EL;
  int32_t B, max_iter;
  const float *P;               // [G][N2][W]
  const float *P1a, *P1b;       // leaf posteriors of even / odd iterations (or NULL)
  const uint64_t *B1a, *B1b;    // leaf decisions of even / odd iterations
  const uint64_t *active, *unsat_last;
  int32_t *iters;
  uint8_t *converged;
  uint8_t *bits;
  float *posterior;
  const int32_t *slot_frame;  // as in VarParams
  int32_t G;
  int32_t flush;  // k_finalize: write only frames that no longer run (lanes not in active)
};

// Outcome of frames still running after the last iteration.
template <int W>
__global__ void k_final_status(const FinalParams p) {
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < p.G * W; s += gridDim.x * blockDim.x) {
    const int g = s / W, w = s % W;
    const int f = lane_frame<W>(p.slot_frame, g, w);
    if (f >= 0 && f < p.B && ((p.active[g] >> w) & 1ull)) {
      p.iters[f] = p.max_iter;
      p.converged[f] = (uint8_t)!((p.unsat_last[g] >> w) & 1ull);
    }
  }
}

// Outputs in user order through an LDS tile of 64 VNs x W frames: reads are
// item rows of W frames, writes are runs of 64 consecutive VNs per frame.
template <int W>
__global__ __launch_bounds__(kBlock) void k_finalize(const FinalParams p) {
  __shared__ float val[64][W + 1];
  __shared__ uint8_t bit[64][W + 1];
  __shared__ uint8_t odd[W];
  __shared__ int32_t frame[W];
  const int g = blockIdx.y;
  const int64_t v0 = (int64_t)blockIdx.x * 64;
  bool any = false;
  if (threadIdx.x < W) {
    int f = lane_frame<W>(p.slot_frame, g, threadIdx.x);
    if (f >= p.B || (p.flush && ((p.active[g] >> threadIdx.x) & 1ull))) f = -1;
    frame[threadIdx.x] = f;
    odd[threadIdx.x] = f >= 0 ? (uint8_t)(p.iters[f] & 1) : 0;
    any = f >= 0;
  }
  if (!__syncthreads_or(any)) return;
  for (int idx = threadIdx.x; idx < W * 64; idx += kBlock) {
    const int v = idx / W, w = idx % W;
    float post = 0.0f;
    uint8_t b = 0;
    if (v0 + v < p.N) {
      const int32_t slot = p.vn_slot[v0 + v];
      if (slot >= 0) {
        post = p.P[((int64_t)g * p.N2 + slot) * W + w];
        b = post < 0.0f;
      } else {
        const int64_t le = -(int64_t)slot - 1;
        b = (uint8_t)(((odd[w] ? p.B1b : p.B1a)[(int64_t)g * p.EL + le] >> w) & 1ull);
        if (p.posterior) post = (odd[w] ? p.P1b : p.P1a)[((int64_t)g * p.EL + le) * W + w];
      }
    }
    val[v][w] = post;
    bit[v][w] = b;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < W * 64; idx += kBlock) {
    const int w = idx / 64, v = idx % 64;
    const int f = frame[w];
    if (f < 0 || v0 + v >= p.N) continue;
    p.bits[(int64_t)f * p.N + v0 + v] = bit[v][w];
    if (p.posterior) p.posterior[(int64_t)f * p.N + v0 + v] = val[v][w];
  }
}

__global__ __launch_bounds__(kBlock) void k_syndrome(const int32_t *all_vn, const int32_t *all_ptr, int64_t N,
                                                     int64_t M, const uint8_t *bits, uint8_t *syn) {
  const int f = blockIdx.y;
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= M) return;
  uint32_t s = 0;
  for (int32_t e = all_ptr[j]; e < all_ptr[j + 1]; ++e) s ^= bits[(int64_t)f * N + all_vn[e]] & 1u;
  syn[(int64_t)f * M + j] = (uint8_t)s;
}

// ----------------------------------------------------------------------------
// Host launch helpers

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Plan {
  int W = 64, G = 1;
  size_t off_c2v = 0, off_P = 0, off_L2 = 0, off_Lphi = 0, off_Lraw = 0, off_P1 = 0, off_synw = 0, off_B1 = 0,
         off_unsat = 0, off_active = 0, off_slot = 0, off_ctab = 0, off_flag = 0, total = 0;
  bool lraw = false, p1 = false;
};

// Compaction table (groups of 64 frames): the number of groups that receive
// frames, their indices, and for each such group the lane each of its 64
// lanes receives a frame from (source slot g * 64 + w, or -1).
inline size_t compact_table_bytes(int G) { return 256 + align256((size_t)G * 4) + (size_t)G * 64 * 4; }

// Frames per group: the smallest supported width that holds min(B, 64).
int choose_interleave(int B) {
  if (B <= 1) return 1;
  if (B <= 4) return 4;
  if (B <= 16) return 16;
  if (B <= 32) return 32;
  return 64;
}

Plan make_plan(const met_code *c, int B, bool post, bool weighted, int W, size_t c2v_bytes = sizeof(float)) {
  Plan pl;
  pl.W = W;
  pl.G = (B + W - 1) / W;
  const size_t GW = (size_t)pl.G * W;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align256(bytes);
    return at;
  };
  // c2v also serves as the staging area of the input transpose.
  pl.off_c2v = take(std::max<size_t>(GW * c->E12 * c2v_bytes, GW * c->N * sizeof(float)));
  pl.off_P = take(GW * c->N2 * sizeof(float));
  pl.off_L2 = take(GW * c->N2 * sizeof(float));
  pl.off_Lphi = take(GW * c->EL * sizeof(float));
  pl.lraw = post || weighted;
  pl.p1 = post;
  pl.off_Lraw = pl.lraw ? take(GW * c->EL * sizeof(float)) : 0;
  pl.off_P1 = pl.p1 ? take(2 * GW * c->EL * sizeof(float)) : 0;
  pl.off_synw = take((size_t)pl.G * c->M * sizeof(uint64_t));
  pl.off_B1 = take(2 * (size_t)pl.G * c->EL * sizeof(uint64_t));
  pl.off_unsat = take(2 * (size_t)pl.G * sizeof(uint64_t));
  pl.off_active = take((size_t)pl.G * sizeof(uint64_t));
  pl.off_slot = take(GW * sizeof(int32_t));
  pl.off_ctab = take(compact_table_bytes(pl.G));
  pl.off_flag = take(sizeof(uint32_t));
  pl.total = o;
  return pl;
}

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) return fail(MET_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

template <int W, int MODE, int IPW, typename CT = float>
void launch_fixed(int shape, unsigned blocks, int G, hipStream_t st, const CheckParams &p, const ClassArgs &c) {
  const dim3 grid(blocks, G), block(kBlock);
  switch (shape) {
    case 0: hipLaunchKernelGGL((k_check_fixed<W, 3, 1, MODE, IPW, CT>), grid, block, 0, st, p, c); break;
    case 1: hipLaunchKernelGGL((k_check_fixed<W, 2, 1, MODE, IPW, CT>), grid, block, 0, st, p, c); break;
    case 2: hipLaunchKernelGGL((k_check_fixed<W, 12, 0, MODE, IPW, CT>), grid, block, 0, st, p, c); break;
    case 3: hipLaunchKernelGGL((k_check_fixed<W, 11, 0, MODE, IPW, CT>), grid, block, 0, st, p, c); break;
    case 4: hipLaunchKernelGGL((k_check_fixed<W, 6, 0, MODE, IPW, CT>), grid, block, 0, st, p, c); break;
    case 5: hipLaunchKernelGGL((k_check_fixed<W, 5, 0, MODE, IPW, CT>), grid, block, 0, st, p, c); break;
    default: hipLaunchKernelGGL((k_check_fixed<W, 4, 0, MODE, IPW, CT>), grid, block, 0, st, p, c); break;
  }
}

template <int W, int MODE>
void launch_fixed_ipw(int ipw, int shape, unsigned blocks, int G, hipStream_t st, const CheckParams &p,
                      const ClassArgs &c) {
  if (W == 64 && ipw == 4)
    launch_fixed<W, MODE, (W == 64 ? 4 : 1)>(shape, blocks, G, st, p, c);
  else if (W == 64 && ipw == 2)
    launch_fixed<W, MODE, (W == 64 ? 2 : 1)>(shape, blocks, G, st, p, c);
  else
    launch_fixed<W, MODE, 1>(shape, blocks, G, st, p, c);
}

// One check-kernel launch over a class: compiled shape (mode, steps per wave)
// or the run-time-degree kernel.  Half-precision and 8-bit message storage are
// compiled for groups of 64 frames with 4 check steps per wave only.
template <int W, typename CT = float>
void launch_check(const CheckParams &p, const ClassArgs &a, int mode, int cn_ipw, int G, hipStream_t st) {
  constexpr bool half = !std::is_same<CT, float>::value;  // half or 8-bit storage
  static_assert(!half || W == 64, "reduced message storage needs groups of 64 frames");
  const bool gen = a.shape == kShapeGeneric;
  const int ipw = (W == 64 && !gen) ? (half ? 4 : cn_ipw) : 1;
  const int64_t per_block = (int64_t)kWavesPerBlock * ipw * (64 / W);
  const unsigned blocks = (unsigned)((a.n_checks + per_block - 1) / per_block);
  if (gen)
    hipLaunchKernelGGL((k_check_generic<W, CT>), dim3(blocks, G), dim3(kBlock), 0, st, p, a);
  else if (half && mode == M_SPECIAL)
    launch_fixed<W, M_SPECIAL, 4, CT>(a.shape, blocks, G, st, p, a);
  else if (half && mode == M_FIRST)
    launch_fixed<W, M_FIRST, 4, CT>(a.shape, blocks, G, st, p, a);
  else if (half)
    launch_fixed<W, M_MAIN, 4, CT>(a.shape, blocks, G, st, p, a);
  else if (mode == M_SPECIAL)
    launch_fixed_ipw<W, M_SPECIAL>(ipw, a.shape, blocks, G, st, p, a);
  else if (mode == M_FIRST)
    launch_fixed_ipw<W, M_FIRST>(ipw, a.shape, blocks, G, st, p, a);
  else
    launch_fixed_ipw<W, M_MAIN>(ipw, a.shape, blocks, G, st, p, a);
}

inline std::vector<ClassArgs> class_args(const met_code *c) {
  std::vector<ClassArgs> out;
  for (const CheckClass &cc : c->classes) {
    ClassArgs a{};
    a.shape = cc.shape;
    a.n_msg = cc.n_msg;
    a.n_leaf = cc.n_leaf;
    a.first_check = cc.first_check;
    a.n_checks = cc.n_checks;
    a.first_msg = cc.first_msg;
    a.first_leaf = cc.first_leaf;
    out.push_back(a);
  }
  return out;
}

// Timer names of the check kernels, by shape.
const char *const kCheckKernelName[kNumFixedShapes + 1] = {
    "k_check<3,1>", "k_check<2,1>", "k_check<12,0>", "k_check<11,0>", "k_check<6,0>", "k_check<5,0>",
    "k_check<4,0>", "k_check_generic"};
static_assert(kShapeMsg[0] == 3 && kShapeLeaf[0] == 1 && kShapeMsg[2] == 12 && kShapeMsg[5] == 5 &&
                  kShapeMsg[6] == 4 && kNumFixedShapes == 7,
              "timer names and kernel switches follow the shape table");

}  // namespace
}  // namespace met
