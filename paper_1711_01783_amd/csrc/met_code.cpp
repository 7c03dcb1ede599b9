// Host side of the decoder library: code construction, derived adjacency,
// bookkeeping and error reporting.  No HIP calls here; everything in this file
// runs without a GPU.
//
// Construction (the paper builds its matrices by progressive edge growth from
// degree distributions that are not published with it; Methods, first
// paragraph).  This project fixes a seeded construction instead:
//   1. VN counts: every VN type but the last gets floor(frac * N + 1e-6) nodes,
//      the last the remainder; nodes are numbered type by type.
//   2. VN sockets per edge type t: S_t = sum over VN types of count * degree.
//   3. Check counts: each edge type belongs to exactly one check type; a check
//      type's anchor is its edge type of smallest non-zero degree d (lowest
//      index on ties) and its count is round-half-up(S_anchor / d).
//   4. Socket balance: the excess m*d - S_t of every (check type, edge type)
//      is spread as -1 / +1 degree over the first checks of that type.
//   5. Per edge type t a SplitMix64 stream (Steele, Lea, Flood 2014) with
//      state0 = mix(seed ^ mix(t + 1)); uniform(n) = (next() * n) >> 64.
//   6. Sockets in node order; the check-socket list is shuffled by Fisher-Yates
//      (i = n-1 .. 1, j = uniform(i + 1)); edge i joins VN socket i and check
//      socket i.
//   7. Multi-edge repair: for each type, for each edge in socket order whose
//      (VN, check) pair occurs more than once, draw j = uniform(E_t) and swap
//      the check ends of i and j when j != i and neither new pair exists yet.
//   8. Edges are sorted by (check, type, VN).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <set>
#include <unordered_map>

#include "met_internal.h"

namespace met {

static thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

void clear_error() { g_last_error.clear(); }

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct SplitMix64 {
  uint64_t state;
  explicit SplitMix64(uint64_t s) : state(s) {}
  uint64_t next() {
    state += kGamma;
    return mix64(state);
  }
  // Multiply-shift reduction to [0, n).
  uint64_t uniform(uint64_t n) {
    unsigned __int128 p = (unsigned __int128)next() * n;
    return (uint64_t)(p >> 64);
  }
};

constexpr long kMaxRepairDraws = 100000;

// Multiplicity of (VN, check) keys: a sorted base plus an overlay of changes.
struct PairCounts {
  std::vector<int64_t> keys;
  std::vector<int32_t> counts;
  std::unordered_map<int64_t, int32_t> delta;
  int32_t get(int64_t k) const {
    auto it = delta.find(k);
    if (it != delta.end()) return it->second;
    auto p = std::lower_bound(keys.begin(), keys.end(), k);
    if (p != keys.end() && *p == k) return counts[p - keys.begin()];
    return 0;
  }
  void set(int64_t k, int32_t v) { delta[k] = v; }
};

}  // namespace

// Derived structures for the decoder: message/leaf split, VN edge lists,
// check classes.
int finalize_code(met_code *c, bool skip_deg1) {
  const int64_t N = c->N, M = c->M, E = c->E;
  std::vector<int32_t> deg(N, 0);
  for (int64_t e = 0; e < E; ++e) deg[c->vn[e]]++;
  // leaf edges: edges to degree-1 variable nodes, when those stay out of the
  // iterations
  auto is_leaf = [&](int32_t v) { return skip_deg1 && deg[v] == 1; };
  c->chk_ptr.assign(M + 1, 0);
  for (int64_t e = 0; e < E; ++e) c->chk_ptr[c->cn[e] + 1]++;
  for (int64_t j = 0; j < M; ++j) c->chk_ptr[j + 1] += c->chk_ptr[j];
  c->max_vn_deg = 0;
  c->n_deg1 = 0;
  c->msg_vn_user.clear();
  c->vn_slot.assign(N, 0);
  std::vector<int32_t> msg_index(N, -1);
  for (int64_t v = 0; v < N; ++v) {
    c->max_vn_deg = std::max(c->max_vn_deg, deg[v]);
    if (deg[v] == 1) c->n_deg1++;
    if (!is_leaf((int32_t)v)) {
      msg_index[v] = (int32_t)c->msg_vn_user.size();
      c->msg_vn_user.push_back((int32_t)v);
    }
  }
  c->N2 = (int64_t)c->msg_vn_user.size();
  c->edge_msgvn.clear();
  c->edge_type_msg.clear();
  c->leaf_vn_user.clear();
  c->leaf_type.clear();
  c->chk_msg_ptr.assign(M + 1, 0);
  c->chk_leaf_ptr.assign(M + 1, 0);
  c->max_check_deg = 0;
  // Decoder order of the checks: within each run of checks of one shape
  // (message and leaf edge counts), checks sorted by their smallest, then
  // largest, message VN, so that checks sharing a VN are processed together
  // and its posterior row is gathered once from HBM for several of them.
  // Only the order of independent check updates changes.
  std::vector<int32_t> nmsg(M), key_lo(M), key_hi(M);
  for (int64_t j = 0; j < M; ++j) {
    const int32_t d = c->chk_ptr[j + 1] - c->chk_ptr[j];
    if (d < 2 || d > MET_MAX_CHECK_DEGREE)
      return fail(MET_EINVAL, "check %lld has degree %d (allowed 2..%d)", (long long)j, d,
                  MET_MAX_CHECK_DEGREE);
    int32_t nm = 0, lo = INT32_MAX, hi = -1;
    for (int32_t e = c->chk_ptr[j]; e < c->chk_ptr[j + 1]; ++e)
      if (!is_leaf(c->vn[e])) {
        ++nm;
        lo = std::min(lo, msg_index[c->vn[e]]);
        hi = std::max(hi, msg_index[c->vn[e]]);
      }
    nmsg[j] = nm;
    key_lo[j] = lo;
    key_hi[j] = hi;
  }
  c->chk_orig.resize(M);
  for (int64_t j = 0; j < M; ++j) c->chk_orig[j] = (int32_t)j;
  for (int64_t a = 0; a < M;) {
    const int32_t nm = nmsg[a], nl = (c->chk_ptr[a + 1] - c->chk_ptr[a]) - nm;
    int64_t b = a + 1;
    while (b < M && nmsg[b] == nm && (c->chk_ptr[b + 1] - c->chk_ptr[b]) - nmsg[b] == nl) ++b;
    std::stable_sort(c->chk_orig.begin() + a, c->chk_orig.begin() + b, [&](int32_t x, int32_t y) {
      return key_lo[x] != key_lo[y] ? key_lo[x] < key_lo[y] : key_hi[x] < key_hi[y];
    });
    a = b;
  }
  c->chk_pos.resize(M);
  for (int64_t jj = 0; jj < M; ++jj) c->chk_pos[c->chk_orig[jj]] = (int32_t)jj;
  for (int64_t jj = 0; jj < M; ++jj) {
    const int64_t j = c->chk_orig[jj];
    const int32_t d = c->chk_ptr[j + 1] - c->chk_ptr[j];
    c->max_check_deg = std::max(c->max_check_deg, d);
    for (int32_t e = c->chk_ptr[j]; e < c->chk_ptr[j + 1]; ++e) {
      const int32_t v = c->vn[e];
      if (is_leaf(v)) {
        c->vn_slot[v] = -(int32_t)c->leaf_vn_user.size() - 1;
        c->leaf_vn_user.push_back(v);
        c->leaf_type.push_back(c->et[e]);
      } else {
        c->edge_msgvn.push_back(msg_index[v]);
        c->edge_type_msg.push_back(c->et[e]);
      }
    }
    c->chk_msg_ptr[jj + 1] = (int32_t)c->edge_msgvn.size();
    c->chk_leaf_ptr[jj + 1] = (int32_t)c->leaf_vn_user.size();
  }
  for (int64_t i = 0; i < c->N2; ++i) c->vn_slot[c->msg_vn_user[i]] = (int32_t)i;
  c->E12 = (int64_t)c->edge_msgvn.size();
  c->EL = (int64_t)c->leaf_vn_user.size();
  // VN-ordered lists of message-edge positions (increasing check order).
  c->vn_ptr.assign(c->N2 + 1, 0);
  for (int64_t e = 0; e < c->E12; ++e) c->vn_ptr[c->edge_msgvn[e] + 1]++;
  for (int64_t i = 0; i < c->N2; ++i) c->vn_ptr[i + 1] += c->vn_ptr[i];
  c->vn_edges.assign(c->E12, 0);
  {
    std::vector<int32_t> fill(c->vn_ptr.begin(), c->vn_ptr.end() - 1);
    for (int64_t e = 0; e < c->E12; ++e) c->vn_edges[fill[c->edge_msgvn[e]]++] = (int32_t)e;
  }
  // Check classes: runs of equal (message, leaf) shape.
  struct Run {
    int32_t nm, nl;
    int64_t first, count;
  };
  std::vector<Run> runs;
  for (int64_t j = 0; j < M; ++j) {
    const int32_t nm = c->chk_msg_ptr[j + 1] - c->chk_msg_ptr[j];
    const int32_t nl = c->chk_leaf_ptr[j + 1] - c->chk_leaf_ptr[j];
    if (!runs.empty() && runs.back().nm == nm && runs.back().nl == nl)
      runs.back().count++;
    else
      runs.push_back({nm, nl, j, 1});
  }
  auto shape_of = [](int32_t nm, int32_t nl) {
    for (int s = 0; s < kNumFixedShapes; ++s)
      if (kShapeMsg[s] == nm && kShapeLeaf[s] == nl) return s;
    return kShapeGeneric;
  };
  auto build_classes = [&](int64_t min_fixed) {
    std::vector<CheckClass> out;
    for (const Run &r : runs) {
      int s = shape_of(r.nm, r.nl);
      if (r.count < min_fixed) s = kShapeGeneric;
      if (s == kShapeGeneric && !out.empty() && out.back().shape == kShapeGeneric) {
        out.back().n_checks += r.count;
        continue;
      }
      CheckClass k;
      k.shape = s;
      k.n_msg = s == kShapeGeneric ? 0 : r.nm;
      k.n_leaf = s == kShapeGeneric ? 0 : r.nl;
      k.first_check = r.first;
      k.n_checks = r.count;
      k.first_msg = c->chk_msg_ptr[r.first];
      k.first_leaf = c->chk_leaf_ptr[r.first];
      out.push_back(k);
    }
    return out;
  };
  c->classes = build_classes(1);
  for (int64_t thr = 2; (int)c->classes.size() > kMaxClasses && thr <= (int64_t)1 << 40; thr *= 4)
    c->classes = build_classes(thr);
  if ((int)c->classes.size() > kMaxClasses) return fail(MET_EINVAL, "too many check classes");
  return MET_OK;
}

}  // namespace met

using met::fail;

static std::atomic<uint64_t> g_next_uid{0};

extern "C" const char *met_last_error(void) { return met::g_last_error.c_str(); }

int met::all_vns_view(const met_code *cc, const met_code **out) {
  met_code *c = const_cast<met_code *>(cc);
  std::lock_guard<std::mutex> lock(c->mu);
  if (!c->all_vns) {
    met_code *v = new (std::nothrow) met_code;
    if (!v) return fail(MET_ENOMEM, "out of host memory");
    v->N = c->N;
    v->M = c->M;
    v->E = c->E;
    v->ntypes = c->ntypes;
    v->vn = c->vn;
    v->cn = c->cn;
    v->et = c->et;
    const int rc = finalize_code(v, false);
    if (rc) {
      delete v;
      return rc;
    }
    v->uid = ++g_next_uid;
    c->all_vns = v;
  }
  *out = c->all_vns;
  return MET_OK;
}

static int sort_and_finalize(met_code *c, std::vector<int32_t> &v, std::vector<int32_t> &ch,
                             std::vector<int8_t> &t) {
  const int64_t E = (int64_t)v.size();
  std::vector<int64_t> key(E);
  std::vector<int32_t> idx(E);
  const int64_t nt = 8;
  for (int64_t e = 0; e < E; ++e) {
    key[e] = ((int64_t)ch[e] * nt + t[e]) * c->N + v[e];
    idx[e] = (int32_t)e;
  }
  std::sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
  c->vn.resize(E);
  c->cn.resize(E);
  c->et.resize(E);
  for (int64_t k = 0; k < E; ++k) {
    c->vn[k] = v[idx[k]];
    c->cn[k] = ch[idx[k]];
    c->et[k] = t[idx[k]];
  }
  c->E = E;
  return met::finalize_code(c);
}

// Steps 1-4, shared by both constructions: validated profile -> node counts,
// node type of every VN, check count and the balanced per-check socket
// counts cdeg[j * T + t].
struct Sockets {
  int T = 0, VT = 0;
  int64_t M = 0;
  std::vector<int64_t> vcount, S;
  std::vector<int32_t> cdeg, vtype;
};

static int prepare_sockets(const met_profile *p, int64_t N, Sockets &sk) {
  const int T = p->n_edge_types;
  if (T < 1 || T > MET_MAX_EDGE_TYPES) return fail(MET_EINVAL, "n_edge_types %d outside 1..%d", T, MET_MAX_EDGE_TYPES);
  if (p->n_vn_types < 1 || p->n_cn_types < 1 || !p->vn_frac || !p->vn_deg || !p->cn_frac || !p->cn_deg)
    return fail(MET_EINVAL, "profile has no node types");
  if (N < 2 || N > ((int64_t)1 << 30)) return fail(MET_EINVAL, "N = %lld outside 2..2^30", (long long)N);
  const int VT = p->n_vn_types, CT = p->n_cn_types;
  for (int k = 0; k < VT * T; ++k)
    if (p->vn_deg[k] < 0 || p->vn_deg[k] > MET_MAX_VN_DEGREE)
      return fail(MET_EINVAL, "VN degree %d outside 0..%d", p->vn_deg[k], MET_MAX_VN_DEGREE);
  for (int k = 0; k < CT * T; ++k)
    if (p->cn_deg[k] < 0) return fail(MET_EINVAL, "negative check degree");
  // 1. VN counts
  std::vector<int64_t> vcount(VT);
  int64_t used = 0;
  for (int k = 0; k < VT; ++k) {
    if (k < VT - 1) {
      const double f = p->vn_frac[k];
      if (!(f >= 0.0 && f <= 1.0)) return fail(MET_EINVAL, "vn_frac[%d] outside [0,1]", k);
      vcount[k] = (int64_t)std::floor(f * (double)N + 1e-6);
    } else {
      vcount[k] = N - used;
    }
    used += vcount[k];
  }
  if (vcount[VT - 1] < 0) return fail(MET_EINVAL, "VN fractions exceed 1");
  for (int k = 0; k < VT; ++k) {
    int dsum = 0;
    for (int t = 0; t < T; ++t) dsum += p->vn_deg[k * T + t];
    if (vcount[k] > 0 && dsum < 1) return fail(MET_EINVAL, "VN type %d has degree 0", k);
  }
  // 2. sockets per type; every edge position is an int32 index
  std::vector<int64_t> S(T, 0);
  int64_t E_total = 0;
  for (int t = 0; t < T; ++t) {
    for (int k = 0; k < VT; ++k) S[t] += vcount[k] * p->vn_deg[k * T + t];
    E_total += S[t];
  }
  if (E_total > (int64_t)INT32_MAX)
    return fail(MET_EINVAL, "%lld edges exceed the int32 edge index", (long long)E_total);
  // 3. check counts
  std::vector<int> owner(T, -1);
  for (int k = 0; k < CT; ++k)
    for (int t = 0; t < T; ++t)
      if (p->cn_deg[k * T + t] > 0) {
        if (owner[t] != -1) return fail(MET_EINVAL, "edge type %d belongs to two check types", t);
        owner[t] = k;
      }
  for (int t = 0; t < T; ++t)
    if (S[t] > 0 && owner[t] == -1) return fail(MET_EINVAL, "edge type %d has no check type", t);
  std::vector<int64_t> ccount(CT, 0);
  for (int k = 0; k < CT; ++k) {
    int anchor = -1;
    for (int t = 0; t < T; ++t) {
      const int d = p->cn_deg[k * T + t];
      if (d > 0 && (anchor < 0 || d < p->cn_deg[k * T + anchor])) anchor = t;
    }
    if (anchor < 0) return fail(MET_EINVAL, "check type %d has no edges", k);
    const int64_t d = p->cn_deg[k * T + anchor];
    ccount[k] = (2 * S[anchor] + d) / (2 * d);
    const double expect = p->cn_frac[k] * (double)N;
    if (std::fabs((double)ccount[k] - expect) > 0.01 * (double)N + 2.0)
      return fail(MET_EINVAL, "check type %d: %lld checks from socket balance, cn_frac implies %.1f", k,
                  (long long)ccount[k], expect);
  }
  int64_t M = 0;
  for (int k = 0; k < CT; ++k) M += ccount[k];
  // 4. per-check degrees with balancing
  std::vector<int32_t> cdeg((size_t)M * T);
  {
    int64_t j0 = 0;
    for (int k = 0; k < CT; ++k) {
      for (int64_t j = 0; j < ccount[k]; ++j)
        for (int t = 0; t < T; ++t) cdeg[(j0 + j) * T + t] = p->cn_deg[k * T + t];
      for (int t = 0; t < T; ++t) {
        const int64_t d = p->cn_deg[k * T + t];
        if (d == 0) continue;
        const int64_t excess = ccount[k] * d - S[t];
        if (std::llabs(excess) > ccount[k]) return fail(MET_EINVAL, "cannot balance sockets of edge type %d", t);
        for (int64_t j = 0; j < std::llabs(excess); ++j) cdeg[(j0 + j) * T + t] += excess > 0 ? -1 : 1;
      }
      j0 += ccount[k];
    }
  }
  for (int64_t j = 0; j < M; ++j) {
    int dsum = 0;
    for (int t = 0; t < T; ++t) dsum += cdeg[j * T + t];
    if (dsum < 2 || dsum > MET_MAX_CHECK_DEGREE)
      return fail(MET_EINVAL, "check %lld would have degree %d (allowed 2..%d)", (long long)j, dsum,
                  MET_MAX_CHECK_DEGREE);
  }
  std::vector<int32_t> vtype(N);
  {
    int64_t v = 0;
    for (int k = 0; k < VT; ++k)
      for (int64_t i = 0; i < vcount[k]; ++i) vtype[v++] = k;
  }
  sk.T = T;
  sk.VT = VT;
  sk.M = M;
  sk.vcount = std::move(vcount);
  sk.S = std::move(S);
  sk.cdeg = std::move(cdeg);
  sk.vtype = std::move(vtype);
  return MET_OK;
}

extern "C" int met_code_build(const met_profile *p, int64_t N, uint64_t seed, met_code **out) { return met::guarded("met_code_build", [&]() -> int {
  met::clear_error();
  if (!p || !out) return fail(MET_EINVAL, "met_code_build: NULL argument");
  *out = nullptr;
  Sockets sk;
  int rc0 = prepare_sockets(p, N, sk);
  if (rc0) return rc0;
  const int T = sk.T;
  const int64_t M = sk.M;
  const std::vector<int64_t> &S = sk.S;
  const std::vector<int32_t> &cdeg = sk.cdeg, &vtype = sk.vtype;
  // 5-6. sockets and shuffles
  std::vector<std::vector<int32_t>> vs(T), cs(T);
  std::vector<met::SplitMix64> rng;
  for (int t = 0; t < T; ++t) {
    rng.emplace_back(met::mix64(seed ^ met::mix64((uint64_t)t + 1)));
    vs[t].reserve(S[t]);
    cs[t].reserve(S[t]);
    for (int64_t v = 0; v < N; ++v)
      for (int r = 0; r < p->vn_deg[vtype[v] * T + t]; ++r) vs[t].push_back((int32_t)v);
    for (int64_t j = 0; j < M; ++j)
      for (int r = 0; r < cdeg[j * T + t]; ++r) cs[t].push_back((int32_t)j);
    if (vs[t].size() != cs[t].size()) return fail(MET_EINVAL, "socket mismatch on edge type %d", t);
    auto &c = cs[t];
    for (int64_t i = (int64_t)c.size() - 1; i >= 1; --i) {
      const int64_t j = (int64_t)rng[t].uniform((uint64_t)(i + 1));
      std::swap(c[i], c[j]);
    }
  }
  // 7. multi-edge repair
  {
    met::PairCounts pc;
    std::vector<int64_t> all;
    for (int t = 0; t < T; ++t)
      for (size_t i = 0; i < vs[t].size(); ++i) all.push_back((int64_t)vs[t][i] * M + cs[t][i]);
    std::sort(all.begin(), all.end());
    bool any_dup = false;
    for (size_t i = 0; i < all.size();) {
      size_t k = i;
      while (k < all.size() && all[k] == all[i]) ++k;
      pc.keys.push_back(all[i]);
      pc.counts.push_back((int32_t)(k - i));
      if (k - i > 1) any_dup = true;
      i = k;
    }
    if (any_dup) {
      for (int t = 0; t < T; ++t) {
        auto &v = vs[t];
        auto &c = cs[t];
        const int64_t Et = (int64_t)v.size();
        std::vector<int64_t> cand;
        for (int64_t i = 0; i < Et; ++i)
          if (pc.get((int64_t)v[i] * M + c[i]) > 1) cand.push_back(i);
        for (int64_t i : cand) {
          long draws = 0;
          for (;;) {
            const int64_t ki = (int64_t)v[i] * M + c[i];
            if (pc.get(ki) <= 1) break;
            if (++draws > met::kMaxRepairDraws) return fail(MET_EINVAL, "multi-edge repair failed");
            const int64_t j = (int64_t)rng[t].uniform((uint64_t)Et);
            if (j == i) continue;
            const int64_t a = (int64_t)v[i] * M + c[j];
            const int64_t b = (int64_t)v[j] * M + c[i];
            if (pc.get(a) != 0 || pc.get(b) != 0) continue;
            const int64_t kj = (int64_t)v[j] * M + c[j];
            pc.set(ki, pc.get(ki) - 1);
            pc.set(kj, pc.get(kj) - 1);
            std::swap(c[i], c[j]);
            pc.set(a, 1);
            pc.set(b, 1);
          }
        }
      }
    }
  }
  met_code *code = new (std::nothrow) met_code();
  if (code) code->uid = g_next_uid.fetch_add(1) + 1;
  if (!code) return fail(MET_ENOMEM, "out of host memory");
  code->N = N;
  code->M = M;
  code->ntypes = T;
  std::vector<int32_t> v, ch;
  std::vector<int8_t> t;
  for (int tt = 0; tt < T; ++tt) {
    v.insert(v.end(), vs[tt].begin(), vs[tt].end());
    ch.insert(ch.end(), cs[tt].begin(), cs[tt].end());
    t.insert(t.end(), vs[tt].size(), (int8_t)tt);
  }
  int rc = sort_and_finalize(code, v, ch, t);
  if (rc != MET_OK) {
    delete code;
    return rc;
  }
  *out = code;
  return MET_OK;
  });
}

// Progressive edge growth (Methods, first paragraph: the paper builds its
// matrices this way).  Edges are placed one at a time, node by node (v =
// 0..N-1) and within a node edge type by edge type; each goes to a check as
// far from its node as the type-t graph built so far allows:
//   * a breadth-first search from v over the type-t edges placed so far gives
//     check layers C_1 (v's type-t checks), C_2, ..., at most depth[t] of them,
//     stopping at the first empty layer;
//   * candidates are the checks with a free type-t socket that are not yet
//     neighbours of v; for k = (number of layers) down to 1 the candidates
//     outside C_1..C_k are taken, and the first k that leaves any decides;
//   * among them the ones with the fewest type-t edges form the tie set, and
//     the edge goes to its r-th check in check order, r = uniform(size) from
//     the SplitMix64 stream numbered T (after the T streams of the random
//     construction), one draw per edge.
// An edge to a check of layer C_k would close a cycle of length 2k, so the
// rule keeps cycles of length <= 2 depth[t] out of the type-t graph wherever
// free sockets allow.  Default depths: with d_v, d_c the largest type-t
// degrees, layer k of a full graph holds about (d_v - 1) g^(k-1) checks,
// g = (d_v - 1)(d_c - 1); the depth is 1 if g = 0 (edges of degree-1 nodes
// close no cycle), else the largest K <= 16 with (d_v - 1) g^(K-1) <= 1024.
//
// Tie sets are found with one Fenwick tree per (edge type, fill level) over
// the checks owning that type (counts, rank and select in O(log M)); the few
// checks a search excludes are skipped by rank.
namespace met {
namespace {

constexpr int kPegMaxDepth = 16;

int peg_default_depth(const met_profile *p, int t) {
  const int T = p->n_edge_types;
  int64_t dv = 0, dc = 0;
  for (int k = 0; k < p->n_vn_types; ++k) dv = std::max<int64_t>(dv, p->vn_deg[k * T + t]);
  for (int k = 0; k < p->n_cn_types; ++k) dc = std::max<int64_t>(dc, p->cn_deg[k * T + t]);
  const int64_t g = std::max<int64_t>(dv - 1, 0) * std::max<int64_t>(dc - 1, 0);
  if (g == 0) return 1;
  int K = 1;
  int64_t layer = (dv - 1) * g;  // size of layer K + 1
  while (K < kPegMaxDepth && layer <= 1024) {
    ++K;
    layer *= g;
  }
  return K;
}

// Membership counts over positions 0..n-1.
struct Fenwick {
  std::vector<int32_t> a;
  int32_t total = 0;
  explicit Fenwick(int64_t n = 0) : a(n + 1, 0) {}
  void add(int64_t i, int32_t d) {
    total += d;
    for (++i; i < (int64_t)a.size(); i += i & -i) a[i] += d;
  }
  int32_t prefix(int64_t i) const {  // members at positions < i
    int32_t s = 0;
    for (; i > 0; i -= i & -i) s += a[i];
    return s;
  }
  int64_t select(int32_t k) const {  // position of the k-th member (0-based)
    int64_t pos = 0;
    int64_t step = 1;
    while (step * 2 < (int64_t)a.size()) step *= 2;
    for (; step > 0; step /= 2)
      if (pos + step < (int64_t)a.size() && a[pos + step] <= k) {
        pos += step;
        k -= a[pos];
      }
    return pos;  // 0-based position
  }
};

}  // namespace
}  // namespace met

extern "C" int met_code_build_peg(const met_profile *p, int64_t N, uint64_t seed, const int32_t *depth,
                                  met_code **out) { return met::guarded("met_code_build_peg", [&]() -> int {
  met::clear_error();
  if (!p || !out) return fail(MET_EINVAL, "met_code_build_peg: NULL argument");
  *out = nullptr;
  Sockets sk;
  int rc0 = prepare_sockets(p, N, sk);
  if (rc0) return rc0;
  const int T = sk.T;
  const int64_t M = sk.M;
  const std::vector<int32_t> &cdeg = sk.cdeg, &vtype = sk.vtype;
  std::vector<int> K(T);
  for (int t = 0; t < T; ++t) {
    K[t] = depth ? depth[t] : met::peg_default_depth(p, t);
    if (K[t] < 1 || K[t] > met::kPegMaxDepth)
      return fail(MET_EINVAL, "depth[%d] = %d outside 1..%d", t, K[t], met::kPegMaxDepth);
  }
  met::SplitMix64 rng(met::mix64(seed ^ met::mix64((uint64_t)T + 1)));
  // checks owning each type: one contiguous run (checks are numbered type by
  // type and every edge type belongs to one check type)
  std::vector<int64_t> own0(T, 0), own_n(T, 0);
  for (int t = 0; t < T; ++t) {
    int64_t lo = -1, hi = -1;
    for (int64_t j = 0; j < M; ++j)
      if (cdeg[j * T + t] > 0) {
        if (lo < 0) lo = j;
        if (hi >= 0 && hi != j - 1) return fail(MET_EINVAL, "checks of edge type %d are not contiguous", t);
        hi = j;
      }
    own0[t] = lo < 0 ? 0 : lo;
    own_n[t] = lo < 0 ? 0 : hi - lo + 1;
  }
  // type-t adjacency as it grows: flat lists with known capacities
  std::vector<std::vector<int64_t>> vptr(T), cptr(T);
  std::vector<std::vector<int32_t>> vlist(T), clist(T), vfill(T), cfill(T);
  std::vector<int> max_cdeg(T, 0);
  for (int t = 0; t < T; ++t) {
    vptr[t].assign(N + 1, 0);
    cptr[t].assign(M + 1, 0);
    for (int64_t v = 0; v < N; ++v) vptr[t][v + 1] = vptr[t][v] + p->vn_deg[vtype[v] * T + t];
    for (int64_t j = 0; j < M; ++j) {
      cptr[t][j + 1] = cptr[t][j] + cdeg[j * T + t];
      max_cdeg[t] = std::max(max_cdeg[t], cdeg[j * T + t]);
    }
    vlist[t].assign(vptr[t][N], 0);
    clist[t].assign(cptr[t][M], 0);
    vfill[t].assign(N, 0);
    cfill[t].assign(M, 0);
  }
  // free checks of each type by fill level (positions within the owner run)
  std::vector<std::vector<met::Fenwick>> level(T);
  for (int t = 0; t < T; ++t) {
    level[t].assign(max_cdeg[t], met::Fenwick(own_n[t]));
    for (int64_t i = 0; i < own_n[t]; ++i) level[t][0].add(i, 1);
  }
  // stamps: search marks per edge, neighbour marks per node
  std::vector<int64_t> cstamp(M, -1), vstamp(N, -1), nstamp(M, -1);
  std::vector<int32_t> clayer(M, 0), frontier, nodes, next, visited, skip;
  std::vector<int32_t> ev, ec;
  std::vector<int8_t> et;
  const int64_t E_total = std::accumulate(sk.S.begin(), sk.S.end(), (int64_t)0);
  ev.reserve(E_total);
  ec.reserve(E_total);
  et.reserve(E_total);
  int64_t stamp = 0;
  for (int64_t v = 0; v < N; ++v) {
    for (int t = 0; t < T; ++t) {
      const int dv = p->vn_deg[vtype[v] * T + t];
      for (int r = 0; r < dv; ++r, ++stamp) {
        // neighbours of v (every type): never a candidate
        visited.clear();
        for (int tt = 0; tt < T; ++tt)
          for (int64_t i = vptr[tt][v]; i < vptr[tt][v] + vfill[tt][v]; ++i) {
            nstamp[vlist[tt][i]] = stamp;
            visited.push_back(vlist[tt][i]);
          }
        // layers of the search over type-t edges
        frontier.clear();
        for (int64_t i = vptr[t][v]; i < vptr[t][v] + vfill[t][v]; ++i) {
          const int32_t c = vlist[t][i];
          if (cstamp[c] != stamp) {
            cstamp[c] = stamp;
            clayer[c] = 1;
            frontier.push_back(c);
            visited.push_back(c);
          }
        }
        vstamp[v] = stamp;
        int layers = 1;
        while (layers < K[t]) {
          nodes.clear();
          for (int32_t c : frontier)
            for (int64_t i = cptr[t][c]; i < cptr[t][c] + cfill[t][c]; ++i) {
              const int32_t u = clist[t][i];
              if (vstamp[u] != stamp) {
                vstamp[u] = stamp;
                nodes.push_back(u);
              }
            }
          next.clear();
          for (int32_t u : nodes)
            for (int64_t i = vptr[t][u]; i < vptr[t][u] + vfill[t][u]; ++i) {
              const int32_t c = vlist[t][i];
              if (cstamp[c] != stamp) {
                cstamp[c] = stamp;
                clayer[c] = layers + 1;
                next.push_back(c);
                visited.push_back(c);
              }
            }
          if (next.empty()) break;
          ++layers;
          frontier.swap(next);
        }
        // the deepest level that leaves a candidate decides; the least filled
        // candidates form the tie set, in check order
        int32_t chosen = -1;
        for (int k = layers; k >= 1 && chosen < 0; --k) {
          for (int f = 0; f < max_cdeg[t] && chosen < 0; ++f) {
            const met::Fenwick &fw = level[t][f];
            if (fw.total == 0) continue;
            // excluded members of this level, in check order (no repeats)
            skip.clear();
            for (int32_t c : visited) {
              const bool excl = nstamp[c] == stamp || (cstamp[c] == stamp && clayer[c] <= k);
              if (!excl || c < own0[t] || c >= own0[t] + own_n[t]) continue;
              if (cfill[t][c] != f || cfill[t][c] >= cdeg[(int64_t)c * T + t]) continue;
              skip.push_back(c);
            }
            std::sort(skip.begin(), skip.end());
            skip.erase(std::unique(skip.begin(), skip.end()), skip.end());
            const int32_t count = fw.total - (int32_t)skip.size();
            if (count <= 0) continue;
            int32_t want = (int32_t)rng.uniform((uint64_t)count);
            for (int32_t c : skip) {  // rank among the level's members, skipping excluded ones
              if (fw.prefix(c - own0[t]) <= want)
                ++want;
              else
                break;
            }
            chosen = (int32_t)(own0[t] + fw.select(want));
          }
        }
        if (chosen < 0)
          return fail(MET_EINVAL, "no check left for an edge of type %d of node %lld", t, (long long)v);
        const int f = cfill[t][chosen];
        level[t][f].add(chosen - own0[t], -1);
        if (f + 1 < cdeg[(int64_t)chosen * T + t]) level[t][f + 1].add(chosen - own0[t], 1);
        vlist[t][vptr[t][v] + vfill[t][v]++] = chosen;
        clist[t][cptr[t][chosen] + cfill[t][chosen]++] = (int32_t)v;
        ev.push_back((int32_t)v);
        ec.push_back(chosen);
        et.push_back((int8_t)t);
      }
    }
  }
  for (int t = 0; t < T; ++t)
    for (int64_t j = 0; j < M; ++j)
      if (cfill[t][j] != cdeg[j * T + t]) return fail(MET_EINVAL, "sockets of edge type %d left unfilled", t);
  met_code *code = new (std::nothrow) met_code();
  if (!code) return fail(MET_ENOMEM, "out of host memory");
  code->uid = g_next_uid.fetch_add(1) + 1;
  code->N = N;
  code->M = M;
  code->ntypes = T;
  int rc = sort_and_finalize(code, ev, ec, et);
  if (rc != MET_OK) {
    delete code;
    return rc;
  }
  *out = code;
  return MET_OK;
  });
}

extern "C" int met_code_from_edges(int64_t N, int64_t M, int64_t E, const int32_t *vn, const int32_t *cn,
                                   const int8_t *etype, met_code **out) { return met::guarded("met_code_from_edges", [&]() -> int {
  met::clear_error();
  if (!out || !vn || !cn) return fail(MET_EINVAL, "met_code_from_edges: NULL argument");
  *out = nullptr;
  if (N < 1 || M < 1 || E < 2 || N > ((int64_t)1 << 30) || M > ((int64_t)1 << 30) || E > ((int64_t)1 << 31) - 1)
    return fail(MET_EINVAL, "sizes N=%lld M=%lld E=%lld out of range", (long long)N, (long long)M, (long long)E);
  std::vector<int32_t> v(vn, vn + E), ch(cn, cn + E);
  std::vector<int8_t> t(E, 0);
  int32_t ntypes = 1;
  for (int64_t e = 0; e < E; ++e) {
    if (v[e] < 0 || v[e] >= N || ch[e] < 0 || ch[e] >= M)
      return fail(MET_EINVAL, "edge %lld has an index out of range", (long long)e);
    if (etype) {
      if (etype[e] < 0 || etype[e] >= MET_MAX_EDGE_TYPES) return fail(MET_EINVAL, "edge type out of range");
      t[e] = etype[e];
      ntypes = std::max<int32_t>(ntypes, etype[e] + 1);
    }
  }
  {
    std::vector<int64_t> keys(E);
    for (int64_t e = 0; e < E; ++e) keys[e] = (int64_t)v[e] * M + ch[e];
    std::sort(keys.begin(), keys.end());
    for (int64_t e = 1; e < E; ++e)
      if (keys[e] == keys[e - 1]) return fail(MET_EINVAL, "repeated (VN, check) pair");
  }
  met_code *code = new (std::nothrow) met_code();
  if (code) code->uid = g_next_uid.fetch_add(1) + 1;
  if (!code) return fail(MET_ENOMEM, "out of host memory");
  code->N = N;
  code->M = M;
  code->ntypes = ntypes;
  int rc = sort_and_finalize(code, v, ch, t);
  if (rc != MET_OK) {
    delete code;
    return rc;
  }
  *out = code;
  return MET_OK;
  });
}

extern "C" int met_code_info(const met_code *c, met_code_stats *o) { return met::guarded("met_code_info", [&]() -> int {
  met::clear_error();
  if (!c || !o) return fail(MET_EINVAL, "met_code_info: NULL argument");
  std::memset(o, 0, sizeof *o);
  o->N = c->N;
  o->M = c->M;
  o->E = c->E;
  for (int64_t e = 0; e < c->E; ++e) o->E_type[c->et[e]]++;
  o->n_deg1 = c->n_deg1;
  o->edges_to_pass = c->E - c->n_deg1;
  o->n_msg_vn = c->N2;
  o->n_msg_edges = c->E12;
  o->n_leaf_edges = c->EL;
  o->n_edge_types = c->ntypes;
  o->n_check_classes = (int32_t)c->classes.size();
  o->max_check_degree = c->max_check_deg;
  o->max_vn_degree = c->max_vn_deg;
  return MET_OK;
  });
}

extern "C" int met_code_export(const met_code *c, int32_t *vn, int32_t *cn, int8_t *etype) { return met::guarded("met_code_export", [&]() -> int {
  met::clear_error();
  if (!c) return fail(MET_EINVAL, "met_code_export: NULL code");
  if (vn) std::memcpy(vn, c->vn.data(), c->E * sizeof(int32_t));
  if (cn) std::memcpy(cn, c->cn.data(), c->E * sizeof(int32_t));
  if (etype) std::memcpy(etype, c->et.data(), c->E * sizeof(int8_t));
  return MET_OK;
  });
}

extern "C" int met_code_classes(const met_code *c, met_check_class *out, int32_t max_entries, int32_t *n) { return met::guarded("met_code_classes", [&]() -> int {
  met::clear_error();
  if (!c || !out || !n || max_entries < 0) return fail(MET_EINVAL, "met_code_classes: NULL argument");
  const int32_t k = std::min<int32_t>(max_entries, (int32_t)c->classes.size());
  std::vector<uint8_t> seen(c->N2);
  for (int32_t i = 0; i < k; ++i) {
    const met::CheckClass &cc = c->classes[i];
    out[i].n_msg = cc.shape == met::kShapeGeneric ? -1 : cc.n_msg;
    out[i].n_leaf = cc.shape == met::kShapeGeneric ? -1 : cc.n_leaf;
    out[i].first_check = cc.first_check;
    out[i].n_checks = cc.n_checks;
    std::fill(seen.begin(), seen.end(), 0);
    int64_t touched = 0;
    const int64_t e0 = c->chk_msg_ptr[cc.first_check], e1 = c->chk_msg_ptr[cc.first_check + cc.n_checks];
    for (int64_t e = e0; e < e1; ++e)
      if (!seen[c->edge_msgvn[e]]) {
        seen[c->edge_msgvn[e]] = 1;
        ++touched;
      }
    out[i].n_msg_vn_touched = touched;
  }
  *n = (int32_t)c->classes.size();
  return MET_OK;
  });
}
