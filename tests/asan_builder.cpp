// Host-only driver of the code builder for an AddressSanitizer /
// UndefinedBehaviorSanitizer build (g++, no GPU code): every construction path
// of met_code.cpp, the derived decoder structures, the all-nodes view, the
// copy-out calls and the validation errors, on the three rate profiles and on
// small random edge lists.  Exit status 0 when every check holds; the
// sanitizers abort on the first invalid access.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "met_internal.h"

namespace {

int g_failures = 0;

void expect(bool ok, const char *what) {
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s\n", what);
    ++g_failures;
  }
}

// Host-side release: no device copy is made in this program, so the handle
// and its all-nodes view are plain host objects.
void release(met_code *c) {
  if (!c) return;
  release(c->all_vns);
  delete c;
}

struct Prof {
  std::vector<double> vf, cf;
  std::vector<int32_t> vd, cd;
  met_profile p;
};

Prof make(double f2, int d1, int d2, double c1, int cd1) {
  Prof r;
  r.vf = {f2, 1.0 - f2};
  r.vd = {d1, d2, 0, 0, 0, 1};
  r.cf = {c1, 1.0 - f2};
  r.cd = {cd1, 0, 0, 0, 3, 1};
  r.p = {3, 2, r.vf.data(), r.vd.data(), 2, r.cf.data(), r.cd.data()};
  return r;
}

void check_code(met_code *c) {
  met_code_stats st;
  expect(met_code_info(c, &st) == MET_OK, "info");
  std::vector<int32_t> vn(st.E), cn(st.E);
  std::vector<int8_t> et(st.E);
  expect(met_code_export(c, vn.data(), cn.data(), et.data()) == MET_OK, "export");
  std::vector<int32_t> vdeg(st.N, 0), cdeg(st.M, 0);
  for (int64_t e = 0; e < st.E; ++e) {
    expect(vn[e] >= 0 && vn[e] < st.N && cn[e] >= 0 && cn[e] < st.M, "edge index in range");
    ++vdeg[vn[e]];
    ++cdeg[cn[e]];
    if (e) expect(cn[e] > cn[e - 1] || (cn[e] == cn[e - 1] && (et[e] > et[e - 1] ||
                                                                (et[e] == et[e - 1] && vn[e] > vn[e - 1]))),
                  "edges sorted by (check, type, variable), no repeated pair");
  }
  int64_t deg1 = 0;
  for (int64_t v = 0; v < st.N; ++v) deg1 += vdeg[v] == 1;
  expect(deg1 == st.n_deg1, "degree-1 count");
  for (int64_t j = 0; j < st.M; ++j) expect(cdeg[j] >= 2 && cdeg[j] <= MET_MAX_CHECK_DEGREE, "check degree");
  met_check_class cls[met::kMaxClasses];
  int32_t n = 0;
  expect(met_code_classes(c, cls, met::kMaxClasses, &n) == MET_OK, "classes");
  int64_t covered = 0;
  for (int k = 0; k < n; ++k) covered += cls[k].n_checks;
  expect(covered == st.M, "classes cover every check");
  // decoder structures: every message edge appears once in the VN edge lists
  std::vector<int32_t> seen(c->E12, 0);
  for (int64_t i = 0; i < c->N2; ++i)
    for (int32_t k = c->vn_ptr[i]; k < c->vn_ptr[i + 1]; ++k) ++seen[c->vn_edges[k]];
  for (int64_t e = 0; e < c->E12; ++e) expect(seen[e] == 1, "message edge listed once");
  const met_code *all = nullptr;
  expect(met::all_vns_view(c, &all) == MET_OK && all && all->EL == 0 && all->E12 == st.E, "all-nodes view");
}

}  // namespace

int main() {
  const Prof profs[3] = {make(0.12, 2, 22, 0.02, 12), make(0.06, 2, 47, 0.01, 12), make(0.03, 2, 97, 0.01, 6)};
  const int64_t sizes[3] = {4096, 20000, 65537};
  for (const Prof &pr : profs)
    for (int64_t n : sizes) {
      met_code *c = nullptr;
      expect(met_code_build(&pr.p, n, 1000 + n, &c) == MET_OK && c, "build");
      if (c) check_code(c);
      release(c);
    }
  // random edge lists: small irregular codes through met_code_from_edges
  uint64_t s = 12345;
  auto rnd = [&](uint64_t m) {
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    return (s >> 33) % m;
  };
  for (int trial = 0; trial < 40; ++trial) {
    const int64_t N = 8 + rnd(60), M = 3 + rnd(20);
    std::vector<int32_t> v, c;
    std::vector<int8_t> t;
    for (int64_t j = 0; j < M; ++j) {
      const int d = 2 + (int)rnd(6);
      std::vector<int32_t> used;
      for (int k = 0; k < d; ++k) {
        int32_t x = (int32_t)rnd(N);
        bool dup = false;
        for (int32_t u : used) dup |= u == x;
        if (dup) continue;
        used.push_back(x);
        v.push_back(x);
        c.push_back((int32_t)j);
        t.push_back((int8_t)rnd(3));
      }
      if (used.size() < 2) {  // keep every check at degree >= 2
        const int32_t x = (used[0] + 1) % (int32_t)N;
        v.push_back(x);
        c.push_back((int32_t)j);
        t.push_back(0);
      }
    }
    met_code *code = nullptr;
    expect(met_code_from_edges(N, M, (int64_t)v.size(), v.data(), c.data(), t.data(), &code) == MET_OK,
           "from_edges");
    if (code) check_code(code);
    release(code);
  }
  // validation paths return errors without touching memory they should not
  met_code *bad = nullptr;
  const int32_t v2[3] = {0, 1, 9}, c2[3] = {0, 0, 0};
  expect(met_code_from_edges(3, 1, 3, v2, c2, nullptr, &bad) == MET_EINVAL && !bad, "index out of range");
  const int32_t v3[2] = {1, 1}, c3[2] = {0, 0};
  expect(met_code_from_edges(3, 1, 2, v3, c3, nullptr, &bad) == MET_EINVAL && !bad, "repeated pair");
  expect(met_code_build(nullptr, 100, 1, &bad) == MET_EINVAL, "NULL profile");
  expect(met_code_build(&profs[0].p, (int64_t)1 << 30, 1, &bad) == MET_EINVAL && !bad, "edge count above int32");
  expect(met_code_info(nullptr, nullptr) == MET_EINVAL, "NULL info");
  if (g_failures) return 1;
  std::printf("asan builder ok\n");
  return 0;
}
