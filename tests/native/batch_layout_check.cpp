// CPU check of the batch host layout (paper_2509_13592_amd/csrc/batch_layout.h), built by
// tests/test_batch_layout_cpu.py with the address and undefined-behaviour sanitizers.
//
// Scenes with ragged grids, array sizes and support lists (built the way a plan builds
// them: each kept element (m1, m2) folds onto spectral bin (m1 mod L1, m2 mod L2), bins
// listed per column k1) are grouped and concatenated; every class's arrays are then
// checked entry by entry against the scenes they came from, and inconsistent tables must
// be refused.  Prints "ok" and returns 0 on success.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "batch_layout.h"

namespace {

struct Entry {
  int k2;
  float omega;
};

struct Scene {
  int L1, L2;
  std::vector<int> sup_ptr, src_ptr, src, scol;
  std::vector<Entry> sup;
  int nscol = 0;
  bool prune_ok = false;
};

int fails = 0;
#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      std::printf("check failed at line %d: %s\n", __LINE__, #c);       \
      ++fails;                                                          \
    }                                                                   \
  } while (0)

Scene make_scene(std::mt19937& rng, int L1, int L2, int M1, int M2) {
  Scene s;
  s.L1 = L1;
  s.L2 = L2;
  std::vector<std::vector<int>> bin_src(static_cast<size_t>(L1) * L2);
  int m = 0;
  std::bernoulli_distribution keep(0.4);
  for (int m2 = 0; m2 < M2; ++m2)
    for (int m1 = 0; m1 < M1; ++m1)
      if (keep(rng) || (m1 == 0 && m2 == 0)) {
        bin_src[static_cast<size_t>(m2 % L2) * L1 + (m1 % L1)].push_back((m << 1) | ((m1 + m2) & 1));
        ++m;
      }
  s.sup_ptr.assign(L1 + 1, 0);
  s.src_ptr.assign(1, 0);
  for (int k1 = 0; k1 < L1; ++k1) {
    s.sup_ptr[k1] = static_cast<int>(s.sup.size());
    for (int k2 = 0; k2 < L2; ++k2) {
      const auto& b = bin_src[static_cast<size_t>(k2) * L1 + k1];
      if (b.empty()) continue;
      s.sup.push_back(Entry{k2, static_cast<float>(L1 * L2 * b.size())});
      for (int c : b) s.src.push_back(c);
      s.src_ptr.push_back(static_cast<int>(s.src.size()));
    }
  }
  s.sup_ptr[L1] = static_cast<int>(s.sup.size());
  for (int k1 = 0; k1 < L1; ++k1)
    if (s.sup_ptr[k1 + 1] > s.sup_ptr[k1]) s.scol.push_back(k1);
  s.nscol = static_cast<int>(s.scol.size());
  const int ncs = (s.nscol + 3) / 4 * 4;
  s.prune_ok = L1 >= 8 && s.nscol >= 1 && ncs <= L1 / 2;
  s.scol.resize(ncs, -1);
  return s;
}

bccb_layout::SceneTables<Entry> view(const Scene& s) {
  bccb_layout::SceneTables<Entry> t;
  t.L1 = s.L1;
  t.L2 = s.L2;
  t.sparse = true;
  t.sup_ptr = &s.sup_ptr;
  t.sup = &s.sup;
  t.src_ptr = &s.src_ptr;
  t.src = &s.src;
  t.prune_ok = s.prune_ok;
  t.nscol = s.nscol;
  t.scol = &s.scol;
  return t;
}

void check_batch(std::mt19937& rng, int nscenes) {
  const int Ls[] = {8, 16, 32, 64, 128, 256};
  const int Ms[] = {1, 3, 5, 12, 16, 20, 32};
  std::vector<Scene> scenes;
  std::vector<std::pair<int, int>> grids;
  for (int i = 0; i < nscenes; ++i) {
    const int L1 = Ls[rng() % 6], L2 = Ls[rng() % 6];
    scenes.push_back(make_scene(rng, L1, L2, Ms[rng() % 7], Ms[rng() % 7]));
    grids.emplace_back(L1, L2);
  }
  std::vector<bccb_layout::SceneTables<Entry>> tables;
  for (const Scene& s : scenes) tables.push_back(view(s));
  const auto classes = bccb_layout::group_by_grid(grids);
  // every scene in exactly one class, in batch order within it, classes by first appearance
  std::vector<int> seen(nscenes, 0);
  int first = -1;
  for (const auto& c : classes) {
    CHECK(!c.scenes.empty());
    CHECK(c.scenes.front() > first);
    first = c.scenes.front();
    for (size_t k = 0; k < c.scenes.size(); ++k) {
      const int i = c.scenes[k];
      CHECK(i >= 0 && i < nscenes);
      if (i < 0 || i >= nscenes) continue;
      ++seen[i];
      CHECK(grids[i].first == c.L1 && grids[i].second == c.L2);
      if (k) CHECK(c.scenes[k] > c.scenes[k - 1]);
    }
  }
  for (int v : seen) CHECK(v == 1);
  for (const auto& c : classes) {
    bccb_layout::ClassSupport<Entry> cs;
    CHECK(bccb_layout::concat_support(tables, c, &cs));
    const size_t n = c.scenes.size();
    CHECK(cs.sup_ptr.size() == n * (c.L1 + 1));
    CHECK(cs.src_ptr.size() == cs.sup.size() + 1);
    CHECK(cs.entry_off.size() == n);
    CHECK(static_cast<size_t>(cs.src_ptr.back()) == cs.src.size());
    for (size_t k = 0; k < n; ++k) {
      const Scene& s = scenes[c.scenes[k]];
      CHECK(cs.max_entries >= static_cast<int>(s.sup.size()));
      for (int k1 = 0; k1 < c.L1; ++k1) {
        const int a = cs.sup_ptr[k * (c.L1 + 1) + k1], b = cs.sup_ptr[k * (c.L1 + 1) + k1 + 1];
        CHECK(a == cs.entry_off[k] + s.sup_ptr[k1] && b == cs.entry_off[k] + s.sup_ptr[k1 + 1]);
        for (int e = a; e < b; ++e) {
          const int le = e - cs.entry_off[k];
          CHECK(cs.sup[e].k2 == s.sup[le].k2 && cs.sup[e].omega == s.sup[le].omega);
          const int n_src = cs.src_ptr[e + 1] - cs.src_ptr[e];
          CHECK(n_src == s.src_ptr[le + 1] - s.src_ptr[le]);
          for (int j = 0; j < n_src && j < s.src_ptr[le + 1] - s.src_ptr[le]; ++j)
            CHECK(cs.src[cs.src_ptr[e] + j] == s.src[s.src_ptr[le] + j]);
        }
      }
    }
    bool all_prune = true;
    for (int i : c.scenes) all_prune = all_prune && scenes[i].prune_ok;
    bccb_layout::KeptColumns kc;
    const bool ok = bccb_layout::kept_columns(tables, c, &kc);
    CHECK(ok == all_prune);
    if (!ok) continue;
    CHECK(kc.ncs % 4 == 0 && kc.scol.size() == n * kc.ncs && kc.colslot.size() == n * c.L1);
    for (size_t k = 0; k < n; ++k) {
      const Scene& s = scenes[c.scenes[k]];
      for (int j = 0; j < kc.ncs; ++j) {
        const int k1 = kc.scol[k * kc.ncs + j];
        CHECK((j < s.nscol) ? k1 == s.scol[j] : k1 == -1);
        if (k1 >= 0) CHECK(kc.colslot[k * c.L1 + k1] == j);
      }
      int kept = 0;
      for (int k1 = 0; k1 < c.L1; ++k1) kept += kc.colslot[k * c.L1 + k1] >= 0;
      CHECK(kept == s.nscol);
    }
  }
}

void check_refusals(std::mt19937& rng) {
  Scene s = make_scene(rng, 16, 8, 5, 4);
  std::vector<std::pair<int, int>> grids(1, {16, 8});
  const auto classes = bccb_layout::group_by_grid(grids);
  bccb_layout::ClassSupport<Entry> cs;
  bccb_layout::KeptColumns kc;
  {
    Scene b = s;
    b.sup_ptr.pop_back();                      // CSR one short
    std::vector<bccb_layout::SceneTables<Entry>> t{view(b)};
    CHECK(!bccb_layout::concat_support(t, classes[0], &cs));
  }
  {
    Scene b = s;
    b.src_ptr.back() += 3;                     // sources past the end
    std::vector<bccb_layout::SceneTables<Entry>> t{view(b)};
    CHECK(!bccb_layout::concat_support(t, classes[0], &cs));
  }
  {
    Scene b = s;
    b.L1 = 32;                                 // scene of another class
    std::vector<bccb_layout::SceneTables<Entry>> t{view(b)};
    CHECK(!bccb_layout::concat_support(t, classes[0], &cs));
  }
  {
    Scene b = s;
    if (b.prune_ok) {
      b.scol[0] = 99;                          // kept column outside the grid
      std::vector<bccb_layout::SceneTables<Entry>> t{view(b)};
      CHECK(!bccb_layout::kept_columns(t, classes[0], &kc));
    }
    b = s;
    b.nscol = static_cast<int>(b.scol.size()) + 1;   // more kept columns than listed
    b.prune_ok = true;
    std::vector<bccb_layout::SceneTables<Entry>> t{view(b)};
    CHECK(!bccb_layout::kept_columns(t, classes[0], &kc));
  }
  {
    bccb_layout::Class bad = classes[0];
    bad.scenes.push_back(7);                   // index past the scene list
    std::vector<bccb_layout::SceneTables<Entry>> t{view(s)};
    CHECK(!bccb_layout::concat_support(t, bad, &cs));
    CHECK(!bccb_layout::kept_columns(t, bad, &kc));
  }
}

}  // namespace

int main() {
  std::mt19937 rng(12345);
  for (int trial = 0; trial < 40; ++trial) check_batch(rng, 1 + static_cast<int>(rng() % 200));
  check_batch(rng, 4096);
  check_refusals(rng);
  if (fails) {
    std::printf("%d checks failed\n", fails);
    return 1;
  }
  std::printf("ok\n");
  return 0;
}
