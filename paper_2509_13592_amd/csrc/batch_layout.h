// Host-side layout of a batched solve: scenes grouped into size classes, their
// spectral-support lists concatenated with per-scene offsets, and the kept-column
// maps of the pruned passes.
//
// Plain C++ with no HIP dependency, so that the exact code the library runs can be
// compiled on its own under the address and undefined-behaviour sanitizers and driven
// with ragged inputs on the CPU.  Every index it writes is checked against the sizes
// it was given; inconsistent inputs make it return false instead of reading or
// writing out of bounds.
#pragma once

#include <algorithm>
#include <cstddef>
#include <map>
#include <utility>
#include <vector>

namespace bccb_layout {

// What one scene's plan contributes (views of the plan's host tables).
template <class Entry>
struct SceneTables {
  int L1 = 0, L2 = 0;
  bool sparse = false;                      // the plan applies Omega from its support lists
  const std::vector<int>* sup_ptr = nullptr;   // [L1 + 1] CSR over spectral columns k1
  const std::vector<Entry>* sup = nullptr;     // [nsup] support bins
  const std::vector<int>* src_ptr = nullptr;   // [nsup + 1] CSR over bins
  const std::vector<int>* src = nullptr;       // snapshot entries folding onto the bins
  bool prune_ok = false;                       // the plan has a kept-column set
  int nscol = 0;                               // kept spectral columns
  const std::vector<int>* scol = nullptr;      // [>= nscol] the kept columns k1
};

// One size class: grid (L1, L2) and the batch indices of its scenes in arena order.
struct Class {
  int L1 = 0, L2 = 0;
  std::vector<int> scenes;
};

// Scenes grouped by grid size, classes in order of first appearance, scenes in batch order.
inline std::vector<Class> group_by_grid(const std::vector<std::pair<int, int>>& grids) {
  std::vector<Class> out;
  std::map<std::pair<int, int>, size_t> index;
  for (size_t i = 0; i < grids.size(); ++i) {
    auto it = index.find(grids[i]);
    if (it == index.end()) {
      Class c;
      c.L1 = grids[i].first;
      c.L2 = grids[i].second;
      it = index.emplace(grids[i], out.size()).first;
      out.push_back(c);
    }
    out[it->second].scenes.push_back(static_cast<int>(i));
  }
  return out;
}

// The support lists of a class's scenes as one set of arrays: sup_ptr [n][L1 + 1] holds
// global entry offsets, src_ptr [total entries + 1] global source offsets.
template <class Entry>
struct ClassSupport {
  std::vector<int> sup_ptr, src_ptr, src, entry_off;
  std::vector<Entry> sup;
  int max_entries = 0;
};

template <class Entry>
bool tables_consistent(const SceneTables<Entry>& t) {
  if (!t.sup_ptr || !t.sup || !t.src_ptr || !t.src) return false;
  const size_t nsup = t.sup->size();
  if (t.L1 < 1 || t.sup_ptr->size() != static_cast<size_t>(t.L1) + 1 || t.src_ptr->size() != nsup + 1) return false;
  if ((*t.sup_ptr)[0] != 0 || static_cast<size_t>((*t.sup_ptr)[t.L1]) != nsup) return false;
  for (int k = 0; k < t.L1; ++k)
    if ((*t.sup_ptr)[k + 1] < (*t.sup_ptr)[k]) return false;
  if ((*t.src_ptr)[0] != 0 || static_cast<size_t>((*t.src_ptr)[nsup]) != t.src->size()) return false;
  for (size_t j = 0; j < nsup; ++j)
    if ((*t.src_ptr)[j + 1] < (*t.src_ptr)[j]) return false;
  return true;
}

template <class Entry>
bool concat_support(const std::vector<SceneTables<Entry>>& scenes, const Class& c, ClassSupport<Entry>* out) {
  ClassSupport<Entry> r;
  r.src_ptr.push_back(0);
  for (int i : c.scenes) {
    if (i < 0 || static_cast<size_t>(i) >= scenes.size()) return false;
    const SceneTables<Entry>& t = scenes[i];
    if (t.L1 != c.L1 || t.L2 != c.L2 || !tables_consistent(t)) return false;
    const int eoff = static_cast<int>(r.sup.size());
    const int soff = static_cast<int>(r.src.size());
    r.entry_off.push_back(eoff);
    r.max_entries = std::max(r.max_entries, static_cast<int>(t.sup->size()));
    for (int v : *t.sup_ptr) r.sup_ptr.push_back(v + eoff);
    r.sup.insert(r.sup.end(), t.sup->begin(), t.sup->end());
    for (size_t j = 1; j < t.src_ptr->size(); ++j) r.src_ptr.push_back((*t.src_ptr)[j] + soff);
    r.src.insert(r.src.end(), t.src->begin(), t.src->end());
  }
  *out = std::move(r);
  return true;
}

// Kept-column maps of a class whose every scene has a kept-column set: ncs = the widest
// scene's count rounded up to a multiple of 4; scol [n][ncs] the kept columns (-1 =
// padding), colslot [n][L1] the slot of each spectral column (-1 = not kept).
struct KeptColumns {
  int ncs = 0;
  std::vector<int> scol, colslot;
};

template <class Entry>
bool kept_columns(const std::vector<SceneTables<Entry>>& scenes, const Class& c, KeptColumns* out) {
  KeptColumns r;
  for (int i : c.scenes) {
    if (i < 0 || static_cast<size_t>(i) >= scenes.size()) return false;
    const SceneTables<Entry>& t = scenes[i];
    if (!t.prune_ok || !t.scol || t.nscol < 1 || static_cast<size_t>(t.nscol) > t.scol->size()) return false;
    r.ncs = std::max(r.ncs, (t.nscol + 3) / 4 * 4);
  }
  const size_t n = c.scenes.size();
  r.scol.assign(n * r.ncs, -1);
  r.colslot.assign(n * static_cast<size_t>(c.L1), -1);
  for (size_t k = 0; k < n; ++k) {
    const SceneTables<Entry>& t = scenes[c.scenes[k]];
    for (int j = 0; j < t.nscol; ++j) {
      const int k1 = (*t.scol)[j];
      if (k1 < 0 || k1 >= c.L1) return false;
      r.scol[k * r.ncs + j] = k1;
      r.colslot[k * c.L1 + k1] = j;
    }
  }
  *out = std::move(r);
  return true;
}

}  // namespace bccb_layout
