// Host-side analysis of the ILU(0) factors (plain C++, no HIP): the sorted
// pattern, the dependency levels of both triangular sweeps, the level-order
// layout of each sweep and its launch plan.  The device factorization and
// sweeps in kernels_ilu.hip run on what these functions produce.
//
// A row of the forward sweep depends on the rows its strictly lower part
// stores, a row of the backward sweep on the rows its strictly upper part
// stores, and a row of the (row-order) factorization on the same rows as in
// the forward sweep; a row's level is one more than the largest level it
// depends on, so the rows of a level are independent of each other.
#pragma once

#include <algorithm>
#include <cstdint>
#include <string>
#include <utility>
#include <vector>

namespace lsba {

constexpr int kIluEll = 4;               // entries per position in the padded copy
constexpr int kIluChainThreads = 1024;   // workgroup of a chained run of levels
constexpr int kIluChainPasses = 4;       // factorization: a level is chained if it fits this
                                         // many passes of the workgroup
constexpr int kIluChainCols = 4;         // sweeps: most columns one lane takes in a chain
constexpr int kIluChainLevels = 2048;    // most levels of one chained run (LDS offsets)
constexpr int kIluThreads = 256;         // workgroup of a one-level launch
constexpr int kIluMaxGrid = 1 << 16;

struct IluLaunch {
  int l0, l1;       // levels [l0, l1) of one launch
  int grid;         // workgroups (1: the levels are chained in one workgroup)
  int lsh;          // 2^lsh lanes per row
  int64_t rows, ents;   // rows and off-diagonal entries the launch covers
};

// One sweep in level order: the positions of level l are [ptr[l], ptr[l+1]),
// rows[k] is the row at position k (rows of a level ascending), its
// off-diagonal entries of the factor part are ci[rp[k] .. rp[k+1]) with
// map[] their places in the sorted pattern, pivmap[k] the place of the pivot
// (backward sweep), lents[l] = rp[ptr[l]], and ecol / emap the first kIluEll
// entries of every position padded to that width (column 0, map -1).
struct IluSweepHost {
  std::vector<int> ptr, rows;
  std::vector<int64_t> rp, map, pivmap, lents, emap;
  std::vector<int> ci, ecol;
};

// Sort each row's columns: srp / sci the sorted pattern, perm[p] the place
// in A of sorted entry p, dg[i] the place of row i's diagonal.  Returns ""
// or the reason the pattern cannot be factored (a row without its diagonal,
// a column stored twice in a row).
inline std::string ilu_sort_pattern(int64_t n, int64_t nnz, const int64_t* rp, const int* ci,
                                    std::vector<int64_t>& srp, std::vector<int>& sci,
                                    std::vector<int64_t>& perm, std::vector<int64_t>& dg) {
  srp.assign(rp, rp + n + 1);
  sci.assign(nnz, 0);
  perm.assign(nnz, 0);
  dg.assign(n, -1);
  std::vector<std::pair<int, int64_t>> row;
  for (int64_t i = 0; i < n; ++i) {
    row.clear();
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p) row.push_back({ci[p], p});
    std::sort(row.begin(), row.end());
    for (size_t q = 0; q < row.size(); ++q) {
      const int64_t p = rp[i] + (int64_t)q;
      sci[p] = row[q].first;
      perm[p] = row[q].second;
      if (q > 0 && row[q].first == row[q - 1].first)
        return "row " + std::to_string(i) + " stores column " + std::to_string(row[q].first) +
               " twice";
      if (row[q].first == i) dg[i] = p;
    }
    if (dg[i] < 0) return "row " + std::to_string(i) + " stores no diagonal entry";
  }
  return "";
}

// Levels and level-order layout of the forward (lower) or backward sweep.
inline IluSweepHost ilu_analyse(int64_t n, const std::vector<int64_t>& srp,
                                const std::vector<int>& sci, const std::vector<int64_t>& dg,
                                bool lower) {
  IluSweepHost h;
  std::vector<int> lev(n, 0);
  int nl = 0;
  auto level_of = [&](int64_t i) {
    int m = -1;
    const int64_t a = lower ? srp[i] : dg[i] + 1, b = lower ? dg[i] : srp[i + 1];
    for (int64_t p = a; p < b; ++p) m = std::max(m, lev[sci[p]]);
    lev[i] = m + 1;
    nl = std::max(nl, m + 2);
  };
  if (lower)
    for (int64_t i = 0; i < n; ++i) level_of(i);
  else
    for (int64_t i = n - 1; i >= 0; --i) level_of(i);
  h.ptr.assign(nl + 1, 0);
  for (int64_t i = 0; i < n; ++i) h.ptr[lev[i] + 1] += 1;
  for (int l = 0; l < nl; ++l) h.ptr[l + 1] += h.ptr[l];
  std::vector<int> fill(h.ptr.begin(), h.ptr.end() - 1);
  h.rows.resize(n);
  for (int64_t i = 0; i < n; ++i) h.rows[fill[lev[i]]++] = (int)i;
  h.rp.resize(n + 1);
  h.rp[0] = 0;
  h.pivmap.resize(lower ? 0 : n);
  for (int64_t k = 0; k < n; ++k) {
    const int64_t i = h.rows[k];
    const int64_t a = lower ? srp[i] : dg[i] + 1, b = lower ? dg[i] : srp[i + 1];
    for (int64_t p = a; p < b; ++p) {
      h.ci.push_back(sci[p]);
      h.map.push_back(p);
    }
    h.rp[k + 1] = h.rp[k] + (b - a);
    if (!lower) h.pivmap[k] = dg[i];
  }
  h.lents.resize(nl + 1);
  for (int l = 0; l <= nl; ++l) h.lents[l] = h.rp[h.ptr[l]];
  h.ecol.assign((size_t)n * kIluEll, 0);
  h.emap.assign((size_t)n * kIluEll, -1);
  for (int64_t k = 0; k < n; ++k)
    for (int u = 0; u < kIluEll && h.rp[k] + u < h.rp[k + 1]; ++u) {
      h.ecol[k * kIluEll + u] = h.ci[h.rp[k] + u];
      h.emap[k * kIluEll + u] = h.rp[k] + u;
    }
  return h;
}

// Launch plan of a sweep for 2^lshift lanes per row.  Factorization
// (lshift = 0, one thread per row, several passes allowed): levels of up to
// kIluChainPasses workgroup passes are chained.  Sweeps: levels of up to
// kIluChainThreads rows whose rows times lanes fit kIluChainCols columns per
// lane are chained, with the lanes per row the widest level of the run
// allows; any other level gets a launch of its own over many workgroups.
inline std::vector<IluLaunch> ilu_make_plan(const std::vector<int>& hptr,
                                            const std::vector<int64_t>& ents, int lshift,
                                            bool factor) {
  std::vector<IluLaunch> plan;
  const int nlev = (int)hptr.size() - 1;
  auto rows_of = [&](int l) { return (int64_t)hptr[l + 1] - hptr[l]; };
  auto chainable = [&](int64_t r) {
    if (factor) return r <= (int64_t)kIluChainThreads * kIluChainPasses;
    return r <= kIluChainThreads && (r << lshift) <= (int64_t)kIluChainThreads * kIluChainCols;
  };
  int l = 0;
  while (l < nlev) {
    const int64_t r = rows_of(l);
    if (!chainable(r)) {
      const int64_t thr = r << lshift;
      const int64_t g = std::min<int64_t>((thr + kIluThreads - 1) / kIluThreads, kIluMaxGrid);
      plan.push_back({l, l + 1, (int)g, lshift, r, ents[l + 1] - ents[l]});
      ++l;
      continue;
    }
    int l1 = l;
    int64_t maxr = 1;
    while (l1 < nlev && chainable(rows_of(l1)) && l1 - l < kIluChainLevels) {
      maxr = std::max(maxr, rows_of(l1));
      ++l1;
    }
    int lsh = lshift;
    if (!factor)
      while (lsh > 0 && (maxr << lsh) > kIluChainThreads) --lsh;
    plan.push_back({l, l1, 1, lsh, (int64_t)hptr[l1] - hptr[l], ents[l1] - ents[l]});
    l = l1;
  }
  return plan;
}

}  // namespace lsba
