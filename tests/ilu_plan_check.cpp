// Checks the host-side ILU(0) analysis (paper_2208_09899_amd/csrc/ilu_plan.h)
// on one sparsity pattern read from a file: int64 n, int64 nnz, int64
// row_ptr[n + 1], int32 col_idx[nnz].  Prints "ERROR <reason>" when the
// analysis rejects the pattern, "OK <levels lower> <levels upper> ..." when
// every invariant holds, and "FAIL <what>" (exit status 1) otherwise.
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "ilu_plan.h"

using namespace lsba;

static int fail(const std::string& m) {
  std::printf("FAIL %s\n", m.c_str());
  return 1;
}

static std::string check_sweep(int64_t n, const std::vector<int64_t>& srp,
                               const std::vector<int>& sci, const std::vector<int64_t>& dg,
                               bool lower, const IluSweepHost& h) {
  const int nl = (int)h.ptr.size() - 1;
  if (h.ptr[0] != 0 || h.ptr[nl] != n) return "level offsets do not cover the rows";
  std::vector<int> level(n, -1);
  for (int l = 0; l < nl; ++l) {
    if (h.ptr[l + 1] <= h.ptr[l]) return "empty level";
    for (int k = h.ptr[l]; k < h.ptr[l + 1]; ++k) {
      const int i = h.rows[k];
      if (i < 0 || i >= n || level[i] >= 0) return "rows are not a permutation";
      if (k > h.ptr[l] && h.rows[k - 1] >= i) return "rows of a level not ascending";
      level[i] = l;
    }
  }
  for (int64_t k = 0; k < n; ++k) {
    const int64_t i = h.rows[k];
    const int64_t a = lower ? srp[i] : dg[i] + 1, b = lower ? dg[i] : srp[i + 1];
    if (h.rp[k + 1] - h.rp[k] != b - a) return "entry count of a position";
    for (int64_t p = a; p < b; ++p) {
      const int64_t q = h.rp[k] + (p - a);
      const int j = sci[p];
      if (h.ci[q] != j || h.map[q] != p) return "entries or their map";
      if (lower ? !(j < i) : !(j > i)) return "entry outside the factor part";
      if (!(level[j] < level[i])) return "a row depends on a row of its own or a later level";
    }
    if (!lower && h.pivmap[k] != dg[i]) return "pivot map";
    for (int u = 0; u < kIluEll; ++u) {
      const bool in = h.rp[k] + u < h.rp[k + 1];
      const int64_t e = k * kIluEll + u;
      if (in ? (h.ecol[e] != h.ci[h.rp[k] + u] || h.emap[e] != h.rp[k] + u)
             : (h.ecol[e] != 0 || h.emap[e] != -1))
        return "padded entry copy";
    }
  }
  // every level's level is one more than its deepest dependency: no level
  // could move earlier
  for (int64_t i = 0; i < n; ++i) {
    const int64_t a = lower ? srp[i] : dg[i] + 1, b = lower ? dg[i] : srp[i + 1];
    int m = -1;
    for (int64_t p = a; p < b; ++p) m = std::max(m, level[sci[p]]);
    if (level[i] != m + 1) return "level is not the longest dependency chain";
  }
  for (int l = 0; l <= nl; ++l)
    if (h.lents[l] != h.rp[h.ptr[l]]) return "entry offsets per level";
  // launch plans
  for (int j = 0; j <= 6; ++j) {
    const bool factor = j == 6;
    const int lshift = factor ? 0 : j;
    const std::vector<IluLaunch> plan = ilu_make_plan(h.ptr, h.lents, lshift, factor);
    int next = 0;
    for (const IluLaunch& L : plan) {
      if (L.l0 != next || L.l1 <= L.l0 || L.l1 > nl) return "plan does not tile the levels";
      next = L.l1;
      if (L.rows != (int64_t)h.ptr[L.l1] - h.ptr[L.l0]) return "plan row count";
      if (L.ents != h.lents[L.l1] - h.lents[L.l0]) return "plan entry count";
      if (L.grid == 1) {
        if (L.l1 - L.l0 > kIluChainLevels) return "chain longer than its LDS offsets";
        if (L.lsh > lshift || L.lsh < 0) return "chain lanes";
        for (int l = L.l0; l < L.l1; ++l) {
          const int64_t r = h.ptr[l + 1] - h.ptr[l];
          if (factor) {
            if (r > (int64_t)kIluChainThreads * kIluChainPasses) return "factor chain level";
          } else {
            if ((r << L.lsh) > kIluChainThreads) return "chain level exceeds the workgroup";
            if ((1 << (lshift - L.lsh)) > kIluChainCols) return "columns per lane";
          }
        }
      } else {
        if (L.l1 != L.l0 + 1) return "one-level launch spans levels";
        if (L.lsh != lshift) return "one-level launch lanes";
        const int64_t thr = L.rows << lshift;
        const int64_t need = (thr + kIluThreads - 1) / kIluThreads;
        if (L.grid < 2 || L.grid != std::min<int64_t>(need, kIluMaxGrid))
          return "one-level launch grid";
      }
    }
    if (next != nl) return "plan ends early";
  }
  return "";
}

int main(int argc, char** argv) {
  if (argc != 2) return fail("usage: ilu_plan_check <pattern file>");
  FILE* fp = std::fopen(argv[1], "rb");
  if (!fp) return fail("cannot open the pattern file");
  int64_t hdr[2];
  if (std::fread(hdr, sizeof(int64_t), 2, fp) != 2) return fail("short header");
  const int64_t n = hdr[0], nnz = hdr[1];
  std::vector<int64_t> rp(n + 1);
  std::vector<int> ci(nnz);
  if (std::fread(rp.data(), sizeof(int64_t), n + 1, fp) != (size_t)(n + 1) ||
      std::fread(ci.data(), sizeof(int), nnz, fp) != (size_t)nnz)
    return fail("short pattern");
  std::fclose(fp);
  std::vector<int64_t> srp, perm, dg;
  std::vector<int> sci;
  const std::string e = ilu_sort_pattern(n, nnz, rp.data(), ci.data(), srp, sci, perm, dg);
  if (!e.empty()) {
    std::printf("ERROR %s\n", e.c_str());
    return 0;
  }
  // the sorted pattern holds A's entries, each row ascending
  for (int64_t i = 0; i < n; ++i)
    for (int64_t p = srp[i]; p < srp[i + 1]; ++p) {
      if (ci[perm[p]] != sci[p] || perm[p] < rp[i] || perm[p] >= rp[i + 1])
        return fail("sort permutation");
      if (p > srp[i] && sci[p - 1] >= sci[p]) return fail("row not ascending");
    }
  const IluSweepHost lo = ilu_analyse(n, srp, sci, dg, true);
  const IluSweepHost up = ilu_analyse(n, srp, sci, dg, false);
  std::string m = check_sweep(n, srp, sci, dg, true, lo);
  if (!m.empty()) return fail("lower: " + m);
  m = check_sweep(n, srp, sci, dg, false, up);
  if (!m.empty()) return fail("upper: " + m);
  std::printf("OK %d %d %zu %zu\n", (int)lo.ptr.size() - 1, (int)up.ptr.size() - 1,
              ilu_make_plan(lo.ptr, lo.lents, 3, false).size(),
              ilu_make_plan(up.ptr, up.lents, 3, false).size());
  return 0;
}
