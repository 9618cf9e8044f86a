// ILU(0) preconditioner: factorization and application, level-scheduled.
//
// The paper's tests on matrices from applications (Sec. 5) precondition with
// an incomplete LU factorization with no fill.  ILU(0) keeps L (unit lower)
// and U (upper) on A's pattern with (L U)_ij = a_ij there; it is Gaussian
// elimination in row order with every update outside the pattern dropped.
// Row i of the elimination reads rows k < i that it stores, and a triangular
// sweep's row reads the rows its factor part stores; both therefore run one
// dependency level at a time: the rows of a level are independent.
//
// Launch plan: a level whose rows (times the lanes per row) fill several
// workgroups gets a launch of its own (the launch boundary orders it after
// the previous level); runs of smaller levels are chained inside ONE
// workgroup of 1024 threads with a workgroup barrier between levels, which
// saves a launch per level where the graph's levels are narrow.  No kernel
// waits on another workgroup.  In a chained run every thread solves at most
// one row per level (a lane takes several columns when the widest level's
// rows times the lanes per row exceed the workgroup), and the loads a level
// issues are independent of each other (its own gathers, the next level's
// right-hand side, the row data of the level after that).  The barrier
// between levels drains every load in flight, so a level costs one memory
// round trip plus the barrier; row data that is cold in L2 sets that round
// trip's length.
//
// Sweep layout: positions in level order (rows of a level ascending), each
// position's off-diagonal entries contiguous, so the lanes of a wavefront
// read neighbouring rows' entries and the s lanes of a row read s contiguous
// elements of each gathered row of the block; the first kIluEll entries of
// every position are repeated in a padded fixed-width array, so that their
// addresses follow from the position alone.
#include <algorithm>
#include <climits>
#include <cmath>

#include "lsba_internal.h"

namespace lsba {

namespace {


// Factorization of the rows of levels [l0, l1) (one thread per row).  The
// updates are evaluated as written (no fused multiply-add), the order of the
// elimination: multipliers by ascending k, each followed by its row's
// updates.
__global__ __launch_bounds__(kIluChainThreads) void ilu_factor_kernel(
    int l0, int l1, const int* __restrict__ lvl_ptr, const int* __restrict__ rows,
    const int64_t* __restrict__ frp, const int* __restrict__ fci,
    const int64_t* __restrict__ fdg, double* fv, unsigned long long* bad) {
#pragma clang fp contract(off)
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int l = l0; l < l1; ++l) {
    const int b = lvl_ptr[l], e = lvl_ptr[l + 1];
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < e - b; t += stride) {
      const int64_t i = rows[b + t];
      const int64_t pe = frp[i + 1], di = fdg[i];
      for (int64_t p = frp[i]; p < di; ++p) {
        const int64_t k = fci[p];
        const double lik = fv[p] / fv[fdg[k]];
        fv[p] = lik;
        // a_ij -= l_ik u_kj for the j > k that rows i and k both store
        int64_t q = p + 1, r = fdg[k] + 1;
        const int64_t re = frp[k + 1];
        while (q < pe && r < re) {
          const int cq = fci[q], cr = fci[r];
          if (cq == cr) {
            const double prod = lik * fv[r];
            fv[q] = fv[q] - prod;
            ++q;
            ++r;
          } else if (cq < cr) {
            ++q;
          } else {
            ++r;
          }
        }
      }
      const double d = fv[di];
      if (!(d != 0.0 && isfinite(d))) atomicMin(bad, (unsigned long long)i);
    }
    if (l + 1 < l1) __syncthreads();
  }
}

// One wide level of a sweep (l1 = l0 + 1) over many workgroups: 2^lshift
// lanes per row, lane c < s owns column c.  Forward (LOWER):
// z_i = y_i - sum_j l_ij z_j; backward: x_i = (z_i - sum_j u_ij x_j) / u_ii.
// Y and Z may be the same block.  (With one workgroup it would also chain
// levels [l0, l1) behind barriers; the launch plan uses ilu_chain_kernel
// for that.)
template <bool LOWER>
__global__ __launch_bounds__(kIluChainThreads) void ilu_sweep_kernel(
    int s, int lshift, int l0, int l1, const int* __restrict__ lvl_ptr,
    const int* __restrict__ rows, const int64_t* __restrict__ rp, const int* __restrict__ ci,
    const double* __restrict__ v, const double* __restrict__ piv, const double* Y, double* Z,
    const Ctl* __restrict__ ctl) {
  if (ctl && ctl->stop) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int lmask = (1 << lshift) - 1;
  for (int l = l0; l < l1; ++l) {
    const int b = lvl_ptr[l], e = lvl_ptr[l + 1];
    const int64_t total = (int64_t)(e - b) << lshift;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
      const int c = (int)(t & lmask);
      if (c < s) {
        const int k = b + (int)(t >> lshift);
        const int64_t i = rows[k];
        double acc = Y[i * s + c];
        const int64_t pe = rp[k + 1];
        for (int64_t p = rp[k]; p < pe; ++p) acc -= v[p] * Z[(int64_t)ci[p] * s + c];
        if (!LOWER) acc = acc / piv[k];
        Z[i * s + c] = acc;
      }
    }
    if (l + 1 < l1) __syncthreads();
  }
}

// A chained run of levels [l0, l1) in one workgroup: thread t solves row
// t >> lsh of each level (when the level has that many), columns
// (t & (2^lsh - 1)) + q 2^lsh.  Every load a level issues is independent of
// the others: the gathers of its own row (columns loaded a level earlier),
// the right-hand side of the next level's row (row loaded a level earlier)
// and the offsets, first entries and pivot of the row two levels on
// (positions from the offsets staged in LDS).  The workgroup barrier between
// levels drains them all, so a level costs one memory round trip.
template <bool LOWER>
__global__ __launch_bounds__(kIluChainThreads) void ilu_chain_kernel(
    int s, int lsh, int l0, int l1, const int* __restrict__ lvl_ptr,
    const int* __restrict__ rows, const int64_t* __restrict__ rp, const int* __restrict__ ci,
    const double* __restrict__ v, const int* __restrict__ ecol, const double* __restrict__ eval,
    const double* __restrict__ piv, const double* Y, double* Z, const Ctl* __restrict__ ctl) {
  if (ctl && ctl->stop) return;
  __shared__ int sp[kIluChainLevels + 1];
  const int nl = l1 - l0;
  for (int t = threadIdx.x; t <= nl; t += blockDim.x) sp[t] = lvl_ptr[l0 + t];
  __syncthreads();
  const int L = 1 << lsh;
  const int slot = threadIdx.x >> lsh;
  const int c0 = threadIdx.x & (L - 1);
  struct Row {
    bool act;
    int cnt;
    int64_t i, p;
    int col[kIluEll];
    double val[kIluEll];
    double d;
  };
  auto meta = [&](int l, Row& r) {
    const int b = sp[l], e = sp[l + 1];
    r.act = slot < e - b;
    const int k = r.act ? b + slot : b;   // a valid position either way
    r.i = rows[k];
    r.p = rp[k];
    r.cnt = (int)(rp[k + 1] - r.p);
#pragma unroll
    for (int u = 0; u < kIluEll; ++u) {
      r.col[u] = ecol[(int64_t)k * kIluEll + u];
      r.val[u] = eval[(int64_t)k * kIluEll + u];
    }
    r.d = LOWER ? 1.0 : piv[k];
  };
  auto rhs = [&](const Row& r, double (&y)[kIluChainCols]) {
#pragma unroll
    for (int q = 0; q < kIluChainCols; ++q) {
      const int c = c0 + q * L;
      y[q] = (r.act && c < s) ? Y[r.i * s + c] : 0.0;
    }
  };
  Row cur, nxt;
  double y[kIluChainCols];
  meta(0, cur);
  rhs(cur, y);
  if (nl > 1) meta(1, nxt);
  for (int l = 0; l < nl; ++l) {
    double acc[kIluChainCols];
#pragma unroll
    for (int q = 0; q < kIluChainCols; ++q) acc[q] = y[q];
    if (cur.act) {
#pragma unroll
      for (int u = 0; u < kIluEll; ++u) {
        if (u < cur.cnt) {
          const int64_t j = cur.col[u];
#pragma unroll
          for (int q = 0; q < kIluChainCols; ++q) {
            const int c = c0 + q * L;
            if (c < s) acc[q] -= cur.val[u] * Z[j * s + c];
          }
        }
      }
      for (int64_t p = cur.p + kIluEll; p < cur.p + cur.cnt; ++p) {
        const int64_t j = ci[p];
        const double vv = v[p];
#pragma unroll
        for (int q = 0; q < kIluChainCols; ++q) {
          const int c = c0 + q * L;
          if (c < s) acc[q] -= vv * Z[j * s + c];
        }
      }
    }
    Row nn{};
    if (l + 1 < nl) rhs(nxt, y);
    if (l + 2 < nl) meta(l + 2, nn);
    if (cur.act) {
#pragma unroll
      for (int q = 0; q < kIluChainCols; ++q) {
        const int c = c0 + q * L;
        if (c < s) Z[cur.i * s + c] = LOWER ? acc[q] : acc[q] / cur.d;
      }
    }
    if (l + 1 < nl) {
      __syncthreads();
      cur = nxt;
      nxt = nn;
    }
  }
}

// dst[i] = src[map[i]], or 0 where map[i] < 0 (padding)
__global__ __launch_bounds__(256) void ilu_gather_kernel(int64_t count,
                                                         const int64_t* __restrict__ map,
                                                         const double* __restrict__ src,
                                                         double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) {
    const int64_t m = map[i];
    dst[i] = m >= 0 ? src[m] : 0.0;
  }
}

void gather(hipStream_t st, int64_t count, const int64_t* map, const double* src, double* dst) {
  if (count <= 0) return;
  const int64_t g = (count + 255) / 256;
  ilu_gather_kernel<<<dim3((unsigned)g), dim3(256), 0, st>>>(count, map, src, dst);
}

template <typename T>
std::string dev_alloc(IluFactors& f, T** p, int64_t count) {
  void* q = nullptr;
  if (hipMalloc(&q, sizeof(T) * (size_t)std::max<int64_t>(count, 1)) != hipSuccess)
    return "device allocation of the ILU(0) factors failed";
  f.mem.push_back(q);
  *p = (T*)q;
  return "";
}

// Copy one sweep's schedule to the device: its arrays are allocated into
// `keep` (the factors), the entry maps of the set-up into `tmp`.
std::string upload(hipStream_t st, IluFactors& keep, IluFactors& tmp, int64_t n, IluSweep& sw,
                   const IluSweepHost& h, bool lower, int64_t** map_dev, int64_t** pivmap_dev,
                   int64_t** emap_dev) {
  std::string e;
  const int64_t ne = (int64_t)h.ci.size();
  sw.nlev = (int)h.ptr.size() - 1;
  if (!(e = dev_alloc(keep, &sw.lvl_ptr, sw.nlev + 1)).empty()) return e;
  if (!(e = dev_alloc(keep, &sw.rows, n)).empty()) return e;
  if (!(e = dev_alloc(keep, &sw.rp, n + 1)).empty()) return e;
  if (!(e = dev_alloc(keep, &sw.ci, ne)).empty()) return e;
  if (!(e = dev_alloc(keep, &sw.v, ne)).empty()) return e;
  if (!(e = dev_alloc(tmp, map_dev, ne)).empty()) return e;
  if (!(e = dev_alloc(keep, &sw.ecol, n * kIluEll)).empty()) return e;
  if (!(e = dev_alloc(keep, &sw.eval, n * kIluEll)).empty()) return e;
  if (!(e = dev_alloc(tmp, emap_dev, n * kIluEll)).empty()) return e;
  if (!lower) {
    if (!(e = dev_alloc(keep, &sw.piv, n)).empty()) return e;
    if (!(e = dev_alloc(tmp, pivmap_dev, n)).empty()) return e;
  }
  auto cp = [&](void* dst, const void* src, size_t bytes) {
    return bytes == 0 || hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st) == hipSuccess;
  };
  bool ok = cp(sw.lvl_ptr, h.ptr.data(), sizeof(int) * h.ptr.size()) &&
            cp(sw.rows, h.rows.data(), sizeof(int) * n) &&
            cp(sw.rp, h.rp.data(), sizeof(int64_t) * (n + 1)) &&
            cp(sw.ci, h.ci.data(), sizeof(int) * ne) &&
            cp(*map_dev, h.map.data(), sizeof(int64_t) * ne) &&
            cp(sw.ecol, h.ecol.data(), sizeof(int) * n * kIluEll) &&
            cp(*emap_dev, h.emap.data(), sizeof(int64_t) * n * kIluEll);
  if (ok && !lower) ok = cp(*pivmap_dev, h.pivmap.data(), sizeof(int64_t) * n);
  if (!ok) return "copy of the ILU(0) level schedule failed";
  for (int j = 0; j < 6; ++j) sw.plan[j] = ilu_make_plan(h.ptr, h.lents, j, false);
  sw.fplan = ilu_make_plan(h.ptr, h.lents, 0, true);
  return "";
}

int lanes_shift_of(int s) {
  int sh = 0;
  while ((1 << sh) < s) ++sh;
  return sh;
}

template <bool LOWER>
void launch_sweep(hipStream_t st, const IluSweep& sw, int s, const double* Y, double* Z,
                  const Ctl* ctl, KTimer* tm) {
  const int lsh = lanes_shift_of(s);
  for (const IluLaunch& L : sw.plan[lsh]) {
    // algorithmic bytes: the off-diagonal entries (value + column), the row
    // list and entry offsets (+ pivots), one read of the input rows and one
    // write of the output rows (the gathered rows are outputs of earlier
    // levels, counted where they were written)
    const double bytes = 12.0 * (double)L.ents + (LOWER ? 12.0 : 20.0) * (double)L.rows +
                         16.0 * (double)L.rows * s;
    if (L.grid == 1)
      launch_k(tm, KK_PRECOND, bytes, ilu_chain_kernel<LOWER>, dim3(1), dim3(kIluChainThreads),
               0, st, s, L.lsh, L.l0, L.l1, (const int*)sw.lvl_ptr, (const int*)sw.rows,
               (const int64_t*)sw.rp, (const int*)sw.ci, (const double*)sw.v,
               (const int*)sw.ecol, (const double*)sw.eval, (const double*)sw.piv, Y, Z, ctl);
    else
      launch_k(tm, KK_PRECOND, bytes, ilu_sweep_kernel<LOWER>, dim3(L.grid), dim3(kIluThreads),
               0, st, s, L.lsh, L.l0, L.l1, (const int*)sw.lvl_ptr, (const int*)sw.rows,
               (const int64_t*)sw.rp, (const int*)sw.ci, (const double*)sw.v,
               (const double*)sw.piv, Y, Z, ctl);
  }
}

}  // namespace

void ilu_free(IluFactors& f) {
  for (void* p : f.mem) (void)hipFree(p);
  f.mem.clear();
  f.frp = nullptr;
  f.fci = nullptr;
  f.fv = nullptr;
  f.lo = IluSweep{};
  f.up = IluSweep{};
}

// On failure the caller releases f with ilu_free.
std::string ilu_build(hipStream_t st, int64_t n, int64_t nnz, const int64_t* rp_h,
                      const int* ci_h, const double* val_dev, IluFactors& f, int64_t* bad_row,
                      bool* bad_input) {
  *bad_row = -1;
  *bad_input = true;
  f.n = n;
  f.nnz = nnz;
  // level positions and row indices are 32-bit
  if (n >= (int64_t)INT_MAX) return "ILU(0) needs n < 2^31 - 1";
  // rows with sorted columns; perm maps a sorted position to A's position
  std::vector<int64_t> srp, perm, dg;
  std::vector<int> sci;
  {
    const std::string e = ilu_sort_pattern(n, nnz, rp_h, ci_h, srp, sci, perm, dg);
    if (!e.empty()) return e;
  }
  *bad_input = false;   // from here on, failures are the device's
  const IluSweepHost lo = ilu_analyse(n, srp, sci, dg, true);
  const IluSweepHost up = ilu_analyse(n, srp, sci, dg, false);
  f.nnz_lo = (int64_t)lo.ci.size();
  f.nnz_up = (int64_t)up.ci.size();
  std::string e;
  int64_t *perm_d = nullptr, *dg_d = nullptr, *lmap = nullptr, *umap = nullptr,
          *pmap = nullptr, *unused = nullptr, *lemap = nullptr, *uemap = nullptr;
  unsigned long long* bad_d = nullptr;
  if (!(e = dev_alloc(f, &f.frp, n + 1)).empty()) return e;
  if (!(e = dev_alloc(f, &f.fci, nnz)).empty()) return e;
  if (!(e = dev_alloc(f, &f.fv, nnz)).empty()) return e;
  // set-up only arrays, freed at the end
  IluFactors tmp;
  auto fail_tmp = [&](const std::string& m) {
    (void)hipStreamSynchronize(st);
    ilu_free(tmp);
    return m;
  };
  if (!(e = dev_alloc(tmp, &perm_d, nnz)).empty()) return fail_tmp(e);
  if (!(e = dev_alloc(tmp, &dg_d, n)).empty()) return fail_tmp(e);
  if (!(e = dev_alloc(tmp, &bad_d, 1)).empty()) return fail_tmp(e);
  const unsigned long long none = ULLONG_MAX;
  if (hipMemcpyAsync(f.frp, srp.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, st) !=
          hipSuccess ||
      (nnz && hipMemcpyAsync(f.fci, sci.data(), sizeof(int) * nnz, hipMemcpyHostToDevice, st) !=
                  hipSuccess) ||
      (nnz && hipMemcpyAsync(perm_d, perm.data(), sizeof(int64_t) * nnz, hipMemcpyHostToDevice,
                             st) != hipSuccess) ||
      hipMemcpyAsync(dg_d, dg.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, st) !=
          hipSuccess ||
      hipMemcpyAsync(bad_d, &none, sizeof(none), hipMemcpyHostToDevice, st) != hipSuccess)
    return fail_tmp("copy of the ILU(0) pattern failed");
  if (!(e = upload(st, f, tmp, n, f.lo, lo, true, &lmap, &unused, &lemap)).empty())
    return fail_tmp(e);
  if (!(e = upload(st, f, tmp, n, f.up, up, false, &umap, &pmap, &uemap)).empty())
    return fail_tmp(e);
  gather(st, nnz, perm_d, val_dev, f.fv);
  for (const IluLaunch& L : f.lo.fplan) {
    const int block = L.grid == 1 ? kIluChainThreads : kIluThreads;
    ilu_factor_kernel<<<dim3(L.grid), dim3(block), 0, st>>>(
        L.l0, L.l1, f.lo.lvl_ptr, f.lo.rows, f.frp, f.fci, dg_d, f.fv, bad_d);
  }
  gather(st, f.nnz_lo, lmap, f.fv, f.lo.v);
  gather(st, f.nnz_up, umap, f.fv, f.up.v);
  gather(st, n, pmap, f.fv, f.up.piv);
  gather(st, n * kIluEll, lemap, f.lo.v, f.lo.eval);
  gather(st, n * kIluEll, uemap, f.up.v, f.up.eval);
  unsigned long long bad = none;
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(&bad, bad_d, sizeof(bad), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail_tmp("ILU(0) factorization kernels failed");
  ilu_free(tmp);
  if (bad != none) {
    *bad_row = (int64_t)bad;
    *bad_input = true;
    return "zero or non-finite pivot in row " + std::to_string(bad);
  }
  return "";
}

void launch_ilu_apply(hipStream_t st, const IluFactors& f, int s, const double* Y, double* Z,
                      const Ctl* ctl, KTimer* tm) {
  launch_sweep<true>(st, f.lo, s, Y, Z, ctl, tm);
  launch_sweep<false>(st, f.up, s, Z, Z, ctl, tm);
}

}  // namespace lsba
