// Small dense kernels off the basis path: the per-column QR update, residual
// estimate and convergence test (with, for Alg. 7, the H column and the J
// recurrence), the end of a cycle, and the loss-of-orthogonality record.
#include "small_common.h"

namespace lsba {

namespace {

// LDS layout of small_side when everything fits (in the order the sources are
// gathered): the column [J; R] (k s x s), Y, Z ((k-1) s x s each), P, R^{-1},
// T2 (k s x s), then at least one column block of H staged per chunk.
__host__ __device__ inline bool side_fits(int s, int k) {
  const int ss = s * s, r0 = (k - 1) * s, ks = k * s;
  const int fixed = ks * s + 2 * r0 * s + 2 * ss + ks * s;
  const int fin = 16 * ss;   // finalize_lds_min
  return fixed + r0 * s <= LDS_DBL && ks * s + fin <= LDS_DBL;
}

// Alg. 7 off the basis path, after loop step k >= 2 (queued on a second
// stream behind small_core of the same step): H_{1:k-1,k-1} = J + Y, for
// k <= m the J recurrence J = ([Z; P] - H_{1:k,1:k-1} Y) R^{-1}, then column
// k-1 is final and goes through finalize_column.  It reads only this step's
// slots (Gram output, R^{-1}, P) and H, J, so it may lag the basis kernels.
// FIT: all operands in LDS (one batched gather); otherwise they live in
// global scratch slots that no basis-path kernel uses.
template <bool FIT, bool FIN>
__global__ __launch_bounds__(NT) void small_side_kernel(Dense d, int k, int m) {
  __shared__ double lds[LDS_DBL];
  Ctl* ctl = d.ctl;
  {
    const int st = ctl->status;
    if (st == ST_CONVERGED || st == ST_ITERCAP) return;
    if (st == ST_FLAGGED && ctl->flag_step <= k) return;
  }
  const int s = d.s, ld = d.ldh, ss = s * s;
  const bool last = (k == m + 1);
  const int ldg = last ? s : 2 * s;
  const int r0 = (k - 1) * s, ks = k * s;
  const int c1 = (k - 2) * s;   // first column of block column k-1
  const double* Gk = d.G + (int64_t)k * d.gstride;
  const Scr sc = make_scr(d);
  double* col;
  double* Yl;
  double* Zl;
  double* Pl;
  double* Ril;
  double* T2;
  double* Hs;
  int hcap;
  if constexpr (FIT) {
    col = lds;
    Yl = col + ks * s;
    Zl = Yl + r0 * s;
    Pl = Zl + r0 * s;
    Ril = Pl + ss;
    T2 = Ril + ss;
    Hs = T2 + ks * s;
    hcap = LDS_DBL - (int)(Hs - lds);
  } else {
    col = sc.bg(7);
    Yl = sc.bg(4);
    Zl = sc.bg(5);
    T2 = sc.bg(6);
    Pl = sc.bg(4) + (int64_t)d.mmax * ss;
    Ril = Pl + ss;
    Hs = lds;
    hcap = LDS_DBL;
  }
  // gather J, R = H_{k,k-1}, Y, Z, P, R^{-1}: element e of the sequence
  const int nJ = r0 * s, nY = r0 * s, nZ = last ? 0 : r0 * s, nP = last ? 0 : ss;
  const int eR = nJ, eY = eR + ss, eZ = eY + nY, eP = eZ + nZ, eRi = eP + nP;
  const int tot = eRi + nP;
  auto src = [&](int e) -> const double* {
    if (e < eR) return d.J + e;
    if (e < eY) return d.H + (int64_t)(r0 + (e - eR) / s) * ld + c1 + (e - eR) % s;
    if (e < eZ) return Gk + (int64_t)((e - eY) / s) * ldg + (e - eY) % s;
    if (e < eP) return Gk + (int64_t)((e - eZ) / s) * ldg + s + (e - eZ) % s;
    if (e < eRi) return d.PS + (int64_t)k * ss + (e - eP);
    return d.RiS + (int64_t)k * ss + (e - eRi);
  };
  auto dst = [&](int e) -> double* {
    if constexpr (FIT) {
      // col, Yl, Zl, Pl, Ril are contiguous in gather order; with no Z the
      // P and R^{-1} slots are skipped (unused on the last step)
      return lds + e;
    } else {
      if (e < eY) return col + e;
      if (e < eZ) return Yl + (e - eY);
      if (e < eP) return Zl + (e - eZ);
      if (e < eRi) return Pl + (e - eP);
      return Ril + (e - eRi);
    }
  };
  for (int base = threadIdx.x; base < tot; base += NT * 16) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = base + u * NT;
      v[u] = *src(e < tot ? e : tot - 1);
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = base + u * NT;
      if (e < tot) *dst(e) = v[u];
    }
  }
  bar();
  // H_{1:k-1,k-1} = J + Y
  for (int e = threadIdx.x; e < r0 * s; e += NT) {
    const double v = col[e] + Yl[e];
    col[e] = v;
    d.H[(int64_t)(e / s) * ld + c1 + (e % s)] = v;
  }
  bar();
  if (!last) {
    // T2 = [Z; P] - H_{1:k,1:k-1} Y.  First the last column block (in col:
    // J + Y above, R below), then H_{1:k-1,1:k-2} from global memory, staged
    // in LDS a few column blocks at a time; row block rb has nonzeros from
    // column block rb - 1 on.
    const double* Ylast = Yl + (int64_t)c1 * s;
    for (int e = threadIdx.x; e < ks * s; e += NT) {
      const int a = e / s, c = e % s;
      double acc = a < r0 ? Zl[e] : Pl[e - r0 * s];
#pragma unroll 8
      for (int t = 0; t < s; ++t) acc = fma(-col[a * s + t], Ylast[t * s + c], acc);
      T2[e] = acc;
    }
    const int nbc = k - 2;   // column blocks of the global part
    if constexpr (FIT) {
      for (int cb0 = 0; cb0 < nbc;) {
        int cb1 = cb0 + 1;
        auto rows_of = [&](int cbe) { return (cbe + 1) * s < r0 ? (cbe + 1) * s : r0; };
        while (cb1 < nbc && rows_of(cb1 + 1) * (cb1 + 1 - cb0) * s <= hcap) ++cb1;
        const int nrows = rows_of(cb1), w = (cb1 - cb0) * s, t0 = cb0 * s;
        const int ntot = nrows * w;
        bar();   // previous chunk consumed (and T2 initialised)
        for (int base = threadIdx.x; base < ntot; base += NT * 16) {
          double v[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            int e = base + u * NT;
            e = e < ntot ? e : ntot - 1;
            const int a = e / w, t = t0 + e % w;
            v[u] = d.H[(int64_t)a * ld + t];
            const int lo = (a / s > 1 ? a / s - 1 : 0) * s;
            v[u] = t >= lo ? v[u] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            const int e = base + u * NT;
            if (e < ntot) Hs[e] = v[u];
          }
        }
        bar();
        for (int e = threadIdx.x; e < nrows * s; e += NT) {
          const int a = e / s, c = e % s;
          const double* hr = Hs + a * w;
          const double* yc = Yl + (int64_t)t0 * s + c;
          double a0 = 0.0, a1 = 0.0;
          int t = 0;
#pragma unroll 4
          for (; t + 1 < w; t += 2) {
            a0 = fma(hr[t], yc[t * s], a0);
            a1 = fma(hr[t + 1], yc[(t + 1) * s], a1);
          }
          if (t < w) a0 = fma(hr[t], yc[t * s], a0);
          T2[e] -= a0 + a1;
        }
        cb0 = cb1;
      }
    } else {
      // operands in global memory: row a against the columns of its band
      bar();
      for (int e = threadIdx.x; e < r0 * s; e += NT) {
        const int a = e / s, c = e % s;
        const int lo = (a / s > 1 ? a / s - 1 : 0) * s;
        const double* hr = d.H + (int64_t)a * ld;
        double a0 = 0.0, a1 = 0.0;
        int t = lo;
#pragma unroll 4
        for (; t + 1 < c1; t += 2) {
          a0 = fma(hr[t], Yl[t * s + c], a0);
          a1 = fma(hr[t + 1], Yl[(t + 1) * s + c], a1);
        }
        if (t < c1) a0 = fma(hr[t], Yl[t * s + c], a0);
        T2[e] -= a0 + a1;
      }
    }
    bar();
    // J = T2 R^{-1}
    rows_x_small(ks, s, T2, s, Ril, 1.0, d.J, s);
    bar();
  }
  if constexpr (FIN)
    finalize_column(d, k - 1, FIT ? lds + ks * s : lds, FIT ? LDS_DBL - ks * s : LDS_DBL, col, s);
}

// Column `col` of H is final: QR update, estimate, convergence test.  Runs
// after the skeleton step that finalised the column, possibly while the basis
// kernels of the next steps are already running; it does nothing once the
// cycle has converged or hit the iteration cap, and nothing for columns past
// a Cholesky flag.
__global__ __launch_bounds__(NT) void small_finalize_kernel(Dense d, int col) {
  __shared__ double lds[LDS_DBL];
  Ctl* ctl = d.ctl;
  const int st = ctl->status;
  if (st == ST_CONVERGED || st == ST_ITERCAP) return;
  if (col > ctl->last_valid) return;
  finalize_column(d, col, lds, LDS_DBL, d.H + (int64_t)(col - 1) * d.s, d.ldh);
}

// End of a cycle: Xi, M, the cospatial factor, the basis-application
// coefficients and the adaptive restart bookkeeping.
__global__ __launch_bounds__(NT) void small_cycle_end_kernel(Dense d) {
  const Scr sc = make_scr(d);
  Ctl* ctl = d.ctl;
  const int s = d.s, ld = d.ldh, ss = s * s;
  CoefLayout lay{s, d.mmax + 1};
  const int j = ctl->j;
  const int status = ctl->status;
  if (threadIdx.x == 0) {
    ctl->cycles += 1;
    ctl->cyc_status = status;
  }
  if (j == 0) {
    // nothing to apply: nv1 = -1 tells the basis application to leave X and U alone
    if (threadIdx.x == 0) {
      ctl->nv1 = -1;
      ctl->nv2_begin = 0;
      ctl->nv2 = 0;
      ctl->cont = 0;
      ctl->stop = 1;
    }
    return;
  }
  const int js = j * s, c0 = (j - 1) * s;
  double* Xi = d.Xi;
  // last block of Xi
  if (d.method == LSBA_FOM) {
    copy(s, s, d.ylast, s, Xi + (int64_t)c0 * s, s);
  } else {
    copy(s, s, d.g + (int64_t)c0 * s, s, Xi + (int64_t)c0 * s, s);
    tri_solve_up(d.Rf + (int64_t)c0 * ld + c0, ld, s, Xi + (int64_t)c0 * s, s, s);
  }
  // block back substitution with the triangular factor
  for (int b = j - 1; b >= 1; --b) {
    const int rb = (b - 1) * s;
    double* xb = Xi + (int64_t)rb * s;
    copy(s, s, d.g + (int64_t)rb * s, s, xb, s);
    mm(s, s, js - (rb + s), -1.0, d.Rf + (int64_t)rb * ld + rb + s, ld, false,
       Xi + (int64_t)(rb + s) * s, s, false, 1.0, xb, s);
    tri_solve_up(d.Rf + (int64_t)rb * ld + rb, ld, s, xb, s, s);
  }
  const bool final_ = (status == ST_CONVERGED || status == ST_ITERCAP);
  // X += V_{1:j} Xi
  set_coef_identity(d, lay.C1());
  copy(js, s, Xi, s, d.coef64 + lay.A(0), s);
  const double* Hsub = d.H + (int64_t)js * ld + c0;
  int nvb = 0, nve = 0;
  if (!final_) {
    if (d.method == LSBA_GMRES) {
      // M = Q_1 ... Q_{j-1} E_j D^{-T} (H_{j+1,j}^T H_{j+1,j})
      double* S = sc.sm(2);
      mm(s, s, s, 1.0, Hsub, ld, true, Hsub, ld, false, 0.0, S, s);
      double* Dt = sc.sm(3);
      for (int e = threadIdx.x; e < ss; e += NT) Dt[e] = d.Dlast[(e % s) * s + (e / s)];
      bar();
      lu_solve(Dt, S, s, s);
      fill(js, s, 0.0, d.M, s);
      copy(s, s, S, s, d.M + (int64_t)c0 * s, s);
      // apply Q_i = (Q_i^T)^T to rows (i-1)s..(i+1)s, i = j-1 .. 1
      double* w2 = sc.sm(4);   // 2s x s
      for (int i = j - 1; i >= 1; --i) {
        double* Mw = d.M + (int64_t)(i - 1) * ss;
        mm(2 * s, s, 2 * s, 1.0, d.Qt + (int64_t)(i - 1) * 4 * ss, 2 * s, true, Mw, s, false,
           0.0, w2, s);
        copy(2 * s, s, w2, s, Mw, s);
      }
      copy(js, s, d.M, s, d.coef64 + lay.B(0), s);
      nvb = 0;
    } else {
      nvb = j;
    }
    set_coef(d, lay.B(j), Hsub, ld, -1.0);
    nve = j + 1;
  }
  if (threadIdx.x == 0) {
    ctl->nv1 = j;
    ctl->nv2_begin = nvb;
    ctl->nv2 = nve;
    if (status == ST_FLAGGED) ctl->m = j;
    ctl->cont = final_ ? 0 : 1;
  }
  bar();
  if (!final_) {
    copy(s, s, Xi + (int64_t)c0 * s, s, d.C, s);
    if (threadIdx.x == 0) {
      ctl->status = ST_RUNNING;
      ctl->stop = 0;
    }
  }
  publish_coef(d);
}

// Loss of orthogonality: G2 = V_{1:kn}^T V_kn is inserted into V^T V; for
// kn >= 2, ||I - V_{1:kn}^T V_{1:kn}||_2 is estimated by power iteration and
// recorded for column kn - 1.
__global__ __launch_bounds__(NT) void small_loo_kernel(Dense d, int kn) {
  Ctl* ctl = d.ctl;
  if (ctl->stop) return;
  const Scr sc = make_scr(d);
  const int s = d.s, ld = d.ldh;
  const int N = kn * s, c0 = (kn - 1) * s;
  for (int e = threadIdx.x; e < N * s; e += NT) {
    const int i = e / s, c = e % s;
    const double v = d.G2[e];
    d.Gv[(int64_t)i * ld + c0 + c] = v;
    d.Gv[(int64_t)(c0 + c) * ld + i] = v;
  }
  bar();
  if (kn < 2) return;
  double* x = sc.bg(0);
  double* y = sc.bg(1);
  for (int i = threadIdx.x; i < N; i += NT) x[i] = 1.0 + 1e-3 * (double)i / (double)N;
  bar();
  double nx = frob(N, 1, x, 1);
  for (int i = threadIdx.x; i < N; i += NT) x[i] /= nx;
  bar();
  double lam = 0.0;
  for (int it = 0; it < 100; ++it) {
    for (int i = threadIdx.x; i < N; i += NT) {
      double acc = 0.0;
      for (int t = 0; t < N; ++t) {
        const double e = ((i == t) ? 1.0 : 0.0) - d.Gv[(int64_t)i * ld + t];
        acc = fma(e, x[t], acc);
      }
      y[i] = acc;
    }
    bar();
    lam = frob(N, 1, y, 1);
    if (!(lam > 0.0)) break;
    for (int i = threadIdx.x; i < N; i += NT) x[i] = y[i] / lam;
    bar();
  }
  if (threadIdx.x == 0) d.loo_hist[kn - 2] = lam;
}

}  // namespace

#define SMALL_LAUNCH(...)                 \
  do {                                    \
    if (tm) tm->begin(st, KK_SMALL);      \
    __VA_ARGS__;                          \
    if (tm) tm->end(st, KK_SMALL, 0.0);   \
  } while (0)

void launch_small_side(hipStream_t st, const Dense& d, int k, int m, bool with_finalize,
                       KTimer* tm) {
  const bool fit = side_fits(d.s, k);
  if (with_finalize) {
    if (fit) SMALL_LAUNCH(small_side_kernel<true, true><<<1, NT, 0, st>>>(d, k, m));
    else SMALL_LAUNCH(small_side_kernel<false, true><<<1, NT, 0, st>>>(d, k, m));
  } else {
    if (fit) SMALL_LAUNCH(small_side_kernel<true, false><<<1, NT, 0, st>>>(d, k, m));
    else SMALL_LAUNCH(small_side_kernel<false, false><<<1, NT, 0, st>>>(d, k, m));
  }
}
void launch_small_finalize(hipStream_t st, const Dense& d, int col, KTimer* tm) {
  SMALL_LAUNCH(small_finalize_kernel<<<1, NT, 0, st>>>(d, col));
}
void launch_small_cycle_end(hipStream_t st, const Dense& d, KTimer* tm) {
  SMALL_LAUNCH(small_cycle_end_kernel<<<1, NT, 0, st>>>(d));
}
void launch_small_loo(hipStream_t st, const Dense& d, int k_new_block, KTimer* tm) {
  SMALL_LAUNCH(small_loo_kernel<<<1, NT, 0, st>>>(d, k_new_block));
}

}  // namespace lsba
