// Small dense steps of the block Arnoldi cycle, in FP64, one workgroup per
// solve.  They consume the reduced Gram products and produce
//   - the Cholesky factors with the breakdown flag (Sec. 4, the NaN-flag),
//   - the skeleton's small updates: Omega, P, J and H (Alg. 7), T and H
//     (Algs. 5, 6),
//   - the coefficients of the next fused block update,
//   - for every final block column j: a progressive block Householder QR of
//     the block Hessenberg H_{1:j+1,1:j} (one 2s x s window per column), the
//     residual estimate of eq. normF_Rm and the convergence test,
//   - at the end of a cycle: Xi (eq. Xm), the BGMRES factor M, the cospatial
//     factor E_j^T Xi_j and the coefficients of X += V Xi and
//     U = V_{1:j+1} [M; -H_{j+1,j}] (Thm. 1).
//
// BGMRES is computed as the least-squares problem
// min ||E_1 B C - H_{j+1,j} Xi||_F, which equals the modified BFOM of eq. Xm
// in exact arithmetic; its residual is the bottom block of the transformed
// right-hand side.  BFOM uses the same QR: after the reflectors of columns
// 1..j-1, H_j is block upper triangular with a full last diagonal block D, so
// the last block of Xi is D^{-1} g_j and the estimate is ||H_{j+1,j} D^{-1} g_j||_F.
// The BGMRES factor M = H_j^{-T} E_j H_{j+1,j}^T H_{j+1,j} becomes
// Q_1 ... Q_{j-1} E_j D^{-T} (H_{j+1,j}^T H_{j+1,j}).
//
// Latency is what matters here: each column's orthogonal factor is kept as an
// explicit 2s x 2s matrix Q_i^T, so bringing a new column through the i-1
// earlier windows costs one small product and one barrier per window; the
// factors are prefetched into LDS (all of them when they fit, else a
// double-buffered ring), and small products split their reduction across
// threads when they have few outputs.
#include "lsba_internal.h"

namespace lsba {

namespace {

constexpr int NT = kSmallThreads;
constexpr int LDS_DBL = 18944;     // 148 KiB of LDS per workgroup
constexpr int G_LDS_MAX = 6144;    // Gram output staged in LDS when it is at most this size

struct Scr {
  double* base;
  int s;
  int64_t big;
  __device__ double* sm(int i) const { return base + (int64_t)i * s * s; }
  __device__ double* bg(int i) const { return base + (int64_t)64 * s * s + (int64_t)i * big; }
};

__device__ __forceinline__ Scr make_scr(const Dense& d) {
  Scr sc;
  sc.base = d.scratch;
  sc.s = d.s;
  sc.big = (int64_t)(d.mmax + 2) * d.s * d.s;
  return sc;
}

__device__ __forceinline__ void bar() { __syncthreads(); }

__device__ double wg_sum(double v) {
  __shared__ double sh[NT / 64];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  bar();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) t += sh[i];
  bar();
  return t;
}

// Y (M x N) = alpha * op(A) op(B) + beta * Y ; op(A) is M x K.  With few
// outputs the reduction over K is split across threads (fixed order of the
// partial sums, so the result does not depend on timing).
__device__ void mm(int M, int N, int K, double alpha, const double* A, int lda, bool tA,
                   const double* B, int ldb, bool tB, double beta, double* Y, int ldy) {
  __shared__ double red[NT];
  const int outs = M * N;
  int ks = 1;
  while (ks * 2 * outs <= NT && ks * 2 <= K && ks < 64) ks *= 2;
  if (ks == 1) {
    for (int e = threadIdx.x; e < outs; e += NT) {
      const int i = e / N, j = e % N;
      double acc = 0.0;
      for (int t = 0; t < K; ++t) {
        const double av = tA ? A[(int64_t)t * lda + i] : A[(int64_t)i * lda + t];
        const double bv = tB ? B[(int64_t)j * ldb + t] : B[(int64_t)t * ldb + j];
        acc = fma(av, bv, acc);
      }
      double* y = Y + (int64_t)i * ldy + j;
      *y = (beta == 0.0 ? 0.0 : beta * *y) + alpha * acc;
    }
    bar();
    return;
  }
  const int t = threadIdx.x;
  if (t < outs * ks) {
    const int e = t % outs, q = t / outs;
    const int i = e / N, j = e % N;
    const int k0 = (int)((int64_t)K * q / ks), k1 = (int)((int64_t)K * (q + 1) / ks);
    double acc = 0.0;
    for (int tt = k0; tt < k1; ++tt) {
      const double av = tA ? A[(int64_t)tt * lda + i] : A[(int64_t)i * lda + tt];
      const double bv = tB ? B[(int64_t)j * ldb + tt] : B[(int64_t)tt * ldb + j];
      acc = fma(av, bv, acc);
    }
    red[t] = acc;
  }
  bar();
  if (t < outs) {
    const int i = t / N, j = t % N;
    double acc = 0.0;
    for (int q = 0; q < ks; ++q) acc += red[q * outs + t];
    double* y = Y + (int64_t)i * ldy + j;
    *y = (beta == 0.0 ? 0.0 : beta * *y) + alpha * acc;
  }
  bar();
}

__device__ void copy(int M, int N, const double* A, int lda, double* Y, int ldy) {
  for (int e = threadIdx.x; e < M * N; e += NT) {
    const int i = e / N, j = e % N;
    Y[(int64_t)i * ldy + j] = A[(int64_t)i * lda + j];
  }
  bar();
}

__device__ void fill(int M, int N, double v, double* Y, int ldy) {
  for (int e = threadIdx.x; e < M * N; e += NT) {
    const int i = e / N, j = e % N;
    Y[(int64_t)i * ldy + j] = v;
  }
  bar();
}

__device__ double frob(int M, int N, const double* A, int lda) {
  double v = 0.0;
  for (int e = threadIdx.x; e < M * N; e += NT) {
    const double x = A[(int64_t)(e / N) * lda + (e % N)];
    v += x * x;
  }
  return sqrt(wg_sum(v));
}

// Upper Cholesky factor R (ld s) of Om + shift I (upper triangle of Om read).
// Returns false (the breakdown flag) when a pivot is not a positive finite number.
__device__ bool chol_up(const double* Om, int ldo, double* R, int s, double shift) {
  __shared__ int okf;
  for (int e = threadIdx.x; e < s * s; e += NT) {
    const int i = e / s, j = e % s;
    R[e] = (j >= i) ? Om[(int64_t)i * ldo + j] + (i == j ? shift : 0.0) : 0.0;
  }
  bar();
  for (int j = 0; j < s; ++j) {
    if (threadIdx.x == 0) {
      double dd = R[j * s + j];
      for (int i = 0; i < j; ++i) dd -= R[i * s + j] * R[i * s + j];
      const int ok = (dd > 0.0) && isfinite(dd);
      okf = ok;
      R[j * s + j] = ok ? sqrt(dd) : 0.0;
    }
    bar();
    if (!okf) return false;
    const double rjj = R[j * s + j];
    for (int l = j + 1 + threadIdx.x; l < s; l += NT) {
      double v = R[j * s + l];
      for (int i = 0; i < j; ++i) v -= R[i * s + j] * R[i * s + l];
      R[j * s + l] = v / rjj;
    }
    bar();
  }
  return true;
}

// Cholesky with the mixed form's shifted fallback: if the plain factorization
// flags, retry with Om + sigma I, sigma = 10 u_fp32 trace(Om).
__device__ bool chol_flag(const Dense& d, const double* Om, int ldo, double* R) {
  const int s = d.s;
  bool ok = chol_up(Om, ldo, R, s, 0.0);
  if (!ok && d.mixed) {
    double tr = 0.0;
    for (int i = 0; i < s; ++i) tr += fabs(Om[(int64_t)i * ldo + i]);
    ok = chol_up(Om, ldo, R, s, 10.0 * 5.9604644775390625e-08 * tr);
  }
  return ok;
}

// Ri = R^{-1} for upper-triangular R (s x s).
__device__ void tri_inv_up(const double* R, int s, double* Ri) {
  for (int c = threadIdx.x; c < s; c += NT) {
    for (int i = s - 1; i >= 0; --i) {
      if (i > c) {
        Ri[i * s + c] = 0.0;
        continue;
      }
      double v = (i == c) ? 1.0 : 0.0;
      for (int l = i + 1; l <= c; ++l) v -= R[i * s + l] * Ri[l * s + c];
      Ri[i * s + c] = v / R[i * s + i];
    }
  }
  bar();
}

// X (s x nrhs, ld ldx) <- R^{-1} X for upper-triangular R (ld ldr).
__device__ void tri_solve_up(const double* R, int ldr, int s, double* X, int ldx, int nrhs) {
  for (int q = threadIdx.x; q < nrhs; q += NT) {
    for (int i = s - 1; i >= 0; --i) {
      double v = X[(int64_t)i * ldx + q];
      for (int l = i + 1; l < s; ++l) v -= R[(int64_t)i * ldr + l] * X[(int64_t)l * ldx + q];
      X[(int64_t)i * ldx + q] = v / R[(int64_t)i * ldr + i];
    }
  }
  bar();
}

// Solve A X = Bm (A: s x s, destroyed; Bm: s x nrhs, overwritten with X) by
// LU with partial pivoting.  Returns false for an exactly singular or
// non-finite pivot.
__device__ bool lu_solve(double* A, double* Bm, int s, int nrhs) {
  __shared__ int piv, okf;
  for (int k = 0; k < s; ++k) {
    if (threadIdx.x == 0) {
      int p = k;
      double best = fabs(A[k * s + k]);
      for (int i = k + 1; i < s; ++i) {
        const double v = fabs(A[i * s + k]);
        if (v > best) {
          best = v;
          p = i;
        }
      }
      piv = p;
      okf = (best > 0.0) && isfinite(best);
    }
    bar();
    if (!okf) return false;
    const int p = piv;
    if (p != k) {
      for (int c = threadIdx.x; c < s + nrhs; c += NT) {
        if (c < s) {
          const double t = A[k * s + c];
          A[k * s + c] = A[p * s + c];
          A[p * s + c] = t;
        } else {
          const int q = c - s;
          const double t = Bm[k * nrhs + q];
          Bm[k * nrhs + q] = Bm[p * nrhs + q];
          Bm[p * nrhs + q] = t;
        }
      }
      bar();
    }
    const int rem = s - k - 1, wid = rem + nrhs;
    const double akk = A[k * s + k];
    for (int e = threadIdx.x; e < rem * wid; e += NT) {
      const int i = k + 1 + e / wid, c = e % wid;
      const double l = A[i * s + k] / akk;
      if (c < rem) {
        const int jj = k + 1 + c;
        A[i * s + jj] -= l * A[k * s + jj];
      } else {
        const int q = c - rem;
        Bm[i * nrhs + q] -= l * Bm[k * nrhs + q];
      }
    }
    bar();
  }
  tri_solve_up(A, s, s, Bm, nrhs, nrhs);
  return true;
}

// Householder QR of the 2s x s window W (ld s, in LDS): W <- [R; 0] and
// Qt (2s x 2s, ld 2s) = Q^T with Q = I - Y T Y^T.  Y, T, tmp are LDS scratch
// (2s x s, s x s, >= 2s x s).
__device__ void window_qr(double* W, int s, double* Qt, double* Y, double* Tq, double* tmp) {
  __shared__ double hh[3];
  const int m2 = 2 * s;
  for (int e = threadIdx.x; e < m2 * s; e += NT) Y[e] = 0.0;
  for (int e = threadIdx.x; e < s * s; e += NT) Tq[e] = 0.0;
  bar();
  for (int c = 0; c < s; ++c) {
    if (threadIdx.x == 0) {
      const double alpha = W[c * s + c];
      double xn2 = 0.0;
      for (int i = c + 1; i < m2; ++i) xn2 += W[i * s + c] * W[i * s + c];
      if (xn2 == 0.0) {
        hh[0] = 0.0;
        hh[1] = alpha;
        hh[2] = 0.0;
      } else {
        const double beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
        hh[0] = (beta - alpha) / beta;
        hh[1] = beta;
        hh[2] = 1.0 / (alpha - beta);
      }
    }
    bar();
    const double tau = hh[0], beta = hh[1], scale = hh[2];
    for (int i = threadIdx.x; i < m2; i += NT)
      Y[i * s + c] = (i < c) ? 0.0 : (i == c ? 1.0 : W[i * s + c] * scale);
    bar();
    for (int q = c + 1 + threadIdx.x; q < s; q += NT) {
      double w = 0.0;
      for (int i = c; i < m2; ++i) w += Y[i * s + c] * W[i * s + q];
      w *= tau;
      for (int i = c; i < m2; ++i) W[i * s + q] -= w * Y[i * s + c];
    }
    // T(0:c, c) = -tau T(0:c, 0:c) (Y(:, 0:c)^T v_c)
    for (int i = threadIdx.x; i < c; i += NT) {
      double v = 0.0;
      for (int r = c; r < m2; ++r) v += Y[r * s + i] * Y[r * s + c];
      tmp[i] = v;
    }
    bar();
    for (int i = c + threadIdx.x; i < m2; i += NT) W[i * s + c] = (i == c) ? beta : 0.0;
    for (int i = threadIdx.x; i < c; i += NT) {
      double v = 0.0;
      for (int l = i; l < c; ++l) v += Tq[i * s + l] * tmp[l];
      Tq[i * s + c] = -tau * v;
    }
    if (threadIdx.x == 0) Tq[c * s + c] = tau;
    bar();
  }
  // Q^T = I - Y T^T Y^T: tmp (s x 2s) = T^T Y^T, then Qt = I - Y tmp
  for (int e = threadIdx.x; e < s * m2; e += NT) {
    const int a = e / m2, r = e % m2;
    double v = 0.0;
    for (int l = 0; l <= a; ++l) v += Tq[l * s + a] * Y[r * s + l];
    tmp[e] = v;
  }
  bar();
  for (int e = threadIdx.x; e < m2 * m2; e += NT) {
    const int r = e / m2, c = e % m2;
    double v = 0.0;
    for (int a = 0; a < s; ++a) v += Y[r * s + a] * tmp[a * m2 + c];
    Qt[e] = (r == c ? 1.0 : 0.0) - v;
  }
  bar();
}

// Write an s x s block (scaled) into the coefficient array.
__device__ void set_coef(const Dense& d, int off, const double* src, int lds, double scale) {
  const int s = d.s;
  for (int e = threadIdx.x; e < s * s; e += NT)
    d.coef64[off + e] = scale * src[(int64_t)(e / s) * lds + (e % s)];
  bar();
}
__device__ void set_coef_identity(const Dense& d, int off) {
  const int s = d.s;
  for (int e = threadIdx.x; e < s * s; e += NT) d.coef64[off + e] = (e / s == e % s) ? 1.0 : 0.0;
  bar();
}

// Mixed form: the block updates read float coefficients.
__device__ void publish_coef(const Dense& d) {
  if (!d.mixed) return;
  CoefLayout lay{d.s, d.mmax + 1};
  float* f = (float*)d.coefT;
  const int tot = lay.total();
  for (int e = threadIdx.x; e < tot; e += NT) f[e] = (float)d.coef64[e];
  bar();
}

// LDS doubles finalize_column needs at least (ring of two slots).
__device__ __forceinline__ int finalize_lds_min(int s) { return 13 * s * s; }

// Column j (1-based) of H is final: bring it through the orthogonal factors of
// columns 1..j-1, factor its window, record the residual estimate, test
// convergence.  `lds` holds nl >= finalize_lds_min(s) doubles of workspace.
__device__ void finalize_column(const Dense& d, int j, double* lds, int nl) {
  const int s = d.s, ld = d.ldh, ss = s * s, q4 = 4 * ss;
  const int c0 = (j - 1) * s;
  Ctl* ctl = d.ctl;
  const double* Hc = d.H + c0;   // column block j (row-major, ld)
  double* Rfc = d.Rf + c0;
  // LDS carve-up: two carry blocks, then a region that holds the ring of
  // (Q_i^T, block row i+1) items during the chain and the window-QR buffers
  // after it.
  double* carry0 = lds;            // ss
  double* carry1 = carry0 + ss;    // ss
  double* ring = carry1 + ss;      // chain: slots of (Q^T: q4, block of h: ss)
  double* qw = ring;               // after: 2ss  [D; H_{j+1,j}] window
  double* Yw = qw + 2 * ss;        //        2ss
  double* Tw = Yw + 2 * ss;        //        ss
  double* tmp = Tw + ss;           //        4ss  (LU scratch, then Q_j^T)
  double* gw = tmp + q4;           //        2ss  (QR scratch, then g window)
  const int slot_sz = q4 + ss;
  const int nslots_fit = (nl - 2 * ss) / slot_sz;
  const int nap = j - 1;
  const bool all = nslots_fit >= nap;
  const int R = all ? (nap > 0 ? nap : 1) : 2;

  // carry <- first block row of the column
  for (int e = threadIdx.x; e < ss; e += NT) carry0[e] = Hc[(int64_t)(e / s) * ld + (e % s)];
  auto item_elem = [&](int i, int e) -> double {   // element e of item i (1-based window)
    if (e < q4) return d.Qt[(int64_t)(i - 1) * q4 + e];
    const int f = e - q4;
    return Hc[(int64_t)(i * s + f / s) * ld + (f % s)];
  };
  if (nap > 0) {
    // items 1..npre go to slots 0..npre-1 (contiguous); loads are batched so
    // that many are in flight at once
    const int npre = all ? nap : 1;
    const int tot = npre * slot_sz;
    for (int base = threadIdx.x; base < tot; base += NT * 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = base + u * NT;
        v[u] = e < tot ? item_elem(e / slot_sz + 1, e % slot_sz) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = base + u * NT;
        if (e < tot) ring[e] = v[u];
      }
    }
  }
  bar();
  constexpr int PF = 5 * kMaxS * kMaxS / NT;   // prefetch registers per thread (ring mode)
  double pf[PF];
  double* cur = carry0;
  double* nxt = carry1;
  const int m2 = 2 * s;
  for (int i = 1; i <= nap; ++i) {
    const bool prefetch = !all && i + 1 <= nap;
    if (prefetch) {
#pragma unroll
      for (int r = 0; r < PF; ++r) {
        const int e = threadIdx.x + r * NT;
        pf[r] = e < slot_sz ? item_elem(i + 1, e) : 0.0;
      }
    }
    const double* sl = ring + (int64_t)((i - 1) % R) * slot_sz;
    const double* Q = sl;              // 2s x 2s
    const double* hb = sl + q4;        // s x s, block row i+1 of the column
    for (int e = threadIdx.x; e < m2 * s; e += NT) {
      const int r = e / s, c = e % s;
      double acc = 0.0;
      for (int t = 0; t < s; ++t) acc = fma(Q[r * m2 + t], cur[t * s + c], acc);
      for (int t = 0; t < s; ++t) acc = fma(Q[r * m2 + s + t], hb[t * s + c], acc);
      if (r < s)
        Rfc[(int64_t)((i - 1) * s + r) * ld + c] = acc;   // final block row i
      else
        nxt[(r - s) * s + c] = acc;                       // carry: block row i+1
    }
    if (prefetch) {
      double* sn = ring + (int64_t)(i % R) * slot_sz;
#pragma unroll
      for (int r = 0; r < PF; ++r) {
        const int e = threadIdx.x + r * NT;
        if (e < slot_sz) sn[e] = pf[r];
      }
    }
    bar();
    double* t = cur;
    cur = nxt;
    nxt = t;
  }
  // D = cur; window [D; H_{j+1,j}] (the ring is free now)
  const double* Hsub = Hc + (int64_t)(j * s) * ld;
  for (int e = threadIdx.x; e < ss; e += NT) {
    d.Dlast[e] = cur[e];
    qw[e] = cur[e];
    qw[ss + e] = Hsub[(int64_t)(e / s) * ld + (e % s)];
  }
  bar();
  double est = 0.0;
  if (d.method == LSBA_FOM) {
    // last block of Xi: D^{-1} g_j ; estimate ||H_{j+1,j} D^{-1} g_j||_F
    double* A = tmp;
    double* Bm = tmp + ss;
    for (int e = threadIdx.x; e < ss; e += NT) {
      A[e] = cur[e];
      Bm[e] = d.g[(int64_t)c0 * s + e];
    }
    bar();
    if (lu_solve(A, Bm, s, s)) {
      double* HY = tmp + 2 * ss;
      for (int e = threadIdx.x; e < ss; e += NT) {
        d.ylast[e] = Bm[e];
        const int i = e / s, c = e % s;
        double acc = 0.0;
        for (int t = 0; t < s; ++t) acc = fma(qw[ss + i * s + t], Bm[t * s + c], acc);
        HY[e] = acc;
      }
      bar();
      est = frob(s, s, HY, s);
    } else {
      for (int e = threadIdx.x; e < ss; e += NT) d.ylast[e] = 0.0;
      bar();
      est = INFINITY;
    }
  }
  double* Qj = tmp;
  window_qr(qw, s, Qj, Yw, Tw, gw);
  for (int e = threadIdx.x; e < 2 * ss; e += NT) gw[e] = d.g[(int64_t)c0 * s + e];
  bar();
  // R_jj -> Rf, Q_j^T -> global, g window <- Q_j^T g window
  for (int e = threadIdx.x; e < ss; e += NT)
    Rfc[(int64_t)(c0 + e / s) * ld + (e % s)] = qw[e];
  for (int e = threadIdx.x; e < q4; e += NT) d.Qt[(int64_t)(j - 1) * q4 + e] = Qj[e];
  for (int e = threadIdx.x; e < 2 * ss; e += NT) {
    const int r = e / s, c = e % s;
    double acc = 0.0;
    for (int t = 0; t < m2; ++t) acc = fma(Qj[r * m2 + t], gw[t * s + c], acc);
    d.g[(int64_t)c0 * s + e] = acc;
    if (r >= s) carry1[(r - s) * s + c] = acc;
  }
  bar();
  if (d.method == LSBA_GMRES) est = frob(s, s, carry1, s);
  if (threadIdx.x == 0) {
    const double rel = est / ctl->nB;
    d.res_hist[j - 1] = rel;
    ctl->j = j;
    ctl->iter += 1;
    ctl->est = rel;
    // convergence or the iteration cap at column j wins over a Cholesky flag
    // raised at a later step that the basis kernels may have reached meanwhile
    if (rel <= ctl->tol) {
      atomicExch(&ctl->status, (int)ST_CONVERGED);
      atomicExch(&ctl->stop, 1);
    } else if (ctl->max_iters > 0 && ctl->iter >= ctl->max_iters) {
      atomicExch(&ctl->status, (int)ST_ITERCAP);
      atomicExch(&ctl->stop, 1);
    }
  }
  bar();
}

// Batched copy of n doubles (many loads in flight per thread).
__device__ void bcopy(const double* __restrict__ src, double* __restrict__ dst, int n) {
  for (int base = threadIdx.x; base < n; base += NT * 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = base + u * NT;
      v[u] = e < n ? src[e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = base + u * NT;
      if (e < n) dst[e] = v[u];
    }
  }
}

// Raise the Cholesky flag at loop step k; `last_valid` is the last block
// column that is final.  A convergence already recorded is kept.
__device__ void raise_flag(Ctl* ctl, int k, int last_valid) {
  if (atomicCAS(&ctl->status, (int)ST_RUNNING, (int)ST_FLAGGED) == (int)ST_RUNNING) {
    ctl->flag_step = k;
    ctl->last_valid = last_valid;
  }
  atomicExch(&ctl->stop, 1);
}

// Rows 0..M-1 of Y (M x s, ld ldy) = A * B with A row-major (lda) read only
// in columns [tlo(a), K) and B (K x s, ld ldb): one thread per (row, group of
// up to 8 columns), so A is read along its rows.  Y may alias nothing.
// alpha scales the product; if Z != null, Y = Z - A*B (Z: M x s, ld ldz).
template <int CG>
__device__ void rowprod(int M, int s, int K, const double* A, int lda, int tlo_blk,
                        const double* B, int ldb, double alpha, const double* Z, int ldz,
                        double* Y, int ldy) {
  const int ng = s / CG;
  for (int w = threadIdx.x; w < M * ng; w += NT) {
    const int a = w / ng, c0 = (w % ng) * CG;
    // tlo_blk >= 0: A is block upper Hessenberg with blocks of s rows, the row
    // block rb has nonzeros from column block max(rb - tlo_blk, 0) on
    const int rb = a / s;
    const int t0 = tlo_blk >= 0 ? (rb > tlo_blk ? rb - tlo_blk : 0) * s : 0;
    double acc[CG];
#pragma unroll
    for (int c = 0; c < CG; ++c) acc[c] = 0.0;
    const double* Ar = A + (int64_t)a * lda;
    for (int t = t0; t < K; ++t) {
      const double av = Ar[t];
      const double* Br = B + (int64_t)t * ldb + c0;
#pragma unroll
      for (int c = 0; c < CG; ++c) acc[c] = fma(av, Br[c], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < CG; ++c) {
      const double v = alpha * acc[c];
      Y[(int64_t)a * ldy + c0 + c] = Z ? Z[(int64_t)a * ldz + c0 + c] - v : v;
    }
  }
  bar();
}

__device__ void rowprod_any(int M, int s, int K, const double* A, int lda, int tlo_blk,
                            const double* B, int ldb, double alpha, const double* Z, int ldz,
                            double* Y, int ldy) {
  if (s % 8 == 0) rowprod<8>(M, s, K, A, lda, tlo_blk, B, ldb, alpha, Z, ldz, Y, ldy);
  else if (s % 4 == 0) rowprod<4>(M, s, K, A, lda, tlo_blk, B, ldb, alpha, Z, ldz, Y, ldy);
  else if (s % 2 == 0) rowprod<2>(M, s, K, A, lda, tlo_blk, B, ldb, alpha, Z, ldz, Y, ldy);
  else rowprod<1>(M, s, K, A, lda, tlo_blk, B, ldb, alpha, Z, ldz, Y, ldy);
}

// Block forward substitution with a unit block lower-triangular matrix
// L = T^T (row-major Lt = Tt, ld): X_b = Rhs_b - sum_{c<b} L_{b,c} X_c for
// b = 0..k-1.  Row blocks of L are staged in LDS (`buf`, cap doubles) in
// chunks, so that each chunk costs one memory latency.  X: k s x s, ld s.
__device__ void fwd_unit(const double* Lt, int ld, const double* Rhs, int ldr, double* X, int k,
                         int s, double* buf, int cap) {
  const int ss = s * s;
  int b = 0;
  while (b < k) {
    int b1 = b, used = 0;
    while (b1 < k && used + b1 * ss <= cap) {
      used += b1 * ss;
      ++b1;
    }
    const bool staged = b1 > b;
    if (!staged) b1 = b + 1;   // one row block too large for the buffer: read it in place
    if (staged) {
      int off = 0;
      for (int c = b; c < b1; ++c) {
        const int w = c * s;   // width of row block c
        for (int base = threadIdx.x; base < s * w; base += NT * 4) {
          double v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int e = base + u * NT;
            v[u] = e < s * w ? Lt[(int64_t)(c * s + e / w) * ld + (e % w)] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int e = base + u * NT;
            if (e < s * w) buf[off + e] = v[u];
          }
        }
        off += s * w;
      }
      bar();
    }
    int off = 0;
    for (int c = b; c < b1; ++c) {
      const int w = c * s;
      copy(s, s, Rhs + (int64_t)c * s * ldr, ldr, X + (int64_t)c * ss, s);
      if (c > 0) {
        const double* Lrow = staged ? buf + off : Lt + (int64_t)(c * s) * ld;
        const int ldl = staged ? w : ld;
        mm(s, s, w, -1.0, Lrow, ldl, false, X, s, false, 1.0, X + (int64_t)c * ss, s);
      }
      off += s * w;
    }
    b = b1;
  }
}

// ------------------------------------------------------------------ kernels

__global__ __launch_bounds__(NT) void small_start_kernel(Dense d, int force) {
  __shared__ double lds[4 * kMaxS * kMaxS];
  Ctl* ctl = d.ctl;
  const int s = d.s, ld = d.ldh, ss = s * s;
  CoefLayout lay{s, d.mmax + 1};
  double* R = lds;
  double* Ri = lds + ss;
  double* G = lds + 2 * ss;
  const bool needT = d.skel != LSBA_BCGSI_LS;
  if (needT)
    for (int64_t e = threadIdx.x; e < (int64_t)ld * ld; e += NT) {
      const double v = ((e / ld) == (e % ld)) ? 1.0 : 0.0;
      d.T[e] = v;
      d.Tt[e] = v;
    }
  for (int e = threadIdx.x; e < ss; e += NT) G[e] = d.G[e];
  bar();
  bool ok = chol_flag(d, G, s, R);
  if (force) ok = false;
  if (threadIdx.x == 0) {
    ctl->j = 0;
    ctl->flag_step = -1;
    ctl->last_valid = 1 << 30;
    if (!ok) {
      ctl->status = ST_FLAGGED;
      ctl->flag_step = 0;
      ctl->last_valid = 0;
      ctl->stop = 1;
    } else {
      ctl->status = ST_RUNNING;
      ctl->stop = 0;
    }
  }
  bar();
  if (!ok) return;
  tri_inv_up(R, s, Ri);
  for (int e = threadIdx.x; e < ss; e += NT) {
    d.Beta[e] = R[e];
    d.Rinv[e] = Ri[e];
    d.coef64[lay.C1() + e] = Ri[e];
    d.coef64[lay.C2() + e] = Ri[e];
  }
  for (int e = threadIdx.x; e < (d.mmax + 1) * ss; e += NT) d.g[e] = 0.0;
  bar();
  mm(s, s, s, 1.0, R, s, false, d.C, s, false, 0.0, d.g, s);
  publish_coef(d);
}

// Algs. 6 (CWY / ICWY) and 7 (BCGSI+LS), loop step k (1-based); m is the
// current basis size, so k = m + 1 only forms V_{m+1}.  Column k-1 of H is
// final after this kernel; its QR update and the convergence test are done by
// small_finalize.
__global__ __launch_bounds__(NT) void small_delayed_kernel(Dense d, int k, int m, int force) {
  __shared__ double lds[LDS_DBL];
  Ctl* ctl = d.ctl;
  if (ctl->stop) return;
  const int s = d.s, ld = d.ldh, ss = s * s;
  CoefLayout lay{s, d.mmax + 1};
  const bool bcgs = d.skel == LSBA_BCGSI_LS;
  const bool icwy = d.skel == LSBA_BMGS_ICWY;
  if (k == 1) {
    // J (or H_{1,1}) = <U, W>;  U <- W - V_1 J
    for (int e = threadIdx.x; e < ss; e += NT) {
      const double v = d.G[e];
      if (bcgs) d.J[e] = v;
      d.H[(int64_t)(e / s) * ld + (e % s)] = v;
      d.coef64[lay.C2() + e] = (e / s == e % s) ? 1.0 : 0.0;
      d.coef64[lay.B(0) + e] = -v;
    }
    bar();
    publish_coef(d);
    return;
  }
  const bool last = (k == m + 1);
  const int ldg = last ? s : 2 * s;
  const int r0 = (k - 1) * s;
  const int ks = k * s;
  // LDS: small matrices, then the Gram output (when it fits), then scratch
  double* Om = lds;
  double* R = Om + ss;
  double* Ri = R + ss;
  double* P = Ri + ss;
  double* T1 = P + ss;
  int lused = 5 * ss;
  const int gsize = ks * ldg;
  const double* Gp = d.G;
  if (gsize <= LDS_DBL - lused) {
    bcopy(d.G, lds + lused, gsize);
    Gp = lds + lused;
    lused += gsize;
  }
  double* scr = lds + lused;          // remaining LDS
  const int scap = LDS_DBL - lused;
  bar();
  const double* Y = Gp;                          // r0 x s
  const double* Z = Gp + s;                      // r0 x s (absent on the last step)
  const double* Omt = Gp + (int64_t)r0 * ldg;    // s x s
  const double* Pt = Omt + s;                    // s x s
  for (int e = threadIdx.x; e < ss; e += NT) Om[e] = Omt[(e / s) * ldg + (e % s)];
  if (bcgs) {
    // H_{1:k-1,k-1} = J + Y ;  Omega = Omega~ - Y^T Y
    for (int e = threadIdx.x; e < r0 * s; e += NT) {
      const int i = e / s, c = e % s;
      d.H[(int64_t)i * ld + (k - 2) * s + c] = d.J[i * s + c] + Y[(int64_t)i * ldg + c];
    }
    bar();
    mm(s, s, r0, -1.0, Y, ldg, true, Y, ldg, false, 1.0, Om, s);
  } else {
    bar();
  }
  bool ok = chol_flag(d, Om, s, R);
  if (force) ok = false;
  if (!ok) {
    if (threadIdx.x == 0) raise_flag(ctl, k, k - 2);
    return;
  }
  for (int e = threadIdx.x; e < ss; e += NT)
    d.H[(int64_t)(r0 + e / s) * ld + (k - 2) * s + (e % s)] = R[e];
  tri_inv_up(R, s, Ri);
  for (int e = threadIdx.x; e < ss; e += NT) {
    d.Rinv[e] = Ri[e];
    d.coef64[lay.C1() + e] = Ri[e];
  }
  if (bcgs) {
    // V_k = (U - V_{1:k-1} Y) R^{-1}
    mm(r0, s, s, -1.0, Y, ldg, false, Ri, s, false, 0.0, d.coef64 + lay.A(0), s);
    if (!last) {
      // P = R^{-T} (P~ - Y^T Z)
      for (int e = threadIdx.x; e < ss; e += NT) T1[e] = Pt[(e / s) * ldg + (e % s)];
      bar();
      mm(s, s, r0, -1.0, Y, ldg, true, Z, ldg, false, 1.0, T1, s);
      mm(s, s, s, 1.0, Ri, s, true, T1, s, false, 0.0, P, s);
      // J = ([Z; P] - H_{1:k,1:k-1} Y) R^{-1}, H block upper Hessenberg:
      // rows of blocks 1..k-1 -> scratch, the last block row (only H_{k,k-1}
      // is nonzero there) handled with P
      double* T2 = (ks * s <= scap) ? scr : d.scratch;
      rowprod_any(r0, s, r0, d.H, ld, 1, Y, ldg, 1.0, Z, ldg, T2, s);
      for (int e = threadIdx.x; e < ss; e += NT) {
        const int i = e / s, c = e % s;
        double acc = 0.0;
        for (int t = 0; t < s; ++t)
          acc = fma(d.H[(int64_t)(r0 + i) * ld + (k - 2) * s + t], Y[(int64_t)((k - 2) * s + t) * ldg + c], acc);
        T2[(r0 + i) * s + c] = P[e] - acc;
      }
      bar();
      mm(ks, s, s, 1.0, T2, s, false, Ri, s, false, 0.0, d.J, s);
      // U = (W - V_{1:k-1} Z - V_k P) R^{-1}
      for (int e = threadIdx.x; e < ss; e += NT) d.coef64[lay.C2() + e] = Ri[e];
      mm(r0, s, s, -1.0, Z, ldg, false, Ri, s, false, 0.0, d.coef64 + lay.B(0), s);
      mm(s, s, s, -1.0, P, s, false, Ri, s, false, 0.0, d.coef64 + lay.D(), s);
    }
  } else if (!last) {
    // P = R^{-T} P~ ;  T_{1:k-1,k} ;  H_{1:k,k}
    mm(s, s, s, 1.0, Ri, s, true, Pt, ldg, false, 0.0, P, s);
    // scratch: YR (r0 x s) and ZPR (ks x s), in LDS when they fit
    const bool fit = (r0 + ks) * s <= scap;
    double* YR = fit ? scr : d.scratch;
    double* ZPR = YR + (int64_t)r0 * s;
    double* scr2 = fit ? scr + (r0 + ks) * s : nullptr;
    const int scap2 = fit ? scap - (r0 + ks) * s : 0;
    mm(r0, s, s, 1.0, Y, ldg, false, Ri, s, false, 0.0, YR, s);
    mm(r0, s, s, 1.0, Z, ldg, false, Ri, s, false, 0.0, ZPR, s);
    mm(s, s, s, 1.0, P, s, false, Ri, s, false, 0.0, ZPR + (int64_t)r0 * s, s);
    double* Tc = d.T + r0;   // rows 0..r0-1 of column block k
    if (icwy) {
      copy(r0, s, YR, s, Tc, ld);
    } else {
      // T_{1:k-1,k} = -T_{1:k-1,1:k-1} (Y R^{-1}); T is block upper triangular
      rowprod_any(r0, s, r0, d.T, ld, 0, YR, s, -1.0, nullptr, 0, Tc, ld);
    }
    // keep T^T: row block k of Tt
    for (int e = threadIdx.x; e < r0 * s; e += NT) {
      const int i = e / s, c = e % s;
      d.Tt[(int64_t)(r0 + c) * ld + i] = Tc[(int64_t)i * ld + c];
    }
    bar();
    double* Hc = d.H + (int64_t)(k - 1) * s;   // column block k, rows 0..ks-1
    if (icwy) {
      // H_{1:k,k} = T^{-T} ([Z; P] R^{-1}): forward substitution with T^T
      double* X = (fit && ks * s <= scap2) ? scr2 : d.scratch + (int64_t)2 * ks * s;
      const int xs = (X == scr2) ? ks * s : 0;
      fwd_unit(d.Tt, ld, ZPR, s, X, k, s, scr2 ? scr2 + xs : nullptr, scr2 ? scap2 - xs : 0);
      copy(ks, s, X, s, Hc, ld);
    } else {
      // H_{1:k,k} = T^T ([Z; P] R^{-1}) = Tt ZPR, Tt block lower triangular
      for (int w = threadIdx.x; w < ks * s; w += NT) {
        const int a = w / s, c = w % s;
        const int tend = (a / s + 1) * s;
        double acc = 0.0;
        for (int t = 0; t < tend; ++t) acc = fma(d.Tt[(int64_t)a * ld + t], ZPR[t * s + c], acc);
        Hc[(int64_t)a * ld + c] = acc;
      }
      bar();
    }
    // U = W R^{-1} - V_{1:k-1} H_{1:k-1,k} - V_k H_{k,k}
    for (int e = threadIdx.x; e < ss; e += NT) d.coef64[lay.C2() + e] = Ri[e];
    for (int e = threadIdx.x; e < r0 * s; e += NT) {
      const int i = e / s, c = e % s;
      d.coef64[lay.B(0) + e] = -Hc[(int64_t)i * ld + c];
    }
    bar();
    set_coef(d, lay.D(), Hc + (int64_t)r0 * ld, ld, -1.0);
  }
  bar();
  publish_coef(d);
}

// Alg. 5, after Y = V_{1:k}^T W: H_{1:k,k} = T^T Y (SVL) or T^{-T} Y (LTS); the
// projection W - V_{1:k} H_{1:k,k} is written by the next block update.
__global__ __launch_bounds__(NT) void small_svl_y_kernel(Dense d, int k) {
  __shared__ double lds[LDS_DBL];
  Ctl* ctl = d.ctl;
  if (ctl->stop) return;
  const int s = d.s, ld = d.ldh;
  CoefLayout lay{s, d.mmax + 1};
  const int ks = k * s;
  double* Hc = d.H + (int64_t)(k - 1) * s;
  const bool fit = 2 * ks * s <= LDS_DBL;
  double* Yl = fit ? lds : d.scratch;
  bcopy(d.G, Yl, ks * s);
  bar();
  if (d.skel == LSBA_BMGS_LTS) {
    double* X = fit ? lds + ks * s : d.scratch + (int64_t)ks * s;
    fwd_unit(d.Tt, ld, Yl, s, X, k, s, fit ? lds + 2 * ks * s : nullptr,
             fit ? LDS_DBL - 2 * ks * s : 0);
    copy(ks, s, X, s, Hc, ld);
  } else {
    for (int w = threadIdx.x; w < ks * s; w += NT) {
      const int a = w / s, c = w % s;
      const int tend = (a / s + 1) * s;
      double acc = 0.0;
      for (int t = 0; t < tend; ++t) acc = fma(d.Tt[(int64_t)a * ld + t], Yl[t * s + c], acc);
      Hc[(int64_t)a * ld + c] = acc;
    }
    bar();
  }
  set_coef_identity(d, lay.C2());
  for (int e = threadIdx.x; e < ks * s; e += NT) {
    const int i = e / s, c = e % s;
    d.coef64[lay.B(0) + e] = -Hc[(int64_t)i * ld + c];
  }
  bar();
  publish_coef(d);
}

// Alg. 5, IntraOrtho of the projected block (CholQR): H_{k+1,k} = chol(X^T X).
__global__ __launch_bounds__(NT) void small_svl_io_kernel(Dense d, int k, int force) {
  __shared__ double lds[3 * kMaxS * kMaxS];
  Ctl* ctl = d.ctl;
  if (ctl->stop) return;
  const int s = d.s, ld = d.ldh, ss = s * s;
  CoefLayout lay{s, d.mmax + 1};
  double* G = lds;
  double* R = lds + ss;
  double* Ri = lds + 2 * ss;
  for (int e = threadIdx.x; e < ss; e += NT) G[e] = d.G2[e];
  bar();
  bool ok = chol_flag(d, G, s, R);
  if (force) ok = false;
  if (!ok) {
    if (threadIdx.x == 0) raise_flag(ctl, k, k - 1);
    return;
  }
  tri_inv_up(R, s, Ri);
  for (int e = threadIdx.x; e < ss; e += NT) {
    d.H[(int64_t)(k * s + e / s) * ld + (k - 1) * s + (e % s)] = R[e];
    d.Rinv[e] = Ri[e];
    d.coef64[lay.C1() + e] = Ri[e];
  }
  bar();
  publish_coef(d);
}

// Alg. 5, after Z = V_{1:k}^T V_{k+1}: T_{1:k,k+1} = -T Z (SVL) or Z (LTS)
// (T_{k+1,k+1} = I from CholQR).  Column k is then final (small_finalize).
__global__ __launch_bounds__(NT) void small_svl_z_kernel(Dense d, int k) {
  __shared__ double lds[LDS_DBL];
  Ctl* ctl = d.ctl;
  if (ctl->stop) return;
  const int s = d.s, ld = d.ldh;
  const int ks = k * s;
  double* Tc = d.T + ks;   // rows 0..ks-1 of column block k+1
  const bool fit = ks * s <= LDS_DBL;
  double* Zl = fit ? lds : d.scratch;
  bcopy(d.G, Zl, ks * s);
  bar();
  if (d.skel == LSBA_BMGS_LTS)
    copy(ks, s, Zl, s, Tc, ld);
  else
    rowprod_any(ks, s, ks, d.T, ld, 0, Zl, s, -1.0, nullptr, 0, Tc, ld);
  for (int e = threadIdx.x; e < ks * s; e += NT) {
    const int i = e / s, c = e % s;
    d.Tt[(int64_t)(ks + c) * ld + i] = Tc[(int64_t)i * ld + c];
  }
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
  finalize_column(d, col, lds, LDS_DBL);
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
    if (tm) tm->begin(st);                \
    __VA_ARGS__;                          \
    if (tm) tm->end(st, KK_SMALL, 0.0);   \
  } while (0)

void launch_small_start(hipStream_t st, const Dense& d, int force_flag, KTimer* tm) {
  SMALL_LAUNCH(small_start_kernel<<<1, NT, 0, st>>>(d, force_flag));
}
void launch_small_delayed(hipStream_t st, const Dense& d, int k, int m, int force_flag,
                          KTimer* tm) {
  SMALL_LAUNCH(small_delayed_kernel<<<1, NT, 0, st>>>(d, k, m, force_flag));
}
void launch_small_finalize(hipStream_t st, const Dense& d, int col, KTimer* tm) {
  SMALL_LAUNCH(small_finalize_kernel<<<1, NT, 0, st>>>(d, col));
}
void launch_small_svl_y(hipStream_t st, const Dense& d, int k, KTimer* tm) {
  SMALL_LAUNCH(small_svl_y_kernel<<<1, NT, 0, st>>>(d, k));
}
void launch_small_svl_io(hipStream_t st, const Dense& d, int k, int force_flag, KTimer* tm) {
  SMALL_LAUNCH(small_svl_io_kernel<<<1, NT, 0, st>>>(d, k, force_flag));
}
void launch_small_svl_z(hipStream_t st, const Dense& d, int k, KTimer* tm) {
  SMALL_LAUNCH(small_svl_z_kernel<<<1, NT, 0, st>>>(d, k));
}
void launch_small_cycle_end(hipStream_t st, const Dense& d, KTimer* tm) {
  SMALL_LAUNCH(small_cycle_end_kernel<<<1, NT, 0, st>>>(d));
}
void launch_small_loo(hipStream_t st, const Dense& d, int k_new_block, KTimer* tm) {
  SMALL_LAUNCH(small_loo_kernel<<<1, NT, 0, st>>>(d, k_new_block));
}

}  // namespace lsba
