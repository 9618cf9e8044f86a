// Device helpers of the small dense kernels (one workgroup per solve, FP64):
// block products, Cholesky with the breakdown flag, triangular solves, the
// window Householder QR and the per-column QR update / convergence test.
// Included by kernels_small.hip and kernels_small_qr.hip only.
#pragma once
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
template <bool TA, bool TB>
__device__ __forceinline__ void mm_t(int M, int N, int K, double alpha, const double* A, int lda,
                     const double* B, int ldb, double beta, double* Y, int ldy,
                     const double* C0 = nullptr, int ldc0 = 0) {
  __shared__ double red[NT];
  const int outs = M * N;
  int ks = 1;
  while (ks * 2 * outs <= NT && ks * 2 <= K && ks < 64) ks *= 2;
  auto dot = [&](int i, int j, int k0, int k1) {
    double a0 = 0.0, a1 = 0.0;
    int t = k0;
#pragma unroll 4
    for (; t + 1 < k1; t += 2) {
      const double x0 = TA ? A[(int64_t)t * lda + i] : A[(int64_t)i * lda + t];
      const double y0 = TB ? B[(int64_t)j * ldb + t] : B[(int64_t)t * ldb + j];
      const double x1 = TA ? A[(int64_t)(t + 1) * lda + i] : A[(int64_t)i * lda + t + 1];
      const double y1 = TB ? B[(int64_t)j * ldb + t + 1] : B[(int64_t)(t + 1) * ldb + j];
      a0 = fma(x0, y0, a0);
      a1 = fma(x1, y1, a1);
    }
    if (t < k1) {
      const double x0 = TA ? A[(int64_t)t * lda + i] : A[(int64_t)i * lda + t];
      const double y0 = TB ? B[(int64_t)j * ldb + t] : B[(int64_t)t * ldb + j];
      a0 = fma(x0, y0, a0);
    }
    return a0 + a1;
  };
  if (ks == 1) {
    for (int e = threadIdx.x; e < outs; e += NT) {
      const int i = e / N, j = e % N;
      const double acc = dot(i, j, 0, K);
      double* y = Y + (int64_t)i * ldy + j;
      const double base = C0 ? C0[(int64_t)i * ldc0 + j] : (beta == 0.0 ? 0.0 : beta * *y);
      *y = base + alpha * acc;
    }
    bar();
    return;
  }
  const int t = threadIdx.x;
  if (t < outs * ks) {
    const int e = t % outs, q = t / outs;
    const int i = e / N, j = e % N;
    const int k0 = (int)((int64_t)K * q / ks), k1 = (int)((int64_t)K * (q + 1) / ks);
    red[t] = dot(i, j, k0, k1);
  }
  bar();
  if (t < outs) {
    const int i = t / N, j = t % N;
    double acc = 0.0;
    for (int q = 0; q < ks; ++q) acc += red[q * outs + t];
    double* y = Y + (int64_t)i * ldy + j;
    const double base = C0 ? C0[(int64_t)i * ldc0 + j] : (beta == 0.0 ? 0.0 : beta * *y);
    *y = base + alpha * acc;
  }
  bar();
}

__device__ __forceinline__ void mm(int M, int N, int K, double alpha, const double* A, int lda, bool tA,
                   const double* B, int ldb, bool tB, double beta, double* Y, int ldy) {
  if (tA) {
    if (tB) mm_t<true, true>(M, N, K, alpha, A, lda, B, ldb, beta, Y, ldy);
    else mm_t<true, false>(M, N, K, alpha, A, lda, B, ldb, beta, Y, ldy);
  } else {
    if (tB) mm_t<false, true>(M, N, K, alpha, A, lda, B, ldb, beta, Y, ldy);
    else mm_t<false, false>(M, N, K, alpha, A, lda, B, ldb, beta, Y, ldy);
  }
}

// Y (M x s, ld ldy) = alpha * A (M x s, ld lda) * Bs (s x s, ld s), no barrier:
// one thread per output entry, the s-term sums unrolled.
__device__ __forceinline__ void rows_x_small(int M, int s, const double* A, int lda, const double* Bs,
                             double alpha, double* Y, int ldy) {
  for (int e = threadIdx.x; e < M * s; e += NT) {
    const int i = e / s, c = e % s;
    const double* a = A + (int64_t)i * lda;
    double a0 = 0.0, a1 = 0.0;
    int t = 0;
#pragma unroll 4
    for (; t + 1 < s; t += 2) {
      a0 = fma(a[t], Bs[t * s + c], a0);
      a1 = fma(a[t + 1], Bs[(t + 1) * s + c], a1);
    }
    if (t < s) a0 = fma(a[t], Bs[t * s + c], a0);
    Y[(int64_t)i * ldy + c] = alpha * (a0 + a1);
  }
}

__device__ __forceinline__ void copy(int M, int N, const double* A, int lda, double* Y, int ldy) {
  for (int e = threadIdx.x; e < M * N; e += NT) {
    const int i = e / N, j = e % N;
    Y[(int64_t)i * ldy + j] = A[(int64_t)i * lda + j];
  }
  bar();
}

__device__ __forceinline__ void fill(int M, int N, double v, double* Y, int ldy) {
  for (int e = threadIdx.x; e < M * N; e += NT) {
    const int i = e / N, j = e % N;
    Y[(int64_t)i * ldy + j] = v;
  }
  bar();
}

__device__ __forceinline__ double frob(int M, int N, const double* A, int lda) {
  double v = 0.0;
  for (int e = threadIdx.x; e < M * N; e += NT) {
    const double x = A[(int64_t)(e / N) * lda + (e % N)];
    v += x * x;
  }
  return sqrt(wg_sum(v));
}

// Upper Cholesky factor R (ld s) of Om + shift I (upper triangle of Om read),
// and dinv[j] = 1 / R[j][j] when dinv is not null.  Returns false (the
// breakdown flag) when a pivot is not a positive finite number.  One
// wavefront does the factorization, lane l owning column l (left-looking: at
// step j lane l >= j forms Om[j][l] - sum_{i<j} R[i][j] R[i][l]; lane j's
// value is the pivot).  Lanes of one wavefront see each other's LDS writes of
// earlier steps in program order, so only the final hand-over needs a barrier.
__device__ __forceinline__ bool chol_up(const double* Om, int ldo, double* R, int s, double shift,
                        double* dinv = nullptr) {
  __shared__ int okf;
  for (int e = threadIdx.x; e < s * s; e += NT) {
    const int i = e / s, j = e % s;
    R[e] = (j >= i) ? Om[(int64_t)i * ldo + j] + (i == j ? shift : 0.0) : 0.0;
  }
  bar();
  if (threadIdx.x < 64) {
    const int l = threadIdx.x;
    int ok = 1;
    for (int j = 0; j < s; ++j) {
      double v = 0.0;
      if (l >= j && l < s) {
        double v0 = R[j * s + l], v1 = 0.0;
        int i = 0;
#pragma unroll 4
        for (; i + 1 < j; i += 2) {
          v0 = fma(-R[i * s + j], R[i * s + l], v0);
          v1 = fma(-R[(i + 1) * s + j], R[(i + 1) * s + l], v1);
        }
        if (i < j) v0 = fma(-R[i * s + j], R[i * s + l], v0);
        v = v0 + v1;
      }
      const double dd = __shfl(v, j, 64);
      if (!(dd > 0.0) || !isfinite(dd)) {
        ok = 0;
        break;
      }
      const double rjj = sqrt(dd);
      const double inv = 1.0 / rjj;
      if (l == j) {
        R[j * s + j] = rjj;
        if (dinv) dinv[j] = inv;
      } else if (l > j && l < s) {
        R[j * s + l] = v * inv;
      }
      __builtin_amdgcn_wave_barrier();
    }
    if (l == 0) okf = ok;
  }
  bar();
  return okf != 0;
}

// Cholesky with the mixed form's shifted fallback: if the plain factorization
// flags, retry with Om + sigma I, sigma = 10 u_fp32 trace(Om).
__device__ bool chol_flag(const Dense& d, const double* Om, int ldo, double* R,
                          double* dinv = nullptr) {
  const int s = d.s;
  bool ok = chol_up(Om, ldo, R, s, 0.0, dinv);
  if (!ok && d.mixed) {
    double tr = 0.0;
    for (int i = 0; i < s; ++i) tr += fabs(Om[(int64_t)i * ldo + i]);
    ok = chol_up(Om, ldo, R, s, 10.0 * 5.9604644775390625e-08 * tr, dinv);
  }
  return ok;
}

// Ri = R^{-1} for upper-triangular R (s x s); dinv[i] = 1 / R[i][i] when
// given (else computed here).  Thread c forms column c bottom-up.
__device__ __forceinline__ void tri_inv_up(const double* R, int s, double* Ri, const double* dinv = nullptr) {
  __shared__ double dl[kMaxS];
  if (!dinv) {
    for (int i = threadIdx.x; i < s; i += NT) dl[i] = 1.0 / R[i * s + i];
    bar();
    dinv = dl;
  }
  for (int c = threadIdx.x; c < s; c += NT) {
    for (int i = s - 1; i > c; --i) Ri[i * s + c] = 0.0;
    Ri[c * s + c] = dinv[c];
    for (int i = c - 1; i >= 0; --i) {
      double v0 = 0.0, v1 = 0.0;
      int l = i + 1;
#pragma unroll 4
      for (; l + 1 <= c; l += 2) {
        v0 = fma(-R[i * s + l], Ri[l * s + c], v0);
        v1 = fma(-R[i * s + l + 1], Ri[(l + 1) * s + c], v1);
      }
      if (l <= c) v0 = fma(-R[i * s + l], Ri[l * s + c], v0);
      Ri[i * s + c] = (v0 + v1) * dinv[i];
    }
  }
  bar();
}

// X (s x nrhs, ld ldx) <- R^{-1} X for upper-triangular R (ld ldr).
__device__ __forceinline__ void tri_solve_up(const double* R, int ldr, int s, double* X, int ldx, int nrhs) {
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
// non-finite pivot.  One wavefront, lane c owning column c of [A | Bm]
// (s + nrhs <= 64); the lanes see each other's LDS writes of earlier
// instructions in program order.
__device__ __forceinline__ bool lu_solve(double* A, double* Bm, int s, int nrhs) {
  __shared__ int okf;
  __shared__ double dinv[kMaxS];
  if (threadIdx.x < 64) {
    const int c = threadIdx.x;
    const int w = s + nrhs;
    double* colp = c < s ? A + c : Bm + (c - s);   // element i of my column: colp[i * ldc]
    const int ldc = c < s ? s : nrhs;
    const bool mine = c < w;
    int ok = 1;
    for (int k = 0; k < s; ++k) {
      int p = k;
      double best = 0.0;
      if (c == k) {
        best = fabs(A[k * s + k]);
        for (int i = k + 1; i < s; ++i) {
          const double v = fabs(A[i * s + k]);
          if (v > best) {
            best = v;
            p = i;
          }
        }
      }
      p = __shfl(p, k, 64);
      best = __shfl(best, k, 64);
      if (!(best > 0.0) || !isfinite(best)) {
        ok = 0;
        break;
      }
      if (mine && p != k) {
        const double t = colp[k * ldc];
        colp[k * ldc] = colp[p * ldc];
        colp[p * ldc] = t;
      }
      __builtin_amdgcn_wave_barrier();
      const double inv = 1.0 / A[k * s + k];
      if (mine && c > k) {
        const double pk = colp[k * ldc];
#pragma unroll 4
        for (int i = k + 1; i < s; ++i) colp[i * ldc] = fma(-(A[i * s + k] * inv), pk, colp[i * ldc]);
      }
      __builtin_amdgcn_wave_barrier();
    }
    if (ok) {
      if (c < s) dinv[c] = 1.0 / A[c * s + c];
      __builtin_amdgcn_wave_barrier();
      if (c >= s && mine) {
        for (int i = s - 1; i >= 0; --i) {
          double v = colp[i * ldc];
#pragma unroll 4
          for (int l = i + 1; l < s; ++l) v = fma(-A[i * s + l], colp[l * ldc], v);
          colp[i * ldc] = v * dinv[i];
        }
      }
    }
    if (c == 0) okf = ok;
  }
  bar();
  return okf != 0;
}

// Householder vector of column c of the 2s x s window W (ld s), by wavefront
// 0 with lane r taking row r: W(:, c) <- beta e_c, Y(:, c) <- v (v_c = 1),
// *tau_out <- tau.
__device__ __forceinline__ void house_col(double* W, int s, double* Y, int c, double* tau_out) {
  const int m2 = 2 * s, r = threadIdx.x;
  const double x = (r > c && r < m2) ? W[r * s + c] : 0.0;
  double xn2 = x * x;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) xn2 += __shfl_xor(xn2, off, 64);
  const double alpha = W[c * s + c];
  double tau = 0.0, beta = alpha, scale = 0.0;
  if (xn2 != 0.0) {
    beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
    tau = (beta - alpha) / beta;
    scale = 1.0 / (alpha - beta);
  }
  __builtin_amdgcn_wave_barrier();
  if (r < m2) {
    Y[r * s + c] = r < c ? 0.0 : (r == c ? 1.0 : x * scale);
    if (r >= c) W[r * s + c] = (r == c) ? beta : 0.0;
  }
  if (r == 0) *tau_out = tau;
}

// Householder QR of the 2s x s window W (ld s, in LDS): W <- [R; 0] and
// Qt (2s x 2s, ld 2s) = Q^T with Q = I - Y T Y^T.  Y, T, tmp are LDS scratch
// (2s x s, s x s, >= 2s x s).  Per column: the s - 1 inner products of v
// with the trailing columns of W (and, for T, with the earlier columns of Y)
// are formed by 16-lane groups; then wavefront 0 updates the next column and
// forms its reflector while the other wavefronts update the rest and T.
__device__ __forceinline__ void window_qr(double* W, int s, double* Qt, double* Y, double* Tq, double* tmp) {
  __shared__ double hh[1];
  __shared__ double wv[2 * kMaxS];
  const int m2 = 2 * s;
  for (int e = threadIdx.x; e < m2 * s; e += NT) Y[e] = 0.0;
  for (int e = threadIdx.x; e < s * s; e += NT) Tq[e] = 0.0;
  bar();
  if (threadIdx.x < 64) house_col(W, s, Y, 0, hh);
  bar();
  const int g = threadIdx.x >> 4, p = threadIdx.x & 15;
  for (int c = 0; c < s; ++c) {
    const double tau = hh[0];
    for (int base = 0; base < s - 1; base += NT / 16) {
      const int dd = base + g;
      const bool valid = dd < s - 1;
      double acc = 0.0;
      if (valid) {
        const double* col = dd < c ? Y + dd : W + dd + 1;
        for (int r = c + p; r < m2; r += 16) acc = fma(col[r * s], Y[r * s + c], acc);
      }
#pragma unroll
      for (int off = 8; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 16);
      if (valid && p == 0) wv[dd] = dd < c ? acc : tau * acc;
    }
    bar();
    if (threadIdx.x < 64) {
      if (c + 1 < s) {
        const int r = threadIdx.x;
        if (r >= c && r < m2) W[r * s + c + 1] = fma(-wv[c], Y[r * s + c], W[r * s + c + 1]);
        __builtin_amdgcn_wave_barrier();
        house_col(W, s, Y, c + 1, hh);
      }
    } else {
      const int t = threadIdx.x - 64;
      const int nq = s - c - 2, nr = m2 - c;
      for (int e = t; e < nq * nr; e += NT - 64) {
        const int q = c + 2 + e / nr, r = c + e % nr;
        W[r * s + q] = fma(-wv[q - 1], Y[r * s + c], W[r * s + q]);
      }
      for (int i = t; i < c; i += NT - 64) {
        double v = 0.0;
        for (int l = i; l < c; ++l) v = fma(Tq[i * s + l], wv[l], v);
        Tq[i * s + c] = -tau * v;
      }
      if (t == 0) Tq[c * s + c] = tau;
    }
    bar();
  }
  // Q^T = I - Y T^T Y^T: tmp (s x 2s) = T^T Y^T, then Qt = I - Y tmp
  for (int e = threadIdx.x; e < s * m2; e += NT) {
    const int a = e / m2, r = e % m2;
    double v = 0.0;
    for (int l = 0; l <= a; ++l) v = fma(Tq[l * s + a], Y[r * s + l], v);
    tmp[e] = v;
  }
  bar();
  for (int e = threadIdx.x; e < m2 * m2; e += NT) {
    const int r = e / m2, c = e % m2;
    double v0 = 0.0, v1 = 0.0;
    int a = 0;
#pragma unroll 4
    for (; a + 1 < s; a += 2) {
      v0 = fma(Y[r * s + a], tmp[a * m2 + c], v0);
      v1 = fma(Y[r * s + a + 1], tmp[(a + 1) * m2 + c], v1);
    }
    if (a < s) v0 = fma(Y[r * s + a], tmp[a * m2 + c], v0);
    Qt[e] = (r == c ? 1.0 : 0.0) - (v0 + v1);
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

// The folded form of an update with a D term: BF(i) = [nb <= i < nv2] B_i +
// [i < nv1] A_i D for i < max(nv1, nv2), and C1D = C1 D.  Reads coefficients
// this workgroup wrote (call after a barrier); ends with a barrier.
__device__ __forceinline__ void fold_coef(const Dense& d, int nv1, int nb, int nv2) {
  const int s = d.s, ss = s * s;
  CoefLayout lay{s, d.mmax + 1};
  double* c = d.coef64;
  const double* D = c + lay.D();
  const int nvm = nv1 > nv2 ? nv1 : nv2;
  for (int e = threadIdx.x; e < (nvm + 1) * ss; e += NT) {
    const int blk = e / ss, f = e % ss, i = f / s, j = f % s;
    if (blk < nvm) {
      double acc = (blk >= nb && blk < nv2) ? c[lay.B(blk) + f] : 0.0;
      if (blk < nv1)
        for (int t = 0; t < s; ++t) acc = fma(c[lay.A(blk) + i * s + t], D[t * s + j], acc);
      c[lay.BF(blk) + f] = acc;
    } else {
      double acc = 0.0;
      for (int t = 0; t < s; ++t) acc = fma(c[lay.C1() + i * s + t], D[t * s + j], acc);
      c[lay.C1D() + f] = acc;
    }
  }
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
__device__ __forceinline__ int finalize_lds_min(int s) { return 16 * s * s; }

// Column j (1-based) of H is final: bring it through the orthogonal factors of
// columns 1..j-1, factor its window, record the residual estimate, test
// convergence.  Hc holds the column's (j + 1) s rows (ld ldc, global memory or
// LDS outside the workspace); `lds` holds nl >= finalize_lds_min(s) doubles of
// workspace.
__device__ __forceinline__ void finalize_column(const Dense& d, int j, double* lds, int nl, const double* Hc,
                                int ldc) {
  const int s = d.s, ld = d.ldh, ss = s * s, q4 = 4 * ss;
  const int c0 = (j - 1) * s;
  Ctl* ctl = d.ctl;
  double* Rfc = d.Rf + c0;
  // LDS carve-up: two carry blocks, the g window and H_{j+1,j} (loaded up
  // front), then a region that holds the ring of (Q_i^T, block row i+1) items
  // during the chain and the window-QR buffers after it.
  double* carry1 = lds;            // ss
  double* carry0 = carry1 + ss;    // ss   first block row of the column
  double* gpre = carry0 + ss;      // 2ss  rows c0 .. c0 + 2s of g
  double* hsub = gpre + 2 * ss;    // ss   H_{j+1,j}
  double* ring = hsub + ss;        // chain: slots of (Q^T: q4, block of h: ss)
  double* qw = ring;               // after: 2ss  [D; H_{j+1,j}] window
  double* Yw = qw + 2 * ss;        //        2ss
  double* Tw = Yw + 2 * ss;        //        ss
  double* tmp = Tw + ss;           //        4ss  (LU scratch, then Q_j^T)
  double* gw = tmp + q4;           //        2ss  (QR scratch)
  const int slot_sz = q4 + ss;
  const int nslots_fit = (nl - 5 * ss) / slot_sz;
  const int nap = j - 1;
  const bool all = nslots_fit >= nap;
  const int R = all ? (nap > 0 ? nap : 1) : 2;

  auto item_elem = [&](int i, int e) -> double {   // element e of item i (1-based window)
    if (e < q4) return d.Qt[(int64_t)(i - 1) * q4 + e];
    const int f = e - q4;
    return Hc[(int64_t)(i * s + f / s) * ldc + (f % s)];
  };
  {
    // One batched pass with two streams kept apart by address space (the
    // column may be in LDS): A = the g window and Q^T of the first items
    // (global), B = carry0, H_{j+1,j} and the h blocks of those items (from
    // Hc).  All loads of a batch are issued before any is used.
    const int npre = nap > 0 ? (all ? nap : 1) : 0;
    const int totA = 2 * ss + npre * q4, totB = 2 * ss + npre * ss;
    const int tot = totA > totB ? totA : totB;
    auto srcA = [&](int e) -> const double* {
      if (e < 2 * ss) return d.g + (int64_t)c0 * s + e;
      const int f = e - 2 * ss;
      return d.Qt + (int64_t)(f / q4) * q4 + (f % q4);
    };
    auto dstA = [&](int e) -> double* {
      if (e < 2 * ss) return gpre + e;
      const int f = e - 2 * ss;
      return ring + (int64_t)(f / q4) * slot_sz + (f % q4);
    };
    auto srcB = [&](int e) -> const double* {
      int row;
      if (e < ss) row = e / s;                             // block row 1
      else if (e < 2 * ss) row = j * s + (e - ss) / s;     // block row j + 1
      else row = ((e - 2 * ss) / ss + 1) * s + ((e - 2 * ss) % ss) / s;   // item h blocks
      return Hc + (int64_t)row * ldc + (e % s);
    };
    auto dstB = [&](int e) -> double* {
      if (e < ss) return carry0 + e;
      if (e < 2 * ss) return hsub + (e - ss);
      const int f = e - 2 * ss;
      return ring + (int64_t)(f / ss) * slot_sz + q4 + (f % ss);
    };
    constexpr int U = 16;
    for (int base = threadIdx.x; base < tot; base += NT * U) {
      double va[U], vb[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = base + u * NT;
        va[u] = *srcA(e < totA ? e : totA - 1);
        vb[u] = *srcB(e < totB ? e : totB - 1);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = base + u * NT;
        if (e < totA) *dstA(e) = va[u];
        if (e < totB) *dstB(e) = vb[u];
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
      // 2s-term product in batches of 8: all operands of a batch are read
      // (clamped indices, zero weights past the end) before the FMAs
      double a0 = 0.0, a1 = 0.0;
      for (int t0 = 0; t0 < s; t0 += 8) {
        double qa[8], qb[8], va[8], vb[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int t = t0 + u < s ? t0 + u : s - 1;
          qa[u] = Q[r * m2 + t];
          qb[u] = Q[r * m2 + s + t];
          va[u] = cur[t * s + c];
          vb[u] = hb[t * s + c];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const double wgt = t0 + u < s ? 1.0 : 0.0;
          a0 = fma(qa[u] * wgt, va[u], a0);
          a1 = fma(qb[u] * wgt, vb[u], a1);
        }
      }
      const double acc = a0 + a1;
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
  for (int e = threadIdx.x; e < ss; e += NT) {
    d.Dlast[e] = cur[e];
    qw[e] = cur[e];
    qw[ss + e] = hsub[e];
  }
  bar();
  double est = 0.0;
  if (d.method == LSBA_FOM) {
    // last block of Xi: D^{-1} g_j ; estimate ||H_{j+1,j} D^{-1} g_j||_F
    double* A = tmp;
    double* Bm = tmp + ss;
    for (int e = threadIdx.x; e < ss; e += NT) {
      A[e] = cur[e];
      Bm[e] = gpre[e];
    }
    bar();
    if (lu_solve(A, Bm, s, s)) {
      double* HY = tmp + 2 * ss;
      for (int e = threadIdx.x; e < ss; e += NT) {
        d.ylast[e] = Bm[e];
        const int i = e / s, c = e % s;
        double acc = 0.0;
#pragma unroll 8
        for (int t = 0; t < s; ++t) acc = fma(hsub[i * s + t], Bm[t * s + c], acc);
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
  // R_jj -> Rf, Q_j^T -> global, g window <- Q_j^T g window
  for (int e = threadIdx.x; e < ss; e += NT)
    Rfc[(int64_t)(c0 + e / s) * ld + (e % s)] = qw[e];
  for (int e = threadIdx.x; e < q4; e += NT) d.Qt[(int64_t)(j - 1) * q4 + e] = Qj[e];
  for (int e = threadIdx.x; e < 2 * ss; e += NT) {
    const int r = e / s, c = e % s;
    double a0 = 0.0, a1 = 0.0;
#pragma unroll 8
    for (int t = 0; t < s; ++t) {
      a0 = fma(Qj[r * m2 + t], gpre[t * s + c], a0);
      a1 = fma(Qj[r * m2 + s + t], gpre[(s + t) * s + c], a1);
    }
    const double acc = a0 + a1;
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
__device__ __forceinline__ void bcopy(const double* __restrict__ src, double* __restrict__ dst, int n) {
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
// column that is final.  A convergence already recorded is kept.  The status
// is published before flag_step / last_valid: a kernel on another stream may
// see FLAGGED with the cycle-start values (-1, 1 << 30).  Readers therefore
// trust only values that a flag at a step they are ordered after can write
// (small_side_kernel: 0 <= flag_step <= k; small_finalize_kernel: a column
// past last_valid), and such a flag is always fully visible to them.
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
__device__ __forceinline__ void rowprod(int M, int s, int K, const double* A, int lda, int tlo_blk,
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

__device__ __forceinline__ void rowprod_any(int M, int s, int K, const double* A, int lda, int tlo_blk,
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
__device__ __forceinline__ void fwd_unit(const double* Lt, int ld, const double* Rhs, int ldr, double* X, int k,
                         int s, double* buf, int cap, bool diag = false) {
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
      if (diag) {
        // a unit lower triangular (not identity) diagonal block: row by row
        bar();
        double* Xc = X + (int64_t)c * ss;
        const double* Ld = Lt + (int64_t)(c * s) * ld + c * s;
        for (int i = 1; i < s; ++i) {
          if (threadIdx.x < s) {
            const int col = threadIdx.x;
            double acc = Xc[i * s + col];
            for (int t = 0; t < i; ++t) acc = fma(-Ld[(int64_t)i * ld + t], Xc[t * s + col], acc);
            Xc[i * s + col] = acc;
          }
          bar();
        }
      }
      off += s * w;
    }
    b = b1;
  }
}

}  // namespace
}  // namespace lsba
