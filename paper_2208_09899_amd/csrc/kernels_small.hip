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
#include <algorithm>

#include "small_common.h"

namespace lsba {

namespace {

// ------------------------------------------------------------------ kernels

// T = T^T = I at the start of a cycle (Algs. 5 and 6), spread over the chip.
__global__ __launch_bounds__(NT) void t_identity_kernel(Dense d) {
  const int64_t ld = d.ldh, tot = ld * ld;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < tot; e += (int64_t)gridDim.x * NT) {
    const double v = ((e / ld) == (e % ld)) ? 1.0 : 0.0;
    d.T[e] = v;
    d.Tt[e] = v;
  }
}

__global__ __launch_bounds__(NT) void small_start_kernel(Dense d, int force) {
  __shared__ double lds[4 * kMaxS * kMaxS];
  Ctl* ctl = d.ctl;
  const int s = d.s, ld = d.ldh, ss = s * s;
  CoefLayout lay{s, d.mmax + 1};
  double* R = lds;
  double* Ri = lds + ss;
  double* G = lds + 2 * ss;
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
  const double* Gk = d.G + (int64_t)k * d.gstride;
  if (k == 1) {
    // J (or H_{1,1}) = <U, W>;  U <- W - V_1 J
    for (int e = threadIdx.x; e < ss; e += NT) {
      const double v = Gk[e];
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
  const double* Gp = Gk;
  if (gsize <= LDS_DBL - lused) {
    bcopy(Gk, lds + lused, gsize);
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
    fold_coef(d, 0, 0, k - 1);
  }
  bar();
  publish_coef(d);
}

// Alg. 7, loop step k >= 2, the part on the basis path.  From this step's
// fused Gram [V_{1:k-1} U]^T [U W] = [Y Z; Omega~ P~]: Omega = Omega~ - Y^T Y,
// its Cholesky factor R = H_{k,k-1} (with the breakdown flag), and the
// coefficients of V_k = (U - V_{1:k-1} Y) R^{-1} and of
// U = (W - V_{1:k-1} Z - V_k P) R^{-1} with P = R^{-T} (P~ - Y^T Z).
// H_{1:k-1,k-1} and the J recurrence feed only the QR / convergence test and
// are left to small_side, which reads R^{-1} and P from this step's slots.
template <bool FIT>
__global__ __launch_bounds__(NT) void small_core_kernel(Dense d, int k, int m, int force) {
  __shared__ double lds[LDS_DBL];
  Ctl* ctl = d.ctl;
  if (ctl->stop) return;
  const int s = d.s, ld = d.ldh, ss = s * s;
  CoefLayout lay{s, d.mmax + 1};
  const bool last = (k == m + 1);
  const int ldg = last ? s : 2 * s;
  const int r0 = (k - 1) * s, ks = k * s;
  const double* Gk = d.G + (int64_t)k * d.gstride;
  double* OmP = lds;            // s x ldg: [Omega | P~ - Y^T Z]
  double* R = OmP + 2 * ss;
  double* Ri = R + ss;
  double* Pn = Ri + ss;
  double* dinv = Pn + ss;       // kMaxS
  const int lused = 5 * ss + kMaxS;
  // FIT: this step's Gram output is copied to LDS (it fits: ks * ldg <= LDS_DBL - lused)
  const double* Gp;
  if constexpr (FIT) {
    bcopy(Gk, lds + lused, ks * ldg);
    Gp = lds + lused;
    bar();
  } else {
    Gp = Gk;
  }
  // [Omega | P~ - Y^T Z] = G(r0.., :) - Y^T [Y Z]
  if constexpr (FIT) {
    mm_t<true, false>(s, ldg, r0, -1.0, Gp, ldg, Gp, ldg, 0.0, OmP, ldg, Gp + (int64_t)r0 * ldg,
                      ldg);
  } else {
    // the Gram output stays in global memory: stream its rows through LDS in
    // chunks (contiguous loads), each thread accumulating its outputs (i, j)
    // of Y^T [Y Z] in a fixed row order
    double* chunk = lds + lused;
    const int crow = (LDS_DBL - lused) / ldg < 64 ? (LDS_DBL - lused) / ldg : 64;
    constexpr int OPT = (kMaxS * 2 * kMaxS + NT - 1) / NT;   // outputs per thread, at most
    double acc[OPT];
#pragma unroll
    for (int u = 0; u < OPT; ++u) acc[u] = 0.0;
    const int nout = s * ldg;
    for (int t0 = 0; t0 < r0; t0 += crow) {
      const int nr = r0 - t0 < crow ? r0 - t0 : crow;
      bar();
      bcopy(Gp + (int64_t)t0 * ldg, chunk, nr * ldg);
      bar();
#pragma unroll
      for (int u = 0; u < OPT; ++u) {
        const int e = threadIdx.x + u * NT;
        if (e < nout) {
          const int i = e / ldg, j = e % ldg;
          double a = acc[u];
          for (int t = 0; t < nr; ++t) a = fma(chunk[t * ldg + i], chunk[t * ldg + j], a);
          acc[u] = a;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < OPT; ++u) {
      const int e = threadIdx.x + u * NT;
      if (e < nout) OmP[e] = Gp[(int64_t)r0 * ldg + e] - acc[u];
    }
    bar();
  }
  bool ok = chol_flag(d, OmP, ldg, R, dinv);
  if (force) ok = false;
  if (!ok) {
    if (threadIdx.x == 0) raise_flag(ctl, k, k - 2);
    return;
  }
  tri_inv_up(R, s, Ri, dinv);
  double* coef = d.coef64;
  // C1 = C2 = R^{-1}; H_{k,k-1} = R;  P = R^{-T} (P~ - Y^T Z)
  for (int e = threadIdx.x; e < ss; e += NT) {
    coef[lay.C1() + e] = Ri[e];
    d.H[(int64_t)(r0 + e / s) * ld + (k - 2) * s + (e % s)] = R[e];
    d.RiS[(int64_t)k * ss + e] = Ri[e];
    if (!last) {
      coef[lay.C2() + e] = Ri[e];
      const int i = e / s, c = e % s;
      double acc = 0.0;
#pragma unroll 8
      for (int t = 0; t < s; ++t) acc = fma(Ri[t * s + i], OmP[t * ldg + s + c], acc);
      Pn[e] = acc;
      d.PS[(int64_t)k * ss + e] = acc;
    }
  }
  double* PR = OmP;   // [Omega | ..] is dead once P is formed
  if (!last) {
    bar();
    // PR = P R^{-1} (D = -PR), then W = R^{-1} PR in R (dead after R^{-1})
    for (int e = threadIdx.x; e < ss; e += NT) {
      const int i = e / s, c = e % s;
      double acc = 0.0;
#pragma unroll 8
      for (int t = 0; t < s; ++t) acc = fma(Pn[i * s + t], Ri[t * s + c], acc);
      PR[e] = acc;
      coef[lay.D() + e] = -acc;
    }
    bar();
    for (int e = threadIdx.x; e < ss; e += NT) {
      const int i = e / s, c = e % s;
      double acc = 0.0;
#pragma unroll 8
      for (int t = 0; t < s; ++t) acc = fma(Ri[i * s + t], PR[t * s + c], acc);
      R[e] = acc;
      coef[lay.C1D() + e] = -acc;   // C1 D = -W
    }
  }
  bar();
  // the s x s coefficients for the precision form's update (the row blocks
  // A, B, BF follow in small_core_rows_kernel, which writes both copies)
  if (d.mixed) {
    float* fc = (float*)d.coefT;
    for (int e = threadIdx.x; e < ss; e += NT) {
      fc[lay.C1() + e] = (float)coef[lay.C1() + e];
      if (!last) {
        fc[lay.C2() + e] = (float)coef[lay.C2() + e];
        fc[lay.D() + e] = (float)coef[lay.D() + e];
        fc[lay.C1D() + e] = (float)coef[lay.C1D() + e];
      }
    }
  }
}

// Alg. 7 core step, second part (after small_core_kernel, k >= 2): one pass
// over the rows of [Y Z], spread over the chip: A = -Y R^{-1},
// B = -Z R^{-1} and the folded B + A D = -Z R^{-1} + Y W, with R^{-1} and
// W = R^{-1} P R^{-1} as the core step left them (its R^{-1} slot and the
// C1 D coefficient, -W).  Each entry is written in FP64 and, for the
// precision form, in FP32.
__global__ __launch_bounds__(NT) void small_core_rows_kernel(Dense d, int k, int m) {
  __shared__ double Ri[kMaxS * kMaxS], Wl[kMaxS * kMaxS];
  Ctl* ctl = d.ctl;
  if (ctl->stop) return;
  const int s = d.s, ss = s * s;
  CoefLayout lay{s, d.mmax + 1};
  const bool last = (k == m + 1);
  const int ldg = last ? s : 2 * s;
  const int r0 = (k - 1) * s;
  const double* Gp = d.G + (int64_t)k * d.gstride;
  double* coef = d.coef64;
  for (int e = threadIdx.x; e < ss; e += NT) {
    Ri[e] = d.RiS[(int64_t)k * ss + e];
    Wl[e] = last ? 0.0 : -coef[lay.C1D() + e];
  }
  bar();
  float* fc = d.mixed ? (float*)d.coefT : nullptr;
  for (int e = blockIdx.x * NT + threadIdx.x; e < r0 * s; e += gridDim.x * NT) {
    const int i = e / s, c = e % s;
    const double* y = Gp + (int64_t)i * ldg;
    double a = 0.0, b = 0.0, f = 0.0;
#pragma unroll 8
    for (int t = 0; t < s; ++t) {
      const double yt = y[t];
      a = fma(yt, Ri[t * s + c], a);
      if (!last) {
        const double zt = y[s + t];
        b = fma(zt, Ri[t * s + c], b);
        f = fma(yt, Wl[t * s + c], f);
      }
    }
    coef[lay.A(0) + e] = -a;
    if (fc) fc[lay.A(0) + e] = (float)(-a);
    if (!last) {
      coef[lay.B(0) + e] = -b;
      coef[lay.BF(0) + e] = f - b;
      if (fc) {
        fc[lay.B(0) + e] = (float)(-b);
        fc[lay.BF(0) + e] = (float)(f - b);
      }
    }
  }
}

// LDS layout of small_cwy (Alg. 6, 2 <= k <= m): small matrices, Y R^{-1},
// [Z; P] R^{-1}, H_{1:k,k}, the new T column, then the Gram output (dead
// once Y R^{-1} and [Z; P] R^{-1} exist) and the staging area for T.
__host__ __device__ inline int cwy_fixed(int s, int k) {
  const int ss = s * s, r0 = (k - 1) * s, ks = k * s;
  return 4 * ss + kMaxS + r0 * s + ks * s + ks * s + r0 * s;
}
__host__ __device__ inline bool cwy_fits(int s, int k) {
  const int r0 = (k - 1) * s, ks = k * s;
  const int g = ks * 2 * s;
  const int stage_min = r0 * s > g ? r0 * s : g;
  return cwy_fixed(s, k) + stage_min <= LDS_DBL;
}

// Alg. 6 (BMGS-CWY / BMGS-ICWY), loop step 2 <= k <= m, all operands in LDS.
// From [Y Z; Omega P~] = [V_{1:k-1} U]^T [U W]: R = chol(Omega) = H_{k,k-1}
// (flag), P = R^{-T} P~, the new T column T_{1:k-1,k} = -T (Y R^{-1}) (CWY) or
// Y R^{-1} (ICWY), H_{1:k,k} = T^T ([Z; P] R^{-1}) (CWY) or T^{-T} ([Z; P]
// R^{-1}) (ICWY) with T = T_{1:k,1:k}, and the coefficients of V_k = U R^{-1}
// and U = W R^{-1} - V_{1:k} H_{1:k,k}.  T is read from global memory once,
// staged in LDS a few rows (CWY) or column blocks (ICWY) at a time.
// LDS doubles small_cwy_rows needs at loop step k.
__host__ __device__ inline int cwy_rows_lds(int s, int k) {
  const int r0 = (k - 1) * s;
  return 6 * r0 * s + 6 * s * s + NT;
}

// Alg. 6 with the explicit T (BMGS-CWY), loop step 2 <= k <= m, split over
// the k block rows: workgroup rb < k - 1 forms block row rb of the new T
// column T_{1:k-1,k} = -T (Y R^{-1}) and of H_{1:k-1,k} = T^T (Z R^{-1}) (each
// needs only its own rows of T, T^T and [Y Z]; every workgroup repeats the
// s x s Cholesky), workgroup k - 1 writes R and the R^{-1} coefficients.  The
// last block row H_{k,k} = P R^{-1} + T_{1:k-1,k}^T (Z R^{-1}) sums one s x s
// term per block row: each workgroup stores its term, and the workgroup that
// arrives last (a counter per loop step) adds them in block-row order.
__global__ __launch_bounds__(NT) void small_cwy_rows_kernel(Dense d, int k, int force) {
  __shared__ double lds[LDS_DBL];
  __shared__ int is_last;
  Ctl* ctl = d.ctl;
  if (ctl->stop) return;
  const int s = d.s, ld = d.ldh, ss = s * s;
  CoefLayout lay{s, d.mmax + 1};
  const int r0 = (k - 1) * s, ldg = 2 * s;
  const int rb = blockIdx.x, a0 = rb * s;
  const bool rowblk = rb < k - 1;
  const double* Gk = d.G + (int64_t)k * d.gstride;
  const Scr sc = make_scr(d);
  double* part = sc.bg(2);          // (k - 1) x ss terms of the last block row
  const int tid = threadIdx.x;
  double* Om = lds;                 // ss  Omega
  double* Pt = Om + ss;             // ss  P~
  double* R = Pt + ss;              // ss
  double* Ri = R + ss;              // ss
  double* Pn = Ri + ss;             // ss  P = R^{-T} P~
  double* dv = Pn + ss;             // ss  (s used: 1 / R_ii)
  double* red = dv + ss;            // NT  split-sum partials
  double* Gs = red + NT;            // r0 x 2s  [Y Z]
  const int wT = r0 - a0, wH = a0 + s;
  double* Tr = Gs + 2 * r0 * s;     // s x wT   T(a0 + i, a0 + u)
  double* Ttr = Tr + s * r0;        // s x wH   T^T(a0 + i, t)
  double* YR = Ttr + s * r0;        // r0 x s   (rows a0 .. r0 used)
  double* ZR = YR + r0 * s;         // r0 x s   (rows 0 .. a0 + s used)
  {
    const int nA = 2 * ss, nG = 2 * r0 * s, nT = rowblk ? s * wT : 0, nH = rowblk ? s * wH : 0;
    const int tot = nA + nG + nT + nH;
    for (int base = tid; base < tot; base += NT * 16) {
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        int e = base + u * NT;
        e = e < tot ? e : tot - 1;
        const double* p;
        if (e < nA) {
          const int f = e % ss;
          p = Gk + (int64_t)(r0 + f / s) * ldg + (e < ss ? 0 : s) + f % s;
        } else if (e < nA + nG) {
          p = Gk + (e - nA);
        } else if (e < nA + nG + nT) {
          const int f = e - nA - nG;
          p = d.T + (int64_t)(a0 + f / wT) * ld + a0 + f % wT;
        } else {
          const int f = e - nA - nG - nT;
          p = d.Tt + (int64_t)(a0 + f / wH) * ld + f % wH;
        }
        v[u] = *p;
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int e = base + u * NT;
        if (e < tot) {
          double* q;
          if (e < nA) q = Om + e;                                  // Om, Pt adjacent
          else if (e < nA + nG) q = Gs + (e - nA);
          else if (e < nA + nG + nT) q = Tr + (e - nA - nG);
          else q = Ttr + (e - nA - nG - nT);
          *q = v[u];
        }
      }
    }
  }
  bar();
  bool ok = chol_flag(d, Om, s, R, dv);
  if (force) ok = false;
  if (!ok) {
    if (rb == 0 && tid == 0) raise_flag(ctl, k, k - 2);
    return;
  }
  tri_inv_up(R, s, Ri, dv);
  double* coef = d.coef64;
  for (int e = tid; e < ss; e += NT) {
    const int i = e / s, c = e % s;
    double acc = 0.0;
#pragma unroll 8
    for (int t = 0; t < s; ++t) acc = fma(Ri[t * s + i], Pt[t * s + c], acc);
    Pn[e] = acc;
    if (!rowblk) {
      d.H[(int64_t)(r0 + i) * ld + (k - 2) * s + c] = R[e];
      coef[lay.C1() + e] = Ri[e];
      coef[lay.C2() + e] = Ri[e];
    }
  }
  // Y R^{-1} on rows a0 .. r0, Z R^{-1} on rows 0 .. a0 + s
  if (rowblk) {
    const int ny = wT * s, nz = wH * s;
    for (int e = tid; e < ny + nz; e += NT) {
      const bool isy = e < ny;
      const int f = isy ? e : e - ny;
      const int row = isy ? a0 + f / s : f / s, c = f % s;
      const double* g = Gs + row * ldg + (isy ? 0 : s);
      double acc = 0.0;
#pragma unroll 8
      for (int t = 0; t < s; ++t) acc = fma(g[t], Ri[t * s + c], acc);
      (isy ? YR : ZR)[row * s + c] = acc;
    }
  }
  bar();
  if (rowblk) {
    // Tc = -T(rows, a0:r0) YR(a0:r0),  Hc = T^T(rows, 0:a0+s) ZR(0:a0+s), the
    // sums split over kp parts when s^2 < NT and added in part order
    const int kp = ss >= NT ? 1 : NT / ss;
    const int pt = ss >= NT ? 0 : tid / ss;
    constexpr int kQ = kMaxS * kMaxS / NT;
    double at[kQ], ah[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) at[q] = ah[q] = 0.0;
    if (pt < kp) {
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        const int e = ss >= NT ? tid + q * NT : tid % ss;
        if (e < ss && (q == 0 || ss >= NT)) {
          const int i = e / s, c = e % s;
          double x = 0.0, y = 0.0;
          for (int u = pt; u < wT; u += kp) x = fma(Tr[i * wT + u], YR[(a0 + u) * s + c], x);
          for (int t = pt; t < wH; t += kp) y = fma(Ttr[i * wH + t], ZR[t * s + c], y);
          at[q] = x;
          ah[q] = y;
        }
      }
    }
    double* Tc = Om;   // Omega, P~ are dead: Tc, Hc (ss each) live there
    double* Hc = Pt;
    if (kp > 1) {
      for (int pass = 0; pass < 2; ++pass) {
        bar();
        if (pt < kp) red[pt * ss + tid % ss] = pass == 0 ? at[0] : ah[0];
        bar();
        for (int e = tid; e < ss; e += NT) {
          double sum = 0.0;
          for (int p = 0; p < kp; ++p) sum += red[p * ss + e];
          (pass == 0 ? Tc : Hc)[e] = pass == 0 ? -sum : sum;
        }
      }
    } else {
      bar();
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        const int e = tid + q * NT;
        if (e < ss) {
          Tc[e] = -at[q];
          Hc[e] = ah[q];
        }
      }
    }
    bar();
    for (int e = tid; e < ss; e += NT) {
      const int i = e / s, c = e % s, a = a0 + i;
      d.H[(int64_t)a * ld + (k - 1) * s + c] = Hc[e];
      coef[lay.B(0) + a * s + c] = -Hc[e];
      coef[lay.BF(0) + a * s + c] = -Hc[e];   // folded form: no A blocks (V_k = U R^{-1})
      d.T[(int64_t)a * ld + r0 + c] = Tc[e];
      d.Tt[(int64_t)(r0 + c) * ld + a] = Tc[e];
      // this block row's term of T_{1:k-1,k}^T (Z R^{-1}): Tc^T ZR(rows)
      double acc = 0.0;
      for (int t = 0; t < s; ++t) acc = fma(Tc[t * s + i], ZR[(a0 + t) * s + c], acc);
      part[(int64_t)rb * ss + e] = acc;
    }
  }
  // arrival: the last workgroup of this loop step finishes the column
  __threadfence();
  bar();
  if (tid == 0) is_last = (atomicAdd(&ctl->arrive[k], 1) == k - 1) ? 1 : 0;
  bar();
  if (!is_last) return;
  __threadfence();
  if (tid == 0) ctl->arrive[k] = 0;
  double* Hl = red;   // ss (red is free)
  for (int e = tid; e < ss; e += NT) {
    const int i = e / s, c = e % s;
    double acc = 0.0;
    for (int t = 0; t < s; ++t) acc = fma(Pn[i * s + t], Ri[t * s + c], acc);   // P R^{-1}
    for (int b = 0; b < k - 1; ++b) acc += part[(int64_t)b * ss + e];
    Hl[e] = acc;
    d.H[(int64_t)(r0 + i) * ld + (k - 1) * s + c] = acc;
    coef[lay.D() + e] = -acc;
  }
  bar();
  // C1 D = -R^{-1} H_{k,k}
  for (int e = tid; e < ss; e += NT) {
    const int i = e / s, c = e % s;
    double acc = 0.0;
    for (int t = 0; t < s; ++t) acc = fma(Ri[i * s + t], Hl[t * s + c], acc);
    coef[lay.C1D() + e] = -acc;
  }
  bar();
  publish_coef(d);
}

// Register-resident BMGS-ICWY step: used when the k s x s block column fits
// kIcRegs doubles per thread and its operands fit in LDS.
constexpr int kIcRegs = 8;
__host__ __device__ inline bool icwy_fast(int s, int k) {
  const int r0 = (k - 1) * s, ss = s * s;
  return k * ss <= kIcRegs * NT && 9 * ss + 5 * r0 * s <= LDS_DBL;
}

// Alg. 6 with the inverse compact WY form (BMGS-ICWY), loop step 2 <= k <= m:
// H_{1:k,k} = X solves T^T X = [Z; P] R^{-1} with T unit block upper
// triangular, its new column block being Y R^{-1}.  Block forward
// substitution, right-looking: once X_b is final, the right-hand sides of the
// later block rows take T(b, c)^T X_b at once, each thread updating the
// entries it owns (in registers).  T(b, c) for c <= k - 2 is read as rows of
// T^T, fetched two steps ahead; T(b, k - 1) is Y R^{-1} (LDS).
__global__ __launch_bounds__(NT) void small_icwy_kernel(Dense d, int k, int force) {
  __shared__ double lds[LDS_DBL];
  Ctl* ctl = d.ctl;
  if (ctl->stop) return;
  const int s = d.s, ld = d.ldh, ss = s * s;
  CoefLayout lay{s, d.mmax + 1};
  const int r0 = (k - 1) * s, ks = k * s, ldg = 2 * s;
  const double* Gk = d.G + (int64_t)k * d.gstride;
  const int tid = threadIdx.x;
  double* Om = lds;              // ss  Omega
  double* Pt = Om + ss;          // ss  P~
  double* R = Pt + ss;           // ss
  double* Ri = R + ss;           // ss
  double* Pn = Ri + ss;          // ss
  double* dv = Pn + ss;          // ss
  double* xb = dv + ss;          // ss  X_b
  double* xn = xb + ss;          // ss  X_{b+1}
  double* Hl = xn + ss;          // ss  X_{k-1}
  double* Gs = Hl + ss;          // r0 x 2s  [Y Z]
  double* YR = Gs + 2 * r0 * s;  // r0 x s
  double* c0b = YR + r0 * s;     // r0 x s   rows of T^T for one step
  double* c1b = c0b + r0 * s;    // r0 x s
  // T^T rows (b+1)s .. r0, columns bs .. bs+s: the step-b terms T(b, c), c <= k-2
  auto nstep = [&](int b) { return b <= k - 3 ? (r0 - (b + 1) * s) * s : 0; };
  {
    const int nA = 2 * ss, nG = 2 * r0 * s, n0 = nstep(0);
    const int tot = nA + nG + n0;
    for (int base = tid; base < tot; base += NT * 16) {
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        int e = base + u * NT;
        e = e < tot ? e : tot - 1;
        const double* p;
        if (e < nA) {
          const int f = e % ss;
          p = Gk + (int64_t)(r0 + f / s) * ldg + (e < ss ? 0 : s) + f % s;
        } else if (e < nA + nG) {
          p = Gk + (e - nA);
        } else {
          const int f = e - nA - nG;
          p = d.Tt + (int64_t)(s + f / s) * ld + f % s;
        }
        v[u] = *p;
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int e = base + u * NT;
        if (e < tot) {
          double* q;
          if (e < nA) q = Om + e;
          else if (e < nA + nG) q = Gs + (e - nA);
          else q = c0b + (e - nA - nG);
          *q = v[u];
        }
      }
    }
  }
  bar();
  bool ok = chol_flag(d, Om, s, R, dv);
  if (force) ok = false;
  if (!ok) {
    if (tid == 0) raise_flag(ctl, k, k - 2);
    return;
  }
  tri_inv_up(R, s, Ri, dv);
  double* coef = d.coef64;
  for (int e = tid; e < ss; e += NT) {
    const int i = e / s, c = e % s;
    double acc = 0.0;
#pragma unroll 8
    for (int t = 0; t < s; ++t) acc = fma(Ri[t * s + i], Pt[t * s + c], acc);
    Pn[e] = acc;
    d.H[(int64_t)(r0 + i) * ld + (k - 2) * s + c] = R[e];
    coef[lay.C1() + e] = Ri[e];
    coef[lay.C2() + e] = Ri[e];
  }
  for (int e = tid; e < r0 * s; e += NT) {
    const int a = e / s, c = e % s;
    double acc = 0.0;
#pragma unroll 8
    for (int t = 0; t < s; ++t) acc = fma(Gs[a * ldg + t], Ri[t * s + c], acc);
    YR[e] = acc;
  }
  bar();
  // right-hand sides [Z; P] R^{-1}, entries e = tid + q NT (row e / s)
  double xr[kIcRegs];
#pragma unroll
  for (int q = 0; q < kIcRegs; ++q) {
    const int e = tid + q * NT;
    const int a = e / s, c = e % s;
    double acc = 0.0;
    if (e < ks * s) {
      const double* g = a < r0 ? Gs + a * ldg + s : Pn + (a - r0) * s;
      for (int t = 0; t < s; ++t) acc = fma(g[t], Ri[t * s + c], acc);
    }
    xr[q] = acc;
    if (a < s && e < ks * s) xb[e] = acc;   // X_0
  }
  double* cur = c0b;
  double* nxt = c1b;
  double pfa[kIcRegs], pfb[kIcRegs];
  auto fetch = [&](int b, double (&pf)[kIcRegs]) {
    const int nn = nstep(b);
#pragma unroll
    for (int q = 0; q < kIcRegs; ++q) {
      const int e = tid + q * NT;
      pf[q] = e < nn ? d.Tt[(int64_t)((b + 1) * s + e / s) * ld + b * s + e % s] : 0.0;
    }
  };
  auto step = [&](int b, double (&pst)[kIcRegs], double (&pld)[kIcRegs]) {
    bar();   // X_b (xb) and the step-b rows of T^T (cur) are in LDS
    fetch(b + 2, pld);
    const int lo = (b + 1) * s;
#pragma unroll
    for (int q = 0; q < kIcRegs; ++q) {
      const int e = tid + q * NT;
      const int a = e / s, c = e % s;
      if (a >= lo && e < ks * s) {
        double x = xr[q];
        if (a < r0) {
          const double* tr = cur + (a - lo) * s;
          for (int t = 0; t < s; ++t) x = fma(-tr[t], xb[t * s + c], x);
        } else {
          for (int t = 0; t < s; ++t) x = fma(-YR[(b * s + t) * s + (a - r0)], xb[t * s + c], x);
        }
        xr[q] = x;
        if (a < lo + s) xn[(a - lo) * s + c] = x;
      }
    }
    const int nn = nstep(b + 1);
#pragma unroll
    for (int q = 0; q < kIcRegs; ++q) {
      const int e = tid + q * NT;
      if (e < nn) nxt[e] = pst[q];
    }
    double* t = cur;
    cur = nxt;
    nxt = t;
    t = xb;
    xb = xn;
    xn = t;
  };
  fetch(1, pfa);
  for (int b = 0; b <= k - 2; b += 2) {
    step(b, pfa, pfb);
    if (b + 1 <= k - 2) step(b + 1, pfb, pfa);
  }
  // H_{1:k,k} = X, the coefficients, the new T column Y R^{-1}
#pragma unroll
  for (int q = 0; q < kIcRegs; ++q) {
    const int e = tid + q * NT;
    if (e < ks * s) {
      const int a = e / s, c = e % s;
      const double x = xr[q];
      d.H[(int64_t)a * ld + (k - 1) * s + c] = x;
      if (a < r0) {
        coef[lay.B(0) + e] = -x;
        coef[lay.BF(0) + e] = -x;   // folded form: no A blocks (V_k = U R^{-1})
      } else {
        coef[lay.D() + (e - r0 * s)] = -x;
        Hl[e - r0 * s] = x;
      }
    }
  }
  for (int e = tid; e < r0 * s; e += NT) {
    const int a = e / s, c = e % s;
    d.T[(int64_t)a * ld + r0 + c] = YR[e];
    d.Tt[(int64_t)(r0 + c) * ld + a] = YR[e];
  }
  bar();
  // C1 D = -R^{-1} H_{k,k}
  for (int e = tid; e < ss; e += NT) {
    const int i = e / s, c = e % s;
    double acc = 0.0;
    for (int t = 0; t < s; ++t) acc = fma(Ri[i * s + t], Hl[t * s + c], acc);
    coef[lay.C1D() + e] = -acc;
  }
  bar();
  publish_coef(d);
}

template <bool ICWY>
__global__ __launch_bounds__(NT) void small_cwy_kernel(Dense d, int k, int force) {
  __shared__ double lds[LDS_DBL];
  Ctl* ctl = d.ctl;
  if (ctl->stop) return;
  const int s = d.s, ld = d.ldh, ss = s * s;
  CoefLayout lay{s, d.mmax + 1};
  const int r0 = (k - 1) * s, ks = k * s, ldg = 2 * s;
  const double* Gk = d.G + (int64_t)k * d.gstride;
  double* Om = lds;
  double* R = Om + ss;
  double* Ri = R + ss;
  double* Pn = Ri + ss;
  double* dinv = Pn + ss;
  double* YR = dinv + kMaxS;     // r0 x s
  double* ZPR = YR + r0 * s;     // ks x s
  double* Hc = ZPR + ks * s;     // ks x s
  double* Tc = Hc + ks * s;      // r0 x s
  double* G = Tc + r0 * s;       // ks x 2s, then the staging area
  double* Ts = G;
  const int tcap = LDS_DBL - (int)(G - lds);
  bcopy(Gk, G, ks * ldg);
  bar();
  for (int e = threadIdx.x; e < ss; e += NT) Om[e] = G[(r0 + e / s) * ldg + (e % s)];
  bar();
  bool ok = chol_flag(d, Om, s, R, dinv);
  if (force) ok = false;
  if (!ok) {
    if (threadIdx.x == 0) raise_flag(ctl, k, k - 2);
    return;
  }
  tri_inv_up(R, s, Ri, dinv);
  double* coef = d.coef64;
  for (int e = threadIdx.x; e < ss; e += NT) {
    d.H[(int64_t)(r0 + e / s) * ld + (k - 2) * s + (e % s)] = R[e];
    coef[lay.C1() + e] = Ri[e];
    coef[lay.C2() + e] = Ri[e];
    const int i = e / s, c = e % s;
    double acc = 0.0;
#pragma unroll 8
    for (int t = 0; t < s; ++t) acc = fma(Ri[t * s + i], G[(r0 + t) * ldg + s + c], acc);
    Pn[e] = acc;   // P = R^{-T} P~
  }
  rows_x_small(r0, s, G, ldg, Ri, 1.0, YR, s);        // Y R^{-1}
  rows_x_small(r0, s, G + s, ldg, Ri, 1.0, ZPR, s);   // Z R^{-1}
  bar();
  rows_x_small(s, s, Pn, s, Ri, 1.0, ZPR + r0 * s, s);   // P R^{-1}
  for (int e = threadIdx.x; e < r0 * s; e += NT) Tc[e] = ICWY ? YR[e] : 0.0;
  for (int e = threadIdx.x; e < ks * s; e += NT) Hc[e] = 0.0;
  bar();   // the Gram output is dead from here on: G becomes the staging area
  if (!ICWY) {
    // T_{1:k-1,1:k-1} is block upper triangular (identity diagonal blocks):
    // rows [t0, t1) restricted to columns [t0, r0) hold all of its nonzeros.
    for (int t0 = 0; t0 < r0;) {
      const int w = r0 - t0;
      int t1 = t0 + s;
      while (t1 + s <= r0 && (t1 + s - t0) * w <= tcap) t1 += s;
      const int tot = (t1 - t0) * w;
      for (int base = threadIdx.x; base < tot; base += NT * 16) {
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          int e = base + u * NT;
          e = e < tot ? e : tot - 1;
          v[u] = d.T[(int64_t)(t0 + e / w) * ld + t0 + (e % w)];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int e = base + u * NT;
          if (e < tot) Ts[e] = v[u];
        }
      }
      bar();
      // Tc(t) -= T(t, t0:r0) YR(t0:r0)   for t in [t0, t1)
      for (int e = threadIdx.x; e < (t1 - t0) * s; e += NT) {
        const int tr = e / s, c = e % s;
        const double* trow = Ts + tr * w;
        double a0 = 0.0, a1 = 0.0;
        int u = 0;
#pragma unroll 4
        for (; u + 1 < w; u += 2) {
          a0 = fma(trow[u], YR[(t0 + u) * s + c], a0);
          a1 = fma(trow[u + 1], YR[(t0 + u + 1) * s + c], a1);
        }
        if (u < w) a0 = fma(trow[u], YR[(t0 + u) * s + c], a0);
        Tc[(t0 + tr) * s + c] -= a0 + a1;
      }
      // Hc(a) += T(t0:t1, a)^T ZPR(t0:t1)   for a in [t0, r0)
      for (int e = threadIdx.x; e < w * s; e += NT) {
        const int a = e / s, c = e % s;
        double a0 = 0.0;
#pragma unroll 4
        for (int tr = 0; tr < t1 - t0; ++tr) a0 = fma(Ts[tr * w + a], ZPR[(t0 + tr) * s + c], a0);
        Hc[(t0 + a) * s + c] += a0;
      }
      bar();
      t0 = t1;
    }
    // last block row of T^T: [Tc^T, I]
    for (int e = threadIdx.x; e < ss; e += NT) {
      const int i = e / s, c = e % s;
      double a0 = ZPR[(r0 + i) * s + c];
      for (int t = 0; t < r0; ++t) a0 = fma(Tc[t * s + i], ZPR[t * s + c], a0);
      Hc[(r0 + i) * s + c] = a0;
    }
    bar();
  } else {
    // block forward substitution with T^T (unit block lower triangular):
    // X_b = ZPR_b - T(0:bs, bs:bs+s)^T X(0:bs), b = 0 .. k-1; column block
    // k-1 of T is Tc (= Y R^{-1}), the others are staged from global memory.
    for (int e = threadIdx.x; e < ss; e += NT) Hc[e] = ZPR[e];
    bar();
    for (int b0 = 1; b0 < k;) {
      // stage column blocks [b0, b1) of rows [0, (b1-1) s) (up to block k-2)
      int b1 = b0 + 1;
      while (b1 < k - 1 && (b1 * s) * ((b1 + 1 - b0) * s) <= tcap) ++b1;
      if (b0 >= k - 1) b1 = k;   // only the new column block is left
      const int w = (b1 - b0) * s;
      const int rows = (b1 - 1) * s;
      const bool global_part = b0 < k - 1;
      if (global_part) {
        const int wg = ((b1 < k - 1 ? b1 : k - 1) - b0) * s;
        const int tot = rows * wg;
        for (int base = threadIdx.x; base < tot; base += NT * 16) {
          double v[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            int e = base + u * NT;
            e = e < tot ? e : tot - 1;
            v[u] = d.T[(int64_t)(e / wg) * ld + b0 * s + (e % wg)];
          }
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            const int e = base + u * NT;
            if (e < tot) Ts[(e / wg) * w + (e % wg)] = v[u];
          }
        }
        bar();
      }
      for (int b = b0; b < b1; ++b) {
        const double* Tcol;
        int ldt;
        if (b == k - 1) {
          Tcol = Tc;
          ldt = s;
        } else {
          Tcol = Ts + (b - b0) * s;
          ldt = w;
        }
        mm_t<true, false>(s, s, b * s, -1.0, Tcol, ldt, Hc, s, 0.0, Hc + b * ss, s,
                          ZPR + b * ss, s);
      }
      b0 = b1;
    }
  }
  // H_{1:k,k}, the new T column (and its transpose), the update coefficients
  for (int e = threadIdx.x; e < ks * s; e += NT) {
    const int i = e / s, c = e % s;
    d.H[(int64_t)i * ld + (k - 1) * s + c] = Hc[e];
    if (i < r0) {
      coef[lay.B(0) + e] = -Hc[e];
      coef[lay.BF(0) + e] = -Hc[e];   // folded form: no A blocks (V_k = U R^{-1})
    } else {
      coef[lay.D() + e - r0 * s] = -Hc[e];
    }
  }
  // C1 D = -R^{-1} H_{k,k}
  for (int e = threadIdx.x; e < ss; e += NT) {
    const int i = e / s, c = e % s;
    double acc = 0.0;
    for (int t = 0; t < s; ++t) acc = fma(Ri[i * s + t], Hc[(r0 + t) * s + c], acc);
    coef[lay.C1D() + e] = -acc;
  }
  for (int e = threadIdx.x; e < r0 * s; e += NT) {
    const int i = e / s, c = e % s;
    d.T[(int64_t)i * ld + r0 + c] = Tc[e];
    d.Tt[(int64_t)(r0 + c) * ld + i] = Tc[e];
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
             fit ? LDS_DBL - 2 * ks * s : 0, d.mgs != 0);
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

// Alg. 5, after Z = V_{1:k}^T V_{k+1}: T_{1:k,k+1} = -T Z T_{k+1,k+1} (SVL)
// or Z T_{k+1,k+1} (LTS), with T_{k+1,k+1} the muscle's factor (I for
// CholQR / HouseQR, unit upper triangular for the MGS muscles).  Column k is
// then final (small_finalize).
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
  if (d.mgs) {
    // times T_{k+1,k+1} (unit upper triangular): column c of a row takes
    // sum_{t <= c} row[t] T_{k+1,k+1}[t][c]; one thread per row of Tc
    bar();
    const double* Tkk = d.T + (int64_t)ks * ld + ks;
    for (int a = threadIdx.x; a < ks; a += NT) {
      double* row = Tc + (int64_t)a * ld;
      for (int c = s - 1; c >= 1; --c) {
        double acc = row[c];
        for (int t = 0; t < c; ++t) acc = fma(row[t], Tkk[(int64_t)t * ld + c], acc);
        row[c] = acc;
      }
    }
  }
  bar();
  for (int e = threadIdx.x; e < ks * s; e += NT) {
    const int i = e / s, c = e % s;
    d.Tt[(int64_t)(ks + c) * ld + i] = Tc[(int64_t)i * ld + c];
  }
}

// Alg. 3 (BCGS-PIP), loop step k (1-based).  From the one fused Gram
// [Y; Omega] = [V_{1:k} W]^T W: H_{1:k,k} = Y, H_{k+1,k} = R = chol(Omega -
// Y^T Y) (the Pythagorean form of the norm of W - V_{1:k} Y, with the
// breakdown flag of Sec. 4), and the coefficients of the one projection
// V_{k+1} = (W - V_{1:k} Y) R^{-1} (C2 = R^{-1}, B_i = -Y_i R^{-1}).
// Column k of H is final afterwards.  FIT: the Gram output is copied to LDS.
template <bool FIT>
__global__ __launch_bounds__(NT) void small_pip_kernel(Dense d, int k, int force) {
  __shared__ double lds[LDS_DBL];
  Ctl* ctl = d.ctl;
  if (ctl->stop) return;
  const int s = d.s, ld = d.ldh, ss = s * s, ks = k * s;
  CoefLayout lay{s, d.mmax + 1};
  double* Om = lds;
  double* R = Om + ss;
  double* Ri = R + ss;
  double* dinv = Ri + ss;   // kMaxS
  const int lused = 3 * ss + kMaxS;
  const double* Gp;
  if constexpr (FIT) {
    bcopy(d.G, lds + lused, (ks + s) * s);
    Gp = lds + lused;
    bar();
  } else {
    Gp = d.G;
  }
  // Omega - Y^T Y
  mm_t<true, false>(s, s, ks, -1.0, Gp, s, Gp, s, 0.0, Om, s, Gp + (int64_t)ks * s, s);
  bool ok = chol_flag(d, Om, s, R, dinv);
  if (force) ok = false;
  if (!ok) {
    if (threadIdx.x == 0) raise_flag(ctl, k, k - 1);
    return;
  }
  tri_inv_up(R, s, Ri, dinv);
  double* coef = d.coef64;
  double* Hc = d.H + (int64_t)(k - 1) * s;
  for (int e = threadIdx.x; e < ss; e += NT) {
    coef[lay.C2() + e] = Ri[e];
    d.Rinv[e] = Ri[e];
    Hc[(int64_t)(ks + e / s) * ld + (e % s)] = R[e];
  }
  // one pass over the rows of Y: H_{1:k,k} = Y and B = -Y R^{-1}
  for (int e = threadIdx.x; e < ks * s; e += NT) {
    const int i = e / s, c = e % s;
    const double* y = Gp + (int64_t)i * s;
    double b = 0.0;
#pragma unroll 8
    for (int t = 0; t < s; ++t) b = fma(y[t], Ri[t * s + c], b);
    coef[lay.B(0) + e] = -b;
    Hc[(int64_t)i * ld + c] = y[c];
  }
  bar();
  publish_coef(d);
}

// Alg. 4 (BCGS-PIO), loop step k (1-based).  Y = H_{1:k,k} = V_{1:k}^T W is
// in G; the IntraOrtho of the block-diagonal [W 0; 0 Y] has the R factor
// [R_W 0; 0 R_H]: with CholQR, R_W = chol(W^T W) (W^T W in G2) and
// R_H = chol(Y^T Y), each flagging; with HouseQR, R_W is the TSQR factor
// already in H_{k+1,k} (it flagged there if it failed) and R_H^T R_H enters
// as Y^T Y (equal to rounding; the ks x s QR of Y is not formed).  Then
// H_{k+1,k} = chol(R_W^T R_W - R_H^T R_H) (flag), H_{1:k,k} = Y and the
// coefficients of V_{k+1} = (W - V_{1:k} Y) R^{-1}, as in BCGS-PIP.
template <bool FIT>
__global__ __launch_bounds__(NT) void small_pio_kernel(Dense d, int k, int force, int house) {
  __shared__ double lds[LDS_DBL];
  Ctl* ctl = d.ctl;
  if (ctl->stop) return;
  const int s = d.s, ld = d.ldh, ss = s * s, ks = k * s;
  CoefLayout lay{s, d.mmax + 1};
  double* RW = lds;
  double* RH = RW + ss;
  double* M = RH + ss;
  double* R = M + ss;
  double* Ri = R + ss;
  double* dinv = Ri + ss;   // kMaxS
  const int lused = 5 * ss + kMaxS;
  const double* Gp;
  if constexpr (FIT) {
    bcopy(d.G, lds + lused, ks * s);
    Gp = lds + lused;
  } else {
    Gp = d.G;
  }
  bar();
  double* Hc = d.H + (int64_t)(k - 1) * s;
  double* Hsub = Hc + (int64_t)ks * ld;   // H_{k+1,k}
  bool ok = true;
  if (house) {
    for (int e = threadIdx.x; e < ss; e += NT) RW[e] = Hsub[(int64_t)(e / s) * ld + (e % s)];
    bar();
    // M = R_W^T R_W - Y^T Y
    mm_t<true, false>(s, s, s, 1.0, RW, s, RW, s, 0.0, R, s);
    bar();
    mm_t<true, false>(s, s, ks, -1.0, Gp, s, Gp, s, 0.0, M, s, R, s);
    bar();
  } else {
    ok = chol_flag(d, d.G2, s, RW);
    if (ok) {
      mm_t<true, false>(s, s, ks, 1.0, Gp, s, Gp, s, 0.0, M, s);   // Y^T Y
      bar();
      ok = chol_flag(d, M, s, RH);
    }
    if (ok) {
      // M = R_W^T R_W - R_H^T R_H
      mm_t<true, false>(s, s, s, 1.0, RW, s, RW, s, 0.0, R, s);
      bar();
      mm_t<true, false>(s, s, s, -1.0, RH, s, RH, s, 0.0, M, s, R, s);
      bar();
    }
  }
  if (ok) ok = chol_flag(d, M, s, R, dinv);
  if (force) ok = false;
  if (!ok) {
    if (threadIdx.x == 0) raise_flag(ctl, k, k - 1);
    return;
  }
  tri_inv_up(R, s, Ri, dinv);
  double* coef = d.coef64;
  for (int e = threadIdx.x; e < ss; e += NT) {
    coef[lay.C2() + e] = Ri[e];
    d.Rinv[e] = Ri[e];
    Hsub[(int64_t)(e / s) * ld + (e % s)] = R[e];
  }
  for (int e = threadIdx.x; e < ks * s; e += NT) {
    const int i = e / s, c = e % s;
    const double* y = Gp + (int64_t)i * s;
    double b = 0.0;
#pragma unroll 8
    for (int t = 0; t < s; ++t) b = fma(y[t], Ri[t * s + c], b);
    coef[lay.B(0) + e] = -b;
    Hc[(int64_t)i * ld + c] = y[c];
  }
  bar();
  publish_coef(d);
}

// Column-wise MGS-SVL / MGS-LTS muscle (Sec. 5; the column version of
// Alg. 5), one phase per launch; the host runs the column loop, each sync a
// Gram product of the block being orthonormalized with itself (its column j
// gives the inner products of column j with the earlier ones), each change
// of the block an in-place update with the coefficients set here.  The
// muscle's R and T live in P and J (unused by the skeletons while a muscle
// runs).  For column j: PROJ h = T^T y (SVL) or T^{-T} y (LTS) from
// y = Q_{1:j-1}^T x_j and x_j -= Q h; NORM r = sqrt(w^T w) (flag when not
// positive finite) and x_j /= r; Z: T_{1:j-1,j} = -T z (SVL) or z (LTS).
// FINISH places R and T: the cycle start (Beta, g = Beta C, the control
// word, T_{1,1} for Alg. 5), Alg. 5's IntraOrtho (H_{k+1,k}, T_{k+1,k+1}) or
// Alg. 2's (H_{k+1,k}).
__device__ void mgs_flag(Ctl* ctl, int mode, int k) {
  if (mode == MGS_START) {
    ctl->status = ST_FLAGGED;
    ctl->flag_step = 0;
    ctl->last_valid = 0;
    ctl->stop = 1;
  } else {
    raise_flag(ctl, k, k - 1);
  }
}

__global__ __launch_bounds__(NT) void small_mgs_kernel(Dense d, int phase, int j, int mode, int k,
                                                      int force) {
  __shared__ double lds[2 * kMaxS * kMaxS];
  Ctl* ctl = d.ctl;
  const int s = d.s, ss = s * s, ld = d.ldh;
  CoefLayout lay{s, d.mmax + 1};
  double* Rm = d.P;
  double* Tm = d.J;
  double* coef = d.coef64;
  const bool lts = d.mgs == 2;
  if (phase == MGS_INIT) {
    if (mode == MGS_START) {
      if (threadIdx.x == 0) {
        ctl->j = 0;
        ctl->flag_step = -1;
        ctl->last_valid = 1 << 30;
        ctl->status = ST_RUNNING;
        ctl->stop = 0;
      }
    } else if (ctl->stop) {
      return;
    }
    for (int e = threadIdx.x; e < ss; e += NT) {
      const double id = (e / s == e % s) ? 1.0 : 0.0;
      Rm[e] = 0.0;
      Tm[e] = id;
      coef[lay.C1() + e] = id;
      coef[lay.C2() + e] = id;
    }
    bar();
    publish_coef(d);
    return;
  }
  if (ctl->stop) return;
  const double* G = d.G2;
  if (phase == MGS_PROJ) {
    double* h = lds;
    if (threadIdx.x == 0) {
      for (int i = 0; i < j; ++i) {
        double acc;
        if (lts) {   // T^T unit lower triangular: forward substitution
          acc = G[i * s + j];
          for (int t = 0; t < i; ++t) acc = fma(-Tm[t * s + i], h[t], acc);
        } else {     // (T^T y)_i = sum_{t <= i} T[t][i] y_t
          acc = 0.0;
          for (int t = 0; t <= i; ++t) acc = fma(Tm[t * s + i], G[t * s + j], acc);
        }
        h[i] = acc;
      }
    }
    bar();
    for (int e = threadIdx.x; e < ss; e += NT) {
      const int r = e / s, c = e % s;
      coef[lay.C1() + e] = (c == j && r < j) ? -h[r] : (r == c ? 1.0 : 0.0);
      if (c == j && r < j) Rm[e] = h[r];
    }
    bar();
    publish_coef(d);
    return;
  }
  if (phase == MGS_NORM) {
    const double rr = G[j * s + j];
    if (!(rr > 0.0) || !isfinite(rr)) {
      if (threadIdx.x == 0) mgs_flag(ctl, mode, k);
      return;
    }
    const double r = sqrt(rr);
    for (int e = threadIdx.x; e < ss; e += NT) {
      const int a = e / s, c = e % s;
      coef[lay.C1() + e] = a == c ? (a == j ? 1.0 / r : 1.0) : 0.0;
    }
    if (threadIdx.x == 0) Rm[j * s + j] = r;
    bar();
    publish_coef(d);
    return;
  }
  if (phase == MGS_Z) {
    for (int i = threadIdx.x; i < j; i += NT) {
      if (lts) {
        Tm[i * s + j] = G[i * s + j];
      } else {
        double acc = 0.0;
        for (int t = i; t < j; ++t) acc = fma(Tm[i * s + t], G[t * s + j], acc);
        Tm[i * s + j] = -acc;
      }
    }
    return;
  }
  // MGS_FINISH
  if (force) {
    if (threadIdx.x == 0) mgs_flag(ctl, mode, k);
    return;
  }
  double* R = lds;
  double* Ri = lds + ss;
  for (int e = threadIdx.x; e < ss; e += NT) R[e] = Rm[e];
  bar();
  tri_inv_up(R, s, Ri);
  for (int e = threadIdx.x; e < ss; e += NT) d.Rinv[e] = Ri[e];
  const bool put_t = d.skel == LSBA_BMGS_SVL || d.skel == LSBA_BMGS_LTS;
  if (mode == MGS_START) {
    for (int e = threadIdx.x; e < ss; e += NT) d.Beta[e] = R[e];
    for (int e = threadIdx.x; e < (d.mmax + 1) * ss; e += NT) d.g[e] = 0.0;
    bar();
    mm(s, s, s, 1.0, R, s, false, d.C, s, false, 0.0, d.g, s);
  } else {
    double* Hsub = d.H + (int64_t)(k * s) * ld + (k - 1) * s;
    for (int e = threadIdx.x; e < ss; e += NT) Hsub[(int64_t)(e / s) * ld + (e % s)] = R[e];
  }
  if (put_t && mode != MGS_IOB) {
    const int o = mode == MGS_START ? 0 : k * s;
    for (int e = threadIdx.x; e < ss; e += NT) {
      const int a = e / s, c = e % s;
      d.T[(int64_t)(o + a) * ld + o + c] = Tm[e];
      d.Tt[(int64_t)(o + c) * ld + o + a] = Tm[e];
    }
  }
  bar();
}

// Alg. 2 (BMGS), loop step k, inner step i (both 1-based): H_{i,k} = V_i^T W
// (the Gram output) and the coefficients of W <- W - V_i H_{i,k}.
__global__ __launch_bounds__(NT) void small_bmgs_kernel(Dense d, int k, int i) {
  Ctl* ctl = d.ctl;
  if (ctl->stop) return;
  const int s = d.s, ld = d.ldh, ss = s * s;
  CoefLayout lay{s, d.mmax + 1};
  double* Hc = d.H + (int64_t)(i - 1) * s * ld + (k - 1) * s;
  for (int e = threadIdx.x; e < ss; e += NT) {
    const double v = d.G[e];
    Hc[(int64_t)(e / s) * ld + (e % s)] = v;
    d.coef64[lay.C2() + e] = (e / s == e % s) ? 1.0 : 0.0;
    d.coef64[lay.B(i - 1) + e] = -v;
  }
  bar();
  publish_coef(d);
}

}  // namespace

#define SMALL_LAUNCH(...)                 \
  do {                                    \
    if (tm) tm->begin(st, KK_SMALL);      \
    __VA_ARGS__;                          \
    if (tm) tm->end(st, KK_SMALL, 0.0);   \
  } while (0)

void launch_small_start(hipStream_t st, const Dense& d, int force_flag, KTimer* tm) {
  if (skel_uses_t(d.skel)) {
    const int64_t tot = (int64_t)d.ldh * d.ldh;
    const int blocks = (int)std::min<int64_t>((tot + NT - 1) / NT, 1024);
    SMALL_LAUNCH(t_identity_kernel<<<blocks, NT, 0, st>>>(d));
  }
  SMALL_LAUNCH(small_start_kernel<<<1, NT, 0, st>>>(d, force_flag));
}
void launch_small_delayed(hipStream_t st, const Dense& d, int k, int m, int force_flag,
                          KTimer* tm) {
  if (d.skel == LSBA_BMGS_CWY && k >= 2 && k <= m && cwy_rows_lds(d.s, k) <= LDS_DBL) {
    SMALL_LAUNCH(small_cwy_rows_kernel<<<k, NT, 0, st>>>(d, k, force_flag));
    return;
  }
  if (d.skel == LSBA_BMGS_ICWY && k >= 2 && k <= m && icwy_fast(d.s, k)) {
    SMALL_LAUNCH(small_icwy_kernel<<<1, NT, 0, st>>>(d, k, force_flag));
    return;
  }
  if (d.skel != LSBA_BCGSI_LS && k >= 2 && k <= m && cwy_fits(d.s, k)) {
    if (d.skel == LSBA_BMGS_ICWY)
      SMALL_LAUNCH(small_cwy_kernel<true><<<1, NT, 0, st>>>(d, k, force_flag));
    else
      SMALL_LAUNCH(small_cwy_kernel<false><<<1, NT, 0, st>>>(d, k, force_flag));
    return;
  }
  if (d.skel == LSBA_BCGSI_LS && k >= 2) {
    const int s = d.s, ldg = (k == m + 1) ? s : 2 * s;
    if (k * s * ldg <= LDS_DBL - (5 * s * s + kMaxS))
      SMALL_LAUNCH(small_core_kernel<true><<<1, NT, 0, st>>>(d, k, m, force_flag));
    else
      SMALL_LAUNCH(small_core_kernel<false><<<1, NT, 0, st>>>(d, k, m, force_flag));
    const int rows = (k - 1) * s * s;
    const int blocks = std::min((rows + NT - 1) / NT, 128);
    SMALL_LAUNCH(small_core_rows_kernel<<<blocks, NT, 0, st>>>(d, k, m));
  }
  else
    SMALL_LAUNCH(small_delayed_kernel<<<1, NT, 0, st>>>(d, k, m, force_flag));
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
void launch_small_pip(hipStream_t st, const Dense& d, int k, int force_flag, KTimer* tm) {
  const int s = d.s;
  if ((k + 1) * s * s <= LDS_DBL - (3 * s * s + kMaxS))
    SMALL_LAUNCH(small_pip_kernel<true><<<1, NT, 0, st>>>(d, k, force_flag));
  else
    SMALL_LAUNCH(small_pip_kernel<false><<<1, NT, 0, st>>>(d, k, force_flag));
}
void launch_small_pio(hipStream_t st, const Dense& d, int k, int force_flag, int house,
                      KTimer* tm) {
  const int s = d.s;
  if (k * s * s <= LDS_DBL - (5 * s * s + kMaxS))
    SMALL_LAUNCH(small_pio_kernel<true><<<1, NT, 0, st>>>(d, k, force_flag, house));
  else
    SMALL_LAUNCH(small_pio_kernel<false><<<1, NT, 0, st>>>(d, k, force_flag, house));
}
void launch_small_mgs(hipStream_t st, const Dense& d, int phase, int j, int mode, int k,
                      int force_flag, KTimer* tm) {
  SMALL_LAUNCH(small_mgs_kernel<<<1, NT, 0, st>>>(d, phase, j, mode, k, force_flag));
}
void launch_t_identity(hipStream_t st, const Dense& d, KTimer* tm) {
  const int64_t tot = (int64_t)d.ldh * d.ldh;
  const int blocks = (int)std::min<int64_t>((tot + NT - 1) / NT, 1024);
  SMALL_LAUNCH(t_identity_kernel<<<blocks, NT, 0, st>>>(d));
}
void launch_small_bmgs(hipStream_t st, const Dense& d, int k, int i, KTimer* tm) {
  SMALL_LAUNCH(small_bmgs_kernel<<<1, NT, 0, st>>>(d, k, i));
}
}  // namespace lsba
