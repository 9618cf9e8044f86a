// Small dense kernels off the basis path: the per-column QR update, residual
// estimate and convergence test (with, for Alg. 7, the H column and the J
// recurrence), the end of a cycle, and the loss-of-orthogonality record.
#include "small_common.h"

namespace lsba {

namespace {

// Alg. 7 off the basis path, after loop step k >= 2 (queued on a second
// stream behind small_core of the same step): H_{1:k-1,k-1} = J + Y and, for
// k <= m, the J recurrence J = ([Z; P] - H_{1:k,1:k-1} Y) R^{-1}.  Every
// quantity here is row-local (row a of the new H column, of T2 and of J
// depends on row a of J, Y, Z, H only), so workgroup rb takes block row rb of
// the k block rows and the kernel runs k workgroups side by side.  It reads
// only this step's slots (Gram output, R^{-1}, P) and H, J, so it may lag the
// basis kernels.
__global__ __launch_bounds__(NT) void small_side_kernel(Dense d, int k, int m) {
  __shared__ double lds[LDS_DBL];
  Ctl* ctl = d.ctl;
  {
    const int st = ctl->status;
    if (st == ST_CONVERGED || st == ST_ITERCAP) return;
    // A flag raised at a loop step <= k was raised by a kernel this one is
    // stream-ordered after, so its flag_step is visible here.  A flag raised
    // concurrently (by a basis-path kernel of a later step) may show its
    // status before its flag_step; whatever value is read then lies outside
    // [0, k], and column k - 1 is still final under that flag, so the step
    // must run.
    const int fs = ctl->flag_step;
    if (fs >= 0 && fs <= k) return;
  }
  const int s = d.s, ld = d.ldh, ss = s * s;
  const bool last = (k == m + 1);
  const int ldg = last ? s : 2 * s;
  const int r0 = (k - 1) * s, c1 = (k - 2) * s;
  const int rb = blockIdx.x, a0 = rb * s;
  const double* Gk = d.G + (int64_t)k * d.gstride;   // [Y Z]: row t holds Y(t, :), Z(t, :)
  const int tid = threadIdx.x;
  // block rb of the new column: J + Y above block row k, R = H_{k,k-1} in it
  double* hc = lds;            // ss
  double* t2 = hc + ss;        // ss
  double* stage = t2 + ss;     // chunks of H rows (s x ck) and Y rows (ck x s); R^{-1}
  for (int e = tid; e < ss; e += NT) {
    const int i = e / s, c = e % s, a = a0 + i;
    double v;
    if (rb < k - 1) {
      v = d.J[(int64_t)a * s + c] + Gk[(int64_t)a * ldg + c];
      d.H[(int64_t)a * ld + c1 + c] = v;
    } else {
      v = d.H[(int64_t)(r0 + i) * ld + c1 + c];
    }
    hc[e] = v;
  }
  if (last) return;
  // T2 rows a0 .. a0 + s: sum over the band t in [lo, r0) of H(a, t) Y(t, :);
  // block row rb of H has nonzeros from column block rb - 1 on, and its
  // entries in the last column block are hc.
  const int lo = (rb > 1 ? rb - 1 : 0) * s;
  const int ck = (LDS_DBL - 2 * ss) / (2 * s);
  double* hs = stage;            // s x ck
  double* ys = stage + s * ck;   // ck x s
  // outputs of this thread: e = tid % ss (+ q NT for s^2 > NT); split of the
  // t range over kp parts when s^2 < NT
  const int kp = ss >= NT ? 1 : NT / ss;
  const int part = ss >= NT ? 0 : tid / ss;
  const bool active = part < kp;
  constexpr int kQ = kMaxS * kMaxS / NT;
  double acc[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) acc[q] = 0.0;
  for (int t0 = lo; t0 < r0; t0 += ck) {
    const int w = (r0 - t0) < ck ? (r0 - t0) : ck;
    bar();   // hc written / previous chunk consumed
    const int nh = s * w;
    for (int base = tid; base < 2 * nh; base += NT * 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        int e = base + u * NT;
        e = e < 2 * nh ? e : 2 * nh - 1;
        if (e < nh) {
          const int i = e / w, t = t0 + e % w;
          v[u] = t < c1 ? d.H[(int64_t)(a0 + i) * ld + t] : hc[i * s + (t - c1)];
        } else {
          const int f = e - nh, t = t0 + f / s;
          v[u] = Gk[(int64_t)t * ldg + f % s];
        }
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = base + u * NT;
        if (e < nh) hs[e] = v[u];
        else if (e < 2 * nh) ys[e - nh] = v[u];
      }
    }
    bar();
    if (active) {
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        const int e = (ss >= NT ? tid + q * NT : tid % ss);
        if (e < ss && (q == 0 || ss >= NT)) {
          const int i = e / s, c = e % s;
          const double* hr = hs + i * w;
          double x0 = 0.0, x1 = 0.0;
          int tt = part;
          for (; tt + kp < w; tt += 2 * kp) {
            x0 = fma(hr[tt], ys[tt * s + c], x0);
            x1 = fma(hr[tt + kp], ys[(tt + kp) * s + c], x1);
          }
          if (tt < w) x0 = fma(hr[tt], ys[tt * s + c], x0);
          acc[q] += x0 + x1;
        }
      }
    }
  }
  bar();
  // T2 = [Z; P] - (sum over the parts), in a fixed order
  if (kp > 1) {
    if (active) stage[part * ss + tid % ss] = acc[0];
    bar();
    for (int e = tid; e < ss; e += NT) {
      double sum = 0.0;
      for (int p = 0; p < kp; ++p) sum += stage[p * ss + e];
      const int i = e / s, c = e % s;
      const double zp = rb < k - 1 ? Gk[(int64_t)(a0 + i) * ldg + s + c]
                                   : d.PS[(int64_t)k * ss + e];
      t2[e] = zp - sum;
    }
  } else {
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int e = tid + q * NT;
      if (e < ss) {
        const int i = e / s, c = e % s;
        const double zp = rb < k - 1 ? Gk[(int64_t)(a0 + i) * ldg + s + c]
                                     : d.PS[(int64_t)k * ss + e];
        t2[e] = zp - acc[q];
      }
    }
  }
  bar();
  // J rows = T2 R^{-1}
  double* ri = stage;
  for (int e = tid; e < ss; e += NT) ri[e] = d.RiS[(int64_t)k * ss + e];
  bar();
  for (int e = tid; e < ss; e += NT) {
    const int i = e / s, c = e % s;
    double x = 0.0;
    for (int u = 0; u < s; ++u) x = fma(t2[i * s + u], ri[u * s + c], x);
    d.J[(int64_t)(a0 + i) * s + c] = x;
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
  finalize_column(d, col, lds, LDS_DBL, d.H + (int64_t)(col - 1) * d.s, d.ldh);
}

// Register-resident back substitution / M chain of small_cycle_end: used
// when the j s x s block coefficient vector fits kCeRegs doubles per thread.
constexpr int kCeRegs = 8;
__host__ __device__ inline bool cycle_end_fast(int s, int j) { return j * s * s <= kCeRegs * NT; }

// Xi = R^{-1} g by block back substitution, right-looking: after block b is
// solved, the rows above it take their update from column block b at once,
// each thread updating the entries of Xi it owns (in registers); the column
// block for the next step is fetched while this one is applied.  The
// diagonal blocks are inverted up front, all of them side by side.  Writes Xi
// to the A coefficients and returns (in LDS, at xlast) its last block.
// GMRES, not final: M = Q_1 ... Q_{j-1} E_j S with S = D^{-T} (H_{j+1,j}^T
// H_{j+1,j}); Q_i touches block rows i, i + 1 only and block row i is still
// zero when it applies, so the chain carries one s x s block w:
// M_{i+1} = Q_i[s:2s, s:2s]^T w and w <- Q_i[s:2s, 0:s]^T w (Q_i^T stored).
__device__ void cycle_end_regs(const Dense& d, int j, bool want_m, double* lds) {
  const int s = d.s, ld = d.ldh, ss = s * s, js = j * s, n = js * s;
  CoefLayout lay{s, d.mmax + 1};
  const int tid = threadIdx.x;
  double* Dg = lds;                    // j x ss   diagonal blocks of R
  double* Ri = Dg + j * ss;            // j x ss   their inverses
  double* rc0 = Ri + j * ss;           // js x s   column block of R above the diagonal
  double* rc1 = rc0 + n;               // js x s   (double buffer)
  double* xb = rc1 + n;                // ss       solved block
  double* xn = xb + ss;                // ss       next block's right-hand side
  double* Qs = xn + ss;                // (j - 1) x (s x 2s)   rows s..2s of each Q_i^T
  double* w0 = Qs + (j - 1) * 2 * ss;  // ss
  double* w1 = w0 + ss;                // ss
  double* Dt = w1 + ss;                // ss
  double xr[kCeRegs];
#pragma unroll
  for (int q = 0; q < kCeRegs; ++q) {
    const int e = tid + q * NT;
    xr[q] = e < n ? d.g[e] : 0.0;
  }
  {
    // one batched gather: diagonal blocks, column block j above its
    // diagonal, rows s..2s of each Q_i^T
    const int nD = j * ss, nR = (j - 1) * ss, nQ = want_m ? (j - 1) * 2 * ss : 0;
    const int tot = nD + nR + nQ;
    for (int base = tid; base < tot; base += NT * 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        int e = base + u * NT;
        e = e < tot ? e : tot - 1;
        const double* p;
        if (e < nD) {
          const int b = e / ss, f = e % ss;
          p = d.Rf + (int64_t)(b * s + f / s) * ld + b * s + f % s;
        } else if (e < nD + nR) {
          const int f = e - nD;
          p = d.Rf + (int64_t)(f / s) * ld + (j - 1) * s + f % s;
        } else {
          const int f = e - nD - nR, i = f / (2 * ss);
          p = d.Qt + (int64_t)i * 4 * ss + 2 * ss + f % (2 * ss);
        }
        v[u] = *p;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = base + u * NT;
        if (e < tot) lds[e < nD ? e : (e < nD + nR ? 2 * nD + (e - nD) : (Qs - lds) + (e - nD - nR))] = v[u];
      }
    }
  }
  bar();
  // inverses of the diagonal blocks: thread (b, c) solves R_bb x = e_c
  if (tid < j * s) {
    const int b = tid / s, c = tid % s;
    const double* R = Dg + b * ss;
    double* X = Ri + b * ss;
    for (int r = s - 1; r >= 0; --r) {
      double x = (r == c) ? 1.0 : 0.0;
      for (int t = r + 1; t < s; ++t) x = fma(-R[r * s + t], X[t * s + c], x);
      X[r * s + c] = r > c ? 0.0 : x / R[r * s + r];
    }
  }
  bar();
  // last block: FOM's comes with the column's test, GMRES solves R_jj x = g_j
  double* coefA = d.coef64 + lay.A(0);
  for (int e = tid; e < ss; e += NT) {
    const int r = e / s, c = e % s;
    double x;
    if (d.method == LSBA_FOM) {
      x = d.ylast[e];
    } else {
      const double* R = Ri + (j - 1) * ss;
      const double* g = d.g + (int64_t)(j - 1) * ss;
      x = 0.0;
      for (int t = 0; t < s; ++t) x = fma(R[r * s + t], g[t * s + c], x);
    }
    xb[e] = x;
    coefA[(int64_t)(j - 1) * ss + e] = x;
  }
  bar();
  // Thread tid owns entries e = tid + q NT of Xi (row e / s, column tid % s
  // for every q: NT is a multiple of s for the power-of-two block sizes; other
  // s take the column per entry).  Column block b - 1 is fetched into
  // registers one step ahead (barriers do not wait for global loads).
  double* cur = rc0;
  double* nxt = rc1;
  double pfa[kCeRegs], pfb[kCeRegs];
  auto fetch = [&](int cb, double (&pf)[kCeRegs]) {   // column block cb, rows above its diagonal
    const int nn = cb >= 2 ? (cb - 1) * ss : 0;
#pragma unroll
    for (int q = 0; q < kCeRegs; ++q) {
      const int e = tid + q * NT;
      pf[q] = e < nn ? d.Rf[(int64_t)(e / s) * ld + (cb - 1) * s + e % s] : 0.0;
    }
  };
  auto step = [&](int b, double (&pst)[kCeRegs], double (&pld)[kCeRegs]) {
    // rows above block b take column block b (cur); block b - 1 (in pst)
    // goes to LDS; block b - 2 is fetched into pld
    fetch(b - 2, pld);
    const int top = (b - 1) * s;
    // column tid % s of the solved block, in registers for s <= 8
    constexpr int kXc = 8;
    double xc[kXc];
    const int cc = tid % s;
#pragma unroll
    for (int t = 0; t < kXc; ++t) xc[t] = t < s ? xb[t * s + cc] : 0.0;
#pragma unroll
    for (int q = 0; q < kCeRegs; ++q) {
      const int e = tid + q * NT;
      const int a = e / s, c = e % s;
      if (a < top) {
        double x = xr[q];
        const double* ra = cur + a * s;
        if (c == cc && s <= kXc) {
#pragma unroll
          for (int t = 0; t < kXc; ++t)
            if (t < s) x = fma(-ra[t], xc[t], x);
        } else {
          for (int t = 0; t < s; ++t) x = fma(-ra[t], xb[t * s + c], x);
        }
        xr[q] = x;
        if (a >= top - s) xn[(a - (top - s)) * s + c] = x;
      }
    }
    const int nn = (b - 2) * ss;
#pragma unroll
    for (int q = 0; q < kCeRegs; ++q) {
      const int e = tid + q * NT;
      if (e < nn) nxt[e] = pst[q];
    }
    bar();
    // block b - 1 = R_{b-1,b-1}^{-1} (its updated right-hand side)
    for (int e = tid; e < ss; e += NT) {
      const int r = e / s, c = e % s;
      const double* R = Ri + (b - 2) * ss;
      double x = 0.0;
      for (int t = 0; t < s; ++t) x = fma(R[r * s + t], xn[t * s + c], x);
      xb[e] = x;
      coefA[(int64_t)(b - 2) * ss + e] = x;
    }
    bar();
    double* t = cur;
    cur = nxt;
    nxt = t;
  };
  fetch(j - 1, pfa);
  for (int b = j; b >= 2; b -= 2) {
    step(b, pfa, pfb);
    if (b - 1 >= 2) step(b - 1, pfb, pfa);
  }
  if (!want_m) return;
  // S = D^{-T} (H_{j+1,j}^T H_{j+1,j})
  const double* Hsub = d.H + (int64_t)js * ld + (j - 1) * s;
  for (int e = tid; e < ss; e += NT) {
    const int r = e / s, c = e % s;
    double x = 0.0;
    for (int t = 0; t < s; ++t) x = fma(Hsub[(int64_t)t * ld + r], Hsub[(int64_t)t * ld + c], x);
    w0[e] = x;
    Dt[e] = d.Dlast[c * s + r];
  }
  bar();
  lu_solve(Dt, w0, s, s);
  bar();
  double* coefB = d.coef64 + lay.B(0);
  double* wc = w0;
  double* wn = w1;
  for (int i = j - 1; i >= 1; --i) {
    const double* Q = Qs + (i - 1) * 2 * ss;   // Q[t * 2s + r] = (Q_i^T)[s + t][r]
    for (int e = tid; e < 2 * ss; e += NT) {
      const int r = e / s, c = e % s;
      double x = 0.0;
      for (int t = 0; t < s; ++t) x = fma(Q[t * 2 * s + r], wc[t * s + c], x);
      if (r < s) wn[r * s + c] = x;
      else coefB[(int64_t)i * ss + (r - s) * s + c] = x;
    }
    bar();
    double* t = wc;
    wc = wn;
    wn = t;
  }
  for (int e = tid; e < ss; e += NT) coefB[e] = wc[e];
  bar();
}

// The same results for any j s^2 (the register form above needs
// j s^2 <= kCeRegs NT): left-looking block back substitution, block b's
// right-hand side g_b - R_{b, b+1:j} Xi_{b+1:j} accumulated over chunks of
// kCeChunk solved rows staged in LDS (with the matching columns of R's block
// row), then the s x s triangular solve with R_bb in LDS, one thread per
// column.  Xi goes to d.Xi (read back by the later blocks' chunks) and to
// the update coefficients.  M's recurrence stages each Q_i slice in LDS.
constexpr int kCeChunk = 128;
constexpr int kCeOut = (kMaxS * kMaxS + NT - 1) / NT;
__device__ void cycle_end_tiled(const Dense& d, int j, bool want_m, double* lds) {
  const int s = d.s, ld = d.ldh, ss = s * s, js = j * s;
  CoefLayout lay{s, d.mmax + 1};
  const int tid = threadIdx.x;
  double* Xb = lds;                     // ss
  double* Rbb = Xb + ss;                // ss
  double* Rch = Rbb + ss;               // s x kCeChunk
  double* Xch = Rch + s * kCeChunk;     // kCeChunk x s
  double* coefA = d.coef64 + lay.A(0);
  for (int bb = j - 1; bb >= 0; --bb) {
    const int r0 = bb * s;
    const bool last = bb == j - 1;
    double acc[kCeOut];
#pragma unroll
    for (int q = 0; q < kCeOut; ++q) acc[q] = 0.0;
    for (int k0 = r0 + s; k0 < js; k0 += kCeChunk) {
      const int kc = min(kCeChunk, js - k0);
      for (int e = tid; e < s * kc; e += NT) {
        const int r = e / kc, t = e % kc;
        Rch[r * kCeChunk + t] = d.Rf[(int64_t)(r0 + r) * ld + k0 + t];
      }
      for (int e = tid; e < kc * s; e += NT) Xch[e] = d.Xi[(int64_t)k0 * s + e];
      bar();
#pragma unroll
      for (int q = 0; q < kCeOut; ++q) {
        const int e = tid + q * NT;
        if (e < ss) {
          const int r = e / s, c = e % s;
          const double* ra = Rch + r * kCeChunk;
          double a0 = 0.0, a1 = 0.0;
          int t = 0;
          for (; t + 1 < kc; t += 2) {
            a0 = fma(ra[t], Xch[t * s + c], a0);
            a1 = fma(ra[t + 1], Xch[(t + 1) * s + c], a1);
          }
          if (t < kc) a0 = fma(ra[t], Xch[t * s + c], a0);
          acc[q] += a0 + a1;
        }
      }
      bar();
    }
    // right-hand side of the block and its diagonal block of R
#pragma unroll
    for (int q = 0; q < kCeOut; ++q) {
      const int e = tid + q * NT;
      if (e < ss) {
        const double rhs = (last && d.method == LSBA_FOM) ? d.ylast[e]
                                                          : d.g[(int64_t)r0 * s + e];
        Xb[e] = rhs - acc[q];
        Rbb[e] = d.Rf[(int64_t)(r0 + e / s) * ld + r0 + e % s];
      }
    }
    bar();
    // FOM's last block comes with the column's test; every other block
    // solves R_bb x = (its right-hand side)
    if (!(last && d.method == LSBA_FOM) && tid < s) {
      const int c = tid;
      for (int r = s - 1; r >= 0; --r) {
        double v = Xb[r * s + c];
        for (int t = r + 1; t < s; ++t) v = fma(-Rbb[r * s + t], Xb[t * s + c], v);
        Xb[r * s + c] = v / Rbb[r * s + r];
      }
    }
    bar();
    for (int e = tid; e < ss; e += NT) {
      d.Xi[(int64_t)r0 * s + e] = Xb[e];
      coefA[(int64_t)bb * ss + e] = Xb[e];
    }
    bar();
  }
  if (!want_m) return;
  double* w0 = Rch;           // ss
  double* w1 = w0 + ss;       // ss
  double* Dt = w1 + ss;       // ss
  double* Qsl = Dt + ss;      // s x 2s: rows s..2s of Q_i^T
  // S = D^{-T} (H_{j+1,j}^T H_{j+1,j})
  const double* Hsub = d.H + (int64_t)js * ld + (j - 1) * s;
  for (int e = tid; e < ss; e += NT) {
    const int r = e / s, c = e % s;
    double x = 0.0;
    for (int t = 0; t < s; ++t) x = fma(Hsub[(int64_t)t * ld + r], Hsub[(int64_t)t * ld + c], x);
    w0[e] = x;
    Dt[e] = d.Dlast[c * s + r];
  }
  bar();
  lu_solve(Dt, w0, s, s);
  bar();
  double* coefB = d.coef64 + lay.B(0);
  double* wc = w0;
  double* wn = w1;
  for (int i = j - 1; i >= 1; --i) {
    const double* Qg = d.Qt + (int64_t)(i - 1) * 4 * ss + 2 * ss;
    for (int e = tid; e < 2 * ss; e += NT) Qsl[e] = Qg[e];
    bar();
    for (int e = tid; e < 2 * ss; e += NT) {
      const int r = e / s, c = e % s;
      double x = 0.0;
      for (int t = 0; t < s; ++t) x = fma(Qsl[t * 2 * s + r], wc[t * s + c], x);
      if (r < s) wn[r * s + c] = x;
      else coefB[(int64_t)i * ss + (r - s) * s + c] = x;
    }
    bar();
    double* t = wc;
    wc = wn;
    wn = t;
  }
  for (int e = tid; e < ss; e += NT) coefB[e] = wc[e];
  bar();
}

// End of a cycle: Xi, M, the cospatial factor, the basis-application
// coefficients and the adaptive restart bookkeeping.
__global__ __launch_bounds__(NT) void small_cycle_end_kernel(Dense d) {
  __shared__ double lds[LDS_DBL];
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
  // arrival counters of split small steps left behind by an early stop
  for (int i = threadIdx.x; i < kMaxM + 2; i += NT) ctl->arrive[i] = 0;
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
  const bool final_ = (status == ST_CONVERGED || status == ST_ITERCAP);
  const bool want_m = !final_ && d.method == LSBA_GMRES;
  // X += V_{1:j} Xi (C1 = I, A = Xi)
  set_coef_identity(d, lay.C1());
  const double* xlast;
  if (cycle_end_fast(s, j)) {
    cycle_end_regs(d, j, want_m, lds);
    xlast = d.coef64 + lay.A(j - 1);
  } else {
    cycle_end_tiled(d, j, want_m, lds);
    xlast = d.coef64 + lay.A(j - 1);
  }
  int nvb = 0, nve = 0;
  if (!final_) {
    nvb = d.method == LSBA_GMRES ? 0 : j;
    set_coef(d, lay.B(j), d.H + (int64_t)js * ld + c0, ld, -1.0);
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
    copy(s, s, xlast, s, d.C, s);
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

void launch_small_side(hipStream_t st, const Dense& d, int k, int m, KTimer* tm) {
  const int rows = (k == m + 1) ? k - 1 : k;   // the last step only writes the H column
  SMALL_LAUNCH(small_side_kernel<<<rows, NT, 0, st>>>(d, k, m));
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
