// HouseQR IntraOrtho (the unconditionally stable muscle of Sec. 3, used by
// the cycle start of every skeleton and by the IntraOrtho step of Alg. 5) as
// a Householder TSQR: the n x s block is cut into chunks of c rows; each
// workgroup factors its chunk by Householder reflections in LDS (FP64),
// keeps the reflectors in place and stacks its s x s triangle; the stack is
// factored the same way until one chunk is left.  The top chunk's R gets the
// sign fix diag(R) >= 0 (zero entries count as +1), which makes Q and R the
// unique factors of a full-rank block; the breakdown flag is raised for an
// exactly zero or non-finite diagonal entry.  Q is then formed top-down:
// each chunk applies its reflectors to [its s rows of the level above; 0].
//
// Reflector convention (as in the per-column window QR): for column j with
// alpha = x_j and sigma = ||x_{j+1:}||^2, beta = -sign(alpha) sqrt(alpha^2 +
// sigma), v = [1; x_{j+1:} / (alpha - beta)], tau = (beta - alpha) / beta,
// H_j = I - tau v v^T; sigma = 0 gives tau = 0 (H_j = I).
#include "lsba_internal.h"

namespace lsba {

namespace {

constexpr int HT = 256;          // threads per workgroup
constexpr int HCHUNK_DBL = 8192; // doubles of one chunk in LDS (c = HCHUNK_DBL / S2 rows)

template <int S2>
constexpr int chunk_rows() {
  return HCHUNK_DBL / S2 < HT ? HT : HCHUNK_DBL / S2;
}

// Sum each of the V values over the 64 lanes (V a power of two <= 64);
// afterwards lane l holds the total of value l >> (6 - log2 V).
template <int V, int Q>
__device__ __forceinline__ void hb_level(double (&v)[V], int lane) {
  constexpr int h = 32 >> Q;
  constexpr int n = V >> Q;
  if constexpr (n > 1) {
    constexpr int half = n / 2;
    const bool up = (lane & h) != 0;
#pragma unroll
    for (int i = 0; i < half; ++i) {
      const double keep = up ? v[i + half] : v[i];
      const double give = up ? v[i] : v[i + half];
      v[i] = keep + __shfl_xor(give, h, 64);
    }
  } else {
    v[0] += __shfl_xor(v[0], h, 64);
  }
}

// Workgroup sums of V per-thread values, returned in out[0..V) (LDS);
// fixed order, ends with a barrier.
template <int V>
__device__ __forceinline__ void block_reduce(double (&v)[V], double* out) {
  __shared__ double part[HT / 64][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  hb_level<V, 0>(v, lane);
  hb_level<V, 1>(v, lane);
  hb_level<V, 2>(v, lane);
  hb_level<V, 3>(v, lane);
  hb_level<V, 4>(v, lane);
  hb_level<V, 5>(v, lane);
  constexpr int sh = (V == 64) ? 0 : (V == 32) ? 1 : (V == 16) ? 2 : (V == 8) ? 3 : (V == 4) ? 4
                     : (V == 2) ? 5 : 6;
  if ((lane & ((1 << sh) - 1)) == 0) part[wave][lane >> sh] = v[0];
  __syncthreads();
  if (threadIdx.x < V) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < HT / 64; ++w) t += part[w][threadIdx.x];
    out[threadIdx.x] = t;
  }
  __syncthreads();
}

// Householder QR of the c x s chunk X (LDS, ld s, rows >= rows_valid are
// zero): R on and above the diagonal of rows 0..s-1, reflector j below the
// diagonal of column j, tau[j] (LDS).  Thread t owns rows t, t + HT, ...
template <int S2>
__device__ void chunk_factor(double* X, int c, int s, double* tau) {
  __shared__ double red[S2 > 1 ? S2 : 2];
  const int t = threadIdx.x;
  const int rpt = c / HT;
  for (int j = 0; j < s; ++j) {
    double sq[1] = {0.0};
    for (int i = 0; i < rpt; ++i) {
      const int r = t + i * HT;
      if (r > j) sq[0] = fma(X[r * s + j], X[r * s + j], sq[0]);
    }
    block_reduce<1>(sq, red);
    const double sigma = red[0];
    const double alpha = X[j * s + j];
    double tj = 0.0, beta = alpha, scale = 0.0;
    if (sigma != 0.0) {
      beta = -copysign(sqrt(alpha * alpha + sigma), alpha);
      tj = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    __syncthreads();   // every thread has read alpha and sigma
    // v in place below the diagonal; dots w_q = tau v^T X(:, q), q > j
    double acc[S2];
#pragma unroll
    for (int q = 0; q < S2; ++q) acc[q] = 0.0;
    for (int i = 0; i < rpt; ++i) {
      const int r = t + i * HT;
      if (r < j) continue;
      double vr = 1.0;
      if (r > j) {
        vr = X[r * s + j] * scale;
        X[r * s + j] = vr;
      }
#pragma unroll
      for (int q = 0; q < S2; ++q)
        if (q > j && q < s) acc[q] = fma(vr, X[r * s + q], acc[q]);
    }
    block_reduce<S2>(acc, red);
    if (t == 0) {
      tau[j] = tj;
      X[j * s + j] = beta;
    }
    for (int i = 0; i < rpt; ++i) {
      const int r = t + i * HT;
      if (r < j) continue;
      const double vr = r == j ? 1.0 : X[r * s + j];
#pragma unroll
      for (int q = 0; q < S2; ++q)
        if (q > j && q < s) X[r * s + q] = fma(-tj * red[q], vr, X[r * s + q]);
    }
    __syncthreads();
  }
}

// E <- H_0 H_1 ... H_{s-1} E for the reflectors of chunk_factor (Y, tau);
// E is c x s (LDS, ld s).
template <int S2>
__device__ void chunk_apply_q(const double* Y, const double* tau, int c, int s, double* E) {
  __shared__ double red[S2 > 1 ? S2 : 2];
  const int t = threadIdx.x;
  const int rpt = c / HT;
  for (int j = s - 1; j >= 0; --j) {
    const double tj = tau[j];
    double acc[S2];
#pragma unroll
    for (int q = 0; q < S2; ++q) acc[q] = 0.0;
    for (int i = 0; i < rpt; ++i) {
      const int r = t + i * HT;
      if (r < j) continue;
      const double vr = r == j ? 1.0 : Y[r * s + j];
#pragma unroll
      for (int q = 0; q < S2; ++q)
        if (q < s) acc[q] = fma(vr, E[r * s + q], acc[q]);
    }
    block_reduce<S2>(acc, red);
    for (int i = 0; i < rpt; ++i) {
      const int r = t + i * HT;
      if (r < j) continue;
      const double vr = r == j ? 1.0 : Y[r * s + j];
#pragma unroll
      for (int q = 0; q < S2; ++q)
        if (q < s) E[r * s + q] = fma(-tj * red[q], vr, E[r * s + q]);
    }
    __syncthreads();
  }
}

template <typename T>
__device__ __forceinline__ void load_chunk(const T* src, int64_t row0, int64_t nrows, int c, int s,
                                           double* X) {
  for (int e = threadIdx.x; e < c * s; e += HT) {
    const int r = e / s;
    X[e] = (row0 + r < nrows) ? (double)src[(row0 + r) * s + (e % s)] : 0.0;
  }
  __syncthreads();
}

// Level factorization: chunk p of `in` (nrows x s) -> reflectors to `refl`
// (same rows; may alias `in`), tau to tau_out[p s ..], R_p to rows p s .. of
// `stack` (s x s, zero below the diagonal).
template <typename T, int S2>
__global__ __launch_bounds__(HT) void house_level_kernel(const T* in, double* refl, int64_t nrows,
                                                         int s, double* tau_out, double* stack,
                                                         const Ctl* ctl) {
  if (ctl && ctl->stop) return;
  constexpr int c = chunk_rows<S2>();
  __shared__ double X[c * S2];
  __shared__ double tau[S2];
  const int64_t row0 = (int64_t)blockIdx.x * c;
  load_chunk<T>(in, row0, nrows, c, s, X);
  chunk_factor<S2>(X, c, s, tau);
  for (int e = threadIdx.x; e < c * s; e += HT) {
    const int r = e / s;
    if (row0 + r < nrows) refl[(row0 + r) * s + (e % s)] = X[e];
  }
  for (int e = threadIdx.x; e < s * s; e += HT) {
    const int i = e / s, j = e % s;
    stack[((int64_t)blockIdx.x * s + i) * s + j] = (j >= i && i < c) ? X[i * s + j] : 0.0;
  }
  if (threadIdx.x < s) tau_out[(int64_t)blockIdx.x * s + threadIdx.x] = tau[threadIdx.x];
}

// Level Q formation: chunk p applies its reflectors (refl rows, tau) to
// [rows p s .. p s + s of qe_above; 0] and writes the c x s result to out1
// (and out2) rows; out may alias refl.
template <typename T, int S2>
__global__ __launch_bounds__(HT) void house_q_kernel(const double* refl, int64_t nrows, int s,
                                                     const double* tau_in, const double* qe_above,
                                                     T* out1, T* out2, const Ctl* ctl) {
  // out1 may alias refl (levels above 0): the chunk is read into LDS first
  if (ctl && ctl->stop) return;
  constexpr int c = chunk_rows<S2>();
  __shared__ double Y[c * S2];
  __shared__ double E[c * S2];
  __shared__ double tau[S2];
  const int64_t row0 = (int64_t)blockIdx.x * c;
  for (int e = threadIdx.x; e < c * s; e += HT) {
    const int r = e / s;
    Y[e] = (row0 + r < nrows) ? refl[(row0 + r) * s + (e % s)] : 0.0;
    E[e] = r < s ? qe_above[((int64_t)blockIdx.x * s + r) * s + (e % s)] : 0.0;
  }
  if (threadIdx.x < s) tau[threadIdx.x] = tau_in[(int64_t)blockIdx.x * s + threadIdx.x];
  __syncthreads();
  chunk_apply_q<S2>(Y, tau, c, s, E);
  for (int e = threadIdx.x; e < c * s; e += HT) {
    const int r = e / s;
    if (row0 + r < nrows) {
      out1[(row0 + r) * s + (e % s)] = (T)E[e];
      if (out2) out2[(row0 + r) * s + (e % s)] = (T)E[e];
    }
  }
}

// Top chunk (nrows <= c rows of `in`): factor, sign fix, flag, bookkeeping
// for the caller (HM_START: the cycle start, as small_start does for CholQR;
// HM_IO: Alg. 5's IntraOrtho at loop step k), then Q of the top chunk
// (E = [D; 0], D the sign fix) to out1/out2 (T) or, when Q continues down,
// to `qtop` (FP64, rows of the stack).
template <typename T, int S2>
__global__ __launch_bounds__(HT) void house_top_kernel(const T* in, int64_t nrows, int s, Dense d,
                                                       int mode, int k, int force, T* out1,
                                                       T* out2, double* qtop) {
  Ctl* ctl = d.ctl;
  if (mode == HM_IO && ctl->stop) return;
  constexpr int c = chunk_rows<S2>();
  __shared__ double X[c * S2];
  __shared__ double E[c * S2];
  __shared__ double tau[S2];
  __shared__ double sg[S2];
  __shared__ int okf;
  load_chunk<T>(in, 0, nrows, c, s, X);
  chunk_factor<S2>(X, c, s, tau);
  if (threadIdx.x == 0) {
    int ok = 1;
    for (int i = 0; i < s; ++i) {
      const double r = i < c ? X[i * s + i] : 0.0;
      ok &= (r != 0.0 && isfinite(r)) ? 1 : 0;
      sg[i] = r < 0.0 ? -1.0 : 1.0;
    }
    for (int e = 0; e < s * s; ++e) ok &= isfinite(X[e]) ? 1 : 0;
    okf = force ? 0 : ok;
  }
  __syncthreads();
  const int ss = s * s;
  const bool ok = okf != 0;
  if (mode == HM_START) {
    if (skel_uses_t(d.skel))
      for (int64_t e = threadIdx.x; e < (int64_t)d.ldh * d.ldh; e += HT) {
        const double v = ((e / d.ldh) == (e % d.ldh)) ? 1.0 : 0.0;
        d.T[e] = v;
        d.Tt[e] = v;
      }
    if (threadIdx.x == 0) {
      ctl->j = 0;
      ctl->flag_step = ok ? -1 : 0;
      ctl->last_valid = ok ? (1 << 30) : 0;
      ctl->status = ok ? ST_RUNNING : ST_FLAGGED;
      ctl->stop = ok ? 0 : 1;
    }
    if (!ok) return;
    // Beta = D R (rows scaled by the sign fix);  g_1 = Beta C
    for (int e = threadIdx.x; e < ss; e += HT) {
      const int i = e / s, j = e % s;
      d.Beta[e] = j >= i ? sg[i] * X[i * s + j] : 0.0;
    }
    for (int e = threadIdx.x; e < (d.mmax + 1) * ss; e += HT) d.g[e] = 0.0;
    __syncthreads();
    for (int e = threadIdx.x; e < ss; e += HT) {
      const int i = e / s, j = e % s;
      double acc = 0.0;
      for (int t = i; t < s; ++t) acc = fma(sg[i] * X[i * s + t], d.C[t * s + j], acc);
      d.g[e] = acc;
    }
  } else {
    if (!ok) {
      if (threadIdx.x == 0) {
        if (atomicCAS(&ctl->status, (int)ST_RUNNING, (int)ST_FLAGGED) == (int)ST_RUNNING) {
          ctl->flag_step = k;
          ctl->last_valid = k - 1;
        }
        atomicExch(&ctl->stop, 1);
      }
      return;
    }
    // H_{k+1,k} = D R
    for (int e = threadIdx.x; e < ss; e += HT) {
      const int i = e / s, j = e % s;
      d.H[(int64_t)(k * s + i) * d.ldh + (k - 1) * s + j] = j >= i ? sg[i] * X[i * s + j] : 0.0;
    }
  }
  // Q of the top chunk applied to [D; 0]
  for (int e = threadIdx.x; e < c * s; e += HT) {
    const int r = e / s, q = e % s;
    E[e] = (r < s && r == q) ? sg[q] : 0.0;
  }
  __syncthreads();
  chunk_apply_q<S2>(X, tau, c, s, E);
  for (int e = threadIdx.x; e < c * s; e += HT) {
    const int r = e / s;
    if (r < nrows) {
      if (qtop) {
        qtop[e] = E[e];
      } else {
        out1[(int64_t)r * s + (e % s)] = (T)E[e];
        if (out2) out2[(int64_t)r * s + (e % s)] = (T)E[e];
      }
    }
  }
}

int chunk_rows_for(int s) {
  const int s2 = s <= 1 ? 1 : s <= 2 ? 2 : s <= 4 ? 4 : s <= 8 ? 8 : s <= 16 ? 16 : 32;
  const int c = HCHUNK_DBL / s2;
  return c < HT ? HT : c;
}

template <typename T, int S2>
void house_s2(hipStream_t st, const Dense& d, int64_t n, int s, const T* X, T* out1, T* out2,
              double* work, int mode, int k, int force, KTimer* tm) {
  constexpr int c = chunk_rows<S2>();
  const Ctl* ctl = mode == HM_IO ? d.ctl : nullptr;
  // level sizes: rows_0 = n, rows_{l+1} = ceil(rows_l / c) * s
  int64_t rows[24];
  int L = 0;
  rows[0] = n;
  while (rows[L] > c) {
    rows[L + 1] = ((rows[L] + c - 1) / c) * s;
    ++L;
  }
  // work: level-0 reflectors (n x s, FP64), stack_l (rows_l x s) for
  // l = 1..L, tau_l (chunks_l x s) for l = 0..L-1
  double* stack[24];
  double* tau[24];
  double* w = work;
  double* refl0 = w;
  if (L > 0) w += n * s;
  for (int l = 1; l <= L; ++l) {
    stack[l] = w;
    w += rows[l] * s;
  }
  for (int l = 0; l < L; ++l) {
    tau[l] = w;
    w += ((rows[l] + c - 1) / c) * s;
  }
  if (tm) tm->begin(st, KK_SMALL);
  // factor levels 0 .. L-1; level 0 keeps its reflectors in out1
  for (int l = 0; l < L; ++l) {
    const int64_t chunks = (rows[l] + c - 1) / c;
    if (l == 0)
      house_level_kernel<T, S2><<<dim3((unsigned)chunks), dim3(HT), 0, st>>>(
          X, refl0, rows[0], s, tau[0], stack[1], ctl);
    else
      house_level_kernel<double, S2><<<dim3((unsigned)chunks), dim3(HT), 0, st>>>(
          stack[l], stack[l], rows[l], s, tau[l], stack[l + 1], ctl);
  }
  if (L == 0) {
    house_top_kernel<T, S2><<<1, HT, 0, st>>>(X, n, s, d, mode, k, force, out1, out2, nullptr);
  } else {
    house_top_kernel<double, S2><<<1, HT, 0, st>>>(stack[L], rows[L], s, d, mode, k, force,
                                                   (double*)nullptr, (double*)nullptr, stack[L]);
    const Ctl* qctl = d.ctl;   // nothing to form after a flag
    for (int l = L - 1; l >= 1; --l) {
      const int64_t chunks = (rows[l] + c - 1) / c;
      house_q_kernel<double, S2><<<dim3((unsigned)chunks), dim3(HT), 0, st>>>(
          stack[l], rows[l], s, tau[l], stack[l + 1], stack[l], (double*)nullptr, qctl);
    }
    const int64_t chunks0 = (n + c - 1) / c;
    house_q_kernel<T, S2><<<dim3((unsigned)chunks0), dim3(HT), 0, st>>>(
        refl0, n, s, tau[0], stack[1], out1, out2, qctl);
  }
  if (tm) tm->end(st, KK_SMALL, 0.0);
  (void)c;
}

}  // namespace

size_t house_work_doubles(int64_t n, int s) {
  const int c = chunk_rows_for(s);
  int64_t rows = n;
  size_t tot = n > c ? (size_t)n * s : 0;   // level-0 reflectors
  while (rows > c) {
    const int64_t chunks = (rows + c - 1) / c;
    tot += (size_t)chunks * s;          // tau of this level
    rows = chunks * s;
    tot += (size_t)rows * s;            // stack of the next level
  }
  return tot + 64;
}

template <typename T>
void launch_house(hipStream_t st, const Dense& d, int64_t n, int s, const T* X, T* out1, T* out2,
                  double* work, int mode, int k, int force, KTimer* tm) {
  if (s <= 1) house_s2<T, 1>(st, d, n, s, X, out1, out2, work, mode, k, force, tm);
  else if (s <= 2) house_s2<T, 2>(st, d, n, s, X, out1, out2, work, mode, k, force, tm);
  else if (s <= 4) house_s2<T, 4>(st, d, n, s, X, out1, out2, work, mode, k, force, tm);
  else if (s <= 8) house_s2<T, 8>(st, d, n, s, X, out1, out2, work, mode, k, force, tm);
  else if (s <= 16) house_s2<T, 16>(st, d, n, s, X, out1, out2, work, mode, k, force, tm);
  else house_s2<T, 32>(st, d, n, s, X, out1, out2, work, mode, k, force, tm);
}
template void launch_house<double>(hipStream_t, const Dense&, int64_t, int, const double*,
                                   double*, double*, double*, int, int, int, KTimer*);
template void launch_house<float>(hipStream_t, const Dense&, int64_t, int, const float*, float*,
                                  float*, double*, int, int, int, KTimer*);

}  // namespace lsba
