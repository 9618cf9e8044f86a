// Sparse block products and FP64 norm reductions.
//
// W = A X with A in CSR and X an n x s row-major block: the block mat-vec of
// every Arnoldi step (Algs. 5-7, "W = A V_k" / "W = A U").  A group of L
// lanes (L = smallest power of two >= s) owns one row; lane c owns column c.
// The row's (col, val) pairs are read by all L lanes at the same address (one
// broadcast per wavefront), and each gather X[col, 0:s] is s contiguous
// elements, so a wavefront reads 64 / L rows' gathers as contiguous segments.
#include "lsba_internal.h"

namespace lsba {

namespace {

inline int lanes_shift(int s) {
  int sh = 0;
  while ((1 << sh) < s) ++sh;
  return sh;
}

template <typename T>
__global__ __launch_bounds__(256) void spmm_kernel(int64_t n, int s, int lshift,
                                                   const int64_t* __restrict__ rp,
                                                   const int* __restrict__ ci,
                                                   const T* __restrict__ val,
                                                   const T* __restrict__ X, T* __restrict__ W,
                                                   const Ctl* __restrict__ ctl) {
  if (ctl && ctl->stop) return;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t row = gid >> lshift;
  const int c = (int)(gid & ((1 << lshift) - 1));
  if (row >= n || c >= s) return;
  const int64_t b = rp[row], e = rp[row + 1];
  T acc = T(0);
  for (int64_t p = b; p < e; ++p) acc += val[p] * X[(int64_t)ci[p] * s + c];
  W[row * s + c] = acc;
}

// Cooperative variant for L >= 8 lanes per row: the L lanes of a row first
// load up to L of the row's (column, value) pairs at once (lane c takes
// entry c of the round), then walk them, receiving each pair by a cross-lane
// shuffle, with the gathers of eight entries in flight before their products
// are added in entry order.  The gather addresses are known one load after
// the row pointer instead of one dependent load per entry.  Workgroups are
// renumbered so that each XCD takes a contiguous range of rows, whose
// neighbours' gathers then hit that XCD's L2.
constexpr int kXcdsSp = 8;

template <typename T, int L>
__global__ __launch_bounds__(256) void spmm_coop_kernel(int64_t n, int s, int64_t nblk,
                                                        int64_t per_xcd,
                                                        const int64_t* __restrict__ rp,
                                                        const int* __restrict__ ci,
                                                        const T* __restrict__ val,
                                                        const T* __restrict__ X,
                                                        T* __restrict__ W,
                                                        const Ctl* __restrict__ ctl) {
  if (ctl && ctl->stop) return;
  constexpr int RPB = 256 / L;   // rows per workgroup
  const int64_t blk = (int64_t)(blockIdx.x % kXcdsSp) * per_xcd + blockIdx.x / kXcdsSp;
  if (blk >= nblk) return;
  const int64_t row = blk * RPB + threadIdx.x / L;
  const int c = threadIdx.x & (L - 1);
  if (row >= n) return;   // whole groups of L lanes leave together
  const int64_t b = rp[row], e = rp[row + 1];
  T acc = T(0);
  const bool col_ok = c < s;
  for (int64_t base = b; base < e; base += L) {
    const int cnt = e - base < L ? (int)(e - base) : L;
    const int my_ci = c < cnt ? ci[base + c] : 0;
    const T my_v = c < cnt ? val[base + c] : T(0);
    for (int j = 0; j < cnt; j += 8) {
      T xv[8], vv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int jj = j + u;
        const int cc = __shfl(my_ci, jj & (L - 1), L);
        vv[u] = __shfl(my_v, jj & (L - 1), L);
        xv[u] = (jj < cnt && col_ok) ? X[(int64_t)cc * s + c] : T(0);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (j + u < cnt) acc += vv[u] * xv[u];
    }
  }
  if (col_ok) W[row * s + c] = acc;
}

// Sum of a value across the workgroup (256 threads), fixed tree order.
__device__ double block_sum_256(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  return r;
}

__global__ __launch_bounds__(256) void residual_kernel(int64_t n, int s, int lshift,
                                                       const int64_t* __restrict__ rp,
                                                       const int* __restrict__ ci,
                                                       const double* __restrict__ val,
                                                       const double* __restrict__ X,
                                                       const double* __restrict__ B,
                                                       double* __restrict__ R,
                                                       double* __restrict__ partial) {
  __shared__ double sh[4];
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t row = gid >> lshift;
  const int c = (int)(gid & ((1 << lshift) - 1));
  double sq = 0.0;
  if (row < n && c < s) {
    const int64_t b = rp[row], e = rp[row + 1];
    double acc = 0.0;
    for (int64_t p = b; p < e; ++p) acc += val[p] * X[(int64_t)ci[p] * s + c];
    const double r = B[row * s + c] - acc;
    if (R) R[row * s + c] = r;
    sq = r * r;
  }
  const double tot = block_sum_256(sq, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void sumsq_partial_kernel(int64_t count,
                                                            const double* __restrict__ x,
                                                            double* __restrict__ partial,
                                                            int64_t per_block) {
  __shared__ double sh[4];
  const int64_t b0 = (int64_t)blockIdx.x * per_block;
  const int64_t b1 = b0 + per_block < count ? b0 + per_block : count;
  double sq = 0.0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += 256) sq += x[i] * x[i];
  const double tot = block_sum_256(sq, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// Per-workgroup sums of (X - Y)^2 over an n x s block (row-major, leading
// dimensions ldx, ldy); each workgroup takes per_block consecutive entries.
__global__ __launch_bounds__(256) void diff_sumsq_partial_kernel(int64_t n, int s,
                                                                 const double* __restrict__ X,
                                                                 int64_t ldx,
                                                                 const double* __restrict__ Y,
                                                                 int64_t ldy,
                                                                 double* __restrict__ partial,
                                                                 int64_t per_block) {
  __shared__ double sh[4];
  const int64_t count = n * s;
  const int64_t b0 = (int64_t)blockIdx.x * per_block;
  const int64_t b1 = b0 + per_block < count ? b0 + per_block : count;
  double sq = 0.0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += 256) {
    const int64_t r = i / s, c = i % s;
    const double d = X[r * ldx + c] - Y[r * ldy + c];
    sq += d * d;
  }
  const double tot = block_sum_256(sq, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void sumsq_final_kernel(const double* __restrict__ partial,
                                                          int nw, double* __restrict__ out) {
  __shared__ double sh[4];
  double v = 0.0;
  for (int i = threadIdx.x; i < nw; i += 256) v += partial[i];
  const double tot = block_sum_256(v, sh);
  if (threadIdx.x == 0) *out = sqrt(tot);
}

template <typename T>
__global__ __launch_bounds__(256) void cast_kernel(int64_t count, const double* __restrict__ in,
                                                   T* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = (T)in[i];
}

template <typename T>
__global__ __launch_bounds__(256) void add_kernel(int64_t count, const T* __restrict__ in,
                                                  double* __restrict__ acc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) acc[i] += (double)in[i];
}

}  // namespace

template <typename T>
void launch_spmm(hipStream_t st, int64_t n, int64_t nnz, int s, const int64_t* rp, const int* ci,
                 const T* val, const T* X, T* W, const Ctl* ctl, KTimer* tm) {
  const int sh = lanes_shift(s);
  const int64_t threads = n << sh;
  const int64_t blocks = (threads + 255) / 256;
  const double bytes =
      (double)nnz * (sizeof(T) + sizeof(int)) + 8.0 * (n + 1) + 2.0 * n * s * sizeof(T);
  if (sh >= 3) {
    const int64_t per_xcd = (blocks + kXcdsSp - 1) / kXcdsSp;
    const dim3 g((unsigned)(per_xcd * kXcdsSp));
    if (sh == 3)
      launch_kf(tm, KK_SPMM, bytes, 2.0 * (double)nnz * s, spmm_coop_kernel<T, 8>, g, dim3(256), 0, st, n, s, blocks,
               per_xcd, rp, ci, val, X, W, ctl);
    else if (sh == 4)
      launch_kf(tm, KK_SPMM, bytes, 2.0 * (double)nnz * s, spmm_coop_kernel<T, 16>, g, dim3(256), 0, st, n, s, blocks,
               per_xcd, rp, ci, val, X, W, ctl);
    else
      launch_kf(tm, KK_SPMM, bytes, 2.0 * (double)nnz * s, spmm_coop_kernel<T, 32>, g, dim3(256), 0, st, n, s, blocks,
               per_xcd, rp, ci, val, X, W, ctl);
    return;
  }
  launch_kf(tm, KK_SPMM, bytes, 2.0 * (double)nnz * s, spmm_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, st, n, s, sh,
           rp, ci, val, X, W, ctl);
}
template void launch_spmm<double>(hipStream_t, int64_t, int64_t, int, const int64_t*, const int*,
                                  const double*, const double*, double*, const Ctl*, KTimer*);
template void launch_spmm<float>(hipStream_t, int64_t, int64_t, int, const int64_t*, const int*,
                                 const float*, const float*, float*, const Ctl*, KTimer*);

void launch_residual(hipStream_t st, int64_t n, int64_t nnz, int s, const int64_t* rp,
                     const int* ci, const double* val, const double* X, const double* B,
                     double* R, double* partial, int* nw_out, KTimer* tm) {
  const int sh = lanes_shift(s);
  const int64_t threads = n << sh;
  const int64_t blocks = (threads + 255) / 256;
  if (tm) tm->begin(st, KK_RESIDUAL);
  residual_kernel<<<dim3((unsigned)blocks), dim3(256), 0, st>>>(n, s, sh, rp, ci, val, X, B, R,
                                                                 partial);
  if (tm)
    tm->end(st, KK_RESIDUAL,
            (double)nnz * 12.0 + 8.0 * (n + 1) + (R ? 3.0 : 2.0) * n * s * sizeof(double));
  *nw_out = (int)blocks;
}

void launch_sumsq_partial(hipStream_t st, int64_t count, const double* x, double* partial,
                          int* nw_out) {
  int64_t per = 256 * 16;
  int64_t blocks = (count + per - 1) / per;
  if (blocks < 1) blocks = 1;
  sumsq_partial_kernel<<<dim3((unsigned)blocks), dim3(256), 0, st>>>(count, x, partial, per);
  *nw_out = (int)blocks;
}

void launch_diff_sumsq_partial(hipStream_t st, int64_t n, int s, const double* X, int64_t ldx,
                               const double* Y, int64_t ldy, double* partial, int* nw_out) {
  const int64_t per = 256 * 16;
  int64_t blocks = (n * s + per - 1) / per;
  if (blocks < 1) blocks = 1;
  diff_sumsq_partial_kernel<<<dim3((unsigned)blocks), dim3(256), 0, st>>>(n, s, X, ldx, Y, ldy,
                                                                         partial, per);
  *nw_out = (int)blocks;
}

void launch_sumsq_final(hipStream_t st, const double* partial, int nw, double* out_norm) {
  sumsq_final_kernel<<<dim3(1), dim3(256), 0, st>>>(partial, nw, out_norm);
}

template <typename T>
void launch_cast(hipStream_t st, int64_t count, const double* in, T* out) {
  const int64_t blocks = (count + 255) / 256;
  cast_kernel<T><<<dim3((unsigned)blocks), dim3(256), 0, st>>>(count, in, out);
}
template void launch_cast<float>(hipStream_t, int64_t, const double*, float*);
template void launch_cast<double>(hipStream_t, int64_t, const double*, double*);

template <typename T>
void launch_add_to_double(hipStream_t st, int64_t count, const T* in, double* acc) {
  const int64_t blocks = (count + 255) / 256;
  add_kernel<T><<<dim3((unsigned)blocks), dim3(256), 0, st>>>(count, in, acc);
}
template void launch_add_to_double<float>(hipStream_t, int64_t, const float*, double*);
template void launch_add_to_double<double>(hipStream_t, int64_t, const double*, double*);

}  // namespace lsba
