// Fused block updates with the basis (the paper's basis_eval / projection):
//
//   out1 = in1 * C1 + sum_{i < nv1} V_i * A_i
//   out2 = in2 * C2 + sum_{nv2_begin <= i < nv2} V_i * B_i + out1 * D
//
// With the coefficients prepared by the small dense step this one pass over
// the basis covers, for example,
//   Alg. 7:  V_k = (U - V_{1:k-1} Y) R^{-1},  U = (W - V_{1:k} [Z; P]) R^{-1}
//   Alg. 6:  V_k = U R^{-1},                  U = W R^{-1} - V_{1:k} H_{1:k,k}
//   Alg. 5:  W - V_{1:k} H_{1:k,k}  and the CholQR scaling X R^{-1}
//   cycle end (Thm. 1):  X += V_{1:j} Xi_j,   U_j = V_{1:j+1} [M; -H_{j+1,j}]
// reading every basis block once and writing at most two blocks.
//
// One thread owns one row: it reads the row of every input block (s
// contiguous elements), keeps both output rows in registers and writes them at
// the end, so in-place updates (out == in) are safe.  The s x s coefficients
// are the same for every thread and are read through the scalar path.
#include "lsba_internal.h"

namespace lsba {

namespace {

template <typename T, int S>
__device__ __forceinline__ void load_row(const T* __restrict__ p, int s, T (&x)[S]) {
#pragma unroll
  for (int t = 0; t < S; ++t) x[t] = (t < s) ? p[t] : T(0);
}

template <typename T, int S>
__device__ __forceinline__ void axpy_mat(const T (&x)[S], const T* __restrict__ C, int s,
                                         T (&o)[S]) {
#pragma unroll
  for (int t = 0; t < S; ++t) {
    if (t < s) {
      const T xv = x[t];
#pragma unroll
      for (int c = 0; c < S; ++c)
        if (c < s) o[c] = fma(xv, C[t * s + c], o[c]);
    }
  }
}

template <typename T, int S, bool EXACT, bool LDSCOEF>
__global__ __launch_bounds__(256) void update_kernel(UpdateArgs<T> a, const Ctl* __restrict__ ctl,
                                                     int obey_stop) {
  if (obey_stop && ctl && ctl->stop) return;
  int nv1 = a.nv1, nb = a.nv2_begin, nv2 = a.nv2;
  if (a.nvp) {
    nv1 = a.nvp[0];
    nb = a.nvp[1];
    nv2 = a.nvp[2];
    if (nv1 < 0) return;
  }
  const int s = EXACT ? S : a.s;
  const T* __restrict__ C = a.coef;
  if constexpr (LDSCOEF) {
    // stage the coefficients used by this launch in LDS once per workgroup;
    // every thread then reads them as broadcasts
    // (same layout as in memory; the A blocks are copied only when used)
    extern __shared__ char smem_raw[];
    T* cl = reinterpret_cast<T*>(smem_raw);
    const int ss = s * s;
    const int a_end = a.lay.A(nv1 > 0 ? nv1 : 0);
    for (int e = threadIdx.x; e < a_end; e += blockDim.x) cl[e] = C[e];
    for (int e = a.lay.C2() + threadIdx.x; e < a.lay.D() + ss; e += blockDim.x) cl[e] = C[e];
    __syncthreads();
    C = cl;
  }
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= a.n) return;
  const int64_t off = row * s;
  const int64_t bstride = a.n * s;
  T o1[S], o2[S], x[S];
#pragma unroll
  for (int c = 0; c < S; ++c) {
    o1[c] = T(0);
    o2[c] = T(0);
  }
  if (a.in1) {
    load_row<T, S>(a.in1 + off, s, x);
    axpy_mat<T, S>(x, C + a.lay.C1(), s, o1);
  }
  const int nvmax = nv1 > nv2 ? nv1 : nv2;
  const int i0 = nv1 > 0 ? 0 : nb;
  for (int i = i0; i < nvmax; ++i) {
    const bool u1 = i < nv1, u2 = (i >= nb) && (i < nv2);
    load_row<T, S>(a.V + (int64_t)i * bstride + off, s, x);
    if (u1) axpy_mat<T, S>(x, C + a.lay.A(i), s, o1);
    if (u2) axpy_mat<T, S>(x, C + a.lay.B(i), s, o2);
  }
  if (a.in2) {
    load_row<T, S>(a.in2 + off, s, x);
    axpy_mat<T, S>(x, C + a.lay.C2(), s, o2);
  }
  if (a.has_D) axpy_mat<T, S>(o1, C + a.lay.D(), s, o2);
  if (a.out1) {
#pragma unroll
    for (int c = 0; c < S; ++c)
      if (c < s) a.out1[off + c] = o1[c];
  }
  if (a.out2 && (a.in2 || nv2 > nb)) {
#pragma unroll
    for (int c = 0; c < S; ++c)
      if (c < s) a.out2[off + c] = o2[c];
  }
}

template <typename T, int S>
void launch_s(hipStream_t st, const UpdateArgs<T>& a, const Ctl* ctl, bool obey) {
  const int64_t blocks = (a.n + 255) / 256;
  // coefficients in LDS for s <= 8 (at most (3 + 2 (m+1)) s^2 elements, 34 KiB
  // for s = 8, m = 30); larger s reads them through the scalar cache
  const size_t coef_bytes = (size_t)a.lay.total() * sizeof(T);
  const bool lds = S <= 8 && coef_bytes <= 64 * 1024;
  if (a.s == S) {
    if (lds)
      update_kernel<T, S, true, true><<<dim3((unsigned)blocks), dim3(256), coef_bytes, st>>>(
          a, ctl, obey ? 1 : 0);
    else
      update_kernel<T, S, true, false><<<dim3((unsigned)blocks), dim3(256), 0, st>>>(
          a, ctl, obey ? 1 : 0);
  } else {
    if (lds)
      update_kernel<T, S, false, true><<<dim3((unsigned)blocks), dim3(256), coef_bytes, st>>>(
          a, ctl, obey ? 1 : 0);
    else
      update_kernel<T, S, false, false><<<dim3((unsigned)blocks), dim3(256), 0, st>>>(
          a, ctl, obey ? 1 : 0);
  }
}

}  // namespace

template <typename T>
double update_bytes(const UpdateArgs<T>& a, int nv1, int nb, int nv2) {
  if (nv1 < 0) return 0.0;
  const int nvmax = nv1 > nv2 ? nv1 : nv2;
  const int i0 = nv1 > 0 ? 0 : nb;
  int blocks = (nvmax > i0 ? nvmax - i0 : 0);
  // inputs (an in-place output reads and writes the same block once each)
  blocks += (a.in1 ? 1 : 0) + (a.in2 && a.in2 != a.in1 ? 1 : 0);
  blocks += (a.out1 ? 1 : 0) + ((a.out2 && (a.in2 || nv2 > nb)) ? 1 : 0);
  return (double)blocks * a.n * a.s * sizeof(T);
}
template double update_bytes<double>(const UpdateArgs<double>&, int, int, int);
template double update_bytes<float>(const UpdateArgs<float>&, int, int, int);

template <typename T>
void launch_update(hipStream_t st, const UpdateArgs<T>& a, const Ctl* ctl, bool obey_stop,
                   KTimer* tm) {
  if (tm) tm->begin(st);
  if (a.s <= 1) launch_s<T, 1>(st, a, ctl, obey_stop);
  else if (a.s <= 2) launch_s<T, 2>(st, a, ctl, obey_stop);
  else if (a.s <= 4) launch_s<T, 4>(st, a, ctl, obey_stop);
  else if (a.s <= 8) launch_s<T, 8>(st, a, ctl, obey_stop);
  else if (a.s <= 16) launch_s<T, 16>(st, a, ctl, obey_stop);
  else launch_s<T, 32>(st, a, ctl, obey_stop);
  if (tm) tm->end(st, KK_UPDATE, a.nvp ? -1.0 : update_bytes(a, a.nv1, a.nv2_begin, a.nv2));
}
template void launch_update<double>(hipStream_t, const UpdateArgs<double>&, const Ctl*, bool,
                                    KTimer*);
template void launch_update<float>(hipStream_t, const UpdateArgs<float>&, const Ctl*, bool,
                                   KTimer*);

}  // namespace lsba
