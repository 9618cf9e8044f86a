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

// The inputs of one launch in order: in1 (if any), the basis blocks
// i0 .. i0 + nbas - 1, in2 (if any).
template <typename T>
struct InputSeq {
  const T* in1;
  const T* in2;
  const T* V;
  int64_t off, bstride;
  int h1, nbas, i0, nv1, nb, nv2;
  __device__ __forceinline__ const T* ptr(int q) const {
    if (q < h1) return in1 + off;
    q -= h1;
    if (q < nbas) return V + (int64_t)(i0 + q) * bstride + off;
    return in2 + off;
  }
};

// Apply input q (its row in x) to the output rows.
template <typename T, int S>
__device__ __forceinline__ void apply_input(const InputSeq<T>& in, int q, const T (&x)[S],
                                            const T* __restrict__ C, const CoefLayout& lay,
                                            int s, T (&o1)[S], T (&o2)[S]) {
  // coefficient blocks for o1 / o2 (null: input does not feed that output)
  const T* c1 = nullptr;
  const T* c2 = nullptr;
  if (q < in.h1) {
    c1 = C + lay.C1();
  } else if (q - in.h1 < in.nbas) {
    const int i = in.i0 + q - in.h1;
    if (i < in.nv1) c1 = C + lay.A(i);
    if (i >= in.nb && i < in.nv2) c2 = C + lay.B(i);
  } else {
    c2 = C + lay.C2();
  }
  if (c1) axpy_mat<T, S>(x, c1, s, o1);
  if (c2) axpy_mat<T, S>(x, c2, s, o2);
}

// Use input q, then start loading input q + NB into the same registers.
template <typename T, int S, int NB>
__device__ __forceinline__ void pipe_step(const InputSeq<T>& in, int nin, int q, T (&x)[S],
                                          const T* __restrict__ C, const CoefLayout& lay,
                                          int s, T (&o1)[S], T (&o2)[S]) {
  if (q < nin) {
    apply_input<T, S>(in, q, x, C, lay, s, o1, o2);
    if (q + NB < nin) load_row<T, S>(in.ptr(q + NB), s, x);
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
  T o1[S], o2[S];
#pragma unroll
  for (int c = 0; c < S; ++c) {
    o1[c] = T(0);
    o2[c] = T(0);
  }
  // The rows of the next NB - 1 inputs are in flight while one is being
  // applied (NB register buffers, named so that every index is static).
  const int nvmax = nv1 > nv2 ? nv1 : nv2;
  InputSeq<T> in;
  in.in1 = a.in1;
  in.in2 = a.in2;
  in.V = a.V;
  in.off = off;
  in.bstride = bstride;
  in.h1 = a.in1 ? 1 : 0;
  in.i0 = nv1 > 0 ? 0 : nb;
  in.nbas = nvmax > in.i0 ? nvmax - in.i0 : 0;
  in.nv1 = nv1;
  in.nb = nb;
  in.nv2 = nv2;
  const int nin = in.h1 + in.nbas + (a.in2 ? 1 : 0);
  constexpr int NB = S <= 8 ? 3 : (S <= 16 ? 2 : 1);
  T x0[S], x1[S], x2[S];
  if (nin > 0) load_row<T, S>(in.ptr(0), s, x0);
  if constexpr (NB > 1)
    if (nin > 1) load_row<T, S>(in.ptr(1), s, x1);
  if constexpr (NB > 2)
    if (nin > 2) load_row<T, S>(in.ptr(2), s, x2);
  for (int q0 = 0; q0 < nin; q0 += NB) {
    pipe_step<T, S, NB>(in, nin, q0, x0, C, a.lay, s, o1, o2);
    if constexpr (NB > 1) pipe_step<T, S, NB>(in, nin, q0 + 1, x1, C, a.lay, s, o1, o2);
    if constexpr (NB > 2) pipe_step<T, S, NB>(in, nin, q0 + 2, x2, C, a.lay, s, o1, o2);
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


// FP64, s = 8, on the matrix cores: [out1 | out2] (16 columns) is one product
// of the inputs (in1, the basis blocks, in2; 8 columns each) with the
// stacked coefficient rows [C1 | C1 D], [A_i | B_i + A_i D], [0 | C2] (the
// folded D term; without D: [C1 | 0], [A_i | B_i], [0 | C2]).  A wavefront
// owns 16 rows: for input q and K-step h, lane l supplies input row
// (row0 + l%16), column 4h + l/16, and coefficient row 4h + l/16, column l%16;
// v_mfma_f64_16x16x4f64 accumulates and lane l ends with rows
// 4r + l/16 (r < 4) of output column l%16.  No LDS: the coefficients are
// read through L1, and four inputs' loads are in flight per lane.
typedef double ud4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ const double* mf_coef(const UpdateArgs<double>& a, const InputSeq<double>& in,
                                                 int q, int lr, bool fold) {
  const CoefLayout& lay = a.lay;
  const double* C = a.coef;
  const bool o2 = lr >= 8;
  if (q < in.h1) return o2 ? (fold ? C + lay.C1D() : nullptr) : C + lay.C1();
  q -= in.h1;
  if (q < in.nbas) {
    const int i = in.i0 + q;
    if (!o2) return i < in.nv1 ? C + lay.A(i) : nullptr;
    if (fold) return C + lay.BF(i);
    return (i >= in.nb && i < in.nv2) ? C + lay.B(i) : nullptr;
  }
  return o2 ? C + lay.C2() : nullptr;
}

template <bool FOLD>
__global__ __launch_bounds__(256) void update_mfma8(UpdateArgs<double> a, const Ctl* __restrict__ ctl,
                                                    int obey_stop) {
  if (obey_stop && ctl && ctl->stop) return;
  int nv1 = a.nv1, nb = a.nv2_begin, nv2 = a.nv2;
  if (a.nvp) {
    nv1 = a.nvp[0];
    nb = a.nvp[1];
    nv2 = a.nvp[2];
    if (nv1 < 0) return;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
  if (row0 >= a.n) return;
  const int lr = lane & 15, lk = lane >> 4;
  const bool rowv = row0 + lr < a.n;
  const int64_t arow = rowv ? row0 + lr : a.n - 1;
  const int nvmax = nv1 > nv2 ? nv1 : nv2;
  InputSeq<double> in;
  in.in1 = a.in1;
  in.in2 = a.in2;
  in.V = a.V;
  in.off = arow * 8;
  in.bstride = a.n * 8;
  in.h1 = a.in1 ? 1 : 0;
  in.i0 = nv1 > 0 ? 0 : nb;
  if (FOLD && nv1 > 0) in.i0 = 0;
  in.nbas = nvmax > in.i0 ? nvmax - in.i0 : 0;
  in.nv1 = nv1;
  in.nb = nb;
  in.nv2 = nv2;
  const int nin = in.h1 + in.nbas + (a.in2 ? 1 : 0);
  const int col = lr & 7;
  ud4 acc = {0.0, 0.0, 0.0, 0.0};
  constexpr int U = 4;
  for (int q0 = 0; q0 < nin; q0 += U) {
    double av[U][2], bv[U][2];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool qv = q0 + u < nin;
      const int q = qv ? q0 + u : nin - 1;
      const double* x = in.ptr(q);
      const double* c = mf_coef(a, in, q, lr, FOLD);
      const bool cv = qv && c != nullptr;
      const double* cc = c ? c : a.coef;
      // padded rows / inputs and absent coefficient blocks contribute exact zeros
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const double xv = x[4 * h + lk];
        const double cvv = cc[(4 * h + lk) * 8 + col];
        av[u][h] = (rowv && qv) ? xv : 0.0;
        bv[u][h] = cv ? cvv : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int h = 0; h < 2; ++h)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][h], bv[u][h], acc, 0, 0, 0);
  }
  const bool w2 = a.out2 && (a.in2 || nv2 > nb);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t row = row0 + 4 * r + lk;
    if (row >= a.n) continue;
    if (lr < 8) {
      if (a.out1) a.out1[row * 8 + col] = acc[r];
    } else if (w2) {
      a.out2[row * 8 + col] = acc[r];
    }
  }
}

template <typename T, int S>
void launch_s(hipStream_t st, const UpdateArgs<T>& a, const Ctl* ctl, bool obey, KTimer* tm,
              double bytes) {
  const int64_t blocks = (a.n + 255) / 256;
  const int ob = obey ? 1 : 0;
  // coefficients in LDS for s <= 8 (at most (3 + 2 (m+1)) s^2 elements, 34 KiB
  // for s = 8, m = 30); larger s reads them through the scalar cache
  if constexpr (sizeof(T) == sizeof(double) && S == 8) {
    if (a.s == 8) {
      const dim3 g((unsigned)((a.n + 63) / 64));
      if (a.has_D)
        launch_k(tm, KK_UPDATE, bytes, update_mfma8<true>, g, dim3(256), 0, st, a, ctl, ob);
      else
        launch_k(tm, KK_UPDATE, bytes, update_mfma8<false>, g, dim3(256), 0, st, a, ctl, ob);
      return;
    }
  }
  // LDS staging covers the coefficients up to D (the folded ones are not read here)
  const size_t coef_bytes = (size_t)(a.lay.D() + a.s * a.s) * sizeof(T);
  const bool lds = S <= 8 && coef_bytes <= 64 * 1024;
  const dim3 g((unsigned)blocks);
  if (a.s == S) {
    if (lds)
      launch_k(tm, KK_UPDATE, bytes, update_kernel<T, S, true, true>, g, dim3(256), coef_bytes,
               st, a, ctl, ob);
    else
      launch_k(tm, KK_UPDATE, bytes, update_kernel<T, S, true, false>, g, dim3(256), 0, st, a,
               ctl, ob);
  } else {
    if (lds)
      launch_k(tm, KK_UPDATE, bytes, update_kernel<T, S, false, true>, g, dim3(256), coef_bytes,
               st, a, ctl, ob);
    else
      launch_k(tm, KK_UPDATE, bytes, update_kernel<T, S, false, false>, g, dim3(256), 0, st, a,
               ctl, ob);
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
  // a launch whose block ranges are read on the device gets its bytes once
  // the host knows them
  const double bytes = a.nvp ? -1.0 : update_bytes(a, a.nv1, a.nv2_begin, a.nv2);
  if (a.s <= 1) launch_s<T, 1>(st, a, ctl, obey_stop, tm, bytes);
  else if (a.s <= 2) launch_s<T, 2>(st, a, ctl, obey_stop, tm, bytes);
  else if (a.s <= 4) launch_s<T, 4>(st, a, ctl, obey_stop, tm, bytes);
  else if (a.s <= 8) launch_s<T, 8>(st, a, ctl, obey_stop, tm, bytes);
  else if (a.s <= 16) launch_s<T, 16>(st, a, ctl, obey_stop, tm, bytes);
  else launch_s<T, 32>(st, a, ctl, obey_stop, tm, bytes);
}
template void launch_update<double>(hipStream_t, const UpdateArgs<double>&, const Ctl*, bool,
                                    KTimer*);
template void launch_update<float>(hipStream_t, const UpdateArgs<float>&, const Ctl*, bool,
                                   KTimer*);

}  // namespace lsba
