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

// FP64, s = 16 or 32, on the matrix cores: [out1 | out2] (2s columns, NT
// tiles of 16) is the product of the input rows [in1 | V_i ... | in2] with
// the stacked coefficient rows, as in update_mfma8.  A workgroup of 8
// wavefronts owns 256 consecutive rows (RG groups of 16 rows per wavefront)
// and walks the inputs in order; for each input the coefficient fragments
// of all its K-steps and output tiles (8 x 4 x 64 doubles for s = 32) are
// staged in LDS once per workgroup, double-buffered, so each wavefront
// reads them conflict-free (lane l reads word l) instead of from L2.  The K
// index of a product may be permuted freely as long as both operands use
// the same order: lane l = (r, q) (row r = l % 16, q = l / 16) loads the
// 16-byte chunks q, q + 4, ... of its row (a wavefront's load covers 16
// rows x 64 contiguous bytes) and K-step h takes column
// c(h, q) = 2q + (h & 1) + 8 (h >> 1) of that row; the coefficient fragment
// of step h holds coefficient row c(h, l / 16).  The next input's rows and
// coefficients are loaded while the current one is multiplied.  Every
// output row depends on its own input rows only, so rows past n read a
// valid row and are not written.  Each 16 x 16 x 4 product is issued as
// four v_mfma_f64_4x4x4f64 with the coefficient fragment rotated across the
// lane groups (Mfma4), twice the FP64 matrix rate of the 16x16x4 form on
// gfx950.  Every global load is unconditional (missing coefficient blocks
// read a valid word and are zeroed when staged), so the compiler's waits on
// them are exact counts and the next input's loads stay in flight through
// the current input's products.
constexpr int kWideRG = 2;

__device__ __forceinline__ int wide_kcol(int h, int q) { return 2 * q + (h & 1) + 8 * (h >> 1); }

template <int S, bool FOLD>
__global__ __launch_bounds__(512) void update_mfma_wide(UpdateArgs<double> a,
                                                        const Ctl* __restrict__ ctl,
                                                        int obey_stop) {
  constexpr int NT = 2 * S / 16;    // output tiles of 16 columns
  constexpr int KS = S / 4;         // K-steps per input block
  constexpr int NCH = S / 8;        // 16-byte chunks per lane and row
  constexpr int RG = kWideRG;
  constexpr int FR = KS * NT * 64;  // doubles of one input's coefficient fragments
  __shared__ double cf[2][FR];
  if (obey_stop && ctl && ctl->stop) return;
  int nv1 = a.nv1, nb = a.nv2_begin, nv2 = a.nv2;
  if (a.nvp) {
    nv1 = a.nvp[0];
    nb = a.nvp[1];
    nv2 = a.nvp[2];
    if (nv1 < 0) return;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  const int64_t wrow0 = (int64_t)blockIdx.x * (8 * RG * 16) + (int64_t)wave * (RG * 16);
  const int nvmax = nv1 > nv2 ? nv1 : nv2;
  InputSeq<double> in;
  in.in1 = a.in1;
  in.in2 = a.in2;
  in.V = a.V;
  in.off = 0;
  in.bstride = a.n * S;
  in.h1 = a.in1 ? 1 : 0;
  in.i0 = nv1 > 0 ? 0 : nb;
  if (FOLD && nv1 > 0) in.i0 = 0;
  in.nbas = nvmax > in.i0 ? nvmax - in.i0 : 0;
  in.nv1 = nv1;
  in.nb = nb;
  in.nv2 = nv2;
  const int nin = in.h1 + in.nbas + (a.in2 ? 1 : 0);
  // this lane's row offsets (rows past n read row n - 1)
  int64_t roff[RG];
#pragma unroll
  for (int g = 0; g < RG; ++g) {
    const int64_t row = wrow0 + 16 * g + lr;
    roff[g] = (row < a.n ? row : a.n - 1) * S + 2 * lq;
  }
  // coefficient fragment entries this thread stages: e = threadIdx.x + 512 u
  constexpr int CPT = (FR + 511) / 512;
  auto coef_load = [&](int q, double (&cv)[CPT], bool (&cok)[CPT]) {
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
      const int e0 = threadIdx.x + 512 * u;
      const int e = e0 < FR ? e0 : FR - 1;
      const int l = e & 63, tq = e >> 6;
      const int t = tq % NT, h = tq / NT;
      const int half = t / (NT / 2);
      const int col = (t % (NT / 2)) * 16 + (l & 15);
      const int krow = wide_kcol(h, l >> 4);
      const double* blk = nullptr;
      if (q < in.h1) {
        blk = half ? (FOLD ? a.coef + a.lay.C1D() : nullptr) : a.coef + a.lay.C1();
      } else if (q - in.h1 < in.nbas) {
        const int i = in.i0 + q - in.h1;
        if (!half) blk = i < nv1 ? a.coef + a.lay.A(i) : nullptr;
        else if (FOLD) blk = a.coef + a.lay.BF(i);
        else blk = (i >= nb && i < nv2) ? a.coef + a.lay.B(i) : nullptr;
      } else {
        blk = half ? a.coef + a.lay.C2() : nullptr;
      }
      cok[u] = blk != nullptr;
      cv[u] = (blk ? blk : a.coef)[krow * S + col];   // a missing block reads a valid word
    }
  };
  auto coef_store = [&](int buf, const double (&cv)[CPT], const bool (&cok)[CPT]) {
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
      const int e = threadIdx.x + 512 * u;
      if (e < FR) cf[buf][e] = cok[u] ? cv[u] : 0.0;
    }
  };
  typedef double dbl2 __attribute__((ext_vector_type(2)));
  auto rows_load = [&](int q, dbl2 (&x)[RG][NCH]) {
    const double* p = in.ptr(q);
#pragma unroll
    for (int g = 0; g < RG; ++g)
#pragma unroll
      for (int j = 0; j < NCH; ++j)
        x[g][j] = *reinterpret_cast<const dbl2*>(p + roff[g] + 8 * j);
  };
  double acc[RG][NT][4];
#pragma unroll
  for (int g = 0; g < RG; ++g)
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[g][t][r] = 0.0;
  dbl2 xc[RG][NCH], xn[RG][NCH];
  double cvn[CPT];
  bool cok[CPT];
  if (nin > 0) {
    coef_load(0, cvn, cok);
    rows_load(0, xc);
    coef_store(0, cvn, cok);
  }
  __syncthreads();
  for (int q = 0; q < nin; ++q) {
    const int buf = q & 1;
    const bool more = q + 1 < nin;
    const int qn = more ? q + 1 : q;   // loads are unconditional (exact waits)
    coef_load(qn, cvn, cok);
    rows_load(qn, xn);
    // the row fragments (RG per K-step) are the rotated operands: fewer
    // than the coefficient fragments (NT per K-step)
#pragma unroll
    for (int h = 0; h < KS; ++h) {
      double bf[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) bf[t] = cf[buf][(h * NT + t) * 64 + lane];
#pragma unroll
      for (int g = 0; g < RG; ++g) {
        const Mfma4 m((h & 1) ? xc[g][h >> 1].y : xc[g][h >> 1].x);
#pragma unroll
        for (int t = 0; t < NT; ++t) m.mac_a(bf[t], acc[g][t]);
      }
    }
    if (more) coef_store(buf ^ 1, cvn, cok);
#pragma unroll
    for (int g = 0; g < RG; ++g)
#pragma unroll
      for (int j = 0; j < NCH; ++j) xc[g][j] = xn[g][j];
    __syncthreads();
  }
  // lane l = 16 i + 4 b + j: acc[g][t][r] = out[row 4 ((b - r) mod 4) + i][tile col 4 b + j]
  const bool w2 = a.out2 && (a.in2 || nv2 > nb);
  const int bq = lr >> 2, jq = lr & 3;
#pragma unroll
  for (int g = 0; g < RG; ++g) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = wrow0 + 16 * g + 4 * ((bq - r) & 3) + lq;
      if (row >= a.n) continue;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int half = t / (NT / 2);
        const int col = (t % (NT / 2)) * 16 + 4 * bq + jq;
        if (!half) {
          if (a.out1) a.out1[row * S + col] = acc[g][t][r];
        } else if (w2) {
          a.out2[row * S + col] = acc[g][t][r];
        }
      }
    }
  }
}

// FP32 blocks, s = 16 or 32, on the BF16 matrix cores with FP32
// accumulation: every FP32 operand x is split into three bf16 parts
// x = h + m + l (h = x rounded to bfloat16, m the rounded remainder, l the
// rounded remainder of that; 24 significant bits in all, like FP32), and
// each product takes the six part products down to 2^-16 relative size
// (l*h, h*l, m*m, m*h, h*m, h*h, smallest first; the dropped ones are below
// 2^-24), so the update keeps FP32 accuracy at the BF16 matrix rate.  Product shape as in update_mfma_wide: [out1 | out2] = the
// input rows times the stacked coefficient rows, one K = s product per
// input block and 16-column output tile (v_mfma_f32_16x16x32_bf16 for
// s = 32, v_mfma_f32_16x16x16bf16_1k for s = 16): lane l holds row l % 16
// and the KPL = s / 4 consecutive input columns KPL (l / 16) .. of it (one
// or two 16-byte loads), the coefficient fragment holds the same rows of
// the coefficient block, and the result rows 4 (l / 16) + r of column l % 16.
// A workgroup of 8 wavefronts owns 256 rows; each input's coefficient
// fragments, already split into the three bf16 parts, are staged in LDS once per
// workgroup, double-buffered; the next input's rows load while the current
// one is multiplied.
typedef short us8 __attribute__((ext_vector_type(8)));
typedef short us4 __attribute__((ext_vector_type(4)));
typedef __bf16 bfv8 __attribute__((ext_vector_type(8)));
typedef __bf16 bfv4 __attribute__((ext_vector_type(4)));
typedef float fv4 __attribute__((ext_vector_type(4)));

// bfloat16 is the upper half of an FP32 word; round to nearest, ties to even.
__device__ __forceinline__ unsigned short bf16_bits(float x) {
  const unsigned int u = __float_as_uint(x);
  return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_value(unsigned short b) {
  return __uint_as_float((unsigned int)b << 16);
}
// x = h + m + l with h, m, l bfloat16 (bit patterns)
__device__ __forceinline__ void bf16_split3(float x, short& h, short& m, short& l) {
  const unsigned short hb = bf16_bits(x);
  const float r1 = x - bf16_value(hb);
  const unsigned short mb = bf16_bits(r1);
  h = (short)hb;
  m = (short)mb;
  l = (short)bf16_bits(r1 - bf16_value(mb));
}

template <int KPL>
__device__ __forceinline__ fv4 mfma_bf16(const short (&a)[KPL], const short (&b)[KPL], fv4 c) {
  if constexpr (KPL == 8) {
    us8 av, bv;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      av[e] = a[e];
      bv[e] = b[e];
    }
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bfv8, av),
                                                   __builtin_bit_cast(bfv8, bv), c, 0, 0, 0);
  } else {
    us4 av, bv;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      av[e] = a[e];
      bv[e] = b[e];
    }
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(bfv4, av),
                                                     __builtin_bit_cast(bfv4, bv), c, 0, 0, 0);
  }
}

template <int S, bool FOLD>
__global__ __launch_bounds__(512) void update_bf16x3(UpdateArgs<float> a,
                                                     const Ctl* __restrict__ ctl, int obey_stop) {
  constexpr int NT = 2 * S / 16;    // output tiles of 16 columns
  constexpr int KPL = S / 4;        // input columns per lane
  constexpr int RG = 2;             // row groups of 16 per wavefront
  constexpr int FR = NT * 64 * KPL; // bf16 values of one part of an input's fragments
  __shared__ short cf[2][3][FR];    // [buffer][h / m / l][tile][lane][KPL]
  if (obey_stop && ctl && ctl->stop) return;
  int nv1 = a.nv1, nb = a.nv2_begin, nv2 = a.nv2;
  if (a.nvp) {
    nv1 = a.nvp[0];
    nb = a.nvp[1];
    nv2 = a.nvp[2];
    if (nv1 < 0) return;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  const int64_t wrow0 = (int64_t)blockIdx.x * (8 * RG * 16) + (int64_t)wave * (RG * 16);
  const int nvmax = nv1 > nv2 ? nv1 : nv2;
  InputSeq<float> in;
  in.in1 = a.in1;
  in.in2 = a.in2;
  in.V = a.V;
  in.off = 0;
  in.bstride = a.n * S;
  in.h1 = a.in1 ? 1 : 0;
  in.i0 = nv1 > 0 ? 0 : nb;
  if (FOLD && nv1 > 0) in.i0 = 0;
  in.nbas = nvmax > in.i0 ? nvmax - in.i0 : 0;
  in.nv1 = nv1;
  in.nb = nb;
  in.nv2 = nv2;
  const int nin = in.h1 + in.nbas + (a.in2 ? 1 : 0);
  int64_t roff[RG];
#pragma unroll
  for (int g = 0; g < RG; ++g) {
    const int64_t row = wrow0 + 16 * g + lr;
    roff[g] = (row < a.n ? row : a.n - 1) * S + KPL * lq;
  }
  // coefficient entries this thread splits and stages: e = threadIdx.x + 512 u
  // over [tile][lane][KPL]
  constexpr int CPT = (FR + 511) / 512;
  auto coef_load = [&](int q, float (&cv)[CPT]) {
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
      const int e = threadIdx.x + 512 * u;
      float v = 0.f;
      if (e < FR) {
        const int t = e / (64 * KPL), rem = e % (64 * KPL);
        const int l = rem / KPL, kk = rem % KPL;
        const int half = t / (NT / 2);
        const int col = (t % (NT / 2)) * 16 + (l & 15);
        const int krow = KPL * (l >> 4) + kk;
        const float* blk = nullptr;
        if (q < in.h1) {
          blk = half ? (FOLD ? a.coef + a.lay.C1D() : nullptr) : a.coef + a.lay.C1();
        } else if (q - in.h1 < in.nbas) {
          const int i = in.i0 + q - in.h1;
          if (!half) blk = i < nv1 ? a.coef + a.lay.A(i) : nullptr;
          else if (FOLD) blk = a.coef + a.lay.BF(i);
          else blk = (i >= nb && i < nv2) ? a.coef + a.lay.B(i) : nullptr;
        } else {
          blk = half ? a.coef + a.lay.C2() : nullptr;
        }
        if (blk) v = blk[krow * S + col];
      }
      cv[u] = v;
    }
  };
  auto coef_store = [&](int buf, const float (&cv)[CPT]) {
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
      const int e = threadIdx.x + 512 * u;
      if (e < FR) {
        short h, m, l;
        bf16_split3(cv[u], h, m, l);
        cf[buf][0][e] = h;
        cf[buf][1][e] = m;
        cf[buf][2][e] = l;
      }
    }
  };
  typedef float flv4 __attribute__((ext_vector_type(4)));
  constexpr int NLD = KPL / 4;   // 16-byte loads per lane and row group
  auto rows_load = [&](int q, flv4 (&x)[RG][NLD]) {
    const float* p = in.ptr(q);
#pragma unroll
    for (int g = 0; g < RG; ++g)
#pragma unroll
      for (int j = 0; j < NLD; ++j) x[g][j] = *reinterpret_cast<const flv4*>(p + roff[g] + 4 * j);
  };
  fv4 acc[RG][NT];
#pragma unroll
  for (int g = 0; g < RG; ++g)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[g][t] = fv4{0.f, 0.f, 0.f, 0.f};
  flv4 xc[RG][NLD], xn[RG][NLD];
  float cvn[CPT];
  if (nin > 0) {
    coef_load(0, cvn);
    rows_load(0, xc);
    coef_store(0, cvn);
  }
  __syncthreads();
  for (int q = 0; q < nin; ++q) {
    const int buf = q & 1;
    const bool more = q + 1 < nin;
    if (more) {
      coef_load(q + 1, cvn);
      rows_load(q + 1, xn);
    }
#pragma unroll
    for (int g = 0; g < RG; ++g) {
      short ah[KPL], am[KPL], al[KPL];
#pragma unroll
      for (int e = 0; e < KPL; ++e) bf16_split3(xc[g][e >> 2][e & 3], ah[e], am[e], al[e]);
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        short bh[KPL], bm[KPL], bl[KPL];
#pragma unroll
        for (int e = 0; e < KPL; ++e) {
          bh[e] = cf[buf][0][(t * 64 + lane) * KPL + e];
          bm[e] = cf[buf][1][(t * 64 + lane) * KPL + e];
          bl[e] = cf[buf][2][(t * 64 + lane) * KPL + e];
        }
        acc[g][t] = mfma_bf16<KPL>(al, bh, acc[g][t]);
        acc[g][t] = mfma_bf16<KPL>(ah, bl, acc[g][t]);
        acc[g][t] = mfma_bf16<KPL>(am, bm, acc[g][t]);
        acc[g][t] = mfma_bf16<KPL>(am, bh, acc[g][t]);
        acc[g][t] = mfma_bf16<KPL>(ah, bm, acc[g][t]);
        acc[g][t] = mfma_bf16<KPL>(ah, bh, acc[g][t]);
      }
    }
    if (more) {
      coef_store(buf ^ 1, cvn);
#pragma unroll
      for (int g = 0; g < RG; ++g)
#pragma unroll
        for (int j = 0; j < NLD; ++j) xc[g][j] = xn[g][j];
    }
    __syncthreads();
  }
  const bool w2 = a.out2 && (a.in2 || nv2 > nb);
#pragma unroll
  for (int g = 0; g < RG; ++g)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = wrow0 + 16 * g + 4 * lq + r;
      if (row >= a.n) continue;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int half = t / (NT / 2);
        const int col = (t % (NT / 2)) * 16 + lr;
        if (!half) {
          if (a.out1) a.out1[row * S + col] = acc[g][t][r];
        } else if (w2) {
          a.out2[row * S + col] = acc[g][t][r];
        }
      }
    }
}

template <typename T, int S>
void launch_s(hipStream_t st, const UpdateArgs<T>& a, const Ctl* ctl, bool obey, KTimer* tm,
              double bytes, double flops) {
  const int64_t blocks = (a.n + 255) / 256;
  const int ob = obey ? 1 : 0;
  // coefficients in LDS for s <= 8 (at most (3 + 2 (m+1)) s^2 elements, 34 KiB
  // for s = 8, m = 30); larger s reads them through the scalar cache
  if constexpr (sizeof(T) == sizeof(double) && S == 8) {
    if (a.s == 8) {
      const dim3 g((unsigned)((a.n + 63) / 64));
      if (a.has_D)
        launch_kf(tm, KK_UPDATE, bytes, flops, update_mfma8<true>, g, dim3(256), 0, st, a, ctl, ob);
      else
        launch_kf(tm, KK_UPDATE, bytes, flops, update_mfma8<false>, g, dim3(256), 0, st, a, ctl, ob);
      return;
    }
  }
  if constexpr (sizeof(T) == sizeof(float) && (S == 16 || S == 32)) {
    if (a.s == S) {
      const dim3 g((unsigned)((a.n + 255) / 256));
      if (a.has_D)
        launch_kf(tm, KK_UPDATE, bytes, flops, update_bf16x3<S, true>, g, dim3(512), 0, st, a, ctl,
                  ob);
      else
        launch_kf(tm, KK_UPDATE, bytes, flops, update_bf16x3<S, false>, g, dim3(512), 0, st, a,
                  ctl, ob);
      return;
    }
  }
  if constexpr (sizeof(T) == sizeof(double) && (S == 16 || S == 32)) {
    if (a.s == S) {
      const dim3 g((unsigned)((a.n + 8 * kWideRG * 16 - 1) / (8 * kWideRG * 16)));
      if (a.has_D)
        launch_kf(tm, KK_UPDATE, bytes, flops, update_mfma_wide<S, true>, g, dim3(512), 0, st, a, ctl, ob);
      else
        launch_kf(tm, KK_UPDATE, bytes, flops, update_mfma_wide<S, false>, g, dim3(512), 0, st, a, ctl,
                 ob);
      return;
    }
  }
  // LDS staging covers the coefficients up to D (the folded ones are not read here)
  const size_t coef_bytes = (size_t)(a.lay.D() + a.s * a.s) * sizeof(T);
  const bool lds = S <= 8 && coef_bytes <= 64 * 1024;
  const dim3 g((unsigned)blocks);
  if (a.s == S) {
    if (lds)
      launch_kf(tm, KK_UPDATE, bytes, flops, update_kernel<T, S, true, true>, g, dim3(256), coef_bytes,
               st, a, ctl, ob);
    else
      launch_kf(tm, KK_UPDATE, bytes, flops, update_kernel<T, S, true, false>, g, dim3(256), 0, st, a,
               ctl, ob);
  } else {
    if (lds)
      launch_kf(tm, KK_UPDATE, bytes, flops, update_kernel<T, S, false, true>, g, dim3(256), coef_bytes,
               st, a, ctl, ob);
    else
      launch_kf(tm, KK_UPDATE, bytes, flops, update_kernel<T, S, false, false>, g, dim3(256), 0, st, a,
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
double update_flops(const UpdateArgs<T>& a, int nv1, int nb, int nv2) {
  if (nv1 < 0) return 0.0;
  const bool w2 = a.out2 && (a.in2 || nv2 > nb);
  int prods = (a.out1 && a.in1 ? 1 : 0) + (a.out1 ? (nv1 > 0 ? nv1 : 0) : 0);
  if (w2) prods += (a.in2 ? 1 : 0) + (nv2 > nb ? nv2 - nb : 0) + (a.has_D ? 1 : 0);
  return 2.0 * (double)prods * a.n * a.s * a.s;
}
template double update_flops<double>(const UpdateArgs<double>&, int, int, int);
template double update_flops<float>(const UpdateArgs<float>&, int, int, int);

template <typename T>
void launch_update(hipStream_t st, const UpdateArgs<T>& a, const Ctl* ctl, bool obey_stop,
                   KTimer* tm) {
  // a launch whose block ranges are read on the device gets its bytes once
  // the host knows them
  const double bytes = a.nvp ? -1.0 : update_bytes(a, a.nv1, a.nv2_begin, a.nv2);
  const double flops = a.nvp ? 0.0 : update_flops(a, a.nv1, a.nv2_begin, a.nv2);
  if (a.s <= 1) launch_s<T, 1>(st, a, ctl, obey_stop, tm, bytes, flops);
  else if (a.s <= 2) launch_s<T, 2>(st, a, ctl, obey_stop, tm, bytes, flops);
  else if (a.s <= 4) launch_s<T, 4>(st, a, ctl, obey_stop, tm, bytes, flops);
  else if (a.s <= 8) launch_s<T, 8>(st, a, ctl, obey_stop, tm, bytes, flops);
  else if (a.s <= 16) launch_s<T, 16>(st, a, ctl, obey_stop, tm, bytes, flops);
  else launch_s<T, 32>(st, a, ctl, obey_stop, tm, bytes, flops);
}
template void launch_update<double>(hipStream_t, const UpdateArgs<double>&, const Ctl*, bool,
                                    KTimer*);
template void launch_update<float>(hipStream_t, const UpdateArgs<float>&, const Ctl*, bool,
                                   KTimer*);

}  // namespace lsba
