// Tall-skinny Gram products G = [L_1 ... L_p]^T [R_1 ... R_q] of n x s blocks:
// the block inner products (the sync points) of the skeletons, e.g. the fused
// [V_{1:k-1} U]^T [U W] of Algs. 6 and 7, V_{1:k}^T W and V_{1:k}^T V_{k+1}
// of Alg. 5, and the Gram X^T X of the CholQR muscle.
//
// Split-n, two stages, deterministic: stage 1 gives each workgroup a chunk of
// rows and writes the chunk's partial G to a workspace; stage 2 sums the
// partials in chunk order.  No floating-point atomics, so every run (and
// every request of a serving batch) reduces in the same order.
//
// Stage 1 (vector FMA): the output (p s) x (q s) is cut into TxT tiles,
// T = min(s, 8); one wavefront owns one tile for one chunk.  Lane l takes the
// chunk's rows l, l+64, ...: for each it loads T contiguous elements of the
// left block row and T of the right block row (consecutive lanes read
// consecutive rows, so a wavefront's loads are contiguous segments) and
// accumulates the T x T outer product in registers.  The 64 lanes are then
// combined by a butterfly of cross-lane shuffles that leaves one finished
// entry per lane.  Workgroups are numbered so that all tiles of one chunk run
// on the same XCD, where their shared block rows are served by that XCD's L2.
#include "lsba_internal.h"

namespace lsba {

namespace {

constexpr int kXcds = 8;

template <typename T>
__device__ __forceinline__ const T* left_ptr(const GramArgs<T>& a, int blk) {
  return blk < a.nv ? a.V + (int64_t)blk * a.n * a.s : a.xl[blk - a.nv];
}

template <int V, int Q>
__device__ __forceinline__ void butterfly_level(double (&v)[V], int lane) {
  constexpr int h = 32 >> Q;      // partner distance
  constexpr int n = V >> Q;       // values still distinct at this level
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

// Sum each of the V values over the 64 lanes of the wavefront (V a power of
// two <= 64); afterwards lane l holds the total of value l >> (6 - log2 V).
// The order of the additions is fixed.
template <int V>
__device__ __forceinline__ double butterfly(double (&v)[V], int lane) {
  butterfly_level<V, 0>(v, lane);
  butterfly_level<V, 1>(v, lane);
  butterfly_level<V, 2>(v, lane);
  butterfly_level<V, 3>(v, lane);
  butterfly_level<V, 4>(v, lane);
  butterfly_level<V, 5>(v, lane);
  return v[0];
}

template <typename T, int TL>
__global__ __launch_bounds__(256) void gram_stage1(GramArgs<T> a, int nchunk, int ngroup,
                                                   int64_t rows_per_chunk,
                                                   double* __restrict__ partial,
                                                   const Ctl* __restrict__ ctl) {
  if (ctl && ctl->stop) return;
  // XCD-aware numbering: hardware workgroup id -> (chunk, tile group)
  const int pid = blockIdx.x;
  const int xcd = pid % kXcds, t = pid / kXcds;
  const int chunk = xcd + kXcds * (t / ngroup);
  const int grp = t % ngroup;
  if (chunk >= nchunk) return;
  const int s = a.s;
  const int PA = (a.nv + a.nxl) * s, QB = a.nxr * s;
  const int tcols = QB / TL;                  // tiles across the right blocks
  const int ntile = (PA / TL) * tcols;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tile = grp * 4 + wave;
  if (tile >= ntile) return;
  const int ta = tile / tcols, tb = tile % tcols;
  const int acol = ta * TL, bcol = tb * TL;   // first output row / column
  const T* __restrict__ L = left_ptr(a, acol / s) + (acol % s);
  const T* __restrict__ Rr = a.xr[bcol / s] + (bcol % s);
  const int64_t r0 = (int64_t)chunk * rows_per_chunk;
  const int64_t r1 = r0 + rows_per_chunk < a.n ? r0 + rows_per_chunk : a.n;
  T acc[TL][TL];
#pragma unroll
  for (int i = 0; i < TL; ++i)
#pragma unroll
    for (int j = 0; j < TL; ++j) acc[i][j] = T(0);
  // rows r0 + lane + 64 q; the rows of the next NB - 1 iterations are in
  // flight while one is multiplied (NB register buffers indexed at compile time)
  constexpr int NB = TL >= 8 ? 2 : 3;
  const int64_t nq = r1 > r0 + lane ? (r1 - (r0 + lane) + 63) / 64 : 0;
  T lv[NB][TL], rv[NB][TL];
  auto load = [&](int64_t q, int b) {
    const int64_t off = (r0 + lane + 64 * q) * s;
#pragma unroll
    for (int i = 0; i < TL; ++i) lv[b][i] = L[off + i];
#pragma unroll
    for (int j = 0; j < TL; ++j) rv[b][j] = Rr[off + j];
  };
#pragma unroll
  for (int b = 0; b < NB; ++b)
    if (b < nq) load(b, b);
  for (int64_t q0 = 0; q0 < nq; q0 += NB) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int64_t q = q0 + b;
      if (q < nq) {
#pragma unroll
        for (int i = 0; i < TL; ++i)
#pragma unroll
          for (int j = 0; j < TL; ++j) acc[i][j] = fma(lv[b][i], rv[b][j], acc[i][j]);
        if (q + NB < nq) load(q + NB, b);
      }
    }
  }
  constexpr int V = TL * TL;
  double v[V];
#pragma unroll
  for (int i = 0; i < TL; ++i)
#pragma unroll
    for (int j = 0; j < TL; ++j) v[i * TL + j] = (double)acc[i][j];
  const double tot = butterfly<V>(v, lane);
  constexpr int sh = (V == 64) ? 0 : (V == 16) ? 2 : (V == 4) ? 4 : 6;
  if ((lane & ((1 << sh) - 1)) == 0) {
    const int e = lane >> sh;
    const int i = e / TL, j = e % TL;
    partial[(int64_t)chunk * PA * QB + (int64_t)(acol + i) * QB + (bcol + j)] = tot;
  }
}

// Stage 2: G[e] = sum over chunks of partial[chunk][e].  A workgroup takes
// 2^ew_log2 consecutive entries and 256 >> ew_log2 groups of threads; group q
// sums chunks q, q + groups, ... (several loads in flight), and the groups'
// sums are added in group order, so the result does not depend on timing.
__global__ __launch_bounds__(256) void gram_stage2(const double* __restrict__ partial, int nchunk,
                                                   int entries, int ew_log2,
                                                   double* __restrict__ out,
                                                   const Ctl* __restrict__ ctl) {
  if (ctl && ctl->stop) return;
  __shared__ double red[256];
  const int ew = 1 << ew_log2, groups = 256 >> ew_log2;
  const int le = threadIdx.x & (ew - 1), q = threadIdx.x >> ew_log2;
  const int e = blockIdx.x * ew + le;
  double v = 0.0;
  if (e < entries) {
    const double* p = partial + e;
    int c = q;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (; c + 3 * groups < nchunk; c += 4 * groups) {
      a0 += p[(int64_t)c * entries];
      a1 += p[(int64_t)(c + groups) * entries];
      a2 += p[(int64_t)(c + 2 * groups) * entries];
      a3 += p[(int64_t)(c + 3 * groups) * entries];
    }
    for (; c < nchunk; c += groups) a0 += p[(int64_t)c * entries];
    v = (a0 + a1) + (a2 + a3);
  }
  red[threadIdx.x] = v;
  __syncthreads();
  if (q == 0 && e < entries) {
    double t = 0.0;
    for (int g = 0; g < groups; ++g) t += red[g * ew + le];
    out[e] = t;
  }
}


// FP64 matrix-core variant (s >= 8): a wavefront owns a 16 x 16 output tile
// (16 consecutive left columns and 16 consecutive right columns, which may
// span several blocks: each lane addresses its own column) for a chunk of rows and feeds v_mfma_f64_16x16x4f64 four rows at a time:
// lane l supplies left[row + l/16][i0 + l%16] and right[row + l/16][j0 + l%16]
// (a wavefront's loads are four 128-byte row segments per operand) and holds
// D[4 q + l/16][l%16], q < 4, of the tile.  The matrix core accumulates
// over the rows, so no cross-lane reduction is needed, and a row element is
// re-read from L2 only by the few tiles that share its block.  Eight row
// groups of loads are in flight per lane.
typedef double gd4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void gram_mfma_f64(GramArgs<double> a, int nchunk, int ngroup,
                                                     int64_t rows_per_chunk,
                                                     double* __restrict__ partial,
                                                     const Ctl* __restrict__ ctl) {
  if (ctl && ctl->stop) return;
  const int pid = blockIdx.x;
  const int xcd = pid % kXcds, t = pid / kXcds;
  const int chunk = xcd + kXcds * (t / ngroup);
  const int grp = t % ngroup;
  if (chunk >= nchunk) return;
  const int s = a.s;
  const int PA = (a.nv + a.nxl) * s, QB = a.nxr * s;
  const int tcols = (QB + 15) / 16;
  const int ntile = ((PA + 15) / 16) * tcols;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tile = grp * 4 + wave;
  if (tile >= ntile) return;
  const int i0 = (tile / tcols) * 16, j0 = (tile % tcols) * 16;
  const int lr = lane & 15, lk = lane >> 4;
  // this lane's left and right columns (zero weight past PA / QB)
  const int ci = i0 + lr, cj = j0 + lr;
  const double wl = ci < PA ? 1.0 : 0.0, wr = cj < QB ? 1.0 : 0.0;
  const int cic = ci < PA ? ci : PA - 1, cjc = cj < QB ? cj : QB - 1;
  const double* __restrict__ L = left_ptr(a, cic / s) + (cic % s);
  const double* __restrict__ R = a.xr[cjc / s] + (cjc % s);
  const int64_t r0 = (int64_t)chunk * rows_per_chunk;
  const int64_t r1 = r0 + rows_per_chunk < a.n ? r0 + rows_per_chunk : a.n;
  gd4 acc = {0.0, 0.0, 0.0, 0.0};
  constexpr int U = 8;   // row groups of 4 in flight
  for (int64_t rb = r0; rb < r1; rb += 4 * U) {
    double av[U], bv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t row = rb + 4 * u + lk;
      const int64_t rr = row < r1 ? row : r1 - 1;   // in-bounds address, zero weight past r1
      av[u] = L[rr * s];
      bv[u] = R[rr * s];
      av[u] = row < r1 ? av[u] * wl : 0.0;
      bv[u] = bv[u] * wr;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
  }
  double* out = partial + (int64_t)chunk * PA * QB;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = i0 + 4 * q + lk;
    if (i < PA && cj < QB) out[(int64_t)i * QB + cj] = acc[q];
  }
}

// FP64 matrix-core Gram for block sizes that are multiples of 16 (s = 16,
// 32): a wavefront owns up to SW (4, 5 or 6) left strips of 16 columns against
// all NTR right tiles of 16 columns (v_mfma_f64_16x16x4f64 tiles, 4 SW NTR
// accumulator doubles per lane) for a chunk of rows; the waves of a
// workgroup share the chunk and differ in their strips.  Each wave loads its
// left fragments itself (one double per lane and strip per group of four
// rows: four rows x 128 contiguous bytes), four groups of rows ahead.  The
// right rows, which every wave needs, are staged once per workgroup in LDS,
// sixteen rows at a time (16-byte loads of whole rows, the next stage in
// flight in registers, two LDS buffers; row stride padded by 128 bytes so
// the four rows of a fragment fall in distinct bank halves), and each wave
// reads its right fragments from there.  So a group of rows costs about one
// global load instruction per strip, and each right row is fetched from
// HBM once per chunk.  Partials go to partial[chunk] in the layout of the
// other stage-1 kernels.  (Measured on MI355X: the 4x4x4 FP64 instruction
// issues at twice this one's rate, but a 4x4x4 form of this kernel, and one
// staging every block in LDS, ran no faster: at these shapes the kernel is
// bound by its memory access, not by the matrix cores.)
constexpr int kWTR = 16;              // rows per right-operand stage
constexpr int kWQB = 64;              // largest right width (two blocks of 32)
constexpr int kWLD = kWQB + 16;       // LDS row stride of a stage (doubles)

template <typename T, int SW, int NTR, int RPT>
__global__ __launch_bounds__(512) void gram_mfma_wide(GramArgs<T> a, int nchunk, int ngroup,
                                                      int wpg, int64_t rows_per_chunk,
                                                      double* __restrict__ partial,
                                                      const Ctl* __restrict__ ctl) {
  __shared__ double rs[2][kWTR * kWLD];
  if (ctl && ctl->stop) return;
  const int pid = blockIdx.x;
  const int xcd = pid % kXcds, t = pid / kXcds;
  const int chunk = xcd + kXcds * (t / ngroup);
  const int grp = t % ngroup;
  if (chunk >= nchunk) return;
  const int s = a.s;
  const int PA = (a.nv + a.nxl) * s, QB = a.nxr * s;
  const int NS = PA >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  // the chunk's ngroup * wpg wavefronts split the NS strips as evenly as
  // possible (counts differ by at most one, the larger counts first)
  const int nw = ngroup * wpg, w = grp * wpg + wave;
  const int base = NS / nw, extra = NS % nw;
  const int st0 = w * base + (w < extra ? w : extra);
  const int nsw = base + (w < extra ? 1 : 0);
  const int lr = lane & 15, lk = lane >> 4;
  // strip base pointers are the same for every lane (a strip never
  // straddles two blocks); the lane's column adds lr
  const T* Lp[SW];
#pragma unroll
  for (int i = 0; i < SW; ++i) {
    const int col = (st0 + (i < nsw ? i : (nsw > 0 ? nsw - 1 : 0))) * 16;
    Lp[i] = left_ptr(a, (col < PA ? col : 0) / s) + (col % s) + lr;
  }
  const int64_t r0 = (int64_t)chunk * rows_per_chunk;
  const int64_t r1 = r0 + rows_per_chunk < a.n ? r0 + rows_per_chunk : a.n;
  const int nst = (int)((r1 - r0 + kWTR - 1) / kWTR);
  // right-stage staging: 16-byte chunk e = threadIdx.x + blockDim.x u of the
  // stage is (row e / cpr, chunk e % cpr); RPT >= chunks per thread.  FP32
  // blocks are widened to FP64 when written to LDS.
  constexpr int EPC = 16 / (int)sizeof(T);      // elements per 16-byte chunk
  const int cpr = QB / EPC;                     // chunks per right row
  const int nchk = kWTR * cpr;
  typedef T wv __attribute__((ext_vector_type(EPC)));
  wv rreg[RPT];
  // Every thread issues the same loads at every stage, none of them under a
  // branch (chunks past the stage and rows past r1 read a valid element; the
  // rows are zeroed only when stored), so the compiler's waits on them are
  // exact counts and the loads of the stage after next stay in flight
  // through this stage.
  auto rload = [&](int st) {
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const int e0 = threadIdx.x + blockDim.x * u;
      const int e = e0 < nchk ? e0 : nchk - 1;
      const int row = e / cpr, col = EPC * (e % cpr);
      const int64_t grow = r0 + (int64_t)st * kWTR + row;
      rreg[u] = *reinterpret_cast<const wv*>(a.xr[col / s] + (col % s) +
                                             (grow < r1 ? grow : r1 - 1) * s);
    }
  };
  auto rstore = [&](int buf, int st) {
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const int e = threadIdx.x + blockDim.x * u;
      if (e < nchk) {
        const bool ok = r0 + (int64_t)st * kWTR + e / cpr < r1;   // rows past r1 contribute 0
        double* dst = &rs[buf][(e / cpr) * kWLD + EPC * (e % cpr)];
#pragma unroll
        for (int q = 0; q < EPC; ++q) dst[q] = ok ? (double)rreg[u][q] : 0.0;
      }
    }
  };
  // left fragments of the four row groups of a stage (slot kq)
  double av[4][SW];
  auto lload = [&](int st, int kq) {
    const int64_t row = r0 + (int64_t)st * kWTR + 4 * kq + lk;
    const int64_t off = (row < r1 ? row : r1 - 1) * s;
#pragma unroll
    for (int i = 0; i < SW; ++i) av[kq][i] = (double)Lp[i][off];   // (Lp[i >= nsw]: a valid strip)
  };
  // each 16 x 16 x 4 product as four 4x4x4 products (Mfma4)
  double acc[SW][NTR][4];
#pragma unroll
  for (int i = 0; i < SW; ++i)
#pragma unroll
    for (int j = 0; j < NTR; ++j)
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[i][j][t] = 0.0;
  if (nst > 0) {
    rload(0);
    rstore(0, 0);
    if (nst > 1) rload(1);
#pragma unroll
    for (int kq = 0; kq < 4; ++kq) lload(0, kq);
  }
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const double* R = rs[st & 1];
    const bool more = st + 1 < nst;
#pragma unroll
    for (int kq = 0; kq < 4; ++kq) {
#pragma unroll
      for (int j = 0; j < NTR; ++j) {
        const Mfma4 m(R[(4 * kq + lk) * kWLD + 16 * j + lr]);
#pragma unroll
        for (int i = 0; i < SW; ++i)
          if (i < nsw) m.mac(av[kq][i], acc[i][j]);
      }
      lload(more ? st + 1 : st, kq);   // unconditional: its waits stay exact
    }
    if (more) rstore((st + 1) & 1, st + 1);
    rload(st + 2 < nst ? st + 2 : nst - 1);
    __syncthreads();
  }
  // lane l = 16 i + 4 g + j: acc[.][.][t] = G[4 g + i][4 ((g - t) mod 4) + j]
  double* out = partial + (int64_t)chunk * PA * QB;
  const int g = lr >> 2, jj = lr & 3;
#pragma unroll
  for (int i = 0; i < SW; ++i)
    if (i < nsw)
#pragma unroll
      for (int j = 0; j < NTR; ++j)
#pragma unroll
        for (int t = 0; t < 4; ++t)
          out[(int64_t)((st0 + i) * 16 + 4 * g + lk) * QB + j * 16 + 4 * ((g - t) & 3) + jj] =
              acc[i][j][t];
}

// FP32 Gram for s = 16, 32 on the BF16 matrix cores with FP32 accumulation
// (the precision form's inner solves).  Each FP32 value x is split into
// three bfloat16 parts x = h + m + l (each the round-to-nearest of what is
// left; 24 significant bits, like FP32) and each product takes the six part
// products down to 2^-16 relative size (l*h, h*l, m*m, m*h, h*m, h*h; the
// dropped ones are below 2^-24), so the Gram keeps FP32 accuracy at the
// BF16 matrix rate.  The contraction runs over rows and
// v_mfma_f32_16x16x32_bf16 wants each lane to hold eight consecutive K
// values: lane l takes column l % 16 of a 16-column strip (A) or tile (B)
// at rows 8 (l / 16) .. 8 (l / 16) + 7.  Row-major blocks do not store
// those together, so a workgroup stages a tile of 32 rows of its left
// blocks and of the right blocks in LDS, split into the three bf16 planes
// and stored column-major: column c of a block keeps its 32 rows in four
// 8-row groups, group g at slot g ^ ((c / 4) mod 4), which puts the
// 16-byte reads of the 16 lanes of a row group in 16 distinct bank
// quarters.  Each thread loads two rows of four columns (two 16-byte
// loads, consecutive threads on consecutive columns), converts each
// column's pair of rows to one packed bf16 word per plane and writes it;
// the tile after next is in flight in registers meanwhile, and LDS is
// double-buffered, one barrier per tile.  Wavefronts split the workgroup's
// 16-column strips (at most 3 each) and take every right tile; partials
// (FP32 per chunk, summed in FP64 across chunks) go to partial[chunk] as
// for the other stage-1 kernels.
constexpr int kBTR = 32;             // rows per staged tile
constexpr int kBMaxBlk = 10;         // s = 32 blocks (left + right) staged per workgroup
constexpr int kBSW = 3;              // strips per wavefront at most
constexpr int kBPlaneShorts = kBMaxBlk * 32 * kBTR;   // one plane of one buffer

typedef short bs8 __attribute__((ext_vector_type(8)));
typedef __bf16 bb8 __attribute__((ext_vector_type(8)));
typedef __bf16 bb2 __attribute__((ext_vector_type(2)));
typedef float bf4acc __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf4acc bmfma(bs8 a, bs8 b, bf4acc c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bb8, a),
                                                 __builtin_bit_cast(bb8, b), c, 0, 0, 0);
}

// Two FP32 values (consecutive rows of one column) to three packed bf16
// words, parts h, m, l in that order; the conversions round to nearest even.
__device__ __forceinline__ void bsplit3_pair(float x0, float x1, unsigned& h, unsigned& m,
                                             unsigned& l) {
  bb2 p;
  p[0] = (__bf16)x0;
  p[1] = (__bf16)x1;
  h = __builtin_bit_cast(unsigned, p);
  const float r0 = x0 - __uint_as_float(h << 16), r1 = x1 - __uint_as_float(h & 0xFFFF0000u);
  p[0] = (__bf16)r0;
  p[1] = (__bf16)r1;
  m = __builtin_bit_cast(unsigned, p);
  p[0] = (__bf16)(r0 - __uint_as_float(m << 16));
  p[1] = (__bf16)(r1 - __uint_as_float(m & 0xFFFF0000u));
  l = __builtin_bit_cast(unsigned, p);
}

// short offset of (column c, row r) inside a block's plane slice
__device__ __forceinline__ int bswz(int c, int r) {
  return c * kBTR + 8 * ((r >> 3) ^ ((c >> 2) & 3)) + (r & 7);
}

template <int NTR>
__global__ __launch_bounds__(512) void gram_bf16(GramArgs<float> a, int nchunk, int ngroup,
                                                 int nlb_max, int64_t rows_per_chunk,
                                                 double* __restrict__ partial,
                                                 const Ctl* __restrict__ ctl) {
  constexpr int TR = kBTR;
  __shared__ __align__(16) short lds[2][3][kBPlaneShorts];
  if (ctl && ctl->stop) return;
  const int pid = blockIdx.x;
  const int xcd = pid % kXcds, t = pid / kXcds;
  const int chunk = xcd + kXcds * (t / ngroup);
  const int grp = t % ngroup;
  if (chunk >= nchunk) return;
  const int s = a.s;
  const int NBL = a.nv + a.nxl;
  const int PA = NBL * s, QB = a.nxr * s;
  const int lb0 = grp * nlb_max;
  const int nlb = NBL - lb0 < nlb_max ? NBL - lb0 : nlb_max;
  if (nlb <= 0) return;
  const int nbs = nlb + a.nxr;                 // blocks staged
  const int bsz = s * TR;                      // shorts per block in one plane
  const int spb = s >> 4;                      // strips per block
  const int NS = nlb * spb;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int base = NS / 8, extra = NS % 8;
  const int st0 = wave * base + (wave < extra ? wave : extra);
  const int nsw = base + (wave < extra ? 1 : 0);
  const int lc = lane & 15, lk = lane >> 4;
  const int64_t r0 = (int64_t)chunk * rows_per_chunk;
  const int64_t r1 = r0 + rows_per_chunk < a.n ? r0 + rows_per_chunk : a.n;
  const int nst = (int)((r1 - r0 + TR - 1) / TR);
  // staging unit e = (block, row pair, 4-column group); a thread's units
  // and their addresses are fixed for the whole chunk
  const int cpr = s >> 2;
  const int upb = (TR / 2) * cpr;
  const int nunit = nbs * upb;
  constexpr int UPT = (kBMaxBlk * 32 * TR / 8 + 511) / 512;
  typedef float fq4 __attribute__((ext_vector_type(4)));
  const float* gb[UPT];     // row r0 of the unit's block, its first column
  int rp2[UPT], lw[UPT];    // first row of the pair; LDS word of its first column
#pragma unroll
  for (int u = 0; u < UPT; ++u) {
    const int e = threadIdx.x + 512 * u;
    const int blk = e < nunit ? e / upb : 0, rem = e % upb;
    const int rp = e < nunit ? rem / cpr : 0, c4 = e < nunit ? rem % cpr : 0;
    const float* bp = blk < nlb ? left_ptr(a, lb0 + blk) : a.xr[blk - nlb];
    gb[u] = bp + r0 * s + 4 * c4;
    rp2[u] = 2 * rp;
    lw[u] = e < nunit ? (blk * bsz + bswz(4 * c4, 2 * rp)) >> 1 : -1;
  }
  // every thread issues the same loads for every tile (inactive units and
  // rows past the chunk read a valid row), so the waits on them are static;
  // the rows past the chunk are zeroed only when the tile is stored
  auto gload = [&](fq4 (&ra)[UPT], fq4 (&rb)[UPT], int st) {
    const int lim = (int)(r1 - r0) - st * TR;          // rows of this tile in the chunk
#pragma unroll
    for (int u = 0; u < UPT; ++u) {
      const float* p0 = gb[u] + (int64_t)(rp2[u] < lim ? st * TR + rp2[u] : 0) * s;
      const float* p1 = gb[u] + (int64_t)(rp2[u] + 1 < lim ? st * TR + rp2[u] + 1 : 0) * s;
      ra[u] = *reinterpret_cast<const fq4*>(p0);
      rb[u] = *reinterpret_cast<const fq4*>(p1);
    }
  };
  auto lstore = [&](int buf, const fq4 (&ra)[UPT], const fq4 (&rb)[UPT], int st) {
    unsigned* H = reinterpret_cast<unsigned*>(&lds[buf][0][0]);
    unsigned* M = reinterpret_cast<unsigned*>(&lds[buf][1][0]);
    unsigned* L = reinterpret_cast<unsigned*>(&lds[buf][2][0]);
    const int lim = (int)(r1 - r0) - st * TR;
#pragma unroll
    for (int u = 0; u < UPT; ++u)
      if (lw[u] >= 0) {
        const bool ok0 = rp2[u] < lim, ok1 = rp2[u] + 1 < lim;   // rows past r1 contribute 0
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int w = lw[u] + (kBTR / 2) * q;
          unsigned h, m, l;
          bsplit3_pair(ok0 ? ra[u][q] : 0.f, ok1 ? rb[u][q] : 0.f, h, m, l);
          H[w] = h;
          M[w] = m;
          L[w] = l;
        }
      }
  };
  bf4acc acc[kBSW][NTR];
#pragma unroll
  for (int i = 0; i < kBSW; ++i)
#pragma unroll
    for (int j = 0; j < NTR; ++j) acc[i][j] = bf4acc{0.f, 0.f, 0.f, 0.f};
  // lane's operand: column c of block blk, rows 8 lk .. 8 lk + 7, one plane
  auto opnd = [&](const short* P, int blk, int c) {
    return *reinterpret_cast<const bs8*>(P + blk * bsz + bswz(c, 8 * lk));
  };
  auto compute = [&](int buf) {
    const short* Ph = &lds[buf][0][0];
    const short* Pm = &lds[buf][1][0];
    const short* Pl = &lds[buf][2][0];
    bs8 bh[NTR], bm[NTR], bl[NTR];
#pragma unroll
    for (int j = 0; j < NTR; ++j) {
      const int col = 16 * j + lc;
      const int blk = nlb + col / s, c = col % s;
      bh[j] = opnd(Ph, blk, c);
      bm[j] = opnd(Pm, blk, c);
      bl[j] = opnd(Pl, blk, c);
    }
#pragma unroll
    for (int i = 0; i < kBSW; ++i)
      if (i < nsw) {
        const int strip = st0 + i;
        const int blk = strip / spb, c = (strip % spb) * 16 + lc;
        const bs8 ah = opnd(Ph, blk, c), am = opnd(Pm, blk, c), al = opnd(Pl, blk, c);
#pragma unroll
        for (int j = 0; j < NTR; ++j) {
          bf4acc x = acc[i][j];
          x = bmfma(al, bh[j], x);
          x = bmfma(ah, bl[j], x);
          x = bmfma(am, bm[j], x);
          x = bmfma(am, bh[j], x);
          x = bmfma(ah, bm[j], x);
          x = bmfma(ah, bh[j], x);
          acc[i][j] = x;
        }
      }
  };
  // Pipeline: at the top of step st, LDS buffer st & 1 holds tile st and
  // the two register sets hold tiles st + 1 and st + 2 in flight (tile
  // numbers past the last clamp to it: a re-read, never out of range).
  fq4 xa[UPT], xb[UPT], ya[UPT], yb[UPT];
  const int last = nst - 1;
  gload(xa, xb, 0);
  gload(ya, yb, last < 1 ? last : 1);
  lstore(0, xa, xb, 0);
  gload(xa, xb, last < 2 ? last : 2);
  __syncthreads();
  for (int st = 0; st < nst; st += 2) {
    // tile st + 1 in y, tile st + 2 in x
    compute(0);
    if (st + 1 < nst) lstore(1, ya, yb, st + 1);
    gload(ya, yb, st + 3 < last ? st + 3 : last);
    __syncthreads();
    if (st + 1 >= nst) break;
    // tile st + 2 in x, tile st + 3 in y
    compute(1);
    if (st + 2 < nst) lstore(0, xa, xb, st + 2);
    gload(xa, xb, st + 4 < last ? st + 4 : last);
    __syncthreads();
  }
  // D layout: lane l holds rows 4 (l / 16) + r of column l % 16
  double* out = partial + (int64_t)chunk * PA * QB;
  const int col0 = lb0 * s;
#pragma unroll
  for (int i = 0; i < kBSW; ++i)
    if (i < nsw)
#pragma unroll
      for (int j = 0; j < NTR; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          out[(int64_t)(col0 + (st0 + i) * 16 + 4 * lk + r) * QB + 16 * j + lc] =
              (double)acc[i][j][r];
}

// Plan of gram_bf16: the left blocks split into ngroup ranges so that at
// most kBMaxBlk s = 32 blocks (twice as many s = 16 ones) are staged per
// workgroup; one workgroup per CU (LDS), so the chunks make two full rounds
// of 256 workgroups; chunks a multiple of 32 rows.
struct BPlan {
  int ntr, nlb_max, ngroup, nchunk;
  int64_t rows;
};

BPlan bplan(int64_t n, int s, int PA, int QB) {
  BPlan p;
  p.ntr = QB / 16;
  const int nbl = PA / s, nbr = QB / s;
  const int cap = kBMaxBlk * (32 / s) - nbr;
  p.ngroup = (nbl + cap - 1) / cap;
  p.nlb_max = (nbl + p.ngroup - 1) / p.ngroup;
  int64_t nchunk = (512 / p.ngroup) / kXcds * kXcds;
  const int64_t maxc = (n + 511) / 512;
  if (nchunk > maxc) nchunk = maxc;
  if (nchunk < 1) nchunk = 1;
  p.rows = (((n + nchunk - 1) / nchunk) + kBTR - 1) / kBTR * kBTR;
  p.nchunk = (int)((n + p.rows - 1) / p.rows);
  return p;
}

struct MPlan {
  int nchunk, ngroup;
  int64_t rows;
};

// Plan of gram_mfma_wide: the row chunk's strips are split over nw
// wavefronts: one per strip while NS <= 4, 4 * ceil(NS / 16) (at most 4
// strips each) while NS <= 16, else 8 per 40 strips (at most 5 each, four
// right tiles) or per 48 strips (at most 6 each, fewer tiles), so that for
// the shapes of a restart cycle one workgroup stages each right row once; 8
// wavefronts per workgroup when that divides nw, else 4 (or nw); enough row
// chunks for about 2048 busy wavefronts (at least 256 rows each, a multiple
// of 16).
struct WPlan {
  int ntr, sw, wpg, ngroup, nchunk;
  int64_t rows;
};

bool use_wide(int s, int QB) { return s % 16 == 0 && (QB == 16 || QB == 32 || QB == 64); }
// gram_bf16 covers FP32 blocks of s = 16 or 32 (its staging sizes assume it)
bool use_bf16(int s, int QB) { return (s == 16 || s == 32) && use_wide(s, QB); }

WPlan wplan(int64_t n, int PA, int QB) {
  WPlan p;
  p.ntr = QB / 16;
  const int ns = PA / 16;
  // above 16 strips: 8 wavefronts per 32 (NTR = 4, at most 4 each) or per
  // 48 strips (at most 6 each); more strips per wavefront at NTR = 4 would
  // leave too few registers for the fragments in flight
  const int big = p.ntr == 4 ? 4 : 6;
  const int nw = ns <= 4 ? ns : (ns <= 16 ? 4 * ((ns + 15) / 16) : 8 * ((ns + 8 * big - 1) / (8 * big)));
  p.sw = ns <= 16 ? 4 : big;
  p.wpg = nw % 8 == 0 ? 8 : (nw % 4 == 0 ? 4 : nw);
  p.ngroup = nw / p.wpg;
  int64_t nchunk = 2048 / nw;
  const int64_t maxc = (n + 255) / 256;
  if (nchunk > maxc) nchunk = maxc;
  if (nchunk < 1) nchunk = 1;
  p.rows = (((n + nchunk - 1) / nchunk) + 15) & ~int64_t(15);
  p.nchunk = (int)((n + p.rows - 1) / p.rows);
  return p;
}

// Plan of gram_mfma_f64: about 2048 workgroups (eight resident waves per
// SIMD), chunks of at least 256 rows.
MPlan mplan(int64_t n, int PA, int QB) {
  MPlan p;
  const int ntile = ((PA + 15) / 16) * ((QB + 15) / 16);
  p.ngroup = (ntile + 3) / 4;
  int64_t nchunk = 2048 / p.ngroup;
  const int64_t maxc = (n + 255) / 256;
  if (nchunk > maxc) nchunk = maxc;
  if (nchunk < 1) nchunk = 1;
  p.rows = (n + nchunk - 1) / nchunk;
  p.nchunk = (int)((n + p.rows - 1) / p.rows);
  return p;
}

bool use_mfma(int s) { return s >= 8; }

struct Plan {
  int tl, nchunk, ngroup;
  int64_t rows;
};

Plan plan(int64_t n, int s, int PA, int QB) {
  Plan p;
  p.tl = s >= 8 ? 8 : (s >= 4 ? 4 : (s >= 2 ? 2 : 1));
  // a tile must not straddle two blocks: T divides s for s in {1, 2, 4, 8, 16, 32};
  // other block sizes fall back to T = 1 (correct, slower)
  if (s % p.tl != 0) p.tl = 1;
  const int ntile = (PA / p.tl) * (QB / p.tl);
  p.ngroup = (ntile + 3) / 4;
  // Rows per lane: 16 by default (enough work per wavefront to amortise the
  // cross-lane reduction), fewer (down to 4) while the grid has under 1024
  // workgroups, more when the partial buffer would pass 8192 partial tiles.
  int64_t rpl = 16;
  auto chunks = [&](int64_t r) { return (n + 64 * r - 1) / (64 * r); };
  while (rpl > 4 && chunks(rpl) * p.ngroup < 1024) rpl >>= 1;
  while (chunks(rpl) * p.ngroup > 8192 && chunks(rpl) > kXcds) rpl <<= 1;
  int64_t nchunk = chunks(rpl);
  if (nchunk < 1) nchunk = 1;
  p.rows = (n + nchunk - 1) / nchunk;
  p.nchunk = (int)((n + p.rows - 1) / p.rows);
  return p;
}

}  // namespace

size_t gram_partial_doubles(int64_t n, int s, int nleft, int nright) {
  // the largest partial buffer any launch with at most this many blocks plans
  size_t best = 0;
  for (int nl = 1; nl <= nleft; ++nl)
    for (int nr = 1; nr <= nright; ++nr) {
      const Plan p = plan(n, s, nl * s, nr * s);
      size_t need = (size_t)p.nchunk * (size_t)(nl * s) * (size_t)(nr * s);
      if (use_mfma(s)) {
        const MPlan q = mplan(n, nl * s, nr * s);
        const size_t nm = (size_t)q.nchunk * (size_t)(nl * s) * (size_t)(nr * s);
        if (nm > need) need = nm;
      }
      if (use_bf16(s, nr * s)) {
        const BPlan qb = bplan(n, s, nl * s, nr * s);
        const size_t nb = (size_t)qb.nchunk * (size_t)(nl * s) * (size_t)(nr * s);
        if (nb > need) need = nb;
      }
      if (use_wide(s, nr * s)) {
        const WPlan q = wplan(n, nl * s, nr * s);
        const size_t nm = (size_t)q.nchunk * (size_t)(nl * s) * (size_t)(nr * s);
        if (nm > need) need = nm;
      }
      if (need > best) best = need;
    }
  return best;
}

static void launch_stage2(hipStream_t st, const double* partial, int nchunk, int entries,
                          double* out, const Ctl* ctl, KTimer* tm) {
  // entries per workgroup: 8 .. 64, aiming at >= 256 workgroups
  int ewl = 3;
  while (ewl < 6 && ((entries + (1 << ewl) - 1) >> ewl) > 256) ++ewl;
  launch_k(tm, KK_GRAM_REDUCE, 0.0, gram_stage2, dim3((entries + (1 << ewl) - 1) >> ewl),
           dim3(256), 0, st, partial, nchunk, entries, ewl, out, ctl);
}

// Distinct input blocks of a Gram launch (a right block that is also a left
// block is read once by the method).
template <typename T>
int distinct_blocks(const GramArgs<T>& a) {
  int cnt = a.nv + a.nxl;
  for (int j = 0; j < a.nxr; ++j) {
    bool dup = false;
    for (int i = 0; i < a.nxl; ++i) dup |= a.xr[j] == a.xl[i];
    const T* p = a.xr[j];
    if (a.nv > 0 && p >= a.V && p < a.V + (int64_t)a.nv * a.n * a.s) dup = true;
    cnt += dup ? 0 : 1;
  }
  return cnt;
}

// The global paradigm's block inner product (Sec. 2.2, Table 1): each s x s
// block of the reduced Gram becomes (1/s) trace(block) I_s.  One wavefront
// per block; the diagonal is summed by a fixed butterfly (s <= 32), so the
// result does not depend on timing.
__global__ __launch_bounds__(64) void gram_globalize(double* __restrict__ out, int s, int QB,
                                                     const Ctl* __restrict__ ctl) {
  if (ctl && ctl->stop) return;
  const int nbj = QB / s;
  const int bi = blockIdx.x / nbj, bj = blockIdx.x % nbj;
  double* blk = out + (int64_t)bi * s * QB + (int64_t)bj * s;
  const int l = threadIdx.x;
  double v = l < s ? blk[(int64_t)l * QB + l] : 0.0;
  // butterfly over the whole wavefront: every lane holds the sum (lanes
  // 32..63 write entries too once s * s > 32)
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  const double t = v / s;
  for (int e = l; e < s * s; e += 64) {
    const int r = e / s, c = e % s;
    blk[(int64_t)r * QB + c] = r == c ? t : 0.0;
  }
}

template <typename T>
void launch_gram_classical(hipStream_t st, const GramArgs<T>& a, double* partial, double* out,
                           const Ctl* ctl, KTimer* tm);

template <typename T>
void launch_gram(hipStream_t st, const GramArgs<T>& a, double* partial, double* out,
                 const Ctl* ctl, KTimer* tm) {
  launch_gram_classical<T>(st, a, partial, out, ctl, tm);
  if (a.glob) {
    const int PA = (a.nv + a.nxl) * a.s, QB = a.nxr * a.s;
    launch_k(tm, KK_GRAM_REDUCE, 0.0, gram_globalize, dim3((PA / a.s) * (QB / a.s)), dim3(64),
             0, st, out, a.s, QB, ctl);
  }
}

template <typename T>
void launch_gram_classical(hipStream_t st, const GramArgs<T>& a, double* partial, double* out,
                           const Ctl* ctl, KTimer* tm) {
  const int PA = (a.nv + a.nxl) * a.s, QB = a.nxr * a.s;
  const double gflops = 2.0 * (double)a.n * PA * QB;
  if constexpr (sizeof(T) == sizeof(float)) {
    if (use_bf16(a.s, QB)) {
      const BPlan q = bplan(a.n, a.s, PA, QB);
      const int nchunk_pad = ((q.nchunk + kXcds - 1) / kXcds) * kXcds;
      const dim3 g(nchunk_pad * q.ngroup), b(512);
      const double bytes = (double)distinct_blocks(a) * a.n * a.s * sizeof(T);
      if (q.ntr == 4)
        launch_kf(tm, KK_GRAM, bytes, gflops, gram_bf16<4>, g, b, 0, st, a, q.nchunk, q.ngroup,
                  q.nlb_max, q.rows, partial, ctl);
      else if (q.ntr == 2)
        launch_kf(tm, KK_GRAM, bytes, gflops, gram_bf16<2>, g, b, 0, st, a, q.nchunk, q.ngroup,
                  q.nlb_max, q.rows, partial, ctl);
      else
        launch_kf(tm, KK_GRAM, bytes, gflops, gram_bf16<1>, g, b, 0, st, a, q.nchunk, q.ngroup,
                  q.nlb_max, q.rows, partial, ctl);
      launch_stage2(st, partial, q.nchunk, PA * QB, out, ctl, tm);
      return;
    }
  }
  if (use_wide(a.s, QB)) {
    {
      const WPlan q = wplan(a.n, PA, QB);
      const int nchunk_pad = ((q.nchunk + kXcds - 1) / kXcds) * kXcds;
      const dim3 g(nchunk_pad * q.ngroup), b(64 * q.wpg);
      const double bytes = (double)distinct_blocks(a) * a.n * a.s * sizeof(T);
      // RPT: 16-byte right-row chunks per thread and stage (every one is
      // loaded, so it is sized to the workgroup: 16 rows x QB / EPC chunks)
      const int epc = 16 / (int)sizeof(T);
      const int per = (16 * (QB / epc) + 64 * q.wpg - 1) / (64 * q.wpg);
      const int rpt = per <= 1 ? 1 : per <= 2 ? 2 : per <= 4 ? 4 : 8;
#define LSBA_WIDE(SW, NTR, RPT)                                                              \
  launch_kf(tm, KK_GRAM, bytes, gflops, gram_mfma_wide<T, SW, NTR, RPT>, g, b, 0, st, a, q.nchunk, \
            q.ngroup, q.wpg, q.rows, partial, ctl)
#define LSBA_WIDE_R(SW, NTR)                                                                 \
  do {                                                                                       \
    if constexpr (sizeof(T) == sizeof(double)) {                                             \
      if (rpt == 1) LSBA_WIDE(SW, NTR, 1);                                                   \
      else if (rpt == 2) LSBA_WIDE(SW, NTR, 2);                                              \
      else if (rpt == 4) LSBA_WIDE(SW, NTR, 4);                                              \
      else LSBA_WIDE(SW, NTR, 8);                                                            \
    } else {                                                                                 \
      if (rpt == 1) LSBA_WIDE(SW, NTR, 1);                                                   \
      else LSBA_WIDE(SW, NTR, 8);                                                            \
    }                                                                                        \
  } while (0)
      if (q.sw == 4) {
        if (q.ntr == 4) LSBA_WIDE_R(4, 4);
        else if (q.ntr == 2) LSBA_WIDE_R(4, 2);
        else LSBA_WIDE_R(4, 1);
      } else {
        if (q.ntr == 2) LSBA_WIDE(6, 2, 1);
        else LSBA_WIDE(6, 1, 1);
      }
#undef LSBA_WIDE_R
#undef LSBA_WIDE
      launch_stage2(st, partial, q.nchunk, PA * QB, out, ctl, tm);
      return;
    }
  }
  if constexpr (sizeof(T) == sizeof(double)) {
    if (use_mfma(a.s)) {
      const MPlan q = mplan(a.n, PA, QB);
      const int nchunk_pad = ((q.nchunk + kXcds - 1) / kXcds) * kXcds;
      launch_kf(tm, KK_GRAM, (double)distinct_blocks(a) * a.n * a.s * sizeof(T), gflops, gram_mfma_f64,
               dim3(nchunk_pad * q.ngroup), dim3(256), 0, st, a, q.nchunk, q.ngroup, q.rows,
               partial, ctl);
      launch_stage2(st, partial, q.nchunk, PA * QB, out, ctl, tm);
      return;
    }
  }
  const Plan p = plan(a.n, a.s, PA, QB);
  const int nchunk_pad = ((p.nchunk + kXcds - 1) / kXcds) * kXcds;
  const int blocks = nchunk_pad * p.ngroup;
  const double bytes = (double)distinct_blocks(a) * a.n * a.s * sizeof(T);
  switch (p.tl) {
    case 8:
      launch_kf(tm, KK_GRAM, bytes, gflops, gram_stage1<T, 8>, dim3(blocks), dim3(256), 0, st, a, p.nchunk,
               p.ngroup, p.rows, partial, ctl);
      break;
    case 4:
      launch_kf(tm, KK_GRAM, bytes, gflops, gram_stage1<T, 4>, dim3(blocks), dim3(256), 0, st, a, p.nchunk,
               p.ngroup, p.rows, partial, ctl);
      break;
    case 2:
      launch_kf(tm, KK_GRAM, bytes, gflops, gram_stage1<T, 2>, dim3(blocks), dim3(256), 0, st, a, p.nchunk,
               p.ngroup, p.rows, partial, ctl);
      break;
    default:
      launch_kf(tm, KK_GRAM, bytes, gflops, gram_stage1<T, 1>, dim3(blocks), dim3(256), 0, st, a, p.nchunk,
               p.ngroup, p.rows, partial, ctl);
  }
  launch_stage2(st, partial, p.nchunk, PA * QB, out, ctl, tm);
}
template void launch_gram<double>(hipStream_t, const GramArgs<double>&, double*, double*,
                                  const Ctl*, KTimer*);
template void launch_gram<float>(hipStream_t, const GramArgs<float>&, double*, double*,
                                 const Ctl*, KTimer*);

}  // namespace lsba
