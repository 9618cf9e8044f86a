// Internal declarations shared by the HIP kernels and the host driver of liblsba.
//
// Device data layout (one solve):
//   block vectors   n x s, row-major (the s entries of a row adjacent), type T
//                   (double in the FP64 form, float for the inner solves of the
//                   mixed form);
//   basis           slots V_1 .. V_{m+1} contiguous: V + i * n * s;
//   small dense     FP64, row-major, in global memory (see Dense below).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "ilu_plan.h"
#include "lsba.h"

namespace lsba {

constexpr int kMaxS = 32;       // largest block size s
constexpr int kMaxM = 128;      // largest basis size m
constexpr int kSmallThreads = 256;

// Per-solve control word, device resident.  Kernels of a restart cycle read
// `stop` and return at once when it is set, so a whole cycle can be queued
// without a host round trip per step.
enum CtlStatus : int {
  ST_RUNNING = 0,     // cycle in progress
  ST_CONVERGED = 1,   // estimate / nB <= tol after column j
  ST_FLAGGED = 2,     // Cholesky breakdown flag; j = last final column
  ST_ITERCAP = 3      // max_iters final columns reached
};

struct Ctl {
  int stop;
  int status;
  int j;                // final block columns of the current cycle
  int m;                // current maximum basis size (shrinks on a flag)
  long long iter;       // final block columns over all cycles
  long long max_iters;  // <= 0: unlimited
  long long a_calls, v_apps, syncs;
  int flag_step;        // loop step whose Cholesky raised the flag
  int nv1, nv2_begin, nv2;   // block ranges of the cycle-end basis application
  int cont;             // 1: another cycle follows
  int cycles;           // cycles completed
  int cyc_status;       // status of the cycle that ended last
  int last_valid;       // after a flag: the last block column that is final
  int pad1;
  double nB;            // ||B||_F of the right-hand side of this solve
  double tol;
  double est;           // last relative residual estimate
  int arrive[kMaxM + 2];   // per loop step: workgroups of a split small step done
};

// Small dense state of one solve (FP64, device, row-major).
struct Dense {
  int s;          // block size
  int mmax;       // allocated basis size
  int ldh;        // leading dimension of H, T, Rf: (mmax + 1) * s
  int skel;       // lsba_skeleton
  int method;     // lsba_method
  int mixed;      // 1: shifted-Cholesky fallback allowed (mixed form)
  int glob;       // 1: global block paradigm (every Gram block -> (1/s) tr I_s)
  int mgs;        // column-wise muscle: 0 none, 1 MGS-SVL, 2 MGS-LTS
  double* H;      // block Hessenberg, (mmax + 2) s rows x ldh
  double* T;      // auxiliary T of Algs. 5 / 6, ldh x ldh
  double* Tt;     // its transpose (kept so that products read rows), ldh x ldh
  double* J;      // auxiliary J of Alg. 7, (mmax + 1) s x s
  double* G;      // reduced Gram output of loop step k at G + k * gstride, up to (k s) x 2 s
  long long gstride;   // 0: one slot (Alg. 5); delayed skeletons keep one slot per step so
                       // that the off-path H / J / QR work may lag the basis kernels
  double* G2;     // second Gram output (muscle Gram / LOO Gram)
  double* Beta;   // factor of IntraOrtho(R0), s x s
  double* C;      // cospatial factor carried between cycles, s x s
  double* Qt;     // Q_i^T of each block column's 2s x 2s window QR, mmax x (2s x 2s)
  double* Rf;     // transformed (triangularised) H columns, (mmax + 1) s x ldh
  double* g;      // transformed right-hand side E_1 B C, (mmax + 1) s x s
  double* Dlast;  // diagonal block of the last column before its own reflector, s x s
  double* ylast;  // FOM: last block of Xi for the last final column, s x s
  double* Xi;     // block coefficient vector, mmax s x s
  double* M;      // BGMRES modification factor, mmax s x s
  double* Rinv;   // inverse of the latest Cholesky factor, s x s
  double* P;      // P of Algs. 6 / 7, s x s
  double* RiS;    // Alg. 7: R^{-1} of loop step k at RiS + k s^2
  double* PS;     // Alg. 7: P of loop step k at PS + k s^2
  double* Gv;     // V^T V of the current cycle (loss-of-orthogonality record), ldh x ldh
  double* scratch;// workspace for the small kernels, >= 8 * ldh * s + 64 * s * s doubles
  double* coef64; // update coefficients (see Coef below), FP64
  void* coefT;    // the same coefficients in the basis type (float copy for the mixed form)
  double* res_hist;
  double* loo_hist;
  Ctl* ctl;
};

// Coefficient layout of the fused block update (both in FP64 and in T):
//   out1 = in1 * C1 + sum_{i < nv1} V_i * A_i
//   out2 = in2 * C2 + sum_{nv2_begin <= i < nv2} V_i * B_i + out1 * D
// Every matrix is s x s row-major (entry (t, c) multiplies input column t
// into output column c).  With D present the same out2 is also
//   in2 * C2 + in1 * (C1 D) + sum_i V_i * (B_i + A_i D)      (BF(i), C1D()),
// the form the matrix-core update uses (one product with all inputs).
// Offsets (in elements) for block size s, mmax:
struct CoefLayout {
  int s, nvmax;
  __host__ __device__ int C1() const { return 0; }
  __host__ __device__ int A(int i) const { return s * s * (1 + i); }
  __host__ __device__ int C2() const { return s * s * (1 + nvmax); }
  __host__ __device__ int B(int i) const { return s * s * (2 + nvmax + i); }
  __host__ __device__ int D() const { return s * s * (2 + 2 * nvmax); }
  __host__ __device__ int BF(int i) const { return s * s * (3 + 2 * nvmax + i); }
  __host__ __device__ int C1D() const { return s * s * (3 + 3 * nvmax); }
  __host__ __device__ int total() const { return s * s * (4 + 3 * nvmax); }
};

// Kernel classes for the device-time statistics (values of lsba_kernel_kind).
enum KernelKind : int {
  KK_SPMM = 0, KK_GRAM = 1, KK_GRAM_REDUCE = 2, KK_UPDATE = 3, KK_SMALL = 4, KK_RESIDUAL = 5,
  KK_PRECOND = 6, KK_COUNT = 7
};

// Optional launch timer: begin()/end() bracket one kernel launch of class
// `kind` on stream st with HIP events (classes outside the timer's mask are
// not bracketed); `bytes` are the launch's algorithmic bytes (inputs the
// method must read plus outputs it must write).
struct KTimer {
  virtual void begin(hipStream_t st, int kind) = 0;
  virtual void end(hipStream_t st, int kind, double bytes) = 0;
  // Two events that a launch of class `kind` records itself at the start and
  // the end of the kernel (hipExtLaunchKernelGGL), so that their interval is
  // the kernel's own duration; false when the class is not timed.
  virtual bool kernel_events(int kind, hipEvent_t* a, hipEvent_t* b) = 0;
  // `flops`: the launch's algorithmic floating-point operations (the
  // products the method needs, 2 per multiply-add)
  virtual void kernel_done(int kind, hipEvent_t a, hipEvent_t b, double bytes,
                           double flops) = 0;
  virtual ~KTimer() {}
};

// Launch `kernel` on st; when tm times class `kind`, the launch records the
// class's events at the kernel's own start and end.
template <typename F, typename... Args>
inline void launch_kf(KTimer* tm, int kind, double bytes, double flops, F kernel, dim3 grid,
                      dim3 block, size_t shmem, hipStream_t st, Args... args) {
  hipEvent_t a = nullptr, b = nullptr;
  if (tm && tm->kernel_events(kind, &a, &b)) {
    hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)shmem, st, a, b, 0, args...);
    tm->kernel_done(kind, a, b, bytes, flops);
  } else {
    kernel<<<grid, block, shmem, st>>>(args...);
  }
}
template <typename F, typename... Args>
inline void launch_k(KTimer* tm, int kind, double bytes, F kernel, dim3 grid, dim3 block,
                     size_t shmem, hipStream_t st, Args... args) {
  launch_kf(tm, kind, bytes, 0.0, kernel, grid, block, shmem, st, args...);
}

// ------------------------------------------------------------------ kernels
// Sparse: W = A X (CSR x row-major block).
template <typename T>
void launch_spmm(hipStream_t st, int64_t n, int64_t nnz, int s, const int64_t* rp, const int* ci,
                 const T* val, const T* X, T* W, const Ctl* ctl, KTimer* tm = nullptr);
// R = B - A X, and per-workgroup partial sums of squares of R written to partial[]
// (nw entries); norms are then reduced in a fixed order by launch_sumsq_final.
void launch_residual(hipStream_t st, int64_t n, int64_t nnz, int s, const int64_t* rp,
                     const int* ci, const double* val, const double* X, const double* B,
                     double* R, double* partial, int* nw_out, KTimer* tm = nullptr);
void launch_sumsq_partial(hipStream_t st, int64_t count, const double* x, double* partial,
                          int* nw_out);
void launch_sumsq_final(hipStream_t st, const double* partial, int nw, double* out_norm);
// partial[w] = sum over workgroup w's entries of (X - Y)^2 (n x s, leading
// dimensions ldx, ldy), nw_out = number of workgroups (n s / 4096 rounded up)
void launch_diff_sumsq_partial(hipStream_t st, int64_t n, int s, const double* X, int64_t ldx,
                               const double* Y, int64_t ldy, double* partial, int* nw_out);
template <typename T>
void launch_cast(hipStream_t st, int64_t count, const double* in, T* out);
template <typename T>
void launch_add_to_double(hipStream_t st, int64_t count, const T* in, double* acc);

// Gram: G = [left blocks]^T [right blocks], deterministic split-n reduction.
template <typename T>
struct GramArgs {
  int64_t n;
  int s;
  const T* V;        // contiguous left blocks V + i n s, i < nv
  int nv;
  const T* xl[2];    // extra left blocks after the contiguous ones
  int nxl;
  const T* xr[2];    // right blocks
  int nxr;
  int glob;          // global paradigm: each s x s block of the result -> (1/s) trace I_s
};
size_t gram_partial_doubles(int64_t n, int s, int nleft, int nright);
template <typename T>
void launch_gram(hipStream_t st, const GramArgs<T>& a, double* partial, double* out,
                 const Ctl* ctl, KTimer* tm = nullptr);

// Fused block update (coefficients in CoefLayout, type T).
template <typename T>
struct UpdateArgs {
  int64_t n;
  int s;
  const T* V;        // basis slots V + i n s
  const T* in1;      // may be null
  const T* in2;      // may be null
  T* out1;           // may be null
  T* out2;           // may be null
  int nv1, nv2_begin, nv2, has_D;
  const int* nvp;    // if non-null: nv1, nv2_begin, nv2 read from nvp[0..2] (device)
  const T* coef;
  CoefLayout lay;
};
// Algorithmic bytes and flops of one update launch with nv1 / nv2_begin / nv2
// block ranges (flops: 2 n s^2 per nonzero s x s coefficient block applied,
// the D term included).
template <typename T>
double update_bytes(const UpdateArgs<T>& a, int nv1, int nb, int nv2);
template <typename T>
double update_flops(const UpdateArgs<T>& a, int nv1, int nb, int nv2);
template <typename T>
void launch_update(hipStream_t st, const UpdateArgs<T>& a, const Ctl* ctl, bool obey_stop,
                   KTimer* tm = nullptr);

// Small dense steps (one workgroup per solve).  The skeleton steps (start,
// delayed, svl_*) are on the critical path of the basis; finalize (QR update,
// estimate, convergence test of one column) can run on a second stream.
void launch_small_start(hipStream_t st, const Dense& d, int force_flag, KTimer* tm = nullptr);
void launch_small_delayed(hipStream_t st, const Dense& d, int k, int m, int force_flag,
                          KTimer* tm = nullptr);
void launch_small_finalize(hipStream_t st, const Dense& d, int col, KTimer* tm = nullptr);
// Alg. 7 off the basis path, after loop step k >= 2: H_{1:k-1,k-1} = J + Y and
// the J recurrence, one workgroup per block row (the QR update / estimate /
// convergence test of column k-1 follows with launch_small_finalize).
void launch_small_side(hipStream_t st, const Dense& d, int k, int m, KTimer* tm = nullptr);
void launch_small_svl_y(hipStream_t st, const Dense& d, int k, KTimer* tm = nullptr);
void launch_small_svl_io(hipStream_t st, const Dense& d, int k, int force_flag,
                         KTimer* tm = nullptr);
void launch_small_svl_z(hipStream_t st, const Dense& d, int k, KTimer* tm = nullptr);
// Alg. 3 (BCGS-PIP), loop step k: H_{1:k,k}, H_{k+1,k} (flag) and the
// projection coefficients from [V_{1:k} W]^T W.
void launch_small_pip(hipStream_t st, const Dense& d, int k, int force_flag,
                      KTimer* tm = nullptr);
// Alg. 4 (BCGS-PIO), loop step k, after Y = V_{1:k}^T W and the IntraOrtho
// of W (CholQR: W^T W in G2; HouseQR: R_W in H_{k+1,k}): H_{1:k,k},
// H_{k+1,k} (flags) and the projection coefficients.
void launch_small_pio(hipStream_t st, const Dense& d, int k, int force_flag, int house,
                      KTimer* tm = nullptr);
// Column-wise MGS-SVL / MGS-LTS muscle, one phase per launch (the host runs
// the column loop between Gram products and in-place block updates).
enum MgsPhase : int { MGS_INIT = 0, MGS_PROJ = 1, MGS_NORM = 2, MGS_Z = 3, MGS_FINISH = 4 };
enum MgsMode : int { MGS_START = 0, MGS_IO5 = 1, MGS_IOB = 2 };
void launch_small_mgs(hipStream_t st, const Dense& d, int phase, int j, int mode, int k,
                      int force_flag, KTimer* tm = nullptr);
void launch_t_identity(hipStream_t st, const Dense& d, KTimer* tm = nullptr);
// Alg. 2 (BMGS), loop step k, inner step i: H_{i,k} = V_i^T W and the
// coefficients of W <- W - V_i H_{i,k}.
void launch_small_bmgs(hipStream_t st, const Dense& d, int k, int i, KTimer* tm = nullptr);
// skeletons that keep the T factor (Algs. 5, 6)
__host__ __device__ inline bool skel_uses_t(int sk) {
  return sk == LSBA_BMGS_SVL || sk == LSBA_BMGS_LTS || sk == LSBA_BMGS_CWY ||
         sk == LSBA_BMGS_ICWY;
}
void launch_small_cycle_end(hipStream_t st, const Dense& d, KTimer* tm = nullptr);
void launch_small_loo(hipStream_t st, const Dense& d, int k_new_block, KTimer* tm = nullptr);

// HouseQR IntraOrtho (TSQR, FP64 inside) of the n x s block X: Q to out1 (and
// out2 if non-null; either may alias X), R with diag(R) >= 0 to the caller's
// state: HM_START -- the cycle start (control word, Beta, g, T = I), HM_IO --
// Alg. 5's IntraOrtho at loop step k (H_{k+1,k}, flag at step k).  `work`
// holds house_work_doubles(n, s) doubles.
enum HouseMode : int { HM_START = 0, HM_IO = 1 };
size_t house_work_doubles(int64_t n, int s);
template <typename T>
void launch_house(hipStream_t st, const Dense& d, int64_t n, int s, const T* X, T* out1, T* out2,
                  double* work, int mode, int k, int force, KTimer* tm = nullptr);

// ------------------------------------------------------------ ILU(0)
// One triangular sweep of the ILU(0) factors in level order: rows of one
// level depend only on rows of earlier levels, so a level's rows are solved
// in parallel.  Position k (0 <= k < n) of the level order holds row rows[k];
// the positions of level l are [lvl_ptr[l], lvl_ptr[l+1]).  The off-diagonal
// entries of position k (strictly lower part for the forward sweep, strictly
// upper part for the backward sweep) are ci/v[rp[k] .. rp[k+1]), columns
// ascending; piv[k] is u_ii (backward sweep only).
struct IluSweep {
  int nlev = 0;
  int* lvl_ptr = nullptr;
  int* rows = nullptr;
  int64_t* rp = nullptr;
  int* ci = nullptr;
  double* v = nullptr;
  double* piv = nullptr;
  // the first kIluEll entries of each position again, padded to that width
  // (column 0, value 0 past the row's count): their loads need only k
  int* ecol = nullptr;
  double* eval = nullptr;
  std::vector<IluLaunch> plan[6];   // sweep launches for 2^j lanes per row, j = 0..5
  std::vector<IluLaunch> fplan;     // factorization launches (one thread per row)
};
// ILU(0) factors of a CSR matrix: the factors on A's pattern with each row's
// columns sorted (fv: strictly lower part = L's multipliers, the rest = U),
// natural row order, plus both sweeps in level order.
struct IluFactors {
  int64_t n = 0, nnz = 0, nnz_lo = 0, nnz_up = 0;
  int64_t* frp = nullptr;
  int* fci = nullptr;
  double* fv = nullptr;
  IluSweep lo, up;
  std::vector<void*> mem;   // every device allocation of the factors
};
// Analyse the pattern (host copies of A's row pointer and column indices),
// then factor A's values (device) on st.  Returns "" on success, else the
// reason; *bad_input is true when the matrix itself is the reason (n too
// large, a missing diagonal, a duplicate column, a zero or non-finite pivot,
// whose row *bad_row receives; else -1) and false for allocation or HIP
// failures.
std::string ilu_build(hipStream_t st, int64_t n, int64_t nnz, const int64_t* rp_h,
                      const int* ci_h, const double* val_dev, IluFactors& f, int64_t* bad_row,
                      bool* bad_input);
void ilu_free(IluFactors& f);
// Z = U^{-1} L^{-1} Y for n x s row-major blocks (Z may alias Y).
void launch_ilu_apply(hipStream_t st, const IluFactors& f, int s, const double* Y, double* Z,
                      const Ctl* ctl, KTimer* tm = nullptr);

// v rotated right by N lanes within each row of 16 lanes (DPP row_ror):
// lane 16 r + i receives the value of lane 16 r + ((i - N) mod 16).
template <int N>
__device__ __forceinline__ double row_ror(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)u, 0x120 + N, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), 0x120 + N, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                          (unsigned long long)(unsigned)lo));
}

// The FP64 16 x 16 x 4 product acc[t] += A B as four v_mfma_f64_4x4x4f64
// (twice the issue rate of v_mfma_f64_16x16x4f64 on gfx950).  a and b hold
// the 16x16x4 operands (lane l: A[l % 16][l / 16], B[l / 16][l % 16]); the
// 4x4x4 instruction multiplies, for each of the four lane groups g = (l % 16)
// / 4, the 4 x 4 blocks A[4 g .. 4 g + 3][:] and B[:][4 g' .. 4 g' + 3] with
// g' = g, so b rotated by 4 t lanes pairs group g with g' = (g - t) mod 4.
// acc[t] at lane l = 16 i + 4 g + j holds D[4 g + i][4 ((g - t) mod 4) + j]
// (mac), or with the rotated operand taken as A, D[4 ((g - t) mod 4) + i][4 g + j]
// (mac_a).
struct Mfma4 {
  double b[4];
  __device__ __forceinline__ explicit Mfma4(double bv) {
    b[0] = bv;
    b[1] = row_ror<4>(bv);
    b[2] = row_ror<8>(bv);
    b[3] = row_ror<12>(bv);
  }
  __device__ __forceinline__ void mac(double a, double (&acc)[4]) const {
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b[t], acc[t], 0, 0, 0);
  }
  // the same product with the stored operand rotated in the A position:
  // acc[t] at lane l = 16 i + 4 g + j holds D[4 ((g - t) mod 4) + i][4 g + j]
  __device__ __forceinline__ void mac_a(double bv, double (&acc)[4]) const {
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = __builtin_amdgcn_mfma_f64_4x4x4f64(b[t], bv, acc[t], 0, 0, 0);
  }
};

}  // namespace lsba
