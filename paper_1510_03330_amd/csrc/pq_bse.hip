// Bethe-Salpeter equations (Eq. PA_F_Phi) of one channel, solved for every
// bosonic transfer q as the dense complex system
//     A F = Gamma,   A = 1 - s Gamma diag(X),
// followed by Phi <- alpha (F - Gamma) + (1 - alpha) Phi.
//
// Blocked elimination without row exchanges on the augmented [A | B]
// (B = Gamma) with panel width NB (128 for complex64, 64 for complex128),
// batched over all q blocks of a channel: every step is one kernel launch over
// (q block, tile) grids. A forward sweep over the panels J = 0, 1, ...:
//   (a) bse_pivot:  P = A_JJ^-1 by Gauss-Jordan on the NB x NB diagonal block,
//                   held in registers (one column per thread and a slice of its
//                   rows), pivot rows and columns broadcast through LDS, stored
//                   transposed (k-major);
//   (b) bse_panel:  pivot rows R_JK = P A_JK for every column right of the
//                   panel in A and every column of B (in place);
//   (c) bse_update: A_IK -= A_IJ R_JK, B_I -= A_IJ R_JB for the rows I below
//                   the panel, a rank-NB update; each wave owns a 64 x 64
//                   (complex64) or 32 x 32 (complex128) tile, reads both
//                   operands straight from L1/L2 (no LDS), and forms each
//                   complex product from three real matrix products.
// The multipliers A_IJ are read k-major (MT[k][i] = A[i][J0 + k]), which makes
// the matrix-core operand loads of (b) and (c) contiguous: the update of panel
// J - 1 writes those of panel J transposed into MT (two buffers, alternating),
// and bse_multcopy copies them for the first panel (formed from Gamma) and a
// ragged last one. The sweep leaves in A the block unit upper triangular
// factor U (the scaled pivot rows) and in B the right-hand sides Y of
// U F = Y. The back substitution then runs over the panels from the last one
// down: B_I -= U_IJ B_J for the rows I above panel J, with the same update
// kernel; (b) also writes the A part of the pivot rows transposed below the
// diagonal block (where the multipliers of that panel are dead), which gives
// the back substitution U k-major with no copy step. This is (4/3) n^3 complex
// multiply-adds per block, the work of an LU factorisation and two n-column
// triangular solves; full Gauss-Jordan, which also clears U, would take
// 1.5 n^3. B then holds F. The mixing Phi <- alpha (F - Gamma) + (1 - alpha)
// Phi is done by each back-substitution launch for the rows it finishes (the
// panel above), and by the last panel's pivot-row step for its own rows.
// Steps (b) and (c) are complex products on the matrix cores
// (v_mfma_f32_32x32x2f32 for complex64, v_mfma_f64_16x16x4f64 for complex128;
// with BF16x3 products, (c) runs on v_mfma_f32_32x32x16_bf16 from operands
// split in LDS, bse_update_bf_kernel).
//
// No row exchanges: A is the identity minus the small-norm kernel s Gamma X,
// and every leading principal block of it stays invertible while the BSE is
// away from its instability. The pivot monitor records the smallest and
// largest pivot modulus of the elimination per block (the same pivots an LU
// factorisation without exchanges meets) and flags weak or non-finite blocks.
#include <float.h>

#include <algorithm>
#include <type_traits>

#include "pq_internal.h"

namespace pq {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kPst = 12;       // per-block monitor doubles (BseCtx::pst)
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------ matrix cores
template <typename T> struct Mma;

template <> struct Mma<float> {   // v_mfma_f32_32x32x2f32
  static constexpr int TM = 32, TN = 32, KS = 2, NV = 16, KV = 1;
  using acc_t = floatx16;
  __device__ static int a_row(int l) { return l & 31; }
  __device__ static int a_k(int l) { return l >> 5; }
  __device__ static int b_col(int l) { return l & 31; }
  __device__ static int b_k(int l) { return l >> 5; }
  __device__ static int c_row(int l, int v) { return 8 * (v >> 2) + 4 * (l >> 5) + (v & 3); }
  __device__ static int c_col(int l) { return l & 31; }
  __device__ static acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
};

template <> struct Mma<double> {  // v_mfma_f64_16x16x4f64
  static constexpr int TM = 16, TN = 16, KS = 4, NV = 4, KV = 1;
  using acc_t = doublex4;
  __device__ static int a_row(int l) { return l & 15; }
  __device__ static int a_k(int l) { return l >> 4; }
  __device__ static int b_col(int l) { return l & 15; }
  __device__ static int b_k(int l) { return l >> 4; }
  __device__ static int c_row(int l, int v) { return (l >> 4) + 4 * v; }
  __device__ static int c_col(int l) { return l & 15; }
  __device__ static acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

// BF16x3 products on v_mfma_f32_32x32x16_bf16: lane l supplies A[l % 32][k]
// and B[k][l % 32] for the 8 consecutive k = 8 (l / 32) .. + 7 of a 16-deep
// step (KV = 8 values per lane); the accumulator layout is that of every
// 32 x 32 matrix-core product (checked with an exact small-integer probe).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
struct MmaBF3 {
  static constexpr int TM = 32, TN = 32, KS = 16, NV = 16, KV = 8;
  using acc_t = floatx16;
  __device__ static int a_row(int l) { return l & 31; }
  __device__ static int a_k(int l) { return 8 * (l >> 5); }
  __device__ static int b_col(int l) { return l & 31; }
  __device__ static int b_k(int l) { return 8 * (l >> 5); }
  __device__ static int c_row(int l, int v) { return 8 * (v >> 2) + 4 * (l >> 5) + (v & 3); }
  __device__ static int c_col(int l) { return l & 31; }
  __device__ static acc_t mma(bf16x8 a, bf16x8 b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};

// A WM x WN complex output tile owned by one wave (default 32 x 32).
template <typename T, int WM = 32, int WN = 32>
struct WTile {
  using M = Mma<T>;
  using C = typename cplx_of<T>::type;
  static constexpr int SR = WM / M::TM, SC = WN / M::TN;
  typename M::acc_t re[SR][SC], im[SR][SC];

  __device__ void zero() {
#pragma unroll
    for (int a = 0; a < SR; ++a)
#pragma unroll
      for (int b = 0; b < SC; ++b)
#pragma unroll
        for (int v = 0; v < M::NV; ++v) { re[a][b][v] = (T)0; im[a][b][v] = (T)0; }
  }
  // element-wise load / store over this lane's elements (tile-relative row, col)
  template <class F> __device__ void load(F f) {
    const int l = threadIdx.x & 63;
#pragma unroll
    for (int a = 0; a < SR; ++a)
#pragma unroll
      for (int b = 0; b < SC; ++b)
#pragma unroll
        for (int v = 0; v < M::NV; ++v) {
          const C c = f(a * M::TM + M::c_row(l, v), b * M::TN + M::c_col(l));
          re[a][b][v] = c.x;
          im[a][b][v] = c.y;
        }
  }
  template <class F> __device__ void store(F f) {
    const int l = threadIdx.x & 63;
#pragma unroll
    for (int a = 0; a < SR; ++a)
#pragma unroll
      for (int b = 0; b < SC; ++b)
#pragma unroll
        for (int v = 0; v < M::NV; ++v) {
          C c;
          c.x = re[a][b][v];
          c.y = im[a][b][v];
          f(a * M::TM + M::c_row(l, v), b * M::TN + M::c_col(l), c);
        }
  }
  // += (sub = false) or -= (sub = true) the product of one k-slab:
  // a[sr] = A(sr*TM + a_row, k0 + a_k), b[sc] = B(k0 + b_k, sc*TN + b_col)
  __device__ void mac(const C (&a)[SR], const C (&b)[SC], bool sub) {
#pragma unroll
    for (int x = 0; x < SR; ++x)
#pragma unroll
      for (int y = 0; y < SC; ++y) {
        const T ar = sub ? -a[x].x : a[x].x, ai = a[x].y;
        re[x][y] = M::mma(ar, b[y].x, re[x][y]);
        re[x][y] = M::mma(sub ? ai : -ai, b[y].y, re[x][y]);
        im[x][y] = M::mma(ar, b[y].y, im[x][y]);
        im[x][y] = M::mma(sub ? -ai : ai, b[y].x, im[x][y]);
      }
  }
};

// Accumulators of a WM x WN complex tile in the three-product form:
//   X1 += (ar + ai) br,  X2 += ar (bi - br),  X3 += ai (br + bi),
//   Re(ab) = X1 - X3,    Im(ab) = X1 + X2
// (three real matrix products per complex product instead of four).
template <typename T, int WM, int WN>
struct Tile3 {
  using M = Mma<T>;
  using C = typename cplx_of<T>::type;
  static constexpr int SR = WM / M::TM, SC = WN / M::TN;
  typename M::acc_t x1[SR][SC], x2[SR][SC], x3[SR][SC];
  template <class F> __device__ void load_c(F f) {     // X1 = 0, X2 = -Im C, X3 = Re C
    const int l = threadIdx.x & 63;
#pragma unroll
    for (int a = 0; a < SR; ++a)
#pragma unroll
      for (int b = 0; b < SC; ++b)
#pragma unroll
        for (int v = 0; v < M::NV; ++v) {
          const C c = f(a * M::TM + M::c_row(l, v), b * M::TN + M::c_col(l));
          x1[a][b][v] = (T)0;
          x2[a][b][v] = -c.y;
          x3[a][b][v] = c.x;
        }
  }
  __device__ void mac(const C (&av)[SR], const C (&bv)[SC]) {
    T as[SR], bd[SC], bs[SC];
#pragma unroll
    for (int x = 0; x < SR; ++x) as[x] = av[x].x + av[x].y;
#pragma unroll
    for (int y = 0; y < SC; ++y) {
      bd[y] = bv[y].y - bv[y].x;
      bs[y] = bv[y].x + bv[y].y;
    }
#pragma unroll
    for (int x = 0; x < SR; ++x)
#pragma unroll
      for (int y = 0; y < SC; ++y) {
        x1[x][y] = M::mma(as[x], bv[y].x, x1[x][y]);
        x2[x][y] = M::mma(av[x].x, bd[y], x2[x][y]);
        x3[x][y] = M::mma(av[x].y, bs[y], x3[x][y]);
      }
  }
  __device__ void mac(const C (&av)[SR][1], const C (&bv)[SC][1]) {
    C a1[SR], b1[SC];
#pragma unroll
    for (int x = 0; x < SR; ++x) a1[x] = av[x][0];
#pragma unroll
    for (int y = 0; y < SC; ++y) b1[y] = bv[y][0];
    mac(a1, b1);
  }
  __device__ void zero() {
#pragma unroll
    for (int a = 0; a < SR; ++a)
#pragma unroll
      for (int b = 0; b < SC; ++b)
#pragma unroll
        for (int v = 0; v < M::NV; ++v) { x1[a][b][v] = (T)0; x2[a][b][v] = (T)0; x3[a][b][v] = (T)0; }
  }
  // started from zero: ab = (X1 - X3, X1 + X2)
  template <class F> __device__ void store_prod(F f) {
    const int l = threadIdx.x & 63;
#pragma unroll
    for (int a = 0; a < SR; ++a)
#pragma unroll
      for (int b = 0; b < SC; ++b)
#pragma unroll
        for (int v = 0; v < M::NV; ++v) {
          C c;
          c.x = x1[a][b][v] - x3[a][b][v];
          c.y = x1[a][b][v] + x2[a][b][v];
          f(a * M::TM + M::c_row(l, v), b * M::TN + M::c_col(l), c);
        }
  }
  template <class F> __device__ void store_c(F f) {    // C - ab = (X3 - X1, -X1 - X2)
    const int l = threadIdx.x & 63;
#pragma unroll
    for (int a = 0; a < SR; ++a)
#pragma unroll
      for (int b = 0; b < SC; ++b)
#pragma unroll
        for (int v = 0; v < M::NV; ++v) {
          C c;
          c.x = x3[a][b][v] - x1[a][b][v];
          c.y = -x1[a][b][v] - x2[a][b][v];
          f(a * M::TM + M::c_row(l, v), b * M::TN + M::c_col(l), c);
        }
  }
};

template <typename C> __device__ inline C cz();
template <> __device__ inline float2 cz<float2>() { return make_float2(0.f, 0.f); }
template <> __device__ inline double2 cz<double2>() { return make_double2(0.0, 0.0); }
template <typename C> __device__ inline C make_cone();
template <> __device__ inline float2 make_cone<float2>() { return make_float2(1.f, 0.f); }
template <> __device__ inline double2 make_cone<double2>() { return make_double2(1.0, 0.0); }

// acc -= a * b
__device__ inline float2 cfms(float2 acc, float2 a, float2 b) {
  acc.x = fmaf(-a.x, b.x, acc.x);
  acc.x = fmaf(a.y, b.y, acc.x);
  acc.y = fmaf(-a.x, b.y, acc.y);
  acc.y = fmaf(-a.y, b.x, acc.y);
  return acc;
}
__device__ inline double2 cfms(double2 acc, double2 a, double2 b) {
  acc.x = fma(-a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(-a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
  return acc;
}
template <typename C> __device__ inline double cabs_d(C a) {
  return sqrt((double)a.x * a.x + (double)a.y * a.y);
}


// Column pointer in the combined column space [A columns right of the panel | B].
template <typename C>
__device__ inline C* colptr(C* A, C* B, int n, int j0, int jb, int c) {
  const int ncolA = n - j0 - jb;
  return c < ncolA ? A + (j0 + jb + c) : B + (c - ncolA);
}

template <typename T>
struct BseCtx {
  using C = typename cplx_of<T>::type;
  int n, Nq, nJ;
  T sign;
  double alpha;
  float weak_ratio;
  const C* gamma;        // [Nq][n][n]
  const double2* chi0;   // [Nq][n]
  C* phi;                // [Nq][n][n]
  C* A;                  // [Nq][n][n]
  C* B;                  // [Nq][n][n]
  C* MT;                 // [3][Nq][NB][n] multipliers, k-major (panel J in buffer J % 3; the
                         //                kernels take the buffer of their panel)
  C* PI;                 // [Nq][NB][NB]   inverse P of the current diagonal block, transposed:
                         //                PI[k][r] = P[r][k] (k-major, like MT)
  double* pst;           // [Nq][kPst]  [0] min |pivot|, [1] max |pivot|, [2] non-finite seen,
                         //             [3] re-solved in FP64, [4] largest |entry| of the
                         //             diagonal-block inverses, [5] error estimate,
                         //             [6] estimate above tol (2: refined estimate pending),
                         //             [7] unresolved, [8], [9] |F v_p|^2 of the two probes
  double kappa_max;      // flag a block whose diagonal-block inverses exceed this
  pq_bse_block_stats* stats;
  const int* active;     // nullable: only blocks < *active are solved (re-solve slots)
  float* pcs;            // complex64 paths: [Nq][ceil(n/64)][n] column sums of |F_ij|^2 over
                         // the 64-row blocks of F, written by the kernels that mix the rows
};

// Column sums of |F_ij|^2 over one 64-row block: the two lanes l and l + 32 of
// a 32-column tile hold different rows of column l % 32 in the matrix-core
// layouts used here, so they are combined and lanes 0 .. 31 store
// (complex64 paths: the norms of the error estimate).
__device__ inline void put_cs(float* pcs, int n, int blk, int rowblk, int col, float v) {
  v += __shfl_xor(v, 32, 64);
  const int nr = (n + 63) / 64;
  if ((threadIdx.x & 63) < 32 && rowblk < nr && col < n) pcs[((size_t)blk * nr + rowblk) * n + col] = v;
}

template <typename T>
__device__ inline bool inactive(const BseCtx<T>& a, int blk) { return a.active && blk >= *a.active; }

// -------------------------------------------------------- first panel
// The system is never materialised before the elimination: the kernels of the
// first panel read Gamma and form A = 1 - s Gamma diag(X) on the fly (B starts
// as Gamma), and their writes create the A and B arrays the later panels use
// (pivot rows from the pivot-row step, every other row from the update).
// Element (i, j) of [A | B] in the combined column index j (< n: A, else B).
template <typename T>
__device__ inline typename cplx_of<T>::type system_elem(const BseCtx<T>& a, int blk, int i, int j) {
  using C = typename cplx_of<T>::type;
  const int n = a.n;
  const bool inA = j < n;
  const int col = inA ? j : j - n;
  const C g = a.gamma[(size_t)blk * n * n + (size_t)i * n + col];
  if (!inA) return g;
  const double2 xv = a.chi0[(size_t)blk * n + col];
  const T sx = a.sign * (T)xv.x, sy = a.sign * (T)xv.y;
  C v;
  v.x = (i == j ? (T)1 : (T)0) - (g.x * sx - g.y * sy);
  v.y = -(g.x * sy + g.y * sx);
  return v;
}

// Multipliers of panel J: A[i][J0 .. J0 + NB) for 32 rows i0 .. i0 + 31,
// through an LDS transpose into MT[k][i]; rows k >= jb of MT (ragged last
// panel) are written as zeros, so the update reads them unmasked. The rows
// i < J0 are the entries U_IJ the back substitution needs (final once the
// forward sweep reaches panel J): except for the last panel, whose MT the back
// substitution reads directly, they go transposed into A[J0 + k][i], the part
// of A left of the diagonal block in the panel's rows, which holds multipliers
// already consumed by the earlier panels (same row stride n as MT). Used for
// the first panel (multipliers formed from Gamma) and a ragged last panel; the
// other panels get both parts from the kernels that produce the values (the
// pivot-row step and the previous update, below).
template <typename T, int NB>
__device__ void copy_multipliers(const BseCtx<T>& a, int blk, int j0, int i0,
                                 typename cplx_of<T>::type (*X)[NB + 1]) {
  using C = typename cplx_of<T>::type;
  const int t = threadIdx.x, nt = blockDim.x, n = a.n;
  const int jb = min(NB, n - j0);
  C* A = a.A + (size_t)blk * n * n;
  C* MT = a.MT + (size_t)blk * NB * n;
  C* UT = j0 != (a.nJ - 1) * NB ? A + (size_t)j0 * n : MT;
  for (int idx = t; idx < 32 * NB; idx += nt) {
    const int r = idx / NB, k = idx - (idx / NB) * NB;
    const int i = min(i0 + r, n - 1), j = j0 + min(k, jb - 1);
    const C v = j0 == 0 ? system_elem(a, blk, i, j) : A[(size_t)i * n + j];
    X[r][k] = k < jb ? v : cz<C>();
  }
  __syncthreads();
  for (int idx = t; idx < 32 * NB; idx += nt) {
    const int k = idx >> 5, r = idx & 31;
    if (i0 + r < n) (i0 + r < j0 ? UT : MT)[(size_t)k * n + i0 + r] = X[r][k];
  }
}

// ------------------------------------------------------------------ pivot
// P = A_JJ^-1 by in-place Gauss-Jordan on the diagonal block (identity outside
// the jb x jb part for a ragged last panel). Thread t holds column j = t % NB
// of the block for the RPT rows r0 .. r0 + RPT - 1 (r0 = RPT t / NB; a wave
// lies inside one row group, so r0 is wave-uniform) in registers (RPT = 32 for
// NB = 128 with 512 threads, 16 for NB = 64). Step c publishes the pivot column
// and row through LDS (double buffered, one barrier per step), then every
// thread updates its entries:
//   row c:           x <- x / p            (column c: x <- 1 / p)
//   other rows r:    x <- x - D[r][c] D[c][j] / p   (column c: x <- -D[r][c] / p)
// Column c is cleared by its owner once published, so one fused multiply-add
// form covers every column; row c is overwritten afterwards by the one wave
// pair that holds it, through a wave-uniform register index.
template <int NB> constexpr int pivot_threads() { return NB >= 128 ? 512 : 256; }

// 1 / z for a pivot. complex64: z scaled by a power of two so that |z|^2 can
// neither overflow nor underflow, then one hardware reciprocal (<= 1 ulp).
__device__ inline float2 pivot_recip(float2 z) {
  int e;
  (void)frexpf(fmaxf(fabsf(z.x), fabsf(z.y)), &e);
  const float a = ldexpf(z.x, -e), b = ldexpf(z.y, -e);
  const float r = __builtin_amdgcn_rcpf(fmaf(a, a, b * b));
  return make_float2(ldexpf(a * r, -e), ldexpf(-b * r, -e));
}
__device__ inline double2 pivot_recip(double2 z) { return crecip(z); }

template <typename T, int NB>
__global__ __launch_bounds__(pivot_threads<NB>()) __attribute__((amdgpu_waves_per_eu(NB >= 128 ? 4 : 3)))
void bse_pivot_kernel(BseCtx<T> a, int j0) {
  using C = typename cplx_of<T>::type;
  constexpr int NT = pivot_threads<NB>();
  constexpr int RPT = NB * NB / NT;
  static_assert(NB % 64 == 0, "a wave must lie inside one row group");
  __shared__ C colbuf[2][NB];
  __shared__ C rowbuf[2][NB];
  __shared__ C pv[NB];
  if (inactive(a, (int)blockIdx.y)) return;
  const int blk = blockIdx.y, t = threadIdx.x, n = a.n;
  const int j = t % NB;
  const int r0 = __builtin_amdgcn_readfirstlane(t / NB) * RPT;
  const int jb = min(NB, n - j0);
  const C* A = a.A + (size_t)blk * n * n;
  T xr[RPT], xi[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int r = r0 + q;
    const int ri = j0 + min(r, jb - 1), ci = j0 + min(j, jb - 1);
    const C v = j0 == 0 ? system_elem(a, blk, ri, ci) : A[(size_t)ri * n + ci];
    const bool in = r < jb && j < jb;
    xr[q] = in ? v.x : (r == j ? (T)1 : (T)0);
    xi[q] = in ? v.y : (T)0;
  }
  for (int c = 0; c < jb; ++c) {
    const int bf = c & 1;
    const int cr = c - r0;                                 // wave-uniform
    const bool own_row = (unsigned)cr < (unsigned)RPT;     // wave-uniform
    if (j == c) {
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        C v;
        v.x = xr[q];
        v.y = xi[q];
        colbuf[bf][r0 + q] = v;
        xr[q] = (T)0;
        xi[q] = (T)0;
      }
    }
    if (own_row) {
      C v;
      if constexpr (sizeof(T) == 4) {
        v.x = xr[cr];
        v.y = xi[cr];
      } else {   // (a dynamic index would put the complex128 block in scratch)
        v = cz<C>();
#pragma unroll
        for (int q = 0; q < RPT; ++q)
          if (q == cr) {
            v.x = xr[q];
            v.y = xi[q];
          }
      }
      rowbuf[bf][j] = v;
    }
    __syncthreads();
    const C piv = colbuf[bf][c];
    if (t == 0) pv[c] = piv;
    const C p = pivot_recip(piv);
    const C rv = rowbuf[bf][j];
    C u;
    u.x = j == c ? p.x : rv.x * p.x - rv.y * p.y;
    u.y = j == c ? p.y : rv.x * p.y + rv.y * p.x;
    // the pivot column is read in chunks of 16 entries (wide broadcast reads
    // issued together), then applied
#pragma unroll
    for (int q0 = 0; q0 < RPT; q0 += 16) {
      C cv[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) cv[q] = colbuf[bf][r0 + q0 + q];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        xr[q0 + q] = fma(-cv[q].x, u.x, fma(cv[q].y, u.y, xr[q0 + q]));
        xi[q0 + q] = fma(-cv[q].x, u.y, fma(-cv[q].y, u.x, xi[q0 + q]));
      }
    }
    if (own_row) {
      if constexpr (sizeof(T) == 4) {
        xr[cr] = u.x;
        xi[cr] = u.y;
      } else {
#pragma unroll
        for (int q = 0; q < RPT; ++q)
          if (q == cr) {
            xr[q] = u.x;
            xi[q] = u.y;
          }
      }
    }
  }
  C* PT = a.PI + (size_t)blk * NB * NB;     // stored transposed: column j of P is row j of PT
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    C v;
    v.x = xr[q];
    v.y = xi[q];
    PT[(size_t)j * NB + r0 + q] = v;
  }
  // pivot monitor: largest |entry|^2 of P (read back from this thread's own
  // stores, which keeps the register-resident block free of extra live
  // values), smallest and largest |pivot|, non-finite pivots
  T xm2 = (T)0;
  for (int q = 0; q < RPT; ++q) {
    const C v = PT[(size_t)j * NB + r0 + q];
    xm2 = fmax(xm2, v.x * v.x + v.y * v.y);
  }
  __syncthreads();                                  // pv complete
  double pmin = DBL_MAX, pmax = 0.0, bad = 0.0;
  if (t < jb) {
    const double ap = cabs_d(pv[t]);
    const bool fin = ap == ap && ap <= DBL_MAX;
    pmin = fin ? ap : DBL_MAX;
    pmax = fin ? ap : 0.0;
    bad = fin ? 0.0 : 1.0;
  }
  for (int o = 32; o > 0; o >>= 1) {
    xm2 = fmax(xm2, __shfl_xor(xm2, o, 64));
    pmin = fmin(pmin, __shfl_xor(pmin, o, 64));
    pmax = fmax(pmax, __shfl_xor(pmax, o, 64));
    bad = fmax(bad, __shfl_xor(bad, o, 64));
  }
  __shared__ double wred[NT / 64][4];
  if ((t & 63) == 0) {
    wred[t >> 6][0] = xm2;
    wred[t >> 6][1] = pmin;
    wred[t >> 6][2] = pmax;
    wred[t >> 6][3] = bad;
  }
  __syncthreads();
  if (t == 0) {
    double xm = 0.0;
    for (int w = 0; w < NT / 64; ++w) {
      xm = fmax(xm, sqrt(wred[w][0]));
      pmin = fmin(pmin, wred[w][1]);
      pmax = fmax(pmax, wred[w][2]);
      bad = fmax(bad, wred[w][3]);
    }
    double* ps = a.pst + (size_t)blk * kPst;
    const bool first = j0 == 0;
    ps[0] = first ? pmin : fmin(ps[0], pmin);
    ps[1] = first ? pmax : fmax(ps[1], pmax);
    ps[2] = (bad > 0.0 || (!first && ps[2] > 0.0)) ? 1.0 : 0.0;
    if (first) ps[3] = 0.0;
    ps[4] = first ? xm : fmax(ps[4], xm);
  }
}

// Multiplier copy of panel J (independent of the diagonal-block inverse; its
// own launch, since sharing the inversion launch halves both kernels' slots):
// 32 rows of A_IJ per workgroup into MT.
template <typename T, int NB>
__global__ __launch_bounds__(kThreads) void bse_multcopy_kernel(BseCtx<T> a, int j0) {
  __shared__ typename cplx_of<T>::type X[32][NB + 1];
  if (inactive(a, (int)blockIdx.y)) return;
  copy_multipliers<T, NB>(a, blockIdx.y, j0, blockIdx.x * 32, X);
}

// Mixing of the solved vertex: Phi <- alpha (F - Gamma) + (1 - alpha) Phi.
template <typename T>
__device__ inline typename cplx_of<T>::type mix_phi(typename cplx_of<T>::type f, typename cplx_of<T>::type g,
                                                    typename cplx_of<T>::type o, T al, T be, bool mix) {
  typename cplx_of<T>::type v;
  v.x = f.x - g.x;
  v.y = f.y - g.y;
  if (mix) {
    v.x = al * v.x + be * o.x;
    v.y = al * v.y + be * o.y;
  }
  return v;
}

// ------------------------------------------------------------------ panel
// One 32-column strip per wave: R = P A_J,strip for RW rows of the panel at
// once (RW / 32 accumulator tiles in the three-product form; NB / RW waves per
// strip), written in place after the whole strip has been read.
// Source of the strip's panel rows: A/B, or (first panel) Gamma with
// A = 1 - s Gamma diag(X) formed per element. colsrc() gives the per-lane
// pointer (row j0 of column c) and the diagonal-term data of the column.
template <typename T>
struct ColSrc {
  using C = typename cplx_of<T>::type;
  const C* p;          // element of row j0 of this column
  T sx, sy;            // s X[col] for an A column (0 for a B column)
  int diag;            // row index whose element gets the unit diagonal (-1: none)
  bool inA;
  __device__ C at(int k, int n, int j0) const {   // row j0 + k
    return form(p[(size_t)k * n], k, j0);
  }
  __device__ C form(C g, int k, int j0) const {    // the element of row j0 + k from its Gamma value
    if (!inA) return g;
    C v;
    v.x = (j0 + k == diag ? (T)1 : (T)0) - (g.x * sx - g.y * sy);
    v.y = -(g.x * sy + g.y * sx);
    return v;
  }
};

template <typename T, bool FIRST>
__device__ inline ColSrc<T> colsrc(const BseCtx<T>& a, int blk, int j0, int jb, int c) {
  ColSrc<T> r;
  const int n = a.n;
  const int ncolA = n - j0 - jb;
  r.inA = FIRST && c < ncolA;
  r.diag = -1;
  r.sx = (T)0;
  r.sy = (T)0;
  if (FIRST) {
    const int col = c < ncolA ? j0 + jb + c : c - ncolA;
    r.p = a.gamma + (size_t)blk * n * n + (size_t)j0 * n + col;
    if (r.inA) {
      const double2 xv = a.chi0[(size_t)blk * n + col];
      r.sx = a.sign * (T)xv.x;
      r.sy = a.sign * (T)xv.y;
      r.diag = col;
    }
  } else {
    r.p = colptr(a.A + (size_t)blk * n * n, a.B + (size_t)blk * n * n, n, j0, jb, c) + (size_t)j0 * n;
  }
  return r;
}

// panel rows per wave: all NB for complex64 (the strip's panel rows are read
// once); 32 for complex128, whose 64-row strip would hold 192 accumulator
// registers and run at one wave per SIMD
template <typename T, int NB> constexpr int panel_rows_per_wave() { return sizeof(T) == 4 ? NB : 32; }

template <typename T, int NB, bool FIRST, int RW = NB, int PFB = 2>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2)))
void bse_panel_kernel(BseCtx<T> a, int j0, int nwb, int mix) {
  using C = typename cplx_of<T>::type;
  using M = Mma<T>;
  using WT = WTile<T>;
  constexpr int SR = WT::SR, SC = WT::SC, KSTEPS = NB / M::KS, NRT = RW / 32, WPS = NB / RW, PFA = 2;
  const int blk = blockIdx.y, t = threadIdx.x, lane = t & 63, wave = t >> 6, n = a.n;
  const int jb = min(NB, n - j0);
  const int ncols = (n - j0 - jb) + n;
  C* A = a.A + (size_t)blk * n * n;
  C* B = a.B + (size_t)blk * n * n;
  static_assert(kWaves % WPS == 0, "the waves of one strip share a workgroup");
  __shared__ C tr_s[kWaves][32][33];            // per-wave transpose tile of the U copy
  if (inactive(a, blk)) return;                 // uniform over the workgroup
  {
    const int ws = blockIdx.x * kWaves + wave;
    const int cs = ws / WPS, rb = (ws % WPS) * RW;      // strip, first panel row of this wave
    // a wave past the last strip computes nothing but still meets the barrier
    // below (both waves of a strip are live or neither is)
    const bool live = cs * 32 < ncols;
    const C* PT = a.PI + (size_t)blk * NB * NB;   // P transposed (k-major)
    const int kb = M::b_k(lane);
    ColSrc<T> cp[SC];
#pragma unroll
    for (int y = 0; y < SC; ++y)
      cp[y] = colsrc<T, FIRST>(a, blk, j0, jb, min(cs * 32 + y * M::TN + M::b_col(lane), ncols - 1));
    const C* pa[NRT][SR];
#pragma unroll
    for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
      for (int xx = 0; xx < SR; ++xx) pa[rt][xx] = PT + (size_t)M::a_k(lane) * NB + rb + rt * 32 + xx * M::TM + M::a_row(lane);
    Tile3<T, 32, 32> acc[NRT];
#pragma unroll
    for (int rt = 0; rt < NRT; ++rt) acc[rt].zero();
    // operands for k-step ks: b from the panel rows of this strip (clamped to
    // the last real row; first touch of these rows, from HBM, so fetched PFB
    // k-steps ahead), a from P (rows outside jb x jb are the identity; shared
    // by every strip of the block, from L2, PFA k-steps ahead)
    auto fetch_a = [&](int ks, C (&av)[NRT][SR]) {
#pragma unroll
      for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
        for (int xx = 0; xx < SR; ++xx) av[rt][xx] = pa[rt][xx][(size_t)ks * M::KS * NB];
    };
    auto fetch_b = [&](int ks, C (&bv)[SC]) {
      const int k = min(ks * M::KS + kb, jb - 1);
#pragma unroll
      for (int y = 0; y < SC; ++y) bv[y] = cp[y].at(k, n, j0);
    };
    C aq[PFA][NRT][SR], bq[PFB][SC];
    if (live) {
#pragma unroll
    for (int s = 0; s < PFB; ++s) fetch_b(s, bq[s]);
#pragma unroll
    for (int s = 0; s < PFA; ++s) fetch_a(s, aq[s]);
#pragma unroll
    for (int ks = 0; ks < KSTEPS; ++ks) {
      C av[NRT][SR], bv[SC];
#pragma unroll
      for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
        for (int xx = 0; xx < SR; ++xx) av[rt][xx] = aq[ks % PFA][rt][xx];
#pragma unroll
      for (int y = 0; y < SC; ++y) bv[y] = bq[ks % PFB][y];
      if (ks + PFB < KSTEPS) fetch_b(ks + PFB, bq[ks % PFB]);
      if (ks + PFA < KSTEPS) fetch_a(ks + PFA, aq[ks % PFA]);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int rt = 0; rt < NRT; ++rt) acc[rt].mac(av[rt], bv);
    }
    }
    // The pivot rows are overwritten in place: with several waves per strip,
    // every wave must have read all NB panel rows of the strip first. The A
    // part of the pivot rows is the U_JK the back substitution needs: it also
    // goes transposed into A[K][J0 + row], below the diagonal block, where the
    // multipliers of panel J are no longer needed (the update reads them from
    // MT), so that the back substitution reads U k-major with no copy step.
    // The transpose goes through a per-wave LDS tile (row stride 33: no bank
    // conflicts on the column-wise writes), so that each store instruction
    // writes two contiguous 32-element runs of A.
    if constexpr (WPS > 1) __syncthreads();
    if (live) {
      const int ncolA = n - j0 - jb;
      const bool tr = cs * 32 < ncolA;            // wave-uniform: the strip has A columns
      C (*ts)[33] = tr_s[wave];
      // the last panel's rows of B are final F: mixed into Phi here, and on the
      // complex64 paths |F_ij X_j|^2 summed per 64-row block (ncolA = 0 there,
      // so the strip is one 32-column tile of F)
      const bool mixes = mix && cs * 32 >= ncolA;
      float fs[2] = {0.f, 0.f};      // |F_ij|^2 of this lane's column, per 64-row block
#pragma unroll
      for (int rt = 0; rt < NRT; ++rt) {
        acc[rt].store_prod([&](int r, int c, C v) {
          const int row = rb + rt * 32 + r, col = cs * 32 + c;
          if (row < jb && col < ncols) {
            colptr(A, B, n, j0, jb, col)[(size_t)(j0 + row) * n] = v;
            if (mixes) {
              const size_t e = (size_t)blk * n * n + (size_t)(j0 + row) * n + (col - ncolA);
              const bool m = a.alpha != 1.0;
              a.phi[e] = mix_phi<T>(v, a.gamma[e], m ? a.phi[e] : cz<C>(), (T)a.alpha, (T)(1.0 - a.alpha), m);
              if constexpr (sizeof(T) == 4) fs[(rb + rt * 32) / 64 % 2] += (float)v.x * v.x + (float)v.y * v.y;
            }
          }
          if (tr) ts[c][r] = v;
        });
        if (tr) {
          // the LDS tile is private to the wave: a wave-scope fence orders the
          // writes above before the reads below (and the reads before the
          // next tile's writes)
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
          for (int it = 0; it < 16; ++it) {
            const int e = it * 64 + lane, c = e >> 5, r = e & 31;
            const int row = rb + rt * 32 + r, col = cs * 32 + c;
            if (row < jb && col < ncolA) A[(size_t)(j0 + jb + col) * n + j0 + row] = ts[c][r];
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
      }
      if constexpr (sizeof(T) == 4) {
        if (mixes && a.pcs) {
          // rows j0 + rb .. + RW: one or two 64-row blocks (j0 is a multiple of 128);
          // lane l holds column l % 32 of the strip
          const int col = cs * 32 + lane % 32 - ncolA;
          put_cs(a.pcs, n, blk, (j0 + rb) / 64, col, fs[0]);
          if (RW > 64) put_cs(a.pcs, n, blk, (j0 + rb) / 64 + 1, col, fs[1]);
        }
      }
    }
  }
}

// ----------------------------------------------------------------- update
// C[i][col] -= sum_k MT[k][i] R[k][col] for the rows row_lo <= i < row_hi and
// the combined columns col_lo <= col < ncols: the forward step takes the rows
// below the panel and every column right of it in A and B, the back
// substitution the rows above the panel and the columns of B. The forward
// step's results in the first ntc combined columns (the columns of the next
// panel) are final multipliers of that panel for the rows below it: those go
// transposed into mtn[col][i], the next panel's MT, instead of into A (where
// nothing reads them: the next pivot-row step writes U there); the next
// panel's diagonal block (the rows below the panel up to mult_row, where the
// multiplier rows start) is stored in A as usual. A forward step may be split
// by rows (the next panel's rows first), mult_row staying the same.
// In the back substitution the rows mix_lo .. row_hi (the panel above, whose F
// is final after this launch) are also mixed into Phi as they are stored
// (Phi <- alpha (F - Gamma) + (1 - alpha) Phi; B keeps F, the next launch's
// operand).
// Tile shape and pipelining of the update: wave tile UWM x UWN, workgroup of
// 2 x 2 waves, operand prefetch PF k-steps ahead; FULL = the panel is NB wide
// (every panel but a ragged last one), so the panel rows need no clamping.
// M3 = complex products with three real matrix products instead of four:
//   X1 += (ar + ai) br,  X2 += ar (bi - br),  X3 += ai (br + bi),
//   Re(ab) = X1 - X3,    Im(ab) = X1 + X2,
// with X3 started at Re C and X2 at -Im C, so C - ab = (X3 - X1, -X1 - X2).
template <typename T_, int UWM_, int UWN_, int PF_, int WPE_, bool FULL_, bool M3_ = true, bool FIRST_ = false,
          bool NT_ = false, bool BF3_ = false>
struct UpdCfg {
  using T = T_;
  static constexpr int UWM = UWM_, UWN = UWN_, PF = PF_, WPE = WPE_;
  static constexpr bool FULL = FULL_, M3 = M3_, FIRST = FIRST_, NT = NT_, BF3 = BF3_;
  static constexpr int WGM = 2 * UWM, WGN = 2 * UWN;
};
// the same tile configuration for the first panel (C read from Gamma)
template <class CF>
using UpdFirst = UpdCfg<typename CF::T, CF::UWM, CF::UWN, CF::PF, CF::WPE, CF::FULL, CF::M3, true, CF::NT, CF::BF3>;

// C tile element access; NT = streaming (non-temporal) hint, so that the C
// stream does not evict the operand panels every workgroup of the block reuses
template <bool NT, typename C>
__device__ inline C ld_c(const C* p) {
  if constexpr (NT) {
    C v;
    v.x = __builtin_nontemporal_load(&p->x);
    v.y = __builtin_nontemporal_load(&p->y);
    return v;
  } else {
    return *p;
  }
}
template <bool NT, typename C>
__device__ inline void st_c(C* p, C v) {
  if constexpr (NT) {
    __builtin_nontemporal_store(v.x, &p->x);
    __builtin_nontemporal_store(v.y, &p->y);
  } else {
    *p = v;
  }
}
// (the ragged-panel form of the complex64 update uses a 64 x 32 tile: the
// clamping of panel rows costs registers the 64 x 64 tile does not have)
template <typename T, bool FULL>
using UpdDefault = typename std::conditional<
    sizeof(T) == 4,
    typename std::conditional<FULL, UpdCfg<T, 64, 64, 2, 2, true, true, false, true>,
                              UpdCfg<T, 64, 32, 2, 3, false, true, false, true>>::type,
    UpdCfg<T, 32, 32, 1, 2, FULL, true, false, true>>::type;

// BF16x3 update of full panels: bse_update_bf_kernel (LDS-staged operands;
// the UWN / PF / FIRST / BF3 fields of this configuration select and shape
// it, the others are unused): a 64 x 64 wave tile (128 x 128 workgroup) with
// loads one step ahead, or (bse_tile = 1) a 64 x 32 wave tile (128 x 64
// workgroup) with loads two steps ahead. A ragged last panel's update takes
// the complex64 FP32 products.
template <bool FULL>
using UpdBF3 = UpdCfg<float, 64, 64, 1, 2, FULL, false, false, true, true>;
template <bool FULL>
using UpdBF3N = UpdCfg<float, 64, 32, 2, 3, FULL, false, false, true, true>;
template <typename T, bool FULL, bool BF3>
using UpdSel = typename std::conditional<BF3 && FULL, UpdBF3<FULL>, UpdDefault<T, FULL>>::type;
// the narrow complex64 tile (bse_tile = 1): 64 x 32 per wave, three waves per
// SIMD, twice the workgroups of the default for the same update
template <bool FULL>
using UpdNarrow = UpdCfg<float, 64, 32, 2, 3, FULL, true, false, true>;

// The four-product form behind the same interface (acc = C, acc -= ab).
template <typename T, int WM, int WN>
struct Tile4 : WTile<T, WM, WN> {
  using C = typename cplx_of<T>::type;
  template <class F> __device__ void load_c(F f) { this->load(f); }
  __device__ void mac(const C (&av)[WTile<T, WM, WN>::SR][1], const C (&bv)[WTile<T, WM, WN>::SC][1]) {
    C a1[WTile<T, WM, WN>::SR], b1[WTile<T, WM, WN>::SC];
#pragma unroll
    for (int x = 0; x < WTile<T, WM, WN>::SR; ++x) a1[x] = av[x][0];
#pragma unroll
    for (int y = 0; y < WTile<T, WM, WN>::SC; ++y) b1[y] = bv[y][0];
    WTile<T, WM, WN>::mac(a1, b1, true);
  }
  template <class F> __device__ void store_c(F f) { this->store(f); }
};

template <typename T, int NB, class CF, int NK = 1>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(CF::WPE)))
void bse_update_kernel(BseCtx<T> a, int j0, int ncb, int row_lo, int row_hi, int col_lo, int col_hi,
                       const typename cplx_of<T>::type* mt0, const typename cplx_of<T>::type* mt1, size_t mt_bs,
                       typename cplx_of<T>::type* mtn, int ntc, int mix_lo, int mult_row) {
  using C = typename cplx_of<T>::type;
  static_assert(!CF::BF3, "the BF16x3 products have their own kernel");
  using M = Mma<T>;
  using UT = typename std::conditional<CF::M3, Tile3<T, CF::UWM, CF::UWN>, Tile4<T, CF::UWM, CF::UWN>>::type;
  static_assert(NK == 1 || CF::FULL, "a paired (rank-2NB) update takes two full panels");
  constexpr int USR = UT::SR, USC = UT::SC, KSTEPS = NB / M::KS, PF = CF::PF, KV = M::KV;
  static_assert(KSTEPS % PF == 0, "the prefetch ring continues across the two panels");
  const unsigned lid = xcd_linear();
  const int blk = lid / gridDim.x, bx = lid - (lid / gridDim.x) * gridDim.x;
  if (inactive(a, blk)) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, n = a.n;
  const int jb = CF::FULL ? NK * NB : min(NB, n - j0);
  const int ncols = min((n - j0 - jb) + n, col_hi);
  const int rb = bx / ncb, cbk = bx - (bx / ncb) * ncb;
  const int wr = wave & 1, wc = wave >> 1;
  const int i0 = row_lo + rb * CF::WGM + wr * CF::UWM;
  const int c0 = col_lo + cbk * CF::WGN + wc * CF::UWN;
  if (i0 >= row_hi || c0 >= ncols) return;
  C* A = a.A + (size_t)blk * n * n;
  C* B = a.B + (size_t)blk * n * n;
  const C* MT = mt0 + (size_t)blk * mt_bs;      // multipliers, k-major with row stride n
  const ptrdiff_t mt_delta = mt1 - mt0;         // to the second panel's (paired update; uniform)
  // Every load below is unconditional from a clamped, in-bounds address, so
  // the loads carry no branches and are issued ahead of the matrix-core work.
  // Lanes of rows or columns that are not stored read finite data that never
  // reaches an output; panel rows k >= jb (ragged last panel) multiply the
  // rows of MT that the multiplier copy wrote as zeros.
  C* cb[USC];
  bool cok[USC];
#pragma unroll
  for (int y = 0; y < USC; ++y) {
    const int col = c0 + y * M::TN + M::b_col(lane);
    cok[y] = col < ncols;
    cb[y] = colptr(A, B, n, j0, jb, cok[y] ? col : 0);
  }
  UT acc;
  if (CF::FIRST) {
    // first panel: C comes from Gamma (A = 1 - s Gamma diag(X), B = Gamma)
    ColSrc<T> src[USC];
#pragma unroll
    for (int y = 0; y < USC; ++y)
      src[y] = colsrc<T, true>(a, blk, 0, jb, cok[y] ? c0 + y * M::TN + M::b_col(lane) : 0);
    acc.load_c([&](int r, int c) -> C { return src[c / M::TN].at(min(i0 + r, n - 1), n, 0); });
  } else {
    acc.load_c([&](int r, int c) -> C { return ld_c<CF::NT>(&cb[c / M::TN][(size_t)min(i0 + r, n - 1) * n]); });
  }
  const int kb = M::b_k(lane), ka = M::a_k(lane);
  const C* bbase[USC];
#pragma unroll
  for (int y = 0; y < USC; ++y) bbase[y] = cb[y] + (size_t)(j0 + (CF::FULL ? kb : 0)) * n;
  const C* abase[USR];
#pragma unroll
  for (int xx = 0; xx < USR; ++xx) abase[xx] = MT + (size_t)ka * n + min(i0 + xx * M::TM + M::a_row(lane), n - 1);
  // each lane takes KV consecutive k per step (1 for the FP32 / FP64 products);
  // panel h of a paired update: rows NB h .. of the pivot-row operand, the
  // multipliers from the second buffer
  auto fetch = [&](int h, int ks, C (&av)[USR][KV], C (&bv)[USC][KV]) {
#pragma unroll
    for (int i = 0; i < KV; ++i) {
      if (CF::FULL) {
#pragma unroll
        for (int y = 0; y < USC; ++y) bv[y][i] = bbase[y][(size_t)(h * NB + ks * M::KS + i) * n];
      } else {
        const int kk = min(ks * M::KS + kb + i, jb - 1);
#pragma unroll
        for (int y = 0; y < USC; ++y) bv[y][i] = bbase[y][(size_t)kk * n];
      }
      const ptrdiff_t ho = h ? mt_delta : 0;
#pragma unroll
      for (int xx = 0; xx < USR; ++xx) av[xx][i] = abase[xx][(ptrdiff_t)(ks * M::KS + i) * n + ho];
    }
  };
  C av[PF][USR][KV], bv[PF][USC][KV];
#pragma unroll
  for (int s = 0; s < PF; ++s) fetch(0, s, av[s], bv[s]);
#pragma unroll
  for (int h = 0; h < NK; ++h) {
#pragma unroll
    for (int ks = 0; ks < KSTEPS; ++ks) {
      const int cur = ks % PF;
      C ca[USR][KV], cbv[USC][KV];
#pragma unroll
      for (int xx = 0; xx < USR; ++xx)
#pragma unroll
        for (int i = 0; i < KV; ++i) ca[xx][i] = av[cur][xx][i];
#pragma unroll
      for (int y = 0; y < USC; ++y)
#pragma unroll
        for (int i = 0; i < KV; ++i) cbv[y][i] = bv[cur][y][i];
      if (ks + PF < KSTEPS)
        fetch(h, ks + PF, av[cur], bv[cur]);
      else if (h + 1 < NK)
        fetch(h + 1, ks + PF - KSTEPS, av[cur], bv[cur]);
      __builtin_amdgcn_sched_barrier(0);     // keep the prefetch ahead of this step's MFMAs
      acc.mac(ca, cbv);
    }
  }
  // wave-uniform (mix_lo is a multiple of the workgroup tile height)
  if (i0 >= mix_lo) {
    const int ncolA = n - j0 - jb;                 // B column = combined column - ncolA
    const C* G = a.gamma + (size_t)blk * n * n;
    C* P = a.phi + (size_t)blk * n * n;
    const T al = (T)a.alpha, be = (T)(1.0 - a.alpha);
    const bool mix = a.alpha != 1.0;
    // complex64: |F_ij|^2 of the finished rows summed per lane (each lane holds
    // one column of each 32-column tile y of the wave's 64 x 64 tile; i0 is a
    // multiple of 64)
    float cs[USC];
#pragma unroll
    for (int y = 0; y < USC; ++y) cs[y] = 0.f;
    acc.store_c([&](int r, int c, C v) {
      const int i = i0 + r;
      const int y = c / M::TN;
      if (cok[y] && i < row_hi) {
        st_c<CF::NT>(&cb[y][(size_t)i * n], v);
        const size_t e = (size_t)i * n + (c0 + c - ncolA);
        P[e] = mix_phi<T>(v, ld_c<true>(&G[e]), mix ? ld_c<true>(&P[e]) : cz<C>(), al, be, mix);
        if constexpr (sizeof(T) == 4) cs[y] += (float)v.x * v.x + (float)v.y * v.y;
      }
    });
    if constexpr (sizeof(T) == 4) {
      if (a.pcs) {
#pragma unroll
        for (int y = 0; y < USC; ++y) put_cs(a.pcs, n, blk, i0 / 64, c0 + y * M::TN + M::b_col(lane) - ncolA, cs[y]);
      }
    }
    return;
  }
  C* MN = mtn + (size_t)blk * NB * n;
  acc.store_c([&](int r, int c, C v) {
    const int i = i0 + r;
    const int y = c / M::TN;
    const bool mult = c0 + c < ntc && i >= mult_row;
    if (cok[y] && i < row_hi && !mult) st_c<CF::NT>(&cb[y][(size_t)i * n], v);
    if (mult && i < row_hi) MN[(size_t)(c0 + c) * n + i] = v;
  });
}

// ------------------------------------------------------ BF16x3 update
// The update above, C -= sum_k MT[k][i] R[k][col], on the bf16 matrix cores
// (v_mfma_f32_32x32x16_bf16, FP32 accumulation) for complex64 operands. Each
// complex product takes four real products,
//   Re C += (-ar) br + ai bi,   Im C += (-ar) bi + (-ai) br,
// and each real product x y the bf16 splits x = xh + xl + O(2^-18 |x|)
// (xh = bf16(x), xl = bf16(x - xh), round to nearest) as xh yh + xh yl + xl yh.
// A workgroup owns a 128 x 128 tile (2 x 2 waves of 64 x 64, two 32 x 32
// accumulator pairs per wave row and column). Per 16-deep step its 256 threads
// load the 128 x 16 slabs of both operands once (thread t: row or column
// t % 128, the eight k of half t / 128; each load instruction reads 64
// consecutive elements of one k row), split them and store the bf16 halves in
// LDS in the operand order of the instruction (lane l: row or column l % 32,
// k = 8 (l / 32) .. + 7, one 16-byte run per lane), double buffered with one
// barrier per step; each wave then reads an operand fragment with one 16-byte
// LDS load. The split is done once per workgroup, not once per wave. The next
// step's global loads are issued before this step's products. The store phase
// (mixing of finished rows, the next panel's multipliers) is that of the FP32
// kernel.
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// two values per conversion; the hi parts are read back from the packed pair
// (a bf16 is the upper half of the float it rounds to)
__device__ inline void split8(const float (&v)[8], bf16x8& hi, bf16x8& lo) {
  u32x4 h, l;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const f32x2 x = {v[2 * e], v[2 * e + 1]};
    const unsigned p = __builtin_bit_cast(unsigned, __builtin_convertvector(x, bf16x2));
    const f32x2 b = {__builtin_bit_cast(float, p << 16), __builtin_bit_cast(float, p & 0xffff0000u)};
    h[e] = p;
    l[e] = __builtin_bit_cast(unsigned, __builtin_convertvector(x - b, bf16x2));
  }
  hi = __builtin_bit_cast(bf16x8, h);
  lo = __builtin_bit_cast(bf16x8, l);
}

__device__ inline bf16x8 neg8(bf16x8 x) {       // exact: sign bits only
  u32x4 u = __builtin_bit_cast(u32x4, x);
  u ^= 0x80008000u;
  return __builtin_bit_cast(bf16x8, u);
}

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

__device__ inline void split4(const float (&v)[4], bf16x4& hi, bf16x4& lo) {
  unsigned h[2], l[2];
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const f32x2 x = {v[2 * e], v[2 * e + 1]};
    const unsigned p = __builtin_bit_cast(unsigned, __builtin_convertvector(x, bf16x2));
    const f32x2 b = {__builtin_bit_cast(float, p << 16), __builtin_bit_cast(float, p & 0xffff0000u)};
    h[e] = p;
    l[e] = __builtin_bit_cast(unsigned, __builtin_convertvector(x - b, bf16x2));
  }
  typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
  hi = __builtin_bit_cast(bf16x4, u32x2{h[0], h[1]});
  lo = __builtin_bit_cast(bf16x4, u32x2{l[0], l[1]});
}

// WN: 32-column groups per wave (wave tile 64 x 32 WN, workgroup tile
// 128 x 64 WN); PFD: operand loads in flight, in steps (a register ring).
// The narrow tile (WN = 1) also spreads the loads of its C tile over the
// steps: its accumulators start at zero and C is added when they are stored,
// so a workgroup does not begin with a burst of C loads that every workgroup
// of the launch makes at the same time (the C stream runs beside the matrix
// products instead of between them).
template <int NB, int NK, bool FIRST, int WN, int PFD>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2)))
void bse_update_bf_kernel(BseCtx<float> a, int j0, int ncb, int row_lo, int row_hi, int col_lo, int col_hi,
                          const float2* mt0, const float2* mt1, size_t mt_bs, float2* mtn, int ntc, int mix_lo,
                          int mult_row) {
  using C = float2;
  using M = MmaBF3;
  constexpr int WR = 128, WC = 64 * WN, SPP = NB / M::KS, KSTEPS = NK * SPP;
  constexpr int KP = M::KS * WC / kThreads;      // k values of one pivot-row column per thread (8 or 4)
  static_assert(NB % M::KS == 0 && kThreads == 2 * WR && (WN == 1 || WN == 2), "staging layout");
  // [buffer][component][32-row / column group][lane]; components: multipliers
  // -Re hi, lo, Im hi, lo; pivot rows Re hi, lo, Im hi, lo
  __shared__ bf16x8 sa[2][4][4][64];
  __shared__ bf16x8 sb[2][4][2 * WN][64];
  const unsigned lid = xcd_linear();
  const int blk = lid / gridDim.x, bx = lid - (lid / gridDim.x) * gridDim.x;
  if (inactive(a, blk)) return;                  // uniform over the workgroup
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, n = a.n;
  constexpr int jb = NK * NB;
  const int ncols = min((n - j0 - jb) + n, col_hi);
  const int rb = bx / ncb, cbk = bx - (bx / ncb) * ncb;
  const int R0 = row_lo + rb * WR, C0 = col_lo + cbk * WC;
  const int wr = wave & 1, wc = wave >> 1;
  const int i0 = R0 + wr * 64, c0 = C0 + wc * 32 * WN;
  // every wave takes part in the staging and the barriers; a wave whose tile
  // lies outside the rows or columns skips only its products and stores
  const bool live = i0 < row_hi && c0 < ncols;
  C* A = a.A + (size_t)blk * n * n;
  C* B = a.B + (size_t)blk * n * n;
  // staging: multiplier row sr (k half kh, 8 k) and pivot-row column sc (k
  // part kp, KP k) of the workgroup tile; clamped, in-bounds addresses (rows
  // past n and columns past ncols load finite data that reaches no output)
  const int sr = t & (WR - 1), kh = t >> 7;
  const int sc = t % WC, kp = t / WC;
  const ptrdiff_t mt_delta = mt1 - mt0;          // to the second panel's multipliers (uniform)
  const C* pa = mt0 + (size_t)blk * mt_bs + (size_t)(8 * kh) * n + min(R0 + sr, n - 1);
  const C* pb = colptr(A, B, n, j0, jb, C0 + sc < ncols ? C0 + sc : 0) + (size_t)(j0 + KP * kp) * n;
  const int ga = sr >> 5, la = (sr & 31) + 32 * kh;
  const int gb = sc >> 5, lb = (sc & 31) + 32 * ((KP * kp) >> 3), hb = ((KP * kp) & 7) / 4;
  C ra[PFD][8], rv[PFD][KP];
  auto load = [&](int s) {
    const int h = s / SPP, ks = s - h * SPP, r = s % PFD;
    const C* p = pa + (h ? mt_delta : 0) + (size_t)(ks * M::KS) * n;
    const C* q = pb + (size_t)(s * M::KS) * n;   // the paired panels' pivot rows are adjacent
#pragma unroll
    for (int e = 0; e < 8; ++e) ra[r][e] = p[(size_t)e * n];
#pragma unroll
    for (int e = 0; e < KP; ++e) rv[r][e] = q[(size_t)e * n];
  };
  auto commit = [&](int s, int buf) {
    const int r = s % PFD;
    {
      float v[8];
      bf16x8 h, l;
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = -ra[r][e].x;
      split8(v, h, l);
      sa[buf][0][ga][la] = h;
      sa[buf][1][ga][la] = l;
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = ra[r][e].y;
      split8(v, h, l);
      sa[buf][2][ga][la] = h;
      sa[buf][3][ga][la] = l;
    }
    if constexpr (KP == 8) {
      float v[8];
      bf16x8 h, l;
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = rv[r][e].x;
      split8(v, h, l);
      sb[buf][0][gb][lb] = h;
      sb[buf][1][gb][lb] = l;
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = rv[r][e].y;
      split8(v, h, l);
      sb[buf][2][gb][lb] = h;
      sb[buf][3][gb][lb] = l;
    } else {
      float v[4];
      bf16x4 h, l;
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] = rv[r][e].x;
      split4(v, h, l);
      reinterpret_cast<bf16x4*>(&sb[buf][0][gb][lb])[hb] = h;
      reinterpret_cast<bf16x4*>(&sb[buf][1][gb][lb])[hb] = l;
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] = rv[r][e].y;
      split4(v, h, l);
      reinterpret_cast<bf16x4*>(&sb[buf][2][gb][lb])[hb] = h;
      reinterpret_cast<bf16x4*>(&sb[buf][3][gb][lb])[hb] = l;
    }
  };
#pragma unroll
  for (int q = 0; q < PFD && q < KSTEPS; ++q) load(q);
  // the C tile (accumulators start at C; Gamma-formed for the first panel)
  C* cb[WN];
  bool cok[WN];
#pragma unroll
  for (int y = 0; y < WN; ++y) {
    const int col = c0 + y * 32 + (lane & 31);
    cok[y] = col < ncols;
    cb[y] = colptr(A, B, n, j0, jb, cok[y] ? col : 0);
  }
  floatx16 re[2][WN], im[2][WN];
  constexpr bool CSPREAD = WN == 1;
  constexpr int NCL = 2 * WN * 16;               // C elements per lane
  constexpr int CPS = (NCL + KSTEPS - 2) / (KSTEPS - 1);   // spread over all steps but the last
  static_assert(KSTEPS >= 2, "a spread C tile needs two steps");
  // first panel: C is formed from Gamma (ColSrc); the spread loads keep only
  // the Gamma column pointer live, the rest of the formula is rebuilt where
  // the elements are stored
  auto first_src = [&](int y) { return colsrc<float, true>(a, blk, 0, jb, cok[y] ? c0 + y * 32 + (lane & 31) : 0); };
  const C* gp[WN];
  if (FIRST) {
#pragma unroll
    for (int y = 0; y < WN; ++y) gp[y] = first_src(y).p;
  }
  // element e of this lane's part of the C tile: x = e / (16 WN), y = e / 16 % WN, v = e % 16
  auto c_row_of = [&](int e) { return min(i0 + (e / (16 * WN)) * 32 + M::c_row(lane, e % 16), n - 1); };
  auto c_ptr = [&](int e) -> const C* {
    const int y = e / 16 % WN;
    return FIRST ? gp[y] + (size_t)c_row_of(e) * n : &cb[y][(size_t)c_row_of(e) * n];
  };
  C cpre[CSPREAD ? NCL : 1];
  if constexpr (CSPREAD) {
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < WN; ++y)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          re[x][y][v] = 0.f;
          im[x][y][v] = 0.f;
        }
  } else if (FIRST) {
    ColSrc<float> src[WN];
#pragma unroll
    for (int y = 0; y < WN; ++y) src[y] = first_src(y);
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < WN; ++y)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const C c = src[y].at(min(i0 + x * 32 + M::c_row(lane, v), n - 1), n, 0);
          re[x][y][v] = c.x;
          im[x][y][v] = c.y;
        }
  } else {
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < WN; ++y)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const C c = ld_c<true>(&cb[y][(size_t)min(i0 + x * 32 + M::c_row(lane, v), n - 1) * n]);
          re[x][y][v] = c.x;
          im[x][y][v] = c.y;
        }
  }
  commit(0, 0);
  if (PFD < KSTEPS) load(PFD);
  __syncthreads();
  // One step is one basic block: the products of step s (every wave, also one
  // outside the rows or columns: clamped data, results never stored), the
  // split and LDS stores of step s + 1 and the loads of step s + 1 + PFD, so
  // that the scheduler can interleave the split (VALU) with the matrix-core
  // products of the same wave instead of running them one after the other.
#pragma unroll
  for (int s = 0; s < KSTEPS; ++s) {
    const int buf = s & 1;
    if constexpr (CSPREAD) {
#pragma unroll
      for (int e = s * CPS; e < (s + 1) * CPS && e < NCL; ++e) cpre[e] = ld_c<true>(c_ptr(e));
    }
    bf16x8 fa[2][6], fb[WN][4];
#pragma unroll
    for (int x = 0; x < 2; ++x) {
#pragma unroll
      for (int c = 0; c < 4; ++c) fa[x][c] = sa[buf][c][2 * wr + x][lane];
      fa[x][4] = neg8(fa[x][2]);
      fa[x][5] = neg8(fa[x][3]);
    }
#pragma unroll
    for (int y = 0; y < WN; ++y)
#pragma unroll
      for (int c = 0; c < 4; ++c) fb[y][c] = sb[buf][c][WN * wc + y][lane];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < WN; ++y) {
        const bf16x8 &ph = fa[x][0], &pl = fa[x][1], &qh = fa[x][2], &ql = fa[x][3], &nqh = fa[x][4],
                     &nql = fa[x][5];
        const bf16x8 &bh = fb[y][0], &bl = fb[y][1], &ih = fb[y][2], &il = fb[y][3];
        re[x][y] = M::mma(pl, bh, re[x][y]);
        re[x][y] = M::mma(ph, bl, re[x][y]);
        re[x][y] = M::mma(ql, ih, re[x][y]);
        re[x][y] = M::mma(qh, il, re[x][y]);
        re[x][y] = M::mma(ph, bh, re[x][y]);
        re[x][y] = M::mma(qh, ih, re[x][y]);
        im[x][y] = M::mma(pl, ih, im[x][y]);
        im[x][y] = M::mma(ph, il, im[x][y]);
        im[x][y] = M::mma(nql, bh, im[x][y]);
        im[x][y] = M::mma(nqh, bl, im[x][y]);
        im[x][y] = M::mma(ph, ih, im[x][y]);
        im[x][y] = M::mma(nqh, bh, im[x][y]);
      }
    if (s + 1 < KSTEPS) {
      commit(s + 1, buf ^ 1);     // its readers (step s - 1) passed the last barrier
      if (s + 1 + PFD < KSTEPS) load(s + 1 + PFD);
      __syncthreads();
    }
  }
  if (!live) return;
  if (FIRST && CSPREAD) {           // the store pointers, not kept through the loop
#pragma unroll
    for (int y = 0; y < WN; ++y) {
      const int col = c0 + y * 32 + (lane & 31);
      cb[y] = colptr(A, B, n, j0, jb, cok[y] ? col : 0);
      asm volatile("" : "+v"(cb[y]));
    }
  }
  ColSrc<float> fsrc[WN];
  int i0e = i0;                     // row origin for the epilogue: the row indices are
  if (FIRST && CSPREAD) {           // recomputed there, not kept through the loop
    asm volatile("" : "+v"(i0e));
#pragma unroll
    for (int y = 0; y < WN; ++y) fsrc[y] = first_src(y);
  }
  auto elem = [&](int x, int y, int v) {
    C r = make_float2(re[x][y][v], im[x][y][v]);
    if constexpr (CSPREAD) {                     // C + (-MT^T R)
      const int e = (x * WN + y) * 16 + v;
      const C c = FIRST ? fsrc[y].form(cpre[e], min(i0e + x * 32 + M::c_row(lane, v), n - 1), 0) : cpre[e];
      r.x = c.x + r.x;
      r.y = c.y + r.y;
    }
    return r;
  };
  if (i0 >= mix_lo) {                            // wave-uniform, as in the FP32 kernel
    const int ncolA = n - j0 - jb;
    const C* G = a.gamma + (size_t)blk * n * n;
    C* P = a.phi + (size_t)blk * n * n;
    const float al = (float)a.alpha, be = (float)(1.0 - a.alpha);
    const bool mix = a.alpha != 1.0;
    float cs[WN];
#pragma unroll
    for (int y = 0; y < WN; ++y) cs[y] = 0.f;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < WN; ++y)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int i = i0 + x * 32 + M::c_row(lane, v);
          if (cok[y] && i < row_hi) {
            const C f = elem(x, y, v);
            st_c<true>(&cb[y][(size_t)i * n], f);
            const size_t e = (size_t)i * n + (c0 + y * 32 + (lane & 31) - ncolA);
            P[e] = mix_phi<float>(f, ld_c<true>(&G[e]), mix ? ld_c<true>(&P[e]) : cz<C>(), al, be, mix);
            cs[y] += f.x * f.x + f.y * f.y;
          }
        }
    if (a.pcs) {
#pragma unroll
      for (int y = 0; y < WN; ++y) put_cs(a.pcs, n, blk, i0 / 64, c0 + y * 32 + (lane & 31) - ncolA, cs[y]);
    }
    return;
  }
  C* MN = mtn + (size_t)blk * NB * n;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < WN; ++y)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int i = i0 + x * 32 + M::c_row(lane, v), c = c0 + y * 32 + (lane & 31);
        const bool mult = c < ntc && i >= mult_row;
        if (cok[y] && i < row_hi && !mult) st_c<true>(&cb[y][(size_t)i * n], elem(x, y, v));
        if (mult && i < row_hi) MN[(size_t)c * n + i] = elem(x, y, v);
      }
}

// ------------------------------------------------- BF16x3 pivot-row step
// The pivot rows R_JK = P A_JK of a full panel (every column right of it in A
// and every column of B) with the products of bse_update_bf_kernel: the
// multiplier operand is P (transposed, k-major with row stride NB), the other
// the panel rows of the column tile (for the first panel A = 1 - s Gamma
// diag(X) formed from Gamma as it is staged), the accumulators start at zero.
// A workgroup owns the 128 panel rows x 128 combined columns (2 x 2 waves of
// 64 x 64). The rows are overwritten in place (every wave has passed the last
// step's barrier, after the staging of the last panel rows, before any
// store); the A part also goes transposed below the diagonal block (the U copy
// the back substitution reads), and the last panel's rows are mixed into Phi
// with their column sums, as in bse_panel_kernel.
template <int NB, bool FIRST>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2)))
void bse_panel_bf_kernel(BseCtx<float> a, int j0, int mix) {
  using C = float2;
  using M = MmaBF3;
  constexpr int W = 128, KSTEPS = NB / M::KS;
  static_assert(NB == W && kThreads == 2 * W, "one workgroup covers the panel rows");
  __shared__ bf16x8 sa[2][4][4][64];
  __shared__ bf16x8 sb[2][4][4][64];
  const unsigned lid = xcd_linear();
  const int blk = lid / gridDim.x, bx = lid - (lid / gridDim.x) * gridDim.x;
  if (inactive(a, blk)) return;                  // uniform over the workgroup
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, n = a.n;
  constexpr int jb = NB;
  const int ncolA = n - j0 - jb, ncols = ncolA + n;
  const int C0 = bx * W;
  const int wr = wave & 1, wc = wave >> 1;
  const int i0 = wr * 64, c0 = C0 + wc * 64;     // panel row, combined column of the wave tile
  const bool live = c0 < ncols;
  C* A = a.A + (size_t)blk * n * n;
  C* B = a.B + (size_t)blk * n * n;
  // staging: row sr of P^T's k slab (k half kh) and combined column sr of the
  // panel rows (clamped: columns past ncols stage finite data no output uses)
  const int sr = t & (W - 1), kh = t >> 7;
  const C* pa = a.PI + (size_t)blk * NB * NB + (size_t)(8 * kh) * NB + sr;
  const int scol = C0 + sr < ncols ? C0 + sr : 0;
  const ColSrc<float> src = colsrc<float, FIRST>(a, blk, j0, jb, scol);
  const C* pb = src.p + (size_t)(8 * kh) * n;
  const int grp = sr >> 5, slot = (sr & 31) + 32 * kh;
  C ra[8], rv[8];
  auto load = [&](int s) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      ra[e] = pa[(size_t)(s * M::KS + e) * NB];
      rv[e] = pb[(size_t)(s * M::KS + e) * n];
    }
  };
  auto commit = [&](int s, int buf) {
    float v[8];
    bf16x8 h, l;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = -ra[e].x;
    split8(v, h, l);
    sa[buf][0][grp][slot] = h;
    sa[buf][1][grp][slot] = l;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = ra[e].y;
    split8(v, h, l);
    sa[buf][2][grp][slot] = h;
    sa[buf][3][grp][slot] = l;
    C b[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) b[e] = FIRST ? src.form(rv[e], s * M::KS + 8 * kh + e, j0) : rv[e];
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = b[e].x;
    split8(v, h, l);
    sb[buf][0][grp][slot] = h;
    sb[buf][1][grp][slot] = l;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = b[e].y;
    split8(v, h, l);
    sb[buf][2][grp][slot] = h;
    sb[buf][3][grp][slot] = l;
  };
  floatx16 re[2][2], im[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        re[x][y][v] = 0.f;
        im[x][y][v] = 0.f;
      }
  load(0);
  commit(0, 0);
  load(1);
  __syncthreads();
#pragma unroll
  for (int s = 0; s < KSTEPS; ++s) {
    const int buf = s & 1;
    bf16x8 fa[2][6], fb[2][4];
#pragma unroll
    for (int x = 0; x < 2; ++x) {
#pragma unroll
      for (int c = 0; c < 4; ++c) fa[x][c] = sa[buf][c][2 * wr + x][lane];
      fa[x][4] = neg8(fa[x][2]);
      fa[x][5] = neg8(fa[x][3]);
    }
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int c = 0; c < 4; ++c) fb[y][c] = sb[buf][c][2 * wc + y][lane];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        const bf16x8 &ph = fa[x][0], &pl = fa[x][1], &qh = fa[x][2], &ql = fa[x][3], &nqh = fa[x][4],
                     &nql = fa[x][5];
        const bf16x8 &bh = fb[y][0], &bl = fb[y][1], &ih = fb[y][2], &il = fb[y][3];
        re[x][y] = M::mma(pl, bh, re[x][y]);
        re[x][y] = M::mma(ph, bl, re[x][y]);
        re[x][y] = M::mma(ql, ih, re[x][y]);
        re[x][y] = M::mma(qh, il, re[x][y]);
        re[x][y] = M::mma(ph, bh, re[x][y]);
        re[x][y] = M::mma(qh, ih, re[x][y]);
        im[x][y] = M::mma(pl, ih, im[x][y]);
        im[x][y] = M::mma(ph, il, im[x][y]);
        im[x][y] = M::mma(nql, bh, im[x][y]);
        im[x][y] = M::mma(nqh, bl, im[x][y]);
        im[x][y] = M::mma(ph, ih, im[x][y]);
        im[x][y] = M::mma(nqh, bh, im[x][y]);
      }
    if (s + 1 < KSTEPS) {
      commit(s + 1, buf ^ 1);
      if (s + 2 < KSTEPS) load(s + 2);
      __syncthreads();
    }
  }
  if (!live) return;
  // the products accumulated -(P A): R is their negative
  const bool mixes = mix && c0 >= ncolA;         // wave-uniform: the last panel has no A columns
  const float al = (float)a.alpha, be = (float)(1.0 - a.alpha);
  const bool m = a.alpha != 1.0;
  float cs[2] = {0.f, 0.f};
#pragma unroll
  for (int y = 0; y < 2; ++y) {
    const int col = c0 + y * 32 + (lane & 31);
    if (col >= ncols) continue;
    C* cp = colptr(A, B, n, j0, jb, col);
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int r = i0 + x * 32 + M::c_row(lane, v);
        const C val = make_float2(-re[x][y][v], -im[x][y][v]);
        cp[(size_t)(j0 + r) * n] = val;
        if (col < ncolA) A[(size_t)(j0 + jb + col) * n + j0 + r] = val;
        if (mixes) {
          const size_t e = (size_t)blk * n * n + (size_t)(j0 + r) * n + (col - ncolA);
          a.phi[e] = mix_phi<float>(val, a.gamma[e], m ? a.phi[e] : cz<C>(), al, be, m);
          cs[y] += val.x * val.x + val.y * val.y;
        }
      }
  }
  if (mixes && a.pcs) {
#pragma unroll
    for (int y = 0; y < 2; ++y) put_cs(a.pcs, n, blk, (j0 + i0) / 64, c0 + y * 32 + (lane & 31) - ncolA, cs[y]);
  }
}

// rows [row_lo, row_hi) with 0 <= row_lo < row_hi <= n, outside the panel;
// combined columns [col_lo, ncols) with col_lo <= n - j0 - jb; multipliers from
// mt (k-major [NB][n] per block) or, ut (back substitution of a full panel),
// from the transposed copy in A's rows J0 .. J0 + NB; the results of the first
// ntc <= min(NB, n - j0 - jb) combined columns also go transposed into mtn
// (forward step: the next panel's multipliers)
template <typename T, int NB, class CF, int NK = 1>
void launch_update(const BseCtx<T>& a, int n, int Nq, int j0, int row_lo, int row_hi, int col_lo, bool ut,
                   typename cplx_of<T>::type* mt, typename cplx_of<T>::type* mtn, int ntc, hipStream_t s,
                   int mix_lo = -1, int mult_row = -1, int col_hi = -1,
                   const typename cplx_of<T>::type* mt1 = nullptr) {
  const auto* mt0 = ut ? a.A + (size_t)j0 * n : mt;
  const size_t mt_bs = ut ? (size_t)n * n : (size_t)NB * n;
  const int jb = std::min(NK * NB, n - j0);
  const int ncols_all = (n - j0 - jb) + n;
  const int ncols = col_hi < 0 ? ncols_all : std::min(col_hi, ncols_all);
  const int nrb = (row_hi - row_lo + CF::WGM - 1) / CF::WGM;
  const int ncb = (ncols - col_lo + CF::WGN - 1) / CF::WGN;
  if constexpr (CF::BF3) {
    static_assert(sizeof(T) == 4 && CF::FULL && CF::UWM == 64 && (CF::UWN == 64 || CF::UWN == 32), "BF16x3 tile");
    hipLaunchKernelGGL((bse_update_bf_kernel<NB, NK, CF::FIRST, CF::UWN / 32, CF::PF>), dim3(nrb * ncb, Nq),
                       dim3(kThreads), 0, s, a, j0,
                       ncb, row_lo, row_hi, col_lo, ncols, mt0, mt1 ? mt1 : mt0, mt_bs, mtn ? mtn : mt,
                       mtn ? ntc : 0, mix_lo < 0 ? n : mix_lo, mult_row < 0 ? row_lo + ntc : mult_row);
  } else {
    hipLaunchKernelGGL((bse_update_kernel<T, NB, CF, NK>), dim3(nrb * ncb, Nq), dim3(kThreads), 0, s, a, j0, ncb,
                       row_lo, row_hi, col_lo, ncols, mt0, mt1 ? mt1 : mt0, mt_bs, mtn ? mtn : mt, mtn ? ntc : 0,
                       mix_lo < 0 ? n : mix_lo, mult_row < 0 ? row_lo + ntc : mult_row);
  }
}

// Per-block statistics (after the error estimate and the FP64 re-solve have
// marked their blocks).
template <typename T>
__global__ __launch_bounds__(kThreads) void bse_stats_kernel(BseCtx<T> a) {
  const int blk = blockIdx.x * blockDim.x + threadIdx.x;
  if (blk >= a.Nq || inactive(a, blk) || !a.stats) return;
  const double* ps = a.pst + (size_t)blk * kPst;
  pq_bse_block_stats st;
  const double ratio = ps[1] > 0.0 ? ps[0] / ps[1] : 0.0;
  const bool weak = ratio < a.weak_ratio || ps[4] > a.kappa_max;
  const bool nonfin = ps[2] > 0.0;
  st.min_pivot = (float)ratio;
  st.growth = (float)ps[4];
  if constexpr (sizeof(T) == 4) {
    const bool probe = ps[6] > 0.0;
    const bool nonfin_est = !(ps[5] <= DBL_MAX);
    st.flags = ((weak || nonfin || probe) ? 1 : 0) | ((nonfin || nonfin_est) ? 2 : 0) | (ps[3] > 0.0 ? 4 : 0) |
               (ps[7] > 0.0 ? 8 : 0) | (probe ? 16 : 0);
    st.err_est = (float)ps[5];
  } else {
    // complex128: weak pivots are only reported; a non-finite block has no
    // more precise path to fall back on
    st.flags = (weak ? 1 : 0) | (nonfin ? 2 | 8 : 0);
    st.err_est = 0.f;
  }
  a.stats[blk] = st;
}

template <typename T>
constexpr int panel_width() { return sizeof(T) == 4 ? 128 : 64; }

// ------------------------------------------------------------ error estimate
// After the complex64 solve, B holds F^ = F + E. With A = 1 - s Gamma diag(X)
// and F = A^-1 Gamma, the inverse is A^-1 = 1 + s F diag(X), and
//   E = A^-1 R,   R = A F^ - Gamma   (the residual of the stored solution).
// The quantity estimated per block is the relative error |E|_F / |F|_F.
// R comes from rounding (the elimination's backward error and the complex64
// storage of F^): it is small, not amplified and without a preferred
// direction, so
//   |E|_F^2 = sum_k |u_k^H R|^2 / sigma_k^2 ~ |R|_F^2 |A^-1|_F^2 / n,
//   |A^-1|_F^2 = n + 2 s Re tr(F X) + |F X|_F^2,
// and |R|_F is sampled through two probe vectors v_p (entries (+-1 +- i)/sqrt(2)
// on a column sample S, from an integer hash of (column, probe); zero elsewhere):
//   y = F^ v,   r = A y - Gamma v = y - s Gamma (X y) - Gamma v = R v,
// evaluated in FP64 on the rows of the same sample, |R|_F^2 ~ (n/|S|)^2 |r_S|^2.
// |F^ X|_F and |F^|_F come from the kernels that mixed the rows (column sums),
// tr(F^ X) from the diagonal: no full pass over F^ or Gamma.
//   screen: est = (|A^-1|_F / n^1/2) (n / |S|) |r_S| / |F^|_F   (max over the probes)
// Where the screen exceeds tol / 2, or |A^-1|_F / n^1/2 exceeds 2 (near the
// instability the residual leans towards the amplified direction, and the
// isotropic screen can be low by a few times), the error of the probes
// themselves is evaluated (one pass over Gamma for r on every row, one over F^):
//   E v = A^-1 r = r + s F (X r) ~ r + s F^ (X r),
//   refined: est2 = max_p |E v_p| / |F^|_F  (8 probes on every column, |v_p|^2 = n,
//            so |E v_p|^2 averages |E|_F^2),
// and decides the flag (est2 > tol); otherwise the screen stands.
// S: every index for n <= 256, else two contiguous chunks of 64 at n/4 and 3n/4.
constexpr int kProbeRows = 4;      // rows per wave, loaded together
constexpr double kDefaultBseTol = 2e-5;
constexpr double kScreen = 2.0;    // margin of the sampled screen
constexpr double kAmp2 = 4.0;      // |A^-1|_F^2 / n above which the probes are evaluated exactly

__device__ inline int probe_ns(int n) { return n <= 256 ? n : 128; }
__device__ inline int probe_chunk(int n, int c) { return ((c == 0 ? n / 4 : (3 * n) / 4) - 32) & ~15; }
__device__ inline int probe_at(int n, int s) { return n <= 256 ? s : probe_chunk(n, s >> 6) + (s & 63); }
__device__ inline bool probe_in(int n, int j) {
  if (n <= 256) return true;
  const int a = probe_chunk(n, 0), b = probe_chunk(n, 1);
  return (j >= a && j < a + 64) || (j >= b && j < b + 64);
}

__device__ inline double2 probe_vec(int j, int p) {
  unsigned x = (unsigned)j * 8u + (unsigned)p + 0x9E3779B9u;
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  const double h = 0.70710678118654752440;
  return mk((x & 1u) ? -h : h, (x & 2u) ? -h : h);
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline void cfma(double2& acc, double2 a, double2 b) {
  acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
  acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
}

// Probe sets: the screen takes kNpScreen probes on the column sample of every
// block; the refined estimate kNpRefine probes on every column of the marked
// blocks (max over the probes: near the instability E is nearly of rank one,
// and one probe's |E v| / |E|_F fluctuates like an exponential variable).
constexpr int kNpScreen = 2, kNpRefine = 8;

template <bool REFINE> __device__ inline bool probe_col(int n, int j) { return REFINE || probe_in(n, j); }

// y_p = F^ v_p on every row. Screen: the sampled columns of every block;
// refined: every column of the blocks with pst[6] = 2. One wave per RPW rows,
// lanes across the columns; grid (ceil(n / (4 RPW)), Nq).
template <int NP, int RPW, bool REFINE>
__global__ __launch_bounds__(kThreads) void probe_y_kernel(const float2* F, int n, const double* pst, double2* y) {
  const int blk = blockIdx.y, lane = threadIdx.x & 63;
  if (REFINE && pst[(size_t)blk * kPst + 6] != 2.0) return;
  const int i0 = (blockIdx.x * kWaves + (threadIdx.x >> 6)) * RPW;
  if (i0 >= n) return;
  const float2* Fb = F + (size_t)blk * n * n;
  const int ns = REFINE ? n : probe_ns(n);
  double2 acc[RPW][NP];
#pragma unroll
  for (int r = 0; r < RPW; ++r)
#pragma unroll
    for (int p = 0; p < NP; ++p) acc[r][p] = mk(0.0, 0.0);
  for (int s = lane; s < ns; s += 64) {
    const int j = REFINE ? s : probe_at(n, s);
    double2 v[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) v[p] = probe_vec(j, p);
    float2 f[RPW];
#pragma unroll
    for (int r = 0; r < RPW; ++r) f[r] = Fb[(size_t)min(i0 + r, n - 1) * n + j];
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      const double2 fd = to_d(f[r]);
#pragma unroll
      for (int p = 0; p < NP; ++p) cfma(acc[r][p], fd, v[p]);
    }
  }
#pragma unroll
  for (int r = 0; r < RPW; ++r)
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const double2 sm = mk(wave_sum(acc[r][p].x), wave_sum(acc[r][p].y));
      if (lane == 0 && i0 + r < n) y[((size_t)blk * NP + p) * n + i0 + r] = sm;
    }
}

// r_p = y_p - s Gamma (X y_p) - Gamma v_p. Screen: on the rows of the sample
// (grid.x over the sample); refined: on every row of the marked blocks.
template <int NP, int RPW, bool REFINE>
__global__ __launch_bounds__(kThreads) void probe_r_kernel(const float2* G, const double2* chi0, const double2* y,
                                                          int n, double sign, const double* pst, double2* r) {
  const int blk = blockIdx.y, lane = threadIdx.x & 63;
  if (REFINE && pst[(size_t)blk * kPst + 6] != 2.0) return;
  const int nrows = REFINE ? n : probe_ns(n);
  const int s0 = (blockIdx.x * kWaves + (threadIdx.x >> 6)) * RPW;
  if (s0 >= nrows) return;
  int rows[RPW];
#pragma unroll
  for (int k = 0; k < RPW; ++k) {
    const int sk = min(s0 + k, nrows - 1);
    rows[k] = REFINE ? sk : probe_at(n, sk);
  }
  const float2* Gb = G + (size_t)blk * n * n;
  const double2* X = chi0 + (size_t)blk * n;
  const double2* yb = y + (size_t)blk * NP * n;
  double2 g[RPW][NP], h[RPW][NP];
#pragma unroll
  for (int k = 0; k < RPW; ++k)
#pragma unroll
    for (int p = 0; p < NP; ++p) g[k][p] = h[k][p] = mk(0.0, 0.0);
  for (int j = lane; j < n; j += 64) {
    const bool in = probe_col<REFINE>(n, j);
    const double2 x = X[j];
    double2 v[NP], z[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      v[p] = in ? probe_vec(j, p) : mk(0.0, 0.0);
      z[p] = cmul(x, yb[(size_t)p * n + j]);
    }
    float2 gv[RPW];
#pragma unroll
    for (int k = 0; k < RPW; ++k) gv[k] = Gb[(size_t)rows[k] * n + j];
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
      const double2 gd = to_d(gv[k]);
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        cfma(g[k][p], gd, v[p]);
        cfma(h[k][p], gd, z[p]);
      }
    }
  }
#pragma unroll
  for (int k = 0; k < RPW; ++k)
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const double2 sg = mk(wave_sum(g[k][p].x), wave_sum(g[k][p].y));
      const double2 sh = mk(wave_sum(h[k][p].x), wave_sum(h[k][p].y));
      const int i = rows[k];
      if (lane == 0 && s0 + k < nrows) {
        const double2 a = yb[(size_t)p * n + i];
        r[((size_t)blk * NP + p) * n + i] = mk(a.x - sign * sh.x - sg.x, a.y - sign * sh.y - sg.y);
      }
    }
}

__device__ inline double safe_ratio(double num2, double den2) {
  if (num2 == 0.0) return 0.0;
  return sqrt(num2 / den2);     // den2 = 0 with num2 > 0: +inf (flagged)
}

// Per block (one workgroup): the screen. Above tol / kScreen, or with |A^-1|_F
// amplifying, with a finite value: refined estimate pending (pst[6] = 2);
// non-finite: flagged (1).
__global__ __launch_bounds__(kThreads) void probe_est_kernel(const double2* r, const float* pcs, const float2* F,
                                                            const double2* chi0, int n, double sign, double tol,
                                                            double* pst) {
  __shared__ double red[kThreads];
  const int blk = blockIdx.x;
  const int ns = probe_ns(n);
  const int nr = (n + 63) / 64;
  double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};    // |r_0|^2, |r_1|^2, |F X|^2, |F|^2, Re tr(F X)
  for (int q = threadIdx.x; q < ns; q += blockDim.x) {
    const int i = probe_at(n, q);
    s[0] += cabs2(r[((size_t)blk * kNpScreen + 0) * n + i]);
    s[1] += cabs2(r[((size_t)blk * kNpScreen + 1) * n + i]);
  }
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    double c = 0.0;
    for (int rb = 0; rb < nr; ++rb) c += (double)pcs[((size_t)blk * nr + rb) * n + j];
    s[2] += c * cabs2(chi0[(size_t)blk * n + j]);
    s[3] += c;
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double2 f = to_d(F[(size_t)blk * n * n + (size_t)i * n + i]), x = chi0[(size_t)blk * n + i];
    s[4] += f.x * x.x - f.y * x.y;
  }
  for (int k = 0; k < 5; ++k) s[k] = block_sum(s[k], red);
  if (threadIdx.x == 0) {
    double* ps = pst + (size_t)blk * kPst;
    const double samp = (double)n / ns;
    const double amp2 = fmax(0.0, 1.0 + (2.0 * sign * s[4] + s[2]) / n);     // |A^-1|_F^2 / n
    double est = sqrt(amp2) * samp * sqrt(fmax(s[0], s[1])) / sqrt(s[3]);
    if (s[0] == 0.0 && s[1] == 0.0) est = s[3] == s[3] ? 0.0 : INFINITY;     // F = 0 exactly
    const bool fin = est <= DBL_MAX;          // false for NaN and +inf
    if (!fin) est = INFINITY;
    ps[5] = est;
    // the refined estimate also wherever A^-1 amplifies (|A^-1|_F / n^1/2 > 2):
    // there the rounding residual need not be isotropic (near the instability
    // it leans towards the amplified direction)
    ps[6] = !fin ? 1.0 : ((est > tol / kScreen || amp2 > kAmp2) ? 2.0 : 0.0);
    ps[8] = s[3];
  }
}

// c_p = r_p + s F^ (X r_p) = E v_p for the marked blocks; writes |c_p|^2 per row.
template <int NP>
__global__ __launch_bounds__(kThreads) void probe_c_kernel(const float2* F, const double2* chi0, const double2* r,
                                                          int n, double sign, const double* pst, double* cq) {
  const int blk = blockIdx.y, lane = threadIdx.x & 63;
  if (pst[(size_t)blk * kPst + 6] != 2.0) return;
  const int i = blockIdx.x * kWaves + (threadIdx.x >> 6);
  if (i >= n) return;
  const float2* Fb = F + (size_t)blk * n * n + (size_t)i * n;
  const double2* X = chi0 + (size_t)blk * n;
  const double2* rb = r + (size_t)blk * NP * n;
  double2 c[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) c[p] = mk(0.0, 0.0);
  for (int j = lane; j < n; j += 64) {
    const double2 x = X[j];
    const double2 fd = to_d(Fb[j]);
#pragma unroll
    for (int p = 0; p < NP; ++p) cfma(c[p], fd, cmul(x, rb[(size_t)p * n + j]));
  }
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const double2 sm = mk(wave_sum(c[p].x), wave_sum(c[p].y));
    if (lane == 0) {
      const double2 a = rb[(size_t)p * n + i];
      cq[((size_t)blk * n + i) * NP + p] = cabs2(mk(a.x + sign * sm.x, a.y + sign * sm.y));
    }
  }
}

// Per block: the refined estimate (max over the probes of (n |E v_p|^2)^1/2 /
// (|v_p| |F^|_F), |v_p|^2 = n) replaces the screen and decides the flag.
template <int NP>
__global__ __launch_bounds__(kThreads) void probe_flag_kernel(const double* cq, int n, double tol, double* pst) {
  __shared__ double red[kThreads];
  const int blk = blockIdx.x;
  double* ps = pst + (size_t)blk * kPst;
  if (ps[6] != 2.0) return;                   // uniform over the workgroup
  double mx = 0.0;
  for (int p = 0; p < NP; ++p) {
    double c = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) c += cq[((size_t)blk * n + i) * NP + p];
    mx = fmax(mx, block_sum(c, red));
  }
  if (threadIdx.x == 0) {
    double est = safe_ratio(mx, ps[8]);
    if (!(est <= DBL_MAX)) est = INFINITY;
    ps[5] = est;
    ps[6] = est > tol ? 1.0 : 0.0;
  }
}

// ------------------------------------------------------ FP64 re-solve
// Flagged blocks of a complex64 elimination are solved again in FP64 from
// Gamma, in S slots (list[0 .. S): block of each slot; list[S]: slots in use;
// list[S + 1]: slots of the first list). Two lists, both in q order:
//  - before any row is mixed (once the forward sweep has met every pivot):
//    the blocks with weak or non-finite pivots; their Phi is saved, and the
//    re-solved block is mixed from the FP64 F and the saved Phi;
//  - after the error estimate: the other blocks it flags; their Phi already
//    holds alpha (F^ - Gamma) + (1 - alpha) Phi_old, so the FP64 F enters as
//    Phi + alpha (F_64 - F^) (no saved copy needed; F^ is still in B).
// Flagged blocks beyond the slots keep the complex64 result and pst[7] = 1.
constexpr int kMaxBlocks = kBseMaxBlocks;   // blocks of one launch sequence (a batch: K Nq)

__device__ inline bool pivot_flagged(const double* ps, float weak, double kappa_max) {
  const double ratio = ps[1] > 0.0 ? ps[0] / ps[1] : 0.0;
  return ps[2] > 0.0 || ratio < weak || ps[4] > kappa_max;
}

__global__ __launch_bounds__(kThreads) void refine_list_kernel(double* pst, int Nq, float weak, double kappa_max,
                                                              int S, int late, int* list) {
  __shared__ unsigned char flag[kMaxBlocks];
  for (int b = threadIdx.x; b < Nq; b += blockDim.x) {
    double* ps = pst + (size_t)b * kPst;
    const bool piv = pivot_flagged(ps, weak, kappa_max);
    flag[b] = late ? (!piv && ps[6] == 1.0) : piv;
    if (!late) {
      ps[3] = 0.0;
      ps[7] = 0.0;
    }
  }
  __syncthreads();                  // (also orders the resets before the overflow marks below)
  if (threadIdx.x == 0) {           // ordered compaction from LDS
    int c = late ? list[S] : 0;
    for (int b = 0; b < Nq; ++b) {
      if (flag[b]) {
        if (c < S) list[c++] = b;
        else pst[(size_t)b * kPst + 7] = 1.0;
      }
    }
    list[S] = c;
    if (!late) list[S + 1] = c;
  }
}

// Gamma and X of the slots [lo, hi) into the complex128 slots (early list: also Phi).
__global__ __launch_bounds__(kThreads) void refine_gather_kernel(const float2* gamma, const double2* chi0,
                                                                  const float2* phi, int n, const int* list, int S,
                                                                  int late, double2* g64, double2* x64, float2* phis) {
  const int slot = blockIdx.y;
  const int lo = late ? list[S + 1] : 0, hi = list[S];
  if (slot < lo || slot >= hi) return;
  const int b = list[slot];
  const size_t nn = (size_t)n * n;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nn; i += (size_t)gridDim.x * blockDim.x) {
    const float2 v = gamma[(size_t)b * nn + i];
    g64[(size_t)slot * nn + i] = mk((double)v.x, (double)v.y);
    if (!late) phis[(size_t)slot * nn + i] = phi[(size_t)b * nn + i];   // Phi before this solve
  }
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < n; i += blockDim.x) x64[(size_t)slot * n + i] = chi0[(size_t)b * n + i];
}

// Phi of a re-solved block from the FP64 solution p64 = F_64 - Gamma:
//   first list:  alpha p64 + (1 - alpha) Phi_saved,
//   second list: Phi + alpha (p64 + Gamma - F^).
// A slot whose FP64 elimination met a non-finite pivot, or (second list) whose
// complex64 F^ is not finite, is left as it is and marked unresolved.
__global__ __launch_bounds__(kThreads) void refine_scatter_kernel(const double2* p64, const float2* phis,
                                                                   const double* pst64, const float2* gamma,
                                                                   const float2* fhat, int n, const int* list, int S,
                                                                   double alpha, float2* phi, double* pst) {
  const int slot = blockIdx.y;
  if (slot >= list[S]) return;
  const int b = list[slot];
  const bool early = slot < list[S + 1];
  double* ps = pst + (size_t)b * kPst;
  const bool ok = !(pst64[(size_t)slot * kPst + 2] > 0.0) && (early || ps[5] <= DBL_MAX);
  if (!ok) {
    if (blockIdx.x == 0 && threadIdx.x == 0) ps[7] = 1.0;
    return;
  }
  const size_t nn = (size_t)n * n;
  const bool mix = alpha != 1.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nn; i += (size_t)gridDim.x * blockDim.x) {
    double2 v = p64[(size_t)slot * nn + i];
    if (early) {
      if (mix) {
        const float2 o = phis[(size_t)slot * nn + i];
        v.x = alpha * v.x + (1.0 - alpha) * (double)o.x;
        v.y = alpha * v.y + (1.0 - alpha) * (double)o.y;
      }
    } else {
      const double2 cur = to_d(phi[(size_t)b * nn + i]);
      const double2 g = to_d(gamma[(size_t)b * nn + i]);
      const double2 f = to_d(fhat[(size_t)b * nn + i]);
      v.x = cur.x + alpha * (v.x + g.x - f.x);
      v.y = cur.y + alpha * (v.y + g.y - f.y);
    }
    phi[(size_t)b * nn + i] = mkf((float)v.x, (float)v.y);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) ps[3] = 1.0;
}

// Re-solve slots per channel: as many as kResolveBudget bytes hold (at least
// 8, at most Nq), or the caller's limit.
constexpr double kResolveBudget = 2.5 * 1024.0 * 1024.0 * 1024.0;

struct BseLayout {
  size_t A, B, MT, PI, pst;
  // complex64 path only: error estimate and FP64 re-solve of flagged blocks
  size_t py, pr, pcs, pcq;
  size_t list, g64, x64, p64, phis, ws64;
  int slots;
  size_t total;
};

template <typename T>
BseLayout bse_layout(const Dims& d, int slots_req = 0);

inline int resolve_slots(const Dims& d, int req) {
  const double nn = (double)d.n * d.n;
  // per slot: Gamma and F in complex128, saved Phi in complex64, and the
  // complex128 elimination's A, B and panels
  const double per = nn * (16.0 + 16.0 + 8.0 + 32.0) + 2.0 * 64 * d.n * 16.0 + 64.0 * 64 * 16.0 + 4096.0;
  int s = (int)std::min<double>(1e6, kResolveBudget / per);
  s = std::max(s, 8);
  if (req > 0) s = req;
  return std::min(s, d.Nq);
}

template <typename T>
BseLayout bse_layout(const Dims& d, int slots_req) {
  using C = typename cplx_of<T>::type;
  constexpr int NB = panel_width<T>();
  const size_t nn = (size_t)d.n * d.n;
  BseLayout L{};
  size_t off = 0;
  auto take = [&](size_t b) { size_t o = off; off += align256(b); return o; };
  L.A = take(sizeof(C) * nn * d.Nq);
  L.B = take(sizeof(C) * nn * d.Nq);
  L.MT = take(3 * sizeof(C) * (size_t)NB * d.n * d.Nq);     // panels rotate through three
  L.PI = take(sizeof(C) * (size_t)NB * NB * d.Nq);
  L.pst = take(sizeof(double) * kPst * (size_t)d.Nq);
  if constexpr (sizeof(T) == 4) {
    const int S = resolve_slots(d, slots_req);
    L.slots = S;
    L.py = take(sizeof(double2) * kNpRefine * (size_t)d.n * d.Nq);
    L.pr = take(sizeof(double2) * kNpRefine * (size_t)d.n * d.Nq);
    L.pcs = take(sizeof(float) * (size_t)((d.n + 63) / 64) * d.n * d.Nq);
    L.pcq = take(sizeof(double) * kNpRefine * (size_t)d.n * d.Nq);
    Dims r = d;
    r.Nq = S;
    L.list = take(sizeof(int) * (S + 2));
    L.g64 = take(sizeof(double2) * nn * S);
    L.x64 = take(sizeof(double2) * (size_t)d.n * S);
    L.p64 = take(sizeof(double2) * nn * S);
    L.phis = take(sizeof(float2) * nn * S);
    L.ws64 = take(bse_layout<double>(r).total);
  }
  L.total = off;
  return L;
}

}  // namespace

size_t bse_ws_bytes(const pq_params& p, const Dims& d, int precision) {
  return precision == PQ_PREC_FP64 ? bse_layout<double>(d).total : bse_layout<float>(d, p.resolve_slots).total;
}

template <typename T, bool BF3 = false>
static hipError_t run_bse(const Dims& d, int channel, double alpha, float weak, double kappa_max, double err_tol,
                          int slots_req, const void* gamma, const double2* chi0, void* phi_io,
                          pq_bse_block_stats* stats, void* ws, hipStream_t s, BseTiming* tm,
                          const int* active = nullptr, int tile = 0, const BseAsync* la = nullptr) {
  using C = typename cplx_of<T>::type;
  constexpr int NB = panel_width<T>();
  static const double kSign[4] = {1.0, 1.0, -1.0, 1.0};
  const BseLayout L = bse_layout<T>(d, slots_req);
  char* w = (char*)ws;
  BseCtx<T> a;
  a.n = d.n;
  a.Nq = d.Nq;
  a.nJ = (d.n + NB - 1) / NB;
  a.sign = (T)kSign[channel];
  a.alpha = alpha;
  a.weak_ratio = weak;
  a.kappa_max = kappa_max;
  a.gamma = (const C*)gamma;
  a.chi0 = chi0;
  a.phi = (C*)phi_io;
  a.A = (C*)(w + L.A);
  a.B = (C*)(w + L.B);
  a.MT = (C*)(w + L.MT);
  a.PI = (C*)(w + L.PI);
  a.pst = (double*)(w + L.pst);
  a.stats = stats;
  a.active = active;
  a.pcs = nullptr;
  if constexpr (sizeof(T) == 4) a.pcs = (float*)(w + L.pcs);
  const int n = d.n;
  // event timing around each launch (kind: 0 init, 1 pivot, 2 panel, 3 update,
  // 4 unused (a separate mixing pass, no longer needed), 5 error estimate and
  // FP64 re-solve)
  // the first failed event call (timing or the look-ahead's stream order)
  hipError_t ev_err = hipSuccess;
  auto note = [&](hipError_t e) {
    if (ev_err == hipSuccess) ev_err = e;
  };
  auto pre = [&](int kind, hipStream_t st) {
    if (tm && tm->used < tm->cap) {
      tm->kind[tm->used] = kind;
      note(hipEventRecord(tm->ev[2 * tm->used], st));
    }
  };
  auto post = [&](hipStream_t st) {
    if (tm && tm->used < tm->cap) {
      note(hipEventRecord(tm->ev[2 * tm->used + 1], st));
      tm->used++;
    }
  };
  if (tm) tm->update_flops = 0.0;
  // Multipliers: three buffers, panel J in buffer J % 3 (a paired update of
  // panels J and J + 1 reads both while writing panel J + 2's). The
  // multiplier copy runs for the first panel (formed from Gamma) and a ragged
  // last panel; every other panel's multipliers come from the previous forward
  // update (rows below the panel) and the pivot-row steps of the earlier
  // panels (the U entries above it, stored in A below the diagonal blocks).
  C* mtb[3] = {a.MT, a.MT + (size_t)NB * n * d.Nq, a.MT + 2 * (size_t)NB * n * d.Nq};
  const int last = (a.nJ - 1) * NB;
  // The mixing is fused into the kernels that finish rows of F: the
  // back-substitution launch of panel J for the rows of panel J - 1, the last
  // panel's pivot-row step for its own rows.
  // complex64 path: the blocks with weak or non-finite pivots (all known once
  // the last pivot is met) are listed and gathered for the FP64 re-solve
  // before any row is mixed, with their Phi (none flagged: empty launches)
  const int S = L.slots;
  int* list = nullptr;
  double2 *g64 = nullptr, *x64 = nullptr, *p64 = nullptr;
  float2* phis = nullptr;
  const unsigned gx = (unsigned)std::min<size_t>(256, ((size_t)n * n + kThreads - 1) / kThreads);
  if constexpr (sizeof(T) == 4) {
    list = (int*)(w + L.list);
    g64 = (double2*)(w + L.g64);
    x64 = (double2*)(w + L.x64);
    p64 = (double2*)(w + L.p64);
    phis = (float2*)(w + L.phis);
  }
  auto refine_gather = [&](int late, hipStream_t st) {
    if constexpr (sizeof(T) == 4) {
      hipLaunchKernelGGL(refine_list_kernel, dim3(1), dim3(kThreads), 0, st, a.pst, d.Nq, weak, kappa_max, S, late,
                         list);
      hipLaunchKernelGGL(refine_gather_kernel, dim3(gx, S), dim3(kThreads), 0, st, (const float2*)gamma, chi0,
                         (const float2*)phi_io, n, list, S, late, g64, x64, phis);
    }
  };
  // the diagonal-block inversion (and, for the first panel and a ragged last
  // one, the multiplier copy) of the panel at j0, then its pivot-row step
  auto pivot_step = [&](int j0, hipStream_t st) {
    const int jb = std::min(NB, n - j0);
    const int pj = j0 / NB;
    pre(1, st);
    hipLaunchKernelGGL((bse_pivot_kernel<T, NB>), dim3(1, d.Nq), dim3(pivot_threads<NB>()), 0, st, a, j0);
    if (j0 == 0 || jb < NB) {
      BseCtx<T> am = a;
      am.MT = mtb[pj % 3];
      hipLaunchKernelGGL((bse_multcopy_kernel<T, NB>), dim3((n + 31) / 32, d.Nq), dim3(kThreads), 0, st, am, j0);
    }
    post(st);
    if (j0 == last) refine_gather(0, st);
  };
  auto panel_step = [&](int j0, hipStream_t st) {
    const int jb = std::min(NB, n - j0);
    const int ncols = (n - j0 - jb) + n;
    constexpr int RW = panel_rows_per_wave<T, NB>();
    const int nwb = ((ncols + 31) / 32 * (NB / RW) + kWaves - 1) / kWaves;
    const int mix = j0 == last ? 1 : 0;
    pre(2, st);
    if constexpr (BF3) {
      if (jb == NB) {                            // full panel: the BF16x3 products
        const unsigned ncb = (unsigned)((ncols + NB - 1) / NB);
        if (j0 == 0)
          hipLaunchKernelGGL((bse_panel_bf_kernel<NB, true>), dim3(ncb, d.Nq), dim3(kThreads), 0, st, a, j0, mix);
        else
          hipLaunchKernelGGL((bse_panel_bf_kernel<NB, false>), dim3(ncb, d.Nq), dim3(kThreads), 0, st, a, j0, mix);
        post(st);
        return;
      }
    }
    if (j0 == 0)
      hipLaunchKernelGGL((bse_panel_kernel<T, NB, true, RW>), dim3(nwb, d.Nq), dim3(kThreads), 0, st, a, j0, nwb, mix);
    else
      hipLaunchKernelGGL((bse_panel_kernel<T, NB, false, RW>), dim3(nwb, d.Nq), dim3(kThreads), 0, st, a, j0, nwb,
                         mix);
    post(st);
  };
  constexpr bool kPair = true;     // paired (rank-2NB) updates of full panels
  // Forward update of NKP panels from j0 (1, or 2 for a paired rank-2NB
  // update) for rows [row_lo, row_hi) and the combined columns below col_hi
  // (the trailing columns right of the panels, then B); the results in the
  // first ntc columns of the rows from mult_row on are the multipliers of the
  // panel after them, written transposed into mtn.
  auto upd = [&](int j0, int nkp, int row_lo, int row_hi, int col_hi, int mult_row, C* mt, C* mt1, C* mtn,
                 int ntc) {
    const int jb = std::min(nkp * NB, n - j0);
    const int ncols = std::min((n - j0 - jb) + n, col_hi < 0 ? n + n : col_hi);
    pre(3, s);
    auto go = [&](auto cfg_first, auto cfg) {
      using CFF = decltype(cfg_first);
      using CFG = decltype(cfg);
      if (kPair && nkp == 2) {
        if constexpr (kPair) {
          if (j0 == 0)
            launch_update<T, NB, CFF, 2>(a, n, d.Nq, j0, row_lo, row_hi, 0, false, mt, mtn, ntc, s, -1, mult_row,
                                         col_hi, mt1);
          else
            launch_update<T, NB, CFG, 2>(a, n, d.Nq, j0, row_lo, row_hi, 0, false, mt, mtn, ntc, s, -1, mult_row,
                                         col_hi, mt1);
        }
      } else if (j0 == 0) {
        launch_update<T, NB, CFF>(a, n, d.Nq, j0, row_lo, row_hi, 0, false, mt, mtn, ntc, s, -1, mult_row, col_hi);
      } else {
        launch_update<T, NB, CFG>(a, n, d.Nq, j0, row_lo, row_hi, 0, false, mt, mtn, ntc, s, -1, mult_row, col_hi);
      }
    };
    if constexpr (BF3) {
      if (tile == 1)
        go(UpdFirst<UpdBF3N<true>>{}, UpdBF3N<true>{});
      else
        go(UpdFirst<UpdBF3<true>>{}, UpdBF3<true>{});
    } else if constexpr (sizeof(T) == 4) {
      if (tile == 1)
        go(UpdFirst<UpdNarrow<true>>{}, UpdNarrow<true>{});
      else
        go(UpdFirst<UpdSel<T, true, BF3>>{}, UpdSel<T, true, BF3>{});
    } else {
      go(UpdFirst<UpdSel<T, true, BF3>>{}, UpdSel<T, true, BF3>{});
    }
    post(s);
    if (tm) tm->update_flops += 8.0 * (double)(row_hi - row_lo) * ncols * jb * d.Nq;
  };
  auto side_pivot = [&](int j0) {
    note(hipEventRecord(la->ready, s));
    note(hipStreamWaitEvent(la->side, la->ready, 0));
    pivot_step(j0, la->side);
    note(hipEventRecord(la->done, la->side));
  };
  // Look-ahead (a second stream given): once the rows of the next panel are
  // updated, its diagonal-block inversion runs on the second stream while the
  // rows below it are updated here. The inversion reads only the next panel's
  // diagonal block and writes its P (the current panel's P is consumed by
  // then) and pivot monitor; the rows below read this panel's pivot rows and
  // multipliers. (The pivot-row step cannot go ahead: it writes the U copy
  // into the rows below, whose old values this update still reads.) Only for a
  // full next panel with rows below it (a ragged one has a multiplier copy,
  // which shares its buffer with the update's multiplier output).
  //
  // Paired panels: for two full panels J, J + 1 with rows below them, the
  // rows of J + 1 (every column) and the columns of J + 1 (the rows below it:
  // its multipliers) are updated by panel J first; J + 1 is then inverted and
  // its pivot rows formed; and the rest, the rows below J + 1 right of it, is
  // updated by both panels at once (depth 2 NB). The flops are those of two
  // single updates; the C tiles of the rows below are read and written once
  // instead of twice.
  bool ahead = false;
  int j0 = 0;
  while (j0 < n) {
    const int jb = std::min(NB, n - j0);
    const int pj = j0 / NB;
    if (ahead)
      note(hipStreamWaitEvent(s, la->done, 0));
    else
      pivot_step(j0, s);
    panel_step(j0, s);
    ahead = false;
    if (j0 + jb >= n) break;                   // the last panel: no rows below
    const int lo = j0 + jb;                    // the next panel's first row
    if (kPair && jb == NB && lo + NB < n) {    // pair panels J and J + 1
      const int hi = lo + NB;                  // the rows below J + 1 start here
      upd(j0, 1, lo, hi, -1, hi, mtb[pj % 3], nullptr, mtb[(pj + 1) % 3], NB);
      if (la) side_pivot(lo);
      upd(j0, 1, hi, n, NB, hi, mtb[pj % 3], nullptr, mtb[(pj + 1) % 3], NB);
      if (la)
        note(hipStreamWaitEvent(s, la->done, 0));
      else
        pivot_step(lo, s);
      panel_step(lo, s);
      const int ntc = std::min(NB, n - hi);    // panel J + 2's columns
      const int mrow = hi + ntc;
      if (la && hi + NB < n) {
        upd(j0, 2, hi, hi + NB, -1, mrow, mtb[pj % 3], mtb[(pj + 1) % 3], mtb[(pj + 2) % 3], ntc);
        side_pivot(hi);
        upd(j0, 2, hi + NB, n, -1, mrow, mtb[pj % 3], mtb[(pj + 1) % 3], mtb[(pj + 2) % 3], ntc);
        ahead = true;
      } else {
        upd(j0, 2, hi, n, -1, mrow, mtb[pj % 3], mtb[(pj + 1) % 3], mtb[(pj + 2) % 3], ntc);
      }
      j0 = hi;
      continue;
    }
    // a single panel: the rows below it
    const int ntc = std::min(NB, n - lo);
    const int mrow = lo + ntc;
    if (la && lo + NB < n) {
      upd(j0, 1, lo, lo + NB, -1, mrow, mtb[pj % 3], nullptr, mtb[(pj + 1) % 3], ntc);
      side_pivot(lo);
      upd(j0, 1, lo + NB, n, -1, mrow, mtb[pj % 3], nullptr, mtb[(pj + 1) % 3], ntc);
      ahead = true;
    } else {
      upd(j0, 1, lo, n, -1, mrow, mtb[pj % 3], nullptr, mtb[(pj + 1) % 3], ntc);
    }
    j0 = lo;
  }
  // Back substitution: the rows of panel J of B hold F once every later panel
  // has been subtracted from them, so going from the last panel down, the
  // rows above panel J take B_I -= U_IJ F_J, with U_IJ read k-major from A
  // below the diagonal blocks (full panels) or from the multiplier copy of a
  // ragged last panel. The rows of panel J - 1 are final after the launch of
  // panel J, which also mixes them into Phi.
  // Paired (two full panels J - 1, J with rows above them): the rows of
  // J - 1 take panel J alone (and are mixed), then every row above J - 1
  // takes both panels at depth 2 NB (their U copies are adjacent rows of A,
  // their F adjacent rows of B) and the rows of J - 2 are mixed.
  auto back = [&](auto cfg, int nkp, int jp, int row_lo, int row_hi, int mix_lo) {
    using CFG = decltype(cfg);
    const int jb = std::min(nkp * NB, n - jp);
    pre(3, s);
    if (nkp == 2) {
      if constexpr (kPair)
        launch_update<T, NB, CFG, 2>(a, n, d.Nq, jp, row_lo, row_hi, n - jp - jb, true, a.MT, nullptr, 0, s, mix_lo,
                                     -1, -1, a.A + (size_t)(jp + NB) * n);
    } else {
      launch_update<T, NB, CFG>(a, n, d.Nq, jp, row_lo, row_hi, n - jp - jb, true, a.MT, nullptr, 0, s, mix_lo);
    }
    post(s);
    if (tm) tm->update_flops += 8.0 * (double)(row_hi - row_lo) * n * jb * d.Nq;
  };
  auto back_full = [&](int nkp, int jp, int row_lo, int row_hi, int mix_lo) {
    if constexpr (sizeof(T) == 4) {
      if (tile == 1) {
        if constexpr (BF3)
          back(UpdBF3N<true>{}, nkp, jp, row_lo, row_hi, mix_lo);
        else
          back(UpdNarrow<true>{}, nkp, jp, row_lo, row_hi, mix_lo);
        return;
      }
    }
    back(UpdSel<T, true, BF3>{}, nkp, jp, row_lo, row_hi, mix_lo);
  };
  for (int j0 = last; j0 > 0;) {
    const int jb = std::min(NB, n - j0);
    if (jb == NB && kPair && j0 - NB > 0) {
      const int j1 = j0 - NB;
      back_full(1, j0, j1, j0, j1);
      back_full(2, j1, 0, j1, j1 - NB);
      j0 -= 2 * NB;
      continue;
    }
    const int mix_lo = j0 - NB;
    if (jb == NB) {
      back_full(1, j0, 0, j0, mix_lo);
    } else {
      pre(3, s);
      launch_update<T, NB, UpdSel<T, false, BF3>>(a, n, d.Nq, j0, 0, j0, n - j0 - jb, false, mtb[(j0 / NB) % 3],
                                                   nullptr, 0, s, mix_lo);
      post(s);
      if (tm) tm->update_flops += 8.0 * (double)j0 * n * jb * d.Nq;
    }
    j0 -= NB;
  }
  if constexpr (sizeof(T) == 4) {
    // error estimate of every block (B holds the complex64 F), then the FP64
    // re-solve of the flagged blocks
    pre(5, s);
    const double sg = kSign[channel];
    const unsigned rows_scr = kWaves * 4, rows_ref = kWaves;
    const unsigned rx_all = (unsigned)((n + rows_scr - 1) / rows_scr);
    const int ns = n <= 256 ? n : 128;
    const unsigned rx_s = (unsigned)((ns + rows_scr - 1) / rows_scr);
    const unsigned rx_ref = (unsigned)((n + rows_ref - 1) / rows_ref);
    double2* py = (double2*)(w + L.py);
    double2* pr = (double2*)(w + L.pr);
    double* pcq = (double*)(w + L.pcq);
    const float2* fh = (const float2*)a.B;
    const float2* gm = (const float2*)gamma;
    const double* cpst = a.pst;
    // screen (every block)
    hipLaunchKernelGGL((probe_y_kernel<kNpScreen, 4, false>), dim3(rx_all, d.Nq), dim3(kThreads), 0, s, fh, n, cpst,
                       py);
    hipLaunchKernelGGL((probe_r_kernel<kNpScreen, 4, false>), dim3(rx_s, d.Nq), dim3(kThreads), 0, s, gm, chi0,
                       (const double2*)py, n, sg, cpst, pr);
    hipLaunchKernelGGL(probe_est_kernel, dim3(d.Nq), dim3(kThreads), 0, s, (const double2*)pr,
                       (const float*)a.pcs, fh, chi0, n, sg, err_tol, a.pst);
    // refined estimate (the marked blocks only; the others exit at once)
    hipLaunchKernelGGL((probe_y_kernel<kNpRefine, 1, true>), dim3(rx_ref, d.Nq), dim3(kThreads), 0, s, fh, n, cpst,
                       py);
    hipLaunchKernelGGL((probe_r_kernel<kNpRefine, 1, true>), dim3(rx_ref, d.Nq), dim3(kThreads), 0, s, gm, chi0,
                       (const double2*)py, n, sg, cpst, pr);
    hipLaunchKernelGGL((probe_c_kernel<kNpRefine>), dim3(rx_ref, d.Nq), dim3(kThreads), 0, s, fh, chi0,
                       (const double2*)pr, n, sg, cpst, pcq);
    hipLaunchKernelGGL((probe_flag_kernel<kNpRefine>), dim3(d.Nq), dim3(kThreads), 0, s, (const double*)pcq, n,
                       err_tol, a.pst);
    refine_gather(1, s);
    Dims r = d;
    r.Nq = S;
    const BseLayout L64 = bse_layout<double>(r);
    hipError_t e = run_bse<double>(r, channel, 1.0, 1e-10f, 1e12, 0.0, 0, g64, x64, p64, nullptr, w + L.ws64, s,
                                   nullptr, list + S);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(refine_scatter_kernel, dim3(gx, S), dim3(kThreads), 0, s, (const double2*)p64,
                       (const float2*)phis, (const double*)(w + L.ws64 + L64.pst), (const float2*)gamma, fh, n,
                       list, S, alpha, (float2*)phi_io, a.pst);
    post(s);
  }
  if (stats)
    hipLaunchKernelGGL((bse_stats_kernel<T>), dim3((d.Nq + kThreads - 1) / kThreads), dim3(kThreads), 0, s, a);
  if (ev_err != hipSuccess) return ev_err;
  return hipGetLastError();
}

namespace {
// Counts over the block stats of one iteration (one workgroup, fixed-order sums).
// nchunks runs of nb stats, stride apart
__global__ __launch_bounds__(kThreads) void bse_summary_kernel(const pq_bse_block_stats* st, int nb, int nchunks,
                                                               size_t stride, double* out) {
  __shared__ double red[kThreads];
  double f = 0.0, r = 0.0, u = 0.0, m = 0.0;
  for (int t = threadIdx.x; t < nb * nchunks; t += blockDim.x) {
    const size_t i = (size_t)(t / nb) * stride + (t % nb);
    const int fl = st[i].flags;
    f += (fl & 1) ? 1.0 : 0.0;
    r += (fl & 4) ? 1.0 : 0.0;
    u += (fl & 8) ? 1.0 : 0.0;
    const double e = st[i].err_est;
    m = fmax(m, e <= DBL_MAX ? e : INFINITY);
  }
  f = block_sum(f, red);
  r = block_sum(r, red);
  u = block_sum(u, red);
  m = block_max(m, red);
  if (threadIdx.x == 0) {
    out[0] = f;
    out[1] = r;
    out[2] = u;
    out[3] = m;
  }
}
}  // namespace

hipError_t launch_bse_summary(const pq_bse_block_stats* stats, int nb, double* out, hipStream_t s, int nchunks,
                              size_t stride) {
  hipLaunchKernelGGL(bse_summary_kernel, dim3(1), dim3(kThreads), 0, s, stats, nb, nchunks, stride, out);
  return hipGetLastError();
}

hipError_t launch_bse(const pq_params& p, const Dims& d, int channel, int precision,
                      const void* gamma, const double2* chi0, void* phi_io, double alpha,
                      pq_bse_block_stats* stats, void* ws, hipStream_t s, BseTiming* tm, const BseAsync* la) {
  if (precision == PQ_PREC_FP64) {
    if (p.storage != PQ_STORE_C128) return hipErrorInvalidValue;
    return run_bse<double>(d, channel, alpha, 1e-10f, 1e12, 0.0, 0, gamma, chi0, phi_io, stats, ws, s, tm, nullptr,
                           0, la);
  }
  if (p.storage != PQ_STORE_C64) return hipErrorInvalidValue;
  // complex64: a block is re-solved in FP64 when its pivot ratio drops below
  // 1e-3, a diagonal-block inverse exceeds 1e3, a pivot is not finite, or its
  // error estimate exceeds bse_tol (default 2e-5)
  const double tol = p.bse_tol > 0.0 ? p.bse_tol : kDefaultBseTol;
  if (precision == PQ_PREC_BF16X3)
    return run_bse<float, true>(d, channel, alpha, 1e-3f, 1e3, tol, p.resolve_slots, gamma, chi0, phi_io, stats, ws,
                                s, tm, nullptr, p.bse_tile, la);
  return run_bse<float>(d, channel, alpha, 1e-3f, 1e3, tol, p.resolve_slots, gamma, chi0, phi_io, stats, ws, s, tm,
                        nullptr, p.bse_tile, la);
}

}  // namespace pq
