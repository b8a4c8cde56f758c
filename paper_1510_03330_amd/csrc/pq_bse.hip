// Bethe-Salpeter equations (Eq. PA_F_Phi) of one channel, solved for every
// bosonic transfer q as the dense complex system
//     A F = Gamma,   A = 1 - s Gamma diag(X),
// followed by Phi <- alpha (F - Gamma) + (1 - alpha) Phi.
//
// Blocked Gauss-Jordan elimination on the augmented [A | B] (B = Gamma) with
// panel width NB and no row exchanges, batched over all q blocks of a channel:
// every step is one kernel launch over (q block, tile) grids. Per panel J:
//   (a) bse_diag:   factor the NB x NB diagonal block in LDS, A_JJ = L_JJ U_JJ,
//                   and invert both triangular factors (one workgroup per block);
//   (b) bse_panel:  row panel U_JK = L_JJ^-1 A_JK for every column right of the
//                   panel in A and every column of B (in place, row tiles
//                   bottom-up), and
//   (c)             multipliers M_IJ = A_IJ U_JJ^-1 for every row, stored k-major
//                   (MT[k][i] = (U_JJ^-T A_IJ^T)[k][i]) so operand loads coalesce;
//   (d) bse_update: A_IK -= M_IJ U_JK, B_I -= M_IJ U_JB for all rows I != J, a
//                   rank-NB update; each wave owns a 64 x 32 (complex64) or
//                   32 x 32 (complex128) tile and reads both operands straight
//                   from L1/L2, so no LDS is needed and four waves share a SIMD.
// After the last panel every row block satisfies U_JJ F_J = B_J; bse_final
// applies F_J = U_JJ^-1 B_J fused with the Phi epilogue. Steps (b)-(d) and the
// final solve are complex products on the matrix cores, four real MFMAs per
// complex product: v_mfma_f32_32x32x2f32 (complex64) or v_mfma_f64_16x16x4f64
// (complex128).
//
// No row exchanges: A is the identity minus the small-norm kernel s Gamma X,
// and every leading principal block of it stays invertible while the BSE is
// away from its instability. The pivot monitor records min|u_jj| / max|u_jj|
// per block and flags weak or non-finite blocks.
#include <float.h>

#include <algorithm>

#include "pq_internal.h"

namespace pq {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------ matrix cores
template <typename T> struct Mma;

template <> struct Mma<float> {   // v_mfma_f32_32x32x2f32
  static constexpr int TM = 32, TN = 32, KS = 2, NV = 16;
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
  static constexpr int TM = 16, TN = 16, KS = 4, NV = 4;
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

// LU of the jb x jb block in D (no exchanges); pivot stats in pst.
template <typename C, int NB>
__device__ void factor_block(C (*D)[NB + 1], int jb, double* pst) {
  const int t = threadIdx.x;
  for (int c = 0; c < jb; ++c) {
    const C piv = D[c][c];
    if (t == 0) {
      const double ap = cabs_d(piv);
      if (!(ap == ap) || ap > DBL_MAX) pst[2] = 1.0;
      pst[0] = fmin(pst[0], ap);
      pst[1] = fmax(pst[1], ap);
    }
    const C rp = cdiv(make_cone<C>(), piv);
    for (int r = c + 1 + t; r < jb; r += blockDim.x) D[r][c] = cmul(D[r][c], rp);
    __syncthreads();
    const int rem = jb - c - 1;
    for (int idx = t; idx < rem * rem; idx += blockDim.x) {
      const int r = c + 1 + idx / rem, cc = c + 1 + idx - (idx / rem) * rem;
      D[r][cc] = cfms(D[r][cc], D[r][c], D[c][cc]);
    }
    __syncthreads();
  }
}

// Both triangular inverses of the factored block D = L U (unit L), written
// into one array: X[i][j] = (L^-1)[i][j] for i > j and (U^-1)[i][j] for i <= j.
// Wave 0 forward-substitutes L X = I and wave 1 back-substitutes U X = I, one
// column per lane, so neither needs a barrier: a lane reads only its own
// column of X (written earlier by itself) and D, which no wave writes here.
// The k-loops are uniform across the wave (entries a lane does not need are
// masked by a select), so the D reads are broadcasts.
template <typename C, int NB>
__device__ void invert_triangles(C (*D)[NB + 1], C (*X)[NB + 1], int jb) {
  const int wave = threadIdx.x >> 6, j = threadIdx.x & 63;
  if (j >= NB) return;
  if (wave == 0) {
    // (L^-1)[i][j] = -sum_{k<i} L[i][k] x_k with x_j = 1, x_k = 0 for k < j
    for (int i = 1; i < jb; ++i) {
      C acc = cz<C>();
#pragma unroll 8
      for (int k = 0; k < i; ++k) {
        C xk = X[k][j];
        if (k <= j) { xk = cz<C>(); if (k == j) xk.x = 1; }
        acc = cfms(acc, D[i][k], xk);
      }
      if (i > j) X[i][j] = acc;
    }
  } else if (wave == 1) {
    // (U^-1)[i][j] = (delta_ij - sum_{k>i} U[i][k] x_k) / U[i][i], x_k = 0 for k > j
    for (int i = jb - 1; i >= 0; --i) {
      C acc = cz<C>();
      if (i == j) acc.x = 1;
#pragma unroll 8
      for (int k = i + 1; k < jb; ++k) {
        C xk = X[k][j];
        if (k > j) xk = cz<C>();
        acc = cfms(acc, D[i][k], xk);
      }
      if (i <= j) X[i][j] = cdiv(acc, D[i][i]);
    }
  }
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
  C* MT;                 // [Nq][NB][n]
  C* LI;                 // [Nq][NB][NB]   L^-1 of the current panel
  C* UI;                 // [Nq][nJ][NB][NB] U^-1 of every panel
  double* pst;           // [Nq][4]  min |pivot|, max |pivot|, non-finite seen
  pq_bse_block_stats* stats;
};

// ------------------------------------------------------------------- init
// A = 1 - s Gamma diag(X), B = Gamma
template <typename T>
__global__ __launch_bounds__(kThreads) void bse_init_kernel(BseCtx<T> a) {
  using C = typename cplx_of<T>::type;
  const int blk = blockIdx.y;
  const int n = a.n;
  const size_t nn = (size_t)n * n;
  const C* G = a.gamma + (size_t)blk * nn;
  C* A = a.A + (size_t)blk * nn;
  C* B = a.B + (size_t)blk * nn;
  const double2* x = a.chi0 + (size_t)blk * n;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < nn; idx += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx / n), j = (int)(idx - (size_t)i * n);
    const C g = G[idx];
    const double2 xv = x[j];
    const T sx = a.sign * (T)xv.x, sy = a.sign * (T)xv.y;
    C v;
    v.x = (i == j ? (T)1 : (T)0) - (g.x * sx - g.y * sy);
    v.y = -(g.x * sy + g.y * sx);
    A[idx] = v;
    B[idx] = g;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double* ps = a.pst + (size_t)blk * 4;
    ps[0] = DBL_MAX;
    ps[1] = 0.0;
    ps[2] = 0.0;
  }
}

// ------------------------------------------------------------------- diag
constexpr int kDiagThreads = kThreads;

// LU of the diagonal block A_JJ in LDS and both triangular inverses: LI gets
// L^-1 (identity outside the jb x jb block), UI[J] gets U^-1 (zero outside).
// The factored block itself is not written back: later steps read only the
// inverses.
template <typename T, int NB>
__global__ __launch_bounds__(kDiagThreads) void bse_diag_kernel(BseCtx<T> a, int j0) {
  using C = typename cplx_of<T>::type;
  __shared__ C D[NB][NB + 1];
  __shared__ C X[NB][NB + 1];
  __shared__ double pst[3];
  const int blk = blockIdx.x, t = threadIdx.x, n = a.n;
  const int jb = min(NB, n - j0);
  const C* A = a.A + (size_t)blk * n * n;
  double* gps = a.pst + (size_t)blk * 4;
  if (t < 3) pst[t] = gps[t];
  for (int idx = t; idx < NB * NB; idx += blockDim.x) {
    const int r = idx / NB, c = idx - (idx / NB) * NB;
    const C v = A[(size_t)(j0 + min(r, jb - 1)) * n + j0 + min(c, jb - 1)];
    D[r][c] = (r < jb && c < jb) ? v : cz<C>();
  }
  __syncthreads();
  factor_block<C, NB>(D, jb, pst);
  invert_triangles<C, NB>(D, X, jb);
  __syncthreads();
  C* LI = a.LI + (size_t)blk * NB * NB;
  C* UI = a.UI + ((size_t)blk * a.nJ + j0 / NB) * NB * NB;
  for (int idx = t; idx < NB * NB; idx += blockDim.x) {
    const int r = idx / NB, c = idx - (idx / NB) * NB;
    const C x = X[r][c];
    C l = cz<C>(), u = cz<C>();
    if (r == c) l.x = 1;
    if (r > c && r < jb) l = x;
    if (r <= c && c < jb) u = x;
    LI[idx] = l;
    UI[idx] = u;
  }
  if (t < 3) gps[t] = pst[t];
}

// ------------------------------------------------------------------ panel
// acc += sum_{k < NB} a(k) b(k) over one full panel: the a operand comes from
// LDS through fa(ks, av), the b operand from global memory through fb(ks, bv)
// with branch-free loads issued PF k-steps ahead of the matrix cores.
// Triangular operands are used whole (their zero half costs matrix-core time
// but keeps the loop fixed-length and fully pipelined).
template <typename T, int NB, class FA, class FB>
__device__ inline void panel_kloop(WTile<T>& acc, FA fa, FB fb) {
  using C = typename cplx_of<T>::type;
  using M = Mma<T>;
  constexpr int SR = WTile<T>::SR, SC = WTile<T>::SC, KSTEPS = NB / M::KS, PF = 2;
  C bq[PF][SC];
#pragma unroll
  for (int s = 0; s < PF; ++s) fb(s, bq[s]);
#pragma unroll
  for (int ks = 0; ks < KSTEPS; ++ks) {
    const int cur = ks % PF;
    C bv[SC], av[SR];
#pragma unroll
    for (int y = 0; y < SC; ++y) bv[y] = bq[cur][y];
    if (ks + PF < KSTEPS) fb(ks + PF, bq[cur]);
    fa(ks, av);
    __builtin_amdgcn_sched_barrier(0);
    acc.mac(av, bv, false);
  }
}

// x < nwb: row-panel workgroups, 4 column strips of 32 each (one per wave);
// x >= nwb: multiplier workgroups, 4 row strips of 32 each.
template <typename T, int NB>
__global__ __launch_bounds__(kThreads) void bse_panel_kernel(BseCtx<T> a, int j0, int nwb) {
  using C = typename cplx_of<T>::type;
  using M = Mma<T>;
  using WT = WTile<T>;
  constexpr int SR = WT::SR, SC = WT::SC;
  __shared__ C X[NB][NB + 1];
  const int blk = blockIdx.y, t = threadIdx.x, lane = t & 63, wave = t >> 6, n = a.n;
  const int jb = min(NB, n - j0);
  const int ncols = (n - j0 - jb) + n;
  C* A = a.A + (size_t)blk * n * n;
  C* B = a.B + (size_t)blk * n * n;
  const bool rowpanel = (int)blockIdx.x < nwb;
  const C* src = rowpanel ? a.LI + (size_t)blk * NB * NB : a.UI + ((size_t)blk * a.nJ + j0 / NB) * NB * NB;
  for (int idx = t; idx < NB * NB; idx += blockDim.x) X[idx / NB][idx % NB] = src[idx];
  __syncthreads();
  const int kb = M::b_k(lane);
  if (rowpanel) {
    // U_JK = L^-1 A_JK in place. Row tile rt of the product needs input rows
    // <= its own last row only (L^-1 is lower triangular), so the tiles go
    // bottom-up; the rows an upper tile has already overwritten meet exact
    // zeros of L^-1.
    const int cs = blockIdx.x * kWaves + wave;
    if (cs * 32 >= ncols) return;
    const C* cp[SC];
#pragma unroll
    for (int y = 0; y < SC; ++y)
      cp[y] = colptr(A, B, n, j0, jb, min(cs * 32 + y * M::TN + M::b_col(lane), ncols - 1)) + (size_t)j0 * n;
    for (int rt = NB / 32 - 1; rt >= 0; --rt) {
      WT acc;
      acc.zero();
      panel_kloop<T, NB>(acc,
          [&](int ks, C (&av)[SR]) {
#pragma unroll
            for (int xx = 0; xx < SR; ++xx) av[xx] = X[rt * 32 + xx * M::TM + M::a_row(lane)][ks * M::KS + M::a_k(lane)];
          },
          [&](int ks, C (&bv)[SC]) {
            const int k = min(ks * M::KS + kb, jb - 1);
#pragma unroll
            for (int y = 0; y < SC; ++y) bv[y] = cp[y][(size_t)k * n];
          });
      acc.store([&](int r, int c, C v) {
        const int row = rt * 32 + r, col = cs * 32 + c;
        if (row < jb && col < ncols) colptr(A, B, n, j0, jb, col)[(size_t)(j0 + row) * n] = v;
      });
    }
  } else {
    // MT = U^-T A_IJ^T: rows k of the panel, columns i = every row of A. Rows
    // jb..NB-1 (ragged last panel) come out exactly zero, since U^-1 is zero
    // outside the jb x jb block; the update reads them unmasked.
    const int is = (blockIdx.x - nwb) * kWaves + wave;
    if (is * 32 >= n) return;
    C* MT = a.MT + (size_t)blk * NB * n;
    const C* rp[SC];
#pragma unroll
    for (int y = 0; y < SC; ++y) rp[y] = A + (size_t)min(is * 32 + y * M::TN + M::b_col(lane), n - 1) * n + j0;
    for (int rt = 0; rt < NB / 32; ++rt) {
      WT acc;
      acc.zero();
      panel_kloop<T, NB>(acc,
          [&](int ks, C (&av)[SR]) {
#pragma unroll
            for (int xx = 0; xx < SR; ++xx) av[xx] = X[ks * M::KS + M::a_k(lane)][rt * 32 + xx * M::TM + M::a_row(lane)];
          },
          [&](int ks, C (&bv)[SC]) {
            const int k = min(ks * M::KS + kb, jb - 1);
#pragma unroll
            for (int y = 0; y < SC; ++y) bv[y] = rp[y][k];
          });
      acc.store([&](int r, int c, C v) {
        const int row = rt * 32 + r, i = is * 32 + c;
        if (i < n) MT[(size_t)row * n + i] = v;
      });
    }
  }
}

// ----------------------------------------------------------------- update
// C[i][col] -= sum_k MT[k][i] U[k][col] for every row i outside the panel.
// Workgroup tile (2 UWM) x (2 UWN), waves 2 x 2, each wave a UWM x UWN tile.
// Tile shape and pipelining of the update: wave tile UWM x UWN, workgroup of
// 2 x 2 waves, operand prefetch PF k-steps ahead; FULL = the panel is NB wide
// (every panel but a ragged last one), so the panel rows need no clamping.
template <typename T, int UWM_, int UWN_, int PF_, int WPE_, bool FULL_>
struct UpdCfg {
  static constexpr int UWM = UWM_, UWN = UWN_, PF = PF_, WPE = WPE_;
  static constexpr bool FULL = FULL_;
  static constexpr int WGM = 2 * UWM, WGN = 2 * UWN;
};
template <typename T, bool FULL>
using UpdDefault = UpdCfg<T, sizeof(T) == 4 ? 64 : 32, 32, sizeof(T) == 4 ? 2 : 1, 4, FULL>;

template <typename T, int NB, class CF>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(CF::WPE)))
void bse_update_kernel(BseCtx<T> a, int j0, int ncb) {
  using C = typename cplx_of<T>::type;
  using M = Mma<T>;
  using UT = WTile<T, CF::UWM, CF::UWN>;
  constexpr int USR = UT::SR, USC = UT::SC, KSTEPS = NB / M::KS, PF = CF::PF;
  const unsigned lid = xcd_linear();
  const int blk = lid / gridDim.x, bx = lid - (lid / gridDim.x) * gridDim.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, n = a.n;
  const int jb = CF::FULL ? NB : min(NB, n - j0);
  const int ncols = (n - j0 - jb) + n;
  const int rb = bx / ncb, cbk = bx - (bx / ncb) * ncb;
  const int wr = wave & 1, wc = wave >> 1;
  const int i0 = rb * CF::WGM + wr * CF::UWM;
  const int c0 = cbk * CF::WGN + wc * CF::UWN;
  if (i0 >= n || c0 >= ncols || (i0 >= j0 && i0 + CF::UWM <= j0 + jb)) return;
  C* A = a.A + (size_t)blk * n * n;
  C* B = a.B + (size_t)blk * n * n;
  const C* MT = a.MT + (size_t)blk * NB * n;
  // Every load below is unconditional from a clamped, in-bounds address, so
  // the loads carry no branches and are issued ahead of the matrix-core work.
  // Lanes of rows or columns that are not stored read finite data that never
  // reaches an output; panel rows k >= jb (ragged last panel) multiply the
  // rows of MT that the panel step wrote as zeros.
  C* cb[USC];
  bool cok[USC];
#pragma unroll
  for (int y = 0; y < USC; ++y) {
    const int col = c0 + y * M::TN + M::b_col(lane);
    cok[y] = col < ncols;
    cb[y] = colptr(A, B, n, j0, jb, cok[y] ? col : 0);
  }
  auto row_ok = [&](int i) { return i < n && !(i >= j0 && i < j0 + jb); };
  UT acc;
  acc.load([&](int r, int c) -> C { return cb[c / M::TN][(size_t)min(i0 + r, n - 1) * n]; });
  const int kb = M::b_k(lane), ka = M::a_k(lane);
  const C* bbase[USC];
#pragma unroll
  for (int y = 0; y < USC; ++y) bbase[y] = cb[y] + (size_t)(j0 + (CF::FULL ? kb : 0)) * n;
  const C* abase[USR];
#pragma unroll
  for (int xx = 0; xx < USR; ++xx) abase[xx] = MT + (size_t)ka * n + min(i0 + xx * M::TM + M::a_row(lane), n - 1);
  auto fetch = [&](int ks, C (&av)[USR], C (&bv)[USC]) {
    if (CF::FULL) {
#pragma unroll
      for (int y = 0; y < USC; ++y) bv[y] = bbase[y][(size_t)(ks * M::KS) * n];
    } else {
      const int kk = min(ks * M::KS + kb, jb - 1);
#pragma unroll
      for (int y = 0; y < USC; ++y) bv[y] = bbase[y][(size_t)kk * n];
    }
#pragma unroll
    for (int xx = 0; xx < USR; ++xx) av[xx] = abase[xx][(size_t)(ks * M::KS) * n];
  };
  C av[PF][USR], bv[PF][USC];
#pragma unroll
  for (int s = 0; s < PF; ++s) fetch(s, av[s], bv[s]);
#pragma unroll
  for (int ks = 0; ks < KSTEPS; ++ks) {
    const int cur = ks % PF;
    C ca[USR], cbv[USC];
#pragma unroll
    for (int xx = 0; xx < USR; ++xx) ca[xx] = av[cur][xx];
#pragma unroll
    for (int y = 0; y < USC; ++y) cbv[y] = bv[cur][y];
    if (ks + PF < KSTEPS) fetch(ks + PF, av[cur], bv[cur]);
    __builtin_amdgcn_sched_barrier(0);     // keep the prefetch ahead of this step's MFMAs
    acc.mac(ca, cbv, true);
  }
  acc.store([&](int r, int c, C v) {
    const int i = i0 + r;
    const int y = c / M::TN;
    if (cok[y] && row_ok(i)) cb[y][(size_t)i * n] = v;
  });
}

template <typename T, int NB, class CF>
void launch_update(const BseCtx<T>& a, int n, int Nq, int j0, hipStream_t s) {
  const int jb = std::min(NB, n - j0);
  const int ncols = (n - j0 - jb) + n;
  const int nrb = (n + CF::WGM - 1) / CF::WGM;
  const int ncb = (ncols + CF::WGN - 1) / CF::WGN;
  hipLaunchKernelGGL((bse_update_kernel<T, NB, CF>), dim3(nrb * ncb, Nq), dim3(kThreads), 0, s, a, j0, ncb);
}

// ------------------------------------------------------------------ final
// F_J = U_JJ^-1 B_J for every panel J, then Phi <- alpha (F - Gamma) + (1 - alpha) Phi.
template <typename T, int NB>
__global__ __launch_bounds__(kThreads) void bse_final_kernel(BseCtx<T> a, int nstripw) {
  using C = typename cplx_of<T>::type;
  using M = Mma<T>;
  using WT = WTile<T>;
  constexpr int SR = WT::SR, SC = WT::SC;
  __shared__ C X[NB][NB + 1];
  const int blk = blockIdx.y, t = threadIdx.x, lane = t & 63, wave = t >> 6, n = a.n;
  const int J = blockIdx.x / nstripw, sw = blockIdx.x - (blockIdx.x / nstripw) * nstripw;
  const int j0 = J * NB, jb = min(NB, n - j0);
  const size_t nn = (size_t)n * n;
  const C* UI = a.UI + ((size_t)blk * a.nJ + J) * NB * NB;
  for (int idx = t; idx < NB * NB; idx += blockDim.x) X[idx / NB][idx % NB] = UI[idx];
  __syncthreads();
  if (blockIdx.x == 0 && t == 0 && a.stats) {
    const double* ps = a.pst + (size_t)blk * 4;
    pq_bse_block_stats st;
    const double ratio = ps[1] > 0.0 ? ps[0] / ps[1] : 0.0;
    st.min_pivot = (float)ratio;
    st.growth = (float)ps[1];
    st.flags = (ps[2] > 0.0 ? 2 : 0) | (ratio < a.weak_ratio ? 1 : 0);
    st.reserved = 0;
    a.stats[blk] = st;
  }
  const int cs = sw * kWaves + wave;
  if (cs * 32 >= n) return;
  const C* B = a.B + (size_t)blk * nn;
  const C* G = a.gamma + (size_t)blk * nn;
  C* P = a.phi + (size_t)blk * nn;
  const T al = (T)a.alpha, be = (T)(1.0 - a.alpha);
  const bool mix = a.alpha != 1.0;
  const int kb = M::b_k(lane);
  const C* cp[SC];
#pragma unroll
  for (int y = 0; y < SC; ++y) cp[y] = B + (size_t)j0 * n + min(cs * 32 + y * M::TN + M::b_col(lane), n - 1);
  for (int rt = 0; rt < NB / 32; ++rt) {
    WT acc;
    acc.zero();
    panel_kloop<T, NB>(acc,
        [&](int ks, C (&av)[SR]) {
#pragma unroll
          for (int xx = 0; xx < SR; ++xx) av[xx] = X[rt * 32 + xx * M::TM + M::a_row(lane)][ks * M::KS + M::a_k(lane)];
        },
        [&](int ks, C (&bv)[SC]) {
          const int k = min(ks * M::KS + kb, jb - 1);
#pragma unroll
          for (int y = 0; y < SC; ++y) bv[y] = cp[y][(size_t)k * n];
        });
    // epilogue: Gamma and the old Phi are gathered with unconditional loads
    // from clamped addresses first, then combined and stored where in range
    auto at = [&](int r, int c) { return (size_t)(j0 + min(rt * 32 + r, jb - 1)) * n + min(cs * 32 + c, n - 1); };
    WT g, old;
    g.load([&](int r, int c) { return G[at(r, c)]; });
    if (mix) old.load([&](int r, int c) { return P[at(r, c)]; });
#pragma unroll
    for (int x = 0; x < SR; ++x)
#pragma unroll
      for (int y = 0; y < SC; ++y)
#pragma unroll
        for (int v = 0; v < M::NV; ++v) {
          const int row = rt * 32 + x * M::TM + M::c_row(lane, v), col = cs * 32 + y * M::TN + M::c_col(lane);
          C o;
          o.x = acc.re[x][y][v] - g.re[x][y][v];
          o.y = acc.im[x][y][v] - g.im[x][y][v];
          if (mix) {
            o.x = al * o.x + be * old.re[x][y][v];
            o.y = al * o.y + be * old.im[x][y][v];
          }
          if (row < jb && col < n) P[(size_t)(j0 + row) * n + col] = o;
        }
  }
}

template <typename T>
constexpr int panel_width() { return sizeof(T) == 4 ? 64 : 32; }

struct BseLayout {
  size_t A, B, MT, LI, UI, pst, total;
};

template <typename T>
BseLayout bse_layout(const Dims& d) {
  using C = typename cplx_of<T>::type;
  constexpr int NB = panel_width<T>();
  const size_t nn = (size_t)d.n * d.n;
  const int nJ = (d.n + NB - 1) / NB;
  BseLayout L{};
  size_t off = 0;
  auto take = [&](size_t b) { size_t o = off; off += align256(b); return o; };
  L.A = take(sizeof(C) * nn * d.Nq);
  L.B = take(sizeof(C) * nn * d.Nq);
  L.MT = take(sizeof(C) * (size_t)NB * d.n * d.Nq);
  L.LI = take(sizeof(C) * (size_t)NB * NB * d.Nq);
  L.UI = take(sizeof(C) * (size_t)NB * NB * nJ * d.Nq);
  L.pst = take(sizeof(double) * 4 * (size_t)d.Nq);
  L.total = off;
  return L;
}

}  // namespace

size_t bse_ws_bytes(const pq_params& p, const Dims& d, int precision) {
  (void)p;
  return precision == PQ_PREC_FP64 ? bse_layout<double>(d).total : bse_layout<float>(d).total;
}

template <typename T>
static hipError_t run_bse(const Dims& d, int channel, double alpha, float weak, const void* gamma,
                          const double2* chi0, void* phi_io, pq_bse_block_stats* stats, void* ws,
                          hipStream_t s, BseTiming* tm) {
  using C = typename cplx_of<T>::type;
  constexpr int NB = panel_width<T>();
  static const double kSign[4] = {1.0, 1.0, -1.0, 1.0};
  const BseLayout L = bse_layout<T>(d);
  char* w = (char*)ws;
  BseCtx<T> a;
  a.n = d.n;
  a.Nq = d.Nq;
  a.nJ = (d.n + NB - 1) / NB;
  a.sign = (T)kSign[channel];
  a.alpha = alpha;
  a.weak_ratio = weak;
  a.gamma = (const C*)gamma;
  a.chi0 = chi0;
  a.phi = (C*)phi_io;
  a.A = (C*)(w + L.A);
  a.B = (C*)(w + L.B);
  a.MT = (C*)(w + L.MT);
  a.LI = (C*)(w + L.LI);
  a.UI = (C*)(w + L.UI);
  a.pst = (double*)(w + L.pst);
  a.stats = stats;
  const int n = d.n;
  // event timing around each launch (kind: 0 init, 1 diag, 2 panel, 3 update, 4 final)
  auto pre = [&](int kind) {
    if (tm && tm->used < tm->cap) {
      tm->kind[tm->used] = kind;
      hipEventRecord(tm->ev[2 * tm->used], s);
    }
  };
  auto post = [&]() {
    if (tm && tm->used < tm->cap) {
      hipEventRecord(tm->ev[2 * tm->used + 1], s);
      tm->used++;
    }
  };
  if (tm) tm->update_flops = 0.0;
  const unsigned init_x = (unsigned)std::min<size_t>(1024, ((size_t)n * n + kThreads - 1) / kThreads);
  pre(0);
  hipLaunchKernelGGL((bse_init_kernel<T>), dim3(init_x, d.Nq), dim3(kThreads), 0, s, a);
  post();
  for (int j0 = 0; j0 < n; j0 += NB) {
    const int jb = std::min(NB, n - j0);
    const int ncols = (n - j0 - jb) + n;
    pre(1);
    hipLaunchKernelGGL((bse_diag_kernel<T, NB>), dim3(d.Nq), dim3(kDiagThreads), 0, s, a, j0);
    post();
    const int nwb = ((ncols + 31) / 32 + kWaves - 1) / kWaves;
    const int nwc = ((n + 31) / 32 + kWaves - 1) / kWaves;
    pre(2);
    hipLaunchKernelGGL((bse_panel_kernel<T, NB>), dim3(nwb + nwc, d.Nq), dim3(kThreads), 0, s, a, j0, nwb);
    post();
    pre(3);
    if (jb == NB)
      launch_update<T, NB, UpdDefault<T, true>>(a, n, d.Nq, j0, s);
    else
      launch_update<T, NB, UpdDefault<T, false>>(a, n, d.Nq, j0, s);
    post();
    if (tm) tm->update_flops += 8.0 * (double)(n - jb) * ncols * jb * d.Nq;
  }
  const int nstripw = ((n + 31) / 32 + kWaves - 1) / kWaves;
  pre(4);
  hipLaunchKernelGGL((bse_final_kernel<T, NB>), dim3(a.nJ * nstripw, d.Nq), dim3(kThreads), 0, s, a, nstripw);
  post();
  return hipGetLastError();
}

hipError_t launch_bse(const pq_params& p, const Dims& d, int channel, int precision,
                      const void* gamma, const double2* chi0, void* phi_io, double alpha,
                      pq_bse_block_stats* stats, void* ws, hipStream_t s, BseTiming* tm) {
  if (precision == PQ_PREC_FP64) {
    if (p.storage != PQ_STORE_C128) return hipErrorInvalidValue;
    return run_bse<double>(d, channel, alpha, 1e-10f, gamma, chi0, phi_io, stats, ws, s, tm);
  }
  if (p.storage != PQ_STORE_C64) return hipErrorInvalidValue;
  return run_bse<float>(d, channel, alpha, 1e-3f, gamma, chi0, phi_io, stats, ws, s, tm);
}

}  // namespace pq
