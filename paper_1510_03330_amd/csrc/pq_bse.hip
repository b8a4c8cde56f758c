// Bethe-Salpeter equations (Eq. PA_F_Phi) of one channel, solved for every
// bosonic transfer q as the dense complex system
//     A F = Gamma,   A = 1 - s Gamma diag(X),
// followed by Phi <- alpha (F - Gamma) + (1 - alpha) Phi.
//
// One workgroup owns one q block for its whole life (persistent per block):
// blocked Gauss-Jordan elimination on the augmented [A | B] (B = Gamma) with
// panel width NB and no row exchanges. Per panel J:
//   (a) factor the NB x NB diagonal block in LDS, A_JJ = L_JJ U_JJ, and invert
//       both triangular factors in LDS;
//   (b) row panel    U_JK = L_JJ^-1 A_JK for every column right of the panel in
//       A and every column of B;
//   (c) multipliers  M_IJ = A_IJ U_JJ^-1 for every row, stored k-major
//       (MT[k][i] = (U_JJ^-T A_IJ^T)[k][i]) so matrix-core operand loads coalesce;
//   (d) update       A_IK -= M_IJ U_JK, B_I -= M_IJ U_JB for all rows I != J.
// After the last panel every row block satisfies U_JJ F_J = B_J, and
// F_J = U_JJ^-1 B_J is fused with the Phi epilogue. Steps (b), (c), (d) and the
// final solve are complex products on the matrix cores, built from four real
// MFMAs per complex product: v_mfma_f32_32x32x2f32 (complex64) or
// v_mfma_f64_16x16x4f64 (complex128), each wave owning 32 x 32 output tiles.
//
// No row exchanges: A is the identity minus the small-norm kernel s Gamma X,
// and every leading principal block of it stays invertible while the BSE is
// away from its instability. The pivot monitor records min|u_jj| / max|u_jj|
// per block and flags weak or non-finite blocks.
#include <float.h>

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

// A 32 x 32 complex output tile owned by one wave.
template <typename T>
struct WTile {
  using M = Mma<T>;
  using C = typename cplx_of<T>::type;
  static constexpr int SR = 32 / M::TM, SC = 32 / M::TN;
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

template <typename T>
struct BseArgs {
  using C = typename cplx_of<T>::type;
  Dims d;
  T sign;
  double alpha;
  float weak_ratio;
  const C* gamma;        // [Nq][n][n]
  const double2* chi0;   // [Nq][n]
  C* phi;                // [Nq][n][n]
  C* A;                  // workspace [Nq][n][n]
  C* B;                  // workspace [Nq][n][n]
  C* MT;                 // workspace [Nq][NB][n]
  pq_bse_block_stats* stats;
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
    for (int r = c + 1 + t; r < jb; r += blockDim.x) D[r][c] = cdiv(D[r][c], piv);
    __syncthreads();
    const int rem = jb - c - 1;
    for (int idx = t; idx < rem * rem; idx += blockDim.x) {
      const int r = c + 1 + idx / rem, cc = c + 1 + idx - (idx / rem) * rem;
      D[r][cc] = cfms(D[r][cc], D[r][c], D[c][cc]);
    }
    __syncthreads();
  }
}

// X = L^-1 of the unit-lower part of D (identity outside the jb x jb block).
template <typename C, int NB>
__device__ void invert_lower(C (*D)[NB + 1], C (*X)[NB + 1], int jb) {
  const int t = threadIdx.x;
  for (int idx = t; idx < NB * NB; idx += blockDim.x) {
    const int r = idx / NB, c = idx - (idx / NB) * NB;
    C z = cz<C>();
    if (r == c) z.x = 1;
    X[r][c] = z;
  }
  __syncthreads();
  // row by row: X[i][j] = -sum_{k=j}^{i-1} L[i][k] X[k][j]  (j < i)
  for (int i = 1; i < jb; ++i) {
    for (int j = t; j < i; j += blockDim.x) {
      C s = cz<C>();
      for (int k = j; k < i; ++k) s = cfms(s, D[i][k], X[k][j]);
      X[i][j] = s;
    }
    __syncthreads();
  }
}

// X = U^-1 of the upper part of D (zero outside the jb x jb block).
template <typename C, int NB>
__device__ void invert_upper(C (*D)[NB + 1], C (*X)[NB + 1], int jb) {
  const int t = threadIdx.x;
  for (int idx = t; idx < NB * NB; idx += blockDim.x) {
    const int r = idx / NB, c = idx - (idx / NB) * NB;
    X[r][c] = cz<C>();
  }
  __syncthreads();
  // rows bottom-up: X[i][i] = 1/U[i][i], X[i][j] = -(sum_{k=i+1}^{j} U[i][k] X[k][j]) / U[i][i]
  for (int i = jb - 1; i >= 0; --i) {
    for (int j = i + t; j < jb; j += blockDim.x) {
      if (j == i) {
        X[i][i] = cdiv(make_cone<C>(), D[i][i]);
      } else {
        C s = cz<C>();
        for (int k = i + 1; k <= j; ++k) s = cfms(s, D[i][k], X[k][j]);
        X[i][j] = cdiv(s, D[i][i]);
      }
    }
    __syncthreads();
  }
}

template <typename T, int NB>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 2)))
void bse_gj_kernel(BseArgs<T> a) {
  using C = typename cplx_of<T>::type;
  using M = Mma<T>;
  using WT = WTile<T>;
  constexpr int SR = WT::SR, SC = WT::SC, KSTEPS = NB / M::KS;
  // LDS arena: the diagonal block D and X (L^-1 in step (b), U^-1 in step (c) and
  // the final solve) during steps (a)-(c); the 128-row multiplier strip S[k][i]
  // during step (d).
  constexpr size_t kDiagBytes = 2 * sizeof(C) * NB * (NB + 1);
  constexpr size_t kStripBytes = sizeof(C) * NB * 128;
  __shared__ __align__(16) char arena[kDiagBytes > kStripBytes ? kDiagBytes : kStripBytes];
  C (*D)[NB + 1] = (C (*)[NB + 1])arena;
  C (*X)[NB + 1] = (C (*)[NB + 1])(arena + sizeof(C) * NB * (NB + 1));
  C (*S)[128] = (C (*)[128])arena;
  __shared__ double pst[3];
  const int n = a.d.n;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int qi = blockIdx.x;
  const size_t nn = (size_t)n * n;
  const C* G = a.gamma + (size_t)qi * nn;
  C* A = a.A + (size_t)qi * nn;
  C* B = a.B + (size_t)qi * nn;
  C* MT = a.MT + (size_t)qi * NB * n;
  const double2* x = a.chi0 + (size_t)qi * n;

  // A = 1 - s Gamma diag(X), B = Gamma
  for (size_t idx = t; idx < nn; idx += blockDim.x) {
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
  if (t == 0) { pst[0] = DBL_MAX; pst[1] = 0.0; pst[2] = 0.0; }
  __threadfence_block();
  __syncthreads();

  for (int j0 = 0; j0 < n; j0 += NB) {
    const int jb = min(NB, n - j0);
    const int ncols = (n - j0 - jb) + n;
    // (a) diagonal block: factor and invert
    for (int idx = t; idx < NB * NB; idx += blockDim.x) {
      const int r = idx / NB, c = idx - (idx / NB) * NB;
      D[r][c] = (r < jb && c < jb) ? A[(size_t)(j0 + r) * n + j0 + c] : cz<C>();
    }
    __syncthreads();
    factor_block<C, NB>(D, jb, pst);
    invert_lower<C, NB>(D, X, jb);
    for (int idx = t; idx < jb * jb; idx += blockDim.x) {
      const int r = idx / jb, c = idx - (idx / jb) * jb;
      A[(size_t)(j0 + r) * n + j0 + c] = D[r][c];
    }
    // (b) U_JK = L^-1 A_JK: each wave owns 32-column strips, all NB rows
    for (int cs = wave; cs * 32 < ncols; cs += kWaves) {
      WT acc[NB / 32];
#pragma unroll
      for (int rt = 0; rt < NB / 32; ++rt) acc[rt].zero();
#pragma unroll 2
      for (int ks = 0; ks < KSTEPS; ++ks) {
        C bv[SC];
#pragma unroll
        for (int y = 0; y < SC; ++y) {
          const int col = cs * 32 + y * M::TN + M::b_col(lane);
          const int k = ks * M::KS + M::b_k(lane);
          bv[y] = (col < ncols && k < jb) ? colptr(A, B, n, j0, jb, col)[(size_t)(j0 + k) * n] : cz<C>();
        }
#pragma unroll
        for (int rt = 0; rt < NB / 32; ++rt) {
          C av[SR];
#pragma unroll
          for (int xx = 0; xx < SR; ++xx) av[xx] = X[rt * 32 + xx * M::TM + M::a_row(lane)][ks * M::KS + M::a_k(lane)];
          acc[rt].mac(av, bv, false);
        }
      }
#pragma unroll
      for (int rt = 0; rt < NB / 32; ++rt) {
        acc[rt].store([&](int r, int c, C v) {
          const int row = rt * 32 + r, col = cs * 32 + c;
          if (row < jb && col < ncols) colptr(A, B, n, j0, jb, col)[(size_t)(j0 + row) * n] = v;
        });
      }
    }
    __syncthreads();
    invert_upper<C, NB>(D, X, jb);
    // (c) MT = U^-T A_IJ^T (rows k of the panel, columns i = all rows of A)
    for (int is = wave; is * 32 < n; is += kWaves) {
      WT acc[NB / 32];
#pragma unroll
      for (int rt = 0; rt < NB / 32; ++rt) acc[rt].zero();
#pragma unroll 2
      for (int ks = 0; ks < KSTEPS; ++ks) {
        C bv[SC];
#pragma unroll
        for (int y = 0; y < SC; ++y) {
          const int i = is * 32 + y * M::TN + M::b_col(lane);
          const int k = ks * M::KS + M::b_k(lane);
          bv[y] = (i < n && k < jb) ? A[(size_t)i * n + j0 + k] : cz<C>();
        }
#pragma unroll
        for (int rt = 0; rt < NB / 32; ++rt) {
          C av[SR];
#pragma unroll
          for (int xx = 0; xx < SR; ++xx) {
            const int row = rt * 32 + xx * M::TM + M::a_row(lane);      // output row c
            const int k = ks * M::KS + M::a_k(lane);
            av[xx] = X[k][row];                                          // (U^-1)^T[row][k]
          }
          acc[rt].mac(av, bv, false);
        }
      }
#pragma unroll
      for (int rt = 0; rt < NB / 32; ++rt) {
        acc[rt].store([&](int r, int c, C v) {
          const int row = rt * 32 + r, i = is * 32 + c;
          if (row < jb && i < n) MT[(size_t)row * n + i] = v;
        });
      }
    }
    __threadfence_block();
    __syncthreads();
    // (d) update of every row outside the panel: C[i][col] -= sum_k MT[k][i] U[k][col].
    // The workgroup stages the multipliers of a 128-row block in LDS; each wave
    // owns 32 rows of it and streams the 32-column tiles of the row panel U,
    // which the four waves read at about the same time (L1/L2 reuse).
    const int nct = (ncols + 31) / 32;
    for (int rb = 0; rb * 128 < n; ++rb) {
      __syncthreads();
      for (int idx = t; idx < NB * 128; idx += blockDim.x) {
        const int k = idx >> 7, x = idx & 127;
        const int i = rb * 128 + x;
        S[k][x] = (k < jb && i < n) ? MT[(size_t)k * n + i] : cz<C>();
      }
      __syncthreads();
      const int i0 = rb * 128 + wave * 32;
      if (i0 >= n || (i0 >= j0 && i0 + 32 <= j0 + jb)) continue;
      for (int ct = 0; ct < nct; ++ct) {
        WT acc;
        C* cb[SC];
        bool cok[SC];
#pragma unroll
        for (int y = 0; y < SC; ++y) {
          const int col = ct * 32 + y * M::TN + M::b_col(lane);
          cok[y] = col < ncols;
          cb[y] = colptr(A, B, n, j0, jb, cok[y] ? col : 0);
        }
        acc.load([&](int r, int c) -> C {
          const int i = i0 + r;
          const int y = c / M::TN;
          const bool ok = cok[y] && i < n && !(i >= j0 && i < j0 + jb);
          return ok ? cb[y][(size_t)i * n] : cz<C>();
        });
#pragma unroll 4
        for (int ks = 0; ks < KSTEPS; ++ks) {
          C av[SR], bv[SC];
          const int k = ks * M::KS + M::b_k(lane);
#pragma unroll
          for (int y = 0; y < SC; ++y)
            bv[y] = (cok[y] && k < jb) ? cb[y][(size_t)(j0 + k) * n] : cz<C>();
#pragma unroll
          for (int xx = 0; xx < SR; ++xx)
            av[xx] = S[ks * M::KS + M::a_k(lane)][wave * 32 + xx * M::TM + M::a_row(lane)];
          acc.mac(av, bv, true);
        }
        acc.store([&](int r, int c, C v) {
          const int i = i0 + r;
          const int y = c / M::TN;
          if (cok[y] && i < n && !(i >= j0 && i < j0 + jb)) cb[y][(size_t)i * n] = v;
        });
      }
    }
    __threadfence_block();
    __syncthreads();
  }

  // F_J = U_JJ^-1 B_J, then Phi <- alpha (F - Gamma) + (1 - alpha) Phi
  C* P = a.phi + (size_t)qi * nn;
  const T al = (T)a.alpha, be = (T)(1.0 - a.alpha);
  const bool mix = a.alpha != 1.0;
  for (int j0 = 0; j0 < n; j0 += NB) {
    const int jb = min(NB, n - j0);
    __syncthreads();
    for (int idx = t; idx < NB * NB; idx += blockDim.x) {
      const int r = idx / NB, c = idx - (idx / NB) * NB;
      D[r][c] = (r < jb && c < jb) ? A[(size_t)(j0 + r) * n + j0 + c] : cz<C>();
    }
    __syncthreads();
    // only the U part is needed (the L part is already applied)
    invert_upper<C, NB>(D, X, jb);
    for (int cs = wave; cs * 32 < n; cs += kWaves) {
      WT acc[NB / 32];
#pragma unroll
      for (int rt = 0; rt < NB / 32; ++rt) acc[rt].zero();
#pragma unroll 2
      for (int ks = 0; ks < KSTEPS; ++ks) {
        C bv[SC];
#pragma unroll
        for (int y = 0; y < SC; ++y) {
          const int col = cs * 32 + y * M::TN + M::b_col(lane);
          const int k = ks * M::KS + M::b_k(lane);
          bv[y] = (col < n && k < jb) ? B[(size_t)(j0 + k) * n + col] : cz<C>();
        }
#pragma unroll
        for (int rt = 0; rt < NB / 32; ++rt) {
          C av[SR];
#pragma unroll
          for (int xx = 0; xx < SR; ++xx) av[xx] = X[rt * 32 + xx * M::TM + M::a_row(lane)][ks * M::KS + M::a_k(lane)];
          acc[rt].mac(av, bv, false);
        }
      }
#pragma unroll
      for (int rt = 0; rt < NB / 32; ++rt) {
        acc[rt].store([&](int r, int c, C f) {
          const int row = rt * 32 + r, col = cs * 32 + c;
          if (row < jb && col < n) {
            const size_t idx = (size_t)(j0 + row) * n + col;
            const C g = G[idx];
            C v;
            v.x = f.x - g.x;
            v.y = f.y - g.y;
            if (mix) {
              const C old = P[idx];
              v.x = al * v.x + be * old.x;
              v.y = al * v.y + be * old.y;
            }
            P[idx] = v;
          }
        });
      }
    }
  }
  if (t == 0 && a.stats) {
    pq_bse_block_stats st;
    const double ratio = pst[1] > 0.0 ? pst[0] / pst[1] : 0.0;
    st.min_pivot = (float)ratio;
    st.growth = (float)pst[1];
    st.flags = (pst[2] > 0.0 ? 2 : 0) | (ratio < a.weak_ratio ? 1 : 0);
    st.reserved = 0;
    a.stats[qi] = st;
  }
}

template <typename T>
constexpr int panel_width() { return sizeof(T) == 4 ? 64 : 32; }

}  // namespace

size_t bse_ws_bytes(const pq_params& p, const Dims& d, int precision) {
  (void)p;
  const size_t es = precision == PQ_PREC_FP64 ? sizeof(double2) : sizeof(float2);
  const int nb = precision == PQ_PREC_FP64 ? panel_width<double>() : panel_width<float>();
  const size_t nn = (size_t)d.n * d.n;
  return align256(es * nn * d.Nq) * 2 + align256(es * (size_t)nb * d.n * d.Nq);
}

template <typename T>
static hipError_t run_bse(const Dims& d, int channel, double alpha, float weak, const void* gamma,
                          const double2* chi0, void* phi_io, pq_bse_block_stats* stats, void* ws,
                          hipStream_t s) {
  using C = typename cplx_of<T>::type;
  constexpr int NB = panel_width<T>();
  static const double kSign[4] = {1.0, 1.0, -1.0, 1.0};
  const size_t nn = (size_t)d.n * d.n;
  char* w = (char*)ws;
  BseArgs<T> a;
  a.d = d;
  a.sign = (T)kSign[channel];
  a.alpha = alpha;
  a.weak_ratio = weak;
  a.gamma = (const C*)gamma;
  a.chi0 = chi0;
  a.phi = (C*)phi_io;
  a.A = (C*)w;
  a.B = (C*)(w + align256(sizeof(C) * nn * d.Nq));
  a.MT = (C*)(w + 2 * align256(sizeof(C) * nn * d.Nq));
  a.stats = stats;
  hipLaunchKernelGGL((bse_gj_kernel<T, NB>), dim3(d.Nq), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_bse(const pq_params& p, const Dims& d, int channel, int precision,
                      const void* gamma, const double2* chi0, void* phi_io, double alpha,
                      pq_bse_block_stats* stats, void* ws, hipStream_t s) {
  if (precision == PQ_PREC_FP64) {
    if (p.storage != PQ_STORE_C128) return hipErrorInvalidValue;
    return run_bse<double>(d, channel, alpha, 1e-10f, gamma, chi0, phi_io, stats, ws, s);
  }
  if (p.storage != PQ_STORE_C64) return hipErrorInvalidValue;
  return run_bse<float>(d, channel, alpha, 1e-3f, gamma, chi0, phi_io, stats, ws, s);
}

}  // namespace pq
