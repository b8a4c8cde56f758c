// Device-side helpers shared by the parquet kernels: complex arithmetic on
// float2/double2, compound-index and momentum arithmetic, block reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "parquet.h"

namespace pq {

// ----------------------------------------------------------------- sizes
struct Dims {
  int Lx, Ly, Nk, Nv, NW, f, Nve, NWe, NG, n, Nq, ntau;
  // elements between the channel arrays of a vertex (Phi, Gamma): Nq n^2 for
  // one instance's [4][Nq][n][n]; K Nq n^2 in a batch of K instances of one
  // box, whose vertices are stored [4][K][Nq][n][n]
  long long cs;
};

// ------------------------------------------------------------- complex
template <typename T> struct cplx_of;
template <> struct cplx_of<float> { using type = float2; };
template <> struct cplx_of<double> { using type = double2; };

__host__ __device__ inline double2 mk(double r, double i) { return make_double2(r, i); }
__host__ __device__ inline float2 mkf(float r, float i) { return make_float2(r, i); }

__device__ inline double2 cadd(double2 a, double2 b) { return mk(a.x + b.x, a.y + b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return mk(a.x - b.x, a.y - b.y); }
__device__ inline double2 cmul(double2 a, double2 b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cscale(double2 a, double s) { return mk(a.x * s, a.y * s); }
__device__ inline double2 cdiv(double2 a, double2 b) {
  // Smith's algorithm
  if (fabs(b.x) >= fabs(b.y)) {
    double r = b.y / b.x, d = b.x + b.y * r;
    return mk((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  } else {
    double r = b.x / b.y, d = b.x * r + b.y;
    return mk((a.x * r + a.y) / d, (a.y * r - a.x) / d);
  }
}
__device__ inline double2 crecip(double2 b) { return cdiv(mk(1.0, 0.0), b); }

__device__ inline float2 cadd(float2 a, float2 b) { return mkf(a.x + b.x, a.y + b.y); }
__device__ inline float2 csub(float2 a, float2 b) { return mkf(a.x - b.x, a.y - b.y); }
__device__ inline float2 cmul(float2 a, float2 b) {
  return mkf(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline float2 cscale(float2 a, float s) { return mkf(a.x * s, a.y * s); }
__device__ inline float2 cdiv(float2 a, float2 b) {
  if (fabsf(b.x) >= fabsf(b.y)) {
    float r = b.y / b.x, d = b.x + b.y * r;
    return mkf((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  } else {
    float r = b.x / b.y, d = b.x * r + b.y;
    return mkf((a.x * r + a.y) / d, (a.y * r - a.x) / d);
  }
}

__device__ inline double2 to_d(float2 a) { return mk((double)a.x, (double)a.y); }
__device__ inline double2 to_d(double2 a) { return a; }
template <typename C> __device__ inline C from_d(double2 a);
template <> __device__ inline double2 from_d<double2>(double2 a) { return a; }
template <> __device__ inline float2 from_d<float2>(double2 a) { return mkf((float)a.x, (float)a.y); }

__device__ inline double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }

// ------------------------------------------------ index arithmetic
// Fermionic box index of n (caller checks range): n + Nv/2.
__device__ inline bool in_fbox(int n, int Nv) { return n >= -Nv / 2 && n <= Nv / 2 - 1; }
__device__ inline bool in_bbox(int m, int Nv) { return m >= -(Nv / 2 - 1) && m <= Nv / 2 - 1; }
__device__ inline int kx_of(int K, int Ly) { return K / Ly; }
__device__ inline int ky_of(int K, int Ly) { return K - (K / Ly) * Ly; }
__device__ inline int kadd(int a, int b, int Lx, int Ly) {
  int ax = a / Ly, ay = a - ax * Ly, bx = b / Ly, by = b - bx * Ly;
  int x = ax + bx; if (x >= Lx) x -= Lx;
  int y = ay + by; if (y >= Ly) y -= Ly;
  return x * Ly + y;
}
__device__ inline int ksub(int a, int b, int Lx, int Ly) {
  int ax = a / Ly, ay = a - ax * Ly, bx = b / Ly, by = b - bx * Ly;
  int x = ax - bx; if (x < 0) x += Lx;
  int y = ay - by; if (y < 0) y += Ly;
  return x * Ly + y;
}

// ------------------------------------------------------ reductions
// Deterministic block reduction of doubles (fixed tree). blockDim.x must be a
// power of two <= 1024; `red` is LDS of blockDim.x doubles.
__device__ inline double block_sum(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

__device__ inline double block_max(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
    if (t < s) red[t] = fmax(red[t], red[t + s]);
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

// Work-item order for a 2-D grid on the 8 XCDs of the chip. Workgroups are
// dealt to the XCDs round-robin by linear id; this returns the logical id so
// that the workgroups one XCD receives are consecutive in logical order (the
// first eighth of the work goes to XCD 0, and so on), which keeps the operands
// that neighbouring work items share in that XCD's own L2. A tail that does
// not divide by 8 keeps the identity order.
__device__ inline unsigned xcd_linear() {
  const unsigned total = gridDim.x * gridDim.y;
  const unsigned lin = blockIdx.y * gridDim.x + blockIdx.x;
  const unsigned per = total >> 3;
  return lin < (per << 3) ? (lin & 7u) * per + (lin >> 3) : lin;
}

}  // namespace pq
