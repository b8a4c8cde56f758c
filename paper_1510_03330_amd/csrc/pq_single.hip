// Single-particle kernels: Dyson equation with the filling condition, the
// bubbles X_ph / X_pp of the Bethe-Salpeter equations, and linear mixing of
// Sigma with its convergence norm. All FP64.
#include <math.h>

#include <algorithm>

#include "pq_internal.h"

namespace pq {

namespace {

constexpr int kThreads = 256;
constexpr int kMaxNk = 1024;

struct DysonArgs {
  Dims d;
  double beta, t, tp, D, filling, mu_fixed, U;
  int mu_mode, local;
  const double2* sigma;
  double2* g;
  double* mu_out;
};

__device__ inline double eps_of(int K, const Dims& d, double t, double tp) {
  int kx = K / d.Ly, ky = K - (K / d.Ly) * d.Ly;
  double cx = cos(2.0 * M_PI * kx / d.Lx), cy = cos(2.0 * M_PI * ky / d.Ly);
  return -2.0 * t * (cx + cy) - 4.0 * tp * cx * cy;
}

__device__ inline double nu_of(int n, double beta) { return (2 * n + 1) * M_PI / beta; }

// Sigma on the G grid: stored on the extended box, zero beyond.
__device__ inline double2 sigma_at(const DysonArgs& a, int n, int K) {
  const int h = a.d.Nve / 2;
  if (n < -h || n > h - 1) return mk(0.0, 0.0);
  return a.sigma[(size_t)(n + h) * a.d.Nk + K];
}

// Lattice G at mu for G-grid row g and momentum K.
__device__ inline double2 g_lattice(const DysonArgs& a, const double* eps, double mu, int gi, int K) {
  int n = gi - a.d.NG / 2;
  double nu = nu_of(n, a.beta);
  double2 s = sigma_at(a, n, K);
  double2 z = mk(mu - eps[K] - s.x, nu - s.y);
  return crecip(z);
}

// Total density per spin at mu: 1/2 + T/N sum Re G + the exact tail beyond the grid.
__device__ double density(const DysonArgs& a, const double* eps, double mu, double* red) {
  const Dims& d = a.d;
  const double T = 1.0 / a.beta;
  double acc = 0.0;
  for (int idx = threadIdx.x; idx < d.NG * d.Nk; idx += blockDim.x) {
    int gi = idx / d.Nk, K = idx - gi * d.Nk;
    acc += g_lattice(a, eps, mu, gi, K).x;
  }
  double sre = block_sum(acc, red);
  double tail = 0.0;
  for (int K = threadIdx.x; K < d.Nk; K += blockDim.x) {
    double xi = eps[K] - mu;
    double partial = 0.0;
    for (int n = 0; n < d.NG / 2; ++n) {
      double nu = nu_of(n, a.beta);
      partial += 1.0 / (nu * nu + xi * xi);
    }
    double full = fabs(xi) < 1e-300 ? a.beta * a.beta / 8.0
                                    : a.beta * tanh(a.beta * xi / 2.0) / (4.0 * xi);
    tail += -xi * (full - partial);
  }
  double stail = block_sum(tail, red);
  return 0.5 + (T / d.Nk) * sre + 2.0 * (T / d.Nk) * stail;
}

__global__ __launch_bounds__(kThreads) void dyson_kernel(DysonArgs a) {
  __shared__ double red[kThreads];
  __shared__ double eps[kMaxNk];
  const Dims& d = a.d;
  for (int K = threadIdx.x; K < d.Nk; K += blockDim.x) eps[K] = a.local ? 0.0 : eps_of(K, d, a.t, a.tp);
  __syncthreads();
  double mu = a.mu_fixed;
  if (!a.local && a.mu_mode == 1) {
    double emin = 1e300, emax = -1e300;
    for (int K = threadIdx.x; K < d.Nk; K += blockDim.x) {
      emin = fmin(emin, eps[K]);
      emax = fmax(emax, eps[K]);
    }
    emin = -block_max(-emin, red);
    emax = block_max(emax, red);
    double lo = emin - 10.0 - fabs(a.U), hi = emax + 10.0 + fabs(a.U);
    for (int it = 0; it < 200; ++it) {
      double mid = 0.5 * (lo + hi);
      double nn = 2.0 * density(a, eps, mid, red);
      if (nn > a.filling) hi = mid; else lo = mid;
      if (hi - lo < 1e-14) break;
    }
    mu = 0.5 * (lo + hi);
  }
  for (int idx = threadIdx.x; idx < d.NG * d.Nk; idx += blockDim.x) {
    int gi = idx / d.Nk, K = idx - gi * d.Nk;
    double2 gv;
    if (a.local) {
      int n = gi - d.NG / 2;
      double nu = nu_of(n, a.beta);
      double sg = nu > 0 ? 1.0 : (nu < 0 ? -1.0 : 0.0);
      double c = 2.0 / (a.D * a.D);
      double2 g0 = mk(0.0, c * (nu - sg * sqrt(nu * nu + a.D * a.D)));
      double2 s = sigma_at(a, n, K);
      gv = crecip(csub(crecip(g0), s));
    } else {
      gv = g_lattice(a, eps, mu, gi, K);
    }
    a.g[idx] = gv;
  }
  if (threadIdx.x == 0) *a.mu_out = a.local ? 0.0 : mu;
}

struct BubbleArgs {
  Dims d;
  double T;
  const double2* g;
  double2* xph;
  double2* xpp;
};

__global__ __launch_bounds__(kThreads) void bubble_kernel(BubbleArgs a) {
  const Dims& d = a.d;
  size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)d.Nq * d.n) return;
  int qi = (int)(idx / d.n), ki = (int)(idx - (size_t)qi * d.n);
  int jm = qi / d.Nk, Q = qi - jm * d.Nk;
  int m = jm - (d.Nv / 2 - 1);
  int in = ki / d.Nk, K = ki - in * d.Nk;
  int n = in - d.Nv / 2;
  const int h = d.NG / 2;
  double2 gk = a.g[(size_t)(n + h) * d.Nk + K];
  double2 gkq = a.g[(size_t)(n + m + h) * d.Nk + kadd(K, Q, d.Lx, d.Ly)];
  double2 gqk = a.g[(size_t)(m - n - 1 + h) * d.Nk + ksub(Q, K, d.Lx, d.Ly)];
  a.xph[idx] = cscale(cmul(gk, gkq), a.T / d.Nk);
  a.xpp[idx] = cscale(cmul(gk, gqk), a.T / (2.0 * d.Nk));
}

__global__ __launch_bounds__(kThreads) void mix_kernel(int count, const double2* snew, double2* sio,
                                                       double alpha, double* dnorm, double* smax) {
  __shared__ double red[kThreads];
  double mx = 0.0, bad = 0.0, sm = 0.0;
  for (int i = threadIdx.x; i < count; i += blockDim.x) {
    double2 a = snew[i], b = sio[i];
    double dr = a.x - b.x, di = a.y - b.y;
    double dd = hypot(dr, di);
    if (!isfinite(a.x) || !isfinite(a.y)) bad = 1.0;
    mx = fmax(mx, dd);
    const double2 c = mk(alpha * a.x + (1.0 - alpha) * b.x, alpha * a.y + (1.0 - alpha) * b.y);
    sio[i] = c;
    sm = fmax(sm, hypot(c.x, c.y));
  }
  mx = block_max(mx, red);
  bad = block_max(bad, red);
  sm = block_max(sm, red);
  if (threadIdx.x == 0) {
    *dnorm = bad > 0.0 ? __builtin_nan("") : mx;
    if (smax) *smax = sm;
  }
}

// storage conversion of a vertex array (complex64 <-> complex128, or a copy)
template <typename S, typename D>
__global__ __launch_bounds__(kThreads) void convert_kernel(const S* src, D* dst, size_t count) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
    const S v = src[i];
    D w;
    w.x = v.x;
    w.y = v.y;
    dst[i] = w;
  }
}

// F = Gamma + Phi over a vertex array (Eq. PA_F_G)
template <typename C>
__global__ __launch_bounds__(kThreads) void vertex_sum_kernel(const C* a, const C* b, C* f, size_t count) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
    const C x = a[i], y = b[i];
    C z;
    z.x = x.x + y.x;
    z.y = x.y + y.y;
    f[i] = z;
  }
}

}  // namespace

hipError_t launch_vertex_sum(const void* a, const void* b, void* f, int storage, size_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<size_t>(16384, (count + kThreads - 1) / kThreads);
  if (storage == PQ_STORE_C64)
    hipLaunchKernelGGL((vertex_sum_kernel<float2>), dim3(blocks), dim3(kThreads), 0, s, (const float2*)a,
                       (const float2*)b, (float2*)f, count);
  else
    hipLaunchKernelGGL((vertex_sum_kernel<double2>), dim3(blocks), dim3(kThreads), 0, s, (const double2*)a,
                       (const double2*)b, (double2*)f, count);
  return hipGetLastError();
}

hipError_t launch_convert(const void* src, int src_storage, void* dst, int dst_storage, size_t count,
                          hipStream_t s) {
  const unsigned blocks = (unsigned)std::min<size_t>(8192, (count + kThreads - 1) / kThreads);
  if (count == 0) return hipSuccess;
  if (src_storage == PQ_STORE_C64 && dst_storage == PQ_STORE_C128)
    hipLaunchKernelGGL((convert_kernel<float2, double2>), dim3(blocks), dim3(kThreads), 0, s,
                       (const float2*)src, (double2*)dst, count);
  else if (src_storage == PQ_STORE_C128 && dst_storage == PQ_STORE_C64)
    hipLaunchKernelGGL((convert_kernel<double2, float2>), dim3(blocks), dim3(kThreads), 0, s,
                       (const double2*)src, (float2*)dst, count);
  else if (src_storage == PQ_STORE_C64)
    hipLaunchKernelGGL((convert_kernel<float2, float2>), dim3(blocks), dim3(kThreads), 0, s,
                       (const float2*)src, (float2*)dst, count);
  else
    hipLaunchKernelGGL((convert_kernel<double2, double2>), dim3(blocks), dim3(kThreads), 0, s,
                       (const double2*)src, (double2*)dst, count);
  return hipGetLastError();
}

hipError_t launch_dyson(const pq_params& p, const Dims& d, const double2* sigma, double2* g,
                        double* mu_out, hipStream_t s) {
  if (d.Nk > kMaxNk) return hipErrorInvalidValue;
  DysonArgs a{d, p.beta, p.t, p.tp, p.D, p.filling, p.mu_fixed, p.U, p.mu_mode, d.Nk == 1 ? 1 : 0,
              sigma, g, mu_out};
  hipLaunchKernelGGL(dyson_kernel, dim3(1), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_bubbles(const pq_params& p, const Dims& d, const double2* g, double2* xph,
                          double2* xpp, hipStream_t s) {
  BubbleArgs a{d, 1.0 / p.beta, g, xph, xpp};
  size_t total = (size_t)d.Nq * d.n;
  unsigned blocks = (unsigned)((total + kThreads - 1) / kThreads);
  hipLaunchKernelGGL(bubble_kernel, dim3(blocks), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_mix(const Dims& d, const double2* snew, double2* sio, double alpha,
                      double* dnorm, hipStream_t s, double* smax) {
  hipLaunchKernelGGL(mix_kernel, dim3(1), dim3(kThreads), 0, s, d.Nve * d.Nk, snew, sio, alpha, dnorm, smax);
  return hipGetLastError();
}

}  // namespace pq

// ------------------------------------------------------ HBM streaming probes
// Reference rates for the memory-bound stages: float4 grid-stride streams,
// eight 16-byte accesses in flight per thread and iteration, non-temporal
// loads (and stores for the copy), up to 16384 workgroups: the fastest of the
// shapes tried on this device (unroll 4, 8, 16; 1024 to 16384 workgroups;
// with and without the non-temporal hint).
namespace pq {
namespace {

constexpr int kHbmUnroll = 8;
typedef float hf4 __attribute__((ext_vector_type(4)));

__device__ inline hf4 nt_ld(const hf4* p) { return __builtin_nontemporal_load(p); }

__global__ __launch_bounds__(256) void hbm_copy_kernel(const hf4* __restrict__ src, hf4* __restrict__ dst,
                                                       size_t count) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + (kHbmUnroll - 1) * stride < count; i += kHbmUnroll * stride) {
    hf4 v[kHbmUnroll];
#pragma unroll
    for (int u = 0; u < kHbmUnroll; ++u) v[u] = nt_ld(src + i + u * stride);
#pragma unroll
    for (int u = 0; u < kHbmUnroll; ++u) __builtin_nontemporal_store(v[u], dst + i + u * stride);
  }
  for (; i < count; i += stride) dst[i] = src[i];
}

__global__ __launch_bounds__(256) void hbm_read_kernel(const hf4* __restrict__ src, size_t count,
                                                       float* __restrict__ out) {
  __shared__ float red[256];
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  float acc = 0.f;
  for (; i + (kHbmUnroll - 1) * stride < count; i += kHbmUnroll * stride) {
    hf4 v[kHbmUnroll];
#pragma unroll
    for (int u = 0; u < kHbmUnroll; ++u) v[u] = nt_ld(src + i + u * stride);
#pragma unroll
    for (int u = 0; u < kHbmUnroll; ++u) acc += (v[u].x + v[u].y) + (v[u].z + v[u].w);
  }
  for (; i < count; i += stride) acc += (src[i].x + src[i].y) + (src[i].z + src[i].w);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void hbm_write_kernel(hf4* __restrict__ dst, size_t count, float value) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const hf4 v = {value, value, value, value};
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) dst[i] = v;
}

}  // namespace

hipError_t launch_hbm_stream(int mode, const void* src, void* dst, size_t bytes, hipStream_t s) {
  const size_t count = bytes / 16;
  const unsigned blocks = (unsigned)std::max<size_t>(1, std::min<size_t>(kHbmStreamBlocks, (count + 255) / 256));
  if (mode == 0)
    hipLaunchKernelGGL(hbm_copy_kernel, dim3(blocks), dim3(256), 0, s, (const hf4*)src, (hf4*)dst, count);
  else if (mode == 1)
    hipLaunchKernelGGL(hbm_read_kernel, dim3(blocks), dim3(256), 0, s, (const hf4*)src, count, (float*)dst);
  else
    hipLaunchKernelGGL(hbm_write_kernel, dim3(blocks), dim3(256), 0, s, (hf4*)dst, count, 1.0f);
  return hipGetLastError();
}

}  // namespace pq
