// Learned warm start: the small multilayer perceptron that maps model
// parameters to kernel functions (forward, backward, Adam), and the reducible
// vertex rebuilt from kernel values (second-level kernel approximation, Sec.
// "Two-level kernel approximations": Phi ~ K1(q) + K2(k;q) + K2(k';q)).
//
// Network: hidden layers h_l = tanh(h_{l-1} W_l^T + b_l), linear output.
// Parameters packed layer by layer as [W_l (out x in, row-major), b_l (out)];
// the forward and input-gradient products use the bf16 copy of the weights
// (round to nearest even), biases, activations and accumulation are FP32.
// Loss: mean squared error over all outputs.
#include <algorithm>
#include <utility>
#include <vector>

#include "pq_internal.h"

namespace pq {

namespace {

constexpr int kT = 16;          // GEMM tile edge (16 x 16 threads)

// C[m][n] = sum_k A(m, k) B(k, n) (+ bias[n]); epilogue 1: tanh; epilogue 2:
// multiply by (1 - E[m][n]^2) (tanh backward). Strided operands; B is bf16
// when BBF. Shapes are small (<= a few thousand), so plain LDS tiles suffice.
template <bool BBF>
__global__ __launch_bounds__(kT* kT) void gemm_kernel(int M, int N, int K, const float* A, int sam, int sak,
                                                      const void* Bv, int sbk, int sbn, float* C, int scm,
                                                      const float* bias, int epi, const float* E) {
  __shared__ float As[kT][kT + 1];
  __shared__ float Bs[kT][kT + 1];
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int m = blockIdx.y * kT + ty, n = blockIdx.x * kT + tx;
  float acc = 0.f;
  for (int k0 = 0; k0 < K; k0 += kT) {
    const int ka = k0 + tx, kb = k0 + ty;
    As[ty][tx] = (m < M && ka < K) ? A[(size_t)m * sam + (size_t)ka * sak] : 0.f;
    float bv = 0.f;
    if (kb < K && n < N) {
      const size_t bi = (size_t)kb * sbk + (size_t)n * sbn;
      if constexpr (BBF) {
        bv = (float)((const __bf16*)Bv)[bi];
      } else {
        bv = ((const float*)Bv)[bi];
      }
    }
    Bs[ty][tx] = bv;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kT; ++k) acc = fmaf(As[ty][k], Bs[k][tx], acc);
    __syncthreads();
  }
  if (m < M && n < N) {
    if (bias) acc += bias[n];
    if (epi == 1) acc = tanhf(acc);
    if (epi == 2) {
      const float e = E[(size_t)m * scm + n];
      acc *= 1.f - e * e;
    }
    C[(size_t)m * scm + n] = acc;
  }
}

// db[o] = sum_b d[b][o]
__global__ __launch_bounds__(256) void colsum_kernel(int B, int O, const float* d, float* db) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= O) return;
  float s = 0.f;
  for (int b = 0; b < B; ++b) s += d[(size_t)b * O + o];
  db[o] = s;
}

// d = 2 (y - t) / count and loss = mean (y - t)^2, in two passes with a fixed
// summation order (deterministic): each workgroup of the first pass sums a
// fixed grid-stride subset into part[blockIdx.x], the second (one workgroup)
// sums the parts.
__device__ inline float block_sum256(float v, float* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  return red[0];
}

__global__ __launch_bounds__(256) void mse_partial_kernel(size_t count, const float* y, const float* t, float* d,
                                                          float* part) {
  __shared__ float red[256];
  float s = 0.f;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
    const float e = y[i] - t[i];
    d[i] = 2.f * e / (float)count;
    s += e * e;
  }
  const float b = block_sum256(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = b;
}

__global__ __launch_bounds__(256) void mse_final_kernel(int nparts, const float* part, size_t count, float* loss) {
  __shared__ float red[256];
  float s = 0.f;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) s += part[i];
  const float b = block_sum256(s, red);
  if (threadIdx.x == 0) *loss = b / (float)count;
}

__global__ __launch_bounds__(256) void adam_kernel(size_t count, float* p, __bf16* pb, float* m, float* v,
                                                   const float* g, float lr, float b1, float b2, float eps,
                                                   float c1, float c2) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float w = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = w;
  pb[i] = (__bf16)w;
}

__global__ __launch_bounds__(256) void to_bf16_kernel(size_t count, const float* p, __bf16* pb) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) pb[i] = (__bf16)p[i];
}

template <typename C>
__global__ __launch_bounds__(256) void phi_from_kernels_kernel(Dims d, const double2* k1, const double2* k2,
                                                               C* phi) {
  const size_t n = d.n, total = 4 * (size_t)d.Nq * n * n;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const size_t kp = i % n, k = (i / n) % n, rq = i / (n * n);      // rq = r Nq + q
    const double2 a = k1[rq], b = k2[rq * n + k], c = k2[rq * n + kp];
    phi[i] = from_d<C>(mk(a.x + b.x + c.x, a.y + b.y + c.y));
  }
}

inline dim3 tiles(int M, int N) { return dim3((N + kT - 1) / kT, (M + kT - 1) / kT); }

}  // namespace

size_t mlp_count(const int32_t* w, int nl) {
  size_t c = 0;
  for (int l = 0; l < nl; ++l) c += (size_t)w[l + 1] * w[l] + w[l + 1];
  return c;
}

hipError_t launch_mlp_forward(const int32_t* w, int nl, const void* pb, const float* p, const float* x, float* acts,
                              int B, hipStream_t s) {
  size_t off = 0, aoff = 0;
  const float* h = x;
  for (int l = 0; l < nl; ++l) {
    const int in = w[l], out = w[l + 1];
    float* y = acts + aoff;
    hipLaunchKernelGGL((gemm_kernel<true>), tiles(B, out), dim3(kT, kT), 0, s, B, out, in, h, in, 1,
                       (const void*)((const __bf16*)pb + off), 1, in, y, out, p + off + (size_t)out * in,
                       l < nl - 1 ? 1 : 0, (const float*)nullptr);
    off += (size_t)out * in + out;
    aoff += (size_t)B * out;
    h = y;
  }
  return hipGetLastError();
}

hipError_t launch_mlp_backward(const int32_t* w, int nl, const void* pb, const float* x, const float* acts,
                               const float* target, float* grad, float* loss, float* scratch, int B, hipStream_t s) {
  int maxw = 0;
  for (int l = 0; l <= nl; ++l) maxw = w[l] > maxw ? w[l] : maxw;
  std::vector<size_t> poff(nl), aoff(nl);
  size_t po = 0, ao = 0;
  for (int l = 0; l < nl; ++l) {
    poff[l] = po;
    aoff[l] = ao;
    po += (size_t)w[l + 1] * w[l] + w[l + 1];
    ao += (size_t)B * w[l + 1];
  }
  float* d = scratch;
  float* dn = scratch + (size_t)B * maxw;
  const size_t nout = (size_t)B * w[nl];
  // the partial sums of the loss live in dn, which the layer loop below
  // writes only after the final pass has read them
  const int nparts = (int)std::min<size_t>({(size_t)1024, (nout + 255) / 256, (size_t)B * maxw});
  hipLaunchKernelGGL(mse_partial_kernel, dim3(nparts), dim3(256), 0, s, nout, acts + aoff[nl - 1], target, d, dn);
  hipLaunchKernelGGL(mse_final_kernel, dim3(1), dim3(256), 0, s, nparts, (const float*)dn, nout, loss);
  for (int l = nl - 1; l >= 0; --l) {
    const int in = w[l], out = w[l + 1];
    const float* hin = l == 0 ? x : acts + aoff[l - 1];
    float* gW = grad + poff[l];
    // gW[o][i] = sum_b d[b][o] hin[b][i]
    hipLaunchKernelGGL((gemm_kernel<false>), tiles(out, in), dim3(kT, kT), 0, s, out, in, B, d, 1, out,
                       (const void*)hin, in, 1, gW, in, (const float*)nullptr, 0, (const float*)nullptr);
    hipLaunchKernelGGL(colsum_kernel, dim3((out + 255) / 256), dim3(256), 0, s, B, out, d, gW + (size_t)out * in);
    if (l > 0) {
      // dn[b][i] = (sum_o d[b][o] W[o][i]) (1 - hin[b][i]^2)
      hipLaunchKernelGGL((gemm_kernel<true>), tiles(B, in), dim3(kT, kT), 0, s, B, in, out, d, out, 1,
                         (const void*)((const __bf16*)pb + poff[l]), in, 1, dn, in, (const float*)nullptr, 2, hin);
      std::swap(d, dn);
    }
  }
  return hipGetLastError();
}

hipError_t launch_mlp_adam(float* p, void* pb, float* m, float* v, const float* g, size_t count, float lr, float b1,
                           float b2, float eps, int step, hipStream_t s) {
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, count, p, (__bf16*)pb, m,
                     v, g, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_mlp_to_bf16(const float* p, void* pb, size_t count, hipStream_t s) {
  hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, count, p, (__bf16*)pb);
  return hipGetLastError();
}

hipError_t launch_phi_from_kernels(const pq_params& p, const Dims& d, const double2* k1, const double2* k2,
                                   void* phi, hipStream_t s) {
  const size_t total = 4 * (size_t)d.Nq * d.n * d.n;
  const unsigned blocks = (unsigned)std::min<size_t>(65536, (total + 255) / 256);
  if (p.storage == PQ_STORE_C64)
    hipLaunchKernelGGL((phi_from_kernels_kernel<float2>), dim3(blocks), dim3(256), 0, s, d, k1, k2, (float2*)phi);
  else
    hipLaunchKernelGGL((phi_from_kernels_kernel<double2>), dim3(blocks), dim3(256), 0, s, d, k1, k2, (double2*)phi);
  return hipGetLastError();
}

}  // namespace pq
