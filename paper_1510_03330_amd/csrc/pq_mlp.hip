// Learned warm start: the small multilayer perceptron that maps model
// parameters to kernel functions (forward, backward, Adam), the factorised
// output head (an orthonormal basis of the training solutions, built by
// Gram-Schmidt, and the expansion of predicted coefficients in it), and the
// reducible vertex rebuilt from kernel values (second-level kernel
// approximation, Sec. "Two-level kernel approximations": Phi ~ K1(q) +
// K2(k;q) + K2(k';q)).
//
// Network: hidden layers h_l = tanh(h_{l-1} W_l^T + b_l), linear output.
// Parameters packed layer by layer as [W_l (out x in, row-major), b_l (out)].
// Every product runs on the bf16 matrix cores (v_mfma_f32_32x32x16_bf16) with
// FP32 accumulation: the weights enter as their bf16 copy (round to nearest
// even), the FP32 activations and gradients as two bf16 terms hi + lo, which
// carries them to about 2^-16 relative, so the products match FP32 operands
// with bf16 weights. Biases, activations and accumulation are FP32.
// Loss: mean squared error over all outputs.
#include <algorithm>
#include <utility>
#include <vector>

#include "pq_internal.h"

namespace pq {

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kGT = 64;          // C tile edge of one workgroup (2 x 2 waves of 32 x 32)
constexpr int kGK = 32;          // K depth staged per LDS round (two 16-deep matrix-core steps)
constexpr int kLd = kGK + 8;     // LDS row stride in bf16 (80 bytes: rows stay 16-byte aligned)

// C[m][n] = sum_k A(m, k) B(k, n) (+ bias[n]); epilogue 1: tanh; epilogue 2:
// multiply by (1 - E[m][n]^2) (tanh backward). A(m, k) = A[m sam + k sak] is
// FP32 and enters as hi + lo; B(k, n) = B[k sbk + n sbn] is the bf16 weight
// array (BSPLIT false, one term) or FP32 (BSPLIT true, hi + lo; the lo x lo
// product is dropped). A 64 x 64 tile per workgroup, LDS rounds of 32 in k,
// zero-filled outside the matrix.
template <bool BSPLIT>
__global__ __launch_bounds__(256) void gemm_mfma_kernel(int M, int N, int K, const float* A, long sam, long sak,
                                                        const void* Bv, long sbk, long sbn, float* C, long scm,
                                                        const float* bias, int epi, const float* E) {
  __shared__ __attribute__((aligned(16))) __bf16 Ahi[kGT][kLd];
  __shared__ __attribute__((aligned(16))) __bf16 Alo[kGT][kLd];
  __shared__ __attribute__((aligned(16))) __bf16 Bhi[kGT][kLd];     // stored [n][k]
  __shared__ __attribute__((aligned(16))) __bf16 Blo[BSPLIT ? kGT : 1][kLd];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w & 1, wn = w >> 1;
  const int m0 = blockIdx.y * kGT, n0 = blockIdx.x * kGT;
  const bool a_kfast = sak == 1, b_kfast = sbk == 1;
  floatx16 acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.f;
  for (int k0 = 0; k0 < K; k0 += kGK) {
#pragma unroll
    for (int i = 0; i < kGT * kGK / 256; ++i) {
      const int e = tid + 256 * i;
      const int am = a_kfast ? e / kGK : e % kGT, ak = a_kfast ? e % kGK : e / kGT;
      float av = 0.f;
      if (m0 + am < M && k0 + ak < K) av = A[(long)(m0 + am) * sam + (long)(k0 + ak) * sak];
      const __bf16 h = (__bf16)av;
      Ahi[am][ak] = h;
      Alo[am][ak] = (__bf16)(av - (float)h);
      const int bn = b_kfast ? e / kGK : e % kGT, bk = b_kfast ? e % kGK : e / kGT;
      const bool in = n0 + bn < N && k0 + bk < K;
      const long bi = (long)(k0 + bk) * sbk + (long)(n0 + bn) * sbn;
      if constexpr (BSPLIT) {
        const float bv = in ? ((const float*)Bv)[bi] : 0.f;
        const __bf16 hb = (__bf16)bv;
        Bhi[bn][bk] = hb;
        Blo[bn][bk] = (__bf16)(bv - (float)hb);
      } else {
        Bhi[bn][bk] = in ? ((const __bf16*)Bv)[bi] : (__bf16)0.f;
      }
    }
    __syncthreads();
    const int ar = wm * 32 + (lane & 31), br = wn * 32 + (lane & 31), kk = 8 * (lane >> 5);
#pragma unroll
    for (int ks = 0; ks < kGK; ks += 16) {
      const bf16x8 ah = *(const bf16x8*)&Ahi[ar][ks + kk];
      const bf16x8 al = *(const bf16x8*)&Alo[ar][ks + kk];
      const bf16x8 bh = *(const bf16x8*)&Bhi[br][ks + kk];
      if constexpr (BSPLIT) {
        const bf16x8 bl = *(const bf16x8*)&Blo[br][ks + kk];
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc, 0, 0, 0);
      }
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  // accumulator element v of lane l: row 8 (v / 4) + 4 (l / 32) + v % 4, column l % 32
  const int n = n0 + wn * 32 + (lane & 31);
  if (n >= N) return;
  const float b = bias ? bias[n] : 0.f;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int m = m0 + wm * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    if (m < M) {
      float val = acc[v] + b;
      if (epi == 1) val = tanhf(val);
      if (epi == 2) {
        const float e = E[(long)m * scm + n];
        val *= 1.f - e * e;
      }
      C[(long)m * scm + n] = val;
    }
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
    const size_t r = rq / d.Nq, q = rq - r * d.Nq;
    const double2 a = k1[rq], b = k2[rq * n + k], c = k2[rq * n + kp];
    phi[r * d.cs + (q * n + k) * n + kp] = from_d<C>(mk(a.x + b.x + c.x, a.y + b.y + c.y));
  }
}

// ---- factorised output head: orthonormal basis of the training outputs ----
// Rows y_i (i < rows, len floats each) are centred on their mean and
// orthonormalised in order by classical Gram-Schmidt with one
// re-orthogonalisation pass; sample i is then y_i = mean + sum_{j<=i} c_ij q_j.
// Dot products accumulate in FP64 over kParts fixed segments of the row and are
// summed in a fixed order (deterministic).

__device__ inline double block_sum256d(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// mean[x] = (1 / rows) sum_i Y[i][x]; Y[i][x] -= mean[x]
__global__ __launch_bounds__(256) void center_kernel(float* Y, int rows, size_t len, float* mean) {
  for (size_t x = (size_t)blockIdx.x * blockDim.x + threadIdx.x; x < len; x += (size_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < rows; ++i) s += Y[(size_t)i * len + x];
    const float mu = (float)(s / rows);
    mean[x] = mu;
    for (int i = 0; i < rows; ++i) Y[(size_t)i * len + x] -= mu;
  }
}

// part[j][b] = sum over segment b of Q_j[x] y[x] for j < nq, and of y[x]^2 for j = nq
__global__ __launch_bounds__(256) void dots_kernel(const float* Q, int nq, size_t len, const float* y,
                                                   double* part) {
  __shared__ double red[256];
  const size_t per = (len + gridDim.x - 1) / gridDim.x;
  const size_t lo = (size_t)blockIdx.x * per, hi = lo + per < len ? lo + per : len;
  for (int j = 0; j <= nq; ++j) {
    const float* q = j < nq ? Q + (size_t)j * len : y;
    double acc = 0.0;
    for (size_t x = lo + threadIdx.x; x < hi; x += blockDim.x) acc += (double)q[x] * (double)y[x];
    const double b = block_sum256d(acc, red);
    if (threadIdx.x == 0) part[(size_t)j * gridDim.x + blockIdx.x] = b;
  }
}

// r[j] = sum_b part[j][b] (in order), j <= nq
__global__ __launch_bounds__(256) void dots_reduce_kernel(const double* part, int nparts, int nq, double* r) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j > nq) return;
  double s = 0.0;
  for (int b = 0; b < nparts; ++b) s += part[(size_t)j * nparts + b];
  r[j] = s;
}

// y[x] -= sum_{j < nq} r[j] Q_j[x]
__global__ __launch_bounds__(256) void project_out_kernel(const float* Q, int nq, size_t len, const double* r,
                                                          float* y) {
  for (size_t x = (size_t)blockIdx.x * blockDim.x + threadIdx.x; x < len; x += (size_t)gridDim.x * blockDim.x) {
    double v = y[x];
    for (int j = 0; j < nq; ++j) v -= r[j] * (double)Q[(size_t)j * len + x];
    y[x] = (float)v;
  }
}

// Row i done: c[i][j] = r1[j] + r2[j] (j < i), c[i][i] = |y_i| after both
// passes; the row is kept (scaled to unit norm) when that norm exceeds 1e-6 of
// the centred row's, else it is dropped (set to zero: no new direction).
__global__ void basis_row_kernel(int i, int rows, const double* r1, const double* r2, const double* r3,
                                 double* c, double* rinv) {
  const int j = threadIdx.x + blockIdx.x * blockDim.x;
  const double nrm = sqrt(r3[0]), orig = sqrt(r1[i]);
  const bool keep = nrm > 1e-6 * orig && nrm > 0.0;
  if (j < rows) c[(size_t)i * rows + j] = j < i ? r1[j] + r2[j] : (j == i && keep ? nrm : 0.0);
  if (j == 0) *rinv = keep ? 1.0 / nrm : 0.0;
}

__global__ __launch_bounds__(256) void scale_row_kernel(float* y, size_t len, const double* rinv) {
  const double a = *rinv;
  for (size_t x = (size_t)blockIdx.x * blockDim.x + threadIdx.x; x < len; x += (size_t)gridDim.x * blockDim.x)
    y[x] = (float)(a * y[x]);
}

// scale = root mean square of c (rows x rows); out[i ld + j] = c[i][j] / scale
__global__ __launch_bounds__(256) void basis_coef_kernel(const double* c, int rows, float* out, int ld,
                                                         float* scale) {
  __shared__ double red[256];
  const size_t cnt = (size_t)rows * rows;
  double s = 0.0;
  for (size_t e = threadIdx.x; e < cnt; e += blockDim.x) s += c[e] * c[e];
  const double tot = block_sum256d(s, red);
  const double rms = tot > 0.0 ? sqrt(tot / (double)cnt) : 1.0;
  for (size_t e = threadIdx.x; e < cnt; e += blockDim.x)
    out[(e / rows) * (size_t)ld + e % rows] = (float)(c[e] / rms);
  if (threadIdx.x == 0) *scale = (float)rms;
}

// out[x] = mean[x] + scale sum_j coef[j] Q_j[x] (FP64 output)
__global__ __launch_bounds__(256) void expand_kernel(const float* Q, int rows, size_t len, const float* mean,
                                                     const float* coef, const float* scale, double* out) {
  const double sc = *scale;
  for (size_t x = (size_t)blockIdx.x * blockDim.x + threadIdx.x; x < len; x += (size_t)gridDim.x * blockDim.x) {
    double v = 0.0;
    for (int j = 0; j < rows; ++j) v += (double)coef[j] * (double)Q[(size_t)j * len + x];
    out[x] = (double)mean[x] + sc * v;
  }
}

constexpr int kBasisParts = 1024;

inline unsigned stream_blocks(size_t len) {
  return (unsigned)std::max<size_t>(1, std::min<size_t>(8192, (len + 255) / 256));
}

inline dim3 gemm_grid(int M, int N) { return dim3((N + kGT - 1) / kGT, (M + kGT - 1) / kGT); }

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
    // y[b][o] = sum_i h[b][i] W[o][i] + bias[o]
    hipLaunchKernelGGL((gemm_mfma_kernel<false>), gemm_grid(B, out), dim3(256), 0, s, B, out, in, h, (long)in, 1L,
                       (const void*)((const __bf16*)pb + off), 1L, (long)in, y, (long)out,
                       p + off + (size_t)out * in, l < nl - 1 ? 1 : 0, (const float*)nullptr);
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
    hipLaunchKernelGGL((gemm_mfma_kernel<true>), gemm_grid(out, in), dim3(256), 0, s, out, in, B, d, 1L,
                       (long)out, (const void*)hin, (long)in, 1L, gW, (long)in, (const float*)nullptr, 0,
                       (const float*)nullptr);
    hipLaunchKernelGGL(colsum_kernel, dim3((out + 255) / 256), dim3(256), 0, s, B, out, d, gW + (size_t)out * in);
    if (l > 0) {
      // dn[b][i] = (sum_o d[b][o] W[o][i]) (1 - hin[b][i]^2)
      hipLaunchKernelGGL((gemm_mfma_kernel<false>), gemm_grid(B, in), dim3(256), 0, s, B, in, out, d, (long)out,
                         1L, (const void*)((const __bf16*)pb + poff[l]), (long)in, 1L, dn, (long)in,
                         (const float*)nullptr, 2, hin);
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

size_t mlp_basis_ws_bytes(int rows) {
  return sizeof(double) * ((size_t)(rows + 1) * kBasisParts + 3 * (size_t)(rows + 1) + (size_t)rows * rows + 1);
}

hipError_t launch_mlp_basis(float* Y, int rows, size_t len, float* mean, float* coef, int ld, float* scale, void* ws,
                            hipStream_t s) {
  double* part = (double*)ws;
  double* r1 = part + (size_t)(rows + 1) * kBasisParts;
  double* r2 = r1 + rows + 1;
  double* r3 = r2 + rows + 1;
  double* c = r3 + rows + 1;
  double* rinv = c + (size_t)rows * rows;
  const unsigned nb = stream_blocks(len);
  const unsigned parts = (unsigned)std::min<size_t>(kBasisParts, (len + 255) / 256);
  hipLaunchKernelGGL(center_kernel, dim3(nb), dim3(256), 0, s, Y, rows, len, mean);
  for (int i = 0; i < rows; ++i) {
    float* y = Y + (size_t)i * len;
    const unsigned rb = (unsigned)((i + 1 + 255) / 256);
    hipLaunchKernelGGL(dots_kernel, dim3(parts), dim3(256), 0, s, (const float*)Y, i, len, (const float*)y, part);
    hipLaunchKernelGGL(dots_reduce_kernel, dim3(rb), dim3(256), 0, s, (const double*)part, (int)parts, i, r1);
    hipLaunchKernelGGL(project_out_kernel, dim3(nb), dim3(256), 0, s, (const float*)Y, i, len, (const double*)r1, y);
    hipLaunchKernelGGL(dots_kernel, dim3(parts), dim3(256), 0, s, (const float*)Y, i, len, (const float*)y, part);
    hipLaunchKernelGGL(dots_reduce_kernel, dim3(rb), dim3(256), 0, s, (const double*)part, (int)parts, i, r2);
    hipLaunchKernelGGL(project_out_kernel, dim3(nb), dim3(256), 0, s, (const float*)Y, i, len, (const double*)r2, y);
    hipLaunchKernelGGL(dots_kernel, dim3(parts), dim3(256), 0, s, (const float*)Y, 0, len, (const float*)y, part);
    hipLaunchKernelGGL(dots_reduce_kernel, dim3(1), dim3(256), 0, s, (const double*)part, (int)parts, 0, r3);
    hipLaunchKernelGGL(basis_row_kernel, dim3((rows + 255) / 256), dim3(256), 0, s, i, rows, (const double*)r1,
                       (const double*)r2, (const double*)r3, c, rinv);
    hipLaunchKernelGGL(scale_row_kernel, dim3(nb), dim3(256), 0, s, y, len, (const double*)rinv);
  }
  hipLaunchKernelGGL(basis_coef_kernel, dim3(1), dim3(256), 0, s, (const double*)c, rows, coef, ld, scale);
  return hipGetLastError();
}

hipError_t launch_mlp_expand(const float* Q, int rows, size_t len, const float* mean, const float* coef,
                             const float* scale, double* out, hipStream_t s) {
  hipLaunchKernelGGL(expand_kernel, dim3(stream_blocks(len)), dim3(256), 0, s, Q, rows, len, mean, coef, scale, out);
  return hipGetLastError();
}

}  // namespace pq
