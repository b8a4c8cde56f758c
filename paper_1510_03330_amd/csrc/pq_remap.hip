// Kernel functions (two-level kernel approximation) and the channel remap of
// the parquet equations (Eqs. PA_Gamma_dm, PA_Gamma_st).
//
// Remap data flow. Every term of Gamma_r at (q, k, k') reads a reducible
// vertex whose first fermionic argument is the output's k. For fixed k and a
// fixed pair of output frequencies (m, n') the Nk x Nk momentum tile (Q, K')
// of a term is a permutation of one Nk x Nk source tile (Q_p, K_b) of
// Phi_r[p][k][b] at one frequency pair (m_p, n_b):
//   ph-bar  (d,m):  m_p = n'-n,       n_b = n+m      Q_p = K'-K,    K_b = K+Q
//   pp      (s,t):  m_p = n+n'+m+1,   n_b = n'       Q_p = K+K'+Q,  K_b = K'
//   st-1    (d,m):  m_p = n'-n,       n_b = m-n'-1   Q_p = K'-K,    K_b = Q-K'
//   st-2    (d,m):  m_p = m-n-n'-1,   n_b = n'       Q_p = Q-K-K',  K_b = K'
// (frequency shifts of ferm+bos, ferm-ferm, ferm+ferm+bos, bos-ferm, bos-ferm-ferm
// sums). A workgroup owns one (k, m) output plane, loads each source tile once
// through LDS with coalesced row reads, and applies the permutation from LDS.
// Source tiles outside the fermionic box are kernel-filled
// (K1(p) + K2(k;p), constant along K_b); transfers outside the bosonic box
// contribute nothing.
#include "pq_internal.h"

namespace pq {

namespace {

constexpr int kThreads = 256;
constexpr int kRemapThreads = 512;

// ------------------------------------------------------- kernel functions
template <typename C>
struct KxArgs {
  Dims d;
  int level, edge_rule;
  const C* phi;
  double2* k1;
  double2* k2;
};

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename C>
__global__ __launch_bounds__(kThreads) void kernel_extract_kernel(KxArgs<C> a) {
  extern __shared__ double2 srow[];   // [2][n]
  const Dims& d = a.d;
  const int r = blockIdx.x / d.Nq, qi = blockIdx.x - (blockIdx.x / d.Nq) * d.Nq;
  const int m = qi / d.Nk - (d.Nv / 2 - 1);
  const size_t n = d.n;
  const size_t ko = (size_t)r * d.Nq + qi;
  if (a.level == 0) {
    for (int k = threadIdx.x; k < d.n; k += blockDim.x) a.k2[ko * n + k] = mk(0, 0);
    if (threadIdx.x == 0) a.k1[ko] = mk(0, 0);
    return;
  }
  const int top = d.Nv / 2 - 1, bot = -d.Nv / 2;
  int e0, e1 = 0, ne = 1;
  if (a.edge_rule == 1) {
    e0 = bot;
  } else if (m == 0) {
    e0 = top; e1 = bot; ne = 2;
  } else if (r < 2) {
    e0 = m > 0 ? top : bot;
  } else {
    e0 = m > 0 ? bot : top;
  }
  const C* blk = a.phi + (size_t)r * d.cs + (size_t)qi * n * n;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  for (int ei = 0; ei < ne; ++ei) {
    const int e = ei == 0 ? e0 : e1;
    const size_t col0 = (size_t)(e + d.Nv / 2) * d.Nk;
    for (int k = wave; k < d.n; k += nw) {
      double sr = 0.0, si = 0.0;
      for (int K = lane; K < d.Nk; K += 64) {
        double2 v = to_d(blk[(size_t)k * n + col0 + K]);
        sr += v.x;
        si += v.y;
      }
      sr = wave_sum(sr);
      si = wave_sum(si);
      if (lane == 0) srow[ei * n + k] = mk(sr / d.Nk, si / d.Nk);
    }
  }
  __syncthreads();
  __shared__ double2 k1s;
  if (threadIdx.x == 0) {
    double kr = 0.0, ki = 0.0;
    for (int ei = 0; ei < ne; ++ei) {
      const int e = ei == 0 ? e0 : e1;
      double sr = 0.0, si = 0.0;
      for (int K = 0; K < d.Nk; ++K) {
        double2 v = srow[ei * n + (size_t)(e + d.Nv / 2) * d.Nk + K];
        sr += v.x;
        si += v.y;
      }
      kr += sr / d.Nk;
      ki += si / d.Nk;
    }
    k1s = mk(kr / ne, ki / ne);
    a.k1[ko] = k1s;
  }
  __syncthreads();
  const double2 K1v = k1s;
  for (int k = threadIdx.x; k < d.n; k += blockDim.x) {
    double2 v = mk(0, 0);
    if (a.level >= 2) {
      double2 s = srow[k];
      if (ne == 2) s = cadd(s, srow[n + k]);
      v = csub(cscale(s, 1.0 / ne), K1v);
    }
    a.k2[ko * n + k] = v;
  }
}

// ------------------------------------------------------------------ remap
template <typename C>
struct RemapArgs {
  Dims d;
  double lam[4];
  const double2* lam_box;   // nullable: local Lambda_r(m; n, n') on the box, [4][NW][Nv][Nv]
  const C* phi;
  const double2* k1;
  const double2* k2;
  C* gamma;
  int xcd_spread;
};

template <typename C> __device__ inline C czero();
template <> __device__ inline float2 czero<float2>() { return make_float2(0.f, 0.f); }
template <> __device__ inline double2 czero<double2>() { return make_double2(0.0, 0.0); }

// non-temporal store of one complex value (Gamma is not read again here)
__device__ inline void st_stream(float2* p, float2 v) {
  typedef float v2 __attribute__((ext_vector_type(2)));
  const v2 w = {v.x, v.y};
  __builtin_nontemporal_store(w, (v2*)p);
}
__device__ inline void st_stream(double2* p, double2 v) {
  typedef double v2 __attribute__((ext_vector_type(2)));
  const v2 w = {v.x, v.y};
  __builtin_nontemporal_store(w, (v2*)p);
}

template <typename C, typename R>
__device__ inline C axpy(C acc, R c, C v) {
  acc.x += c * v.x;
  acc.y += c * v.y;
  return acc;
}

// Coefficients of the eight terms into the two output channels of a pass
// (pass 0 -> d, m; pass 1 -> s, t), Eqs. PA_Gamma_dm and PA_Gamma_st. Term
// order within a pass: pass 0: d ph-bar, m ph-bar, s pp, t pp; pass 1:
// d st-1, m st-1, d st-2, m st-2.
__constant__ float kCoef[2][4][2] = {
    {{-0.5f, -0.5f}, {-1.5f, 0.5f}, {0.5f, -0.5f}, {1.5f, 0.5f}},
    {{0.5f, -0.5f}, {-1.5f, -0.5f}, {0.5f, 0.5f}, {-1.5f, 0.5f}}};

// One workgroup per (k, m) output plane walks the Nv x 2 x 4 (n', pass, term)
// source tiles in a fixed order. The permutation of each geometry depends only
// on (K, Q, K'), so its LDS offsets are tabulated once per workgroup; a
// kernel-filled tile is written into LDS across all its columns so that the
// same offsets apply. The next tile's global loads are issued before the
// current tile is consumed from LDS, so one tile per workgroup is always in
// flight.
template <typename C, int EPT>
__global__ __launch_bounds__(kRemapThreads) void remap_kernel(RemapArgs<C> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  using R = decltype(C().x);
  const Dims& d = a.d;
  const int Nk = d.Nk, Nk2 = Nk * Nk, ld = Nk + 1;
  C* tile = (C*)smem;                                              // Nk rows, padded stride ld
  unsigned short* offs = (unsigned short*)(smem + sizeof(C) * Nk * ld);   // [4][Nk2]

  // block -> (k, m); consecutive logical blocks (same k) stay on one XCD
  const int total = gridDim.x;
  int lin = blockIdx.x;
  if (a.xcd_spread) lin = (blockIdx.x & 7) * (total >> 3) + (blockIdx.x >> 3);
  const int kbi = lin / d.NW, jm = lin - (lin / d.NW) * d.NW;
  const int nk = kbi / Nk - d.Nv / 2, K = kbi - (kbi / Nk) * Nk;
  const int m = jm - (d.Nv / 2 - 1);
  const size_t n = d.n, nn = (size_t)d.n * d.n, chan = (size_t)d.cs;
  const int t = threadIdx.x;

  // output element e = Q Nk + K' reads source (Qp, Kb):
  //   g0 ph-bar: (K'-K, K+Q)  g1 pp: (K+K'+Q, K')  g2 st-1: (K'-K, Q-K')  g3 st-2: (Q-K-K', K')
  for (int e = t; e < Nk2; e += kRemapThreads) {
    const int Q = e / Nk, Kp = e - (e / Nk) * Nk;
    const int Lx = d.Lx, Ly = d.Ly;
    const int kpk = ksub(Kp, K, Lx, Ly);
    offs[0 * Nk2 + e] = (unsigned short)(kpk * ld + kadd(K, Q, Lx, Ly));
    offs[1 * Nk2 + e] = (unsigned short)(kadd(kadd(K, Kp, Lx, Ly), Q, Lx, Ly) * ld + Kp);
    offs[2 * Nk2 + e] = (unsigned short)(kpk * ld + ksub(Q, Kp, Lx, Ly));
    offs[3 * Nk2 + e] = (unsigned short)(ksub(ksub(Q, K, Lx, Ly), Kp, Lx, Ly) * ld + Kp);
  }

  // step s = (n' index, pass, term) -> source tile
  auto info = [&](int s, int& geo, int& src, int& jmp, int& nb, bool& valid) {
    const int in2 = s >> 3, pass = (s >> 2) & 1, term = s & 3;
    const int n2 = in2 - d.Nv / 2;
    geo = pass * 2 + (term >> 1);                    // 0 ph-bar, 1 pp, 2 st-1, 3 st-2
    src = pass == 0 ? term : (term & 1);
    int mp;
    if (geo == 0) { mp = n2 - nk; nb = nk + m; }
    else if (geo == 1) { mp = nk + n2 + m + 1; nb = n2; }
    else if (geo == 2) { mp = n2 - nk; nb = m - n2 - 1; }
    else { mp = m - nk - n2 - 1; nb = n2; }
    valid = in_bbox(mp, d.Nv);
    jmp = mp + d.Nv / 2 - 1;
  };
  C buf[EPT];
  auto fetch = [&](int s) {
    int geo, src, jmp, nb;
    bool valid;
    info(s, geo, src, jmp, nb, valid);
    if (!valid) return;
    if (in_fbox(nb, d.Nv)) {
      const C* base = a.phi + src * chan + (size_t)kbi * n + (size_t)(nb + d.Nv / 2) * Nk;
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const int idx = min(t + i * kRemapThreads, Nk2 - 1);
        const int Qp = idx / Nk, Kb = idx - (idx / Nk) * Nk;
        buf[i] = base[(size_t)(jmp * Nk + Qp) * nn + Kb];
      }
    } else {
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const int idx = min(t + i * kRemapThreads, Nk2 - 1);
        const size_t qo = (size_t)src * d.Nq + jmp * Nk + idx / Nk;
        buf[i] = from_d<C>(cadd(a.k1[qo], a.k2[qo * n + kbi]));
      }
    }
  };
  const int nsteps = d.Nv * 8;
  fetch(0);
  C acc0[EPT], acc1[EPT];
  for (int s = 0; s < nsteps; ++s) {
    int geo, src, jmp, nb;
    bool valid;
    info(s, geo, src, jmp, nb, valid);
    const int pass = (s >> 2) & 1, term = s & 3;
    if (term == 0) {
      // Lambda of the two output channels at (m; n, n'): constant over the
      // momentum plane, since the fully irreducible vertex is local
      C l0 = czero<C>(), l1 = czero<C>();
      if (a.lam_box) {
        const size_t cs = (size_t)d.NW * d.Nv * d.Nv;
        const size_t li = ((size_t)jm * d.Nv + kbi / Nk) * d.Nv + (s >> 3);
        const double2 v0 = a.lam_box[(size_t)(2 * pass) * cs + li];
        const double2 v1 = a.lam_box[(size_t)(2 * pass + 1) * cs + li];
        l0.x = (R)v0.x;
        l0.y = (R)v0.y;
        l1.x = (R)v1.x;
        l1.y = (R)v1.y;
      } else {
        l0.x = (R)a.lam[2 * pass];
        l1.x = (R)a.lam[2 * pass + 1];
      }
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        acc0[i] = l0;
        acc1[i] = l1;
      }
    }
    if (valid) {                                   // uniform across the block
      __syncthreads();
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const int idx = t + i * kRemapThreads;
        if (idx < Nk2) tile[(idx / Nk) * ld + idx % Nk] = buf[i];
      }
      __syncthreads();
    }
    if (s + 1 < nsteps) fetch(s + 1);              // in flight while this tile is consumed
    if (valid) {
      const R c0 = (R)kCoef[pass][term][0], c1 = (R)kCoef[pass][term][1];
      const unsigned short* og = offs + geo * Nk2;
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const int e = min(t + i * kRemapThreads, Nk2 - 1);
        const C v = tile[og[e]];
        acc0[i] = axpy(acc0[i], c0, v);
        acc1[i] = axpy(acc1[i], c1, v);
      }
    }
    if (term == 3) {
      const int in2 = s >> 3;
      C* o0 = a.gamma + (size_t)(2 * pass) * chan;
      C* o1 = a.gamma + (size_t)(2 * pass + 1) * chan;
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const int e = t + i * kRemapThreads;
        if (e < Nk2) {
          const int Q = e / Nk, Kp = e - (e / Nk) * Nk;
          const size_t off = (size_t)(jm * Nk + Q) * nn + (size_t)kbi * n + (size_t)in2 * Nk + Kp;
          st_stream(o0 + off, acc0[i]);                // written once, read by a later stage
          st_stream(o1 + off, acc1[i]);
        }
      }
    }
  }
}

template <typename C, int EPT>
hipError_t run_remap(const Dims& d, const double lam[4], const double2* lam_box, const void* phi,
                     const double2* k1, const double2* k2, void* gamma, hipStream_t s) {
  RemapArgs<C> a;
  a.d = d;
  for (int i = 0; i < 4; ++i) a.lam[i] = lam[i];
  a.lam_box = lam_box;
  a.phi = (const C*)phi;
  a.k1 = k1;
  a.k2 = k2;
  a.gamma = (C*)gamma;
  const int blocks = d.n * d.NW;
  a.xcd_spread = (blocks % 8 == 0) ? 1 : 0;
  size_t lds = sizeof(C) * d.Nk * (d.Nk + 1) + 4 * sizeof(unsigned short) * d.Nk * d.Nk;
  lds = align256(lds);
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)remap_kernel<C, EPT>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((remap_kernel<C, EPT>), dim3(blocks), dim3(kRemapThreads), lds, s, a);
  return hipGetLastError();
}

template <typename C>
hipError_t dispatch_remap(const Dims& d, const double lam[4], const double2* lam_box, const void* phi,
                          const double2* k1, const double2* k2, void* gamma, hipStream_t s) {
  const int need = (d.Nk * d.Nk + kRemapThreads - 1) / kRemapThreads;
  if (need <= 1) return run_remap<C, 1>(d, lam, lam_box, phi, k1, k2, gamma, s);
  if (need <= 2) return run_remap<C, 2>(d, lam, lam_box, phi, k1, k2, gamma, s);
  if (need <= 8) return run_remap<C, 8>(d, lam, lam_box, phi, k1, k2, gamma, s);
  return hipErrorInvalidValue;
}

// Lambda_r = (U, -U, 2U, 0) at every point of a [4][NW][Nv][Nv] box array
__global__ __launch_bounds__(kThreads) void lambda_fill_kernel(double2* lam, size_t per_channel, double U) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 4 * per_channel) return;
  const int r = (int)(i / per_channel);
  const double v = r == 0 ? U : r == 1 ? -U : r == 2 ? 2.0 * U : 0.0;
  lam[i] = mk(v, 0.0);
}

}  // namespace

hipError_t launch_kernel_extract(const pq_params& p, const Dims& d, const void* phi, double2* k1,
                                 double2* k2, hipStream_t s) {
  size_t lds = 2 * sizeof(double2) * (size_t)d.n;
  if (lds > 64 * 1024) return hipErrorInvalidValue;
  if (p.storage == PQ_STORE_C64) {
    KxArgs<float2> a{d, p.kernel_level, p.edge_rule, (const float2*)phi, k1, k2};
    hipLaunchKernelGGL(kernel_extract_kernel<float2>, dim3(4 * d.Nq), dim3(kThreads), lds, s, a);
  } else {
    KxArgs<double2> a{d, p.kernel_level, p.edge_rule, (const double2*)phi, k1, k2};
    hipLaunchKernelGGL(kernel_extract_kernel<double2>, dim3(4 * d.Nq), dim3(kThreads), lds, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_remap(const pq_params& p, const Dims& d, const double lam[4], const double2* lam_box,
                        const void* phi, const double2* k1, const double2* k2, void* gamma, hipStream_t s) {
  if (d.Nk > 64) return hipErrorInvalidValue;
  if (p.storage == PQ_STORE_C64) return dispatch_remap<float2>(d, lam, lam_box, phi, k1, k2, gamma, s);
  return dispatch_remap<double2>(d, lam, lam_box, phi, k1, k2, gamma, s);
}

hipError_t launch_lambda_fill(const Dims& d, double U, double2* lam_box, hipStream_t s) {
  const size_t per = (size_t)d.NW * d.Nv * d.Nv;
  hipLaunchKernelGGL(lambda_fill_kernel, dim3((unsigned)((4 * per + kThreads - 1) / kThreads)), dim3(kThreads), 0, s,
                     lam_box, per, U);
  return hipGetLastError();
}

}  // namespace pq
