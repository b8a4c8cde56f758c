// Host-side declarations shared by the translation units of libparquet.
#pragma once
#include <hip/hip_runtime.h>

#include "parquet.h"
#include "pq_device.h"

namespace pq {

// thread-local error message
void set_error(const char* fmt, ...);
pq_status hip_fail(hipError_t e, const char* what);

// Validates params and fills the device size struct (sets the error on failure).
bool make_dims(const pq_params* p, Dims* d);
pq_dims to_public(const Dims& d);

// Convergence test of one iteration with change dn (max |dSigma|) and max |Sigma|
// smax, on the history dhist[7] / *nhist of the earlier changes (newest first,
// updated here). tol > 0: dn < tol. tol < 0: the estimated distance to the
// fixed point, alpha max(last six changes) / (1 - rho) with rho the geometric
// mean of the last six ratios (< 0.98), below |tol| smax. tol = 0: never.
bool convergence_test(double* dhist, int* nhist, double alpha, double dn, double smax, double tol);

// largest |eps_K| of the lattice (0 in the local mode)
double max_abs_eps(const pq_params& p, const Dims& d);

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

inline size_t elem_bytes(const pq_params& p) {
  return p.storage == PQ_STORE_C64 ? sizeof(float2) : sizeof(double2);
}

// ---- launchers (enqueue only) ----
hipError_t launch_dyson(const pq_params& p, const Dims& d, const double2* sigma, double2* g,
                        double* mu_out, hipStream_t s);
hipError_t launch_bubbles(const pq_params& p, const Dims& d, const double2* g, double2* xph,
                          double2* xpp, hipStream_t s);
// smax (nullable): max |sigma_io| after the mixing
hipError_t launch_mix(const Dims& d, const double2* snew, double2* sio, double alpha,
                      double* dnorm, hipStream_t s, double* smax = nullptr);
// dst[i] = src[i] between complex64 / complex128 storages (count complex elements)
hipError_t launch_convert(const void* src, int src_storage, void* dst, int dst_storage, size_t count,
                          hipStream_t s);
hipError_t launch_kernel_extract(const pq_params& p, const Dims& d, const void* phi, double2* k1,
                                 double2* k2, hipStream_t s);
// lam_box (nullable): local Lambda_r(m; n, n') on the box, [4][NW][Nv][Nv] c128, in place of lam
hipError_t launch_remap(const pq_params& p, const Dims& d, const double lam[4], const double2* lam_box,
                        const void* phi, const double2* k1, const double2* k2, void* gamma, hipStream_t s);
hipError_t launch_lambda_fill(const Dims& d, double U, double2* lam_box, hipStream_t s);
// f = a + b elementwise over count complex elements of the given storage
hipError_t launch_vertex_sum(const void* a, const void* b, void* f, int storage, size_t count, hipStream_t s);
// HBM streaming probes: mode 0 copy src -> dst, 1 read src (dst receives one
// float per workgroup, at most kHbmStreamBlocks), 2 write dst; bytes a multiple of 16
constexpr unsigned kHbmStreamBlocks = 16384;
hipError_t launch_hbm_stream(int mode, const void* src, void* dst, size_t bytes, hipStream_t s);
// learned warm start (pq_mlp.hip)
size_t mlp_count(const int32_t* widths, int n_layers);
hipError_t launch_mlp_forward(const int32_t* widths, int n_layers, const void* params_bf16, const float* params,
                              const float* x, float* acts, int batch, hipStream_t s);
hipError_t launch_mlp_backward(const int32_t* widths, int n_layers, const void* params_bf16, const float* x,
                               const float* acts, const float* target, float* grad, float* loss, float* scratch,
                               int batch, hipStream_t s);
hipError_t launch_mlp_adam(float* params, void* params_bf16, float* m, float* v, const float* grad, size_t count,
                           float lr, float beta1, float beta2, float eps, int step, hipStream_t s);
hipError_t launch_mlp_to_bf16(const float* params, void* params_bf16, size_t count, hipStream_t s);
size_t mlp_basis_ws_bytes(int rows);
hipError_t launch_mlp_basis(float* y, int rows, size_t len, float* mean, float* coef, int ld, float* scale, void* ws,
                            hipStream_t s);
hipError_t launch_mlp_expand(const float* q, int rows, size_t len, const float* mean, const float* coef,
                             const float* scale, double* out, hipStream_t s);
hipError_t launch_phi_from_kernels(const pq_params& p, const Dims& d, const double2* k1, const double2* k2,
                                   void* phi, hipStream_t s);
size_t sigma_ws_bytes(const Dims& d);
// Device address of the static scratch of sigma_sde_no_alloc on the current
// device (looked up once per device, then cached).
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
hipError_t static_scratch(void** out);
hipError_t launch_sigma(const pq_params& p, const Dims& d, const void* phi, const double2* k1,
                        const double2* k2, const double2* lam_box, const double2* g, const double* mu,
                        double2* sigma_out, void* ws, hipStream_t s);
// Sigma~_1 alone (used for the bare-vertex start)
hipError_t launch_sigma1(const pq_params& p, const Dims& d, const double2* g, const double* mu,
                         double2* sigma_out, void* ws, hipStream_t s);
size_t bse_ws_bytes(const pq_params& p, const Dims& d, int precision);
// Optional device-event timing of the BSE launches, by kernel kind
// (0 init, 1 pivot, 2 panel, 3 update, 4 epilogue, 5 error estimate and FP64 re-solve).
struct BseTiming {
  hipEvent_t* ev;     // 2 * cap events
  int cap, used;
  int kind[256];
  double update_flops;
};
// Look-ahead of the BSE elimination: a second stream and two events (created
// by the caller, timing disabled); the next panel's diagonal-block inversion
// runs on the second stream while the rows below it are updated. Not for work
// captured into a graph.
struct BseAsync {
  hipStream_t side;
  hipEvent_t ready, done;
};
hipError_t launch_bse(const pq_params& p, const Dims& d, int channel, int precision,
                      const void* gamma, const double2* chi0, void* phi_io, double alpha,
                      pq_bse_block_stats* stats, void* ws, hipStream_t s, BseTiming* tm = nullptr,
                      const BseAsync* la = nullptr);
// summary of nb block stats into out[0..3]: flagged, re-solved and unresolved
// block counts, largest error estimate (+inf for a non-finite one); with
// nchunks > 1, over nchunks runs of nb stats, stride apart
hipError_t launch_bse_summary(const pq_bse_block_stats* stats, int nb, double* out, hipStream_t s, int nchunks = 1,
                              size_t stride = 0);
// largest number of blocks one BSE launch sequence takes (the refine list)
constexpr int kBseMaxBlocks = 16384;

}  // namespace pq
