// C ABI of libparquet: argument validation, the stateless stage entry points
// and the context API that runs whole parquet iterations on one stream.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <new>

#include <vector>

#include "pq_internal.h"

namespace pq {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

pq_status hip_fail(hipError_t e, const char* what) {
  set_error("%s: %s", what, hipGetErrorString(e));
  return PQ_ERR_HIP;
}

double max_abs_eps(const pq_params& p, const Dims& d) {
  if (d.Nk == 1) return 0.0;
  double mx = 0.0;
  for (int K = 0; K < d.Nk; ++K) {
    int kx = K / d.Ly, ky = K % d.Ly;
    double cx = cos(2.0 * M_PI * kx / d.Lx), cy = cos(2.0 * M_PI * ky / d.Ly);
    double e = -2.0 * p.t * (cx + cy) - 4.0 * p.tp * cx * cy;
    mx = fmax(mx, fabs(e));
  }
  return mx;
}

bool make_dims(const pq_params* p, Dims* d) {
  if (!p) { set_error("null params"); return false; }
  if (p->Lx < 1 || p->Ly < 1 || p->Lx * p->Ly > 64) { set_error("lattice %dx%d outside 1..64 momenta", p->Lx, p->Ly); return false; }
  if (p->Lx * p->Ly > 1 && (p->Lx > 255 || p->Ly > 255)) { set_error("lattice too large"); return false; }
  if (p->Nv < 2 || (p->Nv & 1)) { set_error("Nv must be even and >= 2 (got %d)", p->Nv); return false; }
  if (p->f_ext < 1 || p->f_ext > 16) { set_error("f_ext must be in 1..16"); return false; }
  if (p->kernel_level < 0 || p->kernel_level > 2) { set_error("kernel_level must be 0, 1 or 2"); return false; }
  if (p->edge_rule < 0 || p->edge_rule > 1) { set_error("edge_rule must be 0 or 1"); return false; }
  if (p->mu_mode < 0 || p->mu_mode > 1) { set_error("mu_mode must be 0 or 1"); return false; }
  if (p->storage != PQ_STORE_C64 && p->storage != PQ_STORE_C128) { set_error("bad storage"); return false; }
  if (p->precision == PQ_PREC_FP64 && p->storage != PQ_STORE_C128) { set_error("FP64 BSE needs complex128 storage"); return false; }
  if (p->precision == PQ_PREC_FP32 && p->storage != PQ_STORE_C64) { set_error("FP32 BSE needs complex64 storage"); return false; }
  if (p->precision == PQ_PREC_BF16X3 && p->storage != PQ_STORE_C64) { set_error("BF16x3 BSE needs complex64 storage"); return false; }
  if (p->precision != PQ_PREC_FP64 && p->precision != PQ_PREC_FP32 && p->precision != PQ_PREC_BF16X3) {
    set_error("precision %d not available", p->precision);
    return false;
  }
  if (!(p->beta > 0.0) || !isfinite(p->U) || !isfinite(p->beta)) { set_error("beta must be > 0 and U finite"); return false; }
  if (!(p->alpha > 0.0 && p->alpha <= 1.0)) { set_error("alpha must be in (0, 1]"); return false; }
  if (p->Lx * p->Ly == 1 && !(p->D > 0.0)) { set_error("local mode needs D > 0"); return false; }
  if (p->resolve_slots < 0) { set_error("resolve_slots must be >= 0"); return false; }
  if (p->regulation != 0 && p->regulation != 1) { set_error("regulation must be 0 or 1"); return false; }
  if (p->regulation == 0 && p->f_ext != 1) {
    set_error("without the regulation Sigma lives on the box: f_ext must be 1");
    return false;
  }
  if (!(p->bse_tol >= 0.0 && p->bse_tol <= 1.0)) { set_error("bse_tol must be in [0, 1]"); return false; }
  if (p->bse_tile != 0 && p->bse_tile != 1) { set_error("bse_tile must be 0 or 1"); return false; }
  Dims x;
  x.Lx = p->Lx; x.Ly = p->Ly; x.Nk = p->Lx * p->Ly; x.Nv = p->Nv; x.NW = p->Nv - 1;
  x.f = p->f_ext; x.Nve = p->f_ext * p->Nv; x.NWe = x.Nve - 1; x.NG = 2 * x.Nve;
  x.n = x.Nk * x.Nv; x.Nq = x.Nk * x.NW;
  x.cs = (long long)x.Nq * x.n * x.n;
  if (x.n > 4096) { set_error("BSE dimension %d above 4096", x.n); return false; }
  const double E = x.Nk == 1 ? p->D : 2.0 * max_abs_eps(*p, x);
  x.ntau = 8 * x.f * x.Nv + 64 + 4 * (int)ceil(p->beta * E);
  *d = x;
  return true;
}

bool convergence_test(double* dhist, int* nhist, double alpha, double dn, double smax, double tol) {
  constexpr int W = 6;
  for (int k = W; k > 0; --k) dhist[k] = dhist[k - 1];
  dhist[0] = dn;
  *nhist = *nhist < W + 1 ? *nhist + 1 : W + 1;
  if (tol > 0.0) return dn < tol;
  if (tol == 0.0 || *nhist < W + 1) return false;
  if (!(dhist[W] > 0.0) || !(dn > 0.0)) return dn == 0.0 && *nhist > W;
  const double rho = pow(dn / dhist[W], 1.0 / W);
  double dmax = 0.0;
  for (int k = 0; k < W; ++k) dmax = fmax(dmax, dhist[k]);
  if (!(rho < 0.98)) return false;
  return alpha * dmax / (1.0 - rho) < -tol * smax;
}

pq_dims to_public(const Dims& d) {
  pq_dims o;
  o.Lx = d.Lx; o.Ly = d.Ly; o.Nk = d.Nk; o.Nv = d.Nv; o.NW = d.NW; o.f_ext = d.f;
  o.Nve = d.Nve; o.NWe = d.NWe; o.NG = d.NG; o.n = d.n; o.Nq = d.Nq; o.ntau = d.ntau;
  o.vertex_elems = (int64_t)d.Nq * d.n * d.n;
  return o;
}

}  // namespace pq

using namespace pq;

#define PQ_CHECK_ARG(cond, ...)      \
  do {                               \
    if (!(cond)) {                   \
      set_error(__VA_ARGS__);        \
      return PQ_ERR_ARG;             \
    }                                \
  } while (0)

static pq_status enq(hipError_t e, const char* what) {
  if (e != hipSuccess) return hip_fail(e, what);
  return PQ_OK;
}

extern "C" {

const char* parquet_last_error(void) { return g_err; }

pq_status pq_dims_from_params(const pq_params* p, pq_dims* out) {
  PQ_CHECK_ARG(out, "null output");
  Dims d;
  if (!make_dims(p, &d)) return PQ_ERR_ARG;
  *out = to_public(d);
  return PQ_OK;
}

pq_status dyson_update(const pq_params* p, const void* sigma, void* g_out, void* mu_out,
                       pq_stream stream) {
  Dims d;
  if (!make_dims(p, &d)) return PQ_ERR_ARG;
  PQ_CHECK_ARG(sigma && g_out && mu_out, "null pointer");
  return enq(launch_dyson(*p, d, (const double2*)sigma, (double2*)g_out, (double*)mu_out,
                          (hipStream_t)stream), "dyson_update");
}

pq_status bubble_build(const pq_params* p, const void* g, void* xph, void* xpp, pq_stream stream) {
  Dims d;
  if (!make_dims(p, &d)) return PQ_ERR_ARG;
  PQ_CHECK_ARG(g && xph && xpp, "null pointer");
  return enq(launch_bubbles(*p, d, (const double2*)g, (double2*)xph, (double2*)xpp,
                            (hipStream_t)stream), "bubble_build");
}

pq_status kernel_extract(const pq_params* p, const void* phi, void* k1, void* k2, pq_stream stream) {
  Dims d;
  if (!make_dims(p, &d)) return PQ_ERR_ARG;
  PQ_CHECK_ARG(phi && k1 && k2, "null pointer");
  return enq(launch_kernel_extract(*p, d, phi, (double2*)k1, (double2*)k2, (hipStream_t)stream),
             "kernel_extract");
}

pq_status channel_remap(const pq_params* p, const double lambda[4], const void* lambda_box, const void* phi,
                        const void* k1, const void* k2, void* gamma_out, void* f_out, pq_stream stream) {
  Dims d;
  if (!make_dims(p, &d)) return PQ_ERR_ARG;
  PQ_CHECK_ARG(lambda && phi && k1 && k2 && gamma_out, "null pointer");
  PQ_CHECK_ARG(phi != gamma_out, "phi and gamma_out must not alias");
  PQ_CHECK_ARG(f_out != phi && f_out != gamma_out, "f_out must alias neither phi nor gamma_out");
  hipError_t e = launch_remap(*p, d, lambda, (const double2*)lambda_box, phi, (const double2*)k1,
                              (const double2*)k2, gamma_out, (hipStream_t)stream);
  if (e == hipSuccess && f_out)
    e = launch_vertex_sum(gamma_out, phi, f_out, p->storage, 4 * (size_t)d.Nq * d.n * d.n, (hipStream_t)stream);
  return enq(e, "channel_remap");
}

pq_status sigma_sde_workspace(const pq_params* p, size_t* bytes) {
  Dims d;
  if (!make_dims(p, &d)) return PQ_ERR_ARG;
  PQ_CHECK_ARG(bytes, "null output");
  *bytes = sigma_ws_bytes(d);
  return PQ_OK;
}

pq_status sigma_sde(const pq_params* p, const void* phi, const void* k1, const void* k2,
                    const void* lambda_box, const void* g, const void* mu, void* sigma_out, void* ws,
                    size_t ws_bytes, pq_stream stream) {
  Dims d;
  if (!make_dims(p, &d)) return PQ_ERR_ARG;
  PQ_CHECK_ARG(phi && k1 && k2 && g && mu && sigma_out && ws, "null pointer");
  if (ws_bytes < sigma_ws_bytes(d)) {
    set_error("sigma_sde workspace %zu < %zu bytes", ws_bytes, sigma_ws_bytes(d));
    return PQ_ERR_NOMEM;
  }
  return enq(launch_sigma(*p, d, phi, (const double2*)k1, (const double2*)k2, (const double2*)lambda_box,
                          (const double2*)g, (const double*)mu, (double2*)sigma_out, ws, (hipStream_t)stream),
             "sigma_sde");
}

pq_status sigma_sde_no_alloc(const pq_params* p, const void* phi, const void* k1, const void* k2,
                             const void* lambda_box, const void* g, const void* mu, void* sigma_out,
                             pq_stream stream) {
  Dims d;
  if (!make_dims(p, &d)) return PQ_ERR_ARG;
  PQ_CHECK_ARG(phi && k1 && k2 && g && mu && sigma_out, "null pointer");
  const size_t need = sigma_ws_bytes(d);
  if (need > kStaticScratchBytes) {
    set_error("sigma_sde_no_alloc needs %zu bytes of scratch; the static scratch holds %zu", need,
              kStaticScratchBytes);
    return PQ_ERR_NOMEM;
  }
  void* ws = nullptr;
  hipError_t e = static_scratch(&ws);
  if (e != hipSuccess) return hip_fail(e, "sigma_sde_no_alloc (scratch address)");
  return enq(launch_sigma(*p, d, phi, (const double2*)k1, (const double2*)k2, (const double2*)lambda_box,
                          (const double2*)g, (const double*)mu, (double2*)sigma_out, ws, (hipStream_t)stream),
             "sigma_sde_no_alloc");
}

pq_status bse_workspace(const pq_params* p, size_t* bytes) {
  Dims d;
  if (!make_dims(p, &d)) return PQ_ERR_ARG;
  PQ_CHECK_ARG(bytes, "null output");
  *bytes = bse_ws_bytes(*p, d, p->precision);
  return PQ_OK;
}

pq_status bse_solve(const pq_params* p, int32_t channel, int32_t precision, const void* gamma,
                    const void* chi0, void* phi_io, double alpha, void* stats, void* ws,
                    size_t ws_bytes, pq_stream stream) {
  Dims d;
  if (!make_dims(p, &d)) return PQ_ERR_ARG;
  PQ_CHECK_ARG(channel >= 0 && channel < 4, "channel must be 0..3");
  PQ_CHECK_ARG(precision == p->precision, "precision must match params.precision");
  PQ_CHECK_ARG(gamma && chi0 && phi_io && ws, "null pointer");
  PQ_CHECK_ARG(alpha > 0.0 && alpha <= 1.0, "alpha must be in (0, 1]");
  PQ_CHECK_ARG(gamma != phi_io, "gamma and phi_io must not alias");
  if (ws_bytes < bse_ws_bytes(*p, d, precision)) {
    set_error("bse workspace %zu < %zu bytes", ws_bytes, bse_ws_bytes(*p, d, precision));
    return PQ_ERR_NOMEM;
  }
  return enq(launch_bse(*p, d, channel, precision, gamma, (const double2*)chi0, phi_io, alpha,
                        (pq_bse_block_stats*)stats, ws, (hipStream_t)stream),
             "bse_solve");
}

pq_status sigma_mix(const pq_params* p, const void* sigma_new, void* sigma_io, double alpha,
                    void* dnorm_out, pq_stream stream) {
  Dims d;
  if (!make_dims(p, &d)) return PQ_ERR_ARG;
  PQ_CHECK_ARG(sigma_new && sigma_io && dnorm_out, "null pointer");
  PQ_CHECK_ARG(alpha > 0.0 && alpha <= 1.0, "alpha must be in (0, 1]");
  return enq(launch_mix(d, (const double2*)sigma_new, (double2*)sigma_io, alpha, (double*)dnorm_out,
                        (hipStream_t)stream),
             "sigma_mix");
}

// ------------------------------------------------------ learned warm start
// widths and batch up to 65535 GEMM tiles of 64 (the products put the output
// width and the batch on the grid's second dimension)
constexpr int32_t kMlpMaxWidth = 65535 * 64;
constexpr int32_t kMlpMaxBasisRows = 4096;

static bool mlp_widths_ok(const int32_t* w, int32_t nl) {
  if (!w || nl < 1 || nl > 16) return false;
  for (int l = 0; l <= nl; ++l)
    if (w[l] < 1 || w[l] > kMlpMaxWidth) return false;
  return true;
}

pq_status mlp_param_count(const int32_t* widths, int32_t n_layers, size_t* count) {
  PQ_CHECK_ARG(mlp_widths_ok(widths, n_layers) && count, "bad widths or null output");
  *count = mlp_count(widths, n_layers);
  return PQ_OK;
}

pq_status mlp_forward(const int32_t* widths, int32_t n_layers, const void* params_bf16, const float* params,
                      const float* x, float* acts, int32_t batch, pq_stream stream) {
  PQ_CHECK_ARG(mlp_widths_ok(widths, n_layers) && batch >= 1 && batch <= kMlpMaxWidth, "bad widths or batch");
  PQ_CHECK_ARG(params_bf16 && params && x && acts, "null pointer");
  return enq(launch_mlp_forward(widths, n_layers, params_bf16, params, x, acts, batch, (hipStream_t)stream),
             "mlp_forward");
}

pq_status mlp_backward(const int32_t* widths, int32_t n_layers, const void* params_bf16, const float* x,
                       const float* acts, const float* target, float* grad, float* loss, float* scratch,
                       int32_t batch, pq_stream stream) {
  PQ_CHECK_ARG(mlp_widths_ok(widths, n_layers) && batch >= 1 && batch <= kMlpMaxWidth, "bad widths or batch");
  PQ_CHECK_ARG(params_bf16 && x && acts && target && grad && loss && scratch, "null pointer");
  return enq(launch_mlp_backward(widths, n_layers, params_bf16, x, acts, target, grad, loss, scratch, batch,
                                 (hipStream_t)stream),
             "mlp_backward");
}

pq_status mlp_adam(float* params, void* params_bf16, float* m, float* v, const float* grad, size_t count, float lr,
                   float beta1, float beta2, float eps, int32_t step, pq_stream stream) {
  PQ_CHECK_ARG(params && params_bf16 && m && v && grad && count > 0, "null pointer or empty");
  PQ_CHECK_ARG(step >= 1 && lr > 0.f && beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f, "bad Adam settings");
  return enq(launch_mlp_adam(params, params_bf16, m, v, grad, count, lr, beta1, beta2, eps, step, (hipStream_t)stream),
             "mlp_adam");
}

pq_status mlp_to_bf16(const float* params, void* params_bf16, size_t count, pq_stream stream) {
  PQ_CHECK_ARG(params && params_bf16 && count > 0, "null pointer or empty");
  return enq(launch_mlp_to_bf16(params, params_bf16, count, (hipStream_t)stream), "mlp_to_bf16");
}

pq_status hbm_stream(int32_t mode, const void* src, void* dst, size_t bytes, pq_stream stream) {
  PQ_CHECK_ARG(mode >= 0 && mode <= 2, "mode must be 0 (copy), 1 (read) or 2 (write)");
  PQ_CHECK_ARG(bytes > 0 && bytes % 16 == 0, "bytes must be a positive multiple of 16");
  PQ_CHECK_ARG(mode == 2 || src, "null source");
  PQ_CHECK_ARG(dst, "null destination");
  return enq(launch_hbm_stream(mode, src, dst, bytes, (hipStream_t)stream), "hbm_stream");
}

pq_status mlp_basis_workspace(int32_t rows, size_t* bytes) {
  PQ_CHECK_ARG(rows >= 1 && rows <= kMlpMaxBasisRows && bytes, "bad row count or null output");
  *bytes = mlp_basis_ws_bytes(rows);
  return PQ_OK;
}

pq_status mlp_basis(float* y, int32_t rows, size_t len, float* mean, float* coef, int32_t ld_coef, float* scale,
                    void* ws, pq_stream stream) {
  PQ_CHECK_ARG(rows >= 1 && rows <= kMlpMaxBasisRows && len >= 1 && ld_coef >= rows, "bad sizes");
  PQ_CHECK_ARG(y && mean && coef && scale && ws, "null pointer");
  return enq(launch_mlp_basis(y, rows, len, mean, coef, ld_coef, scale, ws, (hipStream_t)stream), "mlp_basis");
}

pq_status mlp_expand(const float* q, int32_t rows, size_t len, const float* mean, const float* coef,
                     const float* scale, double* out, pq_stream stream) {
  PQ_CHECK_ARG(rows >= 1 && rows <= kMlpMaxBasisRows && len >= 1, "bad sizes");
  PQ_CHECK_ARG(q && mean && coef && scale && out, "null pointer");
  return enq(launch_mlp_expand(q, rows, len, mean, coef, scale, out, (hipStream_t)stream), "mlp_expand");
}

pq_status phi_from_kernels(const pq_params* p, const void* k1, const void* k2, void* phi_out, pq_stream stream) {
  Dims d;
  if (!make_dims(p, &d)) return PQ_ERR_ARG;
  PQ_CHECK_ARG(k1 && k2 && phi_out, "null pointer");
  return enq(launch_phi_from_kernels(*p, d, (const double2*)k1, (const double2*)k2, phi_out, (hipStream_t)stream),
             "phi_from_kernels");
}

}  // extern "C"

// ------------------------------------------------------------- context API
struct pq_ctx {
  pq_params p;
  Dims d;
  hipStream_t s;
  char* ws;
  size_t ws_bytes;
  double2 *sigma, *sigma_new, *g, *xph, *xpp, *k1, *k2, *lam;
  bool has_lam;            // a box Lambda was set (else the scalars (U, -U, 2U, 0))
  double *mu, *dnorm;
  void *phi, *gamma, *bse_ws, *sig_ws;
  size_t bse_bytes, sig_bytes;
  pq_bse_block_stats* bstats;
  int iteration;
  double dhist[7];         // the last changes of Sigma (newest first), for the contraction estimate
  int nhist;
  hipEvent_t ev[8];
  bool have_events;
  hipEvent_t bev[512];   // BSE launch timing of one channel
  bool have_bev;
  BseAsync la;           // BSE look-ahead stream and events (uncaptured iterations only)
  bool have_la;
  hipGraphExec_t graph;  // one whole iteration captured on s (parquet_iterate_batch)
  bool have_graph;
  bool graph_has_lam;    // the box Lambda setting the graph was captured with
};

namespace {

struct CtxLayout {
  size_t sigma, sigma_new, g, mu, dnorm, xph, xpp, k1, k2, lam, phi, gamma, bse, sig, bstats, total;
  size_t bse_bytes, sig_bytes;
};

CtxLayout ctx_layout(const pq_params& p, const Dims& d) {
  CtxLayout L{};
  size_t off = 0;
  auto take = [&](size_t b) { size_t o = off; off += align256(b); return o; };
  const size_t nk = (size_t)d.Nk;
  L.sigma = take(sizeof(double2) * d.Nve * nk);
  L.sigma_new = take(sizeof(double2) * d.Nve * nk);
  L.g = take(sizeof(double2) * d.NG * nk);
  L.mu = take(sizeof(double));
  L.dnorm = take(6 * sizeof(double));      // the norm, the BSE summary (bse_summary), max |Sigma|
  L.xph = take(sizeof(double2) * (size_t)d.Nq * d.n);
  L.xpp = take(sizeof(double2) * (size_t)d.Nq * d.n);
  L.k1 = take(sizeof(double2) * 4 * (size_t)d.Nq);
  L.k2 = take(sizeof(double2) * 4 * (size_t)d.Nq * d.n);
  L.lam = take(sizeof(double2) * 4 * (size_t)d.NW * d.Nv * d.Nv);
  const size_t vb = elem_bytes(p) * (size_t)d.Nq * d.n * d.n * 4;
  L.phi = take(vb);
  L.gamma = take(vb);
  L.bse_bytes = bse_ws_bytes(p, d, p.precision);
  L.bse = take(L.bse_bytes);
  L.sig_bytes = sigma_ws_bytes(d);
  L.sig = take(L.sig_bytes);
  L.bstats = take(sizeof(pq_bse_block_stats) * 4 * (size_t)d.Nq);
  L.total = off;
  return L;
}

size_t field_bytes(const pq_ctx* c, int f) {
  const Dims& d = c->d;
  switch (f) {
    case PQ_FIELD_SIGMA: return sizeof(double2) * d.Nve * (size_t)d.Nk;
    case PQ_FIELD_G: return sizeof(double2) * d.NG * (size_t)d.Nk;
    case PQ_FIELD_PHI:
    case PQ_FIELD_GAMMA:
    case PQ_FIELD_F: return elem_bytes(c->p) * (size_t)d.Nq * d.n * d.n * 4;
    case PQ_FIELD_K1: return sizeof(double2) * 4 * (size_t)d.Nq;
    case PQ_FIELD_K2: return sizeof(double2) * 4 * (size_t)d.Nq * d.n;
    case PQ_FIELD_MU: return sizeof(double);
    case PQ_FIELD_XPH:
    case PQ_FIELD_XPP: return sizeof(double2) * (size_t)d.Nq * d.n;
    case PQ_FIELD_LAMBDA: return sizeof(double2) * 4 * (size_t)d.NW * d.Nv * d.Nv;
    default: return 0;
  }
}

void* field_ptr(pq_ctx* c, int f) {
  switch (f) {
    case PQ_FIELD_SIGMA: return c->sigma;
    case PQ_FIELD_G: return c->g;
    case PQ_FIELD_PHI: return c->phi;
    case PQ_FIELD_GAMMA: return c->gamma;
    case PQ_FIELD_K1: return c->k1;
    case PQ_FIELD_K2: return c->k2;
    case PQ_FIELD_MU: return c->mu;
    case PQ_FIELD_XPH: return c->xph;
    case PQ_FIELD_XPP: return c->xpp;
    case PQ_FIELD_LAMBDA: return c->lam;
    default: return nullptr;
  }
}

// Milliseconds between two recorded events; NaN where they cannot be read.
float elapsed_ms(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  return hipEventElapsedTime(&ms, a, b) == hipSuccess ? ms : __builtin_nanf("");
}

// The launches of one iteration on the context stream: Dyson -> bubbles ->
// kernels -> remap -> Schwinger-Dyson -> BSE (4 channels) -> mixing (writes
// dnorm). Nothing here waits on the host, allocates or clears memory, so the
// sequence can be captured into a graph (record = false, tm = nullptr).
hipError_t enqueue_iteration(pq_ctx* c, bool record, BseTiming* tm, const char** where, bool lookahead = false) {
  const Dims& d = c->d;
  const pq_params& p = c->p;
  const double lam[4] = {p.U, -p.U, 2.0 * p.U, 0.0};
  const size_t vstride = elem_bytes(p) * (size_t)d.Nq * d.n * d.n;
  const double2* lam_box = c->has_lam ? c->lam : nullptr;
  hipError_t e, er = hipSuccess;  // er: the first failed stage-event record
  auto rec = [&](int i) {
    if (record && er == hipSuccess) er = hipEventRecord(c->ev[i], c->s);
  };
  rec(0);
  if ((e = launch_dyson(p, d, c->sigma, c->g, c->mu, c->s)) != hipSuccess) { *where = "dyson"; return e; }
  rec(1);
  if ((e = launch_bubbles(p, d, c->g, c->xph, c->xpp, c->s)) != hipSuccess) { *where = "bubbles"; return e; }
  if ((e = launch_kernel_extract(p, d, c->phi, c->k1, c->k2, c->s)) != hipSuccess) { *where = "kernels"; return e; }
  rec(2);
  if ((e = launch_remap(p, d, lam, lam_box, c->phi, c->k1, c->k2, c->gamma, c->s)) != hipSuccess) {
    *where = "remap";
    return e;
  }
  rec(3);
  if ((e = launch_sigma(p, d, c->phi, c->k1, c->k2, lam_box, c->g, c->mu, c->sigma_new, c->sig_ws, c->s)) !=
      hipSuccess) {
    *where = "sigma";
    return e;
  }
  rec(4);
  for (int r = 0; r < 4; ++r) {
    const double2* x = r < 2 ? c->xph : c->xpp;
    e = launch_bse(p, d, r, p.precision, (char*)c->gamma + r * vstride, x, (char*)c->phi + r * vstride, p.alpha,
                   c->bstats + (size_t)r * d.Nq, c->bse_ws, c->s, r == 0 ? tm : nullptr,
                   lookahead && c->have_la ? &c->la : nullptr);
    if (e != hipSuccess) { *where = "bse"; return e; }
  }
  if ((e = launch_bse_summary(c->bstats, 4 * d.Nq, c->dnorm + 1, c->s)) != hipSuccess) { *where = "bse summary"; return e; }
  rec(5);
  if ((e = launch_mix(d, c->sigma_new, c->sigma, p.alpha, c->dnorm, c->s, c->dnorm + 5)) != hipSuccess) {
    *where = "mix";
    return e;
  }
  rec(6);
  if (er != hipSuccess) *where = "stage events";
  return er;
}

// Convergence test of one iteration. tol > 0: the change of Sigma below tol.
// tol < 0: the estimated distance of the mixed Sigma to the fixed point below
// |tol| max|Sigma|. For a linear iteration with contraction rho the distance
// after a step of size alpha dsigma is at most alpha dsigma / (1 - rho); the
// changes of the parquet iteration oscillate (beating modes), so rho is the
// geometric mean of the last six ratios, (d_k / d_{k-6})^(1/6), and dsigma the
// largest of the last six changes (seven iterations of this state needed, rho
// < 0.98). On the oracle's convergence histories of five small problems this
// stops within 0.42 of the target distance at targets 1e-4 .. 1e-9.
// tol = 0: never.
bool converged_now(pq_ctx* c, double dn, double smax, double tol) {
  return convergence_test(c->dhist, &c->nhist, c->p.alpha, dn, smax, tol);
}

}  // namespace

extern "C" {

pq_status parquet_query_workspace(const pq_params* p, size_t* bytes) {
  Dims d;
  if (!make_dims(p, &d)) return PQ_ERR_ARG;
  PQ_CHECK_ARG(bytes, "null output");
  *bytes = ctx_layout(*p, d).total;
  return PQ_OK;
}

pq_status parquet_init(const pq_params* p, void* ws, size_t ws_bytes, pq_stream stream, pq_ctx** out) {
  Dims d;
  if (!make_dims(p, &d)) return PQ_ERR_ARG;
  PQ_CHECK_ARG(ws && out, "null pointer");
  CtxLayout L = ctx_layout(*p, d);
  if (ws_bytes < L.total) {
    set_error("parquet workspace %zu < %zu bytes", ws_bytes, L.total);
    return PQ_ERR_NOMEM;
  }
  pq_ctx* c = new (std::nothrow) pq_ctx();
  if (!c) { set_error("host allocation failed"); return PQ_ERR_NOMEM; }
  c->p = *p;
  c->d = d;
  c->s = (hipStream_t)stream;
  c->ws = (char*)ws;
  c->ws_bytes = ws_bytes;
  char* w = c->ws;
  c->sigma = (double2*)(w + L.sigma);
  c->sigma_new = (double2*)(w + L.sigma_new);
  c->g = (double2*)(w + L.g);
  c->mu = (double*)(w + L.mu);
  c->dnorm = (double*)(w + L.dnorm);
  c->xph = (double2*)(w + L.xph);
  c->xpp = (double2*)(w + L.xpp);
  c->k1 = (double2*)(w + L.k1);
  c->k2 = (double2*)(w + L.k2);
  c->lam = (double2*)(w + L.lam);
  c->has_lam = false;
  c->phi = w + L.phi;
  c->gamma = w + L.gamma;
  c->bse_ws = w + L.bse;
  c->sig_ws = w + L.sig;
  c->bse_bytes = L.bse_bytes;
  c->sig_bytes = L.sig_bytes;
  c->bstats = (pq_bse_block_stats*)(w + L.bstats);
  c->iteration = 0;
  c->nhist = 0;
  c->have_graph = false;
  c->graph_has_lam = false;
  c->have_events = true;
  for (int i = 0; i < 8; ++i)
    if (hipEventCreate(&c->ev[i]) != hipSuccess) c->have_events = false;
  c->have_bev = true;
  for (int i = 0; i < 512; ++i)
    if (hipEventCreate(&c->bev[i]) != hipSuccess) c->have_bev = false;
  // look-ahead stream (default priority) and its two events
  c->have_la = hipStreamCreateWithFlags(&c->la.side, hipStreamNonBlocking) == hipSuccess;
  if (c->have_la && hipEventCreateWithFlags(&c->la.ready, hipEventDisableTiming) != hipSuccess) {
    (void)hipStreamDestroy(c->la.side);
    c->have_la = false;
  }
  if (c->have_la && hipEventCreateWithFlags(&c->la.done, hipEventDisableTiming) != hipSuccess) {
    (void)hipEventDestroy(c->la.ready);
    (void)hipStreamDestroy(c->la.side);
    c->have_la = false;
  }
  hipError_t e;
  const size_t vb = field_bytes(c, PQ_FIELD_PHI);
  if ((e = hipMemsetAsync(c->phi, 0, vb, c->s)) != hipSuccess) goto fail;
  if ((e = hipMemsetAsync(c->sigma, 0, field_bytes(c, PQ_FIELD_SIGMA), c->s)) != hipSuccess) goto fail;
  if ((e = launch_lambda_fill(d, c->p.U, c->lam, c->s)) != hipSuccess) goto fail;
  if ((e = launch_dyson(c->p, d, c->sigma, c->g, c->mu, c->s)) != hipSuccess) goto fail;
  if ((e = launch_sigma1(c->p, d, c->g, c->mu, c->sigma, c->sig_ws, c->s)) != hipSuccess) goto fail;
  if ((e = hipStreamSynchronize(c->s)) != hipSuccess) goto fail;
  *out = c;
  return PQ_OK;
fail:
  for (int i = 0; i < 8; ++i)
    if (c->have_events) (void)hipEventDestroy(c->ev[i]);
  for (int i = 0; i < 512; ++i)
    if (c->have_bev) (void)hipEventDestroy(c->bev[i]);
  if (c->have_la) {
    (void)hipEventDestroy(c->la.ready);
    (void)hipEventDestroy(c->la.done);
    (void)hipStreamDestroy(c->la.side);
  }
  delete c;
  return hip_fail(e, "parquet_init");
}

pq_status parquet_iterate(pq_ctx* c, int32_t n_iter, double tol, pq_iter_stats* stats,
                          int32_t* iters_done, int32_t* converged) {
  PQ_CHECK_ARG(c, "null context");
  PQ_CHECK_ARG(n_iter >= 0, "n_iter must be >= 0");
  int done = 0, conv = 0;
  pq_status st = PQ_OK;
  for (int it = 0; it < n_iter; ++it) {
    hipError_t e = hipSuccess;
    BseTiming tm;
    tm.ev = c->bev;
    tm.cap = 256;
    tm.used = 0;
    tm.update_flops = 0.0;
    const bool timing = stats && c->have_bev;
    const char* where = nullptr;
    if ((e = enqueue_iteration(c, c->have_events, timing ? &tm : nullptr, &where, true)) != hipSuccess)
      return hip_fail(e, where);
    double res[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, mu = 0.0;  // norm, flagged, re-solved, unresolved,
                                                                 // max estimate, max |Sigma|
    if ((e = hipMemcpyAsync(res, c->dnorm, sizeof(res), hipMemcpyDeviceToHost, c->s)) != hipSuccess) return hip_fail(e, "norm copy");
    if ((e = hipMemcpyAsync(&mu, c->mu, sizeof(double), hipMemcpyDeviceToHost, c->s)) != hipSuccess) return hip_fail(e, "mu copy");
    if ((e = hipStreamSynchronize(c->s)) != hipSuccess) return hip_fail(e, "iteration");
    const double dn = res[0];
    c->iteration++;
    done++;
    if (stats) {
      memset(stats, 0, sizeof(*stats));
      stats->iteration = c->iteration;
      stats->dsigma = dn;
      stats->mu = mu;
      stats->flagged_blocks = (int32_t)res[1];
      stats->resolved_blocks = (int32_t)res[2];
      stats->unresolved_blocks = (int32_t)res[3];
      stats->max_err_est = res[4];
      if (c->have_events) {
        stats->ms_total = elapsed_ms(c->ev[0], c->ev[6]);
        stats->ms_stage[0] = elapsed_ms(c->ev[0], c->ev[1]);
        stats->ms_stage[1] = elapsed_ms(c->ev[1], c->ev[2]);
        stats->ms_stage[3] = elapsed_ms(c->ev[2], c->ev[3]);
        stats->ms_stage[4] = elapsed_ms(c->ev[3], c->ev[4]);
        stats->ms_stage[5] = elapsed_ms(c->ev[4], c->ev[5]);
        stats->ms_stage[6] = elapsed_ms(c->ev[5], c->ev[6]);
      }
      if (timing) {
        for (int i = 0; i < tm.used; ++i) {
          stats->ms_bse_kernel[tm.kind[i]] += elapsed_ms(c->bev[2 * i], c->bev[2 * i + 1]);
          stats->n_bse_launch[tm.kind[i]] += 1;
        }
        stats->update_flops = tm.update_flops;
      }
    }
    if (!(dn == dn)) {
      set_error("non-finite self-energy at iteration %d", c->iteration);
      st = PQ_ERR_NONFINITE;
      break;
    }
    if (res[3] > 0.0) {
      set_error("%d BSE blocks unresolved at iteration %d (no finite FP64 re-solve, or more flagged blocks than "
                "re-solve slots)", (int)res[3], c->iteration);
      st = PQ_ERR_SINGULAR;
      break;
    }
    if (converged_now(c, dn, res[5], tol)) {
      conv = 1;
      break;
    }
  }
  if (st == PQ_OK && tol != 0.0 && !conv && n_iter > 0) {
    set_error("not converged to %g in %d iterations", tol, done);
    st = PQ_ERR_NOT_CONVERGED;
  }
  if (iters_done) *iters_done = done;
  if (converged) *converged = conv;
  return st;
}

pq_status parquet_iterate_batch(pq_ctx* const* ctxs, int32_t count, int32_t n_iter, double tol,
                                int32_t* iters_done, int32_t* converged) {
  PQ_CHECK_ARG(ctxs && count >= 0 && n_iter >= 0, "bad batch arguments");
  for (int i = 0; i < count; ++i) {
    PQ_CHECK_ARG(ctxs[i], "null context %d", i);
    PQ_CHECK_ARG(ctxs[i]->s != nullptr, "context %d has the null stream (graphs need a created stream)", i);
    for (int j = 0; j < i; ++j)
      PQ_CHECK_ARG(ctxs[j] != ctxs[i] && ctxs[j]->s != ctxs[i]->s, "contexts %d and %d share a stream", j, i);
  }
  for (int i = 0; i < count; ++i) {
    pq_ctx* c = ctxs[i];
    if (c->have_graph && c->graph_has_lam != c->has_lam) {
      (void)hipGraphExecDestroy(c->graph);
      c->have_graph = false;
    }
    if (!c->have_graph) {
      hipGraph_t g = nullptr;
      const char* where = nullptr;
      hipError_t e = hipStreamBeginCapture(c->s, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return hip_fail(e, "graph capture (begin)");
      hipError_t ei = enqueue_iteration(c, false, nullptr, &where);
      e = hipStreamEndCapture(c->s, &g);
      if (ei != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(ei, where);
      }
      if (e != hipSuccess) return hip_fail(e, "graph capture (end)");
      e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) return hip_fail(e, "graph instantiate");
      c->have_graph = true;
      c->graph_has_lam = c->has_lam;
    }
    if (iters_done) iters_done[i] = 0;
    if (converged) converged[i] = 0;
  }
  std::vector<char> active(count, 1);
  std::vector<double> res(6 * (size_t)count, 0.0);
  bool nonfinite = false, singular = false;
  for (int it = 0; it < n_iter; ++it) {
    bool any = false;
    for (int i = 0; i < count; ++i) {
      if (!active[i]) continue;
      any = true;
      hipError_t e = hipGraphLaunch(ctxs[i]->graph, ctxs[i]->s);
      if (e != hipSuccess) return hip_fail(e, "graph launch");
    }
    if (!any) break;
    for (int i = 0; i < count; ++i) {
      if (!active[i]) continue;
      pq_ctx* c = ctxs[i];
      double* r = &res[6 * (size_t)i];
      hipError_t e = hipMemcpyAsync(r, c->dnorm, 6 * sizeof(double), hipMemcpyDeviceToHost, c->s);
      if (e == hipSuccess) e = hipStreamSynchronize(c->s);
      if (e != hipSuccess) return hip_fail(e, "batch iteration");
      c->iteration++;
      if (iters_done) iters_done[i]++;
      if (!(r[0] == r[0])) {
        set_error("non-finite self-energy in context %d at iteration %d", i, c->iteration);
        nonfinite = true;
        active[i] = 0;
      } else if (r[3] > 0.0) {
        if (!nonfinite) set_error("context %d: %d BSE blocks unresolved at iteration %d", i, (int)r[3], c->iteration);
        singular = true;
        active[i] = 0;
      } else if (converged_now(c, r[0], r[5], tol)) {
        if (converged) converged[i] = 1;
        active[i] = 0;
      }
    }
  }
  if (nonfinite) return PQ_ERR_NONFINITE;
  if (singular) return PQ_ERR_SINGULAR;
  if (tol != 0.0 && n_iter > 0) {
    for (int i = 0; i < count; ++i)
      if (active[i]) {
        set_error("context %d not converged to %g in %d rounds", i, tol, n_iter);
        return PQ_ERR_NOT_CONVERGED;
      }
  }
  return PQ_OK;
}

pq_status parquet_field_bytes(pq_ctx* c, int32_t field, size_t* bytes) {
  PQ_CHECK_ARG(c && bytes, "null pointer");
  size_t b = field_bytes(c, field);
  PQ_CHECK_ARG(b > 0, "unknown field %d", field);
  *bytes = b;
  return PQ_OK;
}

pq_status parquet_get(pq_ctx* c, int32_t field, void* dev_dst, size_t bytes) {
  PQ_CHECK_ARG(c && dev_dst, "null pointer");
  size_t b = field_bytes(c, field);
  PQ_CHECK_ARG(b > 0 && bytes == b, "field %d needs %zu bytes, got %zu", field, b, bytes);
  if (field == PQ_FIELD_F) {
    // F = Gamma[Phi] + Phi of the current state: kernels and Gamma from the current Phi
    PQ_CHECK_ARG(dev_dst != c->phi && dev_dst != c->gamma, "destination aliases the context state");
    const pq_params& p = c->p;
    const double lam[4] = {p.U, -p.U, 2.0 * p.U, 0.0};
    hipError_t e = launch_kernel_extract(p, c->d, c->phi, c->k1, c->k2, c->s);
    if (e == hipSuccess)
      e = launch_remap(p, c->d, lam, c->has_lam ? c->lam : nullptr, c->phi, c->k1, c->k2, c->gamma, c->s);
    if (e == hipSuccess)
      e = launch_vertex_sum(c->gamma, c->phi, dev_dst, p.storage, 4 * (size_t)c->d.Nq * c->d.n * c->d.n, c->s);
    if (e == hipSuccess) e = hipStreamSynchronize(c->s);
    return e == hipSuccess ? PQ_OK : hip_fail(e, "parquet_get (F)");
  }
  hipError_t e = hipMemcpyAsync(dev_dst, field_ptr(c, field), b, hipMemcpyDeviceToDevice, c->s);
  if (e == hipSuccess) e = hipStreamSynchronize(c->s);
  return e == hipSuccess ? PQ_OK : hip_fail(e, "parquet_get");
}

pq_status parquet_set(pq_ctx* c, int32_t field, const void* dev_src, size_t bytes) {
  PQ_CHECK_ARG(c && dev_src, "null pointer");
  PQ_CHECK_ARG(field != PQ_FIELD_F, "the full vertex F is derived from Phi and cannot be set");
  size_t b = field_bytes(c, field);
  PQ_CHECK_ARG(b > 0 && bytes == b, "field %d needs %zu bytes, got %zu", field, b, bytes);
  hipError_t e = hipMemcpyAsync(field_ptr(c, field), dev_src, b, hipMemcpyDeviceToDevice, c->s);
  if (e == hipSuccess) e = hipStreamSynchronize(c->s);
  if (e == hipSuccess && field == PQ_FIELD_LAMBDA) c->has_lam = true;
  if (field == PQ_FIELD_SIGMA || field == PQ_FIELD_PHI) c->nhist = 0;     // a new state: no contraction history
  return e == hipSuccess ? PQ_OK : hip_fail(e, "parquet_set");
}

pq_status parquet_warm_start(pq_ctx* c, const void* k1, const void* k2, const void* sigma) {
  PQ_CHECK_ARG(c && k1 && k2, "null pointer");
  hipError_t e = launch_phi_from_kernels(c->p, c->d, (const double2*)k1, (const double2*)k2, c->phi, c->s);
  if (e == hipSuccess && sigma)
    e = hipMemcpyAsync(c->sigma, sigma, field_bytes(c, PQ_FIELD_SIGMA), hipMemcpyDeviceToDevice, c->s);
  if (e == hipSuccess) e = hipStreamSynchronize(c->s);
  c->nhist = 0;
  return e == hipSuccess ? PQ_OK : hip_fail(e, "parquet_warm_start");
}

pq_status parquet_copy_state(pq_ctx* dst, pq_ctx* src) {
  PQ_CHECK_ARG(dst && src, "null context");
  PQ_CHECK_ARG(dst != src, "source and destination are the same context");
  const Dims& a = dst->d;
  const Dims& b = src->d;
  PQ_CHECK_ARG(a.Lx == b.Lx && a.Ly == b.Ly && a.Nv == b.Nv && a.f == b.f,
               "contexts describe different boxes (%dx%d Nv=%d f=%d vs %dx%d Nv=%d f=%d)", a.Lx, a.Ly,
               a.Nv, a.f, b.Lx, b.Ly, b.Nv, b.f);
  hipError_t e = hipStreamSynchronize(src->s);
  if (e != hipSuccess) return hip_fail(e, "parquet_copy_state (source stream)");
  const size_t nsig = sizeof(double2) * (size_t)a.Nve * a.Nk;
  if ((e = hipMemcpyAsync(dst->sigma, src->sigma, nsig, hipMemcpyDeviceToDevice, dst->s)) != hipSuccess)
    return hip_fail(e, "parquet_copy_state (sigma)");
  if ((e = hipMemcpyAsync(dst->mu, src->mu, sizeof(double), hipMemcpyDeviceToDevice, dst->s)) != hipSuccess)
    return hip_fail(e, "parquet_copy_state (mu)");
  const size_t count = 4 * (size_t)a.Nq * a.n * a.n;
  if ((e = launch_convert(src->phi, src->p.storage, dst->phi, dst->p.storage, count, dst->s)) != hipSuccess)
    return hip_fail(e, "parquet_copy_state (phi)");
  if (src->has_lam) {
    if ((e = hipMemcpyAsync(dst->lam, src->lam, field_bytes(src, PQ_FIELD_LAMBDA), hipMemcpyDeviceToDevice,
                            dst->s)) != hipSuccess)
      return hip_fail(e, "parquet_copy_state (lambda)");
  }
  if ((e = hipStreamSynchronize(dst->s)) != hipSuccess) return hip_fail(e, "parquet_copy_state");
  dst->iteration = src->iteration;
  // the history of changes goes along: the contraction is a property of the
  // iteration, not of the precision (the first step on the destination's path
  // adds a jump, which only makes the distance estimate larger)
  dst->nhist = src->nhist;
  for (int k = 0; k < 7; ++k) dst->dhist[k] = src->dhist[k];
  if (src->has_lam) dst->has_lam = true;
  return PQ_OK;
}

pq_status parquet_destroy(pq_ctx* c) {
  if (!c) return PQ_OK;
  if (c->have_la) {
    (void)hipStreamSynchronize(c->la.side);
    (void)hipEventDestroy(c->la.ready);
    (void)hipEventDestroy(c->la.done);
    (void)hipStreamDestroy(c->la.side);
  }
  if (c->have_graph) (void)hipGraphExecDestroy(c->graph);
  if (c->have_events)
    for (int i = 0; i < 8; ++i) (void)hipEventDestroy(c->ev[i]);
  if (c->have_bev)
    for (int i = 0; i < 512; ++i) (void)hipEventDestroy(c->bev[i]);
  delete c;
  return PQ_OK;
}

}  // extern "C"
