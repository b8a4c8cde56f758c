// Batched solver: K independent instances of one box (same lattice, Nv,
// f_ext, storage, precision, mixing and BSE settings; any U, beta, t, t',
// filling, kernel level) iterated together.
//
// The reducible vertices of all instances share one arena laid out
// [4][K][Nq][n][n] (Dims::cs = K Nq n^2 between channels), with the bubbles
// [K][Nq][n], so the Bethe-Salpeter blocks of every active instance in one
// channel are contiguous and one BSE launch sequence (Eq. PA_F_Phi) covers all
// (instance, q) blocks. The per-instance stages (Dyson, bubbles, kernel
// functions, channel remap, Schwinger-Dyson; then the mixing) are launched
// instance after instance around it. One round (one iteration of every active
// instance) is captured on one stream into a single HIP graph, replayed until
// the set of active instances changes. An instance that converges, diverges or fails
// is retired: the last active instance's vertex moves into its arena slot, so
// the active blocks stay a contiguous prefix; the retired instance keeps its
// Sigma, G, mu and kernel functions.
//
// The complex64 BSE update (FP32 and BF16x3 products) has two tile shapes
// (bse_tile); at set-up the batch times both on its own block count and keeps
// the faster one.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "pq_internal.h"

using namespace pq;

namespace {

constexpr int kDn = 8;        // doubles per instance: change, BSE summary (4), max |Sigma|, spare

struct BInst {
  pq_params p;
  Dims d;                     // d.cs = K Nq n^2 (the arena's channel stride)
  double2 *sigma, *sigma_new, *g, *k1, *k2;
  double* mu;
  int iteration, nhist, state;
  double dhist[7], last_dn;
};

struct BatchLayout {
  size_t phi, gamma, xph, xpp, bstats, bse, sig, dn, inst, inst_stride, total;
  size_t bse_bytes, sig_bytes;
  size_t sigma, sigma_new, g, k1, k2, mu;     // offsets inside one instance's region
};

bool batch_dims(const pq_params* ps, int K, std::vector<Dims>* dims) {
  if (!ps || K < 1) { set_error("empty batch"); return false; }
  dims->resize(K);
  for (int i = 0; i < K; ++i) {
    if (!make_dims(&ps[i], &(*dims)[i])) return false;
    const pq_params& a = ps[0];
    const pq_params& b = ps[i];
    if (b.Lx != a.Lx || b.Ly != a.Ly || b.Nv != a.Nv || b.f_ext != a.f_ext || b.storage != a.storage ||
        b.precision != a.precision || b.alpha != a.alpha || b.bse_tol != a.bse_tol ||
        b.resolve_slots != a.resolve_slots) {
      set_error("instance %d differs from instance 0 in the box, the precision, alpha or the BSE settings", i);
      return false;
    }
  }
  const Dims& d = (*dims)[0];
  if ((long long)K * d.Nq > kBseMaxBlocks) {
    set_error("batch of %d instances has %lld BSE blocks per channel, above %d", K, (long long)K * d.Nq,
              kBseMaxBlocks);
    return false;
  }
  for (int i = 0; i < K; ++i) (*dims)[i].cs = (long long)K * d.Nq * d.n * d.n;
  return true;
}

BatchLayout batch_layout(const pq_params* ps, const std::vector<Dims>& dims) {
  const int K = (int)dims.size();
  const Dims& d = dims[0];
  const pq_params& p = ps[0];
  BatchLayout L{};
  size_t off = 0;
  auto take = [&](size_t b) { size_t o = off; off += align256(b); return o; };
  const size_t vb = elem_bytes(p) * 4 * (size_t)K * d.Nq * d.n * d.n;
  L.phi = take(vb);
  L.gamma = take(vb);
  L.xph = take(sizeof(double2) * (size_t)K * d.Nq * d.n);
  L.xpp = take(sizeof(double2) * (size_t)K * d.Nq * d.n);
  L.bstats = take(sizeof(pq_bse_block_stats) * 4 * (size_t)K * d.Nq);
  Dims dk = d;
  dk.Nq = K * d.Nq;
  L.bse_bytes = bse_ws_bytes(p, dk, p.precision);
  L.bse = take(L.bse_bytes);
  size_t sb = 0;
  for (int i = 0; i < K; ++i) sb = std::max(sb, sigma_ws_bytes(dims[i]));
  L.sig_bytes = sb;
  L.sig = take(sb);
  L.dn = take(sizeof(double) * kDn * (size_t)K);
  // one instance's own arrays
  size_t io = 0;
  auto itake = [&](size_t b) { size_t o = io; io += align256(b); return o; };
  const size_t nk = (size_t)d.Nk;
  L.sigma = itake(sizeof(double2) * d.Nve * nk);
  L.sigma_new = itake(sizeof(double2) * d.Nve * nk);
  L.g = itake(sizeof(double2) * d.NG * nk);
  L.k1 = itake(sizeof(double2) * 4 * (size_t)d.Nq);
  L.k2 = itake(sizeof(double2) * 4 * (size_t)d.Nq * d.n);
  L.mu = itake(sizeof(double));
  L.inst_stride = io;
  L.inst = take(io * (size_t)K);
  L.total = off;
  return L;
}

// a deterministic non-zero pattern (|v| = 1e-3) for the tile timing
template <typename C>
__global__ void pattern_kernel(C* v, size_t count) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
    const unsigned h = (unsigned)(i * 2654435761u) ^ (unsigned)(i >> 32);
    v[i].x = (h & 1) ? 1e-3 : -1e-3;
    v[i].y = (h & 2) ? 1e-3 : -1e-3;
  }
}

}  // namespace

struct pq_batch {
  int K;
  pq_params p0;
  Dims d0;                    // instance 0's sizes with the arena stride
  BatchLayout L;
  char* ws;
  hipStream_t s;              // the caller's stream (created, not the null stream)
  std::vector<BInst> inst;
  std::vector<int> at_slot;   // slot -> instance
  int active;
  double* dn_host;            // pinned, kDn per instance
  hipGraphExec_t graph;
  bool have_graph;
  int tile;
  float tile_ms[2];
};

namespace {

char* slot_vertex(pq_batch* b, size_t base, int slot) {
  return b->ws + base + elem_bytes(b->p0) * (size_t)slot * b->d0.Nq * b->d0.n * b->d0.n;
}

double2* slot_x(pq_batch* b, size_t base, int slot) {
  return (double2*)(b->ws + base) + (size_t)slot * b->d0.Nq * b->d0.n;
}

double* inst_dn(pq_batch* b, int i) { return (double*)(b->ws + b->L.dn) + (size_t)kDn * i; }

// the stages before the BSE of the instance in a slot
hipError_t enqueue_pre(pq_batch* b, int slot, const char** where) {
  BInst& x = b->inst[b->at_slot[slot]];
  const double lam[4] = {x.p.U, -x.p.U, 2.0 * x.p.U, 0.0};
  hipStream_t s = b->s;
  void* phi = slot_vertex(b, b->L.phi, slot);
  void* gamma = slot_vertex(b, b->L.gamma, slot);
  double2* xph = slot_x(b, b->L.xph, slot);
  double2* xpp = slot_x(b, b->L.xpp, slot);
  hipError_t e;
  if ((e = launch_dyson(x.p, x.d, x.sigma, x.g, x.mu, s)) != hipSuccess) { *where = "dyson"; return e; }
  if ((e = launch_bubbles(x.p, x.d, x.g, xph, xpp, s)) != hipSuccess) { *where = "bubbles"; return e; }
  if ((e = launch_kernel_extract(x.p, x.d, phi, x.k1, x.k2, s)) != hipSuccess) { *where = "kernels"; return e; }
  if ((e = launch_remap(x.p, x.d, lam, nullptr, phi, x.k1, x.k2, gamma, s)) != hipSuccess) { *where = "remap"; return e; }
  if ((e = launch_sigma(x.p, x.d, phi, x.k1, x.k2, nullptr, x.g, x.mu, x.sigma_new, b->ws + b->L.sig, s)) !=
      hipSuccess) {
    *where = "sigma";
    return e;
  }
  return hipSuccess;
}

// the BSE of every active block of the four channels, on the main stream
hipError_t enqueue_bse(pq_batch* b, int nactive, const char** where) {
  const Dims& d = b->d0;
  Dims r = d;
  r.Nq = nactive * d.Nq;
  const size_t chan = elem_bytes(b->p0) * (size_t)d.cs;
  pq_params p = b->p0;
  p.bse_tile = b->tile;
  for (int c = 0; c < 4; ++c) {
    const double2* x = (const double2*)(b->ws + (c < 2 ? b->L.xph : b->L.xpp));
    hipError_t e = launch_bse(p, r, c, p.precision, b->ws + b->L.gamma + c * chan, x, b->ws + b->L.phi + c * chan,
                              p.alpha, (pq_bse_block_stats*)(b->ws + b->L.bstats) + (size_t)c * b->K * d.Nq,
                              b->ws + b->L.bse, b->s, nullptr);
    if (e != hipSuccess) { *where = "bse"; return e; }
  }
  return hipSuccess;
}

hipError_t enqueue_post(pq_batch* b, int slot, const char** where) {
  const int i = b->at_slot[slot];
  BInst& x = b->inst[i];
  hipStream_t s = b->s;
  const Dims& d = b->d0;
  double* dn = inst_dn(b, i);
  hipError_t e = launch_bse_summary((pq_bse_block_stats*)(b->ws + b->L.bstats) + (size_t)slot * d.Nq, d.Nq, dn + 1,
                                    s, 4, (size_t)b->K * d.Nq);
  if (e != hipSuccess) { *where = "bse summary"; return e; }
  if ((e = launch_mix(x.d, x.sigma_new, x.sigma, x.p.alpha, dn, s, dn + 5)) != hipSuccess) { *where = "mix"; return e; }
  return hipSuccess;
}

// one round of the active instances, captured into b->graph
hipError_t capture_round(pq_batch* b, const char** where) {
  if (b->have_graph) {
    (void)hipGraphExecDestroy(b->graph);
    b->have_graph = false;
  }
  const int A = b->active;
  hipError_t e = hipStreamBeginCapture(b->s, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) { *where = "capture begin"; return e; }
  hipError_t err = hipSuccess;
  for (int slot = 0; slot < A && err == hipSuccess; ++slot) err = enqueue_pre(b, slot, where);
  if (err == hipSuccess) err = enqueue_bse(b, A, where);
  for (int slot = 0; slot < A && err == hipSuccess; ++slot) err = enqueue_post(b, slot, where);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(b->s, &g);
  if (err != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return err;
  }
  if (e != hipSuccess) { *where = "capture end"; return e; }
  e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) { *where = "graph instantiate"; return e; }
  b->have_graph = true;
  return hipSuccess;
}

// retire the instances of the given slots (any order): the last active
// instance's vertex moves into each freed slot
hipError_t retire(pq_batch* b, std::vector<int> slots) {
  std::sort(slots.begin(), slots.end(), [](int x, int y) { return x > y; });
  const size_t blk = elem_bytes(b->p0) * (size_t)b->d0.Nq * b->d0.n * b->d0.n;
  const size_t chan = elem_bytes(b->p0) * (size_t)b->d0.cs;
  for (int slot : slots) {
    const int last = b->active - 1;
    if (slot != last) {
      for (int c = 0; c < 4; ++c) {
        char* base = b->ws + b->L.phi + c * chan;
        hipError_t e = hipMemcpyAsync(base + slot * blk, base + last * blk, blk, hipMemcpyDeviceToDevice, b->s);
        if (e != hipSuccess) return e;
      }
      b->at_slot[slot] = b->at_slot[last];
    }
    b->at_slot[last] = -1;
    b->active--;
  }
  return hipStreamSynchronize(b->s);
}

// bare-vertex start of every instance (Phi = 0, Sigma = Sigma~_1), after the
// tile timing when asked
hipError_t batch_setup(pq_batch* b, bool autotune) {
  const BatchLayout& L = b->L;
  const Dims& d = b->d0;
  const int count = b->K;
  const size_t vb = elem_bytes(b->p0) * 4 * (size_t)count * d.Nq * d.n * d.n;
  const size_t xb = sizeof(double2) * (size_t)count * d.Nq * d.n;
  hipError_t e;
  if ((e = hipMemsetAsync(b->ws + L.phi, 0, vb, b->s)) != hipSuccess) return e;
  if ((e = hipMemsetAsync(b->ws + L.xph, 0, xb, b->s)) != hipSuccess) return e;
  if ((e = hipMemsetAsync(b->ws + L.xpp, 0, xb, b->s)) != hipSuccess) return e;
  if (autotune && (b->p0.precision == PQ_PREC_FP32 || b->p0.precision == PQ_PREC_BF16X3)) {
    // Both update tiles on the batch's own block count: Gamma a fixed pattern,
    // X = 0, so every block is the identity system, F = Gamma and the mixing
    // leaves Phi = 0 (the start state).
    const size_t ve = 4 * (size_t)count * d.Nq * d.n * d.n;
    hipLaunchKernelGGL(pattern_kernel<float2>, dim3(4096), dim3(256), 0, b->s, (float2*)(b->ws + L.gamma), ve);
    hipEvent_t t0, t1;
    if ((e = hipEventCreate(&t0)) != hipSuccess) return e;
    if ((e = hipEventCreate(&t1)) != hipSuccess) {
      (void)hipEventDestroy(t0);
      return e;
    }
    const char* where = nullptr;
    for (int tile = 0; tile < 2 && e == hipSuccess; ++tile) {
      b->tile = tile;
      e = enqueue_bse(b, count, &where);                          // warm-up
      if (e == hipSuccess) e = hipEventRecord(t0, b->s);
      for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) e = enqueue_bse(b, count, &where);
      if (e == hipSuccess) e = hipEventRecord(t1, b->s);
      if (e == hipSuccess) e = hipEventSynchronize(t1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
      b->tile_ms[tile] = ms / 2.f;
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (e != hipSuccess) return e;
    b->tile = b->tile_ms[1] < b->tile_ms[0] ? 1 : 0;
    if ((e = hipMemsetAsync(b->ws + L.phi, 0, vb, b->s)) != hipSuccess) return e;
  }
  for (int i = 0; i < count; ++i) {
    BInst& x = b->inst[i];
    if ((e = hipMemsetAsync(x.sigma, 0, sizeof(double2) * d.Nve * (size_t)d.Nk, b->s)) != hipSuccess) return e;
    if ((e = launch_dyson(x.p, x.d, x.sigma, x.g, x.mu, b->s)) != hipSuccess) return e;
    if ((e = launch_sigma1(x.p, x.d, x.g, x.mu, x.sigma, b->ws + L.sig, b->s)) != hipSuccess) return e;
  }
  return hipStreamSynchronize(b->s);
}

}  // namespace

#define PQB_CHECK_ARG(cond, ...) \
  do {                           \
    if (!(cond)) {               \
      set_error(__VA_ARGS__);    \
      return PQ_ERR_ARG;         \
    }                            \
  } while (0)

extern "C" {

pq_status parquet_batch_query_workspace(const pq_params* ps, int32_t count, size_t* bytes) {
  std::vector<Dims> dims;
  if (!batch_dims(ps, count, &dims)) return PQ_ERR_ARG;
  PQB_CHECK_ARG(bytes, "null output");
  *bytes = batch_layout(ps, dims).total;
  return PQ_OK;
}

pq_status parquet_batch_init(const pq_params* ps, int32_t count, void* ws, size_t ws_bytes, pq_stream stream,
                             int32_t autotune, pq_batch** out) {
  std::vector<Dims> dims;
  if (!batch_dims(ps, count, &dims)) return PQ_ERR_ARG;
  PQB_CHECK_ARG(ws && out, "null pointer");
  PQB_CHECK_ARG(stream != nullptr, "the batch needs a created stream (its rounds are captured into graphs)");
  const BatchLayout L = batch_layout(ps, dims);
  if (ws_bytes < L.total) {
    set_error("batch workspace %zu < %zu bytes", ws_bytes, L.total);
    return PQ_ERR_NOMEM;
  }
  pq_batch* b = new (std::nothrow) pq_batch();
  if (!b) { set_error("host allocation failed"); return PQ_ERR_NOMEM; }
  b->K = count;
  b->p0 = ps[0];
  b->d0 = dims[0];
  b->L = L;
  b->ws = (char*)ws;
  b->s = (hipStream_t)stream;
  b->active = count;
  b->have_graph = false;
  b->tile = 0;
  b->tile_ms[0] = b->tile_ms[1] = 0.f;
  b->dn_host = nullptr;
  hipError_t e = hipHostMalloc((void**)&b->dn_host, sizeof(double) * kDn * count, 0);
  if (e != hipSuccess) {
    set_error("batch pinned memory: %s", hipGetErrorString(e));
    delete b;
    return PQ_ERR_HIP;
  }
  b->inst.resize(count);
  b->at_slot.resize(count);
  for (int i = 0; i < count; ++i) {
    BInst& x = b->inst[i];
    x.p = ps[i];
    x.d = dims[i];
    char* base = b->ws + L.inst + L.inst_stride * i;
    x.sigma = (double2*)(base + L.sigma);
    x.sigma_new = (double2*)(base + L.sigma_new);
    x.g = (double2*)(base + L.g);
    x.k1 = (double2*)(base + L.k1);
    x.k2 = (double2*)(base + L.k2);
    x.mu = (double*)(base + L.mu);
    x.iteration = 0;
    x.nhist = 0;
    x.state = PQ_BATCH_RUNNING;
    x.last_dn = 0.0;
    for (double& h : x.dhist) h = 0.0;
    b->at_slot[i] = i;
  }
  e = batch_setup(b, autotune != 0);
  if (e != hipSuccess) {
    (void)hipHostFree(b->dn_host);
    delete b;
    return hip_fail(e, "parquet_batch_init");
  }
  *out = b;
  return PQ_OK;
}

pq_status parquet_batch_iterate(pq_batch* b, int32_t n_iter, double tol, double diverge, int32_t* active_left) {
  PQB_CHECK_ARG(b && n_iter >= 0 && diverge >= 0.0, "bad batch iterate arguments");
  for (int it = 0; it < n_iter && b->active > 0; ++it) {
    const char* where = nullptr;
    hipError_t e = hipSuccess;
    if (!b->have_graph && (e = capture_round(b, &where)) != hipSuccess) return hip_fail(e, where);
    if ((e = hipGraphLaunch(b->graph, b->s)) != hipSuccess) return hip_fail(e, "batch round");
    if ((e = hipMemcpyAsync(b->dn_host, b->ws + b->L.dn, sizeof(double) * kDn * b->K, hipMemcpyDeviceToHost,
                            b->s)) != hipSuccess)
      return hip_fail(e, "batch norms");
    if ((e = hipStreamSynchronize(b->s)) != hipSuccess) return hip_fail(e, "batch round");
    std::vector<int> done;
    for (int slot = 0; slot < b->active; ++slot) {
      BInst& x = b->inst[b->at_slot[slot]];
      const double* r = b->dn_host + (size_t)kDn * b->at_slot[slot];
      const double dn = r[0];
      x.iteration++;
      x.last_dn = dn;
      int st = PQ_BATCH_RUNNING;
      if (!(dn == dn)) st = PQ_BATCH_NONFINITE;
      else if (r[3] > 0.0) st = PQ_BATCH_SINGULAR;
      else if (diverge > 0.0 && dn > diverge) st = PQ_BATCH_DIVERGED;
      else if (convergence_test(x.dhist, &x.nhist, x.p.alpha, dn, r[5], tol)) st = PQ_BATCH_CONVERGED;
      if (st != PQ_BATCH_RUNNING) {
        x.state = st;
        done.push_back(slot);
      }
    }
    if (!done.empty()) {
      if ((e = retire(b, done)) != hipSuccess) return hip_fail(e, "batch retire");
      if (b->have_graph) {
        (void)hipGraphExecDestroy(b->graph);
        b->have_graph = false;
      }
    }
  }
  if (active_left) *active_left = b->active;
  return PQ_OK;
}

pq_status parquet_batch_status(pq_batch* b, int32_t* iterations, int32_t* state, double* dsigma) {
  PQB_CHECK_ARG(b, "null batch");
  for (int i = 0; i < b->K; ++i) {
    if (iterations) iterations[i] = b->inst[i].iteration;
    if (state) state[i] = b->inst[i].state;
    if (dsigma) dsigma[i] = b->inst[i].last_dn;
  }
  return PQ_OK;
}

pq_status parquet_batch_get(pq_batch* b, int32_t instance, int32_t field, void* dev_dst, size_t bytes) {
  PQB_CHECK_ARG(b && dev_dst, "null pointer");
  PQB_CHECK_ARG(instance >= 0 && instance < b->K, "instance %d outside 0..%d", instance, b->K - 1);
  const BInst& x = b->inst[instance];
  const Dims& d = b->d0;
  const void* src = nullptr;
  size_t need = 0;
  switch (field) {
    case PQ_FIELD_SIGMA: src = x.sigma; need = sizeof(double2) * d.Nve * (size_t)d.Nk; break;
    case PQ_FIELD_G: src = x.g; need = sizeof(double2) * d.NG * (size_t)d.Nk; break;
    case PQ_FIELD_MU: src = x.mu; need = sizeof(double); break;
    case PQ_FIELD_K1: src = x.k1; need = sizeof(double2) * 4 * (size_t)d.Nq; break;
    case PQ_FIELD_K2: src = x.k2; need = sizeof(double2) * 4 * (size_t)d.Nq * d.n; break;
    case PQ_FIELD_PHI: {
      int slot = -1;
      for (int j = 0; j < b->active; ++j)
        if (b->at_slot[j] == instance) slot = j;
      PQB_CHECK_ARG(slot >= 0, "the vertex of retired instance %d is no longer kept", instance);
      const size_t blk = elem_bytes(b->p0) * (size_t)d.Nq * d.n * d.n;
      PQB_CHECK_ARG(bytes == 4 * blk, "field %d needs %zu bytes, got %zu", field, 4 * blk, bytes);
      const size_t chan = elem_bytes(b->p0) * (size_t)d.cs;
      for (int c = 0; c < 4; ++c) {
        hipError_t e = hipMemcpyAsync((char*)dev_dst + c * blk, b->ws + b->L.phi + c * chan + slot * blk, blk,
                                      hipMemcpyDeviceToDevice, b->s);
        if (e != hipSuccess) return hip_fail(e, "parquet_batch_get");
      }
      hipError_t e = hipStreamSynchronize(b->s);
      return e == hipSuccess ? PQ_OK : hip_fail(e, "parquet_batch_get");
    }
    default: PQB_CHECK_ARG(false, "field %d is not kept per batch instance", field);
  }
  PQB_CHECK_ARG(bytes == need, "field %d needs %zu bytes, got %zu", field, need, bytes);
  hipError_t e = hipMemcpyAsync(dev_dst, src, need, hipMemcpyDeviceToDevice, b->s);
  if (e == hipSuccess) e = hipStreamSynchronize(b->s);
  return e == hipSuccess ? PQ_OK : hip_fail(e, "parquet_batch_get");
}

pq_status parquet_batch_tile(pq_batch* b, int32_t* tile, float* ms) {
  PQB_CHECK_ARG(b, "null batch");
  if (tile) *tile = b->tile;
  if (ms) {
    ms[0] = b->tile_ms[0];
    ms[1] = b->tile_ms[1];
  }
  return PQ_OK;
}

pq_status parquet_batch_destroy(pq_batch* b) {
  if (!b) return PQ_OK;
  (void)hipStreamSynchronize(b->s);
  if (b->have_graph) (void)hipGraphExecDestroy(b->graph);
  if (b->dn_host) (void)hipHostFree(b->dn_host);
  delete b;
  return PQ_OK;
}

}  // extern "C"
