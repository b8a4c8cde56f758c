/*
 * parquet.h -- C ABI of the MI355X (gfx950) parquet hot-path library.
 *
 * One iteration of the parquet approximation for the Hubbard model, following
 * G. Li, N. Wentzell, P. Pudleiner, P. Thunstroem, K. Held, "Efficient
 * implementation of the parquet equations -- role of the reducible vertex
 * function and its kernel approximation":
 *
 *   Dyson equation (Eq. PA_Dyson)                      -> dyson_update
 *   G G factors of the Bethe-Salpeter equations         -> bubble_build
 *   first/second-level kernel functions                -> kernel_extract
 *   parquet equations with kernel fill (Eqs. PA_Gamma_dm, PA_Gamma_st)
 *                                                       -> channel_remap
 *   regulated Schwinger-Dyson equation (Eq. PA_Sigma with the auxiliary
 *   vertex of Eq. auxiliary_function and the Sigma~_1/Sigma~_2 split)
 *                                                       -> sigma_sde
 *   Bethe-Salpeter equations (Eq. PA_F_Phi) solved as F = [1 - s Gamma X]^-1 Gamma
 *                                                       -> bse_solve
 *   linear mixing and convergence norm                  -> sigma_mix
 *   the whole loop on one device                        -> parquet_* context API
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Sizes: Nk = Lx*Ly momenta, fermionic box Nv (even) with n in [-Nv/2, Nv/2-1],
 * bosonic box NW = Nv-1 with m in [-(Nv/2-1), Nv/2-1]; extended box Nve = f*Nv
 * fermionic / NWe = f*Nv-1 bosonic; Green's-function grid NG = 2*f*Nv;
 * BSE dimension n = Nk*Nv; number of transfers Nq = Nk*NW.
 * Compound indices are frequency-major: k = (n, K) -> (n + Nv/2)*Nk + K,
 * q = (m, Q) -> (m + Nv/2 - 1)*Nk + Q, K = kx*Ly + ky.
 * Layouts (row-major, complex interleaved re/im):
 *   vertex arrays  [4][Nq][n][n]  channels (d, m, s, t), "storage" precision
 *   G              [NG][Nk]        complex double
 *   Sigma          [Nve][Nk]       complex double
 *   X_ph, X_pp     [Nq][n]         complex double
 *   K1             [4][Nq]         complex double
 *   K2             [4][Nq][n]      complex double
 * Storage precision: PQ_STORE_C64 (float2) or PQ_STORE_C128 (double2).
 *
 * Ownership: every pointer is caller-owned device memory (except pq_params and
 * the host stats structs). The library never allocates or frees device memory;
 * scratch comes from the caller's workspace, sized by the *_workspace queries.
 * Asynchrony: stage entry points only enqueue work on the given stream and
 * return; errors of the enqueued kernels surface at the next synchronising
 * call. Invalid sizes or null pointers return PQ_ERR_ARG before anything is
 * enqueued. No C++ exception crosses this interface. parquet_last_error()
 * returns a thread-local message for the last failing call.
 */
#ifndef PARQUET_H
#define PARQUET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void* pq_stream;   /* a hipStream_t (0 = the legacy default stream) */

typedef enum {
  PQ_OK = 0,
  PQ_ERR_ARG = 1,          /* invalid argument, nothing enqueued            */
  PQ_ERR_HIP = 2,          /* a HIP runtime call failed                      */
  PQ_ERR_NOMEM = 3,        /* workspace too small                            */
  PQ_ERR_SINGULAR = 4,     /* context API: a BSE block of the last iteration
                              is unresolved (stats bit 3: no finite FP64
                              solution, or flagged beyond the re-solve slots) */
  PQ_ERR_NOT_CONVERGED = 5,/* context API: n_iter iterations done, the
                              convergence test (tol != 0) not met (the state
                              is valid; call again)                          */
  PQ_ERR_NONFINITE = 6     /* NaN/Inf in Sigma                               */
} pq_status;

typedef enum { PQ_STORE_C128 = 0, PQ_STORE_C64 = 1 } pq_storage;

typedef enum {
  PQ_PREC_FP64 = 0,        /* complex128 elimination, FP64 MFMA              */
  PQ_PREC_FP32 = 1,        /* complex64 elimination, FP32 MFMA               */
  PQ_PREC_BF16X3 = 2       /* complex64 elimination whose rank-NB updates and
                              pivot-row steps (full panels) split each FP32
                              operand into two bf16 parts and keep three of
                              the four cross products on the bf16 matrix
                              cores, FP32 accumulation (per-product relative
                              error ~1e-5); the diagonal-block inversion and
                              ragged panels as PQ_PREC_FP32                   */
} pq_precision;

typedef enum { PQ_CH_D = 0, PQ_CH_M = 1, PQ_CH_S = 2, PQ_CH_T = 3 } pq_channel;

/* Model and numerical parameters of one parquet instance. */
typedef struct {
  int32_t Lx, Ly;          /* lattice; Lx = Ly = 1 selects the local mode    */
  int32_t Nv;              /* fermionic box size, even, >= 2                 */
  int32_t f_ext;           /* extension factor of the regulation box, >= 1   */
  int32_t kernel_level;    /* 0 truncation, 1 K1 only, 2 K1 + K2             */
  int32_t edge_rule;       /* 0 far edge per channel and sign of m, 1 lowest */
  int32_t mu_mode;         /* 0 fixed mu~ = mu_fixed, 1 bisection on filling */
  int32_t storage;         /* pq_storage of the vertex arrays                */
  int32_t precision;       /* pq_precision of the BSE                        */
  int32_t resolve_slots;   /* complex64 BSE: at most this many flagged blocks
                              per channel are re-solved in FP64 (0: as many
                              as a re-solve budget of 2.5 GiB holds, at
                              least 8, at most Nq)                           */
  int32_t regulation;      /* 1: the Schwinger-Dyson equation with the high-
                              frequency regulation (Sigma~_1 + Sigma~_2 + the
                              box part of F - F~); 0: Eq. PA_Sigma plainly
                              summed over the box with the full F, Sigma on
                              the box only (requires f_ext = 1; the ablation
                              the regulation is measured against)           */
  int32_t bse_tile;        /* complex64 (FP32 and BF16x3) BSE update tile: 0
                              the 128 x 128 workgroup tile (64 x 64 per
                              wave), 1 the 128 x 64 tile (64 x 32 per wave:
                              more workgroups for small systems; with BF16x3
                              products also operand loads two steps ahead);
                              complex128 has one tile. Both run the same
                              products in the same order; they agree to FP32
                              rounding (the BF16x3 narrow tile adds C after
                              the products, a different FP32 summation
                              order); the batched solver picks by timing.   */
  double U, beta, t, tp;   /* interaction, inverse temperature, hoppings     */
  double filling;          /* total density n for mu_mode = 1                */
  double D;                /* semicircle half-bandwidth (local mode)         */
  double mu_fixed;
  double alpha;            /* linear mixing of Sigma and Phi, (0, 1]         */
  double bse_tol;          /* complex64 BSE: a block whose estimated relative
                              error |F - F_exact|_F / |F|_F exceeds this is
                              re-solved in FP64 (0 selects 2e-5)             */
} pq_params;

/* Sizes derived from pq_params (filled by pq_dims_from_params). */
typedef struct {
  int32_t Lx, Ly, Nk, Nv, NW, f_ext, Nve, NWe, NG, n, Nq, ntau;
  int64_t vertex_elems;    /* Nq*n*n per channel */
} pq_dims;

/* Validate params and derive sizes; PQ_ERR_ARG if inconsistent. */
pq_status pq_dims_from_params(const pq_params* p, pq_dims* out);

/* Human-readable message of the last failing call on this thread. */
const char* parquet_last_error(void);

/* ------------------------------------------------------------------ stages */

/* Dyson equation (Eq. PA_Dyson) on the G grid: G = 1/(i nu + mu~ - eps_K - Sigma)
 * (lattice, Hartree absorbed into mu~) or 1/(1/G0 - Sigma) (local, semicircle
 * G0). Sigma is taken as zero outside the extended box. With mu_mode = 1, mu~
 * is found by bisection so that 2 n_sigma = filling, the density including the
 * exact tail beyond the grid. sigma: [Nve][Nk] c128 (read); g_out: [NG][Nk]
 * c128 (written); mu_out: one device double (written). */
pq_status dyson_update(const pq_params* p, const void* sigma, void* g_out,
                       void* mu_out, pq_stream stream);

/* X_ph(k;q) = (T/N) G(k) G(k+q), X_pp(k;q) = (T/2N) G(k) G(q-k) for k in the
 * box (the G G factors of Eq. PA_F_Phi). g: [NG][Nk]; xph, xpp: [Nq][n] c128. */
pq_status bubble_build(const pq_params* p, const void* g, void* xph, void* xpp,
                       pq_stream stream);

/* Kernel functions (two-level kernel approximation): K1_r(q) = mean over K,K'
 * of Phi_r at both fermionic arguments on the box edge n_e, K2_r(k;q) = mean
 * over K' of Phi_r^{k,(n_e,K')}(q) - K1_r(q). n_e: the edge away from the
 * stripes (ph channels: top edge for m > 0, bottom for m < 0; pp channels the
 * opposite; both edges averaged at m = 0), or the bottom edge with
 * edge_rule = 1. kernel_level 1 zeroes K2, level 0 zeroes both.
 * phi: [4][Nq][n][n] (storage precision); k1: [4][Nq] c128; k2: [4][Nq][n] c128. */
pq_status kernel_extract(const pq_params* p, const void* phi, void* k1, void* k2,
                         pq_stream stream);

/* Parquet equations (Eqs. PA_Gamma_dm, PA_Gamma_st): for every (q, k, k') in
 * the box, Gamma_r = Lambda_r + the eight remapped reducible vertices
 *   d/m: Phi_{d,m}(k, k+q; k'-k), Psi_{s,t}(k, k'; k+k'+q)
 *   s/t: Phi_{d,m}(k, q-k'; k'-k), Phi_{d,m}(k, k'; q-k-k')
 * with the stored Phi when every argument is inside the box and the kernel
 * value K1(p) + [k1 in box] K2(k1;p) + [k2 in box] K2(k2;p) otherwise (zero
 * when the transfer p leaves the bosonic box). lambda: 4 host doubles
 * (the parquet approximation uses U, -U, 2U, 0). lambda_box: nullable device
 * array [4][Nv-1][Nv][Nv] complex128, a local fully irreducible vertex
 * Lambda_r(m; n, n') (results section: full parquet / parquet DGA take a
 * local Lambda, extended outside the box by U, -U, 2U, 0), index
 * [r][m + Nv/2 - 1][n + Nv/2][n' + Nv/2], used in place of lambda at every
 * momentum. phi, gamma_out: [4][Nq][n][n] storage precision, must not alias.
 * f_out (nullable, same layout, must alias neither): the full vertex
 * F_r = Gamma_r + Phi_r (Eq. PA_F_G), which is Eq. PA_F. */
pq_status channel_remap(const pq_params* p, const double lambda[4], const void* lambda_box,
                        const void* phi, const void* k1, const void* k2, void* gamma_out,
                        void* f_out, pq_stream stream);

/* Workspace bytes for sigma_sde. */
pq_status sigma_sde_workspace(const pq_params* p, size_t* bytes);

/* Regulated Schwinger-Dyson equation (high-frequency regulation subsection):
 *   Sigma(k) = Sigma~_1(k) + Sigma~_2(k) + [k in box] Sigma_box(k)
 * Sigma~_1: second-order diagram over all Matsubara frequencies through
 * imaginary time; Sigma~_2: (F~ - Lambda) summed over the extended box;
 * Sigma_box: (F - F~) over the box, F = Gamma + Phi built from Phi by the
 * parquet equations (no Gamma input needed), F~ from the kernel functions.
 * FP64 accumulation throughout. phi: [4][Nq][n][n]; k1, k2: kernel tables;
 * lambda_box: nullable, the box Lambda of channel_remap; its difference from
 * (U, -U, 2U, 0) is part of F - F~ and adds to Sigma_box (F~ keeps the
 * parquet-approximation values); g: [NG][Nk]; mu: device double from
 * dyson_update; sigma_out: [Nve][Nk] c128. ws: device workspace of
 * sigma_sde_workspace bytes.
 * With params.regulation = 0 (f_ext = 1): Eq. PA_Sigma summed plainly over
 * the box with the full F, computed as the same pieces on the box with
 * Sigma~_1 replaced by the second-order diagram truncated to the box
 * (the plain box sum of F splits exactly that way). */
pq_status sigma_sde(const pq_params* p, const void* phi, const void* k1,
                    const void* k2, const void* lambda_box, const void* g, const void* mu,
                    void* sigma_out, void* ws, size_t ws_bytes, pq_stream stream);

/* sigma_sde without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same computation, its scratch taken from a
 * static device array of 64 MiB that each GPU holds from the library's load
 * until the process ends. No device memory is allocated or freed. Parameter
 * sets whose sigma_sde_workspace exceeds 64 MiB return PQ_ERR_NOMEM before
 * anything is enqueued (the 8x8, Nv = 16, f = 2 box needs 6.9 MB). Every call
 * on one GPU shares that GPU's scratch: calls that overlap on one GPU (other
 * streams, other threads) race; calls on one stream are ordered. The stream
 * must belong to the current device. Arguments as sigma_sde. */
pq_status sigma_sde_no_alloc(const pq_params* p, const void* phi, const void* k1, const void* k2,
                             const void* lambda_box, const void* g, const void* mu, void* sigma_out,
                             pq_stream stream);

/* Workspace bytes for bse_solve on one channel. */
pq_status bse_workspace(const pq_params* p, size_t* bytes);

/* Per-block diagnostics written by bse_solve (device memory, Nq entries). */
typedef struct {
  float min_pivot;       /* smallest |pivot| / largest |pivot| of the block  */
  float growth;          /* largest |entry| of the inverted diagonal blocks
                            (a lower bound of |A^-1| for the last block)     */
  int32_t flags;         /* bit 0: flagged; complex64 paths: for the FP64
                            re-solve (weak pivots: ratio below 1e-3 or growth
                            above 1e3; a non-finite pivot; or an error
                            estimate above the tolerance), complex128 path:
                            weak pivots (ratio below 1e-10 or growth above
                            1e12, a warning only);
                            bit 1: non-finite values in the elimination;
                            bit 2: re-solved in FP64 (complex64 paths);
                            bit 3: unresolved -- flagged but not re-solved
                            (no re-solve slot left, or the FP64 re-solve was
                            not finite), or non-finite on the complex128
                            path; the block's Phi is not trusted;
                            bit 4: error estimate above the tolerance        */
  float err_est;         /* complex64 paths: estimated relative error of the
                            complex64 solution F (before any re-solve; +inf
                            if non-finite); 0 on the complex128 path         */
} pq_bse_block_stats;

/* Bethe-Salpeter equation of one channel (Eq. PA_F_Phi) for every transfer q:
 *   F = [1 - s_r Gamma_r X_r]^-1 Gamma_r,  s = (+1, +1, -1, +1) for (d, m, s, t),
 *   X = X_ph for d, m and X_pp for s, t,
 *   phi_io <- alpha (F - Gamma_r) + (1 - alpha) phi_io   (alpha = 1: plain output).
 * Elimination without row exchanges (A is the identity minus a small-norm
 * kernel); the pivot monitor flags weak blocks in stats (nullable).
 * Error control of the complex64 paths (FP32, BF16x3): after the solve, the
 * relative error |F^ - F|_F / |F|_F of every block's complex64 solution F^ is
 * estimated in FP64 from the residual R = A F^ - Gamma and A^-1 = 1 + s F X
 * (which follows from F = A^-1 Gamma): a screen for every block, with R
 * sampled through two fixed pseudo-random probe vectors on a sample of 128
 * rows and columns (all for n <= 256) and the expected amplification
 * |A^-1|_F / n^1/2 from tr(F X) and |F X|_F, and, where the screen exceeds
 * half the tolerance or |A^-1|_F / n^1/2 exceeds 2, the error E v = A^-1 R v
 * of eight probe vectors itself (max over the probes). Blocks with weak
 * pivots, a non-finite value or an estimate above params.bse_tol (default
 * 2e-5) are solved again in FP64 from the same Gamma and their Phi takes the
 * mixing of the FP64 F; at most resolve_slots blocks per call (in q order,
 * weak-pivot blocks first), the others keep the complex64 result and stats
 * bit 3. The workspace includes the room for the re-solve. Errors of the
 * enqueued kernels cannot be returned by this enqueue-only call: check stats
 * (bit 3) or use the context API, which returns PQ_ERR_SINGULAR for them.
 * gamma: [Nq][n][n] (one channel), chi0: [Nq][n] c128, phi_io: [Nq][n][n],
 * both in storage precision; stats: [Nq] pq_bse_block_stats (device,
 * nullable); ws: bse_workspace bytes. */
pq_status bse_solve(const pq_params* p, int32_t channel, int32_t precision,
                    const void* gamma, const void* chi0, void* phi_io, double alpha,
                    void* stats, void* ws, size_t ws_bytes, pq_stream stream);

/* sigma_io <- alpha sigma_new + (1 - alpha) sigma_io on [Nve][Nk] c128 and
 * dnorm_out (device double) <- max |sigma_new - sigma_io_old|. */
pq_status sigma_mix(const pq_params* p, const void* sigma_new, void* sigma_io,
                    double alpha, void* dnorm_out, pq_stream stream);

/* ------------------------------------------------------ learned warm start */

/* Second-level kernel approximation of the reducible vertex on the whole box
 * (Sec. "Two-level kernel approximations"): phi_out_r(q; k, k') = K1_r(q) +
 * K2_r(k; q) + K2_r(k'; q), from k1 [4][Nq] and k2 [4][Nq][n] complex128;
 * phi_out [4][Nq][n][n] in the storage precision of p. Used to start the
 * iteration from predicted kernel functions instead of the bare vertex. */
pq_status phi_from_kernels(const pq_params* p, const void* k1, const void* k2, void* phi_out,
                           pq_stream stream);

/* Reference streams for the memory-bound stages (not part of the method):
 * mode 0 copies bytes from src to dst, 1 reads bytes from src (dst receives
 * one float per workgroup: at least 64 KiB), 2 writes bytes to dst; float4
 * accesses over a grid of at most 16384 workgroups. bytes: a positive multiple
 * of 16. Measures what a kernel with the same read and write volumes can
 * reach on this device. */
pq_status hbm_stream(int32_t mode, const void* src, void* dst, size_t bytes, pq_stream stream);

/* A multilayer perceptron x [batch][w0] -> tanh hidden layers -> linear output
 * [batch][w_L] (widths: n_layers + 1 host ints). Parameters: params (float)
 * packed layer by layer as [W_l (w_{l+1} x w_l, row-major), b_l (w_{l+1})],
 * mlp_param_count entries, and params_bf16, the same array rounded to bf16
 * (to nearest even). The products run on the bf16 matrix cores with FP32
 * accumulation: weights as their bf16 copy, FP32 activations and gradients as
 * two bf16 terms (hi + lo, about 2^-16 relative), so the result is that of
 * FP32 operands with bf16 weights; biases and activations are FP32. acts:
 * device floats, batch * (w_1 + ... + w_L), the outputs of every layer, the
 * network output last. 1 <= n_layers <= 16, 1 <= widths <= 4194240 and
 * 1 <= batch <= 4194240 (ERR_ARG otherwise). Used for the learned warm start,
 * model parameters -> kernel functions (an addition to the paper's method,
 * which starts from the bare vertex). */
pq_status mlp_param_count(const int32_t* widths, int32_t n_layers, size_t* count);
pq_status mlp_forward(const int32_t* widths, int32_t n_layers, const void* params_bf16, const float* params,
                      const float* x, float* acts, int32_t batch, pq_stream stream);
/* Gradient of the mean squared error between the output (last block of acts,
 * from mlp_forward) and target [batch][w_L] with respect to params (grad:
 * same layout; the weight gradient is taken at the bf16 weights), and the loss
 * itself (one device float). scratch: 2 * batch * max(widths) floats. */
pq_status mlp_backward(const int32_t* widths, int32_t n_layers, const void* params_bf16, const float* x,
                       const float* acts, const float* target, float* grad, float* loss, float* scratch,
                       int32_t batch, pq_stream stream);
/* One bias-corrected Adam step (step counts from 1) on params with moments m,
 * v (count floats each), refreshing params_bf16; mlp_to_bf16 only refreshes it. */
pq_status mlp_adam(float* params, void* params_bf16, float* m, float* v, const float* grad, size_t count,
                   float lr, float beta1, float beta2, float eps, int32_t step, pq_stream stream);
pq_status mlp_to_bf16(const float* params, void* params_bf16, size_t count, pq_stream stream);
/* Factorised output head of the warm-start network. mlp_basis takes rows
 * training outputs y [rows][len] (device floats, overwritten) and leaves in y
 * an orthonormal basis q_0 .. q_{rows-1} of their centred span (classical
 * Gram-Schmidt with one re-orthogonalisation pass, FP64 dot products; a row
 * with no new direction, its residual below 1e-6 of its centred norm, becomes
 * zero), in mean [len] their mean, in coef [rows][ld_coef] (ld_coef >= rows)
 * the coordinates of sample i, y_i = mean + scale sum_j coef[i][j] q_j
 * (zero for j > i), divided by scale [1 float] = their root mean square. The
 * network then predicts the rows coordinates; mlp_expand rebuilds out [len]
 * (device doubles) = mean + scale sum_j coef[j] q_j from one predicted
 * coordinate vector coef [rows] (device floats). ws: mlp_basis_workspace
 * bytes of device memory. 1 <= rows <= 4096, len >= 1. */
pq_status mlp_basis_workspace(int32_t rows, size_t* bytes);
pq_status mlp_basis(float* y, int32_t rows, size_t len, float* mean, float* coef, int32_t ld_coef, float* scale,
                    void* ws, pq_stream stream);
pq_status mlp_expand(const float* q, int32_t rows, size_t len, const float* mean, const float* coef,
                     const float* scale, double* out, pq_stream stream);

/* ------------------------------------------------------------ context API */

typedef struct pq_ctx pq_ctx;

typedef enum {
  PQ_FIELD_SIGMA = 0,  /* [Nve][Nk] c128           */
  PQ_FIELD_G = 1,      /* [NG][Nk] c128            */
  PQ_FIELD_PHI = 2,    /* [4][Nq][n][n] storage    */
  PQ_FIELD_GAMMA = 3,  /* [4][Nq][n][n] storage    */
  PQ_FIELD_K1 = 4,     /* [4][Nq] c128             */
  PQ_FIELD_K2 = 5,     /* [4][Nq][n] c128          */
  PQ_FIELD_MU = 6,     /* 1 double                 */
  PQ_FIELD_XPH = 7,    /* [Nq][n] c128             */
  PQ_FIELD_XPP = 8,    /* [Nq][n] c128             */
  PQ_FIELD_LAMBDA = 9, /* [4][Nv-1][Nv][Nv] c128: local Lambda on the box (channel_remap's
                          lambda_box); (U, -U, 2U, 0) after init; setting it makes the
                          context iterate with it (full parquet / parquet DGA input) */
  PQ_FIELD_F = 10      /* [4][Nq][n][n] storage, get only: the full vertex of the
                          current state, F_r = Gamma_r[Phi] + Phi_r (Eq. PA_F_G), with
                          the kernel functions and Gamma recomputed from the current
                          Phi (this refreshes the K1, K2 and GAMMA fields) */
} pq_field;

typedef struct {
  int32_t iteration;       /* iterations done since init                       */
  int32_t flagged_blocks;  /* BSE blocks flagged (stats bit 0) in the last iteration */
  double dsigma;           /* max |Sigma_new - Sigma_old| of the last iteration */
  double mu;               /* mu~ used by the last iteration                    */
  /* Timings from device events: NaN where an event pair cannot be read. */
  double ms_total;         /* wall time of the last iteration (device events)   */
  double ms_stage[8];      /* dyson, bubbles+kernels, -, remap, sigma, bse (4 channels), mix, - */
  /* BSE of the density channel, per kernel kind (init, pivot and multiplier
   * copy, pivot rows, update, a separate mixing pass (no longer used: 0
   * launches), error estimate and FP64 re-solve): summed device time of its
   * launches and the number of launches. The update includes the back
   * substitution and the mixing fused into it; the last kind runs on the
   * complex64 paths. */
  double ms_bse_kernel[6];
  int32_t n_bse_launch[6];
  int32_t resolved_blocks;   /* blocks re-solved in FP64 (stats bit 2), last iteration */
  int32_t unresolved_blocks; /* unresolved blocks (stats bit 3), last iteration        */
  double update_flops;     /* matrix-core flops of those update launches (8 per complex MAC) */
  double max_err_est;      /* largest BSE error estimate of the last iteration (complex64) */
} pq_iter_stats;

/* Device bytes parquet_init needs in its workspace. */
pq_status parquet_query_workspace(const pq_params* p, size_t* bytes);

/* Bind a context to caller workspace and stream, and set the bare-vertex start:
 * Phi_r = 0, Sigma_0 = Sigma~_1[G_0] (second-order diagram of the Sigma = 0 G;
 * without the regulation its box truncation). */
pq_status parquet_init(const pq_params* p, void* ws, size_t ws_bytes, pq_stream stream,
                       pq_ctx** out);

/* Run up to n_iter iterations (Dyson -> bubbles -> kernels -> remap -> SDE ->
 * BSE -> mixing), stopping early on the convergence test of tol:
 *   tol > 0: the change max|Sigma_new - Sigma_old| is below tol;
 *   tol < 0: the estimated distance of the mixed Sigma to the fixed point is
 *            below |tol| max|Sigma|, i.e. alpha dmax / (1 - rho) < |tol|
 *            max|Sigma| with dmax the largest change of the last six
 *            iterations and rho the contraction per iteration, the geometric
 *            mean of the last six ratios of successive changes (seven
 *            iterations of this state needed, rho < 0.98; the history
 *            restarts after parquet_set of SIGMA or PHI and goes along
 *            with parquet_copy_state);
 *   tol = 0: never (exactly n_iter iterations).
 * Synchronises once per iteration for the norm and a summary of the BSE block
 * flags. stats: host, nullable. Returns PQ_OK (converged, or tol = 0 and n_iter
 * done), PQ_ERR_NOT_CONVERGED (tol != 0 not reached in n_iter),
 * PQ_ERR_NONFINITE (the new self-energy is not finite) or PQ_ERR_SINGULAR (a
 * BSE block is unresolved); the last two stop after the iteration that met
 * them, whose results are kept (*iters_done counts it). */
pq_status parquet_iterate(pq_ctx* ctx, int32_t n_iter, double tol, pq_iter_stats* stats,
                          int32_t* iters_done, int32_t* converged);

/* Iterate several contexts at once, for many small instances that do not fill
 * the GPU alone (each may have its own box and parameters). On first use each
 * context captures one whole iteration (the launches of parquet_iterate,
 * without timing) into a HIP graph on its stream, again after its box Lambda
 * setting changed. Every round replays the graphs of the contexts that are
 * still active, each on its own stream, then reads each norm (one
 * synchronisation per context per round) and retires the converged ones
 * (the test of parquet_iterate with tol), those with a
 * non-finite self-energy and those with an unresolved BSE block (the others
 * continue). Returns the most severe outcome over the contexts:
 * PQ_ERR_NONFINITE, then PQ_ERR_SINGULAR, then PQ_ERR_NOT_CONVERGED (tol != 0
 * and a context still active after n_iter rounds), else PQ_OK.
 * ctxs: count contexts with distinct, created (non-null) streams;
 * iters_done, converged: host arrays of count entries, nullable. Not for
 * contexts another thread uses at the same time. */
pq_status parquet_iterate_batch(pq_ctx* const* ctxs, int32_t count, int32_t n_iter, double tol,
                                int32_t* iters_done, int32_t* converged);

/* Copy a state field out of / into the context (device-to-device, on the
 * context stream; synchronises). bytes must equal the field size. */
pq_status parquet_get(pq_ctx* ctx, int32_t field, void* dev_dst, size_t bytes);
pq_status parquet_set(pq_ctx* ctx, int32_t field, const void* dev_src, size_t bytes);

/* Byte size of a field for this context. */
pq_status parquet_field_bytes(pq_ctx* ctx, int32_t field, size_t* bytes);

/* Warm start of a context: Phi is rebuilt on the whole box from kernel values
 * k1 [4][Nq] and k2 [4][Nq][n] (complex128, device) in the second-level kernel
 * form of Sec. "Two-level kernel approximations" (as phi_from_kernels), in
 * place in the context's storage, and Sigma is taken from sigma [Nve][Nk]
 * (complex128, device) unless it is null. The history of changes used by the
 * relative convergence test restarts. Synchronous on the context's stream. */
pq_status parquet_warm_start(pq_ctx* ctx, const void* k1, const void* k2, const void* sigma);

/* Copy the iteration state of src into dst: Sigma, mu~, the reducible
 * vertices Phi_r (converted between complex64 and complex128 storage as the
 * two contexts require; widening is exact) and the iteration count. Both
 * contexts must describe the same box (Lx, Ly, Nv, f_ext) and live on the
 * current device. Typical use: iterate a complex64/FP32 context until the
 * change of Sigma is small, copy its state into a complex128/FP64 context and
 * finish there, so that the converged solution carries FP64 accuracy while
 * most iterations run on the FP32 path (the parquet iteration is a fixed
 * point map, so the FP32 rounding of the starting state is iterated away).
 * Enqueued on dst's stream after src's stream has been synchronised;
 * synchronises dst's stream. PQ_ERR_ARG if the boxes differ. */
pq_status parquet_copy_state(pq_ctx* dst, pq_ctx* src);

pq_status parquet_destroy(pq_ctx* ctx);

/* ------------------------------------------------------------ batched solver
 * Many independent instances of one box iterated together (an addition to
 * the paper's method, which treats one instance at a time). The count
 * instances ps[0 .. count) must agree in Lx, Ly, Nv, f_ext, storage,
 * precision, alpha, bse_tol and resolve_slots (PQ_ERR_ARG otherwise); U, beta,
 * t, t', the filling, mu_mode, the kernel level, the edge rule and the
 * regulation may differ. No box Lambda (the scalars (U, -U, 2U, 0) of each
 * instance). count * Nq <= 16384.
 *
 * The reducible vertices live in one arena [4][count][Nq][n][n], so the BSE of
 * one channel (Eq. PA_F_Phi) is one launch sequence over every (instance, q)
 * block; the other stages run instance after instance around it, and one
 * round (an iteration of every active instance) is one HIP graph.
 * Each instance keeps its own convergence history and test (tol as in
 * parquet_iterate); an instance that converges, whose Sigma is not finite,
 * whose BSE left a block unresolved, or whose change exceeds diverge (> 0) is
 * retired and no longer iterated (its vertex slot is reused; Sigma, G, mu,
 * K1 and K2 stay readable).
 *
 * parquet_batch_init starts every instance from the bare vertex; with
 * autotune != 0 and complex64 products (FP32 or BF16x3) it first times both update tiles
 * (pq_params.bse_tile) of the batch's BSE on its own block count and keeps the
 * faster (parquet_batch_tile reports the choice and the times, ms per launch
 * sequence of one channel). ws: parquet_batch_query_workspace bytes, owned by
 * the caller. stream: a created stream (not the null stream; the rounds are
 * captured into graphs on it) that the batch uses until it is destroyed;
 * every call is synchronous.
 * parquet_batch_iterate runs up to n_iter rounds, stopping early when no
 * instance is active (active_left: the number still active).
 * parquet_batch_status fills, per instance, the iterations done, the state
 * (pq_batch_state) and the last change of Sigma (arrays of count; each
 * pointer may be null). parquet_batch_get copies one instance's field
 * (PQ_FIELD_SIGMA, G, MU, K1, K2; PHI only while the instance is active) to
 * device memory; bytes must equal the field size. */
typedef struct pq_batch pq_batch;
typedef enum {
  PQ_BATCH_RUNNING = 0,
  PQ_BATCH_CONVERGED = 1,
  PQ_BATCH_DIVERGED = 2,   /* change of Sigma above the diverge bound        */
  PQ_BATCH_NONFINITE = 3,  /* NaN/Inf in Sigma                               */
  PQ_BATCH_SINGULAR = 4    /* a BSE block unresolved                         */
} pq_batch_state;
pq_status parquet_batch_query_workspace(const pq_params* ps, int32_t count, size_t* bytes);
pq_status parquet_batch_init(const pq_params* ps, int32_t count, void* ws, size_t ws_bytes, pq_stream stream,
                             int32_t autotune, pq_batch** out);
pq_status parquet_batch_iterate(pq_batch* b, int32_t n_iter, double tol, double diverge, int32_t* active_left);
pq_status parquet_batch_status(pq_batch* b, int32_t* iterations, int32_t* state, double* dsigma);
pq_status parquet_batch_get(pq_batch* b, int32_t instance, int32_t field, void* dev_dst, size_t bytes);
pq_status parquet_batch_tile(pq_batch* b, int32_t* tile, float* ms);
pq_status parquet_batch_destroy(pq_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* PARQUET_H */
