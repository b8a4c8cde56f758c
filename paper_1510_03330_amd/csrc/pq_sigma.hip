// Regulated Schwinger-Dyson self-energy (high-frequency regulation subsection
// of the paper, Eq. PA_Sigma with the auxiliary vertex):
//
//   Sigma(k) = Sigma~_1(k) + Sigma~_2(k) + [k in box] Sigma_box(k)
//
// Sigma~_1 is the second-order diagram -U^2 G(r)^2 G(-r) over all Matsubara
// frequencies. G is split into its non-interacting pole part (transformed to
// imaginary time analytically, anti-periodic) and a correction supported on
// the extended box (a finite Fourier sum); the tau integral is analytic on
// [0, beta] and is done by Gauss-Legendre quadrature, momenta by direct
// lattice Fourier sums.
//
// Sigma~_2 and Sigma_box are evaluated in "native" variables: every term of
// F - F~ (resp. F~ - Lambda) is a reducible vertex P_r(k, b; p) at its own
// argument triple, so substituting (k', q) -> (b, p) turns both sums into
//   C sum_{p in bosonic box} sum_b { A1 [P_d W16 - P_m (W16 + 2 W25)] + A3 (P_s + P_t) W34 }
// with A1 = G(k+p) G(b+p) G(b), A3 = G(p-b) G(p-k) G(b), C = -U T^2 / 4N^2 and
// integer indicator weights W that encode which original (k', q) lie in the
// summation domain. The box part then only streams Phi (no Gamma, no
// gathers), and the kernel part only needs contiguous rows of K2.
#include <math.h>

#include <mutex>

#include "pq_internal.h"

namespace pq {

namespace {

constexpr int kThreads = 256;
constexpr int kPoles = 128;   // semicircle pole representation (Gauss-Chebyshev)

__device__ inline double nu_of(int n, double beta) { return (2 * n + 1) * M_PI / beta; }

__device__ inline double pole_tau(double e, double tau, double beta) {
  // imaginary-time transform of 1/(i nu - e), 0 < tau < beta
  if (e >= 0.0) return -exp(-e * tau) / (1.0 + exp(-beta * e));
  return -exp(e * (beta - tau)) / (exp(beta * e) + 1.0);
}

__device__ inline void semicircle_pole(int l, double D, double* e, double* c) {
  double th = (l + 1) * M_PI / (kPoles + 1);
  double s = sin(th);
  *e = D * cos(th);
  *c = 2.0 * s * s / (kPoles + 1);
}

__device__ inline double eps_of(int K, const Dims& d, double t, double tp) {
  int kx = K / d.Ly, ky = K - (K / d.Ly) * d.Ly;
  double cx = cos(2.0 * M_PI * kx / d.Lx), cy = cos(2.0 * M_PI * ky / d.Ly);
  return -2.0 * t * (cx + cy) - 4.0 * tp * cx * cy;
}

// exp(+2 pi i (kx rx / Lx + ky ry / Ly)) with the products reduced modulo the lattice
__device__ inline double2 lattice_phase(int K, int R, const Dims& d) {
  int kx = K / d.Ly, ky = K - kx * d.Ly, rx = R / d.Ly, ry = R - rx * d.Ly;
  double ang = 2.0 * M_PI * ((double)((kx * rx) % d.Lx) / d.Lx + (double)((ky * ry) % d.Ly) / d.Ly);
  double s, c;
  sincos(ang, &s, &c);
  return mk(c, s);
}

struct S1Args {
  Dims d;
  double beta, U, t, tp, D;
  int local;
  const double2* g;      // [NG][Nk]
  const double* mu;
  double* tau;           // [ntau]
  double* wt;            // [ntau]
  double2* dg;           // [Nve][Nk]
  double2* gkt;          // [ntau][Nk]
  double2* grt;          // [ntau][Nk] (R)
  double2* trn;          // [Nve][Nk] (R)
  double2* out;          // [Nve][Nk]
};

// Gauss-Legendre nodes/weights on [0, beta], ascending, exactly symmetric.
__global__ void gl_nodes_kernel(S1Args a) {
  const int nt = a.d.ntau;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int half = (nt + 1) / 2;
  if (i >= half) return;
  double x = cos(M_PI * (i + 0.75) / (nt + 0.5));
  double dp = 1.0;
  for (int it = 0; it < 100; ++it) {
    double p0 = 1.0, p1 = x;
    for (int j = 2; j <= nt; ++j) {
      double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
      p0 = p1;
      p1 = p2;
    }
    dp = nt * (x * p1 - p0) / (x * x - 1.0);
    double dx = p1 / dp;
    x -= dx;
    if (fabs(dx) <= 1e-15) {
      // one more evaluation for the derivative at the converged node
      p0 = 1.0; p1 = x;
      for (int j = 2; j <= nt; ++j) {
        double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      dp = nt * (x * p1 - p0) / (x * x - 1.0);
      break;
    }
  }
  double w = 2.0 / ((1.0 - x * x) * dp * dp);
  if ((nt & 1) && i == half - 1) x = 0.0;
  // x is the i-th largest root
  int hi = nt - 1 - i, lo = i;
  a.tau[hi] = 0.5 * a.beta * (x + 1.0);
  a.tau[lo] = 0.5 * a.beta * (1.0 - x);
  a.wt[hi] = 0.5 * a.beta * w;
  a.wt[lo] = 0.5 * a.beta * w;
}

// dG = G - G_pole on the extended box
__global__ void s1_dg_kernel(S1Args a) {
  const Dims& d = a.d;
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d.Nve * d.Nk) return;
  int e = idx / d.Nk, K = idx - e * d.Nk;
  int n = e - d.Nve / 2;
  double nu = nu_of(n, a.beta);
  double2 gv = a.g[(size_t)(n + d.NG / 2) * d.Nk + K];
  double2 gp;
  if (a.local) {
    gp = mk(0.0, 0.0);
    for (int l = 0; l < kPoles; ++l) {
      double el, cl;
      semicircle_pole(l, a.D, &el, &cl);
      gp = cadd(gp, cscale(crecip(mk(-el, nu)), cl));
    }
  } else {
    double xi = eps_of(K, d, a.t, a.tp) - *a.mu;
    gp = crecip(mk(-xi, nu));
  }
  a.dg[idx] = csub(gv, gp);
}

// G(K, tau_j) = pole part + T sum_e dG(e, K) exp(-i nu_e tau_j)
__global__ void s1_gtau_kernel(S1Args a) {
  const Dims& d = a.d;
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d.ntau * d.Nk) return;
  int j = idx / d.Nk, K = idx - j * d.Nk;
  double tau = a.tau[j];
  double pole = 0.0;
  if (a.local) {
    for (int l = 0; l < kPoles; ++l) {
      double el, cl;
      semicircle_pole(l, a.D, &el, &cl);
      pole += cl * pole_tau(el, tau, a.beta);
    }
  } else {
    double xi = eps_of(K, d, a.t, a.tp) - *a.mu;
    pole = pole_tau(xi, tau, a.beta);
  }
  double2 acc = mk(0.0, 0.0);
  for (int e = 0; e < d.Nve; ++e) {
    double nu = nu_of(e - d.Nve / 2, a.beta);
    double s, c;
    sincos(nu * tau, &s, &c);
    acc = cadd(acc, cmul(a.dg[(size_t)e * d.Nk + K], mk(c, -s)));
  }
  a.gkt[idx] = mk(pole + acc.x / a.beta, acc.y / a.beta);
}

// G(R, tau_j) = (1/N) sum_K e^{i K R} G(K, tau_j)
__global__ void s1_gr_kernel(S1Args a) {
  const Dims& d = a.d;
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d.ntau * d.Nk) return;
  int j = idx / d.Nk, R = idx - j * d.Nk;
  double2 acc = mk(0.0, 0.0);
  for (int K = 0; K < d.Nk; ++K) acc = cadd(acc, cmul(lattice_phase(K, R, d), a.gkt[(size_t)j * d.Nk + K]));
  a.grt[idx] = cscale(acc, 1.0 / d.Nk);
}

// T(R, e) = sum_j w_j e^{i nu_e tau_j} U^2 G(R, tau_j)^2 G(-R, beta - tau_j)
__global__ void s1_tr_kernel(S1Args a) {
  const Dims& d = a.d;
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d.Nve * d.Nk) return;
  int e = idx / d.Nk, R = idx - e * d.Nk;
  int rx = R / d.Ly, ry = R - rx * d.Ly;
  int mR = ((d.Lx - rx) % d.Lx) * d.Ly + (d.Ly - ry) % d.Ly;
  double nu = nu_of(e - d.Nve / 2, a.beta);
  double2 acc = mk(0.0, 0.0);
  const int nt = d.ntau;
  for (int j = 0; j < nt; ++j) {
    double2 g1 = a.grt[(size_t)j * d.Nk + R];
    double2 g2 = a.grt[(size_t)(nt - 1 - j) * d.Nk + mR];
    double2 sv = cmul(cmul(g1, g1), g2);
    double s, c;
    sincos(nu * a.tau[j], &s, &c);
    acc = cadd(acc, cscale(cmul(mk(c, s), sv), a.wt[j]));
  }
  a.trn[idx] = cscale(acc, a.U * a.U);
}

// Sigma~_1(K, e) = sum_R e^{-i K R} T(R, e)
__global__ void s1_out_kernel(S1Args a) {
  const Dims& d = a.d;
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d.Nve * d.Nk) return;
  int e = idx / d.Nk, K = idx - e * d.Nk;
  double2 acc = mk(0.0, 0.0);
  for (int R = 0; R < d.Nk; ++R) {
    double2 ph = lattice_phase(K, R, d);
    acc = cadd(acc, cmul(mk(ph.x, -ph.y), a.trn[(size_t)e * d.Nk + R]));
  }
  a.out[idx] = acc;
}

// ------------------------------------------------------------- Sigma~_2
// Re-indexed to native variables (transfer p = (m_p, P), second fermionic
// argument b = (n_b, B)), every term is a product of a G factor of (k, p), the
// indicator weights e16, e25, e34 of the summation domain, which depend on the
// frequencies (n_k, m_p, n_b) only, and momentum-dependent factors of (p, b).
// The momentum sums are therefore done first, once per (p, n_b):
//   U1 = sum_B G(b+p) G(b),  U3 = sum_B G(p-b) G(b),
//   V1d, V1m = sum_B G(b+p) G(b) K2_{d,m}(b;p),  V3st = sum_B G(p-b) G(b) (K2_s + K2_t)(b;p)
// (the V's for b in the box), and the k sum runs over n_b only:
//   s16 = G(k+p) sum e16 U1,  s25 = G(k+p) sum e25 U1,  s34 = G(p-k) sum e34 U3,
//   sk  = G(k+p) sum [e16 V1d - (e16 + 2 e25) V1m] + G(p-k) sum e34 V3st.
struct S2Args {
  Dims d;
  int level;
  const double2* g;
  const double2* k1;     // [4][Nq]
  const double2* k2;     // [4][Nq][n]
  double2* tab;          // [NG][5][Nq]  U1, U3, V1d, V1m, V3st per (n_b, p)
  double2* out;          // [Nve][Nk]  (sum without the constant C)
};

__device__ inline double ind(bool b) { return b ? 1.0 : 0.0; }

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// one wave per (n_b, p): lanes over the momentum B
__global__ __launch_bounds__(kThreads) void s2_tables_kernel(S2Args a) {
  const Dims& d = a.d;
  const int wid = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (wid >= d.NG * d.Nq) return;
  const int nbi = wid / d.Nq, qi = wid - (wid / d.Nq) * d.Nq;
  const int hG = d.NG / 2, nb = nbi - hG;
  const int jm = qi / d.Nk, P = qi - jm * d.Nk, mp = jm - (d.Nv / 2 - 1);
  const bool r1 = nb + mp >= -hG && nb + mp < hG, r3 = mp - nb - 1 >= -hG && mp - nb - 1 < hG;
  const bool kb2 = in_fbox(nb, d.Nv) && a.level >= 2;
  const size_t n = d.n;
  double v[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int B = lane; B < d.Nk; B += 64) {
    const double2 gb = a.g[(size_t)(nb + hG) * d.Nk + B];
    const double2 g1 = r1 ? a.g[(size_t)(nb + mp + hG) * d.Nk + kadd(B, P, d.Lx, d.Ly)] : mk(0, 0);
    const double2 g3 = r3 ? a.g[(size_t)(mp - nb - 1 + hG) * d.Nk + ksub(P, B, d.Lx, d.Ly)] : mk(0, 0);
    const double2 u1 = cmul(g1, gb), u3 = cmul(g3, gb);
    double2 w1d = mk(0, 0), w1m = mk(0, 0), w3 = mk(0, 0);
    if (kb2) {
      const size_t bidx = (size_t)(nb + d.Nv / 2) * d.Nk + B;
      w1d = cmul(u1, a.k2[((size_t)0 * d.Nq + qi) * n + bidx]);
      w1m = cmul(u1, a.k2[((size_t)1 * d.Nq + qi) * n + bidx]);
      w3 = cmul(u3, cadd(a.k2[((size_t)2 * d.Nq + qi) * n + bidx], a.k2[((size_t)3 * d.Nq + qi) * n + bidx]));
    }
    v[0] += u1.x; v[1] += u1.y; v[2] += u3.x; v[3] += u3.y;
    v[4] += w1d.x; v[5] += w1d.y; v[6] += w1m.x; v[7] += w1m.y; v[8] += w3.x; v[9] += w3.y;
  }
  for (int i = 0; i < 10; ++i) v[i] = wave_sum(v[i]);
  if (lane < 5) {
    const double2 o = mk(v[2 * lane], v[2 * lane + 1]);
    a.tab[((size_t)nbi * 5 + lane) * d.Nq + qi] = o;
  }
}

// one workgroup per k point of the extended box; threads over the transfers p
__global__ __launch_bounds__(kThreads) void sigma2_kernel(S2Args a) {
  __shared__ double red[kThreads];
  const Dims& d = a.d;
  const int kid = blockIdx.x;
  const int ek = kid / d.Nk, K = kid - ek * d.Nk;
  const int nk = ek - d.Nve / 2;
  const bool kbox = in_fbox(nk, d.Nv);
  const int kbi = kbox ? (nk + d.Nv / 2) * d.Nk + K : 0;
  const int hF = d.Nve / 2, hBe = d.Nve / 2 - 1, hBb = d.Nv / 2 - 1, hG = d.NG / 2;
  const size_t n = d.n, nq = d.Nq;
  double tr = 0.0, ti = 0.0;
  for (int qi = threadIdx.x; qi < d.Nq; qi += blockDim.x) {
    const int jm = qi / d.Nk, P = qi - jm * d.Nk;
    const int mp = jm - hBb;
    double2 c[4];
    for (int r = 0; r < 4; ++r) {
      c[r] = a.k1[(size_t)r * d.Nq + qi];
      if (kbox && a.level >= 2) c[r] = cadd(c[r], a.k2[((size_t)r * d.Nq + qi) * n + kbi]);
    }
    const int nkp = nk + mp;
    const bool Ye = nkp >= -hF && nkp <= hF - 1;
    const bool Yb = in_fbox(nkp, d.Nv);
    const double2 g_kp = a.g[(size_t)(nkp + hG) * d.Nk + kadd(K, P, d.Lx, d.Ly)];
    const double2 g_pk = a.g[(size_t)(mp - nk - 1 + hG) * d.Nk + ksub(P, K, d.Lx, d.Ly)];
    int lo = min(-hF, min(nk - hBe, -mp - nk - 1 - hBe));
    int hi = max(hF - 1, max(nk + hBe, -mp - nk - 1 + hBe));
    lo = max(lo, -hG);
    hi = min(hi, hG - 1);
    double2 a16 = mk(0, 0), a25 = mk(0, 0), a34 = mk(0, 0), kd = mk(0, 0), km = mk(0, 0), kst = mk(0, 0);
    for (int nb = lo; nb <= hi; ++nb) {
      const bool bFe = nb >= -hF && nb <= hF - 1;
      const bool bFb = in_fbox(nb, d.Nv);
      const int x1 = mp + nk + nb + 1, x2 = nb - nk, x3 = mp - nk - nb - 1;
      double e16 = bFe ? 1.0 + ind(x1 >= -hBe && x1 <= hBe) : 0.0;
      double e25 = Ye ? ind(x2 >= -hBe && x2 <= hBe) + ind(x1 >= -hBe && x1 <= hBe) : 0.0;
      double e34 = bFe ? 1.0 + ind(x3 >= -hBe && x3 <= hBe) : 0.0;
      if (kbox && bFb) {
        e16 -= 1.0 + ind(in_bbox(x1, d.Nv));
        e25 -= Yb ? ind(in_bbox(x2, d.Nv)) + ind(in_bbox(x1, d.Nv)) : 0.0;
        e34 -= 1.0 + ind(in_bbox(x3, d.Nv));
      }
      if (e16 == 0.0 && e25 == 0.0 && e34 == 0.0) continue;
      const double2* t = a.tab + (size_t)(nb + hG) * 5 * nq + qi;
      const double2 u1 = t[0], u3 = t[nq];
      a16 = cadd(a16, cscale(u1, e16));
      a25 = cadd(a25, cscale(u1, e25));
      a34 = cadd(a34, cscale(u3, e34));
      if (bFb && a.level >= 2) {
        kd = cadd(kd, cscale(t[2 * nq], e16));
        km = cadd(km, cscale(t[3 * nq], e16 + 2.0 * e25));
        kst = cadd(kst, cscale(t[4 * nq], e34));
      }
    }
    const double2 s16 = cmul(g_kp, a16), s25 = cmul(g_kp, a25), s34 = cmul(g_pk, a34);
    const double2 sk = cadd(cmul(g_kp, csub(kd, km)), cmul(g_pk, kst));
    double2 contrib = cmul(c[0], s16);
    contrib = csub(contrib, cmul(c[1], cadd(s16, cscale(s25, 2.0))));
    contrib = cadd(contrib, cmul(cadd(c[2], c[3]), s34));
    contrib = cadd(contrib, sk);
    tr += contrib.x;
    ti += contrib.y;
  }
  tr = block_sum(tr, red);
  ti = block_sum(ti, red);
  if (threadIdx.x == 0) a.out[kid] = mk(tr, ti);
}

// ------------------------------------------------------------ Sigma_box
template <typename C>
struct SBArgs {
  Dims d;
  const C* phi;          // [4][Nq][n][n]
  const double2* g;
  double2* partial;      // [n][NW]
};

// 16-byte streaming loads of E consecutive complex values (E = 2 complex64,
// 1 complex128): Phi is read exactly once, so the loads bypass the caches'
// retention (non-temporal), which lets the read stream run closer to the HBM
// read rate.
typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));
template <typename C> struct Row16;
template <> struct Row16<float2> {
  static constexpr int E = 2;
  __device__ static void load(const float2* p, double2 (&o)[2]) {
    const f4v v = __builtin_nontemporal_load((const f4v*)p);
    o[0] = mk(v.x, v.y);
    o[1] = mk(v.z, v.w);
  }
};
template <> struct Row16<double2> {
  static constexpr int E = 1;
  __device__ static void load(const double2* p, double2 (&o)[1]) {
    const d2v v = __builtin_nontemporal_load((const d2v*)p);
    o[0] = mk(v.x, v.y);
  }
};

// One workgroup per (k, m): the box part of Eq. PA_Sigma for row k of the
// four channels at the bosonic index m, summed over Q and k'. Each thread
// takes E consecutive k' per 16-byte load (n is even, rows start 16-byte
// aligned). (Momentum tables in LDS instead of the index arithmetic measured
// slower: the kernel is bound by its loads, not by the integer work.)
template <typename C>
__global__ __launch_bounds__(kThreads) void sigmab_kernel(SBArgs<C> a) {
  __shared__ double red[kThreads];
  using L16 = Row16<C>;
  constexpr int E = L16::E;
  const Dims& d = a.d;
  const int kbi = blockIdx.x / d.NW, jm = blockIdx.x - (blockIdx.x / d.NW) * d.NW;
  const int nk = kbi / d.Nk - d.Nv / 2, K = kbi - (kbi / d.Nk) * d.Nk;
  const int mp = jm - (d.Nv / 2 - 1);
  const int hG = d.NG / 2;
  const int nkp = nk + mp;
  const bool Yb = in_fbox(nkp, d.Nv);
  const size_t n = d.n, nn = (size_t)d.n * d.n, chan = (size_t)d.cs;
  const int ng = d.n / E;                          // load groups per row
  double ar = 0.0, ai = 0.0;
  for (int P = 0; P < d.Nk; ++P) {
    const int qi = jm * d.Nk + P;
    const double2 g_kp = a.g[(size_t)(nkp + hG) * d.Nk + kadd(K, P, d.Lx, d.Ly)];
    const double2 g_pk = a.g[(size_t)(mp - nk - 1 + hG) * d.Nk + ksub(P, K, d.Lx, d.Ly)];
    const C* row = a.phi + (size_t)qi * nn + (size_t)kbi * n;
    for (int gi = threadIdx.x; gi < ng; gi += blockDim.x) {
      double2 pd[E], pm[E], ps[E], pt[E];
      L16::load(row + (size_t)gi * E, pd);
      L16::load(row + chan + (size_t)gi * E, pm);
      L16::load(row + 2 * chan + (size_t)gi * E, ps);
      L16::load(row + 3 * chan + (size_t)gi * E, pt);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int b = gi * E + e;
        const int nb = b / d.Nk - d.Nv / 2, B = b - (b / d.Nk) * d.Nk;
        const int x1 = mp + nk + nb + 1, x2 = nb - nk, x3 = mp - nk - nb - 1;
        const double c16 = 1.0 + ind(in_bbox(x1, d.Nv));
        const double c25 = Yb ? ind(in_bbox(x2, d.Nv)) + ind(in_bbox(x1, d.Nv)) : 0.0;
        const double c34 = 1.0 + ind(in_bbox(x3, d.Nv));
        const double2 gb = a.g[(size_t)(nb + hG) * d.Nk + B];
        const double2 gbp = a.g[(size_t)(nb + mp + hG) * d.Nk + kadd(B, P, d.Lx, d.Ly)];
        const double2 gpb = a.g[(size_t)(mp - nb - 1 + hG) * d.Nk + ksub(P, B, d.Lx, d.Ly)];
        const double2 A1 = cmul(cmul(g_kp, gbp), gb);
        const double2 A3 = cmul(cmul(gpb, g_pk), gb);
        const double2 t1 = csub(cscale(pd[e], c16), cscale(pm[e], c16 + 2.0 * c25));
        const double2 v = cadd(cmul(A1, t1), cmul(A3, cscale(cadd(ps[e], pt[e]), c34)));
        ar += v.x;
        ai += v.y;
      }
    }
  }
  ar = block_sum(ar, red);
  ai = block_sum(ai, red);
  if (threadIdx.x == 0) a.partial[(size_t)kbi * d.NW + jm] = mk(ar, ai);
}

// ------------------------------------------------- local Lambda in the box
// A box Lambda that differs from (U, -U, 2U, 0) adds to Sigma_box the
// Schwinger-Dyson sum of dLambda over the box, with dLambda_dm = Lambda_d -
// Lambda_m - 2U and dLambda_st = Lambda_s + Lambda_t - 2U at (m; n, n'). Since
// Lambda is local, the momentum sums factor through two bubble-like tables
//   B1(n', m; Q) = sum_K' G(n'+m, K'+Q) G(n', K'),
//   B2(n', m; Q) = sum_K' G(m-n'-1, Q-K') G(n', K'),
// and Sigma_box(n, K) gains
//   sum_{n', m} [dLambda_dm sum_Q G(n+m, K+Q) B1 + dLambda_st sum_Q G(m-n-1, Q-K) B2]
// (times the Schwinger-Dyson constant, applied in combine_kernel).
struct LamArgs {
  Dims d;
  double U;
  const double2* g;
  const double2* lam;     // [4][NW][Nv][Nv]
  double2* b1;            // [Nv][NW][Nk]
  double2* b2;
  double2* out;           // [n] (box k)
};

__device__ inline double2 g_at(const LamArgs& a, int nu, int K) {
  return a.g[(size_t)(nu + a.d.NG / 2) * a.d.Nk + K];
}

__global__ __launch_bounds__(kThreads) void lam_tables_kernel(LamArgs a) {
  const Dims& d = a.d;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d.Nv * d.NW * d.Nk) return;
  const int Q = idx % d.Nk, jm = (idx / d.Nk) % d.NW, i2 = idx / (d.Nk * d.NW);
  const int n2 = i2 - d.Nv / 2, m = jm - (d.Nv / 2 - 1);
  double2 s1 = mk(0, 0), s2 = mk(0, 0);
  for (int Kp = 0; Kp < d.Nk; ++Kp) {
    const double2 gk = g_at(a, n2, Kp);
    s1 = cadd(s1, cmul(g_at(a, n2 + m, kadd(Kp, Q, d.Lx, d.Ly)), gk));
    s2 = cadd(s2, cmul(g_at(a, m - n2 - 1, ksub(Q, Kp, d.Lx, d.Ly)), gk));
  }
  a.b1[idx] = s1;
  a.b2[idx] = s2;
}

// one workgroup per box k = (n, K); threads over (n', m)
__global__ __launch_bounds__(kThreads) void lam_sigma_kernel(LamArgs a) {
  __shared__ double red[2][kThreads];
  const Dims& d = a.d;
  const int kbi = blockIdx.x, i1 = kbi / d.Nk, K = kbi - (kbi / d.Nk) * d.Nk;
  const int n = i1 - d.Nv / 2;
  const size_t cs = (size_t)d.NW * d.Nv * d.Nv;
  double sr = 0.0, si = 0.0;
  for (int pr = threadIdx.x; pr < d.Nv * d.NW; pr += blockDim.x) {
    const int i2 = pr / d.NW, jm = pr - (pr / d.NW) * d.NW;
    const int m = jm - (d.Nv / 2 - 1);
    const size_t li = ((size_t)jm * d.Nv + i1) * d.Nv + i2;
    const double2 ldm = csub(csub(a.lam[li], a.lam[cs + li]), mk(2.0 * a.U, 0.0));
    const double2 lst = csub(cadd(a.lam[2 * cs + li], a.lam[3 * cs + li]), mk(2.0 * a.U, 0.0));
    double2 t1 = mk(0, 0), t2 = mk(0, 0);
    const double2* b1 = a.b1 + ((size_t)i2 * d.NW + jm) * d.Nk;
    const double2* b2 = a.b2 + ((size_t)i2 * d.NW + jm) * d.Nk;
    for (int Q = 0; Q < d.Nk; ++Q) {
      t1 = cadd(t1, cmul(g_at(a, n + m, kadd(K, Q, d.Lx, d.Ly)), b1[Q]));
      t2 = cadd(t2, cmul(g_at(a, m - n - 1, ksub(Q, K, d.Lx, d.Ly)), b2[Q]));
    }
    const double2 v = cadd(cmul(ldm, t1), cmul(lst, t2));
    sr += v.x;
    si += v.y;
  }
  red[0][threadIdx.x] = sr;
  red[1][threadIdx.x] = si;
  __syncthreads();
  for (int st = kThreads / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      red[0][threadIdx.x] += red[0][threadIdx.x + st];
      red[1][threadIdx.x] += red[1][threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) a.out[kbi] = mk(red[0][0], red[1][0]);
}

struct CombineArgs {
  Dims d;
  double cfac;
  int has_s2, has_box;
  const double2* s1;
  const double2* s2;
  const double2* partial;
  const double2* lam_part;   // nullable: the box-Lambda term per box k
  double2* out;
};

__global__ void combine_kernel(CombineArgs a) {
  const Dims& d = a.d;
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d.Nve * d.Nk) return;
  int e = idx / d.Nk, K = idx - e * d.Nk;
  int n = e - d.Nve / 2;
  double2 v = a.s1[idx];
  if (a.has_s2) v = cadd(v, cscale(a.s2[idx], a.cfac));
  if (a.has_box && in_fbox(n, d.Nv)) {
    int kbi = (n + d.Nv / 2) * d.Nk + K;
    double2 acc = mk(0, 0);
    for (int j = 0; j < d.NW; ++j) acc = cadd(acc, a.partial[(size_t)kbi * d.NW + j]);
    if (a.lam_part) acc = cadd(acc, a.lam_part[kbi]);
    v = cadd(v, cscale(acc, a.cfac));
  }
  a.out[idx] = v;
}

// ------------------------------------ second order without the regulation
// Eq. PA_Sigma at F = Lambda with both sums truncated to the box (the Sigma~_1
// term of the plain, unregulated equation):
//   -(U^2 T^2 / 2N^2) sum_{q in box} [G(k+q) S_ph(q) + G(q-k) S_pp(q)],
//   S_ph(q) = sum_{k' in box} G(k'+q) G(k'),  S_pp(q) = sum_{k' in box} G(q-k') G(k').
struct S2BoxArgs {
  Dims d;
  double cfac;             // -U^2 T^2 / (2 N^2)
  const double2* g;
  double2* sq;             // [Nq][2]  S_ph, S_pp
  double2* out;            // [Nve][Nk]
};

// one wave per transfer q, lanes over k'
__global__ __launch_bounds__(kThreads) void s2box_tables_kernel(S2BoxArgs a) {
  const Dims& d = a.d;
  const int qi = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (qi >= d.Nq) return;
  const int jm = qi / d.Nk, Q = qi - jm * d.Nk, m = jm - (d.Nv / 2 - 1), hG = d.NG / 2;
  double v[4] = {0, 0, 0, 0};
  for (int kp = lane; kp < d.n; kp += 64) {
    const int n2 = kp / d.Nk - d.Nv / 2, K2 = kp - (kp / d.Nk) * d.Nk;
    const double2 gk = a.g[(size_t)(n2 + hG) * d.Nk + K2];
    const double2 ph = cmul(a.g[(size_t)(n2 + m + hG) * d.Nk + kadd(K2, Q, d.Lx, d.Ly)], gk);
    const double2 pp = cmul(a.g[(size_t)(m - n2 - 1 + hG) * d.Nk + ksub(Q, K2, d.Lx, d.Ly)], gk);
    v[0] += ph.x; v[1] += ph.y; v[2] += pp.x; v[3] += pp.y;
  }
  for (int i = 0; i < 4; ++i) v[i] = wave_sum(v[i]);
  if (lane == 0) {
    a.sq[(size_t)qi * 2] = mk(v[0], v[1]);
    a.sq[(size_t)qi * 2 + 1] = mk(v[2], v[3]);
  }
}

// one workgroup per k (f = 1: the extended box is the box), threads over q
__global__ __launch_bounds__(kThreads) void s2box_kernel(S2BoxArgs a) {
  __shared__ double red[kThreads];
  const Dims& d = a.d;
  const int kid = blockIdx.x, e = kid / d.Nk, K = kid - e * d.Nk;
  const int nk = e - d.Nve / 2, hG = d.NG / 2;
  double tr = 0.0, ti = 0.0;
  for (int qi = threadIdx.x; qi < d.Nq; qi += blockDim.x) {
    const int jm = qi / d.Nk, Q = qi - jm * d.Nk, m = jm - (d.Nv / 2 - 1);
    const double2 gkq = a.g[(size_t)(nk + m + hG) * d.Nk + kadd(K, Q, d.Lx, d.Ly)];
    const double2 gqk = a.g[(size_t)(m - nk - 1 + hG) * d.Nk + ksub(Q, K, d.Lx, d.Ly)];
    const double2 v = cadd(cmul(gkq, a.sq[(size_t)qi * 2]), cmul(gqk, a.sq[(size_t)qi * 2 + 1]));
    tr += v.x;
    ti += v.y;
  }
  tr = block_sum(tr, red);
  ti = block_sum(ti, red);
  if (threadIdx.x == 0) a.out[kid] = mk(a.cfac * tr, a.cfac * ti);
}

struct WsLayout {
  size_t tau, wt, dg, gkt, grt, trn, s1, s2, tab, part, lb1, lb2, lpart, sq, total;
};

WsLayout ws_layout(const Dims& d) {
  WsLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
  L.tau = take(sizeof(double) * d.ntau);
  L.wt = take(sizeof(double) * d.ntau);
  L.dg = take(sizeof(double2) * d.Nve * d.Nk);
  L.gkt = take(sizeof(double2) * (size_t)d.ntau * d.Nk);
  L.grt = take(sizeof(double2) * (size_t)d.ntau * d.Nk);
  L.trn = take(sizeof(double2) * d.Nve * d.Nk);
  L.s1 = take(sizeof(double2) * d.Nve * d.Nk);
  L.s2 = take(sizeof(double2) * d.Nve * d.Nk);
  L.tab = take(sizeof(double2) * 5 * (size_t)d.NG * d.Nq);
  L.part = take(sizeof(double2) * (size_t)d.n * d.NW);
  L.lb1 = take(sizeof(double2) * (size_t)d.Nv * d.NW * d.Nk);
  L.lb2 = take(sizeof(double2) * (size_t)d.Nv * d.NW * d.Nk);
  L.lpart = take(sizeof(double2) * (size_t)d.n);
  L.sq = take(sizeof(double2) * 2 * (size_t)d.Nq);
  L.total = off;
  return L;
}

inline unsigned nblk(size_t total) { return (unsigned)((total + kThreads - 1) / kThreads); }

hipError_t run_sigma1(const pq_params& p, const Dims& d, const double2* g, const double* mu,
                      double2* out, char* ws, hipStream_t s) {
  WsLayout L = ws_layout(d);
  S1Args a{d, p.beta, p.U, p.t, p.tp, p.D, d.Nk == 1 ? 1 : 0, g, mu,
           (double*)(ws + L.tau), (double*)(ws + L.wt), (double2*)(ws + L.dg),
           (double2*)(ws + L.gkt), (double2*)(ws + L.grt), (double2*)(ws + L.trn), out};
  hipLaunchKernelGGL(gl_nodes_kernel, dim3(nblk((d.ntau + 1) / 2)), dim3(kThreads), 0, s, a);
  hipLaunchKernelGGL(s1_dg_kernel, dim3(nblk(d.Nve * d.Nk)), dim3(kThreads), 0, s, a);
  hipLaunchKernelGGL(s1_gtau_kernel, dim3(nblk((size_t)d.ntau * d.Nk)), dim3(kThreads), 0, s, a);
  hipLaunchKernelGGL(s1_gr_kernel, dim3(nblk((size_t)d.ntau * d.Nk)), dim3(kThreads), 0, s, a);
  hipLaunchKernelGGL(s1_tr_kernel, dim3(nblk(d.Nve * d.Nk)), dim3(kThreads), 0, s, a);
  hipLaunchKernelGGL(s1_out_kernel, dim3(nblk(d.Nve * d.Nk)), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace

size_t sigma_ws_bytes(const Dims& d) { return ws_layout(d).total; }

// ------------------------------------------------------ static scratch
// Workspace of sigma_sde_no_alloc: a file-scope device array, one copy per
// device that loads the library, held until the process ends. Host code never
// uses the array's name as an address (on the host it is a stand-in symbol):
// the device address is looked up once per device with hipGetSymbolAddress,
// with that device current, and kept.
namespace {
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// The second-order term: over all frequencies (Sigma~_1 of the regulation) or,
// without the regulation, truncated to the box.
static hipError_t run_second_order(const pq_params& p, const Dims& d, const double2* g, const double* mu,
                                   double2* out, char* ws, hipStream_t s) {
  if (p.regulation != 0) return run_sigma1(p, d, g, mu, out, ws, s);
  const WsLayout L = ws_layout(d);
  const double T = 1.0 / p.beta;
  S2BoxArgs a{d, -p.U * p.U * T * T / (2.0 * d.Nk * (double)d.Nk), g, (double2*)(ws + L.sq), out};
  const unsigned wpb = kThreads / 64;
  hipLaunchKernelGGL(s2box_tables_kernel, dim3((d.Nq + wpb - 1) / wpb), dim3(kThreads), 0, s, a);
  hipLaunchKernelGGL(s2box_kernel, dim3(d.Nve * d.Nk), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_sigma1(const pq_params& p, const Dims& d, const double2* g, const double* mu,
                         double2* sigma_out, void* ws, hipStream_t s) {
  return run_second_order(p, d, g, mu, sigma_out, (char*)ws, s);
}

hipError_t launch_sigma(const pq_params& p, const Dims& d, const void* phi, const double2* k1,
                        const double2* k2, const double2* lam_box, const double2* g, const double* mu,
                        double2* sigma_out, void* wsv, hipStream_t s) {
  char* ws = (char*)wsv;
  WsLayout L = ws_layout(d);
  double2* s1 = (double2*)(ws + L.s1);
  double2* s2 = (double2*)(ws + L.s2);
  double2* part = (double2*)(ws + L.part);
  hipError_t e = run_second_order(p, d, g, mu, s1, ws, s);
  if (e != hipSuccess) return e;
  const int has_s2 = p.kernel_level > 0 ? 1 : 0;
  if (has_s2) {
    S2Args a2{d, p.kernel_level, g, k1, k2, (double2*)(ws + L.tab), s2};
    const unsigned nwav = (unsigned)d.NG * d.Nq, wpb = kThreads / 64;
    hipLaunchKernelGGL(s2_tables_kernel, dim3((nwav + wpb - 1) / wpb), dim3(kThreads), 0, s, a2);
    hipLaunchKernelGGL(sigma2_kernel, dim3(d.Nve * d.Nk), dim3(kThreads), 0, s, a2);
  }
  if (p.storage == PQ_STORE_C64) {
    SBArgs<float2> ab{d, (const float2*)phi, g, part};
    hipLaunchKernelGGL(sigmab_kernel<float2>, dim3(d.n * d.NW), dim3(kThreads), 0, s, ab);
  } else {
    SBArgs<double2> ab{d, (const double2*)phi, g, part};
    hipLaunchKernelGGL(sigmab_kernel<double2>, dim3(d.n * d.NW), dim3(kThreads), 0, s, ab);
  }
  double2* lpart = nullptr;
  if (lam_box) {
    lpart = (double2*)(ws + L.lpart);
    LamArgs al{d, p.U, g, lam_box, (double2*)(ws + L.lb1), (double2*)(ws + L.lb2), lpart};
    hipLaunchKernelGGL(lam_tables_kernel, dim3(nblk((size_t)d.Nv * d.NW * d.Nk)), dim3(kThreads), 0, s, al);
    hipLaunchKernelGGL(lam_sigma_kernel, dim3(d.n), dim3(kThreads), 0, s, al);
  }
  const double T = 1.0 / p.beta;
  CombineArgs ac{d, -p.U * T * T / (4.0 * d.Nk * (double)d.Nk), has_s2, 1, s1, s2, part, lpart, sigma_out};
  hipLaunchKernelGGL(combine_kernel, dim3(nblk(d.Nve * d.Nk)), dim3(kThreads), 0, s, ac);
  return hipGetLastError();
}

}  // namespace pq
