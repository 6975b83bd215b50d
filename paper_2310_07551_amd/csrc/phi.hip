// phi-functions of small dense matrices on the GPU, computed in double-double
// arithmetic and rounded once to FP64.
//
// Section 2.4 computes the phi matrices once, before time stepping, "with a
// rational Pade approach and modified scaling and squaring" (Skaflestad and
// Wright, 2009).  This file does all of it on the device:
//
//  1. X = c A (the FP64 product of the scalar and each entry);
//     s = max(0, ceil(log2 ||X||_1 / theta)),  Y = X / 2^s  (theta = 1, exact).
//  2. The diagonal [m/m] Pade approximant of phi_p at Y, m = 8:
//       D(z) = sum_j d_j z^j,  d_j = (-1)^j C(m, j) / ((2m+p)(2m+p-1)...(2m+p-j+1)),
//       N(z) = sum_i n_i z^i,  n_i = sum_{j<=i} d_j / (p+i-j)!,
//     so that D phi_p - N = O(z^{2m+1}).
//  3. Lower orders by the recurrence phi_k(Y) = Y phi_{k+1}(Y) + I/k!.
//  4. s modified squarings
//       phi_0(2Y) = phi_0(Y)^2,
//       phi_k(2Y) = 2^{-k} [ phi_0(Y) phi_k(Y) + sum_{j=1}^{k} phi_j(Y)/(k-j)! ].
//
// Accuracy.  A squaring maps an error E in phi_0(Y) to about phi_0 E + E
// phi_0; on an eigenvector whose eigenvalue is near zero (the constant vector
// of a Neumann Laplacian, where phi_0 = 1) that doubles it.  s squarings thus
// turn a rounding error of u into 2^s u ~ u ||X||: 2e-11 for the stiffest
// matrix of a 256-point direction of the 3D FitzHugh-Nagumo workload (||X||
// ~ 2e5), enough to move a time step's result by ~1e-12.  Here every matrix
// is a pair of FP64 planes (hi, lo) and every product and sum is done in
// double-double arithmetic (error ~ u^2 per operation), so 2^s u^2 stays far
// below an FP64 ulp, and the result is rounded once.
//
// Deviations.  All stages carry psi_k = phi_k - I/k! instead of phi_k:
//   psi_p(Y)  = D(Y)^{-1} Npsi(Y),  Npsi(z) = N(z) - D(z)/p! = sum_{i>=1} e_i z^i,
//               e_i = sum_{j<i} d_j / (p+i-j)!   (n_0 = d_0/p!, so no constant term);
//   psi_k     = Y psi_{k+1} + Y/(k+1)!;
//   psi_0(2Y) = psi_0^2 + 2 psi_0;
//   psi_k(2Y) = 2^{-k} [ psi_0 psi_k + psi_0/k! + 2 psi_k + sum_{j=1}^{k-1} psi_j/(k-j)! ]   (k >= 1),
// which follow from the formulas above with phi_j = I/j! + psi_j (the identity
// parts sum to I/k!).  On an eigenvector with eigenvalue 0 every psi is
// exactly 0, and a small relative error of the Pade coefficients (they are
// formed in double-double on the host) stays a small relative error of psi
// through the squarings instead of being doubled s times.
//
// D(Y)^{-1} comes from the Newton-Schulz iteration X <- X (2I - D X), whose
// residual I - D X squares at every step.  Because ||Y||_1 <= 1,
// ||I - D(Y)||_1 <= sum_{j>=1} |d_j| = rho (0.64 for p = 0, smaller for
// larger p), so X_0 = I reaches the double-double rounding level after a
// fixed, small number of steps, each two batched GEMMs on all compute units.
//
// A batch shares A and n; every entry has its own scalar c_j and the batch
// uses the largest scaling exponent of its entries (extra squarings of a
// smaller argument only shrink the Pade error).  The matrix products are a
// plain LDS-tiled double-double GEMM: this runs once per step size and is not
// on the time-stepping path.
#include <cmath>
#include <vector>

#include "common.hpp"
#include "pointwise.hpp"

// Double-double arithmetic relies on every sum and product being rounded on
// its own; explicit fma() calls are the only fused operations in this file.
#pragma clang fp contract(off)

namespace setd {
namespace {

constexpr int kPadeM = 8;
constexpr double kTheta = 1.0;
constexpr int kMaxOrder = 6;

// ---- double-double helpers (device and host) ----
struct DD {
  double hi, lo;
};

__host__ __device__ inline DD dd_two_sum(double a, double b) {
  const double s = a + b;
  const double v = s - a;
  return {s, (a - (s - v)) + (b - v)};
}

__host__ __device__ inline DD dd_add(DD a, DD b) {
  const DD s = dd_two_sum(a.hi, b.hi);
  const double e = s.lo + (a.lo + b.lo);
  return dd_two_sum(s.hi, e);
}

__device__ inline DD dd_mul(DD a, DD b) {
  const double p = a.hi * b.hi;
  double e = fma(a.hi, b.hi, -p);
  e = fma(a.hi, b.lo, e);
  e = fma(a.lo, b.hi, e);
  return dd_two_sum(p, e);
}

// a / b for a double-double a and an FP64 b (host).
inline DD hdd_div(DD a, double b) {
  const double q1 = a.hi / b;
  const double r = std::fma(-q1, b, a.hi) + a.lo;   // fma(-q1, b, a.hi) is exact
  return dd_two_sum(q1, r / b);
}

// ---- matrices: block of 2 n^2 doubles, hi plane then lo plane ----
struct GemmDesc {
  const double* A;
  const double* B;
  double* C;
};

// C = alpha A B + diag I + acoef A for n x n column-major double-double
// matrices (alpha = +-1), one descriptor per blockIdx.z; C must not overlap A
// or B.  64 x 64 tile per 256-thread block, 4 x 4 entries per thread; the
// products' rounding errors are carried exactly (fma) and the running sum is
// kept as a two-sum pair per entry.
__global__ void __launch_bounds__(256) gemm_dd_kernel(const GemmDesc* __restrict__ descs, int n, double alpha,
                                                          DD diag, DD acoef) {
  const GemmDesc dsc = descs[blockIdx.z];
  const int64_t nn = (int64_t)n * n;
  __shared__ double Ah[16][65], Al[16][65], Bh[16][65], Bl[16][65];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
  double ch[4][4], cl[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) ch[i][j] = cl[i][j] = 0.0;
  for (int k0 = 0; k0 < n; k0 += 16) {
    for (int e = threadIdx.x; e < 1024; e += 256) {
      const int r = e & 63, kk = e >> 6;
      const bool ina = m0 + r < n && k0 + kk < n;
      const int64_t ia = (m0 + r) + (int64_t)n * (k0 + kk);
      Ah[kk][r] = ina ? dsc.A[ia] : 0.0;
      Al[kk][r] = ina ? dsc.A[nn + ia] : 0.0;
      const int kb = e & 15, c = e >> 4;
      const bool inb = k0 + kb < n && n0 + c < n;
      const int64_t ib = (k0 + kb) + (int64_t)n * (n0 + c);
      Bh[kb][c] = inb ? dsc.B[ib] : 0.0;
      Bl[kb][c] = inb ? dsc.B[nn + ib] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < 16; ++kk) {
      double ah[4], al[4], bh[4], bl[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        ah[i] = Ah[kk][tx + 16 * i];
        al[i] = Al[kk][tx + 16 * i];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        bh[j] = Bh[kk][ty + 16 * j];
        bl[j] = Bl[kk][ty + 16 * j];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const double p = ah[i] * bh[j];
          double e = fma(ah[i], bh[j], -p);
          e = fma(ah[i], bl[j], e);
          e = fma(al[i], bh[j], e);
          const double s = ch[i][j] + p;
          const double v = s - ch[i][j];
          const double t = (ch[i][j] - (s - v)) + (p - v);
          ch[i][j] = s;
          cl[i][j] = cl[i][j] + (t + e);
        }
    }
    __syncthreads();
  }
  const bool use_a = acoef.hi != 0.0 || acoef.lo != 0.0;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      const int r = m0 + tx + 16 * i, c = n0 + ty + 16 * j;
      if (r >= n || c >= n) continue;
      const int64_t idx = r + (int64_t)n * c;
      DD v = dd_two_sum(ch[i][j], cl[i][j]);
      v.hi *= alpha;
      v.lo *= alpha;
      if (r == c) v = dd_add(v, diag);
      if (use_a) v = dd_add(v, dd_mul(acoef, DD{dsc.A[idx], dsc.A[nn + idx]}));
      dsc.C[idx] = v.hi;
      dsc.C[nn + idx] = v.lo;
    }
}

// ||A||_1 (max column sum); NaN if any entry is not finite.
__global__ void norm1_kernel(const double* __restrict__ A, int n, double* __restrict__ out) {
  __shared__ double red[256];
  double best = 0.0;
  bool bad = false;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
      const double v = A[i + (int64_t)n * j];
      bad = bad || !isfinite(v);
      s += fabs(v);
    }
    best = fmax(best, s);
  }
  red[threadIdx.x] = bad ? __builtin_nan("") : best;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
    bool nan = false;
    for (int t = 0; t < (int)blockDim.x; ++t) {
      nan = nan || (red[t] != red[t]);
      m = fmax(m, red[t]);
    }
    *out = nan ? __builtin_nan("") : m;
  }
}

// Y_j = (c_j A) 2^-s for every entry: hi = the FP64 product (scal_j = c_j 2^-s,
// an exact power-of-two scaling of c_j), lo = 0.
__global__ void scale_batch_kernel(const double* __restrict__ A, int64_t nn, const double* __restrict__ scal,
                                   double* __restrict__ W, int64_t stride) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nn) return;
  double* y = W + stride * blockIdx.y;
  y[idx] = scal[blockIdx.y] * A[idx];
  y[nn + idx] = 0.0;
}

struct Coefs {
  DD e[kPadeM + 1];   // Npsi coefficients, e[0] = 0
  DD d[kPadeM + 1];   // denominator, d[0] = 1
};

struct InvFact {
  DD f[kMaxOrder + 2];   // 1/k!
};

// Npsi = sum_{i>=1} e_i Y^i, D = sum d_i Y^i (Y^0 = I); block k-1 holds Y^k.
// Also writes the first Newton-Schulz iterate X_1 = 2I - D over Y^2 (block 1),
// which is not read again.
__global__ void pade_combo_kernel(double* __restrict__ W, int n, int64_t stride, Coefs cf) {
  const int64_t nn = (int64_t)n * n;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nn) return;
  double* w = W + stride * blockIdx.y;
  const bool diag = (idx % n) == (idx / n);
  DD sn{0.0, 0.0};
  DD sd = diag ? cf.d[0] : DD{0.0, 0.0};
  for (int k = 1; k <= kPadeM; ++k) {
    const double* y = w + (int64_t)(k - 1) * 2 * nn;
    const DD yk{y[idx], y[nn + idx]};
    sn = dd_add(sn, dd_mul(cf.e[k], yk));
    sd = dd_add(sd, dd_mul(cf.d[k], yk));
  }
  double* N = w + (int64_t)kPadeM * 2 * nn;
  double* D = w + (int64_t)(kPadeM + 1) * 2 * nn;
  double* X1 = w + 2 * nn;
  N[idx] = sn.hi;
  N[nn + idx] = sn.lo;
  D[idx] = sd.hi;
  D[nn + idx] = sd.lo;
  const DD x1 = dd_add(DD{diag ? 2.0 : 0.0, 0.0}, DD{-sd.hi, -sd.lo});
  X1[idx] = x1.hi;
  X1[nn + idx] = x1.lo;
}

// Modified squaring in deviation form for one entry and all orders at once
// (T_k = psi_0 psi_k already formed; T and the new values share storage):
//   new_0 = T_0 + 2 old_0,
//   new_k = 2^{-k} (T_k + old_0/k! + 2 old_k + sum_{j=1}^{k-1} old_j/(k-j)!).
__global__ void square_combo_kernel(double* __restrict__ W, int n, int64_t stride, int64_t off_old, int64_t off_T,
                                    int p, InvFact f) {
  const int64_t nn = (int64_t)n * n;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nn) return;
  double* w = W + stride * blockIdx.y;
  const double* old = w + off_old;
  double* T = w + off_T;
  auto ld = [&](const double* b, int k) { return DD{b[(int64_t)k * 2 * nn + idx], b[(int64_t)k * 2 * nn + nn + idx]}; };
  const DD o0 = ld(old, 0);
  for (int k = 0; k <= p; ++k) {
    const DD ok = ld(old, k);
    DD s = dd_add(ld(T, k), DD{2.0 * ok.hi, 2.0 * ok.lo});
    if (k >= 1) {
      s = dd_add(s, dd_mul(f.f[k], o0));
      for (int j = 1; j < k; ++j) s = dd_add(s, dd_mul(f.f[k - j], ld(old, j)));
    }
    T[(int64_t)k * 2 * nn + idx] = ldexp(s.hi, -k);
    T[(int64_t)k * 2 * nn + nn + idx] = ldexp(s.lo, -k);
  }
}

// out = I/k! + psi_k rounded to FP64, for output block blockIdx.y = j (p+1) + k.
__global__ void finalize_kernel(const double* __restrict__ W, int n, int64_t stride, int64_t off_res, int p,
                                InvFact f, double* const* __restrict__ outs) {
  const int64_t nn = (int64_t)n * n;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nn) return;
  const int j = blockIdx.y / (p + 1), k = blockIdx.y % (p + 1);
  const double* b = W + stride * j + off_res + (int64_t)k * 2 * nn;
  DD v{b[idx], b[nn + idx]};
  if ((idx % n) == (idx / n)) v = dd_add(v, f.f[k]);
  outs[blockIdx.y][idx] = v.hi + v.lo;
}

struct Buf {
  double* p = nullptr;
  ~Buf() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace

int phi_batch(const double* A, int n, const double* c, int nentries, int p, double* const* out, hipStream_t s) {
  if (nentries <= 0) return SETD_OK;
  if (p < 0 || p > kMaxOrder) {
    set_error("phi order %d outside 0..%d", p, kMaxOrder);
    return SETD_EINVAL;
  }
  const int64_t nn = (int64_t)n * n;
  const int64_t blk_doubles = 2 * nn;   // hi and lo planes
  // entries are processed in chunks that keep the workspace below ~1 GiB
  const int per_entry_blocks = kPadeM + 2 + 2 * (p + 1);
  const int64_t stride = per_entry_blocks * blk_doubles;
  int chunk = (int)std::max<int64_t>(1, (int64_t)(1ll << 27) / stride);
  chunk = std::min(chunk, nentries);

  Buf norm;
  SETD_HIP(hipMalloc(&norm.p, sizeof(double)));
  hipLaunchKernelGGL(norm1_kernel, dim3(1), dim3(256), 0, s, A, n, norm.p);
  SETD_LAUNCHED();
  double anorm = 0.0;
  SETD_HIP(hipMemcpyAsync(&anorm, norm.p, sizeof(double), hipMemcpyDeviceToHost, s));
  SETD_HIP(hipStreamSynchronize(s));
  if (!std::isfinite(anorm)) {
    set_error("phi: matrix has non-finite entries");
    return SETD_ENONFINITE;
  }
  for (int j = 0; j < nentries; ++j)
    if (!std::isfinite(c[j])) {
      set_error("phi: non-finite scalar argument");
      return SETD_ENONFINITE;
    }

  // Pade coefficients in double-double, from exact integers:
  // d_j = (-1)^j C(m, j) / P_j with P_j = (2m+p)(2m+p-1)...(2m+p-j+1) < 2^53.
  Coefs cf;
  InvFact invf;
  int ns_iters = 0;
  {
    const int m = kPadeM;
    double fact[kMaxOrder + kPadeM + 1];   // 0! .. 14!, exact in FP64
    fact[0] = 1.0;
    for (int k = 1; k <= kMaxOrder + kPadeM; ++k) fact[k] = fact[k - 1] * k;
    for (int k = 0; k <= kMaxOrder + 1; ++k) invf.f[k] = hdd_div(DD{1.0, 0.0}, fact[k]);
    double binom = 1.0, P = 1.0;
    double rho = 0.0;
    for (int j = 0; j <= m; ++j) {
      if (j > 0) {
        binom = binom * (m - j + 1) / j;   // exact: C(m, j) is an integer
        P *= (double)(2 * m + p - j + 1);
      }
      cf.d[j] = hdd_div(DD{(j & 1) ? -binom : binom, 0.0}, P);
      if (j > 0) rho += std::fabs(cf.d[j].hi);
    }
    for (int i = 0; i <= m; ++i) {
      DD acc{0.0, 0.0};
      for (int j = 0; j < i; ++j) acc = dd_add(acc, hdd_div(cf.d[j], fact[p + i - j]));
      cf.e[i] = acc;
    }
    // residual bound after X_1 and `ns_iters` further steps: rho^(2^(ns_iters+1))
    double r = rho * rho;
    while (r > 1e-34 && ns_iters < 12) {
      r *= r;
      ++ns_iters;
    }
    if (!(rho < 0.9) || r > 1e-34) {
      set_error("phi: Pade denominator bound %g too large for the inverse iteration", rho);
      return SETD_EINVAL;
    }
  }

  Buf ws, dev;
  SETD_HIP(hipMalloc(&ws.p, (size_t)chunk * stride * sizeof(double)));
  // per chunk: scalars (chunk), gemm descriptors, output pointers.
  // descriptors: (m-1) power products, two parities of the two Newton-Schulz
  // products, the final D^{-1} Npsi, p recurrence products and two parities
  // of (p+1) squaring products, per entry
  const int ndesc_max = chunk * ((kPadeM - 1) + 5 + p + 2 * (p + 1));
  const size_t scal_bytes = ((chunk * sizeof(double) + 63) / 64) * 64;
  const size_t desc_bytes = (size_t)ndesc_max * sizeof(GemmDesc);
  const size_t outp_bytes = (size_t)chunk * (p + 1) * sizeof(double*);
  const size_t dev_bytes = scal_bytes + desc_bytes + outp_bytes;
  SETD_HIP(hipMalloc(&dev.p, dev_bytes));

  for (int e0 = 0; e0 < nentries; e0 += chunk) {
    const int E = std::min(chunk, nentries - e0);
    double cmax = 0.0;
    for (int j = 0; j < E; ++j) cmax = std::max(cmax, std::fabs(c[e0 + j]));
    const double xnorm = cmax * anorm;
    int sq = 0;
    if (xnorm > kTheta) sq = (int)std::ceil(std::log2(xnorm / kTheta));
    if (sq > 1000) {
      set_error("phi: argument norm too large");
      return SETD_EUNSUPPORTED;
    }

    // Host-built tables: scalars, descriptor sets, output pointers.
    std::vector<char> host(dev_bytes, 0);
    double* hs = (double*)host.data();
    for (int j = 0; j < E; ++j) hs[j] = std::ldexp(c[e0 + j], -sq);
    GemmDesc* hd = (GemmDesc*)(host.data() + scal_bytes);
    GemmDesc* dd = (GemmDesc*)((char*)dev.p + scal_bytes);
    double** hout = (double**)(host.data() + scal_bytes + desc_bytes);
    for (int j = 0; j < E; ++j)
      for (int k = 0; k <= p; ++k) hout[j * (p + 1) + k] = out[(int64_t)(e0 + j) * (p + 1) + k];
    // layout of entry j: Ypow[0..m-1] | Npsi | D | bufA[0..p] | bufB[0..p]
    auto blk = [&](int j, int b) { return ws.p + stride * j + (int64_t)b * blk_doubles; };
    const int offA = kPadeM + 2, offB = offA + (p + 1);
    // power chain Y^k = Y^{k-1} Y: one set of E descriptors per k
    int nd = 0;
    GemmDesc* pow_d = hd + nd;
    for (int k = 2; k <= kPadeM; ++k)
      for (int j = 0; j < E; ++j) hd[nd++] = {blk(j, k - 2), blk(j, 0), blk(j, k - 1)};
    // Newton-Schulz on the free power blocks: X in block 1 or 3 by parity,
    // S = 2I - D X in block 2; then bufA[p] = X Npsi
    const int kD = kPadeM + 1, kN = kPadeM;
    GemmDesc* ns_d[2][2];
    for (int par = 0; par < 2; ++par) {
      const int xi = par == 0 ? 1 : 3, xo = par == 0 ? 3 : 1;
      ns_d[par][0] = hd + nd;
      for (int j = 0; j < E; ++j) hd[nd++] = {blk(j, kD), blk(j, xi), blk(j, 2)};
      ns_d[par][1] = hd + nd;
      for (int j = 0; j < E; ++j) hd[nd++] = {blk(j, xi), blk(j, 2), blk(j, xo)};
    }
    GemmDesc* fin_d = hd + nd;
    for (int j = 0; j < E; ++j) hd[nd++] = {blk(j, ns_iters % 2 == 0 ? 1 : 3), blk(j, kN), blk(j, offA + p)};
    // recurrence: bufA[k] = Y bufA[k+1] + Y/(k+1)!
    GemmDesc* rec_d = hd + nd;
    for (int k = p - 1; k >= 0; --k)
      for (int j = 0; j < E; ++j) hd[nd++] = {blk(j, 0), blk(j, offA + k + 1), blk(j, offA + k)};
    // squaring, two parities: T_k = old_0 old_k
    GemmDesc* sq_d[2];
    for (int par = 0; par < 2; ++par) {
      sq_d[par] = hd + nd;
      const int o = par == 0 ? offA : offB, t = par == 0 ? offB : offA;
      for (int j = 0; j < E; ++j)
        for (int k = 0; k <= p; ++k) hd[nd++] = {blk(j, o), blk(j, o + k), blk(j, t + k)};
    }
    if ((size_t)((char*)(hd + nd) - host.data()) > scal_bytes + desc_bytes) {
      set_error("phi: internal descriptor overflow");
      return SETD_EINVAL;
    }
    SETD_HIP(hipMemcpyAsync(dev.p, host.data(), dev_bytes, hipMemcpyHostToDevice, s));
    auto dptr = [&](GemmDesc* hp) { return dd + (hp - hd); };
    const DD zero{0.0, 0.0};

    const dim3 gtile((unsigned)ceil_div(n, 64), (unsigned)ceil_div(n, 64));
    const dim3 ew((unsigned)ceil_div(nn, 256), (unsigned)E);
    // 1. Y = (c/2^s) A
    hipLaunchKernelGGL(scale_batch_kernel, ew, dim3(256), 0, s, A, nn, (const double*)dev.p, ws.p, stride);
    SETD_LAUNCHED();
    // 2. powers
    for (int k = 2; k <= kPadeM; ++k) {
      hipLaunchKernelGGL(gemm_dd_kernel, dim3(gtile.x, gtile.y, E), dim3(256), 0, s, dptr(pow_d + (k - 2) * E), n,
                         1.0, zero, zero);
      SETD_LAUNCHED();
    }
    // 3. Npsi, D, X_1 = 2I - D; Newton-Schulz steps; psi_p(Y) ~ X Npsi
    hipLaunchKernelGGL(pade_combo_kernel, ew, dim3(256), 0, s, ws.p, n, stride, cf);
    SETD_LAUNCHED();
    for (int it = 0; it < ns_iters; ++it) {
      hipLaunchKernelGGL(gemm_dd_kernel, dim3(gtile.x, gtile.y, E), dim3(256), 0, s, dptr(ns_d[it & 1][0]), n, -1.0,
                         DD{2.0, 0.0}, zero);
      SETD_LAUNCHED();
      hipLaunchKernelGGL(gemm_dd_kernel, dim3(gtile.x, gtile.y, E), dim3(256), 0, s, dptr(ns_d[it & 1][1]), n, 1.0,
                         zero, zero);
      SETD_LAUNCHED();
    }
    hipLaunchKernelGGL(gemm_dd_kernel, dim3(gtile.x, gtile.y, E), dim3(256), 0, s, dptr(fin_d), n, 1.0, zero, zero);
    SETD_LAUNCHED();
    // 4. psi_k = Y psi_{k+1} + Y/(k+1)!
    for (int q = 0; q < p; ++q) {
      const int k = p - 1 - q;
      hipLaunchKernelGGL(gemm_dd_kernel, dim3(gtile.x, gtile.y, E), dim3(256), 0, s, dptr(rec_d + q * E), n, 1.0,
                         zero, invf.f[k + 1]);
      SETD_LAUNCHED();
    }
    // 5. s modified squarings
    int cur = 0;   // 0: current values in bufA, 1: in bufB
    for (int it = 0; it < sq; ++it) {
      hipLaunchKernelGGL(gemm_dd_kernel, dim3(gtile.x, gtile.y, E * (p + 1)), dim3(256), 0, s, dptr(sq_d[cur]), n,
                         1.0, zero, zero);
      SETD_LAUNCHED();
      const int64_t off_old = (int64_t)(cur == 0 ? offA : offB) * blk_doubles;
      const int64_t off_T = (int64_t)(cur == 0 ? offB : offA) * blk_doubles;
      hipLaunchKernelGGL(square_combo_kernel, ew, dim3(256), 0, s, ws.p, n, stride, off_old, off_T, p, invf);
      SETD_LAUNCHED();
      cur ^= 1;
    }
    // 6. phi_k = I/k! + psi_k, rounded to FP64, into the caller's blocks
    const int64_t off_res = (int64_t)(cur == 0 ? offA : offB) * blk_doubles;
    hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)ceil_div(nn, 256), (unsigned)(E * (p + 1))), dim3(256), 0, s,
                       (const double*)ws.p, n, stride, off_res, p, invf,
                       (double* const*)((char*)dev.p + scal_bytes + desc_bytes));
    SETD_LAUNCHED();
    SETD_HIP(hipStreamSynchronize(s));   // host tables and workspace are reused by the next chunk
  }
  return SETD_OK;
}

}  // namespace setd
