// phi-functions of small dense matrices, FP64, on the GPU.
//
// Section 2.4 computes the phi matrices once, before time stepping, "with a
// rational Pade approach and modified scaling and squaring" (Skaflestad and
// Wright, 2009).  This file does all of it on the device:
//
//  1. X = c A;  s = max(0, ceil(log2 ||X||_1 / theta)),  Y = X / 2^s  (theta = 1).
//  2. The diagonal [m/m] Pade approximant of phi_p at Y, m = 8:
//       D(z) = sum_j d_j z^j,  d_j = (-1)^j m! (2m+p-j)! / ((2m+p)! j! (m-j)!),
//       N(z) = sum_i n_i z^i,  n_i = sum_{j<=i} d_j / (p+i-j)!,
//     so that D phi_p - N = O(z^{2m+1}); phi_p(Y) ~ D(Y)^{-1} N(Y).
//     D(Y)^{-1} comes from the Newton-Schulz iteration X <- X (2I - D X),
//     whose residual I - D X squares at every step.  Because ||Y||_1 <= 1,
//     ||I - D(Y)||_1 <= sum_{j>=1} |d_j| = rho (0.64 for p = 0, smaller for
//     larger p), so X_0 = I reaches rounding level after a fixed, small
//     number of steps, each two batched GEMMs on all compute units (a
//     pivoted LU keeps one block per matrix busy for n sequential steps).
//  3. Lower orders by the recurrence phi_k(Y) = Y phi_{k+1}(Y) + I/k!.
//  4. s modified squarings
//       phi_0(2Y) = phi_0(Y)^2,
//       phi_k(2Y) = 2^{-k} [ phi_0(Y) phi_k(Y) + sum_{j=1}^{k} phi_j(Y)/(k-j)! ].
//
// A batch shares A and n; every entry has its own scalar c_j and the batch
// uses the largest scaling exponent of its entries (extra squarings of a
// smaller argument only shrink the Pade error).  The matrix products are a
// plain LDS-tiled FP64 GEMM: this runs once per step size and is not on the
// time-stepping path.
#include <cmath>
#include <vector>

#include "common.hpp"
#include "pointwise.hpp"

namespace setd {
namespace {

constexpr int kPadeM = 8;
constexpr double kTheta = 1.0;

struct GemmDesc {
  const double* A;
  const double* B;
  double* C;
};

// C = alpha A B + diag_add * I for n x n column-major matrices, one
// descriptor per blockIdx.z; C must not overlap A or B.  64 x 64 tile per 256-thread block, 4 x 4 per thread.
__global__ void __launch_bounds__(256) gemm_nn_kernel(const GemmDesc* __restrict__ descs, int n, double alpha,
                                                          double diag_add) {
  const GemmDesc dsc = descs[blockIdx.z];
  __shared__ double As[16][65];
  __shared__ double Bs[16][65];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
  double acc[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int k0 = 0; k0 < n; k0 += 16) {
    for (int e = threadIdx.x; e < 1024; e += 256) {
      const int r = e & 63, kk = e >> 6;
      As[kk][r] = (m0 + r < n && k0 + kk < n) ? dsc.A[(m0 + r) + (int64_t)n * (k0 + kk)] : 0.0;
      const int kb = e & 15, c = e >> 4;
      Bs[kb][c] = (k0 + kb < n && n0 + c < n) ? dsc.B[(k0 + kb) + (int64_t)n * (n0 + c)] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][tx + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][ty + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      const int r = m0 + tx + 16 * i, c = n0 + ty + 16 * j;
      if (r < n && c < n) dsc.C[r + (int64_t)n * c] = alpha * acc[i][j] + (r == c ? diag_add : 0.0);
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

// Y_j = scal_j * A for every entry (stride `stride` doubles between entries).
__global__ void scale_batch_kernel(const double* __restrict__ A, int64_t nn, const double* __restrict__ scal,
                                   double* __restrict__ Y0, int64_t stride) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nn) return;
  Y0[stride * blockIdx.y + idx] = scal[blockIdx.y] * A[idx];
}

struct Coefs {
  double n[kPadeM + 1];
  double d[kPadeM + 1];
};

// N = sum n_i Y^i, D = sum d_i Y^i (Y^0 = I); Ypow[k-1] holds Y^k.  Also
// writes the first Newton-Schulz iterate X_1 = 2I - D over Y^2 (Ypow[1]),
// which is not read again.
__global__ void pade_combo_kernel(double* __restrict__ W, int n, int64_t stride, Coefs cf) {
  const int64_t nn = (int64_t)n * n;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nn) return;
  double* w = W + stride * blockIdx.y;
  const bool diag = (idx % n) == (idx / n);
  double sn = diag ? cf.n[0] : 0.0, sd = diag ? cf.d[0] : 0.0;
  for (int k = 1; k <= kPadeM; ++k) {
    const double y = w[(int64_t)(k - 1) * nn + idx];
    sn += cf.n[k] * y;
    sd += cf.d[k] * y;
  }
  w[(int64_t)kPadeM * nn + idx] = sn;        // N
  w[(int64_t)(kPadeM + 1) * nn + idx] = sd;  // D
  w[nn + idx] = (diag ? 2.0 : 0.0) - sd;      // X_1
}

// Modified squaring combination for one entry and all orders at once:
//   new_0 = T_0,  new_k = 2^{-k} (T_k + sum_{j=1}^{k} old_j / (k-j)!),
// where T_k = old_0 old_k.  T and new share storage.
__global__ void square_combo_kernel(double* __restrict__ W, int n, int64_t stride, int64_t off_old, int64_t off_T,
                                    int p) {
  const int64_t nn = (int64_t)n * n;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nn) return;
  double* w = W + stride * blockIdx.y;
  const double* old = w + off_old;
  double* T = w + off_T;
  double inv_fact[8] = {1.0, 1.0, 0.5, 1.0 / 6.0, 1.0 / 24.0, 1.0 / 120.0, 1.0 / 720.0, 1.0 / 5040.0};
  for (int k = 1; k <= p; ++k) {
    double s = T[(int64_t)k * nn + idx];
    for (int j = 1; j <= k; ++j) s += old[(int64_t)j * nn + idx] * inv_fact[k - j];
    T[(int64_t)k * nn + idx] = ldexp(s, -k);
  }
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
  if (p < 0 || p > 6) {
    set_error("phi order %d outside 0..6", p);
    return SETD_EINVAL;
  }
  const int64_t nn = (int64_t)n * n;
  // entries are processed in chunks that keep the workspace below ~1 GiB
  const int per_entry_blocks = kPadeM + 2 + 2 * (p + 1);
  const int64_t stride = per_entry_blocks * nn;
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

  // Pade coefficients (long double, from the closed forms above).
  Coefs cf;
  int ns_iters = 0;
  {
    auto fact = [](int k) {
      long double f = 1.0L;
      for (int i = 2; i <= k; ++i) f *= i;
      return f;
    };
    const int m = kPadeM;
    long double d[kPadeM + 1], nc[kPadeM + 1];
    for (int j = 0; j <= m; ++j)
      d[j] = ((j & 1) ? -1.0L : 1.0L) * fact(m) * fact(2 * m + p - j) / (fact(2 * m + p) * fact(j) * fact(m - j));
    for (int i = 0; i <= m; ++i) {
      long double acc = 0.0L;
      for (int j = 0; j <= i; ++j) acc += d[j] / fact(p + i - j);
      nc[i] = acc;
    }
    for (int i = 0; i <= m; ++i) {
      cf.n[i] = (double)nc[i];
      cf.d[i] = (double)d[i];
    }
    long double rho = 0.0L;
    for (int j = 1; j <= m; ++j) rho += fabsl(d[j]);
    // residual bound after X_1 and `ns_iters` further steps: rho^(2^(ns_iters+1))
    long double r = rho * rho;
    while (r > 1e-22L && ns_iters < 12) {
      r *= r;
      ++ns_iters;
    }
    if (!(rho < 0.9L) || r > 1e-22L) {
      set_error("phi: Pade denominator bound %g too large for the inverse iteration", (double)rho);
      return SETD_EINVAL;
    }
  }

  Buf ws, dev;
  SETD_HIP(hipMalloc(&ws.p, (size_t)chunk * stride * sizeof(double)));
  // per chunk: scalars (chunk) + gemm descriptors
  // descriptors: (m-1) power products, two parities of the two Newton-Schulz
  // products, the final D^{-1} N, p recurrence products and two parities of
  // (p+1) squaring products, per entry
  const int ndesc_max = chunk * ((kPadeM - 1) + 5 + p + 2 * (p + 1));
  const size_t scal_bytes = ((chunk * sizeof(double) + 63) / 64) * 64;
  const size_t dev_bytes = scal_bytes + (size_t)ndesc_max * sizeof(GemmDesc);
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

    // Host-built tables: scalars, then descriptor sets.
    std::vector<char> host(dev_bytes, 0);
    double* hs = (double*)host.data();
    for (int j = 0; j < E; ++j) hs[j] = std::ldexp(c[e0 + j], -sq);
    GemmDesc* hd = (GemmDesc*)(host.data() + scal_bytes);
    GemmDesc* dd = (GemmDesc*)((char*)dev.p + scal_bytes);
    // layout of entry j: Ypow[0..m-1] | N | D | bufA[0..p] | bufB[0..p]
    auto blk = [&](int j, int b) { return ws.p + stride * j + (int64_t)b * nn; };
    const int offA = kPadeM + 2, offB = offA + (p + 1);
    // power chain Y^k = Y^{k-1} Y: one set of E descriptors per k
    int nd = 0;
    GemmDesc* pow_d = hd + nd;
    for (int k = 2; k <= kPadeM; ++k)
      for (int j = 0; j < E; ++j) hd[nd++] = {blk(j, k - 2), blk(j, 0), blk(j, k - 1)};
    // Newton-Schulz on the free power blocks: X in block 1 or 3 by parity,
    // S = 2I - D X in block 2; then bufA[p] = X N
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
    // recurrence: bufA[k] = Y bufA[k+1] + I/k!
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
    if ((size_t)((char*)(hd + nd) - host.data()) > dev_bytes) {
      set_error("phi: internal descriptor overflow");
      return SETD_EINVAL;
    }
    SETD_HIP(hipMemcpyAsync(dev.p, host.data(), dev_bytes, hipMemcpyHostToDevice, s));
    auto dptr = [&](GemmDesc* hp) { return dd + (hp - hd); };

    const dim3 gtile((unsigned)ceil_div(n, 64), (unsigned)ceil_div(n, 64));
    const dim3 ew((unsigned)ceil_div(nn, 256), (unsigned)E);
    // 1. Y = (c/2^s) A
    hipLaunchKernelGGL(scale_batch_kernel, ew, dim3(256), 0, s, A, nn, (const double*)dev.p, ws.p, stride);
    SETD_LAUNCHED();
    // 2. powers
    for (int k = 2; k <= kPadeM; ++k) {
      hipLaunchKernelGGL(gemm_nn_kernel, dim3(gtile.x, gtile.y, E), dim3(256), 0, s, dptr(pow_d + (k - 2) * E), n,
                         1.0, 0.0);
      SETD_LAUNCHED();
    }
    // 3. N, D, X_1 = 2I - D; Newton-Schulz steps; phi_p(Y) ~ X N
    hipLaunchKernelGGL(pade_combo_kernel, ew, dim3(256), 0, s, ws.p, n, stride, cf);
    SETD_LAUNCHED();
    for (int it = 0; it < ns_iters; ++it) {
      hipLaunchKernelGGL(gemm_nn_kernel, dim3(gtile.x, gtile.y, E), dim3(256), 0, s, dptr(ns_d[it & 1][0]), n, -1.0,
                         2.0);
      SETD_LAUNCHED();
      hipLaunchKernelGGL(gemm_nn_kernel, dim3(gtile.x, gtile.y, E), dim3(256), 0, s, dptr(ns_d[it & 1][1]), n, 1.0,
                         0.0);
      SETD_LAUNCHED();
    }
    hipLaunchKernelGGL(gemm_nn_kernel, dim3(gtile.x, gtile.y, E), dim3(256), 0, s, dptr(fin_d), n, 1.0, 0.0);
    SETD_LAUNCHED();
    // 4. phi_k = Y phi_{k+1} + I/k!
    {
      std::vector<double> invf(p + 1, 1.0);
      for (int k = 1; k <= p; ++k) invf[k] = invf[k - 1] / k;
      for (int q = 0; q < p; ++q) {
        const int k = p - 1 - q;
        hipLaunchKernelGGL(gemm_nn_kernel, dim3(gtile.x, gtile.y, E), dim3(256), 0, s, dptr(rec_d + q * E), n,
                           1.0, invf[k]);
        SETD_LAUNCHED();
      }
    }
    // 5. s modified squarings
    int cur = 0;   // 0: current values in bufA, 1: in bufB
    for (int it = 0; it < sq; ++it) {
      hipLaunchKernelGGL(gemm_nn_kernel, dim3(gtile.x, gtile.y, E * (p + 1)), dim3(256), 0, s, dptr(sq_d[cur]), n,
                         1.0, 0.0);
      SETD_LAUNCHED();
      const int64_t off_old = (int64_t)(cur == 0 ? offA : offB) * nn;
      const int64_t off_T = (int64_t)(cur == 0 ? offB : offA) * nn;
      if (p > 0) {
        hipLaunchKernelGGL(square_combo_kernel, ew, dim3(256), 0, s, ws.p, n, stride, off_old, off_T, p);
        SETD_LAUNCHED();
      }
      cur ^= 1;
    }
    // 6. copy out
    const int offR = cur == 0 ? offA : offB;
    for (int j = 0; j < E; ++j)
      for (int k = 0; k <= p; ++k)
        SETD_HIP(hipMemcpyAsync(out[(int64_t)(e0 + j) * (p + 1) + k], blk(j, offR + k), nn * sizeof(double),
                                hipMemcpyDeviceToDevice, s));
    SETD_HIP(hipStreamSynchronize(s));   // host tables and workspace are reused by the next chunk
  }
  return SETD_OK;
}

}  // namespace setd
