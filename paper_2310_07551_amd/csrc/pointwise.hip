// Pointwise and small helper kernels of the split-ETD3 step.
//
//  * packing of the small matrices into the layouts the mode kernels read;
//  * G = g(U), F = K U + G (Algorithms 1-2, first line of the time loop) with
//    K applied as a 3-point stencil per direction when every A_mu is
//    tridiagonal (eq. kronsumv: K t = vec(sum_mu T x_mu A_mu), a tridiagonal
//    A_mu touches the neighbours i_mu - 1, i_mu, i_mu + 1 only);
//  * D = g(U_s) - G (stage differences d_ni of eq. ERK3);
//  * deterministic norms (fixed-order two-pass reductions).
// All of these are bound by HBM bandwidth: one thread per grid point,
// contiguous along i_1, no reuse beyond the stencil neighbours.
#include <algorithm>

#include "common.hpp"
#include "pointwise.hpp"

namespace setd {

// ---------------------------------------------------------------------------
// packing
// ---------------------------------------------------------------------------
template <typename T>
__global__ void pack_kernel(const double* __restrict__ M, int n, int ldp, double scale, bool rowmajor,
                            T* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)ldp * ldp) return;
  const int r = (int)(idx % ldp), c = (int)(idx / ldp);   // out index = r + ldp*c
  // rowmajor: out[i*ldp + p] = M[i, p]  ->  r = p, c = i
  // colmajor: out[i + ldp*p] = M[i, p]  ->  r = i, c = p
  const int i = rowmajor ? c : r, p = rowmajor ? r : c;
  double v = (i < n && p < n) ? scale * M[i + (int64_t)n * p] : 0.0;
  out[idx] = (T)v;
}

// bf16 split: the packed buffer holds np planes of ldp*ldp bf16 values,
// plane k the round-to-nearest-even bf16 of what planes 0..k-1 leave of the
// (FP64) matrix entry, so the entry is ~ the sum of its np pieces.
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__global__ void pack_bf16_kernel(const double* __restrict__ M, int n, int ldp, double scale, bool rowmajor, int np,
                                 uint16_t* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tot = (int64_t)ldp * ldp;
  if (idx >= tot) return;
  const int r = (int)(idx % ldp), c = (int)(idx / ldp);
  const int i = rowmajor ? c : r, p = rowmajor ? r : c;
  double rem = (i < n && p < n) ? scale * M[i + (int64_t)n * p] : 0.0;
  for (int k = 0; k < np; ++k) {
    const uint16_t h = f32_to_bf16_rne((float)rem);
    out[k * tot + idx] = h;
    rem -= (double)bf16_to_f32(h);
  }
}

size_t packed_bytes(int n, int prec) {
  const size_t e = (size_t)packed_ld(n) * packed_ld(n);
  if (prec == SETD_PREC_F64) return e * 8;
  if (prec == SETD_PREC_F32) return e * 4;
  if (prec == SETD_PREC_BF16X3) return e * 6;   // three bf16 planes
  if (prec == SETD_PREC_I8X4) return packed_bytes_i8(n);
  return e * 4;                                 // two bf16 planes
}

int pack_matrix_f64(const double* M, int n, double scale, bool rowmajor, double* out, hipStream_t s) {
  const int ldp = packed_ld(n);
  const int64_t tot = (int64_t)ldp * ldp;
  hipLaunchKernelGGL(pack_kernel<double>, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, s, M, n, ldp, scale,
                     rowmajor, out);
  SETD_LAUNCHED();
  return SETD_OK;
}

int pack_matrix_f32(const double* M, int n, double scale, bool rowmajor, float* out, hipStream_t s) {
  const int ldp = packed_ld(n);
  const int64_t tot = (int64_t)ldp * ldp;
  hipLaunchKernelGGL(pack_kernel<float>, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, s, M, n, ldp, scale,
                     rowmajor, out);
  SETD_LAUNCHED();
  return SETD_OK;
}

int pack_matrix_bf16(const double* M, int n, double scale, bool rowmajor, int np, void* out, hipStream_t s) {
  const int ldp = packed_ld(n);
  const int64_t tot = (int64_t)ldp * ldp;
  hipLaunchKernelGGL(pack_bf16_kernel, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, s, M, n, ldp, scale,
                     rowmajor, np, (uint16_t*)out);
  SETD_LAUNCHED();
  return SETD_OK;
}

// ---------------------------------------------------------------------------
// simple vector helpers
// ---------------------------------------------------------------------------
__global__ void axpby_kernel(const double* __restrict__ x, double* __restrict__ y, int64_t n, double a, double b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (b == 0.0) ? a * x[i] : a * x[i] + b * y[i];
}

__global__ void scale_kernel(double* __restrict__ y, int64_t n, double b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (b == 0.0) ? 0.0 : b * y[i];
}

template <typename T>
__global__ void convert_kernel(const double* __restrict__ x, T* __restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (T)x[i];
}

int launch_axpby(const double* x, double* y, int64_t n, double a, double b, hipStream_t s) {
  if (n == 0) return SETD_OK;
  hipLaunchKernelGGL(axpby_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, x, y, n, a, b);
  SETD_LAUNCHED();
  return SETD_OK;
}

int launch_scale(double* y, int64_t n, double b, hipStream_t s) {
  if (n == 0) return SETD_OK;
  hipLaunchKernelGGL(scale_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, y, n, b);
  SETD_LAUNCHED();
  return SETD_OK;
}

int launch_copy_convert(const double* x, void* y, int64_t n, DType out, hipStream_t s) {
  if (n == 0) return SETD_OK;
  if (out == DType::F64)
    hipLaunchKernelGGL(convert_kernel<double>, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, x, (double*)y, n);
  else
    hipLaunchKernelGGL(convert_kernel<float>, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, x, (float*)y, n);
  SETD_LAUNCHED();
  return SETD_OK;
}

// ---------------------------------------------------------------------------
// reaction, G/F and stage kernels
// ---------------------------------------------------------------------------

// Per-point bodies.  u holds NC fields, component c at u + c * cs;
// point idx has grid indices (i1, i2, i3) with i1 fastest.  D and NC are
// template arguments and every load is unconditional (a clamped index and a
// zero coefficient past the boundary, an exact +0 term), so that a point's
// loads are in flight together: behind a branch, or in a loop with a
// run-time trip count, each would be waited for on its own.
template <typename TF, int D, int NC>
__device__ __forceinline__ void gf_point_at(const double* __restrict__ u, int64_t cs, int64_t idx, int i1, int i2,
                                            int i3, int n1, int n2, int n3, const StencilSet& S, const GParams& gp,
                                            double* __restrict__ G, TF* __restrict__ F) {
  const int idxs[3] = {i1, i2, i3};
  const int ns[3] = {n1, n2, n3};
  const int64_t strides[3] = {1, (int64_t)n1, (int64_t)n1 * n2};

  double uc[2] = {0.0, 0.0}, g[2];
#pragma unroll
  for (int c = 0; c < NC; ++c) uc[c] = u[(int64_t)c * cs + idx];
  reaction(gp, uc[0], uc[1], g[0], g[1]);
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double* __restrict__ uu = u + (int64_t)c * cs;
    double k = 0.0;
#pragma unroll
    for (int mu = 0; mu < D; ++mu) {
      const int i = idxs[mu];
      const int off = c * 3 + mu;
      const bool has_lo = i > 0, has_up = i + 1 < ns[mu];
      const double lo = has_lo ? S.lo[off][i] : 0.0, up = has_up ? S.up[off][i] : 0.0;
      const double xl = uu[idx - (has_lo ? strides[mu] : 0)], xu = uu[idx + (has_up ? strides[mu] : 0)];
      double t = S.di[off][i] * uc[c];
      t += lo * xl;
      t += up * xu;
      k += t;
    }
    G[(int64_t)c * cs + idx] = g[c];
    F[(int64_t)c * cs + idx] = (TF)(k + g[c]);
  }
}

// Same, for a flat point index (the batched kernels); d in {2, 3} and ncomp
// in {1, 2} (the batch is checked at creation), uniform over a block.
template <typename TF>
__device__ __forceinline__ void gf_point(const double* __restrict__ u, int64_t cs, int64_t idx, int ncomp, int d,
                                         int n1, int n2, int n3, const StencilSet& S, const GParams& gp,
                                         double* __restrict__ G, TF* __restrict__ F) {
  const int i1 = (int)(idx % n1);
  const int64_t r = idx / n1;
  const int i2 = (int)(r % n2);
  const int i3 = (d == 3) ? (int)(r / n2) : 0;
  if (d == 3) {
    if (ncomp == 2) gf_point_at<TF, 3, 2>(u, cs, idx, i1, i2, i3, n1, n2, n3, S, gp, G, F);
    else gf_point_at<TF, 3, 1>(u, cs, idx, i1, i2, i3, n1, n2, n3, S, gp, G, F);
  } else {
    if (ncomp == 2) gf_point_at<TF, 2, 2>(u, cs, idx, i1, i2, i3, n1, n2, n3, S, gp, G, F);
    else gf_point_at<TF, 2, 1>(u, cs, idx, i1, i2, i3, n1, n2, n3, S, gp, G, F);
  }
}

__device__ __forceinline__ void g_point(const double* __restrict__ u, int64_t cs, int64_t idx, int ncomp,
                                        const GParams& gp, double* __restrict__ G) {
  double g[2];
  reaction(gp, u[idx], ncomp > 1 ? u[cs + idx] : 0.0, g[0], g[1]);
  for (int c = 0; c < ncomp; ++c) G[(int64_t)c * cs + idx] = g[c];
}

template <typename TD>
__device__ __forceinline__ void stage_d_point(const double* __restrict__ Us, const double* __restrict__ G,
                                              int64_t cs, int64_t idx, int ncomp, const GParams& gp,
                                              TD* __restrict__ D) {
  double g[2];
  reaction(gp, Us[idx], ncomp > 1 ? Us[cs + idx] : 0.0, g[0], g[1]);
  for (int c = 0; c < ncomp; ++c) D[(int64_t)c * cs + idx] = (TD)(g[c] - G[(int64_t)c * cs + idx]);
}

// Writes G_c = g_c(u) and F_c = (K_c u_c) + G_c for every component (F in
// FP64, or FP32 for the reduced-precision Tuckers).  Each thread owns one i1
// and walks RB consecutive i2 rows of one i3 plane, carrying the previous,
// current and next row values of every component in registers, so each
// i2 neighbour is loaded once; the i1 and i3 coefficients are loaded once
// per thread.  The grid is (ceil(n1 / blockDim.x), ceil(n2 / RB), n3): no
// integer division per point.  The sums are formed in the order of
// gf_point_at (direction by direction).  Every neighbour is loaded without
// a branch, from a clamped index, and a neighbour past the boundary gets a
// zero coefficient (an exact +0 term); the component count NC is a template
// argument, so the component loops unroll.  Behind a branch or a run-time
// loop each load would be waited for on its own before the next one issues.
template <typename TF, int RB, int NC>
__global__ void gf_stencil_kernel(const double* __restrict__ u, int64_t N, int d, int n1, int n2, int n3,
                                  StencilSet S, GParams gp, double* __restrict__ G, TF* __restrict__ F) {
  const int i1 = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i1 >= n1) return;
  const int r0 = (int)blockIdx.y * RB, i3 = (int)blockIdx.z;
  const int64_t s2 = n1, s3 = (int64_t)n1 * n2;
  const int64_t base = (int64_t)i3 * s3 + i1;
  double d1[2], l1[2], u1[2], d3[2], l3[2], u3[2], prv[2], cur[2];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int o1 = c * 3, o3 = c * 3 + 2;
    d1[c] = S.di[o1][i1];
    l1[c] = i1 > 0 ? S.lo[o1][i1] : 0.0;
    u1[c] = i1 + 1 < n1 ? S.up[o1][i1] : 0.0;
    d3[c] = d == 3 ? S.di[o3][i3] : 0.0;
    l3[c] = (d == 3 && i3 > 0) ? S.lo[o3][i3] : 0.0;
    u3[c] = (d == 3 && i3 + 1 < n3) ? S.up[o3][i3] : 0.0;
    prv[c] = r0 > 0 ? u[c * N + base + (int64_t)(r0 - 1) * s2] : 0.0;
    cur[c] = u[c * N + base + (int64_t)r0 * s2];
  }
  const int64_t m1 = i1 > 0 ? -1 : 0, p1 = i1 + 1 < n1 ? 1 : 0;                  // clamped i1 neighbours
  const int64_t m3 = (d == 3 && i3 > 0) ? -s3 : 0, p3 = (d == 3 && i3 + 1 < n3) ? s3 : 0;   // and i3
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    const int i2 = r0 + r;
    if (i2 >= n2) break;
    const int64_t idx = base + (int64_t)i2 * s2;
    const bool has_next = i2 + 1 < n2;
    double nxt[2] = {0.0, 0.0}, g[2];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double x = u[c * N + idx + (has_next ? s2 : 0)];
      nxt[c] = has_next ? x : 0.0;
    }
    reaction(gp, cur[0], NC > 1 ? cur[1] : 0.0, g[0], g[1]);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double* __restrict__ uu = u + (int64_t)c * N;
      const int o2 = c * 3 + 1;
      // l1, u1, l3, u3 are zero past the boundary; so are prv and nxt
      const double lo2 = i2 > 0 ? S.lo[o2][i2] : 0.0, up2 = has_next ? S.up[o2][i2] : 0.0;
      double t = d1[c] * cur[c];
      t += l1[c] * uu[idx + m1];
      t += u1[c] * uu[idx + p1];
      double k = 0.0;
      k += t;
      t = S.di[o2][i2] * cur[c];
      t += lo2 * prv[c];
      t += up2 * nxt[c];
      k += t;
      t = d3[c] * cur[c];   // d == 2: zero coefficients, offsets 0 (the point itself)
      t += l3[c] * uu[idx + m3];
      t += u3[c] * uu[idx + p3];
      k += t;
      G[(int64_t)c * N + idx] = g[c];
      F[(int64_t)c * N + idx] = (TF)(k + g[c]);
      prv[c] = cur[c];
      cur[c] = nxt[c];
    }
  }
}

// G_c = g_c(u) only (the dense-K path adds the mode products afterwards).
__global__ void g_kernel(const double* __restrict__ u, int ncomp, int64_t N, GParams gp, double* __restrict__ G) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= N) return;
  g_point(u, N, idx, ncomp, gp, G);
}

// D_c = g_c(Us) - G_c.
template <typename TD>
__global__ void stage_d_kernel(const double* __restrict__ Us, const double* __restrict__ G, int ncomp, int64_t N,
                               GParams gp, TD* __restrict__ D) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= N) return;
  stage_d_point<TD>(Us, G, N, idx, ncomp, gp, D);
}

// ---- batched forms: one launch over the points of every instance ----
// Blocks of 256 points never straddle two instances: instance b owns blocks
// blk[b] .. blk[b+1]-1.
__device__ __forceinline__ int find_inst(const int64_t* __restrict__ blk, int nbatch, int64_t block) {
  int lo = 0, hi = nbatch - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (blk[mid] <= block) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// kind 0: G, F with the stencil; 1: G only; 2: D = g(U_s) - G
__global__ void batch_pointwise_kernel(int kind, const BatchInstDev* __restrict__ inst, const int64_t* __restrict__ blk,
                                       int nbatch, int ncomp, const double* __restrict__ x, double* __restrict__ G,
                                       double* __restrict__ out) {
  const int b = find_inst(blk, nbatch, blockIdx.x);
  const BatchInstDev& I = inst[b];
  const int64_t idx = (int64_t)(blockIdx.x - blk[b]) * blockDim.x + threadIdx.x;
  if (idx >= I.N) return;
  if (kind == 0)
    gf_point<double>(x + I.off, I.cs, idx, ncomp, I.d, I.n[0], I.n[1], I.n[2], I.st, I.gp, G + I.off, out + I.off);
  else if (kind == 1)
    g_point(x + I.off, I.cs, idx, ncomp, I.gp, G + I.off);
  else
    stage_d_point<double>(x + I.off, G + I.off, I.cs, idx, ncomp, I.gp, out + I.off);
}

int launch_batch_pointwise(int kind, const BatchInstDev* inst, const int64_t* blk, int nbatch, int64_t nblocks,
                           int ncomp, int64_t total_points, const double* x, double* G, double* out, hipStream_t s) {
  if (nblocks == 0) return SETD_OK;
  // kind 0 reads u, writes G and F; 1 reads u, writes G; 2 reads U_s and G, writes D
  const double per = kind == 1 ? 16.0 : 24.0;
  ProfScope prof(s, kProfPointwise, 0.0, per * (double)ncomp * (double)total_points);
  hipLaunchKernelGGL(batch_pointwise_kernel, dim3((unsigned)nblocks), dim3(kBatchBlock), 0, s, kind, inst, blk,
                     nbatch, ncomp, x, G, out);
  SETD_LAUNCHED();
  return SETD_OK;
}

int launch_gf_stencil(const double* u, int ncomp, int64_t N, int d, const int* dims, const StencilSet& S,
                      const GParams& gp, double* G, void* F, DType ftype, hipStream_t s) {
  const int n3 = d == 3 ? dims[2] : 1;
  constexpr int RB = 8;   // i2 rows per thread
  const int bx = (int)std::min<int64_t>(256, round_up(dims[0], 64));
  const dim3 grid((unsigned)ceil_div(dims[0], bx), (unsigned)ceil_div(dims[1], RB), (unsigned)n3);
  // reads u once, writes G (FP64) and F
  ProfScope prof(s, kProfPointwise, 0.0, (double)N * ncomp * (8 + 8 + (ftype == DType::F64 ? 8 : 4)));
  auto launch = [&](auto tf, auto nc) {
    using TF = decltype(tf);
    hipLaunchKernelGGL((gf_stencil_kernel<TF, RB, decltype(nc)::value>), grid, dim3(bx), 0, s, u, N, d, dims[0],
                       dims[1], n3, S, gp, G, (TF*)F);
  };
  if (ftype == DType::F64) {
    if (ncomp == 1) launch(0.0, std::integral_constant<int, 1>{});
    else launch(0.0, std::integral_constant<int, 2>{});
  } else {
    if (ncomp == 1) launch(0.0f, std::integral_constant<int, 1>{});
    else launch(0.0f, std::integral_constant<int, 2>{});
  }
  SETD_LAUNCHED();
  return SETD_OK;
}

int launch_g(const double* u, int ncomp, int64_t N, const GParams& gp, double* G, hipStream_t s) {
  hipLaunchKernelGGL(g_kernel, dim3((unsigned)ceil_div(N, 256)), dim3(256), 0, s, u, ncomp, N, gp, G);
  SETD_LAUNCHED();
  return SETD_OK;
}

int launch_stage_d(const double* Us, const double* G, int ncomp, int64_t N, const GParams& gp, void* D,
                   DType dtype, hipStream_t s) {
  const dim3 grid((unsigned)ceil_div(N, 256));
  // reads Us and G, writes D
  ProfScope prof(s, kProfPointwise, 0.0, (double)N * ncomp * (8 + 8 + (dtype == DType::F64 ? 8 : 4)));
  if (dtype == DType::F64)
    hipLaunchKernelGGL(stage_d_kernel<double>, grid, dim3(256), 0, s, Us, G, ncomp, N, gp, (double*)D);
  else
    hipLaunchKernelGGL(stage_d_kernel<float>, grid, dim3(256), 0, s, Us, G, ncomp, N, gp, (float*)D);
  SETD_LAUNCHED();
  return SETD_OK;
}

// ---------------------------------------------------------------------------
// deterministic norms
// ---------------------------------------------------------------------------
// Pass 1: block b reduces a contiguous chunk of x (and x - y): each thread
// strides through it, the 64 lanes of a wave combine by an xor-shuffle
// butterfly, the block's four waves in LDS in wave order.  Pass 2: one block
// reduces the per-block partials the same way.  Every addition happens in an
// order fixed by the launch shape, so repeated calls give identical bits.
constexpr int kNormBlocks = 1024;
constexpr int kNormThreads = 256;

__device__ __forceinline__ double nanmax(double a, double b) {
  return (a != a || b != b) ? __builtin_nan("") : fmax(a, b);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = nanmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Combines the four per-thread values {sum, max, sum, max} of a 256-thread
// block; thread 0 returns the block's result in r.
__device__ __forceinline__ void block_reduce4(double (&r)[4]) {
  __shared__ double w[4][kNormThreads / 64];
  r[0] = wave_sum(r[0]);
  r[1] = wave_max(r[1]);
  r[2] = wave_sum(r[2]);
  r[3] = wave_max(r[3]);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int k = 0; k < 4; ++k) w[k][wave] = r[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 0; k < 4; ++k) r[k] = w[k][0];
    for (int v = 1; v < kNormThreads / 64; ++v) {
      r[0] += w[0][v];
      r[1] = nanmax(r[1], w[1][v]);
      r[2] += w[2][v];
      r[3] = nanmax(r[3], w[3][v]);
    }
  }
}

__global__ void __launch_bounds__(kNormThreads) norm_pass1(const double* __restrict__ x, const double* __restrict__ y,
                                                            int64_t n, double* __restrict__ part) {
  const int64_t chunk = ceil_div_dev(n, (int64_t)gridDim.x);
  const int64_t beg = chunk * blockIdx.x;
  const int64_t end = beg + chunk < n ? beg + chunk : n;
  double r[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t i = beg + threadIdx.x; i < end; i += kNormThreads) {
    const double v = x[i];
    r[0] = fma(v, v, r[0]);
    r[1] = nanmax(r[1], fabs(v));
    if (y) {
      const double e = v - y[i];
      r[2] = fma(e, e, r[2]);
      r[3] = nanmax(r[3], fabs(e));
    }
  }
  block_reduce4(r);
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) part[4 * blockIdx.x + k] = r[k];
}

__global__ void __launch_bounds__(kNormThreads) norm_pass2(const double* __restrict__ part, double* __restrict__ out) {
  double r[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < kNormBlocks; b += kNormThreads) {
    r[0] += part[4 * b];
    r[1] = nanmax(r[1], part[4 * b + 1]);
    r[2] += part[4 * b + 2];
    r[3] = nanmax(r[3], part[4 * b + 3]);
  }
  block_reduce4(r);
  if (threadIdx.x == 0) {
    out[0] = sqrt(r[0]);
    out[1] = r[1];
    out[2] = sqrt(r[2]);
    out[3] = r[3];
  }
}

size_t norm_workspace_bytes() { return (size_t)(4 * kNormBlocks + 4) * sizeof(double); }

int launch_norms(const double* x, const double* y, int64_t n, double* ws, hipStream_t s) {
  hipLaunchKernelGGL(norm_pass1, dim3(kNormBlocks), dim3(kNormThreads), 0, s, x, y, n, ws);
  SETD_LAUNCHED();
  hipLaunchKernelGGL(norm_pass2, dim3(1), dim3(kNormThreads), 0, s, ws, ws + 4 * kNormBlocks);
  SETD_LAUNCHED();
  return SETD_OK;
}

}  // namespace setd
