// Reduced-precision mu-mode products (same operation and job tables as
// mode_f64.hip): operands and intermediates in FP32, the last mode of a
// Tucker written in FP64 on top of an FP64 base.
//
//   SETD_PREC_F32     v_mfma_f32_16x16x4f32, FP32 accumulate.
//   SETD_PREC_BF16X3  v_mfma_f32_16x16x32_bf16 with the three-term split
//                     x = h + m + l (h = bf16(x), m = bf16(x - h),
//                     l = bf16(x - h - m)) and the six products of order
//                     <= 2^-16: hh + hm + mh + hl + lh + mm, FP32 accumulate
//                     (about FP32 accuracy).
//   SETD_PREC_BF16X2  the two-term split x = h + l with hh + hl + lh (about
//                     16 significant bits, half the matrix-core work).
//                     The matrix is split once when it is packed; the tensor
//                     operand is split in registers right after its load.
//
// Per-term scale factors multiply FP32 partial sums (never a bf16 piece, and
// never inside a load, where the multiply would make the wave wait for it).
//
// Operand layouts (probed on gfx950): FP32 16x16x4 and BF16 16x16x32 put
// tile row 4 g + r in register r of lane (g, l); in the bf16 form lane (g, l)
// supplies A[l][8 g + j] and B[8 g + j][l] in slot j.
//
// mode 1 (contraction index contiguous):  MFMA rows = i (matrix, packed
//   row-major), columns = b (tensor columns), k = p.
// modes >= 2:  MFMA rows = a (contiguous tensor index), columns = i, k = p;
//   the FP32 form reads the matrix column-major packed, the bf16 form
//   row-major packed (it needs 8 consecutive p of one row per lane).
#include <cstring>

#include "common.hpp"

#include <cstdlib>

namespace setd {
namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ int64_t remap_xcd_lp(int64_t bid, int64_t per_xcd) {
  return (bid & 7) * per_xcd + (bid >> 3);
}

__device__ __forceinline__ int find_job_lp(const ModeJobs& J, int64_t t) { return find_job(J, t); }

// x = p[0] + p[1] (+ p[2]): each piece the bf16 rounding (RNE) of the FP32
// remainder left by the previous ones.
template <int NP>
__device__ __forceinline__ void split_bf16(const f8& x, bf8 (&p)[NP]) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    float r = x[j];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      const __bf16 h = (__bf16)r;
      p[k][j] = h;
      r -= (float)h;
    }
  }
}

__device__ __forceinline__ f4 mfma_bf(const bf8& a, const bf8& b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// One k-chunk of the split product.  The bf16 matrix-core accumulation was
// measured on gfx950 to round with a small bias toward zero (positive-data
// mode products: mean relative error -2e-8 at n = 256, growing with the
// number of chained accumulations; FP32 MFMA: 1e-10).  A bias does not average
// out over the Tuckers and steps of the integrator, so the leading product
// h*h is formed per chunk from a zero accumulator and added to `main` with an
// FP32 VALU add (round to nearest), and the cross products of order <= 2^-8
// (NP = 2) or <= 2^-16 (NP = 3) chain in their own, 2^8 times smaller,
// accumulator `small` (unscaled; the caller applies the term's scale to it
// once).  `main` receives sc * (chunk of h*h).
template <int NP>
__device__ __forceinline__ void mfma_split(const bf8 (&a)[NP], const bf8 (&b)[NP], float sc, f4& main,
                                           f4& small) {
  if constexpr (NP == 3) {
    small = mfma_bf(a[1], b[1], small);
    small = mfma_bf(a[0], b[2], small);
    small = mfma_bf(a[2], b[0], small);
  }
  small = mfma_bf(a[0], b[1], small);
  small = mfma_bf(a[1], b[0], small);
  main += sc * mfma_bf(a[0], b[0], f4{0.f, 0.f, 0.f, 0.f});
}

// Writes `cnt` consecutive results starting at Y + off (all in range when
// full) as FP32 or, for an FP64 output, base + value.
template <typename TOut, typename TV>
__device__ __forceinline__ void store_run(TOut* __restrict__ Y, const double* __restrict__ base, int64_t off,
                                          const TV* v, int cnt, int valid, bool vec) {
  if (vec && valid >= cnt) {
    if constexpr (sizeof(TOut) == 4) {
      for (int e = 0; e < cnt; e += 4)
        *(f4*)(Y + off + e) = f4{(float)v[e], (float)v[e + 1], (float)v[e + 2], (float)v[e + 3]};
    } else {
      for (int e = 0; e < cnt; e += 2) {
        d2 w = d2{(double)v[e], (double)v[e + 1]};
        if (base) w += *(const d2*)(base + off + e);
        *(d2*)(Y + off + e) = w;
      }
    }
  } else {
    for (int e = 0; e < cnt; ++e) {
      if (e < valid) {
        if constexpr (sizeof(TOut) == 4) {
          Y[off + e] = (float)v[e];
        } else {
          double w = (double)v[e];
          if (base) w += base[off + e];
          Y[off + e] = w;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// FP32 with the accumulation chained on the matrix cores (the layout and
// load scheme of the FP64 kernels: lanes load 4 consecutive p, an interior
// variant without masks in ping-pong registers).  FP32 MFMA accumulator
// layout (probed): lane (g, l) register r holds D[4 g + r][l].
// ---------------------------------------------------------------------------
__device__ __forceinline__ f4 mfma32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int TM, int TN, int MODE, typename TOut>
__global__ void __launch_bounds__(64, 2) mode1_f32c_kernel(const ModeJobs J, int64_t per_xcd) {
  constexpr bool VEC = MODE >= 1;
  const int64_t t = remap_xcd_lp(blockIdx.x, per_xcd);
  if (t >= J.total_tiles) return;
  const ModeJob& jb = J.job[find_job_lp(J, t)];
  const int64_t lt = t - jb.tile_begin;
  const int it = (int)(lt % jb.tiles_i);
  const int64_t bt = lt / jb.tiles_i;
  const int lane = threadIdx.x, g = lane >> 4, l = lane & 15;
  const int n = jb.n, ldp = jb.ldp;
  const int64_t nb = jb.nb;
  const int i0 = it * 16 * TM;
  const int64_t b0 = bt * 16 * TN;
  const float* __restrict__ X = (const float*)jb.X[0];
  const float* __restrict__ PT = (const float*)jb.P[0];
  const float sc = (float)jb.scale[0];
  const float* pa[TM];
#pragma unroll
  for (int m = 0; m < TM; ++m) pa[m] = PT + (int64_t)(i0 + TM * l + m) * ldp + 4 * g;
  const float* pb[TN];
  bool vb[TN];
#pragma unroll
  for (int u = 0; u < TN; ++u) {
    const int64_t b = b0 + 16 * u + l;
    vb[u] = b < nb;
    pb[u] = X + (vb[u] ? b : 0) * (int64_t)n + 4 * g;
  }
  f4 acc[TM][TN];
#pragma unroll
  for (int m = 0; m < TM; ++m)
#pragma unroll
    for (int u = 0; u < TN; ++u) acc[m][u] = f4{0.f, 0.f, 0.f, 0.f};
  auto mma = [&](const f4* ar, const f4* br) {
#pragma unroll
    for (int jj = 0; jj < 4; ++jj)
#pragma unroll
      for (int m = 0; m < TM; ++m)
#pragma unroll
        for (int u = 0; u < TN; ++u) acc[m][u] = mfma32(ar[m][jj], br[u][jj], acc[m][u]);
  };
  if constexpr (MODE == 2) {
    auto load = [&](int p0, f4* ar, f4* br) {
#pragma unroll
      for (int m = 0; m < TM; ++m) ar[m] = *(const f4*)(pa[m] + p0);
#pragma unroll
      for (int u = 0; u < TN; ++u) br[u] = *(const f4*)(pb[u] + p0);
    };
    f4 a0[TM], b0r[TN], a1[TM], b1r[TN];
    load(0, a0, b0r);
    for (int p0 = 0; p0 < n; p0 += 32) {
      load(p0 + 16, a1, b1r);
      mma(a0, b0r);
      load(p0 + 32 < n ? p0 + 32 : p0, a0, b0r);
      mma(a1, b1r);
    }
  } else {
    auto load = [&](int p0, f4* ar, f4* br) {
#pragma unroll
      for (int m = 0; m < TM; ++m) ar[m] = *(const f4*)(pa[m] + p0);
      const bool full = VEC && (p0 + 16 <= n);
#pragma unroll
      for (int u = 0; u < TN; ++u) {
        if (full) {
          br[u] = vb[u] ? *(const f4*)(pb[u] + p0) : f4{0.f, 0.f, 0.f, 0.f};
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) br[u][e] = (vb[u] && p0 + 4 * g + e < n) ? pb[u][p0 + e] : 0.f;
        }
      }
    };
    f4 a[TM], bx[TN];
    load(0, a, bx);
    for (int p0 = 0; p0 < n; p0 += 16) {
      f4 an[TM], bn[TN];
      const bool more = p0 + 16 < n;
      if (more) load(p0 + 16, an, bn);
      mma(a, bx);
      if (more) {
#pragma unroll
        for (int m = 0; m < TM; ++m) a[m] = an[m];
#pragma unroll
        for (int u = 0; u < TN; ++u) bx[u] = bn[u];
      }
    }
  }
  // lane (g, l) owns the 4 TM consecutive rows i0 + 4 TM g + (TM r + m) of
  // column b0 + 16 u + l
  TOut* __restrict__ Y = (TOut*)jb.Y;
  const double* __restrict__ base = (const double*)jb.base;
  const int ir = i0 + 4 * TM * g;
#pragma unroll
  for (int u = 0; u < TN; ++u) {
    if (!vb[u]) continue;
    float v[4 * TM];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int m = 0; m < TM; ++m) v[TM * r + m] = sc * acc[m][u][r];
    store_run<TOut>(Y, base, (b0 + 16 * u + l) * (int64_t)n + ir, v, 4 * TM, n - ir, VEC);
  }
}

template <int TM, int TN, int MODE, typename TOut>
__global__ void __launch_bounds__(64, 2) modeB_f32c_kernel(const ModeJobs J, int64_t per_xcd) {
  constexpr bool VEC = MODE >= 1;
  const int64_t t = remap_xcd_lp(blockIdx.x, per_xcd);
  if (t >= J.total_tiles) return;
  const ModeJob& jb = J.job[find_job_lp(J, t)];
  const int64_t lt = t - jb.tile_begin;
  const int it = (int)(lt % jb.tiles_i);
  const int64_t rest = lt / jb.tiles_i;
  const int64_t at = rest % jb.tiles_a;
  const int64_t b = rest / jb.tiles_a;
  const int lane = threadIdx.x, g = lane >> 4, l = lane & 15;
  const int n = jb.n, ldp = jb.ldp, nterms = jb.nterms;
  const int64_t na = jb.na;
  const int64_t a0 = at * 16 * TM;
  const int i0 = it * 16 * TN;
  const int64_t arow = a0 + TM * l;
  const bool lane_full = arow + TM <= na;
  f4 acc[TM][TN];
#pragma unroll
  for (int m = 0; m < TM; ++m)
#pragma unroll
    for (int u = 0; u < TN; ++u) acc[m][u] = f4{0.f, 0.f, 0.f, 0.f};
  const int64_t slab = na * (int64_t)n * b;
  for (int term = 0; term < nterms; ++term) {
    const float* __restrict__ xb = (const float*)jb.X[term] + slab + arow + na * g;
    const float* __restrict__ pbp = (const float*)jb.P[term] + i0 + TN * l + (int64_t)ldp * g;
    const float sc = (float)jb.scale[term];
    // k-steps per register block: 2 (at 3D FHN 256^3 97.4 TFLOP/s against 95.3 for 4 and 96.5 for 8)
    constexpr int KB = 2;
    auto mmablk = [&](float (*xr)[TM], float (*pr)[TN]) {
#pragma unroll
      for (int k = 0; k < KB; ++k)
#pragma unroll
        for (int u = 0; u < TN; ++u) {
          const float pv = pr[k][u] * sc;
#pragma unroll
          for (int m = 0; m < TM; ++m) acc[m][u] = mfma32(xr[k][m], pv, acc[m][u]);
        }
    };
    auto loadblk = [&](int p0, float (*xr)[TM], float (*pr)[TN]) {
#pragma unroll
      for (int k = 0; k < KB; ++k) {
        const int p = p0 + 4 * k;
        const float* xs = xb + na * (int64_t)p;
        const float* ps = pbp + (int64_t)ldp * p;   // padded: always in range
        if constexpr (MODE == 2) {
          if constexpr (TM == 4) {
            const f4 v = *(const f4*)xs;
#pragma unroll
            for (int m = 0; m < TM; ++m) xr[k][m] = v[m];
          } else {
            const f2 v = *(const f2*)xs;
#pragma unroll
            for (int m = 0; m < TM; ++m) xr[k][m] = v[m];
          }
        } else {
          const bool vp = p + g < n;
          if (VEC && TM == 4 && lane_full && vp) {
            const f4 v = *(const f4*)xs;
#pragma unroll
            for (int m = 0; m < TM; ++m) xr[k][m] = v[m];
          } else if (VEC && TM == 2 && (MODE == 2 || (lane_full && vp))) {
            const f2 v = *(const f2*)xs;
#pragma unroll
            for (int m = 0; m < TM; ++m) xr[k][m] = v[m];
          } else {
#pragma unroll
            for (int m = 0; m < TM; ++m) xr[k][m] = (vp && arow + m < na) ? xs[m] : 0.f;
          }
        }
        if constexpr (TN == 2) {
          const f2 w = *(const f2*)ps;
          pr[k][0] = w[0];
          pr[k][1] = w[1];
        } else if constexpr (TN == 4) {
          const f4 w = *(const f4*)ps;
#pragma unroll
          for (int u = 0; u < TN; ++u) pr[k][u] = w[u];
        } else {
#pragma unroll
          for (int u = 0; u < TN; ++u) pr[k][u] = ps[u];
        }
      }
    };
    if constexpr (MODE == 2) {
      float x0[KB][TM], q0[KB][TN], x1[KB][TM], q1[KB][TN];
      loadblk(0, x0, q0);
      for (int p0 = 0; p0 < n; p0 += 8 * KB) {
        loadblk(p0 + 4 * KB, x1, q1);
        mmablk(x0, q0);
        loadblk(p0 + 8 * KB < n ? p0 + 8 * KB : p0, x0, q0);
        mmablk(x1, q1);
      }
    } else {
      float xr[KB][TM], pr[KB][TN];
      loadblk(0, xr, pr);
      for (int p0 = 0; p0 < n; p0 += 4 * KB) {
        float xn[KB][TM], pn[KB][TN];
        const bool more = p0 + 4 * KB < n;
        if (more) loadblk(p0 + 4 * KB, xn, pn);
        mmablk(xr, pr);
        if (more) {
#pragma unroll
          for (int k = 0; k < KB; ++k) {
#pragma unroll
            for (int m = 0; m < TM; ++m) xr[k][m] = xn[k][m];
#pragma unroll
            for (int u = 0; u < TN; ++u) pr[k][u] = pn[k][u];
          }
        }
      }
    }
  }
  TOut* __restrict__ Y = (TOut*)jb.Y;
  const double* __restrict__ base = (const double*)jb.base;
  const int64_t ar = a0 + 4 * TM * g;
#pragma unroll
  for (int u = 0; u < TN; ++u) {
    const int i = i0 + TN * l + u;
    if (i >= n) continue;
    float v[4 * TM];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int m = 0; m < TM; ++m) v[TM * r + m] = acc[m][u][r];
    store_run<TOut>(Y, base, slab + na * (int64_t)i + ar, v, 4 * TM, (int)(na - ar < 4 * TM ? na - ar : 4 * TM),
                    VEC);
  }
}

// ---------------------------------------------------------------------------
// FP32 mode 1 with the matrix panel in LDS: the scheme of the FP64 panel
// kernel (mode_f64.hip) on FP32 operands, for interior jobs with
// 192 <= n <= 256, n % 64 == 0 and 4 x 4 tiles.  A workgroup of 8 waves
// shares one 64-row panel of P (64 KB), stored in LDS in the order the MFMA
// reads it, so no wave holds P in registers; each wave computes `reps`
// 64 x 64 tiles of the workgroup's column group, its tensor loads one 16-p
// chunk ahead of the products.  The products and their order, and the scale
// applied to the FP32 accumulators, are those of the register kernel: the two
// agree bit for bit.  Measured at 3D FHN 256^3: 110 TFLOP/s against 97 for
// the register kernel (two waves per SIMD; at four, 128 registers forced
// spills: 100).  The same panel for modes >= 2 ran at 90.5 (two waves) and
// 93.6 (four) against 95.2 for the register kernel and is not used.
constexpr int kLds32Waves = 8, kLds32MinN = 192, kLds32MaxN = 256, kLds32Reps = 4;

template <typename TOut>
__global__ void __launch_bounds__(512, 1) mode1_lds32_kernel(const ModeJobs J, int64_t per_xcd, int reps) {
  __shared__ f4 panel[(kLds32MaxN / 16) * 4 * 64];   // 64 KB
  const int64_t w = remap_xcd_lp(blockIdx.x, per_xcd);
  if (w >= J.total_tiles) return;   // uniform over the workgroup
  const ModeJob& jb = J.job[find_job_lp(J, w)];
  const int64_t lw = w - jb.tile_begin;
  const int it = (int)(lw % jb.tiles_i);
  const int64_t bg = lw / jb.tiles_i;
  const int n = jb.n, ldp = jb.ldp, nchunk = n / 16;
  const int i0 = it * 64;
  // fill: entry q = (c * 4 + m) * 64 + lane holds P[i0 + 4 l + m][16 c + 4 g + 0..3]
  {
    const float* __restrict__ PT = (const float*)jb.P[0];
    for (int q = threadIdx.x; q < nchunk * 256; q += 512) {
      const int ln = q & 63, m = (q >> 6) & 3, c = q >> 8;
      panel[q] = *(const f4*)(PT + (int64_t)(i0 + 4 * (ln & 15) + m) * ldp + 16 * c + 4 * (ln >> 4));
    }
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, l = lane & 15;
  const float sc = (float)jb.scale[0];
  for (int rep = 0; rep < reps; ++rep) {
    const int64_t bt = (bg * reps + rep) * kLds32Waves + wave;
    if (bt >= jb.tiles_a) return;   // no barrier follows
    const int64_t b0 = bt * 64;
    const float* __restrict__ X = (const float*)jb.X[0];
    const float* pb[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) pb[u] = X + (b0 + 16 * u + l) * (int64_t)n + 4 * g;
    f4 acc[4][4];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[m][u] = f4{0.f, 0.f, 0.f, 0.f};
    auto load = [&](int c, f4 (&xr)[4]) {
#pragma unroll
      for (int u = 0; u < 4; ++u) xr[u] = *(const f4*)(pb[u] + 16 * c);
    };
    auto mma = [&](int c, const f4 (&xr)[4]) {
      f4 a[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) a[m] = panel[(c * 4 + m) * 64 + lane];
#pragma unroll
      for (int jj = 0; jj < 4; ++jj)
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
          for (int u = 0; u < 4; ++u) acc[m][u] = mfma32(a[m][jj], xr[u][jj], acc[m][u]);
    };
    f4 x0[4], x1[4];
    load(0, x0);
    for (int c = 0; c < nchunk; c += 2) {   // nchunk is even (n % 32 == 0)
      load(c + 1, x1);
      mma(c, x0);
      load(c + 2 < nchunk ? c + 2 : c, x0);
      mma(c + 1, x1);
    }
    // lane (g, l) owns rows i0 + 16 g + 4 r + m of column b0 + 16 u + l
    TOut* __restrict__ Y = (TOut*)jb.Y;
    const double* __restrict__ base = (const double*)jb.base;
    const int ir = i0 + 16 * g;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      float v[16];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int m = 0; m < 4; ++m) v[4 * r + m] = sc * acc[m][u][r];
      store_run<TOut>(Y, base, (b0 + 16 * u + l) * (int64_t)n + ir, v, 16, n - ir, true);
    }
  }
}

// ---------------------------------------------------------------------------
// MODE as for the modes >= 2 kernel (2: n % 32 == 0, nb % (16 TN) == 0).
// One wave per SIMD: bounding these kernels to two (128 registers) made them
// spill and run at a fifth of the speed (3D FHN 256^3: 26 against 115 steps/s).
template <int NP, int TM, int TN, int MODE, typename TOut>
__global__ void __launch_bounds__(64) mode1_bf16_kernel(const ModeJobs J, int64_t per_xcd) {
  constexpr bool VEC = MODE >= 1;
  const int64_t t = remap_xcd_lp(blockIdx.x, per_xcd);
  if (t >= J.total_tiles) return;
  const ModeJob& jb = J.job[find_job_lp(J, t)];
  const int64_t lt = t - jb.tile_begin;
  const int it = (int)(lt % jb.tiles_i);
  const int64_t bt = lt / jb.tiles_i;
  const int lane = threadIdx.x, g = lane >> 4, l = lane & 15;
  const int n = jb.n, ldp = jb.ldp;
  const int64_t nb = jb.nb;
  const int64_t plane = (int64_t)ldp * ldp;
  const int i0 = it * 16 * TM;
  const int64_t b0 = bt * 16 * TN;
  const float* __restrict__ X = (const float*)jb.X[0];
  const __bf16* __restrict__ PH = (const __bf16*)jb.P[0];
  const float sc = (float)jb.scale[0];

  int64_t poff[TM];
#pragma unroll
  for (int m = 0; m < TM; ++m) poff[m] = (int64_t)(i0 + TM * l + m) * ldp + 8 * g;
  const float* pb[TN];
  bool vb[TN];
#pragma unroll
  for (int u = 0; u < TN; ++u) {
    const int64_t b = b0 + 16 * u + l;
    vb[u] = b < nb;
    pb[u] = X + (vb[u] ? b : 0) * (int64_t)n + 8 * g;
  }
  f4 acc[TM][TN], accs[TM][TN];   // leading and cross products (see mfma_split)
#pragma unroll
  for (int m = 0; m < TM; ++m)
#pragma unroll
    for (int u = 0; u < TN; ++u) acc[m][u] = accs[m][u] = f4{0.f, 0.f, 0.f, 0.f};

  // One chunk = 32 p: the matrix pieces and the tensor operand's 8 p values
  // per lane in FP32; chunks alternate between two register sets so that
  // each is loaded one chunk of MFMAs before use.
  auto ldc = [&](int p0, bf8 (&ap)[TM][NP], f8 (&xr)[TN]) {
#pragma unroll
    for (int m = 0; m < TM; ++m)
#pragma unroll
      for (int k = 0; k < NP; ++k) ap[m][k] = *(const bf8*)(PH + k * plane + poff[m] + p0);
    const bool full = MODE == 2 || (VEC && (p0 + 32 <= n));
#pragma unroll
    for (int u = 0; u < TN; ++u) {
      if (MODE == 2 || (full && vb[u])) {
        xr[u] = *(const f8*)(pb[u] + p0);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) xr[u][e] = (vb[u] && p0 + 8 * g + e < n) ? pb[u][p0 + e] : 0.f;
      }
    }
  };
  auto cmp = [&](const bf8 (&ap)[TM][NP], const f8 (&xr)[TN]) {
    bf8 bp[TN][NP];
#pragma unroll
    for (int u = 0; u < TN; ++u) split_bf16<NP>(xr[u], bp[u]);
#pragma unroll
    for (int m = 0; m < TM; ++m)
#pragma unroll
      for (int u = 0; u < TN; ++u) mfma_split<NP>(ap[m], bp[u], sc, acc[m][u], accs[m][u]);
  };
  bf8 a0[TM][NP], a1[TM][NP];
  f8 x0[TN], x1[TN];
  ldc(0, a0, x0);
  int p0 = 0;
  for (; p0 + 32 < n; p0 += 64) {
    ldc(p0 + 32, a1, x1);
    __builtin_amdgcn_sched_barrier(0);
    cmp(a0, x0);
    ldc(p0 + 64 < n ? p0 + 64 : p0, a0, x0);   // the last one re-reads a valid chunk
    __builtin_amdgcn_sched_barrier(0);
    cmp(a1, x1);
  }
  if (p0 < n) cmp(a0, x0);
  TOut* __restrict__ Y = (TOut*)jb.Y;
  const double* __restrict__ base = (const double*)jb.base;
  const int ir = i0 + 4 * TM * g;
#pragma unroll
  for (int u = 0; u < TN; ++u) {
    if (!vb[u]) continue;
    float v[4 * TM];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int m = 0; m < TM; ++m) v[TM * r + m] = acc[m][u][r] + sc * accs[m][u][r];
    store_run<TOut>(Y, base, (b0 + 16 * u + l) * (int64_t)n + ir, v, 4 * TM, n - ir, VEC);
  }
}

// ---------------------------------------------------------------------------
// BF16x3, modes >= 2
// ---------------------------------------------------------------------------
// MODE 0: masked element loads; 1: vector loads; 2: additionally every tile
// interior and n % 32 == 0 (no masks in the k loop).
template <int NP, int TM, int TN, int MODE, typename TOut>
__global__ void __launch_bounds__(64) modeB_bf16_kernel(const ModeJobs J, int64_t per_xcd) {
  constexpr bool VEC = MODE >= 1;
  const int64_t t = remap_xcd_lp(blockIdx.x, per_xcd);
  if (t >= J.total_tiles) return;
  const ModeJob& jb = J.job[find_job_lp(J, t)];
  const int64_t lt = t - jb.tile_begin;
  const int it = (int)(lt % jb.tiles_i);
  const int64_t rest = lt / jb.tiles_i;
  const int64_t at = rest % jb.tiles_a;
  const int64_t b = rest / jb.tiles_a;
  const int lane = threadIdx.x, g = lane >> 4, l = lane & 15;
  const int n = jb.n, ldp = jb.ldp, nterms = jb.nterms;
  const int64_t na = jb.na;
  const int64_t plane = (int64_t)ldp * ldp;
  const int64_t a0 = at * 16 * TM;
  const int i0 = it * 16 * TN;
  const int64_t arow = a0 + TM * l;
  const bool lane_full = arow + TM <= na;
  f4 acc[TM][TN], accs[TM][TN];   // leading and cross products (see mfma_split)
#pragma unroll
  for (int m = 0; m < TM; ++m)
#pragma unroll
    for (int u = 0; u < TN; ++u) acc[m][u] = accs[m][u] = f4{0.f, 0.f, 0.f, 0.f};
  const int64_t slab = na * (int64_t)n * b;
  f4 acct[TM][TN];   // scaled cross products of the finished terms
#pragma unroll
  for (int m = 0; m < TM; ++m)
#pragma unroll
    for (int u = 0; u < TN; ++u) acct[m][u] = f4{0.f, 0.f, 0.f, 0.f};
  for (int term = 0; term < nterms; ++term) {
    const float* __restrict__ xb = (const float*)jb.X[term] + slab + arow;
    const __bf16* __restrict__ PH = (const __bf16*)jb.P[term];
    const float sc = (float)jb.scale[term];
    if (term > 0) {
#pragma unroll
      for (int m = 0; m < TM; ++m)
#pragma unroll
        for (int u = 0; u < TN; ++u) accs[m][u] = f4{0.f, 0.f, 0.f, 0.f};
    }
    // One chunk = 32 p: the tensor operand's 8 p values (8 g + j) x TM rows
    // per lane in FP32 and the matrix pieces; chunks alternate between two
    // register sets so that each is loaded one chunk of MFMAs before use.
    auto ldc = [&](int p0, f8 (&xm)[TM], bf8 (&bp)[TN][NP]) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int p = p0 + 8 * g + j;
        const bool vp = MODE == 2 || p < n;
        const float* xs = xb + na * (int64_t)p;
        if (VEC && TM == 4 && (MODE == 2 || (lane_full && vp))) {
          const f4 v = *(const f4*)xs;
#pragma unroll
          for (int m = 0; m < TM; ++m) xm[m][j] = v[m];
        } else if (VEC && TM == 2 && (MODE == 2 || (lane_full && vp))) {
          const f2 v = *(const f2*)xs;
#pragma unroll
          for (int m = 0; m < TM; ++m) xm[m][j] = v[m];
        } else {
#pragma unroll
          for (int m = 0; m < TM; ++m) xm[m][j] = (vp && arow + m < na) ? xs[m] : 0.f;
        }
      }
#pragma unroll
      for (int u = 0; u < TN; ++u) {
        const int64_t off = (int64_t)(i0 + TN * l + u) * ldp + p0 + 8 * g;
#pragma unroll
        for (int k = 0; k < NP; ++k) bp[u][k] = *(const bf8*)(PH + k * plane + off);
      }
    };
    auto cmp = [&](const f8 (&xm)[TM], const bf8 (&bp)[TN][NP]) {
      bf8 ap[TM][NP];
#pragma unroll
      for (int m = 0; m < TM; ++m) split_bf16<NP>(xm[m], ap[m]);
#pragma unroll
      for (int m = 0; m < TM; ++m)
#pragma unroll
        for (int u = 0; u < TN; ++u) mfma_split<NP>(ap[m], bp[u], sc, acc[m][u], accs[m][u]);
    };
    f8 x0[TM], x1[TM];
    bf8 q0[TN][NP], q1[TN][NP];
    ldc(0, x0, q0);
    int p0 = 0;
    for (; p0 + 32 < n; p0 += 64) {
      ldc(p0 + 32, x1, q1);
      __builtin_amdgcn_sched_barrier(0);
      cmp(x0, q0);
      ldc(p0 + 64 < n ? p0 + 64 : p0, x0, q0);   // the last one re-reads a valid chunk
      __builtin_amdgcn_sched_barrier(0);
      cmp(x1, q1);
    }
    if (p0 < n) cmp(x0, q0);
#pragma unroll
    for (int m = 0; m < TM; ++m)
#pragma unroll
      for (int u = 0; u < TN; ++u) acct[m][u] += sc * accs[m][u];
  }
  TOut* __restrict__ Y = (TOut*)jb.Y;
  const double* __restrict__ base = (const double*)jb.base;
  const int64_t ar = a0 + 4 * TM * g;
#pragma unroll
  for (int u = 0; u < TN; ++u) {
    const int i = i0 + TN * l + u;
    if (i >= n) continue;
    float v[4 * TM];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int m = 0; m < TM; ++m) v[TM * r + m] = acc[m][u][r] + acct[m][u][r];
    store_run<TOut>(Y, base, slab + na * (int64_t)i + ar, v, 4 * TM, (int)(na - ar < 4 * TM ? na - ar : 4 * TM),
                    VEC);
  }
}

int finish_tiles_lp(ModeJobs& J, bool mode1, int TM, int TN) {
  const int64_t tot = assign_tiles(J.job, J.njobs, mode1, TM, TN);
  J.total_tiles = tot;
  J.tiles_per_job = J.njobs > 0 ? tot / J.njobs : 0;
  for (int j = 0; j < J.njobs; ++j)
    if (J.job[j].tile_begin != (int64_t)j * J.tiles_per_job) J.tiles_per_job = 0;
  return SETD_OK;
}

bool aligned_lp(const void* p, uintptr_t a) { return ((uintptr_t)p % a) == 0; }

// bf16 wave tiles (rows x columns of 16): 4 x 4 on the interior path (one
// wave per SIMD; swept at 3D FHN 256^3: BF16x3 113 steps/s against 97 for
// 4 x 2 / 2 x 4 and 78 for 2 x 4 / 2 x 2), smaller ones on the masked paths,
// whose larger register needs would spill at 4 x 4.
constexpr int kTM1 = 4, kTN1 = 4;     // mode 1, interior
constexpr int kTM1s = 4, kTN1s = 2;   // mode 1, masked
constexpr int kTMB = 4, kTNB = 4;     // modes >= 2, interior
constexpr int kTMBs = 2, kTNBs = 2;   // modes >= 2, masked

}  // namespace

namespace {

template <int MODE, typename T>
void go_mode1(int prec, dim3 grid, hipStream_t s, const ModeJobs& J, int64_t per) {
  constexpr int TM = MODE == 2 ? kTM1 : kTM1s, TN = MODE == 2 ? kTN1 : kTN1s;
  if (prec == SETD_PREC_BF16X3)
    hipLaunchKernelGGL((mode1_bf16_kernel<3, TM, TN, MODE, T>), grid, dim3(64), 0, s, J, per);
  else
    hipLaunchKernelGGL((mode1_bf16_kernel<2, TM, TN, MODE, T>), grid, dim3(64), 0, s, J, per);
}

template <int MODE, typename T>
void go_modeB(int prec, dim3 grid, hipStream_t s, const ModeJobs& J, int64_t per) {
  constexpr int TM = MODE == 2 ? kTMB : kTMBs, TN = MODE == 2 ? kTNB : kTNBs;
  if (prec == SETD_PREC_BF16X3)
    hipLaunchKernelGGL((modeB_bf16_kernel<3, TM, TN, MODE, T>), grid, dim3(64), 0, s, J, per);
  else
    hipLaunchKernelGGL((modeB_bf16_kernel<2, TM, TN, MODE, T>), grid, dim3(64), 0, s, J, per);
}

template <typename T>
void go_mode1_m(int mode, int prec, dim3 grid, hipStream_t s, const ModeJobs& J, int64_t per) {
  if (mode == 2) go_mode1<2, T>(prec, grid, s, J, per);
  else if (mode == 1) go_mode1<1, T>(prec, grid, s, J, per);
  else go_mode1<0, T>(prec, grid, s, J, per);
}

template <typename T>
void go_modeB_m(int mode, int prec, dim3 grid, hipStream_t s, const ModeJobs& J, int64_t per) {
  if (mode == 2) go_modeB<2, T>(prec, grid, s, J, per);
  else if (mode == 1) go_modeB<1, T>(prec, grid, s, J, per);
  else go_modeB<0, T>(prec, grid, s, J, per);
}

}  // namespace

namespace {

// FP32 tile shapes: defaults from a sweep at 3D FHN 256^3 (mode 1 4 x 4,
// modes >= 2 4 x 4: 96 TFLOP/s; 4 x 2 / 4 x 2: 90), overridable with
// SETD_TILE_F32_MODE1 / SETD_TILE_F32_MODEB ("4x2" etc.).
void f32_tile(const char* name, int& tm, int& tn) {
  const char* e = std::getenv(name);
  int a = 0, b = 0;
  if (e && std::sscanf(e, "%dx%d", &a, &b) == 2 && (a == 2 || a == 4) && (b == 2 || b == 4)) {
    tm = a;
    tn = b;
  }
}

#define SETD_F32C(KERNEL, TM_, TN_)                                                                  \
  if (tm == TM_ && tn == TN_) {                                                                     \
    if (mode == 2)                                                                                  \
      hipLaunchKernelGGL((KERNEL<TM_, TN_, 2, T>), grid, dim3(64), 0, s, J, per);                    \
    else if (mode == 1)                                                                             \
      hipLaunchKernelGGL((KERNEL<TM_, TN_, 1, T>), grid, dim3(64), 0, s, J, per);                    \
    else                                                                                            \
      hipLaunchKernelGGL((KERNEL<TM_, TN_, 0, T>), grid, dim3(64), 0, s, J, per);                    \
    return;                                                                                         \
  }

template <typename T>
void go_mode1_f32c(int tm, int tn, int mode, dim3 grid, hipStream_t s, const ModeJobs& J, int64_t per) {
  SETD_F32C(mode1_f32c_kernel, 4, 4)
  SETD_F32C(mode1_f32c_kernel, 4, 2)
  SETD_F32C(mode1_f32c_kernel, 2, 4)
  SETD_F32C(mode1_f32c_kernel, 2, 2)
}
template <typename T>
void go_modeB_f32c(int tm, int tn, int mode, dim3 grid, hipStream_t s, const ModeJobs& J, int64_t per) {
  SETD_F32C(modeB_f32c_kernel, 4, 4)
  SETD_F32C(modeB_f32c_kernel, 4, 2)
  SETD_F32C(modeB_f32c_kernel, 2, 4)
  SETD_F32C(modeB_f32c_kernel, 2, 2)
}

int launch_mode1_f32c(ModeJobs& J, DType out, hipStream_t s) {
  int tm = 4, tn = 4;
  f32_tile("SETD_TILE_F32_MODE1", tm, tn);
  finish_tiles_lp(J, true, tm, tn);
  if (J.total_tiles == 0) return SETD_OK;
  bool vec = true, interior = true;
  for (int j = 0; j < J.njobs; ++j) {
    const ModeJob& jb = J.job[j];
    vec = vec && (jb.n % 4 == 0) && aligned_lp(jb.X[0], 16) && aligned_lp(jb.Y, 16) && aligned_lp(jb.base, 16);
    interior = interior && jb.n % 32 == 0 && jb.nb % (16 * tn) == 0;
  }
  const int mode = vec ? (interior ? 2 : 1) : 0;
  double fl = 0.0, by = 0.0;
  if (prof_on()) job_work(J, 4, out == DType::F64 ? 8 : 4, 4, fl, by);
  ProfScope prof(s, kProfMode1LP, fl, by);
  bool lds = mode == 2 && tm == 4 && tn == 4;
  for (int j = 0; j < J.njobs; ++j)
    lds = lds && J.job[j].n >= kLds32MinN && J.job[j].n <= kLds32MaxN && J.job[j].n % 64 == 0;
  if (lds) {   // workgroups: per job tiles_i panels x column groups of 8 * reps tiles
    const int reps = kLds32Reps;
    int64_t tot = 0;
    for (int j = 0; j < J.njobs; ++j) {
      ModeJob& jb = J.job[j];
      jb.tile_begin = tot;
      tot += (int64_t)jb.tiles_i * ceil_div(jb.tiles_a, kLds32Waves * reps);
    }
    J.total_tiles = tot;
    J.tiles_per_job = J.njobs > 0 ? tot / J.njobs : 0;
    for (int j = 0; j < J.njobs; ++j)
      if (J.job[j].tile_begin != (int64_t)j * J.tiles_per_job) J.tiles_per_job = 0;
    const int64_t per = ceil_div(tot, 8);
    if (out == DType::F32)
      hipLaunchKernelGGL(mode1_lds32_kernel<float>, dim3((unsigned)(per * 8)), dim3(64 * kLds32Waves), 0, s, J, per,
                         reps);
    else
      hipLaunchKernelGGL(mode1_lds32_kernel<double>, dim3((unsigned)(per * 8)), dim3(64 * kLds32Waves), 0, s, J, per,
                         reps);
    SETD_LAUNCHED();
    return SETD_OK;
  }
  const int64_t per = ceil_div(J.total_tiles, 8);
  const dim3 grid((unsigned)(per * 8));
  if (out == DType::F32) go_mode1_f32c<float>(tm, tn, mode, grid, s, J, per);
  else go_mode1_f32c<double>(tm, tn, mode, grid, s, J, per);
  SETD_LAUNCHED();
  return SETD_OK;
}

int launch_modeB_f32c(ModeJobs& J, DType out, hipStream_t s) {
  int tm = 4, tn = 4;
  f32_tile("SETD_TILE_F32_MODEB", tm, tn);
  finish_tiles_lp(J, false, tm, tn);
  if (J.total_tiles == 0) return SETD_OK;
  bool vec = true, interior = true;
  for (int j = 0; j < J.njobs; ++j) {
    const ModeJob& jb = J.job[j];
    vec = vec && (jb.na % 4 == 0) && aligned_lp(jb.Y, 16) && aligned_lp(jb.base, 16);
    for (int t = 0; t < jb.nterms; ++t) vec = vec && aligned_lp(jb.X[t], 16);
    interior = interior && jb.n % 32 == 0 && jb.na % (16 * tm) == 0;
  }
  const int mode = vec ? (interior ? 2 : 1) : 0;
  double fl = 0.0, by = 0.0;
  if (prof_on()) job_work(J, 4, out == DType::F64 ? 8 : 4, 4, fl, by);
  ProfScope prof(s, kProfModeBLP, fl, by);
  const int64_t per = ceil_div(J.total_tiles, 8);
  const dim3 grid((unsigned)(per * 8));
  if (out == DType::F32) go_modeB_f32c<float>(tm, tn, mode, grid, s, J, per);
  else go_modeB_f32c<double>(tm, tn, mode, grid, s, J, per);
  SETD_LAUNCHED();
  return SETD_OK;
}

}  // namespace

int launch_mode1_lp(ModeJobs& J, int prec, DType out, hipStream_t s) {
  if (prec == SETD_PREC_F32) return launch_mode1_f32c(J, out, s);
  bool vec = true, interior = true;
  for (int j = 0; j < J.njobs; ++j) {
    const ModeJob& jb = J.job[j];
    vec = vec && (jb.n % 8 == 0) && aligned_lp(jb.X[0], 32) && aligned_lp(jb.Y, 16) && aligned_lp(jb.base, 16);
    interior = interior && jb.n % 32 == 0 && jb.nb % (16 * kTN1) == 0;
  }
  const int mode = vec ? (interior ? 2 : 1) : 0;
  if (mode == 2) finish_tiles_lp(J, true, kTM1, kTN1);
  else finish_tiles_lp(J, true, kTM1s, kTN1s);
  if (J.total_tiles == 0) return SETD_OK;
  double fl = 0.0, by = 0.0;
  if (prof_on()) job_work(J, 4, out == DType::F64 ? 8 : 4, 4, fl, by);
  ProfScope prof(s, kProfMode1LP, fl, by);
  const int64_t per = ceil_div(J.total_tiles, 8);
  const dim3 grid((unsigned)(per * 8));
  if (out == DType::F32) go_mode1_m<float>(mode, prec, grid, s, J, per);
  else go_mode1_m<double>(mode, prec, grid, s, J, per);
  SETD_LAUNCHED();
  return SETD_OK;
}

int launch_modeB_lp(ModeJobs& J, int prec, DType out, hipStream_t s) {
  if (prec == SETD_PREC_F32) return launch_modeB_f32c(J, out, s);
  bool vec = true, interior = true;
  for (int j = 0; j < J.njobs; ++j) {
    const ModeJob& jb = J.job[j];
    vec = vec && (jb.na % 4 == 0) && aligned_lp(jb.Y, 16) && aligned_lp(jb.base, 16);
    for (int t = 0; t < jb.nterms; ++t) vec = vec && aligned_lp(jb.X[t], 16);
    interior = interior && jb.n % 32 == 0 && jb.na % (16 * kTMB) == 0;
  }
  const int mode = vec ? (interior ? 2 : 1) : 0;
  if (mode == 2) finish_tiles_lp(J, false, kTMB, kTNB);
  else finish_tiles_lp(J, false, kTMBs, kTNBs);
  if (J.total_tiles == 0) return SETD_OK;
  double fl = 0.0, by = 0.0;
  if (prof_on()) job_work(J, 4, out == DType::F64 ? 8 : 4, 4, fl, by);
  ProfScope prof(s, kProfModeBLP, fl, by);
  const int64_t per = ceil_div(J.total_tiles, 8);
  const dim3 grid((unsigned)(per * 8));
  if (out == DType::F32) go_modeB_m<float>(mode, prec, grid, s, J, per);
  else go_modeB_m<double>(mode, prec, grid, s, J, per);
  SETD_LAUNCHED();
  return SETD_OK;
}

}  // namespace setd
