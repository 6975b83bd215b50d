// FP64 mu-mode products on the CDNA4 matrix cores (v_mfma_f64_16x16x4_f64).
//
// A mu-mode product S = T x_mu L (Section 2) applies L to every mu-fiber:
// with a = (i_1..i_{mu-1}) flattened (stride 1), i = i_mu and b =
// (i_{mu+1}..i_d) flattened,
//
//     Y[a, i, b] = sum_p L[i, p] X[a, p, b].
//
// Two kernels cover every mode:
//   * mode 1 (no a index): Y = L X as a GEMM over the column-major unfolding
//     X_(1) (n x N/n), no copy.  MFMA rows = i, columns = b, k = p.  The
//     contraction index is the contiguous one, so each lane loads four
//     consecutive p of one column (32 bytes) and uses them over four MFMA
//     k-steps; the matrix is packed row-major (L[i, p] at i*ldp + p) to match.
//   * modes >= 2: for each b, Y[:, :, b] = X[:, :, b] L^T with a contiguous.
//     MFMA rows = a, columns = i, k = p.  Each lane loads TM consecutive a
//     (one row of every row tile) and TN consecutive i of the column-major
//     packed matrix, so every global access is a contiguous 16-32 byte run
//     and a 16-lane group covers a full 128-byte line or more.
//
// Register tiling: a wave owns a (16 TM) x (16 TN) output tile held in
// TM x TN MFMA accumulators; rows of the tile are interleaved (lane row m of
// row-tile t is a0 + TM m + t) so the per-lane loads and the epilogue stores
// are contiguous.  The next k-chunk is loaded into registers while the
// current one feeds the MFMAs.
//
// Each launch runs a table of independent jobs (up to kMaxJobs outputs; each
// may sum up to kMaxTerms inputs along the contraction, which is how the
// terms of a split phi action are accumulated into one output), one wave per
// workgroup, with the block index remapped so that each XCD gets a contiguous
// range of tiles (neighbouring tiles share X or L in that XCD's L2).
#include "common.hpp"

#include <algorithm>
#include <cstdlib>

namespace setd {

__device__ __forceinline__ int64_t remap_xcd(int64_t bid, int64_t per_xcd) {
  return (bid & 7) * per_xcd + (bid >> 3);
}

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// mode 1
// ---------------------------------------------------------------------------
// One wave computes tile `lt` of job `jb`.
template <int TM, int TN, int MODE>
__device__ __forceinline__ void mode1_tile(const ModeJob& jb, int64_t lt) {
  // MODE 0: element loads with bounds checks everywhere; 1: vector loads
  // (aligned operands); 2: additionally every tile interior and n % 32 == 0.
  constexpr bool VEC = MODE >= 1;
  const int it = (int)(lt % jb.tiles_i);
  const int64_t bt = lt / jb.tiles_i;

  const int lane = threadIdx.x, g = lane >> 4, l = lane & 15;
  const int n = jb.n, ldp = jb.ldp;
  const int64_t nb = jb.nb;
  const int i0 = it * 16 * TM;
  const int64_t b0 = bt * 16 * TN;
  const double* __restrict__ X = (const double*)jb.X[0];
  const double* __restrict__ PT = (const double*)jb.P[0];
  const double sc = jb.scale[0];

  // Lanes of group g hold KP consecutive p of each chunk of 4 KP (KP = 2 on
  // the interior path, whose two-deep register ring must fit beside the
  // accumulators in the two-wave budget; 4 elsewhere).
  constexpr int KP = MODE == 2 ? 2 : 4;
  const double* pa[TM];
#pragma unroll
  for (int m = 0; m < TM; ++m) pa[m] = PT + (int64_t)(i0 + TM * l + m) * ldp + KP * g;
  const double* pb[TN];
  bool vb[TN];
#pragma unroll
  for (int u = 0; u < TN; ++u) {
    const int64_t b = b0 + 16 * u + l;
    vb[u] = b < nb;
    pb[u] = X + (vb[u] ? b : 0) * (int64_t)n + KP * g;
  }

  d4 acc[TM][TN];
#pragma unroll
  for (int m = 0; m < TM; ++m)
#pragma unroll
    for (int u = 0; u < TN; ++u) acc[m][u] = d4{0.0, 0.0, 0.0, 0.0};

  // The scale multiplies the operand where it is used, never inside a load:
  // a multiply right after a prefetch would make the wave wait for it.
  auto mma = [&](const d4* ar, const d4* br) {
#pragma unroll
    for (int jj = 0; jj < 4; ++jj)
#pragma unroll
      for (int m = 0; m < TM; ++m) {
        const double av = ar[m][jj] * sc;
#pragma unroll
        for (int u = 0; u < TN; ++u) acc[m][u] = mfma(av, br[u][jj], acc[m][u]);
      }
  };
  if constexpr (MODE == 2) {
    // Interior tile: chunks of 8 p (two k-steps) in a two-deep register ring,
    // no masks and no register copies; each chunk is loaded a whole chunk of
    // MFMAs before its use.  The last loads re-read a valid chunk instead of
    // branching.
    auto load = [&](int p0, d2* ar, d2* br) {
#pragma unroll
      for (int m = 0; m < TM; ++m) ar[m] = *(const d2*)(pa[m] + p0);
#pragma unroll
      for (int u = 0; u < TN; ++u) br[u] = *(const d2*)(pb[u] + p0);
    };
    auto mma2 = [&](const d2* ar, const d2* br) {
#pragma unroll
      for (int jj = 0; jj < 2; ++jj)
#pragma unroll
        for (int m = 0; m < TM; ++m)
#pragma unroll
          for (int u = 0; u < TN; ++u) acc[m][u] = mfma(ar[m][jj], br[u][jj], acc[m][u]);
    };
    d2 a0[TM], b0r[TN], a1[TM], b1r[TN];
    load(0, a0, b0r);
    load(8, a1, b1r);
    for (int p0 = 0; p0 < n; p0 += 16) {
      mma2(a0, b0r);
      load(p0 + 16 < n ? p0 + 16 : p0, a0, b0r);
      mma2(a1, b1r);
      load(p0 + 24 < n ? p0 + 24 : p0 + 8, a1, b1r);
    }
  } else {
    auto load = [&](int p0, d4* ar, d4* br) {
#pragma unroll
      for (int m = 0; m < TM; ++m) ar[m] = *(const d4*)(pa[m] + p0);
      const bool full = VEC && (p0 + 16 <= n);
#pragma unroll
      for (int u = 0; u < TN; ++u) {
        if (full) {
          br[u] = vb[u] ? *(const d4*)(pb[u] + p0) : d4{0.0, 0.0, 0.0, 0.0};
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            br[u][e] = (vb[u] && p0 + 4 * g + e < n) ? pb[u][p0 + e] : 0.0;
        }
      }
    };
    d4 a[TM], bx[TN];
    load(0, a, bx);
    for (int p0 = 0; p0 < n; p0 += 16) {
      d4 an[TM], bn[TN];
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

  // Epilogue.  The FP64 16x16 accumulator holds tile row 4 r + g in register
  // r of lane (g, l), column l; tile row q of row-tile m is output row
  // i0 + TM q + m.  So lane (g, l) owns, for each r, the TM consecutive rows
  // i0 + TM g + 4 TM r + (0..TM-1) of column b0 + 16 u + l.
  // The interior path leaves the scale to the epilogue.
  const double osc = MODE == 2 ? sc : 1.0;
  double* __restrict__ Y = (double*)jb.Y;
  const double* __restrict__ base = (const double*)jb.base;
#pragma unroll
  for (int u = 0; u < TN; ++u) {
    if (!vb[u]) continue;
    const int64_t col = (b0 + 16 * u + l) * (int64_t)n;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ir = i0 + TM * g + 4 * TM * r;
      if (VEC && ir + TM <= n) {
#pragma unroll
        for (int m = 0; m < TM; m += 2) {
          d2 w = d2{acc[m][u][r], acc[m + 1][u][r]} * osc;
          if (base) w += *(const d2*)(base + col + ir + m);
          *(d2*)(Y + col + ir + m) = w;
        }
      } else {
#pragma unroll
        for (int m = 0; m < TM; ++m) {
          if (ir + m < n) {
            double w = acc[m][u][r] * osc;
            if (base) w += base[col + ir + m];
            Y[col + ir + m] = w;
          }
        }
      }
    }
  }
}

// Mode 1 with the matrix panel in LDS (interior jobs, 192 <= n <= 256,
// 4 x 4 tiles).  A workgroup of 8 waves shares one 64-row panel of P, stored
// in LDS in the order the MFMA reads it (chunk of 16 p, row m, lane: 4 p),
// so no wave holds P in registers; each wave then computes `reps` 64 x 64
// tiles of the workgroup's column group (8 * reps column tiles), reading X
// in 32-byte runs per lane (whole cache lines) through a two-deep ring.
// Workgroup w of a job: panel w % tiles_i, column group w / tiles_i.
constexpr int kLdsWaves = 8;
constexpr int kLdsMinN = 192, kLdsMaxN = 256;
// Tiles per wave: 4 measured best at FHN 256^3 (mode 1 at 64.8 TFLOP/s
// against 63.0 with 2, 52.3 with 6 and 58.2 for the register-only kernel);
// below n = 192 the register-only kernel is faster (the panel fill weighs
// more against a shorter contraction).
constexpr int kLdsReps = 4;

__global__ void __launch_bounds__(512, 1) mode1_lds_kernel(const ModeJobs J, int64_t per_xcd, int reps) {
  __shared__ d4 panel[(kLdsMaxN / 16) * 4 * 64];   // 128 KB
  const int64_t w = remap_xcd(blockIdx.x, per_xcd);
  if (w >= J.total_tiles) return;   // uniform over the workgroup
  const int j = find_job(J, w);
  const ModeJob& jb = J.job[j];
  const int64_t lw = w - jb.tile_begin;
  const int it = (int)(lw % jb.tiles_i);
  const int64_t bg = lw / jb.tiles_i;
  const int n = jb.n, ldp = jb.ldp;
  const int nchunk = n / 16;
  const int i0 = it * 64;
  const double* __restrict__ PT = (const double*)jb.P[0];
  // fill: entry q = (c * 4 + m) * 64 + lane holds P[i0 + 4 l + m][16 c + 4 g + 0..3]
  for (int q = threadIdx.x; q < nchunk * 256; q += 512) {
    const int ln = q & 63, m = (q >> 6) & 3, c = q >> 8;
    const int l = ln & 15, g = ln >> 4;
    panel[q] = *(const d4*)(PT + (int64_t)(i0 + 4 * l + m) * ldp + 16 * c + 4 * g);
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6;
  for (int rep = 0; rep < reps; ++rep) {
  const int64_t bt = (bg * reps + rep) * kLdsWaves + wave;
  if (bt >= jb.tiles_a) return;
  const int lane = threadIdx.x & 63, g = lane >> 4, l = lane & 15;
  const int64_t b0 = bt * 64;
  const double* __restrict__ X = (const double*)jb.X[0];
  const double* pb[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) pb[u] = X + (b0 + 16 * u + l) * (int64_t)n + 4 * g;
  d4 acc[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[m][u] = d4{0.0, 0.0, 0.0, 0.0};
  auto load = [&](int c, d4* xr) {
#pragma unroll
    for (int u = 0; u < 4; ++u) xr[u] = *(const d4*)(pb[u] + 16 * c);
  };
  auto mma = [&](int c, const d4* xr) {
    d4 a[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) a[m] = panel[(c * 4 + m) * 64 + lane];
#pragma unroll
    for (int jj = 0; jj < 4; ++jj)
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[m][u] = mfma(a[m][jj], xr[u][jj], acc[m][u]);
  };
  d4 x0[4], x1[4];
  load(0, x0);
  for (int c = 0; c < nchunk; c += 2) {
    load(c + 1, x1);                                 // nchunk is even (n % 32 == 0)
    mma(c, x0);
    load(c + 2 < nchunk ? c + 2 : c, x0);
    mma(c + 1, x1);
  }
  // epilogue as in mode1_tile: lane (g, l) owns rows i0 + 4 g + 16 r + (0..3)
  // of column b0 + 16 u + l
  const double sc = jb.scale[0];
  double* __restrict__ Y = (double*)jb.Y;
  const double* __restrict__ base = (const double*)jb.base;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t col = (b0 + 16 * u + l) * (int64_t)n;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ir = i0 + 4 * g + 16 * r;
      if (ir + 4 <= n) {
#pragma unroll
        for (int m = 0; m < 4; m += 2) {
          d2 v = d2{acc[m][u][r], acc[m + 1][u][r]} * sc;
          if (base) v += *(const d2*)(base + col + ir + m);
          *(d2*)(Y + col + ir + m) = v;
        }
      } else {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          if (ir + m < n) {
            double v = acc[m][u][r] * sc;
            if (base) v += base[col + ir + m];
            Y[col + ir + m] = v;
          }
        }
      }
    }
  }
  }
}

// Job table in the kernel arguments (up to kMaxJobs outputs per launch).
// Two waves per SIMD is the target occupancy: with that register budget the
// accumulators stay in place through the k loop (a tighter default made the
// compiler copy all of them between register files every iteration).
template <int TM, int TN, int MODE>
__global__ void __launch_bounds__(64, 2) mode1_f64_kernel(const ModeJobs J, int64_t per_xcd) {
  const int64_t t = remap_xcd(blockIdx.x, per_xcd);
  if (t >= J.total_tiles) return;
  const int j = find_job(J, t);
  mode1_tile<TM, TN, MODE>(J.job[j], t - J.job[j].tile_begin);
}

// Work list in device memory (any number of jobs, e.g. many independent
// instances): a persistent grid walks the logical tiles with a stride that
// keeps every block on its XCD's contiguous range.
template <int TM, int TN, int MODE>
__global__ void __launch_bounds__(64, 2) mode1_f64_list_kernel(const ModeJob* __restrict__ jobs,
                                                            const int64_t* __restrict__ begins, int njobs,
                                                            int64_t total, int64_t per_xcd) {
  for (int64_t raw = blockIdx.x; raw < 8 * per_xcd; raw += gridDim.x) {
    const int64_t t = remap_xcd(raw, per_xcd);
    if (t >= total) continue;
    const int j = find_job_list(begins, njobs, t);
    mode1_tile<TM, TN, MODE>(jobs[j], t - jobs[j].tile_begin);
  }
}

// ---------------------------------------------------------------------------
// modes >= 2
// ---------------------------------------------------------------------------
template <int TM, int TN, int MODE>
__device__ __forceinline__ void modeB_tile(const ModeJob& jb, int64_t lt) {
  constexpr bool VEC = MODE >= 1;   // as in the mode-1 kernel
  const int it = (int)(lt % jb.tiles_i);
  const int64_t rest = lt / jb.tiles_i;
  const int64_t at = rest % jb.tiles_a;
  const int64_t b = rest / jb.tiles_a;

  const int lane = threadIdx.x, g = lane >> 4, l = lane & 15;
  const int n = jb.n, ldp = jb.ldp, nterms = jb.nterms;
  const int64_t na = jb.na;
  const int64_t a0 = at * 16 * TM;
  const int i0 = it * 16 * TN;
  const int64_t arow = a0 + TM * l;                 // first of this lane's TM rows
  const bool lane_full = arow + TM <= na;

  d4 acc[TM][TN];
#pragma unroll
  for (int m = 0; m < TM; ++m)
#pragma unroll
    for (int u = 0; u < TN; ++u) acc[m][u] = d4{0.0, 0.0, 0.0, 0.0};

  const int64_t slab = na * (int64_t)n * b;
  constexpr bool fast = MODE == 2;   // every tile interior, n % 32 == 0 (checked at launch)
  __builtin_amdgcn_s_setprio(1);   // products ahead of another wave's epilogue on the SIMD
  for (int term = 0; term < nterms; ++term) {
    const double* __restrict__ xb = (const double*)jb.X[term] + slab + arow + na * g;
    const double* __restrict__ pbp = (const double*)jb.P[term] + i0 + TN * l + (int64_t)ldp * g;
    const double sc = jb.scale[term];

    if constexpr (fast) {
      // Interior tile: blocks of KB k-steps (4 KB values of p) in ping-pong
      // registers; the scale is applied to the matrix operand at use.  A
      // 4 x 4 tile takes blocks of 2, so that its ring fits beside the 128
      // accumulator registers at two waves per SIMD.
      constexpr int KB = (TM == 4 && TN == 4) ? 2 : 4;
      auto loadblk = [&](int p0, double (*xr)[TM], double (*pr)[TN]) {
#pragma unroll
        for (int k = 0; k < KB; ++k) {
          const double* xs = xb + na * (int64_t)(p0 + 4 * k);
          if constexpr (TM == 4) {
            const d4 v = *(const d4*)xs;
#pragma unroll
            for (int m = 0; m < TM; ++m) xr[k][m] = v[m];
          } else {
            const d2 v = *(const d2*)xs;
#pragma unroll
            for (int m = 0; m < TM; ++m) xr[k][m] = v[m];
          }
          const double* ps = pbp + (int64_t)ldp * (p0 + 4 * k);
          if constexpr (TN == 4) {
            const d4 v = *(const d4*)ps;
#pragma unroll
            for (int u = 0; u < TN; ++u) pr[k][u] = v[u];
          } else {
            const d2 v = *(const d2*)ps;
#pragma unroll
            for (int u = 0; u < TN; ++u) pr[k][u] = v[u];
          }
        }
      };
      auto mmablk = [&](double (*xr)[TM], double (*pr)[TN]) {
#pragma unroll
        for (int k = 0; k < KB; ++k)
#pragma unroll
          for (int u = 0; u < TN; ++u) {
            const double pv = pr[k][u] * sc;
#pragma unroll
            for (int m = 0; m < TM; ++m) acc[m][u] = mfma(xr[k][m], pv, acc[m][u]);
          }
      };
      double xa[KB][TM], pa[KB][TN], xq[KB][TM], pq[KB][TN];
      loadblk(0, xa, pa);
      for (int p0 = 0; p0 < n; p0 += 8 * KB) {
        loadblk(p0 + 4 * KB, xq, pq);
        mmablk(xa, pa);
        loadblk(p0 + 8 * KB < n ? p0 + 8 * KB : p0, xa, pa);
        mmablk(xq, pq);
      }
      continue;
    }

    auto load = [&](int p0, double* xr, double* pr) {
      const bool vp = p0 + g < n;
      const double* xs = xb + na * (int64_t)p0;
      if (VEC && TM == 4 && lane_full && vp) {
        const d4 v = *(const d4*)xs;
#pragma unroll
        for (int m = 0; m < TM; ++m) xr[m] = v[m];
      } else if (VEC && TM == 2 && lane_full && vp) {
        const d2 v = *(const d2*)xs;
#pragma unroll
        for (int m = 0; m < TM; ++m) xr[m] = v[m];
      } else {
#pragma unroll
        for (int m = 0; m < TM; ++m) xr[m] = (vp && arow + m < na) ? xs[m] : 0.0;
      }
      const double* ps = pbp + (int64_t)ldp * p0;
      if (TN == 4) {
        const d4 v = *(const d4*)ps;
#pragma unroll
        for (int u = 0; u < TN; ++u) pr[u] = v[u];
      } else if (TN == 2) {
        const d2 v = *(const d2*)ps;
#pragma unroll
        for (int u = 0; u < TN; ++u) pr[u] = v[u];
      } else {
#pragma unroll
        for (int u = 0; u < TN; ++u) pr[u] = ps[u];
      }
    };

    double xr[TM], pr[TN];
    load(0, xr, pr);
    for (int p0 = 0; p0 < n; p0 += 4) {
      double xn[TM], pn[TN];
      const bool more = p0 + 4 < n;
      if (more) load(p0 + 4, xn, pn);
#pragma unroll
      for (int u = 0; u < TN; ++u) {
        const double pv = pr[u] * sc;
#pragma unroll
        for (int m = 0; m < TM; ++m) acc[m][u] = mfma(xr[m], pv, acc[m][u]);
      }
      if (more) {
#pragma unroll
        for (int m = 0; m < TM; ++m) xr[m] = xn[m];
#pragma unroll
        for (int u = 0; u < TN; ++u) pr[u] = pn[u];
      }
    }
  }

  __builtin_amdgcn_s_setprio(0);
  // Epilogue (accumulator layout as in the mode-1 kernel): lane (g, l) owns,
  // for each r, the TM consecutive a = a0 + TM g + 4 TM r + (0..TM-1) of
  // column i = i0 + TN l + u.
  double* __restrict__ Y = (double*)jb.Y;
  const double* __restrict__ base = (const double*)jb.base;
#pragma unroll
  for (int u = 0; u < TN; ++u) {
    const int i = i0 + TN * l + u;
    if (i >= n) continue;
    const int64_t off = slab + na * (int64_t)i;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t ar = a0 + TM * g + 4 * TM * r;
      if (VEC && ar + TM <= na) {
#pragma unroll
        for (int m = 0; m < TM; m += 2) {
          d2 w = d2{acc[m][u][r], acc[m + 1][u][r]};
          if (base) w += *(const d2*)(base + off + ar + m);
          *(d2*)(Y + off + ar + m) = w;
        }
      } else {
#pragma unroll
        for (int m = 0; m < TM; ++m) {
          if (ar + m < na) {
            double w = acc[m][u][r];
            if (base) w += base[off + ar + m];
            Y[off + ar + m] = w;
          }
        }
      }
    }
  }
}

// Modes >= 2 with the matrix panel in LDS (interior single-term jobs,
// 192 <= n <= 256, n % 64 == 0, 4 x 4 tiles).  A workgroup of 8 waves shares
// one 64-column panel of P (times the job's scale), stored in LDS in the
// order the MFMA reads it (k-step, lane: 4 columns); each wave computes
// `reps` 64 a x 64 i tiles of the workgroup's group of (a-block, slab) pairs,
// reading X in 32-byte runs per lane through a two-deep ring of 4-k-step
// blocks.  (Multi-term jobs stay on the register kernel: refilling the panel
// for every term cost more than it saved.)
// Workgroup w of a job: panel w % tiles_i, group w / tiles_i of 8 * reps
// (a-block, slab) pairs, pair q = a-block q % tiles_a, slab q / tiles_a.
__global__ void __launch_bounds__(512, 1) modeB_lds_kernel(const ModeJobs J, int64_t per_xcd, int reps) {
  __shared__ d4 panel[(kLdsMaxN / 4) * 64];   // 128 KB
  const int64_t w = remap_xcd(blockIdx.x, per_xcd);
  if (w >= J.total_tiles) return;   // uniform over the workgroup
  const ModeJob& jb = J.job[find_job(J, w)];
  const int64_t lw = w - jb.tile_begin;
  const int it = (int)(lw % jb.tiles_i);
  const int64_t grp = lw / jb.tiles_i;
  const int n = jb.n, ldp = jb.ldp;
  const int64_t na = jb.na;
  const int64_t npairs = (int64_t)jb.tiles_a * jb.nb;
  const int i0 = it * 64;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, l = lane & 15;
  // fill: entry q = kk * 64 + lane' holds sc * P[i0 + 4 l' + 0..3][4 kk + g']
  {
    const double* __restrict__ P = (const double*)jb.P[0];
    const double sc = jb.scale[0];
    for (int q = threadIdx.x; q < (n / 4) * 64; q += 512) {
      const int ln = q & 63, kk = q >> 6;
      panel[q] = *(const d4*)(P + i0 + 4 * (ln & 15) + (int64_t)ldp * (4 * kk + (ln >> 4))) * sc;
    }
  }
  __syncthreads();
  constexpr int KB = 4;
  const double* __restrict__ X = (const double*)jb.X[0];
  // (a-block, slab) pair of repetition r (past the job's pairs: not run), and
  // the lane's first X element of it
  auto pair_of = [&](int r) { return (grp * reps + r) * kLdsWaves + wave; };
  auto xbase = [&](int64_t q) {
    const int64_t at = q % jb.tiles_a, b = q / jb.tiles_a;
    return X + na * (int64_t)n * b + at * 64 + 4 * l + na * g;
  };
  auto loadblk = [&](const double* xb, int p0, d4* xr) {
#pragma unroll
    for (int k = 0; k < KB; ++k) xr[k] = *(const d4*)(xb + na * (int64_t)(p0 + 4 * k));
  };
  d4 xa[KB], xq[KB];
  if (pair_of(0) >= npairs) return;   // no barrier follows
  const double* xb = xbase(pair_of(0));
  loadblk(xb, 0, xa);
  for (int rep = 0; rep < reps; ++rep) {
    const int64_t q = pair_of(rep);
    // the next pair's first block is loaded during this pair's last one
    const bool next = rep + 1 < reps && pair_of(rep + 1) < npairs;
    const double* xn = next ? xbase(pair_of(rep + 1)) : xb;
    __builtin_amdgcn_s_setprio(1);   // products ahead of another wave's epilogue on the SIMD
    const int64_t at = q % jb.tiles_a, b = q / jb.tiles_a;
    const int64_t a0 = at * 64;
    const int64_t slab = na * (int64_t)n * b;
    d4 acc[4][4];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[m][u] = d4{0.0, 0.0, 0.0, 0.0};
    {
      auto mmablk = [&](int p0, const d4* xr) {
#pragma unroll
        for (int k = 0; k < KB; ++k) {
          const d4 pv = panel[(p0 / 4 + k) * 64 + lane];
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int m = 0; m < 4; ++m) acc[m][u] = mfma(xr[k][m], pv[u], acc[m][u]);
        }
      };
      for (int p0 = 0; p0 < n; p0 += 8 * KB) {   // n % 32 == 0
        loadblk(xb, p0 + 4 * KB, xq);
        mmablk(p0, xa);
        const bool last = p0 + 8 * KB >= n;
        loadblk(last ? xn : xb + na * (int64_t)(p0 + 8 * KB), 0, xa);   // unconditional: no branch
        mmablk(p0 + 4 * KB, xq);
      }
    }
    __builtin_amdgcn_s_setprio(0);
    // epilogue as in modeB_tile (TM = TN = 4, every row and column in range)
    double* __restrict__ Y = (double*)jb.Y;
    const double* __restrict__ base = (const double*)jb.base;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t off = slab + na * (int64_t)(i0 + 4 * l + u);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t ar = a0 + 4 * g + 16 * r;
#pragma unroll
        for (int m = 0; m < 4; m += 2) {
          d2 v = d2{acc[m][u][r], acc[m + 1][u][r]};
          if (base) v += *(const d2*)(base + off + ar + m);
          *(d2*)(Y + off + ar + m) = v;
        }
      }
    }
    if (!next) return;
    xb = xn;
  }
}

// Two waves per SIMD, as for mode 1 (with it the 4 x 4 tile fits in 232
// registers).
template <int TM, int TN, int MODE>
__global__ void __launch_bounds__(64, 2) modeB_f64_kernel(const ModeJobs J, int64_t per_xcd) {
  const int64_t t = remap_xcd(blockIdx.x, per_xcd);
  if (t >= J.total_tiles) return;
  const int j = find_job(J, t);
  modeB_tile<TM, TN, MODE>(J.job[j], t - J.job[j].tile_begin);
}

template <int TM, int TN, int MODE>
__global__ void __launch_bounds__(64, 2) modeB_f64_list_kernel(const ModeJob* __restrict__ jobs,
                                                            const int64_t* __restrict__ begins, int njobs,
                                                            int64_t total, int64_t per_xcd) {
  for (int64_t raw = blockIdx.x; raw < 8 * per_xcd; raw += gridDim.x) {
    const int64_t t = remap_xcd(raw, per_xcd);
    if (t >= total) continue;
    const int j = find_job_list(begins, njobs, t);
    modeB_tile<TM, TN, MODE>(jobs[j], t - jobs[j].tile_begin);
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int64_t assign_tiles(ModeJob* jobs, int njobs, bool mode1, int TM, int TN) {
  int64_t tot = 0;
  for (int j = 0; j < njobs; ++j) {
    ModeJob& jb = jobs[j];
    if (mode1) {
      jb.tiles_i = (int)ceil_div(jb.n, 16 * TM);
      jb.tiles_a = (int)ceil_div(jb.nb, 16 * TN);     // tiles along b
    } else {
      jb.tiles_i = (int)ceil_div(jb.n, 16 * TN);
      jb.tiles_a = (int)ceil_div(jb.na, 16 * TM);
    }
    jb.tile_begin = tot;
    tot += (int64_t)jb.tiles_i * jb.tiles_a * (mode1 ? 1 : jb.nb);
  }
  return tot;
}

namespace {
bool aligned(const void* p, uintptr_t a) { return ((uintptr_t)p % a) == 0; }
bool no_interior() {
  static const bool off = std::getenv("SETD_NO_INTERIOR_PATH") != nullptr;
  return off;
}
}  // namespace

int job_mode(const ModeJob& jb, bool mode1, int TM, int TN) {
  bool vec, interior;
  if (mode1) {
    vec = (jb.n % 4 == 0) && aligned(jb.X[0], 32) && aligned(jb.Y, 16) && aligned(jb.base, 16);
    interior = jb.n % 32 == 0 && jb.nb % (16 * TN) == 0;
  } else {
    vec = (jb.na % 4 == 0) && aligned(jb.Y, 16) && aligned(jb.base, 16);
    for (int t = 0; t < jb.nterms; ++t) vec = vec && aligned(jb.X[t], 32);
    interior = jb.n % 32 == 0 && jb.na % (16 * TM) == 0;
  }
  if (!vec) return 0;
  return (interior && !no_interior()) ? 2 : 1;
}

namespace {

struct TileCfg {
  int tm, tn;
};

TileCfg env_tile(const char* name, TileCfg def) {
  const char* s = std::getenv(name);
  if (!s) return def;
  int a = 0, b = 0;
  if (std::sscanf(s, "%dx%d", &a, &b) == 2 && (a == 2 || a == 4) && (b == 2 || b == 4)) return {a, b};
  return def;
}

int finish_tiles(ModeJobs& J, bool mode1, int TM, int TN) {
  J.total_tiles = assign_tiles(J.job, J.njobs, mode1, TM, TN);
  J.tiles_per_job = J.njobs > 0 ? J.total_tiles / J.njobs : 0;
  for (int j = 0; j < J.njobs; ++j)
    if (J.job[j].tile_begin != (int64_t)j * J.tiles_per_job) J.tiles_per_job = 0;
  return SETD_OK;
}

}  // namespace

#define SETD_LAUNCH_MODES(KERNEL, TM_, TN_)                                                    \
  if (cfg.tm == TM_ && cfg.tn == TN_) {                                                       \
    if (mode == 2)                                                                            \
      hipLaunchKernelGGL((KERNEL<TM_, TN_, 2>), grid, dim3(64), 0, s, J, per);                 \
    else if (mode == 1)                                                                       \
      hipLaunchKernelGGL((KERNEL<TM_, TN_, 1>), grid, dim3(64), 0, s, J, per);                 \
    else                                                                                      \
      hipLaunchKernelGGL((KERNEL<TM_, TN_, 0>), grid, dim3(64), 0, s, J, per);                 \
    SETD_LAUNCHED();                                                                          \
    return SETD_OK;                                                                           \
  }

void job_work(const ModeJobs& J, int es_in, int es_out, int es_mat, double& flops, double& bytes) {
  flops = 0.0;
  bytes = 0.0;
  for (int j = 0; j < J.njobs; ++j) {
    const ModeJob& jb = J.job[j];
    const double N = (double)jb.na * jb.n * jb.nb;
    flops += jb.nterms * 2.0 * N * jb.n;
    bytes += jb.nterms * (N * es_in + (double)jb.n * jb.n * es_mat) + N * es_out * (jb.base ? 2.0 : 1.0);
  }
}

int launch_mode1_f64(ModeJobs& J, hipStream_t s) {
  // default from a sweep on MI355X at FHN 256^3 (two waves per SIMD):
  // 4 x 4 53.7, 2 x 4 43.7, 4 x 2 42.2, 2 x 2 34.3 TFLOP/s.  Only the
  // interior variant of the 4 x 4 tile fits the two-wave register budget
  // (its 2-p ring); jobs that need the checked variants take 4 x 2 tiles,
  // which do not spill.
  auto min_mode = [&](int tm, int tn) {
    int m = 2;
    for (int j = 0; j < J.njobs; ++j) m = std::min(m, job_mode(J.job[j], true, tm, tn));
    return m;
  };
  TileCfg def{4, 4};
  if (min_mode(4, 4) < 2) def = TileCfg{4, 2};
  const TileCfg cfg = env_tile("SETD_TILE_MODE1", def);
  finish_tiles(J, true, cfg.tm, cfg.tn);
  if (J.total_tiles == 0) return SETD_OK;
  double fl = 0.0, by = 0.0;
  if (prof_on()) job_work(J, 8, 8, 8, fl, by);
  ProfScope prof(s, kProfMode1F64, fl, by);
  const int mode = min_mode(cfg.tm, cfg.tn);
  bool lds = mode == 2 && cfg.tm == 4 && cfg.tn == 4;
  for (int j = 0; j < J.njobs; ++j)
    lds = lds && J.job[j].n >= kLdsMinN && J.job[j].n <= kLdsMaxN && J.job[j].n % 32 == 0;
  if (lds) {
    // workgroups instead of tiles: per job tiles_i panels x column groups of
    // 8 * reps tiles
    const int reps = kLdsReps;
    int64_t tot = 0;
    for (int j = 0; j < J.njobs; ++j) {
      ModeJob& jb = J.job[j];
      jb.tile_begin = tot;
      tot += (int64_t)jb.tiles_i * ceil_div(jb.tiles_a, kLdsWaves * reps);
    }
    J.total_tiles = tot;
    J.tiles_per_job = J.njobs > 0 ? tot / J.njobs : 0;
    for (int j = 0; j < J.njobs; ++j)
      if (J.job[j].tile_begin != (int64_t)j * J.tiles_per_job) J.tiles_per_job = 0;
    const int64_t per = ceil_div(tot, 8);
    hipLaunchKernelGGL(mode1_lds_kernel, dim3((unsigned)(per * 8)), dim3(64 * kLdsWaves), 0, s, J, per, reps);
    SETD_LAUNCHED();
    return SETD_OK;
  }
  const int64_t per = ceil_div(J.total_tiles, 8);
  const dim3 grid((unsigned)(per * 8));
  SETD_LAUNCH_MODES(mode1_f64_kernel, 4, 4)
  SETD_LAUNCH_MODES(mode1_f64_kernel, 4, 2)
  SETD_LAUNCH_MODES(mode1_f64_kernel, 2, 4)
  SETD_LAUNCH_MODES(mode1_f64_kernel, 2, 2)
  set_error("unsupported mode-1 tile");
  return SETD_EUNSUPPORTED;
}

int launch_modeB_f64(ModeJobs& J, hipStream_t s) {
  // default tiles from sweeps on MI355X: 4 x 4 when every contraction is
  // long (n >= 192; FHN 256^3 last mode 68.4 against 64.2 TFLOP/s for 4 x 2),
  // 4 x 2 otherwise (FHN 128^3: 48.0 against 45.1; fewer, shorter tiles)
  bool long_k = true;
  for (int j = 0; j < J.njobs; ++j) long_k = long_k && J.job[j].n >= kLdsMinN;
  const TileCfg cfg = env_tile("SETD_TILE_MODEB", long_k ? TileCfg{4, 4} : TileCfg{4, 2});
  finish_tiles(J, false, cfg.tm, cfg.tn);
  if (J.total_tiles == 0) return SETD_OK;
  double fl = 0.0, by = 0.0;
  if (prof_on()) job_work(J, 8, 8, 8, fl, by);
  int mode = 2;
  for (int j = 0; j < J.njobs; ++j) mode = std::min(mode, job_mode(J.job[j], false, cfg.tm, cfg.tn));
  bool lds = mode == 2 && cfg.tm == 4;
  for (int j = 0; j < J.njobs; ++j) {
    const ModeJob& jb = J.job[j];
    lds = lds && jb.nterms == 1 && jb.n >= kLdsMinN && jb.n <= kLdsMaxN && jb.n % 64 == 0 && jb.na % 64 == 0;
  }
  // the two kernels are timed as separate classes
  ProfScope prof(s, lds ? kProfModeBPanelF64 : kProfModeBF64, fl, by);
  if (lds) {
    // workgroups: per job n / 64 panels x groups of 8 * reps (a-block, slab)
    // pairs; 4 tiles per wave as in mode 1 (measured at FHN 256^3: the
    // single-term launches go from 62.6 to 65.3 TFLOP/s)
    const int reps = kLdsReps;
    int64_t tot = 0;
    for (int j = 0; j < J.njobs; ++j) {
      ModeJob& jb = J.job[j];
      jb.tiles_i = jb.n / 64;
      jb.tiles_a = (int)(jb.na / 64);
      jb.tile_begin = tot;
      tot += (int64_t)jb.tiles_i * ceil_div((int64_t)jb.tiles_a * jb.nb, (int64_t)kLdsWaves * reps);
    }
    J.total_tiles = tot;
    J.tiles_per_job = J.njobs > 0 ? tot / J.njobs : 0;
    for (int j = 0; j < J.njobs; ++j)
      if (J.job[j].tile_begin != (int64_t)j * J.tiles_per_job) J.tiles_per_job = 0;
    const int64_t per = ceil_div(tot, 8);
    hipLaunchKernelGGL(modeB_lds_kernel, dim3((unsigned)(per * 8)), dim3(64 * kLdsWaves), 0, s, J, per, reps);
    SETD_LAUNCHED();
    return SETD_OK;
  }
  const int64_t per = ceil_div(J.total_tiles, 8);
  const dim3 grid((unsigned)(per * 8));
  SETD_LAUNCH_MODES(modeB_f64_kernel, 4, 4)
  SETD_LAUNCH_MODES(modeB_f64_kernel, 4, 2)
  SETD_LAUNCH_MODES(modeB_f64_kernel, 2, 4)
  SETD_LAUNCH_MODES(modeB_f64_kernel, 2, 2)
  set_error("unsupported mode-b tile");
  return SETD_EUNSUPPORTED;
}

#define SETD_LAUNCH_LIST(KERNEL, TM_, TN_)                                                     \
  if (L.tm == TM_ && L.tn == TN_) {                                                           \
    if (L.mode == 2)                                                                          \
      hipLaunchKernelGGL((KERNEL<TM_, TN_, 2>), grid, dim3(64), 0, s, L.jobs, L.begins, L.njobs, L.total, per); \
    else if (L.mode == 1)                                                                     \
      hipLaunchKernelGGL((KERNEL<TM_, TN_, 1>), grid, dim3(64), 0, s, L.jobs, L.begins, L.njobs, L.total, per); \
    else                                                                                      \
      hipLaunchKernelGGL((KERNEL<TM_, TN_, 0>), grid, dim3(64), 0, s, L.jobs, L.begins, L.njobs, L.total, per); \
    SETD_LAUNCHED();                                                                          \
    return SETD_OK;                                                                           \
  }

int launch_list_f64(const ModeList& L, hipStream_t s) {
  if (L.total == 0) return SETD_OK;
  const int64_t per = ceil_div(L.total, 8);
  // a multiple of 8 blocks, so that block b stays on XCD b % 8 through the
  // whole loop; at most `grid_cap` blocks (0: one block per tile)
  int64_t nblk = per * 8;
  if (L.grid_cap > 0 && nblk > L.grid_cap) nblk = round_up(L.grid_cap, 8);
  const dim3 grid((unsigned)nblk);
  ProfScope prof(s, L.mode1 ? kProfMode1F64 : kProfModeBF64, L.flops, L.bytes);
  if (L.mode1) {
    SETD_LAUNCH_LIST(mode1_f64_list_kernel, 4, 4)
    SETD_LAUNCH_LIST(mode1_f64_list_kernel, 4, 2)
    SETD_LAUNCH_LIST(mode1_f64_list_kernel, 2, 4)
    SETD_LAUNCH_LIST(mode1_f64_list_kernel, 2, 2)
  } else {
    SETD_LAUNCH_LIST(modeB_f64_list_kernel, 4, 4)
    SETD_LAUNCH_LIST(modeB_f64_list_kernel, 4, 2)
    SETD_LAUNCH_LIST(modeB_f64_list_kernel, 2, 4)
    SETD_LAUNCH_LIST(modeB_f64_list_kernel, 2, 2)
  }
  set_error("unsupported tile %dx%d", L.tm, L.tn);
  return SETD_EUNSUPPORTED;
}

}  // namespace setd
