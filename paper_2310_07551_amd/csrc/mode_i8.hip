// FP64 mu-mode products on the int8 matrix cores by error-free slicing
// (the Ozaki scheme of Ozaki, Ogita, Oishi and Rump, 2012, in the integer
// form of Ootomo, Ozaki and Yokota, 2024): SETD_PREC_I8X4.
//
// Each operand vector of the contraction -- a row of the phi matrix, a fibre
// of the tensor along the contracted mode -- is written relative to its own
// power of two 2^E (|x| < 2^E for every entry) as a 30-bit integer
//     q = rint(x 2^(30 - E)) = t3 2^24 + t2 2^16 + t1 2^8 + t0,
// with four signed 8-bit digits t_k (t3 in [-64, 64],
// the others in [-128, 127]).  A product of two entries is then
//     2^(Ex + Ep - 60) sum_{a, b} t^x_a t^p_b 2^(8 (a + b)),
// and the pairs with a + b >= 2 (thirteen of the sixteen; the other three
// weigh at most 2^-44 of |x|max |p|max) are summed over the whole contraction
// on the int8 matrix cores in int32, one accumulator per order a + b, with no
// rounding at all (|sum| <= 4 n 2^14 < 2^31 for n <= 4096).  The five
// accumulators of an output are combined in FP64 and scaled by
// 2^(Ex + Ep - 12).  The error is the rounding of each operand to 30 bits of
// its vector's largest entry: at most 2^-30 of |x|max |p|max per product
// term (unbiased), whatever the cancellation in the sum.
// This is what the reduced-precision forms of FP32 matrix-core arithmetic
// cannot give on the 3D FitzHugh-Nagumo workload, whose F = K u + g is about
// 1e5 times the step's result: their FP32 partial sums round at the scale of
// the terms.
//
// Operands: the phi matrices are sliced once when packed (four int8 planes,
// row-major, plus each row's exponent); the tensor operand is FP64 and is
// sliced in the kernel, once per workgroup: a workgroup owns 32 tensor
// columns and up to 256 matrix rows (eight waves of 32 rows, two per SIMD, so
// one wave's loads overlap the other's products).  Each thread loads 16
// values of one column at once; the block finds every column's
// exponent (phase 1), writes the columns' digit planes to LDS (phase 2), from
// where every wave feeds them to v_mfma_i32_16x16x64_i8 against its own rows'
// planes, the next 64-long step's matrix digits loading while the current
// step's products run (phase 3).
// Contractions longer than 256 take the columns 256 values at a time, the
// exponent pass reading them once before.  Inputs, intermediates and outputs
// stay FP64.
//
// Lane layout (probed on gfx950): lane (g, l) supplies row l of A and column
// l of B at 16 k-slots (g, j); both operands use k = 16 g + j of the current
// 64-long k-step, and register r of lane (g, l) holds D[4 g + r][l].
#include <cstdint>

#include "common.hpp"

namespace setd {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kCols = 32;               // tensor columns per workgroup
constexpr int kWaves = 8;               // waves per workgroup (two per SIMD)
constexpr int kThreads = 64 * kWaves;
constexpr int kTM = 2;                  // 16-row blocks per wave
constexpr int kWaveRows = 16 * kTM;
constexpr int kRows = kWaves * kWaveRows;   // matrix rows per workgroup (256)
constexpr int kChunk = 256;             // contraction values staged in LDS at a time
constexpr int kLdsRow = kChunk + 16;    // bytes per (digit plane, column); +16 spreads the lanes over the banks
constexpr int kBits = 30;
constexpr int kVals = kCols * kChunk / kThreads;   // chunk values per thread in phases 1 and 2 (16)
constexpr int kParts = kChunk / kVals;              // threads per column (16)
constexpr int kBadExp = 1 << 14;        // marks a vector with a non-finite entry (its outputs become NaN)

__device__ __forceinline__ v4i mfma_i8(const v4i& a, const v4i& b, const v4i& c) {
  return __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c, 0, 0, 0);
}

// E with |x| < 2^E for every |x| <= m (m finite, >= 0); 0 for m == 0.
__device__ __forceinline__ int exp_above(double m) {
  int e = 0;
  if (m > 0.0) (void)frexp(m, &e);
  return e;
}

// The four digits of x (|x| < 2^E) as the bytes of one word, t0 lowest:
// w = q + 0x808080 has bytes b0, b1, b2 (unsigned) and a signed top byte
// with q = sum_{k<3} (b_k - 128) 2^(8k) + t3 2^24; b_k - 128 as a signed
// byte is b_k ^ 0x80.
__device__ __forceinline__ uint32_t digit_word(double x, int E) {
  const int q = (int)rint(ldexp(x, kBits - E));   // |q| <= 2^30
  return (uint32_t)(q + 0x00808080) ^ 0x00808080u;
}

// 4 x 4 byte transpose: d[k] gathers byte k of w0..w3 (digit plane k of four
// consecutive values).  v_perm_b32 selects bytes of {S0, S1}, S1 as bytes 0-3.
__device__ __forceinline__ void digit_planes(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3, uint32_t (&d)[4]) {
  const uint32_t lo01 = __builtin_amdgcn_perm(w1, w0, 0x05010400u);   // w0.b0 w1.b0 w0.b1 w1.b1
  const uint32_t hi01 = __builtin_amdgcn_perm(w1, w0, 0x07030602u);   // w0.b2 w1.b2 w0.b3 w1.b3
  const uint32_t lo23 = __builtin_amdgcn_perm(w3, w2, 0x05010400u);
  const uint32_t hi23 = __builtin_amdgcn_perm(w3, w2, 0x07030602u);
  d[0] = __builtin_amdgcn_perm(lo23, lo01, 0x05040100u);
  d[1] = __builtin_amdgcn_perm(lo23, lo01, 0x07060302u);
  d[2] = __builtin_amdgcn_perm(hi23, hi01, 0x05040100u);
  d[3] = __builtin_amdgcn_perm(hi23, hi01, 0x07060302u);
}

// ---- packing of the matrix operand ----
// out: ldp rows of 4 ldp bytes, then ldp int32 row exponents.  Row i holds,
// for every run of 16 contraction indices, the 16 bytes of digit t0, then of
// t1, t2 and t3 (64 bytes): a lane's four digit operands of one k-step are
// one 64-byte block.  One 256-thread block per row.
__global__ void __launch_bounds__(256) pack_i8_kernel(const double* __restrict__ M, int n, int ldp, double scale,
                                                       uint8_t* __restrict__ out) {
  const int i = blockIdx.x;
  __shared__ double red[4];
  double m = 0.0;
  bool bad = false;
  if (i < n)
    for (int p = threadIdx.x; p < n; p += 256) {
      const double v = scale * M[i + (int64_t)n * p];
      bad = bad || !isfinite(v);
      m = fmax(m, fabs(v));
    }
  if (bad) m = __builtin_inf();
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  const bool finite = isfinite(m);
  const int E = finite ? exp_above(m) : kBadExp;
  uint8_t* row = out + (int64_t)i * 4 * ldp;
  for (int p = threadIdx.x; p < ldp; p += 256) {
    const double v = (i < n && p < n && finite) ? scale * M[i + (int64_t)n * p] : 0.0;
    const uint32_t w = finite ? digit_word(v, E) : 0u;
#pragma unroll
    for (int k = 0; k < 4; ++k) row[(p >> 4) * 64 + 16 * k + (p & 15)] = (uint8_t)(w >> (8 * k));
  }
  if (threadIdx.x == 0) ((int*)(out + (int64_t)4 * ldp * ldp))[i] = E;
}

__device__ __forceinline__ int64_t remap_xcd_i8(int64_t bid, int64_t per_xcd) {
  return (bid & 7) * per_xcd + (bid >> 3);
}

// One workgroup (8 waves, two per SIMD): rows row0 .. row0+255 of every
// term's matrix (32 per wave), 32 tensor columns.  MODE1: column b holds
// X[p + n b] (contiguous); otherwise column (a, b) holds X[a + na p + na n b].
// Y = base + sum_t scale_t (P_t X_t).
template <bool MODE1>
__global__ void __launch_bounds__(kThreads, 1) mode_i8_kernel(const ModeJobs J, int64_t per_xcd) {
  const int64_t t = remap_xcd_i8(blockIdx.x, per_xcd);
  if (t >= J.total_tiles) return;   // uniform over the block
  const ModeJob& jb = J.job[find_job(J, t)];
  const int64_t lt = t - jb.tile_begin;
  const int it = (int)(lt % jb.tiles_i);
  const int64_t rest = lt / jb.tiles_i;
  const int n = jb.n, ldp = jb.ldp;
  const int64_t na = jb.na, nb = jb.nb;
  const int64_t ct = MODE1 ? rest : rest % jb.tiles_a;   // column tile
  const int64_t bslab = MODE1 ? 0 : rest / jb.tiles_a;   // b of the column tile (modes >= 2)
  const int64_t c0 = ct * kCols;                          // first b (mode 1) or a (modes >= 2)
  const int64_t ncols = MODE1 ? nb : na;
  const int64_t slab = MODE1 ? 0 : na * (int64_t)n * bslab;
  const int row0 = it * kRows;

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g = lane >> 4, l = lane & 15;
  const int wrow = row0 + kWaveRows * wave;   // this wave's first row
  __shared__ __attribute__((aligned(16))) uint8_t lds[4 * kCols * kLdsRow];
  __shared__ double red[kParts][kCols];
  __shared__ int colexp[kCols];
  // the raw chunk: kVals contiguous values per thread role, rows padded by
  // 16 bytes so that neighbouring lanes use different banks
  constexpr int kRawRow = kVals + 2;
  __shared__ __attribute__((aligned(16))) double raw[kThreads * kRawRow];
  // rows of this wave exist (ldp and the row split are multiples of 32)
  const bool active = wrow < n;
  const int64_t plane = (int64_t)ldp * ldp;

  // Thread roles of phases 1 and 2: column pc, its values kc + kVals ps ..
  // +kVals-1.  MODE1 gives a column kParts neighbouring lanes (each a
  // contiguous run); otherwise 32 lanes read 32 neighbouring columns at one k.
  const int pc = MODE1 ? (tid / kParts) : (tid % kCols);
  const int ps = MODE1 ? (tid % kParts) : (tid / kCols);
  const int64_t cc_p = c0 + pc;
  const bool col_ok = cc_p < ncols;
  const bool vec = MODE1 && (n % 2 == 0);   // 16-byte loads of a column (n even: aligned)
  auto load_vals = [&](const double* __restrict__ X, int kc, double (&v)[kVals]) {
    const int k0 = kc + kVals * ps;
    if (MODE1) {
      const double* src = X + k0 + (int64_t)n * (col_ok ? cc_p : 0);
      if (vec && col_ok && k0 + kVals <= n) {
#pragma unroll
        for (int j = 0; j < kVals; j += 2) {
          const d2 w = *(const d2*)(src + j);
          v[j] = w[0];
          v[j + 1] = w[1];
        }
      } else {
#pragma unroll
        for (int j = 0; j < kVals; ++j) v[j] = (col_ok && k0 + j < n) ? src[j] : 0.0;
      }
    } else {
      const double* src = X + (col_ok ? cc_p : 0) + slab + na * (int64_t)k0;
#pragma unroll
      for (int j = 0; j < kVals; ++j) {
        v[j] = (col_ok && k0 + j < n) ? *src : 0.0;
        src += na;
      }
    }
  };
  // writes the digit planes of v to LDS (column pc, chunk offset kVals ps)
  auto split_vals = [&](const double (&v)[kVals], int E) {
    const bool ok = E != kBadExp;
    uint8_t* dst = lds + pc * kLdsRow + kVals * ps;
#pragma unroll
    for (int j = 0; j < kVals; j += 4) {
      uint32_t w[4], d[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) w[q] = ok ? digit_word(v[j + q], E) : 0u;
      digit_planes(w[0], w[1], w[2], w[3], d);
#pragma unroll
      for (int k = 0; k < 4; ++k) *(uint32_t*)(dst + k * kCols * kLdsRow + j) = d[k];
    }
  };

  double out[kTM][2][4];
#pragma unroll
  for (int m = 0; m < kTM; ++m)
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) out[m][u][r] = 0.0;

  for (int term = 0; term < jb.nterms; ++term) {
    const double* __restrict__ X = (const double*)jb.X[term];
    const uint8_t* __restrict__ P = (const uint8_t*)jb.P[term];
    const int* __restrict__ Pexp = (const int*)(P + 4 * plane);   // after the ldp rows of 4 ldp bytes
    const double sc = jb.scale[term];
    const bool one_chunk = n <= kChunk;

    // phase 1: exponent of every column (a one-chunk contraction keeps its
    // values in LDS for phase 2)
    double* myraw = raw + tid * kRawRow;
    __syncthreads();   // the previous term's readers of colexp / lds / raw are done
    {
      double m = 0.0, z = 0.0;   // z = sum of 0 * v: NaN iff some value is not finite
      for (int kc = 0; kc < n; kc += kChunk) {
        double v[kVals];
        load_vals(X, kc, v);
#pragma unroll
        for (int j = 0; j < kVals; ++j) {
          z = fma(0.0, v[j], z);
          m = fmax(m, fabs(v[j]));
        }
        if (one_chunk) {
#pragma unroll
          for (int j = 0; j < kVals; j += 2) *(d2*)(myraw + j) = d2{v[j], v[j + 1]};
        }
      }
      red[ps][pc] = z != z ? __builtin_inf() : m;
    }
    __syncthreads();
    if (tid < kCols) {
      double m = red[0][tid];
      for (int q = 1; q < kParts; ++q) m = fmax(m, red[q][tid]);
      colexp[tid] = isfinite(m) ? exp_above(m) : kBadExp;
    }

    v4i acc[5][kTM][2];   // [order a + b - 2][row block][column block]
#pragma unroll
    for (int o = 0; o < 5; ++o)
#pragma unroll
      for (int m = 0; m < kTM; ++m)
#pragma unroll
        for (int u = 0; u < 2; ++u) acc[o][m][u] = v4i{0, 0, 0, 0};

    for (int kc = 0; kc < n; kc += kChunk) {
      __syncthreads();   // colexp written; the previous chunk's readers are done
      // phase 2: digit planes of this chunk
      {
        double v[kVals];
        if (one_chunk) {
#pragma unroll
          for (int j = 0; j < kVals; j += 2) {
            const d2 w = *(const d2*)(myraw + j);
            v[j] = w[0];
            v[j + 1] = w[1];
          }
        } else {
          load_vals(X, kc, v);
        }
        split_vals(v, colexp[pc]);
      }
      __syncthreads();
      // phase 3: this wave's rows against the 32 columns, 64 k per step; the
      // next step's matrix digits load while this step's products run
      if (active) {
        const uint8_t* prow = P + (int64_t)(wrow + l) * 4 * ldp + (kc / 16 + g) * 64;
        const int64_t mstride = (int64_t)16 * 4 * ldp;
        const int kend = n - kc < kChunk ? n - kc : kChunk;
        auto load_a = [&](int k64, v4i (&a)[kTM][4]) {
#pragma unroll
          for (int m = 0; m < kTM; ++m) {
            const uint8_t* q = prow + m * mstride + 4 * k64;
#pragma unroll
            for (int s2 = 0; s2 < 4; ++s2) a[m][s2] = *(const v4i*)(q + 16 * s2);
          }
        };
        v4i acur[kTM][4], anext[kTM][4];
        load_a(0, acur);
#pragma unroll
        for (int k64 = 0; k64 < kChunk; k64 += 64) {
          if (k64 >= kend) break;
          if (k64 + 64 < kend) load_a(k64 + 64, anext);
          v4i b[2][4];
#pragma unroll
          for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int s2 = 0; s2 < 4; ++s2)
              b[u][s2] = *(const v4i*)(lds + (s2 * kCols + 16 * u + l) * kLdsRow + k64 + 16 * g);
#pragma unroll
          for (int m = 0; m < kTM; ++m)
#pragma unroll
            for (int u = 0; u < 2; ++u) {
              const v4i* a = acur[m];
              // matrix digit pb (first operand), tensor digit pa, order pa + pb >= 2
              acc[4][m][u] = mfma_i8(a[3], b[u][3], acc[4][m][u]);
              acc[3][m][u] = mfma_i8(a[3], b[u][2], acc[3][m][u]);
              acc[3][m][u] = mfma_i8(a[2], b[u][3], acc[3][m][u]);
              acc[2][m][u] = mfma_i8(a[3], b[u][1], acc[2][m][u]);
              acc[2][m][u] = mfma_i8(a[2], b[u][2], acc[2][m][u]);
              acc[2][m][u] = mfma_i8(a[1], b[u][3], acc[2][m][u]);
              acc[1][m][u] = mfma_i8(a[3], b[u][0], acc[1][m][u]);
              acc[1][m][u] = mfma_i8(a[2], b[u][1], acc[1][m][u]);
              acc[1][m][u] = mfma_i8(a[1], b[u][2], acc[1][m][u]);
              acc[1][m][u] = mfma_i8(a[0], b[u][3], acc[1][m][u]);
              acc[0][m][u] = mfma_i8(a[2], b[u][0], acc[0][m][u]);
              acc[0][m][u] = mfma_i8(a[1], b[u][1], acc[0][m][u]);
              acc[0][m][u] = mfma_i8(a[0], b[u][2], acc[0][m][u]);
            }
          if (k64 + 64 < kend) {
#pragma unroll
            for (int m = 0; m < kTM; ++m)
#pragma unroll
              for (int s2 = 0; s2 < 4; ++s2) acur[m][s2] = anext[m][s2];
          }
        }
      }
    }
    // this term's products:
    // 2^(Ex + Ep - 12) (acc6 + acc5 2^-8 + acc4 2^-16 + acc3 2^-24 + acc2 2^-32)
    if (active) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int ex = colexp[16 * u + l];
#pragma unroll
        for (int m = 0; m < kTM; ++m)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int ep = Pexp[wrow + 16 * m + 4 * g + r];
            double w = (double)acc[0][m][u][r] * 0x1p-32;
            w = fma((double)acc[1][m][u][r], 0x1p-24, w);
            w = fma((double)acc[2][m][u][r], 0x1p-16, w);
            w = fma((double)acc[3][m][u][r], 0x1p-8, w);
            w += (double)acc[4][m][u][r];
            w = (ex == kBadExp || ep == kBadExp) ? __builtin_nan("") : ldexp(w, ex + ep - 12);
            out[m][u][r] = fma(sc, w, out[m][u][r]);
          }
      }
    }
  }
  if (!active) return;   // no barrier follows
  double* __restrict__ Y = (double*)jb.Y;
  const double* __restrict__ base = (const double*)jb.base;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int64_t cc = c0 + 16 * u + l;
    if (cc >= ncols) continue;
#pragma unroll
    for (int m = 0; m < kTM; ++m)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = wrow + 16 * m + 4 * g + r;
        if (i >= n) continue;
        const int64_t o = MODE1 ? i + (int64_t)n * cc : cc + na * (int64_t)i + slab;
        Y[o] = base ? base[o] + out[m][u][r] : out[m][u][r];
      }
  }
}

}  // namespace

size_t packed_bytes_i8(int n) {
  const size_t ldp = (size_t)packed_ld(n);
  return 4 * ldp * ldp + 4 * ldp;
}

int pack_matrix_i8(const double* M, int n, double scale, void* out, hipStream_t s) {
  const int ldp = packed_ld(n);
  hipLaunchKernelGGL(pack_i8_kernel, dim3((unsigned)ldp), dim3(256), 0, s, M, n, ldp, scale, (uint8_t*)out);
  SETD_LAUNCHED();
  return SETD_OK;
}

int launch_mode_i8(ModeJobs& J, bool mode1, hipStream_t s) {
  int64_t tot = 0;
  for (int j = 0; j < J.njobs; ++j) {
    ModeJob& jb = J.job[j];
    jb.tiles_i = (int)ceil_div(jb.n, kRows);
    jb.tiles_a = (int)ceil_div(mode1 ? jb.nb : jb.na, kCols);
    jb.tile_begin = tot;
    tot += (int64_t)jb.tiles_i * jb.tiles_a * (mode1 ? 1 : jb.nb);
  }
  J.total_tiles = tot;
  J.tiles_per_job = J.njobs > 0 ? tot / J.njobs : 0;
  for (int j = 0; j < J.njobs; ++j)
    if (J.job[j].tile_begin != (int64_t)j * J.tiles_per_job) J.tiles_per_job = 0;
  if (tot == 0) return SETD_OK;
  double fl = 0.0, by = 0.0;
  if (prof_on()) job_work(J, 8, 8, 4, fl, by);
  ProfScope prof(s, mode1 ? kProfMode1LP : kProfModeBLP, fl, by);
  const int64_t per = ceil_div(tot, 8);
  const dim3 grid((unsigned)(per * 8));
  if (mode1)
    hipLaunchKernelGGL(mode_i8_kernel<true>, grid, dim3(kThreads), 0, s, J, per);
  else
    hipLaunchKernelGGL(mode_i8_kernel<false>, grid, dim3(kThreads), 0, s, J, per);
  SETD_LAUNCHED();
  return SETD_OK;
}

}  // namespace setd
