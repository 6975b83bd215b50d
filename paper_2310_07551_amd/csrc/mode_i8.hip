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
// and the pairs with a + b >= 2 (thirteen of the sixteen) are summed over
// the whole contraction on the int8 matrix cores in int32, one accumulator
// per order a + b, with no rounding at all (|sum| <= 4 n 2^14 < 2^31 for
// n <= 4096).  The five accumulators of an output are combined in FP64 and
// scaled by 2^(Ex + Ep - 12).  Per product term the error is the rounding of
// each operand to 30 bits of its vector's largest entry (2^(E - 31) <= 2^-30
// of the vector's largest magnitude, unbiased) plus the three dropped pairs,
// 2^(Ex + Ep - 60) (2^14 + 2 2^22) <= 2^-36 |x|max |p|max: about 2^-29 of
// |x|max |p|max in all, whatever the cancellation in the sum.
// This is what the reduced-precision forms of FP32 matrix-core arithmetic
// cannot give on the 3D FitzHugh-Nagumo workload, whose F = K u + g is about
// 1e5 times the step's result: their FP32 partial sums round at the scale of
// the terms.
//
// Two kernels.  The slicing kernel reads an FP64 tensor operand once and
// writes, for every fibre along the contracted mode, its exponent and its
// four digit planes (4 bytes per entry, zero beyond n), tiled in the order the
// matrix cores read them; it is bound by HBM.  The digit GEMM multiplies the
// phi digits (sliced once when the matrix is packed) with those planes: a
// workgroup of 8 waves (two per SIMD) keeps a 64-row panel of the matrix
// digits in LDS, each wave computes 64-row x 16-column output tiles from it,
// and the workgroup walks a run of column groups as one pipeline with the
// tensor digits of later k-steps in flight.  The FP64 combination runs once
// per output.  Where a workgroup's run holds whole fibres of the next mode's
// operand (mode 1 -> 2 for n2 in {128, 256}; mode 3 -> 1 for n1 in
// {128, 256}, the 3D Tucker then taken in the order 3, 1, 2), the GEMM emits
// that operand's digit planes instead of its FP64 product, so only the inputs
// of a Tucker are sliced.  Inputs, the FP64 combination and outputs are FP64.
//
// Lane layout (probed on gfx950): lane (g, l) supplies row l of A and column
// l of B at 16 k-slots (g, j); both operands use k = 16 g + j of the current
// 64-long k-step, and register r of lane (g, l) holds D[4 g + r][l].
#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "common.hpp"
#include "pointwise.hpp"

namespace setd {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kBits = 30;
constexpr int kBadExp = 1 << 14;        // marks a vector with a non-finite entry (its outputs become NaN)
// slicing kernel: 32 fibres per 256-thread workgroup, 8 threads per fibre,
// each 32 consecutive values of a 256-long chunk
constexpr int kSliceCols = 32;
constexpr int kSliceChunk = 256;
constexpr int kStageRow = 4 * kSliceChunk + 16;   // LDS row of one fibre's digits, padded against bank conflicts
// digit buffer tiles: 16 fibres x one 64-long k-step = 4 planes x 64 lanes x 16 bytes
constexpr int kPlaneBytes = 1024;
constexpr int kTileBytes = 4 * kPlaneBytes;
// digit GEMM: 8 waves x (64 rows x 16 columns); the matrix panel holds 64
// rows x 256 contraction values (4 bytes each), rows padded by 16 bytes so
// that neighbouring lanes read different banks
constexpr int kGemmWaves = 8;
constexpr int kPanelRows = 64;
constexpr int kWaveCols = 16;
constexpr int kGroupCols = kGemmWaves * kWaveCols;   // 128 columns per workgroup
constexpr int kPanelK = 256;
constexpr int kPanelRow = 4 * kPanelK + 16;
constexpr int64_t kCus = 256;
constexpr int64_t kMaxSup = 16;   // longest run of column groups

__device__ __forceinline__ v4i mfma_i8(const v4i& a, const v4i& b, const v4i& c) {
  return __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c, 0, 0, 0);
}

// E with |x| < 2^E for every |x| <= m (m finite, >= 0); 0 for m == 0.
__device__ __forceinline__ int exp_above(double m) {
  int e = 0;
  if (m > 0.0) (void)frexp(m, &e);
  return e;
}

// Magnitude key of x: its high word without the sign.  Over finite values
// the exponent field (key >> 20) grows with |x|; inf and NaN have field 0x7FF.
__device__ __forceinline__ int mag_key(double x) { return __double2hiint(x) & 0x7FFFFFFF; }

// Exponent of a tensor fibre from the largest magnitude key k of its entries:
// the frexp exponent of the largest entry (field - 1022) when that entry is
// normal, -1022 when every entry is zero or subnormal (|x| < 2^-1022), and
// kBadExp when some entry is not finite.  |x| < 2^E for every entry.
__device__ __forceinline__ int fibre_exp(int k) {
  const int f = k >> 20;
  return f == 0x7FF ? kBadExp : (f == 0 ? -1022 : f - 1022);
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

// ---- slicing kernel ----
// Job j: X[0] = FP64 tensor, Y = digit buffer.  MODE1: fibre b holds
// X[p + n b] (p contiguous); otherwise fibre c = a + na b holds
// X[a + na p + na n b].  The buffer is tiled the way the matrix cores read
// it: tile (c / 16, p / 64) of kTileBytes at ((c / 16) (ldp / 64) + p / 64)
// kTileBytes holds digit plane s at s kPlaneBytes, and there the 16 bytes of
// slot 4 (c % 16) + (p / 16) % 4: the digits of values p / 16 16 .. + 15 of
// fibre c.  One load instruction of a wave thus reads 1 KB of contiguous
// memory (lane (g, l) takes slot 4 l + g), and a fibre's 64 values of a plane
// are 64 contiguous bytes, so a product that emits the digits of a few
// fibres writes whole 64-byte sectors.  After the tiles of
// round_up(fibres, 16) fibres: one int32 exponent per fibre.
// A workgroup slices 32 fibres that are consecutive in the digit buffer, 256
// values at a time, each thread 32 values of one fibre.  The digit planes are
// assembled in LDS and leave as whole fibre rows (1 KB per fibre and chunk),
// so every store of a wave covers contiguous memory.  For n <= 256 each value
// is read once: it stays in registers between the maximum and the digits.
// The part of slicing after a thread's values are in registers, for a
// 256-thread workgroup of COLS fibres x 256 / COLS threads of COLS
// consecutive values each (COLS 32: 8 threads x 32 values; COLS 16: 16
// threads x 16 values): the fibre exponents (the largest
// magnitude key over the threads of a fibre, in red and colexp) and, per
// 256-long chunk, the digit planes assembled in LDS and written in tile
// order.  v holds this thread's values of chunk 0; for n > 256 reload(kc)
// refills it.  mk: this thread's largest key over all chunks.  Ends with a
// barrier, so the shared arrays may be reused at once.
template <int COLS, typename Reload>
__device__ __forceinline__ void slice_emit(double (&v)[kSliceChunk * COLS / 256], int mk, int n, int ldp, int nv,
                                           int64_t fib0, int pc, int ps, uint8_t* stage, int (*red)[COLS],
                                           int* colexp, uint8_t* __restrict__ D, int* __restrict__ Dexp,
                                           Reload reload) {
  constexpr int TPF = 256 / COLS;                 // threads per fibre
  constexpr int RUNS = kSliceChunk / (16 * TPF);  // 16-value runs per thread and chunk
  const int tid = threadIdx.x;
  red[ps][pc] = mk;
  __syncthreads();
  if (tid < COLS) {
    int mm = red[0][tid];
    for (int q = 1; q < TPF; ++q) mm = max(mm, red[q][tid]);
    const int e = fibre_exp(mm);
    colexp[tid] = e;
    if (tid < nv) Dexp[fib0 + tid] = e;
  }
  __syncthreads();
  const int E = colexp[pc];
  const bool finite = E != kBadExp;
  for (int kc = 0; kc < ldp; kc += kSliceChunk) {
    if (n > kSliceChunk) reload(kc);   // otherwise v still holds the only chunk
    const int kw = ldp - kc < kSliceChunk ? ldp - kc : kSliceChunk;   // multiple of 64
#pragma unroll
    for (int h = 0; h < RUNS; ++h) {
      const int run = RUNS * ps + h;
      if (16 * run >= kw) break;
      uint32_t d[4][4];   // [group of 4 values][plane]
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        uint32_t w[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const uint32_t x = digit_word(v[16 * h + 4 * q + e], E);   // unconditional: no branch
          w[e] = finite ? x : 0u;
        }
        digit_planes(w[0], w[1], w[2], w[3], d[q]);
      }
      uint8_t* o = stage + pc * kStageRow + 64 * run;
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
        *(v4i*)(o + 16 * sp) = v4i{(int)d[0][sp], (int)d[1][sp], (int)d[2][sp], (int)d[3][sp]};
    }
    __syncthreads();
    // 16-byte units in tile order: (local block of 16 fibres, k-step, plane,
    // slot); unit e = tid + 256 it has slot tid % 64, plane tid / 64 and
    // (block, k-step) = (it / ksc, it % ksc), the latter kept incrementally
    const int nks = ldp / 64, ksc = kw / 64;
    const int ln = tid & 63, sp = tid >> 6;
    for (int it = 0, cbl = 0, ks = 0; it < COLS * kw / 1024; ++it) {
      const int pcw = 16 * cbl + (ln >> 2), gg = ln & 3;
      if (pcw < nv) {
        const int64_t f = fib0 + pcw;
        uint8_t* dst = D + (((f >> 4) * nks + kc / 64 + ks) * 4 + sp) * (int64_t)kPlaneBytes + 16 * (4 * (f & 15) + gg);
        *(v4i*)dst = *(const v4i*)(stage + pcw * kStageRow + 64 * (4 * ks + gg) + 16 * sp);
      }
      if (++ks == ksc) {
        ks = 0;
        ++cbl;
      }
    }
    __syncthreads();   // the stage is rewritten by the next chunk
  }
}

template <bool MODE1>
__global__ void __launch_bounds__(256) slice_i8_kernel(const ModeJobs J, int64_t per_xcd) {
  __shared__ __attribute__((aligned(16))) uint8_t stage[kSliceCols * kStageRow];
  __shared__ int red[8][kSliceCols];
  __shared__ int colexp[kSliceCols];
  const int64_t t = remap_xcd_i8(blockIdx.x, per_xcd);
  if (t >= J.total_tiles) return;   // uniform over the block
  const ModeJob& jb = J.job[find_job(J, t)];
  const int64_t lt = t - jb.tile_begin;
  const int n = jb.n, ldp = jb.ldp;
  const int64_t na = jb.na, nb = jb.nb;
  const int64_t nfib = MODE1 ? nb : na;   // fibres per slab
  const int64_t ct = MODE1 ? lt : lt % jb.tiles_a;
  const int64_t bslab = MODE1 ? 0 : lt / jb.tiles_a;
  const int tid = threadIdx.x;
  const int pc = MODE1 ? (tid >> 3) : (tid & 31);   // fibre of this thread
  const int ps = MODE1 ? (tid & 7) : (tid >> 5);    // its 32-value block of a chunk
  const int64_t fa0 = ct * kSliceCols;
  const int nv = (int)(nfib - fa0 < kSliceCols ? nfib - fa0 : kSliceCols);   // fibres of this workgroup
  const bool ok = pc < nv;
  const int64_t fa = fa0 + (ok ? pc : 0);
  const double* __restrict__ X = (const double*)jb.X[0];
  const double* src = MODE1 ? X + (int64_t)n * fa : X + fa + na * (int64_t)n * bslab;
  const int64_t step = MODE1 ? 1 : na;
  const int64_t fib0 = MODE1 ? fa0 : fa0 + na * bslab;
  const int64_t ntot = MODE1 ? nb : na * nb;
  uint8_t* __restrict__ D = (uint8_t*)jb.Y;
  int* __restrict__ Dexp = (int*)(D + ((ntot + 15) & ~(int64_t)15) * 4 * (int64_t)ldp);
  double v[32];
  // modes >= 2, a whole chunk of 32 fibres: value j of every thread at a
  // workgroup-uniform address plus a 32-bit lane offset (no per-value address
  // arithmetic, no branches); otherwise clamped addresses and a select
  const bool whole = !MODE1 && nv == kSliceCols && na <= ((int64_t)1 << 21);
  const uint32_t lane_off = (uint32_t)((pc + na * 32 * ps) * 8);
  auto load = [&](int kc) {
    const int k0 = kc + 32 * ps;
    if (MODE1 && ok && (n % 2 == 0) && k0 + 32 <= n) {
#pragma unroll
      for (int j = 0; j < 32; j += 2) {
        const d2 w = *(const d2*)(src + k0 + j);
        v[j] = w[0];
        v[j + 1] = w[1];
      }
    } else if (whole && kc + kSliceChunk <= n) {
      const char* ub = (const char*)(X + fa0 + na * (int64_t)n * bslab + na * (int64_t)kc);
#pragma unroll
      for (int j = 0; j < 32; ++j) v[j] = *(const double*)(ub + na * 8 * j + lane_off);
    } else {
#pragma unroll
      for (int j = 0; j < 32; ++j) {
        const bool in = ok && k0 + j < n;
        const double x = src[step * (in ? k0 + j : 0)];
        v[j] = in ? x : 0.0;
      }
    }
  };
  // the fibre's largest magnitude key
  int mk = 0;
  for (int kc = 0; kc < n; kc += kSliceChunk) {
    load(kc);
#pragma unroll
    for (int j = 0; j < 32; ++j) mk = max(mk, mag_key(v[j]));
  }
  slice_emit<kSliceCols>(v, mk, n, ldp, nv, fib0, pc, ps, stage, red, colexp, D, Dexp, load);
}

// ---- stage difference and its digits in one pass ----
// D_c = g_c(U_s) - G_c for both components (the stage difference of
// Algorithm 2, formed as the stage kernel forms it), cut straight into the
// digits of its fibres along the last of d modes: fibre a holds the n values
// a + na p (na = N / n), the layout the slicing kernel writes for modes >= 2
// with one slab, into D[c].  The FP64 difference never reaches memory.
// n <= 256.  A 256-thread workgroup takes 16 fibres, 16 threads per fibre and
// 16 consecutive values per thread (the slicing kernel's 32 x 8 x 32 shape
// would hold 4 x 32 operands per thread here).
template <int KIND>
__global__ void __launch_bounds__(256) stage_slice_i8_kernel(const double* __restrict__ Us,
                                                             const double* __restrict__ G, int ncomp, int64_t N,
                                                             int64_t na, int n, int ldp, GParams gp, uint8_t* D0,
                                                             uint8_t* D1, int64_t per_xcd) {
  constexpr int COLS = 16, VPT = 16;   // 16 fibres x 16 threads x 16 values
  __shared__ __attribute__((aligned(16))) uint8_t stage[COLS * kStageRow];
  __shared__ int red[256 / COLS][COLS];
  __shared__ int colexp[COLS];
  const int64_t t = remap_xcd_i8(blockIdx.x, per_xcd);
  if (t * COLS >= na) return;   // uniform over the block
  const int tid = threadIdx.x, pc = tid & (COLS - 1), ps = tid / COLS;
  const int64_t fa0 = t * COLS;
  const int nv = (int)(na - fa0 < COLS ? na - fa0 : COLS);
  const bool ok = pc < nv;
  const int64_t fa = fa0 + (ok ? pc : 0);
  const int64_t coff = ncomp > 1 ? N : 0;   // the second component (a harmless re-read with one)
  const int k0 = VPT * ps;
  double v0[VPT], v1[VPT];
  int m0 = 0, m1 = 0;
  // the 64 loads unconditional (clamped to a valid point) and in flight together
  double uu[VPT], ww[VPT], ga[VPT], gb[VPT];
#pragma unroll
  for (int j = 0; j < VPT; ++j) {
    const bool in = ok && k0 + j < n;
    const int64_t idx = fa + na * (in ? k0 + j : 0);
    uu[j] = Us[idx];
    ww[j] = Us[coff + idx];
    ga[j] = G[idx];
    gb[j] = G[coff + idx];
  }
#pragma unroll
  for (int j = 0; j < VPT; ++j) {
    const bool in = ok && k0 + j < n;
    double g0, g1;
    reaction_of<KIND>(gp, uu[j], ncomp > 1 ? ww[j] : 0.0, g0, g1);
    v0[j] = in ? g0 - ga[j] : 0.0;
    v1[j] = in && ncomp > 1 ? g1 - gb[j] : 0.0;
    m0 = max(m0, mag_key(v0[j]));
    m1 = max(m1, mag_key(v1[j]));
  }
  const int64_t ntot16 = (na + 15) & ~(int64_t)15;
  auto none = [](int) {};
  slice_emit<COLS>(v0, m0, n, ldp, nv, fa0, pc, ps, stage, red, colexp, D0, (int*)(D0 + ntot16 * 4 * (int64_t)ldp),
                   none);
  if (ncomp > 1)
    slice_emit<COLS>(v1, m1, n, ldp, nv, fa0, pc, ps, stage, red, colexp, D1,
                     (int*)(D1 + ntot16 * 4 * (int64_t)ldp), none);
}

// ---- digit GEMM ----
// Job j: X[t] = digit buffer of term t (slicing kernel layout), P[t] = packed
// matrix digits, Y = base + sum_t scale_t P_t X_t.  A workgroup owns row
// panel `it` (64 rows) and a run of `sup` consecutive column groups of 128
// (for modes >= 2 the groups of all slabs in order, tiles_a per slab).  It
// walks the items (group, term, 256-chunk of the contraction) of its run as
// one software pipeline: the tensor digits of the next k-step are always in
// flight, across item and group boundaries, and when the next item needs
// another matrix panel (several terms, or n > 256) that panel is fetched
// during the current item into the second LDS buffer (SWAP; the host picks
// it when some job has several terms or n > 256).  Without SWAP the panel is
// loaded once and the loop has no barrier at all.
// FUSE: 0 = FP64 outputs; 1 = the next mode's digits, any shape; 2 = the same
// when every row block's fibres are evenly spaced (the host checks: n % 16 == 0,
// and for modes >= 2 na / nnext % 16 == 0), with row-block addressing only.
template <bool MODE1, bool SWAP, int FUSE>
__global__ void __launch_bounds__(512, 1) gemm_i8_kernel(const ModeJobs J, int64_t per_xcd, int sup, int nnext) {
  __shared__ __attribute__((aligned(16))) uint8_t panel[2][kPanelRows * kPanelRow];
  __shared__ __attribute__((aligned(16))) int pexp[2][kPanelRows];
  __shared__ int emax[FUSE ? 2 : 1][kGemmWaves][kPanelRows];   // FUSE: magnitude-key maxima per half, wave, row
  __shared__ __attribute__((aligned(16))) int erow[kPanelRows];
  const int64_t t = remap_xcd_i8(blockIdx.x, per_xcd);
  if (t >= J.total_tiles) return;   // uniform over the block
  const ModeJob& jb = J.job[find_job(J, t)];
  const int64_t lt = t - jb.tile_begin;
  const int it = (int)(lt % jb.tiles_i);
  const int n = jb.n, ldp = jb.ldp;
  const int nterms = SWAP ? jb.nterms : 1;   // without SWAP the host guarantees one term, n <= 256
  const int64_t na = jb.na, nb = jb.nb;
  const int64_t nfib = MODE1 ? nb : na;
  const int64_t ntot = MODE1 ? nb : na * nb;
  const int64_t ngroups = (int64_t)jb.tiles_a * (MODE1 ? 1 : nb);
  const int64_t grp0 = (lt / jb.tiles_i) * sup;
  const int ngrp = (int)(ngroups - grp0 < sup ? ngroups - grp0 : sup);
  const int nch = SWAP ? (n + kPanelK - 1) / kPanelK : 1;   // 256-chunks of the contraction
  const int nitems = ngrp * nterms * nch;
  const int row0 = it * kPanelRows;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g = lane >> 4, l = lane & 15;
  const int64_t rowbytes = 4 * (int64_t)ldp;
  const int64_t ntot16 = (ntot + 15) & ~(int64_t)15;   // fibres of the digit tiles
  // FUSE, modes >= 2: next-mode fibres per row of this product (one division per workgroup)
  const int64_t fstride = FUSE && !MODE1 ? na / nnext : 0;

  // Position of an item in the run: column group ct of slab bslab, term tm,
  // contraction chunk ci.  Items advance incrementally: a
  // 64-bit division per item costs more scalar instructions than its k-steps.
  struct Pos {
    int tm, ci;
    int64_t ct, bslab;
  };
  auto first_pos = [&]() __attribute__((always_inline)) {
    Pos p{0, 0, MODE1 ? grp0 : grp0 % jb.tiles_a, MODE1 ? 0 : grp0 / jb.tiles_a};
    return p;
  };
  auto advance = [&](Pos p) __attribute__((always_inline)) {
    if (++p.ci == nch) {
      p.ci = 0;
      if (++p.tm == nterms) {
        p.tm = 0;
        if (++p.ct == jb.tiles_a && !MODE1) {
          p.ct = 0;
          ++p.bslab;
        }
      }
    }
    return p;
  };
  // column of this lane in the item's group (validity, global fibre index)
  auto column = [&](const Pos& p, int64_t& ca, int64_t& fib) __attribute__((always_inline)) {
    ca = p.ct * kGroupCols + kWaveCols * wave + l;
    fib = MODE1 ? ca : ca + na * p.bslab;
  };
  // tensor digits of an item, k-step k: this lane's 4 x 16 bytes (1 KB apart)
  auto bptr = [&](const Pos& p, int k64) __attribute__((always_inline)) {
    int64_t ca, fib;
    column(p, ca, fib);
    const uint8_t* D = (const uint8_t*)jb.X[p.tm];
    const int64_t f = ca < nfib ? fib : 0;
    return D + ((f >> 4) * (ldp / 64) + (p.ci * kPanelK + k64) / 64) * (int64_t)kTileBytes + 16 * (4 * (f & 15) + g);
  };
  // panel of item i: thread tid holds 16-byte unit `lane` of rows wave + 8 r
  v4i pn[8];
  int pen = 0;
  auto fetch_panel = [&](const Pos& p) __attribute__((always_inline)) {
    const uint8_t* P = (const uint8_t*)jb.P[p.tm];
    const int kc = p.ci * kPanelK;
    const int units = (ldp - kc < kPanelK ? ldp - kc : kPanelK) / 4;
#pragma unroll
    for (int r = 0; r < 8; ++r)
      pn[r] = lane < units ? *(const v4i*)(P + (int64_t)(row0 + wave + 8 * r) * rowbytes + 4 * kc + 16 * lane)
                           : v4i{0, 0, 0, 0};
    if (tid < kPanelRows) pen = ((const int*)(P + rowbytes * ldp))[row0 + tid];
  };
  auto store_panel = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int r = 0; r < 8; ++r) *(v4i*)(panel[buf] + (wave + 8 * r) * kPanelRow + 16 * lane) = pn[r];
    if (tid < kPanelRows) pexp[buf][tid] = pen;
  };
  // SWAP: the next item's panel goes into the idle buffer while the current
  // item runs, rows 2 j and 2 j + 1 of every thread's eight at k-step j (the
  // loads are issued before that step's products and stored after them); the
  // units past the chunk's width are never read, so their lanes load a valid
  // address and store whatever it holds
  v4i pq[2];
  auto fetch_rows = [&](const Pos& p, int r0) __attribute__((always_inline)) {
    const uint8_t* P = (const uint8_t*)jb.P[p.tm];
    const int kc = p.ci * kPanelK;
    const int units = (ldp - kc < kPanelK ? ldp - kc : kPanelK) / 4;
    const int u = lane < units ? lane : 0;
#pragma unroll
    for (int h = 0; h < 2; ++h)
      pq[h] = *(const v4i*)(P + (int64_t)(row0 + wave + 8 * (r0 + h)) * rowbytes + 4 * kc + 16 * u);
  };
  auto store_rows = [&](int buf, int r0) __attribute__((always_inline)) {
#pragma unroll
    for (int h = 0; h < 2; ++h) *(v4i*)(panel[buf] + (wave + 8 * (r0 + h)) * kPanelRow + 16 * lane) = pq[h];
  };

  fetch_panel(first_pos());
  store_panel(0);
  int pb = 0;
  __syncthreads();

  double out[4][4];
  double hv[4][4];   // FUSE with two groups per fibre set: the first group's values
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) out[m][r] = 0.0;
  v4i acc[5][4];   // [order a + b - 2][row block]
#pragma unroll
  for (int o = 0; o < 5; ++o)
#pragma unroll
    for (int m = 0; m < 4; ++m) acc[o][m] = v4i{0, 0, 0, 0};

  // state of the current item
  int i = 0, tm = 0, ci = 0, kend = 0, ex = 0;
  Pos cur = first_pos(), nxt = cur;
  auto nxt_pos = [&]() __attribute__((always_inline)) -> const Pos& { return nxt; };
  int64_t ca = 0, fib = 0;
  const uint8_t* bcur = nullptr;
  const uint8_t* bnext = nullptr;
  auto begin_item = [&]() __attribute__((always_inline)) {
    tm = cur.tm;
    ci = cur.ci;
    column(cur, ca, fib);
    nxt = advance(cur);
    const int kc = ci * kPanelK;
    const int kw = ldp - kc < kPanelK ? ldp - kc : kPanelK;
    kend = n - kc < kw ? n - kc : kw;
    // unconditional (clamped) for the same reason as the digit loads below
    ex = ((const int*)((const uint8_t*)jb.X[tm] + ntot16 * rowbytes))[ca < nfib ? fib : 0];
    bcur = bptr(cur, 0);
    bnext = i + 1 < nitems ? bptr(nxt, 0) : bcur;   // after the last item: a harmless reload
    if constexpr (SWAP) pen = ((const int*)((const uint8_t*)jb.P[nxt.tm] + rowbytes * ldp))[row0 + (tid & 63)];
  };
  // FUSE (one term, n <= 256; the next mode's size nnext in {128, 256}):
  // instead of the FP64 product, the digit planes of the operand of the next
  // mode, the one whose index runs fastest along this product's columns.
  // Mode 1: column b is (i2, i3) = (b % n2, b / n2), so the nnext / 128
  // consecutive groups of a run that share i3 hold, for each of the 64 rows
  // i1, the whole mode-2 fibre i1 + n1 i3.  Modes >= 2 (the next mode is 1):
  // column a is (i1, a / n1), and the groups sharing a / n1 hold, for each
  // row i and slab b, the whole mode-1 fibre a / n1 + (na / n1)(i + n b).
  // The first group's values wait in registers (hv); at the last group the
  // fibre exponents are formed from the
  // largest magnitude key over both groups (reduced across lanes with DPP,
  // then across waves in LDS) and every value is cut into its digits exactly
  // as the slicing kernel would, a quad of lanes trading bytes so that each
  // lane stores one 4-byte run of one plane.
  auto fused_digits = [&]() __attribute__((always_inline)) {
    if constexpr (FUSE) {
      const int g2 = nnext / kGroupCols;
      const int half = g2 == 2 ? (int)(cur.ct & 1) : 0;   // which group of the fibre set
      const int64_t set = g2 == 2 ? cur.ct >> 1 : cur.ct;   // MODE1: i3; modes >= 2: a / n1
      // the next mode's fibre through row R of this product
      auto fibre = [&](int R) __attribute__((always_inline)) {
        return MODE1 ? row0 + R + (int64_t)n * set : set + fstride * (row0 + R + (int64_t)n * cur.bslab);
      };
      int hk[4][4];   // magnitude keys of this lane's 16 values
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) hk[m][r] = mag_key(out[m][r]);
      // maximum over the 16 lanes of a row block: swaps within quads, then
      // the half-row and row mirrors (DPP, no LDS traffic)
      auto lane_max = [&](auto ctrl) __attribute__((always_inline)) {
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
          for (int r = 0; r < 4; ++r) hk[m][r] = max(hk[m][r], __builtin_amdgcn_mov_dpp(hk[m][r], decltype(ctrl)::value, 0xF, 0xF, true));
      };
      lane_max(std::integral_constant<int, 0xB1>{});    // quad_perm [1, 0, 3, 2]
      lane_max(std::integral_constant<int, 0x4E>{});    // quad_perm [2, 3, 0, 1]
      lane_max(std::integral_constant<int, 0x141>{});   // row_half_mirror
      lane_max(std::integral_constant<int, 0x140>{});   // row_mirror
      if (l == 0)
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
          for (int r = 0; r < 4; ++r) emax[half][wave][16 * m + 4 * g + r] = hk[m][r];
      if (half != g2 - 1) {
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
          for (int r = 0; r < 4; ++r) hv[m][r] = out[m][r];
        return;
      }
      __syncthreads();
      const int64_t ntot2 = MODE1 ? n * (nb / nnext) : fstride * n * nb;   // fibres of the next mode
      const int ldp2 = nnext, nks2 = nnext / 64;
      uint8_t* __restrict__ Dn = (uint8_t*)jb.Y;
      if (tid < kPanelRows) {
        int bmax = 0;
        for (int h = 0; h < g2; ++h)
          for (int w = 0; w < kGemmWaves; ++w) bmax = max(bmax, emax[h][w][tid]);
        const int E = fibre_exp(bmax);
        erow[tid] = E;
        if (row0 + tid < n) {
          ((int*)(Dn + ((ntot2 + 15) & ~(int64_t)15) * 4 * (int64_t)ldp2))[fibre(tid)] = E;
        }
      }
      __syncthreads();
      v4i Ev[4];   // exponents of this lane's rows 16 m + 4 g + r
#pragma unroll
      for (int m = 0; m < 4; ++m) Ev[m] = *(const v4i*)&erow[16 * m + 4 * g];
      // A quad of lanes holds 4 consecutive values of a row; after a 4 x 4
      // byte transpose in two pair swaps, lane t4 holds their digit plane t4.
      const int t4 = l & 3;
      const uint32_t selA = t4 < 2 ? 0x05040100u : 0x03020706u;    // keep 2 own bytes, take 2 of lane ^ 2
      const uint32_t selB = (t4 & 1) ? 0x03070105u : 0x06020400u;  // interleave with lane ^ 1
      // Destination of value (R, i2): tile (c2 / 16) nks2 + i2 / 64, plane t4,
      // slot 4 (c2 % 16) + (i2 / 16) % 4, byte 4 (l / 4); with
      // i2 = 128 h + 16 wave + l the column part is the same for every row,
      // and the four waves with the same wave / 4 fill a fibre's 64 bytes.
      const uint32_t loff = (uint32_t)((wave >> 2) * kTileBytes + kPlaneBytes * t4 + 16 * (wave & 3) + 4 * (l >> 2));
      // FUSE == 2: row part ((c2 / 16) nks2) kTileBytes + 64 (c2 % 16) =
      // ubase + sm m + sr r + lrow (the rows come in whole blocks of 16 whose
      // fibres are a multiple of 16 apart for modes >= 2, consecutive from a
      // multiple of 16 for mode 1).
      const int64_t tstride = (int64_t)nks2 * kTileBytes;
      int64_t ubase = 0, sm = 0, sr = 0;
      uint32_t lrow = 0;
      if constexpr (MODE1) {
        ubase = ((row0 + (int64_t)n * set) >> 4) * tstride;
        sm = tstride;
        sr = 64;
        lrow = 256 * g;
      } else {
        const int64_t fs = fstride >> 4;
        sr = fs * tstride;
        ubase = ((set >> 4) + fs * (row0 + (int64_t)n * cur.bslab)) * tstride + 64 * (set & 15);
        sm = 16 * sr;
        lrow = (uint32_t)(4 * g * sr);
      }
      // one row block at a time, its four rows side by side (independent
      // operations between each write and the lane exchange that reads it)
      auto emit = [&](auto from_hb, int h) __attribute__((always_inline)) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          if (FUSE == 2 && row0 + 16 * m >= n) break;   // whole row blocks
          uint32_t w[4], x[4], d[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const double v = decltype(from_hb)::value ? hv[m][r]
                                                      : out[m][r];
            const int E = Ev[m][r];
            w[r] = digit_word(v, E);   // unconditional: no branch around the arithmetic
            w[r] = E == kBadExp ? 0u : w[r];
          }
#pragma unroll
          for (int r = 0; r < 4; ++r)
            x[r] = __builtin_amdgcn_perm((uint32_t)__builtin_amdgcn_mov_dpp((int)w[r], 0x4E, 0xF, 0xF, false), w[r], selA);
#pragma unroll
          for (int r = 0; r < 4; ++r)
            d[r] = __builtin_amdgcn_perm((uint32_t)__builtin_amdgcn_mov_dpp((int)x[r], 0xB1, 0xF, 0xF, false), x[r], selB);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            if constexpr (FUSE == 2) {
              uint8_t* dst = Dn + (ubase + sm * m + sr * r + 2 * (int64_t)kTileBytes * h);
              *(uint32_t*)(dst + (lrow + loff)) = d[r];
            } else {
              const int R = 16 * m + 4 * g + r;
              if (row0 + R < n) {
                const int64_t c2 = fibre(R);
                uint8_t* dst = Dn + (((c2 >> 4) * nks2 + 2 * h) * (int64_t)kTileBytes + 64 * (c2 & 15));
                *(uint32_t*)(dst + loff) = d[r];
              }
            }
          }
        }
      };
      if (g2 == 2) {
        emit(std::true_type{}, 0);
        emit(std::false_type{}, 1);
      } else {
        emit(std::false_type{}, 0);
      }
      // No barrier after the digits: the next set's lane maxima overwrite
      // emax only once their writer is past this set's second barrier (the
      // reduction that read them is done), and erow is rewritten only after
      // the next set's first barrier, which every wave reaches after cutting
      // these digits.
    }
  };
  auto end_item = [&]() __attribute__((always_inline)) {
    __builtin_amdgcn_s_setprio(0);
    if (ci == nch - 1) {
      // 2^(Ex + Ep - 12) (acc6 + acc5 2^-8 + acc4 2^-16 + acc3 2^-24 + acc2 2^-32),
      // without branches: a non-finite column has a NaN scale, a non-finite
      // row a NaN high word
      const double sc = ex == kBadExp ? __builtin_nan("") : jb.scale[tm];
      v4i epv[4];   // exponents of this lane's matrix rows 16 m + 4 g + r
#pragma unroll
      for (int m = 0; m < 4; ++m) epv[m] = *(const v4i*)&pexp[pb][16 * m + 4 * g];
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ep = epv[m][r];
          double w = (double)acc[0][m][r] * 0x1p-32;
          w = fma((double)acc[1][m][r], 0x1p-24, w);
          w = fma((double)acc[2][m][r], 0x1p-16, w);
          w = fma((double)acc[3][m][r], 0x1p-8, w);
          w += (double)acc[4][m][r];
          w = ldexp(w, ex + ep - 12);
          w = __hiloint2double(ep == kBadExp ? 0x7FF80000 : __double2hiint(w), __double2loint(w));
          out[m][r] = fma(sc, w, out[m][r]);
          if (SWAP) __builtin_amdgcn_sched_barrier(0);   // one output at a time (registers)
        }
#pragma unroll
      for (int o = 0; o < 5; ++o)
#pragma unroll
        for (int m = 0; m < 4; ++m) acc[o][m] = v4i{0, 0, 0, 0};
      if (tm == nterms - 1) {   // the group's outputs are complete
        if constexpr (FUSE) {
          fused_digits();
        } else if (ca < nfib) {
          double* __restrict__ Y = (double*)jb.Y;
          const double* __restrict__ base = (const double*)jb.base;
          const int64_t slab = MODE1 ? 0 : na * (int64_t)n * cur.bslab;
          if (!MODE1 && row0 + kPanelRows <= n) {
            // modes >= 2, every row inside: one per-lane offset per item plus
            // uniform row steps (no per-row offsets held across the loop)
            const int64_t colb = ca + slab + na * (int64_t)(row0 + 4 * g);
            if (base) {
#pragma unroll
              for (int m0 = 0; m0 < 4; m0 += 2) {
                double bv[2][4];
#pragma unroll
                for (int m = 0; m < 2; ++m)
#pragma unroll
                  for (int r = 0; r < 4; ++r) bv[m][r] = base[colb + na * (16 * (m0 + m) + r)];
#pragma unroll
                for (int m = 0; m < 2; ++m)
#pragma unroll
                  for (int r = 0; r < 4; ++r) out[m0 + m][r] = bv[m][r] + out[m0 + m][r];
              }
            }
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
              for (int r = 0; r < 4; ++r) Y[colb + na * (16 * m + r)] = out[m][r];
          } else {
          // rows past n, or mode 1: the row terms depend on an opaque copy of
          // the sizes, so that the compiler does not hold sixteen per-row
          // offsets in registers across the products (they would spill)
          int64_t nao = MODE1 ? (int64_t)n : na;
          int nl = n - 1;
          asm volatile("" : "+s"(nao), "+s"(nl));
          auto off = [&](int ii) __attribute__((always_inline)) { return MODE1 ? ii + nao * ca : ca + nao * ii + slab; };
          if (base) {   // base values in flight eight at a time (rows past n read row n - 1)
#pragma unroll
            for (int m0 = 0; m0 < 4; m0 += 2) {
              double bv[2][4];
#pragma unroll
              for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                  const int ii = row0 + 16 * (m0 + m) + 4 * g + r;
                  bv[m][r] = base[off(ii < nl ? ii : nl)];
                }
#pragma unroll
              for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int r = 0; r < 4; ++r) out[m0 + m][r] = bv[m][r] + out[m0 + m][r];
            }
          }
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const int i0 = row0 + 16 * m + 4 * g;
            if (MODE1 && (n % 2) == 0 && i0 + 4 <= n) {   // 16-byte aligned runs of 4 rows
              *(d2*)(Y + off(i0)) = d2{out[m][0], out[m][1]};
              *(d2*)(Y + off(i0) + 2) = d2{out[m][2], out[m][3]};
              continue;
            }
            if (row0 + kPanelRows <= n) {   // the whole panel is inside: no per-row branches
#pragma unroll
              for (int r = 0; r < 4; ++r) Y[off(i0 + r)] = out[m][r];
            } else {
#pragma unroll
              for (int r = 0; r < 4; ++r)
                if (i0 + r < n) Y[off(i0 + r)] = out[m][r];
            }
          }
          }
        }
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
          for (int r = 0; r < 4; ++r) out[m][r] = 0.0;
      }
    }
    if (SWAP && i + 1 < nitems) {
      // the rows the item's k-steps did not fetch (items shorter than 4 k-steps)
      for (int r0 = 2 * ((kend + 63) / 64); r0 < 8; r0 += 2) {
        fetch_rows(nxt, r0);
        store_rows(pb ^ 1, r0);
      }
      if (tid < kPanelRows) pexp[pb ^ 1][tid] = pen;
      __syncthreads();   // the next panel is complete; every wave is past this item's reads
      pb ^= 1;
    }
  };
  auto load4 = [&](const uint8_t* p, v4i (&dst)[4]) {
#pragma unroll
    for (int sp = 0; sp < 4; ++sp) dst[sp] = *(const v4i*)(p + kPlaneBytes * sp);
  };
  auto products = [&](int k64, const v4i (&cur)[4]) {
    const uint8_t* pcur = panel[pb];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const uint8_t* pa = pcur + (16 * m + l) * kPanelRow + 4 * k64 + 64 * g;
      v4i a[4];
#pragma unroll
      for (int sp = 0; sp < 4; ++sp) a[sp] = *(const v4i*)(pa + 16 * sp);
      // matrix digit (first operand), tensor digit (second), order >= 2
      acc[4][m] = mfma_i8(a[3], cur[3], acc[4][m]);
      acc[3][m] = mfma_i8(a[3], cur[2], acc[3][m]);
      acc[3][m] = mfma_i8(a[2], cur[3], acc[3][m]);
      acc[2][m] = mfma_i8(a[3], cur[1], acc[2][m]);
      acc[2][m] = mfma_i8(a[2], cur[2], acc[2][m]);
      acc[2][m] = mfma_i8(a[1], cur[3], acc[2][m]);
      acc[1][m] = mfma_i8(a[3], cur[0], acc[1][m]);
      acc[1][m] = mfma_i8(a[2], cur[1], acc[1][m]);
      acc[1][m] = mfma_i8(a[1], cur[2], acc[1][m]);
      acc[1][m] = mfma_i8(a[0], cur[3], acc[1][m]);
      acc[0][m] = mfma_i8(a[2], cur[0], acc[0][m]);
      acc[0][m] = mfma_i8(a[1], cur[1], acc[0][m]);
      acc[0][m] = mfma_i8(a[0], cur[2], acc[0][m]);
      if (SWAP) __builtin_amdgcn_sched_barrier(0);   // one row block's operands at a time (registers)
    }
  };
  // Digit loads are unconditional (clamped addresses), so that the wait
  // before the products counts only the loads they consume: behind a branch
  // the compiler waits for every load in flight.
  //
  // Every item of K k-steps (one term, n <= 256): K rotating buffers, the
  // digits of step s + K - 1 (this item's or the next one's) requested at
  // step s, so each load has K - 1 steps of products to arrive in.
  auto run_fixed = [&](auto kc) __attribute__((always_inline)) {
    constexpr int K = decltype(kc)::value;
    v4i bb[K][4];
    begin_item();
#pragma unroll
    for (int s = 0; s + 1 < K; ++s) load4(bcur + kTileBytes * s, bb[s]);
    for (;;) {
      __builtin_amdgcn_s_setprio(1);   // products first when a SIMD has a wave in its epilogue
#pragma unroll
      for (int s = 0; s < K; ++s) {
        const int t = s + K - 1;
        load4(t < K ? bcur + kTileBytes * t : bnext + kTileBytes * (t - K), bb[(s + K - 1) % K]);
        __builtin_amdgcn_sched_barrier(0);   // the loads go out before the products
        products(64 * s, bb[s]);
      }
      end_item();
      if (++i == nitems) break;
      cur = nxt;
      begin_item();
    }
  };
  // Any items: two buffers trading roles (a register copy of a buffer would
  // wait on its load in flight), the next step's digits requested first.
  auto run_any = [&]() __attribute__((always_inline)) {
    v4i bA[4], bB[4];
    auto kstep = [&](int k64, v4i (&cur)[4], v4i (&nxt)[4]) {
      if constexpr (SWAP) fetch_rows(nxt_pos(), k64 / 32);
      load4(k64 + 64 < kend ? bcur + kTileBytes * ((k64 + 64) / 64) : bnext, nxt);
      __builtin_amdgcn_sched_barrier(0);
      products(k64, cur);
      if constexpr (SWAP) store_rows(pb ^ 1, k64 / 32);
    };
    begin_item();
    load4(bcur, bA);
    for (;;) {
      __builtin_amdgcn_s_setprio(1);
      int k = 0;
      for (; k + 64 < kend; k += 128) {
        kstep(k, bA, bB);
        kstep(k + 64, bB, bA);
      }
      const bool odd = k < kend;
      if (odd) kstep(k, bA, bB);   // the next item's first digits land in bB
      end_item();
      if (++i == nitems) break;
      cur = nxt;
      begin_item();
      if (odd) {
#pragma unroll
        for (int sp = 0; sp < 4; ++sp) bA[sp] = bB[sp];
      }
    }
  };
  const int ksteps = (n + 63) / 64;
  if constexpr (!SWAP) {
    if (ksteps == 4) return run_fixed(std::integral_constant<int, 4>{});
    if (ksteps == 3) return run_fixed(std::integral_constant<int, 3>{});
  }
  run_any();
}

}  // namespace

size_t packed_bytes_i8(int n) {
  const size_t ldp = (size_t)packed_ld(n);
  return 4 * ldp * ldp + 4 * ldp;
}

size_t i8_digit_bytes(int64_t N, int n) {
  const int64_t fibres = N / n;
  return (size_t)round_up(round_up(fibres, (int64_t)16) * 4 * packed_ld(n) + 4 * fibres, 256);
}

int launch_stage_slice_i8(const double* Us, const double* G, int ncomp, int64_t N, int n, const GParams& gp,
                          void* const* D, hipStream_t s) {
  if (n < 1 || n > kSliceChunk || N % n != 0 || ncomp < 1 || ncomp > 2) {
    set_error("stage slicing needs n in 1..%d dividing N and one or two components", kSliceChunk);
    return SETD_EINVAL;
  }
  const int64_t na = N / n;
  const int64_t per = ceil_div(ceil_div(na, 16), 8);   // 16 fibres per workgroup
  // timed with the pointwise kernels: it does the stage kernel's work (and a
  // slicing pass), no mode product
  ProfScope prof(s, kProfPointwise, 0.0, (double)ncomp * N * (16.0 + 4.0));
  auto kern = gp.kind == SETD_G_FHN ? stage_slice_i8_kernel<SETD_G_FHN>
             : gp.kind == SETD_G_SCHNAKENBERG ? stage_slice_i8_kernel<SETD_G_SCHNAKENBERG> : stage_slice_i8_kernel<0>;
  hipLaunchKernelGGL(kern, dim3((unsigned)(per * 8)), dim3(256), 0, s, Us, G, ncomp, N, na, n, packed_ld(n), gp,
                     (uint8_t*)D[0], (uint8_t*)(ncomp > 1 ? D[1] : D[0]), per);
  SETD_LAUNCHED();
  return SETD_OK;
}

int pack_matrix_i8(const double* M, int n, double scale, void* out, hipStream_t s) {
  const int ldp = packed_ld(n);
  hipLaunchKernelGGL(pack_i8_kernel, dim3((unsigned)ldp), dim3(256), 0, s, M, n, ldp, scale, (uint8_t*)out);
  SETD_LAUNCHED();
  return SETD_OK;
}

namespace {

// The digit GEMM of a table of jobs whose X[t] are digit buffers.
int launch_gemm_i8(const ModeJobs& J, bool mode1, hipStream_t s, int fuse_next) {
  // each workgroup takes a run of `sup` column groups of one row panel
  ModeJobs G = J;
  for (int j = 0; j < G.njobs; ++j) {
    ModeJob& jb = G.job[j];
    jb.tiles_i = (int)ceil_div(jb.n, kPanelRows);
    jb.tiles_a = (int)ceil_div(mode1 ? jb.nb : jb.na, kGroupCols);
  }
  // Run length: one 8-wave workgroup fits a CU, so the launch takes about
  // ceil(workgroups / CUs) rounds of (sup + 1) group-times (the one: the
  // panel fill and pipeline start of a workgroup).  The shortest such time,
  // ties to the shorter runs; fused launches with two groups per fibre set
  // need even runs.
  int sup = 1;
  double best = 0.0;
  for (int c = 1; c <= kMaxSup; ++c) {
    if (fuse_next == 2 * kGroupCols && (c & 1)) continue;
    int64_t wgs = 0;
    for (int j = 0; j < G.njobs; ++j) {
      const ModeJob& jb = G.job[j];
      wgs += (int64_t)jb.tiles_i * ceil_div((int64_t)jb.tiles_a * (mode1 ? 1 : jb.nb), c);
    }
    const double t = (double)ceil_div(wgs, kCus) * (c + 1);
    if (best == 0.0 || t < best) {
      best = t;
      sup = c;
    }
  }
  int64_t tot = 0;
  for (int j = 0; j < G.njobs; ++j) {
    ModeJob& jb = G.job[j];
    jb.tile_begin = tot;
    tot += (int64_t)jb.tiles_i * ceil_div((int64_t)jb.tiles_a * (mode1 ? 1 : jb.nb), sup);
  }
  G.total_tiles = tot;
  G.tiles_per_job = G.njobs > 0 ? tot / G.njobs : 0;
  for (int j = 0; j < G.njobs; ++j)
    if (G.job[j].tile_begin != (int64_t)j * G.tiles_per_job) G.tiles_per_job = 0;
  if (tot == 0) return SETD_OK;
  double fl = 0.0, by = 0.0;
  if (prof_on()) job_work(J, 4, fuse_next ? 4 : 8, 4, fl, by);   // digits in, FP64 (or digits) out
  ProfScope prof(s, mode1 ? kProfMode1LP : kProfModeBLP, fl, by);
  bool swap = false;
  for (int j = 0; j < G.njobs; ++j) swap = swap || G.job[j].nterms > 1 || G.job[j].n > kPanelK;
  const int64_t pxcd = ceil_div(tot, 8);
  const dim3 grid((unsigned)(pxcd * 8));
  // the fused form with row-block addressing when every job allows it
  bool aligned = true;
  for (int j = 0; j < G.njobs && fuse_next; ++j) {
    const ModeJob& jb = G.job[j];
    const int64_t fs = mode1 ? 0 : jb.na / fuse_next;
    aligned = aligned && jb.n % 16 == 0 && fs % 16 == 0 && 768 * fs * fuse_next < ((int64_t)1 << 31);
  }
  auto kern = fuse_next ? (aligned ? (mode1 ? gemm_i8_kernel<true, false, 2> : gemm_i8_kernel<false, false, 2>)
                                   : (mode1 ? gemm_i8_kernel<true, false, 1> : gemm_i8_kernel<false, false, 1>))
             : mode1     ? (swap ? gemm_i8_kernel<true, true, 0> : gemm_i8_kernel<true, false, 0>)
                         : (swap ? gemm_i8_kernel<false, true, 0> : gemm_i8_kernel<false, false, 0>);
  hipLaunchKernelGGL(kern, grid, dim3(512), 0, s, G, pxcd, sup, fuse_next);
  SETD_LAUNCHED();
  return SETD_OK;
}

}  // namespace

int launch_mode_i8(ModeJobs& J, bool mode1, void* ws, size_t ws_bytes, hipStream_t s, bool presliced, int fuse_next) {
  if (J.njobs == 0) return SETD_OK;
  if (fuse_next != 0) {
    bool ok = fuse_next == kGroupCols || fuse_next == 2 * kGroupCols;
    for (int j = 0; j < J.njobs; ++j)
      ok = ok && J.job[j].nterms == 1 && J.job[j].n <= kPanelK &&
           (mode1 ? J.job[j].nb % fuse_next == 0 : J.job[j].na % fuse_next == 0);
    if (!ok) {
      set_error("int8 fused slicing needs one term, n <= %d, a next mode of %d or %d dividing the columns", kPanelK,
                kGroupCols, 2 * kGroupCols);
      return SETD_EINVAL;
    }
  }
  if (presliced) return launch_gemm_i8(J, mode1, s, fuse_next);
  // 1. one digit buffer per distinct input tensor of the launch
  const void* inputs[kMaxJobs * kMaxTerms];
  int ninputs = 0;
  int slot_of[kMaxJobs][kMaxTerms];
  size_t per = 0;
  for (int j = 0; j < J.njobs; ++j) {
    const ModeJob& jb = J.job[j];
    per = std::max(per, i8_digit_bytes(jb.na * jb.n * jb.nb, jb.n));
    for (int t = 0; t < jb.nterms; ++t) {
      int k = 0;
      while (k < ninputs && inputs[k] != jb.X[t]) ++k;
      if (k == ninputs) inputs[ninputs++] = jb.X[t];
      slot_of[j][t] = k;
    }
  }
  if (ws == nullptr || (size_t)ninputs * per > ws_bytes) {
    set_error("int8 slicing workspace too small: %zu < %zu bytes", ws_bytes, (size_t)ninputs * per);
    return SETD_EINVAL;
  }
  // 2. slicing launches: one job per distinct input (all jobs of a launch
  // share the regime; inputs shared by several jobs have equal shapes)
  for (int k0 = 0; k0 < ninputs; k0 += kMaxJobs) {
    ModeJobs S;
    S.njobs = 0;
    int64_t tot = 0;
    for (int k = k0; k < std::min(ninputs, k0 + kMaxJobs); ++k) {
      int jj = 0, tt = 0;
      for (int j = 0; j < J.njobs; ++j)
        for (int t = 0; t < J.job[j].nterms; ++t)
          if (slot_of[j][t] == k) jj = j, tt = t;
      ModeJob sj = J.job[jj];
      sj.nterms = 1;
      sj.X[0] = J.job[jj].X[tt];
      sj.Y = (char*)ws + (size_t)k * per;
      sj.base = nullptr;
      sj.tiles_i = 1;
      sj.tiles_a = (int)ceil_div(mode1 ? sj.nb : sj.na, kSliceCols);
      sj.tile_begin = tot;
      tot += (int64_t)sj.tiles_a * (mode1 ? 1 : sj.nb);
      S.job[S.njobs++] = sj;
    }
    S.total_tiles = tot;
    S.tiles_per_job = 0;
    const int64_t pxcd = ceil_div(tot, 8);
    if (mode1)
      hipLaunchKernelGGL(slice_i8_kernel<true>, dim3((unsigned)(pxcd * 8)), dim3(256), 0, s, S, pxcd);
    else
      hipLaunchKernelGGL(slice_i8_kernel<false>, dim3((unsigned)(pxcd * 8)), dim3(256), 0, s, S, pxcd);
    SETD_LAUNCHED();
  }
  for (int j = 0; j < J.njobs; ++j)
    for (int t = 0; t < J.job[j].nterms; ++t) J.job[j].X[t] = (char*)ws + (size_t)slot_of[j][t] * per;
  return launch_gemm_i8(J, mode1, s, fuse_next);
}

}  // namespace setd