// Internal helpers shared by the HIP sources of libsetd (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/setd.h"

namespace setd {

// ---- error reporting (thread-local message, status codes of setd.h) ----
void set_error(const char* fmt, ...);
void clear_error();

#define SETD_CHECK_ARG(cond, ...)                 \
  do {                                            \
    if (!(cond)) {                                \
      ::setd::set_error(__VA_ARGS__);             \
      return SETD_EINVAL;                         \
    }                                             \
  } while (0)

#define SETD_HIP(call)                                                              \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess) {                                                         \
      ::setd::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),      \
                        __FILE__, __LINE__);                                        \
      return e_ == hipErrorOutOfMemory ? SETD_ENOMEM : SETD_EHIP;                   \
    }                                                                               \
  } while (0)

#define SETD_TRY(expr)          \
  do {                          \
    int rc_ = (expr);           \
    if (rc_ != SETD_OK) return rc_; \
  } while (0)

// Launch-error check after a kernel launch.
#define SETD_LAUNCHED()                                                              \
  do {                                                                               \
    hipError_t e_ = hipGetLastError();                                               \
    if (e_ != hipSuccess) {                                                          \
      ::setd::set_error("kernel launch failed: %s (%s:%d)", hipGetErrorString(e_),   \
                        __FILE__, __LINE__);                                         \
      return SETD_EHIP;                                                              \
    }                                                                                \
  } while (0)

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

// ---- device vector types ----
typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));

// Padded size of a packed matrix (rows and columns): multiple of 64 so that a
// 64-row / 64-column wave tile never reads outside it.
inline int packed_ld(int n) { return (int)round_up(n, 64); }

// ---- mu-mode product job tables (see mode_f64.hip) ----
constexpr int kMaxTerms = 3;
constexpr int kMaxJobs = 20;

// One output tensor Y[a, i, b] = base[a, i, b] + sum_t sum_p S_t[i, p] X_t[a, p, b]
// over a (extent na, stride 1), i/p (extent n, stride na), b (extent nb,
// stride na*n).  S_t is scale_t * P_t with P_t a packed matrix.
struct ModeJob {
  const void* X[kMaxTerms];
  const void* P[kMaxTerms];   // packed matrix (layout depends on the kernel)
  double scale[kMaxTerms];
  void* Y;
  const void* base;           // nullable
  int64_t na, nb;
  int n, ldp, nterms;
  int tiles_a, tiles_i;       // tiles along a (or b for mode 1) and i
  int64_t tile_begin;         // first logical tile of this job
};

struct ModeJobs {
  ModeJob job[kMaxJobs];
  int njobs;
  int64_t total_tiles;
  int64_t tiles_per_job;   // > 0 when every job has this many tiles
};

// Job owning logical tile t: one division when all jobs have the same tile
// count, else a binary search over tile_begin (no serial chain of loads).
__device__ __forceinline__ int find_job(const ModeJobs& J, int64_t t) {
  if (J.tiles_per_job > 0) return (int)(t / J.tiles_per_job);
  int lo = 0, hi = J.njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (J.job[mid].tile_begin <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Same search for a job list in device memory, over its compact array of
// first tiles (ascending): 8 bytes per job, so the array of a whole batch
// stays in the scalar cache while the job records themselves do not.
__device__ __forceinline__ int find_job_list(const int64_t* begins, int njobs, int64_t t) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (begins[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

enum class DType : int { F64 = 0, F32 = 1 };

// ---- kernel timing (setd_profile_*), implemented in setd_api.hip ----
enum ProfClass : int {
  kProfMode1F64 = 0,
  kProfModeBF64 = 1,
  kProfMode1LP = 2,
  kProfModeBLP = 3,
  kProfPointwise = 4,
  kProfModeBPanelF64 = 5   // modes >= 2, matrix panel in LDS
};
bool prof_on();
// Records the begin event on construction and the end event on destruction
// (only while profiling is enabled).
struct ProfScope {
  ProfScope(hipStream_t s, int cls, double flops, double bytes);
  ~ProfScope();
  hipStream_t s_;
  int slot_;
};


// Mode-product launchers (implemented in mode_f64.hip / mode_lp.hip).
// `jobs` is filled by the caller except for the tile fields, which the
// launcher computes.  All jobs of one launch share regime (mode 1 or not).
int launch_mode1_f64(ModeJobs& jobs, hipStream_t s);
int launch_modeB_f64(ModeJobs& jobs, hipStream_t s);
// Reduced precision (mode_lp.hip): FP32 tensor inputs, output FP32 or FP64
// (FP64 output adds the optional FP64 base).
int launch_mode1_lp(ModeJobs& jobs, int prec, DType out, hipStream_t s);
int launch_modeB_lp(ModeJobs& jobs, int prec, DType out, hipStream_t s);

// Tile bookkeeping shared by the launchers and the batched work lists:
// fills tiles_i / tiles_a / tile_begin for a TM x TN tile (16 TM rows of the
// MFMA row index, 16 TN columns) and returns the total tile count.
int64_t assign_tiles(ModeJob* jobs, int njobs, bool mode1, int TM, int TN);
// Kernel variant a job can use: 0 = element loads with checks, 1 = vector
// loads (aligned, extents a multiple of 4), 2 = interior fast path.
int job_mode(const ModeJob& jb, bool mode1, int TM, int TN);

// A work list in device memory (FP64): one persistent launch walks all tiles
// of `njobs` jobs, each of which may belong to a different problem instance.
// Every job of a list shares the regime, the tile shape and the variant.
struct ModeList {
  const ModeJob* jobs;   // device
  const int64_t* begins; // device: jobs[j].tile_begin
  int njobs;
  int64_t total;         // tiles
  bool mode1;
  int tm, tn, mode;
  int64_t grid_cap;      // maximum number of workgroups (0: one per tile)
  double flops, bytes;   // algorithmic work, for the kernel timing
};
int launch_list_f64(const ModeList& L, hipStream_t s);

// Algorithmic flops / bytes of a job table (2 N n per term; each input read
// once, output written once, base read once; es = element sizes in bytes).
void job_work(const ModeJobs& J, int es_in, int es_out, int es_mat, double& flops, double& bytes);

// Matrix packing (pointwise.hip).
//   pack_rowmajor: PT[i*ldp + p] = scale*M[i + n p]   (mode-1 operand)
//   pack_colmajor: P [i + ldp*p] = scale*M[i + n p]   (mode >= 2 operand)
// zero outside n x n.
int pack_matrix_f64(const double* M, int n, double scale, bool rowmajor, double* out, hipStream_t s);
int pack_matrix_f32(const double* M, int n, double scale, bool rowmajor, float* out, hipStream_t s);
int pack_matrix_bf16(const double* M, int n, double scale, bool rowmajor, int np, void* out, hipStream_t s);
inline bool is_prec(int p) {
  return p == SETD_PREC_F64 || p == SETD_PREC_F32 || p == SETD_PREC_BF16X3 || p == SETD_PREC_BF16X2 ||
         p == SETD_PREC_I8X4;
}
// Arithmetics whose Tucker inputs and intermediates are stored in FP32 (the
// others keep them in FP64).
inline bool fp32_storage(int p) {
  return p == SETD_PREC_F32 || p == SETD_PREC_BF16X3 || p == SETD_PREC_BF16X2;
}
size_t packed_bytes(int n, int prec);
// Error-free int8 slicing (mode_i8.hip): packed matrix size, packing, the
// digit-buffer size of one FP64 input of N entries contracted along a mode of
// size n, and the mode-product launcher (FP64 tensors, any regime), which
// needs one digit buffer per distinct input of the launch in `ws`.
size_t packed_bytes_i8(int n);
int pack_matrix_i8(const double* M, int n, double scale, void* out, hipStream_t s);
size_t i8_digit_bytes(int64_t N, int n);
// presliced: the jobs' X[t] are already digit buffers (no slicing pass).
// fuse_next = n2 in {128, 256} (mode 1 only): the jobs' Y receive the digit
// buffer of the mode-2 operand instead of the FP64 product.
int launch_mode_i8(ModeJobs& jobs, bool mode1, void* ws, size_t ws_bytes, hipStream_t s, bool presliced = false,
                   int fuse_next = 0);

// Pointwise helpers (pointwise.hip).
int launch_axpby(const double* x, double* y, int64_t n, double a, double b, hipStream_t s);  // y = a x + b y
int launch_scale(double* y, int64_t n, double b, hipStream_t s);                              // y *= b (b == 0 -> 0)
int launch_copy_convert(const double* x, void* y, int64_t n, DType out, hipStream_t s);

}  // namespace setd
