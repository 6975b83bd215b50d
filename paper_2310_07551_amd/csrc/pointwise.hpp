// Interfaces of the pointwise kernels (pointwise.hip) and the phi builder (phi.hip).
#pragma once

#include "common.hpp"

namespace setd {

__host__ __device__ inline int64_t ceil_div_dev(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Reaction parameters as the kernels see them (rho filled in, = 1 if absent).
struct GParams {
  int kind;
  double p[4];
};

// Tridiagonal coefficients of A_mu^(c): index c*3 + mu; arrays of n_mu
// (device).  lo[i] = A[i, i-1], di[i] = A[i, i], up[i] = A[i, i+1].
struct StencilSet {
  const double* lo[6];
  const double* di[6];
  const double* up[6];
};

// One instance of a batch as the batched pointwise kernels see it: its
// fields start at element `off` of every batch-wide field buffer, component c
// at off + c * cs.
struct BatchInstDev {
  int64_t off, cs, N;
  int n[3];
  int d;
  GParams gp;
  StencilSet st;   // tridiagonal coefficients (kind 0 only)
};
constexpr int kBatchBlock = 256;
// kind 0: G = g(u), F = K u + G (stencil); 1: G = g(u); 2: out = g(x) - G.
// blk[b] = first block of instance b (nbatch entries, ascending).
int launch_batch_pointwise(int kind, const BatchInstDev* inst, const int64_t* blk, int nbatch, int64_t nblocks,
                           int ncomp, int64_t total_points, const double* x, double* G, double* out, hipStream_t s);

int launch_gf_stencil(const double* u, int ncomp, int64_t N, int d, const int* dims, const StencilSet& S,
                      const GParams& gp, double* G, void* F, DType ftype, hipStream_t s);
int launch_g(const double* u, int ncomp, int64_t N, const GParams& gp, double* G, hipStream_t s);
int launch_stage_d(const double* Us, const double* G, int ncomp, int64_t N, const GParams& gp, void* D,
                   DType dtype, hipStream_t s);
size_t norm_workspace_bytes();
int launch_norms(const double* x, const double* y, int64_t n, double* ws, hipStream_t s);

// phi-functions of c_j * A for a batch of scalars (phi.hip).  For entry j the
// blocks phi_0..phi_p(c_j A) are written to out[j*(p+1) + k] (device n x n
// column-major).  Synchronises s.
int phi_batch(const double* A, int n, const double* c, int nentries, int p, double* const* out, hipStream_t s);

}  // namespace setd
