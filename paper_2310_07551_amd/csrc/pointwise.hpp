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

// g(u, v) of the two-component kinetics (eq. twocompdisc), rho included:
// KIND is SETD_G_SCHNAKENBERG, SETD_G_FHN or anything else for g = 0.
template <int KIND>
__device__ __forceinline__ void reaction_of(const GParams& P, double u, double v, double& g1, double& g2) {
  if constexpr (KIND == SETD_G_SCHNAKENBERG) {
    const double u2v = u * u * v;
    g1 = P.p[0] * (P.p[1] - u + u2v);
    g2 = P.p[0] * (P.p[2] - u2v);
  } else if constexpr (KIND == SETD_G_FHN) {
    const double rho = P.p[3];
    g1 = rho * (u - u * u * u - v);
    g2 = rho * P.p[0] * (u - P.p[1] * v - P.p[2]);
  } else {
    g1 = 0.0;
    g2 = 0.0;
  }
}
__device__ __forceinline__ void reaction(const GParams& P, double u, double v, double& g1, double& g2) {
  if (P.kind == SETD_G_SCHNAKENBERG)
    reaction_of<SETD_G_SCHNAKENBERG>(P, u, v, g1, g2);
  else if (P.kind == SETD_G_FHN)
    reaction_of<SETD_G_FHN>(P, u, v, g1, g2);
  else
    reaction_of<0>(P, u, v, g1, g2);
}

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
// SETD_PREC_I8X4 (mode_i8.hip): D_c = g_c(Us) - G_c for the ncomp (1 or 2)
// components, written only as the int8 digits of its fibres along the last
// mode of size n (n <= 256, dividing N) into the digit buffers D[c]; the
// bits are those the slicing kernel cuts from the FP64 D of launch_stage_d.
int launch_stage_slice_i8(const double* Us, const double* G, int ncomp, int64_t N, int n, const GParams& gp,
                          void* const* D, hipStream_t s);
size_t norm_workspace_bytes();
int launch_norms(const double* x, const double* y, int64_t n, double* ws, hipStream_t s);

// phi-functions of c_j * A for a batch of scalars (phi.hip).  For entry j the
// blocks phi_0..phi_p(c_j A) are written to out[j*(p+1) + k] (device n x n
// column-major).  Synchronises s.
int phi_batch(const double* A, int n, const double* c, int nentries, int p, double* const* out, hipStream_t s);

}  // namespace setd
