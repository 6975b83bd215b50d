// Host-side helpers shared by the context (setd_api.hip) and the batch
// (batch.hip) implementations.  Not part of the ABI.
#pragma once

#include <cmath>
#include <vector>

#include "common.hpp"
#include "pointwise.hpp"

namespace setd {

// Bank entries of Algorithms 1-2: (stage, ell) pairs.
inline const int kBankStage[5] = {SETD_STAGE_2, SETD_STAGE_3, SETD_STAGE_3, SETD_STAGE_F, SETD_STAGE_F};
inline const int kBankEll[5] = {1, 1, 2, 1, 2};

inline int bank_index(int stage, int ell) {
  for (int e = 0; e < 5; ++e)
    if (kBankStage[e] == stage && kBankEll[e] == ell) return e;
  return -1;
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  int alloc(size_t b) {
    release();
    if (b == 0) return SETD_OK;
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
      p = nullptr;
      set_error("hipMalloc(%zu) failed: %s", b, hipGetErrorString(e));
      return SETD_ENOMEM;
    }
    bytes = b;
    return SETD_OK;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  ~DevBuf() { release(); }
};

// One mu-mode product job with a single term (see ModeJob).
inline ModeJob mk_job(const void* X, const void* P, double scale, void* Y, const void* base, int64_t na, int n,
               int64_t nb) {
  ModeJob j{};
  j.X[0] = X;
  j.P[0] = P;
  j.scale[0] = scale;
  j.nterms = 1;
  j.Y = Y;
  j.base = base;
  j.na = na;
  j.nb = nb;
  j.n = n;
  j.ldp = packed_ld(n);
  return j;
}

inline bool is_tridiagonal(const std::vector<double>& A, int n) {
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i)
      if ((i - j > 1 || j - i > 1) && A[i + (size_t)n * j] != 0.0) return false;
  return true;
}

// Reaction parameters of setd.h checked and copied into the kernels' form.
inline int make_gparams(int g_kind, const double* params, int nparams, int ncomp, GParams& gp) {
  gp.kind = g_kind;
  gp.p[0] = gp.p[1] = gp.p[2] = 0.0;
  gp.p[3] = 1.0;
  if (g_kind == SETD_G_NONE) {
    SETD_CHECK_ARG(nparams == 0 || params != nullptr, "params is NULL");
    return SETD_OK;
  }
  SETD_CHECK_ARG(ncomp == 2, "reaction kind %d needs two components", g_kind);
  SETD_CHECK_ARG(params != nullptr, "params is NULL");
  if (g_kind == SETD_G_SCHNAKENBERG) {
    SETD_CHECK_ARG(nparams == 3, "Schnakenberg takes 3 parameters (gamma, a, b)");
  } else if (g_kind == SETD_G_FHN) {
    SETD_CHECK_ARG(nparams == 3 || nparams == 4, "FitzHugh-Nagumo takes 3 or 4 parameters (eps, a1, a0[, rho])");
  } else {
    SETD_CHECK_ARG(false, "unknown reaction kind %d", g_kind);
  }
  for (int k = 0; k < nparams; ++k) {
    if (!std::isfinite(params[k])) {
      set_error("reaction parameter %d is not finite", k);
      return SETD_ENONFINITE;
    }
    gp.p[k] = params[k];
  }
  return SETD_OK;
}

inline bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const char* x = (const char*)a;
  const char* y = (const char*)b;
  return x < y + nb && y < x + na;
}

}  // namespace setd
