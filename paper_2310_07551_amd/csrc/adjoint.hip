// Adjoint (vector-Jacobian product) of one split-ETD3 step, for gradients of
// a loss of the final state with respect to the initial state, the reaction
// parameters and the size of the diffusion of each component.
//
// The step (eq. exprk3 with the split phi actions S_l, the time loop of
// Algorithms 1 and 2)
//     G = g(U), F = K U + G,
//     U2 = U + tau/3 S1(2) F,            D2 = g(U2) - G,
//     U3 = U + 2tau/3 S1(3) F + 4tau/3 S2(3) D2,   D3 = g(U3) - G,
//     U' = U + tau S1(f) F + 3tau/2 S2(f) D3
// is run backwards.  Each split action S V = sum_i eta_i T(V, {P_{i,mu}})
// has the transpose S^T W = sum_i eta_i T(W, {P_{i,mu}^T}): a Tucker operator
// is the Kronecker product of its matrices acting on vec V (Section 2), so
// the transposed action is the same mu-mode product chain with transposed
// matrices, packed once per step size into the layouts of the forward
// kernels.  K^T is the Kronecker sum of the A_mu^T (a transposed 3-point
// stencil when every A_mu is tridiagonal).  The reaction enters through its
// pointwise 2 x 2 Jacobian transpose and its parameter derivatives.
//
// Diffusion size: with every A_mu^(c) scaled to sigma_c A_mu^(c), the
// derivative at sigma_c = 1 of phi_l(z sigma A) is phi_{l-1}(z A) -
// l phi_l(z A) (term-by-term derivative of the phi series, z phi_l'(z) =
// phi_{l-1}(z) - l phi_l(z)); a split action's derivative is the sum over
// directions of its Tuckers with that direction's matrix replaced (product
// rule), and the K action's is K U = F - G.
//
// Gradient sums are reduced deterministically: fixed grids write per-block
// partial sums, one small kernel adds them in a fixed order to the caller's
// device accumulators.
#include <cmath>
#include <cstring>

#include "ctx.hpp"

namespace setd {
namespace {

constexpr int kRedBlocks = 512;
constexpr int kRedThreads = 256;
// rows of the partial-sum buffer
constexpr int kRowP1 = 0, kRowP2 = 4, kRowP3 = 8, kRowSigK = 12, kRowSigE = 14, kRows = 16;

// J_g(u, v)^T (gu, gv) and the parameter derivatives of <(gu, gv), g(u, v)>.
__device__ __forceinline__ void reaction_vjp(const GParams& P, double u, double v, double gu, double gv, double& ub,
                                             double& vb, double dp[4]) {
  dp[0] = dp[1] = dp[2] = dp[3] = 0.0;
  if (P.kind == SETD_G_SCHNAKENBERG) {
    const double gam = P.p[0], a = P.p[1], b = P.p[2];
    const double uv = u * v, uu = u * u;
    ub = gam * (gu * (2.0 * uv - 1.0) - gv * 2.0 * uv);
    vb = gam * uu * (gu - gv);
    dp[0] = gu * (a - u + uu * v) + gv * (b - uu * v);
    dp[1] = gam * gu;
    dp[2] = gam * gv;
  } else if (P.kind == SETD_G_FHN) {
    const double eps = P.p[0], a1 = P.p[1], a0 = P.p[2], rho = P.p[3];
    const double lin = u - a1 * v - a0;
    ub = rho * (gu * (1.0 - 3.0 * u * u) + gv * eps);
    vb = -rho * (gu + gv * eps * a1);
    dp[0] = rho * gv * lin;
    dp[1] = -rho * eps * gv * v;
    dp[2] = -rho * eps * gv;
    dp[3] = gu * (u - u * u * u - v) + eps * gv * lin;
  } else {
    ub = 0.0;
    vb = 0.0;
  }
}

// Block sum of NV per-thread values into part[(row0 + k) * kRedBlocks + block].
template <int NV>
__device__ __forceinline__ void block_partials(const double (&v)[NV], double* __restrict__ part, int row0) {
  __shared__ double s[NV][kRedThreads];
  for (int k = 0; k < NV; ++k) s[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int w = kRedThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int k = 0; k < NV; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < NV; ++k) part[(row0 + k) * kRedBlocks + blockIdx.x] = s[k][0];
}

// Stage difference adjoint: Xbar = J_g(X)^T Dbar; Gbar = -Dbar (first) or
// Gbar -= Dbar; parameter partials into rows row0..row0+3.
__global__ void __launch_bounds__(kRedThreads) adj_stage_kernel(const double* __restrict__ X,
                                                                const double* __restrict__ Dbar, int ncomp,
                                                                int64_t N, GParams gp, double* __restrict__ Xbar,
                                                                double* __restrict__ Gbar, bool first,
                                                                double* __restrict__ part, int row0) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    const double u = X[i], v = ncomp > 1 ? X[N + i] : 0.0;
    const double gu = Dbar[i], gv = ncomp > 1 ? Dbar[N + i] : 0.0;
    double ub, vb, dp[4];
    reaction_vjp(gp, u, v, gu, gv, ub, vb, dp);
    for (int k = 0; k < 4; ++k) acc[k] += dp[k];
    Xbar[i] = ub;
    Gbar[i] = first ? -gu : Gbar[i] - gu;
    if (ncomp > 1) {
      Xbar[N + i] = vb;
      Gbar[N + i] = first ? -gv : Gbar[N + i] - gv;
    }
  }
  block_partials<4>(acc, part, row0);
}

// Final combination at one grid point:
//   Ubar = Wbar + U3bar + U2bar + K^T Fbar + J_g(U)^T (Gbar + Fbar)
// (in place on ubar), parameter partials (rows kRowP3..) and the K part of
// the diffusion-size derivative <Fbar_c, K_c U_c> = <Fbar_c, F_c - G_c>.
__global__ void __launch_bounds__(kRedThreads) adj_final_kernel(
    const double* __restrict__ U, double* __restrict__ ubar, const double* __restrict__ U3bar,
    const double* __restrict__ U2bar, const double* __restrict__ Fbar, const double* __restrict__ Gbar,
    const double* __restrict__ F, const double* __restrict__ G, const double* __restrict__ KtF, int ncomp, int64_t N,
    int d, int n1, int n2, int n3, StencilSet S, GParams gp, double* __restrict__ part) {
  double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const int ns[3] = {n1, n2, n3};
  const int64_t strides[3] = {1, (int64_t)n1, (int64_t)n1 * n2};
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < N;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int i1 = (int)(idx % n1);
    const int64_t r = idx / n1;
    const int idxs[3] = {i1, (int)(r % n2), d == 3 ? (int)(r / n2) : 0};
    double gb[2] = {0.0, 0.0}, uc[2] = {0.0, 0.0}, kt[2] = {0.0, 0.0};
    for (int c = 0; c < ncomp; ++c) {
      const int64_t o = (int64_t)c * N + idx;
      uc[c] = U[o];
      gb[c] = Gbar[o] + Fbar[o];
      acc[4 + c] += Fbar[o] * (F[o] - G[o]);
      if (KtF) {
        kt[c] = KtF[o];
      } else {
        // (A^T x)_i = A[i-1, i] x_{i-1} + A[i, i] x_i + A[i+1, i] x_{i+1}
        const double* __restrict__ fb = Fbar + (int64_t)c * N;
        double k = 0.0;
        for (int mu = 0; mu < d; ++mu) {
          const int i = idxs[mu];
          const int off = c * 3 + mu;
          double t = S.di[off][i] * fb[idx];
          if (i > 0) t += S.up[off][i - 1] * fb[idx - strides[mu]];
          if (i + 1 < ns[mu]) t += S.lo[off][i + 1] * fb[idx + strides[mu]];
          k += t;
        }
        kt[c] = k;
      }
    }
    double ub, vb, dp[4];
    reaction_vjp(gp, uc[0], uc[1], gb[0], gb[1], ub, vb, dp);
    for (int k = 0; k < 4; ++k) acc[k] += dp[k];
    const double gv[2] = {ub, vb};
    for (int c = 0; c < ncomp; ++c) {
      const int64_t o = (int64_t)c * N + idx;
      ubar[o] = ubar[o] + U3bar[o] + U2bar[o] + kt[c] + gv[c];
    }
  }
  block_partials<6>(acc, part, kRowP3);
}

// sum_c-wise <Ef, Wbar> + <E3, U3bar> + <E2, U2bar> into rows kRowSigE + c.
__global__ void __launch_bounds__(kRedThreads) adj_dots_kernel(const double* __restrict__ Ef,
                                                               const double* __restrict__ Wb,
                                                               const double* __restrict__ E3,
                                                               const double* __restrict__ U3b,
                                                               const double* __restrict__ E2,
                                                               const double* __restrict__ U2b, int ncomp, int64_t N,
                                                               double* __restrict__ part) {
  double acc[2] = {0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
    for (int c = 0; c < ncomp; ++c) {
      const int64_t o = (int64_t)c * N + i;
      acc[c] += Ef[o] * Wb[o] + E3[o] * U3b[o] + E2[o] * U2b[o];
    }
  block_partials<2>(acc, part, kRowSigE);
}

// grad[k] += parameter partials (k < nparams); grad[nparams + c] += diffusion
// partials for the components in sigma_mask.  One wave; row sums in a fixed
// order, so the result does not depend on scheduling.
__global__ void adj_reduce_kernel(const double* __restrict__ part, int nparams, int ncomp, int sigma_mask, bool dots,
                                  double* __restrict__ grad) {
  __shared__ double rs[kRows];
  const int r = threadIdx.x;
  if (r < kRows) {
    double s = 0.0;
    for (int b = 0; b < kRedBlocks; ++b) s += part[r * kRedBlocks + b];
    rs[r] = s;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int k = 0; k < nparams && k < 4; ++k) grad[k] += rs[kRowP1 + k] + rs[kRowP2 + k] + rs[kRowP3 + k];
  for (int c = 0; c < ncomp; ++c)
    if (sigma_mask & (1 << c)) grad[nparams + c] += rs[kRowSigK + c] + (dots ? rs[kRowSigE + c] : 0.0);
}

// Transposed and derivative phi matrices (and transposed A for the dense K
// path), packed for the forward mode kernels.  Synchronises s.
int build_adjoint_bank(setd_ctx* c, hipStream_t s) {
  const int d = c->d, T = c->nterms;
  size_t bytes = 0;
  for (int cc = 0; cc < c->ncomp; ++cc)
    for (int mu = 0; mu < d; ++mu) bytes += (2 * 5 * T + 1) * packed_bytes(c->dims[mu], SETD_PREC_F64);
  SETD_TRY(c->adj_bank_mem.alloc(bytes));
  char* q = (char*)c->adj_bank_mem.p;
  for (int cc = 0; cc < c->ncomp; ++cc)
    for (int mu = 0; mu < d; ++mu) {
      const int n = c->dims[mu];
      const size_t pb = packed_bytes(n, SETD_PREC_F64);
      const size_t nn = (size_t)n * n;
      const bool rowmajor = mu == 0;   // layout the forward kernels read for this direction
      std::vector<double> scal;
      for (int e = 0; e < 5; ++e)
        for (int t = 0; t < T; ++t)
          scal.push_back(stage_scale(kBankStage[e]) * c->tau * c->sp[kBankEll[e]].alpha[t][mu]);
      const int E = (int)scal.size();
      DevBuf A, raw, tmp;
      SETD_TRY(A.alloc(nn * sizeof(double)));
      SETD_HIP(hipMemcpyAsync(A.p, c->Ah[cc][mu].data(), nn * sizeof(double), hipMemcpyHostToDevice, s));
      SETD_TRY(raw.alloc((size_t)E * 3 * nn * sizeof(double)));
      SETD_TRY(tmp.alloc(nn * sizeof(double)));
      std::vector<double*> outs(E * 3);
      for (int k = 0; k < E * 3; ++k) outs[k] = (double*)raw.p + (size_t)k * nn;
      SETD_TRY(phi_batch((const double*)A.p, n, scal.data(), E, 2, outs.data(), s));
      for (int e = 0; e < 5; ++e)
        for (int t = 0; t < T; ++t) {
          const int k = e * T + t;
          const int li = c->sp[kBankEll[e]].ell_i[t];
          // the transpose of M packed in one layout is M packed in the other
          c->bankT[cc][e][t][mu] = q;
          SETD_TRY(pack_matrix_f64(outs[k * 3 + li], n, 1.0, !rowmajor, (double*)q, s));
          q += pb;
          // phi_{l-1} - l phi_l
          SETD_HIP(hipMemcpyAsync(tmp.p, outs[k * 3 + li - 1], nn * sizeof(double), hipMemcpyDeviceToDevice, s));
          SETD_TRY(launch_axpby(outs[k * 3 + li], (double*)tmp.p, (int64_t)nn, -(double)li, 1.0, s));
          c->dbank[cc][e][t][mu] = q;
          SETD_TRY(pack_matrix_f64((const double*)tmp.p, n, 1.0, rowmajor, (double*)q, s));
          q += pb;
        }
      c->ApkT[cc][mu] = q;
      SETD_TRY(pack_matrix_f64((const double*)A.p, n, 1.0, !rowmajor, (double*)q, s));
      q += pb;
      SETD_HIP(hipStreamSynchronize(s));   // A, raw and tmp are released at scope exit
    }
  c->adj_tau = c->tau;
  return SETD_OK;
}

int alloc_adjoint_buffers(setd_ctx* c) {
  const int64_t NN = (int64_t)c->ncomp * c->N;
  const size_t fb = round_up(NN * 8, 256);
  const size_t cb = round_up(c->N * 8, 256);
  const int nfields = 11;
  const int nchain = c->d == 3 ? c->ncomp * 9 * 2 : 0;   // sY: one field each
  SETD_TRY(c->adj_mem.alloc(nfields * fb + nchain * cb + (size_t)kRows * kRedBlocks * 8));
  char* q = (char*)c->adj_mem.p;
  double** f[nfields] = {&c->aD2, &c->aD3, &c->Fbar, &c->Dbar, &c->Gbar, &c->U3bar,
                         &c->U2bar, &c->Ef, &c->E3, &c->E2, &c->KtF};
  for (int k = 0; k < nfields; ++k) {
    *f[k] = (double*)q;
    q += fb;
  }
  if (nchain)
    for (int cc = 0; cc < c->ncomp; ++cc)
      for (int j = 0; j < 9; ++j)
        for (int h = 0; h < 2; ++h) {
          c->sY[cc][j][h] = (double*)q;
          q += cb;
        }
  c->part = (double*)q;
  return SETD_OK;
}

// d = 3: E = sum_k sum_t s_t sum_mu T(V_k, {P_kt with mode mu -> dP_kt,mu})
// for each chain (output k, term t) of one component, sharing the partial
// products between the three derivative Tuckers of a term: with
// X0 = V x1 P1, X1 = V x1 dP1 (mode 1), then X0 <- X0 x2 P2 and
// X1 <- X1 x2 P2 + X0 x2 dP2 (mode 2), the sum is X1 x3 P3 + X0 x3 dP3
// (mode 3): 7 mode products per term instead of 9.
struct SigmaChain {
  const double* V;
  void* const* P;    // packed bank matrices of the term
  void* const* dP;   // packed derivative matrices
  double scale;
  double* A0;        // mode-1 partials
  double* A1;
  double* B0;        // mode-2 partials
  double* B1;
};

int sigma_chains_d3(const int* dims, SigmaChain* ch, int nch, double* const* E, const double* const* Ebase,
                    int nout, int T, hipStream_t s) {
  const int64_t N = (int64_t)dims[0] * dims[1] * dims[2];
  std::vector<ModeJob> jobs;
  for (int k = 0; k < nch; ++k) {
    jobs.push_back(mk_job(ch[k].V, ch[k].P[0], 1.0, ch[k].A0, nullptr, 1, dims[0], N / dims[0]));
    jobs.push_back(mk_job(ch[k].V, ch[k].dP[0], 1.0, ch[k].A1, nullptr, 1, dims[0], N / dims[0]));
  }
  SETD_TRY(launch_f64_jobs(jobs, true, s));
  for (int k = 0; k < nch; ++k) {
    jobs.push_back(mk_job(ch[k].A0, ch[k].P[1], 1.0, ch[k].B0, nullptr, dims[0], dims[1], dims[2]));
    ModeJob jb = mk_job(ch[k].A1, ch[k].P[1], 1.0, ch[k].B1, nullptr, dims[0], dims[1], dims[2]);
    jb.nterms = 2;
    jb.X[1] = ch[k].A0;
    jb.P[1] = ch[k].dP[1];
    jb.scale[1] = 1.0;
    jobs.push_back(jb);
  }
  SETD_TRY(launch_f64_jobs(jobs, false, s));
  // mode 3: output o sums chains o*T .. o*T+T-1; first the X1 x3 P3 terms
  // (onto Ebase[o], or none), then the X0 x3 dP3 terms onto E[o]
  for (int pass = 0; pass < 2; ++pass) {
    for (int o = 0; o < nout; ++o) {
      ModeJob jb{};
      jb.nterms = T;
      for (int t = 0; t < T; ++t) {
        const SigmaChain& q = ch[o * T + t];
        jb.X[t] = pass == 0 ? q.B1 : q.B0;
        jb.P[t] = pass == 0 ? q.P[2] : q.dP[2];
        jb.scale[t] = q.scale;
      }
      jb.Y = E[o];
      jb.base = pass == 0 ? Ebase[o] : E[o];
      jb.na = (int64_t)dims[0] * dims[1];
      jb.nb = 1;
      jb.n = dims[2];
      jb.ldp = packed_ld(dims[2]);
      jobs.push_back(jb);
    }
    SETD_TRY(launch_f64_jobs(jobs, false, s));
  }
  return SETD_OK;
}

// A Tucker output with nterms terms of one bank entry.
TuckerOut mk_out(double* Y, const double* base, const void* X, void* const (*P)[3], double mult, const double* eta,
                 int T, double* const* y1, double* const* y2) {
  TuckerOut o;
  o.Y = Y;
  o.base = base;
  o.nterms = T;
  for (int t = 0; t < T; ++t) o.term[t] = {X, P[t], mult * eta[t], y1[t], y2[t]};
  return o;
}

int adjoint_step(setd_ctx* c, const double* u_in, const double* rec, double* ubar, const GParams& gp, int nparams,
                 int sigma_mask, double* grad, hipStream_t s) {
  const int d = c->d, nc = c->ncomp, T = c->nterms;
  const int64_t N = c->N;
  const double tau = c->tau;
  double* u = const_cast<double*>(u_in);   // read only below
  const int e21 = bank_index(SETD_STAGE_2, 1), e31 = bank_index(SETD_STAGE_3, 1), e32 = bank_index(SETD_STAGE_3, 2),
            ef1 = bank_index(SETD_STAGE_F, 1), ef2 = bank_index(SETD_STAGE_F, 2);
  const double* eta1 = c->sp[1].eta;
  const double* eta2 = c->sp[2].eta;
  auto at = [&](double* p, int cc) { return p + (int64_t)cc * N; };
  // ---- the step's stage quantities G, F, U2, D2, U3, D3: recorded by
  // setd_etd_step_record, or recomputed here ----
  const int64_t NC = (int64_t)nc * N;
  double* rw = const_cast<double*>(rec);   // read only below
  double* const sG = rec ? rw : c->G;
  double* const sF = rec ? rw + NC : c->F;
  double* const sU2 = rec ? rw + 2 * NC : c->U2;
  double* const sD2 = rec ? rw + 3 * NC : c->aD2;
  double* const sU3 = rec ? rw + 4 * NC : c->U3;
  double* const sD3 = rec ? rw + 5 * NC : c->aD3;
  if (!rec) {
    SETD_TRY(compute_gf(c, u, gp, s));
    {
      TuckerOut outs[4];
      int no = 0;
      for (int cc = 0; cc < nc; ++cc) {
        outs[no++] = mk_out(at(sU2, cc), at(u, cc), at(sF, cc), c->bank[cc][e21], tau / 3.0, eta1, T,
                            &c->Y1[cc][0], &c->Y2[cc][0]);
        outs[no++] = mk_out(at(sU3, cc), at(u, cc), at(sF, cc), c->bank[cc][e31], 2.0 * tau / 3.0, eta1, T,
                            &c->Y1[cc][T], &c->Y2[cc][T]);
      }
      SETD_TRY(run_tucker_group(d, c->dims, outs, no, SETD_PREC_F64, s));
    }
    SETD_TRY(launch_stage_d(sU2, sG, nc, N, gp, sD2, DType::F64, s));
    {
      TuckerOut outs[2];
      for (int cc = 0; cc < nc; ++cc)
        outs[cc] = mk_out(at(sU3, cc), at(sU3, cc), at(sD2, cc), c->bank[cc][e32], 4.0 * tau / 3.0, eta2, T,
                          &c->Y1[cc][0], &c->Y2[cc][0]);
      SETD_TRY(run_tucker_group(d, c->dims, outs, nc, SETD_PREC_F64, s));
    }
    SETD_TRY(launch_stage_d(sU3, sG, nc, N, gp, sD3, DType::F64, s));
  }

  // ---- diffusion-size derivatives of the split actions applied to their inputs ----
  // Ef = tau dS1(f) F + 3tau/2 dS2(f) D3, E3 = 2tau/3 dS1(3) F + 4tau/3 dS2(3) D2,
  // E2 = tau/3 dS1(2) F; dS V = sum_i eta_i sum_mu T(V, {P_i with P_{i,mu} -> dP_{i,mu}}).
  const bool dots = sigma_mask != 0;
  if (dots && d == 3) {
    for (int a = 0; a < 2; ++a)
      for (int cc = 0; cc < nc; ++cc) {
        if (!(sigma_mask & (1 << cc))) continue;
        struct {
          double* E;
          double* X;
          int e;
          double mult;
          const double* eta;
        } spec[3] = {
            {c->Ef, a == 0 ? sF : sD3, a == 0 ? ef1 : ef2, a == 0 ? tau : 1.5 * tau, a == 0 ? eta1 : eta2},
            {c->E3, a == 0 ? sF : sD2, a == 0 ? e31 : e32, a == 0 ? 2.0 * tau / 3.0 : 4.0 * tau / 3.0,
             a == 0 ? eta1 : eta2},
            {c->E2, sF, e21, tau / 3.0, eta1}};
        const int nout = a == 0 ? 3 : 2;   // E2 has a phi_1 action only
        SigmaChain ch[9];
        double* E[3];
        const double* Eb[3];
        for (int k = 0; k < nout; ++k) {
          E[k] = at(spec[k].E, cc);
          Eb[k] = a == 0 ? nullptr : E[k];   // the first pass overwrites
          for (int t = 0; t < T; ++t) {
            const int j = k * T + t;
            ch[j] = {at(spec[k].X, cc), c->bank[cc][spec[k].e][t], c->dbank[cc][spec[k].e][t],
                     spec[k].mult * spec[k].eta[t], c->Y1[cc][j], c->Y2[cc][j], c->sY[cc][j][0], c->sY[cc][j][1]};
          }
        }
        SETD_TRY(sigma_chains_d3(c->dims, ch, nout * T, E, Eb, nout, T, s));
      }
  } else if (dots) {
    void* mats[3][3][3];   // [output][term][mu]
    for (int a = 0; a < 2; ++a)
      for (int m0 = 0; m0 < d; ++m0) {
        TuckerOut outs[6];
        int no = 0;
        for (int cc = 0; cc < nc; ++cc) {
          if (!(sigma_mask & (1 << cc))) continue;
          struct {
            double* E;
            double* X;
            int e;
            double mult;
            const double* eta;
          } spec[3] = {
              {c->Ef, a == 0 ? sF : sD3, a == 0 ? ef1 : ef2, a == 0 ? tau : 1.5 * tau, a == 0 ? eta1 : eta2},
              {c->E3, a == 0 ? sF : sD2, a == 0 ? e31 : e32, a == 0 ? 2.0 * tau / 3.0 : 4.0 * tau / 3.0,
               a == 0 ? eta1 : eta2},
              {c->E2, sF, e21, tau / 3.0, eta1}};
          const int nout = a == 0 ? 3 : 2;   // E2 has a phi_1 action only
          for (int k = 0; k < nout; ++k) {
            double* E = at(spec[k].E, cc);
            TuckerOut& o = outs[no++];
            o.Y = E;
            o.base = (a == 0 && m0 == 0) ? nullptr : E;   // the first pass overwrites
            o.nterms = T;
            for (int t = 0; t < T; ++t) {
              for (int mu = 0; mu < d; ++mu)
                mats[k][t][mu] = mu == m0 ? c->dbank[cc][spec[k].e][t][mu] : c->bank[cc][spec[k].e][t][mu];
              o.term[t] = {at(spec[k].X, cc), mats[k][t], spec[k].mult * spec[k].eta[t], c->Y1[cc][k * T + t],
                           c->Y2[cc][k * T + t]};
            }
          }
          // run per component: the matrix arrays in `mats` are reused
          SETD_TRY(run_tucker_group(d, c->dims, outs, no, SETD_PREC_F64, s));
          no = 0;
        }
      }
  }

  // ---- backward ----
  // U' = U + tau S1(f) F + 3tau/2 S2(f) D3
  {
    TuckerOut outs[4];
    int no = 0;
    for (int cc = 0; cc < nc; ++cc) {
      outs[no++] = mk_out(at(c->Fbar, cc), nullptr, at(ubar, cc), c->bankT[cc][ef1], tau, eta1, T, &c->Y1[cc][0],
                          &c->Y2[cc][0]);
      outs[no++] = mk_out(at(c->Dbar, cc), nullptr, at(ubar, cc), c->bankT[cc][ef2], 1.5 * tau, eta2, T,
                          &c->Y1[cc][T], &c->Y2[cc][T]);
    }
    SETD_TRY(run_tucker_group(d, c->dims, outs, no, SETD_PREC_F64, s));
  }
  const dim3 rg(kRedBlocks), rb(kRedThreads);
  // D3 = g(U3) - G
  hipLaunchKernelGGL(adj_stage_kernel, rg, rb, 0, s, sU3, c->Dbar, nc, N, gp, c->U3bar, c->Gbar, true, c->part,
                     kRowP1);
  SETD_LAUNCHED();
  // U3 = U + 2tau/3 S1(3) F + 4tau/3 S2(3) D2
  {
    TuckerOut outs[4];
    int no = 0;
    for (int cc = 0; cc < nc; ++cc) {
      outs[no++] = mk_out(at(c->Fbar, cc), at(c->Fbar, cc), at(c->U3bar, cc), c->bankT[cc][e31], 2.0 * tau / 3.0,
                          eta1, T, &c->Y1[cc][0], &c->Y2[cc][0]);
      outs[no++] = mk_out(at(c->Dbar, cc), nullptr, at(c->U3bar, cc), c->bankT[cc][e32], 4.0 * tau / 3.0, eta2, T,
                          &c->Y1[cc][T], &c->Y2[cc][T]);
    }
    SETD_TRY(run_tucker_group(d, c->dims, outs, no, SETD_PREC_F64, s));
  }
  // D2 = g(U2) - G
  hipLaunchKernelGGL(adj_stage_kernel, rg, rb, 0, s, sU2, c->Dbar, nc, N, gp, c->U2bar, c->Gbar, false, c->part,
                     kRowP2);
  SETD_LAUNCHED();
  // U2 = U + tau/3 S1(2) F
  {
    TuckerOut outs[2];
    for (int cc = 0; cc < nc; ++cc)
      outs[cc] = mk_out(at(c->Fbar, cc), at(c->Fbar, cc), at(c->U2bar, cc), c->bankT[cc][e21], tau / 3.0, eta1, T,
                        &c->Y1[cc][0], &c->Y2[cc][0]);
    SETD_TRY(run_tucker_group(d, c->dims, outs, nc, SETD_PREC_F64, s));
  }
  if (dots) {
    hipLaunchKernelGGL(adj_dots_kernel, rg, rb, 0, s, c->Ef, ubar, c->E3, c->U3bar, c->E2, c->U2bar, nc, N,
                       c->part);
    SETD_LAUNCHED();
  }
  // F = K U + G: K^T Fbar (dense path: mu-mode products with the A_mu^T)
  const double* ktf = nullptr;
  if (!c->tridiag) {
    for (int cc = 0; cc < nc; ++cc) {
      double* out = at(c->KtF, cc);
      const double* fb = at(c->Fbar, cc);
      ModeJobs J;
      J.njobs = 1;
      J.job[0] = mk_job(fb, c->ApkT[cc][0], 1.0, out, nullptr, 1, c->dims[0], N / c->dims[0]);
      SETD_TRY(launch_mode1_f64(J, s));
      int64_t na = c->dims[0];
      for (int mu = 1; mu < d; ++mu) {
        J.njobs = 1;
        J.job[0] = mk_job(fb, c->ApkT[cc][mu], 1.0, out, out, na, c->dims[mu], N / (na * c->dims[mu]));
        SETD_TRY(launch_modeB_f64(J, s));
        na *= c->dims[mu];
      }
    }
    ktf = c->KtF;
  }
  const int n3 = d == 3 ? c->dims[2] : 1;
  hipLaunchKernelGGL(adj_final_kernel, rg, rb, 0, s, u, ubar, c->U3bar, c->U2bar, c->Fbar, c->Gbar, sF, sG, ktf,
                     nc, N, d, c->dims[0], c->dims[1], n3, c->st, gp, c->part);
  SETD_LAUNCHED();
  hipLaunchKernelGGL(adj_reduce_kernel, dim3(1), dim3(64), 0, s, c->part, nparams, nc, sigma_mask, dots, grad);
  SETD_LAUNCHED();
  return SETD_OK;
}

}  // namespace
}  // namespace setd

using namespace setd;

extern "C" int setd_etd_adjoint_step(setd_ctx* c, const double* u, double* ubar, int g_kind, const double* params,
                                     int nparams, int sigma_mask, double* grad, void* stream) {
  clear_error();
  SETD_CHECK_ARG(c != nullptr, "ctx is NULL");
  SETD_CHECK_ARG(u != nullptr && ubar != nullptr, "u and ubar must be non-NULL");
  SETD_CHECK_ARG(sigma_mask >= 0 && sigma_mask < (1 << c->ncomp), "sigma_mask %d has bits beyond the components",
                 sigma_mask);
  SETD_CHECK_ARG(grad != nullptr || (nparams == 0 && sigma_mask == 0), "grad is NULL");
  SETD_CHECK_ARG(!overlap(u, c->ncomp * c->N * 8, ubar, c->ncomp * c->N * 8), "u and ubar overlap");
  if (c->prec != SETD_PREC_F64) {
    set_error("the adjoint step runs in FP64 only");
    return SETD_EUNSUPPORTED;
  }
  GParams gp;
  SETD_TRY(make_gparams(g_kind, params, nparams, c->ncomp, gp));
  hipStream_t s = (hipStream_t)stream;
  if (c->adj_bank_mem.p == nullptr || c->adj_tau != c->tau) SETD_TRY(build_adjoint_bank(c, s));
  if (c->adj_mem.p == nullptr) SETD_TRY(alloc_adjoint_buffers(c));
  return adjoint_step(c, u, nullptr, ubar, gp, nparams, sigma_mask, grad, s);
}

extern "C" int setd_etd_adjoint_step_recorded(setd_ctx* c, const double* u, const double* rec, double* ubar,
                                              int g_kind, const double* params, int nparams, int sigma_mask,
                                              double* grad, void* stream) {
  clear_error();
  SETD_CHECK_ARG(c != nullptr, "ctx is NULL");
  SETD_CHECK_ARG(u != nullptr && rec != nullptr && ubar != nullptr, "u, rec and ubar must be non-NULL");
  SETD_CHECK_ARG(sigma_mask >= 0 && sigma_mask < (1 << c->ncomp), "sigma_mask %d has bits beyond the components",
                 sigma_mask);
  SETD_CHECK_ARG(grad != nullptr || (nparams == 0 && sigma_mask == 0), "grad is NULL");
  const int64_t NC = c->ncomp * c->N;
  SETD_CHECK_ARG(!overlap(u, NC * 8, ubar, NC * 8), "u and ubar overlap");
  SETD_CHECK_ARG(!overlap(rec, 6 * NC * 8, ubar, NC * 8), "rec and ubar overlap");
  if (c->prec != SETD_PREC_F64) {
    set_error("the adjoint step runs in FP64 only");
    return SETD_EUNSUPPORTED;
  }
  GParams gp;
  SETD_TRY(make_gparams(g_kind, params, nparams, c->ncomp, gp));
  hipStream_t s = (hipStream_t)stream;
  if (c->adj_bank_mem.p == nullptr || c->adj_tau != c->tau) SETD_TRY(build_adjoint_bank(c, s));
  if (c->adj_mem.p == nullptr) SETD_TRY(alloc_adjoint_buffers(c));
  return adjoint_step(c, u, rec, ubar, gp, nparams, sigma_mask, grad, s);
}
