// exprk3ds_cplx: the split-ETD3 step with the two-term complex splitting
// (Table 1 complex column for d = 2, Table 2 for d > 2): every split action
// is S_l(c tau) V = Re sum_{i=1,2} eta_i T(V, {phi_{l_i}(c tau alpha_i A_mu)})
// with complex eta_i, alpha_i; the exact phi_l(tau K) V is real and the
// imaginary part of the sum is O(tau^3), so the real part is kept.
//
// Complex arithmetic on the real FP64 kernels:
//   * phi of the complex matrix z A is computed through its real 2n x 2n
//     representation [[Re, -Im], [Im, Re]] (an algebra homomorphism, so
//     phi of the representation represents phi of the matrix): the same
//     Pade / scaling-and-squaring builder as for the real bank;
//   * mode 1 on the real input: Y_r = P_r X, Y_i = P_i X (two jobs);
//   * inner modes: Z_r = Y_r x P_r - Y_i x P_i, Z_i = Y_r x P_i + Y_i x P_r
//     (two-term jobs of the modes >= 2 kernel);
//   * last mode, real part only, with eta folded into the matrices:
//     Re(eta P Y) = Q_r Y_r + Q_i Y_i, Q_r = Re(eta P), Q_i = -Im(eta P);
//     the two Tucker terms of an action are accumulated in two launches.
// A complex Tucker costs 2 + 4 (d - 2) + 2 real mode products against d for
// a real one, so this variant does more work per step than exprk3ds_real
// (two complex Tuckers against three real ones per action for d = 3).
#include <cmath>

#include "ctx.hpp"

namespace setd {
namespace {

// B = [[ar A, -ai A], [ai A, ar A]] (2n x 2n, column-major) for n x n A.
__global__ void embed_complex_kernel(const double* __restrict__ A, int n, double ar, double ai,
                                     double* __restrict__ B) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t m = 2 * (int64_t)n;
  if (idx >= m * m) return;
  const int r = (int)(idx % m), c = (int)(idx / m);
  const int i = r % n, p = c % n;
  const double a = A[i + (int64_t)n * p];
  const bool top = r < n, left = c < n;
  double v;
  if (top == left) v = ar * a;          // diagonal blocks: Re
  else if (!top && left) v = ai * a;    // lower left: Im
  else v = -ai * a;                     // upper right: -Im
  B[idx] = v;
}

// Copies the n x n block at (r0, 0) of a 2n x 2n column-major matrix.
int extract_block(const double* B, int n, int r0, double* out, hipStream_t s) {
  SETD_HIP(hipMemcpy2DAsync(out, (size_t)n * sizeof(double), B + r0, (size_t)2 * n * sizeof(double),
                            (size_t)n * sizeof(double), (size_t)n, hipMemcpyDeviceToDevice, s));
  return SETD_OK;
}

int build_cplx_bank(setd_ctx* c, double tau, hipStream_t s) {
  const int d = c->d;
  size_t bytes = 0;
  for (int cc = 0; cc < c->ncomp; ++cc)
    for (int mu = 0; mu < d; ++mu) bytes += 5 * 2 * 2 * packed_bytes(c->dims[mu], SETD_PREC_F64);
  SETD_TRY(c->cplx_bank_mem.alloc(bytes));
  char* q = (char*)c->cplx_bank_mem.p;
  const SplittingC sc[3] = {SplittingC{}, splitting_cplx(1, d), splitting_cplx(2, d)};
  for (int cc = 0; cc < c->ncomp; ++cc)
    for (int mu = 0; mu < d; ++mu) {
      const int n = c->dims[mu];
      const size_t nn = (size_t)n * n, mm = 4 * nn;
      const bool rowmajor = mu == 0, last = mu == d - 1;
      DevBuf A, B, raw, Pr, Pi, Qr, Qi;
      SETD_TRY(A.alloc(nn * 8));
      SETD_TRY(B.alloc(mm * 8));
      SETD_TRY(Pr.alloc(nn * 8));
      SETD_TRY(Pi.alloc(nn * 8));
      SETD_TRY(Qr.alloc(nn * 8));
      SETD_TRY(Qi.alloc(nn * 8));
      SETD_HIP(hipMemcpyAsync(A.p, c->Ah[cc][mu].data(), nn * 8, hipMemcpyHostToDevice, s));
      for (int ell = 1; ell <= 2; ++ell)
        for (int t = 0; t < 2; ++t) {
          const SplittingC& S = sc[ell];
          const int li = t + 1;   // phi index of term t
          hipLaunchKernelGGL(embed_complex_kernel, dim3((unsigned)ceil_div((int64_t)mm, 256)), dim3(256), 0, s,
                             (const double*)A.p, n, S.al_r[t], S.al_i[t], (double*)B.p);
          SETD_LAUNCHED();
          // the stages that use phi_ell: scalars c_s tau
          std::vector<int> ents;
          std::vector<double> scal;
          for (int e = 0; e < 5; ++e)
            if (kBankEll[e] == ell) {
              ents.push_back(e);
              scal.push_back(stage_scale(kBankStage[e]) * tau);
            }
          const int E = (int)scal.size();
          SETD_TRY(raw.alloc((size_t)E * 3 * mm * 8));
          std::vector<double*> outs(E * 3);
          for (int k = 0; k < E * 3; ++k) outs[k] = (double*)raw.p + (size_t)k * mm;
          SETD_TRY(phi_batch((const double*)B.p, 2 * n, scal.data(), E, 2, outs.data(), s));
          for (int k = 0; k < E; ++k) {
            const double* P = outs[k * 3 + li];
            SETD_TRY(extract_block(P, n, 0, (double*)Pr.p, s));   // Re: upper-left block
            SETD_TRY(extract_block(P, n, n, (double*)Pi.p, s));   // Im: lower-left block
            const double* src_r = (const double*)Pr.p;
            const double* src_i = (const double*)Pi.p;
            if (last) {
              // Q_r = er P_r - ei P_i, Q_i = -(er P_i + ei P_r)
              const double er = S.eta_r[t], ei = S.eta_i[t];
              SETD_HIP(hipMemcpyAsync(Qr.p, Pr.p, nn * 8, hipMemcpyDeviceToDevice, s));
              SETD_TRY(launch_axpby((const double*)Pi.p, (double*)Qr.p, (int64_t)nn, -ei, er, s));
              SETD_HIP(hipMemcpyAsync(Qi.p, Pi.p, nn * 8, hipMemcpyDeviceToDevice, s));
              SETD_TRY(launch_axpby((const double*)Pr.p, (double*)Qi.p, (int64_t)nn, -ei, -er, s));
              src_r = (const double*)Qr.p;
              src_i = (const double*)Qi.p;
            }
            void** slot = c->cbank[cc][ents[k]][t][mu];
            slot[0] = q;
            SETD_TRY(pack_matrix_f64(src_r, n, 1.0, rowmajor, (double*)q, s));
            q += packed_bytes(n, SETD_PREC_F64);
            slot[1] = q;
            SETD_TRY(pack_matrix_f64(src_i, n, 1.0, rowmajor, (double*)q, s));
            q += packed_bytes(n, SETD_PREC_F64);
          }
          SETD_HIP(hipStreamSynchronize(s));   // raw is reused by the next (ell, t)
        }
      SETD_HIP(hipStreamSynchronize(s));
    }
  c->cplx_tau = tau;
  return SETD_OK;
}

// One output of a complex group: Y = base + mult Re(sum_t eta_t T(X_t, {P_t}))
// with the matrices of bank entry e (eta inside the last-mode matrices).
struct CplxOut {
  double* Y;
  const double* base;
  const double* X;
  int comp, e;
  double mult;
  int slot;   // first complex intermediate pair: uses slots slot..slot+1 (one per term)
};

int run_cplx_group(setd_ctx* c, const CplxOut* outs, int nouts, hipStream_t s) {
  const int d = c->d;
  const int64_t N = c->N;
  std::vector<ModeJob> jobs;
  // intermediates of term t of output o: Y1 (re, im) and, for d = 3, Y2 (re, im)
  auto buf = [&](const CplxOut& o, int t, int stage, int part) {
    const int k = (o.slot + t) * (d == 3 ? 4 : 2) + stage * 2 + part;
    return c->cY[o.comp][k];
  };
  for (int o = 0; o < nouts; ++o)
    for (int t = 0; t < 2; ++t)
      for (int part = 0; part < 2; ++part) {
        const CplxOut& out = outs[o];
        jobs.push_back(mk_job(out.X, c->cbank[out.comp][out.e][t][0][part], 1.0, buf(out, t, 0, part), nullptr, 1,
                              c->dims[0], N / c->dims[0]));
      }
  SETD_TRY(launch_f64_jobs(jobs, true, s));
  int64_t na = c->dims[0];
  int cur = 0;   // stage index of the current intermediates
  for (int mu = 1; mu < d - 1; ++mu) {
    const int64_t nb = N / (na * c->dims[mu]);
    for (int o = 0; o < nouts; ++o)
      for (int t = 0; t < 2; ++t) {
        const CplxOut& out = outs[o];
        void* const* P = c->cbank[out.comp][out.e][t][mu];
        for (int part = 0; part < 2; ++part) {
          // re: Y_r P_r - Y_i P_i;  im: Y_r P_i + Y_i P_r
          ModeJob jb = mk_job(buf(out, t, cur, 0), P[part], 1.0, buf(out, t, 1 - cur, part), nullptr, na,
                              c->dims[mu], nb);
          jb.nterms = 2;
          jb.X[1] = buf(out, t, cur, 1);
          jb.P[1] = P[1 - part];
          jb.scale[1] = part == 0 ? -1.0 : 1.0;
          jobs.push_back(jb);
        }
      }
    SETD_TRY(launch_f64_jobs(jobs, false, s));
    cur = 1 - cur;
    na *= c->dims[mu];
  }
  const int mu = d - 1;
  for (int t = 0; t < 2; ++t) {
    for (int o = 0; o < nouts; ++o) {
      const CplxOut& out = outs[o];
      void* const* Q = c->cbank[out.comp][out.e][t][mu];
      ModeJob jb = mk_job(buf(out, t, cur, 0), Q[0], out.mult, out.Y, t == 0 ? out.base : out.Y, na, c->dims[mu], 1);
      jb.nterms = 2;
      jb.X[1] = buf(out, t, cur, 1);
      jb.P[1] = Q[1];
      jb.scale[1] = out.mult;
      jobs.push_back(jb);
    }
    SETD_TRY(launch_f64_jobs(jobs, false, s));
  }
  return SETD_OK;
}

}  // namespace

int prepare_cplx(setd_ctx* c, double tau, hipStream_t s) {
  if (!c->cplx_mem.p) {
    const int per = c->d == 3 ? 4 : 2;          // planes per complex term
    const int nslots = 6;                       // 3 outputs x 2 terms
    const size_t fb = round_up(c->N * 8, 256);
    SETD_TRY(c->cplx_mem.alloc((size_t)c->ncomp * nslots * per * fb));
    char* q = (char*)c->cplx_mem.p;
    for (int cc = 0; cc < c->ncomp; ++cc)
      for (int k = 0; k < nslots * per; ++k) {
        c->cY[cc][k] = (double*)q;
        q += fb;
      }
  }
  if (c->cplx_bank_mem.p == nullptr || c->cplx_tau != tau) SETD_TRY(build_cplx_bank(c, tau, s));
  return SETD_OK;
}

// One exprk3ds_cplx step: the stages of step_once with complex split actions.
int step_cplx_once(setd_ctx* c, double* u, const GParams& gp, hipStream_t s) {
  const int nc = c->ncomp;
  const int64_t N = c->N;
  const double tau = c->tau;
  const int e21 = bank_index(SETD_STAGE_2, 1), e31 = bank_index(SETD_STAGE_3, 1), e32 = bank_index(SETD_STAGE_3, 2),
            ef1 = bank_index(SETD_STAGE_F, 1), ef2 = bank_index(SETD_STAGE_F, 2);
  SETD_TRY(compute_gf(c, u, gp, s));
  {
    CplxOut outs[6];
    int no = 0;
    for (int cc = 0; cc < nc; ++cc) {
      const int64_t o = cc * N;
      outs[no++] = {c->U2 + o, u + o, c->F + o, cc, e21, tau / 3.0, 0};
      outs[no++] = {c->U3 + o, u + o, c->F + o, cc, e31, 2.0 * tau / 3.0, 2};
      outs[no++] = {c->W + o, u + o, c->F + o, cc, ef1, tau, 4};
    }
    SETD_TRY(run_cplx_group(c, outs, no, s));
  }
  SETD_TRY(launch_stage_d(c->U2, c->G, nc, N, gp, c->D, DType::F64, s));
  {
    CplxOut outs[2];
    for (int cc = 0; cc < nc; ++cc)
      outs[cc] = {c->U3 + cc * N, c->U3 + cc * N, c->D + cc * N, cc, e32, 4.0 * tau / 3.0, 0};
    SETD_TRY(run_cplx_group(c, outs, nc, s));
  }
  SETD_TRY(launch_stage_d(c->U3, c->G, nc, N, gp, c->D, DType::F64, s));
  {
    CplxOut outs[2];
    for (int cc = 0; cc < nc; ++cc) outs[cc] = {u + cc * N, c->W + cc * N, c->D + cc * N, cc, ef2, 1.5 * tau, 0};
    SETD_TRY(run_cplx_group(c, outs, nc, s));
  }
  return SETD_OK;
}

}  // namespace setd
