// The integration context (setd_ctx of setd.h) and the Tucker-group runner
// shared by the forward step (setd_api.hip) and the adjoint step
// (adjoint.hip).  Internal to libsetd.
#pragma once

#include <vector>

#include "api_util.hpp"
#include "coeffs.hpp"
#include "common.hpp"
#include "pointwise.hpp"

struct setd_ctx {
  int d = 0, ncomp = 0, prec = SETD_PREC_F64;
  int dims[3] = {1, 1, 1};
  int64_t N = 0;
  double tau = 0.0;
  std::vector<double> Ah[2][3];
  bool tridiag = false;
  setd::StencilSet st{};
  setd::Splitting sp[3];
  int nterms = 0;
  void* bank[2][5][3][3] = {};   // [comp][entry][term][mu] packed FP64 matrix
  void* Apk[2][3] = {};          // packed A for the dense K path
  void* bank2[2][2][3] = {};     // [comp][ell-1][mu] phi_ell(tau A_mu) for etd2rkds
  double *G = nullptr, *F = nullptr, *U2 = nullptr, *U3 = nullptr, *W = nullptr, *D = nullptr;
  double* Y1[2][9] = {};
  double* Y2[2][9] = {};
  double* aux = nullptr;         // FP32 copy of a split_phi_apply input (reduced precision)
  setd::DevBuf i8_mem;           // int8 digit buffers of the Tucker inputs (SETD_PREC_I8X4)
  setd::DevBuf A_mem, stencil_mem, bank_mem, work_mem;
  // one captured step (hipGraph), replayed per step on an internal stream
  hipStream_t gstream = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  double* g_u = nullptr;
  setd::GParams g_gp{};
  const void* g_fn = nullptr;    // which step function the graph holds
  // adjoint step (set up by its first call; rebuilt when tau changes)
  double adj_tau = 0.0;
  setd::DevBuf adj_bank_mem, adj_mem;
  void* bankT[2][5][3][3] = {};   // transposed phi matrices, packed for the forward kernels
  void* dbank[2][5][3][3] = {};   // d/dsigma phi matrices at sigma = 1
  void* ApkT[2][3] = {};          // transposed A (dense K path)
  double *aD2 = nullptr, *aD3 = nullptr, *Fbar = nullptr, *Dbar = nullptr, *Gbar = nullptr;
  double *U3bar = nullptr, *U2bar = nullptr, *Ef = nullptr, *E3 = nullptr, *E2 = nullptr, *KtF = nullptr;
  double* sY[2][9][2] = {};   // d = 3: mode-2 partials of the diffusion-size derivative chains
  double* part = nullptr;         // per-block partial sums of the gradient reductions
  // exprk3ds_cplx (set up by its first step; rebuilt when tau changes)
  double cplx_tau = 0.0;
  setd::DevBuf cplx_bank_mem, cplx_mem;
  void* cbank[2][5][2][3][2] = {};   // [comp][entry][term][mu][re, im]; last mu: eta folded in
  double* cY[2][24] = {};            // complex intermediates (re, im planes)
  ~setd_ctx() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (gstream) (void)hipStreamDestroy(gstream);
  }
};

namespace setd {

// One Tucker-summed output: Y = base + sum_t scale_t T(X_t, {P_t[mu]}).
struct TuckerTerm {
  const void* X;        // FP64, or FP32 for the reduced-precision forms
  void* const* P;       // d packed matrices (layout per pack_for)
  double scale;
  void* Y1;             // intermediates, same type as X
  void* Y2;
};
struct TuckerOut {
  double* Y;
  const double* base;
  int nterms;
  TuckerTerm term[kMaxTerms];
  // SETD_PREC_I8X4 in the order 3, 1, 2 (i8_order312): the terms' X are
  // already digit buffers along the last mode (launch_stage_slice_i8)
  bool x_sliced = false;
};

// Runs all outputs of a group: d grouped launches (or more if a launch would
// exceed kMaxJobs).  dims has d >= 2 entries.  With a reduced-precision
// `prec`, term inputs and Y1/Y2 are FP32 and the outputs FP64.
// SETD_PREC_I8X4 needs digit buffers of i8_slot_bytes each (i8ws): one per
// distinct input of a launch, and for the fused forms one (mode 1 -> mode 2,
// n2 in {128, 256}) or two (d = 3 in the order 3, 1, 2 with n1 and n2 in
// {128, 256}) per chain (term of an output) besides; without room for them
// a group runs the less fused form.
int run_tucker_group(int d, const int* dims, TuckerOut* outs, int nouts, int prec, hipStream_t s,
                     void* i8ws = nullptr, size_t i8bytes = 0);
// Bytes of one int8 digit buffer for any mode of the grid.
size_t i8_slot_bytes(int d, const int* dims);
// Whether run_tucker_group takes a d = 3 group of nchains chains in the
// order 3, 1, 2 (SETD_PREC_I8X4, n1 and n2 in {128, 256}, n3 <= 256, room
// for 2 nchains + 2 digit buffers).  The first 2 nchains buffers of the
// workspace then hold the digits emitted between the products, and buffers
// 2 nchains and 2 nchains + 1 may hold presliced inputs
// (TuckerOut::x_sliced).
bool i8_order312(int d, const int* dims, int nchains, size_t i8bytes);
// Whether the int8 form's products emit the next operand's digits
// (environment variable SETD_I8_EMIT not 0).
bool i8_emit();
// Packs a matrix for the mode kernels of the given arithmetic and direction.
int pack_for(int prec, const double* M, int n, double scale, int mu, void* out, hipStream_t s);
// G = g(U) (FP64) and F = K U + G in the Tucker arithmetic's storage type,
// into c->G and c->F, or into G and F when given (FP64 contexts).
int compute_gf(setd_ctx* c, double* u, const GParams& gp, hipStream_t s, double* G = nullptr, void* F = nullptr);
// The stage quantities of one exprk3ds_real step, each ncomp * N: G = g(U),
// F = K U + G, U2, D2 = g(U2) - G, U3, D3 = g(U3) - G.  F, D2 and D3 are in
// the Tucker arithmetic's storage type.
struct StageBufs {
  double* G;
  void* F;
  double* U2;
  void* D2;
  double* U3;
  void* D3;
};
// One step that keeps its stage quantities in `b` (setd_etd_step_record).
int step_with(setd_ctx* c, double* u, const GParams& gp, hipStream_t s, const StageBufs& b);
// Launches FP64 mode-product jobs of one regime in groups of kMaxJobs.
int launch_f64_jobs(std::vector<ModeJob>& jobs, bool mode1, hipStream_t s);
// exprk3ds_cplx (cplx.hip): complex phi bank for step size tau (synchronises
// s; no-op when already built for tau) and one step.
int prepare_cplx(setd_ctx* c, double tau, hipStream_t s);
int step_cplx_once(setd_ctx* c, double* u, const GParams& gp, hipStream_t s);

}  // namespace setd
