// C ABI of libsetd: argument checking, the phi bank, and the orchestration of
// the split-ETD3 step (the time loop of Algorithms 1 and 2) on top of the
// mode-product and pointwise kernels.
//
// One step, for both components at once (g couples them pointwise):
//   1. G = g(U), F = K U + G                                 (pointwise/stencil)
//   2. the phi_1 Tuckers on F for the three stages (3 x nterms per
//      component) in three grouped launches (one per mode); the last mode
//      sums the terms of each split phi action along the contraction and adds
//      U:  U2 = U + tau/3 S_1(tau/3) F,  U3 = U + 2tau/3 S_1(2tau/3) F,
//          W  = U + tau S_1(tau) F
//   3. D = g(U2) - G
//   4. U3 += 4tau/3 S_2(2tau/3) D
//   5. D = g(U3) - G
//   6. U  = W + 3tau/2 S_2(tau) D
// Every split phi action S_l(c tau) V = sum_i eta_i T(V, {P_{i,s}^(l){mu}})
// (eqs. split2d / splitnd3) costs nterms Tuckers of d mu-mode products.
#include <cmath>
#include <cstdarg>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "coeffs.hpp"
#include "common.hpp"
#include "pointwise.hpp"
#include "api_util.hpp"
#include "ctx.hpp"

namespace setd {

static thread_local char g_err[1024];

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
}
void clear_error() { g_err[0] = 0; }

// Largest tensor setd_tucker_apply accepts: 2^36 elements (512 GiB in FP64,
// more than one GPU holds); keeps every size product far from overflow.
constexpr int64_t kMaxTuckerElems = int64_t(1) << 36;

// ---- kernel timing ----
namespace {
struct ProfRec {
  hipEvent_t b, e;
  int cls;
  double flops, bytes;
};
std::mutex g_prof_mu;
bool g_prof = false;
std::vector<ProfRec> g_recs;
std::vector<hipEvent_t> g_free_events;

hipEvent_t get_event() {
  if (!g_free_events.empty()) {
    hipEvent_t e = g_free_events.back();
    g_free_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

bool prof_on() { return g_prof; }

ProfScope::ProfScope(hipStream_t s, int cls, double flops, double bytes) : s_(s), slot_(-1) {
  if (!g_prof) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  ProfRec r{get_event(), get_event(), cls, flops, bytes};
  if (!r.b || !r.e) return;
  if (hipEventRecord(r.b, s) != hipSuccess) return;
  g_recs.push_back(r);
  slot_ = (int)g_recs.size() - 1;
}

ProfScope::~ProfScope() {
  if (slot_ < 0) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  (void)hipEventRecord(g_recs[slot_].e, s_);
}

namespace {



}  // namespace
}  // namespace setd

using namespace setd;


namespace {



// How a table of jobs is launched: which regime, which arithmetic, and the
// output type (FP64 for the last mode of a Tucker; the reduced-precision
// forms keep their intermediates in FP32).
struct LaunchKind {
  bool mode1;
  int prec;
  DType out;
  void* i8ws = nullptr;      // digit buffers (SETD_PREC_I8X4)
  size_t i8bytes = 0;
  bool presliced = false;    // I8X4: the jobs' inputs are digit buffers already
  int fuse_next = 0;         // I8X4, mode 1: emit the mode-2 digits of this n2
};

int launch_jobs(ModeJobs& J, const LaunchKind& k, hipStream_t s) {
  if (k.prec == SETD_PREC_F64) return k.mode1 ? launch_mode1_f64(J, s) : launch_modeB_f64(J, s);
  if (k.prec == SETD_PREC_I8X4) return launch_mode_i8(J, k.mode1, k.i8ws, k.i8bytes, s, k.presliced, k.fuse_next);
  return k.mode1 ? launch_mode1_lp(J, k.prec, k.out, s) : launch_modeB_lp(J, k.prec, k.out, s);
}

int flush(ModeJobs& J, const LaunchKind& k, hipStream_t s) {
  if (J.njobs == 0) return SETD_OK;
  int rc = launch_jobs(J, k, s);
  J.njobs = 0;
  return rc;
}

int push(ModeJobs& J, const ModeJob& jb, const LaunchKind& k, hipStream_t s) {
  if (J.njobs == kMaxJobs) SETD_TRY(flush(J, k, s));
  J.job[J.njobs++] = jb;
  return SETD_OK;
}

// Packs a matrix for the mode kernels of the given arithmetic: mode 1 reads
// it row-major; modes >= 2 column-major (FP64, FP32) or row-major (bf16).
}  // namespace

int setd::pack_for(int prec, const double* M, int n, double scale, int mu, void* out, hipStream_t s) {
  if (prec == SETD_PREC_F64) return pack_matrix_f64(M, n, scale, mu == 0, (double*)out, s);
  if (prec == SETD_PREC_F32) return pack_matrix_f32(M, n, scale, mu == 0, (float*)out, s);
  if (prec == SETD_PREC_I8X4) return pack_matrix_i8(M, n, scale, out, s);
  return pack_matrix_bf16(M, n, scale, true, prec == SETD_PREC_BF16X3 ? 3 : 2, out, s);
}

namespace {

// Runs all outputs of a group: d grouped launches (or more if a launch
// would exceed kMaxJobs).  dims has d >= 2 entries.  With a reduced-precision
// `prec`, term inputs and Y1/Y2 are FP32 and the outputs FP64.
}  // namespace

int setd::launch_f64_jobs(std::vector<ModeJob>& jobs, bool mode1, hipStream_t s) {
  ModeJobs J;
  J.njobs = 0;
  for (const ModeJob& jb : jobs) {
    J.job[J.njobs++] = jb;
    if (J.njobs == kMaxJobs) {
      SETD_TRY(mode1 ? launch_mode1_f64(J, s) : launch_modeB_f64(J, s));
      J.njobs = 0;
    }
  }
  if (J.njobs) SETD_TRY(mode1 ? launch_mode1_f64(J, s) : launch_modeB_f64(J, s));
  jobs.clear();
  return SETD_OK;
}

size_t setd::i8_slot_bytes(int d, const int* dims) {
  int64_t N = 1;
  for (int mu = 0; mu < d; ++mu) N *= dims[mu];
  size_t b = 0;
  for (int mu = 0; mu < d; ++mu) b = std::max(b, i8_digit_bytes(N, dims[mu]));
  return b;
}

namespace {
bool i8_emit_on() {
  // SETD_I8_EMIT=0 makes every product write its FP64 result and the next one
  // slice it (same order of the modes): the emitted digits must equal these
  const char* e = std::getenv("SETD_I8_EMIT");
  return e == nullptr || e[0] != '0';
}
bool fusable_side(int m) { return m == 128 || m == 256; }
}  // namespace

bool setd::i8_order312(int d, const int* dims, int nchains, size_t i8bytes) {
  return d == 3 && fusable_side(dims[0]) && fusable_side(dims[1]) && dims[2] <= 256 &&
         (size_t)(2 * nchains + 2) * i8_slot_bytes(d, dims) <= i8bytes;
}

bool setd::i8_emit() { return i8_emit_on(); }

int setd::run_tucker_group(int d, const int* dims, TuckerOut* outs, int nouts, int prec, hipStream_t s,
                           void* i8ws, size_t i8bytes) {
  int64_t N = 1;
  for (int mu = 0; mu < d; ++mu) N *= dims[mu];
  const DType mid = fp32_storage(prec) ? DType::F32 : DType::F64;
  int nchains = 0;
  for (int o = 0; o < nouts; ++o) nchains += outs[o].nterms;
  const size_t slot = prec == SETD_PREC_I8X4 ? i8_slot_bytes(d, dims) : 0;
  const bool emit = i8_emit_on();
  bool sliced_in = false;
  for (int o = 0; o < nouts; ++o) sliced_in = sliced_in || outs[o].x_sliced;
  // I8X4, d = 3, n1 and n2 in {128, 256}, n3 <= 256: the products run in the
  // order 3, 1, 2 (the modes commute), so that both intermediates are emitted
  // as digits by the product before them: mode 3 writes the mode-1 digits
  // (slot A of the chain), mode 1 the mode-2 digits (slot B), and only the
  // inputs are sliced (into the slots after them), unless they come sliced
  if (prec == SETD_PREC_I8X4 && i8_order312(d, dims, nchains, i8bytes)) {
    char* base_ws = (char*)i8ws;
    auto slotA = [&](int c) { return (void*)(base_ws + (size_t)c * slot); };
    auto slotB = [&](int c) { return (void*)(base_ws + (size_t)(nchains + c) * slot); };
    LaunchKind k3{false, prec, DType::F64, base_ws + (size_t)2 * nchains * slot, i8bytes - (size_t)2 * nchains * slot};
    k3.fuse_next = emit ? dims[0] : 0;
    if (sliced_in) {
      for (int o = 0; o < nouts; ++o)
        if (!outs[o].x_sliced) {
          set_error("a Tucker group mixes sliced and FP64 inputs");
          return SETD_EINVAL;
        }
      k3.presliced = true;
    }
    LaunchKind k1{true, prec, DType::F64, i8ws, i8bytes};
    k1.presliced = emit;
    k1.fuse_next = emit ? dims[1] : 0;
    LaunchKind k2{false, prec, DType::F64, i8ws, i8bytes};
    k2.presliced = emit;
    ModeJobs J;
    J.njobs = 0;
    int c = 0;
    for (int o = 0; o < nouts; ++o)
      for (int t = 0; t < outs[o].nterms; ++t, ++c) {
        const TuckerTerm& tm = outs[o].term[t];
        SETD_TRY(push(J, mk_job(tm.X, tm.P[2], 1.0, emit ? slotA(c) : tm.Y1, nullptr, (int64_t)dims[0] * dims[1],
                                dims[2], 1), k3, s));
      }
    SETD_TRY(flush(J, k3, s));
    c = 0;
    for (int o = 0; o < nouts; ++o)
      for (int t = 0; t < outs[o].nterms; ++t, ++c) {
        const TuckerTerm& tm = outs[o].term[t];
        SETD_TRY(push(J, mk_job(emit ? slotA(c) : tm.Y1, tm.P[0], 1.0, emit ? slotB(c) : tm.Y2, nullptr, 1, dims[0],
                                (int64_t)dims[1] * dims[2]), k1, s));
      }
    SETD_TRY(flush(J, k1, s));
    c = 0;
    for (int o = 0; o < nouts; ++o) {
      ModeJob jb{};
      jb.nterms = outs[o].nterms;
      for (int t = 0; t < outs[o].nterms; ++t, ++c) {
        jb.X[t] = emit ? slotB(c) : outs[o].term[t].Y2;
        jb.P[t] = outs[o].term[t].P[1];
        jb.scale[t] = outs[o].term[t].scale;
      }
      jb.Y = outs[o].Y;
      jb.base = outs[o].base;
      jb.na = dims[0];
      jb.nb = dims[2];
      jb.n = dims[1];
      jb.ldp = packed_ld(dims[1]);
      SETD_TRY(push(J, jb, k2, s));
    }
    return flush(J, k2, s);
  }
  // I8X4 with n1 <= 256 and n2 in {128, 256}: the mode-1 products emit the
  // mode-2 digits straight into one buffer per chain (the first slots of the
  // workspace; the slicing passes get the rest), and mode 2 reads them
  if (sliced_in) {
    set_error("sliced Tucker inputs need the int8 form in the order 3, 1, 2");
    return SETD_EINVAL;
  }
  const bool fuse = emit && prec == SETD_PREC_I8X4 && d >= 2 && dims[0] <= 256 && (dims[1] == 128 || dims[1] == 256) &&
                    (size_t)(nchains + 1) * slot <= i8bytes;
  char* chain_digits = (char*)i8ws;
  auto chain_slot = [&](int chain) { return (void*)(chain_digits + (size_t)chain * slot); };
  LaunchKind k1{true, prec, mid, i8ws, i8bytes}, kb{false, prec, mid, i8ws, i8bytes},
      klast{false, prec, DType::F64, i8ws, i8bytes};
  if (fuse) {
    k1.i8ws = chain_digits + (size_t)nchains * slot;
    k1.i8bytes = i8bytes - (size_t)nchains * slot;
    k1.fuse_next = dims[1];
  }
  ModeJobs J;
  J.njobs = 0;
  // mode 1 -> Y1 (or the mode-2 digits)
  int chain = 0;
  for (int o = 0; o < nouts; ++o)
    for (int t = 0; t < outs[o].nterms; ++t, ++chain) {
      const TuckerTerm& tm = outs[o].term[t];
      void* y = fuse ? chain_slot(chain) : tm.Y1;
      SETD_TRY(push(J, mk_job(tm.X, tm.P[0], 1.0, y, nullptr, 1, dims[0], N / dims[0]), k1, s));
    }
  SETD_TRY(flush(J, k1, s));
  // inner modes, ping-pong Y1 <-> Y2
  int64_t na = dims[0];
  for (int mu = 1; mu < d - 1; ++mu) {
    const int64_t nb = N / (na * dims[mu]);
    LaunchKind k = kb;
    k.presliced = fuse && mu == 1;
    chain = 0;
    for (int o = 0; o < nouts; ++o)
      for (int t = 0; t < outs[o].nterms; ++t, ++chain) {
        const TuckerTerm& tm = outs[o].term[t];
        const void* src = k.presliced ? chain_slot(chain) : (mu % 2 == 1) ? tm.Y1 : tm.Y2;
        void* dst = (mu % 2 == 1) ? tm.Y2 : tm.Y1;
        SETD_TRY(push(J, mk_job(src, tm.P[mu], 1.0, dst, nullptr, na, dims[mu], nb), k, s));
      }
    SETD_TRY(flush(J, k, s));
    na *= dims[mu];
  }
  // last mode: terms summed along the contraction, base added
  const int mu = d - 1;
  klast.presliced = fuse && mu == 1;
  chain = 0;
  for (int o = 0; o < nouts; ++o) {
    ModeJob jb{};
    jb.nterms = outs[o].nterms;
    for (int t = 0; t < outs[o].nterms; ++t, ++chain) {
      const TuckerTerm& tm = outs[o].term[t];
      jb.X[t] = klast.presliced ? chain_slot(chain) : (mu % 2 == 1) ? tm.Y1 : tm.Y2;
      jb.P[t] = tm.P[mu];
      jb.scale[t] = tm.scale;
    }
    jb.Y = outs[o].Y;
    jb.base = outs[o].base;
    jb.na = na;
    jb.nb = 1;
    jb.n = dims[mu];
    jb.ldp = packed_ld(dims[mu]);
    SETD_TRY(push(J, jb, klast, s));
  }
  return flush(J, klast, s);
}

namespace {


int build_bank(setd_ctx* c, hipStream_t s) {
  const int d = c->d;
  // device copies of A (for phi and the dense K path)
  size_t abytes = 0;
  for (int cc = 0; cc < c->ncomp; ++cc)
    for (int mu = 0; mu < d; ++mu) abytes += (size_t)c->dims[mu] * c->dims[mu] * sizeof(double);
  if (c->A_mem.p == nullptr) {
    SETD_TRY(c->A_mem.alloc(abytes));
    char* q = (char*)c->A_mem.p;
    for (int cc = 0; cc < c->ncomp; ++cc)
      for (int mu = 0; mu < d; ++mu) {
        const size_t b = (size_t)c->dims[mu] * c->dims[mu] * sizeof(double);
        SETD_HIP(hipMemcpyAsync(q, c->Ah[cc][mu].data(), b, hipMemcpyHostToDevice, s));
        q += b;
      }
  }
  auto Adev = [&](int cc, int mu) {
    char* q = (char*)c->A_mem.p;
    for (int k = 0; k < cc * d + mu; ++k) {
      const int m = c->dims[k % d];
      q += (size_t)m * m * sizeof(double);
    }
    return (const double*)q;
  };

  // packed bank (in the context's arithmetic) + packed A (FP64, dense K path)
  size_t bbytes = 0;
  for (int cc = 0; cc < c->ncomp; ++cc)
    for (int mu = 0; mu < d; ++mu)
      bbytes += (5 * c->nterms + 2) * packed_bytes(c->dims[mu], c->prec) + packed_bytes(c->dims[mu], SETD_PREC_F64);
  SETD_TRY(c->bank_mem.alloc(bbytes));
  {
    char* q = (char*)c->bank_mem.p;
    for (int cc = 0; cc < c->ncomp; ++cc)
      for (int mu = 0; mu < d; ++mu) {
        const size_t pb = packed_bytes(c->dims[mu], c->prec);
        for (int e = 0; e < 5; ++e)
          for (int t = 0; t < c->nterms; ++t) {
            c->bank[cc][e][t][mu] = q;
            q += pb;
          }
        for (int l = 0; l < 2; ++l) {
          c->bank2[cc][l][mu] = q;
          q += pb;
        }
        c->Apk[cc][mu] = q;
        q += packed_bytes(c->dims[mu], SETD_PREC_F64);
      }
  }

  for (int cc = 0; cc < c->ncomp; ++cc) {
    // raw phi_0..phi_2 of each direction's scalars; a later direction with
    // the same matrix and the same scalars reuses an earlier one's
    DevBuf raw[3];
    std::vector<double> scal[3];
    std::vector<int> which[3];   // e * 3 + t
    int rep[3];
    for (int mu = 0; mu < d; ++mu) {
      for (int e = 0; e < 5; ++e) {
        const Splitting& S = c->sp[kBankEll[e]];
        for (int t = 0; t < S.nterms; ++t) {
          scal[mu].push_back(stage_scale(kBankStage[e]) * c->tau * S.alpha[t][mu]);
          which[mu].push_back(e * 3 + t);
        }
      }
      scal[mu].push_back(c->tau);   // phi_1, phi_2 (tau A_mu) of the second-order splitting
      which[mu].push_back(-1);
      rep[mu] = mu;
      for (int nu = 0; nu < mu; ++nu)
        if (rep[nu] == nu && c->dims[nu] == c->dims[mu] && c->Ah[cc][nu] == c->Ah[cc][mu] &&
            scal[nu] == scal[mu]) {
          rep[mu] = nu;
          break;
        }
      const int n = c->dims[mu];
      const int E = (int)scal[mu].size();
      const size_t nn = (size_t)n * n;
      if (rep[mu] == mu) {
        SETD_TRY(raw[mu].alloc((size_t)E * 3 * nn * sizeof(double)));
        std::vector<double*> outs(E * 3);
        for (int k = 0; k < E * 3; ++k) outs[k] = (double*)raw[mu].p + (size_t)k * nn;
        SETD_TRY(phi_batch(Adev(cc, mu), n, scal[mu].data(), E, 2, outs.data(), s));
      }
      const double* src = (const double*)raw[rep[mu]].p;
      for (int k = 0; k < E; ++k) {
        if (which[mu][k] < 0) {
          for (int l = 1; l <= 2; ++l)
            SETD_TRY(pack_for(c->prec, src + ((size_t)k * 3 + l) * nn, n, 1.0, mu, c->bank2[cc][l - 1][mu], s));
          continue;
        }
        const int e = which[mu][k] / 3, t = which[mu][k] % 3;
        const int li = c->sp[kBankEll[e]].ell_i[t];
        SETD_TRY(pack_for(c->prec, src + ((size_t)k * 3 + li) * nn, n, 1.0, mu, c->bank[cc][e][t][mu], s));
      }
      SETD_TRY(pack_matrix_f64(Adev(cc, mu), n, 1.0, mu == 0, (double*)c->Apk[cc][mu], s));
    }
    SETD_HIP(hipStreamSynchronize(s));   // raw buffers are released at scope exit
  }
  SETD_HIP(hipStreamSynchronize(s));
  return SETD_OK;
}



// Split phi action outputs for the F group: stage s, ell = 1.
// G = g(U) (FP64) and F = K U + G in the Tucker arithmetic's storage type.
}  // namespace

int setd::compute_gf(setd_ctx* c, double* u, const GParams& gp, hipStream_t s, double* G, void* F) {
  const int d = c->d, nc = c->ncomp;
  const int64_t N = c->N;
  const bool lp = fp32_storage(c->prec);
  const DType tdt = lp ? DType::F32 : DType::F64;
  const size_t es = lp ? 4 : 8;
  if (G == nullptr) G = c->G;
  if (F == nullptr) F = c->F;
  auto Fc_ = [&](int cc) { return (void*)((char*)F + cc * N * es); };
  if (c->tridiag) {
    SETD_TRY(launch_gf_stencil(u, nc, N, d, c->dims, c->st, gp, G, F, tdt, s));
  } else {
    SETD_TRY(launch_g(u, nc, N, gp, G, s));
    for (int cc = 0; cc < nc; ++cc) {
      // FP64 K action into F (or, reduced precision, into W then rounded)
      double* Fc = lp ? c->W + cc * N : (double*)F + cc * N;
      const double* uc = u + cc * N;
      ModeJobs J;
      J.njobs = 1;
      J.job[0] = mk_job(uc, c->Apk[cc][0], 1.0, Fc, G + cc * N, 1, c->dims[0], N / c->dims[0]);
      SETD_TRY(launch_mode1_f64(J, s));
      int64_t na = c->dims[0];
      for (int mu = 1; mu < d; ++mu) {
        J.njobs = 1;
        J.job[0] = mk_job(uc, c->Apk[cc][mu], 1.0, Fc, Fc, na, c->dims[mu], N / (na * c->dims[mu]));
        SETD_TRY(launch_modeB_f64(J, s));
        na *= c->dims[mu];
      }
      if (lp) SETD_TRY(launch_copy_convert(Fc, Fc_(cc), N, DType::F32, s));
    }
  }
  return SETD_OK;
}

namespace {

}  // namespace

// One exprk3ds_real step (the time loop of Algorithms 1 and 2), its stage
// quantities in b.
int setd::step_with(setd_ctx* c, double* u, const GParams& gp, hipStream_t s, const StageBufs& b) {
  const int d = c->d, nc = c->ncomp, T = c->nterms;
  const int64_t N = c->N;
  const double tau = c->tau;
  const int prec = c->prec;
  const bool lp = fp32_storage(prec);
  const DType tdt = lp ? DType::F32 : DType::F64;   // type of F, D and the intermediates
  const size_t es = lp ? 4 : 8;
  auto Fc_ = [&](int cc) { return (void*)((char*)b.F + cc * N * es); };
  auto D2c_ = [&](int cc) { return (void*)((char*)b.D2 + cc * N * es); };
  auto D3c_ = [&](int cc) { return (void*)((char*)b.D3 + cc * N * es); };
  // 1. G, F
  SETD_TRY(compute_gf(c, u, gp, s, b.G, b.F));
  const int e21 = bank_index(SETD_STAGE_2, 1), e31 = bank_index(SETD_STAGE_3, 1), e32 = bank_index(SETD_STAGE_3, 2),
            ef1 = bank_index(SETD_STAGE_F, 1), ef2 = bank_index(SETD_STAGE_F, 2);
  const Splitting& S1 = c->sp[1];
  const Splitting& S2 = c->sp[2];
  // 2. phi_1 actions on F for the three stages
  {
    TuckerOut outs[6];
    int no = 0;
    for (int cc = 0; cc < nc; ++cc) {
      const struct {
        int e;
        double mult;
        double* Y;
      } tg[3] = {{e21, tau / 3.0, b.U2 + cc * N}, {e31, 2.0 * tau / 3.0, b.U3 + cc * N}, {ef1, tau, c->W + cc * N}};
      for (int k = 0; k < 3; ++k) {
        TuckerOut& o = outs[no++];
        o.Y = tg[k].Y;
        o.base = u + cc * N;
        o.nterms = T;
        for (int t = 0; t < T; ++t)
          o.term[t] = {Fc_(cc), c->bank[cc][tg[k].e][t], tg[k].mult * S1.eta[t], c->Y1[cc][k * T + t],
                       c->Y2[cc][k * T + t]};
      }
    }
    SETD_TRY(run_tucker_group(d, c->dims, outs, no, prec, s, c->i8_mem.p, c->i8_mem.bytes));
  }
  // D = g(U_s) - G, the input of the next group.  The int8 form in the order
  // 3, 1, 2 writes only D's digits along mode 3 (the stage difference and
  // the slicing in one pass), unless the stage quantities are being recorded.
  auto stage_diff = [&](const double* Us, void* Dbuf, TuckerOut* outs) -> int {
    const bool own = b.D2 == (void*)c->D && b.D3 == (void*)c->D;
    if (prec == SETD_PREC_I8X4 && own && i8_emit() && i8_order312(d, c->dims, nc * T, c->i8_mem.bytes)) {
      const size_t slot = i8_slot_bytes(d, c->dims);
      void* dg[2];
      for (int cc = 0; cc < 2; ++cc) dg[cc] = (char*)c->i8_mem.p + (size_t)(2 * nc * T + cc) * slot;
      SETD_TRY(launch_stage_slice_i8(Us, b.G, nc, N, c->dims[2], gp, dg, s));
      for (int cc = 0; cc < nc; ++cc) {
        outs[cc].x_sliced = true;
        for (int t = 0; t < T; ++t) outs[cc].term[t].X = dg[cc];
      }
      return SETD_OK;
    }
    return launch_stage_d(Us, b.G, nc, N, gp, Dbuf, tdt, s);
  };
  // 3., 4. D2 = g(U2) - G; U3 += 4tau/3 S_2(2tau/3) D2
  {
    TuckerOut outs[2];
    for (int cc = 0; cc < nc; ++cc) {
      TuckerOut& o = outs[cc];
      o.Y = b.U3 + cc * N;
      o.base = b.U3 + cc * N;
      o.nterms = T;
      for (int t = 0; t < T; ++t)
        o.term[t] = {D2c_(cc), c->bank[cc][e32][t], 4.0 * tau / 3.0 * S2.eta[t], c->Y1[cc][t], c->Y2[cc][t]};
    }
    SETD_TRY(stage_diff(b.U2, b.D2, outs));
    SETD_TRY(run_tucker_group(d, c->dims, outs, nc, prec, s, c->i8_mem.p, c->i8_mem.bytes));
  }
  // 5., 6. D3 = g(U3) - G; U = W + 3tau/2 S_2(tau) D3
  {
    TuckerOut outs[2];
    for (int cc = 0; cc < nc; ++cc) {
      TuckerOut& o = outs[cc];
      o.Y = u + cc * N;
      o.base = c->W + cc * N;
      o.nterms = T;
      for (int t = 0; t < T; ++t)
        o.term[t] = {D3c_(cc), c->bank[cc][ef2][t], 1.5 * tau * S2.eta[t], c->Y1[cc][t], c->Y2[cc][t]};
    }
    SETD_TRY(stage_diff(b.U3, b.D3, outs));
    SETD_TRY(run_tucker_group(d, c->dims, outs, nc, prec, s, c->i8_mem.p, c->i8_mem.bytes));
  }
  return SETD_OK;
}

namespace {

// The step of setd_etd_step: stage quantities in the context's buffers (D2
// and D3 share one).
int step_once(setd_ctx* c, double* u, const GParams& gp, hipStream_t s) {
  return step_with(c, u, gp, s, StageBufs{c->G, c->F, c->U2, c->D, c->U3, c->D});
}

// One etd2rkds step: U2 = U + tau T(F, {phi_1}), D = g(U2) - G,
// U = U2 + tau 2^{d-1} T(D, {phi_2})  (eq. ETD2RK with eq. secondord).
int step2_once(setd_ctx* c, double* u, const GParams& gp, hipStream_t s) {
  const int d = c->d, nc = c->ncomp;
  const int64_t N = c->N;
  const bool lp = fp32_storage(c->prec);
  const DType tdt = lp ? DType::F32 : DType::F64;
  const size_t es = lp ? 4 : 8;
  SETD_TRY(compute_gf(c, u, gp, s));
  TuckerOut outs[2];
  for (int cc = 0; cc < nc; ++cc) {
    TuckerOut& o = outs[cc];
    o.Y = c->U2 + cc * N;
    o.base = u + cc * N;
    o.nterms = 1;
    o.term[0] = {(char*)c->F + cc * N * es, c->bank2[cc][0], c->tau, c->Y1[cc][0], c->Y2[cc][0]};
  }
  SETD_TRY(run_tucker_group(d, c->dims, outs, nc, c->prec, s, c->i8_mem.p, c->i8_mem.bytes));
  SETD_TRY(launch_stage_d(c->U2, c->G, nc, N, gp, c->D, tdt, s));
  const double fact = std::ldexp(1.0, d - 1);   // 2!^{d-1}
  for (int cc = 0; cc < nc; ++cc) {
    TuckerOut& o = outs[cc];
    o.Y = u + cc * N;
    o.base = c->U2 + cc * N;
    o.nterms = 1;
    o.term[0] = {(char*)c->D + cc * N * es, c->bank2[cc][1], c->tau * fact, c->Y1[cc][0], c->Y2[cc][0]};
  }
  return run_tucker_group(d, c->dims, outs, nc, c->prec, s, c->i8_mem.p, c->i8_mem.bytes);
}

typedef int (*StepFn)(setd_ctx*, double*, const GParams&, hipStream_t);

// Graph replay of one step: used unless SETD_GRAPH=0 or the kernel timing is
// on (its event records would be frozen into the graph).
bool use_graph(const setd_ctx* c) {
  (void)c;
  const char* e = std::getenv("SETD_GRAPH");
  if (e && e[0] == '0') return false;
  return !prof_on();
}

void drop_graph(setd_ctx* c) {
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  c->gexec = nullptr;
  c->g_u = nullptr;
}

// Captures one step (kernels only; no memset or memcpy nodes) on the
// context's own stream.
int capture_step(setd_ctx* c, double* u, const GParams& gp, StepFn fn) {
  drop_graph(c);
  if (!c->gstream) SETD_HIP(hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking));
  if (!c->ev_in) SETD_HIP(hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming));
  if (!c->ev_out) SETD_HIP(hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming));
  SETD_HIP(hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal));
  const int rc = fn(c, u, gp, c->gstream);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(c->gstream, &graph);
  if (rc != SETD_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess || !graph) {
    set_error("step capture failed: %s", hipGetErrorString(e));
    return SETD_EHIP;
  }
  const hipError_t ei = hipGraphInstantiate(&c->gexec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) {
    c->gexec = nullptr;
    set_error("graph instantiation failed: %s", hipGetErrorString(ei));
    return SETD_EHIP;
  }
  c->g_u = u;
  c->g_gp = gp;
  c->g_fn = (const void*)fn;
  return SETD_OK;
}

// nsteps applications of `fn` to u (graph replay when possible).
int run_steps(setd_ctx* c, double* u, int nsteps, double tau, int g_kind, const double* params, int nparams,
              hipStream_t s, StepFn fn) {
  SETD_CHECK_ARG(c != nullptr, "ctx is NULL");
  SETD_CHECK_ARG(u != nullptr, "u is NULL");
  SETD_CHECK_ARG(nsteps >= 0, "nsteps < 0");
  SETD_CHECK_ARG(tau > 0.0, "tau must be positive");
  if (!std::isfinite(tau)) {
    set_error("tau is not finite");
    return SETD_ENONFINITE;
  }
  GParams gp;
  SETD_TRY(make_gparams(g_kind, params, nparams, c->ncomp, gp));
  if (tau != c->tau) {
    c->tau = tau;
    SETD_TRY(build_bank(c, s));
    drop_graph(c);
  }
  if (nsteps == 0) return SETD_OK;
  if (use_graph(c)) {
    bool same = c->gexec && c->g_u == u && c->g_fn == (const void*)fn && c->g_gp.kind == gp.kind;
    for (int k = 0; k < 4; ++k) same = same && c->g_gp.p[k] == gp.p[k];
    const int rc = same ? SETD_OK : capture_step(c, u, gp, fn);
    if (rc == SETD_OK) {
      SETD_HIP(hipEventRecord(c->ev_in, s));
      SETD_HIP(hipStreamWaitEvent(c->gstream, c->ev_in, 0));
      for (int k = 0; k < nsteps; ++k) SETD_HIP(hipGraphLaunch(c->gexec, c->gstream));
      SETD_HIP(hipEventRecord(c->ev_out, c->gstream));
      SETD_HIP(hipStreamWaitEvent(s, c->ev_out, 0));
      return SETD_OK;
    }
    drop_graph(c);   // capture failed: fall back to direct launches
    clear_error();
  }
  for (int k = 0; k < nsteps; ++k) SETD_TRY(fn(c, u, gp, s));
  return SETD_OK;
}

}  // namespace

// Scratch memory of setd_tucker_apply_noalloc: the Tucker intermediates and
// packed matrices of one call.  Each GPU the library runs on holds its own
// copy until the process ends.  In host code this name is only a stand-in
// for the device array: kernels and copies get the address that
// hipGetSymbolAddress returns for the current device (noalloc_scratch).
static __device__ __align__(256) unsigned char scratch[SETD_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
int noalloc_scratch(void** out) {
  int dev = 0;
  SETD_HIP(hipGetDevice(&dev));
  SETD_CHECK_ARG(dev >= 0 && dev < kMaxScratchDevices, "device %d outside 0..%d", dev, kMaxScratchDevices - 1);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    SETD_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    SETD_CHECK_ARG(p != nullptr, "no device address for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SETD_OK;
}
}  // namespace

extern "C" {

const char* setd_last_error(void) { return g_err; }

const char* setd_version(void) { return "setd 0.1 (gfx950, FP64 MFMA mode products)"; }

int setd_profile_enable(int on) {
  clear_error();
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof = on != 0;
  return SETD_OK;
}

int setd_profile_read(double* out, int reset) {
  clear_error();
  SETD_CHECK_ARG(out != nullptr, "out is NULL");
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (int k = 0; k < 4 * SETD_PROF_CLASSES; ++k) out[k] = 0.0;
  for (const ProfRec& r : g_recs) {
    SETD_HIP(hipEventSynchronize(r.e));
    float ms = 0.0f;
    SETD_HIP(hipEventElapsedTime(&ms, r.b, r.e));
    double* o = out + 4 * r.cls;
    o[0] += 1.0;
    o[1] += ms;
    o[2] += r.flops;
    o[3] += r.bytes;
  }
  if (reset) {
    for (const ProfRec& r : g_recs) {
      g_free_events.push_back(r.b);
      g_free_events.push_back(r.e);
    }
    g_recs.clear();
  }
  return SETD_OK;
}

int setd_sync(void* stream) {
  clear_error();
  SETD_HIP(hipStreamSynchronize((hipStream_t)stream));
  SETD_HIP(hipGetLastError());
  return SETD_OK;
}

int setd_release_workspace(void) {
  clear_error();
  int dev = 0;
  SETD_HIP(hipGetDevice(&dev));
  hipMemPool_t pool;
  SETD_HIP(hipDeviceGetDefaultMemPool(&pool, dev));
  SETD_HIP(hipMemPoolTrimTo(pool, 0));
  return SETD_OK;
}

int setd_phi_matrices(const double* A, int64_t n, double tau, int ell, double* out, void* stream) {
  clear_error();
  SETD_CHECK_ARG(A != nullptr && out != nullptr, "A and out must be non-NULL");
  SETD_CHECK_ARG(n >= 1 && n <= 4096, "n = %lld outside 1..4096", (long long)n);
  SETD_CHECK_ARG(ell >= 0 && ell <= 4, "ell = %d outside 0..4", ell);
  SETD_CHECK_ARG(!overlap(A, (size_t)n * n * 8, out, (size_t)(ell + 1) * n * n * 8), "out overlaps A");
  if (!std::isfinite(tau)) {
    set_error("tau is not finite");
    return SETD_ENONFINITE;
  }
  hipStream_t s = (hipStream_t)stream;
  std::vector<double*> outs(ell + 1);
  for (int k = 0; k <= ell; ++k) outs[k] = out + (size_t)k * n * n;
  return phi_batch(A, (int)n, &tau, 1, ell, outs.data(), s);
}

int setd_tucker_apply_noalloc(const double* V, double* W, int d, const int64_t* dims, const double* const* M,
                              double alpha, double beta, int prec, void* stream) {
  clear_error();
  // need is 0 for arguments setd_tucker_apply rejects; it reports them below
  // (with a workspace given it never allocates)
  const size_t need = setd_tucker_workspace_bytes(d, dims, prec);
  SETD_CHECK_ARG(need <= (size_t)SETD_NOALLOC_SCRATCH_BYTES,
                 "tensor needs %zu bytes of scratch, more than the %zu bytes setd_tucker_apply_noalloc holds", need,
                 (size_t)SETD_NOALLOC_SCRATCH_BYTES);
  void* ws = nullptr;
  SETD_TRY(noalloc_scratch(&ws));
  return setd_tucker_apply(V, W, d, dims, M, alpha, beta, prec, ws, (size_t)SETD_NOALLOC_SCRATCH_BYTES, stream);
}

size_t setd_tucker_workspace_bytes(int d, const int64_t* dims, int prec) {
  if (d < 1 || d > 8 || dims == nullptr) return 0;
  int64_t N = 1;
  size_t pk = 0;
  for (int mu = 0; mu < d; ++mu) {
    if (dims[mu] < 1 || dims[mu] > 4096 || N > kMaxTuckerElems / dims[mu]) return 0;
    N *= dims[mu];
    pk += round_up(packed_bytes((int)dims[mu], prec), 256);
  }
  if (!is_prec(prec)) return 0;
  // two ping-pong intermediates, plus the FP32 copy of V for reduced precision
  // or one int8 digit buffer for the error-free slicing form
  const int nbuf = fp32_storage(prec) ? 3 : 2;
  size_t dig = 0;
  if (prec == SETD_PREC_I8X4)
    for (int mu = 0; mu < d; ++mu) dig = std::max(dig, i8_digit_bytes(N, (int)dims[mu]));
  return pk + nbuf * round_up(N * (int64_t)sizeof(double), 256) + dig + 256;
}

int setd_tucker_apply(const double* V, double* W, int d, const int64_t* dims, const double* const* M, double alpha,
                      double beta, int prec, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  SETD_CHECK_ARG(d >= 1 && d <= 8, "d = %d outside 1..8", d);
  SETD_CHECK_ARG(dims != nullptr && M != nullptr, "dims and M must be non-NULL");
  SETD_CHECK_ARG(V != nullptr && W != nullptr, "V and W must be non-NULL");
  int64_t N = 1;
  for (int mu = 0; mu < d; ++mu) {
    SETD_CHECK_ARG(dims[mu] >= 1 && dims[mu] <= 4096, "dims[%d] = %lld outside 1..4096", mu, (long long)dims[mu]);
    SETD_CHECK_ARG(N <= kMaxTuckerElems / dims[mu], "the tensor has more than %lld elements",
                   (long long)kMaxTuckerElems);
    N *= dims[mu];
  }
  SETD_CHECK_ARG(!overlap(V, N * 8, W, N * 8), "V and W overlap");
  SETD_CHECK_ARG(is_prec(prec), "bad prec %d", prec);
  if (!std::isfinite(alpha) || !std::isfinite(beta)) {
    set_error("alpha/beta not finite");
    return SETD_ENONFINITE;
  }
  hipStream_t s = (hipStream_t)stream;
  const size_t need = setd_tucker_workspace_bytes(d, dims, prec);
  SETD_CHECK_ARG(ws == nullptr || ws_bytes >= need, "workspace too small: %zu < %zu", ws_bytes, need);

  int modes[8], nm = 0;
  for (int mu = 0; mu < d; ++mu)
    if (M[mu] != nullptr) modes[nm++] = mu;
  // the workspace first, so that a failed allocation leaves W untouched
  void* wsp = ws;
  bool own = false;
  if (nm > 0 && wsp == nullptr) {
    SETD_HIP(hipMallocAsync(&wsp, need, s));
    own = true;
  }
  // beta handling: base = W when beta == 1, none when beta == 0, else scale W first
  const double* base = nullptr;
  if (beta != 0.0) {
    if (beta != 1.0) {
      const int r = launch_scale(W, N, beta, s);
      if (r != SETD_OK) {
        if (own) (void)hipFreeAsync(wsp, s);
        return r;
      }
    }
    base = W;
  }
  if (nm == 0) {
    return launch_axpby(V, W, N, alpha, beta == 0.0 ? 0.0 : 1.0, s);
  }
  const bool lp = fp32_storage(prec);
  const int64_t fb = round_up(N * 8, 256);
  char* q = (char*)round_up((int64_t)(uintptr_t)wsp, 256);
  void* buf[3] = {q, q + fb, q + 2 * fb};
  q += (lp ? 3 : 2) * fb;
  void* P[8] = {};
  int rc = SETD_OK;
  for (int k = 0; k < nm; ++k) q += round_up(packed_bytes((int)dims[modes[k]], prec), 256);
  // the int8 digit buffer (SETD_PREC_I8X4) follows the packed matrices
  void* dig = q;
  size_t dig_bytes = 0;
  if (prec == SETD_PREC_I8X4)
    for (int mu = 0; mu < d; ++mu) dig_bytes = std::max(dig_bytes, i8_digit_bytes(N, (int)dims[mu]));
  q = (char*)round_up((int64_t)(uintptr_t)wsp, 256) + (lp ? 3 : 2) * fb;
  for (int k = 0; k < nm && rc == SETD_OK; ++k) {
    const int mu = modes[k];
    P[mu] = q;
    q += round_up(packed_bytes((int)dims[mu], prec), 256);
    const bool last = (k == nm - 1);
    rc = pack_for(prec, M[mu], (int)dims[mu], last ? alpha : 1.0, mu, P[mu], s);
  }
  // reduced precision: the FP64 input is rounded to FP32 once
  const void* src = V;
  if (lp && rc == SETD_OK) {
    rc = launch_copy_convert(V, buf[2], N, DType::F32, s);
    src = buf[2];
  }
  for (int k = 0; k < nm && rc == SETD_OK; ++k) {
    const int mu = modes[k];
    const bool last = (k == nm - 1);
    void* dst = last ? (void*)W : buf[k & 1];
    int64_t na = 1, nb = 1;
    for (int nu = 0; nu < mu; ++nu) na *= dims[nu];
    for (int nu = mu + 1; nu < d; ++nu) nb *= dims[nu];
    ModeJobs J;
    J.njobs = 1;
    J.job[0] = mk_job(src, P[mu], 1.0, dst, last ? base : nullptr, na, (int)dims[mu], nb);
    const LaunchKind kind{mu == 0, prec, (last || !lp) ? DType::F64 : DType::F32, dig, dig_bytes};
    rc = launch_jobs(J, kind, s);
    src = dst;
  }
  if (own) {
    hipError_t e = hipFreeAsync(wsp, s);
    if (rc == SETD_OK && e != hipSuccess) {
      set_error("hipFreeAsync failed: %s", hipGetErrorString(e));
      rc = SETD_EHIP;
    }
  }
  return rc;
}

int setd_ctx_create(setd_ctx** out, int d, const int64_t* dims, int ncomp, const double* const* A, double tau,
                    int prec, void* stream) {
  clear_error();
  SETD_CHECK_ARG(out != nullptr, "ctx out-pointer is NULL");
  *out = nullptr;
  SETD_CHECK_ARG(d == 2 || d == 3, "d = %d: the split integrator supports d = 2 and d = 3", d);
  SETD_CHECK_ARG(dims != nullptr && A != nullptr, "dims and A must be non-NULL");
  SETD_CHECK_ARG(ncomp == 1 || ncomp == 2, "ncomp = %d outside 1..2", ncomp);
  SETD_CHECK_ARG(tau > 0.0, "tau must be positive");
  if (!std::isfinite(tau)) {
    set_error("tau is not finite");
    return SETD_ENONFINITE;
  }
  SETD_CHECK_ARG(is_prec(prec), "bad prec %d", prec);
  for (int mu = 0; mu < d; ++mu)
    SETD_CHECK_ARG(dims[mu] >= 2 && dims[mu] <= 1024, "dims[%d] = %lld outside 2..1024", mu, (long long)dims[mu]);
  for (int k = 0; k < ncomp * d; ++k) SETD_CHECK_ARG(A[k] != nullptr, "A[%d] is NULL", k);
  hipStream_t s = (hipStream_t)stream;

  setd_ctx* c = new (std::nothrow) setd_ctx();
  if (!c) {
    set_error("out of host memory");
    return SETD_ENOMEM;
  }
  c->d = d;
  c->ncomp = ncomp;
  c->prec = prec;
  c->tau = tau;
  c->N = 1;
  for (int mu = 0; mu < d; ++mu) {
    c->dims[mu] = (int)dims[mu];
    c->N *= dims[mu];
  }
  c->sp[1] = splitting(1, d);
  c->sp[2] = splitting(2, d);
  c->nterms = c->sp[1].nterms;

  int rc = SETD_OK;
  auto fail = [&](int code) {
    delete c;
    return code;
  };
  // host copies of A; tridiagonal check; finiteness
  c->tridiag = true;
  for (int cc = 0; cc < ncomp; ++cc)
    for (int mu = 0; mu < d; ++mu) {
      const int n = c->dims[mu];
      c->Ah[cc][mu].resize((size_t)n * n);
      hipError_t e = hipMemcpy(c->Ah[cc][mu].data(), A[cc * d + mu], (size_t)n * n * 8, hipMemcpyDeviceToHost);
      if (e != hipSuccess) {
        set_error("copying A[%d] failed: %s", cc * d + mu, hipGetErrorString(e));
        return fail(SETD_EHIP);
      }
      for (double v : c->Ah[cc][mu])
        if (!std::isfinite(v)) {
          set_error("A[%d] has non-finite entries", cc * d + mu);
          return fail(SETD_ENONFINITE);
        }
      c->tridiag = c->tridiag && is_tridiagonal(c->Ah[cc][mu], n);
    }
  // stencil coefficients
  if (c->tridiag) {
    size_t tot = 0;
    for (int cc = 0; cc < ncomp; ++cc)
      for (int mu = 0; mu < d; ++mu) tot += 3 * (size_t)c->dims[mu];
    std::vector<double> h(tot);
    size_t o = 0;
    std::vector<size_t> offs;
    for (int cc = 0; cc < ncomp; ++cc)
      for (int mu = 0; mu < d; ++mu) {
        const int n = c->dims[mu];
        const std::vector<double>& M = c->Ah[cc][mu];
        offs.push_back(o);
        for (int i = 0; i < n; ++i) {
          h[o + i] = i > 0 ? M[i + (size_t)n * (i - 1)] : 0.0;
          h[o + n + i] = M[i + (size_t)n * i];
          h[o + 2 * n + i] = i + 1 < n ? M[i + (size_t)n * (i + 1)] : 0.0;
        }
        o += 3 * n;
      }
    if ((rc = c->stencil_mem.alloc(tot * 8)) != SETD_OK) return fail(rc);
    hipError_t e = hipMemcpy(c->stencil_mem.p, h.data(), tot * 8, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      set_error("stencil upload failed: %s", hipGetErrorString(e));
      return fail(SETD_EHIP);
    }
    int k = 0;
    for (int cc = 0; cc < ncomp; ++cc)
      for (int mu = 0; mu < d; ++mu, ++k) {
        const double* base = (const double*)c->stencil_mem.p + offs[k];
        const int n = c->dims[mu];
        c->st.lo[cc * 3 + mu] = base;
        c->st.di[cc * 3 + mu] = base + n;
        c->st.up[cc * 3 + mu] = base + 2 * n;
      }
  }
  // work buffers: G F U2 U3 W D (ncomp*N each) + Y1/Y2 (3*nterms per component)
  {
    const int T = c->nterms;
    const int ny = 3 * T;
    const int64_t fields = 6 * (int64_t)ncomp + (int64_t)ncomp * ny * (d == 3 ? 2 : 1) + 1;
    const size_t fb = round_up(c->N * 8, 256);
    if ((rc = c->work_mem.alloc(fields * fb + 256)) != SETD_OK) return fail(rc);
    char* q = (char*)c->work_mem.p;
    auto take = [&](int64_t nf) {
      double* p = (double*)q;
      q += nf * fb;
      return p;
    };
    c->G = take(ncomp);
    c->F = take(ncomp);
    c->U2 = take(ncomp);
    c->U3 = take(ncomp);
    c->W = take(ncomp);
    c->D = take(ncomp);
    // within G..D, component cc sits at +cc*N; fb-rounding applies per pair
    for (int cc = 0; cc < ncomp; ++cc)
      for (int k = 0; k < ny; ++k) {
        c->Y1[cc][k] = take(1);
        if (d == 3) c->Y2[cc][k] = take(1);
        else c->Y2[cc][k] = nullptr;
      }
    c->aux = take(1);
  }
  // int8 digit buffers: two per chain of the largest group (the phi_1 group:
  // 3 stages x nterms x ncomp) for the fused intermediates' digits, and
  // ncomp + 1 for the inputs of the slicing passes
  if (c->prec == SETD_PREC_I8X4) {
    const size_t slot = i8_slot_bytes(d, c->dims);
    if ((rc = c->i8_mem.alloc((size_t)(6 * c->nterms * ncomp + ncomp + 1) * slot)) != SETD_OK) return fail(rc);
  }
  if ((rc = build_bank(c, s)) != SETD_OK) return fail(rc);
  *out = c;
  return SETD_OK;
}

int setd_ctx_destroy(setd_ctx* ctx) {
  clear_error();
  if (!ctx) return SETD_OK;
  (void)hipDeviceSynchronize();
  delete ctx;
  return SETD_OK;
}

int setd_split_phi_apply(setd_ctx* c, int comp, int ell, int stage, const double* V, double* W, double scale,
                         double beta, void* stream) {
  clear_error();
  SETD_CHECK_ARG(c != nullptr, "ctx is NULL");
  SETD_CHECK_ARG(comp >= 0 && comp < c->ncomp, "comp %d outside 0..%d", comp, c->ncomp - 1);
  SETD_CHECK_ARG(ell == 1 || ell == 2, "ell must be 1 or 2");
  SETD_CHECK_ARG(stage == SETD_STAGE_2 || stage == SETD_STAGE_3 || stage == SETD_STAGE_F, "bad stage %d", stage);
  const int e = bank_index(stage, ell);
  SETD_CHECK_ARG(e >= 0, "stage 2 uses phi_1 only");
  SETD_CHECK_ARG(V != nullptr && W != nullptr, "V and W must be non-NULL");
  SETD_CHECK_ARG(!overlap(V, c->N * 8, W, c->N * 8), "V and W overlap");
  if (!std::isfinite(scale) || !std::isfinite(beta)) {
    set_error("scale/beta not finite");
    return SETD_ENONFINITE;
  }
  hipStream_t s = (hipStream_t)stream;
  const double* base = nullptr;
  if (beta != 0.0) {
    if (beta != 1.0) SETD_TRY(launch_scale(W, c->N, beta, s));
    base = W;
  }
  const Splitting& S = c->sp[ell];
  const void* src = V;
  if (fp32_storage(c->prec)) {   // FP32 forms: round the input to FP32 once
    SETD_TRY(launch_copy_convert(V, c->aux, c->N, DType::F32, s));
    src = c->aux;
  }
  TuckerOut o;
  o.Y = W;
  o.base = base;
  o.nterms = S.nterms;
  for (int t = 0; t < S.nterms; ++t)
    o.term[t] = {src, c->bank[comp][e][t], scale * S.eta[t], c->Y1[0][t], c->Y2[0][t]};
  return run_tucker_group(c->d, c->dims, &o, 1, c->prec, s, c->i8_mem.p, c->i8_mem.bytes);
}

int setd_etd_step(setd_ctx* c, double* u, int nsteps, double tau, int g_kind, const double* params, int nparams,
                  void* stream) {
  clear_error();
  return run_steps(c, u, nsteps, tau, g_kind, params, nparams, (hipStream_t)stream, step_once);
}

int setd_etd_step_record(setd_ctx* c, double* u, double tau, int g_kind, const double* params, int nparams,
                         double* rec, void* stream) {
  clear_error();
  SETD_CHECK_ARG(c != nullptr, "ctx is NULL");
  SETD_CHECK_ARG(u != nullptr && rec != nullptr, "u and rec must be non-NULL");
  const int64_t NC = c->ncomp * c->N;
  SETD_CHECK_ARG(!overlap(u, NC * 8, rec, 6 * NC * 8), "u and rec overlap");
  SETD_CHECK_ARG(tau > 0.0, "tau must be positive");
  if (!std::isfinite(tau)) {
    set_error("tau is not finite");
    return SETD_ENONFINITE;
  }
  if (c->prec != SETD_PREC_F64) {
    set_error("the recorded step runs in FP64 only");
    return SETD_EUNSUPPORTED;
  }
  GParams gp;
  SETD_TRY(make_gparams(g_kind, params, nparams, c->ncomp, gp));
  hipStream_t s = (hipStream_t)stream;
  if (tau != c->tau) {
    c->tau = tau;
    SETD_TRY(build_bank(c, s));
    drop_graph(c);
  }
  const StageBufs b{rec, rec + NC, rec + 2 * NC, rec + 3 * NC, rec + 4 * NC, rec + 5 * NC};
  return step_with(c, u, gp, s, b);
}

int setd_etd2_step(setd_ctx* c, double* u, int nsteps, double tau, int g_kind, const double* params, int nparams,
                   void* stream) {
  clear_error();
  return run_steps(c, u, nsteps, tau, g_kind, params, nparams, (hipStream_t)stream, step2_once);
}

int setd_etd_cplx_step(setd_ctx* c, double* u, int nsteps, double tau, int g_kind, const double* params,
                       int nparams, void* stream) {
  clear_error();
  SETD_CHECK_ARG(c != nullptr, "ctx is NULL");
  SETD_CHECK_ARG(tau > 0.0 && std::isfinite(tau), "tau must be positive and finite");
  if (c->prec != SETD_PREC_F64) {
    set_error("exprk3ds_cplx runs in FP64 only");
    return SETD_EUNSUPPORTED;
  }
  if (nsteps > 0) SETD_TRY(prepare_cplx(c, tau, (hipStream_t)stream));
  return run_steps(c, u, nsteps, tau, g_kind, params, nparams, (hipStream_t)stream, step_cplx_once);
}

int setd_field_norms(const double* x, const double* y, int64_t n, double* out, void* stream) {
  clear_error();
  SETD_CHECK_ARG(x != nullptr && out != nullptr, "x and out must be non-NULL");
  SETD_CHECK_ARG(n >= 0, "n < 0");
  if (n == 0) {
    out[0] = out[1] = out[2] = out[3] = 0.0;
    return SETD_OK;
  }
  hipStream_t s = (hipStream_t)stream;
  void* ws = nullptr;
  SETD_HIP(hipMallocAsync(&ws, norm_workspace_bytes(), s));
  int rc = launch_norms(x, y, n, (double*)ws, s);
  double h[4] = {0, 0, 0, 0};
  if (rc == SETD_OK) {
    hipError_t e = hipMemcpyAsync(h, (double*)ws + norm_workspace_bytes() / 8 - 4, 4 * sizeof(double),
                                  hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) {
      set_error("norm copy failed: %s", hipGetErrorString(e));
      rc = SETD_EHIP;
    }
  }
  (void)hipFreeAsync(ws, s);
  if (rc == SETD_OK) {
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      set_error("sync failed: %s", hipGetErrorString(e));
      rc = SETD_EHIP;
    }
  }
  for (int k = 0; k < 4; ++k) out[k] = y || k < 2 ? h[k] : 0.0;
  return rc;
}

}  // extern "C"
