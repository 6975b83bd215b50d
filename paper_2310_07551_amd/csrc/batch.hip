// Batched split-ETD3: many independent instances of one kind of problem (same
// d, components and tau; each with its own grid, matrices and reaction
// parameters) advanced together.
//
// Small grids cannot fill 256 compute units on their own: a 64 x 64 mu-mode
// product is a few dozen wave tiles.  So every stage of the step (eq. exprk3
// with the split phi actions, the time loop of Algorithms 1 and 2) is one
// launch over the concatenated work of all instances:
//   * the mu-mode products of a Tucker group run from a work list of
//     (instance, output, tile) in device memory, walked by a persistent grid
//     (mode 1, each inner mode, the last mode with its terms summed);
//   * the pointwise kernels (G/F, stage differences) run over the points of
//     all instances, each block inside one instance.
// The work lists are built once for a given state buffer and tile shape, the
// step is captured in a hipGraph and replayed, and the tile shapes are chosen
// by timing candidate shapes on the batch's own work lists.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <unordered_map>
#include <vector>

#include "api_util.hpp"
#include "coeffs.hpp"
#include "common.hpp"
#include "pointwise.hpp"

using namespace setd;

namespace {

constexpr int kNoPacked = -1;

struct Inst {
  int dims[3] = {1, 1, 1};
  int64_t N = 0, cs = 0;    // points; component stride (N rounded up to 8)
  int64_t off = 0;          // component 0 in u and every u-shaped buffer
  int64_t yoff = 0;         // first intermediate field in Y1 / Y2
  int bank[2][3] = {};      // [comp][mu] -> packed phi set (5 x nterms matrices)
  int apk[2][3] = {};       // [comp][mu] -> packed A (dense K path), or kNoPacked
};

// A set of packed matrices shared by every (instance, component, direction)
// with the same matrix A, the same phi scalars and the same packing.
struct PackedSet {
  int n = 0;
  bool rowmajor = false;
  std::vector<double> key;   // A (n*n) followed by the scalars
  uint64_t hash = 0;
  size_t offset = 0;         // bytes into bank_mem
  int count = 0;             // matrices in the set
  const double* A_dev = nullptr;
};

struct Op {
  bool list;                 // mode-product list or pointwise
  ModeList L;
  int pk;
  const double* x;
  double* G;
  double* out;
};

uint64_t fnv(const double* p, size_t n, uint64_t h) {
  const unsigned char* b = (const unsigned char*)p;
  for (size_t k = 0; k < n * sizeof(double); ++k) {
    h ^= b[k];
    h *= 1099511628211ull;
  }
  return h;
}

}  // namespace

struct setd_batch {
  int nb = 0, d = 0, ncomp = 0, nterms = 0;
  double tau = 0.0;
  Splitting sp[3];
  std::vector<Inst> inst;
  std::vector<PackedSet> sets;
  int64_t total = 0;         // elements of u
  int64_t points = 0;        // grid points of all instances
  int64_t ytotal = 0;        // elements of Y1 (and of Y2 when d = 3)
  bool tridiag = true;
  DevBuf bank_mem, stencil_mem, work_mem, inst_mem, list_mem, tune_mem;
  double *G = nullptr, *F = nullptr, *U2 = nullptr, *U3 = nullptr, *W = nullptr, *D = nullptr;
  double *Y1 = nullptr, *Y2 = nullptr;
  std::vector<BatchInstDev> inst_host;
  std::vector<int64_t> blk_host;
  BatchInstDev* inst_dev = nullptr;
  int64_t* blk_dev = nullptr;
  int64_t nblocks = 0;
  // reaction parameters: inst_host holds the latest, inst_dev gets them
  // before the next launch
  bool params_dirty = true;
  // tile choice: {tm, tn, grid cap} for mode 1 and for modes >= 2
  int cfg1[3] = {4, 4, 0}, cfgB[3] = {4, 2, 0};
  bool tuned = false;
  // plan of one step for state buffer plan_u
  std::vector<Op> plan;
  double* plan_u = nullptr;
  // captured step
  hipStream_t gstream = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  ~setd_batch() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (gstream) (void)hipStreamDestroy(gstream);
  }
};

namespace {

double* y1(setd_batch* B, int b, int c, int k) {
  const Inst& I = B->inst[b];
  return B->Y1 + I.yoff + (int64_t)(c * 3 * B->nterms + k) * I.cs;
}
double* y2(setd_batch* B, int b, int c, int k) {
  if (!B->Y2) return nullptr;
  const Inst& I = B->inst[b];
  return B->Y2 + I.yoff + (int64_t)(c * 3 * B->nterms + k) * I.cs;
}
const void* packed(const setd_batch* B, int set, int k) {
  const PackedSet& S = B->sets[set];
  return (const char*)B->bank_mem.p + S.offset + (size_t)k * packed_bytes(S.n, SETD_PREC_F64);
}

// Finds or adds the packed set for (n, A, scalars, layout).
int find_set(setd_batch* B, int n, bool rowmajor, const std::vector<double>& Ah, const std::vector<double>& scal,
             int count, const double* A_dev) {
  std::vector<double> key(Ah);
  key.insert(key.end(), scal.begin(), scal.end());
  const uint64_t h = fnv(key.data(), key.size(), 1469598103934665603ull ^ (uint64_t)n ^ (rowmajor ? 1ull << 40 : 0));
  for (size_t k = 0; k < B->sets.size(); ++k) {
    const PackedSet& S = B->sets[k];
    if (S.hash == h && S.n == n && S.rowmajor == rowmajor && S.key == key) return (int)k;
  }
  PackedSet S;
  S.n = n;
  S.rowmajor = rowmajor;
  S.key = std::move(key);
  S.hash = h;
  S.count = count;
  S.A_dev = A_dev;
  B->sets.push_back(std::move(S));
  return (int)B->sets.size() - 1;
}

// phi bank of every instance (the set-up of Algorithms 1 and 2), one phi
// build per distinct (A, scalars).  Synchronises s.
int build_banks(setd_batch* B, const std::vector<std::vector<double>>& Ah, const double* const* A, hipStream_t s) {
  const int d = B->d, T = B->nterms;
  for (int b = 0; b < B->nb; ++b)
    for (int c = 0; c < B->ncomp; ++c)
      for (int mu = 0; mu < d; ++mu) {
        const int n = B->inst[b].dims[mu];
        const int k = (b * B->ncomp + c) * d + mu;
        std::vector<double> scal;
        for (int e = 0; e < 5; ++e) {
          const Splitting& S = B->sp[kBankEll[e]];
          for (int t = 0; t < T; ++t) scal.push_back(stage_scale(kBankStage[e]) * B->tau * S.alpha[t][mu]);
        }
        B->inst[b].bank[c][mu] = find_set(B, n, mu == 0, Ah[k], scal, 5 * T, A[k]);
        B->inst[b].apk[c][mu] =
            B->tridiag ? kNoPacked : find_set(B, n, mu == 0, Ah[k], std::vector<double>(), 1, A[k]);
      }
  size_t bytes = 0;
  for (PackedSet& S : B->sets) {
    S.offset = bytes;
    bytes += (size_t)S.count * packed_bytes(S.n, SETD_PREC_F64);
  }
  SETD_TRY(B->bank_mem.alloc(bytes));
  for (size_t k = 0; k < B->sets.size(); ++k) {
    const PackedSet& S = B->sets[k];
    const int n = S.n;
    if (S.count == 1) {   // A itself, for the dense K action
      SETD_TRY(pack_matrix_f64(S.A_dev, n, 1.0, S.rowmajor, (double*)packed(B, (int)k, 0), s));
      continue;
    }
    const std::vector<double> scal(S.key.begin() + (size_t)n * n, S.key.end());
    const int E = (int)scal.size();
    const size_t nn = (size_t)n * n;
    DevBuf raw;
    SETD_TRY(raw.alloc((size_t)E * 3 * nn * sizeof(double)));
    std::vector<double*> outs(E * 3);
    for (int j = 0; j < E * 3; ++j) outs[j] = (double*)raw.p + (size_t)j * nn;
    SETD_TRY(phi_batch(S.A_dev, n, scal.data(), E, 2, outs.data(), s));
    for (int e = 0; e < 5; ++e)
      for (int t = 0; t < T; ++t) {
        const int j = e * T + t;
        const int li = B->sp[kBankEll[e]].ell_i[t];
        SETD_TRY(pack_matrix_f64(outs[j * 3 + li], n, 1.0, S.rowmajor, (double*)packed(B, (int)k, j), s));
      }
    SETD_HIP(hipStreamSynchronize(s));   // raw is released at scope exit
  }
  SETD_HIP(hipStreamSynchronize(s));
  return SETD_OK;
}

// ---- work lists ----
struct Term {
  const double* X;
  const void* P[3];
  double scale;
  double* Y1;
  double* Y2;
};
struct Out {
  int b;
  double* Y;
  const double* base;
  int nterms;
  Term term[kMaxTerms];
};

struct PlanBuilder {
  setd_batch* B;
  const int* c1;
  const int* cb;
  std::vector<Op> ops;
  std::vector<std::vector<ModeJob>> lists;   // host jobs of each list op (same order as list ops)

  // Splits jobs by kernel variant and appends one list launch per variant.
  void add_lists(std::vector<ModeJob>& jobs, bool mode1) {
    const int* cfg = mode1 ? c1 : cb;
    std::vector<ModeJob> part[3];
    for (const ModeJob& jb : jobs) part[job_mode(jb, mode1, cfg[0], cfg[1])].push_back(jb);
    for (int m = 2; m >= 0; --m) {
      if (part[m].empty()) continue;
      Op op{};
      op.list = true;
      op.L.njobs = (int)part[m].size();
      op.L.total = assign_tiles(part[m].data(), op.L.njobs, mode1, cfg[0], cfg[1]);
      op.L.mode1 = mode1;
      op.L.tm = cfg[0];
      op.L.tn = cfg[1];
      op.L.mode = m;
      op.L.grid_cap = cfg[2];
      for (const ModeJob& jb : part[m]) {
        const double N = (double)jb.na * jb.n * jb.nb;
        op.L.flops += jb.nterms * 2.0 * N * jb.n;
        op.L.bytes += jb.nterms * (N * 8 + (double)jb.n * jb.n * 8) + N * 8 * (jb.base ? 2.0 : 1.0);
      }
      ops.push_back(op);
      lists.push_back(std::move(part[m]));
    }
    jobs.clear();
  }

  void pointwise(int kind, const double* x, double* G, double* out) {
    Op op{};
    op.list = false;
    op.pk = kind;
    op.x = x;
    op.G = G;
    op.out = out;
    ops.push_back(op);
  }

  // All outputs of one Tucker group over every instance (cf. the grouped
  // launches of the single-instance step): mode 1 into Y1, inner modes
  // ping-pong, last mode summing the terms and adding the base.
  // part: 0 all modes, 1 mode 1 only, 2 modes >= 2 only (for the tuner).
  void group(const std::vector<Out>& outs, int part = 0) {
    const int d = B->d;
    std::vector<ModeJob> jobs;
    if (part != 2) {
      for (const Out& o : outs) {
        const Inst& I = B->inst[o.b];
        for (int t = 0; t < o.nterms; ++t) {
          const Term& tm = o.term[t];
          jobs.push_back(mk_job(tm.X, tm.P[0], 1.0, tm.Y1, nullptr, 1, I.dims[0], I.N / I.dims[0]));
        }
      }
      add_lists(jobs, true);
      if (part == 1) return;
    }
    {
      for (int mu = 1; mu < d - 1; ++mu) {
        for (const Out& o : outs) {
          const Inst& I = B->inst[o.b];
          int64_t na = 1;
          for (int nu = 0; nu < mu; ++nu) na *= I.dims[nu];
          for (int t = 0; t < o.nterms; ++t) {
            const Term& tm = o.term[t];
            const double* src = (mu % 2 == 1) ? tm.Y1 : tm.Y2;
            double* dst = (mu % 2 == 1) ? tm.Y2 : tm.Y1;
            jobs.push_back(mk_job(src, tm.P[mu], 1.0, dst, nullptr, na, I.dims[mu], I.N / (na * I.dims[mu])));
          }
        }
        add_lists(jobs, false);
      }
    }
    const int mu = d - 1;
    for (const Out& o : outs) {
      const Inst& I = B->inst[o.b];
      ModeJob jb{};
      jb.nterms = o.nterms;
      for (int t = 0; t < o.nterms; ++t) {
        const Term& tm = o.term[t];
        jb.X[t] = (mu % 2 == 1) ? tm.Y1 : tm.Y2;
        jb.P[t] = tm.P[mu];
        jb.scale[t] = tm.scale;
      }
      jb.Y = o.Y;
      jb.base = o.base;
      jb.na = I.N / I.dims[mu];
      jb.nb = 1;
      jb.n = I.dims[mu];
      jb.ldp = packed_ld(jb.n);
      jobs.push_back(jb);
    }
    add_lists(jobs, false);
  }

  // Outputs of the phi_1 group on F (stages 2, 3 and final) for every
  // instance; `base` replaces u as the added field when non-null.
  std::vector<Out> f_group(double* u, const double* base_override) {
    const int T = B->nterms;
    const double tau = B->tau;
    const int e21 = bank_index(SETD_STAGE_2, 1), e31 = bank_index(SETD_STAGE_3, 1), ef1 = bank_index(SETD_STAGE_F, 1);
    std::vector<Out> outs;
    for (int b = 0; b < B->nb; ++b) {
      const Inst& I = B->inst[b];
      for (int c = 0; c < B->ncomp; ++c) {
        const int64_t o = I.off + c * I.cs;
        const struct {
          int e;
          double mult;
          double* Y;
        } tg[3] = {{e21, tau / 3.0, B->U2 + o}, {e31, 2.0 * tau / 3.0, B->U3 + o}, {ef1, tau, B->W + o}};
        for (int k = 0; k < 3; ++k) {
          Out out{};
          out.b = b;
          out.Y = tg[k].Y;
          out.base = base_override ? base_override + o : u + o;
          out.nterms = T;
          for (int t = 0; t < T; ++t) {
            Term& tm = out.term[t];
            tm.X = B->F + o;
            for (int mu = 0; mu < B->d; ++mu) tm.P[mu] = packed(B, I.bank[c][mu], tg[k].e * T + t);
            tm.scale = tg[k].mult * B->sp[1].eta[t];
            tm.Y1 = y1(B, b, c, k * T + t);
            tm.Y2 = y2(B, b, c, k * T + t);
          }
          outs.push_back(out);
        }
      }
    }
    return outs;
  }

  // Outputs of a phi_2 group on D: Y = base + mult * S_2 D.
  std::vector<Out> d_group(int e, double mult, double* Yall, const double* baseall) {
    const int T = B->nterms;
    std::vector<Out> outs;
    for (int b = 0; b < B->nb; ++b) {
      const Inst& I = B->inst[b];
      for (int c = 0; c < B->ncomp; ++c) {
        const int64_t o = I.off + c * I.cs;
        Out out{};
        out.b = b;
        out.Y = Yall + o;
        out.base = baseall + o;
        out.nterms = T;
        for (int t = 0; t < T; ++t) {
          Term& tm = out.term[t];
          tm.X = B->D + o;
          for (int mu = 0; mu < B->d; ++mu) tm.P[mu] = packed(B, I.bank[c][mu], e * T + t);
          tm.scale = mult * B->sp[2].eta[t];
          tm.Y1 = y1(B, b, c, t);
          tm.Y2 = y2(B, b, c, t);
        }
        outs.push_back(out);
      }
    }
    return outs;
  }

  // G = g(u), F = K u + G: stencil, or dense mu-mode products of A.
  void gf(double* u) {
    if (B->tridiag) {
      pointwise(0, u, B->G, B->F);
      return;
    }
    pointwise(1, u, B->G, nullptr);
    std::vector<ModeJob> jobs;
    for (int b = 0; b < B->nb; ++b) {
      const Inst& I = B->inst[b];
      for (int c = 0; c < B->ncomp; ++c) {
        const int64_t o = I.off + c * I.cs;
        jobs.push_back(mk_job(u + o, packed(B, I.apk[c][0], 0), 1.0, B->F + o, B->G + o, 1, I.dims[0],
                              I.N / I.dims[0]));
      }
    }
    add_lists(jobs, true);
    for (int mu = 1; mu < B->d; ++mu) {
      for (int b = 0; b < B->nb; ++b) {
        const Inst& I = B->inst[b];
        int64_t na = 1;
        for (int nu = 0; nu < mu; ++nu) na *= I.dims[nu];
        for (int c = 0; c < B->ncomp; ++c) {
          const int64_t o = I.off + c * I.cs;
          jobs.push_back(mk_job(u + o, packed(B, I.apk[c][mu], 0), 1.0, B->F + o, B->F + o, na, I.dims[mu],
                                I.N / (na * I.dims[mu])));
        }
      }
      add_lists(jobs, false);
    }
  }

  // One split-ETD3 step (the time loop of Algorithms 1 and 2).
  void step(double* u) {
    const double tau = B->tau;
    gf(u);
    group(f_group(u, nullptr));
    pointwise(2, B->U2, B->G, B->D);
    group(d_group(bank_index(SETD_STAGE_3, 2), 4.0 * tau / 3.0, B->U3, B->U3));
    pointwise(2, B->U3, B->G, B->D);
    group(d_group(bank_index(SETD_STAGE_F, 2), 1.5 * tau, u, B->W));
  }

  // Uploads every list (job records, then the array of first tiles) into
  // `mem` and points the list ops at it.
  int upload(DevBuf& mem, std::vector<Op>& out) {
    size_t njobs = 0;
    for (const auto& l : lists) njobs += l.size();
    std::vector<ModeJob> all;
    std::vector<int64_t> begins;
    all.reserve(njobs);
    begins.reserve(njobs);
    for (const auto& l : lists)
      for (const ModeJob& jb : l) {
        all.push_back(jb);
        begins.push_back(jb.tile_begin);
      }
    const size_t jbytes = round_up((int64_t)(njobs * sizeof(ModeJob)), 256);
    const size_t need = std::max<size_t>(jbytes + njobs * sizeof(int64_t), 256);
    if (mem.bytes < need) SETD_TRY(mem.alloc(need));
    const ModeJob* jdev = (const ModeJob*)mem.p;
    const int64_t* bdev = (const int64_t*)((char*)mem.p + jbytes);
    if (njobs) {
      SETD_HIP(hipMemcpy(mem.p, all.data(), njobs * sizeof(ModeJob), hipMemcpyHostToDevice));
      SETD_HIP(hipMemcpy((void*)bdev, begins.data(), njobs * sizeof(int64_t), hipMemcpyHostToDevice));
    }
    size_t at = 0, li = 0;
    for (Op& op : ops)
      if (op.list) {
        op.L.jobs = jdev + at;
        op.L.begins = bdev + at;
        at += lists[li++].size();
      }
    out = ops;
    return SETD_OK;
  }
};

int run_op(setd_batch* B, const Op& op, hipStream_t s) {
  if (op.list) return launch_list_f64(op.L, s);
  return launch_batch_pointwise(op.pk, B->inst_dev, B->blk_dev, B->nb, B->nblocks, B->ncomp, B->points, op.x, op.G,
                                op.out, s);
}

int run_ops(setd_batch* B, const std::vector<Op>& ops, hipStream_t s) {
  for (const Op& op : ops) SETD_TRY(run_op(B, op, s));
  return SETD_OK;
}

void drop_graph(setd_batch* B) {
  if (B->gexec) (void)hipGraphExecDestroy(B->gexec);
  B->gexec = nullptr;
}

// Work lists of one step for state buffer u with the current tile choice.
int build_plan(setd_batch* B, double* u) {
  PlanBuilder pb{B, B->cfg1, B->cfgB, {}, {}};
  pb.step(u);
  drop_graph(B);
  SETD_TRY(pb.upload(B->list_mem, B->plan));
  B->plan_u = u;
  return SETD_OK;
}

int capture(setd_batch* B) {
  drop_graph(B);
  if (!B->gstream) SETD_HIP(hipStreamCreateWithFlags(&B->gstream, hipStreamNonBlocking));
  if (!B->ev_in) SETD_HIP(hipEventCreateWithFlags(&B->ev_in, hipEventDisableTiming));
  if (!B->ev_out) SETD_HIP(hipEventCreateWithFlags(&B->ev_out, hipEventDisableTiming));
  SETD_HIP(hipStreamBeginCapture(B->gstream, hipStreamCaptureModeThreadLocal));
  const int rc = run_ops(B, B->plan, B->gstream);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(B->gstream, &graph);
  if (rc != SETD_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess || !graph) {
    set_error("batch step capture failed: %s", hipGetErrorString(e));
    return SETD_EHIP;
  }
  const hipError_t ei = hipGraphInstantiate(&B->gexec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) {
    B->gexec = nullptr;
    set_error("batch graph instantiation failed: %s", hipGetErrorString(ei));
    return SETD_EHIP;
  }
  return SETD_OK;
}

bool batch_use_graph() {
  const char* e = std::getenv("SETD_GRAPH");
  if (e && e[0] == '0') return false;
  return !prof_on();
}

// ---- autotuner ----
// Times the mode-product lists of the phi_1 group on F (the largest group of
// the step; its outputs and intermediates are internal buffers, G stands in
// for the added field) for each candidate tile shape and grid cap, per
// regime, and keeps the fastest.
const int kCand[4][2] = {{2, 2}, {2, 4}, {4, 2}, {4, 4}};
const int kCaps[3] = {0, 2048, 8192};

int time_ops(setd_batch* B, const std::vector<Op>& ops, hipStream_t s, int reps, float& ms) {
  hipEvent_t e0, e1;
  SETD_HIP(hipEventCreate(&e0));
  SETD_HIP(hipEventCreate(&e1));
  int rc = run_ops(B, ops, s);   // warm-up
  if (rc == SETD_OK && hipEventRecord(e0, s) != hipSuccess) rc = SETD_EHIP;
  for (int r = 0; r < reps && rc == SETD_OK; ++r) rc = run_ops(B, ops, s);
  if (rc == SETD_OK && hipEventRecord(e1, s) != hipSuccess) rc = SETD_EHIP;
  if (rc == SETD_OK && hipEventSynchronize(e1) != hipSuccess) rc = SETD_EHIP;
  if (rc == SETD_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = SETD_EHIP;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc == SETD_EHIP) set_error("timing the candidate tiles failed");
  return rc;
}

int tune(setd_batch* B, hipStream_t s) {
  const bool was_prof = prof_on();
  for (int regime = 0; regime < 2; ++regime) {
    float best = 1e30f;
    int bestc[3] = {0, 0, 0};
    for (const auto& cand : kCand)
      for (int cap : kCaps) {
        int c1[3] = {B->cfg1[0], B->cfg1[1], B->cfg1[2]}, cb[3] = {B->cfgB[0], B->cfgB[1], B->cfgB[2]};
        int* c = regime == 0 ? c1 : cb;
        c[0] = cand[0];
        c[1] = cand[1];
        c[2] = cap;
        PlanBuilder pb{B, c1, cb, {}, {}};
        pb.group(pb.f_group(nullptr, B->G), regime == 0 ? 1 : 2);
        std::vector<Op> ops;
        SETD_TRY(pb.upload(B->tune_mem, ops));
        float ms = 0.0f;
        SETD_TRY(time_ops(B, ops, s, 3, ms));
        if (ms < best) {
          best = ms;
          bestc[0] = c[0];
          bestc[1] = c[1];
          bestc[2] = c[2];
        }
      }
    int* dst = regime == 0 ? B->cfg1 : B->cfgB;
    for (int k = 0; k < 3; ++k) dst[k] = bestc[k];
  }
  (void)was_prof;
  B->tuned = true;
  B->plan_u = nullptr;   // rebuild the plan with the new shapes
  drop_graph(B);
  return SETD_OK;
}

bool valid_tile(int tm, int tn) { return (tm == 2 || tm == 4) && (tn == 2 || tn == 4); }

}  // namespace

extern "C" {

int setd_batch_create(setd_batch** out, int nbatch, int d, const int64_t* dims, int ncomp, const double* const* A,
                      double tau, int prec, void* stream) {
  clear_error();
  SETD_CHECK_ARG(out != nullptr, "batch out-pointer is NULL");
  *out = nullptr;
  SETD_CHECK_ARG(nbatch >= 1 && nbatch <= 65536, "nbatch = %d outside 1..65536", nbatch);
  SETD_CHECK_ARG(d == 2 || d == 3, "d = %d: the split integrator supports d = 2 and d = 3", d);
  SETD_CHECK_ARG(dims != nullptr && A != nullptr, "dims and A must be non-NULL");
  SETD_CHECK_ARG(ncomp == 1 || ncomp == 2, "ncomp = %d outside 1..2", ncomp);
  SETD_CHECK_ARG(tau > 0.0, "tau must be positive");
  if (!std::isfinite(tau)) {
    set_error("tau is not finite");
    return SETD_ENONFINITE;
  }
  SETD_CHECK_ARG(is_prec(prec), "bad prec %d", prec);
  if (prec != SETD_PREC_F64) {
    set_error("the batched integrator runs in FP64 only");
    return SETD_EUNSUPPORTED;
  }
  for (int k = 0; k < nbatch * d; ++k)
    SETD_CHECK_ARG(dims[k] >= 2 && dims[k] <= 1024, "dims[%d] = %lld outside 2..1024", k, (long long)dims[k]);
  for (int k = 0; k < nbatch * ncomp * d; ++k) SETD_CHECK_ARG(A[k] != nullptr, "A[%d] is NULL", k);
  hipStream_t s = (hipStream_t)stream;

  setd_batch* B = new (std::nothrow) setd_batch();
  if (!B) {
    set_error("out of host memory");
    return SETD_ENOMEM;
  }
  auto fail = [&](int code) {
    delete B;
    return code;
  };
  B->nb = nbatch;
  B->d = d;
  B->ncomp = ncomp;
  B->tau = tau;
  B->sp[1] = splitting(1, d);
  B->sp[2] = splitting(2, d);
  B->nterms = B->sp[1].nterms;
  const int T = B->nterms;
  B->inst.resize(nbatch);
  for (int b = 0; b < nbatch; ++b) {
    Inst& I = B->inst[b];
    I.N = 1;
    for (int mu = 0; mu < d; ++mu) {
      I.dims[mu] = (int)dims[b * d + mu];
      I.N *= I.dims[mu];
    }
    I.cs = round_up(I.N, 8);
    I.off = B->total;
    I.yoff = B->ytotal;
    B->total += ncomp * I.cs;
    B->ytotal += (int64_t)ncomp * 3 * T * I.cs;
    B->points += I.N;
  }
  // host copies of A; tridiagonal check; finiteness
  std::vector<std::vector<double>> Ah((size_t)nbatch * ncomp * d);
  for (int b = 0; b < nbatch; ++b)
    for (int c = 0; c < ncomp; ++c)
      for (int mu = 0; mu < d; ++mu) {
        const int k = (b * ncomp + c) * d + mu;
        const int n = B->inst[b].dims[mu];
        Ah[k].resize((size_t)n * n);
        hipError_t e = hipMemcpy(Ah[k].data(), A[k], (size_t)n * n * 8, hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
          set_error("copying A[%d] failed: %s", k, hipGetErrorString(e));
          return fail(SETD_EHIP);
        }
        for (double v : Ah[k])
          if (!std::isfinite(v)) {
            set_error("A[%d] has non-finite entries", k);
            return fail(SETD_ENONFINITE);
          }
        B->tridiag = B->tridiag && is_tridiagonal(Ah[k], n);
      }
  int rc = SETD_OK;
  // instance table for the pointwise kernels (+ stencil coefficients)
  B->inst_host.resize(nbatch);
  B->blk_host.resize(nbatch);
  {
    std::vector<double> h;
    std::vector<size_t> where((size_t)nbatch * ncomp * d);
    if (B->tridiag)
      for (int b = 0; b < nbatch; ++b)
        for (int c = 0; c < ncomp; ++c)
          for (int mu = 0; mu < d; ++mu) {
            const int k = (b * ncomp + c) * d + mu;
            const int n = B->inst[b].dims[mu];
            const std::vector<double>& M = Ah[k];
            where[k] = h.size();
            for (int i = 0; i < n; ++i) h.push_back(i > 0 ? M[i + (size_t)n * (i - 1)] : 0.0);
            for (int i = 0; i < n; ++i) h.push_back(M[i + (size_t)n * i]);
            for (int i = 0; i < n; ++i) h.push_back(i + 1 < n ? M[i + (size_t)n * (i + 1)] : 0.0);
          }
    if (!h.empty()) {
      if ((rc = B->stencil_mem.alloc(h.size() * 8)) != SETD_OK) return fail(rc);
      hipError_t e = hipMemcpy(B->stencil_mem.p, h.data(), h.size() * 8, hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        set_error("stencil upload failed: %s", hipGetErrorString(e));
        return fail(SETD_EHIP);
      }
    }
    int64_t blk = 0;
    for (int b = 0; b < nbatch; ++b) {
      const Inst& I = B->inst[b];
      BatchInstDev& D = B->inst_host[b];
      D = BatchInstDev{};
      D.off = I.off;
      D.cs = I.cs;
      D.N = I.N;
      D.d = d;
      for (int mu = 0; mu < 3; ++mu) D.n[mu] = I.dims[mu];
      D.gp.kind = SETD_G_NONE;
      D.gp.p[3] = 1.0;
      if (B->tridiag)
        for (int c = 0; c < ncomp; ++c)
          for (int mu = 0; mu < d; ++mu) {
            const int k = (b * ncomp + c) * d + mu;
            const double* base = (const double*)B->stencil_mem.p + where[k];
            const int n = I.dims[mu];
            D.st.lo[c * 3 + mu] = base;
            D.st.di[c * 3 + mu] = base + n;
            D.st.up[c * 3 + mu] = base + 2 * n;
          }
      B->blk_host[b] = blk;
      blk += ceil_div(I.N, kBatchBlock);
    }
    B->nblocks = blk;
    const size_t ib = round_up((int64_t)(nbatch * sizeof(BatchInstDev)), 256);
    if ((rc = B->inst_mem.alloc(ib + nbatch * sizeof(int64_t))) != SETD_OK) return fail(rc);
    B->inst_dev = (BatchInstDev*)B->inst_mem.p;
    B->blk_dev = (int64_t*)((char*)B->inst_mem.p + ib);
    hipError_t e = hipMemcpy(B->inst_dev, B->inst_host.data(), nbatch * sizeof(BatchInstDev), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(B->blk_dev, B->blk_host.data(), nbatch * sizeof(int64_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      set_error("instance table upload failed: %s", hipGetErrorString(e));
      return fail(SETD_EHIP);
    }
  }
  // work buffers: G F U2 U3 W D (u-shaped) + Y1 (+ Y2 for d = 3), zeroed
  {
    const int64_t elems = 6 * B->total + B->ytotal * (d == 3 ? 2 : 1);
    if ((rc = B->work_mem.alloc((size_t)elems * 8)) != SETD_OK) return fail(rc);
    hipError_t e = hipMemset(B->work_mem.p, 0, (size_t)elems * 8);
    if (e != hipSuccess) {
      set_error("clearing the work buffers failed: %s", hipGetErrorString(e));
      return fail(SETD_EHIP);
    }
    double* q = (double*)B->work_mem.p;
    B->G = q;
    B->F = q + B->total;
    B->U2 = q + 2 * B->total;
    B->U3 = q + 3 * B->total;
    B->W = q + 4 * B->total;
    B->D = q + 5 * B->total;
    B->Y1 = q + 6 * B->total;
    B->Y2 = d == 3 ? B->Y1 + B->ytotal : nullptr;
  }
  if ((rc = build_banks(B, Ah, A, s)) != SETD_OK) return fail(rc);
  *out = B;
  return SETD_OK;
}

int setd_batch_destroy(setd_batch* B) {
  clear_error();
  if (!B) return SETD_OK;
  (void)hipDeviceSynchronize();
  delete B;
  return SETD_OK;
}

int setd_batch_layout(const setd_batch* B, int64_t* off, int64_t* cs) {
  clear_error();
  SETD_CHECK_ARG(B != nullptr, "batch is NULL");
  SETD_CHECK_ARG(off != nullptr, "off is NULL");
  for (int b = 0; b < B->nb; ++b) {
    off[b] = B->inst[b].off;
    if (cs) cs[b] = B->inst[b].cs;
  }
  off[B->nb] = B->total;
  return SETD_OK;
}

int setd_batch_tune(setd_batch* B, void* stream) {
  clear_error();
  SETD_CHECK_ARG(B != nullptr, "batch is NULL");
  return tune(B, (hipStream_t)stream);
}

int setd_batch_set_tiles(setd_batch* B, const int* cfg) {
  clear_error();
  SETD_CHECK_ARG(B != nullptr && cfg != nullptr, "batch and cfg must be non-NULL");
  SETD_CHECK_ARG(valid_tile(cfg[0], cfg[1]) && valid_tile(cfg[3], cfg[4]), "tiles must be 2 or 4 on each side");
  SETD_CHECK_ARG(cfg[2] >= 0 && cfg[5] >= 0, "grid caps must be >= 0");
  for (int k = 0; k < 3; ++k) {
    B->cfg1[k] = cfg[k];
    B->cfgB[k] = cfg[3 + k];
  }
  B->tuned = true;
  B->plan_u = nullptr;
  drop_graph(B);
  return SETD_OK;
}

int setd_batch_info(const setd_batch* B, int64_t* info) {
  clear_error();
  SETD_CHECK_ARG(B != nullptr && info != nullptr, "batch and info must be non-NULL");
  for (int k = 0; k < 3; ++k) {
    info[k] = B->cfg1[k];
    info[3 + k] = B->cfgB[k];
  }
  info[6] = B->tuned ? 1 : 0;
  info[7] = (int64_t)B->plan.size();
  info[8] = B->total;
  info[9] = (int64_t)B->sets.size();
  return SETD_OK;
}

int setd_batch_step(setd_batch* B, double* u, int nsteps, int g_kind, const double* params, int nparams,
                    void* stream) {
  clear_error();
  SETD_CHECK_ARG(B != nullptr, "batch is NULL");
  SETD_CHECK_ARG(u != nullptr, "u is NULL");
  SETD_CHECK_ARG(nsteps >= 0, "nsteps < 0");
  SETD_CHECK_ARG(nparams == 0 || params != nullptr, "params is NULL");
  hipStream_t s = (hipStream_t)stream;
  // per-instance reaction parameters
  for (int b = 0; b < B->nb; ++b) {
    GParams gp;
    SETD_TRY(make_gparams(g_kind, params ? params + (size_t)b * nparams : nullptr, nparams, B->ncomp, gp));
    GParams& cur = B->inst_host[b].gp;
    bool same = cur.kind == gp.kind;
    for (int k = 0; k < 4; ++k) same = same && cur.p[k] == gp.p[k];
    if (!same) {
      cur = gp;
      B->params_dirty = true;
    }
  }
  if (nsteps == 0) return SETD_OK;
  if (B->params_dirty) {
    // ordered after earlier replays (the caller's stream waits for them)
    SETD_HIP(hipMemcpyAsync(B->inst_dev, B->inst_host.data(), B->nb * sizeof(BatchInstDev), hipMemcpyHostToDevice,
                            s));
    SETD_HIP(hipStreamSynchronize(s));
    B->params_dirty = false;
  }
  if (!B->tuned) {
    const char* e = std::getenv("SETD_BATCH_TUNE");
    if (e && e[0] == '0') B->tuned = true;   // keep the default shapes
    else SETD_TRY(tune(B, s));
  }
  if (B->plan_u != u) {
    SETD_HIP(hipStreamSynchronize(s));   // earlier replays may still read the lists
    SETD_TRY(build_plan(B, u));
  }
  if (batch_use_graph()) {
    int rc = B->gexec ? SETD_OK : capture(B);
    if (rc == SETD_OK) {
      SETD_HIP(hipEventRecord(B->ev_in, s));
      SETD_HIP(hipStreamWaitEvent(B->gstream, B->ev_in, 0));
      for (int k = 0; k < nsteps; ++k) SETD_HIP(hipGraphLaunch(B->gexec, B->gstream));
      SETD_HIP(hipEventRecord(B->ev_out, B->gstream));
      SETD_HIP(hipStreamWaitEvent(s, B->ev_out, 0));
      return SETD_OK;
    }
    drop_graph(B);
    clear_error();
  }
  for (int k = 0; k < nsteps; ++k) SETD_TRY(run_ops(B, B->plan, s));
  return SETD_OK;
}

}  // extern "C"
