// C ABI of libngd (include/ngd.h): argument validation, workspace, and the host-side sequencing of
// the device kernels for each entry point.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"

namespace ngd {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

}  // namespace ngd

using namespace ngd;

struct ngd_problem {
  NetDesc net;
  bool ns = false;   // Navier-Stokes rows: two networks (nsd), their own residual kernel
  NsDesc nsd{};
  int dtype;
  int64_t N, P, ldP;
  int max_ell;
  const void *X, *w, *f, *g;
  const int8_t* kind;
  int tp;            // rows per residual workgroup
  int res_blocks;    // residual workgroups per parameter vector
  int nwg;           // one-pass matvec workgroups
  size_t elem;
  // device workspace (one allocation)
  void* base;
  size_t bytes;
  void* partial;     // nwg x ldP, dtype
  double* tsq;       // nwg
  double* loss_part; // res_blocks * kTrials
  double* err_part;  // 4 * kEvalBlocks partial sums of the solution error
  double* diag_work; // kDiagChunks * ldP partial column sums of squares (Gramian diagonal)
  // block RPCholesky workspace (allocated on first use): downdated diagonal, pivots, their count,
  // state {rank, done, kept}, C^T (64 x ldP), F[S', :] (64 x 1024), gathered columns of J (N x 64),
  // the pivot block's factor, kept-row map, block partial sums, residual trace
  void* rp_blob = nullptr;
  double *rp_d, *rp_Ct, *rp_W, *rp_Rt, *rp_part, *rp_trace;
  int64_t *rp_idx, *rp_st;
  int *rp_cnt, *rp_keep;
  void* rp_Jcols;
  double* rp_F = nullptr;  // Woodbury form: F row-major (P x max_ell doubles), on first use
  // full-Gramian solve workspace (allocated on first use): G / its factor (P x ldP), the panels'
  // inverse diagonal blocks, the panel staging rows, substitution partials, y, the pivot word
  void* dr_blob = nullptr;
  double *dr_G, *dr_Linv, *dr_stage, *dr_part, *dr_y;
  int* dr_info;
  double* grad_work; // gradient_chunks(N) x P
  double* vtmp[4];   // P-vectors (FP64)
  double* scal;      // small scalars / dot workspace (128 doubles)
  double* pcg_r;
  double* pcg_z;
  double* pcg_p[2];
  double* pcg_s;     // kDotChunksMax x max_ell: column-chunk partials of the preconditioner dots
  double* pcg_part;  // block partials (P / 256)
  PcgState* pcg_st;
  void* omega;       // max_ell x ldP, dtype
  void* Z;           // N x max_ell, dtype
  void* Q;           // N x max_ell, FP64 (orthonormal basis of range(Z))
  void* Bt;          // max_ell x ldP, dtype
  int64_t ldN;       // row stride of the transposed sketch operands (N rounded up to 64)
  void* Jt;          // P x ldN, J_w^T in BF16 for the BF16 sketch (FP32 problems)
  void* Qt;          // max_ell x ldN, Q^T in the sketch compute type (FP32 problems)
  void* Ob;          // max_ell x ldP, Omega^T in BF16 (FP32 problems)
  void* Jc = nullptr;  // recompute-mode sketch: a block of rows of J_w (jc_rows x ldP, dtype), on first use
  int64_t jc_rows = 0;
  double* nvec[2];   // N-vectors (FP64): recompute-mode J v and adjoint weights
  void* pt;          // ldP, dtype: the current CG direction for the recompute-mode JVP
  int nwg_vjp;       // workgroups of the recompute-mode adjoint product
  float* sk_work;    // split-K partials of the sketch products (FP32 problems)
  int64_t sk_work_elems;
  double* M;         // ell x ell
  double* Ev;        // ell x ell eigenvectors (rows)
  double* F;         // ell x ell
  double* evals;     // ell
  double* gemm_work; // split-K partials of the ell x ell Gram products
  int64_t gemm_work_elems;  // 32 max_ell^2: room for 16 slices, enough to fill the chip with the Gram tiles
  unsigned* cholsync;  // the Cholesky's row-block flags (2 x 64) and error word
  unsigned chol_epoch = 0;
  void* eigw;        // eig workspace
  void* trial;       // kTrials x ldP, dtype (line search)
  double* alphas;    // kTrials
  double* losses;    // kTrials
  // pinned host staging
  void* host;
  // a second stream (default priority) for sketch work that is independent of the FP64 core, and
  // the events that fork it from and join it to the caller's stream
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // kernel timers
  uint32_t timing = 0;  // bit id set: timer id records
  std::vector<hipEvent_t> ev_free;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
  double t_ms[NGD_NUM_TIMERS] = {};
  int64_t t_n[NGD_NUM_TIMERS] = {};
  // iterations of the previous solve (index: plain CG), used to size the first launch chunk
  int64_t last_iters[2] = {4, 4};
  // line-search trials per launch (set at creation from the residual kernel's occupancy), and in the
  // first launch of the next search: 1 while the full step keeps being accepted, ls_batch after a
  // search that had to halve (the same step is chosen either way)
  int ls_batch = 1;
  int ls_first_batch = 1;
  // ell of the last sketch taken without its summary (its core's error words not read yet), or 0
  int64_t unchecked_ell = 0;
};

namespace {

hipEvent_t take_event(ngd_problem* h) {
  if (!h->ev_free.empty()) {
    hipEvent_t e = h->ev_free.back();
    h->ev_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

ngd_status flush_timers(ngd_problem* h) {
  for (auto& p : h->ev_pending) {
    NGD_HIP_TRY(hipEventSynchronize(p.second.second));
    float ms = 0.f;
    NGD_HIP_TRY(hipEventElapsedTime(&ms, p.second.first, p.second.second));
    h->t_ms[p.first] += ms;
    h->t_n[p.first] += 1;
    h->ev_free.push_back(p.second.first);
    h->ev_free.push_back(p.second.second);
  }
  h->ev_pending.clear();
  return NGD_OK;
}

// Forget the last `count` pending records of timer `id` (launches that found the solver done and
// returned at once; they are not launches of the timed kernel's work).
void drop_tail(ngd_problem* h, int id, int64_t count) {
  for (auto it = h->ev_pending.end(); count > 0 && it != h->ev_pending.begin();) {
    --it;
    if (it->first != id) continue;
    h->ev_free.push_back(it->second.first);
    h->ev_free.push_back(it->second.second);
    it = h->ev_pending.erase(it);
    --count;
  }
}

// Run `fn` (which enqueues one kernel sequence on s); when timing is on, bracket it with events.
template <typename F>
ngd_status timed(ngd_problem* h, int id, hipStream_t s, F&& fn) {
  if (id < 0 || !((h->timing >> id) & 1u)) return fn();
  if (h->ev_pending.size() > 4096) {
    ngd_status st = flush_timers(h);
    if (st != NGD_OK) return st;
  }
  hipEvent_t a = take_event(h), b = take_event(h);
  if (!a || !b) {
    set_error("hipEventCreate failed");
    return NGD_ERR_HIP;
  }
  NGD_HIP_TRY(hipEventRecord(a, s));
  ngd_status st = fn();
  NGD_HIP_TRY(hipEventRecord(b, s));
  h->ev_pending.push_back({id, {a, b}});
  return st;
}

// As timed(), for a launcher that starts exactly one kernel: the events are handed to the launch and
// stamped with that kernel's own start and end, so the timer holds kernel time without marker overhead.
template <typename F>
ngd_status timed_kernel(ngd_problem* h, int id, F&& fn) {
  if (id < 0 || !((h->timing >> id) & 1u)) return fn(LaunchEvents{});
  if (h->ev_pending.size() > 4096) {
    ngd_status st = flush_timers(h);
    if (st != NGD_OK) return st;
  }
  LaunchEvents ev{take_event(h), take_event(h)};
  if (!ev.start || !ev.stop) {
    set_error("hipEventCreate failed");
    return NGD_ERR_HIP;
  }
  ngd_status st = fn(ev);
  h->ev_pending.push_back({id, {ev.start, ev.stop}});
  return st;
}

}  // namespace

namespace {

constexpr int kTrials = 8;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

#define NGD_CHECK(cond, msg)          \
  do {                                \
    if (!(cond)) {                    \
      ::ngd::set_error(msg);          \
      return NGD_ERR_INVALID;         \
    }                                 \
  } while (0)

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

ngd_status check_op(const ngd_problem* h, const ngd_operator* op) {
  NGD_CHECK(op != nullptr, "operator is NULL");
  if (op->J == nullptr) {  // recompute mode: J_w products from theta by the JVP / adjoint kernels
    NGD_CHECK(!h->ns, "the recompute mode (J == NULL) is not available for Navier-Stokes rows");
    NGD_CHECK(op->theta != nullptr, "recompute mode (J == NULL) needs theta");
    return NGD_OK;
  }
  NGD_CHECK(op->ldJ >= h->P, "ldJ < P");
  NGD_CHECK(op->ldJ <= h->ldP, "ldJ must not exceed ngd_recommended_ld");
  const int vn = h->dtype == NGD_F64 ? 2 : 4;
  NGD_CHECK(op->ldJ % vn == 0, "ldJ must be a multiple of 16 bytes / element size");
  NGD_CHECK(aligned16(op->J), "J must be 16-byte aligned");
  NGD_CHECK(gram_rows_supported(h->dtype, op->ldJ), "ldJ too large for the one-pass matvec");
  return NGD_OK;
}

// recompute mode: t = J_w v (v: P, dtype) into nvec[0], then the adjoint partials of J_w^T t
ngd_status recompute_rows(ngd_problem* h, const ngd_operator* op, const void* v_dtype, hipStream_t s) {
  NGD_TRY(launch_jvp(h->net, h->dtype, op->theta, v_dtype, h->ldP, 1, h->N, h->X, h->w, h->kind, NGD_F64, h->nvec[0],
                     1, 0, s));
  return launch_vjp(h->net, h->dtype, op->theta, h->N, h->X, h->w, h->f, h->g, h->kind, h->nvec[0], 1, h->partial,
                    h->ldP, h->tsq, h->nwg_vjp, s);
}

// y = (J^T J + lambda I) v, all FP64 P-vectors
ngd_status gram_apply(ngd_problem* h, const ngd_operator* op, const double* v, double lambda, double* y, hipStream_t s) {
  if (op->J == nullptr) {
    NGD_TRY(launch_cast(NGD_F64, v, h->dtype, h->pt, h->P, s));
    NGD_TRY(timed(h, NGD_TIMER_MATVEC_ROWS, s, [&] { return recompute_rows(h, op, h->pt, s); }));
    return launch_gram_reduce(h->dtype, h->partial, h->nwg_vjp, h->ldP, h->P, v, lambda, y, s);
  }
  NGD_TRY(timed_kernel(h, NGD_TIMER_MATVEC_ROWS, [&](LaunchEvents ev) {
    return launch_gram_rows(h->dtype, op->J, op->ldJ, h->N, h->P, v, h->partial, h->tsq, h->nwg, s, ev);
  }));
  return launch_gram_reduce(h->dtype, h->partial, h->nwg, op->ldJ, h->P, v, lambda, y, s);
}

}  // namespace

extern "C" {

const char* ngd_last_error(void) { return g_last_error.c_str(); }

ngd_status ngd_problem_create(const ngd_problem_desc* d, ngd_problem** out) {
  NGD_CHECK(d != nullptr && out != nullptr, "NULL argument");
  *out = nullptr;
  NGD_CHECK(d->n_layers >= 1 && d->n_layers <= kMaxLayers, "n_layers out of range [1, 8]");
  NGD_CHECK(d->widths != nullptr, "widths is NULL");
  NGD_CHECK(d->pde == NGD_PDE_POISSON || d->pde == NGD_PDE_HEAT || d->pde == NGD_PDE_NAVIER_STOKES,
            "unknown pde");
  const bool ns = d->pde == NGD_PDE_NAVIER_STOKES;
  NGD_CHECK(d->dtype == NGD_F64 || d->dtype == NGD_F32, "dtype must be NGD_F64 or NGD_F32");
  NGD_CHECK(d->n_rows >= 1, "n_rows must be >= 1");
  NGD_CHECK(d->X && d->w && d->f && d->g && d->row_kind, "problem data pointer is NULL");
  NGD_CHECK(d->max_ell >= 1, "max_ell must be >= 1");
  NGD_CHECK(d->max_ell <= kMaxEll, "max_ell must be <= 1024");
  NetDesc net{};
  net.n_layers = d->n_layers;
  int64_t off = 0;
  int maxw = 0;
  for (int l = 0; l <= d->n_layers; ++l) {
    NGD_CHECK(d->widths[l] >= 1 && d->widths[l] <= kMaxWidth, "widths out of range [1, 256]");
    net.widths[l] = d->widths[l];
    maxw = std::max(maxw, d->widths[l]);
  }
  NGD_CHECK(ns || d->widths[d->n_layers] == 1, "the output width must be 1");
  NsDesc nsd{};
  if (ns) {
    NGD_CHECK(d->n_layers >= 2, "Navier-Stokes networks need at least one hidden layer");
    NGD_CHECK(d->widths[0] == 2 && d->widths[d->n_layers] == 2,
              "Navier-Stokes velocity network: 2 inputs (x, y) and 2 outputs (u_1, u_2)");
    for (int l = 1; l < d->n_layers; ++l) NGD_CHECK(d->widths[l] <= 64, "Navier-Stokes hidden widths must be <= 64");
    NGD_CHECK(d->viscosity > 0.0, "viscosity must be > 0");
    NGD_TRY(ns_describe(d->n_layers, d->widths, d->viscosity, &nsd));
    NGD_CHECK(ns_lds_bytes(nsd, d->dtype) <= 160 * 1024,
              "Navier-Stokes networks too large for the residual kernel's LDS budget");
  }
  for (int l = 0; l < d->n_layers; ++l) {
    net.woff[l] = off;
    off += (int64_t)net.widths[l] * net.widths[l + 1];
    net.boff[l] = off;
    off += net.widths[l + 1];
  }
  net.P = ns ? nsd.P : off;
  net.d = d->widths[0];
  NGD_CHECK(net.d <= kMaxDim, "input dimension must be <= 6");
  NGD_CHECK(d->pde != NGD_PDE_HEAT || net.d >= 2, "heat needs at least one space and the time input");
  net.nS = d->pde == NGD_PDE_POISSON ? net.d : net.d - 1;
  net.has_t = d->pde == NGD_PDE_HEAT ? 1 : 0;
  net.C = 1 + net.nS + 1 + net.has_t;
  net.pde = d->pde;
  net.max_width = maxw;

  ngd_problem* h = new ngd_problem();
  h->net = net;
  h->ns = ns;
  h->nsd = nsd;
  h->dtype = d->dtype;
  h->N = d->n_rows;
  h->P = net.P;
  h->ldP = (int64_t)align_up((size_t)net.P, 64);
  h->max_ell = (int)std::min<int64_t>(d->max_ell, net.P);
  h->X = d->X;
  h->w = d->w;
  h->f = d->f;
  h->g = d->g;
  h->kind = d->row_kind;
  h->elem = d->dtype == NGD_F64 ? 8 : 4;
  h->tp = residual_block_rows(net, d->dtype);
  h->res_blocks = ns ? ns_blocks(h->N) : (int)((h->N + h->tp - 1) / h->tp);
  // Navier-Stokes trial losses: one per launch (a trial fills the device by itself, so a batch of trials
  // costs their sum and gains only the host round trips)
  h->ls_batch = ns ? 1 : residual_trials_per_launch(net, d->dtype, h->N, kTrials);
  h->nwg = gram_rows_grid(d->dtype, h->N, h->P);
  h->nwg_vjp = vjp_grid(net, d->dtype, h->N, h->nwg);

  const int64_t N = h->N, P = h->P, ldP = h->ldP, L = h->max_ell;
  const size_t e = h->elem;
  std::vector<std::pair<void**, size_t>> plan;
  plan.push_back({&h->partial, (size_t)h->nwg * ldP * e});
  plan.push_back({(void**)&h->tsq, sizeof(double) * 1024});
  plan.push_back({(void**)&h->loss_part, sizeof(double) * (size_t)h->res_blocks * kTrials});
  plan.push_back({(void**)&h->err_part, sizeof(double) * 4 * (size_t)kEvalBlocks});
  plan.push_back({(void**)&h->diag_work, sizeof(double) * (size_t)kDiagChunks * ldP});
  plan.push_back({(void**)&h->grad_work, sizeof(double) * (size_t)gradient_chunks(N) * P});
  for (int i = 0; i < 4; ++i) plan.push_back({(void**)&h->vtmp[i], sizeof(double) * ldP});
  plan.push_back({(void**)&h->scal, sizeof(double) * 256});
  plan.push_back({(void**)&h->pcg_r, sizeof(double) * ldP});
  plan.push_back({(void**)&h->pcg_z, sizeof(double) * ldP});
  plan.push_back({(void**)&h->pcg_p[0], sizeof(double) * ldP});
  plan.push_back({(void**)&h->pcg_p[1], sizeof(double) * ldP});
  plan.push_back({(void**)&h->pcg_s, sizeof(double) * (size_t)L * kDotChunksMax});
  plan.push_back({(void**)&h->pcg_part, sizeof(double) * (size_t)((P + 31) / 32 + 64)});
  plan.push_back({(void**)&h->pcg_st, sizeof(PcgState)});
  plan.push_back({&h->omega, (size_t)L * ldP * e});
  plan.push_back({&h->Z, (size_t)N * L * e});
  plan.push_back({&h->Q, (size_t)N * L * sizeof(double)});
  plan.push_back({&h->Bt, (size_t)L * ldP * e});
  h->ldN = (int64_t)align_up((size_t)N, 64);
  if (d->dtype == NGD_F32) {  // sized for FP32, which also holds the BF16 copies
    plan.push_back({&h->Jt, (size_t)P * h->ldN * 2});
    plan.push_back({&h->Qt, (size_t)L * h->ldN * 4});
    plan.push_back({&h->Ob, (size_t)L * ldP * 2});
    // room for up to 16 slices of the larger sketch product, between 64 and 256 MB
    h->sk_work_elems = std::min<int64_t>((int64_t)64 << 20,
                                         std::max<int64_t>((int64_t)16 << 20, 16 * L * std::max(N, P)));
    plan.push_back({(void**)&h->sk_work, (size_t)h->sk_work_elems * 4});
  }
  plan.push_back({(void**)&h->M, sizeof(double) * (size_t)L * L});
  plan.push_back({(void**)&h->Ev, sizeof(double) * (size_t)L * L});
  plan.push_back({(void**)&h->F, sizeof(double) * (size_t)L * L});
  plan.push_back({(void**)&h->evals, sizeof(double) * (size_t)L});
  h->gemm_work_elems = 32 * (int64_t)L * L;
  plan.push_back({(void**)&h->gemm_work, sizeof(double) * (size_t)h->gemm_work_elems});
  plan.push_back({(void**)&h->cholsync, sizeof(unsigned) * 256});
  plan.push_back({&h->eigw, eig_workspace_bytes((int)L)});
  plan.push_back({&h->trial, (size_t)kTrials * ldP * e});
  plan.push_back({(void**)&h->nvec[0], sizeof(double) * (size_t)N});
  plan.push_back({(void**)&h->nvec[1], sizeof(double) * (size_t)N});
  plan.push_back({&h->pt, (size_t)ldP * e});
  plan.push_back({(void**)&h->alphas, sizeof(double) * kTrials});
  plan.push_back({(void**)&h->losses, sizeof(double) * kTrials});
  size_t total = 0;
  for (auto& p : plan) total += align_up(p.second, 256);
  void* base = nullptr;
  if (const hipError_t e = hipMalloc(&base, total); e != hipSuccess) {
    (void)hipGetLastError();
    delete h;
    set_error("hipMalloc of the workspace failed (" + std::to_string(total) + " bytes): " + hipGetErrorString(e));
    return NGD_ERR_OOM;
  }
  if (hipMemset(base, 0, total) != hipSuccess) {
    (void)hipFree(base);
    delete h;
    set_error("hipMemset of the workspace failed");
    return NGD_ERR_HIP;
  }
  size_t o = 0;
  for (auto& p : plan) {
    *p.first = static_cast<char*>(base) + o;
    o += align_up(p.second, 256);
  }
  h->base = base;
  h->bytes = total;
  if (hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming) != hipSuccess) {
    if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
    if (h->side) (void)hipStreamDestroy(h->side);
    (void)hipFree(h->base);
    delete h;
    set_error("hipStreamCreate / hipEventCreate failed");
    return NGD_ERR_HIP;
  }
  if (hipHostMalloc(&h->host, 4096, hipHostMallocDefault) != hipSuccess) {
    (void)hipEventDestroy(h->ev_join);
    (void)hipEventDestroy(h->ev_fork);
    (void)hipStreamDestroy(h->side);
    (void)hipFree(base);
    delete h;
    set_error("hipHostMalloc failed");
    return NGD_ERR_OOM;
  }
  *out = h;
  return NGD_OK;
}

ngd_status ngd_problem_destroy(ngd_problem* h) {
  if (h == nullptr) return NGD_OK;
  (void)flush_timers(h);
  for (hipEvent_t e : h->ev_free) (void)hipEventDestroy(e);
  if (h->side) {
    (void)hipStreamSynchronize(h->side);
    (void)hipStreamDestroy(h->side);
  }
  if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
  if (h->ev_join) (void)hipEventDestroy(h->ev_join);
  if (h->Jc) (void)hipFree(h->Jc);
  if (h->rp_blob) (void)hipFree(h->rp_blob);
  if (h->rp_F) (void)hipFree(h->rp_F);
  if (h->dr_blob) (void)hipFree(h->dr_blob);
  (void)hipFree(h->base);
  (void)hipHostFree(h->host);
  delete h;
  return NGD_OK;
}

int64_t ngd_num_params(const ngd_problem* h) { return h ? h->P : -1; }
int64_t ngd_recommended_ld(const ngd_problem* h) { return h ? h->ldP : -1; }
int64_t ngd_workspace_bytes(const ngd_problem* h) { return h ? (int64_t)h->bytes : -1; }

ngd_status ngd_residual_jacobian(ngd_problem* h, const void* theta, void* r_w, void* J_w, int64_t ldJ, double* grad,
                                 double* loss, void* stream) {
  NGD_CHECK(h != nullptr && theta != nullptr && r_w != nullptr, "NULL argument");

  if (J_w != nullptr) NGD_CHECK(ldJ >= h->P, "ldJ < P");
  NGD_CHECK(!h->ns || J_w != nullptr || grad == nullptr,
            "the gradient of Navier-Stokes rows needs J_w (no recompute mode)");
  hipStream_t s = S(stream);
  // residual workgroups of this launch (fewer without the Jacobian), each with one loss partial
  const int nb = h->ns ? ns_blocks(h->N) : residual_blocks(h->net, h->dtype, h->N, J_w != nullptr);
  NGD_CHECK(nb <= h->res_blocks, "residual launch exceeds its loss-partial buffer");
  NGD_TRY(timed(h, J_w ? NGD_TIMER_RESIDUAL_JACOBIAN : -1, s, [&] {
    if (h->ns)
      return launch_ns_residual(h->nsd, h->dtype, theta, 0, 1, h->N, h->X, h->w, h->f, h->g, h->kind, r_w, J_w, ldJ,
                                h->loss_part, s);
    return launch_residual_jacobian(h->net, h->dtype, theta, h->N, h->X, h->w, h->f, h->g, h->kind, r_w, J_w, ldJ,
                                    h->loss_part, 0, 1, s, nullptr);
  }));
  if (loss != nullptr) NGD_TRY(launch_reduce_sum(h->loss_part, nb, 1, 0.5, loss, s));
  if (grad != nullptr && J_w != nullptr) {
    // one pass over J_w when its rows suit the one-pass kernel, else the column-sum kernel
    const ngd_operator gop{theta, J_w, ldJ};
    if (ldJ <= h->ldP && ldJ % (h->dtype == NGD_F64 ? 2 : 4) == 0 && aligned16(J_w) &&
        gram_rows_supported(h->dtype, ldJ) && check_op(h, &gop) == NGD_OK) {
      NGD_TRY(launch_grad_rows(h->dtype, J_w, ldJ, h->N, r_w, h->partial, h->nwg, s));
      NGD_TRY(launch_gram_reduce(h->dtype, h->partial, h->nwg, ldJ, h->P, nullptr, 0.0, grad, s));
    } else {
      NGD_TRY(launch_gradient(h->dtype, J_w, ldJ, h->N, h->P, r_w, h->grad_work, grad, s));
    }
  }
  if (grad != nullptr && J_w == nullptr) {
    // recompute mode: grad = J_w^T r_w by the adjoint kernel
    NGD_TRY(launch_cast(h->dtype, r_w, NGD_F64, h->nvec[1], h->N, s));
    NGD_TRY(launch_vjp(h->net, h->dtype, theta, h->N, h->X, h->w, h->f, h->g, h->kind, h->nvec[1], 1, h->partial,
                       h->ldP, h->tsq, h->nwg_vjp, s));
    NGD_TRY(launch_gram_reduce(h->dtype, h->partial, h->nwg_vjp, h->ldP, h->P, nullptr, 0.0, grad, s));
  }
  return NGD_OK;
}

ngd_status ngd_gramian_matvec(ngd_problem* h, const ngd_operator* op, const void* V, int64_t ldV, int64_t k,
                              double lambda, void* Y, int64_t ldY, void* stream) {
  NGD_CHECK(h != nullptr && V != nullptr && Y != nullptr, "NULL argument");
  NGD_TRY(check_op(h, op));
  NGD_CHECK(k >= 1, "k must be >= 1");
  NGD_CHECK(k == 1 || (ldV >= h->P && ldY >= h->P), "ldV, ldY must be >= P");
  NGD_CHECK(lambda >= 0.0, "lambda must be >= 0");
  NGD_CHECK(V != Y, "Y must not alias V");
  hipStream_t s = S(stream);
  const int64_t P = h->P;
  if (k == 1 || op->J == nullptr) {  // one vector at a time (the recompute mode always)
    for (int64_t j = 0; j < k; ++j) {
      const char* Vj = static_cast<const char*>(V) + (size_t)j * ldV * h->elem;
      char* Yj = static_cast<char*>(Y) + (size_t)j * ldY * h->elem;
      NGD_TRY(launch_cast(h->dtype, Vj, NGD_F64, h->vtmp[0], P, s));
      NGD_TRY(gram_apply(h, op, h->vtmp[0], lambda, h->vtmp[1], s));
      NGD_TRY(launch_cast(NGD_F64, h->vtmp[1], h->dtype, Yj, P, s));
    }
    return NGD_OK;
  }
  // block product through the sketch buffers, max_ell columns at a time
  const int gt = h->dtype == NGD_F64 ? G_F64 : G_F32;
  for (int64_t c0 = 0; c0 < k; c0 += h->max_ell) {
    const int64_t kc = std::min<int64_t>(h->max_ell, k - c0);
    const char* Vc = static_cast<const char*>(V) + (size_t)c0 * ldV * h->elem;
    char* Yc = static_cast<char*>(Y) + (size_t)c0 * ldY * h->elem;
    GemmArgs z{h->N, kc, P, op->J, op->ldJ, true, Vc, ldV, true, h->Z, kc, h->dtype, h->dtype, h->dtype, gt, 1.0, 0.0};
    NGD_TRY(launch_gemm(z, s));
    GemmArgs y{kc, P, h->N, h->Z, kc, false, op->J, op->ldJ, false, Yc, ldY, h->dtype, h->dtype, h->dtype, gt, 1.0, 0.0};
    NGD_TRY(launch_gemm(y, s));
    if (lambda != 0.0) NGD_TRY(launch_add_scaled(h->dtype, Vc, ldV, lambda, Yc, ldY, kc, P, s));
  }
  return NGD_OK;
}

ngd_status ngd_jvp(ngd_problem* h, const void* theta, const void* V, int64_t ldV, int64_t k, void* Y, int64_t ldY,
                   void* stream) {
  NGD_CHECK(h != nullptr && theta != nullptr && V != nullptr && Y != nullptr, "NULL argument");
  NGD_CHECK(!h->ns, "ngd_jvp is not available for Navier-Stokes rows");
  NGD_CHECK(k >= 1, "k must be >= 1");
  NGD_CHECK(k == 1 || (ldV >= h->P && ldY >= h->N), "ldV >= P and ldY >= N required");
  return launch_jvp(h->net, h->dtype, theta, V, ldV, k, h->N, h->X, h->w, h->kind, h->dtype, Y, 1, ldY, S(stream));
}

ngd_status ngd_vjp(ngd_problem* h, const void* theta, const void* wv, double* out, void* stream) {
  NGD_CHECK(h != nullptr && theta != nullptr && wv != nullptr && out != nullptr, "NULL argument");
  NGD_CHECK(!h->ns, "ngd_vjp is not available for Navier-Stokes rows");
  hipStream_t s = S(stream);
  NGD_TRY(launch_cast(h->dtype, wv, NGD_F64, h->nvec[1], h->N, s));
  NGD_TRY(launch_vjp(h->net, h->dtype, theta, h->N, h->X, h->w, h->f, h->g, h->kind, h->nvec[1], 1, h->partial,
                     h->ldP, h->tsq, h->nwg_vjp, s));
  return launch_gram_reduce(h->dtype, h->partial, h->nwg_vjp, h->ldP, h->P, nullptr, 0.0, out, s);
}

ngd_status ngd_gaussian_omega(ngd_problem* h, uint64_t seed, uint64_t counter, int64_t ell, void* omega, int64_t ld,
                              void* stream) {
  NGD_CHECK(h != nullptr && omega != nullptr, "NULL argument");
  NGD_CHECK(ell >= 1 && ld >= h->P, "ell >= 1 and ld >= P required");
  return launch_gaussian_omega(h->dtype, seed, counter, h->P, ell, omega, ld, S(stream));
}

namespace {

// Recompute mode: rows [r0, r0 + rows) of J_w at theta into the handle's row-block buffer (allocated on
// first use, at most 128 MB), by the residual/Jacobian kernel on that slice of the points.
ngd_status jc_ensure(ngd_problem* h) {
  if (h->Jc != nullptr) return NGD_OK;
  const int64_t row_bytes = h->ldP * (int64_t)h->elem;
  int64_t rows = std::max<int64_t>(64, (int64_t)(128ll << 20) / row_bytes);
  rows = std::min<int64_t>(rows, h->N);
  if (hipMalloc(&h->Jc, (size_t)rows * row_bytes) != hipSuccess) {
    h->Jc = nullptr;
    set_error("hipMalloc of the recompute-mode row block failed");
    return NGD_ERR_OOM;
  }
  h->jc_rows = rows;
  return NGD_OK;
}

ngd_status jc_rows_at(ngd_problem* h, const void* theta, int64_t r0, int64_t rows, hipStream_t s) {
  const size_t e = h->elem;
  const char* X = static_cast<const char*>(h->X) + (size_t)r0 * h->net.d * e;
  const char* w = static_cast<const char*>(h->w) + (size_t)r0 * e;
  const char* f = static_cast<const char*>(h->f) + (size_t)r0 * e;
  const char* g = static_cast<const char*>(h->g) + (size_t)r0 * e;
  return launch_residual_jacobian(h->net, h->dtype, theta, rows, X, w, f, g, h->kind + r0, nullptr, h->Jc, h->ldP,
                                  h->loss_part, 0, 1, s, nullptr);
}

}  // namespace

// The sketch with a Gaussian test matrix (omega, or generated from seed/counter), or, when `cols` is
// given, with Omega = the identity's columns at those indices, so that Z = J_w Omega is a gather of
// J_w's columns.
ngd_status sketch_impl(ngd_problem* h, const ngd_operator* op, int64_t ell, uint64_t seed, uint64_t counter,
                       const void* omega, int64_t ldO, const int64_t* cols, int32_t sketch_dtype, void* U, int64_t ldU,
                       double* lam_hat, ngd_nystrom_info* info, void* stream, bool defer_eig = false);

ngd_status ngd_nystrom_sketch(ngd_problem* h, const ngd_operator* op, int64_t ell, uint64_t seed, uint64_t counter,
                              const void* omega, int64_t ldO, int32_t sketch_dtype, void* U, int64_t ldU,
                              double* lam_hat, ngd_nystrom_info* info, void* stream) {
  return sketch_impl(h, op, ell, seed, counter, omega, ldO, nullptr, sketch_dtype, U, ldU, lam_hat, info, stream);
}

ngd_status ngd_nystrom_sketch_columns(ngd_problem* h, const ngd_operator* op, int64_t ell, const int64_t* cols,
                                      int32_t sketch_dtype, void* U, int64_t ldU, double* lam_hat,
                                      ngd_nystrom_info* info, void* stream) {
  NGD_CHECK(cols != nullptr, "NULL argument");
  return sketch_impl(h, op, ell, 0, 0, nullptr, 0, cols, sketch_dtype, U, ldU, lam_hat, info, stream);
}

ngd_status ngd_gramian_diagonal(ngd_problem* h, const ngd_operator* op, double* diag, void* stream) {
  NGD_CHECK(h != nullptr && diag != nullptr, "NULL argument");
  NGD_TRY(check_op(h, op));
  hipStream_t s = S(stream);
  const int64_t dw = kDiagChunks * h->ldP;
  if (op->J != nullptr) return launch_colsq(h->dtype, op->J, op->ldJ, h->N, h->P, h->diag_work, dw, 0, diag, s);
  // recompute mode: the rows of J_w a block at a time, each block's squares added in
  NGD_TRY(jc_ensure(h));
  if (h->N == 0) return launch_colsq(h->dtype, nullptr, h->ldP, 0, h->P, h->diag_work, dw, 0, diag, s);
  for (int64_t r0 = 0; r0 < h->N; r0 += h->jc_rows) {
    const int64_t rows = std::min<int64_t>(h->jc_rows, h->N - r0);
    NGD_TRY(jc_rows_at(h, op->theta, r0, rows, s));
    NGD_TRY(launch_colsq(h->dtype, h->Jc, h->ldP, rows, h->P, h->diag_work, dw, r0 > 0 ? 1 : 0, diag, s));
  }
  return NGD_OK;
}

namespace {

// Eigenpairs of B^T B below this fraction of the largest (by the Gershgorin bound of its tridiagonal
// form) come out of the first eigendecomposition as zeros: their vectors carry errors of order
// eps sigma_1 / sigma there.
constexpr double kDropRel = 1e-11;
// FP64 problems resolve every pair below kSplitRel lam_1 a second time, from B projected off the
// pairs above: the projected Gram matrix holds only the small part of the spectrum, so its
// eigendecomposition is accurate relative to that part instead of to lam_1 (forming B^T B squares
// sigma; the projection keeps the small singular values accurate to about eps sigma_1 / sigma).
// Pairs of the second level below kNoiseRel lam_1 are rounding noise of the projection and are
// returned as zeros.
constexpr double kSplitRel = 1e-8;
constexpr double kNoiseRel = 1e-18;

// The thin SVD of B (P x L, given as Bt = B^T, L rows of the working type, ld = ldP; overwritten in
// the FP64 case) through the eigenpairs of B^T B (Alg. 6, svd(B)): lam_hat = sigma^2 descending and
// U = B V Sigma^{-1} as rows. Uses the handle's core buffers M, Ev, F, evals, the eigensolver's
// workspace, vtmp[2] and (FP64) the Omega buffer.
// the Gram matrix B^T B of the core in h->M (FP64)
ngd_status core_gram(ngd_problem* h, void* Bt, int64_t L, hipStream_t s) {
  GemmArgs g5{L, L, h->P, Bt, h->ldP, true, Bt, h->ldP, true, h->M, L, h->dtype, h->dtype, NGD_F64, G_F64, 1.0, 0.0,
              h->gemm_work, h->gemm_work_elems, 1};
  return launch_gemm(g5, s);
}

// non-FP64 problems, once h->M has gone through the eigensolver's batched stages: the rest of it,
// then U^T = (V Sigma^{-1})^T B^T
ngd_status core_svd_finish(ngd_problem* h, void* Bt, int64_t L, void* U, int64_t ldU, double* lam_hat, hipStream_t s) {
  NGD_TRY(launch_sym_eig_rest((int)L, kDropRel, lam_hat, h->Ev, h->eigw, s, h->side, h->ev_join));
  NGD_TRY(launch_whitening(lam_hat, h->Ev, (int)L, h->F, s));
  GemmArgs g6{L, h->P, L, h->F, L, false, Bt, h->ldP, false, U, ldU, NGD_F64, h->dtype, h->dtype, G_F64, 1.0, 0.0};
  return launch_gemm(g6, s);
}

ngd_status core_svd(ngd_problem* h, void* Bt, int64_t L, void* U, int64_t ldU, double* lam_hat, hipStream_t s) {
  const int64_t P = h->P, ldP = h->ldP;
  const int T = h->dtype;
  NGD_TRY(core_gram(h, Bt, L, s));
  NGD_TRY(launch_sym_eig(h->M, (int)L, kDropRel, lam_hat, h->Ev, h->eigw, s, h->side, h->ev_fork, h->ev_join));
  if (T != NGD_F64) {
    NGD_TRY(launch_whitening(lam_hat, h->Ev, (int)L, h->F, s));
    GemmArgs g6{L, P, L, h->F, L, false, Bt, ldP, false, U, ldU, NGD_F64, T, T, G_F64, 1.0, 0.0};
    return launch_gemm(g6, s);
  }
  double* lam_t = h->vtmp[2];
  double* Evt = h->M;  // free: the eigensolver consumed it
  double* X = static_cast<double*>(h->omega);
  // the resolved pairs (lam >= kSplitRel lam_1) give their rows of U directly
  NGD_TRY(launch_split_top(lam_hat, h->Ev, (int)L, kSplitRel, lam_t, Evt, s));
  NGD_TRY(launch_whitening(lam_t, h->Ev, (int)L, h->F, s));
  GemmArgs g6{L, P, L, h->F, L, false, Bt, ldP, false, U, ldU, NGD_F64, T, T, G_F64, 1.0, 0.0};
  NGD_TRY(launch_gemm(g6, s));
  // B_c^T = (I - V_t V_t^T) B^T: X = V_t^T B^T, then B^T -= V_t X
  GemmArgs gx{L, P, L, Evt, L, true, Bt, ldP, false, X, ldP, NGD_F64, T, NGD_F64, G_F64, 1.0, 0.0};
  NGD_TRY(launch_gemm(gx, s));
  GemmArgs gp{L, P, L, Evt, L, false, X, ldP, false, Bt, ldP, NGD_F64, NGD_F64, T, G_F64, -1.0, 1.0};
  NGD_TRY(launch_gemm(gp, s));
  // the small pairs from the eigendecomposition of B_c^T B_c, and their rows of U = B_c y / sqrt(mu)
  GemmArgs g7{L, L, P, Bt, ldP, true, Bt, ldP, true, h->M, L, T, T, NGD_F64, G_F64, 1.0, 0.0,
              h->gemm_work, h->gemm_work_elems, 1};
  NGD_TRY(launch_gemm(g7, s));
  NGD_TRY(launch_sym_eig(h->M, (int)L, kDropRel, h->evals, h->Ev, h->eigw, s, h->side, h->ev_fork, h->ev_join,
                         true));
  NGD_TRY(launch_whitening(h->evals, h->Ev, (int)L, h->F, s));
  GemmArgs g8{L, P, L, h->F, L, false, Bt, ldP, false, X, ldP, NGD_F64, T, NGD_F64, G_F64, 1.0, 0.0};
  NGD_TRY(launch_gemm(g8, s));
  return launch_merge_small(T, lam_t, h->evals, X, ldP, (int)L, P, kNoiseRel, U, ldU, lam_hat, s);
}

}  // namespace

ngd_status rp_ensure(ngd_problem* h);

namespace {

ngd_status dr_ensure(ngd_problem* h) {
  if (h->dr_blob != nullptr) return NGD_OK;
  const size_t P = (size_t)h->P, ldP = (size_t)h->ldP;
  std::vector<std::pair<void**, size_t>> plan = {{(void**)&h->dr_G, 8 * P * ldP},
                                                 {(void**)&h->dr_Linv, direct_panel_inverse_bytes(h->P)},
                                                 {(void**)&h->dr_stage, direct_stage_bytes(h->P)},
                                                 {(void**)&h->dr_part, direct_part_bytes(h->P)},
                                                 {(void**)&h->dr_y, 8 * ldP},
                                                 {(void**)&h->dr_info, 256}};
  size_t total = 0;
  for (auto& e : plan) total += align_up(e.second, 256);
  if (hipMalloc(&h->dr_blob, total) != hipSuccess) {
    (void)hipGetLastError();
    h->dr_blob = nullptr;
    set_error("hipMalloc of the full-Gramian workspace failed (" + std::to_string(total) + " bytes)");
    return NGD_ERR_OOM;
  }
  char* q = static_cast<char*>(h->dr_blob);
  for (auto& e : plan) {
    *e.first = q;
    q += align_up(e.second, 256);
  }
  return NGD_OK;
}

}  // namespace

// NGD full (Alg. 2): G = J_w^T J_w (FP64, lower tiles), G + lambda I = L L^T, d = L^{-T} L^{-1} g.
ngd_status ngd_direct_solve(ngd_problem* h, const ngd_operator* op, const double* g, double lambda, double* d,
                            void* stream) {
  NGD_CHECK(h != nullptr && g != nullptr && d != nullptr, "NULL argument");
  NGD_TRY(check_op(h, op));
  NGD_CHECK(lambda > 0.0 && std::isfinite(lambda), "lambda must be > 0");
  NGD_TRY(dr_ensure(h));
  hipStream_t s = S(stream);
  const int64_t P = h->P, N = h->N, ldG = h->ldP;
  const int T = h->dtype;
  if (op->J != nullptr) {
    GemmArgs gg{P, P, N, op->J, op->ldJ, false, op->J, op->ldJ, false, h->dr_G, ldG, T, T, NGD_F64, G_F64, 1.0, 0.0,
                nullptr, 0, 2};
    NGD_TRY(launch_gemm(gg, s));
  } else {  // recompute mode: the Gramian summed over row blocks of J_w formed from theta
    NGD_TRY(jc_ensure(h));
    for (int64_t r0 = 0; r0 < N; r0 += h->jc_rows) {
      const int64_t rows = std::min<int64_t>(h->jc_rows, N - r0);
      NGD_TRY(jc_rows_at(h, op->theta, r0, rows, s));
      GemmArgs gg{P, P, rows, h->Jc, h->ldP, false, h->Jc, h->ldP, false, h->dr_G, ldG, T, T, NGD_F64, G_F64, 1.0,
                  r0 == 0 ? 0.0 : 1.0, nullptr, 0, 2};
      NGD_TRY(launch_gemm(gg, s));
    }
  }
  NGD_TRY(launch_add_diag(h->dr_G, ldG, P, lambda, s));
  NGD_TRY(launch_blocked_cholesky(h->dr_G, ldG, P, h->dr_Linv, h->dr_stage, h->dr_info, s));
  NGD_TRY(launch_cholesky_solve(h->dr_G, ldG, P, h->dr_Linv, g, h->dr_y, h->dr_part, d, s));
  int* hv = reinterpret_cast<int*>(h->host);
  NGD_HIP_TRY(hipMemcpyAsync(hv, h->dr_info, sizeof(int), hipMemcpyDeviceToHost, s));
  NGD_HIP_TRY(hipStreamSynchronize(s));
  if (hv[0] != 0) {
    set_error("Cholesky factorisation of G + lambda I met a non-positive pivot at index " + std::to_string(hv[0] - 1));
    return NGD_ERR_NOT_PD;
  }
  return NGD_OK;
}

ngd_status ngd_rpcholesky(ngd_problem* h, const ngd_operator* op, const double* diag, int64_t ell_max, int32_t block,
                          uint64_t seed, uint64_t counter, double eps, double* Ft, int64_t ldF, int64_t* rank,
                          double* trace, void* stream) {
  NGD_CHECK(h != nullptr && op != nullptr && diag != nullptr && Ft != nullptr && rank != nullptr, "NULL argument");
  NGD_TRY(check_op(h, op));
  NGD_CHECK(block >= 1 && block <= kRpBlockMax, "block must be in [1, 64]");
  NGD_CHECK(ell_max >= 1 && ell_max <= std::min<int64_t>(kMaxEll, h->P), "ell_max must be in [1, min(1024, P)]");
  NGD_CHECK(ldF >= h->P, "ldF < P");
  NGD_CHECK(eps >= 0.0, "eps must be >= 0");
  NGD_TRY(rp_ensure(h));
  const bool rec = op->J == nullptr;  // recompute mode: J_w's rows a block at a time, every round
  if (rec) NGD_TRY(jc_ensure(h));
  hipStream_t s = S(stream);
  const int64_t P = h->P, N = h->N;
  const int T = h->dtype;
  const int b = block;
  NGD_HIP_TRY(hipMemcpyAsync(h->rp_d, diag, sizeof(double) * P, hipMemcpyDeviceToDevice, s));
  NGD_TRY(launch_zero(Ft, sizeof(double) * (size_t)ell_max * ldF, s));
  NGD_TRY(launch_zero(h->rp_st, sizeof(int64_t) * 4, s));
  const int64_t rounds = (ell_max + b - 1) / b;
  for (int64_t i = 0; i < rounds; ++i) {
    // S' = Unique(b draws ~ d); C^T = (G[:, S'] - F F[S', :]^T)^T = J[:, S']^T J - F[S', :] F^T
    NGD_TRY(launch_sample_pivots(h->rp_d, P, seed, counter, (uint32_t)i, b, 1, h->rp_idx, h->rp_cnt, s, h->rp_st + 1));
    if (!rec) {
      NGD_TRY(launch_gather_cols(T, op->J, op->ldJ, N, h->rp_idx, b, h->rp_Jcols, b, s));
      // (a b x P output over K = N: split K through the core's GEMM workspace, idle here)
      GemmArgs g1{b, P, N, h->rp_Jcols, b, false, op->J, op->ldJ, false, h->rp_Ct, h->ldP, T, T, NGD_F64, G_F64, 1.0,
                  0.0, h->gemm_work, h->gemm_work_elems};
      NGD_TRY(launch_gemm(g1, s));
    } else {
      // C^T summed over row blocks of J_w recomputed from theta
      for (int64_t r0 = 0; r0 < N; r0 += h->jc_rows) {
        const int64_t rows = std::min<int64_t>(h->jc_rows, N - r0);
        NGD_TRY(jc_rows_at(h, op->theta, r0, rows, s));
        NGD_TRY(launch_gather_cols(T, h->Jc, h->ldP, rows, h->rp_idx, b, h->rp_Jcols, b, s));
        GemmArgs g1{b, P, rows, h->rp_Jcols, b, false, h->Jc, h->ldP, false, h->rp_Ct, h->ldP, T, T, NGD_F64, G_F64,
                    1.0, r0 == 0 ? 0.0 : 1.0, h->gemm_work, h->gemm_work_elems};
        NGD_TRY(launch_gemm(g1, s));
      }
    }
    const int64_t kmax = std::min<int64_t>(i * b, ell_max);
    if (kmax > 0) {
      NGD_TRY(launch_rp_gather_f(Ft, ldF, h->rp_idx, b, kmax, h->rp_W, kmax, s));
      GemmArgs g2{b, P, kmax, h->rp_W, kmax, true, Ft, ldF, false, h->rp_Ct, h->ldP, NGD_F64, NGD_F64, NGD_F64, G_F64,
                  -1.0, 1.0};
      NGD_TRY(launch_gemm(g2, s));
    }
    // R = chol(C[S', S']), F[:, r : r + kept] = C R^{-1}, d -= squared row norms; stop on trace < eps
    NGD_TRY(launch_rp_block(h->rp_Ct, h->ldP, h->rp_idx, h->rp_cnt, h->rp_st, ell_max, h->rp_Rt, h->rp_keep, P, Ft,
                            ldF, h->rp_d, h->rp_part, eps, b, h->rp_trace, s));
    // rounds after the stop draw nothing and add nothing, but their products with J_w still run: look
    // at the flag every fourth round, so that at most three such rounds are enqueued
    if (i % 4 == 3 && i + 1 < rounds) {
      int64_t* hd = reinterpret_cast<int64_t*>(h->host);
      NGD_HIP_TRY(hipMemcpyAsync(hd, h->rp_st + 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
      NGD_HIP_TRY(hipStreamSynchronize(s));
      if (hd[0] != 0) break;
    }
  }
  double* hv = reinterpret_cast<double*>(h->host);
  NGD_HIP_TRY(hipMemcpyAsync(hv, h->rp_st, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  NGD_HIP_TRY(hipMemcpyAsync(hv + 1, h->rp_trace, sizeof(double), hipMemcpyDeviceToHost, s));
  NGD_HIP_TRY(hipStreamSynchronize(s));
  int64_t r = 0;
  std::memcpy(&r, hv, sizeof(r));
  *rank = r;
  if (trace != nullptr) *trace = hv[1];
  return NGD_OK;
}

ngd_status ngd_rpchol_precond(ngd_problem* h, const double* Ft, int64_t ldF, int64_t rank, void* U, int64_t ldU,
                              double* lam_hat, void* stream) {
  NGD_CHECK(h != nullptr && Ft != nullptr && U != nullptr && lam_hat != nullptr, "NULL argument");
  NGD_CHECK(rank >= 0 && rank + 1 <= h->max_ell, "rank + 1 must be <= max_ell");
  NGD_CHECK(ldF >= h->P && ldU >= h->P, "ldF and ldU must be >= P");
  hipStream_t s = S(stream);
  const int64_t P = h->P, L = rank;
  const int T = h->dtype;
  NGD_TRY(launch_zero(static_cast<char*>(U) + (size_t)L * ldU * h->elem, (size_t)ldU * h->elem, s));
  NGD_TRY(launch_zero(lam_hat + L, sizeof(double), s));
  if (L == 0) return NGD_OK;
  // the thin SVD of F through the eigenpairs of F^T F (FP64): U = F V Sigma^{-1}, lam = sigma^2
  NGD_TRY(launch_cast_rows(NGD_F64, Ft, ldF, L, P, T, h->Bt, h->ldP, s));
  NGD_TRY(core_svd(h, h->Bt, L, U, ldU, lam_hat, s));
  int* hv = reinterpret_cast<int*>(h->host);
  NGD_HIP_TRY(hipMemcpyAsync(hv, eig_error_flag(h->eigw, (int)L), sizeof(int), hipMemcpyDeviceToHost, s));
  NGD_HIP_TRY(hipStreamSynchronize(s));
  if (hv[0] != 0) {
    set_error("exchange between the workgroups of the tridiagonalisation timed out");
    return NGD_ERR_HIP;
  }
  return NGD_OK;
}

ngd_status ngd_rpchol_precond_woodbury(ngd_problem* h, const double* Ft, int64_t ldF, int64_t rank, double mu,
                                       void* U, int64_t ldU, double* lam_hat, void* stream) {
  NGD_CHECK(h != nullptr && Ft != nullptr && U != nullptr && lam_hat != nullptr, "NULL argument");
  NGD_CHECK(rank >= 0 && rank + 1 <= h->max_ell, "rank + 1 must be <= max_ell");
  NGD_CHECK(ldF >= h->P && ldU >= h->P, "ldF and ldU must be >= P");
  NGD_CHECK(std::isfinite(mu) && mu > 0.0, "mu must be finite and > 0");
  hipStream_t s = S(stream);
  const int64_t P = h->P, L = rank;
  NGD_TRY(launch_zero(static_cast<char*>(U) + (size_t)L * ldU * h->elem, (size_t)ldU * h->elem, s));
  NGD_TRY(launch_woodbury_lam(lam_hat, (int)L, s));
  if (L == 0) return NGD_OK;
  if (h->rp_F == nullptr) {
    if (hipMalloc((void**)&h->rp_F, sizeof(double) * (size_t)P * h->max_ell) != hipSuccess) {
      (void)hipGetLastError();
      h->rp_F = nullptr;
      set_error("hipMalloc of the Woodbury factor's buffer failed");
      return NGD_ERR_OOM;
    }
  }
  // R^T R = F^T F + mu I (FP64 Gram product, the Cholesky factor L = R^T of the core), then
  // W^T = (F L^{-T})^T row by row into U in the working precision
  GemmArgs g{L, L, P, Ft, ldF, true, Ft, ldF, true, h->M, L, NGD_F64, NGD_F64, NGD_F64, G_F64, 1.0, 0.0,
             h->gemm_work, h->gemm_work_elems, 1};
  NGD_TRY(launch_gemm(g, s));
  NGD_TRY(launch_add_diag(h->M, L, L, mu, s));
  // no extra shift; a pivot that rounding left non-positive is floored at 1e-18 tr(M) (far below mu)
  NGD_TRY(launch_shifted_cholesky(h->M, (int)L, 0.0, 1e-18, h->scal + 200, reinterpret_cast<int*>(h->scal + 210),
                                  h->cholsync, ++h->chol_epoch, s));
  NGD_TRY(launch_transpose_cast(NGD_F64, Ft, ldF, L, P, NGD_F64, h->rp_F, L, s));
  NGD_TRY(launch_trsm_q(h->M, (int)L, NGD_F64, h->rp_F, P, nullptr, h->dtype, U, ldU, s));
  int* hv = reinterpret_cast<int*>(h->host);
  NGD_HIP_TRY(hipMemcpyAsync(hv, h->cholsync + 128, sizeof(int), hipMemcpyDeviceToHost, s));
  NGD_HIP_TRY(hipStreamSynchronize(s));
  if (hv[0] != 0) {
    set_error("exchange between the workgroups of the Cholesky factorisation timed out");
    return NGD_ERR_HIP;
  }
  return NGD_OK;
}

ngd_status ngd_sample_pivots(ngd_problem* h, const double* weights, int64_t n_samples, uint64_t seed, uint64_t counter,
                             uint32_t substream, int32_t unique, int64_t* idx, int32_t* count, void* stream) {
  NGD_CHECK(h != nullptr && weights != nullptr && idx != nullptr && count != nullptr, "NULL argument");
  NGD_CHECK(n_samples >= 0 && n_samples <= kMaxSamples, "n_samples must be in [0, 4096]");
  NGD_CHECK(substream < 0x80000000u, "substream must be below 2^31");
  return launch_sample_pivots(weights, h->P, seed, counter, substream, n_samples, unique ? 1 : 0, idx, count,
                              S(stream));
}

// ---- block RPCholesky (Section 4.2.2; block algorithm of the appendix) and its preconditioner ----
ngd_status rp_ensure(ngd_problem* h) {
  if (h->rp_blob != nullptr) return NGD_OK;
  const size_t P = (size_t)h->P, ldP = (size_t)h->ldP, N = (size_t)h->N;
  const size_t nb = (P + 255) / 256;
  std::vector<std::pair<void**, size_t>> plan = {
      {(void**)&h->rp_d, 8 * P},
      {(void**)&h->rp_Ct, 8 * kRpBlockMax * ldP},
      {(void**)&h->rp_W, 8 * (size_t)kRpBlockMax * kMaxEll},
      {(void**)&h->rp_Rt, 8 * (size_t)kRpBlockMax * kRpBlockMax},
      {(void**)&h->rp_part, 8 * nb},
      {(void**)&h->rp_trace, 8},
      {(void**)&h->rp_idx, 8 * (size_t)kRpBlockMax},
      {(void**)&h->rp_st, 8 * 4},
      {(void**)&h->rp_cnt, 4 * 4},
      {(void**)&h->rp_keep, 4 * (size_t)kRpBlockMax},
      {&h->rp_Jcols, (size_t)h->elem * N * kRpBlockMax}};
  size_t total = 0;
  for (auto& e : plan) total += align_up(e.second, 256);
  if (hipMalloc(&h->rp_blob, total) != hipSuccess) {
    h->rp_blob = nullptr;
    set_error("hipMalloc of the RPCholesky workspace failed");
    return NGD_ERR_OOM;
  }
  char* q = static_cast<char*>(h->rp_blob);
  for (auto& e : plan) {
    *e.first = q;
    q += align_up(e.second, 256);
  }
  return NGD_OK;
}

ngd_status sketch_impl(ngd_problem* h, const ngd_operator* op, int64_t ell, uint64_t seed, uint64_t counter,
                       const void* omega, int64_t ldO, const int64_t* cols, int32_t sketch_dtype, void* U, int64_t ldU,
                       double* lam_hat, ngd_nystrom_info* info, void* stream, bool defer_eig) {
  NGD_CHECK(h != nullptr && U != nullptr && lam_hat != nullptr, "NULL argument");
  NGD_TRY(check_op(h, op));
  NGD_CHECK(ell >= 1 && ell <= h->max_ell, "ell must be in [1, min(max_ell, P)]");
  NGD_CHECK(ldU >= h->P, "ldU < P");
  NGD_CHECK(omega == nullptr || ldO >= h->P, "ldO < P");
  int gt;
  if (h->dtype == NGD_F64) {
    NGD_CHECK(sketch_dtype == NGD_F64, "an FP64 problem sketches in FP64");
    gt = G_F64;
  } else {
    NGD_CHECK(sketch_dtype == NGD_F32 || sketch_dtype == NGD_BF16, "an FP32 problem sketches in FP32 or BF16");
    gt = sketch_dtype == NGD_F32 ? G_F32 : G_BF16;
  }
  hipStream_t s = S(stream);
  const int64_t N = h->N, P = h->P, L = ell;
  const int T = h->dtype;
  if (omega == nullptr && cols == nullptr) {
    NGD_TRY(launch_gaussian_omega(T, seed, counter, P, L, h->omega, h->ldP, s));
    omega = h->omega;
    ldO = h->ldP;
  }
  if (cols != nullptr) ldO = h->ldP;  // (no Omega is read; keeps the NT-path checks below well defined)
  // recompute mode: J_w is never stored whole. Each product is formed a block of rows at a time: the
  // residual/Jacobian kernel recomputes the block into a scratch buffer and the block's share of
  // Z = J_w Omega (its rows) or of B^T = Q^T J_w (a rank-`rows` update) follows with the same GEMM
  // kernels as the stored path. Every row of J_w is formed twice per sketch instead of swept ell times
  // by the tangent and adjoint kernels.
  const bool rec = op->J == nullptr;
  if (rec) NGD_TRY(jc_ensure(h));
  const bool nt_rec = rec && T == NGD_F32 && nt_gemm_supported(NGD_F32, NGD_F32, gt, h->jc_rows, L, P, h->ldP, ldO);
  // the NT kernel (large tiles, both operands K-contiguous) serves the FP32 / BF16 sketch
  const int et = gt == G_BF16 ? NGD_BF16 : NGD_F32;
  // The second product reads J in place as a K-major operand in FP32; in BF16 it reads a transposed
  // BF16 copy of J instead (made on the side stream beside the core): with the FP32 operand the BF16
  // product is held to the rate at which its tiles' FP32 rows reach the CUs, and it ran slower than
  // the copy and the product together.
  const bool w_kmajor = et == NGD_F32;
  const bool nt = !rec && T == NGD_F32 && nt_gemm_supported(NGD_F32, NGD_F32, gt, N, L, P, op->ldJ, ldO) &&
                  (w_kmajor ? nt_gemm_supported(NGD_F32, et, gt, P, L, N, op->ldJ, h->ldN, true)
                            : nt_gemm_supported(et, et, gt, P, L, N, h->ldN, h->ldN));
  // Omega^T in the compute type (BF16: a rounded copy, read at half the bytes). A column test matrix
  // has no Omega to read: its Z is a gather.
  const void* om_nt = omega;
  int64_t ld_nt = ldO;
  int om_type = NGD_F32;
  if ((nt || nt_rec) && gt == G_BF16 && cols == nullptr) {
    NGD_TRY(launch_cast_rows(NGD_F32, omega, ldO, L, P, NGD_BF16, h->Ob, h->ldP, s));
    om_nt = h->Ob;
    ld_nt = h->ldP;
    om_type = NGD_BF16;
  }
  // Z = J Omega (N x ell)
  NGD_TRY(timed(h, NGD_TIMER_SKETCH_Z, s, [&] {
    if (cols != nullptr) {  // Omega = columns of the identity: Z is a gather of J's columns
      if (!rec) return launch_gather_cols(T, op->J, op->ldJ, N, cols, L, h->Z, L, s);
      for (int64_t r0 = 0; r0 < N; r0 += h->jc_rows) {
        const int64_t rows = std::min<int64_t>(h->jc_rows, N - r0);
        NGD_TRY(jc_rows_at(h, op->theta, r0, rows, s));
        void* Zr = static_cast<char*>(h->Z) + (size_t)r0 * L * h->elem;
        NGD_TRY(launch_gather_cols(T, h->Jc, h->ldP, rows, cols, L, Zr, L, s));
      }
      return NGD_OK;
    }
    if (rec) {
      for (int64_t r0 = 0; r0 < N; r0 += h->jc_rows) {
        const int64_t rows = std::min<int64_t>(h->jc_rows, N - r0);
        NGD_TRY(jc_rows_at(h, op->theta, r0, rows, s));
        void* Zr = static_cast<char*>(h->Z) + (size_t)r0 * L * h->elem;
        if (nt_rec) {
          NGD_TRY(launch_nt_gemm(NGD_F32, h->Jc, h->ldP, om_type, om_nt, ld_nt, gt, rows, L, P, NGD_F32, Zr, L, false,
                                 1.0, h->sk_work, h->sk_work_elems, s));
        } else {
          GemmArgs g1{rows, L, P, h->Jc, h->ldP, true, omega, ldO, true, Zr, L, T, T, T, gt, 1.0, 0.0};
          NGD_TRY(launch_gemm(g1, s));
        }
      }
      return NGD_OK;
    }
    if (nt) return launch_nt_gemm(NGD_F32, op->J, op->ldJ, om_type, om_nt, ld_nt, gt, N, L, P, NGD_F32, h->Z, L,
                                  false, 1.0, h->sk_work, h->sk_work_elems, s);
    // split K over the Gram products' workspace where the output has too few tiles (small ell)
    GemmArgs g1{N, L, P, op->J, op->ldJ, true, omega, ldO, true, h->Z, L, T, T, T, gt, 1.0, 0.0,
                h->gemm_work, h->gemm_work_elems, 0};
    return launch_gemm(g1, s);
  }));
  // J^T in BF16 for the second product, on the side stream: it overlaps the latency-bound FP64 core
  // below and is joined before the product that reads it
  const bool w_copy = nt && !w_kmajor;
  if (w_copy) {
    NGD_HIP_TRY(hipEventRecord(h->ev_fork, s));
    NGD_HIP_TRY(hipStreamWaitEvent(h->side, h->ev_fork, 0));
    NGD_TRY(timed(h, NGD_TIMER_SKETCH_PREP, h->side, [&] {
      return launch_transpose_cast(NGD_F32, op->J, op->ldJ, N, P, et, h->Jt, h->ldN, h->side);
    }));
    NGD_HIP_TRY(hipEventRecord(h->ev_join, h->side));
  }
  // M = Z^T Z (FP64), eigenpairs, whitening F = V_M D^{-1/2} (pseudo-inverse of the core), and
  // Q = Z F (orthonormal basis of range(Z)) with FP64 accumulation
  NGD_TRY(timed(h, NGD_TIMER_CORE, s, [&] {
    GemmArgs g2{L, L, N, h->Z, L, false, h->Z, L, false, h->M, L, T, T, NGD_F64, G_F64, 1.0, 0.0,
                h->gemm_work, h->gemm_work_elems, 1};
    NGD_TRY(launch_gemm(g2, s));
    // L L^T = M + nu I with nu = c eps tr(M) (the shift of Alg. 6), then Q = Z L^{-T} in FP64; c = 1
    // for FP64 Jacobians (the shift bounds how small an eigenvalue the core resolves), 10 for FP32
    const double shift_rel = (T == NGD_F64 ? 1.0 : 10.0) * 2.220446049250313e-16;
    NGD_TRY(launch_shifted_cholesky(h->M, (int)L, shift_rel, 1e-15, h->scal + 200,
                                    reinterpret_cast<int*>(h->scal + 210), h->cholsync, ++h->chol_epoch, s));
    // one launch: Q in FP64 where a product reads it, Q^T in the compute type on the NT path
    return launch_trsm_q(h->M, (int)L, T, h->Z, N, nt ? nullptr : (double*)h->Q, et, nt ? h->Qt : nullptr, h->ldN,
                         s);
  }));
  // B^T = Q^T J (ell x P); on the NT path as (J^T Q)^T with Q^T in the compute type and J^T read in
  // place from the stored J (FP32, K-major operand) or from its BF16 copy
  if (w_copy) NGD_HIP_TRY(hipStreamWaitEvent(s, h->ev_join, 0));
  NGD_TRY(timed(h, NGD_TIMER_SKETCH_W, s, [&] {
    if (rec) {
      for (int64_t r0 = 0; r0 < N; r0 += h->jc_rows) {
        const int64_t rows = std::min<int64_t>(h->jc_rows, N - r0);
        NGD_TRY(jc_rows_at(h, op->theta, r0, rows, s));
        GemmArgs g4{L, P, rows, (const double*)h->Q + r0 * L, L, false, h->Jc, h->ldP, false, h->Bt, h->ldP,
                    NGD_F64, T, T, gt, 1.0, r0 == 0 ? 0.0 : 1.0};
        NGD_TRY(launch_gemm(g4, s));
      }
      return NGD_OK;
    }
    if (nt && w_kmajor)
      return launch_nt_gemm(NGD_F32, op->J, op->ldJ, et, h->Qt, h->ldN, gt, P, L, N, NGD_F32, h->Bt, h->ldP, true,
                            1.0, h->sk_work, h->sk_work_elems, s, true);
    if (nt) return launch_nt_gemm(et, h->Jt, h->ldN, et, h->Qt, h->ldN, gt, P, L, N, NGD_F32, h->Bt, h->ldP, true,
                                  1.0, h->sk_work, h->sk_work_elems, s);
    GemmArgs g4{L, P, N, h->Q, L, false, op->J, op->ldJ, false, h->Bt, h->ldP, NGD_F64, T, T, gt, 1.0, 0.0,
                h->gemm_work, h->gemm_work_elems, 0};
    return launch_gemm(g4, s);
  }));
  // A = B^T B (FP64) and its eigenpairs lam_hat = Sigma^2, V; U^T = (V Sigma^{-1})^T B^T (FP64
  // problems: the small pairs a second time, from B projected off the resolved ones)
  // defer_eig (FP32 problems, no summary): stop after the Gram matrix B B^T in h->M; the caller
  // tridiagonalises it with other problems' and completes the core with core_svd_finish
  if (defer_eig && h->dtype != NGD_F64 && info == nullptr) {
    NGD_TRY(timed(h, NGD_TIMER_CORE, s, [&] { return core_gram(h, h->Bt, L, s); }));
    h->unchecked_ell = L;
    return NGD_OK;
  }
  NGD_TRY(timed(h, NGD_TIMER_CORE, s, [&] { return core_svd(h, h->Bt, L, U, ldU, lam_hat, s); }));
  // without a summary the call does not synchronise; the next PCG solve with this preconditioner
  // reads the core's error words instead
  h->unchecked_ell = info == nullptr ? L : 0;
  if (info != nullptr) {
    // one gather kernel and one copy into pinned memory: a single host round trip
    double* hv = reinterpret_cast<double*>(h->host);
    NGD_TRY(launch_sketch_info(lam_hat, (int)L, h->scal + 200, eig_error_flag(h->eigw, (int)L),
                               reinterpret_cast<const int*>(h->cholsync + 128), h->scal + 240, s));
    NGD_HIP_TRY(hipMemcpyAsync(hv, h->scal + 240, sizeof(double) * 7, hipMemcpyDeviceToHost, s));
    NGD_HIP_TRY(hipStreamSynchronize(s));
    if (hv[5] != 0.0) {
      set_error("exchange between the workgroups of the tridiagonalisation timed out");
      return NGD_ERR_HIP;
    }
    if (hv[6] != 0.0) {
      set_error("exchange between the workgroups of the Cholesky factorisation timed out");
      return NGD_ERR_HIP;
    }
    info->nu = hv[3];
    info->lam1 = hv[0];
    info->lam_ell = hv[1];
    info->rank = (int32_t)hv[2];
    info->rank_z = (int32_t)(L - (int64_t)hv[4]);
  }
  return NGD_OK;
}

namespace {

// The PCG solve behind ngd_pcg_solve (lambda given) and ngd_pcg_solve_damped (rule != NULL: lambda
// = max(c_lam lam_hat[0], c_loss loss^2) on the device). When the handle's last sketch was taken
// without its summary, its core's error words travel with the PCG state and are checked here.
struct DampingRule {
  double c_lam, c_loss;
  const double* loss;
};

ngd_status pcg_solve_impl(ngd_problem* h, const ngd_operator* op, const double* g, double lambda,
                          const DampingRule* rule, const ngd_precond* prec, double rtol, int64_t maxit, double* d,
                          ngd_pcg_info* info, double* lambda_used, void* stream) {
  NGD_CHECK(h != nullptr && g != nullptr && d != nullptr && info != nullptr, "NULL argument");
  NGD_TRY(check_op(h, op));
  if (rule == nullptr) NGD_CHECK(lambda > 0.0 && std::isfinite(lambda), "lambda must be > 0");
  NGD_CHECK(rtol >= 0.0 && maxit >= 0, "rtol >= 0 and maxit >= 0 required");
  if (prec != nullptr) {
    NGD_CHECK(prec->U != nullptr && prec->lam_hat != nullptr, "preconditioner pointers are NULL");
    NGD_CHECK(prec->ell >= 1 && prec->ell <= h->max_ell && prec->ldU >= h->P, "bad preconditioner ell / ldU");
  }
  hipStream_t s = S(stream);
  const int64_t P = h->P;
  const int plain = prec == nullptr;
  PcgState* hs = reinterpret_cast<PcgState*>(h->host);
  std::memset(hs, 0, sizeof(PcgState));
  hs->lambda = rule != nullptr ? 0.0 : lambda;
  hs->maxit = maxit;
  NGD_HIP_TRY(hipMemcpyAsync(h->pcg_st, hs, sizeof(PcgState), hipMemcpyHostToDevice, s));
  const bool check_sketch = prec != nullptr && h->unchecked_ell > 0 && prec->ell == h->unchecked_ell;
  if (rule != nullptr || check_sketch) {
    NGD_TRY(pcg_launch_setup(h->pcg_st, rule != nullptr ? prec->lam_hat : nullptr, rule != nullptr ? rule->c_lam : 0.0,
                             rule != nullptr ? rule->loss : nullptr, rule != nullptr ? rule->c_loss : 0.0,
                             check_sketch ? eig_error_flag(h->eigw, (int)prec->ell) : nullptr,
                             check_sketch ? h->cholsync + 128 : nullptr, s));
  }
  if (check_sketch) h->unchecked_ell = 0;
  NGD_TRY(pcg_launch_init(g, P, d, h->pcg_r, h->pcg_p[0], h->pcg_part, h->pcg_st, rtol, plain, s));
  double* zsrc = h->pcg_r;
  if (!plain) {
    NGD_TRY(pcg_launch_precond(h->dtype, prec->U, prec->ldU, P, (int)prec->ell, prec->lam_hat, h->pcg_s,
                               h->pcg_r, h->pcg_z, h->pcg_part, h->pcg_st, s));
    zsrc = h->pcg_z;
  }
  // Iterations are enqueued in chunks between host polls of the device state. The first chunk is the
  // previous solve's iteration count; later ones follow the observed residual decay, so that few
  // iterations are enqueued past convergence (they return at once) and few polls are needed.
  int64_t k = 0;
  int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(64, h->last_iters[plain]));
  while (true) {
    const int64_t upto = std::min<int64_t>(maxit, k + chunk);
    for (; k < upto; ++k) {
      double* pprev = h->pcg_p[k & 1];
      double* pcur = h->pcg_p[(k + 1) & 1];
      if (op->J != nullptr) {
        NGD_TRY(timed_kernel(h, NGD_TIMER_MATVEC_ROWS, [&](LaunchEvents ev) {
          return pcg_launch_rows(h->dtype, op->J, op->ldJ, h->N, P, zsrc, pprev, pcur, h->pcg_st, h->partial, h->tsq,
                                 h->nwg, s, ev);
        }));
        NGD_TRY(pcg_launch_update(h->dtype, h->partial, h->nwg, op->ldJ, P, pcur, h->tsq, d, h->pcg_r, h->pcg_part,
                                  h->pcg_st, plain, s));
      } else {
        // recompute mode: the same iteration with J_w p by the JVP and J_w^T (J_w p) by the adjoint kernel
        NGD_TRY(pcg_launch_direction(h->dtype, zsrc, pprev, P, pcur, h->pt, h->pcg_part, h->pcg_st, s));
        NGD_TRY(timed(h, NGD_TIMER_MATVEC_ROWS, s, [&] { return recompute_rows(h, op, h->pt, s); }));
        NGD_TRY(pcg_launch_update(h->dtype, h->partial, h->nwg_vjp, h->ldP, P, pcur, h->tsq, d, h->pcg_r,
                                  h->pcg_part, h->pcg_st, plain, s));
      }
      if (!plain)
        NGD_TRY(timed(h, NGD_TIMER_PRECOND, s, [&] {
          return pcg_launch_precond(h->dtype, prec->U, prec->ldU, P, (int)prec->ell, prec->lam_hat, h->pcg_s,
                                    h->pcg_r, h->pcg_z, h->pcg_part, h->pcg_st, s);
        }));
    }
    NGD_HIP_TRY(hipMemcpyAsync(hs, h->pcg_st, sizeof(PcgState), hipMemcpyDeviceToHost, s));
    NGD_HIP_TRY(hipStreamSynchronize(s));
    if (hs->done || k >= maxit) break;
    // rr_k ~ bnorm2 rate^k: predict the iterations left to reach rtol^2 bnorm2
    int64_t guess = 1;
    if (hs->rr > 0.0 && hs->bnorm2 > 0.0 && hs->rr < hs->bnorm2 && k > 0) {
      const double lrate = std::log(hs->rr / hs->bnorm2) / (double)k;
      const double need = std::log(hs->rtol2bb / hs->rr) / lrate;
      if (std::isfinite(need)) guess = (int64_t)std::ceil(std::max(1.0, need));
    } else {
      guess = chunk;
    }
    chunk = std::max<int64_t>(1, std::min<int64_t>(64, guess));
  }
  if (hs->done) {
    // launches enqueued after the iteration that finished the solve did no work
    const int64_t idle = k - hs->iters;
    if (idle > 0) drop_tail(h, NGD_TIMER_MATVEC_ROWS, idle);
    if (!plain) drop_tail(h, NGD_TIMER_PRECOND, idle + (hs->iters > 0 ? 1 : 0));
  }
  h->last_iters[plain] = hs->iters;
  info->iters = hs->iters;
  info->rel_res = hs->bnorm2 > 0 ? std::sqrt(hs->rr / hs->bnorm2) : 0.0;
  info->converged = hs->converged;
  info->breakdown = hs->breakdown;
  if (lambda_used != nullptr) *lambda_used = hs->lambda;
  if (hs->sketch_err & 1) {
    set_error("exchange between the workgroups of the sketch's tridiagonalisation timed out");
    return NGD_ERR_HIP;
  }
  if (hs->sketch_err & 2) {
    set_error("exchange between the workgroups of the sketch's Cholesky factorisation timed out");
    return NGD_ERR_HIP;
  }
  if (hs->breakdown) {
    set_error("PCG breakdown (non-positive curvature or non-finite value)");
    return NGD_ERR_BREAKDOWN;
  }
  if (!hs->converged) {
    set_error("PCG reached maxit before the tolerance");
    return NGD_ERR_NOT_CONVERGED;
  }
  return NGD_OK;
}

}  // namespace

ngd_status ngd_pcg_solve(ngd_problem* h, const ngd_operator* op, const double* g, double lambda,
                         const ngd_precond* prec, double rtol, int64_t maxit, double* d, ngd_pcg_info* info,
                         void* stream) {
  return pcg_solve_impl(h, op, g, lambda, nullptr, prec, rtol, maxit, d, info, nullptr, stream);
}

ngd_status ngd_pcg_solve_damped(ngd_problem* h, const ngd_operator* op, const double* g, double c_lam,
                                double c_loss, const double* loss, const ngd_precond* prec, double rtol,
                                int64_t maxit, double* d, ngd_pcg_info* info, double* lambda_used, void* stream) {
  NGD_CHECK(prec != nullptr && loss != nullptr, "the damping rule needs the preconditioner and the loss");
  NGD_CHECK(c_lam >= 0.0 && c_loss >= 0.0 && (c_lam > 0.0 || c_loss > 0.0), "c_lam, c_loss >= 0, not both 0");
  const DampingRule rule{c_lam, c_loss, loss};
  return pcg_solve_impl(h, op, g, 0.0, &rule, prec, rtol, maxit, d, info, lambda_used, stream);
}

ngd_status ngd_power_lambda_max(ngd_problem* h, const ngd_operator* op, const double* v0, int32_t iters, double* lam1,
                                double* lam1_dev, void* stream) {
  NGD_CHECK(h != nullptr && v0 != nullptr && lam1 != nullptr, "NULL argument");
  NGD_TRY(check_op(h, op));
  NGD_CHECK(iters >= 1, "iters must be >= 1");
  hipStream_t s = S(stream);
  const int64_t P = h->P;
  double* v = h->vtmp[0];
  double* w = h->vtmp[1];
  double* sc = h->scal;  // [0] v.w, [1] w.w, [2] v0.v0, [8..] dot workspace
  NGD_TRY(launch_dot(v0, v0, P, sc + 8, sc + 2, s));
  NGD_TRY(launch_scale_rsqrt(v0, sc + 2, P, v, s));
  for (int it = 0; it < iters; ++it) {
    NGD_TRY(gram_apply(h, op, v, 0.0, w, s));
    NGD_TRY(launch_dot(v, w, P, sc + 8, sc + 0, s));
    NGD_TRY(launch_dot(w, w, P, sc + 8, sc + 1, s));
    NGD_TRY(launch_scale_rsqrt(w, sc + 1, P, v, s));
  }
  if (lam1_dev != nullptr) NGD_HIP_TRY(hipMemcpyAsync(lam1_dev, sc, sizeof(double), hipMemcpyDeviceToDevice, s));
  double* hv = reinterpret_cast<double*>(h->host);
  NGD_HIP_TRY(hipMemcpyAsync(hv, sc, sizeof(double), hipMemcpyDeviceToHost, s));
  NGD_HIP_TRY(hipStreamSynchronize(s));
  *lam1 = hv[0];
  return NGD_OK;
}

ngd_status ngd_damping(ngd_problem* h, const double* lam1, const double* loss, double c_lam, double c_loss,
                       double* mu, double* mu_host, void* stream) {
  NGD_CHECK(h != nullptr && lam1 != nullptr && mu != nullptr, "NULL argument");
  NGD_CHECK(c_lam >= 0.0 && c_loss >= 0.0 && std::isfinite(c_lam) && std::isfinite(c_loss),
            "c_lam and c_loss must be finite and >= 0");
  hipStream_t s = S(stream);
  NGD_TRY(launch_damping1(lam1, loss, c_lam, c_loss, mu, s));
  if (mu_host != nullptr) {
    double* hv = reinterpret_cast<double*>(h->host);
    NGD_HIP_TRY(hipMemcpyAsync(hv, mu, sizeof(double), hipMemcpyDeviceToHost, s));
    NGD_HIP_TRY(hipStreamSynchronize(s));
    *mu_host = hv[0];
  }
  return NGD_OK;
}

ngd_status ngd_lm_damping(ngd_problem* h, const ngd_operator* op, const double* d, const double* grad, double alpha,
                          double loss0, double loss1, double mu, double mu_floor, double* mu_next, double* rho,
                          void* stream) {
  NGD_CHECK(h != nullptr && d != nullptr && grad != nullptr && mu_next != nullptr, "NULL argument");
  NGD_CHECK(std::isfinite(mu) && mu > 0.0, "mu must be finite and > 0");
  NGD_CHECK(std::isfinite(mu_floor) && mu_floor >= 0.0, "mu_floor must be finite and >= 0");
  NGD_CHECK(std::isfinite(alpha) && alpha >= 0.0, "alpha must be finite and >= 0");
  NGD_TRY(check_op(h, op));
  hipStream_t s = S(stream);
  double* sc = h->scal;  // [4] g^T d, [5] d^T G d, [6] mu_next, [7] rho, [8..] dot workspace
  NGD_TRY(gram_apply(h, op, d, 0.0, h->vtmp[3], s));
  NGD_TRY(launch_dot(grad, d, h->P, sc + 8, sc + 4, s));
  NGD_TRY(launch_dot(d, h->vtmp[3], h->P, sc + 8, sc + 5, s));
  NGD_TRY(launch_lm_damping(sc + 4, sc + 5, alpha, loss0, loss1, mu, mu_floor, sc + 6, s));
  double* hv = reinterpret_cast<double*>(h->host);
  NGD_HIP_TRY(hipMemcpyAsync(hv, sc + 6, sizeof(double) * 2, hipMemcpyDeviceToHost, s));
  NGD_HIP_TRY(hipStreamSynchronize(s));
  *mu_next = hv[0];
  if (rho != nullptr) *rho = hv[1];
  return NGD_OK;
}

ngd_status ngd_next_rank(ngd_problem* h, const double* lam_hat, int64_t ell, double mu, int64_t dell,
                         int64_t offset, int64_t ell_max, int64_t* next_ell, void* stream) {
  NGD_CHECK(h != nullptr && lam_hat != nullptr && next_ell != nullptr, "NULL argument");
  NGD_CHECK(ell >= 1 && dell >= 0 && offset >= 0 && ell_max >= 1, "ell >= 1, dell >= 0, offset >= 0, ell_max >= 1");
  NGD_CHECK(mu >= 0.0 && std::isfinite(mu), "mu must be finite and >= 0");
  hipStream_t s = S(stream);
  int64_t* slot = reinterpret_cast<int64_t*>(h->scal + 250);
  NGD_TRY(launch_next_rank(lam_hat, ell, mu, dell, offset, std::min<int64_t>(ell_max, h->P), slot, s));
  int64_t* hv = reinterpret_cast<int64_t*>(h->host);
  NGD_HIP_TRY(hipMemcpyAsync(hv, slot, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  NGD_HIP_TRY(hipStreamSynchronize(s));
  *next_ell = hv[0];
  return NGD_OK;
}

ngd_status ngd_solution_error(ngd_problem* h, const void* theta, const void* X, int64_t n, const void* u_ref,
                              const void* grad_u_ref, double* sums, void* stream) {
  NGD_CHECK(h != nullptr && sums != nullptr, "NULL argument");
  NGD_CHECK(n >= 0, "n must be >= 0");
  NGD_CHECK(n == 0 || (theta && X && u_ref && grad_u_ref), "NULL argument");
  if (h->ns)
    return launch_ns_velocity_error(h->nsd, h->dtype, theta, X, n, u_ref, grad_u_ref, h->err_part, kEvalBlocks, sums,
                                    S(stream));
  return launch_solution_error(h->net, h->dtype, theta, X, n, u_ref, grad_u_ref, h->err_part, sums, S(stream));
}

ngd_status ngd_line_search(ngd_problem* h, const void* theta, const double* d, const double* grad, double loss0,
                           double c1, int32_t max_halvings, void* theta_out, double* alpha, double* loss_new,
                           void* stream) {
  NGD_CHECK(h != nullptr && theta && d && grad && theta_out && alpha && loss_new, "NULL argument");
  NGD_CHECK(max_halvings >= 0 && c1 >= 0.0, "max_halvings >= 0 and c1 >= 0 required");
  hipStream_t s = S(stream);
  const int64_t P = h->P;
  double* hv = reinterpret_cast<double*>(h->host);  // [0] slope, [8..15] alphas, [16..23] losses
  // the slope comes back with the first batch of trial losses (the trial steps do not depend on it)
  NGD_TRY(launch_dot(grad, d, P, h->scal + 8, h->scal + 0, s));
  NGD_HIP_TRY(hipMemcpyAsync(hv, h->scal, sizeof(double), hipMemcpyDeviceToHost, s));
  int tried = 0;
  double accepted = 0.0, acc_loss = loss0;
  bool found = false;
  int accepted_index = -1;
  int batch = h->ls_first_batch;
  while (!found && tried <= max_halvings) {
    const int nt = std::min(batch, max_halvings + 1 - tried);
    for (int t = 0; t < nt; ++t) hv[8 + t] = std::ldexp(1.0, -(tried + t));
    NGD_HIP_TRY(hipMemcpyAsync(h->alphas, hv + 8, sizeof(double) * nt, hipMemcpyHostToDevice, s));
    NGD_TRY(launch_axpy_theta(h->dtype, theta, d, h->alphas, nt, P, h->trial, h->ldP, s));
    const int nb = h->ns ? ns_blocks(h->N) : residual_blocks(h->net, h->dtype, h->N, false);
    NGD_CHECK(nb <= h->res_blocks, "residual launch exceeds its loss-partial buffer");
    if (h->ns)
      NGD_TRY(launch_ns_residual(h->nsd, h->dtype, h->trial, h->ldP, nt, h->N, h->X, h->w, h->f, h->g, h->kind,
                                 nullptr, nullptr, 0, h->loss_part, s));
    else
      NGD_TRY(launch_residual_jacobian(h->net, h->dtype, h->trial, h->N, h->X, h->w, h->f, h->g, h->kind, nullptr,
                                       nullptr, 0, h->loss_part, h->ldP, nt, s, nullptr));
    NGD_TRY(launch_reduce_sum(h->loss_part, nb, nt, 0.5, h->losses, s));
    NGD_HIP_TRY(hipMemcpyAsync(hv + 16, h->losses, sizeof(double) * nt, hipMemcpyDeviceToHost, s));
    NGD_HIP_TRY(hipStreamSynchronize(s));
    const double slope = hv[0];
    for (int t = 0; t < nt; ++t) {
      const double a = hv[8 + t], Lt = hv[16 + t];
      if (Lt <= loss0 - c1 * a * slope) {
        accepted = a;
        acc_loss = Lt;
        found = true;
        accepted_index = tried + t;
        break;
      }
    }
    tried += nt;
    batch = h->ls_batch;
  }
  h->ls_first_batch = accepted_index == 0 ? 1 : h->ls_batch;
  // theta_out = theta - alpha d (alpha = 0 copies theta), alpha passed by value
  NGD_TRY(launch_axpy_theta(h->dtype, theta, d, nullptr, 1, P, theta_out, h->ldP, s, accepted));
  NGD_HIP_TRY(hipStreamSynchronize(s));
  *alpha = accepted;
  *loss_new = acc_loss;
  return NGD_OK;
}

ngd_status ngd_timing_enable(ngd_problem* h, int32_t enable) {
  return ngd_timing_enable_mask(h, enable != 0 ? (1u << NGD_NUM_TIMERS) - 1u : 0u);
}

ngd_status ngd_timing_enable_mask(ngd_problem* h, uint32_t mask) {
  NGD_CHECK(h != nullptr, "NULL handle");
  NGD_TRY(flush_timers(h));
  h->timing = mask & ((1u << NGD_NUM_TIMERS) - 1u);
  for (int i = 0; i < NGD_NUM_TIMERS; ++i) {
    h->t_ms[i] = 0.0;
    h->t_n[i] = 0;
  }
  return NGD_OK;
}

ngd_status ngd_timing_read(ngd_problem* h, int32_t id, int64_t* launches, double* total_ms) {
  NGD_CHECK(h != nullptr && launches != nullptr && total_ms != nullptr, "NULL argument");
  NGD_CHECK(id >= 0 && id < NGD_NUM_TIMERS, "timer id out of range");
  NGD_TRY(flush_timers(h));
  *launches = h->t_n[id];
  *total_ms = h->t_ms[id];
  return NGD_OK;
}

// ================= batched problems =================

struct ngd_batch {
  std::vector<ngd_problem*> inst;
  int dtype = NGD_F32;
  BatchResidualItem* d_res = nullptr;
  BatchResidualItem* h_res = nullptr;
  PcgBatchItem* d_pcg = nullptr;
  PcgBatchItem* h_pcg = nullptr;
  PcgState* d_states = nullptr;
  PcgState* h_states = nullptr;
  hipStream_t capture = nullptr;      // stream on which the PCG iteration is captured
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<int64_t> graph_key;     // launch shapes the captured graph was built for
  int rows_target = 0;                // autotuned rows per matvec workgroup (0: not tuned yet)
  std::vector<int64_t> tuned_for;     // problem shapes the tuning applies to
  int64_t last_iters = 4;
  // streams (default priority) over which the members' sketches run side by side, and the events
  // that fork them from and join them to the caller's stream; created on first use
  static constexpr int kSketchStreams = 4;
  hipStream_t sk_stream[kSketchStreams] = {};
  hipEvent_t sk_fork = nullptr, sk_join[kSketchStreams] = {};
  int* h_err = nullptr;               // pinned: two error words per member (sketch core checks)
  double* h_ls = nullptr;             // pinned: the line search's decision per member (4 doubles)
};

namespace {

void batch_release(ngd_batch* b) {
  for (int q = 0; q < ngd_batch::kSketchStreams; ++q) {
    if (b->sk_stream[q]) {
      (void)hipStreamSynchronize(b->sk_stream[q]);
      (void)hipStreamDestroy(b->sk_stream[q]);
    }
    if (b->sk_join[q]) (void)hipEventDestroy(b->sk_join[q]);
  }
  if (b->sk_fork) (void)hipEventDestroy(b->sk_fork);
  if (b->h_err) (void)hipHostFree(b->h_err);
  if (b->h_ls) (void)hipHostFree(b->h_ls);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->capture) (void)hipStreamDestroy(b->capture);
  (void)hipFree(b->d_res);
  (void)hipFree(b->d_pcg);
  (void)hipFree(b->d_states);
  (void)hipHostFree(b->h_res);
  (void)hipHostFree(b->h_pcg);
  (void)hipHostFree(b->h_states);
  for (ngd_problem* h : b->inst) ngd_problem_destroy(h);
  delete b;
}

// per-problem matvec workgroups for a target number of rows per workgroup
int batch_nwg(const ngd_problem* h, int rows_target) {
  int64_t w = rows_target > 0 ? (h->N + rows_target - 1) / rows_target : h->nwg;
  return (int)std::max<int64_t>(1, std::min<int64_t>(w, h->nwg));
}

}  // namespace

ngd_status ngd_batch_create(const ngd_problem_desc* descs, int32_t n, ngd_batch** out) {
  NGD_CHECK(descs != nullptr && out != nullptr, "NULL argument");
  NGD_CHECK(n >= 1 && n <= 4096, "batch size out of range [1, 4096]");
  *out = nullptr;
  ngd_batch* b = new ngd_batch();
  b->dtype = descs[0].dtype;
  for (int i = 0; i < n; ++i) {
    if (descs[i].dtype != b->dtype) {
      batch_release(b);
      set_error("all problems of a batch must share one dtype");
      return NGD_ERR_INVALID;
    }
    if (descs[i].pde == NGD_PDE_NAVIER_STOKES) {
      batch_release(b);
      set_error("batches take Poisson and heat problems only");
      return NGD_ERR_INVALID;
    }
    ngd_problem* h = nullptr;
    ngd_status st = ngd_problem_create(&descs[i], &h);
    if (st != NGD_OK) {
      batch_release(b);
      return st;
    }
    b->inst.push_back(h);
  }
  bool ok = hipMalloc(&b->d_res, sizeof(BatchResidualItem) * n) == hipSuccess &&
            hipMalloc(&b->d_pcg, sizeof(PcgBatchItem) * n) == hipSuccess &&
            hipMalloc(&b->d_states, sizeof(PcgState) * n) == hipSuccess &&
            hipHostMalloc(&b->h_res, sizeof(BatchResidualItem) * n, hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc(&b->h_pcg, sizeof(PcgBatchItem) * n, hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc(&b->h_states, sizeof(PcgState) * n, hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc(&b->h_err, sizeof(int) * 2 * n, hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc(&b->h_ls, sizeof(double) * 4 * n, hipHostMallocDefault) == hipSuccess;
  if (!ok) {
    batch_release(b);
    set_error("batch allocation failed");
    return NGD_ERR_OOM;
  }
  *out = b;
  return NGD_OK;
}

ngd_status ngd_batch_destroy(ngd_batch* b) {
  if (b != nullptr) batch_release(b);
  return NGD_OK;
}

int32_t ngd_batch_size(const ngd_batch* b) { return b ? (int32_t)b->inst.size() : -1; }

ngd_problem* ngd_batch_problem(ngd_batch* b, int32_t i) {
  return (b != nullptr && i >= 0 && i < (int32_t)b->inst.size()) ? b->inst[i] : nullptr;
}

ngd_status batch_streams(ngd_batch* b);

ngd_status ngd_batch_residual_jacobian(ngd_batch* b, const void* const* theta, void* const* r_w, void* const* J_w,
                                       const int64_t* ldJ, double* const* grad, double* const* loss, void* stream) {
  NGD_CHECK(b != nullptr && theta != nullptr && r_w != nullptr && J_w != nullptr && ldJ != nullptr, "NULL argument");
  hipStream_t s = S(stream);
  const int n = (int)b->inst.size();
  // the host table is reused by every call: wait until the previous call's copy has been consumed
  NGD_HIP_TRY(hipStreamSynchronize(s));
  // Members are grouped by the LDS their tiles need (how many workgroups share a CU: four or more, two
  // or three, one), and each group is one persistent launch with its own LDS size: a single launch
  // would reserve the widest member's LDS for every tile and hold the narrow ones to its occupancy.
  std::vector<int> tps(n), cls(n);
  std::vector<size_t> ldsb(n);
  for (int i = 0; i < n; ++i) {
    ngd_problem* h = b->inst[i];
    NGD_CHECK(theta[i] != nullptr && r_w[i] != nullptr && J_w[i] != nullptr, "NULL problem pointer");
    NGD_CHECK(ldJ[i] >= h->P, "ldJ < P");
    ldsb[i] = residual_lds_bytes(h->net, h->dtype, &tps[i]);
    const size_t per_cu = ldsb[i] > 0 ? (160 * 1024) / ldsb[i] : 8;
    cls[i] = per_cu >= 4 ? 0 : (per_cu >= 2 ? 1 : 2);
  }
  int slot = 0;
  struct Group { int first, count; int64_t tiles; size_t lds; };
  std::vector<Group> groups;
  for (int c = 0; c < 3; ++c) {
    Group gr{slot, 0, 0, 0};
    for (int i = 0; i < n; ++i) {
      if (cls[i] != c) continue;
      ngd_problem* h = b->inst[i];
      BatchResidualItem& it = b->h_res[slot++];
      it.net = h->net;
      it.theta = theta[i];
      it.X = h->X;
      it.w = h->w;
      it.f = h->f;
      it.g = h->g;
      it.kind = h->kind;
      it.r_w = r_w[i];
      it.J = J_w[i];
      it.ldJ = ldJ[i];
      it.N = h->N;
      it.first_tile = gr.tiles;
      it.TP = tps[i];
      it.loss_part = h->loss_part;
      gr.tiles += (h->N + tps[i] - 1) / tps[i];
      gr.lds = std::max(gr.lds, ldsb[i]);
      ++gr.count;
    }
    if (gr.count > 0) groups.push_back(gr);
  }
  NGD_HIP_TRY(hipMemcpyAsync(b->d_res, b->h_res, sizeof(BatchResidualItem) * n, hipMemcpyHostToDevice, s));
  for (const Group& gr : groups)
    NGD_TRY(launch_batch_residual_jacobian(b->dtype, b->d_res + gr.first, gr.count, gr.tiles, gr.lds, s));
  // each member's loss and gradient (one pass over its J_w) side by side on the batch's streams
  for (int i = 0; i < n; ++i)
    if (grad != nullptr && grad[i] != nullptr) {
      const ngd_operator op{theta[i], J_w[i], ldJ[i]};
      NGD_TRY(check_op(b->inst[i], &op));
    }
  NGD_TRY(batch_streams(b));
  NGD_HIP_TRY(hipEventRecord(b->sk_fork, s));
  for (int q = 0; q < ngd_batch::kSketchStreams; ++q) NGD_HIP_TRY(hipStreamWaitEvent(b->sk_stream[q], b->sk_fork, 0));
  for (int i = 0; i < n; ++i) {
    ngd_problem* h = b->inst[i];
    hipStream_t qs = b->sk_stream[i % ngd_batch::kSketchStreams];
    const int nt = (int)((h->N + tps[i] - 1) / tps[i]);
    if (loss != nullptr && loss[i] != nullptr) NGD_TRY(launch_reduce_sum(h->loss_part, nt, 1, 0.5, loss[i], qs));
    if (grad != nullptr && grad[i] != nullptr) {
      NGD_TRY(launch_grad_rows(h->dtype, J_w[i], ldJ[i], h->N, r_w[i], h->partial, h->nwg, qs));
      NGD_TRY(launch_gram_reduce(h->dtype, h->partial, h->nwg, ldJ[i], h->P, nullptr, 0.0, grad[i], qs));
    }
  }
  for (int q = 0; q < ngd_batch::kSketchStreams; ++q) {
    NGD_HIP_TRY(hipEventRecord(b->sk_join[q], b->sk_stream[q]));
    NGD_HIP_TRY(hipStreamWaitEvent(s, b->sk_join[q], 0));
  }
  return NGD_OK;
}

namespace {

// item numbering of the batched PCG launches for the current per-problem workgroup counts
void batch_pcg_items(ngd_batch* b, int* rows, int* upd, int* dots, int* elem, int* apply) {
  *rows = *upd = *dots = *elem = *apply = 0;
  for (size_t i = 0; i < b->inst.size(); ++i) {
    PcgBatchItem& it = b->h_pcg[i];
    it.nwg = batch_nwg(b->inst[i], b->rows_target);
    it.item0_rows = *rows;
    it.item0_upd = *upd;
    it.item0_dots = *dots;
    it.item0_elem = *elem;
    it.item0_apply = *apply;
    *rows += it.nwg;
    *upd += (int)((it.P + 31) / 32);
    *elem += (int)((it.P + 255) / 256);
    if (!it.plain) {
      *dots += it.ell;
      *apply += (int)((it.P + 255) / 256);
    }
  }
}

}  // namespace

namespace {

// The batched PCG solve behind ngd_batch_pcg_solve (lambda given per problem) and
// ngd_batch_pcg_solve_damped (lambda == NULL: the damping rule on the device from each problem's
// lam_hat[0] and loss).
ngd_status batch_pcg_impl(ngd_batch* b, const ngd_operator* ops, const double* const* g, const double* lambda,
                          const double* const* loss, double c_lam, double c_loss, const ngd_precond* precs,
                          double rtol, int64_t maxit, double* const* d, ngd_pcg_info* infos, double* lambda_used,
                          void* stream) {
  NGD_CHECK(b != nullptr && ops != nullptr && g != nullptr && d != nullptr && infos != nullptr, "NULL argument");
  const bool rule = lambda == nullptr;
  if (rule) NGD_CHECK(precs != nullptr, "the device damping rule needs every problem's preconditioner");
  NGD_CHECK(rtol >= 0.0 && maxit >= 0, "rtol >= 0 and maxit >= 0 required");
  hipStream_t s = S(stream);
  const int n = (int)b->inst.size();
  NGD_HIP_TRY(hipStreamSynchronize(s));  // the host tables are reused by every call
  int64_t max_ld = 0;
  int max_ell = 1;
  std::vector<int64_t> shape;
  for (int i = 0; i < n; ++i) {
    ngd_problem* h = b->inst[i];
    NGD_CHECK(ops[i].J != nullptr, "the batched solve needs stored Jacobians");
    NGD_TRY(check_op(h, &ops[i]));
    if (!rule) NGD_CHECK(lambda[i] > 0.0 && std::isfinite(lambda[i]), "lambda must be > 0");
    NGD_CHECK(g[i] != nullptr && d[i] != nullptr, "NULL problem pointer");
    const ngd_precond* pc = (precs != nullptr && precs[i].U != nullptr) ? &precs[i] : nullptr;
    if (rule) NGD_CHECK(pc != nullptr, "the device damping rule needs every problem's preconditioner");
    if (pc != nullptr) {
      NGD_CHECK(pc->lam_hat != nullptr, "preconditioner pointers are NULL");
      NGD_CHECK(pc->ell >= 1 && pc->ell <= h->max_ell && pc->ldU >= h->P, "bad preconditioner ell / ldU");
    }
    PcgBatchItem& it = b->h_pcg[i];
    it.J = ops[i].J;
    it.ldJ = ops[i].ldJ;
    it.N = h->N;
    it.P = h->P;
    it.g = g[i];
    it.x = d[i];
    it.r = h->pcg_r;
    it.z = h->pcg_z;
    it.p0 = h->pcg_p[0];
    it.p1 = h->pcg_p[1];
    it.s = h->pcg_s;
    it.part = h->pcg_part;
    it.partial = h->partial;
    it.tsq = h->tsq;
    it.st = b->d_states + i;
    it.U = pc ? pc->U : nullptr;
    it.ldU = pc ? pc->ldU : 0;
    it.lam = pc ? pc->lam_hat : nullptr;
    it.loss = rule && loss != nullptr ? loss[i] : nullptr;
    it.mu = rule ? 0.0 : lambda[i];
    it.rtol = rtol;
    it.ell = pc ? (int)pc->ell : 0;
    it.plain = pc == nullptr;
    max_ld = std::max(max_ld, ops[i].ldJ);
    max_ell = std::max(max_ell, it.ell);
    shape.push_back(h->N);
    shape.push_back(ops[i].ldJ);
    PcgState& st = b->h_states[i];
    std::memset(&st, 0, sizeof(PcgState));
    st.lambda = rule ? 0.0 : lambda[i];
    st.maxit = maxit;
  }
  // the core error words of sketches taken without their summary, read back with the solve's state
  std::vector<int> checked;
  for (int i = 0; i < n; ++i) {
    ngd_problem* h = b->inst[i];
    const ngd_precond* pc = (precs != nullptr && precs[i].U != nullptr) ? &precs[i] : nullptr;
    if (pc == nullptr || h->unchecked_ell == 0 || pc->ell != h->unchecked_ell) continue;
    NGD_HIP_TRY(hipMemcpyAsync(b->h_err + 2 * i, eig_error_flag(h->eigw, (int)pc->ell), sizeof(int),
                               hipMemcpyDeviceToHost, s));
    NGD_HIP_TRY(hipMemcpyAsync(b->h_err + 2 * i + 1, h->cholsync + 128, sizeof(int), hipMemcpyDeviceToHost, s));
    h->unchecked_ell = 0;
    checked.push_back(i);
  }
  NGD_TRY(pcg_batch_prepare(b->dtype, max_ld, max_ell));
  int rows, upd, dots, elem, apply;
  // autotune the split of each problem's rows over matvec workgroups (once per set of shapes): time
  // one batched matvec launch per candidate on this solve's first direction; that launch only writes
  // buffers the first iteration rewrites
  const bool tune = b->rows_target == 0 || b->tuned_for != shape;
  if (tune) b->rows_target = 0;
  batch_pcg_items(b, &rows, &upd, &dots, &elem, &apply);
  NGD_HIP_TRY(hipMemcpyAsync(b->d_states, b->h_states, sizeof(PcgState) * n, hipMemcpyHostToDevice, s));
  NGD_HIP_TRY(hipMemcpyAsync(b->d_pcg, b->h_pcg, sizeof(PcgBatchItem) * n, hipMemcpyHostToDevice, s));
  if (rule) NGD_TRY(pcg_batch_launch_damping(b->d_pcg, b->d_states, n, c_lam, c_loss, s));
  NGD_TRY(pcg_batch_launch_init(b->dtype, b->d_pcg, n, elem, s));
  NGD_TRY(pcg_batch_launch_precond(b->dtype, b->d_pcg, n, dots, apply, max_ell, s));
  if (tune) {
    const int cand[4] = {8, 16, 32, 64};
    float best = 1e30f;
    int best_t = 16;
    hipEvent_t e0, e1;
    NGD_HIP_TRY(hipEventCreate(&e0));
    NGD_HIP_TRY(hipEventCreate(&e1));
    for (int t : cand) {
      b->rows_target = t;
      batch_pcg_items(b, &rows, &upd, &dots, &elem, &apply);
      NGD_HIP_TRY(hipStreamSynchronize(s));
      NGD_HIP_TRY(hipMemcpyAsync(b->d_pcg, b->h_pcg, sizeof(PcgBatchItem) * n, hipMemcpyHostToDevice, s));
      float ms_best = 1e30f;
      for (int rep = 0; rep < 3; ++rep) {
        NGD_HIP_TRY(hipEventRecord(e0, s));
        NGD_TRY(pcg_batch_launch_rows(b->dtype, b->d_pcg, n, rows, max_ld, s));
        NGD_HIP_TRY(hipEventRecord(e1, s));
        NGD_HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        NGD_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        ms_best = std::min(ms_best, ms);
      }
      if (ms_best < best) {
        best = ms_best;
        best_t = t;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->rows_target = best_t;
    b->tuned_for = shape;
    batch_pcg_items(b, &rows, &upd, &dots, &elem, &apply);
    NGD_HIP_TRY(hipStreamSynchronize(s));
    NGD_HIP_TRY(hipMemcpyAsync(b->d_pcg, b->h_pcg, sizeof(PcgBatchItem) * n, hipMemcpyHostToDevice, s));
  }
  // one PCG iteration of every problem = 2 (plain CG) or 4 batched launches, captured once as a graph
  std::vector<int64_t> key = {rows, upd, dots, apply, max_ld, max_ell, b->dtype};
  if (b->exec == nullptr || b->graph_key != key) {
    if (b->exec) NGD_HIP_TRY(hipGraphExecDestroy(b->exec));
    if (b->graph) NGD_HIP_TRY(hipGraphDestroy(b->graph));
    b->exec = nullptr;
    b->graph = nullptr;
    if (b->capture == nullptr) NGD_HIP_TRY(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking));
    NGD_HIP_TRY(hipStreamBeginCapture(b->capture, hipStreamCaptureModeRelaxed));
    ngd_status st = pcg_batch_launch_rows(b->dtype, b->d_pcg, n, rows, max_ld, b->capture);
    if (st == NGD_OK) st = pcg_batch_launch_update(b->dtype, b->d_pcg, n, upd, b->capture);
    if (st == NGD_OK) st = pcg_batch_launch_precond(b->dtype, b->d_pcg, n, dots, apply, max_ell, b->capture);
    hipGraph_t graph = nullptr;
    const hipError_t ce = hipStreamEndCapture(b->capture, &graph);
    if (st != NGD_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    NGD_HIP_TRY(ce);
    b->graph = graph;
    NGD_HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->graph_key = key;
  }
  int64_t k = 0;
  int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(64, b->last_iters));
  while (true) {
    const int64_t upto = std::min<int64_t>(maxit, k + chunk);
    for (; k < upto; ++k) NGD_HIP_TRY(hipGraphLaunch(b->exec, s));
    NGD_HIP_TRY(hipMemcpyAsync(b->h_states, b->d_states, sizeof(PcgState) * n, hipMemcpyDeviceToHost, s));
    NGD_HIP_TRY(hipStreamSynchronize(s));
    bool all_done = true;
    for (int i = 0; i < n; ++i) all_done = all_done && (b->h_states[i].done != 0);
    if (all_done || k >= maxit) break;
    chunk = std::min<int64_t>(chunk * 2, 64);
  }
  for (int i : checked) {
    if (b->h_err[2 * i] != 0 || b->h_err[2 * i + 1] != 0) {
      set_error("exchange between the workgroups of a member's sketch core timed out (problem " + std::to_string(i) +
                ")");
      return NGD_ERR_HIP;
    }
  }
  ngd_status ret = NGD_OK;
  int64_t most = 0;
  for (int i = 0; i < n; ++i) {
    const PcgState& st = b->h_states[i];
    if (lambda_used != nullptr) lambda_used[i] = st.lambda;
    infos[i].iters = st.iters;
    infos[i].rel_res = st.bnorm2 > 0 ? std::sqrt(st.rr / st.bnorm2) : 0.0;
    infos[i].converged = st.converged;
    infos[i].breakdown = st.breakdown;
    most = std::max<int64_t>(most, st.iters);
    if (st.breakdown) ret = NGD_ERR_BREAKDOWN;
    else if (!st.converged && ret == NGD_OK) ret = NGD_ERR_NOT_CONVERGED;
  }
  b->last_iters = std::max<int64_t>(1, most);
  if (ret == NGD_ERR_BREAKDOWN) set_error("batched PCG: breakdown in at least one problem");
  else if (ret == NGD_ERR_NOT_CONVERGED) set_error("batched PCG: at least one problem reached maxit");
  return ret;
}

}  // namespace

ngd_status ngd_batch_pcg_solve(ngd_batch* b, const ngd_operator* ops, const double* const* g, const double* lambda,
                               const ngd_precond* precs, double rtol, int64_t maxit, double* const* d,
                               ngd_pcg_info* infos, void* stream) {
  NGD_CHECK(lambda != nullptr, "NULL argument");
  return batch_pcg_impl(b, ops, g, lambda, nullptr, 0.0, 0.0, precs, rtol, maxit, d, infos, nullptr, stream);
}

ngd_status ngd_batch_pcg_solve_damped(ngd_batch* b, const ngd_operator* ops, const double* const* g,
                                      double c_lam, double c_loss, const double* const* loss,
                                      const ngd_precond* precs, double rtol, int64_t maxit, double* const* d,
                                      ngd_pcg_info* infos, double* lambda_used, void* stream) {
  NGD_CHECK(std::isfinite(c_lam) && std::isfinite(c_loss) && c_lam >= 0.0 && c_loss >= 0.0,
            "c_lam and c_loss must be finite and >= 0");
  return batch_pcg_impl(b, ops, g, nullptr, loss, c_lam, c_loss, precs, rtol, maxit, d, infos, lambda_used, stream);
}

// the batch's pool streams and their fork / join events, created on first use
ngd_status batch_streams(ngd_batch* b) {
  if (b->sk_fork != nullptr) return NGD_OK;
  NGD_HIP_TRY(hipEventCreateWithFlags(&b->sk_fork, hipEventDisableTiming));
  for (int q = 0; q < ngd_batch::kSketchStreams; ++q) {
    NGD_HIP_TRY(hipStreamCreateWithFlags(&b->sk_stream[q], hipStreamNonBlocking));
    NGD_HIP_TRY(hipEventCreateWithFlags(&b->sk_join[q], hipEventDisableTiming));
  }
  return NGD_OK;
}

// The members' Nystrom sketches side by side: member i (largest cost first) on pool stream
// i % kSketchStreams, forked from and joined back to the caller's stream; no host round trip.
ngd_status ngd_batch_nystrom_sketch(ngd_batch* b, const ngd_operator* ops, const int64_t* ells, uint64_t seed,
                                    uint64_t counter, int32_t sketch_dtype, void* const* U, const int64_t* ldU,
                                    double* const* lam_hat, void* stream) {
  NGD_CHECK(b != nullptr && ops != nullptr && ells != nullptr && U != nullptr && ldU != nullptr && lam_hat != nullptr,
            "NULL argument");
  const int n = (int)b->inst.size();
  for (int i = 0; i < n; ++i) {
    ngd_problem* h = b->inst[i];
    NGD_TRY(check_op(h, &ops[i]));
    NGD_CHECK(ells[i] >= 1 && ells[i] <= h->max_ell, "ell must be in [1, min(max_ell, P)] for every problem");
    NGD_CHECK(U[i] != nullptr && lam_hat[i] != nullptr && ldU[i] >= h->P, "bad output of a problem");
  }
  NGD_TRY(batch_streams(b));
  hipStream_t s = S(stream);
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  auto cost = [&](int i) { return (double)ells[i] * (double)b->inst[i]->P * (double)(b->inst[i]->N + ells[i]); };
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost(x) > cost(y); });
  // FP32 members: each sketch up to its core's Gram matrix side by side, then every core's
  // tridiagonalisation, multisection, inverse iteration and cluster orthogonalisation in batched
  // launches on the caller's stream (a member's tridiagonalisation is a chain of grid barriers on a
  // few CUs and the next stages are a few waves each: side by side on four streams most of the device
  // idled), then the rest of each core side by side again
  bool batch_eig = true;
  for (int i = 0; i < n; ++i) batch_eig = batch_eig && b->inst[i]->dtype != NGD_F64;
  auto fork = [&] {
    NGD_HIP_TRY(hipEventRecord(b->sk_fork, s));
    for (int q = 0; q < ngd_batch::kSketchStreams; ++q)
      NGD_HIP_TRY(hipStreamWaitEvent(b->sk_stream[q], b->sk_fork, 0));
    return NGD_OK;
  };
  auto join = [&] {
    for (int q = 0; q < ngd_batch::kSketchStreams; ++q) {
      NGD_HIP_TRY(hipEventRecord(b->sk_join[q], b->sk_stream[q]));
      NGD_HIP_TRY(hipStreamWaitEvent(s, b->sk_join[q], 0));
    }
    return NGD_OK;
  };
  NGD_TRY(fork());
  for (int k = 0; k < n; ++k) {
    const int i = order[k];
    hipStream_t qs = b->sk_stream[k % ngd_batch::kSketchStreams];
    // member i's test matrix from its own counter range (counter, i)
    NGD_TRY(sketch_impl(b->inst[i], &ops[i], ells[i], seed, counter + ((uint64_t)i << 32), nullptr, 0, nullptr,
                        sketch_dtype, U[i], ldU[i], lam_hat[i], nullptr, qs, batch_eig));
  }
  NGD_TRY(join());
  if (!batch_eig) return NGD_OK;
  std::vector<EigJob> jobs(n);
  for (int i = 0; i < n; ++i) {
    ngd_problem* h = b->inst[i];
    jobs[i] = EigJob{h->M, (int)ells[i], h->eigw, false, kDropRel, h->side, h->ev_fork, h->ev_join};
  }
  NGD_TRY(launch_sym_eig_tridiag_batch(jobs.data(), n, s));
  NGD_TRY(launch_sym_eig_middle_batch(jobs.data(), n, s));
  NGD_TRY(fork());
  for (int k = 0; k < n; ++k) {
    const int i = order[k];
    hipStream_t qs = b->sk_stream[k % ngd_batch::kSketchStreams];
    NGD_TRY(core_svd_finish(b->inst[i], b->inst[i]->Bt, ells[i], U[i], ldU[i], lam_hat[i], qs));
  }
  return join();
}

// Every member's Armijo line search (as ngd_line_search) with the decisions on the device: each round
// evaluates the next trial steps of every member still searching (side by side on the batch's
// streams) and the host reads back only which members are done, once per round for all of them. The
// accepted step does not depend on how the trials are grouped into launches.
ngd_status ngd_batch_line_search(ngd_batch* b, void* const* theta, double* const* d, double* const* grad,
                                 const double* loss0, double c1, int32_t max_halvings, void* const* theta_out,
                                 double* alpha, double* loss_new, void* stream) {
  NGD_CHECK(b != nullptr && theta && d && grad && loss0 && theta_out && alpha && loss_new, "NULL argument");
  NGD_CHECK(max_halvings >= 0 && c1 >= 0.0, "max_halvings >= 0 and c1 >= 0 required");
  const int n = (int)b->inst.size();
  for (int i = 0; i < n; ++i)
    NGD_CHECK(theta[i] && d[i] && grad[i] && theta_out[i] && std::isfinite(loss0[i]), "bad argument of a problem");
  NGD_TRY(batch_streams(b));
  hipStream_t s = S(stream);
  auto fork = [&] {
    NGD_HIP_TRY(hipEventRecord(b->sk_fork, s));
    for (int q = 0; q < ngd_batch::kSketchStreams; ++q)
      NGD_HIP_TRY(hipStreamWaitEvent(b->sk_stream[q], b->sk_fork, 0));
    return NGD_OK;
  };
  auto join = [&] {
    for (int q = 0; q < ngd_batch::kSketchStreams; ++q) {
      NGD_HIP_TRY(hipEventRecord(b->sk_join[q], b->sk_stream[q]));
      NGD_HIP_TRY(hipStreamWaitEvent(s, b->sk_join[q], 0));
    }
    return NGD_OK;
  };
  // per member: the slope grad^T d, a cleared decision [found, alpha, loss, index] at scal + 100
  NGD_TRY(fork());
  for (int i = 0; i < n; ++i) {
    ngd_problem* h = b->inst[i];
    hipStream_t qs = b->sk_stream[i % ngd_batch::kSketchStreams];
    NGD_TRY(launch_dot(grad[i], d[i], h->P, h->scal + 8, h->scal + 0, qs));
    NGD_TRY(launch_zero(h->scal + 100, sizeof(double) * 4, qs));
  }
  std::vector<int> tried(n, 0), active(n);
  for (int i = 0; i < n; ++i) active[i] = i;
  double* hst = b->h_ls;
  bool first = true;
  while (!active.empty()) {
    for (int i : active) {
      ngd_problem* h = b->inst[i];
      hipStream_t qs = b->sk_stream[i % ngd_batch::kSketchStreams];
      const int batch = first ? h->ls_first_batch : h->ls_batch;
      const int nt = std::min(batch, max_halvings + 1 - tried[i]);
      double* ha = reinterpret_cast<double*>(h->host) + 8;  // this member's pinned staging of the steps
      for (int t = 0; t < nt; ++t) ha[t] = std::ldexp(1.0, -(tried[i] + t));
      NGD_HIP_TRY(hipMemcpyAsync(h->alphas, ha, sizeof(double) * nt, hipMemcpyHostToDevice, qs));
      NGD_TRY(launch_axpy_theta(h->dtype, theta[i], d[i], h->alphas, nt, h->P, h->trial, h->ldP, qs));
      const int nb = residual_blocks(h->net, h->dtype, h->N, false);
      NGD_CHECK(nb <= h->res_blocks, "residual launch exceeds its loss-partial buffer");
      NGD_TRY(launch_residual_jacobian(h->net, h->dtype, h->trial, h->N, h->X, h->w, h->f, h->g, h->kind, nullptr,
                                       nullptr, 0, h->loss_part, h->ldP, nt, qs, nullptr));
      NGD_TRY(launch_reduce_sum(h->loss_part, nb, nt, 0.5, h->losses, qs));
      NGD_TRY(launch_armijo(h->alphas, h->losses, h->scal + 0, loss0[i], c1, nt, tried[i], h->scal + 100, qs));
      NGD_HIP_TRY(hipMemcpyAsync(hst + 4 * (size_t)i, h->scal + 100, sizeof(double) * 4, hipMemcpyDeviceToHost, qs));
      tried[i] += nt;
    }
    NGD_TRY(join());
    NGD_HIP_TRY(hipStreamSynchronize(s));
    std::vector<int> next;
    for (int i : active)
      if (hst[4 * (size_t)i] == 0.0 && tried[i] <= max_halvings) next.push_back(i);
    active.swap(next);
    first = false;
    if (!active.empty()) NGD_TRY(fork());
  }
  // theta_out = theta - alpha d with the accepted alpha (0 when none was: theta_out = theta)
  NGD_TRY(fork());
  for (int i = 0; i < n; ++i) {
    ngd_problem* h = b->inst[i];
    hipStream_t qs = b->sk_stream[i % ngd_batch::kSketchStreams];
    const bool found = hst[4 * (size_t)i] != 0.0;
    alpha[i] = found ? hst[4 * (size_t)i + 1] : 0.0;
    loss_new[i] = found ? hst[4 * (size_t)i + 2] : loss0[i];
    h->ls_first_batch = found && hst[4 * (size_t)i + 3] == 0.0 ? 1 : h->ls_batch;
    NGD_TRY(launch_axpy_theta(h->dtype, theta[i], d[i], nullptr, 1, h->P, theta_out[i], h->ldP, qs, alpha[i]));
  }
  NGD_TRY(join());
  NGD_HIP_TRY(hipStreamSynchronize(s));
  return NGD_OK;
}

// Average time of one batched matvec launch (the PCG iteration's one pass over every J_w) on the
// directions of the last batched solve, from HIP events around `reps` launches on `stream`.
ngd_status ngd_batch_matvec_time(ngd_batch* b, int32_t reps, double* avg_ms, void* stream) {
  NGD_CHECK(b != nullptr && avg_ms != nullptr && reps >= 1, "NULL argument or reps < 1");
  NGD_CHECK(b->rows_target != 0, "no batched solve has run yet");
  hipStream_t s = S(stream);
  int rows, upd, dots, elem, apply;
  batch_pcg_items(b, &rows, &upd, &dots, &elem, &apply);
  int64_t max_ld = 0;
  for (size_t i = 0; i < b->inst.size(); ++i) max_ld = std::max<int64_t>(max_ld, b->h_pcg[i].ldJ);
  const int n = (int)b->inst.size();
  // the solve left every state done, and a done state skips its rows: clear the flags for the timed
  // launches (they rewrite only the direction slot, its norm and the partial sums, which the next
  // solve initialises again) and restore them afterwards
  NGD_HIP_TRY(hipStreamSynchronize(s));
  std::vector<int> done(n);
  for (int i = 0; i < n; ++i) {
    done[i] = b->h_states[i].done;
    b->h_states[i].done = 0;
  }
  NGD_HIP_TRY(hipMemcpyAsync(b->d_states, b->h_states, sizeof(PcgState) * n, hipMemcpyHostToDevice, s));
  hipEvent_t e0, e1;
  NGD_HIP_TRY(hipEventCreate(&e0));
  NGD_HIP_TRY(hipEventCreate(&e1));
  NGD_HIP_TRY(hipEventRecord(e0, s));
  for (int r = 0; r < reps; ++r) NGD_TRY(pcg_batch_launch_rows(b->dtype, b->d_pcg, n, rows, max_ld, s));
  NGD_HIP_TRY(hipEventRecord(e1, s));
  NGD_HIP_TRY(hipEventSynchronize(e1));
  float ms = 0.f;
  NGD_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  for (int i = 0; i < n; ++i) b->h_states[i].done = done[i];
  NGD_HIP_TRY(hipMemcpyAsync(b->d_states, b->h_states, sizeof(PcgState) * n, hipMemcpyHostToDevice, s));
  NGD_HIP_TRY(hipStreamSynchronize(s));
  *avg_ms = ms / reps;
  return NGD_OK;
}


}  // extern "C"
