// extern "C" entry points of libsdgp.so (declared in include/sdgp.h).
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "sdgp_internal.hpp"

struct sdgp_ctx : sdgp::Ctx {};

// Static device workspace of sdgp_lml_grad_noalloc: every device the library
// runs on holds one copy until the process ends.  In host code `scratch` is
// only the host-side stand-in of the symbol; its device address comes from
// hipGetSymbolAddress (kept per device in g_scratch) and only that address
// is ever passed to kernels or copies.
constexpr size_t kScratchBytes = size_t(256) << 20;
constexpr int64_t kNoAllocMaxN = 65535;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;                     // guards g_scratch
char* g_scratch[kMaxDevices] = {};           // device address of `scratch` per device
std::mutex g_scratch_call_mu[kMaxDevices];   // serialises static-workspace calls per device

// Resolves the device address of the static workspace on the current
// device (once per device).
sdgp_status resolve_scratch(int device, std::string* err) {
  if (device < 0 || device >= kMaxDevices) return SDGP_OK;   // the static-workspace call then refuses
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch[device]) return SDGP_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || p == nullptr) {
    *err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
    return SDGP_ERR_HIP;
  }
  g_scratch[device] = static_cast<char*>(p);
  return SDGP_OK;
}
}  // namespace

namespace sdgp {

void Ctx::release_all() {
  for (auto& b : buf)
    if (b.p) { (void)hipFree(b.p); b.p = nullptr; b.bytes = 0; }
  for (auto e : ev_pool) (void)hipEventDestroy(e);
  ev_pool.clear();
  if (gstream) { (void)hipStreamDestroy(gstream); gstream = nullptr; }
  held_bytes = 0;
  ev_used = 0;
}

namespace {

thread_local std::string g_create_error;

template <class F>
sdgp_status guarded(sdgp_ctx* ctx, F&& f) {
  if (!ctx) return SDGP_ERR_INVALID_ARG;
  try {
    SDGP_HIP(hipSetDevice(ctx->device));
    ctx->ev_used = 0;
    f();
    ctx->err.clear();
    return SDGP_OK;
  } catch (const Error& e) {
    ctx->err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    ctx->err = "host allocation failed";
    return SDGP_ERR_OOM;
  } catch (const std::exception& e) {
    ctx->err = e.what();
    return SDGP_ERR_HIP;
  } catch (...) {
    ctx->err = "unknown failure";
    return SDGP_ERR_HIP;
  }
}

// Phases shared by every evaluation on one hyperparameter vector.
struct Assembled {
  KParams kp;
  Bumps b;
  Csr A;
  int64_t candidates = 0;
};

Assembled assemble_all(Ctx* c, const Sorted& s, const sdgp_kernel_desc& d, const double* h, bool add_noise,
                       PhaseTimer* t, bool core_only = false, const CsrOut* out = nullptr) {
  Assembled r;
  r.kp = make_params(d, h);
  r.b = bump_precompute(c, s, r.kp, h);
  if (t) t->mark(2);
  int32_t* iv_ptr;
  int2* iv;
  prune(c, s, r.kp, r.b, &iv_ptr, &iv, core_only);
  if (t) t->mark(3);
  r.A = assemble_sorted(c, s, r.kp, r.b, iv_ptr, iv, add_noise, &r.candidates, t, core_only, out);
  if (t) t->mark(5);
  return r;
}

void check_estimator(const sdgp_estimator* e, int64_t n) {
  require(e != nullptr, "estimator is NULL");
  require(e->kind == SDGP_PROBE_RADEMACHER || e->kind == SDGP_PROBE_IDENTITY, "unknown probe kind");
  if (e->kind == SDGP_PROBE_RADEMACHER) require(e->probes >= 1 && e->probes <= 64, "probes must be 1..64");
  if (e->kind == SDGP_PROBE_IDENTITY) require(n <= 16384, "identity probes need n <= 16384");
  require(e->cg_max_iter >= 1, "cg_max_iter must be >= 1");
  require(e->cg_rtol > 0.0 && std::isfinite(e->cg_rtol), "cg_rtol must be > 0");
  require(e->probe_rtol >= 0.0 && std::isfinite(e->probe_rtol), "probe_rtol must be >= 0");
  require(e->lanczos_steps >= 0, "lanczos_steps must be >= 0");
  require(e->precond == SDGP_PRECOND_NONE || e->precond == SDGP_PRECOND_LOWRANK, "unknown preconditioner");
  require(e->operator_form == SDGP_OPERATOR_ASSEMBLED || e->operator_form == SDGP_OPERATOR_FACTORED,
          "unknown operator form");
  if (e->precond == SDGP_PRECOND_LOWRANK)
    require(e->kind == SDGP_PROBE_RADEMACHER, "the low-rank preconditioner needs Rademacher probes");
  if (e->operator_form == SDGP_OPERATOR_FACTORED)
    require(e->precond == SDGP_PRECOND_LOWRANK, "the factored operator needs the low-rank preconditioner");
}

void finish_timing(Ctx* c, PhaseTimer& t, sdgp_info* info) {
  if (!c->timing || !info) return;
  SDGP_HIP(hipStreamSynchronize(c->stream));
  for (int k = 0; k < 8; ++k) {
    info->ms[k] = 0.0;
    if (t.set[k] && t.set[k + 1]) {
      float ms = 0.0f;
      SDGP_HIP(hipEventElapsedTime(&ms, t.marks[k], t.marks[k + 1]));
      info->ms[k] = ms;
    }
  }
  double tot = 0.0;
  for (auto& pr : c->spmm_events) {
    float ms = 0.0f;
    SDGP_HIP(hipEventElapsedTime(&ms, pr.first, pr.second));
    tot += ms;
  }
  info->spmm_ms = tot;
  info->spmm_launches = (int64_t)c->spmm_events.size();
}

// One LML (+ gradient) evaluation on points already ordered.
sdgp_status evaluate(Ctx* c, const Sorted& s, const double* ys, const sdgp_kernel_desc& d, const double* h,
                     const sdgp_estimator& e, double* lml_out, double* grad_out, sdgp_info* info,
                     PhaseTimer& t) {
  const bool factored = e.operator_form == SDGP_OPERATOR_FACTORED;
  if (factored) require(d.combine == SDGP_COMBINE_SUM, "the factored operator needs the SUM combine");
  Assembled as = assemble_all(c, s, d, h, true, &t, factored);
  const int kind = e.kind == SDGP_PROBE_IDENTITY ? PK_IDENTITY : PK_RADEMACHER;
  const int P = kind == PK_IDENTITY ? (int)s.n : e.probes;
  Precond pc;
  const bool use_pc = e.precond == SDGP_PRECOND_LOWRANK;
  if (use_pc) {
    require(d.combine == SDGP_COMBINE_SUM, "the low-rank preconditioner needs the SUM combine");
    pc = lowrank_precond(c, s, as.kp, as.b);
    pc.lowrank_op = factored ? 1 : 0;
  }
  CgResult cg = block_cg(c, as.A, s, ys, kind, P, e.seed, e.cg_rtol, e.cg_max_iter, nullptr, 0,
                         use_pc ? &pc : nullptr, grad_out != nullptr, &t,
                         kind == PK_RADEMACHER ? e.probe_rtol : 0.0);
  if (cg.not_spd) throw Error(SDGP_ERR_NOT_SPD, "CG met p^T A p <= 0: the covariance is not positive definite");
  t.mark(6);
  const double yKy = dot_device(c, ys, 1, cg.X, cg.R, s.n);
  double logdet = 0.0, se = 0.0, rmin = 0.0, rmax = 0.0;
  slq_from_cg(c, cg, kind, P, s.n, e.lanczos_steps, &logdet, &se, &rmin, &rmax);
  t.mark(7);
  if (lml_out) *lml_out = -0.5 * yKy - 0.5 * logdet;
  if (grad_out) adjoint_gradient(c, s, as.kp, as.b, as.A, cg, kind, P, e.seed, h, grad_out, factored);
  t.mark(8);
  if (info) {
    info->nnz = as.A.nnz;
    info->candidates = as.candidates;
    info->cg_iters = cg.iters;
    info->cg_iters_y = cg.iters_y;
    info->cg_relres_max = cg.relres_max;
    info->yKy = yKy;
    info->logdet = logdet;
    info->logdet_stderr = se;
    info->ritz_min = rmin;
    info->ritz_max = rmax;
  }
  finish_timing(c, t, info);
  return cg.converged ? SDGP_OK : SDGP_ERR_NOT_CONVERGED;
}

}  // namespace
}  // namespace sdgp

using namespace sdgp;

extern "C" {

sdgp_status sdgp_create(sdgp_ctx** out, int device, void* hip_stream) {
  if (!out) return SDGP_ERR_INVALID_ARG;
  *out = nullptr;
  try {
    int count = 0;
    SDGP_HIP(hipGetDeviceCount(&count));
    require(device >= 0 && device < count, "no such HIP device");
    SDGP_HIP(hipSetDevice(device));
    std::string serr;
    if (resolve_scratch(device, &serr) != SDGP_OK) throw Error(SDGP_ERR_HIP, serr);
    sdgp_ctx* c = new sdgp_ctx();
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
      c->cu_count = prop.multiProcessorCount;
      std::string a(prop.gcnArchName);
      c->arch = a.substr(0, a.find(':'));
    }
    if (c->arch.empty()) c->arch = "unknown";
    *out = c;
    return SDGP_OK;
  } catch (const Error& e) {
    g_create_error = e.what();
    return e.code;
  } catch (const std::exception& e) {
    g_create_error = e.what();
    return SDGP_ERR_HIP;
  }
}

void sdgp_destroy(sdgp_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  ctx->release_all();
  delete ctx;
}

const char* sdgp_last_error(const sdgp_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

sdgp_status sdgp_set_timing(sdgp_ctx* ctx, int enable) {
  if (!ctx) return SDGP_ERR_INVALID_ARG;
  ctx->timing = enable != 0;
  return SDGP_OK;
}

int64_t sdgp_num_hyper(const sdgp_kernel_desc* d) {
  if (!d || d->dim < 1 || d->dim > kMaxDim || d->n1 < 0 || d->n1 > kMaxN1 || (d->n1 > 0 && d->n2 < 1))
    return -1;
  return 2 + (int64_t)d->n1 * d->n2 * (3 + d->dim) + 1;
}

sdgp_status sdgp_kernel_nnz(sdgp_ctx* ctx, const sdgp_kernel_desc* desc, const double* x, int64_t n,
                            const double* h, int64_t* nnz_out) {
  return guarded(ctx, [&] {
    require(desc && x && nnz_out, "NULL argument");
    validate(*desc, h, n);
    Sorted s = order_points(ctx, x, n, desc->dim, h[1], false);
    Assembled as = assemble_all(ctx, s, *desc, h, true, nullptr);
    *nnz_out = as.A.nnz;
  });
}

sdgp_status sdgp_kernel_assemble(sdgp_ctx* ctx, const sdgp_kernel_desc* desc, const double* x, int64_t n,
                                 const double* h, int add_noise, int64_t* row_ptr, int32_t* col, double* val,
                                 int64_t capacity, int64_t* nnz_out) {
  sdgp_status st = guarded(ctx, [&] {
    require(desc && x && nnz_out && row_ptr, "NULL argument");
    validate(*desc, h, n);
    Sorted s = order_points(ctx, x, n, desc->dim, h[1], false);
    Assembled as = assemble_all(ctx, s, *desc, h, add_noise != 0, nullptr);
    *nnz_out = as.A.nnz;
    if (as.A.nnz > capacity) throw Error(SDGP_ERR_CAPACITY, "capacity smaller than nnz");
    require(col && val, "NULL col/val");
    canonicalize(ctx, s, as.A, row_ptr, col, val);
    SDGP_HIP(hipStreamSynchronize(ctx->stream));
  });
  return st;
}

sdgp_status sdgp_kernel_assemble_sorted(sdgp_ctx* ctx, const sdgp_kernel_desc* desc, const double* x, int64_t n,
                                        const double* h, int add_noise, int64_t* row_ptr, int32_t* col,
                                        double* val, int32_t* perm, int64_t capacity, int64_t* nnz_out) {
  return guarded(ctx, [&] {
    require(desc && x && nnz_out && row_ptr && perm, "NULL argument");
    validate(*desc, h, n);
    Sorted s = order_points(ctx, x, n, desc->dim, h[1], false);
    // the count's scan and the fill write the caller's arrays directly
    const CsrOut out{row_ptr, col, val, (col && val) ? capacity : -1};
    Assembled as = assemble_all(ctx, s, *desc, h, add_noise != 0, nullptr, false, &out);
    *nnz_out = as.A.nnz;
    if (as.A.nnz > capacity) throw Error(SDGP_ERR_CAPACITY, "capacity smaller than nnz");
    require(col && val, "NULL col/val");
    SDGP_HIP(hipMemcpyAsync(perm, s.perm, n * sizeof(int32_t), hipMemcpyDeviceToDevice, ctx->stream));
    SDGP_HIP(hipStreamSynchronize(ctx->stream));
  });
}

sdgp_status sdgp_csr_spmm(sdgp_ctx* ctx, int64_t n, const int64_t* row_ptr, const int32_t* col,
                          const double* val, const double* X, int32_t R, double* Y) {
  return guarded(ctx, [&] {
    require(row_ptr && col && val && X && Y, "NULL argument");
    require(n >= 1, "n must be >= 1");
    Csr A;
    A.n = n; A.nnz = -1;
    A.row_ptr = const_cast<int64_t*>(row_ptr);
    A.col = const_cast<int32_t*>(col);
    A.val = const_cast<double*>(val);
    spmm(ctx, A, X, R, Y);
  });
}

static sdgp_status lml_common(sdgp_ctx* ctx, const sdgp_kernel_desc* desc, const double* x, const double* y,
                              int64_t n, const double* h, const sdgp_estimator* est, double* lml_out,
                              double* grad_out, sdgp_info* info) {
  sdgp_status inner = SDGP_OK;
  sdgp_status st = guarded(ctx, [&] {
    require(desc && x && y && lml_out, "NULL argument");
    validate(*desc, h, n);
    check_estimator(est, n);
    if (info) std::memset(info, 0, sizeof(*info));
    PhaseTimer t(ctx);
    t.mark(0);
    Sorted s = order_points(ctx, x, n, desc->dim, h[1]);
    double* ys = ctx->get<double>(S_YS, n);
    gather_vector(ctx, s, y, ys);
    t.mark(1);
    inner = evaluate(ctx, s, ys, *desc, h, *est, lml_out, grad_out, info, t);
  });
  if (st != SDGP_OK) return st;
  if (inner == SDGP_ERR_NOT_CONVERGED) ctx->err = "CG did not reach cg_rtol within cg_max_iter";
  return inner;
}

sdgp_status sdgp_lml(sdgp_ctx* ctx, const sdgp_kernel_desc* desc, const double* x, const double* y, int64_t n,
                     const double* h, const sdgp_estimator* est, double* lml_out, sdgp_info* info) {
  return lml_common(ctx, desc, x, y, n, h, est, lml_out, nullptr, info);
}

sdgp_status sdgp_lml_grad(sdgp_ctx* ctx, const sdgp_kernel_desc* desc, const double* x, const double* y,
                          int64_t n, const double* h, const sdgp_estimator* est, double* lml_out,
                          double* grad_out, sdgp_info* info) {
  if (!grad_out) return SDGP_ERR_INVALID_ARG;
  return lml_common(ctx, desc, x, y, n, h, est, lml_out, grad_out, info);
}

sdgp_status sdgp_lml_grad_noalloc(sdgp_ctx* ctx, const sdgp_kernel_desc* desc, const double* x, const double* y,
                                  int64_t n, const double* h, const sdgp_estimator* est, double* lml_out,
                                  double* grad_out, sdgp_info* info) {
  if (!ctx) return SDGP_ERR_INVALID_ARG;
  if (!grad_out) {
    ctx->err = "grad_out is NULL";
    return SDGP_ERR_INVALID_ARG;
  }
  if (n > kNoAllocMaxN) {
    ctx->err = "sdgp_lml_grad_noalloc takes at most " + std::to_string(kNoAllocMaxN) + " points";
    return SDGP_ERR_INVALID_ARG;
  }
  const int dev = ctx->device;
  char* base = (dev >= 0 && dev < kMaxDevices) ? g_scratch[dev] : nullptr;
  if (!base) {
    ctx->err = "no static workspace on this device";
    return SDGP_ERR_HIP;
  }
  std::lock_guard<std::mutex> lk(g_scratch_call_mu[dev]);
  const bool timing = ctx->timing, graph = ctx->use_graph;
  ctx->timing = false;     // events and graphs would allocate
  ctx->use_graph = false;
  ctx->arena = base;
  ctx->arena_cap = kScratchBytes;
  ctx->arena_used = 0;
  for (auto& a : ctx->abuf) a = DevBuf{};
  sdgp_status st = lml_common(ctx, desc, x, y, n, h, est, lml_out, grad_out, info);
  // the next call may reuse the workspace only after this call's device work
  const hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess && st == SDGP_OK) {
    ctx->err = std::string("hipStreamSynchronize: ") + hipGetErrorString(e);
    st = SDGP_ERR_HIP;
  }
  ctx->arena = nullptr;
  ctx->arena_cap = 0;
  ctx->arena_used = 0;
  for (auto& a : ctx->abuf) a = DevBuf{};
  ctx->timing = timing;
  ctx->use_graph = graph;
  return st;
}

sdgp_status sdgp_lml_grad_batched(sdgp_ctx* ctx, const sdgp_kernel_desc* desc, const double* x, const double* y,
                                  int64_t n, const double* H, int32_t B, const sdgp_estimator* est,
                                  double* lml_out, double* grad_out, int32_t* member_status, sdgp_info* info) {
  return guarded(ctx, [&] {
    require(desc && x && y && H && lml_out && grad_out && member_status, "NULL argument");
    require(B >= 1 && B <= 65535, "B must be in 1..65535");
    const int64_t nh = sdgp_num_hyper(desc);
    require(nh > 0, "invalid kernel descriptor");
    check_estimator(est, n);
    validate_shape(*desc, n);
    // The factored operator is not available for populations: a device
    // memory fault met by an earlier version of this path has no shown
    // cause, so the combination is rejected rather than run.
    require(est->operator_form != SDGP_OPERATOR_FACTORED,
            "the factored operator is not available for populations (use SDGP_OPERATOR_ASSEMBLED)");
    const bool factored = false;
    const bool use_pc = est->precond == SDGP_PRECOND_LOWRANK;
    if (use_pc) require(desc->combine == SDGP_COMBINE_SUM, "the low-rank preconditioner needs SUM");
    const int kind = est->kind == SDGP_PROBE_IDENTITY ? PK_IDENTITY : PK_RADEMACHER;
    const int P = kind == PK_IDENTITY ? (int)n : est->probes;
    // shared ordering: the cell side must cover every member's core radius
    double rmax = 0.0;
    for (int m = 0; m < B; ++m) {
      const double r = H[(int64_t)m * nh + 1];
      if (std::isfinite(r) && r > rmax) rmax = r;
    }
    require(rmax > 0.0, "no member has a valid core radius");
    PhaseTimer t0(ctx);
    Sorted s = order_points(ctx, x, n, desc->dim, rmax);
    double* ys = ctx->get<double>(S_YS, n);
    gather_vector(ctx, s, y, ys);
    // validate every member; the valid ones are assembled together, every
    // assembly phase one launch with the member as grid z
    std::vector<int> idx;
    std::vector<const double*> hv;
    for (int m = 0; m < B; ++m) {
      const double* hm = H + (int64_t)m * nh;
      if (info) std::memset(info + m, 0, sizeof(sdgp_info));
      lml_out[m] = NAN;
      for (int64_t k = 0; k < nh; ++k) grad_out[(int64_t)m * nh + k] = NAN;
      try {
        validate(*desc, hm, n);
        idx.push_back(m);
        hv.push_back(hm);
        member_status[m] = SDGP_OK;
      } catch (const Error& e) {
        member_status[m] = e.code;
      }
    }
    if (idx.empty()) return;
    std::vector<PopAssembled> pop = assemble_population(ctx, s, *desc, hv, true);
    std::vector<Precond> pcs;
    std::vector<std::string> pc_failed(pop.size());
    if (use_pc) {
      std::vector<KParams> kps;
      for (const auto& p : pop) kps.push_back(p.kp);
      pcs = lowrank_precond_pop(ctx, s, kps, pop[0].b.F, &pc_failed);
    }
    struct Member {
      int idx;
      KParams kp;
      Bumps b;
      Csr A;
      Precond pc;
      int64_t candidates;
    };
    std::vector<Member> mem;
    for (size_t q = 0; q < pop.size(); ++q) {
      if (!pc_failed[q].empty()) {
        member_status[idx[q]] = SDGP_ERR_INVALID_ARG;
        continue;
      }
      Member mb;
      mb.idx = idx[q];
      mb.kp = pop[q].kp;
      mb.b = pop[q].b;
      mb.A = pop[q].A;
      if (use_pc) mb.pc = pcs[q];
      mb.candidates = pop[q].candidates;
      mem.push_back(mb);
    }
    if (mem.empty()) return;
    // one batched (preconditioned) CG for every valid member
    std::vector<CgMember> cm(mem.size());
    for (size_t q = 0; q < mem.size(); ++q) {
      cm[q].A = mem[q].A;
      cm[q].pc = use_pc ? &mem[q].pc : nullptr;
    }
    std::vector<CgResult> res = block_cg_multi(ctx, cm, s, ys, kind, P, est->seed, est->cg_rtol, est->cg_max_iter,
                                               nullptr, 0, true, ctx->use_graph,
                                               kind == PK_RADEMACHER ? est->probe_rtol : 0.0);
    for (size_t q = 0; q < mem.size(); ++q) {
      const Member& mb = mem[q];
      const int m = mb.idx;
      const double* hm = H + (int64_t)m * nh;
      try {
        const CgResult& cg = res[q];
        if (cg.not_spd) throw Error(SDGP_ERR_NOT_SPD, "CG met p^T A p <= 0");
        const double yKy = dot_device(ctx, ys, 1, cg.X, cg.R, s.n);
        double logdet = 0.0, se = 0.0, rmin = 0.0, rmax2 = 0.0;
        slq_from_cg(ctx, cg, kind, P, s.n, est->lanczos_steps, &logdet, &se, &rmin, &rmax2);
        lml_out[m] = -0.5 * yKy - 0.5 * logdet;
        adjoint_gradient(ctx, s, mb.kp, mb.b, mb.A, cg, kind, P, est->seed, hm, grad_out + (int64_t)m * nh,
                         factored);
        if (info) {
          sdgp_info& I = info[m];
          I.nnz = mb.A.nnz;
          I.candidates = mb.candidates;
          I.cg_iters = cg.iters;
          I.cg_iters_y = cg.iters_y;
          I.cg_relres_max = cg.relres_max;
          I.yKy = yKy;
          I.logdet = logdet;
          I.logdet_stderr = se;
          I.ritz_min = rmin;
          I.ritz_max = rmax2;
        }
        member_status[m] = cg.converged ? SDGP_OK : SDGP_ERR_NOT_CONVERGED;
      } catch (const Error& e) {
        member_status[m] = e.code;
        lml_out[m] = NAN;
        for (int64_t k = 0; k < nh; ++k) grad_out[(int64_t)m * nh + k] = NAN;
        if (e.code == SDGP_ERR_HIP || e.code == SDGP_ERR_OOM) throw;
      }
    }
    (void)t0;
  });
}

sdgp_status sdgp_set_option(sdgp_ctx* ctx, const char* name, int64_t value) {
  if (!ctx || !name) return SDGP_ERR_INVALID_ARG;
  const std::string k(name);
  if (k == "timing") { ctx->timing = value != 0; return SDGP_OK; }
  if (k == "graph") { ctx->use_graph = value != 0; return SDGP_OK; }
  if (k == "union_spmm") {
    if (value < -1 || value > 1) { ctx->err = "union_spmm must be -1, 0 or 1"; return SDGP_ERR_INVALID_ARG; }
    ctx->union_spmm = (int)value;
    return SDGP_OK;
  }
  if (k == "fw_mfma") {
    if (value < -1 || value > 1) { ctx->err = "fw_mfma must be -1, 0 or 1"; return SDGP_ERR_INVALID_ARG; }
    ctx->fw_mfma = (int)value;
    return SDGP_OK;
  }
  if (k == "spmm_blocks") {
    if (value < 0 || value > 65535 || value % 8 != 0) {
      ctx->err = "spmm_blocks must be 0 (default) or a multiple of 8 up to 65535";
      return SDGP_ERR_INVALID_ARG;
    }
    ctx->spmm_blocks = (int)value;
    return SDGP_OK;
  }
  if (k == "autotune") {
    if (value < 0 || value > 2) { ctx->err = "autotune must be 0, 1 or 2"; return SDGP_ERR_INVALID_ARG; }
    ctx->autotune = (int)value;
    return SDGP_OK;
  }
  if (k == "workspace_cap") {
    if (value < 0) { ctx->err = "workspace_cap must be >= 0 (0: no cap)"; return SDGP_ERR_INVALID_ARG; }
    ctx->cap_bytes = (size_t)value;
    return SDGP_OK;
  }
  if (k == "update_blocks") {
    if (value < 0 || value > 65535) { ctx->err = "update_blocks must be 0 (default) .. 65535"; return SDGP_ERR_INVALID_ARG; }
    ctx->update_blocks = (int)value;
    return SDGP_OK;
  }
  ctx->err = "unknown option '" + k + "'";
  return SDGP_ERR_INVALID_ARG;
}

sdgp_status sdgp_get_option(const sdgp_ctx* ctx, const char* name, int64_t* value) {
  if (!ctx || !name || !value) return SDGP_ERR_INVALID_ARG;
  const std::string k(name);
  if (k == "timing") *value = ctx->timing ? 1 : 0;
  else if (k == "graph") *value = ctx->use_graph ? 1 : 0;
  else if (k == "last_y_tail") *value = ctx->last_y_tail;
  else if (k == "union_spmm") *value = ctx->union_spmm;
  else if (k == "fw_mfma") *value = ctx->fw_mfma;
  else if (k == "spmm_blocks") *value = ctx->spmm_blocks;
  else if (k == "update_blocks") *value = ctx->update_blocks;
  else if (k == "autotune") *value = ctx->autotune;
  else if (k == "workspace_cap") *value = (int64_t)ctx->cap_bytes;
  else if (k == "last_spmm_blocks") *value = ctx->last_shape.spmm_blocks;
  else if (k == "last_update_blocks") *value = ctx->last_shape.update_blocks;
  else if (k == "last_union_spmm") *value = ctx->last_shape.union_spmm;
  else if (k == "last_fw_mfma") *value = ctx->last_shape.fw_mfma;
  else if (k == "last_tuned") *value = ctx->last_tuned;
  else return SDGP_ERR_INVALID_ARG;
  return SDGP_OK;
}

sdgp_status sdgp_posterior_mean_var(sdgp_ctx* ctx, const sdgp_kernel_desc* desc, const double* x,
                                    const double* y, int64_t n, const double* h, const double* x0, int64_t n0,
                                    const sdgp_estimator* est, double* mean_out, double* var_out) {
  bool conv = true;
  sdgp_status st = guarded(ctx, [&] {
    require(desc && x && y && x0 && mean_out && var_out && est, "NULL argument");
    validate(*desc, h, n);
    require(est->cg_max_iter >= 1 && est->cg_rtol > 0.0 && std::isfinite(est->cg_rtol), "bad CG options");
    Sorted s = order_points(ctx, x, n, desc->dim, h[1]);
    double* ys = ctx->get<double>(S_YS, n);
    gather_vector(ctx, s, y, ys);
    Assembled as = assemble_all(ctx, s, *desc, h, true, nullptr);
    double* kxx = nullptr;
    Csr K0 = assemble_cross(ctx, s, as.kp, as.b, x0, n0, h, &kxx);
    Precond pc;
    const bool use_pc = est->precond == SDGP_PRECOND_LOWRANK && desc->combine == SDGP_COMBINE_SUM;
    if (use_pc) pc = lowrank_precond(ctx, s, as.kp, as.b);
    CgResult cg = block_cg(ctx, as.A, s, ys, PK_NONE, 0, 0, est->cg_rtol, est->cg_max_iter, nullptr, 0,
                           use_pc ? &pc : nullptr, false, nullptr);
    if (cg.not_spd) throw Error(SDGP_ERR_NOT_SPD, "CG met p^T A p <= 0: the covariance is not positive definite");
    conv = cg.converged;
    spmm(ctx, K0, cg.X, 1, mean_out);
    bool c2 = true;
    posterior_variance(ctx, as.A, s, K0, kxx, est->cg_rtol, est->cg_max_iter, use_pc ? &pc : nullptr, var_out,
                       &c2);
    conv = conv && c2;
    SDGP_HIP(hipStreamSynchronize(ctx->stream));
  });
  if (st != SDGP_OK) return st;
  if (!conv) {
    ctx->err = "CG did not reach cg_rtol within cg_max_iter";
    return SDGP_ERR_NOT_CONVERGED;
  }
  return SDGP_OK;
}

sdgp_status sdgp_logdet_taylor(sdgp_ctx* ctx, const sdgp_kernel_desc* desc, const double* x, int64_t n,
                               const double* h, int32_t probes, int32_t terms, uint64_t seed, double* logdet_out,
                               double* alpha_out) {
  return guarded(ctx, [&] {
    require(desc && x && logdet_out && alpha_out, "NULL argument");
    validate(*desc, h, n);
    Sorted s = order_points(ctx, x, n, desc->dim, h[1]);
    Assembled as = assemble_all(ctx, s, *desc, h, true, nullptr);
    *logdet_out = logdet_taylor(ctx, as.A, s, probes, terms, seed, alpha_out);
  });
}

sdgp_status sdgp_sparsity_bound(const sdgp_kernel_desc* desc, const double* h, double domain_volume,
                                double* s_out) {
  if (!desc || !h || !s_out) return SDGP_ERR_INVALID_ARG;
  if (sdgp_num_hyper(desc) < 0 || !(domain_volume > 0.0) || !std::isfinite(domain_volume))
    return SDGP_ERR_INVALID_ARG;
  const int d = desc->dim;
  const double unit = std::pow(M_PI, d / 2.0) / std::tgamma(d / 2.0 + 1.0);
  double tot = 0.0;
  for (int i = 0; i < desc->n1; ++i)
    for (int j = 0; j < desc->n2; ++j) {
      const double rj = h[2 + (int64_t)(i * desc->n2 + j) * (3 + d) + 2];
      if (!(rj > 0.0) || !std::isfinite(rj)) return SDGP_ERR_INVALID_ARG;
      for (int k = 0; k < desc->n2; ++k) {
        const double rk = h[2 + (int64_t)(i * desc->n2 + k) * (3 + d) + 2];
        if (!(rk > 0.0) || !std::isfinite(rk)) return SDGP_ERR_INVALID_ARG;
        tot += unit * std::pow(rj, d) * unit * std::pow(rk, d);
      }
    }
  *s_out = tot / (domain_volume * domain_volume);
  return SDGP_OK;
}

sdgp_status sdgp_sparsity_objective(double lml, double s, double requirement, double* augmented_out,
                                    int32_t* feasible_out) {
  if (!augmented_out || !feasible_out) return SDGP_ERR_INVALID_ARG;
  if (!std::isfinite(lml) || !std::isfinite(s)) return SDGP_ERR_INVALID_ARG;
  *augmented_out = lml + (1.0 - s) * lml;
  *feasible_out = s < requirement ? 1 : 0;
  return SDGP_OK;
}

sdgp_status sdgp_de_trials(int32_t B, int32_t nh, const double* H, const double* lo, const double* hi, double F,
                           double CR, uint64_t seed, uint64_t generation, double* T) {
  try {
    de_trials(B, nh, H, lo, hi, F, CR, seed, generation, T);
    return SDGP_OK;
  } catch (const Error& e) {
    return (sdgp_status)e.code;
  }
}

sdgp_status sdgp_de_select(int32_t B, int32_t nh, double* H, double* fit, const double* T, const double* ft,
                           int32_t* replaced_out) {
  try {
    const int32_t r = de_select(B, nh, H, fit, T, ft);
    if (replaced_out) *replaced_out = r;
    return SDGP_OK;
  } catch (const Error& e) {
    return (sdgp_status)e.code;
  }
}

sdgp_status sdgp_train_de(sdgp_ctx* ctx, const sdgp_kernel_desc* desc, const double* x, const double* y, int64_t n,
                          double* H, int32_t B, const double* lo, const double* hi, const sdgp_estimator* est,
                          const sdgp_de_options* opt, double* fit, double* history) {
  return guarded(ctx, [&] {
    require(desc && x && y && H && lo && hi && est && opt && fit, "NULL argument");
    require(opt->generations >= 0, "generations must be >= 0");
    require(opt->objective >= SDGP_DE_LML && opt->objective <= SDGP_DE_CONSTRAINED, "unknown objective");
    const int64_t nh = sdgp_num_hyper(desc);
    require(nh > 0, "invalid kernel descriptor");
    require(B >= 4, "differential evolution needs at least 4 members");
    const size_t BN = (size_t)B * nh;
    std::vector<double> T(BN), grad(BN), val(B), ft(B);
    std::vector<int32_t> st(B);
    // fitness of a population: one batched evaluation, failures -> -inf
    auto evaluate = [&](const double* P, double* out) {
      const sdgp_status s = sdgp_lml_grad_batched(ctx, desc, x, y, n, P, B, est, val.data(), grad.data(),
                                                  st.data(), nullptr);
      if (s != SDGP_OK) throw Error(s, std::string("batched evaluation failed: ") + ctx->err);
      for (int32_t m = 0; m < B; ++m) {
        double f = -INFINITY;
        if (st[m] == SDGP_OK && std::isfinite(val[m])) {
          f = val[m];
          if (opt->objective != SDGP_DE_LML) {
            double sp = 0.0, aug = 0.0;
            int32_t feas = 0;
            if (sdgp_sparsity_bound(desc, P + (size_t)m * nh, opt->domain_volume, &sp) != SDGP_OK ||
                sdgp_sparsity_objective(val[m], sp, opt->requirement, &aug, &feas) != SDGP_OK)
              f = -INFINITY;
            else if (opt->objective == SDGP_DE_AUGMENTED)
              f = aug;
            else
              f = feas ? val[m] : -INFINITY;
          }
        }
        out[m] = f;
      }
    };
    auto best = [&]() {
      double b = -INFINITY;
      for (int32_t m = 0; m < B; ++m) b = std::max(b, fit[m]);
      return b;
    };
    evaluate(H, fit);
    if (history) history[0] = best();
    for (int32_t gnr = 1; gnr <= opt->generations; ++gnr) {
      de_trials(B, (int32_t)nh, H, lo, hi, opt->F, opt->CR, opt->seed, (uint64_t)gnr, T.data());
      evaluate(T.data(), ft.data());
      de_select(B, (int32_t)nh, H, fit, T.data(), ft.data());
      if (history) history[gnr] = best();
    }
  });
}

}  // extern "C"
