// Internal declarations shared by the libsdgp translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/sdgp.h"

namespace sdgp {

constexpr int kWave = 64;
constexpr int kMaxDim = 4;
constexpr int kMaxN1 = 64;

// Exception type used inside the library; converted to sdgp_status at the
// ABI boundary.
struct Error : std::runtime_error {
  sdgp_status code;
  Error(sdgp_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define SDGP_HIP(expr)                                                        \
  do {                                                                        \
    hipError_t e_ = (expr);                                                   \
    if (e_ != hipSuccess)                                                     \
      throw ::sdgp::Error(e_ == hipErrorOutOfMemory ? SDGP_ERR_OOM            \
                                                    : SDGP_ERR_HIP,           \
                          std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define SDGP_CHECK_LAUNCH() SDGP_HIP(hipGetLastError())

inline void require(bool ok, const std::string& msg) {
  if (!ok) throw Error(SDGP_ERR_INVALID_ARG, msg);
}

// Growable device buffer owned by a context.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

// Kernel parameters of one hyperparameter vector, in device-friendly form.
struct KParams {
  int dim, n1, n2, core, combine;
  double sigma2, r_core, rc2, inv_rc, noise;
};

// Cell grid of the locality ordering.
struct Grid {
  int dim;
  int G[kMaxDim];          // cells per axis
  double lo[kMaxDim];      // lower corner
  double inv_side[kMaxDim];
  int64_t n_cells;
};

struct Ctx;

// Launch shape of the block CG (the autotuner's search space).  0 / -1 mean
// "the library default": spmm_blocks 0 = 32768 blocks, update_blocks 0 = one
// resident round of the update kernels, union_spmm -1 = union lists from
// 65536 rows, fw_mfma -1 = matrix-core F w products.
struct TuneChoice {
  int spmm_blocks = 0;
  int update_blocks = 0;
  int union_spmm = -1;
  int fw_mfma = -1;
  double ms_per_iter = 0.0;          // measured with this shape (tuner)
  double default_ms_per_iter = 0.0;  // measured with the defaults (tuner)
};

// Persistent store of tuned shapes (tune.cpp): a JSON object keyed by the
// problem class; path from SDGP_TUNE_CACHE, else ~/.cache/sdgp/autotune.json.
bool parse_entry(const std::string& line, TuneChoice* t);
std::string format_entry(const std::string& key, const TuneChoice& t);
std::string tune_cache_path();
bool tune_cache_get(const std::string& path, const std::string& key, TuneChoice* out);
bool tune_cache_put(const std::string& path, const std::string& key, const TuneChoice& t);

// Workspace slots.
enum Slot {
  S_KEYS, S_KEYS_ALT, S_IDX, S_PERM, S_XS, S_YS, S_CELL_START, S_BBOX,
  S_F, S_M, S_BP, S_CELLMASK, S_RUN_CNT, S_RUN_POS, S_RUN_PTR, S_RUNS, S_IV_CNT, S_IV_PTR, S_IV,
  S_ROW_NNZ, S_ROW_PTR, S_COL, S_VAL, S_SORT_TMP, S_COL2, S_VAL2, S_ROWLEN2,
  S_CG_X, S_CG_R, S_CG_P, S_CG_Q, S_CG_SCAL, S_CG_PART, S_CG_HIST_A, S_CG_HIST_B,
  S_CG_STATE, S_ZBITS, S_SLQ_WORK, S_SLQ_OUT, S_ADJ_ROW, S_ADJ_G, S_ADJ_PART,
  S_RED_PART, S_RED_OUT, S_X0S, S_MISC, S_POST, S_COUNTER, S_MASK_CNT, S_MASK_PTR, S_MASK,
  S_CG_V, S_CG_PART2, S_CG_ARGS, S_CG_PARTG, S_CG_G, S_CG_GP, S_PC_PART, S_PC_SINV, S_LR_PART, S_LR_FX, S_LR_FV,
  S_MORTON_KEYS, S_MORTON_KEYS2, S_MORTON_IDS, S_MORTON_ORDER, S_MORTON_SZ, S_MORTON_OFF, S_SCHED,
  S_CG_SRED, S_CG_WRED, S_CG_UCNT, S_CG_UPTR, S_CG_UCOL, S_CG_UVAL, S_QF, S_QM, S_KXX, S_QIV_CNT, S_QIV_PTR, S_QIV, S_QROW_NNZ, S_QROW_PTR, S_QCOL, S_QVAL,
  // population assembly (all members at once)
  S_POP_ARGS, S_POP_RARGS, S_POP_BP, S_POP_F, S_POP_M, S_POP_CM, S_POP_RUNCNT, S_POP_RUNPOS, S_POP_RUNPTR, S_POP_RUNS,
  S_POP_IVCNT, S_POP_IVPTR, S_POP_IV, S_POP_ROWNNZ, S_POP_SCAN, S_POP_ROWPTR, S_POP_COL, S_POP_VAL, S_POP_CAND,
  S_POP_GRAM, S_POP_SINV,
  S_NUM
};

struct Ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  bool timing = false;
  DevBuf buf[S_NUM];
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> spmm_events;
  int cu_count = 256;
  bool use_graph = false;        // replay captured CG iterations (hipGraph)
  int union_spmm = -1;           // CG SpMM over the 4-row union lists: -1 auto, 0 off, 1 on
  int fw_mfma = -1;              // F w products on the matrix cores: -1 auto, 0 off, 1 on
  int update_blocks = 0;         // blocks of the CG update kernels (0: default cap)
  int spmm_blocks = 0;           // blocks of the CG SpMM (0: default cap; multiple of 8)
  int autotune = 1;              // CG launch-shape tuner: 0 off, 1 from 65536 rows, 2 every solve
  std::string arch;              // device architecture (tuner key)
  bool in_trial = false;         // a tuner trial solve is running (shape = trial)
  TuneChoice trial;
  double trial_ms = -1.0;        // ms per timed iteration of the last trial (< 0: not measurable)
  TuneChoice last_shape;         // shape used by the last CG solve
  int last_tuned = 0;            // 0 defaults / options, 1 tuned shape from the store, 2 tuned in that call
  int last_y_tail = 0;           // iterations the last solve ran on y alone (probe columns stopped)
  // Workspace limits.  cap_bytes > 0: get() refuses (SDGP_ERR_OOM) to grow
  // the context's workspace beyond that many bytes.  arena != nullptr
  // (static-workspace calls): get() hands out 256-byte aligned slices of the
  // arena instead of calling hipMalloc; abuf holds those slices per slot.
  size_t cap_bytes = 0;
  size_t held_bytes = 0;
  char* arena = nullptr;
  size_t arena_cap = 0;
  size_t arena_used = 0;
  DevBuf abuf[S_NUM];
  hipStream_t gstream = nullptr; // private default-priority stream for graph capture
  hipStream_t graph_stream() {
    if (!gstream) SDGP_HIP(hipStreamCreateWithFlags(&gstream, hipStreamNonBlocking));
    return gstream;
  }

  template <class T>
  T* get(Slot s, size_t count) {
    size_t need = count * sizeof(T);
    if (need == 0) need = sizeof(T);
    if (arena) {
      DevBuf& a = abuf[s];
      if (a.bytes < need) {
        const size_t cap = (need + need / 8 + 256 + 255) / 256 * 256;   // same slack as hipMalloc'd slots
        if (cap > arena_cap - arena_used)
          throw Error(SDGP_ERR_OOM, "this input needs more device workspace than the static workspace of " +
                                        std::to_string(arena_cap >> 20) + " MiB");
        a.p = arena + arena_used;
        a.bytes = cap;
        arena_used += cap;
      }
      return static_cast<T*>(a.p);
    }
    DevBuf& b = buf[s];
    if (b.bytes < need) {
      const size_t cap = need + need / 8 + 256;
      if (cap_bytes > 0 && held_bytes - b.bytes + cap > cap_bytes)
        throw Error(SDGP_ERR_OOM, "device workspace would exceed the context's workspace_cap of " +
                                      std::to_string(cap_bytes) + " bytes");
      if (b.p) SDGP_HIP(hipFree(b.p));
      held_bytes -= b.bytes;
      b.p = nullptr;
      b.bytes = 0;
      SDGP_HIP(hipMalloc(&b.p, cap));
      b.bytes = cap;
      held_bytes += cap;
    }
    return static_cast<T*>(b.p);
  }
  hipEvent_t event() {
    if (ev_used == ev_pool.size()) {
      hipEvent_t e;
      SDGP_HIP(hipEventCreate(&e));
      ev_pool.push_back(e);
    }
    return ev_pool[ev_used++];
  }
  void release_all();
};

// Phase timer (HIP events on the context stream) used when timing is on.
struct PhaseTimer {
  Ctx* ctx;
  hipEvent_t marks[9];
  bool set[9] = {false};
  explicit PhaseTimer(Ctx* c) : ctx(c) {}
  void mark(int i) {
    if (!ctx->timing) return;
    marks[i] = ctx->event();
    SDGP_HIP(hipEventRecord(marks[i], ctx->stream));
    set[i] = true;
  }
};

// ---------------------------------------------------------------------------
// Assembly (assemble.hip)
// ---------------------------------------------------------------------------
struct Sorted {
  int64_t n;
  Grid grid;
  int32_t* perm;        // sorted position -> caller index
  double4* xs;          // sorted coordinates (padded to 4)
  int32_t* cell_start;  // [n_cells + 1]
  int32_t* cell_of;     // sorted position -> cell (the sorted keys)
  int32_t* sched;       // processing order of rows (points in Morton order)
};

struct Bumps {
  double* F;       // [n, n1] sorted order
  uint64_t* M;     // [n]
  double* bp;      // device copy of bump parameters [n1*n2*(3+dim)]
};

struct Csr {
  int64_t n, nnz;
  int64_t* row_ptr;
  int32_t* col;
  double* val;
};

KParams make_params(const sdgp_kernel_desc& d, const double* h);
void validate_shape(const sdgp_kernel_desc& d, int64_t n);
void validate(const sdgp_kernel_desc& d, const double* h, int64_t n);

// Sort points into grid cells whose side is at least r_cell.
// with_schedule: also the Morton row schedule (sched; null otherwise), which
// the solver and the adjoint walk.
Sorted order_points(Ctx* c, const double* x, int64_t n, int dim, double r_cell, bool with_schedule = true);
void gather_vector(Ctx* c, const Sorted& s, const double* src, double* dst);
Bumps bump_precompute(Ctx* c, const Sorted& s, const KParams& kp, const double* h);
// Candidate column intervals per cell (pruning); returns interval count.
// core_only: only the core supports (the factored SUM operator).
void prune(Ctx* c, const Sorted& s, const KParams& kp, const Bumps& b,
           int32_t** iv_ptr, int2** iv, bool core_only = false);
// Caller-owned CSR arrays: row_ptr (n + 1), col and val (capacity entries).
struct CsrOut {
  int64_t* row_ptr;
  int32_t* col;
  double* val;
  int64_t capacity;
};
// Count + fill; the CSR lives in context buffers (S_ROW_PTR, S_COL, S_VAL),
// or in the caller's arrays when out is given (then, when nnz exceeds
// out->capacity, row_ptr is written and the fill is skipped: col / val of
// the returned Csr are null).
// core_only: store the core part only (K_core + noise on the diagonal).
Csr assemble_sorted(Ctx* c, const Sorted& s, const KParams& kp, const Bumps& b,
                    const int32_t* iv_ptr, const int2* iv, bool add_noise,
                    int64_t* candidates, PhaseTimer* t, bool core_only = false,
                    const CsrOut* out = nullptr);
// Population assembly: members m = 0..B-1 with hyperparameters h[m] on the
// shared ordering s, every phase (bump values, cell masks, bump runs,
// candidate intervals, count, scan, fill) one launch with the member as
// grid z.  Each member's outputs (F, M, bump parameters, CSR) live in
// context storage of the population and stay valid until the next
// population call; a member's CSR is the one assemble_sorted would build.
struct PopAssembled {
  KParams kp;
  Bumps b;
  Csr A;
  int64_t candidates = 0;
};
std::vector<PopAssembled> assemble_population(Ctx* c, const Sorted& s, const sdgp_kernel_desc& d,
                                              const std::vector<const double*>& h, bool add_noise);
// Canonical (caller order, ascending columns) copy of a sorted-order CSR.
void canonicalize(Ctx* c, const Sorted& s, const Csr& k, int64_t* row_ptr,
                  int32_t* col, double* val);
// Cross-covariance kappa between test points (rows, caller order) and the
// sorted training points (columns) as CSR, and the prior variances
// k(x0, x0); requires prune() to have run for the same hyperparameters.
Csr assemble_cross(Ctx* c, const Sorted& s, const KParams& kp, const Bumps& b,
                   const double* x0, int64_t n0, const double* h,
                   double** kxx_out);

// ---------------------------------------------------------------------------
// Solver (solve.hip)
// ---------------------------------------------------------------------------
// Low-rank preconditioner M = c I + F F^T of the SUM combine (F: the sorted
// bump values); Sinv = (c I + F^T F)^{-1} on the device.
struct Precond {
  int apply = 1;        // precondition the CG with M
  int lowrank_op = 0;   // the CSR holds only the core part; A = K_core + F F^T
  int n1 = 0;
  const double* F = nullptr;
  const double* Sinv = nullptr;
  double c = 1.0;
  double logdetM = 0.0;
};

struct CgResult {
  double* V = nullptr;      // [n, R] M^{-1} b when preconditioned and kept
  double* rz0 = nullptr;    // [R] b^T M^{-1} b
  double logdetM = 0.0;
  int iters;
  int iters_y;
  double relres_max;
  bool not_spd;
  bool converged;
  double* X;        // [n, R] solution block (device, context-owned)
  double* hist_a;   // [max_iter, R] CG alphas
  double* hist_b;   // [max_iter, R] CG betas
  int32_t* col_iters;  // [R] device iterations per column
  int R;
};

enum ProbeKind { PK_RADEMACHER = 0, PK_IDENTITY = 2, PK_NONE = 3, PK_DENSE = 4 };

// Block CG on A X = [y, z_1..z_P] (or caller dense RHS when kind==PK_DENSE).
// pc (optional) preconditions every column; keep_v stores M^{-1} b.
// probe_rtol > 0: the probe columns (after y) stop at that tolerance; when
// they have all stopped before y, a single evaluation finishes y alone.
CgResult block_cg(Ctx* c, const Csr& A, const Sorted& s, const double* ys,
                  int kind, int P, uint64_t seed, double rtol, int max_iter,
                  const double* dense_rhs, int dense_R, const Precond* pc,
                  bool keep_v, PhaseTimer* t, double probe_rtol = 0.0);
// All members (own matrix and preconditioner, shared points, probes and
// options) advance together: one launch per kernel with grid z = member.
struct CgMember {
  Csr A;
  const Precond* pc = nullptr;
};
std::vector<CgResult> block_cg_multi(Ctx* c, const std::vector<CgMember>& mem, const Sorted& s,
                                     const double* ys, int kind, int P, uint64_t seed, double rtol,
                                     int max_iter, const double* dense_rhs, int dense_R, bool keep_v,
                                     bool use_graph, double probe_rtol = 0.0);
Precond lowrank_precond(Ctx* c, const Sorted& s, const KParams& kp, const Bumps& b);
// The same for every member of a population (one Gram launch, grid z =
// member); the members' bump values are contiguous from F0 with stride
// n * max(n1, 1).  failed[m] is set to the reason when member m has no
// valid preconditioner (its Precond is then unusable).
std::vector<Precond> lowrank_precond_pop(Ctx* c, const Sorted& s, const std::vector<KParams>& kp,
                                         const double* F0, std::vector<std::string>* failed);
void spmm(Ctx* c, const Csr& A, const double* X, int R, double* Y);
// Y = A X for row-major [n][R] blocks with even R (16-byte aligned).
void spmm_slab(Ctx* c, const Csr& A, const double* X, int R, double* Y);
// Randomised Taylor-series log-det (Boutsidis et al. 2017) on A.
double logdet_taylor(Ctx* c, const Csr& A, const Sorted& s, int P, int terms, uint64_t seed, double* alpha_out);
// Differential evolution (host): trial vectors of one generation, selection
// (returns the number of members replaced).
void de_trials(int32_t B, int32_t nh, const double* H, const double* lo, const double* hi, double F, double CR,
               uint64_t seed, uint64_t generation, double* T);
int32_t de_select(int32_t B, int32_t nh, double* H, double* fit, const double* T, const double* ft);
// Stochastic Lanczos quadrature from CG coefficients of columns 1..R-1.
void slq_from_cg(Ctx* c, const CgResult& cg, int kind, int P, int64_t n,
                 int lanczos_steps, double* logdet, double* stderr_out,
                 double* ritz_min, double* ritz_max);
double dot_device(Ctx* c, const double* a, int64_t stride_a, const double* b,
                  int64_t stride_b, int64_t n);
void probe_bits(Ctx* c, const Sorted& s, int P, uint64_t seed, uint64_t* zbits);
// var[t] = kxx[t] - kappa_t^T A^{-1} kappa_t, by block CG over chunks of 64
// test columns.
void posterior_variance(Ctx* c, const Csr& A, const Sorted& s, const Csr& K0, const double* kxx, double rtol,
                        int max_iter, const Precond* pc, double* var, bool* converged);

// ---------------------------------------------------------------------------
// Adjoint (adjoint.hip)
// ---------------------------------------------------------------------------
// lowrank: A holds only the core part and the bump part is F F^T (SUM).
void adjoint_gradient(Ctx* c, const Sorted& s, const KParams& kp, const Bumps& b,
                      const Csr& A, const CgResult& cg, int kind, int P,
                      uint64_t seed, const double* h, double* grad_host, bool lowrank = false);

}  // namespace sdgp
