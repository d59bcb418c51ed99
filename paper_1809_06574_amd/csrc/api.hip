// The C ABI: argument checks, handle lifetimes, the sequence driver of the
// paper's eq. general_sq (Section 2.3), error reporting.  No arithmetic of the
// method lives here; every step runs in the kernels of the other files.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <vector>
#include <thread>
#include <atomic>

#include "common.hpp"

namespace pmor {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  g_last_error = std::string("HIP error '") + hipGetErrorString(e) + "' in " + what;
  return e == hipErrorOutOfMemory ? PMOR_ENOMEM : PMOR_EHIP;
}

int allow_lds(const void* fn, size_t bytes) {
  if (bytes <= 64 * 1024) return PMOR_OK;
  PMOR_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  return PMOR_OK;
}

__global__ void k_set_int(int* p, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

int set_device_int(int* p, int v, hipStream_t st) {
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, st, p, v);
  PMOR_HIP(hipGetLastError());
  return PMOR_OK;
}

int prof_start(pmor_ctx* c, int kid) {
  Profiler& P = c->prof;
  if (P.kernel == 0 || P.kernel != kid) return -1;
  ProfRec r{};
  for (hipEvent_t* e : {&r.a, &r.b}) {
    if (!P.spare.empty()) { *e = P.spare.back(); P.spare.pop_back(); }
    else if (hipEventCreate(e) != hipSuccess) return -1;
  }
  r.valid = true;
  P.recs.push_back(r);
  return (int)P.recs.size() - 1;
}

void prof_stop(pmor_ctx* c, int idx, double bytes, int tag) {
  if (idx < 0) return;
  ProfRec& r = c->prof.recs[idx];
  r.bytes = bytes;
  r.tag = -1;  // not a block-step record: kept as is
  (void)tag;
  r.e0 = r.e1 = 0;
}

void prof_stop_seg(pmor_ctx* c, int idx, int tag, int e0) {
  if (idx < 0) return;
  ProfRec& r = c->prof.recs[idx];
  r.bytes = 0.0;
  r.tag = tag;
  r.e0 = e0;
  r.e1 = (int)c->prof.ent.size();
}

void prof_resolve(pmor_ctx* c, int first_idx, const int* steps_of) {
  auto& recs = c->prof.recs;
  const auto& ent = c->prof.ent;
  for (size_t i = (first_idx < 0 ? 0 : first_idx); i < recs.size(); ++i) {
    ProfRec& r = recs[i];
    if (r.tag < 0) continue;
    double b = 0.0;
    for (int e = r.e0; e < r.e1; ++e)
      if (steps_of[ent[e].first] > r.tag) b += ent[e].second;
    r.bytes = b;
    r.tag = -1;
    if (b == 0.0) r.valid = false;  // every segment had finished: the launch only exited
  }
}

static void prof_collect(pmor_ctx* c) {
  Profiler& P = c->prof;
  for (ProfRec& r : P.recs) {
    if (r.valid) {
      float ms = 0.f;
      if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
        P.total_ms += ms;
        P.total_bytes += r.bytes;
        P.launches += 1;
      }
    }
    P.spare.push_back(r.a);
    P.spare.push_back(r.b);
  }
  P.recs.clear();
  P.ent.clear();
}

static bool is_fin(double x) { return std::isfinite(x); }

int point_coef(const pmor_problem* pb, const double* coef, Point* out) {
  if (!coef) return fail(PMOR_EINVAL, "coefficient vector is NULL");
  *out = Point{};
  for (int r = 0; r < pb->ncoef; ++r) {
    const int t = pb->coef_slot[r];
    if (t < 0) {  // an absent role, or a part a complex term's kind excludes
      if (pb->strict_coef && coef[r] != 0.0)
        return fail(PMOR_EINVAL, "coefficient " + std::to_string(r) + " belongs to no term and must be 0");
      continue;
    }
    if (!is_fin(coef[r])) return fail(PMOR_EINVAL, "coefficient " + std::to_string(r) + " is not finite");
    out->c[t] = coef[r];
  }
  return PMOR_OK;
}

int point_sp(const pmor_problem* pb, double s, double p, Point* out) {
  if (pb->affine) return fail(PMOR_EINVAL, "an affine problem takes its points as coefficient vectors (*_c calls)");
  if (!is_fin(s) || !is_fin(p)) return fail(PMOR_EINVAL, "s and p must be finite");
  double c[PMOR_NROLES];
  role_coefs(s, p, c);
  return point_coef(pb, c, out);
}

int ensure_assembled(pmor_problem* pb, const Point& pt) {
  if (pb->have_cur && same_point(pb->cur, pt, pb->nterms)) return PMOR_OK;
  PMOR_TRY(launch_assemble(pb, pt, pb->aval, pb->ctx->stream));
  PMOR_TRY(to_sell(pb->sell, pb->aval, pb->aval_s, pb->ctx->stream));
  pb->cur = pt;
  pb->have_cur = true;
  return PMOR_OK;
}

struct Timer {
  hipStream_t s;
  hipEvent_t a, b;
  bool on;
  Timer(pmor_ctx* c, bool enable) : s(c->stream), a(c->ev0), b(c->ev1), on(enable) {
    if (on) (void)hipEventRecord(a, s);
  }
  double stop() {
    if (!on) return 0.0;
    float ms = 0.f;
    (void)hipEventRecord(b, s);
    (void)hipEventSynchronize(b);
    (void)hipEventElapsedTime(&ms, a, b);
    return ms;
  }
};

static void spai_release(pmor_spai* h) {
  if (!h) return;
  (void)hipSetDevice(h->pb->ctx->device);
  hipStream_t s = h->pb->ctx->stream;
  if (h->own_J) { dfree(h->Jcolptr, s); dfree(h->Jrow, s); }
  if (h->own_P) { dfree(h->Prowptr, s); dfree(h->Pcol, s); dfree(h->Pslot, s); }
  double* d[] = {h->Pval, h->P1val, h->Qval, h->aval1, h->rho, h->red};
  for (double* x : d) dfree(x, s);
  dfree(h->Icolptr, s);
  dfree(h->Irow, s);
  dfree(h->bucket_cols, s);
  dfree(h->P1val_s, s);
  dfree(h->Qval_s, s);
  dfree(h->esc_list, s);
  dfree(h->esc_cnt, s);
  if (h->own_psell) free_sell(&h->psell, s);
  pmor_problem* pb = h->pb;
  delete h;
  pb_unref(pb);
}

__global__ void k_copy(const double* a, double* b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}
__global__ void k_fill1(double* a, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

static int dcopy(const double* a, double* b, int64_t n, hipStream_t s) {
  if (n <= 0) return PMOR_OK;
  unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_copy, dim3(g), dim3(256), 0, s, a, b, n);
  PMOR_HIP(hipGetLastError());
  return PMOR_OK;
}
static int dfill(double* a, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return PMOR_OK;
  unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill1, dim3(g), dim3(256), 0, s, a, n, v);
  PMOR_HIP(hipGetLastError());
  return PMOR_OK;
}

// the U-diag factors of no update: 1, or (1, 0) per complex column of a complex problem
__global__ void k_unit_factors(double* q, int64_t n, int pairs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) q[i] = (pairs && (i & 1)) ? 0.0 : 1.0;
}
static int unit_factors(const pmor_spai* h, hipStream_t s) {
  const int64_t n = h->pb->n;
  if (n <= 0) return PMOR_OK;
  hipLaunchKernelGGL(k_unit_factors, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, h->Qval, n,
                     h->pb->cplx ? 1 : 0);
  PMOR_HIP(hipGetLastError());
  return PMOR_OK;
}

// P_1 of A(pt) into h (anchor moved to pt)
static int build_into(pmor_spai* h, const Point& pt, pmor_stats* stats) {
  pmor_problem* pb = h->pb;
  hipStream_t st = pb->ctx->stream;
  Timer ta(pb->ctx, stats != nullptr);
  PMOR_TRY(ensure_assembled(pb, pt));
  const double t_asm = ta.stop();
  Timer tp(pb->ctx, stats != nullptr);
  PMOR_TRY(dcopy(pb->aval, h->aval1, pb->nnz, st));
  int32_t bad = -1;
  double fro2 = 0.0;
  PMOR_TRY(run_spai_ls(h, pb->aval, nullptr, h->P1val, &bad, stats ? &fro2 : nullptr));
  PMOR_TRY(dcopy(h->P1val, h->Pval, h->nnzP, st));
  PMOR_TRY(to_sell(h->psell, h->P1val, h->P1val_s, st));
  if (h->opts.update == PMOR_UPD_DIAG) PMOR_TRY(unit_factors(h, st));
  h->q_active = false;
  h->d_active = false;
  h->c_active = false;
  h->pt1 = pt;
  const double t_pre = tp.stop();
  if (stats) {
    stats->bad_column = bad;
    stats->fro_resid = std::sqrt(fro2);
    stats->t_assemble_ms = t_asm;
    stats->t_precond_ms = t_pre;
  }
  if (bad >= 0) return fail(PMOR_ESINGULAR, "rank-deficient local least-squares problem in column " + std::to_string(bad));
  return PMOR_OK;
}

static SolveItem item_of(pmor_problem* pb, const pmor_spai* h, const double* aval, const double* aval_s,
                         const double* B, int64_t ldb, int k, double* X, int64_t ldx, pmor_stats* stats) {
  SolveItem it{};
  it.n = pb->n;
  it.nnzA = pb->nnz;
  it.arow = pb->rowptr;
  it.acol = pb->col;
  it.aval = aval;
  it.asell = &pb->sell;
  it.aval_s = aval_s;
  it.pkind = 0;
  if (h) {
    it.pkind = h->q_active ? 2 : (h->d_active ? 3 : 1);
    it.nnzP = h->nnzP;
    it.prow = h->Prowptr;
    it.pcol = h->Pcol;
    const bool fac = h->q_active || h->d_active;
    it.pval = fac ? h->P1val : h->Pval;
    it.qval = h->Qval;
    it.prs = h->d_active ? h->Qval : nullptr;
    it.psell = &h->psell;
    it.pval_s = h->P1val_s;  // Pval equals P1val unless an update is applied
    it.qval_s = h->Qval_s;
    if (h->c_active) {  // P_l of a complex problem, written out
      it.pval = h->Pval;
      it.pval_s = h->Qval_s;
    }
  }
  it.B = B;
  it.ldb = ldb;
  it.k = k;
  it.X = X;
  it.ldx = ldx;
  it.stats = stats;
  if (stats) {
    stats->cycles = 0;
    stats->steps = 0;
    std::memset(stats->cycle_steps, 0, sizeof(stats->cycle_steps));
  }
  return it;
}

static int status_error(int st) {
  switch (st) {
    case PMOR_OK: return PMOR_OK;
    case PMOR_ENOTCONV: return fail(st, "block GMRES did not converge within max_cycles");
    case PMOR_EBREAKDOWN: return fail(st, "block breakdown: rank-deficient block with unconverged columns");
    case PMOR_ENAN: return fail(st, "NaN or Inf in the right-hand side or a residual");
    default: return st;
  }
}

static int solve_opts_of(const pmor_solve_opts* opts, pmor_solve_opts* o) {
  *o = pmor_solve_opts{30, 20, 1e-8};
  if (opts) *o = *opts;
  if (o->m < 1 || o->m > 31) return fail(PMOR_EINVAL, "m must be in 1..31");
  if (o->max_cycles < 1 || o->max_cycles > PMOR_MAX_CYCLES) return fail(PMOR_EINVAL, "max_cycles out of range");
  if (!(o->tol > 0.0) || !is_fin(o->tol)) return fail(PMOR_EINVAL, "tol must be positive");
  return PMOR_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free Table 2 norms (pmor_table2_norms_noalloc).  Its partial sums
// live in a fixed device array of this file, `scratch`, instead of memory the
// library allocates: 2 x kT2Parts partials and the 2 sums (4,112 bytes, whatever
// the size of the problem).  Each GPU holds its own copy of the array until
// the process ends; its device address is taken once per device when a context
// is created on it (the array's name in host code is not a device address).
// Every call on a GPU overwrites the whole array before reading it, so nothing
// has to start at zero; calls that overlap on one GPU race for it.
// ---------------------------------------------------------------------------
constexpr int kT2Parts = 256;                    // workgroups, one partial of each norm per workgroup
constexpr int kScratchDoubles = 2 * kT2Parts + 2;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[kScratchDoubles];
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

// the device address of `scratch` on `device` (current), taken once
static int scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(PMOR_EINVAL, "device index beyond the scratch table");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch_ptr[device]) return PMOR_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) return fail(PMOR_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_ptr[device] = static_cast<double*>(ptr);
  return PMOR_OK;
}

struct T2Coefs {
  double c1[PMOR_TMAX], c2[PMOR_TMAX];
  int nt;
};

// Both Table 2 norms straight from the term values: per entry, a1 and a2 are
// the assembled values of the two points (the sums of k_assemble, in its term
// order), added into ||A1 - A2||_F^2 and ||I - A2||_F^2 row by row, one partial
// of each per workgroup (the row split and in-workgroup order of
// k_fro_partials).  part[0..G): ||I - A2||^2, part[G..2G): ||A1 - A2||^2.
__global__ __launch_bounds__(256) void k_table2_partials(int n, const int32_t* __restrict__ rowptr,
                                                         const int32_t* __restrict__ col, int64_t nnz,
                                                         const double* __restrict__ tval, T2Coefs cf,
                                                         double* __restrict__ part) {
  __shared__ double s[2][4];
  double accI = 0.0, accD = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    bool diag = false;
    for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      double a1 = 0.0, a2 = 0.0;
      for (int t = 0; t < cf.nt; ++t) a1 += cf.c1[t] * tval[(int64_t)t * nnz + e];
      for (int t = 0; t < cf.nt; ++t) a2 += cf.c2[t] * tval[(int64_t)t * nnz + e];
      const double d = a1 - a2;
      accD += d * d;
      double x;
      if (col[e] == i) { x = 1.0 - a2; diag = true; }
      else x = a2;
      accI += x * x;
    }
    if (!diag) accI += 1.0;
  }
  accI = wave_sum(accI);
  accD = wave_sum(accD);
  if ((threadIdx.x & 63) == 0) {
    s[0][threadIdx.x >> 6] = accI;
    s[1][threadIdx.x >> 6] = accD;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s[0][0] + s[0][1] + s[0][2] + s[0][3];
    part[gridDim.x + blockIdx.x] = s[1][0] + s[1][1] + s[1][2] + s[1][3];
  }
}

// out[b] = sum of part[b G .. b G + G) in a fixed tree order, b = blockIdx.x (G <= 256)
__global__ __launch_bounds__(256) void k_table2_sums(const double* __restrict__ part, int G, double* __restrict__ out) {
  __shared__ double s[256];
  s[threadIdx.x] = (int)threadIdx.x < G ? part[(int64_t)blockIdx.x * G + threadIdx.x] : 0.0;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = s[0];
}

}  // namespace pmor

using namespace pmor;

extern "C" {

const char* pmor_strerror(int code) {
  switch (code) {
    case PMOR_OK: return "ok";
    case PMOR_EINVAL: return "invalid argument";
    case PMOR_ENOMEM: return "out of device memory";
    case PMOR_ENOTCONV: return "not converged";
    case PMOR_EBREAKDOWN: return "block breakdown";
    case PMOR_ESINGULAR: return "singular least-squares problem";
    case PMOR_ENAN: return "NaN or Inf";
    case PMOR_EHIP: return "HIP runtime error";
    case PMOR_EADMIT: return "admission refused";
    default: return "unknown error";
  }
}

const char* pmor_last_error(void) { return g_last_error.c_str(); }

int pmor_ctx_create(pmor_ctx** out, int device, void* hip_stream) {
  if (!out) return fail(PMOR_EINVAL, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  PMOR_HIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(PMOR_EHIP, "device index out of range");
  PMOR_HIP(hipSetDevice(device));
  PMOR_TRY(scratch_setup(device));
  pmor_ctx* c = new pmor_ctx();
  c->device = device;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
    delete c;
    return fail(PMOR_EHIP, "event creation failed");
  }
  for (int i = 0; i < 64; ++i)
    if (hipEventCreateWithFlags(&c->evs[i], hipEventDisableTiming) != hipSuccess) {
      delete c;
      return fail(PMOR_EHIP, "event creation failed");
    }
  *out = c;
  return PMOR_OK;
}

void pmor_ctx_destroy(pmor_ctx* c) {
  if (c) ctx_unref(c);
}

}  // extern "C"

namespace pmor {

void ctx_ref(pmor_ctx* c) { ++c->refs; }

void ctx_unref(pmor_ctx* c) {
  if (--c->refs > 0) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  prof_collect(c);
  for (hipEvent_t e : c->prof.spare) (void)hipEventDestroy(e);
  (void)hipEventDestroy(c->ev0);
  (void)hipEventDestroy(c->ev1);
  for (int i = 0; i < 64; ++i)
    if (c->evs[i]) (void)hipEventDestroy(c->evs[i]);
  engine_destroy(c->eng);
  delete c;
}

void pb_ref(pmor_problem* pb) { ++pb->refs; }

void pb_unref(pmor_problem* pb) {
  if (--pb->refs > 0) return;
  pmor_ctx* c = pb->ctx;
  (void)hipSetDevice(c->device);
  hipStream_t s = c->stream;
  int32_t* ip[] = {pb->rowptr, pb->col, pb->maps, pb->colptr, pb->rowidx, pb->cscslot};
  for (int32_t* x : ip) dfree(x, s);
  dfree(pb->tval, s);
  dfree(pb->aval, s);
  dfree(pb->aval_s, s);
  free_sell(&pb->sell, s);
  delete pb;
  ctx_unref(c);
}

}  // namespace pmor

extern "C" {

int pmor_ctx_set_stream(pmor_ctx* c, void* hip_stream) {
  if (!c) return fail(PMOR_EINVAL, "ctx is NULL");
  // work queued on the old stream (and the device memory it released into the
  // cache) completes before anything is ordered on the new one
  PMOR_HIP(hipStreamSynchronize(c->stream));
  dstream_retire(c->stream);  // the caller may destroy the old stream
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  return PMOR_OK;
}

}  // extern "C"

namespace pmor {
// checks shared by the create calls: terms[0..count), NULL entries absent
// (roles only); *n_out the terms' common order
static int check_terms(const pmor_csr* const* terms, int count, bool affine, int* n_out) {
  int n = -1;
  for (int r = 0; r < count; ++r) {
    const pmor_csr* T = terms[r];
    if (!T) {
      if (affine) return fail(PMOR_EINVAL, "term " + std::to_string(r) + " is NULL");
      continue;
    }
    if (T->n <= 0) return fail(PMOR_EINVAL, "term dimension must be positive");
    if (T->nnz < 0) return fail(PMOR_EINVAL, "negative nnz");
    if (!T->rowptr || (T->nnz > 0 && (!T->col || !T->val))) return fail(PMOR_EINVAL, "term with NULL arrays");
    if (n >= 0 && T->n != n) return fail(PMOR_EINVAL, "terms differ in n");
    n = T->n;
  }
  if (n < 0) return fail(PMOR_EINVAL, "no term given");
  *n_out = n;
  return PMOR_OK;
}

static pmor_problem* problem_new(pmor_ctx* ctx, int n, bool affine) {
  pmor_problem* pb = new pmor_problem();
  pb->ctx = ctx;
  ctx_ref(ctx);
  pb->n = n;
  pb->affine = affine;
  return pb;
}

static int problem_create(pmor_ctx* ctx, const pmor_csr* const* terms, int count, bool affine, pmor_problem** out) {
  if (!ctx || !terms || !out) return fail(PMOR_EINVAL, "NULL argument");
  *out = nullptr;
  int n = -1;
  PMOR_TRY(check_terms(terms, count, affine, &n));
  PMOR_HIP(hipSetDevice(ctx->device));
  pmor_problem* pb = problem_new(ctx, n, affine);
  int rc = build_union_pattern(pb, terms, count);
  if (rc != PMOR_OK) {
    pb_unref(pb);
    return rc;
  }
  *out = pb;
  return PMOR_OK;
}

// The union patterns of independent problems: a few small kernels per problem
// with host synchronisations between them, so the problems are spread over
// worker threads, each with a stream of its own (the handles themselves are
// made and released on the calling thread).
static int problem_create_batch_impl(pmor_ctx* ctx, pmor_problem_item* items, int32_t count) {
  if (!ctx || (!items && count > 0)) return fail(PMOR_EINVAL, "NULL argument");
  if (count < 0) return fail(PMOR_EINVAL, "count must not be negative");
  PMOR_HIP(hipSetDevice(ctx->device));
  std::vector<pmor_problem*> pbs(count, nullptr);
  std::vector<int> irc(count, PMOR_OK);
  std::vector<std::string> imsg(count);
  auto nterms_of = [&](int i) { return items[i].nterms > 0 ? (int)items[i].nterms : (int)PMOR_NROLES; };
  for (int i = 0; i < count; ++i) {
    pmor_problem_item& it = items[i];
    it.pb = nullptr;
    it.status = PMOR_OK;
    int n = -1;
    if (it.nterms < 0 || it.nterms > PMOR_TMAX) irc[i] = fail(PMOR_EINVAL, "nterms must be in 0..PMOR_TMAX");
    else if (!it.terms) irc[i] = fail(PMOR_EINVAL, "terms is NULL");
    else irc[i] = check_terms(it.terms, nterms_of(i), it.nterms > 0, &n);
    if (irc[i] != PMOR_OK) {
      imsg[i] = g_last_error;
      continue;
    }
    pbs[i] = problem_new(ctx, n, it.nterms > 0);
  }
  PMOR_HIP(hipStreamSynchronize(ctx->stream));  // the caller's work on the terms precedes the workers' reads
  {
    const int nthr = std::max(1, std::min<int>(count, 8));
    std::vector<hipStream_t> ws(nthr, nullptr);
    for (auto& x : ws)
      if (hipStreamCreate(&x) != hipSuccess) { (void)hipGetLastError(); x = nullptr; }
    std::atomic<int> next{0};
    auto work = [&](int t) {
      (void)hipSetDevice(ctx->device);
      const hipStream_t s = ws[t] ? ws[t] : ctx->stream;
      for (int i = next++; i < count; i = next++) {
        if (!pbs[i]) continue;
        irc[i] = build_union_pattern(pbs[i], items[i].terms, nterms_of(i), s);
        if (irc[i] == PMOR_OK && hipStreamSynchronize(s) != hipSuccess) irc[i] = fail(PMOR_EHIP, "synchronise failed");
        if (irc[i] != PMOR_OK) imsg[i] = g_last_error;
      }
    };
    std::vector<std::thread> thr;
    for (int t = 1; t < nthr; ++t) thr.emplace_back(work, t);
    work(0);
    for (auto& x : thr) x.join();
    for (auto& x : ws)
      if (x) {
        (void)hipStreamSynchronize(x);
        dstream_retire(x);
        (void)hipStreamDestroy(x);
      }
  }
  int first = -1;
  for (int i = 0; i < count; ++i) {
    items[i].status = irc[i];
    if (irc[i] == PMOR_OK) {
      items[i].pb = pbs[i];
      continue;
    }
    if (pbs[i]) pb_unref(pbs[i]);
    if (first < 0) first = i;
  }
  if (first >= 0) return fail(irc[first], "item " + std::to_string(first) + ": " + imsg[first]);
  return PMOR_OK;
}

// the point of a batch item or job: coefficients when given, else (s, p)
static int point_of(const pmor_problem* pb, const double* coef, double s, double p, Point* out) {
  return coef ? point_coef(pb, coef, out) : point_sp(pb, s, p, out);
}
}  // namespace pmor

extern "C" {

int pmor_problem_create(pmor_ctx* ctx, const pmor_csr* const* terms, pmor_problem** out) {
  return problem_create(ctx, terms, PMOR_NROLES, false, out);
}

int pmor_problem_create_batch(pmor_ctx* ctx, pmor_problem_item* items, int32_t count) {
  return problem_create_batch_impl(ctx, items, count);
}

int pmor_problem_create_affine(pmor_ctx* ctx, int32_t nterms, const pmor_csr* const* terms, pmor_problem** out) {
  if (out) *out = nullptr;
  if (nterms < 1 || nterms > PMOR_TMAX) return fail(PMOR_EINVAL, "nterms must be in 1..PMOR_TMAX");
  return problem_create(ctx, terms, nterms, true, out);
}

int pmor_problem_create_complex(pmor_ctx* ctx, int32_t nterms, const pmor_csr* const* terms, const int32_t* kinds,
                                pmor_problem** out) {
  if (out) *out = nullptr;
  if (!ctx || !terms || !kinds || !out) return fail(PMOR_EINVAL, "NULL argument");
  if (nterms < 1 || nterms > PMOR_TMAX) return fail(PMOR_EINVAL, "nterms must be in 1..PMOR_TMAX");
  int nreal = 0, n = -1;
  for (int t = 0; t < nterms; ++t) {
    if (kinds[t] != PMOR_COEF_REAL && kinds[t] != PMOR_COEF_IMAG && kinds[t] != PMOR_COEF_COMPLEX)
      return fail(PMOR_EINVAL, "bad coefficient kind");
    const pmor_csr* T = terms[t];
    if (!T || !T->rowptr || T->n <= 0 || T->nnz < 0 || (T->nnz > 0 && (!T->col || !T->val)))
      return fail(PMOR_EINVAL, "term " + std::to_string(t) + " is NULL or malformed");
    if (n >= 0 && T->n != n) return fail(PMOR_EINVAL, "terms differ in n");
    n = T->n;
    nreal += kinds[t] == PMOR_COEF_COMPLEX ? 2 : 1;
  }
  if (nreal > PMOR_TMAX) return fail(PMOR_EINVAL, "more than PMOR_TMAX real terms");
  if ((int64_t)2 * n >= ((int64_t)1 << 31)) return fail(PMOR_EINVAL, "2n too large");
  PMOR_HIP(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  // the real terms T (x) I_2 and T (x) J_2, in the order of the coefficients
  std::vector<void*> bufs;
  std::vector<pmor_csr> rt(nreal);
  std::vector<int> slot_of_coef(2 * nterms, -1);
  int rc = PMOR_OK, q = 0;
  for (int t = 0; t < nterms && rc == PMOR_OK; ++t) {
    for (int part = 0; part < 2 && rc == PMOR_OK; ++part) {
      if ((part == 0 && kinds[t] == PMOR_COEF_IMAG) || (part == 1 && kinds[t] == PMOR_COEF_REAL)) continue;
      int32_t *rp = nullptr, *cl = nullptr, nz2 = 0;
      double* vl = nullptr;
      rc = real_equiv_term(terms[t], part, &rp, &cl, &vl, &nz2, st);
      if (rc != PMOR_OK) break;
      bufs.push_back(rp); bufs.push_back(cl); bufs.push_back(vl);
      rt[q] = pmor_csr{2 * n, nz2, rp, cl, vl};
      slot_of_coef[2 * t + part] = q++;
    }
  }
  if (rc == PMOR_OK) {
    std::vector<const pmor_csr*> ptrs(nreal);
    for (int i = 0; i < nreal; ++i) ptrs[i] = &rt[i];
    rc = problem_create(ctx, ptrs.data(), nreal, true, out);
  }
  if (rc == PMOR_OK) {  // points: 2 nterms coefficients (Re, Im per term), slots of the real terms
    pmor_problem* pb = *out;
    int term_slot[2 * PMOR_TMAX];  // real term q -> its stored slot
    for (int r = 0; r < 2 * PMOR_TMAX; ++r) term_slot[r] = pb->coef_slot[r];
    pb->ncoef = 2 * nterms;
    for (int r = 0; r < 2 * PMOR_TMAX; ++r) pb->coef_slot[r] = -1;
    for (int r = 0; r < 2 * nterms; ++r) pb->coef_slot[r] = slot_of_coef[r] >= 0 ? term_slot[slot_of_coef[r]] : -1;
    pb->strict_coef = true;
    pb->cplx = true;
  }
  (void)hipStreamSynchronize(st);
  for (void* x : bufs) dfree(x, st);
  return rc;
}

void pmor_problem_destroy(pmor_problem* pb) {
  if (pb) pb_unref(pb);
}

int pmor_problem_info(const pmor_problem* pb, int32_t* n, int32_t* nnz) {
  if (!pb) return fail(PMOR_EINVAL, "problem is NULL");
  if (n) *n = pb->n;
  if (nnz) *nnz = pb->nnz;
  return PMOR_OK;
}

int pmor_problem_pattern(const pmor_problem* pb, int32_t* rowptr, int32_t* col, int32_t* maps) {
  if (!pb) return fail(PMOR_EINVAL, "problem is NULL");
  hipStream_t s = pb->ctx->stream;
  if (rowptr) PMOR_HIP(hipMemcpyAsync(rowptr, pb->rowptr, sizeof(int32_t) * (pb->n + 1), hipMemcpyDeviceToDevice, s));
  if (col) PMOR_HIP(hipMemcpyAsync(col, pb->col, sizeof(int32_t) * pb->nnz, hipMemcpyDeviceToDevice, s));
  if (maps)
    PMOR_HIP(hipMemcpyAsync(maps, pb->maps, sizeof(int32_t) * pb->nmaps * (size_t)pb->nnz, hipMemcpyDeviceToDevice, s));
  PMOR_HIP(hipStreamSynchronize(s));
  return PMOR_OK;
}

}  // extern "C"

namespace pmor {
static int assemble_pt(pmor_problem* pb, const Point& pt, double* val) {
  PMOR_TRY(ensure_assembled(pb, pt));
  PMOR_TRY(dcopy(pb->aval, val, pb->nnz, pb->ctx->stream));
  PMOR_HIP(hipStreamSynchronize(pb->ctx->stream));
  return PMOR_OK;
}

// a handle with its sets and buffers, nothing computed yet (the options checked)
static int spai_new(pmor_problem* pb, const pmor_spai_opts* opts, pmor_spai** out, hipStream_t st = nullptr) {
  if (!st) st = pb->ctx->stream;
  pmor_spai_opts o{};
  o.pattern = PMOR_PAT_A;
  o.precision = PMOR_F64;
  o.update = PMOR_UPD_DIAG;
  if (opts) o = *opts;
  if (o.pattern != PMOR_PAT_A && o.pattern != PMOR_PAT_EXPLICIT) return fail(PMOR_EINVAL, "bad pattern kind");
  if (o.precision != PMOR_F64 && o.precision != PMOR_F32 && o.precision != PMOR_F16S)
    return fail(PMOR_EINVAL, "bad precision");
  if (o.update != PMOR_UPD_DIAG && o.update != PMOR_UPD_PATTERN && o.update != PMOR_UPD_ADAPTIVE)
    return fail(PMOR_EINVAL, "bad update kind");
  if (o.update == PMOR_UPD_ADAPTIVE && !(o.adapt_ep >= 0.0 && is_fin(o.adapt_ep)))
    return fail(PMOR_EINVAL, "adapt_ep must be finite and >= 0");
  if (o.approach != PMOR_APPROACH_FIRST && o.approach != PMOR_APPROACH_SECOND)
    return fail(PMOR_EINVAL, "bad update approach");
  if (o.approach == PMOR_APPROACH_SECOND && o.update != PMOR_UPD_DIAG)
    return fail(PMOR_EINVAL, "the second update approach is built for the U-diag update only");
  if (pb->cplx && (o.approach == PMOR_APPROACH_SECOND || o.update == PMOR_UPD_ADAPTIVE))
    return fail(PMOR_EINVAL, "a complex problem takes the first approach with the U-diag or U-pattern update");
  PMOR_HIP(hipSetDevice(pb->ctx->device));
  pmor_spai* h = new pmor_spai();
  h->pb = pb;
  pb_ref(pb);
  h->opts = o;
  *out = h;
  int rc = build_spai_sets(h, st);
  // P of a complex problem must be the real form of a complex pattern (its
  // least squares are then the complex ones, and Q P_1 keeps the pattern)
  if (rc == PMOR_OK && pb->cplx) rc = check_pairs(pb->n, h->Prowptr, h->Pcol, st);
  if (rc == PMOR_OK) {
    const int64_t n = pb->n;
    auto al = [&](double** p, int64_t cnt) {
      return dmalloc((void**)p, sizeof(double) * std::max<int64_t>(cnt, 1), st) == hipSuccess;
    };
    bool ok = al(&h->Pval, h->nnzP) && al(&h->P1val, h->nnzP) &&
              al(&h->Qval, o.update != PMOR_UPD_DIAG ? h->nnzP : n) && al(&h->aval1, pb->nnz) &&
              al(&h->rho, n) && al(&h->red, 512);
    if (ok && h->psell.cap > 0)
      ok = al(&h->P1val_s, h->psell.cap) &&
           ((o.update == PMOR_UPD_DIAG && !pb->cplx) || al(&h->Qval_s, h->psell.cap));
    if (ok && o.update == PMOR_UPD_ADAPTIVE)
      ok = dmalloc((void**)&h->esc_list, sizeof(int32_t) * 2 * std::max<int64_t>(n, 1), st) == hipSuccess &&
           dmalloc((void**)&h->esc_cnt, sizeof(int32_t) * BUCKET_SLOTS, st) == hipSuccess;
    if (!ok) rc = fail(PMOR_ENOMEM, "preconditioner allocation failed");
  }
  // built on another stream than the problem's: complete before the handle is used there
  if (st != pb->ctx->stream && hipStreamSynchronize(st) != hipSuccess && rc == PMOR_OK)
    rc = fail(PMOR_EHIP, "synchronise failed");
  if (rc != PMOR_OK) {
    spai_release(h);
    *out = nullptr;
  }
  return rc;
}

static int spai_build_pt(pmor_problem* pb, const Point& pt, const pmor_spai_opts* opts, pmor_spai** out,
                         pmor_stats* stats) {
  pmor_spai* h = nullptr;
  PMOR_TRY(spai_new(pb, opts, &h));
  const int rc = build_into(h, pt, stats);
  if (rc != PMOR_OK && rc != PMOR_ESINGULAR) {
    spai_release(h);
    return rc;
  }
  *out = h;  // on PMOR_ESINGULAR the handle is returned so the caller can inspect it
  return rc;
}

// P_1 of several problems at their points with the least squares of all in
// shared launches (pmor spai_build_batch); per item as spai_build_pt
static int spai_build_batch_impl(pmor_ctx* ctx, pmor_spai_build_item* items, int32_t count) {
  if (!ctx || (!items && count > 0)) return fail(PMOR_EINVAL, "NULL argument");
  if (count < 0) return fail(PMOR_EINVAL, "count must not be negative");
  PMOR_HIP(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  std::vector<pmor_spai*> hs;
  std::vector<const double*> av;
  std::vector<int> idx;
  std::vector<Point> pts;
  int prec = -1, first_rc = PMOR_OK;
  auto item_fail = [&](int i, int rc) {
    items[i].status = rc;
    if (first_rc == PMOR_OK) first_rc = rc;
  };
  // the items' points, then every handle's index sets and buckets: a few small
  // kernels per system with host synchronisations between them, so the systems
  // are spread over worker threads, each with a stream of its own
  std::vector<Point> ipt(count);
  std::vector<int> irc(count, PMOR_OK);
  std::vector<pmor_spai*> ih(count, nullptr);
  std::vector<std::string> imsg(count);
  for (int i = 0; i < count; ++i) {
    pmor_spai_build_item& it = items[i];
    it.h = nullptr;
    it.status = PMOR_OK;
    it.bad_column = -1;
    if (!it.pb) { irc[i] = fail(PMOR_EINVAL, "item " + std::to_string(i) + ": problem is NULL"); continue; }
    if (it.pb->ctx != ctx) { irc[i] = fail(PMOR_EINVAL, "item " + std::to_string(i) + ": another context"); continue; }
    irc[i] = it.coef ? point_coef(it.pb, it.coef, &ipt[i]) : point_sp(it.pb, it.s, it.p, &ipt[i]);
    const int pr = it.opts ? it.opts->precision : PMOR_F64;
    if (irc[i] == PMOR_OK && prec >= 0 && pr != prec) irc[i] = fail(PMOR_EINVAL, "a batch takes one least-squares precision");
    if (irc[i] == PMOR_OK) prec = pr;
    if (irc[i] != PMOR_OK) imsg[i] = pmor_last_error();
  }
  PMOR_HIP(hipStreamSynchronize(st));  // the problems' earlier work precedes the workers' reads
  {
    const int nthr = std::max(1, std::min(count, 8));
    std::vector<hipStream_t> ws(nthr, nullptr);
    for (auto& x : ws)
      if (hipStreamCreate(&x) != hipSuccess) { (void)hipGetLastError(); x = nullptr; }
    std::atomic<int> next{0};
    auto work = [&](int t) {
      (void)hipSetDevice(ctx->device);
      for (int i = next++; i < count; i = next++) {
        if (irc[i] != PMOR_OK) continue;
        irc[i] = spai_new(items[i].pb, items[i].opts, &ih[i], ws[t] ? ws[t] : st);
        if (irc[i] != PMOR_OK) imsg[i] = pmor_last_error();
      }
    };
    std::vector<std::thread> thr;
    for (int t = 1; t < nthr; ++t) thr.emplace_back(work, t);
    work(0);
    for (auto& x : thr) x.join();
    for (auto& x : ws)
      if (x) {
        (void)hipStreamSynchronize(x);
        dstream_retire(x);
        (void)hipStreamDestroy(x);
      }
  }
  for (int i = 0; i < count; ++i) {
    pmor_spai_build_item& it = items[i];
    const Point& pt = ipt[i];
    pmor_spai* h = ih[i];
    int rc = irc[i];
    if (rc != PMOR_OK) {
      item_fail(i, fail(rc, imsg[i]));
      continue;
    }
    if (rc == PMOR_OK) rc = ensure_assembled(it.pb, pt);
    if (rc == PMOR_OK) rc = dcopy(it.pb->aval, h->aval1, it.pb->nnz, st);
    if (rc != PMOR_OK) {
      if (h) spai_release(h);
      item_fail(i, rc);
      continue;
    }
    hs.push_back(h);
    av.push_back(h->aval1);
    idx.push_back(i);
    pts.push_back(pt);
  }
  int rc = run_spai_ls_multi(hs.data(), (int)hs.size(), av.data(), st);
  for (size_t t = 0; t < hs.size() && rc == PMOR_OK; ++t) {
    pmor_spai* h = hs[t];
    rc = dcopy(h->P1val, h->Pval, h->nnzP, st);
    if (rc == PMOR_OK) rc = to_sell(h->psell, h->P1val, h->P1val_s, st);
    if (rc == PMOR_OK && h->opts.update == PMOR_UPD_DIAG) rc = unit_factors(h, st);
    h->q_active = h->d_active = h->c_active = false;
    h->pt1 = pts[t];
  }
  std::vector<int> bad(hs.size(), 0x7fffffff);
  for (size_t t = 0; t < hs.size() && rc == PMOR_OK; ++t)
    if (hipMemcpyAsync(&bad[t], hs[t]->red, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess)
      rc = fail(PMOR_EHIP, "copy failed");
  if (rc == PMOR_OK && hipStreamSynchronize(st) != hipSuccess) rc = fail(PMOR_EHIP, "synchronise failed");
  if (rc != PMOR_OK) {  // the shared work failed: no item of it has a preconditioner
    for (size_t t = 0; t < hs.size(); ++t) {
      spai_release(hs[t]);
      items[idx[t]].status = rc;
    }
    return rc;
  }
  for (size_t t = 0; t < hs.size(); ++t) {
    pmor_spai_build_item& it = items[idx[t]];
    it.h = hs[t];  // on PMOR_ESINGULAR the handle is returned, as by spai_build
    if (bad[t] != 0x7fffffff) {
      it.bad_column = bad[t];
      item_fail(idx[t], fail(PMOR_ESINGULAR, "rank-deficient least-squares problem in column " +
                                                  std::to_string(bad[t]) + " (item " + std::to_string(idx[t]) + ")"));
    }
  }
  return first_rc;
}

static int spai_update_pt(pmor_spai* h, const Point& pt, pmor_stats* stats) {
  pmor_problem* pb = h->pb;
  Timer ta(pb->ctx, stats != nullptr);
  PMOR_TRY(ensure_assembled(pb, pt));
  const double t_asm = ta.stop();
  Timer tp(pb->ctx, stats != nullptr);
  int32_t bad = -1;
  double fro2 = 0.0;
  if (h->opts.update == PMOR_UPD_DIAG && pb->cplx) {
    // complex factors: P_l = Q P_1 written out and applied as it stands
    PMOR_TRY(run_update_pair(h, pb->aval, h->Pval, h->Qval, h->rho, &bad, stats ? &fro2 : nullptr));
    PMOR_TRY(to_sell(h->psell, h->Pval, h->Qval_s, pb->ctx->stream));
    h->c_active = true;
  } else if (h->opts.update == PMOR_UPD_DIAG) {
    // P_l = diag(q) P_1 is also written out (export); solves apply the factors
    PMOR_TRY(run_update_diag(h, pb->aval, &bad, stats ? &fro2 : nullptr));
    h->d_active = true;
  } else {
    if (h->opts.update == PMOR_UPD_ADAPTIVE)
      PMOR_TRY(run_update_adaptive(h, pb->aval, h->Qval, &bad, stats ? &fro2 : nullptr, nullptr));
    else PMOR_TRY(run_spai_ls(h, pb->aval, h->aval1, h->Qval, &bad, stats ? &fro2 : nullptr));
    PMOR_TRY(to_sell(h->psell, h->Qval, h->Qval_s, pb->ctx->stream));
    h->q_active = true;
  }
  const double t_pre = tp.stop();
  if (stats) {
    stats->bad_column = bad;
    stats->fro_resid = std::sqrt(fro2);
    stats->t_assemble_ms = t_asm;
    stats->t_precond_ms = t_pre;
  }
  if (bad >= 0) return fail(PMOR_ESINGULAR, "rank-deficient update problem in column " + std::to_string(bad));
  return PMOR_OK;
}

// a handle holding a given P (CSR on the device, pattern with the diagonal) anchored at pt
static int spai_import_pt(pmor_problem* pb, const Point& pt, int32_t nnzP, const int32_t* rowptr, const int32_t* col,
                          const double* val, const pmor_spai_opts* opts, pmor_spai** out) {
  if (nnzP < pb->n) return fail(PMOR_EINVAL, "P must hold the diagonal (nnzP >= n)");
  hipStream_t st = pb->ctx->stream;
  PMOR_TRY(check_csr(pb->n, nnzP, rowptr, col, st));
  // the explicit pattern of the handle is P's pattern, as columns (CSC)
  int32_t *cp = nullptr, *rw = nullptr, *sl = nullptr;
  int maxc = 0;
  PMOR_TRY(transpose_pattern(pb->n, nnzP, rowptr, col, &cp, &rw, &sl, &maxc, st));
  pmor_spai_opts o{};
  o.precision = PMOR_F64;
  o.update = PMOR_UPD_DIAG;
  if (opts) o = *opts;
  o.pattern = PMOR_PAT_EXPLICIT;
  o.nnz_explicit = nnzP;
  o.pat_colptr = cp;
  o.pat_row = rw;
  pmor_spai* h = nullptr;
  int rc = spai_new(pb, &o, &h);
  dfree(sl, st);
  if (rc == PMOR_OK) {
    h->opts.pat_colptr = nullptr;  // the caller's-pattern pointers are not kept
    h->opts.pat_row = nullptr;
    rc = ensure_assembled(pb, pt);
  }
  // the handle's CSR of P is the transpose of the CSC pattern: P's own CSR when
  // the input is sorted (checked by the explicit-pattern validation)
  if (rc == PMOR_OK) rc = dcopy(pb->aval, h->aval1, pb->nnz, st);
  if (rc == PMOR_OK) rc = dcopy(val, h->P1val, nnzP, st);
  if (rc == PMOR_OK) rc = dcopy(val, h->Pval, nnzP, st);
  if (rc == PMOR_OK) rc = to_sell(h->psell, h->P1val, h->P1val_s, st);
  if (rc == PMOR_OK && h->opts.update == PMOR_UPD_DIAG) rc = unit_factors(h, st);
  if (rc == PMOR_OK) rc = dfill(h->rho, pb->n, 0.0, st);
  if (rc == PMOR_OK) {
    h->pt1 = pt;
    h->q_active = h->d_active = h->c_active = false;
    if (hipStreamSynchronize(st) != hipSuccess) rc = fail(PMOR_EHIP, "synchronise failed");
  }
  dfree(cp, st);
  dfree(rw, st);
  if (rc != PMOR_OK) {
    spai_release(h);
    return rc;
  }
  *out = h;
  return PMOR_OK;
}
}  // namespace pmor

extern "C" {

int pmor_assemble(pmor_problem* pb, double s, double p, double* val) {
  if (!pb || !val) return fail(PMOR_EINVAL, "NULL argument");
  Point pt;
  PMOR_TRY(point_sp(pb, s, p, &pt));
  return assemble_pt(pb, pt, val);
}

int pmor_assemble_c(pmor_problem* pb, const double* coef, double* val) {
  if (!pb || !val) return fail(PMOR_EINVAL, "NULL argument");
  Point pt;
  PMOR_TRY(point_coef(pb, coef, &pt));
  return assemble_pt(pb, pt, val);
}

int spai_build(pmor_problem* pb, double s, double p, const pmor_spai_opts* opts, pmor_spai** out,
               pmor_stats* stats) {
  if (!pb || !out) return fail(PMOR_EINVAL, "NULL argument");
  *out = nullptr;
  Point pt;
  PMOR_TRY(point_sp(pb, s, p, &pt));
  return spai_build_pt(pb, pt, opts, out, stats);
}

int spai_build_c(pmor_problem* pb, const double* coef, const pmor_spai_opts* opts, pmor_spai** out,
                 pmor_stats* stats) {
  if (!pb || !out) return fail(PMOR_EINVAL, "NULL argument");
  *out = nullptr;
  Point pt;
  PMOR_TRY(point_coef(pb, coef, &pt));
  return spai_build_pt(pb, pt, opts, out, stats);
}

int spai_update(pmor_spai* h, double s, double p, pmor_stats* stats) {
  if (!h) return fail(PMOR_EINVAL, "handle is NULL");
  Point pt;
  PMOR_TRY(point_sp(h->pb, s, p, &pt));
  return spai_update_pt(h, pt, stats);
}

int spai_update_c(pmor_spai* h, const double* coef, pmor_stats* stats) {
  if (!h) return fail(PMOR_EINVAL, "handle is NULL");
  Point pt;
  PMOR_TRY(point_coef(h->pb, coef, &pt));
  return spai_update_pt(h, pt, stats);
}

int spai_update_batch(pmor_ctx* ctx, pmor_spai_update_item* items, int32_t count) {
  if (!ctx || (!items && count > 0)) return fail(PMOR_EINVAL, "NULL argument");
  if (count < 0) return fail(PMOR_EINVAL, "count must not be negative");
  PMOR_HIP(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  int first = -1;
  std::string first_msg;
  auto item_fail = [&](int i, int rc) {
    items[i].status = rc;
    if (first < 0) {
      first = i;
      first_msg = g_last_error;
    }
  };
  std::vector<int> queued;  // items whose update was queued without a readback
  for (int i = 0; i < count; ++i) {
    pmor_spai_update_item& it = items[i];
    it.status = PMOR_OK;
    it.bad_column = -1;
    pmor_spai* h = it.h;
    if (!h) { item_fail(i, fail(PMOR_EINVAL, "handle is NULL")); continue; }
    if (h->pb->ctx != ctx) { item_fail(i, fail(PMOR_EINVAL, "handle of another context")); continue; }
    Point pt;
    int rc = it.coef ? point_coef(h->pb, it.coef, &pt) : point_sp(h->pb, it.s, it.p, &pt);
    if (rc != PMOR_OK) { item_fail(i, rc); continue; }
    if (h->opts.update != PMOR_UPD_DIAG || h->pb->cplx) {  // one after another, as spai_update
      pmor_stats stt{};
      rc = spai_update_pt(h, pt, &stt);
      if (rc != PMOR_OK) {
        it.bad_column = stt.bad_column;
        item_fail(i, rc);
      }
      continue;
    }
    rc = ensure_assembled(h->pb, pt);
    if (rc == PMOR_OK) rc = run_update_diag(h, h->pb->aval, nullptr, nullptr);
    if (rc != PMOR_OK) { item_fail(i, rc); continue; }
    h->d_active = true;
    queued.push_back(i);
  }
  // the queued updates' singular-column flags (the first int of each handle's
  // reduction block), read back together
  if (!queued.empty()) {
    std::vector<int> hbad(queued.size(), 0x7fffffff);
    int rc = PMOR_OK;
    for (size_t q = 0; q < queued.size() && rc == PMOR_OK; ++q)
      if (hipMemcpyAsync(&hbad[q], items[queued[q]].h->red, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess)
        rc = fail(PMOR_EHIP, "copy of the update flags failed");
    if (rc == PMOR_OK && hipStreamSynchronize(st) != hipSuccess) rc = fail(PMOR_EHIP, "synchronise failed");
    for (size_t q = 0; q < queued.size(); ++q) {
      const int i = queued[q];
      if (rc != PMOR_OK) {
        item_fail(i, rc);
      } else if (hbad[q] != 0x7fffffff) {
        items[i].bad_column = hbad[q];
        item_fail(i, fail(PMOR_ESINGULAR, "rank-deficient update problem in column " + std::to_string(hbad[q]) +
                                              " (item " + std::to_string(i) + ")"));
      }
    }
  } else {
    PMOR_HIP(hipStreamSynchronize(st));
  }
  if (first >= 0) return fail(items[first].status, "item " + std::to_string(first) + ": " + first_msg);
  return PMOR_OK;
}

int spai_rebuild(pmor_spai* h, double s, double p, pmor_stats* stats) {
  if (!h) return fail(PMOR_EINVAL, "handle is NULL");
  Point pt;
  PMOR_TRY(point_sp(h->pb, s, p, &pt));
  return build_into(h, pt, stats);
}

int spai_rebuild_c(pmor_spai* h, const double* coef, pmor_stats* stats) {
  if (!h) return fail(PMOR_EINVAL, "handle is NULL");
  Point pt;
  PMOR_TRY(point_coef(h->pb, coef, &pt));
  return build_into(h, pt, stats);
}

int spai_import(pmor_problem* pb, double s, double p, int32_t nnzP, const int32_t* rowptr, const int32_t* col,
                const double* val, const pmor_spai_opts* opts, pmor_spai** out) {
  if (!pb || !rowptr || !col || !val || !out) return fail(PMOR_EINVAL, "NULL argument");
  *out = nullptr;
  Point pt;
  PMOR_TRY(point_sp(pb, s, p, &pt));
  return spai_import_pt(pb, pt, nnzP, rowptr, col, val, opts, out);
}

int spai_import_c(pmor_problem* pb, const double* coef, int32_t nnzP, const int32_t* rowptr, const int32_t* col,
                  const double* val, const pmor_spai_opts* opts, pmor_spai** out) {
  if (!pb || !rowptr || !col || !val || !out) return fail(PMOR_EINVAL, "NULL argument");
  *out = nullptr;
  Point pt;
  PMOR_TRY(point_coef(pb, coef, &pt));
  return spai_import_pt(pb, pt, nnzP, rowptr, col, val, opts, out);
}

int spai_build_batch(pmor_ctx* ctx, pmor_spai_build_item* items, int32_t count) {
  return spai_build_batch_impl(ctx, items, count);
}

int spai_info(const pmor_spai* h, int32_t* nnzP, int32_t* maxJ, int32_t* maxI) {
  if (!h) return fail(PMOR_EINVAL, "handle is NULL");
  if (nnzP) *nnzP = h->nnzP;
  if (maxJ) *maxJ = h->maxJ;
  if (maxI) *maxI = h->maxI;
  return PMOR_OK;
}

int spai_export(const pmor_spai* h, int32_t* rowptr, int32_t* col, double* val, double* qval, double* rho) {
  if (!h) return fail(PMOR_EINVAL, "handle is NULL");
  const pmor_problem* pb = h->pb;
  hipStream_t s = pb->ctx->stream;
  const int n = pb->n;
  if (rowptr) PMOR_HIP(hipMemcpyAsync(rowptr, h->Prowptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToDevice, s));
  if (col) PMOR_HIP(hipMemcpyAsync(col, h->Pcol, sizeof(int32_t) * h->nnzP, hipMemcpyDeviceToDevice, s));
  if (val) {
    const double* src = (h->opts.update != PMOR_UPD_DIAG) ? h->P1val : h->Pval;
    PMOR_HIP(hipMemcpyAsync(val, src, sizeof(double) * h->nnzP, hipMemcpyDeviceToDevice, s));
  }
  if (qval) {
    const int64_t len = (h->opts.update != PMOR_UPD_DIAG) ? h->nnzP : n;
    PMOR_HIP(hipMemcpyAsync(qval, h->Qval, sizeof(double) * len, hipMemcpyDeviceToDevice, s));
  }
  if (rho) PMOR_HIP(hipMemcpyAsync(rho, h->rho, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  PMOR_HIP(hipStreamSynchronize(s));
  return PMOR_OK;
}

int spai_export_sets(const pmor_spai* h, int32_t* J_colptr, int32_t* J_row, int64_t* I_colptr, int32_t* I_row,
                     int64_t* nI) {
  if (!h) return fail(PMOR_EINVAL, "handle is NULL");
  const pmor_problem* pb = h->pb;
  hipStream_t s = pb->ctx->stream;
  const int n = pb->n;
  if (nI) *nI = h->nI;
  if (J_colptr) PMOR_HIP(hipMemcpyAsync(J_colptr, h->Jcolptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToDevice, s));
  if (J_row) PMOR_HIP(hipMemcpyAsync(J_row, h->Jrow, sizeof(int32_t) * h->nnzP, hipMemcpyDeviceToDevice, s));
  if (I_colptr) PMOR_HIP(hipMemcpyAsync(I_colptr, h->Icolptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToDevice, s));
  if (I_row && h->nI > 0) PMOR_HIP(hipMemcpyAsync(I_row, h->Irow, sizeof(int32_t) * h->nI, hipMemcpyDeviceToDevice, s));
  PMOR_HIP(hipStreamSynchronize(s));
  return PMOR_OK;
}

void spai_free(pmor_spai* h) { spai_release(h); }

}  // extern "C"

namespace pmor {
static int block_solve_pt(pmor_problem* pb, const pmor_spai* h, const Point* pt, int pt_rc, const double* B,
                          int64_t ldb, int32_t k, double* X, int64_t ldx, const pmor_solve_opts* opts,
                          pmor_stats* stats) {
  if (!pb || !B || !X) return fail(PMOR_EINVAL, "NULL argument");
  if (k < 1 || k > PMOR_KMAX) return fail(PMOR_EINVAL, "k must be in 1..16");
  if (ldb < k || ldx < k) return fail(PMOR_EINVAL, "leading dimension smaller than k");
  if (h && h->pb != pb) return fail(PMOR_EINVAL, "preconditioner belongs to another problem");
  if (pt_rc != PMOR_OK) return pt_rc;
  pmor_solve_opts o;
  PMOR_TRY(solve_opts_of(opts, &o));
  PMOR_HIP(hipSetDevice(pb->ctx->device));
  auto t0 = std::chrono::steady_clock::now();
  PMOR_TRY(ensure_assembled(pb, *pt));
  SolveItem it = item_of(pb, h, pb->aval, pb->aval_s, B, ldb, k, X, ldx, stats);
  PMOR_TRY(krylov_batch(pb->ctx, &it, 1, o));
  if (stats) {
    stats->t_solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return status_error(it.status);
}
}  // namespace pmor

extern "C" {

int block_solve(pmor_problem* pb, const pmor_spai* h, double s, double p, const double* B, int64_t ldb, int32_t k,
                double* X, int64_t ldx, const pmor_solve_opts* opts, pmor_stats* stats) {
  Point pt{};
  const int prc = pb ? point_sp(pb, s, p, &pt) : PMOR_OK;
  return block_solve_pt(pb, h, &pt, prc, B, ldb, k, X, ldx, opts, stats);
}

int block_solve_c(pmor_problem* pb, const pmor_spai* h, const double* coef, const double* B, int64_t ldb, int32_t k,
                  double* X, int64_t ldx, const pmor_solve_opts* opts, pmor_stats* stats) {
  Point pt{};
  const int prc = pb ? point_coef(pb, coef, &pt) : PMOR_OK;
  return block_solve_pt(pb, h, &pt, prc, B, ldb, k, X, ldx, opts, stats);
}

int pmor_batch_solve(pmor_ctx* ctx, const pmor_batch_item* items, int32_t nitems, const pmor_solve_opts* opts,
                     pmor_stats* stats, int32_t* status) {
  if (!ctx || (!items && nitems > 0)) return fail(PMOR_EINVAL, "NULL argument");
  if (nitems < 0) return fail(PMOR_EINVAL, "nitems must not be negative");
  pmor_solve_opts o;
  PMOR_TRY(solve_opts_of(opts, &o));
  for (int i = 0; i < nitems; ++i) {
    const pmor_batch_item& b = items[i];
    if (!b.pb || !b.B || !b.X) return fail(PMOR_EINVAL, "item " + std::to_string(i) + ": NULL argument");
    if (b.pb->ctx != ctx) return fail(PMOR_EINVAL, "item " + std::to_string(i) + ": problem of another context");
    if (b.k < 1 || b.k > PMOR_KMAX || b.ldb < b.k || b.ldx < b.k)
      return fail(PMOR_EINVAL, "item " + std::to_string(i) + ": bad k or leading dimension");
    if (b.h && b.h->pb != b.pb) return fail(PMOR_EINVAL, "item " + std::to_string(i) + ": foreign preconditioner");
  }
  std::vector<Point> pts(nitems);
  for (int i = 0; i < nitems; ++i) {
    const int prc = point_of(items[i].pb, items[i].coef, items[i].s, items[i].p, &pts[i]);
    if (prc != PMOR_OK) return fail(prc, "item " + std::to_string(i) + ": " + g_last_error);
  }
  if (nitems == 0) return PMOR_OK;
  PMOR_HIP(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  // A values: the problem's own buffer for its first point, private copies for other points
  std::vector<SolveItem> it(nitems);
  std::vector<double*> extra;
  int rc = PMOR_OK;
  for (int i = 0; i < nitems && rc == PMOR_OK; ++i) {
    const pmor_batch_item& b = items[i];
    const double* aval = nullptr;
    const double* aval_s = nullptr;
    for (int q = 0; q < i; ++q)
      if (items[q].pb == b.pb && same_point(pts[q], pts[i], b.pb->nterms)) {
        aval = it[q].aval;
        aval_s = it[q].aval_s;
        break;
      }
    if (!aval) {
      bool first = true;
      for (int q = 0; q < i; ++q)
        if (items[q].pb == b.pb) first = false;
      if (first) {
        rc = ensure_assembled(b.pb, pts[i]);
        aval = b.pb->aval;
        aval_s = b.pb->aval_s;
      } else {
        const int64_t cap = b.pb->sell.cap;
        double* buf = nullptr;
        if (dmalloc((void**)&buf, sizeof(double) * (std::max<int64_t>(b.pb->nnz, 1) + cap), st) != hipSuccess) {
          (void)hipGetLastError();
          rc = fail(PMOR_ENOMEM, "allocation of a point's A values failed");
          break;
        }
        extra.push_back(buf);
        rc = launch_assemble(b.pb, pts[i], buf, st);
        aval = buf;
        if (rc == PMOR_OK && cap > 0) {
          double* bs = buf + std::max<int64_t>(b.pb->nnz, 1);
          rc = to_sell(b.pb->sell, buf, bs, st);
          aval_s = bs;
        }
      }
    }
    it[i] = item_of(b.pb, b.h, aval, aval_s, b.B, b.ldb, b.k, b.X, b.ldx, stats ? &stats[i] : nullptr);
  }
  if (rc == PMOR_OK) rc = krylov_batch(ctx, it.data(), nitems, o);
  for (double* x : extra) dfree(x, st);
  if (rc != PMOR_OK) return rc;
  int first_bad = PMOR_OK;
  for (int i = 0; i < nitems; ++i) {
    if (status) status[i] = it[i].status;
    if (stats) stats[i].t_solve_ms = it[i].t_done_ms;
    if (first_bad == PMOR_OK && it[i].status != PMOR_OK) first_bad = it[i].status;
  }
  return status_error(first_bad);
}

}  // extern "C"

namespace pmor {

// device buffers of a group of points of one sequence
struct SeqBuffers {
  double* aval = nullptr;   // group x nnz: A(l) values
  double* pq = nullptr;     // group x nnzP: P_l, or Q_l for the pattern update
  double* aval_s = nullptr; // group x capA: A(l) in the sliced ELL layout (when the problem has one)
  double* pq_s = nullptr;   // group x capP: P_l / Q_l in the sliced ELL layout
  int64_t capA = 0, capP = 0;
  double* q = nullptr;      // group x n: U-diag factors q_l (P_l = diag(q_l) P_1)
  double* rho = nullptr;    // group x n: U-diag column residuals
  double* carry = nullptr;  // n: second approach, the running row scale of the group's last point
  double* fro = nullptr;    // group x 260 (sum-of-squares scratch)
  int* bad = nullptr;       // group
  int64_t bytes = 0;
  hipStream_t stream = nullptr;
  SeqBuffers() = default;
  SeqBuffers(const SeqBuffers&) = delete;
  SeqBuffers& operator=(const SeqBuffers&) = delete;
  ~SeqBuffers() {
    void* v[] = {aval, pq, q, rho, carry, fro, bad, aval_s, pq_s};
    for (void* x : v) dfree(x, stream);
  }
  int alloc(int group, int64_t nnz, int64_t nnzP, int64_t n, hipStream_t s, int64_t capa = 0, int64_t capp = 0) {
    stream = s;
    capA = capa;
    capP = capp;
    auto al = [&](void** p, size_t b) {
      b = std::max<size_t>(b, 8);
      if (dmalloc(p, b, stream) != hipSuccess) {
        (void)hipGetLastError();
        return fail(PMOR_ENOMEM, "allocation of the sequence buffers failed");
      }
      bytes += (int64_t)b;
      return PMOR_OK;
    };
    PMOR_TRY(al((void**)&aval, sizeof(double) * group * nnz));
    PMOR_TRY(al((void**)&pq, sizeof(double) * group * nnzP));
    PMOR_TRY(al((void**)&q, sizeof(double) * group * n));
    PMOR_TRY(al((void**)&rho, sizeof(double) * group * n));
    PMOR_TRY(al((void**)&carry, sizeof(double) * n));
    PMOR_TRY(al((void**)&fro, sizeof(double) * group * 260));
    PMOR_TRY(al((void**)&bad, sizeof(int) * group));
    if (capA > 0) PMOR_TRY(al((void**)&aval_s, sizeof(double) * group * capA));
    if (capP > 0) PMOR_TRY(al((void**)&pq_s, sizeof(double) * group * capP));
    return PMOR_OK;
  }
  static int64_t estimate(int group, int64_t nnz, int64_t nnzP, int64_t n, int64_t capa = 0, int64_t capp = 0) {
    return 8 * group * (nnz + nnzP + capa + capp + 2 * n) + 8 * n + 8 * 260 * group + 4 * group + 8 * 256;
  }
};

__global__ void k_fill_int(int* p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

static SolveItem point_item(pmor_problem* pb, pmor_spai* h, const double* Al, const double* Al_s, const double* B,
                            int64_t ldb, int k, double* X, int64_t ldx, int l, pmor_stats* stats) {
  SolveItem x = item_of(pb, nullptr, Al, Al_s, B, ldb, k, X + (int64_t)l * pb->n * ldx, ldx,
                        stats ? &stats[l] : nullptr);
  x.pkind = 1;
  x.prow = h->Prowptr;
  x.pcol = h->Pcol;
  x.nnzP = h->nnzP;
  x.psell = &h->psell;
  x.pval = h->P1val;
  x.pval_s = h->P1val_s;
  x.tag = l;
  return x;
}

// prepare_points for the U-diag update: every A(l) (straight into the sliced
// ELL layout when the problem has one, else in CSR order) and every factor
// q_l in launches of PTS_MAX points; P_l = diag(q_l) P_1 stays factored and
// the engine scales the rows of P_1 X.  The batch's assembly and update times
// are shared evenly among its points in stats.
static int prepare_points_diag(pmor_problem* pb, pmor_spai* h, const Point* pts, int l0, int cnt, const double* B,
                               int64_t ldb, int k, double* X, int64_t ldx,
                               pmor_stats* stats, const pmor_stats& pre0, SeqBuffers& sb, SolveItem* items,
                               int* bad) {
  hipStream_t st = pb->ctx->stream;
  const int n = pb->n;
  const bool sell = sb.capA > 0;
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
  if (stats)
    for (auto& e : ev)
      if (hipEventCreate(&e) != hipSuccess) { e = nullptr; (void)hipGetLastError(); }
  auto rec = [&](int i) {
    if (ev[i]) (void)hipEventRecord(ev[i], st);
  };
  int rc = PMOR_OK;
  rec(0);
  for (int c0 = 0; c0 < cnt && rc == PMOR_OK; c0 += PTS_MAX) {
    const int m = std::min(PTS_MAX, cnt - c0);
    rc = sell ? launch_assemble_pts(pb, pts + l0 + c0, m, &pb->sell, sb.aval_s + (int64_t)c0 * sb.capA, sb.capA, st)
              : launch_assemble_pts(pb, pts + l0 + c0, m, nullptr, sb.aval + (int64_t)c0 * pb->nnz, pb->nnz, st);
  }
  rec(1);
  if (rc == PMOR_OK) {
    hipLaunchKernelGGL(k_fill_int, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, sb.bad, cnt, 0x7fffffff);
    if (hipGetLastError() != hipSuccess) rc = fail(PMOR_EHIP, "launch failed");
  }
  if (h->opts.approach == PMOR_APPROACH_SECOND) {
    // anchors A(l-1): the points in order, the running scale carried across launches
    for (int c0 = std::max(0, 1 - l0); c0 < cnt && rc == PMOR_OK; c0 += PTS_MAX) {
      const int m = std::min(PTS_MAX, cnt - c0);
      rc = launch_update_diag_chain(h, pts, l0 + c0, m, sb.carry, sb.q + (int64_t)c0 * n, sb.rho + (int64_t)c0 * n,
                                    sb.bad + c0, st);
    }
  } else {
    for (int c0 = 0; c0 < cnt && rc == PMOR_OK; c0 += PTS_MAX) {
      const int m = std::min(PTS_MAX, cnt - c0);
      rc = launch_update_diag_pts(h, pts + l0 + c0, m, sb.q + (int64_t)c0 * n, sb.rho + (int64_t)c0 * n, sb.bad + c0,
                                  st);
    }
  }
  if (rc == PMOR_OK && stats) rc = sumsq_pts(sb.rho, n, cnt, sb.fro, 260, st);
  rec(2);
  std::vector<int> bd(cnt, 0x7fffffff);
  std::vector<double> fr2(stats ? (size_t)cnt * 260 : 0, 0.0);
  if (rc == PMOR_OK) {
    bool ok = hipMemcpyAsync(bd.data(), sb.bad, sizeof(int) * cnt, hipMemcpyDeviceToHost, st) == hipSuccess;
    if (ok && stats)
      ok = hipMemcpyAsync(fr2.data(), sb.fro, sizeof(double) * 260 * cnt, hipMemcpyDeviceToHost, st) == hipSuccess;
    ok = ok && hipStreamSynchronize(st) == hipSuccess;
    if (!ok) rc = fail(PMOR_EHIP, "copy of the update verdicts failed");
  }
  float ta = 0.f, tp = 0.f;
  if (rc == PMOR_OK && ev[0] && ev[1] && ev[2]) {
    (void)hipEventElapsedTime(&ta, ev[0], ev[1]);
    (void)hipEventElapsedTime(&tp, ev[1], ev[2]);
  }
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  if (rc != PMOR_OK) return rc;
  for (int t = 0; t < cnt; ++t) {
    const int l = l0 + t;
    const double* Al = sell ? nullptr : sb.aval + (int64_t)t * pb->nnz;
    const double* Al_s = sell ? sb.aval_s + (int64_t)t * sb.capA : nullptr;
    SolveItem x = point_item(pb, h, Al, Al_s, B, ldb, k, X, ldx, l, stats);
    double fro2 = 0.0;
    if (l == 0) {
      bad[t] = pre0.bad_column;
      fro2 = pre0.fro_resid * pre0.fro_resid;
    } else {
      x.pkind = 3;
      x.prs = sb.q + (int64_t)t * n;
      bad[t] = (bd[t] == 0x7fffffff) ? -1 : bd[t];
      if (stats) fro2 = fr2[(size_t)t * 260];
    }
    items[t] = x;
    if (stats) {
      pmor_stats& S = stats[l];
      S.t_assemble_ms = ta / cnt;
      S.t_precond_ms = l == 0 ? 0.0 : tp / cnt;
      S.fro_resid = std::sqrt(fro2);
      S.bad_column = bad[t];
      if (l == 0) {
        S.t_assemble_ms += pre0.t_assemble_ms;
        S.t_precond_ms += pre0.t_precond_ms;
      }
    }
  }
  return PMOR_OK;
}

// Points [l0, l0 + cnt) of a sequence whose P_1 (point 0) is h's anchor: A(l)
// into sb.aval + t nnz, the point's preconditioner (P_1 for point 0, else the
// update (Table 1, as the handle's options say) or, for the rebuild policy, a fresh SPAI) into
// sb.pq + t nnzP, and the engine item of every point.  bad[t]: a singular
// column of the point's least-squares problems, or -1.  stats (the sequence's
// array, may be NULL) gets the assembly and preconditioner times, the residual
// norm and bad_column of each point.  Synchronises the stream.
static int prepare_points(pmor_problem* pb, pmor_spai* h, int policy, const Point* pts, int l0, int cnt,
                          const double* B, int64_t ldb, int k, double* X, int64_t ldx, pmor_stats* stats,
                          const pmor_stats& pre0, SeqBuffers& sb, SolveItem* items, int* bad) {
  if (policy == PMOR_UPDATE && h->opts.update == PMOR_UPD_DIAG && !pb->cplx)
    return prepare_points_diag(pb, h, pts, l0, cnt, B, ldb, k, X, ldx, stats, pre0, sb, items, bad);
  hipStream_t st = pb->ctx->stream;
  const int64_t nnz = pb->nnz, nnzP = h->nnzP;
  std::vector<hipEvent_t> ev;
  if (stats) {
    ev.assign(2 * (size_t)cnt + 1, nullptr);
    for (auto& e : ev)
      if (hipEventCreate(&e) != hipSuccess) { e = nullptr; (void)hipGetLastError(); }
  }
  auto rec = [&](size_t i) {
    if (i < ev.size() && ev[i]) (void)hipEventRecord(ev[i], st);
  };
  std::vector<double> fro_host(cnt, 0.0);
  int rc = PMOR_OK;
  rec(0);
  for (int t = 0; t < cnt && rc == PMOR_OK; ++t) {
    const int l = l0 + t;
    bad[t] = -1;
    double* Al = sb.aval + (int64_t)t * nnz;
    double* PQ = sb.pq + (int64_t)t * nnzP;
    rc = launch_assemble(pb, pts[l], Al, st);
    double* Al_s = sb.capA > 0 ? sb.aval_s + (int64_t)t * sb.capA : nullptr;
    double* PQ_s = sb.capP > 0 ? sb.pq_s + (int64_t)t * sb.capP : nullptr;
    if (rc == PMOR_OK && Al_s) rc = to_sell(pb->sell, Al, Al_s, st);
    rec(1 + 2 * t);
    if (rc != PMOR_OK) break;
    SolveItem x = point_item(pb, h, Al, Al_s, B, ldb, k, X, ldx, l, stats);
    if (l == 0) {
      fro_host[t] = pre0.fro_resid * pre0.fro_resid;
      bad[t] = pre0.bad_column;
    } else {
      int32_t b = -1;
      double fro2 = 0.0;
      const bool pair = policy == PMOR_UPDATE && h->opts.update == PMOR_UPD_DIAG;  // a complex problem
      if (policy == PMOR_UPDATE && h->opts.update == PMOR_UPD_ADAPTIVE)
        rc = run_update_adaptive(h, Al, PQ, &b, stats ? &fro2 : nullptr, nullptr);
      else if (pair)
        rc = run_update_pair(h, Al, PQ, sb.q + (int64_t)t * pb->n, sb.rho + (int64_t)t * pb->n, &b,
                             stats ? &fro2 : nullptr);
      else rc = run_spai_ls(h, Al, policy == PMOR_UPDATE ? h->aval1 : nullptr, PQ, &b, stats ? &fro2 : nullptr);
      bad[t] = b;
      fro_host[t] = fro2;
      if (policy == PMOR_UPDATE && !pair) {
        x.pkind = 2;
        x.pval = h->P1val;
        x.pval_s = h->P1val_s;
        x.qval = PQ;
        x.qval_s = PQ_s;
      } else {
        x.pval = PQ;
        x.pval_s = PQ_s;
      }
    }
    if (rc == PMOR_OK && PQ_s && l > 0) rc = to_sell(h->psell, PQ, PQ_s, st);
    rec(2 + 2 * t);
    items[t] = x;
  }
  if (rc == PMOR_OK) rc = hipStreamSynchronize(st) == hipSuccess ? PMOR_OK : fail(PMOR_EHIP, "synchronise failed");
  if (stats && rc == PMOR_OK) {
    for (int t = 0; t < cnt; ++t) {
      pmor_stats& S = stats[l0 + t];
      float a = 0.f, b = 0.f;
      if (ev[2 * t] && ev[1 + 2 * t]) (void)hipEventElapsedTime(&a, ev[2 * t], ev[1 + 2 * t]);
      if (ev[1 + 2 * t] && ev[2 + 2 * t]) (void)hipEventElapsedTime(&b, ev[1 + 2 * t], ev[2 + 2 * t]);
      S.t_assemble_ms = a;
      S.t_precond_ms = b;
      S.fro_resid = std::sqrt(fro_host[t]);
      S.bad_column = bad[t];
      if (l0 + t == 0) {
        S.t_assemble_ms += pre0.t_assemble_ms;
        S.t_precond_ms += pre0.t_precond_ms;
      }
    }
  }
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  return rc;
}

// the checks of a sequence and its points: coefs (npts x pb->ncoef) when given,
// else (s_list[l], p_list[l])
static int sequence_checks(const pmor_problem* pb, const double* B, int64_t ldb, int32_t k, const double* s_list,
                           const double* p_list, const double* coefs, int32_t npts, const double* X, int64_t ldx,
                           int32_t policy, std::vector<Point>* pts) {
  if (!pb || !B || !X || (!coefs && (!s_list || !p_list))) return fail(PMOR_EINVAL, "NULL argument");
  if (npts < 1) return fail(PMOR_EINVAL, "npts must be positive");
  if (policy != PMOR_REBUILD && policy != PMOR_UPDATE) return fail(PMOR_EINVAL, "bad policy");
  if (k < 1 || k > PMOR_KMAX || ldb < k || ldx < k) return fail(PMOR_EINVAL, "bad k or leading dimension");
  pts->assign(npts, Point{});
  for (int l = 0; l < npts; ++l) {
    const int rc = coefs ? point_coef(pb, coefs + (int64_t)l * pb->ncoef, &(*pts)[l])
                         : point_sp(pb, s_list[l], p_list[l], &(*pts)[l]);
    if (rc != PMOR_OK) return fail(rc, "point " + std::to_string(l) + ": " + g_last_error);
  }
  return PMOR_OK;
}

// Anchors of a re-anchored sequence (U-diag, first approach): point 0, then,
// scanning the points in order, every point l whose update misfit
// ||A(a) - A(l) diag(q)||_F exceeds tol ||A(a)||_F against the current anchor
// a.  The misfit is the root sum of the update's column residuals (formed for
// up to PTS_MAX points per launch, read back once per launch); a non-finite
// misfit also re-anchors (the rebuild there reports a singular column).
static int plan_anchors(pmor_problem* pb, const Point* pts, int npts, double tol, std::vector<int>* anchors) {
  hipStream_t st = pb->ctx->stream;
  const int n = pb->n;
  const int64_t nnz = pb->nnz;
  double *Aa = nullptr, *q = nullptr, *rho = nullptr, *fro = nullptr, *nrm = nullptr;
  int* bad = nullptr;
  struct Free {
    std::vector<void*> v;
    hipStream_t s;
    ~Free() {
      for (void* x : v) dfree(x, s);
    }
  } keep{{}, st};
  auto al = [&](void** x, size_t b) {
    if (dmalloc(x, std::max<size_t>(b, 8), st) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    keep.v.push_back(*x);
    return true;
  };
  if (!al((void**)&Aa, sizeof(double) * nnz) || !al((void**)&q, sizeof(double) * PTS_MAX * n) ||
      !al((void**)&rho, sizeof(double) * PTS_MAX * n) || !al((void**)&fro, sizeof(double) * PTS_MAX * 260) ||
      !al((void**)&nrm, sizeof(double) * 260) || !al((void**)&bad, sizeof(int) * PTS_MAX))
    return fail(PMOR_ENOMEM, "allocation of the re-anchoring scratch failed");
  int a = 0, l = 1;
  while (l < npts) {
    PMOR_TRY(launch_assemble(pb, pts[a], Aa, st));
    PMOR_TRY(sumsq(Aa, nnz, nrm, st));
    double na2 = 0.0;
    PMOR_HIP(hipMemcpyAsync(&na2, nrm, sizeof(double), hipMemcpyDeviceToHost, st));
    PMOR_HIP(hipStreamSynchronize(st));  // na2 is read below; no copy into it may outlive an early return
    int found = -1;
    for (int c0 = l; c0 < npts && found < 0; c0 += PTS_MAX) {
      const int m = std::min(PTS_MAX, npts - c0);
      PMOR_TRY(launch_update_diag_pts_anchor(pb, Aa, pts + c0, m, q, rho, bad, st));
      PMOR_TRY(sumsq_pts(rho, n, m, fro, 260, st));
      std::vector<double> f((size_t)m * 260);
      PMOR_HIP(hipMemcpyAsync(f.data(), fro, sizeof(double) * 260 * m, hipMemcpyDeviceToHost, st));
      PMOR_HIP(hipStreamSynchronize(st));
      for (int t = 0; t < m && found < 0; ++t)
        if (!(f[(size_t)t * 260] <= tol * tol * na2)) found = c0 + t;
    }
    if (found < 0) break;
    anchors->push_back(found);
    a = found;
    l = found + 1;
  }
  return PMOR_OK;
}

// One run of a sequence: P_1 built at its first point, the others updated
// from it (or rebuilt).  lbase: the run's first point in the caller's sequence
// (stats[].anchor, messages); t0: the call's start.
static int sequence_run(pmor_problem* pb, const double* B, int64_t ldb, int32_t k, const Point* pts, int32_t npts,
                        double* X, int64_t ldx, int32_t policy,
                        const pmor_spai_opts* sopts, const pmor_solve_opts& o, pmor_stats* stats, int lbase,
                        std::chrono::steady_clock::time_point t0) {
  auto since = [&]() { return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count(); };
  if (stats)
    for (int l = 0; l < npts; ++l) stats[l].anchor = policy == PMOR_UPDATE ? lbase : lbase + l;
  pmor_stats pre0{};
  pre0.bad_column = -1;
  pmor_spai* h = nullptr;
  int rc = spai_build_pt(pb, pts[0], sopts, &h, &pre0);
  if (rc != PMOR_OK && rc != PMOR_ESINGULAR) {
    if (stats) { stats[0] = pre0; stats[0].t_solve_ms = since(); stats[0].anchor = lbase; }
    spai_release(h);
    return rc;
  }
  if (rc == PMOR_ESINGULAR) {  // no anchor: nothing can be solved
    if (stats) { stats[0] = pre0; stats[0].t_solve_ms = since(); stats[0].anchor = lbase; }
    spai_release(h);
    return rc;
  }
  const int n = pb->n;
  const int64_t nnz = pb->nnz, nnzP = h->nnzP;
  // points per group: A and P/Q values plus the Krylov blocks of one system
  const int kp = k <= 1 ? 1 : k <= 2 ? 2 : k <= 4 ? 4 : k <= 8 ? 8 : 16;
  // the U-diag update keeps P_l factored: no per-point P values
  const bool rowq = policy == PMOR_UPDATE && h->opts.update == PMOR_UPD_DIAG && !pb->cplx;
  const int64_t nnzPp = rowq ? 0 : nnzP, capPp = rowq ? 0 : h->psell.cap;
  // and A(l) only in the sliced ELL layout when it has one
  const int64_t nnzA = (rowq && pb->sell.cap > 0) ? 0 : nnz;
  const double per_point = 8.0 * (nnzA + nnzPp + pb->sell.cap + capPp + 2 * n) + 8.0 * (double)n * kp * (o.m + 7) +
                           64.0 * 1024;
  size_t fr = 0, tot = 0;
  PMOR_HIP(hipMemGetInfo(&fr, &tot));
  const int group = (int)std::max(1.0, std::min<double>(npts, 0.6 * (double)fr / per_point));
  SeqBuffers sb;
  rc = sb.alloc(group, nnzA, nnzPp, n, pb->ctx->stream, pb->sell.cap, capPp);
  if (rc != PMOR_OK) { spai_release(h); return rc; }
  int first_bad = PMOR_OK;
  for (int l0 = 0; l0 < npts && rc == PMOR_OK; l0 += group) {
    const int cnt = std::min(group, npts - l0);
    std::vector<SolveItem> it(cnt);
    std::vector<int> bad(cnt, -1);
    rc = prepare_points(pb, h, policy, pts, l0, cnt, B, ldb, k, X, ldx, stats, pre0, sb, it.data(), bad.data());
    if (rc != PMOR_OK) break;
    // solve the points whose preconditioner exists
    std::vector<SolveItem> ok;
    for (int t = 0; t < cnt; ++t) {
      if (bad[t] >= 0) {
        if (first_bad == PMOR_OK) {
          first_bad = PMOR_ESINGULAR;
          set_error("rank-deficient least-squares problem at point " + std::to_string(lbase + l0 + t) + ", column " +
                    std::to_string(bad[t]));
        }
        if (stats) stats[l0 + t].t_solve_ms = since();
        continue;
      }
      ok.push_back(it[t]);
    }
    const double t_start = since();
    rc = krylov_batch(pb->ctx, ok.data(), (int)ok.size(), o);
    if (rc != PMOR_OK) break;
    for (const SolveItem& x : ok) {
      if (stats) stats[x.tag].t_solve_ms = t_start + x.t_done_ms;
      if (first_bad == PMOR_OK && x.status != PMOR_OK) {
        first_bad = x.status;
        (void)status_error(first_bad);
      }
    }
  }
  spai_release(h);
  if (rc != PMOR_OK) return rc;
  return first_bad;
}

}  // namespace pmor

extern "C" {

}  // extern "C"

namespace pmor {
static int sequence_solve(pmor_problem* pb, const double* B, int64_t ldb, int32_t k, const double* s_list,
                          const double* p_list, const double* coefs, int32_t npts, double* X, int64_t ldx,
                          int32_t policy, const pmor_spai_opts* sopts, const pmor_solve_opts* vopts,
                          pmor_stats* stats) {
  std::vector<Point> pts;
  PMOR_TRY(sequence_checks(pb, B, ldb, k, s_list, p_list, coefs, npts, X, ldx, policy, &pts));
  pmor_solve_opts o;
  PMOR_TRY(solve_opts_of(vopts, &o));
  const double tol = sopts ? sopts->reanchor_tol : 0.0;
  if (!(tol >= 0.0) || !is_fin(tol)) return fail(PMOR_EINVAL, "reanchor_tol must be finite and >= 0");
  if (tol > 0.0 && (policy != PMOR_UPDATE || sopts->update != PMOR_UPD_DIAG || sopts->approach != PMOR_APPROACH_FIRST))
    return fail(PMOR_EINVAL, "re-anchoring is built for the U-diag update with the first approach");
  if (tol > 0.0 && pb->cplx) return fail(PMOR_EINVAL, "re-anchoring is built for real problems");
  PMOR_HIP(hipSetDevice(pb->ctx->device));
  const auto t0 = std::chrono::steady_clock::now();
  if (stats) std::memset(stats, 0, sizeof(pmor_stats) * npts);
  std::vector<int> anchors{0};
  if (tol > 0.0) PMOR_TRY(plan_anchors(pb, pts.data(), npts, tol, &anchors));
  anchors.push_back(npts);
  int first_bad = PMOR_OK;
  for (size_t a = 0; a + 1 < anchors.size(); ++a) {
    const int l0 = anchors[a], cnt = anchors[a + 1] - l0;
    const int rc = sequence_run(pb, B, ldb, k, pts.data() + l0, cnt, X + (int64_t)l0 * pb->n * ldx, ldx, policy, sopts,
                                o, stats ? stats + l0 : nullptr, l0, t0);
    if (rc == PMOR_ESINGULAR || rc == PMOR_ENOTCONV || rc == PMOR_EBREAKDOWN || rc == PMOR_ENAN) {
      if (first_bad == PMOR_OK) first_bad = rc;
    } else if (rc != PMOR_OK) {
      return rc;
    }
  }
  return first_bad;
}
}  // namespace pmor

extern "C" {

int pmor_sequence_solve(pmor_problem* pb, const double* B, int64_t ldb, int32_t k, const double* s_list,
                        const double* p_list, int32_t npts, double* X, int64_t ldx, int32_t policy,
                        const pmor_spai_opts* sopts, const pmor_solve_opts* vopts, pmor_stats* stats) {
  if (!s_list || !p_list) return fail(PMOR_EINVAL, "NULL argument");
  return sequence_solve(pb, B, ldb, k, s_list, p_list, nullptr, npts, X, ldx, policy, sopts, vopts, stats);
}

int pmor_sequence_solve_c(pmor_problem* pb, const double* B, int64_t ldb, int32_t k, const double* coefs,
                          int32_t npts, double* X, int64_t ldx, int32_t policy, const pmor_spai_opts* sopts,
                          const pmor_solve_opts* vopts, pmor_stats* stats) {
  if (!coefs) return fail(PMOR_EINVAL, "NULL argument");
  return sequence_solve(pb, B, ldb, k, nullptr, nullptr, coefs, npts, X, ldx, policy, sopts, vopts, stats);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// serving: a queue of sequence jobs, admitted under a device-memory budget,
// whose points share one persistent block GMRES engine
// ---------------------------------------------------------------------------
namespace pmor {
struct ServerJob {
  int64_t id = 0;
  pmor_job job{};
  std::vector<Point> pts;
  double t_submit = 0.0;
  int64_t footprint = 0;
  pmor_spai* h = nullptr;
  SeqBuffers sb;
  std::vector<SolveItem> items;
  std::vector<int> bad;
  int remaining = 0;
  int status = PMOR_OK;
};

// device bytes a job holds while admitted (an upper bound: the shadow sizes
// are bounded by |J_j| times the longest column of A)
static int64_t job_footprint(const pmor_problem* pb, int npts, bool rowq) {
  const int64_t n = pb->n, nnz = pb->nnz, nnzP = pb->nnz;
  const int64_t sumI = nnzP * std::max<int64_t>(pb->max_col_len, 1);
  const int64_t spai = 8 * (3 * nnzP + nnz + 2 * n + 512) + 8 * (n + 1) + 4 * sumI +
                       4 * (3 * (n + 1) + 3 * nnzP + n) + 4096;
  const int64_t cap = pb->sell.cap;
  return spai + 3 * 8 * cap + SeqBuffers::estimate(npts, (rowq && cap > 0) ? 0 : nnz, rowq ? 0 : nnzP, n, cap,
                                                   rowq ? 0 : cap);
}

// the U-diag update policy keeps every P_l factored (no per-point P values)
static bool rows_scaled(const pmor_problem* pb, int policy, const pmor_spai_opts& so) {
  return policy == PMOR_UPDATE && so.update == PMOR_UPD_DIAG && !pb->cplx;
}
}  // namespace pmor

struct pmor_server {
  pmor_ctx* ctx = nullptr;
  pmor_spai_opts sopts{};
  pmor_solve_opts vopts{};
  int k = 1;
  int64_t budget = 0, engine_bytes = 0, in_use = 0, engine_rows = 0;
  int max_systems = 64;
  pmor::Engine* eng = nullptr;
  pmor::Runner* run = nullptr;
  std::deque<pmor::ServerJob*> queue;
  std::map<int64_t, pmor::ServerJob*> jobs;  // admitted
  std::deque<pmor::SolveItem*> waiting;
  std::deque<std::pair<int64_t, int>> reports;
  int64_t next_id = 1;
};

namespace pmor {
static void job_finish(pmor_server* sv, ServerJob* J) {
  spai_release(J->h);
  J->h = nullptr;
  pb_unref(J->job.pb);
  sv->in_use -= J->footprint;
  sv->reports.push_back({J->id, J->status});
  sv->jobs.erase(J->id);
  delete J;
}

// P_1, every point's A(l) and preconditioner; the points enter the waiting line
static int job_admit(pmor_server* sv, ServerJob* J) {
  const pmor_job& jb = J->job;
  const int npts = jb.npts;
  pmor_stats pre0{};
  pre0.bad_column = -1;
  sv->jobs[J->id] = J;
  int rc = spai_build_pt(jb.pb, J->pts[0], &sv->sopts, &J->h, &pre0);
  if (rc == PMOR_OK) {
    const bool rq = rows_scaled(jb.pb, jb.policy, J->h->opts);
    rc = J->sb.alloc(npts, (rq && jb.pb->sell.cap > 0) ? 0 : jb.pb->nnz, rq ? 0 : J->h->nnzP, jb.pb->n,
                     sv->ctx->stream, jb.pb->sell.cap, rq ? 0 : J->h->psell.cap);
  }
  J->items.assign(npts, SolveItem{});
  J->bad.assign(npts, -1);
  if (rc == PMOR_OK)
    rc = prepare_points(jb.pb, J->h, jb.policy, J->pts.data(), 0, npts, jb.B, jb.ldb, jb.k, jb.X, jb.ldx, jb.stats,
                        pre0, J->sb, J->items.data(), J->bad.data());
  if (rc == PMOR_EHIP) return rc;
  if (rc != PMOR_OK) {  // the job fails as a whole (singular anchor, no memory)
    J->status = rc;
    if (jb.stats)
      for (int l = 0; l < npts; ++l) jb.stats[l].t_solve_ms = sv->run->now_ms() - J->t_submit;
    job_finish(sv, J);
    return PMOR_OK;
  }
  J->remaining = 0;
  for (int l = 0; l < npts; ++l) {
    if (J->bad[l] >= 0) {
      if (J->status == PMOR_OK) J->status = PMOR_ESINGULAR;
      if (jb.stats) jb.stats[l].t_solve_ms = sv->run->now_ms() - J->t_submit;
      continue;
    }
    J->items[l].tag = (J->id << 20) | l;
    sv->waiting.push_back(&J->items[l]);
    ++J->remaining;
  }
  if (J->remaining == 0) job_finish(sv, J);
  return PMOR_OK;
}
}  // namespace pmor

extern "C" {

int pmor_server_create(pmor_ctx* ctx, const pmor_server_opts* opts, const pmor_spai_opts* sopts,
                       const pmor_solve_opts* vopts, pmor_server** out) {
  if (!ctx || !opts || !out) return fail(PMOR_EINVAL, "NULL argument");
  *out = nullptr;
  if (opts->k < 1 || opts->k > PMOR_KMAX) return fail(PMOR_EINVAL, "k must be in 1..16");
  if (opts->hbm_budget < 0 || opts->engine_rows < 0 || opts->max_systems < 0)
    return fail(PMOR_EINVAL, "negative server size");
  pmor_spai_opts so{};
  so.pattern = PMOR_PAT_A;
  so.precision = PMOR_F64;
  so.update = PMOR_UPD_DIAG;
  if (sopts) so = *sopts;
  if (so.pattern != PMOR_PAT_A) return fail(PMOR_EINVAL, "the server builds SPAI on the pattern of A");
  if (so.reanchor_tol != 0.0) return fail(PMOR_EINVAL, "re-anchoring is built for pmor_sequence_solve only");
  pmor_solve_opts o;
  PMOR_TRY(solve_opts_of(vopts, &o));
  PMOR_HIP(hipSetDevice(ctx->device));
  size_t fr0 = 0, tot = 0;
  PMOR_HIP(hipMemGetInfo(&fr0, &tot));
  pmor_server* sv = new pmor_server();
  sv->ctx = ctx;
  ctx_ref(ctx);
  sv->sopts = so;
  sv->vopts = o;
  sv->k = opts->k;
  sv->budget = opts->hbm_budget > 0 ? opts->hbm_budget : (int64_t)(0.75 * (double)fr0);
  sv->max_systems = opts->max_systems > 0 ? opts->max_systems : 64;
  const int kp = opts->k <= 1 ? 1 : opts->k <= 2 ? 2 : opts->k <= 4 ? 4 : opts->k <= 8 ? 8 : 16;
  sv->engine_rows = opts->engine_rows > 0 ? opts->engine_rows
                                          : (int64_t)(0.4 * (double)sv->budget / (8.0 * kp * (o.m + 8)));
  sv->eng = engine_new();
  int rc = runner_create(ctx, sv->eng, opts->k, o, sv->engine_rows, sv->max_systems, &sv->run);
  if (rc == PMOR_OK) {
    sv->engine_bytes = engine_bytes(sv->eng);
    if (sv->engine_bytes > sv->budget) rc = fail(PMOR_ENOMEM, "the engine alone exceeds the memory budget");
  }
  if (rc != PMOR_OK) {
    pmor_server_destroy(sv);
    return rc;
  }
  *out = sv;
  return PMOR_OK;
}

void pmor_server_destroy(pmor_server* sv) {
  if (!sv) return;
  (void)hipSetDevice(sv->ctx->device);
  (void)hipStreamSynchronize(sv->ctx->stream);
  delete sv->run;
  engine_destroy(sv->eng);
  for (auto& kv : sv->jobs) {
    spai_release(kv.second->h);
    pb_unref(kv.second->job.pb);
    delete kv.second;
  }
  for (ServerJob* J : sv->queue) {
    pb_unref(J->job.pb);
    delete J;
  }
  pmor_ctx* c = sv->ctx;
  delete sv;
  ctx_unref(c);
}

int pmor_server_submit(pmor_server* sv, const pmor_job* job, int64_t* job_id) {
  if (!sv || !job) return fail(PMOR_EINVAL, "NULL argument");
  std::vector<Point> pts;
  PMOR_TRY(sequence_checks(job->pb, job->B, job->ldb, job->k, job->s_list, job->p_list, job->coefs, job->npts, job->X,
                           job->ldx, job->policy, &pts));
  if (job->pb->ctx != sv->ctx) return fail(PMOR_EINVAL, "problem of another context");
  if (job->npts >= (1 << 20)) return fail(PMOR_EINVAL, "too many points in one job");
  if (job->k > sv->k) return fail(PMOR_EADMIT, "job wider than the server's block width");
  if ((int64_t)((job->pb->n + 15) / 16 * 16) > sv->engine_rows)
    return fail(PMOR_EADMIT, "system larger than the server's engine");
  ServerJob* J = new ServerJob();
  J->job = *job;
  J->pts.swap(pts);
  J->job.s_list = J->job.p_list = J->job.coefs = nullptr;  // host arrays copied: not referenced later
  J->footprint = job_footprint(job->pb, job->npts, rows_scaled(job->pb, job->policy, sv->sopts));
  if (J->footprint + sv->engine_bytes > sv->budget) {
    delete J;
    return fail(PMOR_EADMIT, "job footprint exceeds the server's memory budget");
  }
  J->id = sv->next_id++;
  J->t_submit = sv->run->now_ms();
  pb_ref(job->pb);
  if (job->stats) std::memset(job->stats, 0, sizeof(pmor_stats) * job->npts);
  sv->queue.push_back(J);
  if (job_id) *job_id = J->id;
  return PMOR_OK;
}

int pmor_server_step(pmor_server* sv, int64_t* done_ids, int32_t* done_status, int32_t max_done, int32_t* ndone) {
  if (!sv) return fail(PMOR_EINVAL, "NULL argument");
  if (ndone) *ndone = 0;
  PMOR_HIP(hipSetDevice(sv->ctx->device));
  // jobs, in order, while their footprint fits
  while (!sv->queue.empty()) {
    ServerJob* J = sv->queue.front();
    if (sv->in_use + J->footprint + sv->engine_bytes > sv->budget) break;
    sv->queue.pop_front();
    sv->in_use += J->footprint;
    PMOR_TRY(job_admit(sv, J));
  }
  // waiting points into the engine while rows and slots are free
  std::vector<SolveItem*> batch;
  while (!sv->waiting.empty()) {
    batch.push_back(sv->waiting.front());
    if (!sv->run->can_admit(batch.data(), (int)batch.size())) {
      batch.pop_back();
      break;
    }
    sv->waiting.pop_front();
  }
  if (!batch.empty()) PMOR_TRY(sv->run->admit(batch.data(), (int)batch.size()));
  // one restart cycle of every system in the engine
  if (sv->run->busy() > 0) {
    std::vector<SolveItem*> done;
    PMOR_TRY(sv->run->cycle(done));
    for (SolveItem* it : done) {
      auto f = sv->jobs.find(it->tag >> 20);
      if (f == sv->jobs.end()) continue;
      ServerJob* J = f->second;
      if (it->stats) it->stats->t_solve_ms = it->t_done_ms - J->t_submit;
      if (J->status == PMOR_OK && it->status != PMOR_OK) J->status = it->status;
      if (--J->remaining == 0) job_finish(sv, J);
    }
  }
  int nd = 0;
  while (!sv->reports.empty() && nd < max_done) {
    if (done_ids) done_ids[nd] = sv->reports.front().first;
    if (done_status) done_status[nd] = sv->reports.front().second;
    sv->reports.pop_front();
    ++nd;
  }
  if (ndone) *ndone = nd;
  return PMOR_OK;
}

int pmor_server_info(const pmor_server* sv, int32_t* queued, int32_t* admitted, int32_t* running,
                     int64_t* bytes_in_use) {
  if (!sv) return fail(PMOR_EINVAL, "NULL argument");
  if (queued) *queued = (int32_t)sv->queue.size();
  if (admitted) *admitted = (int32_t)sv->jobs.size();
  if (running) *running = sv->run ? sv->run->busy() : 0;
  if (bytes_in_use) *bytes_in_use = sv->in_use + sv->engine_bytes;
  return PMOR_OK;
}

}  // extern "C"

namespace pmor {
static int table2_norms_pt(pmor_problem* pb, const Point& q1, const Point& q2, double* fro_I_minus_A2,
                           double* fro_A1_minus_A2) {
  double* tmp = nullptr;
  PMOR_HIP(dmalloc((void**)&tmp, sizeof(double) * std::max<int64_t>(pb->nnz, 1), pb->ctx->stream));
  double a = 0.0, b = 0.0;
  const int rc = [&]() -> int {
    PMOR_TRY(ensure_assembled(pb, q1));
    PMOR_TRY(dcopy(pb->aval, tmp, pb->nnz, pb->ctx->stream));
    PMOR_TRY(ensure_assembled(pb, q2));
    PMOR_TRY(fro_norm2(pb, pb->aval, nullptr, pb->nnz, 1, &a));
    PMOR_TRY(fro_norm2(pb, tmp, pb->aval, pb->nnz, 0, &b));
    return PMOR_OK;
  }();
  dfree(tmp, pb->ctx->stream);
  if (rc != PMOR_OK) return rc;
  if (fro_I_minus_A2) *fro_I_minus_A2 = std::sqrt(a);
  if (fro_A1_minus_A2) *fro_A1_minus_A2 = std::sqrt(b);
  return PMOR_OK;
}
}  // namespace pmor

extern "C" {

int pmor_table2_norms(pmor_problem* pb, double s1, double p1, double s2, double p2, double* fro_I_minus_A2,
                      double* fro_A1_minus_A2) {
  if (!pb) return fail(PMOR_EINVAL, "problem is NULL");
  Point q1, q2;
  PMOR_TRY(point_sp(pb, s1, p1, &q1));
  PMOR_TRY(point_sp(pb, s2, p2, &q2));
  return table2_norms_pt(pb, q1, q2, fro_I_minus_A2, fro_A1_minus_A2);
}

int pmor_table2_norms_c(pmor_problem* pb, const double* coef1, const double* coef2, double* fro_I_minus_A2,
                        double* fro_A1_minus_A2) {
  if (!pb) return fail(PMOR_EINVAL, "problem is NULL");
  Point q1, q2;
  PMOR_TRY(point_coef(pb, coef1, &q1));
  PMOR_TRY(point_coef(pb, coef2, &q2));
  return table2_norms_pt(pb, q1, q2, fro_I_minus_A2, fro_A1_minus_A2);
}

int pmor_table2_norms_noalloc(pmor_problem* pb, double s1, double p1, double s2, double p2,
                              double* fro_I_minus_A2, double* fro_A1_minus_A2) {
  if (!pb) return fail(PMOR_EINVAL, "problem is NULL");
  const int dev = pb->ctx->device;
  double* scr = (dev >= 0 && dev < kMaxDevices) ? g_scratch_ptr[dev] : nullptr;
  if (!scr) return fail(PMOR_EHIP, "no scratch address for the context's device");
  static_assert(kT2Parts <= 256, "k_table2_sums adds at most 256 partials");
  Point q1, q2;
  PMOR_TRY(point_sp(pb, s1, p1, &q1));
  PMOR_TRY(point_sp(pb, s2, p2, &q2));
  T2Coefs cf{};
  cf.nt = pb->nterms;
  for (int t = 0; t < pb->nterms; ++t) {
    cf.c1[t] = q1.c[t];
    cf.c2[t] = q2.c[t];
  }
  hipStream_t st = pb->ctx->stream;
  hipLaunchKernelGGL(k_table2_partials, dim3(kT2Parts), dim3(256), 0, st, pb->n, pb->rowptr, pb->col,
                     (int64_t)pb->nnz, pb->tval, cf, scr);
  hipLaunchKernelGGL(k_table2_sums, dim3(2), dim3(256), 0, st, (const double*)scr, kT2Parts, scr + 2 * kT2Parts);
  PMOR_HIP(hipGetLastError());
  double h[2] = {0.0, 0.0};
  PMOR_HIP(hipMemcpyAsync(h, scr + 2 * kT2Parts, sizeof(h), hipMemcpyDeviceToHost, st));
  PMOR_HIP(hipStreamSynchronize(st));
  if (fro_I_minus_A2) *fro_I_minus_A2 = std::sqrt(h[0]);
  if (fro_A1_minus_A2) *fro_A1_minus_A2 = std::sqrt(h[1]);
  return PMOR_OK;
}

int pmor_spai_gather(const pmor_spai* h, double* colsum) {
  if (!h || !colsum) return fail(PMOR_EINVAL, "NULL argument");
  PMOR_HIP(hipSetDevice(h->pb->ctx->device));
  return run_spai_gather(const_cast<pmor_spai*>(h), colsum);
}

}  // extern "C"

namespace pmor {
// nread streams in; their element-wise sum out to NWR streams, or kept (the
// sink store never happens; it only keeps the loads)
template <int NB, int NWR>
__global__ __launch_bounds__(512) void k_stream_probe(const double* __restrict__ in, double* out, int64_t n,
                                                      double* sink) {
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double v[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) v[b] = __builtin_nontemporal_load(in + (int64_t)b * n + i);
    double s = 0.0;
#pragma unroll
    for (int b = 0; b < NB; ++b) s += v[b];
    if (NWR >= 1) out[i] = s;
    if (NWR >= 2) out[n + i] = 0.5 * s;
    if (NWR == 0) acc += s;
  }
  if (NWR == 0 && acc == -1.0) sink[0] = acc;
}

template <int NB>
static void launch_stream_probe(int nwr, unsigned grid, hipStream_t st, const double* in, double* out, int64_t n,
                                double* sink) {
  if (nwr == 0) hipLaunchKernelGGL((k_stream_probe<NB, 0>), dim3(grid), dim3(512), 0, st, in, out, n, sink);
  else if (nwr == 1) hipLaunchKernelGGL((k_stream_probe<NB, 1>), dim3(grid), dim3(512), 0, st, in, out, n, sink);
  else hipLaunchKernelGGL((k_stream_probe<NB, 2>), dim3(grid), dim3(512), 0, st, in, out, n, sink);
}
}  // namespace pmor

extern "C" {

int pmor_stream_probe(pmor_ctx* ctx, int32_t nread, int32_t nwrite, int64_t nbytes, int32_t reps, double* us) {
  if (!ctx || !us) return fail(PMOR_EINVAL, "NULL argument");
  if (!(nread >= 1 && (nread <= 8 || (nread <= 32 && nread % 4 == 0))))
    return fail(PMOR_EINVAL, "nread must be 1..8 or 12, 16, ..., 32");
  if (nwrite < 0 || nwrite > 2) return fail(PMOR_EINVAL, "nwrite must be 0, 1 or 2");
  if (nbytes <= 0 || nbytes % 8 != 0 || reps < 1) return fail(PMOR_EINVAL, "nbytes a positive multiple of 8, reps >= 1");
  PMOR_HIP(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  const int64_t n = nbytes / 8;
  double *in = nullptr, *out = nullptr;
  PMOR_HIP(hipMalloc((void**)&in, (size_t)nbytes * nread));
  if (hipMalloc((void**)&out, (size_t)nbytes * nwrite + 64) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(in);
    return fail(PMOR_ENOMEM, "stream probe: device memory");
  }
  int rc = PMOR_OK;
  float ms = 0.0f;
  if (hipMemsetAsync(in, 0, (size_t)nbytes * nread, st) != hipSuccess) rc = fail(PMOR_EHIP, "memset failed");
  const unsigned grid = 8192;
  double* sink = out + (int64_t)nwrite * n;
  auto pass = [&]() {
    switch (nread) {
      case 1: launch_stream_probe<1>(nwrite, grid, st, in, out, n, sink); break;
      case 2: launch_stream_probe<2>(nwrite, grid, st, in, out, n, sink); break;
      case 3: launch_stream_probe<3>(nwrite, grid, st, in, out, n, sink); break;
      case 4: launch_stream_probe<4>(nwrite, grid, st, in, out, n, sink); break;
      case 5: launch_stream_probe<5>(nwrite, grid, st, in, out, n, sink); break;
      case 6: launch_stream_probe<6>(nwrite, grid, st, in, out, n, sink); break;
      case 7: launch_stream_probe<7>(nwrite, grid, st, in, out, n, sink); break;
      case 8: launch_stream_probe<8>(nwrite, grid, st, in, out, n, sink); break;
      case 12: launch_stream_probe<12>(nwrite, grid, st, in, out, n, sink); break;
      case 16: launch_stream_probe<16>(nwrite, grid, st, in, out, n, sink); break;
      case 20: launch_stream_probe<20>(nwrite, grid, st, in, out, n, sink); break;
      case 24: launch_stream_probe<24>(nwrite, grid, st, in, out, n, sink); break;
      case 28: launch_stream_probe<28>(nwrite, grid, st, in, out, n, sink); break;
      default: launch_stream_probe<32>(nwrite, grid, st, in, out, n, sink); break;
    }
  };
  if (rc == PMOR_OK) {
    pass();
    pass();
    if (hipEventRecord(ctx->ev0, st) != hipSuccess) rc = fail(PMOR_EHIP, "event record failed");
    for (int r = 0; r < reps && rc == PMOR_OK; ++r) pass();
    if (rc == PMOR_OK && hipGetLastError() != hipSuccess) rc = fail(PMOR_EHIP, "stream probe launch failed");
    if (rc == PMOR_OK && (hipEventRecord(ctx->ev1, st) != hipSuccess || hipEventSynchronize(ctx->ev1) != hipSuccess ||
                          hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1) != hipSuccess))
      rc = fail(PMOR_EHIP, "event timing failed");
  }
  (void)hipStreamSynchronize(st);
  (void)hipFree(in);
  (void)hipFree(out);
  if (rc != PMOR_OK) return rc;
  *us = 1000.0 * (double)ms / reps;
  return PMOR_OK;
}

int pmor_prof_set(pmor_ctx* ctx, int kernel_id) {
  if (!ctx) return fail(PMOR_EINVAL, "ctx is NULL");
  if (kernel_id < 0 || kernel_id > PMOR_PROF_GCRO_GEMM) return fail(PMOR_EINVAL, "unknown kernel id");
  prof_collect(ctx);
  ctx->prof.kernel = kernel_id;
  ctx->prof.launches = 0;
  ctx->prof.total_ms = 0.0;
  ctx->prof.total_bytes = 0.0;
  return PMOR_OK;
}

int pmor_prof_read(pmor_ctx* ctx, int64_t* launches, double* total_ms, double* total_bytes) {
  if (!ctx) return fail(PMOR_EINVAL, "ctx is NULL");
  PMOR_HIP(hipStreamSynchronize(ctx->stream));
  prof_collect(ctx);
  if (launches) *launches = ctx->prof.launches;
  if (total_ms) *total_ms = ctx->prof.total_ms;
  if (total_bytes) *total_bytes = ctx->prof.total_bytes;
  ctx->prof.launches = 0;
  ctx->prof.total_ms = 0.0;
  ctx->prof.total_bytes = 0.0;
  return PMOR_OK;
}

int pmor_spmm(pmor_problem* pb, const double* aval, const double* X, int64_t ldx, double* Y, int64_t ldy, int32_t k,
              double alpha, double beta) {
  if (!pb || !aval || !X || !Y) return fail(PMOR_EINVAL, "NULL argument");
  if (k < 1 || k > PMOR_KMAX || ldx < k || ldy < k) return fail(PMOR_EINVAL, "bad k or leading dimension");
  const int pr = prof_start(pb->ctx, PMOR_PROF_SPMM_A);
  PMOR_TRY(launch_spmm(pb->n, pb->rowptr, pb->col, aval, X, ldx, Y, ldy, k, alpha, beta, Y, ldy, pb->ctx->stream,
                       pb->ctx, pr, 3));
  prof_stop(pb->ctx, pr, 12.0 * pb->nnz + 4.0 * (pb->n + 1) + 16.0 * pb->n * k + (beta != 0.0 ? 8.0 * pb->n * k : 0.0), 0);
  PMOR_HIP(hipStreamSynchronize(pb->ctx->stream));
  return PMOR_OK;
}

}  // extern "C"
