// The C ABI: argument checks, handle lifetimes, the sequence driver of the
// paper's eq. general_sq (Section 2.3), error reporting.  No arithmetic of the
// method lives here; every step runs in the kernels of the other files.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>

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
  r.tag = tag;
}

void prof_drop_from(pmor_ctx* c, int first_idx, int tag_limit) {
  auto& recs = c->prof.recs;
  for (size_t i = (first_idx < 0 ? 0 : first_idx); i < recs.size(); ++i)
    if (recs[i].tag >= tag_limit) recs[i].valid = false;
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
}

int ensure_assembled(pmor_problem* pb, double s, double p) {
  if (pb->have_cur && pb->cur_s == s && pb->cur_p == p) return PMOR_OK;
  double c[PMOR_NROLES];
  role_coefs(s, p, c);
  PMOR_TRY(launch_assemble(pb, c, pb->aval, pb->ctx->stream));
  pb->cur_s = s;
  pb->cur_p = p;
  pb->have_cur = true;
  return PMOR_OK;
}

static bool is_fin(double x) { return std::isfinite(x); }

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
  if (h->own_J) { (void)hipFree(h->Jcolptr); (void)hipFree(h->Jrow); }
  if (h->own_P) { (void)hipFree(h->Prowptr); (void)hipFree(h->Pcol); (void)hipFree(h->Pslot); }
  double* d[] = {h->Pval, h->P1val, h->Qval, h->aval1, h->rho, h->red};
  for (double* x : d)
    if (x) (void)hipFree(x);
  if (h->Icolptr) (void)hipFree(h->Icolptr);
  if (h->Irow) (void)hipFree(h->Irow);
  if (h->bucket_cols) (void)hipFree(h->bucket_cols);
  delete h;
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

// P_1 of A(s,p) into h (anchor moved to (s,p))
static int build_into(pmor_spai* h, double s, double p, pmor_stats* stats) {
  pmor_problem* pb = h->pb;
  hipStream_t st = pb->ctx->stream;
  Timer ta(pb->ctx, stats != nullptr);
  PMOR_TRY(ensure_assembled(pb, s, p));
  const double t_asm = ta.stop();
  Timer tp(pb->ctx, stats != nullptr);
  PMOR_TRY(dcopy(pb->aval, h->aval1, pb->nnz, st));
  int32_t bad = -1;
  double fro2 = 0.0;
  PMOR_TRY(run_spai_ls(h, pb->aval, nullptr, h->P1val, &bad, stats ? &fro2 : nullptr));
  PMOR_TRY(dcopy(h->P1val, h->Pval, h->nnzP, st));
  if (h->opts.update == PMOR_UPD_DIAG) PMOR_TRY(dfill(h->Qval, pb->n, 1.0, st));
  h->q_active = false;
  h->s1 = s;
  h->p1 = p;
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
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  prof_collect(c);
  for (hipEvent_t e : c->prof.spare) (void)hipEventDestroy(e);
  (void)hipEventDestroy(c->ev0);
  (void)hipEventDestroy(c->ev1);
  for (int i = 0; i < 64; ++i)
    if (c->evs[i]) (void)hipEventDestroy(c->evs[i]);
  delete c;
}

int pmor_ctx_set_stream(pmor_ctx* c, void* hip_stream) {
  if (!c) return fail(PMOR_EINVAL, "ctx is NULL");
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  return PMOR_OK;
}

int pmor_problem_create(pmor_ctx* ctx, const pmor_csr* const* terms, pmor_problem** out) {
  if (!ctx || !terms || !out) return fail(PMOR_EINVAL, "NULL argument");
  *out = nullptr;
  int n = -1;
  for (int r = 0; r < PMOR_NROLES; ++r) {
    const pmor_csr* T = terms[r];
    if (!T) continue;
    if (T->n <= 0) return fail(PMOR_EINVAL, "term dimension must be positive");
    if (T->nnz < 0) return fail(PMOR_EINVAL, "negative nnz");
    if (!T->rowptr || (T->nnz > 0 && (!T->col || !T->val))) return fail(PMOR_EINVAL, "term with NULL arrays");
    if (n >= 0 && T->n != n) return fail(PMOR_EINVAL, "terms differ in n");
    n = T->n;
  }
  if (n < 0) return fail(PMOR_EINVAL, "no term given");
  PMOR_HIP(hipSetDevice(ctx->device));
  pmor_problem* pb = new pmor_problem();
  pb->ctx = ctx;
  pb->n = n;
  int rc = build_union_pattern(pb, terms);
  if (rc != PMOR_OK) {
    pmor_problem_destroy(pb);
    return rc;
  }
  *out = pb;
  return PMOR_OK;
}

void pmor_problem_destroy(pmor_problem* pb) {
  if (!pb) return;
  int32_t* ip[] = {pb->rowptr, pb->col, pb->maps, pb->colptr, pb->rowidx, pb->cscslot};
  for (int32_t* x : ip)
    if (x) (void)hipFree(x);
  if (pb->tval) (void)hipFree(pb->tval);
  if (pb->aval) (void)hipFree(pb->aval);
  free_workspace(pb->ws);
  delete pb;
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
    PMOR_HIP(hipMemcpyAsync(maps, pb->maps, sizeof(int32_t) * PMOR_NROLES * (size_t)pb->nnz, hipMemcpyDeviceToDevice, s));
  PMOR_HIP(hipStreamSynchronize(s));
  return PMOR_OK;
}

int pmor_assemble(pmor_problem* pb, double s, double p, double* val) {
  if (!pb || !val) return fail(PMOR_EINVAL, "NULL argument");
  if (!is_fin(s) || !is_fin(p)) return fail(PMOR_EINVAL, "s and p must be finite");
  PMOR_TRY(ensure_assembled(pb, s, p));
  PMOR_TRY(dcopy(pb->aval, val, pb->nnz, pb->ctx->stream));
  PMOR_HIP(hipStreamSynchronize(pb->ctx->stream));
  return PMOR_OK;
}

int spai_build(pmor_problem* pb, double s, double p, const pmor_spai_opts* opts, pmor_spai** out,
               pmor_stats* stats) {
  if (!pb || !out) return fail(PMOR_EINVAL, "NULL argument");
  *out = nullptr;
  if (!is_fin(s) || !is_fin(p)) return fail(PMOR_EINVAL, "s and p must be finite");
  pmor_spai_opts o{};
  o.pattern = PMOR_PAT_A;
  o.precision = PMOR_F64;
  o.update = PMOR_UPD_DIAG;
  if (opts) o = *opts;
  if (o.pattern != PMOR_PAT_A && o.pattern != PMOR_PAT_EXPLICIT) return fail(PMOR_EINVAL, "bad pattern kind");
  if (o.precision != PMOR_F64 && o.precision != PMOR_F32) return fail(PMOR_EINVAL, "bad precision");
  if (o.update != PMOR_UPD_DIAG && o.update != PMOR_UPD_PATTERN) return fail(PMOR_EINVAL, "bad update kind");
  PMOR_HIP(hipSetDevice(pb->ctx->device));
  pmor_spai* h = new pmor_spai();
  h->pb = pb;
  h->opts = o;
  int rc = build_spai_sets(h);
  if (rc == PMOR_OK) {
    const int64_t n = pb->n;
    auto al = [&](double** p, int64_t cnt) {
      return hipMalloc((void**)p, sizeof(double) * std::max<int64_t>(cnt, 1)) == hipSuccess;
    };
    bool ok = al(&h->Pval, h->nnzP) && al(&h->P1val, h->nnzP) &&
              al(&h->Qval, o.update == PMOR_UPD_PATTERN ? h->nnzP : n) && al(&h->aval1, pb->nnz) &&
              al(&h->rho, n) && al(&h->red, 512);
    rc = ok ? build_into(h, s, p, stats) : fail(PMOR_ENOMEM, "preconditioner allocation failed");
  }
  if (rc != PMOR_OK && rc != PMOR_ESINGULAR) {
    spai_release(h);
    return rc;
  }
  *out = h;  // on PMOR_ESINGULAR the handle is returned so the caller can inspect it
  return rc;
}

int spai_update(pmor_spai* h, double s, double p, pmor_stats* stats) {
  if (!h) return fail(PMOR_EINVAL, "handle is NULL");
  if (!is_fin(s) || !is_fin(p)) return fail(PMOR_EINVAL, "s and p must be finite");
  pmor_problem* pb = h->pb;
  Timer ta(pb->ctx, stats != nullptr);
  PMOR_TRY(ensure_assembled(pb, s, p));
  const double t_asm = ta.stop();
  Timer tp(pb->ctx, stats != nullptr);
  int32_t bad = -1;
  double fro2 = 0.0;
  if (h->opts.update == PMOR_UPD_DIAG) {
    PMOR_TRY(run_update_diag(h, pb->aval, &bad, stats ? &fro2 : nullptr));
  } else {
    PMOR_TRY(run_spai_ls(h, pb->aval, h->aval1, h->Qval, &bad, stats ? &fro2 : nullptr));
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

int spai_rebuild(pmor_spai* h, double s, double p, pmor_stats* stats) {
  if (!h) return fail(PMOR_EINVAL, "handle is NULL");
  if (!is_fin(s) || !is_fin(p)) return fail(PMOR_EINVAL, "s and p must be finite");
  return build_into(h, s, p, stats);
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
    const double* src = (h->opts.update == PMOR_UPD_PATTERN) ? h->P1val : h->Pval;
    PMOR_HIP(hipMemcpyAsync(val, src, sizeof(double) * h->nnzP, hipMemcpyDeviceToDevice, s));
  }
  if (qval) {
    const int64_t len = (h->opts.update == PMOR_UPD_PATTERN) ? h->nnzP : n;
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

int block_solve(pmor_problem* pb, const pmor_spai* h, double s, double p, const double* B, int64_t ldb, int32_t k,
                double* X, int64_t ldx, const pmor_solve_opts* opts, pmor_stats* stats) {
  if (!pb || !B || !X) return fail(PMOR_EINVAL, "NULL argument");
  if (k < 1 || k > PMOR_KMAX) return fail(PMOR_EINVAL, "k must be in 1..16");
  if (ldb < k || ldx < k) return fail(PMOR_EINVAL, "leading dimension smaller than k");
  if (h && h->pb != pb) return fail(PMOR_EINVAL, "preconditioner belongs to another problem");
  if (!is_fin(s) || !is_fin(p)) return fail(PMOR_EINVAL, "s and p must be finite");
  pmor_solve_opts o{30, 20, 1e-8};
  if (opts) o = *opts;
  if (o.m < 1 || o.m > 31) return fail(PMOR_EINVAL, "m must be in 1..31");
  if (o.max_cycles < 1 || o.max_cycles > PMOR_MAX_CYCLES) return fail(PMOR_EINVAL, "max_cycles out of range");
  if (!(o.tol > 0.0) || !is_fin(o.tol)) return fail(PMOR_EINVAL, "tol must be positive");
  PMOR_HIP(hipSetDevice(pb->ctx->device));
  auto t0 = std::chrono::steady_clock::now();
  PMOR_TRY(ensure_assembled(pb, s, p));
  if (stats) std::memset(stats->cycle_steps, 0, sizeof(stats->cycle_steps));
  int rc = krylov_solve(pb, h, B, ldb, k, X, ldx, o, stats);
  if (stats) {
    stats->t_solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return rc;
}

int pmor_sequence_solve(pmor_problem* pb, const double* B, int64_t ldb, int32_t k, const double* s_list,
                        const double* p_list, int32_t npts, double* X, int64_t ldx, int32_t policy,
                        const pmor_spai_opts* sopts, const pmor_solve_opts* vopts, pmor_stats* stats) {
  if (!pb || !B || !X || !s_list || !p_list) return fail(PMOR_EINVAL, "NULL argument");
  if (npts < 1) return fail(PMOR_EINVAL, "npts must be positive");
  if (policy != PMOR_REBUILD && policy != PMOR_UPDATE) return fail(PMOR_EINVAL, "bad policy");
  pmor_spai* h = nullptr;
  int rc = PMOR_OK;
  for (int l = 0; l < npts && rc == PMOR_OK; ++l) {
    pmor_stats* stl = stats ? &stats[l] : nullptr;
    pmor_stats pre{};
    if (l == 0) rc = spai_build(pb, s_list[0], p_list[0], sopts, &h, stl ? &pre : nullptr);
    else if (policy == PMOR_UPDATE) rc = spai_update(h, s_list[l], p_list[l], stl ? &pre : nullptr);
    else rc = spai_rebuild(h, s_list[l], p_list[l], stl ? &pre : nullptr);
    if (rc != PMOR_OK) break;
    rc = block_solve(pb, h, s_list[l], p_list[l], B, ldb, k, X + (int64_t)l * pb->n * ldx, ldx, vopts, stl);
    if (stl) {
      stl->fro_resid = pre.fro_resid;
      stl->t_assemble_ms = pre.t_assemble_ms;
      stl->t_precond_ms = pre.t_precond_ms;
      stl->bad_column = pre.bad_column;
    }
  }
  spai_release(h);
  return rc;
}

int pmor_table2_norms(pmor_problem* pb, double s1, double p1, double s2, double p2, double* fro_I_minus_A2,
                      double* fro_A1_minus_A2) {
  if (!pb) return fail(PMOR_EINVAL, "problem is NULL");
  double* tmp = nullptr;
  PMOR_HIP(hipMalloc((void**)&tmp, sizeof(double) * std::max<int64_t>(pb->nnz, 1)));
  PMOR_TRY(ensure_assembled(pb, s1, p1));
  PMOR_TRY(dcopy(pb->aval, tmp, pb->nnz, pb->ctx->stream));
  PMOR_TRY(ensure_assembled(pb, s2, p2));
  double a = 0.0, b = 0.0;
  PMOR_TRY(fro_norm2(pb, pb->aval, nullptr, pb->nnz, 1, &a));
  PMOR_TRY(fro_norm2(pb, tmp, pb->aval, pb->nnz, 0, &b));
  (void)hipFree(tmp);
  if (fro_I_minus_A2) *fro_I_minus_A2 = std::sqrt(a);
  if (fro_A1_minus_A2) *fro_A1_minus_A2 = std::sqrt(b);
  return PMOR_OK;
}

int pmor_prof_set(pmor_ctx* ctx, int kernel_id) {
  if (!ctx) return fail(PMOR_EINVAL, "ctx is NULL");
  if (kernel_id < 0 || kernel_id > PMOR_PROF_CGS_UPD_GRAM) return fail(PMOR_EINVAL, "unknown kernel id");
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
  PMOR_TRY(launch_spmm(pb->n, pb->rowptr, pb->col, aval, X, ldx, Y, ldy, k, k, alpha, beta, Y, ldy, nullptr,
                       pb->ctx->stream, pb->ctx, pr, 3));
  prof_stop(pb->ctx, pr, 12.0 * pb->nnz + 4.0 * (pb->n + 1) + 16.0 * pb->n * k + (beta != 0.0 ? 8.0 * pb->n * k : 0.0), 0);
  PMOR_HIP(hipStreamSynchronize(pb->ctx->stream));
  return PMOR_OK;
}

}  // extern "C"
