// Shared definitions of the gfx950 library: handle layouts, device helpers,
// error plumbing.  Host code and kernels of every translation unit include it.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <cstring>

#include <string>
#include <vector>

#include "pmor_spai.h"

namespace pmor {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define PMOR_HIP(expr)                                  \
  do {                                                  \
    hipError_t _e = (expr);                             \
    if (_e != hipSuccess) return pmor::hip_fail(_e, #expr); \
  } while (0)

#define PMOR_TRY(expr)            \
  do {                            \
    int _rc = (expr);             \
    if (_rc != PMOR_OK) return _rc; \
  } while (0)

// ---------------------------------------------------------------------------
// Krylov engine: several independent systems ("segments") advance through the
// block GMRES cycle in lockstep; every kernel launch covers all of them.
// ---------------------------------------------------------------------------
constexpr int KMAX = PMOR_KMAX;
// A block column whose sine to the span of the columns before it is at most
// this is dependent.  Cholesky QR in FP64 resolves sines down to about 1e-7 for
// blocks of up to 2^22 rows (the Gram matrix carries a relative rounding error
// of about sqrt(n) eps), so the verdict does not hinge on the QR algorithm.
constexpr double kDepSine = 1e-6;

// per-segment device state of the current cycle
struct DevState {
  int j;            // block steps completed in the current cycle
  int done;         // the cycle stops (converged, breakdown or max steps)
  int deficient;    // rank-deficient W met in the current step
  int breakdown;    // deficient residual block at the cycle start
  int kact;         // active right-hand sides (<= kp)
  int m;            // restart length
  int nanflag;
  int pad0;
  double tol;
  double wscale;    // max column norm of W = A Z of the current step
  double bnorm[KMAX];
  double est[KMAX]; // least-squares residual estimates / bnorm
  double R1[KMAX * KMAX];     // first Cholesky factor of the step (row-major, upper)
  double R2inv[KMAX * KMAX];  // inverse of the second factor: V_{j+1} = W1 R2inv
  double R1inv[KMAX * KMAX];  // inverse of the first factor (pass 3: W1 = W'' R1inv)
};

// Sliced ELL view of a CSR pattern for the engine's SpMM: 64-row slices,
// column-major inside a slice (entry k of row r at ptr[r/64] + 64 k + r%64);
// padding entries point at their own row with value 0.  Built only when the
// padding stays small (stencil-like rows); cap = 0 means no view.
struct SellView {
  int32_t ns = 0;            // slices
  int64_t cap = 0;           // stored entries (with padding)
  int32_t* ptr = nullptr;    // ns + 1 slice offsets
  int32_t* wid = nullptr;    // ns slice widths
  int32_t* col = nullptr;    // cap columns, -1 for padding (a padded slot gathers nothing)
  int32_t* map = nullptr;    // cap: CSR position of the entry, -1 for padding
};

// one system of a batch (device copy read by every kernel)
struct SegDesc {
  int n;            // rows
  int kact;         // active (nonzero) right-hand sides
  int wg0, G;       // row-kernel workgroups [wg0, wg0 + G) of the logical grid
  int sp0, spG;     // SpMM workgroups [sp0, sp0 + spG)
  int pkind;        // preconditioner: 0 none, 1 P, 2 Q P_1 (factored), 3 diag(q) P_1 (row-scaled)
  int k;            // caller's columns
  int64_t r0;       // first row of the segment in the concatenated blocks
  const int32_t* arow;
  const int32_t* acol;
  const double* aval;
  const int32_t* prow;
  const int32_t* pcol;
  const double* pval;   // P, or P_1 when pkind == 2
  const double* qval;   // Q when pkind == 2
  const double* prs;    // q when pkind == 3 (n row scales)
  // sliced ELL copies (a_sp == nullptr / p_sp == nullptr: use the CSR arrays)
  const int32_t* a_sp;
  const int32_t* a_sw;
  const int32_t* a_sc;
  const double* a_sv;
  const int32_t* p_sp;
  const int32_t* p_sw;
  const int32_t* p_sc;
  const double* p_sv;
  const double* q_sv;
  const double* B;
  int64_t ldb;
  double* X;
  int64_t ldx;
  int cmap[KMAX];   // compacted column c holds caller column cmap[c]
  int cinv[KMAX];   // caller column c sits in compacted column cinv[c], or -1
  double bnorm[KMAX];
};

struct Engine;

// A point of a parametric family: the coefficient of every stored term of its
// problem in term-slot order, A = sum_t c[t] T_t (the affine form of Section
// 1.1, eq. affine_system; for a problem of roles the coefficients of
// s^2 M(p) + s D(p) + K(p)).
struct Point {
  double c[PMOR_TMAX];
};

// HIP-event timing of one chosen kernel class on the context's stream, with the
// algorithmic bytes each timed launch has to move (for roofline reports).
struct ProfRec {
  hipEvent_t a, b;
  double bytes;
  int tag;       // block step of the launch (-1: not a block-step kernel)
  bool valid;
  int e0, e1;    // per-segment byte entries [e0, e1) of a block-step launch
};
struct Profiler {
  int kernel = 0;
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> spare;
  std::vector<std::pair<int, double>> ent;  // (segment, bytes) of block-step launches
  int64_t launches = 0;
  double total_ms = 0.0, total_bytes = 0.0;
};

}  // namespace pmor

struct pmor_ctx {
  std::atomic<int> refs{1};      // the caller's reference + one per problem and server (batch calls take
                                 // references from worker threads)
  int device = 0;
  hipStream_t stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipEvent_t evs[64] = {};       // step events of the Krylov look-ahead
  pmor::Profiler prof;
  pmor::Engine* eng = nullptr;   // Krylov engine buffers (grown on demand)
};

struct pmor_problem {
  std::atomic<int> refs{1};    // the caller's reference + one per preconditioner and queued job
  pmor_ctx* ctx = nullptr;
  int32_t n = 0, nnz = 0;
  int32_t* rowptr = nullptr;   // union pattern, CSR
  int32_t* col = nullptr;
  int32_t* maps = nullptr;     // PMOR_NROLES x nnz
  double* tval = nullptr;      // term values on the union pattern, one array per stored term
  bool affine = false;         // created by pmor_problem_create_affine (points are coefficient vectors)
  int ncoef = 0;               // entries of a point's coefficient vector (PMOR_NROLES for a problem of roles)
  int coef_slot[2 * PMOR_TMAX];  // coefficient index -> index into tval, or -1 (absent role / excluded part)
  bool strict_coef = false;    // a coefficient without a term must be 0 (complex problems)
  bool cplx = false;           // equivalent real form of a complex problem (pmor_problem_create_complex)
  int nmaps = 0;               // rows of maps: PMOR_NROLES (roles) or nterms (affine)
  int nterms = 0;
  int32_t* colptr = nullptr;   // CSC view of the pattern
  int32_t* rowidx = nullptr;
  int32_t* cscslot = nullptr;  // CSC position -> CSR position
  int32_t max_row_len = 0, max_col_len = 0;
  double* aval = nullptr;      // values of the last assembled point
  pmor::SellView sell;         // sliced ELL view of the pattern (engine SpMM)
  double* aval_s = nullptr;    // aval in the sliced ELL layout
  pmor::Point cur{};           // the point aval holds
  bool have_cur = false;
};

struct pmor_spai {
  pmor_problem* pb = nullptr;
  pmor_spai_opts opts{};
  int32_t nnzP = 0;
  int32_t* Jcolptr = nullptr; int32_t* Jrow = nullptr;   // pattern of P (CSC)
  bool own_J = false;
  int64_t* Icolptr = nullptr; int32_t* Irow = nullptr;   // shadows (CSC)
  int64_t nI = 0;
  int32_t* Prowptr = nullptr; int32_t* Pcol = nullptr; int32_t* Pslot = nullptr;
  bool own_P = false;
  int32_t maxJ = 0, maxI = 0;
  double* Pval = nullptr;    // preconditioner applied (P_l for U-diag, P_1 for U-pattern)
  double* P1val = nullptr;   // anchor SPAI P_1
  double* Qval = nullptr;    // U-pattern: Q (P's CSR order); U-diag: q (n)
  double* aval1 = nullptr;   // anchor A(1)
  int32_t* esc_list = nullptr;  // adaptive update: escalated columns, per bucket at its offset (n)
  int32_t* esc_cnt = nullptr;   // adaptive update: escalated columns per bucket (8)
  double* rho = nullptr;     // per-column least-squares residuals
  double* red = nullptr;     // reduction scratch
  int32_t* bucket_cols = nullptr;  // columns sorted into buckets
  int32_t bucket_count[16] = {0};  // per least-squares bucket (slots 0..LS_BUCKETS-1 used)
  int32_t bucket_off[16] = {0};
  int32_t bucket_maxJ[16] = {0};  // largest |J_j| and |I_j| of each bucket (sizes the LDS kernels' launches)
  int32_t bucket_maxI[16] = {0};
  int nbuckets = 0;
  bool identity_order = true;
  bool q_active = false;     // U-pattern update applied (apply Q (P_1 x))
  bool d_active = false;     // U-diag update applied (apply diag(q) (P_1 x), q in Qval)
  bool c_active = false;     // complex U-diag update applied: P_l written out in Pval (Qval_s: its sliced ELL)
  pmor::Point pt1{};          // the anchor point
  pmor::SellView psell;      // sliced ELL view of P's pattern (the problem's for PAT_A)
  bool own_psell = false;
  double* P1val_s = nullptr;  // P1val (= Pval before an update) and Qval in the sliced ELL layout
  double* Qval_s = nullptr;
};

namespace pmor {

// coefficient of each role in A(s,p) = s^2 (M0 + p M1) + s (D0 + p D1) + K0 + p K1
inline void role_coefs(double s, double p, double c[PMOR_NROLES]) {
  c[PMOR_M0] = s * s;
  c[PMOR_M1] = s * s * p;
  c[PMOR_D0] = s;
  c[PMOR_D1] = s * p;
  c[PMOR_K0] = 1.0;
  c[PMOR_K1] = p;
}

// the point (s, p) of a problem of roles (PMOR_EINVAL for an affine problem or
// a non-finite s, p)
int point_sp(const pmor_problem* pb, double s, double p, Point* out);
// the point of the coefficient vector coef (pb->ncoef host values; PMOR_EINVAL
// when coef is NULL or a coefficient of a stored term is not finite)
int point_coef(const pmor_problem* pb, const double* coef, Point* out);
inline bool same_point(const Point& a, const Point& b, int nt) {
  return std::memcmp(a.c, b.c, sizeof(double) * nt) == 0;
}

// Lifetimes: a context lives until its caller and every problem and server of
// it have let it go; a problem until its caller and every preconditioner and
// server job of it have.  Destroy calls may therefore come in any order.
void ctx_ref(pmor_ctx* c);
void ctx_unref(pmor_ctx* c);
void pb_ref(pmor_problem* pb);
void pb_unref(pmor_problem* pb);

// device memory of the library: a cache with stream-ordered reuse (memory.hip)
hipError_t dmalloc(void** p, size_t bytes, hipStream_t s);
void dfree(void* p, hipStream_t s);
void dtrim();
// before a stream of the library or a caller's old stream is destroyed (it is complete)
void dstream_retire(hipStream_t s);

int ensure_assembled(pmor_problem* pb, const Point& pt);
// kernel timing: start returns a record index (-1 when kernel class `kid` is not profiled)
int prof_start(pmor_ctx* c, int kid);
void prof_stop(pmor_ctx* c, int idx, double bytes, int tag);
void prof_stop_seg(pmor_ctx* c, int idx, int tag, int e0);
// resolve the block-step records from first_idx on: a launch counts the bytes of
// the segments that still worked at its step (steps_of[seg] > tag)
void prof_resolve(pmor_ctx* c, int first_idx, const int* steps_of);
// let kernel `fn` use `bytes` of dynamic LDS (above the 64 KiB default)
int allow_lds(const void* fn, size_t bytes);
// device int set by a one-thread kernel (no pageable host source)
int set_device_int(int* p, int v, hipStream_t st);
void engine_destroy(Engine* e);

// Kernel launch that, for a profiled record idx >= 0, lets the dispatch itself
// timestamp the kernel into the record's events (part bit 1: start, bit 2: stop).
template <typename F, typename... Args>
inline void plaunch(pmor_ctx* c, int idx, int part, F kernel, dim3 g, dim3 b, uint32_t shm, hipStream_t s,
                    Args... args) {
  hipEvent_t ea = nullptr, eb = nullptr;
  if (c && idx >= 0) {
    const ProfRec& r = c->prof.recs[idx];
    if (part & 1) ea = r.a;
    if (part & 2) eb = r.b;
  }
  if (ea || eb) hipExtLaunchKernelGGL(kernel, g, b, shm, s, ea, eb, 0, args...);
  else hipLaunchKernelGGL(kernel, g, b, shm, s, args...);
}

// launchers implemented in the kernel translation units
int launch_assemble(pmor_problem* pb, const Point& pt, double* out, hipStream_t st);
// union pattern of terms[0..count) (NULL entries absent); maps rows: one per entry of terms
int build_union_pattern(pmor_problem* pb, const pmor_csr* const* terms, int count, hipStream_t st = nullptr);
// the SPAI index sets and buckets of h (on stream st, or the problem's when null)
int build_spai_sets(pmor_spai* h, hipStream_t st = nullptr);
// PMOR_EINVAL unless (rowptr, col) is an n x n CSR pattern of nnz entries with
// strictly increasing columns per row (synchronises)
int check_csr(int n, int64_t nnz, const int32_t* rowptr, const int32_t* col, hipStream_t st);
// the equivalent real form of complex term T (part 0: T (x) I_2, part 1:
// T (x) J_2), block-closed with the diagonal blocks; arrays allocated here
int real_equiv_term(const pmor_csr* T, int part, int32_t** rp2, int32_t** col2, double** val2, int32_t* nnz2,
                    hipStream_t st);
// PMOR_EINVAL unless the order-n CSR pattern is the real form of a complex one
int check_pairs(int n, const int32_t* rowptr, const int32_t* col, hipStream_t st);
// CSC view (colptr n+1, rowidx, slot: CSC position -> CSR position) allocated here
int transpose_pattern(int n, int64_t nnz, const int32_t* rowptr, const int32_t* col, int32_t** colptr,
                      int32_t** rowidx, int32_t** slot, int* maxcol, hipStream_t st);
// sliced ELL view of a CSR pattern when its padding is at most max_fill x nnz (else v->cap = 0)
// stored slots (padding included) allowed per nonzero before the CSR arrays
// serve instead: a padded slot costs its 12 bytes of column and value only
constexpr double SELL_MAX_FILL = 2.0;
// SELL_MAX_FILL, or PMOR_SELL_MAX_FILL when set (0: always the CSR arrays)
double sell_max_fill();
int build_sell(int n, const int32_t* rowptr, const int32_t* col, int64_t nnz, double max_fill, SellView* v,
               hipStream_t st);
void free_sell(SellView* v, hipStream_t st);
// dst (v->cap) = src (CSR order) permuted into the view; padding 0
int to_sell(const SellView& v, const double* src, double* dst, hipStream_t st);
int run_spai_ls(pmor_spai* h, const double* aval, const double* rhs_aval, double* out_val,
                int32_t* bad_col, double* fro2);
int run_update_diag(pmor_spai* h, const double* aval_l, int32_t* bad_col, double* fro2);
// the U-diag update of a complex problem (2x2 blocks of the real form): factors
// into q (n: Re, Im per complex column), residuals into rho (n), P_l = Q P_1 into pl
// the SPAI least squares of several handles (one stream, one precision) in
// shared bucketed launches; aval[i] the values of handle i's matrix
int run_spai_ls_multi(pmor_spai* const* hs, int count, const double* const* aval, hipStream_t st);
// block GCRO-DR of one system at pt, carrying rec's recycled basis (recycle.hip)
int gcrodr_solve(pmor_problem* pb, const pmor_spai* h, const Point& pt, const double* B, int64_t ldb, int k, double* X,
                 int64_t ldx, const pmor_solve_opts& o, pmor_recycle* rec, pmor_stats* stats);
int run_update_pair(pmor_spai* h, const double* aval_l, double* pl, double* q, double* rho, int32_t* bad_col,
                    double* fro2);
// every column's gathered block A(I_j, J_j) (anchor values) reduced to its sum in colsum (n, device)
int run_spai_gather(pmor_spai* h, double* colsum);
// adaptive Q (PMOR_UPD_ADAPTIVE): Q in P's CSR order into qout, residuals into h->rho;
// *n_esc (may be NULL) = escalated columns
int run_update_adaptive(pmor_spai* h, const double* aval_l, double* qout, int32_t* bad_col, double* fro2,
                        int64_t* n_esc);
// points of a sequence, at most PTS_MAX per call (pts: host array of cnt):
// A(l) into out + l * ostride (CSR order, or the sliced ELL layout of sv when not NULL);
// the U-diag factors q_l, rho_l (stride n) and the first zero column into bad[l]
// (bad must hold 0x7fffffff); per-point sums of squares into out[l * ostride]
constexpr int PTS_MAX = 8;
// least-squares buckets by (|J_j|, |I_j|): 0..7 register kernels (5..7: the LDS
// kernel in FP64), 8 the LDS kernel; BUCKET_SLOTS bounds the per-bucket arrays,
// its last slot counts unsupported columns
constexpr int LS_BUCKETS = 9;
constexpr int BUCKET_SLOTS = 16;
int launch_assemble_pts(pmor_problem* pb, const Point* pts, int cnt, const SellView* sv, double* out, int64_t ostride,
                        hipStream_t st);
int launch_update_diag_pts(pmor_spai* h, const Point* pts, int cnt, double* q, double* rho, int* bad, hipStream_t st);
int sumsq_pts(const double* x, int64_t n, int cnt, double* out, int64_t ostride, hipStream_t st);
// U-diag factors and column residuals of up to PTS_MAX points against the anchor values given
int launch_update_diag_pts_anchor(pmor_problem* pb, const double* anchor, const Point* pts, int cnt, double* q,
                                  double* rho, int* bad, hipStream_t st);
// U-diag update into caller buffers (no host synchronisation): P_l = diag(q) P_1
// into pl, q into q, column residuals into rho, the smallest failing column into
// *dbad (device int, must hold INT_MAX beforehand)
int launch_update_diag(pmor_spai* h, const double* aval_l, const double* anchor, const double* qprev, double* pl,
                       double* q, double* rho, int* dbad);
// pts: the whole sequence (point l0 - 1 is the first anchor)
int launch_update_diag_chain(pmor_spai* h, const Point* pts, int l0, int cnt, double* carry, double* q, double* rho,
                             int* bad, hipStream_t st);
int launch_spmm(int n, const int32_t* rowptr, const int32_t* col, const double* val,
                const double* X, int64_t ldx, double* Y, int64_t ldy, int k,
                double alpha, double beta, const double* Bsrc, int64_t ldb,
                hipStream_t stream, pmor_ctx* pc = nullptr, int pidx = -1, int ppart = 3);
// sum of squares of x[0..n) into dev_scratch[0] (dev_scratch: 258 doubles), deterministic
int sumsq(const double* x, int64_t n, double* dev_scratch, hipStream_t st);
int fro_norm2(pmor_problem* pb, const double* a, const double* b, int64_t len, int mode,
              double* out_host);
// one system of a batched solve
struct SolveItem {
  int n;
  int64_t nnzA, nnzP;
  const int32_t* arow;
  const int32_t* acol;
  const double* aval;
  int pkind;                  // 0 none, 1 P, 2 Q P_1, 3 diag(q) P_1
  const int32_t* prow;
  const int32_t* pcol;
  const double* pval;
  const double* qval;
  const double* prs;          // q of diag(q) P_1 (pkind 3)
  const SellView* asell;      // sliced ELL views (NULL or cap 0: none) and values in them
  const double* aval_s;
  const SellView* psell;
  const double* pval_s;
  const double* qval_s;
  const double* B;
  int64_t ldb;
  int k;
  double* X;
  int64_t ldx;
  pmor_stats* stats;          // may be NULL
  int status;                 // out: PMOR_OK / ENOTCONV / EBREAKDOWN / ENAN
  double t_done_ms;           // out: host time from the engine's start to completion
  int64_t tag;                // caller's bookkeeping
};

// A persistent block GMRES engine over a fixed block width: systems are
// admitted between cycles into free rows and slots; each cycle() advances all
// admitted systems by one restart cycle in lockstep; finished systems leave
// with their X written and status set.
struct Runner {
  virtual ~Runner() {}
  // PMOR_EADMIT (nothing admitted) when rows or slots are lacking; the items
  // must stay valid until cycle() returns them
  virtual int admit(SolveItem* const* items, int n) = 0;
  virtual bool can_admit(SolveItem* const* items, int n) const = 0;
  virtual int cycle(std::vector<SolveItem*>& done) = 0;
  virtual int busy() const = 0;       // admitted, not yet returned
  virtual double now_ms() const = 0;  // host time since the engine's start
};
Engine* engine_new();
int64_t engine_bytes(const Engine* e);
// an engine of block width pad(k) on buffers E for rows_cap concatenated rows and nslots systems
int runner_create(pmor_ctx* ctx, Engine* E, int k, const pmor_solve_opts& o, int64_t rows_cap, int nslots,
                  Runner** out);
// block GMRES(m) for every item, all items in lockstep (one launch per kernel per step)
int krylov_batch(pmor_ctx* ctx, SolveItem* items, int nitems, const pmor_solve_opts& o);

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double shfl_xor_d(double x, int mask) {
  return __shfl_xor(x, mask, 64);
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

template <typename T>
__device__ __forceinline__ T wave_max(T x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    T y = __shfl_xor(x, o, 64);
    x = x > y ? x : y;
  }
  return x;
}

// Broadcast the value held by lane q (q = 0..3) of each aligned group of four lanes.
template <int Q>
__device__ __forceinline__ double quad_bcast(double x) {
  constexpr int ctrl = Q * 0x55;  // quad_perm(Q, Q, Q, Q)
  int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), ctrl, 0xF, 0xF, false);
  int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), ctrl, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Workgroup-to-data mapping that keeps neighbouring workgroups on one XCD:
// the hardware deals consecutive workgroup ids round-robin over the 8 XCDs,
// so logical id = (id % 8) * (G / 8) + id / 8 gives each XCD a contiguous range.
__device__ __forceinline__ int xcd_swizzle(int id, int G) {
  if ((G & 7) != 0) return id;
  return (id & 7) * (G >> 3) + (id >> 3);
}

}  // namespace pmor
