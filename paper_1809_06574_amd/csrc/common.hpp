// Shared definitions of the gfx950 library: handle layouts, device helpers,
// error plumbing.  Host code and kernels of every translation unit include it.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

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
// device state shared by the Krylov kernels of one solve
// ---------------------------------------------------------------------------
constexpr int KMAX = PMOR_KMAX;
constexpr int RED_GROUP = 16;   // workgroups per first-level reduction group
constexpr int MAX_RED_WG = 1024; // row-parallel kernels launch at most this many workgroups

struct DevState {
  int j;            // block steps completed in the current cycle
  int done;         // the cycle stops (converged, breakdown or max steps)
  int deficient;    // rank-deficient W met in the current step
  int breakdown;    // deficient with unconverged columns
  int kact;         // active right-hand sides (<= kp)
  int m;            // restart length
  int nanflag;
  int pad0;
  double tol;
  double wscale;    // max column norm of W = A Z of the current step
  double bnorm[KMAX];
  double est[KMAX]; // least-squares residual estimates / bnorm
  double R1[KMAX * KMAX];    // Cholesky factor, pass 1 (row-major, upper)
  double R1inv[KMAX * KMAX];
  double R2[KMAX * KMAX];
  double R2inv[KMAX * KMAX];
  int counters[2 * MAX_RED_WG / RED_GROUP + 8];  // last-block reduction arrivals
};

// ---------------------------------------------------------------------------
// handles
// ---------------------------------------------------------------------------
struct Workspace {
  int n = 0, kp = 0, m = 0;
  double* V = nullptr;      // (m+1) blocks of n x kp
  double* W = nullptr;      // n x kp
  double* Z = nullptr;      // n x kp
  double* T = nullptr;      // n x kp  (factored preconditioner temp / V Y)
  double* Bc = nullptr;     // n x kp  compacted right-hand sides
  double* Xc = nullptr;     // n x kp  compacted solution
  double* Hbar = nullptr;   // ((m+1) kp) x (m kp), column-major
  double* Hcol = nullptr;   // 2 x (m+1) kp x kp: CGS coefficients of both passes
  double* G = nullptr;      // ((m+1) kp) x kp, column-major (E1 S transformed)
  double* refl = nullptr;   // m kp reflectors, (kp + 2) doubles each
  double* Y = nullptr;      // (m kp) x kp, column-major
  double* part = nullptr;   // reduction partials
  double* part2 = nullptr;  // second-level partials
  double* partg = nullptr;  // per-workgroup partial Gram matrices (two sweeps)
  size_t part_len = 0;
  DevState* st = nullptr;
  DevState* st_host = nullptr;  // pinned mirror
  size_t bytes = 0;
};

// HIP-event timing of one chosen kernel class on the context's stream, with the
// algorithmic bytes each timed launch has to move (for roofline reports).
struct ProfRec {
  hipEvent_t a, b;
  double bytes;
  int tag;       // block step of the launch (skipped steps are discarded)
  bool valid;
};
struct Profiler {
  int kernel = 0;
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> spare;
  int64_t launches = 0;
  double total_ms = 0.0, total_bytes = 0.0;
};

}  // namespace pmor

struct pmor_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipEvent_t evs[64] = {};       // step events of the Krylov look-ahead
  pmor::Profiler prof;
};

struct pmor_problem {
  pmor_ctx* ctx = nullptr;
  int32_t n = 0, nnz = 0;
  int32_t* rowptr = nullptr;   // union pattern, CSR
  int32_t* col = nullptr;
  int32_t* maps = nullptr;     // PMOR_NROLES x nnz
  double* tval = nullptr;      // term values on the union pattern, one array per present role
  int role_slot[PMOR_NROLES];  // index into tval, or -1
  int nterms = 0;
  int32_t* colptr = nullptr;   // CSC view of the pattern
  int32_t* rowidx = nullptr;
  int32_t* cscslot = nullptr;  // CSC position -> CSR position
  int32_t max_row_len = 0, max_col_len = 0;
  double* aval = nullptr;      // values of the last assembled point
  double cur_s = 0, cur_p = 0;
  bool have_cur = false;
  pmor::Workspace ws;
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
  double* rho = nullptr;     // per-column least-squares residuals
  double* red = nullptr;     // reduction scratch
  int32_t* bucket_cols = nullptr;  // columns sorted into buckets
  int32_t bucket_count[8] = {0};
  int32_t bucket_off[8] = {0};
  int nbuckets = 0;
  bool identity_order = true;
  bool q_active = false;     // U-pattern update applied (apply Q (P_1 x))
  double s1 = 0, p1 = 0;
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

int ensure_assembled(pmor_problem* pb, double s, double p);
// kernel timing: start returns a record index (-1 when kernel class `kid` is not profiled)
int prof_start(pmor_ctx* c, int kid);
void prof_stop(pmor_ctx* c, int idx, double bytes, int tag);
void prof_drop_from(pmor_ctx* c, int first_idx, int tag_limit);
// let kernel `fn` use `bytes` of dynamic LDS (above the 64 KiB default)
int allow_lds(const void* fn, size_t bytes);
// device int set by a one-thread kernel (no pageable host source)
int set_device_int(int* p, int v, hipStream_t st);
int ensure_workspace(pmor_problem* pb, int kp, int m);
void free_workspace(pmor::Workspace& ws);

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
int launch_assemble(pmor_problem* pb, const double coef[PMOR_NROLES], double* out, hipStream_t st);
int build_union_pattern(pmor_problem* pb, const pmor_csr* const* terms);
int build_spai_sets(pmor_spai* h);
int run_spai_ls(pmor_spai* h, const double* aval, const double* rhs_aval, double* out_val,
                int32_t* bad_col, double* fro2);
int run_update_diag(pmor_spai* h, const double* aval_l, int32_t* bad_col, double* fro2);
int launch_spmm(int n, const int32_t* rowptr, const int32_t* col, const double* val,
                const double* X, int64_t ldx, double* Y, int64_t ldy, int kp, int kact,
                double alpha, double beta, const double* Bsrc, int64_t ldb,
                const DevState* st, hipStream_t stream, pmor_ctx* pc = nullptr, int pidx = -1,
                int ppart = 3);
int fro_norm2(pmor_problem* pb, const double* a, const double* b, int64_t len, int mode,
              double* out_host);
int krylov_solve(pmor_problem* pb, const pmor_spai* h, const double* B, int64_t ldb, int k,
                 double* X, int64_t ldx, const pmor_solve_opts& o, pmor_stats* stats);

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

// Deterministic two-level cross-workgroup sum.  Every workgroup of a kernel with
// G workgroups writes L partial values at part[g*L .. g*L+L) and calls this
// function (all threads).  The last workgroup of each group of RED_GROUP sums
// its group in order into part2; the last group reducer sums the groups in order
// into out[0..L).  Returns true in the single workgroup that produced out.
__device__ __forceinline__ bool lastblock_sum(double* part, double* part2, int L, int G, int g,
                                              int* counters, double* out) {
  __shared__ int s_flag;
  const int ngroups = (G + RED_GROUP - 1) / RED_GROUP;
  const int grp = g / RED_GROUP;
  const int gsize = min(RED_GROUP, G - grp * RED_GROUP);
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) s_flag = (atomicAdd(&counters[grp], 1) == gsize - 1);
  __syncthreads();
  if (!s_flag) return false;
  __threadfence();
  for (int t = threadIdx.x; t < L; t += blockDim.x) {
    double acc = 0.0;
    for (int q = 0; q < gsize; ++q) acc += part[(size_t)(grp * RED_GROUP + q) * L + t];
    if (ngroups == 1) out[t] = acc; else part2[(size_t)grp * L + t] = acc;
  }
  if (ngroups == 1) {
    __syncthreads();
    if (threadIdx.x == 0) counters[grp] = 0;
    return true;
  }
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    counters[grp] = 0;
    s_flag = (atomicAdd(&counters[ngroups], 1) == ngroups - 1);
  }
  __syncthreads();
  if (!s_flag) return false;
  __threadfence();
  for (int t = threadIdx.x; t < L; t += blockDim.x) {
    double acc = 0.0;
    for (int q = 0; q < ngroups; ++q) acc += part2[(size_t)q * L + t];
    out[t] = acc;
  }
  __syncthreads();
  if (threadIdx.x == 0) counters[ngroups] = 0;
  return true;
}

}  // namespace pmor
