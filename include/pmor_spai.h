/*
 * pmor_spai.h — C ABI of the MI355X (gfx950) library for preconditioned
 * parametric linear solves.
 *
 * What it computes (Singh & Ahuja, "Preconditioned Linear Solves for
 * Parametric Model Order Reduction"):
 *
 *   A(s,p) = s^2 M(p) + s D(p) + K(p)         Section 1.1 (frequency domain),
 *                                              Section 1.2 eq. loewner_eq2
 *   with M(p) = M0 + p M1, D(p) = D0 + p D1, K(p) = K0 + p K1;
 *
 *   P  = argmin ||I - A P||_F  (SPAI)          Section 2.2, one least-squares
 *                                              problem per column of P;
 *   P_l = Q_l P_1,  Q_l = argmin ||A(1) - A(l) Q||_F
 *                                              Section 2.3 (Table 1, first
 *                                              approach) and Section 2.4;
 *   A X = B by block GMRES(m), right-preconditioned (A P X~ = B, X = P X~)
 *                                              Section 2.1 and the footnote
 *                                              of Section 2.2;
 *   the sequence A(l) X(l) = B over points (s, p_l)
 *                                              Section 2.3, eq. general_sq.
 *
 * Conventions for every call:
 *  - Matrix and vector data pointers are DEVICE pointers owned by the caller
 *    (e.g. PyTorch tensors on the library's device).  The library never frees
 *    or retains caller memory beyond the call, except the term matrices given
 *    to pmor_problem_create, which are copied onto the union pattern there.
 *  - Sparse matrices are square, 0-based CSR with int32 row pointers and
 *    strictly increasing int32 column indices per row; values are FP64.
 *  - Dense blocks (B, X) are n x k row-major: element (i, c) at ptr[i*ld + c],
 *    ld >= k.
 *  - Handles (pmor_ctx, pmor_problem, pmor_spai) are owned by the library and
 *    released with their *_destroy / spai_free call.
 *  - All work is ordered on the context's HIP stream.  Calls that fill a
 *    pmor_stats or return a convergence verdict synchronise that stream.
 *  - Return value: PMOR_OK (0) or a negative PMOR_E* code.  No call aborts the
 *    process; pmor_last_error() gives a per-thread message for the last error.
 *  - Handles are not thread-safe: calls on one context must not overlap.
 */
#ifndef PMOR_SPAI_H
#define PMOR_SPAI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------- */
#define PMOR_OK 0
#define PMOR_EINVAL (-1)     /* invalid argument or malformed CSR              */
#define PMOR_ENOMEM (-2)     /* device allocation failed                       */
#define PMOR_ENOTCONV (-3)   /* max cycles reached; X holds the last iterate   */
#define PMOR_EBREAKDOWN (-4) /* rank-deficient block with unconverged columns  */
#define PMOR_ESINGULAR (-5)  /* a local least-squares problem is rank deficient*/
#define PMOR_ENAN (-6)       /* NaN or Inf met in a residual                   */
#define PMOR_EHIP (-7)       /* HIP runtime error (text in pmor_last_error)    */
#define PMOR_EADMIT (-8)     /* request does not fit the memory budget         */

#define PMOR_KMAX 16      /* largest block of right-hand sides                 */
#define PMOR_NROLES 6     /* number of term roles                              */
#define PMOR_MAX_CYCLES 64

/* Term roles: A(s,p) = s^2 (M0 + p M1) + s (D0 + p D1) + (K0 + p K1). */
enum pmor_role { PMOR_M0 = 0, PMOR_M1 = 1, PMOR_D0 = 2, PMOR_D1 = 3, PMOR_K0 = 4, PMOR_K1 = 5 };

/* SPAI sparsity pattern of P (columns J_j of P): */
#define PMOR_PAT_A 0        /* J_j = pattern of column j of A (incl. diagonal) */
#define PMOR_PAT_EXPLICIT 1 /* caller-given CSC pattern                        */
/* Arithmetic of the per-column least-squares problems: */
#define PMOR_F64 0
#define PMOR_F32 1
/* Update kinds (pattern of Q_l, which the paper leaves open): */
#define PMOR_UPD_DIAG 0     /* q_i has the single entry i: P_l = diag(q) P_1  */
#define PMOR_UPD_PATTERN 1  /* q_i on the SPAI pattern J_i, applied as Q_l(P_1 X) */
/* Sequence policies: */
#define PMOR_REBUILD 0      /* a new SPAI of A(l) for every point              */
#define PMOR_UPDATE 1       /* SPAI of A(1), then P_l = Q_l P_1                */

typedef struct pmor_ctx pmor_ctx;
typedef struct pmor_problem pmor_problem;
typedef struct pmor_spai pmor_spai;

/* A term matrix (device pointers, see conventions). */
typedef struct pmor_csr {
  int32_t n;
  int32_t nnz;
  const int32_t* rowptr; /* n+1 */
  const int32_t* col;    /* nnz */
  const double* val;     /* nnz */
} pmor_csr;

typedef struct pmor_spai_opts {
  int32_t pattern;            /* PMOR_PAT_A or PMOR_PAT_EXPLICIT                */
  int32_t precision;          /* PMOR_F64 or PMOR_F32                           */
  int32_t update;             /* PMOR_UPD_DIAG or PMOR_UPD_PATTERN              */
  int32_t nnz_explicit;       /* entries of the explicit pattern                */
  const int32_t* pat_colptr;  /* device, n+1; column j of P may hold rows       */
  const int32_t* pat_row;     /* pat_row[pat_colptr[j]..pat_colptr[j+1]), sorted,*/
                              /* must contain j                                  */
} pmor_spai_opts;

typedef struct pmor_solve_opts {
  int32_t m;          /* block steps per cycle (restart length), 1..64         */
  int32_t max_cycles; /* cycles before PMOR_ENOTCONV, 1..PMOR_MAX_CYCLES        */
  double tol;         /* per-column relative residual ||b-Ax||/||b||           */
} pmor_solve_opts;

typedef struct pmor_stats {
  int32_t k;                 /* right-hand sides solved                         */
  int32_t cycles;            /* restart cycles run                              */
  int32_t steps;             /* block steps, all cycles                         */
  int32_t bad_column;        /* PMOR_ESINGULAR: the offending column, else -1   */
  int32_t cycle_steps[PMOR_MAX_CYCLES];
  double relres[PMOR_KMAX];  /* final true relative residual per column          */
  double fro_resid;          /* build: ||I - A P||_F; update: ||A(1) - A(l)Q||_F */
                             /* (U-diag: with Q = diag(q))                        */
  double t_assemble_ms;      /* device time of the assembly of A(s,p)            */
  double t_precond_ms;       /* device time of the build or update               */
  double t_solve_ms;         /* wall time of block_solve                         */
} pmor_stats;

/* ---- context ----------------------------------------------------------- */
/* Create a context on HIP device `device` that orders its work on
 * `hip_stream` (a hipStream_t; NULL = the null stream).  Errors: PMOR_EHIP
 * when the device cannot be selected, PMOR_EINVAL for out == NULL. */
int pmor_ctx_create(pmor_ctx** out, int device, void* hip_stream);
void pmor_ctx_destroy(pmor_ctx* ctx);
/* Re-point the context at another stream of the same device. */
int pmor_ctx_set_stream(pmor_ctx* ctx, void* hip_stream);

/* ---- problem (one parametric system, Section 1.1 eq. (1)) ---------------- */
/* terms[r] for r in pmor_role: a term matrix, or NULL when absent.  All
 * present terms must share n.  Builds on the device the union pattern of the
 * terms plus the full diagonal (the pattern of every A(s,p), independent of
 * s and p), its CSC view, and copies the term values onto it.  The term
 * arrays are not referenced after the call returns.  Validation on the device:
 * monotone rowptr, nnz = rowptr[n], columns in range and strictly increasing
 * (PMOR_EINVAL otherwise).  Synchronises the stream. */
int pmor_problem_create(pmor_ctx* ctx, const pmor_csr* const* terms, pmor_problem** out);
void pmor_problem_destroy(pmor_problem* pb);
/* n and nnz of the union pattern (host outputs). */
int pmor_problem_info(const pmor_problem* pb, int32_t* n, int32_t* nnz);
/* Copy the union pattern into caller buffers (device): rowptr (n+1), col (nnz)
 * and maps (PMOR_NROLES*nnz; maps[r*nnz + e] = position of A-slot e in term r's
 * value array, -1 where term r has no entry or is absent).  Any output may be
 * NULL. */
int pmor_problem_pattern(const pmor_problem* pb, int32_t* rowptr, int32_t* col, int32_t* maps);
/* Values of A(s,p) on the union pattern into val (device, nnz). */
int pmor_assemble(pmor_problem* pb, double s, double p, double* val);

/* ---- SPAI (Section 2.2) and its update (Sections 2.3-2.4) ---------------- */
/* Build P = argmin ||I - A(s,p) P||_F on the chosen pattern; (s,p) becomes
 * the anchor A(1) of later updates.  Each column j solves
 * min ||e_j(I_j) - A(I_j,J_j) p||_2 by Householder QR, I_j being the rows of
 * A(:,J_j) that hold a nonzero.  opts may be NULL (defaults: PMOR_PAT_A,
 * PMOR_F64, PMOR_UPD_DIAG).  stats may be NULL; when given, the call
 * synchronises and fills fro_resid and t_* fields.  PMOR_ESINGULAR (with
 * stats->bad_column) when |R_kk| <= 10 |I_j| eps max|R| in some column;
 * PMOR_EINVAL when a column's |J_j| or |I_j| exceeds the supported 64 / 256. */
int spai_build(pmor_problem* pb, double s, double p, const pmor_spai_opts* opts,
               pmor_spai** out, pmor_stats* stats);
/* First-approach update at (s,p): Q = argmin ||A(1) - A(s,p) Q||_F on the
 * handle's update pattern; then P = Q P_1 (anchor unchanged).  Errors as
 * spai_build. */
int spai_update(pmor_spai* h, double s, double p, pmor_stats* stats);
/* Recompute the SPAI of A(s,p) in place (the rebuild policy); the anchor is
 * moved to (s,p). */
int spai_rebuild(pmor_spai* h, double s, double p, pmor_stats* stats);
/* The current preconditioner.  P in CSR: rowptr (n+1), col (nnzP), val (nnzP);
 * for PMOR_UPD_PATTERN after an update, val holds P_1 and qval holds Q (same
 * CSR pattern), and the preconditioner is Q P_1; for PMOR_UPD_DIAG, qval (n)
 * holds the diagonal q of the last update (ones before).  rho (n): per-column
 * least-squares residual of the last build or update.  Any output may be NULL;
 * device pointers. */
int spai_info(const pmor_spai* h, int32_t* nnzP, int32_t* maxJ, int32_t* maxI);
int spai_export(const pmor_spai* h, int32_t* rowptr, int32_t* col, double* val,
                double* qval, double* rho);
/* The index sets: J in CSC (colptr n+1, row nnzP) and I in CSC (colptr n+1
 * as int64, row sum|I_j|). */
int spai_export_sets(const pmor_spai* h, int32_t* J_colptr, int32_t* J_row,
                     int64_t* I_colptr, int32_t* I_row, int64_t* nI);
void spai_free(pmor_spai* h);

/* ---- block solve (Section 2.1) ------------------------------------------ */
/* Solve A(s,p) X = B with block GMRES(m) right-preconditioned by h's current
 * preconditioner (h may be NULL: no preconditioner).  X0 = 0.  B, X: n x k
 * row-major device blocks (k in 1..PMOR_KMAX); B is not modified.  Columns of
 * B that are zero get X = 0.  Converged when every column reaches
 * ||b_c - A x_c|| <= tol ||b_c||.  opts NULL: m = 30, tol = 1e-8,
 * max_cycles = 20.  Returns PMOR_ENOTCONV (X = last iterate),
 * PMOR_EBREAKDOWN or PMOR_ENAN on failure.  Synchronises the stream. */
int block_solve(pmor_problem* pb, const pmor_spai* h, double s, double p,
                const double* B, int64_t ldb, int32_t k, double* X, int64_t ldx,
                const pmor_solve_opts* opts, pmor_stats* stats);

/* The whole sequence of Section 2.3 for points (s_list[l], p_list[l]),
 * l < npts: preconditioner at point 0 by spai_build, then for l >= 1 either
 * spai_update (PMOR_UPDATE) or spai_rebuild (PMOR_REBUILD), then block_solve.
 * X: npts consecutive n x k row-major blocks (ldx per block, block stride
 * n*ldx).  stats: npts entries (may be NULL).  Stops at the first error. */
int pmor_sequence_solve(pmor_problem* pb, const double* B, int64_t ldb, int32_t k,
                        const double* s_list, const double* p_list, int32_t npts,
                        double* X, int64_t ldx, int32_t policy,
                        const pmor_spai_opts* sopts, const pmor_solve_opts* vopts,
                        pmor_stats* stats);

/* ---- diagnostics (Section 3.1, Table 2) -------------------------------- */
/* ||I - A(s,p)||_F and ||A(s1,p1) - A(s2,p2)||_F (host outputs; synchronises). */
int pmor_table2_norms(pmor_problem* pb, double s1, double p1, double s2, double p2,
                      double* fro_I_minus_A2, double* fro_A1_minus_A2);

/* ---- kernel-level entry points (timing and parity) --------------------- */
/* Y = beta*Y + alpha*A(s,p)-values-on-pattern * X, with the values in aval
 * (device, nnz) on pb's pattern; X, Y: n x k row-major, ld >= k. */
int pmor_spmm(pmor_problem* pb, const double* aval, const double* X, int64_t ldx,
              double* Y, int64_t ldy, int32_t k, double alpha, double beta);

/* ---- kernel timing (benchmarks) ---------------------------------------- */
/* Time every launch of one kernel class with HIP events recorded on the
 * context's stream around it, and add up the algorithmic bytes each launch must
 * move (the formulas are the library's roofline model).  kernel_id 0 turns the
 * timing off.  Launches of block steps that a converged cycle skipped are not
 * counted.  pmor_prof_read synchronises the stream, returns the totals since the
 * last read and resets them. */
#define PMOR_PROF_SPMM_A 1        /* W = A Z in a block step: 12 nnz + 4(n+1) + 16 n kp */
#define PMOR_PROF_CGS_UPD_DOT 2   /* Gram-Schmidt pass 2: W -= V H; V^T W: 8 n kp (nblk + 2) */
#define PMOR_PROF_CGS_DOT 3       /* Gram-Schmidt pass 1: V^T W: 8 n kp (nblk + 1) */
#define PMOR_PROF_SPAI_LS 4       /* SPAI least squares: 12 nnz + 4 n + 4 (sum|I_j| + nnzP) + 8 nnzP + 8 n */
#define PMOR_PROF_SPMM_P 5        /* Z = P V_j in a block step: 12 nnzP + 4(n+1) + 16 n kp */
#define PMOR_PROF_CGS_UPD_GRAM 6  /* Gram-Schmidt pass 3: W -= V H; W^T W: 8 n kp (nblk + 2) */
int pmor_prof_set(pmor_ctx* ctx, int kernel_id);
int pmor_prof_read(pmor_ctx* ctx, int64_t* launches, double* total_ms, double* total_bytes);

/* ---- errors ------------------------------------------------------------ */
const char* pmor_strerror(int code);
const char* pmor_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PMOR_SPAI_H */
