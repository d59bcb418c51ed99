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
#define PMOR_EBREAKDOWN (-4) /* dependent residual block at a cycle start      */
#define PMOR_ESINGULAR (-5)  /* a local least-squares problem is rank deficient*/
#define PMOR_ENAN (-6)       /* NaN or Inf met in a residual                   */
#define PMOR_EHIP (-7)       /* HIP runtime error (text in pmor_last_error)    */
#define PMOR_EADMIT (-8)     /* request does not fit the memory budget         */

#define PMOR_KMAX 16      /* largest block of right-hand sides                 */
#define PMOR_NROLES 6     /* number of term roles                              */
#define PMOR_TMAX 16      /* most (real) terms of an affine problem            */
#define PMOR_MAX_CYCLES 64

/* Term roles: A(s,p) = s^2 (M0 + p M1) + s (D0 + p D1) + (K0 + p K1). */
enum pmor_role { PMOR_M0 = 0, PMOR_M1 = 1, PMOR_D0 = 2, PMOR_D1 = 3, PMOR_K0 = 4, PMOR_K1 = 5 };

/* SPAI sparsity pattern of P (columns J_j of P): */
#define PMOR_PAT_A 0        /* J_j = pattern of column j of A (incl. diagonal) */
#define PMOR_PAT_EXPLICIT 1 /* caller-given CSC pattern                        */
/* Arithmetic of the per-column least-squares problems: */
#define PMOR_F64 0
#define PMOR_F32 1
#define PMOR_F16S 2   /* gathered block rounded to FP16 with a power-of-two scale per */
                      /* column, arithmetic in FP32                               */
/* Update kinds (pattern of Q_l, which the paper leaves open): */
#define PMOR_UPD_DIAG 0     /* q_i has the single entry i: P_l = diag(q) P_1  */
#define PMOR_UPD_PATTERN 1  /* q_i on the SPAI pattern J_i, applied as Q_l(P_1 X) */
#define PMOR_UPD_ADAPTIVE 2 /* q_i diagonal, escalated to J_i (the U-pattern least */
                            /* squares) where ||A(1)e_i - q_i A(l)e_i|| >         */
                            /* adapt_ep ||A(1)e_i||; applied as Q_l(P_1 X)        */
/* Update approaches (Section 2.3, Table 1): */
#define PMOR_APPROACH_FIRST 0   /* anchor A(1): Q_l = argmin ||A(1) - A(l) Q||_F,  */
                                /* P_l = Q_l P_1 (the paper's choice)              */
#define PMOR_APPROACH_SECOND 1  /* anchor A(l-1): Q_l = argmin ||A(l-1) - A(l) Q||_F,*/
                                /* P_l = Q_l P_{l-1}; built for PMOR_UPD_DIAG only, */
                                /* where it is the row scaling diag(q_l ... q_2) P_1 */
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

/* Options of a preconditioner (spai_build) and of the sequence and server
 * calls.  A zero-filled struct selects the defaults of each field (pattern of
 * A, FP64, U-diag, first approach, no re-anchoring).  PMOR_EINVAL for values
 * outside the ranges below, for the second approach or re-anchoring with
 * another update kind, and for re-anchoring outside pmor_sequence_solve. */
typedef struct pmor_spai_opts {
  int32_t pattern;            /* PMOR_PAT_A or PMOR_PAT_EXPLICIT                */
  int32_t precision;          /* PMOR_F64, PMOR_F32 or PMOR_F16S                */
  int32_t update;             /* PMOR_UPD_DIAG, PMOR_UPD_PATTERN or             */
                              /* PMOR_UPD_ADAPTIVE                               */
  int32_t nnz_explicit;       /* entries of the explicit pattern                */
  const int32_t* pat_colptr;  /* device, n+1; column j of P may hold rows       */
  const int32_t* pat_row;     /* pat_row[pat_colptr[j]..pat_colptr[j+1]), sorted,*/
                              /* must contain j                                  */
  int32_t approach;           /* PMOR_APPROACH_FIRST (0) or PMOR_APPROACH_SECOND */
  double reanchor_tol;        /* pmor_sequence_solve, U-diag first approach: a   */
                              /* point l whose update misfit                     */
                              /* ||A(a) - A(l) Q||_F / ||A(a)||_F against the    */
                              /* current anchor a exceeds this gets a fresh SPAI */
                              /* and anchors the later points (0: never)         */
  double adapt_ep;            /* PMOR_UPD_ADAPTIVE: escalation threshold >= 0    */
} pmor_spai_opts;

typedef struct pmor_solve_opts {
  int32_t m;          /* block steps per cycle (restart length), 1..31         */
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
  double t_solve_ms;         /* block_solve: its wall time; batched calls: wall  */
                             /* time from the call's start until this system's X */
                             /* is final                                         */
  int32_t anchor;            /* pmor_sequence_solve: the point whose SPAI this   */
                             /* point's preconditioner is updated from (itself   */
                             /* when rebuilt); 0 elsewhere                        */
} pmor_stats;

/* ---- context ----------------------------------------------------------- */
/* Create a context on HIP device `device` that orders its work on
 * `hip_stream` (a hipStream_t; NULL = the null stream).  Errors: PMOR_EHIP
 * when the device cannot be selected, PMOR_EINVAL for out == NULL. */
int pmor_ctx_create(pmor_ctx** out, int device, void* hip_stream);
/* Destroy calls may come in any order: the context lives on until its
 * problems and servers are destroyed, a problem until its preconditioners and
 * server jobs are.  Device memory the library releases is kept in a process-wide cache and
 * handed out again (on the stream that released it at once, on another stream
 * once the release has completed on the device); a failed allocation empties
 * the cache and retries. */
void pmor_ctx_destroy(pmor_ctx* ctx);
/* Re-point the context at another stream of the same device.  Synchronises the
 * old stream first, so work queued there (and device memory released on it)
 * is complete before anything is ordered on the new one. */
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
/* The general affine problem of Section 1.1 (eq. affine_system) and Section
 * 2.4: A(l) = sum_t c_t^l T_t over nterms (1..PMOR_TMAX) term matrices, the
 * point l being the coefficient vector c^l (A_0 is a term whose coefficient
 * the caller passes as 1; the paper's gyroscope model of Section 3 has seven
 * terms, six of them with free coefficients such as s^2 d and 1/d).  terms[t]
 * must all be present and share n; validation, pattern and copies as
 * pmor_problem_create.  Points of such a problem are given as coefficient
 * vectors to the *_c calls (nterms host doubles, in the order of terms); the
 * (s, p) calls return PMOR_EINVAL for it.  pmor_problem_create is the special
 * case of six roles with the coefficients of s^2 M(p) + s D(p) + K(p); the *_c
 * calls accept its points too, as PMOR_NROLES coefficients in role order
 * (those of absent roles are ignored). */
int pmor_problem_create_affine(pmor_ctx* ctx, int32_t nterms, const pmor_csr* const* terms, pmor_problem** out);
/* Several problems at once (the batches of independent systems of Section 3:
 * each system is set up on its own, so the set-ups run side by side).  Item i
 * is the call pmor_problem_create (nterms = 0: terms holds PMOR_NROLES role
 * entries, NULL for an absent role) or pmor_problem_create_affine (nterms in
 * 1..PMOR_TMAX); out: pb and status (PMOR_OK, or that call's error; pb NULL on
 * error).  The union patterns are built on worker streams of the library
 * (threads of the calling process), after the work already queued on ctx's
 * stream; every problem is bit for bit the one the single call gives.  Complex
 * problems are not taken here.  Returns PMOR_OK or the first item's failure;
 * synchronises. */
typedef struct pmor_problem_item {
  int32_t nterms;
  const pmor_csr* const* terms;
  pmor_problem* pb;     /* out */
  int32_t status;       /* out */
} pmor_problem_item;
int pmor_problem_create_batch(pmor_ctx* ctx, pmor_problem_item* items, int32_t count);

/* Complex coefficients (the paper's expansion points are complex, Section 3:
 * s = 2 pi f sqrt(-1) makes s theta and s theta d imaginary).  A complex system
 * A x = b with A = sum_t c_t T_t (real T_t, complex c_t) is solved in its
 * equivalent real form: unknown i becomes the pair (Re x_i, Im x_i) at rows
 * 2i, 2i+1, and a complex entry alpha + beta sqrt(-1) the 2x2 block
 * [[alpha, -beta], [beta, alpha]], i.e. A^ = sum_t Re(c_t) (T_t (x) I_2) +
 * Im(c_t) (T_t (x) J_2), J_2 = [[0, -1], [1, 0]].  The problem made here is that
 * real affine problem of order 2n (every call of this header applies to it
 * unchanged: its SPAI is the SPAI of A^, its update and block GMRES those of
 * A^, so X^ holds the complex solution exactly as A^ X^ = B^ holds A X = B).
 * kinds[t] says which parts c_t may have: PMOR_COEF_REAL (T_t (x) I_2 only),
 * PMOR_COEF_IMAG (T_t (x) J_2 only) or PMOR_COEF_COMPLEX (both); at most
 * PMOR_TMAX real terms in all.  Points are given to the *_c calls as 2 nterms
 * doubles (Re c_0, Im c_0, Re c_1, ...); a part a term's kind excludes must be
 * 0 (PMOR_EINVAL otherwise).  B and X are 2n x k real blocks: row 2i the real
 * parts of row i, row 2i+1 its imaginary parts.  n of the problem (info) is 2n.
 * Every term's real form stores whole 2x2 blocks (zeros included), the
 * diagonal blocks among them, so the pattern of A^ is the real form of A's
 * pattern (union of the terms plus the diagonal) and each SPAI column pair
 * 2j, 2j+1 solves the complex least squares of column j (Section 2.2).
 * Updates: PMOR_UPD_DIAG takes the complex factor q_i of Section 2.3, i.e. the
 * 2x2 block [[Re q_i, -Im q_i], [Im q_i, Re q_i]], and writes P_l = Q P_1 out
 * (spai_export's qval holds Re q_i, Im q_i at 2i, 2i+1); PMOR_UPD_PATTERN is
 * the complex U-pattern update as it stands.  The second approach,
 * PMOR_UPD_ADAPTIVE and re-anchoring return PMOR_EINVAL; an explicit or
 * imported P must have a real-form pattern (rows 2i, 2i+1 alike, columns in
 * pairs), else PMOR_EINVAL.  Block GMRES runs on the real blocks as given: with
 * B^ = [R(B), R(sqrt(-1) B)] (2k columns) it is complex block GMRES on B (the
 * real span of both is the complex span of B), and X^'s first k columns are
 * the complex solution.  Frobenius norms reported (stats, Table 2 norms) are
 * those of the real form, sqrt(2) times the complex ones. */
#define PMOR_COEF_REAL 0
#define PMOR_COEF_IMAG 1
#define PMOR_COEF_COMPLEX 2
int pmor_problem_create_complex(pmor_ctx* ctx, int32_t nterms, const pmor_csr* const* terms,
                                const int32_t* kinds, pmor_problem** out);
void pmor_problem_destroy(pmor_problem* pb);
/* n and nnz of the union pattern (host outputs). */
int pmor_problem_info(const pmor_problem* pb, int32_t* n, int32_t* nnz);
/* Copy the union pattern into caller buffers (device): rowptr (n+1), col (nnz)
 * and maps (R*nnz with R = PMOR_NROLES for a problem of roles, nterms for an
 * affine one; maps[r*nnz + e] = position of A-slot e in term r's value array,
 * -1 where term r has no entry or is absent).  Any output may be NULL. */
int pmor_problem_pattern(const pmor_problem* pb, int32_t* rowptr, int32_t* col, int32_t* maps);
/* Values of A(s,p) on the union pattern into val (device, nnz). */
int pmor_assemble(pmor_problem* pb, double s, double p, double* val);
/* Values of A(c) = sum_t coef[t] T_t into val (coef: host, see
 * pmor_problem_create_affine; PMOR_EINVAL for a non-finite coefficient). */
int pmor_assemble_c(pmor_problem* pb, const double* coef, double* val);

/* ---- SPAI (Section 2.2) and its update (Sections 2.3-2.4) ---------------- */
/* Build P = argmin ||I - A(s,p) P||_F on the chosen pattern; (s,p) becomes
 * the anchor A(1) of later updates.  Each column j solves
 * min ||e_j(I_j) - A(I_j,J_j) p||_2 by Householder QR, I_j being the rows of
 * A(:,J_j) that hold a nonzero.  opts may be NULL (defaults: PMOR_PAT_A,
 * PMOR_F64, PMOR_UPD_DIAG).  stats may be NULL; when given, the call
 * synchronises and fills fro_resid and t_* fields.  PMOR_ESINGULAR (with
 * stats->bad_column) when |R_kk| <= 10 |I_j| eps max|R| in some column;
 * PMOR_EINVAL when a column's |J_j| exceeds 64 or its least-squares block does
 * not fit one workgroup's LDS (|I_j| x |J_j| values, about 150 KiB). */
int spai_build(pmor_problem* pb, double s, double p, const pmor_spai_opts* opts,
               pmor_spai** out, pmor_stats* stats);
/* spai_build at the point with coefficient vector coef (host; see
 * pmor_problem_create_affine). */
int spai_build_c(pmor_problem* pb, const double* coef, const pmor_spai_opts* opts,
                 pmor_spai** out, pmor_stats* stats);
/* P_1 of several problems, each at its own point, with the least squares of
 * all of them in shared launches (Section 2.2: every column of every system is
 * a problem of its own): one launch per (|J|, |I|) bucket over the bucket's
 * columns of all systems.  Per item: pb (of ctx), the point coef (host, or NULL
 * for (s, p)), opts (may be NULL; every item the same precision); out: h (the
 * handle, also on PMOR_ESINGULAR as spai_build returns it), status and
 * bad_column.  Each handle is bit for bit the one spai_build gives.  Returns
 * PMOR_OK or the first item's failure; synchronises the stream. */
typedef struct pmor_spai_build_item {
  pmor_problem* pb;
  double s, p;
  const double* coef;
  const pmor_spai_opts* opts;
  pmor_spai* h;         /* out */
  int32_t status;       /* out */
  int32_t bad_column;   /* out */
} pmor_spai_build_item;
int spai_build_batch(pmor_ctx* ctx, pmor_spai_build_item* items, int32_t count);
/* Update at (s,p) (Table 1).  First approach: Q = argmin ||A(1) - A(s,p) Q||_F
 * on the handle's update pattern, then P = Q P_1 (anchor unchanged).  Second
 * approach (U-diag only): q = argmin ||A(prev) - A(s,p) diag(q)||_F, A(prev)
 * being the previous update's (or the build's) matrix, then P = diag(q) P_prev,
 * kept as P_1 with its rows scaled by the running product of the q's; the
 * anchor moves to (s,p).  rho: the step's own residuals
 * ||A(prev) e_i - q_i A(s,p) e_i||.  Errors as spai_build; spai_build returns
 * PMOR_EINVAL for the second approach with PMOR_UPD_PATTERN. */
int spai_update(pmor_spai* h, double s, double p, pmor_stats* stats);
int spai_update_c(pmor_spai* h, const double* coef, pmor_stats* stats);
/* spai_update of several handles (of ctx), each at its own point (the batches
 * of independent systems of Section 3: every system's update is its own).  Per
 * item: h, the point coef (host, or NULL for (s, p)); out: status (as
 * spai_update returns it; PMOR_ESINGULAR with bad_column).  The real U-diag
 * updates (either approach) are queued back to back on ctx's stream and their
 * flags read back together; other update kinds run one after another as
 * spai_update.  Every handle ends bit for bit as after spai_update.  Returns
 * PMOR_OK or the first item's failure; synchronises. */
typedef struct pmor_spai_update_item {
  pmor_spai* h;
  double s, p;
  const double* coef;
  int32_t status;       /* out */
  int32_t bad_column;   /* out */
} pmor_spai_update_item;
int spai_update_batch(pmor_ctx* ctx, pmor_spai_update_item* items, int32_t count);
/* Recompute the SPAI of A(s,p) in place (the rebuild policy); the anchor is
 * moved to (s,p). */
int spai_rebuild(pmor_spai* h, double s, double p, pmor_stats* stats);
int spai_rebuild_c(pmor_spai* h, const double* coef, pmor_stats* stats);
/* A preconditioner from a given P, as the paper's pipeline hands P from one
 * program to another (Section 3): P in CSR on the device (rowptr n+1, col and
 * val nnzP; columns strictly increasing per row, every row holding its
 * diagonal), copied here.  (s,p) or coef is the anchor point A(1) of later
 * updates.  The handle is spai_build's with PMOR_PAT_EXPLICIT on P's pattern
 * (opts: precision, update kind and approach of later updates and rebuilds;
 * its pattern fields are ignored), rho zero until an update.  Export then
 * import gives back the same preconditioner bit for bit.  PMOR_EINVAL for a
 * malformed P.  Synchronises. */
int spai_import(pmor_problem* pb, double s, double p, int32_t nnzP, const int32_t* rowptr,
                const int32_t* col, const double* val, const pmor_spai_opts* opts,
                pmor_spai** out);
int spai_import_c(pmor_problem* pb, const double* coef, int32_t nnzP, const int32_t* rowptr,
                  const int32_t* col, const double* val, const pmor_spai_opts* opts,
                  pmor_spai** out);
/* The current preconditioner.  P in CSR: rowptr (n+1), col (nnzP), val (nnzP);
 * for PMOR_UPD_PATTERN and PMOR_UPD_ADAPTIVE after an update, val holds P_1
 * and qval holds Q (same CSR pattern; an adaptive column that was not
 * escalated holds q_i on its diagonal and zeros), and the preconditioner is
 * Q P_1; for PMOR_UPD_DIAG, qval (n)
 * holds the row scale of P_1 (the last update's q, or with the second approach
 * the product of the q's since the build; ones before any update).  rho (n): per-column
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
 * max_cycles = 20.  Dependent columns (the paper assumes a block Krylov space
 * of full dimension, Section 2.1): a block whose thin QR Y = Q S has a column
 * with S_cc <= 1e-6 ||y_c|| (within that sine of the span of the columns
 * before it) is dependent.  At a cycle start (Y the residual block, e.g. two
 * equal columns of B) the solve ends with PMOR_EBREAKDOWN and X = the last
 * iterate.  In a block step (Y the new block after Gram-Schmidt, also
 * deficient when S_cc <= 1e-14 max ||W_c|| before Gram-Schmidt) the cycle ends
 * there, its least-squares solution updates X and the solve restarts.
 * Returns PMOR_ENOTCONV (X = last iterate), PMOR_EBREAKDOWN, or PMOR_ENAN
 * (NaN/Inf in B: X = 0; in a residual: X = last iterate) on failure.
 * Synchronises the stream. */
int block_solve(pmor_problem* pb, const pmor_spai* h, double s, double p,
                const double* B, int64_t ldb, int32_t k, double* X, int64_t ldx,
                const pmor_solve_opts* opts, pmor_stats* stats);
int block_solve_c(pmor_problem* pb, const pmor_spai* h, const double* coef,
                  const double* B, int64_t ldb, int32_t k, double* X, int64_t ldx,
                  const pmor_solve_opts* opts, pmor_stats* stats);

/* ---- Block GCRO-DR: recycling a subspace across the points of a sequence ----
 * The paper solves its sequences with block GCRO and a recycled subspace
 * (Section 3, Table 5).  A pmor_recycle holds the recycled basis U~ (n x kc,
 * kc <= kr) that one solve leaves for the next.  block_solve_gcrodr solves
 * A(s,p) X = B with right preconditioner h (NULL: none) by block GCRO-DR(m, kr):
 *  - entering: C = A P U~ = Q R, C <- Q, U <- U~ R^{-1} (Op U = C, C orthonormal;
 *    if that QR breaks down the solve starts without recycling);
 *  - each cycle: R = B - A X, projected on C (X += P U C^T R, R -= C C^T R);
 *    block Arnoldi on (I - C C^T) A P with two Gram-Schmidt passes against
 *    [C, V]; y2 = argmin ||E1 S - Hbar y2||; X += P (V y2 - U B y2);
 *  - end of each cycle: the harmonic Ritz vectors of A P on span([U D, V])
 *    (G^T (What^T Vhat) z = mu G^T G z, G = [[D, B], [0, Hbar]], D = diag
 *    (1/||u_i||); the kr of largest |mu|, a conjugate pair as Re z, Im z, a pair
 *    that does not fit ends the choice) become the new C and U;
 *  - the final U is left in rec for the next call.
 * X is overwritten (start X0 = 0).  opts as block_solve (m, max_cycles, tol);
 * stats: cycles, steps, cycle_steps, relres, t_solve_ms.  B must have no zero
 * column (PMOR_EINVAL).  Errors: PMOR_ENOTCONV, PMOR_EBREAKDOWN (dependent
 * residual columns), PMOR_ENAN, PMOR_EINVAL (arguments; rec of another size or
 * context).  Synchronises the stream.  Device work: the library's SpMM, Gram
 * products and tall-skinny products; the small dense work runs on the host. */
typedef struct pmor_recycle pmor_recycle;
/* An empty recycler for problems of order n, recycled dimension at most kr
 * (0..PMOR_KMAX; 0 makes block_solve_gcrodr block GMRES). */
int pmor_recycle_create(pmor_ctx* ctx, int32_t n, int32_t kr, pmor_recycle** out);
void pmor_recycle_destroy(pmor_recycle* r);
/* kc: the recycled dimension held now (host output). */
int pmor_recycle_info(const pmor_recycle* r, int32_t* kc);
/* Forget the recycled basis (the next solve starts without one). */
int pmor_recycle_reset(pmor_recycle* r);
/* U~ into U (device, n x kc, row-major, leading dimension ldu >= kc). */
int pmor_recycle_export(const pmor_recycle* r, double* U, int64_t ldu);
int block_solve_gcrodr(pmor_problem* pb, const pmor_spai* h, double s, double p,
                       const double* B, int64_t ldb, int32_t k, double* X, int64_t ldx,
                       const pmor_solve_opts* opts, pmor_recycle* rec, pmor_stats* stats);
int block_solve_gcrodr_c(pmor_problem* pb, const pmor_spai* h, const double* coef,
                         const double* B, int64_t ldb, int32_t k, double* X, int64_t ldx,
                         const pmor_solve_opts* opts, pmor_recycle* rec, pmor_stats* stats);
/* The harmonic Ritz choice of block GCRO-DR on host matrices (row-major): G
 * and WtV are rows x N (rows >= N); Pk (N x kr, row-major) receives the chosen
 * directions in its first *count columns, mu_re/mu_im (may be NULL, kr each)
 * their eigenvalues mu.  PMOR_ESINGULAR when G^T G is not positive definite
 * or the eigenvalue iteration fails.  Host only (no device work). */
int pmor_harmonic_ritz(int32_t rows, int32_t N, const double* G, const double* WtV, int32_t kr,
                       double* Pk, double* mu_re, double* mu_im, int32_t* count);

/* One system of pmor_batch_solve: A of problem pb at the point coef (host
 * coefficient vector) or, when coef is NULL, at (s,p) (assembled by the
 * library), preconditioned by h's current preconditioner (or NULL), B and X as
 * in block_solve. */
typedef struct pmor_batch_item {
  pmor_problem* pb;
  const pmor_spai* h;
  double s, p;
  const double* B;
  int64_t ldb;
  int32_t k;
  double* X;
  int64_t ldx;
  const double* coef;
} pmor_batch_item;

/* Solve many independent systems together (the batching of the hot path):
 * every system runs block GMRES(m) exactly as block_solve would, and all of them
 * advance in lockstep, each kernel launch covering every unfinished system.  A
 * system's result is bit-identical to its solve alone (its reductions depend on
 * its own sizes only).  Items may share a problem at different points and may
 * share a handle (its current preconditioner is used).  The block width is the
 * largest k of the batch.  status (nitems, host, may be NULL) receives each
 * system's code as block_solve would return it; stats: nitems entries or NULL.
 * Returns PMOR_OK when every system converged, else the first failing system's
 * code.  Device memory: about 8 (m + 6) kp n bytes per system plus nnz(A) values
 * for each extra point of a shared problem.  Synchronises the stream. */
int pmor_batch_solve(pmor_ctx* ctx, const pmor_batch_item* items, int32_t nitems,
                     const pmor_solve_opts* opts, pmor_stats* stats, int32_t* status);

/* The whole sequence of Section 2.3 for points (s_list[l], p_list[l]),
 * l < npts: P_1 = spai_build at point 0; for l >= 1 the update P_l = Q_l P_1
 * (PMOR_UPDATE; with sopts->approach = PMOR_APPROACH_SECOND, P_l = Q_l P_{l-1}
 * anchored at A(l-1), bit for bit as a chain of spai_update calls gives it) or a
 * fresh SPAI of A(l) (PMOR_REBUILD).  The
 * points are independent once P_1 exists, so their systems are solved together
 * as in pmor_batch_solve (in groups sized to the free device memory).
 * X: npts consecutive n x k row-major blocks (ldx per block, block stride
 * n*ldx).  stats: npts entries (may be NULL); t_solve_ms is the wall time from
 * the call's start to the point's final X.  With the U-diag update the A(l)
 * values and the factors q_l are formed for up to 8 points per launch, and
 * P_l = diag(q_l) P_1 is applied in that factored form; t_assemble_ms and
 * t_precond_ms then hold equal shares of those launches.  A point whose update or rebuild
 * meets a singular column is not solved (PMOR_ESINGULAR, X untouched); the
 * others are.  sopts->reanchor_tol > 0 (PMOR_UPDATE, U-diag, first approach;
 * PMOR_EINVAL otherwise): before any solve the points are scanned in order and
 * each point whose update misfit against the current anchor exceeds the
 * tolerance becomes a new anchor (a fresh SPAI, later points updated from it);
 * the runs between anchors are then solved as sequences of their own, and
 * stats[l].anchor names each point's anchor.  Returns the first failing
 * point's code, else PMOR_OK. */
int pmor_sequence_solve(pmor_problem* pb, const double* B, int64_t ldb, int32_t k,
                        const double* s_list, const double* p_list, int32_t npts,
                        double* X, int64_t ldx, int32_t policy,
                        const pmor_spai_opts* sopts, const pmor_solve_opts* vopts,
                        pmor_stats* stats);
/* The same with the points as coefficient vectors: coefs is npts x C (host,
 * row-major, C = the problem's coefficient count; point l at coefs + l*C). */
int pmor_sequence_solve_c(pmor_problem* pb, const double* B, int64_t ldb, int32_t k,
                          const double* coefs, int32_t npts, double* X, int64_t ldx,
                          int32_t policy, const pmor_spai_opts* sopts,
                          const pmor_solve_opts* vopts, pmor_stats* stats);

/* ---- serving: continuous batching of sequence jobs ----------------------- */
/* A server admits whole sequence jobs (one pmor_sequence_solve each) under a
 * device-memory budget and solves the points of all admitted jobs in one
 * persistent block GMRES engine: at every restart-cycle boundary finished
 * points leave it and waiting points of any job join it.  A point's X is bit
 * for bit what pmor_sequence_solve gives for it when it runs alone, whatever
 * else shares the engine.  Single-threaded: all calls on one host thread. */
typedef struct pmor_server pmor_server;

typedef struct pmor_server_opts {
  int64_t hbm_budget;   /* device bytes for the engine and admitted jobs; 0: 75% of free memory */
  int64_t engine_rows;  /* sum of n over the systems the engine holds at once; 0: from the budget */
  int32_t k;            /* widest job (the engine's block width), 1..PMOR_KMAX */
  int32_t max_systems;  /* systems in the engine at once; 0: 64 */
} pmor_server_opts;

typedef struct pmor_job {
  pmor_problem* pb;     /* owned by the caller, alive until the job is reported done */
  const double* B;      /* n x k, ld ldb (device) */
  int64_t ldb;
  int32_t k;
  const double* s_list; /* npts points (host; copied at submission) */
  const double* p_list;
  int32_t npts;
  double* X;            /* npts blocks n x k, ld ldx, block stride n*ldx (device) */
  int64_t ldx;
  int32_t policy;       /* PMOR_UPDATE | PMOR_REBUILD */
  pmor_stats* stats;    /* npts entries or NULL (host, written until the job is done); */
                        /* t_solve_ms = submission to the point's final X            */
  const double* coefs;  /* npts x C coefficient vectors (host, copied at submission), */
                        /* as pmor_sequence_solve_c; NULL: the points (s_list, p_list) */
} pmor_job;

/* sopts, vopts: as pmor_sequence_solve (NULL: defaults; reanchor_tol must be
 * 0).  The engine's buffers are allocated here.  PMOR_ENOMEM when the budget
 * cannot hold them. */
int pmor_server_create(pmor_ctx* ctx, const pmor_server_opts* opts, const pmor_spai_opts* sopts,
                       const pmor_solve_opts* vopts, pmor_server** out);
/* Jobs still held are dropped (their X undefined). */
void pmor_server_destroy(pmor_server* sv);
/* Queue a job (first in, first out).  PMOR_EADMIT when it can never be admitted:
 * its device footprint exceeds the budget, n exceeds the engine's rows or k
 * its block width.  *job_id (host) identifies it in pmor_server_step. */
int pmor_server_submit(pmor_server* sv, const pmor_job* job, int64_t* job_id);
/* One scheduling round: admit queued jobs in order while their footprint fits
 * the free budget (P_1, every point's A(l) and preconditioner are built then),
 * move waiting points into the engine while rows and slots are free, run one
 * restart cycle of every system in the engine, retire finished points and
 * jobs.  done_ids / done_status (host, max_done entries): jobs finished since
 * the last report with their first failing code (PMOR_OK when all points
 * converged); *ndone their count (reports beyond max_done wait for the next
 * call).  Returns an error only for failures of the server itself. */
int pmor_server_step(pmor_server* sv, int64_t* done_ids, int32_t* done_status, int32_t max_done, int32_t* ndone);
/* Host outputs, any may be NULL: queued jobs, admitted jobs, systems in the
 * engine, device bytes reserved (engine + admitted jobs). */
int pmor_server_info(const pmor_server* sv, int32_t* queued, int32_t* admitted, int32_t* running,
                     int64_t* bytes_in_use);

/* ---- diagnostics (Section 3.1, Table 2) -------------------------------- */
/* ||I - A(s,p)||_F and ||A(s1,p1) - A(s2,p2)||_F (host outputs; synchronises). */
int pmor_table2_norms(pmor_problem* pb, double s1, double p1, double s2, double p2,
                      double* fro_I_minus_A2, double* fro_A1_minus_A2);
/* The same for two coefficient vectors (host): ||I - A(coef2)||_F and
 * ||A(coef1) - A(coef2)||_F, e.g. the paper's Table 2 for the points of an
 * affine problem. */
int pmor_table2_norms_c(pmor_problem* pb, const double* coef1, const double* coef2,
                        double* fro_I_minus_A2, double* fro_A1_minus_A2);

/* The same two norms for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops that decide on re-anchoring per point,
 * harnesses that forbid hipMalloc): no hipMalloc, hipFree or other allocating
 * routine on this path.  Both norms are formed in one pass over the term
 * values (A(s1,p1) and A(s2,p2) are not assembled, the problem's assembled
 * values are left as they are) and their partial sums go to a fixed 4,112-byte
 * device array of the library, one per GPU, held until the process ends; it
 * fits every problem size, so no size is rejected.  Calls that overlap on one
 * GPU race for that array.  Host outputs; synchronises the stream.  Errors:
 * PMOR_EINVAL (pb NULL, an affine problem, s or p not finite), PMOR_EHIP. */
int pmor_table2_norms_noalloc(pmor_problem* pb, double s1, double p1, double s2, double p2,
                              double* fro_I_minus_A2, double* fro_A1_minus_A2);

/* ---- kernel-level entry points (timing and parity) --------------------- */
/* Y = beta*Y + alpha*A(s,p)-values-on-pattern * X, with the values in aval
 * (device, nnz) on pb's pattern; X, Y: n x k row-major, ld >= k. */
int pmor_spmm(pmor_problem* pb, const double* aval, const double* X, int64_t ldx,
              double* Y, int64_t ldy, int32_t k, double alpha, double beta);
/* The gather of the SPAI least squares on its own (Section 2.2: the dense block
 * A(I_j, J_j) of every column j, here of the handle's anchor A(1)), read exactly
 * as the FP64 least-squares kernels read it, with each block reduced to the sum
 * of its entries in colsum[j] (device, n).  A data-movement variant of the build
 * for timing (PMOR_PROF_SPAI_GATHER) and parity. */
int pmor_spai_gather(const pmor_spai* h, double* colsum);

/* ---- kernel timing (benchmarks) ---------------------------------------- */
/* Time every launch of one kernel class with HIP events recorded on the
 * context's stream around it, and add up the algorithmic bytes each launch must
 * move (the formulas are the library's roofline model).  kernel_id 0 turns the
 * timing off.  Launches of block steps that a converged cycle skipped are not
 * counted.  pmor_prof_read synchronises the stream, returns the totals since the
 * last read and resets them. */
/* Per system of a launch (n rows, kp block width, nblk V blocks swept): */
/* An array that several systems of one launch share (A's pattern for the points
 * of one problem, P's pattern and P_1's values for the points of one sequence)
 * counts once, split evenly among those systems. */
#define PMOR_PROF_SPMM_A 1        /* W = A Z in a block step: 12 nnz + 4(n+1) + 16 n kp */
#define PMOR_PROF_CGS_UPD_DOT 2   /* pass 2: W -= V H1; V^T W, W^T W: 8 n kp (nblk + 2) */
#define PMOR_PROF_CGS_DOT 3       /* pass 1: V^T W, column norms: 8 n kp (nblk + 1) */
#define PMOR_PROF_SPAI_LS 4       /* SPAI least squares: 12 nnz + 4 n + 4 (sum|I_j| + nnzP) + 8 nnzP + 8 n */
#define PMOR_PROF_SPMM_P 5        /* Z = P V_j, V_j = W1 R2^-1 written: 12 nnzP + 4(n+1) + 24 n kp */
#define PMOR_PROF_CGS_UPD_GRAM 6  /* pass 3: W -= V H2; W R1^-1; Gram: 8 n kp (nblk + 2) */
#define PMOR_PROF_SPAI_GATHER 7   /* gather only (pmor_spai_gather): 12 nnz + 4 n + 4 (sum|I_j| + nnzP) + 8 n */
#define PMOR_PROF_GCRO_GRAM 8     /* block GCRO-DR Gram product [.]^T W (first stage): 8 n (a + b) */
#define PMOR_PROF_GCRO_GEMM 9     /* block GCRO-DR product Y = beta Y + alpha A G: 8 n (a + b) (+ 8 n b read when beta != 0) */
int pmor_prof_set(pmor_ctx* ctx, int kernel_id);
int pmor_prof_read(pmor_ctx* ctx, int64_t* launches, double* total_ms, double* total_bytes);
/* The streaming rate a kernel with a given read/write mix runs against: nread
 * arrays of nbytes each (nread 1..8 or 12, 16, ..., 32; nbytes a positive
 * multiple of 8) read once with non-temporal loads over the whole device, their
 * element-wise sum written to nwrite (0, 1 or 2) more arrays of nbytes (kept in
 * registers when nwrite is 0).  *us: average microseconds of one pass over reps
 * (>= 1) timed passes after two untimed ones, on ctx's stream.  Allocates and
 * frees (nread + nwrite) nbytes of device memory itself (hipMalloc, hipFree) and
 * synchronises.  A measurement aid, no step of the method. */
int pmor_stream_probe(pmor_ctx* ctx, int32_t nread, int32_t nwrite, int64_t nbytes, int32_t reps, double* us);

/* ---- errors ------------------------------------------------------------ */
const char* pmor_strerror(int code);
const char* pmor_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PMOR_SPAI_H */
