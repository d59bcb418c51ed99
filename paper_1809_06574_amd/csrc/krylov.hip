// Block GMRES(m) with right preconditioning (paper, Section 2.1 and the
// footnote of Section 2.2 on right preconditioning) for a batch of
// independent systems ("segments") that advance through the cycle in lockstep:
// every kernel launch below covers all unfinished segments of the batch.
//
// One block step j of every segment:
//   Z = P V_j            V_j = W1 R2^{-1} is formed on the fly from the previous
//                        step's W1 and written by this SpMM
//   W = A Z
//   pass 1:  H1 = [V_0..V_j]^T W and ||W_c||^2
//   pass 2:  W' = W - V H1;   H2 = V^T W' and Gram(W')
//   pass 3:  W'' = W' - V H2; R1 = chol(Gram(W') - H2^T H2); W1 = W'' R1^{-1}; Gram(W1)
//   hess:    R2 = chol(Gram(W1)); H_{j+1,j} = R2 R1; Householder update of the
//            QR of the block Hessenberg matrix, least-squares residual estimates.
// Passes 1-2 are classical Gram-Schmidt with one reorthogonalisation; the thin
// QR W'' = V_{j+1} H_{j+1,j} is Cholesky QR applied twice, its first Gram
// matrix taken from Gram(W') by the identity W''^T W'' = W'^T W' - H2^T H2
// (V^T V = I), so a step sweeps V three times.
// Cycle start: the same pass-2/pass-3/hess kernels with no V blocks give V_0 S = R_0.
// End of cycle: Y = R^{-1} G;  X += P (V Y);  residual B - A X and its norms.
//
// Layout: every n x kp block is row-major (kp contiguous doubles per row); the
// segments' rows are concatenated (each padded to 16 rows) and V holds (m+1)
// such concatenated blocks.  The inner products V^T W and the Gram matrices
// are tall-skinny contractions over the rows done with the FP64 MFMA
// v_mfma_f64_4x4x4f64 for kp in {4, 8, 16}: a wavefront takes 16 rows x 4
// columns (512 contiguous bytes) per operand tile.  Lane l of such a tile holds
// row 16c + (l >> 2), column (l & 3); with the instruction's operand layout
// (A[i][k] at lane 16k + 4b + i, B[k][j] at lane 16k + 4b + j, D[i][j] at lane
// 16i + 4b + j) the same register serves as A or B operand and the four blocks b
// sum rows 4k + b.  kp in {1, 2} use one row per lane.  Cross-workgroup sums
// use a fixed two-level order per segment (no floating-point atomics): results
// are reproducible bit for bit and independent of the other segments of a batch.
#include "common.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

namespace pmor {

// streaming load: the basis and the work block are far larger than the caches
// and are not reread by the same kernel
__device__ __forceinline__ double ldnt(const double* p) { return __builtin_nontemporal_load(p); }

__device__ __forceinline__ double mfma4(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

struct KArgs {
  int m;
  int nbl;             // V blocks of the sweep; < 0: the segment's st->j (end of cycle)
  int mode;            // 0: block step, 1: initial QR of the cycle
  int zero_init;       // update kernels: start from W = 0
  int ignore_done;     // run even when the segment's cycle is done (end-of-cycle V Y)
  int ldh;             // rows of the Hessenberg matrix, (m + 1) kp
  int64_t vstride;     // rows_total * kp
  double* V;
  double* W;           // work block (input/output of the sweeps)
  const SegDesc* seg;
  const int* wtab;     // logical workgroup of the row kernels -> segment (-1: padding)
  const int* slist;    // segments of the one-workgroup-per-segment kernels
  const double* Hsrc;  // update coefficients of segment s at Hsrc + s * hsrc_stride ([basis][rhs])
  int64_t hsrc_stride;
  double hsign;        // the update computes W <- W - hsign * V Hsrc
  double* Hc;          // per segment: H1 (+ kp squared norms) at 0, H2 (+ Gram(W')) at hc2off
  int64_t hcs, hc2off;
  double* Hbar;        // block Hessenberg (column-major, ldh rows), per segment stride hbs
  int64_t hbs;
  double* G;           // transformed E1 S (column-major, ldh rows)
  int64_t gs;
  double* refl;        // Householder reflectors of the Hessenberg QR
  int64_t rfs;
  double* Y;           // R^{-1} G ([basis][rhs])
  int64_t ys;
  double* part;        // per-workgroup partial rows
  int64_t lstride;
  double* partg;       // per-workgroup Gram(W1) partials (kp x kp)
  DevState* st;
  int* hinfo;          // host-mapped {j, done, breakdown, nan} per segment
  int swz;             // row kernels: remap the workgroup index per XCD (few workgroups)
  const double* Hsrc1; // kp = 4 pass 3: pass 2's coefficients (same layout and stride as Hsrc)
};

// The segment of a row kernel's workgroup; false for padding workgroups and
// (check_done) segments whose cycle is over.  Uniform over the workgroup.
struct RowSeg {
  int s, g, G, n, lg;
  int64_t r0;
};

__device__ __forceinline__ bool row_seg(const KArgs& a, bool check_done, RowSeg& r) {
  const int lg = a.swz ? xcd_swizzle(blockIdx.x, gridDim.x) : (int)blockIdx.x;
  const int s = a.wtab[lg];
  if (s < 0) return false;
  if (check_done && a.st[s].done) return false;
  const SegDesc& d = a.seg[s];
  r.s = s;
  r.g = lg - d.wg0;
  r.G = d.G;
  r.n = d.n;
  r.lg = lg;
  r.r0 = d.r0;
  return true;
}

__device__ __forceinline__ int nblocks_of(const KArgs& a, int s) { return a.nbl >= 0 ? a.nbl : a.st[s].j; }

// ---------------------------------------------------------------------------
// cross-workgroup sums: every row-parallel kernel writes one partial row per
// workgroup (part[lg * lstride + t]); these kernels add a segment's rows up in a
// fixed order (no atomics, no inter-workgroup fences).
// ---------------------------------------------------------------------------
// out[s * ostride + ooff + t] = sum_g part[(wg0_s + g) lstride + t]; 8 entries per
// workgroup, 32 lanes per entry, lane r sums g = r, r + 32, ... in order, then a
// fixed tree over the lanes.  fixedG > 0: the segment at list position y owns
// rows [y fixedG, (y + 1) fixedG).
__global__ __launch_bounds__(256) void k_reduce_seg(const double* __restrict__ part, int64_t lstride, int L,
                                                    const SegDesc* seg, const int* slist, int fixedG,
                                                    const DevState* st, int check_done, double* out,
                                                    int64_t ostride, int64_t ooff) {
  const int s = slist[blockIdx.y];
  if (check_done && st[s].done) return;
  const int wg0 = fixedG > 0 ? (int)blockIdx.y * fixedG : seg[s].wg0;
  const int G = fixedG > 0 ? fixedG : seg[s].G;
  const double* p = part + (int64_t)wg0 * lstride;
  __shared__ double sm[8][33];
  const int e = threadIdx.x & 7, r = threadIdx.x >> 3;
  const int t = blockIdx.x * 8 + e;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  if (t < L) {
    int g = r;
    for (; g + 96 < G; g += 128) {
      a0 += p[(int64_t)g * lstride + t];
      a1 += p[(int64_t)(g + 32) * lstride + t];
      a2 += p[(int64_t)(g + 64) * lstride + t];
      a3 += p[(int64_t)(g + 96) * lstride + t];
    }
    for (; g < G; g += 32) a0 += p[(int64_t)g * lstride + t];
  }
  sm[e][r] = (a0 + a1) + (a2 + a3);
  __syncthreads();
  for (int o = 16; o >= 1; o >>= 1) {
    if (r < o) sm[e][r] += sm[e][r + o];
    __syncthreads();
  }
  if (r == 0 && t < L) out[(int64_t)s * ostride + ooff + t] = sm[e][0];
}

// the same sum inside one workgroup of 256 threads, for L <= 256 (result in dst)
__device__ void block_reduce_partials(const double* __restrict__ part, int L, int G, double* dst) {
  __shared__ double sr[256];
  int R = 1;
  while (R * 2 * L <= 256) R *= 2;  // lanes per entry
  const int e = threadIdx.x % L, r = threadIdx.x / L;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  if (r < R) {
    int g = r;
    for (; g + 3 * R < G; g += 4 * R) {
      a0 += part[(size_t)g * L + e];
      a1 += part[(size_t)(g + R) * L + e];
      a2 += part[(size_t)(g + 2 * R) * L + e];
      a3 += part[(size_t)(g + 3 * R) * L + e];
    }
    for (; g < G; g += R) a0 += part[(size_t)g * L + e];
  }
  if (threadIdx.x < R * L) sr[r * L + e] = (a0 + a1) + (a2 + a3);
  __syncthreads();
  for (int o = R / 2; o >= 1; o >>= 1) {
    if (r < o) sr[r * L + e] += sr[(r + o) * L + e];
    __syncthreads();
  }
  if (threadIdx.x < L) dst[threadIdx.x] = sr[threadIdx.x];
  __syncthreads();
}

// ---------------------------------------------------------------------------
// small dense helpers run by one thread
// ---------------------------------------------------------------------------
// Upper Cholesky factor of the leading kact x kact block of the kp x kp
// row-major Gram matrix; padded rows/columns get R = I.  Returns false when a
// pivot is not above thr2.
__device__ bool chol_upper(const double* Gm, int kp, int kact, double thr2, double* R, double* Rinv) {
  bool ok = true;
  for (int i = 0; i < kp * kp; ++i) { R[i] = 0.0; Rinv[i] = 0.0; }
  for (int c = 0; c < kp; ++c) {
    if (c >= kact) { R[c * kp + c] = 1.0; continue; }
    double d = Gm[c * kp + c];
    for (int t = 0; t < c; ++t) d -= R[t * kp + c] * R[t * kp + c];
    if (!(d > thr2)) { ok = false; d = (thr2 > 0.0 ? thr2 : 1e-300); }
    const double rc = sqrt(d);
    R[c * kp + c] = rc;
    for (int c2 = c + 1; c2 < kact; ++c2) {
      double x = Gm[c * kp + c2];
      for (int t = 0; t < c; ++t) x -= R[t * kp + c] * R[t * kp + c2];
      R[c * kp + c2] = x / rc;
    }
  }
  // inverse of the upper triangular R, column by column
  for (int c = 0; c < kp; ++c) {
    for (int r = c; r >= 0; --r) {
      double x = (r == c) ? 1.0 : 0.0;
      for (int t = r + 1; t <= c; ++t) x -= R[r * kp + t] * Rinv[t * kp + c];
      Rinv[r * kp + c] = x / R[r * kp + r];
    }
  }
  return ok;
}

// Pass-3 set-up of a segment (k_p3_setup for kp != 4; every pass-3 workgroup
// for kp = 4, where it is cheap next to the sweep): the Gram matrix of
// W'' = W' - V H2 as Gram(W') - H2^T H2 (sH holds +-H2 in LDS, [basis][rhs]),
// its Cholesky factor R1 and R1^{-1}, and the scale max_c ||W_c|| of the
// deficiency test (block step: norms of pass 1; cycle start: of W itself).
// The block is deficient when a column's sine to the span of the columns
// before it, R1_cc / ||w_c||, is at most kDepSine, or (block step only) a
// pivot is at most 1e-14 max_c ||W_c||.  The sine test is scale-free, so a
// residual column that converged far ahead of the others does not trip it at
// a cycle start.  Stores R1, the scale, the verdict and, in a block step, the
// Hessenberg column block H1 + H2 (when first).
template <int KP>
__device__ void p3_prologue(const KArgs& a, int s, bool first, const double* sH, int nbl, double* sRinv) {
  DevState* st = a.st + s;
  const double* Hc1 = a.Hc + s * a.hcs;
  const double* Hc2 = Hc1 + a.hc2off;
  __shared__ double sG[KP * KP], sR[KP * KP];
  for (int t = threadIdx.x; t < KP * KP; t += blockDim.x) {
    const int c1 = t / KP, c2 = t % KP;
    double x = Hc2[nbl * KP * KP + t];
    for (int b = 0; b < nbl * KP; ++b) x -= sH[b * KP + c1] * sH[b * KP + c2];
    sG[t] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int kact = st->kact;
    double mx = 0.0;
    for (int c = 0; c < kact; ++c) mx = fmax(mx, a.mode == 0 ? Hc1[nbl * KP * KP + c] : sG[c * KP + c]);
    const double ws = sqrt(mx);
    const double thr = a.mode == 0 ? 1e-14 * ws : 0.0;
    bool ok = chol_upper(sG, KP, kact, thr * thr, sR, sRinv);
    for (int c = 0; c < kact; ++c)
      if (!(sR[c * KP + c] > kDepSine * sqrt(sG[c * KP + c]))) ok = false;
    if (first) {
      st->wscale = ws;
      st->deficient = ok ? 0 : 1;
      for (int t = 0; t < KP * KP; ++t) st->R1[t] = sR[t];
    }
  }
  if (first && a.mode == 0) {
    const int j = nbl - 1;
    double* Hb = a.Hbar + s * a.hbs;
    for (int t = threadIdx.x; t < nbl * KP * KP; t += blockDim.x) {
      const int b = t / KP, c = t % KP;
      Hb[b + (int64_t)(j * KP + c) * a.ldh] = Hc1[t] + Hc2[t];
    }
  }
  __syncthreads();
}

// pass-3 set-up of every active segment, once, before the pass-3 sweep of the
// kp = 1, 2, 8, 16 kernels: their workgroups then only load R1^{-1} (dynamic
// LDS: nbl_max KP^2 doubles)
template <int KP>
__global__ __launch_bounds__(256) void k_p3_setup(KArgs a) {
  const int s = a.slist[blockIdx.x];
  if (!a.ignore_done && a.st[s].done) return;
  const int nbl = nblocks_of(a, s);
  extern __shared__ double sH[];
  __shared__ double sRinv[KP * KP];
  const double* Hs = a.Hsrc + s * a.hsrc_stride;
  for (int t = threadIdx.x; t < nbl * KP * KP; t += blockDim.x) sH[t] = Hs[t];
  __syncthreads();
  p3_prologue<KP>(a, s, true, sH, nbl, sRinv);
  for (int t = threadIdx.x; t < KP * KP; t += blockDim.x) a.st[s].R1inv[t] = sRinv[t];
}

__device__ __forceinline__ void load_r1inv(const KArgs& a, int s, int kp2, double* sRinv) {
  for (int t = threadIdx.x; t < kp2; t += blockDim.x) sRinv[t] = a.st[s].R1inv[t];
  __syncthreads();
}

// update-kernel modes
constexpr int UPD_PLAIN = 0;  // W <- W - hsign V Hsrc                       (end-of-cycle V Y)
constexpr int UPD_P2 = 1;     // ... then V^T W and Gram(W)                  (pass 2)
constexpr int UPD_P3 = 2;     // prologue; W <- (W - V H2) R1^{-1}; Gram(W)  (pass 3)
// (kp = 4: pass 2 keeps W' = W - V H1 in registers only, and pass 3 forms it
// again from W with the same operations in the same order, so W' is bit for
// bit the vector pass 2 saw; a block write per step is saved)

// ---------------------------------------------------------------------------
// kp = 4, rows split over the wavefronts: each wavefront streams its own 16-row
// tiles against every V block (at most RS_B), so all of a tile's loads are in
// flight together and no LDS exchange is needed inside the loop.
// ---------------------------------------------------------------------------
constexpr int RS_B = 32;

// sum of a per-wavefront row of L values over the NW wavefronts, in order,
// written as this workgroup's partial row
template <int NW, int ROW>
__device__ __forceinline__ void rs_store_partials(double (*sred)[ROW], int L, double* dst) {
  __syncthreads();
  for (int t = threadIdx.x; t < L; t += 64 * NW) {
    double tot = 0.0;
#pragma unroll
    for (int q = 0; q < NW; ++q) tot += sred[q][t];
    dst[t] = tot;
  }
}

// pass 1: partial [V_0..V_{nbl-1}]^T W (nbl 16 values) and ||W_c||^2 (4 values)
template <int NW, int NB>
__global__ __launch_bounds__(64 * NW) void k_dot4(KArgs a) {
  RowSeg r;
  if (!row_seg(a, true, r)) return;
  const int nbl = a.nbl;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nch = (r.n + 15) >> 4;
  const double* W = a.W + r.r0 * 4;
  const double* V = a.V + r.r0 * 4;
  constexpr int ROW = NB * 16 + 16;
  __shared__ double sred[NW][ROW];
  double acc[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) acc[i] = 0.0;
  double wn = 0.0;
  for (int ch = r.g * NW + w; ch < nch; ch += r.G * NW) {
    const int64_t off = ((int64_t)ch << 6) + lane;  // 16 rows x 4 columns = 64 doubles
    const bool valid = off < (int64_t)r.n * 4;
    const double wt = valid ? ldnt(W + off) : 0.0;
    wn += wt * wt;
    double v[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) v[i] = (i < nbl && valid) ? ldnt(V + (int64_t)i * a.vstride + off) : 0.0;
#pragma unroll
    for (int i = 0; i < NB; ++i)
      if (i < nbl) acc[i] = mfma4(v[i], wt, acc[i]);
  }
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    double x = acc[i];
    x += __shfl_xor(x, 4, 64);
    x += __shfl_xor(x, 8, 64);
    if (i < nbl && ((lane >> 2) & 3) == 0) sred[w][i * 16 + (lane >> 4) * 4 + (lane & 3)] = x;
  }
  wn += __shfl_xor(wn, 4, 64);
  wn += __shfl_xor(wn, 8, 64);
  wn += __shfl_xor(wn, 16, 64);
  wn += __shfl_xor(wn, 32, 64);
  if (lane < 4) sred[w][nbl * 16 + lane] = wn;
  rs_store_partials<NW, ROW>(sred, nbl * 16 + 4, a.part + (int64_t)r.lg * a.lstride);
}

// Lane l of a 16 x 4 tile holds (row 16c + (l >> 2), column l & 3).  Used as the
// A operand of v_mfma_f64_4x4x4f64 a tile contracts over the rows; a product
// tile x M (M 4 x 4) needs the rows as the M index instead, i.e. the 4 x 4
// transpose inside each group of 16 lanes: lane l takes the value of lane
// ((l & 3) << 4) | (l & 12) | (l >> 4).
__device__ __forceinline__ double tile_transpose(double x, int lane) {
  const int src = ((lane & 3) << 4) | (lane & 12) | (lane >> 4);
  return __shfl(x, src, 64);
}

// W <- W - hsign V Hsrc over nbl blocks, then by MODE: nothing, pass 2 (V^T W
// and Gram(W) partials) or pass 3 (W <- W R1^{-1} and Gram(W) partials).  The
// update and the products run on the FP64 MFMA: the transposed V tile is the A
// operand, -hsign H the B operand and W the accumulator (D[i][j] at lane
// 16i + 4b + j is the tile's own layout).
template <int NW, int MODE, int NB>
__global__ __launch_bounds__(64 * NW) void k_upd4(KArgs a) {
  constexpr bool DOT = MODE == UPD_P2, GRAM = MODE != UPD_PLAIN, P3 = MODE == UPD_P3;
  RowSeg r;
  if (!row_seg(a, !a.ignore_done, r)) return;
  const int nbl = nblocks_of(a, r.s);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nch = (r.n + 15) >> 4;
  double* W = a.W + r.r0 * 4;
  const double* V = a.V + r.r0 * 4;
  constexpr int ROW = (DOT ? NB * 16 : 0) + 16;
  __shared__ double sred[GRAM ? NW : 1][ROW];
  // B operand of block i: B[k][j] = -hsign H[4i + k][j], k = lane >> 4, j = lane & 3
  __shared__ double sH[RS_B * 16];
  __shared__ double sH1[P3 ? RS_B * 16 : 1];  // pass 3: pass 2's B operands (-H1)
  __shared__ double sRinv[P3 ? 16 : 1];
  const double* Hs = a.Hsrc + r.s * a.hsrc_stride;
  for (int t = threadIdx.x; t < nbl * 16; t += blockDim.x) sH[t] = -a.hsign * Hs[t];
  if constexpr (P3) {
    const double* H1 = a.Hsrc1 + r.s * a.hsrc_stride;
    for (int t = threadIdx.x; t < nbl * 16; t += blockDim.x) sH1[t] = -1.0 * H1[t];
  }
  __syncthreads();
  if constexpr (P3) p3_prologue<4>(a, r.s, r.g == 0, sH, nbl, sRinv);
  const double* hb = sH + (lane >> 4) * 4 + (lane & 3);
  const double* hb1 = sH1 + (P3 ? (lane >> 4) * 4 + (lane & 3) : 0);
  double rb = 0.0;
  if constexpr (P3) rb = sRinv[(lane >> 4) * 4 + (lane & 3)];
  double acc[DOT ? NB : 1];
#pragma unroll
  for (int i = 0; i < (DOT ? NB : 1); ++i) acc[i] = 0.0;
  double accg = 0.0;
  const bool write = P3 || (MODE == UPD_PLAIN && (nbl > 0 || a.zero_init));
  for (int ch = r.g * NW + w; ch < nch; ch += r.G * NW) {
    const int64_t e = ((int64_t)ch << 6) + lane;
    const bool valid = e < (int64_t)r.n * 4;
    const double wt = (valid && !a.zero_init) ? ldnt(W + e) : 0.0;
    double v[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) v[i] = (i < nbl && valid) ? ldnt(V + (int64_t)i * a.vstride + e) : 0.0;
    double u0 = wt, u1 = 0.0;  // two accumulation chains, added at the end
    if constexpr (P3) {
      // W' = W - V H1 exactly as pass 2 formed it (chains u0, u1), and -V H2
      // in two chains of its own that start from zero (s0, s1), so the four
      // chains run side by side; then W'' = W' + (-V H2).  The tiles are kept
      // transposed.
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int i = 0; i < NB; ++i) v[i] = tile_transpose(v[i], lane);
#pragma unroll
      for (int i = 0; i < NB; i += 2) {
        if (i < nbl) {
          u0 = mfma4(v[i], hb1[16 * i], u0);
          s0 = mfma4(v[i], hb[16 * i], s0);
        }
        if (i + 1 < nbl) {
          u1 = mfma4(v[i + 1], hb1[16 * (i + 1)], u1);
          s1 = mfma4(v[i + 1], hb[16 * (i + 1)], s1);
        }
      }
      u0 = u0 + u1;
      u1 = s0 + s1;
    } else {
#pragma unroll
      for (int i = 0; i < NB; i += 2) {
        if (i < nbl) u0 = mfma4(tile_transpose(v[i], lane), hb[16 * i], u0);
        if (i + 1 < nbl) u1 = mfma4(tile_transpose(v[i + 1], lane), hb[16 * (i + 1)], u1);
      }
    }
    double wnew = u0 + u1;
    if (P3) wnew = mfma4(tile_transpose(wnew, lane), rb, 0.0);
    if (valid && write) W[e] = wnew;
    if (DOT) {
#pragma unroll
      for (int i = 0; i < NB; ++i)
        if (i < nbl) acc[i] = mfma4(v[i], wnew, acc[i]);
    }
    if (GRAM) accg = mfma4(wnew, wnew, accg);
  }
  if (!GRAM) return;
  int L = 0;
  if (DOT) {
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      double x = acc[i];
      x += __shfl_xor(x, 4, 64);
      x += __shfl_xor(x, 8, 64);
      if (i < nbl && ((lane >> 2) & 3) == 0) sred[w][i * 16 + (lane >> 4) * 4 + (lane & 3)] = x;
    }
    L = nbl * 16;
  }
  double x = accg;
  x += __shfl_xor(x, 4, 64);
  x += __shfl_xor(x, 8, 64);
  if (((lane >> 2) & 3) == 0) sred[w][L + (lane >> 4) * 4 + (lane & 3)] = x;
  if (P3) rs_store_partials<NW, ROW>(sred, 16, a.partg + (int64_t)r.lg * 16);
  else rs_store_partials<NW, ROW>(sred, L + 16, a.part + (int64_t)r.lg * a.lstride);
}

// ---------------------------------------------------------------------------
// kp = 8, 16: the NW wavefronts of a workgroup share the rows of a 16-row tile
// and split the V blocks (block i on wavefront i mod NW); their partial updates
// meet in LDS in a fixed order.
// ---------------------------------------------------------------------------
// pass 1: partial H1 and the squared column norms of W
template <int KP, int NW, int BPW>
__global__ __launch_bounds__(64 * NW) void k_dot_mfma(KArgs a) {
  constexpr int NT = KP / 4;
  RowSeg r;
  if (!row_seg(a, true, r)) return;
  const int nbl = a.nbl;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int c4 = lane & 3, rsub = lane >> 2;
  const int nch = (r.n + 15) >> 4;
  const double* W = a.W + r.r0 * KP;
  const double* V = a.V + r.r0 * KP;
  double acc[BPW][NT][NT];
  double wn[NT];
#pragma unroll
  for (int bi = 0; bi < BPW; ++bi)
#pragma unroll
    for (int h = 0; h < NT; ++h)
#pragma unroll
      for (int h2 = 0; h2 < NT; ++h2) acc[bi][h][h2] = 0.0;
#pragma unroll
  for (int h = 0; h < NT; ++h) wn[h] = 0.0;
  for (int ch = r.g; ch < nch; ch += r.G) {
    const int row = (ch << 4) + rsub;
    const bool valid = row < r.n;
    double wt[NT];
#pragma unroll
    for (int h = 0; h < NT; ++h) wt[h] = valid ? W[(int64_t)row * KP + 4 * h + c4] : 0.0;
    if (w == 0) {
#pragma unroll
      for (int h = 0; h < NT; ++h) wn[h] += wt[h] * wt[h];
    }
#pragma unroll
    for (int bi = 0; bi < BPW; ++bi) {
      const int i = w + NW * bi;
      if (i < nbl) {
        const double* Vi = V + (int64_t)i * a.vstride + (int64_t)row * KP + c4;
#pragma unroll
        for (int h = 0; h < NT; ++h) {
          const double v = valid ? Vi[4 * h] : 0.0;
#pragma unroll
          for (int h2 = 0; h2 < NT; ++h2) acc[bi][h][h2] = mfma4(v, wt[h2], acc[bi][h][h2]);
        }
      }
    }
  }
  double* mypart = a.part + (int64_t)r.lg * a.lstride;
#pragma unroll
  for (int bi = 0; bi < BPW; ++bi) {
    const int i = w + NW * bi;
#pragma unroll
    for (int h = 0; h < NT; ++h)
#pragma unroll
      for (int h2 = 0; h2 < NT; ++h2) {
        double x = acc[bi][h][h2];
        x += __shfl_xor(x, 4, 64);
        x += __shfl_xor(x, 8, 64);
        if (i < nbl && ((lane >> 2) & 3) == 0) {
          const int ii = lane >> 4, jj = lane & 3;
          mypart[(i * KP + 4 * h + ii) * KP + 4 * h2 + jj] = x;
        }
      }
  }
  if (w == 0) {
#pragma unroll
    for (int h = 0; h < NT; ++h) {
      double x = wn[h];
      x += __shfl_xor(x, 4, 64);
      x += __shfl_xor(x, 8, 64);
      x += __shfl_xor(x, 16, 64);
      x += __shfl_xor(x, 32, 64);
      if (lane < 4) mypart[nbl * KP * KP + 4 * h + lane] = x;
    }
  }
}

// W <- W - hsign [V_0..V_{nbl-1}] Hsrc, then by MODE (see k_upd4).  Dynamic LDS:
// hsign Hsrc (nbl_max KP^2) and the exchange buffer [2][NW][64][KP/4].
template <int KP, int NW, int BPW, int MODE>
__global__ __launch_bounds__(64 * NW) void k_upd_mfma(KArgs a) {
  constexpr int NT = KP / 4;
  constexpr bool DOT = MODE == UPD_P2, GRAM = MODE != UPD_PLAIN, P3 = MODE == UPD_P3;
  RowSeg r;
  if (!row_seg(a, !a.ignore_done, r)) return;
  const int nbl = nblocks_of(a, r.s);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int c4 = lane & 3, rsub = lane >> 2;
  const int nch = (r.n + 15) >> 4;
  double* W = a.W + r.r0 * KP;
  const double* V = a.V + r.r0 * KP;
  extern __shared__ double sh[];
  double* sH = sh;                          // nbl*KP x KP
  double* su = sh + (size_t)nbl * KP * KP;  // [2][NW][64][NT]
  __shared__ double sRinv[P3 ? KP * KP : 1];
  const double* Hs = a.Hsrc + r.s * a.hsrc_stride;
  for (int t = threadIdx.x; t < nbl * KP * KP; t += blockDim.x) sH[t] = a.hsign * Hs[t];
  __syncthreads();
  if constexpr (P3) load_r1inv(a, r.s, KP * KP, sRinv);
  double acc[DOT ? BPW : 1][NT][NT];
  double accg[GRAM ? NT : 1][NT];
#pragma unroll
  for (int bi = 0; bi < (DOT ? BPW : 1); ++bi)
#pragma unroll
    for (int h = 0; h < NT; ++h)
#pragma unroll
      for (int h2 = 0; h2 < NT; ++h2) acc[bi][h][h2] = 0.0;
#pragma unroll
  for (int h = 0; h < (GRAM ? NT : 1); ++h)
#pragma unroll
    for (int h2 = 0; h2 < NT; ++h2) accg[h][h2] = 0.0;
  const bool write = P3 || nbl > 0 || a.zero_init;
  int buf = 0;
  for (int ch = r.g; ch < nch; ch += r.G) {
    const int row = (ch << 4) + rsub;
    const bool valid = row < r.n;
    double wt[NT], u[NT];
#pragma unroll
    for (int h = 0; h < NT; ++h) {
      wt[h] = (valid && !a.zero_init) ? W[(int64_t)row * KP + 4 * h + c4] : 0.0;
      u[h] = 0.0;
    }
    double vt[BPW][NT];
#pragma unroll
    for (int bi = 0; bi < BPW; ++bi) {
      const int i = w + NW * bi;
      if (i < nbl) {
        const double* Vi = V + (int64_t)i * a.vstride + (int64_t)row * KP + c4;
#pragma unroll
        for (int h = 0; h < NT; ++h) vt[bi][h] = valid ? Vi[4 * h] : 0.0;
        const double* Hi = sH + (size_t)i * KP * KP;
#pragma unroll
        for (int h = 0; h < NT; ++h) {
          const double v0 = quad_bcast<0>(vt[bi][h]);
          const double v1 = quad_bcast<1>(vt[bi][h]);
          const double v2 = quad_bcast<2>(vt[bi][h]);
          const double v3 = quad_bcast<3>(vt[bi][h]);
#pragma unroll
          for (int h2 = 0; h2 < NT; ++h2) {
            const int cc = 4 * h2 + c4;
            double x = u[h2];
            x = fma(v0, Hi[(4 * h + 0) * KP + cc], x);
            x = fma(v1, Hi[(4 * h + 1) * KP + cc], x);
            x = fma(v2, Hi[(4 * h + 2) * KP + cc], x);
            x = fma(v3, Hi[(4 * h + 3) * KP + cc], x);
            u[h2] = x;
          }
        }
      } else {
#pragma unroll
        for (int h = 0; h < NT; ++h) vt[bi][h] = 0.0;
      }
    }
    double wnew[NT];
    if (NW > 1) {
      double* mys = su + ((size_t)(buf * NW + w) * 64 + lane) * NT;
#pragma unroll
      for (int h = 0; h < NT; ++h) mys[h] = u[h];
      __syncthreads();
#pragma unroll
      for (int h = 0; h < NT; ++h) {
        double tot = 0.0;
        for (int q = 0; q < NW; ++q) tot += su[((size_t)(buf * NW + q) * 64 + lane) * NT + h];
        wnew[h] = wt[h] - tot;
      }
      buf ^= 1;
    } else {
#pragma unroll
      for (int h = 0; h < NT; ++h) wnew[h] = wt[h] - u[h];
    }
    if (P3 && w == 0) {
      // W1 = W'' R1^{-1}: column 4 h2 + c4 of the row from the row's KP values
      double o[NT];
#pragma unroll
      for (int h2 = 0; h2 < NT; ++h2) o[h2] = 0.0;
#pragma unroll
      for (int h = 0; h < NT; ++h) {
        const double x0 = quad_bcast<0>(wnew[h]);
        const double x1 = quad_bcast<1>(wnew[h]);
        const double x2 = quad_bcast<2>(wnew[h]);
        const double x3 = quad_bcast<3>(wnew[h]);
#pragma unroll
        for (int h2 = 0; h2 < NT; ++h2) {
          const int cc = 4 * h2 + c4;
          double x = o[h2];
          x = fma(x0, sRinv[(4 * h + 0) * KP + cc], x);
          x = fma(x1, sRinv[(4 * h + 1) * KP + cc], x);
          x = fma(x2, sRinv[(4 * h + 2) * KP + cc], x);
          x = fma(x3, sRinv[(4 * h + 3) * KP + cc], x);
          o[h2] = x;
        }
      }
#pragma unroll
      for (int h = 0; h < NT; ++h) wnew[h] = o[h];
    }
    if (w == 0 && valid && write) {
#pragma unroll
      for (int h = 0; h < NT; ++h) W[(int64_t)row * KP + 4 * h + c4] = wnew[h];
    }
    if (DOT) {
#pragma unroll
      for (int bi = 0; bi < BPW; ++bi)
#pragma unroll
        for (int h = 0; h < NT; ++h)
#pragma unroll
          for (int h2 = 0; h2 < NT; ++h2) acc[bi][h][h2] = mfma4(vt[bi][h], wnew[h2], acc[bi][h][h2]);
    }
    if (GRAM && w == 0) {
#pragma unroll
      for (int h = 0; h < NT; ++h)
#pragma unroll
        for (int h2 = 0; h2 < NT; ++h2) accg[h][h2] = mfma4(wnew[h], wnew[h2], accg[h][h2]);
    }
  }
  if (!GRAM) return;
  double* mypart = P3 ? a.partg + (int64_t)r.lg * KP * KP : a.part + (int64_t)r.lg * a.lstride;
  const int goff = P3 ? 0 : nbl * KP * KP;
  if (DOT) {
#pragma unroll
    for (int bi = 0; bi < BPW; ++bi) {
      const int i = w + NW * bi;
#pragma unroll
      for (int h = 0; h < NT; ++h)
#pragma unroll
        for (int h2 = 0; h2 < NT; ++h2) {
          double x = acc[bi][h][h2];
          x += __shfl_xor(x, 4, 64);
          x += __shfl_xor(x, 8, 64);
          if (i < nbl && ((lane >> 2) & 3) == 0)
            mypart[(i * KP + 4 * h + (lane >> 4)) * KP + 4 * h2 + (lane & 3)] = x;
        }
    }
  }
  if (w == 0) {
#pragma unroll
    for (int h = 0; h < NT; ++h)
#pragma unroll
      for (int h2 = 0; h2 < NT; ++h2) {
        double x = accg[h][h2];
        x += __shfl_xor(x, 4, 64);
        x += __shfl_xor(x, 8, 64);
        if (((lane >> 2) & 3) == 0) mypart[goff + (4 * h + (lane >> 4)) * KP + 4 * h2 + (lane & 3)] = x;
      }
  }
}

// ---------------------------------------------------------------------------
// row-per-lane path (kp = 1, 2): wavefronts split the V blocks of 64-row tiles
// ---------------------------------------------------------------------------
template <int KP, int NW, int BPW>
__global__ __launch_bounds__(64 * NW) void k_dot_row(KArgs a) {
  RowSeg r;
  if (!row_seg(a, true, r)) return;
  const int nbl = a.nbl;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nch = (r.n + 63) >> 6;
  const double* W = a.W + r.r0 * KP;
  const double* V = a.V + r.r0 * KP;
  double acc[BPW][KP][KP];
  double wn[KP];
#pragma unroll
  for (int bi = 0; bi < BPW; ++bi)
#pragma unroll
    for (int x = 0; x < KP; ++x)
#pragma unroll
      for (int y = 0; y < KP; ++y) acc[bi][x][y] = 0.0;
#pragma unroll
  for (int x = 0; x < KP; ++x) wn[x] = 0.0;
  for (int ch = r.g; ch < nch; ch += r.G) {
    const int row = (ch << 6) + lane;
    const bool valid = row < r.n;
    double wt[KP];
#pragma unroll
    for (int x = 0; x < KP; ++x) wt[x] = valid ? W[(int64_t)row * KP + x] : 0.0;
    if (w == 0) {
#pragma unroll
      for (int x = 0; x < KP; ++x) wn[x] += wt[x] * wt[x];
    }
#pragma unroll
    for (int bi = 0; bi < BPW; ++bi) {
      const int i = w + NW * bi;
      if (i < nbl) {
#pragma unroll
        for (int x = 0; x < KP; ++x) {
          const double v = valid ? V[(int64_t)i * a.vstride + (int64_t)row * KP + x] : 0.0;
#pragma unroll
          for (int y = 0; y < KP; ++y) acc[bi][x][y] += v * wt[y];
        }
      }
    }
  }
  double* mypart = a.part + (int64_t)r.lg * a.lstride;
#pragma unroll
  for (int bi = 0; bi < BPW; ++bi) {
    const int i = w + NW * bi;
#pragma unroll
    for (int x = 0; x < KP; ++x)
#pragma unroll
      for (int y = 0; y < KP; ++y) {
        const double sum = wave_sum(acc[bi][x][y]);
        if (i < nbl && lane == 0) mypart[(i * KP + x) * KP + y] = sum;
      }
  }
  if (w == 0) {
#pragma unroll
    for (int x = 0; x < KP; ++x) {
      const double sum = wave_sum(wn[x]);
      if (lane == 0) mypart[nbl * KP * KP + x] = sum;
    }
  }
}

template <int KP, int NW, int BPW, int MODE>
__global__ __launch_bounds__(64 * NW) void k_upd_row(KArgs a) {
  constexpr bool DOT = MODE == UPD_P2, GRAM = MODE != UPD_PLAIN, P3 = MODE == UPD_P3;
  RowSeg r;
  if (!row_seg(a, !a.ignore_done, r)) return;
  const int nbl = nblocks_of(a, r.s);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nch = (r.n + 63) >> 6;
  double* W = a.W + r.r0 * KP;
  const double* V = a.V + r.r0 * KP;
  extern __shared__ double sh[];
  double* sH = sh;
  double* su = sh + (size_t)nbl * KP * KP;  // [2][NW][64][KP]
  __shared__ double sRinv[P3 ? KP * KP : 1];
  const double* Hs = a.Hsrc + r.s * a.hsrc_stride;
  for (int t = threadIdx.x; t < nbl * KP * KP; t += blockDim.x) sH[t] = a.hsign * Hs[t];
  __syncthreads();
  if constexpr (P3) load_r1inv(a, r.s, KP * KP, sRinv);
  double acc[DOT ? BPW : 1][KP][KP];
  double accg[GRAM ? KP : 1][KP];
#pragma unroll
  for (int bi = 0; bi < (DOT ? BPW : 1); ++bi)
#pragma unroll
    for (int x = 0; x < KP; ++x)
#pragma unroll
      for (int y = 0; y < KP; ++y) acc[bi][x][y] = 0.0;
#pragma unroll
  for (int x = 0; x < (GRAM ? KP : 1); ++x)
#pragma unroll
    for (int y = 0; y < KP; ++y) accg[x][y] = 0.0;
  const bool write = P3 || nbl > 0 || a.zero_init;
  int buf = 0;
  for (int ch = r.g; ch < nch; ch += r.G) {
    const int row = (ch << 6) + lane;
    const bool valid = row < r.n;
    double wt[KP], u[KP];
#pragma unroll
    for (int x = 0; x < KP; ++x) {
      wt[x] = (valid && !a.zero_init) ? W[(int64_t)row * KP + x] : 0.0;
      u[x] = 0.0;
    }
    double vt[BPW][KP];
#pragma unroll
    for (int bi = 0; bi < BPW; ++bi) {
      const int i = w + NW * bi;
#pragma unroll
      for (int x = 0; x < KP; ++x)
        vt[bi][x] = (i < nbl && valid) ? V[(int64_t)i * a.vstride + (int64_t)row * KP + x] : 0.0;
      if (i < nbl) {
        const double* Hi = sH + (size_t)i * KP * KP;
#pragma unroll
        for (int x = 0; x < KP; ++x)
#pragma unroll
          for (int y = 0; y < KP; ++y) u[y] = fma(vt[bi][x], Hi[x * KP + y], u[y]);
      }
    }
    double wnew[KP];
    if (NW > 1) {
      double* mys = su + ((size_t)(buf * NW + w) * 64 + lane) * KP;
#pragma unroll
      for (int x = 0; x < KP; ++x) mys[x] = u[x];
      __syncthreads();
#pragma unroll
      for (int x = 0; x < KP; ++x) {
        double tot = 0.0;
        for (int q = 0; q < NW; ++q) tot += su[((size_t)(buf * NW + q) * 64 + lane) * KP + x];
        wnew[x] = wt[x] - tot;
      }
      buf ^= 1;
    } else {
#pragma unroll
      for (int x = 0; x < KP; ++x) wnew[x] = wt[x] - u[x];
    }
    if (P3) {
      double o[KP];
#pragma unroll
      for (int y = 0; y < KP; ++y) {
        double t = 0.0;
#pragma unroll
        for (int x = 0; x < KP; ++x) t = fma(wnew[x], sRinv[x * KP + y], t);
        o[y] = t;
      }
#pragma unroll
      for (int y = 0; y < KP; ++y) wnew[y] = o[y];
    }
    if (w == 0 && valid && write) {
#pragma unroll
      for (int x = 0; x < KP; ++x) W[(int64_t)row * KP + x] = wnew[x];
    }
    if (DOT) {
#pragma unroll
      for (int bi = 0; bi < BPW; ++bi)
#pragma unroll
        for (int x = 0; x < KP; ++x)
#pragma unroll
          for (int y = 0; y < KP; ++y) acc[bi][x][y] += vt[bi][x] * wnew[y];
    }
    if (GRAM && w == 0) {
#pragma unroll
      for (int x = 0; x < KP; ++x)
#pragma unroll
        for (int y = 0; y < KP; ++y) accg[x][y] += wnew[x] * wnew[y];
    }
  }
  if (!GRAM) return;
  double* mypart = P3 ? a.partg + (int64_t)r.lg * KP * KP : a.part + (int64_t)r.lg * a.lstride;
  const int goff = P3 ? 0 : nbl * KP * KP;
  if (DOT) {
#pragma unroll
    for (int bi = 0; bi < BPW; ++bi) {
      const int i = w + NW * bi;
#pragma unroll
      for (int x = 0; x < KP; ++x)
#pragma unroll
        for (int y = 0; y < KP; ++y) {
          const double sum = wave_sum(acc[bi][x][y]);
          if (i < nbl && lane == 0) mypart[(i * KP + x) * KP + y] = sum;
        }
    }
  }
  if (w == 0) {
#pragma unroll
    for (int x = 0; x < KP; ++x)
#pragma unroll
      for (int y = 0; y < KP; ++y) {
        const double sum = wave_sum(accg[x][y]);
        if (lane == 0) mypart[goff + x * KP + y] = sum;
      }
  }
}

// ---------------------------------------------------------------------------
// one-workgroup-per-segment kernels: second Cholesky factor + Hessenberg least
// squares, Y solve, cycle and state initialisation
// ---------------------------------------------------------------------------
// Prologue: Gram(W1) from the pass-3 partials, R2 = chol(Gram(W1)), the
// subdiagonal block H_{j+1,j} = R2 R1 and the deficiency test
// |(R2 R1)_cc| <= 1e-14 max_c ||W_c|| (block steps); R2^{-1} (zero when
// deficient) is kept for the next step's V_{j+1} = W1 R2^{-1}.  Cycle start
// (mode 1): the block is S of R_0 = V_0 S and goes to G; a deficient R_0 ends
// the solve with a breakdown.  A deficient block step ends the cycle only (its
// least-squares solution still updates X, and the solve restarts).  Block
// step: Householder update of the QR
// factorisation of the block Hessenberg matrix for the new block column j, the
// transformed right-hand side G, and the least-squares residual of every column.
template <int KP>
__global__ __launch_bounds__(256) void k_hess(KArgs a) {
  const int s = a.slist[blockIdx.x];
  DevState* st = a.st + s;
  if (st->done) return;
  const SegDesc& d = a.seg[s];
  __shared__ double sG1[KP * KP], sR2[KP * KP], sR2inv[KP * KP], sHs[KP * KP];
  __shared__ int sdef;
  block_reduce_partials(a.partg + (int64_t)d.wg0 * KP * KP, KP * KP, d.G, sG1);
  const int j = st->j, m = st->m, kact = st->kact;
  const int lane = threadIdx.x;
  if (lane == 0) {
    bool ok = chol_upper(sG1, KP, kact, 0.0, sR2, sR2inv) && !st->deficient;
    for (int r = 0; r < KP; ++r)
      for (int c = 0; c < KP; ++c) {
        double x = 0.0;
        if (r < kact && c < kact)
          for (int t = r; t <= c; ++t) x += sR2[r * KP + t] * st->R1[t * KP + c];
        sHs[r * KP + c] = x;
      }
    const double thr = a.mode == 0 ? 1e-14 * st->wscale : 0.0;
    for (int c = 0; c < kact; ++c)
      if (!(fabs(sHs[c * KP + c]) > thr)) ok = false;
    if (!ok)
      for (int t = 0; t < KP * KP; ++t) { sHs[t] = 0.0; sR2inv[t] = 0.0; }
    for (int t = 0; t < KP * KP; ++t) st->R2inv[t] = sR2inv[t];
    sdef = ok ? 0 : 1;
    if (!ok) st->deficient = 1;
  }
  __syncthreads();
  const int ldh = a.ldh;
  double* Hbar = a.Hbar + s * a.hbs;
  double* Gs = a.G + s * a.gs;
  double* refl = a.refl + s * a.rfs;
  volatile int* hf = a.hinfo + 4 * s;
  if (a.mode == 1) {
    if (lane == 0) {
      for (int r = 0; r < KP; ++r)
        for (int c = 0; c < KP; ++c) Gs[r + (int64_t)c * ldh] = sHs[r * KP + c];
      if (sdef) {
        st->breakdown = 1;
        st->done = 1;
        hf[0] = 0;
        hf[1] = 1;
        hf[2] = 1;
        hf[3] = st->nanflag;
        __threadfence_system();
      }
    }
    return;
  }
  extern __shared__ double sh[];
  const int q0 = j * KP, nr = (j + 2) * KP;
  constexpr int RL = KP + 2;                   // stored reflector: tau, v_1..v_KP, (unused)
  double* col = sh;                            // [KP][ldh]
  double* rf = col + (size_t)KP * ldh;         // [q0 + KP][RL]
  double* gw = rf + (size_t)(q0 + KP) * RL;    // [KP][2 KP] window of G
  const int r1 = (j + 1) * KP;
  for (int t = lane; t < KP * nr; t += blockDim.x) {
    const int c = t / nr, r = t % nr;
    col[(size_t)c * ldh + r] = (r < r1) ? Hbar[r + (int64_t)(q0 + c) * ldh] : sHs[(r - r1) * KP + c];
  }
  for (int t = lane; t < q0 * RL; t += blockDim.x) rf[t] = refl[t];
  for (int t = lane; t < KP * 2 * KP; t += blockDim.x) {
    const int c = t / (2 * KP), r = t % (2 * KP);
    gw[c * 2 * KP + r] = Gs[(q0 + r) + (int64_t)c * ldh];
  }
  __syncthreads();
  // earlier reflectors, in order, on the new columns.  Reflector q touches rows
  // q..q+KP; lane t keeps those KP+1 rows of its column in registers, row r at
  // slot r mod (KP+1), retiring row q to LDS and taking in row q+KP+1 each time.
  if (lane < KP) {
    double* x = col + (size_t)lane * ldh;
    double w[KP + 1];
#pragma unroll
    for (int i = 0; i <= KP; ++i) w[i] = x[i];
    for (int base = 0; base < q0; base += KP + 1) {
#pragma unroll
      for (int r = 0; r <= KP; ++r) {
        const int q = base + r;
        if (q < q0) {
          const double* v = rf + (size_t)q * RL;
          double dd = w[r];
#pragma unroll
          for (int i = 1; i <= KP; ++i) dd = fma(v[i], w[(r + i) % (KP + 1)], dd);
          dd *= v[0];
          w[r] -= dd;
#pragma unroll
          for (int i = 1; i <= KP; ++i) w[(r + i) % (KP + 1)] = fma(-dd, v[i], w[(r + i) % (KP + 1)]);
          x[q] = w[r];
          w[r] = (q + KP + 1 < nr) ? x[q + KP + 1] : 0.0;
        }
      }
    }
#pragma unroll
    for (int pidx = 0; pidx <= KP; ++pidx) {
      const int row = q0 + (((pidx - q0) % (KP + 1)) + (KP + 1)) % (KP + 1);
      if (row < nr) x[row] = w[pidx];
    }
  }
  __syncthreads();
  // new reflectors, one column at a time
  for (int t = 0; t < KP; ++t) {
    const int q = q0 + t;
    double* v = rf + (size_t)q * RL;
    if (lane == 0) {
      double* x = col + (size_t)t * ldh;
      const double alpha = x[q];
      double sigma = 0.0;
      for (int r = 1; r <= KP; ++r) sigma += x[q + r] * x[q + r];
      double tau = 0.0, beta = alpha;
      if (sigma != 0.0) {
        const double nrm = sqrt(alpha * alpha + sigma);
        beta = (alpha >= 0.0) ? -nrm : nrm;
        tau = (beta - alpha) / beta;
        const double sc = 1.0 / (alpha - beta);
        for (int r = 1; r <= KP; ++r) v[r] = x[q + r] * sc;
      } else {
        for (int r = 1; r <= KP; ++r) v[r] = 0.0;
      }
      v[0] = tau;
      v[KP + 1] = 0.0;
      x[q] = beta;
      for (int r = 1; r <= KP; ++r) x[q + r] = 0.0;
    }
    __syncthreads();
    const double tau = v[0];
    if (tau != 0.0) {
      double* x = nullptr;
      int off = 0;
      if (lane > t && lane < KP) { x = col + (size_t)lane * ldh; off = q; }
      else if (lane >= KP && lane < 2 * KP) { x = gw + (size_t)(lane - KP) * 2 * KP; off = t; }
      if (x) {
        double dd = x[off];
        for (int r = 1; r <= KP; ++r) dd = fma(v[r], x[off + r], dd);
        dd *= tau;
        x[off] -= dd;
        for (int r = 1; r <= KP; ++r) x[off + r] = fma(-dd, v[r], x[off + r]);
      }
    }
    __syncthreads();
  }
  // write back
  for (int t = lane; t < KP * nr; t += blockDim.x) {
    const int c = t / nr, r = t % nr;
    Hbar[r + (int64_t)(q0 + c) * ldh] = col[(size_t)c * ldh + r];
  }
  for (int t = lane; t < KP * RL; t += blockDim.x) refl[(size_t)q0 * RL + t] = rf[(size_t)q0 * RL + t];
  for (int t = lane; t < KP * 2 * KP; t += blockDim.x) {
    const int c = t / (2 * KP), r = t % (2 * KP);
    Gs[(q0 + r) + (int64_t)c * ldh] = gw[c * 2 * KP + r];
  }
  __syncthreads();
  if (lane == 0) {
    bool done = true;
    for (int c = 0; c < kact; ++c) {
      double sq = 0.0;
      for (int r = KP; r < 2 * KP; ++r) sq += gw[c * 2 * KP + r] * gw[c * 2 * KP + r];
      const double e = sqrt(sq) / st->bnorm[c];
      st->est[c] = e;
      if (!(e <= st->tol)) done = false;
      if (e != e) st->nanflag = 1;
    }
    if (st->deficient) done = true;
    if (st->nanflag) done = true;
    if (j + 1 >= m) done = true;
    st->j = j + 1;
    st->done = done ? 1 : 0;
    hf[0] = j + 1;
    hf[1] = done ? 1 : 0;
    hf[2] = st->breakdown;
    hf[3] = st->nanflag;
    __threadfence_system();
  }
}

// Y = R^{-1} G(0:J, :) with R the triangle of the transformed Hessenberg
// matrix, J = steps * kp; padded positions get y = 0.  Column panels of R go
// through LDS.
template <int KP>
__global__ __launch_bounds__(256) void k_ysolve(KArgs a, int PW) {
  const int s = a.slist[blockIdx.x];
  const DevState* st = a.st + s;
  const int J = st->j * KP;
  const int kact = st->kact;
  const double* Hbar = a.Hbar + s * a.hbs;
  const double* Gs = a.G + s * a.gs;
  double* Y = a.Y + s * a.ys;
  extern __shared__ double sh[];
  double* g = sh;                       // [J][KP]
  double* Rp = g + (size_t)J * KP;      // [PW][J] panel, column-major
  for (int t = threadIdx.x; t < J * KP; t += blockDim.x) {
    const int r = t / KP, c = t % KP;
    g[t] = Gs[r + (int64_t)c * a.ldh];
  }
  for (int p1 = J; p1 > 0; p1 -= PW) {
    const int p0 = p1 - PW > 0 ? p1 - PW : 0;
    __syncthreads();
    for (int t = threadIdx.x; t < (p1 - p0) * p1; t += blockDim.x) {
      const int cc = t / p1, r = t % p1;
      Rp[(size_t)cc * J + r] = Hbar[r + (int64_t)(p0 + cc) * a.ldh];
    }
    __syncthreads();
    for (int i = p1 - 1; i >= p0; --i) {
      const bool pad = (i % KP) >= kact;
      const double* Ri = Rp + (size_t)(i - p0) * J;
      if (threadIdx.x < KP) {
        const double y = pad ? 0.0 : g[i * KP + threadIdx.x] / Ri[i];
        g[i * KP + threadIdx.x] = y;
      }
      __syncthreads();
      for (int t = threadIdx.x; t < i * KP; t += blockDim.x) {
        const int r = t / KP, c = t % KP;
        g[t] = fma(-Ri[r], g[i * KP + c], g[t]);
      }
      __syncthreads();
    }
  }
  for (int t = threadIdx.x; t < J * KP; t += blockDim.x) Y[t] = g[t];
}

// cycle start: G = 0, step counters reset
__global__ __launch_bounds__(256) void k_init_cycle(KArgs a, int kp) {
  const int s = a.slist[blockIdx.x];
  DevState* st = a.st + s;
  double* Gs = a.G + s * a.gs;
  const int rows = (a.m + 1) * kp;
  for (int t = threadIdx.x; t < rows * kp; t += blockDim.x) {
    const int r = t % rows, c = t / rows;
    Gs[r + (int64_t)c * a.ldh] = 0.0;
  }
  if (threadIdx.x == 0) {
    st->j = 0;
    st->done = 0;
    st->deficient = 0;
    st->breakdown = 0;
    st->nanflag = 0;
    volatile int* hf = a.hinfo + 4 * s;
    hf[0] = 0;
    hf[1] = 0;
    hf[2] = 0;
    hf[3] = 0;
    __threadfence_system();
  }
}

// per-solve state from the segment descriptor
__global__ void k_state_init(const SegDesc* seg, const int* slist, DevState* st, int m, double tol) {
  const int s = slist[blockIdx.x];
  DevState* x = st + s;
  const int kact = seg[s].kact;
  if (threadIdx.x == 0) {
    x->j = 0; x->done = 0; x->deficient = 0; x->breakdown = 0;
    x->kact = kact; x->m = m; x->nanflag = 0; x->pad0 = 0;
    x->tol = tol; x->wscale = 0.0;
  }
  if (threadIdx.x < KMAX) {
    x->bnorm[threadIdx.x] = (threadIdx.x < kact) ? seg[s].bnorm[threadIdx.x] : 1.0;
    x->est[threadIdx.x] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// CSR SpMM over the segments of a batch: Y = alpha Op X + beta Bsrc (kp-wide
// row-major blocks of the concatenated layout), LPR lanes per row.  Op is the
// segment's A (which 0), its preconditioner (which 1: identity without one,
// P_1 into Yalt for a factored Q P_1) or Q (which 2, factored segments only).
// CONV: X holds W1 of the previous step; the kernel multiplies by the segment's
// R2^{-1} (M) on the fly, Y = Op (W1 M) = (Op W1) M, and writes V_j = W1 M.
// ---------------------------------------------------------------------------
struct SpArgs {
  const SegDesc* seg;
  const int* stab;      // logical SpMM workgroup -> segment (-1: padding)
  const DevState* st;
  int which;
  int check_done;
  const double* X;
  double* Y;
  double* Yalt;
  const double* Bsrc;
  double alpha, beta;
  double* Vout;
  int vec;              // X rows may be read as double2
  int linear;           // take workgroups in launch order (else the per-XCD remap)
};

// rows per SpMM workgroup: 128 for kp <= 4 (a row's X is at most 32 bytes, and
// twice the rows per workgroup keep more of the gathered rows in its CU's L1),
// 64 for kp 8 and 16
template <int KP>
constexpr int sp_rows() { return KP <= 4 ? 128 : 64; }
// SpMM variants of the batched engine: 1, 2, 4, 8 lanes per row taking the
// row's entries in turn (k_spmm_seg), or the column split (k_spmm_cs)
constexpr int SPMM_COLSPLIT = 16;
static bool spmm_variant_ok(int v) { return v == 1 || v == 2 || v == 4 || v == 8 || v == SPMM_COLSPLIT; }

template <int KP, int LPR, bool CONV>
__global__ __launch_bounds__(sp_rows<KP>() * LPR) void k_spmm_seg(SpArgs a) {
  const int lg = a.linear ? (int)blockIdx.x : xcd_swizzle(blockIdx.x, gridDim.x);
  const int s = a.stab[lg];
  if (s < 0) return;
  if (a.check_done && a.st[s].done) return;
  const SegDesc& d = a.seg[s];
  const int pk = d.pkind;
  const int32_t* rp;
  const int32_t* cl;
  const double* vl;
  const int32_t* sp;   // sliced ELL view, or nullptr for CSR
  const int32_t* sw;
  const int32_t* sc;
  const double* sv;
  bool ident = false;
  double* Y = a.Y;
  double alpha = a.alpha, beta = a.beta;
  const double* Bsrc = a.Bsrc;
  if (a.which == 0) {
    rp = d.arow; cl = d.acol; vl = d.aval;
    sp = d.a_sp; sw = d.a_sw; sc = d.a_sc; sv = d.a_sv;
  } else if (a.which == 1) {
    ident = (pk == 0);
    rp = d.prow; cl = d.pcol; vl = d.pval;
    sp = d.p_sp; sw = d.p_sw; sc = d.p_sc; sv = d.p_sv;
    if (pk == 2) { Y = a.Yalt; alpha = 1.0; beta = 0.0; Bsrc = nullptr; }
  } else {
    if (pk != 2) return;
    rp = d.prow; cl = d.pcol; vl = d.qval;
    sp = d.p_sp; sw = d.p_sw; sc = d.p_sc; sv = d.q_sv;
  }
  __shared__ double sM[CONV ? KP * KP : 1];
  if constexpr (CONV) {
    for (int t = threadIdx.x; t < KP * KP; t += blockDim.x) sM[t] = a.st[s].R2inv[t];
    __syncthreads();
  }
  const int64_t base = d.r0 * KP;
  const double* X = a.X + base;
  Y += base;
  const int local = (lg - d.sp0) * sp_rows<KP>() + (int)threadIdx.x / LPR;
  const int sub = (int)threadIdx.x % LPR;
  const bool valid = local < d.n;
  double acc[KP];
#pragma unroll
  for (int t = 0; t < KP; ++t) acc[t] = 0.0;
  if (valid) {
    if (ident) {
      if (sub == 0) {
#pragma unroll
        for (int t = 0; t < KP; ++t) acc[t] = X[(int64_t)local * KP + t];
      }
    } else if (sp) {
      // sliced ELL: entry k of the row at ptr[slice] + 64 k + row % 64; the LPR
      // lanes of a row take k = sub, sub + LPR, ...  The pattern (columns) and
      // a factored P_1 are shared by the points of a sequence and stay cached;
      // a point's own values stream (nontemporal)
      // Entries go in batches of EB: all column and value loads, then all X
      // rows, then the products in entry order (fewer dependent memory waits).
      // Padded slots (column -1, value 0) gather nothing
      const int64_t base = sp[local >> 6] + (local & 63);
      const int w = sw[local >> 6];
      const bool own = !(a.which == 1 && (pk == 2 || pk == 3));
      constexpr int EB = KP <= 4 ? 8 : (KP == 8 ? 4 : 2);
      for (int k0 = sub; k0 < w; k0 += EB * LPR) {
        int c[EB];
        double v[EB];
#pragma unroll
        for (int t = 0; t < EB; ++t) {
          const int k = k0 + t * LPR;
          const int64_t q = base + (int64_t)k * 64;
          c[t] = -1;  // past the slice width, or a padded slot: no gather
          v[t] = 0.0;
          if (k < w) {
            c[t] = sc[q];
            v[t] = own ? __builtin_nontemporal_load(sv + q) : sv[q];
          }
        }
        if constexpr (KP % 2 == 0) {
          double2 xv[EB][KP / 2];
#pragma unroll
          for (int t = 0; t < EB; ++t) {
            const double2* xr = reinterpret_cast<const double2*>(X + (int64_t)(c[t] < 0 ? 0 : c[t]) * KP);
#pragma unroll
            for (int u = 0; u < KP / 2; ++u) xv[t][u] = c[t] >= 0 ? xr[u] : make_double2(0.0, 0.0);
          }
#pragma unroll
          for (int t = 0; t < EB; ++t) {
            if (k0 + t * LPR < w) {
#pragma unroll
              for (int u = 0; u < KP / 2; ++u) {
                acc[2 * u] = fma(v[t], xv[t][u].x, acc[2 * u]);
                acc[2 * u + 1] = fma(v[t], xv[t][u].y, acc[2 * u + 1]);
              }
            }
          }
        } else {
          double xv[EB][KP];
#pragma unroll
          for (int t = 0; t < EB; ++t)
#pragma unroll
            for (int u = 0; u < KP; ++u) xv[t][u] = c[t] >= 0 ? X[(int64_t)c[t] * KP + u] : 0.0;
#pragma unroll
          for (int t = 0; t < EB; ++t) {
            if (k0 + t * LPR < w) {
#pragma unroll
              for (int u = 0; u < KP; ++u) acc[u] = fma(v[t], xv[t][u], acc[u]);
            }
          }
        }
      }
    } else {
      const int e1 = rp[local + 1];
      if constexpr (KP % 2 == 0) {
        if (a.vec) {
          for (int e = rp[local] + sub; e < e1; e += LPR) {
            const int c = cl[e];
            const double v = vl[e];
            const double2* xr = reinterpret_cast<const double2*>(X + (int64_t)c * KP);
#pragma unroll
            for (int t = 0; t < KP / 2; ++t) {
              const double2 x = xr[t];
              acc[2 * t] = fma(v, x.x, acc[2 * t]);
              acc[2 * t + 1] = fma(v, x.y, acc[2 * t + 1]);
            }
          }
        } else {
          for (int e = rp[local] + sub; e < e1; e += LPR) {
            const int c = cl[e];
            const double v = vl[e];
            const double* xr = X + (int64_t)c * KP;
#pragma unroll
            for (int t = 0; t < KP; ++t) acc[t] = fma(v, xr[t], acc[t]);
          }
        }
      } else {
        for (int e = rp[local] + sub; e < e1; e += LPR) {
          const int c = cl[e];
          const double v = vl[e];
          const double* xr = X + (int64_t)c * KP;
#pragma unroll
          for (int t = 0; t < KP; ++t) acc[t] = fma(v, xr[t], acc[t]);
        }
      }
    }
  }
#pragma unroll
  for (int o = 1; o < LPR; o <<= 1)
#pragma unroll
    for (int t = 0; t < KP; ++t) acc[t] += __shfl_xor(acc[t], o, 64);
  if (!valid) return;
  if (a.which == 1 && pk == 3) {  // P = diag(q) P_1: scale the row of P_1 X
    const double qs = d.prs[local];
#pragma unroll
    for (int t = 0; t < KP; ++t) acc[t] *= qs;
  }
  const int64_t ro = (int64_t)local * KP;
  if constexpr (CONV && LPR == 1 && KP % 2 == 0) {
    // one lane owns the row: both outputs leave as 16-byte stores
    double xr[KP], vo[KP], yo[KP];
#pragma unroll
    for (int u = 0; u < KP; ++u) xr[u] = X[ro + u];
#pragma unroll
    for (int t = 0; t < KP; ++t) {
      double y = 0.0, v = 0.0;
#pragma unroll
      for (int u = 0; u <= t; ++u) {
        y = fma(acc[u], sM[u * KP + t], y);
        v = fma(xr[u], sM[u * KP + t], v);
      }
      vo[t] = v;
      double o = alpha * y;
      if (beta != 0.0) o = fma(beta, Bsrc[base + ro + t], o);
      yo[t] = o;
    }
    double2* vd = reinterpret_cast<double2*>(a.Vout + base + ro);
    double2* yd = reinterpret_cast<double2*>(Y + ro);
#pragma unroll
    for (int t = 0; t < KP / 2; ++t) {
      vd[t] = make_double2(vo[2 * t], vo[2 * t + 1]);
      yd[t] = make_double2(yo[2 * t], yo[2 * t + 1]);
    }
  } else if constexpr (CONV) {
    double xr[KP];
#pragma unroll
    for (int u = 0; u < KP; ++u) xr[u] = X[ro + u];
#pragma unroll
    for (int t = 0; t < KP; ++t) {
      if ((t % LPR) == sub) {
        double y = 0.0, v = 0.0;
#pragma unroll
        for (int u = 0; u <= t; ++u) {
          y = fma(acc[u], sM[u * KP + t], y);
          v = fma(xr[u], sM[u * KP + t], v);
        }
        a.Vout[base + ro + t] = v;
        double o = alpha * y;
        if (beta != 0.0) o = fma(beta, Bsrc[base + ro + t], o);
        Y[ro + t] = o;
      }
    }
  } else if constexpr (LPR == 1 && KP % 2 == 0) {
    double yo[KP];
#pragma unroll
    for (int t = 0; t < KP; ++t) {
      double o = alpha * acc[t];
      if (beta != 0.0) o = fma(beta, Bsrc[base + ro + t], o);
      yo[t] = o;
    }
    double2* yd = reinterpret_cast<double2*>(Y + ro);
#pragma unroll
    for (int t = 0; t < KP / 2; ++t) yd[t] = make_double2(yo[2 * t], yo[2 * t + 1]);
  } else {
#pragma unroll
    for (int t = 0; t < KP; ++t) {
      if ((t % LPR) == sub) {
        double o = alpha * acc[t];
        if (beta != 0.0) o = fma(beta, Bsrc[base + ro + t], o);
        Y[ro + t] = o;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Column-split SpMM over the segments of a batch: the operands and result of
// k_spmm_seg, bit for bit its one-lane-per-row sums (every column adds the
// row's entries in order).  L = KP / 2 lanes share a row and lane sub owns its
// column pair (2 sub, 2 sub + 1), so the X row an entry gathers is one
// contiguous 16 L-byte access of the group instead of KP / 2 accesses of one
// lane; the group's column and value loads take L different entries (R rounds
// per batch) and are passed round by shuffles.  kp = 1: one lane, one column.
// ---------------------------------------------------------------------------
typedef double dbl2 __attribute__((ext_vector_type(2)));  // 16-byte nontemporal stores

template <int KP>
struct CsShape {
  static constexpr int L = KP >= 2 ? KP / 2 : 1;  // lanes per row
  static constexpr int C = KP >= 2 ? 2 : 1;       // columns per lane
  static constexpr int R = KP <= 2 ? 8 : (KP == 4 ? 4 : (KP == 8 ? 2 : 1));  // rounds per batch
};

template <int KP, bool CONV>
__global__ __launch_bounds__(sp_rows<KP>() * CsShape<KP>::L) void k_spmm_cs(SpArgs a) {
  constexpr int L = CsShape<KP>::L, C = CsShape<KP>::C, R = CsShape<KP>::R, EB = L * R;
  const int lg = a.linear ? (int)blockIdx.x : xcd_swizzle(blockIdx.x, gridDim.x);
  const int s = a.stab[lg];
  if (s < 0) return;
  if (a.check_done && a.st[s].done) return;
  const SegDesc& d = a.seg[s];
  const int pk = d.pkind;
  const int32_t *rp, *cl, *sp, *sw, *sc;
  const double *vl, *sv;
  bool ident = false;
  double* Y = a.Y;
  double alpha = a.alpha, beta = a.beta;
  const double* Bsrc = a.Bsrc;
  if (a.which == 0) {
    rp = d.arow; cl = d.acol; vl = d.aval;
    sp = d.a_sp; sw = d.a_sw; sc = d.a_sc; sv = d.a_sv;
  } else if (a.which == 1) {
    ident = (pk == 0);
    rp = d.prow; cl = d.pcol; vl = d.pval;
    sp = d.p_sp; sw = d.p_sw; sc = d.p_sc; sv = d.p_sv;
    if (pk == 2) { Y = a.Yalt; alpha = 1.0; beta = 0.0; Bsrc = nullptr; }
  } else {
    if (pk != 2) return;
    rp = d.prow; cl = d.pcol; vl = d.qval;
    sp = d.p_sp; sw = d.p_sw; sc = d.p_sc; sv = d.q_sv;
  }
  __shared__ double sM[CONV ? KP * KP : 1];
  if constexpr (CONV) {
    for (int t = threadIdx.x; t < KP * KP; t += blockDim.x) sM[t] = a.st[s].R2inv[t];
    __syncthreads();
  }
  const int64_t base = d.r0 * KP;
  const double* X = a.X + base;
  Y += base;
  const int local = (lg - d.sp0) * sp_rows<KP>() + (int)threadIdx.x / L;
  const int sub = (int)threadIdx.x % L;
  const int g0 = ((int)threadIdx.x & 63) - sub;  // first lane of the row's group
  // every lane of a group shares `local`, so groups are wholly valid or not
  if (local >= d.n) return;
  const int64_t ro = (int64_t)local * KP + C * sub;  // this lane's first column
  double acc[C];
#pragma unroll
  for (int q = 0; q < C; ++q) acc[q] = 0.0;
  // one batch: entry j of the group's EB came from lane g0 + j % L, round j / L
  auto batch = [&](const int (&cm)[R], const double (&vm)[R]) {
    int c[EB];
    double v[EB];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int t = 0; t < L; ++t) {
        c[r * L + t] = L > 1 ? __shfl(cm[r], g0 + t, 64) : cm[r];
        v[r * L + t] = L > 1 ? __shfl(vm[r], g0 + t, 64) : vm[r];
      }
    if constexpr (C == 2) {
      const double2* X2 = reinterpret_cast<const double2*>(X);
      double2 x[EB];
#pragma unroll
      for (int j = 0; j < EB; ++j) x[j] = c[j] >= 0 ? X2[(int64_t)c[j] * L + sub] : make_double2(0.0, 0.0);
#pragma unroll
      for (int j = 0; j < EB; ++j) {
        acc[0] = fma(v[j], x[j].x, acc[0]);
        acc[1] = fma(v[j], x[j].y, acc[1]);
      }
    } else {
      double x[EB];
#pragma unroll
      for (int j = 0; j < EB; ++j) x[j] = c[j] >= 0 ? X[c[j]] : 0.0;
#pragma unroll
      for (int j = 0; j < EB; ++j) acc[0] = fma(v[j], x[j], acc[0]);
    }
  };
  if (ident) {
#pragma unroll
    for (int q = 0; q < C; ++q) acc[q] = X[ro + q];
  } else if (sp) {
    // sliced ELL (64-row slices, padded slots hold column -1)
    const int64_t sb = sp[local >> 6] + (local & 63);
    const int w = sw[local >> 6];
    const bool own = !(a.which == 1 && (pk == 2 || pk == 3));
    for (int k0 = 0; k0 < w; k0 += EB) {
      int cm[R];
      double vm[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int k = k0 + r * L + sub;
        const int64_t q = sb + (int64_t)k * 64;
        cm[r] = -1;
        vm[r] = 0.0;
        if (k < w) {
          cm[r] = sc[q];
          vm[r] = own ? __builtin_nontemporal_load(sv + q) : sv[q];
        }
      }
      batch(cm, vm);
    }
  } else {
    const int e0 = rp[local], e1 = rp[local + 1];
    for (int k0 = e0; k0 < e1; k0 += EB) {
      int cm[R];
      double vm[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int e = k0 + r * L + sub;
        cm[r] = -1;
        vm[r] = 0.0;
        if (e < e1) {
          cm[r] = cl[e];
          vm[r] = vl[e];
        }
      }
      batch(cm, vm);
    }
  }
  if (a.which == 1 && pk == 3) {  // P = diag(q) P_1: scale the row of P_1 X
    const double qs = d.prs[local];
#pragma unroll
    for (int q = 0; q < C; ++q) acc[q] *= qs;
  }
  double o[C];
  if constexpr (CONV) {
    // the row's KP values of Op W1 and of W1 from the group, then this lane's
    // columns of (Op W1) M and W1 M (M upper triangular)
    double xr[C];
#pragma unroll
    for (int q = 0; q < C; ++q) xr[q] = X[ro + q];
    double fa[KP], fx[KP];
#pragma unroll
    for (int u = 0; u < KP; ++u) {
      fa[u] = L > 1 ? __shfl(acc[u % C], g0 + u / C, 64) : acc[u % C];
      fx[u] = L > 1 ? __shfl(xr[u % C], g0 + u / C, 64) : xr[u % C];
    }
    double vo[C];
#pragma unroll
    for (int q = 0; q < C; ++q) {
      const int t = C * sub + q;
      double y = 0.0, v = 0.0;
#pragma unroll
      for (int u = 0; u < KP; ++u)
        if (u <= t) {
          y = fma(fa[u], sM[u * KP + t], y);
          v = fma(fx[u], sM[u * KP + t], v);
        }
      vo[q] = v;
      o[q] = alpha * y;
      if (beta != 0.0) o[q] = fma(beta, Bsrc[base + ro + q], o[q]);
    }
    if constexpr (C == 2) __builtin_nontemporal_store(dbl2{vo[0], vo[1]}, reinterpret_cast<dbl2*>(a.Vout + base + ro));
    else __builtin_nontemporal_store(vo[0], a.Vout + base + ro);
  } else {
#pragma unroll
    for (int q = 0; q < C; ++q) {
      o[q] = alpha * acc[q];
      if (beta != 0.0) o[q] = fma(beta, Bsrc[base + ro + q], o[q]);
    }
  }
  // the outputs stream past the caches (nontemporal), which keeps the gathered X
  // rows of the other workgroups cached (measured: SpMM with A 151 -> 142 us
  // and the next pass 1 265 -> 246 us at C1)
  if constexpr (C == 2) __builtin_nontemporal_store(dbl2{o[0], o[1]}, reinterpret_cast<dbl2*>(Y + ro));
  else __builtin_nontemporal_store(o[0], Y + ro);
}

// ---------------------------------------------------------------------------
// single-matrix CSR SpMM with caller leading dimensions (pmor_spmm):
// Y = alpha A X + beta Bsrc, LPR lanes per row
// ---------------------------------------------------------------------------
template <int KP, int LPR>
__global__ __launch_bounds__(256) void k_spmm(int n, const int32_t* __restrict__ rowptr,
                                              const int32_t* __restrict__ col, const double* __restrict__ val,
                                              const double* __restrict__ X, int64_t ldx, double* Y, int64_t ldy,
                                              double alpha, double beta, const double* Bsrc, int64_t ldb) {
  const int64_t gid = (int64_t)xcd_swizzle(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int64_t row = gid / LPR;
  const int sub = (int)(gid % LPR);
  const bool valid = row < n;
  double acc[KP];
#pragma unroll
  for (int t = 0; t < KP; ++t) acc[t] = 0.0;
  if (valid) {
    const int e1 = rowptr[row + 1];
    for (int e = rowptr[row] + sub; e < e1; e += LPR) {
      const int c = col[e];
      const double v = val[e];
      const double* xr = X + (int64_t)c * ldx;
#pragma unroll
      for (int t = 0; t < KP; ++t) acc[t] = fma(v, xr[t], acc[t]);
    }
  }
#pragma unroll
  for (int o = 1; o < LPR; o <<= 1)
#pragma unroll
    for (int t = 0; t < KP; ++t) acc[t] += __shfl_xor(acc[t], o, 64);
  if (!valid) return;
#pragma unroll
  for (int t = 0; t < KP; ++t) {
    if ((t % LPR) == sub) {
      double y = alpha * acc[t];
      if (beta != 0.0) y = fma(beta, Bsrc[row * ldb + t], y);
      Y[row * ldy + t] = y;
    }
  }
}

// lanes per row of the CSR SpMM (1, 2, 4 or 8; 2 measured best for 7-point rows
// at k = 1..8); PMOR_SPMM_LPR overrides the default (16: the engine's column
// split, and 2 lanes for the single-matrix SpMM)
static int spmm_lanes_per_row() {
  static int lpr = [] {
    const char* e = getenv("PMOR_SPMM_LPR");
    const int v = e ? atoi(e) : 2;
    return spmm_variant_ok(v) ? v : 2;
  }();
  return lpr;
}

// SpMM variant tuning for the batched engine.  One value per (block width,
// operator: A or the preconditioner), fixed for the process once chosen, so a
// system's result never depends on the batch it runs in.  The tuner chooses
// only between variants that add a row's entries in the same order (one lane
// per row and the column split), so its choice never changes a result bit;
// 2, 4 and 8 lanes per row split a row's sum and give other roundings, and run
// only when PMOR_SPMM_LPR pins them.  Without the pin the first batch that
// needs a value times the two candidates on its own matrices and keeps the
// faster.  PMOR_TUNE_CACHE names a JSON file of the choices: read before
// tuning (entries other than 1 and the column split are ignored), rewritten
// after it.
namespace tune {
static std::mutex mu;
static std::map<std::string, int> table;
static bool loaded = false;

static std::string key(int kp, int which) {
  return std::string(which == 0 ? "spmm_lanes_A_kp" : "spmm_lanes_P_kp") + std::to_string(kp);
}

// the cache is a flat JSON object of "name": integer pairs
static void load_locked() {
  if (loaded) return;
  loaded = true;
  const char* f = getenv("PMOR_TUNE_CACHE");
  if (!f) return;
  FILE* fp = fopen(f, "r");
  if (!fp) return;
  std::string txt;
  char buf[4096];
  size_t got;
  while ((got = fread(buf, 1, sizeof(buf), fp)) > 0) txt.append(buf, got);
  fclose(fp);
  size_t i = 0;
  while ((i = txt.find('"', i)) != std::string::npos) {
    const size_t j = txt.find('"', i + 1);
    if (j == std::string::npos) break;
    const std::string name = txt.substr(i + 1, j - i - 1);
    size_t c = txt.find(':', j);
    if (c == std::string::npos) break;
    const int v = atoi(txt.c_str() + c + 1);
    if (v == 1 || v == SPMM_COLSPLIT) table[name] = v;
    i = c + 1;
  }
}

static void save_locked() {
  const char* f = getenv("PMOR_TUNE_CACHE");
  if (!f) return;
  FILE* fp = fopen(f, "w");
  if (!fp) return;
  fprintf(fp, "{");
  bool first = true;
  for (const auto& kv : table) {
    fprintf(fp, "%s\n  \"%s\": %d", first ? "" : ",", kv.first.c_str(), kv.second);
    first = false;
  }
  fprintf(fp, "\n}\n");
  fclose(fp);
}

// the chosen value, or 0 when it still has to be measured
static int get(int kp, int which) {
  if (getenv("PMOR_SPMM_LPR")) return spmm_lanes_per_row();
  std::lock_guard<std::mutex> g(mu);
  load_locked();
  auto it = table.find(key(kp, which));
  return it == table.end() ? 0 : it->second;
}

// first writer wins, so every batch of the process sees one value
static int put(int kp, int which, int v) {
  std::lock_guard<std::mutex> g(mu);
  auto it = table.find(key(kp, which));
  if (it != table.end()) return it->second;
  table[key(kp, which)] = v;
  save_locked();
  return v;
}
}  // namespace tune

template <int LPR>
static int launch_spmm_lpr(int n, const int32_t* rowptr, const int32_t* col, const double* val, const double* X,
                           int64_t ldx, double* Y, int64_t ldy, int k, double alpha, double beta, const double* Bsrc,
                           int64_t ldb, hipStream_t stream, pmor_ctx* pc, int pidx, int ppart) {
  const int64_t threads = (int64_t)n * LPR;
  const unsigned grid = (unsigned)((threads + 255) / 256);
  switch (k) {
#define SPMM_CASE(K) \
    case K: plaunch(pc, pidx, ppart, k_spmm<K, LPR>, dim3(grid), dim3(256), 0, stream, n, rowptr, col, val, X, ldx, \
                    Y, ldy, alpha, beta, Bsrc, ldb); break;
    SPMM_CASE(1) SPMM_CASE(2) SPMM_CASE(3) SPMM_CASE(4) SPMM_CASE(5) SPMM_CASE(6) SPMM_CASE(7) SPMM_CASE(8)
    SPMM_CASE(9) SPMM_CASE(10) SPMM_CASE(11) SPMM_CASE(12) SPMM_CASE(13) SPMM_CASE(14) SPMM_CASE(15) SPMM_CASE(16)
#undef SPMM_CASE
    default: return fail(PMOR_EINVAL, "spmm: k out of range");
  }
  PMOR_HIP(hipGetLastError());
  return PMOR_OK;
}

int launch_spmm(int n, const int32_t* rowptr, const int32_t* col, const double* val, const double* X, int64_t ldx,
                double* Y, int64_t ldy, int k, double alpha, double beta, const double* Bsrc, int64_t ldb,
                hipStream_t stream, pmor_ctx* pc, int pidx, int ppart) {
  if (n == 0) return PMOR_OK;
  switch (spmm_lanes_per_row()) {
    case 1: return launch_spmm_lpr<1>(n, rowptr, col, val, X, ldx, Y, ldy, k, alpha, beta, Bsrc, ldb, stream, pc, pidx,
                                      ppart);
    case 4: return launch_spmm_lpr<4>(n, rowptr, col, val, X, ldx, Y, ldy, k, alpha, beta, Bsrc, ldb, stream, pc, pidx,
                                      ppart);
    case 8: return launch_spmm_lpr<8>(n, rowptr, col, val, X, ldx, Y, ldy, k, alpha, beta, Bsrc, ldb, stream, pc, pidx,
                                      ppart);
    default: return launch_spmm_lpr<2>(n, rowptr, col, val, X, ldx, Y, ldy, k, alpha, beta, Bsrc, ldb, stream, pc,
                                       pidx, ppart);
  }
}

// ---------------------------------------------------------------------------
// column norms, gather/scatter of the compacted right-hand sides
// ---------------------------------------------------------------------------
// squared column norms of the segment's W (row kernel grid, 256 threads)
template <int KP>
__global__ __launch_bounds__(256) void k_colnorm_seg(KArgs a) {
  RowSeg r;
  if (!row_seg(a, false, r)) return;
  const double* W = a.W + r.r0 * KP;
  __shared__ double sw[4][KP];
  double acc[KP];
#pragma unroll
  for (int c = 0; c < KP; ++c) acc[c] = 0.0;
  for (int row = r.g * 256 + (int)threadIdx.x; row < r.n; row += r.G * 256) {
#pragma unroll
    for (int c = 0; c < KP; ++c) {
      const double x = W[(int64_t)row * KP + c];
      acc[c] += x * x;
    }
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < KP; ++c) {
    const double sum = wave_sum(acc[c]);
    if (lane == 0) sw[w][c] = sum;
  }
  __syncthreads();
  if (threadIdx.x < KP)
    a.part[(int64_t)r.lg * a.lstride + threadIdx.x] =
        (sw[0][threadIdx.x] + sw[1][threadIdx.x]) + (sw[2][threadIdx.x] + sw[3][threadIdx.x]);
}

// squared column norms of the caller's B of every listed segment: workgroup
// (x, y) writes partials part[(y gridDim.x + x) KMAX + c]
__global__ __launch_bounds__(256) void k_bnorm(const SegDesc* seg, const int* slist, double* part) {
  const SegDesc& d = seg[slist[blockIdx.y]];
  __shared__ double sw[4][KMAX];
  double acc[KMAX];
#pragma unroll
  for (int c = 0; c < KMAX; ++c) acc[c] = 0.0;
  for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < d.n; row += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int c = 0; c < KMAX; ++c)
      if (c < d.k) {
        const double x = d.B[row * d.ldb + c];
        acc[c] += x * x;
      }
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < KMAX; ++c) {
    const double sum = wave_sum(acc[c]);
    if (lane == 0) sw[w][c] = sum;
  }
  __syncthreads();
  if (threadIdx.x < KMAX)
    part[((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * KMAX + threadIdx.x] =
        (sw[0][threadIdx.x] + sw[1][threadIdx.x]) + (sw[2][threadIdx.x] + sw[3][threadIdx.x]);
}

// Bc = W = compacted B, Xc = 0 for every listed segment
__global__ __launch_bounds__(256) void k_gather_seg(const SegDesc* seg, const int* slist, int kp, double* Bc,
                                                    double* W, double* Xc) {
  const SegDesc& d = seg[slist[blockIdx.y]];
  const int64_t len = (int64_t)d.n * kp;
  const int64_t base = d.r0 * kp;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < len; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = t / kp;
    const int c = (int)(t % kp);
    const double b = (c < d.kact) ? d.B[row * d.ldb + d.cmap[c]] : 0.0;
    Bc[base + t] = b;
    W[base + t] = b;
    Xc[base + t] = 0.0;
  }
}

// caller's X from the compacted solution (columns without a compacted slot get 0)
__global__ __launch_bounds__(256) void k_scatter_seg(const SegDesc* seg, const int* slist, int kp, const double* Xc) {
  const SegDesc& d = seg[slist[blockIdx.y]];
  const int64_t len = (int64_t)d.n * d.k;
  const int64_t base = d.r0 * kp;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < len; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = t / d.k;
    const int c = (int)(t % d.k);
    const int ci = d.cinv[c];
    d.X[row * d.ldx + c] = (ci >= 0) ? Xc[base + row * kp + ci] : 0.0;
  }
}

// ---------------------------------------------------------------------------
// host side: engine buffers
// ---------------------------------------------------------------------------
struct DBuf {
  double* p = nullptr;
  int64_t cap = 0;
};

struct Engine {
  DBuf V, W, Z, T, Bc, Xc, Hc, Hbar, G, refl, Y, nrm, part, partg;
  DevState* st = nullptr;
  int64_t st_cap = 0;
  SegDesc* seg_d = nullptr;
  SegDesc* seg_h = nullptr;   // pinned staging
  int64_t seg_cap = 0, seg_h_cap = 0;
  int* tab_d = nullptr;
  int* tab_h = nullptr;       // pinned staging
  int64_t tab_cap = 0, tab_h_cap = 0;
  int* hinfo_h = nullptr;     // host-mapped, 4 ints per segment
  int* hinfo_d = nullptr;
  int64_t hinfo_cap = 0;
  double* nrm_h = nullptr;    // pinned, KMAX per segment
  int64_t nrm_h_cap = 0;
  // strides of the per-segment arrays for the current (kp, m)
  int ldh = 0;
  int64_t hcs = 0, hc2off = 0, hbs = 0, gs = 0, rfs = 0, ys = 0, lstride = 0;
  int64_t bytes = 0;  // device bytes held
};

static int grow(DBuf& b, int64_t need) {
  need = std::max<int64_t>(need, 1);
  if (need <= b.cap) return PMOR_OK;
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.cap = 0;
  if (hipMalloc((void**)&b.p, sizeof(double) * need) != hipSuccess) {
    b.p = nullptr;
    (void)hipGetLastError();
    return fail(PMOR_ENOMEM, "device allocation of the Krylov workspace failed");
  }
  b.cap = need;
  return PMOR_OK;
}

template <typename Tp>
static int grow_host(Tp** p, int64_t& cap, int64_t need, unsigned flags) {
  need = std::max<int64_t>(need, 1);
  if (need <= cap) return PMOR_OK;
  if (*p) (void)hipHostFree(*p);
  *p = nullptr;
  cap = 0;
  if (hipHostMalloc((void**)p, sizeof(Tp) * need, flags) != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(PMOR_ENOMEM, "pinned host allocation failed");
  }
  std::memset(*p, 0, sizeof(Tp) * need);
  cap = need;
  return PMOR_OK;
}

template <typename Tp>
static int grow_dev(Tp** p, int64_t& cap, int64_t need) {
  need = std::max<int64_t>(need, 1);
  if (need <= cap) return PMOR_OK;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  cap = 0;
  if (hipMalloc((void**)p, sizeof(Tp) * need) != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(PMOR_ENOMEM, "device allocation of the Krylov state failed");
  }
  cap = need;
  return PMOR_OK;
}

void engine_destroy(Engine* e) {
  if (!e) return;
  DBuf* bufs[] = {&e->V, &e->W, &e->Z, &e->T, &e->Bc, &e->Xc, &e->Hc, &e->Hbar, &e->G, &e->refl, &e->Y,
                  &e->nrm, &e->part, &e->partg};
  for (DBuf* b : bufs)
    if (b->p) (void)hipFree(b->p);
  if (e->st) (void)hipFree(e->st);
  if (e->seg_d) (void)hipFree(e->seg_d);
  if (e->tab_d) (void)hipFree(e->tab_d);
  if (e->seg_h) (void)hipHostFree(e->seg_h);
  if (e->tab_h) (void)hipHostFree(e->tab_h);
  if (e->hinfo_h) (void)hipHostFree(e->hinfo_h);
  if (e->nrm_h) (void)hipHostFree(e->nrm_h);
  delete e;
}

// buffers for nseg segments over `rows` concatenated rows, `wgs` row-kernel
// workgroups and `tabints` table entries
static int engine_reserve(Engine& E, int kp, int m, int64_t rows, int nseg, int64_t wgs, int64_t tabints) {
  const int64_t kp2 = (int64_t)kp * kp;
  E.ldh = (m + 1) * kp;
  E.hc2off = (m + 2) * kp2 + KMAX;
  E.hcs = 2 * E.hc2off;
  E.hbs = (int64_t)E.ldh * m * kp;
  E.gs = (int64_t)E.ldh * kp;
  E.rfs = (int64_t)(m + 1) * kp * (kp + 2);
  E.ys = (int64_t)E.ldh * kp;
  E.lstride = (m + 1) * kp2 + KMAX;
  const int64_t blk = rows * kp;
  PMOR_TRY(grow(E.V, (m + 1) * blk));
  PMOR_TRY(grow(E.W, blk));
  PMOR_TRY(grow(E.Z, blk));
  PMOR_TRY(grow(E.T, blk));
  PMOR_TRY(grow(E.Bc, blk));
  PMOR_TRY(grow(E.Xc, blk));
  PMOR_TRY(grow(E.Hc, nseg * E.hcs));
  PMOR_TRY(grow(E.Hbar, nseg * E.hbs));
  PMOR_TRY(grow(E.G, nseg * E.gs));
  PMOR_TRY(grow(E.refl, nseg * E.rfs));
  PMOR_TRY(grow(E.Y, nseg * E.ys));
  PMOR_TRY(grow(E.nrm, (int64_t)nseg * KMAX));
  PMOR_TRY(grow(E.part, std::max<int64_t>(wgs * E.lstride, (int64_t)nseg * 64 * KMAX)));
  PMOR_TRY(grow(E.partg, wgs * kp2));
  PMOR_TRY(grow_dev(&E.st, E.st_cap, nseg));
  PMOR_TRY(grow_dev(&E.seg_d, E.seg_cap, nseg));
  PMOR_TRY(grow_dev(&E.tab_d, E.tab_cap, tabints));
  PMOR_TRY(grow_host(&E.seg_h, E.seg_h_cap, nseg, hipHostMallocDefault));
  PMOR_TRY(grow_host(&E.tab_h, E.tab_h_cap, tabints, hipHostMallocDefault));
  if ((int64_t)4 * nseg > E.hinfo_cap) {
    PMOR_TRY(grow_host(&E.hinfo_h, E.hinfo_cap, (int64_t)4 * nseg, hipHostMallocMapped));
    PMOR_HIP(hipHostGetDevicePointer((void**)&E.hinfo_d, E.hinfo_h, 0));
  }
  PMOR_TRY(grow_host(&E.nrm_h, E.nrm_h_cap, (int64_t)nseg * KMAX, hipHostMallocDefault));
  int64_t b = 0;
  for (const DBuf* d : {&E.V, &E.W, &E.Z, &E.T, &E.Bc, &E.Xc, &E.Hc, &E.Hbar, &E.G, &E.refl, &E.Y, &E.nrm, &E.part,
                        &E.partg})
    b += 8 * d->cap;
  E.bytes = b + (int64_t)sizeof(DevState) * E.st_cap + (int64_t)sizeof(SegDesc) * E.seg_cap + 4 * E.tab_cap;
  return PMOR_OK;
}

// ---------------------------------------------------------------------------
// host side: launch configuration per block size
// ---------------------------------------------------------------------------
template <int KP>
struct Fam {
  static constexpr bool RS = (KP == 4);   // rows split over wavefronts
  static constexpr bool ROW = (KP < 4);   // one row per lane
  static constexpr int NW = (KP == 4 || KP == 16) ? 8 : 4;
  static constexpr int BPW = 32 / NW;     // V blocks per wavefront: m + 1 <= 32
  static constexpr int ROWS = RS ? 16 * NW : (ROW ? 64 : 16);  // rows per workgroup iteration
  static constexpr int GMAX = ROW ? 512 : 128;  // kp >= 4: 128 (long streams per wavefront, few partial rows)
};

static int pad_kp(int k) {
  if (k <= 1) return 1;
  if (k <= 2) return 2;
  if (k <= 4) return 4;
  if (k <= 8) return 8;
  return 16;
}

// row-kernel workgroups of an n-row segment: at least two iterations each,
// at most GMAX, a multiple of 8 from 8 on; a function of n and kp only, so a
// segment's sums do not depend on the batch it runs in
static int row_wgs(int n, int rows_per_iter, int gmax) {
  int64_t g = ((int64_t)n + 2 * rows_per_iter - 1) / (2 * rows_per_iter);
  g = std::min<int64_t>(std::max<int64_t>(g, 1), gmax);
  if (g >= 8) g &= ~7;
  return (int)g;
}

// V blocks held in registers by the kp = 4 kernels: the smallest multiple of 4
// that covers the sweep (fewer registers, more wavefronts in flight)
static int rs_nb(int nbl_max) { return std::min(32, std::max(4, (nbl_max + 3) / 4 * 4)); }

// V blocks per wavefront of the kp = 1, 2, 8, 16 kernels, which take block
// i = w + NW bi: the fewest instantiated counts (1..4 for 8 wavefronts, 2, 4,
// 6, 8 for 4) that cover the sweep's nbl_max <= NW BPW blocks.  A smaller count
// holds fewer registers (more wavefronts in flight) and leaves every sum as it
// is: each wavefront still takes its blocks in the same order.
template <int NW, typename Fn>
static void with_bpw(int nbl_max, Fn&& fn) {
  const int need = (nbl_max + NW - 1) / NW;
  if constexpr (NW == 8) {
    switch (need) {
      case 0: case 1: fn(std::integral_constant<int, 1>{}); break;
      case 2: fn(std::integral_constant<int, 2>{}); break;
      case 3: fn(std::integral_constant<int, 3>{}); break;
      default: fn(std::integral_constant<int, 4>{}); break;
    }
  } else {
    static_assert(NW == 4, "4 or 8 wavefronts");
    switch (need) {
      case 0: case 1: case 2: fn(std::integral_constant<int, 2>{}); break;
      case 3: case 4: fn(std::integral_constant<int, 4>{}); break;
      case 5: case 6: fn(std::integral_constant<int, 6>{}); break;
      default: fn(std::integral_constant<int, 8>{}); break;
    }
  }
}

template <typename Fn>
static void with_nb(int nb, Fn&& fn) {
  switch (nb) {
    case 4: fn(std::integral_constant<int, 4>{}); break;
    case 8: fn(std::integral_constant<int, 8>{}); break;
    case 12: fn(std::integral_constant<int, 12>{}); break;
    case 16: fn(std::integral_constant<int, 16>{}); break;
    case 20: fn(std::integral_constant<int, 20>{}); break;
    case 24: fn(std::integral_constant<int, 24>{}); break;
    case 28: fn(std::integral_constant<int, 28>{}); break;
    default: fn(std::integral_constant<int, 32>{}); break;
  }
}

template <int KP>
static void launch_dot(pmor_ctx* c, int pidx, unsigned grid, hipStream_t s, const KArgs& a, int nbl_max) {
  using F = Fam<KP>;
  if constexpr (F::RS) {
    with_nb(rs_nb(nbl_max), [&](auto nb) {
      plaunch(c, pidx, 3, k_dot4<F::NW, decltype(nb)::value>, dim3(grid), dim3(64 * F::NW), 0, s, a);
    });
  }
  else
    with_bpw<F::NW>(nbl_max, [&](auto b) {
      constexpr int B = decltype(b)::value;
      if constexpr (F::ROW) plaunch(c, pidx, 3, k_dot_row<KP, F::NW, B>, dim3(grid), dim3(64 * F::NW), 0, s, a);
      else plaunch(c, pidx, 3, k_dot_mfma<KP, F::NW, B>, dim3(grid), dim3(64 * F::NW), 0, s, a);
    });
}

template <int KP>
static size_t upd_shm(int nbl_max) {
  using F = Fam<KP>;
  if constexpr (F::RS) return 0;
  const int per = F::ROW ? KP : KP / 4;
  return sizeof(double) * ((size_t)nbl_max * KP * KP + (size_t)2 * F::NW * 64 * per);
}

// the update kernels that can need more than 64 KiB of dynamic LDS (kp != 4)
template <int KP, int MODE>
static int allow_upd_lds(int m) {
  using F = Fam<KP>;
  int rc = PMOR_OK;
  if constexpr (!F::RS)
    for (int nb = 0; nb <= F::NW * F::BPW; nb += F::NW)
      with_bpw<F::NW>(nb, [&](auto b) {
        constexpr int B = decltype(b)::value;
        const void* fn;
        if constexpr (F::ROW) fn = (const void*)k_upd_row<KP, F::NW, B, MODE>;
        else fn = (const void*)k_upd_mfma<KP, F::NW, B, MODE>;
        if (rc == PMOR_OK) rc = allow_lds(fn, upd_shm<KP>(m));
      });
  return rc;
}

template <int KP, int MODE>
static void launch_upd(pmor_ctx* c, int pidx, unsigned grid, hipStream_t s, const KArgs& a, int nbl_max) {
  using F = Fam<KP>;
  const uint32_t shm = (uint32_t)upd_shm<KP>(nbl_max);
  if constexpr (F::RS) {
    with_nb(rs_nb(nbl_max), [&](auto nb) {
      plaunch(c, pidx, 3, k_upd4<F::NW, MODE, decltype(nb)::value>, dim3(grid), dim3(64 * F::NW), 0, s, a);
    });
  } else
    with_bpw<F::NW>(nbl_max, [&](auto b) {
      constexpr int B = decltype(b)::value;
      if constexpr (F::ROW) plaunch(c, pidx, 3, k_upd_row<KP, F::NW, B, MODE>, dim3(grid), dim3(64 * F::NW), shm, s, a);
      else plaunch(c, pidx, 3, k_upd_mfma<KP, F::NW, B, MODE>, dim3(grid), dim3(64 * F::NW), shm, s, a);
    });
}

// SpMM launches of at least this many workgroups take them in launch order
constexpr unsigned SPMM_LINEAR_MIN = 16384;

template <int KP, bool CONV>
static void launch_spmm_seg(pmor_ctx* c, int pidx, int part, unsigned grid, int lpr, hipStream_t s,
                            const SpArgs& a0) {
  SpArgs a = a0;
  a.linear = grid >= SPMM_LINEAR_MIN ? 1 : 0;
  constexpr int R = sp_rows<KP>();
  switch (lpr) {
    case SPMM_COLSPLIT:
      plaunch(c, pidx, part, k_spmm_cs<KP, CONV>, dim3(grid), dim3(R * CsShape<KP>::L), 0, s, a);
      break;
    case 1: plaunch(c, pidx, part, k_spmm_seg<KP, 1, CONV>, dim3(grid), dim3(R * 1), 0, s, a); break;
    case 4: plaunch(c, pidx, part, k_spmm_seg<KP, 4, CONV>, dim3(grid), dim3(R * 4), 0, s, a); break;
    case 8: plaunch(c, pidx, part, k_spmm_seg<KP, 8, CONV>, dim3(grid), dim3(R * 8), 0, s, a); break;
    default: plaunch(c, pidx, part, k_spmm_seg<KP, 2, CONV>, dim3(grid), dim3(R * 2), 0, s, a); break;
  }
}

static unsigned chunks(int64_t len, int64_t per, unsigned cap) {
  const int64_t g = (len + per - 1) / per;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}


// ---------------------------------------------------------------------------
// host side: the persistent engine.  Systems are admitted between cycles into
// free row ranges and segment slots; every cycle advances all admitted systems
// in lockstep; finished systems leave (X written) at the end of a cycle.
// ---------------------------------------------------------------------------
template <int KP>
class RunnerT final : public Runner {
  using F = Fam<KP>;

 public:
  RunnerT(pmor_ctx* c, Engine* e, const pmor_solve_opts& o, int64_t rows_cap, int nslots)
      : ctx_(c), E_(*e), o_(o), rows_cap_((rows_cap + 15) / 16 * 16), nslots_(nslots) {}

  int init() {
    sp_rows_ = sp_rows<KP>();
    const int64_t wg_cap = rows_cap_ / (2 * F::ROWS) + nslots_ + 8;
    const int64_t sp_cap = rows_cap_ / sp_rows_ + nslots_ + 8;
    PMOR_TRY(engine_reserve(E_, KP, o_.m, std::max<int64_t>(rows_cap_, 16), nslots_, wg_cap,
                            wg_cap + sp_cap + 2 * (int64_t)nslots_ + 8));
    item_.assign(nslots_, nullptr);
    r0_.assign(nslots_, 0);
    nrows_.assign(nslots_, 0);
    Gw_.assign(nslots_, 0);
    Gs_.assign(nslots_, 0);
    cyc_.assign(nslots_, 0);
    steps_of_.assign(nslots_, 0);
    for (int s = nslots_ - 1; s >= 0; --s) free_slots_.push_back(s);
    free_rows_.clear();
    free_rows_.push_back({0, rows_cap_});
    const int m = o_.m;
    hess_shm_ = sizeof(double) * ((size_t)KP * E_.ldh + (size_t)(m * KP + KP) * (KP + 2) + 2 * KP * KP);
    ys_pw_ = (KP >= 16) ? 8 : 32;
    ys_shm_ = sizeof(double) * ((size_t)m * KP * KP + (size_t)ys_pw_ * m * KP);
    PMOR_TRY(allow_lds((const void*)k_hess<KP>, hess_shm_));
    PMOR_TRY(allow_lds((const void*)k_ysolve<KP>, ys_shm_));
    PMOR_TRY((allow_upd_lds<KP, UPD_PLAIN>(m)));
    PMOR_TRY((allow_upd_lds<KP, UPD_P2>(m)));
    PMOR_TRY((allow_upd_lds<KP, UPD_P3>(m)));
    t0_ = std::chrono::steady_clock::now();
    return PMOR_OK;
  }

  int busy() const override { return (int)(act_.size() + pending_.size()); }
  double now_ms() const override {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0_).count();
  }

  bool can_admit(SolveItem* const* items, int n) const override {
    if ((int)free_slots_.size() < n) return false;
    std::vector<std::pair<int64_t, int64_t>> fr = free_rows_;
    for (int q = 0; q < n; ++q)
      if (take_rows(fr, rows_of(items[q]->n)) < 0) return false;
    return true;
  }

  int admit(SolveItem* const* items, int n) override {
    if (n <= 0) return PMOR_OK;
    for (int q = 0; q < n; ++q)
      if (items[q]->k > KP || items[q]->k < 1) return fail(PMOR_EINVAL, "system wider than the engine's block");
    if (!can_admit(items, n)) return fail(PMOR_EADMIT, "no free rows or slots in the Krylov engine");
    hipStream_t s = ctx_->stream;
    PMOR_HIP(hipStreamSynchronize(s));
    std::vector<int> ns(n);
    for (int q = 0; q < n; ++q) {
      SolveItem* it = items[q];
      const int sl = free_slots_.back();
      free_slots_.pop_back();
      ns[q] = sl;
      item_[sl] = it;
      nrows_[sl] = rows_of(it->n);
      r0_[sl] = take_rows(free_rows_, nrows_[sl]);
      Gw_[sl] = row_wgs(it->n, F::ROWS, F::GMAX);
      Gs_[sl] = (int)(((int64_t)it->n + sp_rows_ - 1) / sp_rows_);
      cyc_[sl] = 0;
      SegDesc& d = E_.seg_h[sl];
      std::memset(&d, 0, sizeof(d));
      d.n = it->n;
      d.k = it->k;
      d.r0 = r0_[sl];
      d.G = Gw_[sl];
      d.spG = Gs_[sl];
      d.pkind = it->pkind;
      d.arow = it->arow; d.acol = it->acol; d.aval = it->aval;
      d.prow = it->prow; d.pcol = it->pcol; d.pval = it->pval; d.qval = it->qval; d.prs = it->prs;
      if (it->asell && it->asell->cap > 0 && it->aval_s) {
        d.a_sp = it->asell->ptr; d.a_sw = it->asell->wid; d.a_sc = it->asell->col; d.a_sv = it->aval_s;
      }
      if (it->pkind != 0 && it->psell && it->psell->cap > 0 && it->pval_s && (it->pkind != 2 || it->qval_s)) {
        d.p_sp = it->psell->ptr; d.p_sw = it->psell->wid; d.p_sc = it->psell->col; d.p_sv = it->pval_s;
        d.q_sv = it->qval_s;
      }
      d.B = it->B; d.ldb = it->ldb;
      d.X = it->X; d.ldx = it->ldx;
      E_.tab_h[q] = sl;
      it->status = PMOR_OK;
      it->t_done_ms = 0.0;
    }
    // norms of the caller's columns
    PMOR_HIP(hipMemcpyAsync(E_.seg_d, E_.seg_h, sizeof(SegDesc) * nslots_, hipMemcpyHostToDevice, s));
    PMOR_HIP(hipMemcpyAsync(E_.tab_d, E_.tab_h, sizeof(int) * n, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_bnorm, dim3(64, n), dim3(256), 0, s, (const SegDesc*)E_.seg_d, (const int*)E_.tab_d,
                       E_.part.p);
    hipLaunchKernelGGL(k_reduce_seg, dim3((KMAX + 7) / 8, n), dim3(256), 0, s, (const double*)E_.part.p,
                       (int64_t)KMAX, KMAX, (const SegDesc*)E_.seg_d, (const int*)E_.tab_d, 64, (const DevState*)E_.st,
                       0, E_.nrm.p, (int64_t)KMAX, (int64_t)0);
    PMOR_HIP(hipGetLastError());
    PMOR_HIP(hipMemcpyAsync(E_.nrm_h, E_.nrm.p, sizeof(double) * nslots_ * KMAX, hipMemcpyDeviceToHost, s));
    PMOR_HIP(hipStreamSynchronize(s));
    std::vector<int> fresh;
    int64_t maxn = 1;
    for (int q = 0; q < n; ++q) {
      const int sl = ns[q];
      SolveItem* it = item_[sl];
      SegDesc& d = E_.seg_h[sl];
      int kact = 0;
      bool nan = false;
      for (int c = 0; c < KMAX; ++c) { d.cinv[c] = -1; d.cmap[c] = 0; d.bnorm[c] = 1.0; }
      for (int c = 0; c < d.k; ++c) {
        const double b = E_.nrm_h[(int64_t)sl * KMAX + c];
        if (!std::isfinite(b)) { nan = true; continue; }
        if (b > 0.0) {
          d.cinv[c] = kact;
          d.cmap[kact] = c;
          d.bnorm[kact] = std::sqrt(b);
          ++kact;
        }
      }
      if (nan) {
        kact = 0;
        for (int c = 0; c < KMAX; ++c) d.cinv[c] = -1;
      }
      d.kact = kact;
      it->status = nan ? PMOR_ENAN : PMOR_OK;
      if (pmor_stats* st = it->stats) {
        st->k = d.k;
        st->cycles = 0;
        st->steps = 0;
        std::memset(st->cycle_steps, 0, sizeof(st->cycle_steps));
        for (int c = 0; c < PMOR_KMAX; ++c) st->relres[c] = 0.0;
      }
      if (kact > 0) {
        fresh.push_back(sl);
        maxn = std::max<int64_t>(maxn, it->n);
      } else {
        pending_.push_back(sl);  // X = 0, returned by the next cycle
      }
    }
    PMOR_HIP(hipMemcpyAsync(E_.seg_d, E_.seg_h, sizeof(SegDesc) * nslots_, hipMemcpyHostToDevice, s));
    const int nf = (int)fresh.size();
    if (nf > 0) {
      for (int t = 0; t < nf; ++t) E_.tab_h[t] = fresh[t];
      PMOR_HIP(hipMemcpyAsync(E_.tab_d, E_.tab_h, sizeof(int) * nf, hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(k_gather_seg, dim3(chunks(maxn * KP, 256, 2048), nf), dim3(256), 0, s,
                         (const SegDesc*)E_.seg_d, (const int*)E_.tab_d, KP, E_.Bc.p, E_.W.p, E_.Xc.p);
      hipLaunchKernelGGL(k_state_init, dim3(nf), dim3(64), 0, s, (const SegDesc*)E_.seg_d, (const int*)E_.tab_d,
                         E_.st, o_.m, o_.tol);
      PMOR_HIP(hipGetLastError());
      for (int sl : fresh) act_.push_back(sl);
    }
    return PMOR_OK;
  }

  int cycle(std::vector<SolveItem*>& done) override {
    hipStream_t s = ctx_->stream;
    const int m = o_.m;
    // the staging buffers are rewritten only after the copies that read them are done
    PMOR_HIP(hipStreamSynchronize(s));
    std::vector<int> fin;  // slots finished in this call
    const int nact = (int)act_.size();
    int64_t Gtot = 0, SPtot = 0;
    int* sl = E_.tab_h;
    if (nact > 0) {
      int64_t g = 0;
      int* wtab = E_.tab_h;
      for (int i : act_) {
        E_.seg_h[i].wg0 = (int)g;
        for (int q = 0; q < Gw_[i]; ++q) wtab[g++] = i;
      }
      Gtot = (g + 7) / 8 * 8;
      while (g < Gtot) wtab[g++] = -1;
      int* stab = wtab + Gtot;
      int64_t q = 0;
      for (int i : act_) {
        E_.seg_h[i].sp0 = (int)q;
        for (int t = 0; t < Gs_[i]; ++t) stab[q++] = i;
      }
      SPtot = (q + 7) / 8 * 8;
      while (q < SPtot) stab[q++] = -1;
      sl = stab + SPtot;
      bool anyq = false;
      for (int t = 0; t < nact; ++t) {
        sl[t] = act_[t];
        if (item_[act_[t]]->pkind == 2) anyq = true;
      }
      PMOR_HIP(hipMemcpyAsync(E_.seg_d, E_.seg_h, sizeof(SegDesc) * nslots_, hipMemcpyHostToDevice, s));
      PMOR_HIP(hipMemcpyAsync(E_.tab_d, E_.tab_h, sizeof(int) * (Gtot + SPtot + nact), hipMemcpyHostToDevice, s));
      bool anyp = false;
      for (int i : act_) anyp = anyp || item_[i]->pkind != 0;
      PMOR_TRY(resolve_lanes(Gtot, SPtot, anyp));
      PMOR_TRY(run_cycle(Gtot, SPtot, nact, anyq));
      // verdicts
      const double t_now = now_ms();
      std::vector<int> next;
      for (int i : act_) {
        SolveItem* it = item_[i];
        const volatile int* hf = E_.hinfo_h + 4 * i;
        const int j = hf[0], brk = hf[2], nanf = hf[3];
        steps_of_[i] = j;
        const SegDesc& d = E_.seg_h[i];
        bool conv = true, nan = nanf != 0;
        double rel[KMAX];
        for (int c = 0; c < d.kact; ++c) {
          rel[c] = std::sqrt(E_.nrm_h[(int64_t)i * KMAX + c]) / d.bnorm[c];
          if (!(rel[c] <= o_.tol)) conv = false;
          if (!std::isfinite(rel[c])) nan = true;
        }
        const int cyc = cyc_[i]++;
        if (pmor_stats* st = it->stats) {
          if (cyc < PMOR_MAX_CYCLES) st->cycle_steps[cyc] = j;
          st->cycles = cyc + 1;
          st->steps += j;
          for (int c = 0; c < d.k; ++c) st->relres[c] = (d.cinv[c] >= 0) ? rel[d.cinv[c]] : 0.0;
        }
        bool over = true;
        if (nan) it->status = PMOR_ENAN;
        else if (conv) it->status = PMOR_OK;
        else if (brk) it->status = PMOR_EBREAKDOWN;
        else if (cyc_[i] >= o_.max_cycles) it->status = PMOR_ENOTCONV;
        else over = false;
        if (over) {
          it->t_done_ms = t_now;
          fin.push_back(i);
        } else {
          next.push_back(i);
        }
      }
      prof_resolve(ctx_, prof_first_, steps_of_.data());
      act_.swap(next);
    }
    for (int i : pending_) {
      item_[i]->t_done_ms = now_ms();
      fin.push_back(i);
    }
    pending_.clear();
    // X of the finished systems (staging region after this cycle's tables)
    if (!fin.empty()) {
      const int64_t off = Gtot + SPtot + nact;
      int* fl = E_.tab_h + off;
      int64_t maxnk = 1;
      for (size_t t = 0; t < fin.size(); ++t) {
        fl[t] = fin[t];
        maxnk = std::max<int64_t>(maxnk, (int64_t)item_[fin[t]]->n * item_[fin[t]]->k);
      }
      PMOR_HIP(hipMemcpyAsync(E_.tab_d + off, fl, sizeof(int) * fin.size(), hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(k_scatter_seg, dim3(chunks(maxnk, 256, 2048), (unsigned)fin.size()), dim3(256), 0, s,
                         (const SegDesc*)E_.seg_d, (const int*)(E_.tab_d + off), KP, (const double*)E_.Xc.p);
      PMOR_HIP(hipGetLastError());
      PMOR_HIP(hipStreamSynchronize(s));
      for (int i : fin) {
        done.push_back(item_[i]);
        item_[i] = nullptr;
        give_rows(r0_[i], nrows_[i]);
        free_slots_.push_back(i);
      }
    }
    return PMOR_OK;
  }

 private:
  static int64_t rows_of(int n) { return std::max<int64_t>(16, ((int64_t)n + 15) / 16 * 16); }

  // first fit over the free row ranges; -1 when nothing fits
  static int64_t take_rows(std::vector<std::pair<int64_t, int64_t>>& fr, int64_t need) {
    for (size_t t = 0; t < fr.size(); ++t)
      if (fr[t].second >= need) {
        const int64_t at = fr[t].first;
        fr[t].first += need;
        fr[t].second -= need;
        if (fr[t].second == 0) fr.erase(fr.begin() + t);
        return at;
      }
    return -1;
  }

  void give_rows(int64_t at, int64_t len) {
    auto& fr = free_rows_;
    size_t t = 0;
    while (t < fr.size() && fr[t].first < at) ++t;
    fr.insert(fr.begin() + t, {at, len});
    if (t + 1 < fr.size() && fr[t].first + fr[t].second == fr[t + 1].first) {
      fr[t].second += fr[t + 1].second;
      fr.erase(fr.begin() + t + 1);
    }
    if (t > 0 && fr[t - 1].first + fr[t - 1].second == fr[t].first) {
      fr[t - 1].second += fr[t].second;
      fr.erase(fr.begin() + t);
    }
  }

  // SpMM variant (lanes per row, or the column split) for A and the
  // preconditioner: the process-wide choice,
  // measured here on this batch's matrices when none exists yet (the buffers T
  // and Z are free at a cycle boundary)
  int resolve_lanes(int64_t Gtot, int64_t SPtot, bool anyp) {
    for (int which = 0; which < 2; ++which) {
      int& lpr = which == 0 ? lprA_ : lprP_;
      if (lpr != 0 || (which == 1 && !anyp)) continue;
      int v = tune::get(KP, which);
      if (v == 0) {
        hipStream_t s = ctx_->stream;
        SpArgs sp{E_.seg_d, E_.tab_d + Gtot, E_.st, which, 0, E_.W.p, E_.T.p, E_.Z.p, nullptr, 1.0, 0.0, nullptr, 1};
        float best_ms = 3.0e38f;
        v = SPMM_COLSPLIT;
        for (int L : {1, SPMM_COLSPLIT}) {
          for (int r = 0; r < 2; ++r) launch_spmm_seg<KP, false>(nullptr, -1, 3, (unsigned)SPtot, L, s, sp);
          PMOR_HIP(hipEventRecord(ctx_->ev0, s));
          for (int r = 0; r < 3; ++r) launch_spmm_seg<KP, false>(nullptr, -1, 3, (unsigned)SPtot, L, s, sp);
          PMOR_HIP(hipEventRecord(ctx_->ev1, s));
          PMOR_HIP(hipEventSynchronize(ctx_->ev1));
          float ms = 0.f;
          PMOR_HIP(hipEventElapsedTime(&ms, ctx_->ev0, ctx_->ev1));
          if (ms < best_ms) { best_ms = ms; v = L; }
        }
        PMOR_HIP(hipGetLastError());
        v = tune::put(KP, which, v);
      }
      lpr = v;
    }
    return PMOR_OK;
  }

  // one restart cycle of every active segment (tables already uploaded)
  int run_cycle(int64_t Gtot, int64_t SPtot, int nact, bool anyq) {
    hipStream_t s = ctx_->stream;
    const int m = o_.m;
    Engine& E = E_;
    KArgs a{};
    a.m = m;
    a.ldh = E.ldh;
    a.vstride = rows_cap_ * KP;
    a.V = E.V.p; a.W = E.W.p;
    a.seg = E.seg_d;
    a.Hc = E.Hc.p; a.hcs = E.hcs; a.hc2off = E.hc2off;
    a.Hbar = E.Hbar.p; a.hbs = E.hbs;
    a.G = E.G.p; a.gs = E.gs;
    a.refl = E.refl.p; a.rfs = E.rfs;
    a.Y = E.Y.p; a.ys = E.ys;
    a.part = E.part.p; a.lstride = E.lstride;
    a.partg = E.partg.p;
    a.st = E.st;
    a.hinfo = E.hinfo_d;
    a.wtab = E.tab_d;
    // few workgroups stream faster with each XCD on its own contiguous rows, a
    // large batch with the XCDs interleaved workgroup by workgroup (pass-1
    // kernel, 20 systems of 262144 rows: 6.9 against 6.8 TB/s).  Results do
    // not depend on the mapping.
    a.swz = Gtot < 1024 ? 1 : 0;
    a.slist = E.tab_d + Gtot + SPtot;
    const int* stab_d = E.tab_d + Gtot;
    const unsigned gR = (unsigned)Gtot, gS = (unsigned)SPtot;
    const int lprA = lprA_ ? lprA_ : 2, lprP = lprP_ ? lprP_ : 2;
    pmor_ctx* ctx = ctx_;
    Profiler& prof = ctx->prof;
    auto prof_seg = [&](int pr, int tag, auto bytes_of) {
      if (pr < 0) return;
      const int e0 = (int)prof.ent.size();
      for (int i : act_) prof.ent.push_back({i, bytes_of(i)});
      prof_stop_seg(ctx, pr, tag, e0);
    };
    auto blkb = [&](int i) { return 8.0 * (double)item_[i]->n * KP; };
    // distinct bytes: an array shared by several systems of the launch (the
    // pattern of A for the points of one problem, P_1 for the points of one
    // sequence) is counted once, split evenly among the systems that share it
    std::map<const void*, int> share;
    for (int i : act_) {
      ++share[item_[i]->acol];
      if (item_[i]->pkind != 0) {
        ++share[item_[i]->pcol];
        ++share[item_[i]->pval];
      }
    }
    auto once = [&](const void* p, double bytes) { return bytes / std::max(1, share[p]); };
    // initial block QR of R_0: V_0 S = R_0 (S -> G)
    hipLaunchKernelGGL(k_init_cycle, dim3(nact), dim3(256), 0, s, a, KP);
    a.mode = 1; a.nbl = 0; a.zero_init = 0; a.ignore_done = 0; a.W = E.W.p;
    a.Hsrc = E.Hc.p + E.hc2off; a.hsrc_stride = E.hcs; a.hsign = 1.0; a.Hsrc1 = E.Hc.p;
    launch_upd<KP, UPD_P2>(ctx, -1, gR, s, a, 0);
    hipLaunchKernelGGL(k_reduce_seg, dim3((KP * KP + 7) / 8, nact), dim3(256), 0, s, (const double*)E.part.p,
                       E.lstride, KP * KP, (const SegDesc*)E.seg_d, a.slist, 0, (const DevState*)E.st, 1, E.Hc.p,
                       E.hcs, E.hc2off);
    if (!F::RS) hipLaunchKernelGGL(k_p3_setup<KP>, dim3(nact), dim3(256), 8, s, a);
    launch_upd<KP, UPD_P3>(ctx, -1, gR, s, a, 0);
    hipLaunchKernelGGL((k_hess<KP>), dim3(nact), dim3(256), 0, s, a);
    PMOR_HIP(hipGetLastError());
    a.mode = 0;
    prof_first_ = (int)prof.recs.size();
    hipEvent_t* evs = ctx->evs;
    const int LOOKAHEAD = 2;
    for (int jj = 0; jj < m; ++jj) {
      // Z = P V_j (V_j = W1 R2^{-1} written on the way); W = A Z
      SpArgs sp{E.seg_d, stab_d, E.st, 1, 1, E.W.p, E.Z.p, E.T.p, nullptr, 1.0, 0.0,
                E.V.p + (int64_t)jj * a.vstride, 1};
      int pr = prof_start(ctx, PMOR_PROF_SPMM_P);
      launch_spmm_seg<KP, true>(ctx, pr, anyq ? 1 : 3, gS, lprP, s, sp);
      if (anyq) {
        SpArgs sq{E.seg_d, stab_d, E.st, 2, 1, E.T.p, E.Z.p, nullptr, nullptr, 1.0, 0.0, nullptr, 1};
        launch_spmm_seg<KP, false>(ctx, pr, 2, gS, lprP, s, sq);
      }
      prof_seg(pr, jj, [&](int i) {
        const SolveItem* x = item_[i];
        // P_1's values and P's pattern (columns, row pointers) may be shared
        const double pat = once(x->pcol, 4.0 * x->nnzP + 4.0 * (x->n + 1));
        const double p1 = once(x->pval, 8.0 * x->nnzP);
        if (x->pkind == 0) return 3.0 * blkb(i);
        if (x->pkind == 1) return pat + p1 + 3.0 * blkb(i);
        if (x->pkind == 3) return pat + p1 + 8.0 * x->n + 3.0 * blkb(i);
        return pat + p1 + 8.0 * x->nnzP + 5.0 * blkb(i);  // Q_l's own values on P's pattern
      });
      SpArgs sa{E.seg_d, stab_d, E.st, 0, 1, E.Z.p, E.W.p, nullptr, nullptr, 1.0, 0.0, nullptr, 1};
      pr = prof_start(ctx, PMOR_PROF_SPMM_A);
      launch_spmm_seg<KP, false>(ctx, pr, 3, gS, lprA, s, sa);
      prof_seg(pr, jj, [&](int i) {
        const SolveItem* x = item_[i];
        return once(x->acol, 4.0 * x->nnzA + 4.0 * (x->n + 1)) + 8.0 * x->nnzA + 2.0 * blkb(i);
      });
      a.nbl = jj + 1;
      const int L1 = (jj + 1) * KP * KP + KP, L2 = (jj + 1) * KP * KP + KP * KP;
      pr = prof_start(ctx, PMOR_PROF_CGS_DOT);
      launch_dot<KP>(ctx, pr, gR, s, a, jj + 1);
      prof_seg(pr, jj, [&](int i) { return blkb(i) * (jj + 2); });
      hipLaunchKernelGGL(k_reduce_seg, dim3((L1 + 7) / 8, nact), dim3(256), 0, s, (const double*)E.part.p,
                         E.lstride, L1, (const SegDesc*)E.seg_d, a.slist, 0, (const DevState*)E.st, 1, E.Hc.p, E.hcs,
                         (int64_t)0);
      a.Hsrc = E.Hc.p; a.hsrc_stride = E.hcs; a.hsign = 1.0;
      pr = prof_start(ctx, PMOR_PROF_CGS_UPD_DOT);
      launch_upd<KP, UPD_P2>(ctx, pr, gR, s, a, jj + 1);
      // kp = 4: W' stays in registers (pass 3 forms it again)
      prof_seg(pr, jj, [&](int i) { return blkb(i) * (jj + (F::RS ? 2 : 3)); });
      hipLaunchKernelGGL(k_reduce_seg, dim3((L2 + 7) / 8, nact), dim3(256), 0, s, (const double*)E.part.p,
                         E.lstride, L2, (const SegDesc*)E.seg_d, a.slist, 0, (const DevState*)E.st, 1, E.Hc.p, E.hcs,
                         E.hc2off);
      a.Hsrc = E.Hc.p + E.hc2off;
      a.Hsrc1 = E.Hc.p;
      if (!F::RS)  // kp = 4: every pass-3 workgroup does the set-up itself (measured faster)
        hipLaunchKernelGGL(k_p3_setup<KP>, dim3(nact), dim3(256), sizeof(double) * (jj + 1) * KP * KP, s, a);
      pr = prof_start(ctx, PMOR_PROF_CGS_UPD_GRAM);
      launch_upd<KP, UPD_P3>(ctx, pr, gR, s, a, jj + 1);
      prof_seg(pr, jj, [&](int i) { return blkb(i) * (jj + 3); });
      hipLaunchKernelGGL((k_hess<KP>), dim3(nact), dim3(256), hess_shm_, s, a);
      PMOR_HIP(hipGetLastError());
      PMOR_HIP(hipEventRecord(evs[jj % 64], s));
      if (jj >= LOOKAHEAD) {
        PMOR_HIP(hipEventSynchronize(evs[(jj - LOOKAHEAD) % 64]));
        bool all = true;
        for (int i : act_)
          if (!((volatile int*)E.hinfo_h)[4 * i + 1]) { all = false; break; }
        if (all) break;
      }
    }
    // Y, X += P (V Y)
    hipLaunchKernelGGL((k_ysolve<KP>), dim3(nact), dim3(256), ys_shm_, s, a, ys_pw_);
    a.nbl = -1; a.Hsrc = E.Y.p; a.hsrc_stride = E.ys; a.hsign = -1.0; a.zero_init = 1; a.ignore_done = 1;
    a.W = E.T.p;
    launch_upd<KP, UPD_PLAIN>(ctx, -1, gR, s, a, m);
    a.W = E.W.p; a.zero_init = 0; a.ignore_done = 0;
    SpArgs sx{E.seg_d, stab_d, E.st, 1, 0, E.T.p, E.Xc.p, E.Z.p, E.Xc.p, 1.0, 1.0, nullptr, 1};
    launch_spmm_seg<KP, false>(ctx, -1, 3, gS, lprP, s, sx);
    if (anyq) {
      SpArgs sx2{E.seg_d, stab_d, E.st, 2, 0, E.Z.p, E.Xc.p, nullptr, E.Xc.p, 1.0, 1.0, nullptr, 1};
      launch_spmm_seg<KP, false>(ctx, -1, 3, gS, lprP, s, sx2);
    }
    // residual R = B - A X into W, and its column norms
    SpArgs sr{E.seg_d, stab_d, E.st, 0, 0, E.Xc.p, E.W.p, nullptr, E.Bc.p, -1.0, 1.0, nullptr, 1};
    launch_spmm_seg<KP, false>(ctx, -1, 3, gS, lprA, s, sr);
    hipLaunchKernelGGL((k_colnorm_seg<KP>), dim3(gR), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_reduce_seg, dim3((KP + 7) / 8, nact), dim3(256), 0, s, (const double*)E.part.p, E.lstride,
                       KP, (const SegDesc*)E.seg_d, a.slist, 0, (const DevState*)E.st, 0, E.nrm.p, (int64_t)KMAX,
                       (int64_t)0);
    PMOR_HIP(hipGetLastError());
    PMOR_HIP(hipMemcpyAsync(E.nrm_h, E.nrm.p, sizeof(double) * nslots_ * KMAX, hipMemcpyDeviceToHost, s));
    PMOR_HIP(hipStreamSynchronize(s));
    return PMOR_OK;
  }

  pmor_ctx* ctx_;
  Engine& E_;
  pmor_solve_opts o_;
  int64_t rows_cap_;
  int nslots_;
  int sp_rows_ = 64;
  int lprA_ = 0, lprP_ = 0;  // SpMM lanes per row for A and for the preconditioner
  size_t hess_shm_ = 0, ys_shm_ = 0;
  int ys_pw_ = 32;
  int prof_first_ = 0;
  std::vector<SolveItem*> item_;
  std::vector<int64_t> r0_, nrows_;
  std::vector<int> Gw_, Gs_, cyc_, steps_of_;
  std::vector<int> act_, pending_, free_slots_;
  std::vector<std::pair<int64_t, int64_t>> free_rows_;
  std::chrono::steady_clock::time_point t0_;
};

int runner_create(pmor_ctx* ctx, Engine* E, int k, const pmor_solve_opts& o, int64_t rows_cap, int nslots,
                  Runner** out) {
  *out = nullptr;
  const int kp = pad_kp(std::max(k, 1));
  if (o.m < 1 || o.m + 1 > 32) return fail(PMOR_EINVAL, "restart length m must be in 1..31");
  if ((int64_t)(o.m + 1) * kp * kp > 8192) return fail(PMOR_EINVAL, "m and k too large for the Hessenberg kernel");
  if (nslots < 1) return fail(PMOR_EINVAL, "the engine needs at least one slot");
  Runner* r = nullptr;
  int rc = PMOR_OK;
  switch (kp) {
#define RUNNER_CASE(K)                                          \
    case K: {                                                   \
      auto* t = new RunnerT<K>(ctx, E, o, rows_cap, nslots);    \
      rc = t->init();                                           \
      r = t;                                                    \
      break;                                                    \
    }
    RUNNER_CASE(1) RUNNER_CASE(2) RUNNER_CASE(4) RUNNER_CASE(8) RUNNER_CASE(16)
#undef RUNNER_CASE
    default: return fail(PMOR_EINVAL, "bad block size");
  }
  if (rc != PMOR_OK) {
    delete r;
    return rc;
  }
  *out = r;
  return PMOR_OK;
}

Engine* engine_new() { return new Engine(); }
int64_t engine_bytes(const Engine* e) { return e ? e->bytes : 0; }

int krylov_batch(pmor_ctx* ctx, SolveItem* items, int nitems, const pmor_solve_opts& o) {
  if (nitems <= 0) return PMOR_OK;
  int kmax = 1;
  int64_t rows = 0;
  for (int i = 0; i < nitems; ++i) {
    kmax = std::max(kmax, items[i].k);
    rows += std::max<int64_t>(16, ((int64_t)items[i].n + 15) / 16 * 16);
  }
  if (!ctx->eng) ctx->eng = new Engine();
  Runner* r = nullptr;
  PMOR_TRY(runner_create(ctx, ctx->eng, kmax, o, rows, nitems, &r));
  std::vector<SolveItem*> ptrs(nitems);
  for (int i = 0; i < nitems; ++i) ptrs[i] = &items[i];
  int rc = r->admit(ptrs.data(), nitems);
  std::vector<SolveItem*> done;
  while (rc == PMOR_OK && r->busy() > 0) rc = r->cycle(done);
  delete r;
  return rc;
}

}  // namespace pmor
