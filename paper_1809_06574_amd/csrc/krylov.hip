// Block GMRES(m) with right preconditioning (paper, Section 2.1 and the
// footnote of Section 2.2 on right preconditioning).
//
// One block step j:   Z = P V_j;  W = A Z;
//   classical Gram-Schmidt twice against [V_0..V_j] (H accumulates both passes);
//   thin QR of W by Cholesky QR applied twice: V_{j+1} H_{j+1,j} = W;
//   Householder update of the QR of the block Hessenberg matrix and the
//   least-squares residual of every column (convergence test on the device).
// End of cycle: Y = R^{-1} G;  X += P (V Y);  residual B - A X.
//
// Layout: every n x kp block is row-major (kp contiguous doubles per row);
// V holds (m+1) such blocks back to back.  The inner products V^T W and the
// Gram matrices W^T W are tall-skinny contractions over the n rows done with
// the FP64 MFMA v_mfma_f64_4x4x4f64 for kp in {4, 8, 16}: a wavefront takes 16
// rows x 4 columns (512 contiguous bytes) per operand tile.  Lane l of such a
// tile holds row 16c + (l >> 2), column (l & 3); with the instruction's
// operand layout (A[i][k] at lane 16k + 4b + i, B[k][j] at lane 16k + 4b + j,
// D[i][j] at lane 16i + 4b + j) the same register serves as A or B operand and
// the four blocks b sum rows 4k + b.  kp in {1, 2} use one row per lane.
// Cross-workgroup sums use a fixed two-level order (no floating-point atomics),
// so every result is reproducible bit for bit.
#include "common.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>

namespace pmor {

__device__ __forceinline__ double mfma4(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

struct KArgs {
  int n;
  int m;
  int64_t vstride;   // n * kp
  double* V;
  double* W;         // work block (input/output of the orthogonalisation)
  const double* Hsrc;  // coefficients for the update kernels ([basis][rhs], row-major)
  double hsign;      // the update computes W <- W - hsign * V Hsrc
  double* Hc1;       // pass-1 coefficients (+ kp squared column norms of W)
  double* Hc2;       // pass-2 coefficients
  double* Gram;      // kp x kp Gram matrix
  double* Hbar;
  int ldh;
  double* G;
  int ldg;
  double* refl;
  double* Y;
  double* part;
  double* part2;
  double* partg0;    // per-workgroup partial Gram matrices of the sweep before the first scaling
  double* partg1;    // ... and of the first scaling sweep
  DevState* st;
  int* hflag;        // host-mapped {steps, done}
  int nbl_mode;      // 0: st->j + 1 blocks, 1: none (initial QR), 2: st->j blocks (V Y)
  int out_block;     // k_scale: 0 = V_{st->j + 1}, 1 = V_0
  int zero_init;     // update kernels: start from W = 0
  int ignore_done;   // run even when the cycle is marked done (end-of-cycle V Y)
};

__device__ __forceinline__ int nblocks_of(const KArgs& a) {
  return a.nbl_mode == 0 ? a.st->j + 1 : (a.nbl_mode == 1 ? 0 : a.st->j);
}

// ---------------------------------------------------------------------------
// cross-workgroup sums: every row-parallel kernel writes one partial row per
// workgroup (part[g * L + t]); these kernels add them up in a fixed order (no
// atomics, no inter-workgroup fences), so results are reproducible bit for bit.
// ---------------------------------------------------------------------------
// out[t] = sum_g part[g L + t]: 8 entries per workgroup, 32 lanes per entry, lane r
// sums g = r, r + 32, ... in order, then a fixed tree over the lanes.
__global__ __launch_bounds__(256) void k_reduce_cols(const double* __restrict__ part, int L, int G, double* out,
                                                     const DevState* st, int check_done) {
  if (check_done && st->done) return;
  __shared__ double s[8][33];
  const int e = threadIdx.x & 7, r = threadIdx.x >> 3;
  const int t = blockIdx.x * 8 + e;
  // four interleaved running sums (g = r + 32 (4q + u)), combined in a fixed order
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  if (t < L) {
    int g = r;
    for (; g + 96 < G; g += 128) {
      a0 += part[(size_t)g * L + t];
      a1 += part[(size_t)(g + 32) * L + t];
      a2 += part[(size_t)(g + 64) * L + t];
      a3 += part[(size_t)(g + 96) * L + t];
    }
    for (; g < G; g += 32) a0 += part[(size_t)g * L + t];
  }
  s[e][r] = (a0 + a1) + (a2 + a3);
  __syncthreads();
  for (int o = 16; o >= 1; o >>= 1) {
    if (r < o) s[e][r] += s[e][r + o];
    __syncthreads();
  }
  if (r == 0 && t < L) out[t] = s[e][0];
}

// the same sum inside one workgroup of 256 threads, for L <= 256 (result in dst)
__device__ void block_reduce_partials(const double* __restrict__ part, int L, int G, double* dst) {
  __shared__ double s[256];
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
  if (threadIdx.x < R * L) s[r * L + e] = (a0 + a1) + (a2 + a3);
  __syncthreads();
  for (int o = R / 2; o >= 1; o >>= 1) {
    if (r < o) s[r * L + e] += s[(r + o) * L + e];
    __syncthreads();
  }
  if (threadIdx.x < L) dst[threadIdx.x] = s[threadIdx.x];
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

// Prologue of the first scaling sweep, run by every workgroup: the Gram matrix
// of W from the previous sweep's partials, its Cholesky factor R1 and R1^{-1}
// (in LDS), the scale max_c ||W_c|| of the deficiency test.  Workgroup 0 also
// stores R1, the scale and the H column block (both passes' coefficients).
__device__ void scale1_prologue(const KArgs& a, int kp, int G, double* sR, double* sRinv, int* sok) {
  DevState* st = a.st;
  __shared__ double sG[KMAX * KMAX];
  block_reduce_partials(a.partg0, kp * kp, G, sG);
  const int nbl = nblocks_of(a);
  if (threadIdx.x == 0) {
    double mx = 0.0;
    for (int c = 0; c < st->kact; ++c)
      mx = fmax(mx, a.nbl_mode == 0 ? a.Hc1[nbl * kp * kp + c] : sG[c * kp + c]);
    const double ws = sqrt(mx);
    const double thr = 1e-14 * ws;
    const bool ok = chol_upper(sG, kp, st->kact, thr * thr, sR, sRinv);
    *sok = ok ? 1 : 0;
    if (blockIdx.x == 0) {
      st->wscale = ws;
      st->deficient = ok ? 0 : 1;
      for (int t = 0; t < kp * kp; ++t) st->R1[t] = sR[t];
    }
  }
  if (blockIdx.x == 0 && a.nbl_mode == 0) {
    const int j = st->j;
    for (int t = threadIdx.x; t < nbl * kp * kp; t += blockDim.x) {
      const int b = t / kp, c = t % kp;
      a.Hbar[b + (int64_t)(j * kp + c) * a.ldh] = a.Hc1[t] + a.Hc2[t];
    }
  }
  __syncthreads();
}

// Prologue of the final scaling sweep, run by every workgroup: R2 from the Gram
// matrix of W R1^{-1}, H_{j+1,j} = R2 R1 (S of the initial block) and the
// deficiency test |(R2 R1)_cc| <= 1e-14 max ||W_c||.  Workgroup 0 stores the
// block into the Hessenberg matrix (or G) and the verdict into the state.
__device__ void scale2_prologue(const KArgs& a, int kp, int G, double* sR2inv, int* sdef) {
  DevState* st = a.st;
  __shared__ double sG[KMAX * KMAX], sR2[KMAX * KMAX], sHs[KMAX * KMAX];
  block_reduce_partials(a.partg1, kp * kp, G, sG);
  if (threadIdx.x == 0) {
    const int kact = st->kact;
    bool ok = chol_upper(sG, kp, kact, 0.0, sR2, sR2inv) && !st->deficient;
    for (int r = 0; r < kp; ++r)
      for (int c = 0; c < kp; ++c) {
        double x = 0.0;
        if (r < kact && c < kact)
          for (int t = r; t <= c; ++t) x += sR2[r * kp + t] * st->R1[t * kp + c];
        sHs[r * kp + c] = x;
      }
    const double thr = 1e-14 * st->wscale;
    for (int c = 0; c < kact; ++c)
      if (!(fabs(sHs[c * kp + c]) > thr)) ok = false;
    if (!ok)
      for (int t = 0; t < kp * kp; ++t) sHs[t] = 0.0;
    *sdef = ok ? 0 : 1;
    if (blockIdx.x == 0) {
      if (a.nbl_mode == 0) {
        const int j = st->j;
        const int r0 = (j + 1) * kp;
        for (int r = 0; r < kp; ++r)
          for (int c = 0; c < kp; ++c) a.Hbar[(r0 + r) + (int64_t)(j * kp + c) * a.ldh] = sHs[r * kp + c];
      } else {
        for (int r = 0; r < kp; ++r)
          for (int c = 0; c < kp; ++c) a.G[r + (int64_t)c * a.ldg] = sHs[r * kp + c];
      }
      if (!ok) {
        st->deficient = 1;
        if (a.nbl_mode != 0) { st->breakdown = 1; st->done = 1; }
      }
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// MFMA path (kp = 4, 8, 16): tiles of 16 rows x 4 columns
// ---------------------------------------------------------------------------
template <int KP, int NW, int BPW>
struct Cfg {
  static constexpr int NT = KP / 4;
};

// pass 1: Hc1 = [V_0..V_j]^T W and the squared column norms of W
template <int KP, int NW, int BPW>
__global__ __launch_bounds__(64 * NW) void k_dot_mfma(KArgs a) {
  constexpr int NT = KP / 4;
  DevState* st = a.st;
  if (st->done) return;
  const int nbl = nblocks_of(a);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int G = gridDim.x, g = blockIdx.x;
  const int c4 = lane & 3, rsub = lane >> 2;
  const int nch = (a.n + 15) >> 4;
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
  for (int ch = xcd_swizzle(g, G); ch < nch; ch += G) {
    const int row = (ch << 4) + rsub;
    const bool valid = row < a.n;
    double wt[NT];
#pragma unroll
    for (int h = 0; h < NT; ++h) wt[h] = valid ? a.W[(int64_t)row * KP + 4 * h + c4] : 0.0;
    if (w == 0) {
#pragma unroll
      for (int h = 0; h < NT; ++h) wn[h] += wt[h] * wt[h];
    }
#pragma unroll
    for (int bi = 0; bi < BPW; ++bi) {
      const int i = w + NW * bi;
      if (i < nbl) {
        const double* Vi = a.V + (int64_t)i * a.vstride + (int64_t)row * KP + c4;
#pragma unroll
        for (int h = 0; h < NT; ++h) {
          const double v = valid ? Vi[4 * h] : 0.0;
#pragma unroll
          for (int h2 = 0; h2 < NT; ++h2) acc[bi][h][h2] = mfma4(v, wt[h2], acc[bi][h][h2]);
        }
      }
    }
  }
  const int L = nbl * KP * KP + KP;
  double* mypart = a.part + (int64_t)g * L;
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

// W <- W - hsign * [V_0..V_{nbl-1}] Hsrc, optionally followed by
//   DOT:  Hc2 = [V..]^T W   (pass 2 of the Gram-Schmidt)
//   GRAM: Gram = W^T W      (pass 3, or the first Cholesky QR sweep)
// The workgroup's NW wavefronts share the rows of a tile and split the V
// blocks; their partial updates meet in LDS (fixed order).
template <int KP, int NW, int BPW, bool DOT, bool GRAM>
__global__ __launch_bounds__(64 * NW) void k_upd_mfma(KArgs a) {
  constexpr int NT = KP / 4;
  DevState* st = a.st;
  if (st->done && !a.ignore_done) return;
  const int nbl = nblocks_of(a);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int G = gridDim.x, g = blockIdx.x;
  const int c4 = lane & 3, rsub = lane >> 2;
  const int nch = (a.n + 15) >> 4;
  extern __shared__ double sh[];
  double* sH = sh;                          // nbl*KP x KP
  double* su = sh + (size_t)nbl * KP * KP;  // [2][NW][64][NT]
  for (int t = threadIdx.x; t < nbl * KP * KP; t += blockDim.x) sH[t] = a.hsign * a.Hsrc[t];
  __syncthreads();
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
  int buf = 0;
  for (int ch = xcd_swizzle(g, G); ch < nch; ch += G) {
    const int row = (ch << 4) + rsub;
    const bool valid = row < a.n;
    double wt[NT], u[NT];
#pragma unroll
    for (int h = 0; h < NT; ++h) {
      wt[h] = (valid && !a.zero_init) ? a.W[(int64_t)row * KP + 4 * h + c4] : 0.0;
      u[h] = 0.0;
    }
    double vt[BPW][NT];
#pragma unroll
    for (int bi = 0; bi < BPW; ++bi) {
      const int i = w + NW * bi;
      if (i < nbl) {
        const double* Vi = a.V + (int64_t)i * a.vstride + (int64_t)row * KP + c4;
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
    if (w == 0 && valid && (nbl > 0 || a.zero_init)) {
#pragma unroll
      for (int h = 0; h < NT; ++h) a.W[(int64_t)row * KP + 4 * h + c4] = wnew[h];
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
  if (!DOT && !GRAM) return;
  const int L = DOT ? nbl * KP * KP : KP * KP;
  double* mypart = a.part + (int64_t)g * L;
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
  } else {
    if (w == 0) {
      double* gp = a.partg0 + (int64_t)g * KP * KP;
#pragma unroll
      for (int h = 0; h < NT; ++h)
#pragma unroll
        for (int h2 = 0; h2 < NT; ++h2) {
          double x = accg[h][h2];
          x += __shfl_xor(x, 4, 64);
          x += __shfl_xor(x, 8, 64);
          if (((lane >> 2) & 3) == 0) gp[(4 * h + (lane >> 4)) * KP + 4 * h2 + (lane & 3)] = x;
        }
    }
  }
}

// W <- W * M (M = a kp x kp upper-triangular inverse kept in DevState),
// optionally with its Gram matrix; writes either W in place or a V block.
template <int KP, int NW, bool GRAM>
__global__ __launch_bounds__(64 * NW) void k_scale_mfma(KArgs a, int Gprev) {
  constexpr int NT = KP / 4;
  DevState* st = a.st;
  if (st->done) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int G = gridDim.x, g = blockIdx.x;
  const int c4 = lane & 3, rsub = lane >> 2;
  const int nch = (a.n + 15) >> 4;
  __shared__ double sR[KMAX * KMAX], sM[KMAX * KMAX];
  __shared__ int sflag;
  if (GRAM) scale1_prologue(a, KP, Gprev, sR, sM, &sflag);
  else scale2_prologue(a, KP, Gprev, sM, &sflag);
  double* out;
  if (GRAM) out = a.W;
  else out = a.V + (int64_t)(a.out_block == 1 ? 0 : st->j + 1) * a.vstride;
  const bool zero = (!GRAM) && sflag;
  double accg[GRAM ? NT : 1][NT];
#pragma unroll
  for (int h = 0; h < (GRAM ? NT : 1); ++h)
#pragma unroll
    for (int h2 = 0; h2 < NT; ++h2) accg[h][h2] = 0.0;
  const int stride = G * NW;
  for (int ch = xcd_swizzle(g, G) * NW + w; ch < nch; ch += stride) {
    const int row = (ch << 4) + rsub;
    const bool valid = row < a.n;
    double wt[NT], o[NT];
#pragma unroll
    for (int h = 0; h < NT; ++h) {
      wt[h] = valid ? a.W[(int64_t)row * KP + 4 * h + c4] : 0.0;
      o[h] = 0.0;
    }
#pragma unroll
    for (int h = 0; h < NT; ++h) {
      const double v0 = quad_bcast<0>(wt[h]);
      const double v1 = quad_bcast<1>(wt[h]);
      const double v2 = quad_bcast<2>(wt[h]);
      const double v3 = quad_bcast<3>(wt[h]);
#pragma unroll
      for (int h2 = 0; h2 < NT; ++h2) {
        const int cc = 4 * h2 + c4;
        double x = o[h2];
        x = fma(v0, sM[(4 * h + 0) * KP + cc], x);
        x = fma(v1, sM[(4 * h + 1) * KP + cc], x);
        x = fma(v2, sM[(4 * h + 2) * KP + cc], x);
        x = fma(v3, sM[(4 * h + 3) * KP + cc], x);
        o[h2] = x;
      }
    }
    if (zero) {
#pragma unroll
      for (int h = 0; h < NT; ++h) o[h] = 0.0;
    }
    if (valid) {
#pragma unroll
      for (int h = 0; h < NT; ++h) out[(int64_t)row * KP + 4 * h + c4] = o[h];
    }
    if (GRAM) {
#pragma unroll
      for (int h = 0; h < NT; ++h)
#pragma unroll
        for (int h2 = 0; h2 < NT; ++h2) accg[h][h2] = mfma4(o[h], o[h2], accg[h][h2]);
    }
  }
  if (!GRAM) return;
  __shared__ double sg[NW][KP * KP];
#pragma unroll
  for (int h = 0; h < NT; ++h)
#pragma unroll
    for (int h2 = 0; h2 < NT; ++h2) {
      double x = accg[h][h2];
      x += __shfl_xor(x, 4, 64);
      x += __shfl_xor(x, 8, 64);
      if (((lane >> 2) & 3) == 0) sg[w][(4 * h + (lane >> 4)) * KP + 4 * h2 + (lane & 3)] = x;
    }
  __syncthreads();
  const int L = KP * KP;
  for (int t = threadIdx.x; t < L; t += blockDim.x) {
    double tot = 0.0;
    for (int q = 0; q < NW; ++q) tot += sg[q][t];
    a.partg1[(int64_t)g * L + t] = tot;
  }
}

// ---------------------------------------------------------------------------
// kp = 4, rows split over the wavefronts: each wavefront streams its own 16-row
// tiles against every V block (at most RS_B), so all of a tile's loads are in
// flight together and no LDS exchange is needed inside the loop.
// ---------------------------------------------------------------------------
constexpr int RS_B = 32;

// sum of a per-wavefront row of L values over the NW wavefronts, in order,
// written as this workgroup's partial row
template <int NW>
__device__ __forceinline__ void rs_store_partials(double (*sred)[RS_B * 16 + 4], int L, double* dst) {
  __syncthreads();
  for (int t = threadIdx.x; t < L; t += 64 * NW) {
    double tot = 0.0;
#pragma unroll
    for (int q = 0; q < NW; ++q) tot += sred[q][t];
    dst[t] = tot;
  }
}

template <int NW>
__global__ __launch_bounds__(64 * NW) void k_dot4(KArgs a) {
  DevState* st = a.st;
  if (st->done) return;
  const int nbl = nblocks_of(a);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int G = gridDim.x, g = blockIdx.x;
  const int nch = (a.n + 15) >> 4;
  __shared__ double sred[NW][RS_B * 16 + 4];
  double acc[RS_B];
#pragma unroll
  for (int i = 0; i < RS_B; ++i) acc[i] = 0.0;
  double wn = 0.0;
  for (int ch = xcd_swizzle(g, G) * NW + w; ch < nch; ch += G * NW) {
    const int64_t off = ((int64_t)ch << 6) + lane;  // 16 rows x 4 columns = 64 doubles
    const bool valid = off < (int64_t)a.n * 4;
    const double wt = valid ? a.W[off] : 0.0;
    wn += wt * wt;
    double v[RS_B];
#pragma unroll
    for (int i = 0; i < RS_B; ++i) v[i] = (i < nbl && valid) ? a.V[(int64_t)i * a.vstride + off] : 0.0;
#pragma unroll
    for (int i = 0; i < RS_B; ++i)
      if (i < nbl) acc[i] = mfma4(v[i], wt, acc[i]);
  }
#pragma unroll
  for (int i = 0; i < RS_B; ++i) {
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
  const int L = nbl * 16 + 4;
  rs_store_partials<NW>(sred, L, a.part + (int64_t)g * L);
}

// Lane l of a 16 x 4 tile holds (row 16c + (l >> 2), column l & 3).  Used as the
// A operand of v_mfma_f64_4x4x4f64 a tile contracts over the rows; the update
// W - V H needs the rows as the M index instead, i.e. the 4 x 4 transpose inside
// each group of 16 lanes: lane l takes the value of lane ((l & 3) << 4) | (l & 12) | (l >> 4).
__device__ __forceinline__ double tile_transpose(double x, int lane) {
  const int src = ((lane & 3) << 4) | (lane & 12) | (lane >> 4);
  return __shfl(x, src, 64);
}

// W <- W - hsign V Hsrc for all blocks, then (DOT) V^T W or (GRAM) W^T W.  Both
// the update and the inner products run on the FP64 MFMA: for the update the
// transposed V tile is the A operand, -hsign H the B operand and W the
// accumulator (D[i][j] at lane 16i + 4b + j is the tile's own layout).
template <int NW, bool DOT, bool GRAM>
__global__ __launch_bounds__(64 * NW) void k_upd4(KArgs a) {
  DevState* st = a.st;
  if (st->done && !a.ignore_done) return;
  const int nbl = nblocks_of(a);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int G = gridDim.x, g = blockIdx.x;
  const int nch = (a.n + 15) >> 4;
  __shared__ double sred[(DOT || GRAM) ? NW : 1][RS_B * 16 + 4];
  // B operand of block i: B[k][j] = -hsign H[4i + k][j], k = lane >> 4, j = lane & 3
  __shared__ double sH[RS_B * 16];
  for (int t = threadIdx.x; t < nbl * 16; t += blockDim.x) sH[t] = -a.hsign * a.Hsrc[t];
  __syncthreads();
  const double* hb = sH + (lane >> 4) * 4 + (lane & 3);
  double acc[DOT ? RS_B : 1];
#pragma unroll
  for (int i = 0; i < (DOT ? RS_B : 1); ++i) acc[i] = 0.0;
  double accg = 0.0;
  for (int ch = xcd_swizzle(g, G) * NW + w; ch < nch; ch += G * NW) {
    const int64_t off = ((int64_t)ch << 6) + lane;
    const bool valid = off < (int64_t)a.n * 4;
    const double wt = (valid && !a.zero_init) ? a.W[off] : 0.0;
    double v[RS_B];
#pragma unroll
    for (int i = 0; i < RS_B; ++i) v[i] = (i < nbl && valid) ? a.V[(int64_t)i * a.vstride + off] : 0.0;
    double u0 = wt, u1 = 0.0;  // two accumulation chains, added at the end
#pragma unroll
    for (int i = 0; i < RS_B; i += 2) {
      if (i < nbl) u0 = mfma4(tile_transpose(v[i], lane), hb[16 * i], u0);
      if (i + 1 < nbl) u1 = mfma4(tile_transpose(v[i + 1], lane), hb[16 * (i + 1)], u1);
    }
    const double wnew = u0 + u1;
    if (valid && (nbl > 0 || a.zero_init)) a.W[off] = wnew;
    if (DOT) {
#pragma unroll
      for (int i = 0; i < RS_B; ++i)
        if (i < nbl) acc[i] = mfma4(v[i], wnew, acc[i]);
    }
    if (GRAM) accg = mfma4(wnew, wnew, accg);
  }
  if (DOT) {
#pragma unroll
    for (int i = 0; i < RS_B; ++i) {
      double x = acc[i];
      x += __shfl_xor(x, 4, 64);
      x += __shfl_xor(x, 8, 64);
      if (i < nbl && ((lane >> 2) & 3) == 0) sred[w][i * 16 + (lane >> 4) * 4 + (lane & 3)] = x;
    }
    const int L = nbl * 16;
    rs_store_partials<NW>(sred, L, a.part + (int64_t)g * L);
  }
  if (GRAM) {
    double x = accg;
    x += __shfl_xor(x, 4, 64);
    x += __shfl_xor(x, 8, 64);
    if (((lane >> 2) & 3) == 0) sred[w][(lane >> 4) * 4 + (lane & 3)] = x;
    rs_store_partials<NW>(sred, 16, a.partg0 + (int64_t)g * 16);
  }
}

// ---------------------------------------------------------------------------
// row-per-lane path (kp = 1, 2)
// ---------------------------------------------------------------------------
template <int KP, int NW, int BPW>
__global__ __launch_bounds__(64 * NW) void k_dot_row(KArgs a) {
  DevState* st = a.st;
  if (st->done) return;
  const int nbl = nblocks_of(a);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int G = gridDim.x, g = blockIdx.x;
  const int nch = (a.n + 63) >> 6;
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
  for (int ch = xcd_swizzle(g, G); ch < nch; ch += G) {
    const int row = (ch << 6) + lane;
    const bool valid = row < a.n;
    double wt[KP];
#pragma unroll
    for (int x = 0; x < KP; ++x) wt[x] = valid ? a.W[(int64_t)row * KP + x] : 0.0;
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
          const double v = valid ? a.V[(int64_t)i * a.vstride + (int64_t)row * KP + x] : 0.0;
#pragma unroll
          for (int y = 0; y < KP; ++y) acc[bi][x][y] += v * wt[y];
        }
      }
    }
  }
  const int L = nbl * KP * KP + KP;
  double* mypart = a.part + (int64_t)g * L;
#pragma unroll
  for (int bi = 0; bi < BPW; ++bi) {
    const int i = w + NW * bi;
#pragma unroll
    for (int x = 0; x < KP; ++x)
#pragma unroll
      for (int y = 0; y < KP; ++y) {
        const double s = wave_sum(acc[bi][x][y]);
        if (i < nbl && lane == 0) mypart[(i * KP + x) * KP + y] = s;
      }
  }
  if (w == 0) {
#pragma unroll
    for (int x = 0; x < KP; ++x) {
      const double s = wave_sum(wn[x]);
      if (lane == 0) mypart[nbl * KP * KP + x] = s;
    }
  }
}

template <int KP, int NW, int BPW, bool DOT, bool GRAM>
__global__ __launch_bounds__(64 * NW) void k_upd_row(KArgs a) {
  DevState* st = a.st;
  if (st->done && !a.ignore_done) return;
  const int nbl = nblocks_of(a);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int G = gridDim.x, g = blockIdx.x;
  const int nch = (a.n + 63) >> 6;
  extern __shared__ double sh[];
  double* sH = sh;
  double* su = sh + (size_t)nbl * KP * KP;  // [2][NW][64][KP]
  for (int t = threadIdx.x; t < nbl * KP * KP; t += blockDim.x) sH[t] = a.hsign * a.Hsrc[t];
  __syncthreads();
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
  int buf = 0;
  for (int ch = xcd_swizzle(g, G); ch < nch; ch += G) {
    const int row = (ch << 6) + lane;
    const bool valid = row < a.n;
    double wt[KP], u[KP];
#pragma unroll
    for (int x = 0; x < KP; ++x) {
      wt[x] = (valid && !a.zero_init) ? a.W[(int64_t)row * KP + x] : 0.0;
      u[x] = 0.0;
    }
    double vt[BPW][KP];
#pragma unroll
    for (int bi = 0; bi < BPW; ++bi) {
      const int i = w + NW * bi;
#pragma unroll
      for (int x = 0; x < KP; ++x) vt[bi][x] = (i < nbl && valid) ? a.V[(int64_t)i * a.vstride + (int64_t)row * KP + x] : 0.0;
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
    if (w == 0 && valid && (nbl > 0 || a.zero_init)) {
#pragma unroll
      for (int x = 0; x < KP; ++x) a.W[(int64_t)row * KP + x] = wnew[x];
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
  if (!DOT && !GRAM) return;
  const int L = DOT ? nbl * KP * KP : KP * KP;
  double* mypart = a.part + (int64_t)g * L;
  if (DOT) {
#pragma unroll
    for (int bi = 0; bi < BPW; ++bi) {
      const int i = w + NW * bi;
#pragma unroll
      for (int x = 0; x < KP; ++x)
#pragma unroll
        for (int y = 0; y < KP; ++y) {
          const double s = wave_sum(acc[bi][x][y]);
          if (i < nbl && lane == 0) mypart[(i * KP + x) * KP + y] = s;
        }
    }
  } else {
    if (w == 0) {
      double* gp = a.partg0 + (int64_t)g * KP * KP;
#pragma unroll
      for (int x = 0; x < KP; ++x)
#pragma unroll
        for (int y = 0; y < KP; ++y) {
          const double s = wave_sum(accg[x][y]);
          if (lane == 0) gp[x * KP + y] = s;
        }
    }
  }
}

template <int KP, int NW, bool GRAM>
__global__ __launch_bounds__(64 * NW) void k_scale_row(KArgs a, int Gprev) {
  DevState* st = a.st;
  if (st->done) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int G = gridDim.x, g = blockIdx.x;
  const int nch = (a.n + 63) >> 6;
  __shared__ double sR[KMAX * KMAX], M[KMAX * KMAX];
  __shared__ int sflag;
  if (GRAM) scale1_prologue(a, KP, Gprev, sR, M, &sflag);
  else scale2_prologue(a, KP, Gprev, M, &sflag);
  double* out;
  if (GRAM) out = a.W;
  else out = a.V + (int64_t)(a.out_block == 1 ? 0 : st->j + 1) * a.vstride;
  const bool zero = (!GRAM) && sflag;
  double Mr[KP][KP];
#pragma unroll
  for (int x = 0; x < KP; ++x)
#pragma unroll
    for (int y = 0; y < KP; ++y) Mr[x][y] = M[x * KP + y];
  double accg[GRAM ? KP : 1][KP];
#pragma unroll
  for (int x = 0; x < (GRAM ? KP : 1); ++x)
#pragma unroll
    for (int y = 0; y < KP; ++y) accg[x][y] = 0.0;
  for (int ch = xcd_swizzle(g, G) * NW + w; ch < nch; ch += G * NW) {
    const int row = (ch << 6) + lane;
    const bool valid = row < a.n;
    double wt[KP], o[KP];
#pragma unroll
    for (int x = 0; x < KP; ++x) { wt[x] = valid ? a.W[(int64_t)row * KP + x] : 0.0; o[x] = 0.0; }
#pragma unroll
    for (int x = 0; x < KP; ++x)
#pragma unroll
      for (int y = 0; y < KP; ++y) o[y] = fma(wt[x], Mr[x][y], o[y]);
    if (zero) {
#pragma unroll
      for (int x = 0; x < KP; ++x) o[x] = 0.0;
    }
    if (valid) {
#pragma unroll
      for (int x = 0; x < KP; ++x) out[(int64_t)row * KP + x] = o[x];
    }
    if (GRAM) {
#pragma unroll
      for (int x = 0; x < KP; ++x)
#pragma unroll
        for (int y = 0; y < KP; ++y) accg[x][y] += o[x] * o[y];
    }
  }
  if (!GRAM) return;
  __shared__ double sg[NW][KP * KP];
#pragma unroll
  for (int x = 0; x < KP; ++x)
#pragma unroll
    for (int y = 0; y < KP; ++y) {
      const double s = wave_sum(accg[x][y]);
      if (lane == 0) sg[w][x * KP + y] = s;
    }
  __syncthreads();
  const int L = KP * KP;
  for (int t = threadIdx.x; t < L; t += blockDim.x) {
    double tot = 0.0;
    for (int q = 0; q < NW; ++q) tot += sg[q][t];
    a.partg1[(int64_t)g * L + t] = tot;
  }
}

// ---------------------------------------------------------------------------
// single-workgroup kernels: Cholesky steps, Hessenberg least squares, Y solve
// ---------------------------------------------------------------------------
// Householder update of the QR factorisation of the block Hessenberg matrix
// for the new block column j, the transformed right-hand side G, and the
// least-squares residual estimate of every column.  One wavefront.
template <int KP>
__global__ __launch_bounds__(64) void k_hess(KArgs a) {
  DevState* st = a.st;
  if (st->done) return;
  extern __shared__ double sh[];
  const int j = st->j, m = st->m, kact = st->kact;
  const int ldh = a.ldh;
  const int q0 = j * KP, nr = (j + 2) * KP;
  constexpr int RL = KP + 2;          // stored reflector: tau, v_1..v_KP, (unused)
  double* col = sh;                   // [KP][ldh]
  double* rf = col + (size_t)KP * ldh;  // [q0 + KP][RL]
  double* gw = rf + (size_t)(q0 + KP) * RL;  // [KP][2 KP] window of G
  const int lane = threadIdx.x;
  for (int t = lane; t < KP * nr; t += 64) {
    const int c = t / nr, r = t % nr;
    col[(size_t)c * ldh + r] = a.Hbar[r + (int64_t)(q0 + c) * ldh];
  }
  for (int t = lane; t < q0 * RL; t += 64) rf[t] = a.refl[t];
  for (int t = lane; t < KP * 2 * KP; t += 64) {
    const int c = t / (2 * KP), r = t % (2 * KP);
    gw[c * 2 * KP + r] = a.G[(q0 + r) + (int64_t)c * a.ldg];
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
          double d = w[r];
#pragma unroll
          for (int i = 1; i <= KP; ++i) d = fma(v[i], w[(r + i) % (KP + 1)], d);
          d *= v[0];
          w[r] -= d;
#pragma unroll
          for (int i = 1; i <= KP; ++i) w[(r + i) % (KP + 1)] = fma(-d, v[i], w[(r + i) % (KP + 1)]);
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
        double d = x[off];
        for (int r = 1; r <= KP; ++r) d = fma(v[r], x[off + r], d);
        d *= tau;
        x[off] -= d;
        for (int r = 1; r <= KP; ++r) x[off + r] = fma(-d, v[r], x[off + r]);
      }
    }
    __syncthreads();
  }
  // write back
  for (int t = lane; t < KP * nr; t += 64) {
    const int c = t / nr, r = t % nr;
    a.Hbar[r + (int64_t)(q0 + c) * ldh] = col[(size_t)c * ldh + r];
  }
  for (int t = lane; t < KP * RL; t += 64) a.refl[(size_t)q0 * RL + t] = rf[(size_t)q0 * RL + t];
  for (int t = lane; t < KP * 2 * KP; t += 64) {
    const int c = t / (2 * KP), r = t % (2 * KP);
    a.G[(q0 + r) + (int64_t)c * a.ldg] = gw[c * 2 * KP + r];
  }
  __syncthreads();
  if (lane == 0) {
    bool done = true;
    for (int c = 0; c < kact; ++c) {
      double s = 0.0;
      for (int r = KP; r < 2 * KP; ++r) s += gw[c * 2 * KP + r] * gw[c * 2 * KP + r];
      const double e = sqrt(s) / st->bnorm[c];
      st->est[c] = e;
      if (!(e <= st->tol)) done = false;
      if (e != e) st->nanflag = 1;
    }
    if (st->deficient) {
      if (!done) st->breakdown = 1;
      done = true;
    }
    if (st->nanflag) done = true;
    if (j + 1 >= m) done = true;
    st->j = j + 1;
    st->done = done ? 1 : 0;
    volatile int* hf = a.hflag;
    hf[0] = j + 1;
    hf[1] = done ? 1 : 0;
    __threadfence_system();
  }
}

// Y = R^{-1} G(0:J, :) with R the triangle of the transformed Hessenberg
// matrix, J = steps * kp; padded positions get y = 0.  Column panels of R go
// through LDS.
template <int KP>
__global__ __launch_bounds__(256) void k_ysolve(KArgs a, int PW) {
  DevState* st = a.st;
  const int J = st->j * KP;
  const int kact = st->kact;
  extern __shared__ double sh[];
  double* g = sh;                       // [J][KP]
  double* Rp = g + (size_t)J * KP;      // [PW][J] panel, column-major
  for (int t = threadIdx.x; t < J * KP; t += blockDim.x) {
    const int r = t / KP, c = t % KP;
    g[t] = a.G[r + (int64_t)c * a.ldg];
  }
  for (int p1 = J; p1 > 0; p1 -= PW) {
    const int p0 = p1 - PW > 0 ? p1 - PW : 0;
    __syncthreads();
    for (int t = threadIdx.x; t < (p1 - p0) * p1; t += blockDim.x) {
      const int cc = t / p1, r = t % p1;
      Rp[(size_t)cc * J + r] = a.Hbar[r + (int64_t)(p0 + cc) * a.ldh];
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
  for (int t = threadIdx.x; t < J * KP; t += blockDim.x) a.Y[t] = g[t];
}

// cycle start: G = 0, step counters reset
__global__ void k_init_cycle(KArgs a, int kp) {
  DevState* st = a.st;
  const int rows = (a.m + 1) * kp;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < rows * kp; t += gridDim.x * blockDim.x) {
    const int r = t % rows, c = t / rows;
    a.G[r + (int64_t)c * a.ldg] = 0.0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->j = 0;
    st->done = 0;
    st->deficient = 0;
    st->breakdown = 0;
    st->nanflag = 0;
    volatile int* hf = a.hflag;
    hf[0] = 0;
    hf[1] = 0;
    __threadfence_system();
  }
}

// ---------------------------------------------------------------------------
// CSR SpMM: Y = alpha A X + beta Bsrc (row-major blocks), LPR lanes per row
// ---------------------------------------------------------------------------
template <int KP, int LPR>
__global__ __launch_bounds__(256) void k_spmm(int n, const int32_t* __restrict__ rowptr,
                                              const int32_t* __restrict__ col, const double* __restrict__ val,
                                              const double* __restrict__ X, int64_t ldx, double* Y, int64_t ldy,
                                              double alpha, double beta, const double* Bsrc, int64_t ldb,
                                              const DevState* st, int vec) {
  if (st && st->done) return;
  const int64_t gid = (int64_t)xcd_swizzle(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int64_t row = gid / LPR;
  const int sub = (int)(gid % LPR);
  const bool valid = row < n;
  double acc[KP];
#pragma unroll
  for (int t = 0; t < KP; ++t) acc[t] = 0.0;
  if (valid) {
    const int e1 = rowptr[row + 1];
    if constexpr (KP % 2 == 0) {
      if (vec) {
        for (int e = rowptr[row] + sub; e < e1; e += LPR) {
          const int c = col[e];
          const double v = val[e];
          const double2* xr = reinterpret_cast<const double2*>(X + (int64_t)c * ldx);
#pragma unroll
          for (int t = 0; t < KP / 2; ++t) {
            const double2 x = xr[t];
            acc[2 * t] = fma(v, x.x, acc[2 * t]);
            acc[2 * t + 1] = fma(v, x.y, acc[2 * t + 1]);
          }
        }
      } else {
        for (int e = rowptr[row] + sub; e < e1; e += LPR) {
          const int c = col[e];
          const double v = val[e];
          const double* xr = X + (int64_t)c * ldx;
#pragma unroll
          for (int t = 0; t < KP; ++t) acc[t] = fma(v, xr[t], acc[t]);
        }
      }
    } else {
      for (int e = rowptr[row] + sub; e < e1; e += LPR) {
        const int c = col[e];
        const double v = val[e];
        const double* xr = X + (int64_t)c * ldx;
#pragma unroll
        for (int t = 0; t < KP; ++t) acc[t] = fma(v, xr[t], acc[t]);
      }
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
// at k = 1..8); PMOR_SPMM_LPR overrides the default
static int spmm_lanes_per_row() {
  static int lpr = [] {
    const char* e = getenv("PMOR_SPMM_LPR");
    const int v = e ? atoi(e) : 2;
    return (v == 1 || v == 2 || v == 4 || v == 8) ? v : 2;
  }();
  return lpr;
}

template <int LPR>
static int launch_spmm_lpr(int n, const int32_t* rowptr, const int32_t* col, const double* val, const double* X,
                           int64_t ldx, double* Y, int64_t ldy, int kp, double alpha, double beta, const double* Bsrc,
                           int64_t ldb, const DevState* st, hipStream_t stream, pmor_ctx* pc, int pidx, int ppart) {
  const int64_t threads = (int64_t)n * LPR;
  const unsigned grid = (unsigned)((threads + 255) / 256);
  const int vec = ((ldx % 2) == 0 && (reinterpret_cast<uintptr_t>(X) % 16) == 0) ? 1 : 0;
  switch (kp) {
#define SPMM_CASE(K) \
    case K: plaunch(pc, pidx, ppart, k_spmm<K, LPR>, dim3(grid), dim3(256), 0, stream, n, rowptr, col, val, X, ldx, \
                    Y, ldy, alpha, beta, Bsrc, ldb, st, vec); break;
    SPMM_CASE(1) SPMM_CASE(2) SPMM_CASE(3) SPMM_CASE(4) SPMM_CASE(5) SPMM_CASE(6) SPMM_CASE(7) SPMM_CASE(8)
    SPMM_CASE(9) SPMM_CASE(10) SPMM_CASE(11) SPMM_CASE(12) SPMM_CASE(13) SPMM_CASE(14) SPMM_CASE(15) SPMM_CASE(16)
#undef SPMM_CASE
    default: return fail(PMOR_EINVAL, "spmm: k out of range");
  }
  PMOR_HIP(hipGetLastError());
  return PMOR_OK;
}

int launch_spmm(int n, const int32_t* rowptr, const int32_t* col, const double* val, const double* X, int64_t ldx,
                double* Y, int64_t ldy, int kp, int kact, double alpha, double beta, const double* Bsrc,
                int64_t ldb, const DevState* st, hipStream_t stream, pmor_ctx* pc, int pidx, int ppart) {
  (void)kact;
  if (n == 0) return PMOR_OK;
  switch (spmm_lanes_per_row()) {
    case 1: return launch_spmm_lpr<1>(n, rowptr, col, val, X, ldx, Y, ldy, kp, alpha, beta, Bsrc, ldb, st, stream, pc,
                                      pidx, ppart);
    case 2: return launch_spmm_lpr<2>(n, rowptr, col, val, X, ldx, Y, ldy, kp, alpha, beta, Bsrc, ldb, st, stream, pc,
                                      pidx, ppart);
    case 8: return launch_spmm_lpr<8>(n, rowptr, col, val, X, ldx, Y, ldy, kp, alpha, beta, Bsrc, ldb, st, stream, pc,
                                      pidx, ppart);
    case 4: return launch_spmm_lpr<4>(n, rowptr, col, val, X, ldx, Y, ldy, kp, alpha, beta, Bsrc, ldb, st, stream, pc,
                                      pidx, ppart);
    default: return launch_spmm_lpr<2>(n, rowptr, col, val, X, ldx, Y, ldy, kp, alpha, beta, Bsrc, ldb, st, stream, pc,
                                       pidx, ppart);
  }
}

// ---------------------------------------------------------------------------
// column norms, gather/scatter of the compacted right-hand sides
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_colnorm2(int n, const double* X, int64_t ldx, int k, double* part,
                                                  double* part2, int* counters, double* out) {
  __shared__ double sw[4][KMAX];
  double acc[KMAX];
  for (int c = 0; c < KMAX; ++c) acc[c] = 0.0;
  for (int row = blockIdx.x * blockDim.x + threadIdx.x; row < n; row += gridDim.x * blockDim.x)
    for (int c = 0; c < k; ++c) {
      const double x = X[(int64_t)row * ldx + c];
      acc[c] += x * x;
    }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int c = 0; c < k; ++c) {
    const double s = wave_sum(acc[c]);
    if (lane == 0) sw[w][c] = s;
  }
  __syncthreads();
  if (threadIdx.x < k) part[(int64_t)blockIdx.x * k + threadIdx.x] =
      sw[0][threadIdx.x] + sw[1][threadIdx.x] + sw[2][threadIdx.x] + sw[3][threadIdx.x];
}

struct ColMap {
  int idx[KMAX];
};

__global__ void k_gather_cols(int n, const double* B, int64_t ldb, int kp, int kact, ColMap cm, double* Bc) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * kp) return;
  const int64_t row = t / kp;
  const int c = (int)(t % kp);
  Bc[t] = (c < kact) ? B[row * ldb + cm.idx[c]] : 0.0;
}

__global__ void k_scatter_cols(int n, const double* Xc, int kp, int k, ColMap inv, double* X, int64_t ldx) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * k) return;
  const int64_t row = t / k;
  const int c = (int)(t % k);
  X[row * ldx + c] = (inv.idx[c] >= 0) ? Xc[row * kp + inv.idx[c]] : 0.0;
}

__global__ void k_fill(double* x, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static int* dev_counters(DevState* st) {
  return reinterpret_cast<int*>(reinterpret_cast<char*>(st) + offsetof(DevState, counters));
}

static int pad_kp(int k) {
  if (k <= 1) return 1;
  if (k <= 2) return 2;
  if (k <= 4) return 4;
  if (k <= 8) return 8;
  return 16;
}

static int row_grid(int n, int rows_per_tile, int gmax = 512) {
  const int tiles = (n + rows_per_tile - 1) / rows_per_tile;
  int g = std::min(tiles, gmax);
  if (g >= 8) g &= ~7;  // a multiple of 8 keeps the XCD swizzle exact
  return std::max(g, 1);
}

void free_workspace(Workspace& ws) {
  double* bufs[] = {ws.V, ws.W, ws.Z, ws.T, ws.Bc, ws.Xc, ws.Hbar, ws.Hcol, ws.G, ws.refl, ws.Y, ws.part, ws.part2,
                    ws.partg};
  for (double* b : bufs)
    if (b) (void)hipFree(b);
  if (ws.st) (void)hipFree(ws.st);
  if (ws.st_host) (void)hipHostFree(ws.st_host);
  ws = Workspace{};
}

int ensure_workspace(pmor_problem* pb, int kp, int m) {
  Workspace& ws = pb->ws;
  if (ws.V && ws.n == pb->n && ws.kp == kp && ws.m >= m) return PMOR_OK;
  free_workspace(ws);
  const int64_t n = pb->n;
  ws.n = pb->n; ws.kp = kp; ws.m = m;
  const int64_t blk = std::max<int64_t>(n * kp, 1);
  const int64_t rows = (int64_t)(m + 1) * kp;
  auto alloc = [&](double** p, int64_t count) -> int {
    hipError_t e = hipMalloc((void**)p, sizeof(double) * std::max<int64_t>(count, 1));
    if (e != hipSuccess) return fail(PMOR_ENOMEM, "device allocation of the Krylov workspace failed");
    ws.bytes += sizeof(double) * count;
    return PMOR_OK;
  };
  PMOR_TRY(alloc(&ws.V, (m + 1) * blk));
  PMOR_TRY(alloc(&ws.W, blk));
  PMOR_TRY(alloc(&ws.Z, blk));
  PMOR_TRY(alloc(&ws.T, blk));
  PMOR_TRY(alloc(&ws.Bc, blk));
  PMOR_TRY(alloc(&ws.Xc, blk));
  PMOR_TRY(alloc(&ws.Hbar, rows * m * kp));
  // Hc1 | Hc2 (coefficients + kp norms each) | Gram (kp x kp) | residual norms (KMAX)
  PMOR_TRY(alloc(&ws.Hcol, 2 * (rows * kp + kp) + kp * kp + 2 * KMAX));
  PMOR_TRY(alloc(&ws.G, rows * kp));
  PMOR_TRY(alloc(&ws.refl, (int64_t)m * kp * (kp + 2) + kp * (kp + 2)));
  PMOR_TRY(alloc(&ws.Y, rows * kp));
  const int64_t L = rows * kp + kp + KMAX;
  ws.part_len = (size_t)L;
  PMOR_TRY(alloc(&ws.part, (int64_t)MAX_RED_WG * L));
  PMOR_TRY(alloc(&ws.part2, (int64_t)(MAX_RED_WG / RED_GROUP + 1) * L));
  PMOR_TRY(alloc(&ws.partg, (int64_t)2 * MAX_RED_WG * KMAX * KMAX));
  PMOR_HIP(hipMalloc((void**)&ws.st, sizeof(DevState)));
  PMOR_HIP(hipMemset(ws.st, 0, sizeof(DevState)));
  PMOR_HIP(hipHostMalloc((void**)&ws.st_host, sizeof(DevState) + 64, hipHostMallocMapped));
  std::memset(ws.st_host, 0, sizeof(DevState) + 64);
  return PMOR_OK;
}

namespace {

struct Launcher {
  pmor_problem* pb;
  const pmor_spai* h;
  int kp;
  int m;
  hipStream_t s;
  KArgs a;
  int G;   // workgroups of the row-parallel kernels
  int* hflag_dev;

  // W <- (P) V_j etc. are done by spmm; these wrap the block kernels
  template <int KP, int NW, int BPW>
  int dot(int pidx = -1) {
    pmor_ctx* c = pb->ctx;
    if constexpr (KP == 4) plaunch(c, pidx, 3, k_dot4<NW>, dim3(G), dim3(64 * NW), 0, s, a);
    else if constexpr (KP >= 4) plaunch(c, pidx, 3, k_dot_mfma<(KP >= 4 ? KP : 4), NW, BPW>, dim3(G), dim3(64 * NW), 0, s, a);
    else plaunch(c, pidx, 3, k_dot_row<(KP < 4 ? KP : 1), NW, BPW>, dim3(G), dim3(64 * NW), 0, s, a);
    PMOR_HIP(hipGetLastError());
    return PMOR_OK;
  }
  template <int KP, int NW, int BPW, bool DOT, bool GRAM>
  int upd(int nbl_max, int pidx = -1) {
    const int per = (KP >= 4) ? (KP / 4) : KP;
    const size_t shm = sizeof(double) * ((size_t)nbl_max * KP * KP + (size_t)2 * NW * 64 * per);
    pmor_ctx* c = pb->ctx;
    if constexpr (KP == 4)
      plaunch(c, pidx, 3, k_upd4<NW, DOT, GRAM>, dim3(G), dim3(64 * NW), 0, s, a);
    else if constexpr (KP >= 4)
      plaunch(c, pidx, 3, k_upd_mfma<(KP >= 4 ? KP : 4), NW, BPW, DOT, GRAM>, dim3(G), dim3(64 * NW), (uint32_t)shm, s, a);
    else
      plaunch(c, pidx, 3, k_upd_row<(KP < 4 ? KP : 1), NW, BPW, DOT, GRAM>, dim3(G), dim3(64 * NW), (uint32_t)shm, s, a);
    PMOR_HIP(hipGetLastError());
    return PMOR_OK;
  }
  template <int KP, int NW, bool GRAM>
  int scale() {
    if constexpr (KP >= 4) hipLaunchKernelGGL((k_scale_mfma<(KP >= 4 ? KP : 4), NW, GRAM>), dim3(G), dim3(64 * NW), 0, s, a, G);
    else hipLaunchKernelGGL((k_scale_row<(KP < 4 ? KP : 1), NW, GRAM>), dim3(G), dim3(64 * NW), 0, s, a, G);
    PMOR_HIP(hipGetLastError());
    return PMOR_OK;
  }
};

// preconditioner application Z = P_l X (P_l = Q P_1 when the pattern update is active)
int apply_P(pmor_problem* pb, const pmor_spai* h, const double* X, double* Z, double* tmp, int kp, int kact,
            const DevState* st, double beta, hipStream_t s, int pidx = -1) {
  const int n = pb->n;
  if (h->q_active) {
    PMOR_TRY(launch_spmm(n, h->Prowptr, h->Pcol, h->P1val, X, kp, tmp, kp, kp, kact, 1.0, 0.0, nullptr, 0, st, s,
                         pb->ctx, pidx, 1));
    return launch_spmm(n, h->Prowptr, h->Pcol, h->Qval, tmp, kp, Z, kp, kp, kact, 1.0, beta, Z, kp, st, s, pb->ctx,
                       pidx, 2);
  }
  return launch_spmm(n, h->Prowptr, h->Pcol, h->Pval, X, kp, Z, kp, kp, kact, 1.0, beta, Z, kp, st, s, pb->ctx, pidx,
                     3);
}

}  // namespace

// identity "matrix" for the unpreconditioned case: a copy kernel
__global__ void k_copy_axpby(int64_t len, const double* X, double* Z, double beta) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x)
    Z[i] = (beta != 0.0) ? Z[i] * beta + X[i] : X[i];
}

template <int KP>
static int run_cycles(pmor_problem* pb, const pmor_spai* h, int kact, const pmor_solve_opts& o, pmor_stats* stats,
                      const double* bnorm, int* steps_out, int* cycles_out, double* relres_out, int* status) {
  constexpr int NW = (KP == 16) ? 16 : (KP == 4 ? 8 : 4);
  constexpr int BPW = 32 / NW;  // V blocks per wavefront: m + 1 <= NW * BPW = 32
  Workspace& ws = pb->ws;
  hipStream_t s = pb->ctx->stream;
  const int n = pb->n, m = o.m;
  const int ldh = (m + 1) * KP;
  Launcher L{pb, h, KP, m, s, KArgs{}, row_grid(n, KP >= 4 ? 16 : 64, KP == 4 ? 256 : 512), nullptr};
  KArgs& a = L.a;
  a.n = n; a.m = m; a.vstride = (int64_t)n * KP;
  a.V = ws.V; a.W = ws.W;
  a.Hc1 = ws.Hcol; a.Hc2 = ws.Hcol + (ldh * KP + KP); a.Gram = ws.Hcol + 2 * (ldh * KP + KP);
  a.Hbar = ws.Hbar; a.ldh = ldh; a.G = ws.G; a.ldg = ldh; a.refl = ws.refl; a.Y = ws.Y;
  a.part = ws.part; a.part2 = ws.part2; a.st = ws.st;
  a.partg0 = ws.partg; a.partg1 = ws.partg + (int64_t)MAX_RED_WG * KMAX * KMAX;
  int* hflag = reinterpret_cast<int*>(reinterpret_cast<char*>(ws.st_host) + sizeof(DevState));
  int* hflag_dev = nullptr;
  PMOR_HIP(hipHostGetDevicePointer((void**)&hflag_dev, hflag, 0));
  a.hflag = hflag_dev;
  // per-solve device state
  DevState& init = *ws.st_host;
  std::memset(&init, 0, offsetof(DevState, counters));
  init.kact = kact; init.m = m; init.tol = o.tol;
  for (int c = 0; c < KMAX; ++c) init.bnorm[c] = (c < kact) ? bnorm[c] : 1.0;
  PMOR_HIP(hipMemcpyAsync(ws.st, &init, offsetof(DevState, counters), hipMemcpyHostToDevice, s));
  const int64_t blk = (int64_t)n * KP;
  const unsigned fgrid = (unsigned)std::min<int64_t>((blk + 255) / 256, 4096);
  // X = 0, W = R_0 = B
  hipLaunchKernelGGL(k_fill, dim3(fgrid), dim3(256), 0, s, ws.Xc, blk, 0.0);
  hipLaunchKernelGGL(k_copy_axpby, dim3(fgrid), dim3(256), 0, s, blk, ws.Bc, ws.W, 0.0);
  PMOR_HIP(hipGetLastError());
  const size_t hess_shm = sizeof(double) * ((size_t)KP * ldh + (size_t)(m * KP + KP) * (KP + 2) + 2 * KP * KP);
  const int ys_pw = (KP >= 16) ? 8 : 32;
  const size_t ys_shm = sizeof(double) * ((size_t)m * KP * KP + (size_t)ys_pw * m * KP);
  PMOR_TRY(allow_lds((const void*)k_hess<KP>, hess_shm));
  PMOR_TRY(allow_lds((const void*)k_ysolve<KP>, ys_shm));
  hipEvent_t* evs = pb->ctx->evs;
  const int LOOKAHEAD = 2;
  int total_steps = 0, cyc = 0;
  *status = PMOR_ENOTCONV;
  for (cyc = 0; cyc < o.max_cycles; ++cyc) {
    const int prof_first = (int)pb->ctx->prof.recs.size();
    // initial block QR of W = R_0: V_0 S = W, S -> G(0:kp, :)
    hipLaunchKernelGGL(k_init_cycle, dim3(64), dim3(256), 0, s, a, KP);
    a.nbl_mode = 1; a.hsign = 1.0; a.Hsrc = ws.Hcol; a.zero_init = 0;
    PMOR_TRY((L.template upd<KP, NW, BPW, false, true>(1)));
    PMOR_TRY((L.template scale<KP, NW, true>()));
    a.out_block = 1;
    PMOR_TRY((L.template scale<KP, NW, false>()));
    a.out_block = 0;
    // Arnoldi steps
    for (int jj = 0; jj < m; ++jj) {
      // Z = P V_j ; W = A Z  (V_j is block jj; the kernels skip once the cycle is done)
      const double* Vj = ws.V + (int64_t)jj * blk;
      const double blkb = 8.0 * (double)n * KP;
      int pr = prof_start(pb->ctx, PMOR_PROF_SPMM_P);
      if (h) PMOR_TRY(apply_P(pb, h, Vj, ws.Z, ws.T, KP, kact, ws.st, 0.0, s, pr));
      else plaunch(pb->ctx, pr, 3, k_copy_axpby, dim3(fgrid), dim3(256), 0, s, blk, (const double*)Vj, ws.Z, 0.0);
      prof_stop(pb->ctx, pr, h ? 12.0 * h->nnzP + 4.0 * (n + 1) + 2 * blkb : 2 * blkb, jj);
      pr = prof_start(pb->ctx, PMOR_PROF_SPMM_A);
      PMOR_TRY(launch_spmm(n, pb->rowptr, pb->col, pb->aval, ws.Z, KP, ws.W, KP, KP, kact, 1.0, 0.0, nullptr, 0,
                           ws.st, s, pb->ctx, pr, 3));
      prof_stop(pb->ctx, pr, 12.0 * pb->nnz + 4.0 * (n + 1) + 2 * blkb, jj);
      a.nbl_mode = 0;
      const int L1 = (jj + 1) * KP * KP + KP, L2 = (jj + 1) * KP * KP;
      pr = prof_start(pb->ctx, PMOR_PROF_CGS_DOT);
      PMOR_TRY((L.template dot<KP, NW, BPW>(pr)));
      prof_stop(pb->ctx, pr, blkb * (jj + 2), jj);
      hipLaunchKernelGGL(k_reduce_cols, dim3((L1 + 7) / 8), dim3(256), 0, s, ws.part, L1, L.G, a.Hc1, ws.st, 1);
      a.Hsrc = a.Hc1; a.hsign = 1.0;
      pr = prof_start(pb->ctx, PMOR_PROF_CGS_UPD_DOT);
      PMOR_TRY((L.template upd<KP, NW, BPW, true, false>(jj + 1, pr)));
      prof_stop(pb->ctx, pr, blkb * (jj + 3), jj);
      hipLaunchKernelGGL(k_reduce_cols, dim3((L2 + 7) / 8), dim3(256), 0, s, ws.part, L2, L.G, a.Hc2, ws.st, 1);
      a.Hsrc = a.Hc2;
      pr = prof_start(pb->ctx, PMOR_PROF_CGS_UPD_GRAM);
      PMOR_TRY((L.template upd<KP, NW, BPW, false, true>(jj + 1, pr)));
      prof_stop(pb->ctx, pr, blkb * (jj + 3), jj);
      PMOR_TRY((L.template scale<KP, NW, true>()));
      PMOR_TRY((L.template scale<KP, NW, false>()));
      hipLaunchKernelGGL((k_hess<KP>), dim3(1), dim3(64), hess_shm, s, a);
      PMOR_HIP(hipGetLastError());
      PMOR_HIP(hipEventRecord(evs[jj % 64], s));
      if (jj >= LOOKAHEAD) {
        PMOR_HIP(hipEventSynchronize(evs[(jj - LOOKAHEAD) % 64]));
        if (((volatile int*)hflag)[1]) break;
      }
    }
    // Y, X += P (V Y)
    hipLaunchKernelGGL((k_ysolve<KP>), dim3(1), dim3(256), ys_shm, s, a, ys_pw);
    a.nbl_mode = 2; a.Hsrc = ws.Y; a.hsign = -1.0; a.zero_init = 1; a.W = ws.T; a.ignore_done = 1;
    PMOR_TRY((L.template upd<KP, NW, BPW, false, false>(m)));
    a.W = ws.W; a.zero_init = 0; a.ignore_done = 0;
    if (h) PMOR_TRY(apply_P(pb, h, ws.T, ws.Xc, ws.Z, KP, kact, nullptr, 1.0, s));
    else hipLaunchKernelGGL(k_copy_axpby, dim3(fgrid), dim3(256), 0, s, blk, ws.T, ws.Xc, 1.0);
    // residual R = B - A X into W, and its column norms
    PMOR_TRY(launch_spmm(n, pb->rowptr, pb->col, pb->aval, ws.Xc, KP, ws.W, KP, KP, kact, -1.0, 1.0, ws.Bc, KP,
                         nullptr, s));
    double* nrm_dev = ws.Hcol + 2 * (ldh * KP + KP) + KP * KP;  // the residual-norm slots after the Gram matrix
    const int cg = std::min(row_grid(n, 256), 256);
    hipLaunchKernelGGL(k_colnorm2, dim3(cg), dim3(256), 0, s, n, ws.W, (int64_t)KP, KP, ws.part, ws.part2,
                       dev_counters(ws.st), nrm_dev);
    hipLaunchKernelGGL(k_reduce_cols, dim3((KP + 7) / 8), dim3(256), 0, s, ws.part, KP, cg, nrm_dev, ws.st, 0);
    PMOR_HIP(hipGetLastError());
    double nrm2[KMAX];
    PMOR_HIP(hipMemcpyAsync(nrm2, nrm_dev, sizeof(double) * KP, hipMemcpyDeviceToHost, s));
    PMOR_HIP(hipMemcpyAsync(ws.st_host, ws.st, offsetof(DevState, R1), hipMemcpyDeviceToHost, s));
    PMOR_HIP(hipStreamSynchronize(s));
    const DevState& hs = *ws.st_host;
    prof_drop_from(pb->ctx, prof_first, hs.j);
    total_steps += hs.j;
    if (stats && cyc < PMOR_MAX_CYCLES) stats->cycle_steps[cyc] = hs.j;
    bool conv = true, nan = hs.nanflag != 0;
    for (int c = 0; c < kact; ++c) {
      relres_out[c] = std::sqrt(nrm2[c]) / bnorm[c];
      if (!(relres_out[c] <= o.tol)) conv = false;
      if (std::isnan(relres_out[c]) || std::isinf(relres_out[c])) nan = true;
    }
    if (nan) { *status = PMOR_ENAN; ++cyc; break; }
    if (conv) { *status = PMOR_OK; ++cyc; break; }
    if (hs.breakdown) { *status = PMOR_EBREAKDOWN; ++cyc; break; }
  }
  *steps_out = total_steps;
  *cycles_out = cyc;
  return PMOR_OK;
}

int krylov_solve(pmor_problem* pb, const pmor_spai* h, const double* B, int64_t ldb, int k, double* X,
                 int64_t ldx, const pmor_solve_opts& o, pmor_stats* stats) {
  hipStream_t s = pb->ctx->stream;
  const int n = pb->n;
  const int kp = pad_kp(k);
  if (o.m + 1 > 32) return fail(PMOR_EINVAL, "restart length m must be <= 31");
  if ((int64_t)(o.m + 1) * kp * kp > 8192) return fail(PMOR_EINVAL, "m and k too large for the Hessenberg kernel");
  PMOR_TRY(ensure_workspace(pb, kp, o.m));
  Workspace& ws = pb->ws;
  // norms of the caller's columns
  double* nrm_dev = ws.Hcol;
  const int cg = std::min(row_grid(n, 256), 256);
  hipLaunchKernelGGL(k_colnorm2, dim3(cg), dim3(256), 0, s, n, B, ldb, k, ws.part, ws.part2, dev_counters(ws.st),
                     nrm_dev);
  hipLaunchKernelGGL(k_reduce_cols, dim3((k + 7) / 8), dim3(256), 0, s, ws.part, k, cg, nrm_dev, ws.st, 0);
  PMOR_HIP(hipGetLastError());
  double bn[KMAX];
  PMOR_HIP(hipMemcpyAsync(bn, nrm_dev, sizeof(double) * k, hipMemcpyDeviceToHost, s));
  PMOR_HIP(hipStreamSynchronize(s));
  ColMap act{}, inv{};
  int kact = 0;
  double bnorm[KMAX];
  for (int c = 0; c < k; ++c) {
    inv.idx[c] = -1;
    if (std::isnan(bn[c]) || std::isinf(bn[c])) return fail(PMOR_ENAN, "NaN or Inf in the right-hand side");
    if (bn[c] > 0.0) {
      inv.idx[c] = kact;
      act.idx[kact] = c;
      bnorm[kact] = std::sqrt(bn[c]);
      ++kact;
    }
  }
  if (stats) {
    stats->k = k;
    for (int c = 0; c < PMOR_KMAX; ++c) stats->relres[c] = 0.0;
  }
  const int64_t blk = (int64_t)n * kp;
  if (kact == 0) {
    hipLaunchKernelGGL(k_scatter_cols, dim3((unsigned)(((int64_t)n * k + 255) / 256)), dim3(256), 0, s, n, ws.Xc,
                       kp, k, inv, X, ldx);
    PMOR_HIP(hipGetLastError());
    PMOR_HIP(hipStreamSynchronize(s));
    if (stats) { stats->cycles = 0; stats->steps = 0; }
    return PMOR_OK;
  }
  hipLaunchKernelGGL(k_gather_cols, dim3((unsigned)((blk + 255) / 256)), dim3(256), 0, s, n, B, ldb, kp, kact, act,
                     ws.Bc);
  PMOR_HIP(hipGetLastError());
  int steps = 0, cycles = 0, status = PMOR_OK;
  double relres[KMAX];
  switch (kp) {
    case 1: PMOR_TRY(run_cycles<1>(pb, h, kact, o, stats, bnorm, &steps, &cycles, relres, &status)); break;
    case 2: PMOR_TRY(run_cycles<2>(pb, h, kact, o, stats, bnorm, &steps, &cycles, relres, &status)); break;
    case 4: PMOR_TRY(run_cycles<4>(pb, h, kact, o, stats, bnorm, &steps, &cycles, relres, &status)); break;
    case 8: PMOR_TRY(run_cycles<8>(pb, h, kact, o, stats, bnorm, &steps, &cycles, relres, &status)); break;
    case 16: PMOR_TRY(run_cycles<16>(pb, h, kact, o, stats, bnorm, &steps, &cycles, relres, &status)); break;
    default: return fail(PMOR_EINVAL, "bad block size");
  }
  hipLaunchKernelGGL(k_scatter_cols, dim3((unsigned)(((int64_t)n * k + 255) / 256)), dim3(256), 0, s, n, ws.Xc, kp, k,
                     inv, X, ldx);
  PMOR_HIP(hipGetLastError());
  PMOR_HIP(hipStreamSynchronize(s));
  if (stats) {
    stats->cycles = cycles;
    stats->steps = steps;
    for (int c = 0; c < k; ++c) stats->relres[c] = (inv.idx[c] >= 0) ? relres[inv.idx[c]] : 0.0;
  }
  if (status == PMOR_ENOTCONV) return fail(status, "block GMRES did not converge within max_cycles");
  if (status == PMOR_EBREAKDOWN) return fail(status, "block breakdown: rank-deficient block with unconverged columns");
  if (status == PMOR_ENAN) return fail(status, "NaN or Inf in a residual");
  return PMOR_OK;
}

}  // namespace pmor
