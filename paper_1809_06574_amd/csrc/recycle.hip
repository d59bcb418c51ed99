// Block GCRO-DR: block GMRES(m) with a recycled subspace carried from one
// system of a sequence to the next (the paper's solver, Section 3 and the
// block GCRO runs of Tables 3 and 5).  Right preconditioning, Op = A P.
//
// Per system: with a recycled basis U~ (n x kc), C = Op U~ = Q R (Cholesky QR
// twice), C <- Q, U <- U~ R^{-1}, so Op U = C with orthonormal C.  Each cycle
// starts from the true residual, projects it on C (X += P U C^T R,
// R -= C C^T R), runs block Arnoldi on (I - C C^T) Op with two classical
// Gram-Schmidt passes against [C, V] (coefficients B against C, H against V)
// and solves the block GMRES least squares y2 = argmin ||E1 S - Hbar y2||; the
// correction is X += P (V y2 - U B y2).  At the end of every cycle the harmonic
// Ritz vectors of Op on span([U D, V]) (the eigenproblem
// G^T (W^T V) z = mu G^T G z with G = [[D, B], [0, Hbar]], the kr of largest
// |mu|) give the new C and U.  The last U is kept for the next system.
//
// Device work is tall-skinny: SpMM with A and P (the library's CSR kernels),
// Gram products [.]^T W in two deterministic stages, and products
// Y = beta Y + alpha A G with the small matrix G staged in LDS.  The small
// dense work (Cholesky, the incremental Householder QR of the block Hessenberg
// matrix, the eigenproblem) runs on the host in FP64.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

#include "common.hpp"

struct pmor_recycle {
  pmor_ctx* ctx = nullptr;
  int n = 0, kr = 0, kc = 0;
  double* U = nullptr;  // n x kr row-major, the first kc columns hold U~
};

namespace pmor {

// ---------------------------------------------------------------------------
// device kernels
// ---------------------------------------------------------------------------
constexpr int GRAM_LDS = 32 * 1024;         // bytes of a row tile staged in LDS
constexpr int64_t GRAM_PART_MAX = 1 << 22;  // doubles of first-stage partial sums (at most)

// part[g][p] = sum over the rows of workgroup g of A[i, p / b] W[i, p % b];
// the rows go through LDS in tiles of tr rows (every thread loads several
// values of a tile before the barrier, which keeps many loads in flight)
template <int PPT>
__global__ __launch_bounds__(256) void k_gram_part(int64_t n, const double* __restrict__ A, int64_t lda, int a,
                                                   const double* __restrict__ W, int64_t ldw, int b, int64_t per,
                                                   int tr, double* __restrict__ part) {
  extern __shared__ double sh[];
  const int w = a + b, ab = a * b;
  double acc[PPT];
#pragma unroll
  for (int q = 0; q < PPT; ++q) acc[q] = 0.0;
  const int64_t r0 = (int64_t)blockIdx.x * per, r1 = min(n, r0 + per);
  for (int64_t base = r0; base < r1; base += tr) {
    const int nr = (int)min((int64_t)tr, r1 - base);
    __syncthreads();
    for (int t = threadIdx.x; t < tr * w; t += 256) {
      const int rr = t / w, cc = t - rr * w;
      double v = 0.0;
      if (rr < nr) v = cc < a ? A[(base + rr) * lda + cc] : W[(base + rr) * ldw + (cc - a)];
      sh[t] = v;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      const int p = threadIdx.x + q * 256;
      if (p < ab) {
        const int ia = p / b, ib = p - ia * b;
        double s = acc[q];
        for (int rr = 0; rr < nr; ++rr) s = fma(sh[rr * w + ia], sh[rr * w + a + ib], s);
        acc[q] = s;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int p = threadIdx.x + q * 256;
    if (p < ab) part[(int64_t)blockIdx.x * ab + p] = acc[q];
  }
}

// out[p] = sum_g part[g][p]: LPE lanes per p, lane l summing g = l, l + LPE,
// ... in order, then a fixed tree over the LPE lanes in LDS (the same order
// for the same G and ab).  Few outputs take many lanes each, so the partials
// of a small Gram product are read with many loads in flight.
template <int LPE>
__global__ __launch_bounds__(256) void k_gram_reduce(int G, int ab, const double* __restrict__ part,
                                                     double* __restrict__ out) {
  constexpr int EPB = 256 / LPE;
  __shared__ double sh[256];
  const int e = threadIdx.x / LPE, l = threadIdx.x - e * LPE;
  const int p = blockIdx.x * EPB + e;
  double s = 0.0;
  if (p < ab)
    for (int g = l; g < G; g += LPE) s += part[(int64_t)g * ab + p];
  sh[threadIdx.x] = s;
  __syncthreads();
#pragma unroll
  for (int o = LPE / 2; o >= 1; o >>= 1) {
    if (l < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (p < ab && l == 0) out[p] = sh[threadIdx.x];
}

// Y = beta Y + alpha A G (A: n x a, G: a x b row-major in LDS; beta 0 reads no Y)
__global__ __launch_bounds__(256) void k_tall_gemm(int64_t n, const double* __restrict__ A, int64_t lda, int a,
                                                   const double* __restrict__ G, int b, double alpha, double beta,
                                                   double* __restrict__ Y, int64_t ldy) {
  extern __shared__ double sg[];
  for (int t = threadIdx.x; t < a * b; t += 256) sg[t] = G[t];
  __syncthreads();
  const int rows = 256 / b;
  const int tr = threadIdx.x / b, c = threadIdx.x - tr * b;
  if (tr >= rows) return;
  const int64_t i = (int64_t)blockIdx.x * rows + tr;
  if (i >= n) return;
  const double* ar = A + i * lda;
  double s = 0.0;
  for (int t = 0; t < a; ++t) s = fma(ar[t], sg[t * b + c], s);
  double* y = Y + i * ldy + c;
  *y = beta == 0.0 ? alpha * s : fma(beta, *y, alpha * s);
}

__global__ void k_copy_cols(int64_t n, int w, const double* __restrict__ src, int64_t lds, double* __restrict__ dst,
                            int64_t ldd) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * w) return;
  const int64_t i = t / w;
  const int c = (int)(t - i * w);
  dst[i * ldd + c] = src[i * lds + c];
}

__global__ void k_add_cols(int64_t n, int w, const double* __restrict__ src, int64_t lds, double* __restrict__ dst,
                           int64_t ldd) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * w) return;
  const int64_t i = t / w;
  const int c = (int)(t - i * w);
  dst[i * ldd + c] += src[i * lds + c];
}

__global__ void k_zero_cols(int64_t n, int w, double* __restrict__ dst, int64_t ldd) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * w) return;
  const int64_t i = t / w;
  dst[i * ldd + (t - i * w)] = 0.0;
}

// ---------------------------------------------------------------------------
// host dense numerics (row-major unless stated)
// ---------------------------------------------------------------------------
namespace dense {

// A = L L^T for SPD A (n x n): the upper factor R = L^T into R; false when a
// pivot is not positive and finite
static bool chol_upper(int n, const double* A, double* R) {
  std::vector<double> L((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double d = A[j * n + j];
    for (int t = 0; t < j; ++t) d -= L[j * n + t] * L[j * n + t];
    if (!(d > 0.0) || !std::isfinite(d)) return false;
    const double l = std::sqrt(d);
    L[j * n + j] = l;
    for (int i = j + 1; i < n; ++i) {
      double s = A[i * n + j];
      for (int t = 0; t < j; ++t) s -= L[i * n + t] * L[j * n + t];
      L[i * n + j] = s / l;
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) R[i * n + j] = L[j * n + i];
  return true;
}

// inverse of an upper-triangular R (n x n) into Ri
static void inv_upper(int n, const double* R, double* Ri) {
  std::fill(Ri, Ri + (size_t)n * n, 0.0);
  for (int c = 0; c < n; ++c) {
    Ri[c * n + c] = 1.0 / R[c * n + c];
    for (int i = c - 1; i >= 0; --i) {
      double s = 0.0;
      for (int t = i + 1; t <= c; ++t) s += R[i * n + t] * Ri[t * n + c];
      Ri[i * n + c] = -s / R[i * n + i];
    }
  }
}

// C (m x n) = A (m x p) B (p x n)
static void matmul(int m, int p, int n, const double* A, const double* B, double* C) {
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int t = 0; t < p; ++t) s += A[i * p + t] * B[t * n + j];
      C[i * n + j] = s;
    }
}

// Householder reflector of x (len entries): H x = beta e_1, H = I - tau v v^T, v[0] = 1
static void house(int len, double* x, double* tau, double* beta) {
  const double alpha = x[0];
  double sigma = 0.0;
  for (int i = 1; i < len; ++i) sigma += x[i] * x[i];
  if (sigma == 0.0) {
    *tau = 0.0;
    *beta = alpha;
    x[0] = 1.0;
    return;
  }
  const double nrm = std::sqrt(alpha * alpha + sigma);
  const double b = alpha >= 0.0 ? -nrm : nrm;
  for (int i = 1; i < len; ++i) x[i] /= (alpha - b);
  x[0] = 1.0;
  *tau = (b - alpha) / b;
  *beta = b;
}

// thin QR with a positive diagonal: A (m x n, m >= n) = Q (m x n) R (n x n)
static bool qr_positive(int m, int n, const double* A, double* Q, double* R) {
  std::vector<double> W(A, A + (size_t)m * n), vs((size_t)n * m, 0.0), taus(n);
  for (int c = 0; c < n; ++c) {
    std::vector<double> x(m - c);
    for (int r = c; r < m; ++r) x[r - c] = W[r * n + c];
    double tau, beta;
    house(m - c, x.data(), &tau, &beta);
    for (int j = c + 1; j < n; ++j) {
      double s = 0.0;
      for (int r = c; r < m; ++r) s += x[r - c] * W[r * n + j];
      for (int r = c; r < m; ++r) W[r * n + j] -= tau * x[r - c] * s;
    }
    W[c * n + c] = beta;
    for (int r = c + 1; r < m; ++r) W[r * n + c] = 0.0;
    for (int r = c; r < m; ++r) vs[(size_t)c * m + r] = x[r - c];
    taus[c] = tau;
  }
  // Q = H_0 ... H_{n-1} applied to the first n columns of the identity
  std::fill(Q, Q + (size_t)m * n, 0.0);
  for (int c = 0; c < n; ++c) Q[c * n + c] = 1.0;
  for (int c = n - 1; c >= 0; --c)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int r = c; r < m; ++r) s += vs[(size_t)c * m + r] * Q[r * n + j];
      for (int r = c; r < m; ++r) Q[r * n + j] -= taus[c] * vs[(size_t)c * m + r] * s;
    }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) R[i * n + j] = j >= i ? W[i * n + j] : 0.0;
  for (int c = 0; c < n; ++c) {
    if (!std::isfinite(R[c * n + c]) || R[c * n + c] == 0.0) return false;
    if (R[c * n + c] < 0.0) {
      for (int j = 0; j < n; ++j) R[c * n + j] = -R[c * n + j];
      for (int r = 0; r < m; ++r) Q[r * n + c] = -Q[r * n + c];
    }
  }
  return true;
}

// Least squares min ||E_1 S - Hbar_j y|| of block GMRES, by Householder QR of
// the block Hessenberg matrix grown one block column at a time.  Storage is
// column-major with leading dimension N = (m + 1) k.
struct HessLS {
  int k = 0, m = 0, N = 0;
  std::vector<double> R, g, v, tau;
  void init(int k_, int m_, const double* S) {  // S: k x k row-major
    k = k_;
    m = m_;
    N = (m + 1) * k;
    R.assign((size_t)N * m * k, 0.0);
    g.assign((size_t)N * k, 0.0);
    v.assign((size_t)m * k * (k + 1), 0.0);
    tau.assign((size_t)m * k, 0.0);
    for (int r = 0; r < k; ++r)
      for (int c = 0; c < k; ++c) g[(size_t)c * N + r] = S[r * k + c];
  }
  void apply(int cr, double* x) const {  // reflector of column cr to a column x (length N)
    const double* vv = &v[(size_t)cr * (k + 1)];
    double s = 0.0;
    for (int i = 0; i <= k; ++i) s += vv[i] * x[cr + i];
    s *= tau[cr];
    for (int i = 0; i <= k; ++i) x[cr + i] -= s * vv[i];
  }
  // block column j of Hbar: H ((j + 2) k rows x k, row-major)
  void add(int j, const double* H) {
    const int rows = (j + 2) * k;
    for (int t = 0; t < k; ++t) {
      double* col = &R[(size_t)(j * k + t) * N];
      for (int r = 0; r < N; ++r) col[r] = r < rows ? H[r * k + t] : 0.0;
      for (int c = 0; c < j * k; ++c) apply(c, col);
    }
    for (int t = 0; t < k; ++t) {
      const int c = j * k + t;
      double* col = &R[(size_t)c * N];
      double x[PMOR_KMAX + 1];
      for (int i = 0; i <= k; ++i) x[i] = col[c + i];
      double tt, beta;
      house(k + 1, x, &tt, &beta);
      for (int i = 0; i <= k; ++i) v[(size_t)c * (k + 1) + i] = x[i];
      tau[c] = tt;
      col[c] = beta;
      for (int i = 1; i <= k; ++i) col[c + i] = 0.0;
      for (int u = t + 1; u < k; ++u) apply(c, &R[(size_t)(j * k + u) * N]);
      for (int u = 0; u < k; ++u) apply(c, &g[(size_t)u * N]);
    }
  }
  double resid(int j, int c) const {  // least-squares residual of column c after block column j
    double s = 0.0;
    for (int r = (j + 1) * k; r < (j + 2) * k; ++r) s += g[(size_t)c * N + r] * g[(size_t)c * N + r];
    return std::sqrt(s);
  }
  void solve(int jd, double* y) const {  // y: jd k x k row-major
    const int n = jd * k;
    for (int c = 0; c < k; ++c)
      for (int i = n - 1; i >= 0; --i) {
        double s = g[(size_t)c * N + i];
        for (int t = i + 1; t < n; ++t) s -= R[(size_t)t * N + i] * y[t * k + c];
        y[i * k + c] = s / R[(size_t)i * N + i];
      }
  }
};

using cd = std::complex<double>;

// Eigenvalues of an upper Hessenberg matrix H (n x n, row-major, destroyed)
// by the Francis double-shift QR iteration in real arithmetic: a 3 x 3
// Householder bulge is chased down the active window [l, hi], which shrinks as
// subdiagonal entries become negligible; 1 x 1 and 2 x 2 diagonal blocks give
// the eigenvalues (a conjugate pair as wr +- i wi, a real one with wi = 0).
// Only the window is updated (no Schur vectors).  False when it does not
// converge.
static bool hess_eig(int n, double* H, double* wr, double* wi) {
  auto h = [&](int r, int c) -> double& { return H[(size_t)r * n + c]; };
  double nrm = 0.0;
  for (int r = 0; r < n; ++r)
    for (int c = std::max(0, r - 1); c < n; ++c) nrm += std::fabs(h(r, c));
  const double eps = 2.220446049250313e-16;
  int hi = n - 1, iter = 0;
  while (hi >= 0) {
    int l = hi;
    for (; l > 0; --l) {
      double s = std::fabs(h(l - 1, l - 1)) + std::fabs(h(l, l));
      if (s == 0.0) s = nrm;
      if (std::fabs(h(l, l - 1)) <= eps * s) {
        h(l, l - 1) = 0.0;
        break;
      }
    }
    if (l == hi) {  // a 1 x 1 block
      wr[hi] = h(hi, hi);
      wi[hi] = 0.0;
      --hi;
      iter = 0;
      continue;
    }
    if (l == hi - 1) {  // a 2 x 2 block
      const double a = h(hi - 1, hi - 1), b = h(hi - 1, hi), c = h(hi, hi - 1), d = h(hi, hi);
      const double p = 0.5 * (a - d), q = p * p + b * c;
      if (q >= 0.0) {
        const double z = p + std::copysign(std::sqrt(q), p);
        wr[hi - 1] = d + z;
        wr[hi] = z != 0.0 ? d - b * c / z : d + z;
        wi[hi - 1] = wi[hi] = 0.0;
      } else {
        wr[hi - 1] = wr[hi] = d + p;
        wi[hi - 1] = std::sqrt(-q);
        wi[hi] = -wi[hi - 1];
      }
      hi -= 2;
      iter = 0;
      continue;
    }
    if (++iter > 40 * n) return false;
    // the double shift: the trailing 2 x 2 block's eigenvalues (sum s, product
    // t), or an exceptional shift after 10 and 20 iterations without deflation
    double s = h(hi - 1, hi - 1) + h(hi, hi);
    double t = h(hi - 1, hi - 1) * h(hi, hi) - h(hi - 1, hi) * h(hi, hi - 1);
    if (iter % 10 == 0) {
      const double x = std::fabs(h(hi, hi - 1)) + std::fabs(h(hi - 1, hi - 2));
      s = 1.5 * x + h(hi, hi);
      t = x * x;
    }
    // first column of (H - s1)(H - s2) in the window
    double x = h(l, l) * h(l, l) + h(l, l + 1) * h(l + 1, l) - s * h(l, l) + t;
    double y = h(l + 1, l) * (h(l, l) + h(l + 1, l + 1) - s);
    double z = h(l + 1, l) * h(l + 2, l + 1);
    for (int k = l; k <= hi - 1; ++k) {
      const int len = k < hi - 1 ? 3 : 2;
      double v[3] = {x, y, len == 3 ? z : 0.0};
      double tau, beta;
      house(len, v, &tau, &beta);
      if (tau != 0.0) {
        const int c0 = std::max(l, k - 1);
        for (int c = c0; c <= hi; ++c) {  // rows k..k+len-1 from the left
          double sm = 0.0;
          for (int i = 0; i < len; ++i) sm += v[i] * h(k + i, c);
          sm *= tau;
          for (int i = 0; i < len; ++i) h(k + i, c) -= sm * v[i];
        }
        const int r1 = std::min(k + 3, hi);
        for (int r = l; r <= r1; ++r) {  // columns k..k+len-1 from the right
          double sm = 0.0;
          for (int i = 0; i < len; ++i) sm += h(r, k + i) * v[i];
          sm *= tau;
          for (int i = 0; i < len; ++i) h(r, k + i) -= sm * v[i];
        }
      }
      if (k > l) {  // the bulge below the subdiagonal is gone
        h(k + 1, k - 1) = 0.0;
        if (len == 3) h(k + 2, k - 1) = 0.0;
      }
      if (k < hi - 1) {
        x = h(k + 1, k);
        y = h(k + 2, k);
        z = k < hi - 2 ? h(k + 3, k) : 0.0;
      }
    }
  }
  return true;
}

using cd = std::complex<double>;

// An eigenvector of the upper Hessenberg H (n x n, row-major) for the
// eigenvalue mu by inverse iteration: (H - sigma I) x = b twice, sigma = mu
// moved by a relative 1e-10 so that the factor is not exactly singular, LU
// with partial pivoting between neighbouring rows (the Hessenberg form keeps
// the factor's work O(n^2)); b a fixed start vector depending on seed.
static void hess_invit(int n, const double* H, cd mu, int seed, std::vector<cd>& x) {
  double hn = 0.0;
  for (int r = 0; r < n; ++r)
    for (int c = std::max(0, r - 1); c < n; ++c) hn = std::max(hn, std::fabs(H[(size_t)r * n + c]));
  const cd sigma = mu + cd(1e-10 * std::max(hn, 1e-300), 0.0);
  std::vector<cd> U((size_t)n * n);
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) U[(size_t)r * n + c] = (c >= r - 1) ? cd(H[(size_t)r * n + c]) : cd(0.0);
  for (int i = 0; i < n; ++i) U[(size_t)i * n + i] -= sigma;
  std::vector<cd> mult(n, cd(0.0));
  std::vector<char> swp(n, 0);
  const double tiny = 2.220446049250313e-16 * std::max(hn, 1e-300);
  for (int c = 0; c + 1 < n; ++c) {
    cd* r0 = &U[(size_t)c * n];
    cd* r1 = &U[(size_t)(c + 1) * n];
    if (std::abs(r1[c]) > std::abs(r0[c])) {
      for (int j = c; j < n; ++j) std::swap(r0[j], r1[j]);
      swp[c] = 1;
    }
    if (std::abs(r0[c]) < tiny) r0[c] = tiny;
    const cd m = r1[c] / r0[c];
    mult[c] = m;
    r1[c] = 0.0;
    for (int j = c + 1; j < n; ++j) r1[j] -= m * r0[j];
  }
  if (std::abs(U[(size_t)(n - 1) * n + n - 1]) < tiny) U[(size_t)(n - 1) * n + n - 1] = tiny;
  x.assign(n, cd(0.0));
  for (int i = 0; i < n; ++i) x[i] = 1.0 + 0.25 * ((i * 7919 + seed * 104729) % 101) / 101.0;
  for (int it = 0; it < 2; ++it) {
    for (int c = 0; c + 1 < n; ++c) {  // the row operations on the right-hand side
      if (swp[c]) std::swap(x[c], x[c + 1]);
      x[c + 1] -= mult[c] * x[c];
    }
    for (int i = n - 1; i >= 0; --i) {
      cd sm = x[i];
      for (int j = i + 1; j < n; ++j) sm -= U[(size_t)i * n + j] * x[j];
      x[i] = sm / U[(size_t)i * n + i];
    }
    double nz = 0.0;
    for (const cd& v : x) nz += std::norm(v);
    nz = std::sqrt(nz);
    for (cd& v : x) v /= nz;
  }
}

// The harmonic Ritz selection: eigenpairs of G^T WtV z = mu G^T G z (G, WtV:
// rows x N row-major) by decreasing |mu|; a real mu (|Im mu| <= 1e-10 max|mu|)
// gives Re z of z scaled to unit norm with its largest entry real and positive,
// a conjugate pair gives Re z, Im z of its member with Im mu > 0, and a pair
// that does not fit in what is left of kr ends the selection.  Pk: N x kr
// row-major (the first returned count of columns used); mu_re/mu_im (may be
// NULL) the selected values.  Returns the count, or -1 when G^T G is not
// positive definite or the iteration fails.  Steps: M = (G^T G)^{-1} G^T WtV by
// Cholesky, M = Qh Hh Qh^T (Householder), the eigenvalues of Hh by the Francis
// iteration, the chosen eigenvectors by inverse iteration on Hh, z = Qh x.
static int harmonic_select(int rows, int N, const double* G, const double* WtV, int kr, double* Pk, double* mu_re,
                           double* mu_im) {
  if (kr <= 0 || N <= 0) return 0;
  std::vector<double> A1((size_t)N * N, 0.0), A2((size_t)N * N, 0.0), Rc((size_t)N * N);
  for (int r = 0; r < rows; ++r) {  // row by row: contiguous accesses
    const double* g = G + (size_t)r * N;
    const double* w = WtV + (size_t)r * N;
    for (int i = 0; i < N; ++i) {
      const double gi = g[i];
      if (gi == 0.0) continue;
      double* a1 = &A1[(size_t)i * N];
      double* a2 = &A2[(size_t)i * N];
      for (int j = 0; j < N; ++j) {
        a1[j] += gi * g[j];
        a2[j] += gi * w[j];
      }
    }
  }
  if (!chol_upper(N, A1.data(), Rc.data())) return -1;
  // M = R^{-1} R^{-T} A2, all columns at once: forward (R^T Y = A2) then back (R M = Y)
  std::vector<double> M(A2);
  for (int i = 0; i < N; ++i) {
    double* mi = &M[(size_t)i * N];
    for (int t = 0; t < i; ++t) {
      const double rti = Rc[(size_t)t * N + i];
      if (rti == 0.0) continue;
      const double* mt = &M[(size_t)t * N];
      for (int c = 0; c < N; ++c) mi[c] -= rti * mt[c];
    }
    const double d = 1.0 / Rc[(size_t)i * N + i];
    for (int c = 0; c < N; ++c) mi[c] *= d;
  }
  for (int i = N - 1; i >= 0; --i) {
    double* mi = &M[(size_t)i * N];
    for (int t = i + 1; t < N; ++t) {
      const double rit = Rc[(size_t)i * N + t];
      if (rit == 0.0) continue;
      const double* mt = &M[(size_t)t * N];
      for (int c = 0; c < N; ++c) mi[c] -= rit * mt[c];
    }
    const double d = 1.0 / Rc[(size_t)i * N + i];
    for (int c = 0; c < N; ++c) mi[c] *= d;
  }
  // Hessenberg form M = Qh Hh Qh^T by Householder reflections
  std::vector<double> Hh(M), Qh((size_t)N * N, 0.0), tmp(N);
  for (int i = 0; i < N; ++i) Qh[(size_t)i * N + i] = 1.0;
  for (int c = 0; c + 2 < N; ++c) {
    const int len = N - c - 1;
    std::vector<double> x(len);
    for (int r = 0; r < len; ++r) x[r] = Hh[(size_t)(c + 1 + r) * N + c];
    double tau, beta;
    house(len, x.data(), &tau, &beta);
    if (tau == 0.0) continue;
    // rows c+1.. : H <- (I - tau v v^T) H, by rows (contiguous)
    std::fill(tmp.begin(), tmp.end(), 0.0);
    for (int r = 0; r < len; ++r) {
      const double* hr = &Hh[(size_t)(c + 1 + r) * N];
      for (int j = 0; j < N; ++j) tmp[j] += x[r] * hr[j];
    }
    for (int r = 0; r < len; ++r) {
      double* hr = &Hh[(size_t)(c + 1 + r) * N];
      const double f = tau * x[r];
      for (int j = 0; j < N; ++j) hr[j] -= f * tmp[j];
    }
    // columns c+1.. : H <- H (I - tau v v^T) and Q <- Q (I - tau v v^T)
    for (int i = 0; i < N; ++i) {
      double* hr = &Hh[(size_t)i * N + c + 1];
      double* qr = &Qh[(size_t)i * N + c + 1];
      double sh = 0.0, sq = 0.0;
      for (int r = 0; r < len; ++r) {
        sh += hr[r] * x[r];
        sq += qr[r] * x[r];
      }
      sh *= tau;
      sq *= tau;
      for (int r = 0; r < len; ++r) {
        hr[r] -= sh * x[r];
        qr[r] -= sq * x[r];
      }
    }
    for (int r = c + 2; r < N; ++r) Hh[(size_t)r * N + c] = 0.0;
  }
  std::vector<double> W(Hh), wr(N), wi(N);
  if (!hess_eig(N, W.data(), wr.data(), wi.data())) return -1;
  std::vector<cd> mu(N);
  double mmax = 0.0;
  for (int i = 0; i < N; ++i) {
    mu[i] = cd(wr[i], wi[i]);
    mmax = std::max(mmax, std::abs(mu[i]));
  }
  const double thr = 1e-10 * mmax;
  auto eigvec = [&](int i, int seed, std::vector<cd>& z) {
    std::vector<cd> x;
    hess_invit(N, Hh.data(), mu[i], seed, x);
    z.assign(N, cd(0.0));
    for (int r = 0; r < N; ++r) {
      const double* q = &Qh[(size_t)r * N];
      cd sm = 0.0;
      for (int t = 0; t < N; ++t) sm += q[t] * x[t];
      z[r] = sm;
    }
    double nz = 0.0;
    for (const cd& v : z) nz += std::norm(v);
    nz = std::sqrt(nz);
    for (cd& v : z) v /= nz;
  };
  std::vector<int> order(N);
  for (int i = 0; i < N; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return std::abs(mu[a]) > std::abs(mu[b]); });
  std::vector<char> used(N, 0);
  int cnt = 0;
  std::vector<cd> z;
  for (int oi = 0; oi < N && cnt < kr; ++oi) {
    const int i = order[oi];
    if (used[i]) continue;
    if (std::abs(mu[i].imag()) <= thr) {
      mu[i] = cd(mu[i].real(), 0.0);
      eigvec(i, cnt, z);
      int tm = 0;
      for (int r = 1; r < N; ++r)
        if (std::abs(z[r]) > std::abs(z[tm])) tm = r;
      const cd ph = std::conj(z[tm]) / std::abs(z[tm]);
      for (int r = 0; r < N; ++r) Pk[(size_t)r * kr + cnt] = (z[r] * ph).real();
      if (mu_re) mu_re[cnt] = mu[i].real();
      if (mu_im) mu_im[cnt] = 0.0;
      used[i] = 1;
      ++cnt;
      continue;
    }
    int j = -1;
    for (int oj = 0; oj < N; ++oj) {
      const int t = order[oj];
      if (used[t] || t == i) continue;
      if (j < 0 || std::abs(mu[t] - std::conj(mu[i])) < std::abs(mu[j] - std::conj(mu[i]))) j = t;
    }
    if (j < 0 || cnt + 2 > kr) break;
    eigvec(mu[i].imag() > 0.0 ? i : j, cnt, z);
    for (int r = 0; r < N; ++r) {
      Pk[(size_t)r * kr + cnt] = z[r].real();
      Pk[(size_t)r * kr + cnt + 1] = z[r].imag();
    }
    if (mu_re) {
      mu_re[cnt] = mu[i].real();
      mu_re[cnt + 1] = mu[j].real();
    }
    if (mu_im) {
      mu_im[cnt] = mu[i].imag();
      mu_im[cnt + 1] = mu[j].imag();
    }
    used[i] = used[j] = 1;
    cnt += 2;
  }
  return cnt;
}

}  // namespace dense

// ---------------------------------------------------------------------------
// the solver
// ---------------------------------------------------------------------------
namespace {

struct Work {
  pmor_ctx* ctx = nullptr;
  hipStream_t st = nullptr;
  int64_t n = 0;
  int k = 0, m = 0, kr = 0;
  int64_t LB = 0;                 // columns of the basis buffer: kr + (m + 1) k
  double* Bs = nullptr;           // n x LB: C at columns [kr - kc, kr), V_j at [kr + j k, kr + (j + 1) k)
  double* U = nullptr;            // n x max(kr, 1): U in its first kc columns
  double *Wt = nullptr, *Z = nullptr, *Z2 = nullptr, *tC = nullptr, *tU = nullptr;
  double* part = nullptr;         // first-stage partial sums of the Gram products
  double* dsm = nullptr;          // device small matrices: SLOTS x slot
  double* hsm = nullptr;          // pinned: SLOTS x slot
  int64_t slot = 0;
  static constexpr int SLOTS = 8;
  bool pend[SLOTS] = {};          // an upload from the slot's pinned buffer may still be in flight
  std::vector<void*> dev;
  ~Work() {
    for (void* p : dev) dfree(p, st);
    if (hsm) (void)hipHostFree(hsm);
  }
  double* ds(int i) { return dsm + (int64_t)i * slot; }
  double* hs(int i) { return hsm + (int64_t)i * slot; }
  double* V(int j) { return Bs + kr + (int64_t)j * k; }
};

int alloc(Work& w) {
  auto al = [&](double** p, int64_t cnt) {
    if (dmalloc((void**)p, sizeof(double) * std::max<int64_t>(cnt, 1), w.st) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    w.dev.push_back(*p);
    return true;
  };
  const int64_t krp = std::max(w.kr, 1), wmax = std::max(w.k, w.kr);
  w.slot = w.LB * wmax + 64;
  const bool ok = al(&w.Bs, w.n * w.LB) && al(&w.U, w.n * krp) && al(&w.Wt, w.n * w.k) && al(&w.Z, w.n * w.k) &&
                  al(&w.Z2, w.n * w.k) && al(&w.tC, w.n * krp) && al(&w.tU, w.n * krp) &&
                  al(&w.part, std::min<int64_t>(GRAM_PART_MAX, 1024 * w.LB * wmax)) &&
                  al(&w.dsm, Work::SLOTS * w.slot);
  if (!ok) return fail(PMOR_ENOMEM, "allocation of the recycling solver's buffers failed");
  if (hipHostMalloc((void**)&w.hsm, sizeof(double) * Work::SLOTS * w.slot, hipHostMallocDefault) != hipSuccess) {
    w.hsm = nullptr;
    (void)hipGetLastError();
    return fail(PMOR_ENOMEM, "pinned host allocation failed");
  }
  return PMOR_OK;
}

// out (a x b, device) = A^T W over n rows
// workgroups of a Gram product with ab outputs: about one per 256 rows, at
// most 1024, and at most GRAM_PART_MAX partial sums
int gram_groups(int64_t n, int ab) {
  int64_t G = std::min<int64_t>(1024, (n + 255) / 256);
  G = std::min<int64_t>(G, std::max<int64_t>(1, GRAM_PART_MAX / std::max(ab, 1)));
  return (int)std::max<int64_t>(G, 1);
}

int gram(Work& w, const double* A, int64_t lda, int a, const double* W, int64_t ldw, int b, double* out) {
  const int ab = a * b;
  if (ab == 0) return PMOR_OK;
  const int G = gram_groups(w.n, ab);
  const int64_t per = (w.n + G - 1) / G;
  const int tr = std::max(1, std::min(64, GRAM_LDS / (int)(sizeof(double) * (a + b))));
  const size_t lds = sizeof(double) * (size_t)tr * (a + b);
  const int ppt = (ab + 255) / 256;
  if (ppt > 36) return fail(PMOR_EINVAL, "Gram product too wide");
  const int pr = prof_start(w.ctx, PMOR_PROF_GCRO_GRAM);
  if (ppt <= 2) {
    plaunch(w.ctx, pr, 3, k_gram_part<2>, dim3(G), dim3(256), lds, w.st, w.n, A, lda, a, W, ldw, b, per, tr, w.part);
  } else if (ppt <= 8) {
    plaunch(w.ctx, pr, 3, k_gram_part<8>, dim3(G), dim3(256), lds, w.st, w.n, A, lda, a, W, ldw, b, per, tr, w.part);
  } else {
    plaunch(w.ctx, pr, 3, k_gram_part<36>, dim3(G), dim3(256), lds, w.st, w.n, A, lda, a, W, ldw, b, per, tr,
            w.part);
  }
  PMOR_HIP(hipGetLastError());
  // algorithmic bytes: the n rows of A's a and W's b columns (W among A's columns is read once)
  const bool w_in_a = lda == ldw && W >= A && W + b <= A + a;
  prof_stop(w.ctx, pr, 8.0 * w.n * (w_in_a ? a : a + b), 0);
  if (ab <= 64) {
    hipLaunchKernelGGL(k_gram_reduce<256>, dim3((unsigned)ab), dim3(256), 0, w.st, G, ab, w.part, out);
  } else if (ab <= 1024) {
    hipLaunchKernelGGL(k_gram_reduce<64>, dim3((unsigned)((ab + 3) / 4)), dim3(256), 0, w.st, G, ab, w.part, out);
  } else {
    hipLaunchKernelGGL(k_gram_reduce<16>, dim3((unsigned)((ab + 15) / 16)), dim3(256), 0, w.st, G, ab, w.part, out);
  }
  PMOR_HIP(hipGetLastError());
  return PMOR_OK;
}

// Y = beta Y + alpha A G (G: a x b on the device)
int tall_gemm(Work& w, const double* A, int64_t lda, int a, const double* G, int b, double alpha, double beta, double* Y,
              int64_t ldy) {
  if (b == 0) return PMOR_OK;
  if (a == 0) {
    if (beta == 0.0) {
      const int64_t tot = w.n * b;
      hipLaunchKernelGGL(k_zero_cols, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, w.st, w.n, b, Y, ldy);
      PMOR_HIP(hipGetLastError());
    }
    return PMOR_OK;
  }
  const int rows = 256 / b;
  const size_t lds = sizeof(double) * (size_t)a * b;
  if (lds > 64 * 1024) PMOR_TRY(allow_lds(reinterpret_cast<const void*>(k_tall_gemm), lds));  // per device, per call
  const int pr = prof_start(w.ctx, PMOR_PROF_GCRO_GEMM);
  plaunch(w.ctx, pr, 3, k_tall_gemm, dim3((unsigned)((w.n + rows - 1) / rows)), dim3(256), lds, w.st, w.n, A, lda, a,
          G, b, alpha, beta, Y, ldy);
  PMOR_HIP(hipGetLastError());
  prof_stop(w.ctx, pr, 8.0 * w.n * (a + b + (beta != 0.0 ? b : 0)), 0);
  return PMOR_OK;
}

int copy_cols(Work& w, const double* src, int64_t lds, double* dst, int64_t ldd, int cols) {
  const int64_t tot = w.n * cols;
  if (tot == 0) return PMOR_OK;
  hipLaunchKernelGGL(k_copy_cols, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, w.st, w.n, cols, src, lds, dst,
                     ldd);
  PMOR_HIP(hipGetLastError());
  return PMOR_OK;
}

int down(Work& w, int s, const double* dev, int64_t cnt) {
  PMOR_HIP(hipMemcpyAsync(w.hs(s), dev, sizeof(double) * cnt, hipMemcpyDeviceToHost, w.st));
  return PMOR_OK;
}
int sync(Work& w) {
  PMOR_HIP(hipStreamSynchronize(w.st));
  for (bool& p : w.pend) p = false;
  return PMOR_OK;
}
// small matrix to the device through the slot's pinned buffer (which is not
// rewritten while an earlier upload from it may still be in flight)
int up(Work& w, int s, const double* host, int64_t cnt) {
  if (w.pend[s]) PMOR_TRY(sync(w));
  std::memcpy(w.hs(s), host, sizeof(double) * cnt);
  PMOR_HIP(hipMemcpyAsync(w.ds(s), w.hs(s), sizeof(double) * cnt, hipMemcpyHostToDevice, w.st));
  w.pend[s] = true;
  return PMOR_OK;
}

// the operator pieces: Y = A X, Y = P X (k columns, leading dimensions)
struct Ops {
  pmor_problem* pb;
  const pmor_spai* h;
  int apply_A(Work& w, const double* X, int64_t ldx, double* Y, int64_t ldy, int k, double alpha, double beta,
              const double* Bsrc, int64_t ldb) const {
    return launch_spmm(pb->n, pb->rowptr, pb->col, pb->aval, X, ldx, Y, ldy, k, alpha, beta, Bsrc, ldb, w.st, pb->ctx,
                       -1, 3);
  }
  // Y = alpha P X + beta Bsrc; without a preconditioner P = I
  int apply_P(Work& w, const double* X, int64_t ldx, double* Y, int64_t ldy, int k, double alpha, double beta,
              const double* Bsrc, int64_t ldb) const {
    if (!h) {
      if (beta != 0.0 || alpha != 1.0) {  // Y = alpha X + beta Bsrc through the identity's CSR-free path
        return fail(PMOR_EINVAL, "internal: identity preconditioner with scaling");
      }
      return copy_cols(w, X, ldx, Y, ldy, k);
    }
    if (h->q_active) {  // P = Q P_1
      PMOR_TRY(launch_spmm(pb->n, h->Prowptr, h->Pcol, h->P1val, X, ldx, w.Z2, k, k, 1.0, 0.0, nullptr, 0, w.st,
                           pb->ctx, -1, 3));
      return launch_spmm(pb->n, h->Prowptr, h->Pcol, h->Qval, w.Z2, k, Y, ldy, k, alpha, beta, Bsrc, ldb, w.st,
                         pb->ctx, -1, 3);
    }
    return launch_spmm(pb->n, h->Prowptr, h->Pcol, h->Pval, X, ldx, Y, ldy, k, alpha, beta, Bsrc, ldb, w.st, pb->ctx,
                       -1, 3);
  }
  // X += P Y (Y: n x k in Z)
  int add_P(Work& w, const double* Y, int64_t ldy, double* X, int64_t ldx, int k) const {
    if (!h) {  // X += Y
      const int64_t tot = w.n * k;
      hipLaunchKernelGGL(k_add_cols, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, w.st, w.n, k, Y, ldy, X, ldx);
      PMOR_HIP(hipGetLastError());
      return PMOR_OK;
    }
    return apply_P(w, Y, ldy, X, ldx, k, 1.0, 1.0, X, ldx);
  }
};

// Cholesky QR twice of Ain (n x c) into Out (Out != Ain): Out = Ain R^{-1},
// R (c x c, host) upper with a positive diagonal; g0 (host, c x c) the Gram
// matrix of Ain when already known.  ok = false when a Cholesky pivot fails.
int cholqr2(Work& w, const double* Ain, int64_t lda, int c, double* Out, int64_t ldo, const double* g0,
            std::vector<double>& R, bool* ok) {
  *ok = false;
  std::vector<double> G((size_t)c * c), R1((size_t)c * c), R1i((size_t)c * c), R2((size_t)c * c),
      R2i((size_t)c * c), Ri((size_t)c * c);
  if (g0) {
    std::memcpy(G.data(), g0, sizeof(double) * c * c);
  } else {
    PMOR_TRY(gram(w, Ain, lda, c, Ain, lda, c, w.ds(0)));
    PMOR_TRY(down(w, 0, w.ds(0), (int64_t)c * c));
    PMOR_TRY(sync(w));
    std::memcpy(G.data(), w.hs(0), sizeof(double) * c * c);
  }
  if (!dense::chol_upper(c, G.data(), R1.data())) return PMOR_OK;
  dense::inv_upper(c, R1.data(), R1i.data());
  PMOR_TRY(up(w, 1, R1i.data(), (int64_t)c * c));
  PMOR_TRY(tall_gemm(w, Ain, lda, c, w.ds(1), c, 1.0, 0.0, Out, ldo));
  PMOR_TRY(gram(w, Out, ldo, c, Out, ldo, c, w.ds(0)));
  PMOR_TRY(down(w, 0, w.ds(0), (int64_t)c * c));
  PMOR_TRY(sync(w));
  std::memcpy(G.data(), w.hs(0), sizeof(double) * c * c);
  if (!dense::chol_upper(c, G.data(), R2.data())) return PMOR_OK;
  dense::inv_upper(c, R2.data(), R2i.data());
  R.assign((size_t)c * c, 0.0);
  dense::matmul(c, c, c, R2.data(), R1.data(), R.data());
  dense::matmul(c, c, c, R1i.data(), R2i.data(), Ri.data());
  PMOR_TRY(up(w, 2, Ri.data(), (int64_t)c * c));
  PMOR_TRY(tall_gemm(w, Ain, lda, c, w.ds(2), c, 1.0, 0.0, Out, ldo));
  *ok = true;
  return PMOR_OK;
}

}  // namespace

int gcrodr_solve(pmor_problem* pb, const pmor_spai* h, const Point& pt, const double* B, int64_t ldb, int k, double* X,
                 int64_t ldx, const pmor_solve_opts& o, pmor_recycle* rec, pmor_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  PMOR_TRY(ensure_assembled(pb, pt));
  Work w;
  w.ctx = pb->ctx;
  w.st = pb->ctx->stream;
  w.n = pb->n;
  w.k = k;
  w.m = o.m;
  w.kr = rec->kr;
  w.LB = w.kr + (int64_t)(w.m + 1) * k;
  PMOR_TRY(alloc(w));
  Ops op{pb, h};
  const int kr = w.kr, m = w.m;
  const int64_t LB = w.LB;
  if (stats) {
    stats->k = k;
    stats->cycles = 0;
    stats->steps = 0;
    stats->bad_column = -1;
    std::memset(stats->cycle_steps, 0, sizeof(stats->cycle_steps));
    for (int c = 0; c < PMOR_KMAX; ++c) stats->relres[c] = 0.0;
  }
  // ||b_c||
  std::vector<double> bnorm(k);
  {
    PMOR_TRY(gram(w, B, ldb, k, B, ldb, k, w.ds(0)));
    PMOR_TRY(down(w, 0, w.ds(0), (int64_t)k * k));
    PMOR_TRY(sync(w));
    for (int c = 0; c < k; ++c) {
      bnorm[c] = std::sqrt(w.hs(0)[c * k + c]);
      if (!(bnorm[c] > 0.0) || !std::isfinite(bnorm[c]))
        return fail(bnorm[c] == 0.0 ? PMOR_EINVAL : PMOR_ENAN,
                    "right-hand side column " + std::to_string(c) + " is zero or not finite (block GCRO-DR)");
    }
  }
  PMOR_TRY(tall_gemm(w, X, ldx, 0, nullptr, k, 1.0, 0.0, X, ldx));  // X = 0
  // entering the system: C = Op U~, C = Q R, U = U~ R^{-1}
  int kc = 0;
  if (rec->kc > 0) {
    const int c0 = rec->kc;
    PMOR_TRY(op.apply_P(w, rec->U, kr, w.tU, kr, c0, 1.0, 0.0, nullptr, 0));
    PMOR_TRY(op.apply_A(w, w.tU, kr, w.tC, kr, c0, 1.0, 0.0, nullptr, 0));
    std::vector<double> R;
    bool ok = false;
    PMOR_TRY(cholqr2(w, w.tC, kr, c0, w.Bs + (kr - c0), LB, nullptr, R, &ok));
    if (ok) {
      std::vector<double> Ri((size_t)c0 * c0);
      dense::inv_upper(c0, R.data(), Ri.data());
      PMOR_TRY(up(w, 3, Ri.data(), (int64_t)c0 * c0));
      PMOR_TRY(tall_gemm(w, rec->U, kr, c0, w.ds(3), c0, 1.0, 0.0, w.U, kr));
      kc = c0;
    }
  }
  std::vector<double> hc((size_t)(kr + (m + 1) * k) * k), Bm((size_t)std::max(kr, 1) * m * k),
      Hbar((size_t)(m + 1) * k * m * k);
  dense::HessLS ls;
  int status = PMOR_ENOTCONV, cycle = 0;
  std::vector<double> rel(k, 0.0);
  for (;; ++cycle) {
    // residual into Wt, projected on C
    PMOR_TRY(op.apply_A(w, X, ldx, w.Wt, k, k, -1.0, 1.0, B, ldb));
    if (kc > 0) {
      double* C = w.Bs + (kr - kc);
      PMOR_TRY(gram(w, C, LB, kc, w.Wt, k, k, w.ds(4)));
      PMOR_TRY(tall_gemm(w, C, LB, kc, w.ds(4), k, -1.0, 1.0, w.Wt, k));
      PMOR_TRY(tall_gemm(w, w.U, kr, kc, w.ds(4), k, 1.0, 0.0, w.Z, k));
      PMOR_TRY(op.add_P(w, w.Z, k, X, ldx, k));
    }
    PMOR_TRY(gram(w, w.Wt, k, k, w.Wt, k, k, w.ds(0)));
    PMOR_TRY(down(w, 0, w.ds(0), (int64_t)k * k));
    PMOR_TRY(sync(w));
    std::vector<double> g0(w.hs(0), w.hs(0) + (size_t)k * k);
    bool fin = true, conv = true;
    for (int c = 0; c < k; ++c) {
      rel[c] = std::sqrt(std::max(g0[c * k + c], 0.0)) / bnorm[c];
      fin = fin && std::isfinite(rel[c]);
      conv = conv && rel[c] <= o.tol;
    }
    if (!fin) {
      status = PMOR_ENAN;
      break;
    }
    if (conv) {
      status = PMOR_OK;
      break;
    }
    if (cycle == o.max_cycles) break;
    std::vector<double> S;
    bool ok = false;
    PMOR_TRY(cholqr2(w, w.Wt, k, k, w.V(0), LB, g0.data(), S, &ok));
    bool dep = !ok;
    for (int c = 0; ok && c < k; ++c)
      if (!(S[c * k + c] > kDepSine * std::sqrt(g0[c * k + c]))) dep = true;
    if (dep) {
      status = PMOR_EBREAKDOWN;
      if (stats && cycle < PMOR_MAX_CYCLES) stats->cycle_steps[cycle] = 0;
      break;
    }
    ls.init(k, m, S.data());
    std::fill(Bm.begin(), Bm.end(), 0.0);
    std::fill(Hbar.begin(), Hbar.end(), 0.0);
    int jd = 0;
    for (int j = 0; j < m; ++j) {
      // W = Op V_j
      const double* Zin = w.V(j);
      int64_t ldz = LB;
      if (h) {
        PMOR_TRY(op.apply_P(w, w.V(j), LB, w.Z, k, k, 1.0, 0.0, nullptr, 0));
        Zin = w.Z;
        ldz = k;
      }
      // W lands in the slot of V_{j+1}, right after [C, V_0..V_j], so that each
      // pass's Gram product [C, V, W]^T W also yields W^T W
      double* Wj = w.V(j + 1);
      PMOR_TRY(op.apply_A(w, Zin, ldz, Wj, LB, k, 1.0, 0.0, nullptr, 0));
      const int nb = kc + (j + 1) * k;  // [C, V_0..V_j]
      const double* basis = w.Bs + (kr - kc);
      for (int pass = 0; pass < 2; ++pass) {
        PMOR_TRY(gram(w, basis, LB, nb + k, Wj, LB, k, w.ds(1 + pass)));
        PMOR_TRY(tall_gemm(w, basis, LB, nb, w.ds(1 + pass), k, -1.0, 1.0, Wj, LB));
        PMOR_TRY(down(w, 1 + pass, w.ds(1 + pass), (int64_t)(nb + k) * k));
      }
      PMOR_TRY(sync(w));
      const double* g1 = w.hs(1);
      const double* g2 = w.hs(2);
      double wscale = 0.0;  // max ||W_c|| before Gram-Schmidt
      for (int c = 0; c < k; ++c) wscale = std::max(wscale, std::sqrt(std::max(g1[(nb + c) * k + c], 0.0)));
      for (int r = 0; r < nb; ++r)
        for (int c = 0; c < k; ++c) hc[(size_t)r * k + c] = g1[r * k + c] + g2[r * k + c];
      // W^T W after the second pass: (W1 - Q H2)^T (W1 - Q H2) = W1^T W1 - H2^T H2 for orthonormal Q
      std::vector<double> gw((size_t)k * k);
      for (int a = 0; a < k; ++a)
        for (int c = 0; c < k; ++c) {
          double v = g2[(nb + a) * k + c];
          for (int r = 0; r < nb; ++r) v -= g2[r * k + a] * g2[r * k + c];
          gw[(size_t)a * k + c] = v;
        }
      // Cholesky QR twice: T1 = W R1^{-1} (into Wt), V_{j+1} = T1 R2^{-1}, H_{j+1,j} = R2 R1
      std::vector<double> Hd((size_t)k * k, 0.0), R1((size_t)k * k), R1i((size_t)k * k), R2((size_t)k * k),
          R2i((size_t)k * k);
      bool okq = dense::chol_upper(k, gw.data(), R1.data());
      if (okq) {
        dense::inv_upper(k, R1.data(), R1i.data());
        PMOR_TRY(up(w, 3, R1i.data(), (int64_t)k * k));
        PMOR_TRY(tall_gemm(w, Wj, LB, k, w.ds(3), k, 1.0, 0.0, w.Wt, k));
        PMOR_TRY(gram(w, w.Wt, k, k, w.Wt, k, k, w.ds(0)));
        PMOR_TRY(down(w, 0, w.ds(0), (int64_t)k * k));
        PMOR_TRY(sync(w));
        okq = dense::chol_upper(k, w.hs(0), R2.data());
      }
      if (okq) {
        dense::inv_upper(k, R2.data(), R2i.data());
        PMOR_TRY(up(w, 4, R2i.data(), (int64_t)k * k));
        PMOR_TRY(tall_gemm(w, w.Wt, k, k, w.ds(4), k, 1.0, 0.0, Wj, LB));
        dense::matmul(k, k, k, R2.data(), R1.data(), Hd.data());
      }
      bool deficient = !okq;
      for (int c = 0; okq && c < k; ++c) {
        if (!(std::fabs(Hd[c * k + c]) > 1e-14 * wscale)) deficient = true;
        if (!(Hd[c * k + c] > kDepSine * std::sqrt(std::max(gw[c * k + c], 0.0)))) deficient = true;
      }
      if (deficient) {
        Hd.assign((size_t)k * k, 0.0);
        PMOR_TRY(tall_gemm(w, nullptr, 0, 0, nullptr, k, 1.0, 0.0, w.V(j + 1), LB));
      }
      // block column j of [B; Hbar]
      std::vector<double> Hcol((size_t)(j + 2) * k * k, 0.0);
      for (int r = 0; r < kc; ++r)
        for (int c = 0; c < k; ++c) Bm[(size_t)r * m * k + j * k + c] = hc[(size_t)r * k + c];
      for (int r = 0; r < (j + 1) * k; ++r)
        for (int c = 0; c < k; ++c) Hcol[(size_t)r * k + c] = hc[(size_t)(kc + r) * k + c];
      for (int r = 0; r < k; ++r)
        for (int c = 0; c < k; ++c) Hcol[(size_t)((j + 1) * k + r) * k + c] = Hd[(size_t)r * k + c];
      for (int r = 0; r < (j + 2) * k; ++r)
        for (int c = 0; c < k; ++c) Hbar[(size_t)r * m * k + j * k + c] = Hcol[(size_t)r * k + c];
      ls.add(j, Hcol.data());
      jd = j + 1;
      bool done = true;
      for (int c = 0; c < k; ++c) done = done && ls.resid(j, c) / bnorm[c] <= o.tol;
      if (deficient || done) break;
    }
    if (stats) {
      if (cycle < PMOR_MAX_CYCLES) stats->cycle_steps[cycle] = jd;
      stats->cycles = cycle + 1;
      stats->steps += jd;
    }
    const int jk = jd * k;
    // X += P (V y2 - U B y2)
    std::vector<double> y((size_t)jk * k);
    ls.solve(jd, y.data());
    PMOR_TRY(up(w, 3, y.data(), (int64_t)jk * k));
    PMOR_TRY(tall_gemm(w, w.V(0), LB, jk, w.ds(3), k, 1.0, 0.0, w.Z, k));
    if (kc > 0) {
      std::vector<double> By((size_t)kc * k, 0.0);
      for (int r = 0; r < kc; ++r)
        for (int c = 0; c < k; ++c) {
          double s = 0.0;
          for (int t = 0; t < jk; ++t) s += Bm[(size_t)r * m * k + t] * y[(size_t)t * k + c];
          By[(size_t)r * k + c] = s;
        }
      PMOR_TRY(up(w, 4, By.data(), (int64_t)kc * k));
      PMOR_TRY(tall_gemm(w, w.U, kr, kc, w.ds(4), k, -1.0, 1.0, w.Z, k));
    }
    PMOR_TRY(op.add_P(w, w.Z, k, X, ldx, k));
    // the recycled space of the next cycle (and system)
    if (kr > 0 && jd > 0) {
      const int rows = kc + (jd + 1) * k, N = kc + jk;
      std::vector<double> G((size_t)rows * N, 0.0), WtV((size_t)rows * N, 0.0), d(kc, 1.0);
      if (kc > 0) {
        const double* basis = w.Bs + (kr - kc);
        PMOR_TRY(gram(w, basis, LB, rows, w.U, kr, kc, w.ds(5)));
        PMOR_TRY(gram(w, w.U, kr, kc, w.U, kr, kc, w.ds(6)));
        PMOR_TRY(down(w, 5, w.ds(5), (int64_t)rows * kc));
        PMOR_TRY(down(w, 6, w.ds(6), (int64_t)kc * kc));
        PMOR_TRY(sync(w));
        for (int i = 0; i < kc; ++i) d[i] = 1.0 / std::sqrt(w.hs(6)[i * kc + i]);
        for (int i = 0; i < kc; ++i) G[(size_t)i * N + i] = d[i];
        for (int i = 0; i < kc; ++i)
          for (int t = 0; t < jk; ++t) G[(size_t)i * N + kc + t] = Bm[(size_t)i * m * k + t];
        for (int r = 0; r < rows; ++r)
          for (int i = 0; i < kc; ++i) WtV[(size_t)r * N + i] = w.hs(5)[r * kc + i] * d[i];
      }
      for (int r = 0; r < (jd + 1) * k; ++r)
        for (int t = 0; t < jk; ++t) G[(size_t)(kc + r) * N + kc + t] = Hbar[(size_t)r * m * k + t];
      for (int t = 0; t < jk; ++t) WtV[(size_t)(kc + t) * N + kc + t] = 1.0;
      std::vector<double> Pk((size_t)N * kr);
      const int kn = dense::harmonic_select(rows, N, G.data(), WtV.data(), kr, Pk.data(), nullptr, nullptr);
      std::vector<double> GP, Q, Rk;
      bool okr = kn > 0;
      if (okr) {
        std::vector<double> P2((size_t)N * kn);
        for (int r = 0; r < N; ++r)
          for (int c = 0; c < kn; ++c) P2[(size_t)r * kn + c] = Pk[(size_t)r * kr + c];
        GP.assign((size_t)rows * kn, 0.0);
        dense::matmul(rows, N, kn, G.data(), P2.data(), GP.data());
        Q.assign((size_t)rows * kn, 0.0);
        Rk.assign((size_t)kn * kn, 0.0);
        okr = dense::qr_positive(rows, kn, GP.data(), Q.data(), Rk.data());
        if (okr) {
          std::vector<double> Rki((size_t)kn * kn), top((size_t)std::max(kc, 1) * kn), bot((size_t)jk * kn);
          dense::inv_upper(kn, Rk.data(), Rki.data());
          // U_new = [U D, V] P_k R^{-1}: the U part D P_top R^{-1}, the V part P_bot R^{-1}
          std::vector<double> Pt((size_t)std::max(kc, 1) * kn, 0.0), Pb((size_t)jk * kn);
          for (int i = 0; i < kc; ++i)
            for (int c = 0; c < kn; ++c) Pt[(size_t)i * kn + c] = d[i] * P2[(size_t)i * kn + c];
          for (int t = 0; t < jk; ++t)
            for (int c = 0; c < kn; ++c) Pb[(size_t)t * kn + c] = P2[(size_t)(kc + t) * kn + c];
          if (kc > 0) dense::matmul(kc, kn, kn, Pt.data(), Rki.data(), top.data());
          dense::matmul(jk, kn, kn, Pb.data(), Rki.data(), bot.data());
          PMOR_TRY(up(w, 5, Q.data(), (int64_t)rows * kn));
          PMOR_TRY(up(w, 6, bot.data(), (int64_t)jk * kn));
          if (kc > 0) PMOR_TRY(up(w, 7, top.data(), (int64_t)kc * kn));
          PMOR_TRY(tall_gemm(w, w.Bs + (kr - kc), LB, rows, w.ds(5), kn, 1.0, 0.0, w.tC, kr));
          PMOR_TRY(tall_gemm(w, w.V(0), LB, jk, w.ds(6), kn, 1.0, 0.0, w.tU, kr));
          if (kc > 0) PMOR_TRY(tall_gemm(w, w.U, kr, kc, w.ds(7), kn, 1.0, 1.0, w.tU, kr));
          PMOR_TRY(copy_cols(w, w.tC, kr, w.Bs + (kr - kn), LB, kn));
          PMOR_TRY(copy_cols(w, w.tU, kr, w.U, kr, kn));
          PMOR_TRY(sync(w));  // the staged coefficients are read before the next upload
          kc = kn;
        }
      }
    }
  }
  if (stats) {
    for (int c = 0; c < k; ++c) stats->relres[c] = rel[c];
    stats->t_solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  // the recycled basis for the next system
  if (kc > 0) PMOR_TRY(copy_cols(w, w.U, kr, rec->U, kr, kc));
  rec->kc = kc;
  PMOR_TRY(sync(w));
  switch (status) {
    case PMOR_OK: return PMOR_OK;
    case PMOR_ENOTCONV: return fail(status, "block GCRO-DR did not converge within max_cycles");
    case PMOR_EBREAKDOWN: return fail(status, "block breakdown: rank-deficient residual block (block GCRO-DR)");
    default: return fail(status, "NaN or Inf in a residual (block GCRO-DR)");
  }
}

int harmonic_select_host(int rows, int N, const double* G, const double* WtV, int kr, double* Pk, double* mu_re,
                         double* mu_im) {
  return dense::harmonic_select(rows, N, G, WtV, kr, Pk, mu_re, mu_im);
}

}  // namespace pmor

namespace pmor {
static int gcrodr_pt(pmor_problem* pb, const pmor_spai* h, const Point* pt, int prc, const double* B, int64_t ldb,
                     int32_t k, double* X, int64_t ldx, const pmor_solve_opts* opts, pmor_recycle* rec,
                     pmor_stats* stats) {
  if (!pb || !B || !X || !rec) return fail(PMOR_EINVAL, "NULL argument");
  if (k < 1 || k > PMOR_KMAX) return fail(PMOR_EINVAL, "k must be in 1..16");
  if (ldb < k || ldx < k) return fail(PMOR_EINVAL, "leading dimension smaller than k");
  if (h && h->pb != pb) return fail(PMOR_EINVAL, "preconditioner belongs to another problem");
  if (rec->n != pb->n) return fail(PMOR_EINVAL, "recycler and problem differ in n");
  if (rec->ctx != pb->ctx) return fail(PMOR_EINVAL, "recycler belongs to another context");
  if (prc != PMOR_OK) return prc;
  pmor_solve_opts o{30, 20, 1e-8};
  if (opts) o = *opts;
  if (o.m < 1 || o.m > 31) return fail(PMOR_EINVAL, "m must be in 1..31");
  if (o.max_cycles < 1 || o.max_cycles > PMOR_MAX_CYCLES) return fail(PMOR_EINVAL, "max_cycles out of range");
  if (!(o.tol > 0.0) || !std::isfinite(o.tol)) return fail(PMOR_EINVAL, "tol must be positive");
  PMOR_HIP(hipSetDevice(pb->ctx->device));
  return gcrodr_solve(pb, h, *pt, B, ldb, k, X, ldx, o, rec, stats);
}
}  // namespace pmor

extern "C" {

int block_solve_gcrodr(pmor_problem* pb, const pmor_spai* h, double s, double p, const double* B, int64_t ldb,
                       int32_t k, double* X, int64_t ldx, const pmor_solve_opts* opts, pmor_recycle* rec,
                       pmor_stats* stats) {
  pmor::Point pt{};
  const int prc = pb ? pmor::point_sp(pb, s, p, &pt) : PMOR_OK;
  return pmor::gcrodr_pt(pb, h, &pt, prc, B, ldb, k, X, ldx, opts, rec, stats);
}

int block_solve_gcrodr_c(pmor_problem* pb, const pmor_spai* h, const double* coef, const double* B, int64_t ldb,
                         int32_t k, double* X, int64_t ldx, const pmor_solve_opts* opts, pmor_recycle* rec,
                         pmor_stats* stats) {
  pmor::Point pt{};
  const int prc = pb ? pmor::point_coef(pb, coef, &pt) : PMOR_OK;
  return pmor::gcrodr_pt(pb, h, &pt, prc, B, ldb, k, X, ldx, opts, rec, stats);
}

int pmor_recycle_create(pmor_ctx* ctx, int32_t n, int32_t kr, pmor_recycle** out) {
  if (out) *out = nullptr;
  if (!ctx || !out) return pmor::fail(PMOR_EINVAL, "NULL argument");
  if (n < 1) return pmor::fail(PMOR_EINVAL, "n must be positive");
  if (kr < 0 || kr > PMOR_KMAX) return pmor::fail(PMOR_EINVAL, "kr must be in 0..16");
  PMOR_HIP(hipSetDevice(ctx->device));
  pmor_recycle* r = new pmor_recycle();
  r->ctx = ctx;
  r->n = n;
  r->kr = kr;
  if (pmor::dmalloc((void**)&r->U, sizeof(double) * (size_t)n * std::max(kr, 1), ctx->stream) != hipSuccess) {
    (void)hipGetLastError();
    delete r;
    return pmor::fail(PMOR_ENOMEM, "allocation of the recycled basis failed");
  }
  pmor::ctx_ref(ctx);
  *out = r;
  return PMOR_OK;
}

void pmor_recycle_destroy(pmor_recycle* r) {
  if (!r) return;
  (void)hipSetDevice(r->ctx->device);
  (void)hipStreamSynchronize(r->ctx->stream);
  pmor::dfree(r->U, r->ctx->stream);
  pmor::ctx_unref(r->ctx);
  delete r;
}

int pmor_recycle_info(const pmor_recycle* r, int32_t* kc) {
  if (!r) return pmor::fail(PMOR_EINVAL, "recycler is NULL");
  if (kc) *kc = r->kc;
  return PMOR_OK;
}

int pmor_recycle_reset(pmor_recycle* r) {
  if (!r) return pmor::fail(PMOR_EINVAL, "recycler is NULL");
  r->kc = 0;
  return PMOR_OK;
}

int pmor_recycle_export(const pmor_recycle* r, double* U, int64_t ldu) {
  if (!r || !U) return pmor::fail(PMOR_EINVAL, "NULL argument");
  if (r->kc == 0) return PMOR_OK;
  if (ldu < r->kc) return pmor::fail(PMOR_EINVAL, "ldu smaller than the recycled dimension");
  PMOR_HIP(hipSetDevice(r->ctx->device));
  PMOR_HIP(hipMemcpy2DAsync(U, sizeof(double) * ldu, r->U, sizeof(double) * r->kr, sizeof(double) * r->kc, r->n,
                            hipMemcpyDeviceToDevice, r->ctx->stream));
  PMOR_HIP(hipStreamSynchronize(r->ctx->stream));
  return PMOR_OK;
}

int pmor_harmonic_ritz(int32_t rows, int32_t N, const double* G, const double* WtV, int32_t kr, double* Pk,
                       double* mu_re, double* mu_im, int32_t* count) {
  if (!G || !WtV || !Pk || !count) return pmor::fail(PMOR_EINVAL, "NULL argument");
  if (rows < N || N < 1 || kr < 0) return pmor::fail(PMOR_EINVAL, "bad sizes");
  const int c = pmor::harmonic_select_host(rows, N, G, WtV, kr, Pk, mu_re, mu_im);
  if (c < 0) return pmor::fail(PMOR_ESINGULAR, "G^T G is not positive definite or the eigen-iteration failed");
  *count = c;
  return PMOR_OK;
}

}  // extern "C"
