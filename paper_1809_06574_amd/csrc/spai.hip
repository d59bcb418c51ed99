// SPAI least squares and the cheap update.
//
// SPAI (paper, Section 2.2): min ||I - A P||_F splits into one least-squares
// problem per column, min ||e_j - A p_j||_2 with p_j supported on J_j; only the
// shadow rows I_j of A(:, J_j) take part, giving the dense |I_j| x |J_j| problem
// A(I_j, J_j) p = e_j(I_j).  The first-approach update (Section 2.3, Table 1;
// Section 2.4) solves the same kind of column problems,
// min ||A(1) e_i - A(l) q_i||_2, with A(1)'s column as right-hand side.
//
// Mapping: one wavefront per column.  Lane l holds rows l, l+64, ... of the
// gathered block (in registers for |J| <= 16, in LDS above), the Householder
// QR runs with one cross-lane reduction per reflector (the column norm and all
// the inner products the reflector needs are summed together), then back
// substitution broadcasts one unknown at a time.
#include <hip/hip_fp16.h>

#include <algorithm>

#include <cstring>
#include <vector>

#include "common.hpp"

namespace pmor {

template <typename T> struct Eps;
template <> struct Eps<double> { static constexpr double v = 2.220446049250313e-16; };
template <> struct Eps<float> { static constexpr double v = 1.1920928955078125e-07; };

__device__ __forceinline__ double readlane_d(double x, int l) {
  int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
  int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float readlane_d(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

// value of column c in CSR row [e, ee) starting the search at e (monotone cursor)
__device__ __forceinline__ double row_lookup(const int32_t* colidx, const double* val, int& e, int ee, int c) {
  while (e < ee && colidx[e] < c) ++e;
  return (e < ee && colidx[e] == c) ? val[e] : 0.0;
}

struct LsArgs {
  int ncols;
  const int32_t* cols;  // bucket column list, or null (then column = col_off + index)
  int col_off;
  const int32_t* rowptr;
  const int32_t* colidx;
  const double* aval;      // matrix of the least-squares problems (A or A(l))
  const double* rhs_aval;  // null: right-hand side e_j; else A(1) values on the same pattern
  const int32_t* Jcolptr;
  const int32_t* Jrow;
  const int64_t* Icolptr;
  const int32_t* Irow;
  const int32_t* Pslot;
  const int32_t* Acolptr;  // CSC view of A's pattern (the LDS kernel gathers by columns)
  const int32_t* Arowidx;
  const int32_t* Acscslot;  // CSC position -> CSR position of the value
  double* out;     // values in P's CSR order
  double* rho;     // per-column residual norm
  int* bad_col;    // smallest singular column (atomicMin)
  // several systems in one launch: the columns of system s are the launch's
  // columns [seg[s], seg[s + 1]) (each system's count padded to whole
  // wavefronts), described by sys[s]; null for a launch of one system
  const LsArgs* sys;
  const int32_t* seg;
  int nsys;
};

// the system of a wavefront's columns in a launch over several systems (every
// wavefront's columns belong to one system): largest s with seg[s] <= w0
__device__ __forceinline__ int ls_system(const int32_t* seg, int nsys, int w0) {
  int lo = 0, hi = nsys - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (seg[mid] <= w0) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// register kernel: 16 lanes (one DPP row) per column, four columns per
// wavefront; |J| <= JMAX (<= 16), |I| <= 16 R.  Lane g of a row holds rows
// g, g + 16, ... of the gathered block.  Sums use a DPP butterfly inside the row
// (quad_perm xor 1, xor 2, row_half_mirror, row_mirror: every lane ends with the
// same bits), broadcasts of row k < 16 use row_newbcast:k.
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ double dpp_row(double x) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(x), __double2loint(x), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(x), __double2hiint(x), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_row(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(x), __float_as_int(x), CTRL, 0xF, 0xF, false));
}

template <typename T>
__device__ __forceinline__ T row_sum(T x) {
  x += dpp_row<0xB1>(x);   // quad_perm(1,0,3,2)
  x += dpp_row<0x4E>(x);   // quad_perm(2,3,0,1)
  x += dpp_row<0x141>(x);  // row_half_mirror
  x += dpp_row<0x140>(x);  // row_mirror
  return x;
}

template <typename T>
__device__ __forceinline__ T row_max(T x) {
  T y;
  y = dpp_row<0xB1>(x); x = x > y ? x : y;
  y = dpp_row<0x4E>(x); x = x > y ? x : y;
  y = dpp_row<0x141>(x); x = x > y ? x : y;
  y = dpp_row<0x140>(x); x = x > y ? x : y;
  return x;
}

// the same over a group of G = 16 or 32 lanes (G = 32: the two rows' results
// added in the same order on both rows, so every lane of the group holds the
// same bits)
template <int G, typename T>
__device__ __forceinline__ T grp_sum(T x) {
  x = row_sum(x);
  if constexpr (G >= 32) {
    const T y = __shfl_xor(x, 16, 64);
    x = ((threadIdx.x & 16) == 0) ? x + y : y + x;
  }
  if constexpr (G == 64) {
    const T y = __shfl_xor(x, 32, 64);
    x = ((threadIdx.x & 32) == 0) ? x + y : y + x;
  }
  return x;
}

template <int G, typename T>
__device__ __forceinline__ T grp_max(T x) {
  x = row_max(x);
  if constexpr (G >= 32) {
    const T y = __shfl_xor(x, 16, 64);
    x = x > y ? x : y;
  }
  if constexpr (G == 64) {
    const T y = __shfl_xor(x, 32, 64);
    x = x > y ? x : y;
  }
  return x;
}

// value of lane k (0..15, a constant after unrolling) of this lane's row
template <typename T>
__device__ __forceinline__ T row_bcast(T x, int k);

// value of lane k (a constant after unrolling) of this lane's group of G lanes
template <int G, typename T>
__device__ __forceinline__ T grp_bcast(T x, int k) {
  if constexpr (G == 16) return row_bcast(x, k);
  else return __shfl(x, (int)(threadIdx.x & ~(unsigned)(G - 1)) + k, 64);
}

// the same for a k known only at run time (uniform over the wavefront)
template <int G, typename T>
__device__ __forceinline__ T grp_bcast_dyn(T x, int k) {
  return __shfl(x, (int)(threadIdx.x & ~(unsigned)(G - 1)) + k, 64);
}

template <typename T>
__device__ __forceinline__ T row_bcast(T x, int k) {
  switch (k) {
    case 0: return dpp_row<0x150>(x);
    case 1: return dpp_row<0x151>(x);
    case 2: return dpp_row<0x152>(x);
    case 3: return dpp_row<0x153>(x);
    case 4: return dpp_row<0x154>(x);
    case 5: return dpp_row<0x155>(x);
    case 6: return dpp_row<0x156>(x);
    case 7: return dpp_row<0x157>(x);
    case 8: return dpp_row<0x158>(x);
    case 9: return dpp_row<0x159>(x);
    case 10: return dpp_row<0x15A>(x);
    case 11: return dpp_row<0x15B>(x);
    case 12: return dpp_row<0x15C>(x);
    case 13: return dpp_row<0x15D>(x);
    case 14: return dpp_row<0x15E>(x);
    default: return dpp_row<0x15F>(x);
  }
}

// FP16 storage with a power-of-two scale per column: x -> half(x 2^-e) 2^e,
// e = ilogb(max|x|) + 1 so the scaled column lies in (-1, 1); the arithmetic
// stays in FP32.
struct Q16Scale {
  float sc, isc;
};
__device__ __forceinline__ Q16Scale q16_scale(float mx) {
  if (!(mx > 0.0f) || !(mx < 3.0e38f)) return {1.0f, 1.0f};
  const int e = ilogbf(mx) + 1;
  return {ldexpf(1.0f, -e), ldexpf(1.0f, e)};
}
__device__ __forceinline__ float q16(float x, Q16Scale q) { return __half2float(__float2half_rn(x * q.sc)) * q.isc; }

template <typename T, int JMAX, int R, bool Q16 = false, int G = 16, bool GO = false, bool MULTI = false>
__global__ __launch_bounds__(256) void k_spai_reg(LsArgs a0) {
  static_assert(G == 16 || G == 32 || G == 64, "groups of one, two or four DPP rows");
  static_assert(JMAX <= G, "row k of R must sit in lane k of the group");
  constexpr int LG = G == 16 ? 4 : (G == 32 ? 5 : 6);
  const int gl = threadIdx.x & (G - 1);
  const int wid = (xcd_swizzle(blockIdx.x, gridDim.x) * 256 + threadIdx.x) >> LG;
  if (wid >= a0.ncols) return;  // whole groups leave together
  LsArgs a = a0;
  int wl = wid;
  if constexpr (MULTI) {
    const int sy = ls_system(a0.seg, a0.nsys, __builtin_amdgcn_readfirstlane(wid));
    a = a0.sys[sy];
    wl = wid - a0.seg[sy];
    if (wl >= a.ncols) return;  // the padding of the system's last wavefront
  }
  const int j = a.cols ? a.cols[wl] : a.col_off + wl;
  const int jb = a.Jcolptr[j];
  const int nj = a.Jcolptr[j + 1] - jb;
  const int64_t ib = a.Icolptr[j];
  const int ni = (int)(a.Icolptr[j + 1] - ib);

  T A_[R][JMAX];
  T b_[R];
  // gather A(I_j, J_j) and the right-hand side: a row's first RW entries are
  // loaded at once (independent loads) and matched against J_j in registers;
  // longer rows continue with a cursor search
  constexpr int RW = 8;
  int Jv[JMAX];
#pragma unroll
  for (int t = 0; t < JMAX; ++t) Jv[t] = (t < nj) ? a.Jrow[jb + t] : -1;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int li = gl + G * r;
    const int row = (li < ni) ? a.Irow[ib + li] : -1;
#pragma unroll
    for (int t = 0; t < JMAX; ++t) A_[r][t] = T(0);
    b_[r] = T(0);
    if (row >= 0) {
      const int e0 = a.rowptr[row];
      const int ee = a.rowptr[row + 1];
      int cc[RW];
      double vv[RW], ww[RW];
#pragma unroll
      for (int u = 0; u < RW; ++u) {
        const bool in = e0 + u < ee;
        cc[u] = in ? a.colidx[e0 + u] : -2;
        vv[u] = in ? a.aval[e0 + u] : 0.0;
        ww[u] = (in && a.rhs_aval) ? a.rhs_aval[e0 + u] : 0.0;
      }
#pragma unroll
      for (int t = 0; t < JMAX; ++t) {
        double x = 0.0;
#pragma unroll
        for (int u = 0; u < RW; ++u) x = (cc[u] == Jv[t]) ? vv[u] : x;
        A_[r][t] = (T)x;
      }
      if (a.rhs_aval) {
        double x = 0.0;
#pragma unroll
        for (int u = 0; u < RW; ++u) x = (cc[u] == j) ? ww[u] : x;
        b_[r] = (T)x;
      } else {
        b_[r] = (row == j) ? T(1) : T(0);
      }
      if (ee - e0 > RW) {  // the rest of a long row
        int e = e0 + RW;
#pragma unroll
        for (int t = 0; t < JMAX; ++t)
          if (t < nj) {
            const double x = row_lookup(a.colidx, a.aval, e, ee, Jv[t]);
            if (x != 0.0) A_[r][t] = (T)x;
          }
        if (a.rhs_aval) {
          int e2 = e0 + RW;
          const double x = row_lookup(a.colidx, a.rhs_aval, e2, ee, j);
          if (x != 0.0) b_[r] = (T)x;
        }
      }
    }
  }
  if constexpr (GO) {  // gather only: the block's sum into rho[j]
    T acc = T(0);
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int t = 0; t < JMAX; ++t) acc += A_[r][t];
    acc = grp_sum<G>(acc);
    if (gl == 0) a.rho[j] = (double)acc;
    return;
  }
  if constexpr (Q16) {
#pragma unroll
    for (int t = 0; t < JMAX; ++t) {
      if (t < nj) {
        T mx = T(0);
#pragma unroll
        for (int r = 0; r < R; ++r) mx = fmaxf(mx, fabsf(A_[r][t]));
        const Q16Scale q = q16_scale(grp_max<G>(mx));
#pragma unroll
        for (int r = 0; r < R; ++r) A_[r][t] = q16(A_[r][t], q);
      }
    }
    if (a.rhs_aval) {
      T mx = T(0);
#pragma unroll
      for (int r = 0; r < R; ++r) mx = fmaxf(mx, fabsf(b_[r]));
      const Q16Scale q = q16_scale(grp_max<G>(mx));
#pragma unroll
      for (int r = 0; r < R; ++r) b_[r] = q16(b_[r], q);
    }
  }
  T minDiag = T(3.0e38);
  // Householder QR, one reflector per column k: one round of group sums gives
  // the column norm and every inner product the reflector needs.  The loop over
  // k stays rolled and every register index is static: column k is picked out
  // by selects and the loops over c run over all columns with a (uniform) test
  // c >= k, so the block never leaves the registers.
  for (int k = 0; k < nj; ++k) {
    T xk[R];  // column k of this lane's rows
#pragma unroll
    for (int r = 0; r < R; ++r) {
      T x = T(0);
#pragma unroll
      for (int t = 0; t < JMAX; ++t) x = (t == k) ? A_[r][t] : x;
      xk[r] = x;
    }
    T s[JMAX + 1];
#pragma unroll
    for (int c = 0; c <= JMAX; ++c) s[c] = T(0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int li = gl + G * r;
      if (li >= k) {
        const T x = xk[r];
#pragma unroll
        for (int c = 0; c < JMAX; ++c)
          if (c >= k) s[c] += x * A_[r][c];
        s[JMAX] += x * b_[r];
      }
    }
    // the sums in chunks of 8 columns: one uniform test per chunk, eight
    // independent reductions inside it
#pragma unroll
    for (int c0 = 0; c0 < JMAX; c0 += 8)
      if (c0 + 8 > k && c0 < nj) {
#pragma unroll
        for (int c = c0; c < c0 + 8 && c < JMAX; ++c) s[c] = grp_sum<G>(s[c]);
      }
    s[JMAX] = grp_sum<G>(s[JMAX]);
    T sig = T(0);
#pragma unroll
    for (int c = 0; c < JMAX; ++c) sig = (c == k) ? s[c] : sig;
    const T alpha = grp_bcast_dyn<G>(xk[0], k);  // row k < nj <= G sits in slot 0 of lane k
    T beta = alpha;
    if (sig != alpha * alpha) {
      const T nrm = sqrt(sig);
      beta = (alpha >= T(0)) ? -nrm : nrm;
      const T rden = T(1) / (beta * (beta - alpha));
      // the reflector's factor of every column replaces its inner product
#pragma unroll
      for (int c = 0; c < JMAX; ++c)
        if (c > k && c < nj) s[c] = (s[c] - beta * grp_bcast_dyn<G>(A_[0][c], k)) * rden;
      s[JMAX] = (s[JMAX] - beta * grp_bcast_dyn<G>(b_[0], k)) * rden;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int li = gl + G * r;
        if (li >= k) {
          const T v = (li == k) ? (alpha - beta) : xk[r];
#pragma unroll
          for (int c = 0; c < JMAX; ++c)
            if (c > k && c < nj) A_[r][c] -= s[c] * v;
          b_[r] -= s[JMAX] * v;
        }
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int li = gl + G * r;
#pragma unroll
      for (int t = 0; t < JMAX; ++t)
        if (t == k) {
          if (li == k) A_[r][t] = beta;
          else if (li > k) A_[r][t] = T(0);
        }
    }
    const T ab = beta < T(0) ? -beta : beta;
    minDiag = ab < minDiag ? ab : minDiag;
  }
  // max |R| over the triangle (rows < nj <= G live in slot 0)
  T mx = T(0);
  if (gl < nj) {
#pragma unroll
    for (int c = 0; c < JMAX; ++c)
      if (c >= gl && c < nj) {
        const T v = A_[0][c] < T(0) ? -A_[0][c] : A_[0][c];
        mx = v > mx ? v : mx;
      }
  }
  const T maxR = grp_max<G>(mx);
  // back substitution R p = (Q^T b)(0:nj), one unknown at a time
  T mine = T(0);
  T p[JMAX];
#pragma unroll
  for (int i = JMAX - 1; i >= 0; --i) {
    if (i < nj) {
      T acc = b_[0];
#pragma unroll
      for (int c = i + 1; c < JMAX; ++c)
        if (c < nj) acc -= A_[0][c] * p[c];
      const T pi = acc / A_[0][i];
      p[i] = grp_bcast<G>(pi, i);
      if (gl == i) mine = pi;
    } else {
      p[i] = T(0);
    }
  }
  // residual: the part of Q^T b below row nj
  T rr = T(0);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int li = gl + G * r;
    if (li >= nj && li < ni) rr += b_[r] * b_[r];
  }
  rr = grp_sum<G>(rr);
  if (gl < nj) a.out[a.Pslot[jb + gl]] = (double)mine;
  if (gl == 0) {
    a.rho[j] = sqrt((double)rr);
    const bool singular = (ni < nj) || !(minDiag > T(10.0 * ni * Eps<T>::v) * maxR);
    if (singular) atomicMin(a.bad_col, j);
  }
}

// ---------------------------------------------------------------------------
// LDS kernel: |J| <= 64, |I| <= 512; one workgroup of LDS_NW wavefronts per
// column, its LDS sized to the largest column of the launch (ldI x (JM + 1)
// values and ldI row indices).  The gather goes by the columns of A: all rows
// of A(:, J_t) lie in I_j (that is how I_j is defined), so thread t takes
// column J_t's entries in CSC order and places each at its row's position in
// I_j, found by binary search in the sorted rows held in LDS.  In the
// Householder steps wavefront w owns the columns k + w CH, k + (w + NW) CH, ...
// (chunks of CH): it forms their inner products with the reflector over all
// rows and updates them, each sum taken by one wavefront in one order, so the
// result does not depend on the number of wavefronts.
// ---------------------------------------------------------------------------
constexpr int LDS_NW = 4;

__device__ __forceinline__ int lds_lower_bound(const int* rows, int len, int r) {
  int lo = 0, hi = len;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (rows[mid] < r) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

template <typename T, bool Q16 = false, bool GO = false, bool MULTI = false>
__global__ __launch_bounds__(64 * LDS_NW) void k_spai_lds(LsArgs a0, int ldI, int JM) {
  constexpr int NW = LDS_NW, NT = 64 * NW;
  extern __shared__ unsigned char smem_raw[];
  T* S = reinterpret_cast<T*>(smem_raw);  // column-major [nj + 1][ldI]: A_hat then rhs (JM >= nj)
  int* Is = reinterpret_cast<int*>(S + (size_t)(JM + 1) * ldI);  // the rows I_j
  __shared__ double sv[66];
  __shared__ T sf[66];  // the reflector's factor per column
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wid = blockIdx.x;
  if (wid >= a0.ncols) return;
  LsArgs a = a0;
  int wl = wid;
  if constexpr (MULTI) {
    const int sy = ls_system(a0.seg, a0.nsys, wid);
    a = a0.sys[sy];
    wl = wid - a0.seg[sy];
    if (wl >= a.ncols) return;
  }
  const int j = a.cols ? a.cols[wl] : a.col_off + wl;
  const int jb = a.Jcolptr[j];
  const int nj = a.Jcolptr[j + 1] - jb;
  const int64_t ib = a.Icolptr[j];
  const int ni = (int)(a.Icolptr[j + 1] - ib);
  T* B = S + (size_t)nj * ldI;  // the right-hand side is column nj of S
  for (int li = tid; li < ni; li += NT) Is[li] = a.Irow[ib + li];
  for (int t = 0; t <= nj; ++t) {
    T* colt = (t < nj) ? S + (size_t)t * ldI : B;
    for (int li = tid; li < ni; li += NT) colt[li] = T(0);
  }
  __syncthreads();
  if (tid < nj) {
    const int c = a.Jrow[jb + tid];
    T* colt = S + (size_t)tid * ldI;
    int q = 0;
    for (int e = a.Acolptr[c]; e < a.Acolptr[c + 1]; ++e) {
      const int r = a.Arowidx[e];
      q += lds_lower_bound(Is + q, ni - q, r);  // rows of A(:, c) ascend: search from the last hit
      colt[q] = (T)a.aval[a.Acscslot[e]];
    }
  }
  if (a.rhs_aval) {  // A(1) e_j on I_j: the entries of column j
    for (int e = a.Acolptr[j] + tid; e < a.Acolptr[j + 1]; e += NT)
      B[lds_lower_bound(Is, ni, a.Arowidx[e])] = (T)a.rhs_aval[a.Acscslot[e]];
  } else if (tid == 0) {
    B[lds_lower_bound(Is, ni, j)] = T(1);
  }
  __syncthreads();
  if constexpr (GO) {  // gather only: the block's sum into rho[j]
    if (w != 0) return;
    T acc = T(0);
    for (int t = 0; t < nj; ++t)
      for (int li = lane; li < ni; li += 64) acc += S[(size_t)t * ldI + li];
    acc = wave_sum(acc);
    if (lane == 0) a.rho[j] = (double)acc;
    return;
  }
  if constexpr (Q16) {
    for (int t = w; t <= nj; t += NW) {
      if (t == nj && !a.rhs_aval) break;
      T* colt = (t < nj) ? S + (size_t)t * ldI : B;
      T mx = T(0);
      for (int li = lane; li < ni; li += 64) mx = fmaxf(mx, fabsf(colt[li]));
      const Q16Scale q = q16_scale(wave_max(mx));
      for (int li = lane; li < ni; li += 64) colt[li] = q16(colt[li], q);
    }
    __syncthreads();
  }
  T minDiag = T(3.0e38);
  constexpr int CH = 8;  // columns per chunk: independent sums side by side
  for (int k = 0; k < nj; ++k) {
    // s[c] = x . a_c for c in [k, nj) and x . b (c = nj), CH columns per pass,
    // the chunks dealt out to the wavefronts
    const T* colk = S + (size_t)k * ldI;
    for (int c0 = k + w * CH; c0 <= nj; c0 += NW * CH) {
      T part[CH];
#pragma unroll
      for (int u = 0; u < CH; ++u) part[u] = T(0);
      for (int li = k + lane; li < ni; li += 64) {
        const T x = colk[li];
#pragma unroll
        for (int u = 0; u < CH; ++u)
          if (c0 + u <= nj) part[u] += x * S[(size_t)(c0 + u) * ldI + li];
      }
#pragma unroll
      for (int u = 0; u < CH; ++u)
        if (c0 + u <= nj) {
          const T t = wave_sum(part[u]);
          if (lane == 0) sv[c0 + u - k] = (double)t;
        }
    }
    __syncthreads();
    const T alpha = colk[k];
    const T sig = (T)sv[0];
    T beta = alpha;
    if (sig != alpha * alpha) {
      const T nrm = sqrt(sig);
      beta = (alpha >= T(0)) ? -nrm : nrm;
      const T denom = beta * (beta - alpha);
      // the factors of every column (a_c(k) is read before any thread writes it)
      for (int c = k + 1 + tid; c <= nj; c += NT) sf[c] = ((T)sv[c - k] - beta * S[(size_t)c * ldI + k]) / denom;
      __syncthreads();
      // wavefront w updates the columns of its chunks, starting after column k
      for (int li = k + lane; li < ni; li += 64) {
        const T v = (li == k) ? (alpha - beta) : colk[li];
        for (int c0 = k + 1 + w * CH; c0 <= nj; c0 += NW * CH) {
#pragma unroll
          for (int u = 0; u < CH; ++u)
            if (c0 + u <= nj) S[(size_t)(c0 + u) * ldI + li] -= sf[c0 + u] * v;
        }
      }
    }
    __syncthreads();
    if (tid == 0) S[(size_t)k * ldI + k] = beta;
    for (int li = k + 1 + tid; li < ni; li += NT) S[(size_t)k * ldI + li] = T(0);
    __syncthreads();
    const T ab = beta < T(0) ? -beta : beta;
    minDiag = ab < minDiag ? ab : minDiag;
  }
  // every wavefront forms max|R| and the residual itself (same values in each)
  T mx = T(0);
  for (int q = lane; q < nj * nj; q += 64) {
    const int r = q % nj, c = q / nj;
    if (r <= c) {
      T v = S[(size_t)c * ldI + r];
      v = v < T(0) ? -v : v;
      mx = v > mx ? v : mx;
    }
  }
  const T maxR = wave_max(mx);
  // back substitution, column oriented: y in B[0:nj]
  for (int i = nj - 1; i >= 0; --i) {
    __syncthreads();
    const T pi = B[i] / S[(size_t)i * ldI + i];
    __syncthreads();
    if (tid == 0) B[i] = pi;
    for (int r = tid; r < i; r += NT) B[r] -= S[(size_t)i * ldI + r] * pi;
  }
  __syncthreads();
  if (w != 0) return;
  T rr = T(0);
  for (int li = nj + lane; li < ni; li += 64) rr += B[li] * B[li];
  rr = wave_sum(rr);
  for (int t = lane; t < nj; t += 64) a.out[a.Pslot[jb + t]] = (double)B[t];
  if (lane == 0) {
    a.rho[j] = sqrt((double)rr);
    const bool singular = (ni < nj) || !(minDiag > T(10.0 * ni * Eps<T>::v) * maxR);
    if (singular) atomicMin(a.bad_col, j);
  }
}

// ---------------------------------------------------------------------------
// Column-owner kernel: |J| <= JM, |I| <= 64, 4-byte values (the (32, 64)
// bucket: against the register kernel's two columns per wavefront it takes 0.54
// of the time on the batch workload; |J| <= 16 takes k_spai_col2 below, two
// columns per workgroup, since one column would leave most lanes idle).  One
// 64-lane workgroup per column j.  Lane c holds column c of A(I_j, J_j), all 64
// rows in registers, and lane |J_j| the right-hand side, so every inner product
// a reflector step needs is a sum inside one lane; only the reflector crosses
// lanes (its owner writes it to LDS, every lane reads it back as a broadcast).
// The reflector loop is unrolled over k, so every register index is static.
// The gather and the back substitution go through LDS as in k_spai_lds.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float readlane_f(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

template <typename T, int JM, bool Q16 = false, bool MULTI = false>
__global__ __launch_bounds__(64) void k_spai_col(LsArgs a0) {
  static_assert(sizeof(T) == 4, "four-byte values");
  constexpr int IM = 64, LD = IM + 1;  // rows; LDS column stride (odd: the column reads spread over the banks)
  __shared__ T S[(JM + 1) * LD];       // column-major: A_hat's columns, then the right-hand side
  __shared__ int Is[IM];
  __shared__ T sv[IM];                 // the reflector's column of the current step
  const int lane = threadIdx.x;
  const int wid = xcd_swizzle(blockIdx.x, gridDim.x);
  if (wid >= a0.ncols) return;
  LsArgs a = a0;
  int wl = wid;
  if constexpr (MULTI) {
    const int sy = ls_system(a0.seg, a0.nsys, wid);
    a = a0.sys[sy];
    wl = wid - a0.seg[sy];
    if (wl >= a.ncols) return;
  }
  const int j = a.cols ? a.cols[wl] : a.col_off + wl;
  const int jb = a.Jcolptr[j];
  const int nj = a.Jcolptr[j + 1] - jb;
  const int64_t ib = a.Icolptr[j];
  const int ni = (int)(a.Icolptr[j + 1] - ib);
  if (lane < ni) Is[lane] = a.Irow[ib + lane];
  for (int q = lane; q < (JM + 1) * LD; q += 64) S[q] = T(0);
  __syncthreads();
  if (lane < nj) {
    const int c = a.Jrow[jb + lane];
    T* colt = S + lane * LD;
    int q = 0;
    for (int e = a.Acolptr[c]; e < a.Acolptr[c + 1]; ++e) {
      const int r = a.Arowidx[e];
      q += lds_lower_bound(Is + q, ni - q, r);  // rows of A(:, c) ascend: search from the last hit
      colt[q] = (T)a.aval[a.Acscslot[e]];
    }
  }
  T* B = S + nj * LD;
  if (a.rhs_aval) {  // A(1) e_j on I_j: the entries of column j
    for (int e = a.Acolptr[j] + lane; e < a.Acolptr[j + 1]; e += 64)
      B[lds_lower_bound(Is, ni, a.Arowidx[e])] = (T)a.rhs_aval[a.Acscslot[e]];
  } else if (lane == 0) {
    B[lds_lower_bound(Is, ni, j)] = T(1);
  }
  __syncthreads();
  // lane c <= nj: its column (lanes beyond take the right-hand side again and
  // are never read)
  const int cl = lane <= nj ? lane : nj;
  T A_[IM];
#pragma unroll
  for (int r = 0; r < IM; ++r) A_[r] = S[cl * LD + r];
  if constexpr (Q16) {
    if (lane < nj || (lane == nj && a.rhs_aval)) {
      T mx = T(0);
#pragma unroll
      for (int r = 0; r < IM; ++r) mx = fmaxf(mx, fabsf(A_[r]));
      const Q16Scale q = q16_scale(mx);
#pragma unroll
      for (int r = 0; r < IM; ++r) A_[r] = q16(A_[r], q);
    }
  }
  T minDiag = T(3.0e38);
#pragma unroll
  for (int k = 0; k < JM; ++k) {
    if (k < nj) {
      if (lane == k) {
#pragma unroll
        for (int r = k; r < IM; ++r) sv[r] = A_[r];
      }
      __syncthreads();
      T x[IM];
      T dot = T(0);
#pragma unroll
      for (int r = k; r < IM; ++r) {
        x[r] = sv[r];
        dot += x[r] * A_[r];
      }
      const T sig = readlane_f(dot, k);
      const T alpha = x[k];
      T beta = alpha;
      if (sig != alpha * alpha) {
        const T nrm = sqrt(sig);
        beta = (alpha >= T(0)) ? -nrm : nrm;
        const T denom = beta * (beta - alpha);
        if (lane > k) {
          const T f = (dot - beta * A_[k]) / denom;
          A_[k] -= f * (alpha - beta);
#pragma unroll
          for (int r = k + 1; r < IM; ++r) A_[r] -= f * x[r];
        }
      }
      if (lane == k) {
        A_[k] = beta;
#pragma unroll
        for (int r = k + 1; r < IM; ++r) A_[r] = T(0);
      }
      const T ab = beta < T(0) ? -beta : beta;
      minDiag = ab < minDiag ? ab : minDiag;
      __syncthreads();  // sv is written again by the next step
    }
  }
  // R (columns 0..nj-1) and Q^T b (column nj) back to LDS
  if (lane <= nj) {
#pragma unroll
    for (int r = 0; r < IM; ++r) S[lane * LD + r] = A_[r];
  }
  __syncthreads();
  T mx = T(0);
  for (int q = lane; q < nj * nj; q += 64) {
    const int r = q % nj, c = q / nj;
    if (r <= c) {
      T v = S[c * LD + r];
      v = v < T(0) ? -v : v;
      mx = v > mx ? v : mx;
    }
  }
  const T maxR = wave_max(mx);
  // back substitution, column oriented: y in B[0:nj]
  for (int i = nj - 1; i >= 0; --i) {
    __syncthreads();
    const T pi = B[i] / S[i * LD + i];
    __syncthreads();
    if (lane == 0) B[i] = pi;
    if (lane < i) B[lane] -= S[i * LD + lane] * pi;
  }
  __syncthreads();
  T rr = T(0);
  for (int li = nj + lane; li < ni; li += 64) rr += B[li] * B[li];
  rr = wave_sum(rr);
  if (lane < nj) a.out[a.Pslot[jb + lane]] = (double)B[lane];
  if (lane == 0) {
    a.rho[j] = sqrt((double)rr);
    const bool singular = (ni < nj) || !(minDiag > T(10.0 * ni * Eps<T>::v) * maxR);
    if (singular) atomicMin(a.bad_col, j);
  }
}

// The same with two columns per 64-lane workgroup for |J| <= 16 (the (16, 64)
// bucket): lanes 32 g .. 32 g + 31 work on the workgroup's column g, each half
// with its own LDS block; the halves share the barriers, so the reflector loop
// runs to the larger |J| of the two and each half works while k is below its own.
template <typename T, bool Q16 = false, bool MULTI = false>
__global__ __launch_bounds__(64) void k_spai_col2(LsArgs a0) {
  static_assert(sizeof(T) == 4, "four-byte values");
  constexpr int JM = 16, IM = 64, LD = IM + 1;
  __shared__ T S[2][(JM + 1) * LD];
  __shared__ int Is[2][IM];
  __shared__ T sv[2][IM];
  const int lane = threadIdx.x, g = lane >> 5, gl = lane & 31;
  const int wid = xcd_swizzle(blockIdx.x, gridDim.x) * 2 + g;
  bool valid = wid < a0.ncols;
  LsArgs a = a0;
  int wl = wid;
  if (MULTI && valid) {
    const int sy = ls_system(a0.seg, a0.nsys, wid);
    a = a0.sys[sy];
    wl = wid - a0.seg[sy];
    valid = wl < a.ncols;
  }
  int j = 0, jb = 0, nj = 0, ni = 0;
  int64_t ib = 0;
  if (valid) {
    j = a.cols ? a.cols[wl] : a.col_off + wl;
    jb = a.Jcolptr[j];
    nj = a.Jcolptr[j + 1] - jb;
    ib = a.Icolptr[j];
    ni = (int)(a.Icolptr[j + 1] - ib);
  }
  const int njmax = max(__builtin_amdgcn_readlane(nj, 0), __builtin_amdgcn_readlane(nj, 32));
  if (njmax == 0) return;  // both halves empty (a column always holds its diagonal)
  T* Sg = S[g];
  int* Ig = Is[g];
  for (int li = gl; li < ni; li += 32) Ig[li] = a.Irow[ib + li];
  for (int q = gl; q < (JM + 1) * LD; q += 32) Sg[q] = T(0);
  __syncthreads();
  if (gl < nj) {
    const int c = a.Jrow[jb + gl];
    T* colt = Sg + gl * LD;
    int q = 0;
    for (int e = a.Acolptr[c]; e < a.Acolptr[c + 1]; ++e) {
      const int r = a.Arowidx[e];
      q += lds_lower_bound(Ig + q, ni - q, r);
      colt[q] = (T)a.aval[a.Acscslot[e]];
    }
  }
  T* B = Sg + nj * LD;
  if (valid) {
    if (a.rhs_aval) {
      for (int e = a.Acolptr[j] + gl; e < a.Acolptr[j + 1]; e += 32)
        B[lds_lower_bound(Ig, ni, a.Arowidx[e])] = (T)a.rhs_aval[a.Acscslot[e]];
    } else if (gl == 0) {
      B[lds_lower_bound(Ig, ni, j)] = T(1);
    }
  }
  __syncthreads();
  const int cl = gl <= nj ? gl : nj;
  T A_[IM];
#pragma unroll
  for (int r = 0; r < IM; ++r) A_[r] = Sg[cl * LD + r];
  if constexpr (Q16) {
    if (valid && (gl < nj || (gl == nj && a.rhs_aval))) {
      T mx = T(0);
#pragma unroll
      for (int r = 0; r < IM; ++r) mx = fmaxf(mx, fabsf(A_[r]));
      const Q16Scale q = q16_scale(mx);
#pragma unroll
      for (int r = 0; r < IM; ++r) A_[r] = q16(A_[r], q);
    }
  }
  T minDiag = T(3.0e38);
#pragma unroll
  for (int k = 0; k < JM; ++k) {
    if (k < njmax) {
      const bool act = k < nj;  // this half still reflects
      if (act && gl == k) {
#pragma unroll
        for (int r = k; r < IM; ++r) sv[g][r] = A_[r];
      }
      __syncthreads();
      if (act) {
        T x[IM];
        T dot = T(0);
#pragma unroll
        for (int r = k; r < IM; ++r) {
          x[r] = sv[g][r];
          dot += x[r] * A_[r];
        }
        const T s0 = readlane_f(dot, k), s1 = readlane_f(dot, 32 + k);
        const T sig = g ? s1 : s0;
        const T alpha = x[k];
        T beta = alpha;
        if (sig != alpha * alpha) {
          const T nrm = sqrt(sig);
          beta = (alpha >= T(0)) ? -nrm : nrm;
          const T denom = beta * (beta - alpha);
          if (gl > k) {
            const T f = (dot - beta * A_[k]) / denom;
            A_[k] -= f * (alpha - beta);
#pragma unroll
            for (int r = k + 1; r < IM; ++r) A_[r] -= f * x[r];
          }
        }
        if (gl == k) {
          A_[k] = beta;
#pragma unroll
          for (int r = k + 1; r < IM; ++r) A_[r] = T(0);
        }
        const T ab = beta < T(0) ? -beta : beta;
        minDiag = ab < minDiag ? ab : minDiag;
      }
      __syncthreads();
    }
  }
  if (valid && gl <= nj) {
#pragma unroll
    for (int r = 0; r < IM; ++r) Sg[gl * LD + r] = A_[r];
  }
  __syncthreads();
  T mx = T(0);
  for (int q = gl; q < nj * nj; q += 32) {
    const int r = q % nj, c = q / nj;
    if (r <= c) {
      T v = Sg[c * LD + r];
      v = v < T(0) ? -v : v;
      mx = v > mx ? v : mx;
    }
  }
  // the maximum over each half's 32 lanes
  for (int o = 16; o >= 1; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
  const T maxR = mx;
  for (int i = njmax - 1; i >= 0; --i) {
    __syncthreads();
    const T pi = i < nj ? B[i] / Sg[i * LD + i] : T(0);
    __syncthreads();
    if (i < nj) {
      if (gl == 0) B[i] = pi;
      if (gl < i) B[gl] -= Sg[i * LD + gl] * pi;
    }
  }
  __syncthreads();
  T rr = T(0);
  for (int li = nj + gl; li < ni; li += 32) rr += B[li] * B[li];
  for (int o = 16; o >= 1; o >>= 1) rr += __shfl_xor(rr, o, 64);
  if (!valid) return;
  if (gl < nj) a.out[a.Pslot[jb + gl]] = (double)B[gl];
  if (gl == 0) {
    a.rho[j] = sqrt((double)rr);
    const bool singular = (ni < nj) || !(minDiag > T(10.0 * ni * Eps<T>::v) * maxR);
    if (singular) atomicMin(a.bad_col, j);
  }
}

// columns per wavefront of bucket b's kernel for values of sizeof(T) bytes
// (a launch over several systems pads each system's count to a multiple)
static int bucket_cpw(int b, int tsize) {
  if (tsize == 4 && b == 5) return 1;  // the column-owner kernels
  if (tsize == 4 && b == 3) return 2;
  if (b <= 4) return 4;
  if (tsize == 4 && (b == 5 || b == 6)) return 2;
  return 1;
}

template <typename T, bool Q16 = false, bool GO = false, bool MULTI = false>
static int launch_bucket(int b, LsArgs a, int maxJ, int maxI, hipStream_t st, pmor_ctx* pc, int pidx, int part) {
  if (a.ncols == 0) return PMOR_OK;
  const unsigned g16 = (unsigned)((a.ncols + 15) / 16);  // 16 columns per workgroup
  const unsigned g32 = (unsigned)((a.ncols + 7) / 8);    // 8 columns (of 32 lanes) per workgroup
  // |J| <= 32 with |I| <= 128 in registers for 4-byte values; FP64 would need
  // 256 registers for the block, so it takes the LDS kernel
  constexpr bool REG32 = sizeof(T) == 4;
  switch (b) {
    case 0: plaunch(pc, pidx, part, k_spai_reg<T, 8, 1, Q16, 16, GO, MULTI>, dim3(g16), dim3(256), 0, st, a); break;
    case 1: plaunch(pc, pidx, part, k_spai_reg<T, 8, 2, Q16, 16, GO, MULTI>, dim3(g16), dim3(256), 0, st, a); break;
    case 2: plaunch(pc, pidx, part, k_spai_reg<T, 8, 4, Q16, 16, GO, MULTI>, dim3(g16), dim3(256), 0, st, a); break;
    case 3:
      if constexpr (REG32 && !GO) {
        plaunch(pc, pidx, part, k_spai_col2<T, Q16, MULTI>, dim3((unsigned)((a.ncols + 1) / 2)), dim3(64), 0, st, a);
        break;
      }
      plaunch(pc, pidx, part, k_spai_reg<T, 16, 4, Q16, 16, GO, MULTI>, dim3(g16), dim3(256), 0, st, a);
      break;
    case 4: plaunch(pc, pidx, part, k_spai_reg<T, 16, 8, Q16, 16, GO, MULTI>, dim3(g16), dim3(256), 0, st, a); break;
    case 5:
      if constexpr (REG32 && !GO) {
        plaunch(pc, pidx, part, k_spai_col<T, 32, Q16, MULTI>, dim3((unsigned)a.ncols), dim3(64), 0, st, a);
        break;
      }
      if constexpr (REG32) {
        plaunch(pc, pidx, part, k_spai_reg<T, 32, 2, Q16, 32, GO, MULTI>, dim3(g32), dim3(256), 0, st, a);
        break;
      }
      [[fallthrough]];
    case 6:
      if constexpr (REG32) {
        plaunch(pc, pidx, part, k_spai_reg<T, 32, 4, Q16, 32, GO, MULTI>, dim3(g32), dim3(256), 0, st, a);
        break;
      }
      [[fallthrough]];
    case 7:  // |J| <= 64 with |I| <= 128: the LDS kernel (measured faster than a 64-lane register form,
             // whose 64-column block left 2 waves per SIMD and spilled scalar registers)
      [[fallthrough]];
    case 8: {
      const int ldI = ((maxI + 7) / 8) * 8;
      const size_t shm = sizeof(T) * (size_t)(maxJ + 1) * ldI + sizeof(int) * (size_t)ldI;
      if (shm > 150 * 1024) return fail(PMOR_EINVAL, "SPAI pattern too large for the LDS least-squares kernel");
      PMOR_TRY(allow_lds((const void*)k_spai_lds<T, Q16, GO, MULTI>, shm));
      plaunch(pc, pidx, part, k_spai_lds<T, Q16, GO, MULTI>, dim3((unsigned)a.ncols), dim3(64 * LDS_NW), (uint32_t)shm, st, a,
              ldI, maxJ);
      break;
    }
    default: return fail(PMOR_EINVAL, "column outside the supported SPAI pattern sizes");
  }
  PMOR_HIP(hipGetLastError());
  return PMOR_OK;
}

__global__ void k_sumsq_partials(const double* x, int64_t n, double* part) {
  __shared__ double s[4];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    acc += x[i] * x[i];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = s[0] + s[1] + s[2] + s[3];
}

// out = sum of part[0..np), np <= 256, by a fixed tree (one workgroup of 256)
__global__ __launch_bounds__(256) void k_sum_in_order(const double* part, int np, double* out) {
  __shared__ double s[256];
  s[threadIdx.x] = (int)threadIdx.x < np ? part[threadIdx.x] : 0.0;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s[0];
}

// sum of squares of x[0..n), deterministic; result left in dev_scratch[0]
int sumsq(const double* x, int64_t n, double* dev_scratch, hipStream_t st) {
  const int np = 256;
  hipLaunchKernelGGL(k_sumsq_partials, dim3(np), dim3(256), 0, st, x, n, dev_scratch + 1);
  hipLaunchKernelGGL(k_sum_in_order, dim3(1), dim3(256), 0, st, dev_scratch + 1, np, dev_scratch);
  PMOR_HIP(hipGetLastError());
  return PMOR_OK;
}

int run_spai_ls(pmor_spai* h, const double* aval, const double* rhs_aval, double* out_val, int32_t* bad_col,
                double* fro2) {
  pmor_problem* pb = h->pb;
  hipStream_t st = pb->ctx->stream;
  int* dbad = reinterpret_cast<int*>(h->red);
  const int big = 0x7fffffff;
  PMOR_TRY(set_device_int(dbad, big, st));
  LsArgs a{};
  a.rowptr = pb->rowptr; a.colidx = pb->col; a.aval = aval; a.rhs_aval = rhs_aval;
  a.Jcolptr = h->Jcolptr; a.Jrow = h->Jrow; a.Icolptr = h->Icolptr; a.Irow = h->Irow;
  a.Pslot = h->Pslot; a.out = out_val; a.rho = h->rho; a.bad_col = dbad;
  a.Acolptr = pb->colptr; a.Arowidx = pb->rowidx; a.Acscslot = pb->cscslot;
  const int pr = prof_start(pb->ctx, PMOR_PROF_SPAI_LS);
  int first_b = -1, last_b = -1;
  for (int b = 0; b < LS_BUCKETS; ++b)
    if (h->bucket_count[b]) { if (first_b < 0) first_b = b; last_b = b; }
  for (int b = 0; b < LS_BUCKETS; ++b) {
    if (h->bucket_count[b] == 0) continue;
    const int part = (b == first_b ? 1 : 0) | (b == last_b ? 2 : 0);
    a.ncols = h->bucket_count[b];
    if (h->identity_order) { a.cols = nullptr; a.col_off = 0; }  // every column sits in bucket b
    else { a.cols = h->bucket_cols + h->bucket_off[b]; a.col_off = 0; }
    const int mj = h->bucket_maxJ[b], mi = h->bucket_maxI[b];
    if (h->opts.precision == PMOR_F32) PMOR_TRY(launch_bucket<float>(b, a, mj, mi, st, pb->ctx, pr, part));
    else if (h->opts.precision == PMOR_F16S)
      PMOR_TRY((launch_bucket<float, true>(b, a, mj, mi, st, pb->ctx, pr, part)));
    else PMOR_TRY(launch_bucket<double>(b, a, mj, mi, st, pb->ctx, pr, part));
  }
  prof_stop(pb->ctx, pr,
            12.0 * pb->nnz + 4.0 * pb->n + 4.0 * ((double)h->nI + h->nnzP) + 8.0 * h->nnzP + 8.0 * pb->n, 0);
  if (bad_col || fro2) {
    double* dsum = h->red + 1;
    PMOR_TRY(sumsq(h->rho, pb->n, dsum, st));
    int hbad = big;
    double hs = 0.0;
    PMOR_HIP(hipMemcpyAsync(&hbad, dbad, sizeof(int), hipMemcpyDeviceToHost, st));
    PMOR_HIP(hipMemcpyAsync(&hs, dsum, sizeof(double), hipMemcpyDeviceToHost, st));
    PMOR_HIP(hipStreamSynchronize(st));
    if (bad_col) *bad_col = (hbad == big) ? -1 : hbad;
    if (fro2) *fro2 = hs;
  }
  return PMOR_OK;
}

// The least squares of several preconditioners in shared launches (Section 2.2:
// every column is a problem of its own, whichever system it belongs to): per
// bucket one launch over that bucket's columns of all systems, each system's
// count padded to whole wavefronts so that a wavefront's columns share one
// system.  hs: the handles (one stream, one precision); aval[i]: the values of
// system i's matrix; results into each handle's P1val, rho and bad column
// (its red[0], set here).
int run_spai_ls_multi(pmor_spai* const* hs, int count, const double* const* aval, hipStream_t st) {
  if (count <= 0) return PMOR_OK;
  const int prec = hs[0]->opts.precision;
  const int tsize = prec == PMOR_F64 ? 8 : 4;
  std::vector<LsArgs> base(count);
  for (int i = 0; i < count; ++i) {
    pmor_spai* h = hs[i];
    pmor_problem* pb = h->pb;
    if (h->opts.precision != prec) return fail(PMOR_EINVAL, "a batch of least squares takes one precision");
    int* dbad = reinterpret_cast<int*>(h->red);
    PMOR_TRY(set_device_int(dbad, 0x7fffffff, st));
    LsArgs& a = base[i];
    a = LsArgs{};
    a.rowptr = pb->rowptr; a.colidx = pb->col; a.aval = aval[i]; a.rhs_aval = nullptr;
    a.Jcolptr = h->Jcolptr; a.Jrow = h->Jrow; a.Icolptr = h->Icolptr; a.Irow = h->Irow;
    a.Pslot = h->Pslot; a.out = h->P1val; a.rho = h->rho; a.bad_col = dbad;
    a.Acolptr = pb->colptr; a.Arowidx = pb->rowidx; a.Acscslot = pb->cscslot;
  }
  // per bucket: the systems' descriptions and the padded column offsets, packed
  // into one device buffer
  struct BucketLaunch {
    int b, nsys, total, maxJ, maxI;
    size_t off_sys, off_seg;
  };
  std::vector<BucketLaunch> bl;
  std::vector<unsigned char> host;
  auto align16 = [](size_t x) { return (x + 15) & ~size_t(15); };
  for (int b = 0; b < LS_BUCKETS; ++b) {
    std::vector<LsArgs> sys;
    std::vector<int32_t> seg{0};
    int mj = 0, mi = 0;
    const int cpw = bucket_cpw(b, tsize);
    for (int i = 0; i < count; ++i) {
      const pmor_spai* h = hs[i];
      const int cnt = h->bucket_count[b];
      if (cnt == 0) continue;
      LsArgs a = base[i];
      a.ncols = cnt;
      a.cols = h->identity_order ? nullptr : h->bucket_cols + h->bucket_off[b];
      a.col_off = 0;
      sys.push_back(a);
      const int64_t next = (int64_t)seg.back() + (cnt + cpw - 1) / cpw * cpw;
      if (next >= ((int64_t)1 << 31)) return fail(PMOR_EINVAL, "too many least-squares columns in one batch");
      seg.push_back((int32_t)next);
      mj = std::max(mj, h->bucket_maxJ[b]);
      mi = std::max(mi, h->bucket_maxI[b]);
    }
    if (sys.empty()) continue;
    BucketLaunch L{b, (int)sys.size(), seg.back(), mj, mi, 0, 0};
    L.off_sys = align16(host.size());
    host.resize(L.off_sys + sizeof(LsArgs) * sys.size());
    std::memcpy(host.data() + L.off_sys, sys.data(), sizeof(LsArgs) * sys.size());
    L.off_seg = align16(host.size());
    host.resize(L.off_seg + sizeof(int32_t) * seg.size());
    std::memcpy(host.data() + L.off_seg, seg.data(), sizeof(int32_t) * seg.size());
    bl.push_back(L);
  }
  if (bl.empty()) return PMOR_OK;
  unsigned char* dev = nullptr;
  PMOR_HIP(dmalloc((void**)&dev, host.size(), st));
  // the descriptions are read by the launches below: a blocking copy, so the
  // host buffer may go when this function returns
  if (hipMemcpyAsync(dev, host.data(), host.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    dfree(dev, st);
    return fail(PMOR_EHIP, "copy of the batch descriptions failed");
  }
  int rc = PMOR_OK;
  pmor_ctx* ctx = hs[0]->pb->ctx;
  const int pr = prof_start(ctx, PMOR_PROF_SPAI_LS);
  double bytes = 0.0;  // the systems' least-squares bytes, as run_spai_ls counts them
  for (int i = 0; i < count; ++i) {
    const pmor_spai* h = hs[i];
    const pmor_problem* pb = h->pb;
    bytes += 12.0 * pb->nnz + 4.0 * pb->n + 4.0 * ((double)h->nI + h->nnzP) + 8.0 * h->nnzP + 8.0 * pb->n;
  }
  for (size_t t = 0; t < bl.size(); ++t) {
    const BucketLaunch& L = bl[t];
    const int part = (t == 0 ? 1 : 0) | (t + 1 == bl.size() ? 2 : 0);
    LsArgs a0{};
    a0.ncols = L.total;
    a0.sys = reinterpret_cast<const LsArgs*>(dev + L.off_sys);
    a0.seg = reinterpret_cast<const int32_t*>(dev + L.off_seg);
    a0.nsys = L.nsys;
    if (prec == PMOR_F32) rc = launch_bucket<float, false, false, true>(L.b, a0, L.maxJ, L.maxI, st, ctx, pr, part);
    else if (prec == PMOR_F16S) rc = launch_bucket<float, true, false, true>(L.b, a0, L.maxJ, L.maxI, st, ctx, pr, part);
    else rc = launch_bucket<double, false, false, true>(L.b, a0, L.maxJ, L.maxI, st, ctx, pr, part);
    if (rc != PMOR_OK) break;
  }
  prof_stop(ctx, pr, bytes, 0);
  dfree(dev, st);  // stream-ordered: reused only after the launches
  return rc;
}

// ---------------------------------------------------------------------------
// U-diag update: q_i = <A(l) e_i, a e_i> / ||A(l) e_i||^2 against the anchor a
// (A(1) for the first approach, A(l-1) for the second), and P_l = diag(q) P_1.
// qprev (second approach): the running row scale of the previous update, so
// that q holds qprev_i q_i and P_l = diag(qprev q) P_1 = diag(q) P_{l-1}.  rho:
// the step's own residual ||a e_i - q_i A(l) e_i||.  (P_l written only when Pl
// is not NULL; the engine can also apply the factors.)
// ---------------------------------------------------------------------------
__global__ void k_update_diag(int n, const int32_t* colptr, const int32_t* cscslot, const double* al,
                              const double* a1, const double* qprev, const int32_t* Prowptr, const double* P1,
                              double* Pl, double* q, double* rho, int* bad_col) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double num = 0.0, den = 0.0;
  for (int e = colptr[i]; e < colptr[i + 1]; ++e) {
    const int s = cscslot[e];
    const double x = al[s], y = a1[s];
    num += x * y;
    den += x * x;
  }
  const double qi = num / den;
  if (!(den > 0.0)) atomicMin(bad_col, i);
  const double qe = qprev ? qprev[i] * qi : qi;
  q[i] = qe;
  // ||a e_i - q_i A(l) e_i|| summed entry by entry once q_i is known (the
  // expanded form ||a e_i||^2 - 2 q num + q^2 den cancels when the fit is
  // tight)
  double r2 = 0.0;
  for (int e = colptr[i]; e < colptr[i + 1]; ++e) {
    const int s = cscslot[e];
    const double d = a1[s] - qi * al[s];
    r2 += d * d;
  }
  rho[i] = sqrt(r2);
  if (Pl)
    for (int e = Prowptr[i]; e < Prowptr[i + 1]; ++e) Pl[e] = qe * P1[e];
}

int launch_update_diag(pmor_spai* h, const double* aval_l, const double* anchor, const double* qprev, double* pl,
                       double* q, double* rho, int* dbad) {
  pmor_problem* pb = h->pb;
  const int n = pb->n;
  if (n == 0) return PMOR_OK;
  hipLaunchKernelGGL(k_update_diag, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, pb->ctx->stream, n, pb->colptr,
                     pb->cscslot, aval_l, anchor, qprev, h->Prowptr, h->P1val, pl, q, rho, dbad);
  PMOR_HIP(hipGetLastError());
  return PMOR_OK;
}

__global__ void k_copy_vals(const double* __restrict__ a, double* __restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

// Gather only: every column's block A(I_j, J_j) of the anchor values, read as
// the FP64 least-squares kernels read it, reduced to its sum in colsum[j] (a
// data-movement variant of the least squares, for timing and parity)
int run_spai_gather(pmor_spai* h, double* colsum) {
  pmor_problem* pb = h->pb;
  hipStream_t st = pb->ctx->stream;
  LsArgs a{};
  a.rowptr = pb->rowptr; a.colidx = pb->col; a.aval = h->aval1; a.rhs_aval = nullptr;
  a.Jcolptr = h->Jcolptr; a.Jrow = h->Jrow; a.Icolptr = h->Icolptr; a.Irow = h->Irow;
  a.Pslot = h->Pslot; a.out = nullptr; a.rho = colsum; a.bad_col = nullptr;
  a.Acolptr = pb->colptr; a.Arowidx = pb->rowidx; a.Acscslot = pb->cscslot;
  const int pr = prof_start(pb->ctx, PMOR_PROF_SPAI_GATHER);
  int first_b = -1, last_b = -1;
  for (int b = 0; b < LS_BUCKETS; ++b)
    if (h->bucket_count[b]) { if (first_b < 0) first_b = b; last_b = b; }
  for (int b = 0; b < LS_BUCKETS; ++b) {
    if (h->bucket_count[b] == 0) continue;
    const int part = (b == first_b ? 1 : 0) | (b == last_b ? 2 : 0);
    a.ncols = h->bucket_count[b];
    a.cols = h->identity_order ? nullptr : h->bucket_cols + h->bucket_off[b];
    a.col_off = 0;
    PMOR_TRY((launch_bucket<double, false, true>(b, a, h->bucket_maxJ[b], h->bucket_maxI[b], st, pb->ctx, pr, part)));
  }
  // the algorithmic bytes of a gather: A once, the index sets, the sums written
  prof_stop(pb->ctx, pr, 12.0 * pb->nnz + 4.0 * pb->n + 4.0 * ((double)h->nI + h->nnzP) + 8.0 * pb->n, 0);
  return PMOR_OK;
}

int run_update_diag(pmor_spai* h, const double* aval_l, int32_t* bad_col, double* fro2) {
  pmor_problem* pb = h->pb;
  hipStream_t st = pb->ctx->stream;
  const int n = pb->n;
  int* dbad = reinterpret_cast<int*>(h->red);
  const int big = 0x7fffffff;
  PMOR_TRY(set_device_int(dbad, big, st));
  // the second approach chains the scales and moves the anchor (aval1) to A(l)
  const bool second = h->opts.approach == PMOR_APPROACH_SECOND;
  PMOR_TRY(launch_update_diag(h, aval_l, h->aval1, second ? h->Qval : nullptr, h->Pval, h->Qval, h->rho, dbad));
  if (second) {
    const unsigned g = (unsigned)std::min<int64_t>((pb->nnz + 255) / 256, 4096);
    if (pb->nnz > 0) hipLaunchKernelGGL(k_copy_vals, dim3(g), dim3(256), 0, st, aval_l, h->aval1, (int64_t)pb->nnz);
    PMOR_HIP(hipGetLastError());
  }
  if (bad_col || fro2) {
    double* dsum = h->red + 1;
    PMOR_TRY(sumsq(h->rho, n, dsum, st));
    double hs = 0.0;
    int hbad = big;
    PMOR_HIP(hipMemcpyAsync(&hs, dsum, sizeof(double), hipMemcpyDeviceToHost, st));
    PMOR_HIP(hipMemcpyAsync(&hbad, dbad, sizeof(int), hipMemcpyDeviceToHost, st));
    PMOR_HIP(hipStreamSynchronize(st));
    if (fro2) *fro2 = hs;
    if (bad_col) *bad_col = (hbad == big) ? -1 : hbad;
  }
  return PMOR_OK;
}

// ---------------------------------------------------------------------------
// U-diag update of a complex problem in its equivalent real form.  The factor
// of complex column i is the complex q_i = <A(l) e_i, A(1) e_i> / ||A(l) e_i||^2
// (first approach, Section 2.3); in the real form it is the 2x2 block
// [[a, -b], [b, a]] (q_i = a + b sqrt(-1)) on rows and columns 2i, 2i+1, and
// with c0, c1 the real columns 2i, 2i+1 of A(l) (c1 the rotation of c0) and t
// the real column 2i of A(1): a = <c0, t> / ||c0||^2, b = <c1, t> / ||c0||^2.
// The pattern is block-closed, so the two columns hold the same rows in the
// same order, and rows 2i, 2i+1 of P the same columns.  q[2i] = a,
// q[2i+1] = b; rho of both real columns, entry by entry; P_l = Q P_1 written
// out: row 2i = a P_1(2i,:) - b P_1(2i+1,:), row 2i+1 = b P_1(2i,:) + a P_1(2i+1,:).
// ---------------------------------------------------------------------------
__global__ void k_update_pair(int m, const int32_t* colptr, const int32_t* cscslot, const double* al,
                              const double* a1, const int32_t* Prowptr, const double* P1, double* Pl, double* q,
                              double* rho, int* bad_col) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int c0 = 2 * i, c1 = 2 * i + 1;
  const int e0 = colptr[c0], e1 = colptr[c1], len = e1 - e0;
  double nre = 0.0, nim = 0.0, den = 0.0;
  for (int k = 0; k < len; ++k) {
    const int s0 = cscslot[e0 + k], s1 = cscslot[e1 + k];
    const double x0 = al[s0], x1 = al[s1], y0 = a1[s0];
    nre += x0 * y0;
    nim += x1 * y0;
    den += x0 * x0;
  }
  const double a = nre / den, b = nim / den;
  if (!(den > 0.0)) atomicMin(bad_col, c0);
  q[c0] = a;
  q[c1] = b;
  double r0 = 0.0, r1 = 0.0;
  for (int k = 0; k < len; ++k) {
    const int s0 = cscslot[e0 + k], s1 = cscslot[e1 + k];
    const double x0 = al[s0], x1 = al[s1];
    const double d0 = a1[s0] - (a * x0 + b * x1);
    const double d1 = a1[s1] - (a * x1 - b * x0);
    r0 += d0 * d0;
    r1 += d1 * d1;
  }
  rho[c0] = sqrt(r0);
  rho[c1] = sqrt(r1);
  const int p0 = Prowptr[c0], p1 = Prowptr[c1], plen = p1 - p0;
  for (int k = 0; k < plen; ++k) {
    const double u = P1[p0 + k], w = P1[p1 + k];
    Pl[p0 + k] = a * u - b * w;
    Pl[p1 + k] = b * u + a * w;
  }
}

int run_update_pair(pmor_spai* h, const double* aval_l, double* pl, double* q, double* rho, int32_t* bad_col,
                    double* fro2) {
  pmor_problem* pb = h->pb;
  hipStream_t st = pb->ctx->stream;
  const int n = pb->n, m = n / 2;
  int* dbad = reinterpret_cast<int*>(h->red);
  const int big = 0x7fffffff;
  PMOR_TRY(set_device_int(dbad, big, st));
  if (m > 0) {
    hipLaunchKernelGGL(k_update_pair, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, m, pb->colptr,
                       pb->cscslot, aval_l, h->aval1, h->Prowptr, h->P1val, pl, q, rho, dbad);
    PMOR_HIP(hipGetLastError());
  }
  if (bad_col || fro2) {
    double* dsum = h->red + 1;
    PMOR_TRY(sumsq(rho, n, dsum, st));
    double hs = 0.0;
    int hbad = big;
    PMOR_HIP(hipMemcpyAsync(&hs, dsum, sizeof(double), hipMemcpyDeviceToHost, st));
    PMOR_HIP(hipMemcpyAsync(&hbad, dbad, sizeof(int), hipMemcpyDeviceToHost, st));
    PMOR_HIP(hipStreamSynchronize(st));
    if (fro2) *fro2 = hs;
    if (bad_col) *bad_col = (hbad == big) ? -1 : hbad;
  }
  return PMOR_OK;
}

// ---------------------------------------------------------------------------
// Adaptive update pattern: every column first takes its U-diag factor q_i;
// a column whose diagonal misfit ||A(1) e_i - q_i A(l) e_i|| exceeds
// ep ||A(1) e_i|| (or is not finite) is escalated to the SPAI pattern J_i, the
// U-pattern least squares with right-hand side A(1) e_i.  Q in P's CSR order: a
// kept column holds q_i on its diagonal and zeros elsewhere, an escalated
// column the least-squares values.
// ---------------------------------------------------------------------------
__global__ void k_update_adaptive_diag(int n, const int32_t* colptr, const int32_t* cscslot, const double* al,
                                       const double* a1, double ep, const int32_t* Jcolptr, const int32_t* Jrow,
                                       const int32_t* Pslot, double* qout, double* rho, int* esc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double num = 0.0, den = 0.0, n11 = 0.0;
  for (int e = colptr[i]; e < colptr[i + 1]; ++e) {
    const int s = cscslot[e];
    const double x = al[s], y = a1[s];
    num += x * y;
    den += x * x;
    n11 += y * y;
  }
  const double qi = num / den;
  double r2 = 0.0;  // entry by entry, as in k_update_diag
  for (int e = colptr[i]; e < colptr[i + 1]; ++e) {
    const int s = cscslot[e];
    const double d = a1[s] - qi * al[s];
    r2 += d * d;
  }
  const double r = sqrt(r2);
  const bool up = !(r <= ep * sqrt(n11));
  esc[i] = up ? 1 : 0;
  rho[i] = up ? 0.0 : r;
  for (int e = Jcolptr[i]; e < Jcolptr[i + 1]; ++e) qout[Pslot[e]] = (!up && Jrow[e] == i) ? qi : 0.0;
}

// the escalated columns of a bucket (column list, or 0..cnt-1 when NULL) into
// out[0..*count); their order follows the atomics, and every column is solved
// on its own, so the values do not depend on it
__global__ void k_compact_cols(int cnt, const int32_t* cols, const int* esc, int32_t* out, int* count) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cnt) return;
  const int c = cols ? cols[j] : j;
  if (esc[c]) out[atomicAdd(count, 1)] = c;
}

__global__ void k_zero_ints(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

int run_update_adaptive(pmor_spai* h, const double* aval_l, double* qout, int32_t* bad_col, double* fro2,
                        int64_t* n_esc) {
  pmor_problem* pb = h->pb;
  hipStream_t st = pb->ctx->stream;
  const int n = pb->n;
  int* dbad = reinterpret_cast<int*>(h->red);
  const int big = 0x7fffffff;
  PMOR_TRY(set_device_int(dbad, big, st));
  int* flags = h->esc_list + n;
  if (n > 0)
    hipLaunchKernelGGL(k_update_adaptive_diag, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, pb->colptr,
                       pb->cscslot, aval_l, h->aval1, h->opts.adapt_ep, h->Jcolptr, h->Jrow, h->Pslot, qout, h->rho,
                       flags);
  hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, st, h->esc_cnt, BUCKET_SLOTS);
  for (int b = 0; b < LS_BUCKETS; ++b) {
    const int cnt = h->bucket_count[b];
    if (cnt == 0) continue;
    const int32_t* cols = h->identity_order ? nullptr : h->bucket_cols + h->bucket_off[b];
    const int off = h->identity_order ? 0 : h->bucket_off[b];
    hipLaunchKernelGGL(k_compact_cols, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, cnt, cols, flags,
                       h->esc_list + off, h->esc_cnt + b);
  }
  PMOR_HIP(hipGetLastError());
  int hc[BUCKET_SLOTS] = {0};
  PMOR_HIP(hipMemcpyAsync(hc, h->esc_cnt, sizeof(int) * BUCKET_SLOTS, hipMemcpyDeviceToHost, st));
  PMOR_HIP(hipStreamSynchronize(st));
  int64_t tot = 0;
  LsArgs a{};
  a.rowptr = pb->rowptr; a.colidx = pb->col; a.aval = aval_l; a.rhs_aval = h->aval1;
  a.Jcolptr = h->Jcolptr; a.Jrow = h->Jrow; a.Icolptr = h->Icolptr; a.Irow = h->Irow;
  a.Pslot = h->Pslot; a.out = qout; a.rho = h->rho; a.bad_col = dbad;
  a.Acolptr = pb->colptr; a.Arowidx = pb->rowidx; a.Acscslot = pb->cscslot;
  for (int b = 0; b < LS_BUCKETS; ++b) {
    if (hc[b] == 0) continue;
    tot += hc[b];
    a.ncols = hc[b];
    a.cols = h->esc_list + (h->identity_order ? 0 : h->bucket_off[b]);
    a.col_off = 0;
    const int mj = h->bucket_maxJ[b], mi = h->bucket_maxI[b];
    if (h->opts.precision == PMOR_F32) PMOR_TRY(launch_bucket<float>(b, a, mj, mi, st, pb->ctx, -1, 0));
    else if (h->opts.precision == PMOR_F16S)
      PMOR_TRY((launch_bucket<float, true>(b, a, mj, mi, st, pb->ctx, -1, 0)));
    else PMOR_TRY(launch_bucket<double>(b, a, mj, mi, st, pb->ctx, -1, 0));
  }
  if (n_esc) *n_esc = tot;
  if (bad_col || fro2) {
    double* dsum = h->red + 1;
    PMOR_TRY(sumsq(h->rho, n, dsum, st));
    int hbad = big;
    double hs = 0.0;
    PMOR_HIP(hipMemcpyAsync(&hbad, dbad, sizeof(int), hipMemcpyDeviceToHost, st));
    PMOR_HIP(hipMemcpyAsync(&hs, dsum, sizeof(double), hipMemcpyDeviceToHost, st));
    PMOR_HIP(hipStreamSynchronize(st));
    if (bad_col) *bad_col = (hbad == big) ? -1 : hbad;
    if (fro2) *fro2 = hs;
  }
  return PMOR_OK;
}

// ---------------------------------------------------------------------------
// assembly: a = sum_r c_r T_r on the union pattern (streaming)
// ---------------------------------------------------------------------------
struct Coefs {
  double c[PMOR_TMAX];
  int nt;
};

__global__ void k_assemble(int64_t nnz, const double* __restrict__ tval, Coefs cf, double* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int t = 0; t < cf.nt; ++t) acc += cf.c[t] * tval[(int64_t)t * nnz + e];
    out[e] = acc;
  }
}

int launch_assemble(pmor_problem* pb, const Point& pt, double* out, hipStream_t st) {
  Coefs cf{};
  cf.nt = pb->nterms;
  for (int t = 0; t < pb->nterms; ++t) cf.c[t] = pt.c[t];
  const int64_t nnz = pb->nnz;
  if (nnz == 0) return PMOR_OK;
  unsigned g = (unsigned)std::min<int64_t>((nnz + 255) / 256, 4096);
  hipLaunchKernelGGL(k_assemble, dim3(g), dim3(256), 0, st, nnz, pb->tval, cf, out);
  PMOR_HIP(hipGetLastError());
  return PMOR_OK;
}

// ---------------------------------------------------------------------------
// the points of a sequence, PTS_MAX per launch: A(l) (into the CSR order or
// straight into the sliced ELL layout) and the U-diag factors, with the term
// values read once for all points of the launch.  A(l) is formed exactly as by
// k_assemble (same terms, same order), so the results match the one-point
// calls bit for bit.
// ---------------------------------------------------------------------------
struct PtsCoefs {
  double c[PTS_MAX][PMOR_TMAX];  // by term slot
  int cnt, nt;
};

// the anchor point and up to PTS_MAX points of a second-approach chain
struct ChainCoefs {
  double c[PTS_MAX + 1][PMOR_TMAX];  // by term slot
  int cnt, nt;
};

static PtsCoefs pts_coefs(const pmor_problem* pb, const Point* pts, int cnt) {
  PtsCoefs pc{};
  pc.cnt = cnt;
  pc.nt = pb->nterms;
  for (int l = 0; l < cnt; ++l)
    for (int t = 0; t < pb->nterms; ++t) pc.c[l][t] = pts[l].c[t];
  return pc;
}

// out[l * ostride + q] = A(l) at CSR position map[q] (q itself when map is NULL), 0 where map[q] < 0
__global__ void k_assemble_pts(int64_t len, const int32_t* __restrict__ map, int64_t nnz,
                               const double* __restrict__ tval, PtsCoefs pc, double* __restrict__ out,
                               int64_t ostride) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < len; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = map ? (int64_t)map[q] : q;
    double tv[PMOR_TMAX];
#pragma unroll
    for (int t = 0; t < PMOR_TMAX; ++t) tv[t] = (e >= 0 && t < pc.nt) ? tval[(int64_t)t * nnz + e] : 0.0;
    for (int l = 0; l < pc.cnt; ++l) {
      double acc = 0.0;
      #pragma unroll
      for (int t = 0; t < PMOR_TMAX; ++t)
          if (t < pc.nt) acc += pc.c[l][t] * tv[t];
      out[(int64_t)l * ostride + q] = e >= 0 ? acc : 0.0;
    }
  }
}

int launch_assemble_pts(pmor_problem* pb, const Point* pts, int cnt, const SellView* sv, double* out, int64_t ostride,
                        hipStream_t st) {
  const int64_t len = sv ? sv->cap : pb->nnz;
  if (len == 0 || cnt <= 0) return PMOR_OK;
  if (cnt > PTS_MAX) return fail(PMOR_EINVAL, "too many points for one assembly launch");
  const PtsCoefs pc = pts_coefs(pb, pts, cnt);
  const unsigned g = (unsigned)std::min<int64_t>((len + 255) / 256, 8192);
  hipLaunchKernelGGL(k_assemble_pts, dim3(g), dim3(256), 0, st, len, sv ? (const int32_t*)sv->map : nullptr,
                     pb->nnz, pb->tval, pc, out, ostride);
  PMOR_HIP(hipGetLastError());
  return PMOR_OK;
}

// U-diag factors of the points of pc: q_l(i), rho_l(i) = ||A(1) e_i - q_l(i) A(l) e_i||
// and the first column with ||A(l) e_i|| = 0 (atomicMin into bad[l])
__global__ void k_update_diag_pts(int n, const int32_t* colptr, const int32_t* cscslot, int64_t nnz,
                                  const double* __restrict__ tval, PtsCoefs pc, const double* __restrict__ a1,
                                  double* q, double* rho, int* bad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double num[PTS_MAX], den[PTS_MAX];
#pragma unroll
  for (int l = 0; l < PTS_MAX; ++l) num[l] = den[l] = 0.0;
  for (int e = colptr[i]; e < colptr[i + 1]; ++e) {
    const int s = cscslot[e];
    double tv[PMOR_TMAX];
#pragma unroll
    for (int t = 0; t < PMOR_TMAX; ++t) tv[t] = t < pc.nt ? tval[(int64_t)t * nnz + s] : 0.0;
    const double y = a1[s];
#pragma unroll
    for (int l = 0; l < PTS_MAX; ++l) {
      if (l < pc.cnt) {
        double x = 0.0;
        #pragma unroll
        for (int t = 0; t < PMOR_TMAX; ++t)
          if (t < pc.nt) x += pc.c[l][t] * tv[t];
        num[l] += x * y;
        den[l] += x * x;
      }
    }
  }
  double qv[PTS_MAX], r2[PTS_MAX];
#pragma unroll
  for (int l = 0; l < PTS_MAX; ++l) {
    qv[l] = l < pc.cnt ? num[l] / den[l] : 0.0;
    r2[l] = 0.0;
  }
  // residuals entry by entry once the factors are known (the column's entries
  // were just read, so the second pass hits the caches)
  for (int e = colptr[i]; e < colptr[i + 1]; ++e) {
    const int s = cscslot[e];
    double tv[PMOR_TMAX];
#pragma unroll
    for (int t = 0; t < PMOR_TMAX; ++t) tv[t] = t < pc.nt ? tval[(int64_t)t * nnz + s] : 0.0;
    const double y = a1[s];
#pragma unroll
    for (int l = 0; l < PTS_MAX; ++l) {
      if (l < pc.cnt) {
        double x = 0.0;
        #pragma unroll
        for (int t = 0; t < PMOR_TMAX; ++t)
          if (t < pc.nt) x += pc.c[l][t] * tv[t];
        const double d = y - qv[l] * x;
        r2[l] += d * d;
      }
    }
  }
#pragma unroll
  for (int l = 0; l < PTS_MAX; ++l) {
    if (l < pc.cnt) {
      if (!(den[l] > 0.0)) atomicMin(bad + l, i);
      q[(int64_t)l * n + i] = qv[l];
      rho[(int64_t)l * n + i] = sqrt(r2[l]);
    }
  }
}

int launch_update_diag_pts_anchor(pmor_problem* pb, const double* anchor, const Point* pts, int cnt, double* q,
                                  double* rho, int* bad, hipStream_t st) {
  const int n = pb->n;
  if (n == 0 || cnt <= 0) return PMOR_OK;
  if (cnt > PTS_MAX) return fail(PMOR_EINVAL, "too many points for one update launch");
  const PtsCoefs pc = pts_coefs(pb, pts, cnt);
  hipLaunchKernelGGL(k_update_diag_pts, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, pb->colptr,
                     pb->cscslot, pb->nnz, pb->tval, pc, anchor, q, rho, bad);
  PMOR_HIP(hipGetLastError());
  return PMOR_OK;
}

int launch_update_diag_pts(pmor_spai* h, const Point* pts, int cnt, double* q, double* rho, int* bad,
                           hipStream_t st) {
  return launch_update_diag_pts_anchor(h->pb, h->aval1, pts, cnt, q, rho, bad, st);
}

// Second approach over points l0 .. l0 + cnt - 1 of a sequence (l0 >= 1, cnt
// <= PTS_MAX): for each point the anchor is the previous point, q_l from
// ||A(l-1) e_i - q A(l) e_i|| and the running scale q_l q_{l-1} ... q_1 into q
// (row t), with the step residual into rho.  Both matrices come from the term
// values with the points' coefficients (pc.c[0]: point l0 - 1, pc.c[t + 1]:
// point l0 + t), each entry once, by the sums of k_assemble, so the factors
// are bit for bit those of a chain of single updates.  carry (n): the running
// scale of point l0 - 1 (ones for l0 = 1), replaced by the last point's.
__global__ void k_update_diag_chain(int n, const int32_t* colptr, const int32_t* cscslot, int64_t nnz,
                                    const double* __restrict__ tval, ChainCoefs pc, int l0, double* carry,
                                    double* q, double* rho, int* bad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double num[PTS_MAX], den[PTS_MAX];
#pragma unroll
  for (int l = 0; l < PTS_MAX; ++l) num[l] = den[l] = 0.0;
  for (int e = colptr[i]; e < colptr[i + 1]; ++e) {
    const int s = cscslot[e];
    double tv[PMOR_TMAX];
#pragma unroll
    for (int t = 0; t < PMOR_TMAX; ++t) tv[t] = t < pc.nt ? tval[(int64_t)t * nnz + s] : 0.0;
    double y = 0.0;  // anchor value (point l0 - 1)
    #pragma unroll
    for (int t = 0; t < PMOR_TMAX; ++t)
          if (t < pc.nt) y += pc.c[0][t] * tv[t];
#pragma unroll
    for (int l = 0; l < PTS_MAX; ++l) {
      if (l < pc.cnt) {
        double x = 0.0;
        #pragma unroll
        for (int t = 0; t < PMOR_TMAX; ++t)
          if (t < pc.nt) x += pc.c[l + 1][t] * tv[t];
        num[l] += x * y;
        den[l] += x * x;
        y = x;  // the next point's anchor
      }
    }
  }
  double qv[PTS_MAX], r2[PTS_MAX];
#pragma unroll
  for (int l = 0; l < PTS_MAX; ++l) {
    qv[l] = l < pc.cnt ? num[l] / den[l] : 0.0;
    r2[l] = 0.0;
  }
  // step residuals ||A(l-1) e_i - q_l A(l) e_i|| entry by entry
  for (int e = colptr[i]; e < colptr[i + 1]; ++e) {
    const int s = cscslot[e];
    double tv[PMOR_TMAX];
#pragma unroll
    for (int t = 0; t < PMOR_TMAX; ++t) tv[t] = t < pc.nt ? tval[(int64_t)t * nnz + s] : 0.0;
    double y = 0.0;
    #pragma unroll
    for (int t = 0; t < PMOR_TMAX; ++t)
          if (t < pc.nt) y += pc.c[0][t] * tv[t];
#pragma unroll
    for (int l = 0; l < PTS_MAX; ++l) {
      if (l < pc.cnt) {
        double x = 0.0;
        #pragma unroll
        for (int t = 0; t < PMOR_TMAX; ++t)
          if (t < pc.nt) x += pc.c[l + 1][t] * tv[t];
        const double d = y - qv[l] * x;
        r2[l] += d * d;
        y = x;
      }
    }
  }
  double qc = l0 >= 2 ? carry[i] : 1.0;
#pragma unroll
  for (int l = 0; l < PTS_MAX; ++l) {
    if (l < pc.cnt) {
      if (!(den[l] > 0.0)) atomicMin(bad + l, i);
      qc = qc * qv[l];
      q[(int64_t)l * n + i] = qc;
      rho[(int64_t)l * n + i] = sqrt(r2[l]);
    }
  }
  carry[i] = qc;
}

int launch_update_diag_chain(pmor_spai* h, const Point* pts, int l0, int cnt, double* carry, double* q, double* rho,
                             int* bad, hipStream_t st) {
  pmor_problem* pb = h->pb;
  const int n = pb->n;
  if (n == 0 || cnt <= 0) return PMOR_OK;
  if (cnt > PTS_MAX) return fail(PMOR_EINVAL, "too many points for one update launch");
  if (l0 < 1) return fail(PMOR_EINVAL, "the update chain starts after the anchor point");
  ChainCoefs pc{};
  pc.cnt = cnt;
  pc.nt = pb->nterms;
  for (int t = 0; t <= cnt; ++t)
    for (int u = 0; u < pb->nterms; ++u) pc.c[t][u] = pts[l0 - 1 + t].c[u];
  hipLaunchKernelGGL(k_update_diag_chain, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, pb->colptr,
                     pb->cscslot, pb->nnz, pb->tval, pc, l0, carry, q, rho, bad);
  PMOR_HIP(hipGetLastError());
  return PMOR_OK;
}

// per point l < cnt: out[l * ostride] = sum of squares of x[l * n ...], with the
// partition and the summation tree of sumsq (partials at out + l * ostride + 1)
__global__ void k_sumsq_partials_pts(const double* x, int64_t n, double* out, int64_t ostride) {
  __shared__ double s[4];
  const double* xl = x + (int64_t)blockIdx.y * n;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    acc += xl[i] * xl[i];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[(int64_t)blockIdx.y * ostride + 1 + blockIdx.x] = s[0] + s[1] + s[2] + s[3];
}

__global__ __launch_bounds__(256) void k_sum_in_order_pts(double* out, int64_t ostride, int np) {
  double* o = out + (int64_t)blockIdx.x * ostride;
  __shared__ double s[256];
  s[threadIdx.x] = (int)threadIdx.x < np ? o[1 + threadIdx.x] : 0.0;
  __syncthreads();
  for (int k = 128; k >= 1; k >>= 1) {
    if ((int)threadIdx.x < k) s[threadIdx.x] += s[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) o[0] = s[0];
}

int sumsq_pts(const double* x, int64_t n, int cnt, double* out, int64_t ostride, hipStream_t st) {
  if (cnt <= 0) return PMOR_OK;
  if (ostride < 257) return fail(PMOR_EINVAL, "sum-of-squares stride too small");
  const int np = 256;
  hipLaunchKernelGGL(k_sumsq_partials_pts, dim3(np, cnt), dim3(256), 0, st, x, n, out, ostride);
  hipLaunchKernelGGL(k_sum_in_order_pts, dim3(cnt), dim3(256), 0, st, out, ostride, np);
  PMOR_HIP(hipGetLastError());
  return PMOR_OK;
}

// ---------------------------------------------------------------------------
// Frobenius norms of Table 2: mode 0: ||a - b||^2, mode 1: ||I - A||^2 (a = A values)
// ---------------------------------------------------------------------------
__global__ void k_fro_partials(int n, const int32_t* rowptr, const int32_t* col, const double* a, const double* b,
                               int mode, double* part) {
  __shared__ double s[4];
  double acc = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    bool diag = false;
    for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      double d;
      if (mode == 0) d = a[e] - b[e];
      else if (col[e] == i) { d = 1.0 - a[e]; diag = true; }
      else d = a[e];
      acc += d * d;
    }
    if (mode == 1 && !diag) acc += 1.0;
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = s[0] + s[1] + s[2] + s[3];
}

int fro_norm2(pmor_problem* pb, const double* a, const double* b, int64_t, int mode, double* out_host) {
  hipStream_t st = pb->ctx->stream;
  double* scratch = nullptr;
  PMOR_HIP(dmalloc((void**)&scratch, sizeof(double) * 260, st));
  hipLaunchKernelGGL(k_fro_partials, dim3(256), dim3(256), 0, st, pb->n, pb->rowptr, pb->col, a, b, mode,
                     scratch + 1);
  hipLaunchKernelGGL(k_sum_in_order, dim3(1), dim3(256), 0, st, scratch + 1, 256, scratch);
  PMOR_HIP(hipGetLastError());
  PMOR_HIP(hipMemcpyAsync(out_host, scratch, sizeof(double), hipMemcpyDeviceToHost, st));
  PMOR_HIP(hipStreamSynchronize(st));
  dfree(scratch, st);
  return PMOR_OK;
}

}  // namespace pmor
