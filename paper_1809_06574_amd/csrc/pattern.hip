// Pattern setup on the device (integer work, bit-exact):
//  * validation of the caller's term CSR arrays;
//  * the union pattern of the terms plus the diagonal (the pattern of every
//    A(s,p) = s^2 M(p) + s D(p) + K(p)), per-term slot maps, packed term values;
//  * the CSC view of a pattern with its CSC -> CSR slot map;
//  * the SPAI index sets: J_j (pattern of column j of P) and the shadow I_j
//    (rows of A(:, J_j) holding a nonzero), and the buckets of columns by
//    (|J_j|, |I_j|) that select the least-squares kernel.
#include <algorithm>
#include <cstdlib>

#include "common.hpp"

namespace pmor {

// ---------------------------------------------------------------------------
// exclusive scan of n int64 counts (out may alias in); out[n] = total
// ---------------------------------------------------------------------------
constexpr int SCAN_T = 256, SCAN_I = 8, SCAN_TILE = SCAN_T * SCAN_I;

__global__ __launch_bounds__(SCAN_T) void k_scan_tile(const int64_t* in, int64_t n, int64_t* out,
                                                      int64_t* sums) {
  __shared__ int64_t s[SCAN_T];
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_I;
  int64_t v[SCAN_I];
  int64_t run = 0;
#pragma unroll
  for (int i = 0; i < SCAN_I; ++i) {
    int64_t x = (base + i < n) ? in[base + i] : 0;
    v[i] = run;
    run += x;
  }
  s[threadIdx.x] = run;
  __syncthreads();
  for (int o = 1; o < SCAN_T; o <<= 1) {
    int64_t add = (threadIdx.x >= o) ? s[threadIdx.x - o] : 0;
    __syncthreads();
    s[threadIdx.x] += add;
    __syncthreads();
  }
  int64_t excl = s[threadIdx.x] - run;
#pragma unroll
  for (int i = 0; i < SCAN_I; ++i)
    if (base + i < n) out[base + i] = v[i] + excl;
  if (threadIdx.x == SCAN_T - 1) sums[blockIdx.x] = s[threadIdx.x];
}

__global__ void k_scan_add(int64_t* out, int64_t n, const int64_t* offs) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += offs[i / SCAN_TILE];
}

__global__ void k_set_total(int64_t* out, int64_t n, const int64_t* in_last, const int64_t* excl_last) {
  if (threadIdx.x == 0 && blockIdx.x == 0) out[n] = *excl_last + *in_last;
}

// the whole scan in one workgroup (sizes up to SCAN_ONE_MAX): thread t owns the
// contiguous chunk [t per, (t + 1) per), sums it, the 1024 sums are scanned in
// LDS, and the chunk is rewritten with its exclusive prefix; buf[n] = total.
// One launch instead of the tile/recursion/add/total sequence, which for the
// pattern set-up of many small systems is mostly launch overhead.
constexpr int SCAN_ONE_T = 1024;
constexpr int64_t SCAN_ONE_MAX = 131072;

__global__ __launch_bounds__(SCAN_ONE_T) void k_scan_one(int64_t* buf, int64_t n) {
  __shared__ int64_t s[2 * (SCAN_ONE_T / 64)];  // wavefront totals, then their inclusive scan
  const int t = threadIdx.x;
  const int64_t per = (n + SCAN_ONE_T - 1) / SCAN_ONE_T;
  const int64_t b = (int64_t)t * per, e = b + per < n ? b + per : n;
  int64_t sum = 0;
  for (int64_t i0 = b; i0 < e; i0 += 8) {
    int64_t v8[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v8[u] = (i0 + u < e) ? buf[i0 + u] : 0;
#pragma unroll
    for (int u = 0; u < 8; ++u) sum += v8[u];
  }
  // inclusive scan of the chunk sums: inside each wavefront by shuffles, then
  // over the 16 wavefront totals (two barriers)
  const int lane = t & 63, w = t >> 6;
  int64_t x = sum;
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) s[w] = x;
  __syncthreads();
  if (w == 0) {
    int64_t v = lane < SCAN_ONE_T / 64 ? s[lane] : 0;
    for (int o = 1; o < SCAN_ONE_T / 64; o <<= 1) {
      const int64_t y = __shfl_up(v, o, 64);
      if (lane >= o) v += y;
    }
    if (lane < SCAN_ONE_T / 64) s[SCAN_ONE_T / 64 + lane] = v;
  }
  __syncthreads();
  // the chunk in blocks of 8: the block's loads are issued together, then its
  // prefixes stored
  int64_t run = x - sum + (w > 0 ? s[SCAN_ONE_T / 64 + w - 1] : 0);
  for (int64_t i0 = b; i0 < e; i0 += 8) {
    int64_t v8[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v8[u] = (i0 + u < e) ? buf[i0 + u] : 0;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (i0 + u < e) {
        buf[i0 + u] = run;
        run += v8[u];
      }
  }
  if (t == SCAN_ONE_T - 1) buf[n] = s[2 * (SCAN_ONE_T / 64) - 1];
}

// in and out have n+1 slots; in[0..n) are counts (in may alias out).
int scan_exclusive(int64_t* buf, int64_t n, hipStream_t st) {
  if (n == 0) {
    PMOR_HIP(hipMemsetAsync(buf, 0, sizeof(int64_t), st));
    return PMOR_OK;
  }
  if (n <= SCAN_ONE_MAX) {
    hipLaunchKernelGGL(k_scan_one, dim3(1), dim3(SCAN_ONE_T), 0, st, buf, n);
    PMOR_HIP(hipGetLastError());
    return PMOR_OK;
  }
  int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
  int64_t* sums = nullptr;
  int64_t* last = nullptr;
  PMOR_HIP(dmalloc((void**)&sums, sizeof(int64_t) * (tiles + 1), st));
  PMOR_HIP(dmalloc((void**)&last, sizeof(int64_t), st));
  PMOR_HIP(hipMemcpyAsync(last, buf + n - 1, sizeof(int64_t), hipMemcpyDeviceToDevice, st));
  hipLaunchKernelGGL(k_scan_tile, dim3((unsigned)tiles), dim3(SCAN_T), 0, st, buf, n, buf, sums);
  PMOR_HIP(hipGetLastError());
  if (tiles > 1) {
    PMOR_TRY(scan_exclusive(sums, tiles, st));
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, buf, n, sums);
    PMOR_HIP(hipGetLastError());
  } else {
    PMOR_HIP(hipMemsetAsync(sums, 0, sizeof(int64_t), st));
  }
  hipLaunchKernelGGL(k_set_total, dim3(1), dim3(1), 0, st, buf, n, last, buf + n - 1);
  PMOR_HIP(hipGetLastError());
  dfree(sums, st);  // stream-ordered: reused only after the kernels above
  dfree(last, st);
  return PMOR_OK;
}

__global__ void k_i64_to_i32(const int64_t* in, int32_t* out, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (int32_t)in[i];
}

// ---------------------------------------------------------------------------
// validation of one CSR term: error bits in *err (1 rowptr, 2 range, 4 order)
// ---------------------------------------------------------------------------
__global__ void k_validate_csr(int n, int nnz, const int32_t* rowptr, const int32_t* col, int* err) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  if (i == 0 && rowptr[0] != 0) atomicOr(err, 1);
  if (i == n) {
    if (rowptr[n] != nnz) atomicOr(err, 1);
    return;
  }
  int a = rowptr[i], b = rowptr[i + 1];
  if (b < a || a < 0 || b > nnz) { atomicOr(err, 1); return; }
  int prev = -1;
  for (int e = a; e < b; ++e) {
    int c = col[e];
    if (c < 0 || c >= n) { atomicOr(err, 2); return; }
    if (c <= prev) { atomicOr(err, 4); return; }
    prev = c;
  }
}

// ---------------------------------------------------------------------------
// union pattern
// ---------------------------------------------------------------------------
struct TermPtrs {
  const int32_t* rowptr[PMOR_TMAX];
  const int32_t* col[PMOR_TMAX];
  const double* val[PMOR_TMAX];
  int present[PMOR_TMAX];
  int slot[PMOR_TMAX];
  int nmaps;  // rows of the slot maps (terms given, present or not)
};

// Walks the sorted column lists of row i of every present term and the diagonal,
// visiting each distinct column once in ascending order: counts[i] = the
// number of distinct columns, maxlen = the longest row.
__global__ void k_union_count(int n, TermPtrs t, int64_t* counts, int* maxlen) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  int cnt = 0;
  if (i < n) {
    int cur[PMOR_TMAX], end[PMOR_TMAX], head[PMOR_TMAX];
#pragma unroll
    for (int r = 0; r < PMOR_TMAX; ++r) {
      cur[r] = t.present[r] ? t.rowptr[r][i] : 0;
      end[r] = t.present[r] ? t.rowptr[r][i + 1] : 0;
      head[r] = cur[r] < end[r] ? t.col[r][cur[r]] : 0x7fffffff;
    }
    bool diag_done = false;
    while (true) {
      int cmin = diag_done ? 0x7fffffff : i;
#pragma unroll
      for (int r = 0; r < PMOR_TMAX; ++r) cmin = min(cmin, head[r]);
      if (cmin == 0x7fffffff) break;
      if (cmin == i) diag_done = true;
#pragma unroll
      for (int r = 0; r < PMOR_TMAX; ++r)
        if (head[r] == cmin) {
          ++cur[r];
          head[r] = cur[r] < end[r] ? t.col[r][cur[r]] : 0x7fffffff;
        }
      ++cnt;
    }
    counts[i] = cnt;
  }
  for (int o = 32; o >= 1; o >>= 1) cnt = max(cnt, __shfl_xor(cnt, o, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(maxlen, cnt);
}

// One thread per entry of the union pattern: entry e is the k-th distinct
// column of its row r (the same walk as k_union_count, stopped at the k-th
// column), so the outputs (columns, the slot maps of every role, the term
// values on the union pattern) leave as coalesced stores.  A row holds a few
// entries, so each thread's walk is short.
// row_of[e] = the row of entry e
__global__ void k_row_of(int n, const int32_t* __restrict__ rowptr, int32_t* __restrict__ row_of) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) row_of[e] = i;
}

__global__ void k_union_fill(int n, TermPtrs t, const int32_t* __restrict__ rowptr_out,
                             const int32_t* row_of, int64_t nnz_out, int32_t* col_out, int32_t* maps,
                             double* tval) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz_out;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = row_of[e];
    const int k = (int)(e - rowptr_out[i]);
    int cur[PMOR_TMAX], end[PMOR_TMAX], head[PMOR_TMAX];
#pragma unroll
    for (int r = 0; r < PMOR_TMAX; ++r) {
      cur[r] = t.present[r] ? t.rowptr[r][i] : 0;
      end[r] = t.present[r] ? t.rowptr[r][i + 1] : 0;
      head[r] = cur[r] < end[r] ? t.col[r][cur[r]] : 0x7fffffff;
    }
    bool diag_done = false;
    for (int cnt = 0;; ++cnt) {
      int cmin = diag_done ? 0x7fffffff : i;
#pragma unroll
      for (int r = 0; r < PMOR_TMAX; ++r) cmin = min(cmin, head[r]);
      if (cmin == 0x7fffffff) break;  // not reached for k < the row's length
      if (cmin == i) diag_done = true;
      if (cnt == k) {
        col_out[e] = cmin;
#pragma unroll
        for (int r = 0; r < PMOR_TMAX; ++r) {
          const bool hit = head[r] == cmin;
          if (r < t.nmaps) maps[(int64_t)r * nnz_out + e] = hit ? cur[r] : -1;
          if (t.present[r]) tval[(int64_t)t.slot[r] * nnz_out + e] = hit ? t.val[r][cur[r]] : 0.0;
        }
        break;
      }
#pragma unroll
      for (int r = 0; r < PMOR_TMAX; ++r)
        if (head[r] == cmin) {
          ++cur[r];
          head[r] = cur[r] < end[r] ? t.col[r][cur[r]] : 0x7fffffff;
        }
    }
  }
}

// ---------------------------------------------------------------------------
// CSC view of a CSR pattern (transpose), rows ascending inside every column
// ---------------------------------------------------------------------------
__global__ void k_col_count(int n, const int32_t* rowptr, const int32_t* col, int64_t* ccount) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) atomicAdd((unsigned long long*)&ccount[col[e]], 1ull);
}

__global__ void k_col_fill(int n, const int32_t* rowptr, const int32_t* col, const int32_t* colptr,
                           int32_t* cursor, int32_t* rowidx, int32_t* slot) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
    int c = col[e];
    int q = colptr[c] + atomicAdd(&cursor[c], 1);
    rowidx[q] = i;
    slot[q] = e;
  }
}

// insertion sort of every column by row (keys unique), carrying the slot map
__global__ void k_col_sort(int n, const int32_t* colptr, int32_t* rowidx, int32_t* slot, int* maxlen) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  int a = colptr[c], b = colptr[c + 1];
  atomicMax(maxlen, b - a);
  for (int q = a + 1; q < b; ++q) {
    int r = rowidx[q], s = slot[q];
    int p = q - 1;
    while (p >= a && rowidx[p] > r) {
      rowidx[p + 1] = rowidx[p];
      slot[p + 1] = slot[p];
      --p;
    }
    rowidx[p + 1] = r;
    slot[p + 1] = s;
  }
}

int check_csr(int n, int64_t nnz, const int32_t* rowptr, const int32_t* col, hipStream_t st) {
  if (n < 1 || nnz < 0 || nnz >= ((int64_t)1 << 31)) return fail(PMOR_EINVAL, "bad pattern size");
  int* derr = nullptr;
  PMOR_HIP(dmalloc((void**)&derr, sizeof(int), st));
  PMOR_HIP(hipMemsetAsync(derr, 0, sizeof(int), st));
  hipLaunchKernelGGL(k_validate_csr, dim3((unsigned)((n + 1 + 255) / 256)), dim3(256), 0, st, n, (int)nnz, rowptr, col,
                     derr);
  PMOR_HIP(hipGetLastError());
  int herr = 0;
  PMOR_HIP(hipMemcpyAsync(&herr, derr, sizeof(int), hipMemcpyDeviceToHost, st));
  PMOR_HIP(hipStreamSynchronize(st));
  dfree(derr, st);
  if (herr) return fail(PMOR_EINVAL, "malformed CSR pattern (rowptr, column range or column order)");
  return PMOR_OK;
}

// ---------------------------------------------------------------------------
// equivalent real form of a complex term (order n -> 2n).  Row i of T, with
// its diagonal entry added (value 0) when absent, becomes rows 2i and 2i+1;
// entry (i, j) becomes the full 2x2 block at columns 2j, 2j+1:
//   part 0 (T (x) I_2): [[v, 0], [0, v]];  part 1 (T (x) J_2): [[0, -v], [v, 0]].
// Every block is stored whole (zeros included), so the union of such terms is
// the real form of a complex pattern: rows 2i and 2i+1 hold the same columns,
// and columns come in pairs 2j, 2j+1.
// ---------------------------------------------------------------------------
__global__ void k_re_count(int n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                           int64_t* __restrict__ cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  bool diag = false;
  for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) diag |= col[e] == i;
  cnt[i] = rowptr[i + 1] - rowptr[i] + (diag ? 0 : 1);
}

__global__ void k_re_fill(int n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                          const double* __restrict__ val, const int64_t* __restrict__ off, int part,
                          int32_t* __restrict__ rp2, int32_t* __restrict__ col2, double* __restrict__ val2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t len = off[i + 1] - off[i];
  const int64_t r0 = 4 * off[i], r1 = r0 + 2 * len;  // starts of rows 2i and 2i+1
  rp2[2 * i] = (int32_t)r0;
  rp2[2 * i + 1] = (int32_t)r1;
  if (i == n - 1) rp2[2 * n] = (int32_t)(4 * off[n]);
  int e = rowptr[i];
  const int e1 = rowptr[i + 1];
  bool diag_done = false;
  for (int64_t k = 0; k < len; ++k) {
    int j;
    double v;
    if (e < e1 && (diag_done || col[e] <= i)) {  // the row's next entry (the diagonal itself when present)
      j = col[e];
      v = val[e];
      ++e;
      if (j == i) diag_done = true;
    } else {  // the absent diagonal, in its sorted place
      j = i;
      v = 0.0;
      diag_done = true;
    }
    const int64_t q0 = r0 + 2 * k, q1 = r1 + 2 * k;
    col2[q0] = 2 * j;
    col2[q0 + 1] = 2 * j + 1;
    col2[q1] = 2 * j;
    col2[q1 + 1] = 2 * j + 1;
    if (part == 0) {
      val2[q0] = v;
      val2[q0 + 1] = 0.0;
      val2[q1] = 0.0;
      val2[q1 + 1] = v;
    } else {
      val2[q0] = 0.0;
      val2[q0 + 1] = -v;
      val2[q1] = v;
      val2[q1 + 1] = 0.0;
    }
  }
}

int real_equiv_term(const pmor_csr* T, int part, int32_t** rp2, int32_t** col2, double** val2, int32_t* nnz2,
                    hipStream_t st) {
  *rp2 = nullptr;
  *col2 = nullptr;
  *val2 = nullptr;
  const int n = T->n;
  PMOR_TRY(check_csr(n, T->nnz, T->rowptr, T->col, st));
  if (4 * ((int64_t)T->nnz + n) >= ((int64_t)1 << 31)) return fail(PMOR_EINVAL, "equivalent real term too large");
  int64_t* off = nullptr;
  PMOR_HIP(dmalloc((void**)&off, sizeof(int64_t) * ((size_t)n + 1), st));
  hipLaunchKernelGGL(k_re_count, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, T->rowptr, T->col, off);
  int rc = hipGetLastError() == hipSuccess ? PMOR_OK : fail(PMOR_EHIP, "launch failed");
  if (rc == PMOR_OK) rc = scan_exclusive(off, n, st);
  int64_t tot = 0;
  if (rc == PMOR_OK && hipMemcpyAsync(&tot, off + n, sizeof(int64_t), hipMemcpyDeviceToHost, st) != hipSuccess)
    rc = fail(PMOR_EHIP, "copy failed");
  if (rc == PMOR_OK && hipStreamSynchronize(st) != hipSuccess) rc = fail(PMOR_EHIP, "synchronise failed");
  if (rc == PMOR_OK) {
    const int64_t nz = 4 * tot;
    if (dmalloc((void**)rp2, sizeof(int32_t) * (2 * (size_t)n + 1), st) != hipSuccess ||
        dmalloc((void**)col2, sizeof(int32_t) * (size_t)nz, st) != hipSuccess ||
        dmalloc((void**)val2, sizeof(double) * (size_t)nz, st) != hipSuccess) {
      (void)hipGetLastError();
      rc = fail(PMOR_ENOMEM, "allocation of an equivalent real term failed");
    } else {
      hipLaunchKernelGGL(k_re_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, T->rowptr, T->col,
                         T->val, off, part, *rp2, *col2, *val2);
      if (hipGetLastError() != hipSuccess) rc = fail(PMOR_EHIP, "launch failed");
      *nnz2 = (int32_t)nz;
    }
  }
  dfree(off, st);
  if (rc != PMOR_OK) {
    dfree(*rp2, st);
    dfree(*col2, st);
    dfree(*val2, st);
    *rp2 = nullptr;
    *col2 = nullptr;
    *val2 = nullptr;
  }
  return rc;
}

// a CSR pattern of order 2m is the real form of a complex one: rows 2i and 2i+1
// hold the same columns, and every row's columns come in pairs 2j, 2j+1
__global__ void k_check_pairs(int m, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col, int* err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int a = rowptr[2 * i], b = rowptr[2 * i + 1], c = rowptr[2 * i + 2];
  bool ok = (b - a == c - b) && ((b - a) % 2 == 0);
  for (int k = 0; ok && k < b - a; k += 2)
    ok = (col[a + k] % 2 == 0) && col[a + k + 1] == col[a + k] + 1 && col[b + k] == col[a + k] &&
         col[b + k + 1] == col[a + k + 1];
  if (!ok) atomicOr(err, 1);
}

int check_pairs(int n, const int32_t* rowptr, const int32_t* col, hipStream_t st) {
  if (n % 2) return fail(PMOR_EINVAL, "odd order");
  int* derr = nullptr;
  PMOR_HIP(dmalloc((void**)&derr, sizeof(int), st));
  PMOR_HIP(hipMemsetAsync(derr, 0, sizeof(int), st));
  const int m = n / 2;
  if (m > 0) hipLaunchKernelGGL(k_check_pairs, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, m, rowptr, col, derr);
  PMOR_HIP(hipGetLastError());
  int herr = 0;
  PMOR_HIP(hipMemcpyAsync(&herr, derr, sizeof(int), hipMemcpyDeviceToHost, st));
  PMOR_HIP(hipStreamSynchronize(st));
  dfree(derr, st);
  if (herr) return fail(PMOR_EINVAL, "the pattern of P is not the real form of a complex pattern");
  return PMOR_OK;
}

// pattern (n x n, nnz entries in CSR) -> CSC arrays allocated here
int transpose_pattern(int n, int64_t nnz, const int32_t* rowptr, const int32_t* col, int32_t** colptr,
                      int32_t** rowidx, int32_t** slot, int* maxcol, hipStream_t st) {
  // counts (int64), cursors (int32) and the maximum in one zeroed scratch block
  int64_t* cc = nullptr;
  const size_t scratch_bytes = sizeof(int64_t) * (n + 1) + sizeof(int32_t) * (n + 2);
  PMOR_HIP(dmalloc((void**)&cc, scratch_bytes, st));
  int32_t* cursor = reinterpret_cast<int32_t*>(cc + (n + 1));
  int* dmax = cursor + (n + 1);
  PMOR_HIP(dmalloc((void**)colptr, sizeof(int32_t) * (n + 1), st));
  PMOR_HIP(dmalloc((void**)rowidx, sizeof(int32_t) * (nnz > 0 ? nnz : 1), st));
  PMOR_HIP(dmalloc((void**)slot, sizeof(int32_t) * (nnz > 0 ? nnz : 1), st));
  PMOR_HIP(hipMemsetAsync(cc, 0, scratch_bytes, st));
  unsigned g = (unsigned)((n + 255) / 256);
  if (n > 0) {
    hipLaunchKernelGGL(k_col_count, dim3(g), dim3(256), 0, st, n, rowptr, col, cc);
    PMOR_HIP(hipGetLastError());
  }
  PMOR_TRY(scan_exclusive(cc, n, st));
  hipLaunchKernelGGL(k_i64_to_i32, dim3((unsigned)((n + 1 + 255) / 256)), dim3(256), 0, st, cc, *colptr,
                     (int64_t)n + 1);
  PMOR_HIP(hipGetLastError());
  if (n > 0) {
    hipLaunchKernelGGL(k_col_fill, dim3(g), dim3(256), 0, st, n, rowptr, col, *colptr, cursor, *rowidx, *slot);
    PMOR_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_col_sort, dim3(g), dim3(256), 0, st, n, *colptr, *rowidx, *slot, dmax);
    PMOR_HIP(hipGetLastError());
  }
  int hmax = 0;
  PMOR_HIP(hipMemcpyAsync(&hmax, dmax, sizeof(int), hipMemcpyDeviceToHost, st));
  PMOR_HIP(hipStreamSynchronize(st));
  *maxcol = hmax;
  dfree(cc, st);
  return PMOR_OK;
}

int build_union_pattern(pmor_problem* pb, const pmor_csr* const* terms, int count, hipStream_t st) {
  if (!st) st = pb->ctx->stream;
  const int n = pb->n;
  if (count < 1 || count > PMOR_TMAX) return fail(PMOR_EINVAL, "term count out of range");
  int* derr = nullptr;
  PMOR_HIP(dmalloc((void**)&derr, sizeof(int) * 2, st));
  PMOR_HIP(hipMemsetAsync(derr, 0, sizeof(int) * 2, st));
  TermPtrs tp{};
  tp.nmaps = count;
  int nt = 0;
  for (int r = 0; r < 2 * PMOR_TMAX; ++r) pb->coef_slot[r] = -1;
  for (int r = 0; r < PMOR_TMAX; ++r) {
    tp.present[r] = 0;
    tp.slot[r] = -1;
    if (r >= count || !terms[r]) continue;
    const pmor_csr* T = terms[r];
    tp.rowptr[r] = T->rowptr;
    tp.col[r] = T->col;
    tp.val[r] = T->val;
    tp.present[r] = 1;
    tp.slot[r] = nt;
    pb->coef_slot[r] = nt++;
    hipLaunchKernelGGL(k_validate_csr, dim3((unsigned)((n + 1 + 255) / 256)), dim3(256), 0, st, n, T->nnz,
                       T->rowptr, T->col, derr);
    PMOR_HIP(hipGetLastError());
  }
  pb->nterms = nt;
  pb->ncoef = count;
  pb->nmaps = count;
  int herr = 0;
  PMOR_HIP(hipMemcpyAsync(&herr, derr, sizeof(int), hipMemcpyDeviceToHost, st));
  PMOR_HIP(hipStreamSynchronize(st));
  if (herr) {
    dfree(derr, st);
    return fail(PMOR_EINVAL, std::string("malformed term CSR (") +
                                 ((herr & 1) ? "rowptr " : "") + ((herr & 2) ? "column-range " : "") +
                                 ((herr & 4) ? "column-order" : "") + ")");
  }
  int64_t* cnt = nullptr;
  PMOR_HIP(dmalloc((void**)&cnt, sizeof(int64_t) * (n + 1), st));
  unsigned g = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_union_count, dim3(g), dim3(256), 0, st, n, tp, cnt, derr + 1);
  PMOR_HIP(hipGetLastError());
  PMOR_TRY(scan_exclusive(cnt, n, st));
  int64_t nnz64 = 0;
  int maxrow = 0;
  PMOR_HIP(hipMemcpyAsync(&nnz64, cnt + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  PMOR_HIP(hipMemcpyAsync(&maxrow, derr + 1, sizeof(int), hipMemcpyDeviceToHost, st));
  PMOR_HIP(hipStreamSynchronize(st));
  if (nnz64 >= ((int64_t)1 << 31)) {
    dfree(cnt, st); dfree(derr, st);
    return fail(PMOR_EINVAL, "union pattern has 2^31 or more entries");
  }
  pb->nnz = (int32_t)nnz64;
  pb->max_row_len = maxrow;
  const int64_t nnz = nnz64;
  PMOR_HIP(dmalloc((void**)&pb->rowptr, sizeof(int32_t) * (n + 1), st));
  PMOR_HIP(dmalloc((void**)&pb->col, sizeof(int32_t) * (nnz > 0 ? nnz : 1), st));
  PMOR_HIP(dmalloc((void**)&pb->maps, sizeof(int32_t) * count * (nnz > 0 ? nnz : 1), st));
  PMOR_HIP(dmalloc((void**)&pb->tval, sizeof(double) * (nt > 0 ? nt : 1) * (nnz > 0 ? nnz : 1), st));
  PMOR_HIP(dmalloc((void**)&pb->aval, sizeof(double) * (nnz > 0 ? nnz : 1), st));
  hipLaunchKernelGGL(k_i64_to_i32, dim3((unsigned)((n + 1 + 255) / 256)), dim3(256), 0, st, cnt, pb->rowptr,
                     (int64_t)n + 1);
  PMOR_HIP(hipGetLastError());
  if (nnz > 0) {
    // the row of every entry goes into pb->col first (each fill thread reads its
    // own entry's row there before it writes the column)
    hipLaunchKernelGGL(k_row_of, dim3(g), dim3(256), 0, st, n, pb->rowptr, pb->col);
    hipLaunchKernelGGL(k_union_fill, dim3((unsigned)std::min<int64_t>((nnz + 255) / 256, 65536)), dim3(256), 0, st,
                       n, tp, pb->rowptr, pb->col, nnz, pb->col, pb->maps, pb->tval);
  }
  PMOR_HIP(hipGetLastError());
  // (no wait here: the transpose below ends with a synchronisation of the same
  // stream, after which the fill has read the caller's term arrays)
  dfree(cnt, st);
  dfree(derr, st);
  int maxcol = 0;
  const int trc = transpose_pattern(n, nnz, pb->rowptr, pb->col, &pb->colptr, &pb->rowidx, &pb->cscslot, &maxcol, st);
  if (trc != PMOR_OK) {
    (void)hipStreamSynchronize(st);  // the fill is done with the caller's terms before the error returns
    return trc;
  }
  pb->max_col_len = maxcol;
  PMOR_TRY(build_sell(n, pb->rowptr, pb->col, nnz, sell_max_fill(), &pb->sell, st));
  if (pb->sell.cap > 0) PMOR_HIP(dmalloc((void**)&pb->aval_s, sizeof(double) * pb->sell.cap, st));
  return PMOR_OK;
}

// ---------------------------------------------------------------------------
// SPAI index sets
// ---------------------------------------------------------------------------
// explicit pattern check: sorted, in range, contains the diagonal (err bits 1, 2, 8)
__global__ void k_validate_pattern(int n, int nnz, const int32_t* colptr, const int32_t* row, int* err) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j > n) return;
  if (j == 0 && colptr[0] != 0) atomicOr(err, 1);
  if (j == n) { if (colptr[n] != nnz) atomicOr(err, 1); return; }
  int a = colptr[j], b = colptr[j + 1];
  if (b < a || a < 0 || b > nnz) { atomicOr(err, 1); return; }
  int prev = -1;
  bool diag = false;
  for (int q = a; q < b; ++q) {
    int r = row[q];
    if (r < 0 || r >= n || r <= prev) { atomicOr(err, 2); return; }
    diag |= (r == j);
    prev = r;
  }
  if (!diag) atomicOr(err, 8);
}

// I_j = sorted union of the rows of A(:, c), c in J_j, by the size of J_j:
//  - |J_j| <= SH_SMALL: one lane merges the |J_j| sorted CSC columns with its
//    cursors and column heads in registers (stencil-like patterns);
//  - larger J_j whose candidate list (sum of |A(:, c)|) fits SH_CAP: one
//    wavefront copies the candidates into LDS, sorts them (bitonic) and keeps
//    the distinct rows;
//  - longer candidate lists: a k-way merge by one lane with the cursors in
//    memory (rare).
// Columns with |J_j| > SH_JMAX are not supported; they report count 0 and
// their |J_j| through maxJ, which the caller turns into an error.
constexpr int SH_SMALL = 8;
constexpr int SH_CAP = 2048;
constexpr int SH_JMAX = 64;

__device__ __forceinline__ int wave_max(int x) {
  for (int o = 32; o >= 1; o >>= 1) x = max(x, __shfl_xor(x, o, 64));
  return x;
}

template <bool FILL>
__global__ __launch_bounds__(256) void k_shadow_small(int n, const int32_t* Jcolptr, const int32_t* Jrow,
                                                      const int32_t* Acolptr, const int32_t* Arowidx,
                                                      int64_t* counts, const int64_t* Icolptr, int32_t* Irow,
                                                      int* maxJ, int* maxI) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  int nj = 0, cnt = 0;
  if (j < n) {
    const int ja = Jcolptr[j];
    nj = Jcolptr[j + 1] - ja;
    if (nj <= SH_SMALL) {
      int cur[SH_SMALL], end[SH_SMALL], head[SH_SMALL];
#pragma unroll
      for (int t = 0; t < SH_SMALL; ++t) {
        cur[t] = 0;
        end[t] = 0;
        if (t < nj) {
          const int c = Jrow[ja + t];
          cur[t] = Acolptr[c];
          end[t] = Acolptr[c + 1];
        }
      }
#pragma unroll
      for (int t = 0; t < SH_SMALL; ++t) head[t] = cur[t] < end[t] ? Arowidx[cur[t]] : 0x7fffffff;
      int64_t pos = FILL ? Icolptr[j] : 0;
      while (true) {
        int rmin = 0x7fffffff;
#pragma unroll
        for (int t = 0; t < SH_SMALL; ++t) rmin = min(rmin, head[t]);
        if (rmin == 0x7fffffff) break;
#pragma unroll
        for (int t = 0; t < SH_SMALL; ++t)
          if (head[t] == rmin) {
            ++cur[t];
            head[t] = cur[t] < end[t] ? Arowidx[cur[t]] : 0x7fffffff;
          }
        if (FILL) Irow[pos + cnt] = rmin;
        ++cnt;
      }
      if (!FILL) counts[j] = cnt;
    } else {
      nj = 0;  // another kernel's column
    }
  }
  if (!FILL) {
    const int mj = wave_max(nj), mi = wave_max(cnt);
    if ((threadIdx.x & 63) == 0) {
      atomicMax(maxJ, mj);
      atomicMax(maxI, mi);
    }
  }
}

// columns SH_SMALL < |J_j| <= SH_JMAX with at most SH_CAP candidates: one
// wavefront per column (grid-stride over the columns, the others skipped) copies
// the candidate rows into LDS, sorts them (bitonic) and keeps the distinct rows.
// With a staging array (tmp, non-null in both passes) the counting pass also
// leaves the distinct rows of column j at tmp + Jcolptr[j] mcl (there are at
// most |J_j| mcl candidates, mcl the longest column of A) and the filling pass
// copies them to their place instead of sorting again.
template <bool FILL>
__global__ __launch_bounds__(64) void k_shadow_sort(int n, const int32_t* Jcolptr, const int32_t* Jrow,
                                                    const int32_t* Acolptr, const int32_t* Arowidx, int64_t* counts,
                                                    const int64_t* Icolptr, int32_t* Irow, int* maxJ, int* maxI,
                                                    int32_t* tmp, int mcl) {
  __shared__ int buf[SH_CAP];
  const int lane = threadIdx.x;
  int mj = 0, mi = 0;
  for (int j = blockIdx.x; j < n; j += gridDim.x) {
    const int ja = Jcolptr[j], nj = Jcolptr[j + 1] - ja;
    if (nj > SH_JMAX) {  // unsupported; reported through maxJ
      if (!FILL && lane == 0) counts[j] = 0;
      mj = max(mj, nj);
      continue;
    }
    if (nj <= SH_SMALL) continue;  // k_shadow_small
    // lane t owns column t of J_j
    int len = 0, c0 = 0;
    if (lane < nj) {
      const int c = Jrow[ja + lane];
      c0 = Acolptr[c];
      len = Acolptr[c + 1] - c0;
    }
    int incl = len;  // inclusive scan over the lanes
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(incl, o, 64);
      if (lane >= o) incl += y;
    }
    const int total = __shfl(incl, 63, 64);
    if (total > SH_CAP) continue;  // k_shadow_merge
    if (FILL && tmp) {  // the counting pass left the rows in tmp
      const int64_t src = (int64_t)ja * mcl, dst = Icolptr[j], cnt = Icolptr[j + 1] - dst;
      for (int64_t q = lane; q < cnt; q += 64) Irow[dst + q] = tmp[src + q];
      continue;
    }
    const int off = incl - len;
    int P = 1;
    while (P < total) P <<= 1;
    __syncthreads();  // the previous column's reads of buf are done
    for (int q = 0; q < len; ++q) buf[off + q] = Arowidx[c0 + q];
    for (int i = total + lane; i < P; i += 64) buf[i] = 0x7fffffff;
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1)
      for (int jj = k >> 1; jj > 0; jj >>= 1) {
        for (int i = lane; i < P; i += 64) {
          const int ixj = i ^ jj;
          if (ixj > i) {
            const int x = buf[i], y = buf[ixj];
            if ((x > y) == ((i & k) == 0)) {
              buf[i] = y;
              buf[ixj] = x;
            }
          }
        }
        __syncthreads();
      }
    // distinct rows, in order
    int64_t pos = FILL ? Icolptr[j] : 0;
    int cnt = 0;
    for (int i0 = 0; i0 < total; i0 += 64) {
      const int i = i0 + lane;
      const bool keep = i < total && (i == 0 || buf[i] != buf[i - 1]);
      const unsigned long long m = __ballot(keep);
      if (FILL && keep) Irow[pos + cnt + __popcll(m & ((1ull << lane) - 1ull))] = buf[i];
      if (!FILL && tmp && keep) tmp[(int64_t)ja * mcl + cnt + __popcll(m & ((1ull << lane) - 1ull))] = buf[i];
      cnt += __popcll(m);
    }
    if (!FILL && lane == 0) counts[j] = cnt;
    mj = max(mj, nj);
    mi = max(mi, cnt);
  }
  // one atomic per workgroup, and none when it cannot raise the maximum
  if (!FILL && lane == 0) {
    if (mj > *(volatile int*)maxJ) atomicMax(maxJ, mj);
    if (mi > *(volatile int*)maxI) atomicMax(maxI, mi);
  }
}

// the columns with more than SH_CAP candidates: k-way merge of the CSC columns, one lane per column
template <bool FILL>
__global__ void k_shadow_merge(int n, const int32_t* Jcolptr, const int32_t* Jrow, const int32_t* Acolptr,
                               const int32_t* Arowidx, int64_t* counts, const int64_t* Icolptr, int32_t* Irow,
                               int* maxJ, int* maxI) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int ja = Jcolptr[j], nj = Jcolptr[j + 1] - ja;
  if (nj <= SH_SMALL || nj > SH_JMAX) return;
  int total = 0;
  for (int t = 0; t < nj; ++t) {
    const int c = Jrow[ja + t];
    total += Acolptr[c + 1] - Acolptr[c];
  }
  if (total <= SH_CAP) return;
  int cur[SH_JMAX], end[SH_JMAX];
  for (int t = 0; t < nj; ++t) {
    int c = Jrow[ja + t];
    cur[t] = Acolptr[c];
    end[t] = Acolptr[c + 1];
  }
  int64_t pos = FILL ? Icolptr[j] : 0;
  int cnt = 0;
  while (true) {
    int rmin = 0x7fffffff;
    for (int t = 0; t < nj; ++t)
      if (cur[t] < end[t]) rmin = min(rmin, Arowidx[cur[t]]);
    if (rmin == 0x7fffffff) break;
    for (int t = 0; t < nj; ++t)
      if (cur[t] < end[t] && Arowidx[cur[t]] == rmin) ++cur[t];
    if (FILL) Irow[pos++] = rmin;
    ++cnt;
  }
  if (!FILL) {
    counts[j] = cnt;
    atomicMax(maxJ, nj);
    atomicMax(maxI, cnt);
  }
}

// jmax: an upper bound of |J_j| known on the host, or -1; tmp, mcl: the
// staging array of k_shadow_sort (or null)
template <bool FILL>
static int launch_shadow(int n, const int32_t* Jcolptr, const int32_t* Jrow, const int32_t* Acolptr,
                         const int32_t* Arowidx, int64_t* counts, const int64_t* Icolptr, int32_t* Irow, int* maxJ,
                         int* maxI, int jmax, hipStream_t st, int32_t* tmp = nullptr, int mcl = 0) {
  if (n <= 0) return PMOR_OK;
  const unsigned g1 = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_shadow_small<FILL>, dim3(g1), dim3(256), 0, st, n, Jcolptr, Jrow, Acolptr, Arowidx, counts,
                     Icolptr, Irow, maxJ, maxI);
  if (jmax >= 0 && jmax <= SH_SMALL) {
    PMOR_HIP(hipGetLastError());
    return PMOR_OK;
  }
  const unsigned gs = (unsigned)std::min(n, 8192);
  hipLaunchKernelGGL(k_shadow_sort<FILL>, dim3(gs), dim3(64), 0, st, n, Jcolptr, Jrow, Acolptr, Arowidx, counts,
                     Icolptr, Irow, maxJ, maxI, tmp, mcl);
  hipLaunchKernelGGL(k_shadow_merge<FILL>, dim3(g1), dim3(256), 0, st, n, Jcolptr, Jrow, Acolptr, Arowidx, counts,
                     Icolptr, Irow, maxJ, maxI);
  PMOR_HIP(hipGetLastError());
  return PMOR_OK;
}

// inv[map[q]] = q
__global__ void k_invert_map(const int32_t* map, int64_t len, int32_t* inv) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < len) inv[map[q]] = (int32_t)q;
}

// bucket of a column: the least-squares kernel that takes it (16, 32 or 64
// lanes per column with R rows each, |I| <= G R, in registers; FP64 takes the
// LDS kernel for buckets 5 to 7; the LDS kernel above, each launch sized to the
// largest column of its bucket)
__host__ __device__ inline int bucket_of(int nj, int ni) {
  if (nj <= 8 && ni <= 16) return 0;
  if (nj <= 8 && ni <= 32) return 1;
  if (nj <= 8 && ni <= 64) return 2;
  if (nj <= 16 && ni <= 64) return 3;
  if (nj <= 16 && ni <= 128) return 4;
  if (nj <= 32 && ni <= 64) return 5;
  if (nj <= 32 && ni <= 128) return 6;
  if (nj <= 64 && ni <= 128) return 7;
  if (nj <= 64 && ni <= 512) return 8;
  return BUCKET_SLOTS - 1;  // unsupported
}

// columns per (|J_j|, |I_j|) bucket from the shadow sizes before their scan
// (counts[j] = |I_j|): a histogram in LDS, one global atomic per bucket and
// workgroup into bcount[0..S) (S = BUCKET_SLOTS); the largest |J_j| and |I_j|
// per bucket into bcount[2S + b], bcount[3S + b]
__global__ void k_bucket_count(int n, const int32_t* Jcolptr, const int64_t* counts, int* bcount) {
  constexpr int S = BUCKET_SLOTS;
  __shared__ int h[S], mj[S], mi[S];
  if (threadIdx.x < S) h[threadIdx.x] = mj[threadIdx.x] = mi[threadIdx.x] = 0;
  __syncthreads();
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) {
    const int nj = Jcolptr[j + 1] - Jcolptr[j], ni = (int)counts[j];
    const int b = bucket_of(nj, ni);
    atomicAdd(&h[b], 1);
    atomicMax(&mj[b], nj);
    atomicMax(&mi[b], ni);
  }
  __syncthreads();
  if (threadIdx.x < S && h[threadIdx.x]) {
    atomicAdd(&bcount[threadIdx.x], h[threadIdx.x]);
    atomicMax(&bcount[2 * S + threadIdx.x], mj[threadIdx.x]);
    atomicMax(&bcount[3 * S + threadIdx.x], mi[threadIdx.x]);
  }
}

// Fill the bucket lists: each workgroup counts its columns per bucket in LDS,
// reserves a range per bucket with one atomic, and writes its columns there in
// order.  The order of the workgroups' ranges inside a bucket may vary between
// runs; every column is still solved on its own, so results do not depend on it.
__global__ __launch_bounds__(256) void k_bucket_fill(int n, const int32_t* Jcolptr, const int64_t* Icolptr,
                                                     const int* boff, int* cursor, int32_t* cols) {
  constexpr int S = BUCKET_SLOTS;
  __shared__ int cnt[S], base[S], pos[S][256];
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = (j < n) ? bucket_of(Jcolptr[j + 1] - Jcolptr[j], (int)(Icolptr[j + 1] - Icolptr[j])) : -1;
  for (int q = 0; q < S; ++q) pos[q][threadIdx.x] = (b == q);
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {  // inclusive scan per bucket
    int v[S];
    for (int q = 0; q < S; ++q) v[q] = (threadIdx.x >= o) ? pos[q][threadIdx.x - o] : 0;
    __syncthreads();
    for (int q = 0; q < S; ++q) pos[q][threadIdx.x] += v[q];
    __syncthreads();
  }
  if (threadIdx.x < S) {
    cnt[threadIdx.x] = pos[threadIdx.x][255];
    base[threadIdx.x] = cnt[threadIdx.x] ? boff[threadIdx.x] + atomicAdd(&cursor[threadIdx.x], cnt[threadIdx.x]) : 0;
  }
  __syncthreads();
  if (b >= 0) cols[base[b] + pos[b][threadIdx.x] - 1] = j;
}

int build_spai_sets(pmor_spai* h, hipStream_t st) {
  pmor_problem* pb = h->pb;
  if (!st) st = pb->ctx->stream;
  const int n = pb->n;
  int* dflag = nullptr;
  PMOR_HIP(dmalloc((void**)&dflag, sizeof(int) * 4, st));
  PMOR_HIP(hipMemsetAsync(dflag, 0, sizeof(int) * 4, st));
  unsigned g = (unsigned)((n + 255) / 256);
  if (h->opts.pattern == PMOR_PAT_A) {
    // J_j = pattern of column j of A; the union pattern holds the full diagonal,
    // so this is the CSC view of A, and P's CSR pattern is A's own.
    h->Jcolptr = pb->colptr; h->Jrow = pb->rowidx; h->own_J = false;
    h->Prowptr = pb->rowptr; h->Pcol = pb->col; h->Pslot = pb->cscslot; h->own_P = false;
    h->psell = pb->sell; h->own_psell = false;
    h->nnzP = pb->nnz;
  } else {
    if (!h->opts.pat_colptr || !h->opts.pat_row || h->opts.nnz_explicit < n) {
      dfree(dflag, st);
      return fail(PMOR_EINVAL, "explicit SPAI pattern: null arrays or fewer than n entries");
    }
    hipLaunchKernelGGL(k_validate_pattern, dim3((unsigned)((n + 1 + 255) / 256)), dim3(256), 0, st, n,
                       h->opts.nnz_explicit, h->opts.pat_colptr, h->opts.pat_row, dflag);
    PMOR_HIP(hipGetLastError());
    int herr = 0;
    PMOR_HIP(hipMemcpyAsync(&herr, dflag, sizeof(int), hipMemcpyDeviceToHost, st));
    PMOR_HIP(hipStreamSynchronize(st));
    if (herr) {
      dfree(dflag, st);
      return fail(PMOR_EINVAL, (herr & 8) ? "explicit SPAI pattern: a column lacks its diagonal"
                                          : "explicit SPAI pattern: malformed CSC");
    }
    const int64_t nnzP = h->opts.nnz_explicit;
    PMOR_HIP(dmalloc((void**)&h->Jcolptr, sizeof(int32_t) * (n + 1), st));
    PMOR_HIP(dmalloc((void**)&h->Jrow, sizeof(int32_t) * nnzP, st));
    PMOR_HIP(hipMemcpyAsync(h->Jcolptr, h->opts.pat_colptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToDevice, st));
    PMOR_HIP(hipMemcpyAsync(h->Jrow, h->opts.pat_row, sizeof(int32_t) * nnzP, hipMemcpyDeviceToDevice, st));
    h->own_J = true;
    // the CSR of P is the transpose of the J sets (read as the CSR of P^T); the
    // transpose's map runs from P's CSR positions to J positions, the least-squares
    // kernels scatter the other way, so it is inverted
    int mx = 0;
    int32_t* back = nullptr;
    PMOR_TRY(transpose_pattern(n, nnzP, h->Jcolptr, h->Jrow, &h->Prowptr, &h->Pcol, &back, &mx, st));
    PMOR_HIP(dmalloc((void**)&h->Pslot, sizeof(int32_t) * nnzP, st));
    hipLaunchKernelGGL(k_invert_map, dim3((unsigned)((nnzP + 255) / 256)), dim3(256), 0, st, back, nnzP, h->Pslot);
    PMOR_HIP(hipGetLastError());
    dfree(back, st);  // stream-ordered: reused only after the inversion
    h->own_P = true;
    h->nnzP = (int32_t)nnzP;
    PMOR_TRY(build_sell(n, h->Prowptr, h->Pcol, nnzP, sell_max_fill(), &h->psell, st));
    h->own_psell = true;
  }
  // shadows: sizes, the bucket histogram and the sizes' scan, read back in one
  // synchronisation; then the rows
  const int jmax = h->opts.pattern == PMOR_PAT_A ? pb->max_col_len : -1;
  int64_t* cnt = nullptr;
  PMOR_HIP(dmalloc((void**)&cnt, sizeof(int64_t) * (n + 1), st));
  // the sorted shadows of the sorting kernel staged between the two passes (one
  // sort instead of two) when |J| mcl bounds fit in 256 MiB
  const int mcl = pb->max_col_len;
  const int64_t tcap = (int64_t)h->nnzP * mcl;
  int32_t* stage = nullptr;
  if (tcap > 0 && tcap <= ((int64_t)64 << 20) && !(jmax >= 0 && jmax <= SH_SMALL))
    PMOR_HIP(dmalloc((void**)&stage, sizeof(int32_t) * tcap, st));
  PMOR_TRY(launch_shadow<false>(n, h->Jcolptr, h->Jrow, pb->colptr, pb->rowidx, cnt, nullptr, nullptr, dflag + 1,
                                dflag + 2, jmax, st, stage, mcl));
  constexpr int S = BUCKET_SLOTS;
  int* bc = nullptr;  // counts [0, S), offsets [S, 2S), largest |J| [2S, 3S), largest |I| [3S, 4S)
  PMOR_HIP(dmalloc((void**)&bc, sizeof(int) * 4 * S, st));
  PMOR_HIP(hipMemsetAsync(bc, 0, sizeof(int) * 4 * S, st));
  hipLaunchKernelGGL(k_bucket_count, dim3(g), dim3(256), 0, st, n, h->Jcolptr, cnt, bc);
  PMOR_HIP(hipGetLastError());
  PMOR_TRY(scan_exclusive(cnt, n, st));
  int hm[2] = {0, 0};
  int hb[S], hx[2 * S];
  PMOR_HIP(hipMemcpyAsync(hm, dflag + 1, sizeof(int) * 2, hipMemcpyDeviceToHost, st));
  PMOR_HIP(hipMemcpyAsync(hb, bc, sizeof(int) * S, hipMemcpyDeviceToHost, st));
  PMOR_HIP(hipMemcpyAsync(hx, bc + 2 * S, sizeof(int) * 2 * S, hipMemcpyDeviceToHost, st));
  PMOR_HIP(hipMemcpyAsync(&h->nI, cnt + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  PMOR_HIP(hipStreamSynchronize(st));
  h->maxJ = hm[0];
  h->maxI = hm[1];
  h->Icolptr = cnt;
  if (h->maxJ > 64 || h->maxI > 512) {
    dfree(bc, st); dfree(dflag, st);
    if (stage) dfree(stage, st);
    return fail(PMOR_EINVAL, "SPAI pattern too large: |J_j| <= 64 and |I_j| <= 512 are supported (got " +
                                 std::to_string(h->maxJ) + ", " + std::to_string(h->maxI) + ")");
  }
  PMOR_HIP(dmalloc((void**)&h->Irow, sizeof(int32_t) * (h->nI > 0 ? h->nI : 1), st));
  PMOR_TRY(launch_shadow<true>(n, h->Jcolptr, h->Jrow, pb->colptr, pb->rowidx, nullptr, h->Icolptr, h->Irow, nullptr,
                               nullptr, jmax, st, stage, mcl));
  if (stage) dfree(stage, st);
  int off = 0, nonempty = 0;
  for (int b = 0; b < S; ++b) {
    h->bucket_count[b] = hb[b];
    h->bucket_off[b] = off;
    h->bucket_maxJ[b] = hx[b];
    h->bucket_maxI[b] = hx[S + b];
    off += hb[b];
    nonempty += hb[b] > 0;
  }
  h->nbuckets = S;
  // when the largest column fits a register kernel, every column takes that one
  // kernel in natural order (no lists, one launch)
  const int bmax = bucket_of(h->maxJ, h->maxI);
  h->identity_order = (bmax <= 4);
  if (h->identity_order) {
    for (int b = 0; b < S; ++b) { h->bucket_count[b] = 0; h->bucket_off[b] = 0; }
    h->bucket_count[bmax] = n;
    h->bucket_maxJ[bmax] = h->maxJ;
    h->bucket_maxI[bmax] = h->maxI;
  }
  for (int b = 0; b < S; ++b) h->identity_order = h->identity_order || (hb[b] == n);
  if (!h->identity_order) {
    int* hb_off = reinterpret_cast<int*>(bc) + S;
    for (int b = 0; b < S; ++b) hb[b] = h->bucket_off[b];
    PMOR_HIP(hipMemcpyAsync(hb_off, hb, sizeof(int) * S, hipMemcpyHostToDevice, st));
    PMOR_HIP(hipMemsetAsync(bc, 0, sizeof(int) * S, st));
    PMOR_HIP(dmalloc((void**)&h->bucket_cols, sizeof(int32_t) * (n > 0 ? n : 1), st));
    hipLaunchKernelGGL(k_bucket_fill, dim3(g), dim3(256), 0, st, n, h->Jcolptr, h->Icolptr, hb_off, bc,
                       h->bucket_cols);
    PMOR_HIP(hipGetLastError());
    PMOR_HIP(hipStreamSynchronize(st));  // hb (host stack) was the source of a copy
  }
  dfree(bc, st);
  dfree(dflag, st);
  (void)nonempty;
  return PMOR_OK;
}

}  // namespace pmor

// ---------------------------------------------------------------------------
// sliced ELL view of a CSR pattern (the engine's SpMM layout)
// ---------------------------------------------------------------------------
namespace pmor {

// width of each 64-row slice (longest row), times 64, one wavefront per slice
__global__ __launch_bounds__(64) void k_sell_width(int n, const int32_t* rowptr, int64_t* w64) {
  const int r = blockIdx.x * 64 + threadIdx.x;
  int len = r < n ? rowptr[r + 1] - rowptr[r] : 0;
  for (int o = 32; o >= 1; o >>= 1) len = max(len, __shfl_xor(len, o, 64));
  if (threadIdx.x == 0) w64[blockIdx.x] = (int64_t)len * 64;
}

__global__ __launch_bounds__(64) void k_sell_fill(int n, const int32_t* rowptr, const int32_t* col,
                                                  const int64_t* off, int32_t* ptr, int32_t* wid, int32_t* scol,
                                                  int32_t* smap) {
  const int s = blockIdx.x, lane = threadIdx.x, r = s * 64 + lane;
  const int64_t base = off[s];
  const int w = (int)((off[s + 1] - base) / 64);
  if (lane == 0) {
    ptr[s] = (int32_t)base;
    wid[s] = w;
    if (s == (int)gridDim.x - 1) ptr[s + 1] = (int32_t)off[s + 1];
  }
  const int e0 = r < n ? rowptr[r] : 0;
  const int len = r < n ? rowptr[r + 1] - e0 : 0;
  for (int k = 0; k < w; ++k) {
    const int64_t q = base + (int64_t)k * 64 + lane;
    if (k < len) {
      scol[q] = col[e0 + k];
      smap[q] = e0 + k;
    } else {
      scol[q] = -1;
      smap[q] = -1;
    }
  }
}

__global__ void k_to_sell(int64_t cap, const int32_t* __restrict__ map, const double* __restrict__ src,
                          double* __restrict__ dst) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < cap; q += (int64_t)gridDim.x * blockDim.x) {
    const int32_t e = map[q];
    dst[q] = e >= 0 ? src[e] : 0.0;
  }
}

double sell_max_fill() {
  const char* e = getenv("PMOR_SELL_MAX_FILL");
  return e ? atof(e) : SELL_MAX_FILL;
}

int build_sell(int n, const int32_t* rowptr, const int32_t* col, int64_t nnz, double max_fill, SellView* v,
               hipStream_t st) {
  *v = SellView{};
  if (n <= 0) return PMOR_OK;
  (void)col;
  const int ns = (n + 63) / 64;
  int64_t* w64 = nullptr;
  PMOR_HIP(dmalloc((void**)&w64, sizeof(int64_t) * (ns + 1), st));
  hipLaunchKernelGGL(k_sell_width, dim3(ns), dim3(64), 0, st, n, rowptr, w64);
  PMOR_HIP(hipGetLastError());
  PMOR_TRY(scan_exclusive(w64, ns, st));
  int64_t cap = 0;
  PMOR_HIP(hipMemcpyAsync(&cap, w64 + ns, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  PMOR_HIP(hipStreamSynchronize(st));
  if (cap <= 0 || (double)cap > max_fill * (double)nnz + 64.0 || cap >= ((int64_t)1 << 31)) {
    dfree(w64, st);
    return PMOR_OK;  // too much padding: the CSR arrays serve
  }
  v->ns = ns;
  v->cap = cap;
  PMOR_HIP(dmalloc((void**)&v->ptr, sizeof(int32_t) * (ns + 1), st));
  PMOR_HIP(dmalloc((void**)&v->wid, sizeof(int32_t) * ns, st));
  PMOR_HIP(dmalloc((void**)&v->col, sizeof(int32_t) * cap, st));
  PMOR_HIP(dmalloc((void**)&v->map, sizeof(int32_t) * cap, st));
  hipLaunchKernelGGL(k_sell_fill, dim3(ns), dim3(64), 0, st, n, rowptr, col, (const int64_t*)w64, v->ptr, v->wid,
                     v->col, v->map);
  PMOR_HIP(hipGetLastError());
  dfree(w64, st);
  return PMOR_OK;
}

void free_sell(SellView* v, hipStream_t st) {
  dfree(v->ptr, st);
  dfree(v->wid, st);
  dfree(v->col, st);
  dfree(v->map, st);
  *v = SellView{};
}

int to_sell(const SellView& v, const double* src, double* dst, hipStream_t st) {
  if (v.cap <= 0) return PMOR_OK;
  const unsigned g = (unsigned)std::min<int64_t>((v.cap + 255) / 256, 8192);
  hipLaunchKernelGGL(k_to_sell, dim3(g), dim3(256), 0, st, v.cap, (const int32_t*)v.map, src, dst);
  PMOR_HIP(hipGetLastError());
  return PMOR_OK;
}

}  // namespace pmor
