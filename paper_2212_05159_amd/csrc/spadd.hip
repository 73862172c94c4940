// Sparse + sparse (Section 3.1.4; Table 1, Sp + Sp rows):
// C = alpha A + beta B on the union of the two patterns, and its VJP
// gA = alpha V on pat(A), gB = beta V on pat(B).
//
// Every kernel works row-parallel with an aligned group of G lanes per
// row (G a power of two dividing 64).  No row is merged serially: the
// position of an entry of A in the union row follows from ranks.  For
// A's entry t with column c, let k = |{B columns < c}| (a binary search
// in B's row) and let d be the number of columns common to both rows
// that are below c.  Then c sits at t + k - d in C's row.  d is the
// number of A entries before t whose column B also stores: a prefix
// count of a per-entry match flag, taken with one ballot per chunk of G
// entries plus a running carry.  B's entries are placed the same way,
// and those whose column A also stores are left to A's side, which adds
// both terms.  The sums round like C_ij = alpha A_ij + beta B_ij done in
// float64 (products and the sum rounded separately), then once to the
// value type, so float64 results are bit-identical to that expression
// and float32 results are its correctly rounded value.
//
// Traffic is row-local and streaming: nothing is gathered through column
// indices, so all three kernels are bound by HBM bandwidth.
#include "internal.hpp"

namespace csrad {
namespace {

constexpr int kAddThreads = 256;

// Lanes of this lane's G-group inside the 64-bit wave mask.
template <int G>
__device__ __forceinline__ unsigned long long group_bits(int lane) {
  if constexpr (G == 64) {
    return ~0ull;
  } else {
    return ((1ull << G) - 1ull) << (lane & ~(G - 1));
  }
}

// Number of entries of the ascending array a[0..len) that are < key.
__device__ __forceinline__ int rank_below(const int32_t* __restrict__ a, int len, int key) {
  int lo = 0, n = len;
  while (n > 0) {
    const int half = n >> 1;
    if (a[lo + half] < key) {
      lo += half + 1;
      n -= half + 1;
    } else {
      n = half;
    }
  }
  return lo;
}

template <typename T>
__device__ __forceinline__ T round_to(double v) {
  return static_cast<T>(v);
}

// Union row lengths: cnt[i] = len_A(i) + len_B(i) - |common columns|.
template <int G>
__global__ __launch_bounds__(kAddThreads) void k_add_count(
    int m, const int32_t* __restrict__ rpA, const int32_t* __restrict__ ciA,
    const int32_t* __restrict__ rpB, const int32_t* __restrict__ ciB, int32_t* __restrict__ cnt) {
  const int row = blockIdx.x * (kAddThreads / G) + threadIdx.x / G;
  if (row >= m) return;  // whole groups leave together
  const int lg = threadIdx.x & (G - 1);
  const unsigned long long gm = group_bits<G>(threadIdx.x & (kWave - 1));
  const int a0 = rpA[row], la = rpA[row + 1] - a0;
  const int b0 = rpB[row], lb = rpB[row + 1] - b0;
  // scan the shorter row against the longer one
  const int32_t* s = la <= lb ? ciA + a0 : ciB + b0;
  const int32_t* l = la <= lb ? ciB + b0 : ciA + a0;
  const int ls = la <= lb ? la : lb, ll = la <= lb ? lb : la;
  int common = 0;
  for (int base = 0; base < ls; base += G) {
    const int t = base + lg;
    bool match = false;
    if (t < ls) {
      const int c = s[t];
      const int k = rank_below(l, ll, c);
      match = k < ll && l[k] == c;
    }
    common += __popcll(__ballot(match) & gm);
  }
  if (lg == 0) cnt[row] = la + lb - common;
}

// Columns (optional) and values of C given C's row pointers.
template <int G, typename T>
__global__ __launch_bounds__(kAddThreads) void k_add_fill(
    int m, const int32_t* __restrict__ rpA, const int32_t* __restrict__ ciA,
    const T* __restrict__ vA, const int32_t* __restrict__ rpB, const int32_t* __restrict__ ciB,
    const T* __restrict__ vB, double alpha, double beta, const int32_t* __restrict__ rpC,
    int32_t* __restrict__ ciC, T* __restrict__ vC) {
  // the products and the sum round separately: no fused multiply-add
  // (the pragma takes the contract flag off the operations written here)
#pragma clang fp contract(off)
  const int row = blockIdx.x * (kAddThreads / G) + threadIdx.x / G;
  if (row >= m) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int lg = threadIdx.x & (G - 1);
  const unsigned long long gm = group_bits<G>(lane);
  const unsigned long long below = gm & ((1ull << lane) - 1ull);
  const int a0 = rpA[row], la = rpA[row + 1] - a0;
  const int b0 = rpB[row], lb = rpB[row + 1] - b0;
  const int c0 = rpC[row], lc = rpC[row + 1] - c0;
  int32_t* cc = ciC ? ciC + c0 : nullptr;
  T* cv = vC + c0;

  int common = 0;  // matched A entries in earlier chunks
  for (int base = 0; base < la; base += G) {
    const int t = base + lg;
    bool match = false;
    int c = 0, k = 0;
    if (t < la) {
      c = ciA[a0 + t];
      k = rank_below(ciB + b0, lb, c);
      match = k < lb && ciB[b0 + k] == c;
    }
    const unsigned long long bal = __ballot(match) & gm;
    const int pos = t + k - common - __popcll(bal & below);
    if (t < la && (unsigned)pos < (unsigned)lc) {  // unless C_rowptr is not this union's
      double v = alpha * static_cast<double>(vA[a0 + t]);
      if (match) {
        const double w = beta * static_cast<double>(vB[b0 + k]);
        v = v + w;
      }
      if (cc) cc[pos] = c;
      cv[pos] = round_to<T>(v);
    }
    common += __popcll(bal);
  }

  common = 0;  // matched B entries in earlier chunks
  for (int base = 0; base < lb; base += G) {
    const int t = base + lg;
    bool match = false;
    int c = 0, k = 0;
    if (t < lb) {
      c = ciB[b0 + t];
      k = rank_below(ciA + a0, la, c);
      match = k < la && ciA[a0 + k] == c;
    }
    const unsigned long long bal = __ballot(match) & gm;
    const int pos = t + k - common - __popcll(bal & below);
    if (t < lb && !match && (unsigned)pos < (unsigned)lc) {
      if (cc) cc[pos] = c;
      cv[pos] = round_to<T>(beta * static_cast<double>(vB[b0 + t]));
    }
    common += __popcll(bal);
  }
}

// VJP: every stored entry of A (B) finds its column in C's row.
template <int G, typename T>
__global__ __launch_bounds__(kAddThreads) void k_add_bwd(
    int m, const int32_t* __restrict__ rpA, const int32_t* __restrict__ ciA,
    const int32_t* __restrict__ rpB, const int32_t* __restrict__ ciB,
    const int32_t* __restrict__ rpC, const int32_t* __restrict__ ciC, const T* __restrict__ gC,
    double alpha, double beta, T* __restrict__ gA, T* __restrict__ gB) {
  const int row = blockIdx.x * (kAddThreads / G) + threadIdx.x / G;
  if (row >= m) return;
  const int lg = threadIdx.x & (G - 1);
  const int c0 = rpC[row], lc = rpC[row + 1] - c0;
  const int32_t* cc = ciC + c0;
  const T* g = gC + c0;
  if (gA) {
    const int a0 = rpA[row], la = rpA[row + 1] - a0;
    for (int t = lg; t < la; t += G) {
      const int k = rank_below(cc, lc, ciA[a0 + t]);  // < lc: pat(A) lies in pat(C)
      gA[a0 + t] = k < lc ? round_to<T>(alpha * static_cast<double>(g[k])) : T(0);
    }
  }
  if (gB) {
    const int b0 = rpB[row], lb = rpB[row + 1] - b0;
    for (int t = lg; t < lb; t += G) {
      const int k = rank_below(cc, lc, ciB[b0 + t]);
      gB[b0 + t] = k < lc ? round_to<T>(beta * static_cast<double>(g[k])) : T(0);
    }
  }
}

// Lanes per row from the mean row length of the longer operand: enough
// that a typical row takes one chunk.
int lanes_for(long long nnz_max, int m) {
  const long long avg = m > 0 ? (nnz_max + m - 1) / m : 0;
  int g = 4;
  while (g < 64 && g < avg) g <<= 1;
  return g;
}

unsigned add_blocks(int m, int g) {
  const int rpb = kAddThreads / g;
  return (unsigned)((m + rpb - 1) / rpb);
}

int check_same_shape(const csrad_csr* A, const csrad_csr* B, bool vals) {
  CSRAD_TRY(check_csr(A, vals));
  CSRAD_TRY(check_csr(B, vals));
  if (A->nrows != B->nrows || A->ncols != B->ncols) return CSRAD_EINVAL;
  if (vals && A->dtype != B->dtype) return CSRAD_EDTYPE;
  return CSRAD_OK;
}

struct SpaddWs {
  int32_t* cnt;
  long long* total;
  void* scan_ws;
  size_t scan_bytes;
};

SpaddWs carve_spadd(Carver& cv, int m) {
  SpaddWs w{};
  w.cnt = cv.take<int32_t>((size_t)m);
  w.total = cv.take<long long>(1);
  w.scan_bytes = scan_workspace(m);
  w.scan_ws = cv.take<char>(w.scan_bytes);
  return w;
}

#define CSRAD_ADD_LANES(G, launch) \
  switch (G) {                     \
    case 4: launch(4); break;      \
    case 8: launch(8); break;      \
    case 16: launch(16); break;    \
    case 32: launch(32); break;    \
    default: launch(64); break;    \
  }

template <typename T>
int spadd_fill_t(const csrad_csr* A, const csrad_csr* B, double alpha, double beta,
                 const int32_t* rpC, int32_t* ciC, T* vC, hipStream_t s) {
  const int m = A->nrows;
  const int g = lanes_for(A->nnz > B->nnz ? A->nnz : B->nnz, m);
  const T* vA = static_cast<const T*>(A->vals);
  const T* vB = static_cast<const T*>(B->vals);
#define CSRAD_FILL(G)                                                                           \
  hipLaunchKernelGGL((k_add_fill<G, T>), dim3(add_blocks(m, G)), dim3(kAddThreads), 0, s, m,  \
                     A->rowptr, A->colind, vA, B->rowptr, B->colind, vB, alpha, beta, rpC, ciC, \
                     vC)
  CSRAD_ADD_LANES(g, CSRAD_FILL)
#undef CSRAD_FILL
  return launch_status();
}

template <typename T>
int spadd_bwd_t(const csrad_csr* A, const csrad_csr* B, const csrad_csr* Cp, const T* gC,
                double alpha, double beta, T* gA, T* gB, hipStream_t s) {
  const int m = A->nrows;
  const int g = lanes_for(A->nnz > B->nnz ? A->nnz : B->nnz, m);
#define CSRAD_BWD(G)                                                                           \
  hipLaunchKernelGGL((k_add_bwd<G, T>), dim3(add_blocks(m, G)), dim3(kAddThreads), 0, s, m,   \
                     A->rowptr, A->colind, B->rowptr, B->colind, Cp->rowptr, Cp->colind, gC,    \
                     alpha, beta, gA, gB)
  CSRAD_ADD_LANES(g, CSRAD_BWD)
#undef CSRAD_BWD
  return launch_status();
}

}  // namespace
}  // namespace csrad

using namespace csrad;

extern "C" int csr_spadd_workspace(const csrad_csr* A, const csrad_csr* B, size_t* bytes) {
  CSRAD_TRY(check_same_shape(A, B, false));
  if (!bytes) return CSRAD_EINVAL;
  Carver cv(nullptr, 0);
  carve_spadd(cv, A->nrows);
  *bytes = cv.off;
  return CSRAD_OK;
}

extern "C" int csr_spadd_symbolic(const csrad_csr* A, const csrad_csr* B, int32_t* C_rowptr,
                                  int64_t* C_nnz_host, void* work, size_t work_bytes,
                                  void* stream) {
  CSRAD_TRY(check_same_shape(A, B, false));
  if (!C_rowptr || !C_nnz_host) return CSRAD_EINVAL;
  hipStream_t s = as_stream(stream);
  const int m = A->nrows;
  Carver cv(work, work_bytes);
  SpaddWs w = carve_spadd(cv, m);
  if (!work || !cv.ok) return CSRAD_EWORKSPACE;
  if (m > 0) {
    const int g = lanes_for(A->nnz > B->nnz ? A->nnz : B->nnz, m);
#define CSRAD_COUNT(G)                                                                       \
  hipLaunchKernelGGL((k_add_count<G>), dim3(add_blocks(m, G)), dim3(kAddThreads), 0, s, m, \
                     A->rowptr, A->colind, B->rowptr, B->colind, w.cnt)
    CSRAD_ADD_LANES(g, CSRAD_COUNT)
#undef CSRAD_COUNT
    CSRAD_TRY(launch_status());
  }
  CSRAD_TRY(scan_exclusive(w.cnt, C_rowptr, m, w.total, w.scan_ws, w.scan_bytes, s));
  long long total = 0;
  if (hipMemcpyAsync(&total, w.total, sizeof(total), hipMemcpyDeviceToHost, s) != hipSuccess)
    return CSRAD_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return CSRAD_EHIP;
  *C_nnz_host = total;
  if (total > INT32_MAX) return CSRAD_EOVERFLOW;
  return CSRAD_OK;
}

extern "C" int csr_spadd_fwd(const csrad_csr* A, const csrad_csr* B, double alpha, double beta,
                             const int32_t* C_rowptr, int32_t* C_colind, void* C_vals,
                             void* stream) {
  CSRAD_TRY(check_same_shape(A, B, true));
  if (!C_rowptr) return CSRAD_EINVAL;
  if (A->nnz == 0 && B->nnz == 0) return CSRAD_OK;  // C is empty
  if (!C_vals) return CSRAD_EINVAL;
  hipStream_t s = as_stream(stream);
  if (A->dtype == CSRAD_F32)
    return spadd_fill_t<float>(A, B, alpha, beta, C_rowptr, C_colind, static_cast<float*>(C_vals),
                               s);
  return spadd_fill_t<double>(A, B, alpha, beta, C_rowptr, C_colind,
                              static_cast<double*>(C_vals), s);
}

extern "C" int csr_spadd_bwd(const csrad_csr* A, const csrad_csr* B, const csrad_csr* C,
                             double alpha, double beta, const void* gC, void* gA, void* gB,
                             void* stream) {
  CSRAD_TRY(check_same_shape(A, B, false));
  CSRAD_TRY(check_csr(C, false));
  if (C->nrows != A->nrows || C->ncols != A->ncols) return CSRAD_EINVAL;
  if (C->dtype != A->dtype || C->dtype != B->dtype) return CSRAD_EDTYPE;
  if (!gA && !gB) return CSRAD_OK;
  if (C->nnz > 0 && !gC) return CSRAD_EINVAL;
  hipStream_t s = as_stream(stream);
  if (A->nrows == 0) return CSRAD_OK;
  if (C->dtype == CSRAD_F32)
    return spadd_bwd_t<float>(A, B, C, static_cast<const float*>(gC), alpha, beta,
                              static_cast<float*>(gA), static_cast<float*>(gB), s);
  return spadd_bwd_t<double>(A, B, C, static_cast<const double*>(gC), alpha, beta,
                             static_cast<double*>(gA), static_cast<double*>(gB), s);
}
