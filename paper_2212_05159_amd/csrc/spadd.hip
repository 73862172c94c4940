// Sparse + sparse (Section 3.1.4; Table 1, Sp + Sp rows):
// C = alpha A + beta B on the union of the two patterns, and its VJP
// gA = alpha V on pat(A), gB = beta V on pat(B).
//
// Every kernel works row-parallel with an aligned group of G lanes per
// row (G a power of two dividing 64).  No row is merged serially: the
// position of an entry of A in the union row follows from ranks.  For
// A's entry t with column c, let k = |{B columns < c}| and let d be the
// number of columns common to both rows that are below c.  Then c sits
// at t + k - d in C's row.  d is the number of A entries before t whose
// column B also stores: a prefix count of a per-entry match flag, taken
// with one ballot over the group.  B's entries are placed the same way,
// and those whose column A also stores are left to A's side, which adds
// both terms.
//
// When both rows fit in the group (at most G entries each, the common
// case with G sized from the mean row length), each lane holds one entry
// of each row and k comes from comparing against the other row's entries
// broadcast lane by lane inside the group: every global load of the row
// is issued at once and nothing waits on a chain of dependent loads.
// Longer rows take chunks of G entries and a binary search in the other
// row for k, with the ballot count carried across chunks.
//
// The sums round like C_ij = alpha A_ij + beta B_ij done in float64
// (products and the sum rounded separately), then once to the value
// type, so float64 results are bit-identical to that expression and
// float32 results are its correctly rounded value.
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

// Value of lane J of this lane's aligned G-group (all lanes of the group
// active): a ds_swizzle in bit-mask mode inside 32-lane halves, a
// readlane for whole-wave groups.
template <int G, int J>
__device__ __forceinline__ int group_lane(int v) {
  if constexpr (G == 64) {
    return __builtin_amdgcn_readlane(v, J);
  } else {
    return __builtin_amdgcn_ds_swizzle(v, (0x1F & ~(G - 1)) | (J << 5));
  }
}

// For a row held one entry per lane of the group (mine, INT_MAX past the
// row's end) against another row held the same way (other): rank = how
// many of the other row's columns are below mine, hit = the group lane
// holding mine in the other row, or -1.
template <int G, int J = 0>
__device__ __forceinline__ void group_rank(int mine, int other, int& rank, int& hit) {
  const int x = group_lane<G, J>(other);
  rank += x < mine ? 1 : 0;
  hit = x == mine ? J : hit;
  if constexpr (J + 1 < G) group_rank<G, J + 1>(mine, other, rank, hit);
}

// Both rows of a sum held in registers (each at most G long): columns,
// ranks in the other row and match flags.  Column indices are below
// INT_MAX, so the padding never equals or undercuts a stored column.
template <int G>
struct RegRows {
  int ca, cb;     // this lane's column of A's and of B's row (or INT_MAX)
  int ra, rb;     // rank of ca among B's columns, of cb among A's
  int ha, hb;     // group lane of the equal column in the other row, or -1
  unsigned long long ma, mb;  // group lanes whose A (B) column the other row stores

  __device__ __forceinline__ void load(const int32_t* __restrict__ ciA, int la,
                                       const int32_t* __restrict__ ciB, int lb, int lg) {
    ca = lg < la ? ciA[lg] : INT_MAX;
    cb = lg < lb ? ciB[lg] : INT_MAX;
  }
  __device__ __forceinline__ void rank(int la, int lb, int lg, unsigned long long gm) {
    ra = rb = 0;
    ha = hb = -1;
    group_rank<G>(ca, cb, ra, ha);
    group_rank<G>(cb, ca, rb, hb);
    ma = __ballot(lg < la && ha >= 0) & gm;
    mb = __ballot(lg < lb && hb >= 0) & gm;
  }
};

template <typename T>
__device__ __forceinline__ T round_to(double v) {
  return static_cast<T>(v);
}

// Row bounds of one row of A, B and (optionally) C.
struct RowSpan {
  int a0, la, b0, lb, c0, lc;
};

// Rows handled by one group: R rows, kAddThreads/G groups per block,
// consecutive groups on consecutive rows for each of the R slots, so a
// wave's loads of one slot are contiguous.  All R rows' loads are issued
// before any of them is used, which keeps R times more loads in flight.
template <int G, int R>
__device__ __forceinline__ int slot_row(int r) {
  constexpr int RPB = kAddThreads / G;
  return blockIdx.x * (RPB * R) + r * RPB + (int)(threadIdx.x / G);
}

template <int G, int R, bool WITH_C>
__device__ __forceinline__ void load_spans(int m, const int32_t* __restrict__ rpA,
                                           const int32_t* __restrict__ rpB,
                                           const int32_t* __restrict__ rpC, RowSpan (&sp)[R]) {
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int row = slot_row<G, R>(r);
    sp[r] = RowSpan{0, 0, 0, 0, 0, 0};
    if (row < m) {
      sp[r].a0 = rpA[row];
      sp[r].la = rpA[row + 1];
      sp[r].b0 = rpB[row];
      sp[r].lb = rpB[row + 1];
      if constexpr (WITH_C) {
        sp[r].c0 = rpC[row];
        sp[r].lc = rpC[row + 1];
      }
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    sp[r].la -= sp[r].a0;
    sp[r].lb -= sp[r].b0;
    sp[r].lc -= sp[r].c0;
  }
}

// Union row lengths: cnt[i] = len_A(i) + len_B(i) - |common columns|.
template <int G, int R>
__global__ __launch_bounds__(kAddThreads) void k_add_count(
    int m, const int32_t* __restrict__ rpA, const int32_t* __restrict__ ciA,
    const int32_t* __restrict__ rpB, const int32_t* __restrict__ ciB, int32_t* __restrict__ cnt) {
  const int lg = threadIdx.x & (G - 1);
  const unsigned long long gm = group_bits<G>(threadIdx.x & (kWave - 1));
  RowSpan sp[R];
  load_spans<G, R, false>(m, rpA, rpB, nullptr, sp);
  RegRows<G> rr[R];
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (sp[r].la <= G && sp[r].lb <= G)
      rr[r].load(ciA + sp[r].a0, sp[r].la, ciB + sp[r].b0, sp[r].lb, lg);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int row = slot_row<G, R>(r);
    const int la = sp[r].la, lb = sp[r].lb;
    int common = 0;
    if (la <= G && lb <= G) {  // both rows in registers (group-uniform branch)
      rr[r].rank(la, lb, lg, gm);
      common = __popcll(rr[r].ma);
    } else {  // scan the shorter row against the longer one by binary search
      const int32_t* s = la <= lb ? ciA + sp[r].a0 : ciB + sp[r].b0;
      const int32_t* l = la <= lb ? ciB + sp[r].b0 : ciA + sp[r].a0;
      const int ls = la <= lb ? la : lb, ll = la <= lb ? lb : la;
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
    }
    if (lg == 0 && row < m) cnt[row] = la + lb - common;
  }
}

// One row of C longer than G on either side: chunks of G entries, binary
// search in the other row, ballot counts carried across chunks.
template <int G, typename T>
__device__ __forceinline__ void fill_row_search(const RowSpan& sp, int lg, unsigned long long gm,
                                                unsigned long long below,
                                                const int32_t* __restrict__ ciA,
                                                const T* __restrict__ vA,
                                                const int32_t* __restrict__ ciB,
                                                const T* __restrict__ vB, double alpha,
                                                double beta, int32_t* cc, T* cv) {
#pragma clang fp contract(off)
  const int a0 = sp.a0, la = sp.la, b0 = sp.b0, lb = sp.lb, lc = sp.lc;
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

// Columns (optional) and values of C given C's row pointers.
template <int G, int R, typename T>
__global__ __launch_bounds__(kAddThreads) void k_add_fill(
    int m, const int32_t* __restrict__ rpA, const int32_t* __restrict__ ciA,
    const T* __restrict__ vA, const int32_t* __restrict__ rpB, const int32_t* __restrict__ ciB,
    const T* __restrict__ vB, double alpha, double beta, const int32_t* __restrict__ rpC,
    int32_t* __restrict__ ciC, T* __restrict__ vC) {
  // the products and the sum round separately: no fused multiply-add
  // (the pragma takes the contract flag off the operations written here)
#pragma clang fp contract(off)
  const int lane = threadIdx.x & (kWave - 1);
  const int lg = threadIdx.x & (G - 1);
  const unsigned long long gm = group_bits<G>(lane);
  const unsigned long long below = gm & ((1ull << lane) - 1ull);
  RowSpan sp[R];
  load_spans<G, R, true>(m, rpA, rpB, rpC, sp);
  RegRows<G> rr[R];
  T xa[R], xb[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    xa[r] = T(0);
    xb[r] = T(0);
    if (sp[r].la <= G && sp[r].lb <= G) {  // both rows in registers
      rr[r].load(ciA + sp[r].a0, sp[r].la, ciB + sp[r].b0, sp[r].lb, lg);
      if (lg < sp[r].la) xa[r] = vA[sp[r].a0 + lg];
      if (lg < sp[r].lb) xb[r] = vB[sp[r].b0 + lg];
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const RowSpan& q = sp[r];
    int32_t* cc = ciC ? ciC + q.c0 : nullptr;
    T* cv = vC + q.c0;
    if (q.la <= G && q.lb <= G) {  // group-uniform branch; rows past m are empty
      RegRows<G>& w = rr[r];
      w.rank(q.la, q.lb, lg, gm);
      // B's value for a matched A column, from the B lane that holds it
      const T yb = __shfl(xb[r], (lane & ~(G - 1)) + (w.ha >= 0 ? w.ha : 0));
      const int pa = lg + w.ra - __popcll(w.ma & below);
      if (lg < q.la && (unsigned)pa < (unsigned)q.lc) {
        double v = alpha * static_cast<double>(xa[r]);
        if (w.ha >= 0) {
          const double u = beta * static_cast<double>(yb);
          v = v + u;
        }
        if (cc) cc[pa] = w.ca;
        cv[pa] = round_to<T>(v);
      }
      const int pb = lg + w.rb - __popcll(w.mb & below);
      if (lg < q.lb && w.hb < 0 && (unsigned)pb < (unsigned)q.lc) {
        if (cc) cc[pb] = w.cb;
        cv[pb] = round_to<T>(beta * static_cast<double>(xb[r]));
      }
    } else {
      fill_row_search<G, T>(q, lg, gm, below, ciA, vA, ciB, vB, alpha, beta, cc, cv);
    }
  }
}

// VJP: every stored entry of A (B) reads V at its position in C's row.
// Rows held in registers place their entries as the numeric pass does
// (C's columns are not read; a matched B entry sits where its A partner
// does, by the same formula) and take V from C's row, which is at most
// 2G long there and is loaded two values per lane together with the
// columns, through a lane shuffle; longer rows search C's row.
template <int G, int R, typename T>
__global__ __launch_bounds__(kAddThreads) void k_add_bwd(
    int m, const int32_t* __restrict__ rpA, const int32_t* __restrict__ ciA,
    const int32_t* __restrict__ rpB, const int32_t* __restrict__ ciB,
    const int32_t* __restrict__ rpC, const int32_t* __restrict__ ciC, const T* __restrict__ gC,
    double alpha, double beta, T* __restrict__ gA, T* __restrict__ gB) {
  const int lane = threadIdx.x & (kWave - 1);
  const int lg = threadIdx.x & (G - 1);
  const unsigned long long gm = group_bits<G>(lane);
  const unsigned long long below = gm & ((1ull << lane) - 1ull);
  RowSpan sp[R];
  load_spans<G, R, true>(m, rpA, rpB, rpC, sp);
  RegRows<G> rr[R];
  T v0[R], v1[R];  // V on C's row (at most 2G long here), lanes lg and lg + G
#pragma unroll
  for (int r = 0; r < R; ++r) {
    v0[r] = T(0);
    v1[r] = T(0);
    if (sp[r].la <= G && sp[r].lb <= G) {
      rr[r].load(ciA + sp[r].a0, sp[r].la, ciB + sp[r].b0, sp[r].lb, lg);
      if (lg < sp[r].lc) v0[r] = gC[sp[r].c0 + lg];
      if (lg + G < sp[r].lc) v1[r] = gC[sp[r].c0 + lg + G];
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const RowSpan& q = sp[r];
    const T* g = gC + q.c0;
    if (q.la <= G && q.lb <= G) {
      RegRows<G>& w = rr[r];
      w.rank(q.la, q.lb, lg, gm);
      const int pa = lg + w.ra - __popcll(w.ma & below);
      const int pb = lg + w.rb - __popcll(w.mb & below);
      // V at a position p of C's row, from the lane that loaded it
      const int gb = lane & ~(G - 1);
      const int sa = gb + (pa & (G - 1)), sb = gb + (pb & (G - 1));
      const T a_lo = __shfl(v0[r], sa), a_hi = __shfl(v1[r], sa);
      const T b_lo = __shfl(v0[r], sb), b_hi = __shfl(v1[r], sb);
      if (gA && lg < q.la)
        gA[q.a0 + lg] = (unsigned)pa < (unsigned)q.lc
                            ? round_to<T>(alpha * static_cast<double>(pa < G ? a_lo : a_hi))
                            : T(0);
      if (gB && lg < q.lb)
        gB[q.b0 + lg] = (unsigned)pb < (unsigned)q.lc
                            ? round_to<T>(beta * static_cast<double>(pb < G ? b_lo : b_hi))
                            : T(0);
    } else {
      const int32_t* cc = ciC + q.c0;
      if (gA) {
        for (int t = lg; t < q.la; t += G) {
          const int k = rank_below(cc, q.lc, ciA[q.a0 + t]);  // < lc: pat(A) lies in pat(C)
          gA[q.a0 + t] = k < q.lc ? round_to<T>(alpha * static_cast<double>(g[k])) : T(0);
        }
      }
      if (gB) {
        for (int t = lg; t < q.lb; t += G) {
          const int k = rank_below(cc, q.lc, ciB[q.b0 + t]);
          gB[q.b0 + t] = k < q.lc ? round_to<T>(beta * static_cast<double>(g[k])) : T(0);
        }
      }
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

// Rows per group (see slot_row).
constexpr int kAddRows = 2;

unsigned add_blocks(int m, int g) {
  const long long rpb = (long long)(kAddThreads / g) * kAddRows;
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
  hipLaunchKernelGGL((k_add_fill<G, kAddRows, T>), dim3(add_blocks(m, G)), dim3(kAddThreads), 0, s, m,  \
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
  hipLaunchKernelGGL((k_add_bwd<G, kAddRows, T>), dim3(add_blocks(m, G)), dim3(kAddThreads), 0, s, m,   \
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
  hipLaunchKernelGGL((k_add_count<G, kAddRows>), dim3(add_blocks(m, G)), dim3(kAddThreads), 0, s, m, \
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
