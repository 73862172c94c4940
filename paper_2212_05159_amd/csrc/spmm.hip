// SpDMM: sparse times dense, forward and backward (Section 3.1.3;
// Table 1, SpDMM row).  No matrix cores: each stored value is used for
// k multiply-adds against one dense row, so the op is HBM-bound.
//
// A group of LPR lanes owns one sparse row; each lane owns VW consecutive
// columns (16-byte vector loads of dense rows), so k = 64 float32 columns
// are one group of 16 lanes and a wavefront works on four rows at once.
// Wider k loops over column chunks of LPR*VW.
//
// Backward (fused, one pass over A^T):
//   gB[j,:]  = sum over column j of A: vals[e] * gC[i,:]       (A^T gC)
//   gvals[e] = <gC[i,:], B[j,:]>                                (gC B^T on pat(A))
// B[j,:] is the same for every entry of column j, so it is loaded once
// and both gradients come out of the same gC row loads.
#include "internal.hpp"

namespace csrad {
namespace {

constexpr int kThreads = 256;

template <typename T, int VW>
__device__ __forceinline__ Vec<T, VW> load_or_zero(const T* p, bool ok) {
  if (ok) return load_vec<T, VW>(p);
  Vec<T, VW> z;
#pragma unroll
  for (int w = 0; w < VW; ++w) z.v[w] = T(0);
  return z;
}

// Entries are taken kBatch at a time: all index/value loads of a batch,
// then all dense-row loads, then the multiply-adds, so each lane keeps
// kBatch independent 16-byte loads in flight.  Short batches are padded by
// repeating the last entry of the row with a zero weight (addresses stay
// valid, no branch), so summation order is the row order.
constexpr int kBatch = 8;

template <typename T, int VW, int LPR>
__global__ __launch_bounds__(kThreads) void k_spmm_fwd(RowOrder ord, int k,
                                                      const int32_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ colind,
                                                      const T* __restrict__ vals,
                                                      const T* __restrict__ B, long long ldb,
                                                      T* __restrict__ C, long long ldc) {
  constexpr int RPB = kThreads / LPR;
  const int b = blockIdx.x;
  const int row = order_row(ord, b, RPB, threadIdx.x / LPR);
  const int l = threadIdx.x % LPR;
  if (row < 0) return;
  const int e0 = rowptr[row], e1 = rowptr[row + 1];
  for (int c0 = 0; c0 < k; c0 += LPR * VW) {
    const int col = c0 + l * VW;
    if (col >= k) break;
    T acc[VW];
#pragma unroll
    for (int w = 0; w < VW; ++w) acc[w] = T(0);
    for (int eb = e0; eb < e1; eb += kBatch) {
      int c[kBatch];
      T a[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int e = min(eb + u, e1 - 1);
        c[u] = ld_stream(&colind[e]);
        a[u] = eb + u < e1 ? ld_stream(&vals[e]) : T(0);
      }
      Vec<T, VW> bv[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) bv[u] = load_vec<T, VW>(B + (long long)c[u] * ldb + col);
#pragma unroll
      for (int u = 0; u < kBatch; ++u)
#pragma unroll
        for (int w = 0; w < VW; ++w) acc[w] += a[u] * bv[u].v[w];
    }
    Vec<T, VW> out;
#pragma unroll
    for (int w = 0; w < VW; ++w) out.v[w] = acc[w];
    store_vec_stream<T, VW>(C + (long long)row * ldc + col, out);
  }
}

// One pass over A^T.  Row j of A^T lists the rows i of column j of A and,
// through perm, the positions e of those entries in A.  Entries are taken
// kBwdBatch at a time (loads first, then arithmetic), padded as above.
constexpr int kBwdBatch = 8;

template <typename T, int VW, int LPR, bool GB, bool GV>
__global__ __launch_bounds__(kThreads) void k_spmm_bwd_t(
    RowOrder ord, int k, const int32_t* __restrict__ rpT, const int32_t* __restrict__ ciT,
    const int32_t* __restrict__ perm, const T* __restrict__ vals, const T* __restrict__ B,
    long long ldb, const T* __restrict__ G, long long ldg, T* __restrict__ gB, long long ldgb,
    T* __restrict__ gv) {
  constexpr int RPB = kThreads / LPR;
  const int b = blockIdx.x;
  const int j = order_row(ord, b, RPB, threadIdx.x / LPR);
  const int l = threadIdx.x % LPR;
  if (j < 0) return;  // whole group leaves together
  const int t0 = rpT[j], t1 = rpT[j + 1];
  for (int c0 = 0; c0 < k; c0 += LPR * VW) {
    const int col = c0 + l * VW;
    const bool act = col < k;
    Vec<T, VW> bj;
    if (GV) bj = load_or_zero<T, VW>(B + (long long)j * ldb + col, act);
    T acc[VW];
#pragma unroll
    for (int w = 0; w < VW; ++w) acc[w] = T(0);
    for (int tb = t0; tb < t1; tb += kBwdBatch) {
      int e[kBwdBatch];
      T a[kBwdBatch];
      Vec<T, VW> g[kBwdBatch];
#pragma unroll
      for (int u = 0; u < kBwdBatch; ++u) {
        const int t = min(tb + u, t1 - 1);
        const int i = ld_stream(&ciT[t]);
        e[u] = ld_stream(&perm[t]);
        g[u] = load_or_zero<T, VW>(G + (long long)i * ldg + col, act);
      }
      if (GB) {
#pragma unroll
        for (int u = 0; u < kBwdBatch; ++u) a[u] = tb + u < t1 ? vals[e[u]] : T(0);
#pragma unroll
        for (int u = 0; u < kBwdBatch; ++u)
#pragma unroll
          for (int w = 0; w < VW; ++w) acc[w] += a[u] * g[u].v[w];
      }
      if (GV) {
#pragma unroll
        for (int u = 0; u < kBwdBatch; ++u) {
          T d = 0;
#pragma unroll
          for (int w = 0; w < VW; ++w) d += g[u].v[w] * bj.v[w];
          d = group_sum<LPR>(d);
          if (l == 0 && tb + u < t1) gv[e[u]] = c0 == 0 ? d : gv[e[u]] + d;
        }
      }
    }
    if (GB && act) {
      Vec<T, VW> out;
#pragma unroll
      for (int w = 0; w < VW; ++w) out.v[w] = acc[w];
      store_vec_stream<T, VW>(gB + (long long)j * ldgb + col, out);
    }
  }
}

// ---------------------------------------------------------------------
// Cooperative variants for groups of >= 16 lanes (k = 64 float32 or
// wider).  Per batch of 8 entries, lanes 0..7 of each 16-lane DPP row load
// the batch's indices and values once; DPP row_newbcast hands entry u to
// every lane of the row; the dense-row loads are predicated on the batch
// length, so no lane loads padding.  This removes the per-lane index and
// value loads that otherwise dominate the load pipeline.
// ---------------------------------------------------------------------
template <int U>
__device__ __forceinline__ int bcast16(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x150 + U, 0xF, 0xF, false);
}
template <int U>
__device__ __forceinline__ float bcast16(float v) {
  return __int_as_float(bcast16<U>(__float_as_int(v)));
}
template <int U>
__device__ __forceinline__ double bcast16(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = bcast16<U>((int)(b & 0xffffffffll));
  const int hi = bcast16<U>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// out[u] = the value of lane S*u of the DPP row, u < N.
template <typename V, int N, int S = 1, int U = 0>
__device__ __forceinline__ void bcast_all(V mine, V (&out)[N]) {
  if constexpr (U < N) {
    out[U] = bcast16<S * U>(mine);
    bcast_all<V, N, S, U + 1>(mine, out);
  }
}


constexpr int kCoop = 8;

template <typename T, int VW, int LPR>
__global__ __launch_bounds__(kThreads) void k_spmm_fwd_coop(RowOrder ord, int k,
                                                           const int32_t* __restrict__ rowptr,
                                                           const int32_t* __restrict__ colind,
                                                           const T* __restrict__ vals,
                                                           const T* __restrict__ B, long long ldb,
                                                           T* __restrict__ C, long long ldc) {
  static_assert(LPR >= 16, "cooperative path needs whole DPP rows");
  constexpr int RPB = kThreads / LPR;
  const int b = blockIdx.x;
  const int row = order_row(ord, b, RPB, threadIdx.x / LPR);
  const int l = threadIdx.x % LPR, lr = threadIdx.x % 16;
  if (row < 0) return;  // whole group leaves together
  const int e0 = rowptr[row], e1 = rowptr[row + 1];
  for (int c0 = 0; c0 < k; c0 += LPR * VW) {
    const int col = c0 + l * VW;
    const bool act = col < k;
    T acc[VW];
#pragma unroll
    for (int w = 0; w < VW; ++w) acc[w] = T(0);
    for (int eb = e0; eb < e1; eb += kCoop) {
      const int cnt = min(kCoop, e1 - eb);
      int myc = 0;
      T myv = 0;
      if (lr < cnt) {
        myc = ld_stream(&colind[eb + lr]);
        myv = ld_stream(&vals[eb + lr]);
      }
      int c[kCoop];
      T a[kCoop];
      bcast_all<int, kCoop>(myc, c);
      bcast_all<T, kCoop>(myv, a);
      Vec<T, VW> bv[kCoop];
#pragma unroll
      for (int u = 0; u < kCoop; ++u) bv[u] = load_or_zero<T, VW>(B + (long long)c[u] * ldb + col, act && u < cnt);
#pragma unroll
      for (int u = 0; u < kCoop; ++u)
#pragma unroll
        for (int w = 0; w < VW; ++w) acc[w] += a[u] * bv[u].v[w];
    }
    if (act) {
      Vec<T, VW> out;
#pragma unroll
      for (int w = 0; w < VW; ++w) out.v[w] = acc[w];
      store_vec_stream<T, VW>(C + (long long)row * ldc + col, out);
    }
  }
}

template <typename T, int VW, int LPR, bool GB, bool GV>
__global__ __launch_bounds__(kThreads) void k_spmm_bwd_coop(
    RowOrder ord, int k, const int32_t* __restrict__ rpT, const int32_t* __restrict__ ciT,
    const int32_t* __restrict__ perm, const T* __restrict__ vals, const T* __restrict__ B,
    long long ldb, const T* __restrict__ G, long long ldg, T* __restrict__ gB, long long ldgb,
    T* __restrict__ gv) {
  static_assert(LPR >= 16, "cooperative path needs whole DPP rows");
  constexpr int RPB = kThreads / LPR;
  const int b = blockIdx.x;
  const int j = order_row(ord, b, RPB, threadIdx.x / LPR);
  const int l = threadIdx.x % LPR, lr = threadIdx.x % 16;
  if (j < 0) return;  // whole group leaves together
  const int t0 = rpT[j], t1 = rpT[j + 1];
  for (int c0 = 0; c0 < k; c0 += LPR * VW) {
    const int col = c0 + l * VW;
    const bool act = col < k;
    Vec<T, VW> bj;
    if (GV) bj = load_or_zero<T, VW>(B + (long long)j * ldb + col, act);
    T acc[VW];
#pragma unroll
    for (int w = 0; w < VW; ++w) acc[w] = T(0);
    // a 16-lane group takes entry u of the batch in lanes 2u and 2u+1 (the
    // layout the scattered row sums leave); wider groups in lane u
    constexpr int S = LPR == 16 ? 2 : 1;
    for (int tb = t0; tb < t1; tb += kCoop) {
      const int cnt = min(kCoop, t1 - tb);
      const int me = lr / S;
      int myi = 0, mye = 0;
      T mya = 0;
      if (me < cnt) {
        myi = ld_stream(&ciT[tb + me]);
        mye = ld_stream(&perm[tb + me]);
        if (GB) mya = vals[mye];
      }
      int i[kCoop];
      bcast_all<int, kCoop, S>(myi, i);
      Vec<T, VW> g[kCoop];
#pragma unroll
      for (int u = 0; u < kCoop; ++u) g[u] = load_or_zero<T, VW>(G + (long long)i[u] * ldg + col, act && u < cnt);
      if (GB) {
        T a[kCoop];
        bcast_all<T, kCoop, S>(mya, a);
#pragma unroll
        for (int u = 0; u < kCoop; ++u)
#pragma unroll
          for (int w = 0; w < VW; ++w) acc[w] += a[u] * g[u].v[w];
        // an empty statement that reads and rewrites acc keeps the
        // multiply-adds here, ahead of the dot products: sunk past them,
        // they would keep the batch's broadcast values live through the
        // reductions and cost occupancy
#pragma unroll
        for (int w = 0; w < VW; ++w) asm volatile("" : "+v"(acc[w]));
      }
      if (GV) {
        T d[kCoop];
#pragma unroll
        for (int u = 0; u < kCoop; ++u) {
          d[u] = 0;
#pragma unroll
          for (int w = 0; w < VW; ++w) d[u] += g[u].v[w] * bj.v[w];
        }
        if constexpr (LPR == 16) {
          static_assert(kCoop == 8, "the scattered row sums take 8 values");
          const T mine = row_sum_scatter8<T>(d, lr);
          if ((lr & 1) == 0 && me < cnt) gv[mye] = c0 == 0 ? mine : gv[mye] + mine;
        } else {
          T mine = 0;
#pragma unroll
          for (int u = 0; u < kCoop; ++u) {
            const T su = group_sum<LPR>(d[u]);
            if (lr == u) mine = su;
          }
          // lane u of the group's first DPP row owns entry u of the batch
          if (l < cnt) gv[mye] = c0 == 0 ? mine : gv[mye] + mine;
        }
      }
    }
    if (GB && act) {
      Vec<T, VW> out;
#pragma unroll
      for (int w = 0; w < VW; ++w) out.v[w] = acc[w];
      store_vec_stream<T, VW>(gB + (long long)j * ldgb + col, out);
    }
  }
}

// gvals only, row-wise over A (no transpose needed):
//   gvals[e] = <gC[i,:], B[col e,:]>, gC[i,:] loaded once per row.
template <typename T, int VW, int LPR>
__global__ __launch_bounds__(kThreads) void k_sddmm_rows(
    RowOrder ord, int k, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
    const T* __restrict__ B, long long ldb, const T* __restrict__ G, long long ldg,
    T* __restrict__ gv) {
  constexpr int RPB = kThreads / LPR;
  const int b = blockIdx.x;
  const int i = order_row(ord, b, RPB, threadIdx.x / LPR);
  const int l = threadIdx.x % LPR;
  if (i < 0) return;
  const int e0 = rowptr[i], e1 = rowptr[i + 1];
  for (int c0 = 0; c0 < k; c0 += LPR * VW) {
    const int col = c0 + l * VW;
    const bool act = col < k;
    const Vec<T, VW> gi = load_or_zero<T, VW>(G + (long long)i * ldg + col, act);
    for (int eb = e0; eb < e1; eb += kBatch) {
      Vec<T, VW> bv[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int c = ld_stream(&colind[min(eb + u, e1 - 1)]);
        bv[u] = load_or_zero<T, VW>(B + (long long)c * ldb + col, act);
      }
      if constexpr (LPR == 16) {
        // the same dots and scattered row sums as the fused backward's
        // 16-lane groups (the two give the same bits): entry u ends in
        // lanes 2u and 2u+1
        static_assert(kBatch == 8, "the scattered row sums take 8 values");
        T d[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
          d[u] = 0;
#pragma unroll
          for (int w = 0; w < VW; ++w) d[u] += gi.v[w] * bv[u].v[w];
        }
        const T mine = row_sum_scatter8<T>(d, l);
        const int e = eb + (l >> 1);
        if ((l & 1) == 0 && e < e1) gv[e] = c0 == 0 ? mine : gv[e] + mine;
      } else {
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
          T d = 0;
#pragma unroll
          for (int w = 0; w < VW; ++w) d += gi.v[w] * bv[u].v[w];
          d = group_sum<LPR>(d);
          if (l == 0 && eb + u < e1) gv[eb + u] = c0 == 0 ? d : gv[eb + u] + d;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------
// Host dispatch.
// ---------------------------------------------------------------------
struct Shape {
  int vw, lpr;
};

template <typename T>
Shape pick_shape(int k, std::initializer_list<long long> lds,
                 std::initializer_list<const void*> ptrs) {
  constexpr int kVec = 16 / sizeof(T);
  bool vec = (k % kVec) == 0;
  for (long long ld : lds) vec = vec && (ld % kVec) == 0;
  for (const void* p : ptrs) vec = vec && (reinterpret_cast<uintptr_t>(p) % 16) == 0;
  const int vw = vec ? kVec : 1;
  const int lanes = (k + vw - 1) / vw;
  int lpr = 1;
  while (lpr < 64 && lpr < lanes) lpr <<= 1;
  return {vw, lpr};
}

#define CSRAD_LPR_SWITCH(lpr, ...)                        \
  switch (lpr) {                                          \
    case 1: { constexpr int L = 1; __VA_ARGS__; } break;   \
    case 2: { constexpr int L = 2; __VA_ARGS__; } break;   \
    case 4: { constexpr int L = 4; __VA_ARGS__; } break;   \
    case 8: { constexpr int L = 8; __VA_ARGS__; } break;   \
    case 16: { constexpr int L = 16; __VA_ARGS__; } break; \
    case 32: { constexpr int L = 32; __VA_ARGS__; } break; \
    default: { constexpr int L = 64; __VA_ARGS__; } break; \
  }

inline dim3 grid_for(const RowOrder& o, int lpr) {
  return dim3((unsigned)order_blocks(o, kThreads / lpr));
}

template <typename T>
int spmm_fwd_t(const csrad_csr* A, int k, const T* B, long long ldb, T* C, long long ldc,
               const csrad_plan* plan, hipStream_t s) {
  const int m = A->nrows;
  if (m == 0) return CSRAD_OK;
  const Shape sh = pick_shape<T>(k, {ldb, ldc}, {B, C});
  const T* v = static_cast<const T*>(A->vals);
  if (sh.vw == 1) {
    CSRAD_LPR_SWITCH(sh.lpr, {
      const RowOrder o = make_order(m, kThreads / L, plan);
      hipLaunchKernelGGL((k_spmm_fwd<T, 1, L>), grid_for(o, L), dim3(kThreads), 0, s, o, k,
                         A->rowptr, A->colind, v, B, ldb, C, ldc);
    });
  } else {
    constexpr int VW = 16 / sizeof(T);
    CSRAD_LPR_SWITCH(sh.lpr, {
      const RowOrder o = make_order(m, kThreads / L, plan);
      if constexpr (L >= 16)
        hipLaunchKernelGGL((k_spmm_fwd_coop<T, VW, L>), grid_for(o, L), dim3(kThreads), 0, s, o,
                           k, A->rowptr, A->colind, v, B, ldb, C, ldc);
      else
        hipLaunchKernelGGL((k_spmm_fwd<T, VW, L>), grid_for(o, L), dim3(kThreads), 0, s, o, k,
                           A->rowptr, A->colind, v, B, ldb, C, ldc);
    });
  }
  return launch_status();
}

template <typename T, int VW, int L>
void launch_bwd_t(const csrad_csr* A, const csrad_csr* At, const int32_t* perm, int k,
                  const T* B, long long ldb, const T* G, long long ldg, T* gB, long long ldgb,
                  T* gv, const csrad_plan* plan, hipStream_t s) {
  const T* v = static_cast<const T*>(A->vals);
  const RowOrder o = make_order(A->ncols, kThreads / L, plan);
  const dim3 grid = grid_for(o, L);
  if constexpr (L >= 16 && VW > 1) {
    if (gB && gv)
      hipLaunchKernelGGL((k_spmm_bwd_coop<T, VW, L, true, true>), grid, dim3(kThreads), 0, s, o, k,
                         At->rowptr, At->colind, perm, v, B, ldb, G, ldg, gB, ldgb, gv);
    else
      hipLaunchKernelGGL((k_spmm_bwd_coop<T, VW, L, true, false>), grid, dim3(kThreads), 0, s, o,
                         k, At->rowptr, At->colind, perm, v, B, ldb, G, ldg, gB, ldgb, gv);
  } else {
    if (gB && gv)
      hipLaunchKernelGGL((k_spmm_bwd_t<T, VW, L, true, true>), grid, dim3(kThreads), 0, s, o, k,
                         At->rowptr, At->colind, perm, v, B, ldb, G, ldg, gB, ldgb, gv);
    else
      hipLaunchKernelGGL((k_spmm_bwd_t<T, VW, L, true, false>), grid, dim3(kThreads), 0, s, o, k,
                         At->rowptr, At->colind, perm, v, B, ldb, G, ldg, gB, ldgb, gv);
  }
}

template <typename T>
int spmm_bwd_t(const csrad_csr* A, const csrad_csr* At, const int32_t* perm, int k, const T* B,
               long long ldb, const T* G, long long ldg, T* gB, long long ldgb, T* gv,
               const csrad_plan* plan, hipStream_t s) {
  if (gB) {
    if (A->ncols == 0) return CSRAD_OK;
    const Shape sh = pick_shape<T>(k, {ldb, ldg, ldgb}, {B, G, gB});
    if (sh.vw == 1) {
      CSRAD_LPR_SWITCH(sh.lpr, (launch_bwd_t<T, 1, L>(A, At, perm, k, B, ldb, G, ldg, gB, ldgb,
                                                      gv, plan, s)));
    } else {
      constexpr int VW = 16 / sizeof(T);
      CSRAD_LPR_SWITCH(sh.lpr, (launch_bwd_t<T, VW, L>(A, At, perm, k, B, ldb, G, ldg, gB, ldgb,
                                                       gv, plan, s)));
    }
    return launch_status();
  }
  // gvals only: row-wise masked product over A, no transpose.
  const int m = A->nrows;
  if (m == 0) return CSRAD_OK;
  const Shape sh = pick_shape<T>(k, {ldb, ldg}, {B, G});
  if (sh.vw == 1) {
    CSRAD_LPR_SWITCH(sh.lpr, {
      const RowOrder o = make_order(m, kThreads / L, plan);
      hipLaunchKernelGGL((k_sddmm_rows<T, 1, L>), grid_for(o, L), dim3(kThreads), 0, s, o, k,
                         A->rowptr, A->colind, B, ldb, G, ldg, gv);
    });
  } else {
    constexpr int VW = 16 / sizeof(T);
    CSRAD_LPR_SWITCH(sh.lpr, {
      const RowOrder o = make_order(m, kThreads / L, plan);
      hipLaunchKernelGGL((k_sddmm_rows<T, VW, L>), grid_for(o, L), dim3(kThreads), 0, s, o, k,
                         A->rowptr, A->colind, B, ldb, G, ldg, gv);
    });
  }
  return launch_status();
}

}  // namespace
}  // namespace csrad

using namespace csrad;

extern "C" int csr_spmm_fwd(const csrad_csr* A, int32_t k, const void* B, int64_t ldb, void* C,
                            int64_t ldc, const csrad_plan* plan, void* stream) {
  CSRAD_TRY(check_csr(A, true));
  CSRAD_TRY(check_plan(plan, A->nrows));
  if (k <= 0 || ldb < k || ldc < k) return CSRAD_EINVAL;
  if ((A->ncols > 0 && !B) || (A->nrows > 0 && !C)) return CSRAD_EINVAL;
  hipStream_t s = as_stream(stream);
  if (A->dtype == CSRAD_F32)
    return spmm_fwd_t<float>(A, k, static_cast<const float*>(B), ldb, static_cast<float*>(C), ldc,
                             plan, s);
  return spmm_fwd_t<double>(A, k, static_cast<const double*>(B), ldb, static_cast<double*>(C), ldc,
                            plan, s);
}

extern "C" int csr_spmm_bwd(const csrad_csr* A, const csrad_csr* At, const int32_t* perm,
                            int32_t k, const void* B, int64_t ldb, const void* gC, int64_t ldgc,
                            void* gB, int64_t ldgb, void* gvals, const csrad_plan* plan,
                            void* stream) {
  CSRAD_TRY(check_csr(A, gB != nullptr));
  CSRAD_TRY(check_plan(plan, gB ? A->ncols : A->nrows));
  if (!gB && !gvals) return CSRAD_OK;
  if (k <= 0 || ldgc < k) return CSRAD_EINVAL;
  if (A->nrows > 0 && !gC) return CSRAD_EINVAL;
  if (gvals && (ldb < k || (A->ncols > 0 && !B))) return CSRAD_EINVAL;
  if (gB) {
    if (ldgb < k || !At) return CSRAD_EINVAL;
    CSRAD_TRY(check_csr(At, false));
    if (At->nrows != A->ncols || At->ncols != A->nrows || At->nnz != A->nnz) return CSRAD_EINVAL;
    if (A->nnz > 0 && !perm) return CSRAD_EINVAL;
  }
  hipStream_t s = as_stream(stream);
  if (A->dtype == CSRAD_F32)
    return spmm_bwd_t<float>(A, At, perm, k, static_cast<const float*>(B), ldb,
                             static_cast<const float*>(gC), ldgc, static_cast<float*>(gB), ldgb,
                             static_cast<float*>(gvals), plan, s);
  return spmm_bwd_t<double>(A, At, perm, k, static_cast<const double*>(B), ldb,
                            static_cast<const double*>(gC), ldgc, static_cast<double*>(gB), ldgb,
                            static_cast<double*>(gvals), plan, s);
}
