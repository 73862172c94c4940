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
constexpr int kUnroll = 4;

template <typename T, int VW>
__device__ __forceinline__ Vec<T, VW> load_or_zero(const T* p, bool ok) {
  if (ok) return load_vec<T, VW>(p);
  Vec<T, VW> z;
#pragma unroll
  for (int w = 0; w < VW; ++w) z.v[w] = T(0);
  return z;
}

template <typename T, int VW, int LPR>
__global__ __launch_bounds__(kThreads) void k_spmm_fwd(int m, int k,
                                                      const int32_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ colind,
                                                      const T* __restrict__ vals,
                                                      const T* __restrict__ B, long long ldb,
                                                      T* __restrict__ C, long long ldc) {
  constexpr int RPB = kThreads / LPR;
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int row = b * RPB + threadIdx.x / LPR;
  const int l = threadIdx.x % LPR;
  if (row >= m) return;
  const int e0 = rowptr[row], e1 = rowptr[row + 1];
  for (int c0 = 0; c0 < k; c0 += LPR * VW) {
    const int col = c0 + l * VW;
    if (col >= k) break;
    T acc[VW];
#pragma unroll
    for (int w = 0; w < VW; ++w) acc[w] = T(0);
    int e = e0;
    for (; e + kUnroll <= e1; e += kUnroll) {
      int c[kUnroll];
      T a[kUnroll];
      Vec<T, VW> bv[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        c[u] = ld_stream(&colind[e + u]);
        a[u] = ld_stream(&vals[e + u]);
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) bv[u] = load_vec<T, VW>(B + (long long)c[u] * ldb + col);
#pragma unroll
      for (int u = 0; u < kUnroll; ++u)
#pragma unroll
        for (int w = 0; w < VW; ++w) acc[w] += a[u] * bv[u].v[w];
    }
    for (; e < e1; ++e) {
      const int c = ld_stream(&colind[e]);
      const T a = ld_stream(&vals[e]);
      const Vec<T, VW> bv = load_vec<T, VW>(B + (long long)c * ldb + col);
#pragma unroll
      for (int w = 0; w < VW; ++w) acc[w] += a * bv.v[w];
    }
    Vec<T, VW> out;
#pragma unroll
    for (int w = 0; w < VW; ++w) out.v[w] = acc[w];
    store_vec<T, VW>(C + (long long)row * ldc + col, out);
  }
}

// One pass over A^T.  Row j of A^T lists the rows i of column j of A and,
// through perm, the positions e of those entries in A.
template <typename T, int VW, int LPR, bool GB, bool GV>
__global__ __launch_bounds__(kThreads) void k_spmm_bwd_t(
    int n, int k, const int32_t* __restrict__ rpT, const int32_t* __restrict__ ciT,
    const int32_t* __restrict__ perm, const T* __restrict__ vals, const T* __restrict__ B,
    long long ldb, const T* __restrict__ G, long long ldg, T* __restrict__ gB, long long ldgb,
    T* __restrict__ gv) {
  constexpr int RPB = kThreads / LPR;
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int j = b * RPB + threadIdx.x / LPR;
  const int l = threadIdx.x % LPR;
  if (j >= n) return;  // whole group leaves together
  const int t0 = rpT[j], t1 = rpT[j + 1];
  for (int c0 = 0; c0 < k; c0 += LPR * VW) {
    const int col = c0 + l * VW;
    const bool act = col < k;
    Vec<T, VW> bj;
    if (GV) bj = load_or_zero<T, VW>(B + (long long)j * ldb + col, act);
    T acc[VW];
#pragma unroll
    for (int w = 0; w < VW; ++w) acc[w] = T(0);
    int t = t0;
    for (; t + 2 <= t1; t += 2) {
      const int i0 = ld_stream(&ciT[t]), i1 = ld_stream(&ciT[t + 1]);
      const int ea = ld_stream(&perm[t]), eb = ld_stream(&perm[t + 1]);
      const Vec<T, VW> g0 = load_or_zero<T, VW>(G + (long long)i0 * ldg + col, act);
      const Vec<T, VW> g1 = load_or_zero<T, VW>(G + (long long)i1 * ldg + col, act);
      if (GB) {
        const T a0 = vals[ea], a1 = vals[eb];
#pragma unroll
        for (int w = 0; w < VW; ++w) acc[w] += a0 * g0.v[w];
#pragma unroll
        for (int w = 0; w < VW; ++w) acc[w] += a1 * g1.v[w];
      }
      if (GV) {
        T d0 = 0, d1 = 0;
#pragma unroll
        for (int w = 0; w < VW; ++w) {
          d0 += g0.v[w] * bj.v[w];
          d1 += g1.v[w] * bj.v[w];
        }
        d0 = group_sum<LPR>(d0);
        d1 = group_sum<LPR>(d1);
        if (l == 0) {
          gv[ea] = c0 == 0 ? d0 : gv[ea] + d0;
          gv[eb] = c0 == 0 ? d1 : gv[eb] + d1;
        }
      }
    }
    if (t < t1) {
      const int i0 = ld_stream(&ciT[t]);
      const int ea = ld_stream(&perm[t]);
      const Vec<T, VW> g0 = load_or_zero<T, VW>(G + (long long)i0 * ldg + col, act);
      if (GB) {
        const T a0 = vals[ea];
#pragma unroll
        for (int w = 0; w < VW; ++w) acc[w] += a0 * g0.v[w];
      }
      if (GV) {
        T d0 = 0;
#pragma unroll
        for (int w = 0; w < VW; ++w) d0 += g0.v[w] * bj.v[w];
        d0 = group_sum<LPR>(d0);
        if (l == 0) gv[ea] = c0 == 0 ? d0 : gv[ea] + d0;
      }
    }
    if (GB && act) {
      Vec<T, VW> out;
#pragma unroll
      for (int w = 0; w < VW; ++w) out.v[w] = acc[w];
      store_vec<T, VW>(gB + (long long)j * ldgb + col, out);
    }
  }
}

// gvals only, row-wise over A (no transpose needed):
//   gvals[e] = <gC[i,:], B[col e,:]>, gC[i,:] loaded once per row.
template <typename T, int VW, int LPR>
__global__ __launch_bounds__(kThreads) void k_sddmm_rows(
    int m, int k, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
    const T* __restrict__ B, long long ldb, const T* __restrict__ G, long long ldg,
    T* __restrict__ gv) {
  constexpr int RPB = kThreads / LPR;
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int i = b * RPB + threadIdx.x / LPR;
  const int l = threadIdx.x % LPR;
  if (i >= m) return;
  const int e0 = rowptr[i], e1 = rowptr[i + 1];
  for (int c0 = 0; c0 < k; c0 += LPR * VW) {
    const int col = c0 + l * VW;
    const bool act = col < k;
    const Vec<T, VW> gi = load_or_zero<T, VW>(G + (long long)i * ldg + col, act);
    for (int e = e0; e < e1; ++e) {
      const int c = ld_stream(&colind[e]);
      const Vec<T, VW> bv = load_or_zero<T, VW>(B + (long long)c * ldb + col, act);
      T d = 0;
#pragma unroll
      for (int w = 0; w < VW; ++w) d += gi.v[w] * bv.v[w];
      d = group_sum<LPR>(d);
      if (l == 0) gv[e] = c0 == 0 ? d : gv[e] + d;
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

inline unsigned blocks_for(int rows, int lpr) {
  const int rpb = kThreads / lpr;
  return (unsigned)((rows + rpb - 1) / rpb);
}

template <typename T>
int spmm_fwd_t(const csrad_csr* A, int k, const T* B, long long ldb, T* C, long long ldc,
               hipStream_t s) {
  const int m = A->nrows;
  if (m == 0) return CSRAD_OK;
  const Shape sh = pick_shape<T>(k, {ldb, ldc}, {B, C});
  const T* v = static_cast<const T*>(A->vals);
  if (sh.vw == 1) {
    CSRAD_LPR_SWITCH(sh.lpr, hipLaunchKernelGGL((k_spmm_fwd<T, 1, L>), dim3(blocks_for(m, L)),
                                                dim3(kThreads), 0, s, m, k, A->rowptr, A->colind,
                                                v, B, ldb, C, ldc));
  } else {
    constexpr int VW = 16 / sizeof(T);
    CSRAD_LPR_SWITCH(sh.lpr, hipLaunchKernelGGL((k_spmm_fwd<T, VW, L>), dim3(blocks_for(m, L)),
                                                dim3(kThreads), 0, s, m, k, A->rowptr, A->colind,
                                                v, B, ldb, C, ldc));
  }
  return launch_status();
}

template <typename T, int VW, int L>
void launch_bwd_t(const csrad_csr* A, const csrad_csr* At, const int32_t* perm, int k,
                  const T* B, long long ldb, const T* G, long long ldg, T* gB, long long ldgb,
                  T* gv, hipStream_t s) {
  const int n = A->ncols;
  const T* v = static_cast<const T*>(A->vals);
  const dim3 grid(blocks_for(n, L));
  if (gB && gv)
    hipLaunchKernelGGL((k_spmm_bwd_t<T, VW, L, true, true>), grid, dim3(kThreads), 0, s, n, k,
                       At->rowptr, At->colind, perm, v, B, ldb, G, ldg, gB, ldgb, gv);
  else
    hipLaunchKernelGGL((k_spmm_bwd_t<T, VW, L, true, false>), grid, dim3(kThreads), 0, s, n, k,
                       At->rowptr, At->colind, perm, v, B, ldb, G, ldg, gB, ldgb, gv);
}

template <typename T>
int spmm_bwd_t(const csrad_csr* A, const csrad_csr* At, const int32_t* perm, int k, const T* B,
               long long ldb, const T* G, long long ldg, T* gB, long long ldgb, T* gv,
               hipStream_t s) {
  if (gB) {
    if (A->ncols == 0) return CSRAD_OK;
    const Shape sh = pick_shape<T>(k, {ldb, ldg, ldgb}, {B, G, gB});
    if (sh.vw == 1) {
      CSRAD_LPR_SWITCH(sh.lpr, (launch_bwd_t<T, 1, L>(A, At, perm, k, B, ldb, G, ldg, gB, ldgb,
                                                      gv, s)));
    } else {
      constexpr int VW = 16 / sizeof(T);
      CSRAD_LPR_SWITCH(sh.lpr, (launch_bwd_t<T, VW, L>(A, At, perm, k, B, ldb, G, ldg, gB, ldgb,
                                                       gv, s)));
    }
    return launch_status();
  }
  // gvals only: row-wise masked product, no transpose.
  const int m = A->nrows;
  if (m == 0) return CSRAD_OK;
  const Shape sh = pick_shape<T>(k, {ldb, ldg}, {B, G});
  if (sh.vw == 1) {
    CSRAD_LPR_SWITCH(sh.lpr, hipLaunchKernelGGL((k_sddmm_rows<T, 1, L>), dim3(blocks_for(m, L)),
                                                dim3(kThreads), 0, s, m, k, A->rowptr, A->colind,
                                                B, ldb, G, ldg, gv));
  } else {
    constexpr int VW = 16 / sizeof(T);
    CSRAD_LPR_SWITCH(sh.lpr, hipLaunchKernelGGL((k_sddmm_rows<T, VW, L>), dim3(blocks_for(m, L)),
                                                dim3(kThreads), 0, s, m, k, A->rowptr, A->colind,
                                                B, ldb, G, ldg, gv));
  }
  return launch_status();
}

}  // namespace
}  // namespace csrad

using namespace csrad;

extern "C" int csr_spmm_fwd(const csrad_csr* A, int32_t k, const void* B, int64_t ldb, void* C,
                            int64_t ldc, void* stream) {
  CSRAD_TRY(check_csr(A, true));
  if (k <= 0 || ldb < k || ldc < k) return CSRAD_EINVAL;
  if ((A->ncols > 0 && !B) || (A->nrows > 0 && !C)) return CSRAD_EINVAL;
  hipStream_t s = as_stream(stream);
  if (A->dtype == CSRAD_F32)
    return spmm_fwd_t<float>(A, k, static_cast<const float*>(B), ldb, static_cast<float*>(C), ldc, s);
  return spmm_fwd_t<double>(A, k, static_cast<const double*>(B), ldb, static_cast<double*>(C), ldc,
                            s);
}

extern "C" int csr_spmm_bwd(const csrad_csr* A, const csrad_csr* At, const int32_t* perm,
                            int32_t k, const void* B, int64_t ldb, const void* gC, int64_t ldgc,
                            void* gB, int64_t ldgb, void* gvals, void* stream) {
  CSRAD_TRY(check_csr(A, gB != nullptr));
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
                             static_cast<float*>(gvals), s);
  return spmm_bwd_t<double>(A, At, perm, k, static_cast<const double*>(B), ldb,
                            static_cast<const double*>(gC), ldgc, static_cast<double*>(gB), ldgb,
                            static_cast<double*>(gvals), s);
}
