// SpMV forward and backward (Section 3.1.1; Table 1, SpMV row).
//
// Forward: short rows (mean length <= 9) by row blocks staged in LDS: a
// block loads the entries of ROWS consecutive rows with coalesced loads
// (several in flight per thread), keeps the products in LDS, and each
// thread sums one row in entry order; longer rows by G lanes per row (G a
// power of two picked from the mean row length), DPP group sum.
// Backward: one pass over A^T (transpose pattern + perm) yields both
//   gx[j] = sum over column j of vals[e] * gy[row e]    (A^T gy)
//   gvals[e] = gy[row e] * x[j]                         (masked outer product)
// with a deterministic gather; without the transpose, an atomic
// scatter forms A^T gy (the paper's reduction-based product).
#include "internal.hpp"

namespace csrad {
namespace {

constexpr int kThreads = 256;

template <typename T, int G>
__global__ __launch_bounds__(kThreads) void k_spmv(int m, const int32_t* __restrict__ rowptr,
                                                  const int32_t* __restrict__ colind,
                                                  const T* __restrict__ vals,
                                                  const T* __restrict__ x, T* __restrict__ y) {
  const int b = blockIdx.x;
  const int row = b * (kThreads / G) + threadIdx.x / G;
  const int sub = threadIdx.x % G;
  T s = 0;
  if (row < m) {
    const int e1 = rowptr[row + 1];
    for (int e = rowptr[row] + sub; e < e1; e += G) s += ld_stream(&vals[e]) * x[ld_stream(&colind[e])];
  }
  s = group_sum<G>(s);
  if (row < m && sub == 0) y[row] = s;
}

// Row blocks of ROWS rows (one per thread), at most CAP entries staged; a
// block with more entries takes its rows one wave each.  A thread stages
// kStreamU entries per round, their loads issued together.
constexpr int kStreamU = 4;
template <typename T, int ROWS, int CAP>
__global__ __launch_bounds__(ROWS) void k_spmv_stream(int m, const int32_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ colind,
                                                      const T* __restrict__ vals,
                                                      const T* __restrict__ x, T* __restrict__ y) {
  __shared__ T prod[CAP];
  const int r0 = blockIdx.x * ROWS;
  if (r0 >= m) return;
  const int r1 = min(r0 + ROWS, m);
  const int e0 = rowptr[r0], cnt = rowptr[r1] - e0;
  if (cnt <= CAP) {
    for (int t = threadIdx.x; t < cnt; t += kStreamU * ROWS) {
      T pr[kStreamU];
#pragma unroll
      for (int u = 0; u < kStreamU; ++u) {
        const int tt = t + u * ROWS;
        pr[u] = tt < cnt ? ld_stream(&vals[e0 + tt]) * x[ld_stream(&colind[e0 + tt])] : T(0);
      }
#pragma unroll
      for (int u = 0; u < kStreamU; ++u)
        if (t + u * ROWS < cnt) prod[t + u * ROWS] = pr[u];
    }
    __syncthreads();
    const int r = r0 + threadIdx.x;
    if (r < r1) {
      const int a = rowptr[r] - e0, b = rowptr[r + 1] - e0;
      T acc = 0;
      for (int t = a; t < b; ++t) acc += prod[t];
      y[r] = acc;
    }
  } else {
    const int lane = threadIdx.x % kWave;
    for (int r = r0 + threadIdx.x / kWave; r < r1; r += ROWS / kWave) {
      T acc = 0;
      for (int e = rowptr[r] + lane; e < rowptr[r + 1]; e += kWave)
        acc += ld_stream(&vals[e]) * x[ld_stream(&colind[e])];
      acc = group_sum<kWave>(acc);
      if (lane == 0) y[r] = acc;
    }
  }
}

// Gather over A^T: output row j of A^T is column j of A.
template <typename T, int G, int U, bool WANT_GX, bool WANT_GV>
__global__ __launch_bounds__(kThreads) void k_spmv_bwd_gather(
    int n, const int32_t* __restrict__ rpT, const int32_t* __restrict__ ciT,
    const int32_t* __restrict__ perm, const T* __restrict__ vals, const T* __restrict__ x,
    const T* __restrict__ gy, T* __restrict__ gx, T* __restrict__ gv) {
  const int b = blockIdx.x;
  const int j = b * (kThreads / G) + threadIdx.x / G;
  const int sub = threadIdx.x % G;
  T s = 0;
  if (j < n) {
    const T xj = WANT_GV ? x[j] : T(0);
    const int t1 = rpT[j + 1];
    // U entries per lane per round (t = sub, sub + G, ...: the lane sums in
    // row order), loads issued stage by stage
    for (int tb = rpT[j] + sub; tb < t1; tb += G * U) {
      int i[U], e[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int t = tb + u * G;
        i[u] = t < t1 ? ld_stream(&ciT[t]) : -1;
        e[u] = t < t1 ? ld_stream(&perm[t]) : -1;
      }
      T g[U], v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        g[u] = i[u] >= 0 ? gy[i[u]] : T(0);
        v[u] = (WANT_GX && i[u] >= 0) ? vals[e[u]] : T(0);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (i[u] < 0) continue;
        if (WANT_GX) s += v[u] * g[u];
        if (WANT_GV) gv[e[u]] = g[u] * xj;
      }
    }
  }
  if (WANT_GX) {
    s = group_sum<G>(s);
    if (j < n && sub == 0) gx[j] = s;
  }
}

// Row-wise pass over A: gvals (always) and, with ATOMIC, gx += vals*gy
// scattered with atomics (gx must be zeroed first).  U entries per lane per
// round, loads issued together.
template <typename T, int G, int U, bool WANT_GV, bool ATOMIC>
__global__ __launch_bounds__(kThreads) void k_spmv_bwd_rows(
    int m, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
    const T* __restrict__ vals, const T* __restrict__ x, const T* __restrict__ gy,
    T* __restrict__ gx, T* __restrict__ gv) {
  const int b = blockIdx.x;
  const int row = b * (kThreads / G) + threadIdx.x / G;
  const int sub = threadIdx.x % G;
  if (row >= m) return;
  const T g = gy[row];
  const int e1 = rowptr[row + 1];
  for (int eb = rowptr[row] + sub; eb < e1; eb += G * U) {
    int c[U];
#pragma unroll
    for (int u = 0; u < U; ++u) c[u] = eb + u * G < e1 ? colind[eb + u * G] : -1;
    T xv[U], va[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      xv[u] = (WANT_GV && c[u] >= 0) ? x[c[u]] : T(0);
      va[u] = (ATOMIC && c[u] >= 0) ? vals[eb + u * G] : T(0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (c[u] < 0) continue;
      if (WANT_GV) gv[eb + u * G] = g * xv[u];
      if (ATOMIC) atomicAdd(&gx[c[u]], va[u] * g);
    }
  }
}

// The two passes of the split backward in one launch: while both have
// blocks left, even blocks run the gather over A^T for g_x (GG lanes per
// row, one entry per lane) and odd blocks the row-wise value gradient over
// A (GR lanes per row, UR entries per lane), so the scattered gather and
// the latency-bound row pass overlap on the CUs instead of running one
// after the other.  Same arithmetic as the two passes alone.
template <typename T, int GG, int GR, int UR>
__global__ __launch_bounds__(kThreads) void k_spmv_bwd_pair(
    int n, int m, int nbg, int nbr, const int32_t* __restrict__ rpT,
    const int32_t* __restrict__ ciT, const int32_t* __restrict__ perm,
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
    const T* __restrict__ vals, const T* __restrict__ x, const T* __restrict__ gy,
    T* __restrict__ gx, T* __restrict__ gv) {
  const int common = min(nbg, nbr);
  const int b = blockIdx.x;
  int kind, idx;
  if (b < 2 * common) {
    kind = b & 1;
    idx = b >> 1;
  } else {
    kind = nbg > nbr ? 0 : 1;
    idx = common + (b - 2 * common);
  }
  if (kind == 0) {
    const int j = idx * (kThreads / GG) + threadIdx.x / GG;
    const int sub = threadIdx.x % GG;
    T s = 0;
    if (j < n) {
      const int t1 = rpT[j + 1];
      for (int t = rpT[j] + sub; t < t1; t += GG) {
        const int i = ld_stream(&ciT[t]);
        const int e = ld_stream(&perm[t]);
        s += vals[e] * gy[i];
      }
    }
    s = group_sum<GG>(s);
    if (j < n && sub == 0) gx[j] = s;
  } else {
    const int row = idx * (kThreads / GR) + threadIdx.x / GR;
    const int sub = threadIdx.x % GR;
    if (row >= m) return;
    const T g = gy[row];
    const int e1 = rowptr[row + 1];
    for (int eb = rowptr[row] + sub; eb < e1; eb += GR * UR) {
      int c[UR];
#pragma unroll
      for (int u = 0; u < UR; ++u) c[u] = eb + u * GR < e1 ? colind[eb + u * GR] : -1;
      T xv[UR];
#pragma unroll
      for (int u = 0; u < UR; ++u) xv[u] = c[u] >= 0 ? x[c[u]] : T(0);
#pragma unroll
      for (int u = 0; u < UR; ++u)
        if (c[u] >= 0) gv[eb + u * GR] = g * xv[u];
    }
  }
}

template <typename T>
__global__ void k_zero(T* p, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = T(0);
}

// Lanes per row from the mean row length: the smallest power of two that
// covers the mean, capped at a full wavefront.
int lanes_for(long long nnz, int rows) {
  if (rows <= 0) return 1;
  const double mean = (double)nnz / rows;
  int g = 1;
  while (g < 64 && g < mean) g <<= 1;
  return g;
}

template <typename T, int G>
void launch_fwd(int m, const csrad_csr* A, const T* x, T* y, hipStream_t s) {
  const int blocks = (m + kThreads / G - 1) / (kThreads / G);
  hipLaunchKernelGGL((k_spmv<T, G>), dim3(blocks), dim3(kThreads), 0, s, m, A->rowptr, A->colind,
                     static_cast<const T*>(A->vals), x, y);
}

template <typename T>
int spmv_fwd_t(const csrad_csr* A, const void* x, void* y, hipStream_t s) {
  const int m = A->nrows;
  if (m == 0) return CSRAD_OK;
  const T* xx = static_cast<const T*>(x);
  T* yy = static_cast<T*>(y);
  const double mean = (double)A->nnz / m;
  if (mean <= 9.0) {
    // 256-row blocks (128^3 Poisson: 0.052 -> 0.048 ms against 128-row
    // blocks; 512 rows 0.047, 8 entries per round no faster)
    hipLaunchKernelGGL((k_spmv_stream<T, 256, 2560>), dim3((m + 255) / 256), dim3(256), 0, s, m,
                       A->rowptr, A->colind, static_cast<const T*>(A->vals), xx, yy);
    return launch_status();
  }
  switch (lanes_for(A->nnz, m)) {
    case 1: launch_fwd<T, 1>(m, A, xx, yy, s); break;
    case 2: launch_fwd<T, 2>(m, A, xx, yy, s); break;
    case 4: launch_fwd<T, 4>(m, A, xx, yy, s); break;
    case 8: launch_fwd<T, 8>(m, A, xx, yy, s); break;
    case 16: launch_fwd<T, 16>(m, A, xx, yy, s); break;
    case 32: launch_fwd<T, 32>(m, A, xx, yy, s); break;
    default: launch_fwd<T, 64>(m, A, xx, yy, s); break;
  }
  return launch_status();
}

template <typename T, int G, int U, bool GX, bool GV>
void launch_gather(const csrad_csr* A, const csrad_csr* At, const int32_t* perm, const T* x,
                   const T* gy, T* gx, T* gv, hipStream_t s) {
  const int n = A->ncols;
  const int blocks = (n + kThreads / G - 1) / (kThreads / G);
  hipLaunchKernelGGL((k_spmv_bwd_gather<T, G, U, GX, GV>), dim3(blocks), dim3(kThreads), 0, s, n,
                     At->rowptr, At->colind, perm, static_cast<const T*>(A->vals), x, gy, gx, gv);
}

template <typename T, int G, int U>
void gather_g(const csrad_csr* A, const csrad_csr* At, const int32_t* perm, const T* x,
              const T* gy, T* gx, T* gv, hipStream_t s) {
  if (gx && gv) launch_gather<T, G, U, true, true>(A, At, perm, x, gy, gx, gv, s);
  else if (gx) launch_gather<T, G, U, true, false>(A, At, perm, x, gy, gx, gv, s);
  else launch_gather<T, G, U, false, true>(A, At, perm, x, gy, gx, gv, s);
}

template <typename T, int G, int U>
void rows_g(const csrad_csr* A, const T* x, const T* gy, T* gx, T* gv, bool atomic,
            hipStream_t s) {
  const int m = A->nrows;
  const int blocks = (m + kThreads / G - 1) / (kThreads / G);
  const T* v = static_cast<const T*>(A->vals);
  if (atomic && gv)
    hipLaunchKernelGGL((k_spmv_bwd_rows<T, G, U, true, true>), dim3(blocks), dim3(kThreads), 0, s,
                       m, A->rowptr, A->colind, v, x, gy, gx, gv);
  else if (atomic)
    hipLaunchKernelGGL((k_spmv_bwd_rows<T, G, U, false, true>), dim3(blocks), dim3(kThreads), 0, s,
                       m, A->rowptr, A->colind, v, x, gy, gx, gv);
  else
    hipLaunchKernelGGL((k_spmv_bwd_rows<T, G, U, true, false>), dim3(blocks), dim3(kThreads), 0, s,
                       m, A->rowptr, A->colind, v, x, gy, gx, gv);
}

// Lanes per row G and entries per lane U from the lanes_for count L: the
// row-wise pass is a chain of dependent gathers per entry, and a CU's
// resident threads cap the chains in flight, so when the rows are many for
// the chip (rows x L at least 8 times the resident threads) a lane takes
// U = 4 entries with their loads issued together (128^3 Poisson: 63 ->
// 41 us); otherwise one entry per lane.
bool batch_entries(long long rows, int lanes) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  return lanes >= 8 && rows * lanes >= 8ll * cus * 2048;
}

#define CSRAD_GU_SWITCH(L, BATCH, ...)                                \
  if (BATCH) {                                                        \
    switch (L) {                                                      \
      case 8: { constexpr int G = 2, U = 4; __VA_ARGS__; } break;      \
      case 16: { constexpr int G = 4, U = 4; __VA_ARGS__; } break;     \
      case 32: { constexpr int G = 8, U = 4; __VA_ARGS__; } break;     \
      default: { constexpr int G = 16, U = 4; __VA_ARGS__; } break;    \
    }                                                                 \
  } else {                                                            \
    switch (L) {                                                      \
      case 1: { constexpr int G = 1, U = 1; __VA_ARGS__; } break;      \
      case 2: { constexpr int G = 2, U = 1; __VA_ARGS__; } break;      \
      case 4: { constexpr int G = 4, U = 1; __VA_ARGS__; } break;      \
      case 8: { constexpr int G = 8, U = 1; __VA_ARGS__; } break;      \
      case 16: { constexpr int G = 16, U = 1; __VA_ARGS__; } break;    \
      case 32: { constexpr int G = 32, U = 1; __VA_ARGS__; } break;    \
      default: { constexpr int G = 64, U = 1; __VA_ARGS__; } break;    \
    }                                                                 \
  }

template <typename T>
int spmv_bwd_t(const csrad_csr* A, const csrad_csr* At, const int32_t* perm, const void* x,
               const void* gy, void* gx, void* gv, hipStream_t s) {
  const T* xx = static_cast<const T*>(x);
  const T* gg = static_cast<const T*>(gy);
  T* gxx = static_cast<T*>(gx);
  T* gvv = static_cast<T*>(gv);
  if (At) {
    if (A->ncols == 0) return CSRAD_OK;
    // one entry per lane: the gather over A^T is bound by its scattered
    // value reads and gradient writes, not by latency chains (batching
    // measured no faster for g_x alone and slower fused)
    const int L = lanes_for(A->nnz, A->ncols);
    CSRAD_GU_SWITCH(L, false, (gather_g<T, G, U>(A, At, perm, xx, gg, gxx, gvv, s)));
    return launch_status();
  }
  // No transpose: row-wise pass, atomics for A^T gy.
  if (gxx && A->ncols > 0) {
    hipLaunchKernelGGL((k_zero<T>), dim3(1024), dim3(256), 0, s, gxx, (long long)A->ncols);
  }
  if (A->nrows == 0) return launch_status();
  const bool atomic = gxx != nullptr;
  const int L = lanes_for(A->nnz, A->nrows);
  CSRAD_GU_SWITCH(L, batch_entries(A->nrows, L),
                  (rows_g<T, G, U>(A, xx, gg, gxx, gvv, atomic, s)));
  return launch_status();
}

template <typename T, int GG, int GR, int UR>
void launch_pair(const csrad_csr* A, const csrad_csr* At, const int32_t* perm, const T* x,
                 const T* gy, T* gx, T* gv, hipStream_t s) {
  const int n = A->ncols, m = A->nrows;
  const int nbg = (n + kThreads / GG - 1) / (kThreads / GG);
  const int nbr = (m + kThreads / GR - 1) / (kThreads / GR);
  if (nbg + nbr == 0) return;
  hipLaunchKernelGGL((k_spmv_bwd_pair<T, GG, GR, UR>), dim3(nbg + nbr), dim3(kThreads), 0, s, n,
                     m, nbg, nbr, At->rowptr, At->colind, perm, A->rowptr, A->colind,
                     static_cast<const T*>(A->vals), x, gy, gx, gv);
}

template <typename T, int GG>
void pair_g(const csrad_csr* A, const csrad_csr* At, const int32_t* perm, const T* x, const T* gy,
            T* gx, T* gv, hipStream_t s) {
  const int L = lanes_for(A->nnz, A->nrows);
  CSRAD_GU_SWITCH(L, batch_entries(A->nrows, L),
                  (launch_pair<T, GG, G, U>(A, At, perm, x, gy, gx, gv, s)));
}

template <typename T>
int spmv_bwd_split_t(const csrad_csr* A, const csrad_csr* At, const int32_t* perm, const void* x,
                     const void* gy, void* gx, void* gv, hipStream_t s) {
  const T* xx = static_cast<const T*>(x);
  const T* gg = static_cast<const T*>(gy);
  T* gxx = static_cast<T*>(gx);
  T* gvv = static_cast<T*>(gv);
  switch (lanes_for(A->nnz, A->ncols)) {
    case 1: pair_g<T, 1>(A, At, perm, xx, gg, gxx, gvv, s); break;
    case 2: pair_g<T, 2>(A, At, perm, xx, gg, gxx, gvv, s); break;
    case 4: pair_g<T, 4>(A, At, perm, xx, gg, gxx, gvv, s); break;
    case 8: pair_g<T, 8>(A, At, perm, xx, gg, gxx, gvv, s); break;
    case 16: pair_g<T, 16>(A, At, perm, xx, gg, gxx, gvv, s); break;
    case 32: pair_g<T, 32>(A, At, perm, xx, gg, gxx, gvv, s); break;
    default: pair_g<T, 64>(A, At, perm, xx, gg, gxx, gvv, s); break;
  }
  return launch_status();
}

}  // namespace
}  // namespace csrad

using namespace csrad;

extern "C" int csr_spmv_fwd(const csrad_csr* A, const void* x, void* y, void* stream) {
  CSRAD_TRY(check_csr(A, true));
  if ((A->ncols > 0 && !x) || (A->nrows > 0 && !y)) return CSRAD_EINVAL;
  hipStream_t s = as_stream(stream);
  return A->dtype == CSRAD_F32 ? spmv_fwd_t<float>(A, x, y, s) : spmv_fwd_t<double>(A, x, y, s);
}

extern "C" int csr_spmv_bwd(const csrad_csr* A, const csrad_csr* At, const int32_t* perm,
                            const void* x, const void* gy, void* gx, void* gvals, void* stream) {
  CSRAD_TRY(check_csr(A, gx != nullptr));
  if (!gx && !gvals) return CSRAD_OK;
  if (A->nrows > 0 && !gy) return CSRAD_EINVAL;
  if (gvals && A->ncols > 0 && !x) return CSRAD_EINVAL;
  if (At) {
    CSRAD_TRY(check_csr(At, false));
    if (At->nrows != A->ncols || At->ncols != A->nrows || At->nnz != A->nnz) return CSRAD_EINVAL;
    if (A->nnz > 0 && !perm) return CSRAD_EINVAL;
  }
  hipStream_t s = as_stream(stream);
  return A->dtype == CSRAD_F32 ? spmv_bwd_t<float>(A, At, perm, x, gy, gx, gvals, s)
                               : spmv_bwd_t<double>(A, At, perm, x, gy, gx, gvals, s);
}

extern "C" int csr_spmv_bwd_split(const csrad_csr* A, const csrad_csr* At, const int32_t* perm,
                                  const void* x, const void* gy, void* gx, void* gvals,
                                  void* stream) {
  CSRAD_TRY(check_csr(A, true));
  if (!At || !gx || !gvals) return CSRAD_EINVAL;
  if (A->nrows > 0 && !gy) return CSRAD_EINVAL;
  if (A->ncols > 0 && !x) return CSRAD_EINVAL;
  CSRAD_TRY(check_csr(At, false));
  if (At->nrows != A->ncols || At->ncols != A->nrows || At->nnz != A->nnz) return CSRAD_EINVAL;
  if (A->nnz > 0 && !perm) return CSRAD_EINVAL;
  hipStream_t s = as_stream(stream);
  return A->dtype == CSRAD_F32 ? spmv_bwd_split_t<float>(A, At, perm, x, gy, gx, gvals, s)
                               : spmv_bwd_split_t<double>(A, At, perm, x, gy, gx, gvals, s);
}
