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
// block with more entries takes its rows one wave each.
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
    for (int t = threadIdx.x; t < cnt; t += 4 * ROWS) {
      T pr[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int tt = t + u * ROWS;
        pr[u] = tt < cnt ? ld_stream(&vals[e0 + tt]) * x[ld_stream(&colind[e0 + tt])] : T(0);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
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
template <typename T, int G, bool WANT_GX, bool WANT_GV>
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
    for (int t = rpT[j] + sub; t < t1; t += G) {
      const int i = ld_stream(&ciT[t]);
      const int e = ld_stream(&perm[t]);
      const T g = gy[i];
      if (WANT_GX) s += vals[e] * g;
      if (WANT_GV) gv[e] = g * xj;
    }
  }
  if (WANT_GX) {
    s = group_sum<G>(s);
    if (j < n && sub == 0) gx[j] = s;
  }
}

// Row-wise pass over A: gvals (always) and, with ATOMIC, gx += vals*gy
// scattered with atomics (gx must be zeroed first).
template <typename T, int G, bool WANT_GV, bool ATOMIC>
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
  for (int e = rowptr[row] + sub; e < e1; e += G) {
    const int c = colind[e];
    if (WANT_GV) gv[e] = g * x[c];
    if (ATOMIC) atomicAdd(&gx[c], vals[e] * g);
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
    hipLaunchKernelGGL((k_spmv_stream<T, 128, 1280>), dim3((m + 127) / 128), dim3(128), 0, s, m,
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

template <typename T, int G, bool GX, bool GV>
void launch_gather(const csrad_csr* A, const csrad_csr* At, const int32_t* perm, const T* x,
                   const T* gy, T* gx, T* gv, hipStream_t s) {
  const int n = A->ncols;
  const int blocks = (n + kThreads / G - 1) / (kThreads / G);
  hipLaunchKernelGGL((k_spmv_bwd_gather<T, G, GX, GV>), dim3(blocks), dim3(kThreads), 0, s, n,
                     At->rowptr, At->colind, perm, static_cast<const T*>(A->vals), x, gy, gx, gv);
}

template <typename T, int G>
void gather_g(const csrad_csr* A, const csrad_csr* At, const int32_t* perm, const T* x,
              const T* gy, T* gx, T* gv, hipStream_t s) {
  if (gx && gv) launch_gather<T, G, true, true>(A, At, perm, x, gy, gx, gv, s);
  else if (gx) launch_gather<T, G, true, false>(A, At, perm, x, gy, gx, gv, s);
  else launch_gather<T, G, false, true>(A, At, perm, x, gy, gx, gv, s);
}

template <typename T, int G>
void rows_g(const csrad_csr* A, const T* x, const T* gy, T* gx, T* gv, bool atomic,
            hipStream_t s) {
  const int m = A->nrows;
  const int blocks = (m + kThreads / G - 1) / (kThreads / G);
  const T* v = static_cast<const T*>(A->vals);
  if (atomic && gv)
    hipLaunchKernelGGL((k_spmv_bwd_rows<T, G, true, true>), dim3(blocks), dim3(kThreads), 0, s, m,
                       A->rowptr, A->colind, v, x, gy, gx, gv);
  else if (atomic)
    hipLaunchKernelGGL((k_spmv_bwd_rows<T, G, false, true>), dim3(blocks), dim3(kThreads), 0, s, m,
                       A->rowptr, A->colind, v, x, gy, gx, gv);
  else
    hipLaunchKernelGGL((k_spmv_bwd_rows<T, G, true, false>), dim3(blocks), dim3(kThreads), 0, s, m,
                       A->rowptr, A->colind, v, x, gy, gx, gv);
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
    switch (lanes_for(A->nnz, A->ncols)) {
      case 1: gather_g<T, 1>(A, At, perm, xx, gg, gxx, gvv, s); break;
      case 2: gather_g<T, 2>(A, At, perm, xx, gg, gxx, gvv, s); break;
      case 4: gather_g<T, 4>(A, At, perm, xx, gg, gxx, gvv, s); break;
      case 8: gather_g<T, 8>(A, At, perm, xx, gg, gxx, gvv, s); break;
      case 16: gather_g<T, 16>(A, At, perm, xx, gg, gxx, gvv, s); break;
      case 32: gather_g<T, 32>(A, At, perm, xx, gg, gxx, gvv, s); break;
      default: gather_g<T, 64>(A, At, perm, xx, gg, gxx, gvv, s); break;
    }
    return launch_status();
  }
  // No transpose: row-wise pass, atomics for A^T gy.
  if (gxx && A->ncols > 0) {
    hipLaunchKernelGGL((k_zero<T>), dim3(1024), dim3(256), 0, s, gxx, (long long)A->ncols);
  }
  if (A->nrows == 0) return launch_status();
  const bool atomic = gxx != nullptr;
  switch (lanes_for(A->nnz, A->nrows)) {
    case 1: rows_g<T, 1>(A, xx, gg, gxx, gvv, atomic, s); break;
    case 2: rows_g<T, 2>(A, xx, gg, gxx, gvv, atomic, s); break;
    case 4: rows_g<T, 4>(A, xx, gg, gxx, gvv, atomic, s); break;
    case 8: rows_g<T, 8>(A, xx, gg, gxx, gvv, atomic, s); break;
    case 16: rows_g<T, 16>(A, xx, gg, gxx, gvv, atomic, s); break;
    case 32: rows_g<T, 32>(A, xx, gg, gxx, gvv, atomic, s); break;
    default: rows_g<T, 64>(A, xx, gg, gxx, gvv, atomic, s); break;
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
