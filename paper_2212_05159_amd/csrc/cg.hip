// Conjugate gradients (the Krylov solver of Section 4.3) and its reverse
// mode, as device-resident steps: scalars never leave the GPU, so a step
// needs no host synchronisation and can be captured in a graph.
//
// Forward step t (x0 = 0, r0 = b, p0 = b, rho0 = b.b):
//   q = A p, sigma = p.q, alpha = rho/sigma, x += alpha p, r -= alpha q,
//   rho' = r.r, beta = rho'/rho, p = r + beta p.
// Once rho is exactly zero, alpha = beta = 0 (converged; no 0/0).
// Dot products accumulate in float64 whatever the vector type: per-block
// partial sums, then one block adds them in a fixed order, so every step is
// bit-reproducible (checkpoint recomputation relies on it).
//
// Reverse step t (adjoints xb, rb, pb, qb of x, r, p, q and rhob of rho_{t+1}):
//   rb += gR_t;  betab = pb.p_t;  rb += pb;  pb *= beta
//   rhob += betab/rho;  rhob_t = -betab rho'/rho^2
//   rb += 2 rhob r_{t+1};  alphab = -rb.q_t + xb.p_t;  qb = -alpha rb;  pb += alpha xb
//   rhob_t += alphab/sigma;  sigmab = -alphab rho/sigma^2
//   qb += sigmab p_t;  pb += sigmab q_t + A^T qb;  gvals[(i,j)] += qb_i p_j
//   rhob = rhob_t
// and after step 0: gb = rb + pb + 2 rhob b.
#include "internal.hpp"

namespace csrad {
namespace {

constexpr int kThreads = 256;
constexpr int kVecBlocksMax = 2048;

// Scalar slots of the device state (float64).
enum : int {
  S_RHO = 0,    // current rho
  S_SIGMA,      // last sigma
  S_ALPHA,      // last alpha
  S_RHO1,       // last rho'
  S_BETA,       // last beta
  S_RHOB,       // reverse: adjoint of rho_{t+1}
  S_RHOB_T,     // reverse: adjoint of rho_t being accumulated
  S_SIGMAB,     // reverse: adjoint of sigma
  S_COUNT = 8
};
constexpr int kHistStride = 5;  // per-step history: rho, sigma, alpha, rho', beta

__device__ double block_sum_double(double v, double* sm) {
  // fixed-order tree: wave butterflies then the 4 wave sums in order
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x / kWave;
  if (threadIdx.x % kWave == 0) sm[w] = v;
  __syncthreads();
  double t = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kThreads / kWave; ++i) t += sm[i];
  __syncthreads();
  return t;
}

// Fixed-order sum of nb partials by one block.
__device__ double reduce_partials(const double* __restrict__ part, int nb, double* sm) {
  double v = 0;
  for (int i = threadIdx.x; i < nb; i += kThreads) v += part[i];
  return block_sum_double(v, sm);
}

template <typename T>
__global__ void k_cg_init(int n, const T* __restrict__ b, T* __restrict__ x, T* __restrict__ r,
                          T* __restrict__ p, double* __restrict__ part) {
  __shared__ double sm[kThreads / kWave];
  double acc = 0;
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
    const T bi = b[i];
    x[i] = T(0);
    r[i] = bi;
    p[i] = bi;
    acc += (double)bi * (double)bi;
  }
  const double s = block_sum_double(acc, sm);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_cg_init_scal(const double* __restrict__ part, int nb, double* __restrict__ scal,
                               int* __restrict__ step) {
  __shared__ double sm[kThreads / kWave];
  const double rho = reduce_partials(part, nb, sm);
  if (threadIdx.x == 0) {
    for (int i = 0; i < S_COUNT; ++i) scal[i] = 0.0;
    scal[S_RHO] = rho;
    *step = 0;
  }
}

// q = A p and the block's share of p.q.
template <typename T, int G>
__global__ __launch_bounds__(kThreads) void k_cg_spmv_dot(int n, const int32_t* __restrict__ rp,
                                                          const int32_t* __restrict__ ci,
                                                          const T* __restrict__ v,
                                                          const T* __restrict__ p,
                                                          T* __restrict__ q,
                                                          T* __restrict__ p_save,
                                                          double* __restrict__ part) {
  __shared__ double sm[kThreads / kWave];
  // G lanes per row; the block strides over row groups (grid capped).
  constexpr int RPB = kThreads / G;
  const int sub = threadIdx.x % G;
  double d = 0;
  for (int base = blockIdx.x * RPB; base < n; base += gridDim.x * RPB) {
    const int row = base + threadIdx.x / G;
    T s = 0;
    if (row < n) {
      const int e1 = rp[row + 1];
      for (int e = rp[row] + sub; e < e1; e += G) s += v[e] * p[ci[e]];
    }
    s = group_sum<G>(s);
    if (row < n && sub == 0) {
      const T pr = p[row];
      q[row] = s;
      if (p_save) p_save[row] = pr;
      d += (double)pr * (double)s;
    }
  }
  d = block_sum_double(d, sm);
  if (threadIdx.x == 0) part[blockIdx.x] = d;
}

__global__ void k_cg_alpha(const double* __restrict__ part, int nb, double* __restrict__ scal) {
  __shared__ double sm[kThreads / kWave];
  const double sigma = reduce_partials(part, nb, sm);
  if (threadIdx.x == 0) {
    const double rho = scal[S_RHO];
    scal[S_SIGMA] = sigma;
    scal[S_ALPHA] = rho != 0.0 ? rho / sigma : 0.0;
  }
}

template <typename T>
__global__ void k_cg_update(int n, const T* __restrict__ p, const T* __restrict__ q,
                            T* __restrict__ x, T* __restrict__ r, T* __restrict__ r_save,
                            const double* __restrict__ scal, double* __restrict__ part) {
  __shared__ double sm[kThreads / kWave];
  const T alpha = (T)scal[S_ALPHA];
  double acc = 0;
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
    x[i] += alpha * p[i];
    const T ri = r[i] - alpha * q[i];
    r[i] = ri;
    if (r_save) r_save[i] = ri;
    acc += (double)ri * (double)ri;
  }
  const double s = block_sum_double(acc, sm);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// rho' and beta; appends the step's scalars to the history and advances
// the step counter.
__global__ void k_cg_beta(const double* __restrict__ part, int nb, double* __restrict__ scal,
                          double* __restrict__ hist, int* __restrict__ step, int hist_cap) {
  __shared__ double sm[kThreads / kWave];
  const double rho1 = reduce_partials(part, nb, sm);
  if (threadIdx.x == 0) {
    const double rho = scal[S_RHO];
    const double beta = rho != 0.0 ? rho1 / rho : 0.0;
    scal[S_RHO1] = rho1;
    scal[S_BETA] = beta;
    const int t = *step;
    if (hist && t >= 0 && t < hist_cap) {
      double* h = hist + (long long)t * kHistStride;
      h[0] = rho;
      h[1] = scal[S_SIGMA];
      h[2] = scal[S_ALPHA];
      h[3] = rho1;
      h[4] = beta;
    }
    scal[S_RHO] = rho1;
    *step = t + 1;
  }
}

template <typename T>
__global__ void k_cg_p(int n, const T* __restrict__ r, T* __restrict__ p,
                       const double* __restrict__ scal) {
  const T beta = (T)scal[S_BETA];
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads)
    p[i] = r[i] + beta * p[i];
}

// ---------------- reverse ----------------
template <typename T>
__global__ void k_cgb_1(int n, const T* __restrict__ p, const T* __restrict__ gR,
                        T* __restrict__ rb, T* __restrict__ pb, const double* __restrict__ h,
                        double* __restrict__ part) {
  __shared__ double sm[kThreads / kWave];
  const T beta = (T)h[4];
  double acc = 0;
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
    const T pbi = pb[i];
    acc += (double)pbi * (double)p[i];
    rb[i] = rb[i] + (gR ? gR[i] : T(0)) + pbi;
    pb[i] = beta * pbi;
  }
  const double s = block_sum_double(acc, sm);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_cgb_r1(const double* __restrict__ part, int nb, const double* __restrict__ h,
                         double* __restrict__ scal) {
  __shared__ double sm[kThreads / kWave];
  const double betab = reduce_partials(part, nb, sm);
  if (threadIdx.x == 0) {
    const double rho = h[0], rho1 = h[3];
    double rt = 0.0;
    if (rho != 0.0) {
      scal[S_RHOB] += betab / rho;
      rt = -betab * rho1 / (rho * rho);
    }
    scal[S_RHOB_T] = rt;
  }
}

template <typename T>
__global__ void k_cgb_2(int n, const T* __restrict__ p, const T* __restrict__ q,
                        const T* __restrict__ r1, const T* __restrict__ xb, T* __restrict__ rb,
                        T* __restrict__ pb, T* __restrict__ qb, const double* __restrict__ h,
                        const double* __restrict__ scal, double* __restrict__ part) {
  __shared__ double sm[kThreads / kWave];
  const T alpha = (T)h[2];
  const T two_rhob = (T)(2.0 * scal[S_RHOB]);
  double acc = 0;
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
    const T rbi = rb[i] + two_rhob * r1[i];
    rb[i] = rbi;
    const T xbi = xb[i];
    acc += -(double)rbi * (double)q[i] + (double)xbi * (double)p[i];
    qb[i] = -alpha * rbi;
    pb[i] += alpha * xbi;
  }
  const double s = block_sum_double(acc, sm);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_cgb_r2(const double* __restrict__ part, int nb, const double* __restrict__ h,
                         double* __restrict__ scal) {
  __shared__ double sm[kThreads / kWave];
  const double alphab = reduce_partials(part, nb, sm);
  if (threadIdx.x == 0) {
    const double rho = h[0], sigma = h[1];
    double rt = scal[S_RHOB_T], sb = 0.0;
    if (rho != 0.0) {
      rt += alphab / sigma;
      sb = -alphab * rho / (sigma * sigma);
    }
    scal[S_SIGMAB] = sb;
    scal[S_RHOB] = rt;  // becomes the adjoint of rho_t for the step before
  }
}

template <typename T>
__global__ void k_cgb_3(int n, const T* __restrict__ p, T* __restrict__ qb,
                        const double* __restrict__ scal) {
  const T sb = (T)scal[S_SIGMAB];
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads)
    qb[i] += sb * p[i];
}

// pb[j] += sigmab q[j] + sum over column j of A: vals * qb[i];
// gvals[e] += qb[i] p[j] for the entries e = (i, j) of column j.
template <typename T, int G>
__global__ __launch_bounds__(kThreads) void k_cgb_4(int n, const int32_t* __restrict__ rpT,
                                                    const int32_t* __restrict__ ciT,
                                                    const int32_t* __restrict__ perm,
                                                    const T* __restrict__ v,
                                                    const T* __restrict__ p,
                                                    const T* __restrict__ q,
                                                    const T* __restrict__ qb,
                                                    T* __restrict__ pb, T* __restrict__ gv,
                                                    const double* __restrict__ scal) {
  const int j = blockIdx.x * (kThreads / G) + threadIdx.x / G;
  const int sub = threadIdx.x % G;
  T s = 0;
  if (j < n) {
    const T pj = p[j];
    const int t1 = rpT[j + 1];
    for (int t = rpT[j] + sub; t < t1; t += G) {
      const int i = ciT[t];
      const int e = perm[t];
      const T g = qb[i];
      s += v[e] * g;
      gv[e] += g * pj;
    }
  }
  s = group_sum<G>(s);
  if (j < n && sub == 0) pb[j] += (T)scal[S_SIGMAB] * q[j] + s;
}

template <typename T>
__global__ void k_cgb_finish(int n, const T* __restrict__ b, const T* __restrict__ rb,
                             const T* __restrict__ pb, const double* __restrict__ scal,
                             T* __restrict__ gb) {
  const T two_rhob = (T)(2.0 * scal[S_RHOB]);
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads)
    gb[i] = rb[i] + pb[i] + two_rhob * b[i];
}

int lanes_for(long long nnz, int rows) {
  if (rows <= 0) return 1;
  const double mean = (double)nnz / rows;
  int g = 1;
  while (g < 64 && g < mean) g <<= 1;
  return g;
}

#define CSRAD_G_SWITCH(g, ...)                            \
  switch (g) {                                            \
    case 1: { constexpr int G = 1; __VA_ARGS__; } break;   \
    case 2: { constexpr int G = 2; __VA_ARGS__; } break;   \
    case 4: { constexpr int G = 4; __VA_ARGS__; } break;   \
    case 8: { constexpr int G = 8; __VA_ARGS__; } break;   \
    case 16: { constexpr int G = 16; __VA_ARGS__; } break; \
    case 32: { constexpr int G = 32; __VA_ARGS__; } break; \
    default: { constexpr int G = 64; __VA_ARGS__; } break; \
  }

int vec_blocks(int n) {
  int b = (n + kThreads - 1) / kThreads;
  return b < 1 ? 1 : (b > kVecBlocksMax ? kVecBlocksMax : b);
}

int spmv_blocks(int n, int g) {
  const int rpb = kThreads / g;
  const int b = (n + rpb - 1) / rpb;
  return b < 1 ? 1 : (b > kVecBlocksMax ? kVecBlocksMax : b);
}

// Workspace: block partials (float64) sized for the larger of the two grids.
size_t cg_partials(int n, int g) {
  const int a = spmv_blocks(n, g), b = vec_blocks(n);
  return (size_t)(a > b ? a : b);
}

int check_square(const csrad_csr* A) {
  CSRAD_TRY(check_csr(A, true));
  if (A->nrows != A->ncols) return CSRAD_EINVAL;
  return CSRAD_OK;
}

template <typename T>
int cg_step_t(const csrad_csr* A, T* x, T* r, T* p, T* q, T* p_save, T* r_save, double* scal,
              int* step, double* hist, int hist_cap, double* part, hipStream_t s) {
  const int n = A->nrows;
  const T* v = static_cast<const T*>(A->vals);
  const int g = lanes_for(A->nnz, n);
  const int nbs = spmv_blocks(n, g), nbv = vec_blocks(n);
  CSRAD_G_SWITCH(g, hipLaunchKernelGGL((k_cg_spmv_dot<T, G>), dim3(nbs), dim3(kThreads), 0, s, n,
                                       A->rowptr, A->colind, v, p, q, p_save, part));
  hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(kThreads), 0, s, part, nbs, scal);
  hipLaunchKernelGGL((k_cg_update<T>), dim3(nbv), dim3(kThreads), 0, s, n, p, q, x, r, r_save,
                     scal, part);
  hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(kThreads), 0, s, part, nbv, scal, hist, step,
                     hist_cap);
  hipLaunchKernelGGL((k_cg_p<T>), dim3(nbv), dim3(kThreads), 0, s, n, r, p, scal);
  return launch_status();
}

template <typename T>
int cg_step_bwd_t(const csrad_csr* A, const csrad_csr* At, const int32_t* perm, const T* p,
                  const T* q, const T* r1, const double* h, const T* gR, T* xb, T* rb, T* pb,
                  T* qb, double* scal, T* gv, double* part, hipStream_t s) {
  const int n = A->nrows;
  const T* v = static_cast<const T*>(A->vals);
  const int nbv = vec_blocks(n);
  hipLaunchKernelGGL((k_cgb_1<T>), dim3(nbv), dim3(kThreads), 0, s, n, p, gR, rb, pb, h, part);
  hipLaunchKernelGGL(k_cgb_r1, dim3(1), dim3(kThreads), 0, s, part, nbv, h, scal);
  hipLaunchKernelGGL((k_cgb_2<T>), dim3(nbv), dim3(kThreads), 0, s, n, p, q, r1, xb, rb, pb, qb, h,
                     scal, part);
  hipLaunchKernelGGL(k_cgb_r2, dim3(1), dim3(kThreads), 0, s, part, nbv, h, scal);
  hipLaunchKernelGGL((k_cgb_3<T>), dim3(nbv), dim3(kThreads), 0, s, n, p, qb, scal);
  const int g = lanes_for(At->nnz, n);
  // one row group per block (no grid stride here)
  const int rpb = kThreads / g;
  CSRAD_G_SWITCH(g, hipLaunchKernelGGL((k_cgb_4<T, G>), dim3((n + rpb - 1) / rpb), dim3(kThreads),
                                       0, s, n, At->rowptr, At->colind, perm, v, p, q, qb, pb, gv,
                                       scal));
  return launch_status();
}

}  // namespace
}  // namespace csrad

using namespace csrad;

extern "C" int csr_cg_workspace(const csrad_csr* A, size_t* bytes) {
  if (!A || !bytes || A->nrows < 0) return CSRAD_EINVAL;
  const int g = lanes_for(A->nnz, A->nrows);
  *bytes = sizeof(double) * cg_partials(A->nrows, g) + 256;
  return CSRAD_OK;
}

extern "C" int csr_cg_init(const csrad_csr* A, const void* b, void* x, void* r, void* p,
                           double* scal, int32_t* step, void* work, size_t work_bytes,
                           void* stream) {
  CSRAD_TRY(check_square(A));
  const int n = A->nrows;
  if (!scal || !step || (n > 0 && (!b || !x || !r || !p))) return CSRAD_EINVAL;
  size_t need = 0;
  CSRAD_TRY(csr_cg_workspace(A, &need));
  if (!work || work_bytes < need) return CSRAD_EWORKSPACE;
  hipStream_t s = as_stream(stream);
  double* part = static_cast<double*>(work);
  const int nbv = vec_blocks(n);
  if (A->dtype == CSRAD_F32)
    hipLaunchKernelGGL((k_cg_init<float>), dim3(nbv), dim3(kThreads), 0, s, n,
                       static_cast<const float*>(b), static_cast<float*>(x),
                       static_cast<float*>(r), static_cast<float*>(p), part);
  else
    hipLaunchKernelGGL((k_cg_init<double>), dim3(nbv), dim3(kThreads), 0, s, n,
                       static_cast<const double*>(b), static_cast<double*>(x),
                       static_cast<double*>(r), static_cast<double*>(p), part);
  hipLaunchKernelGGL(k_cg_init_scal, dim3(1), dim3(kThreads), 0, s, part, nbv, scal, step);
  return launch_status();
}

extern "C" int csr_cg_step(const csrad_csr* A, void* x, void* r, void* p, void* q,
                           void* p_save, void* r_save, double* scal, int32_t* step, double* hist,
                           int32_t hist_cap, void* work, size_t work_bytes, void* stream) {
  CSRAD_TRY(check_square(A));
  if (A->nrows == 0) return CSRAD_OK;
  if (!x || !r || !p || !q || !scal || !step || hist_cap < 0) return CSRAD_EINVAL;
  size_t need = 0;
  CSRAD_TRY(csr_cg_workspace(A, &need));
  if (!work || work_bytes < need) return CSRAD_EWORKSPACE;
  hipStream_t s = as_stream(stream);
  double* part = static_cast<double*>(work);
  if (A->dtype == CSRAD_F32)
    return cg_step_t<float>(A, static_cast<float*>(x), static_cast<float*>(r),
                            static_cast<float*>(p), static_cast<float*>(q),
                            static_cast<float*>(p_save), static_cast<float*>(r_save), scal, step,
                            hist, hist_cap, part, s);
  return cg_step_t<double>(A, static_cast<double*>(x), static_cast<double*>(r),
                           static_cast<double*>(p), static_cast<double*>(q),
                           static_cast<double*>(p_save), static_cast<double*>(r_save), scal, step,
                           hist, hist_cap, part, s);
}

extern "C" int csr_cg_step_bwd(const csrad_csr* A, const csrad_csr* At, const int32_t* perm,
                               const void* p, const void* q, const void* r1,
                               const double* step_hist, const void* gR, void* xb, void* rb,
                               void* pb, void* qb, double* scal, void* gvals, void* work,
                               size_t work_bytes, void* stream) {
  CSRAD_TRY(check_square(A));
  CSRAD_TRY(check_csr(At, false));
  if (At->nrows != A->ncols || At->ncols != A->nrows || At->nnz != A->nnz) return CSRAD_EINVAL;
  if (A->nrows == 0) return CSRAD_OK;
  if (!p || !q || !r1 || !step_hist || !xb || !rb || !pb || !qb || !scal || !gvals ||
      (A->nnz > 0 && !perm))
    return CSRAD_EINVAL;
  size_t need = 0;
  CSRAD_TRY(csr_cg_workspace(A, &need));
  if (!work || work_bytes < need) return CSRAD_EWORKSPACE;
  hipStream_t s = as_stream(stream);
  double* part = static_cast<double*>(work);
  if (A->dtype == CSRAD_F32)
    return cg_step_bwd_t<float>(A, At, perm, static_cast<const float*>(p),
                                static_cast<const float*>(q), static_cast<const float*>(r1),
                                step_hist, static_cast<const float*>(gR), static_cast<float*>(xb),
                                static_cast<float*>(rb), static_cast<float*>(pb),
                                static_cast<float*>(qb), scal, static_cast<float*>(gvals), part, s);
  return cg_step_bwd_t<double>(A, At, perm, static_cast<const double*>(p),
                               static_cast<const double*>(q), static_cast<const double*>(r1),
                               step_hist, static_cast<const double*>(gR), static_cast<double*>(xb),
                               static_cast<double*>(rb), static_cast<double*>(pb),
                               static_cast<double*>(qb), scal, static_cast<double*>(gvals), part, s);
}

extern "C" int csr_cg_finish_bwd(const csrad_csr* A, const void* b, const void* rb,
                                 const void* pb, const double* scal, void* gb, void* stream) {
  CSRAD_TRY(check_square(A));
  const int n = A->nrows;
  if (n == 0) return CSRAD_OK;
  if (!b || !rb || !pb || !scal || !gb) return CSRAD_EINVAL;
  hipStream_t s = as_stream(stream);
  if (A->dtype == CSRAD_F32)
    hipLaunchKernelGGL((k_cgb_finish<float>), dim3(vec_blocks(n)), dim3(kThreads), 0, s, n,
                       static_cast<const float*>(b), static_cast<const float*>(rb),
                       static_cast<const float*>(pb), scal, static_cast<float*>(gb));
  else
    hipLaunchKernelGGL((k_cgb_finish<double>), dim3(vec_blocks(n)), dim3(kThreads), 0, s, n,
                       static_cast<const double*>(b), static_cast<const double*>(rb),
                       static_cast<const double*>(pb), scal, static_cast<double*>(gb));
  return launch_status();
}
