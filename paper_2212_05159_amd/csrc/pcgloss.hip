// The vector and scalar steps of a short PCG unroll and their reverse mode,
// for training a preconditioner on the residual-history loss of Section 4.3:
//   l = sum_{i=1..Nit} w_i ||r_i|| / ||b||.
// One PCG iteration from (r, p, rho = r.z) is
//   q = A p                                   (csr_spmv_fwd: not here)
//   sigma = p.q,  alpha = rho / sigma,  r' = r - alpha q,  nr = ||r'||,
//   acc' = acc + w_i nr / ||b||                                        [res]
//   z' = M^{-1} r'                             (the preconditioner: not here)
//   rho' = r'.z',  beta = rho' / rho,  p' = z' + beta p              [dir]
// and the start rho_0 = b.z_0 with z_0 = M^{-1} b, p_0 = z_0          [start].
// Vectors are float32 or float64, every dot product and scalar float64,
// summed in a fixed order (block partials, then one block), so each call
// is bit-reproducible.  The reverse steps take the upstream adjoints of the
// outputs and write those of the inputs (b is data, not differentiated):
//   res: from (gr', gacc'):  k = gacc' w_i / (||b|| nr),  g = gr' + k r';
//        abar = -q.g;  gr = g;  grho = abar / sigma;
//        sbar = -abar rho / sigma^2;  gq = -alpha g + sbar p;  gp = sbar q
//        (gacc = gacc', left to the caller);
//   dir: from (gp', grho'):  bbar = p.gp';  t = grho' + bbar / rho;
//        gz' = gp' + t r';  gr' = t z';  gp = beta gp';
//        grho = -bbar rho' / rho^2;
//   start: from (grho_0, gp_0):  gz_0 = grho_0 b + gp_0.
#include "internal.hpp"

namespace csrad {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxBlocks = 1024;

int blocks_for(int n) {
  int b = (n + kThreads - 1) / kThreads;
  return b < 1 ? 1 : (b > kMaxBlocks ? kMaxBlocks : b);
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = group_sum<kWave>(v);
  const int w = threadIdx.x / kWave;
  if (threadIdx.x % kWave == 0) sh[w] = v;
  __syncthreads();
  double s = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kThreads / kWave; ++i) s += sh[i];
  __syncthreads();
  return s;  // valid in thread 0
}

// Partial sums of up to two dot products per block: part[b] = a.b over the
// block's grid-stride share, part[nb + b] = c.d (when c is non-null).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_dots(int n, const T* __restrict__ a,
                                                   const T* __restrict__ b,
                                                   const T* __restrict__ c,
                                                   const T* __restrict__ d,
                                                   double* __restrict__ part) {
  __shared__ double sh[kThreads / kWave];
  double s1 = 0, s2 = 0;
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
    s1 += (double)a[i] * (double)b[i];
    if (c) s2 += (double)c[i] * (double)d[i];
  }
  s1 = block_sum(s1, sh);
  if (c) s2 = block_sum(s2, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s1;
    if (c) part[gridDim.x + blockIdx.x] = s2;
  }
}

__device__ __forceinline__ double sum_parts(const double* part, int nb) {
  double s = 0;
  for (int i = 0; i < nb; ++i) s += part[i];
  return s;
}

// start: scal[0] = rho_0 = b.z, scal[1] = ||b||.
__global__ void k_start_scal(const double* __restrict__ part, int nb, double* __restrict__ scal) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    scal[0] = sum_parts(part, nb);
    scal[1] = sqrt(sum_parts(part + nb, nb));
  }
}

// res forward, after the p.q partials: r' = r - alpha q (every block sums
// the partials itself in the same order), then the r'.r' partials.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_res_update(int n, const T* __restrict__ q,
                                                         const T* __restrict__ r,
                                                         const double* __restrict__ rho,
                                                         const double* __restrict__ part, int nb,
                                                         T* __restrict__ r1,
                                                         double* __restrict__ part2) {
  __shared__ double sh[kThreads / kWave];
  __shared__ double s_alpha;
  if (threadIdx.x == 0) {
    const double sigma = sum_parts(part, nb);
    s_alpha = rho[0] / sigma;
  }
  __syncthreads();
  const double alpha = s_alpha;
  double s = 0;
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
    const T v = (T)((double)r[i] - alpha * (double)q[i]);
    r1[i] = v;
    s += (double)v * (double)v;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part2[blockIdx.x] = s;
}

// scal (3 doubles): [0] sigma, [1] alpha, [2] nr; acc' = acc + w nr / ||b||.
__global__ void k_res_scal(const double* __restrict__ part, const double* __restrict__ part2,
                           int nb, const double* __restrict__ rho, double w,
                           const double* __restrict__ bnorm, const double* __restrict__ acc,
                           double* __restrict__ scal, double* __restrict__ acc1) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const double sigma = sum_parts(part, nb);
    const double nr = sqrt(sum_parts(part2, nb));
    scal[0] = sigma;
    scal[1] = rho[0] / sigma;
    scal[2] = nr;
    acc1[0] = acc[0] + w * nr / bnorm[0];
  }
}

// dir forward: rho' = r'.z' (partials done), beta = rho'/rho, p' = z' + beta p.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_dir_update(int n, const T* __restrict__ z,
                                                         const T* __restrict__ p,
                                                         const double* __restrict__ rho,
                                                         const double* __restrict__ part, int nb,
                                                         T* __restrict__ p1,
                                                         double* __restrict__ rho1) {
  __shared__ double s_beta;
  if (threadIdx.x == 0) {
    const double r1 = sum_parts(part, nb);
    s_beta = r1 / rho[0];
    if (blockIdx.x == 0) rho1[0] = r1;
  }
  __syncthreads();
  const double beta = s_beta;
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads)
    p1[i] = (T)((double)z[i] + beta * (double)p[i]);
}

// res reverse.  g = gr1 + k r1 with k = gacc1 w / (||b|| nr); abar = -q.g
// (partials of q.gr1 and q.r1 taken together); then the vectors.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_res_bwd_vec(
    int n, const T* __restrict__ p, const T* __restrict__ q, const T* __restrict__ r1,
    const T* __restrict__ gr1, const double* __restrict__ rho, const double* __restrict__ scal,
    const double* __restrict__ gacc1, double w, const double* __restrict__ bnorm,
    const double* __restrict__ part, int nb, T* __restrict__ gr, T* __restrict__ gq,
    T* __restrict__ gp, double* __restrict__ grho) {
  __shared__ double s_k, s_sbar, s_alpha;
  if (threadIdx.x == 0) {
    const double sigma = scal[0], alpha = scal[1], nr = scal[2];
    const double k = nr > 0 ? gacc1[0] * w / (bnorm[0] * nr) : 0.0;
    const double qg = sum_parts(part, nb) + k * sum_parts(part + nb, nb);
    const double abar = -qg;
    const double sbar = -abar * rho[0] / (sigma * sigma);
    s_k = k;
    s_sbar = sbar;
    s_alpha = alpha;
    if (blockIdx.x == 0) grho[0] = abar / sigma;
  }
  __syncthreads();
  const double k = s_k, sbar = s_sbar, alpha = s_alpha;
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
    const double g = (gr1 ? (double)gr1[i] : 0.0) + k * (double)r1[i];
    gr[i] = (T)g;
    gq[i] = (T)(-alpha * g + sbar * (double)p[i]);
    gp[i] = (T)(sbar * (double)q[i]);
  }
}

// dir reverse.  bbar = p.gp1 (partials done); beta = rho1/rho;
// grho1_tot = grho1 + bbar/rho;  gz1 = gp1 + grho1_tot r1;  gr1 = grho1_tot z1;
// gp = beta gp1;  grho = -bbar rho1 / rho^2.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_dir_bwd_vec(
    int n, const T* __restrict__ r1, const T* __restrict__ z1, const T* __restrict__ gp1,
    const double* __restrict__ rho, const double* __restrict__ rho1,
    const double* __restrict__ grho1, const double* __restrict__ part, int nb,
    T* __restrict__ gr1, T* __restrict__ gz1, T* __restrict__ gp, double* __restrict__ grho) {
  __shared__ double s_t, s_beta;
  if (threadIdx.x == 0) {
    const double bbar = sum_parts(part, nb);
    s_t = (grho1 ? grho1[0] : 0.0) + bbar / rho[0];
    s_beta = rho1[0] / rho[0];
    if (blockIdx.x == 0) grho[0] = -bbar * rho1[0] / (rho[0] * rho[0]);
  }
  __syncthreads();
  const double t = s_t, beta = s_beta;
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
    const double g = gp1 ? (double)gp1[i] : 0.0;
    gz1[i] = (T)(g + t * (double)r1[i]);
    gr1[i] = (T)(t * (double)z1[i]);
    gp[i] = (T)(beta * g);
  }
}

// start reverse: rho_0 = b.z_0 (b constant): gz_0 = grho_0 b + gp_0.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_start_bwd(int n, const T* __restrict__ b,
                                                        const T* __restrict__ gp0,
                                                        const double* __restrict__ grho0,
                                                        T* __restrict__ gz0) {
  const double g = grho0 ? grho0[0] : 0.0;
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads)
    gz0[i] = (T)(g * (double)b[i] + (gp0 ? (double)gp0[i] : 0.0));
}

int ws_check(int n, int dtype, void* work, size_t bytes) {
  if (dtype != CSRAD_F32 && dtype != CSRAD_F64) return CSRAD_EDTYPE;
  if (!work || bytes < sizeof(double) * 2 * (size_t)blocks_for(n)) return CSRAD_EWORKSPACE;
  return CSRAD_OK;
}

template <typename T>
void start_t(int n, const void* b, const void* z, double* scal, double* part, hipStream_t s) {
  const int nb = blocks_for(n);
  const T* bb = static_cast<const T*>(b);
  hipLaunchKernelGGL((k_dots<T>), dim3(nb), dim3(kThreads), 0, s, n, bb, static_cast<const T*>(z),
                     bb, bb, part);
  hipLaunchKernelGGL(k_start_scal, dim3(1), dim3(64), 0, s, part, nb, scal);
}

template <typename T>
void res_fwd_t(int n, const void* p, const void* q, const void* r, const double* rho, double w,
               const double* bnorm, const double* acc, void* r1, double* scal, double* acc1,
               double* part, hipStream_t s) {
  const int nb = blocks_for(n);
  const T* qq = static_cast<const T*>(q);
  hipLaunchKernelGGL((k_dots<T>), dim3(nb), dim3(kThreads), 0, s, n, static_cast<const T*>(p), qq,
                     nullptr, nullptr, part);
  hipLaunchKernelGGL((k_res_update<T>), dim3(nb), dim3(kThreads), 0, s, n, qq,
                     static_cast<const T*>(r), rho, part, nb, static_cast<T*>(r1), part + nb);
  hipLaunchKernelGGL(k_res_scal, dim3(1), dim3(64), 0, s, part, part + nb, nb, rho, w, bnorm, acc,
                     scal, acc1);
}

template <typename T>
int res_bwd_t(int n, const void* p, const void* q, const void* r1, const double* rho,
              const double* scal, double w, const double* bnorm, const void* gr1,
              const double* gacc1, void* gr, void* gq, void* gp, double* grho, double* part,
              hipStream_t s) {
  const int nb = blocks_for(n);
  const T* qq = static_cast<const T*>(q);
  const T* rr = static_cast<const T*>(r1);
  const T* gg = static_cast<const T*>(gr1);
  if (gg) {
    hipLaunchKernelGGL((k_dots<T>), dim3(nb), dim3(kThreads), 0, s, n, qq, gg, qq, rr, part);
  } else {
    CSRAD_TRY(fill_bytes_zero(part, sizeof(double) * nb, s));
    hipLaunchKernelGGL((k_dots<T>), dim3(nb), dim3(kThreads), 0, s, n, qq, rr, nullptr, nullptr,
                       part + nb);
  }
  hipLaunchKernelGGL((k_res_bwd_vec<T>), dim3(nb), dim3(kThreads), 0, s, n,
                     static_cast<const T*>(p), qq, rr, gg, rho, scal, gacc1, w, bnorm, part, nb,
                     static_cast<T*>(gr), static_cast<T*>(gq), static_cast<T*>(gp), grho);
  return CSRAD_OK;
}

template <typename T>
void dir_fwd_t(int n, const void* r1, const void* z1, const double* rho, const void* p,
               double* rho1, void* p1, double* part, hipStream_t s) {
  const int nb = blocks_for(n);
  const T* zz = static_cast<const T*>(z1);
  hipLaunchKernelGGL((k_dots<T>), dim3(nb), dim3(kThreads), 0, s, n, static_cast<const T*>(r1), zz,
                     nullptr, nullptr, part);
  hipLaunchKernelGGL((k_dir_update<T>), dim3(nb), dim3(kThreads), 0, s, n, zz,
                     static_cast<const T*>(p), rho, part, nb, static_cast<T*>(p1), rho1);
}

template <typename T>
int dir_bwd_t(int n, const void* r1, const void* z1, const double* rho, const void* p,
              const double* rho1, const void* gp1, const double* grho1, void* gr1, void* gz1,
              void* gp, double* grho, double* part, hipStream_t s) {
  const int nb = blocks_for(n);
  const T* gg = static_cast<const T*>(gp1);
  if (gg)
    hipLaunchKernelGGL((k_dots<T>), dim3(nb), dim3(kThreads), 0, s, n, static_cast<const T*>(p),
                       gg, nullptr, nullptr, part);
  else
    CSRAD_TRY(fill_bytes_zero(part, sizeof(double) * nb, s));
  hipLaunchKernelGGL((k_dir_bwd_vec<T>), dim3(nb), dim3(kThreads), 0, s, n,
                     static_cast<const T*>(r1), static_cast<const T*>(z1), gg, rho, rho1, grho1,
                     part, nb, static_cast<T*>(gr1), static_cast<T*>(gz1), static_cast<T*>(gp),
                     grho);
  return CSRAD_OK;
}

}  // namespace
}  // namespace csrad

using namespace csrad;

extern "C" int csr_pcgl_workspace(int32_t n, size_t* bytes) {
  if (!bytes || n < 0) return CSRAD_EINVAL;
  *bytes = sizeof(double) * 2 * (size_t)blocks_for(n);
  return CSRAD_OK;
}

extern "C" int csr_pcgl_start(int32_t n, int32_t dtype, const void* b, const void* z,
                              double* scal, void* work, size_t work_bytes, void* stream) {
  if (n <= 0 || !b || !z || !scal) return CSRAD_EINVAL;
  CSRAD_TRY(ws_check(n, dtype, work, work_bytes));
  double* part = static_cast<double*>(work);
  if (dtype == CSRAD_F32) start_t<float>(n, b, z, scal, part, as_stream(stream));
  else start_t<double>(n, b, z, scal, part, as_stream(stream));
  return launch_status();
}

extern "C" int csr_pcgl_res_fwd(int32_t n, int32_t dtype, const void* p, const void* q,
                                const void* r, const double* rho, double w,
                                const double* bnorm, const double* acc, void* r1, double* scal,
                                double* acc1, void* work, size_t work_bytes, void* stream) {
  if (n <= 0 || !p || !q || !r || !rho || !bnorm || !acc || !r1 || !scal || !acc1)
    return CSRAD_EINVAL;
  CSRAD_TRY(ws_check(n, dtype, work, work_bytes));
  double* part = static_cast<double*>(work);
  if (dtype == CSRAD_F32)
    res_fwd_t<float>(n, p, q, r, rho, w, bnorm, acc, r1, scal, acc1, part, as_stream(stream));
  else
    res_fwd_t<double>(n, p, q, r, rho, w, bnorm, acc, r1, scal, acc1, part, as_stream(stream));
  return launch_status();
}

extern "C" int csr_pcgl_res_bwd(int32_t n, int32_t dtype, const void* p, const void* q,
                                const void* r1, const double* rho, const double* scal, double w,
                                const double* bnorm, const void* gr1, const double* gacc1,
                                void* gr, void* gq, void* gp, double* grho, void* work,
                                size_t work_bytes, void* stream) {
  if (n <= 0 || !p || !q || !r1 || !rho || !scal || !bnorm || !gacc1 || !gr || !gq || !gp ||
      !grho)
    return CSRAD_EINVAL;
  CSRAD_TRY(ws_check(n, dtype, work, work_bytes));
  double* part = static_cast<double*>(work);
  hipStream_t s = as_stream(stream);
  if (dtype == CSRAD_F32)
    CSRAD_TRY(res_bwd_t<float>(n, p, q, r1, rho, scal, w, bnorm, gr1, gacc1, gr, gq, gp, grho,
                               part, s));
  else
    CSRAD_TRY(res_bwd_t<double>(n, p, q, r1, rho, scal, w, bnorm, gr1, gacc1, gr, gq, gp, grho,
                                part, s));
  return launch_status();
}

extern "C" int csr_pcgl_dir_fwd(int32_t n, int32_t dtype, const void* r1, const void* z1,
                                const double* rho, const void* p, double* rho1, void* p1,
                                void* work, size_t work_bytes, void* stream) {
  if (n <= 0 || !r1 || !z1 || !rho || !p || !rho1 || !p1) return CSRAD_EINVAL;
  CSRAD_TRY(ws_check(n, dtype, work, work_bytes));
  double* part = static_cast<double*>(work);
  if (dtype == CSRAD_F32) dir_fwd_t<float>(n, r1, z1, rho, p, rho1, p1, part, as_stream(stream));
  else dir_fwd_t<double>(n, r1, z1, rho, p, rho1, p1, part, as_stream(stream));
  return launch_status();
}

extern "C" int csr_pcgl_dir_bwd(int32_t n, int32_t dtype, const void* r1, const void* z1,
                                const double* rho, const void* p, const double* rho1,
                                const void* gp1, const double* grho1, void* gr1, void* gz1,
                                void* gp, double* grho, void* work, size_t work_bytes,
                                void* stream) {
  if (n <= 0 || !r1 || !z1 || !rho || !p || !rho1 || !gr1 || !gz1 || !gp || !grho)
    return CSRAD_EINVAL;
  CSRAD_TRY(ws_check(n, dtype, work, work_bytes));
  double* part = static_cast<double*>(work);
  hipStream_t s = as_stream(stream);
  if (dtype == CSRAD_F32)
    CSRAD_TRY(dir_bwd_t<float>(n, r1, z1, rho, p, rho1, gp1, grho1, gr1, gz1, gp, grho, part, s));
  else
    CSRAD_TRY(dir_bwd_t<double>(n, r1, z1, rho, p, rho1, gp1, grho1, gr1, gz1, gp, grho, part, s));
  return launch_status();
}

extern "C" int csr_pcgl_start_bwd(int32_t n, int32_t dtype, const void* b, const void* gp0,
                                  const double* grho0, void* gz0, void* stream) {
  if (n <= 0 || !b || !gz0) return CSRAD_EINVAL;
  if (dtype != CSRAD_F32 && dtype != CSRAD_F64) return CSRAD_EDTYPE;
  const dim3 g(blocks_for(n));
  if (dtype == CSRAD_F32)
    hipLaunchKernelGGL((k_start_bwd<float>), g, dim3(kThreads), 0, as_stream(stream), n,
                       static_cast<const float*>(b), static_cast<const float*>(gp0), grho0,
                       static_cast<float*>(gz0));
  else
    hipLaunchKernelGGL((k_start_bwd<double>), g, dim3(kThreads), 0, as_stream(stream), n,
                       static_cast<const double*>(b), static_cast<const double*>(gp0), grho0,
                       static_cast<double*>(gz0));
  return launch_status();
}
