// Preconditioned conjugate gradients (Section 4.3) with float64 vectors
// and dot products over float32 or float64 matrix values.  The state lives
// on the device; a step is a fixed sequence of launches and needs no host
// synchronisation.  Once the relative residual ||r||/||b|| reaches the
// tolerance, or a breakdown is detected (p.q not positive and finite, or
// r.z not finite), every later step is a no-op, so the host may run steps
// in chunks and read the state between chunks.
//
// Preconditioners M^{-1}:
//   Jacobi:  z = r / diag(A)
//   factor:  z = L^{-T} (L^{-1} r), L lower triangular with a stored
//            diagonal (M = L L^T), solved level by level.
//   none:    z = r
#include "internal.hpp"

namespace csrad {
namespace {

constexpr int kThreads = 256;
constexpr int kVecBlocksMax = 2048;   // grid of the vector kernels
constexpr int kSpmvBlocksMax = 2048;  // grid of the product kernel

enum : int {
  P_RHO = 0,     // r.z
  P_SIGMA,       // p.q
  P_ALPHA,
  P_BETA,
  P_BNORM,       // ||b||
  P_RES,         // ||r|| / ||b||
  P_DONE,        // 1: converged or broken down
  P_BREAKDOWN,   // 1: breakdown
  P_ITERS,       // steps taken
  P_TOL,
  P_RR,          // r.r
  P_COUNT = 16
};

// Partial sums in the workspace: p.q per product block, r.z and r.r per
// vector block.  Every sum has a fixed partition and a fixed order, so a
// step is deterministic.
struct Parts {
  double* pq;  // kSpmvBlocksMax
  double* rz;  // kVecBlocksMax
  double* rr;  // kVecBlocksMax
};

__device__ double block_sum(double v, double* sm) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if (threadIdx.x % kWave == 0) sm[threadIdx.x / kWave] = v;
  __syncthreads();
  double t = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kThreads / kWave; ++i) t += sm[i];
  __syncthreads();
  return t;
}

__device__ double reduce_parts(const double* __restrict__ part, int nb, double* sm) {
  double v = 0;
  for (int i = threadIdx.x; i < nb; i += kThreads) v += part[i];
  return block_sum(v, sm);
}

int vec_blocks(int n) {
  int b = (n + kThreads - 1) / kThreads;
  return b < 1 ? 1 : (b > kVecBlocksMax ? kVecBlocksMax : b);
}

int lanes_for(long long nnz, int rows) {
  if (rows <= 0) return 1;
  const double mean = (double)nnz / rows;
  int g = 1;
  while (g < 64 && g < mean) g <<= 1;
  return g;
}

int spmv_blocks(int n, int g) {
  const int rpb = kThreads / g;
  int b = (n + rpb - 1) / rpb;
  return b < 1 ? 1 : (b > kSpmvBlocksMax ? kSpmvBlocksMax : b);
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

// 1 / diag(A) (0 where the diagonal is missing or zero).
template <typename TV>
__global__ void k_diag_inv(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                           const TV* __restrict__ v, double* __restrict__ dinv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double d = 0;
  for (int e = rp[i]; e < rp[i + 1]; ++e)
    if (ci[e] == i) d = (double)v[e];
  dinv[i] = d != 0.0 ? 1.0 / d : 0.0;
}

__global__ void k_pcg_init(int n, const double* __restrict__ b, double* __restrict__ x,
                           double* __restrict__ r, double* __restrict__ part) {
  __shared__ double sm[kThreads / kWave];
  double acc = 0;
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
    const double bi = b[i];
    x[i] = 0.0;
    r[i] = bi;
    acc += bi * bi;
  }
  const double s = block_sum(acc, sm);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_pcg_init_scal(const double* __restrict__ part, int nb, double tol,
                                double* __restrict__ scal) {
  __shared__ double sm[kThreads / kWave];
  const double bb = reduce_parts(part, nb, sm);
  if (threadIdx.x == 0) {
    for (int i = 0; i < P_COUNT; ++i) scal[i] = 0.0;
    scal[P_BNORM] = sqrt(bb);
    scal[P_TOL] = tol;
    scal[P_RES] = bb > 0 ? 1.0 : 0.0;
    scal[P_DONE] = bb > 0 ? 0.0 : 1.0;
  }
}

// z = M^{-1} r for the diagonal preconditioners (KIND 0 Jacobi, 2 none)
// with the r.z and r.r partials; KIND 1 (factor) only takes r.z, z having
// come from the solves.
template <int KIND>
__global__ void k_pcg_precond_dots(int n, const double* __restrict__ dinv,
                                   const double* __restrict__ r, double* __restrict__ z,
                                   Parts parts, const double* __restrict__ scal) {
  __shared__ double sm[kThreads / kWave];
  if (scal[P_DONE] != 0.0) return;
  double rz = 0, rr = 0;
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
    const double ri = r[i];
    double zi;
    if (KIND == 0) {
      zi = ri * dinv[i];
      z[i] = zi;
    } else if (KIND == 2) {
      zi = ri;
      z[i] = zi;
    } else {
      zi = z[i];
    }
    rz += ri * zi;
    rr += ri * ri;
  }
  rz = block_sum(rz, sm);
  rr = block_sum(rr, sm);
  if (threadIdx.x == 0) {
    parts.rz[blockIdx.x] = rz;
    parts.rr[blockIdx.x] = rr;
  }
}

// First rho and p = z.
__global__ void k_pcg_start(int n, Parts parts, int nb, const double* __restrict__ z,
                            double* __restrict__ p, double* __restrict__ scal) {
  __shared__ double sm[kThreads / kWave];
  __shared__ double rho_s;
  if (scal[P_DONE] != 0.0) return;
  const double a = reduce_parts(parts.rz, nb, sm);
  if (threadIdx.x == 0) rho_s = a;
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    scal[P_RHO] = rho_s;
    if (!isfinite(rho_s)) {
      scal[P_BREAKDOWN] = 1.0;
      scal[P_DONE] = 1.0;
    }
  }
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) p[i] = z[i];
}

// q = A p and the p.q partial of this block; G lanes per row, the block
// strides over row groups so that the grid stays at most kSpmvBlocksMax.
template <typename TV, int G>
__global__ __launch_bounds__(kThreads) void k_pcg_spmv_dot(int n, const int32_t* __restrict__ rp,
                                                           const int32_t* __restrict__ ci,
                                                           const TV* __restrict__ v,
                                                           const double* __restrict__ p,
                                                           double* __restrict__ q,
                                                           double* __restrict__ part,
                                                           const double* __restrict__ scal) {
  __shared__ double sm[kThreads / kWave];
  if (scal[P_DONE] != 0.0) return;
  constexpr int RPB = kThreads / G;
  const int sub = threadIdx.x % G;
  double d = 0;
  for (int base = blockIdx.x * RPB; base < n; base += gridDim.x * RPB) {
    const int row = base + threadIdx.x / G;
    double s = 0;
    if (row < n) {
      const int e1 = rp[row + 1];
      for (int e = rp[row] + sub; e < e1; e += G) s += (double)v[e] * p[ci[e]];
    }
    s = group_sum<G>(s);
    if (row < n && sub == 0) {
      q[row] = s;
      d += p[row] * s;
    }
  }
  d = block_sum(d, sm);
  if (threadIdx.x == 0) part[blockIdx.x] = d;
}

__global__ void k_pcg_alpha(const double* __restrict__ part, int nb, double* __restrict__ scal) {
  __shared__ double sm[kThreads / kWave];
  if (scal[P_DONE] != 0.0) return;
  const double sigma = reduce_parts(part, nb, sm);
  if (threadIdx.x == 0) {
    scal[P_SIGMA] = sigma;
    if (!(sigma > 0.0) || !isfinite(sigma)) {
      scal[P_ALPHA] = 0.0;
      scal[P_BREAKDOWN] = 1.0;
      scal[P_DONE] = 1.0;
    } else {
      scal[P_ALPHA] = scal[P_RHO] / sigma;
    }
  }
}

// x += alpha p, r -= alpha q, fused with the diagonal preconditioners and
// both dots (KIND 0 Jacobi, 2 none); KIND 1 (factor) only updates x and r.
template <int KIND>
__global__ void k_pcg_update(int n, const double* __restrict__ p, const double* __restrict__ q,
                             double* __restrict__ x, double* __restrict__ r,
                             const double* __restrict__ dinv, double* __restrict__ z, Parts parts,
                             const double* __restrict__ scal) {
  __shared__ double sm[kThreads / kWave];
  if (scal[P_DONE] != 0.0) return;
  const double alpha = scal[P_ALPHA];
  double rz = 0, rr = 0;
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    if (KIND != 1) {
      const double zi = KIND == 0 ? ri * dinv[i] : ri;
      z[i] = zi;
      rz += ri * zi;
      rr += ri * ri;
    }
  }
  if (KIND != 1) {
    rz = block_sum(rz, sm);
    rr = block_sum(rr, sm);
    if (threadIdx.x == 0) {
      parts.rz[blockIdx.x] = rz;
      parts.rr[blockIdx.x] = rr;
    }
  }
}

// rho' = r.z, beta, residual and convergence; counts the step.
__global__ void k_pcg_beta(Parts parts, int nb, double* __restrict__ scal,
                           double* __restrict__ hist, int hist_cap) {
  __shared__ double sm[kThreads / kWave];
  if (scal[P_DONE] != 0.0) return;
  const double a = reduce_parts(parts.rz, nb, sm);
  const double c = reduce_parts(parts.rr, nb, sm);
  if (threadIdx.x == 0) {
    const double rho = scal[P_RHO];
    const double res = sqrt(c) / scal[P_BNORM];
    const int it = (int)scal[P_ITERS];
    scal[P_ITERS] = it + 1;
    scal[P_RES] = res;
    scal[P_RR] = c;
    if (hist && it < hist_cap) hist[it] = res;
    if (!isfinite(a) || !isfinite(res)) {
      scal[P_BREAKDOWN] = 1.0;
      scal[P_DONE] = 1.0;
      scal[P_BETA] = 0.0;
    } else {
      scal[P_BETA] = rho != 0.0 ? a / rho : 0.0;
      scal[P_RHO] = a;
      if (res <= scal[P_TOL]) scal[P_DONE] = 1.0;
    }
  }
}

// p = z + beta p, unless the state became final in this step.
__global__ void k_pcg_p(int n, const double* __restrict__ z, double* __restrict__ p,
                        const double* __restrict__ scal) {
  if (scal[P_DONE] != 0.0) return;
  const double beta = scal[P_BETA];
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads)
    p[i] = z[i] + beta * p[i];
}

struct Precond {
  int kind;  // 0 Jacobi, 1 factor, 2 none
  const double* dinv;
  const csrad_csr* L;
  const csrad_csr* Lt;
  const int32_t* perm;
  int nlevels;
  const int32_t* lp_host;
  const int32_t* lp_dev;
  const int32_t* rows;
};

// z = M^{-1} r followed by the r.z and r.r partials.  The factor solves
// are not conditional on the done flag, so their cost is paid until the
// host stops stepping.
int precond_dots(int n, const Precond& pc, const double* r, double* z, double* y, Parts parts,
                 const double* scal, hipStream_t s) {
  const int nbv = vec_blocks(n);
  if (pc.kind == 0) {
    hipLaunchKernelGGL(k_pcg_precond_dots<0>, dim3(nbv), dim3(kThreads), 0, s, n, pc.dinv, r, z,
                       parts, scal);
  } else if (pc.kind == 1) {
    CSRAD_TRY(trisolve_vec64(pc.L, 1, pc.Lt, pc.perm, false, pc.nlevels, pc.lp_host, pc.lp_dev,
                             pc.rows, r, y, s));
    CSRAD_TRY(trisolve_vec64(pc.L, 1, pc.Lt, pc.perm, true, pc.nlevels, pc.lp_host, pc.lp_dev,
                             pc.rows, y, z, s));
    hipLaunchKernelGGL(k_pcg_precond_dots<1>, dim3(nbv), dim3(kThreads), 0, s, n, pc.dinv, r, z,
                       parts, scal);
  } else {
    hipLaunchKernelGGL(k_pcg_precond_dots<2>, dim3(nbv), dim3(kThreads), 0, s, n, pc.dinv, r, z,
                       parts, scal);
  }
  return launch_status();
}

int check_pc(const csrad_csr* A, int kind, const double* dinv, const csrad_csr* L,
             const csrad_csr* Lt, const int32_t* perm, int nlevels, const int32_t* lp_host,
             const int32_t* lp_dev, const int32_t* rows) {
  if (kind == 0) return dinv ? CSRAD_OK : CSRAD_EINVAL;
  if (kind == 2) return CSRAD_OK;
  if (kind != 1 || !L || !Lt) return CSRAD_EINVAL;
  CSRAD_TRY(check_csr(L, true));
  CSRAD_TRY(check_csr(Lt, false));
  if (L->nrows != A->nrows || L->ncols != A->nrows || Lt->nrows != A->nrows ||
      Lt->nnz != L->nnz)
    return CSRAD_EINVAL;
  if ((L->nnz > 0 && !perm && !Lt->vals) || nlevels < 1 || !lp_host || !lp_dev || !rows)
    return CSRAD_EINVAL;
  if (Lt->vals && Lt->dtype != L->dtype) return CSRAD_EDTYPE;
  if (lp_host[0] != 0 || lp_host[nlevels] != A->nrows) return CSRAD_EINVAL;
  return CSRAD_OK;
}

constexpr size_t kPartsDoubles = kSpmvBlocksMax + 2 * kVecBlocksMax;

Parts carve_parts(void* work) {
  double* w = static_cast<double*>(work);
  return Parts{w, w + kSpmvBlocksMax, w + kSpmvBlocksMax + kVecBlocksMax};
}

}  // namespace
}  // namespace csrad

using namespace csrad;

extern "C" int csr_pcg_workspace(const csrad_csr* A, size_t* bytes) {
  if (!A || !bytes || A->nrows < 0) return CSRAD_EINVAL;
  const int n = A->nrows;
  // partials + the intermediate vector of the factor solves
  *bytes = align_up(sizeof(double) * kPartsDoubles, 256) +
           sizeof(double) * (size_t)(n > 0 ? n : 1) + 256;
  return CSRAD_OK;
}

extern "C" int csr_diag_inv(const csrad_csr* A, double* dinv, void* stream) {
  CSRAD_TRY(check_csr(A, true));
  if (A->nrows != A->ncols) return CSRAD_EINVAL;
  if (A->nrows == 0) return CSRAD_OK;
  if (!dinv) return CSRAD_EINVAL;
  hipStream_t s = as_stream(stream);
  const unsigned g = (unsigned)((A->nrows + 255) / 256);
  if (A->dtype == CSRAD_F32)
    hipLaunchKernelGGL((k_diag_inv<float>), dim3(g), dim3(256), 0, s, A->nrows, A->rowptr,
                       A->colind, static_cast<const float*>(A->vals), dinv);
  else
    hipLaunchKernelGGL((k_diag_inv<double>), dim3(g), dim3(256), 0, s, A->nrows, A->rowptr,
                       A->colind, static_cast<const double*>(A->vals), dinv);
  return launch_status();
}

static int pcg_common(const csrad_csr* A, int kind, const double* dinv, const csrad_csr* L,
                      const csrad_csr* Lt, const int32_t* perm, int nlevels,
                      const int32_t* lp_host, const int32_t* lp_dev, const int32_t* rows,
                      void* work, size_t work_bytes, Precond* pc, Parts* parts, double** y) {
  CSRAD_TRY(check_csr(A, true));
  if (A->nrows != A->ncols) return CSRAD_EINVAL;
  CSRAD_TRY(check_pc(A, kind, dinv, L, Lt, perm, nlevels, lp_host, lp_dev, rows));
  size_t need = 0;
  CSRAD_TRY(csr_pcg_workspace(A, &need));
  if (!work || work_bytes < need) return CSRAD_EWORKSPACE;
  const int n = A->nrows;
  *parts = carve_parts(work);
  *y = reinterpret_cast<double*>(static_cast<char*>(work) +
                                 align_up(sizeof(double) * kPartsDoubles, 256));
  *pc = Precond{kind, dinv, L, Lt, perm, nlevels, lp_host, lp_dev, rows};
  return CSRAD_OK;
}

extern "C" int csr_pcg_init(const csrad_csr* A, int32_t kind, const double* dinv,
                            const csrad_csr* L, const csrad_csr* Lt, const int32_t* perm,
                            int32_t nlevels, const int32_t* lp_host, const int32_t* lp_dev,
                            const int32_t* rows, const double* b, double* x, double* r,
                            double* z, double* p, double tol, double* scal, void* work,
                            size_t work_bytes, void* stream) {
  Precond pc;
  Parts parts;
  double* y;
  CSRAD_TRY(pcg_common(A, kind, dinv, L, Lt, perm, nlevels, lp_host, lp_dev, rows, work,
                       work_bytes, &pc, &parts, &y));
  const int n = A->nrows;
  if (!scal || (n > 0 && (!b || !x || !r || !z || !p))) return CSRAD_EINVAL;
  hipStream_t s = as_stream(stream);
  const int nbv = vec_blocks(n);
  hipLaunchKernelGGL(k_pcg_init, dim3(nbv), dim3(kThreads), 0, s, n, b, x, r, parts.rr);
  hipLaunchKernelGGL(k_pcg_init_scal, dim3(1), dim3(kThreads), 0, s, parts.rr, nbv, tol, scal);
  if (n == 0) return launch_status();
  CSRAD_TRY(precond_dots(n, pc, r, z, y, parts, scal, s));
  hipLaunchKernelGGL(k_pcg_start, dim3(nbv), dim3(kThreads), 0, s, n, parts, nbv, z, p, scal);
  return launch_status();
}

extern "C" int csr_pcg_step(const csrad_csr* A, int32_t kind, const double* dinv,
                            const csrad_csr* L, const csrad_csr* Lt, const int32_t* perm,
                            int32_t nlevels, const int32_t* lp_host, const int32_t* lp_dev,
                            const int32_t* rows, double* x, double* r, double* z, double* p,
                            double* q, double* scal, double* hist, int32_t hist_cap, void* work,
                            size_t work_bytes, void* stream) {
  Precond pc;
  Parts parts;
  double* y;
  CSRAD_TRY(pcg_common(A, kind, dinv, L, Lt, perm, nlevels, lp_host, lp_dev, rows, work,
                       work_bytes, &pc, &parts, &y));
  const int n = A->nrows;
  if (n == 0) return CSRAD_OK;
  if (!x || !r || !z || !p || !q || !scal || hist_cap < 0) return CSRAD_EINVAL;
  hipStream_t s = as_stream(stream);
  const int nbv = vec_blocks(n);
  const int g = lanes_for(A->nnz, n);
  const int nbs = spmv_blocks(n, g);
  if (A->dtype == CSRAD_F32) {
    CSRAD_G_SWITCH(g, hipLaunchKernelGGL((k_pcg_spmv_dot<float, G>), dim3(nbs), dim3(kThreads), 0,
                                         s, n, A->rowptr, A->colind,
                                         static_cast<const float*>(A->vals), p, q, parts.pq, scal));
  } else {
    CSRAD_G_SWITCH(g, hipLaunchKernelGGL((k_pcg_spmv_dot<double, G>), dim3(nbs), dim3(kThreads),
                                         0, s, n, A->rowptr, A->colind,
                                         static_cast<const double*>(A->vals), p, q, parts.pq,
                                         scal));
  }
  hipLaunchKernelGGL(k_pcg_alpha, dim3(1), dim3(kThreads), 0, s, parts.pq, nbs, scal);
  if (kind == 1) {
    hipLaunchKernelGGL(k_pcg_update<1>, dim3(nbv), dim3(kThreads), 0, s, n, p, q, x, r, dinv, z,
                       parts, scal);
    CSRAD_TRY(precond_dots(n, pc, r, z, y, parts, scal, s));
  } else if (kind == 0) {
    hipLaunchKernelGGL(k_pcg_update<0>, dim3(nbv), dim3(kThreads), 0, s, n, p, q, x, r, dinv, z,
                       parts, scal);
  } else {
    hipLaunchKernelGGL(k_pcg_update<2>, dim3(nbv), dim3(kThreads), 0, s, n, p, q, x, r, dinv, z,
                       parts, scal);
  }
  hipLaunchKernelGGL(k_pcg_beta, dim3(1), dim3(kThreads), 0, s, parts, nbv, scal, hist, hist_cap);
  hipLaunchKernelGGL(k_pcg_p, dim3(nbv), dim3(kThreads), 0, s, n, z, p, scal);
  return launch_status();
}
