// Conjugate gradients (the Krylov solver of Section 4.3) and its reverse
// mode, as device-resident steps: scalars never leave the GPU, so a step
// needs no host synchronisation and can be captured in a graph.
//
// Forward step t (x0 = 0, r0 = b, p0 = b, rho0 = b.b):
//   q = A p, sigma = p.q, alpha = rho/sigma, x += alpha p, r -= alpha q,
//   rho' = r.r, beta = rho'/rho, p = r + beta p.
// Once rho is exactly zero, alpha = beta = 0 (converged; no 0/0).
// Dot products accumulate in float64 whatever the vector type: per-block
// partial sums, which every block of the kernel that needs the total adds
// up itself in one fixed order (no separate one-block reduction launches:
// three kernels per forward step, four per reverse step), so every step is
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
  S_RHO = 0,    // rho of the step in flight
  S_SIGMA,      // last sigma
  S_ALPHA,      // last alpha
  S_RHO1,       // last rho' (the current rho between steps)
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
    scal[S_RHO1] = rho;
    *step = 0;
  }
}

// ---------------- row products ----------------
// Row sums y_r = sum_e v[e] x[ci[e]] over a CSR matrix, handed to
// epi(r, y_r) by exactly one thread per row.  Two forms, chosen per matrix:
//
// Staged (mean row length up to kStageCap / kThreads): each block owns a
// contiguous range of 256-row blocks (XCD-aware); a row block's products are
// formed by all threads with coalesced loads of its consecutive entries and
// staged in LDS, then thread r sums row r in entry order.  A row block with
// more entries than the stage holds takes one wave per row.
//
// Lanes: G lanes per row (G the power of two at or above the mean row
// length), the block striding over row groups; lane sums in a fixed tree.
constexpr int kStageCap = 2560;

// Contiguous range [rb0, rb1) of 256-row blocks owned by this block.
__device__ __forceinline__ void owned_row_blocks(int n, int& rb0, int& rb1) {
  const int nrb = (n + kThreads - 1) / kThreads;
  const int per = (nrb + gridDim.x - 1) / gridDim.x;
  rb0 = xcd_block(blockIdx.x, gridDim.x) * per;
  rb1 = min(rb0 + per, nrb);
}

template <typename T, typename Epi>
__device__ __forceinline__ void staged_products(int n, const int32_t* __restrict__ rp,
                                                const int32_t* __restrict__ ci,
                                                const T* __restrict__ v, const T* __restrict__ x,
                                                T* prod, Epi&& epi) {
  int rb0, rb1;
  owned_row_blocks(n, rb0, rb1);
  for (int rb = rb0; rb < rb1; ++rb) {
    const int r0 = rb * kThreads, r1 = min(r0 + kThreads, n);
    const int e0 = rp[r0], cnt = rp[r1] - e0;
    const int r = r0 + threadIdx.x;
    if (cnt <= kStageCap) {
      for (int t = threadIdx.x; t < cnt; t += 4 * kThreads) {
        T pr[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int tt = t + u * kThreads;
          pr[u] = tt < cnt ? v[e0 + tt] * x[ci[e0 + tt]] : T(0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (t + u * kThreads < cnt) prod[t + u * kThreads] = pr[u];
      }
      __syncthreads();
      if (r < r1) {
        const int a = rp[r] - e0, c = rp[r + 1] - e0;
        T acc = 0;
        for (int t = a; t < c; ++t) acc += prod[t];
        epi(r, acc);
      }
      __syncthreads();  // the stage is refilled by the next row block
    } else {
      const int lane = threadIdx.x % kWave;
      for (int rr = r0 + threadIdx.x / kWave; rr < r1; rr += kThreads / kWave) {
        T acc = 0;
        for (int e = rp[rr] + lane; e < rp[rr + 1]; e += kWave) acc += v[e] * x[ci[e]];
        acc = group_sum<kWave>(acc);
        if (lane == 0) epi(rr, acc);
      }
    }
  }
}

template <typename T, int G, typename Epi>
__device__ __forceinline__ void lane_products(int n, const int32_t* __restrict__ rp,
                                              const int32_t* __restrict__ ci,
                                              const T* __restrict__ v, const T* __restrict__ x,
                                              Epi&& epi) {
  constexpr int RPB = kThreads / G;
  const int sub = threadIdx.x % G;
  for (int base = blockIdx.x * RPB; base < n; base += gridDim.x * RPB) {
    const int row = base + threadIdx.x / G;
    T s = 0;
    if (row < n) {
      const int e1 = rp[row + 1];
      for (int e = rp[row] + sub; e < e1; e += G) s += v[e] * x[ci[e]];
    }
    s = group_sum<G>(s);
    if (row < n && sub == 0) epi(row, s);
  }
}

// Row products in the form G names (0: staged).
template <typename T, int G, typename Epi>
__device__ __forceinline__ void row_products(int n, const int32_t* __restrict__ rp,
                                             const int32_t* __restrict__ ci,
                                             const T* __restrict__ v, const T* __restrict__ x,
                                             T* prod, Epi&& epi) {
  if constexpr (G == 0)
    staged_products<T>(n, rp, ci, v, x, prod, epi);
  else
    lane_products<T, G>(n, rp, ci, v, x, epi);
}

// q = A p and the block's share of p.q.
template <typename T, int G>
__global__ __launch_bounds__(kThreads) void k_cg_spmv_dot(int n, const int32_t* __restrict__ rp,
                                                          const int32_t* __restrict__ ci,
                                                          const T* __restrict__ v,
                                                          const T* __restrict__ p,
                                                          T* __restrict__ q,
                                                          T* __restrict__ p_save,
                                                          double* __restrict__ scal,
                                                          double* __restrict__ part) {
  __shared__ double sm[kThreads / kWave];
  __shared__ T prod[G == 0 ? kStageCap : 1];
  // rho of this step is rho' of the step before: no other block of this
  // kernel reads it, so the copy cannot race
  if (blockIdx.x == 0 && threadIdx.x == 0) scal[S_RHO] = scal[S_RHO1];
  double d = 0;
  row_products<T, G>(n, rp, ci, v, p, prod, [&](int r, T acc) {
    const T pr = p[r];
    q[r] = acc;
    if (p_save) p_save[r] = pr;
    d += (double)pr * (double)acc;
  });
  d = block_sum_double(d, sm);
  if (threadIdx.x == 0) part[blockIdx.x] = d;
}

// Every block sums the product kernel's p.q partials itself (same fixed
// order, so all blocks get the same sigma and alpha); block 0 records them.
// Then x += alpha p, r -= alpha q and the block's share of r.r.
template <typename T>
__global__ void k_cg_update(int n, const T* __restrict__ p, const T* __restrict__ q,
                            T* __restrict__ x, T* __restrict__ r, T* __restrict__ r_save,
                            double* __restrict__ scal, const double* __restrict__ part_pq,
                            int nb_pq, double* __restrict__ part_rr) {
  __shared__ double sm[kThreads / kWave];
  __shared__ double s_alpha;
  // the first element's operands are loaded before the partial sums are
  // read, so the two memory round trips overlap
  const int stride = gridDim.x * kThreads;
  int i = blockIdx.x * kThreads + threadIdx.x;
  T pi = T(0), qi = T(0), xi = T(0), ri = T(0);
  if (i < n) {
    pi = p[i];
    qi = q[i];
    xi = x[i];
    ri = r[i];
  }
  const double sigma = reduce_partials(part_pq, nb_pq, sm);
  if (threadIdx.x == 0) {
    const double rho = scal[S_RHO];
    const double a = rho != 0.0 ? rho / sigma : 0.0;
    s_alpha = a;
    if (blockIdx.x == 0) {
      scal[S_SIGMA] = sigma;
      scal[S_ALPHA] = a;
    }
  }
  __syncthreads();
  const T alpha = (T)s_alpha;
  double acc = 0;
  for (; i < n; i += stride) {
    x[i] = xi + alpha * pi;
    const T rn = ri - alpha * qi;
    r[i] = rn;
    if (r_save) r_save[i] = rn;
    acc += (double)rn * (double)rn;
    const int j = i + stride;
    if (j < n) {
      pi = p[j];
      qi = q[j];
      xi = x[j];
      ri = r[j];
    }
  }
  const double s = block_sum_double(acc, sm);
  if (threadIdx.x == 0) part_rr[blockIdx.x] = s;
}

// Every block sums the r.r partials (rho') and forms beta = rho'/rho; block
// 0 records rho' and beta, appends the step's scalars to the history and
// advances the step counter.  rho itself is left for the next product
// kernel to advance, since the other blocks here still read it.  Then
// p = r + beta p.
template <typename T>
__global__ void k_cg_p(int n, const T* __restrict__ r, T* __restrict__ p,
                       double* __restrict__ scal, const double* __restrict__ part_rr, int nb_rr,
                       double* __restrict__ hist, int* __restrict__ step, int hist_cap) {
  __shared__ double sm[kThreads / kWave];
  __shared__ double s_beta;
  const int stride = gridDim.x * kThreads;
  int i = blockIdx.x * kThreads + threadIdx.x;
  T ri = T(0), pi = T(0);
  if (i < n) {  // loaded before the partial sums, as in the update
    ri = r[i];
    pi = p[i];
  }
  const double rho1 = reduce_partials(part_rr, nb_rr, sm);
  if (threadIdx.x == 0) {
    const double rho = scal[S_RHO];
    const double beta = rho != 0.0 ? rho1 / rho : 0.0;
    s_beta = beta;
    if (blockIdx.x == 0) {
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
      *step = t + 1;
    }
  }
  __syncthreads();
  const T beta = (T)s_beta;
  for (; i < n; i += stride) {
    p[i] = ri + beta * pi;
    const int j = i + stride;
    if (j < n) {
      ri = r[j];
      pi = p[j];
    }
  }
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

// Every block sums k_cgb_1's partials (betab) itself; rhob of step t+1
// gains betab/rho (used here only), and block 0 records the betab part of
// the adjoint of rho_t.  Then rb += 2 rhob r_{t+1}, qb = -alpha rb,
// pb += alpha xb and the block's share of alphab = -rb.q + xb.p.
template <typename T>
__global__ void k_cgb_2(int n, const T* __restrict__ p, const T* __restrict__ q,
                        const T* __restrict__ r1, const T* __restrict__ xb, T* __restrict__ rb,
                        T* __restrict__ pb, T* __restrict__ qb, const double* __restrict__ h,
                        double* __restrict__ scal, const double* __restrict__ part_b,
                        int nb_b, double* __restrict__ part_a) {
  __shared__ double sm[kThreads / kWave];
  __shared__ double s_rhob;
  const int stride = gridDim.x * kThreads;
  int i = blockIdx.x * kThreads + threadIdx.x;
  T rbi = T(0), r1i = T(0), xbi = T(0), qi = T(0), pi = T(0), pbi = T(0);
  if (i < n) {  // loaded before the partial sums, as in the forward update
    rbi = rb[i];
    r1i = r1[i];
    xbi = xb[i];
    qi = q[i];
    pi = p[i];
    pbi = pb[i];
  }
  const double betab = reduce_partials(part_b, nb_b, sm);
  if (threadIdx.x == 0) {
    const double rho = h[0], rho1 = h[3];
    double rhob = scal[S_RHOB], rt = 0.0;
    if (rho != 0.0) {
      rhob += betab / rho;
      rt = -betab * rho1 / (rho * rho);
    }
    s_rhob = rhob;
    if (blockIdx.x == 0) scal[S_RHOB_T] = rt;
  }
  __syncthreads();
  const T alpha = (T)h[2];
  const T two_rhob = (T)(2.0 * s_rhob);
  double acc = 0;
  for (; i < n; i += stride) {
    const T rbn = rbi + two_rhob * r1i;
    rb[i] = rbn;
    acc += -(double)rbn * (double)qi + (double)xbi * (double)pi;
    qb[i] = -alpha * rbn;
    pb[i] = pbi + alpha * xbi;
    const int j = i + stride;
    if (j < n) {
      rbi = rb[j];
      r1i = r1[j];
      xbi = xb[j];
      qi = q[j];
      pi = p[j];
      pbi = pb[j];
    }
  }
  const double s = block_sum_double(acc, sm);
  if (threadIdx.x == 0) part_a[blockIdx.x] = s;
}

// Every block sums k_cgb_2's partials (alphab) and forms sigmab; block 0
// sets the adjoint of rho_t (the rhob of the step before) and records
// sigmab.  Then, over the rows i of A: qb_i gets its final value
// g_i = qb_i + sigmab p_i, and every entry e = (i, j) of row i gains
// gvals[e] += g_i p_j.  Staged form (G == 0): each block owns 256-row
// blocks; the row of each entry is spread into LDS so that the entries are
// swept with coalesced accesses.  Lanes form: G lanes per row.
template <typename T, int G>
__global__ __launch_bounds__(kThreads) void k_cgb_3(int n, const int32_t* __restrict__ rp,
                                                    const int32_t* __restrict__ ci,
                                                    const T* __restrict__ p,
                                                    T* __restrict__ qb, T* __restrict__ gv,
                                                    const double* __restrict__ h,
                                                    double* __restrict__ scal,
                                                    const double* __restrict__ part_a, int nb_a) {
  __shared__ double sm[kThreads / kWave];
  __shared__ double s_sb;
  __shared__ T sg[G == 0 ? kThreads : 1];
  __shared__ unsigned char rid[G == 0 ? kStageCap : 1];
  const double alphab = reduce_partials(part_a, nb_a, sm);
  if (threadIdx.x == 0) {
    const double rho = h[0], sigma = h[1];
    double sb = 0.0;
    if (rho != 0.0) sb = -alphab * rho / (sigma * sigma);
    s_sb = sb;
    if (blockIdx.x == 0) {
      double rt = scal[S_RHOB_T];
      if (rho != 0.0) rt += alphab / sigma;
      scal[S_SIGMAB] = sb;
      scal[S_RHOB] = rt;  // becomes the adjoint of rho_t for the step before
    }
  }
  __syncthreads();
  const T sb = (T)s_sb;
  if constexpr (G == 0) {
    int rb0, rb1;
    owned_row_blocks(n, rb0, rb1);
    for (int rb = rb0; rb < rb1; ++rb) {
      const int r0 = rb * kThreads, r1 = min(r0 + kThreads, n);
      const int e0 = rp[r0], cnt = rp[r1] - e0;
      const int r = r0 + threadIdx.x;
      const bool staged = cnt <= kStageCap;
      if (r < r1) {
        const T g = qb[r] + sb * p[r];
        qb[r] = g;
        sg[threadIdx.x] = g;
        if (staged)
          for (int t = rp[r] - e0, c = rp[r + 1] - e0; t < c; ++t) rid[t] = (unsigned char)threadIdx.x;
      }
      __syncthreads();
      if (staged) {
        for (int t = threadIdx.x; t < cnt; t += kThreads) {
          const int e = e0 + t;
          gv[e] += sg[rid[t]] * p[ci[e]];
        }
      } else {
        const int lane = threadIdx.x % kWave;
        for (int rr = r0 + threadIdx.x / kWave; rr < r1; rr += kThreads / kWave) {
          const T g = sg[rr - r0];
          for (int e = rp[rr] + lane; e < rp[rr + 1]; e += kWave) gv[e] += g * p[ci[e]];
        }
      }
      __syncthreads();  // sg and rid are refilled by the next row block
    }
  } else {
    constexpr int RPB = kThreads / G;
    const int sub = threadIdx.x % G;
    for (int base = blockIdx.x * RPB; base < n; base += gridDim.x * RPB) {
      const int row = base + threadIdx.x / G;
      if (row < n) {
        const T g = qb[row] + sb * p[row];
        for (int e = rp[row] + sub; e < rp[row + 1]; e += G) gv[e] += g * p[ci[e]];
        if (sub == 0) qb[row] = g;
      }
    }
  }
}

// pb[j] += sigmab q[j] + (A^T qb)_j, the product taken over the rows of A^T
// with A^T's own values.
template <typename T, int G>
__global__ __launch_bounds__(kThreads) void k_cgb_4(int n, const int32_t* __restrict__ rpT,
                                                    const int32_t* __restrict__ ciT,
                                                    const T* __restrict__ vT,
                                                    const T* __restrict__ q,
                                                    const T* __restrict__ qb,
                                                    T* __restrict__ pb,
                                                    const double* __restrict__ scal) {
  __shared__ T prod[G == 0 ? kStageCap : 1];
  const T sb = (T)scal[S_SIGMAB];
  row_products<T, G>(n, rpT, ciT, vT, qb, prod,
                     [&](int j, T acc) { pb[j] += sb * q[j] + acc; });
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

// Dispatch on a product form: 0 staged, else G lanes per row.
#define CSRAD_FORM_SWITCH(g, ...)                         \
  switch (g) {                                            \
    case 0: { constexpr int G = 0; __VA_ARGS__; } break;   \
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

// Product form of a square matrix: short rows (mean up to kStageCap /
// kThreads entries) take the staged form (0), others G lanes per row.
int product_form(const csrad_csr* A) {
  if ((long long)A->nnz * kThreads <= (long long)kStageCap * A->nrows) return 0;
  return lanes_for(A->nnz, A->nrows);
}

// Blocks of a product launch: the staged form's blocks own 256-row blocks
// (as many as a vector pass); the lanes form strides over row groups.
int product_blocks(int n, int form) { return form == 0 ? vec_blocks(n) : spmv_blocks(n, form); }

// Workspace: block partials (float64): the product kernel's p.q partials,
// then the update's r.r partials (kept apart, since the update's blocks
// still read the former while writing the latter).  The reverse step uses
// the first array.
size_t cg_partials(int n, int form) {
  const int a = product_blocks(n, form), b = vec_blocks(n);
  return (size_t)(a > b ? a : b) + (size_t)b;
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
  const int form = product_form(A);
  const int nbs = product_blocks(n, form), nbv = vec_blocks(n);
  double* part_rr = part + cg_partials(n, form) - nbv;
  CSRAD_FORM_SWITCH(form, hipLaunchKernelGGL((k_cg_spmv_dot<T, G>), dim3(nbs), dim3(kThreads), 0,
                                             s, n, A->rowptr, A->colind, v, p, q, p_save, scal,
                                             part));
  hipLaunchKernelGGL((k_cg_update<T>), dim3(nbv), dim3(kThreads), 0, s, n, p, q, x, r, r_save,
                     scal, part, nbs, part_rr);
  hipLaunchKernelGGL((k_cg_p<T>), dim3(nbv), dim3(kThreads), 0, s, n, r, p, scal, part_rr, nbv,
                     hist, step, hist_cap);
  return launch_status();
}

template <typename T>
int cg_step_bwd_t(const csrad_csr* A, const csrad_csr* At, const T* p, const T* q, const T* r1,
                  const double* h, const T* gR, T* xb, T* rb, T* pb, T* qb, double* scal, T* gv,
                  double* part, hipStream_t s) {
  const int n = A->nrows;
  const int nbv = vec_blocks(n);
  double* part_a = part + nbv;  // within the workspace: nbv <= the first array's size
  hipLaunchKernelGGL((k_cgb_1<T>), dim3(nbv), dim3(kThreads), 0, s, n, p, gR, rb, pb, h, part);
  hipLaunchKernelGGL((k_cgb_2<T>), dim3(nbv), dim3(kThreads), 0, s, n, p, q, r1, xb, rb, pb, qb, h,
                     scal, part, nbv, part_a);
  const int fa = product_form(A), ft = product_form(At);
  CSRAD_FORM_SWITCH(fa, hipLaunchKernelGGL((k_cgb_3<T, G>), dim3(product_blocks(n, fa)),
                                           dim3(kThreads), 0, s, n, A->rowptr, A->colind, p, qb,
                                           gv, h, scal, part_a, nbv));
  CSRAD_FORM_SWITCH(ft, hipLaunchKernelGGL((k_cgb_4<T, G>), dim3(product_blocks(n, ft)),
                                           dim3(kThreads), 0, s, n, At->rowptr, At->colind,
                                           static_cast<const T*>(At->vals), q, qb, pb, scal));
  return launch_status();
}

}  // namespace
}  // namespace csrad

using namespace csrad;

extern "C" int csr_cg_workspace(const csrad_csr* A, size_t* bytes) {
  if (!A || !bytes || A->nrows < 0) return CSRAD_EINVAL;
  *bytes = sizeof(double) * cg_partials(A->nrows, product_form(A)) + 256;
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

extern "C" int csr_cg_step_bwd(const csrad_csr* A, const csrad_csr* At, const void* p,
                               const void* q, const void* r1, const double* step_hist,
                               const void* gR, void* xb, void* rb, void* pb, void* qb,
                               double* scal, void* gvals, void* work, size_t work_bytes,
                               void* stream) {
  CSRAD_TRY(check_square(A));
  CSRAD_TRY(check_csr(At, true));
  if (At->nrows != A->ncols || At->ncols != A->nrows || At->nnz != A->nnz ||
      At->dtype != A->dtype)
    return CSRAD_EINVAL;
  if (A->nrows == 0) return CSRAD_OK;
  if (!p || !q || !r1 || !step_hist || !xb || !rb || !pb || !qb || !scal || !gvals)
    return CSRAD_EINVAL;
  size_t need = 0;
  CSRAD_TRY(csr_cg_workspace(A, &need));
  if (!work || work_bytes < need) return CSRAD_EWORKSPACE;
  hipStream_t s = as_stream(stream);
  double* part = static_cast<double*>(work);
  if (A->dtype == CSRAD_F32)
    return cg_step_bwd_t<float>(A, At, static_cast<const float*>(p), static_cast<const float*>(q),
                                static_cast<const float*>(r1), step_hist,
                                static_cast<const float*>(gR), static_cast<float*>(xb),
                                static_cast<float*>(rb), static_cast<float*>(pb),
                                static_cast<float*>(qb), scal, static_cast<float*>(gvals), part, s);
  return cg_step_bwd_t<double>(A, At, static_cast<const double*>(p),
                               static_cast<const double*>(q), static_cast<const double*>(r1),
                               step_hist, static_cast<const double*>(gR),
                               static_cast<double*>(xb), static_cast<double*>(rb),
                               static_cast<double*>(pb), static_cast<double*>(qb), scal,
                               static_cast<double*>(gvals), part, s);
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
