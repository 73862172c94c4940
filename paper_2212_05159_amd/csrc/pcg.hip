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
//   inverse factor: z = L (L^T r), M = L L^T approximating A^{-1} itself
//            (the form Section 4.3 learns), two sparse products; r.z is
//            taken as ||L^T r||^2 from the first, and the second is fused
//            with the p update.
// init copies A (and, when every level of L is wide, L and L^T by level;
// for the inverse factor, L and L^T whole) into ELL layouts in the
// workspace; the steps read those copies.
#include "internal.hpp"

namespace csrad {
namespace {

constexpr int kThreads = 256;
constexpr int kVecBlocksMax = 2048;   // grid of the vector kernels
constexpr int kSpmvBlocksMax = 8192;  // grid of the product kernel

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
  double* rz;  // kVecBlocksMax, or the factor plan's per-level-block partials
  double* rr;  // kVecBlocksMax
  int nrz;     // number of r.z partials written by the preconditioner step
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

// Block sum for any block size that is a multiple of the wave (sm holds
// one double per wave; fixed order).
__device__ double block_sum_any(double v, double* sm) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if (threadIdx.x % kWave == 0) sm[threadIdx.x / kWave] = v;
  __syncthreads();
  double t = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x / kWave); ++i) t += sm[i];
  __syncthreads();
  return t;
}

// Single-block reductions of block partials run with kRedThreads threads.
constexpr int kRedThreads = 1024;

__device__ double reduce_parts(const double* __restrict__ part, int nb, double* sm) {
  double v = 0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) v += part[i];
  return block_sum_any(v, sm);
}

int vec_blocks(int n) {
  int b = (n + kThreads - 1) / kThreads;
  return b < 1 ? 1 : (b > kVecBlocksMax ? kVecBlocksMax : b);
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
  __shared__ double sm[kRedThreads / kWave];
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
__global__ void k_pcg_start(int n, Parts parts, const double* __restrict__ z,
                            double* __restrict__ p, double* __restrict__ scal) {
  __shared__ double sm[kThreads / kWave];
  __shared__ double rho_s;
  if (scal[P_DONE] != 0.0) return;
  const double a = reduce_parts(parts.rz, parts.nrz, sm);
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

// ---------------------------------------------------------------------
// ELL copies.  The matrix of every PCG step is fixed for a whole solve, so
// init copies it into a sliced ELL layout: rows split into segments (one
// segment for A; for the factor, one per level, rows in level order); a
// segment of R rows and width w keeps slot k of its i-th row at
// col/val[off + k R + i] (col -1 pads short rows).  A thread per row then
// reads its slots with coalesced loads and no row-pointer lookups.  Widths
// come from the device; a segment that would overflow the preallocated
// capacity gets width -1 and its rows are read from the CSR arrays instead.
// For the factors the diagonal is kept apart (diag[q]), so the slots hold
// only off-diagonal entries.
// ---------------------------------------------------------------------
struct Ell {
  int32_t* w;      // [nseg] width, or -1 (rows read from CSR)
  long long* off;  // [nseg] first slot
  int32_t* col;    // [cap]
  void* val;       // [cap] value type of the matrix
  long long cap;
};

// Segment of level-ordered row q: the l with lp[l] <= q < lp[l+1].
__device__ __forceinline__ int segment_of(int q, int nseg, const int32_t* __restrict__ lp) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (lp[mid] <= q) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Width of one segment: the longest row (minus its diagonal when
// skip_diag), one atomicMax per block.
__global__ void k_ell_width(int seg, int q0, int q1, const int32_t* __restrict__ rp,
                            const int32_t* __restrict__ rows, int skip_diag,
                            int32_t* __restrict__ w) {
  __shared__ int sm[kThreads / kWave];
  int m = 0;
  for (int q = q0 + blockIdx.x * kThreads + threadIdx.x; q < q1; q += gridDim.x * kThreads) {
    const int r = rows ? rows[q] : q;
    m = max(m, rp[r + 1] - rp[r] - skip_diag);
  }
  m = wave_max(m);
  if (threadIdx.x % kWave == 0) sm[threadIdx.x / kWave] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < kThreads / kWave; ++i) m = max(m, sm[i]);
    atomicMax(&w[seg], m);
  }
}

// Slot offsets in segment order; a segment that does not fit gets -1.
__global__ void k_ell_offsets(int nseg, const int32_t* __restrict__ lp, int n, long long cap,
                              int32_t* __restrict__ w, long long* __restrict__ off) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  long long run = 0;
  for (int l = 0; l < nseg; ++l) {
    const long long R = lp ? lp[l + 1] - lp[l] : n;
    off[l] = run;
    if (run + (long long)w[l] * R <= cap) run += (long long)w[l] * R;
    else w[l] = -1;
  }
}

// Fills the slots (and, with diag, the diagonal of the factors).
template <typename TV>
__global__ void k_ell_fill(int n, int nseg, const int32_t* __restrict__ lp,
                           const int32_t* __restrict__ rows, const int32_t* __restrict__ rp,
                           const int32_t* __restrict__ ci, const TV* __restrict__ v,
                           const int32_t* __restrict__ perm, const int32_t* __restrict__ w,
                           const long long* __restrict__ off, int32_t* __restrict__ col,
                           TV* __restrict__ val, TV* __restrict__ diag) {
  for (int q = blockIdx.x * kThreads + threadIdx.x; q < n; q += gridDim.x * kThreads) {
    const int l = lp ? segment_of(q, nseg, lp) : 0;
    const int q0 = lp ? lp[l] : 0;
    const long long R = lp ? lp[l + 1] - q0 : n;
    const int ws = w[l];
    const int r = rows ? rows[q] : q;
    const long long base = off[l] + (q - q0);
    int k = 0;
    for (int e = rp[r]; e < rp[r + 1]; ++e) {
      const int c = ci[e];
      const TV x = perm ? v[perm[e]] : v[e];
      if (diag && c == r) {
        diag[q] = x;
      } else if (k < ws) {
        col[base + (long long)k * R] = c;
        val[base + (long long)k * R] = x;
        ++k;
      }
    }
    if (ws >= 0)
      for (; k < ws; ++k) {
        col[base + (long long)k * R] = -1;
        val[base + (long long)k * R] = TV(0);
      }
  }
}

// q = A p over A's ELL copy (or its CSR rows), and the block's p.q partial.
template <typename TV>
__global__ __launch_bounds__(kThreads) void k_pcg_spmv_ell(
    int n, const int32_t* __restrict__ w, const int32_t* __restrict__ col,
    const TV* __restrict__ val, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
    const TV* __restrict__ v, const double* __restrict__ p, double* __restrict__ q,
    double* __restrict__ part, const double* __restrict__ scal) {
  __shared__ double sm[kThreads / kWave];
  // No done check: p does not change once the state is final, so a later
  // step recomputes the same q and partials (the alpha kernel then leaves
  // the state alone); skipping the check saves a dependent load.
  (void)scal;
  const int ws = w[0];
  double d = 0;
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
    double s = 0;
    if (ws >= 0) {
      for (int k = 0; k < ws; ++k) {
        const int c = col[(long long)k * n + i];
        const TV a = val[(long long)k * n + i];
        if (c >= 0) s += (double)a * p[c];
      }
    } else {
      for (int e = rp[i]; e < rp[i + 1]; ++e) s += (double)v[e] * p[ci[e]];
    }
    q[i] = s;
    d += p[i] * s;
  }
  d = block_sum(d, sm);
  if (threadIdx.x == 0) part[blockIdx.x] = d;
}

// out = M in over a one-segment ELL copy of M (or its CSR rows, values
// through perm when given).  MODE 0: nothing else; MODE 1: the block's
// share of <out, out> goes to dot_part[blockIdx.x]; MODE 2: p = out +
// beta p with beta from scal (the whole kernel is skipped once the state
// is final, as the p update is).  Modes 0 and 1 have no done check: their
// inputs do not change once the state is final.
template <typename TV, int MODE>
__global__ __launch_bounds__(kThreads) void k_pcg_ell_apply(
    int n, const int32_t* __restrict__ w, const int32_t* __restrict__ col,
    const TV* __restrict__ val, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
    const TV* __restrict__ v, const int32_t* __restrict__ perm, const double* __restrict__ in,
    double* __restrict__ out, double* __restrict__ p, double* __restrict__ dot_part,
    const double* __restrict__ scal) {
  __shared__ double sm[kThreads / kWave];
  if (MODE == 2 && scal[P_DONE] != 0.0) return;
  const double beta = MODE == 2 ? scal[P_BETA] : 0.0;
  const int ws = w[0];
  double d = 0;
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
    double s = 0;
    if (ws >= 0) {
      for (int k = 0; k < ws; ++k) {
        const int c = col[(long long)k * n + i];
        const TV a = val[(long long)k * n + i];
        if (c >= 0) s += (double)a * in[c];
      }
    } else {
      for (int e = rp[i]; e < rp[i + 1]; ++e)
        s += (double)(perm ? v[perm[e]] : v[e]) * in[ci[e]];
    }
    out[i] = s;
    if (MODE == 1) d += s * s;
    if (MODE == 2) p[i] = s + beta * p[i];
  }
  if (MODE == 1) {
    d = block_sum(d, sm);
    if (threadIdx.x == 0) dot_part[blockIdx.x] = d;
  }
}

int spmv_blocks(int n) {
  int b = (n + kThreads - 1) / kThreads;
  return b < 1 ? 1 : (b > kSpmvBlocksMax ? kSpmvBlocksMax : b);
}

__global__ void k_pcg_alpha(const double* __restrict__ part, int nb, double* __restrict__ scal) {
  __shared__ double sm[kRedThreads / kWave];
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

// x += alpha p, r -= alpha q and the r.r partial, fused with the diagonal
// preconditioners and the r.z partial (KIND 0 Jacobi, 2 none); for KIND 1
// (factor) r.z comes with the solves.
// For the factor with ELL copies, d0 holds 1 / L_ii on the rows of level
// 0 (which have no off-diagonal entry in L) and 0 elsewhere: those rows'
// forward solve y = r / L_ii is done here (a zero L_ii gives inf, as in
// the solve kernels).
template <int KIND>
__global__ void k_pcg_update(int n, const double* __restrict__ p, const double* __restrict__ q,
                             double* __restrict__ x, double* __restrict__ r,
                             const double* __restrict__ dinv, double* __restrict__ z, Parts parts,
                             const double* __restrict__ d0, double* __restrict__ y0,
                             const double* __restrict__ scal) {
  __shared__ double sm[kThreads / kWave];
  if (scal[P_DONE] != 0.0) return;
  const double alpha = scal[P_ALPHA];
  double rz = 0, rr = 0;
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    rr += ri * ri;
    if (KIND == 1 && d0) {
      const double dd = d0[i];
      if (dd != 0.0) y0[i] = ri * dd;
    }
    if (KIND != 1) {
      const double zi = KIND == 0 ? ri * dinv[i] : ri;
      z[i] = zi;
      rz += ri * zi;
    }
  }
  rr = block_sum(rr, sm);
  if (KIND != 1) rz = block_sum(rz, sm);
  if (threadIdx.x == 0) {
    parts.rr[blockIdx.x] = rr;
    if (KIND != 1) parts.rz[blockIdx.x] = rz;
  }
}

// rho' = r.z, beta, residual and convergence; counts the step.
__global__ void k_pcg_beta(Parts parts, int nb, double* __restrict__ scal,
                           double* __restrict__ hist, int hist_cap) {
  __shared__ double sm[kRedThreads / kWave];
  if (scal[P_DONE] != 0.0) return;
  const double a = reduce_parts(parts.rz, parts.nrz, sm);
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

// ---------------------------------------------------------------------
// Factor solves over ELL copies of L and L^T by level.  When every level is
// wide, each level is one segment of the ELL copies (rows in level order),
// and each level is one launch of a thread-per-row kernel.  Levels with
// fewer rows use the general solves.
// ---------------------------------------------------------------------
constexpr int kEllMinRows = 1024;

bool ell_levels(int nlevels, const int32_t* lp_host) {
  for (int l = 0; l < nlevels; ++l)
    if (lp_host[l + 1] - lp_host[l] < kEllMinRows) return false;
  return true;
}

struct FactorPlan {
  bool on;
  Ell fwd;     // off-diagonal entries of L's rows, by level
  Ell bwd;     // off-diagonal entries of L^T's rows, by level
  void* diag;  // [n] diagonal of L, level order
  double* d0;  // [n] 1 / L_ii on level-0 rows, 0 elsewhere, natural order
  int32_t* ident;  // [1] 1 when the level order is the identity (rows[q] == q)
};

// Clears *flag when some rows[q] != q (the flag is set to 1 before).
__global__ void k_rows_identity(int n, const int32_t* __restrict__ rows, int32_t* __restrict__ flag) {
  for (int q = blockIdx.x * kThreads + threadIdx.x; q < n; q += gridDim.x * kThreads)
    if (rows[q] != q) *flag = 0;
}

// d0[rows[q]] = 1 / diag[q] for the level-0 rows q < q1 (d0 zeroed before).
template <typename TV>
__global__ void k_level0_diag(int q1, const int32_t* __restrict__ rows,
                              const TV* __restrict__ diag, double* __restrict__ d0) {
  for (int q = blockIdx.x * kThreads + threadIdx.x; q < q1; q += gridDim.x * kThreads)
    d0[rows[q]] = 1.0 / (double)diag[q];
}

// One level of the solve: x[rows[q]] = (b[rows[q]] - off-diagonal part) /
// diag[q] for q in [q0, q1).  With dot_r set, the block writes its share of
// <dot_r, out> to dot_part[blockIdx.x], where out is x, or z2 when z2 is
// given; with z2 set (the forward solve's last level, whose rows have
// nothing above them in the backward solve) the kernel also finishes those
// rows' backward solve: z2 = x / diagonal.  A level without an ELL copy is
// read from the CSR arrays (rp, ci, v through perm when given), skipping
// the diagonal.
constexpr int kLevelThreads = kThreads;

template <typename TV>
__global__ __launch_bounds__(kLevelThreads) void k_level_ell(
    int seg, int q0, int q1, const int32_t* __restrict__ w, const long long* __restrict__ off,
    const int32_t* __restrict__ col, const TV* __restrict__ val, const TV* __restrict__ diag,
    const int32_t* __restrict__ ident, const int32_t* __restrict__ rows,
    const int32_t* __restrict__ rp, const int32_t* __restrict__ ci, const TV* __restrict__ v,
    const int32_t* __restrict__ perm, const double* __restrict__ b, double* __restrict__ x,
    double* __restrict__ z2, const double* __restrict__ dot_r, double* __restrict__ dot_part,
    const double* __restrict__ scal) {
  __shared__ double sm[kLevelThreads / kWave];
  // No done check: r does not change once the state is final, so a later
  // step recomputes the same y, z and partials.
  (void)scal;
  const int ws = w[seg];
  const bool id = *ident != 0;
  const long long R = q1 - q0, o = off[seg];
  const int i = blockIdx.x * kLevelThreads + threadIdx.x;
  double dot = 0;
  if (i < R) {
    const int q = q0 + i;
    const int row = id ? q : rows[q];
    double acc = 0;
    if (ws >= 0) {
      for (int k = 0; k < ws; ++k) {
        const int c = col[o + (long long)k * R + i];
        const TV a = val[o + (long long)k * R + i];
        if (c >= 0) acc += (double)a * x[c];
      }
    } else {
      for (int e = rp[row]; e < rp[row + 1]; ++e) {
        const int c = ci[e];
        if (c != row) acc += (double)(perm ? v[perm[e]] : v[e]) * x[c];
      }
    }
    const double dg = (double)diag[q];
    const double xr = (b[row] - acc) / dg;
    x[row] = xr;
    double out = xr;
    if (z2) {
      out = xr / dg;
      z2[row] = out;
    }
    if (dot_r) dot = dot_r[row] * out;
  }
  if (dot_r) {
    dot = block_sum_any(dot, sm);
    if (threadIdx.x == 0) dot_part[blockIdx.x] = dot;
  }
}

int level_blocks(int rows) {
  const int b = (rows + kLevelThreads - 1) / kLevelThreads;
  return b < 1 ? 1 : b;
}

// Total number of blocks over the levels (the r.z partials of a step).
int plan_dot_blocks(int nlevels, const int32_t* lp_host) {
  int t = 0;
  for (int l = 0; l < nlevels; ++l) t += level_blocks(lp_host[l + 1] - lp_host[l]);
  return t;
}

struct Precond;
template <typename TV>
void factor_solves_ell(const Precond& pc, const double* r, double* y, double* z, double* rz_parts,
                       const double* scal, hipStream_t s, bool level0_done);

struct Precond {
  int kind;  // 0 Jacobi, 1 factor, 2 none, 3 inverse factor
  const double* dinv;
  const csrad_csr* L;
  const csrad_csr* Lt;
  const int32_t* perm;
  int nlevels;
  const int32_t* lp_host;
  const int32_t* lp_dev;
  const int32_t* rows;
  FactorPlan plan;
  Ell invL, invLt;  // inverse factor: one-segment ELL copies of L and L^T
};

// z = L^{-T} L^{-1} r over the ELL copies, level by level.  The last
// forward level also finishes its rows' backward solve; every level writes
// the r.z partials of its rows (level order, then block order).
template <typename TV>
void factor_solves_ell(const Precond& pc, const double* r, double* y, double* z, double* rz_parts,
                       const double* scal, hipStream_t s, bool level0_done) {
  const FactorPlan& fp = pc.plan;
  const int nl = pc.nlevels, top = nl - 1;
  const int32_t* lp = pc.lp_host;
  const TV* vL = static_cast<const TV*>(pc.L->vals);
  const TV* vT = pc.Lt->vals ? static_cast<const TV*>(pc.Lt->vals) : vL;
  const int32_t* pT = pc.Lt->vals ? nullptr : pc.perm;
  const TV* dg = static_cast<const TV*>(fp.diag);
  const int top_off = plan_dot_blocks(nl, lp) - level_blocks(lp[nl] - lp[top]);
  for (int l = level0_done && top > 0 ? 1 : 0; l < nl; ++l) {
    const bool last = l == top;
    hipLaunchKernelGGL((k_level_ell<TV>), dim3(level_blocks(lp[l + 1] - lp[l])),
                       dim3(kLevelThreads), 0, s, l, lp[l], lp[l + 1], fp.fwd.w, fp.fwd.off,
                       fp.fwd.col, static_cast<const TV*>(fp.fwd.val), dg, fp.ident, pc.rows,
                       pc.L->rowptr,
                       pc.L->colind, vL, nullptr, r, y, last ? z : nullptr, last ? r : nullptr,
                       last ? rz_parts + top_off : nullptr, scal);
  }
  int o = top_off;
  for (int l = top - 1; l >= 0; --l) {
    const int nb = level_blocks(lp[l + 1] - lp[l]);
    o -= nb;
    hipLaunchKernelGGL((k_level_ell<TV>), dim3(nb), dim3(kLevelThreads), 0, s, l, lp[l],
                       lp[l + 1], fp.bwd.w, fp.bwd.off, fp.bwd.col,
                       static_cast<const TV*>(fp.bwd.val), dg, fp.ident, pc.rows, pc.Lt->rowptr,
                       pc.Lt->colind, vT, pT, y, z, nullptr, r,
                       rz_parts + o, scal);
  }
}

// The inverse factor's two products over its ELL copies.  y = L^T r with
// the partials of r.z = r.(L L^T r) = ||y||^2 (vec_blocks grid, as the
// update kernel's, so they fit the r.z slots); then z = L y, fused with
// p = z + beta p inside a step (fuse_p), plain at init.
template <typename TV>
void inverse_factor_y(int n, const Precond& pc, const double* r, double* y, double* rz_parts,
                      hipStream_t s) {
  const TV* vL = static_cast<const TV*>(pc.L->vals);
  const TV* vT = pc.Lt->vals ? static_cast<const TV*>(pc.Lt->vals) : vL;
  const int32_t* pT = pc.Lt->vals ? nullptr : pc.perm;
  hipLaunchKernelGGL((k_pcg_ell_apply<TV, 1>), dim3(vec_blocks(n)), dim3(kThreads), 0, s, n,
                     pc.invLt.w, pc.invLt.col, static_cast<const TV*>(pc.invLt.val),
                     pc.Lt->rowptr, pc.Lt->colind, vT, pT, r, y, nullptr, rz_parts, nullptr);
}

template <typename TV>
void inverse_factor_z(int n, const Precond& pc, const double* y, double* z, double* p,
                      const double* scal, hipStream_t s) {
  const TV* vL = static_cast<const TV*>(pc.L->vals);
  if (p) {
    hipLaunchKernelGGL((k_pcg_ell_apply<TV, 2>), dim3(vec_blocks(n)), dim3(kThreads), 0, s, n,
                       pc.invL.w, pc.invL.col, static_cast<const TV*>(pc.invL.val),
                       pc.L->rowptr, pc.L->colind, vL, nullptr, y, z, p, nullptr, scal);
  } else {
    hipLaunchKernelGGL((k_pcg_ell_apply<TV, 0>), dim3(vec_blocks(n)), dim3(kThreads), 0, s, n,
                       pc.invL.w, pc.invL.col, static_cast<const TV*>(pc.invL.val),
                       pc.L->rowptr, pc.L->colind, vL, nullptr, y, z, nullptr, nullptr, scal);
  }
}

// z = M^{-1} r followed by the r.z and r.r partials.  The factor solves
// are not conditional on the done flag, so their cost is paid until the
// host stops stepping.
// level0_done: the factor's level-0 rows of y were already written (by the
// step's update kernel).
int precond_dots(int n, const Precond& pc, const double* r, double* z, double* y, Parts parts,
                 const double* scal, hipStream_t s, bool level0_done = false) {
  const int nbv = vec_blocks(n);
  if (pc.kind == 0) {
    hipLaunchKernelGGL(k_pcg_precond_dots<0>, dim3(nbv), dim3(kThreads), 0, s, n, pc.dinv, r, z,
                       parts, scal);
  } else if (pc.kind == 1) {
    if (pc.plan.on) {
      if (pc.L->dtype == CSRAD_F32)
        factor_solves_ell<float>(pc, r, y, z, parts.rz, scal, s, level0_done);
      else
        factor_solves_ell<double>(pc, r, y, z, parts.rz, scal, s, level0_done);
    } else {
      CSRAD_TRY(trisolve_vec64(pc.L, 1, pc.Lt, pc.perm, false, pc.nlevels, pc.lp_host,
                               pc.lp_dev, pc.rows, r, y, s));
      CSRAD_TRY(trisolve_vec64(pc.L, 1, pc.Lt, pc.perm, true, pc.nlevels, pc.lp_host, pc.lp_dev,
                               pc.rows, y, z, s));
      hipLaunchKernelGGL(k_pcg_precond_dots<1>, dim3(nbv), dim3(kThreads), 0, s, n, pc.dinv, r,
                         z, parts, scal);
    }
  } else if (pc.kind == 3) {  // init: y = L^T r (+ r.z partials), z = L y
    if (pc.L->dtype == CSRAD_F32) {
      inverse_factor_y<float>(n, pc, r, y, parts.rz, s);
      inverse_factor_z<float>(n, pc, y, z, nullptr, scal, s);
    } else {
      inverse_factor_y<double>(n, pc, r, y, parts.rz, s);
      inverse_factor_z<double>(n, pc, y, z, nullptr, scal, s);
    }
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
  if ((kind != 1 && kind != 3) || !L || !Lt) return CSRAD_EINVAL;
  if (kind == 3) {
    CSRAD_TRY(check_csr(L, true));
    CSRAD_TRY(check_csr(Lt, false));
    if (L->nrows != A->nrows || L->ncols != A->nrows || Lt->nrows != A->nrows ||
        Lt->ncols != A->nrows || Lt->nnz != L->nnz)
      return CSRAD_EINVAL;
    if (L->nnz > 0 && !perm && !Lt->vals) return CSRAD_EINVAL;
    if (Lt->vals && Lt->dtype != L->dtype) return CSRAD_EDTYPE;
    return CSRAD_OK;
  }
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

// Workspace: partials, the intermediate vector of the factor solves, A's
// ELL copy and, for a factor whose levels are all wide, the ELL copies of
// L and L^T by level with the diagonal and the per-level r.z partials.
struct PcgWs {
  Parts parts;
  double* y;
  Ell ellA;
  FactorPlan plan;
  Ell invL, invLt;
};

Ell carve_ell(Carver& cv, int nseg, long long cap, size_t vs) {
  Ell e;
  e.w = cv.take<int32_t>((size_t)nseg);
  e.off = cv.take<long long>((size_t)nseg);
  e.col = cv.take<int32_t>((size_t)cap);
  e.val = cv.take<char>((size_t)cap * vs);
  e.cap = cap;
  return e;
}

long long ell_cap(long long nnz, int n) {
  const long long c = 2 * nnz;
  return c > n ? c : (long long)n;
}

PcgWs carve_pcg(Carver& cv, const csrad_csr* A, const csrad_csr* L, bool with_plan, int nlevels,
                const int32_t* lp_host, bool inverse) {
  const int n = A->nrows;
  PcgWs w;
  double* pd = cv.take<double>(kPartsDoubles);
  w.parts = Parts{pd, pd ? pd + kSpmvBlocksMax : nullptr,
                  pd ? pd + kSpmvBlocksMax + kVecBlocksMax : nullptr, vec_blocks(n)};
  w.y = cv.take<double>((size_t)(n > 0 ? n : 1));
  w.ellA = carve_ell(cv, 1, ell_cap(A->nnz, n), A->dtype == CSRAD_F32 ? 4 : 8);
  w.plan = FactorPlan{};
  w.plan.on = false;
  if (with_plan && L) {
    const size_t vs = L->dtype == CSRAD_F32 ? 4 : 8;
    w.plan.on = true;
    // the solves write one r.z partial per level block
    w.parts.nrz = plan_dot_blocks(nlevels, lp_host);
    w.parts.rz = cv.take<double>((size_t)w.parts.nrz);
    w.plan.fwd = carve_ell(cv, nlevels, ell_cap(L->nnz, n), vs);
    w.plan.bwd = carve_ell(cv, nlevels, ell_cap(L->nnz, n), vs);
    w.plan.diag = cv.take<char>((size_t)(n > 0 ? n : 1) * vs);
    w.plan.d0 = cv.take<double>((size_t)(n > 0 ? n : 1));
    w.plan.ident = cv.take<int32_t>(1);
  }
  w.invL = w.invLt = Ell{};
  if (inverse && L) {
    const size_t vs = L->dtype == CSRAD_F32 ? 4 : 8;
    w.invL = carve_ell(cv, 1, ell_cap(L->nnz, n), vs);
    w.invLt = carve_ell(cv, 1, ell_cap(L->nnz, n), vs);
  }
  return w;
}

// Builds an ELL copy: widths (one launch per segment), offsets, slots.
template <typename TV>
int build_ell(const Ell& e, int n, int nseg, const int32_t* lp_host, const int32_t* lp_dev,
              const int32_t* rows, const int32_t* rp, const int32_t* ci, const TV* v,
              const int32_t* perm, TV* diag, hipStream_t s) {
  CSRAD_TRY(fill_i32(e.w, nseg, 0, s));
  for (int l = 0; l < nseg; ++l) {
    const int q0 = lp_host ? lp_host[l] : 0, q1 = lp_host ? lp_host[l + 1] : n;
    int g = (q1 - q0 + 16 * kThreads - 1) / (16 * kThreads);
    g = g < 1 ? 1 : g;
    hipLaunchKernelGGL(k_ell_width, dim3(g), dim3(kThreads), 0, s, l, q0, q1, rp, rows,
                       diag ? 1 : 0, e.w);
  }
  hipLaunchKernelGGL(k_ell_offsets, dim3(1), dim3(64), 0, s, nseg, lp_dev, n, e.cap, e.w, e.off);
  hipLaunchKernelGGL((k_ell_fill<TV>), dim3(vec_blocks(n)), dim3(kThreads), 0, s, n, nseg, lp_dev,
                     rows, rp, ci, v, perm, e.w, e.off, e.col, static_cast<TV*>(e.val), diag);
  return launch_status();
}

// A's ELL copy.
template <typename TV>
int build_ell_a(const csrad_csr* A, const Ell& ellA, hipStream_t s) {
  return build_ell<TV>(ellA, A->nrows, 1, nullptr, nullptr, nullptr, A->rowptr, A->colind,
                       static_cast<const TV*>(A->vals), nullptr, nullptr, s);
}

// The factor's ELL copies by level (values of L^T from Lt's own values when
// present, else through perm) and its diagonal.
template <typename TV>
int build_ell_factor(int n, const Precond& pc, hipStream_t s) {
  const TV* vL = static_cast<const TV*>(pc.L->vals);
  TV* dg = static_cast<TV*>(pc.plan.diag);
  CSRAD_TRY(build_ell<TV>(pc.plan.fwd, n, pc.nlevels, pc.lp_host, pc.lp_dev, pc.rows,
                          pc.L->rowptr, pc.L->colind, vL, nullptr, dg, s));
  const TV* vT = pc.Lt->vals ? static_cast<const TV*>(pc.Lt->vals) : vL;
  CSRAD_TRY(build_ell<TV>(pc.plan.bwd, n, pc.nlevels, pc.lp_host, pc.lp_dev, pc.rows,
                          pc.Lt->rowptr, pc.Lt->colind, vT, pc.Lt->vals ? nullptr : pc.perm, dg,
                          s));
  CSRAD_TRY(fill_bytes_zero(pc.plan.d0, sizeof(double) * (size_t)n, s));
  CSRAD_TRY(fill_i32(pc.plan.ident, 1, 1, s));
  hipLaunchKernelGGL(k_rows_identity, dim3(vec_blocks(n)), dim3(kThreads), 0, s, n, pc.rows,
                     pc.plan.ident);
  hipLaunchKernelGGL((k_level0_diag<TV>), dim3(vec_blocks(pc.lp_host[1])), dim3(kThreads), 0, s,
                     pc.lp_host[1], pc.rows, dg, pc.plan.d0);
  return launch_status();
}

// The inverse factor's one-segment ELL copies of L and L^T (all entries,
// the diagonal included; L^T's values from Lt's own or through perm).
template <typename TV>
int build_ell_inverse(int n, const Precond& pc, hipStream_t s) {
  const TV* vL = static_cast<const TV*>(pc.L->vals);
  CSRAD_TRY(build_ell<TV>(pc.invL, n, 1, nullptr, nullptr, nullptr, pc.L->rowptr, pc.L->colind,
                          vL, nullptr, nullptr, s));
  const TV* vT = pc.Lt->vals ? static_cast<const TV*>(pc.Lt->vals) : vL;
  return build_ell<TV>(pc.invLt, n, 1, nullptr, nullptr, nullptr, pc.Lt->rowptr, pc.Lt->colind,
                       vT, pc.Lt->vals ? nullptr : pc.perm, nullptr, s);
}

}  // namespace
}  // namespace csrad

using namespace csrad;

extern "C" int csr_pcg_workspace(const csrad_csr* A, const csrad_csr* L, int32_t nlevels,
                                 const int32_t* level_ptr_host, size_t* bytes) {
  if (!A || !bytes || A->nrows < 0) return CSRAD_EINVAL;
  if (L && (L->nnz < 0 || (nlevels > 0 && !level_ptr_host))) return CSRAD_EINVAL;
  const bool plan = L && nlevels > 0 && ell_levels(nlevels, level_ptr_host);
  Carver cv(nullptr, 0);
  carve_pcg(cv, A, L, plan, nlevels, level_ptr_host, L && nlevels == 0);
  *bytes = cv.off + 256;
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
                      void* work, size_t work_bytes, Precond* pc, Parts* parts, double** y,
                      Ell* ellA) {
  CSRAD_TRY(check_csr(A, true));
  if (A->nrows != A->ncols) return CSRAD_EINVAL;
  CSRAD_TRY(check_pc(A, kind, dinv, L, Lt, perm, nlevels, lp_host, lp_dev, rows));
  const bool fac = kind == 1, inv = kind == 3;
  size_t need = 0;
  CSRAD_TRY(csr_pcg_workspace(A, fac || inv ? L : nullptr, fac ? nlevels : 0,
                              fac ? lp_host : nullptr, &need));
  if (!work || work_bytes < need) return CSRAD_EWORKSPACE;
  Carver cv(work, work_bytes);
  PcgWs w = carve_pcg(cv, A, fac || inv ? L : nullptr, fac && ell_levels(nlevels, lp_host),
                      fac ? nlevels : 0, fac ? lp_host : nullptr, inv);
  if (!cv.ok) return CSRAD_EWORKSPACE;
  *parts = w.parts;
  *y = w.y;
  *ellA = w.ellA;
  *pc = Precond{kind, dinv, L, Lt, perm, nlevels, lp_host, lp_dev, rows, w.plan, w.invL, w.invLt};
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
  Ell ellA;
  CSRAD_TRY(pcg_common(A, kind, dinv, L, Lt, perm, nlevels, lp_host, lp_dev, rows, work,
                       work_bytes, &pc, &parts, &y, &ellA));
  const int n = A->nrows;
  if (!scal || (n > 0 && (!b || !x || !r || !z || !p))) return CSRAD_EINVAL;
  hipStream_t s = as_stream(stream);
  const int nbv = vec_blocks(n);
  hipLaunchKernelGGL(k_pcg_init, dim3(nbv), dim3(kThreads), 0, s, n, b, x, r, parts.rr);
  hipLaunchKernelGGL(k_pcg_init_scal, dim3(1), dim3(kRedThreads), 0, s, parts.rr, nbv, tol,
                     scal);
  if (n == 0) return launch_status();
  if (A->dtype == CSRAD_F32) CSRAD_TRY(build_ell_a<float>(A, ellA, s));
  else CSRAD_TRY(build_ell_a<double>(A, ellA, s));
  if (pc.kind == 1 && pc.plan.on) {
    if (L->dtype == CSRAD_F32) CSRAD_TRY(build_ell_factor<float>(n, pc, s));
    else CSRAD_TRY(build_ell_factor<double>(n, pc, s));
  }
  if (pc.kind == 3) {
    if (L->dtype == CSRAD_F32) CSRAD_TRY(build_ell_inverse<float>(n, pc, s));
    else CSRAD_TRY(build_ell_inverse<double>(n, pc, s));
  }
  CSRAD_TRY(precond_dots(n, pc, r, z, y, parts, scal, s));
  hipLaunchKernelGGL(k_pcg_start, dim3(nbv), dim3(kThreads), 0, s, n, parts, z, p, scal);
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
  Ell ellA;
  CSRAD_TRY(pcg_common(A, kind, dinv, L, Lt, perm, nlevels, lp_host, lp_dev, rows, work,
                       work_bytes, &pc, &parts, &y, &ellA));
  const int n = A->nrows;
  if (n == 0) return CSRAD_OK;
  if (!x || !r || !z || !p || !q || !scal || hist_cap < 0) return CSRAD_EINVAL;
  hipStream_t s = as_stream(stream);
  const int nbv = vec_blocks(n);
  const int nbs = spmv_blocks(n);
  if (A->dtype == CSRAD_F32) {
    hipLaunchKernelGGL((k_pcg_spmv_ell<float>), dim3(nbs), dim3(kThreads), 0, s, n, ellA.w,
                       ellA.col, static_cast<const float*>(ellA.val), A->rowptr, A->colind,
                       static_cast<const float*>(A->vals), p, q, parts.pq, scal);
  } else {
    hipLaunchKernelGGL((k_pcg_spmv_ell<double>), dim3(nbs), dim3(kThreads), 0, s, n, ellA.w,
                       ellA.col, static_cast<const double*>(ellA.val), A->rowptr, A->colind,
                       static_cast<const double*>(A->vals), p, q, parts.pq, scal);
  }
  hipLaunchKernelGGL(k_pcg_alpha, dim3(1), dim3(kRedThreads), 0, s, parts.pq, nbs, scal);
  if (kind == 3) {
    // x, r and r.r; y = L^T r with r.z = ||y||^2; rho', beta; then z = L y
    // fused with the p update
    hipLaunchKernelGGL(k_pcg_update<1>, dim3(nbv), dim3(kThreads), 0, s, n, p, q, x, r, dinv, z,
                       parts, nullptr, nullptr, scal);
    if (L->dtype == CSRAD_F32) inverse_factor_y<float>(n, pc, r, y, parts.rz, s);
    else inverse_factor_y<double>(n, pc, r, y, parts.rz, s);
    hipLaunchKernelGGL(k_pcg_beta, dim3(1), dim3(kRedThreads), 0, s, parts, nbv, scal, hist,
                       hist_cap);
    if (L->dtype == CSRAD_F32) inverse_factor_z<float>(n, pc, y, z, p, scal, s);
    else inverse_factor_z<double>(n, pc, y, z, p, scal, s);
    return launch_status();
  } else if (kind == 1) {
    const bool fuse0 = pc.plan.on && nlevels > 1;
    hipLaunchKernelGGL(k_pcg_update<1>, dim3(nbv), dim3(kThreads), 0, s, n, p, q, x, r, dinv, z,
                       parts, fuse0 ? pc.plan.d0 : nullptr, y, scal);
    CSRAD_TRY(precond_dots(n, pc, r, z, y, parts, scal, s, fuse0));
  } else if (kind == 0) {
    hipLaunchKernelGGL(k_pcg_update<0>, dim3(nbv), dim3(kThreads), 0, s, n, p, q, x, r, dinv, z,
                       parts, nullptr, nullptr, scal);
  } else {
    hipLaunchKernelGGL(k_pcg_update<2>, dim3(nbv), dim3(kThreads), 0, s, n, p, q, x, r, dinv, z,
                       parts, nullptr, nullptr, scal);
  }
  hipLaunchKernelGGL(k_pcg_beta, dim3(1), dim3(kRedThreads), 0, s, parts, nbv, scal, hist,
                     hist_cap);
  hipLaunchKernelGGL(k_pcg_p, dim3(nbv), dim3(kThreads), 0, s, n, z, p, scal);
  return launch_status();
}
