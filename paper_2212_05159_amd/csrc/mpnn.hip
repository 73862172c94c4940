// Kernels of the learned preconditioner's message-passing network: the
// dense layers on bf16 matrix cores (the only MFMA use in the library), the
// input preparation on the scaled matrix, and the readout to the values of
// a lower-triangular factor on tril(A)'s pattern.
//
// Dense layer: Y = act([X1 X2] W + b), X1 (n x K1), X2 (n x K2, optional),
// W ((K1+K2) x 32), b (32), act = relu or identity.  One wavefront computes
// a 32-row tile with v_mfma_f32_32x32x16_bf16: operands are rounded to
// bf16, accumulation is float32.  Backward: G = dY * act'(Y);
// dX = G W^T (MFMA), dW = [X1 X2]^T G and db = sum of G rows (MFMA per
// tile, per-block partials, then a fixed-order reduction: deterministic).
#include "internal.hpp"

namespace csrad {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kOut = 32;       // hidden width
constexpr int kTile = 32;      // rows per wavefront
constexpr int kWaves = 4;      // wavefronts per block
constexpr int kMaxK = 64;      // K1 + K2

// Row of accumulator register r for lane l in a 32x32 MFMA result.
__device__ __forceinline__ int acc_row(int r, int l) { return 8 * (r / 4) + 4 * (l / 32) + (r % 4); }

__device__ __forceinline__ float load_x(const float* __restrict__ X1, int K1, long long ld1,
                                        const float* __restrict__ X2, long long ld2, int row,
                                        int k, int n) {
  if (row >= n) return 0.f;
  return k < K1 ? X1[(long long)row * ld1 + k] : X2[(long long)row * ld2 + (k - K1)];
}

// Y = act(X W + b).  Grid: ceil(n / (32 * 4)) blocks of 256 threads.
__global__ __launch_bounds__(256) void k_dense_fwd(int n, int K1, const float* __restrict__ X1,
                                                   long long ld1, int K2,
                                                   const float* __restrict__ X2, long long ld2,
                                                   const float* __restrict__ W,
                                                   const float* __restrict__ b, int relu,
                                                   float* __restrict__ Y) {
  __shared__ __bf16 Ws[kMaxK * kOut];
  const int K = K1 + K2;
  for (int i = threadIdx.x; i < K * kOut; i += 256) Ws[i] = (__bf16)W[i];
  __syncthreads();
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int row0 = (blockIdx.x * kWaves + wave) * kTile;
  if (row0 >= n) return;
  f32x16 acc = {};
  const int m = lane % 32, kh = 8 * (lane / 32);
  for (int k0 = 0; k0 < K; k0 += 16) {
    bf16x8 a, bb;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = k0 + kh + u;
      a[u] = (__bf16)(k < K ? load_x(X1, K1, ld1, X2, ld2, row0 + m, k, n) : 0.f);
      bb[u] = k < K ? Ws[k * kOut + m] : (__bf16)0.f;
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bb, acc, 0, 0, 0);
  }
  const float bias = b ? b[m] : 0.f;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = row0 + acc_row(r, lane);
    if (row < n) {
      float v = acc[r] + bias;
      if (relu) v = v > 0.f ? v : 0.f;
      Y[(long long)row * kOut + m] = v;
    }
  }
}

// dX1 / dX2 = G W^T with G = dY * act'(Y).
__global__ __launch_bounds__(256) void k_dense_bwd_x(int n, int K1, int K2,
                                                     const float* __restrict__ W,
                                                     const float* __restrict__ Y,
                                                     const float* __restrict__ dY, int relu,
                                                     float* __restrict__ dX1, long long ld1,
                                                     float* __restrict__ dX2, long long ld2) {
  __shared__ __bf16 Wt[kOut * kMaxK];  // Wt[c][k] = W[k][c]
  const int K = K1 + K2;
  for (int i = threadIdx.x; i < K * kOut; i += 256) {
    const int k = i / kOut, c = i % kOut;
    Wt[c * kMaxK + k] = (__bf16)W[i];
  }
  __syncthreads();
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int row0 = (blockIdx.x * kWaves + wave) * kTile;
  if (row0 >= n) return;
  const int m = lane % 32, kh = 8 * (lane / 32);
  // A operand (G rows x output columns): two k-steps over the 32 outputs
  bf16x8 ga[2];
  const int grow = row0 + m;
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int c = 16 * s + kh + u;
      float g = 0.f;
      if (grow < n) {
        g = dY[(long long)grow * kOut + c];
        if (relu && !(Y[(long long)grow * kOut + c] > 0.f)) g = 0.f;
      }
      ga[s][u] = (__bf16)g;
    }
  for (int j0 = 0; j0 < K; j0 += 32) {  // 32 input columns per output tile
    f32x16 acc = {};
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      bf16x8 bb;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int c = 16 * s + kh + u;
        const int j = j0 + m;
        bb[u] = j < K ? Wt[c * kMaxK + j] : (__bf16)0.f;
      }
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ga[s], bb, acc, 0, 0, 0);
    }
    const int j = j0 + m;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = row0 + acc_row(r, lane);
      if (row < n && j < K) {
        if (j < K1) {
          if (dX1) dX1[(long long)row * ld1 + j] = acc[r];
        } else if (dX2) {
          dX2[(long long)row * ld2 + (j - K1)] = acc[r];
        }
      }
    }
  }
}

// Per-block partial dW (K x 32) and db (32): each wave takes 32-row tiles,
// dW_tile = X_tile^T G_tile on the matrix cores (k runs over rows).
__global__ __launch_bounds__(256) void k_dense_bwd_w(int n, int K1, const float* __restrict__ X1,
                                                     long long ld1, int K2,
                                                     const float* __restrict__ X2, long long ld2,
                                                     const float* __restrict__ Y,
                                                     const float* __restrict__ dY, int relu,
                                                     float* __restrict__ part) {
  __shared__ float red[kWaves][kMaxK * kOut + kOut];
  const int K = K1 + K2;
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int m = lane % 32, kh = 8 * (lane / 32);
  f32x16 acc[2] = {};
  float dbs = 0.f;
  const int tiles = (n + kTile - 1) / kTile;
  for (int t = blockIdx.x * kWaves + wave; t < tiles; t += gridDim.x * kWaves) {
    const int row0 = t * kTile;
    for (int rs = 0; rs < kTile; rs += 16) {  // k-steps over 16 rows
      bf16x8 gb;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int row = row0 + rs + kh + u;
        float g = 0.f;
        if (row < n) {
          g = dY[(long long)row * kOut + m];
          if (relu && !(Y[(long long)row * kOut + m] > 0.f)) g = 0.f;
        }
        gb[u] = (__bf16)g;
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {  // input-dimension halves of 32
        bf16x8 xa;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int row = row0 + rs + kh + u;
          const int j = 32 * h + m;
          xa[u] = (__bf16)(j < K ? load_x(X1, K1, ld1, X2, ld2, row, j, n) : 0.f);
        }
        acc[h] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa, gb, acc[h], 0, 0, 0);
      }
    }
    // db in float32 from the unrounded gradient: lanes 0..31 own a column
    if (lane < 32)
      for (int rr = 0; rr < kTile; ++rr) {
        const int row = row0 + rr;
        if (row < n) {
          float g = dY[(long long)row * kOut + m];
          if (relu && !(Y[(long long)row * kOut + m] > 0.f)) g = 0.f;
          dbs += g;
        }
      }
  }
  // dW[j][c]: acc[h] register r holds row j = 32h + acc_row(r), column c = m
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int j = 32 * h + acc_row(r, lane);
      if (j < K) red[wave][j * kOut + m] = acc[h][r];
    }
  if (lane < 32) red[wave][K * kOut + m] = dbs;
  __syncthreads();
  for (int i = threadIdx.x; i < K * kOut + kOut; i += 256) {
    float s = 0.f;
    for (int w = 0; w < kWaves; ++w) s += red[w][i];
    part[(long long)blockIdx.x * (kMaxK * kOut + kOut) + i] = s;
  }
}

__global__ void k_dense_reduce(int nb, int K, const float* __restrict__ part,
                               float* __restrict__ dW, float* __restrict__ db) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K * kOut + kOut) return;
  float s = 0.f;
  for (int bidx = 0; bidx < nb; ++bidx) s += part[(long long)bidx * (kMaxK * kOut + kOut) + i];
  if (i < K * kOut) {
    if (dW) dW[i] = s;
  } else if (db) {
    db[i - K * kOut] = s;
  }
}

constexpr int kBwdBlocks = 512;

// Scaled matrix and node inputs.  For row i with d_i = A_ii:
//   ahat[e] = A_e / sqrt(d_i d_j), dsqrt[i] = sqrt(d_i),
//   X0[i] = [1, sum_{j!=i} |ahat_ij|, sum_{j!=i} ahat_ij, (deg_i - 1)/8,
//            sum_{j<i} ahat_ij, sum_{j<i} |ahat_ij|, #{j<i}/8,
//            sum_{j>i} ahat_ij, sum_{j>i} |ahat_ij|, #{j>i}/8, 0 ...] (16 wide);
//   the lower/upper split tells the network where a node sits in the
//   solve order, which the factor depends on.
//   ahatL[t] for the entries of tril(A) (the first entries of each row).
__global__ void k_mpnn_prep(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                            const float* __restrict__ v, const int32_t* __restrict__ rpL,
                            float* __restrict__ ahat, float* __restrict__ ahatL,
                            float* __restrict__ dsqrt, float* __restrict__ X0) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  // diagonal of every row this row touches is needed: read it on the fly
  auto diag = [&](int r) {
    float d = 0.f;
    for (int e = rp[r]; e < rp[r + 1]; ++e)
      if (ci[e] == r) d = v[e];
    return d;
  };
  const float di = diag(i);
  const float si = sqrtf(di > 0.f ? di : 1.f);
  dsqrt[i] = si;
  float s1 = 0.f, s2 = 0.f, lo = 0.f, loa = 0.f, up = 0.f, upa = 0.f;
  int nlo = 0, nup = 0;
  const int e0 = rp[i], e1 = rp[i + 1];
  for (int e = e0; e < e1; ++e) {
    const int j = ci[e];
    const float dj = j == i ? di : diag(j);
    const float a = v[e] / (si * sqrtf(dj > 0.f ? dj : 1.f));
    ahat[e] = a;
    if (j != i) {
      s1 += fabsf(a);
      s2 += a;
    }
    if (j < i) {
      lo += a;
      loa += fabsf(a);
      ++nlo;
    } else if (j > i) {
      up += a;
      upa += fabsf(a);
      ++nup;
    }
  }
  const int lcount = rpL[i + 1] - rpL[i];
  for (int t = 0; t < lcount; ++t) ahatL[rpL[i] + t] = ahat[e0 + t];
  float* x = X0 + (long long)i * 16;
  x[0] = 1.f;
  x[1] = s1;
  x[2] = s2;
  x[3] = (float)(e1 - e0 - 1) / 8.f;
  x[4] = lo;
  x[5] = loa;
  x[6] = (float)nlo / 8.f;
  x[7] = up;
  x[8] = upa;
  x[9] = (float)nup / 8.f;
  for (int k = 10; k < 16; ++k) x[k] = 0.f;
}

__device__ __forceinline__ float softplus(float x) { return x > 20.f ? x : log1pf(expf(x)); }
__device__ __forceinline__ float sigmoid(float x) { return 1.f / (1.f + expf(-x)); }

// L[t] for (i, j) in tril(A):  sqrt(d_i) * (j < i ? ahat (1 + t) : softplus(t + c) + delta)
__global__ void k_mpnn_readout(int n, const int32_t* __restrict__ rpL,
                               const int32_t* __restrict__ ciL, const float* __restrict__ ahatL,
                               const float* __restrict__ dsqrt, const float* __restrict__ t,
                               float c, float delta, float* __restrict__ Lv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float s = dsqrt[i];
  for (int e = rpL[i]; e < rpL[i + 1]; ++e) {
    const int j = ciL[e];
    Lv[e] = s * (j < i ? ahatL[e] * (1.f + t[e]) : softplus(t[e] + c) + delta);
  }
}

__global__ void k_mpnn_readout_bwd(int n, const int32_t* __restrict__ rpL,
                                   const int32_t* __restrict__ ciL,
                                   const float* __restrict__ ahatL,
                                   const float* __restrict__ dsqrt, const float* __restrict__ t,
                                   float c, const float* __restrict__ gL, float* __restrict__ gt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float s = dsqrt[i];
  for (int e = rpL[i]; e < rpL[i + 1]; ++e) {
    const int j = ciL[e];
    gt[e] = gL[e] * s * (j < i ? ahatL[e] : sigmoid(t[e] + c));
  }
}

}  // namespace
}  // namespace csrad

using namespace csrad;

extern "C" int csr_dense_workspace(int32_t n, size_t* bytes) {
  if (!bytes || n < 0) return CSRAD_EINVAL;
  *bytes = sizeof(float) * (size_t)kBwdBlocks * (kMaxK * kOut + kOut) + 256;
  return CSRAD_OK;
}

extern "C" int csr_dense_fwd(int32_t n, int32_t K1, const float* X1, int64_t ld1, int32_t K2,
                             const float* X2, int64_t ld2, const float* W, const float* b,
                             int32_t relu, float* Y, void* stream) {
  if (n < 0 || K1 < 1 || K2 < 0 || K1 + K2 > kMaxK || !W || (n > 0 && (!X1 || !Y)) ||
      (K2 > 0 && !X2) || ld1 < K1 || (K2 > 0 && ld2 < K2))
    return CSRAD_EINVAL;
  if (n == 0) return CSRAD_OK;
  const int blocks = (n + kTile * kWaves - 1) / (kTile * kWaves);
  hipLaunchKernelGGL(k_dense_fwd, dim3(blocks), dim3(256), 0, as_stream(stream), n, K1, X1, ld1,
                     K2, X2, ld2, W, b, relu, Y);
  return launch_status();
}

extern "C" int csr_dense_bwd(int32_t n, int32_t K1, const float* X1, int64_t ld1, int32_t K2,
                             const float* X2, int64_t ld2, const float* W, const float* Y,
                             const float* dY, int32_t relu, float* dX1, float* dX2, float* dW,
                             float* db, void* work, size_t work_bytes, void* stream) {
  if (n < 0 || K1 < 1 || K2 < 0 || K1 + K2 > kMaxK || !W || (n > 0 && (!X1 || !Y || !dY)) ||
      (K2 > 0 && !X2) || ld1 < K1 || (K2 > 0 && ld2 < K2))
    return CSRAD_EINVAL;
  size_t need = 0;
  CSRAD_TRY(csr_dense_workspace(n, &need));
  if ((dW || db) && (!work || work_bytes < need)) return CSRAD_EWORKSPACE;
  hipStream_t s = as_stream(stream);
  const int K = K1 + K2;
  if (n > 0 && (dX1 || dX2)) {
    const int blocks = (n + kTile * kWaves - 1) / (kTile * kWaves);
    hipLaunchKernelGGL(k_dense_bwd_x, dim3(blocks), dim3(256), 0, s, n, K1, K2, W, Y, dY, relu,
                       dX1, ld1, dX2, ld2);
  }
  if (dW || db) {
    float* part = static_cast<float*>(work);
    if (n > 0) {
      hipLaunchKernelGGL(k_dense_bwd_w, dim3(kBwdBlocks), dim3(256), 0, s, n, K1, X1, ld1, K2, X2,
                         ld2, Y, dY, relu, part);
    } else {
      CSRAD_TRY(fill_bytes_zero(part, sizeof(float) * (size_t)kBwdBlocks * (kMaxK * kOut + kOut),
                                s));
    }
    hipLaunchKernelGGL(k_dense_reduce, dim3((K * kOut + kOut + 255) / 256), dim3(256), 0, s,
                       kBwdBlocks, K, part, dW, db);
  }
  return launch_status();
}

extern "C" int csr_mpnn_prep(const csrad_csr* A, const csrad_csr* Lpat, float* ahat, float* ahatL,
                             float* dsqrt, float* X0, void* stream) {
  CSRAD_TRY(check_csr(A, true));
  CSRAD_TRY(check_csr(Lpat, false));
  if (A->dtype != CSRAD_F32) return CSRAD_EDTYPE;
  if (A->nrows != A->ncols || Lpat->nrows != A->nrows) return CSRAD_EINVAL;
  const int n = A->nrows;
  if (n == 0) return CSRAD_OK;
  if (!ahat || !dsqrt || !X0 || (Lpat->nnz > 0 && !ahatL)) return CSRAD_EINVAL;
  hipLaunchKernelGGL(k_mpnn_prep, dim3((n + 255) / 256), dim3(256), 0, as_stream(stream), n,
                     A->rowptr, A->colind, static_cast<const float*>(A->vals), Lpat->rowptr, ahat,
                     ahatL, dsqrt, X0);
  return launch_status();
}

extern "C" int csr_mpnn_readout(const csrad_csr* Lpat, const float* ahatL, const float* dsqrt,
                                const float* t, float c, float delta, float* Lv, void* stream) {
  CSRAD_TRY(check_csr(Lpat, false));
  const int n = Lpat->nrows;
  if (n == 0) return CSRAD_OK;
  if (!ahatL || !dsqrt || !t || !Lv) return CSRAD_EINVAL;
  hipLaunchKernelGGL(k_mpnn_readout, dim3((n + 255) / 256), dim3(256), 0, as_stream(stream), n,
                     Lpat->rowptr, Lpat->colind, ahatL, dsqrt, t, c, delta, Lv);
  return launch_status();
}

extern "C" int csr_mpnn_readout_bwd(const csrad_csr* Lpat, const float* ahatL, const float* dsqrt,
                                    const float* t, float c, const float* gL, float* gt,
                                    void* stream) {
  CSRAD_TRY(check_csr(Lpat, false));
  const int n = Lpat->nrows;
  if (n == 0) return CSRAD_OK;
  if (!ahatL || !dsqrt || !t || !gL || !gt) return CSRAD_EINVAL;
  hipLaunchKernelGGL(k_mpnn_readout_bwd, dim3((n + 255) / 256), dim3(256), 0, as_stream(stream), n,
                     Lpat->rowptr, Lpat->colind, ahatL, dsqrt, t, c, gL, gt);
  return launch_status();
}
