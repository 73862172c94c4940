// Status strings and the CSR pattern validator.
#include "internal.hpp"

namespace csrad {
namespace {

// One thread per row.  Reads are clamped to [0, nnz) so a malformed
// rowptr cannot send the check out of bounds.
__global__ __launch_bounds__(256) void k_validate(int m, int n, int nnz,
                                                  const int32_t* __restrict__ rp,
                                                  const int32_t* __restrict__ ci,
                                                  int32_t* __restrict__ bad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int a = rp[i], b = rp[i + 1];
  bool ok = a >= 0 && b >= a && b <= nnz;
  if (i == 0) ok = ok && a == 0;
  if (i == m - 1) ok = ok && b == nnz;
  if (ok) {
    int prev = -1;
    for (int e = a; e < b; ++e) {
      const int c = ci[e];
      if (c <= prev || c >= n) {
        ok = false;
        break;
      }
      prev = c;
    }
  }
  if (!ok) atomicMin(bad, i);
}

// stats[0] longest row, [1] max |col - row|, [2] non-empty rows.  Each
// block strides over rows, reduces its wave results in LDS and applies
// three atomics, so few atomics meet on the same three addresses.
constexpr int kStatsBlocksMax = 1024;

__global__ __launch_bounds__(256) void k_stats(int m, const int32_t* __restrict__ rp,
                                               const int32_t* __restrict__ ci,
                                               int32_t* __restrict__ st) {
  __shared__ int sm[3][256 / kWave];
  int longest = 0, bw = 0, nonempty = 0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < m; i += gridDim.x * 256) {
    const int a = rp[i], b = rp[i + 1];
    if (b > a) {
      longest = max(longest, b - a);
      bw = max(bw, max(abs(ci[a] - i), abs(ci[b - 1] - i)));
      ++nonempty;
    }
  }
  longest = wave_max(longest);
  bw = wave_max(bw);
  nonempty = group_sum_int<kWave>(nonempty);
  const int w = threadIdx.x / kWave;
  if (threadIdx.x % kWave == 0) {
    sm[0][w] = longest;
    sm[1][w] = bw;
    sm[2][w] = nonempty;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < 256 / kWave; ++k) {
      longest = max(longest, sm[0][k]);
      bw = max(bw, sm[1][k]);
      nonempty += sm[2][k];
    }
    atomicMax(&st[0], longest);
    atomicMax(&st[1], bw);
    atomicAdd(&st[2], nonempty);
  }
}

}  // namespace
}  // namespace csrad

using namespace csrad;

extern "C" int csr_pattern_stats(const csrad_csr* A, int64_t* stats_host, void* work,
                                 size_t work_bytes, void* stream) {
  if (!A || !stats_host) return CSRAD_EINVAL;
  if (A->nrows < 0 || A->ncols < 0 || A->nnz < 0 || !A->rowptr) return CSRAD_EINVAL;
  if (A->nnz > 0 && !A->colind) return CSRAD_EINVAL;
  if (!work || work_bytes < 4 * sizeof(int32_t)) return CSRAD_EWORKSPACE;
  hipStream_t s = as_stream(stream);
  int32_t* st = static_cast<int32_t*>(work);
  CSRAD_TRY(fill_i32(st, 4, 0, s));
  if (A->nrows > 0)
    hipLaunchKernelGGL(k_stats, dim3(std::min((A->nrows + 255) / 256, kStatsBlocksMax)), dim3(256),
                       0, s, A->nrows, A->rowptr, A->colind, st);
  CSRAD_TRY(launch_status());
  int32_t h[4];
  if (hipMemcpyAsync(h, st, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess) return CSRAD_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return CSRAD_EHIP;
  stats_host[0] = h[0];
  stats_host[1] = h[1];
  stats_host[2] = h[2];
  stats_host[3] = A->nnz;
  return CSRAD_OK;
}

extern "C" const char* csr_status_string(int status) {
  switch (status) {
    case CSRAD_OK: return "ok";
    case CSRAD_EINVAL: return "invalid argument (null pointer, shape or size)";
    case CSRAD_EDTYPE: return "unsupported or mismatched value type";
    case CSRAD_EPATTERN: return "malformed CSR pattern";
    case CSRAD_ESINGULAR: return "triangular matrix has a row without a stored diagonal";
    case CSRAD_EWORKSPACE: return "workspace missing or too small";
    case CSRAD_EHIP: return "HIP launch or runtime error";
    case CSRAD_EOVERFLOW: return "result exceeds int32 indexing";
    default: return "unknown status";
  }
}

extern "C" int csr_validate(const csrad_csr* A, int32_t* first_bad_row_host, void* work,
                            size_t work_bytes, void* stream) {
  if (!A || !first_bad_row_host) return CSRAD_EINVAL;
  if (A->nrows < 0 || A->ncols < 0 || A->nnz < 0 || !A->rowptr) return CSRAD_EINVAL;
  if (A->nnz > 0 && !A->colind) return CSRAD_EINVAL;
  if (!work || work_bytes < sizeof(int32_t)) return CSRAD_EWORKSPACE;
  hipStream_t s = as_stream(stream);
  int32_t* bad = static_cast<int32_t*>(work);
  CSRAD_TRY(fill_i32(bad, 1, INT32_MAX, s));
  const int m = A->nrows;
  if (m > 0)
    hipLaunchKernelGGL(k_validate, dim3((m + 255) / 256), dim3(256), 0, s, m, A->ncols, A->nnz,
                       A->rowptr, A->colind, bad);
  CSRAD_TRY(launch_status());
  int32_t host = INT32_MAX;
  if (hipMemcpyAsync(&host, bad, sizeof(host), hipMemcpyDeviceToHost, s) != hipSuccess)
    return CSRAD_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return CSRAD_EHIP;
  *first_bad_row_host = host == INT32_MAX ? -1 : host;
  return host == INT32_MAX ? CSRAD_OK : CSRAD_EPATTERN;
}
