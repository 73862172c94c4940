// Device-wide exclusive prefix sum of int32 counts (tile sums, then
// tile-local scans with the tile offset; with up to kFusedTiles tiles every
// tile adds up the sums before it itself, otherwise one block scans the tile
// sums in between) and small fill helpers.  Used for transpose row pointers,
// SpGEMM row pointers and level pointers.
#include "internal.hpp"

namespace csrad {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;
constexpr int kFusedTiles = 2048;

// Inclusive block scan of one value per thread (256 threads = 4 waves).
template <typename T>
__device__ T block_inclusive_scan(T v, T* smem /* >= 4 */, T* total) {
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    T u = __shfl_up(v, o);
    if (lane >= o) v += u;
  }
  if (lane == kWave - 1) smem[wid] = v;
  __syncthreads();
  T off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kScanThreads / kWave; ++w) {
    if (w < wid) off += smem[w];
    tot += smem[w];
  }
  __syncthreads();
  *total = tot;
  return v + off;
}

__global__ __launch_bounds__(kScanThreads) void k_tile_sums(const int32_t* __restrict__ in, int n,
                                                            long long* __restrict__ part,
                                                            const int32_t* __restrict__ skip) {
  __shared__ long long sm[4];
  if (skip && *skip) return;
  const long long base = (long long)blockIdx.x * kScanTile;
  long long s = 0;
#pragma unroll
  for (int t = 0; t < kScanItems; ++t) {
    long long i = base + (long long)t * kScanThreads + threadIdx.x;
    if (i < n) s += in[i];
  }
  long long tot;
  block_inclusive_scan<long long>(s, sm, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// One block scans the tile sums in place (exclusive) and writes the total.
__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(long long* __restrict__ part, int ntiles,
                                                             long long* __restrict__ total,
                                                             const int32_t* __restrict__ skip) {
  __shared__ long long sm[4];
  if (skip && *skip) return;
  long long carry = 0;
  for (int base = 0; base < ntiles; base += kScanThreads) {
    const int i = base + threadIdx.x;
    long long v = i < ntiles ? part[i] : 0;
    long long tot;
    long long inc = block_inclusive_scan<long long>(v, sm, &tot);
    if (i < ntiles) part[i] = carry + inc - v;
    carry += tot;
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(kScanThreads) void k_tile_scan(const int32_t* __restrict__ in, int n,
                                                            const long long* __restrict__ part,
                                                            const long long* __restrict__ total,
                                                            int32_t* __restrict__ out,
                                                            const int32_t* __restrict__ skip) {
  __shared__ long long sm[4];
  if (skip && *skip) return;
  const long long base = (long long)blockIdx.x * kScanTile + (long long)threadIdx.x * kScanItems;
  long long v[kScanItems];
  long long s = 0;
#pragma unroll
  for (int t = 0; t < kScanItems; ++t) {
    long long i = base + t;
    v[t] = i < n ? in[i] : 0;
    s += v[t];
  }
  long long tot;
  long long inc = block_inclusive_scan<long long>(s, sm, &tot);
  long long run = part[blockIdx.x] + inc - s;
#pragma unroll
  for (int t = 0; t < kScanItems; ++t) {
    long long i = base + t;
    if (i < n) out[i] = (int32_t)run;
    run += v[t];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = (int32_t)*total;
}

// Tile-local scan whose offset this block forms itself from the sums of the
// tiles before it (fixed order, exact in 64 bits); the last tile writes the
// total and out[n].
__global__ __launch_bounds__(kScanThreads) void k_tile_scan_fused(const int32_t* __restrict__ in,
                                                                  int n,
                                                                  const long long* __restrict__ part,
                                                                  int ntiles,
                                                                  long long* __restrict__ total,
                                                                  int32_t* __restrict__ out,
                                                                  const int32_t* __restrict__ skip) {
  __shared__ long long sm[4];
  if (skip && *skip) return;
  long long before = 0;
  for (int t = threadIdx.x; t < (int)blockIdx.x; t += kScanThreads) before += part[t];
  long long pre_tot;
  block_inclusive_scan<long long>(before, sm, &pre_tot);  // pre_tot: sum of earlier tiles
  __syncthreads();  // sm is reused below
  const long long base = (long long)blockIdx.x * kScanTile + (long long)threadIdx.x * kScanItems;
  long long v[kScanItems];
  long long s = 0;
#pragma unroll
  for (int t = 0; t < kScanItems; ++t) {
    long long i = base + t;
    v[t] = i < n ? in[i] : 0;
    s += v[t];
  }
  long long tot;
  long long inc = block_inclusive_scan<long long>(s, sm, &tot);
  long long run = pre_tot + inc - s;
#pragma unroll
  for (int t = 0; t < kScanItems; ++t) {
    long long i = base + t;
    if (i < n) out[i] = (int32_t)run;
    run += v[t];
  }
  if ((int)blockIdx.x == ntiles - 1 && threadIdx.x == 0) {
    *total = pre_tot + tot;
    out[n] = (int32_t)(pre_tot + tot);
  }
}

__global__ void k_fill_i32(int32_t* p, long long n, int32_t value) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = value;
}

__global__ void k_zero_bytes(unsigned char* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

}  // namespace

size_t scan_workspace(int n) {
  const size_t ntiles = (size_t)(n + kScanTile - 1) / kScanTile + 1;
  return align_up(sizeof(long long) * (ntiles + 1), 256) + 256;
}

int scan_exclusive(const int32_t* in, int32_t* out, int n, long long* total_dev, void* work,
                   size_t bytes, hipStream_t s, const int32_t* skip) {
  if (n < 0) return CSRAD_EINVAL;
  const int ntiles = (n + kScanTile - 1) / kScanTile;
  if (bytes < scan_workspace(n) || !work) return CSRAD_EWORKSPACE;
  long long* part = reinterpret_cast<long long*>(work);
  if (ntiles > 0) {
    hipLaunchKernelGGL(k_tile_sums, dim3(ntiles), dim3(kScanThreads), 0, s, in, n, part, skip);
  }
  if (ntiles > 0 && ntiles <= kFusedTiles) {
    hipLaunchKernelGGL(k_tile_scan_fused, dim3(ntiles), dim3(kScanThreads), 0, s, in, n, part,
                       ntiles, total_dev, out, skip);
    return launch_status();
  }
  hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kScanThreads), 0, s, part, ntiles, total_dev,
                     skip);
  hipLaunchKernelGGL(k_tile_scan, dim3(ntiles > 0 ? ntiles : 1), dim3(kScanThreads), 0, s, in, n,
                     part, total_dev, out, skip);
  return launch_status();
}

int fill_i32(int32_t* p, long long n, int32_t value, hipStream_t s) {
  if (n <= 0) return CSRAD_OK;
  long long blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)blocks), dim3(256), 0, s, p, n, value);
  return launch_status();
}

int fill_bytes_zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return CSRAD_OK;
  size_t blocks = (bytes + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_zero_bytes, dim3((unsigned)blocks), dim3(256), 0, s,
                     static_cast<unsigned char*>(p), bytes);
  return launch_status();
}

}  // namespace csrad
