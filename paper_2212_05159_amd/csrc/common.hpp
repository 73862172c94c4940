// Shared device helpers and host-side argument checks for the csrad HIP
// library (gfx950 / CDNA4: 64-lane wavefronts, 256 CUs in 8 XCDs).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/csrad.h"

namespace csrad {

constexpr int kWave = 64;
constexpr int kXcds = 8;

// ---------------------------------------------------------------------
// XCD-aware block order.  The dispatcher hands workgroup b to XCD b % 8.
// Renumbering so that each XCD receives one contiguous range of logical
// blocks keeps neighbouring rows (and the dense rows they gather) in the
// same XCD's L2.  Bijective on [0, nblocks).  The SpMV and SpMM kernels do
// not use it: in dispatch order the eight XCDs sweep one window of rows
// together, so HBM sees one sweep instead of eight and the shared Infinity
// Cache serves the dense rows that several XCDs gather (measured 7-11%
// faster on the 3D Poisson workload).
// ---------------------------------------------------------------------
__device__ __forceinline__ int xcd_block(int b, int nblocks) {
  const int per = nblocks / kXcds, rem = nblocks % kXcds;
  const int x = b % kXcds, idx = b / kXcds;
  return x * per + (x < rem ? x : rem) + idx;
}

// ---------------------------------------------------------------------
// Row traversal order (see csrad_plan).  Natural: logical block lb owns
// rows [lb*rpb, lb*rpb + rpb).  Tiled: rows form the grid
// row = p*stride + q; a tile is `tile` consecutive q for one p and takes
// ceil(tile/rpb) blocks; tiles are ordered q-range major, p minor.
// ---------------------------------------------------------------------
struct RowOrder {
  int m, stride, tile, planes, qtiles, bpt;  // bpt: blocks per tile
};

inline RowOrder make_order(int m, int rpb, const csrad_plan* plan) {
  RowOrder o{m, 0, 0, 0, 0, 0};
  if (plan && plan->row_stride > 0 && plan->row_tile > 0) {
    o.stride = plan->row_stride;
    o.tile = plan->row_tile < o.stride ? plan->row_tile : o.stride;
    o.planes = (m + o.stride - 1) / o.stride;
    o.qtiles = (o.stride + o.tile - 1) / o.tile;
    o.bpt = (o.tile + rpb - 1) / rpb;
  }
  return o;
}

inline long long order_blocks(const RowOrder& o, int rpb) {
  if (o.stride == 0) return ((long long)o.m + rpb - 1) / rpb;
  return (long long)o.qtiles * o.planes * o.bpt;
}

// Row of group g (0 <= g < rpb) in logical block lb, or -1.
__device__ __forceinline__ int order_row(const RowOrder& o, int lb, int rpb, int g) {
  if (o.stride == 0) {
    const int r = lb * rpb + g;
    return r < o.m ? r : -1;
  }
  const int per_q = o.planes * o.bpt;
  const int qt = lb / per_q, rem = lb - qt * per_q;
  const int p = rem / o.bpt, t = rem - p * o.bpt;
  const int off = t * rpb + g;
  const int q = qt * o.tile + off;
  if (off >= o.tile || q >= o.stride) return -1;
  const long long r = (long long)p * o.stride + q;
  return r < o.m ? (int)r : -1;
}

inline int check_plan(const csrad_plan* plan, int rows) {
  if (!plan) return CSRAD_OK;
  if (plan->row_stride < 0 || plan->row_stride > (rows > 0 ? rows : 0)) return CSRAD_EINVAL;
  if (plan->row_stride > 0 && plan->row_tile <= 0) return CSRAD_EINVAL;
  return CSRAD_OK;
}

// ---------------------------------------------------------------------
// Cross-lane reductions over aligned groups of G lanes (G a power of two,
// G <= 64).  Lanes 1,2 apart combine through DPP quad permutes, 4 and 8
// apart through the DPP half-row and row mirrors, 16 apart through a
// ds_swizzle and 32 apart through a bpermute.  Every lane of a group ends
// with the same, bit-identical sum (each step adds the same two values in
// both lanes).  All lanes of the wave must execute the call.
// ---------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float swz16_f32(float v) {
  // bitmask swizzle: and 0x1f, or 0, xor 0x10 -> lane ^ 16 within 32
  return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F));
}
__device__ __forceinline__ double swz16_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_swizzle((int)(b & 0xffffffffll), 0x401F);
  const int hi = __builtin_amdgcn_ds_swizzle((int)(b >> 32), 0x401F);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

constexpr int kDppXor1 = 0xB1;      // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;      // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;
constexpr int kDppMirror = 0x140;

template <int G>
__device__ __forceinline__ float group_sum(float v) {
  if constexpr (G >= 2) v += dpp_f32<kDppXor1>(v);
  if constexpr (G >= 4) v += dpp_f32<kDppXor2>(v);
  if constexpr (G >= 8) v += dpp_f32<kDppHalfMirror>(v);
  if constexpr (G >= 16) v += dpp_f32<kDppMirror>(v);
  if constexpr (G >= 32) v += swz16_f32(v);
  if constexpr (G >= 64) v += __shfl_xor(v, 32);
  return v;
}
template <int G>
__device__ __forceinline__ double group_sum(double v) {
  if constexpr (G >= 2) v += dpp_f64<kDppXor1>(v);
  if constexpr (G >= 4) v += dpp_f64<kDppXor2>(v);
  if constexpr (G >= 8) v += dpp_f64<kDppHalfMirror>(v);
  if constexpr (G >= 16) v += dpp_f64<kDppMirror>(v);
  if constexpr (G >= 32) v += swz16_f64(v);
  if constexpr (G >= 64) v += __shfl_xor(v, 32);
  return v;
}

// Integer group sum (counts); plain bpermute butterflies.
template <int G>
__device__ __forceinline__ int group_sum_int(int v) {
#pragma unroll
  for (int o = 1; o < G; o <<= 1) v += __shfl_xor(v, o);
  return v;
}

// ---------------------------------------------------------------------
// Wave-aggregated atomic increment: lanes holding the same key combine
// into one atomicAdd on counter[key] (a few rounds of "leader takes all
// lanes with its key"; lanes left over after kAggRounds add one by one).
// Returns this lane's slot: the counter's old value plus its rank among
// the lanes that shared the atomic.  Call with the lanes that have an
// element active; every active lane must reach the call.
// ---------------------------------------------------------------------
constexpr int kAggRounds = 4;
__device__ __forceinline__ int wave_agg_add(int32_t* counter, int key) {
  const int lane = __lane_id();
  const unsigned long long lt = (1ull << lane) - 1ull;
  unsigned long long todo = __ballot(1);
  int slot = 0;
  bool done = false;
#pragma unroll
  for (int r = 0; r < kAggRounds; ++r) {
    if (!todo) break;
    const int leader = __ffsll((long long)todo) - 1;
    const int lkey = __builtin_amdgcn_readlane(key, leader);
    const unsigned long long peers = __ballot(!done && key == lkey) & todo;
    int old = 0;
    if (lane == leader) old = atomicAdd(&counter[lkey], __popcll(peers));
    old = __builtin_amdgcn_readlane(old, leader);
    if ((peers >> lane) & 1ull) {
      slot = old + __popcll(peers & lt);
      done = true;
    }
    todo &= ~peers;
  }
  if (!done) slot = atomicAdd(&counter[key], 1);
  return slot;
}

// Wave-aggregated count: like wave_agg_add, but nothing is returned, so
// the atomics need not be waited for (non-returning atomics issue and go)
// and the aggregation rounds are only ballots and shuffles.
__device__ __forceinline__ void wave_agg_count(int32_t* counter, int key) {
  unsigned long long todo = __ballot(1);
  bool done = false;
#pragma unroll
  for (int r = 0; r < kAggRounds; ++r) {
    if (!todo) break;
    const int leader = __ffsll((long long)todo) - 1;
    const int lkey = __builtin_amdgcn_readlane(key, leader);
    const unsigned long long peers = __ballot(!done && key == lkey) & todo;
    if (__lane_id() == leader) atomicAdd(&counter[lkey], __popcll(peers));
    if ((peers >> __lane_id()) & 1ull) done = true;
    todo &= ~peers;
  }
  if (!done) atomicAdd(&counter[key], 1);
}

// Wave-aggregated append to one counter: the lanes with pred set take
// consecutive slots (in lane order) from a single atomicAdd by the first
// of them.  Every lane of the wave must reach the call.  Returns the slot
// (meaningful where pred is set).
__device__ __forceinline__ int wave_append(int32_t* counter, bool pred) {
  const unsigned long long mask = __ballot(pred);
  if (!mask) return 0;
  const int lane = __lane_id();
  const int leader = __ffsll((long long)mask) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(counter, __popcll(mask));
  base = __builtin_amdgcn_readlane(base, leader);
  return base + __popcll(mask & ((1ull << lane) - 1ull));
}

// Maximum of v over the wave (every lane must reach the call).
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}

// Eight sums over one 16-lane DPP row, scattered: every lane holds d[0..7];
// lanes 2u and 2u+1 return the row's sum of d[u].  Each level pairs lanes
// that differ in one bit of u (row mirror: lane bit 3, half-row mirror:
// bit 2, quad swap: bit 1), keeps the half of its values that its bit
// selects and adds the partner's copies of them; a swap of neighbours
// completes the sums.  8 cross-lane moves instead of 32, and the partial
// sums die as they are combined.
template <int CTRL>
__device__ __forceinline__ float dpp_any(float v) {
  return dpp_f32<CTRL>(v);
}
template <int CTRL>
__device__ __forceinline__ double dpp_any(double v) {
  return dpp_f64<CTRL>(v);
}
template <typename T>
__device__ __forceinline__ T row_sum_scatter8(const T (&d)[8], int lr) {
  const bool b3 = lr & 8, b2 = lr & 4, b1 = lr & 2;
  T e[4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
    e[q] = (b3 ? d[4 + q] : d[q]) + dpp_any<kDppMirror>(b3 ? d[q] : d[4 + q]);
  T f[2];
#pragma unroll
  for (int q = 0; q < 2; ++q)
    f[q] = (b2 ? e[2 + q] : e[q]) + dpp_any<kDppHalfMirror>(b2 ? e[q] : e[2 + q]);
  const T h = (b1 ? f[1] : f[0]) + dpp_any<kDppXor2>(b1 ? f[0] : f[1]);
  return h + dpp_any<kDppXor1>(h);
}

// ---------------------------------------------------------------------
// Vector types for 16-byte dense-row accesses.
// ---------------------------------------------------------------------
template <typename T, int VW>
struct alignas(sizeof(T) * VW) Vec {
  T v[VW];
};

template <typename T, int VW>
__device__ __forceinline__ Vec<T, VW> load_vec(const T* p) {
  return *reinterpret_cast<const Vec<T, VW>*>(p);
}
template <typename T, int VW>
__device__ __forceinline__ void store_vec(T* p, const Vec<T, VW>& x) {
  *reinterpret_cast<Vec<T, VW>*>(p) = x;
}

// Streaming store of a whole output row slice that nothing in the kernel
// reads again: kept out of the caches' way of the reused rows.
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
template <typename T, int VW>
__device__ __forceinline__ void store_vec_stream(T* p, const Vec<T, VW>& x) {
  if constexpr (sizeof(T) * VW == 16) {
    u32x4 u;
    __builtin_memcpy(&u, &x, 16);
    __builtin_nontemporal_store(u, reinterpret_cast<u32x4*>(p));
  } else if constexpr (sizeof(T) * VW == 8) {
    u32x2 u;
    __builtin_memcpy(&u, &x, 8);
    __builtin_nontemporal_store(u, reinterpret_cast<u32x2*>(p));
  } else {
    store_vec<T, VW>(p, x);
  }
}

// Streaming loads for data read exactly once (CSR arrays): keep them from
// evicting reused dense rows.
template <typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
  return __builtin_nontemporal_load(p);
}

// ---------------------------------------------------------------------
// Host-side checks.
// ---------------------------------------------------------------------
inline int check_csr(const csrad_csr* A, bool need_vals) {
  if (!A) return CSRAD_EINVAL;
  if (A->nrows < 0 || A->ncols < 0 || A->nnz < 0) return CSRAD_EINVAL;
  if (!A->rowptr) return CSRAD_EINVAL;
  if (A->nnz > 0 && !A->colind) return CSRAD_EINVAL;
  if (need_vals && A->nnz > 0 && !A->vals) return CSRAD_EINVAL;
  if (A->dtype != CSRAD_F32 && A->dtype != CSRAD_F64) return CSRAD_EDTYPE;
  return CSRAD_OK;
}

inline size_t dtype_size(int dtype) { return dtype == CSRAD_F64 ? 8 : 4; }

inline int launch_status() {
  return hipGetLastError() == hipSuccess ? CSRAD_OK : CSRAD_EHIP;
}

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Carves aligned sub-buffers out of a caller workspace.
// Constructed with base == nullptr it only measures (off = bytes needed).
struct Carver {
  char* base;
  size_t cap, off = 0;
  bool ok = true;
  Carver(void* b, size_t c) : base(static_cast<char*>(b)), cap(c) {}
  template <typename T>
  T* take(size_t count) {
    off = align_up(off, 256);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += sizeof(T) * (count ? count : 1);
    if (base && off > cap) ok = false;
    return p;
  }
};

#define CSRAD_TRY(expr)            \
  do {                             \
    int _st = (expr);              \
    if (_st != CSRAD_OK) return _st; \
  } while (0)

}  // namespace csrad
