// Stable CSR transpose (the sparse transpose that the SpDMM backward of
// Section 3.1.3 is built on; every A^T product here gathers over it).
//
// A square pattern is first tried as structurally symmetric: entry (i, j)
// looks up (j, i) in row j by binary search; when every entry finds its
// mirror, the transpose pattern is the pattern itself and perm maps the
// mirror positions (a device flag records the outcome, and the general
// kernels below skip or copy accordingly, so the call stays asynchronous).
// General case, in column blocks of CB = 2^k columns (CB and the block
// count chosen from n and nnz): the entries are first moved into their
// column block's range of the output (per-workgroup LDS histograms over the
// blocks, one device atomic per block a workgroup touches, not one per
// entry), then one workgroup per column block counts its columns in LDS,
// writes their row pointers, groups the block's entries by column (in LDS
// when they fit) and sorts each column by source row.  Patterns with more
// than 2^25 columns take the per-entry form instead: count per column with
// device atomics -> exclusive scan -> scatter with atomic cursors -> the
// same per-column sort.
// Source rows are unique within a column, so the sorted order is unique
// and the result is bit-exact and identical between runs, whichever form
// made it.  Columns are sorted by length class: <= 32 entries by a few
// lanes (rank sort), <= 4096 one workgroup (bitonic in LDS), longer ones in
// 4096-entry LDS-sorted chunks merged by a grid-wide rank computation
// (binary search in every chunk).
#include <algorithm>

#include "internal.hpp"

namespace csrad {
namespace {

constexpr int kShort = 32;
// Grid cap of the kernels that a device flag may switch off (grid-stride
// loops inside): 16 blocks per compute unit keeps the chip full when they
// run and costs a few microseconds of block dispatch when they do not.
constexpr unsigned kGatedGrid = 4096;
constexpr int kChunk = 4096;
constexpr int kSortThreads = 256;

// Column-sorted patterns: when the column indices never decrease over the
// entry array (across row boundaries too, e.g. an aggregation operator whose
// aggregates are contiguous, or its transpose), entry order is already
// column-major order.  The transpose's entries are then the entries in
// their own order: perm is the identity, colindT[e] is the row of e, and
// rowptrT[j] is the first entry with column >= j.  k_mono_probe: each block
// checks its contiguous share of the entries 256 at a time and stops (after
// clearing *mono) at the first slice holding a decrease; before every slice
// thread 0 re-reads the flag past the caches, so that blocks whose share is
// sorted stop once another block has cleared it.  Unsorted patterns
// therefore cost about one slice per block.  Every exit is block-uniform
// (decided through a block reduction).
__global__ __launch_bounds__(256) void k_mono_probe(int nnz, const int32_t* __restrict__ colind,
                                                    int32_t* __restrict__ mono) {
  const long long per = ((long long)nnz + gridDim.x - 1) / gridDim.x;
  const long long a = (long long)blockIdx.x * per, b = min((long long)nnz, a + per);
  for (long long base = a; base < b; base += 256) {
    const bool cleared =
        threadIdx.x == 0 && __hip_atomic_load(mono, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
    if (__syncthreads_or(cleared)) return;
    const long long e = base + threadIdx.x;
    const bool down = e >= 1 && e < b && colind[e - 1] > colind[e];
    if (__syncthreads_or(down)) {
      if (threadIdx.x == 0) *mono = 0;
      return;
    }
  }
}

// Outputs for a column-sorted pattern, one launch:
//  * rowptrT: entry e (0 <= e <= nnz, e = nnz standing for the end) owns the
//    columns j with colind[e-1] < j <= colind[e] (0 <= j and j <= n at the
//    ends) and writes rowptrT[j] = e; every j in [0, n] is owned by exactly
//    one e;
//  * colindT and perm: G lanes per row (G from the mean row length) write
//    the row of each entry and the identity.
template <int G>
__global__ __launch_bounds__(256) void k_mono_out(int m, int nnz, int n,
                                                  const int32_t* __restrict__ rowptr,
                                                  const int32_t* __restrict__ colind,
                                                  int32_t* __restrict__ rowptrT,
                                                  int32_t* __restrict__ colindT,
                                                  int32_t* __restrict__ perm,
                                                  const int32_t* __restrict__ mono) {
  if (*mono == 0) return;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e <= nnz;
       e += (long long)gridDim.x * blockDim.x) {
    const int lo = e == 0 ? 0 : colind[e - 1] + 1;
    const int hi = e == nnz ? n : colind[e];
    for (int j = lo; j <= hi; ++j) rowptrT[j] = (int32_t)e;
  }
  for (long long i = (long long)blockIdx.x * (256 / G) + threadIdx.x / G; i < m;
       i += (long long)gridDim.x * (256 / G)) {
    for (int e = rowptr[i] + threadIdx.x % G; e < rowptr[i + 1]; e += G) {
      colindT[e] = (int32_t)i;
      perm[e] = e;
    }
  }
}

// Symmetric try: entry e = (i, j) finds the position of its mirror (j, i)
// in row j; the transpose's entry at that position is e.  The mirror map is
// an involution, so perm[e] = mirror position is the same permutation,
// written in order.  The transpose's pattern is the pattern itself, so
// rowptrT and colindT are copied on the way.  Clears *sym when some entry
// has no mirror (the general path then rewrites all three outputs).  The
// lookup reads the first kMirrorWin columns of row j with independent loads
// (one round of memory latency instead of a chain of binary-search steps)
// and searches the rest of longer rows.
constexpr int kMirrorWin = 8;

// Unaligned 16- and 8-byte vectors of int32 (global loads need only 4-byte
// alignment on this target).
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x2 __attribute__((ext_vector_type(2)));
typedef i32x4 i32x4_u __attribute__((aligned(4)));
typedef i32x2 i32x2_u __attribute__((aligned(4)));

// Position of column i in the sorted row [a, b) of colind, or -1: the first
// kMirrorWin columns with two 16-byte loads, the rest of a longer row by
// binary search.
__device__ __forceinline__ int mirror_in_row(const int32_t* __restrict__ colind, int nnz, int a,
                                             int b, int i) {
  int v[kMirrorWin];
  if (a + kMirrorWin <= nnz) {
    // two 16-byte loads cover the first 8 columns of the row (entries past
    // the row's end are masked)
    const i32x4 lo = *reinterpret_cast<const i32x4_u*>(colind + a);
    const i32x4 hi = *reinterpret_cast<const i32x4_u*>(colind + a + 4);
    v[0] = lo.x; v[1] = lo.y; v[2] = lo.z; v[3] = lo.w;
    v[4] = hi.x; v[5] = hi.y; v[6] = hi.z; v[7] = hi.w;
#pragma unroll
    for (int u = 0; u < kMirrorWin; ++u) v[u] = a + u < b ? v[u] : -1;
  } else {
#pragma unroll
    for (int u = 0; u < kMirrorWin; ++u) v[u] = a + u < b ? colind[a + u] : -1;
  }
  int pos = -1;
#pragma unroll
  for (int u = 0; u < kMirrorWin; ++u)
    if (v[u] == i) pos = a + u;
  if (pos < 0 && b - a > kMirrorWin && v[kMirrorWin - 1] < i) {
    int lo = a + kMirrorWin, hi = b;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (colind[mid] < i) lo = mid + 1;
      else hi = mid;
    }
    if (lo < b && colind[lo] == i) pos = lo;
  }
  return pos;
}

// Position of column i in row j, or -1.
__device__ __forceinline__ int mirror_pos_win(const int32_t* __restrict__ rowptr,
                                              const int32_t* __restrict__ colind, int nnz, int j,
                                              int i) {
  const i32x2 ab = *reinterpret_cast<const i32x2_u*>(rowptr + j);  // rowptr[j], rowptr[j+1]
  return mirror_in_row(colind, nnz, ab.x, ab.y, i);
}

// Cheap first look: one block checks 256 rows spread over the pattern (the
// first and the last entry of each, two independent mirror lookups per
// thread) and clears *sym on a missing mirror, so that clearly unsymmetric
// patterns (e.g. triangular ones) skip the full pass.
__global__ __launch_bounds__(256) void k_sym_probe(int n, int nnz,
                                                   const int32_t* __restrict__ rowptr,
                                                   const int32_t* __restrict__ colind,
                                                   int32_t* __restrict__ sym,
                                                   const int32_t* __restrict__ mono) {
  if (*mono) {  // the column-sorted path covers it
    if (threadIdx.x == 0) *sym = 0;
    return;
  }
  const int i = (int)(((long long)threadIdx.x * n) / 256 + (n > 256 ? 128 % (n / 256) : 0));
  if (i >= n || (n <= 256 && (int)threadIdx.x >= n)) return;
  const int e0 = rowptr[i], e1 = rowptr[i + 1];
  if (e1 == e0) return;
  const int p0 = mirror_pos_win(rowptr, colind, nnz, colind[e0], i);
  const int p1 = mirror_pos_win(rowptr, colind, nnz, colind[e1 - 1], i);
  if (p0 < 0 || p1 < 0) *sym = 0;
}

// G lanes per row, each lane U of the row's entries at a time (entries l,
// l + G, ...) with the loads of all U mirror lookups issued stage by stage
// (columns, mirror row bounds, mirror windows): the lookups are chains of
// dependent gathers, and U chains per thread keep more of them in flight
// than more lanes would (the resident threads are the cap).
template <int G, int U>
__global__ __launch_bounds__(256) void k_sym_perm(int n, int nnz,
                                                  const int32_t* __restrict__ rowptr,
                                                  const int32_t* __restrict__ colind,
                                                  int32_t* __restrict__ rowptrT,
                                                  int32_t* __restrict__ colindT,
                                                  int32_t* __restrict__ perm,
                                                  int32_t* __restrict__ sym) {
  if (*sym == 0) return;  // uniform over the grid: a capped grid costs little when off
  for (int i = blockIdx.x * (256 / G) + threadIdx.x / G; i < n; i += gridDim.x * (256 / G)) {
    const int e0 = rowptr[i], e1 = rowptr[i + 1];
    if (threadIdx.x % G == 0) {
      rowptrT[i] = e0;
      if (i == n - 1) rowptrT[n] = e1;
    }
    for (int eb = e0 + threadIdx.x % G; eb < e1; eb += G * U) {
      int c[U], a[U], b[U];
#pragma unroll
      for (int u = 0; u < U; ++u) c[u] = eb + u * G < e1 ? colind[eb + u * G] : -1;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        a[u] = 0;
        b[u] = 0;
        if (c[u] >= 0) {
          const i32x2 ab = *reinterpret_cast<const i32x2_u*>(rowptr + c[u]);
          a[u] = ab.x;
          b[u] = ab.y;
        }
      }
      int pos[U];
#pragma unroll
      for (int u = 0; u < U; ++u) pos[u] = c[u] >= 0 ? mirror_in_row(colind, nnz, a[u], b[u], i) : 0;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (c[u] < 0) continue;
        if (pos[u] < 0) {
          *sym = 0;
          return;
        }
        perm[eb + u * G] = pos[u];
        colindT[eb + u * G] = c[u];
      }
    }
  }
}

// Column counts, one (wave-aggregated) atomic per entry; nothing when a fast
// path made the transpose.  Block 0 records that outcome in flags[3]
// (flags[1] | flags[2]: symmetric or column-sorted) for the kernels after it.
__global__ __launch_bounds__(256) void k_count_cols(const int32_t* __restrict__ colind, int nnz,
                                                    int32_t* __restrict__ flags,
                                                    int32_t* __restrict__ cnt) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  const bool fast = (flags[1] | flags[2]) != 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) flags[3] = fast;
  if (fast) return;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += stride)
    wave_agg_count(cnt, colind[e]);
}

// cnt[0 .. len) = 0 and the four path flags, one launch.
__global__ __launch_bounds__(256) void k_tr_init(int32_t* __restrict__ cnt, long long len,
                                                 int32_t* __restrict__ flags, int32_t a, int32_t b,
                                                 int32_t c, int32_t d) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < len;
       i += (long long)gridDim.x * blockDim.x)
    cnt[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    flags[0] = a;
    flags[1] = b;
    flags[2] = c;
    flags[3] = d;
  }
}

__global__ __launch_bounds__(256) void k_copy_i32(const int32_t* __restrict__ src, int n,
                                                  int32_t* __restrict__ dst,
                                                  const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// G lanes per row (G from the mean row length): lanes stride over the row's
// entries.
template <int G>
__global__ __launch_bounds__(256) void k_scatter(int m, const int32_t* __restrict__ rowptr,
                                                 const int32_t* __restrict__ colind,
                                                 int32_t* __restrict__ cursor,
                                                 int2* __restrict__ tkv,
                                                 const int32_t* __restrict__ fast) {
  if (*fast) return;
  const int sub = threadIdx.x % G;
  for (int row = blockIdx.x * (256 / G) + threadIdx.x / G; row < m; row += gridDim.x * (256 / G)) {
    const int e1 = rowptr[row + 1];
    for (int e = rowptr[row] + sub; e < e1; e += G) {
      const int slot = wave_agg_add(cursor, colind[e]);
      tkv[slot] = make_int2(row, e);  // one 8-byte store: (source row, entry)
    }
  }
}

// Short columns (<= kShort entries): G lanes per column, rank sort (keys
// unique).  Lane l ranks entries l, l+G, ... against the whole column; the
// lanes of a group read the same addresses in step.  Longer columns are
// appended to a list for the workgroup kernels.
template <int G>
__global__ __launch_bounds__(256) void k_sort_short(int n, const int32_t* __restrict__ rpT,
                                                    const int2* __restrict__ tkv,
                                                    int32_t* __restrict__ okey,
                                                    int32_t* __restrict__ oval,
                                                    int32_t* __restrict__ long_list,
                                                    int32_t* __restrict__ long_count,
                                                    const int32_t* __restrict__ fast) {
  if (*fast) return;
  const int l = threadIdx.x % G;
  for (int c = blockIdx.x * (256 / G) + threadIdx.x / G; c < n; c += gridDim.x * (256 / G)) {
    const int s = rpT[c], len = rpT[c + 1] - s;
    if (len <= kShort) {
      for (int q = l; q < len; q += G) {
        const int2 kv = tkv[s + q];
        int r = 0;
        for (int u = 0; u < len; ++u) r += tkv[s + u].x < kv.x;
        okey[s + r] = kv.x;
        oval[s + r] = kv.y;
      }
    } else if (l == 0) {
      long_list[atomicAdd(long_count, 1)] = c;
    }
  }
}

// Bitonic sort of P (power of two) key/value pairs in LDS, ascending keys.
__device__ void lds_bitonic(int32_t* key, int32_t* val, int P) {
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < P; i += blockDim.x) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const bool up = (i & k) == 0;
          const int a = key[i], b = key[ixj];
          if ((a > b) == up) {
            key[i] = b;
            key[ixj] = a;
            const int t = val[i];
            val[i] = val[ixj];
            val[ixj] = t;
          }
        }
      }
      __syncthreads();
    }
  }
}

__device__ __forceinline__ int pow2_at_least(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

// Sorts the (key, value) pairs [s, s+len) of src by key in LDS; len <= kChunk.
// The sorted keys and values go to (dst_key, dst_val), or back into src as
// pairs when dst_key is null.
__device__ void sort_range_lds(int2* src, int32_t* dst_key, int32_t* dst_val, int s, int len,
                               int32_t* kk, int32_t* vv) {
  const int P = pow2_at_least(len);
  for (int i = threadIdx.x; i < P; i += blockDim.x) {
    const int2 kv = i < len ? src[s + i] : make_int2(INT32_MAX, 0);
    kk[i] = kv.x;
    vv[i] = kv.y;
  }
  __syncthreads();
  lds_bitonic(kk, vv, P);
  for (int i = threadIdx.x; i < len; i += blockDim.x) {
    if (dst_key) {
      dst_key[s + i] = kk[i];
      dst_val[s + i] = vv[i];
    } else {
      src[s + i] = make_int2(kk[i], vv[i]);
    }
  }
  __syncthreads();
}

// Medium columns (kShort < len <= kChunk): one workgroup each.
__global__ __launch_bounds__(kSortThreads) void k_sort_medium(
    const int32_t* __restrict__ rpT, int2* __restrict__ tkv, int32_t* __restrict__ okey,
    int32_t* __restrict__ oval, const int32_t* __restrict__ long_list,
    const int32_t* __restrict__ long_count) {
  __shared__ int32_t kk[kChunk];
  __shared__ int32_t vv[kChunk];
  const int nl = *long_count;
  for (int t = blockIdx.x; t < nl; t += gridDim.x) {
    const int c = long_list[t];
    const int s = rpT[c], len = rpT[c + 1] - s;
    if (len > kChunk) continue;  // uniform over the block
    sort_range_lds(tkv, okey, oval, s, len, kk, vv);
  }
}

// Long columns, step 1: sort each kChunk-entry chunk in place in the
// scratch arrays.  Every block walks the whole long list and takes the
// chunks whose index matches it modulo the grid size.
__global__ __launch_bounds__(kSortThreads) void k_sort_long_chunks(
    const int32_t* __restrict__ rpT, int2* __restrict__ tkv,
    const int32_t* __restrict__ long_list, const int32_t* __restrict__ long_count) {
  __shared__ int32_t kk[kChunk];
  __shared__ int32_t vv[kChunk];
  const int nl = *long_count;
  for (int t = 0; t < nl; ++t) {
    const int c = long_list[t];
    const int s = rpT[c], len = rpT[c + 1] - s;
    if (len <= kChunk) continue;
    const int nch = (len + kChunk - 1) / kChunk;
    for (int ch = blockIdx.x; ch < nch; ch += gridDim.x) {
      const int cs = s + ch * kChunk;
      const int cl = min(kChunk, s + len - cs);
      sort_range_lds(tkv, nullptr, nullptr, cs, cl, kk, vv);
    }
  }
}

// Number of keys < key in the sorted range [lo, hi).
__device__ __forceinline__ int count_less(const int2* a, int lo, int hi, int key) {
  int l = lo, h = hi;
  while (l < h) {
    const int mid = (l + h) >> 1;
    if (a[mid].x < key) l = mid + 1;
    else h = mid;
  }
  return l - lo;
}

// Long columns, step 2: the final position of each entry is its position
// in its own sorted chunk plus the number of smaller keys in every other
// chunk.
__global__ __launch_bounds__(256) void k_rank_long(const int32_t* __restrict__ rpT,
                                                   const int2* __restrict__ tkv,
                                                   int32_t* __restrict__ okey,
                                                   int32_t* __restrict__ oval,
                                                   const int32_t* __restrict__ long_list,
                                                   const int32_t* __restrict__ long_count) {
  const int nl = *long_count;
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long gsz = (long long)gridDim.x * blockDim.x;
  for (int t = 0; t < nl; ++t) {
    const int c = long_list[t];
    const int s = rpT[c], len = rpT[c + 1] - s;
    if (len <= kChunk) continue;
    const int nch = (len + kChunk - 1) / kChunk;
    for (long long q = gid; q < len; q += gsz) {
      const int my = (int)(q / kChunk);
      const int2 kv = tkv[s + q];
      int r = (int)(q - (long long)my * kChunk);
      for (int ch = 0; ch < nch; ++ch) {
        if (ch == my) continue;
        const int lo = s + ch * kChunk, hi = min(s + len, lo + kChunk);
        r += count_less(tkv, lo, hi, kv.x);
      }
      okey[s + r] = kv.x;
      oval[s + r] = kv.y;
    }
  }
}

// ---------------------------------------------------------------------
// Column-block form of the general transpose.
// ---------------------------------------------------------------------
constexpr int kBkMaxShift = 12;      // at most 4096 columns per block
constexpr int kBkMaxBlocks = 8192;   // at most 8192 column blocks (n <= 2^25)
constexpr int kBkTarget = 2048;      // aimed-for mean entries per column block
constexpr int kBkTileEntries = 4096; // aimed-for entries per row tile
constexpr int kBkLdsBytes = 48896;   // dynamic LDS cap of a column-block workgroup
constexpr int kBkMaxTileRows = 4096; // at most 4096 rows per tile
constexpr int kBkUnroll = 4;         // loads in flight per thread
constexpr int kBkColsThreads = 512;  // threads of a column-block workgroup

struct BkShape {
  int shift = 0, nb = 0;
  bool on = false;
};

// Column-block size 2^shift (at least 32 columns) with a mean of about
// kBkTarget entries per block, and at most kBkMaxBlocks blocks.
BkShape bk_shape(int n, int nnz) {
  BkShape b;
  if (n <= 0 || nnz <= 0 || (long long)n > ((long long)kBkMaxBlocks << kBkMaxShift)) return b;
  int sh = 5;
  while (sh < kBkMaxShift && (2ll << sh) * nnz <= (long long)kBkTarget * n) ++sh;
  while (sh < kBkMaxShift && ((n + (1 << sh) - 1) >> sh) > kBkMaxBlocks) ++sh;
  b.shift = sh;
  b.nb = (n + (1 << sh) - 1) >> sh;
  b.on = true;
  return b;
}

// Entry capacity of the LDS grouping buffer next to the column counters.
// (at most 4096 entries: a smaller buffer keeps more workgroups per CU).
int bk_lds_cap(int shift) {
  return std::min(4096, (kBkLdsBytes - (2 * (1 << shift) + 2) * 4) / 8);
}
int bk_lds_bytes(int shift) { return (2 * (1 << shift) + 2) * 4 + bk_lds_cap(shift) * 8; }

// Column-block counts of the entries [ea, eb) of a row tile into h (LDS),
// kBkUnroll coalesced loads in flight per thread.
__device__ __forceinline__ void bk_tile_counts(const int32_t* __restrict__ colind, int ea, int eb,
                                               int shift, int32_t* h) {
  for (long long base = ea; base < eb; base += 256 * kBkUnroll) {
    int key[kBkUnroll];
#pragma unroll
    for (int u = 0; u < kBkUnroll; ++u) {
      const long long e = base + u * 256 + threadIdx.x;
      key[u] = e < eb ? colind[e] >> shift : -1;
    }
#pragma unroll
    for (int u = 0; u < kBkUnroll; ++u)
      if (key[u] >= 0) atomicAdd(&h[key[u]], 1);
  }
}

// Pass 1: column-block counts of a tile of rows (its entries read flat) in
// LDS; the non-zero ones go to the block totals with one atomic each.
// Block 0 records the fast-path outcome in flags[3] (flags[1] | flags[2]).
__global__ __launch_bounds__(256) void k_bk_count(int m, const int32_t* __restrict__ rowptr,
                                                  const int32_t* __restrict__ colind,
                                                  int rows_per_tile, int shift, int nb,
                                                  int32_t* __restrict__ btotal,
                                                  int32_t* __restrict__ flags) {
  extern __shared__ int32_t h[];  // nb counters
  const bool fast = (flags[1] | flags[2]) != 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) flags[3] = fast;
  if (fast) return;  // uniform over the grid
  for (int b = threadIdx.x; b < nb; b += 256) h[b] = 0;
  __syncthreads();
  const int r0 = blockIdx.x * rows_per_tile, r1 = min(m, r0 + rows_per_tile);
  bk_tile_counts(colind, rowptr[r0], rowptr[r1], shift, h);
  __syncthreads();
  for (int b = threadIdx.x; b < nb; b += 256)
    if (h[b]) atomicAdd(&btotal[b], h[b]);
}

// Pass 2: the same counts again (G lanes per row); one returning atomic per
// non-zero block reserves this tile's slots in the block's output range
// (bbase[b] is the range's start), and every entry then takes a slot with
// an LDS atomic: srow/sent/scol[slot] = (row, entry, column within the
// block).  srow and sent are the colindT and perm outputs, used as staging
// until pass 3.  (Reading the tile's entries flat and finding their rows by
// a search in LDS measured slower than lanes per row here.)
template <int G>
__global__ __launch_bounds__(256) void k_bk_place(int m, const int32_t* __restrict__ rowptr,
                                                  const int32_t* __restrict__ colind,
                                                  int rows_per_tile, int shift, int nb,
                                                  const int32_t* __restrict__ bbase,
                                                  int32_t* __restrict__ brel,
                                                  int32_t* __restrict__ srow,
                                                  int32_t* __restrict__ sent,
                                                  uint16_t* __restrict__ scol,
                                                  const int32_t* __restrict__ fast) {
  extern __shared__ int32_t h[];  // nb counters, then the same array as nb cursors
  if (*fast) return;              // uniform over the grid
  for (int b = threadIdx.x; b < nb; b += 256) h[b] = 0;
  __syncthreads();
  const int r0 = blockIdx.x * rows_per_tile, r1 = min(m, r0 + rows_per_tile);
  for (int row = r0 + (int)threadIdx.x / G; row < r1; row += 256 / G) {
    const int e1 = rowptr[row + 1];
    for (int e = rowptr[row] + (int)threadIdx.x % G; e < e1; e += G)
      atomicAdd(&h[colind[e] >> shift], 1);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nb; b += 256) {
    const int c = h[b];
    if (c) h[b] = bbase[b] + atomicAdd(&brel[b], c);
  }
  __syncthreads();
  const int mask = (1 << shift) - 1;
  for (int row = r0 + (int)threadIdx.x / G; row < r1; row += 256 / G) {
    const int e1 = rowptr[row + 1];
    for (int e = rowptr[row] + (int)threadIdx.x % G; e < e1; e += G) {
      const int col = colind[e];
      const int slot = atomicAdd(&h[col >> shift], 1);
      srow[slot] = row;
      sent[slot] = e;
      scol[slot] = (uint16_t)(col & mask);
    }
  }
}

// Exclusive scan of a[0 .. len) in LDS by the whole block (BT threads,
// each a contiguous run); a[len] = the total.  wsum: BT / 64 ints of LDS.
template <int BT>
__device__ void lds_exclusive_scan(int32_t* a, int len, int32_t* wsum) {
  const int per = (len + BT - 1) / BT;
  const int lo = min(len, (int)threadIdx.x * per), hi = min(len, lo + per);
  int sum = 0;
  for (int i = lo; i < hi; ++i) sum += a[i];
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  int v = sum;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int u = __shfl_up(v, o);
    if (lane >= o) v += u;
  }
  if (lane == kWave - 1) wsum[wid] = v;
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < BT / kWave; ++w) {
    if (w < wid) off += wsum[w];
    tot += wsum[w];
  }
  int run = off + v - sum;
  for (int i = lo; i < hi; ++i) {
    const int x = a[i];
    a[i] = run;
    run += x;
  }
  if (threadIdx.x == 0) a[len] = tot;
  __syncthreads();
}

// Pass 3: one workgroup per column block b (its entries are the output
// range [bbase[b], bbase[b+1]), staged by pass 2).  Counts per column in
// LDS -> exclusive scan -> rowptrT of the block's columns; groups the
// entries by column (in LDS when at most cap of them, else in tkv at their
// output positions); then G lanes per column: columns of at most kShort
// entries are rank-sorted by source row straight into colindT/perm, longer
// ones are left in tkv and listed for the medium/long sorts.  All staged
// inputs are read before the first output is written (block barrier), and
// block ranges are disjoint, so the in-place use of colindT/perm is safe.
template <int G, int BT>
__global__ __launch_bounds__(BT) void k_bk_cols(int n, int shift, int nb, int cap,
                                                 const int32_t* __restrict__ bbase,
                                                 const uint16_t* __restrict__ scol,
                                                 int32_t* __restrict__ colindT,
                                                 int32_t* __restrict__ perm,
                                                 int32_t* __restrict__ rowptrT,
                                                 int2* __restrict__ tkv,
                                                 int32_t* __restrict__ long_list,
                                                 int32_t* __restrict__ long_count,
                                                 const int32_t* __restrict__ fast) {
  extern __shared__ __align__(16) int32_t lds[];
  __shared__ int32_t wsum[BT / kWave];
  if (*fast) return;  // uniform over the grid
  const int cb = 1 << shift;
  int32_t* start = lds;                                    // cb + 1
  int32_t* cur = lds + cb + 1;                             // cb
  int2* lkv = reinterpret_cast<int2*>(lds + 2 * cb + 2);  // cap pairs (8-byte aligned)
  const int b = blockIdx.x;
  const int s0 = bbase[b], s1 = bbase[b + 1], len = s1 - s0;
  const int c0 = b << shift, ncb = min(cb, n - c0);
  for (int c = threadIdx.x; c <= ncb; c += BT) start[c] = 0;
  __syncthreads();
  for (long long base = s0; base < s1; base += BT * kBkUnroll) {
    int c[kBkUnroll];
#pragma unroll
    for (int u = 0; u < kBkUnroll; ++u) {
      const long long i = base + u * BT + threadIdx.x;
      c[u] = i < s1 ? scol[i] : -1;
    }
#pragma unroll
    for (int u = 0; u < kBkUnroll; ++u)
      if (c[u] >= 0) atomicAdd(&start[c[u]], 1);
  }
  __syncthreads();
  lds_exclusive_scan<BT>(start, ncb, wsum);
  for (int c = threadIdx.x; c < ncb; c += BT) {
    cur[c] = start[c];
    rowptrT[c0 + c] = s0 + start[c];
  }
  if (b == nb - 1 && threadIdx.x == 0) rowptrT[n] = s1;
  __syncthreads();
  const bool in_lds = len <= cap;
  for (long long base = s0; base < s1; base += BT * kBkUnroll) {
    int c[kBkUnroll];
    int2 kv[kBkUnroll];
#pragma unroll
    for (int u = 0; u < kBkUnroll; ++u) {
      const long long i = base + u * BT + threadIdx.x;
      c[u] = i < s1 ? scol[i] : -1;
      kv[u] = i < s1 ? make_int2(colindT[i], perm[i]) : make_int2(0, 0);
    }
#pragma unroll
    for (int u = 0; u < kBkUnroll; ++u) {
      if (c[u] < 0) continue;
      const int p = atomicAdd(&cur[c[u]], 1);
      if (in_lds) lkv[p] = kv[u];
      else tkv[s0 + p] = kv[u];
    }
  }
  __syncthreads();
  const int l = threadIdx.x % G;
  for (int c = threadIdx.x / G; c < ncb; c += BT / G) {
    const int st = start[c], lc = start[c + 1] - st;
    if (lc <= kShort) {
      for (int q = l; q < lc; q += G) {
        const int2 kv = in_lds ? lkv[st + q] : tkv[s0 + st + q];
        int r = 0;
        if (in_lds) {
          for (int u = 0; u < lc; ++u) r += lkv[st + u].x < kv.x;
        } else {
          for (int u = 0; u < lc; ++u) r += tkv[s0 + st + u].x < kv.x;
        }
        colindT[s0 + st + r] = kv.x;
        perm[s0 + st + r] = kv.y;
      }
    } else {
      if (in_lds)
        for (int q = l; q < lc; q += G) tkv[s0 + st + q] = lkv[st + q];
      if (l == 0) long_list[atomicAdd(long_count, 1)] = c0 + c;
    }
  }
}

// ---------------------------------------------------------------------
// Stable grouping of n elements by a small key (K <= kSmallKeys): the
// element indices come out ordered by key, ascending index within a key.
// Per tile of kMsTile elements: a key histogram, then a scan over
// (key, tile) gives each tile's base per key; inside a tile the rank of
// an element among equal keys before it comes from wave ballots and
// per-wave counts, chunk by chunk.  No global atomics, deterministic.
// ---------------------------------------------------------------------
constexpr int kSmallKeys = 32;
constexpr int kMsChunks = 8;
constexpr int kMsTile = 256 * kMsChunks;

__global__ __launch_bounds__(256) void k_ms_hist(const int32_t* __restrict__ keys, int n, int K,
                                                 int ntiles, int32_t* __restrict__ hist,
                                                 const int32_t* __restrict__ skip) {
  if (skip && *skip) return;  // uniform over the grid
  __shared__ int h[kSmallKeys];
  if (threadIdx.x < kSmallKeys) h[threadIdx.x] = 0;
  __syncthreads();
  const long long base = (long long)blockIdx.x * kMsTile;
  for (int c = 0; c < kMsChunks; ++c) {
    const long long i = base + c * 256 + threadIdx.x;
    if (i < n) atomicAdd(&h[keys[i]], 1);
  }
  __syncthreads();
  if (threadIdx.x < K) hist[(long long)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Block 0 also writes the key pointers ptr[0 .. K] (ptr[l] = the first
// slot of key l, ptr[K] = n).
__global__ __launch_bounds__(256) void k_ms_scatter(const int32_t* __restrict__ keys, int n,
                                                    int K, int ntiles,
                                                    const int32_t* __restrict__ off,
                                                    int32_t* __restrict__ order,
                                                    int32_t* __restrict__ ptr,
                                                    const int32_t* __restrict__ skip) {
  if (skip && *skip) return;  // uniform over the grid
  if (blockIdx.x == 0 && (int)threadIdx.x <= K)
    ptr[threadIdx.x] = (int)threadIdx.x < K ? off[(long long)threadIdx.x * ntiles] : n;
  __shared__ int wcount[4][kSmallKeys];
  __shared__ int running[kSmallKeys];
  const int lane = __lane_id(), w = threadIdx.x / kWave;
  const unsigned long long lt = (1ull << lane) - 1ull;
  if (threadIdx.x < kSmallKeys) running[threadIdx.x] = 0;
  for (int q = threadIdx.x; q < 4 * kSmallKeys; q += 256) (&wcount[0][0])[q] = 0;
  __syncthreads();
  const long long base = (long long)blockIdx.x * kMsTile;
  for (int c = 0; c < kMsChunks; ++c) {
    const long long i = base + c * 256 + threadIdx.x;
    const bool act = i < n;
    const int key = act ? keys[i] : -1;
    // peers: lanes of this wave with the same key (loop over distinct keys)
    unsigned long long todo = __ballot(act);
    unsigned long long peers = 0;
    while (todo) {
      const int leader = __ffsll((long long)todo) - 1;
      const int lkey = __builtin_amdgcn_readlane(key, leader);
      const unsigned long long m = __ballot(act && key == lkey);
      if (act && key == lkey) peers = m;
      if (lane == leader) wcount[w][lkey] = __popcll(m);
      todo &= ~m;
    }
    __syncthreads();
    if (act) {
      int pre = running[key];
      for (int v = 0; v < w; ++v) pre += wcount[v][key];
      order[off[(long long)key * ntiles + blockIdx.x] + pre + __popcll(peers & lt)] = (int32_t)i;
    }
    __syncthreads();
    if (threadIdx.x < K) {
      int t = 0;
      for (int v = 0; v < 4; ++v) t += wcount[v][threadIdx.x];
      running[threadIdx.x] += t;
    }
    // every wave's counts must be summed before any of them is cleared
    __syncthreads();
    for (int q = threadIdx.x; q < 4 * kSmallKeys; q += 256) (&wcount[0][0])[q] = 0;
    __syncthreads();
  }
}

struct TransposeWs {
  BkShape bk;
  int32_t* bk_total;  // [nb] block totals, then [nb] reservation counters
  int32_t* bk_base;   // [nb + 1] block output ranges
  uint16_t* bk_col;   // [nnz] column within the block, per staged entry
  int32_t* cnt;
  void* scan_ws;
  size_t scan_bytes;
  long long* total;
  int2* tkv;  // scatter slots: (source row, entry)
  int32_t* long_list;
  int32_t* flags;  // [0] long-column count, [1] symmetric path on, [2] column-sorted path on,
                   // [3] either fast path on
  int32_t* long_count;
  int32_t* sym;
  int32_t* mono;
  int32_t* fast;
};

TransposeWs carve_transpose(Carver& cv, int n, int nnz) {
  TransposeWs w;
  w.bk = bk_shape(n, nnz);
  const size_t nb = w.bk.on ? (size_t)w.bk.nb : 0;
  w.bk_total = cv.take<int32_t>(2 * nb);
  w.bk_base = cv.take<int32_t>(nb + 1);
  w.bk_col = cv.take<uint16_t>(w.bk.on ? (size_t)nnz : 0);
  w.cnt = cv.take<int32_t>((size_t)n + 1);
  w.scan_bytes = scan_workspace(n);
  w.scan_ws = cv.take<char>(w.scan_bytes);
  w.total = cv.take<long long>(1);
  w.tkv = cv.take<int2>((size_t)nnz);
  w.long_list = cv.take<int32_t>((size_t)n + 1);
  w.flags = cv.take<int32_t>(4);
  w.long_count = w.flags;
  w.sym = w.flags + 1;
  w.mono = w.flags + 2;
  w.fast = w.flags + 3;
  return w;
}

unsigned grid_for(long long work, int threads, unsigned cap = 65536) {
  long long b = (work + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

template <typename T>
__global__ __launch_bounds__(256) void k_gather_vals(int nnz, const int32_t* __restrict__ perm,
                                                     const T* __restrict__ vals,
                                                     T* __restrict__ out) {
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < nnz;
       t += (long long)gridDim.x * blockDim.x)
    out[t] = vals[perm[t]];
}

}  // namespace

size_t transpose_workspace(int m, int n, int nnz) {
  (void)m;
  Carver cv(nullptr, 0);
  carve_transpose(cv, n, nnz);
  return cv.off + 256;
}

int transpose_pattern(int m, int n, int nnz, const int32_t* rowptr, const int32_t* colind,
                      int32_t* rowptrT, int32_t* colindT, int32_t* perm, void* work, size_t bytes,
                      hipStream_t s) {
  Carver cv(work, bytes);
  TransposeWs w = carve_transpose(cv, n, nnz);
  if (!work || !cv.ok) return CSRAD_EWORKSPACE;
  // zeroes the counters of the form in use (block totals and reservation
  // counters, or per-column counts) and sets the path flags
  int32_t* zero = w.bk.on ? w.bk_total : w.cnt;
  const long long zlen = w.bk.on ? 2ll * w.bk.nb : (long long)n + 1;
  hipLaunchKernelGGL(k_tr_init, dim3(grid_for(zlen, 256, 2048)), dim3(256), 0, s, zero, zlen,
                     w.flags, 0, (m == n && nnz > 0) ? 1 : 0, nnz > 0 ? 1 : 0, 0);
  if (nnz > 0) {
    hipLaunchKernelGGL(k_mono_probe, dim3(grid_for(nnz, 256, 2048)), dim3(256), 0, s, nnz, colind,
                       w.mono);
    int g = 1;
    while (g < 32 && (long long)g * m < nnz) g <<= 1;
    const long long work = std::max((long long)nnz + 1, (long long)m * g);
    const unsigned grid = grid_for(work, 256, 4096);
    switch (g) {
#define CSRAD_MONO_OUT(G)                                                                      \
  hipLaunchKernelGGL((k_mono_out<G>), dim3(grid), dim3(256), 0, s, m, nnz, n, rowptr, colind, \
                     rowptrT, colindT, perm, w.mono)
      case 1: CSRAD_MONO_OUT(1); break;
      case 2: CSRAD_MONO_OUT(2); break;
      case 4: CSRAD_MONO_OUT(4); break;
      case 8: CSRAD_MONO_OUT(8); break;
      case 16: CSRAD_MONO_OUT(16); break;
      default: CSRAD_MONO_OUT(32); break;
#undef CSRAD_MONO_OUT
    }
  }
  if (m == n && nnz > 0) {
    hipLaunchKernelGGL(k_sym_probe, dim3(1), dim3(256), 0, s, m, nnz, rowptr, colind, w.sym,
                       w.mono);
    // lanes from the mean row length; U = 4 entries per lane when the rows
    // are many for the chip (the lookups are latency chains)
    int L = 1;
    while (L < 32 && (long long)L * m < nnz) L <<= 1;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      cus = 256;
    const bool batch = L >= 8 && (long long)m * L >= 8ll * cus * 2048;
    const int gl = batch ? L / 4 : L;
    const unsigned grid = grid_for((long long)m * gl, 256, kGatedGrid);
#define CSRAD_SYM_PERM(G, U)                                                                 \
  hipLaunchKernelGGL((k_sym_perm<G, U>), dim3(grid), dim3(256), 0, s, m, nnz, rowptr, colind, \
                     rowptrT, colindT, perm, w.sym)
    if (batch) {
      switch (gl) {
        case 2: CSRAD_SYM_PERM(2, 4); break;
        case 4: CSRAD_SYM_PERM(4, 4); break;
        default: CSRAD_SYM_PERM(8, 4); break;
      }
    } else {
      switch (gl) {
        case 1: CSRAD_SYM_PERM(1, 1); break;
        case 2: CSRAD_SYM_PERM(2, 1); break;
        case 4: CSRAD_SYM_PERM(4, 1); break;
        case 8: CSRAD_SYM_PERM(8, 1); break;
        case 16: CSRAD_SYM_PERM(16, 1); break;
        default: CSRAD_SYM_PERM(32, 1); break;
      }
    }
#undef CSRAD_SYM_PERM
  }
  if (w.bk.on) {
    // column-block form
    const int nb = w.bk.nb, sh = w.bk.shift;
    // row tiles of about kBkTileEntries entries (64 to kBkMaxTileRows rows)
    const long long rpt = std::min<long long>(
        kBkMaxTileRows, std::max<long long>(64, (long long)kBkTileEntries * m / nnz));
    const unsigned tiles = (unsigned)((m + rpt - 1) / rpt);
    hipLaunchKernelGGL(k_bk_count, dim3(tiles), dim3(256), (size_t)nb * 4, s, m, rowptr, colind,
                       (int)rpt, sh, nb, w.bk_total, w.flags);
    CSRAD_TRY(scan_exclusive(w.bk_total, w.bk_base, nb, w.total, w.scan_ws, w.scan_bytes, s,
                             w.fast));
    int g = 1;
    while (g < 8 && (long long)g * m < nnz) g <<= 1;
    switch (g) {
#define CSRAD_BK_PLACE(G)                                                                    \
  hipLaunchKernelGGL((k_bk_place<G>), dim3(tiles), dim3(256), (size_t)nb * 4, s, m, rowptr, \
                     colind, (int)rpt, sh, nb, w.bk_base, w.bk_total + nb, colindT, perm,   \
                     w.bk_col, w.fast)
      case 1: CSRAD_BK_PLACE(1); break;
      case 2: CSRAD_BK_PLACE(2); break;
      case 4: CSRAD_BK_PLACE(4); break;
      default: CSRAD_BK_PLACE(8); break;
#undef CSRAD_BK_PLACE
    }
    // lanes per column from the mean column length (at most kShort)
    int gc = 1;
    while (gc < kShort && (long long)gc * n < nnz) gc <<= 1;
    const int cap = bk_lds_cap(sh);
    const size_t lb = (size_t)bk_lds_bytes(sh);
    switch (gc) {
#define CSRAD_BK_COLS(G)                                                                    \
  hipLaunchKernelGGL((k_bk_cols<G, kBkColsThreads>), dim3(nb), dim3(kBkColsThreads), lb, s, n, \
                     sh, nb, cap, w.bk_base, w.bk_col, colindT, perm, rowptrT, w.tkv,         \
                     w.long_list, w.long_count, w.fast)
      case 1: CSRAD_BK_COLS(1); break;
      case 2: CSRAD_BK_COLS(2); break;
      case 4: CSRAD_BK_COLS(4); break;
      case 8: CSRAD_BK_COLS(8); break;
      case 16: CSRAD_BK_COLS(16); break;
      default: CSRAD_BK_COLS(32); break;
#undef CSRAD_BK_COLS
    }
  } else {
    // per-entry form (no entries, or more than 2^25 columns)
    if (nnz > 0)
      hipLaunchKernelGGL(k_count_cols, dim3(grid_for(nnz, 256, kGatedGrid)), dim3(256), 0, s,
                         colind, nnz, w.flags, w.cnt);
    CSRAD_TRY(scan_exclusive(w.cnt, rowptrT, n, w.total, w.scan_ws, w.scan_bytes, s, w.fast));
    if (nnz == 0) return launch_status();
    if (n > 0)
      hipLaunchKernelGGL(k_copy_i32, dim3(grid_for(n, 256, 2048)), dim3(256), 0, s, rowptrT, n,
                         w.cnt, w.fast);
    // gated kernels take capped grids with grid-stride loops, so that they
    // cost little when a fast path has made the transpose
    if (m > 0) {
      int g = 1;
      while (g < 8 && (long long)g * m < nnz) g <<= 1;
      const unsigned grid = grid_for((long long)m * g, 256, kGatedGrid);
      switch (g) {
#define CSRAD_SCATTER(G)                                                                     \
  hipLaunchKernelGGL((k_scatter<G>), dim3(grid), dim3(256), 0, s, m, rowptr, colind, w.cnt, \
                     w.tkv, w.fast)
        case 1: CSRAD_SCATTER(1); break;
        case 2: CSRAD_SCATTER(2); break;
        case 4: CSRAD_SCATTER(4); break;
        default: CSRAD_SCATTER(8); break;
#undef CSRAD_SCATTER
      }
    }
    {
      // lanes per column from the mean column length (at most kShort)
      int g = 1;
      while (g < kShort && (long long)g * n < nnz) g <<= 1;
      const unsigned grid = grid_for((long long)n * g, 256, kGatedGrid);
      switch (g) {
#define CSRAD_SORT_SHORT(G)                                                                  \
  hipLaunchKernelGGL((k_sort_short<G>), dim3(grid), dim3(256), 0, s, n, rowptrT, w.tkv,        \
                     colindT, perm, w.long_list, w.long_count, w.fast)
        case 1: CSRAD_SORT_SHORT(1); break;
        case 2: CSRAD_SORT_SHORT(2); break;
        case 4: CSRAD_SORT_SHORT(4); break;
        case 8: CSRAD_SORT_SHORT(8); break;
        case 16: CSRAD_SORT_SHORT(16); break;
        default: CSRAD_SORT_SHORT(32); break;
#undef CSRAD_SORT_SHORT
      }
    }
  }
  hipLaunchKernelGGL(k_sort_medium, dim3(1024), dim3(kSortThreads), 0, s, rowptrT, w.tkv,
                     colindT, perm, w.long_list, w.long_count);
  hipLaunchKernelGGL(k_sort_long_chunks, dim3(256), dim3(kSortThreads), 0, s, rowptrT, w.tkv,
                     w.long_list, w.long_count);
  hipLaunchKernelGGL(k_rank_long, dim3(1024), dim3(256), 0, s, rowptrT, w.tkv, colindT,
                     perm, w.long_list, w.long_count);
  return launch_status();
}

size_t group_small_workspace(int n, int K) {
  const size_t ntiles = (size_t)(n + kMsTile - 1) / kMsTile;
  const size_t cells = ntiles * (size_t)(K > 0 ? K : 1);
  Carver cv(nullptr, 0);
  cv.take<int32_t>(cells);
  cv.take<int32_t>(cells + 1);
  cv.take<char>(scan_workspace((int)cells));
  cv.take<long long>(1);
  return cv.off + 256;
}

int group_small_keys(const int32_t* keys, int n, int K, int32_t* ptr, int32_t* order, void* work,
                     size_t bytes, hipStream_t s, const int32_t* skip) {
  if (K < 1 || K > kSmallKeys || n < 1) return CSRAD_EINVAL;
  const int ntiles = (n + kMsTile - 1) / kMsTile;
  const int cells = ntiles * K;
  Carver cv(work, bytes);
  int32_t* hist = cv.take<int32_t>(cells);
  int32_t* off = cv.take<int32_t>((size_t)cells + 1);
  const size_t sb = scan_workspace(cells);
  void* sws = cv.take<char>(sb);
  long long* total = cv.take<long long>(1);
  if (!work || !cv.ok) return CSRAD_EWORKSPACE;
  hipLaunchKernelGGL(k_ms_hist, dim3(ntiles), dim3(256), 0, s, keys, n, K, ntiles, hist, skip);
  CSRAD_TRY(scan_exclusive(hist, off, cells, total, sws, sb, s, skip));
  hipLaunchKernelGGL(k_ms_scatter, dim3(ntiles), dim3(256), 0, s, keys, n, K, ntiles, off, order,
                     ptr, skip);
  return launch_status();
}

}  // namespace csrad

using namespace csrad;

extern "C" int csr_transpose_workspace(const csrad_csr* A, size_t* bytes) {
  if (!A || !bytes) return CSRAD_EINVAL;
  if (A->nrows < 0 || A->ncols < 0 || A->nnz < 0) return CSRAD_EINVAL;
  *bytes = transpose_workspace(A->nrows, A->ncols, A->nnz);
  return CSRAD_OK;
}

extern "C" int csr_transpose(const csrad_csr* A, int32_t* rowptrT, int32_t* colindT, int32_t* perm,
                             void* work, size_t work_bytes, void* stream) {
  CSRAD_TRY(check_csr(A, false));
  if (!rowptrT || (A->nnz > 0 && (!colindT || !perm))) return CSRAD_EINVAL;
  return transpose_pattern(A->nrows, A->ncols, A->nnz, A->rowptr, A->colind, rowptrT, colindT,
                           perm, work, work_bytes, as_stream(stream));
}

extern "C" int csr_transpose_vals(const csrad_csr* A, const int32_t* perm, void* valsT,
                                  void* stream) {
  CSRAD_TRY(check_csr(A, true));
  if (A->nnz == 0) return CSRAD_OK;
  if (!perm || !valsT) return CSRAD_EINVAL;
  hipStream_t s = as_stream(stream);
  const unsigned g = grid_for(A->nnz, 256);
  if (A->dtype == CSRAD_F32)
    hipLaunchKernelGGL((k_gather_vals<float>), dim3(g), dim3(256), 0, s, A->nnz, perm,
                       static_cast<const float*>(A->vals), static_cast<float*>(valsT));
  else
    hipLaunchKernelGGL((k_gather_vals<double>), dim3(g), dim3(256), 0, s, A->nnz, perm,
                       static_cast<const double*>(A->vals), static_cast<double*>(valsT));
  return launch_status();
}
