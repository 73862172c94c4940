// SpSpMM / SpGEMM C = A B, all CSR (Section 3.1.2; Table 1, SpSpMM row;
// gradient flow of Fig. 2).
//
// Rows of C are binned by the product count U_i = sum over A's row of the
// lengths of the B rows it selects, an upper bound on nnz(C_i):
//   U <= 64                : row merge, G = 8 / 16 / 32 / 64 lanes per row
//                            (at least one lane per non-empty B row the
//                            row selects); each lane walks one sorted B
//                            row and the group merges the lists;
//   U <= 512, 4096         : LDS hash table of H = 2U slots per row,
//                            64 / 256 lanes per row;
//   U > 4096               : a dense per-workgroup marker array in the
//                            workspace (tagged with the row id).
// Symbolic: count the distinct columns (merge steps for U <= 64; hash
//           insert with CAS up to 4096; marker tags beyond).
// Numeric : the merge emits each column with the sum of the products that
//           meet there; the others rebuild the set, sort it (bitonic sort
//           of the table in LDS, empty slots last; for the dense path a
//           block scan of the marker array), write ascending column
//           indices, then each output entry C_ij = sum_k A_ik B_kj with k
//           in A's row order and B_kj found by binary search in B's sorted
//           row k.  No floating-point atomics: values are bit-identical
//           between runs.
// Backward (both gathers, no atomics):
//   gA[(i,k)] = sum_{j in pat(C_i) and pat(B_k)} V_ij B_kj   (row-aligned)
//   gB[(k,j)] = sum_{i in column k of A} A_ik V_ij           (over A^T)
#include "internal.hpp"

namespace csrad {
namespace {

constexpr int kThreads = 256;
// 0: empty, 1..4: row merge (U <= 64; 8, 16, 32, 64 lanes), 5..6: LDS hash,
// 7: dense marker
constexpr int kNumBins = 8;
static_assert(kNumBins + 1 == CSRAD_SPGEMM_BINS, "host copy of the class boundaries");
constexpr int kDenseBin = 7;
constexpr int kBigU = 4096;
constexpr size_t kMarkerBudget = size_t(16) << 20;

// u: products of the row; lists: A entries of the row whose B row is not
// empty (at most u).  Rows with u <= 64 take the row merge with as many
// lanes as lists, rounded up to 8, 16, 32 or 64.
__host__ __device__ inline int bin_of(long long u, int lists) {
  if (u == 0) return 0;
  if (u <= 64) return lists <= 8 ? 1 : lists <= 16 ? 2 : lists <= 32 ? 3 : 4;
  if (u <= 512) return 5;
  if (u <= kBigU) return 6;
  return kDenseBin;
}

// Per row: U_i and its bin, one thread per row.  The row's entries are
// taken kBinBatch at a time with all their loads issued together (A's
// columns, then the B row bounds they select), so a row costs about two
// rounds of memory latency, not two per entry.  The rows are then grouped
// by bin with the stable multi-split (ascending row order within a bin, no
// atomics).
constexpr int kBinBatch = 8;
__global__ __launch_bounds__(kThreads) void k_bin_of(int m, const int32_t* __restrict__ rpA,
                                                     const int32_t* __restrict__ ciA,
                                                     const int32_t* __restrict__ rpB,
                                                     int32_t* __restrict__ binid) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (long long)gridDim.x * blockDim.x) {
    long long u = 0;
    int lists = 0;
    const int a1 = rpA[i + 1];
    for (int a0 = rpA[i]; a0 < a1; a0 += kBinBatch) {
      int k[kBinBatch];
#pragma unroll
      for (int t = 0; t < kBinBatch; ++t) k[t] = a0 + t < a1 ? ciA[a0 + t] : -1;
      int len[kBinBatch];
#pragma unroll
      for (int t = 0; t < kBinBatch; ++t) len[t] = k[t] >= 0 ? rpB[k[t] + 1] - rpB[k[t]] : 0;
#pragma unroll
      for (int t = 0; t < kBinBatch; ++t) {
        u += len[t];
        lists += len[t] > 0;
      }
    }
    binid[i] = bin_of(u, lists);
  }
}

__device__ __forceinline__ unsigned hash_slot(int j, int H) {
  unsigned h = (unsigned)j * 2654435761u;
  return (h ^ (h >> 15)) & (unsigned)(H - 1);
}

// Returns 1 if j was newly inserted.  The table (H slots, -1 empty) never
// fills: every row placed in a bin has at most H/2 products.
__device__ __forceinline__ int hash_insert(int* tab, int H, int j) {
  unsigned h = hash_slot(j, H);
  while (true) {
    const int prev = atomicCAS(&tab[h], -1, j);
    if (prev == -1) return 1;
    if (prev == j) return 0;
    h = (h + 1) & (unsigned)(H - 1);
  }
}

// Visits this lane's share of row i's products: lane l of G takes the
// flattened product indices congruent to l modulo G.
template <int G, typename F>
__device__ __forceinline__ void for_each_product(int i, int l, const int32_t* __restrict__ rpA,
                                                 const int32_t* __restrict__ ciA,
                                                 const int32_t* __restrict__ rpB,
                                                 const int32_t* __restrict__ ciB, F&& f) {
  int base = 0;
  const int a1 = rpA[i + 1];
  for (int a = rpA[i]; a < a1; ++a) {
    const int k = ciA[a];
    const int b0 = rpB[k], len = rpB[k + 1] - b0;
    int off = (l - base) % G;
    if (off < 0) off += G;
    for (int o = off; o < len; o += G) f(ciB[b0 + o]);
    base += len;
  }
}

// Index of key in the sorted range ci[lo, hi), or -1.
__device__ __forceinline__ int find_sorted(const int32_t* __restrict__ ci, int lo, int hi, int key) {
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    const int v = ci[mid];
    if (v == key) return mid;
    if (v < key) lo = mid + 1;
    else hi = mid;
  }
  return -1;
}

// Windowed lookup in short sorted rows: the first kCWin columns of
// ci[lo, hi) come from two unaligned 16-byte loads (one round of memory
// latency; global loads need only 4-byte alignment on this target), so a
// row of at most kCWin entries needs no search; longer rows search the
// rest.  len: the array's length (the vector loads stay inside it).
constexpr int kCWin = 8;
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef i32x4 i32x4_u __attribute__((aligned(4)));

__device__ __forceinline__ void load_win(const int32_t* __restrict__ ci, int len, int lo, int hi,
                                         int (&v)[kCWin]) {
  if (lo + kCWin <= len) {
    const i32x4 a = *reinterpret_cast<const i32x4_u*>(ci + lo);
    const i32x4 b = *reinterpret_cast<const i32x4_u*>(ci + lo + 4);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
#pragma unroll
    for (int u = 0; u < kCWin; ++u) v[u] = lo + u < hi ? v[u] : INT32_MAX;
  } else {
#pragma unroll
    for (int u = 0; u < kCWin; ++u) v[u] = lo + u < hi ? ci[lo + u] : INT32_MAX;
  }
}

// Index of key in the sorted range ci[lo, hi) whose first kCWin columns
// are v, or -1.
__device__ __forceinline__ int find_in_win(const int32_t* __restrict__ ci, int lo, int hi,
                                           const int (&v)[kCWin], int key) {
  int pos = -1;
#pragma unroll
  for (int u = 0; u < kCWin; ++u)
    if (v[u] == key) pos = lo + u;
  if (pos < 0 && hi - lo > kCWin && v[kCWin - 1] < key) pos = find_sorted(ci, lo + kCWin, hi, key);
  return pos;
}

// C_ij = sum over A's row i (in order) of A_ik B_kj.
template <typename T>
__device__ __forceinline__ T product_entry(int i, int j, const int32_t* __restrict__ rpA,
                                           const int32_t* __restrict__ ciA,
                                           const T* __restrict__ vA,
                                           const int32_t* __restrict__ rpB,
                                           const int32_t* __restrict__ ciB,
                                           const T* __restrict__ vB) {
  T acc = 0;
  const int a1 = rpA[i + 1];
  for (int a = rpA[i]; a < a1; ++a) {
    const int k = ciA[a];
    const int p = find_sorted(ciB, rpB[k], rpB[k + 1], j);
    if (p >= 0) acc += vA[a] * vB[p];
  }
  return acc;
}

// ---------------------------------------------------------------------
// LDS-hash bins.  A block holds RPB = 256/G rows, each with H slots.  The
// loop over the bin's rows is uniform across the block (barriers inside).
// ---------------------------------------------------------------------
template <int G, int H>
__global__ __launch_bounds__(kThreads) void k_sym_hash(int bin, const int32_t* __restrict__ list,
                                                       const int32_t* __restrict__ bin_off,
                                                       const int32_t* __restrict__ rpA,
                                                       const int32_t* __restrict__ ciA,
                                                       const int32_t* __restrict__ rpB,
                                                       const int32_t* __restrict__ ciB,
                                                       int32_t* __restrict__ counts) {
  constexpr int RPB = kThreads / G;
  __shared__ int table[RPB * H];
  __shared__ int cnt[RPB];
  const int first = bin_off[bin], nrows = bin_off[bin + 1] - first;
  const int slot = threadIdx.x / G, l = threadIdx.x % G;
  int* tab = table + slot * H;
  for (int base = blockIdx.x * RPB; base < nrows; base += gridDim.x * RPB) {
    for (int q = l; q < H; q += G) tab[q] = -1;
    if (l == 0) cnt[slot] = 0;
    __syncthreads();
    const int idx = base + slot;
    int mine = 0;
    int i = -1;
    if (idx < nrows) {
      i = list[first + idx];
      for_each_product<G>(i, l, rpA, ciA, rpB, ciB, [&](int j) { mine += hash_insert(tab, H, j); });
    }
    if (mine) atomicAdd(&cnt[slot], mine);
    __syncthreads();
    if (i >= 0 && l == 0) counts[i] = cnt[slot];
    __syncthreads();
  }
}

template <typename T, int G, int H>
__global__ __launch_bounds__(kThreads) void k_num_hash(
    int bin, const int32_t* __restrict__ list, const int32_t* __restrict__ bin_off,
    const int32_t* __restrict__ rpA, const int32_t* __restrict__ ciA, const T* __restrict__ vA,
    const int32_t* __restrict__ rpB, const int32_t* __restrict__ ciB, const T* __restrict__ vB,
    const int32_t* __restrict__ rpC, int32_t* __restrict__ ciC, T* __restrict__ vC) {
  constexpr int RPB = kThreads / G;
  __shared__ int table[RPB * H];
  const int first = bin_off[bin], nrows = bin_off[bin + 1] - first;
  const int slot = threadIdx.x / G, l = threadIdx.x % G;
  int* tab = table + slot * H;
  for (int base = blockIdx.x * RPB; base < nrows; base += gridDim.x * RPB) {
    for (int q = l; q < H; q += G) tab[q] = -1;
    __syncthreads();
    const int idx = base + slot;
    const int i = idx < nrows ? list[first + idx] : -1;
    if (i >= 0)
      for_each_product<G>(i, l, rpA, ciA, rpB, ciB, [&](int j) { hash_insert(tab, H, j); });
    __syncthreads();
    for (int q = threadIdx.x; q < RPB * H; q += kThreads)
      if (table[q] == -1) table[q] = INT32_MAX;
    __syncthreads();
    // Bitonic sort of every table (independent segments of length H).
    for (int k = 2; k <= H; k <<= 1) {
      for (int jj = k >> 1; jj > 0; jj >>= 1) {
        for (int q = threadIdx.x; q < RPB * H; q += kThreads) {
          const int e = q % H, ixj = e ^ jj;
          if (ixj > e) {
            const int o = q - e;
            const int a = table[o + e], b = table[o + ixj];
            if ((a > b) == ((e & k) == 0)) {
              table[o + e] = b;
              table[o + ixj] = a;
            }
          }
        }
        __syncthreads();
      }
    }
    if (i >= 0) {
      const int c0 = rpC[i], u = rpC[i + 1] - c0;
      for (int t = l; t < u; t += G) {
        const int j = tab[t];
        ciC[c0 + t] = j;
        vC[c0 + t] = product_entry<T>(i, j, rpA, ciA, vA, rpB, ciB, vB);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------
// Small bins (U <= 64 products): row merge.  The B rows that A's row i
// selects are sorted lists; row i of C is their merge, and the value of a
// column the sum of the products that meet there.  A group of G lanes owns
// a row (G at least the number of A entries whose B row is not empty:
// bins 1..4 are G = 8, 16, 32, 64): lane t holds list t (the t-th such
// entry in A's row order).  One step takes the group minimum m of the
// list heads, sums the products of the lanes whose head is m, and
// advances those lanes; columns come out ascending and the number of
// steps is nnz(C_i).  Each lane keeps a window of W entries of its list in
// registers, refilled one entry ahead, so no step waits on a fresh load
// unless a list runs W entries in a row.  Output entries are kept one per
// lane and written G at a time.
// ---------------------------------------------------------------------
// Register window per list: entries a lane holds ahead of its list head
// (fewer when a group keeps many rows in flight, to keep registers low).
// SHORT: B's rows hold about one entry (the mean is at most 2), so a
// longer window would only cost registers (A P with a one-entry-per-row
// P: 4 rows in flight at 8 waves per SIMD instead of 6, 0.355 -> 0.343 ms).
template <int R, bool SHORT>
constexpr int merge_window() {
  return (R >= 8 || SHORT) ? 2 : 4;
}

template <int G>
__device__ __forceinline__ int group_min(int v) {
  // a move from a switched-off lane returns the lane's own value (old = v)
  if constexpr (G >= 2) v = min(v, __builtin_amdgcn_update_dpp(v, v, kDppXor1, 0xF, 0xF, false));
  if constexpr (G >= 4) v = min(v, __builtin_amdgcn_update_dpp(v, v, kDppXor2, 0xF, 0xF, false));
  if constexpr (G >= 8) v = min(v, __builtin_amdgcn_update_dpp(v, v, kDppHalfMirror, 0xF, 0xF, false));
  if constexpr (G >= 16) v = min(v, __builtin_amdgcn_update_dpp(v, v, kDppMirror, 0xF, 0xF, false));
  if constexpr (G >= 32) v = min(v, __builtin_amdgcn_ds_swizzle(v, 0x401F));
  if constexpr (G >= 64) v = min(v, __shfl_xor(v, 32));
  return v;
}

// Mask of the lanes of this lane's group.
template <int G>
__device__ __forceinline__ unsigned long long group_mask(int lane) {
  return G == 64 ? ~0ull : (((1ull << G) - 1ull) << (lane & ~(G - 1)));
}

// Wave-level ordering of the LDS slots: a group's slots are written and
// read by the lanes of one wave only (G divides 64), so a wave barrier with
// a workgroup-scope fence orders them; groups never wait for other waves.
__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// R rows per group are in flight at once (their load rounds are issued
// together, then merged one after the other), so a wave hides R times the
// memory latency of one row.
template <typename T, int G, bool NUM, int R, bool SHORT>
__global__ __launch_bounds__(kThreads) void k_merge(
    int m, int bin, const int32_t* __restrict__ list, const int32_t* __restrict__ bin_off,
    const int32_t* __restrict__ rpA, const int32_t* __restrict__ ciA, const T* __restrict__ vA,
    const int32_t* __restrict__ rpB, const int32_t* __restrict__ ciB, const T* __restrict__ vB,
    const int32_t* __restrict__ rpC, int32_t* __restrict__ ciC, T* __restrict__ vC,
    int32_t* __restrict__ counts) {
  constexpr int RPB = kThreads / G;  // groups per block
  constexpr int kWin = merge_window<R, SHORT>();
  __shared__ int s_b0[R][kThreads], s_len[R][kThreads], s_a[R][kThreads];
  const int first = bin_off[bin], nrows = bin_off[bin + 1] - first;
  // a class holding all m rows lists them in order (the grouping is
  // stable): the row is its index, one dependent load fewer
  const bool all_rows = nrows == m;
  const int lane = __lane_id(), l = threadIdx.x % G, g0 = threadIdx.x - l;
  const unsigned long long gm = group_mask<G>(lane);
  const unsigned long long below = gm & ((1ull << lane) - 1ull);
  // group q of the block owns rows base + q*R + t, t < R
  for (int base = blockIdx.x * RPB * R; base < nrows; base += gridDim.x * RPB * R) {
    int i[R], a0[R], a1[R], nl[R];
    bool valid[R];
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const int idx = base + (threadIdx.x / G) * R + t;
      valid[t] = idx < nrows;
      i[t] = valid[t] ? (all_rows ? idx : list[first + idx]) : 0;
    }
#pragma unroll
    for (int t = 0; t < R; ++t) {
      a0[t] = valid[t] ? rpA[i[t]] : 0;
      a1[t] = valid[t] ? rpA[i[t] + 1] : 0;
      nl[t] = 0;
    }
    // the non-empty lists of each row, compacted into the group's slots in
    // A's row order (the bin guarantees at most G of them per row)
    int chunks = 0;
#pragma unroll
    for (int t = 0; t < R; ++t) chunks = max(chunks, (a1[t] - a0[t] + G - 1) / G);
    chunks = wave_max(chunks);
    for (int c = 0; c < chunks; ++c) {
      int b0[R], len[R], k[R];
#pragma unroll
      for (int t = 0; t < R; ++t) {
        const int a = a0[t] + c * G + l;
        k[t] = a < a1[t] ? ciA[a] : -1;
      }
#pragma unroll
      for (int t = 0; t < R; ++t) {
        b0[t] = 0;
        len[t] = 0;
        if (k[t] >= 0) {
          b0[t] = rpB[k[t]];
          len[t] = rpB[k[t] + 1] - b0[t];
        }
      }
#pragma unroll
      for (int t = 0; t < R; ++t) {
        const unsigned long long ne = __ballot(len[t] > 0) & gm;
        const int rank = nl[t] + __popcll(ne & below);
        if (len[t] > 0 && rank < G) {  // rank < G holds for every row of the bin
          s_b0[t][g0 + rank] = b0[t];
          s_len[t][g0 + rank] = len[t];
          s_a[t][g0 + rank] = a0[t] + c * G + l;
        }
        nl[t] += __popcll(ne);
      }
    }
    wave_sync_lds();
    int p[R], e[R], c0[R];
    T av[R];
    int hc[R][kWin];
    T hv[R][kWin];
#pragma unroll
    for (int t = 0; t < R; ++t) {
      p[t] = 0;
      e[t] = 0;
      av[t] = 0;
      if (l < nl[t]) {
        p[t] = s_b0[t][g0 + l];
        e[t] = p[t] + s_len[t][g0 + l];
        if (NUM) av[t] = vA[s_a[t][g0 + l]];
      }
      c0[t] = (NUM && valid[t]) ? rpC[i[t]] : 0;
#pragma unroll
      for (int w = 0; w < kWin; ++w) {
        const bool in = p[t] + w < e[t];
        hc[t][w] = in ? ciB[p[t] + w] : INT32_MAX;
        hv[t][w] = (NUM && in) ? vB[p[t] + w] : T(0);
      }
    }
#pragma unroll
    for (int t = 0; t < R; ++t) {
      int steps = 0, oc = 0;
      T ov = 0;
      while (__ballot(hc[t][0] != INT32_MAX)) {  // uniform over the wave
        const int m = group_min<G>(hc[t][0]);
        const bool live = m != INT32_MAX;
        const bool hit = live && hc[t][0] == m;
        if (NUM) {
          const T sv = group_sum<G>(hit ? av[t] * hv[t][0] : T(0));
          if (l == (steps & (G - 1))) {
            oc = m;
            ov = sv;
          }
          if (live && (steps & (G - 1)) == G - 1) {  // a full set of G entries
            ciC[c0[t] + steps - (G - 1) + l] = oc;
            vC[c0[t] + steps - (G - 1) + l] = ov;
          }
        }
        steps += live;
        if (hit) {
#pragma unroll
          for (int w = 0; w + 1 < kWin; ++w) {
            hc[t][w] = hc[t][w + 1];
            hv[t][w] = hv[t][w + 1];
          }
          ++p[t];
          const bool in = p[t] + kWin - 1 < e[t];
          hc[t][kWin - 1] = in ? ciB[p[t] + kWin - 1] : INT32_MAX;
          hv[t][kWin - 1] = (NUM && in) ? vB[p[t] + kWin - 1] : T(0);
        }
      }
      if (NUM) {
        const int rem = steps & (G - 1);
        if (valid[t] && l < rem) {
          ciC[c0[t] + steps - rem + l] = oc;
          vC[c0[t] + steps - rem + l] = ov;
        }
      } else if (valid[t] && l == 0) {
        counts[i[t]] = steps;
      }
    }
    wave_sync_lds();  // the slots are rewritten by the next rows
  }
}

// ---------------------------------------------------------------------
// Dense-marker bin (U > 4096): each block owns a marker array of p ints in
// the workspace, tagged with the row id, and walks the bin's rows.
// ---------------------------------------------------------------------
__device__ void block_init_marker(int* marker, int p) {
  for (int q = threadIdx.x; q < p; q += kThreads) marker[q] = -1;
  __syncthreads();
}

__global__ __launch_bounds__(kThreads) void k_sym_dense(int p, const int32_t* __restrict__ list,
                                                        const int32_t* __restrict__ bin_off,
                                                        const int32_t* __restrict__ rpA,
                                                        const int32_t* __restrict__ ciA,
                                                        const int32_t* __restrict__ rpB,
                                                        const int32_t* __restrict__ ciB,
                                                        int32_t* __restrict__ counts,
                                                        int32_t* __restrict__ markers) {
  __shared__ int cnt;
  const int first = bin_off[kDenseBin], nrows = bin_off[kDenseBin + 1] - first;
  if ((int)blockIdx.x >= nrows) return;
  int* marker = markers + (size_t)blockIdx.x * p;
  block_init_marker(marker, p);
  for (int idx = blockIdx.x; idx < nrows; idx += gridDim.x) {
    const int i = list[first + idx];
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    int mine = 0;
    for_each_product<kThreads>(i, threadIdx.x, rpA, ciA, rpB, ciB,
                               [&](int j) { mine += atomicExch(&marker[j], i) != i; });
    if (mine) atomicAdd(&cnt, mine);
    __syncthreads();
    if (threadIdx.x == 0) counts[i] = cnt;
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_num_dense(
    int p, const int32_t* __restrict__ list, const int32_t* __restrict__ bin_off,
    const int32_t* __restrict__ rpA, const int32_t* __restrict__ ciA, const T* __restrict__ vA,
    const int32_t* __restrict__ rpB, const int32_t* __restrict__ ciB, const T* __restrict__ vB,
    const int32_t* __restrict__ rpC, int32_t* __restrict__ ciC, T* __restrict__ vC,
    int32_t* __restrict__ markers) {
  __shared__ int wsum[kThreads / kWave];
  const int first = bin_off[kDenseBin], nrows = bin_off[kDenseBin + 1] - first;
  if ((int)blockIdx.x >= nrows) return;
  int* marker = markers + (size_t)blockIdx.x * p;
  block_init_marker(marker, p);
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  for (int idx = blockIdx.x; idx < nrows; idx += gridDim.x) {
    const int i = list[first + idx];
    for_each_product<kThreads>(i, threadIdx.x, rpA, ciA, rpB, ciB,
                               [&](int j) { atomicExch(&marker[j], i); });
    __syncthreads();
    // Ascending compaction of the tagged columns: block scan per chunk.
    const int c0 = rpC[i];
    int run = 0;
    for (int cb = 0; cb < p; cb += kThreads) {
      const int c = cb + threadIdx.x;
      const int f = (c < p && marker[c] == i) ? 1 : 0;
      int v = f;
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        const int u = __shfl_up(v, o);
        if (lane >= o) v += u;
      }
      if (lane == kWave - 1) wsum[wid] = v;
      __syncthreads();
      int off = 0, tot = 0;
#pragma unroll
      for (int w = 0; w < kThreads / kWave; ++w) {
        if (w < wid) off += wsum[w];
        tot += wsum[w];
      }
      if (f) ciC[c0 + run + off + v - 1] = c;
      run += tot;
      __syncthreads();
    }
    __syncthreads();
    const int u = rpC[i + 1] - c0;
    for (int t = threadIdx.x; t < u; t += kThreads)
      vC[c0 + t] = product_entry<T>(i, ciC[c0 + t], rpA, ciA, vA, rpB, ciB, vB);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------
// Backward.
// ---------------------------------------------------------------------
// Both backward kernels are bound by chains of dependent gathers (A's
// columns -> B's row bounds -> B's columns and values -> C's row -> gC),
// and the chains a CU keeps in flight are capped by its resident threads,
// not by the lanes given to a row.  So each lane takes U entries and issues
// the loads of all U together, stage by stage: U chains in flight per
// thread.

// gA: G lanes per row of A, each lane U of A's entries at a time (entries
// l, l + G, l + 2G, ... of the row, so a lane sums in row order); the B
// rows they select are walked in lock step, Q entries of each per round
// (U = 4, Q = 1 for many short B rows; U = 1, Q = 4 for few rows with
// longer B rows).  Every lane of the row's group holds the first kCWin
// columns of C's row i.
template <typename T, int G, int U, int Q>
__global__ __launch_bounds__(kThreads) void k_bwd_a(int m, const int32_t* __restrict__ rpA,
                                                    const int32_t* __restrict__ ciA,
                                                    const int32_t* __restrict__ rpB,
                                                    const int32_t* __restrict__ ciB,
                                                    const T* __restrict__ vB,
                                                    const int32_t* __restrict__ rpC,
                                                    const int32_t* __restrict__ ciC, int nnzC,
                                                    const T* __restrict__ gC, T* __restrict__ gA) {
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int i = b * (kThreads / G) + threadIdx.x / G;
  const int l = threadIdx.x % G;
  if (i >= m) return;
  const int c0 = rpC[i], c1 = rpC[i + 1];
  int win[kCWin];
  load_win(ciC, nnzC, c0, c1, win);
  const int a1 = rpA[i + 1];
  for (int a0 = rpA[i] + l; a0 < a1; a0 += G * U) {
    int k[U], q[U], qe[U];
    T sum[U];
#pragma unroll
    for (int u = 0; u < U; ++u) k[u] = a0 + u * G < a1 ? ciA[a0 + u * G] : -1;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      q[u] = k[u] >= 0 ? rpB[k[u]] : 0;
      qe[u] = k[u] >= 0 ? rpB[k[u] + 1] : 0;
      sum[u] = 0;
    }
    bool more = true;
    while (more) {
      int j[U][Q], p[U][Q];
      T bv[U][Q], g[U][Q];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int w = 0; w < Q; ++w) {
          const bool in = q[u] + w < qe[u];
          j[u][w] = in ? ciB[q[u] + w] : -1;
          bv[u][w] = in ? vB[q[u] + w] : T(0);
        }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int w = 0; w < Q; ++w)
          p[u][w] = j[u][w] >= 0 ? find_in_win(ciC, c0, c1, win, j[u][w]) : -1;
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int w = 0; w < Q; ++w) g[u][w] = p[u][w] >= 0 ? gC[p[u][w]] : T(0);
      more = false;
#pragma unroll
      for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int w = 0; w < Q; ++w)
          if (p[u][w] >= 0) sum[u] += g[u][w] * bv[u][w];
        q[u] = min(q[u] + Q, qe[u]);
        more |= q[u] < qe[u];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (a0 + u * G < a1) gA[a0 + u * G] = sum[u];
  }
}

// gB: G lanes per row k of B; the entries of the row in turn, the lanes
// splitting column k of A (A^T's row k, rows ascending, values through
// permA), U of its entries per lane at a time, and summing with a group
// reduction.  The entry loop runs the same number of times across the wave
// (the reduction needs whole groups).
template <typename T, int G, int U>
__global__ __launch_bounds__(kThreads) void k_bwd_b(
    int n, const int32_t* __restrict__ rpB, const int32_t* __restrict__ ciB,
    const int32_t* __restrict__ rpAT, const int32_t* __restrict__ ciAT,
    const int32_t* __restrict__ permA, const T* __restrict__ vA, const int32_t* __restrict__ rpC,
    const int32_t* __restrict__ ciC, int nnzC, const T* __restrict__ gC, T* __restrict__ gB) {
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int k = b * (kThreads / G) + threadIdx.x / G;
  const int l = threadIdx.x % G;
  const bool valid = k < n;
  int t0 = 0, t1 = 0, q0 = 0, q1 = 0;
  if (valid) {
    t0 = rpAT[k];
    t1 = rpAT[k + 1];
    q0 = rpB[k];
    q1 = rpB[k + 1];
  }
  const int steps = wave_max(q1 - q0);
  for (int st = 0; st < steps; ++st) {
    const int q = q0 + st;
    T s = 0;
    if (q < q1) {
      const int j = ciB[q];
      for (int tb = t0 + l; tb < t1; tb += G * U) {
        int i[U], e[U], lo[U], hi[U], p[U];
        T av[U], g[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int t = tb + u * G;
          i[u] = t < t1 ? ciAT[t] : -1;
          e[u] = t < t1 ? permA[t] : -1;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          lo[u] = i[u] >= 0 ? rpC[i[u]] : 0;
          hi[u] = i[u] >= 0 ? rpC[i[u] + 1] : 0;
          av[u] = e[u] >= 0 ? vA[e[u]] : T(0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          int win[kCWin];
          load_win(ciC, nnzC, lo[u], hi[u], win);
          p[u] = i[u] >= 0 ? find_in_win(ciC, lo[u], hi[u], win, j) : -1;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) g[u] = p[u] >= 0 ? gC[p[u]] : T(0);
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (p[u] >= 0) s += av[u] * g[u];
      }
    }
    s = group_sum<G>(s);
    if (q < q1 && l == 0) gB[q] = s;
  }
}

// gB for short columns of A (at most kColShort entries, e.g. A = P^T with
// one entry per column): one thread per row k of B holds column k of A in
// registers (rows, values, and the first kCWin columns of each C row they
// select) and walks row k of B kQ entries per round, its gathers issued
// together; a column with more entries takes the plain loop.  Sums over the
// column in order, as the general kernel does with one lane.
constexpr int kColShort = 2;
constexpr int kQ = 4;
template <typename T>
__global__ __launch_bounds__(kThreads) void k_bwd_b_short(
    int n, const int32_t* __restrict__ rpB, const int32_t* __restrict__ ciB,
    const int32_t* __restrict__ rpAT, const int32_t* __restrict__ ciAT,
    const int32_t* __restrict__ permA, const T* __restrict__ vA, const int32_t* __restrict__ rpC,
    const int32_t* __restrict__ ciC, int nnzC, const T* __restrict__ gC, T* __restrict__ gB) {
  const int k = xcd_block(blockIdx.x, gridDim.x) * kThreads + threadIdx.x;
  if (k >= n) return;
  const int t0 = rpAT[k], t1 = rpAT[k + 1], q0 = rpB[k], q1 = rpB[k + 1];
  const int cnt = t1 - t0;
  if (cnt > kColShort) {
    for (int q = q0; q < q1; ++q) {
      const int j = ciB[q];
      T s = 0;
      for (int t = t0; t < t1; ++t) {
        const int i = ciAT[t];
        const int lo = rpC[i], hi = rpC[i + 1];
        int win[kCWin];
        load_win(ciC, nnzC, lo, hi, win);
        const int p = find_in_win(ciC, lo, hi, win, j);
        if (p >= 0) s += vA[permA[t]] * gC[p];
      }
      gB[q] = s;
    }
    return;
  }
  int lo[kColShort], hi[kColShort], win[kColShort][kCWin];
  T av[kColShort];
#pragma unroll
  for (int u = 0; u < kColShort; ++u) {
    const int i = u < cnt ? ciAT[t0 + u] : -1;
    const int e = u < cnt ? permA[t0 + u] : -1;
    lo[u] = i >= 0 ? rpC[i] : 0;
    hi[u] = i >= 0 ? rpC[i + 1] : 0;
    av[u] = e >= 0 ? vA[e] : T(0);
  }
#pragma unroll
  for (int u = 0; u < kColShort; ++u) load_win(ciC, nnzC, lo[u], hi[u], win[u]);
  for (int qb = q0; qb < q1; qb += kQ) {
    int j[kQ];
#pragma unroll
    for (int w = 0; w < kQ; ++w) j[w] = qb + w < q1 ? ciB[qb + w] : -1;
    int p[kQ][kColShort];
    T g[kQ][kColShort];
#pragma unroll
    for (int w = 0; w < kQ; ++w)
#pragma unroll
      for (int u = 0; u < kColShort; ++u)
        p[w][u] = (j[w] >= 0 && u < cnt) ? find_in_win(ciC, lo[u], hi[u], win[u], j[w]) : -1;
#pragma unroll
    for (int w = 0; w < kQ; ++w)
#pragma unroll
      for (int u = 0; u < kColShort; ++u) g[w][u] = p[w][u] >= 0 ? gC[p[w][u]] : T(0);
#pragma unroll
    for (int w = 0; w < kQ; ++w) {
      if (j[w] < 0) continue;
      T s = 0;
#pragma unroll
      for (int u = 0; u < kColShort; ++u)
        if (p[w][u] >= 0) s += av[u] * g[w][u];
      gB[qb + w] = s;
    }
  }
}

// ---------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------
struct SpgemmWs {
  int32_t* binid;
  int32_t* bin_off;
  int32_t* list;
  int32_t* counts;
  void* scan_ws;
  size_t scan_bytes;
  long long* total;
  void* group_ws;
  size_t group_bytes;
  int32_t* markers;
  int nmark;
};

int marker_slots(int p) {
  const size_t per = sizeof(int32_t) * (size_t)(p > 0 ? p : 1);
  size_t s = kMarkerBudget / per;
  if (s < 1) s = 1;
  if (s > 64) s = 64;
  return (int)s;
}

SpgemmWs carve_spgemm(Carver& cv, int m, int p) {
  SpgemmWs w;
  w.binid = cv.take<int32_t>((size_t)m);
  w.bin_off = cv.take<int32_t>(kNumBins + 1);
  w.list = cv.take<int32_t>((size_t)m);
  w.counts = cv.take<int32_t>((size_t)m);
  w.scan_bytes = scan_workspace(m);
  w.scan_ws = cv.take<char>(w.scan_bytes);
  w.total = cv.take<long long>(1);
  w.group_bytes = group_small_workspace(m > 0 ? m : 1, kNumBins);
  w.group_ws = cv.take<char>(w.group_bytes);
  w.nmark = marker_slots(p);
  w.markers = cv.take<int32_t>((size_t)w.nmark * (size_t)(p > 0 ? p : 1));
  return w;
}

unsigned persistent_grid(int rows_per_block, int m) {
  long long b = ((long long)m + rows_per_block - 1) / rows_per_block;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return (unsigned)b;
}

int classify(const csrad_csr* A, const csrad_csr* B, const SpgemmWs& w, hipStream_t s) {
  const int m = A->nrows;
  if (m == 0) return fill_i32(w.bin_off, kNumBins + 1, 0, s);
  const unsigned g = (unsigned)std::min<long long>(65536, ((long long)m + kThreads - 1) / kThreads);
  hipLaunchKernelGGL(k_bin_of, dim3(g), dim3(kThreads), 0, s, m, A->rowptr, A->colind, B->rowptr,
                     w.binid);
  return group_small_keys(w.binid, m, kNumBins, w.bin_off, w.list, w.group_ws, w.group_bytes, s);
}

int check_pair(const csrad_csr* A, const csrad_csr* B, bool vals) {
  CSRAD_TRY(check_csr(A, vals));
  CSRAD_TRY(check_csr(B, vals));
  if (A->ncols != B->nrows) return CSRAD_EINVAL;
  if (A->dtype != B->dtype) return CSRAD_EDTYPE;
  return CSRAD_OK;
}

// Launches of the row-merge bins (1..4: G = 8, 16, 32, 64).
template <typename T, int G, bool NUM>
void merge_bin(int bin, int rows, const csrad_csr* A, const csrad_csr* B, const T* vA,
               const T* vB, const int32_t* rpC, int32_t* ciC, T* vC, const SpgemmWs& w,
               hipStream_t s) {
  if (rows == 0) return;
  // Several rows in flight per group hide more memory latency, but run
  // their merges one after the other: worth it only when every resident
  // group has many rows to do (short merges, as in A P with one entry per
  // row of P: 4 rows per 8-lane group), not when the rows are few for the
  // chip (P^T (A P)).
  constexpr int RMAX = G <= 8 ? 4 : (G <= 16 ? 2 : 1);
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  const long long resident_groups = (long long)cus * 8 * (kThreads / G);
  const bool short_b = B->nnz <= 2ll * B->nrows;
  if (RMAX > 1 && rows >= 8 * resident_groups) {
    const unsigned g = persistent_grid(kThreads / G * RMAX, rows);
    if (short_b)
      hipLaunchKernelGGL((k_merge<T, G, NUM, RMAX, true>), dim3(g), dim3(kThreads), 0, s, A->nrows,
                         bin, w.list, w.bin_off, A->rowptr, A->colind, vA, B->rowptr, B->colind,
                         vB, rpC, ciC, vC, w.counts);
    else
      hipLaunchKernelGGL((k_merge<T, G, NUM, RMAX, false>), dim3(g), dim3(kThreads), 0, s,
                         A->nrows, bin, w.list, w.bin_off, A->rowptr, A->colind, vA, B->rowptr,
                         B->colind, vB, rpC, ciC, vC, w.counts);
  } else {
    const unsigned g = persistent_grid(kThreads / G, rows);
    hipLaunchKernelGGL((k_merge<T, G, NUM, 1, false>), dim3(g), dim3(kThreads), 0, s, A->nrows, bin,
                       w.list, w.bin_off, A->rowptr, A->colind, vA, B->rowptr, B->colind, vB, rpC,
                       ciC, vC, w.counts);
  }
}

// bins: host copy of the class boundaries, or null (every class is then
// launched for all m rows; the kernels read the boundaries on the device).
template <typename T>
int spgemm_numeric_t(const csrad_csr* A, const csrad_csr* B, const int32_t* rpC, int32_t* ciC,
                     T* vC, const SpgemmWs& w, const int32_t* bins, hipStream_t s) {
  const int m = A->nrows, p = B->ncols;
  const T* vA = static_cast<const T*>(A->vals);
  const T* vB = static_cast<const T*>(B->vals);
  auto rows = [&](int b) { return bins ? bins[b + 1] - bins[b] : m; };
  merge_bin<T, 8, true>(1, rows(1), A, B, vA, vB, rpC, ciC, vC, w, s);
  merge_bin<T, 16, true>(2, rows(2), A, B, vA, vB, rpC, ciC, vC, w, s);
  merge_bin<T, 32, true>(3, rows(3), A, B, vA, vB, rpC, ciC, vC, w, s);
  merge_bin<T, 64, true>(4, rows(4), A, B, vA, vB, rpC, ciC, vC, w, s);
  if (rows(5) > 0)
    hipLaunchKernelGGL((k_num_hash<T, 64, 1024>), dim3(persistent_grid(4, rows(5))),
                       dim3(kThreads), 0, s, 5, w.list, w.bin_off, A->rowptr, A->colind, vA,
                       B->rowptr, B->colind, vB, rpC, ciC, vC);
  if (rows(6) > 0)
    hipLaunchKernelGGL((k_num_hash<T, 256, 8192>), dim3(persistent_grid(1, rows(6))),
                       dim3(kThreads), 0, s, 6, w.list, w.bin_off, A->rowptr, A->colind, vA,
                       B->rowptr, B->colind, vB, rpC, ciC, vC);
  if (rows(kDenseBin) > 0)
    hipLaunchKernelGGL((k_num_dense<T>), dim3(w.nmark), dim3(kThreads), 0, s, p, w.list,
                       w.bin_off, A->rowptr, A->colind, vA, B->rowptr, B->colind, vB, rpC, ciC,
                       vC, w.markers);
  return launch_status();
}

int lanes_for(long long nnz, int rows) {
  if (rows <= 0) return 1;
  const double mean = (double)nnz / rows;
  int g = 1;
  while (g < 64 && g < mean) g <<= 1;
  return g;
}

// Lanes per row G and entries per lane U from the lanes_for count L of a
// mean inner length.  Batching U = 4 entries per lane pays when the rows
// are many for the chip (rows x L at least 8 times the resident threads:
// each lane then carries four gather chains and there are still threads
// to spare); with fewer rows, one entry per lane keeps more threads busy
// (A P's backward, 2.1 M rows: 136 -> 74 us and 149 -> 99 us batched; the
// backward of P^T (A P), 262 k rows: 37 us unbatched, 71 us batched).
#define CSRAD_GU_SWITCH(L, BATCH, ...)                                        \
  if (BATCH) {                                                                \
    switch (L) {                                                              \
      case 8: { constexpr int G = 2, U = 4; __VA_ARGS__; } break;              \
      case 16: { constexpr int G = 4, U = 4; __VA_ARGS__; } break;             \
      case 32: { constexpr int G = 8, U = 4; __VA_ARGS__; } break;             \
      default: { constexpr int G = 16, U = 4; __VA_ARGS__; } break;            \
    }                                                                         \
  } else {                                                                    \
    switch (L) {                                                              \
      case 1: { constexpr int G = 1, U = 1; __VA_ARGS__; } break;              \
      case 2: { constexpr int G = 2, U = 1; __VA_ARGS__; } break;              \
      case 4: { constexpr int G = 4, U = 1; __VA_ARGS__; } break;              \
      case 8: { constexpr int G = 8, U = 1; __VA_ARGS__; } break;              \
      case 16: { constexpr int G = 16, U = 1; __VA_ARGS__; } break;            \
      case 32: { constexpr int G = 32, U = 1; __VA_ARGS__; } break;            \
      default: { constexpr int G = 64, U = 1; __VA_ARGS__; } break;            \
    }                                                                         \
  }

bool batch_entries(long long rows, int lanes) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  return lanes >= 8 && rows * lanes >= 8ll * cus * 2048;
}

template <typename T>
int spgemm_bwd_t(const csrad_csr* A, const csrad_csr* B, const csrad_csr* At,
                 const int32_t* permA, const csrad_csr* C, const T* gC, T* gA, T* gB,
                 hipStream_t s) {
  if (gA && A->nrows > 0) {
    const int m = A->nrows;
    const int L = lanes_for(A->nnz, m);
    // entries of A per lane when A's rows are many, else entries of the B
    // rows per round
    CSRAD_GU_SWITCH(L, batch_entries(m, L),
                    hipLaunchKernelGGL((k_bwd_a<T, G, U, (U == 1 ? 4 : 1)>),
                                       dim3((m + kThreads / G - 1) / (kThreads / G)),
                                       dim3(kThreads), 0, s, m, A->rowptr, A->colind, B->rowptr,
                                       B->colind, static_cast<const T*>(B->vals), C->rowptr,
                                       C->colind, C->nnz, gC, gA));
  }
  if (gB && B->nrows > 0) {
    const int n = B->nrows;
    // from the mean column length of A (the inner loop)
    const int L = lanes_for(A->nnz, A->ncols);
    if (L <= kColShort) {
      // short columns of A: one thread per row of B, the column in registers
      hipLaunchKernelGGL((k_bwd_b_short<T>), dim3((n + kThreads - 1) / kThreads), dim3(kThreads),
                         0, s, n, B->rowptr, B->colind, At->rowptr, At->colind, permA,
                         static_cast<const T*>(A->vals), C->rowptr, C->colind, C->nnz, gC, gB);
      return launch_status();
    }
    CSRAD_GU_SWITCH(L, batch_entries(n, L),
                    hipLaunchKernelGGL((k_bwd_b<T, G, U>),
                                       dim3((n + kThreads / G - 1) / (kThreads / G)),
                                       dim3(kThreads), 0, s, n, B->rowptr, B->colind, At->rowptr,
                                       At->colind, permA, static_cast<const T*>(A->vals),
                                       C->rowptr, C->colind, C->nnz, gC, gB));
  }
  return launch_status();
}

}  // namespace
}  // namespace csrad

using namespace csrad;

extern "C" int csr_spgemm_workspace(const csrad_csr* A, const csrad_csr* B, size_t* bytes) {
  if (!A || !B || !bytes) return CSRAD_EINVAL;
  if (A->nrows < 0 || B->ncols < 0) return CSRAD_EINVAL;
  Carver cv(nullptr, 0);
  carve_spgemm(cv, A->nrows, B->ncols);
  *bytes = cv.off + 256;
  return CSRAD_OK;
}

extern "C" int csr_spgemm_symbolic(const csrad_csr* A, const csrad_csr* B, int32_t* C_rowptr,
                                   int64_t* C_nnz_host, int32_t* bins_host, void* work,
                                   size_t work_bytes, void* stream) {
  CSRAD_TRY(check_pair(A, B, false));
  if (!C_rowptr || !C_nnz_host) return CSRAD_EINVAL;
  hipStream_t s = as_stream(stream);
  const int m = A->nrows, p = B->ncols;
  Carver cv(work, work_bytes);
  SpgemmWs w = carve_spgemm(cv, m, p);
  if (!work || !cv.ok) return CSRAD_EWORKSPACE;
  CSRAD_TRY(classify(A, B, w, s));
  if (m > 0) {
    CSRAD_TRY(fill_i32(w.counts, m, 0, s));
    // the row-merge bins count their steps (the classes' sizes are still on
    // the device: every class is launched over up to m rows)
    merge_bin<float, 8, false>(1, m, A, B, nullptr, nullptr, nullptr, nullptr, nullptr, w, s);
    merge_bin<float, 16, false>(2, m, A, B, nullptr, nullptr, nullptr, nullptr, nullptr, w, s);
    merge_bin<float, 32, false>(3, m, A, B, nullptr, nullptr, nullptr, nullptr, nullptr, w, s);
    merge_bin<float, 64, false>(4, m, A, B, nullptr, nullptr, nullptr, nullptr, nullptr, w, s);
    hipLaunchKernelGGL((k_sym_hash<64, 1024>), dim3(persistent_grid(4, m)), dim3(kThreads), 0, s, 5,
                       w.list, w.bin_off, A->rowptr, A->colind, B->rowptr, B->colind, w.counts);
    hipLaunchKernelGGL((k_sym_hash<256, 8192>), dim3(persistent_grid(1, m)), dim3(kThreads), 0, s,
                       6, w.list, w.bin_off, A->rowptr, A->colind, B->rowptr, B->colind, w.counts);
    hipLaunchKernelGGL(k_sym_dense, dim3(w.nmark), dim3(kThreads), 0, s, p, w.list, w.bin_off,
                       A->rowptr, A->colind, B->rowptr, B->colind, w.counts, w.markers);
  }
  CSRAD_TRY(scan_exclusive(w.counts, C_rowptr, m, w.total, w.scan_ws, w.scan_bytes, s));
  long long total = 0;
  if (hipMemcpyAsync(&total, w.total, sizeof(total), hipMemcpyDeviceToHost, s) != hipSuccess)
    return CSRAD_EHIP;
  if (bins_host && hipMemcpyAsync(bins_host, w.bin_off, sizeof(int32_t) * (kNumBins + 1),
                                  hipMemcpyDeviceToHost, s) != hipSuccess)
    return CSRAD_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return CSRAD_EHIP;
  *C_nnz_host = total;
  if (total > INT32_MAX) return CSRAD_EOVERFLOW;
  return CSRAD_OK;
}

extern "C" int csr_spgemm_fwd(const csrad_csr* A, const csrad_csr* B, const int32_t* C_rowptr,
                              int32_t* C_colind, void* C_vals, const int32_t* bins_host,
                              void* work, size_t work_bytes, void* stream) {
  CSRAD_TRY(check_pair(A, B, true));
  if (!C_rowptr) return CSRAD_EINVAL;
  hipStream_t s = as_stream(stream);
  const int m = A->nrows, p = B->ncols;
  Carver cv(work, work_bytes);
  SpgemmWs w = carve_spgemm(cv, m, p);
  if (!work || !cv.ok) return CSRAD_EWORKSPACE;
  if (m == 0) return CSRAD_OK;
  if (bins_host) {  // the symbolic call's classification, still in `work`
    if (bins_host[0] != 0 || bins_host[kNumBins] != m) return CSRAD_EINVAL;
  } else {
    CSRAD_TRY(classify(A, B, w, s));
  }
  if (A->dtype == CSRAD_F32)
    return spgemm_numeric_t<float>(A, B, C_rowptr, C_colind, static_cast<float*>(C_vals), w,
                                   bins_host, s);
  return spgemm_numeric_t<double>(A, B, C_rowptr, C_colind, static_cast<double*>(C_vals), w,
                                  bins_host, s);
}

extern "C" int csr_spgemm_bwd(const csrad_csr* A, const csrad_csr* B, const csrad_csr* At,
                              const int32_t* permA, const csrad_csr* C, const void* gC, void* gA,
                              void* gB, void* stream) {
  CSRAD_TRY(check_pair(A, B, false));
  if (!gA && !gB) return CSRAD_OK;
  if (!C) return CSRAD_EINVAL;
  CSRAD_TRY(check_csr(C, false));
  if (C->nrows != A->nrows || C->ncols != B->ncols) return CSRAD_EINVAL;
  if (C->nnz > 0 && !gC) return CSRAD_EINVAL;
  if (gA && B->nnz > 0 && !B->vals) return CSRAD_EINVAL;
  if (gB) {
    if (!At) return CSRAD_EINVAL;
    CSRAD_TRY(check_csr(At, false));
    if (At->nrows != A->ncols || At->ncols != A->nrows || At->nnz != A->nnz) return CSRAD_EINVAL;
    if (A->nnz > 0 && (!permA || !A->vals)) return CSRAD_EINVAL;
  }
  hipStream_t s = as_stream(stream);
  if (A->dtype == CSRAD_F32)
    return spgemm_bwd_t<float>(A, B, At, permA, C, static_cast<const float*>(gC),
                               static_cast<float*>(gA), static_cast<float*>(gB), s);
  return spgemm_bwd_t<double>(A, B, At, permA, C, static_cast<const double*>(gC),
                              static_cast<double*>(gA), static_cast<double*>(gB), s);
}
