// SpSpMM / SpGEMM C = A B, all CSR (Section 3.1.2; Table 1, SpSpMM row;
// gradient flow of Fig. 2).
//
// Rows of C are binned by the product count U_i = sum over A's row of the
// lengths of the B rows it selects, an upper bound on nnz(C_i):
//   U <= 8, 16, 32, 64     : 8 / 16 / 32 / 64 lanes per row, one product
//                            per lane, sorted across the lanes in registers;
//   U <= 512, 4096         : LDS hash table of H = 2U slots per row,
//                            64 / 256 lanes per row;
//   U > 4096               : a dense per-workgroup marker array in the
//                            workspace (tagged with the row id).
// Symbolic: count the distinct columns (run heads after the lane sort for
//           U <= 32; hash insert with CAS up to 4096; marker tags beyond).
// Numeric : small bins sum each run of equal columns in k order; the
//           others rebuild the set, sort it (bitonic sort of the table in
//           LDS, empty slots last; for the dense path a block scan of the
//           marker array), write ascending column indices, then each
//           output entry C_ij = sum_k A_ik B_kj with k in A's row order and
//           B_kj found by binary search in B's sorted row k.  No floating
//           point atomics: values are bit-identical between runs.
// Backward (both gathers, no atomics):
//   gA[(i,k)] = sum_{j in pat(C_i) and pat(B_k)} V_ij B_kj   (row-aligned)
//   gB[(k,j)] = sum_{i in column k of A} A_ik V_ij           (over A^T)
#include "internal.hpp"

namespace csrad {
namespace {

constexpr int kThreads = 256;
// 0: empty, 1..4: lanes (U <= 8, 16, 32, 64), 5..6: LDS hash, 7: dense marker
constexpr int kNumBins = 8;
static_assert(kNumBins + 1 == CSRAD_SPGEMM_BINS, "host copy of the class boundaries");
constexpr int kDenseBin = 7;
constexpr int kBigU = 4096;
constexpr size_t kMarkerBudget = size_t(16) << 20;

__host__ __device__ inline int bin_of(long long u) {
  if (u == 0) return 0;
  if (u <= 8) return 1;
  if (u <= 16) return 2;
  if (u <= 32) return 3;
  if (u <= 64) return 4;
  if (u <= 512) return 5;
  if (u <= kBigU) return 6;
  return kDenseBin;
}

// Per row: U_i and its bin.  The rows are then grouped by bin with the
// stable multi-split (ascending row order within a bin, no atomics).
__global__ __launch_bounds__(kThreads) void k_bin_of(int m, const int32_t* __restrict__ rpA,
                                                     const int32_t* __restrict__ ciA,
                                                     const int32_t* __restrict__ rpB,
                                                     int32_t* __restrict__ binid) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
    long long u = 0;
    for (int a = rpA[i]; a < rpA[i + 1]; ++a) {
      const int k = ciA[a];
      u += rpB[k + 1] - rpB[k];
    }
    binid[i] = bin_of(u);
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
// Small bins (U <= G, G = 16 or 64): G lanes per row, no LDS.  Lane l holds
// the row's l-th product in k order (A's row order, then B's row order);
// the G keys (column, product index) are sorted across the lanes by a
// register bitonic network, so equal columns form runs ordered by k.  A
// run's first lane ("head") stands for one output entry: the heads count
// the row (symbolic), give each entry its rank, and sum their run's
// products in lane order, i.e. k ascending (numeric).
// ---------------------------------------------------------------------
__device__ __forceinline__ unsigned long long shfl_xor_key(unsigned long long v, int m) {
  const unsigned lo = (unsigned)__shfl_xor((int)(unsigned)v, m);
  const unsigned hi = (unsigned)__shfl_xor((int)(unsigned)(v >> 32), m);
  return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ unsigned shfl_xor_key(unsigned v, int m) {
  return (unsigned)__shfl_xor((int)v, m);
}

// Lane exchanges within rows of 16 lanes through DPP moves (no LDS
// crossbar): quad permutes, the half-row and row mirrors, and row shifts.
template <int CTRL>
__device__ __forceinline__ unsigned dpp_key(unsigned v) {
  return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ unsigned long long dpp_key(unsigned long long v) {
  const unsigned lo = dpp_key<CTRL>((unsigned)v), hi = dpp_key<CTRL>((unsigned)(v >> 32));
  return ((unsigned long long)hi << 32) | lo;
}

// The value of lane + 1 across the whole wave (DPP wave_shl:1; the last
// lane reads 0).
__device__ __forceinline__ float wave_next(float v) {
  return __uint_as_float(dpp_key<0x130>(__float_as_uint(v)));
}
__device__ __forceinline__ double wave_next(double v) {
  return __longlong_as_double((long long)dpp_key<0x130>((unsigned long long)__double_as_longlong(v)));
}

// The key of lane l ^ M, l the lane's index in its aligned group.  Both
// row shifts of the M = 4 and M = 8 cases run on every lane before the
// select: a DPP move reads nothing from lanes that are switched off.
template <int M, typename K>
__device__ __forceinline__ K partner_key(K key, int l) {
  if constexpr (M == 1) {
    return dpp_key<0xB1>(key);  // quad_perm [1,0,3,2]
  } else if constexpr (M == 2) {
    return dpp_key<0x4E>(key);  // quad_perm [2,3,0,1]
  } else if constexpr (M == 3) {
    return dpp_key<0x1B>(key);  // quad_perm [3,2,1,0]
  } else if constexpr (M == 4 || M == 8) {
    const K down = dpp_key<0x110 + M>(key);  // row_shr:M, lane l - M
    const K up = dpp_key<0x100 + M>(key);    // row_shl:M, lane l + M
    return (l & M) ? down : up;
  } else if constexpr (M == 7) {
    return dpp_key<0x141>(key);  // row_half_mirror
  } else if constexpr (M == 15) {
    return dpp_key<0x140>(key);  // row_mirror
  } else {
    return shfl_xor_key(key, M);
  }
}

template <typename K>
__device__ __forceinline__ K keep(K key, K other, bool keep_min) {
  return keep_min ? (other < key ? other : key) : (other > key ? other : key);
}

// Half-cleaner steps j = J, J/2, ..., 1 of a bitonic merge (ascending).
template <int J, typename K>
__device__ __forceinline__ K merge_steps(K key, int l) {
  if constexpr (J >= 1) {
    key = keep(key, partner_key<J>(key, l), (l & J) == 0);
    return merge_steps<J / 2>(key, l);
  } else {
    return key;
  }
}

// Stages KB = 2, 4, ..., G of the bitonic network in its mirror form: each
// stage compares lane l with l ^ (KB - 1) (the mirror in its KB-block,
// lower half keeps the minimum), then half-cleans with l ^ KB/4, ..., l ^ 1;
// every comparator is ascending, and the exchanges within 16 lanes are DPP
// moves.
template <int KB, int G, typename K>
__device__ __forceinline__ K sort_stages(K key, int l) {
  if constexpr (KB <= G) {
    key = keep(key, partner_key<KB - 1>(key, l), (l & (KB >> 1)) == 0);
    key = merge_steps<KB / 4>(key, l);
    return sort_stages<KB * 2, G>(key, l);
  } else {
    return key;
  }
}

// Ascending sort of one key per lane over aligned groups of G lanes.
template <int G, typename K>
__device__ __forceinline__ K group_sort(K key, int l) {
  return sort_stages<2, G>(key, l);
}

// Inclusive prefix sum over an aligned group of G lanes.  Groups within one
// row of 16 lanes shift by DPP; wider groups shuffle (a row shift does not
// cross into the next row, which their lanes would need).
template <int O, int G>
__device__ __forceinline__ int scan_up(int inc, int l) {
  if constexpr (O < G) {
    int t;
    if constexpr (G <= 16)
      t = __builtin_amdgcn_update_dpp(0, inc, 0x110 + O, 0xF, 0xF, false);  // row_shr:O
    else
      t = __shfl_up(inc, O, G);
    if (l >= O) inc += t;
    return scan_up<O * 2, G>(inc, l);
  } else {
    return inc;
  }
}

// The l-th product of row i, found by the G lanes of the row together: A's
// row is taken G entries at a time, each lane loads one entry and the
// length of the B row it selects, a scan over the group gives every
// entry's first product, and each lane finds the entry holding its product
// by binary search over the scan.  col = INT32_MAX when the row has at most
// l products.  Every lane of the wave must reach the call.
template <int G>
__device__ __forceinline__ void lane_product(int i, bool valid, int l,
                                             const int32_t* __restrict__ rpA,
                                             const int32_t* __restrict__ ciA,
                                             const int32_t* __restrict__ rpB,
                                             const int32_t* __restrict__ ciB, int& col, int& ea,
                                             int& eb) {
  col = INT32_MAX;
  ea = eb = -1;
  const int gbase = __lane_id() & ~(G - 1);
  int a0 = 0, a1 = 0;
  if (valid) {
    a0 = rpA[i];
    a1 = rpA[i + 1];
  }
  const int chunks = wave_max((a1 - a0 + G - 1) / G);
  int before = 0;  // products of the row's earlier chunks
  for (int c = 0; c < chunks; ++c) {
    const int a = a0 + c * G + l;
    int b0 = 0, len = 0;
    if (a < a1) {
      const int k = ciA[a];
      b0 = rpB[k];
      len = rpB[k + 1] - b0;
    }
    const int inc = scan_up<1, G>(len, l);
    const int total = __shfl(inc, gbase + G - 1);
    const int pidx = l - before;  // this lane's product within the chunk
    // first t with inc[t] > pidx (lanes without a product search too)
    int lo = 0, hi = G - 1;
#pragma unroll
    for (int st = G; st > 1; st >>= 1) {
      const int mid = (lo + hi) >> 1;
      const int v = __shfl(inc, gbase + mid);
      if (v > pidx) hi = mid;
      else lo = mid + 1;
    }
    const int t = lo;
    const int st_b0 = __shfl(b0, gbase + t);
    const int st_ex = __shfl(inc - len, gbase + t);
    if (pidx >= 0 && pidx < total) {
      ea = a0 + c * G + t;
      eb = st_b0 + (pidx - st_ex);
      col = ciB[eb];
    }
    before += total;
  }
}

// Mask of the lanes of this lane's group.
template <int G>
__device__ __forceinline__ unsigned long long group_mask(int lane) {
  return G == 64 ? ~0ull : (((1ull << G) - 1ull) << (lane & ~(G - 1)));
}

// Sort key of (column, product index): 32 bits when the column fits in
// 32 - log2(G) bits, else 64.
template <int G>
constexpr int log2_of() {
  return G == 8 ? 3 : G == 16 ? 4 : G == 32 ? 5 : 6;
}

template <int G, typename K>
__device__ __forceinline__ K make_key(int col, int l) {
  constexpr int LG = log2_of<G>();
  if (sizeof(K) == 4)
    return col == INT32_MAX ? (K)0xffffffffu : (K)(((unsigned)col << LG) | (unsigned)l);
  return (K)(((unsigned long long)(unsigned)col << 32) | (unsigned)l);
}
template <int G, typename K>
__device__ __forceinline__ int key_col(K key) {
  constexpr int LG = log2_of<G>();
  if (sizeof(K) == 4) return key == (K)0xffffffffu ? INT32_MAX : (int)((unsigned)key >> LG);
  return (int)((unsigned long long)key >> 32);
}
template <int G, typename K>
__device__ __forceinline__ int key_idx(K key) {
  if (sizeof(K) == 4) return (int)((unsigned)key & (G - 1));
  return (int)((unsigned long long)key & 0xffffffffull);
}

template <int G, typename K>
__global__ __launch_bounds__(kThreads) void k_sym_lanes(int bin, const int32_t* __restrict__ list,
                                                        const int32_t* __restrict__ bin_off,
                                                        const int32_t* __restrict__ rpA,
                                                        const int32_t* __restrict__ ciA,
                                                        const int32_t* __restrict__ rpB,
                                                        const int32_t* __restrict__ ciB,
                                                        int32_t* __restrict__ counts) {
  constexpr int RPB = kThreads / G;
  const int first = bin_off[bin], nrows = bin_off[bin + 1] - first;
  const int lane = __lane_id(), l = threadIdx.x % G;
  const unsigned long long gm = group_mask<G>(lane);
  for (int base = blockIdx.x * RPB; base < nrows; base += gridDim.x * RPB) {
    const int idx = base + threadIdx.x / G;
    const bool valid = idx < nrows;
    const int i = valid ? list[first + idx] : 0;
    int col, ea, eb;
    lane_product<G>(i, valid, l, rpA, ciA, rpB, ciB, col, ea, eb);
    const K key = group_sort<G, K>(make_key<G, K>(col, l), l);
    const int sc = key_col<G, K>(key);
    const int prev = (int)dpp_key<0x138>((unsigned)sc);  // wave_shr:1, lane - 1
    const bool head = sc != INT32_MAX && (l == 0 || prev != sc);
    const int cnt = __popcll(__ballot(head) & gm);
    if (valid && l == 0) counts[i] = cnt;
  }
}

template <typename T, int G, typename K>
__global__ __launch_bounds__(kThreads) void k_num_lanes(
    int bin, const int32_t* __restrict__ list, const int32_t* __restrict__ bin_off,
    const int32_t* __restrict__ rpA, const int32_t* __restrict__ ciA, const T* __restrict__ vA,
    const int32_t* __restrict__ rpB, const int32_t* __restrict__ ciB, const T* __restrict__ vB,
    const int32_t* __restrict__ rpC, int32_t* __restrict__ ciC, T* __restrict__ vC) {
  constexpr int RPB = kThreads / G;
  const int first = bin_off[bin], nrows = bin_off[bin + 1] - first;
  const int lane = __lane_id(), l = threadIdx.x % G;
  const int gbase = lane & ~(G - 1);
  const unsigned long long gm = group_mask<G>(lane);
  const unsigned long long below = gm & ((1ull << lane) - 1ull);
  const unsigned long long above = gm & ~((2ull << lane) - 1ull);
  for (int base = blockIdx.x * RPB; base < nrows; base += gridDim.x * RPB) {
    const int idx = base + threadIdx.x / G;
    const bool valid = idx < nrows;
    const int i = valid ? list[first + idx] : 0;
    int col, ea, eb;
    lane_product<G>(i, valid, l, rpA, ciA, rpB, ciB, col, ea, eb);
    const T prod = ea >= 0 ? vA[ea] * vB[eb] : T(0);
    const K key = group_sort<G, K>(make_key<G, K>(col, l), l);
    const int sc = key_col<G, K>(key);
    const T v = __shfl(prod, gbase + key_idx<G, K>(key));
    const int prev = (int)dpp_key<0x138>((unsigned)sc);  // wave_shr:1, lane - 1
    const bool head = sc != INT32_MAX && (l == 0 || prev != sc);
    const unsigned long long heads = __ballot(head);
    const unsigned long long used = __ballot(sc != INT32_MAX) & gm;
    // run length of a head: up to the next head, else to the last product
    int run = 0;
    if (head) {
      const unsigned long long nxt = heads & above;
      const int end = nxt ? __ffsll((long long)nxt) - 1 : gbase + __popcll(used);
      run = end - lane;
    }
    const int steps = wave_max(run);
    // run sums in lane order (k ascending)
    T acc = v;
    T w = v;
    for (int d = 1; d < steps; ++d) {
      w = wave_next(w);  // now the value of lane + d
      if (d < run) acc += w;
    }
    if (valid && head) {
      const int pos = rpC[i] + __popcll(heads & below);
      ciC[pos] = sc;
      vC[pos] = acc;
    }
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
// gA: G lanes per row of A, lanes over A's entries.
template <typename T, int G>
__global__ __launch_bounds__(kThreads) void k_bwd_a(int m, const int32_t* __restrict__ rpA,
                                                    const int32_t* __restrict__ ciA,
                                                    const int32_t* __restrict__ rpB,
                                                    const int32_t* __restrict__ ciB,
                                                    const T* __restrict__ vB,
                                                    const int32_t* __restrict__ rpC,
                                                    const int32_t* __restrict__ ciC,
                                                    const T* __restrict__ gC, T* __restrict__ gA) {
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int i = b * (kThreads / G) + threadIdx.x / G;
  const int l = threadIdx.x % G;
  if (i >= m) return;
  const int c0 = rpC[i], c1 = rpC[i + 1];
  const int a1 = rpA[i + 1];
  for (int a = rpA[i] + l; a < a1; a += G) {
    const int k = ciA[a];
    T s = 0;
    for (int q = rpB[k]; q < rpB[k + 1]; ++q) {
      const int p = find_sorted(ciC, c0, c1, ciB[q]);
      if (p >= 0) s += gC[p] * vB[q];
    }
    gA[a] = s;
  }
}

// gB: G lanes per row k of B; the entries of the row in turn, the lanes
// splitting column k of A (A^T's row k, rows ascending, values through
// permA) and summing with a group reduction.  The entry loop runs the
// same number of times across the wave (the reduction needs whole groups).
template <typename T, int G>
__global__ __launch_bounds__(kThreads) void k_bwd_b(
    int n, const int32_t* __restrict__ rpB, const int32_t* __restrict__ ciB,
    const int32_t* __restrict__ rpAT, const int32_t* __restrict__ ciAT,
    const int32_t* __restrict__ permA, const T* __restrict__ vA, const int32_t* __restrict__ rpC,
    const int32_t* __restrict__ ciC, const T* __restrict__ gC, T* __restrict__ gB) {
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
  for (int u = 0; u < steps; ++u) {
    const int q = q0 + u;
    T s = 0;
    if (q < q1) {
      const int j = ciB[q];
      for (int t = t0 + l; t < t1; t += G) {
        const int i = ciAT[t];
        const int p = find_sorted(ciC, rpC[i], rpC[i + 1], j);
        if (p >= 0) s += vA[permA[t]] * gC[p];
      }
    }
    s = group_sum<G>(s);
    if (q < q1 && l == 0) gB[q] = s;
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
  unsigned g = (unsigned)((m + kThreads - 1) / kThreads);
  if (g > 8192) g = 8192;
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

// Launches of the lane bins; 32-bit sort keys while (column, product
// index) fits in 32 bits.
template <int G>
bool keys32(int ncols) {
  return (long long)ncols < (1ll << (32 - log2_of<G>())) - 1;
}

template <int G>
void sym_lanes(int bin, const csrad_csr* A, const csrad_csr* B, const SpgemmWs& w,
               hipStream_t s) {
  const unsigned g = persistent_grid(kThreads / G, A->nrows);
  if (keys32<G>(B->ncols))
    hipLaunchKernelGGL((k_sym_lanes<G, unsigned>), dim3(g), dim3(kThreads), 0, s, bin, w.list,
                       w.bin_off, A->rowptr, A->colind, B->rowptr, B->colind, w.counts);
  else
    hipLaunchKernelGGL((k_sym_lanes<G, unsigned long long>), dim3(g), dim3(kThreads), 0, s, bin,
                       w.list, w.bin_off, A->rowptr, A->colind, B->rowptr, B->colind, w.counts);
}

template <typename T, int G>
void num_lanes(int bin, int rows, const csrad_csr* A, const csrad_csr* B, const T* vA,
               const T* vB, const int32_t* rpC, int32_t* ciC, T* vC, const SpgemmWs& w,
               hipStream_t s) {
  if (rows == 0) return;
  const unsigned g = persistent_grid(kThreads / G, rows);
  if (keys32<G>(B->ncols))
    hipLaunchKernelGGL((k_num_lanes<T, G, unsigned>), dim3(g), dim3(kThreads), 0, s, bin, w.list,
                       w.bin_off, A->rowptr, A->colind, vA, B->rowptr, B->colind, vB, rpC, ciC,
                       vC);
  else
    hipLaunchKernelGGL((k_num_lanes<T, G, unsigned long long>), dim3(g), dim3(kThreads), 0, s,
                       bin, w.list, w.bin_off, A->rowptr, A->colind, vA, B->rowptr, B->colind, vB,
                       rpC, ciC, vC);
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
  num_lanes<T, 8>(1, rows(1), A, B, vA, vB, rpC, ciC, vC, w, s);
  num_lanes<T, 16>(2, rows(2), A, B, vA, vB, rpC, ciC, vC, w, s);
  num_lanes<T, 32>(3, rows(3), A, B, vA, vB, rpC, ciC, vC, w, s);
  num_lanes<T, 64>(4, rows(4), A, B, vA, vB, rpC, ciC, vC, w, s);
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

template <typename T>
int spgemm_bwd_t(const csrad_csr* A, const csrad_csr* B, const csrad_csr* At,
                 const int32_t* permA, const csrad_csr* C, const T* gC, T* gA, T* gB,
                 hipStream_t s) {
  if (gA && A->nrows > 0) {
    const int m = A->nrows;
    CSRAD_G_SWITCH(lanes_for(A->nnz, m),
                   hipLaunchKernelGGL((k_bwd_a<T, G>), dim3((m + kThreads / G - 1) / (kThreads / G)),
                                      dim3(kThreads), 0, s, m, A->rowptr, A->colind, B->rowptr,
                                      B->colind, static_cast<const T*>(B->vals), C->rowptr,
                                      C->colind, gC, gA));
  }
  if (gB && B->nrows > 0) {
    const int n = B->nrows;
    // lanes from the mean column length of A (the inner loop)
    CSRAD_G_SWITCH(lanes_for(A->nnz, A->ncols),
                   hipLaunchKernelGGL((k_bwd_b<T, G>), dim3((n + kThreads / G - 1) / (kThreads / G)),
                                      dim3(kThreads), 0, s, n, B->rowptr, B->colind, At->rowptr,
                                      At->colind, permA, static_cast<const T*>(A->vals), C->rowptr,
                                      C->colind, gC, gB));
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
    sym_lanes<8>(1, A, B, w, s);
    sym_lanes<16>(2, A, B, w, s);
    sym_lanes<32>(3, A, B, w, s);
    // counting alone: for U <= 64 an LDS hash with 16 lanes per row beats
    // sorting across a whole wave per row
    hipLaunchKernelGGL((k_sym_hash<16, 128>), dim3(persistent_grid(16, m)), dim3(kThreads), 0, s,
                       4, w.list, w.bin_off, A->rowptr, A->colind, B->rowptr, B->colind,
                       w.counts);
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
