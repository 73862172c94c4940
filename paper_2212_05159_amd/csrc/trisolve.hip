// Sparse triangular solve T x = b and its VJP (Section 3.1.5; Table 1,
// SpSolve row), level-scheduled.
//
// Analysis: the dependency graph of the solve (row i reads row j when T_ij
// is stored on the solve side of the diagonal) is layered by longest path.
//   1. per row: dependency count, stored diagonal check, level-0 rows;
//   2. Kahn's algorithm level by level (dependents of a row are its
//      column, i.e. a row of T^T): a row joins the next level when its last
//      dependency is placed; narrow levels run inside one workgroup, wide
//      ones as grid launches;
//   3. rows are grouped by level, ascending within each level (a stable
//      multi-split by level for up to 32 levels, else the stable transpose
//      of the row -> level map).
// Level sets are unique, so the integer output is bit-exact.
//
// Solve: levels run in order.  A level with many rows is one grid launch;
// runs of small levels are processed by a single workgroup with a barrier
// between levels, so deep, narrow level structures do not pay one launch
// per level.
//
// Adjoint: w = T^{-T} gx runs over T^T (rows of T^T are columns of T)
// visiting T's levels in reverse (every row that column j feeds sits on a
// higher level).  A second pass over T^T writes gvals[(i,j)] = -w_i x_j.
// T must be triangular on the side given by `lower`; a stored entry on
// the other side is a precondition violation.
#include "internal.hpp"

namespace csrad {
namespace {

constexpr int kThreads = 256;
constexpr int kKahnThreads = 1024;
constexpr int kOneBlockThreads = 1024;
constexpr int kOneBlockPasses = 4;

__device__ __forceinline__ bool dep_side(int lower, int row, int col) {
  return lower ? col < row : col > row;
}

constexpr int kUnset = INT32_MAX;
constexpr int kMaxPassBlocks = 4096;  // grid cap of the prep and pull passes

// Step 1: dependency counts, the diagonal check, and level 0 (rows without
// dependencies), counted per block into part.
// Rows counted per block go to part[blockIdx.x] (summed by the level step
// in a fixed order: no contended atomics on one address).
__device__ __forceinline__ void block_count_to(int cnt, int32_t* __restrict__ part) {
  __shared__ int s_cnt;
  if (threadIdx.x == 0) s_cnt = 0;
  __syncthreads();
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
  if (__lane_id() == 0 && cnt) atomicAdd(&s_cnt, cnt);
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = s_cnt;
}

// Sum of part[0 .. np) by one block (fixed order per thread, then LDS).
__device__ __forceinline__ int sum_parts(const int32_t* __restrict__ part, int np) {
  __shared__ int s_sum;
  if (threadIdx.x == 0) s_sum = 0;
  __syncthreads();
  int c = 0;
  for (int b = threadIdx.x; b < np; b += blockDim.x) c += part[b];
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  if (__lane_id() == 0 && c) atomicAdd(&s_sum, c);
  __syncthreads();
  const int r = s_sum;
  __syncthreads();  // every thread has read it before a next call resets it
  return r;
}

// Sums of part[0 .. np) and part[kMaxPassBlocks .. kMaxPassBlocks + np) in
// one pass (both loads in flight together).
__device__ __forceinline__ int2 sum_parts2(const int32_t* __restrict__ part, int np) {
  __shared__ int s_a, s_b;
  if (threadIdx.x == 0) s_a = s_b = 0;
  __syncthreads();
  int a = 0, b = 0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
    a += part[i];
    b += part[kMaxPassBlocks + i];
  }
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o);
    b += __shfl_xor(b, o);
  }
  if (__lane_id() == 0) {
    if (a) atomicAdd(&s_a, a);
    if (b) atomicAdd(&s_b, b);
  }
  __syncthreads();
  return make_int2(s_a, s_b);
}

// Columns of a row read per round (loads issued together) by the
// analysis passes, which walk one row per thread.
constexpr int kRowBatch = 8;

__global__ __launch_bounds__(kThreads) void k_tri_prep(int n, int lower,
                                                       const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ ci,
                                                       int32_t* __restrict__ indeg,
                                                       int32_t* __restrict__ level_of_row,
                                                       int32_t* __restrict__ state,
                                                       int32_t* __restrict__ part) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  int cnt = 0, left = 0;
  for (long long base = (long long)blockIdx.x * blockDim.x; base < n; base += stride) {
    const int i = (int)(base + threadIdx.x);
    bool zero = false;
    if (i < n) {
      int deps = 0;
      bool diag = false;
      const int e1 = rp[i + 1];
      // kRowBatch columns per round with their loads issued together
      for (int eb = rp[i]; eb < e1; eb += kRowBatch) {
        int j[kRowBatch];
#pragma unroll
        for (int u = 0; u < kRowBatch; ++u) j[u] = eb + u < e1 ? ci[eb + u] : -1;
#pragma unroll
        for (int u = 0; u < kRowBatch; ++u) {
          if (j[u] < 0) continue;
          deps += dep_side(lower, i, j[u]);
          diag |= (j[u] == i);
        }
      }
      indeg[i] = deps;
      level_of_row[i] = deps == 0 ? 0 : kUnset;
      zero = deps == 0;
      if (!diag) atomicMin(&state[1], i);
    }
    cnt += zero;
    left += i < n && !zero;
  }
  block_count_to(cnt, part);
  block_count_to(left, part + kMaxPassBlocks);
}

// The frontier (the rows on level state[2]) into the buffer Kahn's
// algorithm reads it from (state[3] ? fb : fa): flag, then compaction at
// the scanned positions.
__global__ void k_tri_flag_level(int n, const int32_t* __restrict__ level_of_row,
                                 const int32_t* __restrict__ state, int32_t* __restrict__ flag) {
  const int L = state[2];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    flag[i] = level_of_row[i] == L;
}

__global__ void k_tri_compact_cur(int n, const int32_t* __restrict__ flag,
                                  const int32_t* __restrict__ pos, int32_t* __restrict__ fa,
                                  int32_t* __restrict__ fb, const int32_t* __restrict__ state) {
  int32_t* front = state[3] ? fb : fa;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    if (flag[i]) front[pos[i]] = i;
}

// Step 2, narrow levels: Kahn's algorithm by levels inside one workgroup.
// Dependents of row j are the rows of column j of T, i.e. row j of T^T; a
// row joins the next level (and gets its level) when its last dependency
// is placed.  Runs while the frontier is non-empty and at most kKahnSmall
// rows; terminates after at most n levels (each level places at least one
// row, and a row enters a frontier only once).  State on the device: [0]
// rows in the current frontier, [2] its level, [3] which buffer holds it.
constexpr int kKahnSmall = 8192;
constexpr int kSpecRounds = 3;
constexpr int kSpecLevels = kSpecRounds + 1;  // levels the speculative rounds can complete

// Releases the dependents of row j (when valid).  The lanes of a wave walk
// their rows' dependents in step so that rows made ready together are
// appended with one atomic per wave.  Every lane of the wave must reach
// the call.
__device__ __forceinline__ void kahn_visit(int j, bool valid, int level, int lower,
                                           const int32_t* __restrict__ rpT,
                                           const int32_t* __restrict__ ciT,
                                           int32_t* __restrict__ indeg, int32_t* __restrict__ nxt,
                                           int* next_n, int32_t* __restrict__ level_of_row) {
  int t0 = 0, len = 0;
  if (valid) {
    t0 = rpT[j];
    len = rpT[j + 1] - t0;
  }
  const int steps = wave_max(len);
  for (int u = 0; u < steps; ++u) {
    bool ready = false;
    int i = 0;
    if (u < len) {
      i = ciT[t0 + u];
      ready = dep_side(lower, i, j) && atomicSub(&indeg[i], 1) == 1;
    }
    const int slot = wave_append(next_n, ready);
    if (ready) {
      level_of_row[i] = level + 1;
      nxt[slot] = i;
    }
  }
}

__global__ __launch_bounds__(kKahnThreads) void k_tri_kahn_small(
    int n, int lower, const int32_t* __restrict__ rpT, const int32_t* __restrict__ ciT,
    int32_t* __restrict__ indeg, int32_t* __restrict__ fa, int32_t* __restrict__ fb,
    int32_t* __restrict__ state, int32_t* __restrict__ level_of_row) {
  __shared__ int next_n;
  int cur_n = state[0];
  int level = state[2];
  int which = state[3];
  while (cur_n > 0 && cur_n <= kKahnSmall && level < n) {
    int* cur = which ? fb : fa;
    int* nxt = which ? fa : fb;
    if (threadIdx.x == 0) next_n = 0;
    __syncthreads();
    for (int base = 0; base < cur_n; base += blockDim.x) {
      const int q = base + threadIdx.x;
      const bool valid = q < cur_n;
      kahn_visit(valid ? cur[q] : 0, valid, level, lower, rpT, ciT, indeg, nxt, &next_n,
                 level_of_row);
    }
    __syncthreads();
    cur_n = next_n;
    which ^= 1;
    ++level;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    state[0] = cur_n;
    state[2] = level;
    state[3] = which;
  }
}

// Step 2, wide levels: one pass over the rows not yet placed.  With the
// frontier on level L placed, a row is ready (level L + 1) when all its
// dependencies sit on levels <= L; otherwise indeg gets the number of
// dependencies still above L (unplaced, or on level L + 1 from this same
// pass: either way above L), which is what Kahn's algorithm needs next.
// The rows placed are counted per block into part.  The frontier's level L is
// state[2]; nothing is done once state[4] is set (the level step after it
// is gated on it too), so rounds may be launched before the host knows
// whether they are needed.
__global__ __launch_bounds__(kThreads) void k_tri_pull(int n, int lower,
                                                       const int32_t* __restrict__ state,
                                                       const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ ci,
                                                       int32_t* __restrict__ level_of_row,
                                                       int32_t* __restrict__ indeg,
                                                       int32_t* __restrict__ part) {
  if (state[4]) return;  // uniform over the grid
  const int L = state[2];
  const long long stride = (long long)gridDim.x * blockDim.x;
  int cnt = 0, left = 0;
  for (long long base = (long long)blockIdx.x * blockDim.x; base < n; base += stride) {
    const int i = (int)(base + threadIdx.x);
    bool placed = false;
    if (i < n && level_of_row[i] == kUnset) {
      int cnt = 0;
      const int e1 = rp[i + 1];
      // kRowBatch columns per round, then their levels, loads issued together
      for (int eb = rp[i]; eb < e1; eb += kRowBatch) {
        int j[kRowBatch];
#pragma unroll
        for (int u = 0; u < kRowBatch; ++u) j[u] = eb + u < e1 ? ci[eb + u] : -1;
        int lv[kRowBatch];
#pragma unroll
        for (int u = 0; u < kRowBatch; ++u)
          lv[u] = (j[u] >= 0 && dep_side(lower, i, j[u])) ? level_of_row[j[u]] : L;
#pragma unroll
        for (int u = 0; u < kRowBatch; ++u) cnt += lv[u] > L;
      }
      if (cnt == 0) {
        level_of_row[i] = L + 1;
        placed = true;
      } else {
        indeg[i] = cnt;
        ++left;
      }
    }
    cnt += placed;
  }
  block_count_to(cnt, part);
  block_count_to(left, part + kMaxPassBlocks);
}

// After a pull pass: state[0] = rows placed (the sum of the np block
// counts), [2] += 1, [4] = no further level (nothing placed, or n
// levels); when the pass placed rows and left none unplaced, the levels
// are complete at once: [2] = the level count, [0] = 0, [4] = 1 (no
// further pass needed to find that nothing is left).  Nothing once [4]
// is set.
__global__ void k_tri_next_level(int n, const int32_t* __restrict__ part, int np,
                                 int32_t* __restrict__ state) {
  if (state[4]) return;
  const int2 tl = sum_parts2(part, np);
  const int t = tl.x, left = tl.y;
  if (threadIdx.x == 0) {
    if (t > 0 && left == 0) {
      state[0] = 0;
      state[2] += 2;
      state[4] = 1;
    } else {
      state[0] = t;
      state[2] += 1;
      state[4] = t == 0 || state[2] >= n;
    }
    state[6] = state[4] ? 0 : 1;
  }
}

// The analysis state, zero but for [1] (the first row without a stored
// diagonal, none yet) and [6] (the gate of the speculative grouping by
// level: 0 once the levels are complete, kept by the level steps).
__global__ void k_tri_state_init(int32_t* __restrict__ state) {
  if (threadIdx.x < 8)
    state[threadIdx.x] = threadIdx.x == 1 ? INT32_MAX : (threadIdx.x == 6 ? 1 : 0);
}

// After the prep pass: state[0] = the level-0 frontier size, [2] = 0,
// [3] = 0, [4] = no level; with every row on level 0 (no dependencies
// anywhere) the levels are complete: [0] = 0, [2] = 1, [4] = 1.
__global__ void k_tri_first_level(const int32_t* __restrict__ part, int np,
                                  int32_t* __restrict__ state) {
  const int2 tl = sum_parts2(part, np);
  const int t = tl.x, left = tl.y;
  if (threadIdx.x == 0) {
    const bool all = t > 0 && left == 0;
    state[0] = all ? 0 : t;
    state[2] = all ? 1 : 0;
    state[3] = 0;
    state[4] = t == 0 || all;
    state[6] = state[4] ? 0 : 1;
  }
}

__global__ void k_iota(int32_t* p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = i;
}

// Solve one row of T x = b on G lanes (also the adjoint solve over T^T
// when PERM is set: values then come through perm).
template <typename TV, typename TX, int G, int U, bool PERM>
__device__ __forceinline__ void solve_row(int r, int sub, int lower, const int32_t* __restrict__ rp,
                                          const int32_t* __restrict__ ci,
                                          const int32_t* __restrict__ perm,
                                          const TV* __restrict__ vals, const TX* __restrict__ b,
                                          TX* __restrict__ x, bool valid) {
  TX s = 0, d = 0;
  if (valid) {
    const int e1 = rp[r + 1];
    // U entries per lane per round (e = sub, sub + G, ...: the lane sums in
    // row order), their loads issued stage by stage without branches:
    // positions past the row's end read its last entry and are masked out,
    // and entries that read no other row (the diagonal) load x at the row
    // itself, whose value is not used
    for (int eb = rp[r] + sub; eb < e1; eb += G * U) {
      int j[U], pe[U];
      TX v[U], xv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = min(eb + u * G, e1 - 1);
        j[u] = ci[e];
        pe[u] = PERM ? perm[e] : e;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        v[u] = (TX)vals[pe[u]];
        xv[u] = x[(j[u] != r && dep_side(lower, r, j[u])) ? j[u] : r];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (eb + u * G >= e1) continue;
        if (j[u] == r) d = v[u];
        else if (dep_side(lower, r, j[u])) s += v[u] * xv[u];
      }
    }
  }
  s = group_sum<G>(s);
  d = group_sum<G>(d);
  if (valid && sub == 0) x[r] = (b[r] - s) / d;
}

template <typename TV, typename TX, int G, int U, bool PERM>
__global__ __launch_bounds__(kThreads) void k_tri_level(int lo, int hi, int lower,
                                                       const int32_t* __restrict__ rows,
                                                       const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ ci,
                                                       const int32_t* __restrict__ perm,
                                                       const TV* __restrict__ vals,
                                                       const TX* __restrict__ b,
                                                       TX* __restrict__ x) {
  const int q = lo + blockIdx.x * (kThreads / G) + threadIdx.x / G;
  const bool valid = q < hi;
  const int r = valid ? rows[q] : 0;
  solve_row<TV, TX, G, U, PERM>(r, threadIdx.x % G, lower, rp, ci, perm, vals, b, x, valid);
}

// A run of consecutive small levels [l0, l1) in one workgroup.  With
// REVERSE the levels run from l1-1 down to l0.
template <typename TV, typename TX, int G, int U, bool PERM, bool REVERSE>
__global__ __launch_bounds__(kOneBlockThreads) void k_tri_levels_block(
    int l0, int l1, int lower, const int32_t* __restrict__ level_ptr,
    const int32_t* __restrict__ rows, const int32_t* __restrict__ rp,
    const int32_t* __restrict__ ci, const int32_t* __restrict__ perm, const TV* __restrict__ vals,
    const TX* __restrict__ b, TX* __restrict__ x) {
  constexpr int RPB = kOneBlockThreads / G;
  for (int t = 0; t < l1 - l0; ++t) {
    const int l = REVERSE ? l1 - 1 - t : l0 + t;
    const int lo = level_ptr[l], hi = level_ptr[l + 1];
    for (int base = lo; base < hi; base += RPB) {
      const int q = base + threadIdx.x / G;
      const bool valid = q < hi;
      const int r = valid ? rows[q] : 0;
      solve_row<TV, TX, G, U, PERM>(r, threadIdx.x % G, lower, rp, ci, perm, vals, b, x, valid);
    }
    __syncthreads();
  }
}

// gvals[(i,j)] = -w_i x_j for the entries of T, written from T^T's side:
// row j of T^T holds column j of T; w there is final once the adjoint
// solve has passed.
template <typename T, int G>
__global__ __launch_bounds__(kThreads) void k_tri_gvals(int n, const int32_t* __restrict__ rpT,
                                                       const int32_t* __restrict__ ciT,
                                                       const int32_t* __restrict__ perm,
                                                       const T* __restrict__ w,
                                                       const T* __restrict__ x,
                                                       T* __restrict__ gv) {
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int j = b * (kThreads / G) + threadIdx.x / G;
  const int sub = threadIdx.x % G;
  if (j >= n) return;
  const T xj = x[j];
  for (int t = rpT[j] + sub; t < rpT[j + 1]; t += G) gv[perm[t]] = -w[ciT[t]] * xj;
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

// Runs the levels: big ones as grid launches, runs of small ones in one
// workgroup.  REVERSE visits levels from last to first.  The first level
// visited reads no other row, so (with nothing stored on the other side of
// the diagonal) its rows hold the diagonal alone: as a grid launch it takes
// one lane per row.
// Past the first level, a row takes half the lanes that its mean length
// asks for (GL), each lane kLevelU entries per round with their loads
// issued together: the solve is a chain of dependent gathers per entry and
// a CU's resident threads cap the chains in flight (128^3 red-black L:
// forward 0.045 -> 0.036 ms, adjoint 0.105 -> 0.095 ms).
constexpr int kLevelSplit = 2, kLevelU = 4;

template <typename TV, typename TX, int GL, bool PERM, bool REVERSE>
void run_levels(int nlevels, const int32_t* lp_host, const int32_t* lp_dev, const int32_t* rows,
                int lower, const int32_t* rp, const int32_t* ci, const int32_t* perm,
                const TV* vals, const TX* b, TX* x, hipStream_t s) {
  constexpr int G = GL >= kLevelSplit ? GL / kLevelSplit : 1, U = kLevelU;
  // A level is worth a grid launch once the single workgroup would need
  // more than kOneBlockPasses passes over it at GL lanes per row (a pass
  // costs a dependent memory round trip; a launch a few of them).
  constexpr int kBig = kOneBlockPasses * (kOneBlockThreads / GL);
  auto big = [&](int l) { return lp_host[l + 1] - lp_host[l] > kBig; };
  int t = 0;
  while (t < nlevels) {
    const int l = REVERSE ? nlevels - 1 - t : t;
    if (big(l)) {
      const int lo = lp_host[l], hi = lp_host[l + 1];
      if (t == 0 && (G > 1 || U > 1)) {
        const unsigned blocks = (unsigned)((hi - lo + kThreads - 1) / kThreads);
        hipLaunchKernelGGL((k_tri_level<TV, TX, 1, 1, PERM>), dim3(blocks), dim3(kThreads), 0, s,
                           lo, hi, lower, rows, rp, ci, perm, vals, b, x);
      } else {
        const int rpb = kThreads / G;
        hipLaunchKernelGGL((k_tri_level<TV, TX, G, U, PERM>), dim3((hi - lo + rpb - 1) / rpb),
                           dim3(kThreads), 0, s, lo, hi, lower, rows, rp, ci, perm, vals, b, x);
      }
      ++t;
      continue;
    }
    int u = t;
    while (u < nlevels && !big(REVERSE ? nlevels - 1 - u : u)) ++u;
    // levels t..u-1 in visiting order
    const int l0 = REVERSE ? nlevels - u : t;
    const int l1 = REVERSE ? nlevels - t : u;
    hipLaunchKernelGGL((k_tri_levels_block<TV, TX, G, U, PERM, REVERSE>), dim3(1),
                       dim3(kOneBlockThreads), 0, s, l0, l1, lower, lp_dev, rows, rp, ci, perm,
                       vals, b, x);
    t = u;
  }
}

template <typename T>
int trisolve_fwd_t(const csrad_csr* Tm, int lower, int nlevels, const int32_t* lp_host,
                   const int32_t* lp_dev, const int32_t* rows, const T* b, T* x, hipStream_t s) {
  const T* v = static_cast<const T*>(Tm->vals);
  CSRAD_G_SWITCH(lanes_for(Tm->nnz, Tm->nrows),
                 (run_levels<T, T, G, false, false>(nlevels, lp_host, lp_dev, rows, lower, Tm->rowptr,
                                                 Tm->colind, nullptr, v, b, x, s)));
  return launch_status();
}

template <typename T>
int trisolve_bwd_t(const csrad_csr* Tm, int lower, const csrad_csr* Tt, const int32_t* perm,
                   int nlevels, const int32_t* lp_host, const int32_t* lp_dev, const int32_t* rows,
                   const T* x, const T* gx, T* gb, T* gv, hipStream_t s) {
  const T* v = static_cast<const T*>(Tm->vals);
  const int n = Tm->nrows;
  // T^T is triangular on the other side: row j of T^T depends on i when
  // (i, j) is on T's solve side, i.e. the opposite orientation.
  const int lower_t = lower ? 0 : 1;
  const int g = lanes_for(Tm->nnz, n);
  CSRAD_G_SWITCH(g, (run_levels<T, T, G, true, true>(nlevels, lp_host, lp_dev, rows, lower_t,
                                                  Tt->rowptr, Tt->colind, perm, v, gx, gb, s)));
  if (gv) {
    CSRAD_G_SWITCH(g, hipLaunchKernelGGL((k_tri_gvals<T, G>),
                                         dim3((n + kThreads / G - 1) / (kThreads / G)),
                                         dim3(kThreads), 0, s, n, Tt->rowptr, Tt->colind, perm, gb,
                                         x, gv));
  }
  return launch_status();
}

// Float64-vector solves over T's value type, for preconditioners: with
// transpose = false x = T^{-1} b over T's levels; with transpose = true
// x = T^{-T} b over T^T with T's levels reversed, reading T^T's own values
// when Tt carries them and T's values through perm otherwise.
template <typename TV>
int trisolve_vec64_t(const csrad_csr* Tm, int lower, const csrad_csr* Tt, const int32_t* perm,
                     bool transpose, int nlevels, const int32_t* lp_host, const int32_t* lp_dev,
                     const int32_t* rows, const double* b, double* x, hipStream_t s) {
  const TV* v = static_cast<const TV*>(Tm->vals);
  const TV* vt = static_cast<const TV*>(Tt ? Tt->vals : nullptr);
  CSRAD_G_SWITCH(lanes_for(Tm->nnz, Tm->nrows), {
    if (transpose && vt)
      run_levels<TV, double, G, false, true>(nlevels, lp_host, lp_dev, rows, lower ? 0 : 1,
                                             Tt->rowptr, Tt->colind, nullptr, vt, b, x, s);
    else if (transpose)
      run_levels<TV, double, G, true, true>(nlevels, lp_host, lp_dev, rows, lower ? 0 : 1,
                                            Tt->rowptr, Tt->colind, perm, v, b, x, s);
    else
      run_levels<TV, double, G, false, false>(nlevels, lp_host, lp_dev, rows, lower, Tm->rowptr,
                                              Tm->colind, nullptr, v, b, x, s);
  });
  return launch_status();
}

struct TriWs {
  int32_t* indeg;
  int32_t* fa;
  int32_t* fb;
  int32_t* counters;  // [0] frontier size, [1] bad row, [2] level, [3] buffer, [4] done
  int32_t* part;      // per-block row counts of the prep and pull passes: [0, kMaxPassBlocks)
                      // rows placed, [kMaxPassBlocks, 2 kMaxPassBlocks) rows left unplaced
  int32_t* flag;
  int32_t* pos;
  void* sws;
  size_t sws_bytes;
  long long* total;
  int32_t* iota;
  int32_t* perm;
  void* tws;
  size_t tws_bytes;
  void* gws;
  size_t gws_bytes;
};

TriWs carve_tri(Carver& cv, int n) {
  TriWs w;
  w.indeg = cv.take<int32_t>((size_t)n);
  w.fa = cv.take<int32_t>((size_t)n);
  w.fb = cv.take<int32_t>((size_t)n);
  w.counters = cv.take<int32_t>(8);
  w.part = cv.take<int32_t>(2 * kMaxPassBlocks);
  w.flag = cv.take<int32_t>((size_t)n + 1);
  w.pos = cv.take<int32_t>((size_t)n + 1);
  w.sws_bytes = scan_workspace(n);
  w.sws = cv.take<char>(w.sws_bytes);
  w.total = cv.take<long long>(1);
  w.iota = cv.take<int32_t>((size_t)n + 1);
  w.perm = cv.take<int32_t>((size_t)n);
  w.tws_bytes = transpose_workspace(n, n, n);
  w.tws = cv.take<char>(w.tws_bytes);
  w.gws_bytes = group_small_workspace(n, 32);
  w.gws = cv.take<char>(w.gws_bytes);
  return w;
}

int check_levels(const csrad_csr* Tm, int nlevels, const int32_t* lp_host, const int32_t* rows) {
  if (nlevels < 0 || (Tm->nrows > 0 && (nlevels == 0 || !lp_host || !rows))) return CSRAD_EINVAL;
  if (Tm->nrows > 0 && (lp_host[0] != 0 || lp_host[nlevels] != Tm->nrows)) return CSRAD_EINVAL;
  return CSRAD_OK;
}

}  // namespace

int trisolve_vec64(const csrad_csr* Tm, int lower, const csrad_csr* Tt, const int32_t* perm,
                   bool transpose, int nlevels, const int32_t* lp_host, const int32_t* lp_dev,
                   const int32_t* rows, const double* b, double* x, hipStream_t s) {
  if (Tm->dtype == CSRAD_F32)
    return trisolve_vec64_t<float>(Tm, lower, Tt, perm, transpose, nlevels, lp_host, lp_dev, rows,
                                   b, x, s);
  return trisolve_vec64_t<double>(Tm, lower, Tt, perm, transpose, nlevels, lp_host, lp_dev, rows,
                                  b, x, s);
}

}  // namespace csrad

using namespace csrad;

extern "C" int csr_trisolve_workspace(const csrad_csr* Tm, size_t* bytes) {
  if (!Tm || !bytes || Tm->nrows < 0) return CSRAD_EINVAL;
  Carver cv(nullptr, 0);
  carve_tri(cv, Tm->nrows);
  *bytes = cv.off + 256;
  return CSRAD_OK;
}

extern "C" int csr_trisolve_analyze(const csrad_csr* Tm, int32_t lower, const csrad_csr* Tt,
                                    int32_t* level_of_row, int32_t* level_ptr,
                                    int32_t* level_rows, int32_t* nlevels_host,
                                    int32_t* level_ptr_host, void* work, size_t work_bytes,
                                    void* stream) {
  CSRAD_TRY(check_csr(Tm, false));
  CSRAD_TRY(check_csr(Tt, false));
  if (Tm->nrows != Tm->ncols || Tt->nrows != Tm->ncols || Tt->ncols != Tm->nrows ||
      Tt->nnz != Tm->nnz)
    return CSRAD_EINVAL;
  if (!level_ptr || !nlevels_host) return CSRAD_EINVAL;
  const int n = Tm->nrows;
  if (n > 0 && (!level_of_row || !level_rows)) return CSRAD_EINVAL;
  hipStream_t s = as_stream(stream);
  Carver cv(work, work_bytes);
  TriWs w = carve_tri(cv, n);
  if (!work || !cv.ok) return CSRAD_EWORKSPACE;
  if (n == 0) {
    *nlevels_host = 0;
    if (level_ptr_host) level_ptr_host[0] = 0;
    CSRAD_TRY(fill_i32(level_ptr, 1, 0, s));
    return hipStreamSynchronize(s) == hipSuccess ? CSRAD_OK : CSRAD_EHIP;
  }
  hipLaunchKernelGGL(k_tri_state_init, dim3(1), dim3(64), 0, s, w.counters);
  const unsigned gn = (unsigned)((n + kThreads - 1) / kThreads < kMaxPassBlocks
                                     ? (n + kThreads - 1) / kThreads
                                     : kMaxPassBlocks);
  const int lw = lower ? 1 : 0;
  hipLaunchKernelGGL(k_tri_prep, dim3(gn), dim3(kThreads), 0, s, n, lw, Tm->rowptr, Tm->colind,
                     w.indeg, level_of_row, w.counters, w.part);
  hipLaunchKernelGGL(k_tri_first_level, dim3(1), dim3(1024), 0, s, w.part, (int)gn, w.counters);
  // One wide-level round: a pull pass and the level step (no compaction:
  // the frontier is materialised only when Kahn's algorithm takes over).
  auto pull_round = [&]() -> int {
    hipLaunchKernelGGL(k_tri_pull, dim3(gn), dim3(kThreads), 0, s, n, lw, w.counters, Tm->rowptr,
                       Tm->colind, level_of_row, w.indeg, w.part);
    hipLaunchKernelGGL(k_tri_next_level, dim3(1), dim3(1024), 0, s, n, w.part, (int)gn, w.counters);
    return launch_status();
  };
  // Coloured orderings have a few wide levels: run kSpecRounds rounds
  // before the first look at the state (each does nothing once the levels
  // are exhausted), which saves a host round trip per level.  If the
  // levels end within those rounds (at most kSpecLevels of them), the rows
  // are grouped by level before that look too (gated on the device), and
  // the one synchronisation returns both the state and the level pointers.
  for (int r = 0; r < kSpecRounds; ++r) CSRAD_TRY(pull_round());
  const bool spec_group = n >= kSpecLevels;  // level_ptr holds kSpecLevels + 1 entries
  if (spec_group) {
    CSRAD_TRY(group_small_keys(level_of_row, n, kSpecLevels, level_ptr, level_rows, w.gws,
                               w.gws_bytes, s, w.counters + 6));
  }
  int32_t host[8];
  int32_t spec_ptr[kSpecLevels + 1];
  auto read_state = [&]() -> int {
    if (hipMemcpyAsync(host, w.counters, sizeof(host), hipMemcpyDeviceToHost, s) != hipSuccess)
      return CSRAD_EHIP;
    return hipStreamSynchronize(s) == hipSuccess ? CSRAD_OK : CSRAD_EHIP;
  };
  if (spec_group &&
      hipMemcpyAsync(spec_ptr, level_ptr, sizeof(spec_ptr), hipMemcpyDeviceToHost, s) != hipSuccess)
    return CSRAD_EHIP;
  CSRAD_TRY(read_state());
  if (host[1] != INT32_MAX) return CSRAD_ESINGULAR;
  if (spec_group && host[4]) {
    // every row placed within the speculative rounds: nl <= kSpecLevels
    // and the grouping above is final (level pointers past nl equal n)
    const int nl = host[2];
    *nlevels_host = nl;
    if (level_ptr_host)
      for (int l = 0; l <= nl; ++l) level_ptr_host[l] = spec_ptr[l];
    return CSRAD_OK;
  }
  bool have_front = false;  // the frontier list is in the Kahn buffer
  while (host[0] > 0 && host[2] < n) {
    if (host[0] <= kKahnSmall) {
      if (!have_front) {
        hipLaunchKernelGGL(k_tri_flag_level, dim3(gn), dim3(kThreads), 0, s, n, level_of_row,
                           w.counters, w.flag);
        CSRAD_TRY(scan_exclusive(w.flag, w.pos, n, w.total, w.sws, w.sws_bytes, s));
        hipLaunchKernelGGL(k_tri_compact_cur, dim3(gn), dim3(kThreads), 0, s, n, w.flag, w.pos,
                           w.fa, w.fb, w.counters);
      }
      // narrow levels inside one workgroup, until the frontier is empty or
      // wide (it then sits in the buffer Kahn's algorithm left it in)
      hipLaunchKernelGGL(k_tri_kahn_small, dim3(1), dim3(kKahnThreads), 0, s, n, lw, Tt->rowptr,
                         Tt->colind, w.indeg, w.fa, w.fb, w.counters, level_of_row);
      CSRAD_TRY(launch_status());
      have_front = true;
    } else {
      // a wide level: one pass over the unplaced rows
      CSRAD_TRY(pull_round());
      have_front = false;
    }
    CSRAD_TRY(read_state());
  }
  const int nl = host[2];
  *nlevels_host = nl;
  // With a stored diagonal everywhere the graph is acyclic (triangular),
  // so Kahn places every row.
  // Group rows by level, ascending within a level: a stable multi-split for
  // few levels, otherwise the stable transpose of the row -> level map.
  if (nl <= 32) {
    CSRAD_TRY(group_small_keys(level_of_row, n, nl, level_ptr, level_rows, w.gws, w.gws_bytes, s));
  } else {
    hipLaunchKernelGGL(k_iota, dim3((n + 1 + 255) / 256 < 4096 ? (n + 1 + 255) / 256 : 4096),
                       dim3(256), 0, s, w.iota, n + 1);
    CSRAD_TRY(transpose_pattern(n, nl, n, w.iota, level_of_row, level_ptr, level_rows, w.perm,
                                w.tws, w.tws_bytes, s));
  }
  if (level_ptr_host &&
      hipMemcpyAsync(level_ptr_host, level_ptr, sizeof(int32_t) * ((size_t)nl + 1),
                     hipMemcpyDeviceToHost, s) != hipSuccess)
    return CSRAD_EHIP;
  return hipStreamSynchronize(s) == hipSuccess ? CSRAD_OK : CSRAD_EHIP;
}

extern "C" int csr_trisolve_fwd(const csrad_csr* Tm, int32_t lower, int32_t nlevels,
                                const int32_t* level_ptr_host, const int32_t* level_ptr,
                                const int32_t* level_rows, const void* b, void* x, void* stream) {
  CSRAD_TRY(check_csr(Tm, true));
  if (Tm->nrows != Tm->ncols) return CSRAD_EINVAL;
  CSRAD_TRY(check_levels(Tm, nlevels, level_ptr_host, level_rows));
  if (Tm->nrows == 0) return CSRAD_OK;
  if (!b || !x || !level_ptr) return CSRAD_EINVAL;
  hipStream_t s = as_stream(stream);
  if (Tm->dtype == CSRAD_F32)
    return trisolve_fwd_t<float>(Tm, lower ? 1 : 0, nlevels, level_ptr_host, level_ptr, level_rows,
                                 static_cast<const float*>(b), static_cast<float*>(x), s);
  return trisolve_fwd_t<double>(Tm, lower ? 1 : 0, nlevels, level_ptr_host, level_ptr, level_rows,
                                static_cast<const double*>(b), static_cast<double*>(x), s);
}

extern "C" int csr_trisolve_bwd(const csrad_csr* Tm, int32_t lower, const csrad_csr* Tt,
                                const int32_t* perm, int32_t nlevels,
                                const int32_t* level_ptr_host, const int32_t* level_ptr,
                                const int32_t* level_rows, const void* x, const void* gx, void* gb,
                                void* gvals, void* stream) {
  CSRAD_TRY(check_csr(Tm, true));
  CSRAD_TRY(check_csr(Tt, false));
  if (Tm->nrows != Tm->ncols || Tt->nrows != Tm->ncols || Tt->ncols != Tm->nrows ||
      Tt->nnz != Tm->nnz)
    return CSRAD_EINVAL;
  CSRAD_TRY(check_levels(Tm, nlevels, level_ptr_host, level_rows));
  if (Tm->nrows == 0) return CSRAD_OK;
  if (!gx || !gb || !level_ptr || (Tm->nnz > 0 && !perm) || (gvals && !x)) return CSRAD_EINVAL;
  hipStream_t s = as_stream(stream);
  if (Tm->dtype == CSRAD_F32)
    return trisolve_bwd_t<float>(Tm, lower ? 1 : 0, Tt, perm, nlevels, level_ptr_host, level_ptr,
                                 level_rows, static_cast<const float*>(x),
                                 static_cast<const float*>(gx), static_cast<float*>(gb),
                                 static_cast<float*>(gvals), s);
  return trisolve_bwd_t<double>(Tm, lower ? 1 : 0, Tt, perm, nlevels, level_ptr_host, level_ptr,
                                level_rows, static_cast<const double*>(x),
                                static_cast<const double*>(gx), static_cast<double*>(gb),
                                static_cast<double*>(gvals), s);
}
