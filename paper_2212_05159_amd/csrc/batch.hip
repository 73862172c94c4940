// Batched operators over a block-diagonal CSR matrix: many independent
// sparse matrices of uneven sizes concatenated along the diagonal, every op
// (SpMV and SpMM forward and backward of Section 3.1.1/3.1.3, the
// triangular solve and its adjoint of Section 3.1.5) as ONE persistent
// launch over a work queue.
//
// Plan.  The host splits every block into tasks of about equal cost
// (rows + stored entries, the length of the block's merge path), each
// aligned to row boundaries, kept in row order.  Each task carries its
// block's variant:
//   rows, G lanes per row (G = 1 ... 64): the row-split traversal;
//   staged: rows of 256 at a time with their entries staged in LDS
//     (short rows);
//   merge: the task's merge path (row ends merged with entry indices) is
//     cut into equal pieces, one per thread (SpMV) or per 16-lane group
//     (SpMM), so a few very long rows spread over the whole workgroup
//     instead of holding one group while the others idle.  Rows cut by a
//     piece boundary are completed from per-piece partial sums in piece
//     order (deterministic; no floating-point atomics).
// For the triangular solves a task is a whole block: one workgroup of 1024
// threads runs the block's levels in order with a barrier between levels,
// so a batch of shallow, independent level structures costs one launch
// instead of one per level; these tasks are ordered by cost, largest first,
// so the long ones start early and the short ones fill the tail.
//
// Queue.  A launch keeps as many workgroups as fit on the chip at once;
// each takes the next task index from device counters: one queue per XCD
// over a contiguous range of the row-ordered tasks (one queue for the
// whole-block tasks), a workgroup moving on to the other queues once its
// own is empty.  The last workgroup to leave resets the counters, so the
// next launch on the stream starts from zero without a memset node
// (launches that share a plan must be ordered on one stream).
#include <hip/hip_cooperative_groups.h>

#include <algorithm>
#include <vector>

#include "internal.hpp"

namespace csrad {
namespace {

constexpr int kThreads = 256;
constexpr int kTriThreads = 1024;       // workgroup of the per-block solves and IC(0)
constexpr int kSlotsPerCu = 4;          // fallback when the occupancy query fails
constexpr int kMergeRowCap = 2048;      // rows of one merge task (staged in LDS)
constexpr int kStageCap = 2560;         // staged variant: entries per 256 rows

enum : int32_t { kKindMerge = 8, kKindStaged = 9 };

struct BTask {
  int32_t r0, r1, kind, block;
};

// ---------------------------------------------------------------------
// Queue.  The tasks are dealt from nq queues (ctr[kNqSlot]: 1, or one per
// XCD), queue q holding the contiguous task range
// [ntasks*q/nq, ntasks*(q+1)/nq).  A workgroup starts on queue
// blockIdx.x % nq (the dispatcher places workgroup b on XCD b % 8, so each
// XCD works through its own range of rows and keeps that range's dense
// operands in its own L2) and moves on to the next queue when its own is
// exhausted.  ctr[0..nq) are the queue heads, ctr[kLeaveSlot] counts the
// workgroups that have left.
// ---------------------------------------------------------------------
constexpr int kQueues = kXcds;
constexpr int kLeaveSlot = kQueues;
constexpr int kNqSlot = kQueues + 1;
constexpr int kCtrWords = kQueues + 2;

// Next task index for this workgroup (thread 0 only); `tried` counts the
// queues found exhausted so far.  ntasks when every queue is exhausted.
__device__ __forceinline__ int fetch_task(unsigned* ctr, int ntasks, int nq, int& tried) {
  const int home = (int)(blockIdx.x % (unsigned)nq);
  while (tried < nq) {
    const int q = (home + tried) % nq;
    const long long lo = (long long)ntasks * q / nq, hi = (long long)ntasks * (q + 1) / nq;
    const unsigned idx = atomicAdd(&ctr[q], 1u);
    if (lo + idx < hi) return (int)(lo + idx);
    ++tried;
  }
  return ntasks;
}

__device__ __forceinline__ void leave_queue(unsigned* ctr, int nq) {
  // the last workgroup out finds every other one gone (each has drawn an
  // index past the end of every queue) and rewinds the queues for the next
  // launch
  if (threadIdx.x == 0 && atomicAdd(&ctr[kLeaveSlot], 1u) == gridDim.x - 1) {
    for (int q = 0; q < nq; ++q) atomicExch(&ctr[q], 0u);
    atomicExch(&ctr[kLeaveSlot], 0u);
  }
}

// Runs body(task) for every task this workgroup draws.  The next index is
// requested while the current task runs.
template <typename F>
__device__ __forceinline__ void run_queue(const BTask* __restrict__ tasks, int ntasks,
                                          unsigned* ctr, F&& body) {
  __shared__ int s_next;
  const int nq = (int)ctr[kNqSlot];
  int tried = 0;  // thread 0's
  if (threadIdx.x == 0) s_next = fetch_task(ctr, ntasks, nq, tried);
  __syncthreads();
  int t = s_next;
  while (t < ntasks) {
    int nxt = 0;
    if (threadIdx.x == 0) nxt = fetch_task(ctr, ntasks, nq, tried);
    const int4 raw = *reinterpret_cast<const int4*>(&tasks[t]);
    body(BTask{raw.x, raw.y, raw.z, raw.w});
    __syncthreads();
    if (threadIdx.x == 0) s_next = nxt;
    __syncthreads();
    t = s_next;
  }
  leave_queue(ctr, nq);
}

// Merge-path split of diagonal d between row ends a[0..nr) (exclusive
// prefix of row lengths shifted: a[i] = end of row i, relative) and the
// entry indices 0..ne-1: returns rows consumed x (entries consumed d - x).
__device__ __forceinline__ int merge_split(const int32_t* a, int nr, int ne, int d) {
  int lo = max(d - ne, 0), hi = min(d, nr);
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] <= d - mid - 1) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// ---------------------------------------------------------------------
// SpMV forward: y = A x over the tasks.
// ---------------------------------------------------------------------
template <typename T, int G>
__device__ __forceinline__ void spmv_rows(const BTask& tk, const int32_t* __restrict__ rp,
                                          const int32_t* __restrict__ ci,
                                          const T* __restrict__ v, const T* __restrict__ x,
                                          T* __restrict__ y) {
  constexpr int RPP = kThreads / G;
  const int sub = threadIdx.x % G;
  for (int base = tk.r0; base < tk.r1; base += RPP) {
    const int r = base + threadIdx.x / G;
    const bool ok = r < tk.r1;
    T s = 0;
    if (ok) {
      const int e1 = rp[r + 1];
      for (int e = rp[r] + sub; e < e1; e += G) s += ld_stream(&v[e]) * x[ld_stream(&ci[e])];
    }
    s = group_sum<G>(s);
    if (ok && sub == 0) y[r] = s;
  }
}

template <typename T>
__device__ __forceinline__ void spmv_staged(const BTask& tk, const int32_t* __restrict__ rp,
                                            const int32_t* __restrict__ ci,
                                            const T* __restrict__ v, const T* __restrict__ x,
                                            T* __restrict__ y, T* prod) {
  for (int r0 = tk.r0; r0 < tk.r1; r0 += kThreads) {
    const int r1 = min(r0 + kThreads, tk.r1);
    const int e0 = rp[r0], cnt = rp[r1] - e0;
    if (cnt <= kStageCap) {
      for (int t = threadIdx.x; t < cnt; t += 4 * kThreads) {
        T pr[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int tt = t + u * kThreads;
          pr[u] = tt < cnt ? ld_stream(&v[e0 + tt]) * x[ld_stream(&ci[e0 + tt])] : T(0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (t + u * kThreads < cnt) prod[t + u * kThreads] = pr[u];
      }
      __syncthreads();
      const int r = r0 + threadIdx.x;
      if (r < r1) {
        const int a = rp[r] - e0, b = rp[r + 1] - e0;
        T acc = 0;
        for (int t = a; t < b; ++t) acc += prod[t];
        y[r] = acc;
      }
      __syncthreads();
    } else {
      const int lane = threadIdx.x % kWave;
      for (int base = r0; base < r1; base += kThreads / kWave) {
        const int r = base + threadIdx.x / kWave;
        T acc = 0;
        if (r < r1)
          for (int e = rp[r] + lane; e < rp[r + 1]; e += kWave)
            acc += ld_stream(&v[e]) * x[ld_stream(&ci[e])];
        acc = group_sum<kWave>(acc);
        if (r < r1 && lane == 0) y[r] = acc;
      }
    }
  }
}

// LDS layout of the merge variants.
template <typename T>
struct MergeLds {
  int32_t rowend[kMergeRowCap];  // end of each task row, relative to the task's first entry
  int32_t xs[kThreads + 1];      // row split of each piece
  int32_t crow[kThreads];        // row of the piece's carry-out, or -1
  int32_t hrow[kThreads];        // row whose tail the piece holds, or -1
  T carry[kThreads];
  T head[kThreads];
};

// Loads the task's row ends and each piece's split; returns (nr, ne, base e0).
template <typename T>
__device__ __forceinline__ void merge_setup(const BTask& tk, const int32_t* __restrict__ rp,
                                            MergeLds<T>& L, int pieces, int& nr, int& ne,
                                            int& e0) {
  nr = tk.r1 - tk.r0;
  e0 = rp[tk.r0];
  ne = rp[tk.r1] - e0;
  for (int i = threadIdx.x; i < nr; i += kThreads) L.rowend[i] = rp[tk.r0 + i + 1] - e0;
  __syncthreads();
  const long long len = (long long)nr + ne;
  for (int p = threadIdx.x; p <= pieces; p += kThreads) {
    const int d = (int)(len * p / pieces);
    L.xs[p] = merge_split(L.rowend, nr, ne, d);
  }
  __syncthreads();
}

__device__ __forceinline__ int row_start(const int32_t* rowend, int i) {
  return i > 0 ? rowend[i - 1] : 0;
}

template <typename T>
__device__ __forceinline__ void spmv_merge(const BTask& tk, const int32_t* __restrict__ rp,
                                           const int32_t* __restrict__ ci,
                                           const T* __restrict__ v, const T* __restrict__ x,
                                           T* __restrict__ y, MergeLds<T>& L) {
  int nr, ne, e0;
  merge_setup<T>(tk, rp, L, kThreads, nr, ne, e0);
  const long long len = (long long)nr + ne;
  const int p = threadIdx.x;
  const int x0 = L.xs[p], x1 = L.xs[p + 1];
  const int y0 = (int)(len * p / kThreads) - x0, y1 = (int)(len * (p + 1) / kThreads) - x1;
  T acc = 0;
  int yy = y0;
  int hrow = -1;
  T head = 0;
  for (int row = x0; row < x1; ++row) {
    const int rend = L.rowend[row];
    for (; yy < rend; ++yy) acc += ld_stream(&v[e0 + yy]) * x[ld_stream(&ci[e0 + yy])];
    if (row == x0 && row_start(L.rowend, row) < y0) {
      hrow = row;  // tail of a row begun by earlier pieces
      head = acc;
    } else {
      y[tk.r0 + row] = acc;
    }
    acc = 0;
  }
  for (; yy < y1; ++yy) acc += ld_stream(&v[e0 + yy]) * x[ld_stream(&ci[e0 + yy])];
  const bool has_carry = x1 < nr && row_start(L.rowend, x1) < y1;
  L.crow[p] = has_carry ? x1 : -1;
  L.carry[p] = acc;
  L.hrow[p] = hrow;
  L.head[p] = head;
  __syncthreads();
  // a chain of pieces carrying into one row is summed in piece order by
  // its first piece, then the tail held by the piece that completes it
  const int r = L.crow[p];
  if (r >= 0 && (p == 0 || L.crow[p - 1] != r)) {
    T s = L.carry[p];
    int q = p + 1;
    while (q < kThreads && L.crow[q] == r) s += L.carry[q++];
    if (q < kThreads && L.hrow[q] == r) s += L.head[q];
    y[tk.r0 + r] = s;
  }
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_batch_spmv(const BTask* __restrict__ tasks,
                                                         int ntasks, unsigned* ctr,
                                                         const int32_t* __restrict__ rp,
                                                         const int32_t* __restrict__ ci,
                                                         const T* __restrict__ v,
                                                         const T* __restrict__ x,
                                                         T* __restrict__ y) {
  __shared__ __align__(16) char smem[sizeof(MergeLds<T>) > kStageCap * sizeof(T)
                                         ? sizeof(MergeLds<T>)
                                         : kStageCap * sizeof(T)];
  run_queue(tasks, ntasks, ctr, [&](const BTask& tk) {
    switch (tk.kind) {
      case 1: spmv_rows<T, 1>(tk, rp, ci, v, x, y); break;
      case 2: spmv_rows<T, 2>(tk, rp, ci, v, x, y); break;
      case 3: spmv_rows<T, 4>(tk, rp, ci, v, x, y); break;
      case 4: spmv_rows<T, 8>(tk, rp, ci, v, x, y); break;
      case 5: spmv_rows<T, 16>(tk, rp, ci, v, x, y); break;
      case 6: spmv_rows<T, 32>(tk, rp, ci, v, x, y); break;
      case 7: spmv_rows<T, 64>(tk, rp, ci, v, x, y); break;
      case kKindMerge: spmv_merge<T>(tk, rp, ci, v, x, y, *reinterpret_cast<MergeLds<T>*>(smem)); break;
      default: spmv_staged<T>(tk, rp, ci, v, x, y, reinterpret_cast<T*>(smem)); break;
    }
  });
}

// ---------------------------------------------------------------------
// SpMV backward over A^T (tasks over A^T's rows, i.e. A's columns):
//   gx[j] = sum_t vals[perm t] gy[ciT t],  gv[perm t] = gy[ciT t] x[j].
// ---------------------------------------------------------------------
template <typename T, int G, bool GX, bool GV>
__device__ __forceinline__ void spmvb_rows(const BTask& tk, const int32_t* __restrict__ rpT,
                                           const int32_t* __restrict__ ciT,
                                           const int32_t* __restrict__ perm,
                                           const T* __restrict__ v, const T* __restrict__ x,
                                           const T* __restrict__ gy, T* __restrict__ gx,
                                           T* __restrict__ gv) {
  constexpr int RPP = kThreads / G;
  const int sub = threadIdx.x % G;
  for (int base = tk.r0; base < tk.r1; base += RPP) {
    const int j = base + threadIdx.x / G;
    const bool ok = j < tk.r1;
    T s = 0;
    if (ok) {
      const T xj = GV ? x[j] : T(0);
      const int t1 = rpT[j + 1];
      for (int t = rpT[j] + sub; t < t1; t += G) {
        const int i = ld_stream(&ciT[t]);
        const int e = ld_stream(&perm[t]);
        const T g = gy[i];
        if (GX) s += v[e] * g;
        if (GV) gv[e] = g * xj;
      }
    }
    if (GX) {
      s = group_sum<G>(s);
      if (ok && sub == 0) gx[j] = s;
    }
  }
}

template <typename T, bool GX, bool GV>
__device__ __forceinline__ void spmvb_merge(const BTask& tk, const int32_t* __restrict__ rpT,
                                            const int32_t* __restrict__ ciT,
                                            const int32_t* __restrict__ perm,
                                            const T* __restrict__ v, const T* __restrict__ x,
                                            const T* __restrict__ gy, T* __restrict__ gx,
                                            T* __restrict__ gv, MergeLds<T>& L) {
  int nr, ne, e0;
  merge_setup<T>(tk, rpT, L, kThreads, nr, ne, e0);
  const long long len = (long long)nr + ne;
  const int p = threadIdx.x;
  const int x0 = L.xs[p], x1 = L.xs[p + 1];
  const int y0 = (int)(len * p / kThreads) - x0, y1 = (int)(len * (p + 1) / kThreads) - x1;
  T acc = 0;
  int yy = y0;
  int hrow = -1;
  T head = 0;
  for (int row = x0; row <= x1 && row < nr; ++row) {
    const int rend = row < x1 ? L.rowend[row] : y1;
    const T xj = GV ? x[tk.r0 + row] : T(0);
    for (; yy < rend; ++yy) {
      const int i = ld_stream(&ciT[e0 + yy]);
      const int e = ld_stream(&perm[e0 + yy]);
      const T g = gy[i];
      if (GX) acc += v[e] * g;
      if (GV) gv[e] = g * xj;
    }
    if (row == x1) break;
    if (GX) {
      if (row == x0 && row_start(L.rowend, row) < y0) {
        hrow = row;
        head = acc;
      } else {
        gx[tk.r0 + row] = acc;
      }
    }
    acc = 0;
  }
  if (GX) {
    const bool has_carry = x1 < nr && row_start(L.rowend, x1) < y1;
    L.crow[p] = has_carry ? x1 : -1;
    L.carry[p] = acc;
    L.hrow[p] = hrow;
    L.head[p] = head;
    __syncthreads();
    const int r = L.crow[p];
    if (r >= 0 && (p == 0 || L.crow[p - 1] != r)) {
      T s = L.carry[p];
      int q = p + 1;
      while (q < kThreads && L.crow[q] == r) s += L.carry[q++];
      if (q < kThreads && L.hrow[q] == r) s += L.head[q];
      gx[tk.r0 + r] = s;
    }
  }
  __syncthreads();
}

template <typename T, bool GX, bool GV>
__global__ __launch_bounds__(kThreads) void k_batch_spmv_bwd(
    const BTask* __restrict__ tasks, int ntasks, unsigned* ctr, const int32_t* __restrict__ rpT,
    const int32_t* __restrict__ ciT, const int32_t* __restrict__ perm, const T* __restrict__ v,
    const T* __restrict__ x, const T* __restrict__ gy, T* __restrict__ gx, T* __restrict__ gv) {
  __shared__ __align__(16) char smem[sizeof(MergeLds<T>)];
  run_queue(tasks, ntasks, ctr, [&](const BTask& tk) {
    switch (tk.kind) {
      case 1: spmvb_rows<T, 1, GX, GV>(tk, rpT, ciT, perm, v, x, gy, gx, gv); break;
      case 2: spmvb_rows<T, 2, GX, GV>(tk, rpT, ciT, perm, v, x, gy, gx, gv); break;
      case 3: spmvb_rows<T, 4, GX, GV>(tk, rpT, ciT, perm, v, x, gy, gx, gv); break;
      case 5: spmvb_rows<T, 16, GX, GV>(tk, rpT, ciT, perm, v, x, gy, gx, gv); break;
      case 6: spmvb_rows<T, 32, GX, GV>(tk, rpT, ciT, perm, v, x, gy, gx, gv); break;
      case 7: spmvb_rows<T, 64, GX, GV>(tk, rpT, ciT, perm, v, x, gy, gx, gv); break;
      case kKindMerge:
        spmvb_merge<T, GX, GV>(tk, rpT, ciT, perm, v, x, gy, gx, gv,
                               *reinterpret_cast<MergeLds<T>*>(smem));
        break;
      default: spmvb_rows<T, 8, GX, GV>(tk, rpT, ciT, perm, v, x, gy, gx, gv); break;
    }
  });
}

// ---------------------------------------------------------------------
// SpMM.  A group of 16 lanes (one DPP row) owns a sparse row; each lane
// owns VW consecutive columns of a chunk of 16*VW columns.  Per batch of 8
// entries, lanes 0..7 of the group load the entries once and DPP
// row_newbcast hands entry u to every lane.
// ---------------------------------------------------------------------
constexpr int kGrp = 16;
constexpr int kGroups = kThreads / kGrp;
constexpr int kEb = 8;

template <int U>
__device__ __forceinline__ int bc16(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x150 + U, 0xF, 0xF, false);
}
template <int U>
__device__ __forceinline__ float bc16(float v) {
  return __int_as_float(bc16<U>(__float_as_int(v)));
}
template <int U>
__device__ __forceinline__ double bc16(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = bc16<U>((int)(b & 0xffffffffll));
  const int hi = bc16<U>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// out[u] = the value of lane S*u of the DPP row, u < kEb.
template <typename V, int S = 1, int U = 0>
__device__ __forceinline__ void bc_all(V mine, V (&out)[kEb]) {
  if constexpr (U < kEb) {
    out[U] = bc16<S * U>(mine);
    bc_all<V, S, U + 1>(mine, out);
  }
}

template <typename T, int VW>
__device__ __forceinline__ Vec<T, VW> ld_or_zero(const T* p, bool ok) {
  if (ok) return load_vec<T, VW>(p);
  Vec<T, VW> z;
#pragma unroll
  for (int w = 0; w < VW; ++w) z.v[w] = T(0);
  return z;
}

// acc += sum over entries [ea, eb) of vals[e] * B[ci[e], col..col+VW)
template <typename T, int VW>
__device__ __forceinline__ void spmm_seg(int ea, int eb, int col, bool act, int lr,
                                         const int32_t* __restrict__ ci,
                                         const T* __restrict__ v, const T* __restrict__ B,
                                         long long ldb, T (&acc)[VW]) {
  for (int e = ea; e < eb; e += kEb) {
    const int cnt = min(kEb, eb - e);
    int myc = 0;
    T myv = 0;
    if (lr < cnt) {
      myc = ld_stream(&ci[e + lr]);
      myv = ld_stream(&v[e + lr]);
    }
    int c[kEb];
    T a[kEb];
    bc_all<int>(myc, c);
    bc_all<T>(myv, a);
    Vec<T, VW> bv[kEb];
#pragma unroll
    for (int u = 0; u < kEb; ++u) bv[u] = ld_or_zero<T, VW>(B + (long long)c[u] * ldb + col, act && u < cnt);
#pragma unroll
    for (int u = 0; u < kEb; ++u)
#pragma unroll
      for (int w = 0; w < VW; ++w) acc[w] += a[u] * bv[u].v[w];
  }
}

template <typename T, int VW>
__device__ __forceinline__ void put_row(T* __restrict__ C, long long ldc, int row, int col,
                                        bool act, const T (&acc)[VW]) {
  if (!act) return;
  Vec<T, VW> o;
#pragma unroll
  for (int w = 0; w < VW; ++w) o.v[w] = acc[w];
  store_vec_stream<T, VW>(C + (long long)row * ldc + col, o);
}

template <typename T, int VW>
__device__ __forceinline__ void spmm_rows(const BTask& tk, int k, const int32_t* __restrict__ rp,
                                          const int32_t* __restrict__ ci,
                                          const T* __restrict__ v, const T* __restrict__ B,
                                          long long ldb, T* __restrict__ C, long long ldc) {
  const int g = threadIdx.x / kGrp, l = threadIdx.x % kGrp;
  for (int row = tk.r0 + g; row < tk.r1; row += kGroups) {
    const int e0 = rp[row], e1 = rp[row + 1];
    for (int c0 = 0; c0 < k; c0 += kGrp * VW) {
      const int col = c0 + l * VW;
      const bool act = col < k;
      T acc[VW];
#pragma unroll
      for (int w = 0; w < VW; ++w) acc[w] = T(0);
      spmm_seg<T, VW>(e0, e1, col, act, l, ci, v, B, ldb, acc);
      put_row<T, VW>(C, ldc, row, col, act, acc);
    }
  }
}

template <typename T, int VW>
struct MergeLdsMM {
  int32_t rowend[kMergeRowCap];
  int32_t xs[kGroups + 1];
  int32_t crow[kGroups];
  int32_t hrow[kGroups];
  T carry[kGroups][kGrp * VW];
  T head[kGroups][kGrp * VW];
};

template <typename T, int VW>
__device__ __forceinline__ void spmm_merge(const BTask& tk, int k,
                                           const int32_t* __restrict__ rp,
                                           const int32_t* __restrict__ ci,
                                           const T* __restrict__ v, const T* __restrict__ B,
                                           long long ldb, T* __restrict__ C, long long ldc,
                                           MergeLdsMM<T, VW>& L) {
  const int nr = tk.r1 - tk.r0;
  const int e0 = rp[tk.r0];
  const int ne = rp[tk.r1] - e0;
  for (int i = threadIdx.x; i < nr; i += kThreads) L.rowend[i] = rp[tk.r0 + i + 1] - e0;
  __syncthreads();
  const long long len = (long long)nr + ne;
  for (int p = threadIdx.x; p <= kGroups; p += kThreads)
    L.xs[p] = merge_split(L.rowend, nr, ne, (int)(len * p / kGroups));
  __syncthreads();
  const int g = threadIdx.x / kGrp, l = threadIdx.x % kGrp;
  const int x0 = L.xs[g], x1 = L.xs[g + 1];
  const int y0 = (int)(len * g / kGroups) - x0, y1 = (int)(len * (g + 1) / kGroups) - x1;
  for (int c0 = 0; c0 < k; c0 += kGrp * VW) {
    const int col = c0 + l * VW;
    const bool act = col < k;
    T acc[VW];
#pragma unroll
    for (int w = 0; w < VW; ++w) acc[w] = T(0);
    int yy = y0, hrow = -1;
    for (int row = x0; row < x1; ++row) {
      const int rend = L.rowend[row];
      spmm_seg<T, VW>(e0 + yy, e0 + rend, col, act, l, ci, v, B, ldb, acc);
      yy = rend;
      if (row == x0 && row_start(L.rowend, row) < y0) {
        hrow = row;
#pragma unroll
        for (int w = 0; w < VW; ++w) L.head[g][l * VW + w] = acc[w];
      } else {
        put_row<T, VW>(C, ldc, tk.r0 + row, col, act, acc);
      }
#pragma unroll
      for (int w = 0; w < VW; ++w) acc[w] = T(0);
    }
    spmm_seg<T, VW>(e0 + yy, e0 + y1, col, act, l, ci, v, B, ldb, acc);
    const bool has_carry = x1 < nr && row_start(L.rowend, x1) < y1;
    if (l == 0) {
      L.crow[g] = has_carry ? x1 : -1;
      L.hrow[g] = hrow;
    }
#pragma unroll
    for (int w = 0; w < VW; ++w) L.carry[g][l * VW + w] = acc[w];
    __syncthreads();
    const int r = L.crow[g];
    if (r >= 0 && (g == 0 || L.crow[g - 1] != r)) {
      T s[VW];
#pragma unroll
      for (int w = 0; w < VW; ++w) s[w] = L.carry[g][l * VW + w];
      int q = g + 1;
      for (; q < kGroups && L.crow[q] == r; ++q)
#pragma unroll
        for (int w = 0; w < VW; ++w) s[w] += L.carry[q][l * VW + w];
      if (q < kGroups && L.hrow[q] == r)
#pragma unroll
        for (int w = 0; w < VW; ++w) s[w] += L.head[q][l * VW + w];
      put_row<T, VW>(C, ldc, tk.r0 + r, col, act, s);
    }
    __syncthreads();
  }
}

template <typename T, int VW>
__global__ __launch_bounds__(kThreads) void k_batch_spmm(const BTask* __restrict__ tasks,
                                                         int ntasks, unsigned* ctr, int k,
                                                         const int32_t* __restrict__ rp,
                                                         const int32_t* __restrict__ ci,
                                                         const T* __restrict__ v,
                                                         const T* __restrict__ B, long long ldb,
                                                         T* __restrict__ C, long long ldc) {
  __shared__ __align__(16) char smem[sizeof(MergeLdsMM<T, VW>)];
  run_queue(tasks, ntasks, ctr, [&](const BTask& tk) {
    if (tk.kind == kKindMerge)
      spmm_merge<T, VW>(tk, k, rp, ci, v, B, ldb, C, ldc,
                        *reinterpret_cast<MergeLdsMM<T, VW>*>(smem));
    else
      spmm_rows<T, VW>(tk, k, rp, ci, v, B, ldb, C, ldc);
  });
}

// ---------------------------------------------------------------------
// SpMM backward over A^T (fused): for row j of A^T (column j of A)
//   gB[j,:] = sum_t vals[perm t] G[ciT t, :]
//   gv[perm t] = <G[ciT t, :], B[j, :]>
// ---------------------------------------------------------------------
template <typename T, int VW, bool GB, bool GV>
__device__ __forceinline__ void spmmb_seg(int ta, int tb, int col, bool act, int lr,
                                          const int32_t* __restrict__ ciT,
                                          const int32_t* __restrict__ perm,
                                          const T* __restrict__ v, const T* __restrict__ G,
                                          long long ldg, const Vec<T, VW>& bj, int c0,
                                          T* __restrict__ gv, T (&acc)[VW]) {
  // entry u of a batch sits in lanes 2u and 2u+1 of the 16-lane group (the
  // layout the scattered row sums leave), as in the per-matrix kernel: the
  // two give the same bits
  static_assert(kGrp == 16 && kEb == 8, "the scattered row sums take 8 values over 16 lanes");
  for (int t = ta; t < tb; t += kEb) {
    const int cnt = min(kEb, tb - t);
    const int me = lr >> 1;
    int myi = 0, mye = 0;
    T mya = 0;
    if (me < cnt) {
      myi = ld_stream(&ciT[t + me]);
      mye = ld_stream(&perm[t + me]);
      if (GB) mya = v[mye];
    }
    int i[kEb];
    bc_all<int, 2>(myi, i);
    Vec<T, VW> g[kEb];
#pragma unroll
    for (int u = 0; u < kEb; ++u) g[u] = ld_or_zero<T, VW>(G + (long long)i[u] * ldg + col, act && u < cnt);
    if (GB) {
      T a[kEb];
      bc_all<T, 2>(mya, a);
#pragma unroll
      for (int u = 0; u < kEb; ++u)
#pragma unroll
        for (int w = 0; w < VW; ++w) acc[w] += a[u] * g[u].v[w];
      // keeps the multiply-adds ahead of the dot products (sunk past them,
      // they would keep the broadcast values live through the reductions)
#pragma unroll
      for (int w = 0; w < VW; ++w) asm volatile("" : "+v"(acc[w]));
    }
    if (GV) {
      T d[kEb];
#pragma unroll
      for (int u = 0; u < kEb; ++u) {
        d[u] = 0;
#pragma unroll
        for (int w = 0; w < VW; ++w) d[u] += g[u].v[w] * bj.v[w];
      }
      const T mine = row_sum_scatter8<T>(d, lr);
      if ((lr & 1) == 0 && me < cnt) gv[mye] = c0 == 0 ? mine : gv[mye] + mine;
    }
  }
}

template <typename T, int VW, bool GB, bool GV>
__device__ __forceinline__ void spmmb_rows(const BTask& tk, int k, const int32_t* __restrict__ rpT,
                                           const int32_t* __restrict__ ciT,
                                           const int32_t* __restrict__ perm,
                                           const T* __restrict__ v, const T* __restrict__ B,
                                           long long ldb, const T* __restrict__ G, long long ldg,
                                           T* __restrict__ gB, long long ldgb,
                                           T* __restrict__ gv) {
  const int g = threadIdx.x / kGrp, l = threadIdx.x % kGrp;
  for (int j = tk.r0 + g; j < tk.r1; j += kGroups) {
    const int t0 = rpT[j], t1 = rpT[j + 1];
    for (int c0 = 0; c0 < k; c0 += kGrp * VW) {
      const int col = c0 + l * VW;
      const bool act = col < k;
      Vec<T, VW> bj;
      if (GV) bj = ld_or_zero<T, VW>(B + (long long)j * ldb + col, act);
      T acc[VW];
#pragma unroll
      for (int w = 0; w < VW; ++w) acc[w] = T(0);
      spmmb_seg<T, VW, GB, GV>(t0, t1, col, act, l, ciT, perm, v, G, ldg, bj, c0, gv, acc);
      if (GB) put_row<T, VW>(gB, ldgb, j, col, act, acc);
    }
  }
}

template <typename T, int VW, bool GB, bool GV>
__device__ __forceinline__ void spmmb_merge(const BTask& tk, int k,
                                            const int32_t* __restrict__ rpT,
                                            const int32_t* __restrict__ ciT,
                                            const int32_t* __restrict__ perm,
                                            const T* __restrict__ v, const T* __restrict__ B,
                                            long long ldb, const T* __restrict__ G, long long ldg,
                                            T* __restrict__ gB, long long ldgb,
                                            T* __restrict__ gv, MergeLdsMM<T, VW>& L) {
  const int nr = tk.r1 - tk.r0;
  const int e0 = rpT[tk.r0];
  const int ne = rpT[tk.r1] - e0;
  for (int i = threadIdx.x; i < nr; i += kThreads) L.rowend[i] = rpT[tk.r0 + i + 1] - e0;
  __syncthreads();
  const long long len = (long long)nr + ne;
  for (int p = threadIdx.x; p <= kGroups; p += kThreads)
    L.xs[p] = merge_split(L.rowend, nr, ne, (int)(len * p / kGroups));
  __syncthreads();
  const int g = threadIdx.x / kGrp, l = threadIdx.x % kGrp;
  const int x0 = L.xs[g], x1 = L.xs[g + 1];
  const int y0 = (int)(len * g / kGroups) - x0, y1 = (int)(len * (g + 1) / kGroups) - x1;
  for (int c0 = 0; c0 < k; c0 += kGrp * VW) {
    const int col = c0 + l * VW;
    const bool act = col < k;
    T acc[VW];
#pragma unroll
    for (int w = 0; w < VW; ++w) acc[w] = T(0);
    int yy = y0, hrow = -1;
    for (int row = x0; row <= x1 && row < nr; ++row) {
      const int rend = row < x1 ? L.rowend[row] : y1;
      Vec<T, VW> bj;
      if (GV) bj = ld_or_zero<T, VW>(B + (long long)(tk.r0 + row) * ldb + col, act);
      spmmb_seg<T, VW, GB, GV>(e0 + yy, e0 + rend, col, act, l, ciT, perm, v, G, ldg, bj, c0, gv,
                               acc);
      yy = rend;
      if (row == x1) break;
      if (GB) {
        if (row == x0 && row_start(L.rowend, row) < y0) {
          hrow = row;
#pragma unroll
          for (int w = 0; w < VW; ++w) L.head[g][l * VW + w] = acc[w];
        } else {
          put_row<T, VW>(gB, ldgb, tk.r0 + row, col, act, acc);
        }
      }
#pragma unroll
      for (int w = 0; w < VW; ++w) acc[w] = T(0);
    }
    if (GB) {
      const bool has_carry = x1 < nr && row_start(L.rowend, x1) < y1;
      if (l == 0) {
        L.crow[g] = has_carry ? x1 : -1;
        L.hrow[g] = hrow;
      }
#pragma unroll
      for (int w = 0; w < VW; ++w) L.carry[g][l * VW + w] = acc[w];
      __syncthreads();
      const int r = L.crow[g];
      if (r >= 0 && (g == 0 || L.crow[g - 1] != r)) {
        T s[VW];
#pragma unroll
        for (int w = 0; w < VW; ++w) s[w] = L.carry[g][l * VW + w];
        int q = g + 1;
        for (; q < kGroups && L.crow[q] == r; ++q)
#pragma unroll
          for (int w = 0; w < VW; ++w) s[w] += L.carry[q][l * VW + w];
        if (q < kGroups && L.hrow[q] == r)
#pragma unroll
          for (int w = 0; w < VW; ++w) s[w] += L.head[q][l * VW + w];
        put_row<T, VW>(gB, ldgb, tk.r0 + r, col, act, s);
      }
    }
    __syncthreads();
  }
}

template <typename T, int VW, bool GB, bool GV>
__global__ __launch_bounds__(kThreads) void k_batch_spmm_bwd(
    const BTask* __restrict__ tasks, int ntasks, unsigned* ctr, int k,
    const int32_t* __restrict__ rpT, const int32_t* __restrict__ ciT,
    const int32_t* __restrict__ perm, const T* __restrict__ v, const T* __restrict__ B,
    long long ldb, const T* __restrict__ G, long long ldg, T* __restrict__ gB, long long ldgb,
    T* __restrict__ gv) {
  __shared__ __align__(16) char smem[sizeof(MergeLdsMM<T, VW>)];
  run_queue(tasks, ntasks, ctr, [&](const BTask& tk) {
    if (tk.kind == kKindMerge)
      spmmb_merge<T, VW, GB, GV>(tk, k, rpT, ciT, perm, v, B, ldb, G, ldg, gB, ldgb, gv,
                                 *reinterpret_cast<MergeLdsMM<T, VW>*>(smem));
    else
      spmmb_rows<T, VW, GB, GV>(tk, k, rpT, ciT, perm, v, B, ldb, G, ldg, gB, ldgb, gv);
  });
}

// ---------------------------------------------------------------------
// Value gradients alone, row-wise over A (the plan of A), for a backward
// split into A^T products over A^T's plan and these coalesced passes:
//   SpMV:  gvals[e] = gy[row e] x[col e]
//   SpMM:  gvals[e] = <gC[row e, :], B[col e, :]>
// ---------------------------------------------------------------------
template <typename T, int G>
__device__ __forceinline__ void sddmv_rows(const BTask& tk, const int32_t* __restrict__ rp,
                                           const int32_t* __restrict__ ci,
                                           const T* __restrict__ x, const T* __restrict__ gy,
                                           T* __restrict__ gv) {
  constexpr int RPP = kThreads / G;
  const int sub = threadIdx.x % G;
  for (int base = tk.r0; base < tk.r1; base += RPP) {
    const int r = base + threadIdx.x / G;
    if (r < tk.r1) {
      const T g = gy[r];
      const int e1 = rp[r + 1];
      for (int e = rp[r] + sub; e < e1; e += G) gv[e] = g * x[ld_stream(&ci[e])];
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_batch_sddmv(const BTask* __restrict__ tasks,
                                                          int ntasks, unsigned* ctr,
                                                          const int32_t* __restrict__ rp,
                                                          const int32_t* __restrict__ ci,
                                                          const T* __restrict__ x,
                                                          const T* __restrict__ gy,
                                                          T* __restrict__ gv) {
  run_queue(tasks, ntasks, ctr, [&](const BTask& tk) {
    switch (tk.kind) {
      case 1: sddmv_rows<T, 1>(tk, rp, ci, x, gy, gv); break;
      case 2: sddmv_rows<T, 2>(tk, rp, ci, x, gy, gv); break;
      case 3: sddmv_rows<T, 4>(tk, rp, ci, x, gy, gv); break;
      case 5: sddmv_rows<T, 16>(tk, rp, ci, x, gy, gv); break;
      case 6: sddmv_rows<T, 32>(tk, rp, ci, x, gy, gv); break;
      case 7: sddmv_rows<T, 64>(tk, rp, ci, x, gy, gv); break;
      default: sddmv_rows<T, 8>(tk, rp, ci, x, gy, gv); break;
    }
  });
}

template <typename T, int VW>
__global__ __launch_bounds__(kThreads) void k_batch_sddmm(
    const BTask* __restrict__ tasks, int ntasks, unsigned* ctr, int k,
    const int32_t* __restrict__ rp, const int32_t* __restrict__ ci, const T* __restrict__ B,
    long long ldb, const T* __restrict__ G, long long ldg, T* __restrict__ gv) {
  run_queue(tasks, ntasks, ctr, [&](const BTask& tk) {
    const int g = threadIdx.x / kGrp, l = threadIdx.x % kGrp;
    for (int row = tk.r0 + g; row < tk.r1; row += kGroups) {
      const int e0 = rp[row], e1 = rp[row + 1];
      for (int c0 = 0; c0 < k; c0 += kGrp * VW) {
        const int col = c0 + l * VW;
        const bool act = col < k;
        const Vec<T, VW> gi = ld_or_zero<T, VW>(G + (long long)row * ldg + col, act);
        for (int eb = e0; eb < e1; eb += kEb) {
          const int cnt = min(kEb, e1 - eb);
          const int myc = l < cnt ? ld_stream(&ci[eb + l]) : 0;
          int c[kEb];
          bc_all<int>(myc, c);
          Vec<T, VW> bv[kEb];
#pragma unroll
          for (int u = 0; u < kEb; ++u)
            bv[u] = ld_or_zero<T, VW>(B + (long long)c[u] * ldb + col, act && u < cnt);
          // the same dots and scattered row sums as the fused backward (the
          // split and fused forms give the same bits): entry u ends in lane 2u
          T d[kEb];
#pragma unroll
          for (int u = 0; u < kEb; ++u) {
            d[u] = 0;
#pragma unroll
            for (int w = 0; w < VW; ++w) d[u] += gi.v[w] * bv[u].v[w];
          }
          const T mine = row_sum_scatter8<T>(d, l);
          const int me = l >> 1;
          if ((l & 1) == 0 && me < cnt) gv[eb + me] = c0 == 0 ? mine : gv[eb + me] + mine;
        }
      }
    }
  });
}

// ---------------------------------------------------------------------
// Triangular solves: a task is one block; lv_lo/lv_hi (nblocks x nlevels)
// give the positions in level_rows of the block's rows on each level.
// x_i = (b_i - sum_{j != i} T_ij x_j) / T_ii, entries in row order.
// ---------------------------------------------------------------------
template <typename TV, typename TX, bool PERM>
__device__ __forceinline__ void tri_row(int r, const int32_t* __restrict__ rp,
                                        const int32_t* __restrict__ ci,
                                        const int32_t* __restrict__ perm,
                                        const TV* __restrict__ vals, const TX* __restrict__ b,
                                        TX* __restrict__ x) {
  // entries 8 at a time: all column/value loads, then all x loads, then the
  // sum in entry order (two or three rounds of memory latency per batch
  // instead of a dependent chain per entry)
  constexpr int W = 8;
  TX s = 0, d = 0;
  const int e0 = rp[r], e1 = rp[r + 1];
  for (int eb = e0; eb < e1; eb += W) {
    int j[W];
    TX v[W], xv[W];
#pragma unroll
    for (int u = 0; u < W; ++u) {
      const bool ok = eb + u < e1;
      j[u] = ok ? ci[eb + u] : r;
      v[u] = ok ? (TX)(PERM ? vals[perm[eb + u]] : vals[eb + u]) : TX(0);
    }
#pragma unroll
    for (int u = 0; u < W; ++u) xv[u] = j[u] != r ? x[j[u]] : TX(0);
#pragma unroll
    for (int u = 0; u < W; ++u) {
      if (eb + u < e1) {
        if (j[u] == r) d = v[u];
        else s += v[u] * xv[u];
      }
    }
  }
  x[r] = (b[r] - s) / d;
}

// Two rows of one level per thread, their loads interleaved (the rows of a
// level are independent): each row's sum still runs in entry order, so the
// result is the one-row tri_row's.
template <typename TX, bool PERM>
__device__ __forceinline__ void tri_rows2(const int (&r)[2], const bool (&valid)[2],
                                          const int32_t* __restrict__ rp,
                                          const int32_t* __restrict__ ci,
                                          const int32_t* __restrict__ perm,
                                          const TX* __restrict__ vals, const TX* __restrict__ b,
                                          TX* __restrict__ x) {
  constexpr int W = 8;
  int e0[2], e1[2];
  TX s[2] = {TX(0), TX(0)}, d[2] = {TX(1), TX(1)};
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    e0[k] = valid[k] ? rp[r[k]] : 0;
    e1[k] = valid[k] ? rp[r[k] + 1] : 0;
  }
  const int nb = max((e1[0] - e0[0] + W - 1) / W, (e1[1] - e0[1] + W - 1) / W);
  for (int bb = 0; bb < nb; ++bb) {
    int j[2][W];
    TX v[2][W], xv[2][W];
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int u = 0; u < W; ++u) {
        const int e = e0[k] + bb * W + u;
        const bool ok = e < e1[k];
        j[k][u] = ok ? ci[e] : r[k];
        v[k][u] = ok ? (PERM ? vals[perm[e]] : vals[e]) : TX(0);
      }
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int u = 0; u < W; ++u) xv[k][u] = j[k][u] != r[k] ? x[j[k][u]] : TX(0);
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int u = 0; u < W; ++u) {
        if (e0[k] + bb * W + u < e1[k]) {
          if (j[k][u] == r[k]) d[k] = v[k][u];
          else s[k] += v[k][u] * xv[k][u];
        }
      }
  }
#pragma unroll
  for (int k = 0; k < 2; ++k)
    if (valid[k]) x[r[k]] = (b[r[k]] - s[k]) / d[k];
}

// A task is a block: its levels in order (ADJ: in reverse, over T^T with
// values through perm), a barrier between levels, two rows per thread per
// pass.  The block's level bounds are staged in LDS first.
constexpr int kLvLds = 1024;

template <typename T, bool ADJ>
__global__ __launch_bounds__(kTriThreads) void k_batch_tri(
    const BTask* __restrict__ tasks, int ntasks, unsigned* ctr, int nlevels,
    const int32_t* __restrict__ lv_lo, const int32_t* __restrict__ lv_hi,
    const int32_t* __restrict__ rows, const int32_t* __restrict__ rp,
    const int32_t* __restrict__ ci, const int32_t* __restrict__ perm, const T* __restrict__ vals,
    const T* __restrict__ b, T* __restrict__ x) {
  __shared__ int s_lo[kLvLds], s_hi[kLvLds];
  const bool staged = nlevels <= kLvLds;
  run_queue(tasks, ntasks, ctr, [&](const BTask& tk) {
    const long long base = (long long)tk.block * nlevels;
    if (staged) {
      for (int l = threadIdx.x; l < nlevels; l += kTriThreads) {
        s_lo[l] = lv_lo[base + l];
        s_hi[l] = lv_hi[base + l];
      }
      __syncthreads();
    }
    for (int s = 0; s < nlevels; ++s) {
      const int l = ADJ ? nlevels - 1 - s : s;
      const int lo = staged ? s_lo[l] : lv_lo[base + l];
      const int hi = staged ? s_hi[l] : lv_hi[base + l];
      if (hi <= lo) continue;  // uniform over the workgroup
      for (int q = lo + threadIdx.x; q < hi; q += 2 * kTriThreads) {
        const int q1 = q + kTriThreads;
        const bool valid[2] = {true, q1 < hi};
        const int r[2] = {rows[q], valid[1] ? rows[q1] : 0};
        tri_rows2<T, ADJ>(r, valid, rp, ci, perm, vals, b, x);
      }
      __syncthreads();
    }
  });
}

// gvals[(i,j)] = -w_i x_j on pat(T), row-wise over T with G lanes per row
// (the adjoint's value gradient, once w is final).
template <typename T, int G>
__global__ __launch_bounds__(kThreads) void k_tri_gvals_rows(int n, const int32_t* __restrict__ rp,
                                                            const int32_t* __restrict__ ci,
                                                            const T* __restrict__ w,
                                                            const T* __restrict__ x,
                                                            T* __restrict__ gv) {
  const int sub = threadIdx.x % G;
  for (long long i = ((long long)blockIdx.x * kThreads + threadIdx.x) / G; i < n;
       i += (long long)gridDim.x * (kThreads / G)) {
    const T wi = -w[i];
    const int e1 = rp[i + 1];
    for (int e = rp[i] + sub; e < e1; e += G) gv[e] = wi * x[ld_stream(&ci[e])];
  }
}

// Level-synchronous variant: ONE cooperative launch over the whole
// block-diagonal matrix.  Level l of the batch is the union of level l of
// every block; all resident workgroups share each level's rows (one row
// per thread, grid-stride), and a grid barrier separates levels.  With ADJ
// the levels run in reverse over T^T (values through perm) and, after a
// last barrier, gvals[(i,j)] = -w_i x_j is written row-wise over T.
template <typename T, bool ADJ>
__global__ __launch_bounds__(kThreads) void k_batch_tri_coop(
    int nlevels, const int32_t* __restrict__ level_ptr, const int32_t* __restrict__ rows,
    const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
    const int32_t* __restrict__ perm, const T* __restrict__ vals, const T* __restrict__ b,
    T* __restrict__ x, const T* __restrict__ xf, int n, const int32_t* __restrict__ rpA,
    const int32_t* __restrict__ ciA, T* __restrict__ gv) {
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int nth = gridDim.x * blockDim.x;
  for (int s = 0; s < nlevels; ++s) {
    const int l = ADJ ? nlevels - 1 - s : s;
    const int lo = level_ptr[l], hi = level_ptr[l + 1];
    for (int q = lo + tid; q < hi; q += nth) tri_row<T, T, ADJ>(rows[q], rp, ci, perm, vals, b, x);
    if (s + 1 < nlevels) grid.sync();  // uniform over the grid
  }
  if (ADJ && gv) {
    grid.sync();
    for (int i = tid; i < n; i += nth) {
      const T wi = x[i];
      for (int e = rpA[i]; e < rpA[i + 1]; ++e) gv[e] = -wi * xf[ciA[e]];
    }
  }
}

// IC(0) on the lower pattern (diagonal last in every row): for the
// entries (i, j) of row i in column order,
//   L_ij = (A_ij - sum_{k<j} L_ik L_jk) / L_jj,   L_ii = sqrt(A_ii - sum_{k<i} L_ik^2),
// the sums over the columns k stored in both rows.  Row i reads rows
// j < i, which sit on lower levels of the lower solve.  A non-positive
// pivot leaves NaN on the diagonal (and in every entry that reads it).
template <typename T>
__global__ __launch_bounds__(kTriThreads) void k_batch_ic0(
    const BTask* __restrict__ tasks, int ntasks, unsigned* ctr, int nlevels,
    const int32_t* __restrict__ lv_lo, const int32_t* __restrict__ lv_hi,
    const int32_t* __restrict__ rows, const int32_t* __restrict__ rp,
    const int32_t* __restrict__ ci, const T* __restrict__ a, T* __restrict__ l) {
  run_queue(tasks, ntasks, ctr, [&](const BTask& tk) {
    const long long base = (long long)tk.block * nlevels;
    for (int lev = 0; lev < nlevels; ++lev) {
      const int lo = lv_lo[base + lev], hi = lv_hi[base + lev];
      if (hi <= lo) continue;
      for (int q = lo + threadIdx.x; q < hi; q += kTriThreads) {
        const int i = rows[q];
        const int e0 = rp[i], e1 = rp[i + 1];
        for (int e = e0; e < e1; ++e) {
          const int j = ci[e];
          T s = 0;
          int p = e0, qq = rp[j];
          const int qe = rp[j + 1] - 1;  // row j without its diagonal
          while (p < e && qq < qe) {
            const int cp = ci[p], cq = ci[qq];
            if (cp == cq) {
              s += l[p] * l[qq];
              ++p;
              ++qq;
            } else if (cp < cq) {
              ++p;
            } else {
              ++qq;
            }
          }
          if (j == i) {
            const T d = a[e] - s;
            l[e] = d > T(0) ? sqrt(d) : T(NAN);
          } else {
            l[e] = (a[e] - s) / l[qe];
          }
        }
      }
      __syncthreads();
    }
  });
}

// Positions of each block's rows inside each level's slice of level_rows
// (rows ascend within a level, and a block's rows are one index range).
__global__ void k_block_levels(int nblocks, int nlevels, const int32_t* __restrict__ brp,
                               const int32_t* __restrict__ level_ptr,
                               const int32_t* __restrict__ rows, int32_t* __restrict__ lv_lo,
                               int32_t* __restrict__ lv_hi) {
  const long long total = (long long)nblocks * nlevels;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const int bk = (int)(idx / nlevels), l = (int)(idx % nlevels);
    const int a = level_ptr[l], z = level_ptr[l + 1];
    auto lower_bound = [&](int key) {
      int lo = a, hi = z;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (rows[mid] < key) lo = mid + 1;
        else hi = mid;
      }
      return lo;
    };
    lv_lo[idx] = lower_bound(brp[bk]);
    lv_hi[idx] = lower_bound(brp[bk + 1]);
  }
}

// ---------------------------------------------------------------------
// Plan construction: task t of block b is chunk c of nch; its rows are
// where the merge-path position r + rowptr[r] crosses c/nch of the block's
// cost (found by binary search; a single long row may leave a chunk empty).
// ---------------------------------------------------------------------
__global__ void k_task_rows(int ntasks, BTask* __restrict__ tasks, const int32_t* __restrict__ chunk,
                            const int32_t* __restrict__ nchunks, const int32_t* __restrict__ brp,
                            const int32_t* __restrict__ rp) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < ntasks; t += gridDim.x * blockDim.x) {
    const int b = tasks[t].block, c = chunk[t], nc = nchunks[t];
    const int R0 = brp[b], R1 = brp[b + 1];
    const long long k0 = (long long)R0 + rp[R0], k1 = (long long)R1 + rp[R1];
    auto find = [&](int cc) {
      if (cc <= 0) return R0;
      if (cc >= nc) return R1;
      const long long target = k0 + (k1 - k0) * cc / nc;
      int lo = R0, hi = R1;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((long long)mid + rp[mid] < target) lo = mid + 1;
        else hi = mid;
      }
      return lo;
    };
    tasks[t].r0 = find(c);
    tasks[t].r1 = find(c + 1);
  }
}

__global__ void k_gather_rp(int nb, const int32_t* __restrict__ brp, const int32_t* __restrict__ rp,
                            int32_t* __restrict__ out) {
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b <= nb; b += gridDim.x * blockDim.x)
    out[b] = rp[brp[b]];
}

// Workspace layout of a plan (see csr_batch_plan_workspace).
struct PlanWs {
  BTask* tasks;
  int32_t* chunk;
  int32_t* nchunks;
  int32_t* brp;
  int32_t* ends;
  unsigned* ctr;
};

// Path items per task: `budget` for row-split tasks; a quarter of it for
// merge tasks, within [256, kMergeRowCap] so a merge task's row ends fit
// the LDS stage (a chunk of the merge path holds at most as many rows as
// path items).
int merge_budget(int budget) {
  const int m = budget / 4;
  return m < 256 ? 256 : (m > kMergeRowCap ? kMergeRowCap : m);
}

long long max_tasks(long long nrows, long long nnz, int nblocks, int budget) {
  if (budget <= 0) return nblocks;
  const int mb = merge_budget(budget);
  const long long unit = budget < mb ? budget : mb;
  return (nrows + nnz) / unit + nblocks + 1;
}

PlanWs carve_plan(Carver& c, long long ntasks_max, int nblocks) {
  PlanWs w;
  w.tasks = c.take<BTask>((size_t)ntasks_max);
  w.chunk = c.take<int32_t>((size_t)ntasks_max);
  w.nchunks = c.take<int32_t>((size_t)ntasks_max);
  w.brp = c.take<int32_t>((size_t)nblocks + 1);
  w.ends = c.take<int32_t>((size_t)nblocks + 1);
  w.ctr = c.take<unsigned>(kCtrWords);
  return w;
}

// Workgroups a persistent launch keeps: as many as fit on the chip at once
// (the occupancy of this kernel at this block size), at most one per task.
template <typename K>
int slots_for(const csrad_batch_plan* plan, K kernel, int threads) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = kSlotsPerCu;
  const long long s = (long long)plan->cus * per_cu;
  return (int)(plan->ntasks < s ? plan->ntasks : s);
}

int check_plan_for(const csrad_batch_plan* plan, int rows) {
  if (!plan || !plan->tasks || !plan->counters) return CSRAD_EINVAL;
  if (plan->nrows != rows || plan->ntasks < 0 || plan->cus <= 0) return CSRAD_EINVAL;
  return CSRAD_OK;
}

int pick_kind(int variant, long long rows, long long nnz) {
  if (variant > 0) return variant;
  // automatic: short rows staged in LDS, else lanes per row from the mean
  const double mean = rows > 0 ? (double)nnz / rows : 0.0;
  if (mean <= 9.0) return kKindStaged;
  int g = 1, kind = 1;
  while (g < 64 && g < mean) {
    g <<= 1;
    ++kind;
  }
  return kind;
}

template <typename T>
int batch_spmm_fwd_t(const csrad_csr* A, const csrad_batch_plan* plan, int k, const T* B,
                     long long ldb, T* C, long long ldc, hipStream_t s) {
  if (plan->ntasks == 0) return CSRAD_OK;
  constexpr int VW = 16 / sizeof(T);
  const BTask* tk = static_cast<const BTask*>(plan->tasks);
  unsigned* ctr = static_cast<unsigned*>(plan->counters);
  const T* v = static_cast<const T*>(A->vals);
  hipLaunchKernelGGL((k_batch_spmm<T, VW>), dim3(slots_for(plan, k_batch_spmm<T, VW>, kThreads)),
                     dim3(kThreads), 0, s, tk,
                     plan->ntasks, ctr, k, A->rowptr, A->colind, v, B, ldb, C, ldc);
  return launch_status();
}

template <typename T>
int batch_spmm_bwd_t(const csrad_csr* A, const csrad_csr* At, const int32_t* perm,
                     const csrad_batch_plan* plan, int k, const T* B, long long ldb, const T* G,
                     long long ldg, T* gB, long long ldgb, T* gv, hipStream_t s) {
  if (plan->ntasks == 0) return CSRAD_OK;
  constexpr int VW = 16 / sizeof(T);
  const BTask* tk = static_cast<const BTask*>(plan->tasks);
  unsigned* ctr = static_cast<unsigned*>(plan->counters);
  const T* v = static_cast<const T*>(A->vals);
  const dim3 grid(slots_for(plan, k_batch_spmm_bwd<T, VW, true, true>, kThreads));
  if (gB && gv)
    hipLaunchKernelGGL((k_batch_spmm_bwd<T, VW, true, true>), grid, dim3(kThreads), 0, s, tk,
                       plan->ntasks, ctr, k, At->rowptr, At->colind, perm, v, B, ldb, G, ldg, gB,
                       ldgb, gv);
  else if (gB)
    hipLaunchKernelGGL((k_batch_spmm_bwd<T, VW, true, false>), grid, dim3(kThreads), 0, s, tk,
                       plan->ntasks, ctr, k, At->rowptr, At->colind, perm, v, B, ldb, G, ldg, gB,
                       ldgb, gv);
  else
    hipLaunchKernelGGL((k_batch_spmm_bwd<T, VW, false, true>), grid, dim3(kThreads), 0, s, tk,
                       plan->ntasks, ctr, k, At->rowptr, At->colind, perm, v, B, ldb, G, ldg, gB,
                       ldgb, gv);
  return launch_status();
}

bool aligned16(const void* p, long long ld, int elem) {
  return (reinterpret_cast<uintptr_t>(p) % 16) == 0 && (ld * elem) % 16 == 0;
}

}  // namespace
}  // namespace csrad

using namespace csrad;

extern "C" int csr_batch_plan_workspace(const csrad_csr* A, int32_t nblocks, int32_t budget,
                                        size_t* bytes) {
  CSRAD_TRY(check_csr(A, false));
  if (!bytes || nblocks < 0) return CSRAD_EINVAL;
  Carver c(nullptr, 0);
  carve_plan(c, max_tasks(A->nrows, A->nnz, nblocks, budget), nblocks);
  *bytes = c.off;
  return CSRAD_OK;
}

extern "C" int csr_batch_plan_build(const csrad_csr* A, int32_t nblocks,
                                    const int32_t* block_rowptr_host, const int32_t* variant_host,
                                    int32_t budget, void* work, size_t work_bytes,
                                    csrad_batch_plan* plan, void* stream) {
  CSRAD_TRY(check_csr(A, false));
  if (!plan || nblocks < 0 || (nblocks > 0 && !block_rowptr_host)) return CSRAD_EINVAL;
  if (nblocks > 0 && (block_rowptr_host[0] != 0 || block_rowptr_host[nblocks] != A->nrows))
    return CSRAD_EINVAL;
  for (int b = 0; b < nblocks; ++b)
    if (block_rowptr_host[b + 1] < block_rowptr_host[b]) return CSRAD_EINVAL;
  if (variant_host)
    for (int b = 0; b < nblocks; ++b)
      if (variant_host[b] < -1 || variant_host[b] > kKindStaged) return CSRAD_EINVAL;
  const long long tmax = max_tasks(A->nrows, A->nnz, nblocks, budget);
  Carver c(work, work_bytes);
  PlanWs w = carve_plan(c, tmax, nblocks);
  if (!work || !c.ok) return CSRAD_EWORKSPACE;
  hipStream_t s = as_stream(stream);
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return CSRAD_EHIP;
  // block boundaries on the device, entry offsets of the boundaries back
  std::vector<int32_t> ends(nblocks + 1, 0);
  if (nblocks > 0) {
    if (hipMemcpyAsync(w.brp, block_rowptr_host, sizeof(int32_t) * (nblocks + 1),
                       hipMemcpyHostToDevice, s) != hipSuccess)
      return CSRAD_EHIP;
    hipLaunchKernelGGL(k_gather_rp, dim3((nblocks + 256) / 256), dim3(256), 0, s, nblocks, w.brp,
                       A->rowptr, w.ends);
    CSRAD_TRY(launch_status());
    if (hipMemcpyAsync(ends.data(), w.ends, sizeof(int32_t) * (nblocks + 1),
                       hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return CSRAD_EHIP;
  }
  // chunks of about `budget` path items (merge tasks: merge_budget(budget))
  std::vector<int> order(nblocks);
  std::vector<long long> cost(nblocks);
  for (int b = 0; b < nblocks; ++b) {
    order[b] = b;
    cost[b] = (long long)(block_rowptr_host[b + 1] - block_rowptr_host[b]) + (ends[b + 1] - ends[b]);
  }
  // Whole-block tasks (budget <= 0): largest blocks first, from one queue,
  // so the long ones start early.  Chunked tasks are about equal in cost:
  // they stay in row order, dealt from one queue per XCD (neighbouring
  // tasks share blocks, so each XCD's L2 holds the dense rows of a few
  // blocks at a time).
  if (budget <= 0)
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return cost[a] > cost[b]; });
  std::vector<BTask> tasks;
  std::vector<int32_t> chunk, nch;
  for (int b : order) {
    const int rows = block_rowptr_host[b + 1] - block_rowptr_host[b];
    const long long nnz = ends[b + 1] - ends[b];
    const int var = variant_host ? variant_host[b] : 0;
    if (var < 0 || rows == 0) continue;  // excluded or empty block
    const int kind = budget <= 0 ? 0 : pick_kind(var, rows, nnz);
    long long n = 1;
    if (budget > 0) {
      const long long bud = kind == kKindMerge ? merge_budget(budget) : budget;
      n = (cost[b] + bud - 1) / bud;
      if (n < 1) n = 1;
    }
    for (long long cc = 0; cc < n; ++cc) {
      tasks.push_back(BTask{0, 0, kind, b});
      chunk.push_back((int32_t)cc);
      nch.push_back((int32_t)n);
    }
  }
  if ((long long)tasks.size() > tmax) return CSRAD_EWORKSPACE;
  const int nt = (int)tasks.size();
  if (nt > 0) {
    if (hipMemcpyAsync(w.tasks, tasks.data(), sizeof(BTask) * nt, hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        hipMemcpyAsync(w.chunk, chunk.data(), sizeof(int32_t) * nt, hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        hipMemcpyAsync(w.nchunks, nch.data(), sizeof(int32_t) * nt, hipMemcpyHostToDevice, s) !=
            hipSuccess)
      return CSRAD_EHIP;
    hipLaunchKernelGGL(k_task_rows, dim3((nt + 255) / 256), dim3(256), 0, s, nt, w.tasks, w.chunk,
                       w.nchunks, w.brp, A->rowptr);
    CSRAD_TRY(launch_status());
  }
  CSRAD_TRY(fill_bytes_zero(w.ctr, kCtrWords * sizeof(unsigned), s));
  const unsigned nq = budget > 0 ? (unsigned)kQueues : 1u;
  if (hipMemcpyAsync(w.ctr + kNqSlot, &nq, sizeof(unsigned), hipMemcpyHostToDevice, s) !=
      hipSuccess)
    return CSRAD_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return CSRAD_EHIP;  // host vectors die here
  // a merge task must fit the LDS stage: check on the host
  if (nt > 0) {
    std::vector<BTask> got(nt);
    if (hipMemcpy(got.data(), w.tasks, sizeof(BTask) * nt, hipMemcpyDeviceToHost) != hipSuccess)
      return CSRAD_EHIP;
    for (const BTask& t : got)
      if (t.kind == kKindMerge && t.r1 - t.r0 > kMergeRowCap) return CSRAD_EINVAL;
  }
  plan->nrows = A->nrows;
  plan->nblocks = nblocks;
  plan->ntasks = nt;
  plan->cus = cus;
  plan->tasks = w.tasks;
  plan->counters = w.ctr;
  plan->block_rowptr = w.brp;
  return CSRAD_OK;
}

extern "C" int csr_batch_spmv_fwd(const csrad_csr* A, const csrad_batch_plan* plan, const void* x,
                                  void* y, void* stream) {
  CSRAD_TRY(check_csr(A, true));
  CSRAD_TRY(check_plan_for(plan, A->nrows));
  if ((A->ncols > 0 && !x) || (A->nrows > 0 && !y)) return CSRAD_EINVAL;
  if (plan->ntasks == 0) return CSRAD_OK;
  hipStream_t s = as_stream(stream);
  const BTask* tk = static_cast<const BTask*>(plan->tasks);
  unsigned* ctr = static_cast<unsigned*>(plan->counters);
  const dim3 grid(A->dtype == CSRAD_F32 ? slots_for(plan, k_batch_spmv<float>, kThreads)
                                        : slots_for(plan, k_batch_spmv<double>, kThreads));
  if (A->dtype == CSRAD_F32)
    hipLaunchKernelGGL((k_batch_spmv<float>), grid, dim3(kThreads), 0, s, tk, plan->ntasks, ctr,
                       A->rowptr, A->colind, static_cast<const float*>(A->vals),
                       static_cast<const float*>(x), static_cast<float*>(y));
  else
    hipLaunchKernelGGL((k_batch_spmv<double>), grid, dim3(kThreads), 0, s, tk, plan->ntasks, ctr,
                       A->rowptr, A->colind, static_cast<const double*>(A->vals),
                       static_cast<const double*>(x), static_cast<double*>(y));
  return launch_status();
}

extern "C" int csr_batch_spmv_bwd(const csrad_csr* A, const csrad_csr* At, const int32_t* perm,
                                  const csrad_batch_plan* planT, const void* x, const void* gy,
                                  void* gx, void* gvals, void* stream) {
  CSRAD_TRY(check_csr(A, gx != nullptr));
  if (!gx && !gvals) return CSRAD_OK;
  if (!At) return CSRAD_EINVAL;
  CSRAD_TRY(check_csr(At, false));
  if (At->nrows != A->ncols || At->ncols != A->nrows || At->nnz != A->nnz) return CSRAD_EINVAL;
  CSRAD_TRY(check_plan_for(planT, At->nrows));
  if ((A->nnz > 0 && !perm) || (A->nrows > 0 && !gy) || (gvals && A->ncols > 0 && !x))
    return CSRAD_EINVAL;
  if (planT->ntasks == 0) return CSRAD_OK;
  hipStream_t s = as_stream(stream);
  const BTask* tk = static_cast<const BTask*>(planT->tasks);
  unsigned* ctr = static_cast<unsigned*>(planT->counters);
  const dim3 grid(A->dtype == CSRAD_F32
                      ? slots_for(planT, k_batch_spmv_bwd<float, true, true>, kThreads)
                      : slots_for(planT, k_batch_spmv_bwd<double, true, true>, kThreads));
#define CSRAD_BATCH_SPMVB(T)                                                                    \
  {                                                                                             \
    const T* v = static_cast<const T*>(A->vals);                                                \
    const T* xx = static_cast<const T*>(x);                                                     \
    const T* gg = static_cast<const T*>(gy);                                                    \
    T* gxx = static_cast<T*>(gx);                                                               \
    T* gvv = static_cast<T*>(gvals);                                                            \
    if (gx && gvals)                                                                            \
      hipLaunchKernelGGL((k_batch_spmv_bwd<T, true, true>), grid, dim3(kThreads), 0, s, tk,     \
                         planT->ntasks, ctr, At->rowptr, At->colind, perm, v, xx, gg, gxx, gvv); \
    else if (gx)                                                                                \
      hipLaunchKernelGGL((k_batch_spmv_bwd<T, true, false>), grid, dim3(kThreads), 0, s, tk,    \
                         planT->ntasks, ctr, At->rowptr, At->colind, perm, v, xx, gg, gxx, gvv); \
    else                                                                                        \
      hipLaunchKernelGGL((k_batch_spmv_bwd<T, false, true>), grid, dim3(kThreads), 0, s, tk,    \
                         planT->ntasks, ctr, At->rowptr, At->colind, perm, v, xx, gg, gxx, gvv); \
  }
  if (A->dtype == CSRAD_F32) CSRAD_BATCH_SPMVB(float) else CSRAD_BATCH_SPMVB(double)
#undef CSRAD_BATCH_SPMVB
  return launch_status();
}

extern "C" int csr_batch_spmm_fwd(const csrad_csr* A, const csrad_batch_plan* plan, int32_t k,
                                  const void* B, int64_t ldb, void* C, int64_t ldc, void* stream) {
  CSRAD_TRY(check_csr(A, true));
  CSRAD_TRY(check_plan_for(plan, A->nrows));
  if (k <= 0 || ldb < k || ldc < k) return CSRAD_EINVAL;
  if ((A->ncols > 0 && !B) || (A->nrows > 0 && !C)) return CSRAD_EINVAL;
  const int es = (int)dtype_size(A->dtype);
  if (k % (16 / es) != 0 || !aligned16(B, ldb, es) || !aligned16(C, ldc, es)) return CSRAD_EINVAL;
  hipStream_t s = as_stream(stream);
  if (A->dtype == CSRAD_F32)
    return batch_spmm_fwd_t<float>(A, plan, k, static_cast<const float*>(B), ldb,
                                   static_cast<float*>(C), ldc, s);
  return batch_spmm_fwd_t<double>(A, plan, k, static_cast<const double*>(B), ldb,
                                  static_cast<double*>(C), ldc, s);
}

extern "C" int csr_batch_spmm_bwd(const csrad_csr* A, const csrad_csr* At, const int32_t* perm,
                                  const csrad_batch_plan* planT, int32_t k, const void* B,
                                  int64_t ldb, const void* gC, int64_t ldgc, void* gB,
                                  int64_t ldgb, void* gvals, void* stream) {
  CSRAD_TRY(check_csr(A, gB != nullptr));
  if (!gB && !gvals) return CSRAD_OK;
  if (!At) return CSRAD_EINVAL;
  CSRAD_TRY(check_csr(At, false));
  if (At->nrows != A->ncols || At->ncols != A->nrows || At->nnz != A->nnz) return CSRAD_EINVAL;
  CSRAD_TRY(check_plan_for(planT, At->nrows));
  if (k <= 0 || ldgc < k || (A->nnz > 0 && !perm) || (A->nrows > 0 && !gC)) return CSRAD_EINVAL;
  if (gvals && (ldb < k || (A->ncols > 0 && !B))) return CSRAD_EINVAL;
  if (gB && ldgb < k) return CSRAD_EINVAL;
  const int es = (int)dtype_size(A->dtype);
  if (k % (16 / es) != 0 || !aligned16(gC, ldgc, es) || (gB && !aligned16(gB, ldgb, es)) ||
      (gvals && !aligned16(B, ldb, es)))
    return CSRAD_EINVAL;
  hipStream_t s = as_stream(stream);
  if (A->dtype == CSRAD_F32)
    return batch_spmm_bwd_t<float>(A, At, perm, planT, k, static_cast<const float*>(B), ldb,
                                   static_cast<const float*>(gC), ldgc, static_cast<float*>(gB),
                                   ldgb, static_cast<float*>(gvals), s);
  return batch_spmm_bwd_t<double>(A, At, perm, planT, k, static_cast<const double*>(B), ldb,
                                  static_cast<const double*>(gC), ldgc, static_cast<double*>(gB),
                                  ldgb, static_cast<double*>(gvals), s);
}

extern "C" int csr_batch_levels_workspace(int32_t nblocks, int32_t nlevels, size_t* bytes) {
  if (!bytes || nblocks < 0 || nlevels < 0) return CSRAD_EINVAL;
  Carver c(nullptr, 0);
  c.take<int32_t>((size_t)nblocks * nlevels);
  c.take<int32_t>((size_t)nblocks * nlevels);
  *bytes = c.off;
  return CSRAD_OK;
}

extern "C" int csr_batch_levels(const csrad_batch_plan* plan, int32_t nlevels,
                                const int32_t* level_ptr, const int32_t* level_rows, void* work,
                                size_t work_bytes, void* stream) {
  if (!plan || !plan->block_rowptr || nlevels < 0 || (nlevels > 0 && (!level_ptr || !level_rows)))
    return CSRAD_EINVAL;
  Carver c(work, work_bytes);
  int32_t* lo = c.take<int32_t>((size_t)plan->nblocks * nlevels);
  int32_t* hi = c.take<int32_t>((size_t)plan->nblocks * nlevels);
  if (!work || !c.ok) return CSRAD_EWORKSPACE;
  const long long total = (long long)plan->nblocks * nlevels;
  if (total == 0) return CSRAD_OK;
  long long blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_block_levels, dim3((unsigned)blocks), dim3(256), 0, as_stream(stream),
                     plan->nblocks, nlevels, plan->block_rowptr, level_ptr, level_rows, lo, hi);
  return launch_status();
}

namespace {
int batch_tri_args(const csrad_csr* T, const csrad_batch_plan* plan, int nlevels,
                   const int32_t* level_rows, const void* lv, size_t lv_bytes) {
  CSRAD_TRY(check_csr(T, true));
  if (T->nrows != T->ncols) return CSRAD_EINVAL;
  CSRAD_TRY(check_plan_for(plan, T->nrows));
  if (nlevels < 0 || (T->nrows > 0 && (!level_rows || !lv))) return CSRAD_EINVAL;
  size_t need = 0;
  CSRAD_TRY(csr_batch_levels_workspace(plan->nblocks, nlevels, &need));
  if (lv_bytes < need) return CSRAD_EWORKSPACE;
  return CSRAD_OK;
}
}  // namespace

extern "C" int csr_batch_trisolve_fwd(const csrad_csr* T, const csrad_batch_plan* plan,
                                      int32_t nlevels, const int32_t* level_rows,
                                      const void* levels_work, size_t levels_bytes,
                                      const void* b, void* x, void* stream) {
  CSRAD_TRY(batch_tri_args(T, plan, nlevels, level_rows, levels_work, levels_bytes));
  if (T->nrows > 0 && (!b || !x)) return CSRAD_EINVAL;
  if (plan->ntasks == 0 || nlevels == 0) return CSRAD_OK;
  Carver c(const_cast<void*>(levels_work), levels_bytes);
  const int32_t* lo = c.take<int32_t>((size_t)plan->nblocks * nlevels);
  const int32_t* hi = c.take<int32_t>((size_t)plan->nblocks * nlevels);
  hipStream_t s = as_stream(stream);
  const BTask* tk = static_cast<const BTask*>(plan->tasks);
  unsigned* ctr = static_cast<unsigned*>(plan->counters);
  const dim3 grid(T->dtype == CSRAD_F32
                      ? slots_for(plan, k_batch_tri<float, false>, kTriThreads)
                      : slots_for(plan, k_batch_tri<double, false>, kTriThreads));
  if (T->dtype == CSRAD_F32)
    hipLaunchKernelGGL((k_batch_tri<float, false>), grid, dim3(kTriThreads), 0, s, tk, plan->ntasks,
                       ctr, nlevels, lo, hi, level_rows, T->rowptr, T->colind, nullptr,
                       static_cast<const float*>(T->vals), static_cast<const float*>(b),
                       static_cast<float*>(x));
  else
    hipLaunchKernelGGL((k_batch_tri<double, false>), grid, dim3(kTriThreads), 0, s, tk, plan->ntasks,
                       ctr, nlevels, lo, hi, level_rows, T->rowptr, T->colind, nullptr,
                       static_cast<const double*>(T->vals), static_cast<const double*>(b),
                       static_cast<double*>(x));
  return launch_status();
}

extern "C" int csr_batch_trisolve_bwd(const csrad_csr* T, const csrad_csr* Tt, const int32_t* perm,
                                      const csrad_batch_plan* plan, int32_t nlevels,
                                      const int32_t* level_rows, const void* levels_work,
                                      size_t levels_bytes, const void* x, const void* gx,
                                      void* gb, void* gvals, void* stream) {
  CSRAD_TRY(batch_tri_args(T, plan, nlevels, level_rows, levels_work, levels_bytes));
  if (!Tt) return CSRAD_EINVAL;
  CSRAD_TRY(check_csr(Tt, false));
  if (Tt->nrows != T->nrows || Tt->nnz != T->nnz) return CSRAD_EINVAL;
  if (T->nrows > 0 && (!gx || !gb || (gvals && !x))) return CSRAD_EINVAL;
  if (T->nnz > 0 && !perm) return CSRAD_EINVAL;
  if (plan->ntasks == 0 || nlevels == 0) return CSRAD_OK;
  Carver c(const_cast<void*>(levels_work), levels_bytes);
  const int32_t* lo = c.take<int32_t>((size_t)plan->nblocks * nlevels);
  const int32_t* hi = c.take<int32_t>((size_t)plan->nblocks * nlevels);
  hipStream_t s = as_stream(stream);
  const BTask* tk = static_cast<const BTask*>(plan->tasks);
  unsigned* ctr = static_cast<unsigned*>(plan->counters);
  const dim3 grid(T->dtype == CSRAD_F32
                      ? slots_for(plan, k_batch_tri<float, true>, kTriThreads)
                      : slots_for(plan, k_batch_tri<double, true>, kTriThreads));
  if (T->dtype == CSRAD_F32)
    hipLaunchKernelGGL((k_batch_tri<float, true>), grid, dim3(kTriThreads), 0, s, tk, plan->ntasks,
                       ctr, nlevels, lo, hi, level_rows, Tt->rowptr, Tt->colind, perm,
                       static_cast<const float*>(T->vals), static_cast<const float*>(gx),
                       static_cast<float*>(gb));
  else
    hipLaunchKernelGGL((k_batch_tri<double, true>), grid, dim3(kTriThreads), 0, s, tk, plan->ntasks,
                       ctr, nlevels, lo, hi, level_rows, Tt->rowptr, Tt->colind, perm,
                       static_cast<const double*>(T->vals), static_cast<const double*>(gx),
                       static_cast<double*>(gb));
  CSRAD_TRY(launch_status());
  if (gvals) {
    const int n = T->nrows;
    const double mean = n > 0 ? (double)T->nnz / n : 0.0;
    const unsigned g = (unsigned)std::min<long long>(((long long)n * 8 + kThreads - 1) / kThreads,
                                                     65536);
    if (mean > 4.0) {
      if (T->dtype == CSRAD_F32)
        hipLaunchKernelGGL((k_tri_gvals_rows<float, 8>), dim3(g), dim3(kThreads), 0, s, n,
                           T->rowptr, T->colind, static_cast<const float*>(gb),
                           static_cast<const float*>(x), static_cast<float*>(gvals));
      else
        hipLaunchKernelGGL((k_tri_gvals_rows<double, 8>), dim3(g), dim3(kThreads), 0, s, n,
                           T->rowptr, T->colind, static_cast<const double*>(gb),
                           static_cast<const double*>(x), static_cast<double*>(gvals));
    } else {
      if (T->dtype == CSRAD_F32)
        hipLaunchKernelGGL((k_tri_gvals_rows<float, 4>), dim3(g), dim3(kThreads), 0, s, n,
                           T->rowptr, T->colind, static_cast<const float*>(gb),
                           static_cast<const float*>(x), static_cast<float*>(gvals));
      else
        hipLaunchKernelGGL((k_tri_gvals_rows<double, 4>), dim3(g), dim3(kThreads), 0, s, n,
                           T->rowptr, T->colind, static_cast<const double*>(gb),
                           static_cast<const double*>(x), static_cast<double*>(gvals));
    }
  }
  return launch_status();
}

extern "C" int csr_batch_ic0(const csrad_csr* Alow, const csrad_batch_plan* plan, int32_t nlevels,
                             const int32_t* level_rows, const void* levels_work,
                             size_t levels_bytes, void* Lvals, void* stream) {
  CSRAD_TRY(batch_tri_args(Alow, plan, nlevels, level_rows, levels_work, levels_bytes));
  if (Alow->nnz > 0 && !Lvals) return CSRAD_EINVAL;
  if (plan->ntasks == 0 || nlevels == 0) return CSRAD_OK;
  Carver c(const_cast<void*>(levels_work), levels_bytes);
  const int32_t* lo = c.take<int32_t>((size_t)plan->nblocks * nlevels);
  const int32_t* hi = c.take<int32_t>((size_t)plan->nblocks * nlevels);
  hipStream_t s = as_stream(stream);
  const BTask* tk = static_cast<const BTask*>(plan->tasks);
  unsigned* ctr = static_cast<unsigned*>(plan->counters);
  const dim3 grid(Alow->dtype == CSRAD_F32 ? slots_for(plan, k_batch_ic0<float>, kTriThreads)
                                           : slots_for(plan, k_batch_ic0<double>, kTriThreads));
  if (Alow->dtype == CSRAD_F32)
    hipLaunchKernelGGL((k_batch_ic0<float>), grid, dim3(kTriThreads), 0, s, tk, plan->ntasks, ctr,
                       nlevels, lo, hi, level_rows, Alow->rowptr, Alow->colind,
                       static_cast<const float*>(Alow->vals), static_cast<float*>(Lvals));
  else
    hipLaunchKernelGGL((k_batch_ic0<double>), grid, dim3(kTriThreads), 0, s, tk, plan->ntasks, ctr,
                       nlevels, lo, hi, level_rows, Alow->rowptr, Alow->colind,
                       static_cast<const double*>(Alow->vals), static_cast<double*>(Lvals));
  return launch_status();
}

extern "C" int csr_batch_sddmv(const csrad_csr* A, const csrad_batch_plan* plan, const void* x,
                               const void* gy, void* gvals, void* stream) {
  CSRAD_TRY(check_csr(A, false));
  CSRAD_TRY(check_plan_for(plan, A->nrows));
  if (A->nnz > 0 && (!gvals || !x || !gy)) return CSRAD_EINVAL;
  if (plan->ntasks == 0 || A->nnz == 0) return CSRAD_OK;
  hipStream_t s = as_stream(stream);
  const BTask* tk = static_cast<const BTask*>(plan->tasks);
  unsigned* ctr = static_cast<unsigned*>(plan->counters);
  if (A->dtype == CSRAD_F32)
    hipLaunchKernelGGL((k_batch_sddmv<float>), dim3(slots_for(plan, k_batch_sddmv<float>, kThreads)),
                       dim3(kThreads), 0, s, tk, plan->ntasks, ctr, A->rowptr, A->colind,
                       static_cast<const float*>(x), static_cast<const float*>(gy),
                       static_cast<float*>(gvals));
  else
    hipLaunchKernelGGL((k_batch_sddmv<double>),
                       dim3(slots_for(plan, k_batch_sddmv<double>, kThreads)), dim3(kThreads), 0,
                       s, tk, plan->ntasks, ctr, A->rowptr, A->colind,
                       static_cast<const double*>(x), static_cast<const double*>(gy),
                       static_cast<double*>(gvals));
  return launch_status();
}

extern "C" int csr_batch_sddmm(const csrad_csr* A, const csrad_batch_plan* plan, int32_t k,
                               const void* B, int64_t ldb, const void* gC, int64_t ldgc,
                               void* gvals, void* stream) {
  CSRAD_TRY(check_csr(A, false));
  CSRAD_TRY(check_plan_for(plan, A->nrows));
  if (k <= 0 || ldb < k || ldgc < k) return CSRAD_EINVAL;
  if (A->nnz > 0 && (!gvals || !B || !gC)) return CSRAD_EINVAL;
  const int es = (int)dtype_size(A->dtype);
  if (k % (16 / es) != 0 || !aligned16(B, ldb, es) || !aligned16(gC, ldgc, es))
    return CSRAD_EINVAL;
  if (plan->ntasks == 0 || A->nnz == 0) return CSRAD_OK;
  hipStream_t s = as_stream(stream);
  const BTask* tk = static_cast<const BTask*>(plan->tasks);
  unsigned* ctr = static_cast<unsigned*>(plan->counters);
  if (A->dtype == CSRAD_F32)
    hipLaunchKernelGGL((k_batch_sddmm<float, 4>),
                       dim3(slots_for(plan, k_batch_sddmm<float, 4>, kThreads)), dim3(kThreads),
                       0, s, tk, plan->ntasks, ctr, k, A->rowptr, A->colind,
                       static_cast<const float*>(B), ldb, static_cast<const float*>(gC), ldgc,
                       static_cast<float*>(gvals));
  else
    hipLaunchKernelGGL((k_batch_sddmm<double, 2>),
                       dim3(slots_for(plan, k_batch_sddmm<double, 2>, kThreads)), dim3(kThreads),
                       0, s, tk, plan->ntasks, ctr, k, A->rowptr, A->colind,
                       static_cast<const double*>(B), ldb, static_cast<const double*>(gC), ldgc,
                       static_cast<double*>(gvals));
  return launch_status();
}

namespace {
// Cooperative launch of k_batch_tri_coop: every workgroup resident at once
// (as many as the occupancy allows on every CU); the runtime refuses a grid
// that cannot be co-resident, and the call then returns CSRAD_EHIP.
template <typename T, bool ADJ>
int tri_coop_launch(int nlevels, const int32_t* level_ptr, const int32_t* rows,
                    const int32_t* rp, const int32_t* ci, const int32_t* perm, const T* vals,
                    const T* b, T* x, const T* xf, int n, const int32_t* rpA, const int32_t* ciA,
                    T* gv, hipStream_t s) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_tri_coop<T, ADJ>, kThreads,
                                                   0) != hipSuccess ||
      per_cu < 1)
    return CSRAD_EHIP;
  long long want = ((long long)n + kThreads - 1) / kThreads;
  const long long cap = (long long)cus * per_cu;
  if (want > cap) want = cap;
  if (want < 1) want = 1;
  void* args[] = {&nlevels, &level_ptr, &rows, &rp, &ci, &perm, &vals, &b, &x, &xf, &n, &rpA,
                  &ciA, &gv};
  if (hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_batch_tri_coop<T, ADJ>),
                                 dim3((unsigned)want), dim3(kThreads), args, 0, s) != hipSuccess)
    return CSRAD_EHIP;
  return launch_status();
}
}  // namespace

extern "C" int csr_batch_trisolve_levels_fwd(const csrad_csr* T, int32_t nlevels,
                                             const int32_t* level_ptr, const int32_t* level_rows,
                                             const void* b, void* x, void* stream) {
  CSRAD_TRY(check_csr(T, true));
  if (T->nrows != T->ncols || nlevels < 0) return CSRAD_EINVAL;
  if (T->nrows == 0 || nlevels == 0) return CSRAD_OK;
  if (!level_ptr || !level_rows || !b || !x) return CSRAD_EINVAL;
  hipStream_t s = as_stream(stream);
  if (T->dtype == CSRAD_F32)
    return tri_coop_launch<float, false>(nlevels, level_ptr, level_rows, T->rowptr, T->colind,
                                         nullptr, static_cast<const float*>(T->vals),
                                         static_cast<const float*>(b), static_cast<float*>(x),
                                         nullptr, T->nrows, nullptr, nullptr, nullptr, s);
  return tri_coop_launch<double, false>(nlevels, level_ptr, level_rows, T->rowptr, T->colind,
                                        nullptr, static_cast<const double*>(T->vals),
                                        static_cast<const double*>(b), static_cast<double*>(x),
                                        nullptr, T->nrows, nullptr, nullptr, nullptr, s);
}

extern "C" int csr_batch_trisolve_levels_bwd(const csrad_csr* T, const csrad_csr* Tt,
                                             const int32_t* perm, int32_t nlevels,
                                             const int32_t* level_ptr, const int32_t* level_rows,
                                             const void* x, const void* gx, void* gb, void* gvals,
                                             void* stream) {
  CSRAD_TRY(check_csr(T, true));
  if (!Tt) return CSRAD_EINVAL;
  CSRAD_TRY(check_csr(Tt, false));
  if (T->nrows != T->ncols || Tt->nrows != T->nrows || Tt->nnz != T->nnz || nlevels < 0)
    return CSRAD_EINVAL;
  if (T->nrows == 0 || nlevels == 0) return CSRAD_OK;
  if (!level_ptr || !level_rows || !gx || !gb || (gvals && !x) || (T->nnz > 0 && !perm))
    return CSRAD_EINVAL;
  hipStream_t s = as_stream(stream);
  if (T->dtype == CSRAD_F32)
    return tri_coop_launch<float, true>(nlevels, level_ptr, level_rows, Tt->rowptr, Tt->colind,
                                        perm, static_cast<const float*>(T->vals),
                                        static_cast<const float*>(gx), static_cast<float*>(gb),
                                        static_cast<const float*>(x), T->nrows, T->rowptr,
                                        T->colind, static_cast<float*>(gvals), s);
  return tri_coop_launch<double, true>(nlevels, level_ptr, level_rows, Tt->rowptr, Tt->colind,
                                       perm, static_cast<const double*>(T->vals),
                                       static_cast<const double*>(gx), static_cast<double*>(gb),
                                       static_cast<const double*>(x), T->nrows, T->rowptr,
                                       T->colind, static_cast<double*>(gvals), s);
}
