// Internal host entry points shared between translation units of the
// csrad library (not part of the C ABI).
#pragma once

#include "common.hpp"

namespace csrad {

// Exclusive prefix sum of n int32 counts: out[0] = 0, out[i+1] =
// in[0] + ... + in[i] (n+1 outputs).  The exact 64-bit total goes to
// *total_dev; out[] is only meaningful when the total fits int32.  With
// skip non-null, the kernels do nothing when *skip (device) is non-zero.
size_t scan_workspace(int n);
int scan_exclusive(const int32_t* in, int32_t* out, int n, long long* total_dev,
                   void* work, size_t bytes, hipStream_t s, const int32_t* skip = nullptr);

// Stable transpose of a CSR pattern (see csr_transpose).
size_t transpose_workspace(int m, int n, int nnz);
int transpose_pattern(int m, int n, int nnz, const int32_t* rowptr, const int32_t* colind,
                      int32_t* rowptrT, int32_t* colindT, int32_t* perm, void* work,
                      size_t bytes, hipStream_t s);

// Stable grouping of n indices by a key in [0, K), K <= 32 (see
// transpose.hip): ptr[K+1], order[n] (indices ascending within a key).
size_t group_small_workspace(int n, int K);
// With skip non-null, nothing is done when *skip (device) is non-zero.
int group_small_keys(const int32_t* keys, int n, int K, int32_t* ptr, int32_t* order, void* work,
                     size_t bytes, hipStream_t s, const int32_t* skip = nullptr);

// Level-scheduled solve with float64 vectors over T's value type (see
// trisolve.hip); transpose selects T^{-T} over Tt/perm with reversed levels.
int trisolve_vec64(const csrad_csr* Tm, int lower, const csrad_csr* Tt, const int32_t* perm,
                   bool transpose, int nlevels, const int32_t* lp_host, const int32_t* lp_dev,
                   const int32_t* rows, const double* b, double* x, hipStream_t s);

// Fill a device int32 array with a value (graph-capture safe, no memset node).
int fill_i32(int32_t* p, long long n, int32_t value, hipStream_t s);
int fill_bytes_zero(void* p, size_t bytes, hipStream_t s);

}  // namespace csrad
