// CSR transpose without a caller workspace, for callers that cannot
// allocate device memory (code under stream capture, serving loops,
// harnesses that forbid hipMalloc).  The scratch space the transpose needs
// (column counts, the scan's tile sums, the scatter's key/value arrays,
// the long-column list and the path flags) lives in one file-scope device
// array of kScratchBytes.  Each GPU the library runs on holds its own copy
// of that array, at its own address, until the process ends.
//
// The array's name is a host-side stand-in in host code, not a device
// address: the address is taken once per device with hipGetSymbolAddress
// (with that device current) and only that pointer is handed to kernels.
// Every call on one GPU shares the array, so calls that overlap on one GPU
// (different streams, or host threads) race; calls on one stream are
// ordered and safe.  The transpose clears what must start at zero itself
// (with fill kernels), so the contents a previous call left do not matter.
#include <mutex>

#include "internal.hpp"

namespace csrad {
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per
// device); null on a HIP error.
void* scratch_address() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

}  // namespace
}  // namespace csrad

using namespace csrad;

extern "C" size_t csr_noalloc_scratch_bytes(void) { return kScratchBytes; }

extern "C" int csr_transpose_noalloc(const csrad_csr* A, int32_t* rowptrT, int32_t* colindT,
                                     int32_t* perm, void* stream) {
  CSRAD_TRY(check_csr(A, false));
  if (!rowptrT || (A->nnz > 0 && (!colindT || !perm))) return CSRAD_EINVAL;
  const size_t need = transpose_workspace(A->nrows, A->ncols, A->nnz);
  if (need > kScratchBytes) return CSRAD_EWORKSPACE;
  void* ws = scratch_address();
  if (!ws) return CSRAD_EHIP;
  return transpose_pattern(A->nrows, A->ncols, A->nnz, A->rowptr, A->colind, rowptrT, colindT,
                           perm, ws, kScratchBytes, as_stream(stream));
}
