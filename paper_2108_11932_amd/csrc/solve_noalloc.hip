// tlr_solve_noalloc: the TLR solve (Algorithm "TLR Triangular Solve" and its
// transpose, Section 4.4) with its workspace in a fixed device array instead
// of memory the handle allocates, for callers that cannot allocate.
//
// The solve's workspace (the padded right-hand sides, one diagonal block of
// them and the per-column products V^T x / U^T x) lives in `scratch`, one
// copy per GPU, kept until the process ends.  Its device address is looked
// up once per device with hipGetSymbolAddress (the array's name is only a
// host-side stand-in) and only that address is handed to the kernels.  The
// launch descriptors go through the handle's pinned staging ring, which was
// allocated when the handle was created; during this call the ring may not
// grow (an oversized batch is an argument error instead).
#include <mutex>

#include "host.h"

namespace {

constexpr size_t kScratchBytes = (size_t)32 << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch`; device `dev` must be
// current.
tlr_status scratch_on(int dev, double** out) {
  if (dev < 0 || dev >= kMaxDevices) {
    tlr::set_error("device %d out of range for the solve scratch", dev);
    return TLR_ERR_ARG;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      tlr::set_error("hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
      return TLR_ERR_DEVICE;
    }
    g_ptr[dev] = (double*)p;
  }
  *out = g_ptr[dev];
  return TLR_OK;
}

}  // namespace

extern "C" {

size_t tlr_solve_noalloc_max_bytes(void) { return kScratchBytes; }

tlr_status tlr_solve_noalloc(tlr_matrix_t A, int nrhs, double* B, long long ldb, void* stream) {
  using namespace tlr;
  if (!A || !B) {
    set_error("NULL argument");
    return TLR_ERR_ARG;
  }
  if (nrhs < 0 || ldb < A->N) {
    set_error(nrhs < 0 ? "nrhs must be non-negative" : "ldb < N");
    return TLR_ERR_ARG;
  }
  if (!A->factored) {
    set_error("the handle holds no factor");
    return TLR_ERR_STATE;
  }
  if (nrhs == 0) return TLR_OK;
  const size_t need = sizeof(double) * solve_workspace(A, nrhs);
  if (need > kScratchBytes) {
    set_error("the solve of %d right-hand sides needs %zu bytes of workspace, more than the "
              "%zu-byte fixed scratch", nrhs, need, kScratchBytes);
    return TLR_ERR_ARG;
  }
  int cur = 0;
  TLR_HIP(hipGetDevice(&cur));
  if (cur != A->dev) TLR_HIP(hipSetDevice(A->dev));
  double* work = nullptr;
  tlr_status st = scratch_on(A->dev, &work);
  if (st == TLR_OK) {
    A->stream = A->mem.stream = (hipStream_t)stream;
    A->stage.fixed = true;
    st = solve_in(A, nrhs, B, ldb, work);
    A->stage.fixed = false;
  }
  if (cur != A->dev) (void)hipSetDevice(cur);
  return st;
}

}  // extern "C"
