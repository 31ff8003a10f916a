// Allocation-free apply_op for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc).  apply_op needs four scratch blocks per chunk of columns: X in
// the library's order (column-major and row-interleaved), A X, and B X before
// it goes back to the caller's order.  Here they live in one file-scope device
// array instead of fresh allocations.
//
// The array exists once per device and is held until the process ends.  Its
// device address is resolved with hipGetSymbolAddress at nullspace_init, with
// the caller's device current, and kept per device: in host code the array's
// name is only a host-side stand-in, so every kernel argument uses the
// resolved address.  Every call on a device shares that device's array:
// calls that overlap in time on one device (other contexts, other streams)
// race on it and must be serialised by the caller.  Nothing in it has to start
// at zero (each chunk writes its blocks before reading them).
#include <mutex>

#include "common.h"
#include "kernels.h"

namespace nsp {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

namespace {
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};  // device address of ``scratch`` on each device
}  // namespace

void noalloc_setup() {
  int dev = 0;
  NSP_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw Error(NSP_ERR_ARG, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[dev]) return;
  void* p = nullptr;
  NSP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (p == nullptr) throw Error(NSP_ERR_HIP, "hipGetSymbolAddress returned NULL for the scratch array");
  g_scratch[dev] = static_cast<double*>(p);
}

// Y = B X like apply_b_colmajor, in chunks of the widest column count whose
// four blocks (3 n + m doubles per column, each block starting on a 256-byte
// boundary) fit in the array.
void apply_b_noalloc(nsp_ctx* c, const double* X, int64_t ldx, double* Y, int64_t ldy, int ncols) {
  const int64_t n = c->n, m = c->m;
  double* s = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (c->device >= 0 && c->device < kMaxDevices) s = g_scratch[c->device];
  }
  if (s == nullptr) throw Error(NSP_ERR_STATE, "scratch array not set up on the context's device");
  auto up = [](int64_t x) { return (x + 31) / 32 * 32; };  // doubles, 256-byte multiples
  auto need = [&](int w) { return (3 * up(n * w) + up(m * w)) * (int64_t)sizeof(double); };
  int wmax = 0;
  for (int w : {kMaxD, 4, 2, 1})
    if (need(w) <= (int64_t)kScratchBytes) { wmax = w; break; }
  if (wmax == 0)
    throw Error(NSP_ERR_ARG, "apply_op_noalloc needs " + std::to_string(need(1)) +
                                 " bytes of scratch for one column (3 n + m doubles), more than its " +
                                 std::to_string(kScratchBytes) + "-byte array");
  double* xc = s;
  double* xr = xc + up(n * wmax);
  double* zr = xr + up(n * wmax);
  double* yr = zr + up(n * wmax);
  apply_b_chunks(c, X, ldx, Y, ldy, ncols, wmax, xc, xr, yr, zr);
}

}  // namespace nsp
