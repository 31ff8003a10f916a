// placeholder; replaced by the Lanczos driver
#include "common.h"
namespace nsp {
void solve(nsp_ctx*) { throw Error(NSP_ERR_STATE, "solver not built yet"); }
void run_backward(nsp_ctx*, const double*, int64_t, double*, double, int64_t, int64_t*) {
  throw Error(NSP_ERR_STATE, "backward not built yet");
}
}  // namespace nsp
