// spotfit_owned.hip -- the lane-owned fit kernel (spotfit_owned.h) for
// batches of spots up to 16 x 16 pixels handed out in index order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spotfit.h"
#include "spotfit_internal.h"
#include "spotfit_owned.h"

namespace sf {
namespace own {

template <int L, int CPL, int WPE, int DT, int OWN>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WPE))) void fit_owned_kernel(KArgs ka) {
  __shared__ OShared sh;
  fit_owned<L, CPL, DT, OWN>(ka, nullptr, ka.queue, (int32_t)ka.n, sh);
}

__global__ void owned_queue_reset_kernel(int32_t* take) {
  if (threadIdx.x == 0) *take = 0;
}

}  // namespace own

// The lane-owned plans, at 2 waves per SIMD (lanes per group, columns per lane,
// spots per group): 4-lane groups with 4 columns per lane (spots up to 16 x 16
// pixels) holding 4 spots (one per lane, 64 per wavefront) or 2 (a lane pair
// per spot: half the pixels in flight, twice the scalar work per spot); 4-lane
// groups with 2 columns per lane (up to 8 x 8), 4 spots; 16-lane groups with 2
// columns per lane (up to 32 x 32) holding 4 spots (4 lanes per spot) or 8.
constexpr int kOwnedWpe = 2;

#define SF_OWNED_KERNELS(X) X(4, 4, 4) X(4, 4, 2) X(4, 2, 4) X(16, 2, 4) X(16, 2, 8)

const void* owned_kernel_symbol(int lanes, int cpl, int own) {
#define SF_OSYM(L, C, O)                               \
  if (lanes == L && cpl == C && own == O)              \
    return reinterpret_cast<const void*>(&own::fit_owned_kernel<L, C, kOwnedWpe, SPOTFIT_U16, O>);
  SF_OWNED_KERNELS(SF_OSYM)
#undef SF_OSYM
  return nullptr;
}

hipError_t launch_owned_kernel(int lanes, int cpl, int own, const KArgs& ka, int grid, hipStream_t st) {
  if (!owned_kernel_symbol(lanes, cpl, own)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(own::owned_queue_reset_kernel, dim3(1), dim3(64), 0, st, ka.queue);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
#define SF_OLAUNCH(L, C, O)                                                                        \
  if (lanes == L && cpl == C && own == O) {                                                        \
    if (ka.dtype == SPOTFIT_U16)                                                                   \
      hipLaunchKernelGGL((own::fit_owned_kernel<L, C, kOwnedWpe, SPOTFIT_U16, O>), dim3(grid), dim3(64), \
                         0, st, ka);                                                               \
    else                                                                                           \
      hipLaunchKernelGGL((own::fit_owned_kernel<L, C, kOwnedWpe, SPOTFIT_F32, O>), dim3(grid), dim3(64), \
                         0, st, ka);                                                               \
  }
  SF_OWNED_KERNELS(SF_OLAUNCH)
#undef SF_OLAUNCH
  return hipGetLastError();
}

}  // namespace sf
