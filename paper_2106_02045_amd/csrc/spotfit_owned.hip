// spotfit_owned.hip -- the lane-owned fit kernel (spotfit_owned.h) for
// batches of spots up to 16 x 16 pixels handed out in index order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spotfit.h"
#include "spotfit_internal.h"
#include "spotfit_owned.h"

namespace sf {
namespace own {

template <int CPL, int WPE, int DT, int OWN>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WPE))) void fit_owned_kernel(KArgs ka) {
  __shared__ OShared sh;
  fit_owned<CPL, DT, OWN>(ka, nullptr, ka.queue, (int32_t)ka.n, sh);
}

__global__ void owned_queue_reset_kernel(int32_t* take) {
  if (threadIdx.x == 0) *take = 0;
}

}  // namespace own

// The lane-owned plans: 4-lane groups of 4 columns per lane (spots up to 16 x
// 16 pixels) at 2 waves per SIMD, holding 4 spots per group (one per lane, 64
// per wavefront) or 2 (a lane pair per spot, 32 per wavefront: half the pixels
// in flight, twice the scalar work per spot).
constexpr int kOwnedCpl = 4, kOwnedWpe = 2;

const void* owned_kernel_symbol(int own) {
  return own == 2 ? reinterpret_cast<const void*>(&own::fit_owned_kernel<kOwnedCpl, kOwnedWpe, SPOTFIT_U16, 2>)
                  : reinterpret_cast<const void*>(&own::fit_owned_kernel<kOwnedCpl, kOwnedWpe, SPOTFIT_U16, 4>);
}

template <int OWN>
static void launch_owned(const KArgs& ka, int grid, hipStream_t st) {
  if (ka.dtype == SPOTFIT_U16)
    hipLaunchKernelGGL((own::fit_owned_kernel<kOwnedCpl, kOwnedWpe, SPOTFIT_U16, OWN>), dim3(grid), dim3(64),
                       0, st, ka);
  else
    hipLaunchKernelGGL((own::fit_owned_kernel<kOwnedCpl, kOwnedWpe, SPOTFIT_F32, OWN>), dim3(grid), dim3(64),
                       0, st, ka);
}

hipError_t launch_owned_kernel(int own, const KArgs& ka, int grid, hipStream_t st) {
  if (own != 2 && own != 4) return hipErrorInvalidValue;
  hipLaunchKernelGGL(own::owned_queue_reset_kernel, dim3(1), dim3(64), 0, st, ka.queue);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (own == 2)
    launch_owned<2>(ka, grid, st);
  else
    launch_owned<4>(ka, grid, st);
  return hipGetLastError();
}

}  // namespace sf
