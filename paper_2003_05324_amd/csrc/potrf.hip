// FP64 Cholesky of one diagonal tile (dpotrf of Algorithm 1) fused with its inverse, the
// forward-solve block and the log-determinant / quadratic-form parts of eq. (2): one
// workgroup per launch on the critical path of the step-ordered factorization.  The body is
// in potrf_dev.h.
#include "potrf_dev.h"

namespace mpgeo {

namespace {

template <int kPotrfThreads>
__global__ __launch_bounds__(kPotrfThreads) void potrf_tile_kernel(PotrfArgs args) {
    potrf_tile_body<kPotrfThreads>(args);
}

}  // namespace

template <int T>
void launch_potrf_threads(const PotrfArgs &a, hipStream_t stream) {
    hipLaunchKernelGGL((potrf_tile_kernel<T>), dim3(1), dim3(T), 0, stream, a);
}

void launch_potrf(const PotrfArgs &a, hipStream_t stream) { launch_potrf_threads<512>(a, stream); }

}  // namespace mpgeo
