// Sums of an array over contiguous ranges of the compacted list, in FP64 and
// in a fixed order: the mass of a pool per z-layer (raster order makes every
// layer a contiguous range) or per brick (brick order), as the layer profiles
// of the paper's diffusion comparison (Sec. IV.B) need.
#include "vg_internal.h"

namespace vg {
namespace {

// One block per range (grid-stride over ranges); each thread sums a strided
// share, then the block adds the shares in a fixed order.  Offsets are
// clamped into [0, n], so no offset can make the kernel read outside x.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_range_sums(const R *__restrict__ x, int64_t n,
                                                       const int64_t *__restrict__ off, int64_t nranges,
                                                       double *__restrict__ out) {
    __shared__ double lds[kWaves];
    for (int64_t r = blockIdx.x; r < nranges; r += gridDim.x) {
        int64_t lo = off[r], hi = off[r + 1];
        lo = lo < 0 ? 0 : (lo > n ? n : lo);
        hi = hi < lo ? lo : (hi > n ? n : hi);
        double v[1] = {0.0};
        for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) v[0] += (double)x[i];
        block_sum<1>(v, lds);
        if (threadIdx.x == 0) out[r] = v[0];
    }
}

}  // namespace
}  // namespace vg

using namespace vg;

extern "C" int vg_range_sums(const void *x_d, int precision, int64_t n, const int64_t *offsets_d, int64_t nranges,
                             double *out_d, void *stream) {
    if (n < 0 || nranges < 0 || (precision != VG_F32 && precision != VG_F64) ||
        (nranges > 0 && (!offsets_d || !out_d || (n > 0 && !x_d)))) {
        set_error("bad range-sum arguments");
        return VG_EINVAL;
    }
    if (nranges == 0) return VG_OK;
    const unsigned grid = (unsigned)(nranges < 65536 ? nranges : 65536);
    if (precision == VG_F64)
        hipLaunchKernelGGL(k_range_sums<double>, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream,
                           (const double *)x_d, n, offsets_d, nranges, out_d);
    else
        hipLaunchKernelGGL(k_range_sums<float>, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream,
                           (const float *)x_d, n, offsets_d, nranges, out_d);
    return launch_status("k_range_sums");
}
