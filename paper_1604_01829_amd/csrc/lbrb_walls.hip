// lbrb_walls.hip -- the moving-wall link kernel (see lbrb_walls.h).
#include "lbrb_layout.h"
#include "lbrb_walls.h"

namespace lbrb {

template <typename Real>
__global__ __launch_bounds__(256) void wall_links_kernel(Real* f, const WallLink* links,
                                                         int64_t n_links)
{
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= n_links) return;
    const WallLink L = links[k];
    Real* p = f + pop_at(L.pop, L.g);
    *p = *p + (Real)L.delta;
}

template <typename Real>
void launch_wall_links(Real* f, const WallLink* links, int64_t n_links, hipStream_t s)
{
    if (n_links <= 0) return;
    const int64_t blocks = (n_links + 255) / 256;
    hipLaunchKernelGGL((wall_links_kernel<Real>), dim3((unsigned)blocks), dim3(256), 0, s, f,
                       links, n_links);
}

template void launch_wall_links<float>(float*, const WallLink*, int64_t, hipStream_t);
template void launch_wall_links<double>(double*, const WallLink*, int64_t, hipStream_t);

}  // namespace lbrb
