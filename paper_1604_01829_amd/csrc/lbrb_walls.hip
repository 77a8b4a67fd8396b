// lbrb_walls.hip -- the moving-wall link kernel and the hole mirrors (see lbrb_walls.h).
#include "lbrb_device.h"
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

// one thread per stored node of the tiles of replicas with holes.  TRANSPOSED: the reverse
// pass's mirror, slot opp(i) of the hole takes population i of x (lambda_opp(i)(h) =
// lambda_i(h + c_i)), so that the transposed pull at a fluid node y = h - c_j reads, from the
// hole's slot j, its own lambda_opp(j)(y): the transpose of halfway bounce-back.
template <typename Real, bool TRANSPOSED>
__global__ __launch_bounds__(kNodeBlock) void mirror_holes_kernel(Real* f, const ReplicaDesc* reps,
                                                                  const RowDesc* rows,
                                                                  const RowDesc* rowinfo,
                                                                  const NodeTile* tiles,
                                                                  const uint8_t* hole)
{
    const NodeTile t = tiles[blockIdx.x];
    if ((int)threadIdx.x >= t.count) return;
    const ReplicaDesc R = reps[t.replica];
    const int64_t local = t.begin + threadIdx.x;
    const int64_t g = R.base + local;
    if (hole[g] == 0) return;
    int x, y, z;
    RowDesc self;
    locate<true>(R, rows, t.row_lo, t.row_hi, local, x, y, z, self);
    for (int i = 1; i < Q; ++i) {
        // c_i in storage coordinates (axes x and z exchanged for a swapped replica)
        const int ci_x = R.swap ? cz_of(i) : cx_of(i), ci_z = R.swap ? cx_of(i) : cz_of(i);
        const int xs = wrap1(x + ci_x, R.nx), ys = wrap1(y + cy_of(i), R.ny),
                  zs = wrap1(z + ci_z, R.nz);
        const RowDesc rd = rowinfo[R.row_base + ys + R.ny * zs];
        const int off = xs - rd.xlo;
        if ((unsigned)off >= (unsigned)rd.len) continue;       // not stored: boundary node
        const int64_t gx = R.base + rd.start + off;
        if (hole[gx] != 0) continue;                             // another hole
        if (TRANSPOSED) f[pop_at(opposite_of(i), g)] = f[pop_at(i, gx)];
        else f[pop_at(i, g)] = f[pop_at(opposite_of(i), gx)];
    }
}

template <typename Real>
void launch_mirror_holes(Real* f, const ReplicaDesc* reps, const RowDesc* rows,
                         const RowDesc* rowinfo, const NodeTile* tiles, int32_t n_tiles,
                         const uint8_t* hole, hipStream_t s)
{
    if (n_tiles <= 0) return;
    hipLaunchKernelGGL((mirror_holes_kernel<Real, false>), dim3(n_tiles), dim3(kNodeBlock), 0, s, f,
                       reps, rows, rowinfo, tiles, hole);
}

template <typename Real>
void launch_mirror_holes_transposed(Real* lam, const ReplicaDesc* reps, const RowDesc* rows,
                                    const RowDesc* rowinfo, const NodeTile* tiles, int32_t n_tiles,
                                    const uint8_t* hole, hipStream_t s)
{
    if (n_tiles <= 0) return;
    hipLaunchKernelGGL((mirror_holes_kernel<Real, true>), dim3(n_tiles), dim3(kNodeBlock), 0, s,
                       lam, reps, rows, rowinfo, tiles, hole);
}

template void launch_mirror_holes<float>(float*, const ReplicaDesc*, const RowDesc*,
                                         const RowDesc*, const NodeTile*, int32_t,
                                         const uint8_t*, hipStream_t);
template void launch_mirror_holes<double>(double*, const ReplicaDesc*, const RowDesc*,
                                          const RowDesc*, const NodeTile*, int32_t,
                                          const uint8_t*, hipStream_t);
template void launch_mirror_holes_transposed<float>(float*, const ReplicaDesc*, const RowDesc*,
                                                    const RowDesc*, const NodeTile*, int32_t,
                                                    const uint8_t*, hipStream_t);
template void launch_mirror_holes_transposed<double>(double*, const ReplicaDesc*, const RowDesc*,
                                                     const RowDesc*, const NodeTile*, int32_t,
                                                     const uint8_t*, hipStream_t);
template void launch_wall_links<float>(float*, const WallLink*, int64_t, hipStream_t);
template void launch_wall_links<double>(double*, const WallLink*, int64_t, hipStream_t);

}  // namespace lbrb
