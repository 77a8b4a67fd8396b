// lbrb_device.h -- device helpers shared by the step kernels and the adjoint kernels:
// index arithmetic, the thread -> node map, the pull of a node's populations (and its
// transpose), the fixed-point spread-force accumulators, the XCD-aware tile order and the
// periodic cell index of a coordinate.
#ifndef LBRB_DEVICE_H
#define LBRB_DEVICE_H

#include <hip/hip_runtime.h>

#include "lbrb_layout.h"

namespace lbrb {

__device__ __forceinline__ int wrap1(int v, int n)
{
    return v < 0 ? v + n : (v >= n ? v - n : v);
}

// A bead record read whole, as eight 16-byte loads in one round.  Read field by field, the
// compiler issues a field's load where it is first used; for fields first used after a
// branch or a barrier that is a dependent round trip of its own.  The empty asm takes every
// loaded word as an operand, so all eight loads are issued before it.
__device__ __forceinline__ BeadRec load_record(const BeadRec* p)
{
    constexpr int kWords = (int)(sizeof(BeadRec) / sizeof(uint4));
    const uint4* src = reinterpret_cast<const uint4*>(p);
    uint4 q[kWords];
#pragma unroll
    for (int k = 0; k < kWords; ++k) q[k] = src[k];
#pragma unroll
    for (int k = 0; k < kWords; ++k) asm volatile("" ::"v"(q[k].x), "v"(q[k].y), "v"(q[k].z), "v"(q[k].w));
    BeadRec B;
    __builtin_memcpy(&B, q, sizeof(BeadRec));
    return B;
}

// A bead record spread over the 8 lanes of its bead: lane j of the group holds bytes
// 16j .. 16j+15 (one coalesced 16-byte load per lane), and a field is gathered from its lane
// by a shuffle where it is used, so no lane keeps the whole record in registers.  Every lane
// of the group must take part in each gather (uniform control flow).
template <int K>   // 32-bit word K (0..31) of the record
__device__ __forceinline__ uint32_t rec_word(const uint4& q)
{
    static_assert(K >= 0 && K < 32, "a bead record has 32 words");
    const uint32_t v = (K & 3) == 0 ? q.x : (K & 3) == 1 ? q.y : (K & 3) == 2 ? q.z : q.w;
    return (uint32_t)__shfl((int)v, K >> 2, 8);
}
template <int K>   // the double at word K
__device__ __forceinline__ double rec_f64(const uint4& q)
{
    const uint64_t lo = rec_word<K>(q), hi = rec_word<K + 1>(q);
    return __longlong_as_double((long long)(lo | (hi << 32)));
}
#define LBRB_REC_WORD(field) ((int)(offsetof(BeadRec, field) / 4))

__device__ __forceinline__ int64_t current_step(const int64_t* p, int64_t arg)
{
    return (p ? *p : 0) + arg;
}

// exact floor(v / n) for 0 <= v < 2^52 via a double reciprocal and one correction
__device__ __forceinline__ int64_t div_exact(int64_t v, int32_t n, double inv)
{
    int64_t q = (int64_t)((double)v * inv);
    int64_t r = v - q * n;
    if (r < 0) q -= 1;
    else if (r >= n) q += 1;
    return q;
}

// coordinates of a local node index
template <bool MASKED>
__device__ __forceinline__ void locate(const ReplicaDesc& R, const RowDesc* __restrict__ rows,
                                       int row_lo, int row_hi, int64_t local, int& x, int& y,
                                       int& z, RowDesc& self)
{
    if constexpr (MASKED) {
        // largest row whose start <= local
        int lo = row_lo, hi = row_hi;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (rows[mid].start <= local) lo = mid; else hi = mid - 1;
        }
        self = rows[lo];
        x = self.xlo + (int)(local - self.start);
        y = self.yz & 0xFFFF;
        z = self.yz >> 16;
    } else {
        const int64_t row = div_exact(local, R.nx, R.inv_nx);
        x = (int)(local - row * R.nx);
        const int64_t zz = div_exact(row, R.ny, R.inv_ny);
        y = (int)(row - zz * R.ny);
        z = (int)zz;
        self.start = 0; self.xlo = 0; self.len = R.nx; self.yz = 0;
    }
}

// locate for a whole workgroup of a node tile (every thread calls it; a barrier inside for
// masked replicas): the descriptors of the rows the tile overlaps are loaded once into LDS
// (tile_rows, kNodeBlock entries: a tile of at most kNodeBlock nodes overlaps at most that many
// non-empty rows) and searched there instead of in global memory
template <bool MASKED>
__device__ __forceinline__ void locate_tile(const ReplicaDesc& R, const RowDesc* __restrict__ rows,
                                            const NodeTile& t, int64_t local, RowDesc* tile_rows,
                                            int& x, int& y, int& z, RowDesc& self)
{
    if constexpr (MASKED) {
        const int nr = t.row_hi - t.row_lo + 1;
        if (nr <= kNodeBlock) {
            if ((int)threadIdx.x < nr) tile_rows[threadIdx.x] = rows[t.row_lo + threadIdx.x];
            __syncthreads();
            locate<true>(R, tile_rows, 0, nr - 1, local, x, y, z, self);
        } else {
            locate<true>(R, rows, t.row_lo, t.row_hi, local, x, y, z, self);
        }
    } else {
        locate<false>(R, rows, t.row_lo, t.row_hi, local, x, y, z, self);
    }
}

// Fluid runs of the 9 rows (y - cy, z - cz), cy, cz in {-1, 0, 1}, at index (cy+1) + 3 (cz+1).
struct Rows9 {
    int32_t st[9], lo[9], ln[9];
};

__device__ __forceinline__ void load_rows9(const RowDesc* __restrict__ rowinfo, int32_t row_base,
                                           int ny, int nz, int y, int z, Rows9& rw)
{
#pragma unroll
    for (int r9 = 0; r9 < 9; ++r9) {
        const int cy = r9 % 3 - 1, cz = r9 / 3 - 1;
        const int yy = wrap1(y - cy, ny), zz = wrap1(z - cz, nz);
        const RowDesc rd = rowinfo[row_base + yy + ny * zz];
        rw.st[r9] = rd.start; rw.lo[r9] = rd.xlo; rw.ln[r9] = rd.len;
    }
}

// Byte offset of population i of local node loc from the replica's first population block:
// 32-bit arithmetic, valid when the replica's populations span at most 4 GiB (a node
// update then addresses memory as one uniform base plus a 32-bit offset per lane).
template <typename Real>
__device__ __forceinline__ uint32_t pop_byte32(uint32_t i, uint32_t loc)
{
    return ((((loc >> kPopBlockLog) * (uint32_t)Q + i) << kPopBlockLog) | (loc & 255u)) *
           (uint32_t)sizeof(Real);
}

template <typename Real, bool NARROW>
__device__ __forceinline__ Real load_pop(const Real* __restrict__ src, int64_t base, int i,
                                         int64_t local)
{
    if constexpr (NARROW) {
        const char* rb = (const char*)(src + (int64_t)Q * base);   // base: multiple of 256
        return *(const Real*)(rb + pop_byte32<Real>((uint32_t)i, (uint32_t)local));
    } else {
        return src[pop_at(i, base + local)];
    }
}

// Masked gather over preloaded rows: element i from x - S c_i (periodic in x) if that node is
// fluid, else population opposite(i) of the node itself (own = its local index).
// sw: the replica is stored with axes x and z exchanged (uniform over the workgroup).  Its
// population j then steps by (c_jz, c_jy, c_jx) in storage, which is the storage step of
// direction k = swap_xz(j): iteration k keeps its geometry and loads population swap_xz(k)
// into d[k], and the pairs (k, swap_xz(k)) are exchanged afterwards.  Same registers, same
// loads, a scalar choice of population per iteration.
template <typename Real, int S, bool NARROW = false>
__device__ __forceinline__ void pull_rows(const Real* __restrict__ src, int64_t base, int nx,
                                          const Rows9& rw, int x, int64_t own, Real d[Q],
                                          bool sw = false)
{
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int cx = S * cx_of(i), cy = S * cy_of(i), cz = S * cz_of(i);
        const int r9 = (cy + 1) + 3 * (cz + 1);
        const int xs = wrap1(x - cx, nx);
        const int off = xs - rw.lo[r9];
        const bool fluid = (unsigned)off < (unsigned)rw.ln[r9];
        const int64_t l = fluid ? (int64_t)rw.st[r9] + off : own;
        const int j = sw ? swap_xz_of(i) : i;
        const int p = fluid ? j : opposite_of(j);
        d[i] = load_pop<Real, NARROW>(src, base, p, l);
    }
    if (sw) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int k = swap_xz_of(i);
            if (k > i) {
                const Real t = d[i];
                d[i] = d[k];
                d[k] = t;
            }
        }
    }
}

// Pre-collision populations of node (x,y,z) (shifted), pulled from the post-collision
// buffer: population i comes from x - c_i, or, if that node is a boundary node, from the
// opposite population of the node itself (halfway bounce-back).  With S = -1 the same gather
// runs along +c_i: element i is taken from x + c_i, or from the opposite population of x
// when x + c_i is a boundary node -- the transpose of streaming, used by the adjoint.
template <typename Real, bool MASKED, int S = 1, bool NARROW = false>
__device__ __forceinline__ void pull(const Real* __restrict__ src, int64_t N,
                                     const ReplicaDesc& R, const RowDesc* __restrict__ rowinfo,
                                     int x, int y, int z, int64_t local, const RowDesc& self,
                                     Real d[Q])
{
    if constexpr (MASKED) {
        // the node's own row is known; the other 8 rows (y - S cy, z - S cz) are loaded
        Rows9 rw;
#pragma unroll
        for (int r9 = 0; r9 < 9; ++r9) {
            const int cy = r9 % 3 - 1, cz = r9 / 3 - 1;
            if (cy == 0 && cz == 0) {
                rw.st[r9] = self.start; rw.lo[r9] = self.xlo; rw.ln[r9] = self.len;
            } else {
                const int yy = wrap1(y - cy, R.ny), zz = wrap1(z - cz, R.nz);
                const RowDesc rd = rowinfo[R.row_base + yy + R.ny * zz];
                rw.st[r9] = rd.start; rw.lo[r9] = rd.xlo; rw.ln[r9] = rd.len;
            }
        }
        pull_rows<Real, S, NARROW>(src, R.base, R.nx, rw, x, local, d, R.swap != 0);
    } else {
        const int xm = wrap1(x - 1, R.nx), xp = wrap1(x + 1, R.nx);
        const int ym = wrap1(y - 1, R.ny), yp = wrap1(y + 1, R.ny);
        const int zm = wrap1(z - 1, R.nz), zp = wrap1(z + 1, R.nz);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int cx = S * cx_of(i), cy = S * cy_of(i), cz = S * cz_of(i);
            const int xs = cx == 0 ? x : (cx > 0 ? xm : xp);
            const int ys = cy == 0 ? y : (cy > 0 ? ym : yp);
            const int zs = cz == 0 ? z : (cz > 0 ? zm : zp);
            const int64_t l = xs + (int64_t)R.nx * (ys + (int64_t)R.ny * zs);
            d[i] = load_pop<Real, NARROW>(src, R.base, i, l);
        }
    }
}

// ------------------------------------------------------------------ spread force
// Bead forces are spread as sums of 64-bit integers, so the total on a node does not depend
// on the order of the atomic additions.  Word 0 counts units of 2^-56 (signed; a node's
// total must stay below 128 in magnitude); in FP64 a second word carries the remainder of
// each contribution in units of 2^-104, which makes the spread exact to far below FP64
// rounding.  A remainder lies in [0, 2^48) and the second word is read back as unsigned, so
// it holds the sum of up to 65535 contributions (beads whose stencil holds the node, times
// MD steps per fluid step) without wrapping.  Layout: the words of a node are contiguous,
// word w of axis ax of node g at gforce[g * spread_stride + 3 w + ax], padded to 32 bytes
// (FP32: 3 words) or 64 bytes (FP64: 6 words), so the atomics on a node and the node
// update's read-and-clear touch one cache line.
// the fixed-point words of one contribution: hi in units of 2^-56, lo (FP64 only) the
// remainder in units of 2^-104
template <typename Real>
__device__ __forceinline__ void spread_words(double val, long long& hi, long long& lo)
{
    const double x = val * 0x1p56;
    const double h = floor(x);
    hi = (long long)h;
    lo = sizeof(Real) == 8 ? (long long)((x - h) * 0x1p48) : 0;
}

// add the spread force of node g to F and clear its words (16-byte loads and stores)
template <typename Real>
__device__ __forceinline__ void take_spread_force(long long* gforce, int64_t g, Real F[3])
{
    constexpr int S = spread_stride<Real>();
    long long* p = gforce + g * S;
    long long w[S];
#pragma unroll
    for (int k = 0; k < S; k += 2) {
        const longlong2 v = *reinterpret_cast<const longlong2*>(p + k);
        w[k] = v.x;
        w[k + 1] = v.y;
    }
#pragma unroll
    for (int k = 0; k < S; k += 2) *reinterpret_cast<longlong2*>(p + k) = make_longlong2(0, 0);
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        double v = (double)w[ax] * 0x1p-56;
        if constexpr (sizeof(Real) == 8) v += (double)(unsigned long long)w[3 + ax] * 0x1p-104;
        F[ax] += (Real)v;
    }
}

// Workgroups are dealt round-robin to the 8 XCDs (separate L2 caches).  Give each XCD a
// contiguous run of tiles so that the halo lines shared by neighbouring tiles are mostly
// reused from the same L2.
__device__ __forceinline__ int xcd_tile(int b, int n)
{
    const int q = n >> 3, r = n & 7, xcd = b & 7, k = b >> 3;
    return xcd * q + min(xcd, r) + k;
}

// periodic cell index and fraction of a coordinate; a non-finite or absurdly large
// coordinate (a diverged body) maps to cell 0 so that no access leaves the box
__device__ __forceinline__ int wrap_floor(double v, int n, double& frac)
{
    if (!(fabs(v) < 1e15)) { frac = 0.0; return 0; }
    const double fl = floor(v);
    frac = v - fl;
    // fl - n floor(fl / n) is exact for |fl| < 2^52; the guard absorbs a quotient rounded up
    double m = fl - (double)n * floor(fl / (double)n);
    if (m >= (double)n) m -= (double)n;
    if (m < 0.0) m += (double)n;
    return (int)m;
}

}  // namespace lbrb

#endif
