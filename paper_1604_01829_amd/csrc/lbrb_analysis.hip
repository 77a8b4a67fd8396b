// lbrb_analysis.hip -- trajectory analysis on the device (the C-ABI functions lb_traj_*
// and the pose recorder behind rb_record_poses).
//
// A trajectory is traj[frame][body][7]: centre (x, y, z; lab frame, unwrapped) and unit
// quaternion (w, x, y, z) of every body at every recording.  The analysis follows Sec. 2.4-2.8
// of the paper: the lab-frame MSD of the centre (eq. (dt_lab)), the lab-frame MSD of the angle
// of a reference vector (eqs. (dr_lab), (delta_theta)), body-frame displacements (each
// recording interval's lab displacement turned into the body frame with the orientation at the
// start of the interval, then summed, Sec. 2.6), body-frame rotation angles by projecting the
// body axes at t onto the planes normal to the axes at t - 1 (Sec. 2.7), and pore-frame
// displacements (the interval's displacement rotated by minus the polar angle of the centre
// about the pore axis at the start of the interval, then summed, Sec. 2.8) with MSDs binned
// by the radial position of each origin frame.
//
// Series are stored body-major, series[body][frame][k], so the MSD kernels read contiguous
// frames.  Every sum runs in a fixed order (thread-strided loops, shuffle + LDS trees): the
// results do not depend on timing.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <cmath>

#include "../../include/lbrb.h"
#include "lbrb_analysis.h"

namespace lbrb {
namespace {

constexpr int kBlock = 256;

// rotation matrix (body -> lab) of a unit quaternion, row-major
__device__ __forceinline__ void rot_of(const double* q, double R[9])
{
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - z * w); R[2] = 2.0 * (x * z + y * w);
    R[3] = 2.0 * (x * y + z * w); R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - x * w);
    R[6] = 2.0 * (x * z - y * w); R[7] = 2.0 * (y * z + x * w); R[8] = 1.0 - 2.0 * (x * x + y * y);
}

// sum over the workgroup of v[0..K), fixed order; the result is valid in thread 0
template <int K>
__device__ __forceinline__ void block_sum(double v[K], double (*part)[K])
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1)
        for (int k = 0; k < K; ++k) v[k] += __shfl_down(v[k], m, 64);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < K; ++k) part[wave][k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 0; k < K; ++k) v[k] = (part[0][k] + part[1][k]) + (part[2][k] + part[3][k]);
}

// ------------------------------------------------------------------ poses

__global__ void record_kernel(const Body* bodies, int n_bodies, double* frame)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_bodies) return;
    const Body& B = bodies[b];
    for (int a = 0; a < 3; ++a) frame[7 * (int64_t)b + a] = B.pos[a];
    for (int a = 0; a < 4; ++a) frame[7 * (int64_t)b + 3 + a] = B.quat[a];
}

// ------------------------------------------------------------------ cumulative series

// per-interval increments of one body between frames n-1 and n
struct LabStep {
    static constexpr int K = 3;
    __device__ static void delta(const double* p0, const double* p1, double, double, double d[K])
    {
        for (int a = 0; a < 3; ++a) d[a] = p1[a] - p0[a];
    }
};

struct BodyStep {
    static constexpr int K = 6;
    // displacement in the body frame at the interval start, and the projection angles
    __device__ static void delta(const double* p0, const double* p1, double, double, double d[K])
    {
        double A[9], Rn[9];
        rot_of(p0 + 3, A);      // columns: body axes at t-1
        rot_of(p1 + 3, Rn);     // columns: body axes at t
        const double dx[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
        for (int a = 0; a < 3; ++a) d[a] = A[a] * dx[0] + A[3 + a] * dx[1] + A[6 + a] * dx[2];
        // axis u of t, minus its component along axis e of t-1, expressed in the t-1 frame
        auto proj = [&](int u, int e, double out[3]) {
            const double v[3] = {Rn[u], Rn[3 + u], Rn[6 + u]};
            const double ee[3] = {A[e], A[3 + e], A[6 + e]};
            const double s = v[0] * ee[0] + v[1] * ee[1] + v[2] * ee[2];
            const double p[3] = {v[0] - ee[0] * s, v[1] - ee[1] * s, v[2] - ee[2] * s};
            for (int r = 0; r < 3; ++r) out[r] = A[r] * p[0] + A[3 + r] * p[1] + A[6 + r] * p[2];
        };
        double k2[3], i2[3], j2[3];
        proj(2, 0, k2);     // z axis onto the plane normal to x
        proj(0, 1, i2);     // x axis onto the plane normal to y
        proj(1, 2, j2);     // y axis onto the plane normal to z
        d[3] = atan(k2[1] / k2[2]);
        d[4] = atan(i2[2] / i2[0]);
        d[5] = atan(j2[0] / j2[1]);
    }
};

struct PoreStep {
    static constexpr int K = 3;
    // displacement rotated by minus the polar angle about the axis (cx, cy) at the start
    __device__ static void delta(const double* p0, const double* p1, double cx, double cy,
                                 double d[K])
    {
        const double th = atan2(p0[1] - cy, p0[0] - cx);
        const double c = cos(th), s = sin(th);
        const double dx = p1[0] - p0[0], dy = p1[1] - p0[1];
        d[0] = c * dx + s * dy;
        d[1] = -s * dx + c * dy;
        d[2] = p1[2] - p0[2];
    }
};

// One workgroup per body: the F - 1 interval increments are cut into 256 contiguous chunks;
// each thread sums its chunk, thread 0 turns the chunk sums into prefixes, then each thread
// writes its chunk's running sums.  out[body][frame][K], 0 at frame 0.
template <class Step>
__global__ __launch_bounds__(kBlock) void cumulate_kernel(const double* __restrict__ traj,
                                                          int n_frames, int n_bodies, double cx,
                                                          double cy, double* __restrict__ out,
                                                          double* __restrict__ radial)
{
    constexpr int K = Step::K;
    __shared__ double pre[kBlock][K];
    const int b = blockIdx.x;
    const int64_t nint = n_frames - 1;
    const int64_t chunk = (nint + kBlock - 1) / kBlock;
    const int64_t i0 = 1 + chunk * threadIdx.x;
    const int64_t i1 = i0 + chunk < nint + 1 ? i0 + chunk : nint + 1;
    auto pose = [&](int64_t f) { return traj + 7 * ((int64_t)f * n_bodies + b); };
    double s[K];
    for (int k = 0; k < K; ++k) s[k] = 0.0;
    for (int64_t n = i0; n < i1; ++n) {
        double d[K];
        Step::delta(pose(n - 1), pose(n), cx, cy, d);
        for (int k = 0; k < K; ++k) s[k] += d[k];
    }
    for (int k = 0; k < K; ++k) pre[threadIdx.x][k] = s[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        double run[K];
        for (int k = 0; k < K; ++k) run[k] = 0.0;
        for (int t = 0; t < kBlock; ++t)
            for (int k = 0; k < K; ++k) {
                const double v = pre[t][k];
                pre[t][k] = run[k];
                run[k] += v;
            }
    }
    __syncthreads();
    double* ob = out + (int64_t)b * n_frames * K;
    if (threadIdx.x == 0)
        for (int k = 0; k < K; ++k) ob[k] = 0.0;
    double run[K];
    for (int k = 0; k < K; ++k) run[k] = pre[threadIdx.x][k];
    for (int64_t n = i0; n < i1; ++n) {
        double d[K];
        Step::delta(pose(n - 1), pose(n), cx, cy, d);
        for (int k = 0; k < K; ++k) {
            run[k] += d[k];
            ob[n * K + k] = run[k];
        }
    }
    if (radial)
        for (int64_t f = threadIdx.x; f < n_frames; f += kBlock) {
            const double* p = pose(f);
            radial[(int64_t)b * n_frames + f] = hypot(p[0] - cx, p[1] - cy);
        }
}

// ------------------------------------------------------------------ MSDs

// The MSD and rotational MSD kernels: one workgroup per block of kLagBlock consecutive lags
// and per body.  The origins are staged kChunk at a time in LDS together with the frames
// the block's lags reach from them, so each frame is read from memory about twice per block
// instead of twice per (origin, lag).  Thread (l, ph) accumulates lag lag0 + l + 1 over the
// origins t = ph mod 4 in increasing order; the four phases are then added in a fixed order.
constexpr int kLagBlock = 64;
constexpr int kChunk = 256;
constexpr int kPhases = kBlock / kLagBlock;
static_assert(kPhases == 4, "four origin phases per lag");

// stage frames f0 .. f0 + n - 1 of a body-major series (K values per frame) into T; frames
// at or beyond n_frames read as zero
template <int K>
__device__ __forceinline__ void stage(const double* __restrict__ sb, int64_t f0, int n,
                                      int n_frames, double (*T)[K])
{
    for (int e = threadIdx.x; e < n * K; e += kBlock) {
        const int64_t f = f0 + e / K;
        T[e / K][e % K] = f < n_frames ? sb[f * K + e % K] : 0.0;
    }
}

// grid (lag block, body): mean over origins of the squared increment of each component
template <int K>
__global__ __launch_bounds__(kBlock) void msd_kernel(const double* __restrict__ s, int n_frames,
                                                     int n_lags, double* __restrict__ out)
{
    __shared__ double A[kChunk][K];                       // origins t0 ..
    __shared__ double Bt[kChunk + kLagBlock - 1][K];      // frames t0 + lag0 + 1 ..
    __shared__ double part[kPhases][kLagBlock][K];
    const int lag0 = blockIdx.x * kLagBlock, b = blockIdx.y;
    const int l = threadIdx.x % kLagBlock, ph = threadIdx.x / kLagBlock;
    const int tau = lag0 + l + 1;
    const double* sb = s + (int64_t)b * n_frames * K;
    double acc[K];
    for (int k = 0; k < K; ++k) acc[k] = 0.0;
    for (int64_t t0 = 0; t0 + lag0 + 1 < n_frames; t0 += kChunk) {
        __syncthreads();
        stage<K>(sb, t0, kChunk, n_frames, A);
        stage<K>(sb, t0 + lag0 + 1, kChunk + kLagBlock - 1, n_frames, Bt);
        __syncthreads();
        // origins t0 + o with t0 + o + tau < n_frames; a counted loop, unrolled, lets the
        // LDS reads of several origins be in flight together
        const int o_end = (int)min<int64_t>(kChunk, n_frames - tau - t0);
#pragma unroll 8
        for (int o = ph; o < o_end; o += kPhases)
            for (int k = 0; k < K; ++k) {
                const double d = Bt[o + l][k] - A[o][k];
                acc[k] += d * d;
            }
    }
    for (int k = 0; k < K; ++k) part[ph][l][k] = acc[k];
    __syncthreads();
    if (ph == 0 && tau <= n_lags)
        for (int k = 0; k < K; ++k) {
            const double v = (part[0][l][k] + part[1][l][k]) + (part[2][l][k] + part[3][l][k]);
            out[((int64_t)b * n_lags + tau - 1) * K + k] = v / (double)(n_frames - tau);
        }
}

// grid (lag block, body): mean over origins of the squared angle between the reference
// vectors; the unit vectors R(q) r / |R(q) r| are computed once per staged frame
__global__ __launch_bounds__(kBlock) void rotation_msd_kernel(const double* __restrict__ traj,
                                                              int n_frames, int n_bodies,
                                                              const double* __restrict__ ref,
                                                              int n_lags, double* __restrict__ out)
{
    __shared__ double A[kChunk][3];
    __shared__ double Bt[kChunk + kLagBlock - 1][3];
    __shared__ double part[kPhases][kLagBlock];
    const int lag0 = blockIdx.x * kLagBlock, b = blockIdx.y;
    const int l = threadIdx.x % kLagBlock, ph = threadIdx.x / kLagBlock;
    const int tau = lag0 + l + 1;
    const double r[3] = {ref[3 * b], ref[3 * b + 1], ref[3 * b + 2]};
    auto unit = [&](int64_t f, double* p) {
        if (f >= n_frames) { p[0] = p[1] = p[2] = 0.0; return; }
        double R[9];
        rot_of(traj + 7 * (f * n_bodies + b) + 3, R);
        for (int a = 0; a < 3; ++a) p[a] = R[3 * a] * r[0] + R[3 * a + 1] * r[1] + R[3 * a + 2] * r[2];
        const double n = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
        for (int a = 0; a < 3; ++a) p[a] /= n;
    };
    double acc = 0.0;
    for (int64_t t0 = 0; t0 + lag0 + 1 < n_frames; t0 += kChunk) {
        __syncthreads();
        for (int e = threadIdx.x; e < kChunk; e += kBlock) unit(t0 + e, A[e]);
        for (int e = threadIdx.x; e < kChunk + kLagBlock - 1; e += kBlock)
            unit(t0 + lag0 + 1 + e, Bt[e]);
        __syncthreads();
        const int o_end = (int)min<int64_t>(kChunk, n_frames - tau - t0);
#pragma unroll 8
        for (int o = ph; o < o_end; o += kPhases) {
            const double* p0 = A[o];
            const double* p1 = Bt[o + l];
            double c = p0[0] * p1[0] + p0[1] * p1[1] + p0[2] * p1[2];
            c = c > 1.0 ? 1.0 : (c < -1.0 ? -1.0 : c);
            const double th = acos(c);
            acc += th * th;
        }
    }
    part[ph][l] = acc;
    __syncthreads();
    if (ph == 0 && tau <= n_lags)
        out[(int64_t)b * n_lags + tau - 1] =
            ((part[0][l] + part[1][l]) + (part[2][l] + part[3][l])) / (double)(n_frames - tau);
}

// grid (lag, bin), for more than kTileBins bins: sums of the squared increments from the
// origins whose radial coordinate lies in [edges[bin], edges[bin+1]), over all bodies, and
// their count (one workgroup per lag and bin, the bodies added in order)
template <int K>
__global__ __launch_bounds__(kBlock) void binned_msd_kernel(const double* __restrict__ s,
                                                            const double* __restrict__ radial,
                                                            int n_frames, int n_bodies,
                                                            const double* __restrict__ edges,
                                                            int n_lags, double* __restrict__ sums,
                                                            double* __restrict__ counts)
{
    __shared__ double part[4][K + 1];
    const int tau = blockIdx.x + 1, bin = blockIdx.y;
    const double lo = edges[bin], hi = edges[bin + 1];
    double acc[K + 1];
    for (int k = 0; k <= K; ++k) acc[k] = 0.0;
    for (int b = 0; b < n_bodies; ++b) {
        const double* sb = s + (int64_t)b * n_frames * K;
        const double* rb = radial + (int64_t)b * n_frames;
        for (int64_t t = threadIdx.x; t + tau < n_frames; t += kBlock) {
            const double r = rb[t];
            if (!(r >= lo && r < hi)) continue;
            for (int k = 0; k < K; ++k) {
                const double d = sb[(t + tau) * K + k] - sb[t * K + k];
                acc[k] += d * d;
            }
            acc[K] += 1.0;
        }
    }
    block_sum<K + 1>(acc, part);
    if (threadIdx.x == 0) {
        const int64_t o = (int64_t)bin * n_lags + blockIdx.x;
        for (int k = 0; k < K; ++k) sums[o * K + k] = acc[k];
        counts[o] = acc[K];
    }
}

// grid (lag block, body), for at most kTileBins bins: the MSD kernel's staging, with each
// staged origin's bin found once.  The lanes of a wave share their origin (they differ in the
// lag), so the bin is uniform across the wave and only its own sums are updated.  Thread
// (l, ph) keeps every bin's sums for lag lag0 + l + 1 in registers; the four phases are added
// in a fixed order and each body's sums are added to the outputs with device atomics, so the
// order in which bodies are added (and the last bits of the sums) is not fixed; the counts
// are whole numbers and exact.
constexpr int kTileBins = 8;

template <int K>
__global__ __launch_bounds__(kBlock) void binned_msd_tiled_kernel(
    const double* __restrict__ s, const double* __restrict__ radial, int n_frames,
    const double* __restrict__ edges, int n_bins, int n_lags, double* __restrict__ sums,
    double* __restrict__ counts)
{
    __shared__ double A[kChunk][K];
    __shared__ double Bt[kChunk + kLagBlock - 1][K];
    __shared__ int bin_of[kChunk];
    __shared__ double part[kPhases][kLagBlock];
    const int lag0 = blockIdx.x * kLagBlock, b = blockIdx.y;
    const int l = threadIdx.x % kLagBlock, ph = threadIdx.x / kLagBlock;
    const int tau = lag0 + l + 1;
    const double* sb = s + (int64_t)b * n_frames * K;
    const double* rb = radial + (int64_t)b * n_frames;
    double acc[kTileBins][K + 1];
#pragma unroll
    for (int q = 0; q < kTileBins; ++q)
        for (int k = 0; k <= K; ++k) acc[q][k] = 0.0;
    for (int64_t t0 = 0; t0 + lag0 + 1 < n_frames; t0 += kChunk) {
        __syncthreads();
        stage<K>(sb, t0, kChunk, n_frames, A);
        stage<K>(sb, t0 + lag0 + 1, kChunk + kLagBlock - 1, n_frames, Bt);
        for (int e = threadIdx.x; e < kChunk; e += kBlock) {
            int j = -1;
            if (t0 + e < n_frames) {
                const double r = rb[t0 + e];
                for (int q = 0; q < n_bins; ++q)
                    if (r >= edges[q] && r < edges[q + 1]) j = q;
            }
            bin_of[e] = j;
        }
        __syncthreads();
        const int o_end = (int)min<int64_t>(kChunk, n_frames - tau - t0);
#pragma unroll 2
        for (int o = ph; o < o_end; o += kPhases) {
            const int j = __builtin_amdgcn_readfirstlane(bin_of[o]);   // uniform in the wave
            if (j < 0) continue;
            double d2[K];
            for (int k = 0; k < K; ++k) {
                const double d = Bt[o + l][k] - A[o][k];
                d2[k] = d * d;
            }
#pragma unroll
            for (int q = 0; q < kTileBins; ++q)
                if (q == j) {
                    for (int k = 0; k < K; ++k) acc[q][k] += d2[k];
                    acc[q][K] += 1.0;
                }
        }
    }
#pragma unroll
    for (int q = 0; q < kTileBins; ++q) {
        if (q >= n_bins) break;
        for (int k = 0; k <= K; ++k) {
            __syncthreads();
            part[ph][l] = acc[q][k];
            __syncthreads();
            if (ph == 0 && tau <= n_lags) {
                const double v = (part[0][l] + part[1][l]) + (part[2][l] + part[3][l]);
                const int64_t o = (int64_t)q * n_lags + tau - 1;
                if (k < K) atomicAdd(sums + o * K + k, v);
                else atomicAdd(counts + o, v);
            }
        }
    }
}

bool frames_ok(const double* p, int32_t n_frames, int32_t n_bodies)
{
    return p && n_frames >= 1 && n_bodies >= 1 && (int64_t)n_frames * n_bodies * 7 < (int64_t(1) << 40);
}

int launched() { return hipGetLastError() == hipSuccess ? LB_OK : LB_ERR_HIP; }

}  // namespace

void launch_record_poses(const Body* bodies, int n_bodies, double* frame, hipStream_t s)
{
    if (n_bodies <= 0) return;
    hipLaunchKernelGGL(record_kernel, dim3((n_bodies + 255) / 256), dim3(256), 0, s, bodies,
                       n_bodies, frame);
}

}  // namespace lbrb

using namespace lbrb;

extern "C" {

int lb_traj_lab_frame(const double* traj, int32_t n_frames, int32_t n_bodies, double* out,
                        void* stream)
{
    if (!frames_ok(traj, n_frames, n_bodies) || !out) return LB_ERR_ARG;
    hipLaunchKernelGGL((cumulate_kernel<LabStep>), dim3(n_bodies), dim3(kBlock), 0,
                       (hipStream_t)stream, traj, n_frames, n_bodies, 0.0, 0.0, out, nullptr);
    return launched();
}

int lb_traj_body_frame(const double* traj, int32_t n_frames, int32_t n_bodies, double* out,
                         void* stream)
{
    if (!frames_ok(traj, n_frames, n_bodies) || !out) return LB_ERR_ARG;
    hipLaunchKernelGGL((cumulate_kernel<BodyStep>), dim3(n_bodies), dim3(kBlock), 0,
                       (hipStream_t)stream, traj, n_frames, n_bodies, 0.0, 0.0, out, nullptr);
    return launched();
}

int lb_traj_pore_frame(const double* traj, int32_t n_frames, int32_t n_bodies, double cx,
                         double cy, double* out, double* radial, void* stream)
{
    if (!frames_ok(traj, n_frames, n_bodies) || !out || !radial || !std::isfinite(cx) ||
        !std::isfinite(cy))
        return LB_ERR_ARG;
    hipLaunchKernelGGL((cumulate_kernel<PoreStep>), dim3(n_bodies), dim3(kBlock), 0,
                       (hipStream_t)stream, traj, n_frames, n_bodies, cx, cy, out, radial);
    return launched();
}

int lb_traj_msd(const double* series, int32_t n_frames, int32_t n_bodies, int32_t k,
                  int32_t n_lags, double* out, void* stream)
{
    if (!frames_ok(series, n_frames, n_bodies) || !out || k < 1 || k > 6 || n_lags < 1 ||
        n_lags >= n_frames || n_bodies > 65535)
        return LB_ERR_ARG;
    const dim3 grid((n_lags + kLagBlock - 1) / kLagBlock, n_bodies);
    hipStream_t s = (hipStream_t)stream;
    switch (k) {
    case 1: hipLaunchKernelGGL((msd_kernel<1>), grid, dim3(kBlock), 0, s, series, n_frames, n_lags, out); break;
    case 2: hipLaunchKernelGGL((msd_kernel<2>), grid, dim3(kBlock), 0, s, series, n_frames, n_lags, out); break;
    case 3: hipLaunchKernelGGL((msd_kernel<3>), grid, dim3(kBlock), 0, s, series, n_frames, n_lags, out); break;
    case 4: hipLaunchKernelGGL((msd_kernel<4>), grid, dim3(kBlock), 0, s, series, n_frames, n_lags, out); break;
    case 5: hipLaunchKernelGGL((msd_kernel<5>), grid, dim3(kBlock), 0, s, series, n_frames, n_lags, out); break;
    default: hipLaunchKernelGGL((msd_kernel<6>), grid, dim3(kBlock), 0, s, series, n_frames, n_lags, out); break;
    }
    return launched();
}

int lb_traj_rotation_msd(const double* traj, int32_t n_frames, int32_t n_bodies,
                           const double* ref_body, int32_t n_lags, double* out, void* stream)
{
    if (!frames_ok(traj, n_frames, n_bodies) || !ref_body || !out || n_lags < 1 ||
        n_lags >= n_frames || n_bodies > 65535)
        return LB_ERR_ARG;
    hipLaunchKernelGGL(rotation_msd_kernel, dim3((n_lags + kLagBlock - 1) / kLagBlock, n_bodies),
                       dim3(kBlock), 0,
                       (hipStream_t)stream, traj, n_frames, n_bodies, ref_body, n_lags, out);
    return launched();
}

int lb_traj_binned_msd(const double* series, const double* radial, int32_t n_frames,
                         int32_t n_bodies, int32_t k, const double* edges, int32_t n_bins,
                         int32_t n_lags, double* sums, double* counts, void* stream)
{
    if (!frames_ok(series, n_frames, n_bodies) || !radial || !edges || !sums || !counts ||
        k < 1 || k > 3 || n_bins < 1 || n_bins > 65535 || n_lags < 1 || n_lags >= n_frames)
        return LB_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (n_bins <= kTileBins && n_bodies <= 65535) {
        if (hipMemsetAsync(sums, 0, sizeof(double) * k * n_bins * (size_t)n_lags, s) != hipSuccess ||
            hipMemsetAsync(counts, 0, sizeof(double) * n_bins * (size_t)n_lags, s) != hipSuccess)
            return LB_ERR_HIP;
        const dim3 tiles((n_lags + kLagBlock - 1) / kLagBlock, n_bodies);
        switch (k) {
        case 1: hipLaunchKernelGGL((binned_msd_tiled_kernel<1>), tiles, dim3(kBlock), 0, s, series, radial, n_frames, edges, n_bins, n_lags, sums, counts); break;
        case 2: hipLaunchKernelGGL((binned_msd_tiled_kernel<2>), tiles, dim3(kBlock), 0, s, series, radial, n_frames, edges, n_bins, n_lags, sums, counts); break;
        default: hipLaunchKernelGGL((binned_msd_tiled_kernel<3>), tiles, dim3(kBlock), 0, s, series, radial, n_frames, edges, n_bins, n_lags, sums, counts); break;
        }
        return launched();
    }
    const dim3 grid(n_lags, n_bins);
    switch (k) {
    case 1: hipLaunchKernelGGL((binned_msd_kernel<1>), grid, dim3(kBlock), 0, s, series, radial, n_frames, n_bodies, edges, n_lags, sums, counts); break;
    case 2: hipLaunchKernelGGL((binned_msd_kernel<2>), grid, dim3(kBlock), 0, s, series, radial, n_frames, n_bodies, edges, n_lags, sums, counts); break;
    default: hipLaunchKernelGGL((binned_msd_kernel<3>), grid, dim3(kBlock), 0, s, series, radial, n_frames, n_bodies, edges, n_lags, sums, counts); break;
    }
    return launched();
}

}  // extern "C"
