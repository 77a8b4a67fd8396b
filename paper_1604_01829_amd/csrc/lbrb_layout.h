// lbrb_layout.h -- device data structures of the library and the kernel launchers.
//
// Fluid storage ("compact rows").  Each replica keeps only its fluid nodes.  A (y,z) row of a
// replica stores the span [xlo, xlo+len) from its first to its last fluid node (one run in
// the common case; with several runs the boundary nodes between them are stored as "holes",
// see lbrb_walls.h); the spans of all non-empty rows are stored back to back in (z, y) order,
// so node (x,y,z) of the span of row (y,z) lives at local index start + x - xlo.  rowinfo[row_base + y + ny z] holds
// (start, xlo, len) of every row (len = 0 for a row without fluid), so a neighbour lookup is
// one load; rows[] lists the non-empty rows in storage order for the thread -> node map.  A replica without boundary nodes is
// "dense": every row is full and the local index is x + nx (y + ny z), computed without
// tables.  Populations are blocked structure-of-arrays: the nodes are cut into blocks of 256
// consecutive global indices g (g = replica base + local index; each replica's base is a
// multiple of 256, N = total padded node count), and a block stores its 19 populations one
// after the other, 256 values each: population i of node g sits at
// f[((g / 256) * 19 + i) * 256 + g % 256] (pop_at below).  A workgroup's stores fill one
// contiguous 19 x 256 block, and the loads of a wavefront stay within a few such blocks,
// which keeps the DRAM streams of the 38 population accesses close together.  Two such
// buffers alternate between steps: one holds the post-collision populations of the previous
// step, the kernel pulls from it and writes the next post-collision state into the other.
#ifndef LBRB_LAYOUT_H
#define LBRB_LAYOUT_H

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbrb_core.h"

namespace lbrb {

constexpr int kNodeBlock = 256;   // threads (= nodes) per node-update workgroup
constexpr int kBeadLanes = 8;     // threads per bead in the coupling kernel (one per corner)
constexpr int kCoupleBlock = 256;
constexpr int kPopBlockLog = 8;   // populations are blocked per 256 nodes
constexpr int kLdsPerCu = 160 * 1024;   // LDS bytes of one gfx950 compute unit
constexpr int kWideTiles = 4;     // node tiles per workgroup of the wide node-update launch

// 64-bit fixed-point words of the spread force per node: 3 (FP32) or 6 (FP64) used, padded to
// 32 or 64 bytes so that a node's words share one cache line
template <typename Real>
constexpr int spread_stride() { return sizeof(Real) == 8 ? 8 : 4; }

// index of population i of global node g in a population buffer
__host__ __device__ __forceinline__ int64_t pop_at(int i, int64_t g)
{
    const int64_t blk = g >> kPopBlockLog;
    return ((blk * Q + i) << kPopBlockLog) + (g & ((1 << kPopBlockLog) - 1));
}
// A fluid step is two launches on one stream: the bead coupling, then the node update whose
// leading workgroups finish the bodies (force/torque sums, second half kick).  With m MD
// steps per fluid step, each of the first m - 1 MD steps adds a coupling launch and a body
// launch before them.

// Storage axes.  A masked replica may be stored with its z axis as the row axis ("swapped":
// storage x = box z, storage z = box x, y unchanged), chosen by the mask so that the stored
// rows run along long fluid runs (a pore along z).  nx, ny, nz, the rows and every kernel's
// (x, y, z) are storage coordinates; the populations keep the box's velocity directions, so a
// pull along c_i steps by (c_iz, c_iy, c_ix) in storage coordinates; the noise streams, the
// fields handed out and the bead positions stay in box coordinates.
struct ReplicaDesc {
    int32_t nx, ny, nz, masked;   // 0: no boundary nodes; 1: masked; 2: masked, with holes
    int64_t base;           // global index of local node 0
    int64_t n_nodes;        // nx*ny*nz
    int64_t n_fluid;
    int32_t row_base;       // first entry of this replica in rows[] and rowinfo[]
    uint32_t key0, key1;    // Philox key (seed)
    int32_t swap;           // 1: stored with box axes x and z exchanged (masked replicas only)
    int32_t pad1;
    double inv_nx, inv_ny;  // for exact index division
};

// index of storage node (x, y, z) in the box's own x-fastest order
__host__ __device__ __forceinline__ int64_t box_index(const ReplicaDesc& R, int x, int y, int z)
{
    return R.swap ? z + (int64_t)R.nz * (y + (int64_t)R.ny * x)
                  : x + (int64_t)R.nx * (y + (int64_t)R.ny * z);
}

struct RowDesc {
    int32_t start;          // local index of the first fluid node of the row
    int32_t xlo, len;       // fluid run [xlo, xlo+len); len = 0: no fluid in the row
    int32_t yz;             // y | z << 16
};

struct NodeTile {
    int32_t replica;
    int32_t count;          // nodes in this tile (<= kNodeBlock)
    int64_t begin;          // local index of the first node
    int32_t row_lo, row_hi; // rows[] range that covers the tile (masked replicas)
    int32_t gt;             // global tile: (replica base + begin) / 256
    int32_t pad;
};

struct DeviceHeader {
    int64_t step;           // completed steps (read by graph-replayed kernels)
    uint32_t err_flags;     // bit 0: spread force out of the fixed-point range
    uint32_t pad;
};

template <typename Real>
struct StepArgs {
    const Real* src;        // post-collision populations of the previous step
    Real* dst;              // post-collision populations of this step
    int64_t N;              // stride between populations
    const ReplicaDesc* reps;
    const RowDesc* rows;      // non-empty rows in storage order
    const RowDesc* rowinfo;   // every row, indexed by row_base + y + ny z
    const NodeTile* tiles;
    int32_t n_tiles;
    int32_t tiles_per_wg;   // node tiles per node-update workgroup (1 or kWideTiles)
    int32_t wg_per_cu;      // node-update workgroups resident per CU at most (0: no cap)
    int32_t thermal;
    int32_t narrow;         // every replica of the group spans at most 4 GiB of populations:
                            // 32-bit byte offsets from a per-replica base
    int32_t stream_stores;  // non-temporal population stores (buffers beyond the caches)
    long long* gforce;      // fixed-point spread force, node-major (spread_stride words)
    uint8_t* flags;         // 1 byte per node: spread force present
    const uint8_t* hole;    // 1 byte per node: the wall id of a hole, 0 otherwise
    CollideParams<Real> cp;
    Real gext[3];
    const int64_t* step_ptr;  // if set, step = *step_ptr + step_arg
    int64_t step_arg;
};

// a bead: body-frame offset, the index of its body and its index in the caller's order, read
// in one 32-byte load (a body's beads are stored in spatial order, see rb_add_raspberry)
struct Bead {
    double off[3];
    int32_t body;
    int32_t user;           // index of the bead within its body in the caller's order
};

// What the coupling needs of a bead in the coming step, written when the body's pose of that
// step is known (the body finishing of the previous step, or the pose prediction after a body
// was added or a state loaded), so that the coupling reads one 128-byte record per bead.
struct BeadRec {
    double r[3];            // lab position, unwrapped
    double dv[3];           // r - centre (lab), for the torque
    double v[3];            // bead velocity (0 for a fixed body)
    double gamma, noise_amp;
    int32_t noise_idx;      // bead index within its replica (counter of its noise)
    int32_t row_base;       // replica geometry: rows of the replica, box, storage base, seed
    int32_t nx, ny, nz, masked;
    int64_t base;
    uint32_t key0, key1;
};
static_assert(sizeof(BeadRec) == 128, "bead record is two 64-byte lines");

struct CoupleArgs {
    const BeadRec* recs;
    double* bead_force;         // 3 per bead, lab frame
    double* bead_torque;        // 3 per bead, lab frame
    int32_t n_beads;
    uint32_t md_step;           // MD step within the fluid step (noise counter block)
    double kT;
    double spread_h;            // the fluid receives -spread_h times the bead force
    DeviceHeader* hdr;
};

// Optional timing of one launch: start/stop events recorded by the dispatch itself
// (hipExtLaunchKernel), so their interval is the kernel's own duration.
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};

struct BodyArgs;
// the bead coupling of one MD step; with wca (bodies with excluded volume and wca_ft set) the
// same launch also writes every body's WCA force and torque for that MD step
template <typename Real>
void launch_couple(const StepArgs<Real>& a, const CoupleArgs& c, hipStream_t s,
                   const LaunchEvents& ev = LaunchEvents{}, const BodyArgs* wca = nullptr);
// Excluded volume (WCA).  A body's sites are body-frame offsets sharing one radius; static
// sites (pore beads) are lab positions with a radius each.  Per replica, a coarse cell grid
// (cells at least one interaction range wide) gives each cell one contiguous list of the
// sites in its neighbourhood (itself and the adjacent cells), and a fine flag grid (cells at
// most 2 wide) marks the cells from which some site may be within range.
struct EvSite {
    double off[3];
    double pad;
};
struct WallSite {
    double p[3];
    double radius;
};
struct WcaRep {
    int32_t first_body, n_bodies;   // the replica's bodies: rep_bodies[first_body ...]
    int32_t cx, cy, cz;             // coarse cells per axis (0: no static sites)
    int32_t cell0;                  // first entry of the replica in nb_start
    int32_t gx, gy, gz;             // fine cells per axis
    int32_t fine0;                  // first entry of the replica in near
    double cw[3];                   // coarse cell widths (>= the largest interaction range)
    double fw[3];                   // fine cell widths (<= 2)
};

// Bodies to finish: per-bead forces/torques of the coupling in, the excluded-volume forces of
// the MD step computed here, body records and the bead records of the next MD step out.
struct BodyArgs {
    Body* bodies;
    const Bead* beads;
    BeadRec* recs;
    const double* bead_force;
    const double* bead_torque;
    int32_t n_bodies;
    int32_t substeps;               // MD steps per fluid step
    double wca_eps;
    double* wca_ft;                 // excluded-volume force and torque of the MD step, 6 per
                                    // body (null: no excluded volume)
    const EvSite* ev;
    const WcaRep* wrep;
    const int32_t* rep_bodies;
    const int32_t* nb_start;        // per replica cx*cy*cz + 1 entries into nb_sites
    const WallSite* nb_sites;       // the static sites of each coarse cell's neighbourhood
    const uint8_t* near;            // fine cells: 1 if a site may be within range
};
// the node update of one tile group; with forces the nodes consume the spread force, with
// bodies != null its leading workgroups finish the bodies
template <typename Real>
void launch_node_step(const StepArgs<Real>& a, bool masked, bool forces, const BodyArgs* bodies,
                      hipStream_t s, const LaunchEvents& ev = LaunchEvents{});
// pose of the coming MD step (parity = MD step count & 1) and bead records of every body
void launch_body_predict(const BodyArgs& b, int parity, hipStream_t s);
// finish the bodies after MD step k (< substeps - 1) of the fluid step read from
// step_ptr + step_arg (or step_arg alone when step_ptr is null)
void launch_body_substep(const BodyArgs& b, const int64_t* step_ptr, int64_t step_arg, int k,
                         hipStream_t s);
void launch_set_step(int64_t* step_ptr, int64_t value, hipStream_t s);
template <typename Real>
void launch_init_equilibrium(Real* f, int64_t N, const ReplicaDesc* reps, const NodeTile* tiles,
                             int32_t n_tiles, Real rho0, const double u0[3], hipStream_t s);
// per-replica observables over a tile range: fields (may be null), partial sums (5 doubles per
// tile: drho, jx, jy, jz, nonfinite count), exported FP64 populations (may be null)
template <typename Real>
void launch_observe(const StepArgs<Real>& a, bool masked, int32_t tile0, int32_t n_tiles,
                    Real* fields, double* partials, double* pops_out, hipStream_t s);

// ------------------------------------------------------------------ reverse pass
// Arguments of one reverse step (deterministic fluid).  The forward state of the step is
// pulled from a.src (post-collision populations of the previous step); the spread force of
// the step must have been recomputed into a.gforce / a.flags by the coupling kernel, and the
// bead records must hold the step's bead positions and velocities.
template <typename Real>
struct AdjArgs {
    StepArgs<Real> a;
    const Real* lam_next;       // adjoint of the pre-collision populations of the next step
    Real* lam_cur;              // adjoint of the pre-collision populations of this step
    Real* lamF;                 // adjoint of the node force density, [axis][node]
    const Bead* beads;
    const BeadRec* recs;        // bead records (fixed bodies: the same for every step)
    const double* bead_force;   // bead forces of this step (lab frame)
    const double* weights;      // dJ/dF_b of this step, 3 per body (global body order)
    double* dr;                 // accumulated dJ/d(bead lab position), 3 per bead
    double* dgam;               // accumulated dJ/dgamma, per bead
    double* Jpart;              // accumulated objective, per bead
    int32_t n_beads;
    // With the body passes (body_adj != null: the adjoint of each body's state after the MD
    // step, kBodyAdjWords per body) the bead pass forms the adjoint of the body's force and
    // lab torque from it (force_torque_adjoint), accumulates dr in the body frame of the
    // step's pose (snap[body].pose[pose_par]) and leaves 12 sums per bead in bead_sums for
    // the body pass: the adjoints of the bead position and velocity, the rotation sum
    // d x dbar + (w x d) x vbar and d x vbar (d = r - R, dbar and vbar the adjoints of the
    // arm and the velocity, w the lab angular velocity).  Without, dr is in the lab frame and
    // the body force's adjoint is the weight.
    // The spread force of an MD step is -spread_h times its bead forces (1 / MD steps).
    const double* body_adj;
    const Body* snap;
    int32_t pose_par;
    double* bead_sums;
    double spread_h;
};

// The body pass of one MD step of a reverse step, after its bead and excluded-volume passes.
// in: the bodies before the MD step (its pose at pose[par]); out: after it; adj: the adjoint
// of each body's state after the MD step (kBodyAdjWords doubles: position, quaternion,
// velocity, body-frame angular velocity, force, body-frame torque).  Adds weights . (force
// after the MD step, excluded volume included) into J[b]; for a free body adds the bead sums
// and the excluded-volume pass's adjoint of the pose (wadj, 6 per body: centre, lab angle
// vector; cleared), and takes adj back through the second half kick, the drift, the rotation
// and the first half kick, to the adjoint of the state before the MD step.
constexpr int kBodyAdjWords = 19;
constexpr int kBeadSumWords = 12;
void launch_adjoint_body_post(const Body* in, const Body* out, int par, const double* weights,
                              const double* bead_sums, double* adj, double* wadj, double* J,
                              int n_bodies, hipStream_t s);
// The excluded-volume pass of one MD step of a reverse step: for every WCA pair of a body's
// site (ba.bodies at pose[par]) with a static site or another body's site, the pair force's
// Jacobian takes the adjoint of the force on the first site (Fbar_b + Tbar_b x d, formed from
// the state adjoint adj and the weights) to both sites' positions, and the torque's arm adds
// f x Tbar_b: into wadj of the free bodies involved (atomic adds).  max_ev: the most sites of
// any body.
void launch_adjoint_wca(const BodyArgs& ba, int par, const double* weights, const double* adj,
                        double* wadj, int max_ev, hipStream_t s);
// the pose part of every bead record from its body's pose[par] (the records a step's coupling
// reads), for recomputing the steps of a window
void launch_records_from_poses(const Body* bodies, int par, const Bead* beads, BeadRec* recs,
                               int n_beads, hipStream_t s);

// node pass: transposed streaming + collision VJP (writes lam_cur, lamF, consumes the force)
template <typename Real>
void launch_adjoint_step(const AdjArgs<Real>& A, bool masked, hipStream_t s);
// bead pass: transpose of spreading, friction and interpolation, and of the velocity
// sampling (adds into lam_cur)
template <typename Real>
void launch_adjoint_beads(const AdjArgs<Real>& A, hipStream_t s);
// the bead pass of A in one launch with the coupling (a, c) of the previous forward step
template <typename Real>
void launch_couple_adj_bead(const StepArgs<Real>& a, const CoupleArgs& c, const AdjArgs<Real>& A,
                            hipStream_t s);

}  // namespace lbrb

#endif
