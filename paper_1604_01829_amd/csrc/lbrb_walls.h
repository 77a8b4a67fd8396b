// lbrb_walls.h -- moving walls: the momentum term of halfway bounce-back off a moving
// boundary node.
//
// A fluid node x whose neighbour x - c_i is a boundary node of wall k takes, at the next
// streaming, the reflected population f*_{opp(i)}(x) + 2 w_i rho0 (c_i . u_k) / c_s^2
// (Ladd's moving-wall rule; the walls of the Stokes-flow set-up of Sec. 2.3 move this way).
// The slot f*_{opp(i)}(x) of the post-collision buffer is read by that reflection and by
// nothing else (its regular destination x - c_i is a boundary node), so the term is added to
// the slot once the node update has written it: a list of (node, population, term) links,
// one per fluid node and direction that faces a moving boundary node, applied by one small
// launch after every step and after each (re-)initialisation of the fluid.
#ifndef LBRB_WALLS_H
#define LBRB_WALLS_H

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbrb {

struct WallLink {
    int64_t g;        // global node index of the fluid node
    int32_t pop;      // population slot opp(i) that the reflection reads
    int32_t pad;
    double delta;     // 6 w_i rho0 (c_i . u_k)
};

// f[pop_at(pop, g)] += delta for every link (links are distinct slots: no atomics)
template <typename Real>
void launch_wall_links(Real* f, const WallLink* links, int64_t n_links, hipStream_t s);

// Holes.  A (y,z) row with several fluid runs stores the span from its first to its last fluid
// node, the boundary nodes between the runs ("holes", hole[g] = their wall id) included, so
// the row keeps one descriptor and the pull looks its neighbours up as before.  A fluid node x
// pulls population i from a hole h = x - c_i as if h were fluid; halfway bounce-back needs the
// opposite post-collision population of x itself there, and the slot i of h is read by x and
// by nothing else.  So after each node update (and the moving-wall links, whose term the
// reflected value carries) every hole copies f*_opp(i)(x) into its slot i for each fluid
// neighbour x = h + c_i.  Holes are updated like fluid nodes by the node kernel (their values
// are never read), and every other consumer -- coupling, observables, export -- treats them as
// boundary nodes.  The reverse pass zeroes the holes' adjoints in its node pass and, once a
// reverse step's adjoint is complete, runs the transposed mirror: for each fluid neighbour
// x = h + c_i, slot opp(i) of h takes lambda_i(x); the transposed pull of x along c_opp(i)
// then reads x's own lambda_i there, the transpose of the bounce-back above.
struct ReplicaDesc;
struct RowDesc;
struct NodeTile;
template <typename Real>
void launch_mirror_holes(Real* f, const ReplicaDesc* reps, const RowDesc* rows,
                         const RowDesc* rowinfo, const NodeTile* tiles, int32_t n_tiles,
                         const uint8_t* hole, hipStream_t s);
template <typename Real>
void launch_mirror_holes_transposed(Real* lam, const ReplicaDesc* reps, const RowDesc* rows,
                                    const RowDesc* rowinfo, const NodeTile* tiles, int32_t n_tiles,
                                    const uint8_t* hole, hipStream_t s);

}  // namespace lbrb

#endif
