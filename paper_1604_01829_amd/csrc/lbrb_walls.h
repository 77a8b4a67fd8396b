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

}  // namespace lbrb

#endif
