/*
 * lbrb.h -- C-ABI of the MI355X (gfx950) raspberry-colloid / lattice-Boltzmann library.
 *
 * The method is the one of Ustach & Faller, "The Raspberry model for protein-like
 * particles: ellipsoids and confinement in cylindrical pores" (arXiv:1604.01829):
 *   - a lattice-Boltzmann fluid that streams and collides with multiple relaxation times
 *     (Sec. 1.1), here on the D3Q19 lattice, thermal (stochastic) or deterministic (Sec. 1.1),
 *     with bounce-back boundary nodes (Sec. 1.1; the pore wall of Sec. 2.3);
 *   - rigid raspberries: beads that are virtual sites of a centre (Sec. 1.2), each coupled to
 *     the fluid by the frictional force of eq. (latticeboltzmannfriction) with the fluid
 *     velocity interpolated between the nearest nodes and a fluctuation-dissipation noise;
 *     the opposite force goes to the fluid;
 *   - forces and torques of the beads summed onto the centre and turned into the body frame;
 *     velocity Verlet for the centre and a quaternion update for its orientation (Sec. 2.3).
 *
 * Conventions.  Lattice units: spacing 1, time step 1.  Node (x,y,z) of a box of nx*ny*nz
 * nodes sits at (x+1/2, y+1/2, z+1/2); the box is periodic in every direction and boundary
 * nodes (a mask) make walls.  Host arrays are x-fastest.  Quaternions are (w,x,y,z) and
 * rotate body-frame vectors into the lab frame.
 *
 * Memory and streams.  The library never allocates device memory for its state: the caller
 * passes one device workspace of lb_workspace_bytes() bytes (for instance a torch tensor)
 * and a HIP stream; the workspace must outlive the context.  Every call enqueues work on
 * that stream.  lb_observables, lb_save_state, lb_load_state, lb_set_boundary_mask and
 * rb_add_raspberry synchronise the stream before returning; lb_rb_step does not.
 *
 * Errors.  Every call returns LB_OK (0) or a negative code; lb_last_error() gives a message.
 * After LB_ERR_HIP the context should be destroyed; after any other code it stays usable.
 * A context is not thread-safe.
 */
#ifndef LBRB_H
#define LBRB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LB_OK 0
#define LB_ERR_ARG (-1)       /* an argument is out of range or inconsistent              */
#define LB_ERR_STATE (-2)     /* the call is not allowed in the context's current state    */
#define LB_ERR_HIP (-3)       /* a HIP runtime call failed                                  */
#define LB_ERR_UNSTABLE (-4)  /* non-finite populations, or a spread force out of range     */
#define LB_ERR_CAPACITY (-5)  /* more bodies/beads than the context was sized for           */

#define LB_PRECISION_F64 0    /* populations and node arithmetic in FP64                     */
#define LB_PRECISION_F32 1    /* FP32 populations stored as f_i - w_i rho0, FP32 arithmetic  */

typedef struct lb_ctx lb_ctx;

/* One independent box.  seed keys all random numbers of the box (Philox4x32-10).          */
typedef struct {
    int32_t nx, ny, nz;
    uint64_t seed;
} lb_replica;

typedef struct {
    int32_t precision;        /* LB_PRECISION_F64 or LB_PRECISION_F32                      */
    double rho0;              /* rest density (> 0)                                         */
    double u0[3];             /* initial uniform fluid velocity                             */
    double tau_shear;         /* relaxation time of the 5 shear modes (> 1/2)               */
    double tau_bulk;          /* relaxation time of the bulk mode (> 1/2)                   */
    double tau_odd;           /* relaxation time of the 6 odd kinetic modes (> 1/2)         */
    double tau_even;          /* relaxation time of the 3 even kinetic modes (> 1/2)        */
    double kT;                /* thermal energy (>= 0); 0 = deterministic fluid and beads   */
    double g_ext[3];          /* force density on every fluid node (not on bodies)          */
    int32_t max_bodies;       /* capacity over all replicas                                 */
    int32_t max_beads;        /* capacity over all replicas                                 */
    int32_t max_wall_links;   /* capacity for moving walls (lb_set_wall_velocity): links
                                 between a fluid node and a moving boundary node, over all
                                 replicas (0 = walls at rest only)                           */
    int32_t md_substeps;      /* MD steps per fluid step (0 or 1: one; the paper uses 2,
                                 Sec. 2.3): each is a velocity-Verlet step of the bodies of
                                 length 1/md_substeps on the frozen fluid, with bead noise of
                                 its own; the fluid receives the MD steps' mean coupling force */
    double wca_epsilon;       /* WCA energy of the excluded volume (Sec. 2.3: kT); 0 = none  */
    int32_t max_ev_sites;     /* capacity: excluded-volume sites over all bodies             */
    int32_t max_wall_sites;   /* capacity: static WCA sites (pore beads) over all replicas   */
} lb_params;

/* Device bytes needed for these parameters and boxes (upper bound, all nodes fluid).
 * Returns 0 if the arguments are invalid.                                                 */
size_t lb_workspace_bytes(const lb_params* params, const lb_replica* replicas,
                          int32_t n_replicas);

/* Create a context.  Lays out the workspace, fills every fluid node with the equilibrium
 * of (rho0, u0) just before a streaming step, and returns the context in *out.
 * dev_workspace: device pointer, 256-byte aligned, ws_bytes >= lb_workspace_bytes().
 * hip_stream: a hipStream_t (NULL = the null stream).                                      */
int lb_init(const lb_params* params, const lb_replica* replicas, int32_t n_replicas,
            void* dev_workspace, size_t ws_bytes, void* hip_stream, lb_ctx** out);

/* Boundary nodes of one replica (the bounce-back rule of Sec. 1.1; the pore wall nodes of
 * Sec. 2.3).  host_mask: nx*ny*nz bytes, x fastest, 0 = fluid node, k = 1..255 = boundary
 * node of wall k (walls are at rest unless lb_set_wall_velocity moves them); copied.
 * Any arrangement of boundary nodes is accepted (obstacles, several pores, porous media).
 * Storage is per (y,z) row from its first to its last fluid node: rows with one fluid run
 * (pores along z, slabs, channels) store fluid nodes only; rows with several runs also store
 * the boundary nodes between the runs, which then cost one node update each and a mirror of
 * their fluid neighbours' reflected populations after every step.  Only before the first step
 * (LB_ERR_STATE otherwise).  Re-initialises that replica's fluid to equilibrium.            */
int lb_set_boundary_mask(lb_ctx* ctx, int32_t replica, const uint8_t* host_mask);

/* Velocity u[3] (lab frame) of wall `wall` (1..255) of one replica: the walls of the
 * Stokes-flow resistance set-up of Sec. 2.3 (eq. (stokesflow)), e.g. the +-y faces of a box.
 * Halfway bounce-back off a moving wall adds 2 w_i rho0 (c_i . u) / c_s^2 to each reflected
 * population (Ladd's moving-wall rule).  Only before the first step (LB_ERR_STATE
 * otherwise); re-initialises that replica's fluid (equilibrium of (rho0, u0) streamed with
 * the moving walls).  LB_ERR_ARG for a bad replica or wall id, LB_ERR_CAPACITY when the
 * links between fluid nodes and moving boundary nodes exceed max_wall_links.             */
int lb_set_wall_velocity(lb_ctx* ctx, int32_t replica, int32_t wall, const double u[3]);

/* Add a raspberry (Sec. 1.2) to a replica.  bead_offsets_body: n_beads*3 body-frame bead
 * positions relative to the centre (a centre bead is just an offset (0,0,0)); mass and
 * principal moments of inertia (ignored when fixed); centre position (lab, unwrapped),
 * orientation quaternion (w,x,y,z; normalised here), lab velocity, body-frame angular
 * velocity; gamma = bead friction of eq. (latticeboltzmannfriction); fixed != 0 holds the
 * body still (its beads have zero velocity, forces are still measured).  All host arrays
 * are copied.  *body_id receives the body's index within its replica.  Bodies may be added
 * at any step; a new body starts with zero force and torque.                              */
int rb_add_raspberry(lb_ctx* ctx, int32_t replica, const double* bead_offsets_body,
                     int32_t n_beads, double mass, const double inertia_body[3],
                     const double pos[3], const double quat_wxyz[4], const double vel[3],
                     const double omega_body[3], double gamma, int32_t fixed,
                     int32_t* body_id);

/* Advance every replica by n_steps time steps (n_steps >= 0).  Each step: half kick and
 * drift of free bodies, bead coupling and force spreading, per-body force/torque sums and
 * the second half kick, then the fused collide-and-stream update of every fluid node.
 * Asynchronous on the context's stream.                                                    */
int lb_rb_step(lb_ctx* ctx, int32_t n_steps);

typedef struct {
    double mass;              /* sum of rho over the replica's fluid nodes (FP64 sum)       */
    double momentum[3];       /* sum of j = sum_i c_i f_i over the fluid nodes              */
    double body_momentum[3];  /* sum of M V over the replica's free bodies                  */
    int64_t step;             /* number of completed steps                                  */
    int32_t finite;           /* 1 if every node's rho and j are finite                     */
} lb_totals;

typedef struct {
    double pos[3];            /* centre, lab frame, unwrapped                               */
    double quat[4];           /* (w,x,y,z)                                                  */
    double vel[3];            /* lab frame                                                  */
    double omega_body[3];     /* body frame                                                 */
    double force[3];          /* sum of bead forces of the last step, lab frame            */
    double torque[3];         /* sum of bead torques of the last step, body frame          */
} rb_state;

/* Observables of one replica after the last completed step (synchronises the stream).
 * out: totals (may be NULL).  bodies: host array of at least (bodies in the replica)
 * records, in the order they were added (may be NULL).  dev_rho_u: device array of
 * 4*nx*ny*nz values of the context precision, node-major (rho, ux, uy, uz) with
 * u = (j + g_ext/2)/rho; boundary nodes get zeros (may be NULL).
 * Returns LB_ERR_UNSTABLE (after filling the outputs) if a population is non-finite or a
 * spread force left the fixed-point range.                                                 */
int lb_observables(lb_ctx* ctx, int32_t replica, lb_totals* out, rb_state* bodies,
                   void* dev_rho_u);

/* Excluded volume of a body (the inner layer of a two-layer raspberry, Sec. 2.1): n_sites
 * body-frame offsets (n_sites*3, host) of sites that take no part in the fluid coupling and
 * repel the static sites of the replica and the sites of its other bodies with the WCA pair
 * potential 4 eps ((s/r)^12 - (s/r)^6) + eps below r = 2^(1/6) s, s = sum of the two radii,
 * eps = wca_epsilon (Sec. 2.3), minimum image in every direction; their forces and torques
 * join the body's.  radius: the sites' Lennard-Jones radius (Sec. 2.1: 0.5).  Replaces
 * earlier sites of the body; n_sites = 0 removes them.  Only before the first step
 * (LB_ERR_STATE); LB_ERR_ARG for bad ids or values, LB_ERR_CAPACITY beyond max_ev_sites.
 * The first lb_rb_step returns LB_ERR_ARG if a box side is shorter than twice the largest
 * interaction range of its replica.                                                        */
int rb_set_excluded_volume(lb_ctx* ctx, int32_t replica, int32_t body_id,
                           const double* offsets_body, int32_t n_sites, double radius);

/* Static WCA sites of one replica (the pore beads of Sec. 2.3): n lab positions (n*3, host)
 * with one Lennard-Jones radius (the paper: 6.25), appended to the replica's sites.  Only
 * before the first step (LB_ERR_STATE); LB_ERR_ARG for bad values, LB_ERR_CAPACITY beyond
 * max_wall_sites.                                                                          */
int lb_add_wall_sites(lb_ctx* ctx, int32_t replica, const double* positions, int32_t n,
                      double radius);

/* ---- trajectory analysis (Sec. 2.4-2.8) ----
 * A trajectory is a device array traj[n_frames][n_bodies][7]: the centre (x, y, z; lab frame,
 * unwrapped) and unit quaternion (w, x, y, z) of every body at every recording.  Series are
 * device arrays stored body-major, series[n_bodies][n_frames][k].  These functions take no
 * context: they launch on `stream` (a hipStream_t; NULL = the default stream) and return
 * LB_OK, LB_ERR_ARG (null pointers, sizes out of range) or LB_ERR_HIP (launch failure)
 * without synchronising.
 *
 * rb_record_poses: every body's centre and quaternion after the last completed step into
 * dev_frame (n_bodies*7 doubles; bodies in the order they were added over all replicas),
 * asynchronously on the context's stream.                                                  */
int rb_record_poses(lb_ctx* ctx, double* dev_frame);

/* Cumulative series, 0 at frame 0.  lab (k = 3): the centre minus its first position.
 * body frame (k = 6): the body-frame displacement (Sec. 2.6: each interval's lab
 * displacement turned into the body frame with the orientation at the start of the
 * interval, summed) and the body-frame rotation angles about x^b, y^b, z^b (Sec. 2.7 and its
 * SI: the body axes at t projected onto the planes normal to the axes at t-1, angles by
 * arctan, summed).  pore frame (k = 3): the displacement rotated by minus the polar angle of
 * the centre about the axis through (cx, cy) parallel to z at the start of each interval
 * (x^p radial, y^p tangential, z^p axial; Sec. 2.8 and its SI), summed; radial[n_bodies]
 * [n_frames] receives each frame's distance from that axis.                                */
int lb_traj_lab_frame(const double* traj, int32_t n_frames, int32_t n_bodies, double* out,
                        void* stream);
int lb_traj_body_frame(const double* traj, int32_t n_frames, int32_t n_bodies, double* out,
                         void* stream);
int lb_traj_pore_frame(const double* traj, int32_t n_frames, int32_t n_bodies, double cx,
                         double cy, double* out, double* radial, void* stream);

/* Mean squared displacement over all time origins for lags 1..n_lags (< n_frames), per body
 * and component: out[n_bodies][n_lags][k], k = 1..6 (eqs. (dt_lab), (dt_body), (dr_body)). */
int lb_traj_msd(const double* series, int32_t n_frames, int32_t n_bodies, int32_t k,
                  int32_t n_lags, double* out, void* stream);

/* Lab-frame rotational MSD (eqs. (dr_lab), (delta_theta)): the mean over origins of
 * arccos(p^(t) . p^(t+tau))^2 for p = R(q) ref, ref_body[n_bodies][3] (device) the body-frame
 * vector from the centre to each body's reference bead: out[n_bodies][n_lags].             */
int lb_traj_rotation_msd(const double* traj, int32_t n_frames, int32_t n_bodies,
                           const double* ref_body, int32_t n_lags, double* out, void* stream);

/* Radially binned MSD (Sec. 2.8): every origin frame t of every body whose radial[b][t]
 * lies in [edges[j], edges[j+1]) (edges: device, n_bins+1 ascending) adds its squared
 * increments over lags 1..n_lags of series (k = 1..3) to sums[n_bins][n_lags][k] and 1 to
 * counts[n_bins][n_lags] (both overwritten).  With at most 8 bins each body's sums are added
 * to the outputs by device atomics, so the order of the bodies in the sums (their last bits)
 * may differ between calls; the counts are exact.  With more bins the bodies are added in
 * order.                                                                                  */
int lb_traj_binned_msd(const double* series, const double* radial, int32_t n_frames,
                         int32_t n_bodies, int32_t k, const double* edges, int32_t n_bins,
                         int32_t n_lags, double* sums, double* counts, void* stream);

/* ---- raspberry construction (Sec. 2.1 and its SI "Details for ellipsoidal raspberry
 * construction") ----
 * rb_relax_shells: n_steps of damped MD for n_shells bead shells at once.  Within a shell the
 * beads repel with the WCA pair potential (sigma, epsilon; cut at 2^(1/6) sigma) and each is
 * held to the closest point r_s of its shell's ellipsoid (semi-axes axes[s][0..2] along the
 * body x, y, z) by U = k_surface |r - r_s|^2; r_s = x a^2 / (t + a^2) per axis with t the
 * root of F(t) = sum (x a / (t + a^2))^2 - 1 on (-min a^2, inf) (bracketed Newton, to the
 * rounding noise of F).  Each bead's pair forces are summed over a pair list in index order,
 * the same terms in the same order as over all beads.  Integration: v <- ((1 - g) v + dt F / mass) / (1 + g), g = damping dt / 2, then
 * r <- r + dt v (the paper's script: leapfrog, damping 1000, dt 0.001, sigma 1.4,
 * epsilon 0.1).  axes (n_shells*3) and counts (n_shells, each 1..2048) are host arrays; the
 * shells' beads are packed one after another in the device arrays dev_pos and dev_vel
 * ([total beads][3], body frame, in/out; dev_vel holds the velocities of the half step
 * before, zeros to start).  Asynchronous on `stream`; LB_ERR_ARG for bad arguments.        */
typedef struct {
    double k_surface;   /* restraint stiffness k                                           */
    double sigma;       /* WCA size                                                         */
    double epsilon;     /* WCA energy                                                       */
    double damping;     /* friction rate                                                    */
    double dt;          /* time step                                                        */
    double mass;        /* bead mass                                                        */
} rb_relax_params;
int rb_relax_shells(int32_t n_shells, const double* axes, const int32_t* counts,
                    double* dev_pos, double* dev_vel, const rb_relax_params* params,
                    int32_t n_steps, void* stream);

/* Number of bodies in a replica, and the per-bead forces (lab frame, FP64, n_beads*3, in
 * the order the beads were given) of the last step of one body, copied to host memory.   */
int lb_body_count(const lb_ctx* ctx, int32_t replica);
int rb_bead_forces(lb_ctx* ctx, int32_t replica, int32_t body_id, double* host_out,
                   int32_t n_beads);

/* The pre-collision populations f_i (not shifted) of one replica as FP64, [i][z][y][x]
 * (19*nx*ny*nz values, zeros on boundary nodes), into a device array.                    */
int lb_export_populations(lb_ctx* ctx, int32_t replica, double* dev_out);

/* Fault injection, for tests of the failure detection (an aid of the library, not a step of
 * the method): population i (0..18) of the fluid node (x, y, z) of one replica, in the current
 * state, becomes a quiet NaN.  The NaN spreads with the next steps, lb_observables then
 * returns LB_ERR_UNSTABLE, and lb_load_state of an earlier checkpoint recovers the run.
 * Synchronises the stream.  LB_ERR_ARG for a node outside the box, a boundary node or i out
 * of range.                                                                                */
int lb_inject_nan(lb_ctx* ctx, int32_t replica, int32_t x, int32_t y, int32_t z, int32_t i);

/* Checkpointing: the complete dynamic state (populations, bodies, step) in bytes that a
 * later lb_load_state of a context with the same parameters, boxes, masks, wall velocities
 * and bodies restores bit for bit (and clears a spread-force overflow reported since, which
 * belongs to the run it replaces).  dev_buf may be NULL to query the size: *bytes receives
 * it.                                                                                      */
int lb_save_state(lb_ctx* ctx, void* dev_buf, size_t* bytes);
int lb_load_state(lb_ctx* ctx, const void* dev_buf, size_t bytes);

/* Execution options.  graph_steps: lb_rb_step replays a HIP graph of this many steps
 * (even, >= 2) and runs the remainder eagerly; 0 = always eager (default 100).
 * timing: when nonzero, every node-update and coupling launch carries a start and a stop
 * HIP event recorded by its dispatch (hipExtLaunchKernel; eager launches only, graphs are
 * not replayed while timing) and lb_kernel_times reports the summed kernel durations (ms)
 * and launch counts since timing was enabled.                                            */
int lb_set_graph_steps(lb_ctx* ctx, int32_t graph_steps);
int lb_set_timing(lb_ctx* ctx, int32_t enable);
int lb_kernel_times(lb_ctx* ctx, double* node_ms, int64_t* node_launches, double* couple_ms,
                    int64_t* couple_launches);

/* How the node update stores the populations.  LB_STORES_STREAMING: non-temporal stores,
 * which bypass the caches -- faster (3-5 % on MI355X) once the two population buffers are far
 * larger than the 256 MB Infinity Cache, much slower (about 25 %) when they fit in it.
 * LB_STORES_CACHED: ordinary stores.  LB_STORES_AUTO (default): the choice of lb_autotune
 * once it has run on this context, else streaming when the populations of the fluid nodes, in
 * both buffers, exceed 256 MiB.                                                            */
#define LB_STORES_AUTO 0
#define LB_STORES_CACHED 1
#define LB_STORES_STREAMING 2
int lb_set_store_policy(lb_ctx* ctx, int32_t policy);

/* Launch settings of the node update, chosen by timing (not in the paper: a property of the
 * GPU).  lb_autotune times the context's own node kernel over its own tiles for every
 * combination of node tiles per workgroup (1 or 4; 256 nodes each), a cap on the node
 * workgroups resident per compute unit (none, 6, 5, 4; by dynamic LDS) and the store kind
 * (ordinary or non-temporal when both population buffers exceed the 256 MB Infinity Cache;
 * ordinary stores only when they fit in it, where the timed launches, which re-read an
 * unchanged buffer, cannot see what non-temporal stores cost the next step's reads; only the
 * forced kind under LB_STORES_CACHED/STREAMING): 16 or 8 settings.  It keeps the fastest
 * for the following steps if it beats the untuned settings by at least
 * 1 % (else the untuned ones).  The timed launches leave the simulation state
 * unchanged (no spread force is consumed, no body is finished; they write the buffer the next
 * step overwrites).  Results are kept for the process per (GPU architecture, precision,
 * thermal, tile counts, fluid nodes, store policy): repeats = 0 takes a kept result when there
 * is one and otherwise times 3 launches per setting; repeats > 0 always times that many and
 * replaces the kept result.  Synchronises the stream.  LB_ERR_ARG for repeats outside
 * 0..1000.  The choice changes no result, only speed.                                       */
typedef struct {
    int32_t tuned;            /* 1 once lb_autotune has run on this context                 */
    int32_t tiles_per_wg;     /* node tiles (256 nodes) per node-update workgroup           */
    int32_t wg_per_cu;        /* cap on node-update workgroups per compute unit (0: none)   */
    int32_t streaming;        /* 1: non-temporal population stores in use                   */
    int32_t candidates;       /* settings timed                                             */
    double node_us_default;   /* one node update of every tile with the untuned settings, us */
    double node_us_tuned;     /* the same with the chosen settings, us                      */
} lb_tuning;
int lb_autotune(lb_ctx* ctx, int32_t repeats);
int lb_get_tuning(const lb_ctx* ctx, lb_tuning* out);
/* Apply settings directly (for instance ones kept from an earlier process): tiles_per_wg
 * 1 or 4, wg_per_cu 0..32, streaming 0/1 (used while the store policy is LB_STORES_AUTO); the
 * other fields are ignored.  LB_ERR_ARG outside those ranges.                               */
int lb_set_tuning(lb_ctx* ctx, const lb_tuning* settings);

/* Reverse-mode derivative of a window of steps (not in the paper: the hand adjoint of the
 * coupled update of Sec. 1.1-1.2 -- streaming with bounce-back, the mode-space collision
 * with its force source, the frictional coupling of eq. (latticeboltzmannfriction) with its
 * interpolated fluid velocity, and the opposite force spread onto the fluid).
 * Objective J = sum_n sum_b a(n,b) . F_b(n) over the next n_steps steps, F_b(n) the summed
 * bead force on body b in step n (a = (1/T,0,0) for every step: time-averaged drag along x).
 * Derivatives with respect to every body's friction gamma and every bead's body-frame
 * offset, holding the window's initial state fixed (populations, body states, and the force
 * and torque of the step before the window).  Bodies may be fixed or free: for a free body
 * the derivative runs through the rigid-body integrator of Sec. 2.3 as well (both half
 * kicks, the drift, the quaternion rotation and the moving bead positions and velocities),
 * which adds a few hundred bytes per body and step to the workspace.  With several MD steps
 * per fluid step (Sec. 2.3), F_b(n) is the force of the fluid step's last MD step (the body
 * force lb_observables reports) and every MD step is differentiated.  WCA excluded volume
 * (Sec. 2.1 inner layers, Sec. 2.3 pore beads) is differentiated through its pair forces,
 * and its force on a body counts in F_b(n).  With kT > 0 the derivative is pathwise: the
 * recomputed steps draw the forward run's counter-based noise, and the bead noise amplitude
 * sqrt(2 kT gamma / dt) is differentiated in gamma (the fluid's noise is additive and leaves
 * the collision's Jacobian unchanged).
 * The call advances the context by n_steps steps (its state afterwards is that of
 * lb_rb_step(n_steps)), keeping the post-collision state every checkpoint_every steps in the
 * caller's device workspace dev_ws (256-byte aligned, at least
 * lb_adjoint_workspace_bytes(ctx, n_steps, checkpoint_every) bytes), then walks the window
 * backwards one segment at a time, recomputing each segment's states from its checkpoint.
 * Host arrays, global body and bead order (the order of the rb_add_raspberry calls over
 * all replicas):
 *   dJ_dF       [n_steps][n_bodies][3]  the weights a(n,b), lab frame;
 *   J           the objective (may be NULL);
 *   dJ_dgamma   [n_bodies];
 *   dJ_doffsets [n_beads][3], body frame.
 * Synchronises the stream.  Errors: LB_ERR_ARG (window, workspace, missing arrays),
 * or the excluded-volume table errors of lb_rb_step.  The adjoint runs in the context precision; its
 * atomic accumulation of sampled-velocity adjoints into the population adjoint is not
 * order-deterministic.                                                                    */
size_t lb_adjoint_workspace_bytes(const lb_ctx* ctx, int32_t n_steps, int32_t checkpoint_every);
int lb_rb_adjoint(lb_ctx* ctx, int32_t n_steps, int32_t checkpoint_every, void* dev_ws,
                  size_t ws_bytes, const double* dJ_dF, double* J, double* dJ_dgamma,
                  double* dJ_doffsets);

/* The reverse pass of lb_rb_adjoint without a caller workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  It runs on a scratch array of LB_NOALLOC_SCRATCH_BYTES (64 MiB) that
 * the library holds on every GPU it runs on until the process ends, and calls no allocating
 * routine; arguments and results as for lb_rb_adjoint.  LB_ERR_ARG when the window needs more
 * than LB_NOALLOC_SCRATCH_BYTES (lb_adjoint_workspace_bytes tells; a longer checkpoint
 * interval needs less), LB_ERR_HIP when the scratch array's address cannot be taken.  Every
 * call on one GPU uses that GPU's array (the parts that must start at zero are cleared by
 * each call), so calls that overlap on one GPU race.                                       */
#define LB_NOALLOC_SCRATCH_BYTES (64 * 1024 * 1024)
int lb_rb_adjoint_noalloc(lb_ctx* ctx, int32_t n_steps, int32_t checkpoint_every,
                          const double* dJ_dF, double* J, double* dJ_dgamma,
                          double* dJ_doffsets);

/* Node counts of one replica: all nodes and fluid nodes.                                  */
int lb_node_counts(const lb_ctx* ctx, int32_t replica, int64_t* n_nodes, int64_t* n_fluid);

/* Storage axis of a replica's rows (a layout choice of the library, not of the method):
 * *axis = 0 when the fluid is stored in rows along x, 2 when lb_set_boundary_mask chose rows
 * along z (the box's axes x and z exchanged in storage) because the mask's x rows are short
 * (under 48 stored nodes on average) and its fluid runs much longer along z, as in a narrow
 * pore along z.  Results do not depend on it; fields,
 * populations and positions are always in the box's own coordinates.  LB_ERR_ARG for a bad
 * replica or a NULL output.                                                                */
int lb_row_axis(const lb_ctx* ctx, int32_t replica, int32_t* axis);

void lb_destroy(lb_ctx* ctx);
const char* lb_last_error(const lb_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
