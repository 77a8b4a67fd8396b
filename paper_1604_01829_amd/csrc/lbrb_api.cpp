// lbrb_api.cpp -- host side of the C-ABI declared in include/lbrb.h.
//
// Owns the layout of the caller's workspace, the compact fluid-row tables built from the
// boundary masks, the tile lists of the launches, the body/bead tables, the HIP-graph replay
// of many steps and the per-kernel event timing.  Every step runs on the caller's stream;
// graphs are captured on a private stream (default priority) and replayed on the caller's.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstddef>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/lbrb.h"
#include "lbrb_layout.h"
#include "lbrb_plan.h"
#include "lbrb_walls.h"
#include "lbrb_analysis.h"

using namespace lbrb;

namespace lbrb {
void noalloc_prepare();   // lbrb_noalloc.hip: the scratch array's address on this device
}

namespace {

constexpr size_t kAlign = 256;
// MI355X's Infinity Cache: population buffers beyond it are stored with non-temporal stores
constexpr double kInfinityCacheBytes = 256.0 * 1024 * 1024;
constexpr uint64_t kStateMagic = 0x4C42524253544154ull;  // "LBRBSTAT"

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// roctx range on the calling thread for the lifetime of the object (seen by rocprofv3
// --marker-trace; a no-op without a profiler)
struct Marker {
    explicit Marker(const char* msg) { roctxRangePushA(msg); }
    ~Marker() { roctxRangePop(); }
    Marker(const Marker&) = delete;
    Marker& operator=(const Marker&) = delete;
};

struct Plan {
    int64_t N = 0;            // padded total node count (stride between populations)
    int64_t rows_cap = 0;     // sum of ny*nz
    int64_t tiles_cap = 0;    // sum of ceil(nodes / 256)
    int64_t bead_cap = 0, body_cap = 0;
    int64_t link_cap = 0;     // moving-wall links
    int64_t ev_cap = 0, site_cap = 0, cells_cap = 0, fine_cap = 0;   // excluded volume
    int gforce_words = 4;     // fixed-point words per node: 3 axes x (1 in FP32, 2 in FP64),
                              // padded to 4 (32 bytes) or 8 (64 bytes)
    size_t off_hdr, off_reps, off_rows, off_rowinfo, off_tiles_d, off_tiles_m, off_fa, off_fb,
        off_gforce, off_flags, off_hole, off_hole_tiles, off_bodies, off_bead_off, off_bead_rec, off_bead_force,
        off_bead_torque, off_partials, off_links, off_ev, off_wrep, off_rep_bodies,
        off_nb_start, off_nb_sites, off_near, off_wca_ft, total;
};

bool valid_params(const lb_params* p)
{
    if (!p) return false;
    if (p->precision != LB_PRECISION_F64 && p->precision != LB_PRECISION_F32) return false;
    if (!(p->rho0 > 0) || !std::isfinite(p->rho0)) return false;
    const double taus[4] = {p->tau_shear, p->tau_bulk, p->tau_odd, p->tau_even};
    for (double t : taus)
        if (!(t > 0.5) || !std::isfinite(t)) return false;
    if (!(p->kT >= 0) || !std::isfinite(p->kT)) return false;
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(p->u0[a]) || !std::isfinite(p->g_ext[a])) return false;
    if (p->max_bodies < 0 || p->max_beads < 0 || p->max_wall_links < 0) return false;
    if (p->md_substeps < 0 || p->md_substeps > 64) return false;
    if (!(p->wca_epsilon >= 0) || !std::isfinite(p->wca_epsilon)) return false;
    if (p->max_ev_sites < 0 || p->max_wall_sites < 0) return false;
    return true;
}

bool make_plan(const lb_params* p, const lb_replica* reps, int32_t n, Plan& pl)
{
    if (!valid_params(p) || !reps || n < 1) return false;
    pl = Plan();
    for (int r = 0; r < n; ++r) {
        const lb_replica& R = reps[r];
        if (R.nx < 1 || R.ny < 1 || R.nz < 1 || R.nx > 32767 || R.ny > 65535 || R.nz > 32767)
            return false;
        const int64_t nodes = (int64_t)R.nx * R.ny * R.nz;
        if (nodes >= (int64_t(1) << 31)) return false;
        pl.N += pad_nodes(nodes);
        // rows of either storage orientation (rows along x or, exchanged, along z)
        pl.rows_cap += (int64_t)R.ny * std::max(R.nx, R.nz);
        pl.tiles_cap += pad_nodes(nodes) / kNodeBlock;
        if (p->max_wall_sites > 0) {
            pl.cells_cap += (int64_t)cells_per_axis_cap(R.nx) * cells_per_axis_cap(R.ny) *
                            cells_per_axis_cap(R.nz) + 1;
            pl.fine_cap += (int64_t)fine_per_axis(R.nx) * fine_per_axis(R.ny) * fine_per_axis(R.nz);
        }
    }
    const size_t real = p->precision == LB_PRECISION_F32 ? sizeof(float) : sizeof(double);
    pl.body_cap = p->max_bodies;
    pl.bead_cap = p->max_beads;
    pl.link_cap = p->max_wall_links;
    pl.ev_cap = p->max_ev_sites;
    pl.site_cap = p->max_wall_sites;
    size_t o = 0;
    auto take = [&](size_t bytes) { const size_t at = o; o = align_up(o + bytes, kAlign); return at; };
    pl.off_hdr = take(sizeof(DeviceHeader));
    pl.off_reps = take(sizeof(ReplicaDesc) * n);
    pl.off_rows = take(sizeof(RowDesc) * pl.rows_cap);
    pl.off_rowinfo = take(sizeof(RowDesc) * pl.rows_cap);
    pl.off_tiles_d = take(sizeof(NodeTile) * pl.tiles_cap);
    pl.off_tiles_m = take(sizeof(NodeTile) * pl.tiles_cap);
    pl.off_fa = take(real * Q * pl.N);
    pl.off_fb = take(real * Q * pl.N);
    pl.gforce_words = p->precision == LB_PRECISION_F32 ? spread_stride<float>()
                                                       : spread_stride<double>();
    pl.off_gforce = take(sizeof(long long) * pl.gforce_words * pl.N);
    pl.off_flags = take(pl.N);
    pl.off_hole = take(pl.N);
    pl.off_hole_tiles = take(sizeof(NodeTile) * pl.tiles_cap);
    pl.off_bodies = take(sizeof(Body) * std::max<int64_t>(pl.body_cap, 1));
    pl.off_bead_off = take(sizeof(Bead) * std::max<int64_t>(pl.bead_cap, 1));
    pl.off_bead_rec = take(sizeof(BeadRec) * std::max<int64_t>(pl.bead_cap, 1));
    pl.off_bead_force = take(sizeof(double) * 3 * std::max<int64_t>(pl.bead_cap, 1));
    pl.off_bead_torque = take(sizeof(double) * 3 * std::max<int64_t>(pl.bead_cap, 1));
    pl.off_partials = take(sizeof(double) * 5 * pl.tiles_cap);
    pl.off_links = take(sizeof(WallLink) * std::max<int64_t>(pl.link_cap, 1));
    pl.off_ev = take(sizeof(EvSite) * std::max<int64_t>(pl.ev_cap, 1));
    pl.off_wrep = take(sizeof(WcaRep) * n);
    pl.off_rep_bodies = take(sizeof(int32_t) * std::max<int64_t>(pl.body_cap, 1));
    pl.off_nb_start = take(sizeof(int32_t) * std::max<int64_t>(pl.cells_cap, 1));
    // a site appears in the neighbourhood lists of at most 27 coarse cells
    pl.off_nb_sites = take(sizeof(WallSite) * 27 * std::max<int64_t>(pl.site_cap, 1));
    pl.off_near = take(std::max<int64_t>(pl.fine_cap, 1));
    pl.off_wca_ft = take(sizeof(double) * 6 * std::max<int64_t>(pl.body_cap, 1));
    pl.total = o;
    return true;
}

struct ReplicaHost {
    int group = 0;            // 0 = dense tiles, 1 = masked tiles
    int64_t n_holes = 0;      // boundary nodes stored inside row spans (lbrb_walls.h)
    int32_t tile0 = 0, n_tiles = 0;
    std::vector<int32_t> bodies;
    std::vector<uint8_t> mask;      // boundary mask as set (wall ids), empty = all fluid
    std::vector<double> uwall;      // 3 per wall id 0..255 once a wall velocity was set
    std::vector<WallLink> links;    // moving-wall links of this replica
    int64_t link0 = 0;              // their first entry in the device list
    std::vector<WallSite> sites;    // static WCA sites
};

struct EvHost {
    std::vector<double> off;        // body-frame offsets of the excluded-volume sites
    double radius = 0.0;
};

struct EventPair { hipEvent_t a, b; };

// Node-update launch settings chosen by lb_autotune (defaults until then)
struct Tuning {
    bool tuned = false;
    int32_t tiles_per_wg = 1;
    int32_t wg_per_cu = 0;
    int32_t streaming = 0;          // non-temporal population stores
    double us_default = 0.0, us_best = 0.0;
    int32_t candidates = 0;
};

}  // namespace

struct lb_ctx {
    lb_params p{};
    Plan plan;
    int32_t n_rep = 0;
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    // device views
    DeviceHeader* hdr = nullptr;
    ReplicaDesc* d_reps = nullptr;
    RowDesc* d_rows = nullptr;
    RowDesc* d_rowinfo = nullptr;
    NodeTile* d_tiles[2] = {nullptr, nullptr};
    void* f[2] = {nullptr, nullptr};
    int cur = 0;
    long long* gforce = nullptr;
    uint8_t* flags = nullptr;
    uint8_t* hole = nullptr;          // per node: wall id of a hole, else 0
    NodeTile* d_hole_tiles = nullptr;  // the tiles of replicas with holes
    std::vector<NodeTile> hole_tiles;
    Body* d_bodies = nullptr;
    Bead* d_beads = nullptr;
    BeadRec* d_recs = nullptr;
    double* d_bead_force = nullptr;
    double* d_bead_torque = nullptr;
    double* d_partials = nullptr;
    WallLink* d_links = nullptr;
    int64_t n_links = 0;
    EvSite* d_ev = nullptr;
    WcaRep* d_wrep = nullptr;
    int32_t* d_rep_bodies = nullptr;
    int32_t* d_nb_start = nullptr;
    WallSite* d_nb_sites = nullptr;
    uint8_t* d_near = nullptr;
    double* d_wca_ft = nullptr;
    std::vector<EvHost> ev;         // per body
    int64_t n_ev = 0, n_sites = 0;
    bool wca_dirty = false;         // site tables to rebuild before the next step
    // host mirrors
    std::vector<ReplicaDesc> reps;
    std::vector<RowDesc> rows;
    std::vector<RowDesc> rowinfo;
    std::vector<NodeTile> tiles[2];
    bool narrow[2] = {true, true};   // tile group addressable with 32-bit byte offsets
    std::vector<ReplicaHost> rh;
    std::vector<Body> bodies0;          // bodies as added (device copy is authoritative)
    std::vector<int32_t> bead_user;     // per stored bead: its index in the caller's order
    int32_t n_bodies = 0, n_beads = 0;
    int64_t step = 0;
    bool pose_stale = true;   // body poses must be recomputed before the next step
    std::string err;
    // graphs are captured on a private stream and replayed on the caller's
    int32_t graph_steps = 100;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    hipStream_t cap_stream = nullptr;
    // timing
    bool timing = false;
    int32_t store_policy = LB_STORES_AUTO;
    Tuning tune;
    std::vector<EventPair> ev_node, ev_couple_t, ev_pool;
};

namespace {

int fail(lb_ctx* c, int code, const std::string& msg)
{
    if (c) c->err = msg;
    return code;
}

#define HIP_TRY(ctx, expr)                                                                \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail((ctx), LB_ERR_HIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

bool is_f32(const lb_ctx* c) { return c->p.precision == LB_PRECISION_F32; }

template <typename Real>
CollideParams<Real> collide_params(const lb_params& p)
{
    CollideParams<Real> cp{};
    const double gb = 1.0 - 1.0 / p.tau_bulk, gs = 1.0 - 1.0 / p.tau_shear;
    const double go = 1.0 - 1.0 / p.tau_odd, ge = 1.0 - 1.0 / p.tau_even;
    cp.rho0 = (Real)p.rho0;
    cp.g_bulk = (Real)gb; cp.g_shear = (Real)gs; cp.g_odd = (Real)go; cp.g_even = (Real)ge;
    cp.h_bulk = (Real)(0.5 * (1.0 + gb));
    cp.h_shear = (Real)(0.5 * (1.0 + gs));
    // b_k of the orthogonal basis
    const double b[Q] = {1.0, 1.0 / 3, 1.0 / 3, 1.0 / 3, 2.0 / 3, 4.0 / 3, 4.0 / 9, 1.0 / 9,
                         1.0 / 9, 1.0 / 9, 2.0 / 3, 2.0 / 3, 2.0 / 3, 2.0 / 9, 2.0 / 9, 2.0 / 9,
                         2.0, 4.0 / 3, 4.0 / 9};
    const double mu = 3.0 * p.kT;
    for (int k = 0; k < Q; ++k) {
        double g = 0.0;
        if (k == 4) g = gb;
        else if (k >= 5 && k <= 9) g = gs;
        else if (k >= 10 && k <= 15) g = go;
        else if (k >= 16) g = ge;
        cp.a_noise[k] = k < 4 ? (Real)0 : (Real)(std::sqrt(mu * p.rho0 * b[k] * (1.0 - g * g)) * std::sqrt(12.0));
    }
    return cp;
}

// whether the populations the steps touch -- the fluid nodes of every replica, in both
// buffers -- exceed the Infinity Cache
bool populations_exceed_cache(const lb_ctx* c)
{
    const double real = c->p.precision == LB_PRECISION_F32 ? 4.0 : 8.0;
    double nodes = 0.0;
    for (int r = 0; r < c->n_rep; ++r) nodes += (double)pad_nodes(c->reps[r].n_fluid);
    return 2.0 * Q * real * nodes > kInfinityCacheBytes;
}

// non-temporal population stores: forced by the policy, else the tuned choice (lb_autotune),
// else once the populations exceed the Infinity Cache
bool streaming_stores(const lb_ctx* c)
{
    if (c->store_policy == LB_STORES_CACHED) return false;
    if (c->store_policy == LB_STORES_STREAMING) return true;
    if (c->tune.tuned) return c->tune.streaming != 0;
    return populations_exceed_cache(c);
}

// launch arguments of one tile group pulling from src and writing dst
template <typename Real>
StepArgs<Real> step_args_on(const lb_ctx* c, int group, const void* src, void* dst)
{
    StepArgs<Real> a{};
    a.src = (const Real*)src;
    a.dst = (Real*)dst;
    a.N = c->plan.N;
    a.reps = c->d_reps;
    a.rows = c->d_rows;
    a.rowinfo = c->d_rowinfo;
    a.tiles = c->d_tiles[group];
    a.n_tiles = (int32_t)c->tiles[group].size();
    a.tiles_per_wg = std::max(1, (int)c->tune.tiles_per_wg);
    a.wg_per_cu = c->tune.wg_per_cu;
    a.thermal = c->p.kT > 0.0 ? 1 : 0;
    a.narrow = c->narrow[group] ? 1 : 0;
    a.stream_stores = streaming_stores(c) ? 1 : 0;
    a.gforce = c->gforce;
    a.flags = c->flags;
    a.hole = c->hole;
    a.cp = collide_params<Real>(c->p);
    for (int ax = 0; ax < 3; ++ax) a.gext[ax] = (Real)c->p.g_ext[ax];
    a.step_ptr = nullptr;
    a.step_arg = c->step;
    return a;
}

template <typename Real>
StepArgs<Real> step_args(const lb_ctx* c, int group, int src_buf)
{
    return step_args_on<Real>(c, group, c->f[src_buf], c->f[src_buf ^ 1]);
}

int md_steps(const lb_ctx* c) { return std::max(1, (int)c->p.md_substeps); }

CoupleArgs couple_args(const lb_ctx* c)
{
    CoupleArgs ca{};
    ca.recs = c->d_recs;
    ca.bead_force = c->d_bead_force;
    ca.bead_torque = c->d_bead_torque;
    ca.n_beads = c->n_beads;
    ca.md_step = 0;
    ca.kT = c->p.kT;
    ca.spread_h = 1.0 / md_steps(c);
    ca.hdr = c->hdr;
    return ca;
}

BodyArgs body_args(const lb_ctx* c)
{
    BodyArgs ba{};
    ba.bodies = c->d_bodies;
    ba.beads = c->d_beads;
    ba.recs = c->d_recs;
    ba.bead_force = c->d_bead_force;
    ba.bead_torque = c->d_bead_torque;
    ba.n_bodies = c->n_bodies;
    ba.substeps = md_steps(c);
    ba.wca_eps = c->p.wca_epsilon;
    ba.wca_ft = (c->n_ev > 0 && c->p.wca_epsilon > 0.0) ? c->d_wca_ft : nullptr;
    ba.ev = c->d_ev;
    ba.wrep = c->d_wrep;
    ba.rep_bodies = c->d_rep_bodies;
    ba.nb_start = c->d_nb_start;
    ba.nb_sites = c->d_nb_sites;
    ba.near = c->d_near;
    return ba;
}

bool any_masked(const lb_ctx* c) { return !c->tiles[1].empty(); }

EventPair get_pair(lb_ctx* c)
{
    if (!c->ev_pool.empty()) {
        EventPair e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    EventPair e{};
    if (hipEventCreate(&e.a) != hipSuccess) e.a = nullptr;
    if (hipEventCreate(&e.b) != hipSuccess) e.b = nullptr;
    return e;
}

// The couplings of one fluid step on stream s, pulling from buffer src_buf; every MD step but
// the last also finishes the bodies.  In capture mode the kernels read the step counter from
// device memory (step_ptr + step_arg).
template <typename Real>
hipError_t enqueue_couple(lb_ctx* c, hipStream_t s, int src_buf, const int64_t* step_ptr,
                          int64_t step_arg, bool timed)
{
    hipError_t err = hipSuccess;
    auto note = [&](hipError_t e) { if (err == hipSuccess && e != hipSuccess) err = e; };
    StepArgs<Real> a = step_args<Real>(c, any_masked(c) ? 1 : 0, src_buf);
    a.step_ptr = step_ptr;
    a.step_arg = step_arg;
    CoupleArgs ca = couple_args(c);
    const BodyArgs ba = body_args(c);
    if (ca.n_beads <= 0) return err;
    const int m = md_steps(c);
    for (int k = 0; k < m; ++k) {
        // MD step k: its own noise block, the fluid gets 1/m of the force
        EventPair e{};
        if (timed) e = get_pair(c);
        ca.md_step = (uint32_t)k;
        launch_couple<Real>(a, ca, s, LaunchEvents{e.a, e.b}, &ba);
        note(hipGetLastError());
        if (timed && e.a && e.b) c->ev_couple_t.push_back(e);
        if (k + 1 < m) {
            launch_body_substep(ba, step_ptr, step_arg, k, s);
            note(hipGetLastError());
        }
    }
    return err;
}

// The node update of one fluid step on stream s, src_buf -> src_buf ^ 1, one launch per tile
// group; the first launch also finishes the bodies.
template <typename Real>
hipError_t enqueue_node(lb_ctx* c, hipStream_t s, int src_buf, const int64_t* step_ptr,
                        int64_t step_arg, bool timed)
{
    hipError_t err = hipSuccess;
    auto note = [&](hipError_t e) { if (err == hipSuccess && e != hipSuccess) err = e; };
    StepArgs<Real> ag[2] = {step_args<Real>(c, 0, src_buf), step_args<Real>(c, 1, src_buf)};
    const BodyArgs ba = body_args(c);
    for (int g = 0; g < 2; ++g) {
        ag[g].step_ptr = step_ptr;
        ag[g].step_arg = step_arg;
    }
    bool finished = ba.n_bodies == 0;
    for (int g = 0; g < 2; ++g) {
        const bool last = g == 1 || ag[1].n_tiles == 0;
        if (ag[g].n_tiles == 0 && !(last && !finished)) continue;
        EventPair e{};
        if (timed) e = get_pair(c);
        launch_node_step<Real>(ag[g], g == 1, c->n_beads > 0, finished ? nullptr : &ba, s,
                               LaunchEvents{e.a, e.b});
        note(hipGetLastError());
        if (timed && e.a && e.b) c->ev_node.push_back(e);
        finished = true;
    }
    return err;
}

// One serial fluid step on stream s: the couplings, then the node update of each tile group
// (the first node launch also finishes the bodies), then the moving-wall links.  Returns the
// first HIP error of the enqueued calls.
template <typename Real>
hipError_t enqueue_step(lb_ctx* c, hipStream_t s, int src_buf, const int64_t* step_ptr,
                        int64_t step_arg, bool capture)
{
    const bool timed = c->timing && !capture;   // timed launches carry their own events
    hipError_t err = enqueue_couple<Real>(c, s, src_buf, step_ptr, step_arg, timed);
    const hipError_t e2 = enqueue_node<Real>(c, s, src_buf, step_ptr, step_arg, timed);
    if (err == hipSuccess) err = e2;
    if (c->n_links > 0 && err == hipSuccess) {
        launch_wall_links<Real>((Real*)c->f[src_buf ^ 1], c->d_links, c->n_links, s);
        err = hipGetLastError();
    }
    if (!c->hole_tiles.empty() && err == hipSuccess) {
        launch_mirror_holes<Real>((Real*)c->f[src_buf ^ 1], c->d_reps, c->d_rows, c->d_rowinfo,
                                  c->d_hole_tiles, (int32_t)c->hole_tiles.size(), c->hole, s);
        err = hipGetLastError();
    }
    return err;
}

void destroy_graphs(lb_ctx* c)
{
    for (int k = 0; k < 2; ++k)
        if (c->gexec[k]) { (void)hipGraphExecDestroy(c->gexec[k]); c->gexec[k] = nullptr; }
}

int build_graph(lb_ctx* c, int parity)
{
    if (!c->cap_stream)
        HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));

    hipGraph_t graph = nullptr;
    HIP_TRY(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t cap_err = hipSuccess;
    int buf = parity;
    for (int k = 0; k < c->graph_steps && cap_err == hipSuccess; ++k) {
        cap_err = is_f32(c) ? enqueue_step<float>(c, c->cap_stream, buf, &c->hdr->step, k, true)
                            : enqueue_step<double>(c, c->cap_stream, buf, &c->hdr->step, k, true);
        buf ^= 1;
    }
    hipError_t end_err = hipStreamEndCapture(c->cap_stream, &graph);
    if (cap_err != hipSuccess || end_err != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        const hipError_t e = cap_err != hipSuccess ? cap_err : end_err;
        return fail(c, LB_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    }
    hipError_t e = hipGraphInstantiate(&c->gexec[parity], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        c->gexec[parity] = nullptr;
        return fail(c, LB_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    return LB_OK;
}

// Build the tiles of every replica from the fluid-row tables, replicas in index order.
void rebuild_tiles(lb_ctx* c)
{
    c->tiles[0].clear();
    c->tiles[1].clear();
    // a group uses 32-bit byte offsets when each of its replicas' populations fit in 4 GiB
    const uint64_t real = is_f32(c) ? sizeof(float) : sizeof(double);
    c->narrow[0] = c->narrow[1] = true;
    for (int r = 0; r < c->n_rep; ++r) {
        const ReplicaDesc& R = c->reps[r];
        if ((uint64_t)Q * (uint64_t)pad_nodes(R.n_nodes) * real > (uint64_t(1) << 32))
            c->narrow[R.masked ? 1 : 0] = false;
    }
    for (int r = 0; r < c->n_rep; ++r) {
        const ReplicaDesc& R = c->reps[r];
        ReplicaHost& H = c->rh[r];
        H.group = R.masked ? 1 : 0;
        std::vector<NodeTile>& T = c->tiles[H.group];
        H.tile0 = (int32_t)T.size();
        append_tiles(R, r, c->rows.data(), c->rowinfo.data(), T);
        H.n_tiles = (int32_t)T.size() - H.tile0;
    }
}

int upload_tables(lb_ctx* c)
{
    // the tiles of replicas with holes, for the mirror launch
    c->hole_tiles.clear();
    for (int r = 0; r < c->n_rep; ++r)
        if (c->reps[r].masked == 2)
            c->hole_tiles.insert(c->hole_tiles.end(), c->tiles[1].begin() + c->rh[r].tile0,
                                 c->tiles[1].begin() + c->rh[r].tile0 + c->rh[r].n_tiles);
    if (!c->hole_tiles.empty())
        HIP_TRY(c, hipMemcpyAsync(c->d_hole_tiles, c->hole_tiles.data(),
                                  sizeof(NodeTile) * c->hole_tiles.size(), hipMemcpyHostToDevice,
                                  c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->d_reps, c->reps.data(), sizeof(ReplicaDesc) * c->n_rep,
                              hipMemcpyHostToDevice, c->stream));
    if (!c->rows.empty())
        HIP_TRY(c, hipMemcpyAsync(c->d_rows, c->rows.data(), sizeof(RowDesc) * c->rows.size(),
                                  hipMemcpyHostToDevice, c->stream));
    if (!c->rowinfo.empty())
        HIP_TRY(c, hipMemcpyAsync(c->d_rowinfo, c->rowinfo.data(), sizeof(RowDesc) * c->rowinfo.size(),
                                  hipMemcpyHostToDevice, c->stream));
    for (int g = 0; g < 2; ++g)
        if (!c->tiles[g].empty())
            HIP_TRY(c, hipMemcpyAsync(c->d_tiles[g], c->tiles[g].data(),
                                      sizeof(NodeTile) * c->tiles[g].size(), hipMemcpyHostToDevice,
                                      c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return LB_OK;
}

// equilibrium of (rho0, u0) in the current buffer for the tiles of one replica (or all)
int init_fluid(lb_ctx* c, int replica)
{
    for (int g = 0; g < 2; ++g) {
        int32_t t0 = 0, nt = (int32_t)c->tiles[g].size();
        if (replica >= 0) {
            if (c->rh[replica].group != g) continue;
            t0 = c->rh[replica].tile0;
            nt = c->rh[replica].n_tiles;
        }
        if (is_f32(c))
            launch_init_equilibrium<float>((float*)c->f[c->cur], c->plan.N, c->d_reps,
                                           c->d_tiles[g] + t0, nt, (float)c->p.rho0, c->p.u0,
                                           c->stream);
        else
            launch_init_equilibrium<double>((double*)c->f[c->cur], c->plan.N, c->d_reps,
                                            c->d_tiles[g] + t0, nt, c->p.rho0, c->p.u0,
                                            c->stream);
    }
    // the fluid starts just before a streaming step: the moving walls' terms go in now
    for (int r = 0; r < c->n_rep; ++r) {
        if (replica >= 0 && r != replica) continue;
        const ReplicaHost& H = c->rh[r];
        if (H.links.empty()) continue;
        if (is_f32(c))
            launch_wall_links<float>((float*)c->f[c->cur], c->d_links + H.link0,
                                     (int64_t)H.links.size(), c->stream);
        else
            launch_wall_links<double>((double*)c->f[c->cur], c->d_links + H.link0,
                                      (int64_t)H.links.size(), c->stream);
    }
    // and the holes reflect what their fluid neighbours hold
    if (!c->hole_tiles.empty()) {
        if (is_f32(c))
            launch_mirror_holes<float>((float*)c->f[c->cur], c->d_reps, c->d_rows, c->d_rowinfo,
                                       c->d_hole_tiles, (int32_t)c->hole_tiles.size(), c->hole,
                                       c->stream);
        else
            launch_mirror_holes<double>((double*)c->f[c->cur], c->d_reps, c->d_rows,
                                        c->d_rowinfo, c->d_hole_tiles,
                                        (int32_t)c->hole_tiles.size(), c->hole, c->stream);
    }
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return LB_OK;
}

int64_t links_without(const lb_ctx* c, int32_t replica)
{
    int64_t n = 0;
    for (int r = 0; r < c->n_rep; ++r)
        if (r != replica) n += (int64_t)c->rh[r].links.size();
    return n;
}

// concatenate the replicas' links (replica order) into the device list
int upload_links(lb_ctx* c)
{
    std::vector<WallLink> all;
    for (int r = 0; r < c->n_rep; ++r) {
        c->rh[r].link0 = (int64_t)all.size();
        all.insert(all.end(), c->rh[r].links.begin(), c->rh[r].links.end());
    }
    c->n_links = (int64_t)all.size();
    if (!all.empty()) {
        HIP_TRY(c, hipMemcpyAsync(c->d_links, all.data(), sizeof(WallLink) * all.size(),
                                  hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    return LB_OK;
}

// the box's own sides of a replica (its storage may exchange axes x and z)
void box_dims(const ReplicaDesc& R, int d[3])
{
    d[0] = R.swap ? R.nz : R.nx;
    d[1] = R.ny;
    d[2] = R.swap ? R.nx : R.nz;
}

BodyBox body_box(const ReplicaDesc& R)
{
    BodyBox x{};
    int d[3];
    box_dims(R, d);
    x.nx = d[0]; x.ny = d[1]; x.nz = d[2]; x.masked = R.masked;
    x.swap = R.swap;
    x.base = R.base;
    x.row_base = R.row_base;
    x.key0 = R.key0; x.key1 = R.key1;
    return x;
}

bool check_replica(lb_ctx* c, int32_t r)
{
    if (r < 0 || r >= c->n_rep) { c->err = "replica index out of range"; return false; }
    return true;
}

// ------------------------------------------------------------------ excluded volume

// WCA tables of every replica from the host records: the bodies of each replica, the
// excluded-volume sites of every body (packed in body order), and for the static sites a
// coarse grid whose cells are at least one interaction range wide (with a margin, so a site
// within range of a point always lies in the point's cell or an adjacent one), one list per
// coarse cell of the sites in that neighbourhood, and a fine grid of flags marking the cells
// whose centre has a site within the range plus half the cell diagonal.
int build_wca(lb_ctx* c)
{
    // bodies: excluded-volume ranges
    std::vector<EvSite> ev;
    for (int32_t b = 0; b < c->n_bodies; ++b) {
        Body& B = c->bodies0[b];
        const EvHost& E = c->ev[b];
        B.first_ev = (int32_t)ev.size();
        B.n_ev = (int32_t)(E.off.size() / 3);
        B.ev_radius = E.radius;
        B.ev_reach = 0.0;
        for (int32_t k = 0; k < B.n_ev; ++k) {
            EvSite e{};
            for (int a = 0; a < 3; ++a) e.off[a] = E.off[3 * (size_t)k + a];
            B.ev_reach = std::max(B.ev_reach, std::sqrt(e.off[0] * e.off[0] + e.off[1] * e.off[1] +
                                                        e.off[2] * e.off[2]));
            ev.push_back(e);
        }
    }
    // replicas: body lists and site grids
    std::vector<WcaRep> wr(c->n_rep);
    std::vector<int32_t> rep_bodies;
    WcaTables wt;
    const std::vector<int32_t>& nb_start = wt.nb_start;
    const std::vector<WallSite>& nb_sites = wt.nb_sites;
    const std::vector<uint8_t>& near = wt.near;
    for (int r = 0; r < c->n_rep; ++r) {
        const ReplicaDesc& R = c->reps[r];
        const ReplicaHost& H = c->rh[r];
        WcaRep& W = wr[r];
        W = WcaRep{};
        W.first_body = (int32_t)rep_bodies.size();
        W.n_bodies = (int32_t)H.bodies.size();
        double ev_r = -1.0;
        for (int32_t b : H.bodies) {
            rep_bodies.push_back(b);
            if (c->bodies0[b].n_ev > 0) ev_r = std::max(ev_r, c->bodies0[b].ev_radius);
        }
        int dims[3];
        box_dims(R, dims);
        if (!wca_grid(dims, ev_r, H.sites, W, wt))
            return fail(c, LB_ERR_ARG, "a box side is shorter than twice the WCA range");
    }
    if ((int64_t)nb_start.size() > c->plan.cells_cap || (int64_t)near.size() > c->plan.fine_cap ||
        (int64_t)nb_sites.size() > 27 * c->plan.site_cap)
        return fail(c, LB_ERR_CAPACITY, "WCA site grids exceed their workspace");
    c->n_ev = (int64_t)ev.size();
    if (!ev.empty())
        HIP_TRY(c, hipMemcpyAsync(c->d_ev, ev.data(), sizeof(EvSite) * ev.size(),
                                  hipMemcpyHostToDevice, c->stream));
    if (!nb_start.empty())
        HIP_TRY(c, hipMemcpyAsync(c->d_nb_start, nb_start.data(), sizeof(int32_t) * nb_start.size(),
                                  hipMemcpyHostToDevice, c->stream));
    if (!nb_sites.empty())
        HIP_TRY(c, hipMemcpyAsync(c->d_nb_sites, nb_sites.data(), sizeof(WallSite) * nb_sites.size(),
                                  hipMemcpyHostToDevice, c->stream));
    if (!near.empty())
        HIP_TRY(c, hipMemcpyAsync(c->d_near, near.data(), near.size(), hipMemcpyHostToDevice,
                                  c->stream));
    if (!rep_bodies.empty())
        HIP_TRY(c, hipMemcpyAsync(c->d_rep_bodies, rep_bodies.data(),
                                  sizeof(int32_t) * rep_bodies.size(), hipMemcpyHostToDevice,
                                  c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->d_wrep, wr.data(), sizeof(WcaRep) * wr.size(),
                              hipMemcpyHostToDevice, c->stream));
    // the bodies' site ranges (set before the first step, so the host records are current
    // apart from what a loaded state changed: copy only these fields)
    const size_t f0 = offsetof(Body, ev_radius), f1 = offsetof(Body, n_ev) + sizeof(int32_t);
    for (int32_t b = 0; b < c->n_bodies; ++b)
        HIP_TRY(c, hipMemcpyAsync((char*)(c->d_bodies + b) + f0, (const char*)&c->bodies0[b] + f0,
                                  f1 - f0, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->wca_dirty = false;
    destroy_graphs(c);
    return LB_OK;
}

// ------------------------------------------------------------------ reverse pass
// Layout of the caller's reverse-pass workspace: checkpoints of the post-collision state
// every K steps, K-1 slots for the states recomputed inside one segment, two adjoint
// population buffers, the adjoints of the node force and velocity, the per-step objective
// weights, the per-bead accumulators, and room to restore the bead forces afterwards; for
// free bodies the body table before every step of the window (and after the last), the
// adjoint of the body states, the bead pass's sums,
// the body tables between the MD steps of one fluid step, zero weights (the objective takes
// the last MD step's force) and room to restore the bead records.
struct AdjPlan {
    int32_t n_ck = 0, n_seg = 0;
    size_t state = 0;
    size_t off_ck, off_seg, off_lam0, off_lam1, off_lamF, off_w, off_dr, off_dg, off_J,
        off_bf, off_save, off_snap, off_badj, off_bsum, off_recs, off_scr, off_zero,
        off_wadj, off_Jb, total;
};

bool any_free(const lb_ctx* c)
{
    for (const Body& B : c->bodies0)
        if (!B.fixed) return true;
    return false;
}

// the most excluded-volume sites of any body
int max_ev_sites(const lb_ctx* c)
{
    size_t m = 0;
    for (const EvHost& E : c->ev) m = std::max(m, E.off.size() / 3);
    return (int)m;
}

// excluded-volume forces act (from the sites as set, whether or not their tables are built)
bool has_wca(const lb_ctx* c)
{
    if (!(c->p.wca_epsilon > 0.0)) return false;
    for (const EvHost& E : c->ev)
        if (!E.off.empty()) return true;
    return false;
}

// the reverse pass runs the body passes (free bodies, several MD steps per fluid step, or
// excluded volume); otherwise it runs the fixed-body schedule, with a fluid step's coupling
// fused into the next reverse step's bead launch
bool body_passes(const lb_ctx* c) { return any_free(c) || md_steps(c) > 1 || has_wca(c); }

bool make_adj_plan(const lb_ctx* c, int32_t T, int32_t K, AdjPlan& ap)
{
    if (!c || T < 1 || K < 1) return false;
    K = std::min(K, T);
    ap = AdjPlan();
    const size_t real = is_f32(c) ? sizeof(float) : sizeof(double);
    const int64_t N = c->plan.N;
    const int64_t nb = std::max<int32_t>(c->n_beads, 1), nbod = std::max<int32_t>(c->n_bodies, 1);
    ap.n_ck = (T + K - 1) / K;
    ap.n_seg = K - 1;
    ap.state = align_up(real * Q * N, kAlign);
    size_t o = 0;
    auto take = [&](size_t bytes) { const size_t at = o; o = align_up(o + bytes, kAlign); return at; };
    ap.off_ck = take(ap.state * ap.n_ck);
    ap.off_seg = take(ap.state * ap.n_seg);
    ap.off_lam0 = take(ap.state);
    ap.off_lam1 = take(ap.state);
    ap.off_lamF = take(real * 3 * N);
    ap.off_w = take(sizeof(double) * 3 * nbod * (size_t)T);
    ap.off_dr = take(sizeof(double) * 3 * nb);
    ap.off_dg = take(sizeof(double) * nb);
    ap.off_J = take(sizeof(double) * nb);
    const int m = md_steps(c);
    ap.off_bf = take(sizeof(double) * 3 * nb * (size_t)std::max(2, m));   // bead forces per MD step
    ap.off_save = take(sizeof(double) * 6 * nb);
    if (body_passes(c)) {
        ap.off_snap = take(sizeof(Body) * nbod * ((size_t)T + 1));
        ap.off_badj = take(sizeof(double) * kBodyAdjWords * nbod);
        ap.off_bsum = take(sizeof(double) * kBeadSumWords * nb);
        ap.off_recs = take(sizeof(BeadRec) * nb);
        ap.off_scr = take(sizeof(Body) * nbod * (size_t)std::max(1, m - 1));
        ap.off_zero = take(sizeof(double) * 3 * nbod);
        ap.off_wadj = take(sizeof(double) * 6 * nbod);
        ap.off_Jb = take(sizeof(double) * nbod);
    } else {
        ap.off_snap = ap.off_badj = ap.off_bsum = ap.off_recs = 0;
        ap.off_scr = ap.off_zero = ap.off_wadj = ap.off_Jb = 0;
    }
    ap.total = o;
    return true;
}

// The couplings of a recomputed fluid step from its stored body table `table` (the bodies
// before the step): the records of its first MD step from the table's pose, then per MD step
// k the coupling, bead forces into bf + k * nbf; between MD steps the bodies are finished as
// the forward step does, into scr + k * n_bodies (the table before MD step k + 1; the
// finishing also writes that step's records).
template <typename Real>
void enqueue_recoupling(lb_ctx* c, hipStream_t s, const StepArgs<Real>& a, int64_t step,
                        const Body* table, Body* scr, double* bf, size_t nbf)
{
    const int m = md_steps(c);
    if (c->n_beads <= 0) return;
    launch_records_from_poses(table, (int)((step * m) & 1), c->d_beads, c->d_recs, c->n_beads, s);
    CoupleArgs ca = couple_args(c);
    for (int k = 0; k < m; ++k) {
        ca.md_step = (uint32_t)k;
        ca.bead_force = bf + nbf * (size_t)k;
        const Body* from = k == 0 ? table : scr + (size_t)c->n_bodies * (k - 1);
        BodyArgs wb = body_args(c);   // the excluded volume at the MD step's poses
        wb.bodies = const_cast<Body*>(from);
        launch_couple<Real>(a, ca, s, LaunchEvents{}, &wb);
        if (k + 1 < m) {
            Body* to = scr + (size_t)c->n_bodies * k;
            (void)hipMemcpyAsync(to, from, sizeof(Body) * (size_t)c->n_bodies, hipMemcpyDeviceToDevice, s);
            BodyArgs ba = body_args(c);
            ba.bodies = to;
            ba.bead_force = ca.bead_force;
            launch_body_substep(ba, nullptr, step, k, s);
        }
    }
}

// forward step without finishing the bodies, src -> dst.  Fixed bodies with one MD step: the
// records hold the only pose; otherwise the couplings are recomputed from the stored body
// table `bodies` of the step (enqueue_recoupling).
template <typename Real>
void enqueue_replay(lb_ctx* c, hipStream_t s, const void* src, void* dst, int64_t step,
                    const Body* bodies, Body* scr, double* bf, size_t nbf)
{
    StepArgs<Real> ag[2] = {step_args_on<Real>(c, 0, src, dst), step_args_on<Real>(c, 1, src, dst)};
    for (auto& a : ag) a.step_arg = step;
    if (bodies)
        enqueue_recoupling<Real>(c, s, any_masked(c) ? ag[1] : ag[0], step, bodies, scr, bf, nbf);
    else if (c->n_beads > 0)
        launch_couple<Real>(any_masked(c) ? ag[1] : ag[0], couple_args(c), s);
    for (int g = 0; g < 2; ++g)
        if (ag[g].n_tiles > 0)
            launch_node_step<Real>(ag[g], g == 1, c->n_beads > 0, nullptr, s);
    if (c->n_links > 0) launch_wall_links<Real>(ag[0].dst, c->d_links, c->n_links, s);
    if (!c->hole_tiles.empty())
        launch_mirror_holes<Real>(ag[0].dst, c->d_reps, c->d_rows, c->d_rowinfo, c->d_hole_tiles,
                                  (int32_t)c->hole_tiles.size(), c->hole, s);
}

// one reverse step at forward step `step` (index n of the window), forward state pulled from
// src.  coupled: the coupling of this step already ran (in the previous reverse step's bead
// launch); prev_src: the state of step - 1, whose coupling then runs in this step's bead launch
// (nullptr: none, as at the start of a segment, whose states the replay rewrites first).
// The bead forces of a reverse step go to one of two buffers by the parity of n.
// snap: with body passes, the stored body tables of the window.  With one MD step and no
// excluded volume the schedule above holds, the records written from table n - 1 for the
// shared coupling and the body pass reading tables n and n + 1; otherwise the couplings of
// step n are recomputed from table n, the MD steps' body passes read the tables before and
// after each of them (table n, the scratch tables of the recompute, table n + 1), and
// prev_src is null.
template <typename Real>
void enqueue_adjoint(lb_ctx* c, hipStream_t s, const void* src, int64_t step, const Real* lam_next,
                     Real* lam_cur, char* ws, const AdjPlan& ap, int64_t n, bool coupled,
                     const void* prev_src, const Body* snap)
{
    double* bf = (double*)(ws + ap.off_bf);
    const size_t nbf = 3 * (size_t)std::max<int32_t>(c->n_beads, 1);
    auto coupling = [&](int64_t k) {
        CoupleArgs ca = couple_args(c);
        ca.bead_force = bf + nbf * (size_t)(k & 1);
        return ca;
    };
    AdjArgs<Real> A[2];
    for (int g = 0; g < 2; ++g) {
        AdjArgs<Real>& X = A[g];
        X = AdjArgs<Real>{};
        X.a = step_args_on<Real>(c, g, src, nullptr);
        X.a.step_arg = step;
        X.lam_next = lam_next;
        X.lam_cur = lam_cur;
        X.lamF = (Real*)(ws + ap.off_lamF);
        X.beads = c->d_beads;
        X.recs = c->d_recs;
        X.bead_force = bf + nbf * (size_t)(n & 1);
        X.weights = (const double*)(ws + ap.off_w) + 3 * (int64_t)c->n_bodies * n;
        X.dr = (double*)(ws + ap.off_dr);
        X.dgam = (double*)(ws + ap.off_dg);
        X.Jpart = (double*)(ws + ap.off_J);
        X.n_beads = c->n_beads;
        if (snap) {
            X.body_adj = (const double*)(ws + ap.off_badj);
            X.bead_sums = (double*)(ws + ap.off_bsum);
            X.spread_h = 1.0 / md_steps(c);
        }
    }
    const int cg = any_masked(c) ? 1 : 0;
    if (snap && md_steps(c) == 1 && !has_wca(c)) {
        // one MD step and no excluded volume: the fixed-body schedule with the body pass after
        // the bead launch.  The bead pass takes the positions from the stored pose of step n,
        // so the records may hold step n - 1's for the coupling recompute sharing its launch.
        const size_t nb = (size_t)c->n_bodies;
        const Body* t0 = snap + nb * n;
        const int par = (int)(step & 1);
        if (c->n_beads > 0 && !coupled) {
            launch_records_from_poses(t0, par, c->d_beads, c->d_recs, c->n_beads, s);
            launch_couple<Real>(A[cg].a, coupling(n), s);
        }
        for (int g = 0; g < 2; ++g) launch_adjoint_step<Real>(A[g], g == 1, s);
        if (c->n_beads <= 0) return;
        AdjArgs<Real> X = A[cg];
        X.snap = t0;
        X.pose_par = par;
        if (prev_src) {
            launch_records_from_poses(t0 - nb, (int)((step - 1) & 1), c->d_beads, c->d_recs,
                                      c->n_beads, s);
            StepArgs<Real> pa = step_args_on<Real>(c, cg, prev_src, nullptr);
            pa.step_arg = step - 1;
            launch_couple_adj_bead<Real>(pa, coupling(n - 1), X, s);
        } else {
            launch_adjoint_beads<Real>(X, s);
        }
        launch_adjoint_body_post(t0, t0 + nb, par, X.weights, (const double*)(ws + ap.off_bsum),
                                 (double*)(ws + ap.off_badj), (double*)(ws + ap.off_wadj),
                                 (double*)(ws + ap.off_Jb), c->n_bodies, s);
        return;
    }
    if (snap) {
        // the MD steps of fluid step n: recompute their couplings (the spread force the node
        // pass takes, each MD step's bead forces and the body tables between them), then the
        // node pass, then each MD step's body and bead passes in reverse order
        const int m = md_steps(c);
        const size_t nb = (size_t)c->n_bodies;
        const Body* t0 = snap + nb * n;
        Body* scr = (Body*)(ws + ap.off_scr);
        enqueue_recoupling<Real>(c, s, A[cg].a, step, t0, scr, bf, nbf);
        for (int g = 0; g < 2; ++g) launch_adjoint_step<Real>(A[g], g == 1, s);
        if (c->n_beads <= 0) return;
        auto table = [&](int k) { return k == 0 ? t0 : k == m ? t0 + nb : scr + nb * (k - 1); };
        double* badj = (double*)(ws + ap.off_badj);
        double* wadj = (double*)(ws + ap.off_wadj);
        const double* zero = (const double*)(ws + ap.off_zero);
        const double* weights = A[cg].weights;
        for (int k = m - 1; k >= 0; --k) {
            const int par = (int)((step * m + k) & 1);
            AdjArgs<Real> X = A[cg];
            X.weights = k == m - 1 ? weights : zero;   // the objective takes the last MD step
            X.bead_force = bf + nbf * (size_t)k;
            X.snap = table(k);
            X.pose_par = par;
            // the recompute left the records of the last MD step in place
            if (k != m - 1)
                launch_records_from_poses(table(k), par, c->d_beads, c->d_recs, c->n_beads, s);
            launch_adjoint_beads<Real>(X, s);
            if (has_wca(c)) {
                BodyArgs wb = body_args(c);
                wb.bodies = const_cast<Body*>(table(k));
                launch_adjoint_wca(wb, par, X.weights, badj, wadj, max_ev_sites(c), s);
            }
            launch_adjoint_body_post(table(k), table(k + 1), par, X.weights,
                                     (const double*)(ws + ap.off_bsum), badj, wadj,
                                     (double*)(ws + ap.off_Jb), c->n_bodies, s);
        }
        return;
    }
    if (c->n_beads > 0 && !coupled) launch_couple<Real>(A[cg].a, coupling(n), s);
    for (int g = 0; g < 2; ++g) launch_adjoint_step<Real>(A[g], g == 1, s);
    if (c->n_beads <= 0) return;
    if (prev_src) {
        StepArgs<Real> pa = step_args_on<Real>(c, cg, prev_src, nullptr);
        pa.step_arg = step - 1;
        launch_couple_adj_bead<Real>(pa, coupling(n - 1), A[cg], s);
    } else {
        launch_adjoint_beads<Real>(A[cg], s);
    }
}

template <typename Real>
int run_adjoint(lb_ctx* c, int32_t T, int32_t K, char* ws, const AdjPlan& ap)
{
    hipStream_t s = c->stream;
    K = std::min(K, T);
    auto ck = [&](int k) { return (void*)(ws + ap.off_ck + ap.state * k); };
    auto seg = [&](int k) { return (void*)(ws + ap.off_seg + ap.state * k); };
    const int64_t step0 = c->step;
    // with body passes: the body table before every step of the window and after the last
    const bool fb = body_passes(c);
    // a fluid step's coupling recompute shares the next reverse step's bead launch (not with
    // several MD steps or excluded volume, whose couplings are recomputed with the body
    // finishing between them)
    const bool fused = !fb || (md_steps(c) == 1 && !has_wca(c));
    Body* snap = fb ? (Body*)(ws + ap.off_snap) : nullptr;
    const size_t table = sizeof(Body) * (size_t)c->n_bodies;
    if (fb) HIP_TRY(c, hipMemcpyAsync(snap, c->d_bodies, table, hipMemcpyDeviceToDevice, s));
    // forward window, keeping a checkpoint every K steps
    for (int32_t n = 0; n < T; ++n) {
        if (n % K == 0)
            HIP_TRY(c, hipMemcpyAsync(ck(n / K), c->f[c->cur], ap.state, hipMemcpyDeviceToDevice, s));
        HIP_TRY(c, enqueue_step<Real>(c, s, c->cur, nullptr, c->step, false));
        c->cur ^= 1;
        c->step += 1;
        if (fb)
            HIP_TRY(c, hipMemcpyAsync(snap + (size_t)c->n_bodies * (n + 1), c->d_bodies, table,
                                      hipMemcpyDeviceToDevice, s));
    }
    const size_t nb = (size_t)std::max<int32_t>(c->n_beads, 1);
    if (fb)
        HIP_TRY(c, hipMemcpyAsync(ws + ap.off_recs, c->d_recs, sizeof(BeadRec) * nb,
                                  hipMemcpyDeviceToDevice, s));
    double* save = (double*)(ws + ap.off_save);
    HIP_TRY(c, hipMemcpyAsync(save, c->d_bead_force, sizeof(double) * 3 * nb, hipMemcpyDeviceToDevice, s));
    HIP_TRY(c, hipMemcpyAsync(save + 3 * nb, c->d_bead_torque, sizeof(double) * 3 * nb,
                              hipMemcpyDeviceToDevice, s));
    // reverse, one segment at a time: recompute the segment's states, then walk it backwards
    Real* lam[2] = {(Real*)(ws + ap.off_lam0), (Real*)(ws + ap.off_lam1)};
    int nxt = 0;
    bool coupled = false;   // the coupling of the next reverse step already ran
    for (int32_t sg = ap.n_ck - 1; sg >= 0; --sg) {
        const int32_t n0 = sg * K, n1 = std::min(T, n0 + K);
        auto state = [&](int32_t j) { return j == 0 ? ck(sg) : seg(j - 1); };
        for (int32_t j = 0; j + 1 < n1 - n0; ++j)
            enqueue_replay<Real>(c, s, state(j), state(j + 1), step0 + n0 + j,
                                 fb ? snap + (size_t)c->n_bodies * (n0 + j) : nullptr,
                                 (Body*)(ws + ap.off_scr), (double*)(ws + ap.off_bf),
                                 3 * (size_t)std::max<int32_t>(c->n_beads, 1));
        HIP_TRY(c, hipGetLastError());
        for (int32_t n = n1 - 1; n >= n0; --n) {
            // the coupling of step n - 1 joins this step's bead launch when its state is at
            // hand and nothing in between rewrites the force accumulators: inside a segment,
            // and across segments of one step each (no replays)
            const void* prev = !fused ? nullptr
                                      : n > n0 ? state(n - 1 - n0) : (K == 1 && n > 0 ? ck(n - 1) : nullptr);
            enqueue_adjoint<Real>(c, s, state(n - n0), step0 + n, lam[nxt], lam[nxt ^ 1], ws, ap, n,
                                  coupled, prev, snap);
            if (!c->hole_tiles.empty())   // the step's adjoint is complete: transposed mirror
                launch_mirror_holes_transposed<Real>(lam[nxt ^ 1], c->d_reps, c->d_rows, c->d_rowinfo,
                                                     c->d_hole_tiles, (int32_t)c->hole_tiles.size(),
                                                     c->hole, s);
            coupled = prev != nullptr;
            nxt ^= 1;
        }
        HIP_TRY(c, hipGetLastError());
    }
    HIP_TRY(c, hipMemcpyAsync(c->d_bead_force, save, sizeof(double) * 3 * nb, hipMemcpyDeviceToDevice, s));
    HIP_TRY(c, hipMemcpyAsync(c->d_bead_torque, save + 3 * nb, sizeof(double) * 3 * nb,
                              hipMemcpyDeviceToDevice, s));
    if (fb)
        HIP_TRY(c, hipMemcpyAsync(c->d_recs, ws + ap.off_recs, sizeof(BeadRec) * nb,
                                  hipMemcpyDeviceToDevice, s));
    return LB_OK;
}

// ------------------------------------------------------------------ autotuner
// The node update's launch settings -- node tiles per workgroup, a cap on the workgroups
// resident per CU (by dynamic LDS), ordinary or non-temporal population stores -- are timed on
// the context's own node kernel over its own tiles: every tile group, the kernel the steps
// launch (with the force path when the context has beads) but without body finishing, pulling
// from the current buffer and writing the other one, which the next step overwrites whole.
// Between steps every spread force has been consumed (flags and words are zero), so the timed
// launches take none and the simulation state is unchanged.  Results are kept per
// (device architecture, precision, thermal, tile counts, fluid nodes) for the process.

struct TuneCand { int32_t per, cap, streaming; };
constexpr double kTuneMargin = 0.01;   // a setting must beat the untuned one by this fraction

std::mutex& tune_mutex() { static std::mutex m; return m; }
std::map<std::string, Tuning>& tune_cache() { static std::map<std::string, Tuning> m; return m; }

std::string tune_key(const lb_ctx* c)
{
    int dev = 0;
    hipDeviceProp_t prop{};
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        arch = prop.gcnArchName;
    int64_t fluid = 0;
    for (int r = 0; r < c->n_rep; ++r) fluid += c->reps[r].n_fluid;
    return arch + "|" + std::to_string(c->p.precision) + "|" + std::to_string(c->p.kT > 0.0) + "|" +
           std::to_string(c->tiles[0].size()) + "|" + std::to_string(c->tiles[1].size()) + "|" +
           std::to_string(fluid) + "|" + std::to_string(c->store_policy);
}

// mean duration (us) of one node update of every tile group with the context's current settings
template <typename Real>
int time_node_update(lb_ctx* c, hipEvent_t e0, hipEvent_t e1, int reps, double& us)
{
    StepArgs<Real> ag[2] = {step_args<Real>(c, 0, c->cur), step_args<Real>(c, 1, c->cur)};
    auto once = [&]() {
        for (int g = 0; g < 2; ++g)
            if (ag[g].n_tiles > 0)
                launch_node_step<Real>(ag[g], g == 1, c->n_beads > 0, nullptr, c->stream);
    };
    once();   // warm-up
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipEventRecord(e0, c->stream));
    for (int k = 0; k < reps; ++k) once();
    HIP_TRY(c, hipEventRecord(e1, c->stream));
    HIP_TRY(c, hipEventSynchronize(e1));
    HIP_TRY(c, hipGetLastError());
    float ms = 0.0f;
    HIP_TRY(c, hipEventElapsedTime(&ms, e0, e1));
    us = 1e3 * (double)ms / reps;
    return LB_OK;
}

template <typename Real>
int autotune_t(lb_ctx* c, int reps, Tuning& best)
{
    std::vector<TuneCand> cands;
    const bool fixed_stores = c->store_policy != LB_STORES_AUTO;
    Tuning saved = c->tune;
    c->tune = Tuning{};
    const int32_t default_streaming = streaming_stores(c) ? 1 : 0;   // the untuned rule
    // The timed launches read a buffer that stays unchanged, while a step reads what the step
    // before wrote: with buffers that fit in the Infinity Cache, non-temporal stores would time
    // faster here and run slower in the steps (their data bypasses the cache the next step
    // reads from), so they are a candidate only for buffers larger than the cache.
    const bool both_kinds = !fixed_stores && populations_exceed_cache(c);
    for (int st = 0; st < 2; ++st) {
        if (!both_kinds && st != default_streaming) continue;
        for (int per : {1, kWideTiles})
            for (int cap : {0, 6, 5, 4}) cands.push_back(TuneCand{per, cap, st});
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(c, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(c, LB_ERR_HIP, "hipEventCreate");
    }
    int rc = LB_OK;
    best = Tuning{};
    bool have = false;
    double t_default = -1.0;
    for (const TuneCand& k : cands) {
        c->tune = Tuning{};
        c->tune.tuned = true;
        c->tune.tiles_per_wg = k.per;
        c->tune.wg_per_cu = k.cap;
        c->tune.streaming = k.streaming;
        double us = 0.0;
        rc = time_node_update<Real>(c, e0, e1, reps, us);
        if (rc != LB_OK) break;
        if (k.per == 1 && k.cap == 0 && k.streaming == default_streaming) t_default = us;
        if (!have || us < best.us_best) {
            best = c->tune;
            best.us_best = us;
            have = true;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != LB_OK) {
        c->tune = saved;
        return rc;
    }
    // the untuned settings stay unless another setting is at least 1 % faster
    if (t_default > 0.0 && best.us_best > (1.0 - kTuneMargin) * t_default) {
        best = Tuning{};
        best.streaming = default_streaming;
        best.us_best = t_default;
    }
    best.candidates = (int32_t)cands.size();
    best.us_default = t_default;
    best.tuned = true;
    c->tune = best;
    return LB_OK;
}

}  // namespace

namespace lbrb {
// error reporting for the entry points of other source files
int set_error(lb_ctx* c, int code, const char* msg) { return fail(c, code, msg); }
}

// ============================================================================ C-ABI

extern "C" {

size_t lb_workspace_bytes(const lb_params* params, const lb_replica* replicas,
                          int32_t n_replicas)
{
    Plan pl;
    if (!make_plan(params, replicas, n_replicas, pl)) return 0;
    return pl.total;
}

int lb_init(const lb_params* params, const lb_replica* replicas, int32_t n_replicas,
            void* dev_workspace, size_t ws_bytes, void* hip_stream, lb_ctx** out)
{
    if (!out) return LB_ERR_ARG;
    *out = nullptr;
    Plan pl;
    if (!make_plan(params, replicas, n_replicas, pl)) return LB_ERR_ARG;
    if (!dev_workspace || ((uintptr_t)dev_workspace % kAlign) != 0 || ws_bytes < pl.total)
        return LB_ERR_ARG;
    lb_ctx* c = new (std::nothrow) lb_ctx();
    if (!c) return LB_ERR_ARG;
    c->p = *params;
    c->plan = pl;
    c->n_rep = n_replicas;
    c->stream = (hipStream_t)hip_stream;
    c->ws = (char*)dev_workspace;
    c->hdr = (DeviceHeader*)(c->ws + pl.off_hdr);
    c->d_reps = (ReplicaDesc*)(c->ws + pl.off_reps);
    c->d_rows = (RowDesc*)(c->ws + pl.off_rows);
    c->d_rowinfo = (RowDesc*)(c->ws + pl.off_rowinfo);
    c->d_tiles[0] = (NodeTile*)(c->ws + pl.off_tiles_d);
    c->d_tiles[1] = (NodeTile*)(c->ws + pl.off_tiles_m);
    c->f[0] = c->ws + pl.off_fa;
    c->f[1] = c->ws + pl.off_fb;
    c->gforce = (long long*)(c->ws + pl.off_gforce);
    c->flags = (uint8_t*)(c->ws + pl.off_flags);
    c->hole = (uint8_t*)(c->ws + pl.off_hole);
    c->d_hole_tiles = (NodeTile*)(c->ws + pl.off_hole_tiles);
    c->d_bodies = (Body*)(c->ws + pl.off_bodies);
    c->d_beads = (Bead*)(c->ws + pl.off_bead_off);
    c->d_recs = (BeadRec*)(c->ws + pl.off_bead_rec);
    c->d_bead_force = (double*)(c->ws + pl.off_bead_force);
    c->d_bead_torque = (double*)(c->ws + pl.off_bead_torque);
    c->d_partials = (double*)(c->ws + pl.off_partials);
    c->d_links = (WallLink*)(c->ws + pl.off_links);
    c->d_ev = (EvSite*)(c->ws + pl.off_ev);
    c->d_wrep = (WcaRep*)(c->ws + pl.off_wrep);
    c->d_rep_bodies = (int32_t*)(c->ws + pl.off_rep_bodies);
    c->d_nb_start = (int32_t*)(c->ws + pl.off_nb_start);
    c->d_nb_sites = (WallSite*)(c->ws + pl.off_nb_sites);
    c->d_near = (uint8_t*)(c->ws + pl.off_near);
    c->d_wca_ft = (double*)(c->ws + pl.off_wca_ft);

    c->reps.resize(n_replicas);
    c->rh.resize(n_replicas);
    c->rows.assign(pl.rows_cap, RowDesc{0, 0, 0, 0});
    c->rowinfo.assign(pl.rows_cap, RowDesc{0, 0, 0, 0});
    int64_t base = 0, row_base = 0;
    for (int r = 0; r < n_replicas; ++r) {
        const lb_replica& in = replicas[r];
        ReplicaDesc& R = c->reps[r];
        R = ReplicaDesc{};
        R.nx = in.nx; R.ny = in.ny; R.nz = in.nz;
        R.masked = 0;
        R.base = base;
        R.n_nodes = (int64_t)in.nx * in.ny * in.nz;
        R.n_fluid = R.n_nodes;
        R.row_base = (int32_t)row_base;
        R.key0 = (uint32_t)(in.seed & 0xFFFFFFFFu);
        R.key1 = (uint32_t)(in.seed >> 32);
        R.inv_nx = 1.0 / in.nx;
        R.inv_ny = 1.0 / in.ny;

        base += pad_nodes(R.n_nodes);
        row_base += (int64_t)in.ny * std::max(in.nx, in.nz);
    }
    rebuild_tiles(c);
    // zero the header, the spread-force accumulators and the flags once
    hipError_t e = hipMemsetAsync(c->ws + pl.off_hdr, 0, sizeof(DeviceHeader), c->stream);
    if (e == hipSuccess)
        e = hipMemsetAsync(c->gforce, 0, sizeof(long long) * pl.gforce_words * pl.N, c->stream);
    // padding nodes are never written by the kernels: clear both buffers once so that a saved
    // state is a deterministic function of the run
    const size_t real = is_f32(c) ? sizeof(float) : sizeof(double);
    for (int k = 0; k < 2 && e == hipSuccess; ++k)
        e = hipMemsetAsync(c->f[k], 0, real * Q * pl.N, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->flags, 0, pl.N, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->hole, 0, pl.N, c->stream);
    if (e != hipSuccess) { lb_destroy(c); return LB_ERR_HIP; }
    int rc = upload_tables(c);
    if (rc == LB_OK) rc = init_fluid(c, -1);
    if (rc != LB_OK) { lb_destroy(c); return rc; }
    noalloc_prepare();
    *out = c;
    return LB_OK;
}

int lb_set_boundary_mask(lb_ctx* c, int32_t replica, const uint8_t* mask)
{
    if (!c) return LB_ERR_ARG;
    if (!check_replica(c, replica) || !mask) return fail(c, LB_ERR_ARG, "bad replica or mask");
    if (c->step != 0) return fail(c, LB_ERR_STATE, "masks can only be set before the first step");
    ReplicaDesc& R = c->reps[replica];
    int box[3];
    box_dims(R, box);
    const int nx = box[0], ny = box[1], nz = box[2];
    // Storage orientation: rows along x, or along z (axes x and z exchanged) when the x rows
    // are short (under 48 stored nodes on average, so that a wavefront of 64 spans several
    // row segments, and its reads of the neighbouring rows fall on more cache lines) and the z
    // rows much longer -- a pore along z.  Longer x rows stay: there the exchanged storage puts
    // neighbouring planes farther apart (measured: a 512-replica batch of pores of sides 32-64
    // gains 2 %, a 128 x 128 x 256 pore with x rows of 63 nodes loses 4 %).
    MaskRows m = compress_mask(nx, ny, nz, mask);
    std::vector<uint8_t> stored_mask(mask, mask + (size_t)nx * ny * nz);
    bool swap = false;
    if (m.any_solid) {
        std::vector<uint8_t> t((size_t)nx * ny * nz);
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x)
                    t[z + (size_t)nz * (y + (size_t)ny * x)] = mask[x + (size_t)nx * (y + (size_t)ny * z)];
        MaskRows mt = compress_mask(nz, ny, nx, t.data());
        // stored nodes plus a cache line's worth of nodes per row
        const double cost_x = (double)m.stored + 16.0 * (double)m.rows.size();
        const double cost_z = (double)mt.stored + 16.0 * (double)mt.rows.size();
        const bool short_x = (double)m.stored < 48.0 * (double)m.rows.size();
        if (short_x && cost_z < 0.9 * cost_x) {
            swap = true;
            m = std::move(mt);
            stored_mask.swap(t);
        }
    }
    const bool any_solid = m.any_solid;
    const int64_t n_holes = m.n_holes;
    // the replica in the chosen storage orientation
    ReplicaDesc Rs = R;
    Rs.swap = swap ? 1 : 0;
    Rs.nx = swap ? nz : nx;
    Rs.nz = swap ? nx : nz;
    // links of the replica's moving walls under the new mask, checked before anything changes
    ReplicaHost& H = c->rh[replica];
    std::vector<WallLink> links;
    if (any_solid) links = build_links(Rs, stored_mask.data(), m.info.data(), H.uwall, c->p.rho0);
    if (links_without(c, replica) + (int64_t)links.size() > c->plan.link_cap)
        return fail(c, LB_ERR_CAPACITY, "moving-wall links exceed max_wall_links");
    // rows of this replica go to rows[row_base ...]; clear the old ones first
    for (int64_t k = 0; k < (int64_t)ny * std::max(nx, nz); ++k) {
        c->rowinfo[R.row_base + k] = RowDesc{0, 0, 0, 0};
        c->rows[R.row_base + k] = RowDesc{0, 0, 0, 0};
    }
    HIP_TRY(c, hipMemsetAsync(c->hole + R.base, 0, (size_t)pad_nodes(R.n_nodes), c->stream));
    if (any_solid) {
        for (size_t k = 0; k < m.rows.size(); ++k) c->rows[R.row_base + k] = m.rows[k];
        for (size_t k = 0; k < m.info.size(); ++k) c->rowinfo[R.row_base + k] = m.info[k];
        R.masked = n_holes > 0 ? 2 : 1;
        R.n_fluid = m.stored;                    // stored nodes: fluid nodes and holes
        R.swap = Rs.swap;
        R.nx = Rs.nx;
        R.nz = Rs.nz;
        H.mask.swap(stored_mask);                // in storage order
        if (n_holes > 0)
            HIP_TRY(c, hipMemcpyAsync(c->hole + R.base, m.holes.data(), m.holes.size(),
                                      hipMemcpyHostToDevice, c->stream));
    } else {
        R.masked = 0;
        R.n_fluid = R.n_nodes;
        R.swap = 0;
        R.nx = nx;
        R.nz = nz;
        H.mask.clear();
    }
    R.inv_nx = 1.0 / R.nx;
    R.inv_ny = 1.0 / R.ny;
    H.n_holes = n_holes;
    H.links.swap(links);
    destroy_graphs(c);
    rebuild_tiles(c);
    int rc = upload_tables(c);
    if (rc == LB_OK) rc = upload_links(c);
    if (rc != LB_OK) return rc;
    // bodies already in this replica carry a copy of its geometry (no step has run yet, so
    // the host records are still the bodies' state)
    for (int32_t b : H.bodies) {
        c->bodies0[b].box = body_box(R);
        HIP_TRY(c, hipMemcpyAsync(c->d_bodies + b, &c->bodies0[b], sizeof(Body),
                                  hipMemcpyHostToDevice, c->stream));
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->pose_stale = true;   // the bead records carry the replica geometry
    return init_fluid(c, replica);
}

int lb_set_wall_velocity(lb_ctx* c, int32_t replica, int32_t wall, const double u[3])
{
    if (!c) return LB_ERR_ARG;
    if (!check_replica(c, replica)) return LB_ERR_ARG;
    if (wall < 1 || wall > 255) return fail(c, LB_ERR_ARG, "wall ids are 1..255");
    if (!u || !std::isfinite(u[0]) || !std::isfinite(u[1]) || !std::isfinite(u[2]))
        return fail(c, LB_ERR_ARG, "missing or non-finite wall velocity");
    if (c->step != 0)
        return fail(c, LB_ERR_STATE, "wall velocities can only be set before the first step");
    const ReplicaDesc& R = c->reps[replica];
    ReplicaHost& H = c->rh[replica];
    std::vector<double> uw = H.uwall;
    if (uw.empty()) uw.assign(3 * 256, 0.0);
    for (int a = 0; a < 3; ++a) uw[3 * (size_t)wall + a] = u[a];
    std::vector<WallLink> links;
    if (!H.mask.empty())
        links = build_links(R, H.mask.data(), &c->rowinfo[R.row_base], uw, c->p.rho0);
    if (links_without(c, replica) + (int64_t)links.size() > c->plan.link_cap)
        return fail(c, LB_ERR_CAPACITY, "moving-wall links exceed max_wall_links");
    H.uwall.swap(uw);
    H.links.swap(links);
    destroy_graphs(c);
    int rc = upload_links(c);
    if (rc != LB_OK) return rc;
    return init_fluid(c, replica);
}

int rb_add_raspberry(lb_ctx* c, int32_t replica, const double* offs, int32_t n_beads,
                     double mass, const double inertia[3], const double pos[3],
                     const double quat[4], const double vel[3], const double omega[3],
                     double gamma, int32_t fixed, int32_t* body_id)
{
    if (!c) return LB_ERR_ARG;
    if (!check_replica(c, replica)) return LB_ERR_ARG;
    if (!offs || n_beads < 1 || !pos || !quat || !inertia || !vel || !omega)
        return fail(c, LB_ERR_ARG, "missing body arrays or no beads");
    if (!(gamma >= 0) || !std::isfinite(gamma)) return fail(c, LB_ERR_ARG, "gamma must be >= 0");
    if (!fixed && (!(mass > 0) || !(inertia[0] > 0) || !(inertia[1] > 0) || !(inertia[2] > 0)))
        return fail(c, LB_ERR_ARG, "a free body needs positive mass and inertia");
    const double qn = std::sqrt(quat[0] * quat[0] + quat[1] * quat[1] + quat[2] * quat[2] +
                                quat[3] * quat[3]);
    if (!(qn > 0) || !std::isfinite(qn)) return fail(c, LB_ERR_ARG, "zero quaternion");
    for (int k = 0; k < 3 * n_beads; ++k)
        if (!std::isfinite(offs[k])) return fail(c, LB_ERR_ARG, "non-finite bead offset");
    if (c->n_bodies + 1 > c->plan.body_cap || (int64_t)c->n_beads + n_beads > c->plan.bead_cap)
        return fail(c, LB_ERR_CAPACITY, "body or bead capacity exceeded");
    Body B{};
    for (int a = 0; a < 3; ++a) {
        B.pos[a] = pos[a];
        B.vel[a] = fixed ? 0.0 : vel[a];
        B.omega[a] = fixed ? 0.0 : omega[a];
        B.inertia[a] = inertia[a];
    }
    for (int a = 0; a < 4; ++a) B.quat[a] = quat[a] / qn;
    B.mass = mass;
    B.gamma = gamma;
    B.dt = 1.0 / md_steps(c);
    // a force held over an MD step dt carries the momentum variance 2 kT gamma dt
    B.noise_amp = std::sqrt(2.0 * c->p.kT * gamma / B.dt) * std::sqrt(12.0);
    B.first_ev = 0;
    B.n_ev = 0;
    B.ev_radius = 0.0;
    B.ev_reach = 0.0;
    B.fixed = fixed ? 1 : 0;
    B.replica = replica;
    B.first_bead = c->n_beads;
    B.n_beads = n_beads;
    int32_t in_rep = 0;
    for (int32_t b : c->rh[replica].bodies) in_rep += c->bodies0[b].n_beads;
    B.first_bead_in_replica = in_rep;
    B.box = body_box(c->reps[replica]);
    // store the beads in spatial (Morton) order of their body-frame offsets, so that the 32
    // beads of a coupling workgroup are neighbours and share stencil nodes; each keeps its
    // index in the caller's order (noise stream, per-bead outputs)
    const std::vector<int32_t> order = spatial_order(offs, n_beads);
    std::vector<Bead> beads(n_beads);
    for (int k = 0; k < n_beads; ++k) {
        for (int a = 0; a < 3; ++a) beads[k].off[a] = offs[3 * order[k] + a];
        beads[k].body = c->n_bodies;
        beads[k].user = order[k];
    }
    HIP_TRY(c, hipMemcpyAsync(c->d_bodies + c->n_bodies, &B, sizeof(Body), hipMemcpyHostToDevice,
                              c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->d_beads + c->n_beads, beads.data(), sizeof(Bead) * n_beads,
                              hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (body_id) *body_id = (int32_t)c->rh[replica].bodies.size();
    c->rh[replica].bodies.push_back(c->n_bodies);
    c->bodies0.push_back(B);
    c->n_bodies += 1;
    c->n_beads += n_beads;
    c->bead_user.insert(c->bead_user.end(), order.begin(), order.end());
    c->ev.push_back(EvHost{});
    c->wca_dirty = true;
    c->pose_stale = true;
    destroy_graphs(c);
    return LB_OK;
}

int rb_set_excluded_volume(lb_ctx* c, int32_t replica, int32_t body_id, const double* offs,
                           int32_t n_sites, double radius)
{
    if (!c) return LB_ERR_ARG;
    if (!check_replica(c, replica)) return LB_ERR_ARG;
    const ReplicaHost& H = c->rh[replica];
    if (body_id < 0 || body_id >= (int32_t)H.bodies.size())
        return fail(c, LB_ERR_ARG, "bad body id");
    if (n_sites < 0 || (n_sites > 0 && !offs) || !(radius >= 0.0) || !std::isfinite(radius))
        return fail(c, LB_ERR_ARG, "bad excluded-volume sites");
    for (int64_t k = 0; k < 3 * (int64_t)n_sites; ++k)
        if (!std::isfinite(offs[k])) return fail(c, LB_ERR_ARG, "non-finite site offset");
    if (c->step != 0)
        return fail(c, LB_ERR_STATE, "excluded volume can only be set before the first step");
    const int32_t g = H.bodies[body_id];
    int64_t total = 0;
    for (int32_t b = 0; b < c->n_bodies; ++b)
        if (b != g) total += (int64_t)(c->ev[b].off.size() / 3);
    if (total + n_sites > c->plan.ev_cap)
        return fail(c, LB_ERR_CAPACITY, "excluded-volume sites exceed max_ev_sites");
    c->ev[g].off.assign(offs, offs + 3 * (size_t)n_sites);
    c->ev[g].radius = radius;
    c->wca_dirty = true;
    return LB_OK;
}

int lb_add_wall_sites(lb_ctx* c, int32_t replica, const double* pos, int32_t n, double radius)
{
    if (!c) return LB_ERR_ARG;
    if (!check_replica(c, replica)) return LB_ERR_ARG;
    if (n < 0 || (n > 0 && !pos) || !(radius >= 0.0) || !std::isfinite(radius))
        return fail(c, LB_ERR_ARG, "bad wall sites");
    for (int64_t k = 0; k < 3 * (int64_t)n; ++k)
        if (!std::isfinite(pos[k])) return fail(c, LB_ERR_ARG, "non-finite site position");
    if (c->step != 0)
        return fail(c, LB_ERR_STATE, "wall sites can only be added before the first step");
    int64_t total = 0;
    for (int r = 0; r < c->n_rep; ++r) total += (int64_t)c->rh[r].sites.size();
    if (total + n > c->plan.site_cap)
        return fail(c, LB_ERR_CAPACITY, "wall sites exceed max_wall_sites");
    for (int32_t k = 0; k < n; ++k) {
        WallSite w{};
        for (int a = 0; a < 3; ++a) w.p[a] = pos[3 * (size_t)k + a];
        w.radius = radius;
        c->rh[replica].sites.push_back(w);
    }
    c->n_sites = total + n;
    c->wca_dirty = true;
    return LB_OK;
}

// Before a run of steps: stale body poses and bead records (predicting a current pose again
// reproduces it bit for bit).
int prepare_bodies(lb_ctx* c, hipStream_t s)
{
    if (!c->pose_stale) return LB_OK;
    launch_body_predict(body_args(c), (int)((c->step * md_steps(c)) & 1), s);
    HIP_TRY(c, hipGetLastError());
    c->pose_stale = false;
    return LB_OK;
}

int lb_rb_step(lb_ctx* c, int32_t n_steps)
{
    if (!c) return LB_ERR_ARG;
    if (n_steps < 0) return fail(c, LB_ERR_ARG, "negative step count");
    if (n_steps == 0) return LB_OK;
    if (c->wca_dirty) {
        const int rc = build_wca(c);
        if (rc != LB_OK) return rc;
    }
    int rc = prepare_bodies(c, c->stream);
    if (rc != LB_OK) return rc;
    int32_t left = n_steps;
    const bool use_graph = c->graph_steps > 0 && !c->timing;
    char name[64];
    while (use_graph && left >= c->graph_steps) {
        if (!c->gexec[c->cur]) {
            rc = build_graph(c, c->cur);
            if (rc != LB_OK) return rc;
        }
        // one range per replay: the steps it enqueues
        std::snprintf(name, sizeof name, "lb_rb_step %lld-%lld", (long long)c->step,
                      (long long)(c->step + c->graph_steps - 1));
        Marker m(name);
        launch_set_step(&c->hdr->step, c->step, c->stream);
        HIP_TRY(c, hipGraphLaunch(c->gexec[c->cur], c->stream));
        c->step += c->graph_steps;
        // an even number of steps leaves the current buffer in place
        left -= c->graph_steps;
    }
    for (; left > 0; --left) {
        std::snprintf(name, sizeof name, "lb_rb_step %lld", (long long)c->step);
        Marker m(name);
        HIP_TRY(c, is_f32(c) ? enqueue_step<float>(c, c->stream, c->cur, nullptr, c->step, false)
                             : enqueue_step<double>(c, c->stream, c->cur, nullptr, c->step, false));
        c->cur ^= 1;
        c->step += 1;
    }
    HIP_TRY(c, hipGetLastError());
    return LB_OK;
}

int lb_observables(lb_ctx* c, int32_t replica, lb_totals* out, rb_state* bodies,
                   void* dev_rho_u)
{
    if (!c) return LB_ERR_ARG;
    if (!check_replica(c, replica)) return LB_ERR_ARG;
    const ReplicaDesc& R = c->reps[replica];
    const ReplicaHost& H = c->rh[replica];
    const size_t real = is_f32(c) ? sizeof(float) : sizeof(double);
    if (dev_rho_u)
        HIP_TRY(c, hipMemsetAsync(dev_rho_u, 0, real * 4 * R.n_nodes, c->stream));
    if (is_f32(c)) {
        StepArgs<float> a = step_args<float>(c, H.group, c->cur);
        launch_observe<float>(a, H.group == 1, H.tile0, H.n_tiles, (float*)dev_rho_u,
                              c->d_partials, nullptr, c->stream);
    } else {
        StepArgs<double> a = step_args<double>(c, H.group, c->cur);
        launch_observe<double>(a, H.group == 1, H.tile0, H.n_tiles, (double*)dev_rho_u,
                               c->d_partials, nullptr, c->stream);
    }
    HIP_TRY(c, hipGetLastError());
    std::vector<double> part(5 * (size_t)H.n_tiles);
    if (H.n_tiles > 0)
        HIP_TRY(c, hipMemcpyAsync(part.data(), c->d_partials, sizeof(double) * part.size(),
                                  hipMemcpyDeviceToHost, c->stream));
    std::vector<Body> bs(c->n_bodies);
    if (c->n_bodies > 0)
        HIP_TRY(c, hipMemcpyAsync(bs.data(), c->d_bodies, sizeof(Body) * c->n_bodies,
                                  hipMemcpyDeviceToHost, c->stream));
    DeviceHeader hdr{};
    HIP_TRY(c, hipMemcpyAsync(&hdr, c->hdr, sizeof(DeviceHeader), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    double s[5] = {0, 0, 0, 0, 0};
    for (int32_t t = 0; t < H.n_tiles; ++t)
        for (int k = 0; k < 5; ++k) s[k] += part[5 * (size_t)t + k];
    lb_totals T{};
    T.mass = (double)(R.n_fluid - H.n_holes) * c->p.rho0 + s[0];
    for (int a = 0; a < 3; ++a) T.momentum[a] = s[1 + a];
    for (int32_t b : H.bodies) {
        if (bs[b].fixed) continue;
        for (int a = 0; a < 3; ++a) T.body_momentum[a] += bs[b].mass * bs[b].vel[a];
    }
    T.step = c->step;
    T.finite = (s[4] == 0.0 && std::isfinite(T.mass)) ? 1 : 0;
    if (out) *out = T;
    if (bodies) {
        for (size_t k = 0; k < H.bodies.size(); ++k) {
            const Body& B = bs[H.bodies[k]];
            rb_state& o = bodies[k];
            for (int a = 0; a < 3; ++a) {
                o.pos[a] = B.pos[a]; o.vel[a] = B.vel[a]; o.omega_body[a] = B.omega[a];
                o.force[a] = B.force[a]; o.torque[a] = B.torque[a];
            }
            for (int a = 0; a < 4; ++a) o.quat[a] = B.quat[a];
        }
    }
    if (!T.finite) return fail(c, LB_ERR_UNSTABLE, "non-finite populations");
    if (hdr.err_flags & 1u) return fail(c, LB_ERR_UNSTABLE, "spread force out of range");
    return LB_OK;
}

int rb_record_poses(lb_ctx* c, double* dev_frame)
{
    if (!c) return LB_ERR_ARG;
    if (!dev_frame) return fail(c, LB_ERR_ARG, "missing frame buffer");
    launch_record_poses(c->d_bodies, c->n_bodies, dev_frame, c->stream);
    HIP_TRY(c, hipGetLastError());
    return LB_OK;
}

int lb_body_count(const lb_ctx* c, int32_t replica)
{
    if (!c || replica < 0 || replica >= c->n_rep) return LB_ERR_ARG;
    return (int)c->rh[replica].bodies.size();
}

int rb_bead_forces(lb_ctx* c, int32_t replica, int32_t body_id, double* host_out, int32_t n)
{
    if (!c) return LB_ERR_ARG;
    if (!check_replica(c, replica)) return LB_ERR_ARG;
    const ReplicaHost& H = c->rh[replica];
    if (body_id < 0 || body_id >= (int32_t)H.bodies.size() || !host_out)
        return fail(c, LB_ERR_ARG, "bad body id");
    const Body& B = c->bodies0[H.bodies[body_id]];
    if (n < B.n_beads) return fail(c, LB_ERR_ARG, "output too small");
    std::vector<double> f(3 * (size_t)B.n_beads);
    HIP_TRY(c, hipMemcpyAsync(f.data(), c->d_bead_force + 3 * (int64_t)B.first_bead,
                              sizeof(double) * f.size(), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (int32_t k = 0; k < B.n_beads; ++k) {
        const int32_t u = c->bead_user[B.first_bead + k];
        for (int a = 0; a < 3; ++a) host_out[3 * (size_t)u + a] = f[3 * (size_t)k + a];
    }
    return LB_OK;
}

int lb_export_populations(lb_ctx* c, int32_t replica, double* dev_out)
{
    if (!c) return LB_ERR_ARG;
    if (!check_replica(c, replica) || !dev_out) return fail(c, LB_ERR_ARG, "bad arguments");
    const ReplicaDesc& R = c->reps[replica];
    const ReplicaHost& H = c->rh[replica];
    HIP_TRY(c, hipMemsetAsync(dev_out, 0, sizeof(double) * Q * R.n_nodes, c->stream));
    if (is_f32(c)) {
        StepArgs<float> a = step_args<float>(c, H.group, c->cur);
        launch_observe<float>(a, H.group == 1, H.tile0, H.n_tiles, nullptr, nullptr, dev_out,
                              c->stream);
    } else {
        StepArgs<double> a = step_args<double>(c, H.group, c->cur);
        launch_observe<double>(a, H.group == 1, H.tile0, H.n_tiles, nullptr, nullptr, dev_out,
                               c->stream);
    }
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return LB_OK;
}

int lb_inject_nan(lb_ctx* c, int32_t replica, int32_t x, int32_t y, int32_t z, int32_t i)
{
    if (!c) return LB_ERR_ARG;
    if (!check_replica(c, replica)) return fail(c, LB_ERR_ARG, "bad replica");
    const ReplicaDesc& R = c->reps[replica];
    int box[3];
    box_dims(R, box);
    if (x < 0 || x >= box[0] || y < 0 || y >= box[1] || z < 0 || z >= box[2] || i < 0 || i >= Q)
        return fail(c, LB_ERR_ARG, "node or population out of range");
    if (R.swap) std::swap(x, z);   // storage coordinates
    int64_t local = x + (int64_t)R.nx * (y + (int64_t)R.ny * z);
    if (R.masked) {
        const RowDesc& d = c->rowinfo[R.row_base + y + (int64_t)R.ny * z];
        const ReplicaHost& H = c->rh[replica];
        if (x < d.xlo || x >= d.xlo + d.len || H.mask[local] != 0)
            return fail(c, LB_ERR_ARG, "not a fluid node");
        local = d.start + (x - d.xlo);
    }
    const int64_t slot = pop_at(i, R.base + local);
    static const float nan32 = std::numeric_limits<float>::quiet_NaN();
    static const double nan64 = std::numeric_limits<double>::quiet_NaN();
    if (is_f32(c))
        HIP_TRY(c, hipMemcpyAsync((float*)c->f[c->cur] + slot, &nan32, sizeof(float),
                                  hipMemcpyHostToDevice, c->stream));
    else
        HIP_TRY(c, hipMemcpyAsync((double*)c->f[c->cur] + slot, &nan64, sizeof(double),
                                  hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return LB_OK;
}

int lb_save_state(lb_ctx* c, void* dev_buf, size_t* bytes)
{
    if (!c || !bytes) return LB_ERR_ARG;
    const size_t real = is_f32(c) ? sizeof(float) : sizeof(double);
    const size_t pops = real * Q * c->plan.N;
    const size_t head = 256, bod = align_up(sizeof(Body) * c->n_bodies, 256);
    const size_t need = head + bod + pops;
    if (!dev_buf) { *bytes = need; return LB_OK; }
    if (*bytes < need) return fail(c, LB_ERR_ARG, "state buffer too small");
    // every byte of the state is written (the header and the padding after the bodies as
    // zeros), so that a saved state is a function of the run alone
    uint64_t h[head / sizeof(uint64_t)] = {kStateMagic, (uint64_t)c->step, (uint64_t)c->n_bodies,
                                           (uint64_t)c->p.precision, (uint64_t)c->plan.N,
                                           (uint64_t)c->n_beads};
    char* d = (char*)dev_buf;
    HIP_TRY(c, hipMemcpyAsync(d, h, head, hipMemcpyHostToDevice, c->stream));
    const size_t used = sizeof(Body) * c->n_bodies;
    if (c->n_bodies > 0)
        HIP_TRY(c, hipMemcpyAsync(d + head, c->d_bodies, used, hipMemcpyDeviceToDevice, c->stream));
    if (bod > used) HIP_TRY(c, hipMemsetAsync(d + head + used, 0, bod - used, c->stream));
    HIP_TRY(c, hipMemcpyAsync(d + head + bod, c->f[c->cur], pops, hipMemcpyDeviceToDevice,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    *bytes = need;
    return LB_OK;
}

int lb_load_state(lb_ctx* c, const void* dev_buf, size_t bytes)
{
    if (!c || !dev_buf) return LB_ERR_ARG;
    const size_t real = is_f32(c) ? sizeof(float) : sizeof(double);
    const size_t pops = real * Q * c->plan.N;
    const size_t head = 256, bod = align_up(sizeof(Body) * c->n_bodies, 256);
    if (bytes < head + bod + pops) return fail(c, LB_ERR_ARG, "state buffer too small");
    uint64_t h[6] = {0, 0, 0, 0, 0, 0};
    const char* d = (const char*)dev_buf;
    HIP_TRY(c, hipMemcpyAsync(h, d, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (h[0] != kStateMagic || h[2] != (uint64_t)c->n_bodies || h[3] != (uint64_t)c->p.precision ||
        h[4] != (uint64_t)c->plan.N || h[5] != (uint64_t)c->n_beads)
        return fail(c, LB_ERR_STATE, "state does not match this context");
    if (c->n_bodies > 0)
        HIP_TRY(c, hipMemcpyAsync(c->d_bodies, d + head, sizeof(Body) * c->n_bodies,
                                  hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->f[c->cur], d + head + bod, pops, hipMemcpyDeviceToDevice,
                              c->stream));
    // a spread-force overflow flagged since belongs to the run being replaced
    HIP_TRY(c, hipMemsetAsync(&c->hdr->err_flags, 0, sizeof(uint32_t), c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->step = (int64_t)h[1];
    c->pose_stale = true;
    return LB_OK;
}

int lb_set_store_policy(lb_ctx* c, int32_t policy)
{
    if (!c) return LB_ERR_ARG;
    if (policy != LB_STORES_AUTO && policy != LB_STORES_CACHED && policy != LB_STORES_STREAMING)
        return fail(c, LB_ERR_ARG, "unknown store policy");
    destroy_graphs(c);
    c->store_policy = policy;
    return LB_OK;
}

int lb_autotune(lb_ctx* c, int32_t repeats)
{
    if (!c) return LB_ERR_ARG;
    if (repeats < 0 || repeats > 1000) return fail(c, LB_ERR_ARG, "repeats must be 0..1000");
    if (c->wca_dirty) {
        const int rc = build_wca(c);
        if (rc != LB_OK) return rc;
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const std::string key = tune_key(c);
    if (repeats == 0) {
        std::lock_guard<std::mutex> lock(tune_mutex());
        auto it = tune_cache().find(key);
        if (it != tune_cache().end()) {
            destroy_graphs(c);
            c->tune = it->second;
            return LB_OK;
        }
    }
    Tuning t;
    Marker m("lb_autotune");
    const int rc = is_f32(c) ? autotune_t<float>(c, repeats > 0 ? repeats : 3, t)
                             : autotune_t<double>(c, repeats > 0 ? repeats : 3, t);
    destroy_graphs(c);
    if (rc != LB_OK) return rc;
    std::lock_guard<std::mutex> lock(tune_mutex());
    tune_cache()[key] = t;
    return LB_OK;
}

int lb_get_tuning(const lb_ctx* c, lb_tuning* out)
{
    if (!c || !out) return LB_ERR_ARG;
    lb_tuning t{};
    t.tuned = c->tune.tuned ? 1 : 0;
    t.tiles_per_wg = std::max(1, (int)c->tune.tiles_per_wg);
    t.wg_per_cu = c->tune.wg_per_cu;
    t.streaming = streaming_stores(c) ? 1 : 0;
    t.candidates = c->tune.candidates;
    t.node_us_default = c->tune.us_default;
    t.node_us_tuned = c->tune.us_best;
    *out = t;
    return LB_OK;
}

int lb_set_tuning(lb_ctx* c, const lb_tuning* t)
{
    if (!c || !t) return LB_ERR_ARG;
    if ((t->tiles_per_wg != 1 && t->tiles_per_wg != kWideTiles) || t->wg_per_cu < 0 ||
        t->wg_per_cu > 32 || (t->streaming != 0 && t->streaming != 1))
        return fail(c, LB_ERR_ARG, "tiles_per_wg 1 or 4, wg_per_cu 0..32, streaming 0 or 1");
    destroy_graphs(c);
    Tuning x{};
    x.tuned = true;
    x.tiles_per_wg = t->tiles_per_wg;
    x.wg_per_cu = t->wg_per_cu;
    x.streaming = t->streaming;
    c->tune = x;
    return LB_OK;
}

int lb_set_graph_steps(lb_ctx* c, int32_t k)
{
    if (!c) return LB_ERR_ARG;
    if (k < 0 || (k > 0 && (k < 2 || (k & 1)))) return fail(c, LB_ERR_ARG, "graph steps must be 0 or even >= 2");
    destroy_graphs(c);
    c->graph_steps = k;
    return LB_OK;
}

int lb_set_timing(lb_ctx* c, int32_t enable)
{
    if (!c) return LB_ERR_ARG;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (auto& e : c->ev_node) c->ev_pool.push_back(e);
    for (auto& e : c->ev_couple_t) c->ev_pool.push_back(e);
    c->ev_node.clear();
    c->ev_couple_t.clear();
    c->timing = enable != 0;
    return LB_OK;
}

int lb_kernel_times(lb_ctx* c, double* node_ms, int64_t* node_n, double* couple_ms,
                    int64_t* couple_n)
{
    if (!c) return LB_ERR_ARG;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    double tn = 0, tc = 0;
    for (auto& e : c->ev_node) { float ms = 0; HIP_TRY(c, hipEventElapsedTime(&ms, e.a, e.b)); tn += ms; }
    for (auto& e : c->ev_couple_t) { float ms = 0; HIP_TRY(c, hipEventElapsedTime(&ms, e.a, e.b)); tc += ms; }
    if (node_ms) *node_ms = tn;
    if (node_n) *node_n = (int64_t)c->ev_node.size();
    if (couple_ms) *couple_ms = tc;
    if (couple_n) *couple_n = (int64_t)c->ev_couple_t.size();
    return LB_OK;
}

int lb_row_axis(const lb_ctx* c, int32_t replica, int32_t* axis)
{
    if (!c || replica < 0 || replica >= c->n_rep || !axis) return LB_ERR_ARG;
    *axis = c->reps[replica].swap ? 2 : 0;
    return LB_OK;
}

int lb_node_counts(const lb_ctx* c, int32_t replica, int64_t* n_nodes, int64_t* n_fluid)
{
    if (!c || replica < 0 || replica >= c->n_rep) return LB_ERR_ARG;
    if (n_nodes) *n_nodes = c->reps[replica].n_nodes;
    if (n_fluid) *n_fluid = c->reps[replica].n_fluid - c->rh[replica].n_holes;
    return LB_OK;
}

void lb_destroy(lb_ctx* c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    destroy_graphs(c);
    for (auto& e : c->ev_node) c->ev_pool.push_back(e);
    for (auto& e : c->ev_couple_t) c->ev_pool.push_back(e);
    for (auto& e : c->ev_pool) {
        if (e.a) (void)hipEventDestroy(e.a);
        if (e.b) (void)hipEventDestroy(e.b);
    }
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    delete c;
}

size_t lb_adjoint_workspace_bytes(const lb_ctx* c, int32_t n_steps, int32_t checkpoint_every)
{
    AdjPlan ap;
    if (!make_adj_plan(c, n_steps, checkpoint_every, ap)) return 0;
    return ap.total;
}

int lb_rb_adjoint(lb_ctx* c, int32_t n_steps, int32_t checkpoint_every, void* dev_ws,
                  size_t ws_bytes, const double* dJ_dF, double* J, double* dJ_dgamma,
                  double* dJ_doffsets)
{
    if (!c) return LB_ERR_ARG;
    AdjPlan ap;
    if (!make_adj_plan(c, n_steps, checkpoint_every, ap))
        return fail(c, LB_ERR_ARG, "the window needs n_steps >= 1 and checkpoint_every >= 1");
    if (!dev_ws || ((uintptr_t)dev_ws % kAlign) != 0 || ws_bytes < ap.total)
        return fail(c, LB_ERR_ARG, "reverse-pass workspace missing, misaligned or too small");
    if (c->wca_dirty) {
        const int rc = build_wca(c);
        if (rc != LB_OK) return rc;
    }
    if (c->n_bodies > 0 && (!dJ_dF || !dJ_dgamma || !dJ_doffsets))
        return fail(c, LB_ERR_ARG, "missing objective weights or gradient outputs");
    char* ws = (char*)dev_ws;
    hipStream_t s = c->stream;
    const size_t nb = (size_t)std::max<int32_t>(c->n_beads, 1);
    if (c->n_bodies > 0)
        HIP_TRY(c, hipMemcpyAsync(ws + ap.off_w, dJ_dF, sizeof(double) * 3 * c->n_bodies * (size_t)n_steps,
                                  hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemsetAsync(ws + ap.off_lam0, 0, ap.state, s));
    HIP_TRY(c, hipMemsetAsync(ws + ap.off_lam1, 0, ap.state, s));
    HIP_TRY(c, hipMemsetAsync(ws + ap.off_dr, 0, sizeof(double) * 3 * nb, s));
    HIP_TRY(c, hipMemsetAsync(ws + ap.off_dg, 0, sizeof(double) * nb, s));
    HIP_TRY(c, hipMemsetAsync(ws + ap.off_J, 0, sizeof(double) * nb, s));
    if (body_passes(c)) {
        const size_t nbod = (size_t)std::max<int32_t>(c->n_bodies, 1);
        HIP_TRY(c, hipMemsetAsync(ws + ap.off_badj, 0, sizeof(double) * kBodyAdjWords * nbod, s));
        HIP_TRY(c, hipMemsetAsync(ws + ap.off_zero, 0, sizeof(double) * 3 * nbod, s));
        HIP_TRY(c, hipMemsetAsync(ws + ap.off_wadj, 0, sizeof(double) * 6 * nbod, s));
        HIP_TRY(c, hipMemsetAsync(ws + ap.off_Jb, 0, sizeof(double) * nbod, s));
    }
    {
        const int rc = prepare_bodies(c, s);
        if (rc != LB_OK) return rc;
    }
    const int parity = (int)(c->step & 1);
    Marker m("lb_rb_adjoint");
    const int rc = is_f32(c) ? run_adjoint<float>(c, n_steps, checkpoint_every, ws, ap)
                             : run_adjoint<double>(c, n_steps, checkpoint_every, ws, ap);
    if (rc != LB_OK) return rc;
    std::vector<double> dr(3 * nb), dg(nb), jp(nb);
    std::vector<Body> bs(c->n_bodies);
    HIP_TRY(c, hipMemcpyAsync(dr.data(), ws + ap.off_dr, sizeof(double) * dr.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipMemcpyAsync(dg.data(), ws + ap.off_dg, sizeof(double) * dg.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipMemcpyAsync(jp.data(), ws + ap.off_J, sizeof(double) * jp.size(), hipMemcpyDeviceToHost, s));
    if (c->n_bodies > 0)
        HIP_TRY(c, hipMemcpyAsync(bs.data(), c->d_bodies, sizeof(Body) * c->n_bodies,
                                  hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    double Jsum = 0.0;
    for (int32_t k = 0; k < c->n_beads; ++k) Jsum += jp[k];
    if (body_passes(c) && c->n_bodies > 0) {   // the body passes took J from the body forces
        std::vector<double> jb(c->n_bodies);
        HIP_TRY(c, hipMemcpy(jb.data(), ws + ap.off_Jb, sizeof(double) * jb.size(), hipMemcpyDeviceToHost));
        for (double v : jb) Jsum += v;
    }
    if (J) *J = Jsum;
    const bool body_frame = body_passes(c);   // the bead pass then accumulated body-frame values
    for (int32_t b = 0; b < c->n_bodies; ++b) {
        const Body& B = bs[b];
        const double* R = B.pose[parity].rot;   // body -> lab; a fixed body keeps one pose
        double g = 0.0;
        for (int32_t k = B.first_bead; k < B.first_bead + B.n_beads; ++k) {
            g += dg[k];
            const double* d = &dr[3 * (size_t)k];
            const size_t u = (size_t)B.first_bead + c->bead_user[k];   // caller's order
            for (int a = 0; a < 3; ++a)
                dJ_doffsets[3 * u + a] =
                    body_frame ? d[a] : R[a] * d[0] + R[3 + a] * d[1] + R[6 + a] * d[2];
        }
        dJ_dgamma[b] = g;
    }
    return LB_OK;
}

const char* lb_last_error(const lb_ctx* c)
{
    if (!c) return "null context";
    return c->err.c_str();
}

}  // extern "C"
