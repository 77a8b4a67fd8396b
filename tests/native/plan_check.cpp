// plan_check.cpp -- the library's host-only planners (paper_1604_01829_amd/csrc/lbrb_plan.cpp)
// against brute-force definitions, built with AddressSanitizer and UndefinedBehaviorSanitizer
// by tests/test_sanitizers.py.  Exits 0 when every check holds; prints the first failure.
//
//   compress_mask  rows, spans, holes and stored counts of random and degenerate masks
//   append_tiles   tiles cover the stored nodes in order, each with the rows it overlaps
//   build_links    the moving-wall links equal the set enumerated node by node
//   spatial_order  a permutation with non-decreasing Morton keys, stable for equal keys
//   wca_grid       every site within range of a point is in the point's neighbourhood list,
//                  every point within range of a site lies in a flagged fine cell
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <tuple>
#include <vector>

#include "../../paper_1604_01829_amd/csrc/lbrb_plan.h"

using namespace lbrb;

#define CHECK(cond, ...)                                                  \
    do {                                                                  \
        if (!(cond)) {                                                    \
            std::fprintf(stderr, "FAIL %s:%d: %s: ", __FILE__, __LINE__, #cond); \
            std::fprintf(stderr, __VA_ARGS__);                            \
            std::fprintf(stderr, "\n");                                   \
            std::exit(1);                                                 \
        }                                                                 \
    } while (0)

// the 19 D3Q19 velocities, written out here (rest, 6 faces, 12 edges)
static const int C19[19][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                               {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                               {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                               {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static std::vector<uint8_t> random_mask(std::mt19937_64& rng, int nx, int ny, int nz, int kind)
{
    std::vector<uint8_t> m((size_t)nx * ny * nz, 0);
    std::uniform_real_distribution<double> u(0.0, 1.0);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                uint8_t v = 0;
                switch (kind) {
                case 0: v = 0; break;                                    // all fluid
                case 1: v = 1; break;                                    // all solid
                case 2: v = u(rng) < 0.3 ? (uint8_t)(1 + (x + y) % 3) : 0; break;   // porous
                case 3: {                                                // a pore along x
                    const double dy = y + 0.5 - ny / 2.0, dz = z + 0.5 - nz / 2.0;
                    v = dy * dy + dz * dz > 0.2 * ny * nz ? 2 : 0;
                    break;
                }
                default:                                                 // slabs: several runs
                    v = (x % 5 == 2 || (y == 0 && z % 2 == 0)) ? 4 : 0;
                }
                m[x + (size_t)nx * (y + (size_t)ny * z)] = v;
            }
    return m;
}

static void check_mask(const std::vector<uint8_t>& mask, int nx, int ny, int nz,
                       const MaskRows& mr)
{
    CHECK(mr.info.size() == (size_t)ny * nz, "info size");
    int64_t stored = 0, holes = 0;
    size_t row = 0;
    bool any = false;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y) {
            const uint8_t* m = &mask[(size_t)nx * (y + (size_t)ny * z)];
            int first = -1, last = -1;
            for (int x = 0; x < nx; ++x) {
                if (m[x]) any = true;
                else { if (first < 0) first = x; last = x; }
            }
            const RowDesc& d = mr.info[(size_t)y + (size_t)ny * z];
            if (first < 0) { CHECK(d.len == 0, "row (%d,%d) has no fluid", y, z); continue; }
            CHECK(d.xlo == first && d.len == last - first + 1 && d.start == stored &&
                      d.yz == (y | (z << 16)),
                  "row (%d,%d): %d %d %d", y, z, d.xlo, d.len, d.start);
            CHECK(row < mr.rows.size() && mr.rows[row].start == d.start &&
                      mr.rows[row].yz == d.yz,
                  "rows[%zu]", row);
            ++row;
            for (int x = first; x <= last; ++x) {
                CHECK(mr.holes[(size_t)stored + (x - first)] == m[x], "hole byte");
                if (m[x]) ++holes;
            }
            stored += d.len;
        }
    CHECK(row == mr.rows.size(), "row count");
    CHECK(stored == mr.stored && (int64_t)mr.holes.size() == stored, "stored");
    CHECK(holes == mr.n_holes && any == mr.any_solid, "holes / any_solid");
}

static ReplicaDesc replica(int nx, int ny, int nz, const MaskRows& mr, int64_t base, int row_base)
{
    ReplicaDesc R{};
    R.nx = nx; R.ny = ny; R.nz = nz;
    R.masked = mr.any_solid ? (mr.n_holes ? 2 : 1) : 0;
    R.base = base;
    R.n_nodes = (int64_t)nx * ny * nz;
    R.n_fluid = mr.any_solid ? mr.stored : R.n_nodes;
    R.row_base = row_base;
    return R;
}

static void check_tiles(const ReplicaDesc& R, const std::vector<RowDesc>& rows,
                        const std::vector<RowDesc>& info)
{
    std::vector<NodeTile> T(3);   // tiles already in the list stay untouched
    append_tiles(R, 7, rows.data(), info.data(), T);
    const int64_t n = R.n_fluid;
    CHECK((int64_t)T.size() - 3 == (n + kNodeBlock - 1) / kNodeBlock, "tile count");
    int64_t next = 0;
    for (size_t k = 3; k < T.size(); ++k) {
        const NodeTile& t = T[k];
        CHECK(t.replica == 7 && t.begin == next && t.count >= 1 && t.count <= kNodeBlock,
              "tile %zu", k);
        CHECK(t.count == kNodeBlock || k + 1 == T.size(), "only the last tile is ragged");
        CHECK(t.gt == (int32_t)((R.base + t.begin) >> kPopBlockLog), "gt");
        next += t.count;
        if (!R.masked) continue;
        // the rows holding the tile's first and last node
        auto row_of = [&](int64_t local) {
            int found = -1;
            for (size_t r = R.row_base; r < rows.size(); ++r)
                if (rows[r].len > 0 && rows[r].start <= local &&
                    local < (int64_t)rows[r].start + rows[r].len)
                    found = (int)r;
            return found;
        };
        CHECK(t.row_lo == row_of(t.begin) && t.row_hi == row_of(t.begin + t.count - 1),
              "tile %zu rows %d..%d", k, t.row_lo, t.row_hi);
    }
    CHECK(next == n, "tiles cover the stored nodes");
}

// The links of a replica whose mask is given in the box's order; with swap the replica is
// stored with axes x and z exchanged (mask, rows and R in storage coordinates), while the
// expected links are enumerated in box coordinates and mapped to the storage node.
static void check_links(const ReplicaDesc& Rbox, const std::vector<uint8_t>& mask,
                        const MaskRows& mr_box, std::mt19937_64& rng, bool swap)
{
    ReplicaDesc R = Rbox;
    MaskRows mr = mr_box;
    std::vector<uint8_t> smask = mask;
    if (swap) {
        const int bx = Rbox.nx, by = Rbox.ny, bz = Rbox.nz;
        for (int z = 0; z < bz; ++z)
            for (int y = 0; y < by; ++y)
                for (int x = 0; x < bx; ++x)
                    smask[z + (size_t)bz * (y + (size_t)by * x)] = mask[x + (size_t)bx * (y + (size_t)by * z)];
        mr = compress_mask(bz, by, bx, smask.data());
        check_mask(smask, bz, by, bx, mr);
        R.nx = bz;
        R.nz = bx;
        R.swap = 1;
        R.n_fluid = mr.stored;
    }
    std::vector<double> uwall(256 * 3, 0.0);
    std::uniform_real_distribution<double> u(-1e-2, 1e-2);
    for (int k : {2, 4})
        for (int a = 0; a < 3; ++a) uwall[3 * k + a] = u(rng);
    uwall[3 * 3 + 1] = 5e-3;   // wall 3 moves along y only: links with c_i . u = 0 drop out
    const double rho0 = 1.25;
    const std::vector<WallLink> got = build_links(R, smask.data(), mr.info.data(), uwall, rho0);
    // a link: (node, direction of the reflected population, delta); the direction -c_i is
    // compared as a vector, so the check does not depend on the library's velocity order
    typedef std::tuple<int64_t, int, int, int, double> Link;
    std::set<Link> want, have;
    const int nx = Rbox.nx, ny = Rbox.ny, nz = Rbox.nz;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                if (mask[x + (size_t)nx * (y + (size_t)ny * z)]) continue;
                // the node's storage coordinates and row
                const int sx = swap ? z : x, sz = swap ? x : z;
                const RowDesc& d = mr.info[(size_t)y + (size_t)ny * sz];
                for (int i = 1; i < 19; ++i) {
                    const int* c = C19[i];
                    const int bx = ((x - c[0]) % nx + nx) % nx;
                    const int by = ((y - c[1]) % ny + ny) % ny;
                    const int bz = ((z - c[2]) % nz + nz) % nz;
                    const int k = mask[bx + (size_t)nx * (by + (size_t)ny * bz)];
                    if (!k) continue;
                    const double cu =
                        c[0] * uwall[3 * k] + c[1] * uwall[3 * k + 1] + c[2] * uwall[3 * k + 2];
                    if (cu == 0.0) continue;
                    const int c2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
                    const double w = c2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0;
                    want.emplace(R.base + d.start + (sx - d.xlo), -c[0], -c[1], -c[2],
                                 6.0 * w * rho0 * cu);
                }
            }
    for (size_t k = 0; k < got.size(); ++k) {
        const int p = got[k].pop;
        have.emplace(got[k].g, cx_of(p), cy_of(p), cz_of(p), got[k].delta);
        if (k) CHECK(pop_at(got[k - 1].pop, got[k - 1].g) < pop_at(got[k].pop, got[k].g),
                     "links sorted by slot, each slot once");
    }
    CHECK(have.size() == got.size() && have.size() == want.size(), "%zu links, want %zu",
          got.size(), want.size());
    for (auto a = have.begin(), b = want.begin(); a != have.end(); ++a, ++b)
        CHECK(std::get<0>(*a) == std::get<0>(*b) && std::get<1>(*a) == std::get<1>(*b) &&
                  std::get<2>(*a) == std::get<2>(*b) && std::get<3>(*a) == std::get<3>(*b) &&
                  std::fabs(std::get<4>(*a) - std::get<4>(*b)) <= 1e-15,
              "link");
}

static uint64_t morton_brute(const double* p, const double lo[3])
{
    uint64_t key = 0;
    uint64_t q[3];
    for (int a = 0; a < 3; ++a) q[a] = (uint64_t)std::floor((p[a] - lo[a]) * 2.0);
    // bit b of axis a goes to bit 3b + a
    for (int b = 20; b >= 0; --b)
        for (int a = 2; a >= 0; --a) key = (key << 1) | ((q[a] >> b) & 1u);
    return key;
}

static void check_order(std::mt19937_64& rng)
{
    for (int n : {0, 1, 2, 57, 400}) {
        std::vector<double> off(3 * (size_t)n);
        std::uniform_real_distribution<double> u(-6.0, 6.0);
        for (double& v : off) v = std::round(u(rng) * 4.0) / 4.0;   // ties on purpose
        const std::vector<int32_t> ord = spatial_order(off.data(), n);
        CHECK((int)ord.size() == n, "order size");
        std::vector<int> seen(n, 0);
        double lo[3] = {1e9, 1e9, 1e9};
        for (int k = 0; k < n; ++k)
            for (int a = 0; a < 3; ++a) lo[a] = std::min(lo[a], off[3 * k + a]);
        for (int k = 0; k < n; ++k) {
            CHECK(ord[k] >= 0 && ord[k] < n && !seen[ord[k]]++, "permutation");
            if (k) {
                const uint64_t a = morton_brute(&off[3 * ord[k - 1]], lo),
                               b = morton_brute(&off[3 * ord[k]], lo);
                CHECK(a < b || (a == b && ord[k - 1] < ord[k]), "Morton order, stable");
            }
        }
    }
}

static int cell_of(double x, double L, double w, int n)
{
    const double xw = x - L * std::floor(x / L);
    const int q = (int)(xw / w);
    return q < 0 ? 0 : (q >= n ? n - 1 : q);
}

static void check_wca(std::mt19937_64& rng)
{
    const double cut = std::pow(2.0, 1.0 / 6.0);
    WcaTables t;
    struct Case { int d[3]; double ev_r, site_r; int n_sites; } cases[] = {
        {{24, 20, 30}, 1.0, 0.7, 300}, {{8, 40, 9}, 1.2, 0.5, 80}, {{64, 64, 64}, 0.5, 0.5, 900},
        {{7, 7, 7}, 1.0, 0.6, 20}};
    for (const Case& cs : cases) {
        std::uniform_real_distribution<double> ux(-0.5, cs.d[0] + 0.5), uy(0, cs.d[1]),
            uz(0, cs.d[2]);
        std::vector<WallSite> sites(cs.n_sites);
        for (WallSite& s : sites) {
            s.p[0] = ux(rng); s.p[1] = uy(rng); s.p[2] = uz(rng);   // some outside [0, L)
            s.radius = cs.site_r;
        }
        WcaRep W{};
        const size_t cells_before = t.nb_start.size(), fine_before = t.near.size();
        CHECK(wca_grid(cs.d, cs.ev_r, sites, W, t), "grid");
        CHECK(W.cell0 == (int32_t)cells_before && W.fine0 == (int32_t)fine_before, "offsets");
        const int ncell = W.cx * W.cy * W.cz;
        CHECK(t.nb_start.size() == cells_before + ncell + 1, "nb_start size");
        for (int k = 0; k < ncell; ++k)
            CHECK(t.nb_start[cells_before + k] <= t.nb_start[cells_before + k + 1], "monotone");
        CHECK(t.nb_start.back() == (int32_t)t.nb_sites.size(), "end");
        CHECK(t.near.size() == fine_before + (size_t)W.gx * W.gy * W.gz, "near size");
        const double range = std::max(cut * 2.0 * cs.ev_r, cut * (cs.ev_r + cs.site_r));
        for (int a = 0; a < 3; ++a) CHECK(W.cw[a] >= range && W.fw[a] <= 2.0, "cell widths");
        std::uniform_real_distribution<double> px(0, cs.d[0]), py(0, cs.d[1]), pz(0, cs.d[2]);
        for (int q = 0; q < 4000; ++q) {
            const double p[3] = {px(rng), py(rng), pz(rng)};
            const int c = cell_of(p[0], cs.d[0], W.cw[0], W.cx) +
                          W.cx * (cell_of(p[1], cs.d[1], W.cw[1], W.cy) +
                                  W.cy * cell_of(p[2], cs.d[2], W.cw[2], W.cz));
            const int32_t b = t.nb_start[W.cell0 + c], e = t.nb_start[W.cell0 + c + 1];
            int fine[3];
            for (int a = 0; a < 3; ++a)
                fine[a] = std::min((int)(p[a] / W.fw[a]), (a == 0 ? W.gx : a == 1 ? W.gy : W.gz) - 1);
            const bool flagged =
                t.near[W.fine0 + fine[0] + (size_t)W.gx * (fine[1] + (size_t)W.gy * fine[2])] != 0;
            for (const WallSite& s : sites) {
                double d2 = 0.0;
                for (int a = 0; a < 3; ++a) {
                    double dd = p[a] - s.p[a];
                    dd -= cs.d[a] * std::round(dd / cs.d[a]);
                    d2 += dd * dd;
                }
                const double r = cut * (cs.ev_r + s.radius);
                if (d2 >= r * r) continue;
                CHECK(flagged, "a point within range of a site lies in an unflagged fine cell");
                int count = 0;
                for (int32_t k = b; k < e; ++k)
                    if (t.nb_sites[k].p[0] == s.p[0] && t.nb_sites[k].p[1] == s.p[1] &&
                        t.nb_sites[k].p[2] == s.p[2])
                        ++count;
                CHECK(count == 1, "site in the neighbourhood list %d times", count);
            }
        }
    }
    // a side shorter than twice the range is refused; no sites or no body sites: no grid
    WcaRep W{};
    const int small[3] = {3, 30, 30};
    CHECK(!wca_grid(small, 1.0, std::vector<WallSite>(1, WallSite{{1, 1, 1}, 1.0}), W, t),
          "short side");
    const int dims[3] = {20, 20, 20};
    const size_t before = t.nb_start.size();
    CHECK(wca_grid(dims, 1.0, {}, W, t) && wca_grid(dims, -1.0, {WallSite{{1, 1, 1}, 1}}, W, t) &&
              t.nb_start.size() == before,
          "no grid needed");
}

int main()
{
    std::mt19937_64 rng(1604);
    const int shapes[][3] = {{1, 1, 1}, {1, 5, 3}, {7, 1, 1}, {13, 11, 9}, {40, 6, 5},
                             {32, 32, 32}, {300, 2, 2}};
    int n_cases = 0;
    for (const auto& s : shapes)
        for (int kind = 0; kind < 5; ++kind) {
            const int nx = s[0], ny = s[1], nz = s[2];
            const std::vector<uint8_t> mask = random_mask(rng, nx, ny, nz, kind);
            const MaskRows mr = compress_mask(nx, ny, nz, mask.data());
            check_mask(mask, nx, ny, nz, mr);
            // the replica's rows placed after another replica's (row_base 5), base 3 tiles in
            const int row_base = 5;
            std::vector<RowDesc> rows(row_base, RowDesc{}), info(row_base, RowDesc{});
            rows.resize(row_base + (size_t)ny * nz, RowDesc{});
            std::copy(mr.rows.begin(), mr.rows.end(), rows.begin() + row_base);
            info.insert(info.end(), mr.info.begin(), mr.info.end());
            const ReplicaDesc R = replica(nx, ny, nz, mr, 3 * kNodeBlock, row_base);
            if (R.n_fluid > 0) check_tiles(R, rows, info);
            if (mr.any_solid) {
                check_links(R, mask, mr, rng, false);
                check_links(R, mask, mr, rng, true);
            }
            ++n_cases;
        }
    check_order(rng);
    check_wca(rng);
    std::printf("plan_check: %d masks, orders and site grids ok\n", n_cases);
    return 0;
}
