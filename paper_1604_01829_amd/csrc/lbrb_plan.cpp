// lbrb_plan.cpp -- host-only planners (declared in lbrb_plan.h): mask compression, node tiles,
// moving-wall links, bead order and excluded-volume grids.  No HIP call: the library uploads
// what these build.
#include "lbrb_plan.h"

#include <algorithm>
#include <cmath>

namespace lbrb {

int cells_per_axis_cap(int n) { return std::min(n, kMaxCellsPerAxis); }
int fine_per_axis(int n) { return (int)std::ceil(n / kFineCell); }

MaskRows compress_mask(int nx, int ny, int nz, const uint8_t* mask)
{
    MaskRows m;
    m.info.assign((size_t)ny * nz, RowDesc{0, 0, 0, 0});
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y) {
            const uint8_t* row = mask + (size_t)nx * (y + (size_t)ny * z);
            int xlo = -1, xhi = -1;
            for (int x = 0; x < nx; ++x) {
                if (row[x]) { m.any_solid = true; continue; }
                if (xlo < 0) xlo = x;
                xhi = x;
            }
            if (xlo < 0) continue;
            RowDesc d{};
            d.start = (int32_t)m.stored;
            d.xlo = xlo;
            d.len = xhi - xlo + 1;
            d.yz = y | (z << 16);
            m.info[(size_t)y + (size_t)ny * z] = d;
            m.rows.push_back(d);
            for (int x = xlo; x <= xhi; ++x) {
                m.holes.push_back(row[x]);
                if (row[x]) ++m.n_holes;
            }
            m.stored += d.len;
        }
    return m;
}

void append_tiles(const ReplicaDesc& R, int32_t r, const RowDesc* rows, const RowDesc* rowinfo,
                  std::vector<NodeTile>& T)
{
    const int64_t n = R.n_fluid;
    int row = R.row_base;   // first row of the replica (masked)
    int last_row = row;
    if (R.masked) {
        // rows of this replica are rows[row_base .. row_base + n_rows)
        int64_t nr = 0;
        for (int64_t k = 0; k < (int64_t)R.ny * R.nz; ++k)
            if (rowinfo[R.row_base + k].len > 0) ++nr;
        last_row = R.row_base + (int)nr - 1;
    }
    for (int64_t b = 0; b < n; b += kNodeBlock) {
        NodeTile t{};
        t.replica = r;
        t.begin = b;
        t.count = (int32_t)std::min<int64_t>(kNodeBlock, n - b);
        const int64_t e = b + t.count - 1;   // last local index of the tile
        if (R.masked) {
            while (row < last_row && rows[row + 1].start <= b) ++row;
            int rh = row;
            while (rh < last_row && rows[rh + 1].start <= e) ++rh;
            t.row_lo = row;
            t.row_hi = rh;
        }
        t.gt = (int32_t)((R.base + b) >> kPopBlockLog);
        T.push_back(t);
    }
}

std::vector<WallLink> build_links(const ReplicaDesc& R, const uint8_t* mask, const RowDesc* info,
                                  const std::vector<double>& uwall, double rho0)
{
    std::vector<WallLink> out;
    if (!mask || uwall.empty()) return out;
    const int nx = R.nx, ny = R.ny, nz = R.nz;
    auto wrapi = [](int v, int n) { v %= n; return v < 0 ? v + n : v; };
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y) {
            const RowDesc& row = info[(size_t)y + (size_t)ny * z];
            for (int x = row.xlo; x < row.xlo + row.len; ++x) {
                if (mask[x + (size_t)nx * (y + (size_t)ny * z)]) continue;   // a hole
                for (int i = 1; i < Q; ++i) {
                    // c_i in storage coordinates (axes x and z exchanged when R.swap)
                    const int sx = R.swap ? cz_of(i) : cx_of(i);
                    const int sz = R.swap ? cx_of(i) : cz_of(i);
                    const int bx = wrapi(x - sx, nx), by = wrapi(y - cy_of(i), ny),
                              bz = wrapi(z - sz, nz);
                    const uint8_t k = mask[bx + (size_t)nx * (by + (size_t)ny * bz)];
                    if (!k) continue;
                    const double* u = &uwall[3 * (size_t)k];
                    const double cu = cx_of(i) * u[0] + cy_of(i) * u[1] + cz_of(i) * u[2];
                    if (cu == 0.0) continue;
                    WallLink L{};
                    L.g = R.base + row.start + (x - row.xlo);
                    L.pop = opposite_of(i);
                    L.delta = 6.0 * weight_of(i) * rho0 * cu;
                    out.push_back(L);
                }
            }
        }
    // in storage order of the slots they update
    std::sort(out.begin(), out.end(), [](const WallLink& a, const WallLink& b) {
        return pop_at(a.pop, a.g) < pop_at(b.pop, b.g);
    });
    return out;
}

std::vector<int32_t> spatial_order(const double* offs, int32_t n)
{
    if (n <= 0) return {};
    double lo[3] = {offs[0], offs[1], offs[2]};
    for (int32_t k = 1; k < n; ++k)
        for (int a = 0; a < 3; ++a) lo[a] = std::min(lo[a], offs[3 * k + a]);
    std::vector<uint64_t> key(n);
    for (int32_t k = 0; k < n; ++k) {
        uint64_t m = 0;
        for (int a = 0; a < 3; ++a) {
            const uint64_t q =
                (uint64_t)std::min(2097151.0, std::floor((offs[3 * k + a] - lo[a]) * 2.0));
            for (int bit = 0; bit < 21; ++bit) m |= ((q >> bit) & 1ull) << (3 * bit + a);
        }
        key[k] = m;
    }
    std::vector<int32_t> order(n);
    for (int32_t k = 0; k < n; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t x, int32_t y) { return key[x] < key[y]; });
    return order;
}

bool wca_grid(const int dims[3], double ev_r, const std::vector<WallSite>& sites_in, WcaRep& W,
              WcaTables& t)
{
    const double cut = std::pow(2.0, 1.0 / 6.0);
    // the largest range of a pair in this replica: body-body and body-site
    double range = ev_r >= 0.0 ? cut * 2.0 * ev_r : 0.0;
    double site_r = -1.0;
    for (const WallSite& w : sites_in) site_r = std::max(site_r, w.radius);
    if (ev_r >= 0.0 && site_r >= 0.0) range = std::max(range, cut * (ev_r + site_r));
    for (int a = 0; a < 3; ++a)
        if (ev_r >= 0.0 && 2.0 * range > dims[a]) return false;
    if (sites_in.empty() || ev_r < 0.0) return true;   // no grid needed
    // coarse grid, sites binned by cell (the kernel's cell rule)
    int nc[3], ng[3];
    for (int a = 0; a < 3; ++a) {
        const int fit = (int)std::floor(dims[a] / (range * (1.0 + 1e-6)));
        nc[a] = std::max(1, std::min(fit, cells_per_axis_cap(dims[a])));
        W.cw[a] = (double)dims[a] / nc[a];
        ng[a] = fine_per_axis(dims[a]);
        W.fw[a] = (double)dims[a] / ng[a];
    }
    W.cx = nc[0]; W.cy = nc[1]; W.cz = nc[2];
    W.gx = ng[0]; W.gy = ng[1]; W.gz = ng[2];
    W.cell0 = (int32_t)t.nb_start.size();
    W.fine0 = (int32_t)t.near.size();
    auto cell_idx = [](double x, double L, double w, int n) {
        const double xw = x - L * std::floor(x / L);
        const int q = (int)(xw / w);
        return q < 0 ? 0 : (q >= n ? n - 1 : q);
    };
    const int ncell = nc[0] * nc[1] * nc[2];
    const size_t site0 = t.sites.size();
    std::vector<std::vector<int32_t>> bins(ncell);
    {
        std::vector<std::vector<WallSite>> sb(ncell);
        for (const WallSite& w : sites_in) {
            const int k = cell_idx(w.p[0], dims[0], W.cw[0], nc[0]) +
                          nc[0] * (cell_idx(w.p[1], dims[1], W.cw[1], nc[1]) +
                                   nc[1] * cell_idx(w.p[2], dims[2], W.cw[2], nc[2]));
            sb[k].push_back(w);
        }
        for (int k = 0; k < ncell; ++k)
            for (const WallSite& w : sb[k]) {
                bins[k].push_back((int32_t)t.sites.size());
                t.sites.push_back(w);
            }
    }
    // neighbourhood lists: the distinct cells c-1, c, c+1 along each axis (all cells of an
    // axis with fewer than three)
    auto span = [](int ci, int n, int& first, int& count) {
        if (n >= 3) { first = ci == 0 ? n - 1 : ci - 1; count = 3; }
        else { first = 0; count = n; }
    };
    for (int z = 0; z < nc[2]; ++z)
        for (int y = 0; y < nc[1]; ++y)
            for (int x = 0; x < nc[0]; ++x) {
                t.nb_start.push_back((int32_t)t.nb_sites.size());
                int f0, n0, f1, n1, f2, n2;
                span(x, nc[0], f0, n0);
                span(y, nc[1], f1, n1);
                span(z, nc[2], f2, n2);
                for (int iz = 0; iz < n2; ++iz)
                    for (int iy = 0; iy < n1; ++iy)
                        for (int ix = 0; ix < n0; ++ix) {
                            const auto& bin = bins[(f0 + ix) % nc[0] +
                                                   nc[0] * ((f1 + iy) % nc[1] +
                                                            nc[1] * ((f2 + iz) % nc[2]))];
                            for (int32_t i : bin) t.nb_sites.push_back(t.sites[i]);
                        }
            }
    t.nb_start.push_back((int32_t)t.nb_sites.size());
    // fine flags: cells whose centre lies within range + half diagonal of a site
    const size_t nfine = (size_t)ng[0] * ng[1] * ng[2];
    std::vector<uint8_t> fl(nfine, 0);
    const double hd = 0.5 * std::sqrt(W.fw[0] * W.fw[0] + W.fw[1] * W.fw[1] + W.fw[2] * W.fw[2]);
    for (size_t k = site0; k < t.sites.size(); ++k) {
        const WallSite& w = t.sites[k];
        const double reach = cut * (ev_r + w.radius) + hd + 1e-6;
        int lo[3], cnt[3];
        for (int a = 0; a < 3; ++a) {
            lo[a] = (int)std::floor((w.p[a] - reach) / W.fw[a]) - 1;
            cnt[a] = std::min(ng[a], (int)std::ceil(2.0 * reach / W.fw[a]) + 4);
        }
        for (int iz = 0; iz < cnt[2]; ++iz)
            for (int iy = 0; iy < cnt[1]; ++iy)
                for (int ix = 0; ix < cnt[0]; ++ix) {
                    const int g[3] = {lo[0] + ix, lo[1] + iy, lo[2] + iz};
                    double d2 = 0.0;
                    int gi[3];
                    for (int a = 0; a < 3; ++a) {
                        gi[a] = ((g[a] % ng[a]) + ng[a]) % ng[a];
                        double dd = (gi[a] + 0.5) * W.fw[a] - w.p[a];
                        dd -= dims[a] * std::round(dd / dims[a]);
                        d2 += dd * dd;
                    }
                    if (d2 <= reach * reach)
                        fl[gi[0] + (size_t)ng[0] * (gi[1] + (size_t)ng[1] * gi[2])] = 1;
                }
    }
    t.near.insert(t.near.end(), fl.begin(), fl.end());
    return true;
}

}  // namespace lbrb
