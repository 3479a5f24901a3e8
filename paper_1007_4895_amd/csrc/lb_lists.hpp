// lb_lists.hpp -- host-side lists that depend only on the decomposition of
// a lattice into its two velocity sets (the coupling of Sec. 2.2, with
// per-tile bands of high-order rows at each wall): the nodes whose
// populations the partner set's stencil reads through the Hermite
// projection, and the nodes that carry periodic row images or pressure
// columns.  Plain C++ (no HIP), so the rules can be checked on the host.
#pragma once
#include <algorithm>
#include <stdint.h>
#include <vector>

#include "lb_internal.hpp"

namespace lbl {

using namespace lbi;

struct Decomp {
    int nx, ny;            // columns; rows are 0..ny
    int xbc, ybc, iface;   // XBC_*, YBC_*, IF_*
    int ntiles, tile_w;    // bands are per tile of tile_w columns
    const int32_t *blo;    // high rows at the bottom wall, per tile
    const int32_t *bhi;    // high rows at the top wall, per tile
};

// region of row j for bands lo/hi of its tile; same rule as the kernels
inline int host_reg(int lo, int hi, int j, int ny, int iface) {
    if (j < lo || j > ny - hi) return REG_HIGH;
    if (iface == IF_PAPER && ((lo > 0 && j == lo) || (hi > 0 && j == ny - hi))) return REG_IFACE;
    return REG_LOW;
}

// Per-step lists: `fin` = nodes needing row images (periodic y) or pressure
// columns, as (i, j, set, 0); `proj` = nodes a stencil of the partner set
// reads (Hermite interface: a node of one set within two nodes, along x or
// y, of a node of the other; beyond a wall there is no node, across a
// periodic boundary the wrapped one), as (i, j), low-set nodes first.  Both
// in row-major order.  Only nodes near a band edge can be projection
// sources: per column, the rows within reach of its own band edges, of the
// rows that wrap (periodic y) and, where a column within two has other
// bands, of the rows between the two columns' edges; the exact test is then
// applied to those candidates alone.  Returns the number of `fin` entries;
// nproj = {low-set, high-set} projection entries.
inline int build_lists(const Decomp &D, std::vector<int32_t> &fin, std::vector<int32_t> &proj, int nproj[2]) {
    fin.clear();
    proj.clear();
    const int nx = D.nx, ny = D.ny, nrow = ny + 1;
    const bool per_y = D.ybc == YBC_PERIODIC, per_x = D.xbc == XBC_PERIODIC;
    const bool press = D.xbc == XBC_PRESSURE;
    std::vector<int> lo(nx), hi(nx);
    for (int i = 0; i < nx; ++i) {
        const int t = D.ntiles == 1 ? 0 : i / D.tile_w;
        lo[i] = D.blo[t];
        hi[i] = D.bhi[t];
    }
    auto reg = [&](int i, int j) { return host_reg(lo[i], hi[i], j, ny, D.iface); };
    auto xwrap = [&](int k) { return k < 0 || k >= nx ? (per_x ? (k + nx) % nx : -1) : k; };
    auto neighbour_in = [&](int i, int j, int want) {
        for (int d = -2; d <= 2; ++d) {
            if (!d) continue;
            int jj = j + d;
            if (jj < 0 || jj > ny) jj = per_y ? (jj + nrow) % nrow : -1;
            if (jj >= 0 && reg(i, jj) == want) return true;
            const int ii = xwrap(i + d);
            if (ii >= 0 && reg(ii, j) == want) return true;
        }
        return false;
    };
    std::vector<std::vector<int>> cand(nrow);   // candidate columns per row, ascending
    if (D.iface == IF_HERMITE) {
        std::vector<int> mark(nrow, -1);
        for (int i = 0; i < nx; ++i) {
            auto add = [&](int a, int b) {
                for (int j = std::max(0, a); j <= std::min(ny, b); ++j)
                    if (mark[j] != i) {
                        mark[j] = i;
                        cand[j].push_back(i);
                    }
            };
            add(lo[i] - 3, lo[i] + 2);
            add(ny - hi[i] - 2, ny - hi[i] + 3);
            if (per_y) {
                add(0, 2);
                add(ny - 2, ny);
            }
            for (int d = -2; d <= 2; ++d) {
                const int k = d ? xwrap(i + d) : -1;
                if (k < 0) continue;
                if (lo[k] != lo[i]) add(std::min(lo[i], lo[k]) - 3, std::max(lo[i], lo[k]) + 2);
                if (hi[k] != hi[i]) add(ny - std::max(hi[i], hi[k]) - 2, ny - std::min(hi[i], hi[k]) + 3);
            }
        }
    }
    std::vector<int32_t> ph;
    for (int j = 0; j < nrow; ++j)
        for (int i : cand[j]) {
            const int r = reg(i, j);
            if (r == REG_IFACE) continue;
            const int set = r == REG_HIGH ? 1 : 0;
            if (neighbour_in(i, j, set ? REG_LOW : REG_HIGH)) {
                std::vector<int32_t> &dst = set ? ph : proj;
                dst.push_back(i);
                dst.push_back(j);
            }
        }
    nproj[0] = int(proj.size() / 2);
    nproj[1] = int(ph.size() / 2);
    proj.insert(proj.end(), ph.begin(), ph.end());
    // row images (periodic y: the first and last two rows), imposed-shear
    // ghost rows (the top row) and pressure columns (the first and last
    // column), row-major
    auto add_fin = [&](int i, int j) {
        const int r = reg(i, j);
        if (r == REG_IFACE) return;
        fin.push_back(i);
        fin.push_back(j);
        fin.push_back(r == REG_HIGH ? 1 : 0);
        fin.push_back(0);
    };
    for (int j = 0; j < nrow; ++j) {
        if (per_y && (j < 2 || j >= nrow - 2)) {
            for (int i = 0; i < nx; ++i) add_fin(i, j);
        } else if (D.ybc == YBC_SHEAR && j == nrow - 1) {
            // the imposed-shear ghost rows above the top row
            for (int i = 0; i < nx; ++i) add_fin(i, j);
        } else if (press) {
            add_fin(0, j);
            if (nx > 1) add_fin(nx - 1, j);
        }
    }
    return int(fin.size() / 4);
}

}  // namespace lbl
