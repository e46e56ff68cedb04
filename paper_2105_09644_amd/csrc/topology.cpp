// Host-side octree topology of a block-structured grid.
//
// The tree solver's octree (Sec. 2.1) is built over the root blocks, the
// refined blocks and the cells inside the blocks.  The root blocks need not
// form a power-of-two array, so a virtual power-of-two root cube covers them;
// octants that hold no leaf cell are simply not created.  Nodes are numbered
// breadth first with the children of a node contiguous, so that a walk can
// fetch a node's children with one coalesced read.
//
// Only the topology is built here (once per set of domains); every quantity
// that depends on the gas is reduced on the GPU.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "tr_internal.h"

namespace tr {

static uint64_t spread3(uint64_t v)
{
    // spreads the low 21 bits of v to every third bit
    v &= 0x1fffff;
    v = (v | (v << 32)) & 0x1f00000000ffffULL;
    v = (v | (v << 16)) & 0x1f0000ff0000ffULL;
    v = (v | (v << 8)) & 0x100f00f00f00f00fULL;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ULL;
    v = (v | (v << 2)) & 0x1249249249249249ULL;
    return v;
}

static uint64_t morton(int32_t x, int32_t y, int32_t z)
{
    // x is the most significant bit of every triple: sorting by key sorts
    // cells by octant (x<<2 | y<<1 | z) at every level
    return (spread3((uint64_t)x) << 2) | (spread3((uint64_t)y) << 1) | spread3((uint64_t)z);
}

std::string build_topology(const tr_domain &d, const tr_params &p, DomTopo &t)
{
    t = DomTopo();
    for (int a = 0; a < 3; ++a)
        if (d.nroot[a] <= 0) return "nroot must be positive";
    if (d.max_level < 0 || d.max_level > 12) return "max_level must be in [0, 12]";
    if (!(d.root_block_cm > 0) || !std::isfinite(d.root_block_cm)) return "root_block_cm must be > 0";
    if (!d.leaf_blocks && d.max_level != 0) return "a uniform grid (leaf_blocks == NULL) needs max_level 0";
    if (d.leaf_blocks && d.n_leaf_blocks <= 0) return "n_leaf_blocks must be positive";
    for (int a = 0; a < 3; ++a) t.nroot[a] = d.nroot[a];
    t.max_level = d.max_level;
    t.root_block_cm = d.root_block_cm;
    const int32_t fine = kBlock << d.max_level;
    t.dx_cm = d.root_block_cm / (double)fine;
    int32_t emax = 0;
    for (int a = 0; a < 3; ++a) {
        int64_t e = (int64_t)d.nroot[a] * fine;
        if (e > (1 << 20)) return "grid too large (more than 2^20 finest cells per axis)";
        t.ext[a] = (int32_t)e;
        emax = std::max(emax, t.ext[a]);
    }
    int32_t root = 1;
    while (root < emax) root *= 2;
    t.root_size = root;

    // ---- leaf cells ----
    const int64_t n = d.leaf_blocks ? d.n_leaf_blocks * 512 : (int64_t)t.ext[0] * t.ext[1] * t.ext[2];
    if (n > (int64_t)INT32_MAX / 2) return "too many cells";
    t.n_cells = n;
    std::vector<int32_t> clo((size_t)n * 3), csz((size_t)n);
    if (!d.leaf_blocks) {
        int64_t c = 0;
        for (int32_t i = 0; i < t.ext[0]; ++i)
            for (int32_t j = 0; j < t.ext[1]; ++j)
                for (int32_t k = 0; k < t.ext[2]; ++k, ++c) {
                    clo[3 * c] = i;
                    clo[3 * c + 1] = j;
                    clo[3 * c + 2] = k;
                    csz[c] = 1;
                }
    } else {
        int64_t c = 0;
        for (int64_t b = 0; b < d.n_leaf_blocks; ++b) {
            const int32_t *e = d.leaf_blocks + 4 * b;
            const int32_t lev = e[0];
            if (lev < 0 || lev > d.max_level) return "leaf block level out of range";
            const int32_t cs = 1 << (d.max_level - lev);
            for (int a = 0; a < 3; ++a)
                if (e[1 + a] < 0 || (int64_t)e[1 + a] >= ((int64_t)d.nroot[a] << lev))
                    return "leaf block index out of range";
            for (int i = 0; i < kBlock; ++i)
                for (int j = 0; j < kBlock; ++j)
                    for (int k = 0; k < kBlock; ++k, ++c) {
                        clo[3 * c] = (e[1] * kBlock + i) * cs;
                        clo[3 * c + 1] = (e[2] * kBlock + j) * cs;
                        clo[3 * c + 2] = (e[3] * kBlock + k) * cs;
                        csz[c] = cs;
                    }
        }
    }
    // the cells must tile the domain: total volume equals the extent
    {
        double v = 0;
        for (int64_t c = 0; c < n; ++c) v += (double)csz[c] * csz[c] * csz[c];
        if (v != (double)t.ext[0] * t.ext[1] * t.ext[2]) return "leaf blocks do not tile the domain";
    }

    // ---- Morton order ----
    std::vector<uint64_t> key((size_t)n);
    for (int64_t c = 0; c < n; ++c) key[c] = morton(clo[3 * c], clo[3 * c + 1], clo[3 * c + 2]);
    std::vector<int32_t> ord((size_t)n);
    std::iota(ord.begin(), ord.end(), 0);
    std::sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
    t.morton = ord;

    // ---- breadth-first build: every node owns a contiguous range of ord ----
    struct Item { int32_t lo[3]; int32_t size; int64_t b, e; };
    std::vector<Item> cur{{{0, 0, 0}, root, 0, n}}, next;
    t.cell_node.assign((size_t)n, -1);
    int64_t base = 0;   // local index of the first node of the current level
    int level = 0;
    while (!cur.empty()) {
        if (level >= kMaxLevels) return "tree too deep";
        t.level_count.push_back((int64_t)cur.size());
        next.clear();
        const int64_t next_base = base + (int64_t)cur.size();
        for (size_t q = 0; q < cur.size(); ++q) {
            const Item &it = cur[q];
            const int64_t id = base + (int64_t)q;
            for (int a = 0; a < 3; ++a) t.lo.push_back(it.lo[a]);
            t.size.push_back(it.size);
            const int32_t c0 = ord[it.b];
            if (it.e - it.b == 1 && csz[c0] == it.size) {
                for (int a = 0; a < 3; ++a)
                    if (clo[3 * c0 + a] != it.lo[a]) return "inconsistent leaf cell";
                t.first.push_back(c0);
                t.nchild.push_back(0);
                t.cell_node[c0] = (int32_t)id;
                continue;
            }
            if (it.size == 1) return "overlapping cells";
            const int32_t half = it.size / 2;
            int32_t nc = 0;
            const int64_t child0 = next_base + (int64_t)next.size();
            int64_t s = it.b;
            for (int o = 0; o < 8; ++o) {
                const int32_t clo3[3] = {it.lo[0] + ((o >> 2) & 1) * half, it.lo[1] + ((o >> 1) & 1) * half,
                                         it.lo[2] + (o & 1) * half};
                int64_t e = s;
                while (e < it.e) {
                    const int32_t c = ord[e];
                    if (csz[c] >= it.size) return "overlapping cells";
                    const int oc = ((clo[3 * c] >= it.lo[0] + half) << 2) |
                                   ((clo[3 * c + 1] >= it.lo[1] + half) << 1) | (clo[3 * c + 2] >= it.lo[2] + half);
                    if (oc != o) break;
                    ++e;
                }
                if (e > s) {
                    next.push_back({{clo3[0], clo3[1], clo3[2]}, half, s, e});
                    ++nc;
                }
                s = e;
            }
            if (s != it.e) return "cells out of Morton order";
            t.first.push_back((int32_t)child0);
            t.nchild.push_back(nc);
        }
        base = next_base;
        cur.swap(next);
        ++level;
    }
    t.depth = level;
    const int64_t nn = (int64_t)t.size.size();
    if (nn > (int64_t)INT32_MAX / 2) return "too many nodes";
    for (int64_t c = 0; c < n; ++c)
        if (t.cell_node[c] < 0) return "cell without node";

    // ---- bounding boxes of the nodes' cells, bottom up ----
    t.olo.assign((size_t)nn * 3, 0);
    t.oext.assign((size_t)nn * 3, 0);
    std::vector<int32_t> ohi((size_t)nn * 3, 0);
    for (int64_t id = nn - 1; id >= 0; --id) {
        if (t.nchild[id] == 0) {
            for (int a = 0; a < 3; ++a) {
                t.olo[3 * id + a] = t.lo[3 * id + a];
                ohi[3 * id + a] = t.lo[3 * id + a] + t.size[id];
            }
        } else {
            for (int a = 0; a < 3; ++a) {
                int32_t lo = INT32_MAX, hi = INT32_MIN;
                for (int q = 0; q < t.nchild[id]; ++q) {
                    const int64_t ch = t.first[id] + q;
                    lo = std::min(lo, t.olo[3 * ch + a]);
                    hi = std::max(hi, ohi[3 * ch + a]);
                }
                t.olo[3 * id + a] = lo;
                ohi[3 * id + a] = hi;
            }
        }
        for (int a = 0; a < 3; ++a) t.oext[3 * id + a] = ohi[3 * id + a] - t.olo[3 * id + a];
    }

    // ---- evaluation points (Sec. 2.2) in finest-cell units ----
    const double L = std::sqrt((double)t.ext[0] * t.ext[0] + (double)t.ext[1] * t.ext[1] +
                               (double)t.ext[2] * t.ext[2]);
    int32_t nr;
    if (p.n_radial > 0) {
        nr = p.n_radial;
        if (nr < 3 || nr > kMaxRadial) return "n_radial must be in [3, 128]";
        t.r_cells.resize(nr);
        for (int i = 0; i < nr; ++i) {
            const double f = (double)i / (double)(nr - 1);
            t.r_cells[i] = L * f * f;
        }
        t.r_coef = L / ((double)(nr - 1) * (double)(nr - 1));
    } else {
        if (!(p.eta_r > 0)) return "eta_r must be > 0";
        nr = (int32_t)(p.eta_r * std::floor(std::sqrt(2.0 * L))) + 1;
        if (nr < 3 || nr > kMaxRadial) return "eq. (Nr) gives N_R outside [3, 128]";
        t.r_cells.resize(nr);
        for (int i = 0; i < nr; ++i) t.r_cells[i] = (double)i * (double)i / (2.0 * p.eta_r * p.eta_r);
        t.r_coef = 1.0 / (2.0 * p.eta_r * p.eta_r);
    }
    t.n_radial = nr;
    return "";
}

}  // namespace tr
