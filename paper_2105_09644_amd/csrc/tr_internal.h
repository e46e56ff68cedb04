// Internal declarations of the TreeRay HIP library (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "treeray.h"

namespace tr {

constexpr int kBlock = 8;          // cells per block edge
constexpr int kMaxRadial = 128;    // evaluation points per ray (two 64-bit masks)
constexpr int kAtabRatios = 4;    // angular-weight table: nodes of 1, 2, 4 and 8 target sizes
constexpr int kMaxLevels = 24;
constexpr int kGlobalList = 1 << 16;   // frontier / accepted-list entries of the fallback walk
constexpr int kFallbackPerCu = 2;       // workgroups per compute unit in the fallback pass
constexpr int kGlNodes = 24;            // Gauss-Legendre nodes of the sphere-deposit quadrature

// Geometry flags packed into NodeGeo.w
constexpr int kSizeMask = (1 << 24) - 1;
constexpr int kPartialBit = 1 << 30;   // node whose cells do not fill its cube
constexpr int kIfBit = 1 << 28;        // node holds an ionisation front (IF MAC)
constexpr int kSrcBit = 1 << 29;       // node holds emission (Src MAC)

// Host-side topology of one domain in breadth-first order.
struct DomTopo {
    int32_t nroot[3] = {0, 0, 0};
    int32_t max_level = 0;
    double root_block_cm = 0;
    double dx_cm = 0;               // finest cell
    int32_t ext[3] = {0, 0, 0};     // extent in finest cells
    int32_t root_size = 0;          // virtual root cube side, finest cells
    int64_t n_cells = 0;
    int32_t depth = 0;              // number of node levels
    // per level: nodes of this domain, breadth-first
    std::vector<int64_t> level_count;
    // node records in BFS order (local numbering 0..n-1, levels concatenated)
    std::vector<int32_t> lo;        // [n][3]
    std::vector<int32_t> size;      // [n]
    std::vector<int32_t> olo, oext; // [n][3] bounding box of the node's cells
    std::vector<int32_t> first;     // local index of first child, or cell index for leaves
    std::vector<int32_t> nchild;    // 0 for leaves
    std::vector<int32_t> cell_node; // [n_cells] local node of each cell
    std::vector<int32_t> morton;    // [n_cells] cells in Morton order
    int32_t n_radial = 0;
    std::vector<double> r_cells;    // evaluation points in finest-cell units
    double r_coef = 0;              // r_i = r_coef i^2
};

// Builds the topology; returns an empty string or an error message.
std::string build_topology(const tr_domain &d, const tr_params &p, DomTopo &out);

// Per-domain constants seen by the kernels.
struct DomDev {
    int32_t root;          // global node index of the root
    int32_t nr;            // evaluation points
    int32_t r_off;         // offset into the radial tables
    int32_t cell_off;      // first global cell
    int32_t n_cells;
    int32_t ext[3];        // extent in finest cells (the period of periodic boundaries)
    double dx_cm;          // finest cell size
    double flux_unit;      // internal flux -> photons cm^-2 s^-1
    double rate_unit;      // internal rate -> photons s^-1
    double alpha_int;      // alpha_B dx^3 / rate_unit
    double rc_inv;         // 1/c of the evaluation points r_i = c i^2 (finest-cell units)
};

}  // namespace tr
