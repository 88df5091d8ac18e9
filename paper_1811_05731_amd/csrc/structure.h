// Host-side H2 block structure: mesh checks, cluster tree, cluster boxes,
// block tree and the node 2-ring (Section 4 of arXiv:1811.05731: index sets
// tied to geometric domains, admissible blocks replaced by low-rank factors).
// Pure C++; compiled without floating-point contraction so that every split
// and admissibility decision is reproducible.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace h2dlp {

struct Cluster {
    int64_t begin = 0, end = 0;   // range of positions in cluster order
    int32_t level = 0, parent = -1, child0 = -1, child1 = -1;
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};   // inflated support box
    bool leaf() const { return child0 < 0; }
    int64_t size() const { return end - begin; }
};

struct Structure {
    int64_t n_nodes = 0, n_tris = 0;
    std::vector<double> xyz;        // N x 3
    std::vector<int32_t> tri;       // T x 3
    std::vector<int64_t> inc_off;   // node -> incident (triangle, local vertex), CSR
    std::vector<int32_t> inc_tri;
    std::vector<int32_t> inc_loc;
    std::vector<int32_t> perm;      // cluster position -> node index
    std::vector<int64_t> iperm;     // node index -> cluster position
    std::vector<Cluster> cl;        // preorder
    std::vector<std::pair<int32_t, int32_t>> far, near;   // (target, source), sorted
    std::vector<int64_t> ring_off;  // per cluster position: 2-ring neighbours (positions, sorted)
    std::vector<int32_t> ring_pos;
    int32_t depth = 0;
};

// Fills `s`; returns an empty string on success, else the reason (EINVAL).
std::string build_structure(Structure& s, const double* xyz, int64_t n_nodes, const int32_t* tri,
                            int64_t n_tris, int leaf, double eta, double alpha, bool want_rings);

bool admissible(const Cluster& t, const Cluster& s, double eta);

}  // namespace h2dlp
