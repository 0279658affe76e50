// Cluster tree / block tree (host).
#pragma once

#include <cstdint>
#include <vector>

#include "bem_internal.hpp"

namespace bem {

struct Cluster {
    int64_t begin = 0, end = 0;   // dofs perm[begin..end)
    double lo[3], hi[3];          // bounding box of the dof points
    double slo[3], shi[3];        // support box
    int child[2] = {-1, -1};
};

struct Block {
    int tau, sigma, admissible;
};

struct Partition {
    std::vector<int32_t> perm;
    std::vector<Cluster> nodes;   // depth-first pre-order, root first
    std::vector<Block> blocks;    // leaves in depth-first order
};

void dof_geometry(const bem_mesh &m, int space, std::vector<double> &pts, std::vector<double> &slo,
                  std::vector<double> &shi);
void build_partition(const std::vector<double> &pts, const std::vector<double> &slo, const std::vector<double> &shi,
                     int leaf_size, double eta, int max_block, Partition &P);
bool admissible(const Cluster &a, const Cluster &b, double eta, int max_block);
double support_distance(const Cluster &a, const Cluster &b);

}  // namespace bem
