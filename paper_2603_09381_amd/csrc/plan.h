// Host-side plan of the recursive proxy solver: tree of cells (a quadtree over grid cells,
// or a hierarchical k-means clustering of the inclusions), near lists and proxy circles
// per level.  Pure C++ (no GPU), unit-testable on any machine.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

struct CellPlan {
  int I = 0, J = 0;              // cell coordinates at its level
  std::vector<int> incl;         // inclusions in the cell, ascending
  std::vector<int> children;     // indices into the level below (Morton order)
  double cx = 0, cy = 0;         // centre: mean of the inclusion centres
  double rc = 0;                 // farthest own boundary node from the centre
  double rho_far = 0;            // nearest node of a far cell (inf if none)
  double Rp = 0;                 // proxy radius (0: no proxy)
  int P = 0;                     // proxy points
  std::vector<int> near;         // near cells of the same level, ascending
};

struct PlanOptions {
  double proxy_ratio;            // radius >= proxy_ratio * r_c
  int proxy_min;                 // minimum (or fixed) number of proxy points
  int near_rule;                 // 0: edge-adjacent + geometric, 1: geometric only,
                                 // 2: eta-admissibility + geometric
  int proxy_rule;                // 0: radius max(ratio r_c, 0.9 rho_far) and adaptive P; 1: fixed
  double id_tol;
  double k_ext;
  int tree = 0;                  // 0: quadtree over grid cells, 1: hierarchical k-means
  int leaf_size = 1;             // tree 1: at most this many inclusions per leaf (1..4)
  double eta = 1.0;              // near_rule 2: near when eta |c_s - c_t| < max(2 r_s, 2 r_t)
};

// Builds levels[0] (one cell per inclusion) up to the single root cell.
// tree 0: grid_ij holds [2m] integer grid coordinates of the inclusions, or is NULL for
// scattered inclusions (grid_assignment below).  tree 1: grid_ij is ignored; levels[0]
// lists the inclusions leaf by leaf, and with leaf_size > 1 levels[1] holds the leaves (up
// to leaf_size inclusions each), which the solver compresses first (levels[0] then has
// centres and radii but no near lists or proxies).
// Returns an empty string on success, else an error message.
std::string build_plan(int m, const int32_t* grid_ij, const double* centers, const int64_t* node_off,
                       const double* x, const double* y, const PlanOptions& o,
                       std::vector<std::vector<CellPlan>>& levels);

uint64_t morton_code(uint32_t i, uint32_t j);

// Tree 1 with leaf_size > 1: the inclusion level is merged into the leaves uncompressed.
inline bool plan_pass_through(const PlanOptions& o) { return o.tree == 1 && o.leaf_size > 1; }

// One k-means split (tree 1): at most four clusters of the inclusions S by weighted Lloyd
// iterations on the node means (px, py) with weights wt; clusters in seed order, members
// in the order of S.
std::vector<std::vector<int>> kmeans_split(const std::vector<int>& S, const std::vector<double>& px,
                                           const std::vector<double>& py, const std::vector<double>& wt);

// Cells of scattered inclusions: [2m] grid coordinates with at most one centre per cell
// (empty when two centres coincide).
std::vector<int32_t> grid_assignment(int m, const double* centers);
