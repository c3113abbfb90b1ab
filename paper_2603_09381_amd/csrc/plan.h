// Host-side plan of the recursive proxy solver: quadtree of cells, near lists and
// proxy circles per level.  Pure C++ (no GPU), unit-testable on any machine.
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
  int near_rule;                 // 0: edge-adjacent + geometric, 1: geometric only
  int proxy_rule;                // 0: radius max(ratio r_c, 0.9 rho_far) and adaptive P; 1: fixed
  double id_tol;
  double k_ext;
};

// Builds levels[0] (one cell per inclusion) up to the single root cell.
// grid_ij: [2m] integer grid coordinates of the inclusions, or NULL for scattered
// inclusions (grid_assignment below).
// Returns an empty string on success, else an error message.
std::string build_plan(int m, const int32_t* grid_ij, const double* centers, const int64_t* node_off,
                       const double* x, const double* y, const PlanOptions& o,
                       std::vector<std::vector<CellPlan>>& levels);

uint64_t morton_code(uint32_t i, uint32_t j);

// Cells of scattered inclusions: [2m] grid coordinates with at most one centre per cell
// (empty when two centres coincide).
std::vector<int32_t> grid_assignment(int m, const double* centers);
