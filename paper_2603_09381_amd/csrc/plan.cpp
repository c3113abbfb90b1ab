// Quadtree, near lists and proxy circles of the recursive proxy solver.
//
// Sec. 3 of arXiv 2603.09381 takes each inclusion as a leaf cell and merges cells up
// a tree; Sec. 4 orders grid cells along the Morton curve and treats the four
// edge-adjacent cells as near field in the proxy method.  Readings used here:
//  * parents are the 2x2 blocks of the grid at the level below (quadtree);
//  * the cell centre is the mean of its inclusion centres, r_c the farthest own node;
//  * near cells: the edge-adjacent cells of the same level plus every same-level cell
//    with a node inside the proxy circle; the circle radius is max(ratio r_c,
//    0.9 rho_far), rho_far the distance to the nearest node of a far cell;
//  * P = max(P_min, 2 ceil(k+ R_p) + 2 ceil(ln tol / ln(r_c / rho_far)) + 16), or a
//    fixed P and radius ratio r_c when the caller fixes them;
//  * no proxy circle when every other cell of the level is near.
// Sec. 4.4 (Discussions) names the extension to arbitrary arrangements: cells from a
// k-means clustering, near pairs by an eta-admissibility test on the distance of the cell
// centres against the cell diameters, several scatterers per leaf.  Readings used here:
//  * the clustered points are the inclusions, each at the mean of its nodes and weighted
//    by its node count (k-means on the integration points with no inclusion split), four
//    clusters per split, top down until every cell holds at most leaf_size inclusions;
//  * seeds: the member farthest from the weighted mean, then each time the member
//    farthest from the seeds so far; Lloyd iterations (nearest centre, weighted mean)
//    until no member moves, at most 100;
//  * a cell's diameter is 2 r_c; near when eta |c_s - c_t| < max(2 r_c,s, 2 r_c,t), then
//    the same proxy-circle closure as above.
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <future>
#include <limits>
#include <map>
#include <thread>
#include <utility>

uint64_t morton_code(uint32_t i, uint32_t j) {
  uint64_t c = 0;
  for (int b = 0; b < 32; ++b) {
    c |= (uint64_t)((i >> b) & 1u) << (2 * b);
    c |= (uint64_t)((j >> b) & 1u) << (2 * b + 1);
  }
  return c;
}

namespace {

// Nearest and farthest node of the inclusions incl from (cx, cy), as std::hypot distances
// (the values the rest of the plan, and its tests, are defined with).  Squared distances
// find the extremes; hypot is then evaluated only for the nodes whose squared distance
// lies within a relative 1e-12 of an extreme, which contains every node hypot can rank
// first (squared distances are off by a few ulps at most).
void node_range(const std::vector<int>& incl, const int64_t* node_off, const double* x, const double* y, double cx,
                double cy, double& dmin, double& dmax) {
  // four independent running extrema (min and max are exact, so the order is free)
  double lo[4], hi[4];
  for (int q = 0; q < 4; ++q) {
    lo[q] = std::numeric_limits<double>::infinity();
    hi[q] = 0;
  }
  for (int j : incl) {
    int64_t i = node_off[j];
    const int64_t e = node_off[j + 1];
    for (; i + 4 <= e; i += 4)
      for (int q = 0; q < 4; ++q) {
        const double dx = x[i + q] - cx, dy = y[i + q] - cy;
        const double d2 = dx * dx + dy * dy;
        lo[q] = d2 < lo[q] ? d2 : lo[q];
        hi[q] = d2 > hi[q] ? d2 : hi[q];
      }
    for (; i < e; ++i) {
      const double dx = x[i] - cx, dy = y[i] - cy;
      const double d2 = dx * dx + dy * dy;
      lo[0] = d2 < lo[0] ? d2 : lo[0];
      hi[0] = d2 > hi[0] ? d2 : hi[0];
    }
  }
  const double lo2 = std::min(std::min(lo[0], lo[1]), std::min(lo[2], lo[3]));
  const double hi2 = std::max(std::max(hi[0], hi[1]), std::max(hi[2], hi[3]));
  const double lo_cut = lo2 * (1.0 + 1e-12), hi_cut = hi2 * (1.0 - 1e-12);
  dmin = std::numeric_limits<double>::infinity();
  dmax = 0;
  for (int j : incl)
    for (int64_t i = node_off[j]; i < node_off[j + 1]; ++i) {
      const double dx = x[i] - cx, dy = y[i] - cy;
      const double d2 = dx * dx + dy * dy;
      if (d2 <= lo_cut) dmin = std::min(dmin, std::hypot(dx, dy));
      if (d2 >= hi_cut) dmax = std::max(dmax, std::hypot(dx, dy));
    }
}

void near_cells(const PlanOptions& o, const int64_t* node_off, const double* x, const double* y,
                std::vector<CellPlan>& cells, int t0, int t1);

void near_and_proxy(const PlanOptions& o, const double* centers, const int64_t* node_off, const double* x,
                    const double* y, std::vector<CellPlan>& cells, bool lists = true) {
  const int nc = (int)cells.size();
  for (int t = 0; t < nc; ++t) {
    CellPlan& c = cells[t];
    double sx = 0, sy = 0;
    for (int j : c.incl) {
      sx += centers[2 * j];
      sy += centers[2 * j + 1];
    }
    c.cx = sx / (double)c.incl.size();
    c.cy = sy / (double)c.incl.size();
    double lo, hi;
    node_range(c.incl, node_off, x, y, c.cx, c.cy, lo, hi);
    c.rc = hi;
  }
  if (nc == 1 || !lists) return;
  // each cell's near list and proxy depend only on the centres and radii above: the cells
  // are split into contiguous ranges handled by up to four threads (the same plan)
  const int nt = nc >= 64 ? std::min(4, std::max(1, (int)std::thread::hardware_concurrency() / 2)) : 1;
  auto range = [&](int t0, int t1) { near_cells(o, node_off, x, y, cells, t0, t1); };
  std::vector<std::future<void>> part;
  for (int k = 1; k < nt; ++k) part.push_back(std::async(std::launch::async, range, nc * k / nt, nc * (k + 1) / nt));
  range(0, nc / nt);
  for (auto& f : part) f.get();
}

void near_cells(const PlanOptions& o, const int64_t* node_off, const double* x, const double* y,
                std::vector<CellPlan>& cells, int t0, int t1) {
  const int nc = (int)cells.size();
  const double inf = std::numeric_limits<double>::infinity();
  std::vector<double> lb(nc), ub(nc), dmin(nc);
  std::vector<char> isnear(nc);
  std::vector<std::pair<double, int>> cand;
  for (int t = t0; t < t1; ++t) {
    CellPlan& c = cells[t];
    // bounds |c_t - c_s| -+ r_s on the distance from the centre of t to the nodes of s
    // (widened by a relative 1e-9 against rounding); exact distances are computed only
    // for the cells the bounds cannot settle
    for (int s = 0; s < nc; ++s) {
      const double ex = cells[s].cx - c.cx, ey = cells[s].cy - c.cy;
      const double cd = std::sqrt(ex * ex + ey * ey);
      const double l = cd - cells[s].rc, u = cd + cells[s].rc;
      lb[s] = l - 1e-9 * (1.0 + std::fabs(l));
      ub[s] = u + 1e-9 * (1.0 + u);
      dmin[s] = -1.0;
      isnear[s] = 0;
    }
    auto dist = [&](int s) {
      if (dmin[s] < 0) {
        double lo, hi;
        node_range(cells[s].incl, node_off, x, y, c.cx, c.cy, lo, hi);
        dmin[s] = lo;
      }
      return dmin[s];
    };
    if (o.near_rule == 0)
      for (int s = 0; s < nc; ++s)
        if (s != t && std::abs(cells[s].I - c.I) + std::abs(cells[s].J - c.J) == 1) isnear[s] = 1;
    if (o.near_rule == 2)
      for (int s = 0; s < nc; ++s) {
        const double ex = cells[s].cx - c.cx, ey = cells[s].cy - c.cy;
        if (s != t && o.eta * std::sqrt(ex * ex + ey * ey) < 2.0 * std::max(c.rc, cells[s].rc)) isnear[s] = 1;
      }
    double rho = inf, Rp = 0;
    bool anyfar = false;
    for (;;) {
      // rho: the nearest node of a far cell; only cells whose lower bound reaches below
      // the smallest upper bound can hold it
      double u = inf;
      anyfar = false;
      for (int s = 0; s < nc; ++s)
        if (s != t && !isnear[s]) {
          anyfar = true;
          u = std::min(u, ub[s]);
        }
      cand.clear();
      for (int s = 0; s < nc; ++s)
        if (s != t && !isnear[s] && lb[s] <= u) cand.push_back({lb[s], s});
      std::sort(cand.begin(), cand.end());
      rho = inf;
      for (const auto& pr : cand) {
        if (pr.first > rho) break;   // nearest first: later cells cannot come closer
        rho = std::min(rho, dist(pr.second));
      }
      if (o.proxy_rule == 0 && anyfar)
        Rp = std::max(o.proxy_ratio * c.rc, 0.9 * rho);
      else
        Rp = o.proxy_ratio * c.rc;
      // every far cell with a node inside the proxy circle becomes near
      bool added = false;
      for (int s = 0; s < nc; ++s)
        if (s != t && !isnear[s] && lb[s] <= Rp && dist(s) <= Rp) {
          isnear[s] = 1;
          added = true;
        }
      if (!added) break;
    }
    c.near.clear();
    for (int s = 0; s < nc; ++s)
      if (isnear[s]) c.near.push_back(s);
    c.rho_far = rho;
    if (anyfar) {
      c.Rp = Rp;
      if (o.proxy_rule == 0) {
        double q = std::min(c.rc / rho, 0.95);
        int P = 2 * (int)std::ceil(o.k_ext * Rp) + 2 * (int)std::ceil(std::log(o.id_tol) / std::log(q)) + 16;
        c.P = std::max(o.proxy_min, P);
      } else {
        c.P = o.proxy_min;
      }
    } else {
      c.Rp = 0;
      c.P = 0;
    }
  }
}

}  // namespace

// Scattered inclusions: a uniform grid of spacing h = 0.99 d_min / sqrt(2) (d_min the
// smallest centre distance) holds at most one centre per cell, as a cell's diagonal is
// shorter than d_min; the quadtree over the occupied cells prunes the empty ones, which
// makes it an adaptive tree with one inclusion per leaf.  Empty result: coincident centres.
std::vector<int32_t> grid_assignment(int m, const double* centers) {
  std::vector<int32_t> ij(2 * (size_t)m, 0);
  if (m == 1) return ij;
  double d2 = std::numeric_limits<double>::infinity();
  for (int i = 0; i < m; ++i)
    for (int j = i + 1; j < m; ++j) {
      const double dx = centers[2 * i] - centers[2 * j];
      const double dy = centers[2 * i + 1] - centers[2 * j + 1];
      d2 = std::min(d2, dx * dx + dy * dy);
    }
  if (!(d2 > 0)) return {};
  const double h = 0.99 * std::sqrt(d2 / 2.0);
  double x0 = centers[0], y0 = centers[1];
  for (int i = 1; i < m; ++i) {
    x0 = std::min(x0, centers[2 * i]);
    y0 = std::min(y0, centers[2 * i + 1]);
  }
  for (int i = 0; i < m; ++i) {
    const double gx = std::floor((centers[2 * i] - x0) / h), gy = std::floor((centers[2 * i + 1] - y0) / h);
    if (gx > 1e9 || gy > 1e9) return {};
    ij[2 * i] = (int32_t)gx;
    ij[2 * i + 1] = (int32_t)gy;
  }
  return ij;
}

std::vector<std::vector<int>> kmeans_split(const std::vector<int>& S, const std::vector<double>& px,
                                           const std::vector<double>& py, const std::vector<double>& wt) {
  const int n = (int)S.size();
  const int k = std::min(4, n);
  const double inf = std::numeric_limits<double>::infinity();
  std::vector<double> cx, cy;
  if (n == 0) return {};
  {
    double sx = 0, sy = 0, sw = 0;
    for (int j : S) {
      sx += wt[j] * px[j];
      sy += wt[j] * py[j];
      sw += wt[j];
    }
    const double mx = sx / sw, my = sy / sw;
    int best = 0;
    double bd = -1;
    for (int i = 0; i < n; ++i) {
      const double dx = px[S[i]] - mx, dy = py[S[i]] - my;
      const double d = dx * dx + dy * dy;
      if (d > bd) {
        bd = d;
        best = i;
      }
    }
    cx.push_back(px[S[best]]);
    cy.push_back(py[S[best]]);
  }
  std::vector<double> dmin(n, inf);
  while ((int)cx.size() < k) {
    int best = -1;
    double bd = 0;
    for (int i = 0; i < n; ++i) {
      const double dx = px[S[i]] - cx.back(), dy = py[S[i]] - cy.back();
      dmin[i] = std::min(dmin[i], dx * dx + dy * dy);
      if (dmin[i] > bd) {
        bd = dmin[i];
        best = i;
      }
    }
    if (best < 0) break;   // every member coincides with a seed
    cx.push_back(px[S[best]]);
    cy.push_back(py[S[best]]);
  }
  const int kk = (int)cx.size();
  std::vector<int> a(n, -1);
  for (int it = 0; it < 100; ++it) {
    bool moved = false;
    for (int i = 0; i < n; ++i) {
      int b = 0;
      double bd = inf;
      for (int c = 0; c < kk; ++c) {
        const double dx = px[S[i]] - cx[c], dy = py[S[i]] - cy[c];
        const double d = dx * dx + dy * dy;
        if (d < bd) {
          bd = d;
          b = c;
        }
      }
      if (b != a[i]) {
        a[i] = b;
        moved = true;
      }
    }
    if (!moved) break;
    for (int c = 0; c < kk; ++c) {
      double sx = 0, sy = 0, sw = 0;
      for (int i = 0; i < n; ++i)
        if (a[i] == c) {
          sx += wt[S[i]] * px[S[i]];
          sy += wt[S[i]] * py[S[i]];
          sw += wt[S[i]];
        }
      if (sw > 0) {   // an emptied cluster keeps its centre
        cx[c] = sx / sw;
        cy[c] = sy / sw;
      }
    }
  }
  std::vector<std::vector<int>> out;
  for (int c = 0; c < kk; ++c) {
    std::vector<int> mem;
    for (int i = 0; i < n; ++i)
      if (a[i] == c) mem.push_back(S[i]);
    if (!mem.empty()) out.push_back(mem);
  }
  return out;
}

namespace {

// Tree 1: k-means clusters split top down, depth by depth, while a cell of the depth holds
// more than leaf_size inclusions (cells within the limit carry on as single children);
// cells of a depth are ordered parent by parent, children in cluster order.
std::string kmeans_levels(int m, const int64_t* node_off, const double* x, const double* y, const PlanOptions& o,
                          std::vector<std::vector<CellPlan>>& levels) {
  if (o.leaf_size < 1 || o.leaf_size > 4) return "leaf_size must be in 1..4";
  std::vector<double> px(m), py(m), wt(m);
  for (int j = 0; j < m; ++j) {
    double sx = 0, sy = 0;
    for (int64_t i = node_off[j]; i < node_off[j + 1]; ++i) {
      sx += x[i];
      sy += y[i];
    }
    wt[j] = (double)(node_off[j + 1] - node_off[j]);
    px[j] = sx / wt[j];
    py[j] = sy / wt[j];
  }
  std::vector<std::vector<std::vector<int>>> depth(1);
  std::vector<std::vector<int>> parent(1);
  depth[0].push_back(std::vector<int>(m));
  for (int j = 0; j < m; ++j) depth[0][0][j] = j;
  parent[0].push_back(-1);
  for (;;) {
    const auto& cur = depth.back();
    bool split = false;
    for (const auto& c : cur) split = split || (int)c.size() > o.leaf_size;
    if (!split) break;
    std::vector<std::vector<int>> nxt;
    std::vector<int> par;
    for (int t = 0; t < (int)cur.size(); ++t) {
      if ((int)cur[t].size() > o.leaf_size) {
        std::vector<std::vector<int>> parts = kmeans_split(cur[t], px, py, wt);
        if (parts.size() < 2) return "inclusions whose node means coincide";
        for (auto& q : parts) {
          nxt.push_back(q);
          par.push_back(t);
        }
      } else {
        nxt.push_back(cur[t]);
        par.push_back(t);
      }
    }
    depth.push_back(nxt);
    parent.push_back(par);
    if (depth.size() > 40) return "tree too deep";
  }
  const int D = (int)depth.size() - 1;
  const bool pass = plan_pass_through(o);
  // level 0: the inclusions leaf by leaf (with leaf_size 1 the leaves themselves)
  std::vector<CellPlan> l0;
  std::vector<int> first(depth[D].size() + 1, 0);
  for (size_t t = 0; t < depth[D].size(); ++t) {
    first[t] = (int)l0.size();
    for (int j : depth[D][t]) {
      CellPlan c;
      c.incl = {j};
      l0.push_back(c);
    }
  }
  first[depth[D].size()] = (int)l0.size();
  levels.push_back(l0);
  for (int d = pass ? D : D - 1; d >= 0; --d) {
    std::vector<CellPlan> cells(depth[d].size());
    for (size_t t = 0; t < depth[d].size(); ++t) {
      cells[t].incl = depth[d][t];
      std::sort(cells[t].incl.begin(), cells[t].incl.end());
    }
    if (d == D)   // the leaves: their inclusions at level 0
      for (size_t t = 0; t < cells.size(); ++t)
        for (int q = first[t]; q < first[t + 1]; ++q) cells[t].children.push_back(q);
    else
      for (size_t q = 0; q < depth[d + 1].size(); ++q) cells[parent[d + 1][q]].children.push_back((int)q);
    levels.push_back(cells);
  }
  return "";
}

}  // namespace

std::string build_plan(int m, const int32_t* grid_ij, const double* centers, const int64_t* node_off,
                       const double* x, const double* y, const PlanOptions& o,
                       std::vector<std::vector<CellPlan>>& levels) {
  levels.clear();
  if (m <= 0) return "no inclusions";
  if (o.tree == 1) {
    if (o.near_rule == 0) return "edge adjacency needs grid cells (tree 0)";
    std::string err = kmeans_levels(m, node_off, x, y, o, levels);
    if (!err.empty()) return err;
    for (size_t l = 0; l < levels.size(); ++l)
      near_and_proxy(o, centers, node_off, x, y, levels[l], !(l == 0 && plan_pass_through(o)));
    return "";
  }
  if (o.tree != 0) return "tree must be 0 or 1";
  std::vector<int32_t> own_grid;
  if (!grid_ij) {
    own_grid = grid_assignment(m, centers);
    if (own_grid.empty()) return "two inclusions share a centre";
    grid_ij = own_grid.data();
  }
  std::map<std::pair<int, int>, std::vector<int>> cur;
  for (int j = 0; j < m; ++j) {
    if (grid_ij[2 * j] < 0 || grid_ij[2 * j + 1] < 0) return "negative grid coordinate";
    cur[{grid_ij[2 * j], grid_ij[2 * j + 1]}].push_back(j);
  }
  for (auto& kv : cur)
    if (kv.second.size() != 1) return "two inclusions share a grid cell";
  int lev = 0;
  for (;;) {
    std::vector<std::pair<uint64_t, std::pair<int, int>>> keys;
    for (auto& kv : cur) keys.push_back({morton_code(kv.first.first, kv.first.second), kv.first});
    std::sort(keys.begin(), keys.end());
    std::vector<CellPlan> cells;
    for (auto& k : keys) {
      CellPlan c;
      c.I = k.second.first;
      c.J = k.second.second;
      c.incl = cur[k.second];
      std::sort(c.incl.begin(), c.incl.end());
      cells.push_back(c);
    }
    if (lev > 0) {
      const std::vector<CellPlan>& prev = levels.back();
      std::map<std::pair<int, int>, int> index;
      for (int t = 0; t < (int)prev.size(); ++t) index[{prev[t].I, prev[t].J}] = t;
      for (auto& c : cells)
        for (int b = 0; b < 2; ++b)
          for (int a = 0; a < 2; ++a) {
            auto it = index.find({2 * c.I + a, 2 * c.J + b});
            if (it != index.end()) c.children.push_back(it->second);
          }
    }
    levels.push_back(cells);
    if (cells.size() == 1) break;
    std::map<std::pair<int, int>, std::vector<int>> nxt;
    for (auto& c : cells) {
      auto& v = nxt[{c.I >> 1, c.J >> 1}];
      v.insert(v.end(), c.incl.begin(), c.incl.end());
    }
    cur.swap(nxt);
    ++lev;
    if (lev > 40) return "tree too deep";
  }
  for (auto& cells : levels) near_and_proxy(o, centers, node_off, x, y, cells);
  return "";
}
