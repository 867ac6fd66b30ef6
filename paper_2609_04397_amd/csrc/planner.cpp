// Host planner: validation, shape classes, and the page layout of both
// directions of the operator (paper, section 3.2: shape classes are counted
// from the distinct (b_i, b_j) and every logical block is mapped to its place
// in a shape-specific buffer; here the buffer of a shape class inside a block
// row is one contiguous run of the row's panel).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <numeric>

#include "../../include/vbcsr.h"
#include "common.hpp"

namespace vbcsr {

int validate_graph(int32_t n, const int32_t *b, const int64_t *row_ptr, const int32_t *col_idx,
                   int64_t n_values, std::string &err) {
  if (n < 0) { err = "n_atoms must be >= 0"; return VBCSR_EINVAL; }
  if (!row_ptr) { err = "row_ptr is NULL"; return VBCSR_EINVAL; }
  if (n > 0 && !b) { err = "block_sizes is NULL"; return VBCSR_EINVAL; }
  if (row_ptr[0] != 0) { err = "row_ptr[0] must be 0"; return VBCSR_EINVAL; }
  int64_t N = 0;
  for (int32_t i = 0; i < n; ++i) {
    if (b[i] <= 0) { err = "block size of atom " + std::to_string(i) + " is <= 0"; return VBCSR_EINVAL; }
    if (b[i] > VBCSR_MAX_BLOCK) {
      err = "block size " + std::to_string(b[i]) + " exceeds VBCSR_MAX_BLOCK";
      return VBCSR_EUNSUPPORTED;
    }
    N += b[i];
    if (row_ptr[i + 1] < row_ptr[i]) { err = "row_ptr is decreasing at row " + std::to_string(i); return VBCSR_EINVAL; }
  }
  if (N > INT32_MAX) { err = "more than 2^31-1 scalar rows"; return VBCSR_EUNSUPPORTED; }
  const int64_t nnzb = row_ptr[n];
  if (nnzb > 0 && !col_idx) { err = "col_idx is NULL"; return VBCSR_EINVAL; }
  int64_t nnz = 0;
  std::vector<int32_t> tmp;
  for (int32_t i = 0; i < n; ++i) {
    tmp.assign(col_idx + row_ptr[i], col_idx + row_ptr[i + 1]);
    for (int32_t j : tmp) {
      if (j < 0 || j >= n) {
        err = "col_idx " + std::to_string(j) + " out of range in row " + std::to_string(i);
        return VBCSR_EINVAL;
      }
      nnz += (int64_t)b[i] * b[j];
    }
    std::sort(tmp.begin(), tmp.end());
    for (size_t t = 1; t < tmp.size(); ++t)
      if (tmp[t] == tmp[t - 1]) {
        err = "duplicate block (" + std::to_string(i) + ", " + std::to_string(tmp[t]) + ")";
        return VBCSR_EDUP;
      }
  }
  if (nnz != n_values) {
    err = "n_values " + std::to_string(n_values) + " != sum of block sizes " + std::to_string(nnz);
    return VBCSR_ESHAPE;
  }
  // The kernels address one block row (forward) or block column (adjoint)
  // with 32-bit byte offsets: its values must stay below 2^31 bytes in FP64.
  constexpr int64_t kPanelMax = (int64_t(1) << 31) / 8;
  std::vector<int64_t> colk(n, 0);
  for (int32_t i = 0; i < n; ++i) {
    int64_t k = 0;
    for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      k += b[col_idx[e]];
      colk[col_idx[e]] += b[i];
    }
    if (k * b[i] >= kPanelMax) {
      err = "block row " + std::to_string(i) + " holds 2^28 or more values";
      return VBCSR_EUNSUPPORTED;
    }
  }
  for (int32_t j = 0; j < n; ++j)
    if (colk[j] * b[j] >= kPanelMax) {
      err = "block column " + std::to_string(j) + " holds 2^28 or more values";
      return VBCSR_EUNSUPPORTED;
    }
  return VBCSR_OK;
}

// Lay out one direction.  `members[r]` lists the graph blocks held by panel r
// together with the atom that indexes their panel columns.
static void layout_direction(int32_t n, const int32_t *b, const std::vector<int64_t> &off,
                             const std::vector<std::vector<std::pair<int32_t, int64_t>>> &members,
                             int64_t nnzb, const std::vector<int64_t> *gbase,
                             const std::vector<int32_t> &order, DirPlan &d) {
  int64_t total_cols = 0;
  for (int32_t r = 0; r < n; ++r)
    for (const auto &m : members[r]) total_cols += b[m.first];
  d.colx.reserve(total_cols);
  if (gbase) d.colg.reserve(total_cols);
  d.rows.resize(n);
  d.vbase16.resize(n);
  d.blk_pos.assign(nnzb, 0);
  d.blk_k0.assign(nnzb, 0);
  d.blk_prow.assign(nnzb, 0);
  int64_t vbase = 0, cbase = 0, vbase16 = 0;
  // panels are laid out and processed in `order` (panel pi holds atom r)
  for (int32_t pi = 0; pi < n; ++pi) {
    const int32_t r = order[pi];
    const int32_t h = b[r];
    int32_t K = 0;
    for (const auto &m : members[r]) K += b[m.first];
    RowDesc rd{};
    rd.vbase = vbase;
    rd.cbase = cbase;
    rd.K = K;
    rd.yrow = (int32_t)off[r];
    rd.b = h;
    d.rows[pi] = rd;
    d.vbase16[pi] = vbase16;
    int32_t k0 = 0;
    for (const auto &m : members[r]) {
      const int32_t c = m.first;     // atom indexing the block's panel columns
      const int64_t k = m.second;    // graph block index
      d.blk_pos[k] = vbase + (int64_t)k0 * h;
      d.blk_k0[k] = k0;
      d.blk_prow[k] = pi;
      for (int32_t q = 0; q < b[c]; ++q) {
        d.colx.push_back((int32_t)(off[c] + q));
        if (gbase) d.colg.push_back((((*gbase)[k] + q) << 7) | b[c]);
      }
      k0 += b[c];
    }
    // panels start on 4-value boundaries (zero padding), so a 16-byte load
    // of values never mixes two panels
    vbase += ((int64_t)h * K + kPanelAlign - 1) / kPanelAlign * kPanelAlign;
    cbase += K;
    vbase16 += (int64_t)h * ((K + 7) / 8 * 8);
  }
  d.n_values = vbase;
  d.n_cols = cbase;
  d.n_values16 = vbase16;
}

// Reverse Cuthill-McKee order of the symmetrised block graph: breadth-first
// from a lowest-degree unvisited atom of each component, neighbours in
// ascending degree, the whole sequence reversed.  Panels processed in this
// order are graph neighbours of the panels processed just before them, so
// the input rows they gather are still in the XCD's L2.
static std::vector<int32_t> rcm_order(int32_t n, const int64_t *row_ptr, const int32_t *col_idx) {
  std::vector<int64_t> deg((size_t)n, 0);
  for (int32_t i = 0; i < n; ++i)
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
      if (col_idx[k] != i) {
        ++deg[i];
        ++deg[col_idx[k]];
      }
  std::vector<int64_t> ap((size_t)n + 1, 0);
  for (int32_t i = 0; i < n; ++i) ap[i + 1] = ap[i] + deg[i];
  std::vector<int32_t> adj((size_t)ap[n]);
  std::vector<int64_t> fill(ap.begin(), ap.end() - 1);
  for (int32_t i = 0; i < n; ++i)
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      const int32_t j = col_idx[k];
      if (j == i) continue;
      adj[fill[i]++] = j;
      adj[fill[j]++] = i;
    }
  auto by_degree = [&](int32_t x, int32_t y) { return deg[x] != deg[y] ? deg[x] < deg[y] : x < y; };
  for (int32_t i = 0; i < n; ++i) std::sort(adj.begin() + ap[i], adj.begin() + ap[i + 1], by_degree);
  std::vector<int32_t> starts((size_t)n);
  std::iota(starts.begin(), starts.end(), 0);
  std::sort(starts.begin(), starts.end(), by_degree);
  std::vector<char> seen((size_t)n, 0);
  std::vector<int32_t> order;
  order.reserve((size_t)n);
  for (int32_t s0 : starts) {
    if (seen[s0]) continue;
    seen[s0] = 1;
    size_t head = order.size();
    order.push_back(s0);
    while (head < order.size()) {
      const int32_t v = order[head++];
      for (int64_t e = ap[v]; e < ap[v + 1]; ++e) {
        const int32_t u = adj[e];
        if (!seen[u]) {
          seen[u] = 1;
          order.push_back(u);
        }
      }
    }
  }
  std::reverse(order.begin(), order.end());
  return order;
}

void build_plan(int32_t n, const int32_t *b, const int64_t *row_ptr, const int32_t *col_idx,
                int32_t row_order, HostPlan &plan) {
  plan.n = n;
  plan.off.assign((size_t)n + 1, 0);
  for (int32_t i = 0; i < n; ++i) plan.off[i + 1] = plan.off[i] + b[i];
  plan.N = plan.off[n];
  plan.nnzb = row_ptr[n];
  const int64_t nnzb = plan.nnzb;
  plan.gbase.assign((size_t)nnzb + 1, 0);
  plan.blk_row.assign((size_t)nnzb, 0);
  std::map<std::pair<int32_t, int32_t>, int32_t> shape_count;
  for (int32_t i = 0; i < n; ++i)
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      const int32_t j = col_idx[k];
      plan.blk_row[k] = i;
      plan.gbase[k + 1] = plan.gbase[k] + (int64_t)b[i] * b[j];
      shape_count[{b[i], b[j]}] += 1;
    }
  plan.nnz = plan.gbase[nnzb];
  plan.shapes.clear();
  for (const auto &kv : shape_count) plan.shapes.push_back({kv.first.first, kv.first.second, kv.second});
  std::vector<int32_t> order((size_t)n);
  std::iota(order.begin(), order.end(), 0);
  if (row_order != VBCSR_ORDER_ATOM) {
    std::vector<int32_t> rcm = rcm_order(n, row_ptr, col_idx);
    // AUTO keeps the caller's order unless RCM at least halves the mean
    // distance, in processing order, between the two atoms of a block
    // (a lattice or a spatially sorted input already has locality)
    bool take = row_order == VBCSR_ORDER_RCM;
    if (!take && nnzb > 0) {
      std::vector<int32_t> pos((size_t)n);
      for (int32_t t = 0; t < n; ++t) pos[rcm[t]] = t;
      double d_atom = 0.0, d_rcm = 0.0;
      for (int32_t i = 0; i < n; ++i)
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
          d_atom += std::abs((double)i - (double)col_idx[k]);
          d_rcm += std::abs((double)pos[i] - (double)pos[col_idx[k]]);
        }
      take = 2.0 * d_rcm <= d_atom;
    }
    if (take) order.swap(rcm);
  }

  // forward: panel i holds the blocks of block row i, ordered by (b_j, j)
  std::vector<std::vector<std::pair<int32_t, int64_t>>> members((size_t)n);
  for (int32_t i = 0; i < n; ++i) {
    auto &m = members[i];
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) m.push_back({col_idx[k], k});
    std::sort(m.begin(), m.end(), [&](const std::pair<int32_t, int64_t> &x,
                                      const std::pair<int32_t, int64_t> &y) {
      if (b[x.first] != b[y.first]) return b[x.first] < b[y.first];
      return x.first < y.first;
    });
  }
  layout_direction(n, b, plan.off, members, nnzb, &plan.gbase, order, plan.fwd);

  // transposed: panel j holds the blocks (i, j) of block column j, ordered by (b_i, i)
  for (auto &m : members) m.clear();
  for (int32_t i = 0; i < n; ++i)
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) members[col_idx[k]].push_back({i, k});
  for (auto &m : members)
    std::sort(m.begin(), m.end(), [&](const std::pair<int32_t, int64_t> &x,
                                      const std::pair<int32_t, int64_t> &y) {
      if (b[x.first] != b[y.first]) return b[x.first] < b[y.first];
      return x.first < y.first;
    });
  layout_direction(n, b, plan.off, members, nnzb, nullptr, order, plan.tr);
}

}  // namespace vbcsr
