// Host planner: validation, shape classes, and the page layout of both
// directions of the operator (paper, section 3.2: shape classes are counted
// from the distinct (b_i, b_j) and every logical block is mapped to its place
// in a shape-specific buffer; here the buffer of a shape class inside a block
// row is one contiguous run of the row's panel).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>

#include "../../include/vbcsr.h"
#include "common.hpp"

namespace vbcsr {

// Run body(r0, r1) over row chunks on up to 16 threads (one for small n).
template <typename F>
static void parallel_rows(int32_t n, F &&body) {
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n < 8192) nt = 1;
  const int32_t chunk = 512;
  std::atomic<int32_t> next{0};
  auto work = [&]() {
    for (;;) {
      const int32_t r0 = next.fetch_add(chunk);
      if (r0 >= n) break;
      body(r0, std::min(n, r0 + chunk));
    }
  };
  std::vector<std::thread> th;
  for (unsigned t = 1; t < nt; ++t) th.emplace_back(work);
  work();
  for (auto &x : th) x.join();
}

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
  // rows are checked in parallel; the error reported is the first in row
  // order (the row is checked again, sequentially, for its message)
  std::vector<int64_t> row_nnz(n, 0);
  std::vector<char> row_bad(n, 0);
  auto check_row = [&](int32_t i, std::vector<int32_t> &tmp, std::string *msg) -> int {
    tmp.assign(col_idx + row_ptr[i], col_idx + row_ptr[i + 1]);
    int64_t s = 0;
    for (int32_t j : tmp) {
      if (j < 0 || j >= n) {
        if (msg) *msg = "col_idx " + std::to_string(j) + " out of range in row " + std::to_string(i);
        return VBCSR_EINVAL;
      }
      s += (int64_t)b[i] * b[j];
    }
    std::sort(tmp.begin(), tmp.end());
    for (size_t t = 1; t < tmp.size(); ++t)
      if (tmp[t] == tmp[t - 1]) {
        if (msg) *msg = "duplicate block (" + std::to_string(i) + ", " + std::to_string(tmp[t]) + ")";
        return VBCSR_EDUP;
      }
    row_nnz[i] = s;
    return VBCSR_OK;
  };
  parallel_rows(n, [&](int32_t r0, int32_t r1) {
    std::vector<int32_t> tmp;
    for (int32_t i = r0; i < r1; ++i) row_bad[i] = check_row(i, tmp, nullptr) != VBCSR_OK;
  });
  int64_t nnz = 0;
  {
    std::vector<int32_t> tmp;
    for (int32_t i = 0; i < n; ++i) {
      if (row_bad[i]) return check_row(i, tmp, &err);
      nnz += row_nnz[i];
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

// Members of every panel as CSR: panel r holds mcol[mptr[r] .. mptr[r+1])
// (the atom indexing the block's panel columns) for graph blocks
// mblk[...], sorted by (b of that atom, atom).
struct Members {
  std::vector<int64_t> mptr;
  std::vector<int32_t> mcol;
  std::vector<int64_t> mblk;
};

static void sort_members(int32_t n, const int32_t *b, Members &M) {
  parallel_rows(n, [&](int32_t r0, int32_t r1) {
    std::vector<std::pair<int32_t, int64_t>> tmp;
    for (int32_t r = r0; r < r1; ++r) {
      const int64_t s0 = M.mptr[r], s1 = M.mptr[r + 1];
      tmp.clear();
      for (int64_t u = s0; u < s1; ++u) tmp.push_back({M.mcol[u], M.mblk[u]});
      std::sort(tmp.begin(), tmp.end(), [&](const std::pair<int32_t, int64_t> &x,
                                            const std::pair<int32_t, int64_t> &y) {
        if (b[x.first] != b[y.first]) return b[x.first] < b[y.first];
        return x.first < y.first;
      });
      for (int64_t u = s0; u < s1; ++u) {
        M.mcol[u] = tmp[u - s0].first;
        M.mblk[u] = tmp[u - s0].second;
      }
    }
  });
}

// Lay out one direction from its members: panels in `order`, each panel's
// values and column-table entries contiguous.
static void layout_direction(int32_t n, const int32_t *b, const std::vector<int64_t> &off,
                             const Members &M, int64_t nnzb, const std::vector<int64_t> *gbase,
                             const std::vector<int32_t> &order, bool with_columns, DirPlan &d) {
  d.rows.resize(n);
  d.vbase16.resize(n);
  d.blk_pos.assign(nnzb, 0);
  d.blk_k0.assign(nnzb, 0);
  d.blk_prow.assign(nnzb, 0);
  // panel widths, then offsets in processing order (panels start on
  // 4-value boundaries, zero padding: a 16-byte load of values never mixes
  // two panels)
  std::vector<int32_t> width(n, 0);
  parallel_rows(n, [&](int32_t r0, int32_t r1) {
    for (int32_t r = r0; r < r1; ++r) {
      int32_t K = 0;
      for (int64_t u = M.mptr[r]; u < M.mptr[r + 1]; ++u) K += b[M.mcol[u]];
      width[r] = K;
    }
  });
  int64_t vbase = 0, cbase = 0, vbase16 = 0;
  for (int32_t pi = 0; pi < n; ++pi) {
    const int32_t r = order[pi];
    const int32_t h = b[r], K = width[r];
    RowDesc rd{};
    rd.vbase = vbase;
    rd.cbase = cbase;
    rd.K = K;
    rd.yrow = (int32_t)off[r];
    rd.b = h;
    d.rows[pi] = rd;
    d.vbase16[pi] = vbase16;
    vbase += ((int64_t)h * K + kPanelAlign - 1) / kPanelAlign * kPanelAlign;
    cbase += K;
    vbase16 += (int64_t)h * ((K + 7) / 8 * 8);
  }
  d.n_values = vbase;
  d.n_cols = cbase;
  d.n_values16 = vbase16;
  if (with_columns) {
    d.colx.assign(cbase, 0);
    if (gbase) d.colg.assign(cbase, 0);
  }
  parallel_rows(n, [&](int32_t p0, int32_t p1) {
    for (int32_t pi = p0; pi < p1; ++pi) {
      const int32_t r = order[pi];
      const RowDesc &rd = d.rows[pi];
      int32_t k0 = 0;
      for (int64_t u = M.mptr[r]; u < M.mptr[r + 1]; ++u) {
        const int32_t c = M.mcol[u];   // atom indexing the block's panel columns
        const int64_t k = M.mblk[u];   // graph block index
        d.blk_pos[k] = rd.vbase + (int64_t)k0 * rd.b;
        d.blk_k0[k] = k0;
        d.blk_prow[k] = pi;
        if (with_columns)
          for (int32_t q = 0; q < b[c]; ++q) {
            d.colx[rd.cbase + k0 + q] = (int32_t)(off[c] + q);
            if (gbase) d.colg[rd.cbase + k0 + q] = (((*gbase)[k] + q) << 7) | b[c];
          }
        k0 += b[c];
      }
    }
  });
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
  parallel_rows(n, [&](int32_t r0, int32_t r1) {
    for (int32_t i = r0; i < r1; ++i) std::sort(adj.begin() + ap[i], adj.begin() + ap[i + 1], by_degree);
  });
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
                int32_t row_order, HostPlan &plan, bool with_columns) {
  plan.n = n;
  plan.off.assign((size_t)n + 1, 0);
  for (int32_t i = 0; i < n; ++i) plan.off[i + 1] = plan.off[i] + b[i];
  plan.N = plan.off[n];
  plan.nnzb = row_ptr[n];
  const int64_t nnzb = plan.nnzb;
  plan.gbase.assign((size_t)nnzb + 1, 0);
  plan.blk_row.assign((size_t)nnzb, 0);
  // shape classes: b <= VBCSR_MAX_BLOCK, a dense table
  std::vector<int64_t> shape_count((VBCSR_MAX_BLOCK + 1) * (VBCSR_MAX_BLOCK + 1), 0);
  for (int32_t i = 0; i < n; ++i)
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      const int32_t j = col_idx[k];
      plan.blk_row[k] = i;
      plan.gbase[k + 1] = plan.gbase[k] + (int64_t)b[i] * b[j];
      shape_count[b[i] * (VBCSR_MAX_BLOCK + 1) + b[j]] += 1;
    }
  plan.nnz = plan.gbase[nnzb];
  plan.shapes.clear();
  for (int32_t bi = 1; bi <= VBCSR_MAX_BLOCK; ++bi)
    for (int32_t bj = 1; bj <= VBCSR_MAX_BLOCK; ++bj)
      if (shape_count[bi * (VBCSR_MAX_BLOCK + 1) + bj])
        plan.shapes.push_back({bi, bj, (int32_t)shape_count[bi * (VBCSR_MAX_BLOCK + 1) + bj]});
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
  Members M;
  M.mptr.assign(row_ptr, row_ptr + n + 1);
  M.mcol.assign(col_idx, col_idx + nnzb);
  M.mblk.resize(nnzb);
  std::iota(M.mblk.begin(), M.mblk.end(), int64_t(0));
  sort_members(n, b, M);
  layout_direction(n, b, plan.off, M, nnzb, &plan.gbase, order, with_columns, plan.fwd);

  // transposed: panel j holds the blocks (i, j) of block column j, ordered by (b_i, i)
  std::fill(M.mptr.begin(), M.mptr.end(), 0);
  for (int64_t k = 0; k < nnzb; ++k) M.mptr[col_idx[k] + 1]++;
  for (int32_t j = 0; j < n; ++j) M.mptr[j + 1] += M.mptr[j];
  {
    std::vector<int64_t> fill(M.mptr.begin(), M.mptr.end() - 1);
    for (int32_t i = 0; i < n; ++i)
      for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
        const int64_t u = fill[col_idx[k]]++;
        M.mcol[u] = i;
        M.mblk[u] = k;
      }
  }
  sort_members(n, b, M);
  layout_direction(n, b, plan.off, M, nnzb, nullptr, order, with_columns, plan.tr);
}

}  // namespace vbcsr
