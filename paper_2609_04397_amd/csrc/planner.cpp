// Host planner: validation, shape classes, and the page layout of both
// directions of the operator (paper, section 3.2: shape classes are counted
// from the distinct (b_i, b_j) and each block is placed in the value storage
// of its class; here the storage of a shape class inside a block row is one
// contiguous run of the row's panel).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <mutex>
#include <numeric>
#include <thread>

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
  RawVec<int32_t> mcol;
  RawVec<int64_t> mblk;
};

// Sort every panel's members by (b, atom); the atoms of a panel are
// distinct, so the order is unique.  A panel already ascending in the atom
// is bucketed by b (stable), any other is sorted on packed keys.
static void sort_members(int32_t n, const int32_t *b, Members &M) {
  parallel_rows(n, [&](int32_t r0, int32_t r1) {
    std::vector<std::pair<uint64_t, int64_t>> keyed;
    std::vector<int32_t> tcol;
    std::vector<int64_t> tblk;
    for (int32_t r = r0; r < r1; ++r) {
      const int64_t s0 = M.mptr[r], s1 = M.mptr[r + 1], len = s1 - s0;
      if (len < 2) continue;
      int32_t *col = M.mcol.data() + s0;
      int64_t *blk = M.mblk.data() + s0;
      bool ascending = true;
      for (int64_t u = 1; u < len && ascending; ++u) ascending = col[u - 1] < col[u];
      if (ascending) {
        int64_t start[VBCSR_MAX_BLOCK + 2] = {};
        for (int64_t u = 0; u < len; ++u) ++start[b[col[u]] + 1];
        for (int v = 1; v <= VBCSR_MAX_BLOCK + 1; ++v) start[v] += start[v - 1];
        tcol.resize(len);
        tblk.resize(len);
        for (int64_t u = 0; u < len; ++u) {
          const int64_t t = start[b[col[u]]]++;
          tcol[t] = col[u];
          tblk[t] = blk[u];
        }
        std::copy(tcol.begin(), tcol.end(), col);
        std::copy(tblk.begin(), tblk.end(), blk);
      } else {
        keyed.resize(len);
        for (int64_t u = 0; u < len; ++u)
          keyed[u] = {(uint64_t)b[col[u]] << 32 | (uint32_t)col[u], blk[u]};
        std::sort(keyed.begin(), keyed.end(),
                  [](const std::pair<uint64_t, int64_t> &x, const std::pair<uint64_t, int64_t> &y) {
                    return x.first < y.first;
                  });
        for (int64_t u = 0; u < len; ++u) {
          col[u] = (int32_t)(uint32_t)keyed[u].first;
          blk[u] = keyed[u].second;
        }
      }
    }
  });
}

// Lay out one direction from its members: panels in `order`, each panel's
// values and column-table entries contiguous.
static void layout_direction(int32_t n, const int32_t *b, const std::vector<int64_t> &off,
                             const Members &M, int64_t nnzb, const RawVec<int64_t> *gbase,
                             const std::vector<int32_t> &order, bool with_columns, DirPlan &d) {
  // panels: the atoms of `order` (all n, or the rows that may hold blocks)
  const int32_t np = (int32_t)order.size();
  d.rows.resize(np);
  d.vbase16.resize(np);
  // every graph block belongs to exactly one panel: the fill below writes
  // each entry once
  d.blk_pos.resize(nnzb);
  d.blk_k0.resize(nnzb);
  d.blk_prow.resize(nnzb);
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
  for (int32_t pi = 0; pi < np; ++pi) {
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
  parallel_rows(np, [&](int32_t p0, int32_t p1) {
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

// Transposed block graph: column j holds the blocks (i, j), ascending in i.
// Threads take contiguous row ranges; each counts its columns, the counts
// give every range its own offsets within each column, and every range then
// writes its blocks in row order, so the result does not depend on
// threading.
struct Transpose {
  std::vector<int64_t> ptr;  // n+1
  RawVec<int32_t> row;       // per entry: i
  RawVec<int64_t> blk;       // per entry: graph block index of (i, j)
};

static void transpose_graph(int32_t n, const int64_t *row_ptr, const int32_t *col_idx,
                            Transpose &T) {
  const int64_t nnzb = row_ptr[n];
  T.ptr.assign((size_t)n + 1, 0);
  T.row.resize(nnzb);
  T.blk.resize(nnzb);
  // ranges: at most 16, fewer when the per-range counts would pass 256 MiB
  int64_t R = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n < 8192 || nnzb < 65536) R = 1;
  R = std::max<int64_t>(1, std::min<int64_t>(R, (int64_t(256) << 20) / (8 * (int64_t)n + 8)));
  std::vector<int32_t> rb((size_t)R + 1, n);
  rb[0] = 0;
  for (int64_t t = 1; t < R; ++t) {
    const int64_t target = nnzb * t / R;
    rb[t] = (int32_t)(std::upper_bound(row_ptr, row_ptr + n + 1, target) - row_ptr - 1);
    rb[t] = std::max(rb[t], rb[t - 1]);
  }
  std::vector<int64_t> cnt((size_t)R * n, 0);
  // ranges whose thread cannot be started run in the caller; an exception
  // is rethrown once every thread has joined
  auto over_ranges = [&](auto &&body) {
    std::exception_ptr err;
    std::mutex mu;
    auto run = [&](int64_t t) {
      try {
        body(t);
      } catch (...) {
        std::lock_guard<std::mutex> lock(mu);
        if (!err) err = std::current_exception();
      }
    };
    std::vector<std::thread> th;
    int64_t started = 1;
    for (; started < R; ++started) {
      try {
        th.emplace_back(run, started);
      } catch (...) {
        break;
      }
    }
    run(0);
    for (int64_t t = started; t < R; ++t) run(t);
    for (auto &x : th) x.join();
    if (err) std::rethrow_exception(err);
  };
  over_ranges([&](int64_t t) {
    int64_t *c = cnt.data() + t * n;
    for (int64_t k = row_ptr[rb[t]]; k < row_ptr[rb[t + 1]]; ++k) ++c[col_idx[k]];
  });
  // column j: range 0's entries first, then range 1's, ...
  int64_t base = 0;
  for (int32_t j = 0; j < n; ++j) {
    T.ptr[j] = base;
    for (int64_t t = 0; t < R; ++t) {
      const int64_t c = cnt[t * n + j];
      cnt[t * n + j] = base;
      base += c;
    }
  }
  T.ptr[n] = base;
  over_ranges([&](int64_t t) {
    int64_t *at = cnt.data() + t * n;
    for (int32_t i = rb[t]; i < rb[t + 1]; ++i)
      for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
        const int64_t u = at[col_idx[k]]++;
        T.row[u] = i;
        T.blk[u] = k;
      }
  });
}

// Reverse Cuthill-McKee order of the symmetrised block graph: breadth-first
// from a lowest-degree unvisited atom of each component, neighbours in
// ascending degree, the whole sequence reversed.  Panels processed in this
// order are graph neighbours of the panels processed just before them, so
// the input rows they gather are still in the XCD's L2.  The neighbours of
// an atom are its off-diagonal blocks' atoms in its row and in its column (a
// pair present in both directions counts twice); ties are broken by the
// atom index.
static std::vector<int32_t> rcm_order(int32_t n, const int64_t *row_ptr, const int32_t *col_idx,
                                      const Transpose &T) {
  std::vector<int64_t> deg((size_t)n, 0);
  parallel_rows(n, [&](int32_t r0, int32_t r1) {
    for (int32_t i = r0; i < r1; ++i) {
      int64_t d = (row_ptr[i + 1] - row_ptr[i]) + (T.ptr[i + 1] - T.ptr[i]);
      for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
        if (col_idx[k] == i) d -= 2;  // the diagonal block is in both lists
      deg[i] = d;
    }
  });
  std::vector<int64_t> ap((size_t)n + 1, 0);
  for (int32_t i = 0; i < n; ++i) ap[i + 1] = ap[i] + deg[i];
  // neighbour lists as (degree, atom) keys, sorted per atom
  RawVec<uint64_t> adj((size_t)ap[n]);
  auto key = [&](int32_t x) { return (uint64_t)deg[x] << 32 | (uint32_t)x; };
  parallel_rows(n, [&](int32_t r0, int32_t r1) {
    for (int32_t i = r0; i < r1; ++i) {
      int64_t u = ap[i];
      for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
        if (col_idx[k] != i) adj[u++] = key(col_idx[k]);
      for (int64_t e = T.ptr[i]; e < T.ptr[i + 1]; ++e)
        if (T.row[e] != i) adj[u++] = key(T.row[e]);
      std::sort(adj.begin() + ap[i], adj.begin() + ap[i + 1]);
    }
  });
  std::vector<uint64_t> starts((size_t)n);
  for (int32_t i = 0; i < n; ++i) starts[i] = key(i);
  std::sort(starts.begin(), starts.end());
  std::vector<char> seen((size_t)n, 0);
  std::vector<int32_t> order;
  order.reserve((size_t)n);
  for (uint64_t sk : starts) {
    const int32_t s0 = (int32_t)(uint32_t)sk;
    if (seen[s0]) continue;
    seen[s0] = 1;
    size_t head = order.size();
    order.push_back(s0);
    while (head < order.size()) {
      const int32_t v = order[head++];
      for (int64_t e = ap[v]; e < ap[v + 1]; ++e) {
        const int32_t u = (int32_t)(uint32_t)adj[e];
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

// Clustered order: the atoms are taken in compact clusters of up to S atoms,
// each grown breadth-first over not yet taken atoms of the symmetrised block
// graph (and listed in ascending atom order), the next cluster seeded on the
// frontier of the previous one.  Panels
// processed together then gather the input rows of one cluster and its halo,
// which stay in the XCD's L2 while the cluster is processed, and consecutive
// clusters share halos.  Deterministic (sequential, neighbours in stored
// order).
// Atoms per cluster of the clustered order (measured: 64 to 4,096 within a
// few per cent of each other on the lattice, the zincblende particle and the
// random three-species structure; 256 best or tied on most products).
constexpr int32_t kClusterAtoms = 256;

static std::vector<int32_t> cluster_order(int32_t n, const int64_t *row_ptr,
                                          const int32_t *col_idx, const Transpose &T,
                                          int32_t S) {
  std::vector<char> seen((size_t)n, 0);
  std::vector<int32_t> order;
  order.reserve((size_t)n);
  std::vector<int32_t> queue;
  int32_t scan = 0, next_seed = -1;
  while ((int32_t)order.size() < n) {
    int32_t seed = next_seed;
    if (seed < 0 || seen[seed]) {
      while (scan < n && seen[scan]) ++scan;
      seed = scan;
    }
    next_seed = -1;
    const size_t c0 = order.size();
    queue.clear();
    queue.push_back(seed);
    seen[seed] = 1;
    size_t head = 0;
    while (head < queue.size()) {
      const int32_t v = queue[head++];
      order.push_back(v);
      if ((int64_t)(order.size() - c0) >= S) break;
      for (int64_t k = row_ptr[v]; k < row_ptr[v + 1]; ++k) {
        const int32_t u = col_idx[k];
        if (!seen[u]) {
          seen[u] = 1;
          queue.push_back(u);
        }
      }
      for (int64_t e = T.ptr[v]; e < T.ptr[v + 1]; ++e) {
        const int32_t u = T.row[e];
        if (!seen[u]) {
          seen[u] = 1;
          queue.push_back(u);
        }
      }
    }
    // atoms queued but not taken go back to the pool; the first of them
    // (adjacent to this cluster) seeds the next one
    for (size_t q = head; q < queue.size(); ++q) seen[queue[q]] = 0;
    if (head < queue.size()) next_seed = queue[head];
    // inside a cluster, ascending atoms: consecutive output rows (and
    // values in the caller's order) where the input order already has them
    std::sort(order.begin() + c0, order.end());
  }
  return order;
}

// Planner statistics on stderr (environment variable VBCSR_LOG set and not
// "0"): sizes, shape classes, the values the panel layout adds (alignment
// padding of the FP64/FP32 pages, 8-column padding of the BF16 pages), and
// how evenly the panels divide the work (largest and mean panel in values,
// the 4-panel workgroups' largest over mean).
static void log_plan(const HostPlan &plan, int32_t row_order) {
  const char *names[] = {"auto (clustered)", "atom", "rcm", "clustered"};
  const DirPlan &F = plan.fwd;
  int64_t vmax = 0, vsum = 0, wmax = 0, wsum = 0, nw = 0, wcur = 0;
  for (size_t r = 0; r < F.rows.size(); ++r) {
    const int64_t v = (int64_t)F.rows[r].b * F.rows[r].K;
    vmax = std::max(vmax, v);
    vsum += v;
    wcur += v;
    if (r % 4 == 3 || r + 1 == F.rows.size()) {
      wmax = std::max(wmax, wcur);
      wsum += wcur;
      ++nw;
      wcur = 0;
    }
  }
  const double np = std::max<double>(1.0, (double)F.rows.size());
  std::fprintf(stderr,
               "vbcsr plan: %d atoms (%d block rows), N %lld, %lld blocks, %lld values, order %s\n"
               "vbcsr plan: %zu shape classes:",
               plan.n, plan.n_rows, (long long)plan.N, (long long)plan.nnzb, (long long)plan.nnz,
               names[row_order >= 0 && row_order <= 3 ? row_order : 0], plan.shapes.size());
  for (const auto &sh : plan.shapes) std::fprintf(stderr, " %dx%d:%d", sh[0], sh[1], sh[2]);
  std::fprintf(stderr,
               "\nvbcsr plan: pages %lld values (+%.3f %% alignment), BF16 pages %lld (+%.3f %%)\n"
               "vbcsr plan: panel values max %lld mean %.1f; workgroup (4 panels) max/mean %.2f; "
               "transposed panels %zu\n",
               (long long)F.n_values, 100.0 * (double)(F.n_values - plan.nnz) / std::max<int64_t>(1, plan.nnz),
               (long long)F.n_values16,
               100.0 * (double)(F.n_values16 - plan.nnz) / std::max<int64_t>(1, plan.nnz),
               (long long)vmax, (double)vsum / np,
               nw ? (double)wmax / ((double)wsum / (double)nw) : 0.0, plan.tr.rows.size());
}

void build_plan(int32_t n, const int32_t *b, const int64_t *row_ptr, const int32_t *col_idx,
                int32_t row_order, HostPlan &plan, bool with_columns, int32_t n_rows) {
  if (n_rows < 0) n_rows = n;
  plan.n = n;
  plan.n_rows = n_rows;
  plan.off.assign((size_t)n + 1, 0);
  for (int32_t i = 0; i < n; ++i) plan.off[i + 1] = plan.off[i] + b[i];
  plan.N = plan.off[n];
  plan.N_rows = plan.off[n_rows];
  plan.nnzb = row_ptr[n];
  const int64_t nnzb = plan.nnzb;
  // graph value offsets: per-row sums, a prefix over rows, then the rows
  // in parallel; shape classes (b <= VBCSR_MAX_BLOCK) counted in a dense table
  std::vector<int64_t> rowv((size_t)n + 1, 0);
  std::vector<int64_t> shape_count((VBCSR_MAX_BLOCK + 1) * (VBCSR_MAX_BLOCK + 1), 0);
  parallel_rows(n, [&](int32_t r0, int32_t r1) {
    int64_t cnt[VBCSR_MAX_BLOCK + 1];
    for (int32_t i = r0; i < r1; ++i) {
      std::fill(cnt, cnt + VBCSR_MAX_BLOCK + 1, 0);
      int64_t v = 0;
      for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
        ++cnt[b[col_idx[k]]];
        v += (int64_t)b[i] * b[col_idx[k]];
      }
      rowv[i + 1] = v;
      for (int32_t bj = 1; bj <= VBCSR_MAX_BLOCK; ++bj)
        if (cnt[bj]) __atomic_fetch_add(&shape_count[b[i] * (VBCSR_MAX_BLOCK + 1) + bj], cnt[bj],
                                        __ATOMIC_RELAXED);
    }
  });
  for (int32_t i = 0; i < n; ++i) rowv[i + 1] += rowv[i];
  plan.gbase.resize((size_t)nnzb + 1);
  plan.blk_row.resize((size_t)nnzb);
  parallel_rows(n, [&](int32_t r0, int32_t r1) {
    for (int32_t i = r0; i < r1; ++i) {
      int64_t g = rowv[i];
      for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
        plan.blk_row[k] = i;
        plan.gbase[k] = g;
        g += (int64_t)b[i] * b[col_idx[k]];
      }
    }
  });
  plan.gbase[nnzb] = rowv[n];
  plan.nnz = rowv[n];
  plan.shapes.clear();
  for (int32_t bi = 1; bi <= VBCSR_MAX_BLOCK; ++bi)
    for (int32_t bj = 1; bj <= VBCSR_MAX_BLOCK; ++bj)
      if (shape_count[bi * (VBCSR_MAX_BLOCK + 1) + bj])
        plan.shapes.push_back({bi, bj, (int32_t)shape_count[bi * (VBCSR_MAX_BLOCK + 1) + bj]});
  Transpose T;
  transpose_graph(n, row_ptr, col_idx, T);
  std::vector<int32_t> order((size_t)n);
  std::iota(order.begin(), order.end(), 0);
  if (row_order == VBCSR_ORDER_CLUSTER || row_order == VBCSR_ORDER_AUTO) {
    order = cluster_order(n, row_ptr, col_idx, T, kClusterAtoms);
  } else if (row_order == VBCSR_ORDER_RCM) {
    order = rcm_order(n, row_ptr, col_idx, T);
  }

  // forward: panel i holds the blocks of block row i, ordered by (b_j, j)
  Members M;
  M.mptr.assign(row_ptr, row_ptr + n + 1);
  M.mcol.resize(nnzb);
  M.mblk.resize(nnzb);
  parallel_rows(n, [&](int32_t r0, int32_t r1) {
    for (int64_t k = row_ptr[r0]; k < row_ptr[r1]; ++k) {
      M.mcol[k] = col_idx[k];
      M.mblk[k] = k;
    }
  });
  sort_members(n, b, M);
  // a rank-local operator has panels only for its first n_rows atoms (the
  // rest have no blocks in their rows); they keep their processing order
  std::vector<int32_t> row_order_fwd;
  if (n_rows < n) {
    row_order_fwd.reserve((size_t)n_rows);
    for (int32_t r : order)
      if (r < n_rows) row_order_fwd.push_back(r);
  }
  layout_direction(n, b, plan.off, M, nnzb, &plan.gbase, n_rows < n ? row_order_fwd : order,
                   with_columns, plan.fwd);

  // transposed: panel j holds the blocks (i, j) of block column j, ordered
  // by (b_i, i)
  M.mptr.swap(T.ptr);
  M.mcol.swap(T.row);
  M.mblk.swap(T.blk);
  sort_members(n, b, M);
  layout_direction(n, b, plan.off, M, nnzb, nullptr, order, with_columns, plan.tr);
  if (const char *lg = std::getenv("VBCSR_LOG"); lg && *lg && *lg != '0') log_plan(plan, row_order);
}

}  // namespace vbcsr
