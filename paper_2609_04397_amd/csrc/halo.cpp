// Rank-local share of a distributed block graph and its halo exchange lists
// (paper, section 3.1: atoms are owned by ranks; a rank stores the block rows
// of its owned atoms over columns that are owned atoms or ghosts, the ghosts
// ordered by owner rank and then by global id, so that each neighbour's ghost
// rows form one contiguous range of the local input vector; section 3.2: the
// forward product first fetches the ghost rows, the adjoint returns the
// contributions of ghost columns to their owners, which add them).
//
// Host code only.  The plan of rank r is computed here from the whole graph
// (one process holds every rank's share on one GPU); in a multi-process
// run, the send lists are what each rank learns from its neighbours' ghost
// lists.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/vbcsr.h"
#include "common.hpp"
#include "kernels.hpp"

using namespace vbcsr;

struct vbcsr_halo {
  int32_t rank = 0, n_ranks = 0;
  int32_t n_owned = 0, n_ghost = 0;
  std::vector<int32_t> gid;        // local atom -> global atom (owned, then ghosts)
  std::vector<int32_t> b;          // local block sizes
  std::vector<int64_t> off;        // local scalar offsets, n_owned + n_ghost + 1
  std::vector<int64_t> row_ptr;    // n_owned + 1
  std::vector<int32_t> col_idx;    // local column ids
  std::vector<int64_t> src_row;    // per owned atom: first graph value of its global row
  std::vector<int64_t> row_vals;   // per owned atom: values of its row
  int64_t n_values = 0;
  std::vector<int64_t> send_ptr;   // n_ranks + 1, scalar rows of the send buffer per rank
  std::vector<int32_t> send_rows;  // local scalar row of every send-buffer row
  std::vector<int64_t> recv_ptr;   // n_ranks + 1, ghost scalar rows (after N_owned) per owner
  std::vector<int32_t> red_rows;   // owned scalar rows that receive adjoint contributions
  std::vector<int64_t> red_ptr;    // red_rows + 1
  std::vector<int64_t> red_pos;    // send-buffer rows adding into each red row, rank order
};

extern "C" {

int vbcsr_halo_create(vbcsr_halo **out, int32_t n_global, const int32_t *block_sizes,
                      const int64_t *row_ptr, const int32_t *col_idx, const int32_t *owner,
                      int32_t rank, int32_t n_ranks) try {
  if (!out) return set_error(VBCSR_EINVAL, "out is NULL");
  *out = nullptr;
  if (n_ranks < 1 || rank < 0 || rank >= n_ranks)
    return set_error(VBCSR_EINVAL, "need 0 <= rank < n_ranks");
  if (n_global > 0 && !owner) return set_error(VBCSR_EINVAL, "owner is NULL");
  std::string err;
  // the graph must be one vbcsr_create would take; with n_values = -1 a
  // well-formed graph fails only the final value count (ESHAPE)
  const int vrc = validate_graph(n_global, block_sizes, row_ptr, col_idx, -1, err);
  if (vrc != VBCSR_ESHAPE && vrc != VBCSR_OK) return set_error(vrc, err);
  for (int32_t i = 0; i < n_global; ++i)
    if (owner[i] < 0 || owner[i] >= n_ranks)
      return set_error(VBCSR_EINVAL, "owner of atom " + std::to_string(i) + " out of range");
  auto H = std::make_unique<vbcsr_halo>();
  H->rank = rank;
  H->n_ranks = n_ranks;
  std::vector<int64_t> gval((size_t)n_global + 1, 0);  // first graph value of each row
  for (int32_t i = 0; i < n_global; ++i) {
    int64_t v = 0;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) v += (int64_t)block_sizes[i] * block_sizes[col_idx[k]];
    gval[i + 1] = gval[i] + v;
  }
  // owned atoms ascending; ghosts: columns of owned rows owned elsewhere,
  // ordered by (owner, global id)
  std::vector<int32_t> local((size_t)n_global, -1);
  for (int32_t i = 0; i < n_global; ++i)
    if (owner[i] == rank) {
      local[i] = (int32_t)H->gid.size();
      H->gid.push_back(i);
    }
  H->n_owned = (int32_t)H->gid.size();
  std::vector<int32_t> ghosts;
  std::vector<char> seen((size_t)n_global, 0);
  for (int32_t u = 0; u < H->n_owned; ++u) {
    const int32_t i = H->gid[u];
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      const int32_t j = col_idx[k];
      if (owner[j] != rank && !seen[j]) {
        seen[j] = 1;
        ghosts.push_back(j);
      }
    }
  }
  std::sort(ghosts.begin(), ghosts.end(), [&](int32_t x, int32_t y) {
    return owner[x] != owner[y] ? owner[x] < owner[y] : x < y;
  });
  for (int32_t j : ghosts) {
    local[j] = (int32_t)H->gid.size();
    H->gid.push_back(j);
  }
  H->n_ghost = (int32_t)ghosts.size();
  const int32_t nl = H->n_owned + H->n_ghost;
  H->b.resize(nl);
  H->off.assign((size_t)nl + 1, 0);
  for (int32_t u = 0; u < nl; ++u) {
    H->b[u] = block_sizes[H->gid[u]];
    H->off[u + 1] = H->off[u] + H->b[u];
  }
  if (H->off[nl] > INT32_MAX) return set_error(VBCSR_EUNSUPPORTED, "more than 2^31-1 local scalar rows");
  // local rows keep the global order of their blocks
  H->row_ptr.assign((size_t)H->n_owned + 1, 0);
  H->src_row.resize(H->n_owned);
  H->row_vals.resize(H->n_owned);
  for (int32_t u = 0; u < H->n_owned; ++u) {
    const int32_t i = H->gid[u];
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) H->col_idx.push_back(local[col_idx[k]]);
    H->row_ptr[u + 1] = (int64_t)H->col_idx.size();
    H->src_row[u] = gval[i];
    H->row_vals[u] = gval[i + 1] - gval[i];
    H->n_values += H->row_vals[u];
  }
  // receive ranges: the ghosts of owner s are contiguous
  H->recv_ptr.assign((size_t)n_ranks + 1, 0);
  for (int32_t g = 0; g < H->n_ghost; ++g) H->recv_ptr[owner[ghosts[g]] + 1] += H->b[H->n_owned + g];
  for (int32_t s = 0; s < n_ranks; ++s) H->recv_ptr[s + 1] += H->recv_ptr[s];
  // send lists: for every other rank s, the owned atoms that a row owned by
  // s references, ascending global id (the order of s's ghosts from us)
  std::vector<std::vector<int32_t>> need((size_t)n_ranks);
  std::vector<int32_t> mark((size_t)n_global, -1);
  for (int32_t s = 0; s < n_ranks; ++s) {
    if (s == rank) continue;
    for (int32_t k0 = 0; k0 < n_global; ++k0) {
      if (owner[k0] != s) continue;
      for (int64_t k = row_ptr[k0]; k < row_ptr[k0 + 1]; ++k) {
        const int32_t j = col_idx[k];
        if (owner[j] == rank && mark[j] != s) {
          mark[j] = s;
          need[s].push_back(j);
        }
      }
    }
    std::sort(need[s].begin(), need[s].end());
  }
  H->send_ptr.assign((size_t)n_ranks + 1, 0);
  for (int32_t s = 0; s < n_ranks; ++s) {
    for (int32_t j : need[s]) {
      const int32_t u = local[j];
      for (int32_t q = 0; q < H->b[u]; ++q) H->send_rows.push_back((int32_t)(H->off[u] + q));
    }
    H->send_ptr[s + 1] = (int64_t)H->send_rows.size();
  }
  // adjoint reduction map: every owned scalar row in the send lists, with
  // the buffer rows that add into it in ascending (rank) order
  const int64_t ns = (int64_t)H->send_rows.size();
  std::vector<int64_t> idx((size_t)ns);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(),
                   [&](int64_t x, int64_t y) { return H->send_rows[x] < H->send_rows[y]; });
  H->red_ptr.push_back(0);
  for (int64_t t = 0; t < ns; ++t) {
    const int32_t r = H->send_rows[idx[t]];
    if (H->red_rows.empty() || H->red_rows.back() != r) {
      if (!H->red_rows.empty()) H->red_ptr.push_back(t);
      H->red_rows.push_back(r);
    }
    H->red_pos.push_back(idx[t]);
  }
  if (!H->red_rows.empty()) H->red_ptr.push_back(ns);
  *out = H.release();
  return VBCSR_OK;
} catch (...) {
  return api_exception("vbcsr_halo_create");
}

int vbcsr_halo_info(const vbcsr_halo *H, int32_t *n_owned, int32_t *n_ghost, int64_t *nnzb,
                    int64_t *n_values, int64_t *n_send_rows, int64_t *n_red_rows) try {
  if (!H) return set_error(VBCSR_EINVAL, "halo handle is NULL");
  if (n_owned) *n_owned = H->n_owned;
  if (n_ghost) *n_ghost = H->n_ghost;
  if (nnzb) *nnzb = (int64_t)H->col_idx.size();
  if (n_values) *n_values = H->n_values;
  if (n_send_rows) *n_send_rows = (int64_t)H->send_rows.size();
  if (n_red_rows) *n_red_rows = (int64_t)H->red_rows.size();
  return VBCSR_OK;
} catch (...) {
  return api_exception("vbcsr_halo_info");
}

int vbcsr_halo_graph(const vbcsr_halo *H, int32_t *gid, int32_t *block_sizes, int64_t *row_ptr,
                     int32_t *col_idx) try {
  if (!H) return set_error(VBCSR_EINVAL, "halo handle is NULL");
  if (gid) std::copy(H->gid.begin(), H->gid.end(), gid);
  if (block_sizes) std::copy(H->b.begin(), H->b.end(), block_sizes);
  if (row_ptr) std::copy(H->row_ptr.begin(), H->row_ptr.end(), row_ptr);
  if (col_idx) std::copy(H->col_idx.begin(), H->col_idx.end(), col_idx);
  return VBCSR_OK;
} catch (...) {
  return api_exception("vbcsr_halo_graph");
}

int vbcsr_halo_local_values(const vbcsr_halo *H, const double *global_values, double *local_values) try {
  if (!H) return set_error(VBCSR_EINVAL, "halo handle is NULL");
  if (H->n_values && (!global_values || !local_values))
    return set_error(VBCSR_EINVAL, "values pointer is NULL");
  int64_t at = 0;
  for (int32_t u = 0; u < H->n_owned; ++u) {
    std::memcpy(local_values + at, global_values + H->src_row[u], sizeof(double) * H->row_vals[u]);
    at += H->row_vals[u];
  }
  return VBCSR_OK;
} catch (...) {
  return api_exception("vbcsr_halo_local_values");
}

int vbcsr_halo_lists(const vbcsr_halo *H, int64_t *send_ptr, int32_t *send_rows, int64_t *recv_ptr,
                     int32_t *red_rows, int64_t *red_ptr, int64_t *red_pos) try {
  if (!H) return set_error(VBCSR_EINVAL, "halo handle is NULL");
  if (send_ptr) std::copy(H->send_ptr.begin(), H->send_ptr.end(), send_ptr);
  if (send_rows) std::copy(H->send_rows.begin(), H->send_rows.end(), send_rows);
  if (recv_ptr) std::copy(H->recv_ptr.begin(), H->recv_ptr.end(), recv_ptr);
  if (red_rows) std::copy(H->red_rows.begin(), H->red_rows.end(), red_rows);
  if (red_ptr) {
    if (H->red_rows.empty())
      red_ptr[0] = 0;
    else
      std::copy(H->red_ptr.begin(), H->red_ptr.end(), red_ptr);
  }
  if (red_pos) std::copy(H->red_pos.begin(), H->red_pos.end(), red_pos);
  return VBCSR_OK;
} catch (...) {
  return api_exception("vbcsr_halo_lists");
}

static bool overlap(const void *a, size_t an, const void *b, size_t bn) {
  const char *pa = static_cast<const char *>(a), *pb = static_cast<const char *>(b);
  return pa < pb + bn && pb < pa + an;
}

int vbcsr_halo_pack(const void *X, int64_t x_rows, int64_t ldx, const int32_t *rows,
                    int64_t nrows, int32_t nrhs, int32_t dtype, void *buf, int64_t ldb,
                    void *stream) try {
  if (dtype != 0 && dtype != 1) return set_error(VBCSR_EINVAL, "dtype must be 0 (double) or 1 (float)");
  if (nrhs <= 0 || nrows < 0 || x_rows < 0) return set_error(VBCSR_EINVAL, "need nrhs >= 1, nrows >= 0, x_rows >= 0");
  if (ldx < nrhs || ldb < nrhs) return set_error(VBCSR_EINVAL, "leading dimension smaller than nrhs");
  if (nrows == 0) return VBCSR_OK;
  if (!rows || !buf || (x_rows > 0 && !X)) return set_error(VBCSR_EINVAL, "pointer is NULL");
  const size_t es = dtype == 0 ? 8 : 4;
  if (x_rows > 0 && overlap(X, ((size_t)(x_rows - 1) * ldx + nrhs) * es, buf,
                            ((size_t)(nrows - 1) * ldb + nrhs) * es))
    return set_error(VBCSR_EINVAL, "X and buf overlap");
  hipError_t e = launch_rows_pack(X, x_rows, ldx, rows, nrows, nrhs, (int)es, buf, ldb,
                                  static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return set_error(VBCSR_EHIP, std::string("halo pack launch: ") + hipGetErrorString(e));
  return VBCSR_OK;
} catch (...) {
  return api_exception("vbcsr_halo_pack");
}

int vbcsr_halo_reduce(void *Y, int64_t y_rows, int64_t ldy, const int32_t *red_rows,
                      const int64_t *red_ptr, const int64_t *red_pos, int64_t n_red,
                      const void *buf, int64_t buf_rows, int64_t ldb, int32_t nrhs, int32_t dtype,
                      void *stream) try {
  if (dtype != 0 && dtype != 1) return set_error(VBCSR_EINVAL, "dtype must be 0 (double) or 1 (float)");
  if (nrhs <= 0 || n_red < 0 || y_rows < 0 || buf_rows < 0)
    return set_error(VBCSR_EINVAL, "need nrhs >= 1 and non-negative sizes");
  if (ldy < nrhs || ldb < nrhs) return set_error(VBCSR_EINVAL, "leading dimension smaller than nrhs");
  if (n_red == 0) return VBCSR_OK;
  if (!Y || !red_rows || !red_ptr || !red_pos || (buf_rows > 0 && !buf))
    return set_error(VBCSR_EINVAL, "pointer is NULL");
  const size_t es = dtype == 0 ? 8 : 4;
  if (buf_rows > 0 && overlap(Y, ((size_t)(y_rows > 0 ? y_rows - 1 : 0) * ldy + nrhs) * es, buf,
                              ((size_t)(buf_rows - 1) * ldb + nrhs) * es))
    return set_error(VBCSR_EINVAL, "Y and buf overlap");
  hipError_t e = launch_rows_reduce(Y, y_rows, ldy, red_rows, red_ptr, red_pos, n_red, buf_rows,
                                    buf, ldb, nrhs, (int)es, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return set_error(VBCSR_EHIP, std::string("halo reduce launch: ") + hipGetErrorString(e));
  return VBCSR_OK;
} catch (...) {
  return api_exception("vbcsr_halo_reduce");
}

void vbcsr_halo_destroy(vbcsr_halo *H) { delete H; }

}  // extern "C"
